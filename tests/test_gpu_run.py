"""GPU tests of the fused persistent run (qcams_run): per-trajectory results
are a pure function of the trajectory id whatever the schedule (grid size,
refill threshold, check interval, instance order, one lane or a quad of
lanes per trajectory); graph replays equal the eager run; the autotuner
returns a valid option set; cross sections agree with the oracle within 3
combined standard errors; the run equals the unfused ABI path; the batched,
mixed-potential and sweep workloads at full size in the benchmark's launch
configuration."""
import math

import numpy as np
import pytest
from scipy import stats

import qcams_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def Q(torch):
    import paper_2304_02731_amd as Q
    Q.lib()
    return Q


def _mixed_energy_workload(per=150):
    """Six instances of very different trajectory lengths (1e3..1e5 K)."""
    inst, first = [], 0
    for Ec, v, j in [(1e3, 0, 0), (3e3, 2, 5), (1e4, 4, 0), (3e4, 0, 5), (6e4, 4, 5), (1e5, 2, 0)]:
        inst.append(W.Instance(Ec, v, j, per, first, 777, W.B_AREA, 0.0, 8.0))
        first += per + 13            # gaps between id ranges
    return W.Workload("mixed_energy", W.h2ca_system(), W.Params(), inst)


def _snapshot(buf):
    st, out = buf["state"], buf["outcome"]
    return dict(d=st.d.cpu().numpy().copy(), nstep=st.nstep.cpu().numpy().copy(),
                nrej=st.nrej.cpu().numpy().copy(), status=st.status.cpu().numpy().copy(),
                label=out.label.cpu().numpy().copy(), vt=out.vt.cpu().numpy().copy(),
                jt=out.jt.cpu().numpy().copy(), od=out.d.cpu().numpy().copy(),
                ids=buf["ids"].cpu().numpy().copy(), xs=buf["xs"].cpu().numpy().copy(),
                hist=buf["hist"].cpu().numpy().copy(), sample=buf["sample"].cpu().numpy().copy())


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("rk", [0, 2], ids=["context_dopri5", "dop853"])
def test_run_is_schedule_independent(Q, torch, rk):
    wl = _mixed_energy_workload()
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ref = None
    for blocks, rm, ce, lpt, lanes in [(0, 1, 1, 1, 4), (3, 1, 1, 1, 1), (5, 64, 1, 0, 4),
                                       (2, 8, 7, 1, 1), (1, 1, 3, 0, 4), (7, 3, 2, 1, 4),
                                       (0, 1, 8, 1, 1), (2, 8, 5, 1, 8), (0, 1, 1, 0, 8)]:
        o = Q.RunOpts(blocks=blocks, refill_min=rm, check_every=ce, lpt=lpt, graph=0, rk=rk,
                      lanes=lanes)
        ctx.run(buf, o)
        torch.cuda.synchronize()
        snap = _snapshot(buf)
        # every counted loop iteration steps between one and all slots of
        # its wave, and a trajectory's trials fall in distinct iterations
        trials = snap["nstep"].astype(np.int64) + snap["nrej"]
        ws = ctx.last_run_wave_steps()
        assert trials.sum() <= ws * (64 // lanes) and ws <= trials.sum(), (ws, trials.sum())
        assert ws >= trials.max()
        if ref is None:
            ref = snap
            # ids at natural positions: instances in id order, consecutive ids
            expect = np.concatenate([np.arange(i.first_id, i.first_id + i.n_traj) for i in wl.instances])
            assert np.array_equal(snap["ids"], expect)
            assert np.all(snap["status"] != Q.RUNNING)
            assert np.array_equal(snap["xs"][:, 0], [i.n_traj for i in wl.instances])
        else:
            _same(ref, snap)
    # the sampled draws equal those of the unfused initial-condition call
    tid = torch.as_tensor(ref["ids"], device="cuda:0")
    st = ctx.new_state(len(tid))
    smp = torch.zeros((Q.NS, len(tid)), dtype=torch.float64, device="cuda:0")
    ctx.init_conditions(tid, st, smp)
    torch.cuda.synchronize()
    assert np.array_equal(smp.cpu().numpy(), ref["sample"])
    d0 = st.d.cpu().numpy()
    for f in (Q.F_TMAX, Q.F_RSTOP, Q.F_E0, Q.F_ESCALE):
        assert np.array_equal(d0[f], ref["d"][f]), f


def test_run_agrees_with_unfused_path(Q, torch):
    """Same trajectories through init / propagate / classify / cross sections
    (one lane per trajectory) and through the fused run (quads): identical
    per-trajectory results, cross sections equal to rounding."""
    wl = _mixed_energy_workload(per=200)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf)
    tid = buf["ids"].clone()
    n = tid.numel()
    st = ctx.new_state(n)
    ctx.init_conditions(tid, st)
    ctx.propagate(st)
    out = ctx.new_outcome(n)
    ctx.classify(st, out)
    xs, _ = ctx.cross_sections(out, tid)
    torch.cuda.synchronize()
    r = _snapshot(buf)
    assert np.array_equal(st.d.cpu().numpy(), r["d"])
    assert np.array_equal(st.nstep.cpu().numpy(), r["nstep"])
    assert np.array_equal(st.nrej.cpu().numpy(), r["nrej"])
    assert np.array_equal(st.status.cpu().numpy(), r["status"])
    assert np.array_equal(out.label.cpu().numpy(), r["label"])
    assert np.array_equal(out.vt.cpu().numpy(), r["vt"])
    assert np.array_equal(out.jt.cpu().numpy(), r["jt"])
    assert np.array_equal(out.d.cpu().numpy(), r["od"], equal_nan=True)
    a, b = xs.cpu().numpy(), r["xs"]
    assert np.allclose(a, b, rtol=1e-13, atol=0.0)


def _system_cases():
    s = W.h2ca_system()
    bc = W.Pair("buck", {"A": 50.0, "b": 1.5, "C6": 40.0})
    generic = W.System(s.masses_amu, (s.pairs[0], bc, s.pairs[2]), "h2 generic")
    mixed = W.config_mixed(per_inst=2)
    # a Buckingham pair whose inner maximum (3.55 a0, 8.3e-3 Eh) is crossed
    # at these energies: trajectories end in COLLAPSE, decided per pair lane
    low = W.Pair("buck", {"A": 2.0, "b": 1.2, "C6": 40.0})
    collapse = W.System(s.masses_amu, (s.pairs[0], low, s.pairs[2]), "h2 low-barrier buck")
    return {"all_morse": (s, _mixed_energy_workload(per=40).instances),
            "lj_morse_buck": (mixed.system, mixed.instances[::40]),
            "generic": (generic, _mixed_energy_workload(per=40).instances),
            "buck_collapse": (collapse, _mixed_energy_workload(per=40).instances)}


@pytest.mark.parametrize("case", ["all_morse", "lj_morse_buck", "generic", "buck_collapse"])
@pytest.mark.parametrize("rk", [1, 2], ids=["dopri5", "dop853"])
def test_quad_lanes_equal_single_lane(Q, torch, case, rk):
    """The quad and octet layouts (four or eight lanes per trajectory, DPP
    exchanges) give the same bits as one lane per trajectory, for every
    kernel specialisation and both RK variants."""
    system, inst = _system_cases()[case]
    ctx = Q.Context(system, W.Params())
    ctx.set_instances(inst)
    buf = ctx.new_run_buffers()
    snaps = []
    for lanes in (1, 4, 8):
        ctx.run(buf, Q.RunOpts(refill_min=1, check_every=4, lpt=1, graph=0, rk=rk, lanes=lanes))
        torch.cuda.synchronize()
        snaps.append(_snapshot(buf))
    _same(snaps[0], snaps[1])
    _same(snaps[0], snaps[2])
    assert np.all(snaps[0]["status"] != Q.RUNNING)
    if case == "buck_collapse":
        assert np.any(snaps[0]["status"] == Q.COLLAPSE)
    print(case, "labels", np.bincount(snaps[0]["label"], minlength=6),
          "status", np.bincount(snaps[0]["status"], minlength=7))


def test_graph_replays_match_eager(Q, torch):
    wl = _mixed_energy_workload(per=64)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf, Q.RunOpts(graph=0, refill_min=1, check_every=1, lpt=1))
    torch.cuda.synchronize()
    ref = _snapshot(buf)
    for rep in range(3):
        # eager work on the same buffers between replays
        buf["xs"].zero_()
        buf["state"].d.fill_(-1.0)
        buf["outcome"].label.fill_(9)
        torch.cuda.synchronize()
        ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=1, lpt=1))
        torch.cuda.synchronize()
        _same(ref, _snapshot(buf))


def test_graph_switch_from_area_to_proposal_sampling(Q, torch):
    """One context, graph mode: a run with area-sampled instances is captured
    before any proposal table exists; then a proposal is installed and
    instances of the same sizes switch to proposal sampling.  The replayed
    run must use the proposal (it equals the eager run on the same context,
    and no trajectory is failed for a missing table)."""
    wl = _mixed_energy_workload(per=64)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=4, lpt=1))
    torch.cuda.synchronize()
    assert np.all(buf["outcome"].label.cpu().numpy() != Q.FAILED)
    q = np.ones(Q.PROP_CELLS)
    q[:1024] *= 8.0
    ctx.proposal_set(q)
    prop = [W.Instance(i.Ec_K, i.v, i.j, i.n_traj, i.first_id, i.seed, W.B_PROPOSAL, 0.0, i.bmax)
            for i in wl.instances]
    ctx.set_instances(prop)
    ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=4, lpt=1))
    torch.cuda.synchronize()
    got = _snapshot(buf)
    assert np.all(got["label"] != Q.FAILED)
    assert np.any(got["sample"][5] != 1.0)      # weights of the proposal
    ctx.run(buf, Q.RunOpts(graph=0, refill_min=1, check_every=4, lpt=1))
    torch.cuda.synchronize()
    _same(got, _snapshot(buf))


@pytest.mark.parametrize("search_rk", [False, True], ids=["schedule", "schedule_and_variant"])
def test_autotune_returns_valid_options(Q, torch, search_rk):
    wl = _mixed_energy_workload(per=32)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    best, ms = ctx.autotune(buf, reps=1, search_rk=search_rk, energy_gate=1e-8)
    assert ms > 0 and best.blocks > 0 and 1 <= best.refill_min <= 64 and best.check_every >= 1
    assert best.rk in ((1, 2) if search_rk else (0,))
    assert best.lanes in (1, 4, 8)
    ctx.run(buf, Q.RunOpts(graph=0, refill_min=1, check_every=1, lpt=1, rk=best.rk))
    torch.cuda.synchronize()
    ref = _snapshot(buf)
    ctx.run(buf, best)
    torch.cuda.synchronize()
    _same(ref, _snapshot(buf))
    ok = ref["label"] != Q.FAILED
    assert np.all(np.abs(ref["od"][3][ok]) < 1e-8)
    print("autotuned", best.as_dict(), "%.2f ms" % ms)


def test_autotune_cache(Q, torch):
    """A second autotune of the same key returns the cached options and time
    without timing again; retune replaces the entry."""
    wl = _mixed_energy_workload(per=24)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    b1, ms1 = ctx.autotune(buf, reps=1)
    ctx2 = Q.Context(wl.system, wl.params)          # another context, same key
    ctx2.set_instances(wl.instances)
    buf2 = ctx2.new_run_buffers()
    b2, ms2 = ctx2.autotune(buf2, reps=1)
    assert b1.as_dict() == b2.as_dict() and ms1 == ms2
    b3, ms3 = ctx2.autotune(buf2, reps=1, retune=True)
    assert ms3 != ms1 and b3.lanes in (1, 4, 8)
    b4, ms4 = ctx.autotune(buf, reps=1)
    assert b4.as_dict() == b3.as_dict() and ms4 == ms3


def test_autotune_cache_is_keyed_on_content(Q, torch):
    """Two workloads with the same numbers of instances and trajectories but
    different content (slow 1e3 K against fast 1e5 K collisions): the second
    is tuned on its own (its time is not the first one's cached time), and
    asking again returns its own cached entry."""
    def wl_at(Ec):
        inst = [W.Instance(Ec, v, 0, 96, 96 * k, 31337, W.B_AREA, 0.0, 8.0)
                for k, v in enumerate((0, 2, 4))]
        return W.Workload("tune_%g" % Ec, W.h2ca_system(), W.Params(), inst)
    res = {}
    for Ec in (1e5, 1e3):
        wl = wl_at(Ec)
        ctx = Q.Context(wl.system, wl.params)
        ctx.set_instances(wl.instances)
        buf = ctx.new_run_buffers()
        b, ms = ctx.autotune(buf, reps=1)
        b2, ms2 = ctx.autotune(buf, reps=1)
        assert b.as_dict() == b2.as_dict() and ms == ms2
        res[Ec] = ms
    print("autotuned ms: 1e5 K %.3f, 1e3 K %.3f" % (res[1e5], res[1e3]))
    assert res[1e3] > 2.0 * res[1e5]


def test_variant_override_equals_context_variant(Q, torch):
    """RunOpts.rk = 2 on a DOPRI5 context equals a DOP853 context's run."""
    wl = _mixed_energy_workload(per=48)
    out = []
    for rk_ctx, rk_opt in [(W.RK_DOP853, 0), (W.RK_DOPRI5, 2)]:
        p = W.Params(rk=rk_ctx)
        ctx = Q.Context(wl.system, p)
        ctx.set_instances(wl.instances)
        buf = ctx.new_run_buffers()
        ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=8, lpt=1, rk=rk_opt))
        torch.cuda.synchronize()
        out.append(_snapshot(buf))
    _same(out[0], out[1])


def test_run_cross_sections_vs_oracle(Q, torch, orc):
    """H2(v=0, j=0) + Ca at 1e4 K, b by area to 8 a0, 500 trajectories:
    reaction and dissociation are energetically closed, and the quench cross
    section matches the oracle's within 3 combined standard errors."""
    wl = W.config_small()
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf)
    torch.cuda.synchronize()
    xs = buf["xs"].cpu().numpy()[0]
    assert xs[0] == 500
    assert xs[1 + Q.R1] == 0 and xs[1 + Q.R2] == 0 and xs[1 + Q.DISS] == 0
    recs, which = orc.run_workload(wl, processes=8)
    ref = orc.cross_sections(wl, recs["label"], np.ones(len(recs)), which)
    for c in range(4):
        comb = math.sqrt(xs[19 + c] ** 2 + ref["dsigma"][0, c] ** 2)
        assert abs(xs[15 + c] - ref["sigma"][0, c]) <= 3 * comb + 1e-12, c
    print("sigma_q GPU %.4f +- %.4f  oracle %.4f +- %.4f" % (xs[15], xs[19], ref["sigma"][0, 0],
                                                           ref["dsigma"][0, 0]))


def test_full_size_bench_configuration(Q, torch, orc):
    """The 100,032-trajectory batched workload in the launch configuration and
    at the tolerances the benchmark times (DOP853 at the Sec. 3.1 example
    tolerances, quads chosen by run size, LPT, graph): every
    trajectory finishes inside the energy gate; sampled trajectories checked
    one by one against the oracle (draws bit-exact, classification of the
    GPU's own final state bit-exact); channel probabilities of the full run
    against the oracle's on a stratified subsample (42 ids of every
    instance, 4032 trajectories), per collision energy and channel and per
    instance and channel, by the exact binomial test at 3 standard errors
    (at most the chance number of the comparisons beyond 3, none beyond
    4.5), and pooled over all instances."""
    wl = W.config_batched()
    wl.params = W.gated_params(wl, W.RK_DOP853)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=8, lpt=1))
    torch.cuda.synchronize()
    used = ctx.last_run_options()
    assert used.lanes == 4 and used.rk == 2 and used.blocks > 0
    r = _snapshot(buf)
    n = len(r["ids"])
    assert n == 100032 and np.all(r["status"] != Q.RUNNING)
    lab, xs = r["label"], r["xs"]
    assert np.array_equal(xs[:, 0], [I.n_traj for I in wl.instances])
    fin = lab != Q.FAILED
    assert fin.mean() > 0.999
    assert np.abs(r["od"][3][fin]).max() < 1e-8
    sys, prm = orc.make_system(wl.system), orc.make_params(wl.params)
    firsts = np.array([I.first_id for I in wl.instances])
    which = np.searchsorted(firsts, r["ids"], side="right") - 1
    rng = np.random.default_rng(5)
    for c in rng.choice(n, 48, replace=False):
        I = wl.instances[which[c]]
        lev = orc.level(sys, I.v, I.j)
        _, _, sm = orc.init(sys, prm, orc.make_instance(I), lev, int(r["ids"][c]))
        assert np.array_equal(r["sample"][:5, c], sm[:5])
        if fin[c]:
            cl = orc.classify(sys, prm, r["d"][:12, c])
            assert (cl["label"], cl["vt"], cl["jt"]) == (lab[c], r["vt"][c], r["jt"][c]), c
    ref = _per_energy_channels_vs_oracle(orc, wl, xs[:, :5], per_inst=42)
    # per instance and channel: the oracle's count of 42 against the GPU's
    # probability from 1042 trajectories
    zs = []
    for k in range(len(wl.instances)):
        for ch in range(4):
            zs.append((_binom_z(int(round(float(ref["P"][k, ch] * 42))), 42, xs[k, 1 + ch], xs[k, 0]),
                       k, ch))
    _assert_z(zs, "(instance, channel)")


def _full_size_run(Q, torch, orc, wl, n_expect, seed):
    """One fused run of a whole workload in the benchmark's launch
    configuration and at its tolerances, then the checks that need no
    per-trajectory oracle integration: every trajectory finished, counts per
    instance, the energy gate, and 48 sampled trajectories one by one (initial
    draws bit-exact; the classification of the GPU's own final state
    bit-exact).  Returns the labels, ids and per-instance results."""
    wl.params = W.gated_params(wl, W.RK_DOP853)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf, Q.RunOpts(graph=1, refill_min=1, check_every=8, lpt=1))
    torch.cuda.synchronize()
    used = ctx.last_run_options()
    st, out = buf["state"], buf["outcome"]
    n = buf["ids"].numel()
    assert n == n_expect
    assert used.rk == 2 and used.blocks > 0 and used.lanes in (1, 4, 8)
    assert not bool((st.status == Q.RUNNING).any())
    lab = out.label.cpu().numpy()
    ids = buf["ids"].cpu().numpy()
    xs = buf["xs"].cpu().numpy()
    assert np.array_equal(xs[:, 0], [I.n_traj for I in wl.instances])
    assert np.array_equal(xs[:, 1:7].sum(axis=1), xs[:, 0])
    fin = lab != Q.FAILED
    assert fin.mean() > 0.999
    dE = out.d[3].cpu().numpy()
    assert np.abs(dE[fin]).max() < 1e-8, float(np.abs(dE[fin]).max())
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(n, 48, replace=False))
    tp = torch.as_tensor(pick, device=buf["ids"].device)
    smp = buf["sample"][:, tp].cpu().numpy()
    dfin = st.d[:12][:, tp].cpu().numpy()
    vt, jt = out.vt[tp].cpu().numpy(), out.jt[tp].cpu().numpy()
    sys, prm = orc.make_system(wl.system), orc.make_params(wl.params)
    firsts = np.array([I.first_id for I in wl.instances])
    which = np.searchsorted(firsts, ids, side="right") - 1
    for k, c in enumerate(pick):
        I = wl.instances[which[c]]
        lev = orc.level(sys, I.v, I.j)
        _, _, sm = orc.init(sys, prm, orc.make_instance(I), lev, int(ids[c]))
        assert np.array_equal(smp[:5, k], sm[:5]), c
        if fin[c]:
            cl = orc.classify(sys, prm, dfin[:, k])
            assert (cl["label"], cl["vt"], cl["jt"]) == (lab[c], vt[k], jt[k]), c
    return lab, ids, xs


def _binom_z(x_o, m, x_g, n_g):
    """Normal deviate of the two-sided exact binomial p-value of the
    oracle's x_o successes in m draws at the GPU's probability x_g / n_g
    (z <= 3: within 3 standard errors, also for the small counts of rare
    channels).  The GPU's estimate is taken as the probability (it comes
    from many times more trajectories), kept half a count away from 0 and 1
    so that a channel the GPU run never (or always) saw is tested at the
    largest (smallest) probability such a count leaves open instead of at
    exactly 0 (1)."""
    p_g = min(max(x_g, 0.5), n_g - 0.5) / n_g
    pv = stats.binomtest(x_o, m, p_g).pvalue
    return float(stats.norm.isf(pv / 2.0)) if pv < 1.0 else 0.0


def _assert_z(zs, what):
    """With K comparisons about 0.27 % lie beyond 3 by chance: the number
    beyond 3 may not exceed the 99.9 % quantile of Binomial(K, 0.0027), and
    none may exceed 4.5."""
    z = np.array([q[0] for q in zs])
    K = len(z)
    allowed = int(stats.binom.ppf(0.999, K, 0.0027))
    beyond = [q for q in zs if q[0] > 3.0]
    print("%d %s comparisons: largest z %.2f, %d beyond 3 (allowed %d); the largest five: %s"
          % (K, what, z.max(), len(beyond), allowed, sorted(zs, key=lambda q: -q[0])[:5]))
    assert len(beyond) <= allowed, beyond
    assert z.max() <= 4.5, max(zs, key=lambda q: q[0])


def _per_energy_channels_vs_oracle(orc, wl, xs, per_inst):
    """Eq. (16), (18): per collision energy and channel, the GPU's full run
    against the oracle's on a stratified subsample (the same number of ids
    from every instance, so both sides weight the (v, j) instances of an
    energy equally).  The oracle's count is tested against the GPU's
    probability (its estimate from ~600x as many trajectories) with the
    exact two-sided binomial test; z is the normal deviate of the same
    p-value, so z <= 3 is "within 3 standard errors", also for the small
    counts of rare channels where the normal approximation fails.  With K
    comparisons about 0.27 % lie beyond 3 by chance: the number beyond 3 may
    not exceed the 99.9 % quantile of Binomial(K, 0.0027), none may exceed
    4.5, and the channels pooled over all energies must be within 3 SE
    (two-proportion test, pooled proportion)."""
    per = [np.arange(I.first_id, I.first_id + I.n_traj, I.n_traj // per_inst,
                     dtype=np.int64)[:per_inst] for I in wl.instances]
    recs, w2 = orc.run_workload(wl, per, processes=16)
    ref = orc.cross_sections(wl, recs["label"], np.ones(len(recs)), w2)
    ecs = np.array([I.Ec_K for I in wl.instances])
    ng = xs[:, 0]
    zs = []
    for E in np.unique(ecs):
        rows = np.nonzero(ecs == E)[0]
        n_g = ng[rows].sum()
        m = per_inst * len(rows)
        for ch in range(4):
            x_g = xs[rows, 1 + ch].sum()
            x_o = int(round(float((ref["P"][rows, ch] * per_inst).sum())))
            zs.append((_binom_z(x_o, m, x_g, n_g), "%.4g" % E, ch, "%.4f" % (x_g / n_g),
                       "%.4f" % (x_o / m)))
    _assert_z(zs, "(E_c, channel)")
    n = ng.sum()
    m = per_inst * len(wl.instances)
    for ch in range(4):
        x_g = xs[:, 1 + ch].sum()
        x_o = float((ref["P"][:, ch] * per_inst).sum())
        p = (x_g + x_o) / (n + m)
        se = math.sqrt(p * (1 - p) * (1.0 / n + 1.0 / m))
        assert abs(x_g / n - x_o / m) <= 3 * se, (ch, x_g / n, x_o / m, se)
    print("pooled P gpu", xs[:, 1:5].sum(axis=0) / n, "oracle subsample",
          (ref["P"] * per_inst).sum(axis=0) / m, "oracle trajectories", m)
    return ref


def test_full_size_mixed_configuration(Q, torch, orc):
    """The 1,001,088-trajectory mixed-potential workload (generalized LJ 12-6,
    Morse, Buckingham; 2112 instances) at full size in the benchmark's launch
    configuration: the checks of _full_size_run, then the channel
    probabilities per collision energy against the oracle on two ids from
    every instance (4224 trajectories)."""
    wl = W.config_mixed()
    lab, ids, xs = _full_size_run(Q, torch, orc, wl, 1001088, seed=11)
    _per_energy_channels_vs_oracle(orc, wl, xs, per_inst=2)


def test_full_size_sweep_configuration(Q, torch, orc):
    """The 10,005,248-trajectory sweep (64 collision energies x v 0-10 x
    j 0-10, 7744 instances) at full size in the benchmark's launch
    configuration: the checks of _full_size_run, then the channel
    probabilities per collision energy against the oracle on two ids from
    every instance (15,488 trajectories)."""
    wl = W.config_sweep()
    lab, ids, xs = _full_size_run(Q, torch, orc, wl, 10005248, seed=13)
    _per_energy_channels_vs_oracle(orc, wl, xs, per_inst=2)
