"""GPU test of qcams_run_noalloc, the fused run whose work buffers live in the
library's static device scratch: through the C ABI it gives exactly what
qcams_run gives on the same installed instances (every per-trajectory field,
the ids, the per-instance cross sections and histograms), on two calls in a
row, the second on a smaller workload; it refuses graph mode and workloads
beyond its stated limit."""
import numpy as np
import pytest

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


def _workload(per, energies):
    inst, first = [], 0
    for Ec, v, j in energies:
        inst.append(W.Instance(Ec, v, j, per, first, 4242, W.B_AREA, 0.0, 8.0))
        first += per + 7
    return W.Workload("noalloc", W.h2ca_system(), W.Params(rk=W.RK_DOP853), inst)


def _poisoned_buffers(ctx, torch):
    """Run buffers filled with values no run writes, so that every compared
    field must have been written by the call under test."""
    buf = ctx.new_run_buffers()
    buf["state"].d.fill_(float("nan"))
    buf["state"].nstep.fill_(-7)
    buf["state"].nrej.fill_(-7)
    buf["state"].status.fill_(250)
    buf["outcome"].label.fill_(250)
    buf["outcome"].vt.fill_(-999)
    buf["outcome"].jt.fill_(-999)
    buf["outcome"].d.fill_(float("nan"))
    buf["ids"].fill_(-1)
    buf["xs"].fill_(float("nan"))
    buf["hist"].fill_(float("nan"))
    buf["sample"].fill_(float("nan"))
    return buf


def _snapshot(buf):
    st, out = buf["state"], buf["outcome"]
    return dict(d=st.d.cpu().numpy().copy(), nstep=st.nstep.cpu().numpy().copy(),
                nrej=st.nrej.cpu().numpy().copy(), status=st.status.cpu().numpy().copy(),
                label=out.label.cpu().numpy().copy(), vt=out.vt.cpu().numpy().copy(),
                jt=out.jt.cpu().numpy().copy(), od=out.d.cpu().numpy().copy(),
                ids=buf["ids"].cpu().numpy().copy(), xs=buf["xs"].cpu().numpy().copy(),
                hist=buf["hist"].cpu().numpy().copy(), sample=buf["sample"].cpu().numpy().copy())


def test_noalloc_run_equals_run_on_two_calls(Q, torch):
    big = _workload(300, [(1e3, 0, 0), (3e3, 2, 5), (1e4, 4, 0), (3e4, 0, 5), (6e4, 4, 5),
                          (1e5, 2, 0)])
    small = _workload(120, [(2e4, 1, 3), (8e4, 3, 0)])
    ctx = Q.Context(big.system, big.params)
    for wl in (big, small):
        print("noalloc vs run: %d instances, %d trajectories" % (len(wl.instances), wl.n_traj),
              flush=True)
        ctx.set_instances(wl.instances)
        opts = Q.RunOpts(blocks=0, refill_min=1, check_every=8, lpt=1, graph=0, rk=0, lanes=0)
        ref = _poisoned_buffers(ctx, torch)
        ctx.run(ref, opts)
        torch.cuda.synchronize()
        ref_ms = ctx.last_run_kernel_ms()
        a = _snapshot(ref)
        got = _poisoned_buffers(ctx, torch)
        ctx.run_noalloc(got, opts)
        torch.cuda.synchronize()
        b = _snapshot(got)
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
        assert not np.isnan(b["d"]).any() and np.all(b["status"] != Q.RUNNING)
        assert np.all(b["label"] <= Q.FAILED)
        assert np.array_equal(b["xs"][:, Q.XS_N], [i.n_traj for i in wl.instances])
        # the run-report calls describe this run
        assert ctx.last_run_kernel_ms() > 0.0 and ref_ms > 0.0
        trials = b["nstep"].astype(np.int64) + b["nrej"]
        lanes = ctx.last_run_options().lanes
        ws = ctx.last_run_wave_steps()
        assert ws >= trials.max() and trials.sum() <= ws * (64 // lanes)


def test_noalloc_run_refuses_graph_and_oversized_work(Q, torch):
    wl = _workload(50, [(1e4, 0, 0)])
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    with pytest.raises(Q.QcamsError, match="graph"):
        ctx.run_noalloc(buf, Q.RunOpts(graph=1))
    # one trajectory beyond the static limit of 2**21: refused before any launch
    n = (1 << 21) + 1
    over = [W.Instance(1e4, 0, 0, n, 0, 1, W.B_AREA, 0.0, 8.0)]
    ctx.set_instances(over)
    big = ctx.new_run_buffers()
    with pytest.raises(Q.QcamsError, match="static scratch limit"):
        ctx.run_noalloc(big)
