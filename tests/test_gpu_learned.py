"""GPU tests of the learned proposal: the BF16-MFMA network against the FP64
oracle evaluated on the same bfloat16-rounded operands (forward, gradient,
Adam, training), the feature map, the proposal tables, importance-sampled
initial conditions against the oracle's, and unbiasedness of the weighted
estimator."""
import math

import numpy as np
import pytest

import qcams_workloads as W
from oracle import mlp as OM

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


def _params(seed=0, scale=1.0):
    th = OM.he_uniform(seed) * scale
    rng = np.random.default_rng(seed + 100)
    # non-zero biases exercise the bias paths
    L = OM.unpack(th)
    L = [(W_, rng.normal(0, 0.05, b.shape)) for W_, b in L]
    return OM.pack(L).astype(np.float32)


def _inputs(n, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    y = rng.integers(0, 4, n).astype(np.int32)
    return x, y


def test_forward_matches_oracle(Q, torch):
    th = _params(0)
    net = Q.MLP(th)
    for n in (1, 64, 333):                       # one row, one tile, ragged tiles
        x, _ = _inputs(n)
        p = net.forward(torch.as_tensor(x, device="cuda:0")).cpu().numpy()
        _, pref, _ = OM.forward(th.astype(np.float64), x.astype(np.float64), use_bf16=True)
        assert np.allclose(p.sum(axis=1), 1.0, atol=1e-5)
        assert np.abs(p - pref).max() < 5e-3, np.abs(p - pref).max()
        assert np.abs(p - pref).mean() < 2e-4
    # all-zero weights except the output bias: softmax of the bias exactly
    th0 = np.zeros(OM.NPARAM, dtype=np.float32)
    th0[-4:] = [0.1, -0.3, 0.7, 0.0]
    net.set_params(th0)
    x, _ = _inputs(70)
    p = net.forward(torch.as_tensor(x, device="cuda:0")).cpu().numpy()
    e = np.exp(th0[-4:] - th0[-4:].max())
    assert np.allclose(p, e / e.sum(), atol=1e-6)


def test_gradient_matches_oracle(Q, torch):
    th = _params(2, scale=0.8)
    net = Q.MLP(th)
    x, y = _inputs(256, seed=4)
    y[::17] = -1                                 # rows without a class contribute nothing
    g, loss = net.gradient(torch.as_tensor(x, device="cuda:0"), torch.as_tensor(y, device="cuda:0"))
    g = g.cpu().numpy().astype(np.float64)
    keep = y >= 0
    # oracle on the kept rows, rescaled to the same mean over all n rows
    lref, gref = OM.backward(th.astype(np.float64), x[keep].astype(np.float64), y[keep], use_bf16=True)
    gref *= keep.sum() / len(y)
    lref *= keep.sum() / len(y)
    assert loss.item() == pytest.approx(lref, rel=2e-3)
    GL, RL = OM.unpack(g), OM.unpack(gref)
    for k in range(4):
        for a, b in zip(GL[k], RL[k]):
            a, b = a.ravel(), b.ravel()
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert cos > 0.9999 and rel < 1e-2, (k, cos, rel)
    # and close to the exact FP64 gradient (no bf16 rounding) at bf16 accuracy
    _, gex = OM.backward(th.astype(np.float64), x[keep].astype(np.float64), y[keep])
    gex *= keep.sum() / len(y)
    assert np.linalg.norm(g - gex) / np.linalg.norm(gex) < 5e-2


def test_adam_matches_oracle(Q, torch):
    th = _params(5)
    net = Q.MLP(th)
    rng = np.random.default_rng(9)
    m = np.zeros(OM.NPARAM)
    v = np.zeros(OM.NPARAM)
    ref = th.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(0, 1e-2, OM.NPARAM).astype(np.float32)
        net.adam(torch.as_tensor(g, device="cuda:0"), 1e-3)
        ref, m, v = OM.adam_step(ref, g.astype(np.float64), m, v, t, lr=1e-3)
    got = net.params().astype(np.float64)
    assert np.abs(got - ref).max() < 1e-6


def test_training_reduces_loss_like_the_oracle(Q, torch):
    """Minibatch Adam on a learnable synthetic task: the GPU's epoch loop
    (captured and replayed) and the FP64 oracle reach similar losses."""
    rng = np.random.default_rng(0)
    n, batch, epochs, lr = 2048, 256, 8, 2e-3
    x = rng.uniform(-1, 1, (n, 6))
    score = np.stack([x[:, 0] + x[:, 1], x[:, 2] - x[:, 3], x[:, 4] * 2, -x[:, 5] - x[:, 0]], 1)
    y = score.argmax(axis=1).astype(np.int32)
    th = _params(7, scale=1.0)
    net = Q.MLP(th)
    xd = torch.as_tensor(x.astype(np.float32), device="cuda:0")
    yd = torch.as_tensor(y, device="cuda:0")
    perm_d = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    loss_d = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    ref = th.astype(np.float64)
    m = np.zeros(OM.NPARAM)
    v = np.zeros(OM.NPARAM)
    t = 0
    losses_gpu, losses_ref = [], []
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        perm_d.copy_(torch.as_tensor(perm))
        net.train_epoch(xd, yd, perm_d, batch, lr, loss_d)
        torch.cuda.synchronize()
        losses_gpu.append(loss_d.item() / (n // batch))
        tot = 0.0
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            l, g = OM.backward(ref, x[idx], y[idx])
            t += 1
            ref, m, v = OM.adam_step(ref, g, m, v, t, lr=lr)
            tot += l
        losses_ref.append(tot / (n // batch))
    print("gpu", np.round(losses_gpu, 4), "oracle", np.round(losses_ref, 4))
    assert losses_gpu[-1] < 0.6 * losses_gpu[0]
    assert abs(losses_gpu[-1] - losses_ref[-1]) < 0.15 * losses_ref[-1] + 0.02
    # accuracy on the training set
    p = net.forward(xd).cpu().numpy()
    assert (p.argmax(axis=1) == y).mean() > 0.8


def test_features_and_labels(Q, torch, orc):
    wl = W.config_small(n_traj=40)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf)
    x, y = ctx.mlp_features(buf["ids"], buf["sample"], buf["outcome"])
    x = x.cpu().numpy()
    y = y.cpu().numpy()
    s = buf["sample"].cpu().numpy()
    lab = buf["outcome"].label.cpu().numpy().astype(np.int32)
    I = wl.instances[0]
    assert np.allclose(x[:, 0], (math.log10(I.Ec_K) - 3) / 2, atol=1e-6)
    assert np.allclose(x[:, 1], s[0] / 10.0, atol=1e-6)
    assert np.allclose(x[:, 2], I.v / 10.0) and np.allclose(x[:, 3], I.j / 10.0)
    assert np.allclose(x[:, 4], s[4], atol=1e-6) and np.allclose(x[:, 5], s[1], atol=1e-6)
    assert np.array_equal(y, np.where(lab < 4, lab, -1))


def _target(Q, n=3000, mode=W.B_PROPOSAL, seed=4242):
    inst = [W.Instance(5.0e4, 4, 0, n, 0, seed, mode, 0.0, 10.0)]
    return W.Workload("target", W.h2ca_system(), W.Params(), inst)


def test_uniform_proposal_has_unit_weights(Q, torch):
    wl = _target(Q, 512)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    q = ctx.proposal_build(None, 0, Q.DISS, 1.0).cpu().numpy()
    assert np.all(q == 1.0 / Q.PROP_CELLS)
    tid = ctx.all_ids()
    st = ctx.new_state(512)
    smp = torch.zeros((Q.NS, 512), dtype=torch.float64, device="cuda:0")
    ctx.init_conditions(tid, st, smp)
    torch.cuda.synchronize()
    assert np.all(smp[5].cpu().numpy() == 1.0)


def test_proposal_draws_match_oracle(Q, torch, orc):
    """A skewed table installed on both sides: the same cells, points and
    weights (a cell may differ only when the cell uniform lies within 1e-12 of
    a cumulative-probability edge)."""
    rng = np.random.default_rng(21)
    q = rng.uniform(0.05, 1.0, Q.PROP_CELLS)
    q[:512] *= 15.0
    wl = _target(Q, 700)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    ctx.proposal_set(q)
    tid = ctx.all_ids()
    st = ctx.new_state(700)
    smp = torch.zeros((Q.NS, 700), dtype=torch.float64, device="cuda:0")
    ctx.init_conditions(tid, st, smp)
    torch.cuda.synchronize()
    s = smp.cpu().numpy()
    d = st.d.cpu().numpy()
    sys, prm = orc.make_system(wl.system), orc.make_params(wl.params)
    inst = orc.make_instance(wl.instances[0])
    lev = orc.level(sys, 4, 0)
    cdf = np.cumsum(q) / q.sum()
    for i in range(700):
        y, aux, so = orc.init(sys, prm, inst, lev, i, prop_q=q)
        if not np.allclose(s[:, i], so, rtol=1e-13, atol=1e-15):
            u5 = orc.uniforms(wl.instances[0].seed, i)[5]
            assert np.abs(cdf - u5).min() < 1e-12, i
            continue
        rel = np.abs(d[:12, i] - y) / np.maximum(np.abs(y), 1.0)
        assert rel.max() < 1e-12, (i, rel.max())


def test_weighted_estimator_is_unbiased(Q, torch):
    """Dissociation of H2(v=4, j=0) + Ca at 5e4 K: importance-sampled runs
    with a skewed proposal agree with plain sampling within 3 combined
    standard errors, and the weights average to 1."""
    n = 6000
    rng = np.random.default_rng(5)
    q = np.ones(Q.PROP_CELLS)
    q[: 8 * 256] *= 6.0                          # over-sample b^2 < bmax^2 / 4
    res = {}
    for mode in (W.B_AREA, W.B_PROPOSAL):
        wl = _target(Q, n, mode, seed=777 + mode)
        ctx = Q.Context(wl.system, wl.params)
        ctx.set_instances(wl.instances)
        if mode == W.B_PROPOSAL:
            ctx.proposal_set(q)
        buf = ctx.new_run_buffers()
        ctx.run(buf)
        torch.cuda.synchronize()
        res[mode] = (buf["xs"].cpu().numpy()[0], buf["sample"][5].cpu().numpy())
    xs_p, w_p = res[W.B_AREA]
    xs_i, w_i = res[W.B_PROPOSAL]
    assert np.all(w_p == 1.0)
    assert abs(w_i.mean() - 1.0) < 4 * w_i.std() / math.sqrt(n)
    for c in range(4):
        comb = math.sqrt(xs_p[19 + c] ** 2 + xs_i[19 + c] ** 2)
        assert abs(xs_p[15 + c] - xs_i[15 + c]) <= 3 * comb + 1e-12, (c, xs_p[15 + c], xs_i[15 + c], comb)
    print("sigma plain", xs_p[15:19], "+-", xs_p[19:23])
    print("sigma IS   ", xs_i[15:19], "+-", xs_i[19:23])


@pytest.fixture(scope="module")
def trained(Q, torch):
    """The network trained as the benchmark trains it: 2e5 trajectories of the
    batched H2 + Ca instances (2084 each), 20 epochs of batch 4096."""
    from paper_2304_02731_amd import learned as L
    wl = W.config_learned_train()
    print("learned: training on %d trajectories" % wl.n_traj, flush=True)
    tr = L.train_network(wl.system, wl.params, wl.instances, epochs=20)
    print("train loss", np.round(tr.train_loss, 4), "val", tr.val_loss, "prior", tr.prior_loss,
          flush=True)
    return wl, tr


def _comparison(Q, trained, n, replicates):
    from paper_2304_02731_amd import learned as L
    wl, tr = trained
    tgt = W.config_learned_target(n_traj=n).instances[0]
    cmp = L.compare(wl.system, wl.params, tgt, tr.net, channel=Q.DISS, n=n,
                    replicates=replicates, alpha=0.1)
    print("n %d x %d replicates: ess %.3f, efficiency %.2f (95%% %.2f-%.2f), sigma plain %.4f, "
          "IS %.4f, var %.3g / %.3g, GPU s %.4f / %.4f"
          % (n, replicates, cmp.ess, cmp.efficiency, cmp.efficiency_ci95[0],
             cmp.efficiency_ci95[1], cmp.sigma_plain[Q.DISS], cmp.sigma_is[Q.DISS],
             cmp.var_plain, cmp.var_is, cmp.gpu_s_plain, cmp.gpu_s_is), flush=True)
    return cmp


R_LEARNED = 32


@pytest.fixture(scope="module")
def comparison(Q, trained):
    """Plain against learned sampling, 32 seeded replicates of 20,000
    trajectories each side."""
    return _comparison(Q, trained, 20000, R_LEARNED)


def test_learned_pipeline_end_to_end(Q, torch, trained, comparison):
    """The trained network beats the class prior, its dissociation proposal
    for H2(v=4, j=0) + Ca at 5e4 K is used (no fallback: ESS per draw >= 0.1),
    and the importance-sampled cross section agrees with plain sampling
    within 3 combined standard errors of the replicate means (Eq. (12)-(13):
    the weighted estimator keeps the average over the sampling measure)."""
    wl, tr = trained
    assert tr.train_loss[-1] < tr.train_loss[0]
    assert np.isfinite(tr.val_loss) and not tr.fallback and tr.val_loss < tr.prior_loss
    R = R_LEARNED
    cmp = comparison
    assert not cmp.fallback
    assert 0.1 <= cmp.ess <= 1.0
    # replicate means of independent seeds on both sides
    se = math.sqrt(cmp.var_plain / R + cmp.var_is / R)
    assert se > 0.0
    assert abs(cmp.sigma_plain[Q.DISS] - cmp.sigma_is[Q.DISS]) <= 3 * se, \
        (cmp.sigma_plain[Q.DISS], cmp.sigma_is[Q.DISS], se)


def test_learned_proposal_gains_over_plain_sampling(Q, torch, comparison):
    """What the trained network gains: the dissociation cross section's
    variance x GPU-seconds with the learned proposal is lower than with plain
    sampling, with the lower end of the 95 % interval of the efficiency ratio
    (F distribution of the replicate-variance ratio) above 1."""
    cmp = comparison
    assert not cmp.fallback
    assert cmp.var_is < cmp.var_plain
    assert cmp.efficiency_ci95[0] > 1.0, cmp.efficiency_ci95
