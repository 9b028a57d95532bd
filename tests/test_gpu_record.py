"""GPU tests of the pair-distance record (qcams_propagate_record): the same
trajectory as qcams_propagate bit for bit; points at the start and after
every accepted step, consistent with the states; against the oracle's
fixed-step states; truncation at rec_max."""
import dataclasses

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


def _pair_distances(x, cA, cB):
    r1, r2 = x[0:3], x[3:6]
    return np.array([np.linalg.norm(r1), np.linalg.norm(r2 - cA * r1), np.linalg.norm(-r2 - cB * r1)])


def _setup(Q, torch, prm, ids, horizon=None):
    wl = W.config_batched(per_inst=8)
    ctx = Q.Context(wl.system, prm)
    ctx.set_instances(wl.instances)
    tid = torch.as_tensor(np.asarray(ids, dtype=np.int64), device="cuda:0")
    st = ctx.new_state(len(ids))
    ctx.init_conditions(tid, st)
    if horizon is not None:
        st.d[Q.F_TMAX].fill_(horizon)
        st.d[Q.F_RSTOP].fill_(1e9)
    return wl, ctx, st


@pytest.mark.parametrize("rk", [W.RK_DOPRI5, W.RK_DOP853], ids=["dopri5", "dop853"])
def test_record_is_the_propagated_trajectory(Q, torch, rk):
    prm = dataclasses.replace(W.Params(), rk=rk)
    ids = np.arange(0, 768, 7)
    wl, ctx, st = _setup(Q, torch, prm, ids)
    st2 = Q.State(st.d.clone(), st.nstep.clone(), st.nrej.clone(), st.status.clone())
    ctx.propagate(st)
    rmax = 100_000
    rec, cnt = ctx.propagate_record(st2, rmax)
    torch.cuda.synchronize()
    for a, b in ((st.d, st2.d), (st.nstep, st2.nstep), (st.nrej, st2.nrej), (st.status, st2.status)):
        assert torch.equal(a, b)
    cnt = cnt.cpu().numpy()
    ns = st.nstep.cpu().numpy()
    assert np.array_equal(cnt, np.minimum(ns + 1, rmax))
    d = st.d.cpu().numpy()
    r = rec.cpu().numpy()
    s = Q.make_system(wl.system)
    mA, mB = s.mass[0], s.mass[1]
    cA, cB = mA / (mA + mB), mB / (mA + mB)
    for c in range(len(ids)):
        pts = r[c, :cnt[c]]
        assert pts[0, 0] == 0.0 and np.all(np.diff(pts[:, 0]) > 0)
        if cnt[c] == ns[c] + 1:      # not truncated: the last point is the final state
            assert pts[-1, 0] == d[Q.F_T, c]
            assert np.allclose(pts[-1, 1:], _pair_distances(d[:6, c], cA, cB), rtol=1e-14, atol=0)


def test_record_against_oracle_fixed_steps(Q, torch, orc):
    """Fixed steps h = 0.5: the point after k steps has the pair distances of
    the oracle's state after k steps, to 1e-9 relative."""
    prm = dataclasses.replace(W.Params(), fixed_step=1, h_fixed=0.5)
    ids = [0, 100, 500]
    wl, ctx, st = _setup(Q, torch, prm, ids, horizon=60.0)
    rec, cnt = ctx.propagate_record(st, 1000)
    torch.cuda.synchronize()
    r, cnt = rec.cpu().numpy(), cnt.cpu().numpy()
    sys, oprm = orc.make_system(wl.system), orc.make_params(prm)
    m = [sys.mass[i] for i in range(3)]
    cA, cB = m[0] / (m[0] + m[1]), m[1] / (m[0] + m[1])
    firsts = np.array([I.first_id for I in wl.instances])
    for c, i in enumerate(ids):
        I = wl.instances[int(np.searchsorted(firsts, i, side="right") - 1)]
        lev = orc.level(sys, I.v, I.j)
        y0, aux, _ = orc.init(sys, oprm, orc.make_instance(I), lev, int(i))
        assert cnt[c] == 121
        for k in (1, 10, 57, 120):
            _, y, a, ns, _ = orc.propagate(sys, oprm, y0, np.r_[0.0, 0.5 * k, 1e9, aux[3], aux[4], 0])
            assert r[c, k, 0] == pytest.approx(0.5 * k, rel=1e-15)
            assert np.allclose(r[c, k, 1:], _pair_distances(y[:6], cA, cB), rtol=1e-9, atol=0)


def test_record_truncates(Q, torch):
    prm = W.Params()
    ids = np.arange(0, 64)
    wl, ctx, st = _setup(Q, torch, prm, ids)
    st2 = Q.State(st.d.clone(), st.nstep.clone(), st.nrej.clone(), st.status.clone())
    ctx.propagate(st)
    rec, cnt = ctx.propagate_record(st2, 16)
    torch.cuda.synchronize()
    assert np.all(cnt.cpu().numpy() == 16)
    assert torch.equal(st.d, st2.d)
    # an already stopped trajectory records nothing
    rec, cnt = ctx.propagate_record(st2, 16)
    torch.cuda.synchronize()
    assert np.all(cnt.cpu().numpy() == 0)
