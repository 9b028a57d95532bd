"""GPU tests of the fixed impact-parameter grid reduction (the paper's
Sec. 4 workflow, Eq. (18)-(19)): group structure; sigma, its error and the
rate against the oracle's trapezoid rule on the same per-b probabilities
(to rounding); and against the oracle's own runs on a subsample of every
b value (within 4 combined standard errors)."""
import math

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


def _grid_run(Q, torch, n_per_b):
    wl = W.config_paper_grid(n_per_b=n_per_b)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances)
    buf = ctx.new_run_buffers()
    ctx.run(buf, Q.RunOpts(graph=0, refill_min=1, check_every=8, lpt=1))
    grid = ctx.grid_cross_sections(buf["xs"])
    torch.cuda.synchronize()
    return wl, ctx, buf["xs"].cpu().numpy(), grid.cpu().numpy()


def test_grid_groups(Q, torch):
    wl = W.config_paper_grid(n_per_b=4)
    extra = W.Instance(3.0e4, 1, 0, 5, wl.instances[-1].first_id + 100, 99, W.B_AREA, 0.0, 5.0)
    ctx = Q.Context(wl.system, wl.params)
    ctx.set_instances(wl.instances + [extra])
    ng, g = ctx.grid_groups()
    assert ng == 10
    assert g[-1] == -1
    assert np.array_equal(g[:-1], np.repeat(np.arange(10), 20))


def test_grid_sigma_matches_oracle_trapezoid(Q, torch, orc):
    """Same per-b P and dP on both sides: sigma and its error to rounding,
    rate = sigma sqrt(2 E_c / mu_123)."""
    wl, ctx, xs, grid = _grid_run(Q, torch, 64)
    assert grid.shape == (10, Q.GRID_STRIDE)
    sys = orc.make_system(wl.system)
    _, mu123, _ = orc.reduced_masses(sys)
    for g in range(10):
        rows = np.arange(20 * g, 20 * g + 20)
        b = np.array([wl.instances[k].b for k in rows])
        Ec = wl.instances[rows[0]].Ec_K
        assert grid[g, Q.G_EC] == Ec and grid[g, Q.G_V] == 1 and grid[g, Q.G_J] == 0
        assert grid[g, Q.G_NB] == 20 and grid[g, Q.G_BMAX] == 4.75 and grid[g, Q.G_N] == 20 * 64
        for c in range(4):
            s, e = orc.sigma_from_grid(b, xs[rows, Q.XS_P + c], xs[rows, Q.XS_DP + c])
            assert grid[g, Q.G_SIGMA + c] == pytest.approx(s, rel=1e-13, abs=1e-15)
            assert grid[g, Q.G_DSIGMA + c] == pytest.approx(e, rel=1e-13, abs=1e-15)
            k = s * math.sqrt(2.0 * Ec * orc.KELVIN / mu123)
            assert grid[g, Q.G_RATE + c] == pytest.approx(k, rel=1e-13, abs=1e-20)


def test_grid_sigma_statistical_vs_oracle(Q, torch, orc):
    """GPU grid sigma from 256 trajectories per b against the oracle's grid
    sigma from every 8th of them (32 per b), per E_c and channel.  The
    oracle's per-b errors use two pseudo-events (Agresti-Coull), so that a
    channel it happens not to see at 32 draws per b keeps a nonzero error."""
    wl, ctx, xs, grid = _grid_run(Q, torch, 256)
    per = [np.arange(I.first_id, I.first_id + I.n_traj, 8, dtype=np.int64) for I in wl.instances]
    recs, which = orc.run_workload(wl, per, processes=8)
    ref = orc.cross_sections(wl, recs["label"], np.ones(len(recs)), which)
    worst = 0.0
    for g in range(10):
        rows = np.arange(20 * g, 20 * g + 20)
        b = np.array([wl.instances[k].b for k in rows])
        m = np.array([len(per[k]) for k in rows], dtype=np.float64)
        for c in range(4):
            P = ref["P"][rows, c]
            pt = (P * m + 2.0) / (m + 4.0)
            s, _ = orc.sigma_from_grid(b, P, ref["dP"][rows, c])
            _, e = orc.sigma_from_grid(b, P, np.sqrt(pt * (1 - pt) / (m + 4.0)))
            comb = math.hypot(e, grid[g, Q.G_DSIGMA + c])
            z = abs(s - grid[g, Q.G_SIGMA + c]) / comb
            worst = max(worst, z)
            assert z <= 4.0, (g, c, s, grid[g, Q.G_SIGMA + c], comb)
    print("largest |z| over 40 (E_c, channel) pairs: %.2f" % worst)
    print("sigma_q by E_c:", grid[:, Q.G_SIGMA])
