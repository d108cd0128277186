"""Pins of the oracle's Lorenz-96 / RK4 / TL / AD part against facts fixed by
the mathematics (the paper defines the model in its numerical-experiments
section and uses the TL and adjoint runs in the sketching and Nystrom sections
without printing them)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O

F, DT = 8.0, 0.025


def _state(n, seed=0, spin=200):
    rng = np.random.default_rng(seed)
    x = F + rng.standard_normal(n)
    return O.rk4_run(x, F, DT, spin)


def test_fixed_point_is_exact():
    # x = F*1 is an exact equilibrium: f(F*1) = (F - F) F - F + F = 0 in exact
    # arithmetic and in IEEE arithmetic, so RK4 must return F*1 bit for bit.
    for n in (4, 5, 40, 1024):
        x = np.full(n, F)
        assert np.all(O.tendency(x, F) == 0.0)
        assert np.array_equal(O.rk4_step(x, F, DT), x)
        assert np.array_equal(O.rk4_run(x, F, DT, 1000), x)


def test_advection_conserves_energy():
    # The quadratic term of Lorenz-96 conserves sum x_i^2:
    # sum_i x_i (x_{i+1} - x_{i-2}) x_{i-1} = 0, so sum x f = -sum x^2 + F sum x.
    # A wrong index or sign in the tendency breaks this identity.
    rng = np.random.default_rng(1)
    for n in (4, 7, 40, 333):
        x = rng.standard_normal(n) * 3.0
        f = O.tendency(x, F)
        lhs = x @ f
        rhs = -(x @ x) + F * x.sum()
        assert abs(lhs - rhs) <= 1e-12 * (np.abs(x) ** 3).sum()


def test_tendency_matches_paper_form_on_small_ring():
    # n = 4 written out by hand from the ODE with the cyclic convention
    # X^(-1) = X^(n-1), X^(0) = X^(n), X^(n+1) = X^(1) (1-based):
    # dX1 = -X3 X4 + X4 X2 - X1 + F, dX2 = -X4 X1 + X1 X3 - X2 + F,
    # dX3 = -X1 X2 + X2 X4 - X3 + F, dX4 = -X2 X3 + X3 X1 - X4 + F.
    X1, X2, X3, X4 = 1.5, -2.0, 0.25, 3.0
    want = [-X3 * X4 + X4 * X2 - X1 + F, -X4 * X1 + X1 * X3 - X2 + F,
            -X1 * X2 + X2 * X4 - X3 + F, -X2 * X3 + X3 * X1 - X4 + F]
    got = O.tendency(np.array([X1, X2, X3, X4]), F)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_rk4_is_fourth_order():
    # Global error against a tight adaptive integrator (scipy DOP853) must fall
    # by ~2^4 when dt halves; a wrong RK4 weight drops the order.
    n = 40
    x0 = _state(n)

    def rhs(_, x):
        return O.tendency(x, F)

    T = 0.5
    ref = solve_ivp(rhs, (0, T), x0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for steps in (20, 40, 80):
        x = O.rk4_run(x0, F, T / steps, steps)
        errs.append(np.linalg.norm(x - ref))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.7) and np.all(orders < 4.3), orders


@pytest.mark.parametrize("n", [8, 40, 101])
def test_tl_step_central_difference(n):
    # TL against central differences of the nonlinear step: error ~ eps^2.
    rng = np.random.default_rng(n)
    x = _state(n, seed=n)
    dx = rng.standard_normal(n)
    tl = O.tl_step(x, dx, F, DT)
    errs = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        fd = (O.rk4_step(x + eps * dx, F, DT) - O.rk4_step(x - eps * dx, F, DT)) / (2 * eps)
        errs.append(np.linalg.norm(fd - tl) / np.linalg.norm(tl))
    ratio = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratio > 3.5) and np.all(ratio < 4.5), (errs, ratio)
    assert errs[-1] < 1e-5


def test_tl_window_forward_difference():
    # Over a 20-step window: one-sided differences converge linearly in eps.
    cfg = dict(n=40, nsteps=20, F=F, dt=DT, obs_dt=1, obs_dx=1, obs_x0=0, sigma_o=1.0)
    x0 = _state(40, seed=3)
    traj = O.nl_traj(cfg, x0)[None]
    dx = np.random.default_rng(3).standard_normal(40)
    g = O.G_apply(cfg, traj, [0], dx[:, None])[:, 0]
    base = O.observe(cfg, traj[0])
    errs = []
    for eps in (1e-4, 1e-5, 1e-6):
        fd = (O.observe(cfg, O.nl_traj(cfg, x0 + eps * dx)) - base) / eps
        errs.append(np.linalg.norm(fd - g) / np.linalg.norm(g))
    assert errs[0] / errs[1] > 7 and errs[1] / errs[2] > 7, errs


@pytest.mark.parametrize("n", [4, 5, 40, 257])
def test_ad_step_is_transpose(n):
    # <M dx, l> = <dx, M^T l> to rounding.
    rng = np.random.default_rng(10 + n)
    x = _state(n, seed=n)
    dx, lam = rng.standard_normal(n), rng.standard_normal(n)
    lhs = O.tl_step(x, dx, F, DT) @ lam
    rhs = dx @ O.ad_step(x, lam, F, DT)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(dx) * np.linalg.norm(lam) * 10


def test_ad_step_matrix_transpose():
    # Assemble M and M^T column by column at n = 12 and compare.
    n = 12
    x = _state(n, seed=5)
    E = np.eye(n)
    M = np.stack([O.tl_step(x, E[i], F, DT) for i in range(n)], axis=1)
    MT = np.stack([O.ad_step(x, E[i], F, DT) for i in range(n)], axis=1)
    np.testing.assert_allclose(MT, M.T, rtol=0, atol=1e-14 * np.abs(M).max())


@pytest.mark.parametrize("obs", [(5, 2, 0), (4, 3, 1), (1, 1, 0)])
def test_window_adjoint(obs):
    # <G v, w> = <v, G^T w> for the whole window with observations.
    obs_dt, obs_dx, obs_x0 = obs
    cfg = dict(n=40, nsteps=20, F=F, dt=DT, obs_dt=obs_dt, obs_dx=obs_dx, obs_x0=obs_x0, sigma_o=0.5)
    nt, nv = O.obs_counts(cfg)
    rng = np.random.default_rng(7)
    traj = np.stack([O.nl_traj(cfg, _state(40, seed=s)) for s in (1, 2)])
    V = rng.standard_normal((40, 3))
    Wm = rng.standard_normal((nt * nv, 3))
    members = [0, 1, 1]
    GV = O.G_apply(cfg, traj, members, V)
    GTW = O.GT_apply(cfg, traj, members, Wm)
    lhs = np.sum(GV * Wm, axis=0)
    rhs = np.sum(V * GTW, axis=0)
    scale = np.linalg.norm(GV, axis=0) * np.linalg.norm(Wm, axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale)


def test_observe_counts_exclude_time_zero():
    # Observation times s = obs_dt, 2 obs_dt, ..., N: 20 steps every 5 with
    # every 2nd of 40 variables gives 4 x 20 = 80 observations.
    cfg = dict(n=40, nsteps=20, obs_dt=5, obs_dx=2, obs_x0=0)
    assert O.obs_counts(cfg) == (4, 20)
    traj = np.arange(21 * 40, dtype=np.float64).reshape(21, 40)
    y = O.observe(cfg, traj)
    assert y.size == 80
    assert y[0] == traj[5, 0] and y[1] == traj[5, 2] and y[20] == traj[10, 0] and y[-1] == traj[20, 38]
