"""Pins of the oracle's covariance, Hessian, right-hand sides, randomized
low-rank approximation, spectral LMP and PCG against what the paper and the
mathematics fix (closed forms, invariants, brute force at tiny sizes)."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


@pytest.fixture(scope="module")
def c1():
    cfg = W.config("C1")
    return O.Problem(cfg, W.problem_normals(cfg))


def _small_cfg(**over):
    # n = 40 with few observations (p = 2 x 5 = 10 < n) so that rank(A) <= p.
    return W.config("C1", obs_dt=10, obs_dx=8, **over)


# ---------------------------------------------------------------- U_B ------
@pytest.mark.parametrize("n,len_b", [(40, 2.0), (64, 4.0), (128, 8.0), (1024, 8.0), (48, 3.0)])
def test_ub_is_symmetric_sqrt_of_b(n, len_b):
    # U_B U_B must reproduce B = sigma_b^2 exp(-d^2/(2 len^2)) (cyclic Gaussian
    # correlation of the experiment set-up), with U_B symmetric, circulant and
    # PSD -- that characterises the unique PSD square root.  It is also compared
    # with the root computed by a dense symmetric eigensolver (LAPACK) where B is
    # well conditioned.
    sb = 1.3
    U = O.build_ub(n, sb, len_b)
    i = np.arange(n)
    d = np.minimum(np.abs(i[:, None] - i[None, :]), n - np.abs(i[:, None] - i[None, :]))
    B = sb ** 2 * np.exp(-d ** 2 / (2 * len_b ** 2))
    assert np.array_equal(U, U.T)
    assert np.array_equal(U[1:, 1:], U[:-1, :-1])
    tol = 6e-9 if len_b < 3 else 1e-13
    np.testing.assert_allclose(U @ U, B, rtol=0, atol=tol * sb ** 2)
    assert np.linalg.eigvalsh(U).min() > -1e-14
    if n <= 64:
        lam, V = np.linalg.eigh(B)
        if lam.min() > 1e-6:
            root = (V * np.sqrt(lam)) @ V.T
            np.testing.assert_allclose(U, root, rtol=0, atol=1e-6 * np.abs(root).max())


@pytest.mark.parametrize("n,D,M", [(1500, 6.0, 10), (300, 6.0, 2), (256, 12.0, 4), (64, 3.0, 10)])
def test_diffusion_ub_real_space_and_normalisation(n, D, M):
    # The diffusion-based U_B (reading of the experiments' C_B) is written from
    # its spectrum.  In real space, M/2 implicit diffusion steps, i.e. M/2
    # applications of the tridiagonal (1 + 2 kappa) I - kappa (shift + shift^T),
    # must turn U_B into a multiple of the identity; B = U_B U_B must have unit
    # correlations on its diagonal (times sigma_b^2); U_B is symmetric,
    # circulant and positive definite.
    sb = 0.8
    U = O.circulant(O.diffusion_ub_row(n, sb, D, M))
    assert np.array_equal(U, U.T)
    assert np.array_equal(U[1:, 1:], U[:-1, :-1])
    assert np.linalg.eigvalsh(U).min() > 0
    B = U @ U
    np.testing.assert_allclose(np.diag(B), sb ** 2, rtol=1e-13)
    kap = O.diffusion_kappa(D, M)
    T = (1 + 2 * kap) * np.eye(n) - kap * (np.roll(np.eye(n), 1, axis=0) + np.roll(np.eye(n), -1, axis=0))
    X = U.copy()
    for _ in range(M // 2):
        X = T @ X
    # rounding in U_B is amplified by ||T||^(M/2) <= (1 + 4 kappa)^(M/2)
    tol = 64 * np.finfo(float).eps * (1 + 4 * kap) ** (M // 2)
    assert X[0, 0] > 0
    assert np.abs(X - X[0, 0] * np.eye(n)).max() <= tol * X[0, 0]


def test_diffusion_daley_length_and_heat_kernel_limit():
    # kappa = D^2 / (2M - 3) makes D the Daley length-scale, -1/c''(0) = D^2, of
    # the correlation c; on the grid the second difference at 0 gives it to
    # O(1/D^2).  As M grows at fixed D the spectrum (1 + 4 kappa sin^2(t/2))^-M
    # tends to exp(-D^2 (1 - cos t)), whose lattice kernel is the discrete heat
    # kernel: c(d) -> I_d(D^2) / I_0(D^2) (modified Bessel functions), with an
    # O(1/M) difference.
    from scipy.special import ive
    for n, D, M in ((1500, 6.0, 10), (1000, 20.0, 10)):
        U = O.circulant(O.diffusion_ub_row(n, 1.0, D, M))
        c = (U @ U)[0]
        d_est = np.sqrt(1.0 / (2.0 * (1.0 - c[1] / c[0])))
        assert abs(d_est - D) < 0.01 * D, (D, d_est)
    n, D = 800, 8.0
    i = np.arange(n)
    heat = ive(np.minimum(i, n - i), D * D) / ive(0, D * D)
    errs = []
    for M in (400, 2000):
        U = O.circulant(O.diffusion_ub_row(n, 1.0, D, M))
        errs.append(np.abs((U @ U)[0] - heat).max())
    assert errs[1] < 2e-4 and errs[1] < errs[0] / 4, errs


def test_diffusion_problem_hessian():
    # The paper's set-up with the diffusion B at reduced size: the Hessian is
    # symmetric, I + A >= I, and rank(A) <= p.
    cfg = W.config("paper", n=120, obs_dx=6, members=2, spinup=200)
    P = O.Problem(cfg, W.problem_normals(cfg))
    assert P.p == 60
    A = P.A(np.eye(120), [0] * 120)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam.min() > -1e-10 * lam.max()
    assert np.sum(lam > 1e-9 * lam.max()) <= P.p


def test_fix_signs_convention():
    # Eigenvector sign reading: the entry of largest magnitude of each column is
    # made positive, the lowest index winning a tie in magnitude.
    S = np.array([[0.1, 0.5, -0.5, 0.0],
                  [-0.9, -0.5, 0.5, 0.0],
                  [0.2, 0.3, 0.1, -1.0]])
    F = O.fix_signs(S)
    want = np.array([[-0.1, 0.5, 0.5, 0.0],
                     [0.9, -0.5, -0.5, 0.0],
                     [-0.2, 0.3, -0.1, 1.0]])
    assert np.array_equal(F, want)
    # idempotent, and a column and its negative map to the same column
    assert np.array_equal(O.fix_signs(F), F)
    assert np.array_equal(O.fix_signs(-S), F)


# ------------------------------------------------------------ Hessian ------
def test_hessian_symmetric_and_above_identity(c1):
    n = c1.cfg["n"]
    for m in (0, 3):
        H = c1.hess(np.eye(n), [m] * n)
        assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
        lam = np.linalg.eigvalsh(0.5 * (H + H.T))
        assert lam.min() >= 1 - 1e-12


def test_hessian_equals_assembled_tl_form(c1):
    # A = U_B^T G^T R^-1 G U_B with G assembled column by column from TL runs
    # only (the hessvec uses the adjoint run for G^T).
    cfg, n = c1.cfg, c1.cfg["n"]
    for m in (0, 7):
        G = O.G_apply(cfg, c1.traj, [m] * n, np.eye(n))
        A_tl = c1.ub.T @ G.T @ G @ c1.ub / cfg["sigma_o"] ** 2
        A = c1.A(np.eye(n), [m] * n)
        np.testing.assert_allclose(A, A_tl, rtol=0, atol=1e-12 * np.abs(A_tl).max())
        # and the right-hand side b = U_B^T G^T R^-1 d
        b_tl = c1.ub.T @ G.T @ c1.d[:, m] / cfg["sigma_o"] ** 2
        np.testing.assert_allclose(c1.b[:, m], b_tl, rtol=0, atol=1e-12 * np.abs(b_tl).max())


def test_rank_bounded_by_observations():
    # I + A has eigenvalue 1 with multiplicity >= n - p (system_with_CVT
    # discussion): with p = 10 < n = 40, A has rank <= 10.
    cfg = _small_cfg()
    P = O.Problem(cfg, W.problem_normals(cfg))
    assert P.p == 10
    lam = np.linalg.eigvalsh(P.A(np.eye(40), [0] * 40))
    assert np.sum(lam > 1e-10 * lam.max()) <= 10
    assert lam.min() > -1e-12 * lam.max()


def test_gamma_linear_limit():
    # Sketch from the EDA structure: with d_0 = 0 (truth = control background,
    # no truth obs error) and perturbations scaled by eps, the RHS difference is
    # gamma_j = eps (U_B^T G^T R^-1 (U_R eta_j - G U_B xi_j)) + O(eps^2), the
    # first-order relation behind cov(gamma) = A + A^2.
    cfg = W.config("C1", members=3)
    z = W.problem_normals(cfg)
    n, p, L = 40, 80, 3
    base = z.copy()
    base[1:1 + n] = 0.0                      # xi_0 = 0
    base[1 + (L + 1) * n:1 + (L + 1) * n + p] = 0.0   # eta_0 = 0
    P0 = O.Problem(cfg, base)
    lin = None
    errs = []
    for eps in (1e-4, 1e-5):
        zz = base.copy()
        zz[1 + n:1 + (L + 1) * n] *= eps
        zz[1 + (L + 1) * n + p:] *= eps
        P = O.Problem(cfg, zz)
        assert np.abs(P.d[:, 0]).max() < 1e-12
        g = P.gamma(L) / eps
        if lin is None:
            xi = base[1 + n:1 + (L + 1) * n].reshape(L, n).T
            eta = base[1 + (L + 1) * n + p:].reshape(L, p).T
            so = cfg["sigma_o"]
            lin = (P0.ub.T @ O.GT_apply(cfg, P0.traj, [0] * L, (so * eta) / so ** 2)
                   - P0.A(xi, [0] * L))
        errs.append(np.linalg.norm(g - lin) / np.linalg.norm(lin))
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 5, errs


@pytest.mark.slow
def test_gamma_covariance_is_A_plus_A2(c1):
    # cov(gamma) = A + A^2 in the linear surrogate (the covariance equation of
    # the EDA-structure subsection), Monte Carlo with 20000 draws at n = 40.
    cfg, n, p = c1.cfg, 40, c1.p
    rng = np.random.default_rng(0)
    draws = 20000
    so = cfg["sigma_o"]
    xi = rng.standard_normal((n, draws))
    eta = rng.standard_normal((p, draws))
    G = O.G_apply(cfg, c1.traj, [0] * n, np.eye(n))
    gam = c1.ub.T @ G.T @ (so * eta - G @ c1.ub @ xi) / so ** 2
    A = c1.A(np.eye(n), [0] * n)
    A = 0.5 * (A + A.T)
    cov = gam @ gam.T / draws
    target = A + A @ A
    err = np.linalg.norm(cov - target) / np.linalg.norm(target)
    assert err < 5 / np.sqrt(draws) * 3, err


# ------------------------------------------------------------ Nystrom ------
def _spd_lowrank(n, r, seed=0, decay=0.7):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    lam = 100.0 * decay ** np.arange(r)
    return (Q * lam) @ Q.T, Q, lam


def test_nystrom_recovers_rank_k_exactly():
    # If rank(A) = r <= ell, range(A Phi) = range(A) and A_N = A (Nystrom
    # subsection: exact when the sketch spans the dominant eigenspace).
    A, Q, lam = _spd_lowrank(60, 8)
    Phi = np.random.default_rng(1).standard_normal((60, 10))
    S, D, _ = O.nystrom(lambda X: A @ X, Phi, 8)
    np.testing.assert_allclose(D, lam, rtol=1e-12)
    np.testing.assert_allclose(S @ np.diag(D) @ S.T, A, atol=1e-11 * lam[0])


def test_nystrom_with_exact_eigenvectors():
    A, Q, lam = _spd_lowrank(50, 20, seed=3, decay=0.8)
    S, D, _ = O.nystrom(lambda X: A @ X, Q[:, :6], 6)
    np.testing.assert_allclose(D, lam[:6], rtol=1e-12)
    np.testing.assert_allclose(np.abs(S.T @ Q[:, :6]), np.eye(6), atol=1e-10)


def test_nystrom_matches_pseudoinverse_definition(c1):
    # Algorithm 1 with k = ell reproduces A_N = A Phi (Phi^T A Phi)^+ (A Phi)^T
    # (the nystrom_approx equation) evaluated with a pseudoinverse.
    Aop = lambda X: c1.A(X, [0] * X.shape[1])
    Phi = c1.gamma(10)
    S, D, info = O.nystrom(Aop, Phi, 10)
    assert info["shift"] == 0.0
    Y = Aop(Phi)
    AN = Y @ np.linalg.pinv(Phi.T @ Y) @ Y.T
    np.testing.assert_allclose(S @ np.diag(D) @ S.T, AN, atol=1e-9 * np.abs(AN).max())
    np.testing.assert_allclose(S.T @ S, np.eye(10), atol=1e-12)


def test_nystrom_eigs_below_true_and_range_invariant(c1):
    # A_N <= A (Loewner), so d_i <= lambda_i(A); A_N depends on range(Phi) only.
    n = 40
    Aop = lambda X: c1.A(X, [0] * X.shape[1])
    lam = np.sort(np.linalg.eigvalsh(Aop(np.eye(n))))[::-1]
    Phi = c1.gamma(10)
    S, D, _ = O.nystrom(Aop, Phi, 10)
    assert np.all(D <= lam[:10] * (1 + 1e-10))
    M = np.random.default_rng(5).standard_normal((10, 10)) + 4 * np.eye(10)
    S2, D2, _ = O.nystrom(Aop, Phi @ M, 10)
    np.testing.assert_allclose(D2, D, rtol=1e-9)
    np.testing.assert_allclose(S2 @ np.diag(D2) @ S2.T, S @ np.diag(D) @ S.T, atol=1e-8 * D[0])


def test_nystrom_shift_fallback():
    # A sketch column in the exact null space of A makes Phi^T A Phi singular
    # (a zero pivot), the Cholesky breaks down and the shift of the
    # Nystrom-variants appendix (Y + nu Phi, nu = eps ||Y||_F) is used; the
    # rank-5 spectrum is still recovered.
    n = 30
    lam = 100.0 * 0.7 ** np.arange(5)
    A = np.diag(np.concatenate([lam, np.zeros(n - 5)]))
    Phi = np.zeros((n, 7))
    Phi[:5, :5] = np.random.default_rng(2).standard_normal((5, 5)) + 3 * np.eye(5)
    Phi[5, 5] = 1.0
    Phi[6, 6] = 1.0
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(Phi.T @ A @ Phi)
    S, D, info = O.nystrom(lambda X: A @ X, Phi, 5)
    assert info["shift"] > 0
    np.testing.assert_allclose(D, lam, rtol=1e-10)
    np.testing.assert_allclose(np.abs(S[:5, :]), np.eye(5), atol=1e-8)


def test_power_pass_improves_eigs(c1):
    Aop = lambda X: c1.A(X, [0] * X.shape[1])
    lam = np.sort(np.linalg.eigvalsh(Aop(np.eye(40))))[::-1]
    Psi = W.gaussian_matrix(c1.cfg, 40, 10).T
    _, D1, _ = O.nystrom(Aop, Psi, 10, q=1)
    _, D2, _ = O.nystrom(Aop, Psi, 10, q=3)
    e1 = np.abs(D1 - lam[:10]) / lam[:10]
    e2 = np.abs(D2 - lam[:10]) / lam[:10]
    assert e2.sum() < e1.sum()


def test_revd_recovers_rank_k_and_rayleigh_ritz():
    A, Q, lam = _spd_lowrank(60, 8, seed=4)
    Phi = np.random.default_rng(4).standard_normal((60, 12))
    S, D = O.revd(lambda X: A @ X, Phi, 8)
    np.testing.assert_allclose(D, lam, rtol=1e-11)
    # general case: S D S^T = Q Q^T A Q Q^T with Q an orthonormal basis of range(A Phi)
    B = A + np.diag(np.linspace(0, 1, 60))
    S, D = O.revd(lambda X: B @ X, Phi, 12)
    Qb, _ = np.linalg.qr(B @ Phi)
    np.testing.assert_allclose(S @ np.diag(D) @ S.T, Qb @ Qb.T @ B @ Qb @ Qb.T, atol=1e-11 * lam[0])


def test_theta_rules():
    D = np.array([50.0, 9.0, 3.0])
    assert O.theta(D, "mid") == (4.0 + 1.0) / 2
    assert O.theta(D, "lamk") == 4.0
    assert O.theta(D, "one") == 1.0


# ---------------------------------------------------------------- LMP ------
def test_lmp_moves_captured_eigenvalues_to_theta():
    # Spectral LMP subsection: with exact eigenpairs (S_k, Lambda_k) of A,
    # P_theta (I + A) s_i = theta s_i, P_theta v = v for v orthogonal to S_k,
    # P_theta = U_theta U_theta, and U_theta (I + A) U_theta has the k captured
    # eigenvalues at theta and the rest unchanged.
    n, k = 30, 5
    A, Q, lam = _spd_lowrank(n, 12, seed=6)
    H = np.eye(n) + A
    S, D = Q[:, :k], lam[:k]
    for th in (1.0, 2.5, 0.5 * (1 + D[-1] + 1)):
        PH = O.lmp_apply(S, D, th, H)
        np.testing.assert_allclose(PH @ S, th * S, atol=1e-11 * lam[0])
        v = np.random.default_rng(1).standard_normal(n)
        v -= S @ (S.T @ v)
        np.testing.assert_allclose(O.lmp_apply(S, D, th, v[:, None])[:, 0], v, atol=1e-14)
        P = O.lmp_apply(S, D, th, np.eye(n))
        U = O.lmp_apply(S, D, th, np.eye(n), which="U")
        np.testing.assert_allclose(U @ U, P, atol=1e-13)
        ev = np.sort(np.linalg.eigvalsh(U @ H @ U))
        want = np.sort(np.concatenate([np.full(k, th), 1 + lam[k:], np.ones(n - 12)]))
        np.testing.assert_allclose(ev, want, atol=1e-10 * lam[0])


# ---------------------------------------------------------------- PCG ------
def test_pcg_matches_dense_cholesky_solve(c1):
    for m in (0, 4):
        x, it, rr, st, _ = O.pcg(lambda v: c1.hess(v[:, None], [m])[:, 0], c1.b[:, m], None, 1e-14, 500)
        assert st == O.CONVERGED
        xe = O.exact_solution(c1, m)
        assert np.linalg.norm(x - xe) <= 1e-11 * np.linalg.norm(xe)


def test_cg_finite_termination_low_rank():
    # I + A has at most p + 1 distinct eigenvalues (p = 10), so CG converges in
    # at most p + 1 iterations in exact arithmetic.
    cfg = _small_cfg()
    P = O.Problem(cfg, W.problem_normals(cfg))
    x, it, rr, st, _ = O.pcg(lambda v: P.hess(v[:, None], [0])[:, 0], P.b[:, 0], None, 1e-10, 100)
    assert st == O.CONVERGED and it <= P.p + 1, it


def test_exact_full_lmp_theta_one_converges_in_one_iteration(c1):
    # With all nonzero eigenpairs of A and theta = 1, P_theta = (I + A)^-1.
    Aop = lambda X: c1.A(X, [0] * X.shape[1])
    lam, V = np.linalg.eigh(Aop(np.eye(40)))
    keep = lam > 1e-9 * lam.max()
    S, D = V[:, keep][:, ::-1], lam[keep][::-1]
    Pop = lambda v: O.lmp_apply(S, D, 1.0, v[:, None])[:, 0]
    x, it, rr, st, _ = O.pcg(lambda v: c1.hess(v[:, None], [0])[:, 0], c1.b[:, 0], Pop, 1e-8, 50)
    assert st == O.CONVERGED and it == 1, (it, rr)


def test_cost_history_decreasing_and_equals_direct_cost(c1):
    # CG decreases the quadratic cost at every iteration (solving-linear-systems
    # section); the history -1/2 x^T (b + r) equals J - c evaluated directly
    # from the cost function (quadratic_cost_function) in the control variable.
    m = 2
    Hop = lambda v: c1.hess(v[:, None], [m])[:, 0]
    S, D, _ = O.nystrom(lambda X: c1.A(X, [0] * X.shape[1]), c1.gamma(10), 10)
    th = O.theta(D)
    Pop = lambda v: O.lmp_apply(S, D, th, v[:, None])[:, 0]
    for pre in (None, Pop):
        xs = []
        hist = None
        for it_max in range(1, 9):
            x, it, rr, st, hist = O.pcg(Hop, c1.b[:, m], pre, 0.0, it_max)
            xs.append(x)
        assert np.all(np.diff(hist) < 0)
        direct = c1.cost(m, np.stack(xs, axis=1)) - c1.cost_c[m]
        np.testing.assert_allclose(hist[1:], direct, rtol=1e-9, atol=1e-9 * abs(hist[-1]))


def test_lmp_accelerates_control_and_members(c1):
    # The paper's qualitative result: the Gamma-built LMP reduces PCG iterations
    # for the control and for perturbed members (ensemble-members results).
    S, D, _ = O.nystrom(lambda X: c1.A(X, [0] * X.shape[1]), c1.gamma(10), 10)
    th = O.theta(D)
    Pop = lambda v: O.lmp_apply(S, D, th, v[:, None])[:, 0]
    for m in (0, 1, 2, 3):
        Hop = lambda v: c1.hess(v[:, None], [m])[:, 0]
        _, it0, _, _, _ = O.pcg(Hop, c1.b[:, m], None, 1e-6, 500)
        _, it1, _, _, _ = O.pcg(Hop, c1.b[:, m], Pop, 1e-6, 500)
        assert it1 < it0, (m, it0, it1)
