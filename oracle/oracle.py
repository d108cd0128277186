"""CPU FP64 oracle of the randomized-preconditioned EDA hot path.

TEST INFRASTRUCTURE ONLY.  A plain, slow, direct transcription of what the
paper defines, used to check the HIP library.  Only tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the library never does, and
this module imports nothing from the library.  Its model part (Lorenz-96, RK4,
TL, AD) is plain C in l96_oracle.c; the linear algebra here uses numpy / LAPACK
routines as single steps (matmul, FFT, QR, Cholesky, SVD, symmetric EVD).

Conventions.  Matrices are in math orientation (an n x l numpy array holds l
column vectors).  Member 0 is the control.  The paper's A is the low-rank part
A = U_B^T G^T R^-1 G U_B; the system matrix is I + A (incremental 4D-Var with
the control-variable transform, the "system_with_CVT" equation).

Readings taken where the paper is silent:
  * observation times exclude t = 0: s = obs_dt, 2 obs_dt, ..., <= N;
  * B = sigma_b^2 C with C the cyclic Gaussian correlation exp(-d^2 / (2 len^2)),
    d the cyclic grid distance; U_B is its symmetric square root in closed form
    (a Gaussian of length len/sqrt(2), see ub_row), and B is taken as U_B U_B,
    equal to sigma_b^2 C to within 5e-9 relative for len >= 2;
  * or (b_kind "diffusion", the paper's own kind of B, named but not defined
    there) the diffusion-based correlation g^2 (I - kappa Lap)^-M with
    kappa = D^2 / (2M - 3) and U_B = sigma_b g (I - kappa Lap)^(-M/2), see
    diffusion_ub_row;
  * control background x^b = x^t_0 + U_B xi_0; members x^b_j = x^b + U_B xi_j,
    y_j = y + sigma_o eta_j (ensemble-formulation section and experiment set-up);
  * the truth is spun up from F*1 with N(0, spin_pert_std^2) added to variable 0;
  * theta "mid" is (lambda_k(I+A) + 1)/2 with lambda_k(I+A) = 1 + d_k;
  * PCG stops on the recurrence residual ||r|| <= rtol ||b|| from x0 = 0.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nsteps", ctypes.c_int32), ("F", ctypes.c_double),
                ("dt", ctypes.c_double), ("obs_dt", ctypes.c_int32), ("obs_dx", ctypes.c_int32),
                ("obs_x0", ctypes.c_int32), ("sigma_o", ctypes.c_double)]


def lib():
    """The compiled model part; built by oracle/build.py."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            raise RuntimeError(f"{_LIBPATH} missing: run `python oracle/build.py`")
        L = ctypes.CDLL(_LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        mp = ctypes.POINTER(_Model)
        i, d = ctypes.c_int, ctypes.c_double
        for name, args in {
            "orc_l96_tendency": [i, d, dp, dp],
            "orc_rk4_step": [i, d, d, dp, dp],
            "orc_rk4_run": [i, d, d, i, dp],
            "orc_nl_traj": [mp, dp, dp],
            "orc_tl_step": [i, d, d, dp, dp, dp],
            "orc_ad_step": [i, d, d, dp, dp, dp],
            "orc_tl_window": [mp, dp, dp, dp],
            "orc_ad_window": [mp, dp, dp, dp],
            "orc_tl_window_batch": [mp, dp, i, ip, dp, dp],
            "orc_ad_window_batch": [mp, dp, i, ip, dp, dp],
            "orc_nl_traj_batch": [mp, i, dp, dp],
        }.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _model(cfg) -> _Model:
    return _Model(cfg["n"], cfg["nsteps"], cfg["F"], cfg["dt"], cfg["obs_dt"], cfg["obs_dx"],
                  cfg["obs_x0"], cfg["sigma_o"])


def obs_counts(cfg) -> tuple[int, int]:
    nt = cfg["nsteps"] // cfg["obs_dt"]
    n, x0, dx = cfg["n"], cfg["obs_x0"], cfg["obs_dx"]
    return nt, (0 if x0 >= n else (n - 1 - x0) // dx + 1)


# --------------------------------------------------------------------------
# Model (numerical-experiments section: Lorenz-96, RK4)
# --------------------------------------------------------------------------
def tendency(x: np.ndarray, F: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_l96_tendency(x.size, F, _p(x), _p(out))
    return out


def rk4_step(x, F, dt):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_rk4_step(x.size, F, dt, _p(x), _p(out))
    return out


def rk4_run(x, F, dt, nsteps):
    x = np.array(x, dtype=np.float64)
    lib().orc_rk4_run(x.size, F, dt, nsteps, _p(x))
    return x


def tl_step(x, dx, F, dt):
    x, dx = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, dx))
    out = np.empty_like(x)
    lib().orc_tl_step(x.size, F, dt, _p(x), _p(dx), _p(out))
    return out


def ad_step(x, lam, F, dt):
    x, lam = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, lam))
    out = np.empty_like(x)
    lib().orc_ad_step(x.size, F, dt, _p(x), _p(lam), _p(out))
    return out


def nl_traj(cfg, x0) -> np.ndarray:
    """(N+1) x n stored trajectory from x0."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    out = np.empty((cfg["nsteps"] + 1, cfg["n"]))
    m = _model(cfg)
    lib().orc_nl_traj(ctypes.byref(m), _p(x0), _p(out))
    return out


def observe(cfg, traj: np.ndarray) -> np.ndarray:
    """Direct observations H x at the observation times: vector of length p,
    ordered (time, variable)."""
    nt, nv = obs_counts(cfg)
    s = cfg["obs_dt"] * np.arange(1, nt + 1)
    return traj[s][:, cfg["obs_x0"]::cfg["obs_dx"]][:, :nv].reshape(-1).copy()


def G_apply(cfg, traj_all: np.ndarray, members, V: np.ndarray) -> np.ndarray:
    """Columns G_m v (TL run about member m's trajectory, observed at the
    observation times).  V: n x nb; returns p x nb."""
    nt, nv = obs_counts(cfg)
    members = np.ascontiguousarray(members, dtype=np.int32)
    Vt = np.ascontiguousarray(V.T)
    out = np.empty((Vt.shape[0], nt * nv))
    m = _model(cfg)
    lib().orc_tl_window_batch(ctypes.byref(m), _p(traj_all), Vt.shape[0],
                              members.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(Vt), _p(out))
    return out.T.copy()


def GT_apply(cfg, traj_all: np.ndarray, members, W: np.ndarray) -> np.ndarray:
    """Columns G_m^T w (AD run).  W: p x nb; returns n x nb."""
    members = np.ascontiguousarray(members, dtype=np.int32)
    Wt = np.ascontiguousarray(W.T)
    out = np.empty((Wt.shape[0], cfg["n"]))
    m = _model(cfg)
    lib().orc_ad_window_batch(ctypes.byref(m), _p(traj_all), Wt.shape[0],
                              members.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(Wt), _p(out))
    return out.T.copy()


# --------------------------------------------------------------------------
# Background-error covariance (incremental 4D-Var section; experiment set-up)
# --------------------------------------------------------------------------
def ub_row(n: int, sigma_b: float, len_b: float) -> np.ndarray:
    """First row r of U_B (U_B[i, j] = r[(i - j) mod n]).

    U_B is the symmetric square root of B = sigma_b^2 C in closed form: a cyclic
    Gaussian of length len/sqrt(2),
        r(d) = sigma_b (2/pi)^(1/4) len^(-1/2) exp(-d^2 / len^2),
    d the cyclic distance.  The lattice sum of two such Gaussians is
    exp(-d^2/(2 len^2)) (1 + O(exp(-pi^2 len^2 / 2))) (Poisson summation), so
    U_B U_B = B up to 5e-9 relative at len = 2 and to rounding at len >= 3;
    U_B is symmetric, circulant and positive definite."""
    i = np.arange(n)
    d = np.minimum(i, n - i).astype(np.float64)
    a = sigma_b * (2.0 / np.pi) ** 0.25 / np.sqrt(len_b)
    return a * np.exp(-d * d / (len_b * len_b))


def diffusion_kappa(daley: float, steps: int) -> float:
    """Diffusion coefficient of an M-step implicit diffusion correlation on a
    line with Daley length-scale D: the spectrum (1 + kappa k^2)^-M has
    -1/c''(0) = kappa (2M - 3), so kappa = D^2 / (2M - 3)."""
    return daley * daley / (2.0 * steps - 3.0)


def diffusion_ub_row(n: int, sigma_b: float, daley: float, steps: int) -> np.ndarray:
    """First row of U_B for the diffusion-based correlation of the experiments
    (B = sigma_b^2 C_B, C_B depending on a Daley length-scale D and a number M
    of diffusion steps, with U_B = U_B^T; the paper names the operator without
    defining it).  Reading: C_B = g^2 (I - kappa Lap)^-M on the ring of n
    points, Lap the second difference, kappa = D^2 / (2M - 3), g normalising
    the diagonal of C_B to one; U_B = sigma_b g (I - kappa Lap)^(-M/2), M even.

    Written from the spectrum: (I - kappa Lap) has eigenvalue
    s_m = 1 + 4 kappa sin^2(pi m / n) on the Fourier mode m, so
        g^2 = n / sum_m s_m^-M,
        r(d) = (1/n) sum_m sigma_b g s_m^(-M/2) cos(2 pi m d / n)."""
    if steps < 2 or steps % 2:
        raise ValueError("the number of diffusion steps must be even and >= 2")
    kap = diffusion_kappa(daley, steps)
    m = np.arange(n)
    s = 1.0 + 4.0 * kap * np.sin(np.pi * m / n) ** 2
    g = np.sqrt(n / np.sum(s ** (-float(steps))))
    lam = sigma_b * g * s ** (-0.5 * steps)
    half = np.cos(2.0 * np.pi * np.outer(np.arange(n // 2 + 1), m) / n) @ lam / n
    return half[np.minimum(m, n - m)]             # r(d) = r(n - d) exactly


def ub_row_for(cfg) -> np.ndarray:
    """U_B's first row for a workload: the cyclic Gaussian (default) or the
    diffusion-based operator (cfg["b_kind"] == "diffusion", Daley length-scale
    len_b, cfg["diff_steps"] steps)."""
    if cfg.get("b_kind", "gauss") == "diffusion":
        return diffusion_ub_row(cfg["n"], cfg["sigma_b"], cfg["len_b"], cfg["diff_steps"])
    return ub_row(cfg["n"], cfg["sigma_b"], cfg["len_b"])


def circulant(r: np.ndarray) -> np.ndarray:
    """The symmetric circulant matrix with first row r (M[i, j] = r[(i - j) mod n])."""
    n = r.size
    i = np.arange(n)
    return r[(i[:, None] - i[None, :]) % n]


def build_ub(n: int, sigma_b: float, len_b: float) -> np.ndarray:
    return circulant(ub_row(n, sigma_b, len_b))


# --------------------------------------------------------------------------
# EDA problem set-up (ensemble-formulation section; experiment set-up)
# --------------------------------------------------------------------------
class Problem:
    """Everything eda_setup produces for one EDA problem, in FP64."""

    def __init__(self, cfg, normals):
        self.cfg = dict(cfg)
        n, N, L = cfg["n"], cfg["nsteps"], cfg["members"]
        nt, nv = obs_counts(cfg)
        p = nt * nv
        self.p = p
        normals = np.asarray(normals, dtype=np.float64)
        z = normals[0]
        xi = normals[1:1 + (L + 1) * n].reshape(L + 1, n).T          # n x (L+1)
        eta = normals[1 + (L + 1) * n:].reshape(L + 1, p).T           # p x (L+1)
        # truth: spin-up from F*1 perturbed at variable 0, then the window run
        x = np.full(n, cfg["F"])
        x[0] = x[0] + cfg["spin_pert_std"] * z
        self.xt0 = rk4_run(x, cfg["F"], cfg["dt"], cfg["spinup"])
        self.xt_traj = nl_traj(cfg, self.xt0)
        # observations y = H x^t + sigma_o eta_0; members y_j = y + sigma_o eta_j
        y = observe(cfg, self.xt_traj) + cfg["sigma_o"] * eta[:, 0]
        Y = np.empty((p, L + 1))
        Y[:, 0] = y
        Y[:, 1:] = y[:, None] + cfg["sigma_o"] * eta[:, 1:]
        self.y = Y
        # U_B and backgrounds
        self.ub = circulant(ub_row_for(cfg))
        UX = self.ub @ xi
        xb = self.xt0 + UX[:, 0]
        XB = np.empty((n, L + 1))
        XB[:, 0] = xb
        XB[:, 1:] = xb[:, None] + UX[:, 1:]
        self.xb = XB
        # member trajectories (member-major, (L+1) x (N+1) x n)
        self.traj = np.stack([nl_traj(cfg, XB[:, j]) for j in range(L + 1)])
        # innovations d_j = y_j - H(x_j traj) and right-hand sides
        # b_j = U_B^T G_j^T R^-1 d_j
        D = np.stack([Y[:, j] - observe(cfg, self.traj[j]) for j in range(L + 1)], axis=1)
        self.d = D
        members = np.arange(L + 1)
        self.b = self.ub.T @ GT_apply(cfg, self.traj, members, D / cfg["sigma_o"] ** 2)
        # constant of the quadratic cost: c_j = 1/2 d_j^T R^-1 d_j
        self.cost_c = 0.5 * np.sum(D * D, axis=0) / cfg["sigma_o"] ** 2

    # ---- operators ----
    def A(self, X: np.ndarray, members) -> np.ndarray:
        """Columns A_m x = U_B^T G_m^T R^-1 G_m U_B x."""
        X = np.asarray(X, dtype=np.float64)
        cfg = self.cfg
        V = self.ub @ X
        W = G_apply(cfg, self.traj, members, V) / cfg["sigma_o"] ** 2
        return self.ub.T @ GT_apply(cfg, self.traj, members, W)

    def hess(self, X: np.ndarray, members) -> np.ndarray:
        """Columns (I + A_m) x."""
        return X + self.A(X, members)

    def gamma(self, ell: int) -> np.ndarray:
        """RHS-difference sketch Gamma = [b_1 - b_0, ..., b_ell - b_0]
        (sketch from the EDA structure, the Gamma equation)."""
        return self.b[:, 1:ell + 1] - self.b[:, [0]]

    def cost(self, m: int, dz: np.ndarray) -> np.ndarray:
        """Quadratic cost J(dx) of the incremental problem with dx = U_B dz,
        written in the control variable: 1/2 dz^T dz + 1/2 ||G U_B dz - d||^2_R^-1."""
        cfg = self.cfg
        Gv = G_apply(cfg, self.traj, [m] * dz.shape[1], self.ub @ dz)
        res = Gv - self.d[:, [m]]
        return 0.5 * np.sum(dz * dz, axis=0) + 0.5 * np.sum(res * res, axis=0) / cfg["sigma_o"] ** 2


# --------------------------------------------------------------------------
# Randomized low-rank approximation (the q-pass Nystrom algorithm; REVD)
# --------------------------------------------------------------------------
def qr_pos(Y: np.ndarray):
    """Economic QR with a positive diagonal of R (unique for full-rank Y)."""
    Q, R = np.linalg.qr(Y)
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s, R * s[:, None]


def fix_signs(S: np.ndarray) -> np.ndarray:
    """Sign convention for eigenvector columns: the entry of largest magnitude
    (lowest index on ties) is positive."""
    idx = np.argmax(np.abs(S), axis=0)
    s = np.where(S[idx, np.arange(S.shape[1])] < 0, -1.0, 1.0)
    return S * s


def _range_sketch(Aop, Phi: np.ndarray, passes: int):
    """Sketch of A's range with `passes` products: Y = A Phi, and each further
    pass replaces Phi by the orthonormal basis of the previous Y (subspace
    iteration).  Returns the Phi of the last product, that Y, and Y = Q R with
    positive diag(R)."""
    Y = Aop(Phi)
    Q, R = qr_pos(Y)
    for _ in range(passes - 1):
        Phi = Q
        Y = Aop(Phi)
        Q, R = qr_pos(Y)
    return Phi, Y, Q, R


def _nystrom_factors(Phi: np.ndarray, Y: np.ndarray, Q: np.ndarray, R: np.ndarray):
    """Ritz pairs of A_N = Y (Phi^T Y)^-1 Y^T (the nystrom_approx equation).

    With Phi^T Y = L L^T (Cholesky; raises LinAlgError when the core is not
    numerically positive definite) and Y = Q R,  A_N = (Q F)(Q F)^T with
    F = R L^-T, so the SVD F = U diag(sig) V^T gives A_N = (Q U) diag(sig^2)
    (Q U)^T.  Returns (S = Q U with the sign convention, sig^2 descending,
    the 2-norm condition number of the core)."""
    core = Phi.T @ Y
    core = 0.5 * (core + core.T)
    Lc = np.linalg.cholesky(core)
    F = np.linalg.solve(Lc, R.T).T               # R L^-T
    U, sig, _ = np.linalg.svd(F)
    return fix_signs(Q @ U), sig * sig, float(np.linalg.cond(core))


def nystrom(Aop, Phi: np.ndarray, k: int, q: int = 1, eps: float = float(np.finfo(np.float64).eps)):
    """Randomized Nystrom approximation of a symmetric positive semidefinite A
    given through Aop(X) = A X, with q products (the paper's Algorithm 1).

    Returns (S_k, D_k, info): S_k n x k with orthonormal columns, D_k the k
    largest approximate eigenvalues (descending); info["shift"] is the shift
    nu used (0 when none was needed) and info["cond_core"] the condition
    number of the Cholesky core Phi^T A Phi.  When the core is not positive
    definite in floating point, the shifted approximation of the Nystrom
    appendix is taken instead: Y + nu Phi with nu = eps ||Y||_F (eps the unit
    roundoff of the products), whose eigenvalues are then lowered by nu.
    """
    Phi, Y, Q, R = _range_sketch(Aop, Phi, q)
    nu = 0.0
    try:
        S, D, cond = _nystrom_factors(Phi, Y, Q, R)
    except np.linalg.LinAlgError:
        nu = eps * np.linalg.norm(Y)
        Ys = Y + nu * Phi
        Qs, Rs = qr_pos(Ys)
        S, D, cond = _nystrom_factors(Phi, Ys, Qs, Rs)
        D = np.maximum(D - nu, 0.0)
    return S[:, :k], D[:k], {"shift": nu, "cond_core": cond}


def revd(Aop, Phi: np.ndarray, k: int):
    """Two-stage randomized EVD with a Rayleigh-Ritz projection (randomized
    eigendecomposition subsection): Q = orth(A Phi), T = Q^T A Q, T = V L V^T,
    S = Q V.  Returns (S_k, D_k)."""
    Q, _ = qr_pos(Aop(Phi))
    Z = Aop(Q)
    T = Q.T @ Z
    T = 0.5 * (T + T.T)
    lam, V = np.linalg.eigh(T)
    order = np.argsort(-lam, kind="stable")
    S = fix_signs(Q @ V[:, order])
    return S[:, :k], lam[order][:k]


def theta(D: np.ndarray, rule: str = "mid") -> float:
    """Scaling of the spectral LMP (spectral LMP subsection; sensitivity study):
    'mid' (lambda_k(I+A) + 1)/2, 'lamk' lambda_k(I+A), 'one' 1, with
    lambda_k(I+A) = 1 + d_k."""
    lk = 1.0 + float(D[-1])
    return {"mid": 0.5 * (lk + 1.0), "lamk": lk, "one": 1.0}[rule]


def lmp_apply(S: np.ndarray, D: np.ndarray, th: float, X: np.ndarray, which: str = "P") -> np.ndarray:
    """P_theta X = X + S (theta (D + I)^-1 - I) S^T X, or the symmetric factor
    U_theta X = X + S (sqrt(theta) (D + I)^-1/2 - I) S^T X (the lmp equation)."""
    if which == "P":
        c = th / (1.0 + D) - 1.0
    else:
        c = np.sqrt(th) / np.sqrt(1.0 + D) - 1.0
    return X + S @ (c[:, None] * (S.T @ X))


# --------------------------------------------------------------------------
# Preconditioned conjugate gradients (solving-linear-systems section)
# --------------------------------------------------------------------------
CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def pcg(Hop, b: np.ndarray, Pop=None, rtol: float = 1e-6, maxit: int = 1000):
    """PCG on (I + A) x = b from x0 = 0 with preconditioner Pop (None: identity).

    Textbook recurrences: r = b, z = P r, p = z, rho = r^T z; per iteration
    q = H p, alpha = rho / p^T q, x += alpha p, r -= alpha q, stop if
    ||r|| <= rtol ||b||, z = P r, rho' = r^T z, p = z + (rho'/rho) p.
    Breakdown (p^T q <= 0, rho' <= 0, or a non-finite value) stops with status 2.
    Also returns the quadratic-cost history J_i - c = -1/2 x_i^T (b + r_i),
    i = 0..iters (c the constant 1/2 d^T R^-1 d).
    """
    P = (lambda v: v) if Pop is None else Pop
    x = np.zeros_like(b)
    r = b.copy()
    z = P(r)
    p = z.copy()
    rho = float(r @ z)
    bnorm = float(np.sqrt(b @ b))
    hist = [0.0]
    status, it = NOT_CONVERGED, 0
    if bnorm == 0.0:
        return x, 0, 0.0, CONVERGED, np.array(hist)
    for it in range(1, maxit + 1):
        q = Hop(p)
        pq = float(p @ q)
        if not (pq > 0.0) or not np.isfinite(pq):
            status, it = BREAKDOWN, it - 1
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        hist.append(-0.5 * float(x @ (b + r)))
        rn = float(np.sqrt(r @ r))
        if rn <= rtol * bnorm:
            status = CONVERGED
            break
        z = P(r)
        rho_new = float(r @ z)
        if not (rho_new > 0.0) or not np.isfinite(rho_new):
            status = BREAKDOWN
            break
        p = z + (rho_new / rho) * p
        rho = rho_new
    relres = float(np.sqrt(r @ r)) / bnorm
    return x, it, relres, status, np.array(hist)


def exact_solution(prob: Problem, m: int) -> np.ndarray:
    """The plain definition of a member's result: the exact solution of
    (I + A_m) dz = b_m, by assembling I + A_m column by column and a Cholesky
    solve."""
    n = prob.cfg["n"]
    H = prob.hess(np.eye(n), [m] * n)
    H = 0.5 * (H + H.T)
    Lc = np.linalg.cholesky(H)
    return np.linalg.solve(Lc.T, np.linalg.solve(Lc, prob.b[:, m]))
