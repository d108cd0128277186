"""GPU parity: every C-ABI call of libeda.so against the CPU oracle on the same
seeded inputs.  Tolerances: bit-exact for the truth trajectory (integer-free
but fixed-order FP64 arithmetic) and for seeded indexing; 1e-12 relative for
FP64 operator results; looser, stated bounds where an iterative method or a
reduced precision is involved (each justified inline)."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_23571_amd import eda  # noqa: E402

CASES = {
    # the n = 40 preset, one ring in a single wave
    "C1": W.config("C1"),
    # ragged ring sizes for 1, 4 and 8 points per thread, unusual observation patterns
    "n203": W.config("C1", n=203, nsteps=15, obs_dt=4, obs_dx=3, obs_x0=1, members=6, ell=5, k=5, len_b=3.0,
                     spinup=300),
    "n1001": W.config("C2", n=1001, nsteps=12, obs_dt=3, obs_dx=2, obs_x0=1, members=5, ell=4, k=4, spinup=200),
    "n2049": W.config("C3", n=2049, nsteps=8, obs_dt=4, obs_dx=5, obs_x0=2, members=3, ell=3, k=3, spinup=100),
}

_cache = {}


def problem(case, mode="banded"):
    key = (case, mode)
    if key not in _cache:
        cfg = CASES[case] if isinstance(case, str) else case
        z = W.problem_normals(cfg)
        print(f"[setup] case={case} mode={mode} n={cfg['n']} L={cfg['members']}", flush=True)
        g = eda.Problem(cfg, z, ub_mode=mode)
        o = _cache.get((case, "oracle"))
        if o is None:
            o = O.Problem(cfg, z)
            _cache[(case, "oracle")] = o
        _cache[key] = (cfg, g, o)
    return _cache[key]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def colrel(A, B):
    """Largest element-wise difference of a column, relative to that column's
    largest magnitude, maximised over the columns (element-wise bar)."""
    A, B = np.atleast_2d(A), np.atleast_2d(B)
    return np.max(np.abs(A - B).max(axis=0) / np.abs(B).max(axis=0))


def elrel(a, b):
    """max_i |a_i - b_i| / max_i |b_i| for vectors."""
    return float(np.abs(a - b).max() / np.abs(b).max())


_exact = {}


def exact(name, o, m):
    """The oracle's exact solution of (I + A_m) dz = b_m (dense assembly and
    Cholesky solve), cached per workload and member."""
    key = (name, m)
    if key not in _exact:
        _exact[key] = O.exact_solution(o, m)
    return _exact[key]


def eig_bars(D, cond_core, c=16.0):
    """Per-eigenvalue relative bars for Nystrom eigenvalues computed by two
    correct FP64 implementations: the Cholesky factor of the core
    Phi^T A Phi carries relative error ~ cond * eps, which moves singular value
    i of T = R C^-1 by ~ cond * eps * sigma_1, i.e. eigenvalue d_i = sigma_i^2
    by ~ 2 cond eps sqrt(d_1 / d_i) relative; c is the safety factor, and the
    floor 1e-13 covers well-conditioned cores."""
    eps = np.finfo(float).eps
    return np.maximum(1e-13, c * 2 * cond_core * eps * np.sqrt(D[0] / D))


def to_np_cols(t, n):
    """[cols, n] tensor -> n x cols numpy."""
    return t.detach().cpu().numpy().reshape(-1, n).T


# ------------------------------------------------------------------ set-up --
@pytest.mark.parametrize("mode", ["banded", "dense"])
@pytest.mark.parametrize("case", list(CASES))
def test_setup_parity(case, mode):
    cfg, g, o = problem(case, mode)
    n, L, N = cfg["n"], cfg["members"], cfg["nsteps"]
    truth = g.field("truth").cpu().numpy().reshape(N + 1, n)
    # the truth follows a chaotic spin-up: only identical arithmetic reproduces it
    assert np.array_equal(truth, o.xt_traj)
    np.testing.assert_allclose(g.field("ubrow").cpu().numpy(), O.ub_row(n, cfg["sigma_b"], cfg["len_b"]),
                               rtol=4e-16, atol=0)
    assert rel(to_np_cols(g.field("xb"), n), o.xb) < 1e-14
    traj = g.field("traj").cpu().numpy().reshape(L + 1, N + 1, n)
    assert rel(traj, o.traj) < 1e-13
    p = o.p
    assert rel(g.field("y").cpu().numpy().reshape(L + 1, p).T, o.y) < 1e-15
    assert rel(g.field("d").cpu().numpy().reshape(L + 1, p).T, o.d) < 1e-12
    b = to_np_cols(g.field("b"), n)
    assert colrel(b, o.b) < 1e-12
    np.testing.assert_allclose(g.field("costc").cpu().numpy(), o.cost_c, rtol=1e-12)


# ---------------------------------------------------------------- hessvec --
@pytest.mark.parametrize("mode", ["banded", "dense"])
@pytest.mark.parametrize("case", list(CASES))
def test_hessvec_member_and_sketch_mode(case, mode):
    cfg, g, o = problem(case, mode)
    n, L = cfg["n"], cfg["members"]
    rng = np.random.default_rng(11)
    X = rng.standard_normal((L + 1, n))
    members = np.arange(L + 1)[::-1].copy()
    Xt = torch.from_numpy(X).cuda()
    YA = to_np_cols(g.hessvec(members, Xt), n)
    YH = to_np_cols(g.hessvec(members, Xt, add_identity=True), n)
    assert colrel(YA, o.A(X.T, members)) < 1e-12
    assert colrel(YH, o.hess(X.T, members)) < 1e-12
    # sketch mode: every column on the control trajectory, width 2 ell
    ell = cfg["ell"]
    Xs = rng.standard_normal((2 * ell, n))
    Ys = to_np_cols(g.hessvec(np.zeros(2 * ell, dtype=np.int32), torch.from_numpy(Xs).cuda()), n)
    assert colrel(Ys, o.A(Xs.T, [0] * (2 * ell))) < 1e-12


@pytest.mark.parametrize("case", ["C1", "n1001"])
def test_hessvec_mixed_precision_bound(case):
    # FP32 TL/AD runs: the error against the FP64 oracle is that of single
    # precision amplified by the window's growth, stated bound 1e-4; it must also
    # be clearly non-zero (the reduced path really ran).
    cfg, g, o = problem(case)
    n = cfg["n"]
    X = np.random.default_rng(3).standard_normal((cfg["ell"], n))
    Y = to_np_cols(g.hessvec(np.zeros(cfg["ell"], dtype=np.int32), torch.from_numpy(X).cuda(), mixed=True), n)
    err = colrel(Y, o.A(X.T, [0] * cfg["ell"]))
    assert 1e-10 < err < 1e-4, err


@pytest.mark.parametrize("case", ["C1", "n1001"])
def test_hessvec_mixed_dense_bf16_bound(case):
    # Dense U_B with EDA_HV_BF16: both U_B products take BF16 operands (unit
    # roundoff 2^-9 each) with FP32 accumulation, the TL/AD runs FP32.  Each
    # product carries about 2^-9 relative rounding from each operand, so the
    # stated bound on the whole A X is 1e-2; it must also exceed the FP32 path's
    # error (the BF16 products really ran).
    cfg, g, o = problem(case, "dense")
    n = cfg["n"]
    X = np.random.default_rng(4).standard_normal((cfg["ell"], n))
    Y = to_np_cols(g.hessvec(np.zeros(cfg["ell"], dtype=np.int32), torch.from_numpy(X).cuda(), mixed="bf16"), n)
    err = colrel(Y, o.A(X.T, [0] * cfg["ell"]))
    assert 1e-5 < err < 1e-2, err


@pytest.mark.parametrize("case", ["C1", "n1001"])
def test_hessvec_mixed_dense_fp32_bound(case):
    # Dense U_B with EDA_HV_MIXED: U_B products with FP32 operands and FP32
    # accumulation, FP32 TL/AD: single-precision rounding amplified by the
    # window, stated bound 1e-4 (as the banded FP32 path), and above 1e-10.
    cfg, g, o = problem(case, "dense")
    n = cfg["n"]
    X = np.random.default_rng(5).standard_normal((cfg["ell"], n))
    Y = to_np_cols(g.hessvec(np.zeros(cfg["ell"], dtype=np.int32), torch.from_numpy(X).cuda(), mixed=True), n)
    err = colrel(Y, o.A(X.T, [0] * cfg["ell"]))
    assert 1e-10 < err < 1e-4, err


@pytest.mark.parametrize("case", ["n203", "n1001", "n2049"])
@pytest.mark.parametrize("mode", ["banded", "dense"])
def test_hessvec_every_geometry(case, mode):
    # Every launch geometry the autotuner may pick (waves per workgroup, time-
    # block length) computes each point with the same formula; only the
    # compiler's FMA contraction may differ between the template instances
    # (points per lane), so the products agree to FP64 rounding (1e-13) with
    # the oracle and each other, member and sketch mode.
    cfg, g, o = problem(case, mode)
    n, L = cfg["n"], cfg["members"]
    Xn = np.random.default_rng(9).standard_normal((L + 1, n))
    X = torch.from_numpy(Xn).cuda()
    cols = np.arange(L + 1, dtype=np.int32)
    exact = o.A(Xn.T, list(range(L + 1))).T + Xn
    exact0 = o.A(Xn.T, [0] * (L + 1)).T
    tried, worst = 0, 0.0
    for w in (1, 2, 4, 8):
        for tb in (1, 2, 0):
            try:
                eda.eda_set_geometry(g.ctx, w, tb)
            except eda.EdaError as e:
                assert e.code == eda.EDA_ERR_UNSUPPORTED
                continue
            tried += 1
            y = g.hessvec(cols, X, add_identity=True).cpu().numpy()
            y0 = g.hessvec(np.zeros(L + 1, dtype=np.int32), X).cpu().numpy()
            e = max(colrel(y.T, exact.T), colrel(y0.T, exact0.T))
            worst = max(worst, e)
            assert e < 1e-12, (w, tb, e)
    eda.eda_set_geometry(g.ctx, 0, 0)
    print(f"[geometry] {case} {mode}: {tried} geometries, worst {worst:.2e}", flush=True)
    assert tried >= 3


def test_hessvec_edge_cases():
    cfg, g, o = problem("C1")
    n = cfg["n"]
    # nb = 0 is a no-op
    X0 = torch.empty((0, n), dtype=torch.float64, device="cuda")
    assert g.hessvec([], X0).shape == (0, n)
    # nb above the workspace bound is rejected
    Xbig = torch.zeros((g.max_cols + 1, n), dtype=torch.float64, device="cuda")
    with pytest.raises(eda.EdaError) as e:
        g.hessvec(np.zeros(g.max_cols + 1, dtype=np.int32), Xbig)
    assert e.value.code == eda.EDA_ERR_INVALID_ARG
    # a zero column maps to zero; linearity
    X = np.random.default_rng(5).standard_normal((3, n))
    X[1] = 0.0
    Y = to_np_cols(g.hessvec([0, 1, 2], torch.from_numpy(X).cuda()), n)
    assert np.all(Y[:, 1] == 0.0)
    Y2 = to_np_cols(g.hessvec([0, 1, 2], torch.from_numpy(2.5 * X).cuda()), n)
    assert colrel(Y2[:, [0, 2]], 2.5 * Y[:, [0, 2]]) < 1e-14


# ----------------------------------------------------------------- sketch --
def _oracle_sketch(o, kind, ell, k, q=1, method="nystrom", phi=None):
    """Oracle Ritz pairs and per-eigenvalue bars for the GPU's (see eig_bars;
    REVD: the Rayleigh quotients of two bases of range(A Phi) that agree to
    cond(Y) eps, which moves d_i by ~ cond(Y) eps d_1 absolute)."""
    Aop = lambda V: o.A(V, [0] * V.shape[1])
    if kind == "rhs_diff":
        phi = o.gamma(ell)
    if method == "nystrom":
        S, D, info = O.nystrom(Aop, phi, k, q)
        bars = eig_bars(D, info["cond_core"])
    else:
        S, D = O.revd(Aop, phi, k)
        condY = np.linalg.cond(Aop(phi))
        bars = np.maximum(1e-13, 16.0 * np.finfo(float).eps * condY * D[0] / D)
    return S, D, bars


def _compare_lmp(g, o, cfg, S, D, th, eig, theta_gpu, bars, label=""):
    err = np.abs(eig - D) / D
    print(f"[eig] {label} max err/bar {np.max(err / bars):.3f}; err[0] {err[0]:.2e} (bar {bars[0]:.1e}), "
          f"err[-1] {err[-1]:.2e} (bar {bars[-1]:.1e})", flush=True)
    assert np.all(err <= bars), (err, bars)
    tol = float(np.max(bars))
    assert abs(theta_gpu - th) <= bars[-1] * th
    n = cfg["n"]
    V = np.random.default_rng(9).standard_normal((min(16, g.max_cols), n))
    Vt = torch.from_numpy(V).cuda()
    for which in ("P", "U"):
        Pg = to_np_cols(g.lmp_apply(Vt, which), n)
        Po = O.lmp_apply(S, D, th, V.T, which)
        assert colrel(Pg, Po) < max(tol, 1e-12), (which, colrel(Pg, Po))
    Sg = g.field("S").cpu().numpy().reshape(-1, n).T
    # eigenvectors compared where the eigenvalue gap is large enough for them to be determined
    gaps = np.abs(np.diff(np.concatenate([[np.inf], D, [0.0]])))
    for i in range(len(D)):
        if min(gaps[i], gaps[i + 1]) > 1e-3 * D[0]:
            assert np.linalg.norm(Sg[:, i] - S[:, i]) < 1e3 * max(tol, 1e-12), i


@pytest.mark.parametrize("case", list(CASES))
def test_nystrom_rhs_diff(case):
    # Algorithm 1 with Phi = Gamma.  CholQR2 (GPU) and Householder QR (oracle)
    # agree to cond(Y) eps, and the Cholesky of the core to cond(core) eps:
    # each eigenvalue is held to its own bar (eig_bars).
    cfg, g, o = problem(case)
    eig, thg = g.sketch_evd("rhs_diff")
    S, D, bars = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"])
    _compare_lmp(g, o, cfg, S, D, O.theta(D), eig, thg, bars, f"nystrom {case}")


LMP_CASES = {
    # ragged: n not a multiple of 16, k not a multiple of 4, 37 columns (3 tiles, the last of 5)
    "n203": (CASES["n203"], 37),
    # one row block per 128 rows, 16 row blocks, every column tile of a C3-sized block (129 = 8 x 16 + 1)
    "n4096": (W.config("C3", nsteps=8, obs_dt=4, members=80, ell=64, k=61, spinup=100), 129),
    # rank above 64 (the wider expansion kernel), n odd, 6 tiles
    "n1001k77": (W.config("C2", n=1001, nsteps=6, obs_dt=3, members=90, ell=80, k=77, spinup=100), 91),
}


@pytest.mark.parametrize("case", list(LMP_CASES))
def test_lmp_block_matches_definition(case):
    # The block LMP (split projection with a fixed-order reduction, then the
    # expansion) against its definition X + S diag(coef) S^T X evaluated by the
    # oracle on the GPU's own Ritz pairs and theta: FP64 to 1e-13.
    cfg, ncols = LMP_CASES[case]
    g = eda.Problem(cfg, W.problem_normals(cfg), max_cols=ncols)
    eig, th = g.sketch_evd("rhs_diff")
    n = cfg["n"]
    S = g.field("S").cpu().numpy().reshape(-1, n).T
    V = np.random.default_rng(11).standard_normal((ncols, n))
    Vt = torch.from_numpy(V).cuda()
    for which in ("P", "U"):
        for nb in (ncols, ncols - 1, 1):
            Pg = to_np_cols(g.lmp_apply(Vt[:nb].contiguous(), which), n)
            Po = O.lmp_apply(S, eig, th, V[:nb].T, which)
            assert colrel(Pg, Po) < 1e-13, (which, nb, colrel(Pg, Po))
    g.close()


@pytest.mark.parametrize("case", ["C1", "n1001"])
def test_revd_and_power_pass(case):
    cfg, g, o = problem(case)
    eig, thg = g.sketch_evd("rhs_diff", method="revd")
    S, D, bars = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"], method="revd")
    _compare_lmp(g, o, cfg, S, D, O.theta(D), eig, thg, bars, f"revd {case}")
    eig, thg = g.sketch_evd("rhs_diff", q=2, theta="lamk")
    S, D, bars = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"], q=2)
    _compare_lmp(g, o, cfg, S, D, O.theta(D, "lamk"), eig, thg, bars, f"q2 {case}")


REVD_CORES = {
    # odd ell: the round-robin ordering of the EVD has an empty slot
    "ell5": CASES["n203"],
    # ell = 64: A and V of the EVD both in LDS
    "ell64": LMP_CASES["n4096"][0],
    # ell = 80: V in the global scratch
    "ell80": LMP_CASES["n1001k77"][0],
}


@pytest.mark.parametrize("case", list(REVD_CORES))
def test_revd_core_sizes(case):
    # REVD (second A-product pass, Jacobi EVD of Q^T A Q) against the oracle's
    # REVD at core sizes that take each path of the EVD kernel.
    cfg = REVD_CORES[case]
    z = W.problem_normals(cfg)
    print(f"[revd] {case} n={cfg['n']} ell={cfg['ell']} k={cfg['k']}", flush=True)
    g = eda.Problem(cfg, z)
    o = O.Problem(cfg, z)
    eig, thg = g.sketch_evd("rhs_diff", method="revd")
    S, D, bars = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"], method="revd")
    _compare_lmp(g, o, cfg, S, D, O.theta(D), eig, thg, bars, f"revd core {case}")
    g.close()


@pytest.mark.parametrize("kind", ["user", "b_psi", "ubt_psi"])
def test_sketch_kinds(kind):
    cfg, g, o = problem("C1")
    n, ell = cfg["n"], cfg["ell"]
    psi = W.gaussian_matrix(cfg, n, ell)          # ell x n (row c = column c)
    phi = {"user": psi.T, "b_psi": o.ub @ o.ub @ psi.T, "ubt_psi": o.ub.T @ psi.T}[kind]
    eig, thg = g.sketch_evd(kind, phi=torch.from_numpy(psi).cuda(), theta="one")
    S, D, bars = _oracle_sketch(o, "user", ell, cfg["k"], phi=phi)
    _compare_lmp(g, o, cfg, S, D, O.theta(D, "one"), eig, thg, bars, f"kind {kind}")


def test_sketch_errors():
    cfg = dict(CASES["C1"])
    g = eda.Problem(cfg, W.problem_normals(cfg))
    X = torch.zeros((2, cfg["n"]), dtype=torch.float64, device="cuda")
    with pytest.raises(eda.EdaError) as e:
        g.lmp_apply(X)
    assert e.value.code == eda.EDA_ERR_ORDER
    with pytest.raises(eda.EdaError) as e:
        g.sketch_evd("rhs_diff", ell=cfg["members"] + 1, k=2)
    assert e.value.code == eda.EDA_ERR_INVALID_ARG
    with pytest.raises(eda.EdaError) as e:
        g.pcg([0], 1e-6, 10, use_lmp=True)
    assert e.value.code == eda.EDA_ERR_ORDER
    g.close()


def test_shifted_pass_against_oracle():
    # ell = 32 RHS differences on small rings: Gamma and A Gamma are numerically
    # rank-deficient, an unshifted Cholesky of the last pass fails and the
    # device-side shifted pass (CholQR3 with the trace shift, then the Nystrom
    # shift nu = eps ||Y||_F) takes over.  Its eigenvalues match the oracle's --
    # which takes Householder QR and its own shift decision.  The core is
    # numerically singular (condition kappa ~ 1/eps), so relative bars do not
    # apply: T = R_Y C^-1 with C the Cholesky factor of the core carries
    # ||dT|| ~ sqrt(kappa) eps ||T||, and Weyl's inequality moves each
    # d_i = sigma_i^2 by at most 2 sigma_1 ||dT|| ~ 2 sqrt(kappa) eps d_1, plus
    # nu where a shift is taken: |d_i - d_i'| <= 16 (2 sqrt(kappa) eps d_1 + nu);
    # the leading eigenvalue to 1e-10 relative.  The LMP still gives the exact
    # solution.  A problem whose shifted pass fails too reports it.
    shapes = ((40, 10, 2.0), (40, 20, 2.0), (128, 10, 2.0), (64, 12, 2.0), (96, 8, 3.0))
    redone = 0
    for i, (n, N, lb) in enumerate(shapes):
        cfg = W.config("C2", n=n, nsteps=N, members=40, ell=32, k=32, len_b=lb, problem_id=300 + i, spinup=100)
        z = W.problem_normals(cfg)
        g = eda.Problem(cfg, z)
        try:
            eig, th = g.sketch_evd("rhs_diff", ell=32, k=32)
            ok = True
        except eda.EdaError as e:
            assert e.code == eda.EDA_ERR_NOT_SPD
            ok = False
        info = g.sketch_info()
        print(f"[shifted] n={n} N={N}: unshifted outcomes {info[:3].tolist()}, redone {info[3]}, failed {info[4]}",
              flush=True)
        assert info[3] == int(info[:3].any()) and info[4] == int(not ok)
        if not ok or not info[3]:
            g.close()
            continue
        redone += 1
        o = O.Problem(cfg, z)
        Aop = lambda V: o.A(V, [0] * V.shape[1])
        S, D, oinfo = O.nystrom(Aop, o.gamma(32), 32)
        eps = np.finfo(float).eps
        nu = eps * np.linalg.norm(Aop(o.gamma(32)))
        bar = 16.0 * (2.0 * np.sqrt(oinfo["cond_core"]) * eps * D[0] + nu)
        dev = np.abs(eig - D)
        print(f"[shifted]   cond(core) {oinfo['cond_core']:.1e}, oracle shift {oinfo['shift']:.1e}, nu {nu:.1e}; "
              f"rel err d_1 {dev[0] / D[0]:.1e}; max |d_i - d_i'| / bar {dev.max() / bar:.3f} "
              f"(bar {bar / D[0]:.1e} d_1)", flush=True)
        assert np.all(np.isfinite(eig)) and np.all(eig >= 0)
        assert dev[0] < 1e-10 * D[0] and np.all(dev <= bar), (dev / D[0], bar / D[0])
        members = [0, 7, cfg["members"]]
        out = g.pcg(members, rtol=1e-10, maxit=3000)
        assert (out["status"] == eda.EDA_MEMBER_CONVERGED).all()
        for j, m in enumerate(members):
            ex = O.exact_solution(o, m)
            assert np.linalg.norm(out["dz"][j].cpu().numpy() - ex) / np.linalg.norm(ex) < 1e-6
        g.close()
    assert redone >= 1


# -------------------------------------------------------------------- PCG --
def test_pcg_c1_fixed_iterations():
    # C1: exactly 50 iterations.  Past convergence to rounding the iterates of
    # two correct implementations wander independently, so the cost histories
    # are compared while J still decreases by more than 1e-13 |J|, and the
    # final solutions against the exact solution.
    cfg, g, o = problem("C1")
    g.sketch_evd("rhs_diff")
    S, D, _ = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"])
    th = O.theta(D)
    L = cfg["members"]
    out = g.pcg(np.arange(L + 1), rtol=0.0, maxit=50, use_lmp=True, history=True)
    assert np.all(out["iters"] == 50)
    for m in (0, 1, L):
        x, it, rr, st, hist = O.pcg(lambda v: o.hess(v[:, None], [m])[:, 0], o.b[:, m],
                                    lambda v: O.lmp_apply(S, D, th, v[:, None])[:, 0], 0.0, 50)
        hg = out["hist"][m]
        meaningful = np.concatenate([[True], np.abs(np.diff(hist)) > 1e-13 * np.abs(hist[-1])])
        cut = np.argmin(meaningful) if not meaningful.all() else len(hist)
        np.testing.assert_allclose(hg[:cut], hist[:cut], rtol=1e-8, atol=1e-10 * abs(hist[-1]))
        xe = O.exact_solution(o, m)
        assert rel(out["dz"][m].cpu().numpy(), xe) < 1e-10


@pytest.mark.parametrize("case", ["n203", "n1001"])
@pytest.mark.parametrize("use_lmp", [False, True])
def test_pcg_converges_like_oracle(case, use_lmp):
    cfg, g, o = problem(case)
    L = cfg["members"]
    if use_lmp:
        g.sketch_evd("rhs_diff")
        S, D, _ = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"])
        th = O.theta(D)
        Pop = lambda v: O.lmp_apply(S, D, th, v[:, None])[:, 0]
    else:
        Pop = None
    out = g.pcg(np.arange(L + 1), rtol=1e-10, maxit=500, use_lmp=use_lmp)
    assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
    assert np.all(out["relres"] <= 1e-10)
    for m in (0, L):
        _, it, _, st, _ = O.pcg(lambda v: o.hess(v[:, None], [m])[:, 0], o.b[:, m], Pop, 1e-10, 500)
        # at rtol 1e-10 the count is rounding-sensitive (different but valid
        # summation orders, and an LMP equal to the oracle's to ~1e-10): allow 5%
        assert abs(int(out["iters"][m]) - it) <= max(2, int(0.05 * it)), (m, out["iters"][m], it)
        xe = O.exact_solution(o, m)
        assert rel(out["dz"][m].cpu().numpy(), xe) < 1e-8


def test_pcg_not_converged_and_deterministic():
    cfg, g, o = problem("n203")
    L = cfg["members"]
    out = g.pcg(np.arange(L + 1), rtol=1e-12, maxit=3, use_lmp=False)
    assert out["code"] == eda.EDA_WARN_NOT_CONVERGED
    assert np.all(out["status"] == eda.EDA_MEMBER_NOT_CONVERGED) and np.all(out["iters"] == 3)
    a = g.pcg([2, 0, 2], rtol=1e-8, maxit=100, use_lmp=False)
    b = g.pcg([2, 0, 2], rtol=1e-8, maxit=100, use_lmp=False)
    assert torch.equal(a["dz"], b["dz"])
    assert torch.equal(a["dz"][0], a["dz"][2])  # same member twice: same bits


@pytest.mark.parametrize("case", ["n1001", "n2049"])
def test_split_iterations_match_whole_columns(case):
    # Split iterations (the Hessian part on P pieces per column) against whole
    # columns (P = 1): independent ring pieces (halos of 12 N + 2 w states on
    # each side, EDA_XCH_OFF) and pieces that share the observed increments
    # (EDA_XCH_OBS, the default: 12 N + 2 w halo states in all, one bounded
    # wait between the TL and AD runs).  The pieces' outputs are the whole
    # column's bits; only the order of the partial sums of p^T (I + A) p
    # differs (it follows the pieces and each piece's lane layout), so after 4
    # iterations the iterates agree to rounding; solved to rtol 1e-10 every
    # form reaches the exact solution.  A wait limit of 0 makes the shared form
    # report EDA_ERR_SYNC, which shows that it ran (it needs pieces of at least
    # 8 N + w states; shorter ones fall back to independent pieces).
    cfg, g, o = problem(case)
    g.sketch_evd("rhs_diff")
    members = np.arange(cfg["members"] + 1)
    ref = None
    shared = []
    worst = 0.0
    for P in (1, 2, 3, 4, 5, 8):
        try:
            eda.eda_set_split(g.ctx, P)
        except eda.EdaError as e:  # a ring of ceil(n / P) + 2 halos longer than n
            assert e.code == eda.EDA_ERR_UNSUPPORTED and P > 2, (P, e.code)
            continue
        for xch in (eda.EDA_XCH_OFF, eda.EDA_XCH_OBS) if P > 1 else (eda.EDA_XCH_OFF,):
            eda.eda_set_exchange(g.ctx, xch)
            dz = g.pcg(members, rtol=0.0, maxit=4)["dz"].cpu().numpy()
            if ref is None:
                ref = dz
            else:
                e = colrel(dz, ref)
                worst = max(worst, e)
                assert e < 1e-12, (P, xch, e)
        if P > 1:
            eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, 0)
            try:
                g.pcg(members, rtol=0.0, maxit=2)
            except eda.EdaError as e:
                assert e.code == eda.EDA_ERR_SYNC, e.code
                shared.append(P)
            eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, -1)
    print(f"[split] {case}: 4 iterations vs whole columns {worst:.1e} (element-wise); shared-observation "
          f"pieces ran for P = {shared}", flush=True)
    assert 2 in shared and 3 in shared
    for P, xch in ((1, eda.EDA_XCH_OFF), (8, eda.EDA_XCH_OFF), (2, eda.EDA_XCH_OBS), (shared[-1], eda.EDA_XCH_OBS)):
        eda.eda_set_split(g.ctx, P)
        eda.eda_set_exchange(g.ctx, xch)
        out = g.pcg(members, rtol=1e-10, maxit=500, history=True)
        assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
        assert np.all(out["relres"] <= 1e-10)
        for m in (0, cfg["members"]):
            xe = O.exact_solution(o, m)
            assert elrel(out["dz"][m].cpu().numpy(), xe) < 1e-8, (P, xch, m)
            h = out["hist"][m][: out["iters"][m] + 1]
            assert np.all(np.diff(h) <= 1e-10 * abs(h[-1]))  # the cost decreases
    eda.eda_set_split(g.ctx, 0)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS)
    a = g.pcg(members, rtol=1e-8, maxit=500)
    b = g.pcg(members, rtol=1e-8, maxit=500)
    assert torch.equal(a["dz"], b["dz"])  # the automatic pieces do not depend on timing


@pytest.mark.parametrize("case", ["n1001", "n2049"])
def test_exchange_iterations_match_whole_columns(case):
    # Wave pieces with halo exchange (eda_set_exchange ON, n >= 512) against
    # whole columns: only the summation order of r^T z and p^T (I + A) p
    # differs, so after 4 iterations the iterates agree to rounding; solved to
    # rtol 1e-10 they reach the exact solution; repeated solves are bit-identical.
    cfg, g, o = problem(case)
    g.sketch_evd("rhs_diff")
    members = np.arange(cfg["members"] + 1)
    eda.eda_set_split(g.ctx, 1)
    ref = g.pcg(members, rtol=0.0, maxit=4)["dz"].cpu().numpy()
    eda.eda_set_split(g.ctx, 0)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_ON)
    dz = g.pcg(members, rtol=0.0, maxit=4)["dz"].cpu().numpy()
    e4 = rel(dz, ref)
    out = g.pcg(members, rtol=1e-10, maxit=500, history=True)
    assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED), out["status"]
    errs = []
    for m in (0, cfg["members"]):
        xe = O.exact_solution(o, m)
        errs.append(elrel(out["dz"][m].cpu().numpy(), xe))
        h = out["hist"][m][: out["iters"][m] + 1]
        assert np.all(np.diff(h) <= 1e-10 * abs(h[-1]))  # the cost decreases
    again = g.pcg(members, rtol=1e-10, maxit=500)
    print(f"[xch] {case}: 4 iterations vs whole columns {e4:.1e}; rtol 1e-10 in {out['iters'].tolist()} "
          f"iterations, element-wise error vs exact {max(errs):.1e}", flush=True)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS)
    assert e4 < 1e-12 and max(errs) < 1e-8
    assert torch.equal(out["dz"], again["dz"])


def test_exchange_after_a_multi_stream_batch():
    # A batch solve (work on many streams) leaves the dealing of workgroups to
    # XCDs starting elsewhere; the exchange form then still pairs neighbours on
    # one XCD (virtual workgroup indices) and solves correctly.
    cfgs = [W.config("C2", n=1024, nsteps=10, members=12, ell=8, k=8, problem_id=41, spinup=200),
            W.config("C2", n=512, nsteps=20, members=9, ell=6, k=6, problem_id=42, spinup=200)]
    probs = [eda.Problem(c, W.problem_normals(c)) for c in cfgs]
    bt = eda.Batch(probs)
    bt.solve(k_cap=8, rtol=1e-8, maxit=500)
    bt.close()
    for c, g in zip(cfgs, probs):
        g.sketch_evd("rhs_diff")
        members = np.arange(c["members"] + 1)
        eda.eda_set_exchange(g.ctx, eda.EDA_XCH_ON)
        out = g.pcg(members, rtol=1e-10, maxit=500)
        assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
        eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OFF)
        ref = g.pcg(members, rtol=1e-10, maxit=500)
        e = rel(out["dz"].cpu().numpy(), ref["dz"].cpu().numpy())
        print(f"[xch] after a batch, n={c['n']}: exchange vs ring pieces {e:.1e}", flush=True)
        assert e < 1e-8
        g.close()


def test_exchange_wait_limit_reports_sync_error():
    # Every wait of the exchange form gives up at once (limit 0, set from the
    # host): the members stop with a breakdown and the solve reports
    # EDA_ERR_SYNC; every kernel still runs to its end.  With the default limit
    # the same context solves normally again.
    cfg, g, o = problem("n1001")
    g.sketch_evd("rhs_diff")
    members = np.arange(cfg["members"] + 1)
    eda.eda_set_split(g.ctx, 0)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_ON, 0)
    with pytest.raises(eda.EdaError) as ei:
        g.pcg(members, rtol=1e-10, maxit=50)
    assert ei.value.code == eda.EDA_ERR_SYNC
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_ON, -1)
    out = g.pcg(members, rtol=1e-10, maxit=500)
    assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OFF)
    off = g.pcg(members, rtol=1e-10, maxit=500)
    assert rel(off["dz"].cpu().numpy(), out["dz"].cpu().numpy()) < 1e-8
    # the same for the pieces that share the observed increments (the default)
    eda.eda_set_split(g.ctx, 2)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, 0)
    with pytest.raises(eda.EdaError) as ei:
        g.pcg(members, rtol=1e-10, maxit=50)
    assert ei.value.code == eda.EDA_ERR_SYNC
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, -1)
    sh = g.pcg(members, rtol=1e-10, maxit=500)
    assert np.all(sh["status"] == eda.EDA_MEMBER_CONVERGED)
    assert rel(sh["dz"].cpu().numpy(), out["dz"].cpu().numpy()) < 1e-8
    eda.eda_set_split(g.ctx, 0)


def _lmp_form_problem(case):
    if case in CASES:
        cfg, g, _ = problem(case)
        return cfg, g, False
    cfg = LMP_CASES[case][0]
    return cfg, eda.Problem(cfg, W.problem_normals(cfg), max_cols=cfg["members"] + 1), True


@pytest.mark.parametrize("case", ["n1001", "n2049", "n4096"])
def test_lmp_one_launch_matches_two_launches(case):
    # The single-launch LMP (a barrier per column tile in device memory between
    # the projection and the expansion) does the two-launch form's arithmetic in
    # the same order: the PCG iterates are the same bits in every iteration form
    # that applies the LMP -- whole columns (P = 1), ring pieces (P = 2, the LMP
    # fused with the update), wave pieces with halo exchange -- and with the
    # dense U_B.  n4096: 81 columns, 6 tiles x 16 row blocks in one launch.
    cfg, g, own = _lmp_form_problem(case)
    g.sketch_evd("rhs_diff")
    members = np.arange(cfg["members"] + 1)
    forms = [("whole columns", 1, eda.EDA_XCH_OFF), ("ring pieces", 2, eda.EDA_XCH_OFF),
             ("shared-observation pieces", 2, eda.EDA_XCH_OBS), ("wave pieces", 0, eda.EDA_XCH_ON)]
    for label, P, xch in forms:
        eda.eda_set_split(g.ctx, P)
        eda.eda_set_exchange(g.ctx, xch)
        out = {}
        for form in (eda.EDA_LMP_FORM_TWO, eda.EDA_LMP_FORM_ONE):
            eda.eda_set_lmp_form(g.ctx, form)
            out[form] = g.pcg(members, rtol=0.0, maxit=6)
        a, b = out[eda.EDA_LMP_FORM_TWO], out[eda.EDA_LMP_FORM_ONE]
        same = torch.equal(a["dz"], b["dz"]) and np.array_equal(a["relres"], b["relres"])
        print(f"[lmp form] {case} {label}: one launch == two launches: {same}", flush=True)
        assert same, (case, label)
    eda.eda_set_split(g.ctx, 0)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS)
    if case == "n1001":
        cfg, gd, _ = problem(case, "dense")
        gd.sketch_evd("rhs_diff")
        res = []
        for form in (eda.EDA_LMP_FORM_TWO, eda.EDA_LMP_FORM_ONE):
            eda.eda_set_lmp_form(gd.ctx, form)
            res.append(gd.pcg(members, rtol=1e-10, maxit=500)["dz"])
        assert torch.equal(res[0], res[1])
    if own:
        g.close()


def test_lmp_one_launch_wait_limit_reports_sync_error():
    # Every tile-barrier wait gives up at once (limit 0, set from the host):
    # the solve reports EDA_ERR_SYNC and every kernel runs to its end.  The
    # two-launch form has no waits and solves normally under the same limit;
    # with the default limit the single launch solves to the same bits.
    cfg, g, o = problem("n1001")
    g.sketch_evd("rhs_diff")
    members = np.arange(cfg["members"] + 1)
    eda.eda_set_split(g.ctx, 1)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OFF, 0)
    eda.eda_set_lmp_form(g.ctx, eda.EDA_LMP_FORM_ONE)
    with pytest.raises(eda.EdaError) as ei:
        g.pcg(members, rtol=1e-10, maxit=50)
    assert ei.value.code == eda.EDA_ERR_SYNC
    eda.eda_set_lmp_form(g.ctx, eda.EDA_LMP_FORM_TWO)
    two = g.pcg(members, rtol=1e-10, maxit=500)
    assert np.all(two["status"] == eda.EDA_MEMBER_CONVERGED)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, -1)
    eda.eda_set_lmp_form(g.ctx, eda.EDA_LMP_FORM_ONE)
    one = g.pcg(members, rtol=1e-10, maxit=500)
    assert torch.equal(one["dz"], two["dz"])
    eda.eda_set_split(g.ctx, 0)


@pytest.mark.parametrize("case", ["n1001", "n2049"])
def test_split_hessvec_matches_whole_columns(case):
    # Hessian products on P pieces per column (independent rings of the
    # piece's states with halos of 12 N + 2 w on each side, and pieces that
    # share the observed increments with 12 N + 2 w in all): every owned output
    # is the whole column's, bit for bit, in member mode and in sketch mode,
    # with and without the identity, with FP64 and with FP32 TL/AD runs; and
    # the oracle agrees.
    cfg, g, o = problem(case)
    n, L = cfg["n"], cfg["members"]
    rng = np.random.default_rng(7)
    X = torch.from_numpy(rng.standard_normal((L + 1, n))).cuda()
    cols = np.arange(L + 1)
    zero = np.zeros(L + 1, dtype=np.int64)
    for cc in (cols, zero):
        for add, mixed in ((False, False), (True, False), (True, True)):
            eda.eda_set_split(g.ctx, 1)
            ref = g.hessvec(cc, X, add_identity=add, mixed=mixed).clone()
            done = 0
            for P in (0, 2, 3, 4, 8):
                try:
                    eda.eda_set_split(g.ctx, P)
                except eda.EdaError as e:
                    assert e.code == eda.EDA_ERR_UNSUPPORTED and P > 2
                    continue
                for xch in (eda.EDA_XCH_OFF, eda.EDA_XCH_OBS):
                    eda.eda_set_exchange(g.ctx, xch)
                    Y = g.hessvec(cc, X, add_identity=add, mixed=mixed)
                    assert torch.equal(Y, ref), (case, P, xch, add, mixed)
                done += 1
            assert done >= 3
    eda.eda_set_split(g.ctx, 0)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS)
    Yc = to_np_cols(g.hessvec(cols, X, add_identity=True), n)
    Xc = X.cpu().numpy().T
    assert colrel(Yc, o.hess(Xc, cols)) < 1e-12
    # five columns (8 pieces each by default) read from and written to column
    # slices of wider buffers (ldx = n + 37, ldy = n + 53): the same values as
    # whole columns, and the padding rows stay as they were
    sel = torch.tensor([3, 0, L, 1, 2], dtype=torch.int32, device="cuda")
    Xw = torch.from_numpy(rng.standard_normal((5, n + 37))).cuda()
    for P in (1, 0):
        eda.eda_set_split(g.ctx, P)
        Yw = torch.full((5, n + 53), 7.25, dtype=torch.float64, device="cuda")
        eda.eda_hessvec(g.ctx, n, sel, Xw[:, :n], Yw[:, :n], eda.EDA_HV_ADD_IDENTITY)
        assert torch.all(Yw[:, n:] == 7.25)
        if P == 1:
            ref = Yw[:, :n].clone()
        else:
            assert torch.equal(Yw[:, :n], ref), case
    eda.eda_set_split(g.ctx, 0)
    Xs = Xw[:, :n].cpu().numpy().T
    assert colrel(to_np_cols(ref.contiguous(), n), o.hess(Xs, sel.cpu().numpy())) < 1e-12


def test_columns_wait_for_a_free_slot():
    # More columns than two pieces each hold on the device (141 columns; half
    # the CUs is 128): 128 start, the control member's column and the last 12
    # wait, and are admitted, each from its own first iteration, as running
    # ones stop.  Every column reaches its own solution with its own
    # iteration count and cost history (against the same members solved in
    # calls of at most 128 columns, where nothing waits, and against the
    # oracle's exact solution); a repeat gives the same bits; with a small
    # maxit the waiting columns end not converged after 0 iterations.
    cap = torch.cuda.get_device_properties(0).multi_processor_count // 2
    cfg = W.config("C2", n=1001, nsteps=12, obs_dt=3, obs_dx=2, obs_x0=1, members=cap + 12, ell=16, k=16,
                   spinup=200)
    nm = cfg["members"] + 1
    z = W.problem_normals(cfg)
    g = eda.Problem(cfg, z)
    g.sketch_evd("rhs_diff")
    members = np.arange(nm)
    waiting = [0] + list(range(cap + 1, nm))
    print(f"[admit] n=1001, {nm} columns, {cap} slots; waiting {waiting}", flush=True)
    out = g.pcg(members, rtol=1e-10, maxit=1000, history=True)
    assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
    assert np.all(out["relres"] <= 1e-10)
    ref_it = np.zeros(nm, dtype=np.int64)
    ref_dz = np.zeros((nm, cfg["n"]))
    ref_h = {}
    for part in (members[:cap], members[cap:]):
        r = g.pcg(part, rtol=1e-10, maxit=1000, history=True)
        assert np.all(r["status"] == eda.EDA_MEMBER_CONVERGED)
        ref_it[part] = r["iters"]
        ref_dz[part] = r["dz"].cpu().numpy()
        for i, m in enumerate(part):
            ref_h[m] = r["hist"][i]
    d = np.abs(out["iters"] - ref_it)
    dz = out["dz"].cpu().numpy()
    e = max(elrel(dz[m], ref_dz[m]) for m in members)
    print(f"[admit] iterations of the waiting columns {out['iters'][waiting].tolist()} (alone "
          f"{ref_it[waiting].tolist()}); max |diff| over all {int(d.max())}; solutions vs calls without "
          f"waiting {e:.1e} element-wise", flush=True)
    assert (d <= np.maximum(3, (0.05 * ref_it).astype(int))).all()
    assert e < 1e-8
    o = O.Problem(cfg, z)
    for m in (0, 1, nm - 1):
        assert elrel(dz[m], O.exact_solution(o, m)) < 1e-8, m
        h, hr = out["hist"][m][: out["iters"][m] + 1], ref_h[m][: ref_it[m] + 1]
        assert h[0] == 0.0 and np.all(np.diff(h) <= 1e-10 * abs(h[-1]))  # the column's own history
        k = min(h.size, hr.size) - 1
        assert abs(h[k] - hr[k]) <= 1e-8 * abs(hr[k]), (m, h[k], hr[k])
    again = g.pcg(members, rtol=1e-10, maxit=1000)
    assert torch.equal(again["dz"], out["dz"])  # admissions do not depend on timing
    few = g.pcg(members, rtol=1e-10, maxit=6)
    assert np.all(few["status"] == eda.EDA_MEMBER_NOT_CONVERGED)
    assert np.all(few["iters"][waiting] == 0)
    assert np.all(np.delete(few["iters"], waiting) == 6)
    g.close()


def test_pieces_that_only_the_shared_form_fits():
    # n = 2048, N = 40: independent ring pieces need ceil(n / P) + 24 N + 4 w
    # states, more than n for every P, so before the shared form no column of
    # this shape was split; shared pieces need ceil(n / P) + 12 N + 2 w (1606
    # for P = 2).  Forced P = 2 and the automatic choice solve like whole
    # columns (to rounding; products bit for bit); a forced P that only the
    # shared form fits is refused at the call when the exchange mode is OFF.
    cfg = W.config("C3", n=2048, nsteps=40, members=5, ell=4, k=4, spinup=200)
    g = eda.Problem(cfg, W.problem_normals(cfg))
    n, L = cfg["n"], cfg["members"]
    members = np.arange(L + 1)
    g.sketch_evd("rhs_diff")
    X = torch.from_numpy(np.random.default_rng(5).standard_normal((L + 1, n))).cuda()
    eda.eda_set_split(g.ctx, 1)
    ref = g.pcg(members, rtol=0.0, maxit=6)["dz"].cpu().numpy()
    hv = g.hessvec(members, X, add_identity=True).clone()
    eda.eda_set_split(g.ctx, 2)
    dz = g.pcg(members, rtol=0.0, maxit=6)["dz"].cpu().numpy()
    e = colrel(dz, ref)
    assert torch.equal(g.hessvec(members, X, add_identity=True), hv)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OFF)
    with pytest.raises(eda.EdaError) as ei:
        g.pcg(members, rtol=0.0, maxit=2)
    assert ei.value.code == eda.EDA_ERR_UNSUPPORTED
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS)
    eda.eda_set_split(g.ctx, 0)  # automatic: 4 shared pieces (8 would be shorter than 8 N + w)
    auto = g.pcg(members, rtol=1e-9, maxit=4000)
    eda.eda_set_split(g.ctx, 1)
    whole = g.pcg(members, rtol=1e-9, maxit=4000)
    eda.eda_set_split(g.ctx, 0)
    ea = colrel(auto["dz"].cpu().numpy(), whole["dz"].cpu().numpy())
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, 0)
    with pytest.raises(eda.EdaError) as ei:  # the automatic choice ran shared pieces
        g.pcg(members, rtol=0.0, maxit=2)
    assert ei.value.code == eda.EDA_ERR_SYNC
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, -1)
    print(f"[only-shared] n=2048 N=40: 6 iterations P=2 vs whole {e:.1e}; rtol 1e-9 automatic vs whole {ea:.1e} "
          f"(iterations {auto['iters'].tolist()} / {whole['iters'].tolist()})", flush=True)
    # 6 iterations: the pieces' partial sums of p^T (I + A) p round otherwise
    # (5e-13 measured); two solves to rtol 1e-9 of this stiffer shape differ
    # by the conditioning times their residuals
    assert e < 1e-11 and ea < 1e-6
    assert np.all(auto["status"] == eda.EDA_MEMBER_CONVERGED)
    assert np.all(whole["status"] == eda.EDA_MEMBER_CONVERGED)
    g.close()


def test_shared_pieces_wait_limit_in_products_and_sketch():
    # With a wait limit of 0 (set from the host) every wait of the pieces that
    # share the observed increments gives up at once: a Hessian product on
    # pieces then leaves NaN in the pieces' rows, and a sketch whose products
    # ran on such pieces reports EDA_ERR_SYNC and keeps no LMP.  Every kernel
    # still runs to its end, and with the default limit the same context gives
    # the whole columns' bits again.
    cfg, g, o = problem("n2049")
    n, L = cfg["n"], cfg["members"]
    X = torch.from_numpy(np.random.default_rng(3).standard_normal((L + 1, n))).cuda()
    cols = np.arange(L + 1)
    eda.eda_set_split(g.ctx, 1)
    ref = g.hessvec(cols, X, add_identity=True).clone()
    eda.eda_set_split(g.ctx, 2)
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, 0)
    Y = g.hessvec(cols, X, add_identity=True)
    assert torch.isnan(Y).all(), "every piece's wait gave up: every row is NaN"
    eda.eda_set_split(g.ctx, 0)
    with pytest.raises(eda.EdaError) as ei:
        g.sketch_evd("rhs_diff")
    assert ei.value.code == eda.EDA_ERR_SYNC
    with pytest.raises(eda.EdaError) as ei:
        g.pcg(np.arange(L + 1), rtol=1e-8, maxit=10)
    assert ei.value.code == eda.EDA_ERR_ORDER  # no LMP was kept
    eda.eda_set_exchange(g.ctx, eda.EDA_XCH_OBS, -1)
    eda.eda_set_split(g.ctx, 2)
    assert torch.equal(g.hessvec(cols, X, add_identity=True), ref)
    eda.eda_set_split(g.ctx, 0)
    g.sketch_evd("rhs_diff")


def test_split_errors():
    cfg, g, o = problem("C1")  # n = 40: no ring shorter than n
    with pytest.raises(eda.EdaError) as e:
        eda.eda_set_split(g.ctx, 2)
    assert e.value.code == eda.EDA_ERR_UNSUPPORTED
    with pytest.raises(eda.EdaError) as e:
        eda.eda_set_split(g.ctx, 3)
    assert e.value.code == eda.EDA_ERR_UNSUPPORTED
    for bad in (-1, 9):
        with pytest.raises(eda.EdaError) as e:
            eda.eda_set_split(g.ctx, bad)
        assert e.value.code == eda.EDA_ERR_INVALID_ARG
    eda.eda_set_split(g.ctx, 1)
    eda.eda_set_split(g.ctx, 0)
    cfg, gd, o = problem("n1001", mode="dense")
    with pytest.raises(eda.EdaError) as e:
        eda.eda_set_split(gd.ctx, 2)
    assert e.value.code == eda.EDA_ERR_UNSUPPORTED


def test_profile_counts_pcg_tlad_launches():
    # the profile covers the TL/AD kernel inside eda_pcg_solve only: one fused
    # launch per iteration (banded U_B); Hessian products outside PCG are not
    # timed; with a period of 5, launches 1, 6, 11 of 12 are timed
    cfg, g, o = problem("C1")
    eda.eda_profile(g.ctx, 1)
    X = torch.from_numpy(np.ones((3, cfg["n"]))).cuda()
    g.hessvec([0, 1, 2], X)
    assert eda.eda_profile_read(g.ctx)[:2] == (0, 0)
    out = g.pcg([0, 1, 2], rtol=0.0, maxit=12, use_lmp=False)
    t, n, ms = eda.eda_profile_read(g.ctx)
    assert (out["iters"] == 12).all()
    assert t == 12 and n == 12 and ms > 0
    eda.eda_profile(g.ctx, 5)
    g.pcg([0, 1, 2], rtol=0.0, maxit=12, use_lmp=False)
    t, n, ms5 = eda.eda_profile_read(g.ctx)
    eda.eda_profile(g.ctx, 0)
    assert t == 3 and n == 12 and 0 < ms5 < ms
    with pytest.raises(eda.EdaError):
        eda.eda_profile(g.ctx, -1)


# ------------------------------------------------- full-size (sampled) ------
_full = {}


def full_oracle(name):
    if name not in _full:
        cfg = W.config(name)
        _full[name] = O.Problem(cfg, W.problem_normals(cfg))
    return _full[name]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,mode", [("C2", "banded"), ("C2", "dense"), ("C3", "banded"), ("C3", "dense")])
def test_full_size_sampled(name, mode):
    # The benchmark configurations at full size, in both U_B forms (the dense
    # form is the bench's plain FP64 form: U_B products as 4096 x 4096 FP64
    # MFMA GEMMs at C3): set-up fields, sampled Hessian columns, the
    # Gamma-Nystrom eigenvalues, and the batched LMP-PCG of every member to
    # rtol 1e-6, whose sampled members are checked by the oracle's true
    # residual.
    cfg = W.config(name)
    z = W.problem_normals(cfg)
    print(f"[full] {name} {mode}", flush=True)
    g = eda.Problem(cfg, z, ub_mode=mode)
    o = full_oracle(name)
    n, L, N = cfg["n"], cfg["members"], cfg["nsteps"]
    assert np.array_equal(g.field("truth").cpu().numpy().reshape(N + 1, n), o.xt_traj)
    assert colrel(to_np_cols(g.field("b"), n), o.b) < 1e-12
    cols = np.array([0, 1, L // 2, L])
    X = np.random.default_rng(1).standard_normal((cols.size, n))
    Y = to_np_cols(g.hessvec(cols, torch.from_numpy(X).cuda(), add_identity=True), n)
    e = colrel(Y, o.hess(X.T, cols))
    print(f"[full] {name} {mode} hessvec element-wise error {e:.2e}", flush=True)
    assert e < 1e-12
    eig, th = g.sketch_evd("rhs_diff")
    _, D, bars = _oracle_sketch(o, "rhs_diff", cfg["ell"], cfg["k"])
    err = np.abs(eig - D) / D
    print(f"[full] {name} {mode} eigenvalues: max err/bar {np.max(err / bars):.3f}, err[0] {err[0]:.1e}, "
          f"err[-1] {err[-1]:.1e}", flush=True)
    assert np.all(err <= bars)
    out = g.pcg(np.arange(L + 1), rtol=1e-6, maxit=2000, use_lmp=True)
    print(f"[full] {name} {mode} iterations min/median/max {out['iters'].min()}/{np.median(out['iters'])}/"
          f"{out['iters'].max()}", flush=True)
    assert np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)
    dz = out["dz"].cpu().numpy()
    for m in (0, L):
        r = o.b[:, m] - o.hess(dz[m][:, None], [m])[:, 0]
        assert np.linalg.norm(r) <= 2e-6 * np.linalg.norm(o.b[:, m])
    g.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,members", [("C2", (0, 64)), ("C3", (0, 1, 64, 128))])
def test_solution_bar_of_the_chosen_form(name, members):
    # The solution bar (reading of the tolerance pair): with the bench's chosen
    # form -- banded U_B, the Gamma-Nystrom sketch with two passes and FP32
    # TL/AD sketch products (C3), or the FP64 single-pass sketch (C2) --
    # members solved to rtol 1e-10 are within 1e-6 relative of the exact
    # solution of (I + A_m) dz = b_m, assembled densely and solved by Cholesky
    # in the oracle, element by element (largest difference over largest
    # magnitude) and in the 2-norm.  At the throughput tolerance 1e-6 the error
    # is printed, not gated (it is bounded only by cond(I + A) 1e-6).
    cfg = W.config(name)
    z = W.problem_normals(cfg)
    g = eda.Problem(cfg, z)
    o = full_oracle(name)
    if name == "C3":
        g.sketch_evd("rhs_diff", q=2, mixed=True)
    else:
        g.sketch_evd("rhs_diff")
    tight = g.pcg(members, rtol=1e-10, maxit=4000, use_lmp=True)
    loose = g.pcg(members, rtol=1e-6, maxit=4000, use_lmp=True)
    assert np.all(tight["status"] == eda.EDA_MEMBER_CONVERGED)
    for i, m in enumerate(members):
        xe = exact(name, o, m)
        dz = tight["dz"][i].cpu().numpy()
        e_el, e_2 = elrel(dz, xe), rel(dz, xe)
        d6 = loose["dz"][i].cpu().numpy()
        print(f"[bar] {name} member {m}: rtol 1e-10 ({tight['iters'][i]} it) element-wise {e_el:.2e}, "
              f"2-norm {e_2:.2e}; rtol 1e-6 ({loose['iters'][i]} it) element-wise {elrel(d6, xe):.2e}, "
              f"2-norm {rel(d6, xe):.2e}", flush=True)
        assert e_el <= 1e-6 and e_2 <= 1e-6
    g.close()
