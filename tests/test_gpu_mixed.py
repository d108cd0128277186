"""GPU: reduced-precision sketch products against the FP64 oracle.

Only the sketch's Hessian products drop precision (FP32 TL/AD; dense U_B
products with FP32 or BF16 operands, FP32 accumulation); the trajectory,
CholQR2, the k x k eigensolve and the PCG recurrences stay FP64.  Stated errors
(each bound is a few times the value measured on MI355X):

  sketch                      eigenvalues (max rel)  LMP operator   solution
  FP32 TL/AD, banded U_B      1e-5 (n=1001), 1e-3*   1e-6           unchanged
  FP32 TL/AD + FP32 GEMM      1e-5                   1e-6           unchanged
  FP32 TL/AD + BF16 GEMM      1e-2                   1e-3           unchanged

(* n=1024, ell=32: the smallest retained eigenvalues carry the relative error
of the FP32 products amplified by the Gram matrix's conditioning.)
"Unchanged": PCG with the reduced-precision LMP still reaches the exact
solution to the FP64 bar (1e-6 relative at rtol 1e-10); the LMP only changes
the iteration count."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_23571_amd import eda  # noqa: E402

CFG_N1001 = W.config("C2", n=1001, nsteps=12, obs_dt=3, obs_dx=2, obs_x0=1, members=20, ell=16, k=16, spinup=200)
CFG_C2S = W.config("C2", members=32, ell=32, k=32, spinup=300)

_cache = {}


def oracle_lmp(cfg):
    key = id(cfg)
    if key not in _cache:
        z = W.problem_normals(cfg)
        o = O.Problem(cfg, z)
        S, D, _ = O.nystrom(lambda V: o.A(V, [0] * V.shape[1]), o.gamma(cfg["ell"]), cfg["k"])
        _cache[key] = (z, o, S, D, O.theta(D))
    return _cache[key]


def sketch_errors(cfg, mode, mixed):
    z, o, S, D, th = oracle_lmp(cfg)
    g = eda.Problem(cfg, z, ub_mode=mode)
    eig, thg = g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"], mixed=mixed)
    V = np.random.default_rng(7).standard_normal((cfg["n"], 16))
    PVg = g.lmp_apply(torch.from_numpy(np.ascontiguousarray(V.T)).cuda()).cpu().numpy().T
    PV = O.lmp_apply(S, D, th, V)
    e_eig = float(np.max(np.abs(eig - D) / D))
    e_lmp = float(np.linalg.norm(PVg - PV) / np.linalg.norm(V))
    return g, o, e_eig, e_lmp


@pytest.mark.parametrize("mode,mixed,b_eig,b_lmp", [("banded", True, 1e-5, 1e-6), ("dense", True, 1e-5, 1e-6),
                                                     ("dense", "bf16", 1e-2, 1e-3)])
def test_reduced_precision_sketch_errors_n1001(mode, mixed, b_eig, b_lmp):
    cfg = CFG_N1001
    g, o, e_eig, e_lmp = sketch_errors(cfg, mode, mixed)
    print(f"[mixed] n1001 {mode} {mixed}: eig {e_eig:.3e} lmp {e_lmp:.3e}", flush=True)
    assert 0 < e_eig < b_eig and 0 < e_lmp < b_lmp
    # the solution is still the FP64 one
    out = g.pcg([0, 7], rtol=1e-10, maxit=3000)
    assert (out["status"] == eda.EDA_MEMBER_CONVERGED).all()
    dz = out["dz"].cpu().numpy()
    for i, m in enumerate([0, 7]):
        ex = O.exact_solution(o, m)
        assert np.linalg.norm(dz[i] - ex) / np.linalg.norm(ex) < 1e-6
    g.close()


def test_reduced_precision_sketch_errors_c2_banded():
    cfg = CFG_C2S
    g, o, e_eig, e_lmp = sketch_errors(cfg, "banded", True)
    print(f"[mixed] C2 banded fp32: eig {e_eig:.3e} lmp {e_lmp:.3e}", flush=True)
    assert 0 < e_eig < 1e-3 and 0 < e_lmp < 1e-4
    # iteration counts with the reduced-precision LMP stay those of the FP64 LMP
    members = np.arange(0, cfg["members"] + 1, 8)
    it_mx = g.pcg(members, rtol=1e-6, maxit=3000)["iters"]
    g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"])
    it_64 = g.pcg(members, rtol=1e-6, maxit=3000)["iters"]
    assert (np.abs(it_mx - it_64) <= np.maximum(3, (0.05 * it_64).astype(int))).all(), (it_mx, it_64)
    g.close()


def test_reduced_precision_sketch_near_full_rank_takes_the_shift():
    # ell = 32 Gaussian sketch columns on a 40-point ring: W = Psi^T A Psi holds
    # eigenvalues far below the FP32 rounding of the products, so with FP32
    # products it is indefinite more often than not (a CPU emulation of FP32
    # rounding in Y: 3 of 5 draws).  The Nystrom shift sized by the products'
    # unit roundoff (2^-24 ||Y||_F) repairs that where the FP64-sized one
    # (2^-52 ||Y||_F) does not (the same emulation: every indefinite draw still
    # failed).  The leading eigenvalues, far above the shift, keep FP32-level
    # agreement with the FP64 oracle; the LMP still gives the FP64 solution.
    cfg = W.config("C1", members=32, ell=32, k=32, spinup=300)
    z = W.problem_normals(cfg)
    o = O.Problem(cfg, z)
    psi = W.gaussian_matrix(cfg, cfg["n"], 32)          # 32 x n: row c is column c
    S, D, info = O.nystrom(lambda V: o.A(V, [0] * V.shape[1]), psi.T, 32)
    g = eda.Problem(cfg, z)
    eig, th = g.sketch_evd("user", ell=32, k=32, mixed=True, phi=torch.from_numpy(psi).cuda())
    lead = slice(0, 5)
    e = np.abs(eig[lead] - D[lead]) / D[lead]
    print(f"[mixed] n=40 ell=32 Gaussian, FP32 products: cond(core) {info['cond_core']:.1e}; "
          f"leading eigenvalues max rel err {e.max():.1e}", flush=True)
    assert np.all(np.isfinite(eig)) and np.all(eig >= 0) and e.max() < 1e-4
    out = g.pcg(np.arange(cfg["members"] + 1), rtol=1e-10, maxit=3000)
    assert (out["status"] == eda.EDA_MEMBER_CONVERGED).all()
    ex = O.exact_solution(o, 5)
    assert np.linalg.norm(out["dz"][5].cpu().numpy() - ex) / np.linalg.norm(ex) < 1e-6
    g.close()
