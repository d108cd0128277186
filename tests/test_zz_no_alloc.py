"""The allocation-free LMP entry point (eda_lmp_apply_noalloc) against
eda_lmp_apply: same kernels and summation order, so the outputs must agree bit
for bit.  Three calls in a row, each smaller than the one before (the largest
at the fixed buffer's limit), across two contexts; one request past the limit
must be refused before anything runs."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_23571_amd import eda  # noqa: E402

ROWS = 256  # rows per partial-projection block
LIMIT = eda.EDA_LMP_NOALLOC_SCRATCH_BYTES // 8


def partial_doubles(n, k, nb):
    return -(-n // ROWS) * k * 16 * -(-nb // 16)


def both(g, X, which):
    w = eda.EDA_LMP_P if which == "P" else eda.EDA_LMP_U
    ref = eda.eda_lmp_apply(g.ctx, g.n, w, X, torch.empty_like(X))
    out = torch.full_like(X, float("nan"))
    eda.eda_lmp_apply_noalloc(g.ctx, g.n, w, X, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_lmp_matches_lmp_apply():
    big = W.config("C3", nsteps=8, obs_dt=4, members=80, ell=64, k=61, spinup=100)
    small = W.config("C1", n=203, nsteps=15, obs_dt=4, obs_dx=3, obs_x0=1, members=6, ell=5, k=5, len_b=3.0,
                     spinup=300)
    n, k = big["n"], big["k"]
    nb_max = max(nb for nb in range(16, 2000, 16) if partial_doubles(n, k, nb) <= LIMIT)
    print(f"[noalloc] n={n} k={k}: largest block within the {LIMIT}-double buffer: {nb_max} columns", flush=True)
    g = eda.Problem(big, W.problem_normals(big), max_cols=nb_max + 16)
    eig, th = g.sketch_evd("rhs_diff")
    rng = np.random.default_rng(3)
    X = torch.from_numpy(rng.standard_normal((nb_max + 16, n))).cuda()
    S = g.field("S").cpu().numpy().reshape(-1, n).T
    for nb, which in ((nb_max, "P"), (17, "U")):
        ref, out = both(g, X[:nb].contiguous(), which)
        same = np.array_equal(ref, out)
        e = float(np.abs(out - O.lmp_apply(S, eig, th, X[:nb].cpu().numpy().T, which).T).max() /
                  np.abs(ref).max())
        print(f"[noalloc] n={n} nb={nb} {which}: bit-identical to eda_lmp_apply: {same}; "
              f"against the definition {e:.1e}", flush=True)
        assert same and e < 1e-13
    # one column tile past the limit: refused, output untouched
    nb_over = nb_max + 1
    assert partial_doubles(n, k, nb_over) > LIMIT
    Xo = X[:nb_over].contiguous()
    Yo = torch.full_like(Xo, 7.0)
    code = eda.lib().eda_lmp_apply_noalloc(g.ctx, eda.EDA_LMP_P, nb_over, ctypes.c_void_p(Xo.data_ptr()), n,
                                           ctypes.c_void_p(Yo.data_ptr()), n)
    torch.cuda.synchronize()
    assert code == eda.EDA_ERR_UNSUPPORTED and bool(torch.all(Yo == 7.0))
    g.close()
    # a second context on the same device (the same buffer), smaller again
    h = eda.Problem(small, W.problem_normals(small))
    h.sketch_evd("rhs_diff")
    Xs = torch.from_numpy(rng.standard_normal((7, small["n"]))).cuda()
    ref, out = both(h, Xs, "P")
    print(f"[noalloc] n={small['n']} nb=7 P: bit-identical: {np.array_equal(ref, out)}", flush=True)
    assert np.array_equal(ref, out)
    h.close()


def test_noalloc_lmp_argument_errors():
    cfg = W.config("C1")
    g = eda.Problem(cfg, W.problem_normals(cfg))
    n = cfg["n"]
    X = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    f = eda.lib().eda_lmp_apply_noalloc
    px, py = ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr())
    assert f(g.ctx, eda.EDA_LMP_P, 3, px, n, py, n) == eda.EDA_ERR_ORDER  # no sketch yet
    g.sketch_evd("rhs_diff")
    assert f(g.ctx, 7, 3, px, n, py, n) == eda.EDA_ERR_INVALID_ARG
    assert f(g.ctx, eda.EDA_LMP_P, 3, px, n - 1, py, n) == eda.EDA_ERR_INVALID_ARG
    assert f(g.ctx, eda.EDA_LMP_P, g.max_cols + 1, px, n, py, n) == eda.EDA_ERR_INVALID_ARG
    assert f(g.ctx, eda.EDA_LMP_P, 0, None, n, None, n) == eda.EDA_OK
    g.close()
