"""Thin Python binding of the C ABI in include/eda.h (libeda.so).

Argument marshalling only: every function here forwards to the HIP library
with raw device pointers taken from torch tensors; torch provides device
memory and the current HIP stream.  Importing works anywhere; any call that
needs the library raises if libeda.so is missing, and device calls raise if no
GPU is visible -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeda.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "eda.h")

# ---- constants (values from include/eda.h) ----
EDA_OK = 0
EDA_ERR_INVALID_ARG = -1
EDA_ERR_WORKSPACE = -2
EDA_ERR_HIP = -3
EDA_ERR_NOT_SPD = -4
EDA_ERR_ORDER = -5
EDA_ERR_UNSUPPORTED = -6
EDA_ERR_SYNC = -7
EDA_WARN_NOT_CONVERGED = 1
EDA_MEMBER_CONVERGED, EDA_MEMBER_NOT_CONVERGED, EDA_MEMBER_BREAKDOWN = 0, 1, 2
EDA_UB_DENSE, EDA_UB_BANDED = 0, 1
EDA_B_GAUSS, EDA_B_DIFFUSION = 0, 1
EDA_HV_ADD_IDENTITY, EDA_HV_MIXED, EDA_HV_BF16 = 1, 2, 4
EDA_SKETCH_RHS_DIFF, EDA_SKETCH_USER, EDA_SKETCH_B_PSI, EDA_SKETCH_UBT_PSI = 0, 1, 2, 3
EDA_METHOD_NYSTROM, EDA_METHOD_REVD = 0, 1
EDA_THETA_MID, EDA_THETA_LAMK, EDA_THETA_ONE = 0, 1, 2
EDA_LMP_P, EDA_LMP_U = 0, 1
EDA_XCH_OFF, EDA_XCH_ON, EDA_XCH_OBS = 0, 1, 2
EDA_LMP_FORM_TWO, EDA_LMP_FORM_ONE = 0, 1
EDA_PROF_TLAD, EDA_PROF_UB_GEMM, EDA_PROF_TLAD_ALL = 0, 1, 2
EDA_LMP_NOALLOC_SCRATCH_BYTES = 4194304
FIELDS = dict(truth=0, xb=1, traj=2, y=3, d=4, b=5, costc=6, ubrow=7, S=8, eig=9)
EDA_FIELD_SKETCH_INFO = 10
THETA_RULES = {"mid": EDA_THETA_MID, "lamk": EDA_THETA_LAMK, "one": EDA_THETA_ONE}


class EdaError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {code} ({strerror(code)})")
        self.code = code


class eda_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nsteps", ctypes.c_int32), ("F", ctypes.c_double),
                ("dt", ctypes.c_double), ("spinup", ctypes.c_int32), ("spin_pert_std", ctypes.c_double),
                ("obs_dt", ctypes.c_int32), ("obs_dx", ctypes.c_int32), ("obs_x0", ctypes.c_int32),
                ("sigma_o", ctypes.c_double), ("sigma_b", ctypes.c_double), ("len_b", ctypes.c_double),
                ("members", ctypes.c_int32), ("max_ell", ctypes.c_int32), ("max_cols", ctypes.c_int32),
                ("ub_mode", ctypes.c_int32), ("b_kind", ctypes.c_int32), ("diff_steps", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libeda.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2605_23571_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64, dbl, u32 = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_uint32)
        cfgp = ctypes.POINTER(eda_config)
        sigs = {
            "eda_workspace_bytes": [cfgp, ctypes.POINTER(sz)],
            "eda_normals_count": [cfgp, ctypes.POINTER(i64)],
            "eda_setup": [cfgp, vp, vp, sz, vp, ctypes.POINTER(vp)],
            "eda_hessvec": [vp, vp, i32, vp, i64, vp, i64, u32],
            "eda_sketch_evd": [vp, i32, vp, i64, i32, i32, i32, i32, i32, u32, vp, vp],
            "eda_lmp_apply": [vp, i32, i32, vp, i64, vp, i64],
            "eda_lmp_apply_noalloc": [vp, i32, i32, vp, i64, vp, i64],
            "eda_pcg_solve": [vp, vp, i32, dbl, i32, i32, vp, i64, vp, vp, vp, vp],
            "eda_field": [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(i64)],
            "eda_profile": [vp, i32],
            "eda_profile_read": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(dbl)],
            "eda_profile_select": [vp, i32],
            "eda_destroy": [vp],
            "eda_set_geometry": [vp, i32, i32],
            "eda_set_split": [vp, i32],
            "eda_set_exchange": [vp, i32, i64],
            "eda_set_lmp_form": [vp, i32],
            "eda_mlp_param_count": [vp, ctypes.POINTER(i64)],
            "eda_mlp_workspace_bytes": [vp, i32, ctypes.POINTER(sz)],
            "eda_mlp_init": [vp, vp, vp, vp],
            "eda_mlp_forward": [vp, i32, vp, vp, vp, vp, sz, vp],
            "eda_mlp_loss_grad": [vp, i32, vp, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(dbl)],
            "eda_mlp_adam": [i64, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, vp],
            "eda_mlp_to_bf16": [i64, vp, vp, vp],
            "eda_mlp_input": [vp, vp],
            "eda_mlp_infer": [vp, vp, vp, vp],
            "eda_sketch_learned": [vp, vp, vp, i32, i32, vp, vp, vp],
            "eda_strerror": [ctypes.c_int],
            "eda_batch_workspace_bytes": [vp, i32, ctypes.POINTER(sz)],
            "eda_batch_create": [vp, i32, vp, sz, vp, ctypes.POINTER(vp)],
            "eda_batch_solve": [vp, i32, dbl, i32, i32, vp],
            "eda_batch_result": [vp, i32, vp, i64, vp, vp, vp],
            "eda_batch_tuning": [vp, i32, vp],
            "eda_batch_timing": [vp, vp],
            "eda_batch_destroy": [vp],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name == "eda_strerror" else ctypes.c_int
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/eda.h."""
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(eda_\w+)\s*\(", txt, flags=re.M)))


def strerror(code: int) -> str:
    return lib().eda_strerror(int(code)).decode()


def _check(fn: str, code: int, ok=(EDA_OK,)):
    if code not in ok:
        raise EdaError(fn, code)
    return code


def make_config(cfg: dict, ub_mode: str = "banded", max_ell: int | None = None, max_cols: int = 0) -> eda_config:
    """eda_config from a workload dict (keys as in workloads.CONFIGS)."""
    return eda_config(cfg["n"], cfg["nsteps"], cfg["F"], cfg["dt"], cfg["spinup"], cfg["spin_pert_std"],
                      cfg["obs_dt"], cfg["obs_dx"], cfg["obs_x0"], cfg["sigma_o"], cfg["sigma_b"], cfg["len_b"],
                      cfg["members"], int(max_ell if max_ell is not None else cfg.get("ell", 1)), int(max_cols),
                      EDA_UB_DENSE if ub_mode == "dense" else EDA_UB_BANDED,
                      EDA_B_DIFFUSION if cfg.get("b_kind", "gauss") == "diffusion" else EDA_B_GAUSS,
                      int(cfg.get("diff_steps", 0)))


def eda_workspace_bytes(c: eda_config) -> int:
    out = ctypes.c_size_t()
    _check("eda_workspace_bytes", lib().eda_workspace_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def eda_normals_count(c: eda_config) -> int:
    out = ctypes.c_int64()
    _check("eda_normals_count", lib().eda_normals_count(ctypes.byref(c), ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------- device ----
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the EDA library runs on the GPU only")
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev_f64(t, rows: int):
    """(pointer, ld) of a [cols, rows] float64 CUDA tensor whose rows are contiguous; ld = the
    stride between columns (>= rows), so a column slice of a wider buffer passes as is."""
    torch = _torch()
    ok = t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.shape[1] == rows
    if ok and t.shape[0] > 1 and rows > 0:
        ok = t.stride(1) == 1 and t.stride(0) >= rows
    elif ok:
        ok = t.is_contiguous()
    if not ok:
        raise ValueError(f"expected a float64 CUDA tensor of shape [cols, {rows}] with contiguous rows")
    return ctypes.c_void_p(t.data_ptr()), (t.stride(0) if t.shape[0] > 1 and rows > 0 else rows)


def eda_setup(c: eda_config, normals, ws):
    """Set up a problem in workspace `ws` (uint8 CUDA tensor); returns the ctx handle."""
    torch = _torch()
    if not (normals.is_cuda and normals.dtype == torch.float64 and normals.is_contiguous()):
        raise ValueError("normals must be a contiguous float64 CUDA tensor")
    if normals.numel() != eda_normals_count(c):
        raise ValueError("normals has the wrong length")
    ctx = ctypes.c_void_p()
    _check("eda_setup", lib().eda_setup(ctypes.byref(c), ctypes.c_void_p(normals.data_ptr()),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(), ctypes.byref(ctx)))
    return ctx


def eda_hessvec(ctx, n: int, col_member, X, Y, flags: int = 0):
    px, ldx = _dev_f64(X, n)
    py, ldy = _dev_f64(Y, n)
    _check("eda_hessvec", lib().eda_hessvec(ctx, ctypes.c_void_p(col_member.data_ptr()), X.shape[0], px, ldx,
                                            py, ldy, flags))
    return Y


def eda_sketch_evd(ctx, n: int, kind: int, phi, ell: int, k: int, q: int = 1, method: int = EDA_METHOD_NYSTROM,
                   theta_rule: int = EDA_THETA_MID, flags: int = 0):
    eig = np.zeros(k)
    th = ctypes.c_double()
    if phi is not None:
        pphi, ldphi = _dev_f64(phi, n)
    else:
        pphi, ldphi = ctypes.c_void_p(), n
    _check("eda_sketch_evd", lib().eda_sketch_evd(ctx, kind, pphi, ldphi, ell, k, q, method, theta_rule, flags,
                                                  eig.ctypes.data_as(ctypes.c_void_p), ctypes.byref(th)))
    return eig, th.value


def eda_lmp_apply(ctx, n: int, which: int, X, Y):
    px, ldx = _dev_f64(X, n)
    py, ldy = _dev_f64(Y, n)
    _check("eda_lmp_apply", lib().eda_lmp_apply(ctx, which, X.shape[0], px, ldx, py, ldy))
    return Y


def eda_lmp_apply_noalloc(ctx, n: int, which: int, X, Y):
    px, ldx = _dev_f64(X, n)
    py, ldy = _dev_f64(Y, n)
    _check("eda_lmp_apply_noalloc", lib().eda_lmp_apply_noalloc(ctx, which, X.shape[0], px, ldx, py, ldy))
    return Y


def eda_pcg_solve(ctx, n: int, members, rtol: float, maxit: int, use_lmp: bool, DZ, history: bool = False):
    members = np.ascontiguousarray(members, dtype=np.int32)
    nm = members.size
    pdz, ldz = _dev_f64(DZ, n)
    iters = np.zeros(nm, dtype=np.int32)
    relres = np.zeros(nm)
    status = np.zeros(nm, dtype=np.int32)
    hist = np.full((nm, maxit + 1), np.nan) if history else None
    code = lib().eda_pcg_solve(ctx, members.ctypes.data_as(ctypes.c_void_p), nm, float(rtol), int(maxit),
                               int(bool(use_lmp)), pdz, ldz, iters.ctypes.data_as(ctypes.c_void_p),
                               relres.ctypes.data_as(ctypes.c_void_p), status.ctypes.data_as(ctypes.c_void_p),
                               hist.ctypes.data_as(ctypes.c_void_p) if history else None)
    _check("eda_pcg_solve", code, ok=(EDA_OK, EDA_WARN_NOT_CONVERGED))
    return dict(iters=iters, relres=relres, status=status, hist=hist, code=code)


def eda_field(ctx, field: int):
    off, cnt = ctypes.c_size_t(), ctypes.c_int64()
    _check("eda_field", lib().eda_field(ctx, field, ctypes.byref(off), ctypes.byref(cnt)))
    return off.value, cnt.value


def eda_profile(ctx, every: int):
    """Time every `every`-th TL/AD launch of eda_pcg_solve (0: off; True: each)."""
    _check("eda_profile", lib().eda_profile(ctx, int(every)))


def eda_profile_read(ctx):
    """(timed launches, all launches, summed duration of the timed ones in ms)"""
    t, n, ms = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check("eda_profile_read", lib().eda_profile_read(ctx, ctypes.byref(t), ctypes.byref(n), ctypes.byref(ms)))
    return t.value, n.value, ms.value


def eda_profile_select(ctx, kind: int):
    _check("eda_profile_select", lib().eda_profile_select(ctx, int(kind)))


def eda_set_geometry(ctx, waves: int, tb: int):
    _check("eda_set_geometry", lib().eda_set_geometry(ctx, int(waves), int(tb)))


def eda_set_exchange(ctx, mode: int, spin_limit: int = -1):
    _check("eda_set_exchange", lib().eda_set_exchange(ctx, int(mode), int(spin_limit)))


def eda_set_lmp_form(ctx, form: int):
    _check("eda_set_lmp_form", lib().eda_set_lmp_form(ctx, int(form)))


def eda_set_split(ctx, pieces: int):
    """Pieces per member column in split PCG iterations (0: automatic)."""
    _check("eda_set_split", lib().eda_set_split(ctx, int(pieces)))


def eda_destroy(ctx):
    _check("eda_destroy", lib().eda_destroy(ctx))


def eda_batch_workspace_bytes(ctxs) -> int:
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    out = ctypes.c_size_t()
    _check("eda_batch_workspace_bytes", lib().eda_batch_workspace_bytes(arr, len(ctxs), ctypes.byref(out)))
    return out.value


def eda_batch_create(ctxs, ws):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    b = ctypes.c_void_p()
    _check("eda_batch_create", lib().eda_batch_create(arr, len(ctxs), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                      _stream(), ctypes.byref(b)))
    return b


def eda_batch_solve(batch, k_cap: int, rtol: float, maxit: int, use_lmp: bool = True) -> tuple[int, int]:
    """Returns (problems whose last Nystrom pass took a shift, of those left without LMP)."""
    fb = (ctypes.c_int32 * 2)()
    _check("eda_batch_solve", lib().eda_batch_solve(batch, int(k_cap), float(rtol), int(maxit), int(bool(use_lmp)),
                                                    fb), ok=(EDA_OK, EDA_WARN_NOT_CONVERGED))
    return int(fb[0]), int(fb[1])


def eda_batch_result(batch, p: int, n: int, m: int, DZ=None):
    iters = np.zeros(m, dtype=np.int32)
    relres = np.zeros(m)
    status = np.zeros(m, dtype=np.int32)
    if DZ is not None:
        pdz, ldz = _dev_f64(DZ, n)
    else:
        pdz, ldz = ctypes.c_void_p(), n
    code = lib().eda_batch_result(batch, int(p), pdz, ldz, iters.ctypes.data_as(ctypes.c_void_p),
                                  relres.ctypes.data_as(ctypes.c_void_p), status.ctypes.data_as(ctypes.c_void_p))
    _check("eda_batch_result", code, ok=(EDA_OK, EDA_WARN_NOT_CONVERGED))
    return dict(iters=iters, relres=relres, status=status, dz=DZ)


def eda_batch_tuning(batch) -> list[dict]:
    out = (ctypes.c_int32 * 11)()
    ncls = lib().eda_batch_tuning(batch, 0, out)
    _check("eda_batch_tuning", min(ncls, 0))
    res = []
    for c in range(ncls):
        lib().eda_batch_tuning(batch, c, out)
        res.append(dict(zip(["n", "problems", "waves", "q", "tb", "grid", "columns", "tune_us", "sketch_waves",
                             "sketch_q", "sketch_tb"], list(out))))
    return res


def eda_batch_timing(batch) -> dict:
    out = (ctypes.c_double * 3)()
    _check("eda_batch_timing", lib().eda_batch_timing(batch, out))
    return dict(sketch_ms=out[0], prelude_ms=out[1], solve_ms=out[2])


def eda_batch_destroy(batch):
    _check("eda_batch_destroy", lib().eda_batch_destroy(batch))


class eda_mlp_dims(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("hidden", ctypes.c_int32), ("k", ctypes.c_int32)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class MLP:
    """The learned-sketch network's parameters on the GPU and its training
    calls (FP32 forward/backward, Adam) and BF16 inference."""

    def __init__(self, n: int, hidden: int = 256, k: int = 32, batch: int = 64):
        torch = _torch()
        self.dims = eda_mlp_dims(n, hidden, k)
        cnt = ctypes.c_int64()
        _check("eda_mlp_param_count", lib().eda_mlp_param_count(ctypes.byref(self.dims), ctypes.byref(cnt)))
        self.count = cnt.value
        self.batch = batch
        wsb = ctypes.c_size_t()
        _check("eda_mlp_workspace_bytes", lib().eda_mlp_workspace_bytes(ctypes.byref(self.dims), batch,
                                                                        ctypes.byref(wsb)))
        self.ws = torch.empty(wsb.value, dtype=torch.uint8, device="cuda")
        self.params = torch.zeros(self.count, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0

    def init(self, normals):
        torch = _torch()
        z = torch.as_tensor(np.ascontiguousarray(normals, dtype=np.float32)).cuda()
        _check("eda_mlp_init", lib().eda_mlp_init(ctypes.byref(self.dims), _ptr(z), _ptr(self.params), _stream()))

    def forward(self, X):
        torch = _torch()
        B = X.shape[0]
        assert B <= self.batch and X.dtype == torch.float32 and X.is_contiguous()
        O = torch.empty((B, self.dims.k * self.dims.n), dtype=torch.float32, device="cuda")
        _check("eda_mlp_forward", lib().eda_mlp_forward(ctypes.byref(self.dims), B, _ptr(self.params), _ptr(X),
                                                        _ptr(O), _ptr(self.ws), self.ws.numel(), _stream()))
        return O

    def loss_grad(self, X, S, D, want_grad: bool = True) -> float:
        """X: [B, n] FP32; S: [B, k, n] (column j of sample b = S[b, j]); D: [B, k]."""
        B = X.shape[0]
        assert B <= self.batch
        loss = ctypes.c_double()
        _check("eda_mlp_loss_grad", lib().eda_mlp_loss_grad(ctypes.byref(self.dims), B, _ptr(self.params), _ptr(X),
                                                            _ptr(S), _ptr(D),
                                                            _ptr(self.grad) if want_grad else None, _ptr(self.ws),
                                                            self.ws.numel(), _stream(), ctypes.byref(loss)))
        return loss.value

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        _check("eda_mlp_adam", lib().eda_mlp_adam(self.count, _ptr(self.params), _ptr(self.grad), _ptr(self.m),
                                                  _ptr(self.v), self.step, lr, beta1, beta2, eps, _stream()))

    def bf16(self):
        torch = _torch()
        p16 = torch.empty(self.count, dtype=torch.int16, device="cuda")
        _check("eda_mlp_to_bf16", lib().eda_mlp_to_bf16(self.count, _ptr(self.params), _ptr(p16), _stream()))
        return p16


def mlp_input(problem) -> "torch.Tensor":
    torch = _torch()
    x = torch.empty(problem.n, dtype=torch.float32, device="cuda")
    _check("eda_mlp_input", lib().eda_mlp_input(problem.ctx, _ptr(x)))
    return x


def mlp_infer(problem, dims: eda_mlp_dims, params16):
    torch = _torch()
    Z = torch.empty((dims.k, dims.n), dtype=torch.float64, device="cuda")
    _check("eda_mlp_infer", lib().eda_mlp_infer(problem.ctx, ctypes.byref(dims), _ptr(params16), _ptr(Z)))
    return Z


def sketch_learned(problem, dims: eda_mlp_dims, params16, k: int, theta: str = "mid"):
    """Returns (eigenvalues, theta, used_learned)."""
    eig = np.zeros(k)
    th = ctypes.c_double()
    used = ctypes.c_int32()
    _check("eda_sketch_learned", lib().eda_sketch_learned(problem.ctx, ctypes.byref(dims), _ptr(params16), k,
                                                          THETA_RULES[theta], eig.ctypes.data_as(ctypes.c_void_p),
                                                          ctypes.byref(th), ctypes.byref(used)))
    return eig, th.value, bool(used.value)


def _lowp_flag(mixed) -> int:
    """False: FP64; True or "fp32": EDA_HV_MIXED; "bf16": EDA_HV_BF16."""
    if mixed == "bf16":
        return EDA_HV_BF16
    return EDA_HV_MIXED if mixed else 0


class Batch:
    """Many Problems solved together (sketch, Nystrom, LMP-PCG of every member)."""

    def __init__(self, problems: list):
        torch = _torch()
        self.problems = list(problems)
        ctxs = [p.ctx for p in self.problems]
        self.ws = torch.empty(eda_batch_workspace_bytes(ctxs), dtype=torch.uint8, device="cuda")
        self.b = eda_batch_create(ctxs, self.ws)

    def solve(self, k_cap: int, rtol: float, maxit: int, use_lmp: bool = True) -> tuple[int, int]:
        return eda_batch_solve(self.b, k_cap, rtol, maxit, use_lmp)

    def result(self, p: int, with_dz: bool = True):
        torch = _torch()
        pr = self.problems[p]
        m = pr.cfg["members"] + 1
        DZ = torch.empty((m, pr.n), dtype=torch.float64, device="cuda") if with_dz else None
        return eda_batch_result(self.b, p, pr.n, m, DZ)

    def tuning(self) -> list[dict]:
        return eda_batch_tuning(self.b)

    def timing(self) -> dict:
        return eda_batch_timing(self.b)

    def close(self):
        if self.b:
            eda_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """One EDA problem on the GPU: owns its workspace tensor and context."""

    def __init__(self, cfg: dict, normals: np.ndarray, ub_mode: str = "banded", max_ell: int | None = None,
                 max_cols: int = 0):
        torch = _torch()
        self.cfg = dict(cfg)
        self.n = cfg["n"]
        self.c = make_config(cfg, ub_mode, max_ell, max_cols)
        self.ws = torch.empty(eda_workspace_bytes(self.c), dtype=torch.uint8, device="cuda")
        self.normals = torch.as_tensor(np.ascontiguousarray(normals, dtype=np.float64)).cuda()
        self.ctx = eda_setup(self.c, self.normals, self.ws)
        self.max_cols = self.c.max_cols if self.c.max_cols > 0 else max(cfg["members"] + 1, 2 * self.c.max_ell)

    def field(self, name: str):
        """A float64 view into the workspace (no copy)."""
        torch = _torch()
        off, cnt = eda_field(self.ctx, FIELDS[name])
        return self.ws[off:off + 8 * cnt].view(torch.float64)

    def sketch_info(self) -> np.ndarray:
        """The last Nystrom sketch's outcomes: the three unshifted Cholesky
        results, whether the shifted pass ran, whether it failed."""
        torch = _torch()
        off, cnt = eda_field(self.ctx, EDA_FIELD_SKETCH_INFO)
        return self.ws[off:off + 4 * cnt].view(torch.int32).cpu().numpy()

    def hessvec(self, members, X, add_identity: bool = False, mixed: bool = False):
        torch = _torch()
        cols = torch.as_tensor(np.asarray(members, dtype=np.int32)).cuda()
        Y = torch.empty_like(X)
        flags = (EDA_HV_ADD_IDENTITY if add_identity else 0) | _lowp_flag(mixed)
        return eda_hessvec(self.ctx, self.n, cols, X, Y, flags)

    def sketch_evd(self, kind: str = "rhs_diff", ell: int | None = None, k: int | None = None, q: int = 1,
                   method: str = "nystrom", theta: str = "mid", phi=None, mixed: bool = False):
        kinds = dict(rhs_diff=EDA_SKETCH_RHS_DIFF, user=EDA_SKETCH_USER, b_psi=EDA_SKETCH_B_PSI,
                     ubt_psi=EDA_SKETCH_UBT_PSI)
        ell = ell or self.cfg["ell"]
        k = k or self.cfg["k"]
        return eda_sketch_evd(self.ctx, self.n, kinds[kind], phi, ell, k, q,
                              EDA_METHOD_NYSTROM if method == "nystrom" else EDA_METHOD_REVD, THETA_RULES[theta],
                              _lowp_flag(mixed))

    def lmp_apply(self, X, which: str = "P"):
        torch = _torch()
        Y = torch.empty_like(X)
        return eda_lmp_apply(self.ctx, self.n, EDA_LMP_P if which == "P" else EDA_LMP_U, X, Y)

    def pcg(self, members, rtol: float, maxit: int, use_lmp: bool = True, history: bool = False):
        torch = _torch()
        members = np.asarray(members, dtype=np.int32)
        DZ = torch.empty((members.size, self.n), dtype=torch.float64, device="cuda")
        out = eda_pcg_solve(self.ctx, self.n, members, rtol, maxit, use_lmp, DZ, history)
        out["dz"] = DZ
        return out

    def close(self):
        if self.ctx:
            eda_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
