"""Workload for profiling the library's GEMM kernels (for example their MFMA
counters under rocprofv3): the dense U_B product of the n = 4096 problem in
FP64 (129 member columns) and with FP32 and BF16 operands (64 sketch
columns), the block LMP (129 columns), the learned sketch's FP32 training
GEMMs (batch 64) and its BF16 inference.

    python -u -m paper_2605_23571_amd.profile_gemms
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import torch  # noqa: E402

import workloads as W  # noqa: E402
from paper_2605_23571_amd import eda  # noqa: E402
from paper_2605_23571_amd import train_sketch as T  # noqa: E402


def main():
    cfg = W.config("C3")
    g = eda.Problem(cfg, W.problem_normals(cfg), ub_mode="dense")
    n, L = cfg["n"], cfg["members"]
    X = torch.randn((L + 1, n), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    cols = torch.arange(L + 1, dtype=torch.int32, device="cuda")
    zero = torch.zeros(64, dtype=torch.int32, device="cuda")
    Xs = X[:64].contiguous(); Ys = torch.empty_like(Xs)
    for _ in range(5):
        eda.eda_hessvec(g.ctx, n, cols, X, Y, eda.EDA_HV_ADD_IDENTITY)
    for fl in (eda.EDA_HV_MIXED, eda.EDA_HV_BF16):
        for _ in range(5):
            eda.eda_hessvec(g.ctx, n, zero, Xs, Ys, fl)
    g.sketch_evd("rhs_diff", ell=64, k=64)
    for _ in range(20):
        g.lmp_apply(X)
    torch.cuda.synchronize()
    g.close()
    net = eda.MLP(T.N, T.HIDDEN, T.K, batch=64)
    net.init(W.mlp_init_normals(net.count))
    Xm = torch.randn((64, T.N), dtype=torch.float32, device="cuda")
    Sm = torch.randn((64, T.K, T.N), dtype=torch.float32, device="cuda")
    Dm = torch.rand((64, T.K), dtype=torch.float32, device="cuda")
    for _ in range(5):
        net.loss_grad(Xm, Sm, Dm)
    p16 = net.bf16()
    c2 = W.config("C2", members=4, ell=4, k=4, spinup=100)
    h = eda.Problem(c2, W.problem_normals(c2))
    dims = eda.eda_mlp_dims(T.N, T.HIDDEN, T.K)
    for _ in range(5):
        eda.mlp_infer(h, dims, p16)
    torch.cuda.synchronize()
    print("[mfma] done", flush=True)


if __name__ == "__main__":
    main()
