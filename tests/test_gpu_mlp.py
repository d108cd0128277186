"""GPU: the learned-sketch network's kernels against the FP64 oracle
(oracle/mlp_oracle.py).  FP32 training kernels: forward, loss, gradient, Adam
within FP32 rounding (bounds below); BF16 inference within a stated bound; the
learned sketch's fallback to the right-hand-side-difference sketch."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp_oracle as M
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_23571_amd import eda  # noqa: E402

DIMS = [(100, 70, 3, 5), (300, 70, 4, 5)]  # ragged tiles; the second takes the split-K path of W3^T dO


def _orth(rng, n, k):
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return q


def make_net(n, h, k, B, seed=0):
    rng = np.random.default_rng(seed)
    net = eda.MLP(n, h, k, batch=B)
    z = rng.standard_normal(net.count).astype(np.float32)
    net.init(z)
    # perturb biases too so that every parameter takes part
    p = net.params.cpu().numpy() + (0.05 * rng.standard_normal(net.count)).astype(np.float32)
    net.params.copy_(torch.from_numpy(p))
    X = M.normalise_input(rng.standard_normal((n, B))).astype(np.float32)
    Ss = [_orth(rng, n, k) for _ in range(B)]
    Ds = [np.sort(rng.uniform(0.2, 4.0, k))[::-1] for _ in range(B)]
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    St = torch.from_numpy(np.stack([s.T for s in Ss]).astype(np.float32)).cuda().contiguous()
    Dt = torch.from_numpy(np.stack(Ds).astype(np.float32)).cuda()
    theta = p.astype(np.float64)
    # the oracle sees exactly the FP32 values the GPU sees
    return net, theta, X.astype(np.float64), [s.astype(np.float32).astype(np.float64) for s in Ss], \
        [d.astype(np.float32).astype(np.float64) for d in Ds], Xt, St, Dt, z


def test_mlp_init_is_he_scaling():
    n, h, k = 100, 70, 3
    net = eda.MLP(n, h, k, batch=2)
    z = np.random.default_rng(1).standard_normal(net.count).astype(np.float32)
    net.init(z)
    ref = M.he_init(z.astype(np.float64), n, h, k)
    assert np.allclose(net.params.cpu().numpy(), ref, rtol=1e-6, atol=0)


@pytest.mark.parametrize("n,h,k,B", DIMS)
def test_mlp_forward_matches_oracle(n, h, k, B):
    net, theta, X, Ss, Ds, Xt, St, Dt, _ = make_net(n, h, k, B)
    O_gpu = net.forward(Xt).cpu().numpy().astype(np.float64)
    Z, _ = M.forward(theta, X, n, h, k)
    O_ref = np.stack([z.reshape(-1, order="F") for z in Z])
    # FP32 products of length <= n with FP32 inputs: relative 1e-5
    assert np.linalg.norm(O_gpu - O_ref) / np.linalg.norm(O_ref) < 1e-5


@pytest.mark.parametrize("n,h,k,B", DIMS)
def test_mlp_loss_and_gradient_match_oracle(n, h, k, B):
    net, theta, X, Ss, Ds, Xt, St, Dt, _ = make_net(n, h, k, B)
    loss = net.loss_grad(Xt, St, Dt)
    g = net.grad.cpu().numpy().astype(np.float64)
    loss_ref, g_ref = M.loss_and_grad(theta, X, Ss, Ds, n, h, k)
    assert loss == pytest.approx(loss_ref, rel=1e-4)
    # FP32 backward through three layers: the whole gradient within 1e-4
    # relative, and each block (W1, b1, ..., b3) within 1e-3
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-4
    for name, val in M.dims_offsets(n, h, k).items():
        if name == "total":
            continue
        off, size = val
        a, r = g[off:off + size], g_ref[off:off + size]
        assert np.linalg.norm(a - r) <= 1e-3 * np.linalg.norm(r) + 1e-12, name


def test_mlp_adam_matches_oracle():
    n, h, k, B = 100, 70, 3, 5
    net, theta, X, Ss, Ds, Xt, St, Dt, _ = make_net(n, h, k, B)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for step in range(1, 4):
        net.loss_grad(Xt, St, Dt)
        g = net.grad.cpu().numpy().astype(np.float64)
        p_before = net.params.cpu().numpy().astype(np.float64)
        net.adam(lr=1e-3)
        th_ref, m, v = M.adam_step(p_before, g, m, v, step, 1e-3)
        assert np.allclose(net.params.cpu().numpy(), th_ref, rtol=1e-5, atol=1e-7)


def test_mlp_training_reduces_loss():
    # a learnable target: the same Ritz pairs for every input
    n, h, k, B = 64, 48, 2, 16
    rng = np.random.default_rng(5)
    net = eda.MLP(n, h, k, batch=B)
    net.init(rng.standard_normal(net.count).astype(np.float32))
    S = _orth(rng, n, k)
    D = np.array([3.0, 1.0])
    St = torch.from_numpy(np.stack([S.T] * B).astype(np.float32)).cuda().contiguous()
    Dt = torch.from_numpy(np.stack([D] * B).astype(np.float32)).cuda()
    first = None
    for it in range(300):
        X = M.normalise_input(rng.standard_normal((n, B))).astype(np.float32)
        loss = net.loss_grad(torch.from_numpy(np.ascontiguousarray(X.T)).cuda(), St, Dt)
        first = loss if first is None else first
        net.adam(lr=2e-3)
    print(f"[mlp] loss {first:.3f} -> {loss:.4f}", flush=True)
    assert loss < 0.1 * first


def _case():
    cfg = W.config("C2", n=203, nsteps=12, obs_dt=3, obs_dx=2, members=8, ell=4, k=4, spinup=200, len_b=3.0)
    z = W.problem_normals(cfg)
    return cfg, z


def test_mlp_bf16_inference_bound():
    cfg, z = _case()
    n, h, k = cfg["n"], 64, 4
    g = eda.Problem(cfg, z)
    rng = np.random.default_rng(6)
    net = eda.MLP(n, h, k, batch=1)
    net.init(rng.standard_normal(net.count).astype(np.float32))
    Zg = eda.mlp_infer(g, net.dims, net.bf16()).cpu().numpy().T  # n x k
    o = O.Problem(cfg, z)
    x = M.normalise_input(o.b[:, 0])
    Zr, _ = M.forward(net.params.cpu().numpy().astype(np.float64), x, n, h, k)
    err = np.linalg.norm(Zg - Zr[0]) / np.linalg.norm(Zr[0])
    # BF16 weights and activations (2^-9 each), FP32 accumulation, three layers
    print(f"[mlp] bf16 inference rel err {err:.2e}", flush=True)
    assert 1e-4 < err < 5e-2
    # the FP32 input matches the definition
    xin = eda.mlp_input(g).cpu().numpy()
    assert np.allclose(xin, x[:, 0], rtol=1e-6)
    g.close()


def test_sketch_learned_and_fallback():
    cfg, z = _case()
    n, h, k = cfg["n"], 64, 4
    g = eda.Problem(cfg, z)
    # zero network: Z = 0, the CholQR of Phi fails -> the RHS-difference sketch
    net0 = eda.MLP(n, h, k, batch=1)
    eig0, th0, used0 = eda.sketch_learned(g, net0.dims, net0.bf16(), k)
    assert not used0
    eig_g, th_g = g.sketch_evd("rhs_diff", ell=k, k=k)
    assert np.array_equal(eig0, eig_g) and th0 == th_g
    # a random network gives a valid sketch: PCG reaches the exact solution
    net = eda.MLP(n, h, k, batch=1)
    net.init(np.random.default_rng(8).standard_normal(net.count).astype(np.float32))
    eig, th, used = eda.sketch_learned(g, net.dims, net.bf16(), k)
    assert used and np.all(np.isfinite(eig)) and np.all(eig >= 0)
    out = g.pcg([0, 3], rtol=1e-10, maxit=2000)
    o = O.Problem(cfg, z)
    dz = out["dz"].cpu().numpy()
    for i, m in enumerate([0, 3]):
        ex = O.exact_solution(o, m)
        assert np.linalg.norm(dz[i] - ex) / np.linalg.norm(ex) < 1e-6
    g.close()
