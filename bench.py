"""Benchmark: ensemble PCG solves per second at relative residual 1e-6.

One step = the hot path for one EDA problem whose inputs (trajectories,
right-hand sides, U_B) are resident in HBM: the RHS-difference (Gamma) Nystrom
sketch of the control member's Hessian (ell Hessian products + CholQR2 +
Nystrom core), the spectral LMP, and batched LMP-PCG of all L + 1 members to
||r|| <= 1e-6 ||b||.  value = members solved per second.  Problem set-up
(spin-up, trajectories, right-hand sides) is done before the timed region and
reported separately.

Forms: "chosen" = banded circulant U_B inside the fused TL/AD kernels, with the
sketch's Hessian products in FP32 (trajectory, CholQR2, eigensolve, LMP and
PCG in FP64); "plain" = dense U_B as FP64 MFMA GEMMs, FP64 throughout.  Hessian-vector products per second
(member mode: every column on its own trajectory; sketch mode: all on the
control trajectory) are reported too, and so is the time of one sketch call per
variant (Nystrom q = 1, 2, reduced precision, REVD), of one LMP application per
column count, and PCG without the LMP.

The roofline entry is for the dominant kernel, the Hessian part of a PCG
iteration (banded U_B, TL run, AD run, banded U_B, vector updates; one
workgroup per member column, or per piece of it): algorithmic bytes per active
column (pcg_kernel_bytes_per_col) x active member-iterations per launch,
divided by the kernel's average launch duration from HIP events recorded on the
launching stream around every 16th launch of the timed steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TF = 78.6
# HIP-event pairs around every 16th fused PCG launch: the average launch is
# measured inside the timed steps while the event records (which sit between
# kernels on the stream) stay out of most iterations
PROFILE_EVERY = 16
# Nystrom passes of the chosen form's sketch (Algorithm 1's q; the plain form
# runs one): at C3 the second pass lowers the longest member's PCG count from
# 660 to 628 for 64 more sketch products (about 1 ms)
CHOSEN_Q = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (dense U_B) form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-no-lmp", action="store_true", help="skip the unpreconditioned PCG leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU-baseline sample time")
    ap.add_argument("--hv-reps", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch (256 problems) measurement")
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-plain", type=int, default=64, help="problems timed through the per-problem path")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-sketch comparison")
    ap.add_argument("--learned-problems", type=int, default=256)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration; untimed)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tlad_C3_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2605_23571_amd", "csrc", "l96_tlad.hip")


def kernel_sha():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(active_per_launch):
    """HBM bytes per launch of the fused PCG kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's reading),
    or None when the summary is missing or was taken on another kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic-json: "):
            t = json.loads(line[len("traffic-json: "):])
            if t.get("kernel_sha") != kernel_sha():
                return None
            return round(t["bytes_per_active_column"] * active_per_launch)
    return None


def pcg_kernel_bytes_per_col(cfg):
    """Algorithmic HBM bytes of one member column in one launch of the Hessian
    part of a PCG iteration (whole column or split): the trajectory read by the
    TL run and again by the AD run (N states of n each), the observed
    increments written and read back (p each), and the vectors: r, z read for
    r^T z; z and the old p read for p; the new p and (I + A) p written.  The
    whole-column kernel also updates x and r (3 n more, not counted); the halos
    of a split column are recomputation, not algorithmic traffic."""
    n, N = cfg["n"], cfg["nsteps"]
    nt, nv = W.obs_counts(cfg)
    return 8 * (2 * N * n + 2 * nt * nv + 6 * n)


def run_form(cfg, z, ub_mode, steps, warmup, hv_reps, mixed=False, keep=False, q=1, lmp_form=None, xch=None):
    import torch
    from paper_2605_23571_amd import eda

    L, n, ell = cfg["members"], cfg["n"], cfg["ell"]
    t0 = time.perf_counter()
    g = eda.Problem(cfg, z, ub_mode=ub_mode)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if lmp_form is not None:
        eda.eda_set_lmp_form(g.ctx, lmp_form)
    if xch is not None:
        eda.eda_set_exchange(g.ctx, xch)
    members = np.arange(L + 1)

    def step():
        g.sketch_evd("rhs_diff", ell=ell, k=cfg["k"], q=q, mixed=mixed)
        return g.pcg(members, rtol=cfg["rtol"], maxit=cfg["maxit"], use_lmp=True)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    eda.eda_profile(g.ctx, PROFILE_EVERY)
    iters_total, outs = 0, []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
        outs.append(out)
        iters_total += int(out["iters"].sum())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed, launches, tlad_ms = eda.eda_profile_read(g.ctx)
    eda.eda_profile(g.ctx, 0)
    conv = all(bool(np.all(o["status"] == eda.EDA_MEMBER_CONVERGED)) for o in outs)
    # Hessian products per second, member mode and sketch mode
    X = torch.randn((L + 1, n), dtype=torch.float64, device="cuda")
    Xs = X[:ell].contiguous()
    cols = torch.arange(L + 1, dtype=torch.int32, device="cuda")
    zero = torch.zeros(ell, dtype=torch.int32, device="cuda")
    Y = torch.empty_like(X)
    Ys = torch.empty_like(Xs)
    hv = {}
    for name, (cc, xx, yy) in {"member_mode": (cols, X, Y), "sketch_mode": (zero, Xs, Ys)}.items():
        eda.eda_hessvec(g.ctx, n, cc, xx, yy, eda.EDA_HV_ADD_IDENTITY)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(hv_reps):
            eda.eda_hessvec(g.ctx, n, cc, xx, yy, eda.EDA_HV_ADD_IDENTITY)
        torch.cuda.synchronize()
        hv[name] = xx.shape[0] * hv_reps / (time.perf_counter() - t1)
    gemm = None
    if ub_mode == "dense":
        # the U_B GEMMs of member-mode products, each launch timed (HIP events)
        eda.eda_profile_select(g.ctx, eda.EDA_PROF_UB_GEMM)
        eda.eda_profile(g.ctx, 1)
        for _ in range(hv_reps):
            eda.eda_hessvec(g.ctx, n, cols, X, Y, eda.EDA_HV_ADD_IDENTITY)
        g_timed, _, g_ms = eda.eda_profile_read(g.ctx)
        eda.eda_profile(g.ctx, 0)
        flops = 2.0 * n * n * (L + 1)  # one n x n by n x (L + 1) product
        gemm = {"avg_launch_ms": g_ms / max(1, g_timed), "flops_per_launch": flops, "launches": g_timed}
        # the TL/AD core (a3 + a4) alone: its launches inside the same products
        eda.eda_profile_select(g.ctx, eda.EDA_PROF_TLAD_ALL)
        for name, (cc, xx, yy) in {"member_mode": (cols, X, Y), "sketch_mode": (zero, Xs, Ys)}.items():
            eda.eda_profile(g.ctx, 1)
            for _ in range(hv_reps):
                eda.eda_hessvec(g.ctx, n, cc, xx, yy, eda.EDA_HV_ADD_IDENTITY)
            t_n, _, t_ms = eda.eda_profile_read(g.ctx)
            eda.eda_profile(g.ctx, 0)
            hv[name + "_tlad_core"] = xx.shape[0] / (t_ms / max(1, t_n) / 1e3)
        eda.eda_profile_select(g.ctx, eda.EDA_PROF_TLAD)
    it = np.concatenate([o["iters"] for o in outs])
    res = dict(solves_per_s=(L + 1) * steps / dt, ms_per_step=1e3 * dt / steps, setup_s=setup_s, converged=conv,
               iters_median=float(np.median(it)), iters_max=int(it.max()), iters_min=int(it.min()),
               tlad_timed=timed, tlad_launches=launches, tlad_ms=tlad_ms, hessvec_per_s=hv,
               active_cols=iters_total, gemm=gemm)
    res["last_dz"] = outs[-1]["dz"]
    res["last_iters"] = np.asarray(outs[-1]["iters"])
    res["problem"] = g if keep else None
    if not keep:
        g.close()
    return res


def lmp_times(cfg, g, reps=200):
    """Wall time of one eda_lmp_apply (P_theta on nb columns: projection and
    expansion launches) in us, for 1, 16 and L + 1 columns, on the context's
    current sketch; the spread against nb shows whether it is latency-bound."""
    import torch
    out = {}
    for nb in (1, 16, cfg["members"] + 1):
        X = torch.randn((nb, cfg["n"]), dtype=torch.float64, device="cuda")
        for _ in range(5):
            g.lmp_apply(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.lmp_apply(X)
        torch.cuda.synchronize()
        out[str(nb)] = round(1e6 * (time.perf_counter() - t0) / reps, 2)
    return out


def copy_bandwidth(mib=1024, reps=5):
    """Attainable HBM bandwidth on this device: a plain device-to-device copy of
    `mib` MiB (read + write bytes) timed with events on torch's stream, GB/s."""
    import torch
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def no_lmp_report(cfg, g, iters_lmp):
    """PCG of every member without a preconditioner (the comparison the paper
    makes for the LMP) on the same problem and rtol: member solves per second
    over one timed call after an untimed one, and the iteration counts beside
    those of the LMP-PCG."""
    import torch
    members = np.arange(cfg["members"] + 1)
    g.pcg(members, rtol=cfg["rtol"], maxit=cfg["maxit"], use_lmp=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = g.pcg(members, rtol=cfg["rtol"], maxit=cfg["maxit"], use_lmp=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = np.asarray(out["iters"])
    from paper_2605_23571_amd import eda
    return {"value": round(members.size / dt, 3), "unit": "solves/s", "maxit": cfg["maxit"],
            "all_converged": bool(np.all(out["status"] == eda.EDA_MEMBER_CONVERGED)),
            "iters_median": float(np.median(it)), "iters_max": int(it.max()),
            "lmp_iters_median": float(np.median(iters_lmp)), "lmp_iters_max": int(np.max(iters_lmp))}


def precision_report(cfg, g, dz_chosen, oracle_lmp, iters_chosen=None):
    """Errors of the reduced-precision sketch (FP32 TL/AD products) at full size:
    against the same sketch with FP64 products on the GPU, and against the CPU
    oracle's FP64 sketch when it is available (eigenvalues D_k, the LMP operator
    on 16 seeded probes, solutions of the oracle's members at the same rtol)."""
    import torch
    rep = {}
    V = np.random.default_rng(11).standard_normal((cfg["n"], 16))
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).cuda()
    eig_mx, th_mx = g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"], q=CHOSEN_Q, mixed=True)
    P_mx = g.lmp_apply(Vt).cpu().numpy().T
    eig_64, th_64 = g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"], q=CHOSEN_Q)
    P_64 = g.lmp_apply(Vt).cpu().numpy().T
    rep["vs_gpu_fp64"] = {"eig_max_rel": float(np.max(np.abs(eig_mx - eig_64) / eig_64)),
                          "theta_rel": float(abs(th_mx - th_64) / th_64),
                          "lmp_rel": float(np.linalg.norm(P_mx - P_64) / np.linalg.norm(V))}
    if iters_chosen is not None:
        # every member solved again with the FP64 sketch's LMP: iteration change
        # and solution difference (both runs stop at the same rtol)
        out = g.pcg(np.arange(cfg["members"] + 1), rtol=cfg["rtol"], maxit=cfg["maxit"], use_lmp=True)
        d_it = np.asarray(iters_chosen) - np.asarray(out["iters"])
        dz64 = out["dz"].cpu().numpy()
        dzr = np.linalg.norm(dz_chosen - dz64, axis=1) / np.linalg.norm(dz64, axis=1)
        rep["vs_gpu_fp64"].update({"iters_delta_median": float(np.median(d_it)),
                                   "iters_delta_max_abs": int(np.max(np.abs(d_it))),
                                   "dz_rel_diff_median": float(np.median(dzr)), "dz_rel_diff_max": float(dzr.max())})
    if oracle_lmp is not None:
        from oracle import oracle as O
        S, D, th, dz_o = oracle_lmp
        P_o = O.lmp_apply(S, D, th, V)
        d = [float(np.linalg.norm(dz_chosen[m] - dz_o[m]) / np.linalg.norm(dz_o[m])) for m in range(len(dz_o))]
        rep["vs_oracle"] = {"eig_max_rel": float(np.max(np.abs(eig_mx - D) / D)),
                            "theta_rel": float(abs(th_mx - th) / th),
                            "lmp_rel": float(np.linalg.norm(P_mx - P_o) / np.linalg.norm(V)),
                            "dz_rel_diff_members": d,
                            "note": "dz: GPU (reduced-precision sketch) and oracle solutions, both stopped at "
                                    f"||r|| <= {cfg['rtol']} ||b||"}
    return rep


def sketch_times(cfg, g, reps=3):
    """Wall time of one eda_sketch_evd call at full size (RHS-difference sketch,
    ell and k of the workload), per variant, in ms: Nystrom with q = 1 and 2
    passes in FP64, the chosen reduced-precision q = 2 Nystrom, and REVD (two
    A-products and the Jacobi EVD).  Each call ends with its eigenvalues on the
    host, so the wall clock brackets the whole device work."""
    import torch
    out = {}
    variants = (("nystrom_q1_fp64", dict(q=1)), ("nystrom_q2_fp64", dict(q=2)),
                ("nystrom_q2_mixed", dict(q=2, mixed=True)), ("revd_fp64", dict(method="revd")))
    for name, kw in variants:
        g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"], **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.sketch_evd("rhs_diff", ell=cfg["ell"], k=cfg["k"], **kw)
        torch.cuda.synchronize()
        out[name] = round(1e3 * (time.perf_counter() - t0) / reps, 3)
    return out


def run_uneven_batch(count, reps, plain_count):
    """Uneven batching: `count` independent problems (n in {40,...,2048}, window
    10/20/40, 8-64 members, k = min(32, members)), every member solved to
    rtol 1e-6 with its problem's Gamma-Nystrom LMP.  Chosen: one batch (per-class
    sketch launches and the Nystrom cores in one captured graph, one persistent
    solve launch for every class in another, autotuned geometry); the first call
    tunes and captures, the timed calls replay.  Plain: the same problems one after another through
    eda_sketch_evd + eda_pcg_solve (first plain_count problems)."""
    import torch
    from paper_2605_23571_amd import eda

    cfgs = W.uneven_problems(count)
    t0 = time.perf_counter()
    probs = [eda.Problem(c, W.problem_normals(c)) for c in cfgs]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    bt = eda.Batch(probs)
    t0 = time.perf_counter()
    bt.solve(k_cap=32, rtol=1e-6, maxit=5000)
    first_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    fb = [0, 0]
    for _ in range(reps):
        f = bt.solve(k_cap=32, rtol=1e-6, maxit=5000)
        fb = [fb[0] + f[0], fb[1] + f[1]]
    dt = (time.perf_counter() - t0) / reps
    cols = sum(c["members"] + 1 for c in cfgs)
    conv, iters = True, []
    for p in range(count):
        r = bt.result(p, with_dz=False)
        conv &= bool((r["status"] == eda.EDA_MEMBER_CONVERGED).all())
        iters.append(r["iters"])
    tun = bt.tuning()
    phases = {k: round(v, 2) for k, v in bt.timing().items()}
    bt.close()
    # plain: host-driven per-problem path on the first plain_count problems
    pc = min(plain_count, count)
    pcols = sum(c["members"] + 1 for c in cfgs[:pc])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, g in zip(cfgs[:pc], probs[:pc]):
        try:
            g.sketch_evd("rhs_diff", ell=c["k"], k=c["k"])
            lmp = True
        except eda.EdaError as e:  # the same rule as the batch: no LMP where the shifted sketch fails
            if e.code != eda.EDA_ERR_NOT_SPD:
                raise
            lmp = False
        g.pcg(np.arange(c["members"] + 1), rtol=1e-6, maxit=5000, use_lmp=lmp)
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    for g in probs:
        g.close()
    it = np.concatenate(iters)
    return {"problems": count, "member_solves": cols, "value": round(cols / dt, 1), "unit": "solves/s",
            "s_per_batch": round(dt, 4), "first_call_s": round(first_s, 3), "setup_s": round(setup_s, 2),
            "all_converged": conv, "shifted_per_call": fb[0] / reps, "without_lmp_per_call": fb[1] / reps, "iters_median": float(np.median(it)), "iters_max": int(it.max()),
            "last_call_phases_ms": phases, "classes": tun,
            "plain": {"problems": pc, "member_solves": pcols, "value": round(pcols / plain_dt, 1),
                      "unit": "solves/s"}}


def run_learned(count):
    """Learned sketch vs the RHS-difference sketch on `count` test problems of
    the n = 1024 preset (64 members): sketch + LMP-PCG of every member to rtol
    1e-6 with each, timed; the committed BF16 network runs the inference."""
    import torch
    from paper_2605_23571_amd import eda
    from paper_2605_23571_amd import train_sketch as T
    net = T.load_bf16()
    if net is None:
        return None
    dims, p16 = net
    t0, _ = W.LEARNED_SPLITS["test"]
    res = {"gamma": {"t": 0.0, "iters": []}, "learned": {"t": 0.0, "iters": []}}
    used, solves = 0, 0
    for pid in range(t0, t0 + count):
        cfg = W.learned_problem(pid)
        g = eda.Problem(cfg, W.problem_normals(cfg))
        members = np.arange(cfg["members"] + 1)
        for name in ("gamma", "learned"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if name == "gamma":
                g.sketch_evd("rhs_diff", ell=32, k=32)
            else:
                used += int(eda.sketch_learned(g, dims, p16, 32)[2])
            out = g.pcg(members, rtol=1e-6, maxit=5000)
            torch.cuda.synchronize()
            res[name]["t"] += time.perf_counter() - t1
            res[name]["iters"].append(out["iters"])
        solves += members.size
        g.close()
    rep = {"problems": count, "learned_used": used, "member_solves": solves}
    for name, r in res.items():
        it = np.concatenate(r["iters"])
        rep[name] = {"solves_per_s": round(solves / r["t"], 1), "iters_median": float(np.median(it)),
                     "iters_mean": round(float(np.mean(it)), 1)}
    rep["iteration_ratio_gamma_over_learned"] = round(rep["gamma"]["iters_mean"] / rep["learned"]["iters_mean"], 3)
    # per problem: mean iterations with Gamma over mean with the learned LMP
    ratios = np.array([np.mean(a) / np.mean(b) for a, b in zip(res["gamma"]["iters"], res["learned"]["iters"])])
    rep["per_problem_ratio"] = {"median": round(float(np.median(ratios)), 4),
                                "p10": round(float(np.percentile(ratios, 10)), 4),
                                "p90": round(float(np.percentile(ratios, 90)), 4),
                                "min": round(float(ratios.min()), 4), "max": round(float(ratios.max()), 4),
                                "learned_fewer": int((ratios > 1).sum()), "gamma_fewer": int((ratios < 1).sum())}
    rep["network"] = T.load_meta().get("recipe", "eig")
    return rep


# ---------------------------------------------------------------- CPU oracle --
# The oracle is timed as it stands on the host cores: one member's PCG per
# worker process (numpy's BLAS at one thread each), members solved concurrently,
# the sketch once per problem on one core and amortised over its members.
_CPU = {}


def _cpu_member(m):
    from oracle import oracle as O
    P, cfg, S, D, th = _CPU["P"], _CPU["cfg"], _CPU["S"], _CPU["D"], _CPU["th"]
    pre = (lambda v: O.lmp_apply(S, D, th, v[:, None])[:, 0]) if S is not None else None
    t0 = time.perf_counter()
    x = O.pcg(lambda v: P.hess(v[:, None], [m])[:, 0], P.b[:, m], pre, cfg["rtol"], cfg["maxit"])[0]
    return m, x, time.perf_counter() - t0


def _cpu_workers():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _cpu_problem(O, cfg, z, q, members, workers):
    """Sketch (one core) + LMP-PCG of `members` on `workers` processes; returns
    (sketch seconds, wall seconds of the member solves, solutions, (S, D, theta))."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    P = O.Problem(cfg, z)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        try:
            S, D, _ = O.nystrom(lambda V: P.A(V, [0] * V.shape[1]), P.gamma(cfg["ell"]), cfg["k"], q)
            th = O.theta(D)
        except np.linalg.LinAlgError:  # the shifted sketch fails too: plain CG, as the library does
            S = D = th = None
        t_sketch = time.perf_counter() - t0
        _CPU.update(P=P, cfg=cfg, S=S, D=D, th=th)
        t1 = time.perf_counter()
        if workers == 1:
            res = [_cpu_member(m) for m in members]
        else:
            with mp.get_context("fork").Pool(workers) as pool:
                res = pool.map(_cpu_member, members, chunksize=1)
        wall = time.perf_counter() - t1
    return t_sketch, wall, {m: x for m, x, _ in res}, (S, D, th)


def cpu_baseline(cfg, z, target_s):
    """The CPU oracle (unchanged) on bounded samples on the host's cores:
    C3 (the metric's workload: the sketch once, amortised over the 129 members,
    then as many members as there are cores, solved concurrently), C1 and C2
    whole, and a 16-problem sample of the uneven batch (each problem's sketch
    and its first members, extrapolated to whole problems by member count).
    value: C3 solves/s on all cores; the one-core figure beside it."""
    import platform
    from oracle import oracle as O
    workers = _cpu_workers()
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    L = cfg["members"]

    def note(msg):
        print(f"[bench] CPU oracle: {msg}", file=sys.stderr, flush=True)

    # C3 sample: one member on one core, then `workers` members at once
    note(f"C3 one member on one core ({workers} cores)")
    t_sk, w1, _, _ = _cpu_problem(O, cfg, z, CHOSEN_Q, [0], 1)
    v1 = 1.0 / (t_sk / (L + 1) + w1)
    mem = list(range(min(L + 1, workers)))
    note(f"C3 {len(mem)} members at once")
    t_sk, wN, dz, lmp = _cpu_problem(O, cfg, z, CHOSEN_Q, mem, workers)
    vN = len(mem) / (t_sk * len(mem) / (L + 1) + wN)
    per = {}
    for name in ("C1", "C2"):
        note(name)
        c = W.config(name)
        zz = W.problem_normals(c)
        ts, wall, _, _ = _cpu_problem(O, c, zz, 1, list(range(c["members"] + 1)), workers)
        per[name] = {"solves_per_s": round((c["members"] + 1) / (ts + wall), 3), "sketch_s": round(ts, 3),
                     "pcg_wall_s": round(wall, 3)}
    # uneven batch: 16 problems, their sketches and first members
    probs = W.uneven_problems(256)[:16]
    tot_s, solves, full_members = 0.0, 0, 0
    per_problem = max(1, workers // 4)
    note(f"{len(probs)} problems of the uneven batch")
    for c in probs:
        zz = W.problem_normals(c)
        mem_c = list(range(min(c["members"] + 1, per_problem)))
        ts, wall, _, _ = _cpu_problem(O, c, zz, 1, mem_c, min(workers, len(mem_c)))
        # whole problem on all cores: the sketch plus its members in rounds of `workers`
        rounds = -(-(c["members"] + 1) // workers)
        tot_s += ts + wall * rounds
        solves += c["members"] + 1
    per["C4_sample"] = {"problems": len(probs), "solves_per_s_extrapolated": round(solves / tot_s, 3),
                        "note": f"each problem's sketch and first {per_problem} members timed; whole problems "
                                "extrapolated as rounds of one member per core"}
    return dict(value=vN, unit="solves/s", cores=workers, kind="oracle", value_1_core=v1, value_all_cores=vN,
                cpu=cpu, per_config=per,
                sample=f"C3: Gamma-Nystrom sketch (ell={cfg['ell']}, q={CHOSEN_Q}) once on one core, amortised over "
                       f"{L + 1} members; LMP-PCG to rtol {cfg['rtol']} of {len(mem)} members at once, one per "
                       f"process ({workers} processes, one BLAS thread each)"), (lmp[0], lmp[1], lmp[2], [dz[m] for m in sorted(dz)])


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1 (a single GPU holds one EDA "
                                   "problem's full member batch; multi-GPU member sharding is not built)"}))
        sys.exit(2)
    cfg = W.config(a.workload)
    z = W.problem_normals(cfg)
    # the CPU oracle first: its worker processes are forked before this
    # process touches the GPU
    cpu_line, oracle_lmp = None, None
    if not a.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cpu_line, oracle_lmp = cpu_baseline(cfg, z, a.cpu_seconds)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] {a.workload} chosen form (banded U_B)", file=sys.stderr, flush=True)
    chosen = run_form(cfg, z, "banded", a.steps, a.warmup, a.hv_reps, mixed=True, keep=True, q=CHOSEN_Q)
    plain = None
    if not a.no_plain:
        print(f"[bench] {a.workload} plain form (dense U_B GEMMs)", file=sys.stderr, flush=True)
        plain = run_form(cfg, z, "dense", max(1, a.steps // 2), 1 if a.warmup else 0, max(2, a.hv_reps // 4))
    # one choice at a time between the plain and the chosen form: the banded
    # U_B, the second Nystrom pass, the FP32 sketch products
    ablation = {}
    if not a.no_plain:
        from paper_2605_23571_amd import eda
        legs = (("banded_q1_fp64", dict(mixed=False, q=1)), ("banded_q2_fp64", dict(mixed=False, q=CHOSEN_Q)),
                ("chosen_lmp_one_launch", dict(mixed=True, q=CHOSEN_Q, lmp_form=eda.EDA_LMP_FORM_ONE)),
                ("chosen_independent_pieces", dict(mixed=True, q=CHOSEN_Q, xch=eda.EDA_XCH_OFF)))
        for name, kw in legs:
            print(f"[bench] {a.workload} {name}", file=sys.stderr, flush=True)
            r = run_form(cfg, z, "banded", max(1, a.steps // 2), 1 if a.warmup else 0, 2, **kw)
            ablation[name] = {"value": round(r["solves_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 3),
                              "iters_median": r["iters_median"], "all_converged": r["converged"]}
    bpc = pcg_kernel_bytes_per_col(cfg)
    # average launch from the sampled HIP-event pairs; bytes per launch from all
    # launches' active columns
    avg_ms = chosen["tlad_ms"] / max(1, chosen["tlad_timed"])
    act_per_launch = chosen["active_cols"] / max(1, chosen["tlad_launches"])
    achieved = bpc * act_per_launch / (avg_ms * 1e-3) / 1e9
    nt, nv = W.obs_counts(cfg)
    attainable = copy_bandwidth()
    line = {
        "metric": "ensemble PCG solves/s at rel-res 1e-6, plain vs chosen; Hess-vec prods/s",
        "value": round(chosen["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(chosen["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (sketch products f32)",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: Lorenz-96 n={cfg['n']}, window {cfg['nsteps']} steps, "
                               f"p={nt * nv} obs ({nt} times x {nv} vars), {cfg['members']} members + control, "
                               f"Gamma-Nystrom ell=k={cfg['k']}, LMP-PCG to rtol {cfg['rtol']}",
                   "form": f"chosen (banded circulant U_B in the fused kernels; q={CHOSEN_Q} Nystrom passes; sketch "
                           "products FP32 TL/AD, everything else FP64; plain: dense U_B GEMMs, q=1, FP64)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(act_per_launch),
                     "kernel": "k_tlad_split_sh<Q> (Hessian part of a PCG iteration: U_B, TL, AD, U_B, (I + A) p "
                               "on 2-8 pieces per column sharing the observed increments; at most half the CUs' "
                               "worth of columns run, the others wait for a free slot; k_tlad<double, Q, 3> whole "
                               "columns where pieces do not fit)",
                     "bytes_per_column": bpc, "avg_launch_ms": round(avg_ms, 4),
                     "launches": chosen["tlad_launches"], "timed_launches": chosen["tlad_timed"], "active_column_iterations": chosen["active_cols"],
                     "kernel_sha": kernel_sha(),
                     "attainable_GBs": round(attainable, 1), "frac_attainable": round(achieved / attainable, 4)},
        "pcg_iterations": {"median": chosen["iters_median"], "min": chosen["iters_min"], "max": chosen["iters_max"],
                           "all_converged": chosen["converged"]},
        "hessvec_per_s": {k: round(v, 1) for k, v in chosen["hessvec_per_s"].items()},
        "setup_s": round(chosen["setup_s"], 3),
    }
    if ablation:
        line["form_steps"] = {
            "plain: dense U_B GEMMs, q=1, FP64": line.get("plain", {}).get("value") if plain is None else
            round(plain["solves_per_s"], 3),
            "banded U_B, q=1, FP64": ablation["banded_q1_fp64"]["value"],
            f"banded U_B, q={CHOSEN_Q}, FP64": ablation["banded_q2_fp64"]["value"],
            f"chosen: banded U_B, q={CHOSEN_Q}, FP32 sketch products": round(chosen["solves_per_s"], 3),
            "chosen with the one-launch LMP (tile barriers)": ablation["chosen_lmp_one_launch"]["value"],
            "chosen with independent ring pieces (full halos, no shared observed increments)":
                ablation["chosen_independent_pieces"]["value"],
            "iters_median": {k: v["iters_median"] for k, v in ablation.items()}}
    if plain and plain.get("gemm"):
        gm = plain["gemm"]
        tf = gm["flops_per_launch"] / (gm["avg_launch_ms"] * 1e-3) / 1e12
        line["plain_roofline"] = {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TF,
                                  "unit": "TFLOP/s", "frac": round(tf / FP64_MFMA_PEAK_TF, 4),
                                  "kernel": f"k_gemm (FP64 MFMA v_mfma_f64_16x16x4f64): U_B ({cfg['n']} x {cfg['n']}) "
                                            f"times {cfg['members'] + 1} member columns, the plain form's U_B product",
                                  "flops_per_launch": gm["flops_per_launch"],
                                  "avg_launch_ms": round(gm["avg_launch_ms"], 4), "timed_launches": gm["launches"]}
    if plain:
        line["plain"] = {"value": round(plain["solves_per_s"], 3), "ms_per_step": round(plain["ms_per_step"], 3),
                         "hessvec_per_s": {k: round(v, 1) for k, v in plain["hessvec_per_s"].items()},
                         "iters_median": plain["iters_median"], "all_converged": plain["converged"]}
    if not a.no_batch:
        print(f"[bench] uneven batch of {a.batch_problems} problems", file=sys.stderr, flush=True)
        line["uneven_batch"] = run_uneven_batch(a.batch_problems, max(1, a.steps), a.batch_plain)
    if not a.no_learned:
        print("[bench] learned sketch vs RHS differences (n = 1024 test problems)", file=sys.stderr, flush=True)
        lr = run_learned(a.learned_problems)
        if lr is not None:
            line["learned_sketch"] = lr
    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line
    g = chosen["problem"]
    line["sketch_ms"] = sketch_times(cfg, g)
    line["lmp_apply_us"] = lmp_times(cfg, g)
    line["reduced_precision_sketch"] = precision_report(cfg, g, chosen["last_dz"].cpu().numpy(), oracle_lmp,
                                                        chosen["last_iters"])
    if not a.no_no_lmp:
        print("[bench] PCG without the LMP", file=sys.stderr, flush=True)
        line["no_lmp"] = no_lmp_report(cfg, g, chosen["last_iters"])
    g.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
