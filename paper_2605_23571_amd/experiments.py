"""The numerical experiments of the paper's Sec. 4 on the GPU library.

Runs the studies of the numerical-experiments section with the library's own
calls (eda_setup, eda_hessvec, eda_sketch_evd, eda_pcg_solve) on the paper's
set-up (Lorenz-96, n = 1500, ten-step window, p = 150, sigma_o = 0.05,
sigma_b = 0.8, the diffusion-based B, L = ell = 20):

  e1  spectrum of I + A for several diffusion parameters D and M (Sec. 4,
      eigenvalue sensitivity to B): the 150 largest eigenvalues;
  e2  relative error of the eigenvalues of I + A that Algorithm 1 returns for
      the five sketching matrices Psi, A Psi (q = 2), B Psi, U_B^T Psi and
      Gamma, against a dense eigensolve; median over random initialisations
      (Sec. 4, randomized LMPs for the control member, eigenvalue figure);
  e3  the quadratic cost J of the control's LMP-PCG against the iteration and
      against the number of A-products (sketch included), median over the
      initialisations, for the five sketches and without LMP (cost figure);
  e4  sensitivity of the Gamma LMP to theta ((lambda_k + 1)/2, lambda_k, 1)
      and to oversampling (k = 20 or 15 of ell = 20): median, minimum and
      maximum of J over the initialisations, and J without LMP;
  e5  the members: the ratio J(no LMP) / J(LMP) per member and iteration for
      one ensemble instance, median, minimum and maximum over the members
      (Sec. 4, randomized LMPs for the ensemble members).

An initialisation is a fresh Gaussian Psi and a fresh ensemble (the members'
background and observation perturbations); the control problem stays the
same, so its Hessian A and the dense reference are computed once.  The dense
reference assembles A from the library's FP64 Hessian products on the unit
vectors and takes numpy's symmetric eigensolver.

    python -m paper_2605_23571_amd.experiments --out results.json [--inits 20]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import workloads as W  # noqa: E402
from paper_2605_23571_amd import eda  # noqa: E402

SKETCHES = ("psi", "a_psi", "b_psi", "ubt_psi", "gamma")


def _torch():
    import torch
    return torch


def dense_hessian(g: eda.Problem, chunk: int | None = None) -> np.ndarray:
    """A of the control member (sketch mode) from Hessian products with the
    unit vectors, symmetrised."""
    torch = _torch()
    n = g.n
    chunk = chunk or g.max_cols
    A = np.empty((n, n))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        E = torch.zeros((c1 - c0, n), dtype=torch.float64, device="cuda")
        E[torch.arange(c1 - c0), torch.arange(c0, c1)] = 1.0
        A[:, c0:c1] = g.hessvec(np.zeros(c1 - c0, dtype=np.int32), E).cpu().numpy().T
    return 0.5 * (A + A.T)


def reference_eigs(cfg: dict, count: int) -> np.ndarray:
    """The `count` largest eigenvalues of I + A for the control of `cfg`."""
    g = eda.Problem(cfg, W.problem_normals(cfg), max_cols=min(cfg["n"], 512))
    lam = np.linalg.eigvalsh(dense_hessian(g))[::-1][:count]
    g.close()
    return 1.0 + lam


def sketch(g: eda.Problem, kind: str, ell: int, k: int, psi, theta: str = "mid"):
    """(eigenvalues of A, theta) from Algorithm 1 with one of the five sketching
    matrices; psi: the Gaussian Psi (ell x n CUDA tensor, row c = column c)."""
    if kind == "gamma":
        return g.sketch_evd("rhs_diff", ell=ell, k=k, theta=theta)
    if kind == "psi":
        return g.sketch_evd("user", ell=ell, k=k, theta=theta, phi=psi)
    if kind == "a_psi":
        return g.sketch_evd("user", ell=ell, k=k, q=2, theta=theta, phi=psi)
    return g.sketch_evd(kind, ell=ell, k=k, theta=theta, phi=psi)


def sketch_products(kind: str) -> int:
    """A-products of a sketch, counting one batched product as one (Sec. 4)."""
    return 2 if kind == "a_psi" else 1


def cost_history(g: eda.Problem, members, iters: int, use_lmp: bool) -> np.ndarray:
    """J_i for i = 0..iters of LMP-PCG (or CG) of `members` (rows)."""
    out = g.pcg(np.asarray(members), rtol=0.0, maxit=iters, use_lmp=use_lmp, history=True)
    c = g.field("costc").cpu().numpy()[np.asarray(members)]
    J = out["hist"][:, :iters + 1] + c[:, None]
    # after a breakdown (the residual at rounding level) J stays where it is
    for row in J:
        bad = ~np.isfinite(row)
        if bad.any():
            first = int(np.argmax(bad))
            row[first:] = row[first - 1]
    return J


def e1_spectrum(base: dict, Ds=(2.0, 4.0, 6.0, 8.0), Ms=(4, 6, 10, 20), count: int = 150) -> dict:
    res = {"D_at_M10": {}, "M_at_D6": {}}
    for D in Ds:
        res["D_at_M10"][str(D)] = reference_eigs(dict(base, len_b=D, diff_steps=10), count).tolist()
    for M in Ms:
        res["M_at_D6"][str(M)] = reference_eigs(dict(base, len_b=6.0, diff_steps=M), count).tolist()
    return res


def e2_to_e4(cfg: dict, inits: int, iters: int, ref: np.ndarray) -> dict:
    torch = _torch()
    n, ell, k = cfg["n"], cfg["ell"], cfg["k"]
    err = {s: [] for s in SKETCHES}
    eigs = {s: [] for s in SKETCHES}
    J = {s: [] for s in SKETCHES}
    sens = {f"{th}_k{kk}": [] for th in ("mid", "lamk", "one") for kk in (k, k - 5)}
    J_none = None
    for i in range(inits):
        g = eda.Problem(cfg, W.ensemble_normals(cfg, i))
        psi = torch.from_numpy(W.gaussian_matrix(cfg, n, ell, draw=i)).cuda()
        if J_none is None:
            J_none = cost_history(g, [0], iters, False)[0]
        for s in SKETCHES:
            eig, _ = sketch(g, s, ell, k, psi)
            lam = 1.0 + eig
            err[s].append(np.abs(ref[:k] - lam) / ref[:k])
            eigs[s].append(eig.tolist())
            J[s].append(cost_history(g, [0], iters, True)[0])
        for th in ("mid", "lamk", "one"):
            for kk in (k, k - 5):
                sketch(g, "gamma", ell, kk, psi, theta=th)
                sens[f"{th}_k{kk}"].append(cost_history(g, [0], iters, True)[0])
        g.close()
    e2 = {s: np.median(np.array(err[s]), axis=0).tolist() for s in SKETCHES}
    e3 = {s: {"median_J": np.median(np.array(J[s]), axis=0).tolist(), "sketch_products": sketch_products(s)}
          for s in SKETCHES}
    e3["none"] = {"median_J": J_none.tolist(), "sketch_products": 0}
    e4 = {key: {"median": np.median(np.array(v), axis=0).tolist(), "min": np.min(np.array(v), axis=0).tolist(),
                "max": np.max(np.array(v), axis=0).tolist()} for key, v in sens.items()}
    e4["none"] = J_none.tolist()
    return {"e2_median_rel_err": e2, "e2_reference_eigs": ref[:k].tolist(), "e3": e3, "e4": e4,
            "e2_eigs_A": eigs}


def e5_members(cfg: dict, iters: int) -> dict:
    L, ell, k = cfg["members"], cfg["ell"], cfg["k"]
    g = eda.Problem(cfg, W.problem_normals(cfg))
    members = np.arange(L + 1)
    J0 = cost_history(g, members, iters, False)
    res = {}
    for th in ("mid", "lamk"):
        for kk in (k, k - 5):
            g.sketch_evd("rhs_diff", ell=ell, k=kk, theta=th)
            J1 = cost_history(g, members, iters, True)
            ratio = J0[1:] / J1[1:]  # perturbed members only
            res[f"{th}_k{kk}"] = {"median": np.median(ratio, axis=0).tolist(), "min": ratio.min(axis=0).tolist(),
                                  "max": ratio.max(axis=0).tolist(),
                                  "control_ratio": (J0[0] / J1[0]).tolist()}
    g.close()
    return res


def run(inits: int = 20, iters: int = 50, spectrum: bool = True) -> dict:
    cfg = W.config("paper")
    t0 = time.time()
    out = {"config": {k: cfg[k] for k in ("n", "nsteps", "obs_dt", "obs_dx", "sigma_o", "sigma_b", "len_b",
                                          "diff_steps", "members", "ell", "k")},
           "inits": inits, "iters": iters}
    ref = reference_eigs(cfg, max(cfg["k"], 150))
    out["reference_eigs_IpA"] = ref.tolist()
    out.update(e2_to_e4(cfg, inits, iters, ref))
    out["e5"] = e5_members(cfg, iters)
    if spectrum:
        out["e1"] = e1_spectrum(cfg)
    out["seconds"] = time.time() - t0
    return out


def summary(res: dict) -> str:
    """Markdown tables of the results (eigenvalue errors at a few indices, J at
    a few iterations)."""
    k = res["config"]["k"]
    idx = [0, 4, 9, 14, k - 1]
    lines = ["E2 median relative error of lambda_i(I + A), i = " + ", ".join(str(i + 1) for i in idx), "",
             "| sketch | " + " | ".join(f"i={i + 1}" for i in idx) + " |", "|---|" + "---|" * len(idx)]
    for s in SKETCHES:
        e = res["e2_median_rel_err"][s]
        lines.append(f"| {s} | " + " | ".join(f"{e[i]:.1e}" for i in idx) + " |")
    its = [1, 2, 5, 10, 20, res["iters"]]
    lines += ["", "E3 median J at PCG iteration (A-products = iteration + sketch products)", "",
              "| sketch | " + " | ".join(f"it {i}" for i in its) + " |", "|---|" + "---|" * len(its)]
    for s in list(SKETCHES) + ["none"]:
        J = res["e3"][s]["median_J"]
        lines.append(f"| {s} | " + " | ".join(f"{J[i]:.4e}" for i in its) + " |")
    lines += ["", "E4 Gamma LMP: median J (min..max over initialisations)", "",
              "| theta, k | " + " | ".join(f"it {i}" for i in its) + " |", "|---|" + "---|" * len(its)]
    for key, v in res["e4"].items():
        if key == "none":
            lines.append("| no LMP | " + " | ".join(f"{v[i]:.4e}" for i in its) + " |")
        else:
            lines.append(f"| {key} | " + " | ".join(f"{v['median'][i]:.4e} ({v['min'][i]:.3e}..{v['max'][i]:.3e})"
                                                    for i in its) + " |")
    lines += ["", "E5 members: J(no LMP) / J(LMP), median (min..max) over the 20 perturbed members", "",
              "| theta, k | " + " | ".join(f"it {i}" for i in its) + " |", "|---|" + "---|" * len(its)]
    for key, v in res["e5"].items():
        lines.append(f"| {key} | " + " | ".join(f"{v['median'][i]:.3f} ({v['min'][i]:.3f}..{v['max'][i]:.3f})"
                                                for i in its) + " |")
    if "e1" in res:
        lines += ["", "E1 eigenvalues of I + A (1st, 20th, 50th, 60th, 150th)", "", "| B | l1 | l20 | l50 | l60 | l150 |",
                  "|---|---|---|---|---|---|"]
        for grp, lab in (("D_at_M10", "D={}, M=10"), ("M_at_D6", "D=6, M={}")):
            for key, ev in res["e1"][grp].items():
                lines.append(f"| {lab.format(key)} | " + " | ".join(f"{ev[i]:.4g}" for i in (0, 19, 49, 59, 149)) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--inits", type=int, default=20)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--no-spectrum", action="store_true")
    a = ap.parse_args()
    res = run(a.inits, a.iters, not a.no_spectrum)
    with open(a.out, "w") as f:
        json.dump(res, f)
    md = summary(res)
    with open(os.path.splitext(a.out)[0] + ".md", "w") as f:
        f.write(md + "\n")
    print(md, flush=True)
    print(f"[experiments] {res['seconds']:.1f} s", flush=True)


if __name__ == "__main__":
    main()
