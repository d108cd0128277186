"""GPU: what the trained learned-sketch network gains over the method without
it.  Test problems (ids from the test range, n = 1024 preset, 64 members): for
each, the right-hand-side-difference sketch (ell = k = 32) and the learned
sketch (k = 32, BF16 inference) build the LMP, PCG solves every member to rtol
1e-6, and the iteration counts are compared; the control member is also solved
to rtol 1e-10 with the learned LMP and compared with the oracle's exact
solution.  The network is the committed one
(paper_2605_23571_amd/weights/); without it the test is skipped."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_23571_amd import eda  # noqa: E402
from paper_2605_23571_amd import train_sketch as T  # noqa: E402

N_TEST = 4


def test_learned_sketch_gain_on_test_problems():
    net = T.load_bf16()
    if net is None:
        pytest.skip("no trained network committed")
    dims, p16 = net
    t0, _ = W.LEARNED_SPLITS["test"]
    rows = []
    for pid in range(t0, t0 + N_TEST):
        cfg = W.learned_problem(pid)
        z = W.problem_normals(cfg)
        g = eda.Problem(cfg, z)
        members = np.arange(cfg["members"] + 1)
        g.sketch_evd("rhs_diff", ell=32, k=32)
        it_g = g.pcg(members, rtol=1e-6, maxit=5000)["iters"]
        _, _, used = eda.sketch_learned(g, dims, p16, 32)
        out = g.pcg(members, rtol=1e-6, maxit=5000)
        assert (out["status"] == eda.EDA_MEMBER_CONVERGED).all()
        it_l = out["iters"]
        rows.append((pid, used, float(np.median(it_g)), float(np.median(it_l))))
        print(f"[gain] problem {pid}: learned used {used}; median PCG iterations Gamma {np.median(it_g):.0f}, "
              f"learned {np.median(it_l):.0f}", flush=True)
        if pid == t0:
            # solution error against the oracle with the learned LMP
            sol = g.pcg([0], rtol=1e-10, maxit=5000)
            ex = O.exact_solution(O.Problem(cfg, z), 0)
            dz = sol["dz"].cpu().numpy()[0]
            assert np.linalg.norm(dz - ex) / np.linalg.norm(ex) < 1e-6
        g.close()
    ratios = np.array([r[2] / r[3] for r in rows])
    gain = float(np.median(ratios))
    print(f"[gain] iteration ratio Gamma / learned: median {gain:.3f}, min {ratios.min():.3f}, "
          f"max {ratios.max():.3f}", flush=True)
    assert all(r[1] for r in rows)  # the network produced usable sketches
    # the stated outcome: parity with the method's own Gamma sketch at equal
    # sketch cost (32 Hessian products), within 3% in median; no gain is
    # claimed (64 test problems measured 0.999, spread 0.985 to 1.014)
    assert 0.97 <= gain
