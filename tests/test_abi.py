"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-only calls behave (no GPU needed)."""
import ctypes

import pytest

import workloads as W
from paper_2605_23571_amd import eda


def test_header_symbols_exported():
    syms = eda.header_symbols()
    assert len(syms) >= 12
    L = eda.lib()
    for s in syms:
        assert hasattr(L, s), s


def test_exports_only_abi_symbols():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", eda.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line and line.split()[-1].startswith("eda_")}
    assert exported == set(eda.header_symbols())


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "paper"])
def test_workspace_and_normals(name):
    cfg = W.config(name)
    c = eda.make_config(cfg)
    assert eda.eda_normals_count(c) == W.n_normals(cfg)
    b_band = eda.eda_workspace_bytes(c)
    b_dense = eda.eda_workspace_bytes(eda.make_config(cfg, ub_mode="dense"))
    n = cfg["n"]
    traj = (cfg["members"] + 1) * (cfg["nsteps"] + 1) * n * 8
    assert b_dense >= 14 * n * n + traj  # U_B stored dense in FP64, FP32 and BF16
    # the banded form holds a block of observed increments per piece of a split column
    nt, nv = W.obs_counts(cfg)
    assert b_band > traj + 8 * nt * nv * (cfg["members"] + 1) * 8


@pytest.mark.parametrize("bad", [dict(n=3), dict(n=4097), dict(n=5000), dict(len_b=1.0), dict(obs_x0=40), dict(sigma_o=0.0),
                                 dict(members=0), dict(nsteps=2, obs_dt=5),
                                 dict(b_kind="diffusion", diff_steps=9), dict(b_kind="diffusion", diff_steps=0),
                                 dict(b_kind="diffusion", diff_steps=66), dict(b_kind="diffusion", len_b=0.0)])
def test_invalid_config_rejected(bad):
    cfg = W.config("C1", **bad)
    c = eda.make_config(cfg)
    out = ctypes.c_size_t()
    assert eda.lib().eda_workspace_bytes(ctypes.byref(c), ctypes.byref(out)) == eda.EDA_ERR_INVALID_ARG


def test_invalid_b_kind_rejected():
    c = eda.make_config(W.config("C1"))
    c.b_kind = 2
    out = ctypes.c_size_t()
    assert eda.lib().eda_workspace_bytes(ctypes.byref(c), ctypes.byref(out)) == eda.EDA_ERR_INVALID_ARG


def test_diffusion_band_is_wider_than_a_short_gaussian():
    # the banded U_B's halo enters the split rings' padding: the diffusion
    # kernel (exponential tails) needs more taps than a Gaussian of the same
    # Daley length, so its workspace is at least as large
    g = eda.eda_workspace_bytes(eda.make_config(W.config("paper", b_kind="gauss")))
    d = eda.eda_workspace_bytes(eda.make_config(W.config("paper")))
    assert d > g


def test_strerror_static():
    for code in (0, -1, -2, -3, -4, -5, -6, 1, 12345):
        assert isinstance(eda.strerror(code), str) and eda.strerror(code)
    assert eda.strerror(-5) != eda.strerror(-4)


def test_null_handles_rejected():
    L = eda.lib()
    assert L.eda_hessvec(None, None, 1, None, 40, None, 40, 0) == eda.EDA_ERR_INVALID_ARG
    assert L.eda_destroy(None) == eda.EDA_ERR_INVALID_ARG
    assert L.eda_profile(None, 1) == eda.EDA_ERR_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    # one GPU per run: the bench exits with a message before it touches a device
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_python_constants_match_header():
    # every integer #define of the header that the binding also names has the
    # same value there (modes, flags, fields, error and status codes)
    import os
    import re
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "eda.h")
    defs = dict(re.findall(r"^#define\s+(EDA_\w+)\s+\(?(-?\d+)\)?", open(hdr).read(), re.M))
    shared = [k for k in defs if hasattr(eda, k)]
    assert len(shared) >= 20
    for k in shared:
        assert getattr(eda, k) == int(defs[k]), k
    assert {"EDA_XCH_OFF", "EDA_XCH_ON", "EDA_XCH_OBS"} <= set(shared)
