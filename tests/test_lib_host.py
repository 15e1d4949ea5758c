"""Host-side checks of the C ABI library (no GPU compute calls)."""
import os
import re
import subprocess

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from oracle.grid import Grid as OracleGrid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfv.h")
LIB = os.path.join(ROOT, "paper_2209_04481_amd", "libcfv.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfv_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        pytest.skip("libcfv.so not built (run __graft_entry__.build())")
    return LIB


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (cfv_[a-z0-9_]+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    from paper_2209_04481_amd import binding
    L = binding.lib()
    for s in declared_symbols():
        assert hasattr(L, s)


@pytest.mark.parametrize("N,Nr,radial", [(8, 16, "geometric"), (5, 7, "log"), (12, 3, "log"),
                                         (3, 1, "log"), (3, 2, "log"), (4, 1, "log"), (2, 2, "log"),
                                         (6, 12, "bcind"), (5, 3, "bcind")])
def test_face_list_bit_exact_vs_geometric_matching(built, N, Nr, radial):
    """Library adjacency (closed-form panel-edge table) vs the oracle's
    point-location derivation: identical canonical face lists."""
    from paper_2209_04481_amd import Grid
    r = ci.radial_nodes(Nr, radial)
    L, R, K = Grid(N, Nr, r).faces()
    oL, oR, oK = OracleGrid(N, Nr, r).face_list()
    assert np.array_equal(L, oL.numpy()) and np.array_equal(R, oR.numpy())
    assert np.array_equal(K.astype(np.int64), oK.numpy())


@pytest.mark.parametrize("N,Nr,radial", [(8, 16, "geometric"), (5, 3, "log"), (3, 1, "log"), (6, 12, "bcind")])
def test_geometry_to_host_matches_the_oracle_vertex_geometry(built, N, Nr, radial):
    """cfv_grid_geometry_to_host (the kernels' separable geometry, rebuilt
    from the per-column tables) against the oracle's cell geometry from the
    vertices: per face of the canonical list the owner's vector area and
    centroid, per cell its volume and centroid."""
    from paper_2209_04481_amd import Grid
    r = ci.radial_nodes(Nr, radial)
    g = Grid(N, Nr, r)
    S, xf, V, xc = g.geometry()
    og = OracleGrid(N, Nr, r)
    cells = torch.arange(og.ncells)
    oxc, oV, oxf, oS = og.cell_geometry(cells)
    nb = og.neighbours(cells)
    emit = (nb >= og.ncells) | (nb > cells[:, None])       # the canonical list's rule
    fS, fx = oS[emit].numpy(), oxf[emit].numpy()
    assert S.shape == fS.shape
    sc = np.abs(fS).max()
    assert np.abs(S - fS).max() <= 1e-13 * sc
    assert np.abs(xf - fx).max() <= 1e-13 * np.abs(fx).max()
    assert np.abs(V - oV.numpy()).max() <= 1e-13 * oV.abs().max().item()
    assert np.abs(xc - oxc.numpy()).max() <= 1e-13 * np.abs(oxc.numpy()).max()


def test_grid_sizes_and_argument_errors(built):
    from paper_2209_04481_amd import CfvError, Grid
    g = Grid(6, 4, ci.radial_nodes(4, "log"))
    assert g.ncells == 6 * 36 * 4 and g.nb == 216
    assert g.nfaces == 6 * 36 * 5 + 12 * 36 * 4
    with pytest.raises(CfvError):
        Grid(6, 4, np.array([1.0, 2.0, 2.0, 3.0, 4.0]))   # not strictly increasing
    with pytest.raises(CfvError):
        Grid(1, 4, ci.radial_nodes(4, "log"))
    with pytest.raises(CfvError, match="16384"):
        Grid(16385, 1, ci.radial_nodes(1, "log"))
    with pytest.raises(CfvError, match="2\\^31"):
        Grid(16384, 8, ci.radial_nodes(8, "log"))   # 1.3e10 cells


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(here, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_cpu_baseline_record_on_a_small_shell():
    """The bench's CPU-baseline leg (the oracle timed on a block of cells)
    clamps its sample to the shell and reports the fields of its record."""
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, here)
    import bench
    inst = ci.make_instance(4, 3, "log", lmax=2, seed=5)
    rec = bench.cpu_baseline({"small": inst}, 10 ** 6, reps=1)
    assert rec["kind"] == "oracle" and rec["value"] > 0 and rec["cores"] >= 1 and rec["nproc"] >= 1
    small = rec["per_workload"]["small"]
    assert small["sample_cells"] == inst.ncells
    for op in ("residual", "jvp"):
        assert small[op]["1_thread_mcells_per_s"] > 0 and small[op]["all_threads_mcells_per_s"] > 0
    assert rec["value"] == small["step_all_threads_mcells_per_s"]
