"""The kernels' phase functions run on the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer (tests/host/cfv_host_harness.cpp), against the
oracle.

The harness emulates each workgroup (its lanes' states and its LDS, a barrier
being the end of a loop over the lanes, the lanes between two barriers run
first to last or last to first), so the residual of the fused march,
the JVP of the two-pass dual march and the VJP's four passes run exactly the
index arithmetic of the GPU kernels.  An access outside any array stops the
run with a sanitizer report; LDS is filled with NaN at the start of every
work item, so a read of an LDS value the item never wrote reaches the
outputs.  Shapes: partial tiles (N not a multiple of 14 or 16), N = 2, one
layer, chunk lengths from 1 to beyond Nr, odd N (polar-axis faces), both
inner laws and two Table 2 outer laws.  Bar: 1e-12 per variable as the GPU
parity tests."""
import ctypes
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import rel_err_per_var
from oracle import mhd, solve
from oracle.grid import Grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12

# (N, Nr, chunk layers, params)
CASES = [
    (5, 6, 4, {}),
    (16, 5, 2, {}),
    (17, 4, 3, {}),
    (2, 2, 1, {}),
    (3, 1, 16, {}),
    (7, 3, 16, {"inner_mode": 1}),
    (6, 4, 5, {"table2": 1}),
    (4, 5, 2, {"table2": 9, "limiter": 0}),
]


def _sanitizer_runtime():
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            return None
        libs.append(p)
    return ":".join(libs)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    pre = _sanitizer_runtime()
    if pre is None:
        pytest.skip("no sanitizer runtime")
    out = tmp_path_factory.mktemp("host") / "libcfv_host.so"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2209_04481_amd", "csrc"),
           os.path.join(HERE, "host", "cfv_host_harness.cpp"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return str(out), pre


RUNNER = r'''
import ctypes, json, sys
import numpy as np
sys.path.insert(0, {root!r})
from paper_2209_04481_amd.binding import CfvParams
L = ctypes.CDLL({lib!r})
P = ctypes.c_void_p
d = np.load({inp!r})
prm = json.loads(open({prm!r}).read())
cp = CfvParams(prm["gamma"], prm["c_h"], prm["G"], prm["vr_star"], prm["rho_b"], prm["T_b"], prm["limiter"],
               prm["inner_mode"], (ctypes.c_double * 8)(*prm["outer_exp"]), prm["outer_vr_mass"], prm["outer_psi_zero"])
N, Nr, kc = int(d["N"]), int(d["Nr"]), int(d["kc"])
ptr = lambda a: a.ctypes.data_as(P)
r, U, br, bth, v, dbr, w = (np.ascontiguousarray(d[k]) for k in ("r", "U", "br", "bth", "v", "dbr", "w"))
R = np.full_like(U, np.nan); Rj = np.full_like(U, np.nan); Jv = np.full_like(U, np.nan)
gU = np.full_like(U, np.nan); gbr = np.full_like(br, np.nan)
flag = ctypes.c_uint(0)
bt = ptr(bth) if prm["inner_mode"] == 1 else None
L.host_set_lane_order(int(d["order"]) if "order" in d.files else 0)
assert L.host_residual(N, Nr, ptr(r), ctypes.byref(cp), ptr(U), ptr(br), bt, kc, ptr(R), ctypes.byref(flag)) == 0
assert L.host_jvp(N, Nr, ptr(r), ctypes.byref(cp), ptr(U), ptr(br), bt, kc, ptr(v), ptr(dbr), ptr(Jv), ptr(Rj)) == 0
assert L.host_vjp(N, Nr, ptr(r), ctypes.byref(cp), ptr(U), ptr(br), bt, kc, ptr(w), ptr(gU), ptr(gbr)) == 0
np.savez({out!r}, R=R, Rj=Rj, Jv=Jv, gU=gU, gbr=gbr, flag=flag.value)
'''


@pytest.mark.parametrize("N,Nr,kc,kw", CASES)
def test_host_emulation_matches_the_oracle(harness, tmp_path, N, Nr, kc, kw):
    lib, pre = harness
    inst = ci.make_instance(N, Nr, "log", lmax=3, seed=300 + 10 * N + Nr)
    inst.U[8] = 1e-3 * np.random.default_rng(N + Nr).standard_normal(inst.ncells)   # psi != 0
    kw = dict(kw)
    case = kw.pop("table2", None)
    if kw.get("inner_mode") == 1:
        kw["inner_btheta"] = torch.tensor(ci.btheta_map(N))
    op = mhd.Params.table2(case, **kw) if case else mhd.Params(**kw)
    bth = ci.btheta_map(N) if op.inner_mode == 1 else np.zeros(6 * N * N)
    v = ci.scaled_direction(inst.U, N)
    dbr = ci.br_direction(6 * N * N, N)
    w = np.random.default_rng(7 + N).standard_normal(inst.U.shape)
    inp = tmp_path / "in.npz"
    np.savez(inp, N=N, Nr=Nr, kc=kc, r=inst.r_nodes, U=inst.U, br=inst.br, bth=bth, v=v, dbr=dbr, w=w)
    prm = tmp_path / "prm.json"
    import json
    prm.write_text(json.dumps({"gamma": op.gamma, "c_h": op.c_h, "G": op.G, "vr_star": op.vr_star, "rho_b": op.rho_b,
                               "T_b": op.T_b, "limiter": int(op.limiter), "inner_mode": int(op.inner_mode),
                               "outer_exp": [float(x) for x in op.outer_exp], "outer_vr_mass": int(op.outer_vr_mass),
                               "outer_psi_zero": int(op.outer_psi_zero)}))
    out = tmp_path / "out.npz"
    script = tmp_path / "run.py"
    script.write_text(RUNNER.format(root=ROOT, lib=lib, inp=str(inp), prm=str(prm), out=str(out)))
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    res = np.load(out)
    g = Grid(N, Nr, inst.r_nodes)
    U, br = torch.tensor(inst.U), torch.tensor(inst.br)
    Ro = mhd.residual(g, U, br, op)
    Jo, _ = solve.jvp(g, U, br, op, torch.tensor(v), torch.tensor(dbr))
    gUo, gbro = solve.vjp(g, U, br, op, torch.tensor(w))
    for name, a, b in (("R (fused march)", res["R"], Ro), ("R (dual march)", res["Rj"], Ro), ("Jv", res["Jv"], Jo),
                       ("gU", res["gU"], gUo), ("gbr", res["gbr"][None], gbro[None])):
        err = float(rel_err_per_var(torch.tensor(a), b).max())
        assert err <= TOL, f"{name}: {err:.2e}"
    # the non-physical flag: set exactly when some face state of the oracle's
    # reconstruction (either side, ghosts included) has rho <= 0 or p <= 0
    st = mhd._Stencil(g, torch.arange(g.ncells))
    fs = mhd.face_states(g, U, br, op, torch.arange(g.ncells), st)
    sides = torch.cat([fs["PL"], fs["PR"]], 1)
    expect = bool(((sides[..., 0] <= 0) | (sides[..., 7] <= 0)).any())
    assert bool(int(res["flag"]) & 1) == expect


def test_host_emulation_outputs_do_not_depend_on_the_chunk_length(harness, tmp_path):
    """Residual, JVP and VJP of one shell for chunks of 1, 2, 5, 16 and 40
    layers (Nr = 11): bitwise equal, since every face flux is evaluated once
    from the same states and every cell sums its faces in a fixed order."""
    lib, pre = harness
    N, Nr = 7, 11
    inst = ci.make_instance(N, Nr, "log", lmax=3, seed=77)
    op = mhd.Params()
    v = ci.scaled_direction(inst.U, 3)
    dbr = ci.br_direction(6 * N * N, 3)
    w = np.random.default_rng(8).standard_normal(inst.U.shape)
    prm = tmp_path / "prm.json"
    import json
    prm.write_text(json.dumps({"gamma": op.gamma, "c_h": op.c_h, "G": op.G, "vr_star": op.vr_star, "rho_b": op.rho_b,
                               "T_b": op.T_b, "limiter": int(op.limiter), "inner_mode": 0,
                               "outer_exp": [float(x) for x in op.outer_exp], "outer_vr_mass": int(op.outer_vr_mass),
                               "outer_psi_zero": int(op.outer_psi_zero)}))
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = {}
    for kc in (16, 1, 2, 5, 40):
        inp, out, script = tmp_path / f"in{kc}.npz", tmp_path / f"out{kc}.npz", tmp_path / f"run{kc}.py"
        np.savez(inp, N=N, Nr=Nr, kc=kc, r=inst.r_nodes, U=inst.U, br=inst.br, bth=np.zeros(6 * N * N), v=v,
                 dbr=dbr, w=w)
        script.write_text(RUNNER.format(root=ROOT, lib=lib, inp=str(inp), prm=str(prm), out=str(out)))
        r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
        res[kc] = np.load(out)
    for kc in (1, 2, 5, 40):
        for name in ("R", "Rj", "Jv", "gU", "gbr"):
            assert np.array_equal(res[kc][name], res[16][name]), f"{name} with chunk {kc}"


def test_host_emulation_outputs_do_not_depend_on_the_lane_order(harness, tmp_path):
    """Between two barriers the GPU runs a workgroup's lanes in any
    interleaving.  The emulation runs the code between two of the kernels'
    barriers lane after lane, first to last and then last to first: a phase
    reading an LDS value another lane writes before the next barrier (a
    missing barrier) would give different results in the two orders.  Partial
    tiles, ring lanes across panel edges, several chunks and both boundary
    layers; residual, JVP and VJP bitwise equal."""
    lib, pre = harness
    N, Nr, kc = 17, 5, 2
    inst = ci.make_instance(N, Nr, "log", lmax=3, seed=91)
    op = mhd.Params()
    v = ci.scaled_direction(inst.U, 5)
    dbr = ci.br_direction(6 * N * N, 5)
    w = np.random.default_rng(9).standard_normal(inst.U.shape)
    prm = tmp_path / "prm.json"
    import json
    prm.write_text(json.dumps({"gamma": op.gamma, "c_h": op.c_h, "G": op.G, "vr_star": op.vr_star, "rho_b": op.rho_b,
                               "T_b": op.T_b, "limiter": int(op.limiter), "inner_mode": 0,
                               "outer_exp": [float(x) for x in op.outer_exp], "outer_vr_mass": int(op.outer_vr_mass),
                               "outer_psi_zero": int(op.outer_psi_zero)}))
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = {}
    for order in (0, 1):
        inp, out, script = tmp_path / f"in{order}.npz", tmp_path / f"out{order}.npz", tmp_path / f"run{order}.py"
        np.savez(inp, N=N, Nr=Nr, kc=kc, order=order, r=inst.r_nodes, U=inst.U, br=inst.br,
                 bth=np.zeros(6 * N * N), v=v, dbr=dbr, w=w)
        script.write_text(RUNNER.format(root=ROOT, lib=lib, inp=str(inp), prm=str(prm), out=str(out)))
        r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
        res[order] = np.load(out)
    for name in ("R", "Rj", "Jv", "gU", "gbr"):
        assert np.all(np.isfinite(res[0][name])), name
        assert np.array_equal(res[0][name], res[1][name]), f"{name} depends on the lane order"


LIMITER_RUNNER = r'''
import ctypes, sys
import numpy as np
L = ctypes.CDLL({lib!r})
d = np.load({inp!r})
P = ctypes.c_void_p
ptr = lambda a: np.ascontiguousarray(a).ctypes.data_as(P)
out = np.zeros((len(d["qc"]), 6))
for c in range(len(d["qc"])):
    o = np.zeros(6)
    L.host_limited_grad_dual(ptr(d["W"][c]), ptr(d["dxf"][c]), ctypes.c_double(d["qc"][c]), ctypes.c_double(d["qcd"][c]),
                             ptr(d["qn"][c]), ptr(d["qnd"][c]), 1, ptr(o))
    out[c] = o
np.save({out!r}, out)
'''


def _limiter_cases():
    """Stencils for the dual limiter: given weights W (so g = sum W_n (q_n -
    q_c) exactly), face offsets and values; exact ties built with powers of
    two, then random ones."""
    cases = []
    e = np.zeros((6, 3))
    W = e.copy(); W[0] = (1.0, 0.0, 0.0)          # g = (q_0 - q_c, 0, 0)
    qn = np.array([1.0, 0.0, 0.0, 0.0, -1.0, 0.0])  # up = down = 1
    for plus, minus in ((2, 3), (3, 2), (5, 1), (1, 5)):
        # projections +4 on face `plus`, -4 on face `minus`: ratios 1/4 and
        # 1/4, an exact tie across signs (the earlier face wins)
        dxf = e.copy(); dxf[plus] = (4.0, 0.0, 0.0); dxf[minus] = (-4.0, 0.0, 0.0)
        cases.append((W, dxf, 0.0, qn))
    # two equal positive projections (same-sign tie), and a ratio of exactly 1
    dxf = e.copy(); dxf[3] = (4.0, 0.0, 0.0); dxf[1] = (4.0, 0.0, 0.0); dxf[2] = (-2.0, 0.0, 0.0)
    cases.append((W, dxf, 0.0, qn))
    dxf = e.copy(); dxf[4] = (1.0, 0.0, 0.0); dxf[0] = (-0.5, 0.0, 0.0)
    cases.append((W, dxf, 0.0, qn))
    rng = np.random.default_rng(11)
    for _ in range(200):
        cases.append((rng.standard_normal((6, 3)) * 0.3, rng.standard_normal((6, 3)), rng.standard_normal(),
                      rng.standard_normal(6)))
    return cases


def test_dual_limiter_choice_matches_the_oracle_scan(harness, tmp_path):
    """The kernels' dual Barth-Jespersen choice (two candidate faces, an
    exact tie between them to the earlier face) against the oracle's scan
    over faces in local order (R7: 1 wins ties, then the first face), value
    and tangent (torch.func.jvp of the oracle), on exact same-sign and
    cross-sign ties in both face orders and on random stencils."""
    lib, pre = harness
    from torch.func import jvp
    cases = _limiter_cases()
    rng = np.random.default_rng(12)
    W = np.stack([c[0] for c in cases]); dxf = np.stack([c[1] for c in cases])
    qc = np.array([c[2] for c in cases]); qn = np.stack([c[3] for c in cases])
    qcd = rng.standard_normal(len(cases)); qnd = rng.standard_normal((len(cases), 6))
    inp, out, script = tmp_path / "lim.npz", tmp_path / "lim.npy", tmp_path / "lim.py"
    np.savez(inp, W=W.reshape(len(cases), 18), dxf=dxf.reshape(len(cases), 18), qc=qc, qcd=qcd, qn=qn, qnd=qnd)
    script.write_text(LIMITER_RUNNER.format(lib=lib, inp=str(inp), out=str(out)))
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    got = np.load(out)
    Wt, dxt = torch.tensor(W), torch.tensor(dxf)

    def glim(qc_, qn_):
        g = torch.einsum("nfa,nf->na", Wt, qn_ - qc_[:, None])
        # one variable: the oracle's shapes carry a variable axis of length 1
        phi = mhd.barth_jespersen(qc_[:, None], qn_[:, :, None], g[:, None, :], dxt)[:, 0]
        return g * phi[:, None]

    val, tan = jvp(glim, (torch.tensor(qc), torch.tensor(qn)), (torch.tensor(qcd), torch.tensor(qnd)))
    assert np.abs(got[:, :3] - val.numpy()).max() <= 1e-14 * max(1.0, float(np.abs(val.numpy()).max()))
    err_t = np.abs(got[:, 3:] - tan.numpy()) / np.maximum(np.abs(tan.numpy()).max(1, keepdims=True), 1e-300)
    assert err_t.max() <= 1e-13, f"tangent differs: {err_t.max():.2e} in case {int(err_t.max(1).argmax())}"


JOIN_RUNNER = r'''
import ctypes
L = ctypes.CDLL({lib!r})
L.host_join_address.restype = ctypes.c_uint64
L.host_join_address.argtypes = [ctypes.c_int, ctypes.c_int]
for hi, lo in {pairs!r}:
    print(L.host_join_address(hi, lo))
'''


def test_uniform_address_halves_join_as_unsigned(harness, tmp_path):
    """The kernels read a launch descriptor and the layer radii with scalar
    loads at an address rebuilt from two readfirstlane halves, which are
    signed 32-bit ints.  Joined as signed, a low half with bit 31 set turned
    the high half into 0xffffffff, an address outside every allocation (a
    GPU memory fault that came and went with the allocation's address)."""
    lib, pre = harness
    pairs = [(0x7F, -0x7FFFE000), (0x7FFF, -1), (0x1234, 0x7FFFFFFF), (0, -0x80000000), (0x7F, 0x1000)]
    script = tmp_path / "join.py"
    script.write_text(JOIN_RUNNER.format(lib=lib, pairs=pairs))
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    got = [int(x) for x in r.stdout.split()]
    want = [((hi & 0xFFFFFFFF) << 32) | (lo & 0xFFFFFFFF) for hi, lo in pairs]
    assert got == want
    assert all(g >> 32 == hi & 0xFFFFFFFF for g, (hi, _) in zip(got, pairs))
