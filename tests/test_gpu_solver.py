"""GPU checks of the implicit step (GMRES on the matrix-free JVP/VJP) and of
the B_r sensitivity, against the oracle and against finite differences."""
import time

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import rel_err_per_var
from oracle import mhd, solve
from oracle.grid import Grid as OGrid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def context(inst, **kw):
    from paper_2209_04481_amd import Context, Grid, Params
    grid = Grid(inst.N, inst.Nr, inst.r_nodes)
    ctx = Context(grid, Params(**kw))
    ctx.set_inner_br(torch.from_numpy(inst.br).cuda())
    return ctx


def test_be_step_gmres30_matches_oracle_tiny():
    """One backward-Euler step, CFL 1e3, GMRES(30) from x0 = 0, no restart:
    the relative-residual history and the new state agree with the oracle."""
    print("case: BE step tiny", flush=True)
    inst = ci.workload("tiny")
    ctx = context(inst)
    U = torch.from_numpy(inst.U).cuda()
    Un, hist = ctx.be_step(U, cfl=1e3, m=30)
    og = OGrid(inst.N, inst.Nr, inst.r_nodes)
    Uo, hist_o, _ = solve.be_step(og, torch.from_numpy(inst.U), torch.from_numpy(inst.br), mhd.Params(), 1e3, 30)
    assert len(hist) == 30
    h, ho = np.asarray(hist), np.asarray(hist_o)
    print("history", h[[0, 9, 19, 29]], "max diff", np.abs(h - ho).max())
    assert np.all(np.abs(h - ho) <= 1e-9 * ho)
    assert float(rel_err_per_var((Un - U).cpu(), Uo - torch.from_numpy(inst.U)).max()) <= 1e-8


@pytest.mark.parametrize("cfl", [1e3, 10.0])
def test_be_step_jacobi_preconditioned_matches_oracle_tiny(cfl):
    """GMRES(30) right-preconditioned by the step's diagonal V/dt: history and
    new state agree with the oracle's preconditioned step."""
    print(f"case: BE step tiny, Jacobi, CFL {cfl}", flush=True)
    inst = ci.workload("tiny")
    ctx = context(inst)
    ctx.set_preconditioner(1)
    U = torch.from_numpy(inst.U).cuda()
    Un, hist = ctx.be_step(U, cfl=cfl, m=30)
    og = OGrid(inst.N, inst.Nr, inst.r_nodes)
    Uo, hist_o, _ = solve.be_step(og, torch.from_numpy(inst.U), torch.from_numpy(inst.br), mhd.Params(), cfl, 30,
                                  jacobi=True)
    h, ho = np.asarray(hist), np.asarray(hist_o)
    print("history", h[[0, 9, len(h) - 1]], "oracle", ho[[0, 9, len(ho) - 1]])
    assert len(h) == len(ho)
    assert np.all(np.abs(h - ho) <= 1e-9 * ho + 1e-13)
    assert float(rel_err_per_var((Un - U).cpu(), Uo - torch.from_numpy(inst.U)).max()) <= 1e-8
    with pytest.raises(Exception):
        ctx.set_preconditioner(2)


def test_be_step_medium_jacobi_converges_further_and_reports_the_true_residual():
    """Medium grid, CFL 1e3, GMRES(30): the Jacobi-preconditioned step ends
    below the unpreconditioned one, and its last history entry is the true
    relative residual |(D + J) x + R| / |R|."""
    print("case: BE step medium, Jacobi", flush=True)
    inst = ci.workload("medium")
    ctx = context(inst)
    U = torch.from_numpy(inst.U).cuda()
    _, hist0 = ctx.be_step(U, cfl=1e3, m=30)
    ctx.set_preconditioner(1)
    Un, hist = ctx.be_step(U, cfl=1e3, m=30)
    torch.cuda.synchronize()
    print("plain", hist0[[9, 29]], "jacobi", hist[[9, 29]])
    assert hist[-1] < hist0[-1]
    x = Un - U
    R = ctx.residual(U)
    D = ctx.local_dt(U, 1e3)
    Ax = ctx.jvp(U, x.contiguous()) + D[None, :] * x
    true_rel = float((Ax + R).norm() / R.norm())
    assert abs(true_rel - hist[-1]) <= 1e-6 * hist[-1]


def test_transpose_solve_is_tight_and_consistent():
    print("case: transpose solve", flush=True)
    inst = ci.make_instance(6, 10, "log", lmax=4, seed=8)
    ctx = context(inst)
    U = torch.from_numpy(inst.U).cuda()
    D = ctx.local_dt(U, 2.0)
    b = torch.randn(9, inst.ncells, dtype=torch.float64, device="cuda")
    x, hist = ctx.solve(U, D, b, transpose=True, m=40, max_restarts=20, rtol=1e-12)
    assert hist[-1] <= 1e-12
    gU, _ = ctx.vjp(U, x, want_br=False)
    Ax = gU + D[None, :] * x
    assert float((Ax - b).norm() / b.norm()) < 1e-10
    # forward and transposed solves are adjoint: <y, A^-1 b> = <A^-T y, b>
    y = torch.randn_like(b)
    xf, _ = ctx.solve(U, D, b, transpose=False, m=40, max_restarts=20, rtol=1e-13)
    xt, _ = ctx.solve(U, D, y, transpose=True, m=40, max_restarts=20, rtol=1e-13)
    lhs, rhs = float((y * xf).sum()), float((xt * b).sum())
    assert abs(lhs - rhs) <= 1e-9 * (abs(lhs) + float((y * xf).abs().sum()) * 1e-3)


def test_be_step_medium_history_is_the_true_residual():
    """Medium grid (1.66M cells): GMRES(30) at CFL 1e3; the reported history
    is monotone and its last entry is the true |(D + J) x + R| / |R|."""
    print("case: BE step medium", flush=True)
    inst = ci.workload("medium")
    ctx = context(inst)
    U = torch.from_numpy(inst.U).cuda()
    t0 = time.time()
    Un, hist = ctx.be_step(U, cfl=1e3, m=30)
    torch.cuda.synchronize()
    print(f"BE step medium: {time.time() - t0:.3f} s, history", hist[[0, 9, 19, 29]])
    assert len(hist) == 30 and np.all(np.diff(hist) <= 1e-15)
    x = Un - U
    R = ctx.residual(U)
    D = ctx.local_dt(U, 1e3)
    Ax = ctx.jvp(U, x.contiguous()) + D[None, :] * x
    true_rel = float((Ax + R).norm() / R.norm())
    assert abs(true_rel - hist[-1]) <= 1e-6 * hist[-1]


@pytest.mark.parametrize("psi_noise", [False, True])
def test_br_sensitivity_matches_the_oracle_exact_gradient(psi_noise):
    """Two implicit steps on a 48-cell grid: the objective equals the
    oracle's (dense solves), the tangent sweep equals the oracle's exact
    gradient (reverse mode through dense Jacobians and solves), and so does
    the adjoint, tightly once psi is not identically zero: with psi = 0 every
    cell sits on the psi limiter's kink at step 0, where the adjoint's
    central difference along the step is direction-dependent."""
    from paper_2209_04481_amd.sensitivity import Sensitivity
    print(f"case: sensitivity vs oracle, psi noise {psi_noise}", flush=True)
    inst = ci.make_instance(2, 2, "log", lmax=2, seed=5)
    U0n = inst.U.copy()
    if psi_noise:
        U0n[8] = np.random.default_rng(6).standard_normal(inst.ncells) * 1e-3 * np.abs(inst.U[4:7]).max()
    ctx = context(inst)
    U0 = torch.from_numpy(U0n).cuda()
    br = torch.from_numpy(inst.br).cuda()
    sens = Sensitivity(ctx, U0, cfl=1.0, nsteps=2, every=1, max_restarts=40, rtol=1e-14, layer=0)
    L, gb = sens.gradient(br)
    assert sens.max_rel <= 1e-13
    og = OGrid(2, 2, inst.r_nodes)
    prm = mhd.Params()
    U0o, bro = torch.from_numpy(U0n), torch.from_numpy(inst.br)
    D0 = solve.local_dt_diag(og, U0o, bro, prm, 1.0)
    Lo, gbo = solve.step_map_sensitivity(og, U0o, bro, prm, D0, 2, solve.layer_objective(og, 0))
    print(f"  L {L:.15e} oracle {Lo:.15e}")
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    rel_adj = float((gb.cpu() - gbo).norm() / gbo.norm())
    print(f"  adjoint vs oracle gradient: {rel_adj:.2e}")
    # the central differences of the step's second-order terms carry about
    # 1e-6 (rounding at a 1e-6 relative step); the psi kink adds about 2e-5
    assert rel_adj <= (5e-6 if psi_noise else 1e-4)
    for q, d in enumerate(_map_dirs(ctx, br, 3)):
        _, tg = sens.tangent(br, d)
        ex = float((gbo * d.cpu()).sum())
        scale = float(gbo.norm() * d.cpu().norm())
        print(f"  dir {q}: tangent {tg:.12e} oracle {ex:.12e} error / (|g| |d|) {abs(tg - ex) / scale:.1e}")
        assert abs(tg - ex) <= 1e-5 * scale


def _map_dirs(ctx, br, k, seed=99):
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.standard_normal(ctx.grid.nb)).cuda() * float(br.abs().max()) * 1e-2
            for _ in range(k)]


# One step, 4-layer grid, CFL 1, objective on layer 0 (where one step moves
# it well above rounding).  Without the limiter the residual is smooth and
# the adjoint matches to FD accuracy.  With Barth-Jespersen limiting, cells at
# a local extremum (and every cell for psi, which starts at zero) sit on a
# kink of the limiter, where the mixed second derivative depends on the
# direction; the one approximate piece of the adjoint (the central difference
# of two VJPs along the step) then differs from the objective's FD at 1e-6.
@pytest.mark.parametrize("limiter,tol", [(0, 1e-7), (1, 1e-5)])
def test_br_sensitivity_one_step_matches_central_differences(limiter, tol):
    """One implicit step: the adjoint and tangent derivatives of L along three
    seeded B_r directions against central differences of L at two step
    sizes (which agree, so the map is smooth there)."""
    from paper_2209_04481_amd.sensitivity import Sensitivity
    print(f"case: one-step sensitivity limiter {limiter}", flush=True)
    inst = ci.make_instance(8, 4, "log", lmax=4, seed=12)
    ctx = context(inst, limiter=limiter)
    U0 = torch.from_numpy(inst.U).cuda()
    br = torch.from_numpy(inst.br).cuda()
    sens = Sensitivity(ctx, U0, cfl=1.0, nsteps=1, max_restarts=16, rtol=1e-13, layer=0)
    L, gb = sens.gradient(br)
    assert sens.max_rel <= 1e-13
    for q, d in enumerate(_map_dirs(ctx, br, 3)):
        fds = [(sens.objective(br + h * d) - sens.objective(br - h * d)) / (2 * h) for h in (1e-3, 1e-4)]
        ad = float((gb * d).sum())
        _, tg = sens.tangent(br, d)
        print(f"  dir {q}: adjoint {ad:.10e} tangent {tg:.10e} fd", " ".join(f"{f:.10e}" for f in fds))
        assert abs(fds[0] - fds[1]) <= 1e-7 * abs(fds[0])
        assert abs(tg - fds[0]) <= 1e-6 * abs(fds[0])
        assert abs(ad - fds[0]) <= tol * abs(fds[0])


# (name, limiter, CFL, objective layer, directions, tolerance): the 4-layer
# grid reaches the outer boundary in 20 steps at CFL 1; on the 120-layer
# medium grid a B_r change travels a few cells, so the objective is taken on
# layer 2.  Over 20 limited steps central differences of L cross limiter
# switches, so the reference is the forward tangent sweep (JVP kernels).
# Adjoint and tangent linearise on the same limiter branches; they differ
# only through the second-order central differences, exactly symmetric
# without the limiter and direction-dependent at limiter kinks (above).
# (Without the limiter the second-order scheme does not stay stable over 20
# steps of this state, and the solves stall: no unlimited multi-step case.)
SENS_CASES = [("outer4", 1, 1.0, None, 3, 1e-4), ("medium", 1, 0.05, 2, 8, 1e-3)]


@pytest.mark.parametrize("name,limiter,cfl,layer,ndir,tol", SENS_CASES)
def test_br_sensitivity_adjoint_matches_tangent(name, limiter, cfl, layer, ndir, tol):
    """dL/dBr after 20 steps (checkpoints every 5) by the adjoint sweep
    against the forward tangent sweep along seeded B_r directions."""
    from paper_2209_04481_amd.sensitivity import Sensitivity
    print(f"case: sensitivity {name}", flush=True)
    inst = ci.workload(name) if name == "medium" else ci.make_instance(8, 4, "log", lmax=4, seed=12)
    ctx = context(inst, limiter=limiter)
    U0 = torch.from_numpy(inst.U).cuda()
    br = torch.from_numpy(inst.br).cuda()
    sens = Sensitivity(ctx, U0, cfl=cfl, nsteps=20, every=5, max_restarts=16, layer=layer)
    t0 = time.time()
    L, gb = sens.gradient(br)
    torch.cuda.synchronize()
    print(f"sensitivity {name}: L = {L:.12e}, gradient {time.time() - t0:.2f} s, worst solve rel {sens.max_rel:.1e}")
    assert sens.max_rel <= 1e-12
    dirs = _map_dirs(ctx, br, ndir)
    t0 = time.time()
    Lt, dLs = sens.tangents(br, dirs, log=lambda s: print("  " + s, flush=True))
    print(f"  {ndir} tangent sweeps sharing one trajectory: {time.time() - t0:.2f} s")
    assert Lt == L
    for q, (d, dL) in enumerate(zip(dirs, dLs)):
        ad = float((gb * d).sum())
        print(f"  dir {q}: tangent {dL:.12e} adjoint {ad:.12e} rel {abs(dL - ad) / abs(dL):.2e}")
        assert abs(dL - ad) <= tol * abs(dL)
    # the shared-trajectory sweep is the single-direction sweep (checked on the small grid)
    if name == "outer4":
        L1, dL1 = sens.tangent(br, dirs[0])
        assert L1 == L and abs(dL1 - dLs[0]) <= 1e-12 * abs(dL1)
