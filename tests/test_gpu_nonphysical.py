"""The non-physical state flag through the C ABI (GPU).

The reconstruction applies no positivity fix-up; instead a face state whose
density or pressure is not positive (NaN included) is recorded in a flag word
that the synchronising entry points turn into status 4.  One cell of a tiny
shell has its energy lowered until its pressure is negative (a host-forced
condition: every kernel still exits normally), and:
  * the residual, the JVP and the VJP set the flag, a normal state leaves it
    clear, and the flag changes no output;
  * a backward-Euler step goes on through such a state (no fix-up) and
    leaves the flag set; a NaN state makes cfv_be_step and cfv_steady return
    status 4 (the march keeps the state before the failing step), and so
    does cfv_solve on a NaN right-hand side;
  * in a batched march an instance with a NaN stops with its state
    unchanged while the others march on, its status word says so, and the
    call returns status 4."""
import numpy as np
import pytest
import torch

import coronal_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make(seed=3, N=4, Nr=6):
    from paper_2209_04481_amd import Context, Grid, Params
    inst = ci.make_instance(N, Nr, "log", lmax=2, seed=seed)
    ctx = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
    ctx.set_inner_br(torch.from_numpy(inst.br).cuda())
    return inst, ctx


def negative_pressure(U, cell):
    """Lower the energy of one cell so that p = (gamma-1)(E - kinetic - magnetic) < 0."""
    U = U.clone()
    rho = U[0, cell]
    kin = 0.5 * (U[1:4, cell] ** 2).sum() / rho
    mag = 0.5 * (U[4:7, cell] ** 2).sum()
    U[7, cell] = 0.5 * (kin + mag)
    return U


def test_flag_clear_on_a_normal_state_and_set_by_every_operator():
    print("case: flag on a 6x4x4x6 shell, cell 3*16+5 forced to negative pressure", flush=True)
    inst, ctx = make()
    U = torch.from_numpy(inst.U)
    Ud = U.cuda()
    v = torch.randn(9, inst.ncells, dtype=torch.float64, generator=torch.Generator().manual_seed(1)).cuda()
    R0 = ctx.residual(Ud)
    Jv0 = ctx.jvp(Ud, v)
    gU0, _ = ctx.vjp(Ud, v)
    assert ctx.status_flags() == 0
    bad = negative_pressure(U, 3 * 16 + 5).cuda()
    for name, call in (("residual", lambda: ctx.residual(bad)), ("jvp", lambda: ctx.jvp(bad, v)),
                       ("vjp", lambda: ctx.vjp(bad, v))):
        assert ctx.status_flags() == 0
        call()
        assert ctx.status_flags() & 1, name
    assert ctx.status_flags() == 0                      # reading clears it
    # the flag changes no output: the normal state again, bit for bit
    assert torch.equal(ctx.residual(Ud), R0)
    assert torch.equal(ctx.jvp(Ud, v), Jv0)
    assert torch.equal(ctx.vjp(Ud, v)[0], gU0)
    assert ctx.status_flags() == 0


def nan_state(U, cell):
    """A NaN in one cell's energy (a host-forced corrupt state)."""
    U = U.clone()
    U[7, cell] = float("nan")
    return U


def test_be_step_reports_and_fails_only_on_non_finite_solves():
    from paper_2209_04481_amd import CfvNonPhysical
    print("case: be_step / steady / solve on forced states, 6x4x4x6", flush=True)
    inst, ctx = make()
    U = torch.from_numpy(inst.U)
    # a negative pressure: the step goes on (no fix-up) and the flag reports it
    bad = negative_pressure(U, 2 * 16 + 7).cuda()
    assert ctx.status_flags() == 0
    Un, _ = ctx.be_step(bad, cfl=10.0, m=5)
    assert bool(torch.isfinite(Un).all())
    assert ctx.status_flags() & 1
    # a NaN: the Krylov solve refuses the non-finite residual
    nan = nan_state(U, 2 * 16 + 7).cuda()
    with pytest.raises(CfvNonPhysical):
        ctx.be_step(nan, cfl=10.0, m=5)
    before = nan.clone()
    with pytest.raises(CfvNonPhysical) as ei:
        ctx.steady(nan, 4, cfl0=2.0, cfl_max=8.0, every=2, m=5)
    assert len(ei.value.cfls) == 1 and np.isnan(ei.value.hist).all()
    assert torch.equal(torch.isnan(nan), torch.isnan(before))   # the state before the failing step
    assert torch.equal(nan[~torch.isnan(nan)], before[~torch.isnan(before)])
    ctx.status_flags()
    # a normal state steps without error and leaves the flag clear
    ctx.be_step(U.cuda(), cfl=10.0, m=5)
    assert ctx.status_flags() == 0
    # a NaN right-hand side
    rhs = torch.zeros(9, inst.ncells, dtype=torch.float64, device="cuda")
    rhs[0, 0] = float("nan")
    diag = torch.ones(inst.ncells, dtype=torch.float64, device="cuda")
    with pytest.raises(CfvNonPhysical):
        ctx.solve(U.cuda(), diag, rhs, m=3)


def test_ensemble_march_stops_the_failing_instance_only():
    from paper_2209_04481_amd import CfvNonPhysical, Ensemble
    print("case: batched runs of 3 instances, the second with a forced negative pressure, then with a NaN",
          flush=True)
    insts, ctxs = [], []
    for q in range(3):
        inst, ctx = make(seed=20 + q, N=4 + q, Nr=5)
        insts.append(inst)
        ctxs.append(ctx)
    U = [torch.from_numpy(i.U).cuda() for i in insts]
    ens = Ensemble(ctxs)
    # residual + JVP of the ensemble: only the instance with the negative pressure is flagged
    Ub = list(U)
    Ub[1] = negative_pressure(U[1].cpu(), 11).cuda()
    v = [torch.ones_like(u) for u in U]
    ens.residual_jvp(Ub, v)
    flags = ens.status_flags()
    assert list(flags & 1) == [0, 1, 0] and not (flags & 2).any()
    assert list(ens.status_flags()) == [0, 0, 0]
    # the batched march: the instance with a NaN stops at its first step, the others march on
    U[1] = nan_state(U[1].cpu(), 11).cuda()
    U1 = U[1].clone()
    U0 = U[0].clone()
    with pytest.raises(CfvNonPhysical) as ei:
        ens.steady(U, 3, cfl0=2.0, cfl_max=8.0, every=2, m=5)
    steps = ei.value.cfls
    assert steps[1] == 1 and steps[0] == 3 and steps[2] == 3
    assert torch.equal(torch.isnan(U[1]), torch.isnan(U1))
    assert torch.equal(U[1][~torch.isnan(U1)], U1[~torch.isnan(U1)])   # the failing instance keeps its state
    assert not torch.equal(U[0], U0)                                     # the others marched
    flags = ens.status_flags()
    assert flags[1] & 2 and not (flags[0] & 2) and not (flags[2] & 2)
