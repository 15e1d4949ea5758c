"""GPU checks of the torch.autograd binding: reverse mode equals the
library's VJP, forward mode (torch.func.jvp and forward_ad) equals its JVP,
and both equal the oracle's derivatives."""
import pytest
import torch

import coronal_inputs as ci
from helpers import rel_err_per_var
from oracle import mhd, solve
from oracle.grid import Grid as OGrid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_04481_amd import Context, Grid, Params
    inst = ci.make_instance(6, 9, "log", lmax=4, seed=31)
    ctx = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
    U = torch.from_numpy(inst.U).cuda()
    br = torch.from_numpy(inst.br).cuda()
    v = torch.from_numpy(ci.scaled_direction(inst.U, 32)).cuda()
    db = torch.from_numpy(ci.br_direction(6 * inst.N ** 2, 33)).cuda()
    w = torch.randn(9, inst.ncells, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(34))
    return inst, ctx, U, br, v, db, w


def test_backward_is_the_library_vjp_and_the_oracle_gradient(setup):
    from paper_2209_04481_amd import residual
    inst, ctx, U, br, v, db, w = setup
    Ur, brr = U.clone().requires_grad_(True), br.clone().requires_grad_(True)
    R = residual(Ur, brr, ctx)
    assert torch.equal(R.detach(), ctx.residual(U))
    (R * w).sum().backward()
    gU, gbr = ctx.vjp(U, w)
    assert torch.equal(Ur.grad, gU) and torch.equal(brr.grad, gbr)
    og = OGrid(inst.N, inst.Nr, inst.r_nodes)
    gUo, gbo = solve.vjp(og, torch.from_numpy(inst.U), torch.from_numpy(inst.br), mhd.Params(), w.cpu())
    assert float(rel_err_per_var(Ur.grad.cpu(), gUo).max()) <= 1e-12
    assert float((brr.grad.cpu() - gbo).abs().max() / gbo.abs().max()) <= 1e-12


def test_forward_mode_is_the_library_jvp(setup):
    from paper_2209_04481_amd import residual
    inst, ctx, U, br, v, db, w = setup
    R, Jv = torch.func.jvp(lambda a, b: residual(a, b, ctx), (U, br), (v, db))
    assert torch.equal(Jv, ctx.jvp(U, v, dbr=db))
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        out = residual(fwAD.make_dual(U, v), br, ctx)
        Jv2 = fwAD.unpack_dual(out).tangent
    assert torch.equal(Jv2, ctx.jvp(U, v))
    og = OGrid(inst.N, inst.Nr, inst.r_nodes)
    Jo, _ = solve.jvp(og, torch.from_numpy(inst.U), torch.from_numpy(inst.br), mhd.Params(), v.cpu(), dbr=db.cpu())
    assert float(rel_err_per_var(Jv.cpu(), Jo).max()) <= 1e-12


def test_only_requested_gradients_are_computed(setup):
    from paper_2209_04481_amd import residual
    inst, ctx, U, br, v, db, w = setup
    Ur = U.clone().requires_grad_(True)
    (residual(Ur, br, ctx) * w).sum().backward()
    assert torch.equal(Ur.grad, ctx.vjp(U, w, want_br=False)[0])
    brr = br.clone().requires_grad_(True)
    (residual(U, brr, ctx) * w).sum().backward()
    assert torch.equal(brr.grad, ctx.vjp(U, w)[1])
