"""The batched ensemble against the oracle (GPU, through the C ABI).

The other ensemble tests compare the batched launch with each instance's own
single-instance launch; these compare it with the CPU oracle directly:

  * the 64-instance, 29.95M-cell ensemble (uneven shells, each its own seeded
    state and magnetogram), residual and JVP with a B_r direction in one
    persistent launch per pass: sampled cells of three instances (the
    smallest 16 x 16 x 40 panels, the largest 48 x 48 x 120, and one between)
    against the oracle on their distance-2 stencils, to 1e-12 per variable;
  * the lockstep backward-Euler step (GMRES on the device for every instance
    at once): small instances against the oracle's backward-Euler step, the
    relative-residual history to 1e-9 and the update to 1e-8 (rounding of
    the Krylov solves grows over the iterations)."""
import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import rel_err_per_var
from oracle import mhd, solve
from oracle.grid import Grid as OGrid

pytestmark = pytest.mark.gpu
TOL = 1e-12


def sample_cells(inst, n, seed):
    """Random cells plus boundary layers and panel edges and corners."""
    rng = np.random.default_rng(seed)
    N, Nr = inst.N, inst.Nr
    picks = list(rng.integers(0, inst.ncells, size=n))
    for p in range(6):
        for (k, j, i) in ((0, 0, 0), (Nr - 1, N - 1, N - 1), (0, N - 1, 0), (Nr // 2, 0, N - 1), (Nr - 1, N // 2, 0),
                          (1, 15, 16), (Nr - 2, 16, 15)):
            if j < N and i < N:
                picks.append(((p * Nr + k) * N + j) * N + i)
    return torch.tensor(sorted(set(int(x) for x in picks)))


@pytest.fixture(scope="module")
def ens64():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_04481_amd import Context, Ensemble, Grid, Params
    print("case: 64-instance ensemble vs oracle (inputs)", flush=True)
    insts = ci.ensemble_instances()
    ctxs, U, v, dbr = [], [], [], []
    for q, inst in enumerate(insts):
        c = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
        c.set_inner_br(torch.from_numpy(inst.br).cuda())
        ctxs.append(c)
        U.append(torch.from_numpy(inst.U).cuda())
        v.append(torch.from_numpy(ci.scaled_direction(inst.U, 900 + q)).cuda())
        dbr.append(torch.from_numpy(ci.br_direction(c.grid.nb, 950 + q)).cuda())
    ens = Ensemble(ctxs)
    R = [torch.full_like(u, float("nan")) for u in U]
    J = [torch.full_like(u, float("nan")) for u in U]
    ens.bind(U, v=v, dbr=dbr, R=R, Jv=J)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ens.capture(s)
    ens.replay(s)
    s.synchronize()
    return insts, v, dbr, R, J


def pick_instances(insts):
    shapes = [(i.N, i.Nr) for i in insts]
    small = shapes.index((16, 40))
    large = shapes.index((48, 120))
    mid = shapes.index((24, 80))
    return [small, mid, large]


def test_batched_residual_and_jvp_match_the_oracle(ens64):
    insts, v, dbr, R, J = ens64
    for q in pick_instances(insts):
        inst = insts[q]
        print(f"case: ensemble instance {q} ({inst.N}, {inst.Nr}) vs oracle", flush=True)
        og = OGrid(inst.N, inst.Nr, inst.r_nodes)
        U = torch.from_numpy(inst.U)
        br = torch.from_numpy(inst.br)
        S = sample_cells(inst, 60, 100 + q)
        Ro = mhd.residual(og, U, br, mhd.Params(), cells=S)
        Jo, _ = solve.jvp(og, U, br, mhd.Params(), v[q].cpu(), dbr[q].cpu(), cells=S)
        Sd = S.cuda()
        assert float(rel_err_per_var(R[q][:, Sd].cpu(), Ro).max()) <= TOL, f"R of instance {q}"
        assert float(rel_err_per_var(J[q][:, Sd].cpu(), Jo).max()) <= TOL, f"Jv of instance {q}"


def test_lockstep_backward_euler_step_matches_the_oracle():
    from paper_2209_04481_amd import Context, Ensemble, Grid, Params
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    shapes = [(4, 5), (5, 7), (6, 4)]
    insts = [ci.make_instance(N, Nr, "log", lmax=3, seed=60 + q) for q, (N, Nr) in enumerate(shapes)]
    ctxs, U = [], []
    for inst in insts:
        c = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
        c.set_inner_br(torch.from_numpy(inst.br).cuda())
        ctxs.append(c)
        U.append(torch.from_numpy(inst.U).cuda())
    m, cfl = 12, 1e3
    print(f"case: lockstep backward-Euler step of {shapes} vs oracle, GMRES({m}), CFL {cfl:g}", flush=True)
    ens = Ensemble(ctxs)
    Un, hist = ens.be_step(U, cfl=cfl, m=m)
    torch.cuda.synchronize()
    for q, inst in enumerate(insts):
        og = OGrid(inst.N, inst.Nr, inst.r_nodes)
        Uo = torch.from_numpy(inst.U)
        Uno, ho, _ = solve.be_step(og, Uo, torch.from_numpy(inst.br), mhd.Params(), cfl, m)
        ho = np.array(ho)
        hb = hist[q].cpu().numpy()[:len(ho)]
        assert np.all(np.abs(hb - ho) <= 1e-9 * np.abs(ho)), f"history of instance {q} {shapes[q]}"
        dx, dxo = (Un[q].cpu() - Uo), (Uno - Uo)
        assert float(rel_err_per_var(dx, dxo).max()) <= 1e-8, f"update of instance {q} {shapes[q]}"
