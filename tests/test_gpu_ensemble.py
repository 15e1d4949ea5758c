"""GPU checks of the batched ensemble launch: every instance's residual and
JVP equal, bit for bit, those of its own single-instance launch, for every
schedule and chunk length, and a captured graph replays to the same bits."""
import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import rel_err_per_var

pytestmark = pytest.mark.gpu

# uneven shapes: partial tiles (N not a multiple of 16), partial chunks, a
# single layer, N = 2, odd N (polar-axis faces)
SHAPES = [(8, 12), (16, 20), (24, 40), (5, 7), (12, 1), (33, 17), (2, 3), (17, 33)]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_04481_amd import Context, Grid, Params
    insts = [ci.make_instance(N, Nr, "log", lmax=4, seed=100 + q) for q, (N, Nr) in enumerate(SHAPES)]
    ctxs, U, v, dbr = [], [], [], []
    for q, inst in enumerate(insts):
        g = Grid(inst.N, inst.Nr, inst.r_nodes)
        c = Context(g, Params())
        c.set_inner_br(torch.from_numpy(inst.br).cuda())
        ctxs.append(c)
        U.append(torch.from_numpy(inst.U).cuda())
        v.append(torch.from_numpy(ci.scaled_direction(inst.U, 500 + q)).cuda())
        dbr.append(torch.from_numpy(ci.br_direction(6 * inst.N ** 2, 700 + q)).cuda())
    R1, J1, R0 = [], [], []
    for c, u, w, b in zip(ctxs, U, v, dbr):
        r = torch.empty_like(u)
        J1.append(c.jvp(u, w, dbr=b, R=r))
        R1.append(r)
        R0.append(c.residual(u))
    torch.cuda.synchronize()
    return ctxs, U, v, dbr, R1, J1, R0


def _same(a, b):
    return torch.equal(a, b) or bool(((a == b) | (torch.isnan(a) & torch.isnan(b))).all())


@pytest.mark.parametrize("queue,bpc,order,kc", [(0, 1, 0, 0), (0, 2, 1, 5), (1, 1, 0, 1), (1, 4, 1, 64),
                                                (1, 2, 1, 8)])
def test_ensemble_matches_single_instance_launches(setup, queue, bpc, order, kc):
    from paper_2209_04481_amd import Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    print(f"case: ensemble schedule queue={queue} bpc={bpc} order={order} chunk={kc}", flush=True)
    ens = Ensemble(ctxs, Tuning(queue, bpc, order, kc))
    R = [torch.full_like(u, float("nan")) for u in U]
    J = [torch.full_like(u, float("nan")) for u in U]
    ens.bind(U, v=v, dbr=dbr, R=R, Jv=J)
    ens.run()
    torch.cuda.synchronize()
    for q in range(len(U)):
        assert _same(R[q], R1[q]), f"R of instance {q} {SHAPES[q]}"
        assert _same(J[q], J1[q]), f"Jv of instance {q} {SHAPES[q]}"
    # residual-only pass
    Rr = [torch.full_like(u, float("nan")) for u in U]
    ens.bind(U, R=Rr)
    ens.run()
    torch.cuda.synchronize()
    for q in range(len(U)):
        assert _same(Rr[q], R0[q]), f"residual of instance {q} {SHAPES[q]}"


def test_ensemble_graph_replays_match_eager(setup):
    from paper_2209_04481_amd import Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    print("case: ensemble graph capture", flush=True)
    ens = Ensemble(ctxs, Tuning(1, 2, 1))
    R = [torch.empty_like(u) for u in U]
    J = [torch.empty_like(u) for u in U]
    ens.bind(U, v=v, dbr=dbr, R=R, Jv=J)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ens.capture(s)
    for rep in range(3):
        for t in R + J:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        ens.replay(s)
        s.synchronize()
        for q in range(len(U)):
            assert _same(R[q], R1[q]) and _same(J[q], J1[q]), f"replay {rep}, instance {q}"
        # eager work of the program between replays
        _ = ctxs[0].residual(U[0])
        torch.cuda.synchronize()


def test_ensemble_chunk_change_after_binding(setup):
    """set_tuning with a new chunk length rebuilds the item lists (longer and
    shorter ones) under a bound run; the outputs keep their bits."""
    from paper_2209_04481_amd import Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    print("case: ensemble chunk change after binding", flush=True)
    ens = Ensemble(ctxs, Tuning(1, 2, 1, 16))
    R = [torch.empty_like(u) for u in U]
    J = [torch.empty_like(u) for u in U]
    ens.bind(U, v=v, dbr=dbr, R=R, Jv=J)
    for kc in (2, 40, 3, 0):
        for t in R + J:
            t.fill_(float("nan"))
        ens.set_tuning(Tuning(0, 2, 1, kc))
        ens.run()
        torch.cuda.synchronize()
        for q in range(len(U)):
            assert _same(R[q], R1[q]) and _same(J[q], J1[q]), f"chunk {kc}, instance {q}"


def test_ensemble_rejects_bad_bindings(setup):
    from paper_2209_04481_amd import CfvError, Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    for kc in (-1, 4097):
        with pytest.raises(CfvError):
            Ensemble(ctxs, Tuning(1, 2, 1, kc))
    ens = Ensemble(ctxs)
    with pytest.raises(CfvError):
        ens.run()  # nothing bound
    with pytest.raises(CfvError):
        ens.bind(U[:-1], R=R1[:-1])
    with pytest.raises(CfvError):
        ens.bind(U, v=v)  # JVP without outputs
    with pytest.raises(CfvError):
        ens.replay(torch.cuda.Stream())  # nothing captured


def test_autotune_picks_a_listed_schedule_and_depth(setup, tmp_path, monkeypatch):
    from paper_2209_04481_amd import Ensemble
    from paper_2209_04481_amd.autotune import CHUNKS, SCHEDULES, autotune
    ctxs, U, v, dbr, R1, J1, R0 = setup
    monkeypatch.setenv("CFV_TUNE_CACHE", str(tmp_path / "tune.json"))
    ens = Ensemble(ctxs)
    R = [torch.empty_like(u) for u in U]
    J = [torch.empty_like(u) for u in U]
    ens.bind(U, v=v, R=R, Jv=J)
    best, ms = autotune(ens, reps=2)
    sched = {(t.queue, t.blocks_per_cu, t.order) for t in SCHEDULES}
    assert (best.queue, best.blocks_per_cu, best.order) in sched and best.chunk_layers in (0,) + tuple(CHUNKS)
    assert len(ms) == len(SCHEDULES) + len(CHUNKS) and min(ms.values()) == ms[repr(best)]
    again, _ = autotune(ens, reps=2)  # from the cache
    assert repr(again) == repr(best)
    ens.run()
    torch.cuda.synchronize()
    for q in range(len(U)):
        assert _same(R[q], R1[q]), f"R of instance {q} under {best}"


def test_ensemble_64_instances_sampled(setup):
    """The 64-instance, 29.95M-cell ensemble: batched output of a sample of
    instances equals their single-instance launches bit for bit."""
    from paper_2209_04481_amd import Context, Ensemble, Grid, Params
    print("case: 64-instance ensemble", flush=True)
    insts = ci.ensemble_instances()
    assert sum(i.ncells for i in insts) == 29_952_000
    ctxs, U, v = [], [], []
    for q, inst in enumerate(insts):
        c = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
        c.set_inner_br(torch.from_numpy(inst.br).cuda())
        ctxs.append(c)
        U.append(torch.from_numpy(inst.U).cuda())
        v.append(torch.from_numpy(ci.scaled_direction(inst.U, 900 + q)).cuda())
    ens = Ensemble(ctxs)
    R, J = ens.residual_jvp(U, v)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for q in sorted(rng.choice(64, 6, replace=False).tolist()):
        r = torch.empty_like(U[q])
        j = ctxs[q].jvp(U[q], v[q], R=r)
        torch.cuda.synchronize()
        assert _same(R[q], r) and _same(J[q], j), f"instance {q} ({insts[q].N}, {insts[q].Nr})"


def test_ensemble_jacobi_be_step_matches_single_instance_steps(setup):
    """The lockstep step with the Jacobi preconditioner (CFL 10, GMRES(12))
    equals each instance's preconditioned cfv_be_step; a step bound before
    the preconditioner changes must be bound again."""
    from paper_2209_04481_amd import CfvError, Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    print("case: ensemble backward-Euler step, Jacobi", flush=True)
    ens = Ensemble(ctxs, Tuning(1, 2, 1))
    ens.set_preconditioner(1)
    Un, hist = ens.be_step(U, cfl=10.0, m=12)
    torch.cuda.synchronize()
    try:
        for q in range(len(U)):
            ctxs[q].set_preconditioner(1)
            Us, hs = ctxs[q].be_step(U[q], cfl=10.0, m=12)
            hb = hist[q].cpu().numpy()
            k = len(hs)
            assert np.all(np.abs(hb[:k] - hs) <= 1e-9 * np.abs(hs) + 1e-300), f"history of instance {q} {SHAPES[q]}"
            dx, dxs = (Un[q] - U[q]).cpu(), (Us - U[q]).cpu()
            assert float(rel_err_per_var(dx, dxs).max()) <= 1e-8, f"step of instance {q} {SHAPES[q]}"
    finally:
        for c in ctxs:
            c.set_preconditioner(0)
    ens.set_preconditioner(0)
    with pytest.raises(CfvError):
        ens.run()  # the bound step was dropped
    with pytest.raises(CfvError):
        ens.set_preconditioner(3)


def test_ensemble_be_step_matches_single_instance_steps(setup):
    """One backward-Euler step (CFL 1e3, GMRES(12)) of every instance in
    lockstep on the device equals cfv_be_step of each instance: the same
    arithmetic except the order of the reductions and where the Givens
    rotations are applied (device vs host)."""
    from paper_2209_04481_amd import Ensemble, Tuning
    ctxs, U, v, dbr, R1, J1, R0 = setup
    print("case: ensemble backward-Euler step", flush=True)
    ens = Ensemble(ctxs, Tuning(1, 2, 1))
    Un, hist = ens.be_step(U, cfl=1e3, m=12)
    torch.cuda.synchronize()
    for q in range(len(U)):
        Us, hs = ctxs[q].be_step(U[q], cfl=1e3, m=12)
        hb = hist[q].cpu().numpy()
        k = len(hs)
        assert k >= 1
        assert np.all(np.abs(hb[:k] - hs) <= 1e-9 * np.abs(hs) + 1e-300), f"history of instance {q} {SHAPES[q]}"
        dx, dxs = (Un[q] - U[q]).cpu(), (Us - U[q]).cpu()
        assert float(rel_err_per_var(dx, dxs).max()) <= 1e-8, f"step of instance {q} {SHAPES[q]}"
    # captured: replays equal the eager run
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ref = [u.clone() for u in Un]
    href = hist.clone()
    ens.capture(s)
    for rep in range(2):
        for u in Un:
            u.fill_(float("nan"))
        hist.zero_()
        torch.cuda.synchronize()
        ens.replay(s)
        s.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(Un, ref)) and torch.equal(hist, href), f"replay {rep}"
