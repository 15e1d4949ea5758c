"""Pins of the oracle's JVP, VJP, GMRES and Eq. 2 monitor (CPU only)."""
import numpy as np
import pytest
import torch

import coronal_inputs as ci
from oracle import mhd, solve
from oracle.grid import Grid

DT = torch.float64


@pytest.fixture(scope="module")
def tiny():
    inst = ci.workload("tiny")
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    return g, torch.tensor(inst.U), torch.tensor(inst.br), inst


def test_jvp_matches_central_differences(tiny):
    g, U, br, inst = tiny
    prm = mhd.Params()
    v = torch.tensor(ci.scaled_direction(inst.U, inst.seed))
    dbr = torch.tensor(ci.br_direction(g.nb, inst.seed))
    Jv, R = solve.jvp(g, U, br, prm, v, dbr)
    assert torch.equal(R, mhd.residual(g, U, br, prm))
    eps = 1e-6
    fd = (mhd.residual(g, U + eps * v, br + eps * dbr, prm)
          - mhd.residual(g, U - eps * v, br - eps * dbr, prm)) / (2 * eps)
    assert float((fd - Jv).norm() / Jv.norm()) < 1e-8


def test_vjp_dot_product_and_fd_columns(tiny):
    g, U, br, inst = tiny
    prm = mhd.Params()
    gen = torch.Generator().manual_seed(3)
    # psi = 0 everywhere puts the limiter on its zero-gradient branch, where
    # w.R is not differentiable in psi; give psi a little noise here.
    U = U.clone()
    U[8] = 1e-3 * torch.randn(g.ncells, dtype=DT, generator=gen)
    w = torch.randn(9, g.ncells, dtype=DT, generator=gen)
    v = torch.tensor(ci.scaled_direction(inst.U, inst.seed + 1))
    dbr = torch.tensor(ci.br_direction(g.nb, inst.seed + 1))
    gU, gb = solve.vjp(g, U, br, prm, w)
    Jv, _ = solve.jvp(g, U, br, prm, v, dbr)
    lhs = float((w * Jv).sum())
    rhs = float((gU * v).sum() + (gb * dbr).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + float((w.abs() * Jv.abs()).sum()))
    # brute force: d(w.R)/dU_{a,c} by central differences for sampled entries
    rng = np.random.default_rng(0)
    scale = U.abs().amax(1)
    for _ in range(12):
        a, c = int(rng.integers(9)), int(rng.integers(g.ncells))
        h = 1e-6 * float(max(abs(U[a, c]), 1e-3 * scale[a], 1e-4))
        Up, Um = U.clone(), U.clone()
        Up[a, c] += h
        Um[a, c] -= h
        fd = float((w * (mhd.residual(g, Up, br, prm) - mhd.residual(g, Um, br, prm))).sum()) / (2 * h)
        assert abs(fd - float(gU[a, c])) <= 1e-6 * abs(fd) + 1e-9 * float(gU[a].abs().max())
    for col in rng.integers(g.nb, size=4):
        h = 1e-6
        bp, bm = br.clone(), br.clone()
        bp[col] += h
        bm[col] -= h
        fd = float((w * (mhd.residual(g, U, bp, prm) - mhd.residual(g, U, bm, prm))).sum()) / (2 * h)
        assert abs(fd - float(gb[col])) <= 1e-6 * abs(fd) + 1e-9 * float(gb.abs().max())


def test_vjp_on_subset_is_exact_locally(tiny):
    """gU at a cell depends only on w within distance 2: restricting w to the
    distance-2 stencil of a sample reproduces the full VJP there."""
    g, U, br, inst = tiny
    prm = mhd.Params()
    w = torch.randn(9, g.ncells, dtype=DT, generator=torch.Generator().manual_seed(4))
    gU, _ = solve.vjp(g, U, br, prm, w)
    sample = torch.tensor([10, 777, 3000])
    st = mhd._Stencil(g, sample)
    T = st.D2
    gUs, _ = solve.vjp(g, U, br, prm, w[:, T], cells=T)
    assert torch.allclose(gUs[:, sample], gU[:, sample], rtol=1e-13, atol=1e-13 * float(gU.abs().max()))


def test_gmres_minimises_over_krylov_space_and_solves_exactly():
    rng = np.random.default_rng(1)
    n = 12
    A = torch.tensor(rng.standard_normal((n, n)) + 4 * np.eye(n))
    b = torch.tensor(rng.standard_normal(n))
    x, hist = solve.gmres(lambda y: A @ y, b, m=n)
    assert torch.allclose(x, torch.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # history: min over the j-dimensional Krylov space, by explicit lstsq
    K = [b]
    for j in range(1, 6):
        Kb = torch.stack(K, 1)
        Q, _ = torch.linalg.qr(Kb)
        y = torch.linalg.lstsq(A @ Q, b).solution
        assert abs(float((b - A @ Q @ y).norm() / b.norm()) - hist[j - 1]) < 1e-12
        K.append(A @ K[-1])
    assert all(hist[i + 1] <= hist[i] + 1e-15 for i in range(len(hist) - 1))


def test_right_preconditioned_gmres_minimises_over_the_preconditioned_space():
    """GMRES on A M^-1 with x = M^-1 y: exact at m = n, its history the
    minimum of |b - A x| over x in M^-1 K_j(A M^-1, b) (explicit lstsq),
    and one iteration when M = A is diagonal."""
    rng = np.random.default_rng(2)
    n = 12
    A = torch.tensor(rng.standard_normal((n, n)) + 4 * np.eye(n))
    d = torch.tensor(rng.uniform(0.5, 20.0, n))
    b = torch.tensor(rng.standard_normal(n))
    Minv = lambda v: v / d
    x, hist = solve.gmres(lambda y: A @ y, b, m=n, precond=Minv)
    assert torch.allclose(x, torch.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    AM = A / d[None, :]
    K = [b]
    for j in range(1, 6):
        Q, _ = torch.linalg.qr(torch.stack(K, 1))
        y = torch.linalg.lstsq(AM @ Q, b).solution
        assert abs(float((b - A @ (Minv(Q @ y))).norm() / b.norm()) - hist[j - 1]) < 1e-12
        K.append(AM @ K[-1])
    D = torch.diag(d)
    x1, h1 = solve.gmres(lambda y: D @ y, b, m=5, precond=Minv)
    assert h1[0] < 1e-14 and torch.allclose(x1, b / d, rtol=1e-14)


def test_eq2_monitor():
    a = torch.tensor([[1.0, 2.0, 3.0], [0.0, 0.0, 1.0]], dtype=DT)
    b = torch.tensor([[1.0, 2.0, 2.0], [3.0, 4.0, 1.0]], dtype=DT)
    out = solve.eq2(a, b)
    assert torch.allclose(out, torch.tensor([0.0, np.log10(5.0)], dtype=DT))


def test_step_map_gradient_matches_central_differences():
    """The oracle's exact B_r gradient after two implicit steps (dense
    Jacobians, reverse mode through the solves) against central differences
    of the objective at two step sizes, with the diagonal held fixed."""
    import numpy as np
    import coronal_inputs as ci
    inst = ci.make_instance(2, 2, "log", lmax=2, seed=5)
    g = Grid(2, 2, inst.r_nodes)
    prm = mhd.Params()
    U0, br = torch.from_numpy(inst.U), torch.from_numpy(inst.br)
    D0 = solve.local_dt_diag(g, U0, br, prm, 1.0)
    lam = solve.layer_objective(g, 0)
    L, gb = solve.step_map_sensitivity(g, U0, br, prm, D0, 2, lam)
    rng = np.random.default_rng(1)
    for _ in range(2):
        d = torch.from_numpy(rng.standard_normal(g.nb)) * float(br.abs().max()) * 1e-2
        fd = []
        for h in (1e-3, 1e-4):
            Lp, _ = solve.step_map_sensitivity(g, U0, br + h * d, prm, D0, 2, lam, want_grad=False)
            Lm, _ = solve.step_map_sensitivity(g, U0, br - h * d, prm, D0, 2, lam, want_grad=False)
            fd.append((Lp - Lm) / (2 * h))
        ad = float((gb * d).sum())
        assert abs(fd[0] - fd[1]) <= 1e-6 * abs(fd[0])
        assert abs(ad - fd[1]) <= 1e-6 * abs(fd[1])


def test_layer_objective_weights():
    """lam picks rho v . r_hat at the upper face centroid of every cell of
    the layer, each with weight 1/(6N^2)."""
    g = Grid(3, 4, torch.linspace(1.0, 2.0, 5, dtype=torch.float64))
    lam = solve.layer_objective(g, 2)
    U = torch.zeros(9, g.ncells, dtype=torch.float64)
    cells = torch.arange(g.ncells)
    p, k, j, i = g.decode(cells)
    _, _, xf, _ = g.cell_geometry(cells)
    rh = xf[:, 1] / torch.linalg.norm(xf[:, 1], dim=-1, keepdim=True)
    U[1:4] = rh.T  # unit radial momentum at every cell
    assert abs(float((lam * U).sum()) - 1.0) < 1e-14
    assert float(lam[:, k != 2].abs().max()) == 0.0
    assert float(lam[[0, 4, 5, 6, 7, 8]].abs().max()) == 0.0
