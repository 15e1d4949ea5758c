"""Pins of the oracle's cubed-sphere grid (CPU only)."""
import math

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from oracle.grid import Grid

DT = torch.float64


def small_grid(N=4, Nr=6, radial="log"):
    return Grid(N, Nr, ci.radial_nodes(Nr, radial))


@pytest.mark.parametrize("N,Nr,radial", [(4, 6, "log"), (8, 16, "geometric"), (6, 5, "log")])
def test_face_counts_and_kinds(N, Nr, radial):
    g = Grid(N, Nr, ci.radial_nodes(Nr, radial))
    L, R, kind = g.face_list()
    nb = 6 * N * N
    assert L.numel() == 6 * N * N * (Nr + 1) + 12 * N * N * Nr - 0 * nb
    assert int((kind == 1).sum()) == nb and int((kind == 2).sum()) == nb
    # canonical orientation: interior faces go from the lower to the higher index
    inter = kind == 0
    assert bool((R[inter] > L[inter]).all())
    assert bool((L[1:] >= L[:-1]).all())


def test_neighbour_reciprocity_and_degree():
    g = small_grid(5, 7)
    cells = torch.arange(g.ncells)
    nb = g.neighbours(cells)
    inner = nb < g.ncells
    back = g.neighbours(nb[inner])
    assert bool((back == cells[:, None].expand_as(nb)[inner][:, None]).any(1).all())
    # every cell has 6 distinct neighbours
    s, _ = torch.sort(nb, dim=1)
    assert bool((s[:, 1:] != s[:, :-1]).all())


@pytest.mark.parametrize("radial", ["log", "bcind"])
def test_point_location_matches_centroid_matching(radial):
    """Independent derivation: pair faces by coincident centroids (brute force
    on the sorted rounded coordinates) and compare with point location; also
    on the extended grid whose last layer (0.01 thick at r = 25) is thinner
    than the curvature of its angular faces."""
    g = Grid(4, 5, ci.radial_nodes(5, radial))
    cells = torch.arange(g.ncells)
    xc, V, xf, S = g.cell_geometry(cells)
    nb = g.neighbours(cells)
    pts = xf.reshape(-1, 3).numpy()
    owner = np.repeat(np.arange(g.ncells), 6)
    key = np.round(pts / 1e-9).astype(np.int64)
    order = np.lexsort(key.T[::-1])
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    match = {}
    for a in np.nonzero(same)[0]:
        fa, fb = order[a], order[a + 1]
        match[fa] = owner[fb]
        match[fb] = owner[fa]
    flat = nb.reshape(-1).numpy()
    for f in range(flat.size):
        if flat[f] < g.ncells:
            assert match[f] == flat[f]
        else:
            assert f not in match


def test_geometric_closure_outward_and_planarity():
    g = small_grid(6, 8)
    cells = torch.arange(g.ncells)
    xc, V, xf, S = g.cell_geometry(cells)
    scale = S.norm(dim=-1).sum(1)
    assert float((S.sum(1).norm(dim=-1) / scale).max()) < 1e-14
    assert bool((((xf - xc[:, None]) * S).sum(-1) > 0).all())
    # angular faces contain the origin: x_f . S_f = 0
    ang = (xf[:, 2:] * S[:, 2:]).sum(-1) / (xf[:, 2:].norm(dim=-1) * S[:, 2:].norm(dim=-1))
    assert float(ang.abs().max()) < 1e-14
    assert bool((V > 0).all())


def test_volume_converges_to_shell_second_order():
    exact = 4.0 * math.pi / 3.0 * (21.5 ** 3 - 1.0)
    errs = []
    for N in (4, 8, 16):
        g = Grid(N, 3, ci.radial_nodes(3, "log"))
        _, V, _, _ = g.cell_geometry(torch.arange(g.ncells))
        errs.append(exact - float(V.sum()))
    assert all(e > 0 for e in errs)          # inscribed polyhedra
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.8


def test_rotation_about_z_maps_grid_onto_itself():
    N, Nr = 4, 3
    g = Grid(N, Nr, ci.radial_nodes(Nr, "log"))
    rot = torch.tensor([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], dtype=DT)
    cells = torch.arange(g.ncells)
    p, k, j, i = g.decode(cells)
    xc, _, _, _ = g.cell_geometry(cells)
    # P0->P1->P2->P3->P0 with the same (i, j); P4: (i, j) -> (N-1-j, i);
    # P5: (i, j) -> (j, N-1-i)
    p2 = torch.where(p < 4, (p + 1) % 4, p)
    i2 = torch.where(p == 4, N - 1 - j, torch.where(p == 5, j, i))
    j2 = torch.where(p == 4, i, torch.where(p == 5, N - 1 - i, j))
    img = g.encode(p2, k, j2, i2)
    assert torch.allclose(xc @ rot.T, xc[img], atol=1e-13, rtol=0)


def test_ghost_centres_mirror_the_boundary_cell():
    g = small_grid(4, 4)
    gids = torch.arange(g.ncells, g.ncells + 2 * g.nb)
    cell, lf, outer, _ = g.ghost_cell(gids)
    xg = g.ghost_centres(gids)
    xc, _, xf, S = g.cell_geometry(cell)
    ar = torch.arange(cell.numel())
    n = S[ar, lf] / S[ar, lf].norm(dim=-1, keepdim=True)
    dI = ((xf[ar, lf] - xc) * n).sum(-1)
    dG = ((xg - xf[ar, lf]) * n).sum(-1)
    assert torch.allclose(dI, dG, rtol=1e-13, atol=0)
    assert bool((dI > 0).all())
    # inner ghosts lie inside the inner radius, outer ghosts outside the outer
    rG = xg.norm(dim=-1)
    assert bool((rG[~outer] < 1.0).all()) and bool((rG[outer] > 21.5 * 0.97).all())
