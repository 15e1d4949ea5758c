"""Cubed-sphere hexahedral shell for the oracle (test infrastructure).

The paper solves on an unstructured shell grid from the inner boundary to
21.5 solar radii (Section 2.1).  The oracle uses a gnomonic equiangular cubed
sphere: panel p maps (a, b) = (tan xi, tan eta), xi, eta in [-pi/4, pi/4], to
the unnormalised directions

    P0 (1, a, b)   P1 (-a, 1, b)   P2 (-1, -a, b)
    P3 (a, -1, b)  P4 (-b, a, 1)   P5 (b, a, -1)

and vertex (p, k, j, i) sits at r_k * d/|d| with d from corner (a_i, b_j).
Cell (p, k, j, i) spans vertices i..i+1, j..j+1, k..k+1 and has index
c = ((p*Nr + k)*N + j)*N + i.

Geometry is computed straight from the eight vertices of each cell:
  face vector area  S = 1/2 (v2 - v0) x (v3 - v1)   (exact for the closed quad)
  face centroid     x_f = mean of its 4 vertices
  cell centroid     x_c = mean of its 8 vertices
  volume            V = 1/3 sum_f x_f . S_f
Faces are listed per cell in the local order (r-, r+, xi-, xi+, eta-, eta+),
with S pointing out of the cell.

Connectivity is derived by *point location*: a point just outside each face
is mapped back to (panel, i, j) by inverting the gnomonic map and to k by the
radial position.  No panel-edge table is used, so this is an independent
derivation of the grid's adjacency.

Ghost cells (Section 4.1: ghost and inner centres equidistant from the
boundary) are the mirror images of the boundary cell's centre in the boundary
face's plane.  Ghost ids: inner ghost of column g = (p*N + j)*N + i is
ncells + g, outer ghost is ncells + 6N^2 + g.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64

# vertex offsets (dk, dj, di) of the four vertices of each local face, ordered
# so that 1/2 (v2 - v0) x (v3 - v1) points out of the cell.
FACE_VERTS = (
    ((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)),   # r-
    ((1, 0, 0), (1, 0, 1), (1, 1, 1), (1, 1, 0)),   # r+
    ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)),   # xi-
    ((0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 1)),   # xi+
    ((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0)),   # eta-
    ((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)),   # eta+
)

KIND_INTERIOR, KIND_INNER, KIND_OUTER = 0, 1, 2


def panel_direction(p: int, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    one = torch.ones_like(a)
    comps = {
        0: (one, a, b), 1: (-a, one, b), 2: (-one, -a, b),
        3: (a, -one, b), 4: (-b, a, one), 5: (b, a, -one),
    }[p]
    return torch.stack(comps, dim=-1)


def locate_panel(y: torch.Tensor):
    """Invert the gnomonic map: (panel, a, b) of direction y (..., 3)."""
    x0, x1, x2 = y[..., 0], y[..., 1], y[..., 2]
    ax = torch.stack([x0, x1, -x0, -x1, x2, -x2], dim=-1)
    p = torch.argmax(ax, dim=-1)
    a = torch.empty_like(x0)
    b = torch.empty_like(x0)
    sel = [
        (x1 / x0, x2 / x0),          # P0: (1, a, b) * x0
        (-x0 / x1, x2 / x1),         # P1: (-a, 1, b) * x1
        (x1 / x0, -x2 / x0),         # P2: (-1, -a, b) * (-x0)
        (-x0 / x1, -x2 / x1),        # P3: (a, -1, b) * (-x1)
        (x1 / x2, -x0 / x2),         # P4: (-b, a, 1) * x2
        (-x1 / x2, -x0 / x2),        # P5: (b, a, -1) * (-x2)
    ]
    for q in range(6):
        m = p == q
        a[m] = sel[q][0][m]
        b[m] = sel[q][1][m]
    return p, a, b


class Grid:
    def __init__(self, N: int, Nr: int, r_nodes):
        self.N, self.Nr = int(N), int(Nr)
        self.r = torch.as_tensor(r_nodes, dtype=DT).clone()
        assert self.r.numel() == self.Nr + 1
        assert bool(torch.all(self.r[1:] > self.r[:-1]))
        self.ncells = 6 * self.N * self.N * self.Nr
        self.nb = 6 * self.N * self.N
        xi = -math.pi / 4 + torch.arange(self.N + 1, dtype=DT) * (math.pi / 2) / self.N
        t = torch.tan(xi)
        bb, aa = torch.meshgrid(t, t, indexing="ij")          # [j', i']
        d = torch.stack([panel_direction(p, aa, bb) for p in range(6)])
        self.corner = d / torch.linalg.norm(d, dim=-1, keepdim=True)  # [p, j', i', 3]

    # ---- indexing ---------------------------------------------------------
    def decode(self, c: torch.Tensor):
        N, Nr = self.N, self.Nr
        i = c % N
        j = (c // N) % N
        k = (c // (N * N)) % Nr
        p = c // (N * N * Nr)
        return p, k, j, i

    def encode(self, p, k, j, i):
        return ((p * self.Nr + k) * self.N + j) * self.N + i

    # ---- geometry ----------------------------------------------------------
    def vertices(self, cells: torch.Tensor) -> torch.Tensor:
        """(n, 2, 2, 2, 3) vertices indexed [dk, dj, di]."""
        p, k, j, i = self.decode(cells)
        out = torch.empty(cells.numel(), 2, 2, 2, 3, dtype=DT)
        for dk in range(2):
            r = self.r[k + dk][:, None]
            for dj in range(2):
                for di in range(2):
                    out[:, dk, dj, di] = r * self.corner[p, j + dj, i + di]
        return out

    def cell_geometry(self, cells: torch.Tensor):
        """Centroid (n,3), volume (n,), face centroids and vector areas (n,6,3)."""
        v = self.vertices(cells)
        xc = v.reshape(-1, 8, 3).mean(dim=1)
        xf = torch.empty(cells.numel(), 6, 3, dtype=DT)
        S = torch.empty(cells.numel(), 6, 3, dtype=DT)
        for f, quad in enumerate(FACE_VERTS):
            q = [v[:, a, b, c] for (a, b, c) in quad]
            xf[:, f] = (q[0] + q[1] + q[2] + q[3]) / 4.0
            S[:, f] = 0.5 * torch.linalg.cross(q[2] - q[0], q[3] - q[1])
        V = (xf * S).sum(-1).sum(-1) / 3.0
        return xc, V, xf, S

    # ---- connectivity by point location ------------------------------------
    def neighbours(self, cells: torch.Tensor) -> torch.Tensor:
        """(n, 6) neighbour id per local face: a cell index, or a ghost id."""
        N, Nr = self.N, self.Nr
        xc, _, xf, S = self.cell_geometry(cells)
        nhat = S / torch.linalg.norm(S, dim=-1, keepdim=True)
        h = ((xf - xc[:, None]) * nhat).sum(-1, keepdim=True)
        # a point just across the face: the offset is tiny so that it stays in
        # the adjacent cell however thick the cells are
        y = xf + 1e-6 * h * nhat
        p, a, b = locate_panel(y)
        step = (math.pi / 2) / N
        i = torch.floor((torch.atan(a) + math.pi / 4) / step).long().clamp(0, N - 1)
        j = torch.floor((torch.atan(b) + math.pi / 4) / step).long().clamp(0, N - 1)
        # radial: the column's radial faces are the bilinear patches r_k B(s, t)
        # through its four corner directions; the ray through y meets them at
        # radii r_k |B(s*, t*)|, with (s*, t*) where B is parallel to y.
        yr = torch.linalg.norm(y, dim=-1) / self._patch_norm_along(p, j, i, y, a, b, step)
        k = torch.searchsorted(self.r, yr.contiguous()) - 1
        out = self.encode(p, k.clamp(0, Nr - 1), j, i)
        g = (p * N + j) * N + i
        out = torch.where(k < 0, self.ncells + g, out)
        out = torch.where(k >= Nr, self.ncells + self.nb + g, out)
        return out

    def _patch_norm_along(self, p, j, i, y, a, b, step, iters: int = 8):
        """|B(s, t)| at the point of the column's unit bilinear patch
        B(s, t) = (1-s)(1-t) c00 + s(1-t) c01 + (1-s)t c10 + st c11 (corner
        directions c_ji) that lies on the ray through y: Gauss-Newton on the
        component of B normal to the ray, from the angular position."""
        c00, c01 = self.corner[p, j, i], self.corner[p, j, i + 1]
        c10, c11 = self.corner[p, j + 1, i], self.corner[p, j + 1, i + 1]
        yh = y / torch.linalg.norm(y, dim=-1, keepdim=True)
        s = (torch.atan(a) + math.pi / 4) / step - i
        t = (torch.atan(b) + math.pi / 4) / step - j
        for _ in range(iters):
            B = ((1 - s) * (1 - t))[..., None] * c00 + (s * (1 - t))[..., None] * c01 \
                + ((1 - s) * t)[..., None] * c10 + (s * t)[..., None] * c11
            Bs = (1 - t)[..., None] * (c01 - c00) + t[..., None] * (c11 - c10)
            Bt = (1 - s)[..., None] * (c10 - c00) + s[..., None] * (c11 - c01)

            def perp(v):
                return v - (v * yh).sum(-1, keepdim=True) * yh
            r, Js, Jt = perp(B), perp(Bs), perp(Bt)
            # 2x2 normal equations of min |r + Js ds + Jt dt|
            a11, a12, a22 = (Js * Js).sum(-1), (Js * Jt).sum(-1), (Jt * Jt).sum(-1)
            g1, g2 = -(Js * r).sum(-1), -(Jt * r).sum(-1)
            det = a11 * a22 - a12 * a12
            s = s + (a22 * g1 - a12 * g2) / det
            t = t + (a11 * g2 - a12 * g1) / det
        B = ((1 - s) * (1 - t))[..., None] * c00 + (s * (1 - t))[..., None] * c01 \
            + ((1 - s) * t)[..., None] * c10 + (s * t)[..., None] * c11
        return torch.linalg.norm(B, dim=-1)

    def is_ghost(self, ids: torch.Tensor) -> torch.Tensor:
        return ids >= self.ncells

    def ghost_cell(self, gid: torch.Tensor):
        """Interior cell and its boundary local face for each ghost id."""
        g = gid - self.ncells
        outer = g >= self.nb
        col = torch.where(outer, g - self.nb, g)
        i = col % self.N
        j = (col // self.N) % self.N
        p = col // (self.N * self.N)
        k = torch.where(outer, torch.full_like(col, self.Nr - 1), torch.zeros_like(col))
        cell = self.encode(p, k, j, i)
        lf = torch.where(outer, torch.ones_like(col), torch.zeros_like(col))
        return cell, lf, outer, col

    def ghost_centres(self, gid: torch.Tensor) -> torch.Tensor:
        """Mirror image of the boundary cell's centroid in its boundary face."""
        cell, lf, _, _ = self.ghost_cell(gid)
        xc, _, xf, S = self.cell_geometry(cell)
        ar = torch.arange(cell.numel())
        xfb = xf[ar, lf]
        n = S[ar, lf] / torch.linalg.norm(S[ar, lf], dim=-1, keepdim=True)
        d = ((xfb - xc) * n).sum(-1, keepdim=True)
        return xc + 2.0 * d * n

    # ---- canonical face list -------------------------------------------------
    def face_list(self, chunk: int = 1 << 20):
        """Canonical faces: cells in increasing order, local faces in order;
        a face is emitted by the cell whose neighbour is a ghost or has a
        larger index.  Returns (L, R, kind) int64 tensors."""
        Ls, Rs, Ks = [], [], []
        for s in range(0, self.ncells, chunk):
            cells = torch.arange(s, min(s + chunk, self.ncells))
            nb = self.neighbours(cells)
            keep = (nb >= self.ncells) | (nb > cells[:, None])
            L = cells[:, None].expand_as(nb)[keep]
            R = nb[keep]
            kind = torch.where(R >= self.ncells + self.nb, KIND_OUTER,
                               torch.where(R >= self.ncells, KIND_INNER, KIND_INTERIOR))
            Ls.append(L)
            Rs.append(R)
            Ks.append(kind)
        return torch.cat(Ls), torch.cat(Rs), torch.cat(Ks)
