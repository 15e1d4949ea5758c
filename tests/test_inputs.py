"""Checks of the seeded input generator (CPU only)."""
import math

import numpy as np

import coronal_inputs as ci


def test_real_harmonics_match_scipy_and_are_orthonormal():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(0)
    th = np.arccos(rng.uniform(-1, 1, 200))
    ph = rng.uniform(0, 2 * math.pi, 200)
    Y = ci.real_harmonics(4, th, ph)
    k = 0
    for l in range(1, 5):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), th, ph)
            ref = y.real if m == 0 else math.sqrt(2) * (-1) ** m * (y.real if m > 0 else y.imag)
            assert np.allclose(Y[k], ref, rtol=1e-12, atol=1e-12)
            k += 1


def test_parker_wind_is_transonic_and_conserves_mass():
    r = np.geomspace(1.0, 21.5, 200)
    v, rho = ci.parker_isothermal(r)
    cs = math.sqrt(ci.T_WIND)
    rc = ci.G_GRAV / (2 * ci.T_WIND)
    assert np.all(np.diff(v) > 0)
    assert np.all((v < cs) == (r < rc))
    assert np.allclose(rho * v * r * r, rho[0] * v[0] * r[0] ** 2, rtol=1e-12)
    u2 = (v / cs) ** 2
    assert np.allclose(u2 - np.log(u2), 4 * np.log(r / rc) + 4 * rc / r - 3, rtol=1e-9, atol=1e-9)


def test_br_map_peak_and_seeding():
    b1 = ci.br_map(12, 5, 42)
    b2 = ci.br_map(12, 5, 42)
    assert np.array_equal(b1, b2)
    assert abs(np.max(np.abs(b1)) - 5.0 * ci.GAUSS) < 1e-9
    dip = ci.br_map(12, 0, 42)
    assert abs(np.max(dip) - 2.0 * ci.GAUSS) < 0.05 * ci.GAUSS


def test_workload_shapes():
    inst = ci.workload("tiny")
    assert inst.U.shape == (9, 6144) and inst.br.shape == (384,)
    assert abs(inst.r_nodes[1] - inst.r_nodes[0] - 0.2344408) < 1e-6
    specs = ci.ensemble_specs()
    assert len(specs) == 64 and sum(6 * N * N * Nr for N, Nr, _ in specs) == 29952000


def test_bc_independent_radii():
    r = ci.radial_nodes(40, "bcind", edge=0.01)
    assert r.shape == (41,) and r[0] == 1.0 and r[-1] == 25.0
    assert np.all(np.diff(r) > 0)
    assert abs((r[-1] - r[-2]) - 0.01) < 1e-12
    # log spacing below the thin edge layer, and 21.5 inside the domain
    q = np.diff(np.log(r[:-1]))
    assert np.allclose(q, q[0], rtol=1e-10) and r[-2] > 21.5
