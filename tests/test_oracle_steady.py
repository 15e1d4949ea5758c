"""Pins of the oracle's march to a steady state: the CFL law of Section 4.1,
the Eq. 2 monitor on the physical quantities, the stopping rule, and that the
march drives a perturbed steady wind back toward equilibrium (CPU only)."""
import math

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import perturbed_parker
from oracle import mhd, solve
from oracle.grid import Grid

DT = torch.float64


def test_cfl_law_of_the_paper():
    # from 2, doubled every `every` steps, up to 128: six doublings
    law = [solve.cfl_law(i, 2.0, 128.0, 300) for i in (0, 299, 300, 599, 600, 1799, 1800, 2100, 10 ** 6)]
    assert law == [2.0, 2.0, 4.0, 4.0, 8.0, 64.0, 128.0, 128.0, 128.0]
    assert solve.cfl_law(5, 2.0, 1000.0, 1) == 64.0 and solve.cfl_law(9, 2.0, 1000.0, 1) == 1000.0


def test_eq2_monitor_on_primitives_by_hand():
    # two cells; the velocity is momentum over density, the pressure from the energy
    gam = 1.5
    Ua = torch.tensor([[2.0, 1.0], [4.0, 3.0], [0.0, 1.0], [2.0, 0.0], [1.0, 0.0], [0.0, 2.0], [0.0, 0.0],
                       [10.0, 8.0], [0.1, 0.0]], dtype=DT)
    Ub = Ua.clone()
    Ub[0, 0] = 4.0          # density doubles in cell 0, momentum kept: V halves
    # primitives by hand: cell 0 a: v = (2, 0, 1), p = 0.5 (10 - 0.5*2*5 - 0.5*1) = 2.25
    #                     cell 0 b: v = (1, 0, 0.5), p = 0.5 (10 - 0.5*4*1.25 - 0.5) = 3.5
    out = solve.eq2_prim(Ua, Ub, gam)
    want = [math.log10(2.0), math.log10(1.0), -math.inf, math.log10(0.5), -math.inf, -math.inf, -math.inf,
            math.log10(1.25), -math.inf]
    for a, b in zip(out.tolist(), want):
        assert a == b or a == pytest.approx(b, rel=1e-14)


def test_march_drives_perturbed_wind_toward_equilibrium():
    g, U, br = perturbed_parker()
    prm = mhd.Params(gamma=1.05, limiter=0)
    R0 = float(mhd.residual(g, U, br, prm).norm())
    Uf, hist, cfls = solve.steady(g, U, br, prm, 8, cfl0=2.0, cfl_max=128.0, every=2, m=20)
    assert cfls == [2.0, 2.0, 4.0, 4.0, 8.0, 8.0, 16.0, 16.0] and hist.shape == (8, 9)
    assert float(mhd.residual(g, Uf, br, prm).norm()) < 0.2 * R0
    # the density and pressure updates shrink as the march settles
    assert float(hist[-1, 0]) < float(hist[0, 0]) - 1.0
    assert float(hist[-1, 7]) < float(hist[0, 7]) - 0.5
    # the history is the monitor of the states the march passes through
    U1, _, _ = solve.be_step(g, U, br, prm, 2.0, 20)
    assert torch.allclose(hist[0], solve.eq2_prim(U, U1, prm.gamma), rtol=1e-12, atol=0)
    # stopping rule: with the threshold between steps 1 and 2 of the density
    # monitor, the march stops after step 2 (the first value below it)
    assert float(hist[2, 0]) < float(hist[1, 0]) < float(hist[0, 0])
    tgt = 0.5 * (float(hist[1, 0]) + float(hist[2, 0]))
    Us, hs, cs = solve.steady(g, U, br, prm, 8, cfl0=2.0, cfl_max=128.0, every=2, m=20, monitor=0, target=tgt)
    assert hs.shape == (3, 9) and torch.equal(hs, hist[:3]) and cs == cfls[:3]
