"""Jeffery orbits on the GPU (Sec. 4.7): a prolate ellipsoid in Couette shear,
FP64, through the C ABI.

  - against the oracle: 40 coupled steps of the reduced setup (a = 8, b = 4 in
    a 40 x 80 x 40 channel) hold the FP64 bars (ellipsoid voxelisation,
    momentum exchange and torque, rotation update);
  - a whole Jeffery period at the paper's Reynolds number 0.08 with 6 cells per
    minor semi-axis (a = 12, b = 6 in a 60 x 120 x 60 channel, top wall at
    0.02): the director turns by pi in T_J = pi (a^2 + b^2) / (a b gd) within
    10 %."""
import math

import numpy as np
import pytest

from tests.parity import TOL, hyd_errs, hyd_info, pop_err, vec_err
from tests.test_oracle_pins import jeffery_angle, jeffery_setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def test_jeffery_setup_matches_oracle(ps, oracle_mod):
    cfg, parts, f0, gd = jeffery_setup(oracle_mod)
    G = ps.Domain(cfg, parts)
    O = oracle_mod.OracleDomain(cfg, parts)
    for D in (G, O):
        D.set_populations(f0)
    worst = {}
    for chunk in (1, 9, 30):
        G.step(chunk)
        O.step(chunk)
        cg, pg, bg = G.solid()
        co, po, bo = O.solid()
        assert np.array_equal(cg, co) and np.array_equal(pg, po) and np.array_equal(bg, bo)
        Pg, Po = G.particles(), O.particles()
        sc = O.scales()
        e = dict(pop=pop_err(G.populations(), O.populations()), omega=vec_err(Pg["omega"], Po["omega"]),
                 quat=vec_err(Pg["quat"], Po["quat"]), **hyd_errs(Pg, Po, sc, "fp64"))
        worst = {k: max(worst.get(k, 0.0), v) for k, v in e.items()}
    print("Jeffery setup, worst errors over 40 steps:", worst, "omega_z", Po["omega"][0, 2], hyd_info(Pg, Po, sc))
    assert Po["omega"][0, 2] < 0
    assert max(worst.values()) < TOL["fp64"]


def test_jeffery_period_fp64(ps, oracle_mod):
    a, b = 12.0, 6.0
    cfg, parts, f0, gd = jeffery_setup(oracle_mod, a, b, L=120, U=0.02, tau=1.4)
    nu = (cfg["tau"] - 0.5) / 3.0
    assert abs(gd * a * a / nu - 0.08) < 1e-3
    TJ = math.pi * (a * a + b * b) / (a * b * gd)
    G = ps.Domain(cfg, parts)
    G.set_populations(f0)
    turned, last, t, every = 0.0, 0.0, 0, 250
    T = None
    while t < 1.3 * TJ:
        G.step(every)
        t += every
        th = jeffery_angle(G.particles()["quat"][0])
        d = th - last
        d -= math.pi * round(d / math.pi)     # the director: angles modulo pi
        prev, turned, last = turned, turned + d, th
        if turned >= math.pi:
            T = t - every + every * (math.pi - prev) / (turned - prev)
            break
    print(f"Jeffery period: measured {T}, theory {TJ:.0f} steps")
    assert T is not None and abs(T - TJ) / TJ < 0.10
