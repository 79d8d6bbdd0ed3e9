"""Parity horizon of a contact-rich coupled case, FP64, measured and reported
(not required: once particles collide, contact onset is decided by the last
bits of positions and the two trajectories part).

The Couette flow of the secondary workload (moving walls at -/+0.02, tau = 0.7,
linear spring-dashpot k_n = 1e3, restitution 0.8, mu = 0.3, density ratio 1.5)
at 48^3 with 250 spheres of radius 3 (solid fraction 0.26) placed with
overlaps of up to 0.3 and random initial velocities of up to 0.01 per
component, so that pairs are in contact from the first step on.  GPU and
oracle start from the same description and step one coupled step at a time;
positions and velocities (velocity floor 0.02, the wall speed) are compared
every step and populations every 25 steps.  Reported: the step of the first
contact, the first step past the FP64 bar (1e-12) and the first past 1e-6.
What holds: the two agree to the FP64 bar at least until the first contact."""
import numpy as np
import pytest

from paper_2512_04997_amd import workloads as W
from tests.parity import TOL, pop_err, vec_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def test_contact_rich_parity_horizon(ps, oracle_mod):
    n = 48
    cfg, _, _ = W.couette_suspension(precision="fp64", n=n, nsph=1)
    pos = W.rsa_spheres(W.SplitMix64(77), 250, np.full(250, 3.0), (n, n, n), [True, True, False], gap=-0.3)
    vel = 0.01 * (2.0 * np.random.default_rng(5).random((len(pos), 3)) - 1.0)
    parts = W.spheres(pos, 3.0, 1.5, vel=vel)
    G = ps.Domain(cfg, parts)
    O = oracle_mod.OracleDomain(cfg, parts)
    first_contact = horizon = h6 = None
    worst = 0.0
    steps = 200
    for s in range(1, steps + 1):
        G.step(1)
        O.step(1)
        Pg, Po = G.particles(), O.particles()
        e = max(vec_err(Pg["pos"], Po["pos"]), vec_err(Pg["vel"], Po["vel"], floor=0.02))
        if s % 25 == 0:
            e = max(e, pop_err(G.populations(), O.populations()))
        if first_contact is None and O.counters()["contacts"] > 0:
            first_contact = s
        if horizon is None and e > TOL["fp64"]:
            horizon = s
        else:
            worst = max(worst, e) if horizon is None else worst
        if h6 is None and e > 1e-6:
            h6 = s
            break
    print(f"contact-rich Couette 48^3, {len(pos)} spheres, FP64: first contact at step {first_contact}, "
          f"past 1e-12 at step {horizon}, past 1e-6 at step {h6} (of {steps}); "
          f"worst error while within the bar {worst:.2e}")
    assert first_contact is not None, "the case must be contact-rich"
    assert horizon is None or horizon >= first_contact
