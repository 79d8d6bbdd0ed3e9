"""State handling on the GPU through the C ABI: checkpoint and restore, the
device flags (unstable, capacity), and cell lists of blown-up states.

  - n steps, a checkpoint, n more steps equal 2n steps bit for bit (populations,
    particle state, pair lists and history, solid slots), on the single-
    workgroup DEM path with the fluid coupled and on the multi-launch DEM path;
  - a host-forced blow-up (tau -> 1/2 with large random velocities) raises
    PSMDEM_E_UNSTABLE at the next sync; reads still return their outputs and
    the flag; rewriting the state clears it;
  - a pair list beyond its capacity surfaces PSMDEM_E_CAPACITY from every read;
  - k_n = 1e3 at dt = 1/2 is an unstable integration whose positions reach
    1e15 within 8 steps: the cell lists of such positions follow the
    definition on both sides (no integer overflow), step by step and from the
    same positions."""
import numpy as np
import pytest

from paper_2512_04997_amd import workloads as W
from tests.parity import linear_shear_populations, pop_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def _snapshot(D):
    P = D.particles() if D.np else {}
    k, h = D.pairs() if D.np else (np.zeros(0, np.uint64), np.zeros((0, 3)))
    c, p, b = D.solid()
    return dict(f=D.populations(), k=k, h=h, c=c, p=p, b=b, **{"P_" + n: v for n, v in P.items()})


def _assert_same(a, b):
    assert a.keys() == b.keys()
    for n in a:
        assert np.array_equal(a[n], b[n]), n


def _couette(ps_, oracle_mod, prec):
    cfg, parts, _ = W.couette_suspension(precision=prec, n=48, nsph=30, radius=4.0)
    cfg["mu"] = 0.3
    f0 = linear_shear_populations(oracle_mod, cfg["n"], 0, 2, cfg["wall_u"][4][0], cfg["wall_u"][5][0])
    return cfg, parts, f0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_checkpoint_n_plus_n_equals_2n(ps, oracle_mod, prec):
    """Coupled Couette suspension (single-workgroup DEM with kept lists and
    saved skip state, in-place populations of both parities): the restored
    domain, which had stepped on its own before, continues bit for bit."""
    cfg, parts, f0 = _couette(ps, oracle_mod, prec)
    A = ps.Domain(cfg, parts)
    A.set_populations(f0)
    A.step(7)
    img = A.state()
    A.step(7)
    B = ps.Domain(cfg, parts)
    B.step(3)
    B.set_state(img)
    B.step(7)
    assert A.info()["n_sub"] > 1 and A.counters()["n_contacts"] >= 0
    _assert_same(_snapshot(A), _snapshot(B))
    assert A.counters()["step"] == B.counters()["step"] == 14
    A.close()
    B.close()


def test_checkpoint_multi_launch_dem(ps):
    """More particles than one workgroup takes (DEM only, walls, contacts):
    the per-substep list flags and buffers are part of the image."""
    box = (72, 64, 60)
    rng = W.SplitMix64(91)
    radii = 1.2 + 0.6 * rng.uniform(2300)
    pos = W.rsa_spheres(rng, 2300, radii, box, [True, True, False], gap=-0.4)
    m = len(pos)
    assert m > 2048
    vel = 0.01 * (rng.uniform(3 * m).reshape(m, 3) - 0.5)
    cfg = W.base_config(box, 0.7, bc=["periodic"] * 4 + ["noslip"] * 2, fluid_on=False, mu=0.3,
                        restitution=0.7, n_sub=5, gravity=[0.0, 0.0, -2e-4])
    parts = W.spheres(pos, radii[:m], 1.6, vel=vel)
    A = ps.Domain(cfg, parts)
    A.step(3)
    img = A.state()
    A.step(3)
    B = ps.Domain(cfg, parts)
    B.set_state(img)
    B.step(3)
    _assert_same(_snapshot(A), _snapshot(B))
    assert A.counters()["n_contacts"] > 100


def test_state_of_another_layout_is_refused(ps):
    a = ps.Domain(W.base_config((32, 16, 16), 0.7, precision="fp32"))
    b = ps.Domain(W.base_config((32, 16, 20), 0.7, precision="fp32"))
    img = a.state()
    with pytest.raises(ps.PsmdemError) as e:
        b.set_state(img)
    assert e.value.code == ps.E_INVALID
    with pytest.raises(ps.PsmdemError):
        a.set_state(img[:-1])
    a.set_state(img)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unstable_flag_raised_and_cleared(ps, oracle_mod, prec):
    """tau = 0.5001 with random velocities of amplitude 0.35 (fluid only):
    the density turns negative within tens of steps (the FP64 oracle: step 43).
    The flag appears at a sync, reads return their data with it, and writing
    populations clears it."""
    n = (16, 16, 16)
    cfg = W.base_config(n, 0.5001, precision=prec)
    rng = np.random.default_rng(1)
    N = n[0] * n[1] * n[2]
    f0 = np.zeros((19, N))
    for c in range(N):
        f0[:, c] = oracle_mod.feq(1.0, 0.35 * (rng.random(3) - 0.5))
    G = ps.Domain(cfg, strict=False)
    G.set_populations(f0)
    assert G.sync() == ps.OK
    flagged = None
    for s in range(1, 31):
        G.step(10)
        if G.sync() == ps.E_UNSTABLE:
            flagged = 10 * s
            break
    print(f"{prec}: unstable flagged after {flagged} steps")
    assert flagged is not None and flagged <= 300
    assert G.counters()["flags"] & 16
    rho, _ = G.fields()
    assert G.flag == ps.E_UNSTABLE
    assert np.any(~(rho > 0) | ~np.isfinite(rho))
    G.set_populations(f0)
    assert G.sync() == ps.OK
    G.strict = True
    G.step(1)
    G.populations()


def test_capacity_overflow_surfaces_from_reads(ps):
    """A pair capacity far below the candidate pairs: every read reports
    PSMDEM_E_CAPACITY (the lists are truncated, the step's results invalid)."""
    box = (48, 40, 36)
    rng = W.SplitMix64(4545)
    radii = 1.4 + 0.6 * rng.uniform(300)
    pos = W.rsa_spheres(rng, 300, radii, box, [True, True, False], gap=-0.5)
    m = len(pos)
    cfg = W.base_config(box, 0.7, bc=["periodic"] * 4 + ["noslip"] * 2, fluid_on=False, n_sub=3,
                        pair_capacity=64)
    G = ps.Domain(cfg, W.spheres(pos, radii[:m], 1.6))
    G.step(1)
    for read in (G.pairs, G.particles, G.cells, G.contacts, G.solid, G.populations):
        with pytest.raises(ps.PsmdemError) as e:
            read()
        assert e.value.code == ps.E_CAPACITY
    assert G.counters()["n_pairs"] > 64 and G.counters()["flags"] & 1
    G.strict = False
    k, _ = G.pairs()
    assert G.flag == ps.E_CAPACITY and len(k) > 64 and np.all(np.diff(k[:64].astype(np.int64)) > 0)


def _blowup_case():
    box = (48, 40, 36)
    rng = W.SplitMix64(4646)
    n = 350
    radii = 1.4 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=0.03)
    m = len(pos)
    vel = 0.006 * (rng.uniform(3 * m).reshape(m, 3) - 0.5)
    parts = W.spheres(pos, radii[:m], 1.6, vel=vel)
    bc = ["periodic", "periodic", "noslip", "noslip", "moving", "moving"]
    wu = [[0.0] * 3 for _ in range(6)]
    wu[4] = [-0.02, 0.01, 0.0]
    wu[5] = [0.02, 0.0, -0.005]
    cfg = W.base_config(box, 0.7, bc=bc, wall_u=wu, precision="fp64", fluid_on=False, mu=0.3, restitution=0.7,
                        n_sub=2, gravity=[0.0, 0.0, -2e-4], kn=1e3)
    return cfg, parts


def test_blown_up_positions_cells_from_the_same_positions(ps, oracle_mod):
    """Seed 4646, 350 spheres, v = 0.006, k_n = 1e3, n_sub = 2: after each of 8
    oracle steps its positions (up to 5e14) go to the GPU, and the GPU's cell
    registrations and candidate pairs for them equal the oracle's bit for bit."""
    cfg, parts = _blowup_case()
    O = oracle_mod.OracleDomain(cfg, parts)
    G = ps.Domain(cfg, parts, strict=False)
    biggest = 0.0
    for step in range(8):
        O.step(1)
        P = O.particles()
        biggest = max(biggest, np.abs(P["pos"]).max())
        G.set_particles(pos=P["pos"], quat=P["quat"], vel=P["vel"], omega=P["omega"])
        G.stage("lists")
        O.stage_lists()
        assert np.array_equal(G.cells(), O.cells()), step
        assert np.array_equal(G.pairs()[0], O.pairs()[0]), step
    assert biggest > 1e13


def test_blown_up_case_steps(ps, oracle_mod):
    """The same case stepped on both sides (the single-workgroup DEM keeps and
    rebuilds its lists across launches): positions stay bit for bit equal while
    they blow up, the pair lists equal the oracle's at every step, and the
    device flags the state as unstable."""
    cfg, parts = _blowup_case()
    O = oracle_mod.OracleDomain(cfg, parts)
    G = ps.Domain(cfg, parts, strict=False)
    for step in range(8):
        G.step(1)
        O.step(1)
        Pg, Po = G.particles(), O.particles()
        assert np.array_equal(Pg["pos"], Po["pos"]), step
        assert np.array_equal(G.pairs()[0], O.pairs()[0]), step
    assert np.abs(Po["pos"]).max() > 1e13
    assert G.sync() == ps.E_UNSTABLE
