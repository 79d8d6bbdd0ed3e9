"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Integer outputs (cell registrations, candidate
pairs, solid-fraction slots) must match bit for bit; floating outputs within
1e-12 (FP64) and 1e-5 (FP32) in the norms of the parity protocol."""
import numpy as np
import pytest

from paper_2512_04997_amd import workloads as W
from tests.parity import (TOL, bar_values, copy_state, force_err, hyd_errs, hyd_info, linear_shear_populations,
                          one_step_errors, pop_err, vec_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    from paper_2512_04997_amd import psmdem
    psmdem.lib()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return psmdem


def _pair(ps, oracle_mod, cfg, parts):
    return ps.Domain(cfg, parts), oracle_mod.OracleDomain(cfg, parts)


def _random_pops(N, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    u = amp * (rng.random((N, 3)) - 0.5)
    rho = 1.0 + 0.05 * (rng.random(N) - 0.5)
    CI = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, -1, 0], [1, 0, 1],
                   [1, 0, -1], [0, 1, 1], [0, 1, -1]])
    CI = np.concatenate([CI, -CI[1:]])
    w = np.array([1 / 3] + [1 / 18] * 3 + [1 / 36] * 6 + [1 / 18] * 3 + [1 / 36] * 6)
    cu = u @ CI.T
    feq = w[None, :] * rho[:, None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u ** 2).sum(1)[:, None])
    f = feq * (1 + 0.01 * (rng.random(feq.shape) - 0.5))
    return f.T.copy()


def _walled(n, tau, prec, **kw):
    bc = ["periodic", "periodic", "noslip", "noslip", "moving", "moving"]
    wu = [[0.0] * 3 for _ in range(6)]
    wu[4] = [-0.02, 0.01, 0.0]
    wu[5] = [0.02, 0.0, -0.005]
    return W.base_config(n, tau, bc=bc, wall_u=wu, precision=prec, **kw)


# --------------------------------------------------------------------------- LBM only
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["periodic", "walls_forcing", "walls_every_face", "trt_walls_forcing",
                                  "trt_magic_every_face"])
def test_lbm_matches_oracle(ps, oracle_mod, prec, kind):
    """Ragged lattice (tiles of 64x4x4 cut in every axis), random near-equilibrium
    populations; several steps cover both in-place parities.  The TRT cases take
    the paper's tau- rule and a free magic parameter."""
    n = (70, 9, 6)
    if kind == "periodic":
        cfg = W.base_config(n, 0.63, precision=prec)
    elif kind in ("walls_forcing", "trt_walls_forcing"):
        cfg = _walled(n, 0.81, prec, body_force=[1e-5, -2e-6, 0.0], kolm_amp=3e-6, kolm_axis=2, kolm_dir=1,
                      collision="trt" if kind.startswith("trt") else "bgk")
    elif kind == "trt_magic_every_face":
        wu = [[0.0] * 3 for _ in range(6)]
        wu[1] = [0.0, 0.01, 0.02]
        wu[4] = [0.015, 0.0, 0.0]
        cfg = W.base_config(n, 0.57, precision=prec, bc=["noslip", "moving", "noslip", "noslip", "moving", "noslip"],
                            wall_u=wu, body_force=[2e-6, 0.0, -3e-6], collision="trt", trt_magic=0.07)
    else:
        wu = [[0.0] * 3 for _ in range(6)]
        wu[0] = [0.0, 0.015, -0.01]
        wu[1] = [0.0, -0.02, 0.0]
        wu[5] = [0.01, 0.0, 0.0]
        cfg = W.base_config(n, 0.74, precision=prec, bc=["moving", "moving", "noslip", "noslip", "noslip", "moving"],
                            wall_u=wu, body_force=[0.0, 3e-6, 0.0])
    G, O = _pair(ps, oracle_mod, cfg, None)
    f0 = _random_pops(G.N, 11)
    G.set_populations(f0)
    O.set_populations(f0)
    for steps in (1, 2, 3):
        G.step(1)
        O.step(1)
        e = pop_err(G.populations(), O.populations())
        assert e < TOL[prec], (steps, e)
    rg, ug = G.fields()
    ro, uo = O.fields()
    assert vec_err(ug, uo) < 10 * TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lbm_low_precision_storage_error_is_stated(ps, oracle_mod, prec):
    """Shifted 16-bit storage with FP32 arithmetic: error stated, loose bound."""
    cfg = _walled((70, 9, 6), 0.81, prec, body_force=[1e-5, 0, 0])
    G, O = _pair(ps, oracle_mod, cfg, None)
    f0 = _random_pops(G.N, 12)
    G.set_populations(f0)
    O.set_populations(f0)
    G.step(4)
    O.step(4)
    e = pop_err(G.populations(), O.populations())
    print(f"{prec} population error after 4 steps: {e:.3e}")
    assert e < (1e-3 if prec == "bf16" else 1e-4)


# --------------------------------------------------------------------------- stages
def _mixed_particles(seed, n, box, periodic, ell_frac=0.5, gap=0.3):
    rng = W.SplitMix64(seed)
    radii = 2.0 + 2.0 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii * 1.6, box, periodic, gap=gap)
    m = len(pos)
    shape = (rng.uniform(m) < ell_frac).astype(np.int32)
    semi = np.stack([radii[:m] * 1.6, radii[:m], radii[:m] * 0.8], 1)
    semi[shape == 0] = (radii[:m] * 1.2)[shape == 0, None]
    return dict(shape=shape, semi=semi, dens=1.3 + rng.uniform(m), pos=pos,
                quat=W.shoemake_quaternions(rng, m),
                vel=0.01 * (rng.uniform(3 * m).reshape(m, 3) - 0.5),
                omega=0.002 * (rng.uniform(3 * m).reshape(m, 3) - 0.5), fixed=np.zeros(m, np.uint8))


def _fcc_cluster(lo, hi, d):
    """Face-centred cubic points with nearest distance d inside the box lo..hi."""
    a = d * np.sqrt(2.0)
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    n = [int((hi[c] - lo[c]) / a) + 1 for c in range(3)]
    pts = [np.array(lo) + np.array([i, j, k]) * a + b
           for i in range(n[0]) for j in range(n[1]) for k in range(n[2]) for b in base]
    return np.array([p for p in pts if np.all(p <= np.array(hi))])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ms", [2, 4])
def test_coupled_steps_three_solids_per_cell(ps, oracle_mod, ms, prec):
    """A face-centred cluster of 70 spheres (R = 3, nearest centres 6.05
    apart) with the distance solid fraction: cells near the triangle centroids
    see three solids.  Four slots run the four-slot LBM-PSM kernels and keep
    all three; two slots drop the smallest.  Two coupled steps against the
    FP64 oracle."""
    box = (48, 40, 36)
    pos = _fcc_cluster((10.3, 9.7, 9.1), (37.0, 30.0, 26.0), 6.05)
    rng = np.random.default_rng(17)
    m = len(pos)
    parts = W.spheres(pos, 3.0, 1.5, vel=0.004 * (rng.random((m, 3)) - 0.5),
                      omega=0.001 * (rng.random((m, 3)) - 0.5))
    # the fluid is driven too, so every three-solid cell carries a real exchange
    cfg = W.base_config(box, 0.7, max_solids=ms, n_sub=4, precision=prec, sf_method="distance",
                        body_force=[2e-6, -1e-6, 0.5e-6], kn=50.0)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(6):
        G.step(1)
        O.step(1)
    cg, pg, bg = G.solid()
    co, po, bo = O.solid()
    assert np.array_equal(cg, co) and np.array_equal(pg, po)
    # beta follows the positions: an FP64 trajectory holds them to round-off,
    # an FP32 one (FP32 populations drive the particles) to the FP32 bar
    assert np.abs(bg - bo).max() < TOL[prec]
    u, cnt = np.unique(co, return_counts=True)
    if ms == 4:
        assert (cnt >= 3).sum() > 10
    else:
        assert G.counters()["n_dropped"] > 0
    Pg, Po = G.particles(), O.particles()
    sc = O.scales()
    assert np.abs(Po["f_hyd"]).min(axis=1).min() > 0 and np.abs(Po["m_hyd"]).max() > 0
    traj = dict(pop=pop_err(G.populations(), O.populations()), vel=vec_err(Pg["vel"], Po["vel"]),
                omega=vec_err(Pg["omega"], Po["omega"]), **hyd_errs(Pg, Po, sc, prec))
    print(f"three solids per cell ({ms} slots, {prec}), trajectory of 6 steps:", traj, hyd_info(Pg, Po, sc))
    if prec == "fp64":
        assert max(traj.values()) < TOL[prec]
    e = one_step_errors(G, O, prec)
    print(f"three solids per cell ({ms} slots, {prec}), one step from the oracle's state:", e)
    assert max(bar_values(e)) < TOL[prec]
    G.close()


@pytest.mark.parametrize("method", ["subdivision", "distance"])
def test_voxelize_bitexact_many_tiles(ps, oracle_mod, method):
    """A lattice of 8320 tiles (64 x 256 x 520), beyond the size whose tile
    lists are ordered inside the per-tile voxelisation kernels: the lists are
    ordered by their own kernel there.  Kept slots bit for bit."""
    box = (64, 256, 520)
    parts = _mixed_particles(131, 200, box, [True, True, True], ell_frac=0.0 if method == "distance" else 0.5)
    cfg = W.base_config(box, 0.7, sf_method=method, max_solids=2)
    assert (box[0] // 64) * (box[1] // 4) * (box[2] // 4) > 8192
    G, O = _pair(ps, oracle_mod, cfg, parts)
    G.stage("voxelize")
    O.stage_voxelize()
    cg, pg, bg = G.solid()
    co, po, bo = O.solid()
    assert len(co) > 50000
    assert np.array_equal(cg, co) and np.array_equal(pg, po)
    if method == "subdivision":
        assert np.array_equal(bg, bo)
    else:
        assert np.max(np.abs(bg - bo)) < 1e-14
    G.close()


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("method", ["subdivision", "distance"])
def test_voxelize_bitexact(ps, oracle_mod, walls, method):
    box = (72, 36, 32)
    periodic = [True, True, not walls]
    parts = _mixed_particles(101 + walls, 40, box, periodic, ell_frac=0.0 if method == "distance" else 0.5)
    if walls:
        cfg = _walled(box, 0.7, "fp64", sf_method=method, max_solids=2)
    else:
        cfg = W.base_config(box, 0.7, sf_method=method, max_solids=2)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    G.stage("voxelize")
    O.stage_voxelize()
    cg, pg, bg = G.solid()
    co, po, bo = O.solid()
    assert len(co) > 1000
    assert np.array_equal(cg, co) and np.array_equal(pg, po)
    if method == "subdivision":
        assert np.array_equal(bg, bo)
    else:
        assert np.max(np.abs(bg - bo)) < 1e-14
    assert G.counters()["n_dropped"] == O.counters()["overflow"]


@pytest.mark.parametrize("walls", [False, True])
def test_dem_lists_bitexact(ps, oracle_mod, walls):
    box = (72, 60, 52)
    periodic = [True, True, not walls]
    parts = _mixed_particles(201 + walls, 120, box, periodic, gap=-1.0)
    cfg = _walled(box, 0.7, "fp64", fluid_on=False) if walls else W.base_config(box, 0.7, fluid_on=False)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    G.stage("lists")
    O.stage_lists()
    assert np.array_equal(G.cells(), O.cells())
    kg, _ = G.pairs()
    ko, _ = O.pairs()
    assert len(ko) > 50
    assert np.array_equal(kg, ko)
    assert np.array_equal(ko, O.brute_pairs())


@pytest.mark.parametrize("law", ["linear", "hertz"])
def test_contacts_match(ps, oracle_mod, law):
    """Overlapping spheres and ellipsoids with walls: contact forces, torques and
    history from a shared state (pairs and history written to both), with the
    linear law and with the Hertz law from the material."""
    box = (64, 48, 40)
    parts = _mixed_particles(301, 90, box, [True, True, False], gap=-3.5)
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.7, n_sub=8, contact_law=law,
                  young=800.0, poisson=0.3)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    O.stage_lists()
    k, _ = O.pairs()
    rng = np.random.default_rng(3)
    hist = 0.05 * (rng.random((len(k), 3)) - 0.5)
    for D in (G, O):
        D.set_pairs(k, hist)
    vp = parts["vel"] * 1.1
    wp = parts["omega"] * 0.9
    G.set_predicted(vp, wp)
    O.set_predicted(vp, wp)
    G.stage("contacts")
    O.stage_contacts()
    kc, Fg, mig, mjg = G.contacts()
    ko, Fo, mio, mjo = O.contacts()
    assert len(ko) > 20
    assert np.array_equal(kc, ko)
    assert np.abs(Fg - Fo).max() <= 1e-12 * np.abs(Fo).max()
    assert np.abs(mig - mio).max() <= 1e-12 * np.abs(mio).max()
    assert np.abs(mjg - mjo).max() <= 1e-12 * np.abs(mjo).max()
    _, hg = G.pairs()
    _, ho = O.pairs()
    assert np.abs(hg - ho).max() <= 1e-12 * max(np.abs(ho).max(), 1e-12)


# --------------------------------------------------------------------------- coupled
def test_settling_sphere_trajectory_fp64(ps, oracle_mod):
    """Plain method, FP64: 32^3 periodic, tau = 0.8, one sphere R = 4 settling
    with density ratio 2 under gravity 1e-5, 200 steps; the whole trajectory
    holds the FP64 bar."""
    cfg, parts, meta = W.settling_sphere()
    G, O = _pair(ps, oracle_mod, cfg, parts)
    worst = {"pop": 0.0, "pos": 0.0, "f": 0.0}
    dv, vmax = 0.0, 0.0
    for chunk in (1, 1, 8, 40, 150):
        G.step(chunk)
        O.step(chunk)
        worst["pop"] = max(worst["pop"], pop_err(G.populations(), O.populations()))
        Pg, Po = G.particles(), O.particles()
        worst["pos"] = max(worst["pos"], vec_err(Pg["pos"], Po["pos"]))
        dv = max(dv, float(np.abs(Pg["vel"] - Po["vel"]).max()))
        vmax = max(vmax, float(np.abs(Po["vel"]).max()))
        sc = O.scales()
        worst["f"] = max(worst["f"], *hyd_errs(Pg, Po, sc, "fp64").values())
    # velocities against the case's own velocity scale: the largest speed of the run
    worst["vel"] = dv / vmax
    print("settling sphere worst errors over 200 steps:", worst, "largest speed %.3e" % vmax,
          hyd_info(Pg, Po, sc))
    assert max(worst.values()) < TOL["fp64"]
    assert O.counters()["step"] == 200


@pytest.mark.parametrize("collision", ["bgk", "trt"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_couette_suspension_steps(ps, oracle_mod, prec, collision):
    """Bounded Couette shear with spheres (48^3, moving walls, contacts and wall
    contacts): three coupled steps from creation, with the BGK or the TRT
    fluid operator inside the PSM collision."""
    cfg, parts, _ = W.couette_suspension(precision=prec, n=48, nsph=30, radius=4.0)
    cfg["mu"] = 0.3
    cfg["collision"] = collision
    G, O = _pair(ps, oracle_mod, cfg, parts)
    assert G.n_sub == O.n_sub
    # the fluid starts on the Couette profile of the walls, so every particle
    # is sheared (and pushed into contacts) from the first step
    f0 = linear_shear_populations(oracle_mod, cfg["n"], 0, 2, cfg["wall_u"][4][0], cfg["wall_u"][5][0])
    G.set_populations(f0)
    O.set_populations(f0)
    worst = {}
    for chunk in (1, 1, 48, 50):
        G.step(chunk)
        O.step(chunk)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        cg, pg, bg = G.solid()
        co, po, bo = O.solid()
        assert np.array_equal(cg, co) and np.array_equal(pg, po)
        Pg, Po = G.particles(), O.particles()
        sc = O.scales()
        e = dict(pop=pop_err(G.populations(), O.populations()), pos=vec_err(Pg["pos"], Po["pos"]),
                 vel=vec_err(Pg["vel"], Po["vel"]), omega=vec_err(Pg["omega"], Po["omega"]),
                 f_dem=force_err(Pg["f_dem"], Po["f_dem"], sc["f_dem"]), **hyd_errs(Pg, Po, sc, prec))
        worst = {k: max(worst.get(k, 0.0), v) for k, v in e.items()}
    print(f"Couette {prec} {collision}, worst errors over 100 steps:", worst, hyd_info(Pg, Po, sc),
          "max |v| %.2e, contacts %d" % (np.abs(Po["vel"]).max(), O.counters()["contacts"]))
    assert np.abs(Po["vel"]).max() > 1e-3
    if prec == "fp64":
        assert max(worst.values()) < TOL[prec]
    else:
        # the FP32 trajectory's state stays within the bar over 100 steps; its
        # forces are compared from the oracle's state below (they follow the
        # diverged state, not the rounding of one step)
        assert max(worst[k] for k in ("pop", "pos", "vel", "omega")) < TOL[prec]
    e = one_step_errors(G, O, prec)
    print(f"Couette {prec} {collision}, one step from the oracle's state at step 100:", e)
    assert max(bar_values(e)) < TOL[prec]


def test_determinism_bitwise(ps):
    """No floating-point atomics: two runs are bitwise identical."""
    cfg, parts, _ = W.couette_suspension(precision="fp32", n=48, nsph=30, radius=4.0)
    out = []
    for _ in range(2):
        G = ps.Domain(cfg, parts)
        G.step(4)
        P = G.particles()
        out.append((G.populations(), P["pos"], P["f_hyd"], P["m_hyd"]))
        G.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_dem_multi_launch_path(ps, oracle_mod):
    """More particles than one workgroup takes: the per-phase kernels with the
    counting-sort cell list (DEM only, walls, friction, contacts)."""
    box = (72, 64, 60)
    rng = W.SplitMix64(77)
    n = 2300
    radii = 1.2 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=-0.4)
    m = len(pos)
    assert m > 2048
    parts = W.spheres(pos, radii[:m], 1.8, vel=0.01 * (rng.uniform(3 * m).reshape(m, 3) - 0.5))
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.6, n_sub=6,
                  gravity=[0.0, 0.0, -1e-4])
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(2):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12
        assert force_err(Pg["f_dem"], Po["f_dem"], O.scales()["f_dem"]) < 1e-12
    assert O.counters()["contacts"] > 50


def test_dem_multi_launch_contacts_form_and_break(ps, oracle_mod):
    """Multi-launch DEM over 48 substeps in which pairs come into contact and
    leave it again while the list is kept: a pair out of contact at its last
    two evaluations writes nothing (its zero outputs and history are already
    in place), so the contact set, forces and trajectory after each step must
    still equal the oracle's, and some pairs must re-enter contact."""
    box = (72, 64, 60)
    rng = W.SplitMix64(91)
    n = 2300
    radii = 1.2 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=0.15)
    m = len(pos)
    assert m > 2048
    parts = W.spheres(pos, radii[:m], 1.8, vel=0.03 * (rng.uniform(3 * m).reshape(m, 3) - 0.5),
                      omega=0.02 * (rng.uniform(3 * m).reshape(m, 3) - 0.5))
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.6, n_sub=6,
                  gravity=[0.0, 0.0, -1e-4])
    G, O = _pair(ps, oracle_mod, cfg, parts)
    seen, left, reentered = set(), 0, 0
    prev = set()
    for step in range(8):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        kg, Fg, _, _ = G.contacts()
        ko, Fo, _, _ = O.contacts()
        assert np.array_equal(kg, ko)
        sc = O.scales()
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12, step
        assert force_err(Pg["f_dem"], Po["f_dem"], sc["f_dem"]) < 1e-12, step
        if len(ko):
            assert np.abs(Fg - Fo).max() <= 1e-12 * max(1.0, float(np.abs(Fo).max()))
        now = set(int(k) for k in ko)
        left += len(prev - now)
        reentered += len((now - prev) & seen)
        seen |= now
        prev = now
    print(f"multi-launch contacts: {len(seen)} pairs touched, {left} separations, {reentered} re-entries")
    assert left > 0 and len(seen) > 50


@pytest.mark.parametrize("kind", ["fast", "dense_slow"])
def test_fused_dem_list_reuse(ps, oracle_mod, kind):
    """The single-workgroup DEM keeps the pair list while no particle changes
    its cells or wall candidates.  'fast': particles cross cells within a
    launch, so rebuilt and kept lists alternate; 'dense_slow': overlapping,
    slowly moving spheres keep their list for many substeps with contacts,
    friction and wall contacts, so the history is carried at the kept index."""
    box = (48, 40, 36)
    rng = W.SplitMix64(4242 if kind == "fast" else 4343)
    n = 400
    radii = 1.4 + 0.6 * rng.uniform(n)
    gap = 0.2 if kind == "fast" else -0.6
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=gap)
    m = len(pos)
    amp = 0.05 if kind == "fast" else 0.004
    vel = amp * (rng.uniform(3 * m).reshape(m, 3) - 0.5)
    parts = W.spheres(pos, radii[:m], 1.6, vel=vel)
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.7, n_sub=9,
                  gravity=[0.0, 0.0, -2e-4])
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(4):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12
        assert force_err(Pg["f_dem"], Po["f_dem"], O.scales()["f_dem"]) < 1e-12
    if kind == "dense_slow":
        assert O.counters()["contacts"] > 20


def test_fused_dem_skip_state_across_launches(ps, oracle_mod):
    """Two substeps per launch: a kept list's quiet pairs are skipped from the
    first substep of a launch only through the state the previous launch
    saved.  Slow, nearly touching spheres keep their lists while contacts
    form and break, so a wrongly skipped pair would show in the forces (a soft
    spring, k_n = 10, keeps the contact resolved at dt = 1/2)."""
    box = (48, 40, 36)
    rng = W.SplitMix64(4646)
    n = 350
    radii = 1.4 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=0.03)
    m = len(pos)
    vel = 0.01 * (rng.uniform(3 * m).reshape(m, 3) - 0.5)
    parts = W.spheres(pos, radii[:m], 1.6, vel=vel)
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.7, n_sub=2,
                  gravity=[0.0, 0.0, -2e-4], kn=10.0)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    contacts, lengths = 0, set()
    for _ in range(12):
        G.step(1)
        O.step(1)
        pg = G.pairs()[0]
        assert np.array_equal(pg, O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12
        assert force_err(Pg["f_dem"], Po["f_dem"], O.scales()["f_dem"]) < 1e-12
        contacts += O.counters()["contacts"]
        lengths.add(len(pg))
    assert contacts > 60 and len(lengths) > 3


def test_fused_dem_state_written_between_steps(ps, oracle_mod):
    """A list kept across launches is dropped when the host writes particles
    or pairs: both sides take the same moved positions and scaled history
    after two steps and must agree again after three more."""
    box = (48, 40, 36)
    rng = W.SplitMix64(4545)
    n = 300
    radii = 1.4 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=-0.5)
    m = len(pos)
    vel = 0.004 * (rng.uniform(3 * m).reshape(m, 3) - 0.5)
    parts = W.spheres(pos, radii[:m], 1.6, vel=vel)
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.7, n_sub=7)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    G.step(2)
    O.step(2)
    P = O.particles()
    moved = P["pos"].copy()
    moved[::3, 0] = (moved[::3, 0] + 0.6) % box[0]
    for D in (G, O):
        D.set_particles(pos=moved, quat=P["quat"], vel=P["vel"], omega=P["omega"], acc=P["acc"],
                        alpha=P["alpha"], f_hyd=P["f_hyd"], m_hyd=P["m_hyd"])
    k, h = O.pairs()
    for D in (G, O):
        D.set_pairs(k, 0.5 * h)
    for _ in range(3):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12
        assert force_err(Pg["f_dem"], Po["f_dem"], O.scales()["f_dem"]) < 1e-12


@pytest.mark.parametrize("n", [600, 2300])
def test_hertz_dem_steps(ps, oracle_mod, n):
    """Hertz law through whole DEM steps: overlapping polydisperse spheres with
    walls, friction and gravity; 600 particles take the single-workgroup
    substeps, 2300 the multi-launch path."""
    box = (40, 36, 30) if n < 1000 else (72, 64, 60)
    rng = W.SplitMix64(88 + n)
    radii = 1.2 + 0.6 * rng.uniform(n)
    pos = W.rsa_spheres(rng, n, radii, box, [True, True, False], gap=-0.4)
    m = len(pos)
    parts = W.spheres(pos, radii[:m], 1.8, vel=0.01 * (rng.uniform(3 * m).reshape(m, 3) - 0.5))
    cfg = _walled(box, 0.7, "fp64", fluid_on=False, mu=0.3, restitution=0.6, n_sub=6,
                  gravity=[0.0, 0.0, -1e-4], contact_law="hertz", young=600.0, poisson=0.25)
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(3):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        assert vec_err(Pg["pos"], Po["pos"]) < 1e-12
        assert vec_err(Pg["vel"], Po["vel"]) < 1e-12
        assert force_err(Pg["f_dem"], Po["f_dem"], O.scales()["f_dem"]) < 1e-12
    assert O.counters()["contacts"] > 20


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_couette_hertz_steps(ps, oracle_mod, prec):
    """The coupled step with the Hertz law and TRT: Couette shear with spheres
    (48^3), three steps from creation against the oracle."""
    cfg, parts, _ = W.couette_suspension(precision=prec, n=48, nsph=30, radius=4.0)
    cfg.update(mu=0.3, contact_law="hertz", young=2e3, poisson=0.3, n_sub=10, collision="trt")
    G, O = _pair(ps, oracle_mod, cfg, parts)
    f0 = linear_shear_populations(oracle_mod, cfg["n"], 0, 2, cfg["wall_u"][4][0], cfg["wall_u"][5][0])
    G.set_populations(f0)
    O.set_populations(f0)
    for _ in range(3):
        G.step(1)
        O.step(1)
        assert np.array_equal(G.pairs()[0], O.pairs()[0])
        Pg, Po = G.particles(), O.particles()
        sc = O.scales()
        e = dict(pop=pop_err(G.populations(), O.populations()), pos=vec_err(Pg["pos"], Po["pos"]),
                 vel=vec_err(Pg["vel"], Po["vel"]), **hyd_errs(Pg, Po, sc, prec))
        print(f"Couette Hertz {prec}:", e, hyd_info(Pg, Po, sc))
        if prec == "fp64":
            assert max(e.values()) < TOL[prec]
    e = one_step_errors(G, O, prec)
    print(f"Couette Hertz {prec}, one step from the oracle's state:", e)
    assert max(bar_values(e)) < TOL[prec]


@pytest.mark.parametrize("phi", [0.15, 0.45])
def test_fluidized_bed_reduced(ps, oracle_mod, phi):
    """The paper's fluidized-bed recipe (D = 20, y walls, gravity -y, density
    1.1, 10 substeps, distance solid fraction, Hertz contacts) on a 128 x 104
    x 128 lattice: 61 spheres by random addition at 0.15, a settled bed of
    183 at 0.45 (the single-workgroup DEM; the full-size bed's 2866-8596
    spheres take the multi-launch path, covered by the settling-bed test);
    two coupled steps against the FP64 oracle, registrations and pairs bit
    for bit."""
    cfg, parts, meta = W.fluidized_bed(precision="fp64", phi=phi, n=(128, 104, 128))
    cfg["collision"] = "trt"
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(2):
        G.step(1)
        O.step(1)
    assert np.array_equal(G.pairs()[0], O.pairs()[0])
    cg, pg, bg = G.solid()
    co, po, bo = O.solid()
    assert np.array_equal(cg, co) and np.array_equal(pg, po)
    assert np.abs(bg - bo).max() < 1e-12
    assert pop_err(G.populations(), O.populations()) < TOL["fp64"]
    Pg, Po = G.particles(), O.particles()
    sc = O.scales()
    assert vec_err(Pg["pos"], Po["pos"]) < TOL["fp64"]
    assert vec_err(Pg["vel"], Po["vel"]) < TOL["fp64"]
    e = hyd_errs(Pg, Po, sc, "fp64")
    print(f"fluidized bed {phi}:", e, hyd_info(Pg, Po, sc))
    assert max(e.values()) < TOL["fp64"]


def test_couette_full_size_fp32(ps, oracle_mod):
    """The Couette workload at its full size (128^3, 500 spheres R = 5, moving
    walls, n_sub = 11) in FP32: two coupled steps from the wall profile
    against the FP64 oracle, pairs and solid slots bit for bit, then one step
    from the oracle's state at the FP32 bars."""
    cfg, parts, meta = W.couette_suspension(precision="fp32")
    G, O = _pair(ps, oracle_mod, cfg, parts)
    assert G.n_sub == O.n_sub == 11
    f0 = linear_shear_populations(oracle_mod, cfg["n"], 0, 2, cfg["wall_u"][4][0], cfg["wall_u"][5][0])
    G.set_populations(f0)
    O.set_populations(f0)
    for _ in range(2):
        G.step(1)
        O.step(1)
    assert np.array_equal(G.pairs()[0], O.pairs()[0])
    cg, pg, _ = G.solid()
    co, po, _ = O.solid()
    assert np.array_equal(cg, co) and np.array_equal(pg, po)
    Pg, Po = G.particles(), O.particles()
    traj = dict(pop=pop_err(G.populations(), O.populations()), pos=vec_err(Pg["pos"], Po["pos"]),
                vel=vec_err(Pg["vel"], Po["vel"]))
    print("Couette 128^3 FP32, two steps:", traj, "max |v| %.2e" % np.abs(Po["vel"]).max())
    assert np.abs(Po["vel"]).max() > 1e-5 and max(traj.values()) < TOL["fp32"]
    e = one_step_errors(G, O, "fp32")
    print("Couette 128^3 FP32, one step from the oracle's state:", e)
    assert max(bar_values(e)) < TOL["fp32"]


def test_settling_bed_multi_launch_coupled(ps, oracle_mod):
    """More particles than the single-workgroup DEM takes, coupled with the
    fluid: polydisperse spheres settling in a box walled on every face
    (n_sub = 32), FP64, two coupled steps against the oracle."""
    cfg, parts, meta = W.settling_bed(precision="fp64", n=(128, 128, 96))
    assert len(parts["pos"]) > 2048
    G, O = _pair(ps, oracle_mod, cfg, parts)
    for _ in range(2):
        G.step(1)
        O.step(1)
    assert np.array_equal(G.pairs()[0], O.pairs()[0])
    assert pop_err(G.populations(), O.populations()) < TOL["fp64"]
    Pg, Po = G.particles(), O.particles()
    sc = O.scales()
    assert vec_err(Pg["pos"], Po["pos"]) < TOL["fp64"]
    assert vec_err(Pg["vel"], Po["vel"]) < TOL["fp64"]
    e = dict(f_dem=force_err(Pg["f_dem"], Po["f_dem"], sc["f_dem"]), **hyd_errs(Pg, Po, sc, "fp64"))
    print("settling bed, multi-launch DEM:", e, hyd_info(Pg, Po, sc))
    assert max(e.values()) < TOL["fp64"]
