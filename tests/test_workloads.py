"""The seeded input generators (no arithmetic of the method): the exact
ellipsoid overlap test used to place the Kolmogorov-ellipsoid workload, and
the placements themselves.

  - the Perram-Wertheim test agrees with a brute-force point-sampling check on
    random pairs of (6.5, 3.5, 3.5) ellipsoids at every orientation;
  - two equal spheres written as ellipsoids overlap exactly when their centres
    are closer than the sum of the radii;
  - the placement of the 64^3 box (98 ellipsoids, the number density of
    50,000 in 512^3) leaves no pair overlapping, with the unit gap, checked by
    point sampling; it is reproducible from its seed; candidates are tested
    against earlier ones of their own batch (a batch of one gives the same
    placement)."""
import numpy as np

from paper_2512_04997_amd import workloads as W


def _rot(q):
    return W._rotation(np.asarray(q, np.float64).reshape(-1, 4))


def _points_inside(semi_a, Ra, ca, semi_b, Rb, cb, samples=6000, seed=0):
    """Any point of ellipsoid a (surface and two inner shells, sampled) inside
    ellipsoid b?"""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(samples, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    pts = np.concatenate([u * semi_a * s for s in (1.0, 0.95, 0.8)])
    world = pts @ Ra.T + ca
    body = (world - cb) @ Rb
    return bool(np.any(np.sum((body / semi_b) ** 2, axis=1) < 1.0))


def test_overlap_test_against_point_sampling():
    rng = np.random.default_rng(7)
    m = 300
    semi = np.array([6.5, 3.5, 3.5])
    qa = rng.normal(size=(m, 4))
    qa /= np.linalg.norm(qa, axis=1)[:, None]
    qb = rng.normal(size=(m, 4))
    qb /= np.linalg.norm(qb, axis=1)[:, None]
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = d * rng.uniform(7.0, 13.0, size=(m, 1))
    A = W.ellipsoid_shape_matrices(np.tile(semi, (m, 1)), qa)
    B = W.ellipsoid_shape_matrices(np.tile(semi, (m, 1)), qb)
    ov = W.ellipsoids_overlap(r, A, B)
    Ra, Rb = _rot(qa), _rot(qb)
    sampled = np.array([_points_inside(semi, Ra[k], np.zeros(3), semi, Rb[k], r[k], seed=k) or
                        _points_inside(semi, Rb[k], r[k], semi, Ra[k], np.zeros(3), seed=k + 1)
                        for k in range(m)])
    # sampling finds no overlap the exact test misses, and misses at most the
    # few overlaps too shallow for its points
    assert not np.any(sampled & ~ov)
    assert 0.2 * m < ov.sum() < 0.9 * m
    assert (ov & ~sampled).sum() <= 0.03 * m


def test_overlap_test_of_spheres():
    m = 200
    rng = np.random.default_rng(3)
    q = rng.normal(size=(2 * m, 4))
    q /= np.linalg.norm(q, axis=1)[:, None]
    A = W.ellipsoid_shape_matrices(np.full((m, 3), 2.0), q[:m])
    B = W.ellipsoid_shape_matrices(np.full((m, 3), 3.0), q[m:])
    dist = np.linspace(4.0, 6.0, m)
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    ov = W.ellipsoids_overlap(d * dist[:, None], A, B)
    far = np.abs(dist - 5.0) > 1e-6
    assert np.array_equal(ov[far], dist[far] < 5.0)


def test_ellipsoid_placement_has_no_overlap_and_is_reproducible():
    cfg, parts, meta = W.kolmogorov_ellipsoids(n=64, precision="fp64")
    pos, quat, semi = parts["pos"], parts["quat"], parts["semi"]
    n = len(pos)
    assert n == 98 and cfg["n"] == (64, 64, 64) and cfg["kolm_amp"] == 1e-6
    assert np.allclose(np.linalg.norm(quat, axis=1), 1.0)
    assert np.all((pos >= 0.0) & (pos < 64.0))
    R = _rot(quat)
    infl = semi[0] + 0.5
    close = 0
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[j] - pos[i]
            d -= 64.0 * np.round(d / 64.0)
            if np.linalg.norm(d) >= 13.0:
                continue
            close += 1
            assert not _points_inside(infl, R[i], np.zeros(3), infl, R[j], d, samples=2000, seed=i * n + j)
            A = W.ellipsoid_shape_matrices(infl[None], quat[i:i + 1])
            B = W.ellipsoid_shape_matrices(infl[None], quat[j:j + 1])
            assert not W.ellipsoids_overlap(d[None], A, B)[0]
    assert close > 20
    _, again, _ = W.kolmogorov_ellipsoids(n=64)
    assert np.array_equal(again["pos"], pos) and np.array_equal(again["quat"], quat)


def test_placement_tests_candidates_within_their_batch():
    box = (40.0, 40.0, 40.0)
    p1, q1 = W.rsa_ellipsoids_periodic(W.SplitMix64(11), 40, [6.0, 3.0, 3.0], box, batch=256)
    # one candidate per batch draws the centre and the orientation of each
    # candidate from a different part of the stream, so compare properties:
    # every pair is separated (with the gap) in both placements
    for pos, quat in ((p1, q1),) + (W.rsa_ellipsoids_periodic(W.SplitMix64(11), 40, [6.0, 3.0, 3.0], box,
                                                                batch=1),):
        A = W.ellipsoid_shape_matrices(np.full((len(pos), 3), 1.0) * [6.5, 3.5, 3.5], quat)
        for i in range(len(pos)):
            d = pos - pos[i]
            d -= 40.0 * np.round(d / 40.0)
            m = np.arange(len(pos)) > i
            assert not np.any(W.ellipsoids_overlap(d[m], np.repeat(A[i:i + 1], m.sum(), 0), A[m]))
    assert len(p1) == 40


def test_polydisperse_addition_in_a_walled_box():
    """The dense settling bed's placement: no two spheres overlap (all pairs,
    brute force), each lies inside the box and its region, the placed volume
    reaches the requested fraction, radii stay in [2, 3], and the same seed
    gives the same bed."""
    box = np.array([48.0, 40.0, 36.0])
    lo = np.array([0.0, 0.0, 0.4 * box[2]])
    region = box[0] * box[1] * 0.6 * box[2]
    pos, r = W.rsa_polydisperse(W.SplitMix64(7), 2.0, 3.0, box, lo, box, 0.3 * region, batch=2048)
    d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    assert np.all(d >= r[:, None] + r[None, :])
    assert np.all(pos - r[:, None] >= lo) and np.all(pos + r[:, None] <= box)
    assert np.all((r >= 2.0) & (r <= 3.0))
    vol = (4.0 / 3.0 * np.pi * r ** 3).sum()
    assert 0.3 * region <= vol < 0.3 * region + 4.0 / 3.0 * np.pi * 27.0
    pos2, r2 = W.rsa_polydisperse(W.SplitMix64(7), 2.0, 3.0, box, lo, box, 0.3 * region, batch=2048)
    assert np.array_equal(pos, pos2) and np.array_equal(r, r2)
