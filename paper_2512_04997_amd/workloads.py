"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method itself: only a counter-based
random generator (SplitMix64, Steele, Lea & Flood 2014), uniform random unit
quaternions (Shoemake, Graphics Gems III, 1992), random sequential addition of
non-overlapping particles, and the configuration dictionaries of the
workloads.  Both the HIP path's tests and the CPU oracle's tests draw their
inputs from here.

A configuration is a plain dict (lattice units, dx = dt = 1) and a particle set
a dict of numpy arrays: shape (n,) int32 0 sphere / 1 ellipsoid, semi (n,3),
dens (n,) density ratio, pos (n,3), quat (n,4) w,x,y,z, vel (n,3),
omega (n,3), fixed (n,) uint8.
"""
import math

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 stream; uniform doubles from the top 53 bits."""

    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next_u64(self, n=None):
        if n is None:
            self.state = (self.state + _GOLDEN) & _MASK
            z = self.state
            z = ((z ^ (z >> 30)) * _M1) & _MASK
            z = ((z ^ (z >> 27)) * _M2) & _MASK
            return z ^ (z >> 31)
        idx = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + idx * np.uint64(_GOLDEN)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * _GOLDEN) & _MASK
        return z

    def uniform(self, n=None):
        if n is None:
            return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def shoemake_quaternions(rng, n):
    """Uniform random unit quaternions (w, x, y, z), Shoemake's method."""
    u = rng.uniform(3 * n).reshape(n, 3)
    a = np.sqrt(1.0 - u[:, 0])
    b = np.sqrt(u[:, 0])
    t1 = 2.0 * math.pi * u[:, 1]
    t2 = 2.0 * math.pi * u[:, 2]
    return np.stack([b * np.cos(t2), a * np.sin(t1), a * np.cos(t1), b * np.sin(t2)], axis=1)


# ---------------------------------------------------------------------------
# contact-law parameter ratios at the paper's Poisson ratio 0.4999: the linear
# law takes k_t/k_n = 3(1-nu)/(2-nu) and gamma_t/gamma_n = sqrt(2(1-nu)/(2-nu))
# ---------------------------------------------------------------------------
NU = 0.4999
KT_RATIO = 3.0 * (1.0 - NU) / (2.0 - NU)
GT_RATIO = math.sqrt(2.0 * (1.0 - NU) / (2.0 - NU))


def rsa_spheres(rng, n, radii, box, periodic, region_lo=None, region_hi=None, gap=1.0,
                wall_gap=1.0, max_attempts=1_000_000):
    """Random sequential addition of spheres with a surface gap.

    radii: (n,) array drawn beforehand; box: (3,) extents; periodic: 3 bools.
    Centres are uniform in [region_lo, region_hi] shrunk by radius + wall_gap on
    walled axes; a candidate is kept when its surface gap to every placed
    sphere (minimum image on periodic axes) is at least `gap`.  Returns (m, 3)
    positions for the first m <= n spheres placed.
    """
    box = np.asarray(box, dtype=np.float64)
    lo = np.zeros(3) if region_lo is None else np.asarray(region_lo, np.float64)
    hi = box.copy() if region_hi is None else np.asarray(region_hi, np.float64)
    per = np.asarray(periodic, dtype=bool)
    radii = np.asarray(radii, dtype=np.float64)
    pos = np.zeros((n, 3))
    placed = 0
    attempts = 0
    for k in range(n):
        r = float(radii[k])
        l = lo.copy()
        h = hi.copy()
        for a in range(3):
            if not per[a]:
                l[a] = max(l[a], r + wall_gap)
                h[a] = min(h[a], box[a] - r - wall_gap)
        # candidates are drawn in batches and tested in draw order; the stream
        # is then rewound to just after the accepted one (SplitMix64 is a
        # counter), so the placements equal those of one draw at a time
        ok = False
        while attempts < max_attempts:
            nb = min(64, max_attempts - attempts)
            st0 = rng.state
            C = l[None, :] + (h - l)[None, :] * rng.uniform(3 * nb).reshape(nb, 3)
            if placed:
                d = C[:, None, :] - pos[None, :placed, :]
                d = np.where(per[None, None, :], d - box[None, None, :] * np.round(d / box[None, None, :]), d)
                dd = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
                clash = np.any(dd < ((r + radii[:placed] + gap) ** 2)[None, :], axis=1)
            else:
                clash = np.zeros(nb, dtype=bool)
            free = np.flatnonzero(~clash)
            if free.size == 0:
                attempts += nb
                continue
            i = int(free[0])
            attempts += i + 1
            rng.state = (st0 + 3 * (i + 1) * _GOLDEN) & _MASK
            c = C[i]
            ok = True
            break
        if not ok:
            break
        pos[k] = c
        placed += 1
    return pos[:placed]


# ---------------------------------------------------------------------------
# exact placement of ellipsoids
# ---------------------------------------------------------------------------
def _rotation(q):
    """Rotation matrices (body to world) of unit quaternions (w, x, y, z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((len(q), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def ellipsoid_shape_matrices(semi, quat):
    """A = R diag(a^2) R^T: the ellipsoid is {x : x^T A^-1 x <= 1} about its centre."""
    R = _rotation(np.asarray(quat, np.float64))
    s = np.asarray(semi, np.float64)
    return np.einsum("nij,nj,nkj->nik", R, s * s, R)


def _r_inv_r(C, r):
    """r^T C^-1 r for symmetric positive definite 3x3 matrices (adjugate form)."""
    a, b, c = C[:, 0, 0], C[:, 0, 1], C[:, 0, 2]
    d, e, f = C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]
    A00, A01, A02 = d * f - e * e, c * e - b * f, b * e - c * d
    A11, A12, A22 = a * f - c * c, b * c - a * e, a * d - b * b
    det = a * A00 + b * A01 + c * A02
    x, y, z = r[:, 0], r[:, 1], r[:, 2]
    return (A00 * x * x + A11 * y * y + A22 * z * z + 2.0 * (A01 * x * y + A02 * x * z + A12 * y * z)) / det


def ellipsoids_overlap(r, A, B, iters=40):
    """Overlap test of ellipsoid pairs (Perram & Wertheim, J. Comput. Phys. 58,
    1985): with shape matrices A, B and centre offset r, the two overlap exactly
    when max over 0 < l < 1 of S(l) = l (1 - l) r^T [(1 - l) A + l B]^-1 r is
    below 1 (S is concave in l).  The maximum is searched by golden sections;
    every evaluated S is a lower bound of it, so touching or nearly touching
    pairs are reported as overlapping (conservative for placement)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0

    def S(l):
        C = (1.0 - l)[:, None, None] * A + l[:, None, None] * B
        return l * (1.0 - l) * _r_inv_r(C, r)

    lo = np.zeros(len(r))
    hi = np.ones(len(r))
    c = hi - g * (hi - lo)
    d = lo + g * (hi - lo)
    fc, fd = S(c), S(d)
    best = np.maximum(fc, fd)
    for _ in range(iters):
        left = fc > fd
        hi = np.where(left, d, hi)
        lo = np.where(left, lo, c)
        nc = np.where(left, hi - g * (hi - lo), d)
        nd = np.where(left, c, lo + g * (hi - lo))
        fx = S(np.where(left, nc, nd))
        fc, fd = np.where(left, fx, fd), np.where(left, fc, fx)
        c, d = nc, nd
        best = np.maximum(best, fx)
    return best < 1.0


def rsa_ellipsoids_periodic(rng, n, semi, box, gap=1.0, batch=None, max_attempts=50_000_000):
    """Random sequential addition of equal ellipsoids in a periodic box with
    an exact overlap test.  Candidates come in batches: `batch` centres
    uniform in the box (3 batch uniforms), then `batch` Shoemake orientations
    (3 batch uniforms).  A candidate is kept when its ellipsoid with every
    semi-axis enlarged by gap/2 overlaps (ellipsoids_overlap, minimum image) no
    kept one's; candidates are tested in draw order against every earlier kept
    one, including those of their own batch, so the result is that of one
    candidate at a time.  Returns (pos (m, 3), quat (m, 4)), m <= n."""
    box = np.asarray(box, np.float64)
    infl = np.asarray(semi, np.float64) + 0.5 * gap
    bound, inner = float(infl.max()), float(infl.min())
    batch = batch or int(min(4096, max(128, n)))
    nc = np.maximum(1, np.floor(box / (2.0 * bound)).astype(np.int64))
    hc = box / nc
    ncell = int(np.prod(nc))
    K = 16
    grid = -np.ones((ncell, K), np.int64)
    gcnt = np.zeros(ncell, np.int64)
    pos = np.zeros((n + 1, 3))
    quat = np.zeros((n, 4))
    Am = np.zeros((n + 1, 3, 3))
    Am[n] = np.eye(3)
    off = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])

    def image(d):
        return d - box * np.round(d / box)

    def cell_id(c):
        return (c[..., 2] * nc[1] + c[..., 1]) * nc[0] + c[..., 0]

    placed = attempts = 0
    while placed < n and attempts < max_attempts:
        nb = min(batch, max_attempts - attempts)
        C = box[None, :] * rng.uniform(3 * nb).reshape(nb, 3)
        Q = shoemake_quaternions(rng, nb)
        attempts += nb
        Ab = ellipsoid_shape_matrices(np.tile(infl, (nb, 1)), Q)
        ci = np.minimum(np.floor(C / hc).astype(np.int64), nc - 1)
        # against the ellipsoids kept before this batch
        nbr = cell_id((ci[:, None, :] + off[None]) % nc)
        idx = grid[nbr].reshape(nb, -1)
        d = image(pos[np.where(idx >= 0, idx, n)] - C[:, None, :])
        dist = np.sqrt(np.sum(d * d, axis=2))
        valid = idx >= 0
        clash = np.any(valid & (dist < 2.0 * inner), axis=1)
        ii, jj = np.nonzero(valid & (dist >= 2.0 * inner) & (dist < 2.0 * bound) & ~clash[:, None])
        if len(ii):
            clash[ii[ellipsoids_overlap(d[ii, jj], Ab[ii], Am[idx[ii, jj]])]] = True
        # overlaps among the batch's survivors (earlier survivor jj, later ii)
        surv = np.flatnonzero(~clash)
        S = len(surv)
        if S == 0:
            continue
        cid = cell_id(ci[surv])
        cnt = np.bincount(cid, minlength=ncell)
        order = np.argsort(cid, kind="stable")
        rank = np.empty(S, np.int64)
        rank[order] = np.arange(S) - np.concatenate([[0], np.cumsum(cnt)[:-1]])[cid[order]]
        tg = -np.ones((ncell, int(cnt.max())), np.int64)
        tg[cid, rank] = np.arange(S)
        jdx = tg[cell_id((ci[surv][:, None, :] + off[None]) % nc)].reshape(S, -1)
        ii, kk = np.nonzero(jdx >= 0)
        jj = jdx[ii, kk]
        ii, jj = ii[jj < ii], jj[jj < ii]
        d2 = image(C[surv[jj]] - C[surv[ii]])
        dist = np.sqrt(np.sum(d2 * d2, axis=1))
        ovl = dist < 2.0 * inner
        m = ~ovl & (dist < 2.0 * bound)
        if np.any(m):
            ovl[m] = ellipsoids_overlap(d2[m], Ab[surv[ii[m]]], Ab[surv[jj[m]]])
        earlier = {}
        for a, b in zip(ii[ovl].tolist(), jj[ovl].tolist()):
            earlier.setdefault(a, []).append(b)
        taken = np.zeros(S, dtype=bool)
        for t in range(S):
            if placed >= n:
                break
            if any(taken[b] for b in earlier.get(t, ())):
                continue
            taken[t] = True
            s = surv[t]
            pos[placed], quat[placed], Am[placed] = C[s], Q[s], Ab[s]
            c = int(cell_id(ci[s]))
            if gcnt[c] >= K:
                raise RuntimeError("grid cell overflow in ellipsoid placement")
            grid[c, gcnt[c]] = placed
            gcnt[c] += 1
            placed += 1
    return pos[:placed], quat[:placed]


def _periodic(bc):
    return [bc[2 * a] == "periodic" for a in range(3)]


def base_config(n, tau, **kw):
    cfg = dict(n=tuple(n), tau=tau, rho0=1.0, bc=["periodic"] * 6, wall_u=[[0.0] * 3] * 6,
               body_force=[0.0] * 3, kolm_amp=0.0, kolm_axis=1, kolm_dir=0,
               gravity=[0.0] * 3, precision="fp64", sf_method="subdivision", sf_subdiv=10,
               fluid_on=True, dem_on=True, n_sub=0, dem_cell=0.0, kn=1e3, restitution=0.8,
               mu=0.3, kt_ratio=KT_RATIO, gt_ratio=GT_RATIO, max_solids=2)
    cfg.update(kw)
    return cfg


def spheres(pos, radii, dens, vel=None, omega=None, fixed=None):
    n = len(pos)
    radii = np.broadcast_to(np.asarray(radii, np.float64), (n,))
    return dict(shape=np.zeros(n, np.int32), semi=np.repeat(radii[:, None], 3, axis=1).copy(),
                dens=np.broadcast_to(np.asarray(dens, np.float64), (n,)).copy(),
                pos=np.asarray(pos, np.float64).reshape(n, 3).copy(),
                quat=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                vel=np.zeros((n, 3)) if vel is None else np.asarray(vel, np.float64).reshape(n, 3),
                omega=np.zeros((n, 3)) if omega is None else np.asarray(omega, np.float64).reshape(n, 3),
                fixed=np.zeros(n, np.uint8) if fixed is None else np.asarray(fixed, np.uint8))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def settling_sphere(precision="fp64", n=32, steps=200):
    """Plain method, one sphere R=4 at the box centre, density ratio 2, settling
    under gravity 1e-5 on a 32^3 periodic lattice, tau = 0.8, 200 steps."""
    cfg = base_config((n, n, n), 0.8, gravity=[0.0, 0.0, -1e-5], precision=precision, n_sub=1)
    c = n / 2.0
    parts = spheres([[c, c, c]], 4.0, 2.0)
    return cfg, parts, dict(workload="settling_sphere_32", steps=steps)


def couette_suspension(precision="fp32", n=128, nsph=500, radius=5.0, seed=1001, steps=1000):
    """Bounded Couette shear: n^3 lattice, moving walls beyond node layers 0 and
    n-1 at -/+0.02 in x, periodic x,y, tau = 0.7; nsph spheres of radius 5 at
    seeded non-overlapping positions, density ratio 1.5; linear spring-dashpot
    k_n = 1e3, restitution 0.8, Coulomb mu = 0.3."""
    bc = ["periodic", "periodic", "periodic", "periodic", "moving", "moving"]
    wu = [[0.0] * 3 for _ in range(6)]
    wu[4] = [-0.02, 0.0, 0.0]
    wu[5] = [0.02, 0.0, 0.0]
    cfg = base_config((n, n, n), 0.7, bc=bc, wall_u=wu, precision=precision, kn=1e3,
                      restitution=0.8, mu=0.3)
    rng = SplitMix64(seed)
    radii = np.full(nsph, radius)
    pos = rsa_spheres(rng, nsph, radii, (n, n, n), _periodic(bc))
    parts = spheres(pos, radius, 1.5)
    return cfg, parts, dict(workload=f"couette_{n}^3_{len(pos)}_spheres", steps=steps)


def serving_job(rng, kind, n, tau, nsph, r_lo=3.0, r_hi=6.0, precision="fp32", max_fraction=0.3):
    """One ensemble job on an n^3 lattice.

    kind 'settle': no-slip walls on every face, gravity (0, 0, -1e-5) on the
    particles, density ratio 2.  kind 'shear': periodic x and y, walls beyond
    node layers 0 and n-1 moving at -/+0.02 in x, density ratio 1.5.  nsph
    sphere radii uniform in [r_lo, r_hi], capped so that the solid volume
    fraction stays at most max_fraction; positions by random sequential
    addition (fewer spheres when the box fills up)."""
    radii = r_lo + (r_hi - r_lo) * rng.uniform(nsph) if nsph > 0 else np.zeros(0)
    vol = np.cumsum(4.0 / 3.0 * np.pi * radii ** 3)
    keep = int(np.searchsorted(vol, max_fraction * n ** 3, side="right"))
    radii = radii[:max(keep, 1 if nsph > 0 else 0)]
    wu = [[0.0] * 3 for _ in range(6)]
    if kind == "shear":
        bc = ["periodic", "periodic", "periodic", "periodic", "moving", "moving"]
        wu[4] = [-0.02, 0.0, 0.0]
        wu[5] = [0.02, 0.0, 0.0]
        cfg = base_config((n, n, n), tau, bc=bc, wall_u=wu, precision=precision)
        dens = 1.5
    else:
        bc = ["noslip"] * 6
        cfg = base_config((n, n, n), tau, bc=bc, gravity=[0.0, 0.0, -1e-5], precision=precision)
        dens = 2.0
    pos = rsa_spheres(rng, len(radii), radii, (n, n, n), _periodic(bc), max_attempts=200 * max(len(radii), 1))
    parts = spheres(pos, radii[:len(pos)], dens)
    return cfg, parts


def serving_stream(njobs=512, rate=50.0, steps=1000, sizes=(32, 64, 96, 128), tau=(0.55, 0.9), nsph=(1, 500),
                   r_lo=3.0, r_hi=6.0, precision="fp32", arrival_seed=4999, job_seed=5000):
    """A Poisson stream of independent settling / shear jobs.

    Arrivals: exponential gaps of mean 1/rate seconds from SplitMix64(arrival_seed).
    Job i, from SplitMix64(job_seed + i): a lattice edge drawn from `sizes`, tau
    uniform in `tau`, kind settle or shear with probability 1/2, a sphere count
    uniform in `nsph` (capped as in serving_job) and `steps` coupled steps.
    Returns a list of (arrival_s, cfg, parts, steps)."""
    arr = SplitMix64(arrival_seed)
    out = []
    t = 0.0
    for k in range(njobs):
        t += -math.log(1.0 - arr.uniform()) / rate
        rng = SplitMix64(job_seed + k)
        u = rng.uniform(4)
        n = int(sizes[min(int(u[0] * len(sizes)), len(sizes) - 1)])
        ta = tau[0] + (tau[1] - tau[0]) * u[1]
        kind = "settle" if u[2] < 0.5 else "shear"
        m = nsph[0] + min(int(u[3] * (nsph[1] - nsph[0] + 1)), nsph[1] - nsph[0])
        cfg, parts = serving_job(rng, kind, n, ta, m, r_lo, r_hi, precision)
        out.append((t, cfg, parts, steps))
    return out


def rsa_grid(rng, n, radii, box, periodic, region_lo=None, region_hi=None, gap=1.0, wall_gap=1.0,
             max_attempts=10_000_000, batch=64):
    """Random sequential addition for many spheres, accelerated by a uniform
    grid (cells of at least 2 max(r) + gap, so every possible clash lies in the
    27 surrounding cells).  Same rules as rsa_spheres: centres uniform in
    [region_lo, region_hi] shrunk by radius + wall_gap on walled axes, surface
    gap at least `gap` (minimum image on periodic axes).  Candidates are drawn
    in batches, tested in draw order, and the stream is rewound to just after
    the accepted one.  Returns (m, 3) positions for the first m <= n spheres."""
    box = np.asarray(box, dtype=np.float64)
    per = np.asarray(periodic, dtype=bool)
    radii = np.asarray(radii, dtype=np.float64)
    lo = np.zeros(3) if region_lo is None else np.asarray(region_lo, np.float64)
    hi = box.copy() if region_hi is None else np.asarray(region_hi, np.float64)
    rmax = float(radii.max()) if n else 1.0
    nc = np.maximum(1, np.floor(box / (2.0 * rmax + gap)).astype(np.int64))
    hc = box / nc
    K = 16
    grid = -np.ones((int(nc[0]), int(nc[1]), int(nc[2]), K), dtype=np.int64)
    gcnt = np.zeros((int(nc[0]), int(nc[1]), int(nc[2])), dtype=np.int64)
    pos = np.zeros((n + 1, 3))
    rad = np.concatenate([radii[:n], [0.0]])
    off = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    placed = 0
    attempts = 0
    for k in range(n):
        r = float(radii[k])
        l = lo.copy()
        h = hi.copy()
        for a in range(3):
            if not per[a]:
                l[a] = max(l[a], r + wall_gap)
                h[a] = min(h[a], box[a] - r - wall_gap)
        ok = False
        while attempts < max_attempts:
            nb = min(batch, max_attempts - attempts)
            st0 = rng.state
            C = l[None, :] + (h - l)[None, :] * rng.uniform(3 * nb).reshape(nb, 3)
            ci = np.minimum(np.floor(C / hc[None, :]).astype(np.int64), nc[None, :] - 1)
            nbr = ci[:, None, :] + off[None, :, :]
            inside = np.all(per[None, None, :] | ((nbr >= 0) & (nbr < nc[None, None, :])), axis=2)
            nbr = nbr % nc[None, None, :]
            idx = grid[nbr[..., 0], nbr[..., 1], nbr[..., 2]]
            idx = np.where(inside[..., None], idx, -1).reshape(nb, -1)
            P = pos[np.where(idx >= 0, idx, n)]
            d = C[:, None, :] - P
            d = np.where(per[None, None, :], d - box[None, None, :] * np.round(d / box[None, None, :]), d)
            dd = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
            lim = (r + rad[np.where(idx >= 0, idx, n)] + gap) ** 2
            clash = np.any((dd < lim) & (idx >= 0), axis=1)
            free = np.flatnonzero(~clash)
            if free.size == 0:
                attempts += nb
                continue
            i = int(free[0])
            attempts += i + 1
            rng.state = (st0 + 3 * (i + 1) * _GOLDEN) & _MASK
            c = ci[i]
            if gcnt[c[0], c[1], c[2]] >= K:
                raise RuntimeError("grid cell overflow in sphere placement")
            grid[c[0], c[1], c[2], gcnt[c[0], c[1], c[2]]] = placed
            gcnt[c[0], c[1], c[2]] += 1
            pos[placed] = C[i]
            placed += 1
            ok = True
            break
        if not ok:
            break
    return pos[:placed]


def rsa_equal_spheres_periodic(rng, n, r, box, gap=1.0, max_attempts=10_000_000):
    """rsa_grid for n equal spheres of radius r in a fully periodic box."""
    return rsa_grid(rng, n, np.full(n, float(r)), box, [True, True, True], gap=gap, max_attempts=max_attempts)


def settling_bed(precision="fp32", n=(256, 256, 128), fraction=0.15, seed=1002, steps=2000):
    """Polydisperse spheres (radius uniform in [2, 3]) placed by random
    sequential addition (surface gap 1) in the top 60 % of a box walled on
    every face, up to a solid fraction `fraction` of that region (0.15: with
    the unit gap the spheres' effective fraction is about 0.26, below the
    addition's jamming limit); tau = 0.6, density ratio 2.5, gravity
    (0, 0, -1e-5) on the particles, the linear contact law of the Couette
    workload, n_sub = 32."""
    bc = ["noslip"] * 6
    cfg = base_config(tuple(n), 0.6, bc=bc, gravity=[0.0, 0.0, -1e-5], precision=precision, n_sub=32,
                      kn=1e3, restitution=0.8, mu=0.3)
    rng = SplitMix64(seed)
    box = np.asarray(n, dtype=np.float64)
    lo = np.array([0.0, 0.0, 0.4 * box[2]])
    region = box[0] * box[1] * 0.6 * box[2]
    # radii drawn first, enough to fill the region at the target fraction
    mean_v = 4.0 / 3.0 * math.pi * 2.5 ** 3 * 1.05
    nmax = int(fraction * region / mean_v) + 1
    radii = 2.0 + rng.uniform(nmax)
    vol = np.cumsum(4.0 / 3.0 * math.pi * radii ** 3)
    m = int(np.searchsorted(vol, fraction * region, side="right"))
    radii = radii[:m]
    pos = rsa_grid(rng, m, radii, box, [False, False, False], region_lo=lo, max_attempts=50 * m)
    parts = spheres(pos, radii[:len(pos)], 2.5)
    return cfg, parts, dict(workload=f"settling_bed_{n[0]}x{n[1]}x{n[2]}_{len(pos)}_spheres", steps=steps)


def rsa_polydisperse(rng, rmin, rmax, box, region_lo, region_hi, target_volume, gap=0.0, wall_gap=0.0,
                     batch=16384, max_attempts=100_000_000):
    """Random sequential addition of spheres whose radii are drawn with their
    centres, in a box walled on every face, until the placed volume reaches
    target_volume.  Candidates come in batches: `batch` radii uniform in
    [rmin, rmax], then `batch` centres (3 uniforms each) uniform over the part of
    [region_lo, region_hi] that keeps the sphere wall_gap inside the box.  A
    candidate is kept when its surface clears every kept sphere's by `gap`
    (a grid of cells at least 2 rmax + gap wide holds them), tested in draw
    order against every earlier kept one, its own batch's included, so the
    result is that of one candidate at a time.  Near the fraction at which the
    addition jams, small candidates fit where large ones do not, so the kept
    radii lean to the small end.  Returns (pos (m, 3), radii (m,))."""
    box = np.asarray(box, np.float64)
    lo = np.asarray(region_lo, np.float64)
    hi = np.asarray(region_hi, np.float64)
    nc = np.maximum(1, np.floor(box / (2.0 * rmax + gap)).astype(np.int64))
    hc = box / nc
    ncell = int(np.prod(nc))
    K = 8  # a cell 2 rmax wide holds fewer than eight spheres of radius rmin / 2 or more
    grid = -np.ones((ncell, K), np.int64)
    gcnt = np.zeros(ncell, np.int64)
    cap = int(target_volume / (4.0 / 3.0 * math.pi * rmin ** 3)) + 2
    pos = np.full((cap + 1, 3), -1e9)
    rad = np.zeros(cap + 1)
    off = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])

    def cell_id(c):
        return (c[..., 2] * nc[1] + c[..., 1]) * nc[0] + c[..., 0]

    def near(cells, table):
        # entries of `table` in the 27 cells around each cell (outside the box: none)
        nbr = cells[:, None, :] + off[None]
        inb = np.all((nbr >= 0) & (nbr < nc), axis=2)
        ids = table[np.where(inb, cell_id(np.clip(nbr, 0, nc - 1)), 0)]
        return np.where(inb[:, :, None], ids, -1).reshape(len(cells), -1)

    placed = attempts = 0
    vol = 0.0
    while vol < target_volume and attempts < max_attempts:
        nb = batch
        R = rmin + (rmax - rmin) * rng.uniform(nb)
        U = rng.uniform(3 * nb).reshape(nb, 3)
        attempts += nb
        lo_c = np.maximum(lo[None, :], 0.0) + (R + wall_gap)[:, None]
        hi_c = np.minimum(hi[None, :], box[None, :]) - (R + wall_gap)[:, None]
        C = lo_c + (hi_c - lo_c) * U
        ci = np.clip(np.floor(C / hc).astype(np.int64), 0, nc - 1)
        # against the spheres kept before this batch
        idx = near(ci, grid)
        j = np.where(idx >= 0, idx, cap)
        d = pos[j] - C[:, None, :]
        clash = np.any((idx >= 0) & (np.sqrt(np.sum(d * d, axis=2)) < rad[j] + R[:, None] + gap), axis=1)
        surv = np.flatnonzero(~clash)
        S = len(surv)
        if S == 0:
            continue
        # among the batch's survivors (earlier survivor jj, later ii)
        cid = cell_id(ci[surv])
        cnt = np.bincount(cid, minlength=ncell)
        order = np.argsort(cid, kind="stable")
        rank = np.empty(S, np.int64)
        rank[order] = np.arange(S) - np.concatenate([[0], np.cumsum(cnt)[:-1]])[cid[order]]
        tg = -np.ones((ncell, int(cnt.max())), np.int64)
        tg[cid, rank] = np.arange(S)
        jdx = near(ci[surv], tg)
        ii, kk = np.nonzero(jdx >= 0)
        jj = jdx[ii, kk]
        ii, jj = ii[jj < ii], jj[jj < ii]
        d2 = C[surv[jj]] - C[surv[ii]]
        ovl = np.sqrt(np.sum(d2 * d2, axis=1)) < R[surv[ii]] + R[surv[jj]] + gap
        earlier = {}
        for a, b in zip(ii[ovl].tolist(), jj[ovl].tolist()):
            earlier.setdefault(a, []).append(b)
        taken = np.zeros(S, dtype=bool)
        for t in range(S):
            if vol >= target_volume:
                break
            if any(taken[b] for b in earlier.get(t, ())):
                continue
            taken[t] = True
            s_ = surv[t]
            c = int(cell_id(ci[s_]))
            if gcnt[c] >= K:
                raise RuntimeError("grid cell overflow in sphere placement")
            pos[placed], rad[placed] = C[s_], R[s_]
            grid[c, gcnt[c]] = placed
            gcnt[c] += 1
            placed += 1
            vol += 4.0 / 3.0 * math.pi * R[s_] ** 3
    return pos[:placed], rad[:placed]


def settling_bed_dense(precision="fp32", n=(256, 256, 128), fraction=0.30, seed=1005, steps=2000):
    """The DEM-heavy settling bed on the 256 x 256 x 128 lattice: polydisperse
    spheres (radius uniform in [2, 3] per candidate) placed by random sequential
    addition without overlap in the top 60 % of a box walled on every face,
    until they fill `fraction` of that region (0.30: about 26,500 spheres);
    tau = 0.6, density ratio 2.5, gravity (0, 0, -1e-5) on the particles, the
    linear contact law of the Couette workload, n_sub = 32."""
    bc = ["noslip"] * 6
    cfg = base_config(tuple(n), 0.6, bc=bc, gravity=[0.0, 0.0, -1e-5], precision=precision, n_sub=32,
                      kn=1e3, restitution=0.8, mu=0.3)
    box = np.asarray(n, dtype=np.float64)
    lo = np.array([0.0, 0.0, 0.4 * box[2]])
    region = box[0] * box[1] * 0.6 * box[2]
    pos, radii = rsa_polydisperse(SplitMix64(seed), 2.0, 3.0, box, lo, box, fraction * region)
    parts = spheres(pos, radii, 2.5)
    return cfg, parts, dict(workload=f"settling_bed_{n[0]}x{n[1]}x{n[2]}_{len(pos)}_spheres", steps=steps)


# sphere counts of the fluidized-bed benchmark at the fractions the paper lists
FLUIDIZED_COUNTS = {0.0: 0, 0.15: 2866, 0.30: 5731, 0.45: 8596}


def fluidized_bed(precision="fp32", phi=0.15, n=(500, 200, 800), radius=10.0, seed=1004, steps=200):
    """The paper's performance configuration (Sec. 5): a lattice of
    500 x 200 x 800 cells, periodic in x and z, no-slip walls in y, gravity
    along -y, spheres of diameter 20 cells at density ratio 1.1, 10 DEM
    substeps per step, the distance-based solid fraction, the TRT operator
    (the paper's choice for its studies), at a solid volume
    fraction phi of the whole box (2866, 5731, 8596 spheres at 0.15, 0.30,
    0.45; other fractions in proportion).  Lattice units: tau = 0.8
    (nu = 0.1) and g = 2.25e-4 make the Stokes settling Reynolds number
    u_s D / nu = 1 (u_s = 0.005); Hertz contacts (Y* = 100, nu = 0.3,
    e = 0.9, mu = 0.3), whose contact time spans well over 10 substeps.
    Placement: up to phi = 0.25 random sequential addition over the whole
    box (surface gap 1, wall gap 1); above it a settled bed, the stand-in for
    the paper's sedimentation-relaxation packing: a face-centred cubic
    lattice (cubic cell 31.25 x 31.25 x 32, nearest centres 22.1 apart)
    filled layer by layer from the y = 0 wall, the top layer in random order,
    every centre jittered by up to 0.5 per axis.  A smaller n keeps the
    recipe (count in proportion to the volume)."""
    nx, ny, nz = (int(v) for v in n)
    nu_p = 0.3
    young = 100.0 * 2.0 * (1.0 - nu_p * nu_p)
    cfg = base_config((nx, ny, nz), 0.8, bc=["periodic", "periodic", "noslip", "noslip", "periodic", "periodic"],
                      gravity=[0.0, -2.25e-4, 0.0], precision=precision, n_sub=10, sf_method="distance",
                      contact_law="hertz", young=young, poisson=nu_p, restitution=0.9, mu=0.3, kn=0.0,
                      collision="trt")
    vol = nx * ny * nz
    vs = 4.0 / 3.0 * math.pi * radius ** 3
    key = round(phi, 2)
    if (nx, ny, nz) == (500, 200, 800) and key in FLUIDIZED_COUNTS:
        count = FLUIDIZED_COUNTS[key]
    else:
        count = int(round(phi / 0.45 * 8596 * vol / (500 * 200 * 800)))
    rng = SplitMix64(seed)
    if count == 0:
        pos = np.zeros((0, 3))
    elif phi <= 0.25:
        radii = np.full(count, radius)
        pos = rsa_spheres(rng, count, radii, (nx, ny, nz), [True, False, True], gap=1.0)
    else:
        ax, az = nx / max(1, int(nx // 31.25)), nz / max(1, int(nz // 32.0))
        ay = 31.25
        cx, cz = int(round(nx / ax)), int(round(nz / az))
        layers = []
        k = 0
        while True:
            y = radius + 1.0 + k * ay / 2
            if y + radius + 1.0 > ny:
                break
            off = k % 2
            layer = []
            for i in range(cx):
                for j in range(cz):
                    # FCC: layer A holds (0, 0) and (1/2, 1/2), layer B (1/2, 0) and (0, 1/2)
                    for (u, w) in (((0.0, 0.0), (0.5, 0.5)) if off == 0 else ((0.5, 0.0), (0.0, 0.5))):
                        layer.append(((i + u + 0.25) * ax, y, (j + w + 0.25) * az))
            layers.append(np.array(layer))
            k += 1
        pts = []
        for L in layers:
            need = count - sum(len(p) for p in pts)
            if need <= 0:
                break
            if need < len(L):
                order = np.argsort(rng.uniform(len(L)), kind="stable")
                L = L[np.sort(order[:need])]
            pts.append(L)
        pos = np.concatenate(pts)
        if len(pos) < count:
            raise ValueError("the settled bed holds %d of %d spheres" % (len(pos), count))
        pos = pos + (rng.uniform(3 * len(pos)).reshape(-1, 3) - 0.5)
        pos[:, 0] %= nx
        pos[:, 2] %= nz
    m = len(pos)
    parts = spheres(pos, radius, 1.1) if m else None
    name = f"fluidized_bed_{nx}x{ny}x{nz}_phi{phi:.2f}_{m}_spheres"
    return cfg, parts, dict(workload=name, steps=steps, phi=phi)


def kolmogorov_ellipsoids(n=512, count=None, precision="fp32", seed=1003, amp=1e-6):
    """Periodic n^3 lattice, tau = 0.55, Kolmogorov forcing of the fluid with
    component x = amp sin(2 pi (y + 1/2) / n); `count` prolate ellipsoids with
    semi-axes (6, 3, 3) (default: 50,000 at 512^3 and the same number density
    at other sizes, 98 at 64^3), density ratio 1.2, uniform random
    orientations (Shoemake), placed by random sequential addition with the
    exact ellipsoid overlap test and a gap of 1 (semi-axes enlarged by 1/2);
    linear contact law k_n = 1e3, e = 0.8, mu = 0.3."""
    cfg = base_config((n, n, n), 0.55, kolm_amp=amp, kolm_axis=1, kolm_dir=0, precision=precision,
                      kn=1e3, restitution=0.8, mu=0.3)
    if count is None:
        count = int(round(50000 * (n / 512.0) ** 3))
    rng = SplitMix64(seed)
    pos, quat = rsa_ellipsoids_periodic(rng, count, [6.0, 3.0, 3.0], (n, n, n))
    m = len(pos)
    parts = dict(shape=np.ones(m, np.int32), semi=np.tile([6.0, 3.0, 3.0], (m, 1)),
                 dens=np.full(m, 1.2), pos=pos, quat=quat, vel=np.zeros((m, 3)), omega=np.zeros((m, 3)),
                 fixed=np.zeros(m, np.uint8))
    return cfg, parts, dict(workload=f"kolmogorov_{n}^3_{m}_ellipsoids", steps=500, warmup=50)
