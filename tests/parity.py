"""Helpers for comparing the HIP path with the CPU oracle (no arithmetic of the
method: norms and scales only).

The floating-point bars are those of the parity protocol: 1e-12 relative in
FP64, 1e-5 in FP32, in these norms:
  populations  max |f_gpu - f_ora| / max |f_ora|, compared as f - w_i;
  vectors      max |a - b| / max |b| (particle positions, velocities), with
               an explicit floor only where a test states the velocity scale
               of its case;
  forces       per particle and component |a - b| / sum_j |term_j|, the L1
               norm of the summands the force is the sum of: the per-cell
               momentum-exchange terms B_k sum_i Omega^s_ik c_i (and their
               torques (r_j - r_k) x term) for F_hyd and M_hyd, the pair
               forces and torques for F_dem and M_dem (the oracle accumulates
               these norms beside the sums).
"""
import numpy as np

W = np.array([1 / 3] + [1 / 18] * 3 + [1 / 36] * 6 + [1 / 18] * 3 + [1 / 36] * 6)

# floating-point bars of the parity protocol
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def pop_err(fg, fo):
    """Populations compared as f - w_i, normalised by max |f|."""
    return float(np.max(np.abs(fg - fo)) / np.max(np.abs(fo)))


def vec_err(a, b, floor=0.0):
    """max |a - b| normalised by max(|b|_inf, floor); floor 0 is purely relative."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    d = float(np.max(np.abs(a - b)))
    s = max(float(np.max(np.abs(b))), floor)
    return d / s if s > 0 else (0.0 if d == 0.0 else float("inf"))


def force_err(a, b, scale):
    """Forces normalised per particle and component by the L1 norm of their
    summands; a component whose summands are all zero must match exactly."""
    a, b, scale = (np.asarray(x, dtype=np.float64) for x in (a, b, scale))
    if a.size == 0:
        return 0.0
    d = np.abs(a - b)
    if np.any((scale == 0) & (d != 0)):
        return float("inf")
    return float((d / np.where(scale > 0, scale, 1.0)).max())


def copy_state(src, dst, pairs=True):
    """Shared input state: canonical populations, particle state, pair list."""
    dst.set_populations(src.populations())
    P = src.particles()
    dst.set_particles(pos=P["pos"], quat=P["quat"], vel=P["vel"], omega=P["omega"], acc=P["acc"],
                      alpha=P["alpha"], f_hyd=P["f_hyd"], m_hyd=P["m_hyd"])
    if pairs:
        k, h = src.pairs()
        dst.set_pairs(k, h)


def linear_shear_populations(oracle_mod, n, axis_u, axis_y, U_lo, U_hi):
    """Equilibrium populations (rho = 1, the oracle's f^eq) of a linear shear
    profile: velocity component axis_u rising from U_lo at the low wall to U_hi
    at the high wall along axis_y (walls on the planes 0 and n of that axis,
    cell centres at index + 1/2).  Layout [19][N], cell x + nx (y + ny z)."""
    N = n[0] * n[1] * n[2]
    idx = np.arange(N)
    coord = [idx % n[0], idx // n[0] % n[1], idx // (n[0] * n[1])]
    layer = coord[axis_y]
    f = np.zeros((19, N))
    for c in range(n[axis_y]):
        u = np.zeros(3)
        u[axis_u] = U_lo + (U_hi - U_lo) * (c + 0.5) / n[axis_y]
        f[:, layer == c] = oracle_mod.feq(1.0, u)[:, None]
    return f
