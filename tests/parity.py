"""Helpers for comparing the HIP path with the CPU oracle (no arithmetic of the
method: norms and scales only)."""
import numpy as np

W = np.array([1 / 3] + [1 / 18] * 3 + [1 / 36] * 6 + [1 / 18] * 3 + [1 / 36] * 6)

# floating-point bars of the parity protocol
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def pop_err(fg, fo):
    """Populations compared as f - w_i, normalised by max |f|."""
    return float(np.max(np.abs(fg - fo)) / np.max(np.abs(fo)))


def vec_err(a, b, floor=1e-3):
    """Vectors normalised by max(|b|_inf, floor)."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)) if np.size(b) else 0.0, floor))


def force_floor(oracle_dom, accel=1e-6):
    """Per-particle force floor: the force accelerating the particle's volume of
    fluid by `accel` per step.  Summands that are pure round-off (a body at rest
    in fluid at rest) are measured against it rather than against themselves."""
    m = oracle_dom.mass()
    dens = np.asarray(oracle_dom._keep["dens"], dtype=np.float64)
    return (accel * m / dens)[:, None]


def force_err(a, b, scale, floor=0.0):
    """Forces normalised per component by the L1 norm of their summands (floored)."""
    a, b, scale = (np.asarray(x, dtype=np.float64) for x in (a, b, scale))
    if a.size == 0:
        return 0.0
    s = np.maximum(np.maximum(scale, floor), 1e-300)
    return float((np.abs(a - b) / s).max())


def copy_state(src, dst, pairs=True):
    """Shared input state: canonical populations, particle state, pair list."""
    dst.set_populations(src.populations())
    P = src.particles()
    dst.set_particles(pos=P["pos"], quat=P["quat"], vel=P["vel"], omega=P["omega"], acc=P["acc"],
                      alpha=P["alpha"], f_hyd=P["f_hyd"], m_hyd=P["m_hyd"])
    if pairs:
        k, h = src.pairs()
        dst.set_pairs(k, h)
