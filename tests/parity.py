"""Helpers for comparing the HIP path with the CPU oracle (no arithmetic of the
method: norms and scales only).

The floating-point bars are those of the parity protocol: 1e-12 relative in
FP64, 1e-5 in FP32, in these norms:
  populations  max |f_gpu - f_ora| / max |f_ora|, compared as f - w_i;
  vectors      max |a - b| / max |b| (particle positions, velocities), or
               against a velocity scale a test states for its case;
  forces       per particle and component |a - b| / S, where S is the
               rounding scale of the sum (the oracle accumulates it beside the
               sums).  A hydrodynamic force is a sum over cells of momentum-
               exchange terms, each a difference of populations of size w_i
               whose result is often many orders smaller: its rounding error is
               a few eps times the magnitudes it is formed from, not times the
               term.  S is therefore those magnitudes, as populations for FP64
               (f, f^eq) and as deviations from the weights (f - w, f^eq - w)
               for FP32, whose shifted storage and arithmetic round the
               deviations.  (The L1 norm of the terms themselves is no bound:
               perturbing every population by one eps moves F_hyd by up to
               10^4-10^5 eps times it, tested on the oracle.)  DEM forces use the
               L1 norm of the pair forces and torques (positions are FP64 in
               every mode).
Comparisons in FP32 follow the protocol's identical input state: the GPU
receives the oracle's state (populations, particles, pair list and history)
and both take one coupled step; longer FP32 trajectories diverge from the FP64
one by accumulated storage rounding, and their errors are printed.
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


def hyd_errs(Pg, Po, sc, prec):
    """F_hyd and M_hyd errors against the rounding scale of the precision."""
    g = "" if prec == "fp64" else "_g"
    return dict(f_hyd=force_err(Pg["f_hyd"], Po["f_hyd"], sc["f_hyd" + g]),
                m_hyd=force_err(Pg["m_hyd"], Po["m_hyd"], sc["m_hyd" + g]))


def hyd_info(Pg, Po, sc):
    """For the record: F_hyd and M_hyd errors against the largest force of the
    set and against the L1 norm of the per-cell terms."""
    return dict(f_hyd_vs_max=vec_err(Pg["f_hyd"], Po["f_hyd"]), m_hyd_vs_max=vec_err(Pg["m_hyd"], Po["m_hyd"]),
                f_hyd_vs_terms=force_err(Pg["f_hyd"], Po["f_hyd"], np.maximum(sc["f_hyd_sum"], 1e-300)),
                m_hyd_vs_terms=force_err(Pg["m_hyd"], Po["m_hyd"], np.maximum(sc["m_hyd_sum"], 1e-300)))


def one_step_errors(G, O, prec, dem=True):
    """The protocol's single step from an identical input state: the GPU
    takes the oracle's state, both step once; errors of populations,
    particle state and forces."""
    copy_state(O, G, pairs=dem and O.np > 0)
    G.step(1)
    O.step(1)
    e = dict(pop=pop_err(G.populations(), O.populations()))
    if O.np:
        Pg, Po = G.particles(), O.particles()
        sc = O.scales()
        e.update(pos=vec_err(Pg["pos"], Po["pos"]), vel=vec_err(Pg["vel"], Po["vel"]),
                 omega=vec_err(Pg["omega"], Po["omega"]), **hyd_errs(Pg, Po, sc, prec))
        if dem:
            e["f_dem"] = force_err(Pg["f_dem"], Po["f_dem"], sc["f_dem"])
        e["info"] = hyd_info(Pg, Po, sc)
    return e


def bar_values(e):
    """The asserted entries of an error dict (the record-only ones removed)."""
    return [v for k, v in e.items() if k != "info"]

