"""Helpers shared by the GPU parity tests (comparison by particle id, tolerances)."""
import numpy as np

# FP32 cell+offset form against the FP64 oracle (single stage from identical state):
# velocities and offsets carry a few binary32 roundings.
TOL_V32 = 4e-6       # relative to the largest speed of the species
TOL_X32 = 2e-6       # in cells
TOL_F64 = 1e-12      # FP64 form: relative
TOL_FIELD = 1e-5     # fields rho, phi, E: rel = max|a - b| / max|b|
TOL_MOMENT = 1e-4    # moments and energies


def by_id(p):
    o = np.argsort(p["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in p.items() if k != "next_id"}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def compare_particles(g, o, dx, f64, vtol=None, xtol=None, exclude=None):
    """Particles of one species from the GPU (g) and the oracle (o), matched by id."""
    G, O = by_id(g), by_id(o)
    if exclude is not None and len(exclude):
        keepg = ~np.isin(G["id"], exclude)
        keepo = ~np.isin(O["id"], exclude)
        G = {k: v[keepg] for k, v in G.items()}
        O = {k: v[keepo] for k, v in O.items()}
    assert np.array_equal(G["id"], O["id"]), (len(G["id"]), len(O["id"]))
    if len(G["id"]) == 0:
        return
    vmax = max(np.max(np.abs(O[k])) for k in ("vx", "vy", "vz"))
    vt = vtol if vtol is not None else (TOL_F64 if f64 else TOL_V32)
    xt = xtol if xtol is not None else (1e-10 if f64 else TOL_X32)
    for k in ("vx", "vy", "vz"):
        d = np.max(np.abs(G[k] - O[k]))
        assert d <= vt * max(vmax, 1e-300), (k, d, vmax)
    dxs = np.max(np.abs(G["x"] - O["x"])) / dx
    assert dxs <= xt, ("x", dxs)


def cell_counts(x, dx, n):
    return np.bincount(np.floor(np.asarray(x) / dx).astype(np.int64), minlength=n)
