"""Seeded synthetic workloads and injected particle states.

This module holds no arithmetic of the method: it only states problem sizes and physical
constants (normalised units eps0 = e = m_e = n0 = T_e = 1, so omega_pe = v_th,e =
lambda_D = 1) and draws plain random inputs with numpy.  Both the GPU library's tests and
the CPU oracle's tests take their inputs from here, so neither side ever feeds the other.

The paper's sheath decks (a double-bounded magnetised layer, 200 particles per cell per
charged species; see its experimental-setup section and the sheath-case table) are not
available, so the workloads below stand in for them at the sizes that section gives and at
the smaller sizes a single GPU and a CPU check can run.
"""
from __future__ import annotations

import copy
import math

import numpy as np

M_ION = 73440.0          # argon-mass ions in electron masses
T_RATIO = 10.0           # T_e / T_i
DX = 0.5                 # lambda_D / 2
DT = 0.1                 # omega_pe dt
B_ANGLE_DEG = 80.0       # angle between B and the x axis
WCE_OVER_WPE = 2.0       # |q_e| B / m_e in units of omega_pe
NGS_EL = 0.01            # n_g sigma, electron elastic (per lambda_D)
NGS_IZ = 0.005           # n_g sigma, electron-impact ionisation
NGS_CX = 1.0             # n_g sigma, ion charge exchange
EPS_IZ = 1.576           # ionisation energy: argon 15.76 eV at T_e = 10 eV


def oblique_B(wce=WCE_OVER_WPE, angle_deg=B_ANGLE_DEG):
    th = math.radians(angle_deg)
    return [wce * math.cos(th), wce * math.sin(th), 0.0]


def species(q, m, T, ppc, ncells, cap_factor=1.25, extra=0):
    """A species record; w = n0 L / P = dx / ppc so that n0 = 1."""
    return {
        "q": float(q), "m": float(m), "w": DX / ppc if ppc > 0 else DX,
        "T": float(T), "ppc": int(ppc),
        "capacity": int(math.ceil(cap_factor * ppc * ncells)) + int(extra),
    }


def ensemble(ncells, ppc, *, T_i=1.0 / T_RATIO, B=None, seed=1, periodic=False,
             nspecies=2, collisions=True, sort_every=0, init_mode=0, E_ext=0.0,
             perturb_amp=0.0, perturb_mode=1, T_e=1.0, cap_factor=1.25, extra=0,
             floating=False, smooth=0, recycle=False, neutral_capacity=0, src_pairs=0,
             src_frac=0.5, cx_relative=False):
    sp = [species(-1.0, 1.0, T_e, ppc, ncells, cap_factor, extra)]
    if nspecies > 1:
        sp.append(species(+1.0, M_ION, T_i, ppc, ncells, cap_factor, extra))
    return {
        "ncells": int(ncells), "periodic": bool(periodic), "nspecies": int(nspecies),
        "collisions": bool(collisions), "init_mode": int(init_mode),
        "dx": DX, "dt": DT, "eps0": 1.0,
        "B": list(B) if B is not None else [0.0, 0.0, 0.0],
        "E_ext": float(E_ext), "seed": int(seed), "sort_every": int(sort_every),
        "species": sp,
        "ngs_el": NGS_EL, "ngs_iz": NGS_IZ, "ngs_cx": NGS_CX, "eps_iz": EPS_IZ,
        "T_n": float(T_i), "m_n": M_ION,
        "perturb_amp": float(perturb_amp), "perturb_mode": int(perturb_mode),
        "floating": bool(floating), "smooth": int(smooth),
        "recycle": bool(recycle), "neutral_capacity": int(neutral_capacity),
        "src_pairs": int(src_pairs), "src_frac": float(src_frac),
        "cx_relative": bool(cx_relative),
    }


# ---- the five workloads -----------------------------------------------------------------
def c1_plain_small(seed=1):
    """256 cells, 100 ppc per species (51,200 particles), B = 0, collisions, 1000 steps."""
    e = ensemble(256, 100, seed=seed, sort_every=0)
    return {"name": "plain-256cells-100ppc", "steps": 1000, "precision": "fp64",
            "ensembles": [e]}


def c2_sheath(seed=1, ncells=100_000, ppc=200):
    """1e5 cells, 200 ppc per species (4.0e7 particles), oblique B, three channels,
    absorbing walls, sort every 20 steps, 1000 steps."""
    e = ensemble(ncells, ppc, seed=seed, B=oblique_B(), sort_every=20)
    return {"name": f"sheath-{ncells}cells-{ppc}ppc", "steps": 1000, "precision": "fp32",
            "ensembles": [e]}


def c3_batched(n_ens=64, seed=12345, scale=1.0):
    """64 independent ensembles: cells log-uniform in [1k, 64k], ppc uniform in [50, 400],
    T_e/T_i uniform in [1, 20], own seeds e + 1, B = 0, sort every 20, 500 steps.
    `scale` shrinks cells for quick checks."""
    rng = np.random.default_rng(seed)
    ens = []
    for k in range(n_ens):
        n = int(1000 * 64 ** rng.random())
        n = max(4, int(n * scale))
        ppc = 50 + int(351 * rng.random())
        ratio = 1.0 + 19.0 * rng.random()
        ens.append(ensemble(n, ppc, T_i=1.0 / ratio, seed=k + 1, sort_every=20))
    return {"name": f"batched-{n_ens}ens", "steps": 500, "precision": "fp32", "ensembles": ens}


def c4_langmuir(ncells=2048, ppc=200, amp=0.01, E_ext=0.0):
    """2048 cells periodic, 200 ppc cold electrons on a fixed ion background, sinusoidal
    perturbation amplitude 0.01 (mode 1), collisionless, 200 steps."""
    e = ensemble(ncells, ppc, periodic=True, nspecies=1, collisions=False, init_mode=1,
                 T_e=0.0, perturb_amp=amp, perturb_mode=1, E_ext=E_ext, cap_factor=1.0)
    return {"name": f"langmuir-{ncells}cells-{ppc}ppc", "steps": 200, "precision": "fp32",
            "ensembles": [e]}


def c5_large(seed=1, ncells=1_000_000, ppc=500):
    """1e6 cells, 500 ppc per species (1.0e9 particles), oblique B, three channels with
    ionisation creating pairs, absorbing walls, sort every 10 steps, 200 steps."""
    e = ensemble(ncells, ppc, seed=seed, B=oblique_B(), sort_every=10)
    return {"name": f"large-{ncells}cells-{ppc}ppc", "steps": 200, "precision": "fp32",
            "ensembles": [e]}


def c6_sheath_recycling(seed=1, ncells=100_000, ppc=200):
    """The uniform-load sheath case with its three species: the 1e5-cell, 200 ppc slab
    with floating walls that keep the absorbed charge and recycle every absorbed ion into a
    D neutral (electrons, ions, neutrals)."""
    e = ensemble(ncells, ppc, seed=seed, B=oblique_B(), sort_every=20, floating=True,
                 recycle=True, neutral_capacity=ppc * ncells // 4)
    return {"name": f"sheath-recycling-{ncells}cells-{ppc}ppc", "steps": 1000,
            "precision": "fp32", "ensembles": [e]}


def c7_sheath_source(seed=1, ncells=100_000, ref_ppc=200, pairs_per_step=20_000,
                     capacity=25_000_000):
    """The non-uniform-load sheath case: an initially empty 1e5-cell slab filled by a
    volumetric source of electron-ion pairs in its left half, floating recycling walls.
    Macro-particle weight as for 200 ppc at the reference density."""
    e = ensemble(ncells, 0, seed=seed, B=oblique_B(), sort_every=20, floating=True,
                 recycle=True, neutral_capacity=capacity // 4, src_pairs=pairs_per_step,
                 src_frac=0.5)
    for sp in e["species"]:
        sp["w"] = DX / ref_ppc
        sp["capacity"] = int(capacity)
    return {"name": f"sheath-source-{ncells}cells", "steps": 1000, "precision": "fp32",
            "ensembles": [e]}


def scaled(work, ncells=None, ppc=None, steps=None):
    """The same physics at a smaller size (cells and/or ppc), for oracle-sized checks."""
    w = copy.deepcopy(work)
    for e in w["ensembles"]:
        n = ncells or e["ncells"]
        for sp in e["species"]:
            p = ppc or sp["ppc"]
            sp["ppc"] = int(p)
            sp["w"] = e["dx"] / p
            sp["capacity"] = int(math.ceil(1.25 * p * n)) + 64
        if e.get("recycle"):
            e["neutral_capacity"] = int(math.ceil(0.25 * (ppc or e["species"][0]["ppc"]) * n)) + 64
        e["ncells"] = int(n)
    if steps is not None:
        w["steps"] = int(steps)
    return w


# ---- injected states ---------------------------------------------------------------------
def random_state(e, n_per_species, seed=0, vscale=None, shuffle_ids=True, sort_by_cell=False,
                 cell_range=None):
    """Random particles whose positions and velocities are exact binary32 values, so the
    same numbers mean the same thing in both precisions.  Returns one dict per species with
    cell (int32), off (float32 in [0,1)), x = (cell + off) dx (float64), vx, vy, vz
    (float32), id (uint32) and next_id."""
    rng = np.random.default_rng(seed)
    out = []
    N = e["ncells"]
    for s, sp in enumerate(e["species"]):
        n = int(n_per_species[s] if hasattr(n_per_species, "__len__") else n_per_species)
        lo, hi = cell_range if cell_range is not None else (0, N)
        cell = rng.integers(lo, hi, size=n).astype(np.int32)
        off = rng.random(n, dtype=np.float32)
        off = np.minimum(off, np.float32(1.0) - np.float32(2.0 ** -24))
        if sort_by_cell:
            order = np.argsort(cell, kind="stable")
            cell, off = cell[order], off[order]
        vth = math.sqrt(sp["T"] / sp["m"]) if vscale is None else vscale[s]
        v = (rng.standard_normal((3, n)) * vth).astype(np.float32)
        ids = rng.permutation(n).astype(np.uint32) if shuffle_ids else np.arange(n, dtype=np.uint32)
        x = (cell.astype(np.float64) + off.astype(np.float64)) * e["dx"]
        out.append({"cell": cell, "off": off, "x": x, "vx": v[0].copy(), "vy": v[1].copy(),
                    "vz": v[2].copy(), "id": ids, "next_id": n})
    return out


def random_field(e, seed=0, amp=0.5):
    """A smooth random node field (binary32-exact values stored as float64)."""
    rng = np.random.default_rng(seed)
    nn = e["ncells"] if e["periodic"] else e["ncells"] + 1
    k = rng.integers(1, 6)
    j = np.arange(nn)
    E = amp * np.sin(2 * np.pi * k * j / max(nn - 1, 1) + rng.random()) + 0.1 * amp * rng.standard_normal(nn)
    return E.astype(np.float32).astype(np.float64)


def quiet_start_state(e):
    """Cold quiet start of one species with a sinusoidal displacement: x0 = (p + 1/2) L / P
    moved by (A / k) sin(k x0), k = 2 pi mode / L, rounded to a binary32 in-cell offset so
    both precisions hold the same positions.  Velocities zero."""
    N, dx = e["ncells"], e["dx"]
    sp = e["species"][0]
    P = sp["ppc"] * N
    L = N * dx
    k = 2 * math.pi * e["perturb_mode"] / L
    x0 = (np.arange(P) + 0.5) * L / P
    x = x0 + (e["perturb_amp"] / k) * np.sin(k * x0)
    x = np.where(x < 0, x + L, x)
    x = np.where(x >= L, x - L, x)
    g = x / dx
    cell = np.floor(g).astype(np.int64)
    off = (g - cell).astype(np.float32).astype(np.float64)
    bump = off >= 1.0
    off[bump] = 0.0
    cell[bump] += 1
    cell[cell >= N] -= N
    z = np.zeros(P)
    return [{"x": (cell + off) * dx, "vx": z.copy(), "vy": z.copy(), "vz": z.copy(),
             "id": np.arange(P, dtype=np.uint32), "next_id": P}]


def rademacher(n, seed=0):
    return np.random.default_rng(seed).choice([-1.0, 1.0], size=n)
