"""Seeded synthetic workloads for the porous-convection lattice Boltzmann step.

This module holds workload recipes (geometry, parameters, wall rules, seeds)
and seeded random population states.  It contains none of the method's
arithmetic: no equilibria, no matrices, no parameter mapping.  Both the
product library's binding and the FP64 oracle receive the same plain dict.

The workloads stand in for the paper's own test problems (there is no dataset):
the cubic porous cavity of Sec. 4.2 (hot and cold x-walls, adiabatic side
walls, buoyancy along z) and channels like those of Sec. 4.1.
"""
from __future__ import annotations

import numpy as np


def face(flow: str, heat: str, T_wall: float = 0.0, u_wall=(0.0, 0.0, 0.0)) -> dict:
    return {"flow": flow, "heat": heat, "T_wall": float(T_wall),
            "u_wall": tuple(float(v) for v in u_wall)}


def cavity(n, *, lattice=19, porosity=0.6, darcy=1e-2, rayleigh=1e4, prandtl=1.0,
           seed=1, noise_amp=1e-3, T_hot=0.5, T_cold=-0.5, forchheimer=1.0,
           mach=0.1, **extra) -> dict:
    """Natural convection in a porous box: isothermal -x (hot) and +x (cold)
    walls, the other four adiabatic, bounce-back everywhere, buoyancy along +z.
    Initial state: rest, T linear between the walls plus seeded uniform noise.
    ``n`` is an edge length or an (nx, ny, nz) tuple; L = nx."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    wl = {
        "nx": int(nx), "ny": int(ny), "nz": int(nz), "q": int(lattice),
        "porosity": float(porosity), "darcy": float(darcy),
        "rayleigh": float(rayleigh), "prandtl": float(prandtl),
        "mach": float(mach), "forchheimer": float(forchheimer),
        "gravity_axis": 2, "length_axis": 0,
        "T_ref": 0.5 * (T_hot + T_cold), "delta_T": float(T_hot - T_cold),
        "faces": [face("wall", "isothermal", T_hot), face("wall", "isothermal", T_cold),
                  face("wall", "adiabatic"), face("wall", "adiabatic"),
                  face("wall", "adiabatic"), face("wall", "adiabatic")],
        "init_axis": 0, "init_T_lo": float(T_hot), "init_T_hi": float(T_cold),
        "seed": int(seed), "noise_amp": float(noise_amp),
    }
    wl.update(extra)
    return wl


def config_cavity_fp64() -> dict:
    """32^3 porous cavity, D3Q19 + D3Q7, FP64: phi 0.6, Da 1e-2, Ra 1e4, Pr 1,
    2000 steps, seed 1."""
    wl = cavity(32, porosity=0.6, darcy=1e-2, rayleigh=1e4, prandtl=1.0, seed=1)
    wl.update(name="cavity32_fp64", precision="fp64", steps=2000)
    return wl


def config_cavity_fp32() -> dict:
    """256^3 porous cavity, D3Q19 + D3Q7, FP32: phi 0.4, Da 1e-4, Ra 1e6, Pr 1,
    seed 2 (20000 steps in the full run)."""
    wl = cavity(256, porosity=0.4, darcy=1e-4, rayleigh=1e6, prandtl=1.0, seed=2)
    wl.update(name="cavity256_fp32", precision="fp32", steps=20000)
    return wl


def periodic_box(shape, *, lattice=19, **extra) -> dict:
    """Fully periodic box with default Sec. 4 rates (no walls)."""
    nx, ny, nz = shape
    wl = {
        "nx": nx, "ny": ny, "nz": nz, "q": lattice,
        "porosity": 0.7, "darcy": 1e-2, "rayleigh": 1e4, "prandtl": 1.0,
        "gravity_axis": 2, "length_axis": 0, "T_ref": 0.0, "delta_T": 1.0,
        "faces": [face("periodic", "periodic")] * 6,
        "init_axis": -1, "seed": 7, "noise_amp": 1e-2,
    }
    wl.update(extra)
    return wl


def random_state(q: int, shape, seed: int, *, f_base=None, amp=0.05, T_amp=0.5):
    """Seeded random pre-collision populations.  f_i = base * (1 + amp U(-1,1)),
    g_k = (T_amp U(-1,1)) / 7 + small noise.  The values are arbitrary positive
    (f) or signed (g) numbers, not equilibria; ``f_base`` defaults to 1/q."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    base = (1.0 / q) if f_base is None else f_base
    f = base * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(q, nz, ny, nx)))
    T = T_amp * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    g = np.broadcast_to(T / 7.0, (7, nz, ny, nx)) * (1.0 + amp * rng.uniform(
        -1.0, 1.0, size=(7, nz, ny, nx)))
    return np.ascontiguousarray(f), np.ascontiguousarray(g)


def channel(shape, *, lattice=15, porosity=0.7, darcy=1e-3, reynolds=10.0, rayleigh=1e5,
            prandtl=1.0, u_in=0.05, seed=3, noise_amp=1e-3, T_hot=0.5, T_cold=-0.5,
            forchheimer=1.0, **extra) -> dict:
    """Mixed convection in a porous channel (the setting of Sec. 4.1, here with a
    throughflow): plug inflow u_in through the -x face (moving-wall bounce-back,
    inlet temperature T_ref), open outlet at +x, heated bottom wall (-y, T_hot)
    and cooled top wall (+y, T_cold), periodic in z, buoyancy along +y.
    Re = u_in H / nu with H = ny.  Initial state: plug flow, T linear in y plus
    seeded uniform noise."""
    nx, ny, nz = shape
    T_ref = 0.5 * (T_hot + T_cold)
    wl = {
        "nx": int(nx), "ny": int(ny), "nz": int(nz), "q": int(lattice),
        "porosity": float(porosity), "darcy": float(darcy), "rayleigh": float(rayleigh),
        "prandtl": float(prandtl), "reynolds": float(reynolds), "u_char": float(u_in),
        "forchheimer": float(forchheimer), "gravity_axis": 1, "length_axis": 1,
        "T_ref": T_ref, "delta_T": float(T_hot - T_cold),
        "faces": [face("wall", "isothermal", T_ref, (u_in, 0.0, 0.0)), face("outlet", "outflow"),
                  face("wall", "isothermal", T_hot), face("wall", "isothermal", T_cold),
                  face("periodic", "periodic"), face("periodic", "periodic")],
        "init_axis": 1, "init_T_lo": float(T_hot), "init_T_hi": float(T_cold),
        "seed": int(seed), "noise_amp": float(noise_amp), "init_u": (float(u_in), 0.0, 0.0),
    }
    wl.update(extra)
    return wl


def config_channel(downscale: bool = False) -> dict:
    """Porous channel 512x128x128 (or its 128x32x32 downscale), D3Q15 + D3Q7:
    phi 0.7, Da 1e-3, Re 10, Ra 1e5, inlet 0.05, seed 3."""
    shape = (128, 32, 32) if downscale else (512, 128, 128)
    wl = channel(shape)
    wl.update(name="channel%dx%dx%d" % shape)
    return wl


def _cavity_draw(rng, edge: int, index: int, seed: int) -> dict:
    """One cavity of the batched and served workloads: porosity U[0.3, 0.9],
    Da log-uniform in [1e-5, 1e-1], Ra log-uniform in [1e3, 1e6], Pr 1."""
    phi = float(rng.uniform(0.3, 0.9))
    da = float(10.0 ** rng.uniform(-5.0, -1.0))
    ra = float(10.0 ** rng.uniform(3.0, 6.0))
    wl = cavity(int(edge), porosity=phi, darcy=da, rayleigh=ra, prandtl=1.0, seed=seed * 1000 + index)
    wl["name"] = f"cavity{edge}_phi{phi:.3f}_Da{da:.2e}_Ra{ra:.2e}"
    return wl


def config_batch(count: int = 64, seed: int = 4) -> list:
    """Independent porous cubic cavities with edge length drawn uniformly from
    {32, 48, 64, 96, 128} and parameters drawn as in ``_cavity_draw``."""
    rng = np.random.default_rng(seed)
    edges = rng.choice(np.array([32, 48, 64, 96, 128]), size=count)
    return [_cavity_draw(rng, int(e), i, seed) for i, e in enumerate(edges)]


def config_serving(count: int = 64, rate: float = 20.0, seed: int = 5, edge_range=(48, 192)) -> list:
    """A Poisson stream of cavity solve requests: exponential inter-arrival
    times of mean 1/rate seconds, edge length log-uniform in edge_range
    (rounded to an integer), parameters as in ``_cavity_draw``.  Returns
    (arrival_seconds, workload) pairs in arrival order."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    lo, hi = np.log(edge_range[0]), np.log(edge_range[1])
    edges = np.rint(np.exp(rng.uniform(lo, hi, size=count))).astype(int)
    return [(float(t[i]), _cavity_draw(rng, int(edges[i]), i, seed)) for i in range(count)]


def melting(nx: int = 400, ny: int = 6, nz: int = 6, *, alpha_ratio: float = 1.0, alpha_s: float = 0.02,
            stefan: float = 1.0, T_hot: float = 1.0, T_melt: float = 0.0, T_init: float = -1.0,
            porosity: float = 1.0, c_pl: float = 1.0, c_ps: float = 1.0, matrix_heat: float = 0.0,
            varpi: float = 0.5, mushy: float = 0.0) -> dict:
    """Two-region conduction melting in a semi-infinite slab (the setting of
    Sec. 4.3): solid at T_init, the -x wall held at T_hot > T_melt from t = 0,
    the +x wall at T_init, periodic in y and z, no flow.  alpha_l =
    alpha_ratio * alpha_s; latent heat from the Stefan number St = c_pl (T_hot
    - T_melt) / L_a.  ``mushy`` > 0 spreads melting over [T_melt, T_melt +
    mushy]."""
    return {
        "name": f"melting{nx}x{ny}x{nz}_ratio{alpha_ratio:g}", "energy": "enthalpy",
        "nx": int(nx), "ny": int(ny), "nz": int(nz), "varpi": float(varpi), "porosity": float(porosity),
        "c_pl": float(c_pl), "c_ps": float(c_ps), "matrix_heat": float(matrix_heat),
        "latent": float(c_pl * (T_hot - T_melt) / stefan), "T_solidus": float(T_melt),
        "T_liquidus": float(T_melt + mushy), "alpha_l": float(alpha_ratio * alpha_s), "alpha_s": float(alpha_s),
        "zeta_e": 1.2, "zeta_nu": 1.2, "T_init": float(T_init),
        "faces": [face("wall", "isothermal", T_hot), face("wall", "isothermal", T_init),
                  face("periodic", "periodic"), face("periodic", "periodic"),
                  face("periodic", "periodic"), face("periodic", "periodic")],
    }
