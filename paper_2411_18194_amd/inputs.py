"""Seeded synthetic inputs for the micromagnetic hot path.

This module builds problem descriptions (grid, material parameters, initial
states, request streams) from a seed.  It holds none of the method's
arithmetic: no field term, torque, demagnetising tensor or time step lives
here.  Both the HIP library's tests/bench and the FP64 oracle's tests take
their inputs from it, so the two sides always see identical arrays.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws in a
fixed, documented order, so a seed fully determines the arrays.

Problem description (a plain ``dict``, SI units throughout):

``n``          (nx, ny, nz) cell counts
``cell``       (dx, dy, dz) cell size in metres
``nsub``       1 (ferromagnet), 2 (two-sublattice antiferro/ferrimagnet) or 3
``gamma``      gyromagnetic ratio, rad/(s T)
per-sublattice lists (length ``nsub``):
  ``Ms`` (A/m), ``A11`` (J/m), ``alpha``, ``Ku1``/``Ku2`` (J/m^3),
  ``anis_u`` (unit 3-vectors), ``Kc1`` (J/m^3), ``cub_c1``/``cub_c2``,
  ``Dint`` (J/m^2, interfacial DMI), ``B1``/``B2`` (J/m^3),
  ``zl_P`` (spin polarisation), ``zl_xi`` (non-adiabaticity)
shared scalars: ``A0`` (homogeneous inter-sublattice exchange, J/m),
  ``A12`` (inhomogeneous inter-sublattice exchange, J/m), ``latcon`` (m),
  ``B_ext`` (T, 3-vector), ``j`` (A/m^2, 3-vector), ``demag`` (bool)
optional per-cell data:
  ``dmi_layer``  int or None: when set, the interfacial DMI acts only in
                 the z-layer with that index (0 = bottom layer)
  ``grain``      uint16 array (nz, ny, nx) of grain ids, with
  ``grain_axes`` float array (ngrains, 3) of uniaxial easy axes; when
                 present these replace ``anis_u`` for every sublattice
``elastic``    None or dict(rho, C11, C12, C44, eta, trac_amp, trac_freq)
               with a shear traction sigma_xz = trac_amp*sin(2 pi f t) on
               the x = 0 face and traction-free faces elsewhere
"""
from __future__ import annotations

import math

import numpy as np

MU_B = 9.2740100783e-24  # J/T (CODATA 2018), used only to document configs
GAMMA = 1.7595e11         # rad/(s T)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def base_params(n, cell, nsub=1):
    """A problem with every interaction switched off."""
    z3 = (0.0, 0.0, 0.0)
    return {
        "n": tuple(int(v) for v in n),
        "cell": tuple(float(v) for v in cell),
        "nsub": int(nsub),
        "gamma": GAMMA,
        "Ms": [0.0] * nsub,
        "A11": [0.0] * nsub,
        "alpha": [0.0] * nsub,
        "Ku1": [0.0] * nsub,
        "Ku2": [0.0] * nsub,
        "anis_u": [(0.0, 0.0, 1.0)] * nsub,
        "Kc1": [0.0] * nsub,
        "cub_c1": [(1.0, 0.0, 0.0)] * nsub,
        "cub_c2": [(0.0, 1.0, 0.0)] * nsub,
        "Dint": [0.0] * nsub,
        "B1": [0.0] * nsub,
        "B2": [0.0] * nsub,
        "zl_P": [0.0] * nsub,
        "zl_xi": [0.0] * nsub,
        "A0": 0.0,
        "A12": 0.0,
        "latcon": 0.35e-9,
        "B_ext": z3,
        "j": z3,
        "demag": False,
        "dmi_layer": None,
        "grain": None,
        "grain_axes": None,
        "elastic": None,
        "solver": "dp45",
        "pbc": (0, 0, 0),
        "dmi_homo": (0.0, 0.0, 0.0),
        "bc": "open",
        "dmi_W": None,
        "dmi_W12": None,
        "grain_exchange_scale": 1.0,
    }


# ---------------------------------------------------------------- states --

def random_unit(g: np.random.Generator, nsub, n):
    """Unit vectors uniform on the sphere: normalised N(0,1)^3 per cell."""
    nx, ny, nz = n
    v = g.standard_normal((nsub, 3, nz, ny, nx))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def gaussian_smooth(field, sigma=3.0, trunc=9):
    """Separable, non-periodic Gaussian blur over the last three axes.

    Taps exp(-k^2/(2 sigma^2)) for |k| <= trunc; near an edge only the taps
    that fall inside the grid are used and their weights are renormalised.
    """
    k = np.arange(-trunc, trunc + 1)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    out = np.asarray(field, dtype=np.float64)
    for axis in (-1, -2, -3):
        n = out.shape[axis]
        acc = np.zeros_like(out)
        wsum = np.zeros(n)
        for off, wk in zip(k, w):
            lo, hi = max(0, -off), min(n, n - off)
            if lo >= hi:
                continue
            dst = [slice(None)] * out.ndim
            src = [slice(None)] * out.ndim
            dst[axis] = slice(lo, hi)
            src[axis] = slice(lo + off, hi + off)
            acc[tuple(dst)] += wk * out[tuple(src)]
            wsum[lo:hi] += wk
        shape = [1] * out.ndim
        shape[axis] = n
        out = acc / wsum.reshape(shape)
    return out


def smoothed_random_unit(g, nsub, n, sigma=3.0, trunc=9):
    """i.i.d. N(0,1) per component and cell, Gaussian-smoothed, normalised."""
    nx, ny, nz = n
    v = g.standard_normal((nsub, 3, nz, ny, nx))
    v = gaussian_smooth(v, sigma, trunc)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def normalise(m):
    return m / np.linalg.norm(m, axis=1, keepdims=True)


# --------------------------------------------------------------- configs --

def config_c1(seed=1):
    """Thin permalloy-like film (standard-problem-4 geometry), FP64, CPU scale.

    64x16x1 cells of 7.8125x7.8125x3 nm, demag + exchange, field
    (-24.6, 4.3, 0) mT.  Initial m uniform on the sphere per cell; the run
    protocol relaxes it with alpha = 1 and no field first.
    """
    p = base_params((64, 16, 1), (7.8125e-9, 7.8125e-9, 3e-9))
    p.update(Ms=[8.0e5], A11=[1.3e-11], alpha=[0.02], demag=True,
             B_ext=(-24.6e-3, 4.3e-3, 0.0))
    m0 = random_unit(rng(seed), 1, p["n"])
    return p, m0


def config_c2(seed=2, n=(512, 512, 16)):
    """Perpendicular film with an interfacial-DMI bottom layer, 2 nm cubes."""
    p = base_params(n, (2e-9, 2e-9, 2e-9))
    p.update(Ms=[1.1e6], A11=[1.5e-11], alpha=[0.1], Ku1=[5e5],
             anis_u=[(0.0, 0.0, 1.0)], Dint=[3e-3], dmi_layer=0,
             B_ext=(0.0, 0.0, 0.05), demag=True)
    m0 = smoothed_random_unit(rng(seed), 1, p["n"])
    return p, m0


C2_CROP = ((224, 288), (224, 288), (0, 4))  # x, y, z cell ranges


def config_c2_crop(seed=2):
    """64x64x4 system cut from the 512x512x16 initial state (own demag)."""
    p, m0 = config_c2(seed)
    (x0, x1), (y0, y1), (z0, z1) = C2_CROP
    pc = dict(p)
    pc["n"] = (x1 - x0, y1 - y0, z1 - z0)
    return pc, np.ascontiguousarray(m0[:, :, z0:z1, y0:y1, x0:x1])


def c2_fixed_dt():
    """Fixed step giving 1667 DP45 steps (~10,002 evaluations) in 0.1 ns."""
    return 0.1e-9 / 1667


def voronoi_grains(g, n, cell, ngrains):
    """Nearest-seed grain map; seeds uniform in the film rectangle.

    Ties go to the lower seed index (argmin order).  Returns (grain ids
    (nz, ny, nx) uint16, seeds (ngrains, 2) in metres).
    """
    nx, ny, nz = n
    dx, dy, _ = cell
    seeds = g.uniform(0.0, 1.0, (ngrains, 2)) * np.array([nx * dx, ny * dy])
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    d2 = ((xc[None, None, :] - seeds[:, 0, None, None]) ** 2
          + (yc[None, :, None] - seeds[:, 1, None, None]) ** 2)
    ids = np.argmin(d2, axis=0).astype(np.uint16)
    return np.broadcast_to(ids, (nz, ny, nx)).copy(), seeds


def config_c3(seed=3, n=(1024, 256, 1)):
    """Polycrystalline two-sublattice antiferromagnet with Zhang-Li current."""
    p = base_params(n, (1e-9, 1e-9, 1e-9), nsub=2)
    p.update(Ms=[4.0e5] * 2, A11=[1e-11] * 2, alpha=[0.01] * 2,
             Ku1=[6e4] * 2, A0=-2.5e-11, A12=-5e-12, latcon=0.35e-9,
             zl_P=[0.5] * 2, zl_xi=[0.1] * 2, j=(1e12, 0.0, 0.0),
             demag=False)
    g = rng(seed)
    ids, _ = voronoi_grains(g, p["n"], p["cell"], 40)
    axes = g.standard_normal((40, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    p["grain"], p["grain_axes"] = ids, axes
    nx, ny, nz = p["n"]
    x = (np.arange(nx) + 0.5) * p["cell"][0]
    delta = math.sqrt(1e-11 / 6e4)
    th = 2.0 * np.arctan(np.exp((x - 512e-9) / delta))
    l = np.zeros((3, nz, ny, nx))
    l[0] = np.sin(th)[None, None, :]
    l[2] = np.cos(th)[None, None, :]
    m = np.stack([l, -l])
    m = m + 1e-3 * g.standard_normal(m.shape)
    return p, normalise(m)


def config_c3_crop(seed=3):
    """128x64 window at x in [448, 576) nm, y in [0, 64) nm of config c3."""
    p, m0 = config_c3(seed)
    pc = dict(p)
    pc["n"] = (128, 64, 1)
    pc["grain"] = np.ascontiguousarray(p["grain"][:, 0:64, 448:576])
    return pc, np.ascontiguousarray(m0[:, :, :, 0:64, 448:576])


def config_c4(seed=4, n=(2048, 64, 1)):
    """NiO-like magnetoelastic two-sublattice racetrack with a shear drive."""
    p = base_params(n, (2e-9, 2e-9, 2e-9), nsub=2)
    C44 = 1.1e11
    p.update(Ms=[4.2e5] * 2, A11=[4.4e-12] * 2, alpha=[2.1e-4] * 2,
             Kc1=[-2e3] * 2, B1=[-6.3e6] * 2, B2=[-6.3e6] * 2,
             A0=-4.6e-11, A12=0.0, latcon=0.42e-9, demag=False,
             elastic=dict(rho=6800.0, C11=3.2e11, C12=1.3e11, C44=C44,
                          eta=1e12, trac_amp=2.0 * C44 * 1e-3,
                          trac_freq=2e9))
    g = rng(seed)
    nx, ny, nz = p["n"]
    l = np.zeros((3, nz, ny, nx))
    l[:] = (1.0 / math.sqrt(3.0))
    m = np.stack([l, -l])
    m = m + 1e-3 * g.standard_normal(m.shape)
    return p, normalise(m)


def config_c4_crop(seed=4):
    """256x64 window at the x = 0 end of config c4 (keeps the drive face)."""
    p, m0 = config_c4(seed)
    pc = dict(p)
    pc["n"] = (256, 64, 1)
    return pc, np.ascontiguousarray(m0[:, :, :, :, 0:256])


C4_FIXED_DT = 1e-14


def request_stream(seed=5, count=4000, rate=200.0):
    """Poisson stream of relaxation requests of mixed size and kind.

    Draw order per request: inter-arrival, nx, ny, nz, cell, kind, six
    parameter scales, then the request's own state seed.  Returns a list of
    dicts with ``t_arrive`` (s), ``params``, ``state_seed`` and ``t_relax``.
    """
    g = rng(seed)
    out = []
    t = 0.0
    for _ in range(count):
        t += g.exponential(1.0 / rate)
        nx = int(round(math.exp(g.uniform(math.log(32), math.log(512)))))
        ny = int(round(math.exp(g.uniform(math.log(32), math.log(512)))))
        nz = int(round(math.exp(g.uniform(0.0, math.log(8)))))
        d = g.uniform(1e-9, 5e-9)
        fm = g.uniform() < 0.7
        s = g.uniform(0.7, 1.3, 6)
        state_seed = int(g.integers(0, 2**31 - 1))
        if fm:
            p = base_params((nx, ny, nz), (d, d, d))
            p.update(Ms=[1.1e6 * s[0]], A11=[1.5e-11 * s[1]],
                     Ku1=[5e5 * s[2]], Dint=[3e-3 * s[3]], dmi_layer=0,
                     alpha=[0.1 * s[4]], B_ext=(0.0, 0.0, 0.05 * s[5]),
                     demag=True)
        else:
            p = base_params((nx, ny, nz), (d, d, d), nsub=2)
            p.update(Ms=[4e5 * s[0]] * 2, A11=[1e-11 * s[1]] * 2,
                     A0=-2.5e-11 * s[2], A12=-5e-12 * s[3],
                     alpha=[0.01 * s[4]] * 2, Ku1=[6e4 * s[5]] * 2,
                     latcon=0.35e-9, demag=False)
        out.append(dict(t_arrive=t, params=p, state_seed=state_seed,
                        t_relax=0.5e-9, tol=1e-5))
    return out


def request_state(req):
    """Initial state of a request: smoothed random field (m2 = -m1 for AFM)."""
    p = req["params"]
    m = smoothed_random_unit(rng(req["state_seed"]), 1, p["n"])
    if p["nsub"] == 2:
        m = np.concatenate([m, -m])
    return m
