"""Seeded synthetic workloads for the multiscale two-component D3Q19 model.

This module only *generates inputs*: voxel classes, porosity, pore types,
constitutive tables and initial densities, plus the plain configuration
constants of each workload.  It contains none of the lattice-Boltzmann
arithmetic (no streaming, collision, forces, table lookups or setup of the
per-voxel constitutive data); both the CPU oracle and the GPU library consume
what it returns.

Voxel classes (paper, Sec. I workflow and Fig. 1): PORE (resolved fluid,
porosity 1), SOLID, GRAY (under-resolved porous medium, 0 < phi < 1).

Workloads:

* ``droplet_slab``      32^3 periodic water droplet (R = 8) in oil with a
                        32x32x8 gray slab of phi = 0.3, FP64, 200 steps.
* ``multiscale_rock``   n^3 Gaussian-random-field rock: 35 % solid, 20 % gray,
                        45 % pore; four Brooks-Corey pore types; water driven
                        in +x from an 8-voxel inlet buffer.  n = 256 is the
                        full-size case, smaller n give the parity minis.
* ``fiber_bundles``     n^3 domain of straight gray cylinders (fiber bundles)
                        in open pore space, single component, tensorial
                        resistivity with anisotropy ratio 10.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

PORE, SOLID, GRAY = 0, 1, 2
TABLE_N = 1025  # samples on [0, 1] for every constitutive curve


# --------------------------------------------------------------------------
# configuration constants
# --------------------------------------------------------------------------
# Bulk minority/majority density ratio of the flat-interface equilibrium of the
# two-component pseudo-potential model at G = 3 (tau = 1, exact-difference
# forcing per component).  It is a configuration constant that fixes the
# saturation normalisation (s_min, s_max), the oil wall potential and phi_avg;
# tests/golden/make_coexistence.py derives it with the CPU oracle and a test
# checks it against a fresh flat-interface run.
COEXISTENCE_RATIO = {3.0: 0.0029912221254390597}

# CSF coefficients kappa of Eq. (4) that scale the surface tension of the
# G = 3 model to 0.5 and 2 times its kappa = 0 value (static quasi-2D droplet,
# R = 7, Laplace's law, as in Sec. III.A); tests/golden/make_kappa.py derives
# them with the CPU oracle and a test re-checks them.
KAPPA_SIGMA_SCALE = {0.5: -0.09562777169572569, 2.0: 0.17510806844983903}


def minority_density(G: float) -> float:
    """Minority density m of a two-component bulk whose majority density is 1."""
    try:
        return COEXISTENCE_RATIO[float(G)]
    except KeyError:
        raise ValueError(f"no coexistence constant for G = {G}; pass m_minor explicitly")


@dataclass
class Params:
    """Model parameters.  Field names are shared with the C ``lbm_params``."""
    nx: int = 32
    ny: int = 32
    nz: int = 32
    ncomp: int = 2
    precision: str = "f64"          # "f64" | "f32" | "f16" | "bf16" (16-bit population storage)
    collision: str = "regularized"  # "regularized" | "bgk"
    tau: tuple = (1.0, 1.0)         # (water, oil)
    G: float = 3.0
    g: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))  # body acceleration per component
    kappa: float = 0.0
    csf_region: str = "gray"        # "gray" | "all"
    phi_max: float = 1.0
    phi_avg: float = 0.0            # filled from m when 0
    m_minor: float = 0.0            # filled from G when 0
    s_min: float = 0.0
    s_max: float = 0.0
    wall_dpsi: tuple = (0.1, -0.1)  # wetting offsets of the solid pseudo-potential (w, o)
    kr_min: float = 1e-4
    c_max: float = 3.5
    c_min: float = 0.575
    hyst: float = 0.05
    eps_n: float = 0.0              # filled by precision when 0
    tensor: bool = False
    sigma_s: float = 1.5
    smooth_radius: int = 5
    eps_g: float = 1e-6
    eps_H: float = 1e-6
    delta_tie: float = 0.05
    outlet_x: int = -1              # -1: nx - 1 (periodic) or nx - 2 (pressure boundaries)
    diag_every: int = 0
    bc_x: str = "periodic"          # "periodic" | "pressure" (reservoirs) | "density" (exact density faces)
    rho_in: tuple = (1.0, 0.0)      # reservoir densities (water, oil) beyond x = 0
    rho_out: tuple = (1.0, 0.0)     # reservoir densities (water, oil) beyond x = nx - 1
    layout: str = "auto"            # population storage: "auto" (fluid-only where supported) | "dense"

    def filled(self) -> "Params":
        p = Params(**asdict(self))
        if p.m_minor == 0.0:
            p.m_minor = minority_density(p.G) if p.ncomp == 2 else 0.0
        m = p.m_minor
        if p.s_min == 0.0 and p.s_max == 0.0:
            p.s_min = m / (1.0 + m)
            p.s_max = 1.0 / (1.0 + m)
        if p.phi_avg == 0.0:
            p.phi_avg = 0.5 * (1.0 + m)
        if p.eps_n == 0.0:
            p.eps_n = 1e-12 if p.precision == "f64" else 1e-7
        if p.outlet_x < 0:
            p.outlet_x = p.nx - 2 if p.bc_x != "periodic" else p.nx - 1
        p.tau = tuple(float(t) for t in p.tau)
        p.rho_in = tuple(float(v) for v in p.rho_in)
        p.rho_out = tuple(float(v) for v in p.rho_out)
        p.g = tuple(tuple(float(v) for v in gg) for gg in p.g)
        return p

    def as_dict(self) -> dict:
        return asdict(self)


# --------------------------------------------------------------------------
# constitutive tables (inputs: the paper's library of K0(phi), Pc(S), Kr(S))
# --------------------------------------------------------------------------
def _grid() -> np.ndarray:
    return np.arange(TABLE_N, dtype=np.float64) / (TABLE_N - 1)


def kozeny_carman_table(d: float = 2.0, phi_hold: float = 0.95) -> np.ndarray:
    """K0(phi) = phi^3 / (1 - phi)^2 * d^2 / 180 sampled on phi = k/1024.
    Samples above ``phi_hold`` repeat the value at ``phi_hold`` (the form
    diverges at phi -> 1; gray porosity never exceeds 0.95 here)."""
    ph = np.minimum(_grid(), phi_hold)
    return ph ** 3 / (1.0 - ph) ** 2 * d * d / 180.0


def brooks_corey_tables(pc_e: float, lam: float, swr: float, cap: float = 10.0):
    """Pc(S) = pc_e * Se^(-1/lam) capped at cap*pc_e, Krw = Se^3,
    Kro = (1 - Se)^3, Se = clamp((S - swr) / (1 - swr), 0, 1)."""
    s = _grid()
    se = np.clip((s - swr) / (1.0 - swr), 0.0, 1.0)
    with np.errstate(divide="ignore", over="ignore"):
        pc = np.where(se > 0.0, pc_e * np.power(np.maximum(se, 1e-300), -1.0 / lam), np.inf)
    pc = np.minimum(pc, cap * pc_e)
    return pc, se ** 3, (1.0 - se) ** 3


def pore_table(K0, Pc, Krw, Kro, phi_ref: float, pc_pm: float, kd=(1.0, 1.0, 1.0)) -> dict:
    return dict(K0=np.asarray(K0, np.float64), Pc=np.asarray(Pc, np.float64),
                Krw=np.asarray(Krw, np.float64), Kro=np.asarray(Kro, np.float64),
                phi_ref=float(phi_ref), Pc_PM=float(pc_pm), kd=tuple(float(v) for v in kd))


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------
def _coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def gaussian_random_field(n: tuple, corr_len: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field: N(0,1) white noise filtered in Fourier
    space with a Gaussian of std corr_len/sqrt(2) (covariance
    exp(-r^2 / (2 corr_len^2)))."""
    nz, ny, nx = n
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    s = corr_len / math.sqrt(2.0)
    kz = 2 * np.pi * np.fft.fftfreq(nz)[:, None, None]
    ky = 2 * np.pi * np.fft.fftfreq(ny)[None, :, None]
    kx = 2 * np.pi * np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
    return np.fft.irfftn(np.fft.rfftn(w) * filt, s=(nz, ny, nx), axes=(0, 1, 2))


def two_phase_densities(water: np.ndarray, m: float):
    rw = np.where(water, 1.0, m)
    ro = np.where(water, m, 1.0)
    return rw.astype(np.float64), ro.astype(np.float64)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def droplet_slab(seed: int = 1001, n: int = 32, radius: float = 8.0, slab: int = 8,
                 kappa: float = -0.045, precision: str = "f64") -> dict:
    """32^3 periodic two-component case: water droplet of radius 8 at a seeded
    uniform random centre in oil; a 32x32x8 gray slab (z < 8) with phi = 0.3;
    one pore type (Kozeny-Carman d = 2, Brooks-Corey Pc = 0.05 Se^-0.5,
    Corey cubic Kr, Swr = 0.1); G = 3, tau = 1 for both components, CSF
    coefficient -0.045 in gray voxels, no body force, 200 steps."""
    p = Params(nx=n, ny=n, nz=n, ncomp=2, precision=precision, tau=(1.0, 1.0), G=3.0,
               kappa=kappa).filled()
    m = p.m_minor
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, n, size=3)
    x, y, z = _coords(n, n, n)
    d = [x - c[0], y - c[1], z - c[2]]
    d = [v - n * np.round(v / n) for v in d]  # minimum image
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    rw = m + (1.0 - m) * 0.5 * (1.0 - np.tanh((r - radius) / 1.5))
    ro = 1.0 + m - rw
    cls = np.full((n, n, n), PORE, np.uint8)
    cls[:slab] = GRAY
    phi = np.where(cls == GRAY, 0.3, 1.0)
    ptype = np.zeros((n, n, n), np.uint8)
    pc, krw, kro = brooks_corey_tables(0.05, 2.0, 0.1)
    tab = pore_table(kozeny_carman_table(2.0), pc, krw, kro, phi_ref=0.3, pc_pm=0.05)
    return dict(name="droplet_slab", params=p, cls=cls, phi=phi, ptype=ptype, tables=[tab],
                rho_w=rw, rho_o=ro, steps=200)


def multiscale_rock(n: int = 256, seed: int = 2001, precision: str = "f32",
                    sigma_scale: float = 0.5, kappa: float = None, buffer: int = 8,
                    margin: int = 6, gw: float = 1e-5, pc_e: float = 0.05,
                    tau: tuple = (1.0, 1.5), edge: float = 1.5,
                    phi_range: tuple = (0.05, 0.4)) -> dict:
    """n^3 synthetic multiscale rock: Gaussian random field (correlation length
    6 voxels) thresholded at its quantiles into 35 % solid, 20 % gray (grain
    rims) and 45 % pore; gray phi ~ U[0.05, 0.4]; pore type ~ U{0..3} with
    Brooks-Corey lambda in {0.5, 1, 2, 3} (Pc_e = 0.05, Swr = 0.1, Corey
    cubic Kr, Kozeny-Carman d = 2, phi_ref = 0.225).  A pore buffer of
    buffer + margin planes at the inlet and margin planes at the outlet (the
    x-periodic wrap joins them; margin at most n/8, none when buffer = 0);
    the first `buffer` planes start as water (tanh edge), the rest as oil; body
    acceleration gw on water along +x; tau_w = 1.0, tau_o = 1.5 (viscosity
    ratio 1:2; at 1:5 the run does not stay valid: tau_w = 0.6 drives the
    minority densities negative in the pores, tau_o = 3 turns the state
    non-finite within a few hundred steps); G = 3.  With a buffer of the 8
    water planes alone (margin 0), the 256^3 rock went non-finite near step
    1750 where the displacement front met the grains next to the inlet; the
    margins keep it finite over 2000 steps in fp32 and fp64.  Surface-tension
    control in the gray voxels at sigma_scale (0.5 or 2) times the kappa = 0
    surface tension, unless kappa is given."""
    if kappa is None:
        kappa = KAPPA_SIGMA_SCALE[float(sigma_scale)]
    p = Params(nx=n, ny=n, nz=n, ncomp=2, precision=precision, tau=tuple(tau), G=3.0,
               g=((gw, 0.0, 0.0), (0.0, 0.0, 0.0)), kappa=kappa).filled()
    f = gaussian_random_field((n, n, n), 6.0, seed)
    q35, q55 = np.quantile(f, [0.35, 0.55])
    cls = np.full((n, n, n), PORE, np.uint8)
    cls[f < q55] = GRAY
    cls[f < q35] = SOLID
    if buffer > 0:
        mg = min(margin, n // 8)
        cls[:, :, :buffer + mg] = PORE
        if mg:
            cls[:, :, n - mg:] = PORE
    rng_phi = np.random.default_rng(seed + 1)
    rng_pt = np.random.default_rng(seed + 2)
    phi = rng_phi.uniform(phi_range[0], phi_range[1], size=(n, n, n))
    phi = np.where(cls == GRAY, phi, np.where(cls == PORE, 1.0, 0.0))
    ptype = rng_pt.integers(0, 4, size=(n, n, n)).astype(np.uint8)
    ptype = np.where(cls == GRAY, ptype, 0).astype(np.uint8)
    K0 = kozeny_carman_table(2.0)
    tabs = []
    for lam in (0.5, 1.0, 2.0, 3.0):
        pc, krw, kro = brooks_corey_tables(pc_e, lam, 0.1)
        tabs.append(pore_table(K0, pc, krw, kro, phi_ref=0.225, pc_pm=pc_e))
    x, _, _ = _coords(n, n, n)
    # water buffer x < buffer with a tanh edge of width 1.5 (periodic in x)
    c = 0.5 * (buffer - 1)
    d = np.abs(x - c)
    d = np.minimum(d, n - d)
    prof = 0.5 * (1.0 - np.tanh((d - 0.5 * buffer) / edge))
    m = p.m_minor
    rw = m + (1.0 - m) * prof
    ro = 1.0 + m - rw
    return dict(name=f"multiscale_rock_{n}", params=p, cls=cls, phi=phi, ptype=ptype,
                tables=tabs, rho_w=rw, rho_o=ro, steps=2000)


def cylinder_bundles(n: int, ncyl: int, seed: int, rmin=3.0, rmax=6.0):
    """Straight infinite cylinders (random point in the box, direction uniform
    on the sphere, radius ~ U[rmin, rmax]); returns a boolean inside mask and
    the list of (point, unit axis, radius)."""
    rng = np.random.default_rng(seed)
    x, y, z = _coords(n, n, n)
    inside = np.zeros((n, n, n), bool)
    cyl = []
    for _ in range(ncyl):
        p0 = rng.uniform(0.0, n, size=3)
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        r = rng.uniform(rmin, rmax)
        dx, dy, dz = x - p0[0], y - p0[1], z - p0[2]
        t = dx * v[0] + dy * v[1] + dz * v[2]
        d2 = dx * dx + dy * dy + dz * dz - t * t
        inside |= d2 <= r * r
        cyl.append((p0, v, r))
    return inside, cyl


def fiber_bundles(n: int = 192, ncyl: int = 40, seed: int = 3001, precision: str = "f32",
                  direction: int = 0, g: float = 1e-5, kd=(1.0, 0.1, 0.1)) -> dict:
    """n^3 single-component domain of gray fiber bundles: ncyl seeded straight
    cylinders (radius 3-6, random orientation) with phi = clamp(0.3 + 0.1 xi,
    0.05, 0.95), xi ~ U[-1, 1]; pore elsewhere; tau = 1; body acceleration g
    along axis ``direction``; principal permeabilities (1, 0.1, 0.1) K0 with
    the first along the fiber axis; tensorial resistivity on; 1000 steps."""
    gv = [0.0, 0.0, 0.0]
    gv[direction] = g
    p = Params(nx=n, ny=n, nz=n, ncomp=1, precision=precision, tau=(1.0, 1.0), G=0.0,
               g=(tuple(gv), (0.0, 0.0, 0.0)), kappa=0.0, tensor=True).filled()
    inside, _ = cylinder_bundles(n, ncyl, seed)
    rng = np.random.default_rng(seed + 1)
    xi = rng.uniform(-1.0, 1.0, size=(n, n, n))
    cls = np.where(inside, GRAY, PORE).astype(np.uint8)
    phi = np.where(inside, np.clip(0.3 + 0.1 * xi, 0.05, 0.95), 1.0)
    ptype = np.zeros((n, n, n), np.uint8)
    pc, krw, kro = brooks_corey_tables(0.05, 2.0, 0.1)
    tab = pore_table(kozeny_carman_table(2.0), pc, krw, kro, phi_ref=0.3, pc_pm=0.05, kd=kd)
    rho = np.ones((n, n, n))
    return dict(name=f"fiber_bundles_{n}", params=p, cls=cls, phi=phi, ptype=ptype,
                tables=[tab], rho_w=rho, rho_o=np.zeros_like(rho), steps=1000)


def uniform_gray(n=(8, 8, 8), phi=0.3, ncomp=1, tau=1.0, g=(1e-5, 0.0, 0.0), kd=(1.0, 1.0, 1.0),
                 tensor=False, precision="f64", K0_const=None) -> dict:
    """Periodic box filled with one gray medium of uniform porosity (Darcy
    closed-form case)."""
    nz, ny, nx = n
    p = Params(nx=nx, ny=ny, nz=nz, ncomp=ncomp, precision=precision, tau=(tau, tau),
               G=3.0 if ncomp == 2 else 0.0, g=(tuple(g), (0.0, 0.0, 0.0)),
               tensor=tensor).filled()
    cls = np.full(n, GRAY, np.uint8)
    ph = np.full(n, float(phi))
    ptype = np.zeros(n, np.uint8)
    K0 = kozeny_carman_table(2.0) if K0_const is None else np.full(TABLE_N, float(K0_const))
    pc, krw, kro = brooks_corey_tables(0.05, 2.0, 0.1)
    tab = pore_table(K0, pc, krw, kro, phi_ref=phi, pc_pm=0.05, kd=kd)
    rho = np.ones(n)
    return dict(name="uniform_gray", params=p, cls=cls, phi=ph, ptype=ptype, tables=[tab],
                rho_w=rho, rho_o=np.zeros(n) if ncomp == 1 else np.full(n, p.m_minor), steps=0)


WORKLOADS = {"droplet_slab": droplet_slab, "multiscale_rock": multiscale_rock,
             "fiber_bundles": fiber_bundles}


def sphere_pack(shape: tuple, porosity: float, seed: int, rmin: float = 3.0,
                rmax: float = 8.0) -> np.ndarray:
    """Periodic box [z][y][x] of class codes: solid spheres (centre uniform in
    the box, radius ~ U[rmin, rmax], voxel centres at integer coordinates) are
    added, overlapping, until the pore fraction falls to `porosity` or below."""
    nz, ny, nx = shape
    if 2 * math.ceil(rmax) + 2 > min(shape):
        raise ValueError("box too small for the sphere radius")
    rng = np.random.default_rng(seed)
    cls = np.zeros(shape, np.uint8)
    target = (1.0 - porosity) * cls.size
    solid = 0
    while solid < target:
        c = rng.uniform(0.0, 1.0, 3) * np.array([nz, ny, nx])
        r = rng.uniform(rmin, rmax)
        R = int(math.ceil(r))
        idx = [np.arange(int(math.floor(ci)) - R, int(math.floor(ci)) + R + 2) for ci in c]
        dz, dy, dx = np.meshgrid(idx[0] - c[0], idx[1] - c[1], idx[2] - c[2], indexing="ij")
        ball = dz * dz + dy * dy + dx * dx <= r * r
        sel = np.ix_(idx[0] % nz, idx[1] % ny, idx[2] % nx)
        sub = cls[sel]
        solid += int(np.count_nonzero(ball & (sub == PORE)))
        sub[ball] = SOLID
        cls[sel] = sub
    return cls


def rev_domains(count: int = 96, seed: int = 4001, lmin: int = 24, lmax: int = 96,
                phi_range: tuple = (0.20, 0.45), rmin: float = 3.0, rmax: float = 8.0) -> list:
    """The batch of the permeability library: `count` cubic sphere packs, edge
    ~ U{lmin..lmax} and target porosity ~ U[phi_range] (seed), each packed by
    sphere_pack with its own seed.  Returns a list of dicts (cls, edge,
    target porosity)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(lmin, lmax + 1))
        phi = float(rng.uniform(*phi_range))
        out.append(dict(cls=sphere_pack((n, n, n), phi, seed * 1000 + k, rmin, rmax), edge=n,
                        target_porosity=phi))
    return out


def pc_sweep_setup(entry_pc: float = 0.3, membrane_phi: float = 0.3, K0: float = 1.0,
                   levels: tuple = (1.05, 1.12, 1.20, 1.30, 1.42), tau: tuple = (1.0, 1.0),
                   precision: str = "f64") -> dict:
    """Inputs of the capillary-pressure sweep: the two-component model (G = 3,
    water-wet walls, no CSF control), the membrane's pore table (Brooks-Corey
    Pc with entry pressure `entry_pc`, lambda = 2, Swr = 0.05, a constant K0
    so that water leaves through it freely, phi_ref = membrane_phi) and the
    inlet oil density of each of the five levels."""
    model = Params(nx=8, ny=8, nz=8, ncomp=2, precision=precision, tau=tuple(tau), G=3.0).filled()
    pc, krw, kro = brooks_corey_tables(entry_pc, 2.0, 0.05)
    tab = pore_table(np.full(TABLE_N, float(K0)), pc, krw, kro, phi_ref=membrane_phi,
                     pc_pm=entry_pc)
    return dict(model=model, membrane_table=tab, membrane_phi=membrane_phi,
                rho_nw_in=tuple(float(v) for v in levels))


def _flux_misfit(seed: int, steps: int, window: int):
    """(target, loss_grad) of the squared flux misfit over steps >= window:
    Q*(n) = 1.1 mean(q_base over the window) (1 + 0.02 xi_n), xi ~ N(0, 1)
    (seed), and L = sum (Q - Q*)^2 with its gradient."""
    xi = np.random.default_rng(seed).standard_normal(steps)
    inside = np.arange(steps) >= window

    def target(q_base):
        return 1.1 * float(np.mean(np.asarray(q_base)[inside])) * (1.0 + 0.02 * xi)

    def loss_grad(q, tgt):
        d = np.where(inside, np.asarray(q, np.float64) - tgt, 0.0)
        return float(np.sum(d * d)), 2.0 * d

    return target, loss_grad


def adjoint_rock(n: int = 96, seed: int = 5001, precision: str = "f32", steps: int = 800,
                 window: int = 200, tau: float = 1.0, g: float = 1e-5,
                 collision: str = "regularized") -> dict:
    """The porosity-gradient workload: the multiscale-rock geometry generator
    (Gaussian random field, correlation length 6, quantiles 35 % solid, 20 %
    gray, 45 % pore; gray phi ~ U[0.05, 0.4], pore type ~ U{0..3}) on an n^3
    box, run with one component (the fluid the library's adjoint covers) from
    rest at density 1, body acceleration g along +x, tau = 1, outlet at
    x = n / 2.  Loss: L = sum over steps n >= window of
    (Q(n) - Q*(n))^2 with a fixed seeded target: `target(q_base)` returns
    Q*(n) = 1.1 mean(q_base over the window) (1 + 0.02 xi_n), xi ~ N(0, 1)
    (seed + 1), from a base run's history; `loss_grad(q, target)` returns
    (L, dL/dQ)."""
    base = multiscale_rock(n=n, seed=seed, precision=precision, buffer=0)
    p = Params(nx=n, ny=n, nz=n, ncomp=1, precision=precision, tau=(tau, tau), G=0.0,
               collision=collision, g=((g, 0.0, 0.0), (0.0, 0.0, 0.0)),
               kappa=0.0, outlet_x=n // 2).filled()
    target, loss_grad = _flux_misfit(seed + 1, steps, window)
    return dict(name=f"adjoint_rock_{n}", params=p, cls=base["cls"], phi=base["phi"],
                ptype=base["ptype"], tables=base["tables"], rho_w=np.ones((n, n, n)),
                rho_o=None, steps=steps, target=target, loss_grad=loss_grad)



def adjoint_rock2(n: int = 96, seed: int = 5001, precision: str = "f32", steps: int = 800,
                  window: int = 200, kappa: float = None) -> dict:
    """The two-component porosity-gradient workload: the multiscale rock of
    `multiscale_rock` at n^3 (seed), with its CSF control in the gray voxels
    (kappa of the 0.5x surface tension unless given), water buffer and body
    force as there, outlet at x = n / 2; loss L = sum over steps n >= window
    of (Q^w(n) - Q*(n))^2 with a seeded target (`target(q_base)`,
    `loss_grad(q, target)`, as in `adjoint_rock`).  The pore buffer is the 8
    water planes alone (no margins), so that the water meets gray voxels and
    residual transfers fire within the first few hundred steps."""
    base = multiscale_rock(n=n, seed=seed, precision=precision, kappa=kappa, margin=0)
    p = base["params"]
    p.outlet_x = n // 2
    target, loss_grad = _flux_misfit(seed + 1, steps, window)
    return dict(base, name=f"adjoint_rock2_{n}", params=p, steps=steps, target=target,
                loss_grad=loss_grad)
