"""Oracle pins for its outputs: the per-link outlet flux, the periodic
Gaussian smoothing of the tensor set-up, and the saturation and speed
diagnostics.  Each is checked against something other than its own formula:
a mass budget, a uniform-acceleration closed form and a hand-listed set of
links for the flux; the variance of the continuous Gaussian (within the
truncation of its radius) and separability for the smoothing; hand-computed
fields for the diagnostics."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Oracle, smooth_periodic
from oracle.lattice import C, W as WQ, Q


def _box(shape, cls=None, ncomp=2, **kw):
    nz, ny, nx = shape
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=ncomp, **kw).filled()
    o = Oracle(p)
    cls = np.zeros(shape, np.uint8) if cls is None else cls
    o.set_geometry(cls, np.where(cls == W.GRAY, 0.3, 1.0), np.zeros(shape, np.uint8),
                   [W.pore_table(W.kozeny_carman_table(), *W.brooks_corey_tables(0.05, 2.0, 0.1),
                                 phi_ref=0.3, pc_pm=0.05)])
    return o


def _random_state(o, rng):
    """Two fluid densities and small random non-equilibrium parts."""
    shape = o.shape
    rw = rng.uniform(0.05, 1.0, shape)
    o.init_fluid(rw, 1.05 - rw if o.ncomp == 2 else None)
    o.f *= 1.0 + 0.05 * rng.standard_normal(o.f.shape)
    o.f = np.where(o.fluid[None, None], o.f, 0.0)


def _slab_mass(o, a, lo, hi):
    """Mass of component a in the voxels lo < x <= hi (indices mod nx), from
    the post-streaming state."""
    xs = [(lo + k) % o.nx for k in range(1, (hi - lo) % o.nx + 1)]
    return float(np.sum(o.f[a][:, :, :, xs]))


@pytest.mark.parametrize("collision", ["regularized", "bgk"])
def test_outlet_flux_is_the_mass_budget_of_a_slab(collision):
    # Between two planes a | a+1 and b | b+1 the mass of the slab a < x <= b
    # changes in one step by exactly Q_a - Q_b: every population that enters
    # or leaves the slab crosses one of the two planes on a fluid-fluid link,
    # and bounce-back at a solid keeps it in its voxel.  A sign error, a plane
    # index off by one or a solid link counted would break the budget.
    rng = np.random.default_rng(11)
    shape = (5, 6, 9)
    cls = np.where(rng.uniform(size=shape) < 0.25, W.SOLID, W.PORE).astype(np.uint8)
    planes = (8, 2, 5)  # 8 | 0 is the periodic wrap
    for trial in range(2):
        runs = {}
        for xf in planes:
            o = _box(shape, cls, ncomp=2, tau=(0.8, 1.3), collision=collision, G=1.5, m_minor=0.05,
                     g=((2e-4, -1e-4, 3e-4), (-1e-4, 2e-4, 0.0)), outlet_x=xf)
            _random_state(o, np.random.default_rng(100 + trial))
            before = [[_slab_mass(o, a, lo, hi) for a in range(2)]
                      for lo, hi in ((2, 5), (5, 8), (8, 2))]
            o.step(1)
            after = [[_slab_mass(o, a, lo, hi) for a in range(2)]
                     for lo, hi in ((2, 5), (5, 8), (8, 2))]
            runs[xf] = (o.Q_last.copy(), before, after)
        for k, (lo, hi) in enumerate(((2, 5), (5, 8), (8, 2))):
            for a in range(2):
                dm = runs[lo][2][k][a] - runs[lo][1][k][a]
                dq = runs[lo][0][a] - runs[hi][0][a]
                assert abs(runs[lo][0][a]) > 1e-4  # a real flux crosses the plane
                assert abs(dm - dq) < 1e-13 * (1.0 + abs(runs[lo][1][k][a]))


def test_outlet_flux_of_uniform_acceleration():
    # An all-pore periodic box accelerated from rest by body forces: the total
    # post-collision momentum of step k is k sum_a rho^a g^a per voxel (the
    # collision exchanges momentum between the components, never creates it),
    # and with every voxel alike the flux through a plane is the plane's
    # summed x momentum, ny nz k sum_a rho^a g^a_x.  With one acceleration for
    # both components nothing is exchanged, and each component's flux is
    # ny nz k rho^a g_x.
    shape = (3, 4, 5)
    area = shape[0] * shape[1]
    rho = (0.9, 0.35)
    for g in (((2.5e-4, 1e-4, 0.0), (-1e-4, 0.0, 3e-4)),
              ((2.5e-4, 1e-4, 0.0), (2.5e-4, 1e-4, 0.0))):
        o = _box(shape, ncomp=2, tau=(0.7, 1.6), G=0.0, m_minor=0.05, g=g, outlet_x=2)
        o.init_fluid(np.full(shape, rho[0]), np.full(shape, rho[1]))
        tot = rho[0] * g[0][0] + rho[1] * g[1][0]
        for k in range(1, 6):
            o.step(1)
            assert abs(o.Q_last.sum() - area * k * tot) < 1e-15 * k * area
            if g[0] == g[1]:
                for a in range(2):
                    assert abs(o.Q_last[a] - area * k * rho[a] * g[a][0]) < 1e-15 * k * area
        assert abs(o.Q_acc.sum() - 15 * area * tot) < 1e-14 * area


def test_outlet_flux_hand_counted_links():
    # 4 x 3 x 1 box, plane 1 | 2, solids at (x, y) = (1, 0) and (2, 2).
    # Directions with c_x = +1 are 1 (1,0,0), 7 (1,1,0), 9 (1,-1,0),
    # 11 (1,0,1), 13 (1,0,-1); with c_x = -1: 2, 8 (-1,-1,0), 10 (-1,1,0),
    # 12, 14.  With nz = 1 the c_z links close on the same row.
    # Out of x = 1 (fluid rows 1 and 2): row 1 -> rows 1 (1, 11, 13), 2 (7,
    # solid: skipped), 0 (9); row 2 -> rows 2 (1, 11, 13: solid, skipped),
    # 0 (7, wraps), 1 (9).
    # Into x = 1 from x = 2 (fluid rows 0 and 1): row 0 -> rows 0 (2, 12, 14:
    # solid at (1, 0), skipped), 2 (8, wraps), 1 (10); row 1 -> rows 1 (2, 12,
    # 14), 0 (8: solid, skipped), 2 (10).
    shape = (1, 3, 4)
    cls = np.zeros(shape, np.uint8)
    cls[0, 0, 1] = W.SOLID
    cls[0, 2, 2] = W.SOLID
    o = _box(shape, cls, ncomp=1, G=0.0, outlet_x=1)
    rng = np.random.default_rng(5)
    post = rng.uniform(0.1, 1.0, (1, Q) + shape)
    o._outlet_flux(post)
    p = post[0]
    out = [(1, 1), (11, 1), (13, 1), (9, 1), (7, 2), (9, 2)]   # (direction, row) at x = 1
    inn = [(8, 0), (10, 0), (2, 1), (12, 1), (14, 1), (10, 1)]  # (direction, row) at x = 2
    expect = sum(p[i, 0, y, 1] for i, y in out) - sum(p[i, 0, y, 2] for i, y in inn)
    assert abs(o.Q_last[0] - expect) < 1e-15
    # the lists above hold every fluid-fluid crossing link: 6 each way
    for i in range(Q):
        assert C[i, 0] != 0 or all(i != d for d, _ in out + inn)


@pytest.mark.parametrize("sigma,radius", [(1.5, 5), (1.0, 5), (0.8, 3)])
def test_smoothing_of_a_delta_is_a_gaussian_of_that_width(sigma, radius):
    # A unit delta smoothed by the normalised, truncated periodic Gaussian:
    # total 1, zero beyond the radius, separable, and along each axis a
    # variance equal to sigma^2 of the continuous Gaussian up to the
    # truncation, whose relative size is below 2 (r/s)^3 exp(-(r+1/2)^2/2s^2)
    # / sqrt(2 pi) (tail of x^2 e^{-x^2/2}); a wrong sigma (the variance taken
    # for the width, a factor 2 in the exponent) is off by tens of per cent.
    n = (13, 14, 15)
    d = np.zeros(n)
    pos = (1, 12, 7)  # near the faces: the periodic wrap is exercised
    d[pos] = 1.0
    s = smooth_periodic(d, sigma, radius)
    assert abs(s.sum() - 1.0) < 1e-14
    prof = []
    for axis in range(3):
        dist = (np.arange(n[axis]) - pos[axis] + n[axis] // 2) % n[axis] - n[axis] // 2
        marg = s.sum(axis=tuple(k for k in range(3) if k != axis))
        assert np.all(marg[np.abs(dist) > radius] == 0.0)
        var = float(np.sum(marg * dist * dist))
        x = (radius + 0.5) / sigma
        bound = 2.0 * x ** 3 * math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi) + 1e-12
        assert abs(var / sigma ** 2 - 1.0) <= bound, (axis, var)
        assert abs(float(np.sum(marg * dist))) < 1e-14  # centred
        prof.append(marg)
    outer = prof[0][:, None, None] * prof[1][None, :, None] * prof[2][None, None, :]
    np.testing.assert_allclose(s, outer, atol=1e-16)


def test_diagnostics_saturation_of_a_hand_made_field():
    # 4^3 box: gray (phi = 0.3) for x < 2, pore elsewhere.  Gray voxels hold
    # water (rho_w = 1, rho_o = m: S = 1) except one with oil plus a residual
    # water amount that makes its total water fraction 1/2 (S = 1/2); pore
    # voxels hold oil (S = 0) except one with equal densities (S = 1/2,
    # since s_min + s_max = 1).  Sw = sum phi S / sum phi.
    shape = (4, 4, 4)
    cls = np.zeros(shape, np.uint8)
    cls[:, :, :2] = W.GRAY
    o = _box(shape, cls, ncomp=2)
    m = o.p.m_minor
    rw = np.where(cls == W.GRAY, 1.0, m)
    ro = np.where(cls == W.GRAY, m, 1.0)
    rw[1, 2, 0], ro[1, 2, 0] = m, 1.0          # gray, oil ...
    o.init_fluid(rw, ro)
    o.r[0][1, 2, 0] = 1.0 - m                  # ... plus residual water: 1 : 1
    rw[3, 0, 3] = ro[3, 0, 3] = 0.5            # pore, S = 1/2
    for a, rr in enumerate((rw, ro)):
        for i in range(Q):
            o.f[a, i] = WQ[i] * rr
    d = o.diagnostics()
    ng, npore = 32, 32
    expect = (0.3 * (ng - 1) * 1.0 + 0.3 * 0.5 + 0.5) / (0.3 * ng + npore)
    assert abs(d["sw"] - expect) < 1e-14
    assert abs(d["mass_w"] - (rw.sum() + 1.0 - m)) < 1e-12
    assert abs(d["mass_o"] - ro.sum()) < 1e-12


def test_diagnostics_max_speed_of_a_hand_made_field():
    # One component, no force: the reported velocity is m / rho.  Rest
    # populations everywhere, with opposite pairs shifted in two voxels:
    # voxel A gets m = (0.02, 0, 0), voxel B m = (0, 0.024, 0.018) (|u| = 0.03).
    shape = (3, 4, 5)
    o = _box(shape, ncomp=1, G=0.0)
    o.init_fluid(np.ones(shape))
    o.f[0, 1, 0, 1, 2] += 0.01
    o.f[0, 2, 0, 1, 2] -= 0.01
    o.f[0, 3, 2, 3, 4] += 0.012
    o.f[0, 4, 2, 3, 4] -= 0.012
    o.f[0, 5, 2, 3, 4] += 0.009
    o.f[0, 6, 2, 3, 4] -= 0.009
    d = o.diagnostics()
    assert abs(d["max_u"] - 0.03) < 1e-15
    assert abs(d["mass_w"] - 60.0) < 1e-12
    f = o.fields()
    assert abs(f["ux"][0, 1, 2] - 0.02) < 1e-16
    assert abs(f["uy"][2, 3, 4] - 0.024) < 1e-16 and abs(f["uz"][2, 3, 4] - 0.018) < 1e-16
