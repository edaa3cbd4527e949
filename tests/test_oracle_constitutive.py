"""Oracle pins for the per-voxel constitutive setup: table interpolation,
Leverett-J scaling (Eq. (5)) and the residual saturations read off the
J-scaled Pc-S curve (residual-component model, Sec. II, Fig. 6)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lerp_table, crossing, gray_parameters, Oracle


def test_lerp_hits_samples_and_is_linear_between():
    rng = np.random.default_rng(1)
    tab = rng.standard_normal(1025)
    k = np.arange(1025)
    np.testing.assert_array_equal(lerp_table(tab, k / 1024.0), tab)
    v = (k[:-1] + 0.25) / 1024.0
    np.testing.assert_allclose(lerp_table(tab, v), 0.75 * tab[:-1] + 0.25 * tab[1:], rtol=1e-14,
                               atol=1e-15)
    # a linear table is reproduced everywhere
    lin = 3.0 - 2.0 * k / 1024.0
    x = rng.uniform(0, 1, 100)
    np.testing.assert_allclose(lerp_table(lin, x), 3.0 - 2.0 * x, rtol=1e-15)


def _bisect(fun, target, lo=0.0, hi=1.0):
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fun(mid) > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("lam", [0.5, 1.0, 2.0, 3.0])
@pytest.mark.parametrize("phi", [0.05, 0.15, 0.225, 0.3, 0.4])
def test_residual_saturations_closed_form(lam, phi):
    swr, pce, pcpm, cmax, cmin, phi_ref = 0.1, 0.05, 0.05, 3.5, 0.575, 0.225
    pc, krw, kro = W.brooks_corey_tables(pce, lam, swr)
    K0 = W.kozeny_carman_table(2.0)
    tab = W.pore_table(K0, pc, krw, kro, phi_ref=phi_ref, pc_pm=pcpm)
    cls = np.full((1, 1, 1), 2, np.uint8)
    k0, sJ, thw, tho = gray_parameters(np.full((1, 1, 1), phi), np.zeros((1, 1, 1), np.uint8),
                                       cls, [tab], cmax, cmin)
    sJ, thw, tho = float(sJ[0, 0, 0]), float(thw[0, 0, 0]), float(tho[0, 0, 0])
    # J scaling with Kozeny-Carman: s_J = [phi_ref/(1-phi_ref)] / [phi/(1-phi)]
    kc = (phi_ref / (1 - phi_ref)) / (phi / (1 - phi))
    assert abs(sJ / kc - 1) < 2e-3  # table interpolation of K0
    # residual water: s_J Pc(S) = c_max Pc_PM with Brooks-Corey Pc
    se = (sJ * pce / (cmax * pcpm)) ** lam
    if se < 1.0 and sJ * 10 * pce >= cmax * pcpm:
        assert abs(thw - (swr + (1 - swr) * se)) < 2e-3
    else:
        assert thw == 0.0
    # residual oil: Pc >= s_J Pc_e everywhere, so a crossing needs s_J Pc_e <= c_min Pc_PM
    if sJ * pce <= cmin * pcpm:
        so = swr + (1 - swr) * (sJ * pce / (cmin * pcpm)) ** lam
        assert abs(tho - (1 - so)) < 2e-3
    else:
        assert tho == 0.0
    # exact crossing of the piecewise-linear interpolant, found by bisection
    f = lambda s: sJ * float(lerp_table(pc, np.array([s]))[0])
    if thw > 0:
        assert abs(thw - _bisect(f, cmax * pcpm)) < 1e-13
    if tho > 0:
        assert abs((1 - tho) - _bisect(f, cmin * pcpm)) < 1e-13


def test_droplet_slab_constants():
    # one pore type, phi = phi_ref: s_J = 1, theta_w = 0.1 + 0.9 (1/3.5)^2, theta_o = 0
    wl = W.droplet_slab()
    k0, sJ, thw, tho = gray_parameters(np.array([0.3]), np.array([0], np.uint8),
                                       np.array([2], np.uint8), wl["tables"], 3.5, 0.575)
    assert abs(sJ[0] - 1.0) < 1e-15
    assert abs(thw[0] - (0.1 + 0.9 / 3.5 ** 2)) < 1e-4
    assert tho[0] == 0.0
    assert abs(k0[0] - 0.3 ** 3 / 0.7 ** 2 * 4 / 180) < 5e-6


def test_crossing_edge_cases():
    y = np.linspace(1.0, 0.0, 1025)
    assert crossing(y, 2.0) is None       # curve entirely below
    assert crossing(y, -1.0) is None      # curve entirely above
    assert crossing(y, 1.0) == 0.0
    assert abs(crossing(y, 0.25) - 0.75) < 1e-15
    flat = np.concatenate([np.full(513, 0.5), np.linspace(0.5, 0.0, 513)[1:]])
    assert crossing(flat, 0.5) == 0.0     # smallest S on a flat run


def _one_voxel(thw, tho):
    p = W.Params(nx=1, ny=1, nz=1, ncomp=2, G=3.0).filled()
    wl = W.droplet_slab()
    o = Oracle(p)
    o.set_geometry(np.full((1, 1, 1), 2, np.uint8), np.full((1, 1, 1), 0.3),
                   np.zeros((1, 1, 1), np.uint8), wl["tables"])
    o.thw[:] = thw
    o.tho[:] = tho
    return o, p


def test_residual_transfer_scripted():
    """A single gray voxel driven through both crossings; trap, release and
    conservation checked against hand-computed amounts."""
    thw, tho = 0.2, 0.15
    o, p = _one_voxel(thw, tho)
    m = p.m_minor
    span = p.s_max - p.s_min
    # start as oil (S < 1/2), then impose a water-rich state: S >= 1/2 + h
    o.init_fluid(np.array([0.1]), np.array([0.9]))
    assert not o.side[0, 0, 0]
    zero = np.zeros((3, 1, 1, 1))
    o.f[0] = o.equilibrium(np.full((1, 1, 1), 0.8), zero)
    o.f[1] = o.equilibrium(np.full((1, 1, 1), 0.2), zero)
    mass0 = o.f.sum(axis=(1, 2, 3, 4))
    o.step(1)
    rT = 1.0
    d_o = min(tho * rT, 0.2 - m)
    assert o.side[0, 0, 0]
    np.testing.assert_allclose(o.r[1, 0, 0, 0], d_o, rtol=1e-14)
    np.testing.assert_allclose(o.f[1].sum(), 0.2 - d_o, rtol=1e-14)
    np.testing.assert_allclose(o.f[0].sum(), 0.8, rtol=1e-14)
    # still water-rich: no second event
    o.step(3)
    np.testing.assert_allclose(o.r[1, 0, 0, 0], d_o, rtol=1e-14)
    # oil comes back: S <= 1/2 - h releases the residual oil and traps water
    o.f[0] = o.equilibrium(np.full((1, 1, 1), 0.1), zero)
    o.f[1] = o.equilibrium(np.full((1, 1, 1), 0.9 - d_o), zero)
    tw, to = 0.1, 0.9 - d_o + d_o
    s = tw / (tw + to)
    assert (s - p.s_min) / span <= 0.5 - p.hyst
    o.step(1)
    assert not o.side[0, 0, 0]
    d_w = min(thw * (tw + to), 0.1 - m)
    np.testing.assert_allclose(o.r[1, 0, 0, 0], 0.0, atol=1e-17)
    np.testing.assert_allclose(o.r[0, 0, 0, 0], d_w, rtol=1e-14)
    np.testing.assert_allclose(o.f[1].sum(), 0.9, rtol=1e-14)
    np.testing.assert_allclose(o.f[0].sum() + o.r[0].sum(), 0.1, rtol=1e-14)
    assert o.r.min() >= 0.0
