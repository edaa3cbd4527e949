"""Pins of the oracle's open x faces (reservoirs of prescribed density beyond
x = 0 and x = nx - 1), independent of its implementation:

* a reservoir at the domain's own uniform rest state changes nothing, for one
  component and for the two-component bulk (the pseudo-potential sum of a
  uniform field vanishes whether its neighbours are voxels or reservoir cells);
* pressure-driven flow in a slit reaches a steady state whose mass flux
  sum_yz j_x is the same through every x (discrete continuity), runs from the
  dense reservoir to the light one, and has the parabolic cross-section of
  Poiseuille flow;
* gray voxels next to an open face are rejected."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle


def run(p, cls, rho_w, rho_o, steps):
    o = Oracle(p)
    shape = cls.shape
    o.set_geometry(cls, np.where(cls == 2, 0.3, 1.0), np.zeros(shape, np.uint8),
                   [W.pore_table(W.kozeny_carman_table(2.0), *W.brooks_corey_tables(0.05, 2.0, 0.1),
                                 phi_ref=0.3, pc_pm=0.05)])
    o.init_fluid(rho_w, rho_o)
    o.step(steps)
    return o


def test_reservoir_at_the_rest_state_is_neutral_one_component():
    p = W.Params(nx=6, ny=5, nz=4, ncomp=1, tau=(0.9, 0.9), G=0.0, bc_x="pressure",
                 rho_in=(1.0, 0.0), rho_out=(1.0, 0.0)).filled()
    cls = np.zeros((4, 5, 6), np.uint8)
    cls[1, 2, 3] = 1
    o = run(p, cls, np.ones(cls.shape), None, 20)
    ref = Oracle(p)
    ref.set_geometry(cls, np.ones(cls.shape), np.zeros(cls.shape, np.uint8), [])
    ref.init_fluid(np.ones(cls.shape))
    assert np.abs(o.f - ref.f).max() < 1e-15


def test_reservoir_at_the_rest_state_is_neutral_two_components():
    m = W.minority_density(3.0)
    p = W.Params(nx=6, ny=5, nz=4, ncomp=2, tau=(1.0, 1.0), bc_x="pressure",
                 rho_in=(1.0, m), rho_out=(1.0, m)).filled()
    cls = np.zeros((4, 5, 6), np.uint8)
    o = run(p, cls, np.ones(cls.shape), np.full(cls.shape, m), 20)
    ev = o.evaluate()
    assert np.abs(ev["rho"][0] - 1.0).max() < 1e-14
    assert np.abs(ev["rho"][1] - m).max() < 1e-14
    assert np.abs(ev["u"]).max() < 1e-14


def test_pressure_driven_slit_is_steady_and_poiseuille_shaped():
    H, L = 6, 12
    p = W.Params(nx=L, ny=H + 2, nz=1, ncomp=1, tau=(1.0, 1.0), G=0.0, bc_x="pressure",
                 rho_in=(1.003, 0.0), rho_out=(0.997, 0.0)).filled()
    cls = np.zeros((1, H + 2, L), np.uint8)
    cls[:, 0, :] = 1
    cls[:, H + 1, :] = 1
    o = run(p, cls, np.ones(cls.shape), None, 4000)
    ev = o.evaluate()
    jx = (ev["rho"][0] * ev["u"][0])[0]          # [y, x]
    flux = jx.sum(axis=0)                       # through every x
    assert flux.min() > 0                       # from the dense reservoir to the light one
    assert np.ptp(flux) < 1e-8 * flux.mean(), flux
    prof = jx[1:H + 1, L // 2]
    y = np.arange(1, H + 1)
    par = (y - 0.5) * (H + 0.5 - y)
    assert np.abs(prof / prof.max() - par / par.max()).max() < 0.02


def test_gray_next_to_an_open_face_is_rejected():
    p = W.Params(nx=8, ny=4, nz=4, ncomp=2, bc_x="pressure").filled()
    cls = np.zeros((4, 4, 8), np.uint8)
    cls[:, :, 1] = 2
    with pytest.raises(ValueError):
        Oracle(p).set_geometry(cls, np.where(cls == 2, 0.3, 1.0), np.zeros(cls.shape, np.uint8),
                               [W.pore_table(W.kozeny_carman_table(2.0),
                                             *W.brooks_corey_tables(0.05, 2.0, 0.1),
                                             phi_ref=0.3, pc_pm=0.05)])


# ---------------------------------------------------------------- exact density faces
def _pulled_moments(o, xb):
    """Density and momentum of each component of the set the voxels of plane
    xb pulled (the oracle's state after streaming), [a] and [a, d]."""
    from oracle.lattice import C
    f = o.f[:, :, :, :, xb]                       # [a, i, z, y]
    rho = f.sum(axis=1)
    mom = np.stack([np.einsum("i,aizy->azy", C[:, d].astype(float), f) for d in range(3)], axis=1)
    return rho, mom


def test_density_faces_impose_the_density_and_no_transverse_momentum():
    """After every step the pulled set of each fluid voxel on a face holds the
    prescribed density of each component and zero momentum along y and z,
    with solid voxels in the face planes and the pseudo-potential force on."""
    m = W.minority_density(3.0)
    rng = np.random.default_rng(5)
    shape = (4, 5, 7)
    cls = np.where(rng.random(shape) < 0.2, 1, 0).astype(np.uint8)
    rin, rout = (1.02, m), (m, 0.99)
    p = W.Params(nx=7, ny=5, nz=4, ncomp=2, tau=(1.0, 1.2), bc_x="density",
                 rho_in=rin, rho_out=rout).filled()
    x = np.arange(7)[None, None, :]
    rw = m + (1 - m) * 0.5 * (1 - np.tanh((x - 3.0) / 1.5)) * np.ones(shape)
    rw = rw * (1 + 0.01 * rng.standard_normal(shape))
    o = Oracle(p)
    o.set_geometry(cls, np.ones(shape), np.zeros(shape, np.uint8), [])
    o.init_fluid(rw, 1 + m - rw)
    for _ in range(5):
        o.step(1)
        for xb, rb in ((0, rin), (6, rout)):
            fl = cls[:, :, xb] != 1
            rho, mom = _pulled_moments(o, xb)
            for a in range(2):
                assert np.abs(rho[a][fl] - rb[a]).max() < 1e-14 * max(rb[a], 1.0), (xb, a)
                assert np.abs(mom[a, 1][fl]).max() < 1e-15, (xb, a)
                assert np.abs(mom[a, 2][fl]).max() < 1e-15, (xb, a)


def test_density_faces_at_the_rest_state_are_neutral():
    p = W.Params(nx=6, ny=5, nz=4, ncomp=1, tau=(0.9, 0.9), G=0.0, bc_x="density",
                 rho_in=(1.0, 0.0), rho_out=(1.0, 0.0)).filled()
    cls = np.zeros((4, 5, 6), np.uint8)
    cls[1, 2, 3] = 1
    cls[2, 1, 0] = 1   # a solid voxel in the inlet plane
    o = run(p, cls, np.ones(cls.shape), None, 20)
    ref = Oracle(W.Params(nx=6, ny=5, nz=4, ncomp=1, tau=(0.9, 0.9), G=0.0).filled())
    ref.set_geometry(cls, np.ones(cls.shape), np.zeros(cls.shape, np.uint8), [])
    ref.init_fluid(np.ones(cls.shape))
    ref.step(20)
    assert np.abs(o.f - ref.f).max() < 1e-15


def test_density_driven_slit_carries_the_poiseuille_mass_flux():
    """Plates at y = 1/2 and H + 1/2 (halfway bounce-back), the density fixed
    at x = 0 and x = nx - 1: the steady mass flux per unit depth equals
    H^3 cs^2 (rho_in - rho_out) / (12 nu (nx - 1)) (plane Poiseuille flow with
    p = cs^2 rho, whose mass flux does not depend on the local density)."""
    H, L = 8, 16
    nu = (1.0 - 0.5) / 3.0
    p = W.Params(nx=L, ny=H + 2, nz=1, ncomp=1, tau=(1.0, 1.0), G=0.0, bc_x="density",
                 rho_in=(1.003, 0.0), rho_out=(0.997, 0.0)).filled()
    cls = np.zeros((1, H + 2, L), np.uint8)
    cls[:, 0, :] = 1
    cls[:, H + 1, :] = 1
    o = run(p, cls, np.ones(cls.shape), None, 6000)
    ev = o.evaluate()
    jx = (ev["rho"][0] * ev["u"][0])[0]
    flux = jx.sum(axis=0)
    assert np.ptp(flux) < 1e-8 * flux.mean(), flux
    expect = H ** 3 * (1.0 / 3.0) * (1.003 - 0.997) / (12.0 * nu * (L - 1))
    assert abs(flux.mean() / expect - 1) < 0.02, (flux.mean(), expect)
    # the imposed densities hold at the faces
    assert abs(ev["rho"][0][0, 1:H + 1, 0].mean() - 1.003) < 1e-12
    assert abs(ev["rho"][0][0, 1:H + 1, L - 1].mean() - 0.997) < 1e-12


def test_density_faces_need_three_planes():
    with pytest.raises(ValueError):
        Oracle(W.Params(nx=2, ny=4, nz=4, ncomp=1, G=0.0, bc_x="density").filled())
