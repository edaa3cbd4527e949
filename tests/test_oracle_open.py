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
