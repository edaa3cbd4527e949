"""Pins of the oracle's single-phase permeability run (K0 = phi <u> nu / g,
the paper's Appendix), independent of its implementation:

* an all-pore box accelerates uniformly: after n steps from rest the reported
  velocity (m + F/2) / rho is (n + 1/2) g exactly, so K0 = (n + 1/2) nu for any
  collision and axis;
* a slit (solid layers at y = 0 and y = H + 1) with the BGK collision at
  tau = 1/2 + sqrt(3)/4 has the exact discrete steady state
  u(y) = g / (2 nu) (y - 1/2) (H + 1/2 - y) (halfway bounce-back), hence
  K0 = sum_y (y - 1/2)(H + 1/2 - y) / (2 (H + 2));
* the wall frame and the mirror are built where the Appendix puts them."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import rev


def params(shape, tau, g, axis, collision="regularized"):
    gv = [0.0, 0.0, 0.0]
    gv[axis] = g
    nz, ny, nx = shape
    return W.Params(nx=nx, ny=ny, nz=nz, ncomp=1, tau=(tau, tau), G=0.0,
                    g=(tuple(gv), (0.0, 0.0, 0.0)), kappa=0.0, collision=collision).filled()


@pytest.mark.parametrize("axis,collision", [(0, "regularized"), (1, "bgk"), (2, "regularized")])
def test_all_pore_box_accelerates_uniformly(axis, collision):
    shape = (3, 4, 5)
    tau, g, n = 0.8, 1e-4, 12
    K, u = rev.permeability(params(shape, tau, g, axis, collision), np.zeros(shape, np.uint8),
                            n, axis)
    nu = (tau - 0.5) / 3
    assert abs(K - (n + 0.5) * nu) < 1e-10 * (n + 0.5) * nu
    assert np.abs(u - (n + 0.5) * g).max() < 1e-10 * (n + 0.5) * g


def test_slit_reaches_exact_discrete_permeability():
    H = 6
    tau = 0.5 + math.sqrt(3) / 4
    g = 1e-6
    cls = np.zeros((1, H + 2, 1), np.uint8)
    cls[:, 0, :] = 1
    cls[:, H + 1, :] = 1
    K, u = rev.permeability(params(cls.shape, tau, g, 0, "bgk"), cls, 1500, 0)
    exact = sum((y - 0.5) * (H + 0.5 - y) for y in range(1, H + 1)) / (2 * (H + 2))
    assert abs(K - exact) < 1e-9 * exact, (K, exact)


def test_side_walls_and_mirror_geometry():
    cls = (np.arange(2 * 3 * 4).reshape(2, 3, 4) % 3 == 0).astype(np.uint8)
    framed, box = rev.with_side_walls(cls, axis=1)   # force along y: walls on x and z faces
    assert framed.shape == (4, 3, 6)
    assert np.array_equal(framed[box], cls)
    assert framed[0].all() and framed[-1].all() and framed[:, :, 0].all() and framed[:, :, -1].all()
    m = rev.mirrored(cls, axis=0)
    assert m.shape == (2, 3, 8)
    assert np.array_equal(m[:, :, :4], cls) and np.array_equal(m[:, :, 4:], cls[:, :, ::-1])


def test_sphere_pack_reaches_target_porosity():
    cls = W.sphere_pack((24, 24, 24), 0.35, seed=5, rmin=3.0, rmax=8.0)
    phi = 1.0 - cls.mean()
    assert 0.30 < phi <= 0.35
