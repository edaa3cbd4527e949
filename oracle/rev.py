"""Single-phase permeability of a fully resolved domain (the paper's
Appendix): K0 = phi <u> nu / g, with <u> the velocity along the driving body
acceleration g averaged over the pore space, phi the pore fraction and
nu = (tau - 1/2) / 3.  The run is the one-component model of model.Oracle on
pore and solid voxels only, started from rest at density 1.  TEST
INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).

The Appendix closes the four sides parallel to the force with walls and
mirrors the domain along the force so that it is periodic there;
`with_side_walls` and `mirrored` build those boxes for the periodic oracle: a
wall is a layer of solid voxels outside each side face (halfway bounce-back
puts it half a voxel beyond the last fluid voxel), and the mirror joins the
box to its reflection along the force.
"""
from __future__ import annotations

import numpy as np

from .model import Oracle, PORE

# numpy axis of each force axis (arrays are [z][y][x]; axis 0 is x)
NP_AXIS = (2, 1, 0)


def with_side_walls(cls, axis):
    """cls framed by a solid layer on both faces normal to each axis other
    than `axis`; returns the framed array and the slices of the original box."""
    cls = np.asarray(cls, np.uint8)
    pads = [(1, 1)] * 3
    pads[NP_AXIS[axis]] = (0, 0)
    out = np.pad(cls, pads, constant_values=1)
    box = tuple(slice(p0, p0 + n) for (p0, _), n in zip(pads, cls.shape))
    return out, box


def mirrored(cls, axis):
    """cls joined to its mirror image along `axis` (twice the length)."""
    cls = np.asarray(cls, np.uint8)
    ax = NP_AXIS[axis]
    return np.concatenate([cls, np.flip(cls, axis=ax)], axis=ax)


def permeability(params, cls, steps, axis=0, with_state=False):
    """Runs the periodic box `cls` (0 pore, 1 solid) for `steps` steps with
    `params` (one component, tau, collision and the body acceleration g along
    `axis`, no gray voxels) and returns (K0, u): u is the velocity field along
    the force, (m + F/2) / rho, zero on solid voxels, and K0 = (sum of u over
    the box / number of voxels) nu / g = phi <u> nu / g.  with_state: also the
    final post-streaming populations f[i][z][y][x]."""
    cls = np.asarray(cls, np.uint8)
    shape = cls.shape
    o = Oracle(params)
    o.set_geometry(cls, np.ones(shape), np.zeros(shape, np.uint8), [])
    o.init_fluid(np.ones(shape))
    o.step(steps)
    u = np.where(cls == PORE, o.evaluate()["u"][axis], 0.0)
    g = float(params.g[0][axis])
    nu = (float(params.tau[0]) - 0.5) / 3.0
    if with_state:
        return u.sum() / cls.size * nu / g, u, o.f[0].copy()
    return u.sum() / cls.size * nu / g, u
