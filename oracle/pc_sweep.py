"""Capillary-pressure sweep of a fully resolved domain (the Pc(Sw) half of
the library runs of the paper's Appendix): a two-component displacement of
the sub-volume between two reservoirs, the pressure difference changed in
steps and the saturation of the sub-volume recorded at a steady state of
each level.  TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark
baseline).

The paper gives the protocol in words only; the reading taken here is a
drainage: the sample starts full of water (wetting with water-wet walls),
an oil region of `buffer_in` planes lies before it (the Appendix's 14
cells), and an oil reservoir beyond x = 0 pushes at a density that rises
level by level against a water reservoir beyond x = nx - 1.  Between the
sample and the outlet a layer of gray voxels acts as a capillary membrane:
an oil-water interface inside gray voxels carries a pressure jump of the
table's Pc (Eq. (1)'s capillary term), so oil stops at it while water
passes.  The level's capillary pressure is the difference of the two
reservoirs' bulk pressures, p = cs^2 (rho_w + rho_o) + cs^2 G rho_w rho_o;
the saturation is the mean of S over the sample's pore voxels.  A level ends
when that saturation changes by at most `tol` over `check_every` steps, or
after `max_steps` steps.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .lattice import CS2
from .model import Oracle, PORE, SOLID, GRAY


def bulk_pressure(rho_w, rho_o, G):
    """Shan-Chen bulk pressure of a uniform mixture (psi = rho)."""
    return CS2 * (rho_w + rho_o) + CS2 * G * rho_w * rho_o


def sweep_box(cls, buffer_in, membrane, buffer_out, side_walls):
    """The run's box along x: buffer_in pore planes, the domain, membrane gray
    planes, buffer_out pore planes; a solid frame on the y and z faces when
    side_walls.  Returns (classes, mask of the domain's pore voxels)."""
    cls = np.asarray(cls, np.uint8)
    nz, ny, nx = cls.shape
    w = 1 if side_walls else 0
    NX = buffer_in + nx + membrane + buffer_out
    box = np.full((nz + 2 * w, ny + 2 * w, NX), PORE, np.uint8)
    inner = (slice(w, w + nz), slice(w, w + ny))
    box[inner + (slice(buffer_in, buffer_in + nx),)] = cls
    box[inner + (slice(buffer_in + nx, buffer_in + nx + membrane),)] = GRAY
    if side_walls:
        box[0, :, :] = box[-1, :, :] = SOLID
        box[:, 0, :] = box[:, -1, :] = SOLID
    sample = np.zeros(box.shape, bool)
    sample[inner + (slice(buffer_in, buffer_in + nx),)] = cls == PORE
    return box, sample


def pc_sweep(cls, model, membrane_table, rho_nw_in, buffer_in=14, membrane=2, buffer_out=2,
             side_walls=True, membrane_phi=0.3, check_every=200, max_steps=4000, tol=1e-4,
             keep=None):
    """One domain's sweep with model.Oracle (fp64).  `model` is a
    workloads.Params of the two-component model.  Returns dict(pc, sw, steps,
    converged) with one entry per level; with keep = [] the oracle's fields
    after each level are appended to it."""
    box, sample = sweep_box(cls, buffer_in, membrane, buffer_out, side_walls)
    NZ, NY, NX = box.shape
    m = float(model.m_minor)
    rho_out = (1.0, m)
    p = replace(model, nx=NX, ny=NY, nz=NZ, ncomp=2, bc_x="pressure",
                g=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)), rho_in=(m, float(rho_nw_in[0])),
                rho_out=rho_out, outlet_x=NX - 2)
    o = Oracle(p)
    phi = np.where(box == GRAY, membrane_phi, np.where(box == PORE, 1.0, 0.0))
    o.set_geometry(box, phi, np.zeros(box.shape, np.uint8), [membrane_table])
    x = np.arange(NX, dtype=np.float64)[None, None, :]
    water = 0.5 * (1.0 + np.tanh((x - (buffer_in - 0.5)) / 1.5)) * np.ones(box.shape)
    rw = m + (1.0 - m) * water
    o.init_fluid(rw, 1.0 + m - rw)
    npore = int(sample.sum())

    def saturation():
        S = o.fields()["S"]
        return float(S[sample].sum() / npore) if npore else 0.0

    out = dict(pc=[], sw=[], steps=[], converged=[])
    prev = saturation()
    for level in rho_nw_in:
        o.p = replace(o.p, rho_in=(m, float(level)))
        steps, conv, cur = 0, False, prev
        while steps < max_steps:
            n = min(check_every, max_steps - steps)
            o.step(n)
            steps += n
            cur = saturation()
            steady = abs(cur - prev) <= tol
            prev = cur
            if steady:
                conv = True
                break
        out["pc"].append(bulk_pressure(m, float(level), p.G) - bulk_pressure(*rho_out, p.G))
        out["sw"].append(cur)
        out["steps"].append(steps)
        out["converged"].append(conv)
        if keep is not None:
            keep.append(o.fields())
    return out
