"""Oracle pin: the vectorised oracle equals an independent scalar nested-loop
step on tiny grids (solids, two pore types, CSF, capillary, resistance,
residual events, unequal relaxation times), to rounding."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle, C, Q
from brute_step import Brute, VELS


def tiny_case(ncomp=2, collision="regularized", seed=11, n=(3, 4, 5), region="gray"):
    nz, ny, nx = n
    rng = np.random.default_rng(seed)
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=ncomp, tau=(0.7, 1.3), G=3.0,
                 g=((2e-4, -1e-4, 5e-5), (0.0, 1e-4, 0.0)), kappa=-0.03, collision=collision,
                 csf_region=region).filled()
    cls = rng.choice([0, 0, 1, 2, 2], size=n).astype(np.uint8)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, size=n), 1.0)
    ptype = np.where(cls == 2, rng.integers(0, 2, size=n), 0).astype(np.uint8)
    K0 = W.kozeny_carman_table()
    tabs = []
    for lam in (1.0, 2.0):
        pc, krw, kro = W.brooks_corey_tables(0.05, lam, 0.1)
        tabs.append(W.pore_table(K0, pc, krw, kro, phi_ref=0.225, pc_pm=0.05))
    rw = rng.uniform(0.05, 1.0, size=n)
    ro = 1.05 - rw
    return p, cls, phi, ptype, tabs, rw, ro, rng


def perturb(o, rng):
    o.f = o.f * (1.0 + 0.02 * rng.standard_normal(o.f.shape))
    o.f = np.where(o.fluid, o.f, 0.0)


def to_brute(o):
    nc = o.ncomp
    pops = [{}, {}]
    idx = {tuple(int(v) for v in C[i]): i for i in range(Q)}
    for z in range(o.nz):
        for y in range(o.ny):
            for x in range(o.nx):
                if o.solid[z, y, x]:
                    continue
                for a in range(nc):
                    pops[a][(x, y, z)] = {c: float(o.f[a, idx[c], z, y, x]) for c in VELS}
    r = [{}, {}]
    side = {}
    for z in range(o.nz):
        for y in range(o.ny):
            for x in range(o.nx):
                for a in range(2):
                    r[a][(x, y, z)] = float(o.r[a, z, y, x])
                side[(x, y, z)] = bool(o.side[z, y, x])
    return pops, r, side


def compare(o, pops, r, side, tol):
    idx = {tuple(int(v) for v in C[i]): i for i in range(Q)}
    worst = 0.0
    for (x, y, z), d in pops[0].items():
        for a in range(o.ncomp):
            for c, val in pops[a][(x, y, z)].items():
                worst = max(worst, abs(val - o.f[a, idx[c], z, y, x]))
    assert worst < tol, worst
    for (x, y, z), val in r[0].items():
        assert abs(val - o.r[0, z, y, x]) < tol
        assert abs(r[1][(x, y, z)] - o.r[1, z, y, x]) < tol
        assert side[(x, y, z)] == bool(o.side[z, y, x])


@pytest.mark.parametrize("ncomp,collision,region",
                         [(2, "regularized", "gray"),
                          (2, "bgk", "all"),
                          (1, "regularized", "gray"),
                          (1, "bgk", "gray")])
def test_oracle_matches_nested_loops(ncomp, collision, region):
    p, cls, phi, ptype, tabs, rw, ro, rng = tiny_case(ncomp, collision, region=region)
    o = Oracle(p)
    o.set_geometry(cls, phi, ptype, tabs)
    o.init_fluid(rw, ro)
    perturb(o, rng)
    if ncomp == 2:
        # flip half of the side flags so that residual events fire
        ev = o.evaluate()
        flip = o.gray & (rng.random(o.shape) < 0.7)
        o.side = np.where(flip, ev["S"] < 0.5, o.side)
        o.r[0] = np.where(o.gray, 0.01 * rng.random(o.shape), 0.0)
    b = Brute(p, cls.tolist(), phi.tolist(), ptype.tolist(), tabs, o.K0.tolist(), o.sJ.tolist(),
              o.thw.tolist(), o.tho.tolist())
    pops, r, side = to_brute(o)
    events = 0
    for _ in range(3):
        before = dict(side)
        pops, r, side = b.step(pops, r, side)
        events += sum(before[v] != side[v] for v in side)
        o.step(1)
        compare(o, pops, r, side, 1e-14)
    if ncomp == 2:
        assert events > 0
