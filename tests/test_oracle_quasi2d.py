"""Quasi-2-D pin: the D3Q19 oracle on an nz = 1 grid, its populations summed
over each in-plane velocity, equals an independent D2Q9 model
(tests/brute_d2q9.py) step by step, for one component with a body force and
for two Shan-Chen components with solid walls (BGK, where the group sums close
on themselves exactly)."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle, C, Q
import brute_d2q9 as B


def group_sums(f3):
    """D3Q19 f[a, i, 1, y, x] -> D2Q9 F[a, k, y, x]."""
    out = np.zeros((f3.shape[0], 9) + f3.shape[3:])
    for k, (ex, ey) in enumerate(B.E):
        for i in range(Q):
            if C[i, 0] == ex and C[i, 1] == ey:
                out[:, k] += f3[:, i, 0]
    return out


@pytest.mark.parametrize("ncomp", [1, 2])
def test_nz1_d3q19_equals_d2q9(ncomp):
    rng = np.random.default_rng(17)
    ny, nx = 12, 15
    cls = np.where(rng.random((1, ny, nx)) < 0.15, 1, 0).astype(np.uint8)
    tau = (0.7, 1.3)
    g = ((2e-4, -1e-4, 0.0), (-1e-4, 5e-5, 0.0))
    p = W.Params(nx=nx, ny=ny, nz=1, ncomp=ncomp, tau=tau, G=3.0 if ncomp == 2 else 0.0,
                 collision="bgk", kappa=0.0, g=g).filled()
    o = Oracle(p)
    o.set_geometry(cls, np.where(cls == 1, 0.0, 1.0), np.zeros_like(cls), [W.uniform_gray()["tables"][0]])
    if ncomp == 2:
        m = p.m_minor
        x = np.arange(nx)[None, None, :]
        rw = np.where((x > 3) & (x < 10), 1.0, m) + 0.01 * rng.random((1, ny, nx))
        o.init_fluid(rw, 1.0 + m - rw)
    else:
        o.init_fluid(1.0 + 0.02 * rng.random((1, ny, nx)))
    F2 = group_sums(o.f)
    solid = cls[0] == 1
    for n in range(25):
        o.step(1)
        F2 = B.step(F2, solid, tau[:ncomp], p.G, [gg[:2] for gg in g[:ncomp]], p.wall_dpsi)
        err = np.abs(group_sums(o.f) - F2).max()
        assert err < 1e-14, (n, err)
    # the run is not trivial: the fluid moved
    assert np.abs(np.einsum("kd,akyx->dyx", B.E.astype(float), F2)).max() > 1e-4
