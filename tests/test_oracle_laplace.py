"""Oracle pins for the interface physics: Laplace's law for a static droplet,
the CSF surface-tension control of Eq. (4) (Sec. III.A: a negative coefficient
lowers sigma while interface thickness and spurious currents stay put), and
the flat-interface coexistence constant used by the workloads."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import Oracle, CS2

HERE = os.path.dirname(os.path.abspath(__file__))


def droplet2d(R, kappa, n=32, steps=1200):
    """Quasi-2D (nz = 1) periodic water droplet in oil; returns the pressure
    jump, max |u| and the 10-90 % interface width on the centre line."""
    p = W.Params(nx=n, ny=n, nz=1, ncomp=2, tau=(1.0, 1.0), G=3.0, kappa=kappa,
                 csf_region="all").filled()
    m = p.m_minor
    cls = np.zeros((1, n, n), np.uint8)
    o = Oracle(p)
    o.set_geometry(cls, np.ones(cls.shape), np.zeros(cls.shape, np.uint8), [])
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - (n - 1) / 2) ** 2 + (y - (n - 1) / 2) ** 2).reshape(1, n, n)
    prof = 0.5 * (1 - np.tanh((r - R) / 1.5))
    o.init_fluid(m + (1 - m) * prof, m + (1 - m) * (1 - prof))
    o.step(steps)
    ev = o.evaluate()
    rw, ro = ev["rho"][0][0], ev["rho"][1][0]
    pr = CS2 * (rw + ro) + CS2 * p.G * rw * ro
    c = n // 2
    dp = pr[c, c] - pr[0, 0]
    umax = float(np.sqrt(ev["u"][0] ** 2 + ev["u"][1] ** 2).max())
    line = rw[c, c:]
    lo, hi = line.min(), line.max()
    xs = np.arange(len(line), dtype=float)
    a = np.interp(lo + 0.9 * (hi - lo), line[::-1], xs[::-1])
    b = np.interp(lo + 0.1 * (hi - lo), line[::-1], xs[::-1])
    return dp, umax, b - a


@pytest.fixture(scope="module")
def base_runs():
    return {R: droplet2d(R, 0.0) for R in (5, 7, 9)}


def test_laplace_law_2d(base_runs):
    Rs = np.array(sorted(base_runs))
    dps = np.array([base_runs[R][0] for R in Rs])
    A = np.vstack([1.0 / Rs, np.ones_like(Rs, dtype=float)]).T
    (sigma, icpt), *_ = np.linalg.lstsq(A, dps, rcond=None)
    fit = A @ np.array([sigma, icpt])
    r2 = 1 - np.sum((dps - fit) ** 2) / np.sum((dps - dps.mean()) ** 2)
    assert sigma > 0.1
    assert r2 > 0.99
    assert abs(icpt) < 0.1 * dps[-1]


def test_csf_lowers_surface_tension_only(base_runs):
    R = 7
    dp0, u0, w0 = base_runs[R]
    dp1, u1, w1 = droplet2d(R, -0.05)
    assert dp1 < 0.8 * dp0            # kappa < 0 lowers sigma = dp R
    assert abs(w1 / w0 - 1) < 0.1     # interface thickness kept
    assert abs(u1 / u0 - 1) < 0.15    # spurious current kept (measured 10 %)


def test_kappa_calibration(base_runs):
    """The stored CSF coefficients (tests/golden/make_kappa.py) still scale the
    droplet's surface tension to 0.5 and 2 times its kappa = 0 value."""
    with open(os.path.join(HERE, "golden", "kappa.json")) as fh:
        gold = json.load(fh)
    dp0 = base_runs[7][0]
    for target, kappa in W.KAPPA_SIGMA_SCALE.items():
        assert kappa == gold["targets"][str(target)]["kappa"]
        dp = droplet2d(7, kappa)[0]
        assert abs(dp / dp0 / target - 1) < 0.01, (target, dp / dp0)


def test_coexistence_constant():
    with open(os.path.join(HERE, "golden", "coexistence.json")) as fh:
        gold = json.load(fh)
    assert gold["ratio"] == W.minority_density(3.0)
    # the stored steady profile is a fixed point of the oracle
    rw = np.array(gold["rho_w"]).reshape(1, 1, -1)
    ro = np.array(gold["rho_o"]).reshape(1, 1, -1)
    n = rw.shape[-1]
    p = W.Params(nx=n, ny=1, nz=1, ncomp=2, G=3.0).filled()
    o = Oracle(p)
    shape = (1, 1, n)
    o.set_geometry(np.zeros(shape, np.uint8), np.ones(shape), np.zeros(shape, np.uint8), [])
    o.init_fluid(rw, ro)
    o.step(300)
    f = o.fields()
    ratio = f["rho_w"][0, 0, 0] / f["rho_w"][0, 0, n // 2]
    assert abs(ratio / gold["ratio"] - 1) < 1e-3
    assert np.max(np.abs(f["rho_w"][0, 0] - rw[0, 0])) < 1e-3
