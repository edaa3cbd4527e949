"""Oracle pins: lattice identities and the moments of the equilibrium, the
force term of Eq. (3) and the Hermite projection of the collision."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import C, W, OPP, Q, CS2, Oracle
from oracle.lattice import W_EXACT


def test_velocity_set_is_d3q19():
    # 19 distinct vectors: all of {-1,0,1}^3 with |c|^2 <= 2 (Sec. II, D3Q19)
    expect = {c for c in itertools.product((-1, 0, 1), repeat=3) if sum(v * v for v in c) <= 2}
    assert len(C) == Q == 19
    assert {tuple(int(v) for v in c) for c in C} == expect
    for i in range(Q):
        assert tuple(C[OPP[i]]) == tuple(-C[i])
        n2 = int(np.dot(C[i], C[i]))
        assert W_EXACT[i] == {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[n2]


def test_isotropy_exact_rationals():
    w = W_EXACT
    assert sum(w) == 1
    for a in range(3):
        assert sum(w[i] * int(C[i, a]) for i in range(Q)) == 0
        for b in range(3):
            s2 = sum(w[i] * int(C[i, a]) * int(C[i, b]) for i in range(Q))
            assert s2 == (Fraction(1, 3) if a == b else 0)
            for c in range(3):
                assert sum(w[i] * int(C[i, a] * C[i, b] * C[i, c]) for i in range(Q)) == 0
                for d in range(3):
                    s4 = sum(w[i] * int(C[i, a] * C[i, b] * C[i, c] * C[i, d]) for i in range(Q))
                    dd = (a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c)
                    assert s4 == Fraction(1, 9) * dd


def _moments(f):
    rho = f.sum(0)
    j = np.array([np.sum(f * C[:, a].reshape((Q,) + (1,) * (f.ndim - 1)), 0) for a in range(3)])
    P = np.array([[np.sum(f * (C[:, a] * C[:, b]).reshape((Q,) + (1,) * (f.ndim - 1)), 0)
                   for b in range(3)] for a in range(3)])
    return rho, j, P


def test_equilibrium_moments():
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 1.5, size=(5,))
    u = rng.uniform(-0.1, 0.1, size=(3, 5))
    feq = Oracle.equilibrium(rho, u)
    r, j, P = _moments(feq)
    np.testing.assert_allclose(r, rho, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(j, rho * u, rtol=0, atol=1e-15)
    for a in range(3):
        for b in range(3):
            np.testing.assert_allclose(P[a, b], rho * (CS2 * (a == b) + u[a] * u[b]),
                                       rtol=0, atol=2e-15)


def test_force_term_moments_and_edm_identity():
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.5, 1.5, size=(6,))
    u = rng.uniform(-0.1, 0.1, size=(3, 6))
    F = rng.uniform(-0.05, 0.05, size=(3, 6))
    S = Oracle.force_term(u, F)
    r, j, P = _moments(S)
    np.testing.assert_allclose(r, 0, atol=1e-16)
    np.testing.assert_allclose(j, F, atol=1e-16)
    for a in range(3):
        for b in range(3):
            np.testing.assert_allclose(P[a, b], u[a] * F[b] + F[a] * u[b], atol=1e-16)
    # exact-difference identity: f_eq(u + F/rho) - f_eq(u) = Eq.(3) at u + F/(2 rho)
    lhs = Oracle.equilibrium(rho, u + F / rho) - Oracle.equilibrium(rho, u)
    rhs = Oracle.force_term(u + F / (2 * rho), F)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=5e-17)
    # ...and it is not the same at the bare velocity (the shift matters)
    assert np.max(np.abs(Oracle.force_term(u, F) - lhs)) > 1e-5


def test_hermite_projection():
    rng = np.random.default_rng(9)
    fneq = rng.standard_normal((Q, 4)) * 1e-3
    f1 = Oracle.hermite_project(fneq)
    r0, j0, P0 = _moments(fneq)
    r1, j1, P1 = _moments(f1)
    # keeps the first and second moments and drops the zeroth
    np.testing.assert_allclose(j1, j0, atol=1e-17)
    np.testing.assert_allclose(r1, 0, atol=1e-17)
    np.testing.assert_allclose(P1, P0, atol=1e-17)
    # idempotent
    np.testing.assert_allclose(Oracle.hermite_project(f1), f1, atol=1e-17)
    # a set already in the span (an equilibrium difference with zero mass) is kept
    u = rng.uniform(-0.05, 0.05, size=(3, 4))
    d = Oracle.force_term(u, rng.uniform(-0.01, 0.01, size=(3, 4)))
    np.testing.assert_allclose(Oracle.hermite_project(d), d, atol=1e-17)
