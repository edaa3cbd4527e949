"""Oracle pins for the tensorial resistivity (Sec. II, Eqs. (6)-(7)):
reductions to the scalar model, principal-axis orientation inside an analytic
fiber bundle, independence from the eigen-solver and the tie-break rule."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Oracle, inverse_permeability, principal_axes, smooth_periodic, CS2


def _cyl_case(n=24, axis=(1.0, 0.0, 0.0), r=5.0, kd=(1.0, 0.1, 0.1), noise=False):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    c = (n - 1) / 2.0
    d = np.stack([x - c, y - c, z - c])
    t = np.tensordot(a, d, axes=1)
    dist = np.sqrt(np.maximum((d ** 2).sum(0) - t * t, 0.0))
    inside = dist <= r
    cls = np.where(inside, 2, 0).astype(np.uint8)
    phi = np.where(inside, 0.3, 1.0)
    if noise:
        rng = np.random.default_rng(0)
        phi = np.where(inside, np.clip(0.3 + 0.1 * rng.uniform(-1, 1, phi.shape), 0.05, 0.95), 1.0)
    pc, krw, kro = W.brooks_corey_tables(0.05, 2.0, 0.1)
    tab = W.pore_table(W.kozeny_carman_table(), pc, krw, kro, 0.3, 0.05, kd=kd)
    K0 = np.where(inside, 1.2e-3, 0.0)
    return cls, phi, np.zeros(cls.shape, np.uint8), [tab], K0, a, dist


def test_unit_multipliers_give_isotropic_tensor():
    cls, phi, pt, tabs, K0, a, dist = _cyl_case(kd=(1.0, 1.0, 1.0), noise=True)
    Kinv, _ = inverse_permeability(phi, cls, pt, K0, tabs, 1.5, 5, 1e-6, 1e-6, 0.05)
    g = cls == 2
    for k in range(3):
        np.testing.assert_allclose(Kinv[k][g] * K0[g], 1.0, rtol=0, atol=1e-13)
    for k in range(3, 6):
        np.testing.assert_allclose(Kinv[k][g] * K0[g], 0.0, atol=1e-13)


@pytest.mark.parametrize("axis,median_deg,worst_deg",
                         [((1, 0, 0), 1.0, 1.0), ((0, 1, 1), 1.0, 1.0), ((1, 2, 3), 2.0, 6.0)])
def test_fiber_axis_is_first_principal_axis(axis, median_deg, worst_deg):
    # lattice-aligned and face-diagonal axes: within 1 degree everywhere; an
    # oblique axis carries the voxelisation staircase (median 2, worst 6 degrees)
    cls, phi, pt, tabs, K0, a, dist = _cyl_case(n=28, axis=axis, r=6.0)
    Kinv, aux = inverse_permeability(phi, cls, pt, K0, tabs, 1.5, 5, 1e-6, 1e-6, 0.05)
    c = 28 // 2
    # voxels 1 .. r-1 from the axis, away from the box faces (lines are not wrapped)
    z, y, x = np.meshgrid(*(np.arange(28),) * 3, indexing="ij")
    central = (np.abs(x - 13.5) < 7) & (np.abs(y - 13.5) < 7) & (np.abs(z - 13.5) < 7)
    sel = (cls == 2) & (dist >= 1.0) & (dist <= 5.0) & central
    cosines = []
    for fi in np.flatnonzero(sel.ravel()):
        iso, E = aux["axes"][int(fi)]
        assert not iso
        cosines.append(abs(float(np.dot(E[:, 0], a))))
    cosines = np.array(cosines)
    assert len(cosines) > 50
    assert np.median(cosines) > math.cos(math.radians(median_deg)), np.median(cosines)
    assert np.min(cosines) > math.cos(math.radians(worst_deg)), np.min(cosines)
    # K along the axis is K0, across it 0.1 K0
    fi = int(np.flatnonzero(sel.ravel())[0])
    zz, yy, xx = np.unravel_index(fi, cls.shape)
    M = np.zeros((3, 3))
    v = Kinv[:, zz, yy, xx]
    M[0, 0], M[1, 1], M[2, 2] = v[:3]
    M[0, 1] = M[1, 0] = v[3]
    M[0, 2] = M[2, 0] = v[4]
    M[1, 2] = M[2, 1] = v[5]
    K = np.linalg.inv(M)
    assert abs(a @ K @ a / K0[zz, yy, xx] - 1.0) < 1e-3


def test_eigensolver_independence():
    # K^-1 from LAPACK's symmetric solver equals the one built from the
    # general (non-symmetric) eigen-solver with the same ordering rule
    rng = np.random.default_rng(4)
    kd = np.array([1.0, 0.3, 0.05])
    for _ in range(200):
        A = rng.standard_normal((3, 3))
        H = A + A.T
        g = rng.standard_normal(3)
        lam = np.linalg.eigvalsh(H)
        a = np.sort(np.abs(lam))
        if a[1] - a[0] <= 0.06 * a[2] or a[2] - a[1] <= 1e-3 * a[2]:
            continue
        iso, E = principal_axes(H, g, 1e-6, 1e-6, 0.05)
        M1 = sum(np.outer(E[:, k], E[:, k]) / kd[k] for k in range(3))
        w, V = np.linalg.eig(H)
        order = np.argsort(np.abs(w.real))
        V = V.real[:, order]
        V /= np.linalg.norm(V, axis=0)
        M2 = sum(np.outer(V[:, k], V[:, k]) / kd[k] for k in range(3))
        np.testing.assert_allclose(M1, M2, rtol=0, atol=1e-12 * np.abs(M1).max())


def test_tie_break_uses_gradient_and_is_basis_free():
    H = np.diag([0.2, 0.2, 3.0])
    g = np.array([0.3, 0.4, 0.7])
    iso, E = principal_axes(H, g, 1e-6, 1e-6, 0.05)
    p = np.array([0.3, 0.4, 0.0]) / 0.5
    assert abs(abs(E[:, 1] @ p) - 1) < 1e-14           # second axis along the in-plane gradient
    assert abs(E[:, 0] @ p) < 1e-14 and abs(E[:, 0][2]) < 1e-14
    # rotating the degenerate pair does not change the result
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    iso2, E2 = principal_axes(R @ H @ R.T + 0.0, g, 1e-6, 1e-6, 0.05)
    M = lambda E: sum(np.outer(E[:, k], E[:, k]) * (k + 1) for k in range(3))
    np.testing.assert_allclose(M(E), M(E2), atol=1e-13)
    # negligible Hessian and gradient: isotropic gate
    iso3, _ = principal_axes(np.zeros((3, 3)), np.zeros(3), 1e-6, 1e-6, 0.05)
    assert iso3


def test_uniform_porosity_tensor_run_equals_scalar_run():
    outs = []
    for tensor in (False, True):
        wl = W.uniform_gray(n=(4, 5, 6), phi=0.25, ncomp=1, tau=0.9, g=(1e-4, 3e-5, 0.0),
                            kd=(1.0, 0.1, 0.1), tensor=tensor)
        p = wl["params"]
        o = Oracle(p)
        o.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
        rng = np.random.default_rng(2)
        o.init_fluid(1.0 + 0.01 * rng.standard_normal(wl["rho_w"].shape))
        o.step(15)
        outs.append(o.fields())
    for k in ("rho_w", "ux", "uy", "uz"):
        np.testing.assert_allclose(outs[1][k], outs[0][k], rtol=0,
                                   atol=1e-13 * np.abs(outs[0][k]).max() + 1e-18)


def test_smoothing_preserves_mean_and_constants():
    rng = np.random.default_rng(6)
    f = rng.standard_normal((6, 7, 8))
    s = smooth_periodic(f, 1.5, 5)
    assert abs(s.mean() - f.mean()) < 1e-14
    np.testing.assert_allclose(smooth_periodic(np.full((5, 5, 5), 0.37), 1.5, 5), 0.37, rtol=1e-15)
