"""Tensorial resistivity setup (paper, Sec. II, Eqs. (6)-(7); the abstract adds
the porosity gradient to the Hessian).  fp64, plain numpy, once per geometry.

Steps, in the paper's order:
1. porosity field for the directional analysis: solid 0, pore 1, gray phi,
   smoothed by a periodic separable Gaussian (std sigma_s, radius r, weights
   normalised to sum 1);
2. gradient g (central differences) and Hessian H (second differences; the
   mixed terms use the four diagonal neighbours) of the smoothed field;
3. principal axes B = eigenvectors of H; the eigenpairs are ordered by
   ascending |lambda| so the first axis is the direction of least porosity
   curvature (a fiber axis);
4. readings where the paper is silent: a voxel whose Hessian and gradient are
   both negligible (max|lambda| <= eps_H and |g| <= eps_g) keeps the isotropic
   K = K0 I; when the two smallest |lambda| are within delta_tie*|lambda_3|
   and the gradient has a component p in their plane with |p| > eps_g, the
   second axis is taken along p and the first perpendicular to it inside that
   plane (the axis of least variation is the one across which phi does not
   change), which makes the choice independent of the eigen-solver's basis;
5. K = B diag(a_k K0) B^T (Eq. (7), B orthonormal so B^-1 = B^T) and the
   stored inverse K^-1 = sum_k e_k e_k^T / (a_k K0).
The eigen-decomposition itself is LAPACK's (numpy.linalg.eigh)."""
import numpy as np


def gaussian_weights(sigma: float, radius: int) -> np.ndarray:
    j = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-j * j / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth_periodic(field: np.ndarray, sigma: float, radius: int) -> np.ndarray:
    w = gaussian_weights(sigma, radius)
    out = field.astype(np.float64)
    for axis in range(3):
        acc = np.zeros_like(out)
        for j, wj in zip(range(-radius, radius + 1), w):
            acc += wj * np.roll(out, -j, axis=axis)  # value at x + j
        out = acc
    return out


def _sh(a, dx=0, dy=0, dz=0):
    """a evaluated at (x+dx, y+dy, z+dz), periodic; arrays are [z, y, x]."""
    return np.roll(a, (-dz, -dy, -dx), axis=(0, 1, 2))


def gradient_hessian(ps: np.ndarray):
    off = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    g = np.zeros((3,) + ps.shape)
    H = np.zeros((3, 3) + ps.shape)
    for a in range(3):
        ea = off[a]
        p_plus = _sh(ps, *ea)
        p_minus = _sh(ps, *[-v for v in ea])
        g[a] = 0.5 * (p_plus - p_minus)
        H[a, a] = p_plus - 2.0 * ps + p_minus
        for b in range(a + 1, 3):
            eb = off[b]
            pp = _sh(ps, *[u + v for u, v in zip(ea, eb)])
            pm = _sh(ps, *[u - v for u, v in zip(ea, eb)])
            mp = _sh(ps, *[-u + v for u, v in zip(ea, eb)])
            mm = _sh(ps, *[-u - v for u, v in zip(ea, eb)])
            H[a, b] = H[b, a] = 0.25 * (pp - pm - mp + mm)
    return g, H


def principal_axes(H3: np.ndarray, g3: np.ndarray, eps_g, eps_H, delta_tie):
    """For one voxel: returns (isotropic?, E) with E[:, k] the k-th axis."""
    lam, vec = np.linalg.eigh(H3)
    gn = np.linalg.norm(g3)
    if np.max(np.abs(lam)) <= eps_H and gn <= eps_g:
        return True, np.eye(3)
    order = np.argsort(np.abs(lam), kind="stable")
    lam = lam[order]
    E = vec[:, order].copy()
    a = np.abs(lam)
    if a[1] - a[0] <= delta_tie * a[2]:
        e3 = E[:, 2]
        p = g3 - np.dot(g3, e3) * e3
        pn = np.linalg.norm(p)
        if pn > eps_g:
            e2 = p / pn
            e1 = np.cross(e3, e2)
            e1 /= np.linalg.norm(e1)
            E[:, 0] = e1
            E[:, 1] = e2
    return False, E


def inverse_permeability(phi, cls, ptype, K0, tables, sigma_s, radius, eps_g, eps_H, delta_tie,
                         PORE=0, GRAY=2, voxels=None):
    """Returns (Kinv[6, ...] in the order xx, yy, zz, xy, xz, yz, aux) where aux
    holds the smoothed field, gradient, Hessian and per-voxel axis matrices for
    tests.  Only gray voxels get a tensor; ``voxels`` optionally restricts the
    eigen-analysis to a list of flat indices (others stay zero)."""
    base = np.where(cls == GRAY, phi, np.where(cls == PORE, 1.0, 0.0))
    ps = smooth_periodic(base, sigma_s, radius)
    g, H = gradient_hessian(ps)
    Kinv = np.zeros((6,) + phi.shape)
    axes = {}
    flat_idx = np.flatnonzero(cls.ravel() == GRAY) if voxels is None else np.asarray(voxels)
    shp = phi.shape
    for fi in flat_idx:
        z, y, x = np.unravel_index(fi, shp)
        H3 = H[:, :, z, y, x]
        g3 = g[:, z, y, x]
        kd = tables[int(ptype[z, y, x])]["kd"]
        k0 = K0[z, y, x]
        iso, E = principal_axes(H3, g3, eps_g, eps_H, delta_tie)
        if iso:
            M = np.eye(3) / k0
        else:
            M = np.zeros((3, 3))
            for k in range(3):
                M += np.outer(E[:, k], E[:, k]) / (kd[k] * k0)
        axes[int(fi)] = (iso, E)
        Kinv[:, z, y, x] = (M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2])
    return Kinv, dict(smoothed=ps, grad=g, hess=H, axes=axes)
