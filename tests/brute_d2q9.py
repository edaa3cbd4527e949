"""An independent D2Q9 Shan-Chen step (BGK collision, halfway bounce-back at
solid voxels, body force and the pseudo-potential force through the force
term of Eq. (3), no gray voxels), written for the quasi-2-D pin of the D3Q19
oracle: a D3Q19 run on an nz = 1 grid, with its populations summed over each
in-plane velocity, must follow this model exactly (the z-copies of an
in-plane velocity carry D2Q9's weights, 1/18 + 2/36 = 1/9 and 1/36, and with
no z variation every moment the BGK step uses is a group sum)."""
import numpy as np

# D2Q9: rest, axes, diagonals
E = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)])
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OP = [0, 2, 1, 4, 3, 6, 5, 8, 7]
CS2 = 1.0 / 3.0


def at(a, ex, ey):
    """a[y, x] evaluated at (x + ex, y + ey), periodic."""
    return np.roll(np.roll(a, -ex, axis=1), -ey, axis=0)


def step(f, solid, tau, G, g, wall_dpsi):
    """f[a, k, y, x] post-streaming D2Q9 populations of ncomp components ->
    the next post-streaming set."""
    nc = f.shape[0]
    fluid = ~solid
    rho = f.sum(axis=1)
    mom = np.einsum("kd,akyx->adyx", E.astype(float), f)
    F = np.zeros_like(mom)
    for a in range(nc):
        F[a, 0] += rho[a] * g[a][0]
        F[a, 1] += rho[a] * g[a][1]
    if nc == 2:
        for a in range(2):
            b = 1 - a
            wall = np.maximum(rho[b] + wall_dpsi[b], 0.0)
            s = np.zeros((2,) + rho.shape[1:])
            for k in range(1, 9):
                ex, ey = E[k]
                psi = np.where(at(solid, ex, ey), wall, at(rho[b], ex, ey))
                s[0] += WT[k] * ex * psi
                s[1] += WT[k] * ey * psi
            F[a] += -G * rho[a] * s
    om = [1.0 / t for t in tau]
    den = sum(rho[a] * om[a] for a in range(nc))
    den = np.where(fluid, den, 1.0)
    up = sum(mom[a] * om[a] for a in range(nc)) / den
    post = np.zeros_like(f)
    for a in range(nc):
        r = np.where(fluid, rho[a], 1.0)
        ua = up + F[a] / (2.0 * r)
        usq = up[0] ** 2 + up[1] ** 2
        uF = ua[0] * F[a, 0] + ua[1] * F[a, 1]
        for k in range(9):
            ex, ey = E[k]
            eu = ex * up[0] + ey * up[1]
            feq = WT[k] * rho[a] * (1 + eu / CS2 + eu * eu / (2 * CS2 ** 2) - usq / (2 * CS2))
            eF = ex * F[a, 0] + ey * F[a, 1]
            ea = ex * ua[0] + ey * ua[1]
            src = WT[k] * (eF / CS2 + (ea * eF - CS2 * uF) / CS2 ** 2)
            post[a, k] = np.where(fluid, feq + (1 - om[a]) * (f[a, k] - feq) + src, 0.0)
    new = np.zeros_like(f)
    for a in range(nc):
        for k in range(9):
            ex, ey = E[k]
            pulled = at(post[a, k], -ex, -ey)
            new[a, k] = np.where(fluid, np.where(at(solid, -ex, -ey), post[a, OP[k]], pulled), 0.0)
    return new
