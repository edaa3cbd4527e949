"""Scalar, voxel-by-voxel re-statement of one model step for tiny grids.

Written independently of the vectorised oracle (its own velocity set, its own
table lookup, explicit neighbour loops) so that an indexing, roll-direction or
vectorisation slip in either one shows up as a mismatch.  Scalar resistance
only (the tensorial setup has its own pins)."""
import math

VELS = [(x, y, z) for z in (-1, 0, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)
        if x * x + y * y + z * z <= 2]
WTS = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}


def weight(c):
    return WTS[c[0] * c[0] + c[1] * c[1] + c[2] * c[2]]


def lerp(tab, v):
    t = v * 1024.0
    k = int(math.floor(t))
    if k > 1023:
        k = 1023
    return tab[k] + (t - k) * (tab[k + 1] - tab[k])


class Brute:
    """State: pop[a][(x,y,z)][c] dictionaries of floats."""

    def __init__(self, p, cls, phi, ptype, tables, K0, sJ, thw, tho):
        self.p = p
        self.nx, self.ny, self.nz = p.nx, p.ny, p.nz
        self.cls, self.phi, self.ptype, self.tables = cls, phi, ptype, tables
        self.K0, self.sJ, self.thw, self.tho = K0, sJ, thw, tho

    def wrap(self, x, y, z):
        return (x % self.nx, y % self.ny, z % self.nz)

    def solid(self, v):
        x, y, z = v
        return self.cls[z][y][x] == 1

    def voxels(self):
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    yield (x, y, z)

    def step(self, pop, r, side):
        p = self.p
        nc = p.ncomp
        cs2 = 1.0 / 3.0
        fluid = [v for v in self.voxels() if not self.solid(v)]
        rho = [{}, {}]
        mom = [{}, {}]
        for a in range(nc):
            for v in fluid:
                rho[a][v] = sum(pop[a][v][c] for c in VELS)
                mom[a][v] = tuple(sum(pop[a][v][c] * c[d] for c in VELS) for d in range(3))

        def nb(v, c):
            return self.wrap(v[0] + c[0], v[1] + c[1], v[2] + c[2])

        def grad(X, v):
            out = [0.0, 0.0, 0.0]
            for c in VELS:
                if c == (0, 0, 0):
                    continue
                n = nb(v, c)
                val = X[v] if self.solid(n) else X[n]
                for d in range(3):
                    out[d] += weight(c) * c[d] * val / cs2
            return out

        span = p.s_max - p.s_min
        S, Sh, rhoT = {}, {}, {}
        for v in fluid:
            if nc == 2:
                tw = rho[0][v] + r[0].get(v, 0.0)
                to = rho[1][v] + r[1].get(v, 0.0)
                s = tw / (tw + to)
                S[v] = min(max((s - p.s_min) / span, 0.0), 1.0)
                Sh[v] = (rho[0][v] / (rho[0][v] + rho[1][v]) - p.s_min) / span
                rhoT[v] = tw + to
            else:
                S[v] = 1.0
        nhat = [{}, {}]
        grad_other = [{}, {}]
        if nc == 2:
            for a in range(2):
                b = 1 - a
                for v in fluid:
                    g = grad(rho[b], v)
                    grad_other[a][v] = g
                    n = math.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
                    nhat[a][v] = [gi / n for gi in g] if n > p.eps_n else [0.0, 0.0, 0.0]
        post = [{}, {}]
        for v in fluid:
            x, y, z = v
            gray = self.cls[z][y][x] == 2
            in_region = gray if p.csf_region == "gray" else True
            rt = sum(rho[a][v] for a in range(nc))
            Fex = []
            for a in range(nc):
                F = [rho[a][v] * p.g[a][d] for d in range(3)]
                if nc == 2:
                    b = 1 - a
                    acc = [0.0, 0.0, 0.0]
                    for c in VELS:
                        if c == (0, 0, 0):
                            continue
                        n = nb(v, c)
                        psi = max(rho[b][v] + p.wall_dpsi[b], 0.0) if self.solid(n) else rho[b][n]
                        for d in range(3):
                            acc[d] += weight(c) * psi * c[d]
                    for d in range(3):
                        F[d] -= p.G * rho[a][v] * acc[d]
                    if p.kappa != 0.0 and in_region:
                        div = 0.0
                        for c in VELS:
                            if c == (0, 0, 0):
                                continue
                            n = nb(v, c)
                            nn = nhat[a][v] if self.solid(n) else nhat[a][n]
                            div += weight(c) * (nn[0] * c[0] + nn[1] * c[1] + nn[2] * c[2]) / cs2
                        g = grad_other[a][v]
                        for d in range(3):
                            F[d] += p.kappa * (-div) * g[d] * rho[a][v] / (p.phi_avg * p.phi_max)
                    if gray:
                        tab = self.tables[self.ptype[z][y][x]]
                        Pc = self.sJ[z][y][x] * lerp(tab["Pc"], S[v])
                        gS = grad(Sh, v)
                        for d in range(3):
                            F[d] -= Pc * rho[a][v] / rt * gS[d]
                Fex.append(F)
            R = 0.0
            if gray:
                if nc == 2:
                    tab = self.tables[self.ptype[z][y][x]]
                    krw = max(lerp(tab["Krw"], S[v]), p.kr_min)
                    kro = max(lerp(tab["Kro"], S[v]), p.kr_min)
                    nuw = cs2 * (p.tau[0] - 0.5)
                    nuo = cs2 * (p.tau[1] - 0.5)
                    cR = 0.0
                    if S[v] > 0:
                        cR += rt * S[v] * nuw / krw
                    if 1.0 - S[v] > 0:
                        cR += rt * (1.0 - S[v]) * nuo / kro
                else:
                    cR = rt * cs2 * (p.tau[0] - 0.5)
                R = cR / self.K0[z][y][x]
            # trapezoidal rule in the resistance
            u = [(sum(mom[a][v][d] for a in range(nc)) + 0.5 * sum(Fex[a][d] for a in range(nc)))
                 / (rt + 0.5 * R) for d in range(3)]
            Ftot = [[Fex[a][d] - rho[a][v] / rt * R * u[d] for d in range(3)] for a in range(nc)]
            den = sum(rho[a][v] / p.tau[a] for a in range(nc))
            up = [sum(mom[a][v][d] / p.tau[a] for a in range(nc)) / den for d in range(3)]
            for a in range(nc):
                ra = rho[a][v]
                Fa = Ftot[a]
                ua = [up[d] + Fa[d] / (2.0 * ra) for d in range(3)]
                # equilibrium velocity: u' (exact-difference forcing) in pore
                # voxels, ua with the force term's 1 - 1/(2 tau) weight in gray ones
                ue = ua if gray else up
                kf = 1.0 - 0.5 / p.tau[a] if gray else 1.0
                feq = {}
                for c in VELS:
                    cu = sum(c[d] * ue[d] for d in range(3))
                    uu = sum(ue[d] * ue[d] for d in range(3))
                    feq[c] = weight(c) * ra * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
                fneq = {c: pop[a][v][c] - feq[c] for c in VELS}
                if p.collision == "regularized":
                    j = [sum(fneq[c] * c[d] for c in VELS) for d in range(3)]
                    Pi = [[sum(fneq[c] * c[d] * c[e] for c in VELS) for e in range(3)]
                          for d in range(3)]
                    tr = Pi[0][0] + Pi[1][1] + Pi[2][2]
                    f1 = {}
                    for c in VELS:
                        cj = sum(c[d] * j[d] for d in range(3))
                        pcc = sum(Pi[d][e] * c[d] * c[e] for d in range(3) for e in range(3))
                        f1[c] = weight(c) * (3.0 * cj + 4.5 * (pcc - tr / 3.0))
                else:
                    f1 = fneq
                out = {}
                for c in VELS:
                    cF = sum(c[d] * Fa[d] for d in range(3))
                    cu = sum(c[d] * ua[d] for d in range(3))
                    uF = sum(ua[d] * Fa[d] for d in range(3))
                    force = kf * weight(c) * (3.0 * cF + 9.0 * (cu * cF - uF / 3.0))
                    out[c] = feq[c] + (1.0 - 1.0 / p.tau[a]) * f1[c] + force
                post[a][v] = out
            # residual transfer
            if nc == 2 and gray:
                m = p.m_minor
                if (not side[v]) and S[v] >= 0.5 + p.hyst:
                    sw = (rho[0][v] + r[0].get(v, 0.0)) / rho[0][v]
                    for c in VELS:
                        post[0][v][c] *= sw
                    r[0][v] = 0.0
                    d_o = max(0.0, min(self.tho[z][y][x] * rhoT[v] - r[1].get(v, 0.0),
                                       rho[1][v] - m))
                    for c in VELS:
                        post[1][v][c] *= 1.0 - d_o / rho[1][v]
                    r[1][v] = r[1].get(v, 0.0) + d_o
                    side[v] = True
                elif side[v] and S[v] <= 0.5 - p.hyst:
                    so = (rho[1][v] + r[1].get(v, 0.0)) / rho[1][v]
                    for c in VELS:
                        post[1][v][c] *= so
                    r[1][v] = 0.0
                    d_w = max(0.0, min(self.thw[z][y][x] * rhoT[v] - r[0].get(v, 0.0),
                                       rho[0][v] - m))
                    for c in VELS:
                        post[0][v][c] *= 1.0 - d_w / rho[0][v]
                    r[0][v] = r[0].get(v, 0.0) + d_w
                    side[v] = False
        # streaming (pull) with halfway bounce-back
        new = [{}, {}]
        for a in range(nc):
            for v in fluid:
                out = {}
                for c in VELS:
                    src = self.wrap(v[0] - c[0], v[1] - c[1], v[2] - c[2])
                    if self.solid(src):
                        out[c] = post[a][v][(-c[0], -c[1], -c[2])]
                    else:
                        out[c] = post[a][src][c]
                new[a][v] = out
        return new, r, side
