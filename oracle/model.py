"""Plain fp64 CPU oracle of the two-component pseudo-potential D3Q19 step with
the multiscale forces (paper, Sec. II).  TEST INFRASTRUCTURE ONLY: it is used by
the tests, by the smoke check and by the benchmark's CPU-baseline leg, never by
the GPU library.

Arrays are numpy, indexed [z, y, x]; populations are f[component, i, z, y, x]
with component 0 = water (w), 1 = oil (o).  The stored state is the
post-streaming population set at time n.  One step (Eq. (2)) is:

1. moments       rho^a = sum_i f_i^a, m^a = sum_i f_i^a c_i; residual-inclusive
                 saturation S (clamped) and mobile saturation S_hat;
2. stencils      isotropic gradient grad X = (1/cs^2) sum_i w_i X(x+c_i) c_i with
                 a solid neighbour taking the value X(x); pseudo-potential
                 force F_SC^a = -G rho^a sum_i w_i psi^b(x+c_i) c_i (b the
                 other component; psi = rho on fluid; a solid neighbour takes
                 the local value plus a wetting offset, max(rho^b(x) + dpsi^b, 0));
                 CSF force of Eq. (4) with phi^a = rho^b, n^a = grad rho^b / |.|,
                 curvature -div n^a, in the configured region (gray);
3. gray voxels   Eq. (1): capillary force -Pc(S) rho_r^a n H, read as
                 -Pc (rho^a/rho) grad S_hat; Brinkman resistance with
                 coefficient c_R = sum_b rho S^b nu^b / max(Kr^b, Kr_min) and
                 resistivity R = c_R K^-1 (scalar K0 or the tensor of
                 Eqs. (6)-(7));
4. velocity      the resistance acts on u = (rho I + R/2)^-1 (m + sum_a F_ex^a / 2)
                 (the trapezoidal rule: its steady states are exactly Darcy's
                 law, under body forces and under pressure gradients alike);
                 F_res^a = -(rho^a/rho) R u, F^a = F_ex^a + F_res^a;
                 u = (m + sum_a F^a / 2) / rho is also the reported velocity;
5. collision     Shan-Chen common velocity u' = sum(m^a/tau^a) / sum(rho^a/tau^a)
                 and ua = u' + F^a / (2 rho^a); non-equilibrium part projected
                 on Hermite orders 1-2 (regularised; BGK optional).  Pore
                 voxels: equilibrium at u', force term of Eq. (3) as the
                 exact-difference increment (Eq. (3) at ua).  Gray voxels:
                 Eq. (3) in its second-order (Guo) form, equilibrium and
                 non-equilibrium part at ua and the force term weighted by
                 1 - 1/(2 tau^a); the post-collision momentum is the same
                 m^a + F^a-sum either way, but the stiff resistance force no
                 longer enters the equilibrium's quadratic terms;
6. residual      trap / release on a saturation crossing (gray voxels);
7. outlet flux   per-link count through the plane x_f | x_f + 1;
8. streaming     pull with halfway bounce-back at solid neighbours, periodic.

Open x faces (bc_x = "pressure"; the pressure inlet and outlet of the paper's
Sec. III.B-D protocols, whose equations it does not give): beyond x = 0 and
x = nx - 1 lie reservoirs of prescribed densities rho_in, rho_out per
component.  A reservoir cell is fluid; it enters the pseudo-potential sum of a
boundary voxel with its density, and the populations it sends into the domain
are the equilibrium at its density and at the mixture velocity of the adjacent
boundary voxel's post-collision set (0 next to a solid voxel).  Gray voxels
and the CSF region must keep two voxels away from both faces, so the other
stencils never reach a reservoir.

Exact density faces (bc_x = "density"; the Zou-He-type density boundaries
that the paper's protocols call for, again without equations there): the same
reservoir cells enter the pseudo-potential sums, but the populations a
boundary voxel pulls across a face are set so that, after streaming, its
density of each component equals the prescribed one and its transverse
momentum is zero.  With s the c_x of the unknown directions (+1 at x = 0, -1
at x = nx - 1), the known pulled values g_j (c_x = 0 or -s, bounce-back at
solid sources included) fix the normal momentum through
    rho = sum_{c_x=0} g + 2 sum_{c_x=-s} g + s J,   J = rho u_x,
and each unknown takes the non-equilibrium bounce-back of its opposite plus
the equilibrium difference, with the transverse sums N_y, N_z of the c_x = 0
values removed:
    g_i = g_opp(i) + 6 w_i s J - c_y N_y - c_z N_z,
    N_y = (1/2) sum_{c_x=0} c_y g,   N_z = (1/2) sum_{c_x=0} c_z g.
(For the face's own plane these reproduce f_i - f_opp(i) = 2 w_i rho c_i.u /
cs^2 of the equilibrium with u = (u_x, 0, 0).)  Needs nx >= 3.
"""
from __future__ import annotations

import numpy as np

from .lattice import C, W, OPP, Q, CS2
from .constitutive import lerp_table, gray_parameters
from .tensor import inverse_permeability

PORE, SOLID, GRAY = 0, 1, 2


def _sh(a, c, sign=1):
    """a evaluated at x + sign*c (periodic); a is [..., z, y, x]."""
    cx, cy, cz = (int(v) * sign for v in c)
    return np.roll(a, (-cz, -cy, -cx), axis=(-3, -2, -1))


class Oracle:
    def __init__(self, params):
        p = params
        self.p = p
        self.nx, self.ny, self.nz = int(p.nx), int(p.ny), int(p.nz)
        self.ncomp = int(p.ncomp)
        if self.ncomp not in (1, 2):
            raise ValueError("ncomp must be 1 or 2")
        self.tau = tuple(float(t) for t in p.tau)[: self.ncomp]
        if min(self.tau) <= 0.5:
            raise ValueError("tau must exceed 1/2")
        self.shape = (self.nz, self.ny, self.nx)
        self.step_count = 0
        self.Q_last = np.zeros(2)
        self.Q_acc = np.zeros(2)
        self.f = None
        bc = getattr(p, "bc_x", "periodic")
        if bc not in ("periodic", "pressure", "density"):
            raise ValueError("bc_x must be periodic, pressure or density")
        self.open_x = bc != "periodic"
        self.exact_density = bc == "density"
        if self.exact_density and self.nx < 3:
            raise ValueError("exact density faces need nx >= 3")

    # ------------------------------------------------------------------ setup
    def set_geometry(self, cls, phi, ptype, tables):
        p = self.p
        cls = np.asarray(cls, np.uint8).reshape(self.shape)
        phi = np.asarray(phi, np.float64).reshape(self.shape)
        ptype = np.asarray(ptype, np.uint8).reshape(self.shape)
        if np.any(cls > 2):
            raise ValueError("class codes are 0 (pore), 1 (solid), 2 (gray)")
        gray = cls == GRAY
        if np.any(gray & ~((phi > 0) & (phi < 1))):
            raise ValueError("gray porosity must lie in (0, 1)")
        if np.any(gray & (ptype >= len(tables))):
            raise ValueError("pore type out of range")
        self.cls, self.phi, self.ptype, self.tables = cls, phi, ptype, tables
        self.solid = cls == SOLID
        self.fluid = ~self.solid
        self.gray = gray
        self.region = gray if p.csf_region == "gray" else self.fluid
        self.K0, self.sJ, self.thw, self.tho = gray_parameters(phi, ptype, cls, tables,
                                                               p.c_max, p.c_min)
        self.Kinv = None
        if p.tensor:
            self.Kinv, self.tensor_aux = inverse_permeability(
                phi, cls, ptype, self.K0, tables, p.sigma_s, p.smooth_radius, p.eps_g, p.eps_H,
                p.delta_tie)
        # solid flags of x + c_i and of x - c_i
        self.nb_solid = np.stack([_sh(self.solid, C[i]) for i in range(Q)])
        self.src_solid = np.stack([_sh(self.solid, C[i], -1) for i in range(Q)])
        if self.open_x:
            # x + c_i (nb) or x - c_i (src) beyond an x face: a reservoir cell,
            # which is fluid
            x = np.arange(self.nx)[None, None, :]
            hi, lo = x == self.nx - 1, x == 0
            self.cross_nb = np.stack([np.broadcast_to(hi if C[i, 0] > 0 else (lo if C[i, 0] < 0
                                      else np.zeros_like(lo)), self.shape) for i in range(Q)])
            self.cross_src = np.stack([np.broadcast_to(lo if C[i, 0] > 0 else (hi if C[i, 0] < 0
                                       else np.zeros_like(lo)), self.shape) for i in range(Q)])
            self.nb_solid = self.nb_solid & ~self.cross_nb
            self.src_solid = self.src_solid & ~self.cross_src
            near = np.zeros(self.nx, bool)
            near[[0, min(1, self.nx - 1), max(self.nx - 2, 0), self.nx - 1]] = True
            if np.any(gray[:, :, near]) or (p.kappa != 0.0 and p.csf_region != "gray"):
                raise ValueError("with open x faces, gray voxels and the CSF region keep two "
                                 "voxels away from both faces")

    def init_fluid(self, rho_w, rho_o=None):
        rho = [np.asarray(rho_w, np.float64).reshape(self.shape)]
        if self.ncomp == 2:
            rho.append(np.asarray(rho_o, np.float64).reshape(self.shape))
        zero = np.zeros((3,) + self.shape)
        self.f = np.zeros((self.ncomp, Q) + self.shape)
        for a in range(self.ncomp):
            self.f[a] = self.equilibrium(np.where(self.fluid, rho[a], 0.0), zero)
        self.r = np.zeros((2,) + self.shape)
        if self.ncomp == 2:
            ev = self.evaluate()
            self.side = self.gray & (ev["S"] >= 0.5)
        else:
            self.side = np.zeros(self.shape, bool)
        self.step_count = 0
        self.Q_last[:] = 0
        self.Q_acc[:] = 0

    # -------------------------------------------------------------- kernels
    @staticmethod
    def equilibrium(rho, u):
        """Second-order Hermite equilibrium w_i rho [1 + c.u/cs2 + (c.u)^2/(2cs4) - u^2/(2cs2)]."""
        usq = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        out = np.empty((Q,) + rho.shape)
        for i in range(Q):
            cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
            out[i] = W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2))
        return out

    @staticmethod
    def force_term(u, F):
        """Eq. (3): w_i [F.c/cs2 + (uF + Fu):(cc - cs2 I)/(2 cs4)]."""
        uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2]
        out = np.empty((Q,) + F.shape[1:])
        for i in range(Q):
            cF = C[i, 0] * F[0] + C[i, 1] * F[1] + C[i, 2] * F[2]
            cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
            out[i] = W[i] * (cF / CS2 + (2.0 * cu * cF - 2.0 * CS2 * uF) / (2 * CS2 * CS2))
        return out

    @staticmethod
    def hermite_project(fneq):
        """Projection of a non-equilibrium set on Hermite orders 1 and 2:
        w_i [c.j/cs2 + Pi:(cc - cs2 I)/(2 cs4)], j and Pi its first two moments."""
        j = np.zeros((3,) + fneq.shape[1:])
        Pi = np.zeros((3, 3) + fneq.shape[1:])
        for i in range(Q):
            for a in range(3):
                if C[i, a]:
                    j[a] += C[i, a] * fneq[i]
                for b in range(3):
                    if C[i, a] and C[i, b]:
                        Pi[a, b] += C[i, a] * C[i, b] * fneq[i]
        trace = Pi[0, 0] + Pi[1, 1] + Pi[2, 2]
        out = np.empty_like(fneq)
        for i in range(Q):
            cj = C[i, 0] * j[0] + C[i, 1] * j[1] + C[i, 2] * j[2]
            pcc = 0.0
            for a in range(3):
                for b in range(3):
                    if C[i, a] and C[i, b]:
                        pcc = pcc + Pi[a, b] * (C[i, a] * C[i, b])
            out[i] = W[i] * (cj / CS2 + (pcc - CS2 * trace) / (2 * CS2 * CS2))
        return out

    def _nbN(self, X, i):
        """X(x + c_i), or X(x) when x + c_i is solid."""
        return np.where(self.nb_solid[i], X, _sh(X, C[i]))

    def gradient(self, X):
        g = np.zeros((3,) + X.shape)
        for i in range(1, Q):
            v = self._nbN(X, i)
            for a in range(3):
                if C[i, a]:
                    g[a] += (W[i] * C[i, a] / CS2) * v
        return g

    def divergence(self, V):
        d = np.zeros(V.shape[1:])
        for i in range(1, Q):
            for a in range(3):
                if C[i, a]:
                    d += (W[i] * C[i, a] / CS2) * self._nbN(V[a], i)
        return d

    def evaluate(self):
        """Moments, saturation, forces and velocities of the current state."""
        p = self.p
        f = self.f
        fl = self.fluid
        nc = self.ncomp
        rho = f.sum(axis=1)
        mom = np.zeros((nc, 3) + self.shape)
        for a in range(nc):
            for i in range(Q):
                for d in range(3):
                    if C[i, d]:
                        mom[a, d] += C[i, d] * f[a, i]
        rho_t = rho.sum(axis=0)
        safe = np.where(fl, rho_t, 1.0)
        out = dict(rho=rho, mom=mom, rho_t=rho_t)
        F_ex = np.zeros((nc, 3) + self.shape)
        for a in range(nc):
            for d in range(3):
                F_ex[a, d] += rho[a] * p.g[a][d]
        if nc == 2:
            span = p.s_max - p.s_min
            tw = rho[0] + self.r[0]
            to = rho[1] + self.r[1]
            s = np.where(fl, tw / np.where(fl, tw + to, 1.0), 0.0)
            S = np.clip((s - p.s_min) / span, 0.0, 1.0)
            S_hat = np.where(fl, (rho[0] / safe - p.s_min) / span, 0.0)
            out.update(S=np.where(fl, S, 0.0), S_hat=S_hat, rhoT=tw + to)
            # pseudo-potential inter-component force
            for a in range(2):
                b = 1 - a
                acc = np.zeros((3,) + self.shape)
                wall = np.maximum(rho[b] + p.wall_dpsi[b], 0.0)
                for i in range(1, Q):
                    psi = np.where(self.nb_solid[i], wall, _sh(rho[b], C[i]))
                    if self.open_x and C[i, 0] != 0:
                        ghost = p.rho_out[b] if C[i, 0] > 0 else p.rho_in[b]
                        psi = np.where(self.cross_nb[i], ghost, psi)
                    for d in range(3):
                        if C[i, d]:
                            acc[d] += W[i] * C[i, d] * psi
                F_ex[a] += -p.G * rho[a] * acc
            # CSF surface-tension control, Eq. (4)
            if p.kappa != 0.0:
                for a in range(2):
                    b = 1 - a
                    gr = self.gradient(rho[b])
                    nrm = np.sqrt(gr[0] ** 2 + gr[1] ** 2 + gr[2] ** 2)
                    big = nrm > p.eps_n
                    nhat = np.where(big, gr / np.where(big, nrm, 1.0), 0.0)
                    curv = -self.divergence(nhat)
                    fcsf = p.kappa * curv * gr * rho[a] / (p.phi_avg * p.phi_max)
                    F_ex[a] += np.where(self.region, fcsf, 0.0)
            # Eq. (1) capillary term on gray voxels
            gS = self.gradient(S_hat)
            Pc = np.zeros(self.shape)
            Krw = np.zeros(self.shape)
            Kro = np.zeros(self.shape)
            for t, tab in enumerate(self.tables):
                sel = self.gray & (self.ptype == t)
                if sel.any():
                    Pc[sel] = self.sJ[sel] * lerp_table(tab["Pc"], S[sel])
                    Krw[sel] = lerp_table(tab["Krw"], S[sel])
                    Kro[sel] = lerp_table(tab["Kro"], S[sel])
            for a in range(2):
                F_ex[a] += np.where(self.gray, -Pc * (rho[a] / safe) * gS, 0.0)
            nu = [CS2 * (t - 0.5) for t in self.tau]
            Sw, So = S, 1.0 - S
            cw = np.where(Sw > 0, rho_t * Sw * nu[0] / np.maximum(Krw, p.kr_min), 0.0)
            co = np.where(So > 0, rho_t * So * nu[1] / np.maximum(Kro, p.kr_min), 0.0)
            cR = np.where(self.gray, cw + co, 0.0)
            out.update(Pc=Pc, Krw=Krw, Kro=Kro)
        else:
            nu = CS2 * (self.tau[0] - 0.5)
            cR = np.where(self.gray, rho_t * nu, 0.0)
            out.update(S=np.where(fl, 1.0, 0.0), S_hat=np.where(fl, 1.0, 0.0), rhoT=rho_t)
        out["cR"] = cR
        # velocity the resistance of Eq. (1) acts on, by the trapezoidal rule:
        # (rho I + R / 2) u = m + sum_a F_ex^a / 2, R = c_R K^-1 (or c_R / K0),
        # F_res = -R u; the steady states are exactly Darcy's law
        b = mom.sum(axis=0) + 0.5 * F_ex.sum(axis=0)
        if self.Kinv is None:
            Rs = np.where(self.gray, cR / np.where(self.gray, self.K0, 1.0), 0.0)
            u = b / (safe + 0.5 * Rs)
            Ru = Rs * u
        else:
            K = self.Kinv
            Rm = np.zeros((3, 3) + self.shape)
            idx = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}
            for (i, j), k in idx.items():
                Rm[i, j] = cR * K[k]
                Rm[j, i] = cR * K[k]
            A = 0.5 * Rm
            for d in range(3):
                A[d, d] += safe
            Am = np.moveaxis(A, (0, 1), (-2, -1))
            bm = np.moveaxis(b, 0, -1)[..., None]
            u = np.moveaxis(np.linalg.solve(Am, bm)[..., 0], -1, 0)
            Ru = np.einsum("ij...,j...->i...", Rm, u)
        F = np.empty_like(F_ex)
        for a in range(nc):
            F[a] = F_ex[a] - (rho[a] / safe) * Ru
        u = np.where(fl, u, 0.0)
        den = sum(rho[a] / self.tau[a] for a in range(nc))
        up = sum(mom[a] / self.tau[a] for a in range(nc)) / np.where(fl, den, 1.0)
        out.update(F_ex=F_ex, F=F, u=u, up=np.where(fl, up, 0.0), Ru=Ru)
        return out

    # ------------------------------------------------------------------ step
    def step(self, n=1):
        for _ in range(int(n)):
            self._one_step()

    def _one_step(self):
        p = self.p
        ev = self.evaluate()
        rho, F, u, up = ev["rho"], ev["F"], ev["u"], ev["up"]
        fl = self.fluid
        post = np.empty_like(self.f)
        for a in range(self.ncomp):
            # the velocity of component a shifted by half its force
            ua = up + F[a] / np.where(fl, 2.0 * rho[a], 1.0)
            # pore voxels: Eq. (3) as the exact-difference-method increment
            # f_eq(rho^a, u' + F^a/rho^a) - f_eq(rho^a, u'), i.e. Eq. (3) at
            # u' + F^a / (2 rho^a), on the equilibrium at u'
            feq = self.equilibrium(rho[a], up)
            fneq = self.f[a] - feq
            f1 = self.hermite_project(fneq) if p.collision == "regularized" else fneq
            edm = feq + (1.0 - 1.0 / self.tau[a]) * f1 + self.force_term(ua, F[a])
            # gray voxels: Eq. (3) in the second-order (Guo) form, with the
            # equilibrium, the non-equilibrium part and the force term all at
            # ua and the force term weighted by 1 - 1/(2 tau^a)
            geq = self.equilibrium(rho[a], ua)
            gneq = self.f[a] - geq
            g1 = self.hermite_project(gneq) if p.collision == "regularized" else gneq
            guo = (geq + (1.0 - 1.0 / self.tau[a]) * g1
                   + (1.0 - 0.5 / self.tau[a]) * self.force_term(ua, F[a]))
            post[a] = np.where(self.gray[None], guo, edm)
            post[a] = np.where(fl, post[a], 0.0)
        if self.ncomp == 2:
            self._residual(post, ev)
        self._outlet_flux(post)
        if self.exact_density:
            self._density_faces(post)
        elif self.open_x:
            self._reservoirs(post)
        new = np.empty_like(post)
        for a in range(self.ncomp):
            for i in range(Q):
                new[a, i] = np.where(self.src_solid[i], post[a, OPP[i]], _sh(post[a, i], C[i], -1))
                new[a, i] = np.where(fl, new[a, i], 0.0)
        self.f = new
        self.step_count += 1

    def _residual(self, post, ev):
        """Residual-component transfer on a saturation crossing (gray voxels)."""
        p = self.p
        S, rho, rhoT = ev["S"], ev["rho"], ev["rhoT"]
        m = p.m_minor
        to_w = self.gray & ~self.side & (S >= 0.5 + p.hyst)
        to_o = self.gray & self.side & (S <= 0.5 - p.hyst)
        rw, ro = self.r[0].copy(), self.r[1].copy()
        safe_w = np.where(self.fluid, rho[0], 1.0)
        safe_o = np.where(self.fluid, rho[1], 1.0)
        # oil -> water: release residual water, trap theta_o of the total as oil
        sc_w = (rho[0] + rw) / safe_w
        d_o = np.maximum(0.0, np.minimum(self.tho * rhoT - ro, rho[1] - m))
        sc_o = 1.0 - d_o / safe_o
        post[0] = np.where(to_w, post[0] * sc_w, post[0])
        post[1] = np.where(to_w, post[1] * sc_o, post[1])
        new_rw = np.where(to_w, 0.0, rw)
        new_ro = np.where(to_w, ro + d_o, ro)
        # water -> oil: release residual oil, trap theta_w of the total as water
        sc_o2 = (rho[1] + ro) / safe_o
        d_w = np.maximum(0.0, np.minimum(self.thw * rhoT - rw, rho[0] - m))
        sc_w2 = 1.0 - d_w / safe_w
        post[1] = np.where(to_o, post[1] * sc_o2, post[1])
        post[0] = np.where(to_o, post[0] * sc_w2, post[0])
        new_ro = np.where(to_o, 0.0, new_ro)
        new_rw = np.where(to_o, rw + d_w, new_rw)
        self.r[0], self.r[1] = new_rw, new_ro
        self.side = np.where(to_w, True, np.where(to_o, False, self.side))

    def _reservoirs(self, post):
        """Open x faces: the populations the reservoir cells send into the
        domain, written where the pull reads them (the slots across the
        periodic wrap, whose own populations leave the domain)."""
        p = self.p
        ends = []
        for x in (0, self.nx - 1):  # boundary planes: mixture velocity of the post set
            rho = post[:, :, :, :, x].sum(axis=(0, 1))
            mom = np.stack([np.einsum("i,aizy->zy", C[:, d].astype(float), post[:, :, :, :, x])
                            for d in range(3)])
            fl = self.fluid[:, :, x]
            ends.append(np.where(fl, mom / np.where(fl, rho, 1.0), 0.0))
        u_in, u_out = ends
        plane = (self.nz, self.ny)
        for a in range(self.ncomp):
            feq_in = self.equilibrium(np.full(plane, p.rho_in[a]), u_in)
            feq_out = self.equilibrium(np.full(plane, p.rho_out[a]), u_out)
            for i in range(Q):
                if C[i, 0] > 0:  # read by the voxels at x = 0 across the wrap
                    post[a, i][:, :, self.nx - 1] = feq_in[i]
                elif C[i, 0] < 0:  # read by the voxels at x = nx - 1
                    post[a, i][:, :, 0] = feq_out[i]

    def _pulled(self, post, a, j, xb):
        """Value that the voxels of plane xb pull in direction j from post
        (component a): post_j at x - c_j, or post_opp(j) at x when that source
        is solid; [z, y].  Only for sources inside the box (c_x of j pointing
        away from the face)."""
        cx, cy, cz = (int(v) for v in C[j])
        src = np.roll(post[a, j][:, :, xb - cx], (cz, cy), axis=(0, 1))
        return np.where(self.src_solid[j][:, :, xb], post[a, OPP[j]][:, :, xb], src)

    def _density_faces(self, post):
        """Exact density faces: the populations the boundary voxels pull across
        each x face, written into the slots they pull them from (the slots
        across the periodic wrap)."""
        p = self.p
        for xb, s, rho_b, wrap in ((0, 1, p.rho_in, self.nx - 1), (self.nx - 1, -1, p.rho_out, 0)):
            fl = self.fluid[:, :, xb]
            for a in range(self.ncomp):
                g = {j: self._pulled(post, a, j, xb) for j in range(Q) if C[j, 0] != s}
                s0 = sum(g[j] for j in g if C[j, 0] == 0)
                sm = sum(g[j] for j in g if C[j, 0] == -s)
                sJ = rho_b[a] - s0 - 2.0 * sm  # s * rho u_x
                Ny = 0.5 * sum(C[j, 1] * g[j] for j in g if C[j, 0] == 0)
                Nz = 0.5 * sum(C[j, 2] * g[j] for j in g if C[j, 0] == 0)
                for i in range(Q):
                    if C[i, 0] != s:
                        continue
                    val = g[OPP[i]] + 6.0 * W[i] * sJ - C[i, 1] * Ny - C[i, 2] * Nz
                    val = np.where(fl, val, 0.0)
                    # the voxel (z, y) pulls direction i from (z - c_z, y - c_y) across the wrap
                    post[a, i][:, :, wrap] = np.roll(val, (-int(C[i, 2]), -int(C[i, 1])), axis=(0, 1))

    def _outlet_flux(self, post):
        xf = int(self.p.outlet_x)
        x1 = (xf + 1) % self.nx
        Qv = np.zeros(2)
        for a in range(self.ncomp):
            tot = 0.0
            for i in range(Q):
                cx, cy, cz = (int(v) for v in C[i])
                if cx == 0:
                    continue
                src = xf if cx == 1 else x1
                dst = x1 if cx == 1 else xf
                fs = self.fluid[:, :, src]
                fd = np.roll(self.fluid[:, :, dst], (-cz, -cy), axis=(0, 1))
                ok = fs & fd
                tot += cx * float(np.sum(np.where(ok, post[a, i][:, :, src], 0.0)))
            Qv[a] = tot
        self.Q_last = Qv
        self.Q_acc = self.Q_acc + Qv

    # --------------------------------------------------------------- outputs
    def fields(self):
        ev = self.evaluate()
        fl = self.fluid
        out = dict(rho_w=np.where(fl, ev["rho"][0], 0.0),
                   rho_o=np.where(fl, ev["rho"][1], 0.0) if self.ncomp == 2 else np.zeros(self.shape),
                   ux=ev["u"][0], uy=ev["u"][1], uz=ev["u"][2], S=ev["S"],
                   r_w=self.r[0].copy(), r_o=self.r[1].copy())
        return out

    def diagnostics(self):
        ev = self.evaluate()
        fl = self.fluid
        phi = np.where(self.gray, self.phi, 1.0)
        mass = [float(np.sum(np.where(fl, ev["rho"][a], 0.0)) + np.sum(self.r[a]))
                for a in range(self.ncomp)]
        if self.ncomp == 1:
            mass.append(0.0)
        sw = float(np.sum(np.where(fl, phi * ev["S"], 0.0)) / np.sum(np.where(fl, phi, 0.0)))
        un = np.sqrt(ev["u"][0] ** 2 + ev["u"][1] ** 2 + ev["u"][2] ** 2)
        return dict(mass_w=mass[0], mass_o=mass[1], sw=sw, q_w=float(self.Q_last[0]),
                    q_o=float(self.Q_last[1]), q_acc_w=float(self.Q_acc[0]),
                    q_acc_o=float(self.Q_acc[1]), max_u=float(np.max(np.where(fl, un, 0.0))),
                    step=self.step_count, nonfinite=int(not np.all(np.isfinite(self.f))))

    def get_state(self):
        return dict(f=self.f.copy(), r=self.r.copy(), side=self.side.copy(),
                    step=self.step_count, Q_acc=self.Q_acc.copy(), Q_last=self.Q_last.copy())

    def set_state(self, st):
        self.f = st["f"].copy()
        self.r = st["r"].copy()
        self.side = st["side"].copy()
        self.step_count = st["step"]
        self.Q_acc = st["Q_acc"].copy()
        self.Q_last = st["Q_last"].copy()
