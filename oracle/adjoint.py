"""Reference gradients of the outlet-flux history with respect to the gray
porosity, for the one-component model (pore, gray and solid voxels, scalar
K0(phi) or the tensorial resistivity of Eqs. (6)-(7), regularised or BGK
collision, trapezoidal resistance, body force; periodic x faces, pressure
reservoirs or exact density faces as in model.Oracle).  TEST
INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).

The step is the one of model.Oracle with one component, and the tensor set-up
the one of tensor.inverse_permeability (smoothing, gradient and Hessian,
eigen-decomposition, ordering by |lambda|, gate and tie-break, Eq. (7)),
transcribed into plain PyTorch CPU fp64 operations so that torch's reverse-mode
autograd gives the exact gradient of this discrete forward map (through the
eigenvectors with torch.linalg.eigh's derivative); tests pin the transcription
to model.Oracle and tensor.inverse_permeability (same fluxes, populations and
K^-1) and the gradient to central finite differences of model.Oracle.  It
serves as the oracle of the GPU library's hand-written discrete adjoint.

Loss convention: the caller supplies dL/dQ(n) for the outlet fluxes
Q(1..N) of N steps (Q(n) measured on the post-collision set of step n, as
model.Oracle does); the result is dL/dphi on every voxel (zero off gray).
"""
from __future__ import annotations

import numpy as np
import torch

from .lattice import C, W, OPP, Q, CS2

PORE, SOLID, GRAY = 0, 1, 2


def _sh(a, c, sign=1):
    """a evaluated at x + sign*c (periodic); a is [..., z, y, x]."""
    cx, cy, cz = (int(v) * sign for v in c)
    return torch.roll(a, (-cz, -cy, -cx), dims=(-3, -2, -1))


def _lerp(tab, v):
    """Linear interpolation of a 1025-sample table at v (differentiable in v)."""
    tab = torch.as_tensor(np.asarray(tab, np.float64))
    n = tab.shape[0] - 1
    t = v * n
    k = torch.clamp(torch.floor(t.detach()), 0, n - 1).long()
    return tab[k] + (t - k) * (tab[k + 1] - tab[k])


def _equilibrium(rho, u):
    usq = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    out = []
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out.append(W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2)))
    return torch.stack(out)


def _force_term(u, F):
    uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2]
    out = []
    for i in range(Q):
        cF = C[i, 0] * F[0] + C[i, 1] * F[1] + C[i, 2] * F[2]
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out.append(W[i] * (cF / CS2 + (2.0 * cu * cF - 2.0 * CS2 * uF) / (2 * CS2 * CS2)))
    return torch.stack(out)


def _collide(f, rho, up, ua, F, tau, collision, gray):
    """Post-collision set of one component: pore voxels take the equilibrium
    at u' and Eq. (3) at ua as the exact-difference increment; gray voxels take
    Eq. (3) in its second-order form, equilibrium and non-equilibrium part at
    ua and the force term weighted by 1 - 1/(2 tau)."""
    def one(ue, kf):
        feq = _equilibrium(rho, ue)
        fneq = f - feq
        f1 = _hermite(fneq) if collision == "regularized" else fneq
        return feq + (1.0 - 1.0 / tau) * f1 + kf * _force_term(ua, F)
    return torch.where(gray, one(ua, 1.0 - 0.5 / tau), one(up, 1.0))


def _hermite(fneq):
    j = [sum(C[i, a] * fneq[i] for i in range(Q) if C[i, a]) for a in range(3)]
    Pi = [[sum(C[i, a] * C[i, b] * fneq[i] for i in range(Q) if C[i, a] and C[i, b])
           for b in range(3)] for a in range(3)]
    trace = Pi[0][0] + Pi[1][1] + Pi[2][2]
    out = []
    for i in range(Q):
        cj = C[i, 0] * j[0] + C[i, 1] * j[1] + C[i, 2] * j[2]
        pcc = sum(Pi[a][b] * float(C[i, a] * C[i, b]) for a in range(3) for b in range(3)
                  if C[i, a] and C[i, b])
        out.append(W[i] * (cj / CS2 + (pcc - CS2 * trace) / (2 * CS2 * CS2)))
    return torch.stack(out)


def _roll(a, dx=0, dy=0, dz=0):
    """a at (x+dx, y+dy, z+dz), periodic, for [z, y, x] arrays."""
    return torch.roll(a, (-dz, -dy, -dx), dims=(0, 1, 2))


def _smooth(a, sigma, radius):
    """Periodic separable Gaussian (weights normalised to 1), z then y then x."""
    j = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-j * j / (2.0 * sigma * sigma))
    w = w / w.sum()
    out = a
    for dim in (0, 1, 2):
        acc = torch.zeros_like(out)
        for jj, wj in zip(range(-radius, radius + 1), w):
            acc = acc + float(wj) * torch.roll(out, -jj, dims=dim)
        out = acc
    return out


def inverse_permeability(phi, cls, ptype, K0, tables, p):
    """K^-1 [6, z, y, x] (xx, yy, zz, xy, xz, yz; zero off gray) as a function
    of the porosity tensor phi and the K0 field: the smoothed porosity (solid
    0, pore 1), its central-difference gradient and Hessian, the eigenpairs
    of the Hessian ordered by ascending |lambda|, the isotropic gate, the
    tie-break that turns the second axis along the gradient's part normal to
    the third, and K^-1 = sum_k e_k e_k^T / (a_k K0)."""
    gray = torch.as_tensor(cls == GRAY)
    base = torch.where(gray, phi, torch.as_tensor(np.where(cls == PORE, 1.0, 0.0)))
    ps = _smooth(base, float(p.sigma_s), int(p.smooth_radius))
    off = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    g = [0.5 * (_roll(ps, *off[a]) - _roll(ps, *[-v for v in off[a]])) for a in range(3)]
    H = [[None] * 3 for _ in range(3)]
    for a in range(3):
        H[a][a] = _roll(ps, *off[a]) - 2.0 * ps + _roll(ps, *[-v for v in off[a]])
        for b in range(a + 1, 3):
            ea, eb = off[a], off[b]
            pp = _roll(ps, *[u + v for u, v in zip(ea, eb)])
            pm = _roll(ps, *[u - v for u, v in zip(ea, eb)])
            mp = _roll(ps, *[-u + v for u, v in zip(ea, eb)])
            mm = _roll(ps, *[-u - v for u, v in zip(ea, eb)])
            H[a][b] = H[b][a] = 0.25 * (pp - pm - mp + mm)
    idx = np.nonzero(cls == GRAY)
    H3 = torch.stack([torch.stack([H[a][b][idx] for b in range(3)], -1) for a in range(3)], -2)
    g3 = torch.stack([g[a][idx] for a in range(3)], -1)
    lam, vec = torch.linalg.eigh(H3)
    order = torch.argsort(lam.detach().abs(), dim=-1, stable=True)
    lam = torch.gather(lam, -1, order)
    E = torch.gather(vec, -1, order[:, None, :].expand(-1, 3, -1))
    al = lam.abs()
    e3 = E[:, :, 2]
    pv = g3 - (g3 * e3).sum(-1, keepdim=True) * e3
    pn = pv.norm(dim=-1)
    tie = ((al[:, 1] - al[:, 0]) <= float(p.delta_tie) * al[:, 2]) & (pn > float(p.eps_g))
    e2t = pv / torch.where(tie, pn, torch.ones_like(pn))[:, None]
    e1t = torch.linalg.cross(e3, e2t, dim=-1)
    e1t = e1t / torch.where(tie, e1t.norm(dim=-1), torch.ones_like(pn))[:, None]
    E = torch.stack([torch.where(tie[:, None], e1t, E[:, :, 0]),
                     torch.where(tie[:, None], e2t, E[:, :, 1]), e3], -1)
    iso = (al.max(-1).values <= float(p.eps_H)) & (g3.norm(dim=-1) <= float(p.eps_g))
    kd = torch.as_tensor(np.array([tables[int(t)]["kd"] for t in ptype[idx]], np.float64))
    k0 = K0[idx]
    M = sum(E[:, :, k, None] * E[:, None, :, k] / (kd[:, k] * k0)[:, None, None]
            for k in range(3))
    M = torch.where(iso[:, None, None], torch.eye(3, dtype=torch.float64) / k0[:, None, None], M)
    out = torch.zeros((6,) + cls.shape, dtype=torch.float64)
    comps = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    return torch.stack([out[c].index_put(tuple(torch.as_tensor(i) for i in idx), M[:, a, b])
                        for c, (a, b) in enumerate(comps)])


class OneComponent:
    """The one-component step in torch; `phi` is a leaf tensor when gradients
    are wanted."""

    def __init__(self, params, cls, ptype, tables):
        p = params
        self.p = p
        self.cls = np.asarray(cls, np.uint8)
        self.shape = self.cls.shape
        self.solid = torch.as_tensor(self.cls == SOLID)
        self.fluid = ~self.solid
        self.gray = torch.as_tensor(self.cls == GRAY)
        self.ptype = np.asarray(ptype, np.uint8)
        self.tables = tables
        self.tau = float(p.tau[0])
        self.g = [float(v) for v in p.g[0]]
        self.tensor = bool(getattr(p, "tensor", False))
        self.src_solid = [_sh(self.solid, C[i], -1) for i in range(Q)]
        bc = getattr(p, "bc_x", "periodic")
        self.faces = bc == "density"
        self.res = bc == "pressure"
        self.open_x = self.faces or self.res
        if self.open_x:
            # a pull across an x face reads the slot the face step wrote, never
            # bounce-back
            nx = self.shape[2]
            for i in range(Q):
                if C[i, 0] != 0:
                    xs = 0 if C[i, 0] > 0 else nx - 1
                    m = self.src_solid[i].clone()
                    m[:, :, xs] = False
                    self.src_solid[i] = m
        fl = self.fluid.numpy()
        xf = int(p.outlet_x)
        x1 = (xf + 1) % self.shape[2]
        # outlet-flux links through x_f | x_f + 1 with both ends fluid: weight
        # +1 on post_i(x_f) for c_x = +1, -1 on post_i(x_f + 1) for c_x = -1
        self.flux_w = torch.zeros((Q,) + self.shape, dtype=torch.float64)
        for i in range(Q):
            cx, cy, cz = (int(v) for v in C[i])
            if cx == 0:
                continue
            src, dst = (xf, x1) if cx == 1 else (x1, xf)
            ok = fl[:, :, src] & np.roll(fl[:, :, dst], (-cz, -cy), axis=(0, 1))
            self.flux_w[i][:, :, src] = torch.as_tensor(cx * ok.astype(np.float64))

    def K0(self, phi):
        K0 = torch.zeros(self.shape, dtype=torch.float64)
        for t, tab in enumerate(self.tables):
            sel = torch.as_tensor((self.cls == GRAY) & (self.ptype == t))
            if bool(sel.any()):
                K0 = torch.where(sel, _lerp(tab["K0"], phi), K0)
        return K0

    def Kinv(self, phi, K0):
        return inverse_permeability(phi, self.cls, self.ptype, K0, self.tables, self.p)

    def step(self, f, K0, Kinv=None):
        """One step from the post-streaming set f; returns (new f, Q).  With
        the tensorial resistivity Kinv is K^-1 [6, z, y, x]."""
        p = self.p
        fl = self.fluid
        rho = f.sum(0)
        mom = [sum(C[i, d] * f[i] for i in range(Q) if C[i, d]) for d in range(3)]
        safe = torch.where(fl, rho, torch.ones_like(rho))
        F_ex = [rho * self.g[d] for d in range(3)]
        nu = CS2 * (self.tau - 0.5)
        cR = torch.where(self.gray, rho * nu, torch.zeros_like(rho))
        b = [mom[d] + 0.5 * F_ex[d] for d in range(3)]
        if Kinv is None:
            Rs = torch.where(self.gray, cR / torch.where(self.gray, K0, torch.ones_like(K0)),
                             torch.zeros_like(rho))
            Ru = [Rs * (b[d] / (safe + 0.5 * Rs)) for d in range(3)]
        else:
            comp = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}
            R = [[cR * Kinv[comp[(min(a, c), max(a, c))]] for c in range(3)] for a in range(3)]
            A = torch.stack([torch.stack([0.5 * R[a][c] + (safe if a == c else 0.0)
                                          for c in range(3)], -1) for a in range(3)], -2)
            u = torch.linalg.solve(A, torch.stack(b, -1)[..., None])[..., 0]
            Ru = [sum(R[a][c] * u[..., c] for c in range(3)) for a in range(3)]
        F = [F_ex[d] - Ru[d] for d in range(3)]
        up = [torch.where(fl, mom[d] / safe, torch.zeros_like(rho)) for d in range(3)]
        ua = [up[d] + F[d] / (2.0 * safe) for d in range(3)]
        post = _collide(f, rho, up, ua, F, self.tau, p.collision, self.gray)
        post = torch.where(fl, post, torch.zeros_like(post))
        Qn = (self.flux_w * post).sum()
        if self.faces:
            post = self._density_faces(post, 0)
        elif self.res:
            post = self._reservoirs([post])[0]
        new = torch.stack([torch.where(self.src_solid[i], post[OPP[i]], _sh(post[i], C[i], -1))
                           for i in range(Q)])
        return torch.where(fl, new, torch.zeros_like(new)), Qn

    def _reservoirs(self, posts):
        """Pressure reservoirs (model.Oracle._reservoirs) on the post sets of
        all components: the slots across the periodic wrap that the boundary
        voxels pull take the equilibrium at the reservoir density and at the
        mixture velocity of the boundary voxel of the same (y, z) row (zero
        when it is solid); the inlet sends c_x = +1, the outlet c_x = -1."""
        p = self.p
        nx = self.shape[2]
        ends = []
        for x in (0, nx - 1):
            rho = sum(post[:, :, :, x].sum(0) for post in posts)
            mom = [sum(C[i, d] * post[i][:, :, x] for post in posts for i in range(Q) if C[i, d])
                   for d in range(3)]
            fl = self.fluid[:, :, x]
            safe = torch.where(fl, rho, torch.ones_like(rho))
            ends.append([torch.where(fl, mom[d] / safe, torch.zeros_like(rho)) for d in range(3)])
        out = []
        for a, post in enumerate(posts):
            feq = [_equilibrium(torch.full_like(ends[0][0], float(r)), u)
                   for r, u in ((p.rho_in[a], ends[0]), (p.rho_out[a], ends[1]))]
            slots = [post[i] for i in range(Q)]
            for i in range(Q):
                if C[i, 0] == 0:
                    continue
                e, col = (0, nx - 1) if C[i, 0] > 0 else (1, 0)
                plane = [slots[i][:, :, x] for x in range(nx)]
                plane[col] = feq[e][i]
                slots[i] = torch.stack(plane, dim=-1)
            out.append(torch.stack(slots))
        return out

    def _density_faces(self, post, a):
        """Exact density faces (model.Oracle._density_faces) for component a:
        the populations the face voxels pull across each x face, written into
        the slots they pull them from."""
        p = self.p
        nx = self.shape[2]
        slots = [post[i] for i in range(Q)]
        for xb, s, rho_b, wrap in ((0, 1, p.rho_in[a], nx - 1), (nx - 1, -1, p.rho_out[a], 0)):
            fl = self.fluid[:, :, xb]
            g = {}
            for j in range(Q):
                if C[j, 0] == s:
                    continue
                cx, cy, cz = (int(v) for v in C[j])
                src = torch.roll(post[j][:, :, xb - cx], (cz, cy), dims=(0, 1))
                g[j] = torch.where(self.src_solid[j][:, :, xb], post[OPP[j]][:, :, xb], src)
            s0 = sum(g[j] for j in g if C[j, 0] == 0)
            sm = sum(g[j] for j in g if C[j, 0] == -s)
            sJ = rho_b - s0 - 2.0 * sm
            Ny = 0.5 * sum(C[j, 1] * g[j] for j in g if C[j, 0] == 0)
            Nz = 0.5 * sum(C[j, 2] * g[j] for j in g if C[j, 0] == 0)
            for i in range(Q):
                if C[i, 0] != s:
                    continue
                val = g[OPP[i]] + 6.0 * W[i] * sJ - C[i, 1] * Ny - C[i, 2] * Nz
                val = torch.where(fl, val, torch.zeros_like(val))
                val = torch.roll(val, (-int(C[i, 2]), -int(C[i, 1])), dims=(0, 1))
                plane = [slots[i][:, :, x] for x in range(nx)]
                plane[wrap] = val
                slots[i] = torch.stack(plane, dim=-1)
        return torch.stack(slots)


def flux_gradient(params, cls, phi, ptype, tables, f0, steps, dL_dQ):
    """Runs `steps` steps from the post-streaming set f0 [Q, z, y, x] and
    returns (Q history [steps], dL/dphi [z, y, x]) for L = sum_n dL_dQ[n] Q(n)."""
    model = OneComponent(params, cls, ptype, tables)
    ph = torch.tensor(np.asarray(phi, np.float64), requires_grad=True)
    K0 = model.K0(ph)
    Kinv = model.Kinv(ph, K0) if model.tensor else None
    f = torch.as_tensor(np.asarray(f0, np.float64))
    hist = []
    for _ in range(int(steps)):
        f, Qn = model.step(f, K0, Kinv)
        hist.append(Qn)
    hist = torch.stack(hist)
    L = (hist * torch.as_tensor(np.asarray(dL_dQ, np.float64))).sum()
    L.backward()
    g = ph.grad.detach().numpy()
    return hist.detach().numpy(), np.where(np.asarray(cls) == GRAY, g, 0.0), f.detach().numpy()


class TwoComponent(OneComponent):
    """The two-component step in torch (Sec. II): the pseudo-potential force
    with wall virtual densities, the CSF surface-tension control of Eq. (4)
    (normals of the other component's density gradient, curvature as their
    divergence, both with the voxel's own value across a solid link), the
    capillary term of Eq. (1) with P_c = s_J(phi) P_c(S) and the gradient of
    the mobile saturation, the resistance c_R = sum_b rho S^b nu^b / max(Kr^b,
    Kr_min) with K0(phi) or K^-1(phi), the common velocity u' and per-component
    collision with the force term at u' + F^a / (2 rho^a), then the residual
    transfer on a saturation crossing (trap and release, with theta_w and
    theta_o the crossings of s_J(phi) P_c with c_max Pc_PM and c_min Pc_PM).
    The events are switches: the gradient is that of the branch each voxel
    takes (the crossing test is made on detached values).  r [2, z, y, x]
    holds the residual amounts at the start."""

    def __init__(self, params, cls, ptype, tables, r):
        super().__init__(params, cls, ptype, tables)
        p = params
        self.region = torch.as_tensor(self.cls == GRAY) if p.csf_region == "gray" else self.fluid
        self.taus = [float(t) for t in p.tau]
        self.gs = [[float(v) for v in p.g[a]] for a in range(2)]
        self.r = torch.as_tensor(np.asarray(r, np.float64))
        self.nb_solid = [_sh(self.solid, C[i]) for i in range(Q)]
        # open faces: a neighbour across an x face is the reservoir cell
        # (fluid, at the face's prescribed density), as in model.Oracle
        self.cross_nb = [None] * Q
        if self.open_x:
            nx = self.shape[2]
            for i in range(1, Q):
                if C[i, 0] != 0:
                    xb = nx - 1 if C[i, 0] > 0 else 0
                    m = torch.zeros(self.shape, dtype=torch.bool)
                    m[:, :, xb] = True
                    self.cross_nb[i] = m
                    self.nb_solid[i] = self.nb_solid[i] & ~m

    def sJ(self, phi, K0):
        out = torch.zeros(self.shape, dtype=torch.float64)
        for t, tab in enumerate(self.tables):
            sel = torch.as_tensor((self.cls == GRAY) & (self.ptype == t))
            if bool(sel.any()):
                ref = torch.tensor(float(tab["phi_ref"]), dtype=torch.float64)
                k0ref = _lerp(tab["K0"], ref).item()
                safe_k = torch.where(sel, K0, torch.ones_like(K0))
                ph_ = torch.where(sel, phi, torch.ones_like(phi))
                val = torch.sqrt((k0ref / tab["phi_ref"]) / (safe_k / ph_))
                out = torch.where(sel, val, out)
        return out

    def _nb(self, X, i):
        return torch.where(self.nb_solid[i], X, _sh(X, C[i]))

    def _grad(self, X):
        """Isotropic gradient with the voxel's own value across a solid link."""
        g = [0.0, 0.0, 0.0]
        for i in range(1, Q):
            v = self._nb(X, i)
            for d in range(3):
                if C[i, d]:
                    g[d] = g[d] + (W[i] * C[i, d] / CS2) * v
        return g

    def thetas(self, sJ):
        """theta_w, theta_o of the gray voxels as functions of s_J: the smallest
        S where the non-increasing s_J P_c(S) equals c Pc_PM (0 when it never
        does), theta_w at c_max, theta_o = 1 - S at c_min."""
        p = self.p
        thw = torch.zeros(self.shape, dtype=torch.float64)
        tho = torch.zeros(self.shape, dtype=torch.float64)
        sj_d = sJ.detach().numpy()
        for t, tab in enumerate(self.tables):
            sel = (self.cls == GRAY) & (self.ptype == t)
            if not sel.any():
                continue
            pc = np.asarray(tab["Pc"], np.float64)
            n = len(pc) - 1
            for c, is_w in ((p.c_max, True), (p.c_min, False)):
                target = c * tab["Pc_PM"]
                kk = np.zeros(self.shape, np.int64)
                found = np.zeros(self.shape, bool)
                for idx in zip(*np.nonzero(sel)):
                    y = sj_d[idx] * pc
                    if y[0] < target or y[n] > target:
                        continue
                    found[idx] = True
                    kk[idx] = int(np.argmax(y <= target))
                km = np.maximum(kk, 1)
                a = sJ * torch.as_tensor(pc[km - 1])
                b = sJ * torch.as_tensor(pc[km])
                sstar = ((torch.as_tensor(km - 1, dtype=torch.float64)
                          + (a - target) / torch.where(torch.as_tensor(found), a - b,
                                                       torch.ones_like(a))) / n)
                sstar = torch.where(torch.as_tensor(found & (kk > 0)), sstar, torch.zeros_like(a))
                val = sstar if is_w else 1.0 - sstar
                val = torch.where(torch.as_tensor(found), val, torch.zeros_like(a))
                if is_w:
                    thw = torch.where(torch.as_tensor(sel), val, thw)
                else:
                    tho = torch.where(torch.as_tensor(sel), val, tho)
        return thw, tho

    def step2(self, f, K0, sJ, Kinv=None, r=None, side=None, thw=None, tho=None):
        """One step from the post-streaming sets f [2, Q, z, y, x] with
        residual amounts r and side flags side; returns (new f, Q^w, new r,
        new side).  Without side flags no residual transfer is made."""
        p = self.p
        if r is None:
            r = self.r
        fl = self.fluid
        rho = [f[a].sum(0) for a in range(2)]
        mom = [[sum(C[i, d] * f[a][i] for i in range(Q) if C[i, d]) for d in range(3)]
               for a in range(2)]
        rho_t = rho[0] + rho[1]
        safe = torch.where(fl, rho_t, torch.ones_like(rho_t))
        F_ex = [[rho[a] * self.gs[a][d] for d in range(3)] for a in range(2)]
        span = p.s_max - p.s_min
        tw, to = rho[0] + r[0], rho[1] + r[1]
        s = torch.where(fl, tw / torch.where(fl, tw + to, torch.ones_like(tw)), torch.zeros_like(tw))
        S = torch.clamp((s - p.s_min) / span, 0.0, 1.0)
        S_hat = torch.where(fl, (rho[0] / safe - p.s_min) / span, torch.zeros_like(tw))
        for a in range(2):
            b = 1 - a
            wall = torch.clamp(rho[b] + p.wall_dpsi[b], min=0.0)
            acc = [0.0, 0.0, 0.0]
            for i in range(1, Q):
                psi = torch.where(self.nb_solid[i], wall, _sh(rho[b], C[i]))
                if self.cross_nb[i] is not None:
                    ghost = p.rho_out[b] if C[i, 0] > 0 else p.rho_in[b]
                    psi = torch.where(self.cross_nb[i], torch.full_like(psi, ghost), psi)
                for d in range(3):
                    if C[i, d]:
                        acc[d] = acc[d] + W[i] * C[i, d] * psi
            for d in range(3):
                F_ex[a][d] = F_ex[a][d] - p.G * rho[a] * acc[d]
        if p.kappa != 0.0:
            for a in range(2):
                b = 1 - a
                gr = self._grad(rho[b])
                nrm = torch.sqrt(gr[0] ** 2 + gr[1] ** 2 + gr[2] ** 2)
                big = nrm > p.eps_n
                safe_n = torch.where(big, nrm, torch.ones_like(nrm))
                nhat = [torch.where(big, gr[d] / safe_n, torch.zeros_like(nrm)) for d in range(3)]
                div = 0.0
                for i in range(1, Q):
                    for d in range(3):
                        if C[i, d]:
                            div = div + (W[i] * C[i, d] / CS2) * self._nb(nhat[d], i)
                curv = -div
                for d in range(3):
                    fc = p.kappa * curv * gr[d] * rho[a] / (p.phi_avg * p.phi_max)
                    F_ex[a][d] = F_ex[a][d] + torch.where(self.region, fc, torch.zeros_like(fc))
        gS = [0.0, 0.0, 0.0]
        for i in range(1, Q):
            v = self._nb(S_hat, i)
            for d in range(3):
                if C[i, d]:
                    gS[d] = gS[d] + (W[i] * C[i, d] / CS2) * v
        Pc = torch.zeros(self.shape, dtype=torch.float64)
        Krw = torch.zeros(self.shape, dtype=torch.float64)
        Kro = torch.zeros(self.shape, dtype=torch.float64)
        for t, tab in enumerate(self.tables):
            sel = torch.as_tensor((self.cls == GRAY) & (self.ptype == t))
            if bool(sel.any()):
                Pc = torch.where(sel, sJ * _lerp(tab["Pc"], S), Pc)
                Krw = torch.where(sel, _lerp(tab["Krw"], S), Krw)
                Kro = torch.where(sel, _lerp(tab["Kro"], S), Kro)
        for a in range(2):
            for d in range(3):
                F_ex[a][d] = F_ex[a][d] + torch.where(self.gray, -Pc * (rho[a] / safe) * gS[d],
                                                      torch.zeros_like(Pc))
        nu = [CS2 * (t - 0.5) for t in self.taus]
        Sw, So = S, 1.0 - S
        cw = torch.where(Sw > 0, rho_t * Sw * nu[0] / torch.clamp(Krw, min=p.kr_min),
                         torch.zeros_like(S))
        co = torch.where(So > 0, rho_t * So * nu[1] / torch.clamp(Kro, min=p.kr_min),
                         torch.zeros_like(S))
        cR = torch.where(self.gray, cw + co, torch.zeros_like(S))
        b = [mom[0][d] + mom[1][d] + 0.5 * (F_ex[0][d] + F_ex[1][d]) for d in range(3)]
        if Kinv is None:
            Rs = torch.where(self.gray, cR / torch.where(self.gray, K0, torch.ones_like(K0)),
                             torch.zeros_like(S))
            Ru = [Rs * (b[d] / (safe + 0.5 * Rs)) for d in range(3)]
        else:
            comp = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}
            R = [[cR * Kinv[comp[(min(a, c), max(a, c))]] for c in range(3)] for a in range(3)]
            A = torch.stack([torch.stack([0.5 * R[a][c] + (safe if a == c else 0.0)
                                          for c in range(3)], -1) for a in range(3)], -2)
            u = torch.linalg.solve(A, torch.stack(b, -1)[..., None])[..., 0]
            Ru = [sum(R[a][c] * u[..., c] for c in range(3)) for a in range(3)]
        F = [[F_ex[a][d] - (rho[a] / safe) * Ru[d] for d in range(3)] for a in range(2)]
        den = rho[0] / self.taus[0] + rho[1] / self.taus[1]
        den = torch.where(fl, den, torch.ones_like(den))
        up = [torch.where(fl, (mom[0][d] / self.taus[0] + mom[1][d] / self.taus[1]) / den,
                          torch.zeros_like(den)) for d in range(3)]
        posts = []
        for a in range(2):
            ra = torch.where(fl, 2.0 * rho[a], torch.ones_like(rho[a]))
            ua = [up[d] + F[a][d] / ra for d in range(3)]
            post = _collide(f[a], rho[a], up, ua, F[a], self.taus[a], p.collision, self.gray)
            posts.append(torch.where(fl, post, torch.zeros_like(post)))
        if side is not None:
            Sd = S.detach()
            g = torch.as_tensor(self.cls == GRAY)
            to_w = g & ~side & (Sd >= 0.5 + p.hyst)
            to_o = g & side & (Sd <= 0.5 - p.hyst)
            rhoT = tw + to
            m = p.m_minor
            sw_ = torch.where(fl, rho[0], torch.ones_like(rho[0]))
            so_ = torch.where(fl, rho[1], torch.ones_like(rho[1]))
            # oil -> water: release residual water, trap theta_o of the total as oil
            sc_w = (rho[0] + r[0]) / sw_
            d_o = torch.clamp(torch.minimum(tho * rhoT - r[1], rho[1] - m), min=0.0)
            sc_o = 1.0 - d_o / so_
            # water -> oil: release residual oil, trap theta_w of the total as water
            sc_o2 = (rho[1] + r[1]) / so_
            d_w = torch.clamp(torch.minimum(thw * rhoT - r[0], rho[0] - m), min=0.0)
            sc_w2 = 1.0 - d_w / sw_
            s0 = torch.where(to_w, sc_w, torch.where(to_o, sc_w2, torch.ones_like(sc_w)))
            s1 = torch.where(to_w, sc_o, torch.where(to_o, sc_o2, torch.ones_like(sc_o)))
            posts = [posts[0] * s0, posts[1] * s1]
            r = torch.stack([torch.where(to_w, torch.zeros_like(r[0]),
                                         torch.where(to_o, r[0] + d_w, r[0])),
                             torch.where(to_w, r[1] + d_o,
                                         torch.where(to_o, torch.zeros_like(r[1]), r[1]))])
            side = torch.where(to_w, torch.ones_like(side), torch.where(to_o, torch.zeros_like(side),
                                                                        side))
        Qn = (self.flux_w * posts[0]).sum()
        if self.faces:
            posts = [self._density_faces(posts[a], a) for a in range(2)]
        elif self.res:
            posts = self._reservoirs(posts)
        new = []
        for a in range(2):
            na = torch.stack([torch.where(self.src_solid[i], posts[a][OPP[i]],
                                          _sh(posts[a][i], C[i], -1)) for i in range(Q)])
            new.append(torch.where(fl, na, torch.zeros_like(na)))
        return torch.stack(new), Qn, r, side


def flux_gradient2(params, cls, phi, ptype, tables, f0, r, steps, dL_dQ, side=None):
    """Two components: runs `steps` steps from the post-streaming sets f0
    [2, Q, z, y, x] with residual amounts r [2, z, y, x] (and, when side
    flags are given, the residual transfer) and returns (Q^w history, dL/dphi,
    final f) for L = sum_n dL_dQ[n] Q^w(n), through K0(phi) (or K^-1(phi)) in
    the resistance, s_J(phi) in the capillary term and theta_w, theta_o(s_J)
    in the residual transfer."""
    model = TwoComponent(params, cls, ptype, tables, r)
    ph = torch.tensor(np.asarray(phi, np.float64), requires_grad=True)
    K0 = model.K0(ph)
    sJ = model.sJ(ph, K0)
    Kinv = model.Kinv(ph, K0) if model.tensor else None
    thw = tho = None
    rr = torch.as_tensor(np.asarray(r, np.float64))
    sd = None
    if side is not None:
        thw, tho = model.thetas(sJ)
        sd = torch.as_tensor(np.asarray(side, bool))
    f = torch.as_tensor(np.asarray(f0, np.float64))
    hist = []
    for _ in range(int(steps)):
        f, Qn, rr, sd = model.step2(f, K0, sJ, Kinv, rr, sd, thw, tho)
        hist.append(Qn)
    hist = torch.stack(hist)
    L = (hist * torch.as_tensor(np.asarray(dL_dQ, np.float64))).sum()
    L.backward()
    g = ph.grad.detach().numpy()
    return hist.detach().numpy(), np.where(np.asarray(cls) == GRAY, g, 0.0), f.detach().numpy()
