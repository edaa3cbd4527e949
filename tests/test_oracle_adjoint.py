"""Pins of the reference gradient (oracle/adjoint.py): its torch forward
reproduces model.Oracle's one-component run (fluxes and populations), and its
autograd gradient of L = sum_n a_n Q(n) with respect to the gray porosity
matches central finite differences of model.Oracle itself."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import adjoint as A
from oracle.lattice import C, Q


def case(collision="regularized", seed=5):
    rng = np.random.default_rng(seed)
    nz, ny, nx = 5, 6, 8
    r = rng.random((nz, ny, nx))
    cls = np.where(r < 0.15, 1, np.where(r < 0.6, 2, 0)).astype(np.uint8)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, cls.shape), np.where(cls == 0, 1.0, 0.0))
    K0 = W.kozeny_carman_table(2.0)
    tabs = [W.pore_table(K0, *W.brooks_corey_tables(0.05, 2.0, 0.1), phi_ref=0.3, pc_pm=0.05)]
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=1, tau=(0.8, 0.8), G=0.0, collision=collision,
                 g=((1e-4, 2e-5, 0.0), (0.0, 0.0, 0.0))).filled()
    return p, cls, phi, np.zeros(cls.shape, np.uint8), tabs


def oracle_history(p, cls, phi, pt, tabs, steps):
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(np.ones(cls.shape))
    f0 = o.f[0].copy()
    qs = []
    for _ in range(steps):
        o.step(1)
        qs.append(o.Q_last[0])
    return f0, np.array(qs), o.f[0]


@pytest.mark.parametrize("collision", ["regularized", "bgk"])
def test_torch_forward_equals_oracle(collision):
    p, cls, phi, pt, tabs = case(collision)
    f0, qs, fN = oracle_history(p, cls, phi, pt, tabs, 15)
    hist, _, f_t = A.flux_gradient(p, cls, phi, pt, tabs, f0, 15, np.ones(15))
    # Q is a signed sum of O(100) populations of size ~0.1: rounding order alone
    # leaves ~1e-15 absolute
    assert np.abs(hist - qs).max() < 1e-14
    assert np.abs(f_t - fN).max() < 1e-14


@pytest.mark.parametrize("collision", ["regularized", "bgk"])
def test_gradient_matches_oracle_finite_differences(collision):
    p, cls, phi, pt, tabs = case(collision)
    steps = 12
    a = np.linspace(1.0, 2.0, steps)            # L = sum_n a_n Q(n)
    f0, _, _ = oracle_history(p, cls, phi, pt, tabs, 1)
    _, grad, _ = A.flux_gradient(p, cls, phi, pt, tabs, f0, steps, a)
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(9)
    # L carries ~1e-15 of rounding noise against a sensitivity of ~1e-6, so
    # eps = 1e-4 (a tenth of a table interval); knots are kept out of reach
    eps = 1e-4
    checked = 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue  # a table knot within reach of the perturbation
        Ls = []
        for s in (1, -1):
            ph = phi.copy()
            ph[v] += s * eps
            _, qs, _ = oracle_history(p, cls, ph, pt, tabs, steps)
            Ls.append(float((a * qs).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        assert abs(grad[v] - fd) < 2e-5 * abs(fd) + 1e-12, (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3
    assert np.all(grad[cls != 2] == 0)


def tensor_case():
    """14^3 gray fibre bundles (3 cylinders), one component, tensorial
    resistivity with multipliers (1, 0.1, 0.1), a skewed body force."""
    wl = W.fiber_bundles(n=14, ncyl=3, precision="f64")
    p = wl["params"]
    p.outlet_x = 6
    p.g = ((1e-4, 3e-5, -2e-5), (0.0, 0.0, 0.0))
    return p, wl["cls"], wl["phi"], wl["ptype"], wl["tables"], wl["rho_w"]


def test_tensor_setup_and_forward_equal_oracle():
    import torch
    from oracle.tensor import inverse_permeability
    p, cls, phi, pt, tabs, rho = tensor_case()
    m = A.OneComponent(p, cls, pt, tabs)
    ph = torch.tensor(phi)
    K0 = m.K0(ph)
    Ki = m.Kinv(ph, K0).numpy()
    ref, aux = inverse_permeability(phi, cls, pt, K0.numpy(), tabs, p.sigma_s, p.smooth_radius,
                                    p.eps_g, p.eps_H, p.delta_tie)
    assert np.abs(Ki - ref).max() < 1e-13 * np.abs(ref).max()
    # the case exercises anisotropic axes (not only the isotropic gate)
    assert sum(not iso for iso, _ in aux["axes"].values()) > 100
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rho)
    f0 = o.f[0].copy()
    qs = []
    for _ in range(10):
        o.step(1)
        qs.append(o.Q_last[0])
    hist, _, fN = A.flux_gradient(p, cls, phi, pt, tabs, f0, 10, np.ones(10))
    assert np.abs(hist - np.array(qs)).max() < 1e-14
    assert np.abs(fN - o.f[0]).max() < 1e-14


def test_tensor_gradient_matches_oracle_finite_differences():
    """dL/dphi through K0(phi) and through K^-1(phi) (smoothing, Hessian,
    eigenvectors): perturbing one voxel moves K^-1 of every gray voxel within
    the smoothing radius."""
    p, cls, phi, pt, tabs, rho = tensor_case()
    steps = 10
    a = np.linspace(1.0, 2.0, steps)
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rho)
    _, grad, _ = A.flux_gradient(p, cls, phi, pt, tabs, o.f[0].copy(), steps, a)
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(3)
    eps = 1e-4
    checked = 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue
        Ls = []
        for s in (1, -1):
            ph = phi.copy()
            ph[v] += s * eps
            oo = Oracle(p)
            oo.set_geometry(cls, ph, pt, tabs)
            oo.init_fluid(rho)
            q = []
            for _ in range(steps):
                oo.step(1)
                q.append(oo.Q_last[0])
            Ls.append(float((a * np.array(q)).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        assert abs(grad[v] - fd) < 1e-4 * abs(fd) + 1e-12, (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3


def two_case(collision="regularized", seed=7):
    """20 x 8 x 6, two components (water in x < 10, oil beyond), random pore /
    solid / gray voxels with two pore types, kappa = 0, skewed body forces."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = 6, 8, 20
    r = rng.random((nz, ny, nx))
    cls = np.where(r < 0.15, 1, np.where(r < 0.5, 2, 0)).astype(np.uint8)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, cls.shape), np.where(cls == 0, 1.0, 0.0))
    pt = np.where(cls == 2, rng.integers(0, 2, cls.shape), 0).astype(np.uint8)
    K0 = W.kozeny_carman_table(2.0)
    tabs = [W.pore_table(K0, *W.brooks_corey_tables(0.05, lam, 0.1), phi_ref=0.225, pc_pm=0.05)
            for lam in (1.0, 2.0)]
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=2, tau=(0.8, 1.2), G=3.0, kappa=0.0,
                 collision=collision,
                 g=((1e-4, 2e-5, 0.0), (0.0, 0.0, -1e-5)), outlet_x=9).filled()
    m = p.m_minor
    x = np.arange(nx)[None, None, :]
    noise = 0.005 * rng.random(cls.shape)
    rw = np.where(x < 10, 1.0 - noise, m + noise)
    return p, cls, phi, pt, tabs, rw, 1.0 + m - rw


def _two_history(p, cls, phi, pt, tabs, rw, ro, steps):
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rw, ro)
    f0, r0, side0 = o.f.copy(), o.r.copy(), o.side.copy()
    q = []
    for _ in range(steps):
        o.step(1)
        q.append(o.Q_last[0])
    events = int(np.sum(o.side != side0)) + int(np.sum(o.r != r0))
    return f0, r0, np.array(q), o.f, events


def test_two_component_forward_equals_oracle():
    p, cls, phi, pt, tabs, rw, ro = two_case()
    f0, r0, q, fN, events = _two_history(p, cls, phi, pt, tabs, rw, ro, 10)
    assert events == 0  # the horizon has no residual event
    hist, _, f_t = A.flux_gradient2(p, cls, phi, pt, tabs, f0, r0, 10, np.ones(10))
    assert np.abs(hist - q).max() < 1e-14
    assert np.abs(f_t - fN).max() < 1e-14


def test_two_component_gradient_matches_oracle_finite_differences():
    """Through K0(phi) in the resistance and s_J(phi) in the capillary term."""
    p, cls, phi, pt, tabs, rw, ro = two_case()
    steps = 10
    a = np.linspace(1.0, 2.0, steps)
    f0, r0, _, _, _ = _two_history(p, cls, phi, pt, tabs, rw, ro, 1)
    _, grad, _ = A.flux_gradient2(p, cls, phi, pt, tabs, f0, r0, steps, a)
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(3)
    eps = 1e-4
    checked = 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue
        Ls = []
        for s in (1, -1):
            ph = phi.copy()
            ph[v] += s * eps
            _, _, q, _, ev = _two_history(p, cls, ph, pt, tabs, rw, ro, steps)
            assert ev == 0
            Ls.append(float((a * q).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        assert abs(grad[v] - fd) < 1e-4 * abs(fd) + 1e-12, (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3


def event_state(p, cls, phi, pt, tabs, rw, ro):
    """The two-component case with half of the gray voxels' side flags turned
    (seed 11) and some residual amounts, so that residual transfers fire."""
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rw, ro)
    S = o.evaluate()["S"]
    gray = cls == 2
    rng = np.random.default_rng(11)
    flip = gray & (rng.random(cls.shape) < 0.5)
    side = o.side.copy()
    side[flip] = ~side[flip]
    r = np.zeros((2,) + cls.shape)
    r[0] = np.where(gray & ~side & (S > 0.5), 0.01, 0.0)
    r[1] = np.where(gray & side & (S < 0.5), 0.02, 0.0)
    return side, r


def _event_history(p, cls, phi, pt, tabs, rw, ro, side, r, steps):
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rw, ro)
    o.side, o.r = side.copy(), r.copy()
    f0 = o.f.copy()
    q, events = [], 0
    for _ in range(steps):
        s0 = o.side.copy()
        o.step(1)
        q.append(o.Q_last[0])
        events += int(np.sum(o.side != s0))
    return f0, np.array(q), o.f, o.r, events


@pytest.mark.parametrize("kappa,region", [(0.0, "gray"), (-0.05, "gray"), (0.03, "all")])
def test_two_component_with_residual_events(kappa, region):
    """Residual transfers (trap and release) fire in this horizon, with and
    without the CSF control: the torch transcription follows the numpy oracle
    through them (theta_w, theta_o as functions of s_J equal the set-up's
    crossings), and its gradient, that of the branch each voxel took, matches
    central finite differences of the oracle at voxels whose perturbed runs
    take the same branches."""
    import torch
    p, cls, phi, pt, tabs, rw, ro = two_case()
    p.kappa, p.csf_region = kappa, region
    side, r = event_state(p, cls, phi, pt, tabs, rw, ro)
    steps = 10
    a = np.linspace(1.0, 2.0, steps)
    f0, q, fN, rN, events = _event_history(p, cls, phi, pt, tabs, rw, ro, side, r, steps)
    assert events > 100 and rN.max() > 0
    m = A.TwoComponent(p, cls, pt, tabs, r)
    ph = torch.tensor(phi)
    thw, tho = m.thetas(m.sJ(ph, m.K0(ph)))
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    assert np.abs(thw.numpy() - o.thw).max() < 1e-14 and np.abs(tho.numpy() - o.tho).max() < 1e-14
    assert o.tho.max() > 0  # both transfers trap something
    hist, grad, fT = A.flux_gradient2(p, cls, phi, pt, tabs, f0, r, steps, a, side=side)
    assert np.abs(hist - q).max() < 1e-14 and np.abs(fT - fN).max() < 1e-14
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(5)
    eps, checked = 1e-4, 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue
        Ls = []
        for s in (1, -1):
            ph2 = phi.copy()
            ph2[v] += s * eps
            _, qq, _, _, ev = _event_history(p, cls, ph2, pt, tabs, rw, ro, side, r, steps)
            assert ev == events
            Ls.append(float((a * qq).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        # L carries ~1e-15 of rounding: 1e-11 of finite-difference noise
        assert abs(grad[v] - fd) < 1e-4 * abs(fd) + 1e-6 * np.abs(grad).max(), (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3


def faces_case(seed=11, bc="density"):
    """One component between open x faces (exact density faces or pressure
    reservoirs): a gray slab (x = 4..6) with solid grains, grains on and next
    to both face planes, no body force, the flow driven by rho_in > rho_out."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = 4, 6, 11
    cls = np.zeros((nz, ny, nx), np.uint8)
    r = rng.random((nz, ny, nx))
    cls[:, :, 4:7] = np.where(r[:, :, 4:7] < 0.7, 2, 0)
    cls[:, :, 2:9] = np.where(r[:, :, 2:9] > 0.9, 1, cls[:, :, 2:9])
    for x in (0, 1, nx - 2, nx - 1):  # grains on and next to the face planes
        cls[:, :, x] = np.where(r[:, :, x] > 0.85, 1, 0)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, cls.shape), np.where(cls == 0, 1.0, 0.0))
    K0 = W.kozeny_carman_table(2.0)
    tabs = [W.pore_table(K0, *W.brooks_corey_tables(0.05, 2.0, 0.1), phi_ref=0.3, pc_pm=0.05)]
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=1, tau=(0.8, 0.8), G=0.0, bc_x=bc,
                 rho_in=(1.01, 0.0), rho_out=(0.99, 0.0), outlet_x=7).filled()
    return p, cls, phi, np.zeros(cls.shape, np.uint8), tabs


@pytest.mark.parametrize("bc", ["density", "pressure"])
def test_torch_forward_with_open_faces_equals_oracle(bc):
    p, cls, phi, pt, tabs = faces_case(bc=bc)
    f0, qs, fN = oracle_history(p, cls, phi, pt, tabs, 15)
    hist, _, f_t = A.flux_gradient(p, cls, phi, pt, tabs, f0, 15, np.ones(15))
    assert np.abs(hist - qs).max() < 1e-14
    assert np.abs(f_t - fN).max() < 1e-14


@pytest.mark.parametrize("bc", ["density", "pressure"])
def test_gradient_with_open_faces_matches_oracle_finite_differences(bc):
    p, cls, phi, pt, tabs = faces_case(bc=bc)
    steps = 12
    a = np.linspace(1.0, 2.0, steps)
    f0, _, _ = oracle_history(p, cls, phi, pt, tabs, 1)
    _, grad, _ = A.flux_gradient(p, cls, phi, pt, tabs, f0, steps, a)
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(3)
    eps = 1e-4
    checked = 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue
        Ls = []
        for s in (1, -1):
            ph = phi.copy()
            ph[v] += s * eps
            _, qs, _ = oracle_history(p, cls, ph, pt, tabs, steps)
            Ls.append(float((a * qs).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        assert abs(grad[v] - fd) < 2e-5 * abs(fd) + 1e-12, (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3


def two_faces_case(seed=13, bc="density"):
    """Two components between open x faces (exact density faces or pressure
    reservoirs; 22 x 8 x 6): water enters at
    x = 0 (rho_in = (1.02, m)) against oil held at x = nx - 1 (rho_out =
    (m, 1.0)); grains everywhere (face planes included), gray voxels (two pore
    types) two planes away
    from both faces; no body force, kappa = 0."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = 6, 8, 22
    r = rng.random((nz, ny, nx))
    cls = np.where(r < 0.15, 1, np.where(r < 0.5, 2, 0)).astype(np.uint8)
    cls[:, :, :2] = np.where(cls[:, :, :2] == 1, 1, 0)  # grains stay, no gray
    cls[:, :, -2:] = np.where(cls[:, :, -2:] == 1, 1, 0)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, cls.shape), np.where(cls == 0, 1.0, 0.0))
    pt = np.where(cls == 2, rng.integers(0, 2, cls.shape), 0).astype(np.uint8)
    K0 = W.kozeny_carman_table(2.0)
    tabs = [W.pore_table(K0, *W.brooks_corey_tables(0.05, lam, 0.1), phi_ref=0.225, pc_pm=0.05)
            for lam in (1.0, 2.0)]
    m = W.minority_density(3.0)
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=2, tau=(0.8, 1.2), G=3.0, kappa=0.0,
                 bc_x=bc, rho_in=(1.02, m), rho_out=(m, 1.0), outlet_x=12).filled()
    x = np.arange(nx)[None, None, :]
    noise = 0.005 * rng.random(cls.shape)
    rw = np.where(x < 6, 1.0 - noise, m + noise)
    return p, cls, phi, pt, tabs, rw, 1.0 + m - rw


@pytest.mark.parametrize("bc", ["density", "pressure"])
def test_two_component_forward_with_open_faces_equals_oracle(bc):
    p, cls, phi, pt, tabs, rw, ro = two_faces_case(bc=bc)
    f0, r0, q, fN, events = _two_history(p, cls, phi, pt, tabs, rw, ro, 10)
    assert events == 0
    hist, _, f_t = A.flux_gradient2(p, cls, phi, pt, tabs, f0, r0, 10, np.ones(10))
    assert np.abs(hist - q).max() < 1e-14
    assert np.abs(f_t - fN).max() < 1e-14


@pytest.mark.parametrize("bc", ["density", "pressure"])
def test_two_component_gradient_with_open_faces_matches_finite_differences(bc):
    p, cls, phi, pt, tabs, rw, ro = two_faces_case(bc=bc)
    steps = 10
    a = np.linspace(1.0, 2.0, steps)
    f0, r0, _, _, _ = _two_history(p, cls, phi, pt, tabs, rw, ro, 1)
    _, grad, _ = A.flux_gradient2(p, cls, phi, pt, tabs, f0, r0, steps, a)
    gray = np.argwhere(cls == 2)
    rng = np.random.default_rng(5)
    eps = 1e-4
    checked = 0
    for k in rng.permutation(len(gray)):
        v = tuple(gray[k])
        t = phi[v] * 1024
        if min(t - np.floor(t), np.ceil(t) - t) < 0.2:
            continue
        Ls = []
        for s in (1, -1):
            ph = phi.copy()
            ph[v] += s * eps
            _, _, q, _, ev = _two_history(p, cls, ph, pt, tabs, rw, ro, steps)
            assert ev == 0
            Ls.append(float((a * q).sum()))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        assert abs(grad[v] - fd) < 1e-4 * abs(fd) + 1e-12, (v, grad[v], fd)
        checked += 1
        if checked == 3:
            break
    assert checked == 3


def _faces_as_constants(monkeypatch):
    """Plants a mistake in the reference gradient: the populations the face
    step writes (the slots across the periodic wrap) are taken as constants."""
    orig_r, orig_d = A.OneComponent._reservoirs, A.OneComponent._density_faces

    def written(self, like):
        m = torch.zeros_like(like, dtype=torch.bool)
        for i in range(Q):
            if C[i, 0] > 0:
                m[i, :, :, -1] = True
            elif C[i, 0] < 0:
                m[i, :, :, 0] = True
        return m

    def res(self, posts):
        return [torch.where(written(self, o), o.detach(), o) for o in orig_r(self, posts)]

    def den(self, post, a):
        o = orig_d(self, post, a)
        return torch.where(written(self, o), o.detach(), o)
    monkeypatch.setattr(A.OneComponent, "_reservoirs", res)
    monkeypatch.setattr(A.OneComponent, "_density_faces", den)


@pytest.mark.parametrize("bc", ["density", "pressure"])
def test_gpu_face_cases_depend_on_the_face_step(bc, monkeypatch):
    """The GPU adjoint's open-face parity cases (faces_case and two_faces_case
    of test_gpu_adjoint) reach gray voxels through the face step within their
    step counts: with the face-written populations taken as constants the
    reference gradient moves by more than ten times those tests' fp32
    tolerances (2e-4 and 1e-3), so a GPU face transpose that dropped its
    dependence would fail them."""
    from test_gpu_adjoint import faces_case, two_faces_case, oracle_gradient

    def ne(x, ref):
        return np.abs(x - ref).max() / np.abs(ref).max()
    c = faces_case("f64", bc=bc)
    a = np.linspace(1.0, 2.0, 40)
    g = oracle_gradient(c, 40, a)[1]
    p, cls, phi, pt, tabs, rw, ro, steps = two_faces_case(bc)
    o = Oracle(p)
    o.set_geometry(cls, phi, pt, tabs)
    o.init_fluid(rw, ro)
    a2 = np.linspace(1.0, 2.0, steps)
    g2 = A.flux_gradient2(p, cls, phi, pt, tabs, o.f.copy(), o.r.copy(), steps, a2)[1]
    gray = cls == 2
    assert np.count_nonzero(g2[gray]) > 0.1 * gray.sum()
    _faces_as_constants(monkeypatch)
    d1 = ne(oracle_gradient(c, 40, a)[1], g)
    d2 = ne(A.flux_gradient2(p, cls, phi, pt, tabs, o.f.copy(), o.r.copy(), steps, a2)[1], g2)
    print(f"{bc}: planted-mistake change {d1:.2e} (one component), {d2:.2e} (two)")
    assert d1 > 10 * 2e-4 and d2 > 10 * 1e-3
