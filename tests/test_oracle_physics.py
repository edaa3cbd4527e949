"""Oracle pins against closed forms and invariants: exact mass conservation
with residual events, momentum conservation of the pseudo-potential force,
the uniform-Darcy steady state of the resistance (scalar and tensorial),
Darcy's law for pressure-driven flow through a gray slab from weak to very
strong resistance, Poiseuille flow with halfway bounce-back, Brinkman channel
convergence, the flat-interface capillary pressure jump of Eq. (1) (and its
persistence under a resistance 5e4 times the density), mirror symmetry and
checkpoint/resume."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Oracle, CS2


def _oracle(wl, **over):
    p = wl["params"]
    for k, v in over.items():
        setattr(p, k, v)
    o = Oracle(p)
    o.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    o.init_fluid(wl["rho_w"], wl["rho_o"])
    return o


def test_mass_conservation_with_residual_events():
    wl = W.droplet_slab()
    o = _oracle(wl)
    # mark every gray voxel below the water-to-oil threshold as water-side,
    # so that the first steps trap water there (a residual event per voxel)
    ev = o.evaluate()
    o.side = np.where(o.gray & (ev["S"] <= 0.5 - wl["params"].hyst), True, o.side)
    d0 = o.diagnostics()
    o.step(100)
    d1 = o.diagnostics()
    assert o.r.sum() > 0.0, "expected residual trapping events"
    assert abs(d1["mass_w"] / d0["mass_w"] - 1) < 1e-13
    assert abs(d1["mass_o"] / d0["mass_o"] - 1) < 1e-13
    assert d1["nonfinite"] == 0
    assert o.r.min() >= 0.0


def test_pseudopotential_conserves_total_momentum():
    # periodic, no gray, no body force, unequal relaxation times
    rng = np.random.default_rng(3)
    n = (6, 7, 8)
    p = W.Params(nx=8, ny=7, nz=6, ncomp=2, tau=(0.8, 1.4), G=3.0).filled()
    cls = np.zeros(n, np.uint8)
    o = Oracle(p)
    o.set_geometry(cls, np.ones(n), np.zeros(n, np.uint8), [])
    rw = rng.uniform(0.1, 1.0, n)
    o.init_fluid(rw, 1.05 - rw)
    o.f *= 1 + 0.01 * rng.standard_normal(o.f.shape)
    ev = o.evaluate()
    assert np.max(np.abs(ev["F"][0])) > 1e-3
    np.testing.assert_allclose(ev["F"].sum(axis=(0, 2, 3, 4)), 0.0, atol=1e-14)
    mom0 = ev["mom"].sum(axis=(0, 2, 3, 4))
    o.step(20)
    mom1 = o.evaluate()["mom"].sum(axis=(0, 2, 3, 4))
    np.testing.assert_allclose(mom1, mom0, atol=1e-13)


def _run_to_steady(o, steps):
    o.step(steps)
    return o.fields()


# Velocities are differences of O(w_i rho) populations, so fp64 resolves them
# to about 1e-17 absolute: the Darcy checks use 1e-12 relative plus 1e-16.
def test_uniform_darcy_scalar():
    # one component: u = g K0 / nu exactly at steady state
    wl = W.uniform_gray(n=(1, 1, 1), phi=0.3, ncomp=1, tau=1.0, g=(1e-3, 2e-4, -3e-4))
    o = _oracle(wl)
    f = _run_to_steady(o, 3000)
    K0 = float(o.K0[0, 0, 0])
    nu = CS2 * 0.5
    for d, key in enumerate(("ux", "uy", "uz")):
        want = wl["params"].g[0][d] * K0 / nu
        assert abs(f[key][0, 0, 0] - want) < 1e-12 * abs(want) + 1e-16
    assert abs(K0 - 0.3 ** 3 / 0.7 ** 2 * 4 / 180) < 5e-6  # Kozeny-Carman sample
    assert abs(1e-5 * K0 / nu - 7.347e-8) < 5e-10


def test_uniform_darcy_two_components():
    wl = W.uniform_gray(n=(1, 1, 1), phi=0.2, ncomp=2, tau=0.8, g=(4e-4, 0.0, 0.0),
                        K0_const=0.05)
    wl["params"].g = ((4e-4, 0.0, 0.0), (-1e-4, 2e-4, 0.0))
    o = _oracle(wl)
    f = _run_to_steady(o, 600)
    ev = o.evaluate()
    R = float(ev["cR"][0, 0, 0] / o.K0[0, 0, 0])
    rho = ev["rho"][:, 0, 0, 0]
    g = wl["params"].g
    for d, key in enumerate(("ux", "uy", "uz")):
        want = (rho[0] * g[0][d] + rho[1] * g[1][d]) / R
        assert abs(f[key][0, 0, 0] - want) < 1e-12 * abs(want) + 1e-16


def test_uniform_darcy_tensor():
    # a rotated principal frame: u = K g / nu along and across the axes
    wl = W.uniform_gray(n=(1, 1, 1), phi=0.3, ncomp=1, tau=1.0, g=(1e-3, 0.0, 0.0),
                        kd=(1.0, 0.1, 0.1), tensor=True, K0_const=0.05)
    o = _oracle(wl)
    # uniform porosity: the gate keeps the isotropic tensor
    np.testing.assert_allclose(o.Kinv[:, 0, 0, 0] * o.K0[0, 0, 0], [1, 1, 1, 0, 0, 0], atol=1e-15)
    rng = np.random.default_rng(5)
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    K0 = float(o.K0[0, 0, 0])
    a = np.array([1.0, 0.1, 0.1])
    Kinv = Qm @ np.diag(1.0 / (a * K0)) @ Qm.T
    o.Kinv[:, 0, 0, 0] = [Kinv[0, 0], Kinv[1, 1], Kinv[2, 2], Kinv[0, 1], Kinv[0, 2], Kinv[1, 2]]
    for gvec in ([1e-3, 0, 0], list(1e-3 * Qm[:, 0]), list(1e-3 * Qm[:, 1])):
        o.p.g = (tuple(gvec), (0.0, 0.0, 0.0))
        o.init_fluid(np.ones((1, 1, 1)))
        f = _run_to_steady(o, 1500)
        u = np.array([f["ux"][0, 0, 0], f["uy"][0, 0, 0], f["uz"][0, 0, 0]])
        want = np.linalg.solve(Kinv, np.array(gvec)) / (CS2 * 0.5)
        np.testing.assert_allclose(u, want, rtol=0, atol=1e-12 * np.max(np.abs(want)) + 1e-16)


def _channel(H, tau, collision, g, gray_K=None):
    ny = H + 2
    p = W.Params(nx=1, ny=ny, nz=1, ncomp=1, tau=(tau, tau), G=0.0, g=((g, 0, 0), (0, 0, 0)),
                 collision=collision).filled()
    fill = 2 if gray_K is not None else 0
    cls = np.full((1, ny, 1), fill, np.uint8)
    cls[:, 0, :] = 1
    cls[:, -1, :] = 1
    tabs = []
    if gray_K is not None:
        pc, krw, kro = W.brooks_corey_tables(0.05, 2, 0.1)
        tabs = [W.pore_table(np.full(1025, gray_K), pc, krw, kro, phi_ref=0.3, pc_pm=0.05)]
    o = Oracle(p)
    o.set_geometry(cls, np.where(cls == 2, 0.3, 1.0), np.zeros(cls.shape, np.uint8), tabs)
    o.init_fluid(np.ones(cls.shape))
    return o


def test_poiseuille_bgk_exact():
    # BGK with (tau - 1/2)^2 = 3/16: halfway bounce-back gives the parabola exactly
    tau = 0.5 + math.sqrt(3) / 4
    H, g = 10, 1e-6
    o = _channel(H, tau, "bgk", g)
    u = _run_to_steady(o, 3000)["ux"][0, :, 0]
    nu = CS2 * (tau - 0.5)
    y = np.arange(H + 2, dtype=float)
    ex = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    assert np.max(np.abs(u[1:-1] - ex[1:-1])) < 1e-10 * np.max(ex)


def test_poiseuille_regularized_second_order():
    tau, g = 1.5, 1e-6
    errs = []
    for H in (6, 12, 24):
        o = _channel(H, tau, "regularized", g)
        u = _run_to_steady(o, int(9 * H * H) + 500)["ux"][0, :, 0]
        nu = CS2 * (tau - 0.5)
        y = np.arange(H + 2, dtype=float)
        ex = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
        errs.append(np.max(np.abs(u[1:-1] - ex[1:-1])) / np.max(ex))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(q - 2.0) < 0.2 for q in orders), (errs, orders)


def test_brinkman_channel_converges():
    tau, g = 1.0, 1e-6
    errs = []
    for H in (8, 16, 32):
        K = (H / 8.0) ** 2
        o = _channel(H, tau, "regularized", g, gray_K=K)
        u = _run_to_steady(o, 40 * H + 300)["ux"][0, :, 0]
        nu = CS2 * (tau - 0.5)
        y = np.arange(H + 2, dtype=float) - (H + 1) / 2.0
        sk = math.sqrt(K)
        ex = g * K / nu * (1 - np.cosh(y / sk) / math.cosh(H / (2 * sk)))
        errs.append(np.max(np.abs(u[1:-1] - ex[1:-1])) / np.max(ex))
    assert errs[2] < 3e-3
    assert errs[0] > errs[1] > errs[2]
    assert math.log2(errs[1] / errs[2]) > 1.6, errs


def test_flat_interface_capillary_jump():
    """Uniform gray column with Pc(S) = P0 and Kr = 1, two flat interfaces at
    rest: p_oil - p_water = P0 (S_hat_w - S_hat_o), p = cs2 rho + cs2 G rho_w rho_o.
    At rest the resistance force vanishes, so pressure carries all of the
    capillary force of Eq. (1) whatever the resistance; the equilibrium reached
    at R / rho = 1/6 is then continued at R / rho = 5e4, where it must stay at
    rest with the same jump."""
    n, P0 = 32, 0.01

    def run(P):
        p = W.Params(nx=n, ny=1, nz=1, ncomp=2, tau=(1.0, 1.0), G=3.0, kappa=0.0).filled()
        m = p.m_minor
        cls = np.full((1, 1, n), 2, np.uint8)
        tab = W.pore_table(np.full(1025, 1.0), np.full(1025, P), np.ones(1025), np.ones(1025),
                           phi_ref=0.3, pc_pm=max(P, 1e-3))
        o = Oracle(p)
        o.set_geometry(cls, np.full(cls.shape, 0.3), np.zeros(cls.shape, np.uint8), [tab])
        x = np.arange(n, dtype=float).reshape(1, 1, n)
        prof = 0.5 * (np.tanh((x - n / 4) / 1.5) - np.tanh((x - 3 * n / 4) / 1.5))
        o.init_fluid(m + (1 - m) * prof, m + (1 - m) * (1 - prof))
        o.step(3000)
        out = []
        for stiff in (False, True):
            if stiff:  # nu / K0 = 5e4
                o.K0 = o.K0 * (CS2 * 0.5) / 5e4
                o.step(300)
            ev = o.evaluate()
            assert np.max(np.abs(ev["u"])) < 1e-8
            rw, ro = ev["rho"][0, 0, 0], ev["rho"][1, 0, 0]
            pr = CS2 * (rw + ro) + CS2 * p.G * rw * ro
            out.append((pr[0] - pr[n // 2], ev["S_hat"][0, 0, n // 2] - ev["S_hat"][0, 0, 0]))
        return out

    (dp0, _), (dp0s, _) = run(0.0)
    (dp1, dS), (dp1s, dSs) = run(P0)
    # inside gray voxels the second-order forcing gives bulk densities a little
    # off the pore voxels' coexistence values that normalise S_hat
    assert abs(dS - 1.0) < 1e-2 and abs(dSs - 1.0) < 1e-2
    assert abs(dp0) < 1e-10 and abs(dp0s) < 1e-10
    assert abs((dp1 - dp0) / (P0 * dS) - 1) < 1e-2
    assert abs((dp1s - dp0s) / (P0 * dSs) - 1) < 1e-2


@pytest.mark.parametrize("ratio", [1.0, 1e2, 1e4, 5e4])
def test_pressure_driven_darcy_through_gray_slab(ratio):
    """A gray slab (R / rho = nu / K0 = ratio) between two pressure reservoirs,
    one component, quasi-1D: inside the slab the mass flux obeys Darcy's law
    J = -(K0 / nu) dp/dx, p = cs2 rho, with the local gradient across the
    flux plane, to 2 % (the flux averaged over two steps, which cancels the
    step-to-step alternation of the gathered momentum under strong
    resistance).  A scheme whose resistance acts on another velocity than
    the one that carries the mass fails by (2 rho + R) / (2 rho) here."""
    nx, xf = 24, 11
    tau = 1.0
    nu = CS2 * (tau - 0.5)
    K0 = nu / ratio
    rin, rout = 1.0005, 0.9995
    p = W.Params(nx=nx, ny=1, nz=1, ncomp=1, tau=(tau, tau), G=0.0, bc_x="pressure",
                 rho_in=(rin, 0.0), rho_out=(rout, 0.0), outlet_x=xf).filled()
    cls = np.zeros((1, 1, nx), np.uint8)
    lo, hi = 6, nx - 6
    cls[..., lo:hi] = 2
    tab = W.pore_table(np.full(1025, K0), np.zeros(1025), np.ones(1025), np.ones(1025),
                       phi_ref=0.3, pc_pm=1e-3)
    o = Oracle(p)
    o.set_geometry(cls, np.where(cls == 2, 0.3, 1.0), np.zeros(cls.shape, np.uint8), [tab])
    x = np.arange(nx, dtype=float)
    rho = np.interp(x, [lo - 0.5, hi - 0.5], [rin, rout])
    o.init_fluid(rho.reshape(1, 1, nx))
    o.step(600)
    q = []
    for _ in range(2):
        o.step(1)
        q.append(o.Q_last[0])
    r = o.fields()["rho_w"][0, 0]
    J = 0.5 * (q[0] + q[1])
    want = -(K0 / nu) * CS2 * (r[xf + 1] - r[xf])
    assert want > 0
    assert abs(J / want - 1.0) < 0.02, (J, want)


def test_centred_droplet_stays_mirror_symmetric():
    n = 12
    p = W.Params(nx=n, ny=n, nz=n, ncomp=2, tau=(1.0, 1.0), G=3.0, kappa=-0.03,
                 csf_region="all").filled()
    m = p.m_minor
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    c = (n - 1) / 2
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    prof = 0.5 * (1 - np.tanh((r - 3.5) / 1.5))
    o = Oracle(p)
    cls = np.zeros((n, n, n), np.uint8)
    o.set_geometry(cls, np.ones(cls.shape), np.zeros(cls.shape, np.uint8), [])
    o.init_fluid(m + (1 - m) * prof, m + (1 - m) * (1 - prof))
    o.step(30)
    f = o.fields()
    rw = f["rho_w"]
    for ax in range(3):
        np.testing.assert_allclose(rw, np.flip(rw, axis=ax), rtol=0, atol=1e-14)
    np.testing.assert_allclose(f["ux"], -np.flip(f["ux"], axis=2), atol=1e-14)


def test_checkpoint_resume_is_bitwise():
    wl = W.droplet_slab()
    a = _oracle(wl)
    a.step(6)
    st = a.get_state()
    a.step(6)
    b = _oracle(W.droplet_slab())
    b.set_state(st)
    b.step(6)
    assert np.array_equal(a.f, b.f)
    assert np.array_equal(a.r, b.r)
    assert np.array_equal(a.side, b.side)
