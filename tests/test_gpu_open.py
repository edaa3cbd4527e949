"""Open x faces on the GPU against the fp64 oracle, through the C ABI, for
both kinds: reservoirs beyond x = 0 and x = nx - 1 (pressure) and exact
density faces of the Zou-He type (density): a two-component displacement with
water entering at the inlet and oil at the outlet through a ragged box with
solid grains, gray voxels and CSF, a single-phase pressure-driven slit, and a
change of the prescribed densities between steps.  On density faces the
reported densities of the face voxels equal the prescribed ones.  Tolerances as in test_gpu_parity: fp64 1e-12 of each field's largest
value; fp32 rounding (6e-8) of O(1) densities accumulated over 60 steps stays
below 1e-4 of each field's scale."""
import numpy as np
import pytest

import workloads as W
from gpu_common import announce, gpu_run, oracle_run, field_errors, diag_errors

pytestmark = pytest.mark.gpu


def displacement(precision="f64", bc="pressure", shape=(9, 10, 21)):
    m = W.minority_density(3.0)
    nz, ny, nx = shape
    rng = np.random.default_rng(71)
    cls = np.zeros((nz, ny, nx), np.uint8)
    core = (slice(None), slice(None), slice(4, nx - 4))
    r = rng.random((nz, ny, nx))
    cls[core] = np.where(r[core] < 0.15, 1, np.where(r[core] < 0.35, 2, 0))
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, cls.shape), np.where(cls == 0, 1.0, 0.0))
    K0 = W.kozeny_carman_table(2.0)
    tabs = [W.pore_table(K0, *W.brooks_corey_tables(0.05, 2.0, 0.1), phi_ref=0.3, pc_pm=0.05)]
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=2, precision=precision, tau=(1.0, 1.2),
                 kappa=-0.05, bc_x=bc, rho_in=(1.02, m), rho_out=(m, 0.99)).filled()
    x = np.arange(nx)[None, None, :]
    prof = 0.5 * (1 - np.tanh((x - 3.0) / 1.5)) * np.ones(cls.shape)
    rw = m + (1 - m) * prof
    return dict(params=p, cls=cls, phi=phi, ptype=np.zeros(cls.shape, np.uint8), tables=tabs,
                rho_w=rw, rho_o=1 + m - rw)


@pytest.mark.parametrize("bc", ["pressure", "density"])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-4)])
def test_open_faces_displacement_matches_oracle(prec, tol, bc):
    wl = displacement(bc=bc)
    steps = 60
    announce(f"open x faces ({bc}) displacement {prec}, {steps} steps")
    lb = gpu_run(wl, steps, prec)
    got, dg = lb.get_fields(), lb.get_diagnostics()
    wl64 = displacement(bc=bc)
    o = oracle_run(wl64, steps)
    ref = o.fields()
    names = ("rho_w", "rho_o", "ux", "uy", "uz", "S") + (("r_w", "r_o") if prec == "f64" else ())
    fe = field_errors(got, ref, names)
    de = diag_errors(dg, o.diagnostics(), ("mass_w", "mass_o", "q_w", "q_o"))
    print(prec, "field errors", {k: f"{v:.2e}" for k, v in fe.items()})
    print(prec, "diag errors", {k: f"{v:.2e}" for k, v in de.items()})
    for k, v in fe.items():
        assert v < tol, (k, v)
    if bc == "density":
        fl = wl["cls"] != 1
        for k, xb, val in (("rho_w", 0, 1.02), ("rho_o", -1, 0.99)):
            err = np.abs(np.asarray(got[k])[:, :, xb][fl[:, :, xb]] - val).max()
            assert err < (1e-13 if prec == "f64" else 1e-6), (k, err)
    lb.destroy()


@pytest.mark.parametrize("bc", ["pressure", "density"])
def test_open_faces_2d_displacement_matches_oracle(bc):
    """nz = 1: a two-dimensional displacement (the paper's 2-D protocols run on
    one plane) through grains and gray voxels, fp64."""
    wl = displacement(bc=bc, shape=(1, 24, 40))
    steps = 80
    announce(f"open x faces ({bc}) 2-D displacement 40x24x1 fp64, {steps} steps")
    lb = gpu_run(wl, steps, "f64")
    got = lb.get_fields()
    o = oracle_run(displacement(bc=bc, shape=(1, 24, 40)), steps)
    fe = field_errors(got, o.fields(), ("rho_w", "rho_o", "ux", "uy", "S"))
    print("2-D field errors", {k: f"{v:.2e}" for k, v in fe.items()})
    assert max(fe.values()) < 1e-12
    lb.destroy()


@pytest.mark.parametrize("bc", ["pressure", "density"])
def test_open_faces_single_phase_slit_matches_oracle(bc):
    H, L = 6, 12
    p = W.Params(nx=L, ny=H + 2, nz=3, ncomp=1, tau=(1.0, 1.0), G=0.0, bc_x=bc,
                 rho_in=(1.003, 0.0), rho_out=(0.997, 0.0)).filled()
    cls = np.zeros((3, H + 2, L), np.uint8)
    cls[:, 0, :] = 1
    cls[:, H + 1, :] = 1
    wl = dict(params=p, cls=cls, phi=np.ones(cls.shape), ptype=np.zeros(cls.shape, np.uint8),
              tables=[], rho_w=np.ones(cls.shape), rho_o=None)
    announce(f"open x faces ({bc}) single-phase slit fp64, 300 steps")
    lb = gpu_run(wl, 300, "f64")
    got = lb.get_fields()
    o = oracle_run(wl, 300)
    ref = o.fields()
    fe = field_errors(got, ref, ("rho_w",))
    # velocities against the speed scale (the transverse components are ~0)
    us = max(np.abs(ref[k]).max() for k in ("ux", "uy", "uz"))
    for k in ("ux", "uy", "uz"):
        fe[k] = float(np.abs(np.asarray(got[k]) - ref[k]).max()) / us
    print("slit field errors", {k: f"{v:.2e}" for k, v in fe.items()})
    assert max(fe.values()) < 1e-12
    lb.destroy()


def test_open_faces_reject_gray_next_to_a_face():
    import paper_2512_21696_amd as L
    wl = displacement()
    wl["cls"][:, :, 1] = 2
    wl["phi"] = np.where(wl["cls"] == 2, 0.3, wl["phi"])
    announce("open x faces: rejected geometry")
    lb = L.lbm_create(wl["params"])
    with pytest.raises(L.LbmError) as e:
        lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    assert e.value.code == L.LBM_E_INVAL
    lb.destroy()


@pytest.mark.parametrize("bc", ["pressure", "density"])
@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_open_faces_16bit_displacement_within_rounding_of_oracle(prec, bc):
    """16-bit storage between open faces: the face values are offsets against
    their slot owner's reference like every other slot, and the face voxels'
    reference sums are corrected to those owners.  Against the fp64 oracle
    within the rounding bounds of the 16-bit tests (density 2 * 2^-p sqrt(n),
    velocity 2^-p sqrt(n) / 3); on density faces the face voxels hold the
    prescribed densities to the rounding of their five face values."""
    from test_gpu_store16 import bound, abs_errors, BITS
    steps = 60
    announce(f"open x faces ({bc}) displacement {prec}, {steps} steps")
    wl = displacement(bc=bc)
    lb = gpu_run(wl, steps, prec)
    got, dg = lb.get_fields(), lb.get_diagnostics()
    lb.destroy()
    o = oracle_run(displacement(bc=bc), steps)
    ref = o.fields()
    names = ("rho_w", "rho_o", "ux", "uy", "uz", "S")
    ae = abs_errors(got, ref, names)
    print(prec, bc, "absolute field errors", {k: f"{v:.2e}" for k, v in ae.items()})
    assert dg["nonfinite"] == 0
    for k, v in ae.items():
        assert v < bound(prec, steps, k), (k, v, bound(prec, steps, k))
    if bc == "density":
        fl = wl["cls"] != 1
        tol = 2.0 ** -BITS[prec] * 2.0
        for k, xb, val in (("rho_w", 0, 1.02), ("rho_o", -1, 0.99)):
            err = np.abs(np.asarray(got[k])[:, :, xb][fl[:, :, xb]] - val).max()
            assert err < tol, (k, err, tol)


@pytest.mark.parametrize("bc", ["pressure", "density"])
def test_reservoir_step_matches_oracle(bc):
    """lbm_set_reservoirs between steps (a pressure step of a quasi-static
    protocol) against the oracle with the same change."""
    import copy
    wl = displacement(bc=bc)
    announce(f"open x faces ({bc}): densities stepped after 30 steps, fp64")
    lb = gpu_run(wl, 30, "f64")
    m = wl["params"].m_minor
    new_in, new_out = (1.05, m), (m, 0.98)
    lb.set_reservoirs(new_in, new_out)
    lb.step(30)
    got = lb.get_fields()
    p = copy.deepcopy(displacement(bc=bc)["params"])
    wl64 = displacement(bc=bc)
    wl64["params"] = p
    o = oracle_run(wl64, 30)
    p.rho_in, p.rho_out = new_in, new_out
    o.step(30)
    fe = field_errors(got, o.fields(), ("rho_w", "rho_o", "ux", "uy", "uz", "S"))
    print("reservoir step field errors", {k: f"{v:.2e}" for k, v in fe.items()})
    assert max(fe.values()) < 1e-12
    lb.destroy()
    import paper_2512_21696_amd as L
    per = W.droplet_slab()
    lb = L.lbm_create(per["params"])
    with pytest.raises(L.LbmError) as e:
        lb.set_reservoirs(new_in, new_out)
    assert e.value.code == L.LBM_E_STATE
    lb.destroy()
