"""16-bit population storage (fp16 / bf16 offsets h = f_i / w_i - rho_ref,
fp32 arithmetic) through the C ABI, against the fp64 oracle.

Tolerances.  Every step rounds each stored offset once, to p = 11 (fp16) or
p = 8 (bf16) significant bits: an absolute error of at most 2^-p |h| in f_i / w_i.
|h| is the deviation of f_i / w_i from the writer's density: O(|u|/cs^2) plus the
non-equilibrium part after a collision, and at most about 1 (densities are
O(1)) for the sets written from a canonical state at initialisation.  Over n steps the independent roundings add up like a random walk,
about 2^-p sqrt(n) in density (weights sum to 1); momentum collects at most
1/6 of it (sum over c_x > 0 of w_i).  The bounds below are twice that, in
absolute terms (densities and saturation on the scale 1, velocities in lattice
units):  density 2 * 2^-p sqrt(n), velocity 2^-p sqrt(n) / 3.  fp32 storage
sits far below both (its test is in test_gpu_parity)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import announce, gpu_run, oracle_run, field_errors, diag_errors

pytestmark = pytest.mark.gpu

BITS = {"f16": 11, "bf16": 8}
VEL = ("ux", "uy", "uz")


def bound(prec, steps, name):
    b = 2.0 ** -BITS[prec] * np.sqrt(steps)
    return b / 3.0 if name in VEL else 2.0 * b


def abs_errors(got, ref, names):
    return {k: float(np.abs(np.asarray(got[k], np.float64) - ref[k]).max()) for k in names}


def _compare(wl, steps, prec, names, label):
    announce(f"{label}: {prec} storage, {steps} steps")
    lb = gpu_run(wl, steps, prec)
    got = lb.get_fields()
    dg = lb.get_diagnostics()
    p64 = wl["params"]
    p64.precision = "f64"
    p64.eps_n = 1e-12
    o = oracle_run(wl, steps, params=p64)
    ref = o.fields()
    fe = field_errors(got, ref, names)
    ae = abs_errors(got, ref, names)
    de = diag_errors(dg, o.diagnostics(), ("mass_w", "mass_o", "sw"))
    print(label, prec, "normalised field errors", {k: f"{v:.2e}" for k, v in fe.items()})
    print(label, prec, "absolute field errors", {k: f"{v:.2e}" for k, v in ae.items()})
    print(label, prec, "field scales", {k: f"{np.abs(ref[k]).max():.2e}" for k in names})
    print(label, prec, "diag errors", {k: f"{v:.2e}" for k, v in de.items()})
    assert dg["nonfinite"] == 0 and dg["step"] == steps
    for k, v in ae.items():
        assert v < bound(prec, steps, k), (k, v, bound(prec, steps, k))
    lb.destroy()
    return fe, de


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_droplet_slab_16bit(prec):
    wl = W.droplet_slab()
    fe, de = _compare(wl, 100, prec, ("rho_w", "rho_o", "ux", "uy", "uz", "S", "r_w", "r_o"),
                      "droplet_slab 32^3")
    # total mass per component (mobile + residual): the roundings of many
    # voxels average out, far below the per-voxel bound
    assert max(de["mass_w"], de["mass_o"]) < bound(prec, 100, "rho_w") / 10, de


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_rock_mini_16bit(prec):
    wl = W.multiscale_rock(n=48, precision="f64")
    _compare(wl, 100, prec, ("rho_w", "rho_o", "ux", "uy", "uz", "S"), "multiscale_rock 48^3")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_fiber_mini_16bit(prec):
    # one component: the reference density is the constant 1
    wl = W.fiber_bundles(n=48, ncyl=5, precision="f64")
    _compare(wl, 100, prec, ("rho_w", "ux", "uy", "uz"), "fiber_bundles 48^3")


def test_fp16_beats_bf16_and_fp32_beats_fp16():
    wl = W.droplet_slab()
    errs = {}
    o = oracle_run(W.droplet_slab(), 50)
    ref = o.fields()
    for prec in ("f32", "f16", "bf16"):
        announce(f"droplet_slab {prec} 50 steps (error ordering)")
        lb = gpu_run(W.droplet_slab(), 50, prec)
        errs[prec] = max(field_errors(lb.get_fields(), ref, ("rho_w", "ux", "uy", "uz")).values())
        lb.destroy()
    print("max field error by storage", errs)
    assert errs["f32"] < errs["f16"] < errs["bf16"]
    del wl


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_checkpoint_resume_bitwise_16bit(prec):
    import paper_2512_21696_amd as L
    wl = W.droplet_slab()
    announce(f"checkpoint/resume droplet_slab {prec}")
    a = gpu_run(wl, 12, prec)
    blob = a.get_state()
    st = a.state_arrays(blob)
    assert st["codes"].dtype == np.uint16 and st["ref"].shape[-1] == 2
    a.step(12)
    fa = a.get_state()
    b = L.lbm_create(wl["params"])
    b.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    b.set_state(blob)
    b.step(12)
    same = b.get_state() == fa  # (a bare assert would diff megabytes on failure)
    assert same, "resumed run differs from the continuous run"
    a.destroy()
    b.destroy()
