"""Batched single-phase permeability runs (lbm_rev_permeability) against the
oracle's run of each domain alone (oracle/rev.py), through the C ABI.

Tolerances.  fp64: the kernel sums in another order than numpy, so fields
agree to rounding: 1e-12 of the largest velocity.  fp32: every step rounds
quantities of the size of the density (1) to 2^-24 relative, and the velocity
is a small difference of them (|u| is at most a few 1e-3 here), so the bound
is absolute: at most one ulp of the unit density, 2^-23, per step, summed
over the n steps (errors persist for a viscous time), n 2^-23 in u and
n 2^-23 nu / g in K.

16-bit storage (fp16, bf16): a stored value is h = f_i / w_i - rho_w, the
offset from the density of the voxel that wrote it, rounded to the nearest
of a format with unit roundoff eps (2^-11 fp16, 2^-8 bf16; fp16 holds 2^12 h,
an exact scaling, so offsets down to 1.5e-8 stay normal and smaller ones err
by at most 2^-36, far below the fp32 term), so a population carries an error
of at most w_i eps |h| per step.  The velocity along an axis takes
sum_i w_i c_ia^2 = 1/3 of that per step.  |h| is at most the largest
|f_i / w_i - 1| plus the largest |rho - 1| of the run; with H twice the sum of
those two on the oracle's final set (the flow accelerates from rest), the
bound is n (eps H / 3 + 2^-23) in u."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import rev
from gpu_common import announce

pytestmark = pytest.mark.gpu


def params(shape, tau, g, axis, collision):
    gv = [0.0, 0.0, 0.0]
    gv[axis] = g
    nz, ny, nx = shape
    return W.Params(nx=nx, ny=ny, nz=nz, ncomp=1, tau=(tau, tau), G=0.0,
                    g=(tuple(gv), (0.0, 0.0, 0.0)), kappa=0.0, collision=collision).filled()


def batch():
    """Four uneven domains: small sphere packs, a slit with a ragged box, an
    all-pore box."""
    a = W.sphere_pack((9, 7, 11), 0.7, seed=11, rmin=1.0, rmax=2.0)
    b = W.sphere_pack((16, 16, 16), 0.5, seed=12, rmin=2.0, rmax=3.0)
    c = np.zeros((6, 10, 1), np.uint8)
    c[:, 0, :] = 1
    c[:, 9, :] = 1
    d = np.zeros((4, 5, 6), np.uint8)
    return [a, b, c, d]


def compare(doms, tau, g, axis, collision, prec, steps, walls=False, mirror=False):
    import paper_2512_21696_amd as L
    announce(f"rev batch {len(doms)} domains {prec} {collision} axis {axis} walls {walls} "
             f"mirror {mirror}, {steps} steps")
    got = L.rev_permeability(doms, tau=tau, g=g, axis=axis, collision=collision, precision=prec,
                             side_walls=walls, mirror=mirror, max_steps=steps, check_every=20,
                             tol=0.0, want_u=True)
    f64 = prec == "f64"
    nu = (tau - 0.5) / 3
    worst = 0.0
    for cls, r in zip(doms, got):
        box = tuple(slice(0, n) for n in cls.shape)
        run = cls
        if mirror:
            run = rev.mirrored(run, axis)
        if walls:
            run, inner = rev.with_side_walls(run, axis)
            box = tuple(slice(s.start, s.start + n) for s, n in zip(inner, cls.shape))
        K, u = rev.permeability(params(run.shape, tau, g, axis, collision), run, steps, axis)
        u = u[box]
        d = np.abs(r["u"] - u).max()
        bound = 1e-12 * np.abs(u).max() if f64 else steps * 2.0 ** -23
        worst = max(worst, d / bound)
        assert d < bound, (cls.shape, d, bound)
        n_run = cls.size * (2 if mirror else 1)
        K_ref = K * run.size / n_run  # the library normalises by its own (unframed) box
        kb = 1e-12 * abs(K_ref) if f64 else steps * 2.0 ** -23 * nu / g
        assert abs(r["K"] - K_ref) < kb, (cls.shape, r["K"], K_ref)
        assert abs(r["phi"] - (1 - cls.mean())) < 1e-15
        assert r["steps"] == steps and not r["converged"]
    print(prec, collision, "worst velocity error / bound", f"{worst:.2e}")


@pytest.mark.parametrize("prec,collision,axis", [("f64", "regularized", 0), ("f64", "bgk", 2),
                                                 ("f32", "regularized", 1), ("f32", "bgk", 0)])
def test_batch_matches_oracle(prec, collision, axis):
    compare(batch(), 0.8, 1e-4, axis, collision, prec, 60)


@pytest.mark.parametrize("walls,mirror", [(True, False), (False, True), (True, True)])
def test_walls_and_mirror_match_oracle(walls, mirror):
    doms = batch()[:2] + [batch()[3]]
    compare(doms, 0.9, 1e-4, 1, "regularized", "f64", 40, walls=walls, mirror=mirror)


def test_batch_equals_single_domain_runs():
    import paper_2512_21696_amd as L
    doms = batch()
    announce("rev batch vs single-domain calls, f64")
    kw = dict(tau=0.8, g=1e-4, axis=0, precision="f64", max_steps=50, check_every=10, tol=0.0,
              want_u=True)
    together = L.rev_permeability(doms, **kw)
    for cls, r in zip(doms, together):
        alone = L.rev_permeability([cls], **kw)[0]
        assert alone["K"] == r["K"] and np.array_equal(alone["u"], r["u"])


def test_slit_converges_to_exact_permeability():
    import paper_2512_21696_amd as L
    H = 6
    cls = np.zeros((3, H + 2, 4), np.uint8)
    cls[:, 0, :] = 1
    cls[:, H + 1, :] = 1
    announce("rev slit convergence, f64 BGK")
    r = L.rev_permeability([cls], tau=0.5 + math.sqrt(3) / 4, g=1e-6, axis=0, collision="bgk",
                           precision="f64", max_steps=20000, check_every=100, tol=1e-12)[0]
    exact = sum((y - 0.5) * (H + 0.5 - y) for y in range(1, H + 1)) / (2 * (H + 2))
    assert r["converged"] and r["steps"] < 20000
    assert abs(r["K"] - exact) < 1e-9 * exact, (r["K"], exact)


@pytest.mark.parametrize("prec,collision,axis", [("f16", "regularized", 0), ("bf16", "bgk", 1),
                                                 ("f16", "bgk", 2), ("bf16", "regularized", 0)])
def test_batch_16bit_storage_matches_oracle(prec, collision, axis):
    import paper_2512_21696_amd as L
    from oracle.lattice import W as WQ
    doms, tau, g, steps = batch(), 0.8, 1e-4, 60
    announce(f"rev batch {len(doms)} domains {prec} {collision} axis {axis}, {steps} steps")
    got = L.rev_permeability(doms, tau=tau, g=g, axis=axis, collision=collision, precision=prec,
                             max_steps=steps, check_every=20, tol=0.0, want_u=True)
    eps = 2.0 ** -11 if prec == "f16" else 2.0 ** -8
    nu = (tau - 0.5) / 3
    worst = 0.0
    for cls, r in zip(doms, got):
        K, u, f = rev.permeability(params(cls.shape, tau, g, axis, collision), cls, steps, axis,
                                   with_state=True)
        pore = cls == 0
        rho = f.sum(axis=0)[pore]
        H = 2.0 * (max(np.abs(f[i][pore] / WQ[i] - 1.0).max() for i in range(19)) +
                   np.abs(rho - 1.0).max())
        bound = steps * (eps * H / 3.0 + 2.0 ** -23)
        d = np.abs(r["u"] - u).max()
        worst = max(worst, d / bound)
        assert d < bound, (cls.shape, d, bound)
        assert abs(r["K"] - K) < bound * nu / g, (cls.shape, r["K"], K)
    print(prec, collision, "worst velocity error / bound", f"{worst:.2e}")


def test_16bit_batch_equals_single_domain_runs():
    import paper_2512_21696_amd as L
    doms = batch()
    announce("rev batch vs single-domain calls, f16")
    kw = dict(tau=0.8, g=1e-4, axis=2, precision="f16", max_steps=50, check_every=10, tol=0.0,
              want_u=True)
    together = L.rev_permeability(doms, **kw)
    for cls, r in zip(doms, together):
        alone = L.rev_permeability([cls], **kw)[0]
        assert alone["K"] == r["K"] and np.array_equal(alone["u"], r["u"])
    # the stored sets are rounded to 16 bits: the fp32 run differs
    f32 = L.rev_permeability(doms[1:2], **dict(kw, precision="f32"))[0]
    assert not np.array_equal(f32["u"], together[1]["u"])


def test_solid_domains():
    """A domain without pore voxels holds no slots: K = phi = 0 in a batch (the
    other domains' results are unchanged) and alone (nothing is launched)."""
    import paper_2512_21696_amd as L
    doms = batch()
    solid = np.ones((5, 4, 6), np.uint8)
    announce("rev batch with an all-solid domain, and an all-solid call, f32")
    kw = dict(tau=0.8, g=1e-4, axis=0, precision="f32", max_steps=40, check_every=10, tol=0.0,
              want_u=True)
    ref = L.rev_permeability(doms, **kw)
    got = L.rev_permeability(doms[:2] + [solid] + doms[2:], **kw)
    for r, g_ in zip(ref, got[:2] + got[3:]):
        assert r["K"] == g_["K"] and np.array_equal(r["u"], g_["u"])
    assert got[2]["K"] == 0.0 and got[2]["phi"] == 0.0 and not got[2]["u"].any()
    alone = L.rev_permeability([solid, solid], **dict(kw, tol=1e-6))
    for r in alone:
        assert r["K"] == 0.0 and r["phi"] == 0.0 and r["converged"] and not r["u"].any()
