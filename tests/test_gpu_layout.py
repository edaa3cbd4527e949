"""Fluid-only population layout (fp32 storage, two components, periodic x):
solid voxels hold no populations, each population array keeps one slot per
fluid voxel.  The layout changes where values live, not what is computed, so
a run in it must agree bitwise with the same run in the dense layout: the
state blob (canonical order, so blobs move between layouts), the fields and
the diagnostics, outlet flux included.

Cases: ragged x and y tiles with the wrap on every axis (72 x 10 x 12: the
fused step's tile and chunk faces and the density fix-up's links); one x tile
exactly (64 wide: the wrap lanes x = 0 and x = nx - 1 in one wave); a
one-voxel x axis (both x neighbours of a voxel are the voxel itself); fully
solid rows and planes; the 48^3 multiscale rock.  Checkpoints resume
bitwise across layouts, and the adjoint, which runs on a dense copy, gives
the dense handle's gradients and leaves the handle in the fluid-only layout
at the same state."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from gpu_common import announce

pytestmark = [pytest.mark.gpu, pytest.mark.skip(
    reason="the fluid-only layout is switched off: its first run of this file stalled without a "
           "GPU fault and the cause is not known")]

STEPS = 40


def _random_case(shape, seed, solid_planes=False):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    p = W.Params(nx=nx, ny=ny, nz=nz, ncomp=2, precision="f32", tau=(1.0, 1.5), G=3.0,
                 kappa=-0.02, csf_region="all", g=((1e-4, 0, 0), (0, -5e-5, 2e-5))).filled()
    cls = rng.choice([0, 0, 0, 1, 2], size=shape).astype(np.uint8)
    if solid_planes:
        cls[nz // 2] = W.SOLID              # a solid z plane
        cls[:, 1, :] = W.SOLID              # solid x rows
        cls[:, :, min(3, nx - 1)] = W.SOLID  # a solid x column
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, shape), 1.0)
    pt = np.where(cls == 2, rng.integers(0, 2, shape), 0).astype(np.uint8)
    tabs = W.multiscale_rock(n=8, precision="f64")["tables"][:2]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - 0.4 * nx) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    prof = 0.5 * (1 - np.tanh((r - 0.3 * min(shape)) / 1.5))
    rw = p.m_minor + (1 - p.m_minor) * np.clip(prof, 0, 1)
    return p, cls, phi, pt, tabs, rw, 1.0 + p.m_minor - rw


def _rock_case():
    wl = W.multiscale_rock(n=48, precision="f32")
    return wl["params"], wl["cls"], wl["phi"], wl["ptype"], wl["tables"], wl["rho_w"], wl["rho_o"]


CASES = {
    "ragged_72x10x12": lambda: _random_case((12, 10, 72), 17),
    "one_tile_64x8x8": lambda: _random_case((8, 8, 64), 23, solid_planes=True),
    "one_voxel_x_1x9x10": lambda: _random_case((10, 9, 1), 29),
    "solid_planes_130x7x9": lambda: _random_case((9, 7, 130), 31, solid_planes=True),
    "rock_48": _rock_case,
}


def _handle(L, p, cls, phi, pt, tabs, layout):
    lb = L.lbm_create(replace(p, layout=layout))
    lb.set_geometry(cls, phi, pt, tabs)
    return lb


def _run(L, case, layout, steps=STEPS):
    p, cls, phi, pt, tabs, rw, ro = case
    lb = _handle(L, p, cls, phi, pt, tabs, layout)
    lay = lb.get_layout()
    lb.init_fluid(rw, ro)
    lb.step(steps)
    f = lb.get_fields()
    d = lb.get_diagnostics()
    blob = lb.get_state()
    lb.destroy()
    return lay, f, d, blob


@pytest.mark.parametrize("name", list(CASES))
def test_fluid_only_layout_is_bitwise_the_dense_run(name):
    import paper_2512_21696_amd as L
    case = CASES[name]()
    p, cls = case[0], case[1]
    nfluid = int((cls != W.SOLID).sum())
    announce(f"layout {name}: {STEPS} fp32 steps, fluid-only vs dense")
    lay_a, fa, da, ba = _run(L, case, "auto")
    lay_d, fd, dd, bd = _run(L, case, "dense")
    assert lay_a["fluid_only"] and not lay_d["fluid_only"]
    assert lay_d["slots"] == cls.size
    assert nfluid <= lay_a["slots"] <= min(cls.size, (nfluid + 63) // 64 * 64)
    assert da["nonfinite"] == 0
    assert ba == bd, "state blobs differ"
    for k in fa:
        assert np.array_equal(fa[k], fd[k]), k
    for k in da:
        assert da[k] == dd[k] or (np.isnan(da[k]) and np.isnan(dd[k])), k


def test_layouts_keep_other_runs_dense():
    """fp64, one component and 16-bit storage keep the dense layout, as does
    fp32 two-component with layout = dense."""
    import paper_2512_21696_amd as L
    p, cls, phi, pt, tabs, rw, ro = _random_case((6, 5, 20), 5)
    announce("layout: which runs take the fluid-only layout")
    for kw, expect in ((dict(), True), (dict(layout="dense"), False), (dict(precision="f64"), False),
                       (dict(precision="f16"), False), (dict(ncomp=1, G=0.0, kappa=0.0), False)):
        q = replace(p, **kw)
        if q.precision == "f64":
            q = replace(q, eps_n=1e-12)
        lb = _handle(L, q, cls, phi, pt, tabs, q.layout)
        assert lb.get_layout()["fluid_only"] == expect, kw
        lb.destroy()


def test_checkpoint_resumes_bitwise_across_layouts():
    import paper_2512_21696_amd as L
    p, cls, phi, pt, tabs, rw, ro = CASES["ragged_72x10x12"]()
    announce("layout: checkpoint at 20 steps, resumed in both layouts")
    lb = _handle(L, p, cls, phi, pt, tabs, "auto")
    lb.init_fluid(rw, ro)
    lb.step(20)
    mid = lb.get_state()
    lb.step(20)
    ref = lb.get_state()
    lb.destroy()
    for layout in ("auto", "dense"):
        lb = _handle(L, p, cls, phi, pt, tabs, layout)
        lb.set_state(mid)
        lb.step(20)
        assert lb.get_state() == ref, layout
        lb.destroy()


def test_adjoint_on_a_fluid_only_handle():
    import paper_2512_21696_amd as L
    p, cls, phi, pt, tabs, rw, ro = _random_case((8, 8, 24), 41)
    n = 12
    dq = np.linspace(1.0, 2.0, n)
    announce(f"layout: two-component fp32 adjoint over {n} steps, fluid-only vs dense handle")
    out = {}
    for layout in ("auto", "dense"):
        lb = _handle(L, p, cls, phi, pt, tabs, layout)
        lb.init_fluid(rw, ro)
        lb.step(3)
        g = lb.adjoint_flux(n, dq, checkpoint_every=4)
        lay = lb.get_layout()
        lb.step(5)
        out[layout] = (g, lay, lb.get_state())
        lb.destroy()
    (ga, la, sa), (gd, ld, sd) = out["auto"], out["dense"]
    assert la["fluid_only"] and not ld["fluid_only"]
    for k in ("Q", "dL_dK0", "dL_dphi"):
        assert np.array_equal(ga[k], gd[k]), k
    assert sa == sd
