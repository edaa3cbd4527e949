"""The debug build (liblbm_debug.so, -DLBM_DEBUG): the same kernels with
device-side index checks, above all where the hardware would hide a bad
index (population accesses through buffer resources read 0 beyond their
range).  A child process loads the debug build (LBM_LIBRARY), runs a set of
small cases through every step variant and reports any failed check as an
LBM_E_DEVICE error; its results must equal the release build's bitwise (the
checks do not touch the arithmetic).

Cases: the fused step with the density push (fp32, two components, ragged
tiles and chunks, CSF everywhere), fp64 and fp16 storage on the droplet slab,
open x faces, a one-component tensorial run, a checkpoint round trip and a
one-component adjoint."""
import json
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from gpu_common import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import workloads as W
import paper_2512_21696_amd as L
from test_gpu_debug import cases
out = {}
for name, (wl, steps, extra) in cases().items():
    print("[debug-case]", name, L.LIB_PATH, flush=True)
    lb = L.lbm_create(wl["params"])
    lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    lb.init_fluid(wl["rho_w"], wl["rho_o"])
    lb.step(steps)
    if extra == "checkpoint":
        blob = lb.get_state()
        lb.set_state(blob)
        lb.step(3)
    res = {k: v for k, v in lb.get_fields().items()}
    res["diag"] = np.array([lb.get_diagnostics()[k] for k in ("mass_w", "mass_o", "q_acc_w", "max_u")])
    if extra == "adjoint":
        g = lb.adjoint_flux(4, np.ones(4))
        res["dL_dphi"] = g["dL_dphi"]
    lb.destroy()
    np.savez(sys.argv[2] + "/" + name + ".npz", **res)
print("[debug-case] done", flush=True)
'''


def cases():
    import workloads as W
    rng = np.random.default_rng(17)
    shape = (12, 10, 72)
    p = W.Params(nx=72, ny=10, nz=12, ncomp=2, precision="f32", tau=(1.0, 1.5), G=3.0,
                 kappa=-0.02, csf_region="all", g=((1e-4, 0, 0), (0, -5e-5, 0))).filled()
    cls = rng.choice([0, 0, 0, 1, 2], size=shape).astype(np.uint8)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, shape), 1.0)
    pt = np.where(cls == 2, rng.integers(0, 2, shape), 0).astype(np.uint8)
    tabs = W.multiscale_rock(n=8, precision="f64")["tables"][:2]
    z, y, x = np.meshgrid(np.arange(12), np.arange(10), np.arange(72), indexing="ij")
    prof = 0.5 * (1 - np.tanh((np.sqrt((x - 10) ** 2 + (y - 5) ** 2 + (z - 6) ** 2) - 4.0) / 1.5))
    rw = p.m_minor + (1 - p.m_minor) * prof
    push = dict(params=p, cls=cls, phi=phi, ptype=pt, tables=tabs, rho_w=rw,
                rho_o=1.0 + p.m_minor - rw)
    drop64 = W.droplet_slab(n=16, radius=4.0, slab=4)
    drop16 = W.droplet_slab(n=16, radius=4.0, slab=4, precision="f16")
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from test_gpu_open import displacement
    fib = W.fiber_bundles(n=24, ncyl=6, precision="f64")
    one = W.uniform_gray(n=(6, 5, 12), phi=0.3, ncomp=1, precision="f64")
    return {"push_f32": (push, 20, "checkpoint"), "droplet_f64": (drop64, 20, ""),
            "droplet_f16": (drop16, 20, ""), "open_f64": (displacement(), 20, ""),
            "fiber_tensor_f64": (fib, 10, ""), "adjoint_f64": (one, 4, "adjoint")}


def test_debug_build_checks_pass_and_match_release():
    import paper_2512_21696_amd as L
    dbg = os.path.join(ROOT, "paper_2512_21696_amd", "liblbm_debug.so")
    assert os.path.exists(dbg), "build the debug library first (__graft_entry__.build())"
    with tempfile.TemporaryDirectory() as d:
        announce("debug build: child process over six small cases")
        env = dict(os.environ, LBM_LIBRARY=dbg)
        r = subprocess.run([sys.executable, "-u", "-c", CHILD, ROOT, d], env=env,
                           capture_output=True, text=True, timeout=600)
        print(r.stdout[-2000:], r.stderr[-2000:])
        assert r.returncode == 0, "debug build reported an error (a failed index check is LBM_E_DEVICE)"
        assert "done" in r.stdout
        for name, (wl, steps, extra) in cases().items():
            announce(f"debug build vs release: {name}")
            lb = L.lbm_create(wl["params"])
            lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
            lb.init_fluid(wl["rho_w"], wl["rho_o"])
            lb.step(steps)
            if extra == "checkpoint":
                lb.set_state(lb.get_state())
                lb.step(3)
            ref = dict(lb.get_fields())
            ref["diag"] = np.array([lb.get_diagnostics()[k]
                                    for k in ("mass_w", "mass_o", "q_acc_w", "max_u")])
            if extra == "adjoint":
                ref["dL_dphi"] = lb.adjoint_flux(4, np.ones(4))["dL_dphi"]
            lb.destroy()
            got = np.load(os.path.join(d, name + ".npz"))
            for k, v in ref.items():
                assert np.array_equal(got[k], v, equal_nan=True), (name, k)
