"""ABI behaviour that needs a device: an allocator hook that returns NULL."""
import ctypes

import pytest

import workloads as W
from gpu_common import announce

pytestmark = pytest.mark.gpu


def test_allocator_hook_returning_null_gives_nomem():
    """lbm_create takes all of its device memory through the hook; a hook that
    returns NULL makes it fail with LBM_E_NOMEM, return no handle and give back
    (through the free hook) nothing it did not get."""
    import torch
    import paper_2512_21696_amd as L
    announce("lbm_create with an allocator hook returning NULL")
    lib = L.load_library()
    p = L.to_c_params(W.droplet_slab(n=16, radius=4.0, slab=4)["params"])
    asked, freed = [], []

    def alloc(nbytes, ctx):
        asked.append(int(nbytes))
        return None

    def free(ptr, ctx):
        freed.append(ptr)

    cbs = (L.ALLOC_FN(alloc), L.FREE_FN(free))
    p.alloc, p.free = cbs
    p.stream = torch.cuda.current_stream().cuda_stream
    h = ctypes.c_void_p()
    rc = lib.lbm_create(ctypes.byref(p), ctypes.byref(h))
    assert rc == L.LBM_E_NOMEM
    assert not h.value
    assert len(asked) >= 1 and all(n > 0 for n in asked)
    assert all(f is None or f == 0 for f in freed)
    assert len(lib.lbm_last_error(None)) > 0


@pytest.mark.parametrize("track", [1, 0])
@pytest.mark.parametrize("case", ["droplet_f64", "rock_f32"])
def test_step_flux_history_equals_per_step_diagnostics(case, track):
    """lbm_step_flux records each step's outlet flux bitwise as the per-step
    lbm_get_diagnostics of a flux-tracking run reports it (q_w, q_o); the
    accumulated flux advances only when the handle tracks it, and the state
    is the one lbm_step reaches."""
    import copy

    import numpy as np

    import paper_2512_21696_amd as L
    wl = (W.droplet_slab(n=16, radius=4.0, slab=4) if case == "droplet_f64"
          else W.multiscale_rock(n=48, precision="f32"))
    n = 12
    announce(f"step_flux {case} track_flux={track}: {n} steps against per-step diagnostics")

    def handle(tr):
        p = copy.copy(wl["params"])
        p.track_flux = tr
        lb = L.lbm_create(p)
        lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
        lb.init_fluid(wl["rho_w"], wl["rho_o"])
        return lb

    lb = handle(1)
    ref = []
    for _ in range(n):
        lb.step(1)
        d = lb.get_diagnostics()
        ref.append((d["q_w"], d["q_o"]))
    acc_ref = lb.get_diagnostics()["q_acc_w"]
    fields_ref = lb.get_fields()
    lb.destroy()
    lb = handle(track)
    q = lb.step_flux(n)
    d = lb.get_diagnostics()
    fields = lb.get_fields()
    lb.destroy()
    assert q.shape == (n, 2)
    assert np.array_equal(q, np.array(ref))
    assert np.all(np.isfinite(q)) and np.any(q[:, 0] != 0.0)
    assert d["q_acc_w"] == (acc_ref if track else 0.0)
    for k in fields_ref:
        assert np.array_equal(fields[k], fields_ref[k]), k
