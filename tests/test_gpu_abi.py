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
