"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and validates arguments on the host."""
import ctypes
import os
import re

import pytest

import paper_2512_21696_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    pat = r"^(?:int|void|const char \*)\s*(lbm_[a-z_]+)\s*\("
    return sorted(set(re.findall(pat, src, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = L.load_library()
    names = header_functions()
    assert set(names) == set(L.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def test_defaults_validate():
    p = L.lbm_params_default()
    assert p.nx == 32 and p.ncomp == 2 and p.precision == 0 and p.track_flux == 1
    assert p.layout == 0  # LBM_LAYOUT_AUTO
    assert abs(p.m_minor - 0.0029912221254390597) < 1e-18
    msg = ctypes.create_string_buffer(256)
    assert L.load_library().lbm_validate_params(ctypes.byref(p), msg, 256) == L.LBM_OK


@pytest.mark.parametrize("field,value,code", [
    ("tau", (0.5, 1.0), L.LBM_E_INVAL), ("ncomp", 3, L.LBM_E_INVAL), ("nx", 0, L.LBM_E_INVAL),
    ("precision", 7, L.LBM_E_UNSUPPORTED), ("outlet_x", 32, L.LBM_E_INVAL),
    ("hyst", 0.5, L.LBM_E_INVAL), ("kr_min", 0.0, L.LBM_E_INVAL), ("layout", 2, L.LBM_E_INVAL)])
def test_invalid_params_rejected_on_host(field, value, code):
    lib = L.load_library()
    p = L.lbm_params_default()
    if field == "tau":
        p.tau[0], p.tau[1] = value
    else:
        setattr(p, field, value)
    msg = ctypes.create_string_buffer(256)
    assert lib.lbm_validate_params(ctypes.byref(p), msg, 256) == code
    assert len(msg.value) > 0
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(p), ctypes.byref(h)) == code
    assert not h.value
    assert len(lib.lbm_last_error(None)) > 0


def test_oversized_grid_unsupported():
    p = L.lbm_params_default()
    p.nx = p.ny = p.nz = 400
    assert L.load_library().lbm_validate_params(ctypes.byref(p), None, 0) == L.LBM_E_UNSUPPORTED


@pytest.mark.parametrize("prec,largest,next_up", [
    (L.PREC["f32"], (384, 384, 383), (384, 384, 384)),   # 2*19*N below 2^31
    (L.PREC["f16"], (384, 384, 383), (384, 384, 384)),
    (L.PREC["f64"], (304, 304, 305), (304, 304, 306))])  # 19*N*8 bytes below 4 GiB
def test_largest_accepted_grid(prec, largest, next_up):
    lib = L.load_library()
    p = L.lbm_params_default()
    p.precision = prec
    p.nx, p.ny, p.nz = largest
    assert lib.lbm_validate_params(ctypes.byref(p), None, 0) == L.LBM_OK
    p.nx, p.ny, p.nz = next_up
    assert lib.lbm_validate_params(ctypes.byref(p), None, 0) == L.LBM_E_UNSUPPORTED


def test_null_handle_calls_fail_cleanly():
    lib = L.load_library()
    assert lib.lbm_step(None, 1) == L.LBM_E_INVAL
    assert lib.lbm_init_fluid(None, None, None) == L.LBM_E_INVAL
    assert lib.lbm_get_layout(None, None, None) == L.LBM_E_INVAL
    lib.lbm_destroy(None)


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import workloads as W
    with pytest.raises(RuntimeError):
        L.lbm_create(W.Params().filled())


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), L.LBM_E_INVAL), (dict(g=0.0), L.LBM_E_INVAL), (dict(axis=3), L.LBM_E_INVAL),
    (dict(check_every=0), L.LBM_E_INVAL), (dict(max_steps=-1), L.LBM_E_INVAL),
    (dict(tol=-1.0), L.LBM_E_INVAL)])
def test_rev_permeability_rejects_bad_arguments_on_host(kw, code):
    import numpy as np
    with pytest.raises(L.LbmError) as e:
        L.rev_permeability([np.zeros((4, 4, 4), np.uint8)], **kw)
    assert e.value.code == code
    assert len(L.load_library().lbm_last_error(None)) > 0


def test_rev_permeability_rejects_unknown_precision_on_host():
    import numpy as np
    lib = L.load_library()
    p = L.lbm_rev_params(tau=1.0, g=1e-5, max_steps=10, check_every=5, precision=7)
    res = (L.lbm_rev_result * 1)()
    doms = (L.lbm_rev_domain * 1)()
    cls = np.zeros((2, 2, 2), np.uint8)
    doms[0].nx = doms[0].ny = doms[0].nz = 2
    doms[0].cls = cls.ctypes.data
    assert lib.lbm_rev_permeability(ctypes.byref(p), doms, 1, res) == L.LBM_E_UNSUPPORTED


def test_rev_permeability_rejects_empty_and_bad_domains_on_host():
    import numpy as np
    lib = L.load_library()
    p = L.lbm_rev_params(tau=1.0, g=1e-5, max_steps=10, check_every=5)
    res = (L.lbm_rev_result * 1)()
    doms = (L.lbm_rev_domain * 1)()
    assert lib.lbm_rev_permeability(ctypes.byref(p), doms, 0, res) == L.LBM_E_INVAL
    assert lib.lbm_rev_permeability(ctypes.byref(p), doms, 1, res) == L.LBM_E_INVAL  # no box
    cls = np.zeros((2, 2, 2), np.uint8)
    doms[0].nx = doms[0].ny = doms[0].nz = 2
    doms[0].cls = None
    assert lib.lbm_rev_permeability(ctypes.byref(p), doms, 1, res) == L.LBM_E_INVAL
    del cls


def _pc_args(**kw):
    import numpy as np
    import workloads as W
    su = W.pc_sweep_setup()
    p = L.lbm_pc_params()
    p.model = L.to_c_params(su["model"])
    p.buffer_in, p.membrane, p.buffer_out, p.side_walls = 4, 2, 2, 1
    p.nlevels = 2
    p.rho_nw_in[0], p.rho_nw_in[1] = 1.05, 1.1
    p.membrane_phi, p.check_every, p.max_steps, p.tol = 0.3, 10, 20, 1e-4
    for k, v in kw.items():
        if k == "precision":
            p.model.precision = v
        else:
            setattr(p, k, v)
    cls = np.zeros((4, 4, 4), np.uint8)
    doms = (L.lbm_rev_domain * 1)()
    doms[0].nz = doms[0].ny = doms[0].nx = 4
    doms[0].cls = cls.ctypes.data
    return p, L.to_c_tables([su["membrane_table"]]), doms, cls


@pytest.mark.parametrize("kw,code", [
    (dict(nlevels=0), L.LBM_E_INVAL), (dict(nlevels=17), L.LBM_E_INVAL),
    (dict(buffer_out=1), L.LBM_E_INVAL), (dict(membrane=0), L.LBM_E_INVAL),
    (dict(buffer_in=0), L.LBM_E_INVAL), (dict(membrane_phi=1.0), L.LBM_E_INVAL),
    (dict(check_every=0), L.LBM_E_INVAL), (dict(max_steps=5), L.LBM_E_INVAL),
    (dict(tol=-1.0), L.LBM_E_INVAL), (dict(precision=2), L.LBM_E_UNSUPPORTED)])
def test_pc_sweep_rejects_bad_arguments_on_host(kw, code):
    lib = L.load_library()
    p, tab, doms, cls = _pc_args(**kw)
    res = (L.lbm_pc_result * 1)()
    assert lib.lbm_rev_pc_sweep(ctypes.byref(p), tab, doms, 1, res) == code
    assert len(lib.lbm_last_error(None)) > 0


def test_pc_sweep_rejects_null_and_bad_levels_on_host():
    lib = L.load_library()
    p, tab, doms, cls = _pc_args()
    res = (L.lbm_pc_result * 1)()
    assert lib.lbm_rev_pc_sweep(ctypes.byref(p), None, doms, 1, res) == L.LBM_E_INVAL
    assert lib.lbm_rev_pc_sweep(ctypes.byref(p), tab, doms, 0, res) == L.LBM_E_INVAL
    p.rho_nw_in[1] = float("nan")
    assert lib.lbm_rev_pc_sweep(ctypes.byref(p), tab, doms, 1, res) == L.LBM_E_INVAL


def test_pc_structs_match_the_header():
    """sizeof of the sweep's structs as the C compiler lays them out."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "%s"\nint main(void){'
           'printf("%%zu %%zu %%zu %%zu\\n", sizeof(lbm_params), sizeof(lbm_pc_params), '
           'sizeof(lbm_pc_result), offsetof(lbm_params, layout));return 0;}\n'
           % os.path.join(ROOT, "include", "lbm.h"))
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "s.c"), os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-o", exe, c], check=True)
        sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                                 check=True).stdout.split()]
    assert sizes == [ctypes.sizeof(L.lbm_params), ctypes.sizeof(L.lbm_pc_params),
                     ctypes.sizeof(L.lbm_pc_result), L.lbm_params.layout.offset]
