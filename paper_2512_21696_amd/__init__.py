"""Python binding of the gfx950 multiscale two-component D3Q19 library.

Argument marshalling only: every step of the method runs in the HIP kernels of
``liblbm.so`` behind the C ABI declared in ``include/lbm.h``.  PyTorch supplies
device memory (its caching allocator is passed in as the allocator hook) and
the stream (the current torch stream).  There is no CPU fallback: importing
this package without the built library, or creating a handle without a GPU,
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY selects another build of the library (the debug build,
# liblbm_debug.so, with device-side index checks)
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_STATE, LBM_E_NONFINITE, \
    LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "LBM_OK", -1: "LBM_E_INVAL", -2: "LBM_E_NOMEM", -3: "LBM_E_DEVICE",
          -4: "LBM_E_STATE", -5: "LBM_E_NONFINITE", -6: "LBM_E_UNSUPPORTED"}
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
STORE16 = ("f16", "bf16")
COLL = {"regularized": 0, "bgk": 1}
REGION = {"gray": 0, "all": 1}
BCX = {"periodic": 0, "pressure": 1, "density": 2}
LAYOUT = {"auto": 0, "dense": 1}
TABLE_N = 1025

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("ncomp", ctypes.c_int32), ("precision", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("tau", ctypes.c_double * 2), ("G", ctypes.c_double), ("g", (ctypes.c_double * 3) * 2),
        ("kappa", ctypes.c_double), ("csf_region", ctypes.c_int32), ("tensor", ctypes.c_int32),
        ("phi_max", ctypes.c_double), ("phi_avg", ctypes.c_double), ("m_minor", ctypes.c_double),
        ("s_min", ctypes.c_double), ("s_max", ctypes.c_double), ("wall_dpsi", ctypes.c_double * 2),
        ("kr_min", ctypes.c_double), ("c_max", ctypes.c_double), ("c_min", ctypes.c_double),
        ("hyst", ctypes.c_double), ("eps_n", ctypes.c_double), ("sigma_s", ctypes.c_double),
        ("smooth_radius", ctypes.c_int32), ("outlet_x", ctypes.c_int32),
        ("eps_g", ctypes.c_double), ("eps_H", ctypes.c_double), ("delta_tie", ctypes.c_double),
        ("diag_every", ctypes.c_int32), ("track_flux", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("rho_in", ctypes.c_double * 2), ("rho_out", ctypes.c_double * 2),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


class lbm_pore_table(ctypes.Structure):
    _fields_ = [("K0", ctypes.c_double * TABLE_N), ("Pc", ctypes.c_double * TABLE_N),
                ("Krw", ctypes.c_double * TABLE_N), ("Kro", ctypes.c_double * TABLE_N),
                ("phi_ref", ctypes.c_double), ("Pc_PM", ctypes.c_double),
                ("kd", ctypes.c_double * 3)]


PC_MAX_LEVELS = 16


class lbm_pc_params(ctypes.Structure):
    _fields_ = [("model", lbm_params), ("buffer_in", ctypes.c_int32),
                ("membrane", ctypes.c_int32), ("buffer_out", ctypes.c_int32),
                ("side_walls", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("rho_nw_in", ctypes.c_double * PC_MAX_LEVELS),
                ("membrane_phi", ctypes.c_double), ("check_every", ctypes.c_int64),
                ("max_steps", ctypes.c_int64), ("tol", ctypes.c_double)]


class lbm_pc_result(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("pc", ctypes.c_double * PC_MAX_LEVELS), ("sw", ctypes.c_double * PC_MAX_LEVELS),
                ("steps", ctypes.c_int64 * PC_MAX_LEVELS),
                ("converged", ctypes.c_int32 * PC_MAX_LEVELS)]


class lbm_fields(ctypes.Structure):
    _fields_ = [("on_device", ctypes.c_int32)] + [
        (k, ctypes.c_void_p) for k in ("rho_w", "rho_o", "ux", "uy", "uz", "S", "r_w", "r_o")]


class lbm_diag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("mass_w", "mass_o", "sw", "q_w", "q_o", "q_acc_w",
                                                "q_acc_o", "max_u")] + [
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class lbm_rev_domain(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("cls", ctypes.c_void_p), ("u_out", ctypes.c_void_p)]


class lbm_rev_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("g", ctypes.c_double), ("axis", ctypes.c_int32),
                ("collision", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("side_walls", ctypes.c_int32), ("mirror", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("max_steps", ctypes.c_int64),
                ("check_every", ctypes.c_int64), ("tol", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class lbm_rev_result(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("phi", ctypes.c_double), ("u_mean", ctypes.c_double),
                ("steps", ctypes.c_int64), ("converged", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("step_ms", ctypes.c_double)]


class lbm_kernel_times(ctypes.Structure):
    _fields_ = [("step_ms", ctypes.c_double), ("step_launches", ctypes.c_int64),
                ("aux_ms", ctypes.c_double), ("aux_launches", ctypes.c_int64),
                ("other_ms", ctypes.c_double), ("other_launches", ctypes.c_int64),
                ("adjoint_ms", ctypes.c_double), ("adjoint_launches", ctypes.c_int64)]


EXPORTS = ["lbm_params_default", "lbm_validate_params", "lbm_create", "lbm_set_geometry",
           "lbm_init_fluid", "lbm_step", "lbm_step_flux", "lbm_get_fields", "lbm_get_diagnostics", "lbm_get_setup",
           "lbm_state_size", "lbm_get_state", "lbm_set_state", "lbm_set_profiling",
           "lbm_get_kernel_times", "lbm_set_reservoirs", "lbm_rev_permeability",
           "lbm_rev_permeability_static", "lbm_rev_pc_sweep", "lbm_adjoint_flux",
           "lbm_get_layout", "lbm_last_error", "lbm_destroy"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblbm.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() or "
                          f"python paper_2512_21696_amd/build.py")
    try:  # torch first, so that the library binds to the HIP runtime torch loaded
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    dp, u8p = P(ctypes.c_double), P(ctypes.c_uint8)
    sig = {
        "lbm_params_default": (None, [P(lbm_params)]),
        "lbm_validate_params": (ctypes.c_int, [P(lbm_params), ctypes.c_char_p, sz]),
        "lbm_create": (ctypes.c_int, [P(lbm_params), P(vp)]),
        "lbm_set_geometry": (ctypes.c_int, [vp, u8p, dp, u8p, P(lbm_pore_table), i32]),
        "lbm_init_fluid": (ctypes.c_int, [vp, dp, dp]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_step_flux": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_double)]),
        "lbm_get_fields": (ctypes.c_int, [vp, P(lbm_fields)]),
        "lbm_get_diagnostics": (ctypes.c_int, [vp, P(lbm_diag)]),
        "lbm_get_setup": (ctypes.c_int, [vp, dp, dp, dp, dp, dp]),
        "lbm_state_size": (ctypes.c_int, [vp, P(sz)]),
        "lbm_get_state": (ctypes.c_int, [vp, vp, sz]),
        "lbm_set_state": (ctypes.c_int, [vp, vp, sz]),
        "lbm_set_profiling": (ctypes.c_int, [vp, i32]),
        "lbm_get_kernel_times": (ctypes.c_int, [vp, P(lbm_kernel_times), i32]),
        "lbm_set_reservoirs": (ctypes.c_int, [vp, dp, dp]),
        "lbm_rev_permeability": (ctypes.c_int, [P(lbm_rev_params), P(lbm_rev_domain), i32,
                                                P(lbm_rev_result)]),
        "lbm_rev_permeability_static": (ctypes.c_int, [P(lbm_rev_params), P(lbm_rev_domain),
                                                       i32, P(lbm_rev_result)]),
        "lbm_rev_pc_sweep": (ctypes.c_int, [P(lbm_pc_params), P(lbm_pore_table),
                                            P(lbm_rev_domain), i32, P(lbm_pc_result)]),
        "lbm_adjoint_flux": (ctypes.c_int, [vp, i64, dp, i64, dp, dp, dp]),
        "lbm_get_layout": (ctypes.c_int, [vp, P(i32), P(i64)]),
        "lbm_last_error": (ctypes.c_char_p, [vp]),
        "lbm_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def lbm_params_default() -> lbm_params:
    p = lbm_params()
    load_library().lbm_params_default(ctypes.byref(p))
    return p


def to_c_params(params) -> lbm_params:
    """workloads.Params (or any object with the same attribute names) -> lbm_params."""
    p = lbm_params_default()
    p.nx, p.ny, p.nz = int(params.nx), int(params.ny), int(params.nz)
    p.ncomp = int(params.ncomp)
    p.precision = PREC[params.precision]
    p.collision = COLL[params.collision]
    for a in range(2):
        p.tau[a] = float(params.tau[a] if a < len(params.tau) else 1.0)
        for d in range(3):
            p.g[a][d] = float(params.g[a][d])
        p.wall_dpsi[a] = float(params.wall_dpsi[a])
    p.G = float(params.G)
    p.kappa = float(params.kappa)
    p.csf_region = REGION[params.csf_region]
    p.bc_x = BCX[getattr(params, "bc_x", "periodic")]
    p.layout = LAYOUT[getattr(params, "layout", "auto")]
    for a in range(2):
        p.rho_in[a] = float(getattr(params, "rho_in", (1.0, 0.0))[a])
        p.rho_out[a] = float(getattr(params, "rho_out", (1.0, 0.0))[a])
    p.tensor = int(bool(params.tensor))
    for k in ("phi_max", "phi_avg", "m_minor", "s_min", "s_max", "kr_min", "c_max", "c_min",
              "hyst", "eps_n", "sigma_s", "eps_g", "eps_H", "delta_tie"):
        setattr(p, k, float(getattr(params, k)))
    p.smooth_radius = int(params.smooth_radius)
    p.outlet_x = int(params.outlet_x)
    p.diag_every = int(getattr(params, "diag_every", 0))
    p.track_flux = int(getattr(params, "track_flux", 1))
    return p


def to_c_tables(tables):
    arr = (lbm_pore_table * max(len(tables), 1))()
    for k, t in enumerate(tables):
        for name in ("K0", "Pc", "Krw", "Kro"):
            a = np.ascontiguousarray(t[name], dtype=np.float64)
            if a.shape != (TABLE_N,):
                raise ValueError(f"table {k} curve {name} must hold {TABLE_N} samples")
            ctypes.memmove(getattr(arr[k], name), a.ctypes.data, a.nbytes)
        arr[k].phi_ref = float(t["phi_ref"])
        arr[k].Pc_PM = float(t["Pc_PM"])
        for d in range(3):
            arr[k].kd[d] = float(t["kd"][d])
    return arr


class Lbm:
    """A handle of the C library.  Methods carry the ABI's names without the
    ``lbm_`` prefix and only marshal arguments."""

    def __init__(self, params, use_torch_memory: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the library has no CPU path")
        self.lib = load_library()
        self.params = params
        self.torch = torch
        cp = to_c_params(params)
        self.device = torch.cuda.current_device()
        self.stream = torch.cuda.current_stream()
        cp.stream = self.stream.cuda_stream
        self._cbs = None
        if use_torch_memory:
            dev, st = self.device, self.stream.cuda_stream

            def _alloc(nbytes, ctx):
                try:
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, st))
                except Exception:
                    return None

            def _free(ptr, ctx):
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:  # interpreter shutdown: torch already torn down
                    pass

            self._cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
            cp.alloc, cp.free = self._cbs
        self.c_params = cp
        h = ctypes.c_void_p()
        rc = self.lib.lbm_create(ctypes.byref(cp), ctypes.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_last_error(None).decode())
        self.h = h
        self.N = int(params.nx) * int(params.ny) * int(params.nz)
        self.shape = (int(params.nz), int(params.ny), int(params.nx))

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.lib.lbm_last_error(self.h).decode())

    def destroy(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # ------------------------------------------------------------------ calls
    def set_geometry(self, cls, phi, pore_type, tables):
        cls = np.ascontiguousarray(cls, dtype=np.uint8).reshape(-1)
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        pt = np.ascontiguousarray(pore_type, dtype=np.uint8).reshape(-1)
        assert cls.size == self.N and phi.size == self.N and pt.size == self.N
        self._fluid = (cls != 1).reshape(self.shape)
        tabs = to_c_tables(tables)
        self._check(self.lib.lbm_set_geometry(
            self.h, cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
            phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            pt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), tabs, len(tables)))

    def init_fluid(self, rho_w, rho_o=None):
        rw = np.ascontiguousarray(rho_w, dtype=np.float64).reshape(-1)
        ro = rw if rho_o is None else np.ascontiguousarray(rho_o, dtype=np.float64).reshape(-1)
        assert rw.size == self.N and ro.size == self.N
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.lbm_init_fluid(self.h, rw.ctypes.data_as(dp), ro.ctypes.data_as(dp)))

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def step_flux(self, n) -> np.ndarray:
        """n steps; the outlet flux of each, shape (n, 2): Q^w, Q^o per step
        (one synchronisation for all of them)."""
        q = np.zeros((int(n), 2), np.float64)
        self._check(self.lib.lbm_step_flux(self.h, int(n),
                                           q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return q

    FIELD_NAMES = ("rho_w", "rho_o", "ux", "uy", "uz", "S", "r_w", "r_o")

    def get_fields(self, names=FIELD_NAMES):
        """Host fp64 arrays shaped [z, y, x]."""
        out = {k: np.zeros(self.N, np.float64) for k in names}
        f = lbm_fields()
        f.on_device = 0
        for k in self.FIELD_NAMES:
            setattr(f, k, out[k].ctypes.data if k in out else None)
        self._check(self.lib.lbm_get_fields(self.h, ctypes.byref(f)))
        return {k: v.reshape(self.shape) for k, v in out.items()}

    def get_fields_device(self, tensors: dict):
        """Writes into caller device tensors (arithmetic dtype: float64 for f64
        runs, float32 otherwise; N elements each)."""
        f = lbm_fields()
        f.on_device = 1
        for k in self.FIELD_NAMES:
            t = tensors.get(k)
            setattr(f, k, t.data_ptr() if t is not None else None)
        self._check(self.lib.lbm_get_fields(self.h, ctypes.byref(f)))

    def get_diagnostics(self) -> dict:
        d = lbm_diag()
        self._check(self.lib.lbm_get_diagnostics(self.h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in lbm_diag._fields_ if k != "pad_"}

    def get_setup(self):
        arrs = [np.zeros(self.N) for _ in range(4)] + [np.zeros(6 * self.N)]
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.lbm_get_setup(self.h, *[a.ctypes.data_as(dp) for a in arrs]))
        K0, sJ, thw, tho, Kinv = arrs
        return dict(K0=K0.reshape(self.shape), sJ=sJ.reshape(self.shape),
                    thw=thw.reshape(self.shape), tho=tho.reshape(self.shape),
                    Kinv=Kinv.reshape((6,) + self.shape))

    def state_size(self) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.lbm_state_size(self.h, ctypes.byref(n)))
        return n.value

    def get_state(self) -> bytes:
        n = self.state_size()
        buf = ctypes.create_string_buffer(n)
        self._check(self.lib.lbm_get_state(self.h, buf, n))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.lbm_set_state(self.h, buf, len(blob)))

    def state_arrays(self, blob: bytes) -> dict:
        """Splits a state blob into its sections (views on the blob): the
        post-streaming populations ``f`` (f64/f32 runs) or their raw 16-bit
        offsets ``codes`` plus the reference densities ``ref`` [z][y][x][a]
        (two-component f16/bf16 runs; codes[a][i] at voxel d decodes as
        w_i (ref[s][a] + h), s = d - c_i, or d itself when d - c_i is solid),
        the residual amounts ``r`` and the side flags ``side``."""
        hdr = 8 + 4 + 4 + 4 * 4 + 8 + 4 * 8
        prec = self.params.precision
        es = 8 if prec == "f64" else 4
        dt = np.float64 if es == 8 else np.float32
        nc = int(self.params.ncomp)
        nf = nc * 19 * self.N
        raw = np.frombuffer(blob, dtype=np.uint8)
        out = {}
        if prec in STORE16:
            out["codes"] = raw[hdr:hdr + nf * 2].view(np.uint16).reshape((nc, 19) + self.shape)
            off = hdr + nf * 2
            if nc == 2:
                out["ref"] = raw[off:off + 2 * self.N * es].view(dt).reshape(self.shape + (2,))
                off += 2 * self.N * es
        else:
            out["f"] = raw[hdr:hdr + nf * es].view(dt).reshape((nc, 19) + self.shape)
            off = hdr + nf * es
        out["r"] = raw[off:off + 2 * self.N * es].view(dt).reshape((2,) + self.shape)
        out["side"] = raw[off + 2 * self.N * es:].reshape(self.shape)
        return out

    def set_reservoirs(self, rho_in, rho_out):
        a = (ctypes.c_double * 2)(*[float(v) for v in rho_in])
        b = (ctypes.c_double * 2)(*[float(v) for v in rho_out])
        self._check(self.lib.lbm_set_reservoirs(self.h, a, b))

    def adjoint_flux(self, nsteps, dL_dQ, checkpoint_every=0):
        """Runs nsteps steps from the current state and returns, for the loss
        L = sum_n dL_dQ[n] Q(n) on their outlet fluxes, a dict with the flux
        history "Q" [nsteps] and the gradients "dL_dK0" and "dL_dphi" as host
        fp64 arrays [z, y, x].  The handle ends nsteps steps on, as after
        step(nsteps)."""
        n = int(nsteps)
        a = np.ascontiguousarray(dL_dQ, dtype=np.float64).reshape(-1)
        if a.size != n:
            raise ValueError("dL_dQ needs one value per step")
        q = np.zeros(n, np.float64)
        gk = np.zeros(self.N, np.float64)
        gp = np.zeros(self.N, np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.lbm_adjoint_flux(self.h, n, a.ctypes.data_as(dp), int(checkpoint_every),
                                              q.ctypes.data_as(dp), gk.ctypes.data_as(dp),
                                              gp.ctypes.data_as(dp)))
        return {"Q": q, "dL_dK0": gk.reshape(self.shape), "dL_dphi": gp.reshape(self.shape)}

    def get_layout(self) -> dict:
        fo, sl = ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.lbm_get_layout(self.h, ctypes.byref(fo), ctypes.byref(sl)))
        return {"fluid_only": bool(fo.value), "slots": int(sl.value)}

    def set_profiling(self, on: bool):
        self._check(self.lib.lbm_set_profiling(self.h, int(bool(on))))

    def get_kernel_times(self, reset=False) -> dict:
        t = lbm_kernel_times()
        self._check(self.lib.lbm_get_kernel_times(self.h, ctypes.byref(t), int(bool(reset))))
        return {k: getattr(t, k) for k, _ in lbm_kernel_times._fields_}


def lbm_create(params, use_torch_memory: bool = True) -> Lbm:
    return Lbm(params, use_torch_memory)


def rev_permeability(domains, tau=1.0, g=1e-5, axis=0, collision="regularized",
                     precision="f32", side_walls=False, mirror=False, max_steps=2000,
                     check_every=100, tol=1e-6, want_u=False, stream=None, static=False):
    """Single-phase permeability K = phi <u> nu / g of every domain (a list of
    uint8 class arrays [z][y][x], 0 pore / 1 solid), all run together by
    lbm_rev_permeability (or, with static=True, by lbm_rev_permeability_static,
    which allocates no device memory).  Returns one dict per domain (K, phi,
    u_mean, steps, converged, and with want_u the final velocity field along
    the force)."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream().cuda_stream
        except ImportError:
            stream = None
    lib = load_library()
    arrs = [np.ascontiguousarray(c, dtype=np.uint8) for c in domains]
    outs = [np.zeros(a.shape) if want_u else None for a in arrs]
    doms = (lbm_rev_domain * len(arrs))()
    for k, a in enumerate(arrs):
        if a.ndim != 3:
            raise ValueError("each domain is a 3-D class array [z][y][x]")
        doms[k].nz, doms[k].ny, doms[k].nx = a.shape
        doms[k].cls = a.ctypes.data
        doms[k].u_out = outs[k].ctypes.data if want_u else None
    p = lbm_rev_params(tau=float(tau), g=float(g), axis=int(axis), collision=COLL[collision],
                       precision=PREC[precision], side_walls=int(bool(side_walls)),
                       mirror=int(bool(mirror)), max_steps=int(max_steps),
                       check_every=int(check_every), tol=float(tol), stream=stream)
    res = (lbm_rev_result * len(arrs))()
    fn = lib.lbm_rev_permeability_static if static else lib.lbm_rev_permeability
    rc = fn(ctypes.byref(p), doms, len(arrs), res)
    if rc != LBM_OK:
        raise LbmError(rc, lib.lbm_last_error(None).decode())
    out = []
    for k in range(len(arrs)):
        r = {n: getattr(res[k], n) for n in ("K", "phi", "u_mean", "steps", "converged",
                                             "step_ms")}
        if want_u:
            r["u"] = outs[k]
        out.append(r)
    return out


def rev_pc_sweep(domains, model, membrane_table, rho_nw_in, buffer_in=14, membrane=2,
                 buffer_out=2, side_walls=True, membrane_phi=0.3, check_every=200,
                 max_steps=4000, tol=1e-4, use_torch_memory=True):
    """Capillary-pressure sweep of every domain (uint8 class arrays [z][y][x],
    0 pore / 1 solid) by lbm_rev_pc_sweep: `model` (workloads.Params of the
    two-component model; grid, reservoirs and forces are set per domain),
    the membrane's pore table (a workloads.pore_table dict) and the inlet oil
    density of every level.  Returns one dict per domain: pc, sw, steps,
    converged (one entry per level)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the library has no CPU path")
    lib = load_library()
    levels = [float(v) for v in rho_nw_in]
    if not 1 <= len(levels) <= PC_MAX_LEVELS:
        raise ValueError(f"1 to {PC_MAX_LEVELS} levels")
    arrs = [np.ascontiguousarray(c, dtype=np.uint8) for c in domains]
    doms = (lbm_rev_domain * len(arrs))()
    for k, a in enumerate(arrs):
        if a.ndim != 3:
            raise ValueError("each domain is a 3-D class array [z][y][x]")
        doms[k].nz, doms[k].ny, doms[k].nx = a.shape
        doms[k].cls = a.ctypes.data
        doms[k].u_out = None
    p = lbm_pc_params()
    p.model = to_c_params(model)
    p.model.stream = torch.cuda.current_stream().cuda_stream
    cbs = None
    if use_torch_memory:
        dev, st = torch.cuda.current_device(), p.model.stream

        def _alloc(nbytes, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, st))
            except Exception:
                return None

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
        p.model.alloc, p.model.free = cbs
    p.buffer_in, p.membrane, p.buffer_out = int(buffer_in), int(membrane), int(buffer_out)
    p.side_walls, p.nlevels = int(bool(side_walls)), len(levels)
    for k, v in enumerate(levels):
        p.rho_nw_in[k] = v
    p.membrane_phi = float(membrane_phi)
    p.check_every, p.max_steps, p.tol = int(check_every), int(max_steps), float(tol)
    tab = to_c_tables([membrane_table])
    res = (lbm_pc_result * len(arrs))()
    rc = lib.lbm_rev_pc_sweep(ctypes.byref(p), tab, doms, len(arrs), res)
    if rc != LBM_OK:
        raise LbmError(rc, lib.lbm_last_error(None).decode())
    n = len(levels)
    return [{"pc": list(res[k].pc[:n]), "sw": list(res[k].sw[:n]),
             "steps": list(res[k].steps[:n]), "converged": list(res[k].converged[:n])}
            for k in range(len(arrs))]


def make_state_blob(lbm: Lbm, f, r, side, step=0, q_last=(0.0, 0.0), q_acc=(0.0, 0.0),
                    ref=None) -> bytes:
    """Builds a state blob (the ABI's checkpoint format) from post-streaming
    populations f[a][i][z][y][x], residual amounts r[2][z][y][x] and side flags.
    For f16/bf16 runs ``f`` holds the raw 16-bit offsets (uint16) and ``ref``
    the reference densities [z][y][x][a] (two components)."""
    import struct
    p = lbm.params
    dt = np.float64 if p.precision == "f64" else np.float32
    hdr = struct.pack("<QIIiiiiq4d", 0x4C424D3251313953, 1, PREC[p.precision], int(p.nx),
                      int(p.ny), int(p.nz), int(p.ncomp), int(step), q_last[0], q_last[1],
                      q_acc[0], q_acc[1])
    if p.precision in STORE16:
        body = np.ascontiguousarray(f, np.uint16).tobytes()
        if int(p.ncomp) == 2:
            if ref is None:
                raise ValueError("16-bit two-component blobs need the reference densities")
            body += np.ascontiguousarray(ref, np.float32).tobytes()
    else:
        body = np.ascontiguousarray(f, dt).tobytes()
    return (hdr + body + np.ascontiguousarray(r, dt).tobytes()
            + np.ascontiguousarray(side, np.uint8).tobytes())
