"""Shared helpers of the GPU parity tests (each test prints the case it runs
before touching the GPU)."""
import sys

import numpy as np

import workloads as W
from oracle import Oracle

FIELDS = ("rho_w", "rho_o", "ux", "uy", "uz", "S", "r_w", "r_o")


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(wl, steps, precision=None, params=None):
    import paper_2512_21696_amd as L
    p = params if params is not None else wl["params"]
    if precision is not None:
        p.precision = precision
        p.eps_n = 1e-12 if precision == "f64" else 1e-7
    lb = L.lbm_create(p)
    lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    lb.init_fluid(wl["rho_w"], wl["rho_o"])
    lb.step(steps)
    return lb


def oracle_run(wl, steps, params=None):
    o = Oracle(params if params is not None else wl["params"])
    o.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    o.init_fluid(wl["rho_w"], wl["rho_o"])
    o.step(steps)
    return o


def field_errors(got, ref, names=FIELDS):
    """Normalised max error per field: max|a - b| / max|b| (0 when both vanish)."""
    out = {}
    for k in names:
        scale = float(np.abs(ref[k]).max())
        diff = float(np.abs(np.asarray(got[k], np.float64) - ref[k]).max())
        out[k] = diff / scale if scale > 0 else diff
    return out


def diag_errors(dg, do, keys=("mass_w", "mass_o", "sw", "q_w", "q_o", "q_acc_w", "q_acc_o",
                              "max_u")):
    out = {}
    for k in keys:
        a, b = dg[k], do[k]
        out[k] = abs(a - b) / max(abs(b), 1e-300) if b != 0 else abs(a)
    return out
