"""Benchmark of the multiscale two-component D3Q19 step on one MI355X.

Workload: the 256^3 synthetic multiscale rock (Gaussian random field,
35 % solid / 20 % gray / 45 % pore, four Brooks-Corey pore types, water driven
in +x, CSF control at half the kappa = 0 surface tension), fp32 storage and
arithmetic.  A step is one full time step of the
method: density pass, CSF normals, the fused collide-stream kernel (forces,
constitutive update, residual transfer, collision, pull streaming) and the
per-step outlet-flux reduction; diagnostics (fp64 reductions with the
non-finite check) run every --diag-every steps inside the timed region.

Prints ONE JSON line.  value = fluid-voxel updates per second / 1e6 over the
timed steps (inputs resident in HBM); the roofline block prices the dominant
kernel (the fused step) with its algorithmic bytes per fluid update divided
by its mean launch time from HIP events on the library's stream.  Unless
--no-compare, the same workload also runs with fp64, fp32, fp16 and bf16
population storage: "storage_comparison" gives each one's MLUPS and its field
errors against the fp64 run after the same number of steps; "fiber_tensor"
times the one-component tensorial-resistivity workload (192^3 fibre bundles).
"""
import argparse
import hashlib
import json
import re
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COMPARED = ("rho_w", "rho_o", "ux", "uy", "uz", "S")
METRIC = "MLUPS (2-comp D3Q19) & % HBM peak; FP16-store vs FP32 MLUPS at stated error"


def algorithmic_bytes(ncomp, es, gray_frac, tensor, pop_es=None):
    """Bytes the method must move per fluid voxel update: every population read
    and written once, the class code, and the per-voxel inputs of gray voxels
    (K0, s_J, theta_w, theta_o, pore type; residual amounts and side flag read
    and written; the six inverse-permeability values for the tensor model).
    With 16-bit storage (pop_es = 2) a two-component voxel also reads its two
    fp32 reference densities."""
    pop_es = es if pop_es is None else pop_es
    pops = 2 * 19 * ncomp * pop_es
    if pop_es == 2 and ncomp == 2:
        pops += 2 * es
    gray = 0.0
    if ncomp == 2:
        gray = 4 * es + 1 + 2 * 2 * es + 2
    else:
        gray = es
    if tensor:
        gray += 6 * es
    return pops + 1 + gray_frac * gray


def kernel_source_hash():
    """Hash of what decides the step kernels' traffic: their sources and the
    runtime's functions that launch them or set their z chunk."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2512_21696_amd", "csrc")
    for f in ("lbm_kernels.hip", "lbm_step_tiled.hip", "lbm_internal.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "lbm_runtime.hip")) as fh:
        rt = fh.read()
    for name in ("ensure_density", "tiled_chunk", "launch_tiled", "launch_density_fix"):
        m = re.search(r"\n[^\n]*\b" + name + r"\(lbm_handle \*h[^{]*\{.*?\n\}\n", rt, re.S)
        if m is None:
            raise RuntimeError(f"{name} not found in lbm_runtime.hip")
        h.update(m.group(0).encode())
    return h.hexdigest()[:16]


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def measured_traffic(workload):
    """HBM traffic per step-kernel launch from the committed rocprofv3 counter
    summary, or None when the kernels changed since it was taken."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as fh:
        rec = json.load(fh).get("records", {}).get(workload)
    if rec is None or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def record_traffic(prefix, workload):
    """Turns four rocprofv3 --pmc passes into the traffic record of one workload:
    <prefix>_fetch and <prefix>_write (FETCH_SIZE, WRITE_SIZE of a short bench
    run), <prefix>_cfetch and <prefix>_cwrite (the same counters on the 1 GiB
    copy of --calibrate-copy, which fix the KiB-to-byte factors).  Each holds
    rocprofv3's run_counter_collection.csv."""
    import csv

    def per_dispatch(tag, name, required=True):
        vals = {}
        with open(f"{prefix}_{tag}/run_counter_collection.csv") as fh:
            for row in csv.DictReader(fh):
                if re.search(r"\b" + name + r"\b", row["Kernel_Name"].replace("<", " ")):
                    vals.setdefault(row["Dispatch_Id"], 0.0)
                    vals[row["Dispatch_Id"]] += float(row["Counter_Value"])
        if not vals:
            if not required:
                return None, 0
            raise SystemExit(f"no dispatch of {name} in {prefix}_{tag}")
        return sum(vals.values()) / len(vals), len(vals)

    gib = float(1 << 30)
    cf, _ = per_dispatch("cfetch", "k_probe_copy_b32")
    cw, _ = per_dispatch("cwrite", "k_probe_copy_b32")
    fs, fw = gib / (cf * 1024), gib / (cw * 1024)
    sf, n_disp = per_dispatch("fetch", "k_step_zm")
    sw, _ = per_dispatch("write", "k_step_zm")
    # the density work of a step: the fix-up after the step's own push, or
    # (storage kinds without the push) the density pass
    aux = "k_density_fix"
    df, nd = per_dispatch("fetch", aux, required=False)
    if not nd:
        aux = "k_density"
        df, _ = per_dispatch("fetch", aux)
    dw, _ = per_dispatch("write", aux)
    rec = {"kernel": "k_step_zm", "kernel_hash": kernel_source_hash(),
           "dispatches": n_disp,
           "fetch_size_kib_per_dispatch": round(sf, 1), "write_size_kib_per_dispatch": round(sw, 1),
           "fetch_scale": round(fs, 4), "write_scale": round(fw, 4),
           "read_bytes_per_launch": int(sf * 1024 * fs), "write_bytes_per_launch": int(sw * 1024 * fw),
           "bytes_per_launch": int(sf * 1024 * fs + sw * 1024 * fw),
           "aux_kernel": {"name": aux, "read_bytes": int(df * 1024 * fs),
                          "write_bytes": int(dw * 1024 * fw)}}
    out = {"note": "HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by "
                   "what the same counter reads for k_probe_copy_b32 (libhbmprobe.so: 1 GiB read "
                   "and 1 GiB written per dispatch); bench.py reports a record only while the "
                   "kernel sources hash to its kernel_hash", "records": {}}
    if os.path.exists(TRAFFIC_JSON):
        with open(TRAFFIC_JSON) as fh:
            old = json.load(fh)
        out["records"] = old.get("records", {})
    out["records"][workload] = rec
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({workload: rec}))


def fiber_permeability(n=192, steps=1000, g=1e-5):
    """The 3 x 3 effective permeability of the fibre bundles, nu <u_i> / g_j
    (mean over the fluid voxels) after `steps` steps from rest with the body
    acceleration along each axis in turn: transient (not converged), fp32."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L
    K = np.zeros((3, 3))
    for j in range(3):
        wf = W.fiber_bundles(n=n, precision="f32", direction=j, g=g)
        p = wf["params"]
        lb = L.lbm_create(p)
        lb.set_geometry(wf["cls"], wf["phi"], wf["ptype"], wf["tables"])
        lb.init_fluid(wf["rho_w"], wf["rho_o"])
        lb.step(steps)
        t = {k: torch.empty(wf["cls"].size, dtype=torch.float32, device="cuda")
             for k in ("ux", "uy", "uz")}
        lb.get_fields_device(t)
        torch.cuda.synchronize()
        lb.destroy()
        fl = torch.from_numpy((wf["cls"] != 1).reshape(-1)).cuda()
        nu = (p.tau[0] - 0.5) / 3.0
        for i, k in enumerate(("ux", "uy", "uz")):
            K[i, j] = nu * float(t[k][fl].double().mean()) / g
    return {"steps": steps, "g": g, "note": "transient, nu <u_i> / g_j over fluid voxels",
            "K": [[float(f"{v:.4e}") for v in row] for row in K]}


def pc_sweep(max_edge=40, count=6):
    """The capillary-pressure half of the library: a five-level drainage sweep
    (workloads.pc_sweep_setup) of the first `count` sphere packs of
    workloads.rev_domains with edge <= max_edge, fp32, 14 oil planes before
    each domain, a 2-plane membrane, side walls; each level until Sw changes
    by at most 1e-3 over 500 steps (20000 steps at most).  Reports every
    domain's Pc(Sw) points and the sweep's voxel updates per second (the
    whole box of each domain, every step, set-up and checks included)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L
    doms = [d["cls"] for d in W.rev_domains() if d["edge"] <= max_edge][:count]
    su = W.pc_sweep_setup(precision="f32")
    kw = dict(buffer_in=14, membrane=2, buffer_out=2, side_walls=True,
              membrane_phi=su["membrane_phi"], check_every=500, max_steps=20000, tol=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = L.rev_pc_sweep(doms, su["model"], su["membrane_table"], su["rho_nw_in"], **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    updates = 0
    for c, r in zip(doms, out):
        nz, ny, nx = c.shape
        updates += sum(r["steps"]) * (nx + 18) * (ny + 2) * (nz + 2)
    return {"domains": len(doms), "edges": [int(c.shape[0]) for c in doms], "storage": "f32",
            "levels_rho_oil_in": list(su["rho_nw_in"]), "seconds": round(dt, 2),
            "box_voxel_mlups": round(updates / dt / 1e6, 1),
            "curves": [{"pc": [round(v, 5) for v in r["pc"]], "sw": [round(v, 4) for v in r["sw"]],
                        "steps": r["steps"], "converged": r["converged"]} for r in out]}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(n_crop=64, steps=40):
    """The fp64 CPU oracle on a bounded sample: an n_crop^3 multiscale rock of
    the same recipe, a few steps, single thread."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    import workloads as W
    from oracle import Oracle
    wl = W.multiscale_rock(n=n_crop, precision="f64")
    o = Oracle(wl["params"])
    o.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    o.init_fluid(wl["rho_w"], wl["rho_o"])
    o.step(1)
    nfl = int(np.sum(wl["cls"] != 1))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": nfl * steps / dt / 1e6, "unit": "MLUPS (fluid voxels)", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_crop}^3 multiscale rock of the same recipe, fp64, {steps} steps "
                      f"after one warm-up step, single thread ({dt:.1f} s)"}


def calibrate_copy(mib=1024, narr=38, reps=5):
    """Yardsticks from libhbmprobe.so: plain copies of a known size (4-byte and
    16-byte accesses per lane), and a read and a write of 38 arrays of 256^3
    floats at the same index, one thread per index (the structure-of-arrays population pattern, 2.55
    GB at 256^3 in fp32).  Their counter readings convert FETCH_SIZE and
    WRITE_SIZE into bytes; their rates are the practical HBM ceiling."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2512_21696_amd", "libhbmprobe.so"))
    lib.hbm_probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_int, ctypes.c_void_p]
    torch.cuda.set_device(0)
    nbytes = mib << 20
    a = torch.arange(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    arr_bytes = narr * (256 ** 3) * 4
    big = torch.ones(arr_bytes // 4, dtype=torch.float32, device="cuda")
    out = torch.empty(256 ** 3, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    res = {}
    cases = [("copy_b32", 0, a, b, nbytes, 2 * nbytes), ("copy_b128", 1, a, b, nbytes, 2 * nbytes),
             ("read_38_arrays", 2, big, out, arr_bytes, arr_bytes),
             ("write_38_arrays", 3, None, big, arr_bytes, arr_bytes)]
    for name, kind, src, dst, size, moved in cases:
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            rc = lib.hbm_probe(kind, src.data_ptr() if src is not None else None, dst.data_ptr(),
                               size, narr, ctypes.c_void_p(st.cuda_stream))
            e1.record(st)
            if rc != 0:
                raise RuntimeError(f"hbm_probe {name} failed: {rc}")
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        best = min(ms[1:]) if len(ms) > 1 else ms[0]
        res[name] = {"bytes_read": size if kind != 3 else 0,
                     "bytes_written": size if kind in (0, 1) else (size if kind == 3 else 0),
                     "ms_best": round(best, 4), "gb_per_s": round(moved / (best * 1e-3) / 1e9, 1)}
    assert torch.equal(a, b)
    print(json.dumps({"yardsticks": res, "reps": reps}), flush=True)


def rev_library(steps=400):
    """The batched permeability library: 96 sphere-pack domains of edge 24..96
    (workloads.rev_domains) run together in fp32.  Fixed work first (`steps`
    steps; the per-step time is the library's HIP-event mean over the step
    launches, packing, set-up and checks excluded), then a run to convergence
    for the K values; then the four storage precisions side by side (the same
    fixed work, and K after 4000 steps against fp64)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L
    wr = W.rev_domains()
    doms = [d["cls"] for d in wr]
    nvox = sum(c.size for c in doms)
    npore = sum(int(np.count_nonzero(c == 0)) for c in doms)
    kw = dict(tau=1.0, g=1e-5, axis=0, precision="f32", check_every=100)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fixed = L.rev_permeability(doms, max_steps=steps, tol=0.0, **kw)
    t1 = time.perf_counter() - t1
    ms = fixed[0]["step_ms"]  # HIP events around the step launches
    t2 = time.perf_counter()
    conv = L.rev_permeability(doms, max_steps=20000, tol=1e-6, **kw)
    t2 = time.perf_counter() - t2
    K = np.array([r["K"] for r in conv])
    # pore voxels only: populations read and written, the 18 neighbour-table
    # entries (16-bit storage also reads and writes the writer's density)
    b = 2 * 19 * 4 + 18 * 4
    # storage precisions side by side: step time of the same fixed work, and K
    # of every domain after `kcmp` steps against the fp64 run's
    kcmp = 4000
    legs, Kp = {}, {}
    for prec in ("f64", "f32", "f16", "bf16"):
        es = {"f64": 8, "f32": 4}.get(prec, 2)
        kp = dict(kw, precision=prec)
        r = L.rev_permeability(doms, max_steps=steps, tol=0.0, **kp)
        pms = r[0]["step_ms"]
        Kp[prec] = np.array([x["K"] for x in L.rev_permeability(doms, max_steps=kcmp, tol=0.0, **kp)])
        bp = 2 * 19 * es + 18 * 4 + (8 if es == 2 else 0)
        legs[prec] = {"ms_per_step": round(pms, 4),
                      "value": round(npore / (pms * 1e-3) / 1e6, 1),
                      "bytes_per_pore_update": bp,
                      "frac": round(bp * npore / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    for prec in legs:
        rel = np.abs(Kp[prec] - Kp["f64"]) / np.abs(Kp["f64"])
        legs[prec]["K_rel_err_vs_f64_max"] = float(rel.max())
        legs[prec]["K_rel_err_vs_f64_median"] = float(np.median(rel))
    return {"workload": f"rev_domains_{len(doms)}", "domains": len(doms), "voxels": nvox,
            "pore_voxels": npore, "storage": "f32", "collision": "regularized", "tau": 1.0,
            "steps": steps, "ms_per_step": round(ms, 4), "call_seconds": round(t1, 3),
            "value": round(npore / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS (pore voxels)",
            "all_voxel_mlups": round(nvox / (ms * 1e-3) / 1e6, 1),
            "bytes_per_pore_update": b,
            "achieved_gbs": round(b * npore / (ms * 1e-3) / 1e9, 1),
            "frac": round(b * npore / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "to_convergence": {"tol": 1e-6, "seconds": round(t2, 2),
                               "converged": int(sum(r["converged"] for r in conv)),
                               "steps_max": int(max(r["steps"] for r in conv)),
                               "K_min": float(K.min()), "K_median": float(np.median(K)),
                               "K_max": float(K.max())},
            "storage_comparison": {"K_after_steps": kcmp, "legs": legs}}


def adjoint_gradient(n=96, steps=800, every=50, precision="f32", kind="rock"):
    """The porosity gradient of a flux loss.  kind "rock": workloads.adjoint_rock
    (the rock generator at n^3, one component, `steps` steps, squared misfit
    over steps 200..steps); kind "fiber": the n^3 gray fibre bundles with the
    tensorial resistivity, L = sum of Q(n) over steps 200..steps.  An untimed
    forward run for the flux history and dL/dQ, then lbm_adjoint_flux with
    checkpoints every `every` steps, timed on the host around the call
    (forward sweep, recomputation, reverse sweep, copies) and per kernel with
    the library's HIP events.  Beside it the plain forward run of the same
    steps."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L
    if kind == "rock":
        wl = W.adjoint_rock(n=n, steps=steps, precision=precision)
    elif kind in ("rock2", "rock2-kappa0"):
        wl = W.adjoint_rock2(n=n, steps=steps, precision=precision,
                             kappa=0.0 if kind == "rock2-kappa0" else None)
    else:
        wl = W.fiber_bundles(n=n, precision=precision)
        wl["params"].outlet_x = n // 2
        lin = np.where(np.arange(steps) >= 200, 1.0, 0.0)
        wl["target"] = lambda q: None
        wl["loss_grad"] = lambda q, t: (float(np.sum(lin * q)), lin)
    cls = wl["cls"]
    n_fluid = int(np.sum(cls != 1))
    gray_frac = float(np.sum(cls == 2)) / n_fluid
    lb = L.lbm_create(wl["params"])
    lb.set_geometry(cls, wl["phi"], wl["ptype"], wl["tables"])
    lb.init_fluid(wl["rho_w"], wl.get("rho_o"))
    start = lb.get_state()
    q = lb.step_flux(steps)[:, 0].copy()  # the flux history, one synchronisation
    loss, dLdQ = wl["loss_grad"](q, wl["target"](q))
    # forward alone
    lb.set_state(start)
    torch.cuda.synchronize()
    lb.set_profiling(True)
    lb.get_kernel_times(reset=True)
    t0 = time.perf_counter()
    lb.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    kf = lb.get_kernel_times(reset=True)
    # gradient
    lb.set_state(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = lb.adjoint_flux(steps, dLdQ, checkpoint_every=every)
    t_adj = time.perf_counter() - t0
    ka = lb.get_kernel_times(reset=True)
    # every level kept (checkpoint_every = steps: no recomputation, steps
    # population sets of HBM), when that fits in 150 GB
    es = 8 if precision == "f64" else 4
    all_levels = None
    if (steps + 2) * 19 * cls.size * es < 150e9:
        lb.set_state(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out_all = lb.adjoint_flux(steps, dLdQ, checkpoint_every=steps)
        t_all = time.perf_counter() - t0
        all_levels = {"gradient_seconds": round(t_all, 4),
                      "gradient_over_forward": round(t_all / t_fwd, 2),
                      "population_sets": steps + 2,
                      "same_gradient": bool(np.array_equal(out_all["dL_dphi"], out["dL_dphi"]))}
    lb.get_kernel_times(reset=True)
    lb.set_profiling(False)
    lb.destroy()
    # per fluid voxel: the recomputed set pulled, the adjoint set gathered and
    # written (storage type), the mask word; gray voxels read K0 and update
    # their fp64 dL/dK0, or (tensor) read K^-1 and update dL/dK^-1
    nc = int(wl["params"].ncomp)
    if nc == 1:
        b = 19 * es + 2 * 19 * es + 4 + gray_frac * ((es + 16) if kind == "rock" else (6 * es + 96))
    else:
        # two components, the reverse step's kernels (timed together; the
        # density, normals and neighbour-sum passes of the level are timed
        # apart): both sets pulled, both adjoint sets gathered and written
        # (3 x 38); the level's neighbour sums read (9), the neighbour part
        # read and written (2 + 2), the stash written and gathered (9 + 9),
        # the densities (2), the mask twice; gray voxels read r (2), K0, s_J,
        # theta (2), side flag and pore type, and update dL/dr and the dL/dK0,
        # dL/ds_J accumulators (4 doubles read and written)
        b = 2 * 19 * es * 3 + 33 * es + 8 + gray_frac * (6 * es + 2 + 64)
        if wl["params"].kappa != 0.0:
            # CSF: curvature (2) and own gradient (3) read, the curvature and
            # gradient adjoints stashed (8), the normals' reverse reading the
            # curvature adjoints (2), normals and gradients (12) and updating
            # the gradient adjoints (12), the gather reading them (6)
            b += 45 * es
    adj_ms = ka["adjoint_ms"] / max(ka["adjoint_launches"], 1)
    achieved = b * n_fluid / (adj_ms * 1e-3) / 1e9
    g = out["dL_dphi"]
    # the same gradient from fp64 storage (the reference the tests hold to
    # finite differences): its error against the largest gradient over the
    # gray voxels
    vs64 = None
    if precision != "f64":
        if kind == "rock":
            w64 = W.adjoint_rock(n=n, steps=steps, precision="f64")
        elif kind in ("rock2", "rock2-kappa0"):
            w64 = W.adjoint_rock2(n=n, steps=steps, precision="f64",
                                  kappa=0.0 if kind == "rock2-kappa0" else None)
        else:
            w64 = None
        if w64 is not None:
            l64 = L.lbm_create(w64["params"])
            l64.set_geometry(cls, w64["phi"], w64["ptype"], w64["tables"])
            l64.init_fluid(w64["rho_w"], w64.get("rho_o"))
            o64 = l64.adjoint_flux(steps, dLdQ, checkpoint_every=every)
            l64.destroy()
            gm = cls == 2
            d = np.abs(g[gm] - o64["dL_dphi"][gm]) / np.abs(o64["dL_dphi"][gm]).max()
            vs64 = {"max": float(d.max()), "p99": float(np.percentile(d, 99)),
                    "flux_history": float(np.abs(out["Q"] - o64["Q"]).max() /
                                          np.abs(o64["Q"]).max())}
    return {"workload": wl["name"], "storage": precision, "components": nc, "steps": steps,
            "tensor": kind == "fiber",
            "checkpoint_every": every, "fluid_voxels": n_fluid,
            "gray_voxels": int(np.sum(cls == 2)), "loss": loss,
            # the adjoint's forward sweep takes every level's densities from the
            # density pass; lbm_step (fp32, two components) from its own push:
            # equal to rounding there, bitwise otherwise
            "dL_dphi_vs_fp64": vs64,
            "flux_history_equal": bool(np.array_equal(out["Q"], q)),
            "flux_history_max_rel_diff": float(np.abs(out["Q"] - q).max() /
                                               max(np.abs(q).max(), 1e-300)),
            "forward_seconds": round(t_fwd, 4), "gradient_seconds": round(t_adj, 4),
            "gradient_over_forward": round(t_adj / t_fwd, 2),
            "all_levels_kept": all_levels,
            "step_kernel_ms": round(kf["step_ms"] / max(kf["step_launches"], 1), 4),
            "reverse_kernel_ms": round(adj_ms, 4),
            "reverse_kernel_launches": int(ka["adjoint_launches"]),
            "recompute_and_forward_step_launches": int(ka["step_launches"]),
            "kappa": float(wl["params"].kappa) if nc == 2 else None,
            "roofline": {"kernel": "k_adj_step" if nc == 1 else
                         ("k_adj_step2 + k_adj_nl2" +
                          (" + k_adj_normals_rev" if wl["params"].kappa != 0.0 else "")),
                         "bound": "hbm",
                         "bytes_per_fluid_update": round(b, 2),
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4)},
            "dL_dphi_max_abs": float(np.abs(g).max()),
            "dL_dphi_nonzero": int(np.count_nonzero(g))}


def precision_drift(n, steps, every=100):
    """The rock run in fp64, fp32, fp16 and bf16 storage side by side from the
    same initial state: per-field error against fp64 (max |X - X_f64| /
    max |X_f64|) at 100, 500, 1000, ... steps, and the global saturation, the
    water outlet flux and the relative mass change of every run every `every`
    steps.  Late-time divergence of an unstable displacement is expected and is
    reported as measured."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L

    torch.cuda.set_device(0)
    wl = W.multiscale_rock(n=n, precision="f64")
    checks = sorted({c for c in (100, 500, 1000, 2000, steps) if c <= steps})
    precs = ("f64", "f32", "f16", "bf16")
    runs = {}
    for prec in precs:
        p = wl["params"]
        p.precision = prec
        p.eps_n = 1e-12 if prec == "f64" else 1e-7
        p.diag_every = every
        lb = L.lbm_create(p)
        lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
        lb.init_fluid(wl["rho_w"], wl["rho_o"])
        runs[prec] = lb
    d0 = {prec: lb.get_diagnostics() for prec, lb in runs.items()}
    series = {prec: [] for prec in precs}
    errs = {prec: {} for prec in precs if prec != "f64"}
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for prec in list(runs):
            try:
                runs[prec].step(k)
            except L.LbmError as exc:  # a run that goes non-finite is reported and dropped
                series[prec].append({"step": done + k, "error": str(exc)})
                errs.pop(prec, None)
                runs.pop(prec).destroy()
        done += k
        if "f64" not in runs:
            break
        torch.cuda.synchronize()
        for prec, lb in runs.items():
            d = lb.get_diagnostics()
            series[prec].append({
                "step": d["step"], "sw": d["sw"], "q_w": d["q_w"], "nonfinite": d["nonfinite"],
                "mass_w_rel": d["mass_w"] / d0[prec]["mass_w"] - 1.0,
                "mass_o_rel": d["mass_o"] / d0[prec]["mass_o"] - 1.0})
        if done in checks:
            ref = {}
            for name in COMPARED:
                t = torch.empty(wl["cls"].size, dtype=torch.float64, device="cuda")
                runs["f64"].get_fields_device({name: t})
                ref[name] = t
            for prec in [q for q in errs if q in runs]:
                e = {}
                for name in COMPARED:
                    t = torch.empty(wl["cls"].size, dtype=torch.float32, device="cuda")
                    runs[prec].get_fields_device({name: t})
                    r = ref[name]
                    sc = r.abs().max().item()
                    d = t.double() - r
                    e[name] = float(f"{d.abs().max().item() / sc:.3e}")
                    e[name + "_rms"] = float(f"{d.square().mean().sqrt().item() / sc:.3e}")
                errs[prec][str(done)] = e
            del ref
            print(f"[drift] step {done}: " + json.dumps({p: errs[p].get(str(done)) for p in errs}),
                  file=sys.stderr, flush=True)
    for lb in runs.values():
        lb.destroy()
    print(json.dumps({"workload": wl["name"], "steps": steps, "compared_to": "f64 storage",
                      "error": "max |X - X_f64| / max |X_f64| per field; *_rms: root mean "
                               "square of X - X_f64 over all voxels / max |X_f64|",
                      "err_vs_f64": errs, "series_every": every, "series": series}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16", "bf16"])
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the runs of the other storage precisions")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only time a plain 1 GiB device copy (counter yardstick) and exit")
    ap.add_argument("--record-traffic", metavar="PREFIX",
                    help="only turn the rocprofv3 counter passes PREFIX_{fetch,write,cfetch,"
                         "cwrite} into the traffic record of --precision's workload (no GPU)")
    ap.add_argument("--rev", action="store_true",
                    help="only run the batched permeability library section and print its JSON, "
                         "then exit")
    ap.add_argument("--adjoint", action="store_true",
                    help="only run the porosity-gradient section and print its JSON, then exit")
    ap.add_argument("--adjoint-case", default="both", choices=["rock", "fiber", "rock2", "rock2-kappa0", "both"],
                    help="with --adjoint: which workload(s) to run")
    ap.add_argument("--drift", type=int, default=0, metavar="STEPS",
                    help="only run the storage precisions side by side for STEPS steps and "
                         "print their field errors against fp64 at checkpoints, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"slab decomposition is a design, not a built path", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.record_traffic:
        record_traffic(args.record_traffic, f"multiscale_rock_{args.n}_{args.precision}")
        return
    if args.drift:
        precision_drift(args.n, args.drift)
        return
    if args.rev:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"rev_library": rev_library(), "pc_sweep": pc_sweep()}), flush=True)
        return
    if args.adjoint:
        import torch
        torch.cuda.set_device(0)
        res = {}
        if args.adjoint_case in ("rock", "both"):
            res["adjoint_gradient"] = adjoint_gradient()
        if args.adjoint_case in ("fiber", "both"):
            res["adjoint_gradient_tensor"] = adjoint_gradient(n=192, steps=1000, kind="fiber")
        if args.adjoint_case in ("rock2", "both"):
            res["adjoint_gradient_two_component"] = adjoint_gradient(kind="rock2")
        if args.adjoint_case == "rock2-kappa0":
            res["adjoint_gradient_two_component_kappa0"] = adjoint_gradient(kind="rock2-kappa0")
        print(json.dumps(res), flush=True)
        return

    import numpy as np
    import torch
    import workloads as W
    import paper_2512_21696_amd as L

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    wl = W.multiscale_rock(n=args.n, precision=args.precision)
    cls = wl["cls"]
    n_fluid = int(np.sum(cls != 1))
    n_gray = int(np.sum(cls == 2))
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated {wl['name']} in {t_gen:.1f}s: fluid {n_fluid}, gray {n_gray}",
          file=sys.stderr, flush=True)

    def run_leg(precision, keep_fields, wl=wl):
        """Setup, warm-up and the timed steps of one storage precision; the
        fields after the last step stay on the device when asked for."""
        cls = wl["cls"]
        p = wl["params"]
        p.precision = precision
        p.eps_n = 1e-12 if precision == "f64" else 1e-7
        p.diag_every = args.diag_every
        lb = L.lbm_create(p)
        t0 = time.perf_counter()
        lb.set_geometry(cls, wl["phi"], wl["ptype"], wl["tables"])
        lb.init_fluid(wl["rho_w"], wl["rho_o"])
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        lb.step(args.warmup)
        torch.cuda.synchronize()
        lb.set_profiling(True)
        lb.get_kernel_times(reset=True)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        lb.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms = e0.elapsed_time(e1)
        kt = lb.get_kernel_times(reset=True)
        lb.set_profiling(False)
        diag = lb.get_diagnostics()
        fields = None
        if keep_fields:
            dt = torch.float64 if precision == "f64" else torch.float32
            fields = {k: torch.empty(cls.size, dtype=dt, device="cuda") for k in COMPARED}
            lb.get_fields_device(fields)
            torch.cuda.synchronize()
        lb.destroy()
        print(f"[bench] {precision}: setup {t_setup:.2f}s, {args.steps} steps in "
              f"{total_ms:.1f} ms; diag {diag}", file=sys.stderr, flush=True)
        return dict(total_ms=total_ms, kt=kt, diag=diag, fields=fields, t_setup=t_setup)

    compare = not args.no_compare
    main_leg = run_leg(args.precision, compare)
    total_ms, kt, diag = main_leg["total_ms"], main_leg["kt"], main_leg["diag"]
    ms_per_step = total_ms / args.steps
    mlups = n_fluid * args.steps / (total_ms * 1e-3) / 1e6
    es = 8 if args.precision == "f64" else 4
    pop_es = 2 if args.precision in ("f16", "bf16") else es
    b_alg = algorithmic_bytes(2, es, n_gray / n_fluid, False, pop_es)
    step_ms = kt["step_ms"] / max(kt["step_launches"], 1)
    achieved = b_alg * n_fluid / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic(wl["name"] + "_" + args.precision)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": wl["name"], "grid": [args.n] * 3, "components": 2,
                   "fluid_voxels": n_fluid, "gray_voxels": n_gray,
                   "sigma_scale": 0.5, "kappa": wl["params"].kappa,
                   "storage": args.precision, "diag_every": args.diag_every,
                   "lups_counted_over": "fluid (pore + gray) voxels",
                   "all_voxel_mlups": round(args.n ** 3 * args.steps / (total_ms * 1e-3) / 1e6, 2),
                   "setup_s": round(main_leg["t_setup"], 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_step_zm (fused collide-stream)",
                     "bytes_per_fluid_update": round(b_alg, 2),
                     "kernel_ms": round(step_ms, 4),
                     # the whole step (fused kernel, density work, flux and
                     # diagnostics) against the same algorithmic bytes
                     "step_achieved": round(b_alg * n_fluid / (ms_per_step * 1e-3) / 1e9, 1),
                     "step_frac": round(b_alg * n_fluid / (ms_per_step * 1e-3) / 1e9 /
                                        HBM_PEAK_GBS, 4),
                     "step_time_share": round(kt["step_ms"] / total_ms, 4),
                     "aux_ms_per_step": round(kt["aux_ms"] / args.steps, 4),
                     "other_ms_per_step": round(kt["other_ms"] / args.steps, 4)},
        "diagnostics": {k: diag[k] for k in ("mass_w", "mass_o", "sw", "max_u", "nonfinite",
                                             "step")},
    }
    if compare:
        # the other storage precisions on the same workload and step count, and
        # their field errors against the fp64 run (itself held to 1e-12 of the
        # oracle by the parity tests) after warm-up + timed steps
        legs = {args.precision: main_leg}
        for prec in ("f64", "f32", "f16", "bf16"):
            if prec not in legs:
                legs[prec] = run_leg(prec, True)
        ref = legs["f64"]["fields"]
        mass0 = legs["f64"]["diag"]
        comp = {}
        for prec in ("f32", "f16", "bf16", "f64"):
            lg = legs[prec]
            t = lg["total_ms"]
            k = lg["kt"]
            e = {}
            if prec != "f64":
                for name in COMPARED:
                    r = ref[name]
                    d = (lg["fields"][name].double() - r).abs().max().item()
                    sc = r.abs().max().item()
                    e[name] = d / sc if sc > 0 else d
                e["mass_w"] = abs(lg["diag"]["mass_w"] - mass0["mass_w"]) / mass0["mass_w"]
                e["mass_o"] = abs(lg["diag"]["mass_o"] - mass0["mass_o"]) / mass0["mass_o"]
            comp[prec] = {
                "value": round(n_fluid * args.steps / (t * 1e-3) / 1e6, 2),
                "ms_per_step": round(t / args.steps, 4),
                "kernel_ms": round(k["step_ms"] / max(k["step_launches"], 1), 4),
                "aux_ms_per_step": round(k["aux_ms"] / args.steps, 4),
                "speedup_vs_f32": None,
                "err_vs_f64_after_steps": args.warmup + args.steps,
                "err_vs_f64": {n: float(f"{v:.3e}") for n, v in e.items()},
            }
        for prec in comp:
            comp[prec]["speedup_vs_f32"] = round(comp["f32"]["ms_per_step"] /
                                                 comp[prec]["ms_per_step"], 3)
        out["storage_comparison"] = {
            "note": "same workload and steps per storage precision; err = max|X - X_f64| / "
                    "max|X_f64| per field after warm-up + timed steps, mass = relative "
                    "difference of total component mass",
            "legs": comp}
        for lg in legs.values():
            lg["fields"] = None
        # the same rock with the surface tension doubled by the CSF control
        w2 = W.multiscale_rock(n=args.n, precision="f32", sigma_scale=2.0)
        l2 = run_leg("f32", False, wl=w2)
        out["sigma_2x"] = {"kappa": w2["params"].kappa, "storage": "f32",
                           "value": round(n_fluid * args.steps / (l2["total_ms"] * 1e-3) / 1e6, 2),
                           "ms_per_step": round(l2["total_ms"] / args.steps, 4),
                           "kernel_ms": round(l2["kt"]["step_ms"] /
                                              max(l2["kt"]["step_launches"], 1), 4),
                           "diagnostics": {k: l2["diag"][k] for k in ("mass_w", "mass_o", "sw",
                                                                       "max_u", "nonfinite")}}
        # the tensorial-resistivity workload: 192^3 gray fibre bundles, one
        # component, principal axes from the smoothed porosity
        wf = W.fiber_bundles(n=192, precision="f32")
        nf_fl = int(np.sum(wf["cls"] != 1))
        nf_gr = int(np.sum(wf["cls"] == 2))
        lf = run_leg("f32", False, wl=wf)
        kf = lf["kt"]
        fms = kf["step_ms"] / max(kf["step_launches"], 1)
        bf = algorithmic_bytes(1, 4, nf_gr / nf_fl, True)
        out["fiber_tensor"] = {
            "workload": wf["name"], "components": 1, "tensor": True, "storage": "f32",
            "fluid_voxels": nf_fl, "gray_voxels": nf_gr,
            "value": round(nf_fl * args.steps / (lf["total_ms"] * 1e-3) / 1e6, 2),
            "unit": "MLUPS", "ms_per_step": round(lf["total_ms"] / args.steps, 4),
            "kernel_ms": round(fms, 4), "bytes_per_fluid_update": round(bf, 2),
            "achieved_gbs": round(bf * nf_fl / (fms * 1e-3) / 1e9, 1),
            "frac": round(bf * nf_fl / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "effective_permeability": fiber_permeability()}
        # the same rock between exact density faces (open x faces: no density
        # push, so the step takes the density pass): water enters at x = 0
        # against oil held at x = nx - 1
        wo = W.multiscale_rock(n=args.n, precision="f32")
        po = wo["params"]
        m = po.m_minor
        po.bc_x = "density"
        po.outlet_x = args.n - 2
        po.rho_in, po.rho_out = (1.0 + 0.02, m), (m, 1.0)
        for a_ in ("cls", "phi", "ptype"):
            wo[a_] = wo[a_].copy()
        wo["cls"][:, :, -2:] = 0          # no gray (or grain) voxel on the outlet planes
        wo["phi"][:, :, -2:] = 1.0
        lo = run_leg("f32", False, wl=wo)
        ko = lo["kt"]
        oms = ko["step_ms"] / max(ko["step_launches"], 1)
        no_fl = int(np.sum(wo["cls"] != 1))
        bo = algorithmic_bytes(2, 4, int(np.sum(wo["cls"] == 2)) / no_fl, False)
        out["open_faces"] = {
            "workload": wo["name"] + "_density_faces", "bc_x": "density", "storage": "f32",
            "rho_in": list(po.rho_in), "rho_out": list(po.rho_out), "fluid_voxels": no_fl,
            "value": round(no_fl * args.steps / (lo["total_ms"] * 1e-3) / 1e6, 2),
            "unit": "MLUPS", "ms_per_step": round(lo["total_ms"] / args.steps, 4),
            "kernel_ms": round(oms, 4), "aux_ms_per_step": round(ko["aux_ms"] / args.steps, 4),
            "bytes_per_fluid_update": round(bo, 2),
            "frac": round(bo * no_fl / (oms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "diagnostics": {k: lo["diag"][k] for k in ("mass_w", "mass_o", "q_acc_w", "q_acc_o",
                                                       "max_u", "nonfinite")}}
    if compare:
        out["rev_library"] = rev_library()
        out["pc_sweep"] = pc_sweep()
        out["adjoint_gradient"] = adjoint_gradient()
        out["adjoint_gradient_tensor"] = adjoint_gradient(n=192, steps=1000, kind="fiber")
        out["adjoint_gradient_two_component"] = adjoint_gradient(kind="rock2")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["host"] = cpu_model()
        out["cpu_baseline"]["nproc"] = os.cpu_count()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
