"""Parity at the benchmark's full sizes and launch configuration: the 256^3
multiscale rock in fp32 and with fp16 / bf16 storage, and the 192^3 gray
fibre bundles (one component, tensorial resistivity) in fp32, run through the
C ABI, then one more step compared voxel by voxel on sampled voxels against
the fp64 oracle; and the 256^3 rock over its full 2000 steps in fp32 and fp64
without a non-finite value.

The oracle cannot run 16.7 M voxels, but the update of one voxel depends only
on the post-streaming populations within three voxels of it (pull: radius 1;
pseudo-potential and grad S_hat: densities at radius 1 of the neighbours that
are pulled from; CSF: normals at radius 1, each from densities at radius 1,
of those neighbours).  So each sampled voxel is checked on a periodic 9^3
crop centred on it (radius 4, one spare layer): the oracle steps the crop
once and the centre's new post-streaming populations, residual amounts and
side flag must match the GPU's.

Tolerances: one fp32 step from the same state differs from the fp64 oracle
only by fp32 rounding, a few ulps of the largest operands (densities O(1)):
1e-5 of each voxel's largest f_i / w_i.  16-bit storage adds one rounding of
the stored offset |h| <= 1: at most 2^-11 for fp16 (tolerance 1e-3) and 2^-8
for bf16 (tolerance 4e-3)."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle, W as WQ, C as CQ, gray_parameters, inverse_permeability
from gpu_common import announce

pytestmark = pytest.mark.gpu

R = 4


def _categories(cls, rng, per=24):
    """Seeded sample of fluid voxels: gray and pore voxels, each in the
    interior and at the other class (next to a solid where the domain has
    solids, else next to the other fluid class), and voxels on the fused
    kernel's tile edges (x = 64 k - 1, 64 k; y = 4 k - 1, 4 k;
    z = 32 k - 1, 32 k) and on the periodic wrap."""
    n = cls.shape[0]
    has_solid = bool((cls == W.SOLID).any())
    picks = []
    for c, cname in ((W.GRAY, "gray"), (W.PORE, "pore")):
        other = cls == W.SOLID if has_solid else (cls != c)
        near = np.zeros_like(other)
        for ax in range(3):
            for sh in (-1, 1):
                near |= np.roll(other, sh, axis=ax)
        where = "solid" if has_solid else ("pore" if c == W.GRAY else "gray")
        for name, sel in ((f"{cname} interior", (cls == c) & ~near),
                          (f"{cname} at {where}", (cls == c) & near)):
            idx = np.flatnonzero(sel)
            take = rng.choice(idx, size=min(per, idx.size), replace=False)
            picks += [(name, int(t)) for t in take]
    fluid = cls != W.SOLID
    edge_x = np.unique([v for k in range(0, n + 1, 64) for v in (k - 1, k)] + [0, 1, n - 2, n - 1])
    edge_y = np.unique([v for k in range(0, n + 1, 4) for v in (k - 1, k)][:12] + [n - 1])
    edge_z = np.unique([v for k in range(0, n + 1, 32) for v in (k - 1, k)] + [n - 1])
    edge_x, edge_y, edge_z = (e[(e >= 0) & (e < n)] for e in (edge_x, edge_y, edge_z))
    got = 0
    while got < 2 * per:
        z = int(rng.choice(edge_z) if rng.random() < 0.5 else rng.integers(n))
        y = int(rng.choice(edge_y) if rng.random() < 0.5 else rng.integers(n))
        x = int(rng.choice(edge_x))
        if fluid[z, y, x]:
            picks.append(("tile edges and wrap", int(np.ravel_multi_index((z, y, x), cls.shape))))
            got += 1
    return picks


def _crop(a, c, lead):
    """Periodic (2R+1)^3 crop of a [..., z, y, x] array around c = (z, y, x)."""
    n = a.shape[-1]
    idx = [np.arange(ci - R, ci + R + 1) % n for ci in c]
    return a[(slice(None),) * lead + np.ix_(*idx)]


def _states(wl, prec, steps):
    import paper_2512_21696_amd as L
    p = wl["params"]
    announce(f"{wl['name']} {prec}: {steps} steps, state, one step, state")
    lb = L.lbm_create(p)
    lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    lb.init_fluid(wl["rho_w"], wl["rho_o"])
    lb.step(steps)
    d0 = lb.get_diagnostics()
    s0 = lb.state_arrays(lb.get_state())
    lb.step(1)
    d1 = lb.get_diagnostics()
    s1 = lb.state_arrays(lb.get_state())
    lb.destroy()
    return s0, s1, d0, d1


def _decoded_crop(st, prec, c, cls):
    """f / w_i (float64) of the (2R+1)^3 crop of a state around c; a 16-bit
    offset pulled by voxel d in direction i decodes as rho_ref(s) + h with s
    the voxel it came from (d - c_i, or d itself when d - c_i is solid);
    solid voxels decode as 0."""
    w = WQ.reshape((1, 19, 1, 1, 1))
    if prec == "f32":
        return _crop(st["f"], c, 2).astype(np.float64) / w
    bits = _crop(st["codes"], c, 2)
    if prec == "f16":
        h = bits.view(np.float16).astype(np.float64)
    else:
        h = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    n = cls.shape[0]
    ref_full = np.moveaxis(st["ref"], -1, 0)  # [a][z][y][x]
    own = _crop(ref_full, c, 1).astype(np.float64)
    refs = np.empty(h.shape)
    for i in range(19):
        shift = (int(CQ[i, 2]), int(CQ[i, 1]), int(CQ[i, 0]))  # (c_z, c_y, c_x)
        idx = [(np.arange(ci - R, ci + R + 1) - d) % n for ci, d in zip(c, shift)]
        src = ref_full[(slice(None),) + np.ix_(*idx)].astype(np.float64)
        src_solid = cls[np.ix_(*idx)] == W.SOLID
        refs[:, i] = np.where(src_solid[None], own, src)
    solid = _crop(cls, c, 0) == W.SOLID
    return np.where(solid[None, None], 0.0, refs + h)


def _sampled_step(wl, prec, tol, steps=20):
    s0, s1, d0, d1 = _states(wl, prec, steps)
    cls = wl["cls"]
    w = WQ.reshape((1, 19, 1, 1, 1))
    picks = _categories(cls, np.random.default_rng(7))
    ncat = len({name for name, _ in picks})
    p = W.Params(**{**wl["params"].as_dict(), "nx": 2 * R + 1, "ny": 2 * R + 1,
                    "nz": 2 * R + 1, "precision": "f64", "outlet_x": 0})
    hy = p.hyst
    Kinv = None
    if p.tensor:
        # the inverse permeability comes from a smoothed porosity field (a
        # wider stencil than the crop): take the oracle's on the whole grid,
        # its eigen-analysis only at the gray voxels within radius 1 of the
        # sampled voxels (all the step at the centre reads)
        K0 = gray_parameters(wl["phi"], wl["ptype"], cls, wl["tables"], p.c_max, p.c_min)[0]
        near = set()
        for _, flat in picks:
            zc, yc, xc = np.unravel_index(flat, cls.shape)
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        v = tuple(np.array([zc + dz, yc + dy, xc + dx]) % cls.shape[0])
                        if cls[v] == W.GRAY:
                            near.add(int(np.ravel_multi_index(v, cls.shape)))
        Kinv = inverse_permeability(wl["phi"], cls, wl["ptype"], K0, wl["tables"], p.sigma_s,
                                    p.smooth_radius, p.eps_g, p.eps_H, p.delta_tie,
                                    voxels=sorted(near))[0]
    worst, skipped = {}, 0
    for name, flat in picks:
        c = np.unravel_index(flat, cls.shape)
        o = Oracle(p)
        o.set_geometry(_crop(cls, c, 0), _crop(wl["phi"], c, 0), _crop(wl["ptype"], c, 0),
                       wl["tables"])
        if Kinv is not None:
            o.Kinv = _crop(Kinv, c, 1)
        o.set_state(dict(f=_decoded_crop(s0, prec, c, cls) * w,
                         r=_crop(s0["r"], c, 1).astype(np.float64),
                         side=_crop(s0["side"], c, 0).astype(bool), step=0,
                         Q_acc=np.zeros(2), Q_last=np.zeros(2)))
        S0 = float(o.evaluate()["S"][R, R, R])
        if min(abs(S0 - 0.5 - hy), abs(S0 - 0.5 + hy)) < 1e-4:
            skipped += 1  # a residual-event switch this close to its threshold may go either way
            continue
        o.step(1)
        got = _decoded_crop(s1, prec, c, cls)[:, :, R, R, R]
        ref = o.f[:, :, R, R, R] / WQ[None, :]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst[name] = max(worst.get(name, 0.0), err)
        assert err < tol, (name, c, err)
        r_got = s1["r"][(slice(None),) + c].astype(np.float64)
        assert np.abs(r_got - o.r[:, R, R, R]).max() < tol, (name, c, r_got, o.r[:, R, R, R])
        assert bool(s1["side"][c]) == bool(o.side[R, R, R]), (name, c)
    print(prec, "worst relative error per category", {k: f"{v:.2e}" for k, v in worst.items()},
          "skipped near a threshold:", skipped)
    assert len(worst) == ncat
    # a property of the whole grid: mass per component (mobile + residual) is
    # carried through the step up to rounding
    for k in ("mass_w", "mass_o")[:int(wl["params"].ncomp)]:
        assert abs(d1[k] - d0[k]) / d0[k] < 1e-6, (k, d0[k], d1[k])


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f16", 1e-3), ("bf16", 4e-3)])
def test_rock256_sampled_step_matches_oracle(prec, tol):
    _sampled_step(W.multiscale_rock(n=256, precision=prec), prec, tol)


def test_fiber192_sampled_step_matches_oracle():
    _sampled_step(W.fiber_bundles(n=192, precision="f32"), "f32", 1e-5)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_rock256_full_run_stays_finite(prec):
    """The benchmark's workload over its 2000 steps: no non-finite value (the
    step checks every diag_every steps), non-negative densities, each
    component's mass (mobile + residual) carried up to rounding, speeds below
    the lattice's 0.1 and a saturation inside (0, 1).  (The net water flux
    through the outlet plane is not signed: over these 2000 steps the
    capillary redistribution of the inlet buffer outweighs the body force.)"""
    import paper_2512_21696_amd as L
    wl = W.multiscale_rock(n=256, precision=prec)
    announce(f"multiscale_rock 256^3 {prec}: 2000 steps in blocks of 250")
    lb = L.lbm_create(wl["params"])
    lb.set_geometry(wl["cls"], wl["phi"], wl["ptype"], wl["tables"])
    lb.init_fluid(wl["rho_w"], wl["rho_o"])
    d0 = lb.get_diagnostics()
    for _ in range(8):
        lb.step(250)
        d = lb.get_diagnostics()
        print(prec, "step", d["step"], "max_u", d["max_u"], "Sw", d["sw"], flush=True)
        assert d["nonfinite"] == 0
        assert d["max_u"] < 0.1
    f = lb.get_fields(names=("rho_w", "rho_o"))
    lb.destroy()
    fluid = wl["cls"] != W.SOLID
    assert f["rho_w"][fluid].min() >= 0.0 and f["rho_o"][fluid].min() >= 0.0
    mtol = 1e-10 if prec == "f64" else 1e-4
    for k in ("mass_w", "mass_o"):
        assert abs(d[k] - d0[k]) / d0[k] < mtol, (k, d0[k], d[k])
    assert 0.0 < d["sw"] < 1.0
