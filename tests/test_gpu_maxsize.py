"""The largest grid the library accepts, through the C ABI: 384 x 384 x 383
voxels (56.5 M) in fp32 with two components, where 2*19*N is within 0.1 % of
2^31 and the last population array of each component ends within 0.1 % of
the 4 GiB that 32-bit byte offsets address.  The geometry is the multiscale
rock of the benchmark's recipe at 128^3, repeated periodically (the repeat is
cut at z = 383, so the z wrap joins two unrelated faces).  After two steps one
more step is compared voxel by voxel against the fp64 oracle on sampled
voxels: the last planes, rows and columns of the arrays (the largest
offsets), the periodic wrap and seeded interior voxels, each on a periodic
9^3 crop around it (the update of one voxel depends on the post-streaming
populations within three voxels; radius 4 keeps one spare layer).

Tolerance as for the 256^3 rock in fp32: one step from the same state
differs from the fp64 oracle only by fp32 rounding of O(1) operands, 1e-5 of
each voxel's largest f_i / w_i."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle, W as WQ
from gpu_common import announce

pytestmark = pytest.mark.gpu

SHAPE = (383, 384, 384)  # z, y, x
R = 4


def _tile(a, lead):
    reps = (1,) * lead + (3, 3, 3)
    t = np.tile(a, reps)
    return np.ascontiguousarray(t[(slice(None),) * lead + tuple(slice(0, n) for n in SHAPE)])


def _crop(a, c, lead):
    idx = [np.arange(ci - R, ci + R + 1) % n for ci, n in zip(c, SHAPE)]
    return a[(slice(None),) * lead + np.ix_(*idx)]


def test_largest_grid_sampled_step_matches_oracle():
    import paper_2512_21696_amd as L
    base = W.multiscale_rock(n=128, precision="f32")
    cls, phi, ptype = _tile(base["cls"], 0), _tile(base["phi"], 0), _tile(base["ptype"], 0)
    rho_w, rho_o = _tile(base["rho_w"], 0), _tile(base["rho_o"], 0)
    nz, ny, nx = SHAPE
    p = W.Params(**{**base["params"].as_dict(), "nx": nx, "ny": ny, "nz": nz})
    announce(f"largest grid {nx}x{ny}x{nz} ({cls.size} voxels) f32: 2 steps, state, one step, state")
    lb = L.lbm_create(p)
    try:
        lb.set_geometry(cls, phi, ptype, base["tables"])
        lb.init_fluid(rho_w, rho_o)
        lb.step(2)
        s0 = lb.state_arrays(lb.get_state())
        lb.step(1)
        s1 = lb.state_arrays(lb.get_state())
        d1 = lb.get_diagnostics()
    finally:
        lb.destroy()
    assert not d1["nonfinite"]
    rng = np.random.default_rng(11)
    fluid = cls != W.SOLID
    picks = []
    for z, y, x in ((nz - 1, ny - 1, nx - 1), (nz - 1, ny - 1, None), (nz - 1, None, None),
                    (nz - 2, None, None), (0, None, None), (None, ny - 1, None),
                    (None, None, nx - 1), (None, None, 0), (None, None, None),
                    (None, None, None), (None, None, None), (None, None, None)):
        for _ in range(1000):  # a fluid voxel with the fixed coordinates
            c = tuple(int(rng.integers(n)) if v is None else v for v, n in zip((z, y, x), SHAPE))
            if fluid[c]:
                picks.append(c)
                break
    assert len(picks) >= 10
    q = W.Params(**{**p.as_dict(), "nx": 2 * R + 1, "ny": 2 * R + 1, "nz": 2 * R + 1,
                    "precision": "f64", "outlet_x": 0})
    worst, skipped = 0.0, 0
    for c in picks:
        o = Oracle(q)
        o.set_geometry(_crop(cls, c, 0), _crop(phi, c, 0), _crop(ptype, c, 0), base["tables"])
        o.set_state(dict(f=_crop(s0["f"], c, 2).astype(np.float64),
                         r=_crop(s0["r"], c, 1).astype(np.float64),
                         side=_crop(s0["side"], c, 0).astype(bool), step=0,
                         Q_acc=np.zeros(2), Q_last=np.zeros(2)))
        S0 = float(o.evaluate()["S"][R, R, R])
        if min(abs(S0 - 0.5 - q.hyst), abs(S0 - 0.5 + q.hyst)) < 1e-4:
            skipped += 1  # a residual-event switch this close to its threshold may go either way
            continue
        o.step(1)
        got = s1["f"][(slice(None), slice(None)) + c].astype(np.float64) / WQ[None, :]
        ref = o.f[:, :, R, R, R] / WQ[None, :]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err < 1e-5, (c, err)
        r_got = s1["r"][(slice(None),) + c].astype(np.float64)
        assert np.abs(r_got - o.r[:, R, R, R]).max() < 1e-5, (c, r_got, o.r[:, R, R, R])
        assert bool(s1["side"][c]) == bool(o.side[R, R, R]), c
    print(f"largest grid: {len(picks)} voxels, worst relative error {worst:.2e}, "
          f"skipped near a threshold: {skipped}")
    assert skipped <= 2
