"""The fused step's own sum of the next level's densities (two components,
fp32 storage).  Each density must equal the sum of the voxel's next pulls:
the run that takes every level's densities from the step's push is compared
with the same run whose densities come from the density pass on every step
(taking a checkpoint makes the next step recompute them).  The two differ
only in the order of the additions, so they agree to rounding; a link
missing from the push (a tile, chunk or wrap edge) would put an error of
w_i rho (>= 1/36) into the pseudo-potential and CSF stencils at once.
16-bit storage keeps the density pass; there the same comparison sets the
pass's reference sums written by the step against the ones it gathers
itself after a checkpoint.

The grid, 72 x 10 x 12, has two x tiles of 64 columns (the second ragged),
three y tiles of 4 rows (the last ragged), three z chunks of 4 planes, the
periodic wrap on every axis, and random pore, solid and gray voxels with
the CSF control everywhere."""
import numpy as np
import pytest

import workloads as W
from gpu_common import announce

pytestmark = pytest.mark.gpu

STEPS = 30
# fp32: a few ulps of O(1) densities grown over the run; 16-bit storage: a
# different last bit of a reference density can move a stored offset by one
# unit in its last place, 2^-11 (fp16) or 2^-8 (bf16) of |h| <= 1, per step,
# adding like a random walk (2 * 2^-p * sqrt(n), as in the 16-bit tests)
TOL = {"f32": 1e-5, "f16": 2 * 2.0 ** -11 * np.sqrt(STEPS), "bf16": 2 * 2.0 ** -8 * np.sqrt(STEPS)}
# total mass: fp32 arithmetic carries it to rounding; 16-bit storage changes it
# by the roundings of the stored offsets, which the two runs take apart
# (measured 8e-6 for bf16 over the 30 steps)
MTOL = {"f32": 1e-6, "f16": 2e-5, "bf16": 1.6e-4}


def _case(prec):
    rng = np.random.default_rng(17)
    shape = (12, 10, 72)
    p = W.Params(nx=72, ny=10, nz=12, ncomp=2, precision=prec, tau=(1.0, 1.5), G=3.0,
                 kappa=-0.02, csf_region="all", g=((1e-4, 0, 0), (0, -5e-5, 0))).filled()
    cls = rng.choice([0, 0, 0, 1, 2], size=shape).astype(np.uint8)
    phi = np.where(cls == 2, rng.uniform(0.1, 0.4, shape), 1.0)
    pt = np.where(cls == 2, rng.integers(0, 2, shape), 0).astype(np.uint8)
    tabs = W.multiscale_rock(n=8, precision="f64")["tables"][:2]
    z, y, x = np.meshgrid(np.arange(12), np.arange(10), np.arange(72), indexing="ij")
    r1 = np.sqrt((x - 10) ** 2 + (y - 5) ** 2 + (z - 6) ** 2)
    r2 = np.sqrt((x - 63) ** 2 + (y - 1) ** 2 + (z - 11) ** 2)  # across the x tile edge and wraps
    prof = 0.5 * (1 - np.tanh((r1 - 4.0) / 1.5)) + 0.5 * (1 - np.tanh((r2 - 3.5) / 1.5))
    rw = p.m_minor + (1 - p.m_minor) * np.clip(prof, 0, 1)
    return p, cls, phi, pt, tabs, rw, 1.0 + p.m_minor - rw


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_pushed_densities_match_the_density_pass(prec):
    import paper_2512_21696_amd as L
    p, cls, phi, pt, tabs, rw, ro = _case(prec)
    runs = []
    for per_step_checkpoint in (False, True):
        announce(f"72x10x12 two components {prec}: {STEPS} steps, "
                 f"{'density pass every step' if per_step_checkpoint else 'pushed densities'}")
        lb = L.lbm_create(p)
        lb.set_geometry(cls, phi, pt, tabs)
        lb.init_fluid(rw, ro)
        for _ in range(STEPS):
            lb.step(1)
            if per_step_checkpoint:
                lb.get_state()
        f = lb.get_fields(names=("rho_w", "rho_o", "ux", "uy", "uz"))
        d = lb.get_diagnostics()
        lb.destroy()
        assert d["nonfinite"] == 0
        runs.append((f, d))
    (fa, da), (fb, db) = runs
    fluid = cls != W.SOLID
    worst = {}
    for k in ("rho_w", "rho_o", "ux", "uy", "uz"):
        scale = 1.0 if k.startswith("rho") else max(np.abs(fb[k][fluid]).max(), 1e-3)
        worst[k] = float(np.abs(fa[k][fluid] - fb[k][fluid]).max()) / scale
    print(prec, "pushed vs density pass", {k: f"{v:.2e}" for k, v in worst.items()})
    assert max(worst.values()) < TOL[prec], worst
    for k in ("mass_w", "mass_o"):
        assert abs(da[k] - db[k]) / db[k] < MTOL[prec], (k, da[k], db[k])
    # the two runs took different summation orders, so both paths did run
    assert any(not np.array_equal(fa[k], fb[k]) for k in fa), "no difference: one path only?"
