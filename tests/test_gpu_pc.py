"""The capillary-pressure sweep (lbm_rev_pc_sweep) through the C ABI against
the oracle's protocol (oracle/pc_sweep.py), on four uneven sphere packs, and a
five-level sweep run to its steady states on the GPU.

Parity: every level runs a fixed number of steps (check_every = max_steps,
tol = 0), so both sides take the same steps; the sample's water saturation
after each level must agree to 1e-12 in fp64 (a mean of O(1) values after
the same arithmetic as the parity tests' fields) and to 1e-5 in fp32 (the
fp32 rounding of the fields, 1e-4 of their scale after 100 steps in
test_gpu_parity, averaged over the sample), and the capillary pressure of
each level, a function of the reservoir densities alone, to 1e-14."""
import numpy as np
import pytest

import workloads as W
from oracle.pc_sweep import pc_sweep
from gpu_common import announce

pytestmark = pytest.mark.gpu

SHAPES = [(6, 7, 9), (7, 6, 6), (6, 8, 7), (8, 6, 10)]  # [z][y][x], uneven on purpose
LEVELS = (1.03, 1.10, 1.18)


def _domains():
    return [W.sphere_pack(s, 0.45, 6100 + k, rmin=1.2, rmax=2.0) for k, s in enumerate(SHAPES)]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sweep_matches_oracle_on_uneven_domains(prec, tol):
    import paper_2512_21696_amd as L
    su = W.pc_sweep_setup(levels=LEVELS, precision=prec)
    doms = _domains()
    kw = dict(buffer_in=4, membrane=2, buffer_out=2, side_walls=True,
              membrane_phi=su["membrane_phi"], check_every=40, max_steps=40, tol=0.0)
    announce(f"Pc sweep {prec}: 4 sphere packs {SHAPES}, {len(LEVELS)} levels x 40 steps")
    got = L.rev_pc_sweep(doms, su["model"], su["membrane_table"], su["rho_nw_in"], **kw)
    su64 = W.pc_sweep_setup(levels=LEVELS)
    worst = 0.0
    for k, d in enumerate(doms):
        ref = pc_sweep(d, su64["model"], su64["membrane_table"], su64["rho_nw_in"], **kw)
        assert got[k]["steps"] == ref["steps"]
        assert np.abs(np.array(got[k]["pc"]) - ref["pc"]).max() < 1e-14
        err = np.abs(np.array(got[k]["sw"]) - ref["sw"]).max()
        worst = max(worst, err)
        assert err < tol, (k, got[k]["sw"], ref["sw"])
    print(prec, "worst Sw difference", worst)


def test_five_level_drainage_reaches_steady_states():
    """Two 24^3-class sphere packs, the five levels of pc_sweep_setup, each run
    until Sw changes by at most 1e-3 over 500 steps, 20000 steps at most: the
    capillary pressure rises and the saturation falls level by level (a
    drainage curve) and stays inside [0, 1], and each domain settles at four
    levels of five at least.  (At the level that crosses a pack's percolation
    threshold the front creeps through one throat after another for tens of
    thousands of steps; measured: one such level in the second pack.)"""
    import paper_2512_21696_amd as L
    su = W.pc_sweep_setup(precision="f32")
    doms = [W.sphere_pack((24, 24, 24), 0.40, 6201), W.sphere_pack((20, 26, 30), 0.35, 6202)]
    announce("Pc sweep f32: two sphere packs, five levels to steady state")
    out = L.rev_pc_sweep(doms, su["model"], su["membrane_table"], su["rho_nw_in"],
                         buffer_in=14, membrane=2, buffer_out=2, side_walls=True,
                         membrane_phi=su["membrane_phi"], check_every=500, max_steps=20000,
                         tol=1e-3)
    for r in out:
        print("pc", np.round(r["pc"], 4), "sw", np.round(r["sw"], 4), "steps", r["steps"])
        assert sum(r["converged"]) >= 4, r
        assert np.all(np.diff(r["pc"]) > 0)
        assert np.all(np.diff(r["sw"]) <= 1e-3), r["sw"]
        assert 0.0 <= min(r["sw"]) and max(r["sw"]) <= 1.0
        assert r["sw"][-1] < r["sw"][0]
