"""The no-allocation variant of the batched permeability library against the
allocating one: two calls in a row on one GPU, the second with fewer and
smaller domains than the first (its scratch keeps the first call's
contents), and a batch larger than the scratch."""
import numpy as np
import pytest

import workloads as W
from gpu_common import announce

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate(sizes):
        out.append(W.sphere_pack((n, n + 2, n + 1), float(rng.uniform(0.3, 0.45)),
                                 seed * 100 + k, rmin=2.0, rmax=4.0))
    return out


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_static_scratch_matches_allocating_call(precision):
    import paper_2512_21696_amd as L
    for call, (sizes, seed) in enumerate((((16, 20, 24, 12, 18), 5), ((12, 10), 6))):
        announce(f"no-allocation permeability, call {call + 1}, {precision}, boxes {sizes}")
        doms = _batch(sizes, seed)
        kw = dict(tau=0.9, g=1e-5, axis=call % 3, precision=precision, max_steps=300,
                  check_every=50, tol=0.0, want_u=True, side_walls=call == 1)
        ref = L.rev_permeability(doms, **kw)
        got = L.rev_permeability(doms, static=True, **kw)
        for r, s in zip(ref, got):
            for k in ("K", "phi", "u_mean", "steps", "converged"):
                assert r[k] == s[k], (call, k, r[k], s[k])
            assert np.array_equal(r["u"], s["u"])
            assert r["K"] > 0 and s["step_ms"] == 0.0


def test_static_scratch_rejects_a_batch_beyond_its_size():
    import paper_2512_21696_amd as L
    announce("no-allocation permeability: a batch beyond the scratch is refused")
    big = [np.zeros((96, 96, 96), np.uint8) for _ in range(2)]
    with pytest.raises(L.LbmError) as ei:
        L.rev_permeability(big, precision="f32", max_steps=10, static=True)
    assert ei.value.code == L.LBM_E_UNSUPPORTED
    assert "static scratch" in str(ei.value)
