"""Writes coexistence.json: the bulk densities of the flat-interface
equilibrium of the two-component pseudo-potential model at G = 3 (tau = 1),
obtained by running the CPU oracle to steady state on a 64-voxel periodic
column with two flat interfaces.  The ratio minority/majority fixes the
saturation normalisation constants (s_min, s_max), the oil wall potential and
phi_avg of the workloads.  Calls only the oracle."""
import json, os, sys
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import Oracle  # noqa: E402


class P:  # parameter record for the oracle
    pass


def run(G=3.0, n=64, steps=8000, m0=0.003):
    p = P()
    p.nx, p.ny, p.nz, p.ncomp = n, 1, 1, 2
    p.tau, p.G, p.g = (1.0, 1.0), G, ((0.0,) * 3, (0.0,) * 3)
    p.kappa, p.csf_region, p.phi_max, p.phi_avg = 0.0, "gray", 1.0, 0.5
    p.m_minor, p.s_min, p.s_max = m0, m0 / (1 + m0), 1 / (1 + m0)
    p.wall_dpsi, p.kr_min, p.c_max, p.c_min, p.hyst = (0.1, -0.1), 1e-4, 3.5, 0.575, 0.05
    p.eps_n, p.tensor, p.collision, p.outlet_x = 1e-12, False, "regularized", n - 1
    o = Oracle(p)
    shape = (1, 1, n)
    o.set_geometry(np.zeros(shape, np.uint8), np.ones(shape), np.zeros(shape, np.uint8), [])
    x = np.arange(n, dtype=float).reshape(shape)
    prof = 0.5 * (np.tanh((x - n / 4) / 1.5) - np.tanh((x - 3 * n / 4) / 1.5))
    o.init_fluid(m0 + (1 - m0) * prof, m0 + (1 - m0) * (1 - prof))
    o.step(steps)
    f = o.fields()
    M = float(f["rho_w"][0, 0, n // 2])
    m = float(f["rho_w"][0, 0, 0])
    return dict(G=G, tau=1.0, n=n, steps=steps, majority=M, minority=m, ratio=m / M,
                max_u=float(np.abs(f["ux"]).max()),
                rho_w=[float(v) for v in f["rho_w"][0, 0]],
                rho_o=[float(v) for v in f["rho_o"][0, 0]])


if __name__ == "__main__":
    out = run()
    with open(os.path.join(HERE, "coexistence.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print({k: v for k, v in out.items() if not k.startswith("rho")})
