"""Writes kappa.json: the CSF coefficients kappa (Eq. (4)) that scale the
surface tension of the two-component pseudo-potential model at G = 3 (tau = 1)
to 0.5 and 2 times its value at kappa = 0, measured as in Sec. III.A with a
static droplet and Laplace's law.

The droplet is quasi-2D (nz = 1), R = 7 on a 32 x 32 periodic box, CSF applied
everywhere, 1200 steps; sigma = dP R (2D Laplace law) with
p = cs^2 (rho_w + rho_o) + cs^2 G rho_w rho_o, dP = p(centre) - p(corner).  A
secant search on kappa brings sigma / sigma_0 to the target within 0.5 %.
Calls only the oracle; the bulk minority density comes from coexistence.json
(written by make_coexistence.py, also from the oracle)."""
import json, os, sys
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import Oracle, CS2  # noqa: E402

N, R, STEPS, G = 32, 7.0, 1200, 3.0


class P:  # parameter record for the oracle
    pass


def params(kappa, m):
    p = P()
    p.nx, p.ny, p.nz, p.ncomp = N, N, 1, 2
    p.tau, p.G, p.g = (1.0, 1.0), G, ((0.0,) * 3, (0.0,) * 3)
    p.kappa, p.csf_region, p.phi_max, p.phi_avg = kappa, "all", 1.0, 0.5 * (1 + m)
    p.m_minor, p.s_min, p.s_max = m, m / (1 + m), 1 / (1 + m)
    p.wall_dpsi, p.kr_min, p.c_max, p.c_min, p.hyst = (0.1, -0.1), 1e-4, 3.5, 0.575, 0.05
    p.eps_n, p.tensor, p.collision, p.outlet_x = 1e-12, False, "regularized", N - 1
    return p


def droplet(kappa, m):
    """Returns (sigma, max |u|, 10-90 % interface width) after STEPS steps."""
    o = Oracle(params(kappa, m))
    shape = (1, N, N)
    o.set_geometry(np.zeros(shape, np.uint8), np.ones(shape), np.zeros(shape, np.uint8), [])
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    r = np.sqrt((x - (N - 1) / 2) ** 2 + (y - (N - 1) / 2) ** 2).reshape(shape)
    prof = 0.5 * (1 - np.tanh((r - R) / 1.5))
    o.init_fluid(m + (1 - m) * prof, m + (1 - m) * (1 - prof))
    o.step(STEPS)
    ev = o.evaluate()
    rw, ro = ev["rho"][0][0], ev["rho"][1][0]
    pr = CS2 * (rw + ro) + CS2 * G * rw * ro
    c = N // 2
    dp = pr[c, c] - pr[0, 0]
    umax = float(np.sqrt(ev["u"][0] ** 2 + ev["u"][1] ** 2).max())
    line = rw[c, c:]
    lo, hi = line.min(), line.max()
    xs = np.arange(len(line), dtype=float)
    a = np.interp(lo + 0.9 * (hi - lo), line[::-1], xs[::-1])
    b = np.interp(lo + 0.1 * (hi - lo), line[::-1], xs[::-1])
    return float(dp * R), umax, float(b - a)


def secant(target, sigma0, m, k0, k1, log):
    f0 = droplet(k0, m)[0] / sigma0 - target
    f1 = droplet(k1, m)[0] / sigma0 - target
    for _ in range(12):
        k2 = k1 - f1 * (k1 - k0) / (f1 - f0)
        res = droplet(k2, m)
        f2 = res[0] / sigma0 - target
        log.append((k2, res[0] / sigma0, res[1], res[2]))
        print(f"  kappa {k2:+.5f}: sigma/sigma0 = {res[0] / sigma0:.4f}", flush=True)
        if abs(f2) < 0.005 * target:
            return k2, res
        k0, f0, k1, f1 = k1, f1, k2, f2
    raise RuntimeError("secant search did not converge")


def main():
    with open(os.path.join(HERE, "coexistence.json")) as fh:
        m = json.load(fh)["ratio"]
    s0, u0, w0 = droplet(0.0, m)
    print(f"sigma_0 = {s0:.6f}, max|u| = {u0:.3e}, width = {w0:.3f}", flush=True)
    out = {"note": __doc__.strip(), "N": N, "R": R, "steps": STEPS, "G": G, "m_minor": m,
           "sigma0": s0, "umax0": u0, "width0": w0, "targets": {}}
    for target, k0, k1 in ((0.5, -0.05, -0.1), (2.0, 0.05, 0.1)):
        log = []
        print(f"target sigma/sigma0 = {target}", flush=True)
        k, (sg, um, wd) = secant(target, s0, m, k0, k1, log)
        out["targets"][str(target)] = {"kappa": k, "sigma_ratio": sg / s0, "umax": um,
                                       "width": wd, "search": log}
    with open(os.path.join(HERE, "kappa.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({t: v["kappa"] for t, v in out["targets"].items()}))


if __name__ == "__main__":
    main()
