"""Per-gray-voxel constitutive setup, once per geometry (fp64, plain numpy).

* Table lookup: every library curve (K0(phi), Pc(S), Krw(S), Kro(S); paper
  Sec. I workflow step iii and Appendix, Fig. 19) is held as 1025 uniform
  samples on [0, 1] and evaluated by linear interpolation:
  t = v * 1024, k = min(floor(t), 1023), value = tab[k] + (t - k)(tab[k+1] - tab[k]).
* K0(x) = lerp(K0_tab[type], phi(x)).
* Leverett-J scaling (Eq. (5)): equal J and equal sigma*cos(theta) give
  Pc(phi) = Pc_ref * sqrt(K0_ref/phi_ref) / sqrt(K0(phi)/phi); the per-voxel
  factor s_J = sqrt((K0_ref/phi_ref) / (K0/phi)) multiplies the tabulated Pc.
* Residual amounts (Sec. II, residual-component model, Fig. 6): the residual
  water saturation theta_w is where the J-scaled Pc-S curve crosses
  Pc^{ref,max} = c_max * Pc_PM; the residual oil saturation theta_o is one
  minus the saturation where it crosses Pc^{ref,min} = c_min * Pc_PM.  The
  curve is the piecewise-linear interpolant, assumed non-increasing; the
  smallest crossing saturation is taken; no crossing on [0, 1] gives 0.
"""
import numpy as np


def lerp_table(tab: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Linear interpolation of a 1025-sample table at v in [0, 1]."""
    tab = np.asarray(tab, np.float64)
    n = tab.shape[-1] - 1
    t = np.asarray(v, np.float64) * n
    k = np.minimum(np.floor(t), n - 1).astype(np.int64)
    k = np.maximum(k, 0)
    fr = t - k
    lo = np.take(tab, k)
    hi = np.take(tab, k + 1)
    return lo + fr * (hi - lo)


def crossing(y: np.ndarray, target: float) -> float:
    """Smallest S in [0, 1] where the piecewise-linear, non-increasing curve with
    samples y_k at S = k/1024 equals target; None when it never does."""
    n = len(y) - 1
    if y[0] < target or y[n] > target:
        return None
    k = int(np.argmax(y <= target))  # first sample at or below target
    if k == 0:
        return 0.0
    a, b = y[k - 1], y[k]
    return ((k - 1) + (a - target) / (a - b)) / n


def gray_parameters(phi, ptype, cls, tables, c_max, c_min, GRAY=2):
    """Per-voxel K0, s_J, theta_w, theta_o (zero outside gray voxels)."""
    shape = phi.shape
    K0 = np.zeros(shape)
    sJ = np.zeros(shape)
    thw = np.zeros(shape)
    tho = np.zeros(shape)
    gray = cls == GRAY
    for t, tab in enumerate(tables):
        sel = gray & (ptype == t)
        if not sel.any():
            continue
        ph = phi[sel]
        k0 = lerp_table(tab["K0"], ph)
        k0ref = float(lerp_table(tab["K0"], np.array([tab["phi_ref"]]))[0])
        sj = np.sqrt((k0ref / tab["phi_ref"]) / (k0 / ph))
        K0[sel] = k0
        sJ[sel] = sj
        pc = np.asarray(tab["Pc"], np.float64)
        tw = np.empty(ph.shape)
        to = np.empty(ph.shape)
        for j, s in enumerate(sj):
            y = s * pc
            cw = crossing(y, c_max * tab["Pc_PM"])
            co = crossing(y, c_min * tab["Pc_PM"])
            tw[j] = 0.0 if cw is None else cw
            to[j] = 0.0 if co is None else 1.0 - co
        thw[sel] = tw
        tho[sel] = to
    return K0, sJ, thw, tho
