// Host-only argument validation of the C ABI (no device call).  Kept in its
// own translation unit so that it can be built and tested without a GPU.
#include "../../include/lbm.h"
#include "lbm_validate.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>

namespace {
// Bulk minority/majority density ratio of the flat-interface equilibrium at
// G = 3 (two components, tau = 1): the default saturation normalisation.
constexpr double kMinorityG3 = 0.0029912221254390597;

int fail(char *msg, size_t len, int code, const char *fmt, double a = 0, double b = 0) {
  if (msg && len) std::snprintf(msg, len, fmt, a, b);
  return code;
}
}  // namespace

extern "C" void lbm_params_default(lbm_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 32;
  p->ncomp = 2;
  p->precision = LBM_PREC_F64;
  p->collision = LBM_COLL_REGULARIZED;
  p->tau[0] = p->tau[1] = 1.0;
  p->G = 3.0;
  p->kappa = 0.0;
  p->csf_region = LBM_CSF_GRAY;
  p->tensor = 0;
  const double m = kMinorityG3;
  p->m_minor = m;
  p->s_min = m / (1.0 + m);
  p->s_max = 1.0 / (1.0 + m);
  p->phi_max = 1.0;
  p->phi_avg = 0.5 * (1.0 + m);
  p->wall_dpsi[0] = 0.1;
  p->wall_dpsi[1] = -0.1;
  p->kr_min = 1e-4;
  p->c_max = 3.5;
  p->c_min = 0.575;
  p->hyst = 0.05;
  p->eps_n = 1e-12;
  p->sigma_s = 1.5;
  p->smooth_radius = 5;
  p->outlet_x = p->nx - 1;
  p->eps_g = 1e-6;
  p->eps_H = 1e-6;
  p->delta_tie = 0.05;
  p->diag_every = 0;
  p->track_flux = 1;
  p->bc_x = LBM_BC_PERIODIC;
  p->layout = LBM_LAYOUT_AUTO;
  p->rho_in[0] = p->rho_out[0] = 1.0;
  p->rho_in[1] = p->rho_out[1] = 0.0;
}

extern "C" int lbm_validate_params(const lbm_params *p, char *msg, size_t len) {
  if (!p) return fail(msg, len, LBM_E_INVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(msg, len, LBM_E_INVAL, "grid sizes must be >= 1");
  const double N = (double)p->nx * p->ny * p->nz;
  if (N * 2 * 19 >= 2147483647.0)
    return fail(msg, len, LBM_E_UNSUPPORTED, "grid too large: 2*19*N must stay below 2^31");
  if (p->ncomp != 1 && p->ncomp != 2) return fail(msg, len, LBM_E_INVAL, "ncomp must be 1 or 2");
  if (p->precision != LBM_PREC_F64 && p->precision != LBM_PREC_F32 &&
      p->precision != LBM_PREC_F16 && p->precision != LBM_PREC_BF16)
    return fail(msg, len, LBM_E_UNSUPPORTED,
                "precision must be LBM_PREC_F64, LBM_PREC_F32, LBM_PREC_F16 or LBM_PREC_BF16");
  // the arithmetic-type arrays (and, in fp64/fp32 runs, the populations) are
  // addressed with 32-bit byte offsets per component
  if (N * 19 * (p->precision == LBM_PREC_F64 ? 8 : 4) >= 4294967295.0)
    return fail(msg, len, LBM_E_UNSUPPORTED,
                "grid too large: one component's populations must stay below 4 GiB");
  if (p->collision != LBM_COLL_REGULARIZED && p->collision != LBM_COLL_BGK)
    return fail(msg, len, LBM_E_INVAL, "unknown collision model");
  for (int a = 0; a < p->ncomp; ++a)
    if (!(p->tau[a] > 0.5) || !std::isfinite(p->tau[a]))
      return fail(msg, len, LBM_E_INVAL, "tau must be finite and > 1/2 (got %g)", p->tau[a]);
  if (!std::isfinite(p->G) || !std::isfinite(p->kappa))
    return fail(msg, len, LBM_E_INVAL, "G and kappa must be finite");
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(p->g[a][d])) return fail(msg, len, LBM_E_INVAL, "body force not finite");
  if (p->csf_region != LBM_CSF_GRAY && p->csf_region != LBM_CSF_ALL)
    return fail(msg, len, LBM_E_INVAL, "unknown CSF region");
  if (p->ncomp == 2) {
    if (!(p->s_max > p->s_min)) return fail(msg, len, LBM_E_INVAL, "s_max must exceed s_min");
    if (!(p->phi_max > 0) || !(p->phi_avg > 0))
      return fail(msg, len, LBM_E_INVAL, "phi_max and phi_avg must be > 0");
    if (!(p->m_minor >= 0)) return fail(msg, len, LBM_E_INVAL, "m_minor must be >= 0");
  }
  if (!(p->kr_min > 0)) return fail(msg, len, LBM_E_INVAL, "kr_min must be > 0");
  if (!(p->hyst >= 0) || !(p->hyst < 0.5))
    return fail(msg, len, LBM_E_INVAL, "hysteresis must be in [0, 1/2)");
  if (!(p->eps_n >= 0)) return fail(msg, len, LBM_E_INVAL, "eps_n must be >= 0");
  if (p->outlet_x < 0 || p->outlet_x >= p->nx)
    return fail(msg, len, LBM_E_INVAL, "outlet_x out of range");
  if (p->tensor) {
    if (!(p->sigma_s > 0)) return fail(msg, len, LBM_E_INVAL, "sigma_s must be > 0");
    if (p->smooth_radius < 0 || p->smooth_radius > 8)
      return fail(msg, len, LBM_E_INVAL, "smooth_radius must be in [0, 8]");
    if (!(p->eps_g >= 0) || !(p->eps_H >= 0) || !(p->delta_tie >= 0))
      return fail(msg, len, LBM_E_INVAL, "tensor thresholds must be >= 0");
  }
  if (p->diag_every < 0) return fail(msg, len, LBM_E_INVAL, "diag_every must be >= 0");
  if (p->bc_x != LBM_BC_PERIODIC && p->bc_x != LBM_BC_PRESSURE && p->bc_x != LBM_BC_DENSITY)
    return fail(msg, len, LBM_E_INVAL, "unknown x boundary");
  if (p->bc_x == LBM_BC_DENSITY && p->nx < 3)
    return fail(msg, len, LBM_E_INVAL, "density faces need nx >= 3");
  if (p->layout != LBM_LAYOUT_AUTO && p->layout != LBM_LAYOUT_DENSE)
    return fail(msg, len, LBM_E_INVAL, "unknown population layout");
  if (p->bc_x != LBM_BC_PERIODIC) {
    if (p->outlet_x > p->nx - 2)
      return fail(msg, len, LBM_E_INVAL, "with open x faces outlet_x must be <= nx - 2");
    if (p->kappa != 0.0 && p->csf_region != LBM_CSF_GRAY)
      return fail(msg, len, LBM_E_INVAL, "open x faces need the CSF region in gray voxels");
    for (int a = 0; a < 2; ++a)
      if (!(p->rho_in[a] >= 0) || !(p->rho_out[a] >= 0) || !std::isfinite(p->rho_in[a]) ||
          !std::isfinite(p->rho_out[a]))
        return fail(msg, len, LBM_E_INVAL, "reservoir densities must be finite and >= 0");
  }
  if ((p->alloc == nullptr) != (p->free == nullptr))
    return fail(msg, len, LBM_E_INVAL, "alloc and free hooks must be given together");
  return LBM_OK;
}

namespace lbm {

int validate_tables(const lbm_pore_table *t, int ntab, char *msg, size_t len) {
  if (ntab < 0 || ntab > LBM_MAX_TYPES) return fail(msg, len, LBM_E_INVAL, "ntab out of range");
  if (ntab > 0 && !t) return fail(msg, len, LBM_E_INVAL, "tables pointer is NULL");
  for (int k = 0; k < ntab; ++k) {
    const lbm_pore_table &tb = t[k];
    if (!(tb.phi_ref > 0 && tb.phi_ref < 1))
      return fail(msg, len, LBM_E_INVAL, "table %g: phi_ref must be in (0,1)", k);
    if (!(tb.Pc_PM > 0) || !std::isfinite(tb.Pc_PM))
      return fail(msg, len, LBM_E_INVAL, "table %g: Pc_PM must be > 0", k);
    for (int d = 0; d < 3; ++d)
      if (!(tb.kd[d] > 0) || !std::isfinite(tb.kd[d]))
        return fail(msg, len, LBM_E_INVAL, "table %g: kd must be > 0", k);
    for (int i = 0; i < LBM_TABLE_N; ++i) {
      if (!std::isfinite(tb.K0[i]) || !std::isfinite(tb.Pc[i]) || !std::isfinite(tb.Krw[i]) ||
          !std::isfinite(tb.Kro[i]))
        return fail(msg, len, LBM_E_INVAL, "table %g: non-finite sample %g", k, i);
      if (i > 0 && !(tb.K0[i] > 0))
        return fail(msg, len, LBM_E_INVAL, "table %g: K0 must be > 0 for phi > 0 (sample %g)", k, i);
      if (tb.Krw[i] < 0 || tb.Krw[i] > 1 || tb.Kro[i] < 0 || tb.Kro[i] > 1)
        return fail(msg, len, LBM_E_INVAL, "table %g: Kr outside [0,1] at sample %g", k, i);
      if (i > 0) {
        if (tb.Pc[i] > tb.Pc[i - 1])
          return fail(msg, len, LBM_E_INVAL, "table %g: Pc increases at sample %g", k, i);
        if (tb.Krw[i] < tb.Krw[i - 1])
          return fail(msg, len, LBM_E_INVAL, "table %g: Krw decreases at sample %g", k, i);
        if (tb.Kro[i] > tb.Kro[i - 1])
          return fail(msg, len, LBM_E_INVAL, "table %g: Kro increases at sample %g", k, i);
      }
    }
  }
  return LBM_OK;
}

int validate_geometry(long long N, const uint8_t *cls, const double *phi, const uint8_t *pt,
                      int ntab, char *msg, size_t len) {
  if (!cls) return fail(msg, len, LBM_E_INVAL, "cls is NULL");
  long long ngray = 0;
  for (long long v = 0; v < N; ++v) {
    if (cls[v] > 2) return fail(msg, len, LBM_E_INVAL, "class code %g at voxel %g", cls[v], (double)v);
    if (cls[v] == 2) ++ngray;
  }
  if (ngray) {
    if (!phi || !pt) return fail(msg, len, LBM_E_INVAL, "phi and pore_type are needed for gray voxels");
    for (long long v = 0; v < N; ++v) {
      if (cls[v] != 2) continue;
      if (!(phi[v] > 0 && phi[v] < 1))
        return fail(msg, len, LBM_E_INVAL, "gray porosity %g outside (0,1) at voxel %g", phi[v], (double)v);
      if (pt[v] >= ntab)
        return fail(msg, len, LBM_E_INVAL, "pore type %g >= ntab at voxel %g", pt[v], (double)v);
    }
  }
  return LBM_OK;
}

int validate_densities(long long N, const uint8_t *cls, const double *rw, const double *ro,
                       int ncomp, char *msg, size_t len) {
  if (!rw || (ncomp == 2 && !ro)) return fail(msg, len, LBM_E_INVAL, "density array is NULL");
  for (long long v = 0; v < N; ++v) {
    if (cls[v] == 1) continue;
    if (!(rw[v] > 0) || !std::isfinite(rw[v]))
      return fail(msg, len, LBM_E_INVAL, "water density %g invalid at voxel %g", rw[v], (double)v);
    if (ncomp == 2 && (!(ro[v] > 0) || !std::isfinite(ro[v])))
      return fail(msg, len, LBM_E_INVAL, "oil density %g invalid at voxel %g", ro[v], (double)v);
  }
  return LBM_OK;
}

}  // namespace lbm
