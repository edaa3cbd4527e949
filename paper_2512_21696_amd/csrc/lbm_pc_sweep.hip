// Capillary-pressure sweep of many small domains (the Pc(Sw) half of the
// library runs of the paper's Appendix): a drainage through each domain
// between two reservoirs, the inlet's oil density raised level by level, the
// sample's water saturation recorded at a steady state of every level.  Host
// code only: each domain runs on a handle of the two-component step with open
// x faces, through the library's own entry points.
#include <cmath>
#include <string>
#include <vector>

namespace lbm {
namespace pc {

int fail(int code, const std::string &msg) {
  g_create_error = msg;
  return code;
}

// bulk pressure of a reservoir state: cs^2 (rho_w + rho_o) + cs^2 G rho_w rho_o
double bulk_pressure(double rw, double ro, double G) { return (rw + ro + G * rw * ro) / 3.0; }

int check_args(const lbm_pc_params *p, const lbm_pore_table *tab, const lbm_rev_domain *doms,
               int32_t ndom, lbm_pc_result *out) {
  if (!p || !tab || !doms || !out) return fail(LBM_E_INVAL, "NULL argument");
  if (ndom < 1) return fail(LBM_E_INVAL, "ndom must be at least 1");
  if (p->nlevels < 1 || p->nlevels > LBM_PC_MAX_LEVELS)
    return fail(LBM_E_INVAL, "nlevels must lie in 1.." + std::to_string(LBM_PC_MAX_LEVELS));
  for (int k = 0; k < p->nlevels; ++k)
    if (!std::isfinite(p->rho_nw_in[k]) || !(p->rho_nw_in[k] > 0.0))
      return fail(LBM_E_INVAL, "rho_nw_in must be finite and positive");
  if (p->buffer_in < 1) return fail(LBM_E_INVAL, "buffer_in must be at least 1");
  if (p->membrane < 1) return fail(LBM_E_INVAL, "membrane must be at least 1");
  if (p->buffer_out < 2)
    return fail(LBM_E_INVAL, "buffer_out must be at least 2 (gray voxels keep two voxels from the face)");
  if (!(p->membrane_phi > 0.0 && p->membrane_phi < 1.0))
    return fail(LBM_E_INVAL, "membrane_phi must lie in (0, 1)");
  if (p->check_every < 1 || p->max_steps < p->check_every)
    return fail(LBM_E_INVAL, "need check_every >= 1 and max_steps >= check_every");
  if (!(p->tol >= 0.0)) return fail(LBM_E_INVAL, "tol must be non-negative");
  if (p->model.precision == LBM_PREC_F16 || p->model.precision == LBM_PREC_BF16)
    return fail(LBM_E_UNSUPPORTED, "the capillary-pressure sweep runs in fp64 or fp32 storage");
  if (!(p->model.m_minor > 0.0)) return fail(LBM_E_INVAL, "model.m_minor must be positive");
  char msg[256] = {0};
  if (lbm::validate_tables(tab, 1, msg, sizeof msg) != LBM_OK)
    return fail(LBM_E_INVAL, std::string("membrane table: ") + msg);
  for (int d = 0; d < ndom; ++d)
    if (doms[d].nx < 1 || doms[d].ny < 1 || doms[d].nz < 1 || !doms[d].cls)
      return fail(LBM_E_INVAL, "domain " + std::to_string(d) + ": empty or without classes");
  return LBM_OK;
}

// One domain: box, handle, levels.  Writes r.
int run_domain(const lbm_pc_params *p, const lbm_pore_table *tab, const lbm_rev_domain &dom,
               lbm_pc_result &r) {
  const int sw = p->side_walls ? 1 : 0;
  const int nx = p->buffer_in + dom.nx + p->membrane + p->buffer_out;
  const int ny = dom.ny + 2 * sw, nz = dom.nz + 2 * sw;
  const size_t N = (size_t)nx * ny * nz;
  const double m = p->model.m_minor;
  const uint8_t *src = static_cast<const uint8_t *>(dom.cls);
  std::vector<uint8_t> cls(N, LBM_PORE), pt(N, 0);
  std::vector<double> phi(N, 1.0), rw(N), ro(N);
  std::vector<char> sample(N, 0);  // the domain's pore voxels: where Sw is measured
  const int x0 = p->buffer_in, x1 = p->buffer_in + dom.nx, x2 = x1 + p->membrane;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t v = ((size_t)z * ny + y) * nx + x;
        const bool frame = sw && (y == 0 || y == ny - 1 || z == 0 || z == nz - 1);
        uint8_t c = LBM_PORE;
        if (frame) {
          c = LBM_SOLID;
        } else if (x >= x0 && x < x1) {
          const size_t s = ((size_t)(z - sw) * dom.ny + (y - sw)) * dom.nx + (x - x0);
          if (src[s] > 1) return fail(LBM_E_INVAL, "domain classes must be 0 (pore) or 1 (solid)");
          c = src[s];
          sample[v] = c == LBM_PORE;
        } else if (x >= x1 && x < x2) {
          c = LBM_GRAY;
        }
        cls[v] = c;
        phi[v] = c == LBM_GRAY ? p->membrane_phi : (c == LBM_PORE ? 1.0 : 0.0);
        // oil in the inlet buffer, water elsewhere, tanh edge of width 1.5
        const double wfrac = 0.5 * (1.0 + std::tanh((x - (x0 - 0.5)) / 1.5));
        rw[v] = m + (1.0 - m) * wfrac;
        ro[v] = 1.0 + m - rw[v];
      }
  lbm_params q = p->model;
  q.nx = nx;
  q.ny = ny;
  q.nz = nz;
  q.ncomp = 2;
  q.bc_x = LBM_BC_PRESSURE;
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d) q.g[a][d] = 0.0;
  q.track_flux = 0;
  q.outlet_x = nx - 2;
  const double rin0[2] = {m, p->rho_nw_in[0]}, rout[2] = {1.0, m};
  q.rho_in[0] = rin0[0];
  q.rho_in[1] = rin0[1];
  q.rho_out[0] = rout[0];
  q.rho_out[1] = rout[1];
  lbm_handle *h = nullptr;
  int rc = lbm_create(&q, &h);
  if (rc != LBM_OK) return rc;  // (lbm_create left its message)
  auto done = [&](int code) -> int {
    if (code != LBM_OK) g_create_error = h->err;
    lbm_destroy(h);
    return code;
  };
  rc = lbm_set_geometry(h, cls.data(), phi.data(), pt.data(), tab, 1);
  if (rc == LBM_OK) rc = lbm_init_fluid(h, rw.data(), ro.data());
  if (rc != LBM_OK) return done(rc);
  size_t npore = 0;
  for (char c : sample) npore += c;
  std::vector<double> S(N);
  lbm_fields fo{};
  fo.on_device = 0;
  fo.S = S.data();
  auto saturation = [&](double *out_sw) -> int {
    const int e = lbm_get_fields(h, &fo);
    if (e != LBM_OK) return e;
    double acc = 0.0;
    for (size_t v = 0; v < N; ++v)
      if (sample[v]) acc += S[v];
    *out_sw = npore ? acc / (double)npore : 0.0;
    return LBM_OK;
  };
  r.nlevels = p->nlevels;
  r.pad_ = 0;
  const double p_out = bulk_pressure(rout[0], rout[1], q.G);
  double prev = 0.0;
  rc = saturation(&prev);
  if (rc != LBM_OK) return done(rc);
  for (int k = 0; k < p->nlevels; ++k) {
    const double rin[2] = {m, p->rho_nw_in[k]};
    rc = lbm_set_reservoirs(h, rin, rout);
    if (rc != LBM_OK) return done(rc);
    int64_t steps = 0;
    int conv = 0;
    double cur = prev;
    while (steps < p->max_steps) {
      const int64_t n = std::min<int64_t>(p->check_every, p->max_steps - steps);
      rc = lbm_step(h, n);
      if (rc == LBM_OK) rc = saturation(&cur);
      if (rc != LBM_OK) return done(rc);
      steps += n;
      const bool steady = std::fabs(cur - prev) <= p->tol;
      prev = cur;
      if (steady) {
        conv = 1;
        break;
      }
    }
    r.pc[k] = bulk_pressure(rin[0], rin[1], q.G) - p_out;
    r.sw[k] = cur;
    r.steps[k] = steps;
    r.converged[k] = conv;
  }
  return done(LBM_OK);
}

}  // namespace pc
}  // namespace lbm

extern "C" int lbm_rev_pc_sweep(const lbm_pc_params *p, const lbm_pore_table *membrane_table,
                                const lbm_rev_domain *doms, int32_t ndom, lbm_pc_result *out) {
  const Range range("lbm_rev_pc_sweep");
  int rc = lbm::pc::check_args(p, membrane_table, doms, ndom, out);
  if (rc != LBM_OK) return rc;
  for (int d = 0; d < ndom; ++d) {
    out[d] = lbm_pc_result{};
    rc = lbm::pc::run_domain(p, membrane_table, doms[d], out[d]);
    if (rc != LBM_OK) {
      g_create_error = "domain " + std::to_string(d) + ": " + g_create_error;
      return rc;
    }
  }
  return LBM_OK;
}
