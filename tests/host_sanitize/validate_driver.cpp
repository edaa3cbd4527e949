// Drives the host-only argument validation of the C ABI (lbm_validate.cpp)
// through valid and invalid inputs, including NULL pointers, empty and
// one-byte message buffers and non-finite values, so that a build with
// AddressSanitizer and UndefinedBehaviorSanitizer checks every path.  Exits
// non-zero when a result differs from the expected status code.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/lbm.h"
#include "../../paper_2512_21696_amd/csrc/lbm_validate.hpp"

static int failures = 0;
static void expect(int got, int want, const char *what) {
  if (got != want) {
    std::fprintf(stderr, "%s: got %d, want %d\n", what, got, want);
    ++failures;
  }
}

static void fill_table(lbm_pore_table &t) {
  for (int i = 0; i < LBM_TABLE_N; ++i) {
    const double s = (double)i / (LBM_TABLE_N - 1);
    t.K0[i] = 1e-3 + s;
    t.Pc[i] = 1.0 - s;
    t.Krw[i] = s;
    t.Kro[i] = 1.0 - s;
  }
  t.phi_ref = 0.3;
  t.Pc_PM = 0.05;
  t.kd[0] = 1.0;
  t.kd[1] = t.kd[2] = 0.1;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  char msg[256];
  char one[1];

  // parameters: defaults, every message buffer size, and each rejected field
  lbm_params p;
  lbm_params_default(&p);
  expect(lbm_validate_params(&p, msg, sizeof msg), LBM_OK, "defaults");
  expect(lbm_validate_params(&p, nullptr, 0), LBM_OK, "defaults, no message");
  expect(lbm_validate_params(nullptr, msg, sizeof msg), LBM_E_INVAL, "NULL params");
  expect(lbm_validate_params(nullptr, one, 1), LBM_E_INVAL, "NULL params, 1-byte message");
  expect(lbm_validate_params(nullptr, msg, 0), LBM_E_INVAL, "NULL params, 0-byte message");
  struct Case {
    const char *name;
    void (*set)(lbm_params &);
    int code;
  };
  const Case cases[] = {
      {"nx 0", [](lbm_params &q) { q.nx = 0; }, LBM_E_INVAL},
      {"nz negative", [](lbm_params &q) { q.nz = -4; }, LBM_E_INVAL},
      {"grid too large", [](lbm_params &q) { q.nx = q.ny = q.nz = 2000; }, LBM_E_UNSUPPORTED},
      {"int overflow grid", [](lbm_params &q) { q.nx = q.ny = q.nz = 2147483647; }, LBM_E_UNSUPPORTED},
      {"ncomp 3", [](lbm_params &q) { q.ncomp = 3; }, LBM_E_INVAL},
      {"precision 9", [](lbm_params &q) { q.precision = 9; }, LBM_E_UNSUPPORTED},
      {"collision 5", [](lbm_params &q) { q.collision = 5; }, LBM_E_INVAL},
      {"tau 1/2", [](lbm_params &q) { q.tau[1] = 0.5; }, LBM_E_INVAL},
      {"tau nan", [](lbm_params &q) { q.tau[0] = std::nan(""); }, LBM_E_INVAL},
      {"tau inf", [](lbm_params &q) { q.tau[0] = HUGE_VAL; }, LBM_E_INVAL},
      {"G nan", [](lbm_params &q) { q.G = std::nan(""); }, LBM_E_INVAL},
      {"g inf", [](lbm_params &q) { q.g[1][2] = HUGE_VAL; }, LBM_E_INVAL},
      {"csf region", [](lbm_params &q) { q.csf_region = 7; }, LBM_E_INVAL},
      {"s range", [](lbm_params &q) { q.s_max = q.s_min; }, LBM_E_INVAL},
      {"phi_max", [](lbm_params &q) { q.phi_max = 0; }, LBM_E_INVAL},
      {"m_minor", [](lbm_params &q) { q.m_minor = -1; }, LBM_E_INVAL},
      {"kr_min", [](lbm_params &q) { q.kr_min = 0; }, LBM_E_INVAL},
      {"hyst", [](lbm_params &q) { q.hyst = 0.5; }, LBM_E_INVAL},
      {"eps_n", [](lbm_params &q) { q.eps_n = -1; }, LBM_E_INVAL},
      {"outlet", [](lbm_params &q) { q.outlet_x = q.nx; }, LBM_E_INVAL},
      {"sigma_s", [](lbm_params &q) { q.tensor = 1; q.sigma_s = 0; }, LBM_E_INVAL},
      {"radius", [](lbm_params &q) { q.tensor = 1; q.smooth_radius = 9; }, LBM_E_INVAL},
      {"tensor eps", [](lbm_params &q) { q.tensor = 1; q.eps_H = -1; }, LBM_E_INVAL},
      {"diag_every", [](lbm_params &q) { q.diag_every = -1; }, LBM_E_INVAL},
      {"bc_x", [](lbm_params &q) { q.bc_x = 4; }, LBM_E_INVAL},
      {"layout", [](lbm_params &q) { q.layout = 3; }, LBM_E_INVAL},
      {"density faces nx 2", [](lbm_params &q) { q.bc_x = LBM_BC_DENSITY; q.nx = 2; q.outlet_x = 0; }, LBM_E_INVAL},
      {"pressure outlet", [](lbm_params &q) { q.bc_x = LBM_BC_PRESSURE; q.outlet_x = q.nx - 1; }, LBM_E_INVAL},
      {"pressure csf", [](lbm_params &q) { q.bc_x = LBM_BC_PRESSURE; q.outlet_x = 1; q.kappa = 0.1; q.csf_region = LBM_CSF_ALL; }, LBM_E_INVAL},
      {"reservoir nan", [](lbm_params &q) { q.bc_x = LBM_BC_PRESSURE; q.outlet_x = 1; q.rho_in[1] = std::nan(""); }, LBM_E_INVAL},
      {"hooks", [](lbm_params &q) { q.alloc = [](size_t, void *) -> void * { return nullptr; }; }, LBM_E_INVAL},
  };
  for (const Case &c : cases) {
    lbm_params q = p;
    c.set(q);
    expect(lbm_validate_params(&q, msg, sizeof msg), c.code, c.name);
    expect(lbm_validate_params(&q, one, 1), c.code, c.name);
    expect(lbm_validate_params(&q, nullptr, 0), c.code, c.name);
    if (c.code != LBM_OK && std::strlen(msg) == 0) {
      std::fprintf(stderr, "%s: empty message\n", c.name);
      ++failures;
    }
  }

  // tables: valid, NULL, out-of-range count and each broken curve
  std::vector<lbm_pore_table> tabs(2);
  fill_table(tabs[0]);
  fill_table(tabs[1]);
  expect(lbm::validate_tables(tabs.data(), 2, msg, sizeof msg), LBM_OK, "tables");
  expect(lbm::validate_tables(nullptr, 0, msg, sizeof msg), LBM_OK, "no tables");
  expect(lbm::validate_tables(nullptr, 1, msg, sizeof msg), LBM_E_INVAL, "NULL tables");
  expect(lbm::validate_tables(tabs.data(), -1, msg, sizeof msg), LBM_E_INVAL, "ntab -1");
  expect(lbm::validate_tables(tabs.data(), LBM_MAX_TYPES + 1, msg, sizeof msg), LBM_E_INVAL,
         "ntab too large");
  struct TCase {
    const char *name;
    void (*set)(lbm_pore_table &);
  };
  const TCase tcases[] = {
      {"phi_ref 1", [](lbm_pore_table &t) { t.phi_ref = 1.0; }},
      {"Pc_PM 0", [](lbm_pore_table &t) { t.Pc_PM = 0.0; }},
      {"kd inf", [](lbm_pore_table &t) { t.kd[2] = HUGE_VAL; }},
      {"K0 nan", [](lbm_pore_table &t) { t.K0[LBM_TABLE_N - 1] = std::nan(""); }},
      {"K0 zero", [](lbm_pore_table &t) { t.K0[3] = 0.0; }},
      {"Krw above 1", [](lbm_pore_table &t) { t.Krw[LBM_TABLE_N - 1] = 1.5; }},
      {"Pc increasing", [](lbm_pore_table &t) { t.Pc[7] = t.Pc[6] + 1.0; }},
      {"Krw decreasing", [](lbm_pore_table &t) { t.Krw[9] = 0.0; }},
      {"Kro increasing", [](lbm_pore_table &t) { t.Kro[9] = 1.0; }},
  };
  for (const TCase &c : tcases) {
    std::vector<lbm_pore_table> bad = tabs;
    c.set(bad[1]);
    expect(lbm::validate_tables(bad.data(), 2, msg, sizeof msg), LBM_E_INVAL, c.name);
    expect(lbm::validate_tables(bad.data(), 2, one, 1), LBM_E_INVAL, c.name);
  }

  // geometry and densities on a small box
  const long long N = 5 * 4 * 3;
  std::vector<uint8_t> cls(N, LBM_PORE), pt(N, 0);
  std::vector<double> phi(N, 1.0), rw(N, 1.0), ro(N, 0.01);
  cls[0] = LBM_SOLID;
  cls[N - 1] = LBM_GRAY;
  phi[N - 1] = 0.25;
  pt[N - 1] = 1;
  expect(lbm::validate_geometry(N, cls.data(), phi.data(), pt.data(), 2, msg, sizeof msg), LBM_OK,
         "geometry");
  expect(lbm::validate_geometry(N, nullptr, phi.data(), pt.data(), 2, msg, sizeof msg), LBM_E_INVAL,
         "NULL cls");
  expect(lbm::validate_geometry(N, cls.data(), nullptr, pt.data(), 2, msg, sizeof msg), LBM_E_INVAL,
         "gray without phi");
  expect(lbm::validate_geometry(N, cls.data(), phi.data(), pt.data(), 1, msg, sizeof msg),
         LBM_E_INVAL, "pore type beyond the tables");
  {
    std::vector<uint8_t> c2 = cls;
    c2[5] = 3;
    expect(lbm::validate_geometry(N, c2.data(), phi.data(), pt.data(), 2, one, 1), LBM_E_INVAL,
           "class 3");
    std::vector<double> p2 = phi;
    p2[N - 1] = nan;
    expect(lbm::validate_geometry(N, cls.data(), p2.data(), pt.data(), 2, msg, sizeof msg),
           LBM_E_INVAL, "gray phi nan");
    p2[N - 1] = 1.0;
    expect(lbm::validate_geometry(N, cls.data(), p2.data(), pt.data(), 2, msg, sizeof msg),
           LBM_E_INVAL, "gray phi 1");
  }
  expect(lbm::validate_densities(N, cls.data(), rw.data(), ro.data(), 2, msg, sizeof msg), LBM_OK,
         "densities");
  expect(lbm::validate_densities(N, cls.data(), rw.data(), nullptr, 1, msg, sizeof msg), LBM_OK,
         "one component");
  expect(lbm::validate_densities(N, cls.data(), rw.data(), nullptr, 2, msg, sizeof msg),
         LBM_E_INVAL, "NULL oil");
  {
    std::vector<double> r2 = rw;
    r2[0] = nan;  // solid voxel: ignored
    expect(lbm::validate_densities(N, cls.data(), r2.data(), ro.data(), 2, msg, sizeof msg), LBM_OK,
           "solid nan ignored");
    r2[1] = -inf;
    expect(lbm::validate_densities(N, cls.data(), r2.data(), ro.data(), 2, one, 1), LBM_E_INVAL,
           "negative density");
  }
  if (failures) std::fprintf(stderr, "%d failures\n", failures);
  else std::printf("validate_driver: all checks passed\n");
  return failures ? 1 : 0;
}
