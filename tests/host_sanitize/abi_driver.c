/* Calls every entry point of the C ABI on paths that the host decides alone:
 * NULL handles and pointers, invalid parameters, tables, domains and sweep
 * settings, and valid calls that reach the device (they return LBM_E_DEVICE
 * where no GPU is present, or run on a tiny case where one is).  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer over a host-only build of
 * the library; exits non-zero when a status differs from the one expected.
 * Plain C: it also checks that the header compiles as C. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/lbm.h"

static int failures = 0;
static void expect(int got, int want, const char *what) {
  if (got != want) {
    fprintf(stderr, "%s: got %d, want %d\n", what, got, want);
    ++failures;
  }
}
static void expect2(int got, int a, int b, const char *what) {
  if (got != a && got != b) {
    fprintf(stderr, "%s: got %d, want %d or %d\n", what, got, a, b);
    ++failures;
  }
}

static void fill_table(lbm_pore_table *t) {
  for (int i = 0; i < LBM_TABLE_N; ++i) {
    const double s = (double)i / (LBM_TABLE_N - 1);
    t->K0[i] = 1e-3 + s;
    t->Pc[i] = 1.0 - s;
    t->Krw[i] = s;
    t->Kro[i] = 1.0 - s;
  }
  t->phi_ref = 0.3;
  t->Pc_PM = 0.05;
  t->kd[0] = 1.0;
  t->kd[1] = t->kd[2] = 0.1;
}

int main(void) {
  lbm_params p;
  lbm_params_default(&p);
  p.nx = 8;
  p.ny = 6;
  p.nz = 4;
  p.outlet_x = p.nx - 1;
  const size_t N = 8 * 6 * 4;
  lbm_handle *h = (lbm_handle *)0x1;

  /* creation */
  expect(lbm_create(NULL, &h), LBM_E_INVAL, "create NULL params");
  expect(h == NULL, 1, "create clears the handle");
  expect(lbm_create(&p, NULL), LBM_E_INVAL, "create NULL out");
  {
    lbm_params q = p;
    q.tau[0] = 0.25;
    expect(lbm_create(&q, &h), LBM_E_INVAL, "create invalid");
    expect(h == NULL, 1, "no handle on failure");
    expect(strlen(lbm_last_error(NULL)) > 0, 1, "creation message");
  }

  /* every handle call with a NULL handle */
  uint8_t *cls = (uint8_t *)calloc(N, 1);
  double *rho = (double *)malloc(N * sizeof(double));
  for (size_t v = 0; v < N; ++v) rho[v] = 1.0;
  lbm_diag d;
  lbm_fields fo;
  memset(&fo, 0, sizeof fo);
  lbm_kernel_times kt;
  size_t bytes = 0;
  int32_t fl = 0;
  int64_t slots = 0;
  const double rin[2] = {1.0, 0.0}, rout[2] = {1.0, 0.0};
  const double dq[2] = {1.0, 1.0};
  char buf[16];
  expect(lbm_set_geometry(NULL, cls, NULL, NULL, NULL, 0), LBM_E_INVAL, "geometry NULL");
  expect(lbm_init_fluid(NULL, rho, rho), LBM_E_INVAL, "init NULL");
  expect(lbm_step(NULL, 1), LBM_E_INVAL, "step NULL");
  double qf[4];
  expect(lbm_step_flux(NULL, 1, qf), LBM_E_INVAL, "step flux NULL");
  expect(lbm_get_fields(NULL, &fo), LBM_E_INVAL, "fields NULL");
  expect(lbm_get_diagnostics(NULL, &d), LBM_E_INVAL, "diagnostics NULL");
  expect(lbm_get_setup(NULL, rho, NULL, NULL, NULL, NULL), LBM_E_INVAL, "setup NULL");
  expect(lbm_state_size(NULL, &bytes), LBM_E_INVAL, "state size NULL");
  expect(lbm_get_state(NULL, buf, sizeof buf), LBM_E_INVAL, "get state NULL");
  expect(lbm_set_state(NULL, buf, sizeof buf), LBM_E_INVAL, "set state NULL");
  expect(lbm_set_reservoirs(NULL, rin, rout), LBM_E_INVAL, "reservoirs NULL");
  expect(lbm_set_profiling(NULL, 1), LBM_E_INVAL, "profiling NULL");
  expect(lbm_get_kernel_times(NULL, &kt, 0), LBM_E_INVAL, "times NULL");
  expect(lbm_get_layout(NULL, &fl, &slots), LBM_E_INVAL, "layout NULL");
  expect(lbm_adjoint_flux(NULL, 2, dq, 0, NULL, NULL, NULL), LBM_E_INVAL, "adjoint NULL");
  expect(lbm_last_error(NULL) != NULL, 1, "last error");
  lbm_destroy(NULL);

  /* a valid handle where a device exists; LBM_E_DEVICE where none does */
  int rc = lbm_create(&p, &h);
  expect2(rc, LBM_OK, LBM_E_DEVICE, "create valid");
  if (rc == LBM_OK) {
    expect(lbm_step(h, 1), LBM_E_STATE, "step before geometry");
    expect(lbm_set_geometry(h, NULL, NULL, NULL, NULL, 0), LBM_E_INVAL, "geometry NULL cls");
    cls[3] = 7;
    expect(lbm_set_geometry(h, cls, NULL, NULL, NULL, 0), LBM_E_INVAL, "geometry bad class");
    cls[3] = 0;
    expect(lbm_set_geometry(h, cls, NULL, NULL, NULL, 0), LBM_OK, "geometry");
    expect(lbm_step(h, 1), LBM_E_STATE, "step before fluid");
    expect(lbm_step_flux(h, 1, qf), LBM_E_STATE, "step flux before fluid");
    expect(lbm_init_fluid(h, rho, rho), LBM_OK, "init");
    expect(lbm_step(h, 2), LBM_OK, "step");
    expect(lbm_step_flux(h, -1, qf), LBM_E_INVAL, "step flux n < 0");
    expect(lbm_step_flux(h, 1, NULL), LBM_E_INVAL, "step flux NULL output");
    expect(lbm_step_flux(h, 2, qf), LBM_OK, "step flux");
    expect(lbm_get_diagnostics(h, &d), LBM_OK, "diagnostics");
    expect(lbm_state_size(h, &bytes), LBM_OK, "state size");
    expect(lbm_get_state(h, buf, sizeof buf), LBM_E_INVAL, "state buffer too small");
    expect(lbm_get_layout(h, &fl, &slots), LBM_OK, "layout");
    lbm_destroy(h);
  }

  /* batched permeability library: host checks, then a tiny valid batch */
  lbm_rev_params rp;
  memset(&rp, 0, sizeof rp);
  rp.tau = 1.0;
  rp.g = 1e-5;
  rp.max_steps = 4;
  rp.check_every = 2;
  lbm_rev_domain dom;
  memset(&dom, 0, sizeof dom);
  dom.nx = dom.ny = dom.nz = 4;
  uint8_t dcls[64];
  memset(dcls, 0, sizeof dcls);
  dcls[5] = LBM_SOLID;
  dom.cls = dcls;
  lbm_rev_result rr[1];
  expect(lbm_rev_permeability(NULL, &dom, 1, rr), LBM_E_INVAL, "rev NULL params");
  expect(lbm_rev_permeability(&rp, NULL, 1, rr), LBM_E_INVAL, "rev NULL domains");
  expect(lbm_rev_permeability(&rp, &dom, 0, rr), LBM_E_INVAL, "rev no domains");
  expect(lbm_rev_permeability(&rp, &dom, 1, NULL), LBM_E_INVAL, "rev NULL results");
  {
    lbm_rev_params q = rp;
    q.tau = 0.5;
    expect(lbm_rev_permeability(&q, &dom, 1, rr), LBM_E_INVAL, "rev tau");
    q = rp;
    q.axis = 3;
    expect(lbm_rev_permeability_static(&q, &dom, 1, rr), LBM_E_INVAL, "rev static axis");
    q = rp;
    q.precision = 9;
    expect(lbm_rev_permeability(&q, &dom, 1, rr), LBM_E_UNSUPPORTED, "rev precision");
    q = rp;
    q.tol = NAN;
    expect(lbm_rev_permeability(&q, &dom, 1, rr), LBM_E_INVAL, "rev tol nan");
    lbm_rev_domain bad = dom;
    bad.cls = NULL;
    expect(lbm_rev_permeability(&rp, &bad, 1, rr), LBM_E_INVAL, "rev NULL cls");
    bad = dom;
    bad.nx = 0;
    expect(lbm_rev_permeability(&rp, &bad, 1, rr), LBM_E_INVAL, "rev empty box");
  }
  expect2(lbm_rev_permeability(&rp, &dom, 1, rr), LBM_OK, LBM_E_DEVICE, "rev valid");
  expect2(lbm_rev_permeability_static(&rp, &dom, 1, rr), LBM_OK, LBM_E_DEVICE, "rev static valid");

  /* capillary-pressure sweep: host checks */
  lbm_pc_params pc;
  memset(&pc, 0, sizeof pc);
  lbm_params_default(&pc.model);
  pc.buffer_in = 2;
  pc.membrane = 1;
  pc.buffer_out = 2;
  pc.nlevels = 2;
  pc.rho_nw_in[0] = 1.05;
  pc.rho_nw_in[1] = 1.1;
  pc.membrane_phi = 0.3;
  pc.check_every = 2;
  pc.max_steps = 4;
  pc.tol = 1e-3;
  lbm_pore_table *tab = (lbm_pore_table *)calloc(1, sizeof(lbm_pore_table));
  fill_table(tab);
  lbm_pc_result pr[1];
  expect(lbm_rev_pc_sweep(NULL, tab, &dom, 1, pr), LBM_E_INVAL, "pc NULL params");
  expect(lbm_rev_pc_sweep(&pc, NULL, &dom, 1, pr), LBM_E_INVAL, "pc NULL table");
  expect(lbm_rev_pc_sweep(&pc, tab, &dom, 0, pr), LBM_E_INVAL, "pc no domains");
  {
    lbm_pc_params q = pc;
    q.nlevels = LBM_PC_MAX_LEVELS + 1;
    expect(lbm_rev_pc_sweep(&q, tab, &dom, 1, pr), LBM_E_INVAL, "pc levels");
    q = pc;
    q.rho_nw_in[1] = -1.0;
    expect(lbm_rev_pc_sweep(&q, tab, &dom, 1, pr), LBM_E_INVAL, "pc level density");
    q = pc;
    q.model.precision = LBM_PREC_BF16;
    expect(lbm_rev_pc_sweep(&q, tab, &dom, 1, pr), LBM_E_UNSUPPORTED, "pc 16-bit");
    q = pc;
    tab->Pc[10] = 5.0;
    expect(lbm_rev_pc_sweep(&q, tab, &dom, 1, pr), LBM_E_INVAL, "pc bad table");
    fill_table(tab);
  }
  expect2(lbm_rev_pc_sweep(&pc, tab, &dom, 1, pr), LBM_OK, LBM_E_DEVICE, "pc valid");

  free(tab);
  free(cls);
  free(rho);
  if (failures) fprintf(stderr, "%d failures\n", failures);
  else printf("abi_driver: all checks passed\n");
  return failures ? 1 : 0;
}
