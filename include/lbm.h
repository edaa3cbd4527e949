/*
 * lbm.h -- C ABI of the multiscale two-component D3Q19 lattice-Boltzmann step
 * for AMD Instinct MI355X (gfx950).
 *
 * The model (paper: "Enhanced numerical models for two-component fluid flow in
 * multiscale porous structures", Sec. II):
 *   - LB equation on D3Q19 with a collision projected on the Hermite space and
 *     the force term of Eq. (3): the exact-difference form in pore voxels, the
 *     second-order (Guo) form in gray voxels (below), Eqs. (2)-(3);
 *   - Shan-Chen pseudo-potential inter-component force;
 *   - CSF surface-tension control, Eq. (4), in under-resolved (gray) voxels;
 *   - the under-resolved-region force of Eq. (1): capillary term
 *     -Pc(Sw) rho_r n H and Brinkman resistance rho nu / (K0(phi) Kr(Sw)) rho_r u,
 *     with u from the trapezoidal rule (below);
 *   - residual-component model (Sec. II, Fig. 6): trapped water/oil amounts read
 *     off the J-scaled (Eq. (5)) Pc-Sw curve at Pc^{ref,max} / Pc^{ref,min};
 *   - tensorial resistivity, Eqs. (6)-(7), principal axes from the Hessian and
 *     gradient of the porosity field.
 *
 * Conventions shared by every call
 *   - Grid: nx * ny * nz voxels, periodic in all directions.  Linear voxel index
 *     v = x + nx * (y + ny * z) (x fastest).  All host arrays are in that order.
 *   - Components: 0 = water (w), 1 = oil (o).  ncomp = 1 runs water only.
 *   - Voxel classes: LBM_PORE (resolved fluid, phi = 1), LBM_SOLID,
 *     LBM_GRAY (under-resolved porous medium, 0 < phi < 1).
 *   - Velocity set (D3Q19), direction order i = 0..18:
 *       (0,0,0),
 *       (+1,0,0) (-1,0,0) (0,+1,0) (0,-1,0) (0,0,+1) (0,0,-1),
 *       (+1,+1,0) (-1,-1,0) (+1,-1,0) (-1,+1,0) (+1,0,+1) (-1,0,-1)
 *       (+1,0,-1) (-1,0,+1) (0,+1,+1) (0,-1,-1) (0,+1,-1) (0,-1,+1);
 *     directions 2k-1 and 2k are opposite.
 *   - Every function returns an lbm_status (0 = LBM_OK).  No exception crosses
 *     the ABI.  On error, lbm_last_error() describes the cause.  A handle is not
 *     thread-safe; calls on one handle must not overlap.
 *   - Device work is enqueued on params.stream (a hipStream_t; NULL = the null
 *     stream).  Calls that hand data to the host synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_E_INVAL = -1,       /* invalid argument (range, monotonicity, size) */
  LBM_E_NOMEM = -2,       /* device allocation failed (hook returned NULL) */
  LBM_E_DEVICE = -3,      /* HIP runtime error (launch, copy, no device) */
  LBM_E_STATE = -4,       /* call out of order (e.g. step before init) */
  LBM_E_NONFINITE = -5,   /* a diagnostic step found NaN/Inf in the state */
  LBM_E_UNSUPPORTED = -6  /* valid request this build does not implement */
} lbm_status;

enum { LBM_PORE = 0, LBM_SOLID = 1, LBM_GRAY = 2 };
/* Precision.  F64 and F32: populations and arithmetic in that type.  F16 and
 * BF16: populations stored in 16 bits, every other array and all arithmetic in
 * fp32.  A stored population is the offset h = f_i / w_i - rho_ref from the
 * equilibrium weight w_i, where rho_ref is the density (of the same component)
 * of the voxel that wrote it (the post-collision set of a voxel is close to
 * its own equilibrium), taken at the level the population was written;
 * two-component runs keep rho_ref per voxel in fp32, one-component runs use
 * rho_ref = 1.  h is then of the order of the local velocity and
 * non-equilibrium part, also next to an interface, so the 16-bit rounding acts
 * on the deviation from the writer's equilibrium rather than on f. */
enum { LBM_PREC_F64 = 0, LBM_PREC_F32 = 1, LBM_PREC_F16 = 2, LBM_PREC_BF16 = 3 };
enum { LBM_COLL_REGULARIZED = 0, LBM_COLL_BGK = 1 };
enum { LBM_CSF_GRAY = 0, LBM_CSF_ALL = 1 };
/* Time discretisation of the Brinkman resistance of Eq. (1) (the paper is
 * silent): the resistance acts on the velocity u = (rho I + R/2)^-1 (m + F_ex/2)
 * (the trapezoidal rule), F_res^a = -(rho^a / rho) R u, which is also the
 * reported velocity (m + sum_a F^a / 2) / rho.  Its steady states are exactly
 * Darcy's law, whether a body force or a pressure gradient drives the flow, and
 * at rest pressure carries all of a force.  Where R >> rho the gathered
 * momentum of a voxel reverses at every step; gray voxels therefore take the
 * force term of Eq. (3) in its second-order form, with the equilibrium, the
 * non-equilibrium part and the force term all at ua = u' + F^a / (2 rho^a) and
 * the force term weighted by 1 - 1/(2 tau^a), which keeps the large resistance
 * force out of the equilibrium's quadratic terms (pore voxels keep the
 * exact-difference form, equilibrium at u').  Both forms give every component
 * the post-collision momentum of the exact-difference form. */
/* Boundaries of the x faces.  PERIODIC: the grid wraps.  PRESSURE: the paper's
 * pressure inlet and outlet (Sec. III.B-D; it gives no equations): beyond
 * x = 0 and x = nx - 1 lie reservoirs of prescribed densities rho_in and
 * rho_out per component.  A reservoir cell is fluid: it enters the
 * pseudo-potential sum of a boundary voxel with its density, and the
 * populations it sends into the domain are the equilibrium at its density and
 * at the mixture velocity of the adjacent boundary voxel's post-collision set
 * (zero next to a solid voxel).  Gray voxels and, with kappa != 0, the CSF
 * region must stay two voxels away from both faces (LBM_CSF_GRAY required; a
 * gray voxel at x in {0, 1, nx-2, nx-1} is rejected by lbm_set_geometry), so
 * no other stencil reaches a reservoir.  With 16-bit storage the populations
 * written across a face are offsets against their slot owner's reference,
 * like every other slot.
 * DENSITY: exact density faces of the Zou-He type (the paper's pressure
 * inlet and outlet read as boundaries that fix the density of each component
 * on the face voxels).  The reservoir cells beyond the faces stay for the
 * pseudo-potential sums, with the same restrictions, but the populations a
 * face voxel pulls across the face are set so that its pulled set holds the
 * prescribed density of each component (rho_in at x = 0, rho_out at
 * x = nx - 1) and no momentum along y and z: with s = +1 at x = 0 and -1 at
 * x = nx - 1 (the c_x of the unknown directions) and g_j the known pulled
 * values (c_x = 0 or -s, bounce-back at solid sources),
 *   s J = rho_b - sum_{c_x=0} g - 2 sum_{c_x=-s} g,
 *   g_i = g_opp(i) + 6 w_i s J - c_y N_y - c_z N_z   (c_x(i) = s),
 *   N_y = (1/2) sum_{c_x=0} c_y g,  N_z = (1/2) sum_{c_x=0} c_z g,
 * i.e. the opposite value plus the difference of the equilibria at velocity
 * (J / rho_b, 0, 0), with the transverse sums of the in-plane values removed.
 * Needs nx >= 3. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_PRESSURE = 1, LBM_BC_DENSITY = 2 };
/* Population storage layout (not part of the model; results are meant to be
 * bitwise the same either way).  DENSE: one slot per voxel.  AUTO: where the
 * fused step pushes the next level's densities (fp32 storage, two components,
 * periodic x) the populations of solid voxels would not be stored, each
 * population array holding one slot per fluid voxel in voxel order, so that
 * the step neither writes nor fetches cache lines for solid voxels.  That
 * fluid-only layout is switched off in this build (its first GPU run stalled
 * without a fault and the cause is not known): AUTO gives the dense layout,
 * which lbm_get_layout reports. */
enum { LBM_LAYOUT_AUTO = 0, LBM_LAYOUT_DENSE = 1 };

#define LBM_TABLE_N 1025 /* samples of every constitutive curve on [0, 1] */
#define LBM_MAX_TYPES 256

/* Model and run parameters.  Fill with lbm_params_default() first. */
typedef struct lbm_params {
  int32_t nx, ny, nz;     /* grid size, each >= 1 */
  int32_t ncomp;          /* 1 or 2 */
  int32_t precision;      /* LBM_PREC_F64 | LBM_PREC_F32 | LBM_PREC_F16 | LBM_PREC_BF16 */
  int32_t collision;      /* LBM_COLL_REGULARIZED (Hermite-projected) | LBM_COLL_BGK */
  double tau[2];          /* relaxation times (water, oil), > 1/2; nu = (tau - 1/2) / 3 */
  double G;               /* pseudo-potential coupling, F^a = -G rho^a sum_i w_i psi^b(x+c_i) c_i */
  double g[2][3];         /* body acceleration per component, force = rho^a g^a */
  double kappa;           /* CSF coefficient of Eq. (4) */
  int32_t csf_region;     /* LBM_CSF_GRAY (paper) | LBM_CSF_ALL (calibration runs) */
  int32_t tensor;         /* 1: tensorial resistivity, Eqs. (6)-(7); 0: scalar K0 */
  double phi_max, phi_avg;/* characteristic values of Eq. (4) */
  double m_minor;         /* bulk minority density (residual trap keeps rho^a >= m) */
  double s_min, s_max;    /* saturation normalisation: S = clamp((s - s_min)/(s_max - s_min)) */
  double wall_dpsi[2];    /* wettability: a solid neighbour enters the pseudo-potential
                             sum with max(rho^b(x) + wall_dpsi[b], 0); (+, -) is water-wet */
  double kr_min;          /* floor of Kr in the resistance */
  double c_max, c_min;    /* Pc^{ref,max} = c_max Pc_PM, Pc^{ref,min} = c_min Pc_PM */
  double hyst;            /* residual event hysteresis h: events at S >= 1/2+h / S <= 1/2-h */
  double eps_n;           /* |grad rho| below which the CSF normal is zero */
  double sigma_s;         /* Gaussian smoothing std of phi for the principal axes */
  int32_t smooth_radius;  /* smoothing stencil radius (<= 8) */
  int32_t outlet_x;       /* outlet flux plane between x_f and x_f + 1 (0 <= x_f < nx;
                             x_f <= nx - 2 with LBM_BC_PRESSURE) */
  double eps_g, eps_H;    /* isotropic gate: max|lambda| <= eps_H and |grad| <= eps_g */
  double delta_tie;       /* tie-break: |l2| - |l1| <= delta_tie |l3| uses the gradient */
  int32_t diag_every;     /* lbm_step checks for non-finite values every k steps (0 = never) */
  int32_t track_flux;     /* 1: accumulate the outlet flux every step */
  int32_t bc_x;           /* LBM_BC_PERIODIC (default) | LBM_BC_PRESSURE | LBM_BC_DENSITY */
  int32_t layout;         /* LBM_LAYOUT_AUTO (default) | LBM_LAYOUT_DENSE */
  double rho_in[2];       /* open faces: densities (water, oil) of the inlet (x = 0) */
  double rho_out[2];      /* open faces: densities of the outlet (x = nx - 1) */
  /* device allocator hook (NULL = hipMalloc/hipFree); ctx is passed through */
  void *(*alloc)(size_t bytes, void *ctx);
  void (*free)(void *ptr, void *ctx);
  void *alloc_ctx;
  void *stream;           /* hipStream_t the library enqueues on */
} lbm_params;

/* One pore type of the constitutive library (paper, Sec. I step ii; Appendix).
 * Each curve holds LBM_TABLE_N uniform samples on [0, 1] and is evaluated by
 * linear interpolation.  K0 is sampled in phi, the others in water saturation.
 * Requirements (else LBM_E_INVAL): all finite, K0 > 0, Pc non-increasing,
 * Krw non-decreasing, Kro non-increasing, Kr in [0, 1], 0 < phi_ref < 1,
 * Pc_PM > 0, kd > 0. */
typedef struct lbm_pore_table {
  double K0[LBM_TABLE_N];
  double Pc[LBM_TABLE_N];
  double Krw[LBM_TABLE_N];
  double Kro[LBM_TABLE_N];
  double phi_ref;  /* reference porosity of the Pc curve (Leverett-J scaling, Eq. (5)) */
  double Pc_PM;    /* critical (entry) pressure of the type */
  double kd[3];    /* principal permeability multipliers a_k (K^D = a_k K0, Eq. (7)),
                      first along the axis of least porosity curvature */
} lbm_pore_table;

/* Field output.  NULL pointers skip a field.  on_device = 0: host arrays of
 * N doubles; on_device = 1: device arrays of N values of the arithmetic type
 * (double for LBM_PREC_F64, float otherwise).  Values are at the current
 * time level: densities, the velocity u = (m + sum_a F^a / 2) / rho with the
 * total force (u = (rho I + R/2)^-1 (m + F_ex/2) in gray voxels),
 * residual-inclusive saturation S and residual amounts; zero in solid voxels. */
typedef struct lbm_fields {
  int32_t on_device;
  void *rho_w, *rho_o, *ux, *uy, *uz, *S, *r_w, *r_o;
} lbm_fields;

/* Global diagnostics, reduced in fp64. */
typedef struct lbm_diag {
  double mass_w, mass_o;  /* mobile + residual mass per component */
  double sw;              /* sum(phi S) / sum(phi) over fluid voxels */
  double q_w, q_o;        /* outlet flux of the last step per component */
  double q_acc_w, q_acc_o;/* outlet flux accumulated since init */
  double max_u;           /* max |u| */
  int64_t step;           /* steps taken since init */
  int32_t nonfinite;      /* 1 if any population or velocity is NaN/Inf */
  int32_t pad_;
} lbm_diag;

/* Per-kernel device time, recorded with HIP events when profiling is on. */
typedef struct lbm_kernel_times {
  double step_ms;   int64_t step_launches;   /* fused collide-stream kernel */
  double aux_ms;    int64_t aux_launches;    /* density / normal passes */
  double other_ms;  int64_t other_launches;  /* flux, diagnostics */
  double adjoint_ms; int64_t adjoint_launches; /* reverse-step kernels of lbm_adjoint_flux */
} lbm_kernel_times;

typedef struct lbm_handle lbm_handle;

/* Fills p with the defaults (32^3, two components, fp64, regularised, tau = 1,
 * G = 3, no force, kappa = 0, gray CSF region, scalar resistivity, the
 * G = 3 coexistence constants, kr_min = 1e-4, c_max = 3.5, c_min = 0.575,
 * h = 0.05, sigma_s = 1.5, radius 5, eps = 1e-6, delta_tie = 0.05, outlet at
 * nx - 1, flux tracking on, no hooks, null stream).  Never fails. */
void lbm_params_default(lbm_params *p);

/* Host-only validation of p (no device call).  Writes a message to msg (may
 * be NULL).  Returns LBM_OK or LBM_E_INVAL / LBM_E_UNSUPPORTED. */
int lbm_validate_params(const lbm_params *p, char *msg, size_t msglen);

/* The run of the paper's workflow step iii (Sec. I: the multiscale two-component
 * simulation with the library's constitutive inputs), with the model
 * parameters of Sec. II (Eqs. (2)-(4) and the gray force of Eq. (1)).
 * Validates p, allocates the device state through the hook and returns a new
 * handle in *out (NULL on failure; LBM_E_NOMEM when the hook returns NULL).
 * The library owns its device memory until lbm_destroy.
 * Errors: LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE. */
int lbm_create(const lbm_params *p, lbm_handle **out);

/* The segmented image of the workflow (Sec. I, Fig. 1: resolved pore, solid and
 * under-resolved gray voxels with their porosity and pore type, and the
 * per-type K0(phi), Pc(Sw), Kr(Sw) library of its step ii).
 * Copies the geometry in (host arrays of N values owned by the caller):
 * cls (LBM_PORE/LBM_SOLID/LBM_GRAY), phi (in (0,1) on gray voxels, ignored
 * elsewhere), pore_type (< ntab on gray voxels) and ntab pore tables; then runs
 * the per-voxel setup on the device: K0(phi), the Leverett-J factor
 * s_J = sqrt((K0_ref/phi_ref) / (K0/phi)) (Eq. (5)), the residual saturations
 * theta_w, theta_o (Sec. II, Fig. 6) and, with tensor = 1, the inverse
 * permeability tensors (Eqs. (6)-(7)).
 * Invalidates the fluid state (lbm_init_fluid is needed again).
 * Errors: LBM_E_INVAL (codes, ranges, table shape), LBM_E_DEVICE. */
int lbm_set_geometry(lbm_handle *h, const uint8_t *cls, const double *phi,
                     const uint8_t *pore_type, const lbm_pore_table *tabs, int32_t ntab);

/* Initial state of Eq. (2) (the paper gives none): sets every fluid voxel to
 * the rest equilibrium of the given densities
 * (host arrays of N doubles; rho_o ignored for ncomp = 1), clears the residual
 * store, sets the side flag of gray voxels to [S >= 1/2] and the step counter
 * and flux accumulators to zero.  Errors: LBM_E_STATE (no geometry),
 * LBM_E_INVAL (non-finite or non-positive density on a fluid voxel). */
int lbm_init_fluid(lbm_handle *h, const double *rho_w, const double *rho_o);

/* Advances n >= 0 time steps of Eq. (2) (collision and force term, Eq. (3),
 * with the pseudo-potential force, the CSF control of Eq. (4) and the gray
 * force of Eq. (1); streaming), asynchronously on the stream.  Every
 * params.diag_every steps it synchronises and returns LBM_E_NONFINITE if the
 * state holds NaN/Inf.  Errors: LBM_E_STATE (no fluid state), LBM_E_DEVICE. */
int lbm_step(lbm_handle *h, int64_t n);

/* lbm_step's n steps with the outlet flux of each step recorded: q_out (host,
 * 2 n doubles, owned by the caller) receives Q^w and Q^o of step k at
 * q_out[2k] and q_out[2k + 1] (Q^o = 0 with one component), the per-link
 * count through the plane x_f | x_f + 1 that lbm_get_diagnostics reports as
 * q_w, q_o (the outlet flux of the paper's displacement runs, Sec. III).  The
 * steps run asynchronously; the call synchronises once, at the end, instead
 * of once per step.  With params.track_flux the accumulated flux advances as
 * with lbm_step; without it, it does not.  Errors: LBM_E_INVAL (n < 0, q_out
 * NULL with n > 0), LBM_E_STATE (no fluid state), LBM_E_NOMEM (the device
 * history of 2 n doubles), LBM_E_DEVICE, LBM_E_NONFINITE (as lbm_step; q_out
 * is then not written). */
int lbm_step_flux(lbm_handle *h, int64_t n, double *q_out);

/* The fields of the workflow's step iii (Sec. I) and of Eq. (1): component
 * densities rho^a, velocity u, saturation Sw and the residual amounts.
 * Evaluates them at the current time level (see lbm_fields) and writes
 * them; synchronises the stream for host outputs.  Errors: LBM_E_STATE (no
 * fluid state), LBM_E_DEVICE. */
int lbm_get_fields(lbm_handle *h, const lbm_fields *out);

/* Global quantities of the paper's displacement runs (Sec. III: mass per
 * component, the pore-volume saturation Sw and the outlet flux per component).
 * Computes them for the current state; synchronises.  Errors: LBM_E_STATE,
 * LBM_E_DEVICE. */
int lbm_get_diagnostics(lbm_handle *h, lbm_diag *out);

/* The per-voxel set-up of lbm_set_geometry (Eqs. (5)-(7), Fig. 6).
 * Per-voxel setup values (host arrays of N doubles, NULL skips): K0, s_J,
 * theta_w, theta_o, and the inverse permeability as 6 arrays of N in the
 * order xx, yy, zz, xy, xz, yz (K0inv6 may be NULL; zero outside gray). */
int lbm_get_setup(lbm_handle *h, double *K0, double *sJ, double *theta_w,
                  double *theta_o, double *K0inv6);

/* Checkpoint of the state of Eq. (2) (the paper describes none).  The state
 * blob holds a header, the post-streaming populations
 * f[a][i][v] (storage type; for F16/BF16 the 16-bit offsets h, followed for
 * two components by the fp32 reference densities rho_ref[v][a]: the offset
 * pulled by voxel v in direction i decodes as w_i (rho_ref[s] + h) with s the
 * voxel it was pulled from, v - c_i, or v itself when v - c_i is solid), the
 * residual amounts r[a][v] (arithmetic type) and the side
 * flags (one byte per voxel).  lbm_state_size gives its size in bytes; get/set
 * copy it to/from a host buffer of exactly that size.  Resuming is bitwise
 * exact. */
int lbm_state_size(const lbm_handle *h, size_t *bytes);
int lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes);
int lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes);

/* Open x faces (bc_x = LBM_BC_PRESSURE or LBM_BC_DENSITY): replaces the
 * densities (water, oil) prescribed at x = 0 and x = nx - 1 from the next step
 * on, as the quasi-static capillary-pressure protocols of the paper's Appendix
 * step the reservoir pressures.  Enqueues nothing.  LBM_E_STATE on a handle with
 * periodic x faces; LBM_E_INVAL for a negative or non-finite density. */
int lbm_set_reservoirs(lbm_handle *h, const double rho_in[2], const double rho_out[2]);

/* Profiling: when on, each launch is bracketed by HIP events on the stream;
 * lbm_get_kernel_times synchronises and returns the accumulated device time
 * since the last reset.  Off by default. */
int lbm_set_profiling(lbm_handle *h, int32_t on);
int lbm_get_kernel_times(lbm_handle *h, lbm_kernel_times *out, int32_t reset);

/* The population layout in use (storage only; see LBM_LAYOUT_AUTO): writes 1
 * to *fluid_only when solid voxels hold no populations, else 0, and the slots
 * of each population array (N in the dense layout; the fluid voxel count
 * rounded up to a multiple of 64, at most N, otherwise).  It is fixed by
 * lbm_set_geometry.  Host only; either pointer may be NULL.  LBM_E_INVAL for a
 * NULL handle. */
int lbm_get_layout(const lbm_handle *h, int32_t *fluid_only, int64_t *slots);

/* ---------------------------------------------------------------------------
 * Batched single-phase permeability of many small domains.
 *
 * The paper's workflow tabulates K0(phi) per pore type from single-phase runs
 * on fully resolved sub-volumes driven by a body force, with K = phi <u> nu / g
 * (Appendix: the domain mirrored along the force and periodic in that
 * direction, the four other sides closed by walls).  lbm_rev_permeability runs
 * any number of such domains of different sizes together: their pore voxels
 * are packed into one array (each domain padded to a multiple of 256 slots,
 * with a table of each slot's 18 pull sources; solid voxels hold nothing) and
 * one launch per time step updates all of them.  Device memory per call:
 * about 2 x 19 stored values + 19 x 4 bytes per pore slot, plus 8 bytes per
 * voxel of the boxes while the table is built.  Each domain is periodic on
 * its own box (or walled on the sides and mirrored, as flags); the model is the
 * one-component case of lbm_step without gray voxels (D3Q19, halfway
 * bounce-back at solid voxels, the regularised or BGK collision, the force
 * term of Eq. (3) for the body force rho g), started from rest at density 1.
 *
 * Every check_every steps the mean velocity along the force is evaluated per
 * domain (velocity (m + F/2)/rho at the post-streaming level, fp64 sums in a
 * fixed order); a domain has converged when it changed by at most tol times
 * its magnitude since the previous check.  The run stops when every domain
 * has converged or after max_steps; tol = 0 runs exactly max_steps.  A domain
 * without pore voxels gives K = phi = u_mean = 0 and counts as converged from
 * the second check (when tol > 0); if no domain has pore voxels nothing is
 * launched and every result is zero (converged when tol > 0, steps 0).
 */
typedef struct {
  int32_t nx, ny, nz;   /* box (each >= 1) */
  int32_t pad_;
  const uint8_t *cls;   /* host [z][y][x]: LBM_PORE or LBM_SOLID; caller-owned, read once */
  double *u_out;        /* optional host [z][y][x] of the given box (the first half
                           when mirrored): final velocity along the force (0 on solid
                           voxels); NULL skips */
} lbm_rev_domain;

typedef struct {
  double tau;           /* relaxation time, > 1/2 */
  double g;             /* body acceleration along axis, > 0 */
  int32_t axis;         /* 0 = x, 1 = y, 2 = z */
  int32_t collision;    /* LBM_COLL_REGULARIZED or LBM_COLL_BGK */
  int32_t precision;    /* populations are held as offsets and the step works on offsets:
                           LBM_PREC_F64 or LBM_PREC_F32 (storage and arithmetic) hold
                           f_i / w_i - 1 from the rest state at density 1;
                           LBM_PREC_F16 / LBM_PREC_BF16 hold f_i / w_i - rho_writer, the
                           offset from the density of the voxel that wrote it, rounded to
                           nearest even in 16 bits (fp16 scaled by 2^12 to stay in its
                           normal range), with fp32 arithmetic and an fp32 array of the
                           writers' densities */
  int32_t side_walls;   /* 1: the four box faces parallel to the force are walls
                           (bounce-back) instead of periodic */
  int32_t mirror;       /* 1: each domain is run joined to its mirror image along the
                           force (twice the length, periodic across both joints) */
  int32_t pad_;
  int64_t max_steps;    /* >= 0 */
  int64_t check_every;  /* >= 1 */
  double tol;           /* >= 0 */
  void *stream;         /* hipStream_t; NULL is the default stream */
} lbm_rev_params;

typedef struct {
  double K;             /* permeability phi <u> nu / g, nu = (tau - 1/2) / 3 */
  double phi;           /* pore fraction of the box */
  double u_mean;        /* mean velocity along the force over the pore voxels */
  int64_t steps;        /* steps at the check where it converged, or all steps run */
  int32_t converged;    /* 1 when the tol criterion was met */
  int32_t pad_;
  double step_ms;       /* mean device time of one batched step of all domains (HIP
                           events around the step launches; the same in every result) */
} lbm_rev_result;

/* Runs the domains doms[0 .. ndom-1] and writes out[0 .. ndom-1] (caller-owned
 * host arrays).  Device memory is allocated and freed inside the call, which
 * returns after the last result is on the host.  Errors: LBM_E_INVAL for an
 * argument out of range (nothing runs), LBM_E_UNSUPPORTED for an unknown
 * precision or more than 2^31 / 19 packed voxels, LBM_E_NOMEM, LBM_E_DEVICE,
 * LBM_E_NONFINITE when a domain's mean velocity is not finite at a check.  The
 * message is lbm_last_error(NULL). */
int lbm_rev_permeability(const lbm_rev_params *p, const lbm_rev_domain *doms, int32_t ndom,
                         lbm_rev_result *out);

/* Bytes of the no-allocation variant's device scratch (one region per GPU). */
#define LBM_REV_SCRATCH_BYTES (64u << 20)

/* lbm_rev_permeability without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, model, results and errors, except:
 *   - every device buffer of the call (packed populations, neighbour table,
 *     slot maps, partial sums) is carved out of a file-scope device array of
 *     LBM_REV_SCRATCH_BYTES bytes, one per GPU, held until the process ends;
 *     its address is looked up once per device on the first call there;
 *   - a batch needing more than that returns LBM_E_UNSUPPORTED before any
 *     launch, with the size it needs in lbm_last_error(NULL) (about 240 bytes
 *     per packed pore slot plus 4 per voxel of the boxes in fp32: roughly
 *     200,000 pore voxels);
 *   - step launches are not timed: step_ms is 0.
 * The call writes every scratch byte it reads before reading it, so a call
 * never depends on what an earlier one left.  All calls on one GPU share its
 * scratch: calls that overlap on one GPU (other host threads, or streams whose
 * work overlaps) race and must be serialised by the caller.  Host staging of
 * the inputs and results is ordinary host memory. */
int lbm_rev_permeability_static(const lbm_rev_params *p, const lbm_rev_domain *doms,
                                int32_t ndom, lbm_rev_result *out);

/* ---------------------------------------------------------------------------
 * Capillary-pressure sweep of many small domains (the Pc(Sw) half of the
 * library runs of the paper's Appendix: Pc measured through a two-component
 * displacement of a resolved sub-volume, with a reservoir region of 14 cells
 * before it and the pressure difference between the two faces changed in
 * steps, a steady state recorded at each level; Sec. II.A describes the same
 * stepping for its fully resolved run).
 *
 * Reading (the paper gives no equations for it): a drainage sweep.  Each
 * domain (lbm_rev_domain: 0 pore, 1 solid, [z][y][x]) is run along x with
 * open faces (LBM_BC_PRESSURE) inside a box of
 *   buffer_in pore planes | the domain | membrane gray planes | buffer_out
 *   pore planes,
 * with a solid frame on the four sides when side_walls = 1 (the walls of the
 * Appendix's runs).  The sample starts filled with water (wetting with the
 * default wall_dpsi), the inlet buffer with oil (tanh edge of width 1.5).
 * The outlet reservoir holds water (rho_w, rho_o) = (1, m); the inlet
 * reservoir holds oil (m, rho_nw_in[k]) at level k, so the capillary pressure
 * of the level is Pc_k = p(m, rho_nw_in[k]) - p(1, m), with the bulk pressure
 * p = cs^2 (rho_w + rho_o) + cs^2 G rho_w rho_o.  The membrane is a capillary
 * barrier of gray voxels (porosity membrane_phi, one pore table given by the
 * caller): oil enters it only above the table's entry pressure, water passes
 * at its K0, so with an entry pressure above the last level the sample's
 * saturation settles at every level instead of the oil breaking through.
 * Levels run in order from one state.  A level ends when the water
 * saturation Sw of the sample's pore voxels (mean of S over them) changes by
 * at most tol over check_every steps, or after max_steps steps.
 *
 * Every model setting comes from `model` (tau, G, wall_dpsi, m_minor,
 * s_min/s_max, collision, kappa with LBM_CSF_GRAY, precision F64 or F32,
 * hooks, stream); the sweep sets the grid, ncomp = 2, bc_x, the reservoirs,
 * zero body force and no flux tracking.  Domains run one after another on
 * the model's stream, each with its own handle (device memory through the
 * hooks, freed before the next).  Errors: LBM_E_INVAL (arguments, levels,
 * buffer_out < 2, membrane < 1, buffer_in < 1, a membrane table that
 * lbm_set_geometry would reject; all checked before any device work),
 * LBM_E_UNSUPPORTED (16-bit
 * storage), and whatever lbm_create and the calls it makes return; the
 * message is in lbm_last_error(NULL).  Results of the domains before a
 * failing one are written. */
#define LBM_PC_MAX_LEVELS 16
typedef struct {
  lbm_params model;        /* two-component model and run settings (see above) */
  int32_t buffer_in;       /* oil planes before the domain (the paper's 14), >= 1 */
  int32_t membrane;        /* gray planes after the domain, >= 1 */
  int32_t buffer_out;      /* pore planes between the membrane and the outlet face, >= 2 */
  int32_t side_walls;      /* 1: solid frame on the four sides, 0: periodic in y and z */
  int32_t nlevels;         /* 1 .. LBM_PC_MAX_LEVELS */
  int32_t pad_;
  double rho_nw_in[LBM_PC_MAX_LEVELS]; /* inlet oil density per level (finite, > 0) */
  double membrane_phi;     /* porosity of the membrane's gray voxels, in (0, 1) */
  int64_t check_every;     /* steps between saturation checks, >= 1 */
  int64_t max_steps;       /* steps per level at most, >= check_every */
  double tol;              /* steady when |delta Sw| <= tol over check_every steps, >= 0 */
} lbm_pc_params;

typedef struct {
  int32_t nlevels;
  int32_t pad_;
  double pc[LBM_PC_MAX_LEVELS];       /* capillary pressure of the level (reservoir pressures) */
  double sw[LBM_PC_MAX_LEVELS];       /* Sw of the sample's pore voxels at the level's end */
  int64_t steps[LBM_PC_MAX_LEVELS];   /* steps the level took */
  int32_t converged[LBM_PC_MAX_LEVELS];
} lbm_pc_result;

int lbm_rev_pc_sweep(const lbm_pc_params *p, const lbm_pore_table *membrane_table,
                     const lbm_rev_domain *doms, int32_t ndom, lbm_pc_result *out);

/* ---------------------------------------------------------------------------
 * Discrete adjoint of the outlet flux with respect to the gray porosity.
 *
 * The gray-region resistance of Eq. (1) makes the flow depend on phi through
 * K0(phi), the per-pore-type table, and, with the tensorial resistivity,
 * through the principal axes of the smoothed porosity (Eqs. (6)-(7)); with two
 * components phi also enters the capillary term through the Leverett-J factor
 * s_J(phi) (Eq. (5)).  Calibrating phi (or the tables) against an observed flux
 * needs dL/dphi.  For one or two components (with the CSF control of Eq. (4)
 * and the residual transfer; scalar K0 or tensor = 1; periodic x faces, exact
 * density faces (LBM_BC_DENSITY), whose face step is linear in the face
 * voxels' known pulls and is reversed by its transpose, or pressure reservoirs
 * (LBM_BC_PRESSURE), whose equilibrium at the boundary voxel's mixture
 * velocity is differentiated at the velocity each forward step recorded;
 * native fp64 or fp32 storage) and a loss
 * L = sum_n dL_dQ[n] Q(n) over the outlet fluxes Q(1..nsteps) of the next
 * nsteps steps from the current state (Q(n) is lbm_diag.q_w after step n: the
 * first component's post-collision populations of step n crossing
 * outlet_x | outlet_x + 1),
 * lbm_adjoint_flux runs those steps and returns dL/dK0 and dL/dphi on every
 * voxel: the exact gradient of the discrete forward map (the step in exact
 * arithmetic, evaluated at the stored states).  Any differentiable loss of the
 * flux history is handled by passing its gradient at the forward history (run
 * the forward first, e.g. with lbm_step and lbm_get_diagnostics, or take
 * Q_out of a first call with zero dL_dQ).
 *
 * Method: a forward sweep of nsteps ordinary steps with the stored set copied
 * to a checkpoint every checkpoint_every steps, then a reverse sweep segment by
 * segment: each segment's stored sets are recomputed from its checkpoint (the
 * last segment keeps them from the forward sweep, so checkpoint_every =
 * nsteps stores every level and recomputes nothing), and
 * one reverse-step kernel per step applies the transposed streaming (a gather
 * from x + c_i, bounce-back links mapped to the opposite slot), adds the flux
 * weights and the transposed collision Jacobian, and accumulates dL/dK0 (or,
 * with the tensor, dL/dK^-1 per gray voxel; with two components also dL/ds_J,
 * and the reverse of the neighbours' pseudo-potential, saturation-gradient and
 * (CSF) density-gradient and normal reads runs as gathering kernels).  The tensor's dL/dK^-1 goes back
 * through the set-up: first-order perturbation of the Hessian's eigenvectors
 * (and of the tie-break's gradient-aligned axis), the transposed gradient and
 * Hessian stencils and the transposed Gaussian smoothing; the derivative is
 * that of the branch each voxel took (isotropic gate, |lambda| ordering, tie
 * test), exact away from those switches.  dL/dphi adds dL/dK0 times the
 * K0(phi) table's slope on the lookup's cell (the right-hand slope on a table
 * knot) and dL/ds_J times ds_J/dphi.  The residual transfers are switches: the
 * gradient is that of the branch each voxel took at each step (the scale
 * factors and trapped amounts differentiated on it, dL/dr carried between
 * steps, dL/dtheta_w and dL/dtheta_o taken to s_J through the crossings of
 * s_J P_c), which is what finite differences see when no transfer moves.
 *
 * Arguments: nsteps >= 1; dL_dQ a host array of nsteps finite doubles;
 * checkpoint_every >= 1, or 0 for ceil(sqrt(nsteps)); Q_out (nsteps), dL_dK0 and
 * dL_dphi (N each, [z][y][x], zero off gray voxels) host arrays owned by the
 * caller, each may be NULL.  Device memory, allocated through the hook and
 * freed before returning: ceil(nsteps / K) + K + 1 population-sized sets of
 * the storage type (19 N values per component, K = checkpoint_every: checkpoints, the
 * recomputed levels of one segment, two adjoint sets) plus 2 N doubles (scalar
 * K0) or 20 N doubles (tensor), and for two components, per kept level, the
 * residual amounts and side flags (2 N values of the storage type and N
 * bytes), plus 15 N (kappa != 0: 35 N) values of the storage type and 5 N
 * doubles; with pressure reservoirs also 8 ny nz doubles per step (the
 * boundary voxels' densities and velocities).  The adjoint populations are kept
 * in the storage type, the reverse arithmetic and the gradient accumulation in
 * fp64.
 * The handle ends nsteps steps on, exactly as after lbm_step(nsteps) (step
 * counter and flux accumulators included).  Synchronises the stream.
 * Errors: LBM_E_INVAL (argument out of range; nothing runs), LBM_E_STATE (no
 * fluid state), LBM_E_UNSUPPORTED (16-bit storage),
 * LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NONFINITE (from a forward step's diagnostics; a failure inside the last
 * segment's forward steps leaves the handle without a fluid state). */
int lbm_adjoint_flux(lbm_handle *h, int64_t nsteps, const double *dL_dQ,
                     int64_t checkpoint_every, double *Q_out, double *dL_dK0,
                     double *dL_dphi);

/* Description of the last error on h (or, when h is NULL, of the last failed
 * call without a handle: lbm_create, lbm_rev_permeability).  Valid until the
 * next call on h. */
const char *lbm_last_error(const lbm_handle *h);

/* Frees the device state (through the hook) and the handle.  NULL is a no-op. */
void lbm_destroy(lbm_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
