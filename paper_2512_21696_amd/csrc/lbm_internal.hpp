// Internal declarations shared by the host runtime and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace lbm {

// Debug builds (-DLBM_DEBUG): device-side index checks.  A failed check sets
// its site's bit in g_dcheck and the kernel goes on (no trap, so a bad index
// never takes the GPU down); the entry points read the bits after their work
// and fail with LBM_E_DEVICE.  Release builds compile the checks away.  The
// sites matter most where the hardware would hide a bad index: population
// accesses through buffer resources read 0 beyond their range.
enum DcheckSite : unsigned {
  DC_PULL = 0,      // fused step: a pulled population beyond its arrays
  DC_STORE = 1,     // fused step: a stored population beyond its arrays
  DC_VOXEL = 2,     // fused step: a per-voxel index beyond N
  DC_DENSITY = 3,   // density pass: a pulled population beyond its arrays
  DC_FIX = 4,       // density fix-up: a source beyond its arrays or the grid
  DC_FLUX = 5,      // outlet flux: a population beyond its arrays
  DC_SCATTER = 6,   // gather / scatter / relayout: an index beyond its arrays
};
#ifdef LBM_DEBUG
__device__ unsigned int g_dcheck;
#define LBM_DCHECK(cond, site)                                            \
  do {                                                                    \
    if (!(cond)) atomicOr(&::lbm::g_dcheck, 1u << (unsigned)(site));     \
  } while (0)
#else
#define LBM_DCHECK(cond, site) ((void)0)
#endif

constexpr int Q = 19;
constexpr int TABLE_N = 1025;

// per-voxel mask word: bit i (0..18) set when x + c_i is a solid voxel;
// class code in bits 24..25.
constexpr uint32_t CLASS_SHIFT = 24;
constexpr uint32_t CLASS_MASK = 3u << CLASS_SHIFT;
constexpr uint32_t SOLID_CODE = 1u;
constexpr uint32_t GRAY_CODE = 2u;

// Scalars of one run, converted once on the host.
struct ModelConsts {
  int nx, ny, nz;
  long long N;
  int ncomp, collision, csf_all, tensor;
  int open_x;        // 1: reservoirs beyond the x faces (pressure or density faces)
  int exact_density; // 1: the faces fix each component's density (Zou-He type)
  double rho_in[2], rho_out[2];
  double tau[2], omega[2], nu[2];
  double G;
  double g[2][3];
  double kappa, csf_scale;  // csf_scale = 1 / (phi_avg phi_max)
  double m_minor, s_min, inv_span;
  double wall_dpsi[2];
  double kr_min, hyst, eps_n;
  int outlet_x;
};

// Population storage: the arithmetic type itself, or 16-bit offsets
// h = f_i / w_i - rho_ref (fp16 or bf16) with fp32 arithmetic.
enum : int { SK_NATIVE = 0, SK_F16 = 2, SK_BF16 = 3 };

// Device buffers of one run (arithmetic type T is float or double).
template <typename T>
struct DevState {
  T *f[2];           // populations, two copies; layout [a][i][v].  16-bit runs:
                     // f[0] is an fp32 decode of the stored set (field
                     // evaluation, initialisation), f[1] is unused
  uint16_t *fc[2];   // 16-bit runs: stored offsets, two copies, layout [a][i][v]
  T *rhoE;           // 16-bit two-component runs: reference densities [v][a]
                     // of the stored offsets (the reader's density)
  T *rho;            // densities at the current level [a][v] (field evaluation)
  T *rho2;           // the same, interleaved [v][a] (fused step)
  T *rho2n;          // the next level's densities, summed by the fused step
                     // from its own post-collision values (fp32 arithmetic,
                     // two components, periodic x), [v][a]
  T *rhoS;           // 16-bit two-component runs: sum_i w_i rho_ref(s_i) over the
                     // sources s_i of each voxel's next pulls [v][a], written by
                     // the fused step for the density pass that follows it
  T *nrm;            // CSF normals [a][3][v] (only when kappa != 0)
  uint32_t *mask;    // neighbour-solid bits and class
  uint8_t *ptype;    // pore type per voxel
  T *K0, *sJ, *thw, *tho;  // gray constitutive values [v]
  T *Kinv;           // inverse permeability [6][v] (tensor runs)
  T *r;              // residual amounts [2][v]
  T *phiT;           // porosity per voxel (1 pore, 0 solid) for diagnostics
  uint8_t *side;     // residual side flag (1 = water)
  T *tab;            // pore tables [type][curve][TABLE_N], curves Pc, Krw, Kro
  double *partial;   // block partials for reductions
  double *acc;       // device accumulators: q_last[2], q_acc[2]
  // Fluid-only population layout (cs != 0): a population array holds cs
  // slots, one per fluid voxel in voxel order.  Per x row (row = y + ny z) and
  // 64-voxel word: cmask the fluid bits, cbase the number of fluid voxels
  // before the word (cw words per row; entry rows * cw is the total).
  const uint64_t *cmask;
  const uint32_t *cbase;
  int cw;
  uint32_t cs;
};

// Where a voxel's populations live: slot = voxel index and array stride N
// (dense), or the fluid-only slot (only fluid voxels have one).
struct PopLayout {
  const uint64_t *cm;
  const uint32_t *cb;
  int cw;
  long long stride;  // elements between population arrays
  __device__ long long slot(long long v, int nx) const {
    if (!cm) return v;
    const long long row = v / nx;
    const int x = (int)(v - row * nx);
    const long long k = row * cw + (x >> 6);
    return (long long)cb[k] + __popcll(cm[k] & ((1ull << (x & 63)) - 1ull));
  }
};

}  // namespace lbm
