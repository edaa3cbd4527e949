// Batched single-phase permeability runs (the REV library of the paper's
// Appendix): many small domains of different sizes, one launch per time step
// for all of them.
//
// Layout: only pore voxels hold populations.  Domain d's pore voxels (x
// fastest, then y, z) occupy slots [poff, poff + npore) of one
// structure-of-arrays population buffer f[i][P], padded to a multiple of 256
// so that a 256-thread block never straddles two domains (blk_dom maps a
// block to its domain).  A neighbour table nbr[i - 1][P] (i = 1..18) holds the
// slot of the pore voxel at x - c_i (across a periodic face, or -1 beyond a
// wall face), -1 when that voxel is solid (halfway bounce-back: the slot's own
// opposite population), and -2 on padding slots.  Sphere packs are mostly
// solid (about 70 % here), so a pore update moves 19 + 19 populations and 18
// table entries instead of the populations of 3 voxels.
// The per-voxel model is the one-component step without gray voxels: pull with
// halfway bounce-back, moments, the regularised or BGK collision and the force
// term of Eq. (3) for the body force rho g, emitted as the quadratic form
// w_i (A + B.c_i + c_i^T C c_i) like the fused step.
//
// Storage: every population is held as an offset, f / w_i - 1 from the rest
// state at density 1 (single-phase flow stays near unit density) in the
// arithmetic type T (fp64 or fp32), or f / w_i - rho_writer from the density
// of the voxel that wrote it, rounded to bf16 or (times 2^12) fp16 (SK), with
// fp32 arithmetic and the writers' density offsets in an fp32 array per
// level; the step works on offsets throughout.
#include <memory>
#include <mutex>

namespace lbm {
namespace rev {

struct Dom {
  int nx, ny, nz;  // box as run (doubled along the force when mirrored)
  int N;           // voxels of the box
  int voff;        // first voxel of the box in the dense class / slot map
  int poff;        // first slot
  int npore;       // pore voxels (slots in use)
  int blk0, nblk;  // its blocks of 256 slots
};

// Neighbour table of every slot.  wall_axes has bit k set when the faces
// normal to axis k are walls; other faces wrap around.  slot_of[voff + v] is
// the slot of voxel v of the box or -1 (solid); vox_of[P] the voxel of slot P
// within its box, -1 on padding.
__global__ __launch_bounds__(256) void k_rev_nbr(const Dom *__restrict__ doms,
                                                 const int *__restrict__ blk_dom,
                                                 const int *__restrict__ slot_of,
                                                 const int *__restrict__ vox_of,
                                                 int *__restrict__ nbr, int Ptot, int wall_axes) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  const int v = vox_of[P];
  if (v < 0) {
    for (int i = 1; i < Q; ++i) nbr[(size_t)(i - 1) * Ptot + P] = -2;
    return;
  }
  const Dom D = doms[blk_dom[blockIdx.x]];
  const int nxy = D.nx * D.ny;
  const int z = v / nxy, y = (v - z * nxy) / D.nx, x = v - z * nxy - y * D.nx;
  for (int i = 1; i < Q; ++i) {
    int xs = x - cx(i), ys = y - cy(i), zs = z - cz(i);
    bool wall = false;
    if (xs < 0 || xs >= D.nx) {
      wall |= (wall_axes & 1) != 0;
      xs = xs < 0 ? D.nx - 1 : 0;
    }
    if (ys < 0 || ys >= D.ny) {
      wall |= (wall_axes & 2) != 0;
      ys = ys < 0 ? D.ny - 1 : 0;
    }
    if (zs < 0 || zs >= D.nz) {
      wall |= (wall_axes & 4) != 0;
      zs = zs < 0 ? D.nz - 1 : 0;
    }
    nbr[(size_t)(i - 1) * Ptot + P] = wall ? -1 : slot_of[D.voff + xs + D.nx * (ys + D.ny * zs)];
  }
}

// Stored value k: the offset h = f / w_i - 1 of a population from the rest
// state at density 1, in T or (16-bit storage) bf16, or fp16 scaled by 2^12:
// the offsets of a slow pore (|u| ~ 1e-6, h ~ 3 c.u) would otherwise fall
// below fp16's smallest normal number (6.1e-5) and keep only a few bits, and
// 2^12 still leaves room for |h| up to 16.
constexpr float kRevF16Scale = 4096.f;
template <typename T, int SK>
__device__ inline T rev_load(const void *__restrict__ f, uint32_t k) {
  if constexpr (SK == SK_NATIVE) return static_cast<const T *>(f)[k];
  else if constexpr (SK == SK_F16)
    return dec16<SK>((uint32_t) static_cast<const uint16_t *>(f)[k]) * (T)(1.0f / kRevF16Scale);
  else return dec16<SK>((uint32_t) static_cast<const uint16_t *>(f)[k]);
}
template <typename T, int SK>
__device__ inline void rev_store(void *__restrict__ f, size_t k, T h) {
  if constexpr (SK == SK_NATIVE) static_cast<T *>(f)[k] = h;
  else if constexpr (SK == SK_F16) static_cast<uint16_t *>(f)[k] = enc16<SK>(h * (T)kRevF16Scale);
  else static_cast<uint16_t *>(f)[k] = enc16<SK>(h);
}

// rest state at density 1 (offset 0, reference 0) on every slot, padding
// included
template <typename T, int SK>
__global__ __launch_bounds__(256) void k_rev_init(void *__restrict__ f, T *__restrict__ ref,
                                                  int Ptot) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  for (int i = 0; i < Q; ++i) rev_store<T, SK>(f, (size_t)i * Ptot + P, (T)0);
  if (ref) ref[P] = (T)0;
}

// The 19 offsets f_i / w_i - 1 slot P pulls from the stored (post-collision)
// set: from the slot at x - c_i, or this slot's opposite population when that
// neighbour is solid or a wall (opposite directions share a weight, so the
// offset carries over unchanged).  16-bit storage keeps each value relative
// to its writer's density, h = f_i / w_i - rho_writer, and ref holds the
// writers' density offsets rho - 1 of that level: the offset from the rest
// state is ref[writer] + h.  (Relative to the rest state alone, a stored value
// would carry the pressure field's density offsets, up to 1e-3 here, beside a
// velocity part down to 1e-6 in a tight pore, which 16-bit rounding then
// loses.)
template <typename T, int SK>
__device__ inline void pull19(const int *__restrict__ nbr, int P, const void *__restrict__ fin,
                              const T *__restrict__ ref, uint32_t Pt, T (&h)[Q]) {
  constexpr bool REF = SK != SK_NATIVE;
  const T own = REF ? ref[P] : (T)0;
  h[0] = rev_load<T, SK>(fin, (uint32_t)P) + own;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int s = nbr[(size_t)(i - 1) * Pt + P];
    const uint32_t k = s >= 0 ? (uint32_t)i * Pt + (uint32_t)s : (uint32_t)opp(i) * Pt + (uint32_t)P;
    h[i] = rev_load<T, SK>(fin, k);
    if (REF) h[i] += s >= 0 ? ref[s] : own;
  }
}

// One time step of every packed domain, in offsets: with f_i = w_i (1 + h_i),
// rho = 1 + d with d = sum_i w_i h_i, m = sum_i w_i c_i h_i, and the second
// moment sum_i w_i c_i c_i (1 + h_i) = I / 3 + sum_i w_i c_i c_i h_i, so every
// moment of the departure from rest is formed from the small offsets and the
// new offsets f_post / w_i - 1 come out of the quadratic form with the unit
// density already taken out (the velocity stays accurate in fp32 at the
// 1e-5 body forces of a permeability run).
template <typename T, bool REG, int SK>
__global__ __launch_bounds__(256) void k_rev_step(const int *__restrict__ nbr,
                                                  const void *__restrict__ fin,
                                                  void *__restrict__ fout,
                                                  const T *__restrict__ ref_in,
                                                  T *__restrict__ ref_out, int Ptot,
                                                  T g0, T g1, T g2, T omega) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  const bool pad = nbr[P] == -2;  // padding slot
  if (__all(pad)) return;
  if (pad) return;
  T h[Q];  // the pulled offsets from the rest state
  pull19<T, SK>(nbr, P, fin, ref_in, (uint32_t)Ptot, h);
  T d = 0, m0 = 0, m1 = 0, m2 = 0, Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T v = (T)wq(i) * h[i];
    d += v;
    if (cx(i)) { m0 += cx(i) * v; Pxx += v; }
    if (cy(i)) { m1 += cy(i) * v; Pyy += v; }
    if (cz(i)) { m2 += cz(i) * v; Pzz += v; }
    if (cx(i) && cy(i)) Pxy += cx(i) * cy(i) * v;
    if (cx(i) && cz(i)) Pxz += cx(i) * cz(i) * v;
    if (cy(i) && cz(i)) Pyz += cy(i) * cz(i) * v;
  }
  const T r = (T)1 + d;
  const T ir = (T)1 / r;
  // common velocity u' = m / rho, force F = rho g, force term at u' + F/(2 rho)
  const T u0 = m0 * ir, u1 = m1 * ir, u2 = m2 * ir;
  const T F0 = r * g0, F1 = r * g1, F2 = r * g2;
  const T a0 = u0 + (T)0.5 * g0, a1 = u1 + (T)0.5 * g1, a2 = u2 + (T)0.5 * g2;
  const T usq = u0 * u0 + u1 * u1 + u2 * u2;
  const T uF = a0 * F0 + a1 * F1 + a2 * F2;
  const T keep = (T)1 - omega;
  const T we = REG ? r : omega * r;  // weight of the equilibrium part
  // A - 1: regularised we - 1 = d; BGK we - 1 + keep = omega d (the keep f_i
  // part adds keep h_i below)
  T A = (REG ? d : omega * d) - (T)1.5 * we * usq - (T)3 * uF;
  const T B0 = (T)3 * (we * u0 + F0), B1 = (T)3 * (we * u1 + F1), B2 = (T)3 * (we * u2 + F2);
  const T er = (T)4.5 * we;
  T Cxx = er * u0 * u0 + (T)9 * a0 * F0;
  T Cyy = er * u1 * u1 + (T)9 * a1 * F1;
  T Czz = er * u2 * u2 + (T)9 * a2 * F2;
  T Cxy = er * u0 * u1 + (T)4.5 * (a0 * F1 + a1 * F0);
  T Cxz = er * u0 * u2 + (T)4.5 * (a0 * F2 + a2 * F0);
  T Cyz = er * u1 * u2 + (T)4.5 * (a1 * F2 + a2 * F1);
  if (REG) {
    // non-equilibrium second moment Pi - rho (I/3 + u u), with the unit
    // density's I/3 taken out; its first moment vanishes for one component
    const T d3 = d * (T)(1.0 / 3.0);
    const T qxx = Pxx - d3 - r * u0 * u0, qyy = Pyy - d3 - r * u1 * u1;
    const T qzz = Pzz - d3 - r * u2 * u2;
    const T qxy = Pxy - r * u0 * u1, qxz = Pxz - r * u0 * u2, qyz = Pyz - r * u1 * u2;
    const T k45 = (T)4.5 * keep;
    A -= (T)1.5 * keep * (qxx + qyy + qzz);
    Cxx += k45 * qxx; Cyy += k45 * qyy; Czz += k45 * qzz;
    Cxy += k45 * qxy; Cxz += k45 * qxz; Cyz += k45 * qyz;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T c0 = (T)cx(i), c1 = (T)cy(i), c2 = (T)cz(i);
    T val = A + B0 * c0 + B1 * c1 + B2 * c2 + Cxx * c0 * c0 + Cyy * c1 * c1 + Czz * c2 * c2 +
            (T)2 * (Cxy * c0 * c1 + Cxz * c0 * c2 + Cyz * c1 * c2);
    if (!REG) val += keep * h[i];
    if (SK != SK_NATIVE) val -= d;  // relative to this voxel's density (its mass is kept)
    rev_store<T, SK>(fout, (size_t)i * Ptot + P, val);
  }
  if (SK != SK_NATIVE) ref_out[P] = d;
}

// Velocity along the force, (m + F/2)_axis / rho, of the post-streaming set
// (the stored set pulled as a step would): per-block fp64 sums over pore
// voxels, and the field when uf is given.
template <typename T, int SK>
__global__ __launch_bounds__(256) void k_rev_velocity(const int *__restrict__ nbr,
                                                      const void *__restrict__ fin,
                                                      const T *__restrict__ ref, int Ptot,
                                                      int axis, T g, T *__restrict__ uf,
                                                      double *__restrict__ partial) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  const bool pore = nbr[P] != -2;
  double val[1] = {0.0};
  T u = 0;
  if (pore) {
    T h[Q];
    pull19<T, SK>(nbr, P, fin, ref, (uint32_t)Ptot, h);
    T d = 0, m = 0;
    for (int i = 0; i < Q; ++i) {
      const int c = axis == 0 ? cx(i) : (axis == 1 ? cy(i) : cz(i));
      const T v = (T)wq(i) * h[i];
      d += v;
      m += c * v;
    }
    const T rho = (T)1 + d;
    u = (m + (T)0.5 * rho * g) / rho;
    val[0] = (double)u;
  }
  if (uf) uf[P] = u;
  block_sum<1>(val, partial + blockIdx.x, false);
}

// per-domain sums of the block partials, one 256-thread block per domain:
// strided partial sums, then a fixed tree (the order depends only on the
// domain's block count, so results are reproducible and batch-independent)
__global__ __launch_bounds__(256) void k_rev_reduce(const Dom *__restrict__ doms,
                                                    const double *__restrict__ partial,
                                                    double *__restrict__ usum) {
  __shared__ double sh[256];
  const Dom D = doms[blockIdx.x];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < D.nblk; b += 256) s += partial[D.blk0 + b];
  sh[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) usum[blockIdx.x] = sh[0];
}

struct DevBuf {  // device allocations and events of one call, freed on every exit path
  std::vector<void *> ptrs;
  std::vector<hipEvent_t> events;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    events.push_back(e);
    return e;
  }
  template <typename U>
  U *get(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(U)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<U *>(p);
  }
};

// Device memory of one call taken from a fixed region (the file-scope scratch
// array of the no-allocation entry point): consecutive 256-byte aligned
// pieces; `need` grows by every request, whether it fits or not, so that a
// run can report the size it needs.
struct Carve {
  char *base;
  size_t cap;
  size_t need = 0;
  template <typename U>
  U *get(size_t n) {
    const size_t bytes = (std::max<size_t>(n, 1) * sizeof(U) + 255) / 256 * 256;
    const size_t at = need;
    need += bytes;
    if (need > cap) return nullptr;
    return reinterpret_cast<U *>(base + at);
  }
};

int fail(int code, const std::string &msg) {
  g_create_error = msg;
  return code;
}

int check(hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T, int SK, typename Mem, typename WriteU>
int run_steps(const lbm_rev_params *p, const lbm_rev_domain *doms, int ndom, lbm_rev_result *out,
              const std::vector<Dom> &hd, const std::vector<int> &slot_of,
              const std::vector<int> &vox_of, const std::vector<int> &blk_dom, int Vtot, int Ptot,
              int nblk, bool want_u, const WriteU &write_u, Mem &mem);

// scratch == nullptr: device memory from hipMalloc, freed on exit, step
// launches timed with HIP events.  Otherwise every device buffer is carved
// out of the scratch region (cap bytes) and nothing is allocated or timed.
template <typename T, int SK>
int run(const lbm_rev_params *p, const lbm_rev_domain *doms, int ndom, lbm_rev_result *out,
        void *scratch = nullptr, size_t cap = 0) {
  const hipStream_t st = (hipStream_t)p->stream;
  const int ax = p->axis;
  // boxes as run, dense offsets, slots of the pore voxels, block table
  std::vector<Dom> hd(ndom);
  long long Vtot_ll = 0;
  for (int d = 0; d < ndom; ++d) {
    int n[3] = {doms[d].nx, doms[d].ny, doms[d].nz};
    if (p->mirror) n[ax] *= 2;
    const long long N = (long long)n[0] * n[1] * n[2];
    if (Vtot_ll + N > (long long)0x7fffffff) return fail(LBM_E_UNSUPPORTED, "more than 2^31 voxels");
    hd[d] = Dom{n[0], n[1], n[2], (int)N, (int)Vtot_ll, 0, 0, 0, 0};
    Vtot_ll += N;
  }
  const int Vtot = (int)Vtot_ll;
  std::vector<int> slot_of((size_t)Vtot, -1), vox_of;
  long long Ptot_ll = 0;
  for (int d = 0; d < ndom; ++d) {
    Dom &D = hd[d];
    D.poff = (int)Ptot_ll;
    const int bx = doms[d].nx, by = doms[d].ny;
    int np = 0;
    for (int z = 0; z < D.nz; ++z)
      for (int y = 0; y < D.ny; ++y)
        for (int x = 0; x < D.nx; ++x) {
          int s[3] = {x, y, z};
          if (p->mirror) {  // the second half is the mirror image of the first
            const int L = (&doms[d].nx)[ax];
            if (s[ax] >= L) s[ax] = 2 * L - 1 - s[ax];
          }
          const uint8_t c = doms[d].cls[(size_t)s[0] + (size_t)bx * (s[1] + (size_t)by * s[2])];
          if (c != LBM_PORE && c != LBM_SOLID)
            return fail(LBM_E_INVAL, "domain classes must be LBM_PORE or LBM_SOLID");
          if (c == LBM_PORE) {
            const int v = x + D.nx * (y + D.ny * z);
            slot_of[(size_t)D.voff + v] = D.poff + np++;
            vox_of.push_back(v);
          }
        }
    const long long ppad = ((long long)np + 255) / 256 * 256;
    if (Ptot_ll + ppad > (long long)(0x7fffffff / Q))
      return fail(LBM_E_UNSUPPORTED, "more than 2^31 / 19 pore voxels");
    vox_of.resize((size_t)(Ptot_ll + ppad), -1);
    D.npore = np;
    D.blk0 = (int)(Ptot_ll / 256);
    D.nblk = (int)(ppad / 256);
    Ptot_ll += ppad;
  }
  const int Ptot = (int)Ptot_ll;
  const int nblk = Ptot / 256;
  std::vector<int> blk_dom((size_t)std::max(nblk, 1), 0);
  for (int d = 0; d < ndom; ++d)
    for (int b = 0; b < hd[d].nblk; ++b) blk_dom[(size_t)hd[d].blk0 + b] = d;
  const bool want_u = [&] {
    for (int d = 0; d < ndom; ++d)
      if (doms[d].u_out) return true;
    return false;
  }();
  auto write_u = [&](const std::vector<T> &hu) {  // slots back to the callers' boxes
    for (int d = 0; d < ndom; ++d) {
      if (!doms[d].u_out) continue;
      const Dom &D = hd[d];
      const int L = (&doms[d].nx)[ax];
      std::fill(doms[d].u_out, doms[d].u_out + (size_t)doms[d].nx * doms[d].ny * doms[d].nz, 0.0);
      for (int k = 0; k < D.npore; ++k) {
        const int v = vox_of[(size_t)D.poff + k];
        const int z = v / (D.nx * D.ny), y = (v / D.nx) % D.ny, x = v % D.nx;
        const int c[3] = {x, y, z};
        if (c[ax] >= L) continue;  // the mirrored half
        doms[d].u_out[(size_t)x + (size_t)doms[d].nx * (y + (size_t)doms[d].ny * z)] =
            hu.empty() ? 0.0 : (double)hu[(size_t)D.poff + k];
      }
    }
  };
  const double nu = (p->tau - 0.5) / 3.0;
  if (nblk == 0) {  // no pore voxel anywhere: nothing flows
    write_u({});
    for (int d = 0; d < ndom; ++d)
      out[d] = lbm_rev_result{0.0, 0.0, 0.0, 0, p->tol > 0 ? 1 : 0, 0, 0.0};
    return LBM_OK;
  }

  if (scratch) {
    Carve mem{static_cast<char *>(scratch), cap};
    return run_steps<T, SK>(p, doms, ndom, out, hd, slot_of, vox_of, blk_dom, Vtot, Ptot, nblk,
                            want_u, write_u, mem);
  }
  DevBuf mem;
  return run_steps<T, SK>(p, doms, ndom, out, hd, slot_of, vox_of, blk_dom, Vtot, Ptot, nblk,
                          want_u, write_u, mem);
}

// The device part of run(): buffers from `mem` (DevBuf or Carve), set-up,
// the step loop with its convergence checks, results.
template <typename T, int SK, typename Mem, typename WriteU>
int run_steps(const lbm_rev_params *p, const lbm_rev_domain *doms, int ndom, lbm_rev_result *out,
              const std::vector<Dom> &hd, const std::vector<int> &slot_of,
              const std::vector<int> &vox_of, const std::vector<int> &blk_dom, int Vtot, int Ptot,
              int nblk, bool want_u, const WriteU &write_u, Mem &mem) {
  const hipStream_t st = (hipStream_t)p->stream;
  const int ax = p->axis;
  const double nu = (p->tau - 0.5) / 3.0;
  constexpr bool timed = std::is_same<Mem, DevBuf>::value;
  Dom *ddom = mem.template get<Dom>(ndom);
  int *dblk = mem.template get<int>(nblk);
  int *dslot = mem.template get<int>(Vtot);
  int *dvox = mem.template get<int>(Ptot);
  int *dnbr = mem.template get<int>((size_t)(Q - 1) * Ptot);
  const size_t es = SK == SK_NATIVE ? sizeof(T) : 2;  // bytes per stored value
  void *fa = mem.template get<uint8_t>((size_t)Q * Ptot * es);
  void *fb = mem.template get<uint8_t>((size_t)Q * Ptot * es);
  T *uf = want_u ? mem.template get<T>(Ptot) : nullptr;
  // 16-bit storage: the writers' density offsets, one array per level
  T *ra = SK != SK_NATIVE ? mem.template get<T>(Ptot) : nullptr;
  T *rb = SK != SK_NATIVE ? mem.template get<T>(Ptot) : nullptr;
  double *partial = mem.template get<double>(nblk);
  double *usum = mem.template get<double>(ndom);
  if (!ddom || !dblk || !dslot || !dvox || !dnbr || !fa || !fb || (want_u && !uf) || !partial ||
      !usum || (SK != SK_NATIVE && (!ra || !rb))) {
    if constexpr (!timed)
      return fail(LBM_E_UNSUPPORTED, "the domains need " + std::to_string(mem.need) +
                                         " bytes of device memory; the static scratch holds " +
                                         std::to_string(mem.cap));
    return fail(LBM_E_NOMEM, "device allocation failed");
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if constexpr (timed) {
    ev0 = mem.event();
    ev1 = mem.event();
    if (!ev0 || !ev1) return fail(LBM_E_DEVICE, "hipEventCreate failed");
  }
  double step_ms_total = 0.0;
  int rc = check(hipMemcpyAsync(ddom, hd.data(), ndom * sizeof(Dom), hipMemcpyHostToDevice, st),
                 "copy domains");
  if (rc == LBM_OK)
    rc = check(hipMemcpyAsync(dblk, blk_dom.data(), nblk * sizeof(int), hipMemcpyHostToDevice, st),
               "copy block table");
  if (rc == LBM_OK)
    rc = check(hipMemcpyAsync(dslot, slot_of.data(), (size_t)Vtot * sizeof(int),
                              hipMemcpyHostToDevice, st),
               "copy slot map");
  if (rc == LBM_OK)
    rc = check(hipMemcpyAsync(dvox, vox_of.data(), (size_t)Ptot * sizeof(int),
                              hipMemcpyHostToDevice, st),
               "copy slot voxels");
  if (rc != LBM_OK) return rc;
  const int wall_axes = p->side_walls ? (7 & ~(1 << ax)) : 0;
  hipLaunchKernelGGL(k_rev_nbr, dim3(nblk), dim3(256), 0, st, ddom, dblk, dslot, dvox, dnbr, Ptot,
                     wall_axes);
  hipLaunchKernelGGL((k_rev_init<T, SK>), dim3(nblk), dim3(256), 0, st, fa, ra, Ptot);

  const T gv[3] = {ax == 0 ? (T)p->g : (T)0, ax == 1 ? (T)p->g : (T)0, ax == 2 ? (T)p->g : (T)0};
  const T omega = (T)(1.0 / p->tau);
  const bool reg = p->collision == LBM_COLL_REGULARIZED;
  std::vector<double> hsum(ndom), prev(ndom, 0.0);
  std::vector<int64_t> conv_step(ndom, -1);
  int64_t done = 0;
  bool have_prev = false;
  auto measure = [&](T *u_field) -> int {
    hipLaunchKernelGGL((k_rev_velocity<T, SK>), dim3(nblk), dim3(256), 0, st, dnbr, fa,
                       (const T *)ra, Ptot, ax, (T)p->g, u_field, partial);
    hipLaunchKernelGGL(k_rev_reduce, dim3(ndom), dim3(256), 0, st, ddom, partial, usum);
    int r = check(hipMemcpyAsync(hsum.data(), usum, ndom * sizeof(double), hipMemcpyDeviceToHost, st),
                  "copy sums");
    if (r == LBM_OK) r = check(hipStreamSynchronize(st), "step");
    if (r != LBM_OK) return r;
    for (int d = 0; d < ndom; ++d)
      if (!std::isfinite(hsum[d]))
        return fail(LBM_E_NONFINITE, "non-finite velocity in domain " + std::to_string(d) +
                                         " at step " + std::to_string((long long)done));
    return LBM_OK;
  };
  while (true) {
    rc = measure(nullptr);
    if (rc != LBM_OK) return rc;
    bool all = true;
    for (int d = 0; d < ndom; ++d) {
      if (conv_step[d] < 0 && have_prev && p->tol > 0 &&
          std::fabs(hsum[d] - prev[d]) <= p->tol * std::fabs(hsum[d]))
        conv_step[d] = done;
      all = all && conv_step[d] >= 0;
      prev[d] = hsum[d];
    }
    have_prev = true;
    if (all || done >= p->max_steps) break;
    const int64_t k = std::min<int64_t>(p->check_every, p->max_steps - done);
    if (timed) {
      rc = check(hipEventRecord(ev0, st), "event");
      if (rc != LBM_OK) return rc;
    }
    for (int64_t s = 0; s < k; ++s) {
      if (reg)
        hipLaunchKernelGGL((k_rev_step<T, true, SK>), dim3(nblk), dim3(256), 0, st, dnbr, fa, fb,
                           (const T *)ra, rb, Ptot, gv[0], gv[1], gv[2], omega);
      else
        hipLaunchKernelGGL((k_rev_step<T, false, SK>), dim3(nblk), dim3(256), 0, st, dnbr, fa, fb,
                           (const T *)ra, rb, Ptot, gv[0], gv[1], gv[2], omega);
      std::swap(fa, fb);
      std::swap(ra, rb);
    }
    rc = check(hipGetLastError(), "step launch");
    float ms = 0.f;
    if (timed) {
      if (rc == LBM_OK) rc = check(hipEventRecord(ev1, st), "event");
      if (rc == LBM_OK) rc = check(hipEventSynchronize(ev1), "step");
      if (rc == LBM_OK) rc = check(hipEventElapsedTime(&ms, ev0, ev1), "event time");
    }
    if (rc != LBM_OK) return rc;
    step_ms_total += ms;
    done += k;
  }
  if (want_u) {
    rc = measure(uf);
    if (rc != LBM_OK) return rc;
    std::vector<T> hu((size_t)Ptot);
    rc = check(hipMemcpyAsync(hu.data(), uf, (size_t)Ptot * sizeof(T), hipMemcpyDeviceToHost, st),
               "copy velocity");
    if (rc == LBM_OK) rc = check(hipStreamSynchronize(st), "copy velocity");
    if (rc != LBM_OK) return rc;
    write_u(hu);
  }
  for (int d = 0; d < ndom; ++d) {
    const double N = (double)hd[d].N;
    out[d].K = hsum[d] / N * nu / p->g;
    out[d].phi = (double)hd[d].npore / N;
    out[d].u_mean = hd[d].npore > 0 ? hsum[d] / (double)hd[d].npore : 0.0;
    out[d].steps = conv_step[d] >= 0 ? conv_step[d] : done;
    out[d].converged = conv_step[d] >= 0;
    out[d].pad_ = 0;
    out[d].step_ms = done > 0 ? step_ms_total / (double)done : 0.0;
  }
  return LBM_OK;
}

// The no-allocation entry point's device memory: one file-scope array per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in for the symbol):
// scratch_address() looks up its device address once per device, with that
// device current, and every later use goes through that pointer.
static __device__ __align__(256) unsigned char scratch[LBM_REV_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void **out) {
  int dev = 0;
  int rc = check(hipGetDevice(&dev), "hipGetDevice");
  if (rc != LBM_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_E_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    rc = check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc != LBM_OK) return rc;
    if (!ptr) return fail(LBM_E_DEVICE, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

int check_args(const lbm_rev_params *p, const lbm_rev_domain *doms, int32_t ndom,
               lbm_rev_result *out) {
  if (!p || !doms || !out) return fail(LBM_E_INVAL, "NULL argument");
  if (ndom < 1) return fail(LBM_E_INVAL, "ndom must be at least 1");
  if (!(p->tau > 0.5)) return fail(LBM_E_INVAL, "tau must exceed 1/2");
  if (!(p->g > 0.0) || !std::isfinite(p->g)) return fail(LBM_E_INVAL, "g must be positive");
  if (p->axis < 0 || p->axis > 2) return fail(LBM_E_INVAL, "axis must be 0, 1 or 2");
  if (p->collision != LBM_COLL_REGULARIZED && p->collision != LBM_COLL_BGK)
    return fail(LBM_E_INVAL, "unknown collision");
  if (p->max_steps < 0 || p->check_every < 1 || !(p->tol >= 0.0))
    return fail(LBM_E_INVAL, "max_steps >= 0, check_every >= 1 and tol >= 0 are required");
  if ((p->side_walls != 0 && p->side_walls != 1) || (p->mirror != 0 && p->mirror != 1))
    return fail(LBM_E_INVAL, "side_walls and mirror are 0 or 1");
  for (int d = 0; d < ndom; ++d) {
    if (doms[d].nx < 1 || doms[d].ny < 1 || doms[d].nz < 1 || !doms[d].cls)
      return fail(LBM_E_INVAL, "domain " + std::to_string(d) + ": box >= 1 and classes required");
    if ((long long)doms[d].nx * doms[d].ny * doms[d].nz * (p->mirror ? 2 : 1) > 0x7fffffff / Q)
      return fail(LBM_E_UNSUPPORTED, "domain " + std::to_string(d) + " is too large");
  }
  if (p->precision < LBM_PREC_F64 || p->precision > LBM_PREC_BF16)
    return fail(LBM_E_UNSUPPORTED, "unknown precision");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(LBM_E_DEVICE, "no HIP device");
  return LBM_OK;
}

int dispatch(const lbm_rev_params *p, const lbm_rev_domain *doms, int32_t ndom,
             lbm_rev_result *out, void *scr, size_t cap) {
  switch (p->precision) {
    case LBM_PREC_F64: return run<double, SK_NATIVE>(p, doms, ndom, out, scr, cap);
    case LBM_PREC_F32: return run<float, SK_NATIVE>(p, doms, ndom, out, scr, cap);
    case LBM_PREC_F16: return run<float, SK_F16>(p, doms, ndom, out, scr, cap);
    default: return run<float, SK_BF16>(p, doms, ndom, out, scr, cap);
  }
}

}  // namespace rev
}  // namespace lbm

extern "C" int lbm_rev_permeability_static(const lbm_rev_params *p, const lbm_rev_domain *doms,
                                           int32_t ndom, lbm_rev_result *out) {
  const Range range("lbm_rev_permeability_static");
  int rc = lbm::rev::check_args(p, doms, ndom, out);
  if (rc != LBM_OK) return rc;
  void *scr = nullptr;
  rc = lbm::rev::scratch_address(&scr);
  if (rc != LBM_OK) return rc;
  return lbm::rev::dispatch(p, doms, ndom, out, scr, (size_t)LBM_REV_SCRATCH_BYTES);
}

extern "C" int lbm_rev_permeability(const lbm_rev_params *p, const lbm_rev_domain *doms,
                                    int32_t ndom, lbm_rev_result *out) {
  const Range range("lbm_rev_permeability");
  const int rc = lbm::rev::check_args(p, doms, ndom, out);
  if (rc != LBM_OK) return rc;
  return lbm::rev::dispatch(p, doms, ndom, out, nullptr, 0);
}
