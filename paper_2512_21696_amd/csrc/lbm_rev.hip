// Batched single-phase permeability runs (the REV library of the paper's
// Appendix): many small domains of different sizes packed into one voxel
// array, one launch per time step for all of them.
//
// Packing: domain d occupies packed voxels [voff, voff + N) of one
// structure-of-arrays population buffer f[i][V], padded to a multiple of 256 so
// that a 256-thread block never straddles two domains; blk_dom maps a block to
// its domain.  Padding voxels are marked solid and never touched by a pull.
// The per-voxel model is the one-component step without gray voxels: pull with
// halfway bounce-back (resolved from the neighbour mask, so a wall face of the
// box is just a solid neighbour), moments, the regularised or BGK collision
// and the force term of Eq. (3) for the body force rho g, emitted as the
// quadratic form w_i (A + B.c_i + c_i^T C c_i) like the fused step.
//
// Storage: the arithmetic type T (fp64 or fp32), or 16-bit offsets (fp16 or
// bf16, SK) with fp32 arithmetic: a stored value of direction class i is
// h = f / w_i - 1, the population's departure from the rest state at density 1
// (single-phase flow stays near unit density), decoded as f = w_i (1 + h).
#include <memory>

namespace lbm {
namespace rev {

struct Dom {
  int nx, ny, nz;  // box as run (doubled along the force when mirrored)
  int N;           // voxels of the box
  int voff;        // first packed voxel
  int blk0, nblk;  // its blocks of 256 packed voxels
};

__device__ inline void local_xyz(const Dom &D, int v, int &x, int &y, int &z) {
  const int nxy = D.nx * D.ny;
  z = v / nxy;
  const int r = v - z * nxy;
  y = r / D.nx;
  x = r - y * D.nx;
}

// Class code and neighbour-solid bits of every packed voxel.  wall_axes has
// bit k set when the faces normal to axis k are walls (a neighbour beyond
// them counts as solid); other faces wrap around.
__global__ __launch_bounds__(256) void k_rev_mask(const Dom *__restrict__ doms,
                                                  const int *__restrict__ blk_dom,
                                                  const uint8_t *__restrict__ cls,
                                                  uint32_t *__restrict__ mask, int wall_axes) {
  const int V = blockIdx.x * 256 + threadIdx.x;
  const Dom D = doms[blk_dom[blockIdx.x]];
  const int v = V - D.voff;
  if (v >= D.N) {
    mask[V] = SOLID_CODE << CLASS_SHIFT;
    return;
  }
  int x, y, z;
  local_xyz(D, v, x, y, z);
  uint32_t m = (cls[V] == 1 ? SOLID_CODE : 0u) << CLASS_SHIFT;
  for (int i = 1; i < Q; ++i) {
    int xs = x + cx(i), ys = y + cy(i), zs = z + cz(i);
    bool solid = false;
    if (xs < 0 || xs >= D.nx) {
      if (wall_axes & 1) solid = true;
      xs = xs < 0 ? D.nx - 1 : 0;
    }
    if (ys < 0 || ys >= D.ny) {
      if (wall_axes & 2) solid = true;
      ys = ys < 0 ? D.ny - 1 : 0;
    }
    if (zs < 0 || zs >= D.nz) {
      if (wall_axes & 4) solid = true;
      zs = zs < 0 ? D.nz - 1 : 0;
    }
    if (!solid) solid = cls[D.voff + xs + D.nx * (ys + D.ny * zs)] == 1;
    if (solid) m |= 1u << i;
  }
  mask[V] = m;
}

// Stored slot k of direction class i (opposite directions share a weight).
template <typename T, int SK>
__device__ inline T rev_load(const void *__restrict__ f, uint32_t k, int i) {
  if constexpr (SK == SK_NATIVE) return static_cast<const T *>(f)[k];
  else return (T)wq(i) * ((T)1 + dec16<SK>((uint32_t) static_cast<const uint16_t *>(f)[k]));
}
// zero: a solid slot (never read), stored as zero bits
template <typename T, int SK>
__device__ inline void rev_store(void *__restrict__ f, size_t k, int i, T val, bool zero) {
  if constexpr (SK == SK_NATIVE) static_cast<T *>(f)[k] = zero ? (T)0 : val;
  else
    static_cast<uint16_t *>(f)[k] =
        zero ? (uint16_t)0 : enc16<SK>(val * (T)(1.0 / wq(i)) - (T)1);
}

// rest state at density 1 on pore voxels (16-bit: offset 0), zeros elsewhere
template <typename T, int SK>
__global__ __launch_bounds__(256) void k_rev_init(void *__restrict__ f,
                                                  const uint32_t *__restrict__ mask, int Vtot) {
  const int V = blockIdx.x * 256 + threadIdx.x;
  if (V >= Vtot) return;
  const bool pore = ((mask[V] >> CLASS_SHIFT) & 3u) != SOLID_CODE;
  for (int i = 0; i < Q; ++i) rev_store<T, SK>(f, (size_t)i * Vtot + V, i, (T)wq(i), !pore);
}

// The 19 populations voxel V pulls from the stored (post-collision) set:
// f_i from x - c_i, or this voxel's opposite slot when x - c_i is solid.
template <typename T, int SK>
__device__ inline void pull19(const Dom &D, uint32_t mk, int V, const void *__restrict__ fin,
                              uint32_t Vt, T (&f)[Q]) {
  int x, y, z;
  local_xyz(D, V - D.voff, x, y, z);
  const int X3[3] = {x == 0 ? D.nx - 1 : x - 1, x, x == D.nx - 1 ? 0 : x + 1};
  const int Y3[3] = {y == 0 ? D.ny - 1 : y - 1, y, y == D.ny - 1 ? 0 : y + 1};
  const int Z3[3] = {z == 0 ? D.nz - 1 : z - 1, z, z == D.nz - 1 ? 0 : z + 1};
  f[0] = rev_load<T, SK>(fin, (uint32_t)V, 0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const uint32_t src =
        (uint32_t)(D.voff + X3[1 - cx(i)] + D.nx * (Y3[1 - cy(i)] + D.ny * Z3[1 - cz(i)]));
    const uint32_t k = ((mk >> opp(i)) & 1u) ? (uint32_t)opp(i) * Vt + (uint32_t)V
                                              : (uint32_t)i * Vt + src;
    f[i] = rev_load<T, SK>(fin, k, i);
  }
}

// One time step of every packed domain.
template <typename T, bool REG, int SK>
__global__ __launch_bounds__(256) void k_rev_step(const Dom *__restrict__ doms,
                                                  const int *__restrict__ blk_dom,
                                                  const void *__restrict__ fin,
                                                  void *__restrict__ fout,
                                                  const uint32_t *__restrict__ mask, int Vtot,
                                                  T g0, T g1, T g2, T omega) {
  const int V = blockIdx.x * 256 + threadIdx.x;
  const Dom D = doms[blk_dom[blockIdx.x]];
  const uint32_t mk = mask[V];
  const bool solid = ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  // no pull ever reads a solid slot: a wave of solid voxels (or padding) has
  // nothing to do; solid lanes of mixed waves store zeros so that every store
  // covers whole lines
  if (__all(solid)) return;
  // solid lanes store zeros only when their 128-byte line holds a fluid voxel
  // (16-bit storage: one line per wave, which holds one here)
  constexpr int LPL = 128 / (SK == SK_NATIVE ? (int)sizeof(T) : 2);
  constexpr uint64_t LMASK = LPL >= 64 ? ~0ull : ((1ull << (LPL & 63)) - 1ull);
  const uint64_t live = __ballot(!solid);
  const int lane = threadIdx.x & 63;
  const bool dead_line = solid && ((live >> (lane / LPL * LPL % 64)) & LMASK) == 0ull;
  const uint32_t Vt = (uint32_t)Vtot;
  T f[Q];  // the pulled set
  if (!solid) {
    pull19<T, SK>(D, mk, V, fin, Vt, f);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = (T)0;
  }
  T rho = 0, m0 = 0, m1 = 0, m2 = 0, Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T v = f[i];
    rho += v;
    if (cx(i)) { m0 += cx(i) * v; Pxx += v; }
    if (cy(i)) { m1 += cy(i) * v; Pyy += v; }
    if (cz(i)) { m2 += cz(i) * v; Pzz += v; }
    if (cx(i) && cy(i)) Pxy += cx(i) * cy(i) * v;
    if (cx(i) && cz(i)) Pxz += cx(i) * cz(i) * v;
    if (cy(i) && cz(i)) Pyz += cy(i) * cz(i) * v;
  }
  const T r = solid ? (T)1 : rho;
  const T ir = (T)1 / r;
  // common velocity u' = m / rho, force F = rho g, force term at u' + F/(2 rho)
  const T u0 = m0 * ir, u1 = m1 * ir, u2 = m2 * ir;
  const T F0 = r * g0, F1 = r * g1, F2 = r * g2;
  const T a0 = u0 + (T)0.5 * g0, a1 = u1 + (T)0.5 * g1, a2 = u2 + (T)0.5 * g2;
  const T usq = u0 * u0 + u1 * u1 + u2 * u2;
  const T uF = a0 * F0 + a1 * F1 + a2 * F2;
  const T keep = (T)1 - omega;
  const T we = REG ? r : omega * r;  // weight of the equilibrium part
  T A = we * ((T)1 - (T)1.5 * usq) - (T)3 * uF;
  const T B0 = (T)3 * (we * u0 + F0), B1 = (T)3 * (we * u1 + F1), B2 = (T)3 * (we * u2 + F2);
  const T er = (T)4.5 * we;
  T Cxx = er * u0 * u0 + (T)9 * a0 * F0;
  T Cyy = er * u1 * u1 + (T)9 * a1 * F1;
  T Czz = er * u2 * u2 + (T)9 * a2 * F2;
  T Cxy = er * u0 * u1 + (T)4.5 * (a0 * F1 + a1 * F0);
  T Cxz = er * u0 * u2 + (T)4.5 * (a0 * F2 + a2 * F0);
  T Cyz = er * u1 * u2 + (T)4.5 * (a1 * F2 + a2 * F1);
  if (REG) {
    // non-equilibrium second moment; its first moment vanishes for one component
    const T cs2 = (T)(1.0 / 3.0);
    const T qxx = Pxx - r * (cs2 + u0 * u0), qyy = Pyy - r * (cs2 + u1 * u1);
    const T qzz = Pzz - r * (cs2 + u2 * u2);
    const T qxy = Pxy - r * u0 * u1, qxz = Pxz - r * u0 * u2, qyz = Pyz - r * u1 * u2;
    const T k45 = (T)4.5 * keep;
    A -= (T)1.5 * keep * (qxx + qyy + qzz);
    Cxx += k45 * qxx; Cyy += k45 * qyy; Czz += k45 * qzz;
    Cxy += k45 * qxy; Cxz += k45 * qxz; Cyz += k45 * qyz;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T c0 = (T)cx(i), c1 = (T)cy(i), c2 = (T)cz(i);
    T val = (T)wq(i) * (A + B0 * c0 + B1 * c1 + B2 * c2 + Cxx * c0 * c0 + Cyy * c1 * c1 +
                        Czz * c2 * c2 + (T)2 * (Cxy * c0 * c1 + Cxz * c0 * c2 + Cyz * c1 * c2));
    if (!REG) val += keep * f[i];
    if (!dead_line) rev_store<T, SK>(fout, (size_t)i * Vtot + V, i, val, solid);
  }
}

// Velocity along the force, (m + F/2)_axis / rho, of the post-streaming set
// (the stored set pulled as a step would): per-block fp64 sums over pore
// voxels, and the field when uf is given.
template <typename T, int SK>
__global__ __launch_bounds__(256) void k_rev_velocity(const Dom *__restrict__ doms,
                                                      const int *__restrict__ blk_dom,
                                                      const void *__restrict__ fin,
                                                      const uint32_t *__restrict__ mask, int Vtot,
                                                      int axis, T g, T *__restrict__ uf,
                                                      double *__restrict__ partial) {
  const int V = blockIdx.x * 256 + threadIdx.x;
  const uint32_t mk = mask[V];
  const bool pore = ((mk >> CLASS_SHIFT) & 3u) != SOLID_CODE;
  double val[1] = {0.0};
  T u = 0;
  if (pore) {
    const Dom D = doms[blk_dom[blockIdx.x]];
    T f[Q];
    pull19<T, SK>(D, mk, V, fin, (uint32_t)Vtot, f);
    T rho = 0, m = 0;
    for (int i = 0; i < Q; ++i) {
      const int c = axis == 0 ? cx(i) : (axis == 1 ? cy(i) : cz(i));
      rho += f[i];
      m += c * f[i];
    }
    u = (m + (T)0.5 * rho * g) / rho;
    val[0] = (double)u;
  }
  if (uf) uf[V] = u;
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

int fail(int code, const std::string &msg) {
  g_create_error = msg;
  return code;
}

int check(hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T, int SK>
int run(const lbm_rev_params *p, const lbm_rev_domain *doms, int ndom, lbm_rev_result *out) {
  const hipStream_t st = (hipStream_t)p->stream;
  const int ax = p->axis;
  // boxes as run, packing offsets, block table
  std::vector<Dom> hd(ndom);
  long long Vtot_ll = 0;
  for (int d = 0; d < ndom; ++d) {
    int n[3] = {doms[d].nx, doms[d].ny, doms[d].nz};
    if (p->mirror) n[ax] *= 2;
    const long long N = (long long)n[0] * n[1] * n[2];
    const long long Npad = (N + 255) / 256 * 256;
    if (Vtot_ll + Npad > (long long)(0x7fffffff / Q))
      return fail(LBM_E_UNSUPPORTED, "more than 2^31 / 19 packed voxels");
    hd[d] = Dom{n[0], n[1], n[2], (int)N, (int)Vtot_ll, (int)(Vtot_ll / 256), (int)(Npad / 256)};
    Vtot_ll += Npad;
  }
  const int Vtot = (int)Vtot_ll;
  const int nblk = Vtot / 256;
  std::vector<int> blk_dom(nblk);
  std::vector<uint8_t> hcls((size_t)Vtot, 1);
  std::vector<long long> npore(ndom, 0);
  for (int d = 0; d < ndom; ++d) {
    const Dom &D = hd[d];
    for (int b = 0; b < D.nblk; ++b) blk_dom[D.blk0 + b] = d;
    const int bx = doms[d].nx, by = doms[d].ny;
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
          hcls[(size_t)D.voff + x + (size_t)D.nx * (y + (size_t)D.ny * z)] = c;
          npore[d] += c == LBM_PORE;
        }
  }
  const bool want_u = [&] {
    for (int d = 0; d < ndom; ++d)
      if (doms[d].u_out) return true;
    return false;
  }();

  DevBuf mem;
  Dom *ddom = mem.get<Dom>(ndom);
  int *dblk = mem.get<int>(nblk);
  uint8_t *dcls = mem.get<uint8_t>(Vtot);
  uint32_t *dmask = mem.get<uint32_t>(Vtot);
  const size_t es = SK == SK_NATIVE ? sizeof(T) : 2;  // bytes per stored value
  void *fa = mem.get<uint8_t>((size_t)Q * Vtot * es);
  void *fb = mem.get<uint8_t>((size_t)Q * Vtot * es);
  T *uf = want_u ? mem.get<T>(Vtot) : nullptr;
  double *partial = mem.get<double>(nblk);
  double *usum = mem.get<double>(ndom);
  if (!ddom || !dblk || !dcls || !dmask || !fa || !fb || (want_u && !uf) || !partial || !usum)
    return fail(LBM_E_NOMEM, "device allocation failed");
  hipEvent_t ev0 = mem.event(), ev1 = mem.event();
  if (!ev0 || !ev1) return fail(LBM_E_DEVICE, "hipEventCreate failed");
  double step_ms_total = 0.0;
  int rc = check(hipMemcpyAsync(ddom, hd.data(), ndom * sizeof(Dom), hipMemcpyHostToDevice, st),
                 "copy domains");
  if (rc == LBM_OK)
    rc = check(hipMemcpyAsync(dblk, blk_dom.data(), nblk * sizeof(int), hipMemcpyHostToDevice, st),
               "copy block table");
  if (rc == LBM_OK)
    rc = check(hipMemcpyAsync(dcls, hcls.data(), (size_t)Vtot, hipMemcpyHostToDevice, st),
               "copy classes");
  if (rc != LBM_OK) return rc;
  const int wall_axes = p->side_walls ? (7 & ~(1 << ax)) : 0;
  hipLaunchKernelGGL(k_rev_mask, dim3(nblk), dim3(256), 0, st, ddom, dblk, dcls, dmask, wall_axes);
  hipLaunchKernelGGL((k_rev_init<T, SK>), dim3(nblk), dim3(256), 0, st, fa, dmask, Vtot);

  const T gv[3] = {ax == 0 ? (T)p->g : (T)0, ax == 1 ? (T)p->g : (T)0, ax == 2 ? (T)p->g : (T)0};
  const T omega = (T)(1.0 / p->tau);
  const bool reg = p->collision == LBM_COLL_REGULARIZED;
  const double nu = (p->tau - 0.5) / 3.0;
  std::vector<double> hsum(ndom), prev(ndom, 0.0);
  std::vector<int64_t> conv_step(ndom, -1);
  int64_t done = 0;
  bool have_prev = false;
  auto measure = [&](T *u_field) -> int {
    hipLaunchKernelGGL((k_rev_velocity<T, SK>), dim3(nblk), dim3(256), 0, st, ddom, dblk, fa, dmask,
                       Vtot, ax, (T)p->g, u_field, partial);
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
    rc = check(hipEventRecord(ev0, st), "event");
    if (rc != LBM_OK) return rc;
    for (int64_t s = 0; s < k; ++s) {
      if (reg)
        hipLaunchKernelGGL((k_rev_step<T, true, SK>), dim3(nblk), dim3(256), 0, st, ddom, dblk, fa, fb,
                           dmask, Vtot, gv[0], gv[1], gv[2], omega);
      else
        hipLaunchKernelGGL((k_rev_step<T, false, SK>), dim3(nblk), dim3(256), 0, st, ddom, dblk, fa,
                           fb, dmask, Vtot, gv[0], gv[1], gv[2], omega);
      std::swap(fa, fb);
    }
    rc = check(hipGetLastError(), "step launch");
    if (rc == LBM_OK) rc = check(hipEventRecord(ev1, st), "event");
    if (rc == LBM_OK) rc = check(hipEventSynchronize(ev1), "step");
    float ms = 0.f;
    if (rc == LBM_OK) rc = check(hipEventElapsedTime(&ms, ev0, ev1), "event time");
    if (rc != LBM_OK) return rc;
    step_ms_total += ms;
    done += k;
  }
  if (want_u) {
    rc = measure(uf);
    if (rc != LBM_OK) return rc;
    std::vector<T> hu((size_t)Vtot);
    rc = check(hipMemcpyAsync(hu.data(), uf, (size_t)Vtot * sizeof(T), hipMemcpyDeviceToHost, st),
               "copy velocity");
    if (rc == LBM_OK) rc = check(hipStreamSynchronize(st), "copy velocity");
    if (rc != LBM_OK) return rc;
    for (int d = 0; d < ndom; ++d) {
      if (!doms[d].u_out) continue;
      const Dom &D = hd[d];
      for (int z = 0; z < doms[d].nz; ++z)
        for (int y = 0; y < doms[d].ny; ++y)
          for (int x = 0; x < doms[d].nx; ++x)
            doms[d].u_out[(size_t)x + (size_t)doms[d].nx * (y + (size_t)doms[d].ny * z)] =
                (double)hu[(size_t)D.voff + x + (size_t)D.nx * (y + (size_t)D.ny * z)];
    }
  }
  for (int d = 0; d < ndom; ++d) {
    const double N = (double)hd[d].N;
    out[d].K = hsum[d] / N * nu / p->g;
    out[d].phi = (double)npore[d] / N;
    out[d].u_mean = npore[d] > 0 ? hsum[d] / (double)npore[d] : 0.0;
    out[d].steps = conv_step[d] >= 0 ? conv_step[d] : done;
    out[d].converged = conv_step[d] >= 0;
    out[d].pad_ = 0;
    out[d].step_ms = done > 0 ? step_ms_total / (double)done : 0.0;
  }
  return LBM_OK;
}

}  // namespace rev
}  // namespace lbm

extern "C" int lbm_rev_permeability(const lbm_rev_params *p, const lbm_rev_domain *doms,
                                    int32_t ndom, lbm_rev_result *out) {
  using lbm::rev::fail;
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
  switch (p->precision) {
    case LBM_PREC_F64: return lbm::rev::run<double, lbm::SK_NATIVE>(p, doms, ndom, out);
    case LBM_PREC_F32: return lbm::rev::run<float, lbm::SK_NATIVE>(p, doms, ndom, out);
    case LBM_PREC_F16: return lbm::rev::run<float, lbm::SK_F16>(p, doms, ndom, out);
    default: return lbm::rev::run<float, lbm::SK_BF16>(p, doms, ndom, out);
  }
}
