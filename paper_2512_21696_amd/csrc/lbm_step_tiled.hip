// The fused collide-stream kernel of one time step (gfx950).
//
// A block owns a column of 64 x 4 voxels (one wavefront per x-row, so every
// population load and store of a wave covers 256 contiguous bytes) and
// marches along z through a chunk of planes.  A rolling window in LDS holds
// five planes of (rho_w, rho_o) on the column plus a radius-2 halo (periodic
// wrap; +inf marks a solid cell) with the mobile saturation S_hat of each
// cell, and one plane of the CSF normals
// n^a = grad rho^b / |grad rho^b| on the column plus a radius-1 halo.  Each
// density plane is staged once and serves every stencil of the step
// (pseudo-potential sum, grad rho^b, the normals, grad S_hat); each normal
// plane is consumed as soon as it is made, its contributions to the
// curvature -div n^a of the voxels on the planes below, on and above it
// summed in registers.  Blocks are numbered so that the blocks resident
// on one XCD (dispatch is round-robin over the 8 XCDs) cover neighbouring
// columns, which keeps halo re-reads inside that XCD's L2.
//
// Collision: with the Hermite-projected (regularised) operator the
// post-collision set depends on the gathered populations only through their
// first moments (rho, rho u, the second-moment tensor), so the pull
// accumulates those ten moments per component on the fly (pairing opposite
// directions).  Equilibrium, projected non-equilibrium part and the force term
// of Eq. (3) are each a quadratic form w_i (A + B.c_i + c_i^T C c_i), so the
// 19 outgoing populations follow from ten coefficients per component.  The
// BGK variant keeps the populations.
//
// fp32 runs use the hardware reciprocal and reciprocal square root (1 ulp);
// fp64 runs divide exactly.
//
// 16-bit storage (fp16 or bf16, fp32 arithmetic): a stored population is the
// offset h = f_i / w_i - rho_ref, rho_ref being the density of the voxel that
// wrote it, at the level it was written.  A voxel's post-collision set is close
// to its own equilibrium, so h is of the order of its velocity and
// non-equilibrium part even where the neighbour that pulls it lies across an
// interface.  The writer encodes with its own density; the reader decodes each
// pulled value with the reference of the voxel it came from, which the block
// stages in LDS (three planes of the previous level's densities).
#include <type_traits>

namespace lbm {
namespace zm {
constexpr int TX = 64, TY = 4;
constexpr int NT = TX * TY;
constexpr int R = 2;
constexpr int HX = TX + 2 * R, HY = TY + 2 * R;
constexpr int NH = HX * HY;  // density plane cells
constexpr int MX = TX + 2, MY = TY + 2;
constexpr int NM = MX * MY;  // normal plane cells
constexpr int RS = 5;        // density planes z-2 .. z+2
constexpr int ZC = 32;       // planes per block without an occupancy figure (halved on small grids)
__host__ __device__ constexpr int hoff(int i) { return cx(i) + HX * cy(i); }
__host__ __device__ constexpr int moff(int i) { return cx(i) + MX * cy(i); }
}  // namespace zm

// Run constants pre-converted to the arithmetic type, so the kernel reads
// them as scalar operands instead of converting inside the loop.
template <typename T>
struct KC {
  int nx, ny, nz, csf_all, tensor, collision, open_x;
  long long N;
  T g[2][3], omega[2], nu[2], wall_dpsi[2], rho_in[2], rho_out[2];
  T G, kappa, csf_fac, s_min, inv_span, kr_min, hyst, m_minor, eps_n2;
};

template <typename T>
KC<T> make_kc(const ModelConsts &m) {
  KC<T> k{};
  k.nx = m.nx; k.ny = m.ny; k.nz = m.nz; k.N = m.N;
  k.csf_all = m.csf_all; k.tensor = m.tensor; k.collision = m.collision;
  k.open_x = m.open_x;
  for (int a = 0; a < 2; ++a) {
    k.rho_in[a] = (T)m.rho_in[a];
    k.rho_out[a] = (T)m.rho_out[a];
    for (int d = 0; d < 3; ++d) k.g[a][d] = (T)m.g[a][d];
    k.omega[a] = (T)m.omega[a];
    k.nu[a] = (T)m.nu[a];
    k.wall_dpsi[a] = (T)m.wall_dpsi[a];
  }
  k.G = (T)m.G; k.kappa = (T)m.kappa;
  k.csf_fac = (T)(m.kappa * m.csf_scale);  // kappa / (phi_avg phi_max)
  k.s_min = (T)m.s_min; k.inv_span = (T)m.inv_span; k.kr_min = (T)m.kr_min;
  k.hyst = (T)m.hyst; k.m_minor = (T)m.m_minor; k.eps_n2 = (T)(m.eps_n * m.eps_n);
  return k;
}

template <typename T> __device__ inline T rcp(T x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }
template <typename T> __device__ inline T rsq(T x);
template <> __device__ inline float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsq<double>(double x) { return 1.0 / sqrt(x); }

template <typename T> struct vec4 { T x, y, z, w; };
template <typename T> struct alignas(2 * sizeof(T)) vec2 { T x, y; };

__device__ inline int wrapn(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}
// Raw buffer access with 32-bit byte offsets (one resource per component's
// 19 population arrays, which stay below 4 GiB).
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ inline rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ inline float bload(rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline double bload(rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// Population stores are marked non-temporal (cache-policy bit 1, NT): the
// new set is not read again within the step, and streaming it past the L2
// leaves the L2 to the pulled lines that neighbouring tiles share.
constexpr int kStoreNT = 2;
__device__ inline void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kStoreNT);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ inline void bstore(rsrc_t r, uint32_t voff, uint32_t soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, voff, soff, kStoreNT);
}

__device__ inline uint32_t bload16(rsrc_t r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
__device__ inline void bstore16(rsrc_t r, uint32_t voff, uint32_t soff, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, voff, soff, kStoreNT);
}
template <int SK> __device__ inline float dec16(uint32_t bits);
template <> __device__ inline float dec16<SK_F16>(uint32_t bits) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
}
template <> __device__ inline float dec16<SK_BF16>(uint32_t bits) {
  return __builtin_bit_cast(float, bits << 16);
}
// round to nearest even
template <int SK> __device__ inline uint16_t enc16(float x);
template <> __device__ inline uint16_t enc16<SK_F16>(float x) {
  return __builtin_bit_cast(uint16_t, (_Float16)x);
}
template <> __device__ inline uint16_t enc16<SK_BF16>(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
// One pulled value: the population itself (native storage) or its stored
// offset h (16-bit storage).  off is the element index within the component.
template <typename T, int SK>
__device__ inline T pull_value(rsrc_t r, uint32_t off) {
  if constexpr (SK == SK_NATIVE) return bload(r, off * (uint32_t)sizeof(T), (T)0);
  else return (T)dec16<SK>(bload16(r, off * 2u));
}

// Raw pulled value (the population, or the 16-bit offset's bits) and its
// conversion to the arithmetic type, split so the loads can be issued a plane
// ahead of their use.
template <typename T, int SK>
__device__ inline auto pull_raw(rsrc_t r, uint32_t off) {
  if constexpr (SK == SK_NATIVE) return bload(r, off * (uint32_t)sizeof(T), (T)0);
  else return bload16(r, off * 2u);
}
// The same with the population array's start as a scalar byte offset.
template <typename T, int SK>
__device__ inline auto pull_raw_s(rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (SK == SK_NATIVE) {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
  }
}
// Keeps a running scalar offset in one SGPR: the compiler may not fold the
// per-direction offsets into 19 loop-invariant registers (which it would then
// spill into vector lanes and reload on every use).
__device__ inline void keep_scalar(uint32_t &so) { asm volatile("" : "+s"(so)); }

template <typename T, int SK, typename L>
__device__ inline T pull_decode(L raw) {
  if constexpr (SK == SK_NATIVE) return raw;
  else return (T)dec16<SK>(raw);
}

__device__ inline int rslot(int z) { return (z + 10) % 5; }

// Writes the 19 populations w_i (A + B.c_i + c_i^T C c_i) * sc (plus
// keep * sc * f_i for BGK) of one component; voff is the voxel's byte offset
// within its plane, sbase the byte offset of the plane.
// SKIPZ: lanes with `zero` set store nothing (fluid-only layout: a solid
// voxel has no slot).
template <typename T, bool REG, bool OUTV = false, bool SKIPZ = false>
__device__ __forceinline__ void emit_post(rsrc_t out, uint32_t voff, uint32_t sbase,
                                          uint32_t Nbytes, T A, T B0, T B1, T B2, T Cxx, T Cyy,
                                          T Czz, T Cxy, T Cxz, T Cyz, T sc, const T *fpop,
                                          T keep, bool zero, T *outv = nullptr) {
  const T w0 = (T)(1.0 / 3.0) * sc, w1 = (T)(1.0 / 18.0) * sc, w2 = (T)(1.0 / 36.0) * sc;
  T v[Q];
  v[0] = w0 * A;
  const T ax = A + Cxx, ay = A + Cyy, az = A + Czz;
  v[1] = w1 * (ax + B0);
  v[2] = w1 * (ax - B0);
  v[3] = w1 * (ay + B1);
  v[4] = w1 * (ay - B1);
  v[5] = w1 * (az + B2);
  v[6] = w1 * (az - B2);
  const T exy = ax + Cyy, exz = ax + Czz, eyz = ay + Czz;
  const T dxy = (T)2 * Cxy, dxz = (T)2 * Cxz, dyz = (T)2 * Cyz;
  const T pxy = exy + dxy, mxy = exy - dxy, pxz = exz + dxz, mxz = exz - dxz;
  const T pyz = eyz + dyz, myz = eyz - dyz;
  const T s01 = B0 + B1, d01 = B0 - B1, s02 = B0 + B2, d02 = B0 - B2, s12 = B1 + B2,
          d12 = B1 - B2;
  v[7] = w2 * (pxy + s01);
  v[8] = w2 * (pxy - s01);
  v[9] = w2 * (mxy + d01);
  v[10] = w2 * (mxy - d01);
  v[11] = w2 * (pxz + s02);
  v[12] = w2 * (pxz - s02);
  v[13] = w2 * (mxz + d02);
  v[14] = w2 * (mxz - d02);
  v[15] = w2 * (pyz + s12);
  v[16] = w2 * (pyz - s12);
  v[17] = w2 * (myz + d12);
  v[18] = w2 * (myz - d12);
  if (!SKIPZ || !zero) {
    uint32_t so = sbase;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T val = v[i];
      if (!REG) val += keep * sc * fpop[i];
      bstore(out, voff, so, SKIPZ ? val : (zero ? (T)0 : val));
      so += Nbytes;
      keep_scalar(so);
    }
  }
  if (OUTV) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T val = v[i];
      if (!REG) val += keep * sc * fpop[i];
      outv[i] = zero ? (T)0 : val;  // the value its readers will pull
    }
  }
}

// 16-bit variant: stores enc((A + B.c_i + c_i^T C c_i) sc - ref) where ref
// is the writing voxel's density (plus keep * sc * g_i, g_i = f_i / w_i, for
// BGK).
template <int SK, bool REG, bool OUTV = false>
__device__ __forceinline__ void emit_post16(rsrc_t out, uint32_t voff, uint32_t sbase,
                                            uint32_t Nbytes, float A, float B0, float B1,
                                            float B2, float Cxx, float Cyy, float Czz, float Cxy,
                                            float Cxz, float Cyz, float sc, const float *gpop,
                                            float keep, bool zero, float ref,
                                            float *outv = nullptr) {
  float v[Q];
  v[0] = A;
  const float ax = A + Cxx, ay = A + Cyy, az = A + Czz;
  v[1] = ax + B0;
  v[2] = ax - B0;
  v[3] = ay + B1;
  v[4] = ay - B1;
  v[5] = az + B2;
  v[6] = az - B2;
  const float exy = ax + Cyy, exz = ax + Czz, eyz = ay + Czz;
  const float dxy = 2.f * Cxy, dxz = 2.f * Cxz, dyz = 2.f * Cyz;
  const float pxy = exy + dxy, mxy = exy - dxy, pxz = exz + dxz, mxz = exz - dxz;
  const float pyz = eyz + dyz, myz = eyz - dyz;
  const float s01 = B0 + B1, d01 = B0 - B1, s02 = B0 + B2, d02 = B0 - B2, s12 = B1 + B2,
              d12 = B1 - B2;
  v[7] = pxy + s01;
  v[8] = pxy - s01;
  v[9] = mxy + d01;
  v[10] = mxy - d01;
  v[11] = pxz + s02;
  v[12] = pxz - s02;
  v[13] = mxz + d02;
  v[14] = mxz - d02;
  v[15] = pyz + s12;
  v[16] = pyz - s12;
  v[17] = myz + d12;
  v[18] = myz - d12;
  uint32_t so = sbase;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float val = v[i] * sc;
    if (!REG) val += keep * sc * gpop[i];
    val -= ref;
    const uint16_t code = zero ? (uint16_t)0 : enc16<SK>(val);
    bstore16(out, voff, so, code);
    // the population its readers decode, w_i (ref + h)
    if (OUTV) outv[i] = zero ? 0.f : (float)wq(i) * (ref + dec16<SK>(code));
    so += Nbytes;
    keep_scalar(so);
  }
}

// Densities of the current level for the fused step: the pull of every
// population (bounce-back at solid sources) summed per component, written
// interleaved [v][rho_w, rho_o].  Solid voxels get +inf in both slots: the
// fused step recognises solid halo cells by it (a fluid density is finite),
// and never uses the value itself.  With 16-bit storage
// rho = sum_i w_i (rho_ref(s_i) + h_i), s_i the voxel the offset was pulled
// from (its writer) and rho_ref from rhoE.
template <typename T, int NC, int SK, bool GATHER>
__global__ __launch_bounds__(256) void k_density(const void *__restrict__ fin,
                                                 T *__restrict__ rho2, const T *__restrict__ rhoE,
                                                 const T *__restrict__ rhoS,
                                                 const uint32_t *__restrict__ mask, int nx, int ny,
                                                 int nz, long long N) {
  const uint32_t v = blockIdx.x * 256u + threadIdx.x;
  if (v >= (uint32_t)N) return;
  const uint32_t mk = mask[v];
  vec2<T> *out = reinterpret_cast<vec2<T> *>(rho2);
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) {
    out[v] = vec2<T>{(T)INFINITY, (T)INFINITY};
    return;
  }
  const uint32_t N32 = (uint32_t)N;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const uint32_t z = v / nxy;
  const uint32_t rem = v - z * nxy;
  const uint32_t y = rem / (uint32_t)nx;
  const uint32_t x = rem - y * (uint32_t)nx;
  const uint32_t X3[3] = {x == 0 ? nx - 1 : x - 1, x, x == (uint32_t)nx - 1 ? 0 : x + 1};
  const uint32_t Y3[3] = {(y == 0 ? ny - 1 : y - 1) * nx, y * nx,
                          (y == (uint32_t)ny - 1 ? 0 : y + 1) * nx};
  const uint32_t Z3[3] = {(z == 0 ? nz - 1 : z - 1) * nxy, z * nxy,
                          (z == (uint32_t)nz - 1 ? 0 : z + 1) * nxy};
  constexpr uint32_t ES = SK == SK_NATIVE ? (uint32_t)sizeof(T) : 2u;
  T r[2] = {0, 0};
  // 16-bit storage: the reference part sum_i w_i rho_ref(s_i) comes from
  // the step that wrote the set (rhoS), or is gathered here (GATHER)
  constexpr bool gather = SK != SK_NATIVE && GATHER;
  T q[2] = {0, 0};
  if constexpr (SK != SK_NATIVE && !GATHER) {
    const vec2<T> e = reinterpret_cast<const vec2<T> *>(rhoS)[v];
    q[0] = e.x;
    q[1] = e.y;
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const rsrc_t rin = make_rsrc((const char *)fin + (size_t)a * Q * N * ES, (uint32_t)(Q * N * ES));
    T v0 = pull_value<T, SK>(rin, v);
    if constexpr (gather) v0 += rhoE[2 * v + a];
    T axis = 0, diag = 0;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const int j = i + 1;
      // sources: x - c_i for i, x + c_i for j; this voxel under bounce-back
      const bool bi = (mk >> j) & 1u, bj = (mk >> i) & 1u;
      const uint32_t si = bi ? v : X3[1 - cx(i)] + Y3[1 - cy(i)] + Z3[1 - cz(i)];
      const uint32_t sj = bj ? v : X3[1 + cx(i)] + Y3[1 + cy(i)] + Z3[1 + cz(i)];
      const uint32_t oi = bi ? (uint32_t)j * N32 + v : (uint32_t)i * N32 + si;
      const uint32_t oj = bj ? (uint32_t)i * N32 + v : (uint32_t)j * N32 + sj;
      LBM_DCHECK(si < N32 && sj < N32 && oi < Q * N32 && oj < Q * N32, DC_DENSITY);
      T pair = pull_value<T, SK>(rin, oi) + pull_value<T, SK>(rin, oj);
      // 16-bit: each offset decodes with its writer's reference density
      if constexpr (gather) pair += rhoE[2 * si + a] + rhoE[2 * sj + a];
      if (i < 7) axis += pair;
      else diag += pair;
    }
    if constexpr (SK == SK_NATIVE) r[a] = v0 + axis + diag;
    else r[a] = q[a] + ((T)(1.0 / 3.0) * v0 + (T)(1.0 / 18.0) * axis + (T)(1.0 / 36.0) * diag);
  }
  out[v] = vec2<T>{r[0], r[1]};
}

template <typename T, int NC, bool REG, int SK, bool PUSH = false, bool CMP = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_step_zm(const KC<T> mc, const void *__restrict__ fin,
                                                 void *__restrict__ fout, const DevState<T> s,
                                                 const int tiles_x, const int tiles_y,
                                                 const int zc, const int ntiles) {
  using namespace zm;
  constexpr bool STENCIL = NC == 2;
  using T4 = vec4<T>;
  using T2 = vec2<T>;
  __shared__ T2 srho[STENCIL ? RS : 1][STENCIL ? NH : 1];  // rho_w, rho_o (+inf: solid)
  __shared__ T sshat[STENCIL ? RS : 1][STENCIL ? NH : 1];  // mobile saturation S_hat
  // (n^w_d, n^o_d) of one plane; the push exchange of the next level's
  // densities reuses the space between the normals' last read and their next
  // write (a barrier on each side)
  constexpr int NRM_BYTES = 3 * (STENCIL ? NM : 1) * (int)sizeof(T2);
  // rows 0 .. TY-2 send up, rows 1 .. TY-1 send down: [TY-1][TX][c_z + 1][NC] each
  constexpr int PUSH_ROW = TX * 3 * NC;
  constexpr int PUSH_BYTES = PUSH ? 2 * (TY - 1) * PUSH_ROW * (int)sizeof(T) : 0;
  static_assert(PUSH_BYTES <= NRM_BYTES || !STENCIL, "the push exchange fits the normals' space");
  __shared__ __align__(16) unsigned char snrm_raw[NRM_BYTES > PUSH_BYTES ? NRM_BYTES : PUSH_BYTES];
  T2(*snrm)[STENCIL ? NM : 1] = reinterpret_cast<T2(*)[STENCIL ? NM : 1]>(snrm_raw);
  T *const spush_up = reinterpret_cast<T *>(snrm_raw);
  T *const spush_dn = spush_up + (TY - 1) * PUSH_ROW;
  __shared__ int sxw[HX], syw[HY];
  __shared__ int sxg[HX];  // open x faces: 1 beyond x = 0, 2 beyond x = nx-1 (reservoir cells)
  // 16-bit storage, two components: reference densities (the writers'
  // densities of the previous level) of planes z-1 .. z+1 on the tile plus a
  // radius-1 halo, in a ring of three planes
  constexpr bool REFS = SK != SK_NATIVE && NC == 2;
  __shared__ T2 sref[REFS ? 3 : 1][REFS ? NM : 1];

  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int per = nb / 8;  // the grid is a multiple of 8: bijection on [0, nb)
  const int tl = (b % 8) * per + b / 8;
  if (tl >= ntiles) return;  // whole block leaves together
  const int bx = tl % tiles_x;
  const int by = (tl / tiles_x) % tiles_y;
  const int bzc = tl / (tiles_x * tiles_y);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nx = mc.nx, ny = mc.ny, nz = mc.nz;
  const long long N = mc.N;
  const uint32_t N32 = (uint32_t)N;
  static_assert(!CMP || (TX == 64 && SK == SK_NATIVE), "fluid-only layout: one 64-voxel word per tile row");
  // population array stride: every voxel, or (fluid-only layout) every fluid voxel
  const uint32_t NSTR = CMP ? s.cs : N32;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const int x0 = bx * TX, y0 = by * TY;
  const int zs = bzc * zc;
  const int ze = zs + zc < nz ? zs + zc : nz;
  const bool csf = STENCIL && mc.kappa != (T)0;
  constexpr uint32_t ES = SK == SK_NATIVE ? (uint32_t)sizeof(T) : 2u;  // population element
  constexpr bool S16 = SK != SK_NATIVE;
  const T2 *rho2 = reinterpret_cast<const T2 *>(s.rho2);

  // Staging of one density plane: each thread owns up to 3 cells of the
  // (64+4) x (4+4) plane; the global loads are issued one plane ahead into
  // registers and written to LDS after the barrier-free voxel work.
  constexpr int CPT = (NH + NT - 1) / NT;
  uint32_t cell_g[CPT];  // in-plane voxel index of each owned cell
  uint32_t cell_res = 0;  // 2 bits per owned cell: reservoir cell (open x faces)
  T2 pre_r[CPT];
  if (STENCIL) {
    if (tid < HX) {
      const int xu = x0 + tid - R;
      sxw[tid] = wrapn(xu, nx);
      sxg[tid] = mc.open_x ? (xu < 0 ? 1 : (xu >= nx ? 2 : 0)) : 0;
    }
    if (tid < HY) syw[tid] = wrapn(y0 + tid - R, ny);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int k = tid + q * NT;
      const int kk = k < NH ? k : 0;
      const int lx = kk % HX, ly = kk / HX;
      cell_g[q] = (uint32_t)sxw[lx] + (uint32_t)nx * (uint32_t)syw[ly];
      cell_res |= (uint32_t)sxg[lx] << (2 * q);
    }
  }
  auto fetch_rho = [&](int zz) {
    const uint32_t zoff = (uint32_t)wrapn(zz, nz) * nxy;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      if (tid + q * NT < NH) {
        const uint32_t rc = (cell_res >> (2 * q)) & 3u;
        if (rc == 0u) pre_r[q] = rho2[zoff + cell_g[q]];
        else pre_r[q] = rc == 1u ? T2{mc.rho_in[0], mc.rho_in[1]} : T2{mc.rho_out[0], mc.rho_out[1]};
      }
    }
  };
  auto store_rho = [&](int zz) {
    const int sl = rslot(zz);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int k = tid + q * NT;
      if (k < NH) {
        const T2 e = pre_r[q];
        srho[sl][k] = e;
        sshat[sl][k] = __builtin_isinf(e.x) ? (T)0 : (e.x * rcp(e.x + e.y) - mc.s_min) * mc.inv_span;
      }
    }
  };
  // staging of one reference plane (same pattern on the 66 x 6 normal tile)
  constexpr int CPE = (NM + NT - 1) / NT;
  uint32_t ecell_g[CPE];
  T2 pre_e[CPE];
  if (REFS) {
#pragma unroll
    for (int q = 0; q < CPE; ++q) {
      const int k = tid + q * NT;
      const int kk = k < NM ? k : 0;
      const int lx = kk % MX, ly = kk / MX;
      ecell_g[q] = (uint32_t)sxw[lx + 1] + (uint32_t)nx * (uint32_t)syw[ly + 1];
    }
  }
  auto fetch_ref = [&](int zz) {
    const uint32_t zoff = (uint32_t)wrapn(zz, nz) * nxy;
#pragma unroll
    for (int q = 0; q < CPE; ++q)
      if (tid + q * NT < NM) pre_e[q] = reinterpret_cast<const T2 *>(s.rhoE)[zoff + ecell_g[q]];
  };
  auto store_ref = [&](int zz) {
    const int sl = (zz + 3) % 3;
#pragma unroll
    for (int q = 0; q < CPE; ++q) {
      const int k = tid + q * NT;
      if (k < NM) sref[sl][k] = pre_e[q];
    }
  };

  // CSF normals of plane zz from the density planes zz-1 .. zz+1 (a solid
  // neighbour takes the cell's own density; solid cells get a zero normal)
  auto make_normals = [&](int zz) {
    const int sc0 = rslot(zz);
    for (int k = tid; k < NM; k += NT) {
      const int mx_ = k % MX, my_ = k / MX;
      const int c = (mx_ + 1) + HX * (my_ + 1);
      const T2 self = srho[sc0][c];
      const bool sol = __builtin_isinf(self.x);
      T gw0 = 0, gw1 = 0, gw2 = 0, go0 = 0, go1 = 0, go2 = 0;  // grad rho_w, grad rho_o
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const T2 e = srho[rslot(zz + cz(i))][c + hoff(i)];
        const bool ns = __builtin_isinf(e.x);
        const T vw = ns ? self.x : e.x;
        const T vo = ns ? self.y : e.y;
        if (cx(i)) { gw0 += (T)(gw(i) * cx(i)) * vw; go0 += (T)(gw(i) * cx(i)) * vo; }
        if (cy(i)) { gw1 += (T)(gw(i) * cy(i)) * vw; go1 += (T)(gw(i) * cy(i)) * vo; }
        if (cz(i)) { gw2 += (T)(gw(i) * cz(i)) * vw; go2 += (T)(gw(i) * cz(i)) * vo; }
      }
      // n^w follows grad rho_o, n^o follows grad rho_w
      const T qo = go0 * go0 + go1 * go1 + go2 * go2;
      const T qw = gw0 * gw0 + gw1 * gw1 + gw2 * gw2;
      const T io = qo > mc.eps_n2 ? rsq(qo) : (T)0;
      const T iw = qw > mc.eps_n2 ? rsq(qw) : (T)0;
      snrm[0][k] = sol ? T2{0, 0} : T2{go0 * io, gw0 * iw};
      snrm[1][k] = sol ? T2{0, 0} : T2{go1 * io, gw1 * iw};
      snrm[2][k] = sol ? T2{0, 0} : T2{go2 * io, gw2 * iw};
    }
  };

  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < nx && y < ny;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  // byte offsets of the 3 x 3 in-plane neighbours (x - 1 .. x + 1, y - 1 .. y + 1)
  uint32_t XYE[3][3];
#pragma unroll
  for (int bb = 0; bb < 3; ++bb)
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
      XYE[bb][aa] = ((uint32_t)(aa == 0 ? xm : (aa == 1 ? x : xp)) +
                     (uint32_t)(bb == 0 ? ym : (bb == 1 ? y : yp)) * (uint32_t)nx) * ES;
  const uint32_t vxy = (uint32_t)x + (uint32_t)y * (uint32_t)nx;  // in-plane voxel index
  const int c = (tx + R) + HX * (ty + R);
  const int cn = (tx + 1) + MX * (ty + 1);
  const T cs2 = (T)CS2;

  // Masks of this thread's voxel on planes z, z+1, z+2, and the CSF
  // curvature sums -div n^a of those planes, accumulated as the normal
  // planes arrive: the normals of plane p serve the voxels of planes p-1, p,
  // p+1 through the directions with c_z = p - (their plane); a solid link
  // takes the voxel's own normal.
  uint32_t M[3] = {0u, 0u, 0u};
  T Dw[3] = {0, 0, 0}, Do[3] = {0, 0, 0};
  auto mask_at = [&](int zz) -> uint32_t {
    return inside ? s.mask[vxy + (uint32_t)wrapn(zz, nz) * nxy] : 0u;
  };
  auto accum = [&](auto BASE) {  // BASE: plane of the normals minus z
    constexpr int base = decltype(BASE)::value;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int o = base - cz(i);  // target plane minus z
      if (o < 0 || o > 2) continue;
      const T k = ((M[o] >> i) & 1u) ? (T)0 : (T)gw(i);
      const int u = cn + moff(i);
      if (cx(i)) { const T2 n = snrm[0][u]; Dw[o] += k * (T)cx(i) * n.x; Do[o] += k * (T)cx(i) * n.y; }
      if (cy(i)) { const T2 n = snrm[1][u]; Dw[o] += k * (T)cy(i) * n.x; Do[o] += k * (T)cy(i) * n.y; }
      if (cz(i)) { const T2 n = snrm[2][u]; Dw[o] += k * (T)cz(i) * n.x; Do[o] += k * (T)cz(i) * n.y; }
    }
    if constexpr (base >= 0 && base <= 2) {
      const uint32_t mk = M[base];
      if (mk & 0x7fffeu) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const T on = ((mk >> i) & 1u) ? (T)gw(i) : (T)0;
          if (cx(i)) s0 += (T)cx(i) * on;
          if (cy(i)) s1 += (T)cy(i) * on;
          if (cz(i)) s2 += (T)cz(i) * on;
        }
        const T2 n0 = snrm[0][cn], n1 = snrm[1][cn], n2 = snrm[2][cn];
        Dw[base] += s0 * n0.x + s1 * n1.x + s2 * n2.x;
        Do[base] += s0 * n0.y + s1 * n1.y + s2 * n2.y;
      }
    }
  };
  auto advance = [&](int znext) {  // shift the windows to plane znext
    M[0] = M[1];
    M[1] = M[2];
    M[2] = mask_at(znext + 2);
    Dw[0] = Dw[1]; Dw[1] = Dw[2]; Dw[2] = 0;
    Do[0] = Do[1]; Do[1] = Do[2]; Do[2] = 0;
  };

  M[0] = mask_at(zs);
  M[1] = mask_at(zs + 1);
  M[2] = mask_at(zs + 2);
  if (STENCIL) {
    for (int zz = zs - 2; zz <= zs + 1; ++zz) {
      fetch_rho(zz);
      store_rho(zz);
    }
    if (REFS) {
      for (int zz = zs - 1; zz <= zs; ++zz) {
        fetch_ref(zz);
        store_ref(zz);
      }
    }
    __syncthreads();
    if (csf) {
      make_normals(zs - 1);
      __syncthreads();
      accum(std::integral_constant<int, -1>{});
      __syncthreads();
      make_normals(zs);
      __syncthreads();
      accum(std::integral_constant<int, 0>{});
    }
    fetch_rho(zs + 2);
    if (REFS) fetch_ref(zs + 1);
  }

  rsrc_t rin[NC], rout[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    rin[a] = make_rsrc((const char *)fin + (size_t)a * Q * NSTR * ES, (uint32_t)(Q * NSTR * ES));
    rout[a] = make_rsrc((char *)fout + (size_t)a * Q * NSTR * ES, (uint32_t)(Q * NSTR * ES));
  }

  // Fluid-only layout: the slot of a fluid voxel is the number of fluid voxels
  // before it.  A wave is one tile row, so the 64-voxel word of the rows
  // (y', z') it pulls from is the tile's (bx) and every row index is
  // wave-uniform (scalar loads); mbcnt counts the fluid voxels of the word
  // below this lane.  row_word gives the row's first word.
  const int tyu = __builtin_amdgcn_readfirstlane(ty);
  auto row_word = [&](int yy, int zq) -> uint32_t {
    return ((uint32_t)yy + (uint32_t)ny * (uint32_t)zq) * (uint32_t)s.cw;
  };
  // slot of x + dx (|dx| <= 1, a fluid voxel) in the row starting at word k
  // (the tables are read-only here: constant address space, scalar loads)
  using cu64 = __attribute__((address_space(4))) const uint64_t;
  using cu32 = __attribute__((address_space(4))) const uint32_t;
  cu64 *const cmask = (cu64 *)s.cmask;
  cu32 *const cbase = (cu32 *)s.cbase;
  auto slot_at = [&](int dx, uint32_t k) -> uint32_t {
    const uint64_t m = cmask[k + bx];
    const uint32_t cb = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, cbase[k + bx]));
    if (dx == 0) return cb;
    if (dx < 0) return x == 0 ? cbase[k + s.cw] - 1u : cb - 1u;  // (x = 0: the row's last voxel)
    return x == nx - 1 ? cbase[k] : cb + (uint32_t)((m >> tx) & 1ull);  // (the row's first)
  };


  // The pull of plane z+1 is issued while plane z computes, so each wave keeps
  // its next plane's loads in flight (and ahead of its own stores).
  using LT = typename std::conditional<S16, uint32_t, T>::type;
  LT pf[NC][Q];
  auto issue = [&](int zz, uint32_t mkz) {
    const uint32_t zo = (uint32_t)zz * nxy;
    const uint32_t vv = vxy + zo;
    const int zm1 = zz == 0 ? nz - 1 : zz - 1, zp1 = zz == nz - 1 ? 0 : zz + 1;
    const uint32_t NE = NSTR * ES;
    const uint32_t ZE[3] = {(uint32_t)zm1 * nxy * ES, zo * ES, (uint32_t)zp1 * nxy * ES};
    const int yu = y0 + tyu;
    const int Yr[3] = {yu == 0 ? ny - 1 : yu - 1, yu, yu == ny - 1 ? 0 : yu + 1};
    const int Zr[3] = {zm1, zz, zp1};
    const uint32_t vE = CMP ? slot_at(0, row_word(yu, zz)) * ES : vv * ES;
    // a solid voxel's pulls are never used: its lane loads nothing
    if (((mkz >> CLASS_SHIFT) & 3u) == SOLID_CODE) {
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int i = 0; i < Q; ++i) pf[a][i] = (LT)0;
      return;
    }
    LBM_DCHECK((uint64_t)vE + ES <= (uint64_t)Q * NSTR * ES && vv < N32, DC_PULL);
#pragma unroll
    for (int a = 0; a < NC; ++a) pf[a][0] = pull_raw_s<T, SK>(rin[a], vE, 0u);
    // pair (i, j = i + 1) of opposite directions, both addressed from the
    // scalar start i N of array i: pull source of i is x - c_i (array i), of
    // j is x + c_i (array j = i + 1, one N further); bounce-back takes the
    // opposite population of this voxel when the source is solid
    uint32_t so = NE;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const int j = i + 1;
      uint32_t si, sj;  // source offsets of i and j
      if constexpr (CMP) {
        si = slot_at(-cx(i), row_word(Yr[1 - cy(i)], Zr[1 - cz(i)])) * ES;
        sj = slot_at(cx(i), row_word(Yr[1 + cy(i)], Zr[1 + cz(i)])) * ES;
      } else {
        si = XYE[1 - cy(i)][1 - cx(i)] + ZE[1 - cz(i)];
        sj = XYE[1 + cy(i)][1 + cx(i)] + ZE[1 + cz(i)];
      }
      const uint32_t oi = ((mkz >> j) & 1u) ? vE + NE : si;
      const uint32_t oj = ((mkz >> i) & 1u) ? vE : sj + NE;
      LBM_DCHECK((uint64_t)oi + so + ES <= (uint64_t)Q * NSTR * ES &&
                     (uint64_t)oj + so + ES <= (uint64_t)Q * NSTR * ES,
                 DC_PULL);
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        pf[a][i] = pull_raw_s<T, SK>(rin[a], oi, so);
        pf[a][j] = pull_raw_s<T, SK>(rin[a], oj, so);
      }
      so += 2 * NE;
      keep_scalar(so);
    }
  };
  auto all_solid = [](uint32_t mkz) { return __all(((mkz >> CLASS_SHIFT) & 3u) == SOLID_CODE); };
  if (inside && !all_solid(M[0])) issue(zs, M[0]);
  // pushed densities of planes z - 1, z, z + 1 at this thread's column
  T Pp[NC], Pc[NC], Pn[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) Pp[a] = Pc[a] = Pn[a] = (T)0;
  uint32_t Mlast = 0u;

  for (int z = zs; z < ze; advance(++z)) {
    if (STENCIL) {
      // plane z+2 reuses the slot of plane z-3, which no wave still reads;
      // the barrier also ends every read of the previous normal plane
      store_rho(z + 2);
      __syncthreads();
      if (REFS) {
        // plane z+1 takes the slot of plane z-2, whose last reader (plane
        // z-1's pulls) finished before the barrier above; the next barrier
        // orders it before this plane's pulls
        store_ref(z + 1);
        if (!csf) __syncthreads();
      }
      if (csf) {
        make_normals(z + 1);
        __syncthreads();
        accum(std::integral_constant<int, 1>{});
      }
      if (z + 1 < ze) {
        fetch_rho(z + 3);
        if (REFS) fetch_ref(z + 2);
      }
    }
    // The push of the next level's densities: every post-collision value goes
    // to the voxel that will pull it (x + c_i), or stays here when x + c_i is
    // solid (bounce-back).  Links within this tile and chunk that do not wrap
    // around the grid are summed here: along x by lane shifts, across rows
    // through LDS, across planes in registers (Pp, Pc, Pn hold the planes
    // z - 1, z, z + 1 of this thread's column).  k_density_fix adds the
    // links leaving the tile or chunk, or wrapping, after the step.
    // gself, gzp, gzm: this component's values for planes z, z + 1, z - 1
    // from this row (after the lane shifts); the values for the rows above
    // and below go to LDS ([row][tx][c_z + 1][a]), which reuses the normals'
    // space: the barrier below ends every read of the normals of this plane.
    T gself[PUSH ? NC : 1], gzp[PUSH ? NC : 1], gzm[PUSH ? NC : 1];
    T *const my_up = spush_up + (ty < TY - 1 ? ty : 0) * PUSH_ROW + tx * 3 * NC;
    T *const my_dn = spush_dn + (ty >= 1 ? ty - 1 : 0) * PUSH_ROW + tx * 3 * NC;
    auto push_zero = [&]() {
#pragma unroll
      for (int k = 0; k < 3 * NC; ++k) {
        if (ty < TY - 1) my_up[k] = (T)0;
        if (ty >= 1) my_dn[k] = (T)0;
      }
    };
    if constexpr (PUSH) {
#pragma unroll
      for (int a = 0; a < NC; ++a) gself[a] = gzp[a] = gzm[a] = (T)0;
      if (csf) __syncthreads();
    }
    auto push_comp = [&](int a, const T *pvv, uint32_t mkp) {
      const bool ox_p = tx + 1 < TX && x + 1 < nx, ox_m = tx >= 1;
      const bool oy_p = ty + 1 < TY && y + 1 < ny, oy_m = ty >= 1;
      const bool oz_p = z + 1 < ze, oz_m = z - 1 >= zs;
      T own = pvv[0];
      auto take = [&](int i, bool ok) -> T {
        if ((mkp >> i) & 1u) {  // x + c_i solid: it comes back here
          own += pvv[i];
          return (T)0;
        }
        return ok ? pvv[i] : (T)0;
      };
      // lane tx takes the +x values of lane tx - 1 and the -x values of lane
      // tx + 1 (lanes beyond the grid's last column left the voxel work, so
      // their lane is never read)
      const bool rl = tx >= 1, rr = tx + 1 < TX && x + 1 < nx;
      auto from_left = [&](T val) -> T {
        const T r = __shfl_up(val, 1);
        return rl ? r : (T)0;
      };
      auto from_right = [&](T val) -> T {
        const T r = __shfl_down(val, 1);
        return rr ? r : (T)0;
      };
      // one class (c_y, c_z) at a time: its c_x = 0 value plus the +x value
      // of the lane to the left and the -x value of the lane to the right
      auto cls3 = [&](int i0_, int ip, int im, bool ok) -> T {
        const T c0 = take(i0_, ok);
        const T l = from_left(take(ip, ok && ox_p));
        const T r = from_right(take(im, ok && ox_m));
        return c0 + l + r;
      };
      const T gyp = cls3(3, 7, 10, oy_p);  // (., +1, 0)
      const T gym = cls3(4, 9, 8, oy_m);   // (., -1, 0)
      if (ty < TY - 1) {  // the top row's up values are zero: they leave the tile
        my_up[0 * NC + a] = take(17, oy_p && oz_m);  // (0, +1, -1)
        my_up[1 * NC + a] = gyp;
        my_up[2 * NC + a] = take(15, oy_p && oz_p);  // (0, +1, +1)
      } else {
        (void)take(17, false);
        (void)take(15, false);
      }
      if (ty >= 1) {  // the bottom row's down values likewise
        my_dn[0 * NC + a] = take(16, oy_m && oz_m);  // (0, -1, -1)
        my_dn[1 * NC + a] = gym;
        my_dn[2 * NC + a] = take(18, oy_m && oz_p);  // (0, -1, +1)
      } else {
        (void)take(16, false);
        (void)take(18, false);
      }
      gzp[a] = cls3(5, 11, 14, oz_p);  // (., 0, +1)
      gzm[a] = cls3(6, 13, 12, oz_m);  // (., 0, -1)
      const T gx = from_left(take(1, ox_p)) + from_right(take(2, ox_m));  // (., 0, 0)
      gself[a] = own + gx;
    };
    do {
    if (!inside) {
      if constexpr (PUSH) push_zero();
      break;
    }
    const uint32_t zoff = (uint32_t)z * nxy;
    const uint32_t v = vxy + zoff;
    LBM_DCHECK(v < N32 && x < nx && y < ny, DC_VOXEL);
    const uint32_t mk = M[0];
    const uint32_t cl = (mk >> CLASS_SHIFT) & 3u;
    // Solid lanes of a wave that also holds fluid voxels run along (their
    // results are discarded).  In the dense layout they store zeros, so that
    // every population store of the wave writes whole cache lines instead of
    // partial ones; in the fluid-only layout they have no slot and store
    // nothing.
    const bool solid = cl == SOLID_CODE;
    const bool skip = all_solid(mk);
    const bool skip_next = z + 1 >= ze || all_solid(M[1]);
    const bool gray = cl == GRAY_CODE;

    // a1 + a2: the pulled populations of this plane (bounce-back resolved at
    // issue) summed into moments over opposite pairs.  16-bit storage: each
    // pulled offset decodes with the reference density of the voxel it came
    // from (this voxel's own under bounce-back), g = ref + h = f_i / w_i.
    T rho[NC], mom[NC][3], P[NC][6];  // P: xx, yy, zz, xy, xz, yz
    T f[REG ? 1 : NC][REG ? 1 : Q];   // BGK: f_i (native) or f_i / w_i (16-bit)
    if (!skip) {
      // reference planes z-1, z, z+1 in the ring, and this voxel's references
      const int es[3] = {(z + 2) % 3, z % 3, (z + 1) % 3};
      T2 Ro2 = T2{(T)1, (T)1};
      if (REFS) Ro2 = sref[es[1]][cn];
      const T Ro[2] = {Ro2.x, Ro2.y};
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        T g0 = pull_decode<T, SK>(pf[a][0]);
        if (S16) g0 += Ro[a];
        if (!REG) f[REG ? 0 : a][0] = g0;
        rho[a] = S16 ? (T)(1.0 / 3.0) * g0 : g0;
        mom[a][0] = mom[a][1] = mom[a][2] = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) P[a][d] = 0;
      }
#pragma unroll
      for (int i = 1; i < Q; i += 2) {
        const int j = i + 1;
        // pull of i from x - c_i, of j from x + c_i; bounce-back when solid
        const bool bbi = (mk >> j) & 1u, bbj = (mk >> i) & 1u;
        // 16-bit: the references of both sources, both components in one read
        T2 Ri2 = Ro2, Rj2 = Ro2;
        if (REFS) {
          if (!bbi) Ri2 = sref[es[1 - cz(i)]][cn - moff(i)];
          if (!bbj) Rj2 = sref[es[1 + cz(i)]][cn + moff(i)];
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          T fi = pull_decode<T, SK>(pf[a][i]);
          T fj = pull_decode<T, SK>(pf[a][j]);
          if (S16) {
            fi += a == 0 ? Ri2.x : Ri2.y;
            fj += a == 0 ? Rj2.x : Rj2.y;
          }
          if (!REG) {
            f[REG ? 0 : a][i] = fi;
            f[REG ? 0 : a][j] = fj;
          }
          if (S16) {
            const T w = i < 7 ? (T)(1.0 / 18.0) : (T)(1.0 / 36.0);
            fi *= w;
            fj *= w;
          }
          const T sm = fi + fj, df = fi - fj;
          rho[a] += sm;
          if (cx(i)) { mom[a][0] += cx(i) > 0 ? df : -df; P[a][0] += sm; }
          if (cy(i)) { mom[a][1] += cy(i) > 0 ? df : -df; P[a][1] += sm; }
          if (cz(i)) { mom[a][2] += cz(i) > 0 ? df : -df; P[a][2] += sm; }
          if (cx(i) && cy(i)) P[a][3] += cx(i) * cy(i) > 0 ? sm : -sm;
          if (cx(i) && cz(i)) P[a][4] += cx(i) * cz(i) > 0 ? sm : -sm;
          if (cy(i) && cz(i)) P[a][5] += cy(i) * cz(i) > 0 ? sm : -sm;
        }
      }
    }
    if (!skip_next) issue(z + 1, M[1]);
    if (skip) {
      if constexpr (PUSH) push_zero();
      break;
    }
    T rt = rho[0];
    if (NC == 2) rt = rho[0] + rho[1];
    const T irt = rcp(rt);

    T Fex[NC][3];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) Fex[a][d] = rho[a] * mc.g[a][d];

    T S = 1, rw_res = 0, ro_res = 0, rhoT = rt, cR = 0;
    if (NC == 2) {
      if (gray) {
        rw_res = s.r[v];
        ro_res = s.r[N + v];
      }
      const T tw = rho[0] + rw_res, to = rho[1] + ro_res;
      rhoT = tw + to;
      S = (tw * rcp(rhoT) - mc.s_min) * mc.inv_span;
      S = S < (T)0 ? (T)0 : (S > (T)1 ? (T)1 : S);
      // a3: pseudo-potential sums acc_b = sum_i w_i c_i psi_b(x + c_i); a solid
      // neighbour enters with the local density plus the wetting offset
      T pw[2];
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) {
        const T p_ = rho[bb] + mc.wall_dpsi[bb];
        pw[bb] = p_ > (T)0 ? p_ : (T)0;
      }
      T aw0 = 0, aw1 = 0, aw2 = 0, ao0 = 0, ao1 = 0, ao2 = 0;
      // 16-bit storage: the reference part sum_i w_i rho_ref(s_i) of the next
      // level's densities (this level's densities are the next references;
      // a solid neighbour means bounce-back, whose writer is this voxel)
      const T2 eown = srho[rslot(z)][c];
      T qw = (T)(1.0 / 3.0) * eown.x, qo = (T)(1.0 / 3.0) * eown.y;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const T2 e = srho[rslot(z + cz(i))][c + hoff(i)];
        const bool sol = (mk >> i) & 1u;
        const T vw = sol ? pw[0] : e.x;
        const T vo = sol ? pw[1] : e.y;
        if (cx(i)) { aw0 += (T)(wq(i) * cx(i)) * vw; ao0 += (T)(wq(i) * cx(i)) * vo; }
        if (cy(i)) { aw1 += (T)(wq(i) * cy(i)) * vw; ao1 += (T)(wq(i) * cy(i)) * vo; }
        if (cz(i)) { aw2 += (T)(wq(i) * cz(i)) * vw; ao2 += (T)(wq(i) * cz(i)) * vo; }
        if (S16 && !PUSH) {
          qw += (T)wq(i) * (sol ? eown.x : e.x);
          qo += (T)wq(i) * (sol ? eown.y : e.y);
        }
      }
      if (S16 && !PUSH) reinterpret_cast<T2 *>(s.rhoS)[v] = T2{qw, qo};
      {
        const T kw = -mc.G * rho[0], ko = -mc.G * rho[1];
        Fex[0][0] += kw * ao0; Fex[0][1] += kw * ao1; Fex[0][2] += kw * ao2;
        Fex[1][0] += ko * aw0; Fex[1][1] += ko * aw1; Fex[1][2] += ko * aw2;
      }
      // a3: CSF surface-tension control, Eq. (4).  The Neumann gradient of
      // rho_b differs from 3 acc_b only through the solid links.
      if (csf && (gray || mc.csf_all)) {
        T sw0 = 0, sw1 = 0, sw2 = 0;  // sum over solid links of w_i c_i
        if (mk & 0x7fffeu) {
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const T on = ((mk >> i) & 1u) ? (T)wq(i) : (T)0;
            if (cx(i)) sw0 += (T)cx(i) * on;
            if (cy(i)) sw1 += (T)cy(i) * on;
            if (cz(i)) sw2 += (T)cz(i) * on;
          }
        }
        const T dw = pw[0] - rho[0], dox = pw[1] - rho[1];
        const T grw0 = (T)3 * (aw0 - dw * sw0), grw1 = (T)3 * (aw1 - dw * sw1),
                grw2 = (T)3 * (aw2 - dw * sw2);
        const T gro0 = (T)3 * (ao0 - dox * sw0), gro1 = (T)3 * (ao1 - dox * sw1),
                gro2 = (T)3 * (ao2 - dox * sw2);
        const T dvw = Dw[0], dvo = Do[0];  // div n^w, div n^o
        // F_csf^a = kappa (-div n^a) grad rho^b rho^a / (phi_avg phi_max)
        const T kw = -mc.csf_fac * dvw * rho[0], ko = -mc.csf_fac * dvo * rho[1];
        Fex[0][0] += kw * gro0; Fex[0][1] += kw * gro1; Fex[0][2] += kw * gro2;
        Fex[1][0] += ko * grw0; Fex[1][1] += ko * grw1; Fex[1][2] += ko * grw2;
      }
      // a4: capillary term of Eq. (1) and the resistance coefficient
      if (gray) {
        const T shat0 = (rho[0] * irt - mc.s_min) * mc.inv_span;
        T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const T val = ((mk >> i) & 1u) ? shat0 : sshat[rslot(z + cz(i))][c + hoff(i)];
          if (cx(i)) g0 += (T)(gw(i) * cx(i)) * val;
          if (cy(i)) g1 += (T)(gw(i) * cy(i)) * val;
          if (cz(i)) g2 += (T)(gw(i) * cz(i)) * val;
        }
        const int t = s.ptype[v];
        const T *tb = s.tab + (size_t)t * 3 * TABLE_N;
        const T Pc = s.sJ[v] * lerp_tab<T>(tb, S);
        const T krw = lerp_tab<T>(tb + TABLE_N, S);
        const T kro = lerp_tab<T>(tb + 2 * TABLE_N, S);
        const T kw = -Pc * rho[0] * irt, ko = -Pc * rho[1] * irt;
        Fex[0][0] += kw * g0; Fex[0][1] += kw * g1; Fex[0][2] += kw * g2;
        Fex[1][0] += ko * g0; Fex[1][1] += ko * g1; Fex[1][2] += ko * g2;
        const T Sw = S, So = (T)1 - S;
        const T krmin = mc.kr_min;
        const T cw = Sw > (T)0 ? rt * Sw * mc.nu[0] * rcp(krw > krmin ? krw : krmin) : (T)0;
        const T co = So > (T)0 ? rt * So * mc.nu[1] * rcp(kro > krmin ? kro : krmin) : (T)0;
        cR = cw + co;
      }
    } else if (gray) {
      cR = rt * mc.nu[0];
    }

    // a5: velocity the resistance acts on, u = (rho I + R/2)^-1 (m + sum F_ex / 2)
    // (trapezoidal rule)
    const T h = (T)0.5;
    T b0 = 0, b1 = 0, b2 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      b0 += mom[a][0]; b1 += mom[a][1]; b2 += mom[a][2];
      e0 += Fex[a][0]; e1 += Fex[a][1]; e2 += Fex[a][2];
    }
    b0 = b0 + h * e0;
    b1 = b1 + h * e1;
    b2 = b2 + h * e2;
    T Ru0 = 0, Ru1 = 0, Ru2 = 0;
    if (gray && mc.tensor) {
      const T *K = s.Kinv;
      const T Rxx = cR * K[v], Ryy = cR * K[N + v], Rzz = cR * K[2 * N + v];
      const T Rxy = cR * K[3 * N + v], Rxz = cR * K[4 * N + v], Ryz = cR * K[5 * N + v];
      const T a00 = rt + h * Rxx, a11 = rt + h * Ryy, a22 = rt + h * Rzz;
      const T a01 = h * Rxy, a02 = h * Rxz, a12 = h * Ryz;
      const T c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22,
              c02 = a01 * a12 - a02 * a11;
      const T c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12,
              c22 = a00 * a11 - a01 * a01;
      const T idet = rcp(a00 * c00 + a01 * c01 + a02 * c02);
      const T u0 = (c00 * b0 + c01 * b1 + c02 * b2) * idet;
      const T u1 = (c01 * b0 + c11 * b1 + c12 * b2) * idet;
      const T u2 = (c02 * b0 + c12 * b1 + c22 * b2) * idet;
      Ru0 = Rxx * u0 + Rxy * u1 + Rxz * u2;
      Ru1 = Rxy * u0 + Ryy * u1 + Ryz * u2;
      Ru2 = Rxz * u0 + Ryz * u1 + Rzz * u2;
    } else if (gray) {
      const T Rs = cR * rcp(s.K0[v]);
      const T q = Rs * rcp(rt + h * Rs);
      Ru0 = q * b0;
      Ru1 = q * b1;
      Ru2 = q * b2;
    }

    // a6: Shan-Chen common velocity u'
    T den = 0, up0 = 0, up1 = 0, up2 = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const T om = mc.omega[a];
      den += rho[a] * om;
      up0 += mom[a][0] * om; up1 += mom[a][1] * om; up2 += mom[a][2] * om;
    }
    const T iden = rcp(den);
    up0 *= iden; up1 *= iden; up2 *= iden;
    const T usq = up0 * up0 + up1 * up1 + up2 * up2;

    // a7: residual transfer (gray voxels) as per-component scale factors
    T scale[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) scale[a] = 1;
    if (NC == 2 && gray) {
      const uint8_t sd = s.side[v];
      const T hy = mc.hyst;
      const T m = mc.m_minor;
      if (!sd && S >= (T)0.5 + hy) {
        scale[0] = (rho[0] + rw_res) / rho[0];
        T d = s.tho[v] * rhoT - ro_res;
        const T cap = rho[NC - 1] - m;
        d = d < cap ? d : cap;
        d = d > (T)0 ? d : (T)0;
        scale[NC - 1] = (T)1 - d / rho[NC - 1];
        s.r[v] = 0;
        s.r[N + v] = ro_res + d;
        s.side[v] = 1;
      } else if (sd && S <= (T)0.5 - hy) {
        scale[NC - 1] = (rho[NC - 1] + ro_res) / rho[NC - 1];
        T d = s.thw[v] * rhoT - rw_res;
        const T cap = rho[0] - m;
        d = d < cap ? d : cap;
        d = d > (T)0 ? d : (T)0;
        scale[0] = (T)1 - d / rho[0];
        s.r[N + v] = 0;
        s.r[v] = rw_res + d;
        s.side[v] = 0;
      }
    }

    // a6: collision + force term (Eq. (3)) as quadratic forms.  Pore voxels:
    // equilibrium at u' and Eq. (3) at ua = u' + F^a / (2 rho^a) (the exact
    // difference).  Gray voxels: Eq. (3) in its second-order form, the
    // equilibrium and the non-equilibrium part at ua and the force term
    // weighted by 1 - omega/2, so that the resistance force (R >> rho) stays
    // out of the equilibrium's quadratic terms.
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const T ra = rho[a];
      const T kr = ra * irt;
      const T Fa0 = Fex[a][0] - kr * Ru0, Fa1 = Fex[a][1] - kr * Ru1, Fa2 = Fex[a][2] - kr * Ru2;
      const T ih2 = (T)0.5 * rcp(ra);
      const T ua0 = up0 + Fa0 * ih2, ua1 = up1 + Fa1 * ih2, ua2 = up2 + Fa2 * ih2;
      const T om = mc.omega[a];
      const T keep = (T)1 - om;
      // equilibrium velocity ve and force weight kf
      const T ve0 = gray ? ua0 : up0, ve1 = gray ? ua1 : up1, ve2 = gray ? ua2 : up2;
      const T kf = gray ? (T)1 - (T)0.5 * om : (T)1;
      const T vsq = gray ? ua0 * ua0 + ua1 * ua1 + ua2 * ua2 : usq;
      const T kF0 = kf * Fa0, kF1 = kf * Fa1, kF2 = kf * Fa2;
      const T uF = ua0 * kF0 + ua1 * kF1 + ua2 * kF2;
      const T we = REG ? (T)1 : om;  // weight of the equilibrium part
      const T wr = we * ra;
      T A = wr * ((T)1 - (T)1.5 * vsq) - (T)3 * uF;
      T B0 = (T)3 * (wr * ve0 + kF0);
      T B1 = (T)3 * (wr * ve1 + kF1);
      T B2 = (T)3 * (wr * ve2 + kF2);
      const T er = (T)4.5 * wr;
      T Cxx = er * ve0 * ve0 + (T)9 * ua0 * kF0;
      T Cyy = er * ve1 * ve1 + (T)9 * ua1 * kF1;
      T Czz = er * ve2 * ve2 + (T)9 * ua2 * kF2;
      T Cxy = er * ve0 * ve1 + (T)4.5 * (ua0 * kF1 + ua1 * kF0);
      T Cxz = er * ve0 * ve2 + (T)4.5 * (ua0 * kF2 + ua2 * kF0);
      T Cyz = er * ve1 * ve2 + (T)4.5 * (ua1 * kF2 + ua2 * kF1);
      if (REG) {
        // projected non-equilibrium part: j - rho ve, Pi - rho (cs2 I + ve ve)
        const T jn0 = mom[a][0] - ra * ve0, jn1 = mom[a][1] - ra * ve1, jn2 = mom[a][2] - ra * ve2;
        const T qxx = P[a][0] - ra * (cs2 + ve0 * ve0);
        const T qyy = P[a][1] - ra * (cs2 + ve1 * ve1);
        const T qzz = P[a][2] - ra * (cs2 + ve2 * ve2);
        const T qxy = P[a][3] - ra * ve0 * ve1;
        const T qxz = P[a][4] - ra * ve0 * ve2;
        const T qyz = P[a][5] - ra * ve1 * ve2;
        const T k3 = (T)3 * keep, k45 = (T)4.5 * keep;
        A -= (T)1.5 * keep * (qxx + qyy + qzz);
        B0 += k3 * jn0; B1 += k3 * jn1; B2 += k3 * jn2;
        Cxx += k45 * qxx; Cyy += k45 * qyy; Czz += k45 * qzz;
        Cxy += k45 * qxy; Cxz += k45 * qxz; Cyz += k45 * qyz;
      }
      const T sc = NC == 2 ? scale[a] : (T)1;
      T pv[PUSH ? Q : 1];  // the values written (the push's input)
      LBM_DCHECK(CMP || (uint64_t)(vxy + zoff) * ES + (uint64_t)(Q - 1) * N32 * ES + ES <=
                            (uint64_t)Q * N32 * ES,
                 DC_STORE);
      if constexpr (CMP) {
        emit_post<T, REG, PUSH, true>(rout[a], slot_at(0, row_word(y0 + tyu, z)) * ES, 0u,
                                      NSTR * ES, A, B0, B1, B2, Cxx, Cyy, Czz, Cxy, Cxz, Cyz, sc,
                                      f[REG ? 0 : a], keep, solid, pv);
      } else if constexpr (!S16) {
        emit_post<T, REG, PUSH>(rout[a], vxy * ES, zoff * ES, N32 * ES, A, B0, B1, B2, Cxx, Cyy,
                                Czz, Cxy, Cxz, Cyz, sc, f[REG ? 0 : a], keep, solid, pv);
      } else {
        // reference of every outgoing slot: this voxel's density of this
        // level (exactly the value the density pass wrote, which becomes the
        // readers' reference array)
        const float ref = NC == 2 ? reinterpret_cast<const float *>(&srho[rslot(z)][c])[a] : 1.f;
        emit_post16<SK, REG, PUSH>(rout[a], vxy * 2u, zoff * 2u, N32 * 2u, A, B0, B1, B2, Cxx,
                                   Cyy, Czz, Cxy, Cxz, Cyz, sc, f[REG ? 0 : a], keep, solid, ref,
                                   reinterpret_cast<float *>(pv));
      }
      if constexpr (PUSH) push_comp(a, pv, mk);
    }
    } while (0);

    if constexpr (PUSH) {
      __syncthreads();
      // row y - 1's up values and row y + 1's down values
      const T *below = spush_up + (ty >= 1 ? ty - 1 : 0) * PUSH_ROW + tx * 3 * NC;
      const T *above = spush_dn + (ty + 1 < TY ? ty : 0) * PUSH_ROW + tx * 3 * NC;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        T r[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T ru = ty >= 1 ? below[k * NC + a] : (T)0;
          const T rd = ty + 1 < TY ? above[k * NC + a] : (T)0;
          r[k] = ru + rd;
        }
        Pc[a] += gself[a] + r[1];
        Pn[a] += gzp[a] + r[2];
        Pp[a] += gzm[a] + r[0];
      }
      const uint32_t mkp = inside ? M[0] : 0u;
      // plane z - 1 has all its in-tile contributions now
      if (inside && z - 1 >= zs) {
        const bool sol = ((Mlast >> CLASS_SHIFT) & 3u) == SOLID_CODE;
        reinterpret_cast<T2 *>(s.rho2n)[(size_t)vxy + (size_t)(z - 1) * nxy] =
            sol ? T2{(T)INFINITY, (T)INFINITY} : T2{Pp[0], Pp[NC - 1]};
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        Pp[a] = Pc[a];
        Pc[a] = Pn[a];
        Pn[a] = (T)0;
      }
      Mlast = mkp;
    }
  }
  if constexpr (PUSH) {
    if (inside) {  // the chunk's last plane: the next chunk's first plane adds to it in k_density_fix
      const bool sol = ((Mlast >> CLASS_SHIFT) & 3u) == SOLID_CODE;
      reinterpret_cast<T2 *>(s.rho2n)[(size_t)vxy + (size_t)(ze - 1) * nxy] =
          sol ? T2{(T)INFINITY, (T)INFINITY} : T2{Pp[0], Pp[NC - 1]};
    }
  }
}

// The next level's densities, second part.  With the push, the fused step
// summed every link whose two ends lie in one tile and one z chunk without
// crossing the periodic wrap; this adds the values of the other links, read
// back from the new set exactly as the next step will pull them (16-bit
// storage: w_i (rho_ref(s) + h), rho_ref(s) the writer's density of the
// level just left, `rref`), so that each density is the sum of the voxel's
// next pulls.  Only voxels on a face of a tile or chunk have such links, and
// a solid source means bounce-back, which the step summed at the voxel itself.
// CMP: the new set is in the fluid-only layout (L); solid sources have no
// slot and are not read.
template <typename T, int SK, bool CMP = false>
__global__ __launch_bounds__(256) void k_density_fix(const void *__restrict__ fnew,
                                                     T *__restrict__ rho2n,
                                                     const T *__restrict__ rref,
                                                     const uint32_t *__restrict__ mask, int nx,
                                                     int ny, int nz, int zc, long long N,
                                                     const PopLayout L) {
  using namespace zm;
  const uint32_t v = blockIdx.x * 256u + threadIdx.x;
  if (v >= (uint32_t)N) return;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const int z = (int)(v / nxy);
  const uint32_t rem = v - (uint32_t)z * nxy;
  const int y = (int)(rem / (uint32_t)nx);
  const int x = (int)(rem - (uint32_t)y * (uint32_t)nx);
  const int tx = x % TX, ty = y % TY, tz = z % zc;
  const bool face = tx == 0 || tx == TX - 1 || x == nx - 1 || ty == 0 || ty == TY - 1 ||
                    y == ny - 1 || tz == 0 || tz == zc - 1 || z == nz - 1;
  if (!face) return;
  // which links leave the step's reach follows from the position alone: a
  // source beyond the grid (the wrap) or in another tile or chunk along some
  // axis.  Their loads, the mask and the partial density are all issued
  // before any of them is used (one memory round trip per wave).
  auto cut = [](int src, int dst, int n, int t) { return src < 0 || src >= n || src / t != dst / t; };
  const uint32_t mk = mask[v];
  if (CMP && ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  const vec2<T> part = reinterpret_cast<const vec2<T> *>(rho2n)[v];
  T val[Q - 1][2];
  uint32_t need = 0u;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int xs = x - cx(i), ys = y - cy(i), zs = z - cz(i);
    const bool cross = (cx(i) != 0 && cut(xs, x, nx, TX)) || (cy(i) != 0 && cut(ys, y, ny, TY)) ||
                       (cz(i) != 0 && cut(zs, z, nz, zc));
    val[i - 1][0] = val[i - 1][1] = (T)0;
    if (!cross) continue;
    need |= 1u << i;
    if (CMP && ((mk >> opp(i)) & 1u)) continue;  // solid source: no slot
    const uint32_t sv = (uint32_t)(xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs)) +
                        (uint32_t)(ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys)) * (uint32_t)nx +
                        (uint32_t)(zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs)) * nxy;
    const size_t ss = CMP ? (size_t)L.slot(sv, nx) : (size_t)sv;
    LBM_DCHECK(sv < (uint32_t)N && ss < (size_t)(CMP ? L.stride : N), DC_FIX);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const size_t k = (size_t)(a * Q + i) * (size_t)(CMP ? L.stride : N) + ss;
      if constexpr (SK == SK_NATIVE) {
        val[i - 1][a] = reinterpret_cast<const T *>(fnew)[k];
      } else {
        const uint16_t code = reinterpret_cast<const uint16_t *>(fnew)[k];
        val[i - 1][a] = (float)wq(i) * (rref[2 * (size_t)sv + a] + dec16<SK>(code));
      }
    }
  }
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  // a solid source means bounce-back, which the step summed at the voxel itself
  T add[2] = {(T)0, (T)0};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!((need >> i) & 1u) || ((mk >> opp(i)) & 1u)) continue;
    add[0] += val[i - 1][0];
    add[1] += val[i - 1][1];
  }
  if (need) {
    vec2<T> r = part;
    r.x += add[0];
    r.y += add[1];
    reinterpret_cast<vec2<T> *>(rho2n)[v] = r;
  }
}

// ---------------------------------------------------------------------------
// 16-bit storage: conversions between the stored offsets and fp32 populations
// (field evaluation, initialisation) and the per-step outlet flux.

// Reference density of component a of the slots stored at voxel v: the
// density of v (their writer) at the level they were written.
__device__ inline float writer_ref(const float *rhoE, long long v, int a, int nc) {
  return nc == 1 ? 1.f : rhoE[2 * v + a];
}

// stored offsets (slot layout) -> fp32 populations f = w_i (rho_ref + h)
// (open x faces: a solid voxel on a face also decodes its slots that the
// voxels across the face pull)
template <int SK>
__global__ __launch_bounds__(256) void k_decode(const uint16_t *__restrict__ codes,
                                                const float *__restrict__ rhoE,
                                                const uint32_t *__restrict__ mask,
                                                float *__restrict__ out, int nx, int ny, int nz,
                                                long long N, int nc, int open_x) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const uint32_t mk = mask[v];
  const bool solid = ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  const int x = (int)(v % nx);
  for (int a = 0; a < nc; ++a) {
    const float ref = writer_ref(rhoE, v, a, nc);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const size_t k = (size_t)(a * Q + i) * N + v;
      const bool crossing = open_x && cx(i) != 0 && (x + cx(i) < 0 || x + cx(i) >= nx);
      float val = 0.f;
      if (!solid || crossing) val = (float)wq(i) * (ref + dec16<SK>(codes[k]));
      out[k] = val;
    }
  }
}

// reference densities of a canonical (post-streaming) fp32 set: rho = sum_i f_i
__global__ __launch_bounds__(256) void k_ref_canonical(const float *__restrict__ C,
                                                       float *__restrict__ rhoE,
                                                       const uint32_t *__restrict__ mask,
                                                       long long N) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const bool solid = ((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  for (int a = 0; a < 2; ++a) {
    float r = 0.f;
    if (!solid) {
#pragma unroll
      for (int i = 0; i < Q; ++i) r += C[(size_t)(a * Q + i) * N + v];
    }
    rhoE[2 * v + a] = r;
  }
}

// canonical fp32 set -> stored offsets (the streaming of k_scatter, encoded
// against the reader's reference)
// (open x faces: a solid voxel on a face also stores the slots that a fluid
// voxel across the face pulls, as k_scatter does)
template <int SK>
__global__ __launch_bounds__(256) void k_scatter_enc(const float *__restrict__ C,
                                                     uint16_t *__restrict__ codes,
                                                     const float *__restrict__ rhoE,
                                                     const uint32_t *__restrict__ mask, int nx,
                                                     int ny, int nz, long long N, int nc,
                                                     int open_x) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const uint32_t mk = mask[v];
  const bool solid = ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  const Nbr nb((int)v, nx, ny, nz);
  for (int a = 0; a < nc; ++a) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      uint16_t code = 0;
      const float inv_w = i == 0 ? 3.f : (i < 7 ? 18.f : 36.f);
      if (!solid) {
        const bool bb = i > 0 && ((mk >> i) & 1u);
        const float val = bb ? C[(size_t)(a * Q + opp(i)) * N + v]
                             : C[(size_t)(a * Q + i) * N + nb.at(cx(i), cy(i), cz(i))];
        code = enc16<SK>(val * inv_w - writer_ref(rhoE, v, a, nc));
      } else if (open_x && cx(i) != 0 && (nb.x + cx(i) < 0 || nb.x + cx(i) >= nx)) {
        const int rd = nb.at(cx(i), cy(i), cz(i));
        if (((mask[rd] >> CLASS_SHIFT) & 3u) != SOLID_CODE)
          code = enc16<SK>(C[(size_t)(a * Q + i) * N + rd] * inv_w - writer_ref(rhoE, v, a, nc));
      }
      codes[(size_t)(a * Q + i) * N + v] = code;
    }
  }
}

// Open x faces with 16-bit storage.  A pulled value decodes as
// w_i (rho_ref + h) with the reference of the slot's owner (refs [v][a], the
// densities of the level the set was written at; 1 for one component), and
// the face kernels encode what they write against the same owner's
// reference, so every reader (the step, the density pass, the decode)
// decodes the face values unchanged.
template <int SK>
__device__ inline float pulled16(const uint16_t *codes, const float *refs, long long N, int nc,
                                 int a, int i, long long owner) {
  return (float)wq(i) * (writer_ref(refs, owner, a, nc) + dec16<SK>(codes[(size_t)(a * Q + i) * N + owner]));
}

// Exact density faces (the formula of k_density_faces) on 16-bit offsets.
template <int SK, int NC>
__global__ __launch_bounds__(256) void k_density_faces16(const ModelConsts mc,
                                                         uint16_t *__restrict__ codes,
                                                         const float *__restrict__ refs,
                                                         const uint32_t *__restrict__ mask) {
  const long long N = mc.N;
  const int nx = mc.nx, ny = mc.ny, nz = mc.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * ny * nz) return;
  const int face = k / (ny * nz);
  const int r = k - face * ny * nz;
  const int y = r % ny, z = r / ny;
  const int xb = face == 0 ? 0 : nx - 1, s = face == 0 ? 1 : -1, wrap = face == 0 ? nx - 1 : 0;
  const long long vb = xb + (long long)nx * (y + (long long)ny * z);
  const uint32_t mk = mask[vb];
  const bool fluid = ((mk >> CLASS_SHIFT) & 3u) != SOLID_CODE;
  auto at = [&](int xx, int yy, int zz) -> long long {
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
    return xx + (long long)nx * (yy + (long long)ny * zz);
  };
  for (int a = 0; a < NC; ++a) {
    float g[Q];
    float s0 = 0, sm = 0, ny2 = 0, nz2 = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      g[j] = 0;
      if (cx(j) == s) continue;
      const float v = ((mk >> opp(j)) & 1u)
                          ? pulled16<SK>(codes, refs, N, NC, a, opp(j), vb)
                          : pulled16<SK>(codes, refs, N, NC, a, j, at(xb - cx(j), y - cy(j), z - cz(j)));
      g[j] = v;
      if (cx(j) == 0) {
        s0 += v;
        ny2 += (float)cy(j) * v;
        nz2 += (float)cz(j) * v;
      } else {
        sm += v;
      }
    }
    const float Ny = 0.5f * ny2, Nz = 0.5f * nz2;
    const float sJ = (float)(face == 0 ? mc.rho_in[a] : mc.rho_out[a]) - s0 - 2.f * sm;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cx(i) != s) continue;
      const float val = g[opp(i)] + (float)(6.0 * wq(i)) * sJ - (float)cy(i) * Ny - (float)cz(i) * Nz;
      const long long owner = at(wrap, y - cy(i), z - cz(i));
      const float inv_w = i < 7 ? 18.f : 36.f;
      codes[(size_t)(a * Q + i) * N + owner] =
          fluid ? enc16<SK>(val * inv_w - writer_ref(refs, owner, a, NC)) : (uint16_t)0;
    }
  }
}

// Reservoir faces (the reading of k_reservoirs) on 16-bit offsets.
template <int SK, int NC>
__global__ __launch_bounds__(256) void k_reservoirs16(const ModelConsts mc,
                                                      uint16_t *__restrict__ codes,
                                                      const float *__restrict__ refs,
                                                      const uint32_t *__restrict__ mask) {
  const long long N = mc.N;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mc.ny * mc.nz) return;
  const long long v0 = (long long)k * mc.nx, v1 = v0 + mc.nx - 1;
  float u[2][3];
  const long long vb[2] = {v0, v1};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const bool fluid = ((mask[vb[e]] >> CLASS_SHIFT) & 3u) != SOLID_CODE;
    float rho = 0, m0 = 0, m1 = 0, m2 = 0;
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const float f = pulled16<SK>(codes, refs, N, NC, a, i, vb[e]);
        rho += f;
        m0 += (float)cx(i) * f;
        m1 += (float)cy(i) * f;
        m2 += (float)cz(i) * f;
      }
    const float ir = fluid ? 1.f / rho : 0.f;
    u[e][0] = m0 * ir;
    u[e][1] = m1 * ir;
    u[e][2] = m2 * ir;
  }
  for (int a = 0; a < NC; ++a) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (cx(i) == 0) continue;
      const int e = cx(i) > 0 ? 0 : 1;  // inlet reservoir sends c_x = +1, outlet c_x = -1
      const float r = (float)(e == 0 ? mc.rho_in[a] : mc.rho_out[a]);
      const float cu = (float)cx(i) * u[e][0] + (float)cy(i) * u[e][1] + (float)cz(i) * u[e][2];
      const float usq = u[e][0] * u[e][0] + u[e][1] * u[e][1] + u[e][2] * u[e][2];
      const float geq = r * (1.f + 3.f * cu + 4.5f * cu * cu - 1.5f * usq);  // f_eq / w_i
      const long long owner = e == 0 ? v1 : v0;
      codes[(size_t)(a * Q + i) * N + owner] = enc16<SK>(geq - writer_ref(refs, owner, a, NC));
    }
  }
}

// Two components: the fused step wrote rhoS[v] = sum_i w_i rho_ref(s_i) over
// the sources s_i of v's next pulls with the reservoir densities for the
// sources beyond an open face; those pulls read slots whose reference is their
// owner's (the voxel across the wrap), so a face voxel's sum takes the
// difference.  One thread per face voxel.
__global__ __launch_bounds__(256) void k_rhoS_faces(const ModelConsts mc, float *__restrict__ rhoS,
                                                    const float *__restrict__ refs,
                                                    const uint32_t *__restrict__ mask) {
  const int nx = mc.nx, ny = mc.ny, nz = mc.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * ny * nz) return;
  const int face = k / (ny * nz);
  const int r = k - face * ny * nz;
  const int y = r % ny, z = r / ny;
  const int xb = face == 0 ? 0 : nx - 1, out = face == 0 ? -1 : 1, wrap = face == 0 ? nx - 1 : 0;
  const long long v = xb + (long long)nx * (y + (long long)ny * z);
  if (((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  float add[2] = {0.f, 0.f};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (cx(i) != out) continue;  // x + c_i beyond the face
    int yy = y + cy(i), zz = z + cz(i);
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
    const long long owner = wrap + (long long)nx * (yy + (long long)ny * zz);
    for (int a = 0; a < 2; ++a) {
      const float res = (float)(face == 0 ? mc.rho_in[a] : mc.rho_out[a]);
      add[a] += (float)wq(i) * (refs[2 * owner + a] - res);
    }
  }
  rhoS[2 * v] += add[0];
  rhoS[2 * v + 1] += add[1];
}

// per-link outlet flux through the plane x_f | x_f + 1 from the stored offsets
template <int SK, int NC>
__global__ void k_flux16(const ModelConsts mc, const uint16_t *__restrict__ codes,
                         const float *__restrict__ rhoE, const uint32_t *__restrict__ mask,
                         double *__restrict__ partial) {
  const long long N = mc.N;
  const int nyz = mc.ny * mc.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double val[2] = {0.0, 0.0};
  if (k < nyz) {
    const int x0 = mc.outlet_x;
    const int x1 = x0 + 1 == mc.nx ? 0 : x0 + 1;
    const long long base = (long long)k * mc.nx;
    const long long v0 = base + x0, v1 = base + x1;
    const uint32_t m0 = mask[v0], m1 = mask[v1];
    const bool f0 = ((m0 >> CLASS_SHIFT) & 3u) != SOLID_CODE;
    const bool f1 = ((m1 >> CLASS_SHIFT) & 3u) != SOLID_CODE;
    // every offset and reference is loaded (any voxel's slots are valid) and
    // the links taken afterwards, so all loads of a thread are in flight at once
    uint16_t cd[NC][10];
    float ref[2][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      ref[0][a] = writer_ref(rhoE, v0, a, NC);
      ref[1][a] = writer_ref(rhoE, v1, a, NC);
      int n = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (cx(i) != 0) cd[a][n++] = codes[(size_t)(a * Q + i) * N + (cx(i) == 1 ? v0 : v1)];
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double q = 0.0;
      int n = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (cx(i) == 0) continue;
        const float h = dec16<SK>(cd[a][n++]);
        if (cx(i) == 1) {
          const double pv = (double)((float)wq(i) * (ref[0][a] + h));
          q = f0 && !((m0 >> i) & 1u) ? q + pv : q;
        } else {
          const double pv = (double)((float)wq(i) * (ref[1][a] + h));
          q = f1 && !((m1 >> i) & 1u) ? q - pv : q;
        }
      }
      val[a] = q;
    }
  }
  block_sum<2>(val, partial + (size_t)blockIdx.x * 2, false);
}

}  // namespace lbm
