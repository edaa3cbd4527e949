// The fused collide-stream kernel of one time step (gfx950).
//
// A block owns a column of 64 x 4 voxels (one wavefront per x-row, so every
// population load and store of a wave is 256 contiguous bytes) and marches
// along z through a chunk of ZC planes.  Rolling windows in LDS hold, per
// plane, the densities of both components and the mobile saturation S_hat on
// the column plus a radius-2 halo (periodic wrap), a solid flag per cell, and
// the CSF normals n^a = grad rho^b / |grad rho^b| on the column plus a
// radius-1 halo.  Each plane is staged once and used by three consecutive
// voxel planes, so every stencil of the step (pseudo-potential sum,
// grad rho^b, curvature -div n^a, grad S_hat) reads LDS only.  Blocks are
// numbered so that the blocks resident on one XCD (dispatch is round-robin
// over the 8 XCDs) cover neighbouring columns, keeping halo re-reads in that
// XCD's L2.
//
// Collision: with the Hermite-projected (regularised) operator the
// post-collision set depends on the gathered populations only through their
// first moments (rho, rho u, the second-moment tensor), so the pull
// accumulates those ten moments per component on the fly.  Equilibrium,
// projected non-equilibrium part and the force term of Eq. (3) are each a
// quadratic form w_i (A + B.c_i + c_i^T C c_i), so the 19 outgoing
// populations follow from ten coefficients per component.  The BGK variant
// keeps the populations.
namespace lbm {
namespace zm {
constexpr int TX = 64, TY = 4;
constexpr int NT = TX * TY;
constexpr int R = 2;
constexpr int HX = TX + 2 * R, HY = TY + 2 * R;
constexpr int NH = HX * HY;          // density plane cells
constexpr int MX = TX + 2, MY = TY + 2;
constexpr int NM = MX * MY;          // normal plane cells
constexpr int RS = 4;                // density planes z-1 .. z+2
constexpr int MS = 3;                // normal planes z-1 .. z+1
constexpr int ZC = 32;               // planes per block
__host__ __device__ constexpr int hoff(int i) { return cx(i) + HX * cy(i); }
__host__ __device__ constexpr int moff(int i) { return cx(i) + MX * cy(i); }
}  // namespace zm

// Run constants pre-converted to the arithmetic type, so the kernel reads
// them as scalar (SGPR) operands instead of converting inside the loop.
template <typename T>
struct KC {
  int nx, ny, nz, csf_all, tensor, collision;
  long long N;
  T g[2][3], omega[2], nu[2], wall_dpsi[2];
  T G, kappa, csf_den, s_min, span, kr_min, hyst, m_minor, eps_n;
};

template <typename T>
KC<T> make_kc(const ModelConsts &m) {
  KC<T> k{};
  k.nx = m.nx; k.ny = m.ny; k.nz = m.nz; k.N = m.N;
  k.csf_all = m.csf_all; k.tensor = m.tensor; k.collision = m.collision;
  for (int a = 0; a < 2; ++a) {
    for (int d = 0; d < 3; ++d) k.g[a][d] = (T)m.g[a][d];
    k.omega[a] = (T)m.omega[a];
    k.nu[a] = (T)m.nu[a];
    k.wall_dpsi[a] = (T)m.wall_dpsi[a];
  }
  k.G = (T)m.G; k.kappa = (T)m.kappa; k.csf_den = (T)(1.0 / m.csf_scale);
  k.s_min = (T)m.s_min; k.span = (T)(1.0 / m.inv_span); k.kr_min = (T)m.kr_min;
  k.hyst = (T)m.hyst; k.m_minor = (T)m.m_minor; k.eps_n = (T)m.eps_n;
  return k;
}

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
__device__ inline void bstore(rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ inline void bstore(rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}

__device__ inline int rslot(int z) { return (z + 8) & 3; }
__device__ inline int mslot(int z) { return (z + 9) % 3; }

// Writes the 19 populations w_i (A + B.c_i + c_i^T C c_i) * sc (plus keep*f_i
// for BGK) of one component.
template <typename T, bool REG>
__device__ __forceinline__ void emit_post(rsrc_t out, uint32_t vox, uint32_t N, T A, T B0, T B1, T B2,
                                          T Cxx, T Cyy, T Czz, T Cxy, T Cxz, T Cyz, T sc,
                                          const T *fpop, T keep) {
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
  const T exy = A + Cxx + Cyy, exz = A + Cxx + Czz, eyz = A + Cyy + Czz;
  const T dxy = (T)2 * Cxy, dxz = (T)2 * Cxz, dyz = (T)2 * Cyz;
  v[7] = w2 * (exy + B0 + B1 + dxy);
  v[8] = w2 * (exy - B0 - B1 + dxy);
  v[9] = w2 * (exy + B0 - B1 - dxy);
  v[10] = w2 * (exy - B0 + B1 - dxy);
  v[11] = w2 * (exz + B0 + B2 + dxz);
  v[12] = w2 * (exz - B0 - B2 + dxz);
  v[13] = w2 * (exz + B0 - B2 - dxz);
  v[14] = w2 * (exz - B0 + B2 - dxz);
  v[15] = w2 * (eyz + B1 + B2 + dyz);
  v[16] = w2 * (eyz - B1 - B2 + dyz);
  v[17] = w2 * (eyz + B1 - B2 - dyz);
  v[18] = w2 * (eyz - B1 + B2 - dyz);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    T val = v[i];
    if (!REG) val += keep * sc * fpop[i];
    bstore(out, ((uint32_t)i * N + vox) * (uint32_t)sizeof(T), val);
  }
}

template <typename T, int NC, bool REG>
__global__ __launch_bounds__(256) void k_step_zm(const KC<T> mc, const T *__restrict__ fin,
                                                 T *__restrict__ fout, const DevState<T> s,
                                                 const int tiles_x, const int tiles_y,
                                                 const int chunks_z, const int ntiles) {
  using namespace zm;
  constexpr bool STENCIL = NC == 2;
  __shared__ T srho[STENCIL ? RS : 1][NC][STENCIL ? NH : 1];
  __shared__ T sS[STENCIL ? RS : 1][STENCIL ? NH : 1];
  __shared__ uint8_t ssol[STENCIL ? RS : 1][STENCIL ? NH : 1];
  __shared__ T snrm[STENCIL ? MS : 1][STENCIL ? 6 : 1][STENCIL ? NM : 1];
  __shared__ int sxw[HX], syw[HY];

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
  const long long nxy = (long long)nx * ny;
  const int x0 = bx * TX, y0 = by * TY;
  const int zs = bzc * ZC;
  const int ze = zs + ZC < nz ? zs + ZC : nz;
  const bool csf = STENCIL && mc.kappa != (T)0;
  const T span = mc.span;

  if (tid < HX) sxw[tid] = wrapn(x0 + tid - R, nx);
  if (tid < HY) syw[tid] = wrapn(y0 + tid - R, ny);
  __syncthreads();

  // stage one density plane (global plane zz, periodic) into its ring slot
  auto load_rho = [&](int zz) {
    const int sl = rslot(zz);
    const long long zoff = (long long)wrapn(zz, nz) * nxy;
    for (int k = tid; k < NH; k += NT) {
      const int lx = k % HX, ly = k / HX;
      const long long g = zoff + sxw[lx] + (long long)nx * syw[ly];
      const bool sol = ((s.mask[g] >> CLASS_SHIFT) & 3u) == SOLID_CODE;
      ssol[sl][k] = sol;
      const T rw = s.rho[g];
      srho[sl][0][k] = rw;
      if (NC == 2) {
        const T ro = s.rho[N + g];
        srho[sl][NC - 1][k] = ro;
        sS[sl][k] = sol ? (T)0 : (rw / (rw + ro) - mc.s_min) / span;
      }
    }
  };
  // CSF normals of plane zz from the density planes zz-1 .. zz+1
  auto make_normals = [&](int zz) {
    const int ms = mslot(zz);
    for (int k = tid; k < NM; k += NT) {
      const int mx_ = k % MX, my_ = k / MX;
      const int c = (mx_ + 1) + HX * (my_ + 1);
      const int sc0 = rslot(zz);
      const bool sol = ssol[sc0][c];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T self = srho[sc0][1 - a][c];
        T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int sl = rslot(zz + cz(i));
          const int cc = c + hoff(i);
          const T val = ssol[sl][cc] ? self : srho[sl][1 - a][cc];
          if (cx(i)) g0 += (T)(gw(i) * cx(i)) * val;
          if (cy(i)) g1 += (T)(gw(i) * cy(i)) * val;
          if (cz(i)) g2 += (T)(gw(i) * cz(i)) * val;
        }
        const T n = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
        const bool big = !sol && n > mc.eps_n;
        snrm[ms][a * 3 + 0][k] = big ? g0 / n : (T)0;
        snrm[ms][a * 3 + 1][k] = big ? g1 / n : (T)0;
        snrm[ms][a * 3 + 2][k] = big ? g2 / n : (T)0;
      }
    }
  };

  if (STENCIL) {
    for (int zz = zs - 2; zz <= zs + 1; ++zz) load_rho(zz);
    __syncthreads();
    if (csf) {
      make_normals(zs - 1);
      make_normals(zs);
    }
  }

  const int x = x0 + tx, y = y0 + ty;
  const bool inside = x < nx && y < ny;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int X3[3] = {xm, x, xp};
  const int Y3[3] = {ym * nx, y * nx, yp * nx};
  const int c = (tx + R) + HX * (ty + R);
  const int cn = (tx + 1) + MX * (ty + 1);
  const T cs2 = (T)CS2;

  for (int z = zs; z < ze; ++z) {
    if (STENCIL) {
      __syncthreads();  // previous plane done with the slot reused below
      load_rho(z + 2);
      __syncthreads();
      if (csf) {
        make_normals(z + 1);
        __syncthreads();
      }
    }
    if (!inside) continue;
    const long long v = x + (long long)nx * y + (long long)z * nxy;
    const uint32_t v32 = (uint32_t)v;
    const uint32_t N32 = (uint32_t)N;
    const uint32_t mk = s.mask[v];
    const uint32_t cl = (mk >> CLASS_SHIFT) & 3u;
    if (cl == SOLID_CODE) continue;
    const bool gray = cl == GRAY_CODE;
    const int zm1 = z == 0 ? nz - 1 : z - 1, zp1 = z == nz - 1 ? 0 : z + 1;
    const uint32_t Z3[3] = {(uint32_t)(zm1 * nxy), (uint32_t)(z * nxy), (uint32_t)(zp1 * nxy)};

    // a1 + a2: pull with bounce-back, moments accumulated on the fly
    T rho[NC], mom[NC][3], P[NC][6];
    T f[REG ? 1 : NC][REG ? 1 : Q];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const rsrc_t rin = make_rsrc(fin + (size_t)a * Q * N, (uint32_t)(Q * N * sizeof(T)));
      T r = 0, m0 = 0, m1 = 0, m2 = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int j = opp(i);
        const uint32_t e = ((mk >> j) & 1u)
                               ? (uint32_t)j * N32 + v32
                               : (uint32_t)i * N32 + (uint32_t)(X3[1 - cx(i)] + Y3[1 - cy(i)]) +
                                     Z3[1 - cz(i)];
        const T val = bload(rin, e * (uint32_t)sizeof(T), (T)0);
        if (!REG) f[REG ? 0 : a][REG ? 0 : i] = val;
        r += val;
        if (cx(i)) { m0 += (T)cx(i) * val; pxx += val; }
        if (cy(i)) { m1 += (T)cy(i) * val; pyy += val; }
        if (cz(i)) { m2 += (T)cz(i) * val; pzz += val; }
        if (cx(i) && cy(i)) pxy += (T)(cx(i) * cy(i)) * val;
        if (cx(i) && cz(i)) pxz += (T)(cx(i) * cz(i)) * val;
        if (cy(i) && cz(i)) pyz += (T)(cy(i) * cz(i)) * val;
      }
      rho[a] = r;
      mom[a][0] = m0; mom[a][1] = m1; mom[a][2] = m2;
      P[a][0] = pxx; P[a][1] = pyy; P[a][2] = pzz; P[a][3] = pxy; P[a][4] = pxz; P[a][5] = pyz;
    }
    __builtin_amdgcn_sched_barrier(0);
    T rt = rho[0];
    if (NC == 2) rt = rho[0] + rho[1];

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
      const T sat = tw / (tw + to);
      S = (sat - mc.s_min) / span;
      S = S < (T)0 ? (T)0 : (S > (T)1 ? (T)1 : S);
      rhoT = tw + to;
      // a3: pseudo-potential force (solid neighbours: local density + wetting offset)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int bb = 1 - a;
        T pw = rho[bb] + mc.wall_dpsi[bb];
        pw = pw > (T)0 ? pw : (T)0;
        T acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const T psi = ((mk >> i) & 1u) ? pw : srho[rslot(z + cz(i))][bb][c + hoff(i)];
          if (cx(i)) acc0 += (T)(wq(i) * cx(i)) * psi;
          if (cy(i)) acc1 += (T)(wq(i) * cy(i)) * psi;
          if (cz(i)) acc2 += (T)(wq(i) * cz(i)) * psi;
        }
        const T k = -mc.G * rho[a];
        Fex[a][0] += k * acc0;
        Fex[a][1] += k * acc1;
        Fex[a][2] += k * acc2;
        __builtin_amdgcn_sched_barrier(0);
      }
      // a3: CSF surface-tension control, Eq. (4)
      if (csf && (gray || mc.csf_all)) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const T self = rho[1 - a];
          const int m0s = mslot(z);
          T gr0 = 0, gr1 = 0, gr2 = 0, dv = 0;
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const bool sol = (mk >> i) & 1u;
            const T val = sol ? self : srho[rslot(z + cz(i))][1 - a][c + hoff(i)];
            const int ms = sol ? m0s : mslot(z + cz(i));
            const int u = sol ? cn : cn + moff(i);
            if (cx(i)) gr0 += (T)(gw(i) * cx(i)) * val;
            if (cy(i)) gr1 += (T)(gw(i) * cy(i)) * val;
            if (cz(i)) gr2 += (T)(gw(i) * cz(i)) * val;
            if (cx(i)) dv += (T)(gw(i) * cx(i)) * snrm[ms][a * 3 + 0][u];
            if (cy(i)) dv += (T)(gw(i) * cy(i)) * snrm[ms][a * 3 + 1][u];
            if (cz(i)) dv += (T)(gw(i) * cz(i)) * snrm[ms][a * 3 + 2][u];
          }
          const T k = mc.kappa * (-dv);
          const T sc = mc.csf_den;
          Fex[a][0] += k * gr0 * rho[a] / sc;
          Fex[a][1] += k * gr1 * rho[a] / sc;
          Fex[a][2] += k * gr2 * rho[a] / sc;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // a4: capillary term of Eq. (1) and the resistance coefficient
      if (gray) {
        const T shat0 = (rho[0] / rt - mc.s_min) / span;
        T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const T val = ((mk >> i) & 1u) ? shat0 : sS[rslot(z + cz(i))][c + hoff(i)];
          if (cx(i)) g0 += (T)(gw(i) * cx(i)) * val;
          if (cy(i)) g1 += (T)(gw(i) * cy(i)) * val;
          if (cz(i)) g2 += (T)(gw(i) * cz(i)) * val;
        }
        const int t = s.ptype[v];
        const T *tb = s.tab + (size_t)t * 3 * TABLE_N;
        const T Pc = s.sJ[v] * lerp_tab<T>(tb, S);
        const T krw = lerp_tab<T>(tb + TABLE_N, S);
        const T kro = lerp_tab<T>(tb + 2 * TABLE_N, S);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const T k = -Pc * (rho[a] / rt);
          Fex[a][0] += k * g0;
          Fex[a][1] += k * g1;
          Fex[a][2] += k * g2;
        }
        const T Sw = S, So = (T)1 - S;
        const T krmin = mc.kr_min;
        const T cw = Sw > (T)0 ? rt * Sw * mc.nu[0] / (krw > krmin ? krw : krmin) : (T)0;
        const T co = So > (T)0 ? rt * So * mc.nu[1] / (kro > krmin ? kro : krmin) : (T)0;
        cR = cw + co;
      }
    } else if (gray) {
      cR = rt * mc.nu[0];
    }

    // a5: semi-implicit velocity u = (rho I + R/2)^-1 (m + sum F_ex / 2)
    T b0 = 0, b1 = 0, b2 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      b0 += mom[a][0]; b1 += mom[a][1]; b2 += mom[a][2];
      e0 += Fex[a][0]; e1 += Fex[a][1]; e2 += Fex[a][2];
    }
    b0 = b0 + (T)0.5 * e0;
    b1 = b1 + (T)0.5 * e1;
    b2 = b2 + (T)0.5 * e2;
    T Ru0 = 0, Ru1 = 0, Ru2 = 0;
    if (gray && mc.tensor) {
      const T *K = s.Kinv;
      const T Rxx = cR * K[v], Ryy = cR * K[N + v], Rzz = cR * K[2 * N + v];
      const T Rxy = cR * K[3 * N + v], Rxz = cR * K[4 * N + v], Ryz = cR * K[5 * N + v];
      const T h = (T)0.5;
      const T a00 = rt + h * Rxx, a11 = rt + h * Ryy, a22 = rt + h * Rzz;
      const T a01 = h * Rxy, a02 = h * Rxz, a12 = h * Ryz;
      const T c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22,
              c02 = a01 * a12 - a02 * a11;
      const T c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12,
              c22 = a00 * a11 - a01 * a01;
      const T det = a00 * c00 + a01 * c01 + a02 * c02;
      const T u0 = (c00 * b0 + c01 * b1 + c02 * b2) / det;
      const T u1 = (c01 * b0 + c11 * b1 + c12 * b2) / det;
      const T u2 = (c02 * b0 + c12 * b1 + c22 * b2) / det;
      Ru0 = Rxx * u0 + Rxy * u1 + Rxz * u2;
      Ru1 = Rxy * u0 + Ryy * u1 + Ryz * u2;
      Ru2 = Rxz * u0 + Ryz * u1 + Rzz * u2;
    } else if (gray) {
      const T Rs = cR / s.K0[v];
      const T den = rt + (T)0.5 * Rs;
      Ru0 = Rs * (b0 / den);
      Ru1 = Rs * (b1 / den);
      Ru2 = Rs * (b2 / den);
    }

    // a6: Shan-Chen common velocity u'
    T den = 0, up0 = 0, up1 = 0, up2 = 0;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const T om = mc.omega[a];
      den += rho[a] * om;
      up0 += mom[a][0] * om; up1 += mom[a][1] * om; up2 += mom[a][2] * om;
    }
    up0 /= den; up1 /= den; up2 /= den;
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

    // a6: collision + exact-difference force term (Eq. (3)) as quadratic forms
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const T ra = rho[a];
      const T kr = rho[a] / rt;
      const T Fa0 = Fex[a][0] - kr * Ru0, Fa1 = Fex[a][1] - kr * Ru1, Fa2 = Fex[a][2] - kr * Ru2;
      const T h2 = (T)2 * ra;
      const T ua0 = up0 + Fa0 / h2, ua1 = up1 + Fa1 / h2, ua2 = up2 + Fa2 / h2;
      const T uF = ua0 * Fa0 + ua1 * Fa1 + ua2 * Fa2;
      const T om = mc.omega[a];
      const T keep = (T)1 - om;
      // equilibrium part (weight omega for BGK, 1 for the projected form)
      const T we = REG ? (T)1 : om;
      T A = we * ra * ((T)1 - (T)1.5 * usq) - (T)3 * uF;
      T B0 = (T)3 * (we * ra * up0 + Fa0);
      T B1 = (T)3 * (we * ra * up1 + Fa1);
      T B2 = (T)3 * (we * ra * up2 + Fa2);
      const T er = (T)4.5 * we * ra;
      T Cxx = er * up0 * up0 + (T)9 * ua0 * Fa0;
      T Cyy = er * up1 * up1 + (T)9 * ua1 * Fa1;
      T Czz = er * up2 * up2 + (T)9 * ua2 * Fa2;
      T Cxy = er * up0 * up1 + (T)4.5 * (ua0 * Fa1 + ua1 * Fa0);
      T Cxz = er * up0 * up2 + (T)4.5 * (ua0 * Fa2 + ua2 * Fa0);
      T Cyz = er * up1 * up2 + (T)4.5 * (ua1 * Fa2 + ua2 * Fa1);
      if (REG) {
        // projected non-equilibrium part: j - rho u', Pi - rho (cs2 I + u'u')
        const T jn0 = mom[a][0] - ra * up0, jn1 = mom[a][1] - ra * up1, jn2 = mom[a][2] - ra * up2;
        const T qxx = P[a][0] - ra * (cs2 + up0 * up0);
        const T qyy = P[a][1] - ra * (cs2 + up1 * up1);
        const T qzz = P[a][2] - ra * (cs2 + up2 * up2);
        const T qxy = P[a][3] - ra * up0 * up1;
        const T qxz = P[a][4] - ra * up0 * up2;
        const T qyz = P[a][5] - ra * up1 * up2;
        const T k3 = (T)3 * keep, k45 = (T)4.5 * keep;
        A -= (T)1.5 * keep * (qxx + qyy + qzz);
        B0 += k3 * jn0; B1 += k3 * jn1; B2 += k3 * jn2;
        Cxx += k45 * qxx; Cyy += k45 * qyy; Czz += k45 * qzz;
        Cxy += k45 * qxy; Cxz += k45 * qxz; Cyz += k45 * qyz;
      }
      const T sc = NC == 2 ? scale[a] : (T)1;
      const rsrc_t rout = make_rsrc(fout + (size_t)a * Q * N, (uint32_t)(Q * N * sizeof(T)));
      emit_post<T, REG>(rout, v32, N32, A, B0, B1, B2, Cxx, Cyy, Czz, Cxy, Cxz, Cyz, sc,
                        f[REG ? 0 : a], keep);
    }
  }
}

}  // namespace lbm
