// Device kernels of the multiscale two-component D3Q19 step (gfx950).
//
// Storage: populations f[a][i][v] (structure of arrays, x fastest), two copies.
// The stored copy holds the post-collision populations of the last step; a
// step pulls them along -c_i (halfway bounce-back at solid neighbours), which
// gives the post-streaming set at the current time level, and writes the new
// post-collision set into the other copy at the same voxel.
//
// The arithmetic follows the paper's Sec. II (Eqs. (1)-(7)) with the readings
// documented in the header lbm.h.
#include "lbm_internal.hpp"

#include <math.h>

namespace lbm {

// ------------------------------------------------------------------ lattice
constexpr int kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr uint64_t pack(const int (&c)[Q]) {
  uint64_t r = 0;
  for (int i = 0; i < Q; ++i) r |= (uint64_t)(c[i] + 1) << (2 * i);
  return r;
}
constexpr uint64_t PCX = pack(kCX), PCY = pack(kCY), PCZ = pack(kCZ);

__host__ __device__ constexpr int cx(int i) { return (int)((PCX >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cy(int i) { return (int)((PCY >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cz(int i) { return (int)((PCZ >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wq(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
constexpr double CS2 = 1.0 / 3.0;
// coefficient of the isotropic gradient: w_i c_i / cs^2 per unit component
__host__ __device__ constexpr double gw(int i) { return wq(i) / CS2; }

__device__ inline int wrapc(int v, int n) {
  if (v < 0) v += n;
  if (v < 0) v += n;
  if (v >= n) v -= n;
  if (v >= n) v -= n;
  return v;
}

// Wrapped coordinates of x-2..x+2 (and y, z) for stencils up to radius 2.
struct Nbr {
  int X[5], Y[5], Z[5];
  int nx, nxy, x;
  __device__ Nbr(int v, int nx_, int ny, int nz) {
    nx = nx_;
    nxy = nx_ * ny;
    x = v % nx_;
    int t = v / nx_;
    int y = t % ny;
    int z = t / ny;
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
      X[d + 2] = wrapc(x + d, nx_);
      Y[d + 2] = wrapc(y + d, ny) * nx_;
      Z[d + 2] = wrapc(z + d, nz) * nxy;
    }
  }
  __device__ int at(int dx, int dy, int dz) const { return X[dx + 2] + Y[dy + 2] + Z[dz + 2]; }
};

template <typename T>
__device__ inline T lerp_tab(const T *tab, T v) {
  T t = v * (T)(TABLE_N - 1);
  T fl = floor(t);
  int k = (int)fl;
  if (k > TABLE_N - 2) k = TABLE_N - 2;
  if (k < 0) k = 0;
  T fr = t - (T)k;
  T lo = tab[k];
  T hi = tab[k + 1];
  return lo + fr * (hi - lo);
}

// ------------------------------------------------------------------ reductions
template <int NV>
__device__ inline void block_sum(double (&val)[NV], double *out_row, bool maxlast) {
  // deterministic: wave shuffles then a fixed-order pass over the waves
  __shared__ double sh[NV][16];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = val[k];
    for (int off = 32; off > 0; off >>= 1) {
      double y = __shfl_down(x, off, 64);
      x = (maxlast && k == NV - 1) ? fmax(x, y) : x + y;
    }
    if (lane == 0) sh[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double x = sh[k][0];
      for (int w = 1; w < nw; ++w)
        x = (maxlast && k == NV - 1) ? fmax(x, sh[k][w]) : x + sh[k][w];
      out_row[k] = x;
    }
  }
}

// ------------------------------------------------------------------ setup
// With open x faces (pressure boundaries) a neighbour beyond a face is a
// reservoir cell, which is fluid.
__global__ void k_mask(const uint8_t *__restrict__ cls, uint32_t *__restrict__ mask, int nx,
                       int ny, int nz, long long N, int open_x) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  Nbr nb((int)v, nx, ny, nz);
  const int x = (int)(v % nx);
  uint32_t m = (uint32_t)cls[v] << CLASS_SHIFT;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const bool beyond = open_x && (x + cx(i) < 0 || x + cx(i) >= nx);
    if (!beyond && cls[nb.at(cx(i), cy(i), cz(i))] == SOLID_CODE) m |= 1u << i;
  }
  mask[v] = m;
}

// Open x faces: the populations the reservoir cells send into the domain,
// written into the slots that the boundary voxels pull across the periodic
// wrap (slots whose own populations leave the domain): the equilibrium at the
// reservoir density and at the mixture velocity of the adjacent boundary
// voxel's post-collision set.  One thread per (y, z) row.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_reservoirs(const ModelConsts mc, T *__restrict__ post,
                                                    const uint32_t *__restrict__ mask) {
  const long long N = mc.N;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mc.ny * mc.nz) return;
  const long long v0 = (long long)k * mc.nx, v1 = v0 + mc.nx - 1;
  T u[2][3];
  const long long vb[2] = {v0, v1};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const bool fluid = ((mask[vb[e]] >> CLASS_SHIFT) & 3u) != SOLID_CODE;
    T rho = 0, m0 = 0, m1 = 0, m2 = 0;
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T f = post[(size_t)(a * Q + i) * N + vb[e]];
        rho += f;
        m0 += (T)cx(i) * f;
        m1 += (T)cy(i) * f;
        m2 += (T)cz(i) * f;
      }
    const T ir = fluid ? (T)1 / rho : (T)0;
    u[e][0] = m0 * ir;
    u[e][1] = m1 * ir;
    u[e][2] = m2 * ir;
  }
  for (int a = 0; a < NC; ++a) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (cx(i) == 0) continue;
      const int e = cx(i) > 0 ? 0 : 1;  // inlet reservoir sends c_x = +1, outlet c_x = -1
      const T r = (T)(e == 0 ? mc.rho_in[a] : mc.rho_out[a]);
      const T cu = (T)cx(i) * u[e][0] + (T)cy(i) * u[e][1] + (T)cz(i) * u[e][2];
      const T usq = u[e][0] * u[e][0] + u[e][1] * u[e][1] + u[e][2] * u[e][2];
      const T feq = (T)wq(i) * r * ((T)1 + (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * usq);
      post[(size_t)(a * Q + i) * N + (e == 0 ? v1 : v0)] = feq;
    }
  }
}

// Exact density faces (Zou-He type): for every fluid voxel on a face, the
// populations it will pull across the face, chosen so that its pulled set
// holds the prescribed density of each component and no momentum along y and
// z.  With s = +1 at x = 0 and -1 at x = nx - 1 (the c_x of the unknown
// directions) and g_j its known pulled values (c_x = 0 or -s; bounce-back at
// a solid source): s J = rho_b - sum_{c_x=0} g - 2 sum_{c_x=-s} g and
// g_i = g_opp(i) + 6 w_i s J - c_y N_y - c_z N_z with N_y, N_z half the
// transverse sums of the c_x = 0 values.  Each value goes into the slot the
// voxel pulls it from (across the periodic wrap).  One thread per face voxel;
// the slots written (c_x = s arrays on the far plane) are never among the
// values read (nx >= 3).
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_density_faces(const ModelConsts mc, T *__restrict__ post,
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
    T g[Q];
    T s0 = 0, sm = 0, ny2 = 0, nz2 = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      g[j] = 0;
      if (cx(j) == s) continue;
      const T v = ((mk >> opp(j)) & 1u) ? post[(size_t)(a * Q + opp(j)) * N + vb]
                                        : post[(size_t)(a * Q + j) * N +
                                               at(xb - cx(j), y - cy(j), z - cz(j))];
      g[j] = v;
      if (cx(j) == 0) {
        s0 += v;
        ny2 += (T)cy(j) * v;
        nz2 += (T)cz(j) * v;
      } else {
        sm += v;
      }
    }
    const T Ny = (T)0.5 * ny2, Nz = (T)0.5 * nz2;
    const T sJ = (T)(face == 0 ? mc.rho_in[a] : mc.rho_out[a]) - s0 - (T)2 * sm;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cx(i) != s) continue;
      const T val = g[opp(i)] + (T)(6.0 * wq(i)) * sJ - (T)cy(i) * Ny - (T)cz(i) * Nz;
      post[(size_t)(a * Q + i) * N + at(wrap, y - cy(i), z - cz(i))] = fluid ? val : (T)0;
    }
  }
}

// Per gray voxel (fp64): K0 = lerp(K0_tab, phi), s_J (Leverett-J, Eq. (5)),
// residual saturations at the crossings of s_J Pc(S) with c Pc_PM.
__device__ double crossing_s(const double *pc, double sj, double target, bool *found) {
  const int n = TABLE_N - 1;
  if (sj * pc[0] < target || sj * pc[n] > target) {
    *found = false;
    return 0.0;
  }
  *found = true;
  // first k with sj*pc[k] <= target (the curve is non-increasing)
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (sj * pc[mid] <= target) hi = mid;
    else lo = mid + 1;
  }
  if (lo == 0) return 0.0;
  double a = sj * pc[lo - 1], b = sj * pc[lo];
  return ((double)(lo - 1) + (a - target) / (a - b)) / (double)n;
}

template <typename T>
__global__ void k_setup_gray(const double *__restrict__ phi, const uint8_t *__restrict__ pt,
                             const uint32_t *__restrict__ mask, const double *__restrict__ tabs,
                             const double *__restrict__ tabmeta, double c_max, double c_min,
                             long long N, T *K0, T *sJ, T *thw, T *tho, double *K0d, T *phiT) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t cl = (mask[v] >> CLASS_SHIFT) & 3u;
  if (cl != GRAY_CODE) {
    K0[v] = 0; sJ[v] = 0; thw[v] = 0; tho[v] = 0; K0d[v] = 0.0;
    phiT[v] = (cl == SOLID_CODE) ? (T)0 : (T)1;
    return;
  }
  const int t = pt[v];
  const double *K0t = tabs + (size_t)t * 4 * TABLE_N;
  const double *Pct = K0t + TABLE_N;
  const double phi_ref = tabmeta[t * 8 + 0], pcpm = tabmeta[t * 8 + 1];
  const double ph = phi[v];
  double k0 = lerp_tab<double>(K0t, ph);
  double k0ref = lerp_tab<double>(K0t, phi_ref);
  double sj = sqrt((k0ref / phi_ref) / (k0 / ph));
  bool fw, fo;
  double sw = crossing_s(Pct, sj, c_max * pcpm, &fw);
  double so = crossing_s(Pct, sj, c_min * pcpm, &fo);
  K0[v] = (T)k0;
  K0d[v] = k0;
  sJ[v] = (T)sj;
  thw[v] = (T)(fw ? sw : 0.0);
  tho[v] = (T)(fo ? 1.0 - so : 0.0);
  phiT[v] = (T)ph;
}

// Separable periodic Gaussian of the porosity field along one axis (fp64).
__global__ void k_smooth(const double *__restrict__ in, double *__restrict__ out, int nx, int ny,
                         int nz, long long N, int axis, int radius, const double *__restrict__ w) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  int x = (int)(v % nx);
  long long t = v / nx;
  int y = (int)(t % ny);
  int z = (int)(t / ny);
  double acc = 0.0;
  for (int j = -radius; j <= radius; ++j) {
    int xx = x, yy = y, zz = z;
    if (axis == 0) zz = ((z + j) % nz + nz) % nz;
    else if (axis == 1) yy = ((y + j) % ny + ny) % ny;
    else xx = ((x + j) % nx + nx) % nx;
    acc += w[j + radius] * in[xx + (long long)nx * (yy + (long long)ny * zz)];
  }
  out[v] = acc;
}

__global__ void k_base_phi(const uint32_t *__restrict__ mask, const double *__restrict__ phi,
                           double *__restrict__ out, long long N) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t cl = (mask[v] >> CLASS_SHIFT) & 3u;
  out[v] = cl == GRAY_CODE ? phi[v] : (cl == SOLID_CODE ? 0.0 : 1.0);
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (fp64).
// On return A holds the eigenvalues on its diagonal and V the eigenvectors as
// columns.
__device__ void jacobi3(double A[3][3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off == 0.0 || off <= 1e-36 * dia) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        double apq = A[p][q];
        if (apq == 0.0) continue;
        double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A J
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- J^T A
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        A[p][q] = A[q][p] = 0.0;
        for (int k = 0; k < 3; ++k) {  // V <- V J
          double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// Principal axes from the Hessian (ordered by |lambda|), gradient tie-break,
// isotropic gate, and K^-1 = sum_k e_k e_k^T / (a_k K0)  (Eqs. (6)-(7)).
template <typename T>
__global__ void k_axes(const double *__restrict__ ps, const uint32_t *__restrict__ mask,
                       const uint8_t *__restrict__ pt, const double *__restrict__ K0d,
                       const double *__restrict__ tabmeta, int nx, int ny, int nz, long long N,
                       double eps_g, double eps_H, double delta_tie, T *__restrict__ Kinv) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t cl = (mask[v] >> CLASS_SHIFT) & 3u;
  if (cl != GRAY_CODE) {
    for (int k = 0; k < 6; ++k) Kinv[(size_t)k * N + v] = (T)0;
    return;
  }
  Nbr nb((int)v, nx, ny, nz);
  auto P = [&](int dx, int dy, int dz) { return ps[nb.at(dx, dy, dz)]; };
  const double p0 = P(0, 0, 0);
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double g[3], H[3][3];
  for (int a = 0; a < 3; ++a) {
    const int *ea = off[a];
    double pp = P(ea[0], ea[1], ea[2]);
    double pm = P(-ea[0], -ea[1], -ea[2]);
    g[a] = 0.5 * (pp - pm);
    H[a][a] = pp - 2.0 * p0 + pm;
    for (int b = a + 1; b < 3; ++b) {
      const int *eb = off[b];
      double v_pp = P(ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2]);
      double v_pm = P(ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]);
      double v_mp = P(-ea[0] + eb[0], -ea[1] + eb[1], -ea[2] + eb[2]);
      double v_mm = P(-ea[0] - eb[0], -ea[1] - eb[1], -ea[2] - eb[2]);
      H[a][b] = H[b][a] = 0.25 * (v_pp - v_pm - v_mp + v_mm);
    }
  }
  const double k0 = K0d[v];
  const int t = pt[v];
  const double kd[3] = {tabmeta[t * 8 + 2], tabmeta[t * 8 + 3], tabmeta[t * 8 + 4]};
  double A[3][3], E[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = H[i][j];
  jacobi3(A, E);
  double lam[3] = {A[0][0], A[1][1], A[2][2]};
  double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double amax = fmax(fabs(lam[0]), fmax(fabs(lam[1]), fabs(lam[2])));
  if (amax <= eps_H && gn <= eps_g) {
    for (int i = 0; i < 3; ++i) M[i][i] = 1.0 / k0;
  } else {
    int ord[3] = {0, 1, 2};  // stable sort by |lambda|
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && fabs(lam[ord[j]]) < fabs(lam[ord[j - 1]]); --j) {
        int tmp = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = tmp;
      }
    double e[3][3];  // e[k] = k-th axis
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) e[k][d] = E[d][ord[k]];
    double a0 = fabs(lam[ord[0]]), a1 = fabs(lam[ord[1]]), a2 = fabs(lam[ord[2]]);
    if (a1 - a0 <= delta_tie * a2) {
      double ge3 = g[0] * e[2][0] + g[1] * e[2][1] + g[2] * e[2][2];
      double p[3] = {g[0] - ge3 * e[2][0], g[1] - ge3 * e[2][1], g[2] - ge3 * e[2][2]};
      double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      if (pn > eps_g) {
        double e2[3] = {p[0] / pn, p[1] / pn, p[2] / pn};
        double e1[3] = {e[2][1] * e2[2] - e[2][2] * e2[1], e[2][2] * e2[0] - e[2][0] * e2[2],
                        e[2][0] * e2[1] - e[2][1] * e2[0]};
        double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int d = 0; d < 3; ++d) {
          e[0][d] = e1[d] / n1;
          e[1][d] = e2[d];
        }
      }
    }
    for (int k = 0; k < 3; ++k) {
      double s = kd[k] * k0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] += e[k][i] * e[k][j] / s;
    }
  }
  Kinv[0 * (size_t)N + v] = (T)M[0][0];
  Kinv[1 * (size_t)N + v] = (T)M[1][1];
  Kinv[2 * (size_t)N + v] = (T)M[2][2];
  Kinv[3 * (size_t)N + v] = (T)M[0][1];
  Kinv[4 * (size_t)N + v] = (T)M[0][2];
  Kinv[5 * (size_t)N + v] = (T)M[1][2];
}

// ------------------------------------------------------------------ state moves
// post-streaming set C (canonical) -> stored pre-streaming set B such that the
// pull of the next step reproduces C:  B_i(y) = C_i(y + c_i), or C_opp(i)(y)
// when y + c_i is solid.
template <typename T>
__global__ void k_scatter(const T *__restrict__ C, T *__restrict__ B,
                          const uint32_t *__restrict__ mask, int nx, int ny, int nz, long long N,
                          int ncomp, int open_x, const PopLayout L) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t mk = mask[v];
  bool solid = ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  if (solid && L.cm) return;  // fluid-only layout: a solid voxel has no slot
  const long long sl = L.slot(v, nx);
  LBM_DCHECK(sl >= 0 && sl < L.stride, DC_SCATTER);
  Nbr nb((int)v, nx, ny, nz);
  for (int a = 0; a < ncomp; ++a) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T val = 0;
      const int rd = nb.at(cx(i), cy(i), cz(i));  // the voxel that pulls slot i
      if (!solid) {
        if ((mk >> i) & 1u) val = C[(size_t)(a * Q + opp(i)) * N + v];
        else val = C[(size_t)(a * Q + i) * N + rd];
      } else if (open_x && cx(i) != 0 && (nb.x + cx(i) < 0 || nb.x + cx(i) >= nx) &&
                 ((mask[rd] >> CLASS_SHIFT) & 3u) != SOLID_CODE) {
        // open x faces: a fluid boundary voxel pulls this slot of a solid
        // voxel across the wrap (its reservoir population)
        val = C[(size_t)(a * Q + i) * N + rd];
      }
      B[(size_t)(a * Q + i) * L.stride + sl] = val;
    }
  }
}

// stored set B -> post-streaming set C (the pull of a step, without collision)
template <typename T>
__global__ void k_gather(const T *__restrict__ B, T *__restrict__ C,
                         const uint32_t *__restrict__ mask, int nx, int ny, int nz, long long N,
                         int ncomp, const PopLayout L) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t mk = mask[v];
  bool solid = ((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  Nbr nb((int)v, nx, ny, nz);
  const long long sl = solid ? 0 : L.slot(v, nx);
  LBM_DCHECK(sl >= 0 && sl < L.stride, DC_SCATTER);
  for (int a = 0; a < ncomp; ++a) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T val = 0;
      if (!solid) {
        const int j = opp(i);
        if ((mk >> j) & 1u) val = B[(size_t)(a * Q + j) * L.stride + sl];
        else val = B[(size_t)(a * Q + i) * L.stride + L.slot(nb.at(-cx(i), -cy(i), -cz(i)), nx)];
      }
      C[(size_t)(a * Q + i) * N + v] = val;
    }
  }
}

// Between the dense and the fluid-only population layouts (to_fluid = 1:
// dense src into fluid-only dst; 0: fluid-only src into dense dst, zero at
// solid voxels, as the dense step leaves them).
template <typename T>
__global__ void k_relayout(const T *__restrict__ src, T *__restrict__ dst,
                           const uint32_t *__restrict__ mask, int nx, long long N, int ncomp,
                           const PopLayout L, int to_fluid) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const bool solid = ((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  if (solid && to_fluid) return;
  const long long sl = solid ? 0 : L.slot(v, nx);
  for (int a = 0; a < ncomp; ++a)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const size_t kd = (size_t)(a * Q + i) * N + v, kf = (size_t)(a * Q + i) * L.stride + sl;
      if (to_fluid) dst[kf] = src[kd];
      else dst[kd] = solid ? (T)0 : src[kf];
    }
}

template <typename T>
__global__ void k_equilibrium_rest(const double *__restrict__ rw, const double *__restrict__ ro,
                                   T *__restrict__ C, const uint32_t *__restrict__ mask,
                                   long long N, int ncomp) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  bool solid = ((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE;
  for (int a = 0; a < ncomp; ++a) {
    double rho = solid ? 0.0 : (a == 0 ? rw[v] : ro[v]);
#pragma unroll
    for (int i = 0; i < Q; ++i) C[(size_t)(a * Q + i) * N + v] = (T)(wq(i) * rho * 1.0);
  }
}

// ------------------------------------------------------------------ densities
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ B, T *__restrict__ rho,
                                                 const uint32_t *__restrict__ mask, int nx, int ny,
                                                 int nz, long long N) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t mk = mask[v];
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) {
#pragma unroll
    for (int a = 0; a < NC; ++a) rho[(size_t)a * N + v] = 0;
    return;
  }
  Nbr nb((int)v, nx, ny, nz);
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int j = opp(i);
      T fi = ((mk >> j) & 1u) ? B[(size_t)(a * Q + j) * N + v]
                              : B[(size_t)(a * Q + i) * N + nb.at(-cx(i), -cy(i), -cz(i))];
      s += fi;
    }
    rho[(size_t)a * N + v] = s;
  }
}

// CSF normals n^a = grad rho^b / |grad rho^b| (zero below eps_n), fluid voxels.
template <typename T>
__global__ void k_normals(const T *__restrict__ rho, T *__restrict__ nrm,
                          const uint32_t *__restrict__ mask, int nx, int ny, int nz, long long N,
                          double eps_n) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  uint32_t mk = mask[v];
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) {
    for (int k = 0; k < 6; ++k) nrm[(size_t)k * N + v] = 0;
    return;
  }
  Nbr nb((int)v, nx, ny, nz);
  for (int a = 0; a < 2; ++a) {
    const T *rb = rho + (size_t)(1 - a) * N;
    const T self = rb[v];
    T gr[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      T val = ((mk >> i) & 1u) ? self : rb[nb.at(cx(i), cy(i), cz(i))];
      if (cx(i)) gr[0] += (T)(gw(i) * cx(i)) * val;
      if (cy(i)) gr[1] += (T)(gw(i) * cy(i)) * val;
      if (cz(i)) gr[2] += (T)(gw(i) * cz(i)) * val;
    }
    T n = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    bool big = n > (T)eps_n;
    for (int d = 0; d < 3; ++d) nrm[(size_t)(a * 3 + d) * N + v] = big ? gr[d] / n : (T)0;
  }
}

template <typename T>
__global__ void k_init_side(const T *__restrict__ rho, const uint32_t *__restrict__ mask,
                            uint8_t *__restrict__ side, T *__restrict__ r, long long N,
                            double s_min, double span) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  r[v] = 0;
  r[N + v] = 0;
  uint32_t cl = (mask[v] >> CLASS_SHIFT) & 3u;
  uint8_t sd = 0;
  if (cl == GRAY_CODE) {
    T tw = rho[v], to = rho[N + v];
    T s = tw / (tw + to);
    T S = (s - (T)s_min) / (T)span;
    S = S < (T)0 ? (T)0 : (S > (T)1 ? (T)1 : S);
    sd = S >= (T)0.5 ? 1 : 0;
  }
  side[v] = sd;
}

// ------------------------------------------------------------------ the step
struct FieldsOut {
  void *rho_w, *rho_o, *ux, *uy, *uz, *S, *r_w, *r_o;
};

enum { MODE_STEP = 0, MODE_FIELDS = 1, MODE_DIAG = 2 };

// One voxel of the step (MODE_STEP), of the field evaluation (MODE_FIELDS) or
// of the diagnostics (MODE_DIAG: the voxel's contributions are left in dsum,
// reduced by the caller once all lanes have converged).
template <typename T, int NC, int MODE, typename O>
__device__ __forceinline__ void step_voxel(const ModelConsts &mc, const T *__restrict__ fin,
                                           T *__restrict__ fout, const DevState<T> &s,
                                           const FieldsOut &fo, const long long v,
                                           double (&dsum)[6]) {
  const long long N = mc.N;
  const bool active = v < N;
  uint32_t mk = active ? s.mask[v] : (SOLID_CODE << CLASS_SHIFT);
  const uint32_t cl = (mk >> CLASS_SHIFT) & 3u;
  if (cl == SOLID_CODE) {
    if (MODE == MODE_FIELDS && active) {
      O *outs[8] = {(O *)fo.rho_w, (O *)fo.rho_o, (O *)fo.ux, (O *)fo.uy,
                    (O *)fo.uz,    (O *)fo.S,     (O *)fo.r_w, (O *)fo.r_o};
      for (int k = 0; k < 8; ++k)
        if (outs[k]) outs[k][v] = (O)0;
    }
    return;
  }
  const bool gray = cl == GRAY_CODE;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  const T cs2 = (T)CS2;

  // a1: pull with halfway bounce-back
  T f[NC][Q];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int j = opp(i);
      f[a][i] = ((mk >> j) & 1u) ? fin[(size_t)(a * Q + j) * N + v]
                                 : fin[(size_t)(a * Q + i) * N + nb.at(-cx(i), -cy(i), -cz(i))];
    }
  }
  // a2: moments
  T rho[NC], mom[NC][3];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    T r = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) r += f[a][i];
    rho[a] = r;
    T m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cx(i)) m0 += (T)cx(i) * f[a][i];
      if (cy(i)) m1 += (T)cy(i) * f[a][i];
      if (cz(i)) m2 += (T)cz(i) * f[a][i];
    }
    mom[a][0] = m0; mom[a][1] = m1; mom[a][2] = m2;
  }
  T rt = rho[0];
  if (NC == 2) rt = rho[0] + rho[1];

  T Fex[NC][3];
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) Fex[a][d] = rho[a] * (T)mc.g[a][d];

  T S = 1, rw_res = 0, ro_res = 0, rhoT = rt, cR = 0;
  const T span = (T)(1.0 / mc.inv_span);
  if (NC == 2) {
    if (gray) {
      rw_res = s.r[v];
      ro_res = s.r[N + v];
    }
    const T tw = rho[0] + rw_res, to = rho[1] + ro_res;
    const T sat = tw / (tw + to);
    S = (sat - (T)mc.s_min) / span;
    S = S < (T)0 ? (T)0 : (S > (T)1 ? (T)1 : S);
    rhoT = tw + to;
    // a3: pseudo-potential force
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int b = 1 - a;
      const T *rb = s.rho + (size_t)b * N;
      T pw = rho[b] + (T)mc.wall_dpsi[b];
      pw = pw > (T)0 ? pw : (T)0;
      T acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        T psi = ((mk >> i) & 1u) ? pw : rb[nb.at(cx(i), cy(i), cz(i))];
        if (mc.open_x && cx(i) != 0) {  // a reservoir cell beyond an x face
          const int xn = nb.x + cx(i);
          if (xn < 0) psi = (T)mc.rho_in[b];
          else if (xn >= mc.nx) psi = (T)mc.rho_out[b];
        }
        if (cx(i)) acc0 += (T)(wq(i) * cx(i)) * psi;
        if (cy(i)) acc1 += (T)(wq(i) * cy(i)) * psi;
        if (cz(i)) acc2 += (T)(wq(i) * cz(i)) * psi;
      }
      const T c = -(T)mc.G * rho[a];
      Fex[a][0] += c * acc0;
      Fex[a][1] += c * acc1;
      Fex[a][2] += c * acc2;
    }
    // a3: CSF surface-tension control, Eq. (4)
    if (mc.kappa != 0.0 && (gray || mc.csf_all)) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int b = 1 - a;
        const T *rb = s.rho + (size_t)b * N;
        const T *na = s.nrm + (size_t)(a * 3) * N;
        const T self = rb[v];
        const T n0 = na[v], n1 = na[N + v], n2 = na[2 * N + v];
        T gr0 = 0, gr1 = 0, gr2 = 0, dv = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const bool sol = (mk >> i) & 1u;
          const int u = nb.at(cx(i), cy(i), cz(i));
          const T val = sol ? self : rb[u];
          if (cx(i)) gr0 += (T)(gw(i) * cx(i)) * val;
          if (cy(i)) gr1 += (T)(gw(i) * cy(i)) * val;
          if (cz(i)) gr2 += (T)(gw(i) * cz(i)) * val;
          if (cx(i)) dv += (T)(gw(i) * cx(i)) * (sol ? n0 : na[u]);
          if (cy(i)) dv += (T)(gw(i) * cy(i)) * (sol ? n1 : na[N + u]);
          if (cz(i)) dv += (T)(gw(i) * cz(i)) * (sol ? n2 : na[2 * N + u]);
        }
        const T curv = -dv;
        const T k = (T)mc.kappa * curv;
        const T sc = (T)(1.0 / mc.csf_scale);
        Fex[a][0] += k * gr0 * rho[a] / sc;
        Fex[a][1] += k * gr1 * rho[a] / sc;
        Fex[a][2] += k * gr2 * rho[a] / sc;
      }
    }
    // a4: capillary term of Eq. (1) and the resistance coefficient
    if (gray) {
      const T *rw = s.rho;
      const T *ro = s.rho + N;
      const T shat0 = (rho[0] / rt - (T)mc.s_min) / span;
      T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        T val = shat0;
        if (!((mk >> i) & 1u)) {
          const int u = nb.at(cx(i), cy(i), cz(i));
          const T a_ = rw[u], b_ = ro[u];
          val = (a_ / (a_ + b_) - (T)mc.s_min) / span;
        }
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
        const T c = -Pc * (rho[a] / rt);
        Fex[a][0] += c * g0;
        Fex[a][1] += c * g1;
        Fex[a][2] += c * g2;
      }
      const T Sw = S, So = (T)1 - S;
      const T krmin = (T)mc.kr_min;
      const T cw = Sw > (T)0 ? rt * Sw * (T)mc.nu[0] / (krw > krmin ? krw : krmin) : (T)0;
      const T co = So > (T)0 ? rt * So * (T)mc.nu[1] / (kro > krmin ? kro : krmin) : (T)0;
      cR = cw + co;
    }
  } else if (gray) {
    cR = rt * (T)mc.nu[0];
  }

  // a5: velocity the resistance acts on, u = (rho I + R/2)^-1 (m + sum F_ex / 2)
  // (trapezoidal rule), which is also the reported velocity (m + sum F / 2) / rho
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
  T u0, u1, u2, Ru0 = 0, Ru1 = 0, Ru2 = 0;
  if (gray && mc.tensor) {
    const T *K = s.Kinv;
    const T kxx = K[v], kyy = K[N + v], kzz = K[2 * N + v];
    const T kxy = K[3 * N + v], kxz = K[4 * N + v], kyz = K[5 * N + v];
    const T Rxx = cR * kxx, Ryy = cR * kyy, Rzz = cR * kzz;
    const T Rxy = cR * kxy, Rxz = cR * kxz, Ryz = cR * kyz;
    const T a00 = rt + h * Rxx, a11 = rt + h * Ryy, a22 = rt + h * Rzz;
    const T a01 = h * Rxy, a02 = h * Rxz, a12 = h * Ryz;
    // symmetric 3x3 solve by the adjugate
    const T c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const T c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const T det = a00 * c00 + a01 * c01 + a02 * c02;
    u0 = (c00 * b0 + c01 * b1 + c02 * b2) / det;
    u1 = (c01 * b0 + c11 * b1 + c12 * b2) / det;
    u2 = (c02 * b0 + c12 * b1 + c22 * b2) / det;
    Ru0 = Rxx * u0 + Rxy * u1 + Rxz * u2;
    Ru1 = Rxy * u0 + Ryy * u1 + Ryz * u2;
    Ru2 = Rxz * u0 + Ryz * u1 + Rzz * u2;
  } else {
    const T Rs = gray ? cR / s.K0[v] : (T)0;
    const T den = rt + h * Rs;
    u0 = b0 / den; u1 = b1 / den; u2 = b2 / den;
    Ru0 = Rs * u0; Ru1 = Rs * u1; Ru2 = Rs * u2;
  }

  if (MODE == MODE_FIELDS) {
    auto put = [&](void *p, T val) {
      if (p) ((O *)p)[v] = (O)val;
    };
    put(fo.rho_w, rho[0]);
    put(fo.rho_o, NC == 2 ? rho[NC - 1] : (T)0);
    put(fo.ux, u0); put(fo.uy, u1); put(fo.uz, u2);
    put(fo.S, S);
    put(fo.r_w, rw_res); put(fo.r_o, ro_res);
    return;
  }
  if (MODE == MODE_DIAG) {
    const double ph = (double)s.phiT[v];
    dsum[0] = (double)rho[0] + (double)rw_res;
    dsum[1] = NC == 2 ? (double)rho[NC - 1] + (double)ro_res : 0.0;
    dsum[2] = ph * (double)S;
    dsum[3] = ph;
    const double un = sqrt((double)u0 * u0 + (double)u1 * u1 + (double)u2 * u2);
    dsum[4] = isfinite(un) && isfinite(dsum[0]) && isfinite(dsum[1]) ? 0.0 : 1.0;
    dsum[5] = isfinite(un) ? un : 0.0;
    return;
  }

  // total force per component: F^a = F_ex^a - (rho^a / rho) R u
  T F[NC][3];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const T c = rho[a] / rt;
    F[a][0] = Fex[a][0] - c * Ru0;
    F[a][1] = Fex[a][1] - c * Ru1;
    F[a][2] = Fex[a][2] - c * Ru2;
  }
  // a6: Shan-Chen common velocity u'
  T den = 0, up0 = 0, up1 = 0, up2 = 0;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const T om = (T)mc.omega[a];
    den += rho[a] * om;
    up0 += mom[a][0] * om; up1 += mom[a][1] * om; up2 += mom[a][2] * om;
  }
  up0 /= den; up1 /= den; up2 /= den;
  const T usq = up0 * up0 + up1 * up1 + up2 * up2;

  // a7 (residual transfer) decides per-component scale factors applied to f_post
  T scale[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) scale[a] = 1;
  if (NC == 2 && gray) {
    const uint8_t sd = s.side[v];
    const T hy = (T)mc.hyst;
    const T m = (T)mc.m_minor;
    if (!sd && S >= (T)0.5 + hy) {
      // oil -> water: release residual water, trap theta_o of the total as oil
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
      // water -> oil: release residual oil, trap theta_w of the total as water
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

  // a6: collision (Hermite-projected or BGK) + exact-difference force (Eq. (3))
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    const T ra = rho[a];
    T feq[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T cu = (T)cx(i) * up0 + (T)cy(i) * up1 + (T)cz(i) * up2;
      feq[i] = (T)wq(i) * ra * ((T)1 + cu / cs2 + cu * cu / ((T)2 * cs2 * cs2) - usq / ((T)2 * cs2));
    }
    T f1[Q];
    if (mc.collision == 0) {
      T j0 = 0, j1 = 0, j2 = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T d = f[a][i] - feq[i];
        if (cx(i)) j0 += (T)cx(i) * d;
        if (cy(i)) j1 += (T)cy(i) * d;
        if (cz(i)) j2 += (T)cz(i) * d;
        if (cx(i)) pxx += d;
        if (cy(i)) pyy += d;
        if (cz(i)) pzz += d;
        if (cx(i) && cy(i)) pxy += (T)(cx(i) * cy(i)) * d;
        if (cx(i) && cz(i)) pxz += (T)(cx(i) * cz(i)) * d;
        if (cy(i) && cz(i)) pyz += (T)(cy(i) * cz(i)) * d;
      }
      const T tr = pxx + pyy + pzz;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T cj = (T)cx(i) * j0 + (T)cy(i) * j1 + (T)cz(i) * j2;
        T pcc = 0;
        if (cx(i)) pcc += pxx;
        if (cy(i)) pcc += pyy;
        if (cz(i)) pcc += pzz;
        if (cx(i) && cy(i)) pcc += (T)(2 * cx(i) * cy(i)) * pxy;
        if (cx(i) && cz(i)) pcc += (T)(2 * cx(i) * cz(i)) * pxz;
        if (cy(i) && cz(i)) pcc += (T)(2 * cy(i) * cz(i)) * pyz;
        f1[i] = (T)wq(i) * (cj / cs2 + (pcc - cs2 * tr) / ((T)2 * cs2 * cs2));
      }
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) f1[i] = f[a][i] - feq[i];
    }
    const T Fa0 = F[a][0], Fa1 = F[a][1], Fa2 = F[a][2];
    const T h2 = (T)2 * ra;
    const T ua0 = up0 + Fa0 / h2, ua1 = up1 + Fa1 / h2, ua2 = up2 + Fa2 / h2;
    const T uF = ua0 * Fa0 + ua1 * Fa1 + ua2 * Fa2;
    const T keep = (T)1 - (T)mc.omega[a];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T cF = (T)cx(i) * Fa0 + (T)cy(i) * Fa1 + (T)cz(i) * Fa2;
      const T cu = (T)cx(i) * ua0 + (T)cy(i) * ua1 + (T)cz(i) * ua2;
      const T src =
          (T)wq(i) * (cF / cs2 + ((T)2 * cu * cF - (T)2 * cs2 * uF) / ((T)2 * cs2 * cs2));
      T post = feq[i] + keep * f1[i] + src;
      if (NC == 2) post = post * scale[a];
      fout[(size_t)(a * Q + i) * N + v] = post;
    }
  }
}

template <typename T, int NC, int MODE, typename O>
__global__ __launch_bounds__(256) void k_step(const ModelConsts mc, const T *__restrict__ fin,
                                              T *__restrict__ fout, const DevState<T> s,
                                              const FieldsOut fo) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double dsum[6] = {0, 0, 0, 0, 0, 0};  // mass_w, mass_o, phi S, phi, nonfinite, max|u|
  step_voxel<T, NC, MODE, O>(mc, fin, fout, s, fo, v, dsum);
  if (MODE == MODE_DIAG) block_sum<6>(dsum, s.partial + (size_t)blockIdx.x * 6, true);
}

// Outlet flux through the plane x_f | x_f+1, counted per link from the
// post-collision set (links with a solid end are skipped).
template <typename T, int NC>
__global__ void k_flux(const ModelConsts mc, const T *__restrict__ post,
                       const uint32_t *__restrict__ mask, double *__restrict__ partial,
                       const PopLayout L) {
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
    const long long s0 = f0 ? L.slot(v0, mc.nx) : 0, s1 = f1 ? L.slot(v1, mc.nx) : 0;
    LBM_DCHECK(v0 < N && v1 < N && s0 < L.stride && s1 < L.stride, DC_FLUX);
    // every value is loaded (the slots are valid for any voxel) and the
    // links taken afterwards, so all loads of a thread are in flight at once
    T p[NC][10];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      int n = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i)
        if (cx(i) != 0) p[a][n++] = post[(size_t)(a * Q + i) * L.stride + (cx(i) == 1 ? s0 : s1)];
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double q = 0.0;
      int n = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (cx(i) == 0) continue;
        const double pv = (double)p[a][n++];
        if (cx(i) == 1) q = f0 && !((m0 >> i) & 1u) ? q + pv : q;
        else q = f1 && !((m1 >> i) & 1u) ? q - pv : q;
      }
      val[a] = q;
    }
  }
  block_sum<2>(val, partial + (size_t)blockIdx.x * 2, false);
}

// Fixed-order sum of block partials (nv values per block), one block of 256
// threads: strided partial sums then a fixed tree, so results are
// deterministic for a given launch shape.
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partial, int nblocks,
                                                  int nv, int maxlast, double *__restrict__ out,
                                                  int accumulate) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  for (int k = 0; k < nv; ++k) {
    const bool mx = maxlast && k == nv - 1;
    double x = 0.0;
    for (int b = t; b < nblocks; b += 256) {
      const double y = partial[(size_t)b * nv + k];
      x = mx ? fmax(x, y) : x + y;
    }
    sh[t] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) sh[t] = mx ? fmax(sh[t], sh[t + w]) : sh[t] + sh[t + w];
      __syncthreads();
    }
    if (t == 0) {
      if (accumulate) {  // out[0..nv) = last values, out[nv..2nv) += last values
        out[k] = sh[0];
        out[nv + k] += sh[0];
      } else {
        out[k] = sh[0];
      }
    }
    __syncthreads();
  }
}

}  // namespace lbm
