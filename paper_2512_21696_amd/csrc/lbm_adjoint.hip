// Discrete adjoint of the one-component step: the gradient of a loss on the
// outlet-flux history with respect to K0 (and, through the K0(phi) table, to
// the gray porosity), by a reverse sweep over recomputed states.
//
// Forward map of one step (Sec. II of the paper with one component; this is
// what the fused step computes in exact arithmetic):
//   pull      f_i(x) = post_i(x - c_i), or post_opp(i)(x) when x - c_i is solid;
//   moments   rho, m = sum c_i f_i, Pi = sum c_i c_i^T f_i (Phi below is
//             linear in Pi, so its reverse needs rho and m only);
//   Eq. (1)   R_s = rho nu / K0 on gray voxels (0 elsewhere),
//             u = (m + h rho g) / (rho + h R_s), F = rho g - R_s u, h = 1/2
//             (the trapezoidal rule);
//   collision post_i = w_i (A + B.c_i + c_i^T C c_i) with u' = m / rho,
//             ua = u' + F / (2 rho), omega = 1 / tau, the equilibrium
//             velocity ve = u' and kf = 1 in pore voxels, ve = ua and
//             kf = 1 - omega / 2 in gray voxels, and
//               equilibrium  A = e rho (1 - ve.ve / 2cs2), B = e rho ve / cs2,
//                            C = e rho ve ve^T / 2cs4,
//               force (Eq. (3))  A = -kf ua.F / cs2, B = kf F / cs2,
//                            C = kf (ua F^T + F ua^T) / 2cs4,
//               regularised non-equilibrium  B = (1 - omega) j / cs2,
//                            A = -(1 - omega) tr P / 2cs2, C = (1 - omega) P / 2cs4,
//                            j = m - rho ve, P = Pi - rho cs2 I - rho ve ve^T,
//             e = 1 (regularised) or omega (BGK, which also keeps (1 - omega) f_i);
//   flux      Q(n) = sum over the outlet links of post_i(x_f) (c_x = +1) minus
//             post_i(x_f + 1) (c_x = -1), both ends fluid.
//
// Reverse of step n at a fluid voxel x, given lam (dL/df of the post-streaming
// set that step n produced):
//   lam_post_j(x) = lam_opp(j)(x) when x + c_j is solid, else lam_j(x + c_j)
//                   (the transpose of the pull), plus dL/dQ(n) times the
//                   link's flux weight;
//   Lambda0, Lambda1, Lambda2 = sum_j w_j lam_post_j (1, c_j, c_j c_j^T) turn
//   sum_j lam_post_j post_j into the scalar Phi = A Lambda0 + B.Lambda1 + C:Lambda2,
//   whose arithmetic is swept backwards by hand to dPhi/drho, dPhi/dm,
//   dPhi/dPi and dPhi/dK0; then
//   lam'_k(x) = dPhi/drho + c_k.dPhi/dm + c_k^T (dPhi/dPi) c_k
//               (+ (1 - omega) lam_post_k for BGK) is dL/df of the set step n
//   read, and dL/dK0(x) gains dPhi/dK0.
namespace lbm {
namespace adj {

// XCD-aware voxel order of the stencil kernels: the chip hands consecutive
// blocks to its 8 XCDs in turn, so a plain linear order spreads the
// neighbouring planes of a voxel over all of them and each XCD's L2 re-fetches
// the neighbours' values.  Remapped, each XCD takes one contiguous run of
// voxels.  The grid must be a multiple of 8 blocks (blocks8).
__device__ inline long long xcd_voxel() {
  const long long per = gridDim.x / 8;
  return ((long long)(blockIdx.x % 8) * per + blockIdx.x / 8) * blockDim.x + threadIdx.x;
}

// Exact density faces: the transpose of the face step on the adjoint of the
// next level (indexed like the pulled values: lam[a][i][w] is dL/d of the
// value w pulls in direction i, component a).  A face voxel's unknown pulls
// g_i (c_x(i) = s) are linear in its known pulls g_j of the same level,
//   dg_i/dg_j = [j = opp(i)] - 6 w_i - (c_y(i) c_y(j) + c_z(i) c_z(j)) / 2  (c_x(j) = 0)
//             = [j = opp(i)] - 12 w_i                                       (c_x(j) = -s),
// so each lam[i][v] moves onto the knowns' entries, and the unknowns' entries
// become zero (the post-collision values the periodic pull would have brought
// across the face are overwritten).  Two components: the density of a fluid
// face voxel is the prescribed one whatever the level's values (the sum of
// its pulls' derivatives vanishes), so the adjoint of the next level's density
// there (rnl, added to every pull of the voxel by the reverse step) is zeroed.
// One thread per face voxel; it touches only its own entries.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_density_faces(const ModelConsts mc,
                                                           T *__restrict__ lam,
                                                           T *__restrict__ rnl,
                                                           const uint32_t *__restrict__ mask) {
  const long long N = mc.N;
  const int nx = mc.nx, ny = mc.ny, nz = mc.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * ny * nz) return;
  const int face = k / (ny * nz);
  const int r = k - face * ny * nz;
  const int y = r % ny, z = r / ny;
  const int xb = face == 0 ? 0 : nx - 1, s = face == 0 ? 1 : -1;
  const long long v = xb + (long long)nx * (y + (long long)ny * z);
  if (((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  for (int a = 0; a < mc.ncomp; ++a) {
    T *const la = lam + (size_t)a * Q * N;
    double l[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) l[i] = (double)la[(size_t)i * N + v];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cx(i) != s) continue;
      const double li = l[i];
      l[i] = 0.0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if (cx(j) == s) continue;
        double c = j == opp(i) ? 1.0 : 0.0;
        if (cx(j) == 0) c -= 6.0 * wq(i) + 0.5 * (double)(cy(i) * cy(j) + cz(i) * cz(j));
        else c -= 12.0 * wq(i);
        l[j] += c * li;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) la[(size_t)i * N + v] = (T)l[i];
    if (rnl) rnl[2 * v + a] = (T)0;
  }
}

// Pressure reservoirs: the transpose of the reservoir face step on the
// adjoint of the next level (lam, indexed like the pulled values).  The step
// wrote, into the slots across the periodic wrap that the boundary voxels
// pull, f_i = w_i rho_res (1 + 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u) with u the
// mixture velocity m / rho of the post-collision sets (both components) of
// the boundary voxel of the same (y, z) row (zero when it is solid); rec holds
// that rho and u per step (k_res_record).  Reverse, per row end: dL/du is the
// sum over the written slots of their adjoint times
// w_i rho_res (3 c_i + 9 (c_i.u) c_i - 3 u); the written slots' adjoint
// becomes zero (the values they held reach nothing); then every post-collision
// value f_j^b of a fluid boundary voxel gets (c_j - u).dL/du / rho.  The
// adjoint of a post-collision value is the entry of the voxel that pulls it
// (x + c_j in direction j, or the voxel's own entry in direction opp(j) across
// a solid link; a link across an x face is never one) plus, with two
// components, that puller's rnl (the adjoint of its next density, which the
// reverse step adds to each of its pulls): a zeroed slot takes -rnl.  Both
// ends' dL/du are taken before any value gets its share, since each end's
// written slots are values of the other end.  A written slot whose puller is
// solid has no reader and adds nothing; its entry is cleared, because it can
// hold the share a fluid boundary voxel across the face gave it two reverse
// steps earlier (the two adjoint sets alternate and the reverse step never
// writes a solid voxel's entries), and then gets this step's share, which the
// boundary voxel's gather reads there.  One thread per (y, z) row; it touches
// only the entries of its row's two boundary voxels, so rows do not overlap.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_reservoirs(const ModelConsts mc,
                                                        T *__restrict__ lam,
                                                        const T *__restrict__ rnl,
                                                        const uint32_t *__restrict__ mask,
                                                        const double *__restrict__ rec) {
  const long long N = mc.N;
  const int nx = mc.nx, ny = mc.ny, nz = mc.nz;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ny * nz) return;
  const int y = k % ny, z = k / ny;
  const double *const rk = rec + 8LL * k;
  double ub[2][3] = {{0, 0, 0}, {0, 0, 0}};
  for (int e = 0; e < 2; ++e) {
    const int s = e == 0 ? 1 : -1;          // c_x of the directions the reservoir sends
    const int xp = e == 0 ? 0 : nx - 1;     // the plane that pulls them
    const double *const u = rk + 4 * e + 1;
    for (int a = 0; a < mc.ncomp; ++a) {
      // the reservoir density and the weights as the forward rounds them
      const double r = (double)(T)(e == 0 ? mc.rho_in[a] : mc.rho_out[a]);
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        if (cx(i) != s) continue;
        const int yy = (y + cy(i) + ny) % ny, zz = (z + cz(i) + nz) % nz;
        const long long w = xp + (long long)nx * (yy + (long long)ny * zz);
        T *const li = lam + ((size_t)a * Q + i) * N + w;
        if (((mask[w] >> CLASS_SHIFT) & 3u) == SOLID_CODE) {
          *li = (T)0;  // no reader; the entry may hold a value left two steps back
          continue;
        }
        const T rn = rnl ? rnl[2 * w + a] : (T)0;
        const double pb = (double)*li + (double)rn;
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double sc = pb * (double)(T)wq(i) * r;
        ub[e][0] += sc * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * u[0]);
        ub[e][1] += sc * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * u[1]);
        ub[e][2] += sc * (3.0 * cz(i) + 9.0 * cu * cz(i) - 3.0 * u[2]);
        *li = -rn;
      }
    }
  }
  for (int e = 0; e < 2; ++e) {
    const long long vb = (e == 0 ? 0 : nx - 1) + (long long)nx * (y + (long long)ny * z);
    const uint32_t mk = mask[vb];
    if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) continue;  // u = 0 whatever its values
    const double rho = rk[4 * e];
    const double *const u = rk + 4 * e + 1;
    const double base = -(u[0] * ub[e][0] + u[1] * ub[e][1] + u[2] * ub[e][2]) / rho;
    const Nbr nb((int)vb, nx, ny, nz);
    for (int b = 0; b < mc.ncomp; ++b)
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const bool wall = (mk >> j) & 1u;
        const size_t t = wall ? ((size_t)b * Q + opp(j)) * N + vb
                              : ((size_t)b * Q + j) * N + nb.at(cx(j), cy(j), cz(j));
        const double add = (cx(j) * ub[e][0] + cy(j) * ub[e][1] + cz(j) * ub[e][2]) / rho + base;
        lam[t] = (T)((double)lam[t] + add);
      }
  }
}

// The adjoint populations are stored in the state's type (fp64 or fp32); the
// arithmetic is fp64 throughout and dL/dK0 accumulates in fp64.  One thread
// per voxel; the grid is a multiple of 8 blocks and block b takes the voxel
// range (b % 8) * (grid / 8) + b / 8, so that each XCD (blocks are dealt to
// the 8 XCDs round-robin) sweeps one contiguous z slab and the y and z
// neighbours of its gathers stay in its own L2.
//
// With the tensorial resistivity (TENS) a gray voxel solves
// (rho I + h c_R K^-1) u = m + h rho g with c_R = rho nu and takes
// F = rho g - c_R K^-1 u; the reverse of that solve gives dL/dK^-1, accumulated
// per gray voxel in gk[6][v] (xx, yy, zz, xy, xz, yz: the derivative with
// respect to each stored component, an off-diagonal one standing for both of
// its entries).  Without it gk[v] accumulates dL/dK0.
template <typename T, bool REG, bool TENS>
__global__ __launch_bounds__(256) void k_adj_step(const ModelConsts mc,
                                                  const T *__restrict__ post,
                                                  const T *__restrict__ lin,
                                                  T *__restrict__ lout,
                                                  const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ K0,
                                                  const T *__restrict__ Kinv,
                                                  double *__restrict__ gk, const double a) {
  const long long N = mc.N;
  const int per = gridDim.x / 8;
  const long long blk = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const long long v = blk * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const uint32_t mk = mask[v];
  const uint32_t cl = (mk >> CLASS_SHIFT) & 3u;
  if (cl == SOLID_CODE) return;  // never read: its entries stay zero
  const bool gray = cl == GRAY_CODE;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  const int x1 = mc.outlet_x + 1 == mc.nx ? 0 : mc.outlet_x + 1;
  const bool at0 = nb.x == mc.outlet_x, at1 = nb.x == x1;
  // (tensor) a gray voxel's K^-1 and its dL/dK^-1 accumulators, loaded ahead
  // of the gathers so that their latency overlaps them (the updates at the
  // end add to these values; their six read-after-write round trips would
  // otherwise follow one another)
  double p_K[6] = {0, 0, 0, 0, 0, 0}, p_gk[6] = {0, 0, 0, 0, 0, 0};
  if (TENS && gray) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      p_K[q] = (double)Kinv[(size_t)q * N + v];
      p_gk[q] = gk[(size_t)q * N + v];
    }
  }

  double lp[Q];
  double rho = 0, m0 = 0, m1 = 0, m2 = 0;
  double L0 = 0, L1x = 0, L1y = 0, L1z = 0;
  double Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int j = opp(i);
    const uint32_t N32 = (uint32_t)N, v32 = (uint32_t)v;
    const uint32_t src = ((mk >> j) & 1u) ? (uint32_t)j * N32 + v32
                                          : (uint32_t)i * N32 + (uint32_t)nb.at(-cx(i), -cy(i), -cz(i));
    const double fi = (double)post[src];
    const bool wall = (mk >> i) & 1u;
    const uint32_t li = wall ? (uint32_t)j * N32 + v32
                             : (uint32_t)i * N32 + (uint32_t)nb.at(cx(i), cy(i), cz(i));
    double l = (double)lin[li];
    if (cx(i) == 1 && at0 && !wall) l += a;
    if (cx(i) == -1 && at1 && !wall) l -= a;
    lp[i] = l;
    rho += fi;
    if (cx(i)) m0 += cx(i) * fi;
    if (cy(i)) m1 += cy(i) * fi;
    if (cz(i)) m2 += cz(i) * fi;
    const double wl = wq(i) * l;
    L0 += wl;
    if (cx(i)) { L1x += cx(i) * wl; Mxx += wl; }
    if (cy(i)) { L1y += cy(i) * wl; Myy += wl; }
    if (cz(i)) { L1z += cz(i) * wl; Mzz += wl; }
    if (cx(i) && cy(i)) Mxy += (cx(i) * cy(i)) * wl;
    if (cx(i) && cz(i)) Mxz += (cx(i) * cz(i)) * wl;
    if (cy(i) && cz(i)) Myz += (cy(i) * cz(i)) * wl;
  }

  // forward quantities of the voxel
  const double cs2 = CS2;
  constexpr double ics2 = 3.0, ics4 = 9.0;  // 1 / c_s^2, 1 / c_s^4
  const double om = mc.omega[0], keep = 1.0 - om, e = REG ? 1.0 : om;
  const double h = 0.5;
  const double g0 = mc.g[0][0], g1 = mc.g[0][1], g2 = mc.g[0][2];
  const bool tens = TENS && gray;
  const double b0 = m0 + h * rho * g0, b1 = m1 + h * rho * g1, b2 = m2 + h * rho * g2;
  double k0 = 1.0, r = 0.0, Rs = 0.0, den = rho, cR = 0.0;
  double K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Ai[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double u0, u1, u2, F0, F1, F2, w0 = 0, w1 = 0, w2 = 0;
  if (tens) {
    cR = rho * mc.nu[0];
    K[0][0] = p_K[0];
    K[1][1] = p_K[1];
    K[2][2] = p_K[2];
    K[0][1] = K[1][0] = p_K[3];
    K[0][2] = K[2][0] = p_K[4];
    K[1][2] = K[2][1] = p_K[5];
    const double hc = h * cR;
    const double a00 = rho + hc * K[0][0], a11 = rho + hc * K[1][1], a22 = rho + hc * K[2][2];
    const double a01 = hc * K[0][1], a02 = hc * K[0][2], a12 = hc * K[1][2];
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22,
                 c02 = a01 * a12 - a02 * a11;
    const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12,
                 c22 = a00 * a11 - a01 * a01;
    const double idet = 1.0 / (a00 * c00 + a01 * c01 + a02 * c02);
    Ai[0][0] = c00 * idet; Ai[1][1] = c11 * idet; Ai[2][2] = c22 * idet;
    Ai[0][1] = Ai[1][0] = c01 * idet;
    Ai[0][2] = Ai[2][0] = c02 * idet;
    Ai[1][2] = Ai[2][1] = c12 * idet;
    u0 = Ai[0][0] * b0 + Ai[0][1] * b1 + Ai[0][2] * b2;
    u1 = Ai[1][0] * b0 + Ai[1][1] * b1 + Ai[1][2] * b2;
    u2 = Ai[2][0] * b0 + Ai[2][1] * b1 + Ai[2][2] * b2;
    w0 = K[0][0] * u0 + K[0][1] * u1 + K[0][2] * u2;
    w1 = K[1][0] * u0 + K[1][1] * u1 + K[1][2] * u2;
    w2 = K[2][0] * u0 + K[2][1] * u1 + K[2][2] * u2;
    F0 = rho * g0 - cR * w0; F1 = rho * g1 - cR * w1; F2 = rho * g2 - cR * w2;
  } else {
    if (gray) {
      k0 = (double)K0[v];
      r = mc.nu[0] / k0;
    }
    Rs = rho * r;
    den = rho + h * Rs;
    u0 = b0 / den; u1 = b1 / den; u2 = b2 / den;
    F0 = rho * g0 - Rs * u0; F1 = rho * g1 - Rs * u1; F2 = rho * g2 - Rs * u2;
  }
  const double ir = 1.0 / rho;
  const double p0 = m0 * ir, p1 = m1 * ir, p2 = m2 * ir;  // u'
  const double a0 = p0 + 0.5 * F0 * ir, a1 = p1 + 0.5 * F1 * ir, a2 = p2 + 0.5 * F2 * ir;  // ua
  // equilibrium velocity ve (u' in pore voxels, ua in gray ones) and the
  // force term's weight kf (1, or 1 - omega/2 in gray voxels)
  const double v0 = gray ? a0 : p0, v1 = gray ? a1 : p1, v2 = gray ? a2 : p2;
  const double kf = gray ? 1.0 - 0.5 * om : 1.0;
  const double vsq = v0 * v0 + v1 * v1 + v2 * v2;

  // reverse sweep of Phi
  double rb = 0, pb0 = 0, pb1 = 0, pb2 = 0, Fb0 = 0, Fb1 = 0, Fb2 = 0, ab0 = 0, ab1 = 0, ab2 = 0;
  double vb0 = 0, vb1 = 0, vb2 = 0, mb0 = 0, mb1 = 0, mb2 = 0;
  // A terms
  rb += e * (1.0 - vsq * (0.5 * ics2)) * L0;
  const double vsqb = -e * rho * (0.5 * ics2) * L0;
  const double uFb = -kf * L0 * ics2;
  // B terms
  rb += e * (v0 * L1x + v1 * L1y + v2 * L1z) * ics2;
  vb0 += e * rho * L1x * ics2; vb1 += e * rho * L1y * ics2; vb2 += e * rho * L1z * ics2;
  Fb0 += kf * L1x * ics2; Fb1 += kf * L1y * ics2; Fb2 += kf * L1z * ics2;
  // C terms (M = Lambda2, symmetric)
  const double Mv0 = Mxx * v0 + Mxy * v1 + Mxz * v2;
  const double Mv1 = Mxy * v0 + Myy * v1 + Myz * v2;
  const double Mv2 = Mxz * v0 + Myz * v1 + Mzz * v2;
  rb += e * (v0 * Mv0 + v1 * Mv1 + v2 * Mv2) * (0.5 * ics4);
  vb0 += e * rho * Mv0 * ics4; vb1 += e * rho * Mv1 * ics4; vb2 += e * rho * Mv2 * ics4;
  ab0 += kf * (Mxx * F0 + Mxy * F1 + Mxz * F2) * ics4;
  ab1 += kf * (Mxy * F0 + Myy * F1 + Myz * F2) * ics4;
  ab2 += kf * (Mxz * F0 + Myz * F1 + Mzz * F2) * ics4;
  Fb0 += kf * (Mxx * a0 + Mxy * a1 + Mxz * a2) * ics4;
  Fb1 += kf * (Mxy * a0 + Myy * a1 + Myz * a2) * ics4;
  Fb2 += kf * (Mxz * a0 + Myz * a1 + Mzz * a2) * ics4;
  // regularised non-equilibrium: first order j = m - rho ve (identically 0
  // at ve = u'), second order P = Pi - rho cs2 I - rho ve ve; dPhi/dP is also
  // dPhi/dPi
  double Bxx = 0, Byy = 0, Bzz = 0, Bxy = 0, Bxz = 0, Byz = 0;
  if (REG) {
    const double kj = keep * ics2;
    mb0 += kj * L1x; mb1 += kj * L1y; mb2 += kj * L1z;
    rb -= kj * (v0 * L1x + v1 * L1y + v2 * L1z);
    vb0 -= kj * rho * L1x; vb1 -= kj * rho * L1y; vb2 -= kj * rho * L1z;
    const double c = keep * (0.5 * ics4), d = -keep * (0.5 * ics2) * L0;
    Bxx = c * Mxx + d; Byy = c * Myy + d; Bzz = c * Mzz + d;
    Bxy = c * Mxy; Bxz = c * Mxz; Byz = c * Myz;
    const double Bv0 = Bxx * v0 + Bxy * v1 + Bxz * v2;
    const double Bv1 = Bxy * v0 + Byy * v1 + Byz * v2;
    const double Bv2 = Bxz * v0 + Byz * v1 + Bzz * v2;
    rb += -cs2 * (Bxx + Byy + Bzz) - (v0 * Bv0 + v1 * Bv1 + v2 * Bv2);
    vb0 -= 2 * rho * Bv0; vb1 -= 2 * rho * Bv1; vb2 -= 2 * rho * Bv2;
  }
  // ua.F
  ab0 += F0 * uFb; ab1 += F1 * uFb; ab2 += F2 * uFb;
  Fb0 += a0 * uFb; Fb1 += a1 * uFb; Fb2 += a2 * uFb;
  // ve.ve, then ve = ua (gray) or u' (pore)
  vb0 += 2 * v0 * vsqb; vb1 += 2 * v1 * vsqb; vb2 += 2 * v2 * vsqb;
  if (gray) { ab0 += vb0; ab1 += vb1; ab2 += vb2; }
  else { pb0 += vb0; pb1 += vb1; pb2 += vb2; }
  // ua = u' + F / 2rho
  pb0 += ab0; pb1 += ab1; pb2 += ab2;
  Fb0 += 0.5 * ab0 * ir; Fb1 += 0.5 * ab1 * ir; Fb2 += 0.5 * ab2 * ir;
  rb -= 0.5 * (ab0 * F0 + ab1 * F1 + ab2 * F2) * ir * ir;
  // u' = m / rho
  mb0 += pb0 * ir; mb1 += pb1 * ir; mb2 += pb2 * ir;
  rb -= (pb0 * p0 + pb1 * p1 + pb2 * p2) * ir;
  rb += g0 * Fb0 + g1 * Fb1 + g2 * Fb2;
  double Rsb = 0.0;
  if (tens) {
    // F = rho g - c_R w, w = K^-1 u
    const double Rub[3] = {-Fb0, -Fb1, -Fb2};
    const double u[3] = {u0, u1, u2};
    double cRb = Rub[0] * w0 + Rub[1] * w1 + Rub[2] * w2;
    const double wb[3] = {cR * Rub[0], cR * Rub[1], cR * Rub[2]};
    double Kb[3][3], ub[3];
    for (int i = 0; i < 3; ++i) {
      ub[i] = K[i][0] * wb[0] + K[i][1] * wb[1] + K[i][2] * wb[2];
      for (int j = 0; j < 3; ++j) Kb[i][j] = wb[i] * u[j];
    }
    // u = A^-1 b, A = rho I + h c_R K^-1 (symmetric)
    double bb[3];
    for (int i = 0; i < 3; ++i) bb[i] = Ai[i][0] * ub[0] + Ai[i][1] * ub[1] + Ai[i][2] * ub[2];
    double AK = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double Ab = -bb[i] * u[j];
        AK += Ab * K[i][j];
        Kb[i][j] += h * cR * Ab;
        if (i == j) rb += Ab;
      }
    cRb += h * AK;
    mb0 += bb[0]; mb1 += bb[1]; mb2 += bb[2];
    rb += h * (g0 * bb[0] + g1 * bb[1] + g2 * bb[2]);
    // c_R = rho nu
    rb += mc.nu[0] * cRb;
    const long long NN = N;
    gk[v] = p_gk[0] + Kb[0][0];
    gk[NN + v] = p_gk[1] + Kb[1][1];
    gk[2 * NN + v] = p_gk[2] + Kb[2][2];
    gk[3 * NN + v] = p_gk[3] + (Kb[0][1] + Kb[1][0]);
    gk[4 * NN + v] = p_gk[4] + (Kb[0][2] + Kb[2][0]);
    gk[5 * NN + v] = p_gk[5] + (Kb[1][2] + Kb[2][1]);
  } else {
    // F = rho g - R_s u
    Rsb = -(u0 * Fb0 + u1 * Fb1 + u2 * Fb2);
    const double ub0 = -Rs * Fb0, ub1 = -Rs * Fb1, ub2 = -Rs * Fb2;
    // u = (m + h rho g) / den
    const double idn = 1.0 / den;
    const double bb0 = ub0 * idn, bb1 = ub1 * idn, bb2 = ub2 * idn;
    const double denb = -(ub0 * u0 + ub1 * u1 + ub2 * u2) * idn;
    mb0 += bb0; mb1 += bb1; mb2 += bb2;
    rb += h * (g0 * bb0 + g1 * bb1 + g2 * bb2);
    rb += denb;
    Rsb += h * denb;
    // R_s = rho nu / K0
    rb += r * Rsb;
  }

#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double l = rb;
    if (cx(k)) l += cx(k) * mb0;
    if (cy(k)) l += cy(k) * mb1;
    if (cz(k)) l += cz(k) * mb2;
    if (REG) {
      if (cx(k)) l += Bxx;
      if (cy(k)) l += Byy;
      if (cz(k)) l += Bzz;
      if (cx(k) && cy(k)) l += (2 * cx(k) * cy(k)) * Bxy;
      if (cx(k) && cz(k)) l += (2 * cx(k) * cz(k)) * Bxz;
      if (cy(k) && cz(k)) l += (2 * cy(k) * cz(k)) * Byz;
    } else {
      l += keep * lp[k];
    }
    lout[(size_t)k * N + v] = (T)l;
  }
  if (gray && !tens) gk[v] += -(r / k0) * (rho * Rsb);
}

// ---------------------------------------------------------------------------
// Two components (Sec. II without the CSF control, and for horizons without
// residual events).  Forward quantities at a fluid voxel x, per component a
// (b = 1 - a), with rho_t = rho^w + rho^o:
//   F_ex^a = rho^a g^a - G rho^a sum_i w_i c_i psi^b(x + c_i)   (psi = rho, or
//            max(rho^b(x) + dpsi^b, 0) across a solid link)
//          - P_c (rho^a / rho_t) grad S_hat                       (gray voxels)
//   S_hat = (rho^w / rho_t - s_min) / span (own value across a solid link),
//   S = clamp(((rho^w + r^w) / (rho_t + r^w + r^o) - s_min) / span, 0, 1),
//   P_c = s_J P_c(S), c_R = rho_t S nu^w / max(Kr^w(S), Kr_min)
//                         + rho_t (1 - S) nu^o / max(Kr^o(S), Kr_min),
//   u = (rho_t I + h c_R K^-1)^-1 (m^w + m^o + h (F_ex^w + F_ex^o)), h = 1/2,
//   F^a = F_ex^a - (rho^a / rho_t) c_R K^-1 u,
//   u' = (omega^w m^w + omega^o m^o) / (omega^w rho^w + omega^o rho^o),
//   post^a = w_i (A^a + B^a.c_i + c_i^T C^a c_i) as for one component, with
//   ua^a = u' + F^a / (2 rho^a), the force term at ua^a, the equilibrium
//   feq(rho^a, ve^a) with ve^a = u' (pore) or ua^a and the force term weighted
//   by 1 - omega^a / 2 (gray), and, regularised, the first-order part
//   j^a = m^a - rho^a ve^a of the non-equilibrium.
// The reverse of the force's neighbour reads is split off: k_adj_step2 keeps
// dL/d(acc^a) and dL/d(grad S_hat) of each voxel (stash[9][v]), k_adj_nl2
// gathers them into the neighbours' dL/drho^a (rnl[v][2]), which the next
// reverse step adds to every population of those voxels as it gathers.
// Residual transfer (gray voxels; the branch the forward state takes): on a
// crossing the post-collision sets are scaled, post^a <- s^a post^a, with
//   oil -> water (side 0, S >= 1/2 + h): s^w = (rho^w + r^w) / rho^w,
//     d = max(min(theta_o rho_T - r^o, rho^o - m), 0), s^o = 1 - d / rho^o,
//     r^w <- 0, r^o <- r^o + d;
//   water -> oil (side 1, S <= 1/2 - h): the mirror with theta_w;
// rho_T = rho^w + r^w + rho^o + r^o.  The residual amounts are state: lr[2][v]
// carries dL/dr from step to step (updated in place), and gth[2][v]
// accumulates dL/dtheta_w, dL/dtheta_o.
template <typename T, bool REG, bool TENS, typename AT = double>
__global__ __launch_bounds__(256) void k_adj_step2(
    const ModelConsts mc, const T *__restrict__ post, const T *__restrict__ rho2,
    const T *__restrict__ rres, const uint8_t *__restrict__ side, const T *__restrict__ nrmb,
    const T *__restrict__ inb, const T *__restrict__ lin, const T *__restrict__ rnl, T *__restrict__ lout,
    T *__restrict__ stash,
    const uint32_t *__restrict__ mask, const T *__restrict__ K0, const T *__restrict__ Kinv,
    const T *__restrict__ sJ, const T *__restrict__ thw, const T *__restrict__ tho,
    const uint8_t *__restrict__ ptype, const T *__restrict__ tab, double *__restrict__ gk,
    double *__restrict__ gsj, double *__restrict__ lr, double *__restrict__ gth,
    const double an) {
  // the run's constants in the arithmetic type
  const AT mG = (AT)mc.G, mkappa = (AT)mc.kappa, mcsf = (AT)mc.csf_scale, mminor = (AT)mc.m_minor;
  const AT msmin = (AT)mc.s_min, mspan = (AT)mc.inv_span, mkrmin = (AT)mc.kr_min, mhyst = (AT)mc.hyst;
  const AT mnu[2] = {(AT)mc.nu[0], (AT)mc.nu[1]}, momg[2] = {(AT)mc.omega[0], (AT)mc.omega[1]};
  const AT mwd[2] = {(AT)mc.wall_dpsi[0], (AT)mc.wall_dpsi[1]};
  const AT mg[2][3] = {{(AT)mc.g[0][0], (AT)mc.g[0][1], (AT)mc.g[0][2]},
                       {(AT)mc.g[1][0], (AT)mc.g[1][1], (AT)mc.g[1][2]}};
  const long long N = mc.N;
  const int per = gridDim.x / 8;
  const long long blk = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const long long v = blk * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const uint32_t mk = mask[v];
  const uint32_t cl = (mk >> CLASS_SHIFT) & 3u;
  if (cl == SOLID_CODE) return;
  const bool gray = cl == GRAY_CODE;
  const bool tens = TENS && gray;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  const int x1 = mc.outlet_x + 1 == mc.nx ? 0 : mc.outlet_x + 1;
  const bool at0 = nb.x == mc.outlet_x, at1 = nb.x == x1;
  const AT cs2 = CS2;
  constexpr AT ics2 = AT(3.0), ics4 = AT(9.0);  // 1 / c_s^2, 1 / c_s^4

  // a gray voxel's inputs and accumulators, none of which depends on the
  // gathers below, loaded ahead of them so that their latency overlaps the
  // gathers' (the updates further down add to these values)
  AT p_rres[2] = {0, 0}, p_gS[3] = {0, 0, 0}, p_sj = 0, p_k0 = 1, p_thw = 0, p_tho = 0;
  AT p_K[6] = {0, 0, 0, 0, 0, 0};
  double p_lr[2] = {0, 0}, p_gsj = 0, p_gk[6] = {0, 0, 0, 0, 0, 0};
  const T *p_tb = tab;
  bool p_side = false;
  // the level's neighbour sums of every fluid voxel, and (CSF region) its
  // density gradients and curvatures
  AT p_inb[6], p_cg[2][3] = {{0, 0, 0}, {0, 0, 0}}, p_curv[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < 6; ++q) p_inb[q] = (AT)inb[(size_t)q * N + v];
  const bool csfv = (AT)mc.kappa != AT(0.0) && (gray || mc.csf_all);
  if (csfv) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int d = 0; d < 3; ++d) p_cg[a][d] = (AT)nrmb[(size_t)(6 * a + d) * N + v];
      p_curv[a] = (AT)inb[(size_t)(9 + a) * N + v];
    }
  }
  if (gray) {
    p_rres[0] = (AT)rres[v];
    p_rres[1] = (AT)rres[N + v];
#pragma unroll
    for (int d = 0; d < 3; ++d) p_gS[d] = (AT)inb[(size_t)(6 + d) * N + v];
    p_tb = tab + (size_t)ptype[v] * 3 * TABLE_N;
    p_sj = (AT)sJ[v];
    p_thw = (AT)thw[v];
    p_tho = (AT)tho[v];
    p_side = side[v] != 0;
    p_lr[0] = lr[v];
    p_lr[1] = lr[N + v];
    p_gsj = gsj[v];
    if (TENS) {
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        p_K[q] = (AT)Kinv[(size_t)q * N + v];
        p_gk[q] = gk[(size_t)q * N + v];
      }
    } else {
      p_k0 = (AT)K0[v];
      p_gk[0] = gk[v];
    }
  }

  // pulls, moments and the gathered adjoint of the post-collision sets
  AT rho[2], m[2][3], L0[2], L1[2][3], M2[2][6];  // M2: xx, yy, zz, xy, xz, yz
  AT Pi[2][6], lf[2];  // second moments (regularised), sum_i lam_i f_i (BGK)
  AT lp[REG ? 1 : 2][REG ? 1 : Q];
  const uint32_t N32 = (uint32_t)N, v32 = (uint32_t)v;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    rho[a] = 0; L0[a] = 0; lf[a] = 0;
    for (int d = 0; d < 3; ++d) { m[a][d] = 0; L1[a][d] = 0; }
    for (int d = 0; d < 6; ++d) { M2[a][d] = 0; Pi[a][d] = 0; }
  }
  // one direction at a time for both components (each component's sums keep
  // their order): the addresses serve both, and the neighbour's dL/drho pair
  // is one load
  const vec2<T> *rnl2 = reinterpret_cast<const vec2<T> *>(rnl);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int j = opp(i);
    const uint32_t src = ((mk >> j) & 1u) ? (uint32_t)j * N32 + v32
                                          : (uint32_t)i * N32 + (uint32_t)nb.at(-cx(i), -cy(i), -cz(i));
    const bool wall = (mk >> i) & 1u;
    const uint32_t y = wall ? v32 : (uint32_t)nb.at(cx(i), cy(i), cz(i));
    const uint32_t li = wall ? (uint32_t)j * N32 + v32 : (uint32_t)i * N32 + y;
    const vec2<T> rn = rnl2[y];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const T *pa = post + (size_t)a * Q * N;
      const T *la = lin + (size_t)a * Q * N;
      const AT fi = (AT)pa[src];
      rho[a] += fi;
      if (cx(i)) m[a][0] += cx(i) * fi;
      if (cy(i)) m[a][1] += cy(i) * fi;
      if (cz(i)) m[a][2] += cz(i) * fi;
      if (REG) {
        if (cx(i)) Pi[a][0] += fi;
        if (cy(i)) Pi[a][1] += fi;
        if (cz(i)) Pi[a][2] += fi;
        if (cx(i) && cy(i)) Pi[a][3] += (cx(i) * cy(i)) * fi;
        if (cx(i) && cz(i)) Pi[a][4] += (cx(i) * cz(i)) * fi;
        if (cy(i) && cz(i)) Pi[a][5] += (cy(i) * cz(i)) * fi;
      }
      AT l = (AT)la[li] + (AT)(a == 0 ? rn.x : rn.y);
      if (a == 0 && cx(i) == 1 && at0 && !wall) l += an;
      if (a == 0 && cx(i) == -1 && at1 && !wall) l -= an;
      if (!REG) {
        lp[REG ? 0 : a][REG ? 0 : i] = l;
        lf[a] += l * fi;
      }
      const AT wl = (AT)wq(i) * l;
      L0[a] += wl;
      if (cx(i)) { L1[a][0] += cx(i) * wl; M2[a][0] += wl; }
      if (cy(i)) { L1[a][1] += cy(i) * wl; M2[a][1] += wl; }
      if (cz(i)) { L1[a][2] += cz(i) * wl; M2[a][2] += wl; }
      if (cx(i) && cy(i)) M2[a][3] += (cx(i) * cy(i)) * wl;
      if (cx(i) && cz(i)) M2[a][4] += (cx(i) * cz(i)) * wl;
      if (cy(i) && cz(i)) M2[a][5] += (cy(i) * cz(i)) * wl;
    }
  }

  // forward quantities
  const AT rt = rho[0] + rho[1], irt = AT(1.0) / rt;
  const AT irho[2] = {AT(1.0) / rho[0], AT(1.0) / rho[1]};
  const AT h = AT(0.5);
  const AT ispan = mspan;
  AT Fex[2][3], acc[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int b = 1 - a;
    AT pw = rho[b] + mwd[b];
    pw = pw > AT(0.0) ? pw : AT(0.0);
    // the fluid links' sum comes from the inputs pass, the solid links read pw
    AT s0 = p_inb[3 * a], s1 = p_inb[3 * a + 1], s2 = p_inb[3 * a + 2];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const AT w = ((mk >> i) & 1u) ? (AT)wq(i) * pw : AT(0.0);
      if (cx(i)) s0 += cx(i) * w;
      if (cy(i)) s1 += cy(i) * w;
      if (cz(i)) s2 += cz(i) * w;
    }
    acc[a][0] = s0; acc[a][1] = s1; acc[a][2] = s2;
    for (int d = 0; d < 3; ++d) Fex[a][d] = rho[a] * mg[a][d] - mG * rho[a] * acc[a][d];
  }
  // CSF control, Eq. (4), on the region's voxels: g^a = grad rho^b and the
  // normals n^a = g^a / |g^a| of the level (nrmb rows 6a..6a+2: g, 6a+3..: n),
  // curv^a = -div n^a (own normal across a solid link), F^a += kap curv g rho^a
  const AT kap = mkappa * mcsf;
  AT cg[2][3] = {{0, 0, 0}, {0, 0, 0}}, curv[2] = {0, 0};
  if (csfv) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int d = 0; d < 3; ++d) cg[a][d] = p_cg[a][d];
      curv[a] = p_curv[a];
#pragma unroll
      for (int d = 0; d < 3; ++d) Fex[a][d] += kap * curv[a] * cg[a][d] * rho[a];
    }
  }
  // gray: saturation, tables, capillary force, resistance coefficient
  AT S = 0, Sraw = 0, tw = 0, to = 0, gS[3] = {0, 0, 0}, Pct = 0, dPct = 0, Krw = 0,
         dKrw = 0, Kro = 0, dKro = 0, sj = 0, Pc = 0, kw = 1, ko = 1, ikw = 1, iko = 1, cR = 0;
  const AT shat0 = (rho[0] * irt - msmin) * ispan;
  if (gray) {
    tw = rho[0] + p_rres[0];
    to = rho[1] + p_rres[1];
    Sraw = (tw / (tw + to) - msmin) * ispan;
    S = Sraw < AT(0.0) ? AT(0.0) : (Sraw > AT(1.0) ? AT(1.0) : Sraw);
#pragma unroll
    for (int d = 0; d < 3; ++d) gS[d] = p_gS[d];
#pragma unroll
    for (int i = 1; i < Q; ++i) {  // solid links read this voxel's own S_hat
      const AT w = ((mk >> i) & 1u) ? (AT)gw(i) * shat0 : AT(0.0);
      if (cx(i)) gS[0] += cx(i) * w;
      if (cy(i)) gS[1] += cy(i) * w;
      if (cz(i)) gS[2] += cz(i) * w;
    }
    const T *tb = p_tb;
    const AT t = S * (AT)(TABLE_N - 1);
    int k = (int)floor(t);
    k = k > TABLE_N - 2 ? TABLE_N - 2 : (k < 0 ? 0 : k);
    const AT fr = t - (AT)k;
    auto lookup = [&](const T *c, AT &val, AT &slope) {
      const AT lo = (AT)c[k], hi = (AT)c[k + 1];
      val = lo + fr * (hi - lo);
      slope = (hi - lo) * (AT)(TABLE_N - 1);
    };
    lookup(tb, Pct, dPct);
    lookup(tb + TABLE_N, Krw, dKrw);
    lookup(tb + 2 * TABLE_N, Kro, dKro);
    sj = p_sj;
    Pc = sj * Pct;
    for (int a = 0; a < 2; ++a)
      for (int d = 0; d < 3; ++d) Fex[a][d] += -Pc * (rho[a] * irt) * gS[d];
    kw = Krw > mkrmin ? Krw : mkrmin;
    ko = Kro > mkrmin ? Kro : mkrmin;
    ikw = AT(1.0) / kw;
    iko = AT(1.0) / ko;
    const AT cw = S > AT(0.0) ? rt * S * mnu[0] * ikw : AT(0.0);
    const AT co = AT(1.0) - S > AT(0.0) ? rt * (AT(1.0) - S) * mnu[1] * iko : AT(0.0);
    cR = cw + co;
  }
  // resistance
  AT bvec[3], u[3], Ru[3], K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}},
                                  Ai[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, wv[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) bvec[d] = m[0][d] + m[1][d] + h * (Fex[0][d] + Fex[1][d]);
  AT k0 = AT(1.0), Rs = AT(0.0), den = rt;
  if (tens) {
    K[0][0] = p_K[0];
    K[1][1] = p_K[1];
    K[2][2] = p_K[2];
    K[0][1] = K[1][0] = p_K[3];
    K[0][2] = K[2][0] = p_K[4];
    K[1][2] = K[2][1] = p_K[5];
    const AT hc = h * cR;
    const AT a00 = rt + hc * K[0][0], a11 = rt + hc * K[1][1], a22 = rt + hc * K[2][2];
    const AT a01 = hc * K[0][1], a02 = hc * K[0][2], a12 = hc * K[1][2];
    const AT c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22,
                 c02 = a01 * a12 - a02 * a11;
    const AT c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12,
                 c22 = a00 * a11 - a01 * a01;
    const AT idet = AT(1.0) / (a00 * c00 + a01 * c01 + a02 * c02);
    Ai[0][0] = c00 * idet; Ai[1][1] = c11 * idet; Ai[2][2] = c22 * idet;
    Ai[0][1] = Ai[1][0] = c01 * idet;
    Ai[0][2] = Ai[2][0] = c02 * idet;
    Ai[1][2] = Ai[2][1] = c12 * idet;
    for (int i = 0; i < 3; ++i) u[i] = Ai[i][0] * bvec[0] + Ai[i][1] * bvec[1] + Ai[i][2] * bvec[2];
    for (int i = 0; i < 3; ++i) {
      wv[i] = K[i][0] * u[0] + K[i][1] * u[1] + K[i][2] * u[2];
      Ru[i] = cR * wv[i];
    }
  } else {
    if (gray) {
      k0 = p_k0;
      Rs = cR / k0;  // once per voxel
    }
    den = rt + h * Rs;
    const AT idn0 = AT(1.0) / den;
    for (int d = 0; d < 3; ++d) {
      u[d] = bvec[d] * idn0;
      Ru[d] = Rs * u[d];
    }
  }
  AT F[2][3];
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d) F[a][d] = Fex[a][d] - (rho[a] * irt) * Ru[d];
  const AT om[2] = {momg[0], momg[1]};
  const AT D = om[0] * rho[0] + om[1] * rho[1], iD = AT(1.0) / D;
  AT up[3];
  for (int d = 0; d < 3; ++d) up[d] = (om[0] * m[0][d] + om[1] * m[1][d]) * iD;

  // residual transfer: which branch, the scale factors, and dL/ds^a =
  // sum_i lam_post_i post_i of the unscaled set; the adjoint of the unscaled
  // set is s^a times the gathered one
  int ev = 0;  // 1: oil -> water, 2: water -> oil
  AT sc[2] = {AT(1.0), AT(1.0)}, scb[2] = {AT(0.0), AT(0.0)}, dtr = AT(0.0), rw0 = AT(0.0), ro0 = AT(0.0);
  if (gray) {
    const bool sd = p_side;
    if (!sd && S >= AT(0.5) + mhyst) ev = 1;
    else if (sd && S <= AT(0.5) - mhyst) ev = 2;
  }
  if (ev) {
    rw0 = p_rres[0];
    ro0 = p_rres[1];
    const AT rhoT = tw + to, mm = mminor;
    if (ev == 1) {
      sc[0] = (rho[0] + rw0) * irho[0];
      AT d = p_tho * rhoT - ro0;
      const AT cap = rho[1] - mm;
      d = d < cap ? d : cap;
      dtr = d > AT(0.0) ? d : AT(0.0);
      sc[1] = AT(1.0) - dtr * irho[1];
    } else {
      sc[1] = (rho[1] + ro0) * irho[1];
      AT d = p_thw * rhoT - rw0;
      const AT cap = rho[0] - mm;
      d = d < cap ? d : cap;
      dtr = d > AT(0.0) ? d : AT(0.0);
      sc[0] = AT(1.0) - dtr * irho[0];
    }
    for (int a = 0; a < 2; ++a) {
      const AT keep = AT(1.0) - om[a], e = REG ? AT(1.0) : om[a], ra = rho[a];
      AT ua[3], ve[3];
      for (int d = 0; d < 3; ++d) {
        ua[d] = up[d] + F[a][d] * AT(0.5) * irho[a];
        ve[d] = gray ? ua[d] : up[d];
      }
      const AT kf = gray ? AT(1.0) - AT(0.5) * om[a] : AT(1.0);
      AT uF = 0, pl = 0, FL = 0, vsq = 0;
      for (int d = 0; d < 3; ++d) {
        uF += ua[d] * F[a][d];
        pl += ve[d] * L1[a][d];
        FL += F[a][d] * L1[a][d];
        vsq += ve[d] * ve[d];
      }
      const AT *Mv = M2[a];
      const AT Mm[3][3] = {{Mv[0], Mv[3], Mv[4]}, {Mv[3], Mv[1], Mv[5]}, {Mv[4], Mv[5], Mv[2]}};
      AT uMu = 0, aMF = 0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          uMu += ve[i] * Mm[i][j] * ve[j];
          aMF += ua[i] * Mm[i][j] * F[a][j];
        }
      // equilibrium and force parts of A L0 + B.L1 + C:M
      AT phi_a = e * ra * (AT(1.0) - vsq * (AT(0.5) * ics2)) * L0[a] - kf * uF * ics2 * L0[a] +
                     e * ra * pl * ics2 + kf * FL * ics2 + e * ra * uMu * (AT(0.5) * ics4) +
                     kf * aMF * ics4;
      if (REG) {
        const AT *P = Pi[a];
        const AT Pm[3][3] = {{P[0], P[3], P[4]}, {P[3], P[1], P[5]}, {P[4], P[5], P[2]}};
        AT tr = 0, PM = 0, jl = 0;
        for (int i = 0; i < 3; ++i) {
          for (int j = 0; j < 3; ++j) {
            const AT pn = Pm[i][j] - (i == j ? ra * cs2 : AT(0.0)) - ra * ve[i] * ve[j];
            PM += pn * Mm[i][j];
            if (i == j) tr += pn;
          }
          jl += (m[a][i] - ra * ve[i]) * L1[a][i];
        }
        phi_a += keep * (-tr * (AT(0.5) * ics2) * L0[a] + jl * ics2 + PM * (AT(0.5) * ics4));
      } else {
        phi_a += keep * lf[a];
      }
      scb[a] = phi_a;
      L0[a] *= sc[a];
      for (int d = 0; d < 3; ++d) L1[a][d] *= sc[a];
      for (int d = 0; d < 6; ++d) M2[a][d] *= sc[a];
      if (!REG)
        for (int i = 0; i < Q; ++i) lp[REG ? 0 : a][REG ? 0 : i] *= sc[a];
    }
  }

  // reverse sweep; per component the equilibrium velocity ve is u' (pore)
  // or ua (gray), and kf the force term's weight (1 or 1 - omega/2)
  AT rb[2] = {0, 0}, mb[2][3] = {{0, 0, 0}, {0, 0, 0}}, Pb[2][6];
  AT upb[3] = {0, 0, 0}, Fb[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const AT keep = AT(1.0) - om[a], e = REG ? AT(1.0) : om[a];
    const AT ra = rho[a], ir2 = AT(0.5) * irho[a];
    const AT kf = gray ? AT(1.0) - AT(0.5) * om[a] : AT(1.0);
    AT ua[3], ve[3];
    for (int d = 0; d < 3; ++d) {
      ua[d] = up[d] + F[a][d] * ir2;
      ve[d] = gray ? ua[d] : up[d];
    }
    const AT vsq = ve[0] * ve[0] + ve[1] * ve[1] + ve[2] * ve[2];
    const AT *Mv = M2[a];
    const AT Mm[3][3] = {{Mv[0], Mv[3], Mv[4]}, {Mv[3], Mv[1], Mv[5]}, {Mv[4], Mv[5], Mv[2]}};
    AT Fbar[3] = {0, 0, 0}, uab[3] = {0, 0, 0}, veb[3] = {0, 0, 0};
    rb[a] += e * (AT(1.0) - vsq * (AT(0.5) * ics2)) * L0[a];
    const AT vsqb = -e * ra * (AT(0.5) * ics2) * L0[a];
    const AT uFb = -kf * L0[a] * ics2;
    AT pl = 0, pMp = 0;
    for (int d = 0; d < 3; ++d) pl += ve[d] * L1[a][d];
    rb[a] += e * pl * ics2;
    for (int d = 0; d < 3; ++d) {
      veb[d] += e * ra * L1[a][d] * ics2;
      Fbar[d] += kf * L1[a][d] * ics2;
    }
    for (int i = 0; i < 3; ++i) {
      const AT Mu = Mm[i][0] * ve[0] + Mm[i][1] * ve[1] + Mm[i][2] * ve[2];
      pMp += ve[i] * Mu;
      veb[i] += e * ra * Mu * ics4;
      uab[i] += kf * (Mm[i][0] * F[a][0] + Mm[i][1] * F[a][1] + Mm[i][2] * F[a][2]) * ics4;
      Fbar[i] += kf * (Mm[i][0] * ua[0] + Mm[i][1] * ua[1] + Mm[i][2] * ua[2]) * ics4;
    }
    rb[a] += e * pMp * (AT(0.5) * ics4);
    for (int d = 0; d < 6; ++d) Pb[a][d] = 0;
    if (REG) {
      const AT c = keep * (AT(0.5) * ics4), dd = -keep * (AT(0.5) * ics2) * L0[a];
      AT B[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = c * Mm[i][j] + (i == j ? dd : AT(0.0));
      Pb[a][0] = B[0][0]; Pb[a][1] = B[1][1]; Pb[a][2] = B[2][2];
      Pb[a][3] = B[0][1]; Pb[a][4] = B[0][2]; Pb[a][5] = B[1][2];
      AT pBp = 0;
      for (int i = 0; i < 3; ++i) {
        const AT Bu = B[i][0] * ve[0] + B[i][1] * ve[1] + B[i][2] * ve[2];
        pBp += ve[i] * Bu;
        veb[i] += -AT(2.0) * ra * Bu;
      }
      rb[a] += -cs2 * (B[0][0] + B[1][1] + B[2][2]) - pBp;
      // first-order part j^a = m^a - rho^a ve
      AT pj = 0;
      for (int d = 0; d < 3; ++d) {
        const AT jb = keep * L1[a][d] * ics2;
        mb[a][d] += jb;
        pj += ve[d] * jb;
        veb[d] += -ra * jb;
      }
      rb[a] += -pj;
    }
    AT abF = 0;
    for (int d = 0; d < 3; ++d) {
      veb[d] += AT(2.0) * ve[d] * vsqb;
      if (gray) uab[d] += veb[d];
      else upb[d] += veb[d];
      uab[d] += F[a][d] * uFb;
      Fbar[d] += ua[d] * uFb;
      upb[d] += uab[d];
      Fbar[d] += uab[d] * ir2;
      abF += uab[d] * F[a][d];
    }
    rb[a] += -abF * ir2 * irho[a];
    for (int d = 0; d < 3; ++d) Fb[a][d] = Fbar[d];
  }
  {
    AT pu = 0;
    for (int d = 0; d < 3; ++d) pu += upb[d] * up[d];
    for (int a = 0; a < 2; ++a) {
      for (int d = 0; d < 3; ++d) mb[a][d] += om[a] * upb[d] * iD;
      rb[a] += -om[a] * pu * iD;
    }
  }
  // F^a = F_ex^a - (rho^a / rho_t) R u
  AT Rub[3] = {0, 0, 0}, rtb = 0, Fexb[2][3], twb = 0, tob = 0;
  for (int a = 0; a < 2; ++a) {
    AT FR = 0;
    for (int d = 0; d < 3; ++d) {
      Fexb[a][d] = Fb[a][d];
      Rub[d] += -(rho[a] * irt) * Fb[a][d];
      FR += Fb[a][d] * Ru[d];
    }
    rb[a] += -FR * irt;
    rtb += rho[a] * FR * irt * irt;
  }
  AT cRb = 0, bb[3];
  if (tens) {
    cRb = Rub[0] * wv[0] + Rub[1] * wv[1] + Rub[2] * wv[2];
    AT wb[3], ub[3], Kb[3][3];
    for (int i = 0; i < 3; ++i) wb[i] = cR * Rub[i];
    for (int i = 0; i < 3; ++i) {
      ub[i] = K[i][0] * wb[0] + K[i][1] * wb[1] + K[i][2] * wb[2];
      for (int j = 0; j < 3; ++j) Kb[i][j] = wb[i] * u[j];
    }
    for (int i = 0; i < 3; ++i) bb[i] = Ai[i][0] * ub[0] + Ai[i][1] * ub[1] + Ai[i][2] * ub[2];
    AT AK = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const AT Ab = -bb[i] * u[j];
        AK += Ab * K[i][j];
        Kb[i][j] += h * cR * Ab;
        if (i == j) rtb += Ab;
      }
    cRb += h * AK;
    gk[v] = p_gk[0] + Kb[0][0];
    gk[N + v] = p_gk[1] + Kb[1][1];
    gk[2 * N + v] = p_gk[2] + Kb[2][2];
    gk[3 * N + v] = p_gk[3] + (Kb[0][1] + Kb[1][0]);
    gk[4 * N + v] = p_gk[4] + (Kb[0][2] + Kb[2][0]);
    gk[5 * N + v] = p_gk[5] + (Kb[1][2] + Kb[2][1]);
  } else {
    AT Rsb = 0, ub[3];
    for (int d = 0; d < 3; ++d) {
      Rsb += u[d] * Rub[d];
      ub[d] = Rs * Rub[d];
    }
    const AT idn = AT(1.0) / den;
    AT denb = 0;
    for (int d = 0; d < 3; ++d) {
      bb[d] = ub[d] * idn;
      denb += -ub[d] * u[d] * idn;
    }
    rtb += denb;
    Rsb += h * denb;
    if (gray) {
      const AT ik0 = AT(1.0) / k0;
      cRb = Rsb * ik0;
      gk[v] = p_gk[0] + -Rsb * cR * ik0 * ik0;
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d) {
      mb[a][d] += bb[d];
      Fexb[a][d] += h * bb[d];
    }
  // CSF: this voxel's part; dL/dcurv^a and dL/dg^a of the force term are
  // stashed (rows 9, 10 and 11..16) for the normals' and gradients' reverse
  if (mkappa != AT(0.0)) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      AT cb = AT(0.0), gb[3] = {0, 0, 0};
      if (csfv) {
        const AT gFc = cg[a][0] * Fexb[a][0] + cg[a][1] * Fexb[a][1] + cg[a][2] * Fexb[a][2];
        rb[a] += kap * curv[a] * gFc;
        cb = kap * rho[a] * gFc;
        for (int d = 0; d < 3; ++d) gb[d] = kap * curv[a] * rho[a] * Fexb[a][d];
      }
      stash[(size_t)(9 + a) * N + v] = (T)cb;
      for (int d = 0; d < 3; ++d) stash[(size_t)(11 + 3 * a + d) * N + v] = (T)gb[d];
    }
  }
  // F_ex: body force, pseudo-potential force (own part; the neighbours'
  // part is stashed), capillary term
  AT gSb[3] = {0, 0, 0}, Pcb = 0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int b = 1 - a;
    AT gF = 0, aF = 0, gFS = 0;
    for (int d = 0; d < 3; ++d) {
      gF += mg[a][d] * Fexb[a][d];
      aF += acc[a][d] * Fexb[a][d];
      gFS += gS[d] * Fexb[a][d];
    }
    rb[a] += gF - mG * aF;
    const AT accb[3] = {-mG * rho[a] * Fexb[a][0], -mG * rho[a] * Fexb[a][1],
                            -mG * rho[a] * Fexb[a][2]};
    for (int d = 0; d < 3; ++d) stash[(size_t)(3 * a + d) * N + v] = (T)accb[d];
    if (rho[b] + mwd[b] > AT(0.0)) {  // solid links read max(rho^b + dpsi^b, 0)
      AT wsum = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const AT t = (AT)wq(i) * (cx(i) * accb[0] + cy(i) * accb[1] + cz(i) * accb[2]);
        wsum += ((mk >> i) & 1u) ? t : AT(0.0);
      }
      rb[b] += wsum;
    }
    if (gray) {
      Pcb += -(rho[a] * irt) * gFS;
      rb[a] += -Pc * gFS * irt;
      rtb += Pc * rho[a] * gFS * irt * irt;
      for (int d = 0; d < 3; ++d) gSb[d] += -Pc * (rho[a] * irt) * Fexb[a][d];
    }
  }
  if (gray) {
    for (int d = 0; d < 3; ++d) stash[(size_t)(6 + d) * N + v] = (T)gSb[d];
    // c_R
    AT Sb = 0;
    if (S > AT(0.0)) {
      rtb += cRb * S * mnu[0] * ikw;
      Sb += cRb * rt * mnu[0] * ikw;
      if (Krw > mkrmin) Sb += -cRb * rt * S * mnu[0] * ikw * ikw * dKrw;
    }
    if (AT(1.0) - S > AT(0.0)) {
      rtb += cRb * (AT(1.0) - S) * mnu[1] * iko;
      Sb += -cRb * rt * mnu[1] * iko;
      if (Kro > mkrmin) Sb += -cRb * rt * (AT(1.0) - S) * mnu[1] * iko * iko * dKro;
    }
    // P_c = s_J P_c(S)
    gsj[v] = p_gsj + Pcb * Pct;
    Sb += Pcb * sj * dPct;
    if (Sraw > AT(0.0) && Sraw < AT(1.0)) {
      const AT itt = AT(1.0) / (tw + to), sb = Sb * ispan;
      twb += sb * to * itt * itt;
      tob += -sb * tw * itt * itt;
    }
    // grad S_hat: the links to solid neighbours read this voxel's S_hat
    AT shb = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const AT t = (AT)gw(i) * (cx(i) * gSb[0] + cy(i) * gSb[1] + cz(i) * gSb[2]);
      shb += ((mk >> i) & 1u) ? t : AT(0.0);
    }
    rb[0] += shb * ispan * rho[1] * irt * irt;
    rb[1] += -shb * ispan * rho[0] * irt * irt;
  }
  rb[0] += rtb;
  rb[1] += rtb;
  if (gray) {
    // residual amounts: dL/dr after the step comes in, dL/dr before it goes out
    AT rbw = AT(0.0), rbo = AT(0.0);
    const AT lw = (AT)p_lr[0], lo_ = (AT)p_lr[1];
    if (ev) {
      const AT rhoT = tw + to;
      AT db = AT(0.0), rTb = AT(0.0);
      if (ev == 1) {
        rb[0] += scb[0] * (-rw0 * irho[0] * irho[0]);
        rbw += scb[0] * irho[0];
        db += -scb[1] * irho[1];
        rb[1] += scb[1] * dtr * irho[1] * irho[1];
        rbo += lo_;  // r^o <- r^o + d; r^w <- 0
        db += lo_;
        const AT raw = p_tho * rhoT - ro0, cap = rho[1] - mminor;
        if (raw < cap && raw > AT(0.0)) {
          gth[N + v] += db * rhoT;
          rTb += db * p_tho;
          rbo -= db;
        } else if (raw >= cap && cap > AT(0.0)) {
          rb[1] += db;
        }
      } else {
        rb[1] += scb[1] * (-ro0 * irho[1] * irho[1]);
        rbo += scb[1] * irho[1];
        db += -scb[0] * irho[0];
        rb[0] += scb[0] * dtr * irho[0] * irho[0];
        rbw += lw;  // r^w <- r^w + d; r^o <- 0
        db += lw;
        const AT raw = p_thw * rhoT - rw0, cap = rho[0] - mminor;
        if (raw < cap && raw > AT(0.0)) {
          gth[v] += db * rhoT;
          rTb += db * p_thw;
          rbw -= db;
        } else if (raw >= cap && cap > AT(0.0)) {
          rb[0] += db;
        }
      }
      twb += rTb;
      tob += rTb;
    } else {
      rbw += lw;
      rbo += lo_;
    }
    // t_w = rho^w + r^w, t_o = rho^o + r^o
    rb[0] += twb;
    rb[1] += tob;
    lr[v] = rbw + twb;
    lr[N + v] = rbo + tob;
  }

#pragma unroll
  for (int a = 0; a < 2; ++a) {
    T *lo = lout + (size_t)a * Q * N;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      AT l = rb[a];
      if (cx(k)) l += cx(k) * mb[a][0];
      if (cy(k)) l += cy(k) * mb[a][1];
      if (cz(k)) l += cz(k) * mb[a][2];
      if (REG) {
        if (cx(k)) l += Pb[a][0];
        if (cy(k)) l += Pb[a][1];
        if (cz(k)) l += Pb[a][2];
        if (cx(k) && cy(k)) l += (2 * cx(k) * cy(k)) * Pb[a][3];
        if (cx(k) && cz(k)) l += (2 * cx(k) * cz(k)) * Pb[a][4];
        if (cy(k) && cz(k)) l += (2 * cy(k) * cz(k)) * Pb[a][5];
      } else {
        l += (AT(1.0) - om[a]) * lp[REG ? 0 : a][REG ? 0 : k];
      }
      lo[(size_t)k * N + v] = (T)l;
    }
  }
}

// The CSF normals of a level from its density field: per component a the
// gradient g^a of rho^b (b = 1 - a; the voxel's own value across a solid link)
// and n^a = g^a / |g^a| (0 when |g^a| <= eps_n), rows 6a..6a+2 and 6a+3..6a+5.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_normals(const ModelConsts mc,
                                                     const T *__restrict__ rho2,
                                                     const uint32_t *__restrict__ mask,
                                                     T *__restrict__ nrmb) {
  const long long N = mc.N;
  const long long v = xcd_voxel();
  if (v >= N) return;
  const uint32_t mk = mask[v];
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int b = 1 - a;
    double g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const bool wall = (mk >> i) & 1u;
      const size_t y = wall ? (size_t)v : (size_t)nb.at(cx(i), cy(i), cz(i));
      const double r = (double)rho2[2 * y + b];
      if (cx(i)) g0 += gw(i) * cx(i) * r;
      if (cy(i)) g1 += gw(i) * cy(i) * r;
      if (cz(i)) g2 += gw(i) * cz(i) * r;
    }
    const double n2 = g0 * g0 + g1 * g1 + g2 * g2;
    const double in = n2 > mc.eps_n * mc.eps_n ? 1.0 / sqrt(n2) : 0.0;
    const double g[3] = {g0, g1, g2};
    for (int d = 0; d < 3; ++d) {
      nrmb[(size_t)(6 * a + d) * N + v] = (T)g[d];
      nrmb[(size_t)(6 * a + 3 + d) * N + v] = (T)(g[d] * in);
    }
  }
}

// Neighbour sums of the level that the two-component reverse step reads
// (fluid links only; the step adds its solid links from its own values):
// rows 0..2 and 3..5 sum_i w_i c_i rho^b(x + c_i) for the pseudo-potential
// force of component a (b = 1 - a), rows 6..8 sum_i (w_i / cs2) c_i S_hat(x + c_i),
// and (CSF, from the normals) rows 9, 10 curv^a = -div n^a (own normal across
// a solid link).
template <typename T, bool CSF>
__global__ __launch_bounds__(256) void k_adj_inputs2(const ModelConsts mc,
                                                     const T *__restrict__ rho2,
                                                     const T *__restrict__ nrmb,
                                                     const uint32_t *__restrict__ mask,
                                                     T *__restrict__ inb) {
  const long long N = mc.N;
  const long long v = xcd_voxel();
  if (v >= N) return;
  const uint32_t mk = mask[v];
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  double a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const bool wall = (mk >> i) & 1u;
    const size_t y = wall ? (size_t)v : (size_t)nb.at(cx(i), cy(i), cz(i));
    double rw = (double)rho2[2 * y], ro = (double)rho2[2 * y + 1];
    // open x faces: a neighbour beyond a face is the reservoir cell at the
    // face's prescribed densities (as in the forward step)
    if (mc.open_x && cx(i) != 0 && (nb.x + cx(i) < 0 || nb.x + cx(i) >= mc.nx)) {
      rw = cx(i) > 0 ? mc.rho_out[0] : mc.rho_in[0];
      ro = cx(i) > 0 ? mc.rho_out[1] : mc.rho_in[1];
    }
    const double f = wall ? 0.0 : 1.0;
    const double sh = f * (rw / (rw + ro) - mc.s_min) * mc.inv_span;
    const int c[3] = {cx(i), cy(i), cz(i)};
    for (int d = 0; d < 3; ++d) {
      if (!c[d]) continue;
      a0[d] += f * wq(i) * c[d] * ro;  // water's force reads psi^o
      a1[d] += f * wq(i) * c[d] * rw;
      gs[d] += gw(i) * c[d] * sh;
    }
  }
  // (CSF a template switch and every store last: no branch or store between
  // the two groups of gathers)
  double dv[2] = {0, 0};
  if (CSF) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const bool wall = (mk >> i) & 1u;
        const size_t y = wall ? (size_t)v : (size_t)nb.at(cx(i), cy(i), cz(i));
        if (cx(i)) dv[a] += gw(i) * cx(i) * (double)nrmb[(size_t)(6 * a + 3) * N + y];
        if (cy(i)) dv[a] += gw(i) * cy(i) * (double)nrmb[(size_t)(6 * a + 4) * N + y];
        if (cz(i)) dv[a] += gw(i) * cz(i) * (double)nrmb[(size_t)(6 * a + 5) * N + y];
      }
    }
  }
  for (int d = 0; d < 3; ++d) {
    inb[(size_t)d * N + v] = (T)a0[d];
    inb[(size_t)(3 + d) * N + v] = (T)a1[d];
    inb[(size_t)(6 + d) * N + v] = (T)gs[d];
  }
  if (CSF) {
    inb[(size_t)9 * N + v] = (T)(-dv[0]);
    inb[(size_t)10 * N + v] = (T)(-dv[1]);
  }
}

// CSF normals' reverse at a fluid voxel y: dL/dn^a(y) gathered from the
// curvature reads of the voxels x = y - c_i (and of y itself across its solid
// links), carried to dL/dg^a(y) through n = g / |g|, added to the force
// term's own dL/dg^a(y) (stash rows 11..16).  It then leaves the neighbour
// part what it reads: rows 0..5 become rows 0..5 + 3 x rows 11..16, and rows
// 11, 12 this voxel's own solid-link part of each component's sum.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_normals_rev(const ModelConsts mc,
                                                         const T *__restrict__ nrmb,
                                                         const uint32_t *__restrict__ mask,
                                                         T *__restrict__ stash) {
  const long long N = mc.N;
  const long long v = xcd_voxel();
  if (v >= N) return;
  const uint32_t mk = mask[v];
  if (((mk >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  // every load of both components before the first store: the stores go to
  // the same array (rows 11..16), so loads after them could not move ahead
  T cb[2][Q];  // [a][0]: this voxel's curvature adjoint, [a][i]: x = y - c_i's
  double g[2][3], n[2][3], sg[2][3], sp[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    cb[a][0] = stash[(size_t)(9 + a) * N + v];
#pragma unroll
    for (int i = 1; i < Q; ++i) cb[a][i] = stash[(size_t)(9 + a) * N + nb.at(-cx(i), -cy(i), -cz(i))];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g[a][d] = (double)nrmb[(size_t)(6 * a + d) * N + v];
      n[a][d] = (double)nrmb[(size_t)(6 * a + 3 + d) * N + v];
      sg[a][d] = (double)stash[(size_t)(11 + 3 * a + d) * N + v];
      sp[a][d] = (double)stash[(size_t)(3 * a + d) * N + v];  // pseudo-potential rows
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    double nbar[3] = {0, 0, 0};
    const double cbv = (double)cb[a][0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const bool wall = (mk >> i) & 1u;
      // the voxel x = y - c_i read n(y) through its link i; y's own solid
      // links read its own normal
      const double c = (double)cb[a][i] + (wall ? cbv : 0.0);
      if (cx(i)) nbar[0] += -gw(i) * cx(i) * c;
      if (cy(i)) nbar[1] += -gw(i) * cy(i) * c;
      if (cz(i)) nbar[2] += -gw(i) * cz(i) * c;
    }
    const double n2 = g[a][0] * g[a][0] + g[a][1] * g[a][1] + g[a][2] * g[a][2];
    if (n2 > mc.eps_n * mc.eps_n) {
      const double in = 1.0 / sqrt(n2);
      const double nn = n[a][0] * nbar[0] + n[a][1] * nbar[1] + n[a][2] * nbar[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) sg[a][d] = (double)(T)(sg[a][d] + (nbar[d] - nn * n[a][d]) * in);
    }
  }
  // The neighbours' part reads, per link, the pseudo-potential row and the
  // density-gradient row of the same component with weights w_i and
  // w_i / cs2 = 3 w_i: it gets their sum (rows 0..5 <- rows 0..5 + 3 rows
  // 11..16) and, in rows 11 and 12, this voxel's own part, the sum over its
  // solid links (the gradient's read of its own density; links whose other
  // end lies across an open face are not taken) of (w_i / cs2) c_i . row.
  double own[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const bool across = mc.open_x && cx(i) != 0 && (nb.x - cx(i) < 0 || nb.x - cx(i) >= mc.nx);
    if (!((mk >> i) & 1u) || across) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      double t = 0;
      if (cx(i)) t += cx(i) * sg[a][0];
      if (cy(i)) t += cy(i) * sg[a][1];
      if (cz(i)) t += cz(i) * sg[a][2];
      own[a] += gw(i) * t;
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
      stash[(size_t)(3 * a + d) * N + v] = (T)(sp[a][d] + 3.0 * sg[a][d]);
    stash[(size_t)(11 + a) * N + v] = (T)own[a];
  }
}

// The neighbours' part of the force's reverse: dL/drho^b(y) from the
// pseudo-potential reads of every fluid voxel x = y - c_i, dL/drho^w,o(y)
// through S_hat(y) from the saturation-gradient reads of gray voxels, and
// (CSF) dL/drho^b(y) from the density-gradient reads behind the normals and
// the force term (own value across a solid link).
// Every neighbour value is loaded without a branch between the loads (the
// open-face and solid-link cases select their terms afterwards), so a wave
// keeps all its gathers in flight instead of waiting on each direction's.
template <typename T, bool CSF>
__global__ __launch_bounds__(256) void k_adj_nl2(const ModelConsts mc,
                                                 const T *__restrict__ rho2,
                                                 const T *__restrict__ stash,
                                                 const uint32_t *__restrict__ mask,
                                                 T *__restrict__ rnl) {
  const long long N = mc.N;
  const long long v = xcd_voxel();
  if (v >= N) return;
  if (((mask[v] >> CLASS_SHIFT) & 3u) == SOLID_CODE) return;  // stays zero
  const Nbr nb((int)v, mc.nx, mc.ny, mc.nz);
  // (CSF) the normals' reverse has added 3 x the density-gradient rows to the
  // pseudo-potential rows (both read with w_i and w_i / cs2 = 3 w_i) and left
  // this voxel's solid-link part in rows 11 and 12
  const double own1 = CSF ? (double)stash[(size_t)11 * N + v] : 0.0;
  const double own0 = CSF ? (double)stash[(size_t)12 * N + v] : 0.0;
  double r0 = 0, r1 = 0, shb = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    // open x faces: the voxel x - c_i across a face read a reservoir cell, not x
    const bool across = mc.open_x && cx(i) != 0 && (nb.x - cx(i) < 0 || nb.x - cx(i) >= mc.nx);
    const size_t x = (size_t)nb.at(-cx(i), -cy(i), -cz(i));
    auto dot = [&](int c0, size_t at) {
      double s = 0;
      if (cx(i)) s += cx(i) * (double)stash[(size_t)c0 * N + at];
      if (cy(i)) s += cy(i) * (double)stash[(size_t)(c0 + 1) * N + at];
      if (cz(i)) s += cz(i) * (double)stash[(size_t)(c0 + 2) * N + at];
      return s;
    };
    const double d0 = dot(0, x), d3 = dot(3, x), d6 = dot(6, x);
    // water's force reads psi^o (and, CSF, g^w = grad rho^o), oil's psi^w
    // (g^o = grad rho^w)
    r1 = across ? r1 : r1 + wq(i) * d0;
    r0 = across ? r0 : r0 + wq(i) * d3;
    shb = across ? shb : shb + gw(i) * d6;
  }
  r1 += own1;
  r0 += own0;
  const double aw = (double)rho2[2 * v], ao = (double)rho2[2 * v + 1];
  const double tt = aw + ao, span = 1.0 / mc.inv_span;
  rnl[2 * v] = (T)(r0 + shb / span * ao / (tt * tt));
  rnl[2 * v + 1] = (T)(r1 - shb / span * aw / (tt * tt));
}

// d theta / d s_J of a residual saturation: theta is the smallest S* where
// s_J P_c(S*) = target on the piecewise-linear table, so on the crossed cell
// (k-1, k) dS*/ds_J = target / (s_J^2 (P_c[k-1] - P_c[k])) / (TABLE_N - 1);
// zero where the curve never reaches the target or already starts below it.
__device__ inline double dcross_dsj(const double *pc, double sj, double target) {
  const int n = TABLE_N - 1;
  if (sj * pc[0] < target || sj * pc[n] > target) return 0.0;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sj * pc[mid] <= target) hi = mid;
    else lo = mid + 1;
  }
  if (lo == 0) return 0.0;
  return target / (sj * sj * (pc[lo - 1] - pc[lo])) / (double)n;
}

// dL/dphi on gray voxels: dL/dK0 times the K0(phi) table's slope on the
// lookup's cell, plus (two components) dL/ds_J, with the residual
// saturations' dL/dtheta_w (at c_max Pc_PM) and dL/dtheta_o (at c_min Pc_PM,
// theta_o = 1 - S*) carried to s_J, through
// s_J = sqrt((K0_ref / phi_ref) phi / K0(phi)), plus (tensor) the transposed
// smoothing's result gbase (the porosity field the smoothing read is phi
// there).  gbase, gsj and gth may be null.
__global__ __launch_bounds__(256) void k_adj_phi2(const double *__restrict__ gbase,
                                                  const double *__restrict__ gK0,
                                                  const double *__restrict__ gsj,
                                                  const double *__restrict__ gth,
                                                  const double *__restrict__ phi,
                                                  const uint8_t *__restrict__ pt,
                                                  const uint32_t *__restrict__ mask,
                                                  const double *__restrict__ tabs,
                                                  const double *__restrict__ tabmeta,
                                                  double c_max, double c_min, long long N,
                                                  double *__restrict__ out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  if (((mask[v] >> CLASS_SHIFT) & 3u) != GRAY_CODE) {
    out[v] = 0.0;
    return;
  }
  const int ty = pt[v];
  const double *tab = tabs + (size_t)ty * 4 * TABLE_N;
  const double ph = phi[v];
  const double t = ph * (double)(TABLE_N - 1);
  int k = (int)floor(t);
  k = k > TABLE_N - 2 ? TABLE_N - 2 : (k < 0 ? 0 : k);
  const double slope = (tab[k + 1] - tab[k]) * (double)(TABLE_N - 1);
  const double k0 = lerp_tab<double>(tab, ph);
  const double phi_ref = tabmeta[ty * 8 + 0];
  const double k0ref = lerp_tab<double>(tab, phi_ref);
  const double sj = sqrt((k0ref / phi_ref) / (k0 / ph));
  const double dsj = 0.5 * sj * (1.0 / ph - slope / k0);
  double gs = gsj ? gsj[v] : 0.0;
  if (gth) {
    const double pcpm = tabmeta[ty * 8 + 1];
    const double *pc = tab + TABLE_N;
    gs += gth[v] * dcross_dsj(pc, sj, c_max * pcpm) - gth[N + v] * dcross_dsj(pc, sj, c_min * pcpm);
  }
  out[v] = (gbase ? gbase[v] : 0.0) + gK0[v] * slope + gs * dsj;
}

// ---------------------------------------------------------------------------
// Tensorial resistivity: dL/dK^-1 back to the smoothed porosity.
//
// The set-up (Eqs. (6)-(7)) builds, per gray voxel, the gradient g and Hessian
// H of the smoothed porosity p_s, the eigenpairs (lambda_k, e_k) of H ordered by
// |lambda|, and K^-1 = sum_k d_k e_k e_k^T with d_k = 1 / (a_k K0).  Away from
// the switches (the isotropic gate, the ordering, the tie test) its derivative
// is, with G the symmetric dL/dK^-1 (an off-diagonal stored component split
// over its two entries):
//   K0        dL/dK0 = -G : K^-1 / K0;
//   axes      dL/dH = sum_{j != k} (e_j^T G e_k)(d_k - d_j) / (lambda_k - lambda_j)
//             e_j e_k^T (first-order eigenvector perturbation);
//   tie-break (the two smallest |lambda| within delta_tie |lambda_3|, second axis
//             along p = g - (g.e_3) e_3): K^-1 = d_1 I + (d_2 - d_1) e_2 e_2^T
//             + (d_3 - d_1) e_3 e_3^T with e_2 = p / |p|, so the sweep runs back
//             through the normalisation and the projection to dL/dg and to
//             dL/de_3, and e_3's perturbation to dL/dH;
//   gate      K^-1 = I / K0: no dependence on p_s.
// Output per gray voxel hb[9][v]: dL/dH_xx, _yy, _zz, _xy, _xz, _yz (the
// off-diagonal ones standing for both entries), dL/dg_x, _y, _z; zero
// elsewhere.  gK0[v] receives dL/dK0.
__global__ __launch_bounds__(256) void k_adj_axes(const double *__restrict__ ps,
                                                  const uint32_t *__restrict__ mask,
                                                  const uint8_t *__restrict__ pt,
                                                  const double *__restrict__ phi,
                                                  const double *__restrict__ tabs,
                                                  const double *__restrict__ tabmeta, int nx,
                                                  int ny, int nz, long long N, double eps_g,
                                                  double eps_H, double delta_tie,
                                                  const double *__restrict__ gKi,
                                                  double *__restrict__ hb,
                                                  double *__restrict__ gK0) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  if (((mask[v] >> CLASS_SHIFT) & 3u) != GRAY_CODE) {
    for (int c = 0; c < 9; ++c) hb[(size_t)c * N + v] = 0.0;
    gK0[v] = 0.0;
    return;
  }
  const Nbr nb((int)v, nx, ny, nz);
  auto P = [&](int dx, int dy, int dz) { return ps[nb.at(dx, dy, dz)]; };
  const double p0 = P(0, 0, 0);
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double g[3], H[3][3];
  for (int a = 0; a < 3; ++a) {
    const int *ea = off[a];
    const double pp = P(ea[0], ea[1], ea[2]);
    const double pm = P(-ea[0], -ea[1], -ea[2]);
    g[a] = 0.5 * (pp - pm);
    H[a][a] = pp - 2.0 * p0 + pm;
    for (int b = a + 1; b < 3; ++b) {
      const int *eb = off[b];
      const double v_pp = P(ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2]);
      const double v_pm = P(ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]);
      const double v_mp = P(-ea[0] + eb[0], -ea[1] + eb[1], -ea[2] + eb[2]);
      const double v_mm = P(-ea[0] - eb[0], -ea[1] - eb[1], -ea[2] - eb[2]);
      H[a][b] = H[b][a] = 0.25 * (v_pp - v_pm - v_mp + v_mm);
    }
  }
  const int t = pt[v];
  const double k0 = lerp_tab<double>(tabs + (size_t)t * 4 * TABLE_N, phi[v]);
  const double kd[3] = {tabmeta[t * 8 + 2], tabmeta[t * 8 + 3], tabmeta[t * 8 + 4]};
  double G[3][3];
  G[0][0] = gKi[v];
  G[1][1] = gKi[N + v];
  G[2][2] = gKi[2 * N + v];
  G[0][1] = G[1][0] = 0.5 * gKi[3 * N + v];
  G[0][2] = G[2][0] = 0.5 * gKi[4 * N + v];
  G[1][2] = G[2][1] = 0.5 * gKi[5 * N + v];
  double A[3][3], E[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = H[i][j];
  jacobi3(A, E);
  const double lam[3] = {A[0][0], A[1][1], A[2][2]};
  const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const double amax = fmax(fabs(lam[0]), fmax(fabs(lam[1]), fabs(lam[2])));
  double Hb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, gb[3] = {0, 0, 0};
  double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (amax <= eps_H && gn <= eps_g) {
    for (int i = 0; i < 3; ++i) M[i][i] = 1.0 / k0;
  } else {
    int ord[3] = {0, 1, 2};  // stable sort by |lambda|, as the set-up
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && fabs(lam[ord[j]]) < fabs(lam[ord[j - 1]]); --j) {
        const int tmp = ord[j];
        ord[j] = ord[j - 1];
        ord[j - 1] = tmp;
      }
    double e[3][3], l[3], d[3];
    for (int k = 0; k < 3; ++k) {
      for (int c = 0; c < 3; ++c) e[k][c] = E[c][ord[k]];
      l[k] = lam[ord[k]];
      d[k] = 1.0 / (kd[k] * k0);
    }
    const double a0 = fabs(l[0]), a1 = fabs(l[1]), a2 = fabs(l[2]);
    bool tied = false;
    double e2[3], pn = 0.0, pv[3] = {0, 0, 0};
    if (a1 - a0 <= delta_tie * a2) {
      const double ge3 = g[0] * e[2][0] + g[1] * e[2][1] + g[2] * e[2][2];
      for (int c = 0; c < 3; ++c) pv[c] = g[c] - ge3 * e[2][c];
      pn = sqrt(pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2]);
      tied = pn > eps_g;
    }
    if (!tied) {
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) M[i][j] += d[k] * e[k][i] * e[k][j];
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
          if (j == k || l[k] == l[j]) continue;
          double Gjk = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Gjk += e[j][a] * G[a][b] * e[k][b];
          const double c = Gjk * (d[k] - d[j]) / (l[k] - l[j]);
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Hb[a][b] += c * e[j][a] * e[k][b];
        }
    } else {
      for (int c = 0; c < 3; ++c) e2[c] = pv[c] / pn;
      const double *e3 = e[2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          M[i][j] = (i == j ? d[0] : 0.0) + (d[1] - d[0]) * e2[i] * e2[j] +
                    (d[2] - d[0]) * e3[i] * e3[j];
      double eb2[3], eb3[3];
      for (int i = 0; i < 3; ++i) {
        eb2[i] = 2.0 * (d[1] - d[0]) * (G[i][0] * e2[0] + G[i][1] * e2[1] + G[i][2] * e2[2]);
        eb3[i] = 2.0 * (d[2] - d[0]) * (G[i][0] * e3[0] + G[i][1] * e3[1] + G[i][2] * e3[2]);
      }
      // e2 = p / |p|
      const double s2 = eb2[0] * e2[0] + eb2[1] * e2[1] + eb2[2] * e2[2];
      double pb[3];
      for (int c = 0; c < 3; ++c) pb[c] = (eb2[c] - s2 * e2[c]) / pn;
      // p = g - (g.e3) e3
      const double pe3 = pb[0] * e3[0] + pb[1] * e3[1] + pb[2] * e3[2];
      const double ge3 = g[0] * e3[0] + g[1] * e3[1] + g[2] * e3[2];
      for (int c = 0; c < 3; ++c) {
        gb[c] = pb[c] - pe3 * e3[c];
        eb3[c] += -pe3 * g[c] - ge3 * pb[c];
      }
      // e3 = the eigenvector of the largest |lambda|
      for (int j = 0; j < 2; ++j) {
        if (l[2] == l[j]) continue;
        const double c =
            (eb3[0] * e[j][0] + eb3[1] * e[j][1] + eb3[2] * e[j][2]) / (l[2] - l[j]);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) Hb[a][b] += c * e[j][a] * e3[b];
      }
    }
  }
  double gk0 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) gk0 -= G[i][j] * M[i][j];
  gK0[v] = gk0 / k0;
  hb[v] = Hb[0][0];
  hb[N + v] = Hb[1][1];
  hb[2 * N + v] = Hb[2][2];
  hb[3 * N + v] = Hb[0][1] + Hb[1][0];
  hb[4 * N + v] = Hb[0][2] + Hb[2][0];
  hb[5 * N + v] = Hb[1][2] + Hb[2][1];
  hb[6 * N + v] = gb[0];
  hb[7 * N + v] = gb[1];
  hb[8 * N + v] = gb[2];
}

// Transpose of the gradient and Hessian stencils: dL/dp_s at y gathers the
// stencil coefficients of every voxel whose g or H read p_s(y).
__global__ __launch_bounds__(256) void k_adj_hess_t(const double *__restrict__ hb, int nx,
                                                    int ny, int nz, long long N,
                                                    double *__restrict__ out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const Nbr nb((int)v, nx, ny, nz);
  auto B = [&](int c, int dx, int dy, int dz) { return hb[(size_t)c * N + nb.at(dx, dy, dz)]; };
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double acc = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int *ea = off[a];
    acc += 0.5 * (B(6 + a, -ea[0], -ea[1], -ea[2]) - B(6 + a, ea[0], ea[1], ea[2]));
    acc += B(a, -ea[0], -ea[1], -ea[2]) - 2.0 * B(a, 0, 0, 0) + B(a, ea[0], ea[1], ea[2]);
  }
  const int pair[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int q = 0; q < 3; ++q) {
    const int *ea = off[pair[q][0]], *eb = off[pair[q][1]];
    const int c = 3 + q;
    acc += 0.25 * (B(c, -ea[0] - eb[0], -ea[1] - eb[1], -ea[2] - eb[2]) -
                   B(c, -ea[0] + eb[0], -ea[1] + eb[1], -ea[2] + eb[2]) -
                   B(c, ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]) +
                   B(c, ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2]));
  }
  out[v] = acc;
}

}  // namespace adj
}  // namespace lbm

// ------------------------------------------------------------------ host side
namespace {

template <typename T, bool REG, bool TENS>
void launch_adj_step_t(lbm_handle *h, const T *post, const T *lin, T *lout, double *gk,
                       double a) {
  DevState<T> &s = state<T>(h);
  const unsigned nb = (blocks(h->N) + 7) / 8 * 8;
  hipLaunchKernelGGL((adj::k_adj_step<T, REG, TENS>), dim3(nb), dim3(256), 0, h->st, h->mc, post,
                     lin, lout, s.mask, s.K0, (const T *)s.Kinv, gk, a);
}

// Buffers of the two-component reverse: the level's density field, residual
// amounts and side flags, the neighbour-part stash and gathers, dL/dr, and the
// s_J and theta accumulators.
template <typename T>
struct Rev2 {
  T *dens, *stash, *rnl_in, *rnl_out, *nrmb, *inb;
  const T *r;
  const uint8_t *side;
  double *gsj, *lr, *gth;
};

// blocks of 256 for n threads, rounded up to a multiple of 8 (xcd_voxel)
unsigned blocks8(long long n) { return (blocks(n) + 7) / 8 * 8; }

template <typename T, bool REG, bool TENS>
void launch_adj_step2_t(lbm_handle *h, const T *post, const T *lin, T *lout, double *gk,
                        double a, const Rev2<T> &b) {
  DevState<T> &s = state<T>(h);
  const unsigned nb = (blocks(h->N) + 7) / 8 * 8;
  // fp32 storage reverses in fp32 arithmetic (the accumulators stay fp64)
  hipLaunchKernelGGL((adj::k_adj_step2<T, REG, TENS, T>), dim3(nb), dim3(256), 0, h->st, h->mc,
                     post, (const T *)b.dens, b.r, b.side, (const T *)b.nrmb,
                     (const T *)b.inb, lin,
                     (const T *)b.rnl_in, lout,
                     b.stash, s.mask, s.K0, (const T *)s.Kinv, s.sJ, (const T *)s.thw,
                     (const T *)s.tho, s.ptype, s.tab, gk, b.gsj, b.lr, b.gth, a);
}

// One reverse step: one component, or (two components) the density pass of
// the level, the local reverse and the gather of the neighbours' part.
// With pressure reservoirs, res holds the step's boundary densities and
// velocities (k_res_record).
template <typename T>
void launch_reverse(lbm_handle *h, const T *post, const T *lin, T *lout, double *gk, double a,
                    const Rev2<T> &b, const double *res) {
  DevState<T> &s = state<T>(h);
  const bool reg = h->p.collision == LBM_COLL_REGULARIZED;
  const bool ten = h->p.tensor != 0;
  const unsigned rb = blocks((long long)h->p.ny * h->p.nz);
  if (h->p.ncomp == 1) {
    Timed tm(h, K_ADJ);
    if (h->mc.exact_density)
      hipLaunchKernelGGL((adj::k_adj_density_faces<T>), dim3(blocks(2LL * h->p.ny * h->p.nz)),
                         dim3(256), 0, h->st, h->mc, const_cast<T *>(lin), (T *)nullptr, s.mask);
    else if (res)
      hipLaunchKernelGGL((adj::k_adj_reservoirs<T>), dim3(rb), dim3(256), 0, h->st, h->mc,
                         const_cast<T *>(lin), (const T *)nullptr, s.mask, res);
    if (ten) {
      if (reg) launch_adj_step_t<T, true, true>(h, post, lin, lout, gk, a);
      else launch_adj_step_t<T, false, true>(h, post, lin, lout, gk, a);
    } else {
      if (reg) launch_adj_step_t<T, true, false>(h, post, lin, lout, gk, a);
      else launch_adj_step_t<T, false, false>(h, post, lin, lout, gk, a);
    }
    return;
  }
  if (h->mc.exact_density) {
    Timed tm(h, K_ADJ);
    hipLaunchKernelGGL((adj::k_adj_density_faces<T>), dim3(blocks(2LL * h->p.ny * h->p.nz)),
                       dim3(256), 0, h->st, h->mc, const_cast<T *>(lin), b.rnl_in, s.mask);
  } else if (res) {
    Timed tm(h, K_ADJ);
    hipLaunchKernelGGL((adj::k_adj_reservoirs<T>), dim3(rb), dim3(256), 0, h->st, h->mc,
                       const_cast<T *>(lin), (const T *)b.rnl_in, s.mask, res);
  }
  {
    Timed tm(h, K_AUX);
    hipLaunchKernelGGL((k_density<T, 2, SK_NATIVE, false>), dim3(blocks(h->N)), dim3(256), 0,
                       h->st, (const void *)post, b.dens, (const T *)nullptr, (const T *)nullptr,
                       s.mask, h->p.nx, h->p.ny, h->p.nz, h->N);
  }
  {
    Timed tm(h, K_AUX);
    if (h->p.kappa != 0.0)
      hipLaunchKernelGGL((adj::k_adj_normals<T>), dim3(blocks8(h->N)), dim3(256), 0, h->st,
                         h->mc, (const T *)b.dens, s.mask, b.nrmb);
    if (h->p.kappa != 0.0)
      hipLaunchKernelGGL((adj::k_adj_inputs2<T, true>), dim3(blocks8(h->N)), dim3(256), 0, h->st,
                         h->mc, (const T *)b.dens, (const T *)b.nrmb, s.mask, b.inb);
    else
      hipLaunchKernelGGL((adj::k_adj_inputs2<T, false>), dim3(blocks8(h->N)), dim3(256), 0,
                         h->st, h->mc, (const T *)b.dens, (const T *)b.nrmb, s.mask, b.inb);
  }
  Timed tm(h, K_ADJ);
  if (ten) {
    if (reg) launch_adj_step2_t<T, true, true>(h, post, lin, lout, gk, a, b);
    else launch_adj_step2_t<T, false, true>(h, post, lin, lout, gk, a, b);
  } else {
    if (reg) launch_adj_step2_t<T, true, false>(h, post, lin, lout, gk, a, b);
    else launch_adj_step2_t<T, false, false>(h, post, lin, lout, gk, a, b);
  }
  if (h->p.kappa != 0.0)
    hipLaunchKernelGGL((adj::k_adj_normals_rev<T>), dim3(blocks8(h->N)), dim3(256), 0, h->st,
                       h->mc, (const T *)b.nrmb, s.mask, b.stash);
  if (h->p.kappa != 0.0)
    hipLaunchKernelGGL((adj::k_adj_nl2<T, true>), dim3(blocks8(h->N)), dim3(256), 0, h->st, h->mc,
                       (const T *)b.dens, (const T *)b.stash, s.mask, b.rnl_out);
  else
    hipLaunchKernelGGL((adj::k_adj_nl2<T, false>), dim3(blocks8(h->N)), dim3(256), 0, h->st,
                       h->mc, (const T *)b.dens, (const T *)b.stash, s.mask, b.rnl_out);
}

// The fused step from fin into fout (two components: after the density pass
// of fin into the handle's density buffer).
// Two components: the residual amounts and side flags of the new level (rout,
// sout, which hold a copy of the old level's on entry) are updated in place by
// the step, through the handle's state pointers swapped for the launch.
template <typename T>
void launch_recompute(lbm_handle *h, const T *fin, T *fout, T *rout = nullptr,
                      uint8_t *sout = nullptr) {
  DevState<T> &s = state<T>(h);
  const bool reg = h->p.collision == LBM_COLL_REGULARIZED;
  if (h->p.ncomp == 2) {
    {
      Timed tm(h, K_AUX);
      hipLaunchKernelGGL((k_density<T, 2, SK_NATIVE, false>), dim3(blocks(h->N)), dim3(256), 0,
                         h->st, (const void *)fin, s.rho2, (const T *)nullptr, (const T *)nullptr,
                         s.mask, h->p.nx, h->p.ny, h->p.nz, h->N);
    }
    T *const r_own = s.r;
    uint8_t *const s_own = s.side;
    s.r = rout;
    s.side = sout;
    {
      Timed tm(h, K_STEP);
      if (reg) launch_tiled<T, 2, true>(h, fin, fout);
      else launch_tiled<T, 2, false>(h, fin, fout);
    }
    s.r = r_own;
    s.side = s_own;
    if (h->mc.exact_density)
      hipLaunchKernelGGL((k_density_faces<T, 2>), dim3(blocks(2LL * h->p.ny * h->p.nz)), dim3(256),
                         0, h->st, h->mc, fout, s.mask);
    else if (h->mc.open_x)
      hipLaunchKernelGGL((k_reservoirs<T, 2>), dim3(blocks((long long)h->p.ny * h->p.nz)),
                         dim3(256), 0, h->st, h->mc, fout, s.mask);
    return;
  }
  Timed tm(h, K_STEP);
  if (reg) launch_tiled<T, 1, true>(h, fin, fout);
  else launch_tiled<T, 1, false>(h, fin, fout);
  if (h->mc.exact_density)  // the face populations, as the step applies them
    hipLaunchKernelGGL((k_density_faces<T, 1>), dim3(blocks(2LL * h->p.ny * h->p.nz)), dim3(256), 0,
                       h->st, h->mc, fout, s.mask);
  else if (h->mc.open_x)
    hipLaunchKernelGGL((k_reservoirs<T, 1>), dim3(blocks((long long)h->p.ny * h->p.nz)),
                       dim3(256), 0, h->st, h->mc, fout, s.mask);
}

// dL/dK^-1 (tensor runs) back to dL/dK0 and to the porosity through the
// set-up: the smoothed porosity is rebuilt with the set-up's own kernels, the
// axes kernel turns dL/dK^-1 into dL/dH, dL/dg and dL/dK0, then the transposed
// stencils and the transposed smoothing (a symmetric periodic convolution per
// axis, applied in the reverse axis order) carry dL/dH and dL/dg back to the
// porosity field (gbase).
template <typename T>
int tensor_gradient(lbm_handle *h, const double *gKi, double *gK0, double *gbase,
                    std::vector<void *> &tmp) {
  DevState<T> &s = state<T>(h);
  const long long N = h->N;
  const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
  bool ok = true;
  double *sm1 = alloc_into<double>(h, tmp, (size_t)N, &ok);
  double *hb = alloc_into<double>(h, tmp, (size_t)9 * N, &ok);
  double *wts = alloc_into<double>(h, tmp, 32, &ok);
  if (!ok) return set_err(h, LBM_E_NOMEM, "device allocation failed in adjoint_flux");
  const int R = h->p.smooth_radius;
  std::vector<double> w(2 * R + 1);
  double sum = 0.0;
  for (int j = -R; j <= R; ++j) {
    w[j + R] = std::exp(-(double)(j * j) / (2.0 * h->p.sigma_s * h->p.sigma_s));
    sum += w[j + R];
  }
  for (double &x : w) x /= sum;
  int rc = hip_check(h, hipMemcpyAsync(wts, w.data(), w.size() * sizeof(double),
                                       hipMemcpyHostToDevice, h->st),
                     "copy smoothing weights");
  // w is host staging for that copy and ends with this function
  if (rc == LBM_OK) rc = hip_check(h, hipStreamSynchronize(h->st), "copy smoothing weights");
  if (rc != LBM_OK) return rc;
  const dim3 gr(blocks(N)), bl(256);
  double *sm2 = gbase;
  Timed tm(h, K_OTHER);
  hipLaunchKernelGGL(k_base_phi, gr, bl, 0, h->st, s.mask, h->geom_phi, sm1, N);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm1, sm2, nx, ny, nz, N, 0, R, wts);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm2, sm1, nx, ny, nz, N, 1, R, wts);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm1, sm2, nx, ny, nz, N, 2, R, wts);
  hipLaunchKernelGGL(adj::k_adj_axes, gr, bl, 0, h->st, sm2, s.mask, s.ptype, h->geom_phi,
                     h->geom_tabs, h->geom_meta, nx, ny, nz, N, h->p.eps_g, h->p.eps_H,
                     h->p.delta_tie, gKi, hb, gK0);
  hipLaunchKernelGGL(adj::k_adj_hess_t, gr, bl, 0, h->st, hb, nx, ny, nz, N, sm1);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm1, sm2, nx, ny, nz, N, 2, R, wts);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm2, sm1, nx, ny, nz, N, 1, R, wts);
  hipLaunchKernelGGL(k_smooth, gr, bl, 0, h->st, sm1, sm2, nx, ny, nz, N, 0, R, wts);
  return hip_check(h, hipGetLastError(), "tensor gradient kernels");
}

// Forward sweep: nsteps ordinary steps of the handle, the stored set copied
// into a checkpoint at the start of every segment of K steps and the outlet
// flux of every step recorded on the device.  Reverse sweep, segment by
// segment from the last: the segment's stored sets are recomputed from its
// checkpoint with the same fused step into a scratch ring, then the reverse
// step runs from the segment's last step down to its first.
template <typename T>
int adjoint_t(lbm_handle *h, int64_t n, const double *dLdQ, int64_t K, double *Qout,
              double *gK0_out, double *gphi_out) {
  DevState<T> &s = state<T>(h);
  const long long N = h->N;
  const int nc = h->p.ncomp;
  const size_t SN = (size_t)nc * Q * N;  // one population set
  if (K <= 0) K = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)n)));
  K = std::min<int64_t>(K, n);
  const int64_t nseg = (n + K - 1) / K;
  std::vector<void *> tmp;
  bool ok = true;
  T *ck = alloc_into<T>(h, tmp, (size_t)nseg * SN, &ok);
  T *ring = K > 1 ? alloc_into<T>(h, tmp, (size_t)(K - 1) * SN, &ok) : nullptr;
  T *lam = alloc_into<T>(h, tmp, 2 * SN, &ok);
  const size_t ngk = h->p.tensor ? (size_t)6 * N : (size_t)N;  // dL/dK^-1 or dL/dK0
  double *gk = alloc_into<double>(h, tmp, ngk, &ok);
  double *gk0 = h->p.tensor ? alloc_into<double>(h, tmp, (size_t)N, &ok) : gk;
  double *gbase = h->p.tensor ? alloc_into<double>(h, tmp, (size_t)N, &ok) : nullptr;
  double *gp = alloc_into<double>(h, tmp, (size_t)N, &ok);
  double *qh = alloc_into<double>(h, tmp, (size_t)2 * n, &ok);
  // pressure reservoirs: every step's boundary densities and velocities
  const size_t RR = (size_t)8 * h->p.ny * h->p.nz;
  double *resv = h->mc.open_x && !h->mc.exact_density
                     ? alloc_into<double>(h, tmp, (size_t)n * RR, &ok) : nullptr;
  // two components: the residual amounts and side flags of every kept level
  // (checkpoints and ring, like the populations), the reverse's buffers
  T *dens = nullptr, *stash = nullptr, *rnl = nullptr, *ckR = nullptr, *ringR = nullptr,
    *nrmb = nullptr, *inb = nullptr;
  const int nstash = h->p.kappa != 0.0 ? 17 : 9;
  uint8_t *ckS = nullptr, *ringS = nullptr;
  double *gsj = nullptr, *lr = nullptr, *gth = nullptr;
  if (nc == 2) {
    dens = alloc_into<T>(h, tmp, (size_t)2 * N, &ok);
    stash = alloc_into<T>(h, tmp, (size_t)nstash * N, &ok);
    if (h->p.kappa != 0.0) nrmb = alloc_into<T>(h, tmp, (size_t)12 * N, &ok);
    inb = alloc_into<T>(h, tmp, (size_t)11 * N, &ok);
    rnl = alloc_into<T>(h, tmp, (size_t)4 * N, &ok);
    ckR = alloc_into<T>(h, tmp, (size_t)nseg * 2 * N, &ok);
    ckS = alloc_into<uint8_t>(h, tmp, (size_t)nseg * N, &ok);
    if (K > 1) {
      ringR = alloc_into<T>(h, tmp, (size_t)(K - 1) * 2 * N, &ok);
      ringS = alloc_into<uint8_t>(h, tmp, (size_t)(K - 1) * N, &ok);
    }
    gsj = alloc_into<double>(h, tmp, (size_t)N, &ok);
    lr = alloc_into<double>(h, tmp, (size_t)2 * N, &ok);
    gth = alloc_into<double>(h, tmp, (size_t)2 * N, &ok);
  }
  auto finish = [&](int rc) {
    h->res_rec = nullptr;
    (void)hipStreamSynchronize(h->st);
    for (void *p : tmp) dev_free(h, p);
    return rc;
  };
  if (!ok) return finish(set_err(h, LBM_E_NOMEM, "device allocation failed in adjoint_flux"));
  const unsigned fb = blocks((long long)h->p.ny * h->p.nz);
  int rc = LBM_OK;
  // the step stores nothing for a wave of solid voxels, so the ring's slots
  // of those voxels keep what the allocation held; the reservoirs read a solid
  // boundary voxel's set (its velocity is m * 0), so with them the ring starts
  // at zero, like the handle's own sets
  if (resv && ring)
    rc = hip_check(h, hipMemsetAsync(ring, 0, (size_t)(K - 1) * SN * sizeof(T), h->st),
                   "clear the ring");
  const size_t RB = (size_t)2 * N * sizeof(T);  // residual amounts of one level
  auto copy_rs = [&](T *rdst, uint8_t *sdst, const T *rsrc, const uint8_t *ssrc) {
    int e = hip_check(h, hipMemcpyAsync(rdst, rsrc, RB, hipMemcpyDeviceToDevice, h->st),
                      "copy residual amounts");
    if (e == LBM_OK)
      e = hip_check(h, hipMemcpyAsync(sdst, ssrc, (size_t)N, hipMemcpyDeviceToDevice, h->st),
                    "copy side flags");
    return e;
  };
  // every level's densities come from the density pass, in the forward sweep
  // as in its recomputations, so both give the same sets
  h->rho2_valid = false;
  // forward sweep.  The last segment keeps its levels: each of its steps but
  // the last writes its new set straight into the ring (the handle's buffer
  // pointers are swapped for it and put back at the end), so that segment is
  // not recomputed, and checkpoint_every = nsteps recomputes nothing.
  T *const own0 = s.f[0], *const own1 = s.f[1];
  h->res_rec = resv;
  for (int64_t sg = 0; sg < nseg && rc == LBM_OK; ++sg) {
    rc = hip_check(h, hipMemcpyAsync(ck + sg * SN, s.f[h->cur], SN * sizeof(T),
                                     hipMemcpyDeviceToDevice, h->st),
                   "checkpoint copy");
    if (rc == LBM_OK && nc == 2)
      rc = copy_rs(ckR + (size_t)sg * 2 * N, ckS + (size_t)sg * N, s.r, s.side);
    const int64_t m = std::min<int64_t>(K, n - sg * K);
    const bool keep = sg == nseg - 1;
    T *const spare = s.f[1 - h->cur];
    for (int64_t k = 0; k < m && rc == LBM_OK; ++k) {
      if (keep) s.f[1 - h->cur] = k < m - 1 ? ring + k * SN : spare;
      rc = step_t<T>(h, 1, false);
      if (rc != LBM_OK) break;
      Timed tm(h, K_OTHER);
      if (nc == 2)
        hipLaunchKernelGGL((k_flux<T, 2>), dim3(fb), dim3(256), 0, h->st, h->mc, s.f[h->cur],
                           s.mask, s.partial, pop_layout<T>(h));
      else
        hipLaunchKernelGGL((k_flux<T, 1>), dim3(fb), dim3(256), 0, h->st, h->mc, s.f[h->cur],
                           s.mask, s.partial, pop_layout<T>(h));
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, h->st, s.partial, (int)fb, 2, 0,
                         qh + 2 * (sg * K + k), 0);
      if (keep && nc == 2 && k < m - 1)
        rc = copy_rs(ringR + (size_t)k * 2 * N, ringS + (size_t)k * N, s.r, s.side);
    }
    if (keep) {
      if (rc == LBM_OK) {  // the final set is in `spare`, one of the handle's buffers
        s.f[1 - h->cur] = s.f[h->cur] == own0 ? own1 : own0;
      } else {  // a failed step: the handle's buffers come back, the state is lost
        s.f[0] = own0;
        s.f[1] = own1;
        h->has_fluid = false;
      }
    }
  }
  h->res_rec = nullptr;
  // reverse sweep; the loss does not depend on the set after the last step
  if (rc == LBM_OK)
    rc = hip_check(h, hipMemsetAsync(lam, 0, 2 * SN * sizeof(T), h->st), "clear adjoint");
  if (rc == LBM_OK)
    rc = hip_check(h, hipMemsetAsync(gk, 0, ngk * sizeof(double), h->st), "clear gradient");
  if (rc == LBM_OK && nc == 2) {
    rc = hip_check(h, hipMemsetAsync(rnl, 0, (size_t)4 * N * sizeof(T), h->st), "clear");
    if (rc == LBM_OK)
      rc = hip_check(h, hipMemsetAsync(stash, 0, (size_t)nstash * N * sizeof(T), h->st), "clear");
    if (rc == LBM_OK && nrmb)
      rc = hip_check(h, hipMemsetAsync(nrmb, 0, (size_t)12 * N * sizeof(T), h->st), "clear");
    if (rc == LBM_OK)
      rc = hip_check(h, hipMemsetAsync(gsj, 0, (size_t)N * sizeof(double), h->st), "clear");
    if (rc == LBM_OK)
      rc = hip_check(h, hipMemsetAsync(lr, 0, (size_t)2 * N * sizeof(double), h->st), "clear");
    if (rc == LBM_OK)
      rc = hip_check(h, hipMemsetAsync(gth, 0, (size_t)2 * N * sizeof(double), h->st), "clear");
  }
  int cl = 0;
  for (int64_t sg = nseg - 1; sg >= 0 && rc == LBM_OK; --sg) {
    const int64_t m = std::min<int64_t>(K, n - sg * K);
    auto level = [&](int64_t k) -> T * { return k == 0 ? ck + sg * SN : ring + (k - 1) * SN; };
    auto levelR = [&](int64_t k) -> T * {
      return k == 0 ? ckR + (size_t)sg * 2 * N : ringR + (size_t)(k - 1) * 2 * N;
    };
    auto levelS = [&](int64_t k) -> uint8_t * {
      return k == 0 ? ckS + (size_t)sg * N : ringS + (size_t)(k - 1) * N;
    };
    if (sg < nseg - 1)
      for (int64_t k = 1; k < m && rc == LBM_OK; ++k) {
        if (nc == 2) {
          rc = copy_rs(levelR(k), levelS(k), levelR(k - 1), levelS(k - 1));
          if (rc == LBM_OK) launch_recompute<T>(h, level(k - 1), level(k), levelR(k), levelS(k));
        } else {
          launch_recompute<T>(h, level(k - 1), level(k));
        }
      }
    for (int64_t k = m - 1; k >= 0 && rc == LBM_OK; --k) {
      Rev2<T> b{};
      if (nc == 2) {
        b.dens = dens;
        b.stash = stash;
        b.nrmb = nrmb;
        b.inb = inb;
        b.rnl_in = rnl + (size_t)cl * 2 * N;
        b.rnl_out = rnl + (size_t)(1 - cl) * 2 * N;
        b.r = levelR(k);
        b.side = levelS(k);
        b.gsj = gsj;
        b.lr = lr;
        b.gth = gth;
      }
      launch_reverse<T>(h, level(k), lam + cl * SN, lam + (1 - cl) * SN, gk, dLdQ[sg * K + k], b,
                        resv ? resv + (size_t)(sg * K + k) * RR : nullptr);
      cl = 1 - cl;
    }
    rc = hip_check(h, hipGetLastError(), "adjoint launches");
  }
  // the recomputation used the handle's density buffer
  h->rho2_valid = false;
  if (rc == LBM_OK && h->p.tensor) rc = tensor_gradient<T>(h, gk, gk0, gbase, tmp);
  if (rc == LBM_OK) {
    Timed tm(h, K_OTHER);
    hipLaunchKernelGGL(adj::k_adj_phi2, dim3(blocks(N)), dim3(256), 0, h->st,
                       (const double *)gbase, (const double *)gk0, (const double *)gsj,
                       (const double *)gth, h->geom_phi, s.ptype, s.mask, h->geom_tabs,
                       h->geom_meta, h->p.c_max, h->p.c_min, N, gp);
    rc = hip_check(h, hipGetLastError(), "gradient kernel");
  }
  std::vector<double> qv;
  if (rc == LBM_OK && Qout) {
    qv.resize((size_t)2 * n);
    rc = hip_check(h, hipMemcpyAsync(qv.data(), qh, qv.size() * sizeof(double),
                                     hipMemcpyDeviceToHost, h->st),
                   "copy flux history");
  }
  if (rc == LBM_OK && gK0_out)
    rc = hip_check(h, hipMemcpyAsync(gK0_out, gk0, (size_t)N * sizeof(double),
                                     hipMemcpyDeviceToHost, h->st),
                   "copy dL/dK0");
  if (rc == LBM_OK && gphi_out)
    rc = hip_check(h, hipMemcpyAsync(gphi_out, gp, (size_t)N * sizeof(double),
                                     hipMemcpyDeviceToHost, h->st),
                   "copy dL/dphi");
  if (rc == LBM_OK) rc = hip_check(h, hipStreamSynchronize(h->st), "adjoint");
  if (rc == LBM_OK && Qout)
    for (int64_t k = 0; k < n; ++k) Qout[k] = qv[(size_t)2 * k];
  return finish(rc);
}

}  // namespace

extern "C" int lbm_adjoint_flux(lbm_handle *h, int64_t nsteps, const double *dL_dQ,
                                int64_t checkpoint_every, double *Q_out, double *dL_dK0,
                                double *dL_dphi) {
  const Range range("lbm_adjoint_flux");
  if (!h) return LBM_E_INVAL;
  if (nsteps < 1 || !dL_dQ || checkpoint_every < 0)
    return set_err(h, LBM_E_INVAL, "adjoint_flux: need nsteps >= 1, dL_dQ, checkpoint_every >= 0");
  for (int64_t k = 0; k < nsteps; ++k)
    if (!std::isfinite(dL_dQ[k]))
      return set_err(h, LBM_E_INVAL, "adjoint_flux: non-finite dL_dQ");
  if (h->sk != SK_NATIVE)
    return set_err(h, LBM_E_UNSUPPORTED, "adjoint_flux: native fp64 or fp32 storage only");
  if (!h->has_geom || !h->has_fluid) return set_err(h, LBM_E_STATE, "adjoint_flux: no fluid state");
  // the sweeps keep whole population sets (checkpoints, ring): dense layout
  // for their duration
  const bool fluid_only = h->compact;
  int rc = fluid_only ? set_layout_t<float>(h, false) : LBM_OK;
  if (rc != LBM_OK) return rc;
  rc = h->es == 8 ? adjoint_t<double>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi)
                  : adjoint_t<float>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi);
  if (fluid_only) {
    const int rc2 = set_layout_t<float>(h, true);
    if (rc == LBM_OK) rc = rc2;
  }
  return dcheck(h, rc);
}
