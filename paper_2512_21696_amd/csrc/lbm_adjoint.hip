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
//             u = (m + h rho g) / (rho + h R_s), F = rho g - R_s u,
//             h = 1/2 (semi-implicit) or 1 (implicit);
//   collision post_i = w_i (A + B.c_i + c_i^T C c_i) with u' = m / rho,
//             ua = u' + F / (2 rho), omega = 1 / tau and
//               equilibrium  A = e rho (1 - u'.u' / 2cs2), B = e rho u' / cs2,
//                            C = e rho u' u'^T / 2cs4,
//               force (Eq. (3))  A = -ua.F / cs2, B = F / cs2,
//                            C = (ua F^T + F ua^T) / 2cs4,
//               regularised non-equilibrium  A = -(1 - omega) tr P / 2cs2,
//                            C = (1 - omega) P / 2cs4, P = Pi - rho cs2 I - rho u' u'^T,
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

  double lp[Q];
  double rho = 0, m0 = 0, m1 = 0, m2 = 0;
  double L0 = 0, L1x = 0, L1y = 0, L1z = 0;
  double Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int j = opp(i);
    const double fi = (double)(((mk >> j) & 1u)
                                   ? post[(size_t)j * N + v]
                                   : post[(size_t)i * N + nb.at(-cx(i), -cy(i), -cz(i))]);
    const bool wall = (mk >> i) & 1u;
    double l = (double)(wall ? lin[(size_t)j * N + v]
                             : lin[(size_t)i * N + nb.at(cx(i), cy(i), cz(i))]);
    if (!wall && at0 && cx(i) == 1) l += a;
    if (!wall && at1 && cx(i) == -1) l -= a;
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
  const double cs2 = CS2, cs4 = CS2 * CS2;
  const double om = mc.omega[0], keep = 1.0 - om, e = REG ? 1.0 : om;
  const double h = mc.res_implicit ? 1.0 : 0.5;
  const double g0 = mc.g[0][0], g1 = mc.g[0][1], g2 = mc.g[0][2];
  const bool tens = TENS && gray;
  const double b0 = m0 + h * rho * g0, b1 = m1 + h * rho * g1, b2 = m2 + h * rho * g2;
  double k0 = 1.0, r = 0.0, Rs = 0.0, den = rho, cR = 0.0;
  double K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Ai[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double u0, u1, u2, F0, F1, F2, w0 = 0, w1 = 0, w2 = 0;
  if (tens) {
    cR = rho * mc.nu[0];
    K[0][0] = (double)Kinv[v];
    K[1][1] = (double)Kinv[N + v];
    K[2][2] = (double)Kinv[2 * N + v];
    K[0][1] = K[1][0] = (double)Kinv[3 * N + v];
    K[0][2] = K[2][0] = (double)Kinv[4 * N + v];
    K[1][2] = K[2][1] = (double)Kinv[5 * N + v];
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
  const double usq = p0 * p0 + p1 * p1 + p2 * p2;
  const double a0 = p0 + 0.5 * F0 * ir, a1 = p1 + 0.5 * F1 * ir, a2 = p2 + 0.5 * F2 * ir;  // ua

  // reverse sweep of Phi
  double rb = 0, pb0 = 0, pb1 = 0, pb2 = 0, Fb0 = 0, Fb1 = 0, Fb2 = 0, ab0 = 0, ab1 = 0, ab2 = 0;
  // A terms
  rb += e * (1.0 - usq / (2 * cs2)) * L0;
  const double usqb = -e * rho / (2 * cs2) * L0;
  const double uFb = -L0 / cs2;
  // B terms
  rb += e * (p0 * L1x + p1 * L1y + p2 * L1z) / cs2;
  pb0 += e * rho * L1x / cs2; pb1 += e * rho * L1y / cs2; pb2 += e * rho * L1z / cs2;
  Fb0 += L1x / cs2; Fb1 += L1y / cs2; Fb2 += L1z / cs2;
  // C terms (M = Lambda2, symmetric)
  const double Mp0 = Mxx * p0 + Mxy * p1 + Mxz * p2;
  const double Mp1 = Mxy * p0 + Myy * p1 + Myz * p2;
  const double Mp2 = Mxz * p0 + Myz * p1 + Mzz * p2;
  rb += e * (p0 * Mp0 + p1 * Mp1 + p2 * Mp2) / (2 * cs4);
  pb0 += e * rho * Mp0 / cs4; pb1 += e * rho * Mp1 / cs4; pb2 += e * rho * Mp2 / cs4;
  ab0 += (Mxx * F0 + Mxy * F1 + Mxz * F2) / cs4;
  ab1 += (Mxy * F0 + Myy * F1 + Myz * F2) / cs4;
  ab2 += (Mxz * F0 + Myz * F1 + Mzz * F2) / cs4;
  Fb0 += (Mxx * a0 + Mxy * a1 + Mxz * a2) / cs4;
  Fb1 += (Mxy * a0 + Myy * a1 + Myz * a2) / cs4;
  Fb2 += (Mxz * a0 + Myz * a1 + Mzz * a2) / cs4;
  // regularised non-equilibrium: dPhi/dP, which is also dPhi/dPi
  double Bxx = 0, Byy = 0, Bzz = 0, Bxy = 0, Bxz = 0, Byz = 0;
  if (REG) {
    const double c = keep / (2 * cs4), d = -keep / (2 * cs2) * L0;
    Bxx = c * Mxx + d; Byy = c * Myy + d; Bzz = c * Mzz + d;
    Bxy = c * Mxy; Bxz = c * Mxz; Byz = c * Myz;
    const double Bp0 = Bxx * p0 + Bxy * p1 + Bxz * p2;
    const double Bp1 = Bxy * p0 + Byy * p1 + Byz * p2;
    const double Bp2 = Bxz * p0 + Byz * p1 + Bzz * p2;
    rb += -cs2 * (Bxx + Byy + Bzz) - (p0 * Bp0 + p1 * Bp1 + p2 * Bp2);
    pb0 -= 2 * rho * Bp0; pb1 -= 2 * rho * Bp1; pb2 -= 2 * rho * Bp2;
  }
  // ua.F
  ab0 += F0 * uFb; ab1 += F1 * uFb; ab2 += F2 * uFb;
  Fb0 += a0 * uFb; Fb1 += a1 * uFb; Fb2 += a2 * uFb;
  // ua = u' + F / 2rho
  pb0 += ab0; pb1 += ab1; pb2 += ab2;
  Fb0 += 0.5 * ab0 * ir; Fb1 += 0.5 * ab1 * ir; Fb2 += 0.5 * ab2 * ir;
  rb -= 0.5 * (ab0 * F0 + ab1 * F1 + ab2 * F2) * ir * ir;
  // u'.u'
  pb0 += 2 * p0 * usqb; pb1 += 2 * p1 * usqb; pb2 += 2 * p2 * usqb;
  // u' = m / rho
  double mb0 = pb0 * ir, mb1 = pb1 * ir, mb2 = pb2 * ir;
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
    gk[v] += Kb[0][0];
    gk[NN + v] += Kb[1][1];
    gk[2 * NN + v] += Kb[2][2];
    gk[3 * NN + v] += Kb[0][1] + Kb[1][0];
    gk[4 * NN + v] += Kb[0][2] + Kb[2][0];
    gk[5 * NN + v] += Kb[1][2] + Kb[2][1];
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

// dL/dphi = dL/dK0 * dK0/dphi on gray voxels: the slope of the linear
// interpolation in the K0(phi) table, on the same table cell as the lookup.
__global__ __launch_bounds__(256) void k_adj_phi(const double *__restrict__ gK0,
                                                 const double *__restrict__ phi,
                                                 const uint8_t *__restrict__ pt,
                                                 const uint32_t *__restrict__ mask,
                                                 const double *__restrict__ tabs, long long N,
                                                 double *__restrict__ out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  if (((mask[v] >> CLASS_SHIFT) & 3u) != GRAY_CODE) {
    out[v] = 0.0;
    return;
  }
  const double *tab = tabs + (size_t)pt[v] * 4 * TABLE_N;  // curve 0 of each type is K0
  const double t = phi[v] * (double)(TABLE_N - 1);
  int k = (int)floor(t);
  k = k > TABLE_N - 2 ? TABLE_N - 2 : (k < 0 ? 0 : k);
  out[v] = gK0[v] * (tab[k + 1] - tab[k]) * (double)(TABLE_N - 1);
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

// dL/dphi on gray voxels with the tensor: the transposed smoothing's result
// (the porosity field the smoothing read is phi there) plus dL/dK0 times the
// K0 table's slope.
__global__ __launch_bounds__(256) void k_adj_phi_tensor(const double *__restrict__ gbase,
                                                        const double *__restrict__ gK0,
                                                        const double *__restrict__ phi,
                                                        const uint8_t *__restrict__ pt,
                                                        const uint32_t *__restrict__ mask,
                                                        const double *__restrict__ tabs,
                                                        long long N, double *__restrict__ out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  if (((mask[v] >> CLASS_SHIFT) & 3u) != GRAY_CODE) {
    out[v] = 0.0;
    return;
  }
  const double *tab = tabs + (size_t)pt[v] * 4 * TABLE_N;
  const double t = phi[v] * (double)(TABLE_N - 1);
  int k = (int)floor(t);
  k = k > TABLE_N - 2 ? TABLE_N - 2 : (k < 0 ? 0 : k);
  out[v] = gbase[v] + gK0[v] * (tab[k + 1] - tab[k]) * (double)(TABLE_N - 1);
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

template <typename T>
void launch_adj_step(lbm_handle *h, const T *post, const T *lin, T *lout, double *gk,
                     double a) {
  Timed tm(h, K_ADJ);
  const bool reg = h->p.collision == LBM_COLL_REGULARIZED;
  if (h->p.tensor) {
    if (reg) launch_adj_step_t<T, true, true>(h, post, lin, lout, gk, a);
    else launch_adj_step_t<T, false, true>(h, post, lin, lout, gk, a);
  } else {
    if (reg) launch_adj_step_t<T, true, false>(h, post, lin, lout, gk, a);
    else launch_adj_step_t<T, false, false>(h, post, lin, lout, gk, a);
  }
}

// dL/dK^-1 (tensor runs) back to dL/dK0 and dL/dphi: the smoothed porosity is
// rebuilt with the set-up's own kernels, the axes kernel turns dL/dK^-1 into
// dL/dH, dL/dg and dL/dK0, then the transposed stencils and the transposed
// smoothing (a symmetric periodic convolution per axis, applied in the reverse
// axis order) carry dL/dH and dL/dg back to the porosity.
template <typename T>
int tensor_gradient(lbm_handle *h, const double *gKi, double *gK0, double *gphi,
                    std::vector<void *> &tmp) {
  DevState<T> &s = state<T>(h);
  const long long N = h->N;
  const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
  bool ok = true;
  double *sm1 = alloc_into<double>(h, tmp, (size_t)N, &ok);
  double *sm2 = alloc_into<double>(h, tmp, (size_t)N, &ok);
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
  if (rc != LBM_OK) return rc;
  const dim3 gr(blocks(N)), bl(256);
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
  hipLaunchKernelGGL(adj::k_adj_phi_tensor, gr, bl, 0, h->st, sm2, gK0, h->geom_phi, s.ptype,
                     s.mask, h->geom_tabs, N, gphi);
  return hip_check(h, hipGetLastError(), "tensor gradient kernels");
}

template <typename T>
void launch_recompute(lbm_handle *h, const T *fin, T *fout) {
  Timed tm(h, K_STEP);
  if (h->p.collision == LBM_COLL_REGULARIZED) launch_tiled<T, 1, true>(h, fin, fout);
  else launch_tiled<T, 1, false>(h, fin, fout);
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
  const size_t QN = (size_t)Q * N;
  if (K <= 0) K = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)n)));
  K = std::min<int64_t>(K, n);
  const int64_t nseg = (n + K - 1) / K;
  std::vector<void *> tmp;
  bool ok = true;
  T *ck = alloc_into<T>(h, tmp, (size_t)nseg * QN, &ok);
  T *ring = K > 1 ? alloc_into<T>(h, tmp, (size_t)(K - 1) * QN, &ok) : nullptr;
  T *lam = alloc_into<T>(h, tmp, 2 * QN, &ok);
  const size_t ngk = h->p.tensor ? (size_t)6 * N : (size_t)N;  // dL/dK^-1 or dL/dK0
  double *gk = alloc_into<double>(h, tmp, ngk, &ok);
  double *gk0 = h->p.tensor ? alloc_into<double>(h, tmp, (size_t)N, &ok) : gk;
  double *gp = alloc_into<double>(h, tmp, (size_t)N, &ok);
  double *qh = alloc_into<double>(h, tmp, (size_t)2 * n, &ok);
  auto finish = [&](int rc) {
    (void)hipStreamSynchronize(h->st);
    for (void *p : tmp) dev_free(h, p);
    return rc;
  };
  if (!ok) return finish(set_err(h, LBM_E_NOMEM, "device allocation failed in adjoint_flux"));
  const unsigned fb = blocks((long long)h->p.ny * h->p.nz);
  int rc = LBM_OK;
  // forward sweep.  The last segment keeps its levels: each of its steps but
  // the last writes its new set straight into the ring (the handle's buffer
  // pointers are swapped for it and put back at the end), so that segment is
  // not recomputed, and checkpoint_every = nsteps recomputes nothing.
  T *const own0 = s.f[0], *const own1 = s.f[1];
  for (int64_t sg = 0; sg < nseg && rc == LBM_OK; ++sg) {
    rc = hip_check(h, hipMemcpyAsync(ck + sg * QN, s.f[h->cur], QN * sizeof(T),
                                     hipMemcpyDeviceToDevice, h->st),
                   "checkpoint copy");
    const int64_t m = std::min<int64_t>(K, n - sg * K);
    const bool keep = sg == nseg - 1;
    T *const spare = s.f[1 - h->cur];
    for (int64_t k = 0; k < m && rc == LBM_OK; ++k) {
      if (keep) s.f[1 - h->cur] = k < m - 1 ? ring + k * QN : spare;
      rc = step_t<T>(h, 1);
      if (rc != LBM_OK) break;
      Timed tm(h, K_OTHER);
      hipLaunchKernelGGL((k_flux<T, 1>), dim3(fb), dim3(256), 0, h->st, h->mc, s.f[h->cur],
                         s.mask, s.partial);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, h->st, s.partial, (int)fb, 2, 0,
                         qh + 2 * (sg * K + k), 0);
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
  // reverse sweep; the loss does not depend on the set after the last step
  if (rc == LBM_OK)
    rc = hip_check(h, hipMemsetAsync(lam, 0, 2 * QN * sizeof(T), h->st), "clear adjoint");
  if (rc == LBM_OK)
    rc = hip_check(h, hipMemsetAsync(gk, 0, ngk * sizeof(double), h->st), "clear gradient");
  int cl = 0;
  for (int64_t sg = nseg - 1; sg >= 0 && rc == LBM_OK; --sg) {
    const int64_t m = std::min<int64_t>(K, n - sg * K);
    auto level = [&](int64_t k) -> T * { return k == 0 ? ck + sg * QN : ring + (k - 1) * QN; };
    if (sg < nseg - 1)
      for (int64_t k = 1; k < m; ++k) launch_recompute<T>(h, level(k - 1), level(k));
    for (int64_t k = m - 1; k >= 0; --k) {
      launch_adj_step<T>(h, level(k), lam + cl * QN, lam + (1 - cl) * QN, gk, dLdQ[sg * K + k]);
      cl = 1 - cl;
    }
    rc = hip_check(h, hipGetLastError(), "adjoint launches");
  }
  if (rc == LBM_OK && h->p.tensor) {
    rc = tensor_gradient<T>(h, gk, gk0, gp, tmp);
  } else if (rc == LBM_OK) {
    Timed tm(h, K_OTHER);
    hipLaunchKernelGGL(adj::k_adj_phi, dim3(blocks(N)), dim3(256), 0, h->st, gk, h->geom_phi,
                       s.ptype, s.mask, h->geom_tabs, N, gp);
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
  if (!h) return LBM_E_INVAL;
  if (nsteps < 1 || !dL_dQ || checkpoint_every < 0)
    return set_err(h, LBM_E_INVAL, "adjoint_flux: need nsteps >= 1, dL_dQ, checkpoint_every >= 0");
  for (int64_t k = 0; k < nsteps; ++k)
    if (!std::isfinite(dL_dQ[k]))
      return set_err(h, LBM_E_INVAL, "adjoint_flux: non-finite dL_dQ");
  if (h->p.ncomp != 1 || h->mc.open_x || h->sk != SK_NATIVE)
    return set_err(h, LBM_E_UNSUPPORTED,
                   "adjoint_flux: one component, periodic x faces and native storage only");
  if (!h->has_geom || !h->has_fluid) return set_err(h, LBM_E_STATE, "adjoint_flux: no fluid state");
  return h->es == 8 ? adjoint_t<double>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi)
                    : adjoint_t<float>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi);
}
