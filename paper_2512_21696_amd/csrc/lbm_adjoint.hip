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
template <typename T, bool REG>
__global__ __launch_bounds__(256) void k_adj_step(const ModelConsts mc,
                                                  const T *__restrict__ post,
                                                  const T *__restrict__ lin,
                                                  T *__restrict__ lout,
                                                  const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ K0,
                                                  double *__restrict__ gK0, const double a) {
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
  const double k0 = gray ? (double)K0[v] : 1.0;
  const double r = gray ? mc.nu[0] / k0 : 0.0;
  const double Rs = rho * r, den = rho + h * Rs;
  const double u0 = (m0 + h * rho * g0) / den, u1 = (m1 + h * rho * g1) / den,
               u2 = (m2 + h * rho * g2) / den;
  const double F0 = rho * g0 - Rs * u0, F1 = rho * g1 - Rs * u1, F2 = rho * g2 - Rs * u2;
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
  // F = rho g - R_s u
  rb += g0 * Fb0 + g1 * Fb1 + g2 * Fb2;
  double Rsb = -(u0 * Fb0 + u1 * Fb1 + u2 * Fb2);
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
  if (gray) gK0[v] += -(r / k0) * (rho * Rsb);
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

}  // namespace adj
}  // namespace lbm

// ------------------------------------------------------------------ host side
namespace {

template <typename T>
void launch_adj_step(lbm_handle *h, const T *post, const T *lin, T *lout, double *gk,
                     double a) {
  DevState<T> &s = state<T>(h);
  Timed tm(h, K_ADJ);
  const unsigned nb = (blocks(h->N) + 7) / 8 * 8;
  if (h->p.collision == LBM_COLL_REGULARIZED)
    hipLaunchKernelGGL((adj::k_adj_step<T, true>), dim3(nb), dim3(256), 0, h->st, h->mc, post, lin,
                       lout, s.mask, s.K0, gk, a);
  else
    hipLaunchKernelGGL((adj::k_adj_step<T, false>), dim3(nb), dim3(256), 0, h->st, h->mc, post,
                       lin, lout, s.mask, s.K0, gk, a);
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
  double *gk = alloc_into<double>(h, tmp, (size_t)N, &ok);
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
    rc = hip_check(h, hipMemsetAsync(gk, 0, (size_t)N * sizeof(double), h->st), "clear gradient");
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
  if (rc == LBM_OK) {
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
    rc = hip_check(h, hipMemcpyAsync(gK0_out, gk, (size_t)N * sizeof(double),
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
  if (h->p.ncomp != 1 || h->p.tensor || h->mc.open_x || h->sk != SK_NATIVE)
    return set_err(h, LBM_E_UNSUPPORTED,
                   "adjoint_flux: one component, scalar K0, periodic x faces and native storage "
                   "only");
  if (!h->has_geom || !h->has_fluid) return set_err(h, LBM_E_STATE, "adjoint_flux: no fluid state");
  return h->es == 8 ? adjoint_t<double>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi)
                    : adjoint_t<float>(h, nsteps, dL_dQ, checkpoint_every, Q_out, dL_dK0, dL_dphi);
}
