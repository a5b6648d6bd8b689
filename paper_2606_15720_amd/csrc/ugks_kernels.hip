// gfx950 kernels of the UGKS phase-space step (staged form).
//
// Each kernel is one numbered part of the one-step algorithm (Sec. 2.2) for
// the BGK-Shakhov model of Sec. 2.1.  Velocity is the fast (lane) index:
// h is stored [cell][k] with k contiguous, so every per-(cell, velocity)
// kernel issues coalesced 64-lane loads and stores, and every per-face or
// per-cell quantity (geometry, interface coefficients) is wave-uniform.
// Sums over velocity use wave shuffles plus LDS in a fixed order, so the
// results are deterministic.
#include "ugks_device.h"

namespace ugks {

using namespace dev;

namespace {

// ---------------------------------------------------------------------------
template <int D>
__global__ void k_prims(int64_t nc, GasP g, const double* __restrict__ W, double* __restrict__ prim,
                        int32_t* flag, int check) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nc) return;
  if (check && *flag) return;
  bool ok = prim_of<D>(&W[i * (D + 2)], g, &prim[i * NPRIM]);
  if (!ok) atomicOr(flag, 1);
}

// Heat flux q_i = 1/2 sum_k w_k c_k (|c_k|^2 h_ik + b_ik), c = u - U_i.
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_heatflux(DevVel v, const T* __restrict__ h,
                                                  const T* __restrict__ b,
                                                  const double* __restrict__ prim,
                                                  double* __restrict__ q, const int32_t* flag) {
  __shared__ double lds[3 * 16];
  if (*flag) return;
  const int64_t i = blockIdx.x;
  const double* P = &prim[i * NPRIM];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < v.nvp; k += TPB) {
    double c[3], c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      c[d] = v.u[d * v.nvp + k] - P[1 + d];
      c2 += c[d] * c[d];
    }
    double hv = ld(h, i * v.nvp + k);
    double bv = v.has_b ? ld(b, i * v.nvp + k) : 0.0;
    double s = v.w[k] * (c2 * hv + bv);
    for (int d = 0; d < D; ++d) acc[d] += s * c[d];
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) q[i * 3 + d] = d < D ? 0.5 * acc[d] : 0.0;
  }
}

// Venkatakrishnan's limiter factor of one cell field (Sec. 2.1 reconstruction
// with an optional limiter): vi is the cell's value, [vmin, vmax] the range
// of the cell and its stencil values, g its least-squares gradient.  At each
// face d- = g.(x_f - x_i) and d+ the room left toward the bound on its side;
// psi = (d+^2 + eps^2 + 2 d- d+) / (d+^2 + 2 d-^2 + d- d+ + eps^2); the
// factor is min(1, min_faces psi).
template <int D>
__device__ __forceinline__ double venkat_phi(const DevMesh& m, int64_t i, int nfc, double vi,
                                             double vmin, double vmax, const double* g) {
  const double eps2 = m.veps2[i];
  double phi = 1.0;
  for (int p = 0; p < nfc; ++p) {
    const int f = m.cface[i * MAXF + p];
    const double* dx = m.csign[i * MAXF + p] > 0.0 ? &m.fdxL[f * 3] : &m.fdxR[f * 3];
    double dm = 0.0;
    for (int d = 0; d < D; ++d) dm += g[d] * dx[d];
    if (dm == 0.0) continue;
    const double dp = dm > 0.0 ? vmax - vi : vmin - vi;
    const double psi = (dp * dp + eps2 + 2.0 * dm * dp) / (dp * dp + 2.0 * dm * dm + dm * dp + eps2);
    phi = fmin(phi, psi);
  }
  return phi;
}

// Macroscopic least-squares gradients of W (step 4).
template <int D>
__device__ __forceinline__ void gradW_at(int64_t i, const DevMesh& m, const DevBC* __restrict__ bcs,
                                         const GasP& g, const double* __restrict__ W,
                                         double* __restrict__ gW, const int32_t* flag) {
  if (*flag) return;
  const int nfc = m.nfc[i];
  const double* Wi = &W[i * (D + 2)];
  double acc[3][5], vmin[5], vmax[5];
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 5; ++v) acc[d][v] = 0.0;
  for (int v = 0; v < D + 2; ++v) vmin[v] = vmax[v] = Wi[v];
  for (int p = 0; p < nfc; ++p) {
    const int f = m.cface[i * MAXF + p];
    const int j = m.cnbr[i * MAXF + p];
    double nb[5];
    if (j >= 0) {
      for (int v = 0; v < D + 2; ++v) nb[v] = W[(int64_t)j * (D + 2) + v];
    } else if (m.fbc[f] == UGKS_BC_WALL) {
      for (int v = 0; v < D + 2; ++v) nb[v] = Wi[v];
    } else {
      ghost_state<D>(m.fbc[f], bcs[m.fbcid[f]], &m.fnorm[f * 3], Wi, g.R, g.K, nb);
    }
    for (int v = 0; v < D + 2; ++v) {
      vmin[v] = fmin(vmin[v], nb[v]);
      vmax[v] = fmax(vmax[v], nb[v]);
    }
    for (int d = 0; d < D; ++d) {
      const double G = m.lsG[(i * 3 + d) * MAXF + p];
      for (int v = 0; v < D + 2; ++v) acc[d][v] += G * (nb[v] - Wi[v]);
    }
  }
  if (m.limiter)
    for (int v = 0; v < D + 2; ++v) {
      double gv[3] = {acc[0][v], acc[1][v], acc[2][v]};
      const double phi = venkat_phi<D>(m, i, nfc, Wi[v], vmin[v], vmax[v], gv);
      for (int d = 0; d < D; ++d) acc[d][v] *= phi;
    }
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 5; ++v) gW[(i * 3 + d) * 5 + v] = (d < D && v < D + 2) ? acc[d][v] : 0.0;
}

template <int D>
__global__ void k_gradW(DevMesh m, const DevBC* __restrict__ bcs, GasP g, const double* __restrict__ W,
                        double* __restrict__ gW, const int32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < m.nc) gradW_at<D>(i, m, bcs, g, W, gW, flag);
}

// Interface equilibrium data of every face (steps 6.1-6.6), wall Maxwellian
// data of wall faces.
template <int D>
__device__ __forceinline__ void face_eq_at(int64_t f, const DevMesh& m, const DevBC* __restrict__ bcs,
                                           const GasP& g, const double* __restrict__ W,
                                           const double* __restrict__ gW,
                                           const double* __restrict__ q, double* __restrict__ frec,
                                           int32_t* flag) {
  if (*flag) return;
  double* R = &frec[f * FREC];
  const int kind = m.fbc[f];
  const int L = m.fL[f];
  if (kind == UGKS_BC_WALL) {
    const DevBC& bc = bcs[m.fbcid[f]];
    double lamw = 1.0 / (2.0 * g.R * bc.T);
    R[FR_C0] = maxw_norm<D>(lamw);
    R[FR_LAM] = lamw;
    for (int d = 0; d < 3; ++d) R[FR_U + d] = d < D ? bc.U[d] : 0.0;
    // free transport of the incident member over the step (h_f - t u.grad h),
    // and the re-emitted Maxwellian as g(u) times a constant polynomial
    R[FR_G] = g.dt;
    R[FR_G + 1] = -0.5 * g.dt * g.dt;
    for (int x = 0; x < 20; ++x) {
      R[FR_PH + x] = x == 0 ? 1.0 : 0.0;
      R[FR_PB + x] = x == 0 ? (g.K + 3.0 - D) / (2.0 * lamw) : 0.0;
    }
    return;
  }
  const bool ghost = kind != UGKS_BC_INTERIOR;
  const int Rc = ghost ? -1 : m.fR[f];
  const double* n = &m.fnorm[f * 3];
  double Wg[5];
  if (ghost) {
    ghost_state<D>(kind, bcs[m.fbcid[f]], n, &W[(int64_t)L * (D + 2)], g.R, g.K, Wg);
    double Pg[NPRIM];
    prim_of<D>(Wg, g, Pg);
    R[FR_GRHO] = Pg[0];
    for (int d = 0; d < 3; ++d) R[FR_GU + d] = Pg[1 + d];
    R[FR_GLAM] = Pg[4];
    R[FR_GC] = Pg[0] * maxw_norm<D>(Pg[4]);
  }
  // 6.1 reconstructed states on both sides
  double Wl[5], Wr[5];
  for (int v = 0; v < D + 2; ++v) {
    double sl = W[(int64_t)L * (D + 2) + v];
    for (int d = 0; d < D; ++d) sl += m.fdxL[f * 3 + d] * gW[((int64_t)L * 3 + d) * 5 + v];
    Wl[v] = sl;
    if (ghost) {
      Wr[v] = Wg[v];
    } else {
      double sr = W[(int64_t)Rc * (D + 2) + v];
      for (int d = 0; d < D; ++d) sr += m.fdxR[f * 3 + d] * gW[((int64_t)Rc * 3 + d) * 5 + v];
      Wr[v] = sr;
    }
  }
  double Pl[NPRIM], Pr[NPRIM];
  if (!prim_of<D>(Wl, g, Pl)) {
    for (int v = 0; v < D + 2; ++v) Wl[v] = W[(int64_t)L * (D + 2) + v];
    prim_of<D>(Wl, g, Pl);
  }
  if (!prim_of<D>(Wr, g, Pr)) {
    for (int v = 0; v < D + 2; ++v) Wr[v] = ghost ? Wg[v] : W[(int64_t)Rc * (D + 2) + v];
    prim_of<D>(Wr, g, Pr);
  }
  // 6.2 interface state from the two half-range Maxwellians
  double W0[5] = {0, 0, 0, 0, 0};
  const double* Ps[2] = {Pl, Pr};
  for (int s = 0; s < 2; ++s) {
    const double* P = Ps[s];
    double rho = P[0], lam = P[4];
    double Un = 0.0;
    for (int d = 0; d < D; ++d) Un += P[1 + d] * n[d];
    double Ut2 = 0.0, Ut[3];
    for (int d = 0; d < D; ++d) {
      Ut[d] = P[1 + d] - Un * n[d];
      Ut2 += Ut[d] * Ut[d];
    }
    double mo[3];
    half_range(Un, lam, s == 0 ? 1.0 : -1.0, mo);
    W0[0] += rho * mo[0];
    for (int d = 0; d < D; ++d) W0[1 + d] += rho * (mo[1] * n[d] + mo[0] * Ut[d]);
    W0[D + 1] += 0.5 * rho * (mo[2] + mo[0] * (Ut2 + (g.K + 2.0) / (2.0 * lam)));
  }
  // 6.3 interface primitives, relaxation time and time coefficients
  double P0[NPRIM];
  if (!prim_of<D>(W0, g, P0)) {
    atomicOr(flag, 2);
    return;
  }
  const double rho0 = P0[0], lam0 = P0[4];
  double U0[3] = {P0[1], P0[2], P0[3]};
  R[FR_C0] = rho0 * maxw_norm<D>(lam0);
  R[FR_LAM] = lam0;
  for (int d = 0; d < 3; ++d) R[FR_U + d] = U0[d];
  R[FR_SH] = 4.0 * (1.0 - g.Pr) * lam0 * lam0 / ((g.K + 5.0) * rho0);
  const double kxi = g.K + 3.0 - D;
  time_coeffs(g.dt, P0[5], &R[FR_G]);
  // 6.4 spatial slopes from the averaged gradient
  double a[3][5];
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 5; ++v) a[d][v] = 0.0;
  for (int d = 0; d < D; ++d) {
    double bvec[5];
    for (int v = 0; v < D + 2; ++v) {
      double gl = gW[((int64_t)L * 3 + d) * 5 + v];
      double gr = ghost ? 0.0 : gW[((int64_t)Rc * 3 + d) * 5 + v];
      bvec[v] = 0.5 * (gl + gr) / rho0;
    }
    slope_solve<D>(bvec, U0, lam0, g.K + 3.0, a[d]);
  }
  // 6.5 time slope from compatibility
  Moments<D> M;
  M.init(U0, lam0, kxi);
  double r[5], At[5];
  time_slope_rhs<D>(M, a, r);
  slope_solve<D>(r, U0, lam0, g.K + 3.0, At);
  for (int d = 0; d < 3; ++d)
    for (int v = 0; v < 5; ++v) R[FR_A + d * 5 + v] = (d < D && v < D + 2) ? a[d][v] : 0.0;
  for (int v = 0; v < 5; ++v) R[FR_AT + v] = v < D + 2 ? At[v] : 0.0;
  // 6.6 interface heat flux
  double q0[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    double ql = q[(int64_t)L * 3 + d];
    double qr = ghost ? 0.0 : q[(int64_t)Rc * 3 + d];
    q0[d] = d < D ? 0.5 * (ql + qr) : 0.0;
    R[FR_Q + d] = q0[d];
  }
  // All equilibrium terms of the time-integrated interface distribution,
  //   Gamma3 (g0 + g0+) + Gamma4 u.grad g0 + Gamma5 d_t g0,
  // equal g0(u) times a cubic polynomial in u: PH for h, PB for b.
  {
    using Cb = Cubic<D>;
    double PH[Cb::N], PB[Cb::N];
    for (int x = 0; x < Cb::N; ++x) PH[x] = PB[x] = 0.0;
    const double kap = kxi / (2.0 * lam0);                             // B0 / H0
    const double xi4 = kxi * (kxi + 2.0) / (4.0 * lam0 * lam0);       // int xi^4 g / H0
    const double G3 = R[FR_G + 2], G4 = R[FR_G + 3], G5 = R[FR_G + 4];
    const double sh = R[FR_SH];
    double a0v[3], a4v[3], Am[9], Atl[3];
    for (int d = 0; d < D; ++d) {
      a0v[d] = a[d][0];
      a4v[d] = a[d][D + 1];
      Atl[d] = At[1 + d];
      for (int e = 0; e < D; ++e) Am[d * 3 + e] = a[d][1 + e];
    }
    // Gamma3 (1 + H0+/H0)
    Cb::add_const(PH, G3);
    Cb::add_shakhov(PH, G3 * sh, U0, q0, lam0, 2.0 + D);
    // Gamma4 sum_d u_d (P_d + a_d4 kap / 2), P_d = a_d0 + a_d.u + a_d4 |u|^2 / 2
    Cb::add_lin(PH, G4, a0v);
    Cb::add_mat(PH, G4, Am, 3);
    Cb::add_lin_u2(PH, 0.5 * G4, a4v);
    Cb::add_lin(PH, 0.5 * G4 * kap, a4v);
    // Gamma5 (P_A + A4 kap / 2)
    Cb::add_const(PH, G5 * (At[0] + 0.5 * At[D + 1] * kap));
    Cb::add_lin(PH, G5, Atl);
    Cb::add_u2(PH, 0.5 * G5 * At[D + 1]);
    if (kxi > 0.0) {
      Cb::add_const(PB, G3 * kap);
      Cb::add_shakhov(PB, G3 * sh * kap, U0, q0, lam0, (double)D);
      Cb::add_lin(PB, G4 * kap, a0v);
      Cb::add_mat(PB, G4 * kap, Am, 3);
      Cb::add_lin_u2(PB, 0.5 * G4 * kap, a4v);
      Cb::add_lin(PB, 0.5 * G4 * xi4, a4v);
      Cb::add_const(PB, G5 * (kap * At[0] + 0.5 * At[D + 1] * xi4));
      Cb::add_lin(PB, G5 * kap, Atl);
      Cb::add_u2(PB, 0.5 * G5 * kap * At[D + 1]);
    }
    for (int x = 0; x < 20; ++x) {
      R[FR_PH + x] = x < Cb::N ? PH[x] : 0.0;
      R[FR_PB + x] = x < Cb::N ? PB[x] : 0.0;
    }
  }
}

template <int D>
__global__ void k_face_eq(DevMesh m, const DevBC* __restrict__ bcs, GasP g,
                          const double* __restrict__ W, const double* __restrict__ gW,
                          const double* __restrict__ q, double* __restrict__ frec, int32_t* flag) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < m.nf) face_eq_at<D>(f, m, bcs, g, W, gW, q, frec, flag);
}

// Microscopic gradients of h (and b) for every (cell, velocity) (step 5).
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_grad_micro(DevMesh m, DevVel v,
                                                    const double* __restrict__ frec,
                                                    const T* __restrict__ h, const T* __restrict__ b,
                                                    double* __restrict__ gh, double* __restrict__ gb,
                                                    const int32_t* flag) {
  const int64_t nch = (v.nvp + TPB - 1) / TPB;
  const int64_t i = blockIdx.x / nch;
  const int64_t k = (blockIdx.x % nch) * TPB + threadIdx.x;
  if (k >= v.nvp || *flag) return;
  const int64_t nvp = v.nvp;
  const double hi = ld(h, i * nvp + k);
  const bool hb = v.has_b;
  const double bi = hb ? ld(b, i * nvp + k) : 0.0;
  double ah[3] = {0, 0, 0}, ab[3] = {0, 0, 0};
  double hmin = hi, hmax = hi, bmin = bi, bmax = bi;
  const int nfc = m.nfc[i];
  for (int p = 0; p < nfc; ++p) {
    const int j = m.cnbr[i * MAXF + p];
    double hn, bn;
    if (j >= 0) {
      hn = ld(h, (int64_t)j * nvp + k);
      bn = hb ? ld(b, (int64_t)j * nvp + k) : 0.0;
    } else {
      const int f = m.cface[i * MAXF + p];
      if (m.fbc[f] == UGKS_BC_WALL) {
        hn = hi;
        bn = bi;
      } else {
        const double* R = &frec[(int64_t)f * FREC];
        double c2 = 0.0;
        for (int d = 0; d < D; ++d) {
          double c = v.u[d * nvp + k] - R[FR_GU + d];
          c2 += c * c;
        }
        hn = R[FR_GC] * exp(-R[FR_GLAM] * c2);
        bn = v.kxi / (2.0 * R[FR_GLAM]) * hn;
      }
    }
    hmin = fmin(hmin, hn);
    hmax = fmax(hmax, hn);
    bmin = fmin(bmin, bn);
    bmax = fmax(bmax, bn);
    for (int d = 0; d < D; ++d) {
      const double G = m.lsG[(i * 3 + d) * MAXF + p];
      ah[d] += G * (hn - hi);
      if (hb) ab[d] += G * (bn - bi);
    }
  }
  if (m.limiter) {
    const double ph = venkat_phi<D>(m, i, nfc, hi, hmin, hmax, ah);
    const double pb = hb ? venkat_phi<D>(m, i, nfc, bi, bmin, bmax, ab) : 1.0;
    for (int d = 0; d < D; ++d) {
      ah[d] *= ph;
      ab[d] *= pb;
    }
  }
  for (int d = 0; d < D; ++d) {
    gh[(i * 3 + d) * nvp + k] = ah[d];
    if (hb) gb[(i * 3 + d) * nvp + k] = ab[d];
  }
}

// Wall density from the zero normal mass flux condition (step 7).
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_wall_rho(DevMesh m, DevVel v, GasP g,
                                                  const T* __restrict__ h,
                                                  const double* __restrict__ gh,
                                                  double* __restrict__ frec, const int32_t* flag) {
  __shared__ double lds[2 * 16];
  if (*flag) return;
  const int f = m.walls[blockIdx.x];
  const int L = m.fL[f];
  const int64_t nvp = v.nvp;
  double* R = &frec[(int64_t)f * FREC];
  const double lamw = R[FR_LAM], Cw = R[FR_C0];
  const double dt = g.dt;
  double acc[2] = {0.0, 0.0};
  for (int64_t k = threadIdx.x; k < nvp; k += TPB) {
    double un = 0.0;
    for (int d = 0; d < D; ++d) un += v.u[d * nvp + k] * m.fnorm[f * 3 + d];
    if (un > 0.0) {
      double hf = ld(h, (int64_t)L * nvp + k), ugh = 0.0;
      for (int d = 0; d < D; ++d) {
        double gd = gh[((int64_t)L * 3 + d) * nvp + k];
        hf += m.fdxL[f * 3 + d] * gd;
        ugh += v.u[d * nvp + k] * gd;
      }
      acc[0] += v.w[k] * un * (dt * hf - 0.5 * dt * dt * ugh);
    } else if (un < 0.0) {
      double c2 = 0.0;
      for (int d = 0; d < D; ++d) {
        double c = v.u[d * nvp + k] - R[FR_U + d];
        c2 += c * c;
      }
      acc[1] += v.w[k] * un * Cw * exp(-lamw * c2);
    }
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) R[FR_RHOW] = -acc[0] / (dt * acc[1]);
}

// Time-integrated microscopic flux of one (face, velocity) (steps 6.7, 7).
template <int D, typename T>
__device__ __forceinline__ void face_flux(const DevMesh& m, const DevVel& v, const GasP& g,
                                          const double* R, int64_t f, int64_t k,
                                          const T* __restrict__ h, const T* __restrict__ b,
                                          const double* __restrict__ gh,
                                          const double* __restrict__ gb, double& FH, double& FB) {
  const int64_t nvp = v.nvp;
  const int kind = m.fbc[f];
  const int L = m.fL[f];
  double uk[3] = {0, 0, 0};
  double un = 0.0;
  for (int d = 0; d < D; ++d) {
    uk[d] = v.u[d * nvp + k];
    un += uk[d] * m.fnorm[f * 3 + d];
  }
  const double dt = g.dt;
  const double KXI = v.kxi;
  const bool hb = v.has_b;
  double ih = 0.0, ib = 0.0;
  if (kind == UGKS_BC_WALL) {
    if (un > 0.0) {
      double hf = ld(h, (int64_t)L * nvp + k), bf = hb ? ld(b, (int64_t)L * nvp + k) : 0.0;
      double ugh = 0.0, ugb = 0.0;
      for (int d = 0; d < D; ++d) {
        double gd = gh[((int64_t)L * 3 + d) * nvp + k];
        hf += m.fdxL[f * 3 + d] * gd;
        ugh += uk[d] * gd;
        if (hb) {
          double gbd = gb[((int64_t)L * 3 + d) * nvp + k];
          bf += m.fdxL[f * 3 + d] * gbd;
          ugb += uk[d] * gbd;
        }
      }
      ih = dt * hf - 0.5 * dt * dt * ugh;
      ib = dt * bf - 0.5 * dt * dt * ugb;
    } else if (un < 0.0) {
      double c2 = 0.0;
      for (int d = 0; d < D; ++d) {
        double c = uk[d] - R[FR_U + d];
        c2 += c * c;
      }
      double Hw = R[FR_C0] * exp(-R[FR_LAM] * c2);
      ih = dt * R[FR_RHOW] * Hw;
      ib = dt * R[FR_RHOW] * KXI / (2.0 * R[FR_LAM]) * Hw;
    }
    FH = un * ih;
    FB = un * ib;
    return;
  }
  const bool ghost = kind != UGKS_BC_INTERIOR;
  double hf, bf = 0.0, ugh = 0.0, ugb = 0.0;
  if (un <= 0.0 && ghost) {
    double c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double c = uk[d] - R[FR_GU + d];
      c2 += c * c;
    }
    hf = R[FR_GC] * exp(-R[FR_GLAM] * c2);
    bf = KXI / (2.0 * R[FR_GLAM]) * hf;
  } else {
    const bool left = un > 0.0;
    const int64_t up = left ? L : m.fR[f];
    const double* dx = left ? &m.fdxL[f * 3] : &m.fdxR[f * 3];
    hf = ld(h, up * nvp + k);
    if (hb) bf = ld(b, up * nvp + k);
    for (int d = 0; d < D; ++d) {
      double gd = gh[(up * 3 + d) * nvp + k];
      hf += dx[d] * gd;
      ugh += uk[d] * gd;
      if (hb) {
        double gbd = gb[(up * 3 + d) * nvp + k];
        bf += dx[d] * gbd;
        ugb += uk[d] * gbd;
      }
    }
  }
  // interface equilibrium, its Shakhov correction and derivative terms
  const double lam0 = R[FR_LAM];
  double c2 = 0.0, cq = 0.0, u2 = v.u2[k];
  for (int d = 0; d < D; ++d) {
    double c = uk[d] - R[FR_U + d];
    c2 += c * c;
    cq += c * R[FR_Q + d];
  }
  const double H0 = R[FR_C0] * exp(-lam0 * c2);
  const double B0 = KXI / (2.0 * lam0) * H0;
  const double sh = R[FR_SH] * cq;
  const double H0p = sh * (2.0 * lam0 * c2 - 2.0 - D) * H0;
  const double B0p = sh * (2.0 * lam0 * c2 - D) * KXI / (2.0 * lam0) * H0;
  const double xi4 = KXI * (KXI + 2.0) / (4.0 * lam0 * lam0);
  double uH = 0.0, uB = 0.0;
  for (int d = 0; d < D; ++d) {
    const double* ad = &R[FR_A + d * 5];
    double Pd = ad[0] + 0.5 * ad[D + 1] * u2;
    for (int c = 0; c < D; ++c) Pd += ad[1 + c] * uk[c];
    uH += uk[d] * (Pd * H0 + 0.5 * ad[D + 1] * B0);
    uB += uk[d] * (Pd * B0 + 0.5 * ad[D + 1] * xi4 * H0);
  }
  const double* At = &R[FR_AT];
  double PA = At[0] + 0.5 * At[D + 1] * u2;
  for (int c = 0; c < D; ++c) PA += At[1 + c] * uk[c];
  const double tH = PA * H0 + 0.5 * At[D + 1] * B0;
  const double tB = PA * B0 + 0.5 * At[D + 1] * xi4 * H0;
  const double* G = &R[FR_G];
  ih = G[0] * hf + G[1] * ugh + G[2] * (H0 + H0p) + G[3] * uH + G[4] * tH;
  ib = G[0] * bf + G[1] * ugb + G[2] * (B0 + B0p) + G[3] * uB + G[4] * tB;
  FH = un * ih;
  FB = un * ib;
}

// Microscopic fluxes of one face for every velocity, and the face's
// macroscopic flux F = sum_k w_k (H, u H, (|u|^2 H + B)/2) (Eq. macro_flux).
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_flux(DevMesh m, DevVel v, GasP g,
                                              const double* __restrict__ frec,
                                              const T* __restrict__ h, const T* __restrict__ b,
                                              const double* __restrict__ gh,
                                              const double* __restrict__ gb,
                                              double* __restrict__ fh, double* __restrict__ fb,
                                              double* __restrict__ F, const int32_t* flag) {
  __shared__ double lds[5 * 16];
  if (*flag) return;
  const int64_t f = blockIdx.x;
  const double* R = &frec[f * FREC];
  const int64_t nvp = v.nvp;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = threadIdx.x; k < nvp; k += TPB) {
    double FH, FB;
    face_flux<D, T>(m, v, g, R, f, k, h, b, gh, gb, FH, FB);
    fh[f * nvp + k] = FH;
    if (v.has_b) fb[f * nvp + k] = FB;
    const double wk = v.w[k];
    acc[0] += wk * FH;
    for (int d = 0; d < D; ++d) acc[1 + d] += wk * v.u[d * nvp + k] * FH;
    acc[D + 1] += wk * 0.5 * (v.u2[k] * FH + FB);
  }
  block_sum<5>(acc, lds);
  if (threadIdx.x == 0)
    for (int x = 0; x < 5; ++x) F[f * 5 + x] = x < D + 2 ? acc[x] : 0.0;
}

// Reduced Maxwellian and Shakhov correction of a cell at one velocity.
template <int D>
__device__ __forceinline__ void cell_equilibrium(const double* P, const double* qv, const GasP& g,
                                                 const double* uk, double& Hs, double& Bs) {
  const double KXI = g.K + 3.0 - D, Pr = g.Pr;
  const double rho = P[0], lam = P[4];
  double c2 = 0.0, cq = 0.0;
  for (int d = 0; d < D; ++d) {
    double c = uk[d] - P[1 + d];
    c2 += c * c;
    cq += c * qv[d];
  }
  const double H = rho * maxw_norm<D>(lam) * exp(-lam * c2);
  const double pre = 4.0 * (1.0 - Pr) * lam * lam / ((g.K + 5.0) * rho) * cq;
  const double Hp = pre * (2.0 * lam * c2 - 2.0 - D) * H;
  const double Bp = pre * (2.0 * lam * c2 - D) * KXI / (2.0 * lam) * H;
  Hs = H + Hp;
  Bs = KXI / (2.0 * lam) * H + Bp;
}

// First stage (Eq. f_tilde).
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_stage1(DevMesh m, DevVel v, GasP g,
                                                const double* __restrict__ prim,
                                                const double* __restrict__ q,
                                                const T* __restrict__ h, const T* __restrict__ b,
                                                const double* __restrict__ fh,
                                                const double* __restrict__ fb, T* __restrict__ ht,
                                                T* __restrict__ bt, const int32_t* flag) {
  const int64_t nch = (v.nvp + TPB - 1) / TPB;
  const int64_t i = blockIdx.x / nch;
  const int64_t k = (blockIdx.x % nch) * TPB + threadIdx.x;
  if (k >= v.nvp || *flag) return;
  const int64_t nvp = v.nvp;
  double sh = 0.0, sb = 0.0;
  const int nfc = m.nfc[i];
  for (int p = 0; p < nfc; ++p) {
    const int64_t f = m.cface[i * MAXF + p];
    const double s = m.csign[i * MAXF + p] * area_for(g, i, m.farea[f]);
    sh += s * fh[f * nvp + k];
    if (v.has_b) sb += s * fb[f * nvp + k];
  }
  const double* P = &prim[i * NPRIM];
  double uk[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) uk[d] = v.u[d * nvp + k];
  double Hs, Bs;
  cell_equilibrium<D>(P, &q[i * 3], g, uk, Hs, Bs);
  const double c = dt_cell(g, i) / (2.0 * P[5]);
  const double iv = 1.0 / m.vol[i];
  const double hv = ld(h, i * nvp + k);
  st(ht, i * nvp + k, hv - sh * iv + c * (Hs - hv));
  if (v.has_b) {
    const double bv = ld(b, i * nvp + k);
    st(bt, i * nvp + k, bv - sb * iv + c * (Bs - bv));
  }
}

// Conservative update (Eq. macro_update) and per-cell residual parts.
template <int D>
__global__ void k_macro_update(DevMesh m, GasP g, const double* __restrict__ W, const double* __restrict__ F,
                               double* __restrict__ Wn, double* __restrict__ cellred,
                               const int32_t* flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m.nc || *flag) return;
  double acc[5] = {0, 0, 0, 0, 0};
  const int nfc = m.nfc[i];
  for (int p = 0; p < nfc; ++p) {
    const int64_t f = m.cface[i * MAXF + p];
    const double s = m.csign[i * MAXF + p] * area_for(g, i, m.farea[f]);
    for (int x = 0; x < D + 2; ++x) acc[x] += s * F[f * 5 + x];
  }
  const double V = m.vol[i];
  for (int x = 0; x < D + 2; ++x) Wn[i * (D + 2) + x] = W[i * (D + 2) + x] - acc[x] / V;
  const double dr = Wn[i * (D + 2)] - W[i * (D + 2)];
  cellred[i * 3 + 0] = V * dr * dr;
  cellred[i * 3 + 1] = V;
  cellred[i * 3 + 2] = V * W[i * (D + 2)] * W[i * (D + 2)];
}

// Second stage (Eq. f_final) with the equilibrium of W^{n+1} and q^n.
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_stage2(DevVel v, GasP g, const double* __restrict__ primn,
                                                const double* __restrict__ q,
                                                const T* __restrict__ ht, const T* __restrict__ bt,
                                                T* __restrict__ h, T* __restrict__ b,
                                                const int32_t* flag) {
  const int64_t nch = (v.nvp + TPB - 1) / TPB;
  const int64_t i = blockIdx.x / nch;
  const int64_t k = (blockIdx.x % nch) * TPB + threadIdx.x;
  if (k >= v.nvp || *flag) return;
  const int64_t nvp = v.nvp;
  const double* P = &primn[i * NPRIM];
  double uk[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) uk[d] = v.u[d * nvp + k];
  double Hs, Bs;
  cell_equilibrium<D>(P, &q[i * 3], g, uk, Hs, Bs);
  const double a = dt_cell(g, i) / (2.0 * P[5]);
  const double inv = 1.0 / (1.0 + a);
  st(h, i * nvp + k, (ld(ht, i * nvp + k) + a * Hs) * inv);
  if (v.has_b) st(b, i * nvp + k, (ld(bt, i * nvp + k) + a * Bs) * inv);
}

// Residual of the density: one block, fixed summation order.
__device__ __forceinline__ void residual_of(int64_t nc, const double* __restrict__ cellred,
                                            double* __restrict__ resid, const int32_t* flag,
                                            double* lds) {
  if (*flag) return;
  double acc[3] = {0, 0, 0};
  for (int64_t i = threadIdx.x; i < nc; i += blockDim.x)
    for (int x = 0; x < 3; ++x) acc[x] += cellred[i * 3 + x];
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    double nrm = sqrt(acc[0] / acc[1]);
    if (resid[3] == 0.0) resid[3] = nrm;
    resid[0] = resid[3] > 0.0 ? nrm / resid[3] : 0.0;
    resid[1] = nrm / sqrt(acc[2] / acc[1]);
  }
}

__global__ __launch_bounds__(1024) void k_residual(int64_t nc, const double* __restrict__ cellred,
                                                   double* __restrict__ resid, const int32_t* flag) {
  __shared__ double lds[3 * 16];
  residual_of(nc, cellred, resid, flag, lds);
}

template <int D>
__global__ void k_commit_W(int64_t nc, const double* __restrict__ Wn, double* __restrict__ W,
                           const int32_t* flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nc * (D + 2) || *flag) return;
  W[i] = Wn[i];
}

template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_init_maxwellian(DevVel v, const double* __restrict__ prim,
                                                         T* __restrict__ h, T* __restrict__ b) {
  const int64_t nch = (v.nvp + TPB - 1) / TPB;
  const int64_t i = blockIdx.x / nch;
  const int64_t k = (blockIdx.x % nch) * TPB + threadIdx.x;
  if (k >= v.nvp) return;
  const double* P = &prim[i * NPRIM];
  double c2 = 0.0;
  for (int d = 0; d < D; ++d) {
    double c = v.u[d * v.nvp + k] - P[1 + d];
    c2 += c * c;
  }
  const double H = P[0] * maxw_norm<D>(P[4]) * exp(-P[4] * c2);
  st(h, i * v.nvp + k, H);
  if (v.has_b) st(b, i * v.nvp + k, v.kxi / (2.0 * P[4]) * H);
}

// Discrete moments sum_k w_k psi_k (h, b) per cell.
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_moments(DevVel v, const T* __restrict__ h,
                                                 const T* __restrict__ b, double* __restrict__ out) {
  __shared__ double lds[5 * 16];
  const int64_t i = blockIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t k = threadIdx.x; k < v.nvp; k += TPB) {
    double wh = v.w[k] * ld(h, i * v.nvp + k);
    double wb = v.has_b ? v.w[k] * ld(b, i * v.nvp + k) : 0.0;
    acc[0] += wh;
    for (int d = 0; d < D; ++d) acc[1 + d] += wh * v.u[d * v.nvp + k];
    acc[D + 1] += 0.5 * (wh * v.u2[k] + wb);
  }
  block_sum<5>(acc, lds);
  if (threadIdx.x == 0)
    for (int x = 0; x < D + 2; ++x) out[i * (D + 2) + x] = acc[x];
}

// Per-cell CFL bound 2 V_i / max_k sum_j S_j |u_k . n_j|.
template <int D>
__global__ __launch_bounds__(TPB) void k_dt_cells(DevMesh m, DevVel v, double* __restrict__ out) {
  __shared__ double lds[16];
  const int64_t i = blockIdx.x;
  const int nfc = m.nfc[i];
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < v.nvp; k += TPB) {
    if (k >= v.nv) break;
    double s = 0.0;
    for (int p = 0; p < nfc; ++p) {
      const int64_t f = m.cface[i * MAXF + p];
      double un = 0.0;
      for (int d = 0; d < D; ++d) un += v.u[d * v.nvp + k] * m.fnorm[f * 3 + d];
      s += m.farea[f] * fabs(un);
    }
    mx = fmax(mx, s);
  }
  mx = block_max(mx, lds);
  if (threadIdx.x == 0) out[i] = 2.0 * m.vol[i] / mx;
}

inline unsigned blocks_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

// ---- batched forms: one launch covers every case of a batch ---------------
__device__ __forceinline__ int case_of(const int64_t* __restrict__ off, int n, int64_t t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int D>
__global__ void k_gradW_b(BatchDev bd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= bd.cell_off[bd.n]) return;
  const int c = case_of(bd.cell_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  gradW_at<D>(t - bd.cell_off[c], C.m, C.bcs, C.g, C.B.W, C.B.gW, C.B.flag);
}

template <int D>
__global__ void k_face_eq_b(BatchDev bd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= bd.face_off[bd.n]) return;
  const int c = case_of(bd.face_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  face_eq_at<D>(t - bd.face_off[c], C.m, C.bcs, C.g, C.B.W, C.B.gW, C.B.q, C.B.frec, C.B.flag);
}

// one block per case
__global__ __launch_bounds__(1024) void k_residual_b(BatchDev bd) {
  __shared__ double lds[3 * 16];
  const CaseDev& C = bd.cases[blockIdx.x];
  residual_of(C.m.nc, C.B.cellred, C.B.resid, C.B.flag, lds);
}

template <int D>
__global__ void k_commit_W_b(BatchDev bd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= bd.cell_off[bd.n]) return;
  const int c = case_of(bd.cell_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  if (*C.B.flag) return;
  const int64_t i = t - bd.cell_off[c];
  for (int x = 0; x < D + 2; ++x) C.B.W[i * (D + 2) + x] = C.B.Wn[i * (D + 2) + x];
}

}  // namespace

#define UGKS_DISPATCH_D(D_, ...)          \
  do {                                    \
    if ((D_) == 2) {                      \
      constexpr int DD = 2;               \
      __VA_ARGS__;                        \
    } else {                              \
      constexpr int DD = 3;               \
      __VA_ARGS__;                        \
    }                                     \
  } while (0)

#define UGKS_DISPATCH_DT(D_, P_, ...)                  \
  do {                                                 \
    if ((P_) == UGKS_FP32) {                           \
      using TT = float;                                \
      UGKS_DISPATCH_D(D_, __VA_ARGS__);                \
    } else {                                           \
      using TT = double;                               \
      UGKS_DISPATCH_D(D_, __VA_ARGS__);                \
    }                                                  \
  } while (0)

hipError_t launch_prims(int D, const DevMesh& m, const GasP& g, const double* W, double* prim,
                        int32_t* flag, int checkflag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_prims<DD><<<blocks_for(m.nc, 256), 256, 0, s>>>(m.nc, g, W, prim, flag, checkflag));
  return hipGetLastError();
}

hipError_t launch_heatflux(int D, int prec, const DevMesh& m, const DevVel& v, const void* h,
                           const void* b, const double* prim, double* q, const int32_t* flag,
                           hipStream_t s) {
  UGKS_DISPATCH_DT(D, prec, k_heatflux<DD, TT><<<(unsigned)m.nc, TPB, 0, s>>>(
      v, (const TT*)h, (const TT*)b, prim, q, flag));
  return hipGetLastError();
}

hipError_t launch_gradW(int D, const DevMesh& m, const DevBC* bcs, const GasP& g, const double* W,
                        double* gW, const int32_t* flag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_gradW<DD><<<blocks_for(m.nc, 128), 128, 0, s>>>(m, bcs, g, W, gW, flag));
  return hipGetLastError();
}

hipError_t launch_face_eq(int D, const DevMesh& m, const DevBC* bcs, const GasP& g,
                          const double* W, const double* gW, const double* q, double* frec,
                          int32_t* flag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_face_eq<DD><<<blocks_for(m.nf, 64), 64, 0, s>>>(m, bcs, g, W, gW, q, frec, flag));
  return hipGetLastError();
}

hipError_t launch_grad_micro(int D, int prec, const DevMesh& m, const DevVel& v,
                             const double* frec, const void* h, const void* b, double* gh,
                             double* gb, const int32_t* flag, hipStream_t s) {
  const unsigned grid = blocks_for(v.nvp, TPB) * (unsigned)m.nc;
  UGKS_DISPATCH_DT(D, prec, k_grad_micro<DD, TT><<<grid, TPB, 0, s>>>(
      m, v, frec, (const TT*)h, (const TT*)b, gh, gb, flag));
  return hipGetLastError();
}

hipError_t launch_flux(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                       const double* frec, const void* h, const void* b, const double* gh,
                       const double* gb, double* fh, double* fb, double* F, const int32_t* flag,
                       hipStream_t s) {
  UGKS_DISPATCH_DT(D, prec, k_flux<DD, TT><<<(unsigned)m.nf, TPB, 0, s>>>(
      m, v, g, frec, (const TT*)h, (const TT*)b, gh, gb, fh, fb, F, flag));
  return hipGetLastError();
}

hipError_t launch_stage1(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                         const double* prim, const double* q, const void* h, const void* b,
                         const double* fh, const double* fb, void* ht, void* bt,
                         const int32_t* flag, hipStream_t s) {
  const unsigned grid = blocks_for(v.nvp, TPB) * (unsigned)m.nc;
  UGKS_DISPATCH_DT(D, prec, k_stage1<DD, TT><<<grid, TPB, 0, s>>>(
      m, v, g, prim, q, (const TT*)h, (const TT*)b, fh, fb, (TT*)ht, (TT*)bt, flag));
  return hipGetLastError();
}

hipError_t launch_macro_update(int D, const DevMesh& m, const GasP& g, const double* W, const double* F,
                               double* Wn, double* cellred, const int32_t* flag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_macro_update<DD><<<blocks_for(m.nc, 256), 256, 0, s>>>(m, g, W, F, Wn, cellred, flag));
  return hipGetLastError();
}

hipError_t launch_stage2(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                         const double* primn, const double* q, const void* ht, const void* bt,
                         void* h, void* b, const int32_t* flag, hipStream_t s) {
  const unsigned grid = blocks_for(v.nvp, TPB) * (unsigned)m.nc;
  UGKS_DISPATCH_DT(D, prec, k_stage2<DD, TT><<<grid, TPB, 0, s>>>(
      v, g, primn, q, (const TT*)ht, (const TT*)bt, (TT*)h, (TT*)b, flag));
  return hipGetLastError();
}

hipError_t launch_residual(const DevMesh& m, const double* cellred, double* resid,
                           const int32_t* flag, hipStream_t s) {
  k_residual<<<1, 1024, 0, s>>>(m.nc, cellred, resid, flag);
  return hipGetLastError();
}

hipError_t launch_commit_W(int D, const DevMesh& m, const double* Wn, double* W,
                           const int32_t* flag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_commit_W<DD><<<blocks_for(m.nc * (DD + 2), 256), 256, 0, s>>>(m.nc, Wn, W, flag));
  return hipGetLastError();
}

hipError_t launch_init_maxwellian(int D, int prec, const DevMesh& m, const DevVel& v,
                                  const double* prim, void* h, void* b, hipStream_t s) {
  const unsigned grid = blocks_for(v.nvp, TPB) * (unsigned)m.nc;
  UGKS_DISPATCH_DT(D, prec, k_init_maxwellian<DD, TT><<<grid, TPB, 0, s>>>(v, prim, (TT*)h, (TT*)b));
  return hipGetLastError();
}

hipError_t launch_moments(int D, int prec, const DevMesh& m, const DevVel& v, const void* h,
                          const void* b, double* out, hipStream_t s) {
  UGKS_DISPATCH_DT(D, prec, k_moments<DD, TT><<<(unsigned)m.nc, TPB, 0, s>>>(v, (const TT*)h, (const TT*)b, out));
  return hipGetLastError();
}

hipError_t launch_dt_cells(int D, const DevMesh& m, const DevVel& v, double* cellval,
                           hipStream_t s) {
  UGKS_DISPATCH_D(D, k_dt_cells<DD><<<(unsigned)m.nc, TPB, 0, s>>>(m, v, cellval));
  return hipGetLastError();
}

hipError_t launch_wall_rho(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                           const void* h, const double* gh, double* frec, const int32_t* flag,
                           hipStream_t s) {
  if (m.nwall == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_wall_rho<DD, TT><<<(unsigned)m.nwall, TPB, 0, s>>>(
      m, v, g, (const TT*)h, gh, frec, flag));
  return hipGetLastError();
}

hipError_t launch_gradW_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  const unsigned grid = (unsigned)((ncell + 127) / 128);
  if (D == 2) k_gradW_b<2><<<grid, 128, 0, s>>>(bd);
  else k_gradW_b<3><<<grid, 128, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_face_eq_b(int D, const BatchDev& bd, int64_t nface, hipStream_t s) {
  if (nface == 0) return hipSuccess;
  const unsigned grid = (unsigned)((nface + 63) / 64);
  if (D == 2) k_face_eq_b<2><<<grid, 64, 0, s>>>(bd);
  else k_face_eq_b<3><<<grid, 64, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_residual_b(const BatchDev& bd, hipStream_t s) {
  if (bd.n == 0) return hipSuccess;
  k_residual_b<<<(unsigned)bd.n, 1024, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_commit_W_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  const unsigned grid = (unsigned)((ncell + 255) / 256);
  if (D == 2) k_commit_W_b<2><<<grid, 256, 0, s>>>(bd);
  else k_commit_W_b<3><<<grid, 256, 0, s>>>(bd);
  return hipGetLastError();
}

}  // namespace ugks
