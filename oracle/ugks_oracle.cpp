// Plain FP64 CPU oracle of one UGKS phase-space time step.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the HIP library is checked against.  Only tests, the smoke
// check and the benchmark's CPU-baseline leg may load it; the product path
// never does.  It shares no code, header or table with the HIP library.
//
// What it computes (paper Sec. 2.1 and the one-step algorithm of Sec. 2.2):
//   * BGK-Shakhov model with reduced distributions h = int f dxi and
//     b = int xi^2 f dxi (Eqs. reduced_hb, reduced_bgk), K >= 0 internal
//     degrees of freedom, K_xi = K + 3 - D (Eq. Kxi_def).  For a monatomic
//     gas in 3-D K_xi = 0, so b = B = B+ = 0 and b is not stored.
//   * Reduced Maxwellian H, B (Eqs. H_def, B_def) and Shakhov corrections
//     H+, B+ (Eqs. H_plus, B_plus).
//   * Finite-volume update with time-integrated interface fluxes
//     (Eqs. fv_micro_update, micro_flux, HB_flux, macro_update, macro_flux).
//   * Interface distribution from the characteristic integral solution with
//     upwind second-order reconstruction and a first-order equilibrium
//     expansion (Eqs. integral_solution, initial_reconstruction,
//     equilibrium_expansion, interface_distribution, c123, c45), integrated
//     over [0, dt].
//   * Diffuse Maxwell walls with the wall density from the zero normal mass
//     flux condition (Eqs. wall_bc, wall_maxwellian, wall_density_condition).
//   * Two-stage trapezoidal collision update (Eqs. f_tilde, f_final).
//
// Readings of points the paper leaves open (the same ones the library uses):
//   R1 K > 0: the Shakhov correction g A c.q (2 lambda (c^2 + xi^2) - alpha)
//      of Eq. shakhov_fp takes alpha = K + 5 (zero momentum) and
//      A = 4 (1 - Pr) lambda^2 / ((K + 5) rho) (heat flux (1 - Pr) q), so
//      H+ = A c.q (2 lambda c^2 - D - 2) H and
//      B+ = A c.q (K_xi / 2 lambda)(2 lambda c^2 - D) H; for K = 0 these are
//      Eqs. H_plus, B_plus.  lambda = (K + 3) rho / (4 (rho E - rho U^2 / 2)).
//   R2 units rho0 = T0 = 1, speed unit sqrt(2RT0), R = 1/2.
//   R3 hard-sphere viscosity mu = mu_ref (T/T_ref)^omega, tau = mu / p.
//   R5 dt = CFL * min_i 2 V_i / max_k sum_{j in faces(i)} S_j |u_k . n_j|.
//   R6 unweighted least squares over face neighbours; one mirror ghost per
//      boundary face at offset 2((x_f - x_i).n)n; wall ghost value = the
//      cell's own value; far-field / outflow ghost = Maxwellian of W_g.
//   R8 the macroscopic reconstruction uses the conservative variables.
//   R9 interface state W0 from the analytic half-range moments of the left
//      and right reconstructed Maxwellians.
//   R10 grad W0 = (grad W_L + grad W_R)/2, ghost gradients 0.
//   R11 spatial slopes a_d and time slope A from Gaussian moments of g0.
//   R12 q0 = (q_L + q_R)/2, ghost q = 0.
//   R14 wall incident part h_f - t u.grad h over the step.
//   R16 far-field ghost = W_inf if U_inf.n < 0 else W_L; outflow ghost = W_L.
//   R17 the Shakhov term of the stage-2 equilibrium uses q^n.
//   R18 time coefficients by closed form for dt/tau >= 1/2, series below.
//   R7 optional slope limiter: Venkatakrishnan's (1995) smooth limiter on the
//      least-squares gradient of every cell field it is applied to, each
//      conservative component of W and each (cell, velocity) of h and b:
//      with v_max, v_min over the cell and its stencil values, at each face
//      d- = g.(x_f - x_i), d+ = v_max - v_i (d- > 0) or v_min - v_i (d- < 0),
//      psi = (d+^2 + eps^2 + 2 d- d+) / (d+^2 + 2 d-^2 + d- d+ + eps^2)
//      (psi = 1 where d- = 0), phi = min(1, min_faces psi), g -> phi g,
//      eps^2 = (K V_i^(1/D))^3.  Off by default.
//   R26 optional local time steps for steady problems (the paper has none;
//      its conclusion names steady-state acceleration as future work): cell
//      i advances by dt_i = dt b_i / min_j b_j, b_i the cell's R5 bound;
//      every face still integrates over the global dt, and cell i applies
//      the face integrals scaled by dt_i / dt and relaxes over dt_i.  A fixed
//      point of the global step is a fixed point of this one.  Off by default.
//
// Layout (oracle's own choice): distributions are velocity-major,
// h[k * n_cells + i], so one velocity is swept over all cells at a time, which
// is the sequential-in-velocity reading of the two-stage update.
// Every velocity sum runs over k ascending; OpenMP parallelises over cells or
// faces only, so results do not depend on the thread count.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <array>
#include <map>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum { BC_INTERIOR = 0, BC_WALL = 1, BC_FARFIELD = 2, BC_OUTFLOW = 3 };

// ---------------------------------------------------------------------------
// Gaussian moments and the Gram systems for the slopes (step 6.4-6.5).
// A monomial is u_1^e1 u_2^e2 u_3^e3 (xi^2)^m; a polynomial is a map from
// exponents to coefficients.
using Mono = std::array<int, 4>;
using Poly = std::map<Mono, double>;

Poly poly_mul(const Poly& a, const Poly& b) {
  Poly r;
  for (auto& x : a)
    for (auto& y : b) {
      Mono m;
      for (int i = 0; i < 4; ++i) m[i] = x.first[i] + y.first[i];
      r[m] += x.second * y.second;
    }
  return r;
}

// E[X^n] for X ~ N(mean, var): E[X^{n+1}] = mean E[X^n] + n var E[X^{n-1}].
double normal_raw_moment(int n, double mean, double var) {
  double m0 = 1.0, m1 = mean;
  if (n == 0) return m0;
  for (int k = 1; k < n; ++k) {
    double m2 = mean * m1 + k * var * m0;
    m0 = m1;
    m1 = m2;
  }
  return m1;
}

// E[(xi^2)^m] for K_xi independent N(0, var) components.
double xi2_moment(int m, int kxi, double var) {
  double r = 1.0;
  for (int j = 0; j < m; ++j) r *= (kxi + 2.0 * j) * var;
  return r;
}

struct Gauss {
  int D, kxi;
  double U[3];
  double var;  // 1/(2 lambda)
  double expect(const Poly& p) const {
    double s = 0.0;
    for (auto& t : p) {
      double v = t.second;
      for (int d = 0; d < 3; ++d) {
        if (t.first[d] == 0) continue;
        v *= normal_raw_moment(t.first[d], d < D ? U[d] : 0.0, var);
      }
      v *= xi2_moment(t.first[3], kxi, var);
      s += v;
    }
    return s;
  }
};

// Collision invariants psi = (1, u_1..u_D, (|u|^2 + xi^2)/2) (Eq. collision_invariant).
std::vector<Poly> invariants(int D) {
  std::vector<Poly> psi(D + 2);
  psi[0][Mono{0, 0, 0, 0}] = 1.0;
  for (int d = 0; d < D; ++d) {
    Mono m{0, 0, 0, 0};
    m[d] = 1;
    psi[1 + d][m] = 1.0;
  }
  for (int d = 0; d < D; ++d) {
    Mono m{0, 0, 0, 0};
    m[d] = 2;
    psi[D + 1][m] = 0.5;
  }
  psi[D + 1][Mono{0, 0, 0, 1}] = 0.5;
  return psi;
}

// Dense Cholesky solve of the SPD system M x = r (n <= 5).
bool cholesky_solve(int n, std::vector<double> M, std::vector<double>& x, const std::vector<double>& r) {
  for (int j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
    if (!(s > 0.0)) return false;
    M[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
      M[i * n + j] = t / M[j * n + j];
    }
  }
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double t = r[i];
    for (int k = 0; k < i; ++k) t -= M[i * n + k] * y[k];
    y[i] = t / M[i * n + i];
  }
  x.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < n; ++k) t -= M[k * n + i] * x[k];
    x[i] = t / M[i * n + i];
  }
  return true;
}

// Gram matrix M_ab = E[psi_a psi_b] under the normalised Maxwellian.
std::vector<double> gram(const Gauss& g, const std::vector<Poly>& psi) {
  int n = (int)psi.size();
  std::vector<double> M(n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) M[a * n + b] = g.expect(poly_mul(psi[a], psi[b]));
  return M;
}

// ---------------------------------------------------------------------------
// Time-integrated coefficients Gamma_1..5 = int_0^dt c_1..c_5 dt (Eqs. c123, c45).
void gamma_coeffs(double dt, double tau, double G[5]) {
  double x = dt / tau;
  if (x >= 0.5) {
    double E = -std::expm1(-x);  // 1 - exp(-x)
    G[0] = tau * E;
    G[1] = tau * tau * (x * (1.0 - E) - E);
    G[2] = tau * (x - E);
    G[3] = tau * tau * (2.0 * E - x * (2.0 - E));
    G[4] = tau * tau * (0.5 * x * x - x + E);
    return;
  }
  // Power series of the same expressions (exact rearrangements of exp(-x)).
  double s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
  double xn = 1.0;  // x^n / n!
  for (int n = 1; n <= 60; ++n) {
    xn *= x / n;
    double sg = (n % 2 == 1) ? 1.0 : -1.0;  // (-1)^(n+1)
    s1 += sg * xn;
    if (n >= 2) {
      s2 += sg * (n - 1) * xn;   // (-1)^(n-1) (n-1) x^n/n!
      s3 += -sg * xn;            // (-1)^n x^n / n!
    }
    if (n >= 3) {
      s4 += sg * (2 - n) * xn;
      s5 += sg * xn;
    }
    if (xn < 1e-40) break;
  }
  G[0] = tau * s1;
  G[1] = tau * tau * s2;
  G[2] = tau * s3;
  G[3] = tau * tau * s4;
  G[4] = tau * tau * s5;
}

struct Prim {
  double rho, U[3], lam, tau;
  bool ok;
};

}  // namespace

// ---------------------------------------------------------------------------
struct oracle_ctx {
  int D, K, kxi, nr, nbc, limiter;
  int64_t nc, nf, nv;
  double Pr, Rg, Tref, muref, omega, dt;
  std::vector<double> vol, cen, farea, fnorm, fcen, fshift;
  std::vector<int64_t> fL, fR;
  std::vector<int> fbc, fbcid;
  std::vector<double> u, w;
  std::vector<int> bckind;
  std::vector<double> bcrho, bcU, bcT;
  // cell -> faces
  std::vector<std::vector<int64_t>> cfaces;
  // least-squares coefficient matrix per cell: G_i is D x m_i, stored row-major
  std::vector<std::vector<double>> lsG;
  // state
  std::vector<double> W, h, b, q;
  std::vector<double> rho_hist0, rho_prev;
  double res_norm0 = 0.0, last_res = -1.0, last_change = 0.0;
  int64_t steps_done = 0;
  // diagnostics of the last step
  std::vector<double> F;       // nf x (D+2)
  std::vector<double> rhow;    // nf (wall faces only)
  std::vector<double> fW0;     // nf x (D+2)
  std::vector<double> ftau0;   // nf
  std::string err;

  int NW() const { return D + 2; }

  double mu_of_T(double T) const { return muref * std::pow(T / Tref, omega); }

  // Primitive variables of W (step 1).
  Prim prim(const double* Wc) const {
    Prim p;
    p.rho = Wc[0];
    double u2 = 0.0;
    for (int d = 0; d < 3; ++d) p.U[d] = 0.0;
    for (int d = 0; d < D; ++d) {
      p.U[d] = Wc[1 + d] / p.rho;
      u2 += p.U[d] * p.U[d];
    }
    double eint = Wc[D + 1] - 0.5 * p.rho * u2;  // = 3 rho / (4 lambda)
    p.lam = (K + 3.0) * p.rho / (4.0 * eint);
    p.ok = (p.rho > 0.0) && (eint > 0.0) && std::isfinite(p.lam);
    double pres = p.rho / (2.0 * p.lam);
    double T = 1.0 / (2.0 * Rg * p.lam);
    p.tau = mu_of_T(T) / pres;
    return p;
  }

  // Reduced Maxwellian H (Eq. H_def) at velocity k.
  double H_at(double rho, const double* U, double lam, int64_t k) const {
    double c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double c = u[k * D + d] - U[d];
      c2 += c * c;
    }
    return rho * std::pow(lam / M_PI, 0.5 * D) * std::exp(-lam * c2);
  }

  // Shakhov corrections H+, B+ (Eqs. H_plus, B_plus with K = 0).
  void shakhov(double rho, const double* U, double lam, const double* qv, int64_t k, double H,
               double& Hp, double& Bp) const {
    double cq = 0.0, c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double c = u[k * D + d] - U[d];
      cq += c * qv[d];
      c2 += c * c;
    }
    double pre = 4.0 * (1.0 - Pr) * lam * lam / ((K + 5.0) * rho) * cq;
    Hp = pre * (2.0 * lam * c2 - 2.0 - D) * H;
    Bp = pre * (2.0 * lam * c2 - D) * kxi / (2.0 * lam) * H;
  }

  // Ghost state of a far-field / outflow boundary face (R16).
  void ghost_W(int64_t f, const double* WL, double* Wg) const {
    int id = fbcid[f];
    bool use_inf = false;
    if (fbc[f] == BC_FARFIELD) {
      double un = 0.0;
      for (int d = 0; d < D; ++d) un += bcU[id * 3 + d] * fnorm[f * D + d];
      use_inf = un < 0.0;
    }
    if (use_inf) {
      double rho = bcrho[id], T = bcT[id];
      double U2 = 0.0;
      Wg[0] = rho;
      for (int d = 0; d < D; ++d) {
        Wg[1 + d] = rho * bcU[id * 3 + d];
        U2 += bcU[id * 3 + d] * bcU[id * 3 + d];
      }
      Wg[D + 1] = 0.5 * rho * U2 + 0.5 * (K + 3.0) * rho * Rg * T;  // K internal degrees (R1)
    } else {
      for (int v = 0; v < NW(); ++v) Wg[v] = WL[v];
    }
  }

  // Least-squares stencil of cell i (O0): offsets of the face neighbours or
  // mirror ghosts.
  void stencil_offsets(int64_t i, std::vector<double>& A) const {
    A.clear();
    for (int64_t f : cfaces[i]) {
      double off[3] = {0, 0, 0};
      if (fbc[f] == BC_INTERIOR) {
        bool isL = fL[f] == i;
        int64_t j = isL ? fR[f] : fL[f];
        double sg = isL ? 1.0 : -1.0;
        for (int d = 0; d < D; ++d) off[d] = cen[j * D + d] + sg * fshift[f * D + d] - cen[i * D + d];
      } else {
        double dn = 0.0;
        for (int d = 0; d < D; ++d) dn += (fcen[f * D + d] - cen[i * D + d]) * fnorm[f * D + d];
        for (int d = 0; d < D; ++d) off[d] = 2.0 * dn * fnorm[f * D + d];
      }
      for (int d = 0; d < D; ++d) A.push_back(off[d]);
    }
  }

  void build_ls() {
    lsG.assign(nc, {});
    std::vector<double> A;
    for (int64_t i = 0; i < nc; ++i) {
      stencil_offsets(i, A);
      int m = (int)cfaces[i].size();
      // normal matrix N = A^T A, invert by cofactors (D <= 3)
      double N[9] = {0};
      for (int p = 0; p < m; ++p)
        for (int r = 0; r < D; ++r)
          for (int c = 0; c < D; ++c) N[r * 3 + c] += A[p * D + r] * A[p * D + c];
      double Ni[9] = {0};
      if (D == 2) {
        double det = N[0] * N[4] - N[1] * N[3];
        Ni[0] = N[4] / det; Ni[1] = -N[1] / det; Ni[3] = -N[3] / det; Ni[4] = N[0] / det;
      } else {
        double a = N[0], b_ = N[1], c = N[2], d = N[3], e = N[4], f = N[5], g = N[6], hh = N[7], k = N[8];
        double det = a * (e * k - f * hh) - b_ * (d * k - f * g) + c * (d * hh - e * g);
        Ni[0] = (e * k - f * hh) / det; Ni[1] = (c * hh - b_ * k) / det; Ni[2] = (b_ * f - c * e) / det;
        Ni[3] = (f * g - d * k) / det; Ni[4] = (a * k - c * g) / det; Ni[5] = (c * d - a * f) / det;
        Ni[6] = (d * hh - e * g) / det; Ni[7] = (b_ * g - a * hh) / det; Ni[8] = (a * e - b_ * d) / det;
      }
      std::vector<double> G(D * m);
      for (int r = 0; r < D; ++r)
        for (int p = 0; p < m; ++p) {
          double s = 0.0;
          for (int c = 0; c < D; ++c) s += Ni[r * 3 + c] * A[p * D + c];
          G[r * m + p] = s;
        }
      lsG[i] = G;
    }
  }

  // Gradient of a cell field given per-face neighbour values (step 4/5).
  // nb[p] is the stencil value through face p of cell i.  `exact` gives the
  // plain least-squares gradient whatever the order and limiter.
  void ls_grad(int64_t i, double vi, const double* nb, double* g, bool exact = false) const {
    if (first_order && !exact) {  // piecewise-constant reconstruction
      for (int d = 0; d < D; ++d) g[d] = 0.0;
      return;
    }
    int m = (int)cfaces[i].size();
    const std::vector<double>& G = lsG[i];
    for (int d = 0; d < D; ++d) {
      double s = 0.0;
      for (int p = 0; p < m; ++p) s += G[d * m + p] * (nb[p] - vi);
      g[d] = s;
    }
    if (limiter == 1 && !exact) venkatakrishnan(i, vi, nb, g);
  }

  // Offset x_f - x_i of face f's centroid from cell i's (as seen from R
  // across a periodic seam, the face centroid is shifted back).
  void face_offset(int64_t i, int64_t f, double* dx) const {
    const bool right = fbc[f] == BC_INTERIOR && fR[f] == i && fL[f] != i;
    for (int d = 0; d < D; ++d)
      dx[d] = fcen[f * D + d] - (right ? fshift[f * D + d] : 0.0) - cen[i * D + d];
  }

  // Reading R7: Venkatakrishnan's limiter scales the gradient g of a cell
  // field with value vi and stencil values nb.
  void venkatakrishnan(int64_t i, double vi, const double* nb, double* g) const {
    const int m = (int)cfaces[i].size();
    double vmax = vi, vmin = vi;
    for (int p = 0; p < m; ++p) {
      vmax = std::max(vmax, nb[p]);
      vmin = std::min(vmin, nb[p]);
    }
    const double h = std::pow(vol[i], 1.0 / D);
    const double eps2 = std::pow(limiter_k * h, 3);
    double phi = 1.0;
    for (int p = 0; p < m; ++p) {
      double dx[3];
      face_offset(i, cfaces[i][p], dx);
      double dm = 0.0;
      for (int d = 0; d < D; ++d) dm += g[d] * dx[d];
      if (dm == 0.0) continue;
      const double dp = dm > 0.0 ? vmax - vi : vmin - vi;
      const double psi = (dp * dp + eps2 + 2.0 * dm * dp) / (dp * dp + 2.0 * dm * dm + dm * dp + eps2);
      phi = std::min(phi, psi);
    }
    for (int d = 0; d < D; ++d) g[d] *= phi;
  }

  // The step bound of cell i (R5 without the CFL number):
  // 2 V_i / max_k sum_{j in faces(i)} S_j |u_k . n_j|.
  double cell_bound(int64_t i) const {
    double mx = 0.0;
    for (int64_t k = 0; k < nv; ++k) {
      double s = 0.0;
      for (int64_t f : cfaces[i]) {
        double un = 0.0;
        for (int d = 0; d < D; ++d) un += u[k * D + d] * fnorm[f * D + d];
        s += farea[f] * std::fabs(un);
      }
      mx = std::max(mx, s);
    }
    return 2.0 * vol[i] / mx;
  }

  double compute_dt(double cfl) const {
    double best = INFINITY;
    for (int64_t i = 0; i < nc; ++i) best = std::min(best, cell_bound(i));
    return cfl * best;
  }

  // Local time steps for steady problems (reading R26): cell i advances by
  // dt_i = dt * b_i / min_j b_j, b_i its R5 bound, so the most restrictive
  // cell keeps the global dt.  Faces integrate over the global dt; cell i
  // applies their integrals as rates over dt, for its own dt_i.
  bool lts = false;
  std::vector<double> dtc;
  void set_local_dt(bool on) {
    lts = on;
    dtc.clear();
    if (!on) return;
    std::vector<double> bnd(nc);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nc; ++i) bnd[i] = cell_bound(i);
    double mn = INFINITY;
    for (int64_t i = 0; i < nc; ++i) mn = std::min(mn, bnd[i]);
    dtc.resize(nc);
    for (int64_t i = 0; i < nc; ++i) dtc[i] = dt * (bnd[i] / mn);
  }
  double dt_cell(int64_t i) const { return lts ? dtc[i] : dt; }
  // S_f as cell i applies it: times dt_i / dt under local steps
  double area_for(int64_t i, int64_t f) const { return lts ? farea[f] * (dtc[i] / dt) : farea[f]; }

  // Heat flux of every cell (step 2, Eq. reduced_heat_flux).
  void heat_flux(const std::vector<Prim>& P) {
    q.assign(nc * D, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
      double acc[3] = {0, 0, 0};
      for (int64_t k = 0; k < nv; ++k) {
        double c[3], c2 = 0.0;
        for (int d = 0; d < D; ++d) {
          c[d] = u[k * D + d] - P[i].U[d];
          c2 += c[d] * c[d];
        }
        double hv = h[k * nc + i];
        double bv = nr == 2 ? b[k * nc + i] : 0.0;
        for (int d = 0; d < D; ++d) acc[d] += w[k] * c[d] * (c2 * hv + bv);
      }
      for (int d = 0; d < D; ++d) q[i * D + d] = 0.5 * acc[d];
    }
  }

  int step_once();
  bool first_order = false;  // zero every least-squares gradient
  double limiter_k = 0.0;    // Venkatakrishnan's K (reading R7)
  void macro_grad(const std::vector<double>& Wg, std::vector<double>& gW, bool exact = false) const;
};

extern "C" {

oracle_ctx* oracle_create(int D, int64_t nc, int64_t nf, const double* vol, const double* cen,
                          const int64_t* fcells, const double* farea, const double* fnorm,
                          const double* fcen, const double* fshift, const int32_t* fbc,
                          const int32_t* fbcid, int64_t nv, const double* u, const double* w,
                          int K, double Pr, double Rg, double Tref, double muref, double omega,
                          double cfl, double dt, int nbc, const int32_t* bckind, const double* bcrho,
                          const double* bcU, const double* bcT, const double* W0) {
  if ((D != 2 && D != 3) || K < 0 || nc <= 0 || nf <= 0 || nv <= 0) return nullptr;
  oracle_ctx* o = new oracle_ctx();
  o->D = D;
  o->K = K;
  o->kxi = K + 3 - D;
  o->nr = o->kxi > 0 ? 2 : 1;
  o->nc = nc; o->nf = nf; o->nv = nv;
  o->Pr = Pr; o->Rg = Rg; o->Tref = Tref; o->muref = muref; o->omega = omega;
  o->limiter = 0;
  o->vol.assign(vol, vol + nc);
  o->cen.assign(cen, cen + nc * D);
  o->farea.assign(farea, farea + nf);
  o->fnorm.assign(fnorm, fnorm + nf * D);
  o->fcen.assign(fcen, fcen + nf * D);
  if (fshift) o->fshift.assign(fshift, fshift + nf * D);
  else o->fshift.assign(nf * D, 0.0);
  o->fL.resize(nf); o->fR.resize(nf);
  for (int64_t f = 0; f < nf; ++f) { o->fL[f] = fcells[2 * f]; o->fR[f] = fcells[2 * f + 1]; }
  o->fbc.assign(fbc, fbc + nf);
  o->fbcid.assign(fbcid, fbcid + nf);
  o->u.assign(u, u + nv * D);
  o->w.assign(w, w + nv);
  o->nbc = nbc;
  o->bckind.assign(bckind, bckind + nbc);
  o->bcrho.assign(bcrho, bcrho + nbc);
  o->bcU.assign(bcU, bcU + 3 * nbc);
  o->bcT.assign(bcT, bcT + nbc);
  o->cfaces.assign(nc, {});
  for (int64_t f = 0; f < nf; ++f) {
    o->cfaces[o->fL[f]].push_back(f);
    if (o->fbc[f] == BC_INTERIOR) o->cfaces[o->fR[f]].push_back(f);
  }
  o->build_ls();
  o->dt = dt > 0.0 ? dt : o->compute_dt(cfl);
  o->W.assign(W0, W0 + nc * (D + 2));
  // initial distributions: the reduced Maxwellian of W0 (h = H, b = B)
  o->h.assign(nc * nv, 0.0);
  if (o->nr == 2) o->b.assign(nc * nv, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    Prim p = o->prim(&o->W[i * (D + 2)]);
    for (int64_t k = 0; k < nv; ++k) {
      double H = o->H_at(p.rho, p.U, p.lam, k);
      o->h[k * nc + i] = H;
      if (o->nr == 2) o->b[k * nc + i] = o->kxi / (2.0 * p.lam) * H;
    }
  }
  o->rho_prev.resize(nc);
  for (int64_t i = 0; i < nc; ++i) o->rho_prev[i] = o->W[i * (D + 2)];
  return o;
}

void oracle_destroy(oracle_ctx* o) { delete o; }

double oracle_dt(const oracle_ctx* o) { return o->dt; }

int oracle_step(oracle_ctx* o, int nsteps, double* residual_out) {
  for (int s = 0; s < nsteps; ++s) {
    int rc = o->step_once();
    if (rc) return rc;
  }
  if (residual_out) {
    residual_out[0] = o->last_res;
    residual_out[1] = o->last_change;
  }
  return 0;
}

// W: nc x (D+2); h, b: nc x nv (cell-major, as the library exposes them); q: nc x D
void oracle_get_state(const oracle_ctx* o, double* W, double* h, double* b, double* q) {
  int64_t nc = o->nc, nv = o->nv;
  if (W) std::memcpy(W, o->W.data(), sizeof(double) * nc * (o->D + 2));
  if (h)
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t k = 0; k < nv; ++k) h[i * nv + k] = o->h[k * nc + i];
  if (b)
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t k = 0; k < nv; ++k) b[i * nv + k] = o->nr == 2 ? o->b[k * nc + i] : 0.0;
  if (q) {
    // heat flux of the current state
    oracle_ctx* m = const_cast<oracle_ctx*>(o);
    std::vector<Prim> P(nc);
    for (int64_t i = 0; i < nc; ++i) P[i] = m->prim(&m->W[i * (m->D + 2)]);
    std::vector<double> save = m->q;
    m->heat_flux(P);
    std::memcpy(q, m->q.data(), sizeof(double) * nc * m->D);
    m->q = save;
  }
}

// Overwrite the state (h, b cell-major).  Used by tests that start from a
// non-equilibrium distribution.
void oracle_set_state(oracle_ctx* o, const double* W, const double* h, const double* b) {
  int64_t nc = o->nc, nv = o->nv;
  if (W) std::memcpy(o->W.data(), W, sizeof(double) * nc * (o->D + 2));
  if (h)
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t k = 0; k < nv; ++k) o->h[k * nc + i] = h[i * nv + k];
  if (b && o->nr == 2)
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t k = 0; k < nv; ++k) o->b[k * nc + i] = b[i * nv + k];
  for (int64_t i = 0; i < nc; ++i) o->rho_prev[i] = o->W[i * (o->D + 2)];
}

// Diagnostics of the last step: macroscopic face fluxes F (nf x (D+2)),
// wall densities (nf, 0 elsewhere), interface states W0 (nf x (D+2)) and tau0.
void oracle_get_faces(const oracle_ctx* o, double* F, double* rhow, double* W0, double* tau0) {
  int64_t nf = o->nf;
  int nw = o->D + 2;
  if (F && !o->F.empty()) std::memcpy(F, o->F.data(), sizeof(double) * nf * nw);
  if (rhow && !o->rhow.empty()) std::memcpy(rhow, o->rhow.data(), sizeof(double) * nf);
  if (W0 && !o->fW0.empty()) std::memcpy(W0, o->fW0.data(), sizeof(double) * nf * nw);
  if (tau0 && !o->ftau0.empty()) std::memcpy(tau0, o->ftau0.data(), sizeof(double) * nf);
}

// ---- Stand-alone pieces, exported so the tests can pin them one by one ----

void oracle_gamma(double dt, double tau, double* G) { gamma_coeffs(dt, tau, G); }

// Half-range moments <u_n^m>_{+/-}, m = 0..nm-1, of a 1-D Maxwellian with mean
// Un and parameter lam, normalised to unit density (step 6.2).
void oracle_half_moments(double Un, double lam, int sign, int nm, double* out) {
  double m0 = 0.5 * std::erfc(-sign * std::sqrt(lam) * Un);
  double m1 = Un * m0 + sign * std::exp(-lam * Un * Un) / (2.0 * std::sqrt(M_PI * lam));
  out[0] = m0;
  if (nm > 1) out[1] = m1;
  for (int m = 0; m + 2 < nm; ++m) out[m + 2] = Un * out[m + 1] + (m + 1) / (2.0 * lam) * out[m];
}

// Interface state W0 from left/right conservative states and the unit normal
// (a gas of K internal degrees of freedom).
int oracle_interface_state_k(int D, int K, const double* Wl, const double* Wr, const double* n,
                             double* W0);
int oracle_interface_state(int D, const double* Wl, const double* Wr, const double* n, double* W0) {
  return oracle_interface_state_k(D, 0, Wl, Wr, n, W0);
}

// Slopes: given the interface state (rho, U, lam) and conservative-variable
// derivatives dW (D rows of D+2), return the spatial slopes a (D x (D+2)) and the
// time slope A (D+2), each in the psi basis (step 6.4-6.5).
int oracle_slopes_k(int D, int K, double rho, const double* U, double lam, const double* dW,
                    double* a, double* A);
int oracle_slopes(int D, double rho, const double* U, double lam, const double* dW, double* a,
                  double* A) {
  return oracle_slopes_k(D, 0, rho, U, lam, dW, a, A);
}

// Gram matrix E[psi psi^T] (normalised) for a check of the solve.
void oracle_gram_k(int D, int K, const double* U, double lam, double* M) {
  Gauss g{D, K + 3 - D, {0, 0, 0}, 1.0 / (2.0 * lam)};
  for (int d = 0; d < D; ++d) g.U[d] = U[d];
  std::vector<Poly> psi = invariants(D);
  std::vector<double> G = gram(g, psi);
  std::copy(G.begin(), G.end(), M);
}
void oracle_gram(int D, const double* U, double lam, double* M) { oracle_gram_k(D, 0, U, lam, M); }

// E[u_d psi psi^T] (normalised), D x (D+2) x (D+2).
void oracle_gram_u_k(int D, int K, const double* U, double lam, double* Mu) {
  Gauss g{D, K + 3 - D, {0, 0, 0}, 1.0 / (2.0 * lam)};
  for (int d = 0; d < D; ++d) g.U[d] = U[d];
  std::vector<Poly> psi = invariants(D);
  int n = D + 2;
  for (int d = 0; d < D; ++d) {
    Poly ud;
    Mono m{0, 0, 0, 0};
    m[d] = 1;
    ud[m] = 1.0;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) Mu[(d * n + a) * n + b] = g.expect(poly_mul(ud, poly_mul(psi[a], psi[b])));
  }
}
void oracle_gram_u(int D, const double* U, double lam, double* Mu) { oracle_gram_u_k(D, 0, U, lam, Mu); }

// Least-squares coefficients of cell i (D x m, row-major) and m.
int oracle_ls_coeffs(const oracle_ctx* o, int64_t i, double* G) {
  int m = (int)o->cfaces[i].size();
  if (G) std::copy(o->lsG[i].begin(), o->lsG[i].end(), G);
  return m;
}

}  // extern "C"

// ---------------------------------------------------------------------------
int oracle_interface_state_k(int D, int K, const double* Wl, const double* Wr, const double* n,
                             double* W0) {
  const int kxi = K + 3 - D;
  const double* Ws[2] = {Wl, Wr};
  int sgn[2] = {+1, -1};
  for (int v = 0; v < D + 2; ++v) W0[v] = 0.0;
  for (int s = 0; s < 2; ++s) {
    const double* Wc = Ws[s];
    double rho = Wc[0], U[3] = {0, 0, 0}, u2 = 0.0;
    for (int d = 0; d < D; ++d) { U[d] = Wc[1 + d] / rho; u2 += U[d] * U[d]; }
    double lam = (K + 3.0) * rho / (4.0 * (Wc[D + 1] - 0.5 * rho * u2));
    double Un = 0.0;
    for (int d = 0; d < D; ++d) Un += U[d] * n[d];
    double Ut[3], ut2 = 0.0;
    for (int d = 0; d < D; ++d) { Ut[d] = U[d] - Un * n[d]; ut2 += Ut[d] * Ut[d]; }
    double hm[3];
    oracle_half_moments(Un, lam, sgn[s], 3, hm);
    W0[0] += rho * hm[0];
    for (int d = 0; d < D; ++d) W0[1 + d] += rho * (hm[1] * n[d] + hm[0] * Ut[d]);
    W0[D + 1] += 0.5 * rho * (hm[2] + hm[0] * (ut2 + (D - 1 + kxi) / (2.0 * lam)));
  }
  return 0;
}

int oracle_slopes_k(int D, int K, double rho, const double* U, double lam, const double* dW,
                    double* a, double* A) {
  Gauss g{D, K + 3 - D, {0, 0, 0}, 1.0 / (2.0 * lam)};
  for (int d = 0; d < D; ++d) g.U[d] = U[d];
  std::vector<Poly> psi = invariants(D);
  int n = D + 2;
  std::vector<double> M = gram(g, psi);
  std::vector<double> x;
  for (int d = 0; d < D; ++d) {
    std::vector<double> r(n);
    for (int v = 0; v < n; ++v) r[v] = dW[d * n + v] / rho;
    if (!cholesky_solve(n, M, x, r)) return -1;
    for (int v = 0; v < n; ++v) a[d * n + v] = x[v];
  }
  // compatibility: E[psi (A.psi)] = - sum_d E[u_d psi (a_d . psi)]
  std::vector<double> r(n, 0.0);
  for (int d = 0; d < D; ++d) {
    Poly ad;  // a_d . psi
    for (int v = 0; v < n; ++v)
      for (auto& t : psi[v]) ad[t.first] += a[d * n + v] * t.second;
    Poly ud;
    Mono m{0, 0, 0, 0};
    m[d] = 1;
    ud[m] = 1.0;
    Poly uad = poly_mul(ud, ad);
    for (int v = 0; v < n; ++v) r[v] -= g.expect(poly_mul(psi[v], uad));
  }
  if (!cholesky_solve(n, M, x, r)) return -1;
  for (int v = 0; v < n; ++v) A[v] = x[v];
  return 0;
}

// ---------------------------------------------------------------------------
// Least-squares gradients of every conservative component of every cell
// (step 4), with the ghost rules of R6: the neighbour's value through an
// interior face, the cell's own value through a wall, the ghost state Wg of
// a far-field or outflow face.  gW[(i*D + d)*nw + v] = d W_v / d x_d.
void oracle_ctx::macro_grad(const std::vector<double>& Wg, std::vector<double>& gW, bool exact) const {
  const int nw = NW();
  auto nbW = [&](int64_t i, int64_t f, int v) -> double {
    if (fbc[f] == BC_INTERIOR) return W[(fL[f] == i ? fR[f] : fL[f]) * nw + v];
    if (fbc[f] == BC_WALL) return W[i * nw + v];
    return Wg[f * nw + v];
  };
  gW.assign(nc * D * nw, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nc; ++i) {
    int m = (int)cfaces[i].size();
    std::vector<double> nb(m);
    for (int v = 0; v < nw; ++v) {
      for (int p = 0; p < m; ++p) nb[p] = nbW(i, cfaces[i][p], v);
      double g[3];
      ls_grad(i, W[i * nw + v], nb.data(), g, exact);
      for (int d = 0; d < D; ++d) gW[(i * D + d) * nw + v] = g[d];
    }
  }
}

// ---------------------------------------------------------------------------
// One time step (the numbered steps follow the one-step algorithm).
int oracle_ctx::step_once() {
  const int nw = NW();
  // 1. primitives and relaxation time of W^n
  std::vector<Prim> P(nc);
  for (int64_t i = 0; i < nc; ++i) {
    P[i] = prim(&W[i * nw]);
    if (!P[i].ok) { err = "non-positive density or temperature"; return -4; }
  }
  // 2. heat flux q^n
  heat_flux(P);
  // 3. ghost states of far-field / outflow faces
  std::vector<double> Wg(nf * nw, 0.0);
  for (int64_t f = 0; f < nf; ++f)
    if (fbc[f] == BC_FARFIELD || fbc[f] == BC_OUTFLOW) ghost_W(f, &W[fL[f] * nw], &Wg[f * nw]);
  std::vector<Prim> Pg(nf);
  for (int64_t f = 0; f < nf; ++f)
    if (fbc[f] == BC_FARFIELD || fbc[f] == BC_OUTFLOW) Pg[f] = prim(&Wg[f * nw]);

  // 4. macroscopic gradients
  std::vector<double> gW;
  macro_grad(Wg, gW);

  // 6.1-6.6 interface equilibrium data of every non-wall face
  struct FaceEq {
    double rho0, U0[3], lam0, tau0, G[5], a[3][5], A[5], q0[3];
    double W0[5];
  };
  std::vector<FaceEq> fe(nf);
  bool bad = false;
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < nf; ++f) {
    if (fbc[f] == BC_WALL) continue;
    FaceEq& e = fe[f];
    int64_t L = fL[f];
    bool ghost = fbc[f] != BC_INTERIOR;
    int64_t R = ghost ? -1 : fR[f];
    double Wl[5], Wr[5];
    for (int v = 0; v < nw; ++v) {
      double sl = 0.0, sr = 0.0;
      for (int d = 0; d < D; ++d) {
        sl += (fcen[f * D + d] - cen[L * D + d]) * gW[(L * D + d) * nw + v];
        if (!ghost) sr += (fcen[f * D + d] - fshift[f * D + d] - cen[R * D + d]) * gW[(R * D + d) * nw + v];
      }
      Wl[v] = W[L * nw + v] + sl;
      Wr[v] = ghost ? Wg[f * nw + v] : W[R * nw + v] + sr;
    }
    // first-order fallback if a reconstructed state is not physical
    if (!prim(Wl).ok)
      for (int v = 0; v < nw; ++v) Wl[v] = W[L * nw + v];
    if (!prim(Wr).ok)
      for (int v = 0; v < nw; ++v) Wr[v] = ghost ? Wg[f * nw + v] : W[R * nw + v];
    oracle_interface_state_k(D, K, Wl, Wr, &fnorm[f * D], e.W0);
    Prim p0 = prim(e.W0);
    if (!p0.ok) { bad = true; continue; }
    e.rho0 = p0.rho; e.lam0 = p0.lam; e.tau0 = p0.tau;
    for (int d = 0; d < 3; ++d) e.U0[d] = p0.U[d];
    gamma_coeffs(dt, p0.tau, e.G);
    double dW[3 * 5];
    for (int d = 0; d < D; ++d)
      for (int v = 0; v < nw; ++v)
        dW[d * nw + v] = 0.5 * (gW[(L * D + d) * nw + v] + (ghost ? 0.0 : gW[(R * D + d) * nw + v]));
    double a[15], A[5];
    if (oracle_slopes_k(D, K, p0.rho, p0.U, p0.lam, dW, a, A)) { bad = true; continue; }
    for (int d = 0; d < D; ++d)
      for (int v = 0; v < nw; ++v) e.a[d][v] = a[d * nw + v];
    for (int v = 0; v < nw; ++v) e.A[v] = A[v];
    for (int d = 0; d < D; ++d) e.q0[d] = 0.5 * (q[L * D + d] + (ghost ? 0.0 : q[R * D + d]));
  }
  if (bad) { err = "non-physical interface state"; return -4; }

  // micro ghost values (R6): wall -> own value; far field -> ghost Maxwellian
  auto ghost_h = [&](int64_t f, int64_t k, double& hv, double& bv) {
    const Prim& g = Pg[f];
    hv = H_at(g.rho, g.U, g.lam, k);
    bv = kxi / (2.0 * g.lam) * hv;
  };
  // gradients of h (and b) of cell i at velocity k
  auto micro_grad = [&](int64_t i, int64_t k, double* gh, double* gb) {
    int m = (int)cfaces[i].size();
    double nbh[8], nbb[8];
    double hi = h[k * nc + i], bi = nr == 2 ? b[k * nc + i] : 0.0;
    for (int p = 0; p < m; ++p) {
      int64_t f = cfaces[i][p];
      if (fbc[f] == BC_INTERIOR) {
        int64_t j = fL[f] == i ? fR[f] : fL[f];
        nbh[p] = h[k * nc + j];
        nbb[p] = nr == 2 ? b[k * nc + j] : 0.0;
      } else if (fbc[f] == BC_WALL) {
        nbh[p] = hi;
        nbb[p] = bi;
      } else {
        ghost_h(f, k, nbh[p], nbb[p]);
      }
    }
    ls_grad(i, hi, nbh, gh);
    if (nr == 2) ls_grad(i, bi, nbb, gb);
    else for (int d = 0; d < D; ++d) gb[d] = 0.0;
  };

  // 7 (first half). wall density of every wall face (Eq. wall_density_condition)
  rhow.assign(nf, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t f = 0; f < nf; ++f) {
    if (fbc[f] != BC_WALL) continue;
    int64_t L = fL[f];
    int id = fbcid[f];
    double Tw = bcT[id];
    double lamw = 1.0 / (2.0 * Rg * Tw);
    double Uw[3] = {bcU[id * 3], bcU[id * 3 + 1], bcU[id * 3 + 2]};
    double incident = 0.0, reflected = 0.0;
    for (int64_t k = 0; k < nv; ++k) {
      double un = 0.0;
      for (int d = 0; d < D; ++d) un += u[k * D + d] * fnorm[f * D + d];
      if (un > 0.0) {
        double gh[3], gb[3];
        micro_grad(L, k, gh, gb);
        double hf = h[k * nc + L], ugh = 0.0;
        for (int d = 0; d < D; ++d) {
          hf += (fcen[f * D + d] - cen[L * D + d]) * gh[d];
          ugh += u[k * D + d] * gh[d];
        }
        double ih = dt * hf - 0.5 * dt * dt * ugh;
        incident += w[k] * un * ih;
      } else if (un < 0.0) {
        reflected += w[k] * un * H_at(1.0, Uw, lamw, k);
      }
    }
    rhow[f] = -incident / (dt * reflected);
  }

  // 5-9. sweep the velocity space one point at a time
  F.assign(nf * nw, 0.0);
  fW0.assign(nf * nw, 0.0);
  ftau0.assign(nf, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    if (fbc[f] == BC_WALL) continue;
    for (int v = 0; v < nw; ++v) fW0[f * nw + v] = fe[f].W0[v];
    ftau0[f] = fe[f].tau0;
  }
  std::vector<double> ht(nc * nv), bt(nr == 2 ? nc * nv : 0);
  std::vector<double> gh(nc * D), gb(nc * D);
  std::vector<double> Hf(nf), Bf(nf);
  const double xi4_fac = kxi * (kxi + 2.0);
  for (int64_t k = 0; k < nv; ++k) {
    const double* uk = &u[k * D];
    double u2 = 0.0;
    for (int d = 0; d < D; ++d) u2 += uk[d] * uk[d];
    // 5. microscopic gradients at this velocity
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) micro_grad(i, k, &gh[i * D], &gb[i * D]);
    // 6.7 / 7. time-integrated microscopic fluxes through every face
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
      double un = 0.0;
      for (int d = 0; d < D; ++d) un += uk[d] * fnorm[f * D + d];
      int64_t L = fL[f];
      double ih = 0.0, ib = 0.0;
      if (fbc[f] == BC_WALL) {
        int id = fbcid[f];
        double lamw = 1.0 / (2.0 * Rg * bcT[id]);
        double Uw[3] = {bcU[id * 3], bcU[id * 3 + 1], bcU[id * 3 + 2]};
        if (un > 0.0) {
          double hf = h[k * nc + L], bf = nr == 2 ? b[k * nc + L] : 0.0, ugh = 0.0, ugb = 0.0;
          for (int d = 0; d < D; ++d) {
            double dx = fcen[f * D + d] - cen[L * D + d];
            hf += dx * gh[L * D + d];
            bf += dx * gb[L * D + d];
            ugh += uk[d] * gh[L * D + d];
            ugb += uk[d] * gb[L * D + d];
          }
          ih = dt * hf - 0.5 * dt * dt * ugh;
          ib = dt * bf - 0.5 * dt * dt * ugb;
        } else if (un < 0.0) {
          double Hw = H_at(1.0, Uw, lamw, k);
          ih = dt * rhow[f] * Hw;
          ib = dt * rhow[f] * kxi / (2.0 * lamw) * Hw;
        }
      } else {
        const FaceEq& e = fe[f];
        bool ghost = fbc[f] != BC_INTERIOR;
        // upwind reconstruction (Eq. initial_reconstruction)
        // u_n > 0: left cell; u_n <= 0: right cell (or the ghost Maxwellian with
        // zero gradient); at u_n = 0 the flux vanishes whichever side is used
        double hf, bf, ugh = 0.0, ugb = 0.0;
        if (un <= 0.0 && ghost) {
          ghost_h(f, k, hf, bf);
        } else {
          int64_t up = un > 0.0 ? L : fR[f];
          // face centroid as seen from R is shifted back by the periodic translation
          double shift_sign = un > 0.0 ? 0.0 : 1.0;
          hf = h[k * nc + up];
          bf = nr == 2 ? b[k * nc + up] : 0.0;
          for (int d = 0; d < D; ++d) {
            double dx = fcen[f * D + d] - shift_sign * fshift[f * D + d] - cen[up * D + d];
            hf += dx * gh[up * D + d];
            bf += dx * gb[up * D + d];
            ugh += uk[d] * gh[up * D + d];
            ugb += uk[d] * gb[up * D + d];
          }
        }
        // interface equilibrium and its derivatives (Eq. equilibrium_expansion)
        double H0 = H_at(e.rho0, e.U0, e.lam0, k);
        double B0 = kxi / (2.0 * e.lam0) * H0;
        double H0p, B0p;
        shakhov(e.rho0, e.U0, e.lam0, e.q0, k, H0, H0p, B0p);
        double xi4 = xi4_fac / (4.0 * e.lam0 * e.lam0);
        double uH = 0.0, uB = 0.0;
        for (int d = 0; d < D; ++d) {
          double Pd = e.a[d][0] + 0.5 * e.a[d][D + 1] * u2;
          for (int c = 0; c < D; ++c) Pd += e.a[d][1 + c] * uk[c];
          uH += uk[d] * (Pd * H0 + 0.5 * e.a[d][D + 1] * B0);
          uB += uk[d] * (Pd * B0 + 0.5 * e.a[d][D + 1] * xi4 * H0);
        }
        double PA = e.A[0] + 0.5 * e.A[D + 1] * u2;
        for (int c = 0; c < D; ++c) PA += e.A[1 + c] * uk[c];
        double tH = PA * H0 + 0.5 * e.A[D + 1] * B0;
        double tB = PA * B0 + 0.5 * e.A[D + 1] * xi4 * H0;
        // time integral of the interface distribution (Eq. interface_distribution)
        ih = e.G[0] * hf + e.G[1] * ugh + e.G[2] * (H0 + H0p) + e.G[3] * uH + e.G[4] * tH;
        ib = e.G[0] * bf + e.G[1] * ugb + e.G[2] * (B0 + B0p) + e.G[3] * uB + e.G[4] * tB;
      }
      double Hk = un * ih, Bk = un * ib;
      Hf[f] = Hk;
      Bf[f] = Bk;
      // 6.8 macroscopic flux (Eq. macro_flux), accumulated over k ascending
      double* Fj = &F[f * nw];
      Fj[0] += w[k] * Hk;
      for (int d = 0; d < D; ++d) Fj[1 + d] += w[k] * uk[d] * Hk;
      Fj[D + 1] += w[k] * 0.5 * (u2 * Hk + Bk);
    }
    // 9. first stage (Eq. f_tilde)
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
      double sh = 0.0, sb = 0.0;
      for (int64_t f : cfaces[i]) {
        double sg = fL[f] == i ? 1.0 : -1.0;
        sh += sg * area_for(i, f) * Hf[f];
        sb += sg * area_for(i, f) * Bf[f];
      }
      const Prim& p = P[i];
      double H = H_at(p.rho, p.U, p.lam, k);
      double Hp, Bp;
      shakhov(p.rho, p.U, p.lam, &q[i * D], k, H, Hp, Bp);
      double B = kxi / (2.0 * p.lam) * H;
      double c = dt_cell(i) / (2.0 * p.tau);
      double hv = h[k * nc + i];
      ht[k * nc + i] = hv - sh / vol[i] + c * (H + Hp - hv);
      if (nr == 2) {
        double bv = b[k * nc + i];
        bt[k * nc + i] = bv - sb / vol[i] + c * (B + Bp - bv);
      }
    }
  }
  // 8. macroscopic update (Eq. macro_update)
  std::vector<double> Wn(W);
  for (int64_t i = 0; i < nc; ++i) {
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t f : cfaces[i]) {
      double sg = fL[f] == i ? 1.0 : -1.0;
      for (int v = 0; v < nw; ++v) acc[v] += sg * area_for(i, f) * F[f * nw + v];
    }
    for (int v = 0; v < nw; ++v) Wn[i * nw + v] = W[i * nw + v] - acc[v] / vol[i];
  }
  // 10-11. new equilibrium and the second stage (Eq. f_final)
  std::vector<Prim> Pn(nc);
  for (int64_t i = 0; i < nc; ++i) {
    Pn[i] = prim(&Wn[i * nw]);
    if (!Pn[i].ok) { err = "non-positive density or temperature after update"; return -4; }
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nc; ++i) {
    const Prim& p = Pn[i];
    double a = dt_cell(i) / (2.0 * p.tau);
    for (int64_t k = 0; k < nv; ++k) {
      double H = H_at(p.rho, p.U, p.lam, k);
      double Hp, Bp;
      shakhov(p.rho, p.U, p.lam, &q[i * D], k, H, Hp, Bp);
      h[k * nc + i] = (ht[k * nc + i] + a * (H + Hp)) / (1.0 + a);
      if (nr == 2) {
        double B = kxi / (2.0 * p.lam) * H;
        b[k * nc + i] = (bt[k * nc + i] + a * (B + Bp)) / (1.0 + a);
      }
    }
  }
  // 12. residual of the density (R20)
  double num = 0.0, den = 0.0, rn = 0.0;
  for (int64_t i = 0; i < nc; ++i) {
    double d = Wn[i * nw] - W[i * nw];
    num += vol[i] * d * d;
    den += vol[i];
    rn += vol[i] * W[i * nw] * W[i * nw];
  }
  double nrm = std::sqrt(num / den);
  // normalise by the first step that changed the density (a gas at rest can
  // keep rho unchanged for the first step)
  if (res_norm0 == 0.0) res_norm0 = nrm;
  last_res = res_norm0 > 0.0 ? nrm / res_norm0 : 0.0;
  last_change = nrm / std::sqrt(rn / den);
  W.swap(Wn);
  ++steps_done;
  return 0;
}

// Local time steps (reading R26): on = 1 gives every cell its own step.
extern "C" void oracle_set_local_dt(oracle_ctx* o, int on) { o->set_local_dt(on != 0); }

// The cells' steps, [nc] (the global dt everywhere when off).
extern "C" void oracle_local_dt(const oracle_ctx* o, double* dtc) {
  for (int64_t i = 0; i < o->nc; ++i) dtc[i] = o->dt_cell(i);
}

// Reconstruction order: 1 = first order (all gradients zero), 2 = least squares.
extern "C" void oracle_set_order(oracle_ctx* o, int order) { o->first_order = order == 1; }

// Slope limiter (reading R7): kind 0 = none, 1 = Venkatakrishnan with constant K.
extern "C" void oracle_set_limiter(oracle_ctx* o, int kind, double K) {
  o->limiter = kind == 1 ? 1 : 0;
  o->limiter_k = K;
}

// Gradients of h and b at velocity k of the current state, as the next step
// reconstructs them (order and limiter applied), [nc*D] each.
extern "C" void oracle_micro_grad(const oracle_ctx* o, int64_t k, double* gh, double* gb) {
  const int D = o->D;
  std::vector<double> Wg(o->nf * o->NW(), 0.0);
  for (int64_t f = 0; f < o->nf; ++f)
    if (o->fbc[f] == BC_FARFIELD || o->fbc[f] == BC_OUTFLOW)
      o->ghost_W(f, &o->W[o->fL[f] * o->NW()], &Wg[f * o->NW()]);
  for (int64_t i = 0; i < o->nc; ++i) {
    const int m = (int)o->cfaces[i].size();
    std::vector<double> nbh(m), nbb(m);
    const double hi = o->h[k * o->nc + i], bi = o->nr == 2 ? o->b[k * o->nc + i] : 0.0;
    for (int p = 0; p < m; ++p) {
      const int64_t f = o->cfaces[i][p];
      if (o->fbc[f] == BC_INTERIOR) {
        const int64_t j = o->fL[f] == i ? o->fR[f] : o->fL[f];
        nbh[p] = o->h[k * o->nc + j];
        nbb[p] = o->nr == 2 ? o->b[k * o->nc + j] : 0.0;
      } else if (o->fbc[f] == BC_WALL) {
        nbh[p] = hi;
        nbb[p] = bi;
      } else {
        const double* Wf = &Wg[f * o->NW()];
        Prim g = o->prim(Wf);
        nbh[p] = o->H_at(g.rho, g.U, g.lam, k);
        nbb[p] = o->kxi / (2.0 * g.lam) * nbh[p];
      }
    }
    o->ls_grad(i, hi, nbh.data(), &gh[i * D]);
    if (o->nr == 2) o->ls_grad(i, bi, nbb.data(), &gb[i * D]);
    else
      for (int d = 0; d < D; ++d) gb[i * D + d] = 0.0;
  }
}

// Gradients of W of the current state as the next step reconstructs them
// (order and limiter applied), [nc*D*(D+2)].
extern "C" void oracle_macro_grad(const oracle_ctx* o, double* gW) {
  const int nw = o->NW();
  std::vector<double> Wg(o->nf * nw, 0.0);
  for (int64_t f = 0; f < o->nf; ++f)
    if (o->fbc[f] == BC_FARFIELD || o->fbc[f] == BC_OUTFLOW) o->ghost_W(f, &o->W[o->fL[f] * nw], &Wg[f * nw]);
  std::vector<double> g;
  o->macro_grad(Wg, g, false);
  std::copy(g.begin(), g.end(), gW);
}

// Least-squares gradients of the current state (steps 3-4 only; nothing
// advances), whatever the reconstruction order.
extern "C" void oracle_grad_W(const oracle_ctx* o, double* gW) {
  const int nw = o->NW();
  std::vector<double> Wg(o->nf * nw, 0.0);
  for (int64_t f = 0; f < o->nf; ++f)
    if (o->fbc[f] == BC_FARFIELD || o->fbc[f] == BC_OUTFLOW) o->ghost_W(f, &o->W[o->fL[f] * nw], &Wg[f * nw]);
  std::vector<double> g;
  o->macro_grad(Wg, g, true);
  std::copy(g.begin(), g.end(), gW);
}

extern "C" const char* oracle_last_error(const oracle_ctx* o) { return o->err.c_str(); }
extern "C" int64_t oracle_steps_done(const oracle_ctx* o) { return o->steps_done; }

// Threads the oracle's parallel loops use.
extern "C" int oracle_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Set the threads of the following parallel loops (n >= 1); the results do
// not depend on it (every reduction over velocities is sequential).
extern "C" void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
