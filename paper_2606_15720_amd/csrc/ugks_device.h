// Device helpers shared by the staged kernels and the fused sweep.
#pragma once

#include "ugks_internal.h"

#include <cmath>

namespace ugks {
namespace dev {

constexpr int TPB = 256;  // threads per block for velocity-parallel kernels

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return static_cast<double>(p[i]);
}
template <typename T>
__device__ __forceinline__ void st(T* p, int64_t i, double v) {
  p[i] = static_cast<T>(v);
}

// (lambda/pi)^(D/2)
template <int D>
__device__ __forceinline__ double maxw_norm(double lam) {
  double r = lam * M_1_PI;
  if constexpr (D == 2) return r;
  else return r * sqrt(r);
}

// Primitive variables of a conservative state of a gas with K internal
// degrees of freedom: lambda = (K + 3) rho / (4 (rho E - rho|U|^2/2)), p = rho/(2 lambda),
// T = 1/(2 R lambda), tau = mu(T)/p with mu = mu_ref (T/T_ref)^omega.
template <int D>
__device__ __forceinline__ bool prim_of(const double* W, const GasP& g, double* P) {
  double rho = W[0];
  double u2 = 0.0;
  double U[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < D; ++d) {
    U[d] = W[1 + d] / rho;
    u2 += U[d] * U[d];
  }
  double eint = W[D + 1] - 0.5 * rho * u2;
  double lam = (g.K + 3.0) * rho / (4.0 * eint);
  double p = rho / (2.0 * lam);
  double T = 1.0 / (2.0 * g.R * lam);
  double tau = g.muref * pow(T / g.Tref, g.omega) / p;
  P[0] = rho;
  P[1] = U[0];
  P[2] = U[1];
  P[3] = U[2];
  P[4] = lam;
  P[5] = tau;
  P[6] = p;
  P[7] = 0.0;
  return (rho > 0.0) && (eint > 0.0) && isfinite(lam) && isfinite(tau);
}

// Conservative state of (rho, U, T) for a gas with K internal degrees of freedom.
template <int D>
__device__ __forceinline__ void cons_of(double rho, const double* U, double T, double R, double K,
                                        double* W) {
  double u2 = 0.0;
  W[0] = rho;
  for (int d = 0; d < D; ++d) {
    W[1 + d] = rho * U[d];
    u2 += U[d] * U[d];
  }
  W[D + 1] = 0.5 * rho * u2 + 0.5 * (K + 3.0) * rho * R * T;
}

// Far-field / outflow ghost state: free stream when it enters through the
// face, otherwise the interior state.
template <int D>
__device__ __forceinline__ void ghost_state(int kind, const DevBC& bc, const double* n,
                                            const double* Wi, double R, double K, double* Wg) {
  bool inflow = false;
  if (kind == UGKS_BC_FARFIELD) {
    double un = 0.0;
    for (int d = 0; d < D; ++d) un += bc.U[d] * n[d];
    inflow = un < 0.0;
  }
  if (inflow) {
    cons_of<D>(bc.rho, bc.U, bc.T, R, K, Wg);
  } else {
    for (int v = 0; v < D + 2; ++v) Wg[v] = Wi[v];
  }
}

// Reduce N per-thread values over a block of TPB threads; the result is
// valid in thread 0.  Fixed order: wave shuffle tree, then waves in order.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* lds) {
#pragma unroll
  for (int n = 0; n < N; ++n) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v[n] += __shfl_down(v[n], off, WAVE);
  }
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  if (lane == 0)
#pragma unroll
    for (int n = 0; n < N; ++n) lds[n * 16 + wv] = v[n];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
      double s = lds[n * 16];
      for (int w = 1; w < nw; ++w) s += lds[n * 16 + w];
      v[n] = s;
    }
  }
}

__device__ __forceinline__ double block_max(double v, double* lds) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, WAVE));
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) v = fmax(v, lds[w]);
  }
  return v;
}

// ---------------------------------------------------------------------------
// Interface equilibrium (steps 6.1-6.6)

// Half-range moments <u_n^m>_{s}, m = 0, 1, 2, of a unit-density 1-D
// Maxwellian with mean Un; s = +1 for u_n > 0, -1 for u_n < 0.
__device__ __forceinline__ void half_range(double Un, double lam, double s, double* m) {
  double sl = sqrt(lam);
  m[0] = 0.5 * erfc(-s * sl * Un);
  m[1] = Un * m[0] + s * exp(-lam * Un * Un) / (2.0 * sqrt(M_PI * lam));
  m[2] = Un * m[1] + m[0] / (2.0 * lam);
}

// Solve E[psi psi^T] a = b for a Maxwellian (U, lam) with N = K + 3
// translational plus internal degrees of freedom, by elimination of a_0, a_j, a_E.
template <int D>
__device__ __forceinline__ void slope_solve(const double* b, const double* U, double lam, double N,
                                            double* a) {
  double UU = 0.0, UR = 0.0, Rj[3];
  for (int d = 0; d < D; ++d) {
    UU += U[d] * U[d];
    Rj[d] = b[1 + d] - U[d] * b[0];
    UR += U[d] * Rj[d];
  }
  double e2 = UU + N / (2.0 * lam);
  double RE = 2.0 * b[D + 1] - e2 * b[0];
  double aE = 4.0 * lam * lam / N * (RE - 2.0 * UR);
  double a0 = b[0] - 0.5 * aE * e2;
  for (int d = 0; d < D; ++d) {
    double aj = 2.0 * lam * Rj[d] - U[d] * aE;
    a[1 + d] = aj;
    a0 -= U[d] * aj;
  }
  a[0] = a0;
  a[D + 1] = aE;
}

// Gaussian moment tables for the time slope.
template <int D>
struct Moments {
  double m[3][6];   // E[u_d^n], n <= 5 (m[d][0] = 1; unused dims are delta at 0)
  double x1, x2;    // E[xi^2], E[xi^4]
  __device__ void init(const double* U, double lam, double kxi) {
    double var = 1.0 / (2.0 * lam);
    for (int d = 0; d < 3; ++d) {
      double mu = d < D ? U[d] : 0.0;
      m[d][0] = 1.0;
      m[d][1] = mu;
      for (int n = 1; n < 5; ++n) m[d][n + 1] = mu * m[d][n] + n * var * m[d][n - 1];
      if (d >= D)
        for (int n = 1; n < 6; ++n) m[d][n] = 0.0;
    }
    x1 = kxi * var;
    x2 = kxi * (kxi + 2.0) * var * var;
  }
  // E[u^e] for an exponent vector
  __device__ double E(int e0, int e1, int e2) const { return m[0][e0] * m[1][e1] * m[2][e2]; }
  // E[u^e psi_E] with psi_E = (|u|^2 + xi^2)/2
  __device__ double Epe(int e0, int e1, int e2) const {
    double s = x1 * E(e0, e1, e2);
    s += E(e0 + 2, e1, e2);
    if (D >= 2) s += E(e0, e1 + 2, e2);
    if (D >= 3) s += E(e0, e1, e2 + 2);
    return 0.5 * s;
  }
  // E[u^e psi_E^2]
  __device__ double Epe2(int e0, int e1, int e2) const {
    int e[3] = {e0, e1, e2};
    double s = x2 * E(e0, e1, e2);
    for (int g = 0; g < D; ++g) {
      int f[3] = {e[0], e[1], e[2]};
      f[g] += 2;
      s += 2.0 * x1 * E(f[0], f[1], f[2]);
      for (int hh = 0; hh < D; ++hh) {
        int k[3] = {f[0], f[1], f[2]};
        k[hh] += 2;
        s += E(k[0], k[1], k[2]);
      }
    }
    return 0.25 * s;
  }
};

// r_alpha = -sum_d E[u_d psi_alpha (a_d . psi)]  (compatibility condition for
// the time slope).
template <int D>
__device__ __forceinline__ void time_slope_rhs(const Moments<D>& M, const double (*a)[5], double* r) {
  for (int al = 0; al < D + 2; ++al) r[al] = 0.0;
  for (int d = 0; d < D; ++d) {
    int ed[3] = {0, 0, 0};
    ed[d] = 1;
    // alpha = 0: psi_0 = 1
    {
      double t = a[d][0] * M.E(ed[0], ed[1], ed[2]);
      for (int e = 0; e < D; ++e) {
        int k[3] = {ed[0], ed[1], ed[2]};
        k[e] += 1;
        t += a[d][1 + e] * M.E(k[0], k[1], k[2]);
      }
      t += a[d][D + 1] * M.Epe(ed[0], ed[1], ed[2]);
      r[0] -= t;
    }
    // alpha = f: psi_f = u_f
    for (int f = 0; f < D; ++f) {
      int ef[3] = {ed[0], ed[1], ed[2]};
      ef[f] += 1;
      double t = a[d][0] * M.E(ef[0], ef[1], ef[2]);
      for (int e = 0; e < D; ++e) {
        int k[3] = {ef[0], ef[1], ef[2]};
        k[e] += 1;
        t += a[d][1 + e] * M.E(k[0], k[1], k[2]);
      }
      t += a[d][D + 1] * M.Epe(ef[0], ef[1], ef[2]);
      r[1 + f] -= t;
    }
    // alpha = E: psi_E
    {
      double t = a[d][0] * M.Epe(ed[0], ed[1], ed[2]);
      for (int e = 0; e < D; ++e) {
        int k[3] = {ed[0], ed[1], ed[2]};
        k[e] += 1;
        t += a[d][1 + e] * M.Epe(k[0], k[1], k[2]);
      }
      t += a[d][D + 1] * M.Epe2(ed[0], ed[1], ed[2]);
      r[D + 1] -= t;
    }
  }
}

// Time integrals of c_1..c_5 over [0, dt]; closed forms for dt/tau >= 1/2,
// power series of the same functions below (they are exact rearrangements of
// exp(-x); the closed forms cancel catastrophically for small x).
__device__ __forceinline__ void time_coeffs(double dt, double tau, double* G) {
  double x = dt / tau;
  if (x >= 0.5) {
    double E = -expm1(-x);
    G[0] = tau * E;
    G[1] = tau * tau * (x * (1.0 - E) - E);
    G[2] = tau * (x - E);
    G[3] = tau * tau * (2.0 * E - x * (2.0 - E));
    G[4] = tau * tau * (0.5 * x * x - x + E);
    return;
  }
  // term t_n = (-x)^n / n!; accumulate each series by its own coefficient
  double t = 1.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0;
  for (int n = 1; n <= 40; ++n) {
    t *= -x / n;           // (-1)^n x^n / n!
    s1 -= t;               // (-1)^(n+1) x^n/n!
    s2 -= (n - 1) * t;     // (-1)^(n-1) (n-1) x^n/n!
    s3 += (n >= 2) ? t : 0.0;
    s4 -= (n >= 3) ? (2 - n) * t : 0.0;
    s5 -= (n >= 3) ? t : 0.0;
    if (fabs(t) < 1e-40) break;
  }
  G[0] = tau * s1;
  G[1] = tau * tau * s2;
  G[2] = tau * s3;
  G[3] = tau * tau * s4;
  G[4] = tau * tau * s5;
}


// ---------------------------------------------------------------------------
// Cubic polynomials in the molecular velocity.  Monomial order:
//   3-D: 1 | x y z | xx yy zz xy xz yz | xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
//   2-D: 1 | x y   | xx yy xy          | xxx xxy xyy yyy
// The even part is the constant and quadratic terms, the odd part the linear
// and cubic terms, so P(-u) = E(u) - O(u) when P(u) = E(u) + O(u).
// Every cubic term the scheme produces is of the form (w . u)|u|^2 (the
// energy slope's u.grad part and the Shakhov factor): add_lin_u2 is the only
// builder of cubic terms, so the coefficient of u_a^3 is the kappa_a of
// P = c + l.u + u^T Q u + (kappa . u)|u|^2, which is how the sweeps read it.
template <int D>
struct Cubic {
  static constexpr int NQ = D == 3 ? 6 : 3;
  static constexpr int NC = D == 3 ? 10 : 4;
  static constexpr int N = 1 + D + NQ + NC;
  static constexpr int Q0 = 1 + D;        // first quadratic
  static constexpr int C0 = 1 + D + NQ;   // first cubic
  __host__ __device__ static int qi(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    if (a == b) return Q0 + a;
    return Q0 + (D == 3 ? a + b + 2 : 2);
  }
  __host__ __device__ static int ci(int a, int b, int c) {
    // sort a <= b <= c
    if (a > b) { int t = a; a = b; b = t; }
    if (b > c) { int t = b; b = c; c = t; }
    if (a > b) { int t = a; a = b; b = t; }
    if (D == 2) return C0 + a + b + c;
    // lexicographic index of the sorted triple among the 10 3-D cubics
    int base = a == 0 ? 0 : (a == 1 ? 6 : 9);
    int rem;
    if (a == 0) rem = (b == 0) ? c : (b == 1 ? 2 + c : 5);
    else if (a == 1) rem = (b == 1) ? c - 1 : 2;
    else rem = 0;
    return C0 + base + rem;
  }
  // P += s
  __device__ static void add_const(double* P, double s) { P[0] += s; }
  // P += s (w . u)
  __device__ static void add_lin(double* P, double s, const double* w) {
    for (int a = 0; a < D; ++a) P[1 + a] += s * w[a];
  }
  // P += s |u|^2
  __device__ static void add_u2(double* P, double s) {
    for (int a = 0; a < D; ++a) P[qi(a, a)] += s;
  }
  // P += s (w1 . u)(w2 . u)
  __device__ static void add_linlin(double* P, double s, const double* w1, const double* w2) {
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) P[qi(a, b)] += s * w1[a] * w2[b];
  }
  // P += s sum_{a,b} M[a][b] u_a u_b, M given row-major with stride ld
  __device__ static void add_mat(double* P, double s, const double* M, int ld) {
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) P[qi(a, b)] += s * M[a * ld + b];
  }
  // P += s (w . u) |u|^2
  __device__ static void add_lin_u2(double* P, double s, const double* w) {
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) P[ci(a, b, b)] += s * w[a];
  }
  // Shakhov factor S(u) = (c.q)(2 lam |c|^2 - m), c = u - U, times s.
  __device__ static void add_shakhov(double* P, double s, const double* U, const double* q,
                                     double lam, double m) {
    double UU = 0.0, beta = 0.0;
    for (int a = 0; a < D; ++a) {
      UU += U[a] * U[a];
      beta += U[a] * q[a];
    }
    const double alpha = 2.0 * lam * UU - m;
    // (u.q - beta)(2 lam |u|^2 - 4 lam U.u + alpha)
    add_lin_u2(P, s * 2.0 * lam, q);
    add_linlin(P, -s * 4.0 * lam, q, U);
    add_lin(P, s * alpha, q);
    add_u2(P, -s * 2.0 * lam * beta);
    add_lin(P, s * 4.0 * lam * beta, U);
    add_const(P, -s * alpha * beta);
  }
};

}  // namespace dev
}  // namespace ugks
