// Fused velocity sweep for tensor-product, mirror-symmetric velocity sets.
//
// A work item is one cell and one block of its velocity space.  Each lane
// owns a mirror pair of velocities (u, -u): for every face of the cell
// exactly one of the two leaves the cell, so the lane evaluates one
// time-integrated flux from the cell's own reconstruction (outgoing) and one
// from the neighbour's reconstruction (incoming), with no divergence between
// lanes.  The face and cell data are wave-uniform:
//   * the Maxwellians g0, g_cell and the wall Maxwellian factor over the
//     velocity axes and are staged in LDS once per work item, so
//     exp(-lambda |u - U|^2) is a product of three table entries;
//   * every equilibrium term of the interface distribution (Eqs.
//     interface_distribution, c123, c45 integrated over the step) is g0(u)
//     times a cubic polynomial c + l.u + u^T Q u + (kappa . u)|u|^2, evaluated
//     with the even/odd split P(-u) = E(u) - O(u);
//   * those polynomials and the least-squares stencils of the cell and of
//     each neighbour are read from the face and cell records through the
//     scalar cache.
// The conservative update needs, per cell, sum_j sigma_j S_j F_j / V with
// F_j = sum_k w_k psi_k H_jk (Eqs. macro_update, macro_flux); the sweep
// regroups that sum by velocity, sum_k w_k psi_k (sum_j sigma_j S_j H_jk / V),
// accumulates it per lane and reduces it once per work item, so there are no
// atomics and the result is deterministic.  The first stage (Eq. f_tilde) is
// applied in the same pass.  All loads of an iteration (the cell's stencil at
// u and -u, each neighbour's stencil at the incoming member) are issued
// before any arithmetic so their latency overlaps.  In 2-D the b equation
// (same transport and relaxation, its own equilibrium polynomials) runs as a
// second pass over the block after h, except in the batched form, whose
// short work items carry h and b in one pass.  Stage 2 (Eq. f_final) and
// the heat flux of the new distribution are fused in a second kernel.
#include <type_traits>

#include "ugks_device.h"

namespace ugks {

using namespace dev;

namespace {

constexpr int SWF = 4;      // faces per cell on the fused path (triangles, quads, tets)
constexpr int SWT = 256;    // threads per work-group
constexpr int NAX = 64;     // nodes per velocity axis (max)

// A wave-uniform row of f in the global address space, kept opaque in
// scalar registers, so that every load from it is one scalar base plus a
// 32-bit per-lane byte offset (no reassociated 64-bit vector addresses).
typedef const __attribute__((address_space(1))) char grow_t;

template <typename T>
__device__ __forceinline__ grow_t* srow(const T* p) {
  grow_t* g = (grow_t*)p;
  __asm__("" : "+s"(g));
  return g;
}

// Per-cell and per-face records are read-only during the sweep; read
// through the constant address space their wave-uniform loads are always
// scalar loads, also where the record pointers themselves come from memory
// (the batched form).
typedef const __attribute__((address_space(4))) int32_t crec_i_t;
template <typename X>
using crec_t = const __attribute__((address_space(4))) X;

template <typename T, typename C>
__device__ __forceinline__ C ldo(grow_t* row, uint32_t off) {
  return static_cast<C>(*(const __attribute__((address_space(1))) T*)(row + off));
}

// Even and odd parts of a cubic P = c + l.u + u^T Q u + (kappa . u)|u|^2
// (monomial order of Cubic<D>; kappa_a is the coefficient of u_a^3, the only
// cubic form the scheme builds) at u, with v2 = |u|^2:
//   E = c + u^T Q u,  O = l.u + (kappa . u) v2,  P(u) = E + O,  P(-u) = E - O.
template <int D, typename C, typename PT>
__device__ __forceinline__ void cubic_eo(PT P, const C* v, C v2, C& E, C& O) {
  if constexpr (D == 3) {
    const C x = v[0], y = v[1], z = v[2];
    // quadratics xx yy zz xy xz yz = P[4..9]; u_a^3 at P[10], P[16], P[19]
    E = P[0] + x * (P[4] * x + P[7] * y + P[8] * z) + y * (P[5] * y + P[9] * z) + P[6] * z * z;
    O = (P[1] * x + P[2] * y + P[3] * z) + (P[10] * x + P[16] * y + P[19] * z) * v2;
  } else {
    const C x = v[0], y = v[1];
    // quadratics xx yy xy = P[3..5]; u_a^3 at P[6], P[9]
    E = P[0] + x * (P[3] * x + P[5] * y) + P[4] * y * y;
    O = (P[1] * x + P[2] * y) + (P[6] * x + P[9] * y) * v2;
  }
}

// Venkatakrishnan's limiter factor (Sec. 2.1 reconstruction with the
// optional limiter) of a gradient g of a field with cell value vi and stencil
// range [vmin, vmax]: at each of four faces with offsets off[q * stride + d]
// from the centroid, d- = g.off, d+ = vmax - vi (d- > 0) or vmin - vi,
// psi = (d+^2 + eps^2 + 2 d- d+) / (d+^2 + 2 d-^2 + d- d+ + eps^2) (psi = 1
// where d- = 0); returns min(1, min_faces psi).  The minimum is kept as a
// fraction and divided once.
template <int D, typename C, typename PT>
__device__ __forceinline__ C venkat_phi(C vi, C vmin, C vmax, const C* g, PT off, int stride, C eps2) {
  C Nm = C(1), Dm = C(1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    C dm = C(0);
#pragma unroll
    for (int d = 0; d < D; ++d) dm += g[d] * off[q * stride + d];
    const C dp = dm > C(0) ? vmax - vi : vmin - vi;
    C N = dp * dp + eps2 + C(2) * dm * dp;
    C Dn = dp * dp + C(2) * dm * dm + dm * dp + eps2;
    if (dm == C(0)) N = Dn = C(1);
    const bool lt = N * Dm < Nm * Dn;
    Nm = lt ? N : Nm;
    Dm = lt ? Dn : Dm;
  }
  return Nm / Dm;
}

// Per-cell first-stage data of one step: dt/(2 tau), K_xi/(2 lambda) and the
// Shakhov polynomials H+/H, B+/B of the cell's equilibrium (Eqs. H_plus, B_plus).
template <int D>
__device__ __forceinline__ void cell_prep_at(int64_t i, const GasP& g, const double* __restrict__ W,
                                             const double* __restrict__ q,
                                             double* __restrict__ prim, double* __restrict__ cs,
                                             int32_t* flag) {
  if (*flag) return;
  double* P = &prim[i * NPRIM];
  if (!prim_of<D>(&W[i * (D + 2)], g, P)) {
    atomicOr(flag, 1);
    return;
  }
  using Cb = Cubic<D>;
  double SH[Cb::N], SB[Cb::N];
  for (int x = 0; x < Cb::N; ++x) SH[x] = SB[x] = 0.0;
  const double lam = P[4], rho = P[0];
  const double sh = 4.0 * (1.0 - g.Pr) * lam * lam / ((g.K + 5.0) * rho);
  const double U[3] = {P[1], P[2], P[3]};
  const double qc[3] = {q[i * 3], q[i * 3 + 1], q[i * 3 + 2]};
  Cb::add_shakhov(SH, sh, U, qc, lam, 2.0 + D);
  Cb::add_shakhov(SB, sh, U, qc, lam, (double)D);
  double* C = &cs[i * CSREC];
  C[CS_CC] = dt_cell(g, i) / (2.0 * P[5]);
  C[CS_KAP] = (g.K + 3.0 - D) / (2.0 * lam);
  C[CS_NORM] = rho * maxw_norm<D>(lam);
  for (int x = 0; x < 20; ++x) {
    C[CS_SH + x] = x < Cb::N ? SH[x] : 0.0;
    C[CS_SB + x] = x < Cb::N ? SB[x] : 0.0;
  }
}

template <int D>
__global__ void k_cell_prep(int64_t nc, GasP g, const double* __restrict__ W,
                            const double* __restrict__ q, double* __restrict__ prim,
                            double* __restrict__ cs, int32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nc) cell_prep_at<D>(i, g, W, q, prim, cs, flag);
}

// Axis tables of every face Maxwellian and every cell Maxwellian of the
// step, tab[e][d][n] = scale_d exp(-lambda (a_n - U_d)^2) with the density
// and normalisation folded into d = 0, so that g(u) at a tensor point is a
// product of D entries.  Entities 0..nf-1 are faces (interface g0, or on a
// wall the re-emitted Maxwellian scaled by rho_w dt), nf..nf+nc-1 cells.
template <int D>
__device__ __forceinline__ void tables_at(int64_t t, int64_t nf, int na,
                                          const double* __restrict__ axis,
                                          const int32_t* __restrict__ fbc, const GasP& g,
                                          const double* __restrict__ frec,
                                          const double* __restrict__ prim,
                                          const double* __restrict__ cs, double* __restrict__ tabs,
                                          const int32_t* __restrict__ flag) {
  const int64_t per = (int64_t)D * na;
  if (*flag) return;
  const int64_t e = t / per;
  const int r = (int)(t % per), d = r / na, n = r % na;
  const double a = axis[n];
  double lam, U, scale = 1.0;
  if (e < nf) {
    const double* R = &frec[e * FREC];
    lam = R[FR_LAM];
    U = R[FR_U + d];
    if (d == 0)  // rho0 (lambda0/pi)^(D/2), or rho_w dt (lambda_w/pi)^(D/2) on a wall
      scale = fbc[e] == UGKS_BC_WALL ? R[FR_C0] * R[FR_RHOW] * g.dt : R[FR_C0];
  } else {
    const int64_t i = e - nf;
    lam = prim[i * NPRIM + 4];
    U = prim[i * NPRIM + 1 + d];
    if (d == 0) scale = cs[i * CSREC + CS_NORM];
  }
  tabs[e * per + d * na + n] = scale * exp(-lam * (a - U) * (a - U));
}

template <int D>
__global__ void k_tables(int64_t nf, int64_t nc, int na, const double* __restrict__ axis,
                         const int32_t* __restrict__ fbc, GasP g, const double* __restrict__ frec,
                         const double* __restrict__ prim, const double* __restrict__ cs,
                         double* __restrict__ tabs, const int32_t* __restrict__ flag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < (nf + nc) * (int64_t)D * na) tables_at<D>(t, nf, na, axis, fbc, g, frec, prim, cs, tabs, flag);
}

// LDS of one sweep work item: the Maxwellian axis tables of the cell's four
// faces and of the cell, the velocity nodes and the reduction scratch.
template <typename C>
struct SweepLds {
  C tab[SWF][3][NAX];
  C ctab[3][NAX];
  C ax[NAX];
  double red[5 * 16];
};

// One work item of the fused sweep: cell ic, velocity block `chunk`.
// Every read-only array is its own __restrict__ argument so that the
// compiler can prove no store of the sweep clobbers it and serve the
// wave-uniform reads from the scalar cache.
template <int D, typename T, typename C, bool SPLIT, bool LIM = false, bool SPARSE = false,
          bool NB = false>
__device__ __forceinline__ void sweep_item(
    const FusedMesh& fm, int64_t nvp, const SweepSched& sc, const int32_t* __restrict__ crec_i,
    const C* __restrict__ crec_d, const C* __restrict__ crec_l, const int32_t* __restrict__ vidx,
    const double* __restrict__ w, const C* __restrict__ cs, const C* __restrict__ frec,
    const C* __restrict__ tabs, const T* __restrict__ h, const T* __restrict__ b,
    T* __restrict__ ht, T* __restrict__ bt, double* __restrict__ dWp,
    const int32_t* __restrict__ flag, int64_t ic, int64_t chunk, SweepLds<C>& L) {
  if (*flag) return;
  // every pointer below is wave-uniform: its loads are scalar loads
  crec_i_t* ci0 = (crec_i_t*)(crec_i + ic * CRI);
  crec_t<C>* cd0 = (crec_t<C>*)(crec_d + ic * CRD);
  crec_t<C>* cc0 = (crec_t<C>*)(cs + ic * CSREC);
  crec_t<C>* frc = (crec_t<C>*)frec;
  crec_t<C>* cl0 = LIM ? (crec_t<C>*)(crec_l + ic * CRL) : nullptr;
  const unsigned nthr = blockDim.x;  // lanes of the work-group, one mirror pair each
  const int na = fm.na;
  {
    // Stage this cell's face and cell tables in LDS (faces 0..3, then the
    // cell).  The five table entities are scalar loads; each wave copies
    // whole (entity, axis) rows, one node per lane (na <= 64, and the
    // work-group is 1, 2 or 4 waves), and with the row loop unrolled all of
    // a wave's loads are in flight together.
    const int64_t ent[5] = {(int64_t)ci0[CRI_F0], (int64_t)ci0[CRI_F0 + CRI_FS],
                            (int64_t)ci0[CRI_F0 + 2 * CRI_FS], (int64_t)ci0[CRI_F0 + 3 * CRI_FS],
                            sc.nf + ic};
    const unsigned lane = threadIdx.x & 63u;
    const unsigned wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned wmask = (nthr >> 6) - 1;
    if (lane < (unsigned)na) {
      C v[5 * D];
#pragma unroll
      for (int row = 0; row < 5 * D; ++row)
        if (((unsigned)row & wmask) == wv) v[row] = tabs[(ent[row / D] * D + row % D) * na + lane];
#pragma unroll
      for (int row = 0; row < 5 * D; ++row)
        if (((unsigned)row & wmask) == wv) {
          if (row / D < 4) L.tab[row / D][row % D][lane] = v[row];
          else L.ctab[row % D][lane] = v[row];
        }
      if (wv == 0) L.ax[lane] = fm.axis[lane];
    }
    __syncthreads();
  }
  constexpr int NM = D + 2;
  const unsigned nv = (unsigned)fm.nv;
  const unsigned npairs = (unsigned)fm.npairs;
  const unsigned kbeg = (unsigned)(chunk * sc.chunk_pairs);
  const unsigned kend = (unsigned)min((int64_t)npairs, (chunk + 1) * sc.chunk_pairs);
  // Row r of h (or b) starts r * rowb bytes in.  Row indices are 32-bit and
  // non-negative, and a row is under 4 GiB, so the offset is one 32x32->64
  // scalar multiply.
  const uint32_t rowb = (uint32_t)nvp * (uint32_t)sizeof(T);
  auto row_of = [rowb](const T* base, int32_t r) {
    return srow((const char*)base + (uint64_t)(uint32_t)r * rowb);
  };
  // per-lane moments sum_k w_k psi_k (net outflow of the cell at u_k): the
  // conservative update of the cell is W - sum (Eq. macro_update regrouped
  // by velocity: sum_j sigma S_j F_j / V = sum_k w_k psi_k sum_j sigma S_j H_jk / V)
  double mw[NM];
#pragma unroll
  for (int x = 0; x < NM; ++x) mw[x] = 0.0;

  // In 2-D, h and b run as two passes over the block (each pass's records
  // and row addresses then fit the scalar registers, where h and b together
  // spill them), except for the batched form: the items of its small cases
  // run only a few iterations, whose dependent-load latency two passes would
  // pay twice, so there one pass carries both.
  if constexpr (D == 2 && !SPLIT) {
    // (64-bit row arithmetic here: the 32-bit form costs this body scalar
    // registers it does not have)
    constexpr bool B2 = true;
    const T* __restrict__ hi = h + ic * nvp;
    const T* __restrict__ bi = b + ic * nvp;
    // the packed axis indices of the next pair are loaded one iteration ahead
    int pk_next = kbeg + threadIdx.x < kend ? vidx[kbeg + threadIdx.x] : 0;
    for (unsigned kp = kbeg + threadIdx.x; kp < kend; kp += nthr) {
      // The cell and face records are loop invariant but too large to keep in
      // scalar registers for the whole loop: an opaque uniform zero added to
      // their addresses makes them scalar re-loads (scalar cache) each
      // iteration instead of hoisted, spilled registers.
      int z;
      __asm__ volatile("s_mov_b32 %0, 0" : "=s"(z));
      crec_i_t* ci = ci0 + z;
      crec_t<C>* cd = cd0 + z;
      crec_t<C>* cc = cc0 + z;
      const unsigned k0 = kp, k1 = nv - 1 - kp;
      const int pk = pk_next;
      pk_next = vidx[min(kp + nthr, kend - 1)];
      int id[3], im[3];
  #pragma unroll
      for (int d = 0; d < 3; ++d) {
        id[d] = (pk >> (8 * d)) & 255;
        im[d] = na - 1 - id[d];
      }
      C vv[3] = {C(0), C(0), C(0)};
  #pragma unroll
      for (int d = 0; d < D; ++d) vv[d] = L.ax[id[d]];
      // orientation of u against every outward normal
      C sp[4];
  #pragma unroll
      for (int p = 0; p < 4; ++p) {
        C s = C(0);
  #pragma unroll
        for (int d = 0; d < D; ++d) s += vv[d] * cd[CRD_F0 + CRD_FS * p + 0 + d];
        sp[p] = s;
      }
      // ---- the cell's own stencil at u and -u (4 rows, padded) ----
      const uint32_t o0 = k0 * (uint32_t)sizeof(T), o1 = k1 * (uint32_t)sizeof(T);
      grow_t* rhi = srow(hi);
      const C h0 = ldo<T, C>(rhi, o0), h1 = ldo<T, C>(rhi, o1);
      C b0 = C(0), b1 = C(0);
      if (B2) {
        grow_t* rbi = srow(bi);
        b0 = ldo<T, C>(rbi, o0);
        b1 = ldo<T, C>(rbi, o1);
      }
      C os0[4], os1[4], ob0[4], ob1[4];
  #pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t cell = ci[2 + s];
        grow_t* rh = srow(h + cell * nvp);
        os0[s] = ldo<T, C>(rh, o0);
        os1[s] = ldo<T, C>(rh, o1);
        ob0[s] = ob1[s] = C(0);
        if (B2) {
          grow_t* rb = srow(b + cell * nvp);
          ob0[s] = ldo<T, C>(rb, o0);
          ob1[s] = ldo<T, C>(rb, o1);
        }
      }
      // ---- every neighbour's value and stencil at the incoming member ----
      // Slot p of the own stencil is the row across face p, and slot 0 of
      // neighbour p's stencil is this cell: both are already in registers.
      C nh[4], nhs[4][4], nb[4], nbs[4][4];
  #pragma unroll
      for (int p = 0; p < 4; ++p) {
        crec_i_t* fi = ci + CRI_F0 + CRI_FS * p;
        const bool in1 = sp[p] > C(0);  // the incoming member is -u
        uint32_t oin = in1 ? o1 : o0;
        __asm__("" : "+v"(oin));  // keep the select on the offset, not on 64-bit addresses
        nh[p] = in1 ? os1[p] : os0[p];
        nb[p] = B2 ? (in1 ? ob1[p] : ob0[p]) : C(0);
        nhs[p][0] = in1 ? h1 : h0;
        nbs[p][0] = B2 ? (in1 ? b1 : b0) : C(0);
  #pragma unroll
        for (int r = 1; r < 4; ++r) {
          const int64_t cell = fi[5 + r];
          nhs[p][r] = ldo<T, C>(srow(h + cell * nvp), oin);
          nbs[p][r] = B2 ? ldo<T, C>(srow(b + cell * nvp), oin) : C(0);
        }
      }
      // ---- arithmetic ----
      C g0[3] = {C(0), C(0), C(0)}, g1[3] = {C(0), C(0), C(0)}, gb0[3] = {C(0), C(0), C(0)}, gb1[3] = {C(0), C(0), C(0)};
  #pragma unroll
      for (int s = 0; s < 4; ++s) {
        const C d0 = os0[s] - h0, d1 = os1[s] - h1;
        const C e0 = ob0[s] - b0, e1 = ob1[s] - b1;
  #pragma unroll
        for (int d = 0; d < D; ++d) {
          const C G = cd[d * 4 + s];
          g0[d] += G * d0;
          g1[d] += G * d1;
          if (B2) {
            gb0[d] += G * e0;
            gb1[d] += G * e1;
          }
        }
      }
      C ug0 = C(0), ug1 = C(0), ub0 = C(0), ub1 = C(0);
  #pragma unroll
      for (int d = 0; d < D; ++d) {
        ug0 += vv[d] * g0[d];
        ug1 -= vv[d] * g1[d];
        if (B2) {
          ub0 += vv[d] * gb0[d];
          ub1 -= vv[d] * gb1[d];
        }
      }
      C v2 = C(0);
  #pragma unroll
      for (int d = 0; d < D; ++d) v2 += vv[d] * vv[d];
      C acc0 = C(0), acc1 = C(0), accb0 = C(0), accb1 = C(0);
  #pragma unroll
      for (int p = 0; p < 4; ++p) {
        crec_t<C>* fd = cd + CRD_F0 + CRD_FS * p;
        crec_t<C>* R = frc + (int64_t)ci[CRI_F0 + CRI_FS * p] * FREC;
        const bool pos = sp[p] > C(0);
        const C as = fabs(sp[p]);
        const C G1 = R[FR_G], G2 = R[FR_G + 1];
        // outgoing member: the cell's own reconstruction at the face
        const C us = pos ? ug0 : ug1;
        C hf = pos ? h0 : h1;
  #pragma unroll
        for (int d = 0; d < D; ++d) hf += fd[4 + d] * (pos ? g0[d] : g1[d]);
        // incoming member: the neighbour's reconstruction at the face (all
        // zero rows on a wall)
        const C sgn_in = pos ? -1.0 : 1.0;  // u_in = sgn_in * u
        const C hj = nh[p], bj = nb[p];
        C gj[3] = {C(0), C(0), C(0)}, gbj[3] = {C(0), C(0), C(0)};
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const C dh = nhs[p][r] - hj, db = nbs[p][r] - bj;
  #pragma unroll
          for (int d = 0; d < D; ++d) {
            const C G = fd[10 + d * 4 + r];
            gj[d] += G * dh;
            if (B2) gbj[d] += G * db;
          }
        }
        C hfj = hj, ugj = C(0);
  #pragma unroll
        for (int d = 0; d < D; ++d) {
          hfj += fd[7 + d] * gj[d];
          ugj += vv[d] * gj[d];
        }
        ugj *= sgn_in;
        // g0 (or the scaled wall Maxwellian) at u and -u from the axis tables,
        // times the equilibrium polynomial (constant on a wall)
        C e0 = L.tab[p][0][id[0]], e1 = L.tab[p][0][im[0]];
  #pragma unroll
        for (int d = 1; d < D; ++d) {
          e0 *= L.tab[p][d][id[d]];
          e1 *= L.tab[p][d][im[d]];
        }
        C E, O;
        cubic_eo<D>(R + FR_PH, vv, v2, E, O);
        const C q0 = e0 * (E + O), q1 = e1 * (E - O);
        const C eqm = fd[22];  // 0 on a wall: no equilibrium term going out
        const C eqo = eqm * (pos ? q0 : q1);
        const C eqi = pos ? q1 : q0;
        const C out = as * (G1 * hf + G2 * us + eqo);
        const C in = -as * (G1 * hfj + G2 * ugj + eqi);
        C outb = 0.0, inb = 0.0;
        if (B2) {
          C bfo = pos ? b0 : b1;
          const C ubs = pos ? ub0 : ub1;
  #pragma unroll
          for (int d = 0; d < D; ++d) bfo += fd[4 + d] * (pos ? gb0[d] : gb1[d]);
          C bfj = bj, ubj = C(0);
  #pragma unroll
          for (int d = 0; d < D; ++d) {
            bfj += fd[7 + d] * gbj[d];
            ubj += vv[d] * gbj[d];
          }
          ubj *= sgn_in;
          C Eb, Ob;
          cubic_eo<D>(R + FR_PB, vv, v2, Eb, Ob);
          const C r0 = e0 * (Eb + Ob), r1 = e1 * (Eb - Ob);
          outb = as * (G1 * bfo + G2 * ubs + eqm * (pos ? r0 : r1));
          inb = -as * (G1 * bfj + G2 * ubj + (pos ? r1 : r0));
        }
        // fluxes at u and at -u along this cell's outward normal, times S/V
        const C sv = fd[3];
        acc0 += sv * (pos ? out : in);
        acc1 += sv * (pos ? in : out);
        if (B2) {
          accb0 += sv * (pos ? outb : inb);
          accb1 += sv * (pos ? inb : outb);
        }
      }
      // moments of the net outflow (the zero velocity of an odd grid once)
      {
        const double a0 = w[k0] * (double)acc0, a1 = (k1 != k0) ? w[k1] * (double)acc1 : 0.0;
        mw[0] += a0 + a1;
  #pragma unroll
        for (int d = 0; d < D; ++d) mw[1 + d] += (double)vv[d] * (a0 - a1);
        double e = 0.5 * (double)v2 * (a0 + a1);
        if (B2) e += 0.5 * (w[k0] * (double)accb0 + ((k1 != k0) ? w[k1] * (double)accb1 : 0.0));
        mw[D + 1] += e;
      }
      // first stage with the cell's BGK-Shakhov equilibrium at u and -u
      C c0 = L.ctab[0][id[0]], c1 = L.ctab[0][im[0]];
  #pragma unroll
      for (int d = 1; d < D; ++d) {
        c0 *= L.ctab[d][id[d]];
        c1 *= L.ctab[d][im[d]];
      }
      C E, O;
      cubic_eo<D>(cc + CS_SH, vv, v2, E, O);
      const C ccoll = cc[CS_CC];
      T* __restrict__ hto = ht + ic * nvp;
      st(hto, k0, h0 - acc0 + ccoll * (c0 * (C(1) + E + O) - h0));
      if (k1 != k0) st(hto, k1, h1 - acc1 + ccoll * (c1 * (C(1) + E - O) - h1));
      if (B2) {
        C Eb, Ob;
        cubic_eo<D>(cc + CS_SB, vv, v2, Eb, Ob);
        const C kc = cc[CS_KAP];
        T* __restrict__ bto = bt + ic * nvp;
        st(bto, k0, b0 - accb0 + ccoll * (kc * c0 * (C(1) + Eb + Ob) - b0));
        if (k1 != k0) st(bto, k1, b1 - accb1 + ccoll * (kc * c1 * (C(1) + Eb - Ob) - b1));
      }
    }
  } else {
    // One pass over the block's mirror pairs for one reduced distribution:
    // X = 0 is h (mass, momentum and its share of the energy), X = 1 is b
    // (2-D only: the rest of the energy).  The b equation has the same
    // transport and relaxation as h with its own equilibrium polynomials.
    auto pass = [&](auto xtag) {
      constexpr int X = decltype(xtag)::value;
      const T* __restrict__ f = X ? b : h;
      T* __restrict__ fto = (X ? bt : ht) + ic * nvp;
      grow_t* rfi = srow(f + ic * nvp);
      // the packed axis indices of the next pair are loaded one iteration ahead
      int pk_next = kbeg + threadIdx.x < kend ? vidx[kbeg + threadIdx.x] : 0;
      for (unsigned kp = kbeg + threadIdx.x; kp < kend; kp += nthr) {
        // FP32: the wave takes a higher issue priority while it issues the
        // iteration's gathers, so that they start early (measured 2-6 %
        // faster in FP32, slower in FP64)
        if constexpr (sizeof(C) == 4) __builtin_amdgcn_s_setprio(1);
        // The cell and face records are loop invariant but too large to keep
        // in scalar registers for the whole loop: an opaque uniform zero
        // added to their addresses makes them scalar re-loads (scalar cache)
        // each iteration instead of hoisted, spilled registers.
        int z;
        __asm__ volatile("s_mov_b32 %0, 0" : "=s"(z));
        crec_i_t* ci = ci0 + z;
        crec_t<C>* cd = cd0 + z;
        crec_t<C>* cc = cc0 + z;
        // a pair's two points: k and its mirror; a sparse set lists them
        // (a point without a mirror in the set has the pad slot nv as a
        // partner: weight 0, never stored)
        unsigned k0 = kp, k1 = nv - 1 - kp;
        if constexpr (SPARSE) {
          k0 = (unsigned)fm.pairs[2 * kp];
          k1 = (unsigned)fm.pairs[2 * kp + 1];
        }
        const bool has1 = k1 != k0 && (!SPARSE || k1 < nv);
        const int pk = pk_next;
        pk_next = vidx[min(kp + nthr, kend - 1)];
        int id[3], im[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          id[d] = (pk >> (8 * d)) & 255;
          im[d] = na - 1 - id[d];
        }
        C vv[3] = {C(0), C(0), C(0)};
#pragma unroll
        for (int d = 0; d < D; ++d) vv[d] = L.ax[id[d]];
        // orientation of u against every outward normal
        C sp[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          C s = C(0);
#pragma unroll
          for (int d = 0; d < D; ++d) s += vv[d] * cd[CRD_F0 + CRD_FS * p + 0 + d];
          sp[p] = s;
        }
        // ---- the cell's own stencil at u and -u (4 rows, padded) ----
        const uint32_t o0 = k0 * (uint32_t)sizeof(T), o1 = k1 * (uint32_t)sizeof(T);
        const C f0 = ldo<T, C>(rfi, o0), f1 = ldo<T, C>(rfi, o1);
        C os0[4], os1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          grow_t* rs = row_of(f, ci[2 + s]);
          os0[s] = ldo<T, C>(rs, o0);
          os1[s] = ldo<T, C>(rs, o1);
        }
        // ---- every neighbour's value and stencil at the incoming member ----
        // Slot p of the own stencil is the row across face p, and slot 0 of
        // neighbour p's stencil is this cell: both are already in registers.
        C nh[4], nhs[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          crec_i_t* fi = ci + CRI_F0 + CRI_FS * p;
          const bool in1 = sp[p] > C(0);  // the incoming member is -u
          uint32_t oin = in1 ? o1 : o0;
          __asm__("" : "+v"(oin));  // keep the select on the offset, not on 64-bit addresses
          nh[p] = in1 ? os1[p] : os0[p];
          nhs[p][0] = in1 ? f1 : f0;
#pragma unroll
          for (int r = 1; r < 4; ++r) nhs[p][r] = ldo<T, C>(row_of(f, fi[5 + r]), oin);
        }
        if constexpr (sizeof(C) == 4) __builtin_amdgcn_s_setprio(0);
        // ---- arithmetic ----
        C g0[3] = {C(0), C(0), C(0)}, g1[3] = {C(0), C(0), C(0)};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const C d0 = os0[s] - f0, d1 = os1[s] - f1;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const C G = cd[d * 4 + s];
            g0[d] += G * d0;
            g1[d] += G * d1;
          }
        }
        crec_t<C>* cl = LIM ? cl0 + z : nullptr;
        if constexpr (LIM) {
          // the cell's own gradients at u and -u, limited (a wall slot's
          // zero row stands for the cell's own value in the bounds)
          C lo0 = f0, hi0 = f0, lo1 = f1, hi1 = f1;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const C wm = cl[1 + s];
            const C v0 = wm * f0 + os0[s], v1 = wm * f1 + os1[s];
            lo0 = fmin(lo0, v0);
            hi0 = fmax(hi0, v0);
            lo1 = fmin(lo1, v1);
            hi1 = fmax(hi1, v1);
          }
          const C e2 = cl[0];
          const C p0 = venkat_phi<D>(f0, lo0, hi0, g0, cd + CRD_F0 + 4, CRD_FS, e2);
          const C p1 = venkat_phi<D>(f1, lo1, hi1, g1, cd + CRD_F0 + 4, CRD_FS, e2);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            g0[d] *= p0;
            g1[d] *= p1;
          }
        }
        C ug0 = C(0), ug1 = C(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          ug0 += vv[d] * g0[d];
          ug1 -= vv[d] * g1[d];
        }
        C v2 = C(0);
#pragma unroll
        for (int d = 0; d < D; ++d) v2 += vv[d] * vv[d];
        C acc0 = C(0), acc1 = C(0);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          crec_t<C>* fd = cd + CRD_F0 + CRD_FS * p;
          crec_t<C>* R = frc + (uint64_t)(uint32_t)ci[CRI_F0 + CRI_FS * p] * FREC;
          const bool pos = sp[p] > C(0);
          const C as = fabs(sp[p]);
          const C G1 = R[FR_G], G2 = R[FR_G + 1];
          // outgoing member: the cell's own reconstruction at the face
          const C us = pos ? ug0 : ug1;
          C ff = pos ? f0 : f1;
#pragma unroll
          for (int d = 0; d < D; ++d) ff += fd[4 + d] * (pos ? g0[d] : g1[d]);
          // incoming member: the neighbour's reconstruction at the face (all
          // zero rows on a wall)
          const C sgn_in = pos ? -1.0 : 1.0;  // u_in = sgn_in * u
          const C fj = nh[p];
          C gj[3] = {C(0), C(0), C(0)};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const C df = nhs[p][r] - fj;
#pragma unroll
            for (int d = 0; d < D; ++d) gj[d] += fd[10 + d * 4 + r] * df;
          }
          if constexpr (LIM) {
            // the neighbour's gradient at the incoming member, limited with
            // its own stencil bounds and face offsets
            crec_t<C>* Fr = cl + CRL_F0 + CRL_FS * p;
            C lo = fj, hi = fj;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const C vr = Fr[1 + r] * fj + nhs[p][r];
              lo = fmin(lo, vr);
              hi = fmax(hi, vr);
            }
            const C pj = venkat_phi<D>(fj, lo, hi, gj, Fr + 5, 3, Fr[0]);
#pragma unroll
            for (int d = 0; d < D; ++d) gj[d] *= pj;
          }
          C ffj = fj, ugj = C(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            ffj += fd[7 + d] * gj[d];
            ugj += vv[d] * gj[d];
          }
          ugj *= sgn_in;
          // g0 (or the scaled wall Maxwellian) at u and -u from the axis
          // tables, times the equilibrium polynomial (constant on a wall)
          C e0 = L.tab[p][0][id[0]], e1 = L.tab[p][0][im[0]];
#pragma unroll
          for (int d = 1; d < D; ++d) {
            e0 *= L.tab[p][d][id[d]];
            e1 *= L.tab[p][d][im[d]];
          }
          C E, O;
          cubic_eo<D>(R + (X ? FR_PB : FR_PH), vv, v2, E, O);
          const C q0 = e0 * (E + O), q1 = e1 * (E - O);
          const C eqm = fd[22];  // 0 on a wall: no equilibrium term going out
          const C eqo = eqm * (pos ? q0 : q1);
          const C eqi = pos ? q1 : q0;
          const C out = as * (G1 * ff + G2 * us + eqo);
          const C in = -as * (G1 * ffj + G2 * ugj + eqi);
          // fluxes at u and at -u along this cell's outward normal, times S/V
          const C sv = fd[3];
          acc0 += sv * (pos ? out : in);
          acc1 += sv * (pos ? in : out);
        }
        // moments of the net outflow (the zero velocity of an odd grid once)
        {
          const double a0 = w[k0] * (double)acc0, a1 = has1 ? w[k1] * (double)acc1 : 0.0;
          if constexpr (X == 0) {
            mw[0] += a0 + a1;
#pragma unroll
            for (int d = 0; d < D; ++d) mw[1 + d] += (double)vv[d] * (a0 - a1);
            mw[D + 1] += 0.5 * (double)v2 * (a0 + a1);
          } else {
            mw[D + 1] += 0.5 * (a0 + a1);
          }
        }
        // first stage with the cell's BGK-Shakhov equilibrium at u and -u
        C c0 = L.ctab[0][id[0]], c1 = L.ctab[0][im[0]];
#pragma unroll
        for (int d = 1; d < D; ++d) {
          c0 *= L.ctab[d][id[d]];
          c1 *= L.ctab[d][im[d]];
        }
        if constexpr (X == 1) {  // the b equilibrium carries the internal-energy factor
          const C kc = cc[CS_KAP];
          c0 = kc * c0;
          c1 = kc * c1;
        }
        C E, O;
        cubic_eo<D>(cc + (X ? CS_SB : CS_SH), vv, v2, E, O);
        const C ccoll = cc[CS_CC];
        st(fto, k0, f0 - acc0 + ccoll * (c0 * (C(1) + E + O) - f0));
        if (has1) st(fto, k1, f1 - acc1 + ccoll * (c1 * (C(1) + E - O) - f1));
      }
    };
    pass(std::integral_constant<int, 0>{});
    // b: always in 2-D; in 3-D for a gas with internal degrees of freedom
    if constexpr (D == 2 || NB) pass(std::integral_constant<int, 1>{});
  }
  block_sum<NM>(mw, L.red);
  if (threadIdx.x == 0)
    for (int x = 0; x < 5; ++x) dWp[(ic * sc.nchunk + chunk) * 5 + x] = x < NM ? mw[x] : 0.0;
}


// Single case: the sweep computes in the storage type T (FP32 storage uses
// FP32 copies of the records and tables; moment sums stay FP64).  The FP32
// body fits in half the registers; its bound asks for the occupancy that
// hides the gathers' latency (measured: 7 waves per SIMD, no spills).  NB:
// a 3-D gas with internal degrees of freedom, whose b runs a second pass.
template <int D, typename T, bool LIM, bool SPARSE, bool NB>
__global__ __launch_bounds__(SWT, (sizeof(T) == 4 ? 6 : 4)) void k_sweep(
    FusedMesh fm, int64_t nvp, SweepSched sc, const int32_t* __restrict__ crec_i,
    const T* __restrict__ crec_d, const T* __restrict__ crec_l, const int32_t* __restrict__ vidx,
    const double* __restrict__ w, const T* __restrict__ cs, const T* __restrict__ frec,
    const T* __restrict__ tabs, const T* __restrict__ h, const T* __restrict__ b,
    T* __restrict__ ht, T* __restrict__ bt, double* __restrict__ dWp,
    const int32_t* __restrict__ flag) {
  __shared__ SweepLds<T> L;
  // Work item = (cell, velocity block).  Blocks are dealt round-robin to the
  // 8 XCDs; XCD x takes tiles x, x+8, ... of sc.tile consecutive (Z-order)
  // cells and runs all of a tile's cells through velocity block 0, then 1,
  // ..., so the stencil rows of one tile and one velocity block are what
  // its L2 must hold.
  const int64_t xcd = blockIdx.x % 8, local = blockIdx.x / 8;
  const int64_t per_tile = sc.nchunk * sc.tile;
  const int64_t tile = (local / per_tile) * 8 + xcd;
  const int64_t rem = local % per_tile;
  const int64_t chunk = rem / sc.tile;
  const int64_t ic = tile * sc.tile + rem % sc.tile;
  if (ic >= fm.nc) return;
  sweep_item<D, T, T, true, LIM, SPARSE, NB>(fm, nvp, sc, crec_i, crec_d, crec_l, vidx, w, cs, frec,
                                             tabs, h, b, ht, bt, dWp, flag, ic, chunk, L);
}

// The fused sweep over a batch of cases: a persistent grid walks a list of
// (case, cell, velocity block) work items; item w runs on block w mod the
// grid size, and the host orders the list so that the blocks of one XCD
// (block index mod 8) take whole tiles of one case.  In 2-D, where one pass
// carries h and b, the bound trades a few spilled scalar registers for a
// third wave per SIMD.
template <int D, typename T>
__global__ __launch_bounds__(SWT, (D == 3 ? 4 : 3)) void k_sweep_b(BatchDev bd) {
  // computes in the storage type, as the single case does: an FP32 batch
  // reads the FP32 copies of its records and tables
  __shared__ SweepLds<T> L;
  // The work list and the case table are read-only for the whole launch:
  // read through the constant address space they are scalar loads, so the
  // case's pointers and sizes land in scalar registers as kernel arguments do.
  typedef const __attribute__((address_space(4))) int32_t citem_t;
  typedef const __attribute__((address_space(4))) CaseDev ccase_t;
  citem_t* items = (citem_t*)bd.items;
  ccase_t* cases = (ccase_t*)bd.cases;
  for (int64_t it = blockIdx.x; it < bd.nitems; it += gridDim.x) {
    const int c = items[4 * it];
    if (c < 0) continue;  // padding
    const int64_t ic = items[4 * it + 1], chunk = items[4 * it + 2];
    FusedMesh fm;
    fm.nc = cases[c].fm.nc;
    fm.nv = cases[c].fm.nv;
    fm.na = cases[c].fm.na;
    fm.axis = cases[c].fm.axis;
    fm.vidx = cases[c].fm.vidx;
    fm.npairs = cases[c].fm.npairs;
    fm.crec_i = cases[c].fm.crec_i;
    fm.crec_d = cases[c].fm.crec_d;
    SweepSched sc;
    sc.nf = cases[c].sc.nf;
    sc.tile = cases[c].sc.tile;
    sc.nchunk = cases[c].sc.nchunk;
    sc.chunk_pairs = cases[c].sc.chunk_pairs;
    const int64_t nvp = cases[c].v.nvp;
    const double* w = cases[c].v.w;
    const T *crec_d, *cs, *frec, *tabs;
    if constexpr (sizeof(T) == 4) {
      crec_d = cases[c].fm.crec_d32;
      cs = cases[c].B.cs32;
      frec = cases[c].B.frec32;
      tabs = cases[c].B.tabs32;
    } else {
      crec_d = cases[c].fm.crec_d;
      cs = cases[c].B.cs;
      frec = cases[c].B.frec;
      tabs = cases[c].B.tabs;
    }
    const T* h = (const T*)cases[c].B.h;
    const T* b = (const T*)cases[c].B.b;
    T* ht = (T*)cases[c].B.ht;
    T* bt = (T*)cases[c].B.bt;
    double* dW = cases[c].B.dW;
    const int32_t* flag = cases[c].B.flag;
    __syncthreads();  // the previous item's readers of L are done
    sweep_item<D, T, T, false>(fm, nvp, sc, fm.crec_i, crec_d, nullptr, fm.vidx, w, cs, frec, tabs, h, b,
                               ht, bt, dW, flag, ic, chunk, L);
  }
}

// Conservative update of the fused path: W^{n+1} = W^n - dW.
// The partial sums of the velocity blocks are added in block order.
template <int D>
__device__ __forceinline__ void apply_dW_at(int64_t i, int64_t nchunk, const double* __restrict__ vol,
                                            const double* __restrict__ W,
                                            const double* __restrict__ dWp, double* __restrict__ Wn,
                                            double* __restrict__ cellred, const int32_t* flag) {
  if (*flag) return;
  for (int x = 0; x < D + 2; ++x) {
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) s += dWp[(i * nchunk + c) * 5 + x];
    Wn[i * (D + 2) + x] = W[i * (D + 2) + x] - s;
  }
  const double V = vol[i];
  const double dr = Wn[i * (D + 2)] - W[i * (D + 2)];
  cellred[i * 3 + 0] = V * dr * dr;
  cellred[i * 3 + 1] = V;
  cellred[i * 3 + 2] = V * W[i * (D + 2)] * W[i * (D + 2)];
}

template <int D>
__global__ void k_apply_dW(int64_t nc, int64_t nchunk, const double* __restrict__ vol,
                           const double* __restrict__ W, const double* __restrict__ dWp,
                           double* __restrict__ Wn, double* __restrict__ cellred, const int32_t* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nc) apply_dW_at<D>(i, nchunk, vol, W, dWp, Wn, cellred, flag);
}

// Second stage (Eq. f_final) fused with the heat flux of the result.
// csn holds dt/(2 tau^{n+1}) and the Shakhov polynomials of W^{n+1} with q^n.
struct Stage2Lds {
  double ctab[3][NAX];
  double ax[NAX];
  double red[3 * 16];
};

template <int D, typename T>
__device__ __forceinline__ void stage2_q_cell(int64_t ic, const FusedMesh& fm, int64_t nvp,
                                              const double* __restrict__ w,
                                              const double* __restrict__ primn,
                                              const double* __restrict__ csn,
                                              const T* __restrict__ ht, const T* __restrict__ bt,
                                              T* __restrict__ h, T* __restrict__ b,
                                              double* __restrict__ qn, const int32_t* flag,
                                              Stage2Lds& L) {
  if (*flag) return;
  double(&ctab)[3][NAX] = L.ctab;
  double(&ax)[NAX] = L.ax;
  const int na = fm.na;
  const double* __restrict__ P = primn + ic * NPRIM;
  const double* __restrict__ cc = csn + ic * CSREC;
  for (int t = threadIdx.x; t < D * na; t += SWT) {
    const int d = t / na, n = t % na;
    const double a = fm.axis[n], U = P[1 + d], lam = P[4];
    ctab[d][n] = (d == 0 ? cc[CS_NORM] : 1.0) * exp(-lam * (a - U) * (a - U));
  }
  for (int t = threadIdx.x; t < na; t += SWT) ax[t] = fm.axis[t];
  __syncthreads();
  const double A = cc[CS_CC];
  const double inv = 1.0 / (1.0 + A);
  const double kc = cc[CS_KAP];
  const double U0 = P[1], U1 = P[2], U2 = P[3];
  const T* __restrict__ hti = ht + ic * nvp;
  T* __restrict__ hi = h + ic * nvp;
  double acc[3] = {0.0, 0.0, 0.0};
  const unsigned nv = (unsigned)fm.nv;
  crec_t<double>* csh = (crec_t<double>*)(cc + CS_SH);  // scalar loads of the uniform polynomials
  crec_t<double>* csb = (crec_t<double>*)(cc + CS_SB);
  // b: always in 2-D; in 3-D when the gas has internal degrees of freedom
  const bool hb = bt != nullptr;
  const T* __restrict__ bti = hb ? bt + ic * nvp : nullptr;
  auto body = [&](unsigned k, int pk, double htk, double btk, double wk) {
    double vv[3] = {0, 0, 0};
    double c0 = 1.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = (pk >> (8 * d)) & 255;
      vv[d] = ax[i];
      c0 *= ctab[d][i];
    }
    const double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
    double E, O;
    cubic_eo<D>(csh, vv, v2, E, O);
    const double hn = (htk + A * c0 * (1.0 + E + O)) * inv;
    __builtin_nontemporal_store((T)hn, &hi[k]);
    double bn = 0.0;
    if (hb) {
      double Eb, Ob;
      cubic_eo<D>(csb, vv, v2, Eb, Ob);
      bn = (btk + A * kc * c0 * (1.0 + Eb + Ob)) * inv;
      st(b + ic * nvp, k, bn);
    }
    // heat flux of h^{n+1} about U^{n+1} (Eq. reduced_heat_flux)
    const double c[3] = {vv[0] - U0, vv[1] - U1, D == 3 ? vv[2] - U2 : 0.0};
    double c2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) c2 += c[d] * c[d];
    const double s = wk * (c2 * hn + bn);
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] += s * c[d];
  };
  // four velocities per lane per pass, all their loads issued together, so
  // each lane keeps several HBM reads in flight
  constexpr unsigned UN = 4;
  unsigned k = threadIdx.x;
  for (; k + (UN - 1) * SWT < nv; k += UN * SWT) {
    int pk[UN];
    T hv[UN], bv[UN];
    double wv[UN];
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      hv[u] = __builtin_nontemporal_load(&hti[k + u * SWT]);
      bv[u] = hb ? bti[k + u * SWT] : T(0);
    }
    // the HBM reads go out first, the small cached arrays next, and no
    // arithmetic is moved between them
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      pk[u] = fm.vidx[k + u * SWT];
      wv[u] = w[k + u * SWT];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) body(k + u * SWT, pk[u], (double)hv[u], (double)bv[u], wv[u]);
  }
  for (; k < nv; k += SWT) body(k, fm.vidx[k], ld(hti, k), hb ? ld(bti, k) : 0.0, w[k]);
  block_sum<3>(acc, L.red);
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) qn[ic * 3 + d] = d < D ? 0.5 * acc[d] : 0.0;
}

template <int D, typename T>
__global__ __launch_bounds__(SWT) void k_stage2_q(FusedMesh fm, int64_t nvp,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ primn,
                                                  const double* __restrict__ csn,
                                                  const T* __restrict__ ht, const T* __restrict__ bt,
                                                  T* __restrict__ h, T* __restrict__ b,
                                                  double* __restrict__ qn, const int32_t* flag) {
  __shared__ Stage2Lds L;
  const int64_t per = (fm.nc + 7) / 8;
  const int64_t ic = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (ic >= fm.nc) return;
  stage2_q_cell<D, T>(ic, fm, nvp, w, primn, csn, ht, bt, h, b, qn, flag, L);
}

// Wall density with the wall cell's gradient evaluated in place.
struct WallLds {
  double ax[NAX];
  double wx[3][NAX];  // axis factors of the wall Maxwellian, C_w folded into the first
  double red[2 * 16];
  double red2[5 * 16];
};

// Wall density of one wall face: the incident free transport of the wall
// cell (its gradient evaluated in place) against the re-emitted wall
// Maxwellian, whose value at a tensor point is a product of three LDS
// axis factors (no per-velocity exp).
template <int D, typename T, bool LIM = false, bool BF = false>
__device__ __forceinline__ void wall_rho_at(int64_t wi, const DevMesh& m, const DevVel& v,
                                            const FusedMesh& fm, const GasP& g,
                                            const T* __restrict__ h, double* __restrict__ frec,
                                            const int32_t* flag, WallLds& S,
                                            const T* __restrict__ b = nullptr) {
  if (*flag) return;
  const int f = m.walls[wi];
  const int64_t L = m.fL[f];
  const int64_t nvp = v.nvp;
  double* R = &frec[(int64_t)f * FREC];
  const double lamw = R[FR_LAM], Cw = R[FR_C0], dt = g.dt;
  const int na = fm.na;
  for (int t = threadIdx.x; t < D * na; t += blockDim.x) {
    const int d = t / na, n = t % na;
    const double c = fm.axis[n] - R[FR_U + d];
    S.wx[d][n] = (d == 0 ? Cw : 1.0) * exp(-lamw * c * c);
  }
  for (int t = threadIdx.x; t < na; t += blockDim.x) S.ax[t] = fm.axis[t];
  __syncthreads();
  double nrm[3] = {0, 0, 0}, dxl[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    nrm[d] = m.fnorm[f * 3 + d];
    dxl[d] = m.fdxL[f * 3 + d];
  }
  // The wall cell's padded stencil from its fused record: the row across
  // each face (a neighbour, the zero row with coefficient 0 across a wall,
  // the ghost row across a far-field or outflow face) and the least-squares
  // coefficients, wave-uniform for the whole loop.
  crec_i_t* ci = (crec_i_t*)(fm.crec_i + L * CRI);
  crec_t<double>* cd = (crec_t<double>*)(fm.crec_d + L * CRD);
  const T* __restrict__ hl_row = h + L * nvp;
  const T* hs_row[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) hs_row[s] = h + (int64_t)ci[2 + s] * nvp;
  double acc[2] = {0.0, 0.0};
  // with BF: the wall flux's moments, incident (time-integrated free transport
  // of the wall cell's h, and b in 2-D) and reflected (per unit rho_w dt)
  double bfi[D + 2], bfr[D + 2];
#pragma unroll
  for (int x = 0; x < D + 2; ++x) bfi[x] = bfr[x] = 0.0;
  // Four velocities per lane per pass: their axis indices are loaded one
  // pass ahead, and the rows of the incident ones (u.n > 0, the only ones
  // that read f) are loaded together before any arithmetic.
  constexpr unsigned UN = 4;
  const unsigned nb = blockDim.x, nv = (unsigned)v.nv;
  int pkn[UN];
#pragma unroll
  for (unsigned u = 0; u < UN; ++u) {
    const unsigned kk = threadIdx.x + u * nb;
    pkn[u] = kk < nv ? fm.vidx[kk] : 0;
  }
  for (unsigned k0 = threadIdx.x; k0 < nv; k0 += UN * nb) {
    int pk[UN];
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      pk[u] = pkn[u];
      const unsigned kk = k0 + (UN + u) * nb;
      pkn[u] = kk < nv ? fm.vidx[kk] : 0;
    }
    double uu[UN][3], un[UN];
    int id[UN][3];
    bool inc[UN], out[UN];
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      const bool valid = k0 + u * nb < nv;
      un[u] = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        id[u][d] = (pk[u] >> (8 * d)) & 255;
        uu[u][d] = d < D ? S.ax[id[u][d]] : 0.0;
        if (d < D) un[u] += uu[u][d] * nrm[d];
      }
      inc[u] = valid && un[u] > 0.0;
      out[u] = valid && un[u] < 0.0;
    }
    double hl[UN], hs[UN][4], wk[UN];
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      const unsigned kk = k0 + u * nb;
      hl[u] = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) hs[u][s] = 0.0;
      if (inc[u]) {
        hl[u] = ld(hl_row, kk);
#pragma unroll
        for (int s = 0; s < 4; ++s) hs[u][s] = ld(hs_row[s], kk);
      }
      wk[u] = (inc[u] || out[u]) ? v.w[kk] : 0.0;
    }
#pragma unroll
    for (unsigned u = 0; u < UN; ++u) {
      if (inc[u]) {
        // incident: free transport of the wall cell's reconstruction
        double gr[3] = {0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double dh = hs[u][s] - hl[u];
#pragma unroll
          for (int d = 0; d < D; ++d) gr[d] += cd[d * 4 + s] * dh;
        }
        if constexpr (LIM) {
          // the wall cell's gradient limited as the sweep limits it
          crec_t<double>* cl = (crec_t<double>*)(fm.crec_l + L * CRL);
          double lo = hl[u], hi = hl[u];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const double vs = cl[1 + s] * hl[u] + hs[u][s];
            lo = fmin(lo, vs);
            hi = fmax(hi, vs);
          }
          const double ph = venkat_phi<D>(hl[u], lo, hi, gr, cd + CRD_F0 + 4, CRD_FS, cl[0]);
#pragma unroll
          for (int d = 0; d < D; ++d) gr[d] *= ph;
        }
        double hf = hl[u], ugh = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          hf += dxl[d] * gr[d];
          ugh += uu[u][d] * gr[d];
        }
        acc[0] += wk[u] * un[u] * (dt * hf - 0.5 * dt * dt * ugh);
        if constexpr (BF) {
          const double fh = wk[u] * un[u] * (dt * hf - 0.5 * dt * dt * ugh);
          double u2 = 0.0;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            bfi[1 + d] += uu[u][d] * fh;
            u2 += uu[u][d] * uu[u][d];
          }
          bfi[0] += fh;
          bfi[D + 1] += 0.5 * u2 * fh;
          if (b != nullptr) {
            // the b part of the energy: the same free transport of the wall cell's b
            const unsigned kk = k0 + u * nb;
            const T* __restrict__ bl_row = b + L * nvp;
            const double bl = ld(bl_row, kk);
            double gb[3] = {0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const double db = ld(b + (int64_t)ci[2 + s] * nvp, kk) - bl;
#pragma unroll
              for (int d = 0; d < D; ++d) gb[d] += cd[d * 4 + s] * db;
            }
            if constexpr (LIM) {
              crec_t<double>* cl = (crec_t<double>*)(fm.crec_l + L * CRL);
              double lo = bl, hi = bl;
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const double vs = cl[1 + s] * bl + ld(b + (int64_t)ci[2 + s] * nvp, kk);
                lo = fmin(lo, vs);
                hi = fmax(hi, vs);
              }
              const double pb = venkat_phi<D>(bl, lo, hi, gb, cd + CRD_F0 + 4, CRD_FS, cl[0]);
#pragma unroll
              for (int d = 0; d < D; ++d) gb[d] *= pb;
            }
            double bf = bl, ugb = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
              bf += dxl[d] * gb[d];
              ugb += uu[u][d] * gb[d];
            }
            bfi[D + 1] += 0.5 * wk[u] * un[u] * (dt * bf - 0.5 * dt * dt * ugb);
          }
        }
      } else if (out[u]) {
        double M = S.wx[0][id[u][0]];
#pragma unroll
        for (int d = 1; d < D; ++d) M *= S.wx[d][id[u][d]];
        acc[1] += wk[u] * un[u] * M;
        if constexpr (BF) {
          const double fm_ = wk[u] * un[u] * M;
          double u2 = 0.0;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            bfr[1 + d] += uu[u][d] * fm_;
            u2 += uu[u][d] * uu[u][d];
          }
          bfr[0] += fm_;
          // the re-emitted b = K_xi/(2 lambda_w) H_w adds to the energy
          bfr[D + 1] += 0.5 * (u2 + v.kxi / (2.0 * lamw)) * fm_;
        }
      }
    }
  }
  block_sum<2>(acc, S.red);
  if constexpr (BF) {
    __syncthreads();
    block_sum<D + 2>(bfi, S.red2);
    __syncthreads();
    block_sum<D + 2>(bfr, S.red2);
  }
  if (threadIdx.x == 0) {
    const double rhow = -acc[0] / (dt * acc[1]);
    R[FR_RHOW] = rhow;
    // the wall face's time-integrated flux of mass, momentum and energy
    // (Eq. macro_flux): incident part plus rho_w dt times the re-emitted part
    if constexpr (BF)
      for (int x = 0; x < D + 2; ++x) R[FR_BF + x] = bfi[x] + rhow * dt * bfr[x];
  }
}

// One work-group per wall face (256 lanes measured faster than 1024).
constexpr int WALLT = 256;

template <int D, typename T>
__global__ __launch_bounds__(WALLT) void k_wall_rho_inline(DevMesh m, DevVel v, FusedMesh fm, GasP g,
                                                         const T* __restrict__ h,
                                                         double* __restrict__ frec,
                                                         const int32_t* flag, const T* b_bf,
                                                         int track) {
  __shared__ WallLds S;
  // with tracking the pass also keeps each wall face's flux; b_bf is the b
  // array where b is stored (its part of the energy flux), else null
  if (track) {
    if (fm.crec_l) wall_rho_at<D, T, true, true>(blockIdx.x, m, v, fm, g, h, frec, flag, S, b_bf);
    else wall_rho_at<D, T, false, true>(blockIdx.x, m, v, fm, g, h, frec, flag, S, b_bf);
  } else {
    if (fm.crec_l) wall_rho_at<D, T, true>(blockIdx.x, m, v, fm, g, h, frec, flag, S);
    else wall_rho_at<D, T, false>(blockIdx.x, m, v, fm, g, h, frec, flag, S);
  }
}

// Ghost rows of the far-field / outflow faces: the Maxwellian of the face's
// ghost state W_g (written by the interface-equilibrium pass), h and, where
// b is stored, b = K_xi/(2 lambda_g) h, so the sweep reads them as neighbour rows.
template <int D, typename T>
__device__ __forceinline__ void ghost_row_at(int64_t m, int64_t nc, const int32_t* __restrict__ ffaces,
                                             const DevVel& v, const double* __restrict__ frec,
                                             T* __restrict__ h, T* __restrict__ b,
                                             const int32_t* flag) {
  if (*flag) return;
  const double* R = &frec[(int64_t)ffaces[m] * FREC];
  const double C = R[FR_GC], lam = R[FR_GLAM];
  const double U[3] = {R[FR_GU], R[FR_GU + 1], R[FR_GU + 2]};
  const int64_t row = (nc + 1 + m) * v.nvp;
  for (int64_t k = threadIdx.x; k < v.nvp; k += blockDim.x) {
    double hv = 0.0;
    if (k < v.nv) {
      double c2 = 0.0;
      for (int d = 0; d < D; ++d) {
        const double c = v.u[d * v.nvp + k] - U[d];
        c2 += c * c;
      }
      hv = C * exp(-lam * c2);
    }
    st(h, row + k, hv);
    if (v.has_b) st(b, row + k, v.kxi / (2.0 * lam) * hv);
  }
}

template <int D, typename T>
__global__ __launch_bounds__(SWT) void k_ghost_rows(int64_t nc, const int32_t* __restrict__ ffaces,
                                                    DevVel v, const double* __restrict__ frec,
                                                    T* __restrict__ h, T* __restrict__ b,
                                                    const int32_t* flag) {
  ghost_row_at<D, T>(blockIdx.x, nc, ffaces, v, frec, h, b, flag);
}

// ---- batched forms: one launch covers every case of a batch ---------------
// Element t of a flattened range belongs to case c with off[c] <= t < off[c+1].
__device__ __forceinline__ int case_of(const int64_t* __restrict__ off, int n, int64_t t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// elements per lane of the batch's flattened element-wise kernels (k_tables_b,
// k_to_f32_b)
constexpr int PER_LANE = 16;

// next = 0: W^n, q -> prim, cs;  next = 1: W^{n+1}, q -> primn, csn
template <int D>
__global__ void k_cell_prep_b(BatchDev bd, int next) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= bd.cell_off[bd.n]) return;
  const int c = case_of(bd.cell_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  const int64_t i = t - bd.cell_off[c];
  if (next) cell_prep_at<D>(i, C.g, C.B.Wn, C.B.q, C.B.primn, C.B.csn, C.B.flag);
  else cell_prep_at<D>(i, C.g, C.B.W, C.B.q, C.B.prim, C.B.cs, C.B.flag);
}

template <int D>
__global__ void k_tables_b(BatchDev bd) {
  // each wave takes PER_LANE consecutive runs of 64 entries; a lane searches
  // for an entry's case only when it leaves the previous entry's case
  const int64_t lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t n = bd.tab_off[bd.n];
  int c = 0;
  int64_t lo = 0, hi = 0;
  for (int j = 0; j < PER_LANE; ++j) {
    const int64_t t = (wave * PER_LANE + j) * 64 + lane;
    if (t >= n) break;
    if (t < lo || t >= hi) {
      c = case_of(bd.tab_off, bd.n, t);
      lo = bd.tab_off[c];
      hi = bd.tab_off[c + 1];
    }
    const CaseDev& C = bd.cases[c];
    tables_at<D>(t - lo, C.m.nf, C.fm.na, C.fm.axis, C.m.fbc, C.g, C.B.frec, C.B.prim, C.B.cs,
                 C.B.tabs, C.B.flag);
  }
}

// FP32 copies of every case's per-step face records, cell records and axis
// tables (an FP32 batch's sweep computes from them): three flattened ranges.
// Each wave converts PER_LANE consecutive runs of 64 elements, so that the
// search for an element's case (a chain of dependent loads) is made once per
// case a lane meets, not once per element.
__global__ void k_to_f32_b(BatchDev bd, int64_t nfr, int64_t ncs, int64_t ntab) {
  const int64_t lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  // the case of the lane's previous element: its range kind, the range's
  // first unit (face, cell or table entry) and end, and the arrays
  int kind_c = -1;
  int64_t lo = 0, hi = 0;
  const double* src = nullptr;
  float* dst = nullptr;
  for (int j = 0; j < PER_LANE; ++j) {
    const int64_t t = (wave * PER_LANE + j) * 64 + lane;
    int kind;
    int64_t e, unit;  // element within its range, and the unit holding it
    const int64_t* off;
    if (t < nfr) {
      kind = 0, e = t, unit = t / FREC, off = bd.face_off;
    } else if (t - nfr < ncs) {
      kind = 1, e = t - nfr, unit = e / CSREC, off = bd.cell_off;
    } else if (t - nfr - ncs < ntab) {
      kind = 2, e = t - nfr - ncs, unit = e, off = bd.tab_off;
    } else {
      break;
    }
    if (kind != kind_c || unit < lo || unit >= hi) {
      const int c = case_of(off, bd.n, unit);
      const CaseDev& C = bd.cases[c];
      kind_c = kind;
      lo = off[c];
      hi = off[c + 1];
      src = kind == 0 ? C.B.frec : kind == 1 ? C.B.cs : C.B.tabs;
      dst = kind == 0 ? C.B.frec32 : kind == 1 ? C.B.cs32 : C.B.tabs32;
    }
    const int64_t i = e - lo * (kind == 0 ? FREC : kind == 1 ? CSREC : 1);
    dst[i] = (float)src[i];
  }
}

template <int D>
__global__ void k_apply_dW_b(BatchDev bd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= bd.cell_off[bd.n]) return;
  const int c = case_of(bd.cell_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  apply_dW_at<D>(t - bd.cell_off[c], C.sc.nchunk, C.m.vol, C.B.W, C.B.dW, C.B.Wn, C.B.cellred,
                 C.B.flag);
}

// one block per cell of the batch
template <int D, typename T>
__global__ __launch_bounds__(SWT) void k_stage2_q_b(BatchDev bd) {
  __shared__ Stage2Lds L;
  const int64_t t = blockIdx.x;
  const int c = case_of(bd.cell_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  stage2_q_cell<D, T>(t - bd.cell_off[c], C.fm, C.v.nvp, C.v.w, C.B.primn, C.B.csn,
                      (const T*)C.B.ht, (const T*)C.B.bt, (T*)C.B.h, (T*)C.B.b, C.B.qn, C.B.flag,
                      L);
}

// one block per far-field / outflow face of the batch
template <int D, typename T>
__global__ __launch_bounds__(SWT) void k_ghost_rows_b(BatchDev bd) {
  const int64_t t = blockIdx.x;
  const int c = case_of(bd.ff_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  ghost_row_at<D, T>(t - bd.ff_off[c], C.m.nc, C.fm.ffaces, C.v, C.B.frec, (T*)C.B.h, (T*)C.B.b,
                     C.B.flag);
}

// one block per wall face of the batch
template <int D, typename T>
__global__ __launch_bounds__(WALLT) void k_wall_rho_b(BatchDev bd) {
  __shared__ WallLds S;
  const int64_t t = blockIdx.x;
  const int c = case_of(bd.wall_off, bd.n, t);
  const CaseDev& C = bd.cases[c];
  wall_rho_at<D, T>(t - bd.wall_off[c], C.m, C.v, C.fm, C.g, (const T*)C.B.h, C.B.frec, C.B.flag,
                    S);
}

}  // namespace

#define UGKS_DISPATCH_D(D_, ...) \
  do {                           \
    if ((D_) == 2) {             \
      constexpr int DD = 2;      \
      __VA_ARGS__;               \
    } else {                     \
      constexpr int DD = 3;      \
      __VA_ARGS__;               \
    }                            \
  } while (0)

#define UGKS_DISPATCH_DT(D_, P_, ...)   \
  do {                                  \
    if ((P_) == UGKS_FP32) {            \
      using TT = float;                 \
      UGKS_DISPATCH_D(D_, __VA_ARGS__); \
    } else {                            \
      using TT = double;                \
      UGKS_DISPATCH_D(D_, __VA_ARGS__); \
    }                                   \
  } while (0)

// precision only (the dimension fixed by the kernel named)
#define UGKS_DISPATCH_T(P_, ...)      \
  do {                                \
    if ((P_) == UGKS_FP32) {          \
      using TT = float;               \
      __VA_ARGS__;                    \
    } else {                          \
      using TT = double;              \
      __VA_ARGS__;                    \
    }                                 \
  } while (0)

hipError_t launch_apply_dW(int D, const DevMesh& m, int64_t nchunk, const double* W,
                          const double* dWp, double* Wn, double* cellred, const int32_t* flag,
                          hipStream_t s) {
  const unsigned grid = (unsigned)((m.nc + 255) / 256);
  UGKS_DISPATCH_D(D, k_apply_dW<DD><<<grid, 256, 0, s>>>(m.nc, nchunk, m.vol, W, dWp, Wn, cellred, flag));
  return hipGetLastError();
}

hipError_t launch_tables(int D, const DevMesh& m, const FusedMesh& fm, const GasP& g,
                         const double* frec, const double* prim, const double* cs, double* tabs,
                         const int32_t* flag, hipStream_t s) {
  const int64_t n = (m.nf + m.nc) * (int64_t)D * fm.na;
  const unsigned grid = (unsigned)((n + 255) / 256);
  UGKS_DISPATCH_D(D, k_tables<DD><<<grid, 256, 0, s>>>(m.nf, m.nc, fm.na, fm.axis, m.fbc, g, frec,
                                                        prim, cs, tabs, flag));
  return hipGetLastError();
}

hipError_t launch_cell_prep(int D, int64_t nc, const GasP& g, const double* W, const double* q,
                            double* prim, double* cs, int32_t* flag, hipStream_t s) {
  const unsigned grid = (unsigned)((nc + 127) / 128);
  UGKS_DISPATCH_D(D, k_cell_prep<DD><<<grid, 128, 0, s>>>(nc, g, W, q, prim, cs, flag));
  return hipGetLastError();
}

hipError_t launch_sweep(int D, int prec, const FusedMesh& fm, const DevVel& v, const GasP& g,
                        const SweepSched& sc, const void* crec_d, const void* crec_l,
                        const void* cs, const void* frec,
                        const void* tabs, const void* h, const void* b, void* ht, void* bt,
                        double* dWp, const int32_t* flag, hipStream_t s) {
  const int64_t ntile = (fm.nc + sc.tile - 1) / sc.tile;
  const unsigned grid = (unsigned)(((ntile + 7) / 8) * 8 * sc.nchunk * sc.tile);
  // a sparse set's pairs carry their own packed axis indices
  const int32_t* pv = fm.sparse ? fm.pvidx : fm.vidx;
#define UGKS_SWEEP_ARGS                                                                       \
  fm, v.nvp, sc, fm.crec_i, (const TT*)crec_d, (const TT*)crec_l, pv, v.w, (const TT*)cs,      \
      (const TT*)frec, (const TT*)tabs, (const TT*)h, (const TT*)b, (TT*)ht, (TT*)bt, dWp, flag
#define UGKS_SWEEP_NB(LIMV, SPV)                                                             \
  do {                                                                                        \
    if (D == 3 && b)                                                                          \
      UGKS_DISPATCH_T(prec, (k_sweep<3, TT, LIMV, SPV, true><<<grid, SWT, 0, s>>>(UGKS_SWEEP_ARGS))); \
    else                                                                                      \
      UGKS_DISPATCH_DT(D, prec, (k_sweep<DD, TT, LIMV, SPV, false><<<grid, SWT, 0, s>>>(UGKS_SWEEP_ARGS))); \
  } while (0)
  if (fm.sparse) {
    if (crec_l) UGKS_SWEEP_NB(true, true);
    else UGKS_SWEEP_NB(false, true);
  } else {
    if (crec_l) UGKS_SWEEP_NB(true, false);
    else UGKS_SWEEP_NB(false, false);
  }
#undef UGKS_SWEEP_NB
#undef UGKS_SWEEP_ARGS
  return hipGetLastError();
}

// FP64 -> FP32 copies of the sweep's per-step records (FP32 compute form)
__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ fa, int64_t na,
                         const double* __restrict__ b, float* __restrict__ fb, int64_t nb,
                         const double* __restrict__ c, float* __restrict__ fc, int64_t nc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < na) fa[t] = (float)a[t];
  else if (t < na + nb) fb[t - na] = (float)b[t - na];
  else if (t < na + nb + nc) fc[t - na - nb] = (float)c[t - na - nb];
}

hipError_t launch_to_f32(const double* a, float* fa, int64_t na, const double* b, float* fb,
                         int64_t nb, const double* c, float* fc, int64_t nc, hipStream_t s) {
  const int64_t n = na + nb + nc;
  if (n == 0) return hipSuccess;
  k_to_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, fa, na, b, fb, nb, c, fc, nc);
  return hipGetLastError();
}

hipError_t launch_stage2_q(int D, int prec, const FusedMesh& fm, const DevVel& v,
                           const double* primn, const double* csn, const void* ht, const void* bt,
                           void* h, void* b, double* qn, const int32_t* flag, hipStream_t s) {
  const unsigned grid = (unsigned)(((fm.nc + 7) / 8) * 8);
  UGKS_DISPATCH_DT(D, prec, k_stage2_q<DD, TT><<<grid, SWT, 0, s>>>(
      fm, v.nvp, v.w, primn, csn, (const TT*)ht, (const TT*)bt, (TT*)h, (TT*)b, qn, flag));
  return hipGetLastError();
}

hipError_t launch_wall_rho_inline(int D, int prec, const DevMesh& m, const DevVel& v,
                                  const FusedMesh& fm, const GasP& g, const void* h, double* frec,
                                  const int32_t* flag, hipStream_t s, int track, const void* b_bf) {
  if (m.nwall == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_wall_rho_inline<DD, TT><<<(unsigned)m.nwall, WALLT, 0, s>>>(
      m, v, fm, g, (const TT*)h, frec, flag, (const TT*)b_bf, track));
  return hipGetLastError();
}

// The step's boundary flux, added to the running sum acc[0..D+1]: the sum
// over boundary faces of S_f F_f, from the wall records' fluxes (fused path,
// FR_BF) or from the face fluxes (staged path, every boundary face).  One
// work-group; each lane adds its faces in order, then a fixed reduction.
template <int D>
__global__ __launch_bounds__(256) void k_bflux(DevMesh m, const double* __restrict__ frec,
                                               const double* __restrict__ F, int staged,
                                               double* __restrict__ acc, const int32_t* flag) {
  __shared__ double red[5 * 16];
  if (*flag) return;
  double s[D + 2];
  for (int x = 0; x < D + 2; ++x) s[x] = 0.0;
  if (staged) {
    for (int64_t f = threadIdx.x; f < m.nf; f += 256)
      if (m.fR[f] < 0)
        for (int x = 0; x < D + 2; ++x) s[x] += m.farea[f] * F[f * 5 + x];
  } else {
    for (int64_t wi = threadIdx.x; wi < m.nwall; wi += 256) {
      const int64_t f = m.walls[wi];
      for (int x = 0; x < D + 2; ++x) s[x] += m.farea[f] * frec[f * FREC + FR_BF + x];
    }
  }
  block_sum<D + 2>(s, red);
  if (threadIdx.x == 0)
    for (int x = 0; x < D + 2; ++x) acc[x] += s[x];
}

hipError_t launch_bflux(int D, const DevMesh& m, const double* frec, const double* F, int staged,
                        double* acc, const int32_t* flag, hipStream_t s) {
  UGKS_DISPATCH_D(D, k_bflux<DD><<<1, 256, 0, s>>>(m, frec, F, staged, acc, flag));
  return hipGetLastError();
}

// ---- batched launchers ------------------------------------------------------
hipError_t launch_cell_prep_b(int D, const BatchDev& bd, int64_t ncell, int next, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  const unsigned grid = (unsigned)((ncell + 127) / 128);
  UGKS_DISPATCH_D(D, k_cell_prep_b<DD><<<grid, 128, 0, s>>>(bd, next));
  return hipGetLastError();
}

hipError_t launch_to_f32_b(const BatchDev& bd, int64_t nface, int64_t ncell, int64_t ntab,
                           hipStream_t s) {
  const int64_t n = nface * FREC + ncell * CSREC + ntab;
  if (n == 0) return hipSuccess;
  const int64_t waves = (n + 64 * PER_LANE - 1) / (64 * PER_LANE);
  k_to_f32_b<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(bd, nface * FREC, ncell * CSREC, ntab);
  return hipGetLastError();
}

hipError_t launch_tables_b(int D, const BatchDev& bd, int64_t ntab, hipStream_t s) {
  if (ntab == 0) return hipSuccess;
  const int64_t waves = (ntab + 64 * PER_LANE - 1) / (64 * PER_LANE);
  const unsigned grid = (unsigned)((waves + 3) / 4);
  UGKS_DISPATCH_D(D, k_tables_b<DD><<<grid, 256, 0, s>>>(bd));
  return hipGetLastError();
}

hipError_t launch_apply_dW_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  const unsigned grid = (unsigned)((ncell + 255) / 256);
  UGKS_DISPATCH_D(D, k_apply_dW_b<DD><<<grid, 256, 0, s>>>(bd));
  return hipGetLastError();
}

hipError_t launch_stage2_q_b(int D, int prec, const BatchDev& bd, int64_t ncell, hipStream_t s) {
  if (ncell == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_stage2_q_b<DD, TT><<<(unsigned)ncell, SWT, 0, s>>>(bd));
  return hipGetLastError();
}

hipError_t launch_wall_rho_b(int D, int prec, const BatchDev& bd, int64_t nwall, hipStream_t s) {
  if (nwall == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_wall_rho_b<DD, TT><<<(unsigned)nwall, WALLT, 0, s>>>(bd));
  return hipGetLastError();
}

hipError_t launch_ghost_rows(int D, int prec, const FusedMesh& fm, const DevVel& v,
                             const double* frec, void* h, void* b, const int32_t* flag,
                             hipStream_t s) {
  if (fm.nff == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_ghost_rows<DD, TT><<<(unsigned)fm.nff, SWT, 0, s>>>(
      fm.nc, fm.ffaces, v, frec, (TT*)h, (TT*)b, flag));
  return hipGetLastError();
}

hipError_t launch_ghost_rows_b(int D, int prec, const BatchDev& bd, int64_t nff, hipStream_t s) {
  if (nff == 0) return hipSuccess;
  UGKS_DISPATCH_DT(D, prec, k_ghost_rows_b<DD, TT><<<(unsigned)nff, SWT, 0, s>>>(bd));
  return hipGetLastError();
}

hipError_t launch_sweep_b(int D, int prec, const BatchDev& bd, int64_t grid, int threads,
                          hipStream_t s) {
  if (bd.nitems == 0) return hipSuccess;
  if (threads % 64 != 0 || threads < 64 || threads > SWT) return hipErrorInvalidValue;
  UGKS_DISPATCH_DT(D, prec, k_sweep_b<DD, TT><<<(unsigned)grid, threads, 0, s>>>(bd));
  return hipGetLastError();
}

int sweep_b_blocks_per_cu(int D, int prec, int threads) {
  int n = 0;
  hipError_t e = hipSuccess;
  UGKS_DISPATCH_DT(D, prec, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &n, reinterpret_cast<const void*>(&k_sweep_b<DD, TT>), threads, 0));
  return e == hipSuccess ? n : 0;
}

}  // namespace ugks
