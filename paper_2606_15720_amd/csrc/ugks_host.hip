// Host side of the gfx950 UGKS library: the C ABI declared in ugks.h.
//
// ugks_create validates the mesh and velocity set, renumbers nothing the
// caller can see (all outputs come back in the caller's order), precomputes
// the least-squares coefficients of every cell (unweighted, one row per face
// neighbour or mirror ghost), pads the velocity set with zero-weight points
// to a multiple of the velocity block, fixes the time step from the CFL bound
// and allocates every device buffer once.  ugks_step only enqueues kernels.
#include "ugks_host_util.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <fstream>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <sstream>

using namespace ugks;
using namespace ugks::host;

namespace {

thread_local std::string g_create_error;

// Solve the D x D SPD normal system by Cholesky; returns false if singular.
bool chol_inverse(int D, const double* N, double* Ninv) {
  double Lm[9] = {0};
  for (int j = 0; j < D; ++j) {
    double s = N[j * 3 + j];
    for (int k = 0; k < j; ++k) s -= Lm[j * 3 + k] * Lm[j * 3 + k];
    if (!(s > 0.0)) return false;
    Lm[j * 3 + j] = std::sqrt(s);
    for (int i = j + 1; i < D; ++i) {
      double t = N[i * 3 + j];
      for (int k = 0; k < j; ++k) t -= Lm[i * 3 + k] * Lm[j * 3 + k];
      Lm[i * 3 + j] = t / Lm[j * 3 + j];
    }
  }
  for (int col = 0; col < D; ++col) {
    double y[3], x[3];
    for (int i = 0; i < D; ++i) {
      double t = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= Lm[i * 3 + k] * y[k];
      y[i] = t / Lm[i * 3 + i];
    }
    for (int i = D - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < D; ++k) t -= Lm[k * 3 + i] * x[k];
      x[i] = t / Lm[i * 3 + i];
    }
    for (int i = 0; i < D; ++i) Ninv[i * 3 + col] = x[i];
  }
  return true;
}


// The checks of a case's arguments that need no mesh traversal: pointers,
// sizes, dimension and gas constants.
void check_case_args(const ugks_mesh* mesh, const ugks_velocity* vel, const ugks_gas* gas,
                     const double* W0) {
  fail_if(!mesh || !vel || !gas || !W0, "null argument");
  const int D = mesh->dim;
  fail_if(D != 2 && D != 3, "mesh.dim must be 2 or 3");
  fail_if(gas->K < 0, "gas.K (internal degrees of freedom) must be >= 0");
  const int64_t nc = mesh->n_cells, nf = mesh->n_faces, nv = vel->nv;
  fail_if(nc <= 0 || nf <= 0 || nv <= 0, "empty mesh or velocity set");
  fail_if(nc >= (int64_t)INT32_MAX || nf >= (int64_t)INT32_MAX, "mesh too large for 32-bit indices");
  fail_if(!mesh->cell_volume || !mesh->cell_centroid || !mesh->face_cells || !mesh->face_area ||
              !mesh->face_normal || !mesh->face_centroid || !mesh->face_bc || !mesh->face_bc_id ||
              !vel->u || !vel->w,
          "null mesh or velocity array");
  fail_if(!(gas->Pr > 0.0) || !(gas->R > 0.0) || !(gas->T_ref > 0.0) || !(gas->mu_ref > 0.0),
          "gas constants must be positive");
}

void build(ugks_ctx* c, const ugks_mesh* mesh, const ugks_velocity* vel, const ugks_gas* gas,
           const ugks_bc* bcs, int32_t n_bc, const double* W0, const ugks_options* opt) {
  check_case_args(mesh, vel, gas, W0);
  const int D = mesh->dim;
  const int64_t nc = mesh->n_cells, nf = mesh->n_faces, nv = vel->nv;
  int prec = opt && opt->precision ? opt->precision : UGKS_FP64;
  fail_if(prec != UGKS_FP64 && prec != UGKS_FP32, "precision must be 64 or 32");
  int Bv = opt && opt->block_v ? opt->block_v : 0;
  fail_if(Bv < 0 || Bv % WAVE != 0, "block_v must be 0 or a positive multiple of 64");
  const int tile = opt && opt->tile_cells ? opt->tile_cells : 0;
  fail_if(tile < 0, "tile_cells must be >= 0");
  const int lim = opt ? opt->limiter : 0;
  const double limk = opt ? opt->limiter_k : 0.0;
  fail_if(lim != 0 && lim != 1, "limiter must be 0 (none) or 1 (Venkatakrishnan)");
  fail_if(lim == 1 && !(limk >= 0.0 && std::isfinite(limk)), "limiter_k must be finite and >= 0");
  c->D = D;
  // K_xi = K + 3 - D internal and out-of-plane dimensions (Eq. Kxi_def); b
  // is carried when there are any (always in 2-D)
  c->kxi = gas->K + 3 - D;
  c->nr = c->kxi > 0 ? 2 : 1;
  c->prec = prec;
  c->Bv = Bv;
  c->flags = opt ? opt->flags : 0;
  c->nc = nc;
  c->nf = nf;
  c->nv = nv;
  // rows are padded to whole waves; the velocity block of the sweep is a
  // scheduling unit and needs no padding
  c->nvp = (nv + WAVE - 1) / WAVE * WAVE;
  {
    // a point whose mirror -u_k is not in the set is paired with a pad slot
    // on the fused sweep: keep at least one
    std::set<std::vector<double>> pts;
    for (int64_t k = 0; k < nv; ++k) pts.insert(std::vector<double>(vel->u + k * D, vel->u + (k + 1) * D));
    bool all_mirrored = true;
    for (int64_t k = 0; k < nv && all_mirrored; ++k) {
      std::vector<double> m(D);
      for (int d = 0; d < D; ++d) m[d] = -vel->u[k * D + d];
      all_mirrored = pts.count(m) > 0;
    }
    if (!all_mirrored && c->nvp == nv) c->nvp += WAVE;
  }

  // ---- mesh validation and cell -> face tables --------------------------
  for (int64_t i = 0; i < nc; ++i)
    fail_if(!(mesh->cell_volume[i] > 0.0), "non-positive cell volume");
  std::vector<int32_t> nfc(nc, 0), cface(nc * MAXF, -1), cnbr(nc * MAXF, -1);
  std::vector<double> csign(nc * MAXF, 0.0);
  std::vector<int32_t> fL(nf), fR(nf), fbc(nf), fbcid(nf), walls;
  std::vector<double> farea(nf), fnorm(nf * 3, 0.0), fdxL(nf * 3, 0.0), fdxR(nf * 3, 0.0),
      fmir(nf * 3, 0.0);
  // ---- cell renumbering: Z-order (Morton) of the centroids, so that cells
  // with nearby indices are spatial neighbours (they run together and share
  // stencil rows in cache); the caller never sees this order
  std::vector<int64_t> perm(nc), inv(nc);
  {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < nc; ++i)
      for (int d = 0; d < D; ++d) {
        lo[d] = std::min(lo[d], mesh->cell_centroid[i * D + d]);
        hi[d] = std::max(hi[d], mesh->cell_centroid[i * D + d]);
      }
    std::vector<std::pair<uint64_t, int64_t>> key(nc);
    for (int64_t i = 0; i < nc; ++i) {
      uint64_t code = 0;
      for (int d = 0; d < D; ++d) {
        const double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
        uint64_t qd = (uint64_t)std::min(1048575.0, std::floor((mesh->cell_centroid[i * D + d] - lo[d]) / span * 1048576.0));
        for (int bit = 0; bit < 20; ++bit) code |= ((qd >> bit) & 1ull) << (bit * D + d);
      }
      key[i] = {(c->flags & 4) ? (uint64_t)i : code, i};
    }
    std::stable_sort(key.begin(), key.end());
    for (int64_t i = 0; i < nc; ++i) {
      perm[i] = key[i].second;
      inv[key[i].second] = i;
    }
  }
  std::vector<double> cen(nc * 3, 0.0), vol(nc);
  for (int64_t i = 0; i < nc; ++i) {
    vol[i] = mesh->cell_volume[perm[i]];
    for (int d = 0; d < D; ++d) cen[i * 3 + d] = mesh->cell_centroid[perm[i] * D + d];
  }
  std::vector<double> closure(nc * 3, 0.0), asum(nc, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    int64_t L = mesh->face_cells[2 * f], R = mesh->face_cells[2 * f + 1];
    int kind = mesh->face_bc[f];
    fail_if(L < 0 || L >= nc, "face_cells L out of range");
    fail_if(kind < 0 || kind > 3, "unknown face_bc");
    fail_if(kind == UGKS_BC_INTERIOR && (R < 0 || R >= nc || R == L), "interior face needs a distinct R");
    fail_if(kind != UGKS_BC_INTERIOR && R != -1, "boundary face must have R = -1");
    L = inv[L];
    if (R >= 0) R = inv[R];
    fail_if(!(mesh->face_area[f] > 0.0), "non-positive face area");
    double nn = 0.0;
    for (int d = 0; d < D; ++d) nn += mesh->face_normal[f * D + d] * mesh->face_normal[f * D + d];
    fail_if(std::fabs(nn - 1.0) > 1e-10, "face normal is not a unit vector");
    if (kind != UGKS_BC_INTERIOR) {
      int id = mesh->face_bc_id[f];
      fail_if(id < 0 || id >= n_bc || !bcs, "face_bc_id out of range");
      fail_if(bcs[id].kind != kind, "face_bc does not match the boundary table kind");
      if (kind == UGKS_BC_WALL) {
        double un = 0.0;
        for (int d = 0; d < D; ++d) un += bcs[id].U[d] * mesh->face_normal[f * D + d];
        fail_if(std::fabs(un) > 1e-12, "wall velocity must be tangential");
        walls.push_back((int32_t)f);
      }
    }
    fL[f] = (int32_t)L;
    fR[f] = (int32_t)R;
    fbc[f] = kind;
    fbcid[f] = mesh->face_bc_id[f];
    farea[f] = mesh->face_area[f];
    double dn = 0.0;
    for (int d = 0; d < D; ++d) {
      double n = mesh->face_normal[f * D + d];
      double xf = mesh->face_centroid[f * D + d];
      double sh = mesh->face_shift ? mesh->face_shift[f * D + d] : 0.0;
      fnorm[f * 3 + d] = n;
      fdxL[f * 3 + d] = xf - cen[L * 3 + d];
      if (R >= 0) fdxR[f * 3 + d] = xf - sh - cen[R * 3 + d];
      dn += (xf - cen[L * 3 + d]) * n;
    }
    for (int d = 0; d < D; ++d) fmir[f * 3 + d] = 2.0 * dn * fnorm[f * 3 + d];
    auto add = [&](int64_t cell, int64_t nb, double s) {
      fail_if(nfc[cell] >= MAXF, "a cell has more than 8 faces");
      int p = nfc[cell]++;
      cface[cell * MAXF + p] = (int32_t)f;
      cnbr[cell * MAXF + p] = (int32_t)nb;
      csign[cell * MAXF + p] = s;
      for (int d = 0; d < D; ++d) closure[cell * 3 + d] += s * farea[f] * fnorm[f * 3 + d];
      asum[cell] += farea[f];
    };
    add(L, R, 1.0);
    if (R >= 0) add(R, L, -1.0);
  }
  for (int64_t i = 0; i < nc; ++i) {
    fail_if(nfc[i] < D + 1, "a cell has fewer than D+1 faces");
    double cl = 0.0;
    for (int d = 0; d < D; ++d) cl += closure[i * 3 + d] * closure[i * 3 + d];
    fail_if(std::sqrt(cl) > 1e-9 * asum[i], "a cell is not closed (sum S n != 0)");
  }
  // ---- least-squares coefficients --------------------------------------
  std::vector<double> lsG(nc * 3 * MAXF, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    double off[MAXF][3] = {{0}};
    for (int p = 0; p < nfc[i]; ++p) {
      int f = cface[i * MAXF + p];
      int j = cnbr[i * MAXF + p];
      for (int d = 0; d < D; ++d) {
        if (j >= 0) {
          // offset to the neighbour's centroid (periodic image for a shifted face)
          double sh = mesh->face_shift ? mesh->face_shift[f * D + d] : 0.0;
          double s = csign[i * MAXF + p];
          off[p][d] = cen[j * 3 + d] + s * sh - cen[i * 3 + d];
        } else {
          off[p][d] = fmir[f * 3 + d];
        }
      }
    }
    double N[9] = {0}, Ni[9];
    for (int p = 0; p < nfc[i]; ++p)
      for (int r = 0; r < D; ++r)
        for (int s = 0; s < D; ++s) N[r * 3 + s] += off[p][r] * off[p][s];
    fail_if(!chol_inverse(D, N, Ni), "degenerate least-squares stencil");
    for (int d = 0; d < D; ++d)
      for (int p = 0; p < nfc[i]; ++p) {
        double s = 0.0;
        for (int e = 0; e < D; ++e) s += Ni[d * 3 + e] * off[p][e];
        lsG[(i * 3 + d) * MAXF + p] = s;
      }
  }
  // first-order reconstruction: every gradient of the step, macroscopic and
  // microscopic, is zero (piecewise-constant states on both sides of each
  // face); the true coefficients are kept for the warm start's features
  std::vector<double> lsG_true;
  if (opt && (opt->flags & 16)) {
    lsG_true = lsG;
    std::fill(lsG.begin(), lsG.end(), 0.0);
  }
  // ---- velocity set -----------------------------------------------------
  const int64_t nvp = c->nvp;
  std::vector<double> u(3 * nvp, 0.0), w(nvp, 0.0), u2(nvp, 0.0);
  for (int64_t k = 0; k < nv; ++k) {
    fail_if(!(vel->w[k] > 0.0), "velocity weights must be positive");
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
      double x = vel->u[k * D + d];
      fail_if(!std::isfinite(x), "non-finite velocity");
      u[d * nvp + k] = x;
      s += x * x;
    }
    w[k] = vel->w[k];
    u2[k] = s;
  }
  // ---- fused-path eligibility ----------------------------------------------
  // A tensor product of one symmetric 1-D node set, first axis slowest, so
  // that point k and its mirror -u_k = u_{nv-1-k} are known by index.
  std::vector<double> ax;
  {
    std::vector<double> a0;
    for (int64_t k = 0; k < nv; ++k) a0.push_back(vel->u[k * D]);
    std::sort(a0.begin(), a0.end());
    a0.erase(std::unique(a0.begin(), a0.end()), a0.end());
    bool ok = !(c->flags & 2);
    const int64_t na = (int64_t)a0.size();
    int64_t prod = 1;
    for (int d = 0; d < D; ++d) prod *= na;
    ok = ok && prod == nv && na <= 64;
    for (int64_t n = 0; ok && n < na; ++n) ok = a0[na - 1 - n] == -a0[n];
    for (int64_t k = 0; ok && k < nv; ++k) {
      int64_t r = k;
      for (int d = D - 1; d >= 0 && ok; --d) {
        ok = vel->u[k * D + d] == a0[r % na];
        r /= na;
      }
    }
    bool mesh_ok = !(c->flags & 2);
    for (int64_t f = 0; mesh_ok && f < nf; ++f)
      mesh_ok = mesh->face_bc[f] >= UGKS_BC_INTERIOR && mesh->face_bc[f] <= UGKS_BC_OUTFLOW;
    for (int64_t i = 0; mesh_ok && i < nc; ++i) mesh_ok = nfc[i] <= 4;
    ok = ok && mesh_ok;
    if (ok) {
      ax = a0;
      c->fmesh.na = (int)na;
    } else if (mesh_ok) {
      // Sparse tensor set: every coordinate of every point is a node of one
      // 1-D set A = -A of at most 64 nodes (a locally refined set whose levels
      // are lattices is one), so the Maxwellians still factor over the axes.
      std::vector<double> aa;
      for (int64_t k = 0; k < nv * D; ++k) {
        aa.push_back(vel->u[k]);
        aa.push_back(-vel->u[k]);
      }
      std::sort(aa.begin(), aa.end());
      aa.erase(std::unique(aa.begin(), aa.end()), aa.end());
      if ((int64_t)aa.size() <= 64) {
        ax = aa;
        c->fmesh.na = (int)aa.size();
        c->fmesh.sparse = true;
        ok = true;
      }
    }
    c->fused = ok;
  }
  // ---- initial state check ---------------------------------------------
  for (int64_t i = 0; i < nc; ++i) {
    const double* Wi = &W0[i * (D + 2)];
    double rho = Wi[0], m2 = 0.0;
    for (int d = 0; d < D; ++d) m2 += Wi[1 + d] * Wi[1 + d];
    fail_if(!(rho > 0.0), "initial density must be positive");
    fail_if(!(Wi[D + 1] - 0.5 * m2 / rho > 0.0), "initial internal energy must be positive");
  }
  // ---- stream -------------------------------------------------------------
  if (opt && opt->stream) {
    c->stream = (hipStream_t)opt->stream;
    c->own_stream = false;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  // ---- device buffers ---------------------------------------------------
  DevMesh& m = c->mesh;
  m.nc = nc;
  m.nf = nf;
  m.vol = upload(c, vol);
  m.cen = upload(c, cen);
  m.nfc = upload(c, nfc);
  m.cface = upload(c, cface);
  m.cnbr = upload(c, cnbr);
  m.csign = upload(c, csign);
  m.lsG = upload(c, lsG);
  c->lsG_exact = lsG_true.empty() ? m.lsG : upload(c, lsG_true);
  m.fL = upload(c, fL);
  m.fR = upload(c, fR);
  m.fbc = upload(c, fbc);
  m.fbcid = upload(c, fbcid);
  m.farea = upload(c, farea);
  m.fnorm = upload(c, fnorm);
  m.fdxL = upload(c, fdxL);
  m.fdxR = upload(c, fdxR);
  m.fmir = upload(c, fmir);
  m.walls = upload(c, walls);
  m.nwall = (int64_t)walls.size();
  m.limiter = lim;
  if (lim) {
    std::vector<double> veps2(nc);
    for (int64_t i = 0; i < nc; ++i) veps2[i] = std::pow(limk * std::pow(vol[i], 1.0 / D), 3);
    m.veps2 = upload(c, veps2);
  }
  DevVel& v = c->vel;
  v.nv = nv;
  v.nvp = nvp;
  v.u = upload(c, u);
  v.w = upload(c, w);
  v.u2 = upload(c, u2);
  v.kxi = (double)c->kxi;
  v.has_b = c->nr == 2 ? 1 : 0;
  std::vector<DevBC> hb(std::max(n_bc, 1));
  for (int i = 0; i < n_bc; ++i) {
    hb[i].kind = bcs[i].kind;
    hb[i].rho = bcs[i].rho;
    for (int d = 0; d < 3; ++d) hb[i].U[d] = bcs[i].U[d];
    hb[i].T = bcs[i].T;
    fail_if(bcs[i].kind != UGKS_BC_OUTFLOW && !(bcs[i].T > 0.0), "boundary temperature must be positive");
  }
  c->bcs = upload(c, hb);
  // ---- time step (R5), and the local steps of reading R26 -------------------
  c->gas.Pr = gas->Pr;
  c->gas.R = gas->R;
  c->gas.Tref = gas->T_ref;
  c->gas.muref = gas->mu_ref;
  c->gas.omega = gas->omega;
  c->gas.K = (double)gas->K;
  const bool lts = (c->flags & 128) != 0;
  fail_if(lts && (c->flags & 64),
          "local time steps (flags bit 7) and boundary-flux tracking (bit 6) exclude each other");
  std::vector<double> dtc;
  {
    fail_if(!(gas->dt > 0.0) && !(gas->cfl > 0.0), "cfl must be positive when dt = 0");
    // each cell's bound 2 V_i / max_k sum_j S_j |u_k . n_j|
    std::vector<double> bound;
    double mn = INFINITY;
    if (!(gas->dt > 0.0) || lts) {
      double* cellv = dalloc<double>(c, nc);
      HIP_TRY(launch_dt_cells(D, m, v, cellv, c->stream));
      bound.resize(nc);
      HIP_TRY(hipMemcpyAsync(bound.data(), cellv, nc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      for (double x : bound) mn = std::min(mn, x);
      fail_if(!(mn > 0.0) || !std::isfinite(mn), "could not derive a time step");
    }
    c->gas.dt = gas->dt > 0.0 ? gas->dt : gas->cfl * mn;
    if (lts) {
      // cell i advances by dt b_i / min b (the most restrictive cell keeps dt)
      dtc.resize(nc);
      for (int64_t i = 0; i < nc; ++i) dtc[i] = c->gas.dt * (bound[i] / mn);
      c->gas.dtc = upload(c, dtc);
    }
  }
  if (c->fused) {
    // Static records of the fused sweep: the cell's faces, its least-squares
    // stencil and, per face, the neighbour's stencil, all wave-uniform.
    // Every cell is padded to the same shape (4 faces, 4-row stencils) so the
    // sweep runs one straight-line body:
    //   * a missing stencil row points at a real row with coefficient 0;
    //   * a wall face's "neighbour" rows point at the all-zero row nc (so the
    //     incoming free transport vanishes) and its equilibrium polynomial is
    //     the constant 1 (or K_xi/(2 lambda_w) for b), so the incoming flux
    //     is the re-emitted wall Maxwellian; the outgoing member's
    //     equilibrium term is switched off by the multiplier 0;
    //   * a far-field or outflow face's neighbour is a ghost row (rows
    //     nc+1 ... of h and b, refilled every step with the ghost Maxwellian)
    //     whose stencil is itself with coefficient 0, i.e. the ghost value
    //     with zero gradient; the ghost row also enters the least-squares
    //     stencil of the cell that owns the face, as its mirror-ghost row;
    //   * a missing face (cells with 3 faces) repeats face 0 with S/V = 0.
    const int32_t zero_row = (int32_t)nc;
    std::vector<int32_t> ghost_row(nf, -1), ffaces;
    for (int64_t f = 0; f < nf; ++f)
      if (fbc[f] == UGKS_BC_FARFIELD || fbc[f] == UGKS_BC_OUTFLOW) {
        ghost_row[f] = (int32_t)(nc + 1 + (int64_t)ffaces.size());
        ffaces.push_back((int32_t)f);
      }
    std::vector<int32_t> ci(nc * CRI, 0);
    std::vector<double> cdr(nc * CRD, 0.0);
    // Stencil slot p of a cell is its face p: the neighbour's row with the
    // least-squares coefficients of that face, the ghost row of a far-field
    // face, or the zero row with coefficient 0 at a wall (the wall ghost is the
    // cell's own value and adds nothing); slots past the cell's faces carry
    // the cell itself with coefficient 0.  So slot p of the cell's own stencil
    // is also the neighbour row read through face p.
    auto stencil = [&](int64_t cell, int32_t* cells, double* G /* [d*4 + s] */) {
      for (int p = 0; p < 4; ++p) {
        int32_t row = (int32_t)cell;
        bool coef = false;
        if (p < nfc[cell]) {
          const int f = cface[cell * MAXF + p];
          const int j = cnbr[cell * MAXF + p];
          if (j >= 0) {
            row = j;
            coef = true;
          } else if (ghost_row[f] >= 0) {
            row = ghost_row[f];
            coef = true;
          } else {
            row = zero_row;
          }
        }
        cells[p] = row;
        for (int d = 0; d < 3; ++d) G[d * 4 + p] = coef ? lsG[(cell * 3 + d) * MAXF + p] : 0.0;
      }
    };
    for (int64_t i = 0; i < nc; ++i) {
      int32_t* I = &ci[i * CRI];
      double* Dd = &cdr[i * CRD];
      I[0] = nfc[i];
      I[1] = 4;
      stencil(i, &I[2], Dd);
      for (int p = 0; p < 4; ++p) {
        const int pp = p < nfc[i] ? p : 0;
        int32_t* fi = &I[CRI_F0 + CRI_FS * p];
        double* fd = &Dd[CRD_F0 + CRD_FS * p];
        const int f = cface[i * MAXF + pp];
        const double sg = csign[i * MAXF + pp];
        const int j = cnbr[i * MAXF + pp];
        fi[0] = f;
        fi[1] = fbc[f];
        fi[2] = (p < nfc[i] && sg > 0.0) ? 1 : 0;
        const int32_t gr = ghost_row[f];
        fi[3] = j >= 0 ? j : (gr >= 0 ? gr : zero_row);
        fi[4] = 4;
        if (j >= 0) {
          // the neighbour's stencil with this cell's row (through the shared
          // face) moved to slot 0: the sweep reads that value from registers
          stencil(j, &fi[5], &fd[10]);
          int q = 0;
          for (int t = 0; t < nfc[j]; ++t)
            if (cface[j * MAXF + t] == f) q = t;
          if (q != 0) {
            std::swap(fi[5], fi[5 + q]);
            for (int d = 0; d < 3; ++d) std::swap(fd[10 + d * 4], fd[10 + d * 4 + q]);
          }
        } else {
          // zero or ghost row: its own value with zero gradient
          for (int r = 0; r < 4; ++r) {
            fi[5 + r] = fi[3];
            for (int d = 0; d < 3; ++d) fd[10 + d * 4 + r] = 0.0;
          }
        }
        for (int d = 0; d < 3; ++d) {
          fd[0 + d] = sg * fnorm[f * 3 + d];
          fd[4 + d] = sg > 0.0 ? fdxL[f * 3 + d] : fdxR[f * 3 + d];
          fd[7 + d] = j >= 0 ? (sg > 0.0 ? fdxR[f * 3 + d] : fdxL[f * 3 + d]) : 0.0;
        }
        fd[3] = p < nfc[i] ? farea[f] / vol[i] : 0.0;
        // local steps: the face's integral over dt, applied for dt_i
        if (lts && p < nfc[i]) fd[3] *= dtc[i] / c->gas.dt;
        // equilibrium term of the outgoing member: none at a wall
        fd[22] = (j >= 0 || gr >= 0) ? 1.0 : 0.0;
      }
    }
    std::vector<int32_t> vidx(nv);
    const int64_t na = c->fmesh.na;
    if (!c->fmesh.sparse) {
      for (int64_t k = 0; k < nv; ++k) {
        int64_t r = k;
        int32_t packed = 0;
        for (int d = D - 1; d >= 0; --d) {
          packed |= (int32_t)(r % na) << (8 * d);
          r /= na;
        }
        vidx[k] = packed;
      }
      c->fmesh.npairs = (nv + 1) / 2;
    } else {
      // node indices of every coordinate, then mirror pairs: point k with the
      // point at the mirrored indices, itself (u = 0), or a pad slot whose
      // weight is 0 and which is never stored (a "phantom" partner)
      std::map<std::vector<int32_t>, int64_t> at;
      std::vector<std::vector<int32_t>> ids(nv, std::vector<int32_t>(D));
      for (int64_t k = 0; k < nv; ++k) {
        int32_t packed = 0;
        for (int d = 0; d < D; ++d) {
          const double x = vel->u[k * D + d];
          const int32_t n = (int32_t)(std::lower_bound(ax.begin(), ax.end(), x) - ax.begin());
          ids[k][d] = n;
          packed |= n << (8 * d);
        }
        vidx[k] = packed;
        at[ids[k]] = k;
      }
      std::vector<int32_t> pairs, pvidx;
      std::vector<char> done(nv, 0);
      for (int64_t k = 0; k < nv; ++k) {
        if (done[k]) continue;
        std::vector<int32_t> m(D);
        for (int d = 0; d < D; ++d) m[d] = (int32_t)na - 1 - ids[k][d];
        auto it = at.find(m);
        int64_t k1 = (int64_t)nv;  // pad slot
        if (it != at.end() && !done[it->second]) k1 = it->second;
        done[k] = 1;
        if (k1 < nv) done[k1] = 1;
        pairs.push_back((int32_t)k);
        pairs.push_back((int32_t)k1);
        pvidx.push_back(vidx[k]);
      }
      c->fmesh.npairs = (int64_t)pvidx.size();
      c->fmesh.pairs = upload(c, pairs);
      c->fmesh.pvidx = upload(c, pvidx);
    }
    c->fmesh.nc = nc;
    c->fmesh.nv = nv;
    c->fmesh.axis = upload(c, ax);
    c->fmesh.vidx = upload(c, vidx);
    c->fmesh.crec_i = upload(c, ci);
    c->fmesh.crec_d = upload(c, cdr);
    if (prec == UGKS_FP32) c->fmesh.crec_d32 = upload(c, std::vector<float>(cdr.begin(), cdr.end()));
    if (lim) {
      // Limiter record (reading R7): what the sweep needs beyond the stencil
      // to limit the cell's gradient and each neighbour's.
      std::vector<double> lr(nc * CRL, 0.0);
      auto eps2_of = [&](int64_t cell) { return std::pow(limk * std::pow(vol[cell], 1.0 / D), 3); };
      auto wall_slot = [&](int64_t cell, int p) {
        if (p >= nfc[cell]) return false;
        return cnbr[cell * MAXF + p] < 0 && ghost_row[cface[cell * MAXF + p]] < 0;
      };
      for (int64_t i = 0; i < nc; ++i) {
        double* Lr = &lr[i * CRL];
        Lr[0] = eps2_of(i);
        for (int p = 0; p < 4; ++p) Lr[1 + p] = wall_slot(i, p) ? 1.0 : 0.0;
        for (int p = 0; p < 4 && p < nfc[i]; ++p) {
          const int f = cface[i * MAXF + p];
          const int j = cnbr[i * MAXF + p];
          if (j < 0) continue;  // wall or ghost: the incoming side has no gradient
          double* Fr = &Lr[CRL_F0 + CRL_FS * p];
          Fr[0] = eps2_of(j);
          // the neighbour's slots in record order: the shared face at slot 0
          int order[4] = {0, 1, 2, 3};
          for (int t = 0; t < nfc[j]; ++t)
            if (cface[j * MAXF + t] == f) std::swap(order[0], order[t]);
          for (int r = 0; r < 4; ++r) {
            const int t = order[r];
            Fr[1 + r] = wall_slot(j, t) ? 1.0 : 0.0;
            if (t >= nfc[j]) continue;
            const int fj = cface[j * MAXF + t];
            const bool left = csign[j * MAXF + t] > 0.0;
            for (int d = 0; d < 3; ++d) Fr[5 + 3 * r + d] = left ? fdxL[fj * 3 + d] : fdxR[fj * 3 + d];
          }
        }
      }
      c->fmesh.crec_l = upload(c, lr);
      if (prec == UGKS_FP32) c->fmesh.crec_l32 = upload(c, std::vector<float>(lr.begin(), lr.end()));
    }
    c->fmesh.nff = (int64_t)ffaces.size();
    c->fmesh.ffaces = upload(c, ffaces);
  }
  c->cell_perm = perm;
  c->face_perm.resize(nf);
  for (int64_t f = 0; f < nf; ++f) c->face_perm[f] = f;

  StepBuffers& B = c->buf;
  const size_t esz = prec == UGKS_FP32 ? sizeof(float) : sizeof(double);
  const int NW = D + 2;
  B.W = dalloc<double>(c, nc * NW);
  B.Wn = dalloc<double>(c, nc * NW);
  B.prim = dalloc<double>(c, nc * NPRIM);
  B.primn = dalloc<double>(c, nc * NPRIM);
  B.q = dalloc<double>(c, nc * 3);
  B.qn = dalloc<double>(c, nc * 3);
  B.gW = dalloc<double>(c, nc * 15);
  B.frec = dalloc<double>(c, nf * FREC);
  B.F = dalloc<double>(c, nf * 5);
  if (c->fused) {
    // velocity block: B_v velocities = B_v/2 mirror pairs per work item
    const int64_t npairs = c->fmesh.npairs;
    // (at least 32 pairs, or all: the batched form's smallest block, whose
    // per-block moment buffer below is sized from this)
    int64_t cp = Bv ? Bv / 2 : 2048;
    cp = std::max<int64_t>(std::min<int64_t>(32, npairs), std::min<int64_t>(cp, npairs));
    c->sched.nf = nf;
    c->sched.chunk_pairs = cp;
    c->sched.nchunk = (npairs + cp - 1) / cp;
    c->sched.tile = tile ? tile : 32;
    c->Bv = (int)(2 * cp);
    B.dW = dalloc<double>(c, nc * c->sched.nchunk * 5);
    B.tabs = dalloc<double>(c, (nf + nc) * (int64_t)D * c->fmesh.na);
    B.cs = dalloc<double>(c, nc * CSREC);
    B.csn = dalloc<double>(c, nc * CSREC);
    if (prec == UGKS_FP32) {
      B.frec32 = dalloc<float>(c, nf * FREC);
      B.cs32 = dalloc<float>(c, nc * CSREC);
      B.tabs32 = dalloc<float>(c, (nf + nc) * (int64_t)D * c->fmesh.na);
      // defined before the first step (the batched autotuner times the sweep on them)
      HIP_TRY(hipMemset(B.frec32, 0, nf * FREC * sizeof(float)));
      HIP_TRY(hipMemset(B.cs32, 0, nc * CSREC * sizeof(float)));
      HIP_TRY(hipMemset(B.tabs32, 0, (nf + nc) * (int64_t)D * c->fmesh.na * sizeof(float)));
    }
  } else {
    B.dW = dalloc<double>(c, nc * 5);
  }
  // row nc of h and b stays zero: the fused sweep's wall faces read it;
  // rows nc+1 ... are the fused sweep's far-field ghost rows
  const int64_t rows = nc + 1 + (c->fused ? c->fmesh.nff : 0);
  B.h = dalloc<char>(c, (size_t)rows * nvp * esz);
  B.ht = dalloc<char>(c, (size_t)nc * nvp * esz);
  B.b = c->nr == 2 ? (void*)dalloc<char>(c, (size_t)rows * nvp * esz) : nullptr;
  B.bt = c->nr == 2 ? (void*)dalloc<char>(c, (size_t)nc * nvp * esz) : nullptr;
  HIP_TRY(hipMemset(B.h, 0, (size_t)rows * nvp * esz));
  if (B.b) HIP_TRY(hipMemset(B.b, 0, (size_t)rows * nvp * esz));
  if (!c->fused) {
    // the staged sweep keeps every gradient and microscopic flux in HBM
    B.gradh = dalloc<double>(c, (size_t)nc * 3 * nvp);
    B.gradb = c->nr == 2 ? dalloc<double>(c, (size_t)nc * 3 * nvp) : nullptr;
    B.fluxh = dalloc<double>(c, (size_t)nf * nvp);
    B.fluxb = c->nr == 2 ? dalloc<double>(c, (size_t)nf * nvp) : nullptr;
  }
  B.resid = dalloc<double>(c, 8);
  B.cellred = dalloc<double>(c, nc * 3);
  B.flag = dalloc<int32_t>(c, 4);
  B.bflux = dalloc<double>(c, 5);
  HIP_TRY(hipMemsetAsync(B.frec, 0, nf * FREC * sizeof(double), c->stream));
  HIP_TRY(hipMemsetAsync(B.resid, 0, 8 * sizeof(double), c->stream));
  HIP_TRY(hipMemsetAsync(B.bflux, 0, 5 * sizeof(double), c->stream));
  HIP_TRY(hipMemsetAsync(B.flag, 0, 4 * sizeof(int32_t), c->stream));
  HIP_TRY(hipMemsetAsync(B.q, 0, nc * 3 * sizeof(double), c->stream));
  std::vector<double> W0p(nc * NW);
  for (int64_t i = 0; i < nc; ++i)
    for (int x = 0; x < NW; ++x) W0p[i * NW + x] = W0[perm[i] * NW + x];
  HIP_TRY(hipMemcpy(B.W, W0p.data(), nc * NW * sizeof(double), hipMemcpyHostToDevice));

  // ---- initial distributions: the reduced Maxwellian of W0 ---------------
  HIP_TRY(launch_prims(D, m, c->gas, B.W, B.prim, B.flag, 0, c->stream));
  HIP_TRY(launch_init_maxwellian(D, prec, m, v, B.prim, B.h, B.b, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
}

int set_err(ugks_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

// Kernel kinds timed by ugks_profile_enable.
enum KernelKind {
  KK_PRIMS, KK_HEATFLUX, KK_GRADW, KK_FACE_EQ, KK_WALL, KK_SWEEP, KK_STAGE1, KK_GRAD_MICRO,
  KK_FLUX, KK_MACRO, KK_STAGE2, KK_RESID, KK_COMMIT, KK_TABLES, KK_COUNT
};
const char* const kKernelNames[KK_COUNT] = {
    "cell_prims", "heat_flux", "macro_gradient", "face_equilibrium", "wall_density",
    "sweep", "stage1", "micro_gradient", "face_flux", "macro_update", "stage2", "residual",
    "commit", "maxwell_tables"};

hipEvent_t take_event(ugks_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_TRY(hipEventCreate(&e));
  return e;
}

// Records an event pair around one launch when profiling is on.
struct Timed {
  ugks_ctx* c;
  int kind;
  hipEvent_t a = nullptr;
  Timed(ugks_ctx* c_, int k) : c(c_), kind(k) {
    if (c->profiling) {
      a = take_event(c);
      HIP_TRY(hipEventRecord(a, c->stream));
    }
  }
  ~Timed() noexcept(false) {
    // no second record while a failed launch is unwinding
    if (c->profiling && a && std::uncaught_exceptions() == 0) {
      hipEvent_t b = take_event(c);
      HIP_TRY(hipEventRecord(b, c->stream));
      c->prof_events.push_back({kind, {a, b}});
    }
  }
};
#define TIMED(kind, call)        \
  do {                           \
    Timed _t(c, kind);           \
    HIP_TRY(call);               \
  } while (0)

// One time step of the fused path, enqueued.
void enqueue_step_fused(ugks_ctx* c) {
  const int D = c->D, P = c->prec;
  const DevMesh& m = c->mesh;
  const DevVel& v = c->vel;
  const GasP& g = c->gas;
  StepBuffers& B = c->buf;
  hipStream_t s = c->stream;
  // 2 heat flux of h^n: carried over from the previous second stage once valid
  if (!c->q_valid) {
    TIMED(KK_PRIMS, launch_prims(D, m, g, B.W, B.prim, B.flag, 1, s));
    TIMED(KK_HEATFLUX, launch_heatflux(D, P, m, v, B.h, B.b, B.prim, B.q, B.flag, s));
    c->q_valid = true;
  }
  // 1 primitives of W^n and the cell equilibrium data of the first stage
  TIMED(KK_PRIMS, launch_cell_prep(D, c->nc, g, B.W, B.q, B.prim, B.cs, B.flag, s));
  // 4 macroscopic reconstruction; 6.1-6.6 interface equilibrium
  TIMED(KK_GRADW, launch_gradW(D, m, c->bcs, g, B.W, B.gW, B.flag, s));
  TIMED(KK_FACE_EQ, launch_face_eq(D, m, c->bcs, g, B.W, B.gW, B.q, B.frec, B.flag, s));
  // 7 far-field ghost rows (the wall cells' stencils may read them), then
  // the wall densities
  if (c->fmesh.nff)
    TIMED(KK_WALL, launch_ghost_rows(D, P, c->fmesh, v, B.frec, B.h, B.b, B.flag, s));
  // (with boundary-flux tracking the wall pass also keeps each wall face's flux)
  const bool track = (c->flags & 64) != 0;
  TIMED(KK_WALL, launch_wall_rho_inline(D, P, m, v, c->fmesh, g, B.h, B.frec, B.flag, s, track ? 1 : 0,
                                        track ? (const void*)B.b : nullptr));
  if (track) TIMED(KK_RESID, launch_bflux(D, m, B.frec, B.F, 0, B.bflux, B.flag, s));
  // Maxwellian axis tables of every face and cell of this step
  TIMED(KK_TABLES, launch_tables(D, m, c->fmesh, g, B.frec, B.prim, B.cs, B.tabs, B.flag, s));
  // 5, 6.7-6.8, 9: the fused velocity sweep
  if (P == UGKS_FP32) {
    // the FP32 sweep reads FP32 copies of this step's records and tables
    TIMED(KK_TABLES, launch_to_f32(B.frec, B.frec32, c->nf * FREC, B.cs, B.cs32, c->nc * CSREC,
                                   B.tabs, B.tabs32, (c->nf + c->nc) * (int64_t)D * c->fmesh.na, s));
    TIMED(KK_SWEEP, launch_sweep(D, P, c->fmesh, v, g, c->sched, c->fmesh.crec_d32, c->fmesh.crec_l32, B.cs32,
                                 B.frec32, B.tabs32, B.h, B.b, B.ht, B.bt, B.dW, B.flag, s));
  } else {
    TIMED(KK_SWEEP, launch_sweep(D, P, c->fmesh, v, g, c->sched, c->fmesh.crec_d, c->fmesh.crec_l, B.cs, B.frec,
                                 B.tabs, B.h, B.b, B.ht, B.bt, B.dW, B.flag, s));
  }
  // 8 conservative update; 10 new equilibrium (with q^n, reading R17)
  TIMED(KK_MACRO, launch_apply_dW(D, m, c->sched.nchunk, B.W, B.dW, B.Wn, B.cellred, B.flag, s));
  TIMED(KK_PRIMS, launch_cell_prep(D, c->nc, g, B.Wn, B.q, B.primn, B.csn, B.flag, s));
  // 11 second stage and the heat flux of h^{n+1}
  TIMED(KK_STAGE2, launch_stage2_q(D, P, c->fmesh, v, B.primn, B.csn, B.ht, B.bt, B.h, B.b, B.qn,
                                    B.flag, s));
  std::swap(B.q, B.qn);
  if (!(c->flags & 1)) TIMED(KK_RESID, launch_residual(m, B.cellred, B.resid, B.flag, s));
  TIMED(KK_COMMIT, launch_commit_W(D, m, B.Wn, B.W, B.flag, s));
}

// One time step, enqueued (the one-step algorithm).
void enqueue_step(ugks_ctx* c) {
  if (c->fused) {
    enqueue_step_fused(c);
    return;
  }
  const int D = c->D, P = c->prec;
  const DevMesh& m = c->mesh;
  const DevVel& v = c->vel;
  const GasP& g = c->gas;
  StepBuffers& B = c->buf;
  hipStream_t s = c->stream;
  // 1-2 primitives and heat flux of the current state
  TIMED(KK_PRIMS, launch_prims(D, m, g, B.W, B.prim, B.flag, 1, s));
  TIMED(KK_HEATFLUX, launch_heatflux(D, P, m, v, B.h, B.b, B.prim, B.q, B.flag, s));
  // 3-4 ghost states and macroscopic reconstruction
  TIMED(KK_GRADW, launch_gradW(D, m, c->bcs, g, B.W, B.gW, B.flag, s));
  // 6.1-6.6 interface equilibrium data
  TIMED(KK_FACE_EQ, launch_face_eq(D, m, c->bcs, g, B.W, B.gW, B.q, B.frec, B.flag, s));
  // 5 microscopic reconstruction
  TIMED(KK_GRAD_MICRO, launch_grad_micro(D, P, m, v, B.frec, B.h, B.b, B.gradh, B.gradb, B.flag, s));
  // 7 wall densities
  TIMED(KK_WALL, launch_wall_rho(D, P, m, v, g, B.h, B.gradh, B.frec, B.flag, s));
  // 6.7-6.8 microscopic fluxes and their moments
  TIMED(KK_FLUX, launch_flux(D, P, m, v, g, B.frec, B.h, B.b, B.gradh, B.gradb, B.fluxh, B.fluxb,
                              B.F, B.flag, s));
  if (c->flags & 64) TIMED(KK_RESID, launch_bflux(D, m, B.frec, B.F, 1, B.bflux, B.flag, s));
  // 9 first stage
  TIMED(KK_STAGE1, launch_stage1(D, P, m, v, g, B.prim, B.q, B.h, B.b, B.fluxh, B.fluxb, B.ht,
                                B.bt, B.flag, s));
  // 8 conservative update, 10 new equilibrium
  TIMED(KK_MACRO, launch_macro_update(D, m, g, B.W, B.F, B.Wn, B.cellred, B.flag, s));
  TIMED(KK_PRIMS, launch_prims(D, m, g, B.Wn, B.primn, B.flag, 1, s));
  // 11 second stage
  TIMED(KK_STAGE2, launch_stage2(D, P, m, v, g, B.primn, B.q, B.ht, B.bt, B.h, B.b, B.flag, s));
  // 12 residual, commit W^{n+1}
  if (!(c->flags & 1)) TIMED(KK_RESID, launch_residual(m, B.cellred, B.resid, B.flag, s));
  TIMED(KK_COMMIT, launch_commit_W(D, m, B.Wn, B.W, B.flag, s));
}

}  // namespace

// ===========================================================================
// Batched form
// ===========================================================================
struct ugks_batch_impl;

namespace {

// Autotuner cache: case shape -> (velocity-block pairs, tile cells, time),
// batch shape list -> lanes per work-group.
struct TuneCase {
  int64_t chunk_pairs = 0, tile = 0;
  double us = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneCase> g_tune_case;
std::map<std::string, int> g_tune_batch;

std::string case_key(int D, int prec, int threads, int64_t nc, int64_t nv) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%d %d %d %lld %lld", D, prec, threads, (long long)nc, (long long)nv);
  return buf;
}

}  // namespace

struct ugks_batch {
  std::vector<ugks_ctx*> cases;
  int D = 0, prec = 64, flags = 0, nr = 1;
  int threads = 256;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void*> allocations;
  CaseDev* cases_dev[2] = {nullptr, nullptr};  // even / odd step: q and qn swapped
  int64_t* offs = nullptr;                    // cell, face, wall, tab, ghost offsets, [5][n+1]
  int32_t* items = nullptr;
  int64_t nitems = 0, grid = 0;
  int64_t ncell = 0, nface = 0, nwall = 0, ntab = 0, nff = 0;
  int32_t* flags_dev = nullptr;  // [4*n]
  double* resid_dev = nullptr;   // [8*n]
  int parity = 0;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  bool use_graph = true, tuned = false;
  int64_t tune_timings = 0, steps_done = 0;
  std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

template <typename T>
T* balloc(ugks_batch* b, size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
  b->allocations.push_back(p);
  return static_cast<T*>(p);
}

BatchDev batch_dev(const ugks_batch* b, int par) {
  BatchDev bd{};
  bd.cases = b->cases_dev[par];
  bd.n = (int32_t)b->cases.size();
  const int64_t n1 = bd.n + 1;
  bd.cell_off = b->offs;
  bd.face_off = b->offs + n1;
  bd.wall_off = b->offs + 2 * n1;
  bd.tab_off = b->offs + 3 * n1;
  bd.ff_off = b->offs + 4 * n1;
  bd.items = b->items;
  bd.nitems = b->nitems;
  return bd;
}

// Device case table of one parity from the sub-contexts' buffers.
void upload_cases(ugks_batch* b) {
  const size_t n = b->cases.size();
  for (int par = 0; par < 2; ++par) {
    std::vector<CaseDev> h(n);
    for (size_t i = 0; i < n; ++i) {
      const ugks_ctx* c = b->cases[i];
      CaseDev& d = h[i];
      d.m = c->mesh;
      d.v = c->vel;
      d.g = c->gas;
      d.fm = c->fmesh;
      d.sc = c->sched;
      d.bcs = c->bcs;
      d.B = c->buf;
      if (par) std::swap(d.B.q, d.B.qn);
    }
    if (!b->cases_dev[par]) b->cases_dev[par] = balloc<CaseDev>(b, n);
    HIP_TRY(hipMemcpy(b->cases_dev[par], h.data(), n * sizeof(CaseDev), hipMemcpyHostToDevice));
  }
}

// Work list of the batched sweep.  Tiles of each case go to the XCD queue
// with the least work so far; queue x holds the items of its tiles, velocity
// block by velocity block; queues are padded to one length and interleaved
// so that item w lands on a work-group with index = w (mod 8), i.e. on XCD w mod 8.
std::vector<int32_t> work_list(const ugks_batch* b, const std::vector<int64_t>& only) {
  std::vector<std::vector<int32_t>> q(8);
  std::vector<double> load(8, 0.0);
  auto add_case = [&](int64_t ci) {
    const ugks_ctx* c = b->cases[ci];
    const SweepSched& sc = c->sched;
    const int64_t ntile = (c->nc + sc.tile - 1) / sc.tile;
    for (int64_t t = 0; t < ntile; ++t) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      const int64_t c0 = t * sc.tile, c1 = std::min(c->nc, c0 + sc.tile);
      for (int64_t ch = 0; ch < sc.nchunk; ++ch)
        for (int64_t ic = c0; ic < c1; ++ic) {
          q[x].push_back((int32_t)ci);
          q[x].push_back((int32_t)ic);
          q[x].push_back((int32_t)ch);
          q[x].push_back(0);
        }
      load[x] += (double)(c1 - c0) * (double)((c->nv + 1) / 2);
    }
  };
  if (only.empty())
    for (int64_t ci = 0; ci < (int64_t)b->cases.size(); ++ci) add_case(ci);
  else
    for (int64_t ci : only) add_case(ci);
  size_t len = 0;
  for (auto& v : q) len = std::max(len, v.size() / 4);
  std::vector<int32_t> out(8 * len * 4, 0);
  for (size_t j = 0; j < len; ++j)
    for (int x = 0; x < 8; ++x) {
      int32_t* o = &out[(8 * j + x) * 4];
      if (j < q[x].size() / 4) std::memcpy(o, &q[x][4 * j], 4 * sizeof(int32_t));
      else o[0] = -1;
    }
  return out;
}

int64_t sweep_grid(const ugks_batch* b, int64_t nitems) {
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int per = std::max(1, sweep_b_blocks_per_cu(b->D, b->prec, b->threads));
  int64_t g = (int64_t)ncu * per;
  g = std::min<int64_t>(g, nitems);
  g = std::max<int64_t>(8, g / 8 * 8);
  return g;
}

void set_items(ugks_batch* b, const std::vector<int32_t>& items, int32_t** dst, int64_t* cap) {
  const int64_t n = (int64_t)items.size() / 4;
  if (n > *cap) {
    *dst = balloc<int32_t>(b, items.size());
    *cap = n;
  }
  HIP_TRY(hipMemcpy(*dst, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
}

// The phases of one step for every case of the batch.
void enqueue_batch_step(ugks_batch* b, int par) {
  const int D = b->D, P = b->prec;
  const BatchDev bd = batch_dev(b, par);
  hipStream_t s = b->stream;
  // 1 primitives of W^n and the first-stage cell data
  HIP_TRY(launch_cell_prep_b(D, bd, b->ncell, 0, s));
  // 4 macroscopic reconstruction; 6.1-6.6 interface equilibrium
  HIP_TRY(launch_gradW_b(D, bd, b->ncell, s));
  HIP_TRY(launch_face_eq_b(D, bd, b->nface, s));
  // 7 wall densities; far-field ghost rows
  HIP_TRY(launch_ghost_rows_b(D, P, bd, b->nff, s));
  HIP_TRY(launch_wall_rho_b(D, P, bd, b->nwall, s));
  // Maxwellian axis tables
  HIP_TRY(launch_tables_b(D, bd, b->ntab, s));
  // the FP32 form's sweep computes from FP32 copies of the step's records
  if (P == UGKS_FP32) HIP_TRY(launch_to_f32_b(bd, b->nface, b->ncell, b->ntab, s));
  // 5, 6.7-6.8, 9: the fused velocity sweep, one persistent launch
  HIP_TRY(launch_sweep_b(D, P, bd, b->grid, b->threads, s));
  // 8 conservative update; 10 new equilibrium
  HIP_TRY(launch_apply_dW_b(D, bd, b->ncell, s));
  HIP_TRY(launch_cell_prep_b(D, bd, b->ncell, 1, s));
  // 11 second stage with the heat flux of h^{n+1}
  HIP_TRY(launch_stage2_q_b(D, P, bd, b->ncell, s));
  // 12 residuals, commit W^{n+1}
  if (!(b->flags & 1)) HIP_TRY(launch_residual_b(bd, s));
  HIP_TRY(launch_commit_W_b(D, bd, b->ncell, s));
}

// Average duration of `reps` launches of the batched sweep over `items`.
double time_sweep(ugks_batch* b, const std::vector<int32_t>& items, int32_t** buf, int64_t* cap,
                  int reps) {
  upload_cases(b);  // the kernels read each case's schedule from the case table
  set_items(b, items, buf, cap);
  BatchDev bd = batch_dev(b, 0);
  bd.items = *buf;
  bd.nitems = (int64_t)items.size() / 4;
  const int64_t g = sweep_grid(b, bd.nitems);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(launch_sweep_b(b->D, b->prec, bd, g, b->threads, b->stream));  // warm-up
  HIP_TRY(hipEventRecord(e0, b->stream));
  for (int r = 0; r < reps; ++r) HIP_TRY(launch_sweep_b(b->D, b->prec, bd, g, b->threads, b->stream));
  HIP_TRY(hipEventRecord(e1, b->stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tune_timings += reps + 1;
  return 1e3 * ms / reps;
}

void apply_sched(ugks_ctx* c, int64_t chunk_pairs, int64_t tile) {
  const int64_t npairs = c->fmesh.npairs;
  // at least 32 pairs (or all): the per-block moment buffer was sized for that
  chunk_pairs = std::max(std::min<int64_t>(32, npairs), std::min(chunk_pairs, npairs));
  c->sched.chunk_pairs = chunk_pairs;
  c->sched.nchunk = (npairs + chunk_pairs - 1) / chunk_pairs;
  c->sched.tile = std::max<int64_t>(1, std::min(tile, c->nc));
  c->Bv = (int)(2 * chunk_pairs);
}

// Autotuner: for each lane count, each case's velocity block and tile by
// timing that case's sweep alone, then the lane count by timing the whole
// batch's sweep; shapes found in the cache are not timed again.
void autotune(ugks_batch* b) {
  const int64_t n = (int64_t)b->cases.size();
  int32_t* buf = nullptr;
  int64_t cap = 0;
  std::string bkey = "batch";
  for (ugks_ctx* c : b->cases) bkey += " " + case_key(b->D, b->prec, 0, c->nc, c->nv);
  int best_threads = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_batch.find(bkey);
    if (it != g_tune_batch.end()) best_threads = it->second;
  }
  const int cand_threads[3] = {64, 128, 256};
  double best_t = INFINITY;
  for (int th : cand_threads) {
    if (best_threads && th != best_threads) continue;
    b->threads = th;
    for (int64_t i = 0; i < n; ++i) {
      ugks_ctx* c = b->cases[i];
      const std::string key = case_key(b->D, b->prec, th, c->nc, c->nv);
      TuneCase tc;
      bool hit = false;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_case.find(key);
        if (it != g_tune_case.end()) {
          tc = it->second;
          hit = true;
        }
      }
      if (!hit) {
        const int64_t npairs = c->fmesh.npairs;
        tc.us = INFINITY;
        int64_t last_cp = -1;
        // velocity blocks from 64 velocities (half a wave of pairs) up to the whole set
        for (int mult2 : {1, 2, 4, 8, 16, 1 << 21}) {
          if (mult2 == 1 && th != 64) continue;
          const int64_t cp = std::min<int64_t>(npairs, (int64_t)mult2 * th / 2);
          if (cp == last_cp) continue;
          last_cp = cp;
          for (int64_t tile : {16, 64, 256}) {
            if (tile > 16 && tile / 4 >= c->nc) continue;
            apply_sched(c, cp, tile);
            const double us = time_sweep(b, work_list(b, {i}), &buf, &cap, 3);
            if (us < tc.us) tc = {c->sched.chunk_pairs, c->sched.tile, us};
          }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_case[key] = tc;
      }
      apply_sched(c, tc.chunk_pairs, tc.tile);
    }
    if (best_threads) break;  // cached lane count: schedules applied above
    const double t = time_sweep(b, work_list(b, {}), &buf, &cap, 3);
    if (t < best_t) {
      best_t = t;
      best_threads = th;
    }
  }
  if (b->threads != best_threads) {
    // re-apply the winning lane count's schedules (all cached by now)
    b->threads = best_threads;
    for (int64_t i = 0; i < n; ++i) {
      ugks_ctx* c = b->cases[i];
      std::lock_guard<std::mutex> lk(g_tune_mu);
      const TuneCase& tc = g_tune_case[case_key(b->D, b->prec, best_threads, c->nc, c->nv)];
      apply_sched(c, tc.chunk_pairs, tc.tile);
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_batch[bkey] = best_threads;
}

void batch_build(ugks_batch* b, const ugks_case* cases, int32_t n, const ugks_options* opt) {
  fail_if(!cases || n < 1, "need at least one case");
  const int prec = opt && opt->precision ? opt->precision : UGKS_FP64;
  fail_if(prec != UGKS_FP64 && prec != UGKS_FP32, "precision must be 64 or 32");
  const int fixed_bv = opt ? opt->block_v : 0, fixed_tile = opt ? opt->tile_cells : 0;
  fail_if(fixed_bv < 0 || fixed_bv % WAVE != 0, "block_v must be 0 or a positive multiple of 64");
  fail_if(fixed_tile < 0, "tile_cells must be >= 0");
  if (opt && (opt->flags & 128))
    throw std::pair<int, std::string>(UGKS_EUNSUPPORTED,
                                      "the batched form runs one global step (no local time steps)");
  for (int32_t i = 0; i < n; ++i)
    if (cases && cases[i].gas && cases[i].gas->K != 0)
      throw std::pair<int, std::string>(UGKS_EUNSUPPORTED, "case " + std::to_string(i) +
                                        ": the batched form takes monatomic gases (K = 0) only");
  if (opt && opt->limiter)
    throw std::pair<int, std::string>(UGKS_EUNSUPPORTED,
                                      "the batched sweep has no limiter");
  // every case's arguments, and one dimension for all, before any device work
  for (int32_t i = 0; i < n; ++i) {
    const ugks_case& k = cases[i];
    try {
      check_case_args(k.mesh, k.vel, k.gas, k.W0);
    } catch (InvalidArg& e) {
      throw InvalidArg{"case " + std::to_string(i) + ": " + e.msg};
    } catch (std::pair<int, std::string>& e) {
      throw std::pair<int, std::string>(e.first, "case " + std::to_string(i) + ": " + e.second);
    }
    fail_if(k.mesh->dim != cases[0].mesh->dim,
            "case " + std::to_string(i) + ": every case needs the same dimension");
  }
  b->prec = prec;
  b->flags = opt ? opt->flags : 0;
  b->use_graph = !(b->flags & 8);
  if (opt && opt->stream) {
    b->stream = (hipStream_t)opt->stream;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
  }
  b->flags_dev = balloc<int32_t>(b, 4 * (size_t)n);
  b->resid_dev = balloc<double>(b, 8 * (size_t)n);
  HIP_TRY(hipMemset(b->flags_dev, 0, 4 * (size_t)n * sizeof(int32_t)));
  HIP_TRY(hipMemset(b->resid_dev, 0, 8 * (size_t)n * sizeof(double)));
  for (int32_t i = 0; i < n; ++i) {
    const ugks_case& k = cases[i];
    ugks_options o{};
    o.precision = prec;
    o.block_v = 64;  // smallest velocity block: sizes the per-block moment buffer
    o.tile_cells = 0;
    o.flags = b->flags & ~(2 | 8);
    o.stream = b->stream;
    std::unique_ptr<ugks_ctx> c(new ugks_ctx());
    try {
      build(c.get(), k.mesh, k.vel, k.gas, k.bcs, k.n_bc, k.W0, &o);
    } catch (InvalidArg& e) {
      ugks_destroy(c.release());
      throw InvalidArg{"case " + std::to_string(i) + ": " + e.msg};
    } catch (std::pair<int, std::string>& e) {
      ugks_destroy(c.release());
      throw std::pair<int, std::string>(e.first, "case " + std::to_string(i) + ": " + e.second);
    } catch (...) {
      ugks_destroy(c.release());
      throw;
    }
    ugks_ctx* cc = c.release();
    b->cases.push_back(cc);
    if (i == 0) {
      b->D = cc->D;
      b->nr = cc->nr;
    }
    fail_if(cc->D != b->D, "case " + std::to_string(i) + ": every case needs the same dimension");
    if (!cc->fused || cc->fmesh.sparse)
      throw std::pair<int, std::string>(
          UGKS_EUNSUPPORTED, "case " + std::to_string(i) +
                                 ": the batched form needs the fused sweep over a full tensor "
                                 "product velocity set (symmetric nodes, at most 4 faces per cell)");
    // flags and residuals of all cases side by side: one copy reads them all
    cc->buf.flag = b->flags_dev + 4 * i;
    cc->buf.resid = b->resid_dev + 8 * i;
    // heat flux of the initial state
    HIP_TRY(launch_prims(cc->D, cc->mesh, cc->gas, cc->buf.W, cc->buf.prim, cc->buf.flag, 1, b->stream));
    HIP_TRY(launch_heatflux(cc->D, cc->prec, cc->mesh, cc->vel, cc->buf.h, cc->buf.b, cc->buf.prim,
                            cc->buf.q, cc->buf.flag, b->stream));
    cc->q_valid = true;
  }
  // case-offset tables
  const int64_t n1 = n + 1;
  std::vector<int64_t> off(5 * n1, 0);
  for (int32_t i = 0; i < n; ++i) {
    const ugks_ctx* c = b->cases[i];
    off[i + 1] = off[i] + c->nc;
    off[n1 + i + 1] = off[n1 + i] + c->nf;
    off[2 * n1 + i + 1] = off[2 * n1 + i] + c->mesh.nwall;
    off[3 * n1 + i + 1] = off[3 * n1 + i] + (c->nf + c->nc) * (int64_t)c->D * c->fmesh.na;
    off[4 * n1 + i + 1] = off[4 * n1 + i] + c->fmesh.nff;
  }
  b->ncell = off[n];
  b->nface = off[n1 + n];
  b->nwall = off[2 * n1 + n];
  b->ntab = off[3 * n1 + n];
  b->nff = off[4 * n1 + n];
  b->offs = balloc<int64_t>(b, off.size());
  HIP_TRY(hipMemcpy(b->offs, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  upload_cases(b);
  // the step's phases up to the sweep once, so the autotuner times the
  // sweep on this batch's own records
  {
    const BatchDev bd = batch_dev(b, 0);
    HIP_TRY(launch_cell_prep_b(b->D, bd, b->ncell, 0, b->stream));
    HIP_TRY(launch_gradW_b(b->D, bd, b->ncell, b->stream));
    HIP_TRY(launch_face_eq_b(b->D, bd, b->nface, b->stream));
    HIP_TRY(launch_ghost_rows_b(b->D, b->prec, bd, b->nff, b->stream));
    HIP_TRY(launch_wall_rho_b(b->D, b->prec, bd, b->nwall, b->stream));
    HIP_TRY(launch_tables_b(b->D, bd, b->ntab, b->stream));
  }
  if (fixed_bv || fixed_tile) {
    b->threads = 256;
    for (ugks_ctx* c : b->cases)
      apply_sched(c, fixed_bv ? fixed_bv / 2 : 2048, fixed_tile ? fixed_tile : 256);
  } else {
    autotune(b);
    b->tuned = true;
  }
  upload_cases(b);
  const std::vector<int32_t> items = work_list(b, {});
  int64_t cap = 0;
  set_items(b, items, &b->items, &cap);
  b->nitems = (int64_t)items.size() / 4;
  b->grid = sweep_grid(b, b->nitems);
  HIP_TRY(hipStreamSynchronize(b->stream));
  int32_t f0 = 0;
  std::vector<int32_t> fl(4 * (size_t)n);
  HIP_TRY(hipMemcpy(fl.data(), b->flags_dev, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t i = 0; i < n; ++i) f0 |= fl[4 * i];
  fail_if(f0 != 0, "non-positive density or temperature in an initial state");
  if (b->use_graph) {
    for (int par = 0; par < 2; ++par) {
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_batch_step(b, par);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIP_TRY(hipStreamEndCapture(b->stream, &b->graph[par]));
      HIP_TRY(hipGraphInstantiate(&b->exec[par], b->graph[par], nullptr, nullptr, 0));
    }
  }
}

int batch_err(ugks_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  else g_batch_create_error = msg;
  return code;
}

}  // namespace


extern "C" {

int ugks_create(const ugks_mesh* mesh, const ugks_velocity* vel, const ugks_gas* gas,
                const ugks_bc* bcs, int32_t n_bc, const double* W0, const ugks_options* opt,
                ugks_ctx** out) {
  if (!out) return set_err(nullptr, UGKS_EINVAL, "out is NULL");
  Range range("ugks_create");
  std::unique_ptr<ugks_ctx> c(new ugks_ctx());
  try {
    build(c.get(), mesh, vel, gas, bcs, n_bc, W0, opt);
  } catch (const InvalidArg& e) {
    ugks_destroy(c.release());
    return set_err(nullptr, UGKS_EINVAL, e.msg);
  } catch (const std::pair<int, std::string>& e) {
    ugks_destroy(c.release());
    return set_err(nullptr, e.first, e.second);
  } catch (const HipFail& e) {
    ugks_destroy(c.release());
    int code = (e.e == hipErrorOutOfMemory) ? UGKS_ENOMEM : UGKS_EHIP;
    return set_err(nullptr, code, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    ugks_destroy(c.release());
    return set_err(nullptr, UGKS_ENOMEM, "host memory allocation failed");
  } catch (...) {
    ugks_destroy(c.release());
    return set_err(nullptr, UGKS_EHIP, "internal error");
  }
  *out = c.release();
  return UGKS_OK;
}

namespace {

// Capture one step per order of the q / q^{n+1} buffers as HIP graphs.  The
// step records kernels only (no memset or copy), and two captures swap the
// buffers twice, so the context ends as it started.
void capture_step_graphs(ugks_ctx* c) {
  c->graph_q0 = c->buf.q;
  for (int par = 0; par < 2; ++par) {
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_step(c);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIP_TRY(hipStreamEndCapture(c->stream, &c->graph[par]));
    HIP_TRY(hipGraphInstantiate(&c->graph_exec[par], c->graph[par], nullptr, nullptr, 0));
  }
}

// One step: a graph replay where asked for (flags bit 5) and where one
// applies (not profiling, the heat flux of the current f known, a stream
// that can be captured), else the kernels one by one.  Both run the same
// kernels with the same arguments.
void run_step(ugks_ctx* c) {
  const bool graphs = (c->flags & 32) && !c->profiling && c->stream != nullptr;
  if (!graphs || !c->q_valid) {
    enqueue_step(c);
    return;
  }
  if (!c->graph_exec[0]) capture_step_graphs(c);
  const int par = c->buf.q == c->graph_q0 ? 0 : 1;
  HIP_TRY(hipGraphLaunch(c->graph_exec[par], c->stream));
  if (c->fused) std::swap(c->buf.q, c->buf.qn);  // as the fused step does on the host
}

}  // namespace

int ugks_step(ugks_ctx* c, int32_t n_steps, double* residual_out) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  if (n_steps < 0) return set_err(c, UGKS_EINVAL, "n_steps < 0");
  Range range("ugks_step");
  try {
    for (int32_t s = 0; s < n_steps; ++s) run_step(c);
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, c->buf.flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    double res[2] = {0.0, 0.0};
    if (residual_out)
      HIP_TRY(hipMemcpyAsync(res, c->buf.resid, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (flag) {
      // leave the flag set: the state is the last completed step and further
      // steps would repeat the failure
      return set_err(c, UGKS_ENUMERIC, "non-positive density or temperature (flag " +
                                           std::to_string(flag) + ")");
    }
    c->steps_done += n_steps;
    if (residual_out) {
      residual_out[0] = res[0];
      residual_out[1] = res[1];
    }
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_moments(ugks_ctx* c, int32_t which, double* out, int32_t on_device) {
  if (!c || !out) return set_err(c, UGKS_EINVAL, "null argument");
  const int D = c->D;
  try {
    int64_t ncol = which == 2 ? D : D + 2;
    std::vector<double> lib(c->nc * (which == 2 ? 3 : ncol));
    if (which == 0) {
      HIP_TRY(hipMemcpyAsync(lib.data(), c->buf.W, c->nc * ncol * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    } else if (which == 1) {
      double* tmp = c->buf.cellred;  // reuse: needs nc*(D+2) <= nc*3? no: use Wn scratch
      tmp = c->buf.Wn;
      HIP_TRY(launch_moments(D, c->prec, c->mesh, c->vel, c->buf.h, c->buf.b, tmp, c->stream));
      HIP_TRY(hipMemcpyAsync(lib.data(), tmp, c->nc * ncol * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    } else if (which == 2) {
      HIP_TRY(launch_prims(D, c->mesh, c->gas, c->buf.W, c->buf.prim, c->buf.flag, 0, c->stream));
      HIP_TRY(launch_heatflux(D, c->prec, c->mesh, c->vel, c->buf.h, c->buf.b, c->buf.prim, c->buf.qn,
                              c->buf.flag, c->stream));
      HIP_TRY(hipMemcpyAsync(lib.data(), c->buf.qn, c->nc * 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    } else {
      return set_err(c, UGKS_EINVAL, "which must be 0, 1 or 2");
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<double> user(c->nc * ncol);
    int64_t stride = which == 2 ? 3 : ncol;
    for (int64_t i = 0; i < c->nc; ++i)
      for (int64_t x = 0; x < ncol; ++x) user[c->cell_perm[i] * ncol + x] = lib[i * stride + x];
    if (on_device)
      HIP_TRY(hipMemcpy(out, user.data(), user.size() * sizeof(double), hipMemcpyHostToDevice));
    else
      std::memcpy(out, user.data(), user.size() * sizeof(double));
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}


int ugks_boundary_flux(ugks_ctx* c, double* out, int32_t* complete) {
  if (!c || !out) return set_err(c, UGKS_EINVAL, "null argument");
  if (!(c->flags & 64))
    return set_err(c, UGKS_EINVAL, "boundary-flux tracking is off (options.flags bit 6)");
  try {
    double acc[5];
    HIP_TRY(hipMemcpyAsync(acc, c->buf.bflux, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int x = 0; x < c->D + 2; ++x) out[x] = acc[x];
    if (complete) *complete = (!c->fused || c->fmesh.nff == 0) ? 1 : 0;
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_get_state(ugks_ctx* c, double* W, double* h, double* b) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  try {
    const int64_t nc = c->nc, nv = c->nv, nvp = c->nvp;
    if (W) {
      int rc = ugks_moments(c, 0, W, 0);
      if (rc) return rc;
    }
    void* src[2] = {c->buf.h, c->buf.b};
    double* dst[2] = {h, b};
    for (int r = 0; r < 2; ++r) {
      if (!dst[r]) continue;
      if (r == 1 && c->nr == 1) {
        std::fill(b, b + nc * nv, 0.0);
        continue;
      }
      if (c->prec == UGKS_FP32) {
        std::vector<float> tmp(nc * nvp);
        HIP_TRY(hipMemcpy(tmp.data(), src[r], tmp.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nc; ++i)
          for (int64_t k = 0; k < nv; ++k) dst[r][c->cell_perm[i] * nv + k] = tmp[i * nvp + k];
      } else {
        std::vector<double> tmp(nc * nvp);
        HIP_TRY(hipMemcpy(tmp.data(), src[r], tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nc; ++i)
          for (int64_t k = 0; k < nv; ++k) dst[r][c->cell_perm[i] * nv + k] = tmp[i * nvp + k];
      }
    }
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_set_state(ugks_ctx* c, const double* W, const double* h, const double* b) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  try {
    const int64_t nc = c->nc, nv = c->nv, nvp = c->nvp;
    const int NW = c->D + 2;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (W) {
      std::vector<double> lib(nc * NW);
      for (int64_t i = 0; i < nc; ++i)
        for (int x = 0; x < NW; ++x) lib[i * NW + x] = W[c->cell_perm[i] * NW + x];
      HIP_TRY(hipMemcpy(c->buf.W, lib.data(), lib.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    void* dst[2] = {c->buf.h, c->buf.b};
    const double* src[2] = {h, b};
    for (int r = 0; r < c->nr; ++r) {
      if (!src[r]) continue;
      if (c->prec == UGKS_FP32) {
        std::vector<float> tmp(nc * nvp, 0.0f);
        for (int64_t i = 0; i < nc; ++i)
          for (int64_t k = 0; k < nv; ++k) tmp[i * nvp + k] = (float)src[r][c->cell_perm[i] * nv + k];
        HIP_TRY(hipMemcpy(dst[r], tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice));
      } else {
        std::vector<double> tmp(nc * nvp, 0.0);
        for (int64_t i = 0; i < nc; ++i)
          for (int64_t k = 0; k < nv; ++k) tmp[i * nvp + k] = src[r][c->cell_perm[i] * nv + k];
        HIP_TRY(hipMemcpy(dst[r], tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
      }
    }
    // a new state restarts the residual normalisation and the boundary-flux
    // sum, and clears a failure
    HIP_TRY(hipMemset(c->buf.bflux, 0, 5 * sizeof(double)));
    c->q_valid = false;
    HIP_TRY(hipMemset(c->buf.resid, 0, 8 * sizeof(double)));
    HIP_TRY(hipMemset(c->buf.flag, 0, 4 * sizeof(int32_t)));
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_face_data(ugks_ctx* c, double* F, double* rho_w) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  try {
    const int64_t nf = c->nf;
    const int NW = c->D + 2;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (F) {
      std::vector<double> lib(nf * 5);
      HIP_TRY(hipMemcpy(lib.data(), c->buf.F, lib.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t f = 0; f < nf; ++f)
        for (int x = 0; x < NW; ++x) F[c->face_perm[f] * NW + x] = lib[f * 5 + x];
    }
    if (rho_w) {
      std::vector<double> lib(nf * FREC);
      HIP_TRY(hipMemcpy(lib.data(), c->buf.frec, lib.size() * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<int32_t> kind(nf);
      HIP_TRY(hipMemcpy(kind.data(), c->mesh.fbc, nf * sizeof(int32_t), hipMemcpyDeviceToHost));
      for (int64_t f = 0; f < nf; ++f)
        rho_w[c->face_perm[f]] = kind[f] == UGKS_BC_WALL ? lib[f * FREC + FR_RHOW] : 0.0;
    }
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_info(const ugks_ctx* c, ugks_info_t* out) {
  if (!c || !out) return UGKS_EINVAL;
  out->dim = c->D;
  out->n_r = c->nr;
  out->precision = c->prec;
  out->block_v = c->Bv;
  out->n_cells = c->nc;
  out->n_faces = c->nf;
  out->nv = c->nv;
  out->nv_padded = c->nvp;
  out->dt = c->gas.dt;
  out->steps_done = c->steps_done;
  out->device_bytes = c->bytes;
  out->fused = c->fused ? 1 : 0;
  out->tile_cells = c->fused ? (int32_t)c->sched.tile : 0;
  return UGKS_OK;
}

int ugks_profile_enable(ugks_ctx* c, int32_t on) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  try {
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& e : c->prof_events) {
      c->event_pool.push_back(e.second.first);
      c->event_pool.push_back(e.second.second);
    }
    c->prof_events.clear();
    c->profiling = on != 0;
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

int ugks_profile_read(ugks_ctx* c, ugks_kernel_time* out, int32_t max, int32_t* n_out) {
  if (!c) return set_err(nullptr, UGKS_EINVAL, "ctx is NULL");
  try {
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tot[KK_COUNT] = {0};
    int64_t cnt[KK_COUNT] = {0};
    for (auto& e : c->prof_events) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e.second.first, e.second.second));
      tot[e.first] += ms;
      cnt[e.first] += 1;
    }
    int n = 0;
    for (int k = 0; k < KK_COUNT; ++k) {
      if (!cnt[k]) continue;
      if (out && n < max) {
        std::memset(out[n].name, 0, sizeof(out[n].name));
        std::strncpy(out[n].name, kKernelNames[k], sizeof(out[n].name) - 1);
        out[n].launches = cnt[k];
        out[n].total_ms = tot[k];
      }
      ++n;
    }
    if (n_out) *n_out = n;
  } catch (const HipFail& e) {
    return set_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(set_err, c)
  return UGKS_OK;
}

void ugks_destroy(ugks_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int par = 0; par < 2; ++par) {
    if (c->graph_exec[par]) (void)hipGraphExecDestroy(c->graph_exec[par]);
    if (c->graph[par]) (void)hipGraphDestroy(c->graph[par]);
  }
  for (auto& e : c->prof_events) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  for (void* p : c->allocations) (void)hipFree(p);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* ugks_last_error(const ugks_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}


int ugks_batch_create(const ugks_case* cases, int32_t n_cases, const ugks_options* opt,
                      ugks_batch** out) {
  if (!out) return batch_err(nullptr, UGKS_EINVAL, "out is NULL");
  Range range("ugks_batch_create");
  std::unique_ptr<ugks_batch> b(new ugks_batch());
  try {
    batch_build(b.get(), cases, n_cases, opt);
  } catch (const InvalidArg& e) {
    ugks_batch_destroy(b.release());
    return batch_err(nullptr, UGKS_EINVAL, e.msg);
  } catch (const std::pair<int, std::string>& e) {
    ugks_batch_destroy(b.release());
    return batch_err(nullptr, e.first, e.second);
  } catch (const HipFail& e) {
    ugks_batch_destroy(b.release());
    int code = (e.e == hipErrorOutOfMemory) ? UGKS_ENOMEM : UGKS_EHIP;
    return batch_err(nullptr, code, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    ugks_batch_destroy(b.release());
    return batch_err(nullptr, UGKS_ENOMEM, "host memory allocation failed");
  } catch (...) {
    ugks_batch_destroy(b.release());
    return batch_err(nullptr, UGKS_EHIP, "internal error");
  }
  *out = b.release();
  return UGKS_OK;
}

int ugks_batch_step(ugks_batch* b, int32_t n_steps, double* residual_out) {
  if (!b) return batch_err(nullptr, UGKS_EINVAL, "batch is NULL");
  if (n_steps < 0) return batch_err(b, UGKS_EINVAL, "n_steps < 0");
  Range range("ugks_batch_step");
  const size_t n = b->cases.size();
  try {
    for (int32_t s = 0; s < n_steps; ++s) {
      if (b->use_graph) HIP_TRY(hipGraphLaunch(b->exec[b->parity], b->stream));
      else enqueue_batch_step(b, b->parity);
      b->parity ^= 1;
    }
    std::vector<int32_t> fl(4 * n);
    std::vector<double> rs(8 * n);
    HIP_TRY(hipMemcpyAsync(fl.data(), b->flags_dev, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(rs.data(), b->resid_dev, rs.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < n; ++i)
      if (fl[4 * i]) {
        return batch_err(b, UGKS_ENUMERIC, "case " + std::to_string(i) +
                                               ": non-positive density or temperature");
      }
    b->steps_done += n_steps;
    for (ugks_ctx* c : b->cases) c->steps_done += n_steps;
    if (residual_out)
      for (size_t i = 0; i < n; ++i) {
        residual_out[2 * i] = rs[8 * i];
        residual_out[2 * i + 1] = rs[8 * i + 1];
      }
  } catch (const HipFail& e) {
    return batch_err(b, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(batch_err, b)
  return UGKS_OK;
}

int ugks_batch_moments(ugks_batch* b, int32_t i, int32_t which, double* out, int32_t on_device) {
  if (!b) return batch_err(nullptr, UGKS_EINVAL, "batch is NULL");
  if (i < 0 || i >= (int32_t)b->cases.size()) return batch_err(b, UGKS_EINVAL, "case index out of range");
  ugks_ctx* c = b->cases[i];
  // the batch alternates q and qn by step parity; the case's own view is the
  // even one, so after an odd number of steps its scratch qn is the current q
  if (b->parity) std::swap(c->buf.q, c->buf.qn);
  int rc = ugks_moments(c, which, out, on_device);
  if (b->parity) std::swap(c->buf.q, c->buf.qn);
  if (rc) batch_err(b, rc, c->err);
  return rc;
}

int ugks_batch_get_state(ugks_batch* b, int32_t i, double* W, double* h, double* bb) {
  if (!b) return batch_err(nullptr, UGKS_EINVAL, "batch is NULL");
  if (i < 0 || i >= (int32_t)b->cases.size()) return batch_err(b, UGKS_EINVAL, "case index out of range");
  int rc = ugks_get_state(b->cases[i], W, h, bb);
  if (rc) batch_err(b, rc, b->cases[i]->err);
  return rc;
}

int ugks_batch_case_info(ugks_batch* b, int32_t i, ugks_info_t* out) {
  if (!b || !out) return UGKS_EINVAL;
  if (i < 0 || i >= (int32_t)b->cases.size()) return batch_err(b, UGKS_EINVAL, "case index out of range");
  return ugks_info(b->cases[i], out);
}

int ugks_batch_info(const ugks_batch* b, ugks_batch_info_t* out) {
  if (!b || !out) return UGKS_EINVAL;
  out->n_cases = (int32_t)b->cases.size();
  out->dim = b->D;
  out->precision = b->prec;
  out->threads = b->threads;
  out->work_items = b->nitems;
  out->grid = b->grid;
  out->graph = b->use_graph ? 1 : 0;
  out->tuned = b->tuned ? 1 : 0;
  out->tune_timings = b->tune_timings;
  out->steps_done = b->steps_done;
  return UGKS_OK;
}

void ugks_batch_destroy(ugks_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (int par = 0; par < 2; ++par) {
    if (b->exec[par]) (void)hipGraphExecDestroy(b->exec[par]);
    if (b->graph[par]) (void)hipGraphDestroy(b->graph[par]);
  }
  for (ugks_ctx* c : b->cases) ugks_destroy(c);
  for (void* p : b->allocations) (void)hipFree(p);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* ugks_batch_last_error(const ugks_batch* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int ugks_autotune_save(const char* path) {
  try {
    if (!path) return UGKS_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ofstream f(path);
    if (!f) return UGKS_EINVAL;
    f << "ugks-autotune 1\n";
    for (auto& e : g_tune_case)
      f << "case " << e.first << " : " << e.second.chunk_pairs << " " << e.second.tile << " "
        << e.second.us << "\n";
    for (auto& e : g_tune_batch) f << e.first << " : " << e.second << "\n";
    return f.good() ? UGKS_OK : UGKS_EINVAL;
  } catch (...) {
    return UGKS_EHIP;  // no exception crosses the ABI
  }
}

int ugks_autotune_load(const char* path) {
  try {
    if (!path) return UGKS_EINVAL;
    std::ifstream f(path);
    if (!f) return UGKS_EINVAL;
    std::string line;
    if (!std::getline(f, line) || line != "ugks-autotune 1") return UGKS_EINVAL;
    std::map<std::string, TuneCase> cs;
    std::map<std::string, int> bs;
    while (std::getline(f, line)) {
      if (line.empty()) continue;
      const size_t sep = line.find(" : ");
      if (sep == std::string::npos) return UGKS_EINVAL;
      const std::string key = line.substr(0, sep);
      std::istringstream val(line.substr(sep + 3));
      if (key.rfind("case ", 0) == 0) {
        TuneCase t;
        if (!(val >> t.chunk_pairs >> t.tile >> t.us) || t.chunk_pairs < 1 || t.tile < 1)
          return UGKS_EINVAL;
        cs[key.substr(5)] = t;
      } else if (key.rfind("batch", 0) == 0) {
        int th = 0;
        if (!(val >> th) || (th != 64 && th != 128 && th != 256)) return UGKS_EINVAL;
        bs[key] = th;
      } else {
        return UGKS_EINVAL;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : cs) g_tune_case[e.first] = e.second;
    for (auto& e : bs) g_tune_batch[e.first] = e.second;
    return UGKS_OK;
  } catch (...) {
    return UGKS_EHIP;  // no exception crosses the ABI
  }
}

void ugks_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_case.clear();
  g_tune_batch.clear();
}

}  // extern "C"
