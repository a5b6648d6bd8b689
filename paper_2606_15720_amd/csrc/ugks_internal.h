// Internal declarations of the gfx950 UGKS library: the context, device
// records and the kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ugks.h"

namespace ugks {

constexpr int MAXF = 8;    // faces per cell
constexpr int NPRIM = 8;   // rho, U[3], lambda, tau, p, spare
constexpr int FREC = 96;   // doubles per face record
constexpr int WAVE = 64;

// Face record layout (doubles).  Interior / far-field faces hold the
// interface equilibrium data; wall faces hold the wall Maxwellian data.
enum FaceRec : int {
  FR_C0 = 0,     // rho0 (lambda0/pi)^(D/2)   | wall: (lambda_w/pi)^(D/2)
  FR_LAM = 1,    // lambda0                    | wall: lambda_w
  FR_U = 2,      // U0[3]                      | wall: U_w[3]
  FR_SH = 5,     // 4 (1-Pr) lambda0^2 / (5 rho0)
  FR_Q = 6,      // q0[3]
  FR_G = 9,      // Gamma_1..5
  FR_A = 14,     // a[d][0..4], d < 3 (15)
  FR_AT = 29,    // A[0..4]
  FR_RHOW = 34,  // wall: rho_w (written by the wall pass)
  FR_GRHO = 35,  // ghost: rho_g, U_g[3], lambda_g (far field / outflow)
  FR_GU = 36,
  FR_GLAM = 39,
  FR_GC = 40,    // ghost: rho_g (lambda_g/pi)^(D/2)
  FR_PH = 48,    // cubic polynomial PH(u) of the h-equation equilibrium terms (20)
  FR_PB = 68,    // cubic polynomial PB(u) of the b-equation equilibrium terms (20, 2-D)
  FR_BF = 88,    // wall: the step's flux of mass, momentum, energy (boundary-flux tracking)
};

struct DevMesh {
  int64_t nc, nf;
  // cells
  const double* vol;        // [nc]
  const double* cen;        // [nc*3]
  const int32_t* nfc;       // [nc] faces per cell
  const int32_t* cface;     // [nc*MAXF] face ids
  const int32_t* cnbr;      // [nc*MAXF] neighbour cell, -1 for a boundary face
  const double* csign;      // [nc*MAXF] +1 if the cell is L of the face, -1 if R
  const double* lsG;        // [nc*3*MAXF] least-squares coefficients G[d][p]
  // faces
  const int32_t* fL;        // [nf]
  const int32_t* fR;        // [nf] (-1 boundary)
  const int32_t* fbc;       // [nf]
  const int32_t* fbcid;     // [nf]
  const double* farea;      // [nf]
  const double* fnorm;      // [nf*3]
  const double* fdxL;       // [nf*3] x_f - x_L
  const double* fdxR;       // [nf*3] x_f - shift - x_R
  const double* fmir;       // [nf*3] mirror ghost offset from L: 2((x_f-x_L).n) n
  const int32_t* walls;     // [nwall] ids of the wall faces
  int64_t nwall;
  int32_t limiter = 0;      // 1: Venkatakrishnan's limiter on every reconstruction gradient
  const double* veps2 = nullptr;  // [nc] its eps^2 = (K V^(1/D))^3
};

// Static per-cell records of the fused sweep (built once at create).
// Integer record (CRI ints per cell):
//   [0] faces, [1] own stencil size, [2..5] own stencil cells,
//   face p at CRI_F0 + CRI_FS p: [0] face id, [1] kind, [2] 1 if the cell is L,
//   [3] neighbour cell (-1 on a wall), [4] neighbour stencil size,
//   [5..8] neighbour stencil cells.
// Double record (CRD doubles per cell):
//   [d*4 + s] own least-squares coefficients G[d][s],
//   face p at CRD_F0 + CRD_FS p: [0..2] outward unit normal, [3] S/V,
//   [4..6] x_f - x_cell, [7..9] x_f - x_neighbour, [10 + d*4 + r] the
//   neighbour's coefficients G[d][r], [22] 1 (0 on a wall: the outgoing
//   member has no equilibrium term).
constexpr int CRI = 48, CRI_F0 = 6, CRI_FS = 10;
constexpr int CRD = 112, CRD_F0 = 12, CRD_FS = 24;
// Limiter record of the fused path (CRL doubles per cell, only with the
// limiter): [0] eps^2 of the cell, [1..4] 1 where own stencil slot s is a
// wall (its row is the zero row; its value for the bounds is the cell's own),
// then per face p at CRL_F0 + CRL_FS p: [0] eps^2 of the neighbour, [1..4]
// the neighbour's wall slots, [5 + 3 r + d] the offset of the neighbour's
// face in its stencil slot r from its centroid (slot order of the record).
constexpr int CRL = 88, CRL_F0 = 8, CRL_FS = 20;
// Per-cell, per-step record of the fused path (CSREC doubles per cell).
constexpr int CSREC = 48, CS_CC = 0, CS_KAP = 1, CS_NORM = 2, CS_SH = 4, CS_SB = 24;

struct FusedMesh {
  int64_t nc, nv;
  int na;                   // nodes per velocity axis
  const double* axis;       // [na] symmetric 1-D nodes
  const int32_t* vidx;      // [nv] packed axis indices of point k (8 bits per axis, first axis low)
  const int32_t* crec_i;    // [nc*CRI]
  const double* crec_d;     // [nc*CRD]
  const float* crec_d32;    // [nc*CRD] FP32 copy (FP32 compute form), else null
  bool sparse = false;      // points on the tensor product of `axis`, not all of it
  int64_t npairs = 0;       // mirror pairs of the sweep
  const int32_t* pairs = nullptr;  // sparse: [2*npairs] (k, mirror of k, or the pad slot nv)
  const int32_t* pvidx = nullptr;  // sparse: [npairs] packed axis indices of each pair's first point
  const double* crec_l = nullptr;  // [nc*CRL] limiter record, null without the limiter
  const float* crec_l32 = nullptr; // its FP32 copy (FP32 compute form)
  const int32_t* ffaces;    // [nff] far-field / outflow faces; face m owns ghost row nc+1+m
  int64_t nff;
};

// Schedule of the fused sweep: work item = (cell, velocity block of
// chunk_pairs mirror pairs); tiles of `tile` consecutive cells per XCD.
struct SweepSched {
  int64_t nf;             // face count (cell tables follow the face tables)
  int64_t tile;           // cells per tile
  int64_t nchunk;         // velocity blocks
  int64_t chunk_pairs;    // mirror pairs per velocity block
};

struct DevVel {
  int64_t nv, nvp;          // true and padded counts
  const double* u;          // [3*nvp] SoA: u[d*nvp + k]
  const double* w;          // [nvp]
  const double* u2;         // [nvp]
  // internal and out-of-plane dimensions of the full velocity space,
  // K_xi = K + 3 - D (Eq. Kxi_def); b is carried when K_xi > 0
  double kxi = 0.0;
  int32_t has_b = 0;
};

struct DevBC {
  int32_t kind;
  double rho, U[3], T;
};

struct GasP {
  double Pr, R, Tref, muref, omega, dt;
  double K = 0.0;  // internal degrees of freedom (0: monatomic)
  // local time steps (flags bit 7): per-cell steps dt_i [nc], or null for
  // the global dt everywhere.  Faces always integrate over the global dt.
  const double* dtc = nullptr;
};

// The step cell i advances by.
__host__ __device__ inline double dt_cell(const GasP& g, int64_t i) { return g.dtc ? g.dtc[i] : g.dt; }
// S_f as cell i applies it: times dt_i / dt under local steps
__host__ __device__ inline double area_for(const GasP& g, int64_t i, double S) {
  return g.dtc ? S * (g.dtc[i] / g.dt) : S;
}

// Kernel launchers (ugks_kernels.hip).  Each returns hipGetLastError().
struct StepBuffers {
  double* W;       // [nc*(D+2)] state W^n
  double* Wn;      // [nc*(D+2)] W^{n+1}
  double* prim;    // [nc*NPRIM] of W^n
  double* primn;   // [nc*NPRIM] of W^{n+1}
  double* q;       // [nc*3] heat flux of h^n
  double* qn;      // [nc*3] heat flux of h^{n+1} (fused path)
  double* gW;      // [nc*3*5]
  double* frec;    // [nf*FREC]
  double* F;       // [nf*5] face fluxes (staged sweep)
  double* dW;      // [nc*nchunk*5] per-(cell, velocity block) net outflow moments (fused sweep)
  double* tabs;    // [(nf+nc)*D*na] Maxwellian axis tables of the step (fused sweep)
  double* cs;      // [nc*CSREC] per-step cell record of W^n (fused sweep)
  double* csn;     // [nc*CSREC] per-step cell record of W^{n+1}
  float* frec32;   // FP32 copies of frec, cs, tabs for the FP32 sweep (null in FP64)
  float* cs32;
  float* tabs32;
  void* h;         // [nc*nvp] storage type
  void* b;         // [nc*nvp] (2-D only)
  void* ht;        // [nc*nvp] first-stage result
  void* bt;
  double* gradh;   // [nc*3*nvp] microscopic gradients (staged sweep)
  double* gradb;
  double* fluxh;   // [nf*nvp] time-integrated microscopic fluxes (staged sweep)
  double* fluxb;
  double* resid;   // [8] residual accumulators and state
  double* bflux;   // [5] running boundary flux (with boundary-flux tracking)
  double* cellred; // [nc*3] per-cell residual contributions
  int32_t* flag;   // numeric error flag
};

// One case of a batch as the batched kernels see it (an array of these in
// device memory; the pointers are the case's own buffers).
struct CaseDev {
  DevMesh m;
  DevVel v;
  GasP g;
  FusedMesh fm;
  SweepSched sc;
  const DevBC* bcs;
  StepBuffers B;
};

// A batch of cases run by one launch per phase: flattened element ranges
// with case-offset tables (prefix sums) and the sweep's work list.
struct BatchDev {
  const CaseDev* cases;     // [n]
  int32_t n;
  const int64_t* cell_off;  // [n+1] cells
  const int64_t* face_off;  // [n+1] faces
  const int64_t* wall_off;  // [n+1] wall faces
  const int64_t* tab_off;   // [n+1] Maxwellian axis-table entries, (nf+nc)*D*na
  const int64_t* ff_off;    // [n+1] far-field / outflow faces (ghost rows)
  const int32_t* items;     // [4*nitems] sweep work items: case (-1 = padding), cell, block, 0
  int64_t nitems;
};

hipError_t launch_prims(int D, const DevMesh& m, const GasP& g, const double* W, double* prim,
                        int32_t* flag, int checkflag, hipStream_t s);
hipError_t launch_heatflux(int D, int prec, const DevMesh& m, const DevVel& v, const void* h,
                           const void* b, const double* prim, double* q, const int32_t* flag,
                           hipStream_t s);
hipError_t launch_gradW(int D, const DevMesh& m, const DevBC* bcs, const GasP& g, const double* W,
                        double* gW, const int32_t* flag, hipStream_t s);
hipError_t launch_face_eq(int D, const DevMesh& m, const DevBC* bcs, const GasP& g,
                          const double* W, const double* gW, const double* q, double* frec,
                          int32_t* flag, hipStream_t s);
hipError_t launch_grad_micro(int D, int prec, const DevMesh& m, const DevVel& v,
                             const double* frec, const void* h, const void* b, double* gh,
                             double* gb, const int32_t* flag, hipStream_t s);
hipError_t launch_wall_rho(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                           const void* h, const double* gh, double* frec, const int32_t* flag,
                           hipStream_t s);
hipError_t launch_flux(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                       const double* frec, const void* h, const void* b, const double* gh,
                       const double* gb, double* fh, double* fb, double* F, const int32_t* flag,
                       hipStream_t s);
hipError_t launch_stage1(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                         const double* prim, const double* q, const void* h, const void* b,
                         const double* fh, const double* fb, void* ht, void* bt,
                         const int32_t* flag, hipStream_t s);
hipError_t launch_macro_update(int D, const DevMesh& m, const GasP& g, const double* W, const double* F,
                               double* Wn, double* cellred, const int32_t* flag, hipStream_t s);
hipError_t launch_stage2(int D, int prec, const DevMesh& m, const DevVel& v, const GasP& g,
                         const double* primn, const double* q, const void* ht, const void* bt,
                         void* h, void* b, const int32_t* flag, hipStream_t s);
hipError_t launch_residual(const DevMesh& m, const double* cellred, double* resid,
                           const int32_t* flag, hipStream_t s);
hipError_t launch_commit_W(int D, const DevMesh& m, const double* Wn, double* W,
                           const int32_t* flag, hipStream_t s);
hipError_t launch_init_maxwellian(int D, int prec, const DevMesh& m, const DevVel& v,
                                  const double* prim, void* h, void* b, hipStream_t s);
hipError_t launch_moments(int D, int prec, const DevMesh& m, const DevVel& v, const void* h,
                          const void* b, double* out, hipStream_t s);
hipError_t launch_dt_cells(int D, const DevMesh& m, const DevVel& v, double* cellval,
                           hipStream_t s);
// fused sweep (ugks_sweep.hip)
hipError_t launch_cell_prep(int D, int64_t nc, const GasP& g, const double* W, const double* q,
                            double* prim, double* cs, int32_t* flag, hipStream_t s);
// crec_d, cs, frec, tabs: FP64 records, or their FP32 copies when prec is FP32
hipError_t launch_sweep(int D, int prec, const FusedMesh& fm, const DevVel& v, const GasP& g,
                        const SweepSched& sc, const void* crec_d, const void* crec_l,
                        const void* cs, const void* frec,
                        const void* tabs, const void* h, const void* b, void* ht, void* bt,
                        double* dWp, const int32_t* flag, hipStream_t s);
hipError_t launch_to_f32(const double* a, float* fa, int64_t na, const double* b, float* fb,
                         int64_t nb, const double* c, float* fc, int64_t nc, hipStream_t s);
hipError_t launch_tables(int D, const DevMesh& m, const FusedMesh& fm, const GasP& g,
                         const double* frec, const double* prim, const double* cs, double* tabs,
                         const int32_t* flag, hipStream_t s);
hipError_t launch_apply_dW(int D, const DevMesh& m, int64_t nchunk, const double* W,
                          const double* dWp, double* Wn, double* cellred, const int32_t* flag,
                          hipStream_t s);
hipError_t launch_stage2_q(int D, int prec, const FusedMesh& fm, const DevVel& v,
                           const double* primn, const double* csn, const void* ht, const void* bt,
                           void* h, void* b, double* qn, const int32_t* flag, hipStream_t s);
hipError_t launch_wall_rho_inline(int D, int prec, const DevMesh& m, const DevVel& v,
                                  const FusedMesh& fm, const GasP& g, const void* h, double* frec,
                                  const int32_t* flag, hipStream_t s, int track = 0,
                                  const void* b_bf = nullptr);
hipError_t launch_bflux(int D, const DevMesh& m, const double* frec, const double* F, int staged,
                        double* acc, const int32_t* flag, hipStream_t s);
hipError_t launch_ghost_rows(int D, int prec, const FusedMesh& fm, const DevVel& v,
                             const double* frec, void* h, void* b, const int32_t* flag,
                             hipStream_t s);

// batched forms (one launch per phase over every case of a batch)
hipError_t launch_cell_prep_b(int D, const BatchDev& bd, int64_t ncell, int next, hipStream_t s);
hipError_t launch_gradW_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s);
hipError_t launch_face_eq_b(int D, const BatchDev& bd, int64_t nface, hipStream_t s);
hipError_t launch_wall_rho_b(int D, int prec, const BatchDev& bd, int64_t nwall, hipStream_t s);
hipError_t launch_to_f32_b(const BatchDev& bd, int64_t nface, int64_t ncell, int64_t ntab,
                           hipStream_t s);
hipError_t launch_tables_b(int D, const BatchDev& bd, int64_t ntab, hipStream_t s);
hipError_t launch_ghost_rows_b(int D, int prec, const BatchDev& bd, int64_t nff, hipStream_t s);
hipError_t launch_sweep_b(int D, int prec, const BatchDev& bd, int64_t grid, int threads,
                          hipStream_t s);
// resident work-groups of the batched sweep per CU at `threads` lanes
int sweep_b_blocks_per_cu(int D, int prec, int threads);
hipError_t launch_apply_dW_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s);
hipError_t launch_stage2_q_b(int D, int prec, const BatchDev& bd, int64_t ncell, hipStream_t s);
hipError_t launch_residual_b(const BatchDev& bd, hipStream_t s);
hipError_t launch_commit_W_b(int D, const BatchDev& bd, int64_t ncell, hipStream_t s);

}  // namespace ugks

struct ugks_ctx {
  int D = 0, kxi = 0, nr = 0, prec = 64, Bv = 64, flags = 0;
  bool fused = false;       // tensor-product symmetric velocity set, walls / interior only
  bool q_valid = false;     // buf.q holds the heat flux of the current h
  // HIP graphs of one step, one per order of the q / q^{n+1} buffers (the
  // step swaps them); graph_q0 is buf.q when graph 0 was captured
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  const double* graph_q0 = nullptr;
  ugks::FusedMesh fmesh{};  // static records of the fused sweep
  ugks::SweepSched sched{};
  int64_t nc = 0, nf = 0, nv = 0, nvp = 0;
  int64_t steps_done = 0;
  ugks::GasP gas{};
  std::vector<int64_t> cell_perm;   // library cell c -> caller cell
  std::vector<int64_t> face_perm;   // library face f -> caller face
  std::vector<int64_t> vel_perm;    // library velocity k -> caller velocity (k < nv)
  ugks::DevMesh mesh{};
  const double* lsG_exact = nullptr;  // least-squares coefficients even under first-order reconstruction
  ugks::DevVel vel{};
  ugks::DevBC* bcs = nullptr;
  ugks::StepBuffers buf{};
  std::vector<void*> allocations;
  int64_t bytes = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // kernel timing (ugks_profile_enable): event pairs per launch, in order
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_events;
  std::vector<hipEvent_t> event_pool;
  std::string err;
};
