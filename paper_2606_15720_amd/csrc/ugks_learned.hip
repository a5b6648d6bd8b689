// Learned warm start on gfx950: per-cell features, stress / heat-flux
// targets, a 9-64-64-9 tanh network (bf16 MFMA inference, FP32 training
// kernels with Adam) and the Grad-type initial distribution.
//
// The network closes the moment hierarchy the way a Chapman-Enskog
// expansion does (Sec. 2.1: the BGK-Shakhov relaxation toward H+, B+ carries
// the stress and heat flux of f); it maps dimensionless gradients of the
// macroscopic state to sigma/p and q/(p sqrt(2RT)), and the initial f is
// Grad's 13-moment form about the Maxwellian of W built from them.
//
// Inference is one wave per 16 cells on v_mfma_f32_16x16x16_bf16 in the
// transposed form Z^T = W Z_prev^T: a layer's 16x16 output tile (hidden
// units x cells) lands in exactly the register layout the next layer's B
// operand needs, so the three layers chain in registers without LDS.
#include "ugks_device.h"
#include "ugks_host_util.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

// Device memory of ugks_mlp_forward_noalloc: the padded input rows, then the
// padded output rows, of at most UGKS_NOALLOC_MAX_ROWS rows (8 MiB).  Each
// GPU holds its own copy until the process ends.  Host code never uses this
// name as an address: it takes the device address that hipGetSymbolAddress
// returns on each device.
static __device__ __align__(256) float scratch[2 * UGKS_NOALLOC_MAX_ROWS * 16];

namespace ugks {

using namespace dev;

namespace {

constexpr int NFEAT = 9, NOUT = 9, HID = 64;
constexpr int P_W1 = 0, P_B1 = P_W1 + HID * NFEAT, P_W2 = P_B1 + HID, P_B2 = P_W2 + HID * HID,
              P_W3 = P_B2 + HID, P_B3 = P_W3 + NOUT * HID, NPARAM = P_B3 + NOUT;
static_assert(NPARAM == 5385, "parameter layout");
constexpr int FS = 16;  // padded row of features and outputs (floats)

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// ---------------------------------------------------------------------------
// Features of every cell from W and its least-squares gradient gW
// (gW[(i*3 + d)*5 + v] = dW_v/dx_d), in FP64, stored as float rows of 16.
template <int D>
__global__ void k_features(int64_t nc, GasP g, const double* __restrict__ W,
                           const double* __restrict__ gW, float* __restrict__ feat) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double* Wi = &W[i * (D + 2)];
  double P[NPRIM];
  const bool ok = prim_of<D>(Wi, g, P);
  float* F = &feat[i * FS];
  for (int j = 0; j < FS; ++j) F[j] = 0.0f;
  if (!ok) {
    F[0] = NAN;  // outside every training box: the cell falls back to the Maxwellian
    return;
  }
  const double rho = P[0], tau = P[5], lam = P[4];
  const double RT = 0.5 / lam;
  const double E = Wi[D + 1] / rho;
  double dU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // dU[d][a] = dU_a/dx_d
  double dTT[3] = {0, 0, 0}, dr[3] = {0, 0, 0};
  for (int d = 0; d < D; ++d) {
    const double* G = &gW[(i * 3 + d) * 5];
    dr[d] = G[0];
    double UdU = 0.0;
    for (int a = 0; a < D; ++a) {
      dU[d][a] = (G[1 + a] - P[1 + a] * G[0]) / rho;
      UdU += P[1 + a] * dU[d][a];
    }
    const double dE = (G[D + 1] - E * G[0]) / rho;
    dTT[d] = (dE - UdU) / (1.5 * RT);
  }
  const double div = dU[0][0] + dU[1][1] + dU[2][2];
  const double L = tau * sqrt(2.0 * RT);
  F[0] = (float)(tau * (dU[0][0] - div / 3.0));
  F[1] = (float)(tau * (dU[1][1] - div / 3.0));
  F[2] = (float)(tau * 0.5 * (dU[0][1] + dU[1][0]));
  F[3] = (float)(tau * 0.5 * (dU[0][2] + dU[2][0]));
  F[4] = (float)(tau * 0.5 * (dU[1][2] + dU[2][1]));
  for (int d = 0; d < 3; ++d) F[5 + d] = (float)(L * dTT[d]);
  F[8] = (float)(L * sqrt(dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2]) / rho);
}

// Targets of every cell from its distribution: sigma/p (xx yy zz xy xz yz)
// and q/(p sqrt(2RT)), one work-group per cell, sums over velocity in a
// fixed order (wave shuffles, then waves in order).
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_targets(DevVel v, GasP g, const double* __restrict__ W,
                                                 const T* __restrict__ h, const T* __restrict__ b,
                                                 float* __restrict__ targ) {
  __shared__ double red[9 * 16];
  const int64_t i = blockIdx.x;
  double P[NPRIM];
  prim_of<D>(&W[i * (D + 2)], g, P);
  const double p = P[6], RT = 0.5 / P[4];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // Pxx Pyy Pzz Pxy Pxz Pyz qx qy qz
  for (int64_t k = threadIdx.x; k < v.nv; k += TPB) {
    double c[3] = {0, 0, 0};
    double c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      c[d] = v.u[d * v.nvp + k] - P[1 + d];
      c2 += c[d] * c[d];
    }
    const double wk = v.w[k];
    const double hk = wk * ld(h, i * v.nvp + k);
    const double bk = D == 2 ? wk * ld(b, i * v.nvp + k) : 0.0;
    acc[0] += c[0] * c[0] * hk;
    acc[1] += c[1] * c[1] * hk;
    acc[2] += D == 2 ? bk : c[2] * c[2] * hk;
    acc[3] += c[0] * c[1] * hk;
    acc[4] += c[0] * c[2] * hk;
    acc[5] += c[1] * c[2] * hk;
    const double e = c2 * hk + bk;
    for (int d = 0; d < 3; ++d) acc[6 + d] += 0.5 * c[d] * e;
  }
  block_sum<9>(acc, red);
  if (threadIdx.x == 0) {
    float* o = &targ[i * FS];
    for (int j = 0; j < FS; ++j) o[j] = 0.0f;
    for (int j = 0; j < 6; ++j) o[j] = (float)((acc[j] - (j < 3 ? p : 0.0)) / p);
    const double s = p * sqrt(2.0 * RT);
    for (int d = 0; d < 3; ++d) o[6 + d] = (float)(acc[6 + d] / s);
  }
}

// ---------------------------------------------------------------------------
// Network inference: y = out_scale * N(in_scale * x), N with bf16 weights and
// layer inputs, FP32 accumulation, FP32 biases and tanh.  One wave per tile
// of 16 rows; pb holds the weights as bf16, each matrix zero-padded to
// whole 16x16 tiles: W1 64x16, W2 64x64, W3 16x64.
struct MlpDev {
  const short* w1;     // [64*16]
  const short* w2;     // [64*64]
  const short* w3;     // [16*64]
  const float* p;      // FP32 parameters (biases read from here)
  const float* in_scale;
  const float* out_scale;
};

__global__ __launch_bounds__(256) void k_mlp_infer(MlpDev net, const float* __restrict__ x,
                                                   int64_t n, float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 15, grp = lane >> 4;  // A: row i = lane%16, k = 4*(lane/16)+e
  // weights of this lane, per 16x16 tile
  short4_t a1[4], a2[4][4], a3[4];
  for (int t = 0; t < 4; ++t)
    for (int e = 0; e < 4; ++e) a1[t][e] = net.w1[(16 * t + row) * 16 + 4 * grp + e];
  for (int t = 0; t < 4; ++t)
    for (int s = 0; s < 4; ++s)
      for (int e = 0; e < 4; ++e) a2[t][s][e] = net.w2[(16 * t + row) * 64 + 16 * s + 4 * grp + e];
  for (int s = 0; s < 4; ++s)
    for (int e = 0; e < 4; ++e) a3[s][e] = net.w3[row * 64 + 16 * s + 4 * grp + e];
  // biases in the output layout: D[unit = 4*(lane/16)+r][cell = lane%16]
  float4_t c1[4], c2[4], c3;
  for (int t = 0; t < 4; ++t)
    for (int r = 0; r < 4; ++r) {
      c1[t][r] = net.p[P_B1 + 16 * t + 4 * grp + r];
      c2[t][r] = net.p[P_B2 + 16 * t + 4 * grp + r];
    }
  for (int r = 0; r < 4; ++r) {
    const int u = 4 * grp + r;
    c3[r] = u < NOUT ? net.p[P_B3 + u] : 0.0f;
  }
  const int64_t ntile = (n + 15) / 16;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave; tile < ntile; tile += nwave) {
    const int64_t cell = tile * 16 + row;  // B operand / output column of this lane
    const bool live = cell < n;
    // B = X^T: features 4*grp .. 4*grp+3 of this lane's cell
    short4_t bx;
    for (int e = 0; e < 4; ++e) {
      const int f = 4 * grp + e;
      const float v = (live && f < NFEAT) ? x[cell * FS + f] * net.in_scale[f] : 0.0f;
      bx[e] = bf16_bits(v);
    }
    short4_t b2[4];
    for (int t = 0; t < 4; ++t) {
      float4_t z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[t], bx, c1[t], 0, 0, 0);
      for (int r = 0; r < 4; ++r) b2[t][r] = bf16_bits(tanhf(z[r]));
    }
    short4_t b3[4];
    for (int t = 0; t < 4; ++t) {
      float4_t z = c2[t];
      for (int s = 0; s < 4; ++s) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[t][s], b2[s], z, 0, 0, 0);
      for (int r = 0; r < 4; ++r) b3[t][r] = bf16_bits(tanhf(z[r]));
    }
    float4_t z = c3;
    for (int s = 0; s < 4; ++s) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3[s], b3[s], z, 0, 0, 0);
    if (live)
      for (int r = 0; r < 4; ++r) {
        const int u = 4 * grp + r;
        if (u < NOUT) y[cell * FS + u] = z[r] * net.out_scale[u];
      }
  }
}

// Staging rows of the allocation-free inference: the caller's rows of 9
// floats to padded rows of FS floats, and back.
__global__ void k_rows_in(const float* __restrict__ x, int64_t rows, float* __restrict__ xs) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * FS) return;
  const int64_t r = t / FS;
  const int j = (int)(t % FS);
  xs[t] = j < NFEAT ? x[r * NFEAT + j] : 0.0f;
}

__global__ void k_rows_out(const float* __restrict__ ys, int64_t rows, float* __restrict__ y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * NOUT) return;
  const int64_t r = t / NOUT;
  const int j = (int)(t % NOUT);
  y[t] = ys[r * FS + j];
}

// FP32 parameters -> the padded bf16 tiles of k_mlp_infer
__global__ void k_mlp_pack(const float* __restrict__ p, short* __restrict__ w1,
                           short* __restrict__ w2, short* __restrict__ w3) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 64 * 16) {
    const int j = t / 16, k = t % 16;
    w1[t] = k < NFEAT ? bf16_bits(p[P_W1 + j * NFEAT + k]) : (short)0;
  }
  if (t < 64 * 64) w2[t] = bf16_bits(p[P_W2 + t]);
  if (t < 16 * 64) {
    const int j = t / 64, k = t % 64;
    w3[t] = j < NOUT ? bf16_bits(p[P_W3 + j * HID + k]) : (short)0;
  }
}

// ---------------------------------------------------------------------------
// Training, FP32.  Per sample: forward, loss and the back-propagated layer
// errors; then per parameter the sum over samples (chunk partials, then the
// chunks in order), then Adam.
struct TrainWs {
  float* xs;    // [n*16] normalised inputs
  float* a1;    // [n*64]
  float* a2;    // [n*64]
  float* d1;    // [n*64] dL/dz1
  float* d2;    // [n*64] dL/dz2
  float* dy;    // [n*16] dL/dy
  float* loss;  // [n]
};

__global__ __launch_bounds__(256) void k_mlp_fb(const float* __restrict__ p,
                                                const float* __restrict__ in_scale,
                                                const float* __restrict__ out_scale,
                                                const float* __restrict__ x,
                                                const float* __restrict__ t, int64_t n,
                                                TrainWs ws) {
  __shared__ float sp[NPARAM];
  for (int j = threadIdx.x; j < NPARAM; j += blockDim.x) sp[j] = p[j];
  __syncthreads();
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  float xs[NFEAT];
  for (int k = 0; k < NFEAT; ++k) {
    xs[k] = x[s * FS + k] * in_scale[k];
    ws.xs[s * FS + k] = xs[k];
  }
  float a1[HID], a2[HID];
  for (int j = 0; j < HID; ++j) {
    float z = sp[P_B1 + j];
    for (int k = 0; k < NFEAT; ++k) z += sp[P_W1 + j * NFEAT + k] * xs[k];
    a1[j] = tanhf(z);
  }
  for (int j = 0; j < HID; ++j) {
    float z = sp[P_B2 + j];
    for (int k = 0; k < HID; ++k) z += sp[P_W2 + j * HID + k] * a1[k];
    a2[j] = tanhf(z);
  }
  const float inv_n = 1.0f / (float)n;
  float dy[NOUT];
  float loss = 0.0f;
  for (int j = 0; j < NOUT; ++j) {
    float y = sp[P_B3 + j];
    for (int k = 0; k < HID; ++k) y += sp[P_W3 + j * HID + k] * a2[k];
    const float r = y - t[s * FS + j] / out_scale[j];
    loss += r * r;
    dy[j] = 2.0f * r * inv_n;
    ws.dy[s * FS + j] = dy[j];
  }
  ws.loss[s] = loss;
  float d2[HID];
  for (int k = 0; k < HID; ++k) {
    float e = 0.0f;
    for (int j = 0; j < NOUT; ++j) e += sp[P_W3 + j * HID + k] * dy[j];
    d2[k] = e * (1.0f - a2[k] * a2[k]);
    ws.a2[s * HID + k] = a2[k];
    ws.d2[s * HID + k] = d2[k];
  }
  for (int k = 0; k < HID; ++k) {
    float e = 0.0f;
    for (int j = 0; j < HID; ++j) e += sp[P_W2 + j * HID + k] * d2[j];
    ws.a1[s * HID + k] = a1[k];
    ws.d1[s * HID + k] = e * (1.0f - a1[k] * a1[k]);
  }
}

// partial[c][j] = sum over samples of chunk c of the parameter-j gradient term
__global__ __launch_bounds__(256) void k_mlp_wgrad(TrainWs ws, int64_t n, int64_t chunk,
                                                   float* __restrict__ partial) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (j >= NPARAM) return;
  const int64_t s0 = c * chunk, s1 = min(n, s0 + chunk);
  float acc = 0.0f;
  if (j < P_B1) {
    const int u = j / NFEAT, k = j % NFEAT;
    for (int64_t s = s0; s < s1; ++s) acc += ws.d1[s * HID + u] * ws.xs[s * FS + k];
  } else if (j < P_W2) {
    const int u = j - P_B1;
    for (int64_t s = s0; s < s1; ++s) acc += ws.d1[s * HID + u];
  } else if (j < P_B2) {
    const int u = (j - P_W2) / HID, k = (j - P_W2) % HID;
    for (int64_t s = s0; s < s1; ++s) acc += ws.d2[s * HID + u] * ws.a1[s * HID + k];
  } else if (j < P_W3) {
    const int u = j - P_B2;
    for (int64_t s = s0; s < s1; ++s) acc += ws.d2[s * HID + u];
  } else if (j < P_B3) {
    const int u = (j - P_W3) / HID, k = (j - P_W3) % HID;
    for (int64_t s = s0; s < s1; ++s) acc += ws.dy[s * FS + u] * ws.a2[s * HID + k];
  } else {
    const int u = j - P_B3;
    for (int64_t s = s0; s < s1; ++s) acc += ws.dy[s * FS + u];
  }
  partial[c * NPARAM + j] = acc;
}

// gradient = chunk partials added in order; optional Adam update
__global__ __launch_bounds__(256) void k_mlp_adam(const float* __restrict__ partial, int64_t nchunk,
                                                  float* __restrict__ grad, float* __restrict__ p,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  int do_update, float lr, float beta1, float beta2,
                                                  float eps, float bc1, float bc2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NPARAM) return;
  float g = 0.0f;
  for (int64_t c = 0; c < nchunk; ++c) g += partial[c * NPARAM + j];
  grad[j] = g;
  if (!do_update) return;
  const float mj = beta1 * m[j] + (1.0f - beta1) * g;
  const float vj = beta2 * v[j] + (1.0f - beta2) * g * g;
  m[j] = mj;
  v[j] = vj;
  p[j] -= lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
}

// loss = sum over samples (fixed order: one block, strided, then the waves in order)
__global__ __launch_bounds__(1024) void k_mlp_loss(const float* __restrict__ loss, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[16];
  double acc[1] = {0.0};
  for (int64_t s = threadIdx.x; s < n; s += blockDim.x) acc[0] += loss[s];
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) *out = acc[0] / (double)n;
}

// ---------------------------------------------------------------------------
// Grad-type initial distribution (reduced over the internal dimension in
// 2-D), one work-group per cell; a cell whose features leave the training
// box (or are not finite) keeps the Maxwellian.
template <int D, typename T>
__global__ __launch_bounds__(TPB) void k_grad_init(DevVel v, GasP g, const double* __restrict__ W,
                                                   const float* __restrict__ feat,
                                                   const float* __restrict__ out,
                                                   const float* __restrict__ lo,
                                                   const float* __restrict__ hi, T* __restrict__ h,
                                                   T* __restrict__ b, int32_t* __restrict__ nfall) {
  const int64_t i = blockIdx.x;
  double P[NPRIM];
  prim_of<D>(&W[i * (D + 2)], g, P);
  bool use = true;
  for (int j = 0; j < NFEAT; ++j) {
    const float f = feat[i * FS + j];
    use = use && (f >= lo[j]) && (f <= hi[j]);  // false for NaN
  }
  for (int j = 0; j < NOUT; ++j) use = use && isfinite(out[i * FS + j]);
  double s[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, r[3] = {0, 0, 0};
  if (use) {
    const float* o = &out[i * FS];
    s[0][0] = o[0];
    s[1][1] = o[1];
    s[2][2] = o[2];
    s[0][1] = s[1][0] = o[3];
    s[0][2] = s[2][0] = o[4];
    s[1][2] = s[2][1] = o[5];
    const double tr = (s[0][0] + s[1][1] + s[2][2]) / 3.0;
    for (int a = 0; a < 3; ++a) s[a][a] -= tr;
    for (int d = 0; d < 3; ++d) r[d] = o[6 + d];
    if (D == 2) {
      s[0][2] = s[2][0] = s[1][2] = s[2][1] = 0.0;
      r[2] = 0.0;
    }
  } else if (threadIdx.x == 0) {
    atomicAdd(nfall, 1);
  }
  const double rho = P[0], lam = P[4];
  const double nrm = rho * maxw_norm<D>(lam);
  const double sq = 2.0 * sqrt(lam);
  for (int64_t k = threadIdx.x; k < v.nvp; k += TPB) {
    if (k >= v.nv) {
      st(h, i * v.nvp + k, 0.0);
      if (D == 2) st(b, i * v.nvp + k, 0.0);
      continue;
    }
    double c[3] = {0, 0, 0};
    double c2 = 0.0;
    for (int d = 0; d < D; ++d) {
      c[d] = v.u[d * v.nvp + k] - P[1 + d];
      c2 += c[d] * c[d];
    }
    double quad = 0.0, rc = 0.0;
    for (int a = 0; a < D; ++a) {
      rc += r[a] * c[a];
      for (int bb = 0; bb < D; ++bb) quad += s[a][bb] * c[a] * c[bb];
    }
    const double H = nrm * exp(-lam * c2);
    if (D == 3) {
      st(h, i * v.nvp + k, H * (1.0 + lam * quad + sq * rc * (0.4 * lam * c2 - 1.0)));
    } else {
      st(h, i * v.nvp + k, H * (1.0 + lam * quad + 0.5 * s[2][2] + sq * rc * (0.4 * lam * c2 - 0.8)));
      st(b, i * v.nvp + k,
         H / (2.0 * lam) * (1.0 + lam * quad + 1.5 * s[2][2] + sq * rc * (0.4 * lam * c2 - 0.4)));
    }
  }
}

}  // namespace
}  // namespace ugks

// ===========================================================================
// C ABI of the learned warm start
// ===========================================================================
using namespace ugks;
using namespace ugks::host;

struct ugks_mlp {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = -1;  // the device the network's memory lives on
  std::vector<void*> allocations;
  float* p = nullptr;  // FP32 parameters
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  short* w1 = nullptr;
  short* w2 = nullptr;
  short* w3 = nullptr;
  float* in_scale = nullptr;
  float* out_scale = nullptr;
  float* lo = nullptr;
  float* hi = nullptr;
  double* loss = nullptr;  // device scalar
  int64_t adam_steps = 0;
  // training workspace (grown on demand)
  int64_t ws_n = 0, ws_chunks = 0;
  TrainWs ws{};
  float* partial = nullptr;
  float* xdev = nullptr;
  float* tdev = nullptr;
  int64_t xcap = 0;
  std::string err;
};

namespace {

thread_local std::string g_mlp_create_error;

template <typename T>
T* malloc_into(std::vector<void*>& list, size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
  list.push_back(p);
  return static_cast<T*>(p);
}

int mlp_err(ugks_mlp* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  else g_mlp_create_error = msg;
  return code;
}

int ctx_err(ugks_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

MlpDev mlp_dev(const ugks_mlp* n) {
  MlpDev d;
  d.w1 = n->w1;
  d.w2 = n->w2;
  d.w3 = n->w3;
  d.p = n->p;
  d.in_scale = n->in_scale;
  d.out_scale = n->out_scale;
  return d;
}

void mlp_pack(ugks_mlp* n) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, n->stream, n->p, n->w1, n->w2, n->w3);
  HIP_TRY(hipGetLastError());
}

void mlp_infer(const ugks_mlp* n, const float* x, int64_t rows, float* y, hipStream_t s) {
  if (rows == 0) return;
  const int64_t tiles = (rows + 15) / 16;
  const int64_t blocks = std::min<int64_t>((tiles + 3) / 4, 4096);
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(256), 0, s, mlp_dev(n), x, rows, y);
  HIP_TRY(hipGetLastError());
}

// Device address of the file-scope scratch array on the current device,
// looked up once per device (every GPU holds its own copy of the array).
std::mutex g_scratch_mu;
float* g_scratch_dev[64] = {};

float* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[device] = static_cast<float*>(ptr);
  }
  return g_scratch_dev[device];
}

// Inputs as device rows of 16 floats: copy (and pad) from the caller's rows of 9.
float* stage_rows(ugks_mlp* n, const float* src, int64_t rows, int on_device, float** slot,
                  int64_t* cap) {
  if (rows > *cap) {
    *slot = malloc_into<float>(n->allocations, (size_t)rows * FS);
    *cap = rows;
  }
  HIP_TRY(hipMemset2DAsync(*slot, FS * sizeof(float), 0, FS * sizeof(float), rows, n->stream));
  HIP_TRY(hipMemcpy2DAsync(*slot, FS * sizeof(float), src, 9 * sizeof(float), 9 * sizeof(float), rows,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, n->stream));
  return *slot;
}

void grow_ws(ugks_mlp* n, int64_t rows, int64_t chunks) {
  if (rows > n->ws_n) {
    TrainWs& w = n->ws;
    w.xs = malloc_into<float>(n->allocations, rows * FS);
    w.a1 = malloc_into<float>(n->allocations, rows * HID);
    w.a2 = malloc_into<float>(n->allocations, rows * HID);
    w.d1 = malloc_into<float>(n->allocations, rows * HID);
    w.d2 = malloc_into<float>(n->allocations, rows * HID);
    w.dy = malloc_into<float>(n->allocations, rows * FS);
    w.loss = malloc_into<float>(n->allocations, rows);
    n->ws_n = rows;
  }
  if (chunks > n->ws_chunks) {
    n->partial = malloc_into<float>(n->allocations, (size_t)chunks * NPARAM);
    n->ws_chunks = chunks;
  }
}

constexpr int64_t kChunk = 256;  // samples per gradient partial

// gradient (and optionally one Adam step) of the mean squared error over rows
// [0, rows) of x, t (device rows of 16)
void mlp_grad_step(ugks_mlp* n, const float* x, const float* t, int64_t rows, bool update, float lr) {
  const int64_t chunks = (rows + kChunk - 1) / kChunk;
  grow_ws(n, rows, chunks);
  hipLaunchKernelGGL(k_mlp_fb, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, n->stream, n->p,
                     n->in_scale, n->out_scale, x, t, rows, n->ws);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((NPARAM + 255) / 256, (unsigned)chunks), dim3(256), 0,
                     n->stream, n->ws, rows, kChunk, n->partial);
  HIP_TRY(hipGetLastError());
  float bc1 = 1.0f, bc2 = 1.0f;
  if (update) {
    n->adam_steps += 1;
    bc1 = 1.0f - std::pow(0.9f, (float)n->adam_steps);
    bc2 = 1.0f - std::pow(0.999f, (float)n->adam_steps);
  }
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, n->stream, n->partial,
                     chunks, n->grad, n->p, n->m, n->v, update ? 1 : 0, lr, 0.9f, 0.999f, 1e-8f,
                     bc1, bc2);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(1024), 0, n->stream, n->ws.loss, rows, n->loss);
  HIP_TRY(hipGetLastError());
}

}  // namespace

extern "C" {

int ugks_mlp_create(const float* params, const float* in_scale, const float* out_scale, void* stream,
                    ugks_mlp** out) {
  if (!out || !params || !in_scale || !out_scale) return mlp_err(nullptr, UGKS_EINVAL, "null argument");
  for (int j = 0; j < NPARAM; ++j)
    if (!std::isfinite(params[j])) return mlp_err(nullptr, UGKS_EINVAL, "parameters must be finite");
  for (int j = 0; j < 9; ++j)
    if (!(in_scale[j] > 0.0f) || !(out_scale[j] > 0.0f) || !std::isfinite(in_scale[j]) ||
        !std::isfinite(out_scale[j]))
      return mlp_err(nullptr, UGKS_EINVAL, "scales must be positive and finite");
  std::unique_ptr<ugks_mlp> n(new ugks_mlp());
  try {
    HIP_TRY(hipGetDevice(&n->device));
    if (stream) {
      n->stream = (hipStream_t)stream;
    } else {
      HIP_TRY(hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking));
      n->own_stream = true;
    }
    auto& A = n->allocations;
    n->p = malloc_into<float>(A, NPARAM);
    n->m = malloc_into<float>(A, NPARAM);
    n->v = malloc_into<float>(A, NPARAM);
    n->grad = malloc_into<float>(A, NPARAM);
    n->w1 = malloc_into<short>(A, 64 * 16);
    n->w2 = malloc_into<short>(A, 64 * 64);
    n->w3 = malloc_into<short>(A, 16 * 64);
    n->in_scale = malloc_into<float>(A, 16);
    n->out_scale = malloc_into<float>(A, 16);
    n->lo = malloc_into<float>(A, 16);
    n->hi = malloc_into<float>(A, 16);
    n->loss = malloc_into<double>(A, 1);
    HIP_TRY(hipMemcpy(n->p, params, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(n->m, 0, NPARAM * sizeof(float)));
    HIP_TRY(hipMemset(n->v, 0, NPARAM * sizeof(float)));
    HIP_TRY(hipMemcpy(n->in_scale, in_scale, 9 * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(n->out_scale, out_scale, 9 * sizeof(float), hipMemcpyHostToDevice));
    // until a box is set every finite feature is inside it
    std::vector<float> lo(16, -INFINITY), hi(16, INFINITY);
    HIP_TRY(hipMemcpy(n->lo, lo.data(), 16 * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(n->hi, hi.data(), 16 * sizeof(float), hipMemcpyHostToDevice));
    mlp_pack(n.get());
    HIP_TRY(hipStreamSynchronize(n->stream));
  } catch (const HipFail& e) {
    ugks_mlp_destroy(n.release());
    return mlp_err(nullptr, e.e == hipErrorOutOfMemory ? UGKS_ENOMEM : UGKS_EHIP,
                   std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    ugks_mlp_destroy(n.release());
    return mlp_err(nullptr, UGKS_ENOMEM, "host memory allocation failed");
  } catch (...) {
    ugks_mlp_destroy(n.release());
    return mlp_err(nullptr, UGKS_EHIP, "internal error");
  }
  *out = n.release();
  return UGKS_OK;
}

int ugks_mlp_get_params(ugks_mlp* n, float* params) {
  if (!n || !params) return mlp_err(n, UGKS_EINVAL, "null argument");
  try {
    HIP_TRY(hipMemcpyAsync(params, n->p, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

int ugks_mlp_set_box(ugks_mlp* n, const float* lo, const float* hi) {
  if (!n || !lo || !hi) return mlp_err(n, UGKS_EINVAL, "null argument");
  for (int j = 0; j < 9; ++j)
    if (!(lo[j] <= hi[j])) return mlp_err(n, UGKS_EINVAL, "box bounds must satisfy lo <= hi");
  try {
    HIP_TRY(hipMemcpyAsync(n->lo, lo, 9 * sizeof(float), hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemcpyAsync(n->hi, hi, 9 * sizeof(float), hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

int ugks_mlp_forward(ugks_mlp* n, const float* x, int64_t rows, float* y, int32_t on_device) {
  if (!n || (rows > 0 && (!x || !y)) || rows < 0) return mlp_err(n, UGKS_EINVAL, "bad argument");
  try {
    float* xd = stage_rows(n, x, rows, on_device, &n->xdev, &n->xcap);
    float* yd = malloc_into<float>(n->allocations, (size_t)rows * FS);
    mlp_infer(n, xd, rows, yd, n->stream);
    HIP_TRY(hipMemcpy2DAsync(y, 9 * sizeof(float), yd, FS * sizeof(float), 9 * sizeof(float), rows,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    (void)hipFree(yd);
    n->allocations.pop_back();
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

int ugks_mlp_forward_noalloc(ugks_mlp* n, const float* x, int64_t rows, float* y) {
  static_assert(FS == 16, "scratch rows are 16 floats");
  if (!n) return mlp_err(n, UGKS_EINVAL, "null network");
  if (rows < 0 || rows > UGKS_NOALLOC_MAX_ROWS)
    return mlp_err(n, UGKS_EINVAL, "rows must be in [0, " + std::to_string(UGKS_NOALLOC_MAX_ROWS) +
                                       "] for the allocation-free inference");
  if (rows > 0 && (!x || !y)) return mlp_err(n, UGKS_EINVAL, "null input or output");
  if (rows == 0) return UGKS_OK;
  try {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != n->device || dev < 0 || dev >= 64)
      return mlp_err(n, UGKS_EINVAL, "the network's device must be the current device");
    float* xs = noalloc_scratch(dev);
    float* ys = xs + (size_t)UGKS_NOALLOC_MAX_ROWS * FS;
    const int64_t tin = rows * FS, tout = rows * NOUT;
    hipLaunchKernelGGL(k_rows_in, dim3((unsigned)((tin + 255) / 256)), dim3(256), 0, n->stream, x, rows, xs);
    HIP_TRY(hipGetLastError());
    mlp_infer(n, xs, rows, ys, n->stream);
    hipLaunchKernelGGL(k_rows_out, dim3((unsigned)((tout + 255) / 256)), dim3(256), 0, n->stream, ys, rows, y);
    HIP_TRY(hipGetLastError());
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

int ugks_mlp_loss_grad(ugks_mlp* n, const float* x, const float* t, int64_t rows, float* grad,
                       double* loss, int32_t on_device) {
  if (!n || !x || !t || rows <= 0) return mlp_err(n, UGKS_EINVAL, "bad argument");
  try {
    float* xd = stage_rows(n, x, rows, on_device, &n->xdev, &n->xcap);
    int64_t tcap = 0;
    float* td = nullptr;
    td = stage_rows(n, t, rows, on_device, &td, &tcap);
    mlp_grad_step(n, xd, td, rows, false, 0.0f);
    if (grad) HIP_TRY(hipMemcpyAsync(grad, n->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (loss) HIP_TRY(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    (void)hipFree(td);
    n->allocations.erase(std::find(n->allocations.begin(), n->allocations.end(), (void*)td));
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

int ugks_mlp_train(ugks_mlp* n, const float* x, const float* t, int64_t rows, int64_t batch,
                   int32_t steps, float lr, int32_t on_device, double* loss_out) {
  if (!n || !x || !t || rows <= 0 || batch <= 0 || steps < 0 || !(lr > 0.0f))
    return mlp_err(n, UGKS_EINVAL, "bad argument");
  Range range("ugks_mlp_train");
  try {
    float* xd = stage_rows(n, x, rows, on_device, &n->xdev, &n->xcap);
    int64_t tcap = 0;
    float* td = nullptr;
    td = stage_rows(n, t, rows, on_device, &td, &tcap);
    batch = std::min(batch, rows);
    std::vector<double> losses(steps);
    int64_t at = 0;
    for (int32_t k = 0; k < steps; ++k) {
      if (at + batch > rows) at = 0;  // consecutive slices of the caller's (shuffled) order
      mlp_grad_step(n, xd + at * FS, td + at * FS, batch, true, lr);
      if (loss_out) HIP_TRY(hipMemcpyAsync(&losses[k], n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
      at += batch;
    }
    mlp_pack(n);
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (loss_out) std::copy(losses.begin(), losses.end(), loss_out);
    (void)hipFree(td);
    n->allocations.erase(std::find(n->allocations.begin(), n->allocations.end(), (void*)td));
  } catch (const HipFail& e) {
    return mlp_err(n, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(mlp_err, n)
  return UGKS_OK;
}

void ugks_mlp_destroy(ugks_mlp* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (void* p : n->allocations) (void)hipFree(p);
  if (n->own_stream && n->stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

const char* ugks_mlp_last_error(const ugks_mlp* n) {
  return n ? n->err.c_str() : g_mlp_create_error.c_str();
}

int ugks_snapshot(ugks_ctx* c, float* feat, float* targ) {
  if (!c || (!feat && !targ)) return ctx_err(c, UGKS_EINVAL, "null argument");
  if (c->gas.K != 0.0)
    return ctx_err(c, UGKS_EUNSUPPORTED, "the learned closure is defined for monatomic gases (K = 0)");
  const int D = c->D;
  try {
    StepBuffers& B = c->buf;
    hipStream_t s = c->stream;
    const int64_t nc = c->nc;
    float* fd = dalloc<float>(c, (size_t)nc * FS);
    float* td = dalloc<float>(c, (size_t)nc * FS);
    HIP_TRY(launch_prims(D, c->mesh, c->gas, B.W, B.prim, B.flag, 0, s));
    DevMesh mg = c->mesh;
    mg.lsG = c->lsG_exact;  // features use the true gradient at any reconstruction order
    mg.limiter = 0;         // and unlimited
    HIP_TRY(launch_gradW(D, mg, c->bcs, c->gas, B.W, B.gW, B.flag, s));
    const unsigned g1 = (unsigned)((nc + 127) / 128);
    if (D == 2) hipLaunchKernelGGL(k_features<2>, dim3(g1), dim3(128), 0, s, nc, c->gas, B.W, B.gW, fd);
    else hipLaunchKernelGGL(k_features<3>, dim3(g1), dim3(128), 0, s, nc, c->gas, B.W, B.gW, fd);
    HIP_TRY(hipGetLastError());
    if (c->prec == UGKS_FP32) {
      if (D == 2) hipLaunchKernelGGL((k_targets<2, float>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, (const float*)B.h, (const float*)B.b, td);
      else hipLaunchKernelGGL((k_targets<3, float>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, (const float*)B.h, (const float*)B.b, td);
    } else {
      if (D == 2) hipLaunchKernelGGL((k_targets<2, double>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, (const double*)B.h, (const double*)B.b, td);
      else hipLaunchKernelGGL((k_targets<3, double>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, (const double*)B.h, (const double*)B.b, td);
    }
    HIP_TRY(hipGetLastError());
    std::vector<float> hf(nc * FS), ht(nc * FS);
    HIP_TRY(hipMemcpyAsync(hf.data(), fd, hf.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ht.data(), td, ht.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nc; ++i) {
      const int64_t u = c->cell_perm[i];
      for (int j = 0; j < 9; ++j) {
        if (feat) feat[u * 9 + j] = hf[i * FS + j];
        if (targ) targ[u * 9 + j] = ht[i * FS + j];
      }
    }
    // scratch: released now (the allocation list keeps the rest)
    for (float* p : {fd, td}) {
      (void)hipFree(p);
      c->allocations.erase(std::find(c->allocations.begin(), c->allocations.end(), (void*)p));
      c->bytes -= (int64_t)(nc * FS * sizeof(float));
    }
  } catch (const HipFail& e) {
    return ctx_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(ctx_err, c)
  return UGKS_OK;
}

int ugks_warm_start(ugks_ctx* c, const ugks_mlp* net, const double* W, int64_t* n_fallback) {
  if (!c || !net) return ctx_err(c, UGKS_EINVAL, "null argument");
  if (c->gas.K != 0.0)
    return ctx_err(c, UGKS_EUNSUPPORTED, "the learned closure is defined for monatomic gases (K = 0)");
  const int D = c->D;
  Range range("ugks_warm_start");
  try {
    StepBuffers& B = c->buf;
    hipStream_t s = c->stream;
    const int64_t nc = c->nc;
    if (W) {
      int rc = ugks_set_state(c, W, nullptr, nullptr);
      if (rc) return rc;
    }
    HIP_TRY(hipStreamSynchronize(net->stream));  // the network's last update is done
    float* fd = dalloc<float>(c, (size_t)nc * FS);
    float* od = dalloc<float>(c, (size_t)nc * FS);
    int32_t* cnt = dalloc<int32_t>(c, 1);
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t), s));
    HIP_TRY(launch_prims(D, c->mesh, c->gas, B.W, B.prim, B.flag, 0, s));
    DevMesh mg = c->mesh;
    mg.lsG = c->lsG_exact;  // features use the true gradient at any reconstruction order
    mg.limiter = 0;         // and unlimited
    HIP_TRY(launch_gradW(D, mg, c->bcs, c->gas, B.W, B.gW, B.flag, s));
    const unsigned g1 = (unsigned)((nc + 127) / 128);
    if (D == 2) hipLaunchKernelGGL(k_features<2>, dim3(g1), dim3(128), 0, s, nc, c->gas, B.W, B.gW, fd);
    else hipLaunchKernelGGL(k_features<3>, dim3(g1), dim3(128), 0, s, nc, c->gas, B.W, B.gW, fd);
    HIP_TRY(hipGetLastError());
    mlp_infer(net, fd, nc, od, s);
    if (c->prec == UGKS_FP32) {
      if (D == 2) hipLaunchKernelGGL((k_grad_init<2, float>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, fd, od, net->lo, net->hi, (float*)B.h, (float*)B.b, cnt);
      else hipLaunchKernelGGL((k_grad_init<3, float>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, fd, od, net->lo, net->hi, (float*)B.h, (float*)B.b, cnt);
    } else {
      if (D == 2) hipLaunchKernelGGL((k_grad_init<2, double>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, fd, od, net->lo, net->hi, (double*)B.h, (double*)B.b, cnt);
      else hipLaunchKernelGGL((k_grad_init<3, double>), dim3((unsigned)nc), dim3(TPB), 0, s, c->vel, c->gas, B.W, fd, od, net->lo, net->hi, (double*)B.h, (double*)B.b, cnt);
    }
    HIP_TRY(hipGetLastError());
    int32_t nf = 0;
    HIP_TRY(hipMemcpyAsync(&nf, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (n_fallback) *n_fallback = nf;
    c->q_valid = false;  // the next step takes the heat flux of the new f
    HIP_TRY(hipMemsetAsync(B.resid, 0, 8 * sizeof(double), s));  // residuals restart from here
    for (void* p : {(void*)fd, (void*)od, (void*)cnt}) {
      (void)hipFree(p);
      c->allocations.erase(std::find(c->allocations.begin(), c->allocations.end(), p));
    }
    c->bytes -= (int64_t)(2 * nc * FS * sizeof(float) + sizeof(int32_t));
  } catch (const HipFail& e) {
    return ctx_err(c, UGKS_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } UGKS_CATCH_REST(ctx_err, c)
  return UGKS_OK;
}

}  // extern "C"
