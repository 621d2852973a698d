// Learned warm start: scene features, the network's products on the matrix
// cores (BF16 x BF16 -> FP32, v_mfma_f32_16x16x32_bf16), loss, backward, Adam,
// and the moves between the solver state and the network's rows.
//
// Product kernel: 64 x 64 output tile per 256-thread workgroup, K in steps of
// 32. Both operand tiles are staged in LDS k-contiguous ([row][k] for A,
// [column][k] for B) so that every lane's MFMA operand is one 16-byte LDS read:
// lane l of a 16 x 16 x 32 product supplies A[row l % 16][k 8 (l / 16) .. + 7] and
// B[k 8 (l / 16) .. + 7][column l % 16]. A stored transposed (dW = X^T dY) or
// B stored untransposed (Y = X W) are transposed while being staged. Each wave
// computes a 32 x 32 quarter of the tile as 2 x 2 products.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>

#include "traj_internal.h"
#include "traj_mlp.h"

namespace traj {
int api_fail(int code, const char* fmt, ...);
}

namespace {

using traj::NC;
using traj::WAVE;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDK = BK + 8;  // LDS row stride (elements): 80 bytes, keeps 16-byte reads aligned
constexpr int GEMM_THREADS = 256;

__device__ __forceinline__ uint16_t f2bf(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);  // round to nearest even
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K;
  int lda, ldb;           // leading dimension of A and B as stored
  const float* bias;      // [N] or NULL
  int relu;
  float* C32;             // [M][N] or NULL
  uint16_t* C16;          // [M][N] BF16 copy of the result, or NULL
  const uint16_t* mask;   // [M][N] BF16: result *= (mask > 0) before C16 (gradient through ReLU)
};

template <bool TA, bool TB>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[BM * LDK];
  __shared__ __align__(16) uint16_t Bs[BN * LDK];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wr = w >> 1, wc = w & 1;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const uint4 zero = make_uint4(0, 0, 0, 0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // ---- stage A: As[m][k] = op(A)[m0 + m][k0 + k]
    if (!TA) {
      const int m = t >> 2, kc = (t & 3) * 8;
      uint4 v = zero;
      if (m0 + m < g.M && k0 + kc < g.K)
        v = *reinterpret_cast<const uint4*>(g.A + (size_t)(m0 + m) * g.lda + k0 + kc);
      *reinterpret_cast<uint4*>(As + m * LDK + kc) = v;
    } else {
      const int k = t >> 3, mc = (t & 7) * 8;
      uint4 v = zero;
      if (k0 + k < g.K && m0 + mc < g.M)
        v = *reinterpret_cast<const uint4*>(g.A + (size_t)(k0 + k) * g.lda + m0 + mc);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int i = 0; i < 8; ++i) As[(mc + i) * LDK + k] = e[i];
    }
    // ---- stage B: Bs[n][k] = op(B)[k0 + k][n0 + n]
    if (TB) {
      const int n = t >> 2, kc = (t & 3) * 8;
      uint4 v = zero;
      if (n0 + n < g.N && k0 + kc < g.K)
        v = *reinterpret_cast<const uint4*>(g.B + (size_t)(n0 + n) * g.ldb + k0 + kc);
      *reinterpret_cast<uint4*>(Bs + n * LDK + kc) = v;
    } else {
      const int k = t >> 3, nc = (t & 7) * 8;
      uint4 v = zero;
      if (k0 + k < g.K && n0 + nc < g.N)
        v = *reinterpret_cast<const uint4*>(g.B + (size_t)(k0 + k) * g.ldb + n0 + nc);
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[(nc + i) * LDK + k] = e[i];
    }
    __syncthreads();
    bf8 a[2], b[2];
    const int r = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf8*>(As + (wr * 32 + i * 16 + r) * LDK + kq);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf8*>(Bs + (wc * 32 + j * 16 + r) * LDK + kq);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // ---- epilogue: lane l holds rows 4 (l / 16) + r, column l % 16 of each product
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc * 32 + j * 16 + (lane & 15);
      if (col >= g.N) continue;
      const float bias = g.bias != nullptr ? g.bias[col] : 0.f;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = m0 + wr * 32 + i * 16 + 4 * (lane >> 4) + rr;
        if (row >= g.M) continue;
        float v = acc[i][j][rr] + bias;
        if (g.relu) v = fmaxf(v, 0.f);
        const size_t o = (size_t)row * g.N + col;
        if (g.mask != nullptr && !(bf2f(g.mask[o]) > 0.f)) v = 0.f;
        if (g.C32 != nullptr) g.C32[o] = v;
        if (g.C16 != nullptr) g.C16[o] = f2bf(v);
      }
    }
  }
}

hipError_t gemm(bool ta, bool tb, const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(GEMM_THREADS), 0, st, g);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(GEMM_THREADS), 0, st, g);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(GEMM_THREADS), 0, st, g);
  else hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(GEMM_THREADS), 0, st, g);
  return hipGetLastError();
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n, int cols, int ld_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = i / cols, c = i - r * cols;
  y[r * ld_out + c] = f2bf(x[i]);
}

// ---------------------------------------------------------------- features
// One wavefront per scene; lanes = obstacles (at most 64). The rank of obstacle j
// is the number of obstacles with a smaller (d2, index).
__global__ void k_features(const int32_t* __restrict__ obs_off, const float* __restrict__ ego,
                           const float* __restrict__ obs, int n_scenes, float* __restrict__ feat) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  if (s >= n_scenes) return;
  const float* e = ego + 8 * s;
  const int o0 = obs_off[s], m = obs_off[s + 1] - o0;
  float v = 0.f;  // feature `lane` of the scene
  if (o0 < 0 || m < 0 || m > 64) {
    v = __builtin_nanf("");
  } else {
    if (lane == 0) v = e[2] * (1.f / 30.f);
    float d2 = __builtin_inff();
    if (lane < m) {
      const float* o = obs + 4 * (o0 + lane);
      const float dx = o[0] - e[0], dy = o[1] - e[1];
      d2 = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
    }
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const float dj = __shfl(d2, j, 64);
      rank += (dj < d2) || (dj == d2 && j < lane);
    }
    // the obstacle of rank r fills features 1 + 4 r .. 4 + 4 r
    for (int r = 0; r < 10; ++r) {
      const unsigned long long b = __ballot(lane < m && rank == r);
      if (b == 0ull) break;
      const int j = __builtin_ctzll(b);
      const int comp = lane - 1 - 4 * r;
      if (comp >= 0 && comp < 4) {
        const float* o = obs + 4 * (o0 + j);
        v = comp < 2 ? (o[comp] - e[comp]) * 0.01f : (o[comp] - e[comp]) * (1.f / 30.f);
      }
    }
  }
  feat[(size_t)s * TRAJ_N_FEAT + lane] = v;
}

// ---------------------------------------------------------------- loss
// One workgroup per row: dy = bf16(2 (y - t) / n_total), row sum of (y - t)^2.
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ target, const float* __restrict__ mean,
                       const float* __restrict__ stdv, int n_out, float inv_total, uint16_t* __restrict__ dy,
                       float* __restrict__ row_loss) {
  __shared__ float part[256 / 64];
  const int r = blockIdx.x;
  float acc = 0.f;
  for (int c = threadIdx.x; c < n_out; c += blockDim.x) {
    const size_t o = (size_t)r * n_out + c;
    const float tn = (target[o] - mean[c]) / stdv[c];
    const float d = y[o] - tn;
    acc = fmaf(d, d, acc);
    dy[o] = f2bf(2.f * d * inv_total);
  }
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) row_loss[r] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ void k_loss_total(const float* __restrict__ row_loss, int rows, float inv_total, float* __restrict__ loss) {
  __shared__ double part[256 / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) acc += row_loss[i];
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = (float)(((part[0] + part[1]) + (part[2] + part[3])) * (double)inv_total);
}

// bias gradient: column sums (FP32, fixed order) of a BF16 matrix [rows][cols].
// A workgroup takes 64 columns; its 16 waves sum the rows r = slice (mod 16) of
// them (one 128-byte row segment per wave and load), and the 16 partial sums are
// added in slice order.
constexpr int COLSUM_SLICES = 16;
__global__ __launch_bounds__(WAVE * COLSUM_SLICES) void k_colsum_bf16(const uint16_t* __restrict__ x, int rows,
                                                                      int cols, float* __restrict__ out) {
  __shared__ float part[COLSUM_SLICES][WAVE];
  const int lane = threadIdx.x & (WAVE - 1), sl = threadIdx.x / WAVE;
  const int c = blockIdx.x * WAVE + lane;
  float acc = 0.f;
  if (c < cols)
    for (int r = sl; r < rows; r += COLSUM_SLICES) acc += bf2f(x[(size_t)r * cols + c]);
  part[sl][lane] = acc;
  __syncthreads();
  if (sl == 0 && c < cols) {
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < COLSUM_SLICES; ++i) sum += part[i][lane];
    out[c] = sum;
  }
}

__global__ void k_adam(float* __restrict__ p, uint16_t* __restrict__ pb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

__global__ void k_sync_bf16(const float* __restrict__ p, uint16_t* __restrict__ pb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

// Column mean and deviation (FP64 sums, fixed order): a workgroup takes 64
// columns; its 16 waves sum the rows r = slice (mod 16), and the partial sums are
// added in slice order, first for the mean, then for the squared deviations.
__global__ __launch_bounds__(WAVE * COLSUM_SLICES) void k_colstats(const float* __restrict__ rows, int n_rows,
                                                                   int n_cols, float* __restrict__ mean,
                                                                   float* __restrict__ stdv) {
  __shared__ double part[COLSUM_SLICES][WAVE];
  __shared__ double mu_s[WAVE];
  const int lane = threadIdx.x & (WAVE - 1), sl = threadIdx.x / WAVE;
  const int c = blockIdx.x * WAVE + lane;
  double s = 0.0;
  if (c < n_cols)
    for (int r = sl; r < n_rows; r += COLSUM_SLICES) s += rows[(size_t)r * n_cols + c];
  part[sl][lane] = s;
  __syncthreads();
  if (sl == 0) {
    double t = 0.0;
    for (int i = 0; i < COLSUM_SLICES; ++i) t += part[i][lane];
    mu_s[lane] = t / n_rows;
  }
  __syncthreads();
  const double mu = mu_s[lane];
  double q = 0.0;
  if (c < n_cols)
    for (int r = sl; r < n_rows; r += COLSUM_SLICES) {
      const double d = rows[(size_t)r * n_cols + c] - mu;
      q += d * d;
    }
  part[sl][lane] = q;  // every read of the first pass's sums came before the barrier above
  __syncthreads();
  if (sl == 0 && c < n_cols) {
    double t = 0.0;
    for (int i = 0; i < COLSUM_SLICES; ++i) t += part[i][lane];
    double sd = sqrt(t / n_rows);
    if (sd < 1e-5 * fmax(1.0, fabs(mu))) sd = 1.0;
    mean[c] = (float)mu;
    stdv[c] = (float)sd;
  }
}

// state <-> rows: thread per (scene, goal slot, value)
__global__ void k_state_rows(const int32_t* __restrict__ goal_off, const float* __restrict__ c,
                             const float* __restrict__ lam, int n_scenes, int n_goals, int gps,
                             float* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = 6 * NC * gps;
  if (i >= (int64_t)n_scenes * per) return;
  const int s = (int)(i / per), e = (int)(i - (int64_t)s * per);
  const int slot = e / (6 * NC), qk = e - slot * 6 * NC, qq = qk / NC, k = qk - qq * NC;
  const int g0 = goal_off[s];
  float v = __builtin_nanf("");
  if (goal_off[s + 1] - g0 == gps && g0 >= 0 && g0 + gps <= n_goals) {
    const float* src = qq < 3 ? c : lam;
    v = src[((size_t)(qq % 3) * NC + k) * n_goals + g0 + slot];
  }
  rows[i] = v;
}

__global__ void k_rows_state(const int32_t* __restrict__ goal_off, const float* __restrict__ y,
                             const float* __restrict__ mean, const float* __restrict__ stdv, int n_scenes,
                             int n_goals, int gps, float* __restrict__ c, float* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = 6 * NC * gps;
  if (i >= (int64_t)n_scenes * per) return;
  const int s = (int)(i / per), e = (int)(i - (int64_t)s * per);
  const int slot = e / (6 * NC), qk = e - slot * 6 * NC, qq = qk / NC, k = qk - qq * NC;
  const int g0 = goal_off[s];
  if (goal_off[s + 1] - g0 != gps || g0 < 0 || g0 + gps > n_goals) return;
  float* dst = qq < 3 ? c : lam;
  dst[((size_t)(qq % 3) * NC + k) * n_goals + g0 + slot] = fmaf(y[i], stdv[e], mean[e]);
}

int64_t param_count(const traj_mlp_dims& d) {
  int64_t n = 0;
  int fi = d.n_in;
  for (int l = 0; l <= d.n_layers; ++l) {
    const int fo = l < d.n_layers ? d.n_hidden : d.n_out;
    n += (int64_t)fi * fo + fo;
    fi = fo;
  }
  return n;
}

// offsets of W_l and b_l (l = 0 .. n_layers) in the packed array
void layer_offsets(const traj_mlp_dims& d, int l, int64_t& w, int64_t& b, int& fi, int& fo) {
  int64_t off = 0;
  int in = d.n_in;
  for (int i = 0;; ++i) {
    const int out = i < d.n_layers ? d.n_hidden : d.n_out;
    if (i == l) {
      w = off;
      b = off + (int64_t)in * out;
      fi = in;
      fo = out;
      return;
    }
    off += (int64_t)in * out + out;
    in = out;
  }
}

// element offset of the input of layer l (l = 0 .. n_layers) in the activation
// buffer: a0 [batch][n_in], then a1 .. a_L [batch][n_hidden]
int64_t act_offset(const traj_mlp_dims& d, int batch, int l) {
  return l == 0 ? 0 : (int64_t)batch * d.n_in + (int64_t)(l - 1) * batch * d.n_hidden;
}

bool dims_ok(const traj_mlp_dims* d) {
  return d != nullptr && d->n_in > 0 && d->n_hidden > 0 && d->n_out > 0 && d->n_in % 8 == 0 &&
         d->n_hidden % 8 == 0 && d->n_out % 8 == 0 && d->n_layers >= 1 && d->n_layers <= 8;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

extern "C" {

int traj_mlp_param_count(const traj_mlp_dims* dims, int64_t* count) {
  if (!dims_ok(dims) || count == nullptr) return traj::api_fail(TRAJ_E_INVAL, "bad network dimensions");
  *count = param_count(*dims);
  return TRAJ_OK;
}

int traj_mlp_sync_bf16(const traj_mlp* net, void* stream) {
  if (net == nullptr || !dims_ok(&net->dims) || !net->params || !net->params_bf16)
    return traj::api_fail(TRAJ_E_INVAL, "bad network");
  const int64_t n = param_count(net->dims);
  hipLaunchKernelGGL(k_sync_bf16, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, net->params,
                     net->params_bf16, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mlp_sync_bf16: %s", hipGetErrorString(e));
}

int traj_features(const traj_batch* batch, float* feat, void* stream) {
  if (batch == nullptr || feat == nullptr || batch->n_scenes < 0) return traj::api_fail(TRAJ_E_INVAL, "NULL argument");
  if (batch->n_scenes == 0) return TRAJ_OK;
  if (!batch->obs_off || !batch->ego || !batch->obs) return traj::api_fail(TRAJ_E_INVAL, "batch has NULL arrays");
  hipLaunchKernelGGL(k_features, dim3(batch->n_scenes), dim3(64), 0, (hipStream_t)stream, batch->obs_off, batch->ego,
                     batch->obs, batch->n_scenes, feat);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_features: %s", hipGetErrorString(e));
}

int traj_mlp_forward(const traj_mlp* net, const float* x, int batch, uint16_t* acts, float* y, void* stream) {
  if (net == nullptr || !dims_ok(&net->dims) || !net->params || !net->params_bf16 || !x || !acts || !y || batch < 0)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mlp_forward: bad arguments");
  if (batch == 0) return TRAJ_OK;
  const traj_mlp_dims& d = net->dims;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n0 = (int64_t)batch * d.n_in;
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n0, 256)), dim3(256), 0, st, x, acts, n0, d.n_in, d.n_in);
  hipError_t e = hipGetLastError();
  for (int l = 0; l <= d.n_layers && e == hipSuccess; ++l) {
    int64_t wo, bo;
    int fi, fo;
    layer_offsets(d, l, wo, bo, fi, fo);
    GemmArgs g = {};
    g.A = acts + act_offset(d, batch, l);
    g.lda = fi;
    g.B = net->params_bf16 + wo;
    g.ldb = fo;
    g.M = batch;
    g.N = fo;
    g.K = fi;
    g.bias = net->params + bo;
    if (l < d.n_layers) {
      g.relu = 1;
      g.C16 = acts + act_offset(d, batch, l + 1);
    } else {
      g.C32 = y;
    }
    e = gemm(false, false, g, st);
  }
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mlp_forward: %s", hipGetErrorString(e));
}

int traj_mlp_loss(const traj_mlp_dims* dims, const float* y, const float* target, const float* mean,
                  const float* stdv, int batch, uint16_t* dy, float* row_loss, float* loss, void* stream) {
  if (!dims_ok(dims) || !y || !target || !mean || !stdv || !dy || !row_loss || !loss || batch < 0)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mlp_loss: bad arguments");
  if (batch == 0) return TRAJ_OK;
  hipStream_t st = (hipStream_t)stream;
  const float inv_total = (float)(1.0 / ((double)batch * dims->n_out));
  hipLaunchKernelGGL(k_loss, dim3(batch), dim3(256), 0, st, y, target, mean, stdv, dims->n_out, inv_total, dy,
                     row_loss);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, st, row_loss, batch, inv_total, loss);
    e = hipGetLastError();
  }
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mlp_loss: %s", hipGetErrorString(e));
}

int traj_mlp_backward(const traj_mlp* net, const uint16_t* acts, const uint16_t* dy, int batch, uint16_t* work,
                      void* stream) {
  if (net == nullptr || !dims_ok(&net->dims) || !net->params_bf16 || !net->grad || !acts || !dy || !work ||
      batch < 0)
    return traj::api_fail(TRAJ_E_INVAL, "traj_mlp_backward: bad arguments");
  if (batch == 0) return TRAJ_OK;
  const traj_mlp_dims& d = net->dims;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const uint16_t* g = dy;  // gradient at the output of layer l (BF16, [batch][fo])
  for (int l = d.n_layers; l >= 0 && e == hipSuccess; --l) {
    int64_t wo, bo;
    int fi, fo;
    layer_offsets(d, l, wo, bo, fi, fo);
    // dW_l = a_l^T g   ([fi][fo], K = batch)
    GemmArgs gw = {};
    gw.A = acts + act_offset(d, batch, l);
    gw.lda = fi;
    gw.B = g;
    gw.ldb = fo;
    gw.M = fi;
    gw.N = fo;
    gw.K = batch;
    gw.C32 = net->grad + wo;
    e = gemm(true, false, gw, st);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_colsum_bf16, dim3(blocks_for(fo, WAVE)), dim3(WAVE * COLSUM_SLICES), 0, st, g, batch, fo,
                       net->grad + bo);
    e = hipGetLastError();
    if (e != hipSuccess || l == 0) break;
    // g_{l-1} = bf16((g W_l^T) * (a_l > 0))   ([batch][fi], K = fo)
    uint16_t* out = work + (size_t)(l & 1) * batch * d.n_hidden;
    GemmArgs gx = {};
    gx.A = g;
    gx.lda = fo;
    gx.B = net->params_bf16 + wo;
    gx.ldb = fo;
    gx.M = batch;
    gx.N = fi;
    gx.K = fo;
    gx.mask = acts + act_offset(d, batch, l);
    gx.C16 = out;
    e = gemm(false, true, gx, st);
    g = out;
  }
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mlp_backward: %s", hipGetErrorString(e));
}

int traj_mlp_adam(const traj_mlp* net, int step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (net == nullptr || !dims_ok(&net->dims) || !net->params || !net->params_bf16 || !net->grad || !net->adam_m ||
      !net->adam_v || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return traj::api_fail(TRAJ_E_INVAL, "traj_mlp_adam: bad arguments");
  const int64_t n = param_count(net->dims);
  const float c1 = (float)(1.0 - pow((double)beta1, step)), c2 = (float)(1.0 - pow((double)beta2, step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, net->params,
                     net->params_bf16, net->grad, net->adam_m, net->adam_v, n, lr, beta1, beta2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_mlp_adam: %s", hipGetErrorString(e));
}

int traj_colstats(const float* rows, int n_rows, int n_cols, float* mean, float* stdv, void* stream) {
  if (!rows || !mean || !stdv || n_rows < 1 || n_cols < 0) return traj::api_fail(TRAJ_E_INVAL, "traj_colstats: bad arguments");
  if (n_cols == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_colstats, dim3(blocks_for(n_cols, WAVE)), dim3(WAVE * COLSUM_SLICES), 0, (hipStream_t)stream,
                     rows, n_rows, n_cols, mean, stdv);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_colstats: %s", hipGetErrorString(e));
}

int traj_state_rows(const traj_batch* batch, const traj_state* state, int goals_per_scene, float* rows,
                    void* stream) {
  if (!batch || !state || !rows || goals_per_scene < 1 || batch->n_scenes < 0 || !state->c || !state->lam ||
      (batch->n_scenes > 0 && !batch->goal_off))
    return traj::api_fail(TRAJ_E_INVAL, "traj_state_rows: bad arguments");
  const int64_t n = (int64_t)batch->n_scenes * 6 * traj::NC * goals_per_scene;
  if (n == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_state_rows, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, batch->goal_off,
                     state->c, state->lam, batch->n_scenes, batch->n_goals, goals_per_scene, rows);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_state_rows: %s", hipGetErrorString(e));
}

int traj_rows_state(const traj_batch* batch, traj_state* state, int goals_per_scene, const float* y,
                    const float* mean, const float* stdv, void* stream) {
  if (!batch || !state || !y || !mean || !stdv || goals_per_scene < 1 || batch->n_scenes < 0 || !state->c ||
      !state->lam || (batch->n_scenes > 0 && !batch->goal_off))
    return traj::api_fail(TRAJ_E_INVAL, "traj_rows_state: bad arguments");
  const int64_t n = (int64_t)batch->n_scenes * 6 * traj::NC * goals_per_scene;
  if (n == 0) return TRAJ_OK;
  hipLaunchKernelGGL(k_rows_state, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, batch->goal_off, y,
                     mean, stdv, batch->n_scenes, batch->n_goals, goals_per_scene, state->c, state->lam);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_rows_state: %s", hipGetErrorString(e));
}

int traj_gemm_bf16(int ta, int tb, int M, int N, int K, const uint16_t* A, const uint16_t* B, const float* bias,
                   int relu, float* C, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 0 || M % 8 || N % 8 || K % 8)
    return traj::api_fail(TRAJ_E_INVAL, "traj_gemm_bf16: NULL operand or size not a multiple of 8");
  GemmArgs g = {};
  g.A = A;
  g.B = B;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = ta ? M : K;
  g.ldb = tb ? K : N;
  g.bias = bias;
  g.relu = relu;
  g.C32 = C;
  hipError_t e = gemm(ta != 0, tb != 0, g, (hipStream_t)stream);
  return e == hipSuccess ? TRAJ_OK : traj::api_fail(TRAJ_E_HIP, "traj_gemm_bf16: %s", hipGetErrorString(e));
}

}  // extern "C"
