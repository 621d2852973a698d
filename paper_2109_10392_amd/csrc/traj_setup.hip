// Operator setup: basis, Gram matrices and KKT inverses in FP64 on the GPU.
//
// Remark 1 of the paper: Q, F, F_o, P, P', P'' do not depend on the goal, so
// the KKT matrices of the x/y step (eq. 17) and heading step (eq. 19) are the
// same for the whole batch and are inverted once (eqs. 18, 20). F is block
// diagonal in (x, y) and so is A, hence eq. 17 splits exactly into one system
// per axis; each is formed and inverted here:
//   x, y:   [[Q + rho F_ax^T F_ax, A^T], [A, 0]],  F_ax^T F_ax = m P^T P + P''^T P'' + P'^T P'
//   psi:    [[Q + rho P^T P,       A^T], [A, 0]]
//   cold:   [[Q,                   A^T], [A, 0]]   (boundary-only minimum acceleration)
// with Q = P''^T P'' (the sum of squared accelerations, eq. 8a).
#include "traj_internal.h"

namespace traj {
namespace {

constexpr int SETUP_THREADS = 256;

__device__ double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Bernstein polynomial B_{deg,k}(tau); zero outside 0 <= k <= deg.
__device__ double bern(int deg, int k, double tau) {
  if (k < 0 || k > deg) return 0.0;
  double p = 1.0, q = 1.0;
  for (int i = 0; i < k; ++i) p *= tau;
  for (int i = 0; i < deg - k; ++i) q *= (1.0 - tau);
  return binom(deg, k) * p * q;
}

// In-place Gauss-Jordan inversion with partial pivoting of an nk x nk matrix
// stored as an augmented nk x 2nk array in shared memory.
__device__ void gauss_jordan(double* aug, int nk, double* fac, int* piv) {
  const int W = 2 * nk;
  const int tid = threadIdx.x;
  for (int col = 0; col < nk; ++col) {
    if (tid == 0) {
      int p = col;
      double best = fabs(aug[col * W + col]);
      for (int r = col + 1; r < nk; ++r) {
        double v = fabs(aug[r * W + col]);
        if (v > best) { best = v; p = r; }
      }
      *piv = p;
    }
    __syncthreads();
    const int p = *piv;
    if (p != col) {
      for (int j = tid; j < W; j += blockDim.x) {
        double t = aug[col * W + j];
        aug[col * W + j] = aug[p * W + j];
        aug[p * W + j] = t;
      }
    }
    __syncthreads();
    const double pivot = aug[col * W + col];
    __syncthreads();
    for (int j = tid; j < W; j += blockDim.x) aug[col * W + j] /= pivot;
    __syncthreads();
    for (int r = tid; r < nk; r += blockDim.x) fac[r] = aug[r * W + col];
    __syncthreads();
    for (int e = tid; e < nk * W; e += blockDim.x) {
      int r = e / W, j = e % W;
      if (r != col) aug[e] -= fac[r] * aug[col * W + j];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(SETUP_THREADS) void k_setup(const ShapeDesc* shapes, SolverConst kc, float* tables,
                                                         double* tables64) {
  extern __shared__ double sm[];
  const ShapeDesc sd = shapes[blockIdx.x];
  const int n = sd.n, m = sd.m;
  const int tid = threadIdx.x;
  const double tf = (double)sd.t_f;
  const double rho = (double)kc.rho;

  double* P = sm;                 // [n][NC]
  double* Pd = P + n * NC;        // [n][NC]
  double* Pdd = Pd + n * NC;      // [n][NC]
  double* Gpp = Pdd + n * NC;     // P^T P
  double* Gdd = Gpp + NC * NC;    // P''^T P''  (= Q)
  double* Gd = Gdd + NC * NC;     // P'^T P'
  double* aug = Gd + NC * NC;     // [KMAX][2 KMAX]
  double* fac = aug + KMAX * 2 * KMAX;
  int* piv = (int*)(fac + KMAX);
  // the inverses go straight to the FP64 table in global memory
  double* Minv = tables64 + sd.table64_off;  // [SYS_COUNT][KMAX][KMAX]

  const int deg = NC - 1;
  for (int e = tid; e < n * NC; e += blockDim.x) {
    const int i = e / NC, k = e % NC;
    const double tau = (double)i / (double)(n - 1);
    P[e] = bern(deg, k, tau);
    Pd[e] = deg * (bern(deg - 1, k - 1, tau) - bern(deg - 1, k, tau)) / tf;
    Pdd[e] = deg * (deg - 1) * (bern(deg - 2, k - 2, tau) - 2.0 * bern(deg - 2, k - 1, tau) + bern(deg - 2, k, tau)) /
             (tf * tf);
  }
  __syncthreads();
  for (int e = tid; e < NC * NC; e += blockDim.x) {
    const int r = e / NC, c = e % NC;
    double spp = 0, sdd = 0, sd1 = 0;
    for (int i = 0; i < n; ++i) {
      spp += P[i * NC + r] * P[i * NC + c];
      sdd += Pdd[i * NC + r] * Pdd[i * NC + c];
      sd1 += Pd[i * NC + r] * Pd[i * NC + c];
    }
    Gpp[e] = spp;
    Gdd[e] = sdd;
    Gd[e] = sd1;
  }
  __syncthreads();

  for (int sys = 0; sys < SYS_COUNT; ++sys) {
    const int ne = (sys == SYS_Y || sys == SYS_0Y) ? NY : (sys == SYS_P ? NP : NX);
    const int nk = NC + ne;
    const int W = 2 * nk;
    for (int e = tid; e < nk * W; e += blockDim.x) {
      const int r = e / W, c = e % W;
      double v = 0.0;
      if (c >= nk) {
        v = (c - nk == r) ? 1.0 : 0.0;
      } else if (r < NC && c < NC) {
        const int q = r * NC + c;
        if (sys == SYS_X || sys == SYS_Y)
          v = Gdd[q] + rho * (m * Gpp[q] + Gdd[q] + Gd[q]);
        else if (sys == SYS_P)
          v = Gdd[q] + rho * Gpp[q];
        else
          v = Gdd[q];
      } else if (r >= NC && c >= NC) {
        v = 0.0;
      } else {
        // constraint row `row` against coefficient `col`
        const int row = (r >= NC) ? r - NC : c - NC;
        const int col = (r >= NC) ? c : r;
        const int last = (n - 1) * NC + col;
        if (sys == SYS_P) {
          const double rows[NP] = {P[col], Pd[col], P[last], Pd[last]};
          v = rows[row];
        } else {
          const double rows[NY] = {P[col], Pd[col], Pdd[col], P[last], Pd[last], Pdd[last]};
          v = rows[row];
        }
      }
      aug[e] = v;
    }
    __syncthreads();
    gauss_jordan(aug, nk, fac, piv);
    for (int e = tid; e < KMAX * KMAX; e += blockDim.x) {
      const int r = e / KMAX, c = e % KMAX;
      Minv[sys * KMAX * KMAX + e] = (r < nk && c < nk) ? aug[r * W + nk + c] : 0.0;
    }
    __syncthreads();
  }

  // FP32 tables
  float* T = tables + sd.table_off;
  for (int e = tid; e < n * NC; e += blockDim.x) {
    const int i = e / NC, k = e % NC;
    T[tab_basis(n, 0) + k * n + i] = (float)P[e];
    T[tab_basis(n, 1) + k * n + i] = (float)Pd[e];
    T[tab_basis(n, 2) + k * n + i] = (float)Pdd[e];
  }
  const double* Mx = Minv + SYS_X * KMAX * KMAX;
  const double* My = Minv + SYS_Y * KMAX * KMAX;
  const double* Mp = Minv + SYS_P * KMAX * KMAX;
  const double* M0x = Minv + SYS_0X * KMAX * KMAX;
  const double* M0y = Minv + SYS_0Y * KMAX * KMAX;
  for (int e = tid; e < NC * NC; e += blockDim.x) {
    const int r = e / NC, c = e % NC;
    // M (rho F_ax^T F_ax): the part of M rho F^T g that is linear in the previous c
    double mgx = 0, mgy = 0;
    for (int j = 0; j < NC; ++j) {
      const double g = rho * (m * Gpp[j * NC + c] + Gdd[j * NC + c] + Gd[j * NC + c]);
      mgx += Mx[r * KMAX + j] * g;
      mgy += My[r * KMAX + j] * g;
    }
    double* A64 = tables64 + sd.table64_off;
    A64[T64_MGX + e] = mgx;
    A64[T64_MX + e] = Mx[r * KMAX + c];
    A64[T64_MGY + e] = mgy;
    A64[T64_MY + e] = My[r * KMAX + c];
    T[tab_square(n, SQ_MGX) + e] = (float)mgx;
    T[tab_square(n, SQ_MX) + e] = (float)Mx[r * KMAX + c];
    T[tab_square(n, SQ_MGY) + e] = (float)mgy;
    T[tab_square(n, SQ_MY) + e] = (float)My[r * KMAX + c];
    T[tab_square(n, SQ_MP) + e] = (float)Mp[r * KMAX + c];
  }
  float* Bt = T + tab_bnd(n);
  for (int e = tid; e < NC * NY; e += blockDim.x) {
    const int r = e / NY, c = e % NY;
    if (c < NX) {
      Bt[BND_MBX + r * NX + c] = (float)Mx[r * KMAX + NC + c];
      Bt[BND_M0BX + r * NX + c] = (float)M0x[r * KMAX + NC + c];
      Bt[BND_MBP + r * NP + c] = (float)Mp[r * KMAX + NC + c];
    }
    Bt[BND_MBY + r * NY + c] = (float)My[r * KMAX + NC + c];
    double* A64 = tables64 + sd.table64_off;
    if (c < NX) A64[T64_MBX + r * NX + c] = Mx[r * KMAX + NC + c];
    A64[T64_MBY + r * NY + c] = My[r * KMAX + NC + c];
    Bt[BND_M0BY + r * NY + c] = (float)M0y[r * KMAX + NC + c];
  }
}

// Packed product tiles of every shape (layout next to tab_pack), from the FP32
// basis that k_setup wrote.
__global__ void k_pack(const ShapeDesc* __restrict__ shapes, float* __restrict__ tables) {
  const ShapeDesc sd = shapes[blockIdx.x];
  float* T = tables + sd.table_off;
  const int n = sd.n;
  float4* out = reinterpret_cast<float4*>(T + tab_pack(n));
  const int total = n_tiles(n) * PACK_SLOTS * WAVE;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int l = e % WAVE, s = (e / WAVE) % PACK_SLOTS, w = e / (WAVE * PACK_SLOTS);
    const int j = l & 15, q = l >> 4, mi = s % 3;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = s < 3 ? TILE_T * w + j : TILE_T * w + 4 * q + r;
      const int k = s < 3 ? 4 * q + r : j;
      v[r] = (t < n && k < NC) ? T[tab_basis(n, mi) + k * n + t] : 0.f;
    }
    out[e] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

}  // namespace

hipError_t launch_setup(const ShapeDesc* d_shapes, int n_shapes, const SolverConst& k, float* d_tables,
                        double* d_tables64, int max_n, hipStream_t stream) {
  const size_t smem = sizeof(double) * (3 * (size_t)max_n * NC + 3 * NC * NC + KMAX * 2 * KMAX + KMAX) + 16;
  hipLaunchKernelGGL(k_setup, dim3(n_shapes), dim3(SETUP_THREADS), smem, stream, d_shapes, k, d_tables, d_tables64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack, dim3(n_shapes), dim3(256), 0, stream, d_shapes, d_tables);
  return hipGetLastError();
}

}  // namespace traj
