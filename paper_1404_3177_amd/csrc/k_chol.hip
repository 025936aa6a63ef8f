// Newton direction (Eq. 6): delta = (-H)^{-1} g through the Cholesky factor
// of A = -H, always in FP64.
//
// Blocked right-looking factorisation with 64-wide panels on the lower
// triangle of A (row-major, in place):
//   diag  : one workgroup factors the 64x64 diagonal block in LDS and
//           checks every pivot against the round-off floor
//           n * eps * max_k A_kk (a pivot at or below it means -H is not
//           numerically positive definite);
//   trsm  : L21 = A21 L11^{-T}, one thread per row, L11 in LDS;
//   update: A22 -= L21 L21^T on the lower 64x64 tiles, FP64 MFMA.
// Then L z = g and L^T delta = z panel by panel: each workgroup re-solves
// the small diagonal system itself and updates its share of the remaining
// right-hand side, so one launch per panel suffices and no two workgroups
// write the same entry.  A failure flag in device memory makes every later
// launch return at once.
#include <cmath>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = 64;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// A <- -H on the lower triangle (the factorisation reads nothing else)
__global__ void k_negate_lower(double *A, int64_t n) {
  const int64_t r = blockIdx.y;
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c <= r && r < n) A[r * n + c] = -A[r * n + c];
}

__global__ __launch_bounds__(256) void k_floor(const double *A, int64_t n,
                                               double *floor_out,
                                               int32_t *info) {
  __shared__ double red[256];
  double m = 0.0;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = A[i * n + i];
    if (!isfinite(v)) bad = true;
    m = fmax(m, v);
  }
  red[threadIdx.x] = bad ? INFINITY : m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = red[0];
    *floor_out = double(n) * 2.220446049250313e-16 * mx;
    info[0] = isfinite(mx) ? 0 : 1;
  }
}

__global__ __launch_bounds__(256) void k_chol_diag(double *A, int64_t n,
                                                   int64_t j0,
                                                   const double *floor_p,
                                                   int32_t *info) {
  __shared__ double L[NB][NB + 1];
  __shared__ int fail;
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NB, n - j0);
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e / jb, j = e - (e / jb) * jb;
    L[i][j] = (j <= i) ? A[(j0 + i) * n + j0 + j] : 0.0;
  }
  if (tid == 0) fail = 0;
  const double fl = *floor_p;
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    if (tid == 0) {
      const double d = L[k][k];
      if (!(d > fl) || !isfinite(d)) {
        fail = 1;
        info[0] = int(j0 + k + 1);
      } else {
        L[k][k] = sqrt(d);
      }
    }
    __syncthreads();
    if (fail) return;
    const double dk = L[k][k];
    for (int i = k + 1 + tid; i < jb; i += 256) L[i][k] /= dk;
    __syncthreads();
    const int m = jb - k - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + (e - (e / m) * m);
      if (j <= i) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e / jb, j = e - (e / jb) * jb;
    if (j <= i) A[(j0 + i) * n + j0 + j] = L[i][j];
  }
}

// rows below the panel: x L11^T = a  ->  x_c = (a_c - sum_{k<c} x_k L_ck)/L_cc
__global__ __launch_bounds__(64) void k_chol_trsm(double *A, int64_t n,
                                                  int64_t j0,
                                                  const int32_t *info) {
  __shared__ double L[NB][NB + 1];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NB, n - j0);
  const int64_t j1 = j0 + jb;
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 64) {
    const int i = e / jb, j = e - (e / jb) * jb;
    L[i][j] = (j <= i) ? A[(j0 + i) * n + j0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t r = j1 + int64_t(blockIdx.x) * 64 + tid;
  if (r >= n) return;
  double x[NB];
  double *row = A + r * n + j0;
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = c < jb ? row[c] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < jb) {
      double s = x[c];
#pragma unroll
      for (int k = 0; k < c; ++k) s = fma(-x[k], L[c][k], s);
      x[c] = s / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < jb) row[c] = x[c];
}

// trailing update on lower tiles: A[R][C] -= L21[R] . L21[C], FP64 MFMA
__global__ __launch_bounds__(256) void k_chol_update(double *A, int64_t n,
                                                     int64_t j0,
                                                     const int32_t *info) {
  __shared__ double Ar[NB][NB + 1];
  __shared__ double Ac[NB][NB + 1];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NB, n - j0);
  const int64_t j1 = j0 + jb;
  // lower-triangular tile index
  const int64_t b = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int64_t tj = b - ti * (ti + 1) / 2;
  const int64_t R0 = j1 + ti * NB, C0 = j1 + tj * NB;
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, k = e - (e / NB) * NB;
    const int64_t rr = R0 + i, cc = C0 + i;
    Ar[i][k] = (rr < n && k < jb) ? A[rr * n + j0 + k] : 0.0;
    Ac[i][k] = (cc < n && k < jb) ? A[cc * n + j0 + k] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
  const int ar = 16 * wv + (lane & 15);
  for (int ks = 0; ks < (jb + 3) / 4; ++ks) {
    const int k = 4 * ks + (lane >> 4);
    const double av = Ar[ar][k];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double bv = Ac[16 * t + (lane & 15)][k];
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = R0 + 16 * wv + (lane >> 4) + 4 * r;
      const int64_t cc = C0 + 16 * t + (lane & 15);
      if (rr < n && cc < n && cc <= rr) A[rr * n + cc] -= acc[t][r];
    }
  }
}

// forward substitution, panel j0: z_p = L11^{-1} y_p, then y_r -= L_rp z_p
__global__ __launch_bounds__(256) void k_chol_fwd(const double *A, int64_t n,
                                                  int64_t j0, double *y,
                                                  double *z,
                                                  const int32_t *info) {
  __shared__ double L[NB][NB + 1];
  __shared__ double zp[NB];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NB, n - j0);
  const int64_t j1 = j0 + jb;
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e / jb, j = e - (e / jb) * jb;
    L[i][j] = (j <= i) ? A[(j0 + i) * n + j0 + j] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    // lane j holds unknown j; each step broadcasts one finished value
    double zl = tid < jb ? y[j0 + tid] : 0.0;
    for (int c = 0; c < jb; ++c) {
      const double part = wsum((tid < c) ? L[c][tid] * zl : 0.0);
      if (tid == c) zl = (zl - part) / L[c][c];
    }
    zp[tid] = zl;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < jb) z[j0 + tid] = zp[tid];
  const int64_t r = j1 + int64_t(blockIdx.x) * 256 + tid;
  if (r < n) {
    const double *row = A + r * n + j0;
    double s = 0.0;
    for (int c = 0; c < jb; ++c) s = fma(row[c], zp[c], s);
    y[r] -= s;
  }
}

// backward substitution, panel j0: d_p = L11^{-T} z_p, then
// z_c -= sum_r L_rc d_r for the columns c < j0
__global__ __launch_bounds__(256) void k_chol_bwd(const double *A, int64_t n,
                                                  int64_t j0, double *z,
                                                  double *delta,
                                                  const int32_t *info) {
  __shared__ double L[NB][NB + 1];
  __shared__ double dp[NB];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NB, n - j0);
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e / jb, j = e - (e / jb) * jb;
    L[i][j] = (j <= i) ? A[(j0 + i) * n + j0 + j] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    double dl = tid < jb ? z[j0 + tid] : 0.0;
    for (int c = jb - 1; c >= 0; --c) {
      const double part = wsum((tid > c && tid < jb) ? L[tid][c] * dl : 0.0);
      if (tid == c) dl = (dl - part) / L[c][c];
    }
    dp[tid] = dl;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < jb) delta[j0 + tid] = dp[tid];
  const int64_t c = int64_t(blockIdx.x) * 256 + tid;
  if (c < j0) {
    double s = 0.0;
    for (int r = 0; r < jb; ++r) s = fma(A[(j0 + r) * n + c], dp[r], s);
    z[c] -= s;
  }
}

}  // namespace

int chol_solve_run(Ctx *c, double *A, int64_t n, const double *g,
                   double *delta, int32_t *info, hipStream_t s) {
  void *scr;
  MNL_TRY(ws_get(c, S_CHOL, size_t(2 * n + 8) * 8, &scr));
  double *y = static_cast<double *>(scr);
  double *z = y + n;
  double *floor_p = z + n;
  MNL_HIP(c, hipMemcpyAsync(y, g, size_t(n) * 8, hipMemcpyDeviceToDevice, s));
  {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_negate_lower, grid, dim3(256), 0, s, A, n);
  }
  hipLaunchKernelGGL(k_floor, dim3(1), dim3(256), 0, s, A, n, floor_p, info);
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int64_t jb = std::min<int64_t>(NB, n - j0);
    const int64_t rest = n - j0 - jb;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, n, j0,
                       floor_p, info);
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_trsm, dim3((unsigned)((rest + 63) / 64)),
                         dim3(64), 0, s, A, n, j0, info);
      const int64_t T = (rest + NB - 1) / NB;
      hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)),
                         dim3(256), 0, s, A, n, j0, info);
    }
  }
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int64_t jb = std::min<int64_t>(NB, n - j0);
    const int64_t rest = n - j0 - jb;
    const unsigned gr = (unsigned)std::max<int64_t>(1, (rest + 255) / 256);
    hipLaunchKernelGGL(k_chol_fwd, dim3(gr), dim3(256), 0, s, A, n, j0, y, z,
                       info);
  }
  const int64_t last = ((n - 1) / NB) * NB;
  for (int64_t j0 = last; j0 >= 0; j0 -= NB) {
    const unsigned gr = (unsigned)std::max<int64_t>(1, (j0 + 255) / 256);
    hipLaunchKernelGGL(k_chol_bwd, dim3(gr), dim3(256), 0, s, A, n, j0, z,
                       delta, info);
  }
  MNL_HIP(c, hipGetLastError());
  return MNL_OK;
}

}  // namespace mnl
