// Newton direction (Eq. 6): delta = (-H)^{-1} g through the Cholesky factor
// of A = -H, always in FP64.
//
// The matrix buffer has n + 1 rows: rows 0..n-1 hold H (row-major), row n
// holds g^T.  Factoring the augmented lower triangle
//     [ A    ]   [ L    ] [ L^T  z ]
//     [ g^T  ] = [ z^T  ]
// by blocked right-looking Cholesky leaves z = L^{-1} g in row n, so the
// forward substitution comes out of the factorisation.  Per 32-wide panel:
//   diag  : one wave factors the diagonal block in registers (LDL^T form,
//           then scaled), checks the pivots against the round-off floor
//           n * eps * max_k A_kk and writes L11 to scratch;
//   trsm  : rows below the panel solve x L11^T = a, one row per thread;
//   update: puts L11 in place, then A22 -= L21 L21^T on the lower 64x64
//           tiles, FP64 MFMA.
// Then L^T delta = z by 64-wide panels from the bottom: each workgroup
// re-solves the panel's small triangular system itself and updates its
// share of the remaining right-hand side, so one launch per panel suffices
// and no two workgroups write the same entry.  A failure flag in device
// memory makes every later launch return at once.
#include <cmath>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NBF = 32;   // factorisation panel width
constexpr int NBS = 64;   // backward-solve panel width
constexpr int TILE = 64;  // trailing-update tile

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// A <- -H on the lower triangle of rows 0..n-1 (nothing else is read)
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

// Diagonal block of panel j0 (width jb <= NBF), one wave: lane i keeps row
// i in registers; each LDL^T step broadcasts the finished column through
// LDS.  Pivots are checked against the round-off floor; L11 goes to
// scratch (l11, row-major NBF x NBF, identity rows past jb) and is put into
// A by the next trailing-update launch.
__global__ __launch_bounds__(64) void k_chol_diag(const double *A, int64_t n,
                                                  int64_t j0,
                                                  const double *floor_p,
                                                  double *l11, int32_t *info) {
  __shared__ double col[NBF];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NBF, n - j0);
  const int tid = threadIdx.x;
  const bool mine = tid < jb;
  double a[NBF];
  {
    const double *src = A + (j0 + (mine ? tid : 0)) * n + j0;
#pragma unroll
    for (int j = 0; j < NBF; ++j)
      a[j] = (mine && j <= tid && j < jb) ? src[j] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NBF; ++k) {
    if (k < jb) {
      if (tid < jb) col[tid] = a[k];
      __syncthreads();
      const double lik = a[k] / col[k];
#pragma unroll
      for (int j = k + 1; j < NBF; ++j)
        if (j <= tid) a[j] = fma(-lik, col[j], a[j]);
      __syncthreads();
    }
  }
  double d = 0.0;
#pragma unroll
  for (int j = 0; j < NBF; ++j)
    if (j == tid) d = a[j];
  if (tid < jb) col[tid] = d;
  __syncthreads();
  const double fl = *floor_p;
  for (int k = 0; k < jb; ++k) {
    const double dk = col[k];
    if (!(dk > fl) || !isfinite(dk)) {
      if (tid == 0) info[0] = int(j0 + k + 1);
      return;
    }
  }
  if (tid < NBF) {
    double *dst = l11 + tid * NBF;
#pragma unroll
    for (int j = 0; j < NBF; ++j) {
      double v;
      if (!mine) v = (j == tid) ? 1.0 : 0.0;
      else if (j < tid) v = a[j] / sqrt(col[j]);
      else if (j == tid) v = sqrt(col[j]);
      else v = 0.0;
      dst[j] = v;
    }
  }
}

// rows below panel j0: x L11^T = a, one row per thread in registers, L11
// broadcast from LDS (its padding rows are the identity, so no bounds on
// the column index are needed)
__global__ __launch_bounds__(64) void k_chol_trsm(double *A, int64_t n,
                                                  int64_t nrows, int64_t j0,
                                                  const double *l11,
                                                  const int32_t *info) {
  __shared__ double L[NBF][NBF + 1];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NBF, n - j0);
  const int tid = threadIdx.x;
  for (int e = tid; e < NBF * NBF; e += 64)
    L[e / NBF][e % NBF] = l11[e];
  __syncthreads();
  const int64_t r = j0 + jb + int64_t(blockIdx.x) * 64 + tid;
  if (r >= nrows) return;
  double x[NBF];
  double *row = A + r * n + j0;
#pragma unroll
  for (int c = 0; c < NBF; ++c) x[c] = c < jb ? row[c] : 0.0;
  // the runtime bound keeps the compiler from hoisting all of L11 into
  // registers ahead of the substitution
#pragma unroll
  for (int c = 0; c < NBF; ++c) {
    if (c < jb) {
      double s0 = x[c];
#pragma unroll
      for (int k = 0; k < c; ++k) s0 = fma(-x[k], L[c][k], s0);
      x[c] = s0 / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < NBF; ++c)
    if (c < jb) row[c] = x[c];
}

// trailing update on lower tiles of rows/cols >= j0 + jb (rows up to
// nrows - 1, columns up to n - 1): A[R][C] -= L21[R] . L21[C], FP64 MFMA
__global__ __launch_bounds__(256) void k_chol_update(double *A, int64_t n,
                                                     int64_t nrows, int64_t j0,
                                                     const double *l11,
                                                     const int32_t *info) {
  __shared__ double Ar[TILE][NBF + 1];
  __shared__ double Ac[TILE][NBF + 1];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NBF, n - j0);
  const int64_t j1 = j0 + jb;
  if (blockIdx.x == 0) {
    // the panel's factored diagonal block, written by k_chol_panel
    for (int e = threadIdx.x; e < jb * jb; e += 256) {
      const int i = e / jb, j = e - (e / jb) * jb;
      if (j <= i) A[(j0 + i) * n + j0 + j] = l11[i * NBF + j];
    }
  }
  const int64_t b = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int64_t tj = b - ti * (ti + 1) / 2;
  const int64_t R0 = j1 + ti * TILE, C0 = j1 + tj * TILE;
  const int tid = threadIdx.x;
  for (int e = tid; e < TILE * NBF; e += 256) {
    const int i = e / NBF, k = e - (e / NBF) * NBF;
    const int64_t rr = R0 + i, cc = C0 + i;
    Ar[i][k] = (rr < nrows && k < jb) ? A[rr * n + j0 + k] : 0.0;
    Ac[i][k] = (cc < n && k < jb) ? A[cc * n + j0 + k] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
  const int ar = 16 * wv + (lane & 15);
#pragma unroll
  for (int ks = 0; ks < NBF / 4; ++ks) {
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
      if (rr < nrows && cc < n && cc <= rr) A[rr * n + cc] -= acc[t][r];
    }
  }
}

// backward substitution, panel j0: d_p = L11^{-T} z_p, then
// z_c -= sum_r L_rc d_r for the columns c < j0
__global__ __launch_bounds__(256) void k_chol_bwd(const double *A, int64_t n,
                                                  int64_t j0, double *z,
                                                  double *delta,
                                                  const int32_t *info) {
  __shared__ double L[NBS][NBS + 1];
  __shared__ double dp[NBS];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NBS, n - j0);
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
    // independent partial sums keep many loads in flight
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const double *colp = A + j0 * n + c;
#pragma unroll 16
    for (int r = 0; r < jb; ++r) s[r & 3] = fma(colp[int64_t(r) * n], dp[r], s[r & 3]);
    z[c] -= (s[0] + s[1]) + (s[2] + s[3]);
  }
}

}  // namespace

int chol_solve_run(Ctx *c, double *A, int64_t n, const double *g,
                   double *delta, int32_t *info, hipStream_t s) {
  void *scr;
  MNL_TRY(ws_get(c, S_CHOL, size_t(n + 8 + NBF * NBF) * 8, &scr));
  double *z = static_cast<double *>(scr);
  double *floor_p = z + n;
  double *l11 = floor_p + 8;
  const int64_t nrows = n + 1;
  // g^T as row n of the augmented matrix
  MNL_HIP(c, hipMemcpyAsync(A + n * n, g, size_t(n) * 8,
                            hipMemcpyDeviceToDevice, s));
  {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_negate_lower, grid, dim3(256), 0, s, A, n);
  }
  hipLaunchKernelGGL(k_floor, dim3(1), dim3(256), 0, s, A, n, floor_p, info);
  for (int64_t j0 = 0; j0 < n; j0 += NBF) {
    const int64_t jb = std::min<int64_t>(NBF, n - j0);
    const int64_t rest = nrows - j0 - jb;   // >= 1: the g row
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, s, A, n, j0,
                       floor_p, l11, info);
    hipLaunchKernelGGL(k_chol_trsm, dim3((unsigned)((rest + 63) / 64)),
                       dim3(64), 0, s, A, n, nrows, j0, l11, info);
    const int64_t T = (rest + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(T * (T + 1) / 2)),
                       dim3(256), 0, s, A, n, nrows, j0, l11, info);
  }
  MNL_HIP(c, hipMemcpyAsync(z, A + n * n, size_t(n) * 8,
                            hipMemcpyDeviceToDevice, s));
  const int64_t last = ((n - 1) / NBS) * NBS;
  for (int64_t j0 = last; j0 >= 0; j0 -= NBS) {
    const unsigned gr = (unsigned)std::max<int64_t>(1, (j0 + 255) / 256);
    hipLaunchKernelGGL(k_chol_bwd, dim3(gr), dim3(256), 0, s, A, n, j0, z,
                       delta, info);
  }
  MNL_HIP(c, hipGetLastError());
  return MNL_OK;
}

}  // namespace mnl
