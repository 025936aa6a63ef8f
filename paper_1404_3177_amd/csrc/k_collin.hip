// Collinearity check of the data (Sec. 2.3 linDepTol, App. B): the
// variables to keep so that X, every Z_k and the differenced generic data
// stacked over alternatives have full column rank.
//
// Column-order QR with tolerance tol drops column j when its part
// orthogonal to the kept columns before it has norm below tol times its
// own norm.  On the Gram matrix G = M^T M the same quantity is a Schur
// complement: after equilibrating G to unit diagonal, eliminating the kept
// columns in order leaves the squared residual ratio of column j on the
// diagonal, so column j goes when that pivot is below tol^2 (or when the
// column is zero).  The Gram matrices are library GEMMs over the
// observations (X^T X, the K blocks Z_k^T Z_k as one strided batch, and
// Ytil^T Ytil over the N (K - 1) stacked rows of Ytil_k = Y_k - Y_0, which
// a small kernel forms first); one workgroup per Gram matrix then runs the
// ordered elimination.  The Gram route squares the condition number: it
// agrees with the QR criterion while kappa(kept columns)^2 eps << tol^2.
#include <algorithm>
#include <vector>

#include <rocblas/rocblas.h>

#include "mnl_common.h"

namespace mnl {

namespace {

// Ytil[i][k - 1][c] = Y[i][k][c] - Y[i][0][c], k = 1..K-1
__global__ __launch_bounds__(256) void k_ydiff(const double *Y, int64_t N,
                                               int K, int g, double *Yt) {
  const int64_t cnt = N * (K - 1) * g;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * 256) {
    const int64_t i = e / (int64_t(K - 1) * g);
    const int64_t r = e - i * (int64_t(K - 1) * g);
    const int k = 1 + int(r / g), c = int(r % g);
    Yt[e] = Y[(i * K + k) * g + c] - Y[i * K * g + c];
  }
}

// Ordered elimination on each Gram matrix (block b: matrix b of size n,
// column-major n x n at G + b n^2, lower triangle used, overwritten).
// keep[b n + j] = 1 if column j is kept.
__global__ __launch_bounds__(256) void k_ordered_elim(double *G, int n,
                                                      double tol2,
                                                      int32_t *keep) {
  double *A = G + int64_t(blockIdx.x) * n * n;
  int32_t *kp = keep + int64_t(blockIdx.x) * n;
  const int t = threadIdx.x;
  __shared__ double dg[1024];  // 1 / sqrt(G_jj), 0 for a zero column
  for (int j = t; j < n; j += 256) {
    const double d = A[int64_t(j) * n + j];
    dg[j] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  // unit diagonal (zero columns become zero)
  const int64_t tri = int64_t(n) * (n + 1) / 2;
  for (int64_t e = t; e < tri; e += 256) {
    int64_t l = int64_t((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
    while ((l + 1) * (l + 2) / 2 <= e) ++l;
    while (l * (l + 1) / 2 > e) --l;
    const int64_t i = e - l * (l + 1) / 2;   // i <= l: entry (l, i) lower
    A[i * n + l] *= dg[i] * dg[l];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double piv = A[int64_t(j) * n + j];
    const bool kj = dg[j] > 0.0 && piv >= tol2;
    if (t == 0) kp[j] = kj ? 1 : 0;
    if (kj) {
      // A[l][i] -= A[l][j] A[i][j] / piv for j < i <= l
      const int m = n - j - 1;
      const int64_t cnt = int64_t(m) * (m + 1) / 2;
      const double inv = 1.0 / piv;
      for (int64_t e = t; e < cnt; e += 256) {
        int64_t l = int64_t((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
        while ((l + 1) * (l + 2) / 2 <= e) ++l;
        while (l * (l + 1) / 2 > e) --l;
        const int64_t i = e - l * (l + 1) / 2;
        const int64_t L = j + 1 + l, I = j + 1 + i;
        A[I * n + L] -= A[int64_t(j) * n + L] * A[int64_t(j) * n + I] * inv;
      }
    }
    __syncthreads();
  }
}

// out[r][c'] = in[r][sel[c']] for a row-major [rows][cols] matrix
__global__ __launch_bounds__(256) void k_gather_cols(const double *in,
                                                     int64_t rows, int cols,
                                                     const int32_t *sel,
                                                     int cout, double *out) {
  const int64_t cnt = rows * cout;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * 256) {
    const int64_t r = e / cout;
    const int c = int(e - r * cout);
    out[e] = in[r * cols + sel[c]];
  }
}

unsigned grid_for(int64_t cnt) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (cnt + 255) / 256));
}

}  // namespace

int collinear_run(Ctx *c, const Dims &d, const mnl_problem *pr, double tol,
                  int32_t *keep_x, int32_t *keep_y, int32_t *keep_z,
                  hipStream_t s) {
  const int p = d.p, g = d.g, a = d.a, K = d.K;
  const int64_t N = d.N;
  if (p > 1024 || g > 1024 || a > 1024)
    return set_error(c, MNL_ERR_UNSUPPORTED, "more than 1024 columns");
  // Gram matrices: X (p^2), Z_0..Z_{K-1} (K a^2), Ytil (g^2); masks
  const size_t ng = size_t(p) * p + size_t(K) * a * a + size_t(g) * g;
  const size_t nk = size_t(p) + size_t(K) * a + size_t(g);
  void *gv, *yv = nullptr;
  MNL_TRY(ws_get(c, S_COLLIN, (ng + nk) * 8, &gv));
  double *Gx = (double *)gv, *Gz = Gx + size_t(p) * p,
         *Gy = Gz + size_t(K) * a * a;
  int32_t *kd = (int32_t *)(Gy + size_t(g) * g);
  void *hv;
  MNL_TRY(blas_get(c, s, &hv));
  rocblas_handle hb = static_cast<rocblas_handle>(hv);
  const double one = 1.0, zero = 0.0;
  rocblas_status st = rocblas_status_success;
  // row-major [N][cols] data are column-major cols x N: G = M M^T
  if (p > 0 && st == rocblas_status_success)
    st = rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_transpose,
                       p, p, rocblas_int(N), &one, pr->X, p, pr->X, p, &zero,
                       Gx, p);
  if (a > 0 && st == rocblas_status_success)
    st = rocblas_dgemm_strided_batched(
        hb, rocblas_operation_none, rocblas_operation_transpose, a, a,
        rocblas_int(N), &one, pr->Z, rocblas_int(int64_t(K) * a), a, pr->Z,
        rocblas_int(int64_t(K) * a), a, &zero, Gz, a, int64_t(a) * a, K);
  if (g > 0 && st == rocblas_status_success) {
    const int64_t rows = N * (K - 1);
    MNL_TRY(ws_get(c, S_XX, size_t(rows) * g * 8 + 8, &yv));
    c->xx_epoch = ~uint64_t(0);   // the X o X cache no longer holds its data
    hipLaunchKernelGGL(k_ydiff, dim3(grid_for(rows * g)), dim3(256), 0, s,
                       pr->Y, N, K, g, (double *)yv);
    if (rows > 0)
      st = rocblas_dgemm(hb, rocblas_operation_none,
                         rocblas_operation_transpose, g, g, rocblas_int(rows),
                         &one, (const double *)yv, g, (const double *)yv, g,
                         &zero, Gy, g);
    else
      MNL_HIP(c, hipMemsetAsync(Gy, 0, size_t(g) * g * 8, s));
  }
  if (st != rocblas_status_success)
    return set_error(c, MNL_ERR_HIP, "rocblas Gram product failed (%d)",
                     int(st));
  const double tol2 = tol * tol;
  int32_t *kx = kd, *kz = kx + p, *ky = kz + size_t(K) * a;
  if (p > 0)
    hipLaunchKernelGGL(k_ordered_elim, dim3(1), dim3(256), 0, s, Gx, p, tol2,
                       kx);
  if (a > 0)
    hipLaunchKernelGGL(k_ordered_elim, dim3(K), dim3(256), 0, s, Gz, a, tol2,
                       kz);
  if (g > 0)
    hipLaunchKernelGGL(k_ordered_elim, dim3(1), dim3(256), 0, s, Gy, g, tol2,
                       ky);
  MNL_HIP(c, hipGetLastError());
  std::vector<int32_t> h(nk);
  MNL_HIP(c, hipMemcpyAsync(h.data(), kd, nk * 4, hipMemcpyDeviceToHost, s));
  MNL_HIP(c, hipStreamSynchronize(s));
  for (int j = 0; j < p; ++j) keep_x[j] = h[j];
  for (int j = 0; j < a; ++j) {
    int32_t k_all = 1;
    for (int k = 0; k < K; ++k) k_all &= h[p + size_t(k) * a + j];
    keep_z[j] = k_all;
  }
  for (int j = 0; j < g; ++j) keep_y[j] = h[p + size_t(K) * a + j];
  return MNL_OK;
}

int select_columns_run(Ctx *c, const Dims &d, const mnl_problem *pr,
                       const int32_t *keep_x, const int32_t *keep_y,
                       const int32_t *keep_z, double *X_out, double *Y_out,
                       double *Z_out, hipStream_t s) {
  std::vector<int32_t> sel;
  int nx = 0, ny = 0, nz = 0;
  for (int j = 0; j < d.p; ++j)
    if (keep_x[j]) sel.push_back(j), ++nx;
  for (int j = 0; j < d.g; ++j)
    if (keep_y[j]) sel.push_back(j), ++ny;
  for (int j = 0; j < d.a; ++j)
    if (keep_z[j]) sel.push_back(j), ++nz;
  if ((nx && !X_out) || (ny && !Y_out) || (nz && !Z_out))
    return set_error(c, MNL_ERR_ARG, "NULL output for kept columns");
  void *sv;
  MNL_TRY(ws_get(c, S_COLLIN, sel.size() * 4 + 8, &sv));
  int32_t *sd = (int32_t *)sv;
  if (!sel.empty()) {
    MNL_HIP(c, hipMemcpyAsync(sd, sel.data(), sel.size() * 4,
                              hipMemcpyHostToDevice, s));
    // the host vector must outlive the copy
    MNL_HIP(c, hipStreamSynchronize(s));
  }
  const int64_t NK = d.N * d.K;
  if (nx)
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(d.N * nx)), dim3(256), 0,
                       s, pr->X, d.N, d.p, sd, nx, X_out);
  if (ny)
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(NK * ny)), dim3(256), 0,
                       s, pr->Y, NK, d.g, sd + nx, ny, Y_out);
  if (nz)
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(NK * nz)), dim3(256), 0,
                       s, pr->Z, NK, d.a, sd + nx + ny, nz, Z_out);
  MNL_HIP(c, hipGetLastError());
  return MNL_OK;
}

}  // namespace mnl
