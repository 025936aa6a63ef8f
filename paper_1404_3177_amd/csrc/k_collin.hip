// Collinearity check of the data (Sec. 2.4 linDepTol, App. B): the
// variables to keep so that X, every Z_k and the differenced generic data
// stacked over alternatives have full column rank.
//
// Column-order QR with tolerance tol drops column j when its part
// orthogonal to the kept columns before it has norm below tol times its
// own norm.  On the Gram matrix G = M^T M the same quantity is a Schur
// complement: after equilibrating G to unit diagonal, eliminating the kept
// columns in order leaves the squared residual ratio of column j on the
// diagonal, so column j goes when that pivot is below tol^2 (or when the
// column is zero).  The Gram matrices (X^T X, the K blocks Z_k^T Z_k, and
// Ytil^T Ytil over the N (K - 1) stacked rows of Ytil_k = Y_k - Y_0) come
// from one pass over the observations (k_gram: tiles of observations staged
// in LDS, each thread owning up to 16 Gram entries, Ytil formed on the fly;
// per-workgroup partials summed in a fixed order).  Shapes beyond its
// limits take library GEMMs instead (Ytil then formed in the workspace).
// One workgroup per Gram matrix then runs the ordered elimination.  The Gram route squares the condition number: it
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

// One Gram entry: the LDS offsets (within an observation's staged row
// [x | y | z]) of its two columns, its kind (0: product, 2: differenced
// generic data summed over alternatives 1..K-1) and its two destinations
// in the column-major Gram storage.
struct GramEnt {
  int32_t oj, ol, kind, dst, dst2, pad;
};
constexpr int kGramEPT = 16;   // entries per thread at most

// Partial Gram entries of workgroup b over its observation range.
__global__ __launch_bounds__(256) void k_gram(const double *X,
                                              const double *Y,
                                              const double *Z, int64_t N,
                                              int p, int K, int g, int a,
                                              const GramEnt *ent, int E,
                                              int T, double *partial) {
  extern __shared__ double sm[];
  const int t = threadIdx.x;
  const int rowlen = p + K * g + K * a;
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = int64_t(blockIdx.x) * chunk;
  const int64_t i1 = i0 + chunk < N ? i0 + chunk : N;
  double acc[kGramEPT];
  GramEnt me[kGramEPT];
#pragma unroll
  for (int q = 0; q < kGramEPT; ++q) {
    acc[q] = 0.0;
    const int e = t + 256 * q;
    me[q] = e < E ? ent[e] : GramEnt{0, 0, -1, 0, 0, 0};
  }
  for (int64_t ib = i0; ib < i1; ib += T) {
    const int nt = int(i1 - ib < T ? i1 - ib : T);
    for (int x = t; x < nt * p; x += 256)
      sm[(x / p) * rowlen + x % p] = X[ib * p + x];
    const int kg = K * g, ka = K * a;
    for (int x = t; x < nt * kg; x += 256)
      sm[(x / kg) * rowlen + p + x % kg] = Y[ib * kg + x];
    for (int x = t; x < nt * ka; x += 256)
      sm[(x / ka) * rowlen + p + kg + x % ka] = Z[ib * ka + x];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGramEPT; ++q) {
      const GramEnt m = me[q];
      if (m.kind < 0) continue;
      double s = acc[q];
      if (m.kind == 0) {
        for (int o = 0; o < nt; ++o) {
          const double *r = sm + o * rowlen;
          s = fma(r[m.oj], r[m.ol], s);
        }
      } else {
        for (int o = 0; o < nt; ++o) {
          const double *r = sm + o * rowlen;
          const double yj = r[m.oj], yl = r[m.ol];
          for (int k = 1; k < K; ++k)
            s = fma(r[m.oj + k * g] - yj, r[m.ol + k * g] - yl, s);
        }
      }
      acc[q] = s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kGramEPT; ++q) {
    const int e = t + 256 * q;
    if (e < E) partial[int64_t(blockIdx.x) * E + e] = acc[q];
  }
}

// Gram entries: the G partials of each entry summed in order, written to
// both of its places
__global__ __launch_bounds__(256) void k_gram_reduce(const double *partial,
                                                     int G, int E,
                                                     const GramEnt *ent,
                                                     double *out) {
  const int e = int(blockIdx.x) * 256 + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int b = 0; b < G; ++b) s += partial[int64_t(b) * E + e];
  out[ent[e].dst] = s;
  out[ent[e].dst2] = s;
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
  // one pass of k_gram when the entries and a staged row fit
  const int64_t rowlen = int64_t(p) + int64_t(K) * (g + a);
  const int64_t E = int64_t(p) * (p + 1) / 2 + int64_t(K) * a * (a + 1) / 2 +
                    int64_t(g) * (g + 1) / 2;
  if (E <= 256 * kGramEPT && rowlen <= 8192) {
    std::vector<GramEnt> ent;
    ent.reserve(size_t(E));
    for (int l = 0; l < p; ++l)
      for (int j = 0; j <= l; ++j)
        ent.push_back({j, l, 0, j + l * p, l + j * p, 0});
    const int zo = p + K * g;
    for (int k = 0; k < K; ++k)
      for (int l = 0; l < a; ++l)
        for (int j = 0; j <= l; ++j) {
          const int base = p * p + k * a * a;
          ent.push_back({zo + k * a + j, zo + k * a + l, 0, base + j + l * a,
                         base + l + j * a, 0});
        }
    for (int l = 0; l < g; ++l)
      for (int j = 0; j <= l; ++j) {
        const int base = p * p + K * a * a;
        ent.push_back({p + j, p + l, 2, base + j + l * g, base + l + j * g,
                       0});
      }
    const int T = int(std::max<int64_t>(1, std::min<int64_t>(16, 8192 / rowlen)));
    const int G = int(std::max<int64_t>(
        1, std::min<int64_t>(512, (N + 4 * T - 1) / (4 * T))));
    void *ev, *pv;
    MNL_TRY(ws_get(c, S_CG, size_t(E) * sizeof(GramEnt) + 8, &ev));
    MNL_TRY(ws_get(c, S_PARTIAL, size_t(G) * size_t(E) * 8, &pv));
    MNL_HIP(c, hipMemcpyAsync(ev, ent.data(), ent.size() * sizeof(GramEnt),
                              hipMemcpyHostToDevice, s));
    const int lds = int(T * rowlen * 8);
    MNL_HIP(c, raise_lds_limit(reinterpret_cast<const void *>(&k_gram), lds));
    hipLaunchKernelGGL(k_gram, dim3(G), dim3(256), lds, s, pr->X, pr->Y, pr->Z,
                       N, p, K, g, a, (const GramEnt *)ev, int(E), T,
                       (double *)pv);
    hipLaunchKernelGGL(k_gram_reduce, dim3(unsigned((E + 255) / 256)),
                       dim3(256), 0, s, (const double *)pv, G, int(E),
                       (const GramEnt *)ev, Gx);
    MNL_HIP(c, hipGetLastError());
    // the host table must outlive its copy
    MNL_HIP(c, hipStreamSynchronize(s));
  } else {
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
    c->xx[0].epoch = ~uint64_t(0);   // the FP64 chi no longer holds its data
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
  }
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
