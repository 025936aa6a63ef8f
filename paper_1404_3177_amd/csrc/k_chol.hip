// Newton direction (Eq. 6): delta = (-H)^{-1} g through the factorisation
// A = -H = L D L^T (L unit lower triangular, D diagonal), always in FP64.
//
// The matrix buffer has n + 1 rows: rows 0..n-1 hold H (row-major), row n
// holds g^T.  Factoring the augmented lower triangle
//     [ A    ]   [ L    ] [ D ] [ L^T  y ]
//     [ g^T  ] = [ y^T  ]
// leaves y = D^{-1} L^{-1} g in row n, so the forward substitution comes out
// of the factorisation and delta = L^{-T} y needs one unit-triangular solve.
// One launch per 32-wide panel (k_chol_step) factors the panel and updates
// the trailing lower triangle with FP64 MFMA; the first launch reads -H
// directly.  Then L^T delta = y by 64-wide panels from the bottom: each
// workgroup re-solves the panel's small unit-triangular system itself and
// updates its share of the remaining right-hand side, so one launch per
// panel suffices and no two workgroups write the same entry.  A failure flag
// in device memory makes every later launch return at once.  In A, the
// diagonal holds D and the strict lower triangle the multipliers of L.
//
// Large systems factor by outer panels of NBO columns: the 32-wide steps
// update only the columns of their outer panel (all rows below), then one
// FP64-MFMA launch (k_chol_syrk) applies L21 (D L21^T) to the lower
// triangle of the trailing square by 128 x 128 tiles, and a small kernel
// applies the update to the g row.  Each trailing entry is then read and
// written once per outer panel instead of once per 32-wide step.
//
// The same factorisation gives the summary's standard errors: with n more
// rows holding the identity below the g row, the augmented factor leaves
// R L^{-T} D^{-1} = L^{-T} D^{-1} =: X in them (the rows are eliminated like
// the g row), and diag((-H)^{-1}) = diag(L^{-T} D^{-1} L^{-1}) is
// sum_k X_ik^2 D_k.
#include <cmath>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NBF = 32;   // factorisation panel width
constexpr int NBS = 64;   // backward-solve panel width
constexpr int TILE = 64;  // trailing-update tile
constexpr int NBO = 256;  // outer panel width of the blocked factorisation
constexpr int64_t kOuterMin = 2048;  // smallest n factored by outer panels

// Round-off floor of the pivots, n * eps * max_k A_kk with A = -H, and g^T
// into row n of the matrix buffer.
__global__ __launch_bounds__(256) void k_floor(double *Hm, int64_t n,
                                               const double *g,
                                               double *floor_out,
                                               int32_t *info) {
  __shared__ double red[256];
  double m = 0.0;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = -Hm[i * n + i];
    if (!isfinite(v)) bad = true;
    m = fmax(m, v);
    Hm[n * n + i] = g ? g[i] : 0.0;
  }
  red[threadIdx.x] = bad ? INFINITY : m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h)
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = red[0];
    *floor_out = double(n) * 2.220446049250313e-16 * mx;
    info[0] = isfinite(mx) ? 0 : 1;
  }
}

// 1 / d to within an ulp: hardware estimate and two Newton steps
__device__ inline double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(e, r, r);
  e = fma(-d, r, 1.0);
  return fma(e, r, r);
}

// One step of the blocked right-looking LDL^T factorisation, panel j0
// (width jb <= NBF), in a single launch.  Workgroup b owns the lower 64x64
// tile (ti, tj) of the trailing rows [j1, nrows) x columns [j1, cend),
// j1 = j0 + jb; tiles are enumerated by rows (the whole lower triangle, when
// tcols covers every tile column) or by the tcols tile columns (an outer
// panel: cend ends it, and at least one tile column exists so that every
// panel row is factored).  Every wave factors the panel's diagonal block itself
// (lanes 0..31 hold its rows) while lanes 32..63 carry 32 panel rows of tile
// row ti (waves 0, 1) or tile column tj (waves 2, 3) through the same column
// steps, so the diagonal factor and the panel's triangular solve are one
// chain with no barrier across waves.  The multiplier rows then feed the
// FP64-MFMA update A22 -= L21 D L21^T of the tile.  The panel's columns are
// only read in this launch: its factor goes to scratch `cur` and the next
// launch (or k_chol_copy) writes it into A, so no workgroup overwrites what
// another still reads.  With neg set (the first panel) rows 0..n-1 of the
// buffer still hold H and every value read from them is negated (row n is
// g itself).  Pivots are checked against the round-off floor.
__global__ __launch_bounds__(256) void k_chol_step(
    double *A, int64_t n, int64_t nrows, int64_t j0, const double *prev,
    int64_t j0p, double *cur, const double *floor_p, int32_t *info, int neg,
    int64_t cend, int64_t tcols) {
  __shared__ double Pr[TILE][NBF + 1];
  __shared__ double Pc[TILE][NBF + 1];
  __shared__ double colb[4][128];
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // one read of the failure flag for the whole workgroup (other workgroups
  // may set it meanwhile), so every wave takes the same branch
  if (tid == 0) fail = info[0];
  __syncthreads();
  if (fail) return;
  const int jb = (int)min<int64_t>(NBF, n - j0);
  const int64_t j1 = j0 + jb;
  const int64_t b = blockIdx.x;
  const int64_t T = (nrows - j1 + TILE - 1) / TILE;
  int64_t ti, tj;
  if (tcols >= T) {
    ti = (int64_t)((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    tj = b - ti * (ti + 1) / 2;
  } else {
    // column tj holds tiles ti = tj .. T-1 (tcols <= NBO / TILE columns)
    int64_t rem = b;
    tj = 0;
    while (rem >= T - tj) {
      rem -= T - tj;
      ++tj;
    }
    ti = tj + rem;
  }
  const int64_t R0 = j1 + ti * TILE, C0 = j1 + tj * TILE;
  const bool same = ti == tj;

  // my row: lanes < 32 a row of the diagonal block (identity past jb),
  // lanes >= 32 a panel row (zero when out of range).  The matrix buffer
  // carries NBF doubles of padding, so all NBF entries of a row can be
  // loaded unconditionally and masked afterwards.
  const bool diag = lane < NBF;
  int64_t prow = -1;
  if (!diag) {
    const int64_t i = int64_t(wv & 1) * 32 + (lane - NBF);
    if (wv < 2) prow = R0 + i < nrows ? R0 + i : -1;
    else if (!same) prow = C0 + i < n ? C0 + i : -1;
  }
  const int ncols = diag ? (lane < jb ? lane + 1 : 0) : (prow >= 0 ? jb : 0);
  const int64_t srow = diag ? j0 + min(lane, jb - 1) : (prow >= 0 ? prow : 0);
  const double sgn = (neg && srow < n) ? -1.0 : 1.0;
  double x[NBF];
  {
    const double *s1 = A + srow * n + j0;
    if (((srow * n + j0) & 1) == 0) {
      const double2 *s2 = reinterpret_cast<const double2 *>(s1);
#pragma unroll
      for (int k = 0; k < NBF / 2; ++k) {
        const double2 v = s2[k];
        x[2 * k] = v.x;
        x[2 * k + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NBF; ++k) x[k] = s1[k];
    }
  }
  // the tile this workgroup updates, loaded while the chain runs
  const bool upd = C0 < cend;
  double tv[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = R0 + 16 * wv + (lane >> 4) + 4 * r;
      const int64_t cc = C0 + 16 * t + (lane & 15);
      tv[t][r] = (upd && rr < nrows && cc < cend && cc <= rr) ? A[rr * n + cc] : 0.0;
    }
#pragma unroll
  for (int k = 0; k < NBF; ++k) {
    const double one = (diag && k == lane) ? 1.0 : 0.0;
    x[k] = k < ncols ? sgn * x[k] : one;
  }
  // column steps, branch-free: lanes publish column k of the diagonal rows
  // through this wave's LDS buffer (lanes >= 32 write to a dummy half; LDS
  // operations of one wave complete in order), every lane forms its
  // multiplier with the reciprocal of the pivot and updates its remaining
  // entries
  const double fl = *floor_p;
  int bad = NBF;
  double dmine = 1.0;
  double *cbw = &colb[wv][0];
#pragma unroll
  for (int k = 0; k < NBF; ++k) {
    cbw[lane] = x[k];
    __builtin_amdgcn_wave_barrier();
    const double dk = cbw[k];
    const bool ok = dk > fl && isfinite(dk);
    bad = (k < jb && !ok && bad == NBF) ? k : bad;
    dmine = lane == k ? dk : dmine;
    const double r = recip(dk);
    const bool act = !diag || lane > k;
    const double l = act ? x[k] * r : 0.0;
#pragma unroll
    for (int j = k + 1; j < NBF; ++j) x[j] = fma(-l, cbw[j], x[j]);
    x[k] = act ? l : x[k];
    __builtin_amdgcn_wave_barrier();
  }
  if (bad < NBF) {
    if (tid == 0) info[0] = int(j0 + bad + 1);
    return;  // the same pivot fails in every wave of every workgroup
  }
  // x now holds the multipliers (and d on a diagonal row's own entry);
  // D goes to this wave's buffer, L21 D to Pr and L21 to Pc
  double *dds = &colb[wv][64];
  if (diag) dds[lane] = dmine;
  __builtin_amdgcn_wave_barrier();
  if (!diag) {
    const int i = (wv & 1) * 32 + (lane - NBF);
    if (wv < 2) {
#pragma unroll
      for (int k = 0; k < NBF; ++k) Pr[i][k] = x[k] * dds[k];
      if (same) {
#pragma unroll
        for (int k = 0; k < NBF; ++k) Pc[i][k] = x[k];
      }
    } else if (!same) {
#pragma unroll
      for (int k = 0; k < NBF; ++k) Pc[i][k] = x[k];
    }
  }
  __syncthreads();
  if (upd) {
    // A[R][C] -= L21[R] D L21[C]^T, lower part
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
    const int ar = 16 * wv + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < NBF / 4; ++ks) {
      const int k = 4 * ks + (lane >> 4);
      const double av = Pr[ar][k];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double bv = Pc[16 * t + (lane & 15)][k];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = R0 + 16 * wv + (lane >> 4) + 4 * r;
        const int64_t cc = C0 + 16 * t + (lane & 15);
        const double sr = (neg && rr < n) ? -1.0 : 1.0;
        if (rr < nrows && cc < cend && cc <= rr)
          A[rr * n + cc] = sr * tv[t][r] - acc[t][r];
      }
    }
  }
  // this panel's factor to scratch
  if (!diag) {
    if (wv < 2 && tj == 0 && prow >= 0) {
      double2 *dst = reinterpret_cast<double2 *>(cur + prow * NBF);
#pragma unroll
      for (int k = 0; k < NBF / 2; ++k) dst[k] = double2{x[2 * k], x[2 * k + 1]};
    }
  } else if (b == 0 && wv == 0 && lane < jb) {
#pragma unroll
    for (int k = 0; k < NBF; ++k)
      if (k <= lane) cur[(j0 + lane) * NBF + k] = x[k];
  }
  // the previous panel's factor into A (columns nobody reads here)
  if (prev) {
    const int64_t cnt = (nrows - j0p) * NBF;
    for (int64_t e = int64_t(blockIdx.x) * 256 + tid; e < cnt;
         e += int64_t(gridDim.x) * 256) {
      const int64_t r = j0p + e / NBF;
      const int k = int(e % NBF);
      if (r - j0p >= NBF || k <= r - j0p) A[r * n + j0p + k] = prev[r * NBF + k];
    }
  }
}

// the last panel's factor into A, and y (row n) into z (if given)
__global__ __launch_bounds__(256) void k_chol_copy(double *A, int64_t n,
                                                   int64_t nrows, int64_t j0p,
                                                   const double *prev,
                                                   double *z,
                                                   const int32_t *info) {
  if (info[0]) return;
  const int64_t cnt = (nrows - j0p) * NBF;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * 256) {
    const int64_t r = j0p + e / NBF;
    const int k = int(e % NBF);
    if (j0p + k < n && (r - j0p >= NBF || k <= r - j0p))
      A[r * n + j0p + k] = prev[r * NBF + k];
  }
  if (!z) return;
  for (int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x; c < n;
       c += int64_t(gridDim.x) * 256)
    z[c] = c >= j0p ? prev[n * NBF + (c - j0p)] : A[n * n + c];
}

// Trailing update of an outer panel on FP64 MFMA:
//   C[r][c] = beta C[r][c] - sum_k A[r][k] B[c][k],  k < kdim,
// row-major operands with strides lda, ldb, ldc; r < M, c < Nc.  One
// workgroup per TE x TE tile of C (lower: only tiles with tile row >=
// tile column, the lower triangle of a symmetric update; the upper part of
// a diagonal tile is written too and never read), four waves of TE/2 x
// TE/2 (16 x 16 MFMA tiles).  The k extent streams through LDS in chunks
// of SYK (k-major, so each fragment read is 16 consecutive doubles), the
// next chunk's loads in registers while this chunk's MFMAs run.  128-wide
// tiles read each operand half as often; 64-wide ones split a small
// trailing square over more workgroups (the launch takes whichever needs
// fewer rounds of MFMA work).
template <int TE>
struct SyrkCfg {
  static constexpr int SYK = TE == 128 ? 8 : 16;   // k chunk
  static constexpr int SYP = TE + 2;   // LDS row length of a k slice
  static constexpr int NF = TE / 32;   // 16-wide fragments per wave edge
  static constexpr int NU = TE / (512 / SYK);   // row passes of a load
};
template <int TE>
__global__ __launch_bounds__(256, TE == 128 ? 2 : 4) void k_chol_syrk(
    const double *Amat, int64_t lda, const double *Bmat, int64_t ldb,
    double *C, int64_t ldc, int64_t M, int64_t Nc, int kdim, double beta,
    int lower, const int32_t *info) {
  using Cf = SyrkCfg<TE>;
  constexpr int SYK = Cf::SYK, SYP = Cf::SYP, NF = Cf::NF, NU = Cf::NU;
  static_assert(NU >= 1 && NU * (512 / SYK) == TE, "load passes");
  __shared__ double As[2][SYK][SYP];
  __shared__ double Bs[2][SYK][SYP];
  if (info[0]) return;
  // tile of this workgroup
  int64_t ti, tj;
  const int64_t b = blockIdx.x;
  if (lower) {
    ti = int64_t((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    tj = b - ti * (ti + 1) / 2;
  } else {
    const int64_t tcn = (Nc + TE - 1) / TE;
    ti = b / tcn;
    tj = b - ti * tcn;
  }
  const int64_t r0 = ti * TE, c0 = tj * TE;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * (TE / 2), wc = (wv & 1) * (TE / 2);
  // loads: thread -> rows tid / (SYK / 2) + (512 / SYK) u, k pair
  // 2 (tid % (SYK / 2)) of a chunk
  constexpr int KP = SYK / 2, RP = 256 / KP;
  const int lr = tid / KP, lk = 2 * (tid % KP);
  double2 ra[NU], rb[NU];
  auto load = [&](int kc) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int64_t r = r0 + lr + RP * u, c = c0 + lr + RP * u;
      ra[u] = r < M ? *reinterpret_cast<const double2 *>(Amat + r * lda + kc + lk)
                    : double2{0.0, 0.0};
      rb[u] = c < Nc ? *reinterpret_cast<const double2 *>(Bmat + c * ldb + kc + lk)
                     : double2{0.0, 0.0};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      As[buf][lk][lr + RP * u] = ra[u].x;
      As[buf][lk + 1][lr + RP * u] = ra[u].y;
      Bs[buf][lk][lr + RP * u] = rb[u].x;
      Bs[buf][lk + 1][lr + RP * u] = rb[u].y;
    }
  };
  d4 acc[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = d4{0, 0, 0, 0};
  const int nch = kdim / SYK;
  load(0);
  store(0);
  __syncthreads();
  const int kb = lane >> 4, l16 = lane & 15;
  for (int ch = 0; ch < nch; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < nch) load((ch + 1) * SYK);
#pragma unroll
    for (int ks = 0; ks < SYK / 4; ++ks) {
      double av[NF], bv[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) av[i] = As[cur][4 * ks + kb][wr + 16 * i + l16];
#pragma unroll
      for (int j = 0; j < NF; ++j) bv[j] = Bs[cur][4 * ks + kb][wc + 16 * j + l16];
#pragma unroll
      for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j],
                                                           acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nch) store(cur ^ 1);
    __syncthreads();
  }
  // lane holds rows (lane >> 4) + 4 q of each 16 x 16 tile, column lane & 15
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int64_t c = c0 + wc + 16 * j + l16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + wr + 16 * i + kb + 4 * q;
        if (r < M && c < Nc) {
          double *cp = C + r * ldc + c;
          *cp = beta * *cp - acc[i][j][q];
        }
      }
    }
}

// Launch the trailing update with the tile edge that finishes first: the
// rounds of resident workgroups (two 128-wide or four 64-wide per CU)
// times the MFMA work a round puts on a CU (a 64-wide tile is a quarter
// of a 128-wide one).
hipError_t launch_syrk(Ctx *c, const double *Amat, int64_t lda,
                       const double *Bmat, int64_t ldb, double *C,
                       int64_t ldc, int64_t M, int64_t Nc, int kdim,
                       double beta, int lower, const int32_t *info,
                       hipStream_t s) {
  // both tile edges take the k extent in whole chunks (8 or 16)
  if (kdim % 16) return hipErrorInvalidValue;
  const int64_t cus = device_cus(c);
  auto tiles = [&](int64_t te) {
    const int64_t tr = (M + te - 1) / te, tc = (Nc + te - 1) / te;
    return lower ? tr * (tr + 1) / 2 : tr * tc;
  };
  const int64_t t128 = tiles(128), t64 = tiles(64);
  const int64_t w128 = 8 * ((t128 + 2 * cus - 1) / (2 * cus));
  const int64_t w64 = 4 * ((t64 + 4 * cus - 1) / (4 * cus));
  if (w64 < w128)
    hipLaunchKernelGGL(k_chol_syrk<64>, dim3((unsigned)t64), dim3(256), 0, s,
                       Amat, lda, Bmat, ldb, C, ldc, M, Nc, kdim, beta, lower,
                       info);
  else
    hipLaunchKernelGGL(k_chol_syrk<128>, dim3((unsigned)t128), dim3(256), 0,
                       s, Amat, lda, Bmat, ldb, C, ldc, M, Nc, kdim, beta,
                       lower, info);
  return hipGetLastError();
}

// Operands of an outer panel's trailing update, columns [J0, J0 + NBO):
// W[i][k] = L[J1 + i][J0 + k] D_k for the trailing rows i < n - J1 (the
// trailing update then forms L21 W^T), and the g row's own update
// A[n][j] -= sum_k L[j][J0 + k] D_k y_k, one wave per column j, the 256
// products summed in a fixed order.  Blocks [0, nbw) form W, the rest the
// g row.
__global__ __launch_bounds__(256) void k_outer_prep(double *A, int64_t n,
                                                    int64_t J0, double *W,
                                                    int64_t nbw,
                                                    const int32_t *info) {
  __shared__ double dy[NBO];
  if (info[0]) return;
  const int64_t J1 = J0 + NBO, m = n - J1;
  const int tid = threadIdx.x;
  if (int64_t(blockIdx.x) < nbw) {
    const int64_t e = int64_t(blockIdx.x) * 256 + tid;
    if (e < m * NBO) {
      const int64_t i = e / NBO;
      const int k = int(e - i * NBO);
      W[e] = A[(J1 + i) * n + J0 + k] * A[(J0 + k) * (n + 1)];
    }
    return;
  }
  // D_k y_k for the wave products
  for (int k = tid; k < NBO; k += 256)
    dy[k] = A[(J0 + k) * (n + 1)] * A[n * n + J0 + k];
  __syncthreads();
  const int lane = tid & 63;
  const int64_t j = J1 + (int64_t(blockIdx.x) - nbw) * 4 + (tid >> 6);
  if (j >= n) return;
  const double *Lj = A + j * n + J0;
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < NBO / 64; ++q) v = fma(Lj[q * 64 + lane], dy[q * 64 + lane], v);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) A[n * n + j] -= v;
}

// Rows n + 1 .. 2n of the matrix buffer := the identity (row n + 1 + i
// holds e_i^T).
__global__ __launch_bounds__(256) void k_eye_rows(double *A, int64_t n) {
  const int64_t cnt = n * n;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < cnt;
       e += int64_t(gridDim.x) * 256) {
    const int64_t i = e / n, j = e - i * n;
    A[(n + 1) * n + e] = i == j ? 1.0 : 0.0;
  }
}

// Standard errors from the augmented factor: one wave per coefficient i,
// v_i = sum_{k >= i} X_ik^2 D_k over row n + 1 + i (X_ik = 0 for k < i),
// lane-strided partial sums combined by a fixed butterfly.  se = sqrt(v),
// z = theta / se, p = erfc(|z| / sqrt 2) (z and p optional).
__global__ __launch_bounds__(256) void k_inv_diag(const double *A, int64_t n,
                                                  const double *theta,
                                                  double *se, double *zv,
                                                  double *pv,
                                                  const int32_t *info) {
  if (info[0]) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double *xr = A + (n + 1 + i) * n;
  double v = 0.0;
  for (int64_t k = i + lane; k < n; k += 64) {
    const double x = xr[k];
    v = fma(x * x, A[k * (n + 1)], v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) {
    const double s = sqrt(v);
    se[i] = s;
    const double z = theta[i] / s;
    if (zv) zv[i] = z;
    if (pv) pv[i] = erfc(fabs(z) * 0.70710678118654752440);
  }
}

// Covariance entries from the augmented factor: V[a][b] =
// sum_k X[ia][k] X[ib][k] D_k over k >= max(ia, ib) (X = L^{-T} D^{-1}
// upper triangular), one wave per entry; the products commute, so
// V[a][b] and V[b][a] are bitwise equal.
__global__ __launch_bounds__(256) void k_cov_sub(const double *A, int64_t n,
                                                 const int32_t *idx, int s,
                                                 double *V,
                                                 const int32_t *info) {
  if (info[0]) return;
  const int lane = threadIdx.x & 63;
  const int64_t e = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (e >= int64_t(s) * s) return;
  const int a = int(e / s), b = int(e - int64_t(a) * s);
  const int64_t ia = idx[a], ib = idx[b];
  const double *xa = A + (n + 1 + ia) * n, *xb = A + (n + 1 + ib) * n;
  double v = 0.0;
  for (int64_t k = (ia > ib ? ia : ib) + lane; k < n; k += 64)
    v = fma(xa[k] * xb[k], A[k * (n + 1)], v);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) V[e] = v;
}

// out = sgn (A - B) for n x n matrices (B optional), then the vector
// x - x0 (x0 optional) into out[n^2 ..] (the g row of the buffer)
__global__ __launch_bounds__(256) void k_signed_copy(const double *A,
                                                     const double *B,
                                                     const double *x,
                                                     const double *x0,
                                                     double sgn, int64_t n,
                                                     double *out) {
  const int64_t cnt = n * n;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < cnt + n;
       e += int64_t(gridDim.x) * 256) {
    if (e < cnt) {
      out[e] = sgn * (B ? A[e] - B[e] : A[e]);
    } else {
      const int64_t j = e - cnt;
      out[e] = x0 ? x[j] - x0[j] : x[j];
    }
  }
}

// x^T A^{-1} x = sum_k D_k y_k^2 with y = D^{-1} L^{-1} x the factor's g
// row; one workgroup, fixed-order tree
__global__ __launch_bounds__(256) void k_quad(const double *A, int64_t n,
                                              double *out,
                                              const int32_t *info) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double v = 0.0;
  if (!info[0])
    for (int64_t k = t; k < n; k += 256) {
      const double y = A[n * n + k];
      v = fma(y * y, A[k * (n + 1)], v);
    }
  red[t] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0];
}

__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), l);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), l);
  return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}

// backward substitution L^T delta = y, panel j0 (jb <= NBS rows): every
// workgroup solves the panel's unit-triangular system in one wave (lane t
// holds column t of the panel's L in registers, delta_c is broadcast by
// readlane), then subtracts L[panel][c]^T delta_panel from its 64-column
// chunk of z (four row groups, summed in a fixed order).  Every load is
// issued at the start, so the chain and the update wait on one round trip.
__global__ __launch_bounds__(256) void k_chol_bwd(const double *A, int64_t n,
                                                  int64_t j0, double *z,
                                                  double *delta,
                                                  const int32_t *info) {
  __shared__ double dp[NBS];
  __shared__ double part[4][64];
  if (info[0]) return;
  const int jb = (int)min<int64_t>(NBS, n - j0);
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  // this thread's share of the update: column c, rows grp, grp + 4, ...
  const int64_t c = int64_t(blockIdx.x) * 64 + lane;
  double av[NBS / 4];
#pragma unroll
  for (int u = 0; u < NBS / 4; ++u) {
    const int r = grp + 4 * u;
    av[u] = (c < j0 && r < jb) ? A[(j0 + r) * n + c] : 0.0;
  }
  if (grp == 0) {
    double lcol[NBS];
#pragma unroll
    for (int cc = 0; cc < NBS; ++cc)
      lcol[cc] = (cc < jb && lane < cc) ? A[(j0 + cc) * n + j0 + lane] : 0.0;
    // rows past jb are identity rows, so the chain always has NBS steps
    double zt = lane < jb ? z[j0 + lane] : 0.0;
    double dl = 0.0;
#pragma unroll
    for (int cc = NBS - 1; cc >= 0; --cc) {
      const double dc = readlane_f64(zt, cc);
      dl = lane == cc ? dc : dl;
      zt = fma(-lcol[cc], dc, zt);
    }
    dp[lane] = dl;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < jb) delta[j0 + tid] = dp[tid];
  double s2[2] = {0.0, 0.0};
#pragma unroll
  for (int u = 0; u < NBS / 4; ++u) s2[u & 1] = fma(av[u], dp[grp + 4 * u], s2[u & 1]);
  part[grp][lane] = s2[0] + s2[1];
  __syncthreads();
  if (grp == 0 && c < j0)
    z[c] -= (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

}  // namespace

size_t chol_workspace_bytes(int64_t n, int64_t extra) {
  const int64_t nrows = n + 1 + extra;
  const int64_t w = n >= kOuterMin ? (n - NBO) * NBO : 0;
  return size_t(n + 8 + 2 * nrows * NBF + w) * 8;
}

int chol_solve_run(Ctx *c, double *A, int64_t n, const double *g,
                   double *delta, int32_t *info, hipStream_t s,
                   int64_t extra) {
  void *scr;
  if (extra != 0 && extra != n)
    return set_error(c, MNL_ERR_ARG, "identity rows must number n");
  const int64_t nrows = n + 1 + extra;
  const bool outer = n >= kOuterMin;
  // two panel buffers of nrows x NBF (each a multiple of 256 bytes, so
  // both stay 16-byte aligned), z, floor, then W of the outer panels
  MNL_TRY(ws_get(c, S_CHOL, chol_workspace_bytes(n, extra), &scr));
  double *pbuf[2] = {static_cast<double *>(scr),
                     static_cast<double *>(scr) + nrows * NBF};
  double *z = pbuf[1] + nrows * NBF;
  double *floor_p = z + n;
  double *W = floor_p + 8;
  hipLaunchKernelGGL(k_floor, dim3(1), dim3(256), 0, s, A, n, g, floor_p,
                     info);
  if (extra) {
    const unsigned gr = (unsigned)std::min<int64_t>(4096, (n * n + 255) / 256);
    hipLaunchKernelGGL(k_eye_rows, dim3(gr), dim3(256), 0, s, A, n);
  }
  int step = 0;
  int64_t j0p = -1;
  const int64_t wo = outer ? NBO : n;
  for (int64_t J0 = 0; J0 < n; J0 += wo) {
    const int64_t J1 = std::min<int64_t>(n, J0 + wo);
    const bool last_outer = J1 == n;
    for (int64_t j0 = J0; j0 < J1; j0 += NBF, ++step) {
      const int64_t jb = std::min<int64_t>(NBF, n - j0);
      const int64_t rest = nrows - j0 - jb;   // >= 1: the g row
      const int64_t T = (rest + TILE - 1) / TILE;
      // inside an outer panel only its own columns are updated
      const int64_t tc =
          last_outer ? T
                     : std::max<int64_t>(1, (J1 - j0 - jb + TILE - 1) / TILE);
      const int64_t nblk = tc >= T ? T * (T + 1) / 2 : tc * T - tc * (tc - 1) / 2;
      const double *prev = j0p >= 0 ? pbuf[(step - 1) & 1] : nullptr;
      hipLaunchKernelGGL(k_chol_step, dim3((unsigned)nblk), dim3(256), 0, s, A,
                         n, nrows, j0, prev, j0p, pbuf[step & 1], floor_p,
                         info, j0 == 0 ? 1 : 0, last_outer ? n : J1, tc);
      j0p = j0;
    }
    if (last_outer) break;
    // close the outer panel: its last step's factor into A, the operands of
    // the trailing update, then A22 -= L21 D L21^T on the lower triangle
    // (the first panel's trailing block still holds H: beta = -1 forms
    // A = -H on the way)
    {
      const int64_t cnt = (nrows - j0p) * NBF;
      const unsigned gr = (unsigned)std::min<int64_t>(1024, (cnt + 255) / 256);
      hipLaunchKernelGGL(k_chol_copy, dim3(gr), dim3(256), 0, s, A, n, nrows,
                         j0p, pbuf[(step - 1) & 1], (double *)nullptr, info);
      j0p = -1;
    }
    const int64_t m = n - J1;
    const int64_t nbw = (m * NBO + 255) / 256, nbg = (m + 3) / 4;
    hipLaunchKernelGGL(k_outer_prep, dim3((unsigned)(nbw + nbg)), dim3(256), 0,
                       s, A, n, J0, W, nbw, info);
    const double beta = J0 == 0 ? -1.0 : 1.0;
    MNL_HIP(c, launch_syrk(c, A + J1 * n + J0, n, W, int64_t(NBO),
                           A + J1 * n + J1, n, m, m, NBO, beta, 1, info, s));
    if (extra) {
      // identity rows: X[:, J1:n] -= X[:, J0:J1] (L21 D)^T, the same update
      // as the g row's (these rows are never negated, so beta = 1)
      double *Xr = A + (n + 1) * n;
      MNL_HIP(c, launch_syrk(c, Xr + J0, n, W, int64_t(NBO), Xr + J1, n,
                             extra, m, NBO, 1.0, 0, info, s));
    }
  }
  {
    const int64_t cnt = std::max<int64_t>((nrows - j0p) * NBF, n);
    const unsigned gr = (unsigned)std::min<int64_t>(1024, (cnt + 255) / 256);
    hipLaunchKernelGGL(k_chol_copy, dim3(gr), dim3(256), 0, s, A, n, nrows,
                       j0p, pbuf[(step - 1) & 1], delta ? z : nullptr, info);
  }
  if (!delta) {
    MNL_HIP(c, hipGetLastError());
    return MNL_OK;
  }
  const int64_t last = ((n - 1) / NBS) * NBS;
  for (int64_t j0 = last; j0 >= 0; j0 -= NBS) {
    const unsigned gr = (unsigned)std::max<int64_t>(1, (j0 + 63) / 64);
    hipLaunchKernelGGL(k_chol_bwd, dim3(gr), dim3(256), 0, s, A, n, j0, z,
                       delta, info);
  }
  MNL_HIP(c, hipGetLastError());
  return MNL_OK;
}

hipError_t launch_cov_sub(const double *A, int64_t n, const int32_t *idx,
                          int s, double *V, const int32_t *info,
                          hipStream_t st) {
  const int64_t waves = int64_t(s) * s;
  hipLaunchKernelGGL(k_cov_sub, dim3((unsigned)((waves + 3) / 4)), dim3(256),
                     0, st, A, n, idx, s, V, info);
  return hipGetLastError();
}

hipError_t launch_signed_copy(const double *A, const double *B,
                              const double *x, const double *x0, double sgn,
                              int64_t n, double *out, hipStream_t s) {
  const unsigned gr = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>(4096, (n * n + n + 255) / 256));
  hipLaunchKernelGGL(k_signed_copy, dim3(gr), dim3(256), 0, s, A, B, x, x0,
                     sgn, n, out);
  return hipGetLastError();
}

hipError_t launch_quad(const double *A, int64_t n, double *out,
                       const int32_t *info, hipStream_t s) {
  hipLaunchKernelGGL(k_quad, dim3(1), dim3(256), 0, s, A, n, out, info);
  return hipGetLastError();
}

hipError_t launch_inv_diag(const double *A, int64_t n, const double *theta,
                           double *se, double *z, double *pval,
                           const int32_t *info, hipStream_t s) {
  const unsigned gr = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL(k_inv_diag, dim3(gr), dim3(256), 0, s, A, n, theta, se,
                     z, pval, info);
  return hipGetLastError();
}

}  // namespace mnl
