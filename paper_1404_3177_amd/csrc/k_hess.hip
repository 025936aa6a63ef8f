// Block Hessian of the multinomial-logit log-likelihood (Eq. 10).
//
// With phi_ik the features that alternative k's coefficients see
// (x_i for beta_k, z_ik for gamma_k), every alternative-specific block is
//   H_nm = -sum_i w_i P_in (delta_nm - P_im) phi_in phi_im^T        (Eq. 10)
// and the generic (alpha) blocks take the centred form obtained from Eq. 10
// with sum_k P_ik = 1 (App. A derivation):
//   H_{beta_n,alpha}  = -X^T D(w P_n) (Y_n - Ybar)
//   H_{gamma_n,alpha} = -Z_n^T D(w P_n) (Y_n - Ybar)
//   H_{alpha,alpha}   = -sum_i w_i sum_k P_ik (y_ik - ybar_i)(y_ik - ybar_i)^T
//
// Work split (A = -H is accumulated, H written at the end):
//  * BB tiles (beta-beta, the bulk): one GEMM C = Omega^T (X o X) whose
//    rows are alternative pairs n <= m (omega_i = w P_n (delta - P_m)) and
//    whose columns are feature pairs a <= b (x_a x_b).  Both operands are
//    generated on the fly from LDS-staged P and X, so each block's two
//    symmetries (H_nm = H_mn^T and X^T W X symmetric) are used and the
//    per-observation weights W_nm are never stored.
//  * XG tiles (beta-gamma and gamma-gamma): C = sum_i (w P_n phi_n)(P_m z_m)
//    for rows over all alternative-specific coefficients and columns over
//    the gamma coefficients (upper triangle only for gamma-gamma).
//  * per-alternative kernel: the delta_nm parts of the XG blocks
//    (sum_i w P_n phi_n z_n^T) and all alpha blocks.
// Tiles of both GEMM kinds run in one launch on MFMA (FP64, FP32 or BF16
// operands), split over observations; the split partials are summed in a
// fixed order, so the result is reproducible.
#include <algorithm>
#include <map>
#include <tuple>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kRows = 64;        // rows per workgroup tile (4 waves x 16)
constexpr int kTN = 4;           // 16-column MFMA tiles per wave
constexpr int kCols = 16 * kTN;  // columns per workgroup tile
constexpr int kMaxCols = 128;    // staged alternatives per BB row tile

enum TileType { T_BB = 0, T_XG = 1 };

struct Tile {
  int32_t type, row0, col0, split;
  int32_t obs0, obs1, pad0, pad1;
};

// MFMA traits --------------------------------------------------------------
template <int PREC> struct MF;
template <> struct MF<0> {
  using T = double;       // staged operand type
  using Acc = d4;
  static constexpr int KSTEP = 4, KC = 16;
  __device__ static int out_row(int l, int r) { return (l >> 4) + 4 * r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <> struct MF<1> {
  using T = float;
  using Acc = f4;
  static constexpr int KSTEP = 4, KC = 32;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <> struct MF<2> {
  using T = float;
  using Acc = f4;
  static constexpr int KSTEP = 32, KC = 64;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};

struct HessDev {
  Dims d;
  const double *X, *Z, *w;
  const double *P;
  const float *P32;
  const Tile *tiles;
  // BB tables
  const int32_t *bb_cols;    // [n_row_tiles][kMaxCols]
  const int32_t *bb_ncol;    // [n_row_tiles]
  const uint32_t *bb_row;    // per pair row: ln | lm << 8 | diag << 16 | valid << 17
  const uint32_t *bb_combo;  // per combo col: a | b << 16 (0xffffffff = pad)
  int64_t bb_M, bb_N;        // padded partial dims
  int64_t xg_M, xg_N;
  void *part_bb, *part_xg;   // [S][M][N] accumulator type
  int64_t nrow_bb, ncombo;   // valid rows / cols
  int64_t nrow_xg, ncol_xg;
};

template <int PREC>
__device__ inline typename MF<PREC>::Acc mfma_step(
    typename MF<PREC>::Acc c, const float *av, const float *bv);

template <typename T>
__device__ inline T ldg_op(const double *p64, const float *p32, int64_t idx);
template <>
__device__ inline double ldg_op<double>(const double *p64, const float *,
                                        int64_t idx) {
  return p64[idx];
}
template <>
__device__ inline float ldg_op<float>(const double *p64, const float *p32,
                                      int64_t idx) {
  return p32 ? p32[idx] : (float)p64[idx];
}

// Generated-operand GEMM over a tile list.
template <int PREC>
__global__ __launch_bounds__(kThreads) void k_hess_tiles(HessDev H) {
  using M = MF<PREC>;
  using T = typename M::T;
  extern __shared__ double smd[];
  T *sm = reinterpret_cast<T *>(smd);
  const Tile tile = H.tiles[blockIdx.x];
  const Dims d = H.d;
  const int K = d.K, p = d.p, a = d.a;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int KC = M::KC;
  const int lrow = 16 * wv + (lane & 15);      // generation row in tile
  const int row = tile.row0 + lrow;
  typename M::Acc acc[kTN];
#pragma unroll
  for (int t = 0; t < kTN; ++t) acc[t] = M::zero();

  if (tile.type == T_BB) {
    const int rt = tile.row0 / kRows;
    const int ncol = H.bb_ncol[rt];
    const int32_t *cols = H.bb_cols + int64_t(rt) * kMaxCols;
    // LDS: Ps[KC][kMaxCols], Xs[KC][p], ws[KC]
    T *Ps = sm;
    T *Xs = Ps + KC * kMaxCols;
    T *Ws = Xs + KC * p;
    const uint32_t rinfo = (row < H.nrow_bb) ? H.bb_row[row] : 0u;
    const int ln = rinfo & 0xff, lm = (rinfo >> 8) & 0xff;
    const T dg = (rinfo >> 16) & 1 ? T(1) : T(0);
    const bool rvalid = (rinfo >> 17) & 1;
    int ca[kTN], cb[kTN];
#pragma unroll
    for (int t = 0; t < kTN; ++t) {
      const int col = tile.col0 + 16 * t + (lane & 15);
      uint32_t ci = (col < H.ncombo) ? H.bb_combo[col] : 0xffffffffu;
      ca[t] = (ci == 0xffffffffu) ? -1 : int(ci & 0xffff);
      cb[t] = (ci == 0xffffffffu) ? -1 : int(ci >> 16);
    }
    for (int i0 = tile.obs0; i0 < tile.obs1; i0 += KC) {
      const int nobs = min(KC, tile.obs1 - i0);
      for (int idx = tid; idx < KC * ncol; idx += kThreads) {
        const int j = idx / ncol, c = idx - j * ncol;
        Ps[j * kMaxCols + c] =
            j < nobs ? ldg_op<T>(H.P, H.P32, int64_t(i0 + j) * K + cols[c])
                     : T(0);
      }
      for (int idx = tid; idx < KC * p; idx += kThreads) {
        const int j = idx / p, f = idx - j * p;
        Xs[idx] = j < nobs ? T(d.N > 0 ? H.X[int64_t(i0 + j) * p + f] : 0)
                           : T(0);
      }
      for (int j = tid; j < KC; j += kThreads)
        Ws[j] = j < nobs ? T(H.w ? H.w[i0 + j] : 1.0) : T(0);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KC / M::KSTEP; ++ks) {
        if constexpr (PREC == 2) {
          const int jb = ks * 32 + 8 * (lane >> 4);
          bf8 av;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int j = jb + q;
            float om = rvalid ? Ws[j] * Ps[j * kMaxCols + ln] *
                                    (dg - Ps[j * kMaxCols + lm])
                              : 0.0f;
            av[q] = (__bf16)om;
          }
#pragma unroll
          for (int t = 0; t < kTN; ++t) {
            bf8 bv;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int j = jb + q;
              float xx = ca[t] >= 0 ? Xs[j * p + ca[t]] * Xs[j * p + cb[t]]
                                    : 0.0f;
              bv[q] = (__bf16)xx;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t],
                                                             0, 0, 0);
          }
        } else {
          const int j = ks * 4 + (lane >> 4);
          const T om = rvalid ? Ws[j] * Ps[j * kMaxCols + ln] *
                                    (dg - Ps[j * kMaxCols + lm])
                              : T(0);
#pragma unroll
          for (int t = 0; t < kTN; ++t) {
            const T xx = ca[t] >= 0 ? Xs[j * p + ca[t]] * Xs[j * p + cb[t]]
                                    : T(0);
            if constexpr (PREC == 0)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(om, xx, acc[t], 0,
                                                            0, 0);
            else
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(om, xx, acc[t], 0,
                                                            0, 0);
          }
        }
      }
      __syncthreads();
    }
  } else {  // T_XG
    // LDS: Ps[KC][K], Xs[KC][p], Zs[KC][K*a], ws[KC]
    T *Ps = sm;
    T *Xs = Ps + KC * K;
    T *Zs = Xs + KC * p;
    T *Ws = Zs + KC * K * a;
    const int64_t nbrow = int64_t(K - 1) * p;
    // A row: w P_n phi_nf
    int an = 0, af = 0;
    bool arow_z = false, avalid = row < H.nrow_xg;
    if (avalid) {
      if (row < nbrow) {
        an = 1 + row / p;
        af = row - (an - 1) * p;
      } else {
        const int r2 = int(row - nbrow);
        an = r2 / a;
        af = r2 - an * a;
        arow_z = true;
      }
    }
    int bm[kTN], bc[kTN];
#pragma unroll
    for (int t = 0; t < kTN; ++t) {
      const int col = tile.col0 + 16 * t + (lane & 15);
      if (col < H.ncol_xg) {
        bm[t] = col / a;
        bc[t] = col - bm[t] * a;
      } else {
        bm[t] = -1;
        bc[t] = 0;
      }
    }
    for (int i0 = tile.obs0; i0 < tile.obs1; i0 += KC) {
      const int nobs = min(KC, tile.obs1 - i0);
      for (int idx = tid; idx < KC * K; idx += kThreads) {
        const int j = idx / K;
        Ps[idx] = j < nobs ? ldg_op<T>(H.P, H.P32, int64_t(i0) * K + idx)
                           : T(0);
      }
      for (int idx = tid; idx < KC * p; idx += kThreads) {
        const int j = idx / p;
        Xs[idx] = j < nobs ? T(H.X[int64_t(i0) * p + idx]) : T(0);
      }
      const int za = K * a;
      for (int idx = tid; idx < KC * za; idx += kThreads) {
        const int j = idx / za;
        Zs[idx] = j < nobs ? T(H.Z[int64_t(i0) * za + idx]) : T(0);
      }
      for (int j = tid; j < KC; j += kThreads)
        Ws[j] = j < nobs ? T(H.w ? H.w[i0 + j] : 1.0) : T(0);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < KC / M::KSTEP; ++ks) {
        if constexpr (PREC == 2) {
          const int jb = ks * 32 + 8 * (lane >> 4);
          bf8 av;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int j = jb + q;
            float v = 0.0f;
            if (avalid)
              v = Ws[j] * Ps[j * K + an] *
                  (arow_z ? Zs[(j * K + an) * a + af] : Xs[j * p + af]);
            av[q] = (__bf16)v;
          }
#pragma unroll
          for (int t = 0; t < kTN; ++t) {
            bf8 bv;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int j = jb + q;
              float v = bm[t] >= 0
                            ? Ps[j * K + bm[t]] * Zs[(j * K + bm[t]) * a + bc[t]]
                            : 0.0f;
              bv[q] = (__bf16)v;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t],
                                                             0, 0, 0);
          }
        } else {
          const int j = ks * 4 + (lane >> 4);
          T av = T(0);
          if (avalid)
            av = Ws[j] * Ps[j * K + an] *
                 (arow_z ? Zs[(j * K + an) * a + af] : Xs[j * p + af]);
#pragma unroll
          for (int t = 0; t < kTN; ++t) {
            const T bv = bm[t] >= 0
                             ? Ps[j * K + bm[t]] * Zs[(j * K + bm[t]) * a + bc[t]]
                             : T(0);
            if constexpr (PREC == 0)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0,
                                                            0, 0);
            else
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0,
                                                            0, 0);
          }
        }
      }
      __syncthreads();
    }
  }

  // epilogue: this split's partial tile
  using AccT = typename std::conditional<PREC == 0, double, float>::type;
  AccT *part;
  int64_t Mp, Np;
  if (tile.type == T_BB) {
    part = reinterpret_cast<AccT *>(H.part_bb);
    Mp = H.bb_M;
    Np = H.bb_N;
  } else {
    part = reinterpret_cast<AccT *>(H.part_xg);
    Mp = H.xg_M;
    Np = H.xg_N;
  }
  AccT *base = part + (int64_t(tile.split) * Mp + tile.row0 + 16 * wv) * Np +
               tile.col0;
#pragma unroll
  for (int t = 0; t < kTN; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = M::out_row(lane, r);
      const int ocol = 16 * t + (lane & 15);
      base[int64_t(orow) * Np + ocol] = acc[t][r];
    }
  }
}

// Per-alternative sums for the delta_nm parts and the alpha blocks:
//   out[n][r][s] = sum_i w_i P_in L_in[r] R_in[s]
// with L = (x_i, z_in, y_in - ybar_i), R = (z_in, y_in - ybar_i).
// Workgroup: alternatives [n0, n0 + nb) x one observation range; each
// thread owns up to kJ outputs.
constexpr int kJ = 8;
constexpr int kAltTB = 16;

__global__ __launch_bounds__(kThreads) void k_hess_alt(
    Dims d, const double *X, const double *Y, const double *Z,
    const double *w, const double *P, const double *Ybar, int nb,
    int64_t obs_chunk, double *out /* [S][K][nl][nr] */) {
  extern __shared__ double sm[];
  const int K = d.K, p = d.p, g = d.g, a = d.a;
  const int nl = p + a + g, nr = a + g;
  const int n0 = blockIdx.x * nb;
  const int nbe = min(nb, K - n0);
  const int64_t i_begin = int64_t(blockIdx.y) * obs_chunk;
  const int64_t i_end = min(d.N, i_begin + obs_chunk);
  // LDS: L[kAltTB][nb][nl] (u * L) and R[kAltTB][nb][nr]
  double *Ls = sm;
  double *Rs = Ls + kAltTB * nb * nl;
  const int tid = threadIdx.x;
  const int nout = nbe * nl * nr;
  double acc[kJ];
#pragma unroll
  for (int j = 0; j < kJ; ++j) acc[j] = 0.0;
  for (int64_t i0 = i_begin; i0 < i_end; i0 += kAltTB) {
    const int nobs = (int)min<int64_t>(kAltTB, i_end - i0);
    // stage u*L and R for every (obs, alternative)
    for (int idx = tid; idx < kAltTB * nbe; idx += kThreads) {
      const int j = idx / nbe, q = idx - j * nbe;
      const int n = n0 + q;
      double *L = Ls + (j * nb + q) * nl;
      double *Rr = Rs + (j * nb + q) * nr;
      if (j >= nobs) {
        for (int r = 0; r < nl; ++r) L[r] = 0.0;
        for (int r = 0; r < nr; ++r) Rr[r] = 0.0;
        continue;
      }
      const int64_t i = i0 + j;
      const double u = (w ? w[i] : 1.0) * P[i * K + n];
      for (int f = 0; f < p; ++f) L[f] = u * X[i * p + f];
      for (int c = 0; c < a; ++c) {
        const double z = Z[(i * K + n) * a + c];
        L[p + c] = u * z;
        Rr[c] = z;
      }
      for (int c = 0; c < g; ++c) {
        const double yc = Y[(i * K + n) * g + c] - Ybar[i * g + c];
        L[p + a + c] = u * yc;
        Rr[a + c] = yc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int o = tid + jj * kThreads;
      if (o < nout) {
        const int q = o / (nl * nr);
        const int rem = o - q * nl * nr;
        const int r = rem / nr, s = rem - (rem / nr) * nr;
        double sacc = acc[jj];
        for (int j = 0; j < nobs; ++j)
          sacc = fma(Ls[(j * nb + q) * nl + r], Rs[(j * nb + q) * nr + s],
                     sacc);
        acc[jj] = sacc;
      }
    }
    __syncthreads();
  }
  double *ob = out + (int64_t(blockIdx.y) * K + n0) * nl * nr;
#pragma unroll
  for (int jj = 0; jj < kJ; ++jj) {
    const int o = tid + jj * kThreads;
    if (o < nout) ob[o] = acc[jj];
  }
}

// ---- assembly into H (Hessian sign) ----------------------------------------------

template <typename AccT>
__global__ void k_assemble_bb(Dims d, const AccT *part, int S, int64_t Mp,
                              int64_t Np, const int32_t *pair_nm,
                              const uint32_t *combo, int64_t nrow,
                              int64_t ncombo, double *Hm) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nrow * ncombo) return;
  const int64_t r = e / ncombo, q = e - (e / ncombo) * ncombo;
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += (double)part[(int64_t(s) * Mp + r) * Np + q];
  const int n = pair_nm[r] & 0xffff, m = pair_nm[r] >> 16;
  const int fa = combo[q] & 0xffff, fb = combo[q] >> 16;
  const int64_t np = d.np, p = d.p;
  const int64_t ra = (n - 1) * p + fa, rb = (n - 1) * p + fb;
  const int64_t ca = (m - 1) * p + fa, cb = (m - 1) * p + fb;
  v = -v;
  Hm[ra * np + cb] = v;
  Hm[rb * np + ca] = v;
  Hm[cb * np + ra] = v;
  Hm[ca * np + rb] = v;
}

template <typename AccT>
__global__ void k_assemble_xg(Dims d, const AccT *part, int S, int64_t Mp,
                              int64_t Np, const double *alt, int Salt,
                              double *Hm) {
  const int64_t nrow = int64_t(d.K - 1) * d.p + int64_t(d.K) * d.a;
  const int64_t ncol = int64_t(d.K) * d.a;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nrow * ncol) return;
  const int64_t r = e / ncol, c = e - (e / ncol) * ncol;
  const int64_t offg = d.off_gamma();
  const int64_t gc = offg + c;
  if (r >= offg && r > gc) return;  // lower gamma-gamma triangle: mirrored
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += (double)part[(int64_t(s) * Mp + r) * Np + c];
  // delta_nm term of the same-alternative block
  const int m = int(c / d.a), cz = int(c - (c / d.a) * d.a);
  int n, rl;
  if (r < offg) {
    n = 1 + int(r / d.p);
    rl = int(r - int64_t(n - 1) * d.p);
  } else {
    n = int((r - offg) / d.a);
    rl = d.p + int(r - offg - int64_t(n) * d.a);
  }
  if (n == m) {
    const int nl = d.p + d.a + d.g, nr = d.a + d.g;
    double dsum = 0.0;
    for (int s = 0; s < Salt; ++s)
      dsum += alt[((int64_t(s) * d.K + n) * nl + rl) * nr + cz];
    v -= dsum;
  }
  const int64_t np = d.np;
  Hm[r * np + gc] = v;
  Hm[gc * np + r] = v;
}

// alpha rows/cols: beta-alpha, gamma-alpha, alpha-alpha
__global__ void k_assemble_alpha(Dims d, const double *alt, int Salt,
                                 double *Hm) {
  const int64_t offg = d.off_gamma(), offa = d.off_alpha();
  const int64_t np = d.np;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= offa * d.g + int64_t(d.g) * d.g) return;
  const int nl = d.p + d.a + d.g, nr = d.a + d.g;
  if (e < offa * d.g) {
    const int64_t r = e / d.g;
    const int c = int(e - r * d.g);
    int n, rl;
    if (r < offg) {
      n = 1 + int(r / d.p);
      rl = int(r - int64_t(n - 1) * d.p);
    } else {
      n = int((r - offg) / d.a);
      rl = d.p + int(r - offg - int64_t(n) * d.a);
    }
    double v = 0.0;
    for (int s = 0; s < Salt; ++s)
      v += alt[((int64_t(s) * d.K + n) * nl + rl) * nr + d.a + c];
    Hm[r * np + offa + c] = -v;
    Hm[(offa + c) * np + r] = -v;
  } else {
    const int64_t q = e - offa * d.g;
    const int c1 = int(q / d.g), c2 = int(q - (q / d.g) * d.g);
    if (c1 > c2) return;  // written by its mirror
    double v = 0.0;
    for (int s = 0; s < Salt; ++s)
      for (int n = 0; n < d.K; ++n)
        v += alt[((int64_t(s) * d.K + n) * nl + d.p + d.a + c1) * nr + d.a +
                 c2];
    Hm[(offa + c1) * np + offa + c2] = -v;
    Hm[(offa + c2) * np + offa + c1] = -v;
  }
}

// ---- host-side plan -------------------------------------------------------------

struct Plan {
  Dims d;
  int prec;
  int S = 1;                     // observation splits of the GEMM tiles
  int ntiles = 0;
  int64_t bb_M = 0, bb_N = 0, xg_M = 0, xg_N = 0;
  int64_t nrow_bb = 0, ncombo = 0, nrow_xg = 0, ncol_xg = 0;
  size_t lds = 0;
  // alt kernel
  int alt_nb = 1, alt_S = 1;
  int64_t alt_chunk = 0;
  size_t alt_lds = 0;
  bool need_alt = false;
  // device tables (one allocation)
  void *dev = nullptr;
  size_t dev_bytes = 0;
  Tile *tiles = nullptr;
  int32_t *bb_cols = nullptr, *bb_ncol = nullptr, *pair_nm = nullptr;
  uint32_t *bb_row = nullptr, *bb_combo = nullptr;
};

using Key = std::tuple<int64_t, int, int, int, int, int>;
struct Cache {
  std::map<Key, Plan *> plans;
};

int build_plan(Ctx *c, const Dims &d, int prec, Plan **out) {
  if (!c->hess_cache) c->hess_cache = new Cache;
  Cache *cache = static_cast<Cache *>(c->hess_cache);
  Key key{d.N, d.K, d.p, d.g, d.a, prec};
  auto it = cache->plans.find(key);
  if (it != cache->plans.end()) {
    *out = it->second;
    return MNL_OK;
  }
  if (d.p > 255 || d.K > 32767)
    return set_error(c, MNL_ERR_UNSUPPORTED, "Hessian tiles need p <= 255");
  Plan *pl = new Plan;
  pl->d = d;
  pl->prec = prec;
  const int KC = prec == 0 ? MF<0>::KC : (prec == 1 ? MF<1>::KC : MF<2>::KC);
  const int K = d.K, p = d.p, a = d.a, g = d.g;

  // BB rows: pairs n <= m over alternatives 1..K-1, row-major
  std::vector<int32_t> pair_nm;
  for (int n = 1; n < K; ++n)
    for (int m = n; m < K; ++m) pair_nm.push_back(n | (m << 16));
  const int64_t nrow_bb = p > 0 ? int64_t(pair_nm.size()) : 0;
  std::vector<uint32_t> combo;
  for (int fa = 0; fa < p; ++fa)
    for (int fb = fa; fb < p; ++fb) combo.push_back(uint32_t(fa) | (uint32_t(fb) << 16));
  const int64_t ncombo = int64_t(combo.size());
  const int64_t nrt_bb = (nrow_bb + kRows - 1) / kRows;
  const int64_t nct_bb = (ncombo + kCols - 1) / kCols;
  std::vector<int32_t> bb_cols(std::max<int64_t>(nrt_bb, 1) * kMaxCols, 0);
  std::vector<int32_t> bb_ncol(std::max<int64_t>(nrt_bb, 1), 0);
  std::vector<uint32_t> bb_row(std::max<int64_t>(nrow_bb, 1), 0);
  for (int64_t t = 0; t < nrt_bb; ++t) {
    std::vector<int> alts;
    const int64_t r1 = std::min<int64_t>(nrow_bb, (t + 1) * kRows);
    for (int64_t r = t * kRows; r < r1; ++r) {
      alts.push_back(pair_nm[r] & 0xffff);
      alts.push_back(pair_nm[r] >> 16);
    }
    std::sort(alts.begin(), alts.end());
    alts.erase(std::unique(alts.begin(), alts.end()), alts.end());
    bb_ncol[t] = int(alts.size());
    for (size_t q = 0; q < alts.size(); ++q) bb_cols[t * kMaxCols + q] = alts[q];
    for (int64_t r = t * kRows; r < r1; ++r) {
      const int n = pair_nm[r] & 0xffff, m = pair_nm[r] >> 16;
      const uint32_t ln = uint32_t(std::lower_bound(alts.begin(), alts.end(), n) - alts.begin());
      const uint32_t lm = uint32_t(std::lower_bound(alts.begin(), alts.end(), m) - alts.begin());
      bb_row[r] = ln | (lm << 8) | (uint32_t(n == m) << 16) | (1u << 17);
    }
  }
  pl->nrow_bb = nrow_bb;
  pl->ncombo = ncombo;
  pl->bb_M = nrt_bb * kRows;
  pl->bb_N = nct_bb * kCols;

  // XG rows: all alternative-specific coefficients; columns: gamma ones
  const int64_t offg = d.off_gamma();
  const int64_t nrow_xg = a > 0 ? offg + int64_t(K) * a : 0;
  const int64_t ncol_xg = a > 0 ? int64_t(K) * a : 0;
  const int64_t nrt_xg = (nrow_xg + kRows - 1) / kRows;
  const int64_t nct_xg = (ncol_xg + kCols - 1) / kCols;
  pl->nrow_xg = nrow_xg;
  pl->ncol_xg = ncol_xg;
  pl->xg_M = nrt_xg * kRows;
  pl->xg_N = nct_xg * kCols;

  // output tiles, then observation splits
  std::vector<std::pair<int, std::pair<int, int>>> out_tiles;
  for (int64_t rt = 0; rt < nrt_bb; ++rt)
    for (int64_t ct = 0; ct < nct_bb; ++ct)
      out_tiles.push_back({T_BB, {int(rt * kRows), int(ct * kCols)}});
  for (int64_t rt = 0; rt < nrt_xg; ++rt)
    for (int64_t ct = 0; ct < nct_xg; ++ct) {
      const int64_t r0 = rt * kRows, c0 = ct * kCols;
      // gamma-gamma below the diagonal is mirrored, not computed
      if (r0 >= offg && r0 > offg + c0 + kCols - 1) continue;
      out_tiles.push_back({T_XG, {int(r0), int(c0)}});
    }
  const int64_t nout = int64_t(out_tiles.size());
  int S = 1;
  if (nout > 0) {
    const int64_t target = 1024;
    S = int(std::max<int64_t>(1, (target + nout - 1) / nout));
    const int64_t max_s = std::max<int64_t>(1, d.N / 256);
    S = int(std::min<int64_t>(S, max_s));
  }
  int64_t chunk = (d.N + S - 1) / S;
  chunk = (chunk + KC - 1) / KC * KC;
  S = int((d.N + chunk - 1) / chunk);
  pl->S = S;
  std::vector<Tile> tiles;
  for (int s = 0; s < S; ++s)
    for (auto &ot : out_tiles) {
      Tile t{};
      t.type = ot.first;
      t.row0 = ot.second.first;
      t.col0 = ot.second.second;
      t.split = s;
      t.obs0 = int(s * chunk);
      t.obs1 = int(std::min<int64_t>(d.N, (s + 1) * chunk));
      tiles.push_back(t);
    }
  if (d.N > (int64_t(1) << 31) - 1024)
    return set_error(c, MNL_ERR_UNSUPPORTED, "N too large for Hessian tiles");
  pl->ntiles = int(tiles.size());

  // LDS per workgroup (max over tile kinds)
  const size_t esz = prec == 0 ? 8 : 4;
  size_t lds_bb = nrow_bb ? size_t(KC) * (kMaxCols + p + 1) * esz : 0;
  size_t lds_xg = nrow_xg ? size_t(KC) * (K + p + size_t(K) * a + 1) * esz : 0;
  pl->lds = std::max(lds_bb, lds_xg);
  if (pl->lds > 150 * 1024) {
    delete pl;
    return set_error(c, MNL_ERR_UNSUPPORTED, "Hessian tile LDS too large");
  }

  // per-alternative kernel
  pl->need_alt = (a + g) > 0;
  if (pl->need_alt) {
    const int nl = p + a + g, nr = a + g;
    int nb = std::max(1, (kJ * kThreads) / (nl * nr));
    nb = std::min(nb, K);
    while (nb > 1 && size_t(kAltTB) * nb * (nl + nr) * 8 > 64 * 1024) --nb;
    if (nl * nr > kJ * kThreads) {
      delete pl;
      return set_error(c, MNL_ERR_UNSUPPORTED, "too many alpha/gamma features");
    }
    pl->alt_nb = nb;
    const int ngrp = (K + nb - 1) / nb;
    int Sa = std::max(1, 512 / ngrp);
    Sa = int(std::min<int64_t>(Sa, std::max<int64_t>(1, d.N / 256)));
    int64_t ch = (d.N + Sa - 1) / Sa;
    Sa = int((d.N + ch - 1) / ch);
    pl->alt_S = Sa;
    pl->alt_chunk = ch;
    pl->alt_lds = size_t(kAltTB) * nb * (nl + nr) * 8;
  }

  // device tables
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t o_tiles = 0;
  size_t o_cols = al(o_tiles + tiles.size() * sizeof(Tile));
  size_t o_ncol = al(o_cols + bb_cols.size() * 4);
  size_t o_row = al(o_ncol + bb_ncol.size() * 4);
  size_t o_combo = al(o_row + bb_row.size() * 4);
  size_t o_pair = al(o_combo + std::max<size_t>(combo.size(), 1) * 4);
  size_t total = al(o_pair + std::max<size_t>(pair_nm.size(), 1) * 4);
  if (hipMalloc(&pl->dev, total) != hipSuccess) {
    (void)hipGetLastError();
    delete pl;
    return set_error(c, MNL_ERR_OOM, "Hessian tables");
  }
  pl->dev_bytes = total;
  char *base = static_cast<char *>(pl->dev);
  pl->tiles = reinterpret_cast<Tile *>(base + o_tiles);
  pl->bb_cols = reinterpret_cast<int32_t *>(base + o_cols);
  pl->bb_ncol = reinterpret_cast<int32_t *>(base + o_ncol);
  pl->bb_row = reinterpret_cast<uint32_t *>(base + o_row);
  pl->bb_combo = reinterpret_cast<uint32_t *>(base + o_combo);
  pl->pair_nm = reinterpret_cast<int32_t *>(base + o_pair);
  auto up = [&](void *dst, const void *src, size_t n) {
    return n ? hipMemcpy(dst, src, n, hipMemcpyHostToDevice) : hipSuccess;
  };
  if (up(pl->tiles, tiles.data(), tiles.size() * sizeof(Tile)) != hipSuccess ||
      up(pl->bb_cols, bb_cols.data(), bb_cols.size() * 4) != hipSuccess ||
      up(pl->bb_ncol, bb_ncol.data(), bb_ncol.size() * 4) != hipSuccess ||
      up(pl->bb_row, bb_row.data(), bb_row.size() * 4) != hipSuccess ||
      up(pl->bb_combo, combo.data(), combo.size() * 4) != hipSuccess ||
      up(pl->pair_nm, pair_nm.data(), pair_nm.size() * 4) != hipSuccess) {
    (void)hipFree(pl->dev);
    delete pl;
    return set_error(c, MNL_ERR_HIP, "uploading Hessian tables");
  }
  cache->plans[key] = pl;
  *out = pl;
  return MNL_OK;
}

template <int PREC>
hipError_t launch_tiles(const Plan &pl, const HessDev &hd, hipStream_t s) {
  if (pl.ntiles == 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&k_hess_tiles<PREC>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hess_tiles<PREC>, dim3(pl.ntiles), dim3(kThreads),
                     pl.lds, s, hd);
  return hipGetLastError();
}

template <typename AccT>
hipError_t launch_assemble(const Plan &pl, const HessArgs &h, void *pbb,
                           void *pxg, const double *alt, hipStream_t s) {
  const Dims &d = pl.d;
  if (pl.nrow_bb > 0) {
    const int64_t n = pl.nrow_bb * pl.ncombo;
    hipLaunchKernelGGL(k_assemble_bb<AccT>, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, s, d, (const AccT *)pbb, pl.S, pl.bb_M,
                       pl.bb_N, pl.pair_nm, pl.bb_combo, pl.nrow_bb,
                       pl.ncombo, h.H);
  }
  if (pl.nrow_xg > 0) {
    const int64_t n = pl.nrow_xg * pl.ncol_xg;
    hipLaunchKernelGGL(k_assemble_xg<AccT>, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, s, d, (const AccT *)pxg, pl.S, pl.xg_M,
                       pl.xg_N, alt, pl.alt_S, h.H);
  }
  if (d.g > 0) {
    const int64_t n = d.off_alpha() * d.g + int64_t(d.g) * d.g;
    hipLaunchKernelGGL(k_assemble_alpha, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, s, d, alt, pl.alt_S, h.H);
  }
  return hipGetLastError();
}

}  // namespace

int hessian_run(Ctx *c, const HessArgs &h, hipStream_t s) {
  Plan *pl;
  MNL_TRY(build_plan(c, h.d, h.prec, &pl));
  const Dims &d = h.d;
  const size_t asz = h.prec == 0 ? 8 : 4;
  const size_t bytes_bb = size_t(pl->S) * pl->bb_M * pl->bb_N * asz;
  const size_t bytes_xg = size_t(pl->S) * pl->xg_M * pl->xg_N * asz;
  const int nl = d.p + d.a + d.g, nr = d.a + d.g;
  const size_t bytes_alt =
      pl->need_alt ? size_t(pl->alt_S) * d.K * nl * nr * 8 : 0;
  const size_t o_xg = (bytes_bb + 255) & ~size_t(255);
  const size_t o_alt = (o_xg + bytes_xg + 255) & ~size_t(255);
  void *ws;
  MNL_TRY(ws_get(c, S_HPART, o_alt + bytes_alt, &ws));
  char *wb = static_cast<char *>(ws);
  void *pbb = wb, *pxg = wb + o_xg;
  double *alt = reinterpret_cast<double *>(wb + o_alt);

  if (pl->need_alt) {
    const int ngrp = (d.K + pl->alt_nb - 1) / pl->alt_nb;
    MNL_HIP(c, hipFuncSetAttribute(
                   reinterpret_cast<const void *>(&k_hess_alt),
                   hipFuncAttributeMaxDynamicSharedMemorySize,
                   (int)pl->alt_lds));
    hipLaunchKernelGGL(k_hess_alt, dim3(ngrp, pl->alt_S), dim3(kThreads),
                       pl->alt_lds, s, d, h.X, h.Y, h.Z, h.w, h.P, h.Ybar,
                       pl->alt_nb, pl->alt_chunk, alt);
    MNL_HIP(c, hipGetLastError());
  }
  HessDev hd;
  hd.d = d;
  hd.X = h.X;
  hd.Z = h.Z;
  hd.w = h.w;
  hd.P = h.P;
  hd.P32 = h.prec == 0 ? nullptr : h.P32;
  hd.tiles = pl->tiles;
  hd.bb_cols = pl->bb_cols;
  hd.bb_ncol = pl->bb_ncol;
  hd.bb_row = pl->bb_row;
  hd.bb_combo = pl->bb_combo;
  hd.bb_M = pl->bb_M;
  hd.bb_N = pl->bb_N;
  hd.xg_M = pl->xg_M;
  hd.xg_N = pl->xg_N;
  hd.part_bb = pbb;
  hd.part_xg = pxg;
  hd.nrow_bb = pl->nrow_bb;
  hd.ncombo = pl->ncombo;
  hd.nrow_xg = pl->nrow_xg;
  hd.ncol_xg = pl->ncol_xg;
  if (c->ev_ready && pl->ntiles > 0) {
    MNL_HIP(c, hipEventRecord(c->ev_h0, s));
  }
  if (h.prec == 0) {
    MNL_HIP(c, launch_tiles<0>(*pl, hd, s));
  } else if (h.prec == 1) {
    MNL_HIP(c, launch_tiles<1>(*pl, hd, s));
  } else {
    MNL_HIP(c, launch_tiles<2>(*pl, hd, s));
  }
  if (c->ev_ready && pl->ntiles > 0) {
    MNL_HIP(c, hipEventRecord(c->ev_h1, s));
    c->hess_pending = true;
  }
  if (h.prec == 0)
    MNL_HIP(c, (launch_assemble<double>(*pl, h, pbb, pxg, alt, s)));
  else
    MNL_HIP(c, (launch_assemble<float>(*pl, h, pbb, pxg, alt, s)));
  return MNL_OK;
}

void hessian_cache_free(Ctx *c) {
  if (!c->hess_cache) return;
  Cache *cache = static_cast<Cache *>(c->hess_cache);
  for (auto &kv : cache->plans) {
    if (kv.second->dev) (void)hipFree(kv.second->dev);
    delete kv.second;
  }
  delete cache;
  c->hess_cache = nullptr;
}

}  // namespace mnl
