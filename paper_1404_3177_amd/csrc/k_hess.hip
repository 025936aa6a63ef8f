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
//  * beta-beta blocks (the bulk): k_bb.hip;
//  * XG tiles (beta-gamma and gamma-gamma): C = sum_i (w P_n phi_n)(P_m z_m)
//    for rows over all alternative-specific coefficients and columns over
//    the gamma coefficients (upper triangle only for gamma-gamma), on MFMA
//    (FP64, FP32 or BF16 operands) from LDS-staged P, X and Z, split over
//    observations; the split partials are summed in a fixed order, so the
//    result is reproducible;
//  * per-alternative kernel: the delta_nm parts of the XG blocks
//    (sum_i w P_n phi_n z_n^T) and all alpha blocks.
#include <algorithm>
#include <map>
#include <tuple>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;    // small kernels

struct Tile {
  int32_t row0, col0, split, obs0;
  int32_t obs1, pad0, pad1, pad2;
};

// MFMA traits --------------------------------------------------------------
// T: staged input type; OT: operand type in LDS; KCX: most observations per
// round (a multiple of KSTEP, the observations per MFMA); TN: most
// 16-column MFMA tiles per wave; NW: waves per workgroup (16 rows each),
// chosen so that accumulators plus operands fit the register file at
// NW / 4 waves per SIMD.
template <int PREC> struct MF;
template <> struct MF<0> {
  using T = double;
  using OT = double;
  using Acc = d4;
  static constexpr int KSTEP = 4, KCX = 32, TN = 8, NW = 16;
  __device__ static int out_row(int l, int r) { return (l >> 4) + 4 * r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <> struct MF<1> {
  using T = float;
  using OT = float;
  using Acc = f4;
  static constexpr int KSTEP = 4, KCX = 16, TN = 16, NW = 8;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};
template <> struct MF<2> {
  using T = float;
  using OT = __bf16;
  using Acc = f4;
  static constexpr int KSTEP = 32, KCX = 32, TN = 16, NW = 8;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static Acc zero() { return Acc{0, 0, 0, 0}; }
};

struct HessDev {
  Dims d;
  const double *X, *Z, *w;
  const double *P;
  const float *P32;
  const Tile *tiles;
  int64_t xg_M, xg_N;        // padded partial dims
  void *part_xg;             // [S][M][N] accumulator type
  int64_t nrow_xg, ncol_xg;  // valid rows / cols
  int kc_xg;                 // observations per round
  int nbuf_xg;               // raw input buffers (2: next round streams in)
};

__host__ __device__ constexpr int align16(int bytes) {
  return (bytes + 15) & ~15;
}

// LDS layout of one workgroup (bytes); shared by the kernel and the host.
// The raw region of a round is P rows, X, Z and w, back to back.
struct TileLds {
  // raw inputs of a round: P rows and Z in the staged type (P as P or P32
  // are stored), X and w in FP64; one or two buffers
  int rx, rz, rw, rawsz;
  int raw0, opa, opb, total;
};

template <int PREC>
__host__ __device__ inline TileLds tile_lds(int KC, int K, int p, int a,
                                            int bn, int nbuf) {
  using M = MF<PREC>;
  constexpr int kRows = 16 * M::NW;
  const int tsz = sizeof(typename M::T), osz = sizeof(typename M::OT);
  const int kp = PREC == 2 ? KC + 8 : KC;   // padded k extent (bf16 rows)
  TileLds L;
  L.rx = align16(KC * K * tsz);
  L.rz = L.rx + KC * p * 8;
  L.rw = L.rz + align16(KC * K * a * tsz);
  L.rawsz = align16(L.rw + KC * 8);
  int o = 0;
  L.raw0 = o; o += nbuf * L.rawsz;
  L.opa = o;  o = align16(o + kRows * kp * osz);
  L.opb = o;  o = align16(o + bn * kp * osz);
  L.total = o;
  return L;
}

// Wait for this wave's LDS operations, then the workgroup barrier; global
// loads still in flight (asynchronous copies into LDS) are not waited for.
__device__ inline void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt / expcnt untouched
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Generated-operand GEMM over the XG tile list.  Per round of KC
// observations: the raw inputs (P rows, X, Z, w) sit in LDS; the workgroup
// forms the A tile (rows: alternative-specific coefficients (n, feature),
// w P_n phi_n) and the B tile (16 tn gamma columns (m, c), P_m z_mc) in the
// MFMA operand type, then each wave runs 16 rows x 16 tn columns of MFMAs
// from LDS.  Several workgroups share a CU, so one's loads overlap
// another's MFMAs.
template <int PREC, int TNV>
__global__ __launch_bounds__(64 * MF<PREC>::NW) void k_hess_tiles(HessDev H) {
  using M = MF<PREC>;
  constexpr int kRows = 16 * M::NW, NT = 64 * M::NW;
  using T = typename M::T;
  using OT = typename M::OT;
  constexpr int TNM = TNV;
  extern __shared__ double smd[];
  char *smb = reinterpret_cast<char *>(smd);
  const Tile tile = H.tiles[blockIdx.x];
  const Dims d = H.d;
  const int K = d.K, p = d.p, a = d.a;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int bn = 16 * TNV;
  const int KC = H.kc_xg;
  const int kp = PREC == 2 ? KC + 8 : KC;
  const int nbuf = H.nbuf_xg;
  const TileLds L = tile_lds<PREC>(KC, K, p, a, bn, nbuf);
  OT *opa = reinterpret_cast<OT *>(smb + L.opa);
  OT *opb = reinterpret_cast<OT *>(smb + L.opb);
  // raw buffer b of the round: P rows, then X, Z, w (FP64)
  auto rawp = [&](int b) {
    return reinterpret_cast<T *>(smb + L.raw0 + b * L.rawsz);
  };
  auto rawd = [&](int b, int off) {
    return reinterpret_cast<double *>(smb + L.raw0 + b * L.rawsz + off);
  };
  // start from zeros in both raw buffers: the slots past the last
  // observation keep stale (finite) values that meet a zero weight
  for (int e = tid; e < nbuf * L.rawsz / 4; e += NT)
    reinterpret_cast<uint32_t *>(smb + L.raw0)[e] = 0u;
  __syncthreads();
  // stage one round of raw inputs into buffer b: the contiguous blocks (P
  // rows, X, Z) stream straight into LDS asynchronously, split over the
  // waves in 64-dword pieces; converted values and w are copied directly
  auto stage = [&](int b, int i0, int nobs) {
    auto wg_copy = [&](const void *src, void *dst, int ndw) {
      const uint32_t *s32 = static_cast<const uint32_t *>(src);
      char *d8 = static_cast<char *>(dst);
      for (int c = 64 * wv; c < ndw; c += 64 * (NT / 64)) {
        if (c + lane < ndw)
          __builtin_amdgcn_global_load_lds(s32 + c + lane,
                                           (lds_void_t *)(d8 + 4 * c), 4, 0,
                                           0);
      }
    };
    T *Pw = rawp(b);
    if constexpr (PREC == 0) {
      wg_copy(H.P + int64_t(i0) * K, Pw, 2 * nobs * K);
    } else if (H.P32) {
      wg_copy(H.P32 + int64_t(i0) * K, Pw, nobs * K);
    } else {
      for (int e = tid; e < nobs * K; e += NT)
        Pw[e] = T(H.P[int64_t(i0) * K + e]);
    }
    wg_copy(H.X + int64_t(i0) * p, rawd(b, L.rx), 2 * nobs * p);
    if constexpr (PREC == 0) {
      wg_copy(H.Z + int64_t(i0) * K * a, rawd(b, L.rz), 2 * nobs * K * a);
    } else {
      T *Zw = reinterpret_cast<T *>(smb + L.raw0 + b * L.rawsz + L.rz);
      const int za = K * a;
      batched_copy<8>(
          nobs * za, tid, NT,
          [&](int e) { return T(H.Z[int64_t(i0) * za + e]); },
          [&](int e, T v) { Zw[e] = v; });
    }
    // w streams in like the rest: a plain load here would make the
    // compiler wait for every copy in flight before storing it
    double *Ww = rawd(b, L.rw);
    if (H.w) {
      wg_copy(H.w + i0, Ww, 2 * nobs);
      for (int e = nobs + tid; e < KC; e += NT) Ww[e] = 0.0;
    } else {
      for (int e = tid; e < KC; e += NT) Ww[e] = e < nobs ? 1.0 : 0.0;
    }
  };

  typename M::Acc acc[TNM];
#pragma unroll
  for (int t = 0; t < TNM; ++t) acc[t] = M::zero();

  stage(0, tile.obs0, min(KC, tile.obs1 - tile.obs0));
  __syncthreads();
  // per-thread operand roles, fixed for the tile (no division in the loop):
  // A row: beta_n feature f (rows below (K-1) p) or gamma_n variable
  const int nb_rows = int(int64_t(K - 1) * p);
  const int ra = tid & (kRows - 1), ka0 = tid / kRows;  // NT / kRows = 4
  bool a_ok = false, a_z = false;
  int a_ln = 0, a_f = 0;
  {
    const int row = tile.row0 + ra;
    if (row < H.nrow_xg) {
      a_ok = true;
      if (row < nb_rows) {
        a_ln = 1 + row / p;
        a_f = row - (a_ln - 1) * p;
      } else {
        const int r2 = row - nb_rows;
        a_ln = r2 / a;
        a_f = r2;
        a_z = true;
      }
    }
  }
  // B: kbs threads share a column when bn divides the workgroup
  const int kbs = (NT % bn == 0) ? NT / bn : 1;
  const int cbx = (NT % bn == 0) ? tid % bn : tid;
  const int kb0 = (NT % bn == 0) ? tid / bn : 0;
  bool b_ok = false;
  int b_f1 = 0, b_f2 = 0;
  if (cbx < bn) {
    const int col = tile.col0 + cbx;
    b_ok = col < H.ncol_xg;
    b_f1 = col / a;
    b_f2 = col;
  }
  int cur = 0;
  for (int i0 = tile.obs0; i0 < tile.obs1;
       i0 += KC, cur = nbuf == 2 ? cur ^ 1 : 0) {
    const T *Ps = rawp(cur);
    const double *Xs = rawd(cur, L.rx);
    const T *Zs = reinterpret_cast<const T *>(smb + L.raw0 +
                                              cur * L.rawsz + L.rz);
    const double *Ws = rawd(cur, L.rw);
    // ---- form the operand tiles for this round ------------------------------
    // A: thread -> row ra, observations ka0, ka0 + 4, ...
    if (a_ok) {
      for (int k = ka0; k < KC; k += NT / kRows) {
        const T v = T(Ws[k]) * Ps[k * K + a_ln] *
                    T(a_z ? Zs[k * K * a + a_f] : Xs[k * p + a_f]);
        if constexpr (PREC == 2) opa[ra * kp + k] = (__bf16)v;
        else opa[k * kRows + ra] = v;
      }
    } else {
      for (int k = ka0; k < KC; k += NT / kRows) {
        if constexpr (PREC == 2) opa[ra * kp + k] = (__bf16)0.0f;
        else opa[k * kRows + ra] = OT(0);
      }
    }
    // B: thread -> column cbx, observations kb0, kb0 + kbs, ...
    if (cbx < bn) {
      for (int k = kb0; k < KC; k += kbs) {
        const T v = b_ok ? Ps[k * K + b_f1] * T(Zs[k * K * a + b_f2]) : T(0);
        if constexpr (PREC == 2) opb[cbx * kp + k] = (__bf16)v;
        else opb[k * bn + cbx] = v;
      }
    }
    // the next round streams into the other raw buffer during the MFMAs
    const int i1 = i0 + KC;
    if (nbuf == 2 && i1 < tile.obs1) stage(cur ^ 1, i1, min(KC, tile.obs1 - i1));
    lds_barrier();

    // ---- MFMAs from LDS --------------------------------------------------------

    const int arow = 16 * wv + (lane & 15);
    if constexpr (PREC == 2) {
      for (int ks = 0; ks < KC / 32; ++ks) {
        const int kb = 32 * ks + 8 * (lane >> 4);
        const bf8 av = *reinterpret_cast<const bf8 *>(opa + arow * kp + kb);
        const OT *bp = opb + (lane & 15) * kp + kb;
        bf8 bv[TNM];
#pragma unroll
        for (int t = 0; t < TNM; ++t)
          bv[t] = *reinterpret_cast<const bf8 *>(bp + 16 * t * kp);
#pragma unroll
        for (int t = 0; t < TNM; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[t], acc[t],
                                                           0, 0, 0);
      }
    } else {
      // operands of k-step ks + 1 are loaded while those of ks feed the
      // MFMAs (the last step reloads its own, unused)
      const int nks = KC / 4;
      const OT *ap = opa + (lane >> 4) * kRows + arow;
      const OT *bp = opb + (lane >> 4) * bn + (lane & 15);
      OT av = ap[0];
      OT bv[TNM];
#pragma unroll
      for (int t = 0; t < TNM; ++t) bv[t] = bp[16 * t];
      for (int ks = 0; ks < nks; ++ks) {
        const int kn = ks + 1 < nks ? ks + 1 : ks;
        const OT avn = ap[kn * 4 * kRows];
        OT bvn[TNM];
#pragma unroll
        for (int t = 0; t < TNM; ++t) bvn[t] = bp[kn * 4 * bn + 16 * t];
#pragma unroll
        for (int t = 0; t < TNM; ++t) {
          if constexpr (PREC == 0)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[t], acc[t],
                                                          0, 0, 0);
          else
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[t], acc[t],
                                                          0, 0, 0);
        }
        av = avn;
#pragma unroll
        for (int t = 0; t < TNM; ++t) bv[t] = bvn[t];
      }
    }
    // every wave is done with the operand tiles and the next round landed
    __syncthreads();
    if (nbuf == 1 && i1 < tile.obs1) {
      // one raw buffer: the next round is staged after this round's MFMAs
      stage(0, i1, min(KC, tile.obs1 - i1));
      __syncthreads();
    }
  }

  // epilogue: this split's partial tile
  using AccT = typename std::conditional<PREC == 0, double, float>::type;
  AccT *part = reinterpret_cast<AccT *>(H.part_xg);
  AccT *base = part +
               (int64_t(tile.split) * H.xg_M + tile.row0 + 16 * wv) * H.xg_N +
               tile.col0;
#pragma unroll
  for (int t = 0; t < TNM; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int orow = M::out_row(lane, r);
      const int ocol = 16 * t + (lane & 15);
      base[int64_t(orow) * H.xg_N + ocol] = acc[t][r];
    }
  }
}

// Per-alternative sums for the delta_nm parts and the alpha blocks:
//   out[n][l][r] = sum_i w_i P_in L_in[l] R_in[r]
// with L = (x_i, z_in, y_in - ybar_i), R = (z_in, y_in - ybar_i): for each
// alternative n a small GEMM over the observations, on FP64 MFMA.
// Workgroup: nb = 4 NQ alternatives x one observation range; wave w owns
// alternatives w, w + 4, ... with all NRT 16-row tiles of L for each, so
// per k-step the R operand and w P_n are read once for NRT MFMAs.  Per tile
// of 16 observations X, the Z and Y slices of the workgroup's alternatives,
// Ybar and w P are staged in LDS with contiguous row copies.
constexpr int kAltTB = 16;
constexpr int kAltNR = 16;   // most a + g handled (one MFMA column tile)

template <int NRT>
__global__ __launch_bounds__(kThreads) void k_hess_alt(
    Dims d, const double *X, const double *Y, const double *Z,
    const double *w, const double *P, const double *Ybar, int nb, int ngrp,
    int64_t obs_chunk, int xr, double *out /* [S][K][nl][nr] */) {
  constexpr int NQ = NRT == 1 ? 8 : (NRT == 2 ? 4 : (NRT <= 4 ? 2 : 1));
  extern __shared__ double sm[];
  // xr = p: every row of L; xr = 0: only the z and y rows (the x rows come
  // from k_hess_altx), written at their places p.. of the output rows
  const int K = d.K, p = xr, g = d.g, a = d.a, pf = d.p;
  const int nl = p + a + g, nr = a + g, nlf = pf + a + g, lo = pf - p;
  const int grp = blockIdx.x % ngrp, split = blockIdx.x / ngrp;
  const int n0 = grp * nb;
  const int nbe = min(nb, K - n0);
  const int64_t i_begin = int64_t(split) * obs_chunk;
  const int64_t i_end = min(d.N, i_begin + obs_chunk);
  // two LDS buffers, each: Xs [TB][p], Zs [TB][nb][a], Ys [TB][nb][g],
  // Yb [TB][g] (Ybar), Ps [TB][nb] (P), Ws [TB] (weights, 0 past the end)
  // and one zero slot, the source of every padding operand entry
  const int oZ = kAltTB * p, oY = oZ + kAltTB * nb * a,
            oB = oY + kAltTB * nb * g, oP = oB + kAltTB * g,
            oW = oP + kAltTB * nb, o0 = oW + kAltTB, bsz = o0 + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // stale values are multiplied by a zero weight, so start from zeros
  // (never NaN) and load only whole rows of real observations
  for (int e = tid; e < 2 * bsz; e += kThreads) sm[e] = 0.0;
  __syncthreads();
  auto stage = [&](int b, int64_t i0) {
    double *B = sm + b * bsz;
    const int nobs = (int)min<int64_t>(kAltTB, i_end - i0);
    // the tile's X rows, Ybar rows and weights are contiguous in memory:
    // one copy each, its 64-dword pieces spread over the waves
    auto wg_copy = [&](const double *src, double *dst, int ndw) {
      const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);
      char *d8 = reinterpret_cast<char *>(dst);
      for (int c = 64 * wv; c < ndw; c += kThreads) {
        if (c + lane < ndw)
          __builtin_amdgcn_global_load_lds(s32 + c + lane,
                                           (lds_void_t *)(d8 + 4 * c), 4, 0, 0);
      }
    };
    if (p) wg_copy(X + i0 * p, B, 2 * nobs * p);
    wg_copy(Ybar + i0 * g, B + oB, 2 * nobs * g);
    if (w) wg_copy(w + i0, B + oW, 2 * nobs);
    // per observation, the slices of the workgroup's alternatives
    for (int j = wv; j < nobs; j += kThreads / kWave) {
      const int64_t ii = i0 + j;
      wave_copy_lds(Z + (ii * K + n0) * a, B + oZ + j * nb * a, 2 * nbe * a,
                    lane);
      wave_copy_lds(Y + (ii * K + n0) * g, B + oY + j * nb * g, 2 * nbe * g,
                    lane);
      wave_copy_lds(P + ii * K + n0, B + oP + j * nb, 2 * nbe, lane);
    }
    // unit weights without w, zero weights past the last observation
    if (wv == 0 && lane < kAltTB && (!w || lane >= nobs))
      B[oW + lane] = lane < nobs ? 1.0 : 0.0;
  };
  d4 acc[NQ][NRT];
#pragma unroll
  for (int j = 0; j < NQ; ++j)
#pragma unroll
    for (int r = 0; r < NRT; ++r) acc[j][r] = d4{0, 0, 0, 0};

  const int ntile = (int)((i_end - i_begin + kAltTB - 1) / kAltTB);
  if (ntile > 0) stage(0, i_begin);
  __syncthreads();
  // Operand roles of this lane, fixed for the kernel, as LDS offsets
  // base + ob * (observation stride) + q * (alternative stride) so that the
  // loop has no branch: entries that are padding read the zero slot.
  // B column r = rl: z_qr or y_q,r-a, minus ybar_r-a for the latter.
  const int rl = lane & 15, obq = lane >> 4;
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  int bB = o0, bSo = 0, bSq = 0, bY = o0, bYo = 0;
  if (rl < a) {
    bB = oZ + rl; bSo = nb * a; bSq = a;
  } else if (rl < nr) {
    bB = oY + rl - a; bSo = nb * g; bSq = g; bY = oB + rl - a; bYo = g;
  }
  // A rows l = 16 rt + rl: x_l (l < p) in every tile, z / y - ybar only in
  // the rows p .. nl-1, which (NRT = ceil(nl / 16), nr <= 16) lie in the
  // last two tiles: slot 0 is tile NRT-2, slot 1 tile NRT-1
  int aB[2], aSo[2], aSq[2], aY[2], aYo[2];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) {
    const int l = 16 * (NRT - 2 + s2) + rl;
    aB[s2] = o0; aSo[s2] = 0; aSq[s2] = 0; aY[s2] = o0; aYo[s2] = 0;
    if (l >= p && l < p + a) {
      aB[s2] = oZ + l - p; aSo[s2] = nb * a; aSq[s2] = a;
    } else if (l >= p + a && l < nl) {
      aB[s2] = oY + l - p - a; aSo[s2] = nb * g; aSq[s2] = g;
      aY[s2] = oB + l - p - a; aYo[s2] = g;
    }
  }
  // slot 0 holds such rows only when they reach into tile NRT-2
  const bool two = NRT >= 2 && p < 16 * (NRT - 1);
  for (int t = 0; t < ntile; ++t) {
    const int cur = t & 1;
    // the next tile streams into the other buffer while this one is used
    if (t + 1 < ntile) stage(cur ^ 1, i_begin + int64_t(t + 1) * kAltTB);
    const double *B = sm + cur * bsz;
    const double *Ps = B + oP, *Ws = B + oW;
#pragma unroll 1
    for (int ks = 0; ks < kAltTB / 4; ++ks) {
      const int ob = 4 * ks + obq;
      const double wo = Ws[ob];
      // observation-only parts, shared by the workgroup's alternatives
      double xv[NRT];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt) {
        const int l = 16 * rt + rl;
        xv[rt] = B[l < p ? ob * p + l : o0];
      }
      const double ybB = B[bY + ob * bYo];
      const double ybA0 = two ? B[aY[0] + ob * aYo[0]] : 0.0;
      const double ybA1 = B[aY[1] + ob * aYo[1]];
      // every wave runs all NQ alternative slots: past the workgroup's last
      // alternative the staged P is zero, so those products add nothing
      // (and are not written out)
#pragma unroll
      for (int jq = 0; jq < NQ; ++jq) {
        const int q = wvu + 4 * jq;   // wave-uniform
        // the weight scales the R operand, so the x rows of L (the same for
        // every alternative) feed the MFMAs unscaled
        const double u = wo * Ps[ob * nb + q];
        const double bv = (B[bB + ob * bSo + q * bSq] - ybB) * u;
        const double z0 =
            two ? B[aB[0] + ob * aSo[0] + q * aSq[0]] - ybA0 : 0.0;
        const double z1 = B[aB[1] + ob * aSo[1] + q * aSq[1]] - ybA1;
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
          const double lv =
              rt == NRT - 1 ? xv[rt] + z1 : (rt == NRT - 2 ? xv[rt] + z0 : xv[rt]);
          acc[jq][rt] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(lv, bv, acc[jq][rt], 0, 0, 0);
        }
      }
    }
    // this tile's reads are done and the next tile has landed
    __syncthreads();
  }
#pragma unroll
  for (int jq = 0; jq < NQ; ++jq) {
    const int q = wv + 4 * jq;
    if (q >= nbe) continue;
    double *ob = out + ((int64_t(split) * K + n0 + q) * nlf) * nr;
    const int r = lane & 15;
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = 16 * rt + (lane >> 4) + 4 * i;
        if (l < nl && r < nr) ob[(l + lo) * nr + r] = acc[jq][rt][i];
      }
    }
  }
}

// The x rows of the per-alternative sums for all alternatives at once:
//   out[n][l][r] = sum_i x_il (w_i P_in R_in[r]),  l < p,
// a product X^T B' over the observations with B' columns (n, r) packed 16
// to an MFMA tile (K (a + g) columns), B' formed in registers from P, the
// z / y values, Ybar and w staged in LDS.  One workgroup of 8 waves per
// observation range reads X and Y once; wave v owns column tiles 4 v ..
// 4 v + 3 and all NRT 16-row tiles of X, so per k-step each A fragment
// feeds 4 MFMAs and each formed B fragment NRT.
constexpr int kAxThreads = 512;
template <int NRT>
__global__ __launch_bounds__(kAxThreads) void k_hess_altx(
    Dims d, const double *X, const double *Y, const double *Z,
    const double *w, const double *P, const double *Ybar, int rb,
    int64_t obs_chunk, double *out /* [S][K][nl][nr] */) {
  extern __shared__ double sm[];
  const int K = d.K, p = d.p, g = d.g, a = d.a;
  const int nr = a + g, nl = p + a + g, Ka = K * a, Kg = K * g;
  const int split = blockIdx.x;
  const int64_t i_begin = int64_t(split) * obs_chunk;
  const int64_t i_end = min(d.N, i_begin + obs_chunk);
  // two buffers: Xs [rb][p], Ps [rb][K], Zs [rb][K a], Ys [rb][K g],
  // Yb [rb][g], Ws [rb] (0 past the range), then one zero slot
  const int oP = rb * p, oZ = oP + rb * K, oY = oZ + rb * Ka,
            oB = oY + rb * Kg, oW = oB + rb * g, o0 = oW + rb, bsz = o0 + 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < 2 * bsz; e += kAxThreads) sm[e] = 0.0;
  __syncthreads();
  auto stage = [&](int b, int64_t i0) {
    double *B = sm + b * bsz;
    const int nobs = (int)min<int64_t>(rb, i_end - i0);
    auto wg_copy = [&](const double *src, double *dst, int ndw) {
      const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);
      char *d8 = reinterpret_cast<char *>(dst);
      for (int c = 64 * wv; c < ndw; c += kAxThreads)
        if (c + lane < ndw)
          __builtin_amdgcn_global_load_lds(s32 + c + lane,
                                           (lds_void_t *)(d8 + 4 * c), 4, 0, 0);
    };
    wg_copy(X + i0 * p, B, 2 * nobs * p);
    wg_copy(P + i0 * K, B + oP, 2 * nobs * K);
    if (a) wg_copy(Z + i0 * Ka, B + oZ, 2 * nobs * Ka);
    if (g) {
      wg_copy(Y + i0 * Kg, B + oY, 2 * nobs * Kg);
      wg_copy(Ybar + i0 * g, B + oB, 2 * nobs * g);
    }
    if (w) wg_copy(w + i0, B + oW, 2 * nobs);
    // unit weights without w, zero weights past the range
    if (tid < rb && (!w || tid >= nobs)) B[oW + tid] = tid < nobs ? 1.0 : 0.0;
  };
  // this lane's B columns (one per column tile): alternative, the offset of
  // its z or y value in an observation row, the Ybar offset (zero slot for
  // z), as offsets base + observation * stride so the loop has no branch
  const int kb = lane >> 4, l16 = lane & 15;
  int cP[4], cR[4], cRs[4], cY[4], cYs[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = 64 * wv + 16 * t + l16;
    cP[t] = o0; cR[t] = o0; cRs[t] = 0; cY[t] = o0; cYs[t] = 0;
    if (col < K * nr) {
      const int n = col / nr, r = col - n * nr;
      cP[t] = oP + n;
      if (r < a) {
        cR[t] = oZ + n * a + r; cRs[t] = Ka;
      } else {
        cR[t] = oY + n * g + (r - a); cRs[t] = Kg;
        cY[t] = oB + (r - a); cYs[t] = g;
      }
    }
  }
  int cX[NRT];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt) cX[rt] = 16 * rt + l16;
  d4 acc[NRT][4];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[rt][t] = d4{0, 0, 0, 0};
  const int nround = (int)((i_end - i_begin + rb - 1) / rb);
  if (nround > 0) stage(0, i_begin);
  for (int t0 = 0; t0 < nround; ++t0) {
    const int cur = t0 & 1;
    // this round's copies landed and every wave is done with the buffer
    // the next copies overwrite
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (t0 + 1 < nround) stage(cur ^ 1, i_begin + int64_t(t0 + 1) * rb);
    const double *B = sm + cur * bsz;
    for (int ks = 0; ks < rb / 4; ++ks) {
      const int o = 4 * ks + kb;
      const double wo = B[oW + o];
      double av[NRT], bv[4];
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
        av[rt] = B[cX[rt] < p ? o * p + cX[rt] : o0];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bv[t] = wo * B[cP[t] == o0 ? o0 : cP[t] + o * K] *
                (B[cR[t] + o * cRs[t]] - B[cY[t] + o * cYs[t]]);
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[rt][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bv[t],
                                                            acc[rt][t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = 64 * wv + 16 * t + l16;
    if (col >= K * nr) continue;
    const int n = col / nr, r = col - n * nr;
    double *ob = out + ((int64_t(split) * K + n) * nl) * nr + r;
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = 16 * rt + kb + 4 * i;
        if (l < p) ob[l * nr] = acc[rt][t][i];
      }
  }
}

// sum the observation splits of the per-alternative sums in a fixed order
__global__ void k_alt_reduce(const double *alt, int S, int64_t n,
                             double *red) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int s2 = 0;
  for (; s2 + 8 <= S; s2 += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += alt[int64_t(s2 + u) * n + e];
  }
  for (; s2 < S; ++s2) acc[s2 & 7] += alt[int64_t(s2) * n + e];
  red[e] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
           ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// ---- assembly into H (Hessian sign) ----------------------------------------------

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
  int S = 1;                     // observation splits of the XG tiles
  int ntiles = 0;
  int64_t xg_M = 0, xg_N = 0, nrow_xg = 0, ncol_xg = 0;
  size_t lds = 0;
  int kc_xg = 4, nbuf_xg = 1;
  int tn = 1;                    // 16-column MFMA tiles per workgroup tile
  // alt kernel
  int alt_nb = 1, alt_S = 1, alt_nrt = 1, alt_ngrp = 1;
  int64_t alt_chunk = 0;
  size_t alt_lds = 0;
  bool need_alt = false;
  // x rows of the per-alternative sums in k_hess_altx (else in k_hess_alt)
  bool altx = false;
  int altx_nrt = 1, altx_rb = 8;
  size_t altx_lds = 0;
  // tables: host copies (kept until the plan is freed, so an asynchronous
  // upload never reads freed memory) and one device allocation
  std::vector<Tile> h_tiles;
  void *dev = nullptr;
  size_t dev_bytes = 0;
  Tile *tiles = nullptr;
};

using Key = std::tuple<int64_t, int, int, int, int, int>;
struct Cache {
  std::map<Key, Plan *> plans;
};

}  // namespace

// Compute units of the context's device (256 on MI355X when the device
// cannot be queried, e.g. for host-only footprint queries).
int device_cus(Ctx *c) {
  if (c->ncu > 0) return c->ncu;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount,
                            c->device) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  c->ncu = n;
  return n;
}

namespace {

// Host part of a plan: tiling, split counts, LDS sizes and the tile list
// (in pl's host vector).  On error the caller deletes pl.
int plan_host(Ctx *c, const Dims &d, int prec, Plan *pl) {
  if (d.p > 255 || d.K > 4095)
    return set_error(c, MNL_ERR_UNSUPPORTED,
                     "Hessian tiles need p <= 255 and K < 4096");
  pl->d = d;
  pl->prec = prec;
  const int KSTEP = prec == 2 ? 32 : 4;
  const int kRows = 16 * (prec == 0 ? MF<0>::NW : (prec == 1 ? MF<1>::NW : MF<2>::NW));
  const int NT = 4 * kRows;
  const int KCX0 = prec == 0 ? MF<0>::KCX : (prec == 1 ? MF<1>::KCX : MF<2>::KCX);
  const int TNMAX = prec == 0 ? MF<0>::TN : (prec == 1 ? MF<1>::TN : MF<2>::TN);
  const int K = d.K, p = d.p, a = d.a, g = d.g;
  // column tiling: tn 16-column MFMA tiles per workgroup tile (the kernel
  // is specialised on it), as few tiles of padding as possible with at most
  // TNMAX per workgroup tile
  auto n16_of = [](int64_t ncols) { return (ncols + 15) / 16; };
  int tnu = 1;
  {
    const int64_t n16 = n16_of(a > 0 ? int64_t(K) * a : 0);
    if (n16 > 0) {
      const int64_t nct = (n16 + TNMAX - 1) / TNMAX;
      tnu = std::max(tnu, int((n16 + nct - 1) / nct));
    }
  }
  pl->tn = tnu;

  // XG rows: all alternative-specific coefficients; columns: gamma ones
  const int64_t offg = d.off_gamma();
  const int64_t nrow_xg = a > 0 ? offg + int64_t(K) * a : 0;
  const int64_t ncol_xg = a > 0 ? int64_t(K) * a : 0;
  const int64_t nrt_xg = (nrow_xg + kRows - 1) / kRows;
  const int64_t nct_xg = (n16_of(ncol_xg) + tnu - 1) / tnu;
  const int cw_xg = 16 * tnu;
  pl->nrow_xg = nrow_xg;
  pl->ncol_xg = ncol_xg;
  pl->xg_M = nrt_xg * kRows;
  pl->xg_N = std::max<int64_t>(nct_xg * cw_xg, 16);

  // output tiles, then observation splits
  struct OutTile { int row0, col0; };
  std::vector<OutTile> out_tiles;
  for (int64_t rt = 0; rt < nrt_xg; ++rt)
    for (int64_t ct = 0; ct < nct_xg; ++ct) {
      const int64_t r0 = rt * kRows, c0 = ct * cw_xg;
      // gamma-gamma below the diagonal is mirrored, not computed
      if (r0 >= offg && r0 > offg + c0 + cw_xg - 1) continue;
      out_tiles.push_back({int(r0), int(c0)});
    }
  const int64_t nout = int64_t(out_tiles.size());
  int S = 1;
  if (nout > 0) {
    // observation splits: the count whose workgroups fill the device's
    // resident slots (CUs x workgroups per CU) best in whole rounds; a
    // larger count must gain 2 points of fill to be taken (each split adds
    // a partial tile to write and reduce)
    const int64_t slots = int64_t(device_cus(c)) * std::max(1, 16 * 64 / NT);
    const int64_t max_s =
        std::max<int64_t>(1, std::min<int64_t>(64, d.N / 128));
    double best = -1.0;
    for (int sc = 1; sc <= max_s; ++sc) {
      const int64_t wg = int64_t(sc) * nout;
      const int64_t rounds = (wg + slots - 1) / slots;
      const double fill = double(wg) / double(rounds * slots);
      if (fill > best + 0.02) {
        best = fill;
        S = sc;
      }
    }
  }
  // split boundaries at multiples of 64 (BF16) or 32 observations
  int64_t chunk = (d.N + S - 1) / S;
  const int KCR = prec == 2 ? 64 : 32;
  chunk = (chunk + KCR - 1) / KCR * KCR;
  S = int((d.N + chunk - 1) / chunk);
  pl->S = S;
  // XCD-aware order: workgroup b runs on XCD b % 8, so the tiles of one
  // observation split are given ids of one residue and share that XCD's L2
  std::vector<Tile> tiles;
  {
    std::vector<std::vector<Tile>> q(8);
    for (int sp = 0; sp < S; ++sp)
      for (auto &ot : out_tiles) {
        Tile t{};
        t.row0 = ot.row0;
        t.col0 = ot.col0;
        t.split = sp;
        t.obs0 = int(sp * chunk);
        t.obs1 = int(std::min<int64_t>(d.N, (sp + 1) * chunk));
        q[sp % 8].push_back(t);
      }
    size_t pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    size_t left = size_t(S) * out_tiles.size();
    while (left) {
      for (int x = 0; x < 8 && left; ++x) {
        // an exhausted queue lends its slot to the longest remaining one
        int src = x;
        if (pos[src] >= q[src].size()) {
          size_t best = 0;
          for (int y = 0; y < 8; ++y)
            if (q[y].size() - pos[y] > best) { best = q[y].size() - pos[y]; src = y; }
        }
        tiles.push_back(q[src][pos[src]++]);
        --left;
      }
    }
  }
  if (d.N > (int64_t(1) << 31) - 1024) {
    return set_error(c, MNL_ERR_UNSUPPORTED, "N too large for Hessian tiles");
  }
  pl->ntiles = int(tiles.size());

  auto lds_of = [&](int kc, int bn, int nbuf) -> size_t {
    if (prec == 0) return tile_lds<0>(kc, K, p, a, bn, nbuf).total;
    if (prec == 1) return tile_lds<1>(kc, K, p, a, bn, nbuf).total;
    return tile_lds<2>(kc, K, p, a, bn, nbuf).total;
  };
  // observations per round: the largest multiple of the MFMA's observation
  // count that keeps LDS small enough for several workgroups per CU
  // (double-buffered raw inputs if they fit; one buffer otherwise)
  auto pick_kc = [&](int kc0, int bn, int *nbuf) -> int {
    // 16-wave workgroups own a CU; 8-wave ones share it with a second
    const size_t budget = kRows >= 192 ? size_t(150 * 1024) : size_t(78 * 1024);
    for (int nb2 = 2; nb2 >= 1; --nb2) {
      for (int kc = kc0; kc >= KSTEP; kc -= KSTEP) {
        if (lds_of(kc, bn, nb2) <= budget) {
          *nbuf = nb2;
          return kc;
        }
      }
    }
    *nbuf = 1;
    return lds_of(KSTEP, bn, 1) > 150 * 1024 ? 0 : KSTEP;
  };
  pl->nbuf_xg = 1;
  pl->kc_xg = nrow_xg ? pick_kc(KCX0, cw_xg, &pl->nbuf_xg) : KSTEP;
  if (pl->kc_xg == 0) {
    return set_error(c, MNL_ERR_UNSUPPORTED,
                     "Hessian tile exceeds LDS (p=%d K=%d a=%d)", p, K, a);
  }
  pl->lds = nrow_xg ? lds_of(pl->kc_xg, cw_xg, pl->nbuf_xg) : size_t(0);

  // per-alternative kernel
  pl->need_alt = (a + g) > 0;
  if (pl->need_alt) {
    const int nr = a + g;
    if (nr > kAltNR)
      return set_error(c, MNL_ERR_UNSUPPORTED,
                       "more than %d alternative-varying variables", kAltNR);
    // the x rows go to k_hess_altx when its columns (alternative, r) fit
    // one workgroup's 32 column tiles, p <= 64 and its staged rounds fit
    // in LDS; then k_hess_alt keeps the z and y rows (one row tile)
    // It pays when the X rows that the one-kernel path reads once per group
    // of alternatives outweigh the second read of the z and y data:
    // (groups - 1) p > K (a + g) values per observation
    pl->altx = false;
    const int nrt1 = (p + a + g + 15) / 16;
    const int nb1 = 4 * (nrt1 == 1 ? 8 : (nrt1 == 2 ? 4 : (nrt1 <= 4 ? 2 : 1)));
    const int64_t groups1 = (K + nb1 - 1) / nb1;
    if (p >= 1 && p <= 64 && int64_t(K) * nr <= 8 * 4 * 16 &&
        (groups1 - 1) * p > int64_t(K) * nr) {
      for (int rb = 8; rb >= 4 && !pl->altx; rb -= 4) {
        const size_t bsz = size_t(rb) * (p + K + size_t(K) * (a + g) + g + 1) + 1;
        if (2 * bsz * 8 <= 150 * 1024) {
          pl->altx = true;
          pl->altx_rb = rb;
          pl->altx_lds = 2 * bsz * 8;
          pl->altx_nrt = (p + 15) / 16;
        }
      }
    }
    const int pr = pl->altx ? 0 : p;   // rows of L taken from X in k_hess_alt
    const int nl = pr + a + g;
    int nrt = (nl + 15) / 16;
    if (nrt > 8)
      return set_error(c, MNL_ERR_UNSUPPORTED, "more than 128 features");
    const int nq = nrt == 1 ? 8 : (nrt == 2 ? 4 : (nrt <= 4 ? 2 : 1));
    const int nb = 4 * nq;
    pl->alt_nrt = nrt;
    pl->alt_nb = nb;
    const int ngrp = (K + nb - 1) / nb;
    pl->alt_ngrp = ngrp;
    // one round of resident workgroups (at most 3 per CU: register and
    // LDS limits), split evenly over the alternative groups
    pl->alt_lds = 2 * (size_t(kAltTB) *
                           (pr + size_t(nb) * a + size_t(nb) * g + g + nb + 1) +
                       1) * 8;
    const int wpc = int(std::max<size_t>(
        1, std::min<size_t>(3, (160 * 1024) / pl->alt_lds)));
    // the x-row kernel shares the observation ranges: one range per its
    // resident workgroups
    // (two resident workgroups per CU for one row tile of X, whose
    // registers allow that, else one)
    const int xpc =
        pl->altx && pl->altx_nrt == 1
            ? int(std::max<size_t>(1, std::min<size_t>(
                                          2, (160 * 1024) / pl->altx_lds)))
            : 1;
    int Sa = pl->altx ? xpc * device_cus(c)
                      : std::max(1, wpc * device_cus(c) / ngrp);
    Sa = int(std::min<int64_t>(Sa, std::max<int64_t>(1, d.N / 64)));
    int64_t ch = (d.N + Sa - 1) / Sa;
    ch = (ch + kAltTB - 1) / kAltTB * kAltTB;
    Sa = int((d.N + ch - 1) / ch);
    pl->alt_S = Sa;
    pl->alt_chunk = ch;
    if (pl->alt_lds > 150 * 1024)
      return set_error(c, MNL_ERR_UNSUPPORTED, "per-alternative tile too big");
  }

  // the tile list (one allocation)
  pl->dev_bytes = (std::max<size_t>(tiles.size(), 1) * sizeof(Tile) + 255) &
                  ~size_t(255);
  pl->h_tiles = std::move(tiles);
  return MNL_OK;
}

// Device copy of a plan's tile list.  A context in stream-ordered mode takes
// the memory from its pool and uploads on its stream; otherwise the upload
// is synchronous.
int plan_upload(Ctx *c, Plan *pl) {
  if (c->capturing)
    return set_error(c, MNL_ERR_HIP, "Hessian tables inside a capture");
  hipError_t e;
  if (c->pool)
    e = hipMallocFromPoolAsync(&pl->dev, pl->dev_bytes, c->pool, c->ostream);
  else
    e = hipMalloc(&pl->dev, pl->dev_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    pl->dev = nullptr;
    return set_error(c, MNL_ERR_OOM, "Hessian tables");
  }
  pl->tiles = static_cast<Tile *>(pl->dev);
  auto up = [&](void *dst, const void *src, size_t n) {
    if (!n) return hipSuccess;
    return c->pool ? hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice,
                                    c->ostream)
                   : hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
  };
  if (up(pl->tiles, pl->h_tiles.data(), pl->h_tiles.size() * sizeof(Tile)) !=
      hipSuccess)
    return set_error(c, MNL_ERR_HIP, "uploading Hessian tables");
  return MNL_OK;
}

void plan_free(Ctx *c, Plan *pl) {
  if (pl->dev) {
    if (c->pool) (void)hipFreeAsync(pl->dev, c->ostream);
    else (void)hipFree(pl->dev);
  }
  delete pl;
}

int build_plan(Ctx *c, const Dims &d, int prec, Plan **out) {
  if (!c->hess_cache) c->hess_cache = new Cache;
  Cache *cache = static_cast<Cache *>(c->hess_cache);
  Key key{d.N, d.K, d.p, d.g, d.a, prec};
  auto it = cache->plans.find(key);
  if (it != cache->plans.end()) {
    *out = it->second;
    return MNL_OK;
  }
  Plan *pl = new Plan;
  int rc = plan_host(c, d, prec, pl);
  if (rc == MNL_OK) rc = plan_upload(c, pl);
  if (rc != MNL_OK) {
    plan_free(c, pl);
    return rc;
  }
  cache->plans[key] = pl;
  *out = pl;
  return MNL_OK;
}

// Split-partial workspace of hessian_run: offsets of the XG partials, the
// per-alternative partials and their reduction, and the total.
struct PartLayout {
  size_t o_xg, o_alt, o_red, total, n_alt;
};

PartLayout part_layout(const Plan &pl) {
  const Dims &d = pl.d;
  const size_t asz = pl.prec == 0 ? 8 : 4;
  const size_t bytes_xg = size_t(pl.S) * pl.xg_M * pl.xg_N * asz;
  const int nl = d.p + d.a + d.g, nr = d.a + d.g;
  PartLayout L;
  L.n_alt = pl.need_alt ? size_t(d.K) * nl * nr : 0;
  const size_t bytes_alt = size_t(pl.alt_S) * L.n_alt * 8;
  L.o_xg = 0;
  L.o_alt = (L.o_xg + bytes_xg + 255) & ~size_t(255);
  L.o_red = (L.o_alt + bytes_alt + 255) & ~size_t(255);
  L.total = L.o_red + L.n_alt * 8 + 256;
  return L;
}

template <int PREC, int TNV>
hipError_t launch_tiles_tn(const Plan &pl, const HessDev &hd, hipStream_t s) {
  hipError_t e = raise_lds_limit(
      reinterpret_cast<const void *>(&k_hess_tiles<PREC, TNV>), (int)pl.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_hess_tiles<PREC, TNV>), dim3(pl.ntiles),
                     dim3(64 * MF<PREC>::NW), pl.lds, s, hd);
  return hipGetLastError();
}

// the instantiation for the plan's column-tile width
template <int PREC, int TNV = MF<PREC>::TN>
hipError_t launch_tiles(const Plan &pl, const HessDev &hd, hipStream_t s) {
  if (pl.ntiles == 0) return hipSuccess;
  if (pl.tn == TNV) return launch_tiles_tn<PREC, TNV>(pl, hd, s);
  if constexpr (TNV > 1) return launch_tiles<PREC, TNV - 1>(pl, hd, s);
  return hipErrorInvalidValue;
}

template <int NRT>
hipError_t launch_alt_nrt(const Plan &pl, const HessArgs &h, double *part,
                          hipStream_t s) {
  hipError_t e = raise_lds_limit(
      reinterpret_cast<const void *>(&k_hess_alt<NRT>), (int)pl.alt_lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_hess_alt<NRT>), dim3(pl.alt_ngrp * pl.alt_S),
                     dim3(kThreads), pl.alt_lds, s, pl.d, h.X, h.Y, h.Z, h.w,
                     h.P, h.Ybar, pl.alt_nb, pl.alt_ngrp, pl.alt_chunk,
                     pl.altx ? 0 : pl.d.p, part);
  return hipGetLastError();
}

template <int NRT>
hipError_t launch_altx_nrt(const Plan &pl, const HessArgs &h, double *part,
                           hipStream_t s) {
  hipError_t e = raise_lds_limit(
      reinterpret_cast<const void *>(&k_hess_altx<NRT>), (int)pl.altx_lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_hess_altx<NRT>), dim3(pl.alt_S), dim3(kAxThreads),
                     pl.altx_lds, s, pl.d, h.X, h.Y, h.Z, h.w, h.P, h.Ybar,
                     pl.altx_rb, pl.alt_chunk, part);
  return hipGetLastError();
}

hipError_t launch_altx(const Plan &pl, const HessArgs &h, double *part,
                       hipStream_t s) {
  switch (pl.altx_nrt) {
    case 1: return launch_altx_nrt<1>(pl, h, part, s);
    case 2: return launch_altx_nrt<2>(pl, h, part, s);
    case 3: return launch_altx_nrt<3>(pl, h, part, s);
    default: return launch_altx_nrt<4>(pl, h, part, s);
  }
}

hipError_t launch_alt(const Plan &pl, const HessArgs &h, double *part,
                      hipStream_t s) {
  switch (pl.alt_nrt) {
    case 1: return launch_alt_nrt<1>(pl, h, part, s);
    case 2: return launch_alt_nrt<2>(pl, h, part, s);
    case 3: return launch_alt_nrt<3>(pl, h, part, s);
    case 4: return launch_alt_nrt<4>(pl, h, part, s);
    case 5: return launch_alt_nrt<5>(pl, h, part, s);
    case 6: return launch_alt_nrt<6>(pl, h, part, s);
    case 7: return launch_alt_nrt<7>(pl, h, part, s);
    default: return launch_alt_nrt<8>(pl, h, part, s);
  }
}

template <typename AccT>
hipError_t launch_assemble(const Plan &pl, const HessArgs &h, void *pxg,
                           const double *alt, hipStream_t s) {
  const Dims &d = pl.d;
  if (pl.nrow_xg > 0) {
    const int64_t n = pl.nrow_xg * pl.ncol_xg;
    hipLaunchKernelGGL(k_assemble_xg<AccT>, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, s, d, (const AccT *)pxg, pl.S, pl.xg_M,
                       pl.xg_N, alt, 1, h.H);
  }
  if (d.g > 0) {
    const int64_t n = d.off_alpha() * d.g + int64_t(d.g) * d.g;
    hipLaunchKernelGGL(k_assemble_alpha, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, s, d, alt, 1, h.H);
  }
  return hipGetLastError();
}

}  // namespace

int hessian_run(Ctx *c, const HessArgs &h, hipStream_t s) {
  Plan *pl;
  MNL_TRY(build_plan(c, h.d, h.prec, &pl));
  const Dims &d = h.d;
  const PartLayout L = part_layout(*pl);
  const size_t n_alt = L.n_alt;
  void *ws;
  MNL_TRY(ws_get(c, S_HPART, L.total, &ws));
  char *wb = static_cast<char *>(ws);
  void *pxg = wb + L.o_xg;
  double *alt_part = reinterpret_cast<double *>(wb + L.o_alt);
  double *alt = reinterpret_cast<double *>(wb + L.o_red);

  if (pl->need_alt) {
    if (pl->altx) MNL_HIP(c, launch_altx(*pl, h, alt_part, s));
    MNL_HIP(c, launch_alt(*pl, h, alt_part, s));
    hipLaunchKernelGGL(k_alt_reduce, dim3((unsigned)((n_alt + 255) / 256)),
                       dim3(256), 0, s, alt_part, pl->alt_S, int64_t(n_alt),
                       alt);
    MNL_HIP(c, hipGetLastError());
  }
  // beta-beta blocks (timed: the Hessian's dominant kernel)
  MNL_TRY(bb_run(c, h, s));
  HessDev hd;
  hd.d = d;
  hd.X = h.X;
  hd.Z = h.Z;
  hd.w = h.w;
  hd.P = h.P;
  hd.P32 = h.prec == 0 ? nullptr : h.P32;
  hd.tiles = pl->tiles;
  hd.xg_M = pl->xg_M;
  hd.xg_N = pl->xg_N;
  hd.part_xg = pxg;
  hd.nrow_xg = pl->nrow_xg;
  hd.ncol_xg = pl->ncol_xg;
  hd.kc_xg = pl->kc_xg;
  hd.nbuf_xg = pl->nbuf_xg;
  if (h.prec == 0) {
    MNL_HIP(c, launch_tiles<0>(*pl, hd, s));
  } else if (h.prec == 1) {
    MNL_HIP(c, launch_tiles<1>(*pl, hd, s));
  } else {
    MNL_HIP(c, launch_tiles<2>(*pl, hd, s));
  }
  if (h.prec == 0)
    MNL_HIP(c, (launch_assemble<double>(*pl, h, pxg, alt, s)));
  else
    MNL_HIP(c, (launch_assemble<float>(*pl, h, pxg, alt, s)));
  return MNL_OK;
}

void hessian_cache_free(Ctx *c) {
  if (!c->hess_cache) return;
  Cache *cache = static_cast<Cache *>(c->hess_cache);
  for (auto &kv : cache->plans) plan_free(c, kv.second);
  delete cache;
  c->hess_cache = nullptr;
}

int hessian_footprint(Ctx *c, const Dims &d, int prec, size_t *part_bytes,
                      size_t *table_bytes) {
  Plan pl;
  MNL_TRY(plan_host(c, d, prec, &pl));
  size_t bb_ws = 0, bb_tab = 0;
  MNL_TRY(bb_footprint(c, d, prec, &bb_ws, &bb_tab));
  *part_bytes = part_layout(pl).total + bb_ws;
  *table_bytes = pl.dev_bytes + bb_tab;
  return MNL_OK;
}


}  // namespace mnl
