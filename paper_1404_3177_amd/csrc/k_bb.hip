// Beta-beta blocks of the Hessian (Eq. 10, Sec. 3.3): the bulk of the
// Hessian and the part the paper's block-symmetric formulation speeds up.
//
// For alternatives 1 <= n <= m <= K-1 the block is
//   H_nm = -X^T W_nm X,  W_nm = diag(w_i P_in (delta_nm - P_im)),
// H_mn = H_nm^T, and each block is itself symmetric.  All unique entries
// come from one product whose rows are alternative pairs (n, m) and whose
// columns are feature pairs a <= b:
//   C[(n,m)][(a,b)] = sum_i omega_i(n,m) chi_i(a,b),
//   omega_i(n,m) = P_in (delta_nm - P_im),  chi_i(a,b) = w_i x_ia x_ib,
// which is half the flops of the blocks' dense products (the observation
// weight rides with the data-only operand).
//
// Neither operand is stored whole:
//  * chi depends on the data only.  It is formed once per fit, in the MFMA
//    operand type, in the order the MFMA B operand takes it
//    (k_xx_frag): per round of KR observations and 16 feature pairs, one
//    contiguous fragment block.  A workgroup streams its column tile of
//    it into LDS with asynchronous 16-byte copies (no registers held).
//  * omega depends on theta.  P is transposed once per Hessian into
//    observation blocks [N/KR][K][RS] (k_p_blocks), each column padded as
//    its copy in LDS; the alternatives a row tile needs stream into LDS
//    per round, each run of consecutive alternatives in 1 KB pieces of
//    16-byte copies, and each wave forms its omega fragments in
//    registers, in MFMA A-operand order, right before the MFMAs that
//    consume them.  The rounding to the MFMA type happens after omega is
//    formed in FP32 (mixed precision) or FP64.
// A workgroup of NWV waves (8, or 4 for few pair rows) owns 64 NWV pair rows
// x 16 TNB feature pairs; every wave runs 64 rows (4 A fragments) x all TNB
// B fragments, so each B fragment read from LDS feeds 4 MFMAs and each
// formed A fragment TNB.
// The observations are split in S contiguous ranges; partial tiles are
// summed in a fixed order by the assembly kernel (bitwise reproducible).
#include <algorithm>
#include <map>
#include <tuple>

#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kMaxStage = 128;   // staged alternatives per row tile
// copy pieces per row tile: each run of consecutive staged alternatives
// goes to LDS in 1 KB pieces (at most 34 full pieces for 128 columns, plus
// one partial piece per run)
constexpr int kMaxPieces = 192;
// A fragments (16 pair rows each) per wave: 4, or 3 where 384-row tiles
// pad the pair rows and columns less (8-wave tiles; up to 7 B fragments
// then in FP64 and 12 in FP32 and BF16, LDS allowing, so that a formed
// omega fragment feeds more MFMAs)
constexpr int kTMA = 4;
constexpr int tnmax3(int prec) { return prec == 0 ? 7 : 12; }
constexpr int kBlkAlt = 32;      // alternatives per pair block (large K)

// Per precision: T = P / w / omega type, XT = chi type, KR observations per
// round, RS = LDS row stride of a staged P column (elements; padded so the
// fragment reads of 16 lanes fall on distinct banks), TNMAX = most B
// fragments per wave (register budget: kTMA x TNMAX accumulators).
template <int PREC> struct BBT;
template <> struct BBT<0> {
  using T = double;
  using XT = double;
  using Acc = d4;
  static constexpr int KR = 32, RS = 34, TNMAX = 5;
  __device__ static int out_row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct BBT<1> {
  using T = float;
  using XT = float;
  using Acc = f4;
  static constexpr int KR = 64, RS = 68, TNMAX = 8;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct BBT<2> {
  using T = float;
  using XT = __bf16;
  using Acc = f4;
  static constexpr int KR = 64, RS = 68, TNMAX = 8;
  __device__ static int out_row(int l, int r) { return 4 * (l >> 4) + r; }
};

struct BBConst {
  int kr, rs, tnmax, esz, xsz, asz;
};
BBConst bb_const(int prec) {
  if (prec == 0) return {32, 34, 5, 8, 8, 8};
  if (prec == 1) return {64, 68, 8, 4, 4, 4};
  return {64, 68, 8, 4, 2, 4};
}

__host__ __device__ constexpr int al16(int b) { return (b + 15) & ~15; }

// LDS layout of one of the two round buffers: staged P columns (plus one
// zero column that padding rows read), then the B tile.
struct BBLds {
  int b, bufsz;
};
__host__ __device__ inline BBLds bb_lds(int kr, int rs, int esz, int xsz,
                                        int pcols, int tnb) {
  BBLds L;
  L.b = al16((pcols + 1) * rs * esz);
  L.bufsz = al16(L.b + tnb * 16 * kr * xsz);
  return L;
}

struct BBTile {
  int32_t rt, ct, split, ob0, ob1, pad0, pad1, pad2;
};

struct BBDev {
  const void *PT;           // [nob][K][RS] T: P by observation blocks,
                            // each column padded as in LDS
  const void *XX;           // [nob][ncgx][16 KR] XT: chi in fragment order
  const BBTile *tiles;
  const int32_t *pieces;    // [nrt][kMaxPieces][2] copy pieces: source
                            // dword offset in an observation block, LDS
                            // byte offset | 16-byte lanes << 24
  const int32_t *npiece;    // [nrt]
  const uint32_t *rowinfo;  // [Mp] ln | lm << 8 | delta << 16
  void *part;               // [S][Mp][Np] accumulator type
  int64_t Mp, Np;
  int K, pcols, ncgx;
};

template <int PREC, int TNB, int NWV, int TMA>
__global__ __launch_bounds__(64 * NWV, 2) void k_bb(BBDev D) {
  constexpr int kWaves = NWV;
  constexpr int RW = 16 * TMA;               // pair rows per wave
  using C = BBT<PREC>;
  using T = typename C::T;
  using XT = typename C::XT;
  using Acc = typename C::Acc;
  constexpr int KR = C::KR, RS = C::RS;
  constexpr int XF = 16 * KR;               // chi elements per group/round
  constexpr int BCH = TNB * XF * int(sizeof(XT)) / 1024;  // 1 KB B chunks
  static_assert(TNB * XF * int(sizeof(XT)) % 1024 == 0, "B tile in 1 KB");
  extern __shared__ double smd[];
  char *sm = reinterpret_cast<char *>(smd);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const BBTile tl = D.tiles[blockIdx.x];
  const BBLds L = bb_lds(KR, RS, int(sizeof(T)), int(sizeof(XT)), D.pcols,
                         TNB);
  // the wave index as a scalar: the copy loops are then scalar
  const int wvs = __builtin_amdgcn_readfirstlane(wv);
  // this wave's copy pieces of the tile's staged P columns (pieces wvs,
  // wvs + NWV, ...): lane i holds the i-th, so a copy takes its offsets
  // with a lane read and no memory wait
  constexpr int PPW = kMaxPieces / kWaves;   // most pieces per wave
  static_assert(PPW <= 64, "one lane per piece");
  const int npc = D.npiece[tl.rt];
  const int npw = npc > wvs ? (npc - wvs + kWaves - 1) / kWaves : 0;
  int psrc = 0, pdst = 0;
  if (lane < npw) {
    const int32_t *pe =
        D.pieces + (int64_t(tl.rt) * kMaxPieces + wvs + kWaves * lane) * 2;
    psrc = pe[0];
    pdst = pe[1];
  }

  // the zero column (index pcols) of both buffers, read by padding rows
  for (int e = tid; e < 2 * RS; e += 64 * kWaves) {
    const int b = e / RS, o = e - b * RS;
    reinterpret_cast<T *>(sm + b * L.bufsz)[D.pcols * RS + o] = T(0);
  }
  // this lane's A rows (one per fragment): LDS offsets of P_n and P_m
  int offn[TMA], offm[TMA];
  T dg[TMA];
  {
    const int64_t r0 = int64_t(tl.rt) * (RW * kWaves) + RW * wv + (lane & 15);
#pragma unroll
    for (int j = 0; j < TMA; ++j) {
      const uint32_t info = D.rowinfo[r0 + 16 * j];
      offn[j] = int(info & 0xffu) * RS;
      offm[j] = int((info >> 8) & 0xffu) * RS;
      dg[j] = (info >> 16) & 1u ? T(1) : T(0);
    }
  }
  // fragments with no diagonal pair in any row of this wave (wave-uniform)
  bool offd[TMA];
#pragma unroll
  for (int j = 0; j < TMA; ++j)
    offd[j] = __builtin_amdgcn_ballot_w64(dg[j] != T(0)) == 0;

  // asynchronous copies of round ob into buffer b: the staged P columns
  // (laid out in HBM as in LDS) and the B tile go in 1 KB pieces of
  // 16-byte lanes
  const uint32_t *pt32 = static_cast<const uint32_t *>(D.PT);
  const char *xx8 = static_cast<const char *>(D.XX);
  constexpr int PDW = RS * int(sizeof(T)) / 4;   // dwords per padded column
  static_assert(RS * int(sizeof(T)) % 16 == 0, "16-byte column pieces");
  auto piece = [&](char *buf, const uint32_t *src, int i) {
    const int ps = __builtin_amdgcn_readlane(psrc, i);
    const int pd = __builtin_amdgcn_readlane(pdst, i);
    if (lane < (pd >> 24))
      __builtin_amdgcn_global_load_lds(src + ps + 4 * lane,
                                       (lds_void_t *)(buf + (pd & 0xffffff)),
                                       16, 0, 0);
  };
  auto stage = [&](int b, int ob) {
    char *buf = sm + b * L.bufsz;
    const uint32_t *src = pt32 + int64_t(ob) * D.K * PDW;
    for (int i = 0; i < npw; ++i) piece(buf, src, i);
    const char *xs =
        xx8 + (int64_t(ob) * D.ncgx + int64_t(tl.ct) * TNB) * XF * sizeof(XT);
    for (int q = wvs; q < BCH; q += kWaves)
      __builtin_amdgcn_global_load_lds(xs + q * 1024 + lane * 16,
                                       (lds_void_t *)(buf + L.b + q * 1024),
                                       16, 0, 0);
  };

  Acc acc[TMA][TNB];
#pragma unroll
  for (int j = 0; j < TMA; ++j)
#pragma unroll
    for (int t = 0; t < TNB; ++t) acc[j][t] = Acc{0, 0, 0, 0};

  __syncthreads();   // zero columns in place
  stage(0, tl.ob0);
  __builtin_amdgcn_s_waitcnt(0);   // every counter: this wave's copies landed
  __syncthreads();
  int cur = 0;
  const int kb = lane >> 4;
  for (int ob = tl.ob0; ob < tl.ob1; ++ob, cur ^= 1) {
    // the next round streams into the other buffer during this one
    constexpr bool kSpread = PREC != 2 && TNB >= 3;
    if (!kSpread && ob + 1 < tl.ob1) stage(cur ^ 1, ob + 1);
    const char *buf = sm + cur * L.bufsz;
    const T *Ps = reinterpret_cast<const T *>(buf);
    const XT *Bs = reinterpret_cast<const XT *>(buf + L.b);
    if constexpr (PREC == 2) {
      // forming omega is the BF16 kernel's VALU load: a fragment none of
      // whose rows is a diagonal pair (n = m, delta = 1) takes
      // omega = -(P_n P_m), one product per element instead of two ops
#pragma unroll
      for (int ks = 0; ks < KR / 32; ++ks) {
        // lane: row lane & 15 of each A fragment, observations o .. o + 7
        const int o = 32 * ks + 8 * kb;
        bf8 bv[TNB];
#pragma unroll
        for (int t = 0; t < TNB; ++t)
          bv[t] = *reinterpret_cast<const bf8 *>(Bs + t * XF + ks * 512 +
                                                 lane * 8);
#pragma unroll
        for (int j = 0; j < TMA; ++j) {
          const f4 n0 = *reinterpret_cast<const f4 *>(Ps + offn[j] + o);
          const f4 n1 = *reinterpret_cast<const f4 *>(Ps + offn[j] + o + 4);
          const f4 m0 = *reinterpret_cast<const f4 *>(Ps + offm[j] + o);
          const f4 m1 = *reinterpret_cast<const f4 *>(Ps + offm[j] + o + 4);
          bf8 av;
          if (offd[j]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              av[e] = (__bf16)(-(n0[e] * m0[e]));
              av[4 + e] = (__bf16)(-(n1[e] * m1[e]));
            }
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              av[e] = (__bf16)(n0[e] * (dg[j] - m0[e]));
              av[4 + e] = (__bf16)(n1[e] * (dg[j] - m1[e]));
            }
          }
#pragma unroll
          for (int t = 0; t < TNB; ++t)
            acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                av, bv[t], acc[j][t], 0, 0, 0);
        }
      }
    } else if constexpr (TNB >= 3) {
      // one k-step of software pipeline with the instruction order fixed
      // (scheduling barriers): the LDS reads of step ks + 1 go out between
      // the first three MFMAs of step ks, and its A fragments are formed
      // between the last four, at least five MFMAs after those reads; a
      // wave then waits on LDS only at the start of a round
      constexpr int NQ = TMA * TNB, NKS = KR / 4, NHALF = NKS / 2;
      // the next round's copies go out over the first half of the round,
      // between MFMAs: step ks < NHALF issues this wave's P pieces
      // CPK ks .. CPK ks + CPK - 1 and B pieces BPK ks .. BPK ks + BPK - 1
      // (at most 4 pieces per step; a wave's pieces past 4 NHALF, which
      // only many short runs of alternatives give, go out in one loop)
      constexpr int CPK = std::min(4, (PPW + NHALF - 1) / NHALF);
      constexpr int BPW = (BCH + kWaves - 1) / kWaves;
      constexpr int BPK = (BPW + NHALF - 1) / NHALF;
      const bool copy = ob + 1 < tl.ob1;
      char *nbuf = sm + (cur ^ 1) * L.bufsz;
      const uint32_t *nsrc = pt32 + int64_t(ob + 1) * D.K * PDW;
      const char *nxs = xx8 + (int64_t(ob + 1) * D.ncgx + int64_t(tl.ct) * TNB) *
                                  XF * sizeof(XT);
      T bv[TNB], av[TMA];
      {
#pragma unroll
        for (int t = 0; t < TNB; ++t) bv[t] = Bs[t * XF + lane];
#pragma unroll
        for (int j = 0; j < TMA; ++j)
          av[j] = Ps[offn[j] + kb] * (dg[j] - Ps[offm[j] + kb]);
      }
#pragma unroll
      for (int ks = 0; ks < KR / 4; ++ks) {
        const bool more = ks + 1 < KR / 4;
        const int o = 4 * (ks + 1) + kb;
        T bn[TNB], pn[TMA], pm[TMA], an[TMA];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = q / TNB, t = q % TNB;
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (PREC == 0)
            acc[j][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                av[j], bv[t], acc[j][t], 0, 0, 0);
          else
            acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                av[j], bv[t], acc[j][t], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          if (ks < NHALF && q == 3 && copy) {
#pragma unroll
            for (int u = 0; u < CPK; ++u) {
              const int i = CPK * ks + u;
              if (i < PPW && i < npw) piece(nbuf, nsrc, i);
            }
            if (ks == 0)
              for (int i = CPK * NHALF; i < npw; ++i) piece(nbuf, nsrc, i);
          }
          if (ks < NHALF && q == 4 && copy) {
#pragma unroll
            for (int u = 0; u < BPK; ++u) {
              const int m = wvs + kWaves * (BPK * ks + u);
              if (m < BCH)
                __builtin_amdgcn_global_load_lds(
                    nxs + m * 1024 + lane * 16,
                    (lds_void_t *)(nbuf + L.b + m * 1024), 16, 0, 0);
            }
          }
          if (more) {
            if (q == 0) {
#pragma unroll
              for (int u = 0; u < TNB; ++u)
                bn[u] = Bs[u * XF + (ks + 1) * 64 + lane];
            } else if (q == 1) {
#pragma unroll
              for (int i = 0; i < TMA; ++i) pn[i] = Ps[offn[i] + o];
            } else if (q == 2) {
#pragma unroll
              for (int i = 0; i < TMA; ++i) pm[i] = Ps[offm[i] + o];
            } else if (q >= NQ - TMA) {
              const int i = q - (NQ - TMA);
              an[i] = pn[i] * (dg[i] - pm[i]);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (more) {
#pragma unroll
          for (int j = 0; j < TMA; ++j) av[j] = an[j];
#pragma unroll
          for (int t = 0; t < TNB; ++t) bv[t] = bn[t];
        }
      }
    } else {
      // operands one k-step ahead: the LDS reads of step ks + 1 are in
      // flight while step ks's MFMAs run (lane: row lane & 15 of each A
      // fragment, observation 4 ks + lane / 16)
      T bv[TNB], pn[TMA], pm[TMA];
      auto load = [&](int ks, T *b, T *n, T *m) {
        const int o = 4 * ks + kb;
#pragma unroll
        for (int t = 0; t < TNB; ++t) b[t] = Bs[t * XF + ks * 64 + lane];
#pragma unroll
        for (int j = 0; j < TMA; ++j) {
          n[j] = Ps[offn[j] + o];
          m[j] = Ps[offm[j] + o];
        }
      };
      load(0, bv, pn, pm);
#pragma unroll
      for (int ks = 0; ks < KR / 4; ++ks) {
        T bv2[TNB], pn2[TMA], pm2[TMA];
        if (ks + 1 < KR / 4) load(ks + 1, bv2, pn2, pm2);
#pragma unroll
        for (int j = 0; j < TMA; ++j) {
          const T av = pn[j] * (dg[j] - pm[j]);
#pragma unroll
          for (int t = 0; t < TNB; ++t) {
            if constexpr (PREC == 0)
              acc[j][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                  av, bv[t], acc[j][t], 0, 0, 0);
            else
              acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  av, bv[t], acc[j][t], 0, 0, 0);
          }
        }
        if (ks + 1 < KR / 4) {
#pragma unroll
          for (int t = 0; t < TNB; ++t) bv[t] = bv2[t];
#pragma unroll
          for (int j = 0; j < TMA; ++j) {
            pn[j] = pn2[j];
            pm[j] = pm2[j];
          }
        }
      }
    }
    // the next round's copies have landed and nobody reads this buffer
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  using AT = typename std::conditional<PREC == 0, double, float>::type;
  AT *base = static_cast<AT *>(D.part) +
             (int64_t(tl.split) * D.Mp + int64_t(tl.rt) * (RW * kWaves) +
              RW * wv) * D.Np +
             int64_t(tl.ct) * TNB * 16;
#pragma unroll
  for (int j = 0; j < TMA; ++j)
#pragma unroll
    for (int t = 0; t < TNB; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        base[int64_t(16 * j + C::out_row(lane, r)) * D.Np + 16 * t +
             (lane & 15)] = AT(acc[j][t][r]);
}

// chi_i(a,b) = w_i x_ia x_ib in B-fragment order: element index
// ((ob * ncgx + cg) * NKS + ks) * 64 + lane (times 8 for BF16), holding
// observation ob KR + ks KSTEP + lane / 16 (+ 8 (lane / 16) + e for BF16,
// KSTEP 32) and feature pair 16 cg + lane % 16; zero past N and past the
// last pair; w NULL reads as ones.  The product is taken in FP64 and
// rounded once (BF16: through FP32, as the other mixed operands).
template <int PREC>
__global__ __launch_bounds__(256) void k_xx_frag(
    const double *X, const double *w, int p, int64_t N, const uint32_t *combo,
    int64_t ncombo, int ncgx, int64_t nob, typename BBT<PREC>::XT *xx) {
  using XT = typename BBT<PREC>::XT;
  constexpr int KR = BBT<PREC>::KR;
  constexpr int NKS = PREC == 2 ? KR / 32 : KR / 4;
  const int64_t total = nob * ncgx * NKS * 64;
  for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * 256) {
    const int l = int(idx & 63);
    const int64_t gk = idx >> 6;
    const int ks = int(gk % NKS);
    const int64_t grp = gk / NKS;
    const int cg = int(grp % ncgx);
    const int64_t ob = grp / ncgx;
    const int64_t col = int64_t(cg) * 16 + (l & 15);
    int fa = 0, fb = 0;
    const bool cok = col < ncombo;
    if (cok) {
      const uint32_t cq = combo[col];
      fa = int(cq & 0xffff);
      fb = int(cq >> 16);
    }
    if constexpr (PREC == 2) {
      const int64_t i0 = ob * KR + 32 * ks + 8 * (l >> 4);
      bf8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t i = i0 + e;
        const double x = (cok && i < N)
                             ? (w ? w[i] : 1.0) * X[i * p + fa] * X[i * p + fb]
                             : 0.0;
        v[e] = (__bf16)float(x);
      }
      *reinterpret_cast<bf8 *>(xx + idx * 8) = v;
    } else {
      const int64_t i = ob * KR + 4 * ks + (l >> 4);
      const double x = (cok && i < N)
                           ? (w ? w[i] : 1.0) * X[i * p + fa] * X[i * p + fb]
                           : 0.0;
      xx[idx] = XT(x);
    }
  }
}

// P [N][K] (FP64) -> PT [nob][K][RS] in T (0 past N; the RS - KR padding
// entries of a column are not written), the layout of the staged columns
// in LDS; one workgroup per block of KR observations and 64 alternatives,
// transposed through LDS.
template <typename T, int KR, int RS>
__global__ __launch_bounds__(256) void k_p_blocks(const double *P, int K,
                                                  int64_t N, T *PT) {
  __shared__ double tile[KR][65];
  const int64_t ob = blockIdx.x;
  const int k0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < KR * 64; e += 256) {
    const int i = e >> 6, k = e & 63;
    const int64_t obs = ob * KR + i;
    tile[i][k] = (obs < N && k0 + k < K) ? P[obs * K + k0 + k] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < KR * 64; e += 256) {
    const int k = e / KR, i = e - k * KR;
    if (k0 + k < K) PT[(ob * K + k0 + k) * RS + i] = T(tile[i][k]);
  }
}

// Sum the split partials of a pair row / feature pair entry in a fixed
// order and write its four places in H (Hessian sign): rows (n, a), (n, b)
// against columns (m, b), (m, a), and the mirrored ones.
template <typename AT>
__global__ void k_bb_assemble(const AT *part, int S, int64_t Mp, int64_t Np,
                              const int32_t *pair_nm, const uint32_t *combo,
                              int64_t ncombo, int64_t p, int64_t np,
                              double *H) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= Mp * ncombo) return;
  const int64_t r = e / ncombo, q = e - r * ncombo;
  const int32_t nm = pair_nm[r];
  if (nm == 0) return;   // padding row
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += (double)part[(int64_t(s) * Mp + r) * Np + q];
  const int n = nm & 0xffff, m = nm >> 16;
  const int fa = combo[q] & 0xffff, fb = combo[q] >> 16;
  const int64_t ra = (n - 1) * p + fa, rb = (n - 1) * p + fb;
  const int64_t ca = (m - 1) * p + fa, cb = (m - 1) * p + fb;
  v = -v;
  H[ra * np + cb] = v;
  H[rb * np + ca] = v;
  H[cb * np + ra] = v;
  H[ca * np + rb] = v;
}

// ---- host plan ------------------------------------------------------------

struct BBPlan {
  Dims d;
  int prec = 0, tnb = 1, nw = 8, tma = kTMA, S = 1, ntiles = 0, pcols = 0,
      ncgx = 0;
  int64_t npairs = 0, Mp = 0, Np = 0, ncombo = 0, nob = 0, nrt = 0;
  size_t lds = 0;
  std::vector<BBTile> h_tiles;
  std::vector<int32_t> h_pieces, h_npiece, h_pair;
  std::vector<uint32_t> h_row, h_combo;
  size_t o_pieces = 0, o_npiece = 0, o_row = 0, o_combo = 0, o_pair = 0;
  size_t dev_bytes = 0;
  void *dev = nullptr;
  BBTile *tiles = nullptr;
  int32_t *pieces = nullptr, *npiece = nullptr, *pair = nullptr;
  uint32_t *row = nullptr, *combo = nullptr;
};

using BBKey = std::tuple<int64_t, int, int, int>;
struct BBCache {
  std::map<BBKey, BBPlan *> plans;
};

int bb_plan_host(Ctx *c, const Dims &d, int prec, BBPlan *pl) {
  if (d.p > 255)
    return set_error(c, MNL_ERR_UNSUPPORTED,
                     "beta-beta Hessian blocks need p <= 255");
  if (d.N > (int64_t(1) << 40))
    return set_error(c, MNL_ERR_UNSUPPORTED, "N too large");
  pl->d = d;
  pl->prec = prec;
  const BBConst bc = bb_const(prec);
  const int Lk = d.K - 1, p = d.p;
  // workgroups of 8 waves (512 pair rows), or of 4 when that pads at least
  // 10% fewer rows (few alternatives; two such workgroups share a CU)
  {
    const int64_t np = int64_t(Lk) * (Lk + 1) / 2;
    const int64_t r8 = (np + 511) / 512 * 512, r4 = (np + 255) / 256 * 256;
    pl->nw = (Lk <= kMaxStage && r4 < 0.9 * double(r8)) ? 4 : 8;
  }
  // pair rows: n <= m over alternatives 1..K-1, row-major within blocks of
  // kBlkAlt alternatives when there are more than a tile can stage; a row
  // tile closes early (padding rows) when its next pair would need more
  // than kMaxStage staged alternatives
  std::vector<std::pair<int, int>> pairs;
  if (Lk <= kMaxStage) {
    for (int n = 1; n <= Lk; ++n)
      for (int m = n; m <= Lk; ++m) pairs.push_back({n, m});
  } else {
    const int nb = (Lk + kBlkAlt - 1) / kBlkAlt;
    for (int bi = 0; bi < nb; ++bi)
      for (int bj = bi; bj < nb; ++bj)
        for (int n = 1 + bi * kBlkAlt; n <= std::min(Lk, (bi + 1) * kBlkAlt); ++n)
          for (int m = std::max(n, 1 + bj * kBlkAlt);
               m <= std::min(Lk, (bj + 1) * kBlkAlt); ++m)
            pairs.push_back({n, m});
  }
  pl->npairs = int64_t(pairs.size());
  // rows of R pairs per tile: row_nm gets n | m << 16 per row (0 =
  // padding), tcols the staged alternatives of each tile
  auto tile_rows = [&](int R, std::vector<int32_t> &row_nm,
                       std::vector<std::vector<int>> &tcols) {
    std::vector<char> in(size_t(d.K), 0);
    std::vector<int> cur;
    auto close_tile = [&]() {
      while (row_nm.size() % R) row_nm.push_back(0);
      std::sort(cur.begin(), cur.end());
      tcols.push_back(cur);
      for (int a : cur) in[a] = 0;
      cur.clear();
    };
    for (auto &pr : pairs) {
      const int need = (in[pr.first] ? 0 : 1) +
                       (in[pr.second] || pr.second == pr.first ? 0 : 1);
      if (int(cur.size()) + need > kMaxStage) close_tile();
      for (int a : {pr.first, pr.second})
        if (!in[a]) {
          in[a] = 1;
          cur.push_back(a);
        }
      row_nm.push_back(pr.first | (pr.second << 16));
      if (row_nm.size() % R == 0) {
        std::sort(cur.begin(), cur.end());
        tcols.push_back(cur);
        for (int a : cur) in[a] = 0;
        cur.clear();
      }
    }
    if (row_nm.size() % R) close_tile();
  };
  // feature pairs a <= b; column groups of 16, TNB groups per tile: the
  // least padded columns, weighted by the per-tile cost of forming and
  // staging the A operand (a tile of TNB groups re-forms it once per TNB)
  std::vector<uint32_t> combo;
  for (int fa = 0; fa < p; ++fa)
    for (int fb = fa; fb < p; ++fb)
      combo.push_back(uint32_t(fa) | (uint32_t(fb) << 16));
  pl->ncombo = int64_t(combo.size());
  const int64_t ncg = (pl->ncombo + 15) / 16;
  auto pick_tnb = [&](int lo, int hi) {
    int tnb = lo;
    double best = 1e300;
    for (int t = lo; t <= hi; ++t) {
      const double cost = double((ncg + t - 1) / t * t) * (1.0 + 0.5 / t);
      if (cost <= best) {
        best = cost;
        tnb = t;
      }
    }
    return tnb;
  };
  std::vector<int32_t> row_nm;
  std::vector<std::vector<int>> tcols;
  int R = 16 * kTMA * pl->nw;
  tile_rows(R, row_nm, tcols);
  int tnb = pick_tnb(1, bc.tnmax);
  // 8-wave tiles: three A fragments per wave (384 rows) when that pads the
  // pair rows times columns at least 2% less
  if (pl->nw == 8) {
    std::vector<int32_t> row3;
    std::vector<std::vector<int>> tc3;
    const int R3 = 16 * 3 * pl->nw;
    tile_rows(R3, row3, tc3);
    int pc3 = 1;
    for (auto &tc : tc3) pc3 = std::max(pc3, int(tc.size()));
    // the most B fragments whose two round buffers fit in LDS
    int hi3 = tnmax3(prec);
    while (hi3 > 3 &&
           2 * size_t(bb_lds(bc.kr, bc.rs, bc.esz, bc.xsz, pc3, hi3).bufsz) >
               160 * 1024)
      --hi3;
    const int tnb3 = pick_tnb(3, hi3);
    const double w4 = double(row_nm.size()) * double((ncg + tnb - 1) / tnb * tnb);
    const double w3 = double(row3.size()) * double((ncg + tnb3 - 1) / tnb3 * tnb3);
    if (2 * size_t(bb_lds(bc.kr, bc.rs, bc.esz, bc.xsz, pc3, tnb3).bufsz) <=
            160 * 1024 &&
        w3 <= 0.98 * w4) {
      pl->tma = 3;
      R = R3;
      tnb = tnb3;
      row_nm.swap(row3);
      tcols.swap(tc3);
    }
  }
  pl->nrt = int64_t(tcols.size());
  pl->Mp = pl->nrt * R;
  int pcols = 1;
  for (auto &tc : tcols) pcols = std::max(pcols, int(tc.size()));
  pl->pcols = pcols;
  // copy pieces of each row tile: runs of consecutive staged alternatives
  // (contiguous in the padded P blocks and in LDS) cut into 1 KB pieces
  std::vector<int32_t> pieces(size_t(std::max<int64_t>(pl->nrt, 1)) * kMaxPieces * 2, 0);
  std::vector<int32_t> npiece(size_t(std::max<int64_t>(pl->nrt, 1)), 0);
  const int colb = bc.rs * bc.esz;   // bytes per padded column
  std::vector<uint32_t> rowinfo(size_t(std::max<int64_t>(pl->Mp, 1)),
                                uint32_t(pcols) | (uint32_t(pcols) << 8));
  for (int64_t t = 0; t < pl->nrt; ++t) {
    const auto &tc = tcols[t];
    int np = 0;
    for (size_t q0 = 0; q0 < tc.size();) {
      size_t q1 = q0 + 1;
      while (q1 < tc.size() && tc[q1] == tc[q1 - 1] + 1) ++q1;
      const int64_t bytes = int64_t(q1 - q0) * colb;
      for (int64_t off = 0; off < bytes; off += 1024, ++np) {
        if (np >= kMaxPieces)
          return set_error(c, MNL_ERR_UNSUPPORTED, "beta-beta copy pieces");
        const int64_t nb = std::min<int64_t>(1024, bytes - off);
        pieces[(t * kMaxPieces + np) * 2] =
            int32_t((int64_t(tc[q0]) * colb + off) / 4);
        pieces[(t * kMaxPieces + np) * 2 + 1] =
            int32_t((int64_t(q0) * colb + off) | ((nb / 16) << 24));
      }
      q0 = q1;
    }
    npiece[t] = np;
    for (int64_t r = t * R; r < (t + 1) * R; ++r) {
      const int32_t nm = row_nm[r];
      if (nm == 0) continue;
      const int n = nm & 0xffff, m = nm >> 16;
      const uint32_t ln = uint32_t(std::lower_bound(tc.begin(), tc.end(), n) - tc.begin());
      const uint32_t lm = uint32_t(std::lower_bound(tc.begin(), tc.end(), m) - tc.begin());
      rowinfo[r] = ln | (lm << 8) | (uint32_t(n == m) << 16);
    }
  }
  pl->tnb = tnb;
  const int64_t nct = (ncg + tnb - 1) / tnb;
  pl->ncgx = int(nct * tnb);
  pl->Np = int64_t(pl->ncgx) * 16;
  pl->nob = (d.N + bc.kr - 1) / bc.kr;
  const BBLds L = bb_lds(bc.kr, bc.rs, bc.esz, bc.xsz, pcols, tnb);
  pl->lds = size_t(2) * L.bufsz;
  if (pl->lds > 160 * 1024)
    return set_error(c, MNL_ERR_UNSUPPORTED, "beta-beta tile exceeds LDS");

  // observation splits: the count whose workgroups fill the resident slots
  // (one 8-wave or two 4-wave workgroups per CU, as LDS allows) best in
  // whole rounds; a larger count must gain 2 points of fill
  const int64_t nout = pl->nrt * nct;
  int S = 1;
  if (nout > 0) {
    const int per_cu = std::max<int>(
        1, std::min<int>(pl->nw == 4 ? 2 : 1,
                         int((160 * 1024) / std::max<size_t>(pl->lds, 1))));
    const int64_t slots = int64_t(device_cus(c)) * per_cu;
    const int64_t max_s = std::max<int64_t>(1, std::min<int64_t>(64, pl->nob / 4));
    double bestf = -1.0;
    for (int sc = 1; sc <= max_s; ++sc) {
      const int64_t wg = sc * nout;
      const int64_t rounds = (wg + slots - 1) / slots;
      const double fill = double(wg) / double(rounds * slots);
      if (fill > bestf + 0.02) {
        bestf = fill;
        S = sc;
      }
    }
  }
  const int64_t chunk = (pl->nob + S - 1) / S;
  S = int((pl->nob + chunk - 1) / chunk);
  pl->S = S;
  // XCD-aware order: workgroup b runs on XCD b % 8, so the tiles of one
  // observation split get ids of one residue and share that XCD's L2 (the
  // B column tiles are read by every row tile of the split)
  std::vector<BBTile> tiles;
  {
    std::vector<std::vector<BBTile>> q(8);
    for (int sp = 0; sp < S; ++sp)
      for (int64_t ct = 0; ct < nct; ++ct)
        for (int64_t rt = 0; rt < pl->nrt; ++rt) {
          BBTile t{};
          t.rt = int(rt);
          t.ct = int(ct);
          t.split = sp;
          t.ob0 = int(sp * chunk);
          t.ob1 = int(std::min<int64_t>(pl->nob, (sp + 1) * chunk));
          q[sp % 8].push_back(t);
        }
    size_t pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    size_t left = size_t(S) * size_t(nout);
    while (left) {
      for (int x = 0; x < 8 && left; ++x) {
        int src = x;
        if (pos[src] >= q[src].size()) {
          size_t most = 0;
          for (int y = 0; y < 8; ++y)
            if (q[y].size() - pos[y] > most) {
              most = q[y].size() - pos[y];
              src = y;
            }
        }
        tiles.push_back(q[src][pos[src]++]);
        --left;
      }
    }
  }
  pl->ntiles = int(tiles.size());
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  pl->o_pieces = al(tiles.size() * sizeof(BBTile));
  pl->o_npiece = al(pl->o_pieces + pieces.size() * 4);
  pl->o_row = al(pl->o_npiece + npiece.size() * 4);
  pl->o_combo = al(pl->o_row + rowinfo.size() * 4);
  pl->o_pair = al(pl->o_combo + std::max<size_t>(combo.size(), 1) * 4);
  pl->dev_bytes = al(pl->o_pair + std::max<size_t>(row_nm.size(), 1) * 4);
  pl->h_tiles = std::move(tiles);
  pl->h_pieces = std::move(pieces);
  pl->h_npiece = std::move(npiece);
  pl->h_row = std::move(rowinfo);
  pl->h_combo = std::move(combo);
  pl->h_pair = std::move(row_nm);
  return MNL_OK;
}

int bb_plan_upload(Ctx *c, BBPlan *pl) {
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
    return set_error(c, MNL_ERR_OOM, "beta-beta tables");
  }
  char *base = static_cast<char *>(pl->dev);
  pl->tiles = reinterpret_cast<BBTile *>(base);
  pl->pieces = reinterpret_cast<int32_t *>(base + pl->o_pieces);
  pl->npiece = reinterpret_cast<int32_t *>(base + pl->o_npiece);
  pl->row = reinterpret_cast<uint32_t *>(base + pl->o_row);
  pl->combo = reinterpret_cast<uint32_t *>(base + pl->o_combo);
  pl->pair = reinterpret_cast<int32_t *>(base + pl->o_pair);
  auto up = [&](void *dst, const void *src, size_t n) {
    if (!n) return hipSuccess;
    return c->pool ? hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice,
                                    c->ostream)
                   : hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
  };
  if (up(pl->tiles, pl->h_tiles.data(), pl->h_tiles.size() * sizeof(BBTile)) !=
          hipSuccess ||
      up(pl->pieces, pl->h_pieces.data(), pl->h_pieces.size() * 4) != hipSuccess ||
      up(pl->npiece, pl->h_npiece.data(), pl->h_npiece.size() * 4) != hipSuccess ||
      up(pl->row, pl->h_row.data(), pl->h_row.size() * 4) != hipSuccess ||
      up(pl->combo, pl->h_combo.data(), pl->h_combo.size() * 4) != hipSuccess ||
      up(pl->pair, pl->h_pair.data(), pl->h_pair.size() * 4) != hipSuccess)
    return set_error(c, MNL_ERR_HIP, "uploading beta-beta tables");
  return MNL_OK;
}

void bb_plan_free(Ctx *c, BBPlan *pl) {
  if (pl->dev) {
    if (c->pool) (void)hipFreeAsync(pl->dev, c->ostream);
    else (void)hipFree(pl->dev);
  }
  delete pl;
}

int bb_plan_get(Ctx *c, const Dims &d, int prec, BBPlan **out) {
  if (!c->bb_cache) c->bb_cache = new BBCache;
  BBCache *cache = static_cast<BBCache *>(c->bb_cache);
  BBKey key{d.N, d.K, d.p, prec};
  auto it = cache->plans.find(key);
  if (it != cache->plans.end()) {
    *out = it->second;
    return MNL_OK;
  }
  BBPlan *pl = new BBPlan;
  int rc = bb_plan_host(c, d, prec, pl);
  if (rc == MNL_OK) rc = bb_plan_upload(c, pl);
  if (rc != MNL_OK) {
    bb_plan_free(c, pl);
    return rc;
  }
  cache->plans[key] = pl;
  *out = pl;
  return MNL_OK;
}

struct BBWs {
  size_t pt, part, xx;
};
BBWs bb_ws_bytes(const BBPlan &pl) {
  const BBConst bc = bb_const(pl.prec);
  BBWs w;
  w.pt = size_t(pl.nob) * pl.d.K * bc.rs * bc.esz;
  w.part = size_t(pl.S) * pl.Mp * pl.Np * bc.asz;
  w.xx = size_t(pl.nob) * pl.ncgx * 16 * bc.kr * bc.xsz;
  return w;
}

template <int PREC, int TNB, int NWV, int TMA>
hipError_t launch_bb_nw(const BBPlan &pl, const BBDev &D, hipStream_t s) {
  hipError_t e = raise_lds_limit(
      reinterpret_cast<const void *>(&k_bb<PREC, TNB, NWV, TMA>), int(pl.lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_bb<PREC, TNB, NWV, TMA>), dim3(pl.ntiles),
                     dim3(64 * NWV), pl.lds, s, D);
  return hipGetLastError();
}

template <int PREC, int TNB>
hipError_t launch_bb_tnb(const BBPlan &pl, const BBDev &D, hipStream_t s) {
  if constexpr (TNB >= 3 && TNB <= tnmax3(PREC)) {
    if (pl.tma == 3)
      return pl.nw == 8 ? launch_bb_nw<PREC, TNB, 8, 3>(pl, D, s)
                        : hipErrorInvalidValue;
  }
  if constexpr (TNB <= BBT<PREC>::TNMAX) {
    if (pl.tma == kTMA)
      return pl.nw == 4 ? launch_bb_nw<PREC, TNB, 4, kTMA>(pl, D, s)
                        : launch_bb_nw<PREC, TNB, 8, kTMA>(pl, D, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int TNB = (tnmax3(PREC) > BBT<PREC>::TNMAX
                                  ? tnmax3(PREC) : BBT<PREC>::TNMAX)>
hipError_t launch_bb(const BBPlan &pl, const BBDev &D, hipStream_t s) {
  if (pl.tnb == TNB) return launch_bb_tnb<PREC, TNB>(pl, D, s);
  if constexpr (TNB > 1) return launch_bb<PREC, TNB - 1>(pl, D, s);
  return hipErrorInvalidValue;
}

template <int PREC>
int bb_run_prec(Ctx *c, const BBPlan &pl, const HessArgs &h, hipStream_t s) {
  using C = BBT<PREC>;
  using T = typename C::T;
  using XT = typename C::XT;
  // the call's dims (n_p): one cached plan serves every (g, a) of an (N, K, p)
  const Dims &d = h.d;
  const BBWs wb = bb_ws_bytes(pl);
  void *ptv, *partv, *xxv;
  MNL_TRY(ws_get(c, S_PT, wb.pt, &ptv));
  MNL_TRY(ws_get(c, S_BBPART, wb.part, &partv));
  MNL_TRY(ws_get(c, PREC == 0 ? S_XX : S_XX_LP, wb.xx, &xxv));
  T *PT = static_cast<T *>(ptv);
  // chi depends on the data only: formed once per top-level call (a fit
  // reuses it for all of its Hessians)
  Ctx::XXState &xs = c->xx[PREC == 0 ? 0 : 1];
  if (!(xs.X == h.X && xs.w == h.w && xs.N == d.N && xs.p == d.p &&
        xs.prec == PREC && xs.epoch == c->call_epoch && xs.buf == xxv)) {
    const int64_t total = pl.nob * pl.ncgx * (PREC == 2 ? C::KR / 32 : C::KR / 4) * 64;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL((k_xx_frag<PREC>), dim3(unsigned(blocks)), dim3(256), 0,
                       s, h.X, h.w, d.p, d.N, pl.combo, pl.ncombo, pl.ncgx,
                       pl.nob, static_cast<XT *>(xxv));
    MNL_HIP(c, hipGetLastError());
    xs.X = h.X;
    xs.w = h.w;
    xs.N = d.N;
    xs.p = d.p;
    xs.prec = PREC;
    xs.epoch = c->call_epoch;
    xs.buf = xxv;
  }
  hipLaunchKernelGGL((k_p_blocks<T, C::KR, C::RS>),
                     dim3(unsigned(pl.nob), unsigned((d.K + 63) / 64)),
                     dim3(256), 0, s, h.P, d.K, d.N, PT);
  MNL_HIP(c, hipGetLastError());
  BBDev D;
  D.PT = PT;
  D.XX = xxv;
  D.tiles = pl.tiles;
  D.pieces = pl.pieces;
  D.npiece = pl.npiece;
  D.rowinfo = pl.row;
  D.part = partv;
  D.Mp = pl.Mp;
  D.Np = pl.Np;
  D.K = d.K;
  D.pcols = pl.pcols;
  D.ncgx = pl.ncgx;
  const bool timed = c->ev_ready;
  if (timed) MNL_HIP(c, hipEventRecord(c->ev_h0, s));
  MNL_HIP(c, launch_bb<PREC>(pl, D, s));
  if (timed) {
    MNL_HIP(c, hipEventRecord(c->ev_h1, s));
    c->hess_pending = true;
  }
  using AT = typename std::conditional<PREC == 0, double, float>::type;
  const int64_t n = pl.Mp * pl.ncombo;
  hipLaunchKernelGGL(k_bb_assemble<AT>, dim3(unsigned((n + 255) / 256)),
                     dim3(256), 0, s, static_cast<const AT *>(partv), pl.S,
                     pl.Mp, pl.Np, pl.pair, pl.combo, pl.ncombo, int64_t(d.p),
                     d.np, h.H);
  MNL_HIP(c, hipGetLastError());
  return MNL_OK;
}

}  // namespace

int bb_run(Ctx *c, const HessArgs &h, hipStream_t s) {
  const Dims &d = h.d;
  if (d.K < 2 || d.p < 1) return MNL_OK;
  BBPlan *pl;
  MNL_TRY(bb_plan_get(c, d, h.prec, &pl));
  if (h.prec == 0) return bb_run_prec<0>(c, *pl, h, s);
  if (h.prec == 1) return bb_run_prec<1>(c, *pl, h, s);
  return bb_run_prec<2>(c, *pl, h, s);
}

int bb_footprint(Ctx *c, const Dims &d, int prec, size_t *ws_bytes,
                 size_t *table_bytes) {
  *ws_bytes = 0;
  *table_bytes = 0;
  if (d.K < 2 || d.p < 1) return MNL_OK;
  BBPlan pl;
  MNL_TRY(bb_plan_host(c, d, prec, &pl));
  const BBWs w = bb_ws_bytes(pl);
  *ws_bytes = (w.pt + 256) + w.part + w.xx;
  *table_bytes = pl.dev_bytes;
  return MNL_OK;
}

void bb_cache_free(Ctx *c) {
  if (!c->bb_cache) return;
  BBCache *cache = static_cast<BBCache *>(c->bb_cache);
  for (auto &kv : cache->plans) bb_plan_free(c, kv.second);
  delete cache;
  c->bb_cache = nullptr;
}

}  // namespace mnl
