// Fused pass over the observations: utilities, choice probabilities,
// log-likelihood and gradient in one read of X, Y and Z.
//
//   U_ik = x_i.beta_k + z_ik.gamma_k + y_ik.alpha     (Eq. 1, beta_0 = 0)
//   P_i  = softmax_k(U_i)                              (Eqs. 3-4: softmax is
//          invariant to the per-row shift that turns U into the normalised
//          V of Eq. 2, so no differencing of the data is needed)
//   l    = sum_i w_i (U_{i,c_i} - logsumexp_k U_ik)    (Eq. 5)
//   g    = sum_i w_i J_i^T (e_i - P_i)                 (Eq. 9 chunk by chunk)
//   Ybar_i = sum_k P_ik y_ik                            (used by the centred
//          alpha blocks of the Hessian)
//
// A workgroup (4 waves) walks tiles of 16 observations with a fixed stride,
// so every sum has a fixed partition for a given shape and the result is
// bitwise reproducible.  Per tile:
//   1. X of the tile goes to LDS transposed (one coalesced read);
//   2. X beta for the 16 observations on FP64 MFMA (16 x 16 output tiles,
//      beta gathered from theta), into LDS;
//   3. one wave per observation, lanes over alternatives: the Y and Z terms
//      (read straight from HBM), max / exp / sum by DPP reductions, P and
//      Ybar to HBM, residual R_ik = w_i (e_ik - P_ik) back into LDS, the
//      gamma gradient into per-wave LDS sums;
//   4. the beta gradient X^T R on FP64 MFMA, accumulated in registers
//      across all of the workgroup's tiles.
// At the end each workgroup writes one partial row, reduced in a fixed
// order by k_pass_reduce.
//
// Hessian-vector mode (HV): with v in theta's place, step 2 and the Y/Z
// terms give u_i = J_i v, the utilities of v.  With the probabilities P at
// the current theta read from HBM, s_ik = P_ik (u_ik - sum_k' P_ik' u_ik')
// is (diag P_i - P_i P_i^T) u_i, and R_ik = -w_i s_ik takes the residual's
// place, so the gradient sums give H v = -sum_i w_i J_i^T (diag P_i -
// P_i P_i^T) J_i v, the Hessian of Eq. 10 applied to v, without forming H.
#include "mnl_common.h"

namespace mnl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kTB = 16;           // observations per tile (MFMA rows)
constexpr int kXS = kTB + 1;      // LDS row stride of the transposed X tile

// Lane permutation of a double by DPP (both 32-bit halves).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL,
                                             0xf, 0xf, false);
  return __builtin_bit_cast(double,
                            (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}
__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), l);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), l);
  return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}
// Wave-wide sum / max: butterflies within each 16-lane row (lane xor 1,
// xor 2, then the mirrored half-row and row: every lane of a row combines
// the same two values, so the row agrees bitwise), then the four row
// results in a fixed order.  Every lane must be active.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) +
         (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
              fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

struct Lay {  // LDS layout, offsets in doubles
  int Kp, p16, cap;
  int xs, us, ws, gz, gam, alf, red, ch, ysc, lg;
  int yb, ys;     // y-row buffers (two per wave) and their stride
  int total;
};

// register slots for the z and y values of one alternative
__host__ __device__ inline int pass_cap(const Dims &d) {
  const int mx = d.a > d.g ? d.a : d.g;
  return mx <= 4 ? 4 : (mx <= 8 ? 8 : 16);
}

__host__ __device__ inline Lay make_lay(const Dims &d, bool yl = false) {
  Lay L;
  L.Kp = (d.K + 15) & ~15;
  L.p16 = (d.p + 15) & ~15;
  L.cap = pass_cap(d);
  int o = 0;
  L.xs = o;  o += L.p16 * kXS;                // X^T tile [p16][kXS]
  L.us = o;  o += kTB * L.Kp;                 // U, then e, then R [kTB][Kp]
  L.ws = o;  o += kTB;                        // weights
  L.gz = o;  o += kWaves * d.K * d.a;         // gamma gradient per wave
  L.gam = o; o += d.K * d.a;                  // gamma
  L.alf = o; o += d.g;                        // alpha
  L.red = o; o += kWaves * (1 + d.g);         // loglik, alpha grad per wave
  L.ch = o;  o += kTB / 2;                    // choices, two per double
  // Ybar transpose: per wave CAP rows of 64 values, one padding slot after
  // every CAP values, so the transposed reads hit distinct banks
  L.ysc = o; o += d.g > 0 ? kWaves * L.cap * (kWave + kWave / L.cap) : 0;
  L.lg = o;  o += 2 * kTB;                    // max and sum per observation
  // y rows of one observation (K g values), two buffers per wave: the
  // wave's next observation streams in while the current one is used
  L.ys = (d.K * d.g + 1) & ~1;
  o = (o + 1) & ~1;
  L.yb = o;  o += yl ? kWaves * 2 * L.ys : 0;
  L.total = o;
  return L;
}

// NTW: beta-gradient MFMA tiles per wave; CAP: register slots for the z
// and y values of one alternative (>= a and >= g); ZR: a > 0 (without Z
// no register is spent on z, gamma or the gamma gradient).  With NTW <= 2
// and CAP <= 8 the kernel is held to 168 VGPRs for three waves per SIMD:
// more loads in flight per CU outweigh the few registers spilled.
// YL: the y rows reach the wave through LDS, copied asynchronously one
// observation ahead (K g even, Y 16-byte aligned); otherwise each
// observation reads them from global memory when it starts.
template <int NTW, int CAP, bool ZR, bool HV, bool YL>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(NTW <= 2 && CAP <= 8 ? 3 : 1))) void
k_pass(PassArgs A, int64_t stride) {
  constexpr int CZ = ZR ? CAP : 1;
  extern __shared__ double sm[];
  const Dims d = A.d;
  const Lay L = make_lay(d, YL);
  const int K = d.K, p = d.p, g = d.g, a = d.a, Kp = L.Kp, p16 = L.p16;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  double *xs = sm + L.xs, *us = sm + L.us, *ws = sm + L.ws, *gz = sm + L.gz,
         *gam = sm + L.gam, *alf = sm + L.alf, *red = sm + L.red,
         *lgm = sm + L.lg, *lgs = sm + L.lg + kTB;
  int32_t *chs = reinterpret_cast<int32_t *>(sm + L.ch);
  const double *th = A.theta;
  const int64_t offg = d.off_gamma(), offa = d.off_alpha();
  const int Ka = K * a;
  for (int e = tid; e < Ka; e += kThreads) gam[e] = th[offg + e];
  for (int e = tid; e < g; e += kThreads) alf[e] = th[offa + e];
  for (int e = tid; e < kWaves * Ka; e += kThreads) gz[e] = 0.0;
  for (int e = tid; e < kWaves * (1 + g); e += kThreads) red[e] = 0.0;
  // beta-gradient tiles (16 features x 16 alternatives), wave wv owns
  // tiles wv, wv + 4, ... of the row-major tile grid
  const int nct = Kp / 16, nbt = (p16 / 16) * nct;
  d4 acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) acc[j] = d4{0, 0, 0, 0};
  double lsum = 0.0;  // per lane: choice terms of its alternatives, and
                      // on lane 0 the log-normalisers
  const int p4 = (p + 3) / 4;
  __syncthreads();
  // lane k < 64 keeps gamma_k and its gamma-gradient sums in registers
  // (alternatives past 64 use the per-wave LDS sums)
  double gamr[CZ], gzr[CZ];
#pragma unroll
  for (int c = 0; c < CZ; ++c) {
    gamr[c] = (ZR && c < a && lane < K) ? gam[lane * a + c] : 0.0;
    gzr[c] = 0.0;
  }

  const int64_t ntiles = (d.N + kTB - 1) / kTB;
  // y rows through LDS: 16-byte copies of observation gn into buffer b of
  // this wave (no registers held while they are in flight)
  double *ybuf = sm + L.yb + wv * 2 * L.ys;
  const int nyb = K * g * 8;
  auto ycopy = [&](int64_t gn, int b) {
    const uint32_t *src =
        reinterpret_cast<const uint32_t *>(A.Y + gn * int64_t(K) * g);
    char *dst = reinterpret_cast<char *>(ybuf + b * L.ys);
    for (int o = 0; o < nyb; o += 1024)
      if (o + 16 * lane < nyb)
        __builtin_amdgcn_global_load_lds(src + o / 4 + 4 * lane,
                                         (lds_void_t *)(dst + o), 16, 0, 0);
  };
  int ypar = 0;
  if constexpr (YL) {
    const int64_t g0 = int64_t(blockIdx.x) * kTB + wv;
    if (g0 < d.N) ycopy(g0, 0);
  }
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = t * kTB;
    const int nobs = (int)((d.N - i0) < kTB ? (d.N - i0) : kTB);

    // ---- 1. X^T, w and choices of the tile -----------------------------------
    {
      const double *srx = A.X + i0 * p;
      const int nx = nobs * p;
      for (int e = tid; e < kTB * p16; e += kThreads) {
        const int i = e / p16, aa = e - i * p16;
        xs[aa * kXS + i] = (aa < p && i < nobs) ? srx[i * p + aa] : 0.0;
      }
      (void)nx;
      if (tid < kTB) {
        ws[tid] = tid < nobs ? (A.w ? A.w[i0 + tid] : 1.0) : 0.0;
        // an out-of-range choice (rejected when validation is on) is
        // clamped so that no access leaves the tile
        // (no choices: predictions only, alternative 0 stands in)
        int c = (tid < nobs && A.choice) ? A.choice[i0 + tid] : 0;
        chs[tid] = c < 0 ? 0 : (c >= K ? K - 1 : c);
      }
    }
    __syncthreads();

    // ---- 2. X beta on MFMA -----------------------------------------------------
    for (int ct = wv; ct < nct; ct += kWaves) {
      d4 u = d4{0, 0, 0, 0};
      const int kc = ct * 16 + (lane & 15);
      for (int ks = 0; ks < p4; ++ks) {
        const int aa = 4 * ks + (lane >> 4);
        const double av = xs[aa * kXS + (lane & 15)];
        const double bv = (aa < p && kc >= 1 && kc < K)
                              ? th[int64_t(kc - 1) * p + aa] : 0.0;
        u = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, u, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) us[((lane >> 4) + 4 * r) * Kp + kc] = u[r];
    }
    __syncthreads();

    // ---- 3. softmax, log-likelihood, residuals, Ybar, gamma gradient ----------
    // Lane k holds alternative k of the first 64 (its z and y values in
    // registers, loaded once); alternatives past 64 are revisited in chunks.
    for (int i = wv; i < nobs; i += kWaves) {
      const double wi = ws[i];
      const int ci = chs[i];
      const int64_t gi = i0 + i;
      const double *yr;
      if constexpr (YL) {
        // wait for every vector memory operation of the wave, this
        // observation's row copies among them (also the previous
        // observation's stores, and at a tile's first observation the
        // tile's loads); the copy of the wave's next observation, in this
        // tile or its first of the next, goes to the other buffer
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        int64_t gn = -1;
        if (i + kWaves < nobs) {
          gn = gi + kWaves;
        } else if (t + gridDim.x < ntiles) {
          const int64_t fn = (t + gridDim.x) * kTB + wv;
          if (fn < d.N) gn = fn;
        }
        if (gn >= 0) ycopy(gn, ypar ^ 1);
        yr = ybuf + ypar * L.ys;
        ypar ^= 1;
      } else {
        yr = A.Y + gi * K * g;
      }
      const double *zr = A.Z + gi * Ka;
      double *ui = us + i * Kp;
      double zv[CZ], yv[CAP];
      const bool own = lane < K;
#pragma unroll
      for (int c = 0; c < CZ; ++c)
        zv[c] = (ZR && c < a && own) ? zr[lane * a + c] : 0.0;
#pragma unroll
      for (int c = 0; c < CAP; ++c)
        yv[c] = (c < g && own) ? yr[lane * g + c] : 0.0;
      // alternatives 64..127 (one more chunk): their y values load with
      // the first chunk's, one round trip for both, instead of being read
      // from memory in each loop below
      // (kernels held to three waves per SIMD have no registers for it)
      constexpr bool kY2 = !HV && CAP >= 8 && !(NTW <= 2 && CAP <= 8);
      constexpr int C2 = kY2 ? CAP : 1;
      const bool two = kY2 && K > kWave && K <= 2 * kWave;
      double yv2[C2];
#pragma unroll
      for (int c = 0; c < C2; ++c)
        yv2[c] = (two && c < g && kWave + lane < K)
                     ? yr[(kWave + lane) * g + c] : 0.0;
      double m = -INFINITY;
      {
        double u = -INFINITY;
        if (own) {
          u = ui[lane];
#pragma unroll
          for (int c = 0; c < CZ; ++c)
            if (ZR && c < a) u = fma(zv[c], gamr[c], u);
#pragma unroll
          for (int c = 0; c < CAP; ++c)
            if (c < g) u = fma(yv[c], alf[c], u);
          ui[lane] = u;
        }
        m = u;
      }
      for (int k0 = kWave; k0 < K; k0 += kWave) {
        const int k = k0 + lane;
        if (k < K) {
          double u = ui[k];
          for (int c = 0; c < a; ++c) u = fma(zr[k * a + c], gam[k * a + c], u);
          if (two) {
#pragma unroll
            for (int c = 0; c < C2; ++c)
              if (c < g) u = fma(yv2[c], alf[c], u);
          } else {
            for (int c = 0; c < g; ++c) u = fma(yr[k * g + c], alf[c], u);
          }
          ui[k] = u;
          m = fmax(m, u);
        }
      }
      if constexpr (HV) {
        const double *pin = A.Pin + gi * K;
        double pu = 0.0;
        for (int k0 = 0; k0 < K; k0 += kWave) {
          const int k = k0 + lane;
          if (k < K) pu = fma(pin[k], ui[k], pu);
        }
        const double ub = wave_sum(pu);
        for (int k0 = 0; k0 < K; k0 += kWave) {
          const int k = k0 + lane;
          if (k < K) {
            const double R = -wi * (pin[k] * (ui[k] - ub));
            ui[k] = R;
            if (k0 == 0) {
#pragma unroll
              for (int c = 0; c < CZ; ++c)
                if (ZR && c < a) gzr[c] = fma(R, zv[c], gzr[c]);
            } else {
              double *gzk = gz + wv * Ka + k * a;
              for (int c = 0; c < a; ++c) gzk[c] = fma(R, zr[k * a + c], gzk[c]);
            }
          }
        }
        if (g > 0) {
          // alpha part: sum_k R_ik y_ikc, all c reduced together as for Ybar
          double part[CAP];
          const double R0 = own ? ui[lane] : 0.0;
#pragma unroll
          for (int c = 0; c < CAP; ++c) part[c] = (c < g) ? R0 * yv[c] : 0.0;
          for (int k0 = kWave; k0 < K; k0 += kWave) {
            const int k = k0 + lane;
            if (k < K) {
              const double R = ui[k];
#pragma unroll
              for (int c = 0; c < CAP; ++c)
                if (c < g) part[c] = fma(R, yr[k * g + c], part[c]);
            }
          }
          constexpr int RS = kWave + kWave / CAP;   // padded row
          double *scr = sm + L.ysc + wv * (CAP * RS);
#pragma unroll
          for (int c = 0; c < CAP; ++c)
            if (c < g) scr[c * RS + lane + lane / CAP] = part[c];
          __builtin_amdgcn_wave_barrier();
          constexpr int LPC = kWave / CAP;
          const int cl = lane / LPC, jl = lane % LPC;
          double yb = 0.0;
          if (cl < g) {
#pragma unroll
            for (int q = 0; q < CAP; ++q)
              yb += scr[cl * RS + jl * (CAP + 1) + q];
          }
          yb += dpp_f64<0xB1>(yb);
          if constexpr (LPC >= 4) yb += dpp_f64<0x4E>(yb);
          if constexpr (LPC >= 8) yb += dpp_f64<0x141>(yb);
          if constexpr (LPC >= 16) yb += dpp_f64<0x140>(yb);
          __builtin_amdgcn_wave_barrier();
          if (jl == 0 && cl < g) red[wv * (1 + g) + 1 + cl] += yb;
        }
        continue;
      }
      m = wave_max(m);
      double s = 0.0;
      for (int k0 = 0; k0 < K; k0 += kWave) {
        const int k = k0 + lane;
        if (k < K) {
          const double u = ui[k];
          const double e = exp(u - m);
          if (k == ci) lsum += wi * u;  // U at the choice, one lane
          s += e;
          ui[k] = e;
        }
      }
      s = wave_sum(s);
      // the log-normaliser is taken after the tile's observations, one
      // observation per lane
      if (lane == 0) {
        lgm[i] = m;
        lgs[i] = s;
      }
      const double inv = 1.0 / s;
      if (g > 0) {
        // Ybar_c = sum_k P_k y_kc, all c reduced together
        double part[CAP];
        const double P0 = own ? ui[lane] * inv : 0.0;
#pragma unroll
        for (int c = 0; c < CAP; ++c) part[c] = (c < g) ? P0 * yv[c] : 0.0;
        for (int k0 = kWave; k0 < K; k0 += kWave) {
          const int k = k0 + lane;
          if (k < K) {
            const double P = ui[k] * inv;
            if (two) {
#pragma unroll
              for (int c = 0; c < C2; ++c)
                if (c < g) part[c] = fma(P, yv2[c], part[c]);
            } else {
#pragma unroll
              for (int c = 0; c < CAP; ++c)
                if (c < g) part[c] = fma(P, yr[k * g + c], part[c]);
            }
          }
        }
        // all g sums at once: the 64 x CAP partial values go through this
        // wave's LDS block transposed, lane (c, j) adds CAP of them in order
        // and each group of 64 / CAP lanes combines its results by DPP
        // (every lane of a group ends with the same bits)
        constexpr int RS = kWave + kWave / CAP;   // padded row
        double *scr = sm + L.ysc + wv * (CAP * RS);
#pragma unroll
        for (int c = 0; c < CAP; ++c)
          if (c < g) scr[c * RS + lane + lane / CAP] = part[c];
        __builtin_amdgcn_wave_barrier();
        constexpr int LPC = kWave / CAP;
        const int cl = lane / LPC, jl = lane % LPC;
        double yb = 0.0;
        if (cl < g) {
#pragma unroll
          for (int q = 0; q < CAP; ++q)
            yb += scr[cl * RS + jl * (CAP + 1) + q];
        }
        yb += dpp_f64<0xB1>(yb);
        if constexpr (LPC >= 4) yb += dpp_f64<0x4E>(yb);
        if constexpr (LPC >= 8) yb += dpp_f64<0x141>(yb);
        if constexpr (LPC >= 16) yb += dpp_f64<0x140>(yb);
        __builtin_amdgcn_wave_barrier();
        if (jl == 0 && cl < g) {
          if (A.Ybar) A.Ybar[gi * g + cl] = yb;
          // alpha gradient: w_i (y_{i,c_i} - ybar_i)   (Eq. 9, centred)
          red[wv * (1 + g) + 1 + cl] += wi * (yr[ci * g + cl] - yb);
        }
      }
      const int64_t row = gi * K;
      for (int k0 = 0; k0 < K; k0 += kWave) {
        const int k = k0 + lane;
        if (k < K) {
          const double P = ui[k] * inv;
          if (A.P) A.P[row + k] = P;
          if (A.P32) A.P32[row + k] = (float)P;
          const double R = wi * ((k == ci ? 1.0 : 0.0) - P);
          ui[k] = R;
          if (k0 == 0) {
#pragma unroll
            for (int c = 0; c < CZ; ++c)
              if (ZR && c < a) gzr[c] = fma(R, zv[c], gzr[c]);
          } else {
            double *gzk = gz + wv * Ka + k * a;
            for (int c = 0; c < a; ++c) gzk[c] = fma(R, zr[k * a + c], gzk[c]);
          }
        }
      }
    }
    // log-normalisers of this wave's observations of the tile, lane q
    // taking observation wv + 4 q
    {
      const int iq = wv + kWaves * lane;
      if (!HV && lane < kTB / kWaves && iq < nobs)
        lsum -= ws[iq] * (lgm[iq] + log(lgs[iq]));
    }
    __syncthreads();

    // ---- 4. beta gradient X^T R on MFMA ---------------------------------------
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int bt = wv + kWaves * j;
      if (bt < nbt) {
        const int rt = bt / nct, ct = bt - rt * nct;
        const double *xa = xs + (16 * rt + (lane & 15)) * kXS + (lane >> 4);
        const double *rb = us + (lane >> 4) * Kp + 16 * ct + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < kTB / 4; ++ks)
          acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              xa[4 * ks], rb[4 * ks * Kp], acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---- this workgroup's partial row --------------------------------------------
  // the register gamma-gradient sums join the per-wave LDS sums
  if (ZR && lane < K) {
#pragma unroll
    for (int c = 0; c < CZ; ++c)
      if (c < a) gz[wv * Ka + lane * a + c] = gzr[c];
  }
  __syncthreads();
  double *out = A.partial + int64_t(blockIdx.x) * stride;
  lsum = wave_sum(lsum);
  if (lane == 0) red[wv * (1 + g)] = lsum;
  __syncthreads();
  if (tid == 0) {
    double l = 0.0;
    for (int v = 0; v < kWaves; ++v) l += red[v * (1 + g)];
    out[0] = l;
  }
  for (int c = tid; c < g; c += kThreads) {
    double s = 0.0;
    for (int v = 0; v < kWaves; ++v) s += red[v * (1 + g) + 1 + c];
    out[1 + offa + c] = s;
  }
  for (int e = tid; e < Ka; e += kThreads) {
    double s = 0.0;
    for (int v = 0; v < kWaves; ++v) s += gz[v * Ka + e];
    out[1 + offg + e] = s;
  }
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int bt = wv + kWaves * j;
    if (bt < nbt) {
      const int rt = bt / nct, ct = bt - rt * nct;
      const int kk = 16 * ct + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int aa = 16 * rt + (lane >> 4) + 4 * r;
        if (aa < p && kk >= 1 && kk < K)
          out[1 + int64_t(kk - 1) * p + aa] = acc[j][r];
      }
    }
  }
}

// Sum the partial rows: 64 columns per workgroup, 16 groups of rows each
// summed with four accumulators, the group sums added in a fixed order.
__global__ __launch_bounds__(1024) void k_pass_reduce(
    const double *__restrict__ partial, int grid, int64_t stride, int64_t np,
    double *loglik, double *grad) {
  __shared__ double red[16][64];
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t j = int64_t(blockIdx.x) * 64 + col;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j <= np) {
    int q = 0;
    for (int b = grp; b < grid; b += 16, ++q)
      acc[q & 3] += partial[int64_t(b) * stride + j];
  }
  red[grp][col] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (grp == 0 && j <= np) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += red[q][col];
    if (j == 0) {
      if (loglik) *loglik = s;
    } else if (grad) {
      grad[j - 1] = s;
    }
  }
}

}  // namespace

int pass_plan(const Dims &d, PassPlan *plan) {
  const Lay L = make_lay(d);
  const int nbt = (L.p16 / 16) * (L.Kp / 16);
  const int per_wave = (nbt + kWaves - 1) / kWaves;
  int ntw = 1;
  while (ntw < per_wave) ntw *= 2;
  if (ntw > 32) return MNL_ERR_UNSUPPORTED;
  const int mx = d.a > d.g ? d.a : d.g;
  if (mx > 16) return MNL_ERR_UNSUPPORTED;
  plan->cap = L.cap;
  if (size_t(L.total) * 8 > 160 * 1024) return MNL_ERR_UNSUPPORTED;
  plan->ntw = ntw;
  plan->tb = kTB;
  plan->lds_bytes = size_t(L.total) * 8;
  const int64_t ntiles = (d.N + kTB - 1) / kTB;
  // kernels with at most two beta tiles per wave and eight value slots are
  // built for three waves per SIMD (three workgroups per CU, LDS allowing):
  // one round of 3 x 256 workgroups; the others hold two waves per SIMD (one
  // round of 2 x 256) or one (two rounds).  The count depends on the shape
  // alone, so the sums are deterministic.
  const int gmax =
      (ntw <= 2 && L.cap <= 8 && 3 * plan->lds_bytes <= 160 * 1024) ? 768
                                                                     : 512;
  // two workgroups per CU with eight value slots: the y rows go through
  // LDS when both workgroups' buffers fit
  plan->yl = 0;
  if (gmax == 512 && L.cap == 8 && d.g > 0 && (d.K * d.g) % 2 == 0) {
    const Lay Ly = make_lay(d, true);
    if (2 * size_t(Ly.total) * 8 <= 160 * 1024) {
      plan->yl = 1;
      plan->lds_bytes = size_t(Ly.total) * 8;
    }
  }
  plan->grid = (int)(ntiles < gmax ? ntiles : gmax);
  plan->stride = 1 + d.np;
  return MNL_OK;
}

namespace {
template <int J, int C, bool Z, bool H, bool Y>
hipError_t launch_pass_k(const PassPlan &plan, const PassArgs &a,
                         hipStream_t s) {
  const size_t lds = plan.lds_bytes;
  hipError_t e = raise_lds_limit(
      reinterpret_cast<const void *>(&k_pass<J, C, Z, H, Y>), (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pass<J, C, Z, H, Y>), dim3(plan.grid),
                     dim3(kThreads), lds, s, a, plan.stride);
  return hipSuccess;
}
// the y rows go through LDS where the plan allows it and Y is 16-byte
// aligned (the Hessian-vector mode reads them from global memory)
template <int J, int C, bool Z, bool H>
hipError_t launch_pass_y(const PassPlan &plan, const PassArgs &a,
                         hipStream_t s) {
  if constexpr (C == 8 && !H) {
    if (plan.yl && (reinterpret_cast<uintptr_t>(a.Y) & 15) == 0)
      return launch_pass_k<J, C, Z, H, true>(plan, a, s);
  }
  return launch_pass_k<J, C, Z, H, false>(plan, a, s);
}
}  // namespace

hipError_t launch_pass(const PassPlan &plan, const PassArgs &a,
                       hipStream_t s) {
#define MNL_PASS_LAUNCH3(J, C, Z, H)                                          \
  do {                                                                        \
    hipError_t e_ = launch_pass_y<J, C, Z, H>(plan, a, s);                    \
    if (e_ != hipSuccess) return e_;                                          \
  } while (0)
#define MNL_PASS_LAUNCH2(J, C, Z)                                             \
  do {                                                                        \
    if (a.Pin) MNL_PASS_LAUNCH3(J, C, Z, true);                               \
    else MNL_PASS_LAUNCH3(J, C, Z, false);                                    \
  } while (0)
#define MNL_PASS_LAUNCH(J, C)                                                 \
  do {                                                                        \
    if (a.d.a > 0) MNL_PASS_LAUNCH2(J, C, true);                              \
    else MNL_PASS_LAUNCH2(J, C, false);                                       \
  } while (0)
#define MNL_PASS_CAP(J)                                                       \
  do {                                                                        \
    if (plan.cap == 4) MNL_PASS_LAUNCH(J, 4);                                 \
    else if (plan.cap == 8) MNL_PASS_LAUNCH(J, 8);                            \
    else MNL_PASS_LAUNCH(J, 16);                                              \
  } while (0)
  switch (plan.ntw) {
    case 1: MNL_PASS_CAP(1); break;
    case 2: MNL_PASS_CAP(2); break;
    case 4: MNL_PASS_CAP(4); break;
    case 8: MNL_PASS_CAP(8); break;
    case 16: MNL_PASS_CAP(16); break;
    default: MNL_PASS_CAP(32); break;
  }
#undef MNL_PASS_CAP
#undef MNL_PASS_LAUNCH
#undef MNL_PASS_LAUNCH2
#undef MNL_PASS_LAUNCH3
  return hipGetLastError();
}

hipError_t launch_pass_reduce(const PassPlan &plan, const double *partial,
                              double *loglik, double *grad, int64_t np,
                              hipStream_t s) {
  const int64_t n = np + 1;
  dim3 block(1024), grid((unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(k_pass_reduce, grid, block, 0, s, partial, plan.grid,
                     plan.stride, np, loglik, grad);
  return hipGetLastError();
}

// ---- small vector kernels ---------------------------------------------------------

namespace {
__global__ void k_axpy(const double *x, const double *d, double t, double *out,
                       int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fma(t, d[i], x[i]);
}

__global__ __launch_bounds__(256) void k_sumsq(const double *x, int64_t n,
                                               double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(x[i], x[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// The scalars one Newton-step decision needs, in one buffer for one copy
// to the host: out[0] the factorisation status (0 without one), out[1]
// l = lg[0], out[2] |g|^2 over lg[1..n] (summed as k_sumsq does).
__global__ __launch_bounds__(256) void k_scalars(const double *lg, int64_t n,
                                                 const int32_t *status,
                                                 double *out) {
  __shared__ double red[256];
  const double *x = lg + 1;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(x[i], x[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = status ? double(status[0]) : 0.0;
    out[1] = lg[0];
    out[2] = red[0];
  }
}

__global__ void k_validate(Dims d, const double *X, const double *Y,
                           const double *Z, const double *w,
                           const int32_t *choice, int32_t *flags) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  int bad_choice = (choice[i] < 0 || choice[i] >= d.K) ? 1 : 0;
  int bad = 0;
  for (int j = 0; j < d.p; ++j) bad |= !isfinite(X[i * d.p + j]);
  for (int64_t j = 0; j < int64_t(d.K) * d.g; ++j)
    bad |= !isfinite(Y[i * d.K * d.g + j]);
  for (int64_t j = 0; j < int64_t(d.K) * d.a; ++j)
    bad |= !isfinite(Z[i * d.K * d.a + j]);
  if (w) bad |= !(isfinite(w[i]) && w[i] >= 0.0);
  if (bad_choice) atomicAdd(&flags[0], 1);
  if (bad) atomicAdd(&flags[1], 1);
}
}  // namespace

hipError_t launch_axpy(const double *x, const double *d, double t, double *out,
                       int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, x, d, t, out, n);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double *x, int64_t n, double *out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_scalars(const double *lg, int64_t n, const int32_t *status,
                          double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars, dim3(1), dim3(256), 0, s, lg, n, status, out);
  return hipGetLastError();
}

hipError_t launch_validate(const Dims &d, const double *X, const double *Y,
                           const double *Z, const double *w,
                           const int32_t *choice, int32_t *flags,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((d.N + 255) / 256)),
                     dim3(256), 0, s, d, X, Y, Z, w, choice, flags);
  return hipGetLastError();
}

// ---- truncated conjugate gradients (inexact Newton) ----------------------------

namespace {
// sum over threads of one workgroup of 1024, in a fixed tree order; every
// thread returns the total
__device__ inline double block_sum_1024(double v, double *red) {
  const int t = threadIdx.x;
  __syncthreads();   // red may still be read from a previous sum
  red[t] = v;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  return red[0];
}

// d = 0, r = p = g, scal[0] = g.g
__global__ __launch_bounds__(1024) void k_cg_init(const double *g, double *d,
                                                  double *r, double *p,
                                                  int64_t n, double *scal) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double gi = g[i];
    d[i] = 0.0;
    r[i] = gi;
    p[i] = gi;
    s = fma(gi, gi, s);
  }
  s = block_sum_1024(s, red);
  if (threadIdx.x == 0) {
    scal[0] = s;
    scal[1] = 0.0;
  }
}

// One conjugate-gradient step on (-H) d = g given Hp = H p:
// pAp = p.(-H p); if pAp > 0: alpha = rr / pAp, d += alpha p,
// r -= alpha (-H p), rr' = r.r, p = r + (rr' / rr) p.  scal[0] holds rr
// (updated), scal[1] receives pAp (d, r, p untouched when pAp <= 0).
__global__ __launch_bounds__(1024) void k_cg_update(const double *Hp,
                                                    double *d, double *r,
                                                    double *p, int64_t n,
                                                    double *scal) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s = fma(p[i], -Hp[i], s);
  const double pAp = block_sum_1024(s, red);
  const double rr = scal[0];
  if (!(pAp > 0.0)) {
    if (threadIdx.x == 0) scal[1] = pAp;
    return;   // uniform: every thread holds the same pAp
  }
  const double alpha = rr / pAp;
  s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    d[i] = fma(alpha, p[i], d[i]);
    const double ri = fma(alpha, Hp[i], r[i]);
    r[i] = ri;
    s = fma(ri, ri, s);
  }
  const double rr_new = block_sum_1024(s, red);
  const double beta = rr_new / rr;
  for (int64_t i = threadIdx.x; i < n; i += 1024) p[i] = fma(beta, p[i], r[i]);
  if (threadIdx.x == 0) {
    scal[0] = rr_new;
    scal[1] = pAp;
  }
}
}  // namespace

hipError_t launch_cg_init(const double *g, double *d, double *r, double *p,
                          int64_t n, double *scal, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1024), 0, s, g, d, r, p, n,
                     scal);
  return hipGetLastError();
}

hipError_t launch_cg_update(const double *Hp, double *d, double *r, double *p,
                            int64_t n, double *scal, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(1), dim3(1024), 0, s, Hp, d, r, p, n,
                     scal);
  return hipGetLastError();
}

}  // namespace mnl
