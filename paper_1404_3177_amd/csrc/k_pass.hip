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
// One workgroup (4 waves) walks tiles of TB observations with a fixed
// stride, so every sum has a fixed partition for a given shape and the
// result is bitwise reproducible.  Per tile:
//   1. stage X (transposed), Y, Z, w, choice of the tile in LDS (coalesced);
//   2. U = X beta^T as a register-blocked product from LDS, plus the Y/Z
//      terms;
//   3. one wave per row: max / exp / sum by wave reductions, P and Ybar to
//      HBM, residual R_ik = w_i (e_ik - P_ik) back into LDS;
//   4. gradient partials: beta (X^T R) and gamma (sum_i R_ik z_ik) live in
//      registers owned by fixed threads across tiles; alpha in LDS.
// At the end each workgroup writes one partial row, reduced in a fixed
// order by k_pass_reduce.
#include "mnl_common.h"

namespace mnl {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct Lay {  // LDS layout, offsets in doubles
  int Kp, tb;
  int bs, gs, as, xs, us, ys, zs, ws, gacc, lacc, ch;  // ch: int offset
  int total;                                           // doubles
};

__host__ __device__ inline Lay make_lay(const Dims &d, int tb, bool beta_lds) {
  Lay L;
  L.Kp = (d.K + 1) & ~1;
  L.tb = tb;
  int o = 0;
  L.bs = o; o += beta_lds ? d.p * L.Kp : 0;
  L.gs = o; o += d.K * d.a;
  L.as = o; o += d.g;
  L.xs = o; o += d.p * tb;
  L.us = o; o += tb * L.Kp;
  L.ys = o; o += tb * d.K * d.g;
  L.zs = o; o += tb * d.K * d.a;
  L.ws = o; o += tb;
  L.gacc = o; o += kWaves * d.g;
  L.lacc = o; o += kWaves;
  L.ch = o;  o += (tb + 1) / 2;  // int32 choices packed two per double
  L.total = o;
  return L;
}

template <bool BETA_LDS, int JMAX>
__global__ __launch_bounds__(kThreads) void k_pass(PassArgs A, int tb,
                                                   int64_t stride) {
  extern __shared__ double sm[];
  const Dims d = A.d;
  const Lay L = make_lay(d, tb, BETA_LDS);
  const int K = d.K, p = d.p, g = d.g, a = d.a, Kp = L.Kp;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  double *bs = sm + L.bs, *gs = sm + L.gs, *as = sm + L.as, *xs = sm + L.xs,
         *us = sm + L.us, *ys = sm + L.ys, *zs = sm + L.zs, *ws = sm + L.ws,
         *gacc = sm + L.gacc, *lacc = sm + L.lacc;
  int32_t *chs = reinterpret_cast<int32_t *>(sm + L.ch);
  const double *th = A.theta;
  const int64_t offg = d.off_gamma(), offa = d.off_alpha();

  // coefficients: beta_s[a][k] (k = 0 column is the base, all zero)
  if (BETA_LDS) {
    for (int idx = tid; idx < p * Kp; idx += kThreads) {
      int aa = idx / Kp, k = idx - aa * Kp;
      bs[idx] = (k >= 1 && k < K) ? th[int64_t(k - 1) * p + aa] : 0.0;
    }
  }
  for (int idx = tid; idx < K * a; idx += kThreads) gs[idx] = th[offg + idx];
  for (int idx = tid; idx < g; idx += kThreads) as[idx] = th[offa + idx];
  for (int idx = tid; idx < kWaves * g; idx += kThreads) gacc[idx] = 0.0;
  if (tid < kWaves) lacc[tid] = 0.0;

  // gradient accumulators owned by this thread
  const int pp2 = (p + 1) / 2, kp2 = Kp / 2;
  const int nub = pp2 * kp2;       // beta 2x2 units
  const int nug = K * a;           // gamma units
  double gb[JMAX][4];
  double gg[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    gb[j][0] = gb[j][1] = gb[j][2] = gb[j][3] = 0.0;
    gg[j] = 0.0;
  }
  double lsum = 0.0;  // wave-uniform
  __syncthreads();

  const int64_t ntiles = (d.N + tb - 1) / tb;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = t * tb;
    const int nobs = (int)((d.N - i0) < tb ? (d.N - i0) : tb);

    // ---- 1. stage the tile ---------------------------------------------
    {
      const double *srx = A.X + i0 * p;
      const int nx = nobs * p;
      batched_copy<8>(
          tb * p, tid, kThreads,
          [&](int e) { return e < nx ? srx[e] : 0.0; },
          [&](int e, double v) {
            const int i = e / p;
            xs[(e - i * p) * tb + i] = v;
          });
      const double *src = A.Y + i0 * K * g;
      batched_copy<8>(
          nobs * K * g, tid, kThreads, [&](int e) { return src[e]; },
          [&](int e, double v) { ys[e] = v; });
      const double *srz = A.Z + i0 * K * a;
      batched_copy<8>(
          nobs * K * a, tid, kThreads, [&](int e) { return srz[e]; },
          [&](int e, double v) { zs[e] = v; });
    }
    for (int i = tid; i < tb; i += kThreads) {
      ws[i] = (i < nobs) ? (A.w ? A.w[i0 + i] : 1.0) : 0.0;
      // an out-of-range choice (rejected when validation is on) is clamped
      // so that no access leaves the tile
      int c = (i < nobs) ? A.choice[i0 + i] : 0;
      chs[i] = c < 0 ? 0 : (c >= K ? K - 1 : c);
    }
    __syncthreads();

    // ---- 2. utilities ------------------------------------------------------
    {
      const int tb2 = tb / 2;
      const int nu = tb2 * kp2;
      for (int u = tid; u < nu; u += kThreads) {
        const int iu = u % tb2, ku = u / tb2;
        const int i = 2 * iu, k = 2 * ku;
        double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
        for (int aa = 0; aa < p; ++aa) {
          const double x0 = xs[aa * tb + i], x1 = xs[aa * tb + i + 1];
          double b0, b1;
          if (BETA_LDS) {
            b0 = bs[aa * Kp + k];
            b1 = bs[aa * Kp + k + 1];
          } else {
            b0 = (k >= 1 && k < K) ? th[int64_t(k - 1) * p + aa] : 0.0;
            b1 = (k + 1 < K) ? th[int64_t(k) * p + aa] : 0.0;
          }
          c00 = fma(x0, b0, c00);
          c01 = fma(x0, b1, c01);
          c10 = fma(x1, b0, c10);
          c11 = fma(x1, b1, c11);
        }
        double cc[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
        for (int di = 0; di < 2; ++di) {
#pragma unroll
          for (int dk = 0; dk < 2; ++dk) {
            const int ii = i + di, kk = k + dk;
            double v = cc[di][dk];
            if (kk < K && ii < nobs) {
              for (int c = 0; c < a; ++c)
                v = fma(zs[(ii * K + kk) * a + c], gs[kk * a + c], v);
              for (int c = 0; c < g; ++c)
                v = fma(ys[(ii * K + kk) * g + c], as[c], v);
            }
            us[ii * Kp + kk] = v;
          }
        }
      }
    }
    __syncthreads();

    // ---- 3. softmax, log-likelihood, residuals, Ybar --------------------------
    for (int i = wv; i < nobs; i += kWaves) {
      const double wi = ws[i];
      const int ci = chs[i];
      double m = -INFINITY;
      for (int k = lane; k < K; k += kWave) m = fmax(m, us[i * Kp + k]);
      m = wave_max(m);
      const double uci = us[i * Kp + ci];
      double s = 0.0;
      for (int k = lane; k < K; k += kWave) {
        const double e = exp(us[i * Kp + k] - m);
        us[i * Kp + k] = e;
        s += e;
      }
      s = wave_sum(s);
      lsum += wi * (uci - (m + log(s)));
      const double inv = 1.0 / s;
      const int64_t row = (i0 + i) * K;
      for (int c = 0; c < g; ++c) {
        double yb = 0.0;
        for (int k = lane; k < K; k += kWave)
          yb = fma(us[i * Kp + k] * inv, ys[(i * K + k) * g + c], yb);
        yb = wave_sum(yb);
        if (lane == 0) {
          if (A.Ybar) A.Ybar[(i0 + i) * g + c] = yb;
          // alpha gradient: w_i (y_{i,c_i} - ybar_i)   (Eq. 9, centred)
          gacc[wv * g + c] += wi * (ys[(i * K + ci) * g + c] - yb);
        }
      }
      for (int k = lane; k < K; k += kWave) {
        const double P = us[i * Kp + k] * inv;
        if (A.P) A.P[row + k] = P;
        if (A.P32) A.P32[row + k] = (float)P;
        us[i * Kp + k] = wi * ((k == ci ? 1.0 : 0.0) - P);
      }
      if (Kp > K && lane == 0) us[i * Kp + K] = 0.0;
    }
    // rows beyond nobs contribute nothing
    for (int idx = nobs * Kp + tid; idx < tb * Kp; idx += kThreads)
      us[idx] = 0.0;
    __syncthreads();

    // ---- 4. gradient partials ------------------------------------------------
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const int u = tid + j * kThreads;
      if (u < nub) {
        const int ku = u % kp2, au = u / kp2;
        const int k = 2 * ku, a0 = 2 * au;
        const bool has1 = (a0 + 1) < p;
        double s00 = gb[j][0], s01 = gb[j][1], s10 = gb[j][2], s11 = gb[j][3];
        for (int i = 0; i < nobs; ++i) {
          const double r0 = us[i * Kp + k], r1 = us[i * Kp + k + 1];
          const double x0 = xs[a0 * tb + i];
          const double x1 = has1 ? xs[(a0 + 1) * tb + i] : 0.0;
          s00 = fma(x0, r0, s00);
          s01 = fma(x0, r1, s01);
          s10 = fma(x1, r0, s10);
          s11 = fma(x1, r1, s11);
        }
        gb[j][0] = s00; gb[j][1] = s01; gb[j][2] = s10; gb[j][3] = s11;
      }
      if (u < nug) {
        const int k = u / a, c = u - (u / a) * a;
        double s0 = gg[j];
        for (int i = 0; i < nobs; ++i)
          s0 = fma(us[i * Kp + k], zs[(i * K + k) * a + c], s0);
        gg[j] = s0;
      }
    }
    __syncthreads();
  }

  // ---- write this workgroup's partial row ---------------------------------------
  double *out = A.partial + int64_t(blockIdx.x) * stride;
  if (lane == 0) lacc[wv] = lsum;
  __syncthreads();
  if (tid == 0) {
    double l = 0.0;
    for (int v = 0; v < kWaves; ++v) l += lacc[v];
    out[0] = l;
  }
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int u = tid + j * kThreads;
    if (u < nub) {
      const int ku = u % kp2, au = u / kp2;
      const int k = 2 * ku, a0 = 2 * au;
      const double v[4] = {gb[j][0], gb[j][1], gb[j][2], gb[j][3]};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int aa = a0 + (q >> 1), kk = k + (q & 1);
        if (aa < p && kk >= 1 && kk < K)
          out[1 + int64_t(kk - 1) * p + aa] = v[q];
      }
    }
    if (u < nug) out[1 + offg + u] = gg[j];
  }
  for (int c = tid; c < g; c += kThreads) {
    double s = 0.0;
    for (int v = 0; v < kWaves; ++v) s += gacc[v * g + c];
    out[1 + offa + c] = s;
  }
}

__global__ void k_pass_reduce(const double *__restrict__ partial, int grid,
                              int64_t stride, int64_t np, double *loglik,
                              double *grad) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j > np) return;
  // eight independent partial sums in a fixed order: deterministic, and
  // many loads in flight
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = 0;
  for (; b + 8 <= grid; b += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += partial[int64_t(b + u) * stride + j];
  }
  for (; b < grid; ++b) acc[b & 7] += partial[int64_t(b) * stride + j];
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                   ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if (j == 0) {
    if (loglik) *loglik = s;
  } else if (grad) {
    grad[j - 1] = s;
  }
}

}  // namespace

int pass_plan(const Dims &d, PassPlan *plan) {
  const int Kp = (d.K + 1) & ~1;
  const int pp2 = (d.p + 1) / 2;
  const int64_t nub = int64_t(pp2) * (Kp / 2);
  const int64_t nug = int64_t(d.K) * d.a;
  const int64_t need = nub > nug ? nub : nug;
  if (need <= 8 * kThreads) plan->jmax = 8;
  else if (need <= 16 * kThreads) plan->jmax = 16;
  else return MNL_ERR_UNSUPPORTED;
  const bool beta_lds = int64_t(d.p) * Kp * 8 <= 64 * 1024;
  plan->beta_in_lds = beta_lds;
  const size_t budget = 80 * 1024;
  int tb = 64;
  while (tb > 2) {
    Lay L = make_lay(d, tb, beta_lds);
    if (size_t(L.total) * 8 <= budget) break;
    tb /= 2;
  }
  Lay L = make_lay(d, tb, beta_lds);
  if (size_t(L.total) * 8 > 150 * 1024) return MNL_ERR_UNSUPPORTED;
  plan->tb = tb;
  plan->lds_bytes = size_t(L.total) * 8;
  const int64_t ntiles = (d.N + tb - 1) / tb;
  plan->grid = (int)(ntiles < 512 ? ntiles : 512);
  plan->stride = 1 + d.np;
  return MNL_OK;
}

hipError_t launch_pass(const PassPlan &plan, const PassArgs &a,
                       hipStream_t s) {
  dim3 grid(plan.grid), block(kThreads);
  const size_t lds = plan.lds_bytes;
#define MNL_PASS_LAUNCH(BL, J)                                                \
  do {                                                                        \
    hipError_t e_ = raise_lds_limit(                                          \
        reinterpret_cast<const void *>(&k_pass<BL, J>), (int)lds);            \
    if (e_ != hipSuccess) return e_;                                          \
    hipLaunchKernelGGL((k_pass<BL, J>), grid, block, lds, s, a, plan.tb,      \
                       plan.stride);                                          \
  } while (0)
  if (plan.beta_in_lds) {
    if (plan.jmax == 8) MNL_PASS_LAUNCH(true, 8);
    else MNL_PASS_LAUNCH(true, 16);
  } else {
    if (plan.jmax == 8) MNL_PASS_LAUNCH(false, 8);
    else MNL_PASS_LAUNCH(false, 16);
  }
#undef MNL_PASS_LAUNCH
  return hipGetLastError();
}

hipError_t launch_pass_reduce(const PassPlan &plan, const double *partial,
                              double *loglik, double *grad, int64_t np,
                              hipStream_t s) {
  const int64_t n = np + 1;
  dim3 block(256), grid((unsigned)((n + 255) / 256));
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
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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

hipError_t launch_validate(const Dims &d, const double *X, const double *Y,
                           const double *Z, const double *w,
                           const int32_t *choice, int32_t *flags,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((d.N + 255) / 256)),
                     dim3(256), 0, s, d, X, Y, Z, w, choice, flags);
  return hipGetLastError();
}

}  // namespace mnl
