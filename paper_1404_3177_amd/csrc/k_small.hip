// Many small fits at once: the Newton-Raphson fit of Sec. 3.1 (Eqs. 2-6,
// 9-10 and the halving line search) run by one workgroup per fit, on chip.
//
// A served stream holds many fits too small to fill the device (a few
// thousand observations, tens of coefficients), whose multi-kernel steps
// are bound by launch and host round-trip latency.  k_fit_small is a
// persistent kernel over a device work list of fit descriptors: each
// workgroup takes the next fit (an atomic counter) and iterates it to its
// stop rule without the host, with theta, the gradient, the Newton
// direction and the whole matrix A = -H (then its L D L^T factor) in LDS.
// One iteration: the Eq. 10 Hessian accumulated over chunks of
// observations staged in LDS, the factorisation with the pivot floor,
// the two triangular solves and the line search, whose trial passes also
// form the gradient at the trial point (kept if the trial is accepted).
// Every sum runs in an order fixed by the fit's own shape, so a fit's
// result does not depend on the other fits of the batch.  FP64 throughout.
#include <cmath>
#include <cstring>

#include "mnl_common.h"

namespace mnl {

namespace {

constexpr int kSmThreads = 256;  // 4 waves
constexpr int kSmWaves = kSmThreads / 64;
constexpr int kSmK = 64, kSmG = 8, kSmNP = 128;
// dynamic LDS of a workgroup at most: 160 KiB less room for the kernel's
// static LDS (the work-list slot)
constexpr size_t kSmLdsMax = 160 * 1024 - 256;
constexpr int kSmChMax = 64, kSmChMin = 4;   // observations per chunk

// A fit of the work list with its LDS layout (offsets in doubles).
struct SmallFit {
  int64_t N;
  int K, p, g, a, np, nbg, npair;   // nbg: beta and gamma coefficients;
                                    // npair: g (g + 1) / 2
  int nbgp;                  // nbg rounded up to a multiple of 16
  int ch;                    // observations per staged chunk
  int seg;                   // lanes per observation (power of two >= K)
  int oA, oTh, oG, oDl, oTr, oTg, oPart, oRed, oAlt, oFoff;
  int oBuf0, oBuf1;          // two staged chunks, each laid out as:
  int bX, bZ, bY, bW, bC;    // X [ch][p], Z [ch][K a], Y [ch][K g], w [ch],
                             // choice [ch] (int32), as in global memory
  int oP, oQ, oS, oU;        // per-chunk products (see chunk_eval)
  int lds_doubles, pad;
  const double *X, *Y, *Z, *w;
  const int32_t *choice;
  const double *theta0;     // NULL: zeros
  double *theta;            // output
};
struct SmallOpts {
  double gtol, ftol, ls_tol_ulps;
  int maxiter, ls_max;
};
struct SmallInfo {
  int iters, ls_iters, ls_backtracks, stop_reason, n_hess, n_pass;
  double loglik, grad_norm, loglik_diff;
  // device clock ticks of the phases: first pass, Hessians, factorisations
  // and solves, line-search passes
  uint64_t tk_first, tk_hess, tk_chol, tk_ls;
};

__device__ inline double seg_max(double v, int seg) {
  for (int o = seg >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double seg_sum(double v, int seg) {
  for (int o = seg >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Asynchronous copy of n dwords from global memory into LDS by the whole
// workgroup: 64-dword blocks go round-robin to the waves, and each lane's
// dword lands straight in LDS (no registers).  A wave's copies have landed
// after its s_waitcnt vmcnt(0).
__device__ inline void wg_copy_lds(const void *src, double *dst, int n) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t *s = static_cast<const uint32_t *>(src);
  char *dc = reinterpret_cast<char *>(dst);
  for (int c = wv * 64; c < n; c += kSmThreads)
    if (c + lane < n)
      __builtin_amdgcn_global_load_lds(s + c + lane,
                                       (lds_void_t *)(dc + 4 * c), 4, 0, 0);
}

// Start staging observations i0 .. i0 + nobs - 1 into buffer b.  Without
// weights the buffer's w holds ones, written once per fit.
__device__ inline void issue_chunk(const SmallFit &F, int64_t i0, int nobs,
                                   double *b) {
  const int p = F.p, Ka = F.K * F.a, Kg = F.K * F.g;
  if (p) wg_copy_lds(F.X + i0 * p, b + F.bX, 2 * nobs * p);
  if (Ka) wg_copy_lds(F.Z + i0 * Ka, b + F.bZ, 2 * nobs * Ka);
  if (Kg) wg_copy_lds(F.Y + i0 * Kg, b + F.bY, 2 * nobs * Kg);
  if (F.w) wg_copy_lds(F.w + i0, b + F.bW, 2 * nobs);
  wg_copy_lds(F.choice + i0, b + F.bC, nobs);
}

// Run body(i0, nobs, buffer) over the chunks of the fit's observations in
// order, the next chunk's copy in flight while the current one is used.
template <typename Body>
__device__ inline void for_chunks(const SmallFit &F, double *sm, Body body) {
  const int64_t N = F.N, ch = F.ch;
  const int nch = int((N + ch - 1) / ch);
  auto nob = [&](int c) { return int(min(ch, N - int64_t(c) * ch)); };
  issue_chunk(F, 0, nob(0), sm + F.oBuf0);
  for (int c = 0; c < nch; ++c) {
    // chunk c has landed, and every wave is done with chunk c - 1, whose
    // buffer the next copy overwrites
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nch)
      issue_chunk(F, int64_t(c + 1) * ch, nob(c + 1),
                  sm + ((c + 1) & 1 ? F.oBuf1 : F.oBuf0));
    body(nob(c), sm + (c & 1 ? F.oBuf1 : F.oBuf0));
  }
  __syncthreads();
}

// One staged chunk at theta th: for each observation the utilities of
// Eq. 1 (base alternative's beta = 0) and the softmax (Eqs. 2-3).  Wave v,
// lane l takes observation slot l / seg of the wave's q = 64 / seg,
// alternative k = l % seg.  Then, into LDS:
//  HESS: U_r = P_{alt(r)} phi_r for the beta / gamma coefficients (phi:
//        the x or z value of coefficient r) [ch][nbg], Ybar = sum_k P_k y_k
//        [ch][g], and S_uv = sum_k P_k (y_k - Ybar)_u (y_k - Ybar)_v [ch]
//        [npair] (u >= v);
//  else: the residuals R_k = w (delta_{k,c} - P_k) of the gradient
//        (Eq. 9) [ch][K] and their generic sums Ra_v = sum_k R_k y_kv
//        [ch][g]; the observation's weighted log-likelihood term (Eq. 5)
//        goes to *lacc of the chosen alternative's lane.
template <bool HESS>
__device__ void chunk_eval(const SmallFit &F, const double *th, int nobs,
                           const double *b, double *sm, double *lacc) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = F.K, p = F.p, g = F.g, a = F.a, seg = F.seg;
  const int q = 64 / seg, k = lane & (seg - 1);
  const bool alt = k < K;
  const double *Xs = b + F.bX, *Zs = b + F.bZ, *Ys = b + F.bY, *Ws = b + F.bW;
  const int *Cs = reinterpret_cast<const int *>(b + F.bC);
  const double *thg = th + (K - 1) * p, *tha = thg + K * a;
  for (int j0 = wv * q; j0 < F.ch; j0 += kSmWaves * q) {
    const int j = j0 + lane / seg;
    const bool on = j < nobs && alt;
    const double *xj = Xs + j * p, *zk = Zs + (j * K + k) * a,
                 *yk = Ys + (j * K + k) * g;
    double u = 0.0;
    if (on) {
      if (k >= 1) {
        const double *bk = th + (k - 1) * p;
#pragma unroll 4
        for (int c = 0; c < p; ++c) u = fma(xj[c], bk[c], u);
      }
      for (int c = 0; c < a; ++c) u = fma(zk[c], thg[k * a + c], u);
      for (int c = 0; c < g; ++c) u = fma(yk[c], tha[c], u);
    }
    if (!alt) u = -INFINITY;
    const double m = seg_max(u, seg);
    const double e = alt ? exp(u - m) : 0.0;
    const double s = seg_sum(e, seg);
    const double P = e / s;
    const bool row = j < F.ch && k == 0;   // one lane writes per observation
    if (HESS) {
      if (on) {
        double *uj = sm + F.oU + j * F.nbgp;
        if (k >= 1)
          for (int c = 0; c < p; ++c) uj[(k - 1) * p + c] = P * xj[c];
        for (int c = 0; c < a; ++c)
          uj[(K - 1) * p + k * a + c] = P * zk[c];
      }
      double yb[kSmG];
#pragma unroll
      for (int v = 0; v < kSmG; ++v) {
        if (v >= g) break;
        yb[v] = seg_sum(on ? P * yk[v] : 0.0, seg);
        if (row) sm[F.oQ + j * g + v] = yb[v];
      }
      int pi = 0;
#pragma unroll
      for (int v = 0; v < kSmG; ++v) {
        if (v >= g) break;
#pragma unroll
        for (int w2 = 0; w2 <= v; ++w2, ++pi) {
          const double t = seg_sum(
              on ? P * (yk[v] - yb[v]) * (yk[w2] - yb[w2]) : 0.0, seg);
          if (row) sm[F.oS + j * F.npair + pi] = t;
        }
      }
    } else {
      const int ci = Cs[j < F.ch ? j : 0];
      const double w = on ? Ws[j] : 0.0;
      if (on && k == ci) *lacc = fma(w, u - (m + log(s)), *lacc);
      const double r = on ? w * ((k == ci ? 1.0 : 0.0) - P) : 0.0;
      if (on) sm[F.oP + j * K + k] = r;
      for (int v = 0; v < g; ++v) {
        const double t = seg_sum(on ? r * yk[v] : 0.0, seg);
        if (row) sm[F.oQ + j * g + v] = t;
      }
    }
  }
}

// The fused pass at theta th (LDS): l into *l_out, the gradient into grad
// (LDS).  Thread t < n_p owns gradient entry t and adds each chunk's
// observations in order (beta_k,v: sum_j R_jk x_jv; gamma_k,v: sum_j R_jk
// z_jkv; alpha_v: sum_j Ra_jv); l is summed over the lanes by a fixed
// butterfly, then over the waves in wave order.
__device__ void small_pass(const SmallFit &F, const double *th, double *grad,
                           double *l_out, double *sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = F.K, p = F.p, g = F.g, a = F.a, np = F.np, Ka = K * a;
  const double *R = sm + F.oP, *Ra = sm + F.oQ;
  int kind = 3, kk = 0, off = 0;
  if (tid < (K - 1) * p) {
    kind = 0;
    kk = 1 + tid / p;
    off = tid % p;
  } else if (tid < F.nbg) {
    kind = 1;
    off = tid - (K - 1) * p;
    kk = off / a;
  } else if (tid < np) {
    kind = 2;
    off = tid - F.nbg;
  }
  double gacc = 0.0, lacc = 0.0;
  for_chunks(F, sm, [&](int nobs, const double *b) {
    chunk_eval<false>(F, th, nobs, b, sm, &lacc);
    __syncthreads();
    double t = gacc;
    if (kind == 0) {
      const double *Xs = b + F.bX + off;
#pragma unroll 8
      for (int j = 0; j < nobs; ++j) t = fma(R[j * K + kk], Xs[j * p], t);
    } else if (kind == 1) {
      const double *Zs = b + F.bZ + off;
#pragma unroll 8
      for (int j = 0; j < nobs; ++j) t = fma(R[j * K + kk], Zs[j * Ka], t);
    } else if (kind == 2) {
#pragma unroll 8
      for (int j = 0; j < nobs; ++j) t += Ra[j * g + off];
    }
    gacc = t;
  });
  double *part = sm + F.oPart;
  const double lw = seg_sum(lacc, 64);
  if (lane == 0) part[wv] = lw;
  if (tid < np) grad[tid] = gacc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int v = 0; v < kSmWaves; ++v) s += part[v];
    *l_out = s;
  }
  __syncthreads();
}

// sum of v[j]^2, j < n, in a fixed order (every thread gets it)
__device__ double small_sumsq(const double *v, int n, double *sm,
                              const SmallFit &F) {
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int j = tid; j < n; j += kSmThreads) s = fma(v[j], v[j], s);
  double *red = sm + F.oRed;
  red[tid] = s;
  __syncthreads();
  for (int h = kSmThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Offset of entry (r, c), r >= c, of a row-major packed lower triangle.
__device__ inline int tix(int r, int c) { return r * (r + 1) / 2 + c; }

// Packed lower-triangle index e -> (r, c), r >= c, row-major.
__device__ inline void tri_rc(int e, int *r, int *c) {
  int rr = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
  while (rr * (rr + 1) / 2 > e) --rr;
  *r = rr;
  *c = e - rr * (rr + 1) / 2;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// A = -H of Eq. 10 into the lower triangle of the LDS matrix.  With U_r =
// P_{alt(r)} phi_r (phi: the x or z value of coefficient r), the beta /
// gamma block is sum_i w [delta_{alt(r),alt(c)} U_r phi_c - U_r U_c]: the
// second term, U^T diag(w) U, is a dense product run on FP64 MFMA (16 x 16
// tiles of the lower triangle, four observations per k-step, one tile
// pair per wave at a time, accumulated in place in A chunk by chunk); the
// first term (pairs of one alternative), the alpha rows in the centred form
// (w U_c (y_{alt(c), v} - Ybar_v)) and the alpha-alpha block (w S_uv) are
// sums that thread t adds entry by entry (entries t, t + 256, ...).  Every
// entry's terms are added in observation order.
__device__ void small_hessian(const SmallFit &F, const double *th,
                              double *sm) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int K = F.K, p = F.p, g = F.g, a = F.a, np = F.np, nbg = F.nbg;
  const int nb = (K - 1) * p, Ka = K * a, Kg = K * g, npair = F.npair;
  const int nbp = F.nbgp;
  const int T = nbp / 16, ntp = T * (T + 1) / 2;
  // scalar entries: same-alternative pairs of alternative 0 (gamma_0),
  // then of alternatives 1 .. K-1 (beta_k then gamma_k), then alpha rows
  const int B = p + a, t0 = a * (a + 1) / 2, tb = B * (B + 1) / 2;
  const int n_same = t0 + (K - 1) * tb, n_sc = n_same + g * nbg + npair;
  const int *cfoff = reinterpret_cast<const int *>(sm + F.oFoff);
  const int *calt = reinterpret_cast<const int *>(sm + F.oAlt);
  double *Am = sm + F.oA;
  const double *U = sm + F.oU, *Yb = sm + F.oQ, *S = sm + F.oS;
  for (int e = tid; e < np * (np + 1) / 2; e += kSmThreads) Am[e] = 0.0;
  const int kb = lane >> 4, l16 = lane & 15;
  for_chunks(F, sm, [&](int nobs, const double *b) {
    chunk_eval<true>(F, th, nobs, b, sm, nullptr);
    __syncthreads();
    const double *W = b + F.bW;
    // dense part: A -= U^T diag(w) U on the lower tile pairs
    for (int tp = wv; tp < ntp; tp += kSmWaves) {
      int ti, tj;
      tri_rc(tp, &ti, &tj);
      const int rb = 16 * ti, cb = 16 * tj;
      // the lane's A-operand row and B-operand column exist (the region
      // past nbg holds the pass's residuals, not zeros)
      const bool ra = rb + l16 < nbg, ca = cb + l16 < nbg;
      d4 acc;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rb + kb + 4 * q, c = cb + l16;
        acc[q] = r < nbg && c <= r ? Am[tix(r, c)] : 0.0;
      }
      for (int j0 = 0; j0 < nobs; j0 += 4) {
        const int j = j0 + kb;
        const bool in = j < nobs;
        const double av = in && ra ? -W[j] * U[j * nbp + rb + l16] : 0.0;
        const double bv = in && ca ? U[j * nbp + cb + l16] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rb + kb + 4 * q, c = cb + l16;
        if (r < nbg && c <= r) Am[tix(r, c)] = acc[q];
      }
    }
    __syncthreads();
    for (int e = tid; e < n_sc; e += kSmThreads) {
      int r, c;
      double s;
      if (e < n_same) {
        // sum_j w U_r phi_c over a pair of one alternative
        int k, lr, lc;
        if (e < t0) {
          k = 0;
          tri_rc(e, &lr, &lc);
          r = nb + lr;
          c = nb + lc;
        } else {
          k = 1 + (e - t0) / tb;
          tri_rc((e - t0) % tb, &lr, &lc);
          r = lr < p ? (k - 1) * p + lr : nb + k * a + (lr - p);
          c = lc < p ? (k - 1) * p + lc : nb + k * a + (lc - p);
        }
        s = Am[tix(r, c)];
        const double *Ur = U + r;
        const double *ph = c < nb ? b + F.bX + cfoff[c] : b + F.bZ + cfoff[c];
        const int st = c < nb ? p : Ka;
#pragma unroll 4
        for (int j = 0; j < nobs; ++j)
          s = fma(W[j] * Ur[j * nbp], ph[j * st], s);
      } else if (e < n_same + g * nbg) {
        const int e2 = e - n_same, v = e2 / nbg;
        c = e2 - v * nbg;
        r = nbg + v;
        s = Am[tix(r, c)];
        const double *Uc = U + c;
        const double *y = b + F.bY + calt[c] * g + v, *yb = Yb + v;
#pragma unroll 4
        for (int j = 0; j < nobs; ++j)
          s = fma(W[j] * Uc[j * nbp], y[j * Kg] - yb[j * g], s);
      } else {
        int vr, vc;
        tri_rc(e - n_same - g * nbg, &vr, &vc);
        r = nbg + vr;
        c = nbg + vc;
        s = Am[tix(r, c)];
        const double *Sp = S + vr * (vr + 1) / 2 + vc;
#pragma unroll 4
        for (int j = 0; j < nobs; ++j) s = fma(W[j], Sp[j * npair], s);
      }
      Am[tix(r, c)] = s;
    }
  });
}

// L D L^T of A (lower triangle in place: D on the diagonal, the unit
// factor's multipliers below) with the pivot floor n eps max_k A_kk, then
// the direction dl = A^{-1} g by L y = g, D z = y, L^T dl = z (one wave,
// each entry's sum in a fixed order).  Returns false on every thread when
// a pivot is not above the floor or not finite (A is then garbage).
__device__ bool small_solve(const SmallFit &F, double *sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = F.np;
  double *A = sm + F.oA, *red = sm + F.oRed;
  double m = 0.0;
  for (int j = tid; j < n; j += kSmThreads) m = fmax(m, A[tix(j, j)]);
  red[tid] = m;
  __syncthreads();
  for (int h = kSmThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double floor = double(n) * 2.220446049250313e-16 * red[0];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = A[tix(k, k)];
    if (!(d > floor) || !isfinite(d)) return false;   // uniform
    const int m2 = n - k - 1, cnt = m2 * (m2 + 1) / 2;
    const double rd = 1.0 / d;
    for (int e = tid; e < cnt; e += kSmThreads) {
      int r, c;
      tri_rc(e, &r, &c);
      const int i = k + 1 + r, j = k + 1 + c;
      A[tix(i, j)] = fma(-A[tix(i, k)] * rd, A[tix(j, k)], A[tix(i, j)]);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += kSmThreads) A[tix(i, k)] *= rd;
    __syncthreads();
  }
  const double *gv = sm + F.oG;
  double *x = sm + F.oDl;
  if (wv == 0) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = lane; j < i; j += 64) s = fma(A[tix(i, j)], x[j], s);
      s = seg_sum(s, 64);
      if (lane == 0) x[i] = gv[i] - s;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
    for (int i = lane; i < n; i += 64) x[i] /= A[tix(i, i)];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int i = n - 1; i >= 0; --i) {
      double s = 0.0;
      for (int j = i + 1 + lane; j < n; j += 64) s = fma(A[tix(j, i)], x[j], s);
      s = seg_sum(s, 64);
      if (lane == 0) x[i] -= s;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  return true;
}

// The descriptor's address, hidden from the optimiser: each phase reads the
// fields it needs (scalar loads) instead of values derived from them for
// every phase being kept live across the whole iteration loop.
__device__ inline const SmallFit &fresh(const SmallFit *p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return *reinterpret_cast<const SmallFit *>(v);
}

__global__ __launch_bounds__(kSmThreads, 3) void k_fit_small(
    const SmallFit *fits, int nfits, const SmallOpts *opts, SmallInfo *info,
    int *counter) {
  extern __shared__ double sm[];
  __shared__ int next;
  const int tid = threadIdx.x;
  for (;;) {
    // the next fit of the work list; every workgroup leaves once it is
    // exhausted
    if (tid == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int f = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (f >= nfits) return;
    const SmallFit *Fp = fits + f;
    const SmallFit &F = fresh(Fp);
    const SmallOpts o = opts[f];
    const int np = F.np;
    double *th = sm + F.oTh, *gr = sm + F.oG, *dl = sm + F.oDl,
           *tr = sm + F.oTr, *tg = sm + F.oTg;
    int *calt = reinterpret_cast<int *>(sm + F.oAlt);
    int *cfoff = reinterpret_cast<int *>(sm + F.oFoff);
    for (int j = tid; j < np; j += kSmThreads) {
      th[j] = F.theta0 ? F.theta0[j] : 0.0;
      // alternative of the coefficient and its offset in an x or z row
      if (j < (F.K - 1) * F.p) {
        calt[j] = 1 + j / F.p;
        cfoff[j] = j % F.p;
      } else if (j < F.nbg) {
        const int c = j - (F.K - 1) * F.p;
        calt[j] = c / F.a;
        cfoff[j] = c;
      }
    }
    if (!F.w)
      for (int j = tid; j < F.ch; j += kSmThreads)
        sm[F.oBuf0 + F.bW + j] = sm[F.oBuf1 + F.bW + j] = 1.0;
    __syncthreads();
    double *lv = sm + F.oRed + kSmThreads - 1;   // a pass's l
    double l = 0.0, dlast = NAN, gnorm = 0.0;
    int iters = 0, ls_iters = 0, backtracks = 0, n_hess = 0, n_pass = 1;
    int reason = MNL_STOP_NONE;
    uint64_t tk0 = wall_clock64(), tk_hess = 0, tk_chol = 0, tk_ls = 0;
    small_pass(fresh(Fp), th, gr, lv, sm);
    l = *lv;
    __syncthreads();
    gnorm = sqrt(small_sumsq(gr, np, sm, fresh(Fp)));
    const uint64_t tk_first = wall_clock64() - tk0;
    for (;;) {
      if (!isfinite(l) || !isfinite(gnorm)) {
        reason = MNL_STOP_NONFINITE;
        break;
      }
      if (gnorm <= o.gtol) {
        reason = MNL_STOP_GTOL;
        break;
      }
      if (iters >= o.maxiter) {
        reason = MNL_STOP_MAXITER;
        break;
      }
      const uint64_t tk1 = wall_clock64();
      small_hessian(fresh(Fp), th, sm);
      n_hess += 1;
      const uint64_t tk2 = wall_clock64();
      tk_hess += tk2 - tk1;
      const bool pd = small_solve(fresh(Fp), sm);
      const uint64_t tk3 = wall_clock64();
      tk_chol += tk3 - tk2;
      if (!pd) {
        reason = MNL_STOP_NOT_PD;
        break;
      }
      // halving line search from the full step: accept l_t >= l - tau
      const double tau = o.ls_tol_ulps * 2.220446049250313e-16 * fabs(l);
      double t = 1.0, lt = 0.0;
      bool ok = false;
      for (int trial = 1; trial <= o.ls_max + 1; ++trial) {
        for (int j = tid; j < np; j += kSmThreads) tr[j] = fma(t, dl[j], th[j]);
        __syncthreads();
        small_pass(fresh(Fp), tr, tg, lv, sm);
        lt = *lv;
        __syncthreads();
        n_pass += 1;
        ls_iters += 1;
        if (isfinite(lt) && lt >= l - tau) {
          backtracks += trial - 1;
          ok = true;
          break;
        }
        t *= 0.5;
      }
      tk_ls += wall_clock64() - tk3;
      if (!ok) {
        backtracks += o.ls_max;
        reason = MNL_STOP_LS_FAIL;
        break;
      }
      for (int j = tid; j < np; j += kSmThreads) {
        th[j] = tr[j];
        gr[j] = tg[j];
      }
      __syncthreads();
      iters += 1;
      dlast = lt - l;
      l = lt;
      gnorm = sqrt(small_sumsq(gr, np, sm, fresh(Fp)));
      if (fabs(dlast) < o.ftol) {
        reason = MNL_STOP_FTOL;
        break;
      }
    }
    for (int j = tid; j < np; j += kSmThreads) fresh(Fp).theta[j] = th[j];
    if (tid == 0) {
      SmallInfo r;
      r.iters = iters;
      r.ls_iters = ls_iters;
      r.ls_backtracks = backtracks;
      r.stop_reason = reason;
      r.n_hess = n_hess;
      r.n_pass = n_pass;
      r.loglik = l;
      r.grad_norm = gnorm;
      r.loglik_diff = dlast;
      r.tk_first = tk_first;
      r.tk_hess = tk_hess;
      r.tk_chol = tk_chol;
      r.tk_ls = tk_ls;
      info[f] = r;
    }
    __syncthreads();
  }
}

int pow2_at_least(int x) {
  int v = 1;
  while (v < x) v <<= 1;
  return v;
}

// LDS layout of a fit with chunks of ch observations; returns the doubles.
int small_layout(const Dims &d, int ch, SmallFit *F) {
  auto ev = [](int x) { return (x + 1) & ~1; };   // 16-byte aligned offsets
  const int K = d.K, p = d.p, g = d.g, a = d.a, np = int(d.np);
  F->K = K;
  F->p = p;
  F->g = g;
  F->a = a;
  F->np = np;
  F->nbg = (K - 1) * p + K * a;
  F->nbgp = (F->nbg + 15) / 16 * 16;
  F->npair = g * (g + 1) / 2;
  F->ch = ch;
  F->seg = pow2_at_least(K);
  int o = 0;
  F->oA = o;    o += ev(np * (np + 1) / 2);
  F->oTh = o;   o += ev(np);
  F->oG = o;    o += ev(np);
  F->oDl = o;   o += ev(np);
  F->oTr = o;   o += ev(np);
  F->oTg = o;   o += ev(np);
  F->oPart = o; o += kSmWaves;
  F->oRed = o;  o += kSmThreads;
  F->oAlt = o;  o += ev((np + 1) / 2);
  F->oFoff = o; o += ev((np + 1) / 2);
  int bo = 0;
  F->bX = bo;   bo += ev(ch * p);
  F->bZ = bo;   bo += ev(ch * K * a);
  F->bY = bo;   bo += ev(ch * K * g);
  F->bW = bo;   bo += ev(ch);
  F->bC = bo;   bo += ev((ch + 1) / 2);
  F->oBuf0 = o; o += bo;
  F->oBuf1 = o; o += bo;
  // the pass's residuals and the Hessian's U products share a region
  F->oP = F->oU = o;
  o += std::max(ev(ch * K), ch * F->nbgp);
  F->oQ = o;    o += ev(ch * g);
  F->oS = o;    o += ev(ch * F->npair);
  F->lds_doubles = o;
  return o;
}

}  // namespace

bool small_fit_shape_ok(const Dims &d) {
  if (d.K > kSmK || d.g > kSmG || d.np > kSmNP) return false;
  SmallFit F;
  return size_t(small_layout(d, kSmChMin, &F)) * 8 <= kSmLdsMax;
}

bool batch_eligible(const Dims &d, const mnl_fit_opts &o) {
  return o.prec == MNL_PREC_FP64 && o.method == MNL_METHOD_NEWTON &&
         !o.validate && small_fit_shape_ok(d) &&
         double(d.N) * double(d.np) * double(d.np) <=
             double(MNL_BATCH_MAX_WORK);
}

size_t small_fit_workspace_bytes(int nfits) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(size_t(nfits) * sizeof(SmallFit)) +
         al(size_t(nfits) * sizeof(SmallOpts)) + 256 +
         al(size_t(nfits) * sizeof(SmallInfo));
}

int small_fit_run(Ctx *c, int nfits, const mnl_problem *probs,
                  const double *const *theta0, const mnl_fit_opts *opts,
                  double *const *theta_out, mnl_fit_info *infos,
                  hipStream_t s) {
  if (nfits < 0 || (nfits > 0 && (!probs || !theta_out || !infos)))
    return set_error(c, MNL_ERR_ARG, "NULL problems, outputs or reports");
  if (nfits == 0) return MNL_OK;
  MNL_HIP(c, hipSetDevice(c->device));
  const double t_start = now_ms();
  // workgroups per CU that registers allow; a fit's chunk is the largest
  // whose layout leaves room for that many (a function of the shape alone)
  const void *kern = reinterpret_cast<const void *>(&k_fit_small);
  MNL_HIP(c, raise_lds_limit(kern, int(kSmLdsMax)));
  int occ_regs = 0;
  MNL_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_regs, kern,
                                                          kSmThreads, 0));
  const size_t lds_each = (kSmLdsMax + 256) / size_t(std::max(occ_regs, 1)) -
                          256;
  std::vector<SmallFit> h(nfits);
  std::vector<SmallOpts> ho(nfits);
  size_t lds = 0;
  for (int f = 0; f < nfits; ++f) {
    Dims d;
    MNL_TRY(check_problem(c, &probs[f], &d));
    mnl_fit_opts o;
    if (opts) o = opts[f];
    else mnl_default_opts(&o);
    MNL_TRY(check_opts(c, &o));
    if (o.prec != MNL_PREC_FP64 || o.method != MNL_METHOD_NEWTON ||
        o.validate)
      return set_error(c, MNL_ERR_UNSUPPORTED,
                       "fit %d: batched fits take FP64 Newton steps without "
                       "validation", f);
    if (!small_fit_shape_ok(d))
      return set_error(c, MNL_ERR_UNSUPPORTED,
                       "fit %d beyond the batched limits (K <= %d, n_p <= "
                       "%d, LDS layout <= %zu bytes)", f, kSmK, kSmNP,
                       kSmLdsMax);
    if (!theta_out[f])
      return set_error(c, MNL_ERR_ARG, "NULL theta_out of fit %d", f);
    SmallFit &F = h[f];
    int ch = kSmChMax;
    while (ch > kSmChMin && size_t(small_layout(d, ch, &F)) * 8 > lds_each)
      ch /= 2;
    small_layout(d, ch, &F);
    F.N = d.N;
    F.pad = 0;
    F.X = probs[f].X;
    F.Y = probs[f].Y;
    F.Z = probs[f].Z;
    F.w = probs[f].w;
    F.choice = probs[f].choice;
    F.theta0 = theta0 ? theta0[f] : nullptr;
    F.theta = theta_out[f];
    lds = std::max(lds, size_t(F.lds_doubles) * 8);
    SmallOpts &so = ho[f];
    so.gtol = o.gtol;
    so.ftol = o.ftol;
    so.ls_tol_ulps = o.ls_tol_ulps;
    so.maxiter = o.maxiter;
    so.ls_max = o.ls_max;
  }
  // work list: descriptors, options, the counter, the reports
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_opt = al(size_t(nfits) * sizeof(SmallFit));
  const size_t o_cnt = o_opt + al(size_t(nfits) * sizeof(SmallOpts));
  const size_t o_inf = o_cnt + 256;
  void *ws;
  MNL_TRY(ws_get(c, S_BATCH, small_fit_workspace_bytes(nfits), &ws));
  char *b = static_cast<char *>(ws);
  MNL_HIP(c, hipMemcpyAsync(b, h.data(), size_t(nfits) * sizeof(SmallFit),
                            hipMemcpyHostToDevice, s));
  MNL_HIP(c, hipMemcpyAsync(b + o_opt, ho.data(),
                            size_t(nfits) * sizeof(SmallOpts),
                            hipMemcpyHostToDevice, s));
  MNL_HIP(c, hipMemsetAsync(b + o_cnt, 0, sizeof(int), s));
  int per_cu = 0;
  MNL_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern,
                                                          kSmThreads, lds));
  const int grid = std::min(nfits, device_cus(c) * std::max(per_cu, 1));
  hipLaunchKernelGGL(k_fit_small, dim3(grid), dim3(kSmThreads), lds, s,
                     reinterpret_cast<const SmallFit *>(b), nfits,
                     reinterpret_cast<const SmallOpts *>(b + o_opt),
                     reinterpret_cast<SmallInfo *>(b + o_inf),
                     reinterpret_cast<int *>(b + o_cnt));
  MNL_HIP(c, hipGetLastError());
  std::vector<SmallInfo> hi(nfits);
  MNL_HIP(c, hipMemcpyAsync(hi.data(), b + o_inf,
                            size_t(nfits) * sizeof(SmallInfo),
                            hipMemcpyDeviceToHost, s));
  MNL_HIP(c, hipStreamSynchronize(s));
  const double dt = now_ms() - t_start;
  int khz = 0;   // rate of the device's constant clock
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate,
                            c->device) != hipSuccess || khz <= 0) {
    (void)hipGetLastError();
    khz = 0;
  }
  const double ms_per_tick = khz > 0 ? 1.0 / double(khz) : 0.0;
  for (int f = 0; f < nfits; ++f) {
    mnl_fit_info &I = infos[f];
    std::memset(&I, 0, sizeof I);
    I.iters = hi[f].iters;
    I.ls_iters = hi[f].ls_iters;
    I.ls_backtracks = hi[f].ls_backtracks;
    I.stop_reason = hi[f].stop_reason;
    I.n_hess = hi[f].n_hess;
    I.n_pass = hi[f].n_pass;
    I.loglik = hi[f].loglik;
    I.grad_norm = hi[f].grad_norm;
    I.loglik_diff = hi[f].loglik_diff;
    I.t_total = dt;
    I.t_loglik_grad = double(hi[f].tk_first) * ms_per_tick;
    I.t_hessian = double(hi[f].tk_hess) * ms_per_tick;
    I.t_chol = double(hi[f].tk_chol) * ms_per_tick;
    I.t_ls = double(hi[f].tk_ls) * ms_per_tick;
  }
  return MNL_OK;
}

}  // namespace mnl
