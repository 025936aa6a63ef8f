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
constexpr int kSmK = 64, kSmNP = 128;
constexpr size_t kSmLdsMax = 160 * 1024;
constexpr size_t kSmLdsTwo = 80 * 1024;   // two workgroups per CU

// A fit of the work list with its LDS layout (offsets in doubles).
struct SmallFit {
  int64_t N;
  int K, p, g, a, np, nbg;   // nbg: beta and gamma coefficients
  int ch;                    // observations per staged chunk
  int seg;                   // lanes per observation (power of two >= K)
  int ld;                    // row stride of A
  int drow;                  // doubles per staged observation
  int oA, oTh, oG, oDl, oTr, oTg, oPart, oRed, oAlt, oFoff;
  int oRow, oW, oCh, oP, oYb, oU;
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
// sum over the lanes that share lane % seg (one per observation slot)
__device__ inline double across_segs(double v, int seg) {
  for (int o = seg; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Stage observations i0 .. i0 + nobs - 1 into LDS: row j = [x_j (p) |
// z_j (K a) | y_j (K g)], the weight and the choice.  Rows past nobs are
// left as they are (never read).
__device__ void stage_chunk(const SmallFit &F, int64_t i0, int nobs,
                            double *sm) {
  const int tid = threadIdx.x;
  const int p = F.p, Ka = F.K * F.a, Kg = F.K * F.g, dr = F.drow;
  double *row = sm + F.oRow;
  if (p)
    batched_copy<4>(nobs * p, tid, kSmThreads,
                    [&](int e) { return F.X[i0 * p + e]; },
                    [&](int e, double v) {
                      const int j = e / p;
                      row[j * dr + (e - j * p)] = v;
                    });
  if (Ka)
    batched_copy<4>(nobs * Ka, tid, kSmThreads,
                    [&](int e) { return F.Z[i0 * Ka + e]; },
                    [&](int e, double v) {
                      const int j = e / Ka;
                      row[j * dr + p + (e - j * Ka)] = v;
                    });
  if (Kg)
    batched_copy<4>(nobs * Kg, tid, kSmThreads,
                    [&](int e) { return F.Y[i0 * Kg + e]; },
                    [&](int e, double v) {
                      const int j = e / Kg;
                      row[j * dr + p + Ka + (e - j * Kg)] = v;
                    });
  int *chs = reinterpret_cast<int *>(sm + F.oCh);
  for (int j = tid; j < F.ch; j += kSmThreads) {
    sm[F.oW + j] = j < nobs ? (F.w ? F.w[i0 + j] : 1.0) : 0.0;
    chs[j] = j < nobs ? F.choice[i0 + j] : -1;
  }
}

// One staged chunk at theta th: for each observation the utilities of
// Eq. 1 (base alternative's beta = 0) and the softmax (Eqs. 2-3), then
// either (HESS) P, U_r = P_{alt(r)} phi_r for the beta / gamma coefficients
// and Ybar = sum_k P_k y_k into LDS, or the residuals R_jk = w_j (delta_{k,
// c_j} - P_jk) of the gradient (Eq. 9) into LDS and the observation's
// weighted log-likelihood term (Eq. 5) into *lacc of the chosen
// alternative's lane.  Wave v, lane l takes observation slot l / seg of
// the wave's q = 64 / seg, alternative l % seg.
template <bool HESS>
__device__ void chunk_eval(const SmallFit &F, const double *th, int nobs,
                           double *sm, double *lacc) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = F.K, p = F.p, g = F.g, a = F.a, seg = F.seg;
  const int q = 64 / seg, k = lane & (seg - 1);
  const bool alt = k < K;
  const int *chs = reinterpret_cast<const int *>(sm + F.oCh);
  const double *thg = th + (K - 1) * p, *tha = thg + K * a;
  for (int j0 = wv * q; j0 < F.ch; j0 += kSmWaves * q) {
    const int j = j0 + lane / seg;
    const bool obs = j < nobs;
    const double *rj = sm + F.oRow + j * F.drow;
    double u = 0.0;
    if (obs && alt) {
      if (k >= 1) {
        const double *bk = th + (k - 1) * p;
        for (int c = 0; c < p; ++c) u = fma(rj[c], bk[c], u);
      }
      for (int c = 0; c < a; ++c) u = fma(rj[p + k * a + c], thg[k * a + c], u);
      const double *yk = rj + p + K * a + k * g;
      for (int c = 0; c < g; ++c) u = fma(yk[c], tha[c], u);
    }
    if (!alt) u = -INFINITY;
    const double m = seg_max(u, seg);
    const double e = alt ? exp(u - m) : 0.0;
    const double s = seg_sum(e, seg);
    const double P = e / s;
    if (HESS) {
      if (j < F.ch && alt) {
        sm[F.oP + j * K + k] = P;
        double *uj = sm + F.oU + j * F.nbg;
        if (k >= 1)
          for (int c = 0; c < p; ++c) uj[(k - 1) * p + c] = P * rj[c];
        for (int c = 0; c < a; ++c)
          uj[(K - 1) * p + k * a + c] = P * rj[p + k * a + c];
      }
      for (int c = 0; c < g; ++c) {
        const double t =
            seg_sum(obs && alt ? P * rj[p + K * a + k * g + c] : 0.0, seg);
        if (j < F.ch && k == 0) sm[F.oYb + j * g + c] = t;
      }
    } else if (obs && alt) {
      const double w = sm[F.oW + j];
      const int ci = chs[j];
      if (k == ci) *lacc = fma(w, u - (m + log(s)), *lacc);
      sm[F.oP + j * K + k] = w * ((k == ci ? 1.0 : 0.0) - P);
    }
  }
}

// The fused pass at theta th (LDS): l into *l_out, the gradient into grad
// (LDS).  Thread t < n_p owns gradient entry t and adds each chunk's
// observations in order (beta_k,c: sum_j R_jk x_jc; gamma_k,c: sum_j R_jk
// z_jkc; alpha_c: sum_j sum_k R_jk y_jkc); l is summed over the lanes by a
// fixed butterfly, then over the waves in wave order.
__device__ void small_pass(const SmallFit &F, const double *th, double *grad,
                           double *l_out, double *sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = F.K, p = F.p, g = F.g, a = F.a, np = F.np, dr = F.drow;
  const double *R = sm + F.oP, *row = sm + F.oRow;
  // what entry tid of the gradient reads: R column and row offset
  int kind = 3, kk = 0, off = 0;
  if (tid < (K - 1) * p) {
    kind = 0;
    kk = 1 + tid / p;
    off = tid % p;
  } else if (tid < F.nbg) {
    kind = 1;
    const int c = tid - (K - 1) * p;
    kk = c / a;
    off = p + c;
  } else if (tid < np) {
    kind = 2;
    off = p + K * a + (tid - F.nbg);
  }
  double gacc = 0.0, lacc = 0.0;
  for (int64_t i0 = 0; i0 < F.N; i0 += F.ch) {
    const int nobs = int(F.N - i0 < F.ch ? F.N - i0 : F.ch);
    stage_chunk(F, i0, nobs, sm);
    __syncthreads();
    chunk_eval<false>(F, th, nobs, sm, &lacc);
    __syncthreads();
    if (kind < 2) {
      for (int j = 0; j < nobs; ++j)
        gacc = fma(R[j * K + kk], row[j * dr + off], gacc);
    } else if (kind == 2) {
      for (int j = 0; j < nobs; ++j) {
        double t = 0.0;
        for (int k = 0; k < K; ++k)
          t = fma(R[j * K + k], row[j * dr + off + k * g], t);
        gacc += t;
      }
    }
    __syncthreads();
  }
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

// Packed lower-triangle index e -> (r, c), r >= c, row-major.
__device__ inline void tri_rc(int e, int *r, int *c) {
  int rr = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
  while (rr * (rr + 1) / 2 > e) --rr;
  *r = rr;
  *c = e - rr * (rr + 1) / 2;
}

// A = -H of Eq. 10 into the lower triangle of the LDS matrix.  With U_r =
// P_{alt(r)} phi_r (phi: the x or z value of coefficient r) the beta /
// gamma entries are sum_i w U_r (delta phi_c - U_c) (delta: same
// alternative); the alpha rows use the centred form: sum_i w U_c
// (y_{alt(c), v} - ybar_v) and sum_i w sum_k P_k (y_k - ybar)_v
// (y_k - ybar)_u.  Thread t owns entries t, t + 256, ... and adds each
// chunk's observations in order.
__device__ void small_hessian(const SmallFit &F, const double *th,
                              double *sm) {
  const int tid = threadIdx.x;
  const int K = F.K, p = F.p, g = F.g, a = F.a, np = F.np, nbg = F.nbg;
  const int ntri = np * (np + 1) / 2, dr = F.drow, yoff = p + K * a;
  const int *calt = reinterpret_cast<const int *>(sm + F.oAlt);
  const int *cfoff = reinterpret_cast<const int *>(sm + F.oFoff);
  double *Am = sm + F.oA;
  const double *W = sm + F.oW, *U = sm + F.oU, *row = sm + F.oRow,
               *Pc = sm + F.oP, *Yb = sm + F.oYb;
  double unused = 0.0;
  for (int64_t i0 = 0; i0 < F.N; i0 += F.ch) {
    const int nobs = int(F.N - i0 < F.ch ? F.N - i0 : F.ch);
    stage_chunk(F, i0, nobs, sm);
    __syncthreads();
    chunk_eval<true>(F, th, nobs, sm, &unused);
    __syncthreads();
    for (int e = tid; e < ntri; e += kSmThreads) {
      int r, c;
      tri_rc(e, &r, &c);
      double *dst = Am + r * F.ld + c;
      double s = i0 == 0 ? 0.0 : *dst;
      if (r < nbg) {
        if (calt[r] == calt[c]) {
          const int fo = cfoff[c];
          for (int j = 0; j < nobs; ++j)
            s = fma(W[j] * U[j * nbg + r], row[j * dr + fo] - U[j * nbg + c], s);
        } else {
          for (int j = 0; j < nobs; ++j)
            s = fma(-W[j] * U[j * nbg + r], U[j * nbg + c], s);
        }
      } else if (c < nbg) {
        const int v = r - nbg, yo = yoff + calt[c] * g + v;
        for (int j = 0; j < nobs; ++j)
          s = fma(W[j] * U[j * nbg + c], row[j * dr + yo] - Yb[j * g + v], s);
      } else {
        const int vr = r - nbg, vc = c - nbg;
        for (int j = 0; j < nobs; ++j) {
          const double *yj = row + j * dr + yoff;
          const double br = Yb[j * g + vr], bc = Yb[j * g + vc];
          double t = 0.0;
          for (int kk = 0; kk < K; ++kk)
            t = fma(Pc[j * K + kk] * (yj[kk * g + vr] - br),
                    yj[kk * g + vc] - bc, t);
          s = fma(W[j], t, s);
        }
      }
      *dst = s;
    }
    __syncthreads();
  }
}

// L D L^T of A (lower triangle in place: D on the diagonal, the unit
// factor's multipliers below) with the pivot floor n eps max_k A_kk, then
// the direction dl = A^{-1} g by L y = g, D z = y, L^T dl = z (one wave,
// each entry's sum in a fixed order).  Returns false on every thread when
// a pivot is not above the floor or not finite (A is then garbage).
__device__ bool small_solve(const SmallFit &F, double *sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = F.np, LD = F.ld;
  double *A = sm + F.oA, *red = sm + F.oRed;
  double m = 0.0;
  for (int j = tid; j < n; j += kSmThreads) m = fmax(m, A[j * LD + j]);
  red[tid] = m;
  __syncthreads();
  for (int h = kSmThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double floor = double(n) * 2.220446049250313e-16 * red[0];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = A[k * LD + k];
    if (!(d > floor) || !isfinite(d)) return false;   // uniform
    const int m2 = n - k - 1, cnt = m2 * (m2 + 1) / 2;
    const double rd = 1.0 / d;
    for (int e = tid; e < cnt; e += kSmThreads) {
      int r, c;
      tri_rc(e, &r, &c);
      const int i = k + 1 + r, j = k + 1 + c;
      A[i * LD + j] = fma(-A[i * LD + k] * rd, A[j * LD + k], A[i * LD + j]);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += kSmThreads) A[i * LD + k] *= rd;
    __syncthreads();
  }
  const double *gv = sm + F.oG;
  double *x = sm + F.oDl;
  if (wv == 0) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = lane; j < i; j += 64) s = fma(A[i * LD + j], x[j], s);
      s = seg_sum(s, 64);
      if (lane == 0) x[i] = gv[i] - s;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
    for (int i = lane; i < n; i += 64) x[i] /= A[i * LD + i];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int i = n - 1; i >= 0; --i) {
      double s = 0.0;
      for (int j = i + 1 + lane; j < n; j += 64) s = fma(A[j * LD + i], x[j], s);
      s = seg_sum(s, 64);
      if (lane == 0) x[i] -= s;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(kSmThreads, 2) void k_fit_small(
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
    const SmallFit F = fits[f];
    const SmallOpts o = opts[f];
    const int np = F.np;
    double *th = sm + F.oTh, *gr = sm + F.oG, *dl = sm + F.oDl,
           *tr = sm + F.oTr, *tg = sm + F.oTg;
    int *calt = reinterpret_cast<int *>(sm + F.oAlt);
    int *cfoff = reinterpret_cast<int *>(sm + F.oFoff);
    for (int j = tid; j < np; j += kSmThreads) {
      th[j] = F.theta0 ? F.theta0[j] : 0.0;
      if (j < (F.K - 1) * F.p) {
        calt[j] = 1 + j / F.p;
        cfoff[j] = j % F.p;
      } else if (j < F.nbg) {
        const int c = j - (F.K - 1) * F.p;
        calt[j] = c / F.a;
        cfoff[j] = F.p + c;
      }
    }
    __syncthreads();
    double *lv = sm + F.oRed + kSmThreads - 1;   // a pass's l
    double l = 0.0, dlast = NAN, gnorm = 0.0;
    int iters = 0, ls_iters = 0, backtracks = 0, n_hess = 0, n_pass = 1;
    int reason = MNL_STOP_NONE;
    uint64_t tk0 = wall_clock64(), tk_hess = 0, tk_chol = 0, tk_ls = 0;
    small_pass(F, th, gr, lv, sm);
    l = *lv;
    __syncthreads();
    gnorm = sqrt(small_sumsq(gr, np, sm, F));
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
      small_hessian(F, th, sm);
      n_hess += 1;
      const uint64_t tk2 = wall_clock64();
      tk_hess += tk2 - tk1;
      const bool pd = small_solve(F, sm);
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
        small_pass(F, tr, tg, lv, sm);
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
      gnorm = sqrt(small_sumsq(gr, np, sm, F));
      if (fabs(dlast) < o.ftol) {
        reason = MNL_STOP_FTOL;
        break;
      }
    }
    for (int j = tid; j < np; j += kSmThreads) F.theta[j] = th[j];
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
  F->ch = ch;
  F->seg = pow2_at_least(K);
  F->ld = np | 1;
  F->drow = p + K * a + K * g;
  int o = 0;
  F->oA = o;    o += ev(np * F->ld);
  F->oTh = o;   o += ev(np);
  F->oG = o;    o += ev(np);
  F->oDl = o;   o += ev(np);
  F->oTr = o;   o += ev(np);
  F->oTg = o;   o += ev(np);
  F->oPart = o; o += kSmWaves;
  F->oRed = o;  o += kSmThreads;
  F->oAlt = o;  o += ev((np + 1) / 2);
  F->oFoff = o; o += ev((np + 1) / 2);
  F->oRow = o;  o += ev(ch * F->drow);
  F->oW = o;    o += ev(ch);
  F->oCh = o;   o += ev((ch + 1) / 2);
  F->oP = o;    o += ev(ch * K);
  F->oYb = o;   o += ev(ch * g);
  F->oU = o;    o += ev(ch * F->nbg);
  F->lds_doubles = o;
  return o;
}

}  // namespace

bool small_fit_shape_ok(const Dims &d) {
  if (d.K > kSmK || d.np > kSmNP) return false;
  SmallFit F;
  return size_t(small_layout(d, 16, &F)) * 8 <= kSmLdsMax;
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
    // the largest chunk that keeps two workgroups per CU, else the
    // smallest
    int ch = 64;
    while (ch > 16 && size_t(small_layout(d, ch, &F)) * 8 > kSmLdsTwo) ch /= 2;
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
  MNL_HIP(c, raise_lds_limit(reinterpret_cast<const void *>(&k_fit_small),
                             int(lds)));
  const int per_cu = lds <= kSmLdsTwo ? 2 : 1;
  const int grid = std::min(nfits, device_cus(c) * per_cu);
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
