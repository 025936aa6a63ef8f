"""Hypothesis tests of fitted models (Sec. 2.4: lrtest, waldtest,
scoretest, hmftest).

Each statistic is a likelihood difference (mnl_lrtest) or a quadratic form
that the library evaluates on the device (mnl_covariance, mnl_quadform);
p-values come from the library's chi-square tail (mnl_chi2_sf).  This
module only selects coefficients and data subsets.
"""
from __future__ import annotations

from . import Context, Problem, chi2_sf, lr_stat


def lrtest(loglik_full: float, loglik_restricted: float, df: int):
    """Likelihood-ratio test: (2 (l_full - l_restricted), df, p)."""
    stat, p = lr_stat(loglik_full, loglik_restricted, df)
    return stat, df, p


def waldtest(ctx: Context, prob: Problem, theta, idx):
    """Wald test of theta[idx] = 0 at the fitted theta:
    theta_S^T V_SS^{-1} theta_S with V = (-H)^{-1}."""
    import torch
    sel = torch.as_tensor(list(idx), dtype=torch.long, device=theta.device)
    V = ctx.covariance(prob, theta, list(idx))
    stat = ctx.quadform(V, theta.index_select(0, sel))
    return stat, len(sel), chi2_sf(stat, len(sel))


def scoretest(ctx: Context, prob: Problem, theta_restricted, df: int):
    """Rao score test: g^T (-H)^{-1} g of the full model at the restricted
    estimate (restricted coefficients set to zero in theta_restricted)."""
    _, g, _ = ctx.loglik_grad(prob, theta_restricted)
    H = ctx.hessian(prob, theta_restricted)
    stat = ctx.quadform(H, g, hessian_sign=True)
    return stat, df, chi2_sf(stat, df)


def subset_problem(prob: Problem, alts):
    """The data restricted to the alternatives `alts` (alts[0] must be the
    base alternative 0): observations choosing another alternative are
    dropped, alternatives are renumbered in the order given."""
    import torch
    alts = [int(k) for k in alts]
    if not alts or alts[0] != 0 or len(set(alts)) != len(alts) or \
            min(alts) < 0 or max(alts) >= prob.K:
        raise ValueError("alts must start with 0 and list distinct "
                         "alternatives")
    X, Y, Z, choice, w = prob._refs
    dev = X.device
    lut = torch.full((prob.K,), -1, dtype=torch.int32, device=dev)
    lut[torch.as_tensor(alts, device=dev)] = torch.arange(
        len(alts), dtype=torch.int32, device=dev)
    newc = lut[choice.long()]
    rows = torch.nonzero(newc >= 0).flatten()
    ka = torch.as_tensor(alts, dtype=torch.long, device=dev)

    def take(t):
        return t.index_select(0, rows).index_select(1, ka).contiguous()
    return Problem(X.index_select(0, rows).contiguous(), take(Y), take(Z),
                   newc.index_select(0, rows).contiguous(),
                   None if w is None else w.index_select(0, rows).contiguous())


def common_coefficients(K: int, p: int, g: int, a: int, alts):
    """Indices in the full model's theta (Eq. 8 order) of each coefficient
    of the model on the alternatives `alts`, in that model's order."""
    idx = []
    for j in alts[1:]:
        idx += [(j - 1) * p + c for c in range(p)]
    off = (K - 1) * p
    for j in alts:
        idx += [off + j * a + c for c in range(a)]
    off += K * a
    idx += [off + c for c in range(g)]
    return idx


def hmftest(ctx: Context, prob: Problem, theta_full, alts, **fit_opts):
    """Hausman-McFadden test of IIA: refit on the alternatives `alts`
    (alts[0] = 0) and compare the common coefficients,
    d^T (V_sub - V_full)^{-1} d with d = theta_sub - theta_full.
    Returns (stat, df, p, theta_sub, fit info of the subset fit)."""
    import torch
    sub = subset_problem(prob, alts)
    theta_sub, info = ctx.fit(sub, **fit_opts)
    idx = common_coefficients(prob.K, prob.p, prob.g, prob.a, list(alts))
    V_full = ctx.covariance(prob, theta_full, idx)
    V_sub = ctx.covariance(sub, theta_sub)
    sel = torch.as_tensor(idx, dtype=torch.long, device=theta_full.device)
    stat = ctx.quadform(V_sub, theta_sub, B=V_full,
                        x0=theta_full.index_select(0, sel))
    return stat, len(idx), chi2_sf(stat, len(idx)), theta_sub, info
