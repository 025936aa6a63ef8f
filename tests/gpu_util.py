"""Helpers shared by the GPU parity tests (device copies, tolerances)."""
import numpy as np


def device_problem(pr):
    import paper_1404_3177_amd as mnl
    return mnl.Problem.from_numpy(pr, device="cuda")


def theta_tensor(theta):
    import torch
    return torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float64)).cuda()


def grad_scale(pr):
    """Per-coefficient bound on sum_i |term_i| of the gradient sums (Eq. 9):
    |e_ik - P_ik| <= 1, so sum_i w_i |feature_i| bounds each component."""
    w = np.ones(pr.N) if pr.w is None else pr.w
    K, p, g, a = pr.K, pr.p, pr.g, pr.a
    sx = w @ np.abs(pr.X) if p else np.zeros(0)
    parts = [np.tile(sx, K - 1)]
    if a:
        parts.append(np.einsum("i,ika->ka", w, np.abs(pr.Z)).ravel())
    if g:
        parts.append(np.einsum("i,ikc->c", w, np.abs(pr.Y)) * 2.0)
    return np.concatenate(parts) + 1e-300


def abs_jacobian_sums(pr):
    """A_i = sum_k |dU_ik/dtheta| per observation, [N, n_p] (un-normalised
    utility of Eq. 1, theta in Eq. 8 order)."""
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    A = np.zeros((N, pr.n_params))
    if p:
        A[:, :(K - 1) * p] = np.tile(np.abs(pr.X), (1, K - 1))
    if a:
        A[:, (K - 1) * p:(K - 1) * p + K * a] = np.abs(pr.Z).reshape(N, K * a)
    if g:
        A[:, (K - 1) * p + K * a:] = np.abs(pr.Y).sum(axis=1)
    return A


def hess_scale(pr):
    """Elementwise bound on sum_i |term_i| of each Hessian entry: with
    |W_kk'| <= 1, |H_jl| terms sum to at most sum_i w_i A_ij A_il."""
    A = abs_jacobian_sums(pr)
    w = np.ones(pr.N) if pr.w is None else pr.w
    return A.T @ (w[:, None] * A) + 1e-300


# error bounds on Hessian entries relative to hess_scale:
#  fp64: rounding of length-N sums, far below 1e-12 at these sizes;
#  fp32: operands rounded to 2^-24, FP32 accumulation of split chunks;
#  bf16: each operand rounded to 2^-9, so every product is within 2^-8
#        relative, plus FP32 accumulation.
HESS_TOL = {"fp64": 1e-12, "fp32": 5e-5, "bf16": 2.0 ** -7}
