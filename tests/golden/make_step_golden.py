"""Write oracle Newton steps and trajectories at the largest workload sizes.

Calls only the FP64 CPU oracle and the seeded generator (no GPU code).
Outputs, under tests/golden/:

  step_c3.npz   400,000 observations, K = 100, p = 51, g = 5 at theta = 0:
                l, the gradient (Eq. 9) and the Newton direction of Eq. 6
                solved against the full Eq. 10 Hessian (alpha-alpha block
                included), plus the largest diagonal entry of -H.
  traj_c5.npz   50,000 observations, K = 500, p = 11, weighted, coefficient
                sd 3: the oracle fit from zero at gradient tolerance 1e-8
                (per iteration theta, l, ||g||, line-search trials; the stop
                reason and the iteration of the stop).

    python tests/golden/make_step_golden.py c3 c5 [--c5-maxiter N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import mnl_ref as R  # noqa: E402

GTOL = 1e-8


def c3():
    t0 = time.time()
    pr = synth.make_config("c3")
    th = np.zeros(pr.n_params)
    l0 = R.loglik(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    g0 = R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    print(f"c3: l, g ({time.time() - t0:.0f}s)", flush=True)
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    print(f"c3: Hessian ({time.time() - t0:.0f}s)", flush=True)
    delta = R.newton_direction(H, g0)
    np.savez(os.path.join(HERE, "step_c3.npz"), loglik=l0, grad=g0,
             delta=delta, max_diag=float(np.max(-np.diag(H))))
    print(f"c3: |g|={np.linalg.norm(g0):.6e} |delta|={np.linalg.norm(delta):.6e}"
          f" ({time.time() - t0:.0f}s)", flush=True)


def c5(maxiter):
    t0 = time.time()
    pr = synth.make_config("c5")
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0,
                                              maxiter=maxiter), record=True)
    np.savez(os.path.join(HERE, "traj_c5.npz" if maxiter >= 50 else f"traj_c5_it{maxiter}.npz"),
             stop_reason=res.stop_reason, iters=res.iters,
             ls_iters=res.ls_iters, loglik=res.loglik,
             grad_norm=res.grad_norm, maxiter=maxiter, gtol=GTOL,
             hist_theta=np.array([h["theta"] for h in res.history]),
             hist_loglik=np.array([h["loglik"] for h in res.history]),
             hist_grad_norm=np.array([h["grad_norm"] for h in res.history]),
             hist_trials=np.array([h["trials"] for h in res.history]),
             theta=res.theta)
    print(f"c5: iters={res.iters} ls={res.ls_iters} stop={res.stop_reason} "
          f"|g|={res.grad_norm:.3e} l={res.loglik:.6f} "
          f"({time.time() - t0:.0f}s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=["c3", "c5"])
    ap.add_argument("--c5-maxiter", type=int, default=50)
    args = ap.parse_args()
    for name in args.names:
        if name == "c3":
            c3()
        else:
            c5(args.c5_maxiter)


if __name__ == "__main__":
    main()
