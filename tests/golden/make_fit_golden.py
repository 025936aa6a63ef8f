"""Write oracle fit trajectories for the workload configurations.

Calls only the FP64 CPU oracle and the seeded generator.  Output:
tests/golden/fit_<name>.npz with the fitted theta, log-likelihood,
gradient norm, stop reason, iteration and line-search counts, and the
per-iteration thetas / log-likelihoods / gradient norms.

    python tests/golden/make_fit_golden.py c1 c2 [--maxiter N]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--maxiter", type=int, default=50)
    args = ap.parse_args()
    for name in args.names:
        t0 = time.time()
        pr = synth.make_config(name)
        res = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0,
                                                  maxiter=args.maxiter),
                            record=True)
        hist_theta = np.array([h["theta"] for h in res.history])
        np.savez(os.path.join(HERE, f"fit_{name}.npz"),
                 theta=res.theta, loglik=res.loglik, grad_norm=res.grad_norm,
                 stop_reason=res.stop_reason, iters=res.iters,
                 ls_iters=res.ls_iters, gtol=GTOL,
                 hist_theta=hist_theta,
                 hist_loglik=np.array([h["loglik"] for h in res.history]),
                 hist_grad_norm=np.array([h["grad_norm"] for h in res.history]),
                 hist_trials=np.array([h["trials"] for h in res.history]))
        print(f"{name}: iters={res.iters} ls={res.ls_iters} "
              f"stop={res.stop_reason} |g|={res.grad_norm:.3e} "
              f"l={res.loglik:.6f} ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main()
