"""Write the oracle's coefficient tables at the fitted workload optima.

Calls only the FP64 CPU oracle and the seeded generator.  Reads the fitted
theta of tests/golden/fit_<name>.npz (itself written by the oracle) and
writes tests/golden/summary_<name>.npz with the standard errors, Wald
statistics and p-values of the summary method at that theta, and the
extreme eigenvalues of -H and max |H_jl| (for error bounds).

    python tests/golden/make_summary_golden.py c1 c2
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import mnl_ref as R  # noqa: E402


def main():
    for name in sys.argv[1:]:
        t0 = time.time()
        pr = synth.make_config(name)
        theta = np.load(os.path.join(HERE, f"fit_{name}.npz"))["theta"]
        H = R.hessian(theta, pr.X, pr.Y, pr.Z, None, pr.w)
        se, z, pval = R.summary(theta, pr.X, pr.Y, pr.Z, pr.w, H=H)
        lam = np.linalg.eigvalsh(-H)
        np.savez(os.path.join(HERE, f"summary_{name}.npz"), theta=theta,
                 se=se, z=z, pval=pval, lam_min=lam[0], lam_max=lam[-1],
                 hmax=np.abs(H).max())
        print(f"{name}: n_p={theta.size} se in [{se.min():.3e}, "
              f"{se.max():.3e}] ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main()
