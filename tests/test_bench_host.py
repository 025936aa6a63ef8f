"""Host-side parts of bench.py: the one-GPU rule and the algorithmic work
formulas its roofline uses."""
import os
import subprocess
import sys

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_hessian_flops_count_unique_entries():
    # beta-beta kernel: (K-1)K/2 pair rows x p(p+1)/2 feature pairs; the
    # whole Hessian adds all (K-1)p x K a beta-gamma entries, the
    # gamma-gamma upper blocks and the alpha rows
    pr = synth.make_config("c2")
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    u_bb = 49 * 50 // 2 * (21 * 22 // 2)
    u_bg = 49 * 21 * 50 * 5
    u_gg = 50 * 49 // 2 * 25 + 50 * 15
    assert bench.hess_kernel_flops(pr) == 2.0 * N * u_bb
    u_alpha = (K - 1) * p * g + K * a * g + g * (g + 1) // 2
    assert bench.hess_total_flops(pr) == \
        2.0 * N * (u_bb + u_bg + u_gg + u_alpha)
    # the 400,000-individual workload: 4950 x 1326 unique beta-beta
    # entries, 5.25 TFLOP per launch
    c3 = synth.make_config("c3", N=10)
    assert bench.hess_kernel_flops(c3) == 2.0 * 10 * 4950 * 1326


def test_pass_bytes_are_the_algorithmic_traffic():
    pr = synth.make_config("c2")
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    reads = N * (p + K * g + K * a) * 8 + 4 * N
    writes = N * K * 8 + N * g * 8
    assert bench.pass_bytes(pr) == float(reads + writes)
    assert bench.predict_bytes(pr) == float(N * (p + K * g + K * a) * 8 +
                                            N * K * 8)
