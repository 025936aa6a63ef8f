"""FP64 CPU oracle of the Newton-Raphson multinomial-logit fit.

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the GPU library.
"""
from . import mnl_ref  # noqa: F401
