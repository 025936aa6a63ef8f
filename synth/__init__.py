"""Seeded synthetic multinomial-logit problems.

This package only draws random data.  It simulates the data-generating
process of the random-utility model (Sec. 2.2: each individual picks the
alternative of highest utility, the unobserved part being i.i.d. Gumbel) and
contains none of the estimation method's arithmetic (no probabilities, no
likelihood, no derivatives).  Both the CPU oracle and the GPU path read their
inputs from here; neither imports the other.
"""
from .gen import (  # noqa: F401
    Problem,
    CONFIGS,
    make_problem,
    make_config,
    serving_request_shapes,
    serving_request,
    serving_arrivals,
    ServingStream,
)
