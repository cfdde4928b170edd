"""CPU oracle for the lambda-leveling loop and the lambda-skeleton, and (in
``oracle.deriche``) for the gradient front-end (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls it, and the two share no
code: the oracle computes every connectivity number by flood fill over the
8-ring (``thin_oracle.c``), the product from its own tables.
"""
from .oracle import (  # noqa: F401
    ADJ_8_4,
    ADJ_4_8,
    OP_LEVELING,
    OP_SKELETON,
    OracleError,
    build,
    classify,
    classify_patch,
    count_destructible,
    count_lowerable,
    queue,
    ring_offsets,
    sweep,
    sweep_dirty,
    sweep_ordered,
)
