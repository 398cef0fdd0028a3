"""FP64 CPU oracle: test infrastructure only (see ``oracle.c``).

Importable by the tests, the smoke check and the benchmark's CPU-baseline leg;
never by the product package.
"""
from .oracle import (BREAKDOWN, DIRICHLET, NOCONV, NONFINITE, OK, ZEROFLUX,  # noqa: F401
                     Oracle, SolveInfo, build, load, num_threads, set_num_threads)
