"""GPU parity bars, and a record of each case's margin.

Fixed bars (relative L2): 1e-12 for FP64 results and 1e-5 for FP32 results,
both against the FP64 oracle.

Trajectory bar.  BiCGStab and CG amplify rounding, so after k iterations two
correct implementations that round differently agree only to about the
oracle's own sensitivity s: the relative change of its k-th iterate when b
(and x0) are perturbed by one ulp, 2u with u = 2^-53.  The GPU's iterates
differ from the oracle's by rounding injected at every operator application:

  * the face coefficients: the harmonic mean's reciprocal takes one Newton
    step from the hardware estimate, measured accurate to 2^-48.7 = 20 u
    (the oracle divides, correctly rounded);
  * the 7-term operator sum in another order: up to 7 u;
  * the staged updates (p', s) as fused multiply-adds: up to 3 u.

That is about 30 u = 15 times the one-ulp perturbation per application.
Errors injected at different applications are independent, so they add like
a random walk: over m applications the expected drift is 15 sqrt(m) s.  The
bar is therefore max(floor, 15 sqrt(m) s) with m = 2k for BiCGStab and
m = k (+1 for w0 = A r0) for CG with one reduction.  At k = 20 BiCGStab
iterations that is 95 s.

Every check prints one line, and appends it to the file named by the
PARITY_BAR_LOG environment variable when set:
  label  observed  bound  observed/bound  [observed/s]
"""
from __future__ import annotations

import math
import os

import numpy as np

from tests.oracle_helpers import rel_l2

FP64_TOL = 1e-12
FP32_TOL = 1e-5
ULP_FACTOR = 15.0      # rounding per operator application, in one-ulp units (see above)


def trajectory_factor(applications: int) -> float:
    return ULP_FACTOR * math.sqrt(max(int(applications), 1))


def trajectory_bound(sens: float, applications: int, floor: float = FP64_TOL) -> float:
    return max(floor, trajectory_factor(applications) * sens)


def sensitivity(run, b, x0, eps: float = 2.0 ** -52, seeds=(0, 1), perturb_x0: bool = True):
    """max over seeds of ||run(b', x0') - run(b, x0)|| / ||run(b, x0)|| for
    one-ulp relative perturbations of b (and of x0) in random directions;
    run(b, x0) returns the oracle's k-th iterate."""
    ref = run(b, x0)
    worst = 0.0
    for sd in seeds:
        xi = np.random.default_rng(sd).choice([-1.0, 1.0], size=np.shape(b))
        worst = max(worst, rel_l2(run(b * (1 + eps * xi), x0), ref))
        if perturb_x0 and np.any(x0):
            worst = max(worst, rel_l2(run(b, x0 * (1 + eps * xi)), ref))
    return worst


def check(label: str, observed: float, bound: float, sens: float | None = None) -> None:
    ratio = observed / bound if bound > 0 else math.inf
    line = f"{label}  observed {observed:.3e}  bound {bound:.3e}  ratio {ratio:.3f}"
    if sens:
        line += f"  observed/s {observed / sens:.2f}"
    print(line, flush=True)
    path = os.environ.get("PARITY_BAR_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")
    assert observed <= bound, line
