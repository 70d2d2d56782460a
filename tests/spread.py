"""Iteration-count checks against the rounding-only spread of the oracle.

With two FGS sweeps the Gram systems are solved only roughly, and the outer
iteration count to a tolerance depends on rounding: the oracle's own runs
with every Gram entry moved by one unit in the last place (seeded random
directions) give, on the 2D Poisson 64^2 system with s = 4, counts from 291
to 483 at 1e-8 and from 438 to 632 at 1e-12 (60 runs each).  The device
rounds differently everywhere (sums of n terms in another order), so its
count is one more draw from that kind of distribution: it must lie within
four standard deviations of the perturbed oracle runs' mean (at least two
iterations plus 2 %, for systems whose runs all agree).
"""
import numpy as np

import oracle


def perturbed_counts(A, b, *, s, sweeps, interval, tol, runs, **kw):
    """Outer-iteration counts of the oracle, unperturbed (seed 0) and with
    one-ulp Gram perturbations (seeds 1..runs-1)."""
    counts = []
    for seed in range(runs):
        _, r = oracle.sspcg(A, b, s=s, sweeps=sweeps, interval=interval, tol=tol,
                            perturb_seed=seed, **kw)
        assert r["status"] == oracle.OK
        counts.append(r["iters"])
    return np.array(counts)


def within_spread(count: int, counts) -> bool:
    counts = np.asarray(counts, dtype=float)
    m, sd = counts.mean(), counts.std()
    return abs(count - m) <= max(4.0 * sd, 2.0 + 0.02 * m)
