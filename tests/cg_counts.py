"""Iteration-count agreement between two CG runs of the same system.

In floating point, CG's iteration count depends on the rounding of its inner
products and updates: the search directions lose conjugacy at a rate set by
those roundings, and a run that sums in another order (the GPU's block and
lane trees against the oracle's sequential sums, or a different kernel shape)
can reach the stopping test a few iterations earlier or later on an
ill-conditioned system.  Counts are therefore compared with a small slack;
the solutions themselves are compared at the stated tolerances.
"""


def iters_close(a, b):
    """|a - b| <= max(2, 2% of the larger count)."""
    return abs(int(a) - int(b)) <= max(2, (2 * max(int(a), int(b)) + 99) // 100)
