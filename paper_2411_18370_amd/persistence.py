"""Candidate choice with a persistence requirement (Sec. VI.B): the loudest
template by the power statistic whose weighted number count (Eq.
number_count) reaches a minimum, set in units of the number count's noise
standard deviation above its noise mean (3 in the paper).

The library's toplist is the exact top-k by power, and it gives each entry's
exact number count and number-count critical ratio; the loudest template that
passes is therefore the first passing entry.  When no entry of the top k passes,
the answer lies deeper than the toplist (None: evaluate again with a larger k).
"""
from __future__ import annotations

from . import fasttracks as ft


def loudest_persistent(ctx: ft.Context, sub: int, k: int, n_sigma: float = 3.0):
    """(candidate, nc, z_nc) of sub-band `sub` after an evaluation with the power
    statistic, or None when none of its top-k passes z_nc >= n_sigma."""
    tops = ctx.toplist(sub, k)
    nc, z = ctx.toplist_number_count(sub, k)
    for cand, n, zz in zip(tops, nc, z):
        if zz >= n_sigma:
            return cand, float(n), float(zz)
    return None
