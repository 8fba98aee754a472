"""Ahead-of-time hyperbox partition and candidate selection (Sec. IV.B, VI.A).

The search region of a random binary bank is cut into a regular grid of boxes
in the uniform-density coordinates xi, so every box holds the same coordinate
volume and hence the same expected number of templates; the search step keeps
the loudest template of each box (ft_eval_binary_boxes, exact).  The divisions
per coordinate follow the resolution cells at the region's centre: boxes are
about equally many cells wide along every coordinate.

Selection (Sec. VI.A): the box maxima, sorted by critical ratio, give N_cand
follow-up candidates after N_reject of the loudest boxes are set aside.  A
signal in a selected box is detected when it beats that box's candidate, in a
rejected box never, elsewhere when it beats the last selected candidate; with
that rule the semi-analytic estimate (Sec. V) gives D^p for each N_reject, and
the N_reject with the largest D^p is chosen.
"""
from __future__ import annotations

import numpy as np

from . import mismatch, sensitivity

COORDS = ("f0", "alpha", "sdec", "ap", "omega", "phib")


def cells(region, t_sft, t_obs, vmax):
    """Resolution cells across the region along each coordinate, at its centre."""
    r = region
    mid = {c: 0.5 * (r[c + "_lo"] + r[c + "_hi"]) for c in COORDS}
    d = mismatch.resolutions(mid["f0"], mid["ap"], mid["omega"], t_sft, t_obs, vmax)
    return np.array([(r[c + "_hi"] - r[c + "_lo"]) / d[i] for i, c in enumerate(COORDS)])


def partition(region, t_sft, t_obs, vmax, o, per_box, min_boxes=1, max_boxes=1 << 26):
    """Divisions n_div[6] of a regular partition whose boxes hold about per_box of
    the bank's o N(region) templates (Eq. N_binary), with at least min_boxes boxes."""
    n_bank = o * mismatch.n_templates(region, t_sft, t_obs, vmax)
    target = min(max(float(min_boxes), n_bank / per_box), float(max_boxes))
    c = cells(region, t_sft, t_obs, vmax)

    def divs(side):
        return np.maximum(1, np.round(c / side)).astype(np.int64)

    lo, hi = -30.0, 60.0  # log of the box side in cells; the box count falls as it grows
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.prod(divs(np.exp(mid)).astype(float)) >= target:
            lo = mid
        else:
            hi = mid
    n_div = divs(np.exp(lo))
    while np.prod(n_div.astype(float)) > max_boxes:
        n_div[np.argmax(n_div)] -= 1
    return [int(x) for x in n_div]


def box_z(res):
    """Critical ratios of the box maxima of ft_eval_binary_boxes (records with
    index, z), nan for empty boxes: the z_box that thresholds() takes."""
    return np.where(res["index"] >= 0, res["z"], np.nan)


def thresholds(z_box, n_cand, n_reject):
    """Detection threshold on z per box: boxes sorted by z (descending, ties to
    the lower box), the first n_reject rejected (+inf), the next n_cand selected
    (their own z); any other box takes the last selected z (+inf when none is
    selected).  Empty boxes (z = nan) sort last and are never selected."""
    z = np.asarray(z_box, np.float64)
    key = np.where(np.isnan(z), -np.inf, z)
    order = np.lexsort((np.arange(z.size), -key))
    rejected = order[:n_reject]
    selected = order[n_reject:n_reject + n_cand]
    selected = selected[~np.isnan(z[selected])]
    last = z[selected[-1]] if selected.size else np.inf
    thr = np.full(z.size, last)
    thr[selected] = z[selected]
    thr[rejected] = np.inf
    return thr


def depth_for_selection(q, m_samples, z_box, n_cand, n_reject, p=0.95, seed=0):
    """D^p of the search with this selection: population samples fall in boxes
    uniformly (boxes hold equal xi volume), each with its box's threshold."""
    thr = thresholds(z_box, n_cand, n_reject)
    rng = np.random.default_rng(seed + 1)
    box = rng.integers(0, thr.size, np.asarray(q).shape[0])
    return sensitivity.depth_at(q, m_samples, p, thr[box], seed=seed)


def optimize_reject(q, m_samples, z_box, n_cand, rejects, p=0.95, seed=0):
    """(best n_reject, [(n_reject, D^p)]) over the candidate numbers of rejected boxes."""
    table = [(int(r), depth_for_selection(q, m_samples, z_box, n_cand, int(r), p, seed)) for r in rejects]
    best = max(table, key=lambda t: (t[1], -t[0]))
    return best[0], table
