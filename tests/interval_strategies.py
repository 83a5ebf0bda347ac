"""Hypothesis strategies for random exposure sets (test inputs only): each of
up to J instruments places non-overlapping exposures on a coarse time grid,
so that equal times (an end and a start, two starts, two ends) and
zero-length exposures are frequent, and the merged set of a series overlaps
at most J deep."""
import numpy as np
from hypothesis import strategies as st

GRID = 0.25


@st.composite
def exposure_series(draw, max_instruments=4, max_per_instrument=8):
    J = draw(st.integers(1, max_instruments))
    ts, te = [], []
    for _ in range(J):
        n = draw(st.integers(0, max_per_instrument))
        t = 0.0
        for _ in range(n):
            t += GRID * draw(st.integers(0, 4))          # gap (0: back to back)
            d = GRID * draw(st.integers(0, 3))           # duration (0: instantaneous)
            ts.append(t)
            te.append(t + d)
            t += d
    ts, te = np.array(ts, dtype=np.float64), np.array(te, dtype=np.float64)
    o = np.argsort(ts, kind="stable")
    return ts[o], te[o], J
