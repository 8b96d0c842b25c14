"""Kaplan-Meier estimate of the censoring survival function G(t) = Pr(C > t).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The Fine-Gray IPCW weights (Sec. 2.2, the weight definition right after
eq. fg_l) use the Kaplan-Meier estimate of G(t) = Pr(C > t), the survival
function of the censoring time.  The roles of "event" and "censored" are
swapped: a censored observation (status 0) is a censoring "event", every
observed failure (status 1 or 2) is a "censored" observation for C.

Reading taken where the paper is silent: the product-limit estimator

    G(t) = prod over distinct censoring times c <= t of (1 - m_c / n_c),

with m_c the number of censored subjects whose observed time equals c and
n_c = #{r : y_r >= c} the number still under observation at c.  G is
right-continuous (a censoring at c is already counted in G(c)), matching
the definition Pr(C > t).
"""
import numpy as np


def km_censoring(y, status):
    """Return ``(times, values)``: the distinct censoring times in increasing
    order and G evaluated at each of them (right-continuous step function)."""
    y = np.asarray(y, dtype=np.float64)
    status = np.asarray(status)
    cens_times = y[status == 0]
    times, m = np.unique(cens_times, return_counts=True)
    y_sorted = np.sort(y)
    # n_c = #{r : y_r >= c}
    n = y_sorted.size - np.searchsorted(y_sorted, times, side="left")
    values = np.empty(times.size, dtype=np.float64)
    g = 1.0
    for k in range(times.size):
        g = g * (1.0 - m[k] / n[k])
        values[k] = g
    return times, values


def km_eval(times, values, t):
    """G(t) for each t: the product over censoring times c <= t (1 if none)."""
    t = np.asarray(t, dtype=np.float64)
    k = np.searchsorted(times, t, side="right")  # number of censoring times <= t
    out = np.ones(t.shape, dtype=np.float64)
    has = k > 0
    out[has] = values[k[has] - 1]
    return out
