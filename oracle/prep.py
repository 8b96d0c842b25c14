"""Integer preparation for the scan form (Sec. 2.7).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.7 arranges the subjects by observed time in decreasing order, which
makes R_1(Y_i) a prefix of that order.  Subjects with equal times form a tie
run; all of them belong to each other's risk set (y_r >= Y_i), so the risk
sum for any subject of a run is the inclusive prefix up to the run's last
position.

* ``order``    -- stable ordering by decreasing y; equal times keep
                  increasing original index.  ``order[k]`` is the original
                  index of the subject at sorted position k.
* ``run_end``  -- for each sorted position, the last position of its run.
* ``d_end``    -- at the last position of each run, the number of events in
                  the run (Cox: status != 0, Fine-Gray: status == 1); 0 at
                  every other position.
"""
import numpy as np


def order(y):
    y = np.asarray(y, dtype=np.float64)
    idx = np.arange(y.size)
    # lexsort: last key is primary -> decreasing y, then increasing index
    return np.lexsort((idx, -y)).astype(np.int64)


def run_end(y_sorted):
    y_sorted = np.asarray(y_sorted, dtype=np.float64)
    n = y_sorted.size
    out = np.empty(n, dtype=np.int64)
    last = n - 1
    for k in range(n - 1, -1, -1):
        if k < n - 1 and y_sorted[k] != y_sorted[k + 1]:
            last = k
        out[k] = last
    return out


def d_end(y_sorted, ev_sorted):
    """Events per run, stored at the run's last position."""
    ev_sorted = np.asarray(ev_sorted).astype(np.int64)
    ends = run_end(y_sorted)
    d = np.zeros(ev_sorted.size, dtype=np.int64)
    np.add.at(d, ends, ev_sorted)
    return d


def event_indicator(model, status):
    status = np.asarray(status)
    if model == "cox":
        return (status != 0).astype(np.int64)
    if model == "fg":
        return (status == 1).astype(np.int64)
    raise ValueError(model)


def csc_sorted_rows(col_ptr, rows, vals, inv_order):
    """Relabel CSC rows to sorted positions and sort each column by position.

    Returns (rows_sorted, vals_sorted) with the same ``col_ptr``."""
    col_ptr = np.asarray(col_ptr, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    pos = inv_order[rows]
    out_r = np.empty_like(pos)
    out_v = None if vals is None else np.empty(len(vals), dtype=np.float64)
    for j in range(col_ptr.size - 1):
        a, b = col_ptr[j], col_ptr[j + 1]
        o = np.argsort(pos[a:b], kind="stable")
        out_r[a:b] = pos[a:b][o]
        if vals is not None:
            out_v[a:b] = np.asarray(vals[a:b], dtype=np.float64)[o]
    return out_r, out_v
