"""Cross-validation replicates (Sec. 2.8).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

k-fold cross-validation splits the subjects into k partitions; for each
partition the model is fitted by cyclic coordinate descent on the other
k - 1 partitions, and the fit is scored by the predictive log-likelihood of
the held-out partition.  Repeating the split r times gives k r replicates
(Sec. 3.3 uses 10 x 10).  A replicate is given here as a training mask over
the subjects (1 = training).

The definitions are taken literally on subsets:
  * the fit of a replicate is CCD (Secs. 2.3-2.4, one coordinate after the
    other in column order, the order of the workflow of Sec. 2.7's figure)
    on the data set made of its training subjects alone -- their risk sets,
    their event counts and, for Fine-Gray, the Kaplan-Meier estimate of the
    censoring distribution from the training subjects;
  * the held-out score is the log partial (Cox) or pseudo- (Fine-Gray)
    likelihood of the held-out subjects as a data set of their own, at the
    linear predictor X beta of the fitted beta (reading: the paper names the
    predictive log-likelihood of the partition without writing it out; this
    is the plain log-likelihood of that partition).
Nothing here computes a risk-set sum itself: the coordinate values come from
``oracle.scan`` and the likelihood from ``oracle.adjoint.loglik_eta``.
"""
import numpy as np

from . import ccd, scan
from .adjoint import loglik_eta


def subset(y, status, col_ptr, rows, vals, keep):
    """The data set of the subjects with keep != 0, renumbered in their
    original relative order; the CSC columns are restricted to them."""
    keep = np.asarray(keep) != 0
    idx = np.nonzero(keep)[0]
    new = np.full(keep.size, -1, dtype=np.int64)
    new[idx] = np.arange(idx.size)
    col_ptr = np.asarray(col_ptr, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    p = col_ptr.size - 1
    cp = np.zeros(p + 1, dtype=np.int64)
    rr, vv = [], []
    for j in range(p):
        r = rows[col_ptr[j]:col_ptr[j + 1]]
        m = keep[r]
        rr.append(new[r[m]])
        if vals is not None:
            vv.append(np.asarray(vals)[col_ptr[j]:col_ptr[j + 1]][m])
        cp[j + 1] = cp[j] + int(m.sum())
    rows_s = np.concatenate(rr) if rr else np.zeros(0, np.int64)
    vals_s = None if vals is None else (np.concatenate(vv) if vv else np.zeros(0))
    return (np.asarray(y, dtype=np.float64)[idx], np.asarray(status)[idx], cp, rows_s,
            vals_s, idx)


def column(n, col_ptr, rows, vals, j):
    """Column j as a dense vector of length n."""
    x = np.zeros(n)
    lo, hi = int(col_ptr[j]), int(col_ptr[j + 1])
    x[np.asarray(rows[lo:hi], dtype=np.int64)] = 1.0 if vals is None else vals[lo:hi]
    return x


def ccd_sweeps(model, y, status, col_ptr, rows, vals, eta, penalty, lam, sweeps,
               beta=None, delta=None):
    """`sweeps` cyclic passes over the coordinates from the state
    (eta = X beta, beta, trust widths delta).  Returns beta, delta, eta and
    per coordinate visit (g', g'', scale of g', scale of g'')."""
    n = np.asarray(y).size
    p = np.asarray(col_ptr).size - 1
    pr = scan.Prepared(model, y, status)
    eta = np.array(eta, dtype=np.float64)
    beta = np.zeros(p) if beta is None else np.array(beta, dtype=np.float64)
    delta = np.ones(p) if delta is None else np.array(delta, dtype=np.float64)
    hist = []
    for _ in range(sweeps):
        for j in range(p):
            x = column(n, col_ptr, rows, vals, j)
            r = pr.coordinate(eta, x)
            beta[j], delta[j], step = ccd.update(r["g1"], r["g2"], beta[j], delta[j],
                                                 penalty, lam)
            eta = eta + step * x
            hist.append((r["g1"], r["g2"], r["scale_g1"], r["scale_g2"]))
    return beta, delta, eta, hist


def fit_replicate(model, y, status, col_ptr, rows, vals, train, penalty, lam, sweeps):
    """CCD on the training subjects of one replicate, from beta = 0.
    Returns beta, delta, the linear predictor X beta of EVERY subject, and
    the coordinate history."""
    ys, ss, cp, rr, vv, idx = subset(y, status, col_ptr, rows, vals, train)
    beta, delta, _, hist = ccd_sweeps(model, ys, ss, cp, rr, vv, np.zeros(ys.size),
                                      penalty, lam, sweeps)
    n = np.asarray(y).size
    eta_all = np.zeros(n)
    for j in range(beta.size):
        if beta[j] != 0.0:
            eta_all += beta[j] * column(n, col_ptr, rows, vals, j)
    return beta, delta, eta_all, hist


def heldout_loglik(model, y, status, eta, train):
    """Predictive log-likelihood of the held-out subjects (train == 0) at
    the per-subject linear predictor eta."""
    ho = np.asarray(train) == 0
    if not np.any(ho):
        return 0.0
    return loglik_eta(model, np.asarray(y)[ho], np.asarray(status)[ho],
                      np.asarray(eta)[ho])


def training_loglik(model, y, status, eta, train):
    """Log-likelihood of the training subjects alone at eta."""
    tr = np.asarray(train) != 0
    if not np.any(tr):
        return 0.0
    return loglik_eta(model, np.asarray(y)[tr], np.asarray(status)[tr],
                      np.asarray(eta)[tr])


def path(model, y, status, col_ptr, rows, vals, train, penalty, gammas, sweeps):
    """A replicate along a path of penalty strengths: CCD on the training
    subjects, warm-started from the previous strength (beta, trust widths,
    eta carried over), `sweeps` sweeps per strength; after each, the
    held-out log-likelihood at the fitted beta.  Returns one value per
    strength."""
    ys, ss_, cp, rr, vv, idx = subset(y, status, col_ptr, rows, vals, train)
    n = np.asarray(y).size
    p = np.asarray(col_ptr).size - 1
    beta = np.zeros(p)
    delta = np.ones(p)
    eta = np.zeros(ys.size)
    out = []
    for g in gammas:
        beta, delta, eta, _ = ccd_sweeps(model, ys, ss_, cp, rr, vv, eta, penalty, g, sweeps,
                                         beta, delta)
        eta_all = np.zeros(n)
        for j in range(p):
            if beta[j] != 0.0:
                eta_all += beta[j] * column(n, col_ptr, rows, vals, j)
        out.append(heldout_loglik(model, y, status, eta_all, train))
    return np.array(out)
