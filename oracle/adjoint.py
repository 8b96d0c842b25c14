"""The full gradient of the log (pseudo-)likelihood with respect to eta.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

With l = sum_{i event} [eta_i - log S0_i] and S0_i = sum_r W_ir exp(eta_r)
(Sec. 2.1 eq. cox_l with W the risk-set indicator; Sec. 2.2 eq. fg_l with W
the IPCW weights of the Fine-Gray risk set), the chain rule gives

    dl/deta_m = 1{m event} - exp(eta_m) sum_{i event} W_im / S0_i ,

which for Cox is the vector delta - P delta of Sec. 2.9 (P built from
I(y_m >= y_i) exp(eta_m) / S0_i); X' of it is the gradient in beta that a
proximal-gradient step needs, and Sec. 2.9 notes that the prefix-sum form
of Sec. 2.7 brings it to O(N).

``eta_gradient_brute`` evaluates the chain-rule form from the O(N^2) weight
matrices of ``oracle.risk``.  ``eta_gradient_scan`` is the O(N) form with
the subjects by decreasing time: for Cox, W_im = 1{y_m >= Y_i}, so the inner
sum runs over the events whose tie run ends at or after m's position -- a
suffix sum of d_k / S0_k over run ends k.  For Fine-Gray a subject m with a
competing event also belongs, with weight G(Y_i) / G(y_m), to the risk sets
of the events at later times Y_i > y_m, i.e. of the run ends before m's run
in this order -- a prefix sum of d_k G(Y_k) / S0_k.  Breslow ties, as
everywhere in this oracle.
"""
import numpy as np

from .km import km_censoring, km_eval
from .prep import d_end, event_indicator, order
from .risk import _as, cox_risk_matrix, fg_weight_matrix


def eta_gradient_brute(model, y, status, eta):
    """dl/deta (subject order) from the definition; complex eta allowed."""
    y, status, eta, _ = _as(y, status, eta, None)
    if model == "cox":
        ev = np.nonzero(status != 0)[0]
        W = cox_risk_matrix(y, ev)
    elif model == "fg":
        ev = np.nonzero(status == 1)[0]
        W = fg_weight_matrix(y, status, ev)
    else:
        raise ValueError(model)
    e = np.exp(eta)
    s0 = W @ e
    grad = -e * (W.T @ (1.0 / s0))
    grad[ev] += 1.0
    return grad


def loglik_eta(model, y, status, eta):
    """l(eta) = sum_{i event} [eta_i - log S0_i] in the O(N) scan form
    (inclusive prefix at each run end times the run's event count)."""
    y = np.asarray(y, dtype=np.float64)
    status = np.asarray(status).astype(np.int64)
    eta = np.asarray(eta, dtype=np.float64)
    s0, d, _, _, o = _scan_parts(model, y, status, eta)
    ev = event_indicator(model, status)
    at = d > 0
    return float(np.sum(eta[ev == 1]) - np.sum(d[at] * np.log(s0[at])))


def _scan_parts(model, y, status, eta):
    o = order(y)
    ys = y[o]
    st = status[o]
    e = np.exp(eta[o])
    ev = event_indicator(model, status)[o]
    d = d_end(ys, ev).astype(np.float64)
    p0 = np.cumsum(e)                        # inclusive prefix of e
    if model == "cox":
        return p0, d, None, None, o
    times, values = km_censoring(y, status)
    g = km_eval(times, values, ys)           # G(y) at every position
    w = np.divide(1.0, g, out=np.zeros_like(g), where=(st == 2))  # competing events
    pw = np.cumsum(e * w)
    # S0 at a run end k: prefix up to k plus G(Y_k) times the weighted
    # sum over the subjects after k's run (competing events only)
    s0 = p0 + g * (pw[-1] - pw)
    return s0, d, g, w, o


def eta_gradient_scan(model, y, status, eta):
    """dl/deta (subject order) by the prefix/suffix sums described above."""
    y = np.asarray(y, dtype=np.float64)
    status = np.asarray(status).astype(np.int64)
    eta = np.asarray(eta, dtype=np.float64)
    s0, d, g, w, o = _scan_parts(model, y, status, eta)
    n = y.size
    q = np.zeros(n)
    at = d > 0
    q[at] = d[at] / s0[at]
    # suffix sums: for position m, the run ends at or after m (q is zero
    # elsewhere, so the suffix from m equals the suffix from m's run end)
    r = np.cumsum(q[::-1])[::-1]
    e = np.exp(eta[o])
    ev = event_indicator(model, status)[o].astype(np.float64)
    grad_sorted = ev - e * r
    if model == "fg":
        q2 = np.zeros(n)
        q2[at] = d[at] * g[at] / s0[at]
        before = np.concatenate(([0.0], np.cumsum(q2)[:-1]))  # run ends before m
        grad_sorted -= e * w * before
    grad = np.empty(n)
    grad[o] = grad_sorted
    return grad
