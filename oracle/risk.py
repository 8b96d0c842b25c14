"""Plain O(N^2) risk-set definitions (no sorting, no scans).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Notation follows the paper: y_i observed time, status s_i in {0 censored,
1 event (Fine-Gray: primary event), 2 competing event}, eta_i = x_i' beta,
x_j the covariate column along which the coordinate derivatives are taken.

Cox (Sec. 2.1, eq. cox_l; risk set R_1(Y_i) = {r : y_r >= Y_i}):

    l     = sum_{i: d_i=1} [ eta_i - log S0_i ],
    S_m,i = sum_{r in R_1(Y_i)} exp(eta_r) x_rj^m            (m = 0, 1, 2)
    g'    = sum_{i: d_i=1} (x_ij - S1_i/S0_i)
    g''   = -sum_{i: d_i=1} (S2_i/S0_i - (S1_i/S0_i)^2)

g' and g'' are the first and second derivatives of l along beta_j
(Sec. 2.4); the form is eqs. cox_g/cox_h of Sec. 2.7 before the
prefix-sum substitution.  Ties are handled exactly as the risk set is
written (y_r >= Y_i includes the tied subjects, i.e. Breslow's form).
For the Cox model every non-zero status counts as an event.

Fine-Gray (Sec. 2.2, eq. fg_l): the sums run over subjects with a primary
event (s_i = 1) and each risk-set term carries the IPCW weight

    w_r(t) = I(C_r >= min(T_r, t)) G(t) / G(min(Y_r, t)),

with G the Kaplan-Meier censoring survival (``oracle.km``), over the risk
set R(Y_i) = {r : y_r >= Y_i} union {r : y_r < Y_i and eps_r != 1}.  From
the observed data, s_r != 0 means T_r = y_r <= C_r and s_r = 0 means
C_r = y_r < T_r, which decides the indicator.

All functions accept complex ``eta`` (used by the complex-step checks).
"""
import numpy as np

from .km import km_censoring, km_eval


def _as(y, status, eta, xj):
    y = np.asarray(y, dtype=np.float64)
    status = np.asarray(status).astype(np.int64)
    eta = np.asarray(eta)
    if not np.iscomplexobj(eta):
        eta = eta.astype(np.float64)
    xj = None if xj is None else np.asarray(xj, dtype=np.float64)
    return y, status, eta, xj


def _weighted_sums(weights, eta, xj):
    """S_m = sum_r weights[:, r] * exp(eta_r) * x_rj^m for m = 0, 1, 2."""
    e = np.exp(eta)
    s0 = weights @ e
    if xj is None:
        return s0, None, None
    s1 = weights @ (e * xj)
    s2 = weights @ (e * xj * xj)
    return s0, s1, s2


def cox_risk_matrix(y, idx):
    """Row k is the indicator of R_1(Y_i) = {r : y_r >= Y_i} for i = idx[k]."""
    return (y[None, :] >= y[idx][:, None]).astype(np.float64)


def cox_brute(y, status, eta, xj):
    """Cox log partial likelihood and its coordinate derivatives.

    Returns a dict with ``loglik``, ``g1`` (g'), ``g2`` (g'') and the
    per-event ratios ``G`` = S1/S0 and ``H`` = S2/S0 (event order)."""
    y, status, eta, xj = _as(y, status, eta, xj)
    ev = np.nonzero(status != 0)[0]
    M = cox_risk_matrix(y, ev)
    s0, s1, s2 = _weighted_sums(M, eta, xj)
    loglik = np.sum(eta[ev] - np.log(s0))
    G = s1 / s0
    H = s2 / s0
    g1 = np.sum(xj[ev] - G)
    g2 = -np.sum(H - G * G)
    return {"loglik": loglik, "g1": g1, "g2": g2, "G": G, "H": H,
            "S0": s0}


def cox_loglik(y, status, eta):
    y, status, eta, _ = _as(y, status, eta, None)
    ev = np.nonzero(status != 0)[0]
    s0, _, _ = _weighted_sums(cox_risk_matrix(y, ev), eta, None)
    return np.sum(eta[ev] - np.log(s0))


def fg_weight_matrix(y, status, idx, times=None, values=None):
    """Row k holds w_r(Y_i) for r in R(Y_i) and 0 outside it, i = idx[k].

    (Sec. 2.2: risk set R(Y_i) and the IPCW weight w_r(t).)"""
    if times is None:
        times, values = km_censoring(y, status)
    t = y[idx][:, None]                       # evaluation time Y_i
    yr = y[None, :]
    sr = status[None, :]
    in_risk = (yr >= t) | ((yr < t) & (sr != 1))
    # I(C_r >= min(T_r, t)) from the observed data
    ind = (sr != 0) | (yr >= t)
    keep = in_risk & ind
    G_t = km_eval(times, values, np.broadcast_to(t, keep.shape))
    G_m = km_eval(times, values, np.minimum(np.broadcast_to(yr, keep.shape),
                                            np.broadcast_to(t, keep.shape)))
    W = np.zeros(keep.shape, dtype=np.float64)
    W[keep] = G_t[keep] / G_m[keep]
    return W


def fg_brute(y, status, eta, xj):
    """Fine-Gray log pseudo-likelihood and its coordinate derivatives."""
    y, status, eta, xj = _as(y, status, eta, xj)
    ev = np.nonzero(status == 1)[0]
    W = fg_weight_matrix(y, status, ev)
    s0, s1, s2 = _weighted_sums(W, eta, xj)
    loglik = np.sum(eta[ev] - np.log(s0))
    G = s1 / s0
    H = s2 / s0
    g1 = np.sum(xj[ev] - G)
    g2 = -np.sum(H - G * G)
    return {"loglik": loglik, "g1": g1, "g2": g2, "G": G, "H": H,
            "S0": s0}


def fg_loglik(y, status, eta):
    y, status, eta, _ = _as(y, status, eta, None)
    ev = np.nonzero(status == 1)[0]
    s0, _, _ = _weighted_sums(fg_weight_matrix(y, status, ev), eta, None)
    return np.sum(eta[ev] - np.log(s0))


def brute(model, y, status, eta, xj):
    """Dispatch on ``model`` in {"cox", "fg"}."""
    if model == "cox":
        return cox_brute(y, status, eta, xj)
    if model == "fg":
        return fg_brute(y, status, eta, xj)
    raise ValueError(model)


def loglik(model, y, status, eta):
    if model == "cox":
        return cox_loglik(y, status, eta)
    if model == "fg":
        return fg_loglik(y, status, eta)
    raise ValueError(model)
