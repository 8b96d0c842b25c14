"""The risk-set definitions of ``oracle.risk`` in 50-digit arithmetic.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Pure-Python loops over ``mpmath.mpf``; meant for N <= a few hundred.  The
Kaplan-Meier factors are also formed in multiprecision, so the only FP64
quantities are the inputs themselves.  Definitions: Sec. 2.1 (eq. cox_l)
and Sec. 2.2 (eq. fg_l and the IPCW weight), see ``oracle.risk``.
"""
import mpmath

DPS = 50


def _km_mp(y, status):
    """Multiprecision Kaplan-Meier censoring survival G(t), right-continuous:
    product over censoring times c <= t of (1 - m_c / #{y >= c})."""
    ctimes = sorted(set(float(y[i]) for i in range(len(y)) if status[i] == 0))
    fac = []
    for c in ctimes:
        m = sum(1 for i in range(len(y)) if status[i] == 0 and y[i] == c)
        n = sum(1 for i in range(len(y)) if y[i] >= c)
        fac.append((c, 1 - mpmath.mpf(m) / n))

    def G(t):
        g = mpmath.mpf(1)
        for c, f in fac:
            if c <= t:
                g *= f
        return g
    return G


def exact(model, y, status, eta, xj):
    """Return (loglik, g1, g2) as ``mpmath.mpf`` for model "cox" or "fg"."""
    with mpmath.workdps(DPS):
        n = len(y)
        e = [mpmath.exp(mpmath.mpf(float(v))) for v in eta]
        x = [mpmath.mpf(float(v)) for v in xj]
        if model == "fg":
            G = _km_mp(y, status)
        ll = mpmath.mpf(0)
        g1 = mpmath.mpf(0)
        g2 = mpmath.mpf(0)
        for i in range(n):
            if model == "cox" and status[i] == 0:
                continue
            if model == "fg" and status[i] != 1:
                continue
            t = y[i]
            s0 = s1 = s2 = mpmath.mpf(0)
            for r in range(n):
                if model == "cox":
                    if y[r] < t:
                        continue
                    w = mpmath.mpf(1)
                else:
                    if y[r] >= t:
                        w = mpmath.mpf(1)          # R_1, weight G(t)/G(t)
                    elif status[r] == 2:
                        w = G(t) / G(y[r])        # R_2, C_r >= T_r = y_r
                    else:
                        continue                  # not in R, or weight 0
                s0 += w * e[r]
                s1 += w * e[r] * x[r]
                s2 += w * e[r] * x[r] * x[r]
            gi = s1 / s0
            hi = s2 / s0
            ll += mpmath.mpf(float(eta[i])) - mpmath.log(s0)
            g1 += x[i] - gi
            g2 -= hi - gi * gi
        return ll, g1, g2
