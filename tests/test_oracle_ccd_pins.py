"""Pins of the oracle's coordinate-descent loop, its penalty path, the
relabelling of the design to sorted positions and the penalty value.

Each one is checked against something the oracle does not compute itself:
a sweep worked by hand (which coordinate moves first, with which linear
predictor and which clipped step), the optimality (KKT) conditions of the
penalised objective at convergence with g' taken from the O(N^2) risk-set
definition, the uniqueness of the optimum (a warm-started path and a cold
start reach the same point), and hand-relabelled designs.
"""
import math

import numpy as np
import pytest

import gen
from oracle import ccd, cv, prep, risk


# ---------------------------------------------------------------- one sweep by hand

def _hand_data():
    # times 1 < 2 < 3 < 4, events at 1, 3, 4; two 0/1 columns
    y = np.array([1.0, 2.0, 3.0, 4.0])
    s = np.array([1, 0, 1, 1])
    x0 = np.array([1.0, 0.0, 1.0, 0.0])
    x1 = np.array([0.0, 1.0, 1.0, 0.0])
    cp, rows, _ = gen.csc_from_dense(np.stack([x0, x1], axis=1))
    return y, s, x0, x1, cp, rows


def test_sweep_hand_example_unpenalised():
    """Cyclic order, the linear predictor after each step, the trust region.

    Coordinate 0 at eta = 0: g' = 1, g'' = -1/2 (risk sets {all}, {3, 4},
    {4} hold 2, 1, 0 subjects with x0 = 1), Newton step 2, clipped to the
    initial width 1; the width becomes max(2 * 2, 1/2) = 4.  Coordinate 1
    then sees eta = x0 (e = E at the subjects with x0 = 1, E = exp(1)):
    at time 1 the risk set is everyone, S0 = 2E + 2, S1 = 1 + E, G = 1/2;
    at time 3 it is {3, 4}, S0 = E + 1, S1 = E; at time 4 it is {4},
    S1 = 0.  So g' = 1/(E+1) - 1/2 and g'' = -(1/4 + E/(E+1)^2), and the
    step -g'/g'' (|step| < 1) is taken whole.  Taking coordinate 1 first,
    or with a stale eta = 0, gives g' = 0 and no step; updating eta with
    the unclipped step 2 gives a different value."""
    y, s, x0, x1, cp, rows = _hand_data()
    E = math.e
    g1 = 1.0 / (E + 1.0) - 0.5
    g2 = -(0.25 + E / (E + 1.0) ** 2)
    s1 = -g1 / g2
    beta, delta, eta, hist = cv.ccd_sweeps("cox", y, s, cp, rows, None, np.zeros(4),
                                           ccd.PENALTY_NONE, 0.0, 1)
    assert hist[0][0] == pytest.approx(1.0, abs=1e-15)
    assert hist[0][1] == pytest.approx(-0.5, abs=1e-15)
    assert hist[1][0] == pytest.approx(g1, rel=1e-14)
    assert hist[1][1] == pytest.approx(g2, rel=1e-14)
    np.testing.assert_allclose(beta, [1.0, s1], rtol=1e-14)
    np.testing.assert_allclose(delta, [4.0, max(2 * abs(s1), 0.5)], rtol=1e-14)
    np.testing.assert_allclose(eta, x0 * 1.0 + x1 * s1, rtol=1e-14, atol=1e-15)


def test_sweep_hand_example_l1():
    """The same data with gamma = 1/2: coordinate 0 leaves zero since
    g' - gamma = 1/2 > 0 (step (1/2)/(1/2) = 1, width max(2, 1/2) = 2);
    coordinate 1 stays at zero since |1/(E+1) - 1/2| < 1/2."""
    y, s, x0, x1, cp, rows = _hand_data()
    beta, delta, eta, _ = cv.ccd_sweeps("cox", y, s, cp, rows, None, np.zeros(4),
                                        ccd.PENALTY_L1, 0.5, 1)
    np.testing.assert_allclose(beta, [1.0, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(delta, [2.0, 0.5], rtol=0, atol=1e-15)
    np.testing.assert_allclose(eta, x0, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- KKT at convergence

def _kkt_data(model, valued):
    """A small design with a few clear effects, so that l1 keeps some
    coefficients at zero and moves others."""
    rng = np.random.default_rng(7 if model == "cox" else 8)
    n, p = 260, 5
    if valued:
        X = rng.normal(0.0, 1.0, (n, p))
    else:
        X = (rng.random((n, p)) < 0.35).astype(np.float64)
    b_true = np.array([1.2, -0.9, 0.0, 0.0, 0.6])
    eta = X @ b_true
    T = rng.exponential(1.0, n) / np.exp(eta)
    C = rng.exponential(1.5, n)
    y = np.minimum(T, C)
    if model == "cox":
        s = (T <= C).astype(np.int64)
    else:
        kind = np.where(rng.random(n) < 0.6, 1, 2)
        s = np.where(T <= C, kind, 0).astype(np.int64)
    cp, rows, vals = gen.csc_from_dense(X)
    return y, s, X, cp, rows, (vals if valued else None)


def _converge(model, y, s, cp, rows, vals, penalty, lam, max_sweeps=600):
    n, p = y.size, cp.size - 1
    beta, delta, eta = np.zeros(p), np.ones(p), np.zeros(n)
    for k in range(max_sweeps):
        b_old = beta.copy()
        beta, delta, eta, _ = cv.ccd_sweeps(model, y, s, cp, rows, vals, eta, penalty, lam, 1,
                                            beta, delta)
        if np.max(np.abs(beta - b_old)) < 1e-14:
            return beta, eta, k + 1
    raise AssertionError("oracle CCD did not converge")


@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("valued", [False, True])
@pytest.mark.parametrize("penalty,lam", [(ccd.PENALTY_L1, 6.0), (ccd.PENALTY_L2, 0.4)])
def test_ccd_sweeps_converge_to_kkt(model, valued, penalty, lam):
    """At the fixed point of the oracle's CCD loop the optimality conditions
    of l(beta) + pi(beta) hold (Secs. 2.3-2.4), with g' and g'' from the
    O(N^2) risk-set definition at eta = X beta: l1, |g'_j| <= gamma where
    beta_j = 0 and g'_j = gamma sgn(beta_j) elsewhere; l2, g'_j = beta_j/tau.
    The eta the loop carries is X beta."""
    y, s, X, cp, rows, vals = _kkt_data(model, valued)
    beta, eta, _ = _converge(model, y, s, cp, rows, vals, penalty, lam)
    np.testing.assert_allclose(eta, X @ beta, rtol=1e-12, atol=1e-12)
    for j in range(X.shape[1]):
        r = risk.brute(model, y, s, X @ beta, X[:, j])
        g1, g2 = float(r["g1"]), float(r["g2"])
        tol = 1e-9 * (abs(g2) + 1.0)
        if penalty == ccd.PENALTY_L1:
            if beta[j] == 0.0:
                assert abs(g1) <= lam + tol, (j, g1)
            else:
                assert abs(g1 - lam * np.sign(beta[j])) <= tol, (j, g1, beta[j])
        else:
            assert abs(g1 - beta[j] / lam) <= tol, (j, g1, beta[j])
    if penalty == ccd.PENALTY_L1:
        assert np.any(beta == 0.0) and np.any(beta != 0.0), beta


# ---------------------------------------------------------------- path vs cold start

@pytest.mark.parametrize("model", ["cox", "fg"])
def test_path_equals_cold_start_at_convergence(model):
    """The penalised objective has one maximiser, so the warm-started path
    of oracle.cv.path, converged at each strength, scores the same held-out
    likelihood as a fit started from zero at that strength; its first
    strength is a cold start and agrees bit for bit."""
    y, s, X, cp, rows, vals = _kkt_data(model, False)
    train = gen.cv_folds(3, y.size, 4, 1)[1]
    gammas = [8.0, 3.0]
    sweeps = 300
    got = cv.path(model, y, s, cp, rows, vals, train, ccd.PENALTY_L1, gammas, sweeps)
    for k, g in enumerate(gammas):
        beta, _, eta_all, _ = cv.fit_replicate(model, y, s, cp, rows, vals, train,
                                               ccd.PENALTY_L1, g, sweeps)
        want = cv.heldout_loglik(model, y, s, eta_all, train)
        if k == 0:
            assert got[0] == want
        else:
            assert got[k] == pytest.approx(want, rel=1e-11, abs=1e-11)
        # the score is the held-out likelihood at X beta of all subjects
        ho = train == 0
        assert want == pytest.approx(risk.loglik(model, y[ho], s[ho], (X @ beta)[ho]),
                                     rel=1e-12)
    assert got[0] != got[1]


# ---------------------------------------------------------------- design relabelling

def test_csc_sorted_rows_hand_example():
    """Five subjects with times 2, 5, 2, 1, 5: by decreasing time (ties by
    increasing index) the order is 1, 4, 0, 2, 3, so subjects 0..4 sit at
    positions 2, 0, 3, 4, 1.  Column 0 holds subjects 0, 3, 4 (values 10,
    30, 40) -> positions 2, 4, 1 -> ascending 1, 2, 4 with values 40, 10,
    30; column 1 holds subjects 2, 1 (values 7, 8, given out of order) ->
    positions 3, 0 -> 0, 3 with values 8, 7."""
    y = np.array([2.0, 5.0, 2.0, 1.0, 5.0])
    o = prep.order(y)
    np.testing.assert_array_equal(o, [1, 4, 0, 2, 3])
    inv = np.empty_like(o)
    inv[o] = np.arange(5)
    np.testing.assert_array_equal(inv, [2, 0, 3, 4, 1])
    col_ptr = np.array([0, 3, 5])
    rows = np.array([0, 3, 4, 2, 1])
    vals = np.array([10.0, 30.0, 40.0, 7.0, 8.0])
    rs, vs = prep.csc_sorted_rows(col_ptr, rows, vals, inv)
    np.testing.assert_array_equal(rs, [1, 2, 4, 0, 3])
    np.testing.assert_array_equal(vs, [40.0, 10.0, 30.0, 8.0, 7.0])
    rs2, vs2 = prep.csc_sorted_rows(col_ptr, rows, None, inv)
    np.testing.assert_array_equal(rs2, rs)
    assert vs2 is None


# ---------------------------------------------------------------- penalty value

def test_penalty_value_hand():
    """Sec. 2.3: -gamma sum |beta_j| and -sum beta_j^2 / (2 tau)."""
    b = [1.0, -2.0, 0.0, 0.5]
    assert ccd.penalty_value(b, ccd.PENALTY_NONE, 3.0) == 0.0
    assert ccd.penalty_value(b, ccd.PENALTY_L1, 0.5) == -1.75
    assert ccd.penalty_value(b, ccd.PENALTY_L2, 2.0) == -(1 + 4 + 0.25) / 4.0
