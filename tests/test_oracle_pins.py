"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed by the paper or by
mathematics: hand-derived values on tiny data, the log-rank closed form,
50-digit arithmetic, finite differences and complex steps of the
likelihood, invariances and reductions between the two models.
"""
import math

import numpy as np
import pytest
from fractions import Fraction

from oracle import ccd, exact, km, prep, risk, scan
import gen


# ---------------------------------------------------------------- helpers

def _rand_problem(seed, n, model, ties=0, binary=False):
    rng = np.random.default_rng(seed)
    y = rng.exponential(1.0, n)
    if ties:
        y = gen.force_ties(y, ties)
    if model == "cox":
        status = (rng.random(n) < 0.6).astype(np.int64)
    else:
        u = rng.random(n)
        status = np.where(u < 0.35, 1, np.where(u < 0.65, 2, 0)).astype(np.int64)
    eta = rng.normal(0.0, 0.7, n)
    if binary:
        xj = (rng.random(n) < 0.3).astype(np.float64)
    else:
        xj = rng.normal(0.0, 1.0, n)
    return y, status, eta, xj


# ---------------------------------------------------------------- KM

def test_km_hand_example():
    # censoring times 1, 3, 5 with 6, 4, 2 subjects still observed:
    # G = 5/6, 5/6*3/4 = 5/8, 5/8*1/2 = 5/16
    y = np.array([1, 2, 3, 4, 5, 6], float)
    s = np.array([0, 1, 0, 2, 0, 1])
    t, v = km.km_censoring(y, s)
    got = km.km_eval(t, v, np.array([0.5, 1, 2, 3, 4, 5, 6, 7]))
    want = [1, 5 / 6, 5 / 6, 5 / 8, 5 / 8, 5 / 16, 5 / 16, 5 / 16]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_km_ties_and_no_censoring():
    # two censorings tied at t=2 with four subjects observed there: G(2)=1/2
    t, v = km.km_censoring(np.array([2, 2, 2, 3.0]), np.array([0, 1, 0, 2]))
    assert km.km_eval(t, v, np.array([2.0]))[0] == 0.5
    t, v = km.km_censoring(np.array([1, 2, 3.0]), np.array([1, 2, 1]))
    np.testing.assert_array_equal(km.km_eval(t, v, np.array([0, 1, 5.0])), 1.0)


# ---------------------------------------------------------------- hand examples

def test_cox_hand_example():
    # y=1,2,3,4  events at 1,3,4  x=1,0,1,0  eta=0
    # risk sums: t=1 -> S0=4,S1=2; t=3 -> S0=2,S1=1; t=4 -> S0=1,S1=0
    y = np.array([1, 2, 3, 4.0]); s = np.array([1, 0, 1, 1])
    x = np.array([1, 0, 1, 0.0]); eta = np.zeros(4)
    r = risk.cox_brute(y, s, eta, x)
    assert r["g1"] == pytest.approx(1.0, abs=1e-15)
    assert r["g2"] == pytest.approx(-0.5, abs=1e-15)
    assert r["loglik"] == pytest.approx(-3 * math.log(2), abs=1e-14)


def test_cox_hand_example_ties():
    # two events tied at t=1 share the full risk set {1,2,3}: G = 2/3 each
    y = np.array([1, 1, 2.0]); s = np.array([1, 1, 0])
    x = np.array([1, 0, 1.0]); eta = np.zeros(3)
    r = risk.cox_brute(y, s, eta, x)
    assert r["g1"] == pytest.approx(-1 / 3, abs=1e-15)
    assert r["g2"] == pytest.approx(-4 / 9, abs=1e-15)
    assert r["loglik"] == pytest.approx(-2 * math.log(3), abs=1e-14)


def test_fg_hand_example():
    # y=1,2,3,4  status 2,0,1,1  x=1,0,1,0  eta=0.  G(t)=1 for t<2, 2/3 after.
    # event at 3: R1={3,4} w=1, competing subject at 1 has w=G(3)/G(1)=2/3
    #   S0=8/3, S1=5/3, G=5/8
    # event at 4: R1={4}, competing subject at 1 w=2/3: S0=5/3, S1=2/3, G=2/5
    y = np.array([1, 2, 3, 4.0]); s = np.array([2, 0, 1, 1])
    x = np.array([1, 0, 1, 0.0]); eta = np.zeros(4)
    r = risk.fg_brute(y, s, eta, x)
    assert r["g1"] == pytest.approx(float(Fraction(3, 8) - Fraction(2, 5)),
                                    abs=1e-15)
    assert r["g2"] == pytest.approx(-759 / 1600, abs=1e-15)
    assert r["loglik"] == pytest.approx(-math.log(8 / 3) - math.log(5 / 3),
                                        abs=1e-14)


# ---------------------------------------------------------------- closed form

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cox_logrank_closed_form(seed):
    """At beta = 0 with one binary covariate and distinct times, the Cox
    score is the log-rank O - E and minus the Hessian its variance
    sum n1*n0/n^2 (counts of subjects at risk in each group)."""
    rng = np.random.default_rng(seed)
    n = 300
    y = rng.permutation(n).astype(float) + 1
    s = (rng.random(n) < 0.7).astype(int)
    x = (rng.random(n) < 0.4).astype(float)
    o_minus_e = 0.0
    var = 0.0
    for i in range(n):
        if s[i] != 1:
            continue
        at_risk = [r for r in range(n) if y[r] >= y[i]]
        n_all = len(at_risk)
        n1 = sum(1 for r in at_risk if x[r] == 1)
        n0 = n_all - n1
        o_minus_e += x[i] - n1 / n_all
        var += n1 * n0 / n_all ** 2
    r = risk.cox_brute(y, s, np.zeros(n), x)
    assert r["g1"] == pytest.approx(o_minus_e, rel=1e-12, abs=1e-12)
    assert -r["g2"] == pytest.approx(var, rel=1e-12)
    sc = scan.scan("cox", y, s, np.zeros(n), x)
    assert sc["g1"] == pytest.approx(o_minus_e, rel=1e-12, abs=1e-12)
    assert -sc["g2"] == pytest.approx(var, rel=1e-12)


# ---------------------------------------------------------------- exact arithmetic

@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,ties", [(0, 0), (1, 7), (2, 3)])
def test_brute_matches_50_digit(model, seed, ties):
    y, s, eta, x = _rand_problem(seed, 40, model, ties=ties)
    ll, g1, g2 = exact.exact(model, y, s, eta, x)
    r = risk.brute(model, y, s, eta, x)
    assert r["loglik"] == pytest.approx(float(ll), rel=1e-13)
    assert r["g1"] == pytest.approx(float(g1), rel=1e-11, abs=1e-12)
    assert r["g2"] == pytest.approx(float(g2), rel=1e-12)


# ---------------------------------------------------------------- brute vs scan

@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,n,ties", [(3, 1, 0), (4, 2, 0), (5, 57, 0),
                                          (6, 600, 0), (7, 900, 25),
                                          (8, 1500, 4), (9, 2000, 300)])
def test_scan_matches_brute(model, seed, n, ties):
    y, s, eta, x = _rand_problem(seed, n, model, ties=ties)
    r = risk.brute(model, y, s, eta, x)
    c = scan.scan(model, y, s, eta, x)
    scale_g1 = np.sum(np.abs(x[prep.event_indicator(model, s) == 1])) + \
        np.sum(np.abs(r["G"])) + 1e-300
    assert abs(c["g1"] - r["g1"]) <= 1e-12 * scale_g1
    assert c["g2"] == pytest.approx(r["g2"], rel=1e-12, abs=1e-300)
    assert c["loglik"] == pytest.approx(r["loglik"], rel=1e-12, abs=1e-300)


def test_scan_binary_covariate_with_all_censored_and_all_events():
    for model in ("cox", "fg"):
        y, _, eta, x = _rand_problem(11, 300, model, binary=True)
        for s in (np.zeros(300, int), np.ones(300, int)):
            r = risk.brute(model, y, s, eta, x)
            c = scan.scan(model, y, s, eta, x)
            assert c["g1"] == pytest.approx(r["g1"], rel=1e-12, abs=1e-12)
            assert c["g2"] == pytest.approx(r["g2"], rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------- derivatives

@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,n,ties", [(12, 200, 0), (13, 1000, 20), (14, 2000, 0)])
def test_central_fd(model, seed, n, ties):
    """g' and g'' are the derivatives of l along beta_j (Sec. 2.4):
    central differences with h = 1e-6 in FP64, relative error <= 1e-6."""
    y, s, eta, x = _rand_problem(seed, n, model, ties=ties)
    h = 1e-6
    r = risk.brute(model, y, s, eta, x)
    lp = risk.loglik(model, y, s, eta + h * x)
    lm = risk.loglik(model, y, s, eta - h * x)
    fd1 = (lp - lm) / (2 * h)
    assert abs(fd1 - r["g1"]) <= 1e-6 * max(abs(r["g1"]), 1.0)
    g1p = risk.brute(model, y, s, eta + h * x, x)["g1"]
    g1m = risk.brute(model, y, s, eta - h * x, x)["g1"]
    fd2 = (g1p - g1m) / (2 * h)
    assert abs(fd2 - r["g2"]) <= 1e-6 * abs(r["g2"])


@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,n,ties", [(15, 300, 0), (16, 1200, 40)])
def test_complex_step(model, seed, n, ties):
    """Complex step h = 1e-30: Im l(eta + i h x_j) / h = g' and
    Im g'(eta + i h x_j) / h = g'' to near machine precision."""
    y, s, eta, x = _rand_problem(seed, n, model, ties=ties)
    h = 1e-30
    r = risk.brute(model, y, s, eta, x)
    etac = eta + 1j * h * x
    cs1 = np.imag(risk.loglik(model, y, s, etac)) / h
    cs2 = np.imag(risk.brute(model, y, s, etac, x)["g1"]) / h
    assert cs1 == pytest.approx(r["g1"], rel=1e-11, abs=1e-11)
    assert cs2 == pytest.approx(r["g2"], rel=1e-12)


# ---------------------------------------------------------------- invariances

@pytest.mark.parametrize("model", ["cox", "fg"])
def test_shift_and_permutation_invariance(model):
    y, s, eta, x = _rand_problem(17, 800, model, ties=30)
    base = risk.brute(model, y, s, eta, x)
    sh = risk.brute(model, y, s, eta + 3.25, x)
    for k in ("g1", "g2", "loglik"):
        assert sh[k] == pytest.approx(base[k], rel=1e-11, abs=1e-11)
    perm = np.random.default_rng(0).permutation(y.size)
    pr = scan.scan(model, y[perm], s[perm], eta[perm], x[perm])
    for k in ("g1", "g2", "loglik"):
        assert pr[k] == pytest.approx(base[k], rel=1e-11, abs=1e-11)


@pytest.mark.parametrize("model", ["cox", "fg"])
def test_constant_column_and_indicator(model):
    y, s, eta, _ = _rand_problem(18, 500, model, ties=10)
    r = risk.brute(model, y, s, eta, np.full(500, 2.5))
    assert abs(r["g1"]) < 1e-11 and abs(r["g2"]) < 1e-11
    xb = (np.random.default_rng(1).random(500) < 0.2).astype(float)
    r = risk.brute(model, y, s, eta, xb)
    np.testing.assert_allclose(r["H"], r["G"], rtol=1e-14)
    assert r["g2"] == pytest.approx(-np.sum(r["G"] * (1 - r["G"])), rel=1e-12)
    assert r["g2"] <= 0


def test_event_at_largest_time_contributes_nothing():
    y = np.array([5.0, 1.0, 2.0, 3.0]); s = np.array([1, 0, 0, 0])
    r = risk.cox_brute(y, s, np.array([0.3, -1, 2, 0.1]), np.array([2.0, 1, 0, 4]))
    assert r["g1"] == 0.0 and r["g2"] == 0.0


def test_hessian_nonpositive():
    for seed in range(5):
        for model in ("cox", "fg"):
            y, s, eta, x = _rand_problem(40 + seed, 400, model, ties=seed * 5)
            assert risk.brute(model, y, s, eta, x)["g2"] <= 0


# ---------------------------------------------------------------- model reductions

def test_fg_without_competing_events_is_cox():
    y, s, eta, x = _rand_problem(19, 700, "cox", ties=15)
    fg = risk.fg_brute(y, s, eta, x)
    cx = risk.cox_brute(y, s, eta, x)
    for k in ("g1", "g2", "loglik"):
        assert fg[k] == pytest.approx(cx[k], rel=1e-13, abs=1e-13)


def test_fg_without_censoring_is_cox_with_competing_times_at_infinity():
    """With no censoring G = 1, and the Fine-Gray risk set of an event at
    Y_i is {y_r >= Y_i} plus every earlier competing event with weight 1:
    the Cox risk set after moving competing events past every time."""
    rng = np.random.default_rng(20)
    n = 600
    y = rng.exponential(1.0, n)
    s = np.where(rng.random(n) < 0.5, 1, 2)
    eta = rng.normal(0, 0.5, n); x = rng.normal(0, 1, n)
    fg = risk.fg_brute(y, s, eta, x)
    y2 = np.where(s == 2, y.max() + 1.0, y)
    s2 = (s == 1).astype(int)
    cx = risk.cox_brute(y2, s2, eta, x)
    for k in ("g1", "g2", "loglik"):
        assert fg[k] == pytest.approx(cx[k], rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------- CCD update

def test_ccd_branches():
    N, L1, L2 = ccd.PENALTY_NONE, ccd.PENALTY_L1, ccd.PENALTY_L2
    # plain Newton: -g'/g''
    assert ccd.newton_step(2.0, -4.0, 0.3, N, 0) == 0.5
    # l2: (g' - b/tau) / -(g'' - 1/tau)
    assert ccd.newton_step(2.0, -4.0, 1.0, L2, 2.0) == pytest.approx(1.5 / 4.5)
    # l1 at zero: positive direction, negative direction, stay
    assert ccd.newton_step(3.0, -2.0, 0.0, L1, 1.0) == 1.0
    assert ccd.newton_step(-3.0, -2.0, 0.0, L1, 1.0) == -1.0
    assert ccd.newton_step(0.5, -2.0, 0.0, L1, 1.0) == 0.0
    # l1 away from zero: (g' - gamma sgn b) / -g''
    assert ccd.newton_step(3.0, -2.0, 0.5, L1, 1.0) == 1.0
    # l1 sign crossing stops at zero
    assert ccd.newton_step(-5.0, -2.0, 0.5, L1, 1.0) == -0.5
    # trust region: applied step clipped to Delta, width from the Newton step
    b, d, a = ccd.update(10.0, -2.0, 0.0, 1.0, N, 0)
    assert (b, d, a) == (1.0, 10.0, 1.0)
    b, d, a = ccd.update(0.1, -1.0, 0.0, 1.0, N, 0)
    assert (b, d, a) == (0.1, 0.5, 0.1)
    # non-negative curvature: no step
    assert ccd.newton_step(1.0, 0.0, 0.0, N, 0) == 0.0


# ---------------------------------------------------------------- prep

def test_prep_order_runs_and_counts():
    y = np.array([3.0, 1.0, 3.0, 2.0, 3.0, 1.0])
    s = np.array([1, 0, 0, 1, 1, 1])
    o = prep.order(y)
    np.testing.assert_array_equal(o, [0, 2, 4, 3, 1, 5])
    ys = y[o]
    np.testing.assert_array_equal(prep.run_end(ys), [2, 2, 2, 3, 5, 5])
    np.testing.assert_array_equal(prep.d_end(ys, s[o]), [0, 0, 2, 1, 0, 1])


# ---------------------------------------------------------------- full gradient in eta

@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,n,ties", [(21, 1, 0), (22, 9, 0), (23, 120, 15), (24, 400, 0)])
def test_eta_gradient_complex_step(model, seed, n, ties):
    """dl/deta_m from the chain-rule definition equals the complex-step
    derivative Im l(eta + i h e_m) / h of the likelihood itself (h = 1e-30),
    for every m (ties included)."""
    y, s, eta, _ = _rand_problem(seed, n, model, ties=ties)
    from oracle import adjoint
    g = adjoint.eta_gradient_brute(model, y, s, eta)
    h = 1e-30
    for m in range(n):
        etac = eta.astype(np.complex128)
        etac[m] += 1j * h
        cs = np.imag(risk.loglik(model, y, s, etac)) / h
        assert cs == pytest.approx(g[m], rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("seed,n,ties", [(25, 1, 0), (26, 2, 0), (27, 300, 0), (28, 900, 40),
                                          (29, 2000, 300)])
def test_eta_gradient_scan_matches_brute(model, seed, n, ties):
    """The O(N) prefix/suffix form equals the O(N^2) definition; its inner
    product with a column is the coordinate gradient g' (the directional
    derivative of l along x_j); it sums to zero (l(eta + c) = l(eta))."""
    from oracle import adjoint
    y, s, eta, x = _rand_problem(seed, n, model, ties=ties)
    gb = adjoint.eta_gradient_brute(model, y, s, eta)
    gs = adjoint.eta_gradient_scan(model, y, s, eta)
    scale = np.sum(np.abs(gb)) + 1.0
    assert np.max(np.abs(gs - gb)) <= 1e-12 * scale
    r = risk.brute(model, y, s, eta, x)
    assert float(np.dot(x, gs)) == pytest.approx(r["g1"], rel=1e-11, abs=1e-11 * scale)
    assert abs(float(np.sum(gs))) <= 1e-11 * scale
    assert adjoint.loglik_eta(model, y, s, eta) == pytest.approx(
        risk.loglik(model, y, s, eta), rel=1e-12, abs=1e-12)


def test_eta_gradient_hand_example():
    """Three subjects, times 3 > 2 > 1, all events, e = (1, 2, 4): the risk
    sets at the event times 3, 2, 1 have S0 = 1, 3, 7, and a subject's
    derivative is 1 - e_m times the sum of 1/S0 over the events whose risk
    set holds it (event times at or below its own time): subject at t=3:
    1 - 1 (1/1 + 1/3 + 1/7); t=2: 1 - 2 (1/3 + 1/7); t=1: 1 - 4 (1/7)."""
    from oracle import adjoint
    y = np.array([3.0, 2.0, 1.0])
    s = np.array([1, 1, 1])
    eta = np.log([1.0, 2.0, 4.0])
    want = np.array([1 - (1 + 1 / 3 + 1 / 7), 1 - 2 * (1 / 3 + 1 / 7), 1 - 4 / 7])
    np.testing.assert_allclose(adjoint.eta_gradient_brute("cox", y, s, eta), want, rtol=1e-14)
    np.testing.assert_allclose(adjoint.eta_gradient_scan("cox", y, s, eta), want, rtol=1e-14)


# ---------------------------------------------------------------- cross-validation

def _cv_problem(model, seed, n, p):
    d = gen.cox_data(seed, n, p, 0.2) if model == "cox" else gen.fg_data(seed, n, p, 0.2)
    return d


@pytest.mark.parametrize("model", ["cox", "fg"])
def test_cv_fit_equals_fit_on_smaller_data_set(model):
    """A replicate's fit is CCD on the training subjects as a data set of
    their own: built independently here from the dense design restricted to
    the training rows, it gives the same beta bit for bit."""
    from oracle import cv
    d = _cv_problem(model, 3, 300, 6)
    train = gen.cv_folds(5, d["n"], 5, 1)[2]
    beta, delta, eta_all, hist = cv.fit_replicate(model, d["y"], d["status"], d["col_ptr"],
                                                  d["rows"], None, train, ccd.PENALTY_L1, 1.0, 2)
    X = np.stack([gen.dense_column(d["n"], d["col_ptr"], d["rows"], None, j)
                  for j in range(d["p"])], axis=1)
    tr = train == 1
    cp, rr, vv = gen.csc_from_dense(X[tr])
    b2, d2, eta2, _ = cv.ccd_sweeps(model, d["y"][tr], d["status"][tr], cp, rr, None,
                                    np.zeros(int(tr.sum())), ccd.PENALTY_L1, 1.0, 2)
    assert np.array_equal(beta, b2) and np.array_equal(delta, d2)
    np.testing.assert_allclose(eta_all, X @ beta, rtol=1e-13, atol=1e-13)
    assert np.any(beta != 0.0)


@pytest.mark.parametrize("model", ["cox", "fg"])
def test_cv_fit_ignores_heldout_subjects(model):
    """Changing the times, statuses and covariates of held-out subjects
    leaves the training fit unchanged (a risk set or KM estimate over all
    subjects would not)."""
    from oracle import cv
    d = _cv_problem(model, 4, 250, 5)
    train = gen.cv_folds(6, d["n"], 4, 1)[1]
    ho = np.nonzero(train == 0)[0]
    fit = cv.fit_replicate(model, d["y"], d["status"], d["col_ptr"], d["rows"], None, train,
                           ccd.PENALTY_NONE, 0.0, 1)
    y2 = d["y"].copy()
    s2 = d["status"].copy()
    rng = np.random.default_rng(0)
    y2[ho] = rng.exponential(1.0, ho.size)
    s2[ho] = 2 if model == "fg" else 0
    rows = np.asarray(d["rows"])
    keep = np.isin(rows, ho, invert=True)      # drop the held-out non-zeros
    cp = np.concatenate(([0], np.cumsum([int(keep[d["col_ptr"][j]:d["col_ptr"][j + 1]].sum())
                                         for j in range(d["p"])])))
    fit2 = cv.fit_replicate(model, y2, s2, cp, rows[keep], None, train, ccd.PENALTY_NONE,
                            0.0, 1)
    assert np.array_equal(fit[0], fit2[0])
    # the full-data fit differs (the held-out subjects matter there)
    full = cv.fit_replicate(model, d["y"], d["status"], d["col_ptr"], d["rows"], None,
                            np.ones(d["n"], np.uint8), ccd.PENALTY_NONE, 0.0, 1)
    assert not np.array_equal(fit[0], full[0])


def test_cv_heldout_loglik_hand_example():
    """Held-out subjects at times 3 > 2 > 1, all events, e = (1, 2, 4):
    the held-out risk sets give S0 = 1, 3, 7, so the predictive
    log-likelihood is (0 + log 2 + log 4) - (log 1 + log 3 + log 7).
    Training subjects interleaved with them (any time, status, eta) do not
    enter; the training likelihood is the same form on the training set."""
    from oracle import cv
    y = np.array([3.0, 2.5, 2.0, 1.5, 1.0, 0.5])
    s = np.array([1, 1, 1, 0, 1, 1])
    eta = np.log([1.0, 5.0, 2.0, 7.0, 4.0, 3.0])
    train = np.array([0, 1, 0, 1, 0, 1], np.uint8)
    want = math.log(2) + math.log(4) - (math.log(1) + math.log(3) + math.log(7))
    assert cv.heldout_loglik("cox", y, s, eta, train) == pytest.approx(want, rel=1e-14)
    # training set: times 2.5 (event, e 5), 1.5 (censored, e 7), 0.5 (event, e 3)
    want_tr = math.log(5) + math.log(3) - (math.log(5) + math.log(15))
    assert cv.training_loglik("cox", y, s, eta, train) == pytest.approx(want_tr, rel=1e-14)


def test_cv_folds_partition():
    m = gen.cv_folds(1, 1003, 10, 3)
    assert m.shape == (30, 1003)
    for t in range(3):
        held = 1 - m[t * 10:(t + 1) * 10].astype(int)
        assert np.all(held.sum(axis=0) == 1)            # held out exactly once
        sizes = held.sum(axis=1)
        assert sizes.max() - sizes.min() <= 1
