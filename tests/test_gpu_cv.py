"""GPU: cross-validation replicates in one launch (ss_cv_*) against the
oracle's definition (oracle.cv: CCD on each replicate's training subset, the
held-out log-likelihood on the held-out subset).

Checks:
  * preparation, bit for bit: the training events per run end (as the
    sequence of (time, count) over run ends with training events, which
    does not depend on where the positions sit) and c_j per replicate;
  * sweeps: g' and g'' of every coordinate visit of every replicate within
    the condition-scaled bound (1e-10 for one sweep, 1e-9 over repeated
    sweeps as for the single-problem sweep), beta and delta, eta = X beta
    for every subject including the held-out ones;
  * training and held-out log-likelihoods against the oracle at the GPU's
    eta;
  * a replicate that trains on everyone equals the single-problem sweep;
    replicates without training events take zero steps; determinism;
  * the 10 x 10 cross-validation design at N = 1e5, P = 1000 (sampled
    replicates against the oracle over the whole sweep).
"""
import numpy as np
import pytest

import gen
from oracle import ccd as occd, cv as ocv, prep as oprep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2204_08183_amd import survscan as ss  # noqa: E402

DEV = "cuda:0"
PEN = {"none": occd.PENALTY_NONE, "l1": occd.PENALTY_L1, "l2": occd.PENALTY_L2}


def cox_case(n, p, seed, ties=0, density=0.1):
    d = gen.cox_data(seed, n, p, density)
    if ties:
        d["y"] = gen.force_ties(d["y"], ties)
    return d


def fg_case(n, p, seed, ties=0, density=0.1):
    d = gen.fg_data(seed, n, p, density)
    if ties:
        d["y"] = gen.force_ties(d["y"], ties)
    return d


def make_cv(d, train, model="cox"):
    prob = ss.Problem(model, d["y"], d["status"], d["col_ptr"], d["rows"], None, DEV)
    return prob, ss.CrossValidation(prob, train)


def run_end_counts(y_sorted, d):
    at = np.nonzero(d)[0]
    return list(zip(y_sorted[at].tolist(), d[at].tolist()))


def test_cv_prepare_matches_oracle():
    d = cox_case(20001, 7, 1, ties=300)
    train = gen.cv_folds(3, d["n"], 5, 2)
    prob, cvp = make_cv(d, train)
    perm = prob.perm.cpu().numpy()
    ys = d["y"][perm]
    d8 = cvp.sorted_view(cvp.d8_r).cpu().numpy().astype(np.int64)
    d32 = cvp.sorted_view(cvp.d32_r).cpu().numpy()
    dr = np.where(d8 == 255, d32, d8)
    ts = cvp.sorted_view(cvp.train_s).cpu().numpy()
    c = cvp.c.cpu().numpy().reshape(cvp.reps, d["p"])
    pad = cvp.train_s.view(cvp.reps, cvp.stride)[:, d["n"]:].cpu().numpy()
    assert np.all(pad == 0)
    for r in range(cvp.reps):
        tr = train[r] == 1
        assert np.array_equal(ts[r], train[r][perm])
        ysub = d["y"][tr]
        o = oprep.order(ysub)
        want_d = oprep.d_end(ysub[o], oprep.event_indicator("cox", d["status"][tr])[o])
        assert run_end_counts(ys, dr[r]) == run_end_counts(ysub[o], want_d), r
        for j in range(d["p"]):
            x = ocv.column(d["n"], d["col_ptr"], d["rows"], None, j)
            want_c = float(np.sum(x[tr] * (d["status"][tr] != 0)))
            assert c[r, j] == want_c, (r, j)


def test_cv_prepare_long_tie_runs():
    """Runs of more than 255 training events (the int32 escape)."""
    d = cox_case(6000, 3, 2, ties=4)
    d["status"] = np.ones(d["n"], np.int8)
    train = gen.cv_folds(4, d["n"], 3, 1)
    prob, cvp = make_cv(d, train)
    perm = prob.perm.cpu().numpy()
    d8 = cvp.sorted_view(cvp.d8_r).cpu().numpy().astype(np.int64)
    d32 = cvp.sorted_view(cvp.d32_r).cpu().numpy()
    dr = np.where(d8 == 255, d32, d8)
    assert np.any(d8 == 255)
    for r in range(cvp.reps):
        tr = train[r] == 1
        ysub = d["y"][tr]
        o = oprep.order(ysub)
        want_d = oprep.d_end(ysub[o], np.ones(int(tr.sum()), np.int64))
        assert run_end_counts(d["y"][perm], dr[r]) == run_end_counts(ysub[o], want_d)


def check_sweeps(d, train, penalty, lam, sweeps, tol, reps_to_check=None, model="cox"):
    prob, cvp = make_cv(d, train, model)
    R, p, n = cvp.reps, d["p"], d["n"]
    g12 = torch.zeros(R * p * 3, dtype=torch.float64, device=DEV)
    hist_gpu = []
    for _ in range(sweeps):
        cvp.sweep(penalty, lam, g12_out=g12)
        hist_gpu.append(g12.cpu().numpy().reshape(R, p, 3).copy())
    beta = cvp.beta.cpu().numpy().reshape(R, p)
    delta = cvp.delta.cpu().numpy().reshape(R, p)
    perm = prob.perm.cpu().numpy()
    eta_s = cvp.sorted_view(cvp.eta).cpu().numpy()
    e_s = cvp.sorted_view(cvp.e).cpu().numpy()
    ll = cvp.loglik().cpu().numpy()
    assert cvp.workspace_error() == 0
    for r in (range(R) if reps_to_check is None else reps_to_check):
        b, dl, eta_all, hist = ocv.fit_replicate(model, d["y"], d["status"], d["col_ptr"],
                                                 d["rows"], None, train[r], PEN[penalty], lam,
                                                 sweeps)
        for s in range(sweeps):
            for j in range(p):
                g1, g2, s1, s2 = hist[s * p + j]
                got = hist_gpu[s][r, j]
                assert abs(got[0] - g1) <= tol * s1, (r, s, j, got[0], g1)
                assert abs(got[1] - g2) <= tol * max(s2, 1e-300), (r, s, j, got[1], g2)
        np.testing.assert_allclose(beta[r], b, rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(delta[r], dl, rtol=1e-8, atol=1e-12)
        eta = np.empty(n)
        eta[perm] = eta_s[r]
        np.testing.assert_allclose(eta, eta_all, rtol=1e-9, atol=1e-11)
        tr = train[r] == 1
        np.testing.assert_allclose(e_s[r], np.where(tr[perm], np.exp(eta_s[r]), 0.0), rtol=1e-15)
        # likelihoods at the GPU's eta
        lt = ocv.training_loglik(model, d["y"], d["status"], eta, train[r])
        lh = ocv.heldout_loglik(model, d["y"], d["status"], eta, train[r])
        assert ll[r, 0] == pytest.approx(lt, rel=1e-11, abs=1e-11)
        assert ll[r, 1] == pytest.approx(lh, rel=1e-11, abs=1e-11)
    return prob, cvp


HALVES = ["two", "one"]


def _halves(monkeypatch, halves):
    """Two workgroups per replicate (the default when they fit) or one."""
    if halves == "one":
        monkeypatch.setenv("SURVSCAN_CV_HALVES", "1")
    else:
        monkeypatch.delenv("SURVSCAN_CV_HALVES", raising=False)


@pytest.mark.parametrize("halves", HALVES)
@pytest.mark.parametrize("penalty,lam", [("l1", 2.0), ("l2", 1.0), ("none", 0.0)])
def test_cv_sweeps_match_oracle(penalty, lam, halves, monkeypatch):
    _halves(monkeypatch, halves)
    d = cox_case(7000, 8, 5, density=0.2)
    train = gen.cv_folds(6, d["n"], 4, 2)
    check_sweeps(d, train, penalty, lam, 2, 1e-9)


@pytest.mark.parametrize("halves", HALVES)
# chunks of 8192 positions, strides of 16384: 16384 fills its stride,
# 16385 and 50001 leave a chunk of pure padding that the sweep skips
@pytest.mark.parametrize("n,p,ties", [(1, 2, 0), (3, 2, 0), (8193, 4, 0), (50001, 5, 40),
                                      (24577, 3, 0), (16384, 3, 0), (16385, 3, 5)])
def test_cv_sizes_and_ties(n, p, ties, halves, monkeypatch):
    _halves(monkeypatch, halves)
    d = cox_case(n, p, 7, ties=ties, density=0.3 if n < 10 else 0.1)
    train = gen.cv_folds(8, n, 3, 2) if n >= 3 else np.ones((2, n), np.uint8)
    check_sweeps(d, train, "l1", 0.5, 1, 1e-10)


def test_cv_everyone_training_equals_single_sweep():
    d = cox_case(30000, 6, 9)
    train = np.ones((2, d["n"]), np.uint8)
    prob, cvp = make_cv(d, train)
    g12 = torch.zeros(2 * d["p"] * 3, dtype=torch.float64, device=DEV)
    cvp.sweep("l1", 1.0, g12_out=g12)
    single = torch.zeros(3 * d["p"], dtype=torch.float64, device=DEV)
    prob.sweep("l1", 1.0, g12_out=single)
    got = g12.cpu().numpy().reshape(2, d["p"], 3)
    want = single.cpu().numpy().reshape(d["p"], 3)
    np.testing.assert_allclose(got[0, :, :2], want[:, :2], rtol=1e-10, atol=1e-9)
    assert np.array_equal(got[0], got[1])
    np.testing.assert_allclose(cvp.beta.cpu().numpy()[:d["p"]], prob.beta.cpu().numpy(),
                               rtol=1e-10, atol=1e-13)


def test_cv_no_training_events():
    """A replicate whose training subjects are all censored and one with
    no training subjects: g' = g'' = 0, no step, likelihoods 0 where
    there are no events."""
    d = cox_case(5000, 4, 10)
    train = np.ones((3, d["n"]), np.uint8)
    train[0, d["status"] != 0] = 0          # training subjects all censored
    train[1, :] = 0                         # nobody trains
    prob, cvp = make_cv(d, train)
    g12 = torch.zeros(3 * d["p"] * 3, dtype=torch.float64, device=DEV)
    cvp.sweep("none", 0.0, g12_out=g12)
    got = g12.cpu().numpy().reshape(3, d["p"], 3)
    assert np.all(got[:2] == 0.0)
    assert np.all(cvp.beta.cpu().numpy().reshape(3, d["p"])[:2] == 0.0)
    ll = cvp.loglik().cpu().numpy()
    assert ll[0, 0] == 0.0 and ll[1, 0] == 0.0
    assert ll[2, 1] == 0.0                  # nothing held out
    want = ocv.heldout_loglik("cox", d["y"], d["status"], np.zeros(d["n"]), train[1])
    assert ll[1, 1] == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("halves", HALVES)
def test_cv_deterministic_and_set_eta(halves, model, monkeypatch):
    _halves(monkeypatch, halves)
    d = cox_case(40000, 5, 11) if model == "cox" else fg_case(40000, 5, 11)
    train = gen.cv_folds(12, d["n"], 5, 1)
    outs = []
    for _ in range(2):
        prob, cvp = make_cv(d, train, model)
        rng = np.random.default_rng(3)
        eta0 = rng.normal(0.0, 0.3, (cvp.reps, d["n"]))
        cvp.set_eta(eta0)
        g12 = torch.zeros(cvp.reps * d["p"] * 3, dtype=torch.float64, device=DEV)
        cvp.sweep("l1", 0.3, g12_out=g12)
        cvp.sweep("l1", 0.3, g12_out=g12)
        outs.append((g12.cpu().numpy().copy(), cvp.eta.cpu().numpy().copy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    # first sweep from a non-zero eta against the oracle (replicate 2)
    prob, cvp = make_cv(d, train, model)
    cvp.set_eta(eta0)
    g12 = torch.zeros(cvp.reps * d["p"] * 3, dtype=torch.float64, device=DEV)
    cvp.sweep("l1", 0.3, g12_out=g12)
    got = g12.cpu().numpy().reshape(cvp.reps, d["p"], 3)
    r = 2
    tr = train[r] == 1
    ys, sts, cp, rr, _, idx = ocv.subset(d["y"], d["status"], d["col_ptr"], d["rows"], None, tr)
    _, _, _, hist = ocv.ccd_sweeps(model, ys, sts, cp, rr, None, eta0[r][idx],
                                   occd.PENALTY_L1, 0.3, 1)
    for j in range(d["p"]):
        g1, g2, s1, s2 = hist[j]
        assert abs(got[r, j, 0] - g1) <= 1e-10 * s1
        assert abs(got[r, j, 1] - g2) <= 1e-10 * s2


def test_cv_rejects_unsupported():
    d = cox_case(3000, 2, 13)
    prob = ss.Problem("cox", d["y"], d["status"], d["col_ptr"], d["rows"], None, DEV)
    cvp = ss.CrossValidation(prob, gen.cv_folds(1, d["n"], 3, 1))
    lib = ss.load()
    args = [ss._p(cvp.eta), ss._p(cvp.e), ss._p(cvp.d8_r), ss._p(cvp.d32_r),
            ss._p(cvp.train_s), ss._p(cvp.xbits), ss._p(cvp.c), ss._p(cvp.beta),
            ss._p(cvp.delta), None, cvp.ws.ptr, cvp.ws.nbytes, None]
    args = args[:7] + [None, None] + args[7:]   # w_r, g_r: Fine-Gray only
    # Fine-Gray without its weights
    assert lib.ss_cv_sweep(ss.FINE_GRAY, 0, 0.0, prob.n, prob.p, 3, 0, 2,
                           *args) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(5, 0, 0.0, prob.n, prob.p, 3, 0, 2, *args) == ss.SS_EUNSUPPORTED
    assert lib.ss_cv_sweep(ss.COX, 0, 0.0, prob.n, prob.p, 3, 0, 3, *args) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(ss.COX, 0, 0.0, prob.n, prob.p, 0, 0, 2, *args) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(ss.COX, 9, 0.0, prob.n, prob.p, 3, 0, 2, *args) == ss.SS_EUNSUPPORTED
    assert lib.ss_cv_sweep(ss.COX, 1, 0.0, prob.n, prob.p, 3, 0, 2, *args) == ss.SS_EINVAL
    assert lib.ss_cv_sweep(ss.COX, 2, -1.0, prob.n, prob.p, 3, 0, 2, *args) == ss.SS_EINVAL
    # an empty coordinate range is a no-op that still resynchronises e
    assert lib.ss_cv_sweep(ss.COX, 0, 0.0, prob.n, prob.p, 3, 1, 1, *args) == ss.SS_OK
    short = args[:-3] + [cvp.ws.ptr, cvp.ws.nbytes - 1, None]
    assert lib.ss_cv_sweep(ss.COX, 0, 0.0, prob.n, prob.p, 3, 0, 2, *short) == ss.SS_EWORKSPACE
    valued = ss.Problem("cox", d["y"], d["status"], d["col_ptr"], d["rows"],
                        np.ones(d["rows"].size), DEV)
    with pytest.raises(ss.SurvScanError):
        ss.CrossValidation(valued, gen.cv_folds(1, d["n"], 3, 1))
    fg = gen.fg_data(1, 3000, 2, 0.1)
    fprob = ss.Problem("fg", fg["y"], fg["status"], fg["col_ptr"], fg["rows"],
                       np.ones(fg["rows"].size), DEV)
    with pytest.raises(ss.SurvScanError):
        ss.CrossValidation(fprob, gen.cv_folds(1, 3000, 3, 1))


@pytest.mark.parametrize("halves", HALVES)
def test_cv_ten_by_ten_design(halves, monkeypatch):
    _halves(monkeypatch, halves)
    """10-fold x 10-repetition cross-validation at N = 1e5, P = 1000 (the
    Sec. 3.3 design at its smallest size), one l1 sweep: replicates 0, 57
    and 99 against the oracle over all 1000 coordinates."""
    d = cox_case(100_000, 1000, 0, density=0.05)
    train = gen.cv_folds(0, d["n"], 10, 10)
    check_sweeps(d, train, "l1", float(np.sqrt(2.0)), 1, 1e-10, reps_to_check=(0, 57, 99))


@pytest.mark.parametrize("halves", HALVES)
def test_cv_many_steps_in_one_launch(halves, monkeypatch):
    _halves(monkeypatch, halves)
    """More non-zero steps in one launch than the kernel holds before it
    brings eta up to date (no penalty: every coordinate moves), checked
    against the oracle over two sweeps."""
    d = cox_case(2500, 700, 14, density=0.05)
    train = gen.cv_folds(15, d["n"], 5, 1)[:2]
    check_sweeps(d, train, "none", 0.0, 2, 1e-9)


@pytest.mark.parametrize("model", ["cox", "fg"])
@pytest.mark.parametrize("reps", [1, 150])
def test_cv_replicate_counts(reps, model, monkeypatch):
    """One replicate, and more replicates than fit two workgroups each on
    the device at once (the launch then takes one workgroup per replicate
    by itself); sampled replicates against the oracle."""
    monkeypatch.delenv("SURVSCAN_CV_HALVES", raising=False)
    d = cox_case(9000, 4, 16, density=0.1) if model == "cox" else \
        fg_case(9000, 4, 16, density=0.1)
    rng = np.random.default_rng(17)
    train = (rng.random((reps, d["n"])) < 0.8).astype(np.uint8)
    check_sweeps(d, train, "l1", 0.7, 2, 1e-9,
                 reps_to_check=(0,) if reps == 1 else (0, 77, reps - 1), model=model)


def test_cv_path_matches_oracle():
    """Sec. 2.8 over a path of l1 strengths with warm starts: the held-out
    log-likelihood of every replicate at every strength, and the chosen
    strength, against the oracle's path on the training subsets."""
    d = cox_case(3000, 8, 18, density=0.2)
    train = gen.cv_folds(19, d["n"], 5, 1)
    gammas = [16.0, 8.0, 4.0, 2.0, 1.0]
    prob = ss.Problem("cox", d["y"], d["status"], d["col_ptr"], d["rows"], None, DEV)
    scores, best = ss.cv_path(prob, train, gammas, sweeps=3)
    assert scores.shape == (len(gammas), train.shape[0])
    want = np.stack([ocv.path("cox", d["y"], d["status"], d["col_ptr"], d["rows"], None,
                              train[r], occd.PENALTY_L1, gammas, 3)
                     for r in range(train.shape[0])], axis=1)
    np.testing.assert_allclose(scores, want, rtol=1e-9, atol=1e-9)
    assert best == gammas[int(want.mean(axis=1).argmax())]
    assert len(set(np.round(scores.mean(axis=1), 6))) > 1   # the path moves


# ---------------------------------------------------------------- Fine-Gray
def test_cv_fg_prepare_km_matches_oracle():
    """Per replicate: the Kaplan-Meier estimate of the censoring
    distribution of its training subjects and of its held-out subjects at
    every sorted position, and the training competing-event weights, against
    the oracle's estimate on the subsets (with tie runs across the folds)."""
    from oracle import km as okm
    d = fg_case(20001, 3, 21, ties=700)
    train = gen.cv_folds(22, d["n"], 4, 2)
    prob, cvp = make_cv(d, train, "fg")
    perm = prob.perm.cpu().numpy()
    ys = d["y"][perm]
    st = d["status"][perm]
    g_r = cvp.sorted_view(cvp.g_r).cpu().numpy()
    g_h = cvp.sorted_view(cvp.g_h).cpu().numpy()
    w_r = cvp.sorted_view(cvp.w_r).cpu().numpy()
    pad = cvp.w_r.view(cvp.reps, cvp.stride)[:, d["n"]:].cpu().numpy()
    assert np.all(pad == 0.0)
    for r in range(cvp.reps):
        tr = train[r] == 1
        for mask, got in ((tr, g_r[r]), (~tr, g_h[r])):
            t, v = okm.km_censoring(d["y"][mask], d["status"][mask])
            np.testing.assert_allclose(got, okm.km_eval(t, v, ys), rtol=1e-12, atol=0)
        want_w = np.where(tr[perm] & (st == 2), 1.0 / g_r[r], 0.0)
        np.testing.assert_array_equal(w_r[r], want_w)
        # c_j counts training events of type 1 only
        c = cvp.c.cpu().numpy().reshape(cvp.reps, d["p"])
        for j in range(d["p"]):
            x = ocv.column(d["n"], d["col_ptr"], d["rows"], None, j)
            assert c[r, j] == float(np.sum(x[tr] * (d["status"][tr] == 1)))


@pytest.mark.parametrize("halves", HALVES)
@pytest.mark.parametrize("penalty,lam", [("l1", 2.0), ("l2", 1.0), ("none", 0.0)])
def test_cv_fg_sweeps_match_oracle(penalty, lam, halves, monkeypatch):
    _halves(monkeypatch, halves)
    d = fg_case(7000, 8, 23, density=0.2)
    train = gen.cv_folds(24, d["n"], 4, 2)
    check_sweeps(d, train, penalty, lam, 2, 1e-9, model="fg")


@pytest.mark.parametrize("halves", HALVES)
# chunks of 4096 positions: 16384 fills its stride, 16385, 40961 and 50001
# leave chunks of pure padding; the halves split the chunks 12:13
@pytest.mark.parametrize("n,p,ties", [(1, 2, 0), (3, 2, 0), (8193, 4, 0), (50001, 5, 40),
                                      (16384, 3, 0), (16385, 3, 5), (40961, 3, 30)])
def test_cv_fg_sizes_and_ties(n, p, ties, halves, monkeypatch):
    _halves(monkeypatch, halves)
    d = fg_case(n, p, 25, ties=ties, density=0.3 if n < 10 else 0.1)
    train = gen.cv_folds(26, n, 3, 2) if n >= 3 else np.ones((2, n), np.uint8)
    check_sweeps(d, train, "l1", 0.5, 1, 1e-10, model="fg")


@pytest.mark.parametrize("halves", HALVES)
def test_cv_fg_many_steps_in_one_launch(halves, monkeypatch):
    """More non-zero steps than the kernel holds before eta is brought up to
    date, so the carried weighted totals cross that update too."""
    _halves(monkeypatch, halves)
    d = fg_case(2500, 700, 27, density=0.05)
    train = gen.cv_folds(28, d["n"], 5, 1)[:2]
    check_sweeps(d, train, "none", 0.0, 2, 1e-9, model="fg")


def test_cv_fg_everyone_training_equals_single_sweep():
    d = fg_case(30000, 6, 29)
    train = np.ones((2, d["n"]), np.uint8)
    prob, cvp = make_cv(d, train, "fg")
    g12 = torch.zeros(2 * d["p"] * 3, dtype=torch.float64, device=DEV)
    cvp.sweep("l1", 1.0, g12_out=g12)
    single = torch.zeros(3 * d["p"], dtype=torch.float64, device=DEV)
    prob.sweep("l1", 1.0, g12_out=single)
    got = g12.cpu().numpy().reshape(2, d["p"], 3)
    want = single.cpu().numpy().reshape(d["p"], 3)
    np.testing.assert_allclose(got[0, :, :2], want[:, :2], rtol=1e-10, atol=1e-9)
    assert np.array_equal(got[0], got[1])


@pytest.mark.parametrize("halves", HALVES)
def test_cv_fg_ten_by_ten_design(halves, monkeypatch):
    """10 x 10 cross-validation of the Fine-Gray model at N = 1e5,
    P = 1000, one l1 sweep: replicates 0, 57 and 99 against the oracle."""
    _halves(monkeypatch, halves)
    d = fg_case(100_000, 1000, 0, density=0.05)
    train = gen.cv_folds(0, d["n"], 10, 10)
    check_sweeps(d, train, "l1", float(np.sqrt(2.0)), 1, 1e-10, reps_to_check=(0, 57, 99),
                 model="fg")


def test_cv_fg_path_matches_oracle():
    d = fg_case(3000, 8, 30, density=0.2)
    train = gen.cv_folds(31, d["n"], 5, 1)
    gammas = [16.0, 8.0, 4.0, 2.0, 1.0]
    prob = ss.Problem("fg", d["y"], d["status"], d["col_ptr"], d["rows"], None, DEV)
    scores, best = ss.cv_path(prob, train, gammas, sweeps=3)
    want = np.stack([ocv.path("fg", d["y"], d["status"], d["col_ptr"], d["rows"], None,
                              train[r], occd.PENALTY_L1, gammas, 3)
                     for r in range(train.shape[0])], axis=1)
    np.testing.assert_allclose(scores, want, rtol=1e-9, atol=1e-9)
    assert best == gammas[int(want.mean(axis=1).argmax())]
