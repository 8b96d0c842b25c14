"""ss_grad_hess_noalloc (scratch in a file-scope device array) against
ss_grad_hess (caller workspace) and the oracle, through the C ABI: two
calls in a row on one device, the second with a smaller problem, for both
models, plus the argument checks that need no launch."""

import numpy as np
import pytest
import torch

import gen
from oracle import scan as oscan
from paper_2204_08183_amd import survscan as ss

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-10


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _case(model, n, p, seed, ties, valued):
    d = gen.cox_data(seed, n, p, 0.1) if model == "cox" else gen.fg_data(seed, n, p, 0.1)
    y = gen.force_ties(d["y"], ties) if ties else d["y"]
    rng = np.random.default_rng(seed + 77)
    vals = rng.normal(0.0, 1.0, d["rows"].size) if valued else None
    eta = rng.normal(0.0, 0.5, n)
    prob = ss.Problem(model, y, d["status"], d["col_ptr"], d["rows"], vals, DEV)
    prob.set_eta(eta)
    return prob, d, y, vals, eta


def _noalloc(prob, j, out):
    return ss.load().ss_grad_hess_noalloc(
        prob.model, prob.n, prob.p, int(j), ss._p(prob.e), ss._p(prob.d8), ss._p(prob.d32),
        ss._p(prob.w_comp), ss._p(prob.g_end), ss._p(prob.col_ptr), ss._p(prob.rows_sorted),
        ss._p(prob.vals_sorted), ss._p(prob.chunk_ptr), ss._p(prob.c), ss._p(out),
        ss._stream(prob.device))


@pytest.mark.parametrize("model", ["cox", "fg"])
def test_noalloc_matches_workspace_entry_point(model):
    # first call: 3 columns at N = 300,000 (147 tiles of 2048, a ragged
    # tail, tie runs across tile boundaries); second call: a smaller
    # problem (N = 5,000) on the same device array
    for n, p, seed, ties, valued in ((300_001, 3, 5, 20_000, False), (5_000, 2, 6, 0, True)):
        prob, d, y, vals, eta = _case(model, n, p, seed, ties, valued)
        pr = oscan.Prepared(model, y, d["status"])
        for j in range(p):
            want = prob.grad_hess(j).cpu().numpy()
            out = torch.full((4,), np.nan, dtype=torch.float64, device=DEV)
            assert _noalloc(prob, j, out) == ss.SS_OK
            got = out.cpu().numpy()
            assert got[3] == 0.0, "a bounded wait gave up"
            x = gen.dense_column(n, d["col_ptr"], d["rows"], vals, j)
            orc = pr.coordinate(eta, x)
            # the workspace entry point and the oracle both bound the result
            for k, scale in ((0, orc["scale_g1"]), (1, orc["scale_g2"]), (2, orc["scale_L"])):
                assert abs(got[k] - want[k]) <= TOL * scale, (model, n, j, k, got[k], want[k])
                assert abs(got[k] - orc[("g1", "g2", "L")[k]]) <= TOL * scale, (model, n, j, k)
        assert prob.workspace_error() == 0


def test_noalloc_rejects_bad_arguments():
    prob, d, y, vals, eta = _case("cox", 3000, 2, 9, 0, False)
    lib = ss.load()
    out = torch.zeros(4, dtype=torch.float64, device=DEV)
    args = [ss._p(prob.e), ss._p(prob.d8), ss._p(prob.d32), None, None, ss._p(prob.col_ptr),
            ss._p(prob.rows_sorted), None, ss._p(prob.chunk_ptr), ss._p(prob.c), ss._p(out),
            ss._stream(prob.device)]
    too_big = (1 << 25) + 1
    assert lib.ss_grad_hess_noalloc(ss.COX, too_big, prob.p, 0, *args) == ss.SS_EINVAL
    assert lib.ss_grad_hess_noalloc(ss.COX, prob.n, prob.p, 2, *args) == ss.SS_EINVAL
    assert lib.ss_grad_hess_noalloc(7, prob.n, prob.p, 0, *args) == ss.SS_EUNSUPPORTED
    # Fine-Gray without its weight arrays
    assert lib.ss_grad_hess_noalloc(ss.FINE_GRAY, prob.n, prob.p, 0, *args) == ss.SS_EINVAL
    assert lib.ss_noalloc_scratch_bytes() >= lib.ss_workspace_bytes(ss.COX, 1 << 25)
