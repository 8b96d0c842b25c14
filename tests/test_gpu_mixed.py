"""GPU: the FP32-storage paths (ss_exp_f32; ss_grad_hess_mixed, the
deterministic reduce-then-scan of the accuracy study; ss_grad_hess_f32, FP32
e inside the single-pass fused kernel) against the FP64 oracle.

e is kept as exp(eta - m) in FP32 (m = max eta) and the scans and sums run in
plain FP32, compensated FP32 (two-sum), FP32 inside tiles with an FP64 carry
between tiles ("f32x64"), or FP64.  Checks:
  * FP64 accumulation against the oracle evaluated on the same FP32-rounded
    e: the FP64 bound of the parity tests (1e-10, condition-scaled);
  * both FP32 accumulations against the oracle on the original FP64 e: the
    FP32 bound 1e-5, condition-scaled (storage rounding plus accumulation);
  * the shift: g' and g'' do not move, sum d log S0 moves by m sum d.
test_mixed_report prints the maximum and median condition-scaled errors over
many coordinates for each accumulation (the M5 measurement).
"""
import time

import numpy as np
import pytest

import gen
from oracle import prep as oprep, scan as oscan

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2204_08183_amd import survscan as ss  # noqa: E402

from test_gpu_parity import make_case, gpu_problem, xcol  # noqa: E402

DEV = "cuda:0"
TOL64 = 1e-10
TOL32 = 1e-5


def rounded_eta(prob, e32):
    """Subject-order eta whose exp is the FP32 e the GPU holds (shifted)."""
    e_sorted = e32.double().cpu().numpy()
    perm = prob.perm.cpu().numpy()
    eta = np.empty(prob.n)
    eta[perm] = np.log(e_sorted)
    return eta


def scaled_errors(got, want, shift_sum=0.0):
    g1, g2, L = (float(v) for v in got)
    return (abs(g1 - want["g1"]) / want["scale_g1"],
            abs(g2 - want["g2"]) / want["scale_g2"],
            abs(L + shift_sum - want["L"]) / max(want["scale_L"], 1e-300))


def assert_within(got, want, tol, shift_sum=0.0, what=""):
    """|got - want| <= tol * scale for g', g'' and sum d log S0 (no division,
    so that degenerate cases with a zero scale must match exactly)."""
    g1, g2, L = (float(v) for v in got)
    assert abs(g1 - want["g1"]) <= tol * want["scale_g1"] + 1e-300, (what, g1, want["g1"])
    assert abs(g2 - want["g2"]) <= tol * want["scale_g2"] + 1e-300, (what, g2, want["g2"])
    assert abs(L + shift_sum - want["L"]) <= tol * want["scale_L"] + 1e-300, \
        (what, L + shift_sum, want["L"])


CASES = [("cox", 20000, 6, 0, 30, False), ("cox", 60001, 4, 1, 0, True),
         ("fg", 20000, 6, 2, 30, False), ("fg", 60001, 4, 3, 0, True)]


@pytest.mark.parametrize("model,n,p,seed,ties,valued", CASES)
def test_mixed_matches_oracle(model, n, p, seed, ties, valued):
    c = make_case(model, n, p, seed, ties, 0.1, valued)
    prob = gpu_problem(model, c)
    e32, shift = prob.make_e32()
    m = float(shift.cpu()[0])
    assert m == pytest.approx(float(np.max(c["eta"])), abs=0.0)
    nev = float(np.sum(oprep.event_indicator(model, c["status"])))
    pr = oscan.Prepared(model, c["y"], c["status"])
    eta_r = rounded_eta(prob, e32)
    for j in range(p):
        x = xcol(c, j)
        want_r = pr.coordinate(eta_r, x)       # same FP32 inputs, FP64 arithmetic
        want = pr.coordinate(c["eta"], x)      # the FP64 definition
        got = prob.grad_hess_mixed(j, e32, "f64").cpu().numpy()
        e1, e2, eL = scaled_errors(got, want_r)
        assert max(e1, e2, eL) <= TOL64, (model, n, j, "f64", e1, e2, eL)
        for acc in ("f32", "f32c", "f32x64"):
            got = prob.grad_hess_mixed(j, e32, acc).cpu().numpy()
            e1, e2, eL = scaled_errors(got, want, m * nev)
            assert max(e1, e2, eL) <= TOL32, (model, n, j, acc, e1, e2, eL)


F32_CASES = CASES + [
    ("cox", 1, 2, 40, 0, False), ("fg", 2, 2, 41, 0, True), ("cox", 2047, 3, 42, 0, False),
    ("fg", 2049, 3, 43, 100, False), ("cox", 100_000, 3, 44, 50, True),
    # 4096-position tiles (above 1.5M), tie runs across their boundaries
    ("cox", 2_000_003, 2, 45, 1500, False), ("fg", 1_900_000, 2, 46, 400_000, True),
]


@pytest.mark.parametrize("model,n,p,seed,ties,valued", F32_CASES)
def test_fused_f32_matches_oracle(model, n, p, seed, ties, valued):
    """Single-pass FP32-storage kernel: with FP64 sums it is the FP64 kernel
    on rounded inputs (1e-10 against the oracle on the same rounded e);
    with FP32 sums inside tiles and the FP64 carry, within the FP32 bound
    of the FP64 definition."""
    c = make_case(model, n, p, seed, ties, 0.1, valued)
    prob = gpu_problem(model, c)
    e32, shift = prob.make_e32()
    m = float(shift.cpu()[0])
    nev = float(np.sum(oprep.event_indicator(model, c["status"])))
    pr = oscan.Prepared(model, c["y"], c["status"])
    eta_r = rounded_eta(prob, e32)
    for j in range(p):
        x = xcol(c, j)
        want_r = pr.coordinate(eta_r, x)
        want = pr.coordinate(c["eta"], x)
        got = prob.grad_hess_f32(j, e32, "f64").cpu().numpy()
        assert_within(got, want_r, TOL64, 0.0, (model, n, j, "f64"))
        got = prob.grad_hess_f32(j, e32, "f32x64").cpu().numpy()
        assert_within(got, want, TOL32, m * nev, (model, n, j, "f32x64"))
    assert prob.workspace_error() == 0


def test_fused_f32_rejects_bad_arguments():
    c = make_case("cox", 3000, 2, 8, 0, 0.2, False)
    prob = gpu_problem("cox", c)
    e32, _ = prob.make_e32()
    out = torch.empty(3, dtype=torch.float64, device=DEV)
    lib = ss.load()

    def call(acc, ptr):
        return lib.ss_grad_hess_f32(ss.COX, acc, prob.n, prob.p, 0, ptr, prob.d8.data_ptr(),
                                    prob.d32.data_ptr(), None, None, prob.col_ptr.data_ptr(),
                                    prob.rows_sorted.data_ptr(), None,
                                    prob.chunk_ptr.data_ptr(), prob.c.data_ptr(),
                                    out.data_ptr(), prob.ws.ptr, prob.ws.nbytes, None)
    assert call(ss.ACC_F32, e32.data_ptr()) == ss.SS_EINVAL
    assert call(ss.ACC_F32_COMP, e32.data_ptr()) == ss.SS_EINVAL
    assert call(ss.ACC_F64, e32.data_ptr() + 4) == ss.SS_EINVAL  # not 16-byte aligned
    assert call(ss.ACC_F64, e32.data_ptr()) == ss.SS_OK


def test_mixed_shift_overflow():
    """eta far above the FP32 exp range: the shift keeps e32 finite."""
    c = make_case("cox", 5000, 3, 7, 0, 0.2, False, eta_shift=500.0)
    prob = gpu_problem("cox", c)
    e32, shift = prob.make_e32()
    assert torch.isfinite(e32).all().item()
    assert float(e32.max().cpu()) == 1.0
    pr = oscan.Prepared("cox", c["y"], c["status"])
    nev = float(np.sum(oprep.event_indicator("cox", c["status"])))
    m = float(shift.cpu()[0])
    for j in range(3):
        want = pr.coordinate(c["eta"], xcol(c, j))
        for acc in ("f32c", "f32x64"):
            got = prob.grad_hess_mixed(j, e32, acc).cpu().numpy()
            assert max(scaled_errors(got, want, m * nev)) <= TOL32


def test_mixed_rejects_bad_accumulation():
    c = make_case("cox", 3000, 2, 8, 0, 0.2, False)
    prob = gpu_problem("cox", c)
    e32, _ = prob.make_e32()
    out = torch.empty(3, dtype=torch.float64, device=DEV)
    rc = ss.load().ss_grad_hess_mixed(ss.COX, 7, prob.n, prob.p, 0, e32.data_ptr(),
                                      prob.d8.data_ptr(), prob.d32.data_ptr(), None, None,
                                      prob.col_ptr.data_ptr(), prob.rows_sorted.data_ptr(),
                                      None, prob.chunk_ptr.data_ptr(), prob.c.data_ptr(),
                                      out.data_ptr(), prob.ws.ptr, prob.ws.nbytes, None)
    assert rc == ss.SS_EINVAL


def _report_config(name, model, c, coords):
    prob = gpu_problem(model, c)
    e32, shift = prob.make_e32()
    m = float(shift.cpu()[0])
    nev = float(np.sum(oprep.event_indicator(model, c["status"])))
    pr = oscan.Prepared(model, c["y"], c["status"])
    errs = {acc: [] for acc in ("f32", "f32c", "f32x64", "f64")}
    for j in coords:
        want = pr.coordinate(c["eta"], xcol(c, j))
        for acc in errs:
            got = prob.grad_hess_mixed(j, e32, acc).cpu().numpy()
            errs[acc].append(scaled_errors(got, want, m * nev)[:2])
    timing = {}
    for acc in errs:
        out = torch.empty(3, dtype=torch.float64, device=DEV)
        prob.grad_hess_mixed(0, e32, acc, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            prob.grad_hess_mixed(0, e32, acc, out)
        torch.cuda.synchronize()
        timing[acc] = (time.perf_counter() - t0) / 20 * 1e6
    fused = {acc: [] for acc in ("f64", "f32x64")}
    for j in coords:
        want = pr.coordinate(c["eta"], xcol(c, j))
        for acc in fused:
            got = prob.grad_hess_f32(j, e32, acc).cpu().numpy()
            fused[acc].append(scaled_errors(got, want, m * nev)[:2])
    ftime = {}
    for acc in fused:
        out = torch.empty(3, dtype=torch.float64, device=DEV)
        prob.grad_hess_f32(0, e32, acc, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            prob.grad_hess_f32(0, e32, acc, out)
        torch.cuda.synchronize()
        ftime[acc] = (time.perf_counter() - t0) / 20 * 1e6
    out64 = torch.empty(3, dtype=torch.float64, device=DEV)
    prob.grad_hess(0, out64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        prob.grad_hess(0, out64)
    torch.cuda.synchronize()
    t64 = (time.perf_counter() - t0) / 20 * 1e6
    lines = []
    for acc, e in errs.items():
        e = np.array(e)
        lines.append("M5 %-34s %-5s g' max %.2e med %.2e | g'' max %.2e med %.2e | %7.1f us"
                     % (name, acc, e[:, 0].max(), np.median(e[:, 0]), e[:, 1].max(),
                        np.median(e[:, 1]), timing[acc]))
    for acc, e in fused.items():
        e = np.array(e)
        lines.append("M5 %-34s fused-f32 %-6s g' max %.2e med %.2e | g'' max %.2e med %.2e | "
                     "%7.1f us" % (name, acc, e[:, 0].max(), np.median(e[:, 0]), e[:, 1].max(),
                                   np.median(e[:, 1]), ftime[acc]))
        errs["fused_" + acc] = fused[acc]
    lines.append("M5 %-34s fp64 fused path                                              "
                 "          | %7.1f us" % (name, t64))
    return lines, errs


def test_mixed_report(capsys):
    """M5: condition-scaled errors against the FP64 oracle over many
    coordinates (M3/M4 designs at N = 1e6, M1 tuple data at N = 1e6)."""
    out = []
    worst = 0.0
    for model in ("cox", "fg"):
        d = gen.cox_data(0, 1_000_000, 100, 0.05) if model == "cox" else \
            gen.fg_data(0, 1_000_000, 100, 0.05)
        rng = np.random.default_rng(11)
        c = {"y": d["y"], "status": d["status"], "col_ptr": d["col_ptr"], "rows": d["rows"],
             "vals": None, "eta": rng.normal(0.0, 0.5, d["n"]), "n": d["n"], "p": d["p"]}
        lines, errs = _report_config("%s N=1e6 P=100 0/1 X" % model, model, c, range(100))
        out += lines
        worst = max(worst, max(np.max(np.array(e)) for e in errs.values()))
    u = gen.uniform_tuple_data(1, 1_000_000)
    c = {"y": u["y"], "status": u["status"], "col_ptr": u["col_ptr"], "rows": u["rows"],
         "vals": u["vals"], "eta": u["eta"], "n": u["n"], "p": 1}
    lines, errs = _report_config("cox N=1e6 Uniform(1,2) tuple", "cox", c, [0])
    out += lines
    worst = max(worst, max(np.max(np.array(e)) for e in errs.values()))
    with capsys.disabled():
        print()
        for line in out:
            print(line)
    assert worst <= TOL32
