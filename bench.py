#!/usr/bin/env python3
"""Throughput of the Cox / Fine-Gray coordinate-descent hot path on one GPU.

A step is one cyclic-coordinate-descent sweep over all P coordinates of the
l1-regularised Cox model followed by one sweep of the l1-regularised
Fine-Gray model (gamma = sqrt(2)), each coordinate being the sparse update
of X beta, the fused scan -> transform -> reduce for g' and g'', and the
coordinate update, all on the GPU.  Data: the paper's synthetic design at
its largest size, N = 1e6 subjects, P = 1000 indicator covariates at 5%
density (seed 0), already prepared and resident in HBM when timing starts.

One JSON line is printed.  Besides the throughput it carries
  roofline      the fused Cox kernel at N = 2^27 (its HBM-bound size), timed
                with HIP events on its own stream;
  cpu_baseline  the FP64 oracle (serial C scan) on a bounded sample, one
                thread; cpu_baseline_all_cores: the same scan on every host
                core, coordinates in parallel;
  roofline_fg   the Fine-Gray gradient and Hessian at N = 2^27;
  precision     FP32 storage of e in the same single-pass kernel at N = 2^27;
  context       our fused kernel at N = 1e5 next to the paper's GV100 time;
  paper_sizes   the fused kernel at N = 1e5 ... 1e6 and the sweeps at
                N = 1e5 (latency-bound sizes, not an HBM fraction);
  eta_gradient  the full gradient in eta at N = 1e6 and 2^27, and X' times
                it formed in sorted order (no permutation);
  fit           the l1 fits of both models to convergence at N = 1e6, with
                the largest violation of the optimality conditions;
  cv            10-fold x 10-repetition cross-validation (100 replicates) at
                N = 1e5, P = 1000, Cox and Fine-Gray: one l1 sweep of every
                replicate in one launch, next to the replicates as problems
                of their own swept on 1, 2, 4 or 8 streams.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FUSED_SRC = os.path.join(ROOT, "paper_2204_08183_amd", "csrc", "fused.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_cox_n134217728_traffic.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=1000)
    ap.add_argument("--density", type=float, default=0.05)
    ap.add_argument("--roof-n", type=int, default=1 << 27)
    ap.add_argument("--roof-reps", type=int, default=20)
    ap.add_argument("--cpu-coords", type=int, default=400,
                    help="coordinates per model in the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-context", action="store_true")
    ap.add_argument("--no-cv", action="store_true")
    ap.add_argument("--record-traffic", nargs=4, metavar="CSV",
                    help="write the roofline kernel's calibrated traffic from rocprofv3 "
                         "--pmc CSVs: FETCH_SIZE, WRITE_SIZE (of --only roofline), "
                         "FETCH_SIZE, WRITE_SIZE (of --copy-calibration)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--only", choices=["cv", "eta_gradient", "fit", "precision", "roofline",
                                       "roofline_fg"],
                    help="only run one of the secondary measurements (for profiling)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash():
    with open(FUSED_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def event_time_us(torch, fn, reps):
    """Average device time per call of fn() between two events on the
    current stream (the stream the library launches on)."""
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def tuned(prob, **kw):
    """Runs the library's autotuner on a problem (launch shapes only; the
    results do not depend on them) and returns what it picked."""
    res = prob.autotune(**kw)
    out = {}
    if res["grad_hess"]:
        out["grad_hess_ipt"] = res["grad_hess"][0]
        out["grad_hess_us_by_ipt"] = dict(zip(("4", "8", "16", "32"),
                                              [round(t, 2) for t in res["grad_hess"][1]]))
    if res.get("sweep"):
        out["sweep_shape"] = res["sweep"][0]
        out["sweep_us_by_shape"] = dict(zip(("256x16", "512x8", "256x8", "512x16"),
                                            [round(t, 1) for t in res["sweep"][1]]))
    return out


def roofline(torch, ss, gen, n, reps):
    log("roofline workload: uniform(1,2) tuple, dense valued column, N=%d" % n)
    u = gen.uniform_tuple_data(1, n)
    prob = ss.Problem("cox", u["y"], u["status"], u["col_ptr"], u["rows"], u["vals"],
                      "cuda:0")
    prob.set_eta(u["eta"])
    nnz = int(u["rows"].size)
    del u
    tune = tuned(prob, j=0, reps=5, sweep=False)
    out = torch.empty(3, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        prob.grad_hess(0, out=out)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda: prob.grad_hess(0, out=out), reps)
    # algorithmic bytes: e (8) and the event count (1) per subject, plus the
    # column's row index (4) and value (8) per non-zero
    algo = n * (8 + 1) + nnz * (4 + 8)
    achieved = algo / (us * 1e-6) / 1e9
    ipt = ss.tune_get(ss.TUNE_GRAD_HESS, "cox", "f64", True, n)  # the tile shape launched
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_sha") == kernel_hash() and t.get("n") == n and t.get("ipt") == ipt:
            traffic = t.get("bytes_per_launch")
    err = prob.workspace_error()
    copy_gbs = copy_peak_gbs(torch)
    del prob
    torch.cuda.empty_cache()
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_fused<256,%d,cox,vals>" % ipt, "n": n, "nnz": nnz,
            "algo_bytes_per_launch": algo, "avg_us": round(us, 2), "reps": reps,
            "copy_peak_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
            "wait_errors": err, "tuning": tune}


def roofline_fg(torch, ss, gen, n, reps):
    """The Fine-Gray gradient and Hessian (a4) at N = 2^27 on the Sec. 3.2
    competing-risks design with one 0/1 column at 5% density.  Algorithmic
    bytes per coordinate: e, w and G(Y) (8 each) and the event count (1) per
    subject, plus 4 per non-zero.  Two ways to run it:
      standalone        ss_grad_hess: a totals pass (sum e w x^m), then the
                        scan pass (the totals are needed before the scan);
      in_sweep          one coordinate inside a sweep that launches per
                        coordinate (the size is above the persistent
                        sweep's): one launch, the totals carried in closed
                        form from the previous coordinate, plus that
                        coordinate's update of X beta."""
    import numpy as np
    p = 4
    log("Fine-Gray at N=%d: Sec. 3.2 design, %d 0/1 columns at 5%%" % (n, p))
    d = gen.fg_data(3, n, p, 0.05)
    eta = np.random.default_rng(5).normal(0.0, 0.5, n)
    prob = ss.Problem("fg", d["y"], d["status"], d["col_ptr"], d["rows"], None, "cuda:0")
    prob.set_eta(eta)
    nnz = int(d["col_ptr"][1] - d["col_ptr"][0])
    nnz_all = int(d["rows"].size)
    del d, eta
    tune = tuned(prob, j=0, reps=3, sweep=False)
    out = torch.empty(3, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        prob.grad_hess(0, out=out)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda: prob.grad_hess(0, out=out), reps)
    algo = n * (3 * 8 + 1) + nnz * 4
    res = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "n": n, "nnz": nnz,
           "algo_bytes_per_coordinate": algo, "tuning": tune,
           "standalone": {"avg_us": round(us, 2), "launches": 2,
                          "achieved": round(algo / (us * 1e-6) / 1e9, 1),
                          "frac": round(algo / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}
    # the per-coordinate path of a sweep over the p columns: one launch each
    # (the first also runs the totals pass)
    os.environ["SURVSCAN_SWEEP"] = "launch"
    try:
        prob.sweep("l1", 1.0)
        torch.cuda.synchronize()
        us_sw = event_time_us(torch, lambda: prob.sweep("l1", 1.0), 3)
    finally:
        del os.environ["SURVSCAN_SWEEP"]
    per = us_sw / p
    # per coordinate: the scan pass plus the update of the previous column
    # (28 bytes per non-zero) and the next column's indices for the carry
    algo_c = n * (3 * 8 + 1) + (nnz_all // p) * (4 + 4 + 28)
    res["in_sweep"] = {"avg_us_per_coordinate": round(per, 2), "launches_per_coordinate": 1,
                       "p": p, "achieved": round(algo_c / (per * 1e-6) / 1e9, 1),
                       "frac": round(algo_c / (per * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                       "algo_bytes_per_coordinate": algo_c}
    res["wait_errors"] = prob.workspace_error()
    del prob
    torch.cuda.empty_cache()
    return res


def record_traffic(paths, n):
    """Writes the calibrated per-launch HBM traffic of the roofline kernel
    from four rocprofv3 --pmc CSV files (FETCH_SIZE and WRITE_SIZE of
    `bench.py --only roofline`, then of `bench.py --copy-calibration`)."""
    import csv
    import statistics

    def values(path, pick):
        out = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if pick(r["Kernel_Name"]):
                    out.append(float(r["Counter_Value"]))
        return out

    fetch_p, write_p, cfetch_p, cwrite_p = paths
    ipt = 16
    with open(fetch_p) as f:
        names = {r["Kernel_Name"] for r in csv.DictReader(f) if "k_fused<256" in r["Kernel_Name"]}
    # the roofline kernel: Cox, valued column, FP64, the most launched shape
    counts = {}
    for nm in names:
        if ", 0, true, false, false, double, false>" in nm:
            counts[nm] = len(values(fetch_p, lambda k, nm=nm: k == nm))
    name = max(counts, key=counts.get)
    ipt = int(name.split("k_fused<256, ")[1].split(",")[0])
    fetch = statistics.median(values(fetch_p, lambda k: k == name))
    write = statistics.median(values(write_p, lambda k: k == name))
    copy = lambda k: "copyBuffer" in k  # noqa: E731
    cf = statistics.median(values(cfetch_p, copy))
    cw = statistics.median(values(cwrite_p, copy))
    gib_kib = (1 << 27) * 8 / 1024.0  # the calibration copy: 1 GiB read, 1 GiB written
    fs, ws = gib_kib / cf, gib_kib / cw
    rec = {"kernel": "k_fused<256,%d,cox,vals>" % ipt, "n": n, "ipt": ipt,
           "kernel_sha": kernel_hash(), "fetch_kib_raw_median": fetch,
           "write_kib_raw_median": write, "fetch_scale": round(fs, 5),
           "write_scale": round(ws, 5), "fetch_bytes_per_launch": int(fetch * 1024 * fs),
           "write_bytes_per_launch": int(write * 1024 * ws),
           "bytes_per_launch": int(fetch * 1024 * fs + write * 1024 * ws),
           "algo_bytes_per_launch": n * (8 + 1) + n * (4 + 8)}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def precision(torch, ss, gen, n, reps):
    """FP32 storage of e in the single-pass fused kernel against the FP64
    kernel at N = 2^27, on a 0/1 column at 5% density (the Sec. 3.2
    design's column; e ~ U(1,2), delta ~ Bernoulli(0.5)) and on the dense
    valued column of the roofline workload.  Algorithmic bytes per launch:
    e (8 or 4) and the event count (1) per subject, plus 4 per non-zero
    (+ 8 for a value)."""
    res = {}
    for label, density, valued in (("01_col_5pct", 0.05, False), ("dense_valued", 1.0, True)):
        u = gen.uniform_tuple_data(1, n, density)
        prob = ss.Problem("cox", u["y"], u["status"], u["col_ptr"], u["rows"],
                          u["vals"] if valued else None, "cuda:0")
        prob.set_eta(u["eta"])
        nnz = int(u["rows"].size)
        del u
        e32, _ = prob.make_e32()
        out = torch.empty(3, dtype=torch.float64, device="cuda:0")
        col = nnz * (4 + (8 if valued else 0))
        row = {"tuned_ipt": {}}
        for storage in ("f64", "f32", "f32x64"):
            t = tuned(prob, j=0, reps=5, sweep=False, storage=storage, e32=e32)
            row["tuned_ipt"][storage] = t["grad_hess_ipt"]
        for name, fn, se in (("f64", lambda: prob.grad_hess(0, out=out), 8),
                             ("f32_storage_f64_sums",
                              lambda: prob.grad_hess_f32(0, e32, "f64", out), 4),
                             ("f32_storage_f32_tile_sums_f64_carry",
                              lambda: prob.grad_hess_f32(0, e32, "f32x64", out), 4)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            us = event_time_us(torch, fn, reps)
            algo = n * (se + 1) + col
            row[name] = {"avg_us": round(us, 2), "algo_bytes_per_launch": algo,
                         "achieved_gbs": round(algo / (us * 1e-6) / 1e9, 1),
                         "frac": round(algo / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        row["wait_errors"] = prob.workspace_error()
        res[label] = row
        del prob, e32
        torch.cuda.empty_cache()
    return res


def copy_peak_gbs(torch):
    """Measured device-to-device copy rate (read + write bytes), 1 GiB each way."""
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda: b.copy_(a), 10)
    nbytes = 2 * a.numel() * 8
    del a, b
    torch.cuda.empty_cache()
    return nbytes / (us * 1e-6) / 1e9


def context(torch, ss, gen):
    """Our fused kernel at the paper's Table 1 size (N = 1e5, U(1,2))."""
    u = gen.uniform_tuple_data(2, 100_000)
    prob = ss.Problem("cox", u["y"], u["status"], u["col_ptr"], u["rows"], u["vals"],
                      "cuda:0")
    prob.set_eta(u["eta"])
    tune = tuned(prob, j=0, reps=20, sweep=False)
    out = torch.empty(3, dtype=torch.float64, device="cuda:0")
    for _ in range(5):
        prob.grad_hess(0, out=out)
    torch.cuda.synchronize()
    us = event_time_us(torch, lambda: prob.grad_hess(0, out=out), 200)
    return {"fused_us_n1e5_ours_back_to_back": round(us, 2),
            "fused_us_n1e5_paper_gv100": 5.2, "tuned_ipt": tune["grad_hess_ipt"],
            "note": "paper Table 1, steps (2)-(4) fused, N=1e5, Uniform(1,2); other GPU"}


def paper_sizes(torch, ss, gen):
    """The paper's own sizes, latency-bound and cache-resident (not an HBM
    fraction): the fused kernel on Uniform(1,2) tuples at N = 1e5 ... 1e6
    (Table 1 workload), and the l1 sweeps of the Sec. 3.2 designs at
    N = 1e5 (the headline covers N = 1e6)."""
    fused = {}
    for n in (100_000, 200_000, 500_000, 1_000_000):
        u = gen.uniform_tuple_data(2, n)
        prob = ss.Problem("cox", u["y"], u["status"], u["col_ptr"], u["rows"], u["vals"],
                          "cuda:0")
        prob.set_eta(u["eta"])
        tuned(prob, j=0, reps=20, sweep=False)
        out = torch.empty(3, dtype=torch.float64, device="cuda:0")
        for _ in range(5):
            prob.grad_hess(0, out=out)
        torch.cuda.synchronize()
        fused[str(n)] = round(event_time_us(torch, lambda: prob.grad_hess(0, out=out), 100), 2)
    sweeps = {}
    gamma = math.sqrt(2.0)
    for model in ("cox", "fg"):
        d = gen.cox_data(0, 100_000, 1000, 0.05) if model == "cox" else \
            gen.fg_data(0, 100_000, 1000, 0.05)
        prob = ss.Problem(model, d["y"], d["status"], d["col_ptr"], d["rows"], None, "cuda:0")
        tuned(prob, j=0, reps=10, sweep=True, penalty="l1", lam=gamma)
        prob.sweep("l1", gamma)
        torch.cuda.synchronize()
        us = event_time_us(torch, lambda: prob.sweep("l1", gamma), 5)
        sweeps[model] = {"us_per_coordinate": round(us / d["p"], 3),
                         "coords_per_s": round(d["p"] / (us * 1e-6), 1)}
    return {"fused_us_uniform_tuple_by_n": fused,
            "l1_sweep_n1e5_p1000": sweeps,
            "note": "back-to-back launches timed with HIP events; latency-bound sizes"}


def eta_gradient(torch, ss, gen):
    """The full gradient in eta (ss_eta_gradient, Cox) on the Uniform(1,2)
    tuple workload: time per call and algorithmic bandwidth, counting each
    input read once and the output written once (perm 4, status 1, eta 8,
    e 8, d 1, grad 8 = 30 bytes per subject)."""
    res = {}
    for n in (1_000_000, 1 << 27):
        u = gen.uniform_tuple_data(1, n)
        prob = ss.Problem("cox", u["y"], u["status"], u["col_ptr"], u["rows"], u["vals"],
                          "cuda:0")
        prob.set_eta(u["eta"])
        del u
        grad = torch.empty(n, dtype=torch.float64, device="cuda:0")
        ll = torch.empty(1, dtype=torch.float64, device="cuda:0")
        prob.eta_gradient(grad, ll)
        torch.cuda.synchronize()
        us = event_time_us(torch, lambda: prob.eta_gradient(grad, ll), 10)
        gb = torch.empty(1, dtype=torch.float64, device="cuda:0")
        prob.beta_gradient(gb, None, ll)
        torch.cuda.synchronize()
        us_b = event_time_us(torch, lambda: prob.beta_gradient(gb, None, ll), 10)
        # X' (dl/deta) of the dense column: status, eta, e, d per subject
        # (18 bytes) and the column's index and value per non-zero (12)
        algo_b = 30.0 * n
        res[str(n)] = {"us": round(us, 1), "algo_gbs": round(30.0 * n / (us * 1e3), 1),
                       "frac_of_hbm_peak": round(30.0 * n / (us * 1e3) / HBM_PEAK_GBS, 4),
                       "beta_gradient_us": round(us_b, 1),
                       "beta_gradient_algo_gbs": round(algo_b / (us_b * 1e3), 1),
                       "beta_gradient_frac_of_hbm_peak": round(algo_b / (us_b * 1e3) /
                                                               HBM_PEAK_GBS, 4)}
        del prob, grad
        torch.cuda.empty_cache()
    return res


def subset_problem(ss, d, keep, model):
    """The data set of the subjects with keep != 0 (CSC columns restricted
    to them, rows renumbered), prepared as a problem of its own."""
    import numpy as np
    keep = np.asarray(keep) != 0
    idx = np.nonzero(keep)[0]
    new = np.full(keep.size, -1, dtype=np.int64)
    new[idx] = np.arange(idx.size)
    rows = np.asarray(d["rows"], dtype=np.int64)
    m = keep[rows]
    csum = np.concatenate([[0], np.cumsum(m, dtype=np.int64)])
    cp = csum[np.asarray(d["col_ptr"], dtype=np.int64)]
    return ss.Problem(model, d["y"][idx], d["status"][idx], cp, new[rows[m]].astype(np.int32),
                      None, "cuda:0")


def cross_validation(torch, ss, gen):
    """Sec. 3.3 design at its smallest size: 10 x 10 cross-validation of the
    l1 model (gamma = sqrt 2) at N = 1e5, P = 1000, Cox and Fine-Gray; one
    sweep of all 100 replicates in one launch, next to the paper's way
    (Sec. 2.8): every replicate a problem of its own (its training subjects),
    their single-problem sweeps spread over s = 1, 2, 4, 8 streams."""
    n, p, reps = 100_000, 1000, 100
    gamma = math.sqrt(2.0)
    train = gen.cv_folds(0, n, 10, 10)
    out = {"workload": "10-fold x 10 cross-validation, l1, N=1e5, P=1000, 0.05 density",
           "replicates": reps}
    for model in ("cox", "fg"):
        d = gen.cox_data(0, n, p, 0.05) if model == "cox" else gen.fg_data(0, n, p, 0.05)
        prob = ss.Problem(model, d["y"], d["status"], d["col_ptr"], d["rows"], None, "cuda:0")
        cvp = ss.CrossValidation(prob, train)
        cvp.sweep("l1", gamma)
        torch.cuda.synchronize()
        us_cv = event_time_us(torch, lambda: cvp.sweep("l1", gamma), 3)
        err = cvp.workspace_error()
        del cvp, prob
        torch.cuda.empty_cache()
        # the multi-stream baseline
        probs = [subset_problem(ss, d, train[r], model) for r in range(reps)]
        for pr in probs:
            pr.sweep("l1", gamma)
        torch.cuda.synchronize()
        streams_ms = {}
        for ns in (1, 2, 4, 8):
            streams = [torch.cuda.Stream() for _ in range(ns)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r, pr in enumerate(probs):
                with torch.cuda.stream(streams[r % ns]):
                    pr.sweep("l1", gamma)
            torch.cuda.synchronize()
            streams_ms[str(ns)] = round((time.perf_counter() - t0) * 1e3, 3)
        # the same with one launch per coordinate (the sweep as the paper's
        # CPU-driven loop launches it; launches of different streams can
        # overlap, the cooperative persistent sweep above cannot)
        launch_ms = {}
        os.environ["SURVSCAN_SWEEP"] = "launch"
        try:
            for pr in probs:
                pr.sweep("l1", gamma)
            for ns in (1, 2, 4, 8):
                streams = [torch.cuda.Stream() for _ in range(ns)]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for r, pr in enumerate(probs):
                    with torch.cuda.stream(streams[r % ns]):
                        pr.sweep("l1", gamma)
                torch.cuda.synchronize()
                launch_ms[str(ns)] = round((time.perf_counter() - t0) * 1e3, 3)
        finally:
            del os.environ["SURVSCAN_SWEEP"]
        err += sum(pr.workspace_error() for pr in probs)
        best = min(min(streams_ms.values()), min(launch_ms.values()))
        out[model] = {"sweep_ms_all_replicates_one_launch": round(us_cv / 1e3, 3),
                      "replicate_coords_per_s": round(reps * p / (us_cv * 1e-6), 1),
                      "multi_stream_sweep_ms_by_streams": streams_ms,
                      "multi_stream_per_coordinate_launches_ms_by_streams": launch_ms,
                      "speedup_one_launch_vs_best_multi_stream": round(best / (us_cv / 1e3), 2),
                      "wait_errors": err}
        del probs
        torch.cuda.empty_cache()
    return out


def fit_to_convergence(torch, ss, cox, fg, tol=1e-15):
    """Sec. 3.2 / Fig. 5 at the paper's largest size: the l1 fit (gamma =
    sqrt 2) of both models from beta = 0 to convergence (relative change of
    the penalised log-likelihood below `tol` over a sweep), whole sweeps on
    the GPU; then the largest violation of the optimality conditions over
    all coordinates, in units of |g''_j| (what is left of a Newton step)."""
    import numpy as np
    gamma = math.sqrt(2.0)
    res = {}
    for model, d in (("cox", cox), ("fg", fg)):
        prob = ss.Problem(model, d["y"], d["status"], d["col_ptr"], d["rows"], None,
                          "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps = prob.fit("l1", gamma, max_sweeps=400, tol=tol)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        beta = prob.beta.cpu().numpy()
        g = torch.empty((d["p"], 3), dtype=torch.float64, device="cuda:0")
        for j in range(d["p"]):
            prob.grad_hess(j, out=g[j])
        g = g.cpu().numpy()
        zero = beta == 0.0
        viol = np.where(zero, np.abs(g[:, 0]) - gamma,
                        np.abs(g[:, 0] - gamma * np.sign(beta))) / np.abs(g[:, 1])
        res[model] = {"sweeps": int(sweeps), "seconds": round(secs, 4),
                      "nonzero_coefficients": int(np.count_nonzero(~zero)),
                      "kkt_max_violation_over_abs_g2": float(np.max(viol)),
                      "wait_errors": prob.workspace_error()}
        del prob
        torch.cuda.empty_cache()
    return res


def cpu_baseline(gen, cox, fg, coords):
    """The oracle as it stands: serial C scan per coordinate + CCD update."""
    import numpy as np

    from oracle import ccd as occd, scan as oscan
    total = 0
    t0 = time.perf_counter()
    for model, d in (("cox", cox), ("fg", fg)):
        pr = oscan.Prepared(model, d["y"], d["status"])
        eta = np.zeros(d["n"])
        beta = np.zeros(d["p"])
        delta = np.ones(d["p"])
        for j in range(min(coords, d["p"])):
            x = gen.dense_column(d["n"], d["col_ptr"], d["rows"], None, j)
            r = pr.coordinate(eta, x)
            beta[j], delta[j], step = occd.update(r["g1"], r["g2"], beta[j], delta[j],
                                                  occd.PENALTY_L1, math.sqrt(2.0))
            if step != 0.0:
                eta = eta + step * x
            total += 1
    dt = time.perf_counter() - t0
    return {"value": round(total / dt, 2), "unit": "coords/s", "cores": 1, "kind": "oracle",
            "sample": "first %d coordinates of one l1 CCD sweep (gamma=sqrt 2) on each of the "
                      "Cox and Fine-Gray N=%d P=%d data sets, from beta=0; serial C scan with "
                      "compensated sums, single thread; %.1f s" % (coords, cox["n"], cox["p"],
                                                                  dt)}


def cpu_baseline_all_cores(gen, cox, coords_per_thread=60):
    """The same oracle scan on all host cores: independent coordinates at
    fixed beta = 0 (Cox, N = 1e6), one C call per coordinate per thread
    (ctypes releases the interpreter lock during the call)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle import scan as oscan
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else \
        (os.cpu_count() or 1)
    pr = oscan.Prepared("cox", cox["y"], cox["status"])
    eta_s = np.zeros(cox["n"])
    total = min(cox["p"], threads * coords_per_thread)
    cols = [np.ascontiguousarray(
        gen.dense_column(cox["n"], cox["col_ptr"], cox["rows"], None, j)[pr.order])
        for j in range(total)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda x: pr.coordinate_sorted(eta_s, x), cols))
    dt = time.perf_counter() - t0
    return {"value": round(total / dt, 2), "unit": "coords/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d coordinates of the Cox N=%d P=%d data set at beta=0 (gradient and "
                      "Hessian only, no update), spread over %d threads; %.1f s"
                      % (total, cox["n"], cox["p"], threads, dt)}


def host_cpu():
    """The host the CPU baselines ran on: its CPU model and os.cpu_count()."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count()}


def copy_calibration(torch):
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    if args.record_traffic:
        record_traffic(args.record_traffic, args.roof_n)
        return

    import numpy as np  # noqa: F401
    import torch

    import gen
    from paper_2204_08183_amd import survscan as ss

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ss.load()
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.only == "cv":
        print(json.dumps({"cv": cross_validation(torch, ss, gen)}), flush=True)
        return
    if args.only == "roofline":
        print(json.dumps({"roofline": roofline(torch, ss, gen, args.roof_n, args.roof_reps)}),
              flush=True)
        return
    if args.only == "roofline_fg":
        print(json.dumps({"roofline_fg": roofline_fg(torch, ss, gen, args.roof_n,
                                                     args.roof_reps)}), flush=True)
        return
    if args.only == "precision":
        print(json.dumps({"precision": precision(torch, ss, gen, args.roof_n, args.roof_reps)}),
              flush=True)
        return
    if args.only == "eta_gradient":
        print(json.dumps({"eta_gradient": eta_gradient(torch, ss, gen)}), flush=True)
        return

    log("generating Cox and Fine-Gray data N=%d P=%d density=%g" % (args.n, args.p,
                                                                   args.density))
    cox = gen.cox_data(0, args.n, args.p, args.density)
    fg = gen.fg_data(0, args.n, args.p, args.density)
    if args.only == "fit":
        print(json.dumps({"fit": fit_to_convergence(torch, ss, cox, fg)}), flush=True)
        return
    t0 = time.perf_counter()
    pc = ss.Problem("cox", cox["y"], cox["status"], cox["col_ptr"], cox["rows"], None,
                    "cuda:0")
    pf = ss.Problem("fg", fg["y"], fg["status"], fg["col_ptr"], fg["rows"], None, "cuda:0")
    torch.cuda.synchronize()
    prepare_s = time.perf_counter() - t0
    gamma = math.sqrt(2.0)
    log("autotuning launch shapes")
    tuning = {"cox": tuned(pc, j=0, reps=10, sweep=True, penalty="l1", lam=gamma),
              "fg": tuned(pf, j=0, reps=10, sweep=True, penalty="l1", lam=gamma)}

    def step():
        pc.sweep("l1", gamma)
        pf.sweep("l1", gamma)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    coords = 2 * args.p * args.steps
    value = coords / elapsed
    # per-model sweep time (events, after the timed region)
    cox_us = event_time_us(torch, lambda: pc.sweep("l1", gamma), 2)
    fg_us = event_time_us(torch, lambda: pf.sweep("l1", gamma), 2)
    wait_errors = pc.workspace_error() + pf.workspace_error()
    log("step %.3f ms (cox sweep %.3f ms, fg sweep %.3f ms)" % (ms_per_step, cox_us / 1e3,
                                                                 fg_us / 1e3))
    nnz = int(cox["rows"].size)
    del pc, pf
    torch.cuda.empty_cache()

    line = {
        "metric": "CCD coordinate gradient+Hessian evaluations/s (Cox + Fine-Gray, FP64)",
        "value": round(value, 1),
        "unit": "coords/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "l1 CCD sweep, Cox then Fine-Gray, N=%d subjects, P=%d indicator "
                        "covariates at %g density, gamma=sqrt(2) (paper Sec. 3.2 design)"
                        % (args.n, args.p, args.density),
            "n": args.n, "p": args.p, "density": args.density, "nnz_cox": nnz,
            "penalty": "l1", "gamma": gamma, "seed": 0,
        },
        "rows_per_s": round(value * args.n, 1),
        "cox_sweep_ms": round(cox_us / 1e3, 4),
        "fg_sweep_ms": round(fg_us / 1e3, 4),
        "us_per_coordinate_cox": round(cox_us / args.p, 3),
        "us_per_coordinate_fg": round(fg_us / args.p, 3),
        "prepare_s_both_models": round(prepare_s, 3),
        "wait_errors": wait_errors,
        "tuning": tuning,
    }
    if not args.no_roofline:
        line["roofline"] = roofline(torch, ss, gen, args.roof_n, args.roof_reps)
    if not args.no_roofline:
        line["roofline_fg"] = roofline_fg(torch, ss, gen, args.roof_n, args.roof_reps)
        log("FP32 storage of e at N=%d" % args.roof_n)
        line["precision"] = precision(torch, ss, gen, args.roof_n, args.roof_reps)
    if not args.no_context:
        line["context"] = context(torch, ss, gen)
    if not args.no_context:
        log("paper sizes: fused N=1e5..1e6, sweeps at N=1e5")
        line["paper_sizes"] = paper_sizes(torch, ss, gen)
    if not args.no_context:
        log("gradient in eta: N=1e6 and 2^27")
        line["eta_gradient"] = eta_gradient(torch, ss, gen)
    if not args.no_cv:
        log("cross-validation: 100 replicates, N=1e5, P=1000")
        line["cv"] = cross_validation(torch, ss, gen)
    if not args.no_context:
        log("l1 fits to convergence, N=%d, P=%d" % (args.n, args.p))
        line["fit"] = fit_to_convergence(torch, ss, cox, fg)
    if not args.no_cpu:
        log("cpu baseline (oracle) on %d coordinates per model" % args.cpu_coords)
        line["cpu_baseline"] = cpu_baseline(gen, cox, fg, args.cpu_coords)
        if "fit" in line:
            # the oracle's coordinate rate times the fits' coordinate count
            cps = line["cpu_baseline"]["value"]
            for m in ("cox", "fg"):
                f = line["fit"][m]
                f["oracle_seconds_extrapolated_1_core"] = round(f["sweeps"] * args.p / cps, 1)
        log("cpu baseline (oracle) on all host cores")
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(gen, cox)
        host = host_cpu()
        line["cpu_baseline"].update(host)
        line["cpu_baseline_all_cores"].update(host)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
