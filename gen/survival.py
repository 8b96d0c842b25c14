"""Synthetic data following the paper's designs (Sec. 3.1 and Sec. 3.2).

Random numbers: ``numpy.random.default_rng(seed)``; the draw order of each
function is fixed and documented in its docstring, so a seed reproduces the
same data set anywhere.

Readings of the design where the paper is ambiguous:
  * "5% of the entries chosen uniformly": every entry of X is 1 with
    probability ``density`` independently (a Bernoulli process per column,
    drawn as geometric gaps between consecutive non-zero rows);
  * beta_j ~ N(0,1) x Bernoulli: the text says that on average 80% of the
    coefficients are zero, so a coefficient is non-zero with probability
    ``nonzero_frac`` = 0.2;
  * T_i ~ Exponential(x_i' beta) is read as rate exp(x_i' beta) (a Cox
    model with unit baseline hazard);
  * the censoring mechanism is not given: C_i ~ Exponential(1), independent
    of x;
  * Fine-Gray: the primary event follows the Fine & Gray unit exponential
    mixture with mass 1-p at infinity, P(eps=1|x) = 1 - (1-p)^exp(x'beta1);
    given eps = 1 the time is drawn by inverting F_1(t|x)/P(eps=1|x);
    given eps = 2 it is Exponential(rate exp(x'beta2)); beta2 = -beta1,
    p = 0.5.
"""
import numpy as np


def indicator_design(rng, n, p, density):
    """Sparse 0/1 design in CSC form with rows ascending inside a column.

    Draw order: for j = 0..p-1, geometric gaps until the row index passes n.
    Returns (col_ptr int64[p+1], rows int32[nnz])."""
    cols = []
    for _ in range(p):
        if density >= 1.0:
            cols.append(np.arange(n, dtype=np.int64))
            continue
        if density <= 0.0 or n == 0:
            cols.append(np.zeros(0, dtype=np.int64))
            continue
        expect = int(n * density + 10 * np.sqrt(n * density + 1) + 16)
        pos = []
        last = -1
        while True:
            gaps = rng.geometric(density, size=expect)
            r = last + np.cumsum(gaps)
            pos.append(r)
            last = int(r[-1])
            if last >= n:
                break
        r = np.concatenate(pos)
        cols.append(r[r < n])
    counts = np.array([c.size for c in cols], dtype=np.int64)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    rows = (np.concatenate(cols) if cols else np.zeros(0)).astype(np.int32)
    return col_ptr, rows


def linear_predictor(n, col_ptr, rows, vals, beta):
    """eta = X beta for a CSC design (vals None means all non-zeros are 1)."""
    eta = np.zeros(n, dtype=np.float64)
    for j in range(len(col_ptr) - 1):
        if beta[j] == 0.0:
            continue
        a, b = col_ptr[j], col_ptr[j + 1]
        x = 1.0 if vals is None else vals[a:b]
        np.add.at(eta, rows[a:b], x * beta[j])
    return eta


def dense_column(n, col_ptr, rows, vals, j):
    x = np.zeros(n, dtype=np.float64)
    a, b = col_ptr[j], col_ptr[j + 1]
    x[rows[a:b]] = 1.0 if vals is None else vals[a:b]
    return x


def csc_from_dense(X):
    """CSC arrays (col_ptr, rows int32, vals float64) of a dense matrix."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    rows, vals = [], []
    for j in range(p):
        nz = np.nonzero(X[:, j])[0]
        rows.append(nz)
        vals.append(X[nz, j])
        col_ptr[j + 1] = col_ptr[j] + nz.size
    return (col_ptr, np.concatenate(rows).astype(np.int32),
            np.concatenate(vals).astype(np.float64))


def _coefficients(rng, p, nonzero_frac):
    """beta_j ~ N(0,1) x Bernoulli(nonzero_frac); draws normals then uniforms."""
    z = rng.standard_normal(p)
    keep = rng.random(p) < nonzero_frac
    return np.where(keep, z, 0.0)


def cox_data(seed, n, p, density=0.05, nonzero_frac=0.2):
    """Sec. 3.2 Cox design.

    Draw order: design (indicator_design), beta, T (exponential), C."""
    rng = np.random.default_rng(seed)
    col_ptr, rows = indicator_design(rng, n, p, density)
    beta = _coefficients(rng, p, nonzero_frac)
    eta = linear_predictor(n, col_ptr, rows, None, beta)
    T = rng.exponential(1.0, size=n) / np.exp(eta)
    C = rng.exponential(1.0, size=n)
    y = np.minimum(T, C)
    status = (T <= C).astype(np.int8)
    return {"n": n, "p": p, "y": y, "status": status, "col_ptr": col_ptr,
            "rows": rows, "vals": None, "beta_true": beta}


def fg_data(seed, n, p, density=0.05, nonzero_frac=0.2, pmix=0.5):
    """Sec. 3.2 Fine-Gray design (competing risks).

    Draw order: design, beta1, U (event type), V (time given type), C."""
    rng = np.random.default_rng(seed)
    col_ptr, rows = indicator_design(rng, n, p, density)
    beta1 = _coefficients(rng, p, nonzero_frac)
    beta2 = -beta1
    eta1 = linear_predictor(n, col_ptr, rows, None, beta1)
    eta2 = linear_predictor(n, col_ptr, rows, None, beta2)
    r1 = np.exp(eta1)
    p1 = 1.0 - (1.0 - pmix) ** r1               # P(eps = 1 | x)
    U = rng.random(n)
    V = rng.random(n)
    primary = U < p1
    # eps = 1: solve F_1(t|x) = V * P(eps=1|x) for t
    inner = 1.0 - V * p1
    T1 = -np.log(1.0 - (1.0 - inner ** (1.0 / r1)) / pmix)
    # eps = 2: exponential with rate exp(x' beta2), from the same uniform
    T2 = -np.log1p(-V) / np.exp(eta2)
    T = np.where(primary, T1, T2)
    C = rng.exponential(1.0, size=n)
    y = np.minimum(T, C)
    status = np.where(T <= C, np.where(primary, 1, 2), 0).astype(np.int8)
    return {"n": n, "p": p, "y": y, "status": status, "col_ptr": col_ptr,
            "rows": rows, "vals": None, "beta_true": beta1}


def uniform_tuple_data(seed, n, density=1.0):
    """Sec. 3.1 kernel-fusion workload: inputs drawn from Uniform(1, 2).

    e ~ U(1,2) (the exp(X beta) vector), one covariate column whose
    non-zero values are U(1,2) (dense by default), event indicator
    Bernoulli(0.5), observed times U(0,1) (distinct with overwhelming
    probability; a tie would be handled exactly anyway).
    Draw order: e, x values, design rows (if sparse), delta, times."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(1.0, 2.0, size=n)
    xv = rng.uniform(1.0, 2.0, size=n)
    if density >= 1.0:
        rows = np.arange(n, dtype=np.int32)
    else:
        rows = np.nonzero(rng.random(n) < density)[0].astype(np.int32)
    vals = xv[rows]
    status = (rng.random(n) < 0.5).astype(np.int8)
    y = rng.random(n)
    col_ptr = np.array([0, rows.size], dtype=np.int64)
    return {"n": n, "p": 1, "y": y, "status": status, "col_ptr": col_ptr,
            "rows": rows, "vals": vals, "eta": np.log(e)}


def force_ties(y, levels):
    """Round observed times onto ``levels`` distinct values (forces ties)."""
    y = np.asarray(y, dtype=np.float64)
    q = np.quantile(y, np.linspace(0, 1, levels + 1)[1:-1]) if levels > 1 else []
    return np.searchsorted(np.asarray(q), y).astype(np.float64) + 1.0


def cv_folds(seed, n, k=10, repeats=10):
    """Training masks of k-fold cross-validation repeated `repeats` times
    (Sec. 2.8; 10 folds x 10 repetitions in Sec. 3.3).  Repetition t draws a
    random partition of the subjects into k folds of sizes differing by at
    most one; replicate t*k + f trains on every subject outside fold f.
    Returns uint8 [repeats*k, n], 1 = training subject."""
    rng = np.random.default_rng(seed)
    masks = np.ones((repeats * k, n), dtype=np.uint8)
    for t in range(repeats):
        fold = rng.permutation(n) % k
        for f in range(k):
            masks[t * k + f, fold == f] = 0
    return masks
