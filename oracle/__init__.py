"""FP64 CPU oracle for the Cox / Fine-Gray coordinate gradient and Hessian.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only ``tests/``, the smoke check
in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written from the paper (Yang, Schuemie, Ji & Suchard,
"Massive Parallelization of Massive Sample-size Survival Analysis",
arXiv 2204.08183) and shares no code with the HIP library:

* ``risk``    -- the plain O(N^2) risk-set definitions of the Cox log partial
                 likelihood (Sec. 2.1, eq. cox_l) and the Fine-Gray log
                 pseudo-likelihood with its IPCW weights (Sec. 2.2, eq. fg_l),
                 together with their first and second derivatives along one
                 coordinate (Sec. 2.4).
* ``exact``   -- the same definitions evaluated in 50-digit ``mpmath``
                 arithmetic for tiny inputs.
* ``km``      -- the Kaplan-Meier estimate of the censoring survival function
                 G(t) = Pr(C > t) that the Fine-Gray weights use (Sec. 2.2).
* ``prep``    -- the integer preparation the scan form needs: ordering by
                 decreasing observed time, tie runs and per-run event counts
                 (Sec. 2.7).
* ``scan``    -- the serial O(N) scan form of Sec. 2.7 (eqs. cox_g, cox_h,
                 fg_g, fg_h), in plain C with compensated sums.
* ``ccd``     -- the one-dimensional penalised Newton step with trust region
                 and the l1 directional-derivative rule (Secs. 2.3-2.4).
* ``adjoint`` -- the gradient of the log-likelihood in the linear predictor
                 for every subject (Sec. 2.9), brute force and O(N) scan form.
* ``cv``      -- cross-validation replicates (Sec. 2.8): CCD on a training
                 subset, the predictive log-likelihood of the held-out one.

Every function computes in IEEE double precision unless stated otherwise.
"""
