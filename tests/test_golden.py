"""The oracle against the hand-derived examples in tests/golden (each file
cites its passage and carries its derivation): the O(N^2) definition and
the O(N) scan form both reproduce the exact values."""
import numpy as np
import pytest

import golden
from oracle import adjoint, risk, scan


@pytest.mark.parametrize("name", golden.NAMES)
def test_coordinate_examples(name):
    g = golden.load(name)
    y, s, x, eta = (np.array(g[k], dtype=float) for k in ("y", "status", "x", "eta"))
    s = s.astype(int)
    b = risk.brute(g["model"], y, s, eta, x)
    for got in (b, scan.scan(g["model"], y, s, eta, x)):
        assert got["g1"] == pytest.approx(g["g1"], rel=1e-14, abs=1e-15)
        assert got["g2"] == pytest.approx(g["g2"], rel=1e-14, abs=1e-15)
        assert got["loglik"] == pytest.approx(g["loglik"], rel=1e-14, abs=1e-15)


def test_eta_gradient_example():
    g = golden.load("eta_gradient_hand")
    y, s = np.array(g["y"], float), np.array(g["status"], int)
    eta = np.array(g["eta"])
    for f in (adjoint.eta_gradient_brute, adjoint.eta_gradient_scan):
        np.testing.assert_allclose(f(g["model"], y, s, eta), g["grad"], rtol=1e-14,
                                   atol=1e-15)
