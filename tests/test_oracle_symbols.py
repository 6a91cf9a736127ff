"""Pins of the oracle's Fourier analysis against printed values (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import symbols

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("case", GOLD["tau_star"]["cases"])
def test_tau_star_printed_values(case):
    v = symbols.tau_star(case["r"], case["psibar"])
    assert round(v, case["digits"]) == case["value"]


def test_tau_star_infinite_in_liquid_regime():
    assert symbols.tau_star(-0.3, -0.4) == math.inf  # psibar^2 > -r/3


@pytest.mark.parametrize("tau,r,psibar", [(0.1, -0.35, 0.0), (0.5, -0.3, -0.25), (2.0, -0.35, -0.3)])
def test_numeric_eigenvalues_match_printed_sets(tau, r, psibar):
    for k2 in np.linspace(0.0, 32.0, 97):
        A = symbols.sym_A(k2, tau, r, psibar)
        ev = np.linalg.eigvals(A @ np.linalg.inv(symbols.sym_PCH(k2, tau)))
        third = symbols.eig_printed_QCH(k2, tau, r, psibar)
        # two eigenvalues are 1, the third is the printed expression
        rest = sorted(ev, key=lambda z: abs(z - 1.0))
        assert abs(rest[0] - 1) < 1e-6 and abs(rest[1] - 1) < 1e-6 or abs(third - 1) < 1e-6
        assert min(abs(ev - third)) < 1e-9 * max(1.0, abs(third))
        if tau < 1.0:
            evq = np.linalg.eigvals(A @ np.linalg.inv(symbols.sym_P(k2, tau)))
            thq = symbols.eig_printed_Q(k2, tau, r, psibar)
            assert min(abs(evq - thq)) < 1e-9 * max(1.0, abs(thq))


def test_tau_natural():
    """Denominator of the third eigenvalue of Q: zero at tau = 1, |k| = 1, positive below."""
    def den(k2, tau):
        st = math.sqrt(tau)
        return tau * k2 ** 3 + (st - 2 * tau) * k2 ** 2 - st * k2 + 1
    assert abs(den(1.0, GOLD["tau_natural"]["value"])) < 1e-15
    k2 = np.linspace(0, 50, 20001)
    for tau in (0.1, 0.5, 0.9, 0.99):
        assert den(k2, tau).min() > 0
    assert den(k2, 1.2).min() < 0


def test_rho_printed_ranges():
    g = GOLD["rho"]
    rq = symbols.rho_sigma("Q", g["tau"], g["r"], g["psibar"], dim=2)
    rch = symbols.rho_sigma("QCH", g["tau"], g["r"], g["psibar"], dim=2)
    r0 = symbols.rho_sigma("A0", g["tau"], g["r"], g["psibar"], dim=2)
    lo, hi = g["QCH_range"]
    assert lo <= rch <= hi
    assert rq < rch < r0
    assert r0 > 0.95 and abs(r0 - g["A0_approx"]) < 0.03
