"""Pins for the closed-form constants of SSA and D-SSA (oracle side).

Each check compares with something the paper fixes or a library routine:
the printed eps defaults, Eq. 14's constraint, the IMM form of the sample
cap (Eq. 13 with delta/3, as Lemma 4 states), Table 3's D-SSA sample
counts, and lgamma for ln C(n,k).
"""
import json
import math
from pathlib import Path

import pytest

GOLD = Path(__file__).parent / "golden"
ONE_M = 1.0 - math.exp(-1.0)


def test_upsilon_closed_form(oracle_lib):
    # Table 1: Upsilon(eps, delta) = (2 + 2eps/3) ln(1/delta) / eps^2.
    # At delta = 1/e the log is 1; at eps = 1, delta = e^-3 it is 3 * 8/3.
    assert oracle_lib.upsilon(0.1, math.exp(-1.0)) == pytest.approx((2 + 0.2 / 3) / 0.01, rel=1e-14)
    assert oracle_lib.upsilon(1.0, math.exp(-3.0)) == pytest.approx(8.0, rel=1e-14)
    assert oracle_lib.upsilon(0.5, 0.25) == pytest.approx((2 + 1 / 3) * math.log(4) * 4, rel=1e-14)


@pytest.mark.parametrize("n,k", [(10, 3), (15233, 50), (1 << 20, 100), (41_700_000, 1000), (5, 5), (7, 1)])
def test_ln_choose_vs_lgamma(oracle_lib, n, k):
    ref = math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)
    assert oracle_lib.ln_choose(n, k) == pytest.approx(ref, rel=1e-11, abs=1e-9)


def test_eps_defaults_match_printed(oracle_lib):
    g = json.loads((GOLD / "eps_defaults.json").read_text())
    c = oracle_lib.ssa_constants(15233, 50, g["eps"], 1 / 15233)
    a, b = g["eps1_printed"]
    assert c["eps1"] == pytest.approx(a / b, abs=1.5e-3)
    a, b = g["eps2_printed"]
    assert c["eps2"] == pytest.approx(a / b, abs=1.5e-3)
    assert c["eps3"] == c["eps2"]


@pytest.mark.parametrize("eps", [0.02, 0.05, 0.1, 0.2, 0.3, 0.5])
def test_eps_defaults_meet_eq14_with_equality(oracle_lib, eps):
    c = oracle_lib.ssa_constants(1000, 10, eps, 1e-3)
    e1, e2, e3 = c["eps1"], c["eps2"], c["eps3"]
    lhs = ONE_M * (e1 + e2 + e1 * e2 + e3) / ((1 + e1) * (1 + e2))
    assert lhs == pytest.approx(eps, rel=1e-12)
    assert 0 < e1 and 0 < e2 < 1 and 0 < e3 < 1


@pytest.mark.parametrize("n,k,eps", [(15233, 50, 0.1), (1 << 20, 100, 0.1), (4_800_000, 500, 0.05), (100, 1, 0.2)])
def test_nmax_equals_imm_bound_with_delta_over_3(oracle_lib, n, k, eps):
    # Algorithm 1 writes N_max through Upsilon(eps, delta/6/C(n,k)); Lemma 4
    # says it is Eq. 13's simplified IMM threshold with delta replaced by
    # delta/3: 8(1-1/e)(ln(2/(delta/3)) + ln C(n,k)) / eps^2 * n/k.
    delta = 1.0 / n
    lnc = math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)
    imm = 8 * ONE_M * (math.log(2 / (delta / 3)) + lnc) / eps**2 * n / k
    c = oracle_lib.ssa_constants(n, k, eps, delta)
    d = oracle_lib.dssa_constants(n, k, eps, delta)
    assert c["n_max"] == pytest.approx(imm, rel=1e-9)
    assert d["n_max"] == pytest.approx(imm, rel=1e-9)


@pytest.mark.parametrize("n,k,eps", [(15233, 50, 0.1), (1 << 20, 100, 0.1), (37000, 1, 0.1), (3000, 30, 0.3)])
def test_iteration_caps_and_lambdas(oracle_lib, n, k, eps):
    delta = 1.0 / n
    c = oracle_lib.ssa_constants(n, k, eps, delta)
    d = oracle_lib.dssa_constants(n, k, eps, delta)
    ratio = 2 * c["n_max"] / oracle_lib.upsilon(eps, delta / 3)
    # i_max = t_max = ceil(log2(2 N_max / Upsilon(eps, delta/3)))
    assert 2 ** (c["i_max"] - 1) < ratio <= 2 ** c["i_max"]
    assert d["t_max"] == c["i_max"]
    # Lambda = Upsilon(eps, delta/(3 i_max)); SSA Lambda1 with eps3; D-SSA Lambda1 = 1 + (1+eps) Lambda
    assert c["lambda"] == pytest.approx(oracle_lib.upsilon(eps, delta / (3 * c["i_max"])), rel=1e-15)
    assert d["lambda1"] == pytest.approx(1 + (1 + eps) * d["lambda"], rel=1e-15)
    lam1 = (1 + c["eps1"]) * (1 + c["eps2"]) * oracle_lib.upsilon(c["eps3"], delta / (3 * c["i_max"]))
    assert c["lambda1"] == pytest.approx(lam1, rel=1e-15)
    # SSA's eps3 = eps2 < eps, so Lambda1 > Lambda
    assert c["lambda1"] > c["lambda"]


def test_table3_dssa_counts_are_lambda_times_power_of_two(oracle_lib):
    # D-SSA ends iteration t holding R_t and R^c_t, 2 N_t = ceil(Lambda) 2^t
    # sets. Table 3's printed (rounded) counts must sit on that grid.
    g = json.loads((GOLD / "table3_dssa.json").read_text())
    eps = g["eps"]
    for name, row in g["graphs"].items():
        n = row["n"]
        for k, count in row["dssa_rr"].items():
            d = oracle_lib.dssa_constants(n, int(k), eps, 1.0 / n)
            x = math.log2(count / math.ceil(d["lambda"]))
            t = round(x)
            assert abs(x - t) < 0.05, (name, k, x)
            assert 1 <= t <= d["t_max"], (name, k, t)


def test_argument_checks(oracle_lib):
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.ssa_constants(10, 0, 0.1, 0.1)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.ssa_constants(10, 11, 0.1, 0.1)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.dssa_constants(10, 1, 0.7, 0.1)  # eps >= 1 - 1/e
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.dssa_constants(10, 1, 0.1, 1.0)
