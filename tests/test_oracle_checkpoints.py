"""Pins for the checkpoint conditions of SSA (Algorithm 1) and D-SSA
(Algorithm 4) in the oracle.

Every logged iteration of many oracle runs is re-derived here from the
logged integers and the constants (pinned in test_oracle_constants.py), in
algebraic forms other than the ones the oracle evaluates, and with the
oracle's separately pinned Max-Coverage and Estimate-Inf as the only
building blocks.

D-SSA, iteration t, N_t = ceil(Lambda) 2^(t-1) sets in each half:
  * D1 holds iff the integer Cov_c reaches ceil(Lambda1); eps_t is logged as
    -1 when it does not;
  * with I^c = n Cov_c / N_t the printed n (1+eps) / (2^(t-1) I^c) equals
    (1+eps) ceil(Lambda) / Cov_c (reading R15), so
        eps2 = eps sqrt((1+eps) ceil(Lambda) / Cov_c),
        eps3 = eps2 sqrt((1-1/e-eps) / (1+eps/3)),
        1 + eps1 = Cov / Cov_c,
        eps_t = ((1+eps1)(1+eps2) - 1)(1-1/e-eps) + (1-1/e) eps3;
  * the run ends at the first iteration with D1 and eps_t <= eps (D2), or at
    the first whose N_t reaches N_max.
SSA, iteration t, |R| = ceil(Lambda) 2^(t-1):
  * Cov equals a fresh Max-Coverage of the stream's first |R| sets;
  * Estimate-Inf runs iff Cov >= Lambda1 (C1), on the derived stream K_t
    with eps2 and delta / (3 i_max), capped at
    T_max = 2 |R| (1+eps2)/(1-eps2) eps3^2/eps2^2. The test runs it without
    a cap and applies the cap itself: T = min(T_free, floor(T_max)), and
    I_c = -1 when the cap is what ended it;
  * C2: the run ends at the first C1 iteration with n Cov/|R| <= (1+eps1) I_c.

Inputs are chosen so that each rule decides something: a graph where
Lambda <= Cov_c < Lambda1 at some iteration (D1 against the wrong bound
would pass there), runs where (1+eps1) I_c < n Cov/|R| <= (1+eps2) I_c (C2
with the wrong epsilon would stop there), and a run where Estimate-Inf needs
more than half of T_max (a cap without its factor 2 would end it early).
The last uses a graph without edges: every RR set is {source}, I(S) = |S|
exactly, and with k close to n/2 and few samples per node the greedy's
estimate runs well above I(S) while Cov only just reaches Lambda1.
"""
import math

import numpy as np
import pytest

ONE_M = 1.0 - math.exp(-1.0)
EMPTY_U32 = np.array([], np.uint32)


def edgeless(oracle_lib, n):
    return oracle_lib.Graph(oracle_lib.IC, n, EMPTY_U32, EMPTY_U32, np.array([], np.float32))


def check_dssa_log(n, eps, st, d):
    """Every iteration of one D-SSA run against Algorithm 4; returns the
    iterations whose Cov_c lay in [Lambda, Lambda1)."""
    lam_c, lam1_c = math.ceil(d["lambda"]), math.ceil(d["lambda1"])
    between = 0
    last_pass = None
    T = st["iterations"]
    for t in range(1, T + 1):
        nt, cov, cov_c, e_t = (st["it_sets"][t - 1], st["it_cov"][t - 1], st["it_cov_c"][t - 1],
                               st["it_eps_t"][t - 1])
        assert nt == lam_c << (t - 1)
        if d["lambda"] <= cov_c < d["lambda1"]:
            between += 1
        if cov_c < lam1_c:  # D1 fails
            assert e_t == -1.0, (t, cov_c, lam1_c)
            d2 = False
        else:
            eps2 = eps * math.sqrt((1.0 + eps) * lam_c / cov_c)
            eps3 = eps2 * math.sqrt((ONE_M - eps) / (1.0 + eps / 3.0))
            ratio = cov / cov_c
            want = (ratio * (1.0 + eps2) - 1.0) * (ONE_M - eps) + ONE_M * eps3
            assert e_t == pytest.approx(want, rel=1e-12, abs=1e-14), (t, cov, cov_c)
            d2 = e_t <= eps
            last_pass = (ratio - 1.0, eps2, eps3, want, n * cov_c / nt)
        capped = nt >= d["n_max"]
        if t < T:
            assert not d2 and not capped, t
        else:
            assert d2 or capped
            assert st["stopped_by_cap"] == (not d2)
            assert st["n_sets"] == 2 * nt and st["cov"] == cov and st["cov_c"] == cov_c
    if last_pass is not None:
        e1, e2, e3, et, ic = last_pass
        assert st["eps1"] == pytest.approx(e1, rel=1e-12, abs=1e-14)
        assert st["eps2"] == pytest.approx(e2, rel=1e-12)
        assert st["eps3"] == pytest.approx(e3, rel=1e-12)
        assert st["eps_t"] == pytest.approx(et, rel=1e-12, abs=1e-14)
        assert st["i_c"] == pytest.approx(ic, rel=1e-12)
    return between


def check_ssa_log(oracle_lib, og, k, eps, split, delta, key, seeds, st):
    """Every iteration of one SSA run against Algorithm 1 (C1, Estimate-Inf
    with its cap, C2); returns (iterations where C2 with eps2 in place of
    eps1 would decide differently, iterations where Estimate-Inf needed more
    than half of its cap)."""
    n = og.n
    c = oracle_lib.ssa_constants(n, k, eps, delta)
    e1, e2, e3 = split if split is not None else (c["eps1"], c["eps2"], c["eps3"])
    lam_c = math.ceil(c["lambda"])
    lam1 = (1 + e1) * (1 + e2) * oracle_lib.upsilon(e3, delta / (3 * c["i_max"]))
    delta2p = delta / (3 * c["i_max"])
    pool = oracle_lib.Pool(og, key)
    c2_window = over_half = 0
    T_it = st["iterations"]
    for t in range(1, T_it + 1):
        size = st["it_sets"][t - 1]
        assert size == lam_c << (t - 1)
        pool.extend(size)
        s_t, cov = pool.max_coverage(k)
        assert cov == st["it_cov"][t - 1]
        T_log, ic_log = st["it_cov_c"][t - 1], st["it_eps_t"][t - 1]
        if cov < lam1:  # C1 fails: no Estimate-Inf
            assert T_log == 0 and ic_log == -1.0, t
            stop = False
        else:
            t_max = 2.0 * size * (1.0 + e2) / (1.0 - e2) * (e3 * e3) / (e2 * e2)
            ic_free, T_free = og.estimate_inf(s_t, e2, delta2p, 1e15, oracle_lib.derived_key(key, t))
            assert ic_free > 0
            if T_free <= math.floor(t_max):
                assert T_log == T_free and ic_log == ic_free, (t, T_log, T_free)
            else:
                assert T_log == math.floor(t_max) and ic_log == -1.0, (t, T_log, t_max)
            over_half += T_free > t_max / 2
            i_hat = n * cov / size
            stop = i_hat <= (1.0 + e1) * ic_log
            if ic_log > 0 and (1.0 + e1) * ic_log < i_hat <= (1.0 + e2) * ic_log:
                c2_window += 1
        capped = size >= c["n_max"]
        if t < T_it:
            assert not stop and not capped, t
        else:
            assert stop or capped
            assert st["stopped_by_cap"] == (not stop)
            assert seeds.tolist() == s_t.tolist()
            assert st["n_sets"] == size and st["cov"] == cov
    return c2_window, over_half


@pytest.mark.parametrize("model", [0, 1])
def test_dssa_checkpoints_on_chung_lu(oracle_lib, synth_lib, model):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, g.w_ic if model == 0 else g.w_lt)
    runs = 0
    for k, eps in ((10, 0.1), (3, 0.2), (40, 0.3)):
        d = oracle_lib.dssa_constants(g.n, k, eps, 1.0 / g.n)
        for key in range(10):
            _, st = og.dssa(k, eps, 1.0 / g.n, key)
            check_dssa_log(g.n, eps, st, d)
            runs += 1
    assert runs >= 30


def test_dssa_d1_between_lambda_and_lambda1(oracle_lib):
    # No edges: every set is {source}, so k seeds cover a fraction close to
    # k/n of any half. With k/n = 21/80 the verification half of iteration 3
    # (4 ceil(Lambda) sets) holds about 1.05 Lambda covered sets: at least
    # Lambda, below Lambda1 = 1 + 1.1 Lambda.
    n, k, eps = 80, 21, 0.1
    og = edgeless(oracle_lib, n)
    d = oracle_lib.dssa_constants(n, k, eps, 1.0 / n)
    between = 0
    for key in range(20):
        _, st = og.dssa(k, eps, 1.0 / n, key)
        between += check_dssa_log(n, eps, st, d)
    assert between >= 10


@pytest.mark.parametrize("model", [0, 1])
def test_ssa_checkpoints_default_split(oracle_lib, synth_lib, model):
    g = synth_lib.make("cl_small")
    og = oracle_lib.Graph(model, g.n, g.src, g.dst, g.w_ic if model == 0 else g.w_lt)
    for k, eps in ((10, 0.2), (50, 0.3)):
        for key in range(8):
            seeds, st = og.ssa(k, eps, 1.0 / g.n, key)
            check_ssa_log(oracle_lib, og, k, eps, None, 1.0 / g.n, key, seeds, st)


def test_ssa_c2_window_on_edgeless_graph(oracle_lib):
    # I(S) = k for every S here, and the greedy's estimate sits a few percent
    # above it at early checkpoints: between (1+eps1) I_c and (1+eps2) I_c.
    n, k, eps = 200, 100, 0.1
    og = edgeless(oracle_lib, n)
    window = 0
    for key in range(10):
        seeds, st = og.ssa(k, eps, 1.0 / n, key)
        w, _ = check_ssa_log(oracle_lib, og, k, eps, None, 1.0 / n, key, seeds, st)
        window += w
    assert window >= 10


def test_ssa_estimate_inf_cap_decides(oracle_lib):
    # A split with eps2 != eps3 and tiny eps1 (Eq. 14 holds: 0.0153 <= 0.1).
    # With n = 6000, k = 2600 and no edges, C1 first holds at |R| = 128
    # ceil(Lambda) with Cov about 1.06 Lambda1 while n Cov/|R| is about 1.2 k,
    # so Estimate-Inf needs about 0.56 T_max sets.
    n, k, eps, delta = 6000, 2600, 0.1, 0.5
    split = (0.002, 0.01, 0.0125)
    assert oracle_lib.eps_admissible(eps, *split)
    og = edgeless(oracle_lib, n)
    over = 0
    for key in range(2):
        seeds, st = og.ssa_eps(k, eps, *split, delta, key)
        _, o = check_ssa_log(oracle_lib, og, k, eps, split, delta, key, seeds, st)
        over += o
    assert over >= 2
