"""Pins of the performance model (Sec. III-B) against the paper's Table I
and against the algebra of Eqs. 3-6."""
import math
import os

import numpy as np
import pytest

from paper_2501_09398_amd import perfmodel as pm


def table1(golden_dir):
    rows = []
    for line in open(os.path.join(golden_dir, "table1_fit_coefficients.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    return rows


def test_eq5_equals_eq3_with_eq4():
    rng = np.random.default_rng(0)
    for _ in range(100):
        T_l, T_k, T_i, T_a = rng.uniform(1e-6, 1e-4, 4)
        I_k = 10000
        for S in pm.divisors(I_k):
            e3 = pm.exec_time_eq3(T_l, T_k, T_i, T_a, S, I_k // S)
            e5 = pm.exec_time_eq5(T_l, T_k, T_i, T_a, S, I_k)
            assert abs(e3 - e5) <= 1e-12 * e3
            a, b = pm.eq6_coefficients(T_l, T_k, T_i, T_a, I_k)
            assert abs(a / S + b - e5) <= 1e-12 * e5


def test_gain_condition_observation_1():
    # Larger batches lower T_E exactly when T_i < T_a.
    lo = pm.exec_time_eq5(1e-5, 2e-6, 1e-6, 3e-6, 10, 10000)
    hi = pm.exec_time_eq5(1e-5, 2e-6, 1e-6, 3e-6, 100, 10000)
    assert hi < lo
    lo = pm.exec_time_eq5(1e-5, 2e-6, 4e-6, 3e-6, 10, 10000)
    hi = pm.exec_time_eq5(1e-5, 2e-6, 4e-6, 3e-6, 100, 10000)
    assert hi > lo


def test_table1_synthetic_recovery(golden_dir):
    # Data generated from Table I's coefficients plus noise at the stated MAE
    # is fitted back to within a few standard errors.
    rng = np.random.default_rng(1)
    S = np.array(pm.divisors(10000, 1, 2500), dtype=float)
    for thr, kc, bc, mae_c, a, b, mae_e in table1(golden_dir):
        tc = kc * S + bc + rng.laplace(0, mae_c, S.size)
        te = a / S + b + rng.laplace(0, mae_e, S.size)
        fc, fe = pm.fit_creation(S, tc), pm.fit_execution(S, te)
        # standard errors of ordinary least squares; Laplace(scale m) has
        # mean absolute deviation m and standard deviation sqrt(2) m
        Ac = np.stack([S, np.ones_like(S)], 1)
        Ae = np.stack([1 / S, np.ones_like(S)], 1)
        se_c = np.sqrt(2) * mae_c * np.sqrt(np.diag(np.linalg.inv(Ac.T @ Ac)))
        se_e = np.sqrt(2) * mae_e * np.sqrt(np.diag(np.linalg.inv(Ae.T @ Ae)))
        assert abs(fc.k_c - kc) < 5 * se_c[0] and abs(fc.b_c - bc) < 5 * se_c[1]
        assert abs(fe.a - a) < 5 * se_e[0] and abs(fe.b - b) < 5 * se_e[1]
        assert 0.3 * mae_c < fc.mae < 3 * mae_c
        # noiseless data is recovered exactly
        fc0, fe0 = pm.fit_creation(S, kc * S + bc), pm.fit_execution(S, a / S + b)
        assert math.isclose(fc0.k_c, kc, rel_tol=1e-9) and math.isclose(fc0.b_c, bc, rel_tol=1e-9)
        assert math.isclose(fe0.a, a, rel_tol=1e-9) and math.isclose(fe0.b, b, rel_tol=1e-9)


def test_table1_optimum_in_papers_range(golden_dir):
    # Sec. IV-A finds the optimal iteration batch at 50-100 kernels for
    # I_k = 10,000; the model with Table I's coefficients agrees.
    expected_closed = [65.1, 50.3, 36.3]
    expected_divisor = [80, 50, 40]
    for row, sc, sd in zip(table1(golden_dir), expected_closed, expected_divisor):
        _, kc, bc, _, a, b, _ = row
        m = pm.Model(pm.CreationFit(kc, bc, 0), pm.ExecutionFit(a, b, 0), K=1)
        assert abs(m.s_closed_form() - sc) < 0.05
        best, _ = m.best(pm.divisors(10000))
        assert best == sd
        assert 35 <= best <= 100


def test_table1_speedup_ratio_s1_vs_s100(golden_dir):
    # Modelled T(S=1)/T(S=100): the smallest workload gains most (Obs. III).
    ratios = []
    for _, kc, bc, _, a, b, _ in table1(golden_dir):
        m = pm.Model(pm.CreationFit(kc, bc, 0), pm.ExecutionFit(a, b, 0))
        ratios.append(float(m.total(1) / m.total(100)))
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert abs(ratios[0] - 1.369) < 2e-3


def test_speedup_error_quadrature():
    s, e = pm.speedup([2.0, 2.0, 2.0], [1.0, 1.0, 1.0])
    assert s == 2.0 and e == 0.0
    base = np.array([10.0, 12.0])
    graph = np.array([5.0, 5.0])
    s, e = pm.speedup(base, graph)
    assert math.isclose(s, 2.2)
    assert math.isclose(e, 2.2 * (1.0 / 11.0))


def test_divisors():
    assert pm.divisors(10000, 1, 2000)[:6] == [1, 2, 4, 5, 8, 10]
    assert len(pm.divisors(10000, 1, 2000)) == 22
    assert pm.divisors(1000) == [1, 2, 4, 5, 8, 10, 20, 25, 40, 50, 100, 125, 200, 250, 500, 1000]


def test_fit_standard_errors_match_polyfit_covariance():
    """The coefficient standard errors of Eq. 2 and Eq. 6 equal the square
    roots of the covariance numpy's polyfit reports (residual variance over
    n - 2 degrees of freedom)."""
    rng = np.random.default_rng(1)
    x = np.array([4, 8, 20, 40, 80, 200, 400, 800], float)
    y = 4.2e-6 * x + 1.6e-4 + rng.normal(0, 5e-5, x.size)
    f = pm.fit_creation(x, y)
    p, cov = np.polyfit(x, y, 1, cov=True)
    assert np.isclose(f.k_c, p[0]) and np.isclose(f.b_c, p[1])
    assert np.isclose(f.k_c_se, np.sqrt(cov[0, 0]), rtol=1e-9) and np.isclose(f.b_c_se, np.sqrt(cov[1, 1]), rtol=1e-9)
    S = np.array([1, 2, 5, 10, 20, 50, 100], float)
    t = 1.77e-2 / S + 4.56e-2 + rng.normal(0, 1e-4, S.size)
    e = pm.fit_execution(S, t)
    p, cov = np.polyfit(1.0 / S, t, 1, cov=True)
    assert np.isclose(e.a_se, np.sqrt(cov[0, 0]), rtol=1e-9) and np.isclose(e.b_se, np.sqrt(cov[1, 1]), rtol=1e-9)


def test_trace_gaps_synthetic_timeline():
    """A synthetic trace laid out as Eq. 3 describes it: graph jobs of I
    launches of S nodes (kernel T_k, node gap T_i, graph gap T_a), then a
    per-launch job (gap T_a0 between launches): the analyser recovers each
    gap class exactly."""
    K, b, iters, Tk, Ti, Ta, Ta0 = 2, 5, 20, 3000, 700, 9000, 4000
    rows, t = [], 0
    for job in range(2):
        for j in range(K * iters):
            rows.append(("k%d" % (j % K), t, t + Tk, 64))
            t += Tk + (Ta if (j + 1) % (K * b) == 0 else Ti)
        t += 10 ** 7                                       # host work between jobs
    for j in range(K * iters):
        rows.append(("k%d" % (j % K), t, t + Tk, 64))
        t += Tk + Ta0
    r = pm.trace_gaps(rows, K, b, iters, 2, 1)
    assert r["T_i_in_graph_gap"]["median_us"] == Ti / 1e3
    assert r["T_a_between_graphs_gap"]["median_us"] == Ta / 1e3
    assert r["T_a_between_graphs_gap"]["n"] == 2 * (iters // b - 1)
    assert r["T_a_per_launch_gap"]["median_us"] == Ta0 / 1e3
    assert r["graph_kernel_duration"]["median_us"] == Tk / 1e3
