"""Scenario generation as random convex combinations of seven operating cases
(Case study, problem setup), on synthetic base cases standing in for the
paper's measurements: the weights lie on the simplex, the scenarios in the
convex hull of the cases, the feed rows are the same combinations of the
cases' feed rows, and the sample mean approaches the cases' centroid (the mean
of uniform simplex weights is 1/7 each).
"""

import numpy as np
import pytest
from scipy.optimize import linprog

from absorber_inputs import CONFIGS, N_BASE_CASES, base_cases, convex_combinations, feed_table


def test_weights_on_the_simplex_and_exact_combination():
    C = base_cases()
    assert C.shape == (N_BASE_CASES, 3) and np.abs(C).max() <= 0.2
    X, w = convex_combinations(C, 500, 7)
    assert X.shape == (500, 3) and w.shape == (500, N_BASE_CASES)
    assert (w >= 0).all() and np.allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.allclose(X, w @ C, rtol=0, atol=1e-15)


def test_scenarios_in_the_convex_hull():
    # feasibility of lambda >= 0, sum lambda = 1, C^T lambda = x, found
    # independently of the sampler's weights
    C = base_cases()
    X, _ = convex_combinations(C, 40, 11)
    A = np.vstack([C.T, np.ones((1, N_BASE_CASES))])
    for x in X:
        r = linprog(np.zeros(N_BASE_CASES), A_eq=A, b_eq=np.r_[x, 1.0], bounds=[(0, None)] * N_BASE_CASES)
        assert r.status == 0
    # a point outside the bounding box of the cases is not in the hull
    out = C.max(axis=0) + 0.01
    r = linprog(np.zeros(N_BASE_CASES), A_eq=A, b_eq=np.r_[out, 1.0], bounds=[(0, None)] * N_BASE_CASES)
    assert r.status == 2


def test_feed_rows_are_the_same_combination(params):
    C = base_cases()
    X, w = convex_combinations(C, 64, 3)
    Fc = feed_table(C, params)
    assert np.allclose(feed_table(X, params), w @ Fc, rtol=1e-14, atol=1e-12)


def test_sample_mean_approaches_the_centroid():
    C = base_cases()
    X, w = convex_combinations(C, 20000, 5)
    # Dirichlet(1,...,1): each weight has mean 1/K and variance (K-1)/(K^2 (K+1))
    K = N_BASE_CASES
    sd = np.sqrt((K - 1) / (K * K * (K + 1)) / X.shape[0])
    assert np.abs(w.mean(axis=0) - 1.0 / K).max() <= 5 * sd
    assert np.allclose(X.mean(axis=0), C.mean(axis=0), atol=5 * sd * np.abs(C).max() * K)


def test_convex_workload():
    w = CONFIGS["C6"]
    assert w.sampler == "convex" and w.pert().shape == (w.n_scen, 3)
    C = base_cases(amplitude=w.amplitude)
    assert (w.pert().min(axis=0) >= C.min(axis=0) - 1e-15).all()
    assert (w.pert().max(axis=0) <= C.max(axis=0) + 1e-15).all()
