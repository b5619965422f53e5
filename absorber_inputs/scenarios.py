"""Scenario sampling, workload definitions and problem-size accounting.

The paper samples its scenarios as random convex combinations of seven measured
operating cases (Case study, problem setup); those measurements are not
published with the text.  Two synthetic stand-ins are provided, both drawn
from NumPy PCG64 generators with fixed seeds:

* iid uniform relative perturbations of the nominal flue-gas flow, CO2 mole
  fraction and inlet temperature (the benchmarked workloads);
* the paper's sampling scheme applied to seven synthetic base cases (relative
  perturbations drawn once from their own seed in place of the measurements):
  each scenario is a convex combination of the seven cases with weights drawn
  uniformly from the simplex (Dirichlet(1, ..., 1)).

N2 absorbs the change of the CO2 fraction so the gas fractions still sum to
one.  The feed table is affine in the perturbations, so a convex combination
of perturbations gives the same convex combination of the cases' feed rows.
"""

from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass

import numpy as np

NF = 18  # doubles per feed-table row, see the package docstring

_HERE = os.path.dirname(os.path.abspath(__file__))


def load_params(path: str | None = None) -> dict:
    """Return the problem constants (params.json) as a dict."""
    with open(path or os.path.join(_HERE, "params.json")) as fh:
        return json.load(fh)


def perturbations(n_scen: int, amplitude: float, seed: int) -> np.ndarray:
    """Relative perturbations u ~ U(-a, a) of (gas flow, y_CO2, T_gas), shape (S, 3).

    Row order is the scenario order.
    """
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, (n_scen, 3))


N_BASE_CASES = 7


def base_cases(seed: int = 6, amplitude: float = 0.20) -> np.ndarray:
    """Seven synthetic operating cases standing in for the paper's measured ones:
    relative perturbations (gas flow, y_CO2, T_gas), shape (7, 3)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, (N_BASE_CASES, 3))


def convex_combinations(cases: np.ndarray, n_scen: int, seed: int):
    """Scenarios as random convex combinations of the base cases: weights w
    (S, K) uniform on the simplex (Dirichlet(1, ..., 1)), perturbations w @ cases.
    Returns (perturbations (S, 3), weights (S, K))."""
    cases = np.asarray(cases, dtype=np.float64)
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(cases.shape[0]), n_scen)
    return w @ cases, w


def feed_table(pert: np.ndarray, params: dict | None = None) -> np.ndarray:
    """Build the (S, NF) feed table from relative perturbations (S, 3)."""
    p = params or load_params()
    pert = np.asarray(pert, dtype=np.float64).reshape(-1, 3)
    S = pert.shape[0]
    g, l = p["feed_gas"], p["feed_liquid"]
    F = np.zeros((S, NF), dtype=np.float64)
    F[:, 0] = g["V0"] * (1.0 + pert[:, 0])
    yC = g["y"][0] * (1.0 + pert[:, 1])
    F[:, 1] = yC
    F[:, 2] = g["y"][1]
    F[:, 4] = g["y"][3]
    F[:, 3] = 1.0 - yC - g["y"][1] - g["y"][3]  # N2 rebalances the sum
    F[:, 5] = g["T"] * (1.0 + pert[:, 2])  # relative in kelvin
    F[:, 6] = l["L"]
    F[:, 7:16] = np.asarray(l["x"], dtype=np.float64)[None, :]
    F[:, 16] = l["T"]
    F[:, 17] = p["P_abs"]
    return F


@dataclass(frozen=True)
class Workload:
    name: str
    n_stages: int
    n_scen: int
    amplitude: float
    seed: int
    description: str
    sampler: str = "uniform"  # "uniform": iid perturbations; "convex": combinations of the base cases

    def pert(self) -> np.ndarray:
        if self.sampler == "convex":
            return convex_combinations(base_cases(amplitude=self.amplitude), self.n_scen, self.seed)[0]
        return perturbations(self.n_scen, self.amplitude, self.seed)

    def feeds(self, params: dict | None = None) -> np.ndarray:
        return feed_table(self.pert(), params)


# The five workloads: sizes follow the paper's case study (10 stages, up to
# 5000 scenarios, problem-size paragraph of the numerical results).
CONFIGS = {
    "C1": Workload("C1", 8, 4, 0.10, 0, "8 stages x 4 scenarios, +-10%, seed 0"),
    "C2": Workload("C2", 10, 500, 0.10, 1, "10 stages x 500 scenarios, +-10%, seed 1"),
    "C3": Workload("C3", 10, 5000, 0.20, 2, "10 stages x 5000 scenarios, +-20%, seed 2"),
    "C4": Workload("C4", 10, 5000, 0.20, 3, "warm-start test instance, 10 x 5000, +-20%, seed 3"),
    # the paper's sampling scheme on synthetic base cases (seed 6, +-20%)
    "C6": Workload("C6", 10, 5000, 0.20, 7, "10 x 5000, convex combinations of 7 base cases, seed 7", "convex"),
}

# warm-start training data: 20000 single-scenario problems, +-20%, seed 4
TRAIN_SET = Workload("train", 10, 20000, 0.20, 4, "20000 single-scenario problems, seed 4")


def batch_problems(n_problems: int = 64, seed: int = 5, amplitude: float = 0.15,
                   n_min: int = 8, n_max: int = 60, s_min: int = 50, s_max: int = 2000):
    """Uneven batch of independent design problems.

    Returns a list of (n_stages, pert (S_p, 3)).  Stage counts are uniform in
    [n_min, n_max], scenario counts log-uniform in [s_min, s_max]; all draws come
    from one generator in problem order.
    """
    rng = np.random.default_rng(seed)
    n_st = rng.integers(n_min, n_max + 1, n_problems)
    s_cnt = np.rint(np.exp(rng.uniform(math.log(s_min), math.log(s_max), n_problems))).astype(int)
    out = []
    for p in range(n_problems):
        out.append((int(n_st[p]), rng.uniform(-amplitude, amplitude, (int(s_cnt[p]), 3))))
    return out


def dims(n_stages: int, n_scen: int) -> dict:
    """Problem-size accounting of the deterministic equivalent.

    Per stage: 30 variables (11 liquid and 11 vapour mole fractions, L, V, T and
    5 reaction extents), 9 of them fixed to zero (the vapour fractions of the 7
    non-volatile species and the liquid fractions of N2 and O2), 21 MESH
    equalities and 1 hydraulic inequality; plus the shared diameter.
    """
    N, S = int(n_stages), int(n_scen)
    return {
        "n_var_total": 30 * N * S + 1,
        "n_var_free": 21 * N * S + 1,
        "n_eq": 21 * N * S,
        "n_fixed": 9 * N * S,
        "n_ineq": N * S,
        "kkt_dim": 43 * N * S + 1,
    }
