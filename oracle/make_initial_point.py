"""Write the cold-start liquid composition into absorber_inputs/params.json.

TEST INFRASTRUCTURE / DATA SCRIPT: uses only the oracle and NumPy/SciPy.

The cold start gives every stage of every scenario the lean solvent as it
enters the column: its apparent composition (MEA, H2O, CO2) speciated by the
five liquid-phase equilibria R1-R5 at the inlet temperature, with ideal
activities (Case study: reactions, Kent-Eisenberg constants and ideal phases).
The speciated composition x solves

    sum_i nu_ir ln x_i = ln K_r(T)      r = 1..5
    sum_i x_i = 1
    the amine backbone, carbon and oxygen atoms keep their apparent ratios
    the liquid is electrically neutral

Run:  python -m oracle.make_initial_point
"""

from __future__ import annotations

import json
import os

import numpy as np
from scipy.optimize import least_squares

from absorber_inputs import load_params

from . import model as M

O_ATOMS = np.array([1, 1, 0, 3, 3, 1, 3, 2, 1])  # O atoms in the 9 liquid species
CHARGE = np.array([0, 1, 1, -1, -1, -1, -2, 0, 0])


def speciate(params: dict) -> np.ndarray:
    P = M.OracleParams(params)
    nu = P.nu.numpy()[:M.NLIQ]
    T = params["feed_liquid"]["T"]
    lnK = (P.A + P.B / T + P.C * np.log(T) + P.D * T).numpy()
    xa = np.asarray(params["feed_liquid"]["x"], dtype=np.float64)
    amine0 = xa[0] + xa[1] + xa[3]
    carbon0 = xa[3] + xa[4] + xa[6] + xa[7]
    oxy0 = O_ATOMS @ xa

    def res(lx):
        x = np.exp(lx)
        amine = x[0] + x[1] + x[3]
        carbon = x[3] + x[4] + x[6] + x[7]
        return np.concatenate([nu.T @ lx - lnK,
                               [x.sum() - 1.0,
                                amine / carbon - amine0 / carbon0,
                                amine / (O_ATOMS @ x) - amine0 / oxy0,
                                CHARGE @ x]])

    guess = np.log(np.array([0.07, 0.02, 1e-12, 0.02, 2e-4, 1e-6, 5e-5, 1e-7, 0.87]))
    sol = least_squares(res, guess, xtol=1e-15, ftol=1e-15, gtol=1e-15)
    if np.abs(res(sol.x)).max() > 1e-12:
        raise RuntimeError("speciation did not converge")
    return np.exp(sol.x)


def main():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "absorber_inputs", "params.json")
    p = load_params(path)
    x = speciate(p)
    text = open(path).read()
    old = json.dumps(p["initial_point"]["x"])
    new = json.dumps([float(v) for v in x])
    text = text.replace('"x": ' + old, '"x": ' + new, 1) if old in text else text
    with open(path, "w") as fh:
        fh.write(text)
    print("initial liquid composition:", new)


if __name__ == "__main__":
    main()
