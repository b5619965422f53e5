"""Pins of the oracle's residual forms against physical anchors.

Each test builds a stage state for which a textbook fact fixes the value of
one row of the equilibrium model (the row must vanish, or change by a known
amount), so a wrong species index, a wrong sign, a wrong temperature or a
dropped term in that row fails here:

* reaction equilibrium (3a): at a pH equal to a pK the acid and its conjugate
  base are present in equal amounts; neutral water has equal H+ and OH-;
  van 't Hoff with the reaction enthalpies fixes the temperature dependence;
* Raoult's law (9a): water boils at 373.15 K under 101325 Pa and has a vapour
  pressure of 7.38 kPa at 313.15 K;
* Henry's law (9b): CO2 dissolves in water at 25 C with 0.034 mol/(L atm); its
  Henry constant rises with temperature (2400 K van 't Hoff slope) and with the
  amine fraction (the N2O analogy ratio of the readings);
* energy balance (6): summed over a column with Q = 0 the stage balances
  telescope to enthalpy in = enthalpy out, which the converged C1 states must
  satisfy with enthalpies computed here from the component data;
* physical direction of the converged profiles: gas CO2 falls from the bottom
  to the top of the column and the liquid CO2 loading rises downwards.
"""

import math

import numpy as np
import pytest
import torch

from absorber_inputs import CONFIGS, feed_table
from oracle import ipm
from oracle import model as M

LN10 = math.log(10.0)
C_LIQ = 43.0  # mol/L, total liquid molarity of the mole-fraction reading of the K values
MEA, MEAH, H, MEACOO, HCO3, OH, CO3, CO2, H2O = range(9)


def stage_rows(params, x, T, y=None, P=101325.0):
    """All 22 rows of a one-stage column at liquid fractions x (9), vapour y (4), T."""
    Z = np.zeros((1, M.NV))
    Z[0, 0:9] = x
    Z[0, 9:13] = y if y is not None else [0.1, 0.1, 0.7, 0.1]
    Z[0, M.IL], Z[0, M.IV], Z[0, M.IT] = 40.0, 10.0, T
    feed = feed_table(np.zeros((1, 3)), params)[0].copy()
    feed[17] = P
    P_ = M.OracleParams(params)
    return M.scenario_constraints(torch.from_numpy(Z), torch.tensor(1.0, dtype=torch.float64),
                                  torch.from_numpy(feed), P_).numpy()[0]


def liquid(**kw):
    """A liquid composition with every species at a distinct small value, then kw."""
    x = np.array([0.011, 0.013, 0.017, 0.019, 0.023, 0.029, 0.031, 0.037, 0.8])
    for k, v in kw.items():
        x[globals()[k]] = v
    return x


# ---------------------------------------------------------------- (3a)
def test_r1_amine_protonation_at_its_pka(params):
    # MEAH+ = MEA + H+ with pKa 9.50 at 298.15 K: equal MEA and MEAH+ at x_H+ = Ka
    x = liquid(MEA=0.05, MEAH=0.05, H=10 ** -9.50 / C_LIQ)
    assert abs(stage_rows(params, x, 298.15)[11]) < 1e-10


def test_r2_bicarbonate_dissociation_at_its_pka(params):
    # HCO3- = H+ + CO3-- with pKa2 10.33
    x = liquid(HCO3=0.02, CO3=0.02, H=10 ** -10.33 / C_LIQ)
    assert abs(stage_rows(params, x, 298.15)[12]) < 1e-10


def test_r3_neutral_water(params):
    # pure water at 298.15 K: [H+] = [OH-] = 1e-7 mol/L, 55.5 mol/L of water
    x = liquid(H2O=1.0, H=1e-7 / 55.5, OH=1e-7 / 55.5)
    assert abs(stage_rows(params, x, 298.15)[13]) < 1e-10


def test_r4_carbamate_reversion_constant(params):
    # MEACOO- + H2O = MEA + HCO3- with K = 0.033 mol/L on a 0.87 water fraction
    # basis: [MEA][HCO3-]/[MEACOO-] = 0.033 mol/L at x_H2O = 0.87
    x = liquid(H2O=0.87, MEACOO=0.02, MEA=0.02, HCO3=0.033 / C_LIQ)
    assert abs(stage_rows(params, x, 298.15)[14]) < 1e-10


def test_r5_co2_hydration_at_its_pka(params):
    # H2O + CO2 = H+ + HCO3- with pKa1 6.35: equal CO2 and HCO3- at [H+] = Ka1
    x = liquid(H2O=0.87, CO2=0.01, HCO3=0.01, H=10 ** -6.35 / C_LIQ)
    assert abs(stage_rows(params, x, 298.15)[15]) < 1e-10


@pytest.mark.parametrize("r,dH", [(0, 50.0e3), (1, 14.7e3), (2, 55.8e3), (3, 20.0e3), (4, 9.2e3)])
def test_reaction_rows_follow_van_t_hoff(params, r, dH):
    # d ln K / d(1/T) = -dH / R: the row sum nu ln x - ln K(T) at fixed x falls by
    # dH / R (1/T1 - 1/T2) from T1 to T2 (all five reactions are endothermic)
    x = liquid()
    T1, T2 = 298.15, 333.15
    drop = stage_rows(params, x, T1)[11 + r] - stage_rows(params, x, T2)[11 + r]
    assert drop == pytest.approx(dH / params["R"] * (1 / T1 - 1 / T2), rel=1e-12)


def test_reaction_rows_use_the_right_species(params):
    # doubling one species' fraction moves ln x_i by ln 2 in exactly the reactions
    # it takes part in, with its stoichiometric sign (products +, reactants -)
    base = stage_rows(params, liquid(), 310.0)[11:16]
    nu = np.array(params["nu"], dtype=float)
    for i in range(9):
        x = liquid()
        x[i] *= 2.0
        moved = stage_rows(params, x, 310.0)[11:16] - base
        assert np.allclose(moved, nu[i] * math.log(2.0), atol=1e-12), i


# ---------------------------------------------------------------- (9a), (9b)
def test_raoult_water_boils_at_one_atmosphere(params):
    x = liquid(H2O=0.8)
    r = stage_rows(params, x, 373.15, y=[0.05, 0.8, 0.1, 0.05], P=101325.0)
    assert abs(r[18]) / 101325.0 < 1e-9
    # 313.15 K, 2 atm: y_H2O = x_H2O 7380 Pa / P
    P = 2 * 101325.0
    r = stage_rows(params, x, 313.15, y=[0.05, 0.8 * 7380.0 / P, 0.5, 0.1], P=P)
    assert abs(r[18]) / P < 1e-9


def test_henry_co2_in_water(params):
    # 0.034 mol/(L atm) in 55.5 mol/L of water: H = 55.5 / 0.034 atm (within the
    # 1 % of the rounded textbook figure), and the row vanishes at P y = x H
    H_book = 55.5 / 0.034 * 101325.0
    H298 = math.exp(params["henry_lnH298"])
    assert abs(H298 - H_book) / H_book < 0.01
    x = liquid(MEA=0.0, MEAH=0.0, MEACOO=0.0, H2O=0.98, CO2=1e-4)
    P = 101325.0
    r = stage_rows(params, x, 298.15, y=[1e-4 * H298 / P, 0.03, 0.9, 0.05], P=P)
    assert abs(r[19]) / P < 1e-12


def test_henry_rises_with_temperature_and_amine(params):
    H298 = math.exp(params["henry_lnH298"])
    P = 101325.0
    # 323.15 K in water: H = H298 exp(2400 (1/298.15 - 1/323.15))
    x = liquid(MEA=0.0, MEAH=0.0, MEACOO=0.0, H2O=0.98, CO2=1e-4)
    H323 = H298 * math.exp(2400.0 * (1 / 298.15 - 1 / 323.15))
    r = stage_rows(params, x, 323.15, y=[1e-4 * H323 / P, 0.03, 0.9, 0.05], P=P)
    assert abs(r[19]) / P < 1e-12
    assert 1.5 < H323 / H298 < 2.2  # CO2 is about half as soluble at 50 C as at 25 C
    # half of the apparent solvent is amine: ln H gains half of ln 1.3
    x = liquid(MEA=0.1, MEAH=0.1, MEACOO=0.1, H2O=0.3, CO2=1e-4)
    Hmix = H298 * 1.3 ** 0.5
    r = stage_rows(params, x, 298.15, y=[1e-4 * Hmix / P, 0.03, 0.9, 0.05], P=P)
    assert abs(r[19]) / P < 1e-12


def test_vaporisation_enthalpy_of_water(params):
    # h^V_H2O - h^L_H2O at 298.15 K is the heat of vaporisation, 43.99 kJ/mol
    dh = params["hV_ref"][1] - params["hL_ref"][8]
    assert dh == pytest.approx(43.99e3, rel=1e-3)


# ---------------------------------------------------------------- (6), profiles
def _h(T, href, a, b, Tref):
    return np.asarray(href) + np.asarray(a) * (T - Tref) + 0.5 * np.asarray(b) * (T * T - Tref * Tref)


@pytest.fixture(scope="module")
def c1_solution(params):
    w = CONFIGS["C1"]
    F = w.feeds(params)
    r = ipm.solve(params, F, w.n_stages)
    assert r.status == ipm.SUCCESS
    return F, r.x[:-1].reshape(F.shape[0], w.n_stages, M.NV)


def test_column_enthalpy_closure(params, c1_solution):
    # Q = 0: liquid in at the top (lean solvent at T_liq) plus gas in at the
    # bottom (flue gas at T_gas) carry the enthalpy of liquid out at the bottom
    # plus gas out at the top
    F, Z = c1_solution
    Tr = params["Tref"]
    hL = lambda x, T: float(x @ _h(T, params["hL_ref"], params["cpL_a"], params["cpL_b"], Tr))  # noqa: E731
    hV = lambda y, T: float(y @ _h(T, params["hV_ref"], params["cpV_a"], params["cpV_b"], Tr))  # noqa: E731
    for s in range(F.shape[0]):
        f = F[s]
        h_in = f[6] * hL(f[7:16], f[16]) + f[0] * hV(f[1:5], f[5])
        bot, top = Z[s, 0], Z[s, -1]
        h_out = bot[M.IL] * hL(bot[0:9], bot[M.IT]) + top[M.IV] * hV(top[9:13], top[M.IT])
        scale = abs(f[6] * hL(f[7:16], f[16])) + abs(f[0] * hV(f[1:5], f[5]))
        assert abs(h_in - h_out) <= 1e-9 * scale, (s, h_in, h_out)


def test_profiles_point_the_physical_way(params, c1_solution):
    F, Z = c1_solution
    for s in range(F.shape[0]):
        yco2 = Z[s, :, 9]
        assert np.all(np.diff(yco2) < 0), yco2          # gas CO2 absorbed on the way up
        assert yco2[0] < F[s, 1]                        # already below the feed on stage 1
        x = Z[s, :, 0:9]
        loading = (x[:, CO2] + x[:, MEACOO] + x[:, HCO3] + x[:, CO3]) / (x[:, MEA] + x[:, MEAH] + x[:, MEACOO])
        assert np.all(np.diff(loading) < 0), loading    # rich at the bottom, lean at the top
        lean = F[s, 7:16]
        assert loading[-1] > lean[CO2] / lean[MEA]      # the top stage already absorbed some
        # water: every stage's y_H2O P / x_H2O is the vapour pressure at its own T,
        # between the column's coldest and hottest stage values
        T = Z[s, :, M.IT]
        ps = lambda TT: math.exp(params["psat_a"] - params["psat_b"] / TT)  # noqa: E731
        ratio = Z[s, :, 10] * F[s, 17] / x[:, H2O]
        assert np.all(ratio >= ps(T.min()) * (1 - 1e-9)) and np.all(ratio <= ps(T.max()) * (1 + 1e-9))
