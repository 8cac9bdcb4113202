"""Pins of the oracle's closed forms and tables against mathematics that fixes them (CPU).

Each check is independent of the oracle's own arithmetic: an integral of the
differential form against the closed total, a textbook limit, a symmetry, the
derivative relation tying the restricted stopping power to the delta-ray cross
section, or adaptive quadrature of a tabulated integral.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W

ME = 0.51099895
RE = 2.8179403262e-13
NA = 6.02214076e23


def quad(f, a, b, **kw):
    v, err = integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-12, limit=400, **kw)
    return v


@pytest.mark.parametrize("E", [0.02, 0.1, 1.0, 10.0, 1e3, 1e5])
def test_kn_total_is_integral_of_differential(orc, E):
    k = E / ME
    e0 = 1.0 / (1.0 + 2.0 * k)
    tot = quad(lambda e: orc.closed("kn_dsigma", E, e), e0, 1.0, points=None)
    assert tot == pytest.approx(orc.closed("kn_sigma", E), rel=1e-9)


def test_kn_limits(orc):
    thomson = 8.0 * math.pi / 3.0 * RE ** 2
    # Thomson limit k -> 0: sigma = sigma_T (1 - 2k + ...)
    E = 1e-4 * ME
    assert orc.closed("kn_sigma", E) == pytest.approx(thomson * (1 - 2e-4), rel=1e-6)
    # forward scattering (eps = 1) is Thomson's r_e^2 per steradian: d sigma/d eps at eps=1
    # equals (pi r_e^2/k) * 2
    E = 3.0
    assert orc.closed("kn_dsigma", E, 1.0) == pytest.approx(2 * math.pi * RE ** 2 / (E / ME), rel=1e-14)
    # ultra-relativistic: sigma -> pi r_e^2 (ln 2k + 1/2)/k
    E = 1e6
    k = E / ME
    assert orc.closed("kn_sigma", E) == pytest.approx(math.pi * RE ** 2 * (math.log(2 * k) + 0.5) / k,
                                                      rel=1e-5)


def test_photoelectric_law(orc):
    # the configured law: 1e-6 barn * Z^5 * (100 keV / E)^3.5
    assert orc.closed("pe_sigma", 82.0, 0.1) == pytest.approx(1e-30 * 82.0 ** 5, rel=1e-15)
    r = orc.closed("pe_sigma", 18.0, 0.2) / orc.closed("pe_sigma", 18.0, 0.1)
    assert r == pytest.approx(2.0 ** -3.5, rel=1e-14)


@pytest.mark.parametrize("E", [1.2, 2.0, 10.0, 1e3, 1e5])
def test_pair_total_is_integral(orc, E):
    X0 = 0.5
    a = ME / E
    tot = quad(lambda x: orc.closed("pair_dSigma", X0, E, x), a, 1 - a)
    assert tot == pytest.approx(orc.closed("pair_Sigma", X0, E), rel=1e-10)


def test_pair_limits(orc):
    X0 = 0.7
    # high-energy limit 7/(9 X0); zero at and below threshold
    assert orc.closed("pair_Sigma", X0, 1e9) == pytest.approx(7.0 / 9.0 / X0, rel=1e-8)
    assert orc.closed("pair_Sigma", X0, 2 * ME) == 0.0
    assert orc.closed("pair_Sigma", X0, 2 * ME * (1 + 1e-9)) > 0.0


@pytest.mark.parametrize("T,kc", [(0.05, 0.011), (1.0, 0.117), (1e3, 0.1), (1e5, 1.0)])
def test_brems_total_and_soft_loss(orc, T, kc):
    X0 = 0.556
    tot = quad(lambda k: orc.closed("brems_dSigma", X0, T, k), kc, T)
    assert tot == pytest.approx(orc.closed("brems_Sigma", X0, T, kc), rel=1e-10)
    soft = quad(lambda k: k * orc.closed("brems_dSigma", X0, T, k), 0.0, kc)
    assert soft == pytest.approx(orc.closed("brems_Srad", X0, T, kc), rel=1e-10)


def test_brems_defines_radiation_length(orc):
    # all radiated energy per unit length = T / X0 in this spectrum
    for T in (0.1, 10.0, 1e4):
        assert orc.closed("brems_Srad", 0.3, T, T) == pytest.approx(T / 0.3, rel=1e-14)


@pytest.mark.parametrize("T,Tc", [(0.1, 0.02), (1.0, 0.265), (30.0, 1.02), (1e4, 0.5)])
def test_moller_total_and_symmetry(orc, T, Tc):
    tot = quad(lambda e: orc.closed("moller_dsigma", T, e), Tc / T, 0.5)
    assert tot == pytest.approx(orc.closed("moller_sigma", T, Tc), rel=1e-10)
    # identical particles: symmetric under eps <-> 1 - eps
    for e in (0.01, 0.1, 0.3):
        assert orc.closed("moller_dsigma", T, e) == pytest.approx(orc.closed("moller_dsigma", T, 1 - e),
                                                                  rel=1e-12)


@pytest.mark.parametrize("T,Tc", [(0.1, 0.02), (1.0, 0.265), (30.0, 1.02), (1e4, 0.5)])
def test_bhabha_total(orc, T, Tc):
    tot = quad(lambda e: orc.closed("bhabha_dsigma", T, e), Tc / T, 1.0)
    assert tot == pytest.approx(orc.closed("bhabha_sigma", T, Tc), rel=1e-10)


def test_bhabha_ultrarelativistic_form(orc):
    # beta -> 1: the bracket tends to (1/eps - 1 + eps)^2
    T = 1e7
    pref = 2 * math.pi * RE ** 2 * ME / T
    for e in (0.05, 0.3, 0.9):
        assert orc.closed("bhabha_dsigma", T, e) / pref == pytest.approx((1 / e - 1 + e) ** 2, rel=1e-6)


@pytest.mark.parametrize("T", [0.02, 0.5, 10.0, 1e4])
def test_heitler_total_is_half_range_integral(orc, T):
    g = T / ME + 1
    emin = 0.5 * (1 - math.sqrt((g - 1) / (g + 1)))
    Z = 82.0
    tot = quad(lambda e: orc.closed("heitler_dsigma", Z, T, e), emin, 1 - emin)
    # the photon-1 spectrum over the full range counts each annihilation once
    assert tot == pytest.approx(orc.closed("heitler_sigma", Z, T), rel=1e-9)


def test_heitler_high_energy_limit(orc):
    T = 1e6
    g = T / ME + 1
    Z = 18.0
    lim = Z * math.pi * RE ** 2 / g * (math.log(2 * g) - 1)
    assert orc.closed("heitler_sigma", Z, T) == pytest.approx(lim, rel=1e-4)


@pytest.mark.parametrize("positron", [0, 1])
@pytest.mark.parametrize("T,cut", [(0.2, 0.03), (2.0, 0.3), (50.0, 1.0), (5e3, 1.02)])
def test_restricted_stopping_power_tied_to_delta_cross_section(orc, positron, T, cut):
    """dS/d(cut) = n_el * cut * d sigma/d T_delta at T_delta = cut, and the restricted
    plus the hard-collision integral equals the unrestricted stopping power."""
    n_el, I = 2.7e24, 823e-6
    h = cut * 1e-5
    dS = (orc.closed("scol", positron, n_el, I, T, cut + h) -
          orc.closed("scol", positron, n_el, I, T, cut - h)) / (2 * h)
    ds_name = "bhabha_dsigma" if positron else "moller_dsigma"
    expect = n_el * cut * orc.closed(ds_name, T, cut / T) / T
    assert dS == pytest.approx(expect, rel=1e-6)
    tmax = T if positron else T / 2
    hard = quad(lambda td: n_el * td * orc.closed(ds_name, T, td / T) / T, cut, tmax)
    unres = orc.closed("scol", positron, n_el, I, T, 10 * T)
    assert orc.closed("scol", positron, n_el, I, T, cut) + hard == pytest.approx(unres, rel=1e-9)


@pytest.mark.parametrize("positron", [0, 1])
@pytest.mark.parametrize("T", [0.012, 0.3, 5.0, 200.0, 1e4])
@pytest.mark.parametrize("I", [823e-6, 188e-6])
def test_restricted_at_largest_cut_is_unrestricted_icru37(orc, positron, T, I):
    """With the cut at the largest energy transfer (T/2 for e-, T for e+) the restricted
    collision stopping power is the unrestricted ICRU 37 (Berger-Seltzer) formula, written
    here in its own standard form:  S = 2 pi r_e^2 m n_el / beta^2 [ln(tau^2 (tau+2) / (2 I^2))
    + F(tau)], F- = 1 - beta^2 + (tau^2/8 - (2 tau + 1) ln 2)/(tau+1)^2,
    F+ = 2 ln 2 - beta^2/12 (23 + 14/(tau+2) + 10/(tau+2)^2 + 4/(tau+2)^3)."""
    n_el = 2.7e24
    tau = T / ME
    g = tau + 1.0
    b2 = 1.0 - 1.0 / (g * g)
    Im = I / ME
    if positron:
        y = tau + 2.0
        F = 2 * math.log(2) - b2 / 12 * (23 + 14 / y + 10 / y ** 2 + 4 / y ** 3)
    else:
        F = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (g * g)
    S = 2 * math.pi * RE ** 2 * ME * n_el / b2 * (math.log(tau * tau * (tau + 2) / (2 * Im * Im)) + F)
    cut = T if positron else T / 2
    assert orc.closed("scol", positron, n_el, I, T, cut) == pytest.approx(S, rel=1e-12)


def test_stopping_power_cut_saturates(orc):
    n_el, I = 1e24, 188e-6
    T = 3.0
    e = orc.closed("scol", 0, n_el, I, T, T / 2)
    assert orc.closed("scol", 0, n_el, I, T, T) == e
    p = orc.closed("scol", 1, n_el, I, T, T)
    assert orc.closed("scol", 1, n_el, I, T, 5 * T) == p


def test_radiation_length_pdg_fit(orc):
    # the PDG fit 716.4 A / (Z (Z+1) ln(287/sqrt Z)) g/cm^2 agrees with Tsai's tabulated
    # radiation lengths (lead 6.37, argon 19.55 g/cm^2) to better than 2.5%
    x0 = orc.closed("radiation_length", 82.0, 207.2, 1.0)
    assert x0 == pytest.approx(6.37, rel=0.025)
    x0 = orc.closed("radiation_length", 18.0, 39.948, 1.0)
    assert x0 == pytest.approx(19.55, rel=0.025)


@pytest.mark.parametrize("name,params", [
    ("kn", [0.011, 0.1, 1.0, 10.0, 1e3, 1e5]),
    ("moller", [0.05, 1.0, 100.0, 1e5]),
    ("bhabha", [0.05, 1.0, 100.0, 1e5]),
    ("heitler", [0.011, 0.5, 10.0, 1e5]),
])
def test_acceptance_ratios_within_unit_interval(orc, name, params):
    for T in params:
        if name == "kn":
            k = T / ME
            lo, hi = 1 / (1 + 2 * k), 1.0
        elif name == "moller":
            lo, hi = 1e-6, 0.5
        elif name == "bhabha":
            lo, hi = 1e-6, 1.0
        else:
            g = T / ME + 1
            lo = 0.5 * (1 - math.sqrt((g - 1) / (g + 1)))
            hi = 1 - lo
        for e in np.linspace(lo, hi, 2001):
            a = orc.closed("accept_" + name, T, float(e))
            assert -1e-12 <= a <= 1 + 1e-12, (name, T, e, a)


# ------------------------------------------------------------------ tables

@pytest.fixture(scope="module")
def cal_world(orc):
    wl = W.calorimeter(1)
    return orc.World(wl.materials, wl.options, wl.geometry), wl


def test_grid(cal_world):
    w, _ = cal_world
    assert w.grid_energy(0) == pytest.approx(1e-3, rel=1e-15)
    assert w.grid_energy(199) == pytest.approx(1e5, rel=1e-13)
    assert w.grid_energy(99) * (1e8 ** (0.5 / 199)) == pytest.approx(10.0 ** (-3 + 8 * 99.5 / 199), rel=1e-13)


def test_table_nodes_are_closed_forms(orc, cal_world):
    w, wl = cal_world
    for m, (Z, A, rho, I) in enumerate(wl.materials):
        n_at = rho * NA / A
        X0 = orc.closed("radiation_length", Z, A, rho)
        Tc, kc = w.cut_electron(m), w.cut_gamma(m)
        for i in (10, 57, 99, 150, 199):
            E = w.grid_energy(i)
            assert w.node(m, 0, 0, i) == pytest.approx(Z * n_at * orc.closed("kn_sigma", E), rel=1e-15)
            assert w.node(m, 0, 1, i) == pytest.approx(n_at * orc.closed("pe_sigma", Z, E), rel=1e-15)
            assert w.node(m, 0, 2, i) == pytest.approx(orc.closed("pair_Sigma", X0, E), rel=1e-15)
            assert w.node(m, 1, 0, i) == pytest.approx(Z * n_at * orc.closed("moller_sigma", E, Tc), rel=1e-15)
            assert w.node(m, 1, 1, i) == pytest.approx(orc.closed("brems_Sigma", X0, E, kc), rel=1e-15)
            assert w.node(m, 2, 0, i) == pytest.approx(Z * n_at * orc.closed("bhabha_sigma", E, Tc), rel=1e-15)
            assert w.node(m, 2, 2, i) == pytest.approx(n_at * orc.closed("heitler_sigma", Z, E), rel=1e-15)


def test_interpolation_is_linear_in_log_energy(cal_world):
    """Mid-interval photoelectric value: PE ~ E^-3.5 = exp(-3.5 ln E), so the linear-in-ln E
    midpoint over-estimates by exactly cosh(3.5 Delta/2)."""
    w, wl = cal_world
    d = math.log(1e8) / 199
    for i in (30, 80, 120):
        Em = math.sqrt(w.grid_energy(i) * w.grid_energy(i + 1))
        ratio = w.interp(0, 0, 1, Em) / (w.node(0, 0, 1, i) * math.exp(-3.5 * d / 2))
        assert ratio == pytest.approx(math.cosh(3.5 * d / 2), rel=1e-12)


def test_range_table_against_adaptive_quadrature(orc, cal_world):
    w, wl = cal_world
    for m, (Z, A, rho, I) in enumerate(wl.materials):
        n_el = Z * rho * NA / A
        X0 = orc.closed("radiation_length", Z, A, rho)
        Tc, kc = w.cut_electron(m), w.cut_gamma(m)
        for s, pos in ((1, 0), (2, 1)):
            def S(T):
                return orc.closed("scol", pos, n_el, I, T, Tc) + orc.closed("brems_Srad", X0, T, T if kc > T else kc)
            for i in (30, 100, 199):
                Ei = w.grid_energy(i)
                R = quad(lambda l: math.exp(l) / S(math.exp(l)), math.log(1e-3), math.log(Ei))
                assert w.node(m, s, 3, i) == pytest.approx(R, rel=1e-9)


def test_range_inverse_round_trip(cal_world):
    w, _ = cal_world
    for T in (0.0123, 0.7, 13.0, 999.0):
        r = w.interp(0, 1, 3, T)
        assert w.range_inverse(0, 1, r) == pytest.approx(T, rel=1e-13)


def test_production_thresholds(orc, cal_world):
    """e+- threshold: unrestricted CSDA range equals the 0.7 mm cut (within the linear-in-ln T
    interpolation of the range); photon threshold: 5 mean free paths equal the cut."""
    w, wl = cal_world
    L = wl.options.production_cut
    for m, (Z, A, rho, I) in enumerate(wl.materials):
        n_at = rho * NA / A
        n_el = Z * n_at
        X0 = orc.closed("radiation_length", Z, A, rho)
        Tc = w.cut_electron(m)
        R = quad(lambda l: math.exp(l) / (orc.closed("scol", 0, n_el, I, math.exp(l), 1e9) + math.exp(l) / X0),
                 math.log(1e-3), math.log(Tc))
        assert R == pytest.approx(L, rel=2e-3)
        kc = w.cut_gamma(m)
        if kc > 0.010001:
            sig = n_el * orc.closed("kn_sigma", kc) + n_at * orc.closed("pe_sigma", Z, kc) + orc.closed("pair_Sigma", X0, kc)
            assert 5.0 / sig == pytest.approx(L, rel=2e-2)
