"""Chi-square of the oracle's interaction samplers against their analytic spectra (CPU).

Each sampler is fed independent uniforms from numpy's seeded generator; the
histogram of the sampled variable is compared with the differential cross
section integrated over each bin.  A mistake in an envelope, an acceptance
ratio or a variable change shows up as a chi-square far above the number of
degrees of freedom.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

ME = 0.51099895
N = 40000


def _draw(orc, name, params, rng, n=N):
    out = np.empty(n)
    for i in range(n):
        u = rng.random(256)
        v, used = orc.sample(name, params, u)
        assert used > 0
        out[i] = v[0] if isinstance(v, tuple) else v
    return out


def _chi2(samples, edges, pdf):
    counts, _ = np.histogram(samples, edges)
    w = np.array([integrate.quad(pdf, a, b, epsrel=1e-10)[0] for a, b in zip(edges[:-1], edges[1:])])
    expect = w / w.sum() * len(samples)
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    dof = len(counts) - 1
    return chi2, dof, stats.chi2.sf(chi2, dof)


@pytest.mark.parametrize("E", [0.05, 1.0, 100.0])
def test_klein_nishina_spectrum(orc, E):
    rng = np.random.default_rng(11)
    s = _draw(orc, "kn", [E], rng)
    e0 = 1 / (1 + 2 * E / ME)
    edges = np.exp(np.linspace(math.log(e0), 0.0, 31))
    chi2, dof, p = _chi2(s, edges, lambda e: orc.closed("kn_dsigma", E, e))
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("E", [1.5, 10.0, 1e4])
def test_pair_spectrum(orc, E):
    rng = np.random.default_rng(12)
    s = _draw(orc, "pair", [E], rng)
    a = ME / E
    edges = np.linspace(a, 1 - a, 31)
    chi2, dof, p = _chi2(s, edges, lambda x: orc.closed("pair_dSigma", 1.0, E, x))
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("T,kc", [(2.0, 0.117), (1000.0, 0.0118)])
def test_brems_spectrum(orc, T, kc):
    rng = np.random.default_rng(13)
    s = _draw(orc, "brems", [T, kc], rng)
    edges = np.exp(np.linspace(math.log(kc), math.log(T), 31))
    chi2, dof, p = _chi2(s, edges, lambda k: orc.closed("brems_dSigma", 1.0, T, k))
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("T,Tc", [(3.0, 0.265), (1000.0, 1.02)])
def test_moller_spectrum(orc, T, Tc):
    rng = np.random.default_rng(14)
    s = _draw(orc, "moller", [T, Tc], rng)
    edges = 1.0 / np.linspace(T / Tc, 2.0, 31)
    chi2, dof, p = _chi2(s, edges, lambda e: orc.closed("moller_dsigma", T, e))
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("T,Tc", [(3.0, 0.265), (1000.0, 1.02)])
def test_bhabha_spectrum(orc, T, Tc):
    rng = np.random.default_rng(15)
    s = _draw(orc, "bhabha", [T, Tc], rng)
    edges = 1.0 / np.linspace(T / Tc, 1.0, 31)
    chi2, dof, p = _chi2(s, edges, lambda e: orc.closed("bhabha_dsigma", T, e))
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("T", [0.3, 50.0])
def test_annihilation_spectrum(orc, T):
    rng = np.random.default_rng(16)
    s = _draw(orc, "heitler", [T], rng)
    g = T / ME + 1
    emin = 0.5 * (1 - math.sqrt((g - 1) / (g + 1)))
    edges = np.exp(np.linspace(math.log(emin), math.log(1 - emin), 31))
    chi2, dof, p = _chi2(s, edges, lambda e: orc.closed("heitler_dsigma", 1.0, T, e))
    assert p > 1e-4, (chi2, dof)


def test_sampler_reports_short_draw_supply(orc):
    v, used = orc.sample("pair", [10.0], np.array([0.5]))
    assert used == -1
