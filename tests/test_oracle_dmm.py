"""Pins of the pitch-angle diffusion models (section 2.1, Eq. 5, and the power
law of the synthetic workloads) and of their normalisation by lambda_par."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import fte_workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _g(model, mu, q, eps):
    am = abs(mu)
    if model == "iso":
        return 1 - mu * mu
    if model == "eq5":
        return (am / (1 + am) + eps) * (1 - mu * mu)
    return (1 - mu * mu) * am ** (q - 1)


@pytest.mark.parametrize("model,q,eps", [("iso", 0, 0), ("eq5", 0, GOLD["eps_resonance_gap"]["value"]),
                                         ("eq5", 0, 0.2), ("power_q", 5 / 3, 0), ("power_q", 1.3, 0)])
def test_normalisation_integral_by_quadrature(orc, model, q, eps):
    # I = Int_{-1}^{1} (1-mu^2)^2 / g(mu) dmu from the definition, by adaptive quadrature
    f = lambda m: (1 - m * m) ** 2 / _g(model, m, q, eps)
    pts = [0.0] if model != "iso" else None
    val = integrate.quad(f, -1, 0, limit=200, points=None)[0] + integrate.quad(f, 0, 1, limit=200)[0]
    del pts
    assert orc.dmm_integral(model, q, eps) == pytest.approx(val, rel=1e-9)


def test_paper_eq5_scale(orc):
    # with the paper's eps (section 2.1, Eq. 5) the MFP-consistent scale is
    # D0 = 3 v I / (8 lambda); I from quadrature of the definition
    eps = GOLD["eps_resonance_gap"]["value"]
    f = lambda m: (1 - m) * (1 + m) ** 2 / ((1 + eps) * m + eps)
    I = 2 * integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert orc.dmm_integral("eq5", 0, eps) == pytest.approx(I, rel=1e-12)
    assert 2.2 < 3 * I / 8 < 2.4


@pytest.mark.parametrize("model", ["iso", "eq5", "power_q"])
def test_mean_free_path_recovered(orc, model):
    # kappa_par = (v^2/8) Int (1-mu^2)^2 / D dmu and lambda = 3 kappa / v must
    # give back lambda_ref, using the oracle's own D(mu)
    P = 0.0146
    v = W.C_LIGHT * P / math.sqrt(1 + P * P)
    lam = 0.3 * W.AU
    p = dict(mass=W.M_P, dmm_model=model, lambda_ref=lam, q=5 / 3, eps=0.048, dt=1.0)
    f = lambda m: (1 - m * m) ** 2 / orc.dmm(p, P, m)[0]
    I = integrate.quad(f, -1, 0, limit=400)[0] + integrate.quad(f, 0, 1, limit=400)[0]
    kappa = v * v / 8 * I
    assert 3 * kappa / v == pytest.approx(lam, rel=1e-7)


@pytest.mark.parametrize("model", ["iso", "eq5", "power_q"])
def test_dmm_derivative(orc, model):
    P = 0.0146
    p = dict(mass=W.M_P, dmm_model=model, lambda_ref=0.3 * W.AU, q=5 / 3, eps=0.048, dt=1.0)
    for mu in [-0.93, -0.5, -0.11, 0.07, 0.33, 0.8, 0.999]:
        h = 1e-6
        fd = (orc.dmm(p, P, mu + h)[0] - orc.dmm(p, P, mu - h)[0]) / (2 * h)
        assert orc.dmm(p, P, mu)[1] == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # sgn(0) = 0: the drift vanishes at mu = 0 by symmetry
    assert orc.dmm(p, P, 0.0)[1] == 0.0


def test_power_q_floor(orc):
    # |mu|^(q-2) is evaluated with |mu| floored at mu_floor; D itself is not
    P = 0.0146
    p = dict(mass=W.M_P, dmm_model="power_q", lambda_ref=0.3 * W.AU, q=5 / 3, mu_floor=1e-4, dt=1.0)
    d_small = orc.dmm(p, P, 1e-7)[1]
    d_floor = orc.dmm(p, P, 1e-4)[1]
    assert d_small == pytest.approx(d_floor, rel=1e-2)
    assert np.isfinite(d_small)


def test_literal_prefactor(orc):
    P = 0.0146
    v = W.C_LIGHT * P / math.sqrt(1 + P * P)
    lam = 0.3 * W.AU
    p = dict(mass=W.M_P, dmm_model="power_q", dmm_norm=1, lambda_ref=lam, q=5 / 3, dt=1.0)
    mu = 0.5
    D = orc.dmm(p, P, mu)[0]
    assert D == pytest.approx(v / lam * (1 - mu * mu) * mu ** (2 / 3), rel=1e-12)
