"""Pins of the oracle's absorbing layers (an option of this implementation,
not of the paper): over a width h in front of each radial boundary the weight
decays at the rate k0 (1 - d/h)^2, d the distance to the boundary, so that a
particle crossing the layer at radial speed v keeps the fraction
exp(-Int k dt) = exp(-k0 h / (3 v)) of its weight, and the hard sphere behind
the layer retires what is left.  The particles stream along a radial line
(mu = +-1 in a uniform field along x, no flow, no scattering), so that the
step sum of the rates is a midpoint rule of that integral."""
import math

import numpy as np
import pytest

import fte_workloads as W

AU = W.AU
E100 = 100 * W.KEV
EPS100 = E100 / (W.M_P * W.C_LIGHT ** 2)
P100 = math.sqrt(EPS100 * (EPS100 + 2))
V100 = W.C_LIGHT * P100 / math.sqrt(1 + P100 ** 2)

R_IN, R_OUT = 0.1 * AU, 1.0 * AU
H = 0.01 * AU
K0 = 3 * V100 / H                  # k0 h / (3 v) = 1
N_LAYER = 2000                     # steps across the layer


def _params(dt, layer=True):
    return dict(mass=W.M_P, dmm_model="iso", lambda_ref=1e30, dt=dt, bg_kind="uniform", bg=[0, 0, 0, 1, 0, 0],
                r_in=R_IN, r_out=R_OUT, check_bounds=1, absorb_layer=H if layer else 0.0,
                absorb_rate=K0 if layer else 0.0)


def _streamer(orc, x0, mu):
    p = orc.Particles(1)
    p.x[:] = (x0, 0.0, 0.0)
    p.mu[:] = mu
    p.lnp[:] = math.log(P100)
    p.w[:] = 1.0
    p.pid[:] = 0
    return p


@pytest.mark.parametrize("n_layer", [N_LAYER, N_LAYER // 2])
def test_inner_layer_survival(orc, n_layer):
    """Inward at mu = -1 from 10.5 steps outside the layer: the weight stays 1
    until the layer, is exp(-1) half a step before r_in (midpoint rule,
    relative error ~ (v dt / h)^2), and the next step retires the particle at
    r_in with that weight."""
    dt = H / (V100 * n_layer)
    step = V100 * dt
    par = _params(dt)
    p = _streamer(orc, R_IN + H + 10.5 * step, -1.0)
    orc.run(par, None, p, 0, 10, None)
    assert p.status[0] == 0 and p.w[0] == 1.0
    orc.run(par, None, p, 10, n_layer, None)
    assert p.status[0] == 0
    assert p.x[0, 0] == pytest.approx(R_IN + 0.5 * step, rel=1e-9)
    assert p.w[0] == pytest.approx(math.exp(-1.0), rel=1e-5)
    w_last = p.w[0]
    orc.run(par, None, p, 10 + n_layer, 1, None)
    assert p.status[0] == 1 and p.w[0] == w_last


def test_outer_layer_survival(orc):
    """Outward at mu = +1 through the layer inside r_out: the same fraction."""
    dt = H / (V100 * N_LAYER)
    step = V100 * dt
    par = _params(dt)
    p = _streamer(orc, R_OUT - H - 10.5 * step, 1.0)
    orc.run(par, None, p, 0, 10 + N_LAYER, None)
    assert p.status[0] == 0
    assert p.w[0] == pytest.approx(math.exp(-1.0), rel=1e-5)
    orc.run(par, None, p, 10 + N_LAYER, 1, None)
    assert p.status[0] == 2


def test_layer_off_and_outside(orc):
    """No layer: the weight never changes; with the layer, a particle that
    stays outside it (at rest at mu = 0, up to the 1e-30-scale scattering)
    keeps its weight."""
    dt = H / (V100 * N_LAYER)
    step = V100 * dt
    p = _streamer(orc, R_IN + 0.5 * step + H, -1.0)
    orc.run(_params(dt, layer=False), None, p, 0, N_LAYER, None)
    assert p.status[0] == 0 and p.w[0] == 1.0
    q = _streamer(orc, 0.5 * AU, 0.0)
    orc.run(_params(dt), None, q, 0, 1000, None)
    assert q.status[0] == 0 and q.w[0] == 1.0
    assert abs(np.linalg.norm(q.x[0]) - 0.5 * AU) < 1e-6 * H
