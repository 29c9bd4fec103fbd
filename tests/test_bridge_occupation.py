"""The occupation density at mu = 0 that the step kernel's tangents use for
Eq. 5's Dirac term when kink_sigma < 0 (gradient mode): for a Brownian motion
of diffusion s2 (variance s2 h after a time h) pinned at a and b over a step
of length h, the expected time spent per unit length at 0 is

    Int_0^h g_t(a) g_(h-t)(b) dt / g_h(b - a),   g_t(x) the N(0, s2 t) density,

which in closed form is sqrt(2 pi h) / (2 s) erfcx(z) exp(-(a b + |a b|) / (s2 h)),
z = (|a| + |b|) / (s sqrt(2 h)).  These checks pin that closed form against
its definition by quadrature and against the unconditional local time, and
the kernel's asymptotic erfcx against scipy's."""
import math

import numpy as np
import pytest
from scipy import integrate, special


def _gauss(x, var):
    return math.exp(-x * x / (2 * var)) / math.sqrt(2 * math.pi * var)


def _closed(a, b, s2, h):
    s = math.sqrt(s2)
    z = (abs(a) + abs(b)) / (s * math.sqrt(2 * h))
    return math.sqrt(2 * math.pi * h) / (2 * s) * special.erfcx(z) * math.exp(-(a * b + abs(a * b)) / (s2 * h))


def _definition(a, b, s2, h):
    f = lambda t: _gauss(a, s2 * t) * _gauss(b, s2 * (h - t))
    num, _ = integrate.quad(f, 0.0, h, epsabs=0.0, epsrel=1e-12, limit=400, points=[h / 2])
    return num / _gauss(b - a, s2 * h)


@pytest.mark.parametrize("a,b", [(0.01, 0.02), (0.02, 0.01), (-0.01, 0.015), (0.03, -0.002), (-0.02, -0.05),
                                 (0.0, 0.01), (0.1, 0.12), (-0.004, 0.004)])
@pytest.mark.parametrize("s2,h", [(1e-3, 1.0), (0.2, 0.05)])
def test_closed_form_matches_definition(a, b, s2, h):
    got, want = _closed(a, b, s2, h), _definition(a, b, s2, h)
    assert got == pytest.approx(want, rel=1e-8, abs=1e-300)


@pytest.mark.parametrize("a", [0.0, 0.01, -0.03])
def test_mean_over_end_points_is_the_local_time(a):
    """Averaged over the free end point b ~ N(a, s2 h) the bridge occupation is
    the expected local time at 0 of the free motion, Int_0^h g_t(a) dt."""
    s2, h = 1e-3, 1.0
    sd = math.sqrt(s2 * h)
    avg, _ = integrate.quad(lambda b: _closed(a, b, s2, h) * _gauss(b - a, s2 * h), a - 12 * sd, a + 12 * sd,
                            points=[0.0] if abs(a) < 12 * sd else None, limit=400, epsrel=1e-11)
    free, _ = integrate.quad(lambda t: _gauss(a, s2 * t), 0.0, h, limit=400, epsrel=1e-11)
    if a == 0.0:
        free = math.sqrt(2 * h / (math.pi * s2))       # Int_0^h (2 pi s2 t)^-1/2 dt
    assert avg == pytest.approx(free, rel=1e-7)


def _erfcx_series(z):
    t = 1.0 / (z * z)
    return 1.0 / (z * math.sqrt(math.pi)) * (1 - 0.5 * t + 0.75 * t * t - 1.875 * t ** 3)


@pytest.mark.parametrize("z,rel", [(8.0, 5e-7), (26.0, 3e-11), (100.0, 1e-15)])
def test_asymptotic_erfcx(z, rel):
    """The series the kernel switches to (z >= 8 in FP32, z >= 26 in FP64)."""
    assert _erfcx_series(z) == pytest.approx(float(special.erfcx(z)), rel=rel)
    assert abs(_erfcx_series(z) / special.erfcx(z) - 1) < 7 / z ** 8
