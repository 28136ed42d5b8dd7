"""Time-to-solution analysis (Sec. IV) against closed forms and scipy."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1806_08815_amd import tts


def test_r99_closed_forms():
    assert tts.r99(0.5) == pytest.approx(math.log(0.01) / math.log(0.5))
    assert tts.r99(0.5) == pytest.approx(6.643856189774724)
    assert tts.r99(0.99) == pytest.approx(1.0)
    assert tts.r99(1.0) == 1.0
    assert math.isinf(tts.r99(0.0))
    # P(at least one success in R99 runs) = 0.99
    for th in (0.01, 0.2, 0.7):
        R = tts.r99(th)
        assert 1 - (1 - th) ** R == pytest.approx(0.99)


def test_jeffreys_posterior_matches_scipy():
    for y, r in [(0, 10), (3, 10), (10, 10), (57, 100)]:
        a, b = tts.jeffreys_posterior(y, r)
        assert (a, b) == (0.5 + y, 0.5 + r - y)
        med = tts._beta_median(a, b)
        assert med == pytest.approx(stats.beta(a, b).median(), rel=1e-9, abs=1e-12)
        for xv in (0.1, 0.5, 0.9):
            assert tts._betainc(a, b, xv) == pytest.approx(stats.beta(a, b).cdf(xv), rel=1e-9)


def test_posterior_samples_distribution():
    s = tts.posterior_r99_samples(20, 100, n=20000, seed=3)
    a, b = tts.jeffreys_posterior(20, 100)
    th = 1 - np.exp(np.log(0.01) / s)
    ks = stats.kstest(th, stats.beta(a, b).cdf)
    assert ks.pvalue > 1e-3


def test_tts99_measured_uses_ceil_r99():
    calls = []

    def launch(R):
        calls.append(R)
        return 0.001 * R

    out = tts.tts99_measured(50, 100, launch)
    want = math.ceil(tts.r99(stats.beta(50.5, 50.5).median()))
    assert calls == [want] and out["replicas"] == want
    none = tts.tts99_measured(0, 100, launch)
    assert none["tts_s"] > 0
    assert tts.success_count([3, 1, 1, 5], 1) == 2
