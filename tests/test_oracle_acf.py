"""Pins of the oracle's autocorrelation (choice of the sampling interval T_s): the direct
definition equals an FFT computation of the same sums, an alternating series has the closed
form acf(k) = (-1)^k, and a first-order autoregressive series has acf(k) = phi^k and the
integrated time (1 + phi) / (2 (1 - phi)) within their statistical errors."""
import numpy as np
import pytest

import ttcf_inputs as I


def test_definition_equals_fft(orc):
    x = I.ar1_series(4000, 0.8, 3)
    a = orc.acf(x, 200)
    d = x - x.mean()
    n = len(d)
    f = np.fft.rfft(d, 2 * n)
    full = np.fft.irfft(f * np.conj(f), 2 * n)[:200]
    ref = full / (n - np.arange(200))
    np.testing.assert_allclose(a, ref / ref[0], rtol=1e-10, atol=1e-12)


def test_alternating_series_closed_form(orc):
    x = np.tile([1.0, -1.0], 500)
    a = orc.acf(x, 10)
    np.testing.assert_allclose(a, [(-1.0) ** k for k in range(10)], atol=1e-15)
    fb, tau = orc.acf_summary(a, 0.5)
    assert fb == 1 and tau == 0.5


def test_ar1_decay_and_correlation_time(orc):
    phi = 0.9
    x = I.ar1_series(400000, phi, 5)
    a = orc.acf(x, 60)
    k = np.arange(60)
    # statistical error of an estimated acf at lag k is about sqrt((1+phi^2)/((1-phi^2) n))
    err = np.sqrt((1 + phi ** 2) / ((1 - phi ** 2) * len(x)))
    assert np.abs(a - phi ** k).max() < 6 * err
    fb, tau = orc.acf_summary(a, np.exp(-2.0))
    assert fb == int(np.ceil(2.0 / -np.log(phi))) or fb == int(np.ceil(2.0 / -np.log(phi))) + 1
    assert tau == pytest.approx((1 + phi) / (2 * (1 - phi)), rel=0.1)
