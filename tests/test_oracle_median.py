"""Pins of the oracle's running-median de-reddening (Sec. 5.2).

The paper subtracts a running median of user-chosen width and states the
filter's defining property: a constant impulse narrower than half the window
passes through x - median unchanged. The pins: that property, brute force
(a sort of every window) on small inputs, a monotone series being left
unchanged where the whole window fits (a monotone run is a root of the
median filter), the lower-median reading at the ends, and constant series.
"""
import numpy as np
import pytest

import oracle


def brute(x, window):
    h = window // 2
    n = x.size
    med = np.empty(n)
    for i in range(n):
        w = np.sort(x[max(0, i - h):min(n, i + h + 1)])
        med[i] = w[(w.size - 1) // 2]
    return x - med, med


@pytest.mark.parametrize("n,window", [(1, 1), (7, 1), (7, 3), (50, 5), (50, 49), (50, 99),
                                      (301, 31), (1000, 257)])
def test_running_median_equals_brute_force(n, window):
    g = np.random.default_rng(n * 1000 + window)
    x = g.standard_normal(n)
    x[::7] = np.round(x[::7])  # some ties
    y, med = oracle.running_median(x, window)
    yb, mb = brute(x, window)
    assert np.array_equal(med, mb)
    assert np.array_equal(y, yb)


def test_constant_impulse_narrower_than_half_the_window_passes_unchanged():
    # Sec. 5.2: the running median leaves intact any constant impulse whose
    # width is less than half the window; on a constant background the
    # de-reddened series is exactly the impulse
    g = np.random.default_rng(11)
    for window in (5, 31, 101, 1001):
        for trial in range(5):
            n = 5 * window + 17
            c = float(g.normal() * 10)
            a = float(g.uniform(1, 20)) * (1 if trial % 2 else -1)
            width = int(g.integers(1, (window + 1) // 2))  # < window / 2
            # away from the ends, where every window touching it is whole
            start = int(g.integers(window, n - window - width))
            x = np.full(n, c)
            x[start:start + width] += a
            y, med = oracle.running_median(x, window)
            want = np.zeros(n)
            want[start:start + width] = a
            assert np.array_equal(med, np.full(n, c)), (window, width)
            assert np.array_equal(y, x - c)
            assert np.allclose(y, want, rtol=0, atol=1e-12 * abs(a))


def test_wider_impulse_is_not_left_intact():
    # the property is sharp: an impulse wider than half the window moves the
    # median of the windows centred on it
    n, window, width = 400, 101, 60
    x = np.zeros(n)
    x[150:150 + width] = 5.0
    y, med = oracle.running_median(x, window)
    assert med[150 + width // 2] == 5.0


def test_monotone_series_is_a_root_where_the_window_fits():
    n, window = 500, 41
    x = np.cumsum(np.random.default_rng(3).uniform(0.1, 1.0, n))
    y, med = oracle.running_median(x, window)
    h = window // 2
    assert np.array_equal(y[h:n - h], np.zeros(n - 2 * h))
    # near the start the cut window [0, i + h] has its lower median at (i + h) // 2
    for i in range(h):
        assert med[i] == x[(i + h) // 2]


def test_lower_median_at_the_ends_by_hand():
    # window 3 on [4, 1, 3, 2]: output 0 sees {4, 1} (two samples, lower
    # median 1), output 3 sees {3, 2} (lower median 2)
    x = np.array([4.0, 1.0, 3.0, 2.0])
    y, med = oracle.running_median(x, 3)
    assert list(med) == [1.0, 3.0, 2.0, 2.0]
    assert list(y) == [3.0, -2.0, 1.0, 0.0]


def test_constant_series_gives_zero():
    y, med = oracle.running_median(np.full(123, 7.25), 11)
    assert (y == 0).all() and (med == 7.25).all()


def test_even_window_is_refused():
    with pytest.raises(ValueError):
        oracle.running_median(np.zeros(10), 4)
