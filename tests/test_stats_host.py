"""CPU checks of the host post-processing in paper_2005_08736_amd.stats: the
three-point time derivative is exact on quadratics at any spacing and second
order on a smooth decay."""
import math

import numpy as np
import pytest

from paper_2005_08736_amd import stats


def test_time_derivative_exact_on_quadratics_nonuniform():
    rng = np.random.default_rng(3)
    t = np.cumsum(rng.uniform(0.5, 1.5, size=9))
    f = 2.0 - 0.7 * t + 0.3 * t * t
    assert np.allclose(stats.time_derivative(t, f), -0.7 + 0.6 * t, rtol=1e-12, atol=1e-12)


def test_time_derivative_second_order():
    errs = []
    for n in (21, 41):
        t = np.linspace(0.0, 1.0, n) ** 1.2  # nonuniform
        errs.append(np.abs(stats.time_derivative(t, np.exp(-2 * t)) + 2 * np.exp(-2 * t)).max())
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_time_derivative_rejects_bad_histories():
    with pytest.raises(ValueError):
        stats.time_derivative([0.0, 1.0], [1.0, 2.0])
    with pytest.raises(ValueError):
        stats.time_derivative([0.0, 2.0, 1.0], [1.0, 2.0, 3.0])
