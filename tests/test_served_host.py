"""Host-side pieces of the served form (no GPU): nearest-rank quantiles and
Poisson arrival times."""
import numpy as np

from paper_2306_08252_amd import inputs as I
from paper_2306_08252_amd import served as S


def test_nearest_rank_definition():
    x = [15, 20, 35, 40, 50]  # the textbook nearest-rank example
    assert S.nearest_rank(x, 0.05) == 15
    assert S.nearest_rank(x, 0.30) == 20
    assert S.nearest_rank(x, 0.40) == 20
    assert S.nearest_rank(x, 0.50) == 35
    assert S.nearest_rank(x, 1.00) == 50
    y = np.arange(1, 101)
    assert S.nearest_rank(y, 0.99) == 99 and S.nearest_rank(y, 0.5) == 50


def test_poisson_arrivals_rate_and_order():
    draws = I.splitmix64(I.stream_seed("served-arrivals"), 200000)
    t = S.poisson_arrivals(draws, 1000.0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    # exponential gaps: mean 1/rate and standard deviation 1/rate, within 5 sigma
    assert abs(gaps.mean() - 1e-3) < 5 * 1e-3 / np.sqrt(len(gaps))
    assert abs(gaps.std() - 1e-3) < 0.02 * 1e-3
