"""Host-side pieces of the serving loop (no GPU): arrival processes and the
frame order that plays a rendered sequence forward and back."""
import numpy as np

from paper_1905_02082_amd import serving


def test_poisson_arrivals_start_and_rate():
    rng = np.random.default_rng(0)
    a = serving.poisson_arrivals(20000, 1.5, 30.0, rng)
    assert a[0] == 1.5 and np.all(np.diff(a) >= 0)
    assert abs((a[-1] - a[0]) / (len(a) - 1) - 1 / 30.0) < 1e-3   # mean gap of a rate-30 process


def test_ping_pong_is_continuous():
    o = serving.ping_pong(5, 13)
    assert o.tolist() == [0, 1, 2, 3, 4, 3, 2, 1, 0, 1, 2, 3, 4]
    assert serving.ping_pong(1, 4).tolist() == [0, 0, 0, 0]
