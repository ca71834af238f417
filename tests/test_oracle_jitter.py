"""Pins of the oracle's counter-based jitter generator."""
import os

import numpy as np


def test_splitmix64_reference_sequence(orc):
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    ref = [int(l, 16) for l in open(path) if l.strip() and not l.startswith("#")]
    got = [int(v) for v in orc.splitmix64(0, np.arange(3))]
    assert got == ref


def test_jitter_bounds_and_uniformity(orc):
    """Jitter stays in [-amp, amp), is non-cumulative (depends on the step,
    not on earlier steps) and is close to uniform."""
    n = 200000
    x0 = np.full(n, 0.5, np.float32)
    amp = np.float32(0.1 / 1024)
    xs = orc.jitter(x0, x0, x0, 3, amp, 20180503)
    for a in xs:
        d = a.astype(np.float64) - 0.5
        ulp = float(np.spacing(np.float32(0.5)))      # the FP32 add rounds to x0's lattice
        assert d.min() >= -amp - ulp and d.max() <= amp + ulp
        hist, _ = np.histogram(d, bins=10, range=(-amp, amp))
        assert np.all(np.abs(hist / (n / 10) - 1) < 0.05)
    again = orc.jitter(x0, x0, x0, 3, amp, 20180503)
    assert all(np.array_equal(a, b) for a, b in zip(xs, again))
    other = orc.jitter(x0, x0, x0, 4, amp, 20180503)
    assert not np.array_equal(xs[0], other[0])
