"""Host-side pieces of the serving form (no GPU): the workload generator and
the latency percentile."""
import numpy as np

import instances as I
from paper_1810_05231_amd.serving import percentile


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50
    assert percentile(xs, 99) == 99
    assert percentile(xs, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert percentile([5, 1, 4, 2, 3], 50) == 3


def test_serving_stream_shape_and_seed():
    a = I.serving_stream(40, seed=1, rate=10.0)
    b = I.serving_stream(40, seed=1, rate=10.0)
    assert [(r[0], r[1], r[2].n, r[2].name) for r in a] == [(r[0], r[1], r[2].n, r[2].name) for r in b]
    ns = np.array([r[2].n for r in a])
    assert ns.min() >= 100 and ns.max() <= 2000
    arr = np.array([r[1] for r in a])
    assert np.all(np.diff(arr) >= 0) and arr[0] > 0
    kinds = {r[2].name.split("_")[0] for r in a}
    assert kinds == {"maxcut", "equip"}
    # G(n, 8/n): mean degree about 8
    deg = np.mean([2 * r[2].meta["edges"] / r[2].n for r in a])
    assert 6.5 < deg < 9.5


def test_serving_stream_poisson_rate():
    a = I.serving_stream(400, seed=2, rate=20.0, n_lo=100, n_hi=120)
    arr = np.array([r[1] for r in a])
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.2 / 20.0
    z = I.serving_stream(5, seed=2, rate=None, n_lo=100, n_hi=120)
    assert all(r[1] == 0.0 for r in z)
