"""The bandwidth measurements the benchmark reports beside the published peak: a streaming copy
and a streaming read over 1 GiB return finite, plausible rates, and bad arguments are refused."""
import numpy as np
import pytest

import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = qt.Context(0)
    yield c
    c.close()


def test_stream_bandwidth_measurements(ctx):
    print("[gpu] streaming copy and read bandwidth, 1 GiB", flush=True)
    c = qt.measure_copy_bandwidth(ctx, 1 << 30, 5)
    r = qt.measure_read_bandwidth(ctx, 1 << 30, 5)
    print(f"[gpu]   copy {c:.0f} GB/s, read {r:.0f} GB/s", flush=True)
    # above any plausible floor, and below the 8 TB/s peak plus what the 256 MB MALL could add
    for v in (c, r):
        assert np.isfinite(v) and 500.0 < v < 12000.0
    for bad in [(8, 1), (1 << 20, 0)]:
        with pytest.raises(qt.QtError):
            qt.measure_read_bandwidth(ctx, *bad)
        with pytest.raises(qt.QtError):
            qt.measure_copy_bandwidth(ctx, *bad)
