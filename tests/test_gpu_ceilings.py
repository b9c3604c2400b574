"""The library's streaming-read probe (read_bandwidth), which measures the read ceilings that
the path-sum kernels' rooflines are stated against."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def test_read_bandwidth_levels(sf):
    import torch
    buf = torch.ones(1 << 28, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rates = {}
    for nbytes, reps in ((1 << 28, 10), (1 << 21, 2000)):
        ms = sf.read_bandwidth(buf, nbytes, reps, 0, stream)
        assert ms > 0.0
        rates[nbytes] = nbytes * reps / (ms * 1e-3) / 1e9
    # plausible bytes per second, and a buffer that fits the L2s is read faster than one that does not
    for r in rates.values():
        assert 100.0 < r < 200_000.0, rates
    assert rates[1 << 21] > rates[1 << 28], rates
    # a grid given explicitly
    assert sf.read_bandwidth(buf, 1 << 20, 4, 64, stream) > 0.0
