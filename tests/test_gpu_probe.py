"""The streaming-bandwidth probe (a measurement utility stated beside the
roofline): each kind runs and times its pass, the copy moves the source into
the destination, the write fills the destination, and the rates it implies
stay below the device's 8 TB/s (buffers of 1 GiB, beyond the last-level
cache)."""
import pytest

pytestmark = pytest.mark.gpu

PEAK = 8e12


def test_stream_probe_kinds():
    import torch
    from paper_2512_04997_amd import probe
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    torch.cuda.set_device(0)
    nbytes = 1 << 30
    a = torch.arange(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    torch.cuda.synchronize()
    ms = probe.stream("copy", a.data_ptr(), b.data_ptr(), nbytes, grid=4096, reps=3)
    assert ms > 0 and 2 * nbytes / (ms * 1e-3) < PEAK
    assert torch.equal(a, b)
    ms = probe.stream("read", a.data_ptr(), b.data_ptr(), nbytes, grid=4096, reps=3)
    assert ms > 0 and nbytes / (ms * 1e-3) < PEAK
    ms = probe.stream("write", a.data_ptr(), b.data_ptr(), nbytes, grid=4096, reps=3)
    assert ms > 0 and nbytes / (ms * 1e-3) < PEAK
    q = b.view(-1, 4)
    assert bool((q[:, 0] == 1).all()) and bool((q[:, 3] == 4).all())
    del a, b
    torch.cuda.empty_cache()
