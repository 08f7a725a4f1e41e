"""The binding's checks of caller-supplied output buffers (host mode: numpy arrays).

They run before any address reaches the library, so an undersized, mistyped or
non-contiguous array raises RaptorError(E_INVALID) instead of letting the library's copies
run past its end.  No GPU is needed: the checks are plain Python."""
import numpy as np
import pytest

from paper_1801_10452_amd import raptor as R


def test_accepts_a_matching_array():
    a = np.zeros((2, 3, 4))
    assert R._out(a, 24, "f8", R.MEM_HOST, 0, "images") == a.ctypes.data
    assert R._out(None, 24, "f8", R.MEM_HOST, 0, "images") is None
    s = np.zeros((3, 4), np.int32)
    assert R._out(s, 12, "i4", R.MEM_HOST, 0, "ray_status") == s.ctypes.data


@pytest.mark.parametrize("bad,why", [
    (np.zeros(23), "elements"),                       # one element short
    (np.zeros(24, np.float32), "float64"),            # wrong dtype
    (np.zeros((4, 12))[:, ::2], "contiguous"),        # a strided view
    ([0.0] * 24, "numpy"),                            # not an array
])
def test_rejects_mismatched_host_buffers(bad, why):
    with pytest.raises(R.RaptorError) as ei:
        R._out(bad, 24, "f8", R.MEM_HOST, 0, "images")
    assert ei.value.status == R.E_INVALID
    assert why in str(ei.value)


def test_rejects_read_only_and_wrong_int_type():
    a = np.zeros(24)
    a.setflags(write=False)
    with pytest.raises(R.RaptorError):
        R._out(a, 24, "f8", R.MEM_HOST, 0, "images")
    with pytest.raises(R.RaptorError):
        R._out(np.zeros(12, np.int64), 12, "i4", R.MEM_HOST, 0, "ray_steps")


def test_device_mode_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(R.RaptorError) as ei:
        R._out(np.zeros(24), 24, "f8", R.MEM_DEVICE, 0, "images")
    assert "torch tensor" in str(ei.value)
    with pytest.raises(R.RaptorError) as ei:
        R._out(torch.zeros(24, dtype=torch.float64), 24, "f8", R.MEM_DEVICE, 0, "images")
    assert "cuda" in str(ei.value)
    with pytest.raises(R.RaptorError):
        R._out(torch.zeros(24, dtype=torch.float32), 24, "f8", R.MEM_DEVICE, 0, "images")
