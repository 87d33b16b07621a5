"""The bandwidth-calibration kernels (etd_calib_stream) move the data they
claim to: a copy (plain or non-temporal stores) equals its source, a write
sweep stores (i, i) at 16-byte element i, a read sweep leaves its sink
untouched."""

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["copy", "copy_nt", "copy_ranges", "write", "write_nt", "read"])
def test_calibration_sweeps_move_the_right_bytes(kind):
    import torch
    from paper_2001_11220_amd.etd import calib_stream
    n = (1 << 20) + 48  # doubles; not a multiple of the grid's stride
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    sink = torch.zeros(8, dtype=torch.float64, device="cuda")
    src, dst = {"copy": (x, y), "copy_nt": (x, y), "copy_ranges": (x, y), "write": (None, y),
                "write_nt": (None, y), "read": (x, sink)}[kind]
    calib_stream(kind, src, dst, n * 8, 512)
    torch.cuda.synchronize()
    if kind.startswith("copy"):
        assert torch.equal(y, x)
    elif kind.startswith("write"):
        i = torch.arange(n // 2, dtype=torch.float64, device="cuda")
        assert torch.equal(y.view(-1, 2)[:, 0], i) and torch.equal(y.view(-1, 2)[:, 1], i)
    else:
        assert torch.equal(sink, torch.zeros_like(sink))
