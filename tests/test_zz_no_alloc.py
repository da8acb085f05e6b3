"""fgs_l1_loss_noalloc, the L1 loss for callers that cannot allocate: its
partial sums live in the library's own per-GPU array instead of a
caller-provided buffer.  Checked through the C ABI against fgs_l1_loss (same
kernels: equal bit for bit) on two calls in a row, the second on a smaller
input, so a stale partial from the first call would show."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2409_04751_amd import _lib as L  # noqa: E402

pytestmark = pytest.mark.gpu


def _stream():
    return int(torch.cuda.current_stream().cuda_stream)


def _both(img, tgt):
    n = img.numel()
    partials = torch.empty(L.FGS_L1_PARTIALS, dtype=torch.float64, device="cuda")
    ref = torch.empty((), dtype=torch.float32, device="cuda")
    got = torch.full((), float("nan"), dtype=torch.float32, device="cuda")
    L.fgs_l1_loss(img.data_ptr(), tgt.data_ptr(), n, partials.data_ptr(), ref.data_ptr(), _stream())
    rc = L.fgs_l1_loss_noalloc(img.data_ptr(), tgt.data_ptr(), n, got.data_ptr(), _stream())
    assert rc == L.FGS_OK, L.fgs_last_error()
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_loss_equals_loss_two_calls_second_smaller():
    rng = np.random.default_rng(21)
    big = [torch.from_numpy(rng.random((3, 1168, 1752), dtype=np.float32)).cuda() for _ in range(2)]
    small = [torch.from_numpy(rng.random((3, 37, 53), dtype=np.float32)).cuda() for _ in range(2)]
    for img, tgt in (big, small):
        ref, got = _both(img, tgt)
        assert torch.equal(ref, got), (float(ref), float(got))
        want = float(np.abs(img.cpu().numpy().astype(np.float64) - tgt.cpu().numpy()).mean())
        assert abs(float(got) - want) <= 1e-6 * want


def test_noalloc_loss_rejects_bad_arguments():
    img = torch.zeros(16, device="cuda")
    out = torch.zeros((), device="cuda")
    assert L.fgs_l1_loss_noalloc(img.data_ptr(), img.data_ptr(), 0, out.data_ptr(), _stream()) == L.FGS_ERR_ARG
    assert L.fgs_l1_loss_noalloc(img.data_ptr(), img.data_ptr(), 1 << 31, out.data_ptr(), _stream()) == \
        L.FGS_ERR_OVERFLOW
    assert L.fgs_l1_loss_noalloc(img.data_ptr() + 4, img.data_ptr(), 8, out.data_ptr(), _stream()) == L.FGS_ERR_ARG
    assert L.fgs_l1_loss_noalloc(None, img.data_ptr(), 8, out.data_ptr(), _stream()) == L.FGS_ERR_ARG
