"""Host-side argument checks of the Python binding (no GPU needed): every
tensor handed to a kernel must be on the right device, contiguous, of an
allowed dtype, of exactly the stated shape and 16-byte aligned."""
import pytest
import torch

from paper_2505_19154_amd._lib import FhError
from paper_2505_19154_amd.raster import check_tensor

F32 = (torch.float32,)


def test_accepts_a_matching_tensor():
    check_tensor(torch.zeros(10, 3), "x", (10, 3), F32, "cpu")


@pytest.mark.parametrize("bad, why", [
    (lambda: torch.zeros(10, 3, dtype=torch.float64), "dtype"),
    (lambda: torch.zeros(10, 3, dtype=torch.float16), "dtype"),
    (lambda: torch.zeros(9, 3), "shape"),
    (lambda: torch.zeros(30), "shape"),
    (lambda: torch.zeros(3, 10).t(), "contiguous"),
    (lambda: torch.zeros(41)[1:31].view(10, 3), "aligned"),
    (lambda: [[0.0] * 3] * 10, "tensor"),
])
def test_rejects(bad, why):
    with pytest.raises(FhError, match=why):
        check_tensor(bad(), "x", (10, 3), F32, "cpu")


def test_rejects_wrong_device():
    with pytest.raises(FhError, match="cuda"):
        check_tensor(torch.zeros(10, 3), "x", (10, 3), F32, "cuda")
