"""The Python binding checks every block before its pointer crosses the C ABI
(the library reads and writes through raw pointers): host tensors, wrong
dtypes and non-2-D arguments are refused with ValueError before any library
call (these run without a GPU)."""

import pytest
import torch


def test_host_tensors_refused(cd):
    X = torch.zeros(100, 4, dtype=torch.float64)
    with pytest.raises(ValueError, match="CUDA"):
        cd.orthonormalize(None, X)
    with pytest.raises(ValueError, match="CUDA"):
        cd.tsqr(X)
    with pytest.raises(ValueError, match="CUDA"):
        cd.cluster(X, 3)
    with pytest.raises(ValueError, match="CUDA"):
        cd.subspace_loss(X.float(), X)


def test_block_checks(cd):
    # the checks themselves, on host tensors with the device test left out
    t = torch.zeros(10, 3, dtype=torch.float64)
    with pytest.raises(ValueError, match="CUDA"):
        cd._block(t, "t", 10, (torch.float64,))
    assert cd._same_device(torch.device("cpu"), "cpu")
    assert not cd._same_device(torch.device("cpu"), "cuda")
