"""GPU: the random whole-row gather measurement (chebdav_probe_gather).  On a
table of ones every gather adds the row's element count to the live sum, so
the output pins the number of gathers performed and that each read a whole
row; argument errors return before any launch."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row_bytes", [128, 256, 512])
def test_probe_gather_reads_whole_rows(cd, dev, row_bytes):
    import torch
    rows = 50_000
    table = torch.ones(rows * row_bytes // 8, dtype=torch.float64, device="cuda")
    print("case probe gather row_bytes=%d" % row_bytes, flush=True)
    done, out = cd.probe_gather(table, row_bytes, 1_000_003, seed=7)
    torch.cuda.synchronize()
    assert done >= 1_000_003 and done % 16 == 0
    total = float(out.double().sum().cpu())
    assert total == done * (row_bytes // 8)


def test_probe_gather_zero_and_errors(cd, dev):
    import torch
    table = torch.zeros(4096, dtype=torch.float64, device="cuda")
    done, out = cd.probe_gather(table, 512, 0)
    torch.cuda.synchronize()
    assert done == 0 and float(out.abs().sum().cpu()) == 0.0
    with pytest.raises(cd.ChebdavError) as ei:
        cd.probe_gather(table, 64, 10)
    assert ei.value.status == cd.EINVAL
    with pytest.raises(cd.ChebdavError) as ei:
        cd.probe_gather(table[1:4001], 128, 10)  # 8-byte offset: not 16-byte aligned
    assert ei.value.status == cd.EINVAL
