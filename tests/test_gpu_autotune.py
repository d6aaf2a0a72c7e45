"""The autotuner records a shape per size bucket and results stay identical."""
import numpy as np
import pytest
import torch

from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results():
    wl = workload.clustered_loguniform(n=100_000, m=5_000, curve=sfc.MORTON, seed=31)
    pts = torch.as_tensor(wl.points).cuda()
    q = torch.as_tensor(wl.queries).cuda()
    d = torch.as_tensor(wl.delta).cuda()
    idx = sfc.Index(pts, sfc.MORTON, refine=True)
    want = idx.query(q, d)
    best, ms = sfc.autotune_build(pts, sfc.MORTON)
    assert best in (8, 12, 16, 20, 24) and len(ms) == 5 and all(v > 0 for v in ms.values())
    bq, msq = sfc.autotune_query(idx, q, d)
    assert 0 <= bq <= 4 and len(msq) == 5
    idx2 = sfc.Index(pts, sfc.MORTON, refine=True)
    got = idx2.query(q, d)
    assert torch.equal(want[0], got[0]) and torch.equal(want[1], got[1])


def test_stats_rows_match_ranges():
    wl = workload.clustered_loguniform(n=60_000, m=3_000, curve=sfc.HILBERT, seed=32)
    pts = torch.as_tensor(wl.points).cuda()
    q = torch.as_tensor(wl.queries).cuda()
    d = torch.as_tensor(wl.delta).cuda()
    idx = sfc.Index(pts, sfc.HILBERT)
    off, ids = idx.query(q, d)
    _, _, b, e, nr = idx.query_ranges(q, d)
    b, e, nr = (t.cpu().numpy().astype(np.int64) for t in (b, e, nr))
    mask = np.arange(b.shape[1])[None, :] < nr[:, None]
    lens = np.where(mask, e - b, 0)
    st = idx.last_stats()
    assert st["candidates"] == lens.sum()
    assert st["rows"] == ((lens + 63) // 64).sum()
    assert st["reported"] == ids.numel() and st["queries"] == 3_000
