"""sfc_query_batch_static (the library's fixed scratch, no allocation)
against sfc_query_batch through the C ABI: offsets and ids bit for bit on
two calls in a row, the second with a smaller batch, then the error paths
(a batch too large for the scratch, an ids buffer too small)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV)


def static_call(idx, q, d, offsets, ids):
    total = ctypes.c_uint64(0)
    st = sfc.lib().sfc_query_batch_static(idx.handle, sfc._ptr(q), sfc._ptr(d), q.shape[0],
                                          sfc._ptr(offsets), sfc._ptr(ids), ids.numel(),
                                          ctypes.byref(total))
    return st, int(total.value)


@pytest.mark.parametrize("curve,search,refine", [(sfc.HILBERT, sfc.BINARY, True),
                                                  (sfc.MORTON, sfc.LEARNED, True),
                                                  (sfc.MORTON, sfc.STREE, False)])
def test_static_scratch_equals_query_batch(curve, search, refine):
    wl = workload.clustered_loguniform(n=1 << 20, m=30_000, curve=curve, seed=21)
    idx = sfc.Index(dev(wl.points), curve, search=search, refine=refine)
    for m in (30_000, 7_000):   # the second call smaller than the first
        print(f"static scratch: curve={curve} search={search} refine={refine} m={m}", flush=True)
        q, d = dev(wl.queries[:m]), dev(wl.delta[:m])
        want_off, want_ids = idx.query(q, d)
        offsets = torch.full((m + 1,), -1, dtype=torch.int64, device=DEV)
        ids = torch.full((want_ids.numel() + 5,), -1, dtype=torch.int32, device=DEV)
        st, total = static_call(idx, q, d, offsets, ids)
        assert st == sfc.SFC_OK, sfc.status_string(st)
        assert total == want_ids.numel()
        assert torch.equal(offsets, want_off)
        assert torch.equal(ids[:total], want_ids)
        assert (ids[total:] == -1).all()
    idx.close()


def test_static_scratch_limits():
    wl = workload.uniform_fixed_radius(n=1 << 16, m=4000, curve=sfc.MORTON)
    idx = sfc.Index(dev(wl.points), sfc.MORTON)
    q, d = dev(wl.queries), dev(wl.delta)
    want_off, want_ids = idx.query(q, d)
    # an ids buffer too small: offsets and the total are written
    offsets = torch.empty(4001, dtype=torch.int64, device=DEV)
    small = torch.empty(10, dtype=torch.int32, device=DEV)
    st, total = static_call(idx, q, d, offsets, small)
    assert st == sfc.SFC_ERR_CAPACITY and total == want_ids.numel()
    assert torch.equal(offsets, want_off)
    # more queries than the fixed scratch holds: refused before any work
    big = 1 << 20
    qb = torch.full((big, 2), 0.5, dtype=torch.float64, device=DEV)
    db = torch.zeros(big, dtype=torch.float64, device=DEV)
    ob = torch.empty(big + 1, dtype=torch.int64, device=DEV)
    st, _ = static_call(idx, qb, db, ob, small)
    assert st == sfc.SFC_ERR_SCRATCH
    # an empty batch
    st, total = static_call(idx, q[:0], d[:0], offsets, small)
    assert st == sfc.SFC_OK and total == 0 and int(offsets[0]) == 0
    # and the index still answers the same afterwards
    off2, ids2 = idx.query(q, d)
    assert torch.equal(off2, want_off) and torch.equal(ids2, want_ids)
    idx.close()
