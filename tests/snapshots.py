"""Host record of an updated index for the GPU update and serving tests:
which ids each epoch sees, and the oracle's answers over that snapshot."""
import os

import numpy as np

import oracle

THREADS = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))

LIVE = 0xFFFFFFFF


class Model:
    """Host record of every id handed out: point, insert and erase epochs,
    and the compaction policy (drop tombstones with era <= oldest once they
    reach a tenth of the stored entries)."""

    def __init__(self, pts, hold=False):
        self.xy = np.asarray(pts, np.float64).reshape(-1, 2).copy()
        n = len(self.xy)
        self.ins = np.zeros(n, np.int64)
        self.era = np.full(n, LIVE, np.int64)
        self.stored = np.ones(n, bool)
        self.epoch = 0
        self.oldest = 0
        self.hold = hold
        self.compactions = 0

    def _after_update(self):
        if not self.hold:
            self.oldest = self.epoch
        self._maybe_compact()

    def _droppable(self):
        return self.stored & (self.era <= self.oldest)

    def _maybe_compact(self):
        d = self._droppable()
        if d.sum() > 0 and d.sum() * 10 >= self.stored.sum():
            self.stored &= ~d
            self.compactions += 1

    def insert(self, pts):
        self.epoch += 1
        k = len(pts)
        first = len(self.xy)
        self.xy = np.concatenate([self.xy, pts])
        self.ins = np.concatenate([self.ins, np.full(k, self.epoch)])
        self.era = np.concatenate([self.era, np.full(k, LIVE)])
        self.stored = np.concatenate([self.stored, np.ones(k, bool)])
        self._after_update()
        return np.arange(first, first + k)

    def erase(self, ids):
        self.epoch += 1
        cnt = 0
        for i in ids:
            if 0 <= i < len(self.xy) and self.stored[i] and self.era[i] == LIVE:
                self.era[i] = self.epoch
                cnt += 1
        self._after_update()
        return cnt

    def retire(self, e):
        self.oldest = max(self.oldest, e)
        self._maybe_compact()

    def visible(self, e):
        return np.nonzero(self.stored & (self.ins <= e) & (e < self.era))[0]

    def reference(self, qs, ds, epochs, curve, metric=oracle.L2):
        """Oracle answers (offsets, ids) for queries at the given epochs."""
        m = len(qs)
        per_q = [None] * m
        for e in np.unique(epochs):
            sel = np.nonzero(epochs == e)[0]
            ids = self.visible(e)
            if len(ids) == 0:
                for j in sel:
                    per_q[j] = np.zeros(0, np.uint32)
                continue
            off, idx = oracle.query(oracle.build(self.xy[ids], curve), qs[sel], ds[sel], curve,
                                    nthreads=THREADS, metric=metric)
            for t, j in enumerate(sel):
                per_q[j] = ids[idx[off[t]:off[t + 1]]].astype(np.uint32)
        offsets = np.zeros(m + 1, np.uint64)
        offsets[1:] = np.cumsum([len(r) for r in per_q])
        return offsets, (np.concatenate(per_q) if m else np.zeros(0, np.uint32))
