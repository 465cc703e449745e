"""Serving form: a request loop that codes streamed images of several sizes
against a resident dictionary and updates that dictionary online.

Design (host loop over the C calls; every arithmetic step runs in the library):

* One learner context per grid size, each on its own stream, so that batches
  of different sizes overlap on the device.  All contexts start from the same
  spatial dictionary; each keeps its own history at its grid size, and the
  dictionary update is the shared-dictionary DictOCSC over all grids that have
  seen requests (``ocsc_dict_update_group``).
* Continuous batching: a request is admitted to its grid's pending slots as
  they free up; whenever a grid's stream has no batch in flight, the requests
  of that grid that have arrived (up to ``max_launch`` and the free slots) are
  coded in one launch sequence (``ocsc_code_append``), their input copied from
  pinned host memory on the same stream.  A request completes when the event
  recorded after its batch has completed; latency = completion - arrival.
* The pending slots per grid (the device state a request occupies until its
  history is folded) are sized so that all contexts fit the HBM budget.
* Each grid's code-update launch shapes are autotuned at start-up for a full
  launch (``ocsc_autotune``).  A context keeps its shape for every launch
  size, so a request's codes do not depend on what it was batched with.
* ``cholesky=True`` serves in the precision form: each fold adds the pending
  samples to the history on the matrix cores and rebuilds C from FP64
  Cholesky factors, instead of folding sample after sample.
* Every ``update_every`` completed requests the pending samples of every grid
  are accumulated and one shared dictionary update is enqueued; requests
  coded afterwards carry the next dictionary version.  A grid whose slots are
  full accumulates early (its fold runs before its next batch).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    grid: int               # side of the square grid
    image: object           # host array (grid x grid), float32
    done: float = math.nan  # completion time (seconds from the start)
    version: int = -1       # dictionary version the request was coded with
    codes: object = None    # device tensor (K x grid x grid) when kept


def slot_bytes(K: int, n: int, real_bytes: int = 4, cholesky: bool = False) -> int:
    """Device bytes one pending slot of an n x n context holds (contexts with
    more than one slot): the sample and code spectra, the frequency-major copy
    of the code spectra that the history fold reads, the code-ADMM dual and
    transform workspace (and, in the precision form, a codes buffer)."""
    Pf, P = n * (n // 2 + 1), n * n
    spec = 2 * real_bytes
    b = Pf * spec * 2 + 3 * K * Pf * spec + K * P * real_bytes
    if n > 128:
        b += K * Pf * spec
    if cholesky:
        b += K * P * real_bytes
    return b


def fixed_bytes(K: int, n: int, real_bytes: int = 4, cholesky: bool = False) -> int:
    """Device bytes of an n x n context independent of its slots (C, and H in
    the precision form, dominate)."""
    Pf = n * (n // 2 + 1)
    fs = (K * (K + 1) + 3) // 4 * 4
    return Pf * fs * real_bytes * (2 if cholesky else 1) + 8 * K * Pf * 2 * real_bytes


def plan_slots(K: int, grids: Sequence[int], shares: Sequence[float], budget: float,
               max_launch: Dict[int, int], cholesky: bool = False) -> Dict[int, int]:
    """Pending slots per grid: what remains of the budget after the fixed
    state, split in proportion to share x slot size, at least one launch's
    worth per grid."""
    free = budget - sum(fixed_bytes(K, n, cholesky=cholesky) for n in grids)
    weights = [s * slot_bytes(K, n, cholesky=cholesky) for s, n in zip(shares, grids)]
    tot = sum(weights)
    out = {}
    for n, w in zip(grids, weights):
        slots = int(free * w / tot // slot_bytes(K, n, cholesky=cholesky)) if free > 0 else 0
        slots = min(slots, 65535 // K)
        if slots < max_launch[n]:
            raise ValueError(f"HBM budget too small for the {n}x{n} grid")
        out[n] = slots
    return out


@dataclass
class _Grid:
    n: int
    model: object
    stream: object
    slots: int
    max_launch: int
    queue: List[Request] = field(default_factory=list)
    inflight: Optional[tuple] = None   # (event, requests, codes tensor)
    pending: int = 0                   # slots holding coded, not yet folded samples
    xbuf: object = None                # pinned host staging
    xdev: object = None


class Server:
    def __init__(self, K: int, filt: int, D0, grids: Sequence[int] = (64, 128, 256, 512),
                 shares: Sequence[float] = (8, 4, 2, 1), lam: float = 1.0, rho: float = 1.0,
                 update_every: int = 256, budget: float = 64e9, max_launch: Optional[Dict[int, int]] = None,
                 iters_code: int = 10, iters_dict: int = 10, keep_codes: bool = False, device: str = "cuda:0",
                 slots: Optional[Dict[int, int]] = None, autotune: bool = True, cholesky: bool = False):
        import torch
        from paper_1706_06972_amd.ocsc import OCSC
        self.torch = torch
        self.K, self.update_every, self.keep_codes = K, update_every, keep_codes
        self.device = torch.device(device)
        max_launch = max_launch or {64: 64, 128: 32, 256: 8, 512: 2}
        self.slots = dict(slots) if slots else plan_slots(K, grids, shares, budget, max_launch, cholesky)
        self.grids: Dict[int, _Grid] = {}
        for n in grids:
            st = torch.cuda.Stream(device=self.device)
            with torch.cuda.stream(st):
                m = OCSC(K, filt, filt, n, n, lam, rho, iters_code=iters_code, iters_dict=iters_dict,
                         max_batch=self.slots[n], precision="f32", cholesky=cholesky, device=self.device)
                m.set_dictionary(D0)
                if autotune:   # launch shapes for full launches of this grid, kept for every launch size
                    m.autotune(min(max_launch[n], self.slots[n]))
            g = _Grid(n, m, st, self.slots[n], max_launch[n])
            g.xbuf = torch.empty((g.max_launch, n, n), dtype=torch.float32, pin_memory=True)
            g.xdev = torch.empty((g.max_launch, n, n), dtype=torch.float32, device=self.device)
            self.grids[n] = g
        torch.cuda.synchronize(self.device)
        self.version = 0
        self.updates = 0
        self._since_update = 0
        self.log: list = []   # ("code", grid, request ids) / ("accumulate", grid) / ("update", grids)

    # -- device steps ---------------------------------------------------------
    def _launch(self, g: _Grid):
        torch = self.torch
        free = g.slots - g.pending
        if free <= 0:
            g.model.history_accumulate()           # fold runs before this grid's next batch
            g.pending = 0
            free = g.slots
            self.log.append(("accumulate", g.n))
        take = g.queue[:min(len(g.queue), g.max_launch, free)]
        del g.queue[:len(take)]
        B = len(take)
        for i, r in enumerate(take):
            g.xbuf[i].copy_(torch.from_numpy(r.image))
        with torch.cuda.stream(g.stream):
            g.xdev[:B].copy_(g.xbuf[:B], non_blocking=True)
            codes = torch.empty((B, self.K, g.n, g.n), dtype=torch.float32, device=self.device)
            g.model.code_append(g.xdev[:B], codes)
            ev = torch.cuda.Event()
            ev.record(g.stream)
        g.pending += B
        for r in take:
            r.version = self.version
        g.inflight = (ev, take, codes)
        self.log.append(("code", g.n, [r.rid for r in take]))

    def _dictionary_update(self):
        from paper_1706_06972_amd.ocsc import OCSC
        members = []
        for g in self.grids.values():
            if g.pending:
                g.model.history_accumulate()
                g.pending = 0
            if g.model.count > 0:
                members.append(g)
        if members:
            OCSC.dict_update_group([g.model for g in members])
            self.version += 1
            self.updates += 1
            self.log.append(("update", [g.n for g in members]))

    # -- the loop ---------------------------------------------------------------
    def run(self, requests: List[Request]) -> dict:
        """Serve requests (sorted by arrival) in real time; returns the metrics."""
        pending = list(requests)
        nxt = 0
        done = 0
        t0 = time.perf_counter()
        while done < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                r = pending[nxt]
                self.grids[r.grid].queue.append(r)
                nxt += 1
            for g in self.grids.values():
                if g.inflight is not None and g.inflight[0].query():
                    tdone = time.perf_counter() - t0
                    _, reqs, codes = g.inflight
                    for i, r in enumerate(reqs):
                        r.done = tdone
                        if self.keep_codes:
                            r.codes = codes[i]
                    done += len(reqs)
                    self._since_update += len(reqs)
                    g.inflight = None
                if self._since_update >= self.update_every:
                    self._since_update -= self.update_every
                    self._dictionary_update()
                if g.inflight is None and g.queue:
                    self._launch(g)
            if nxt < len(pending) and all(g.inflight is None and not g.queue for g in self.grids.values()):
                wait = pending[nxt].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        wall = time.perf_counter() - t0
        return summarize(requests, wall, self.updates)

    def close(self):
        for g in self.grids.values():
            g.model.close()


def summarize(requests: List[Request], wall: float, updates: int, warmup: int = 0) -> dict:
    import numpy as np
    rs = requests[warmup:]
    lat = np.array([r.done - r.arrival for r in rs])
    span = max(r.done for r in rs) - min(r.arrival for r in rs)
    offered = len(rs) / max(rs[-1].arrival - rs[0].arrival, 1e-9)
    return {"requests": len(rs), "p50_ms": 1000 * float(np.percentile(lat, 50)),
            "p99_ms": 1000 * float(np.percentile(lat, 99)), "mean_ms": 1000 * float(lat.mean()),
            "images_per_s": len(rs) / span, "offered_per_s": offered, "wall_s": wall,
            "dictionary_updates": updates}


def poisson_requests(n: int, rate: float, grids: Sequence[int], shares: Sequence[float], seed: int = 0,
                     content: float = 0.5) -> List[Request]:
    """n requests with exponential inter-arrival gaps (mean 1/rate) and grid
    sizes drawn with the given shares; each image is synthetic content of
    n/2 x n/2 (the shape recipe of the synthetic workloads) on its grid."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    p = np.asarray(shares, dtype=np.float64)
    sizes = rng.choice(len(grids), size=n, p=p / p.sum())
    cache = {}
    out = []
    for i, (a, si) in enumerate(zip(arrivals, sizes)):
        g = grids[si]
        if g not in cache:   # a pool of distinct images per grid, reused round robin
            wl = synth.Workload(name=f"serve{g}", pad_h=g, pad_w=g, content_h=int(g * content),
                                content_w=int(g * content), k_true=16, density=0.01, sigma_z=10.0, noise=0.01,
                                K=16, filt_h=11, filt_w=11, lam=1.0, rho=1.0, iters_code=10, iters_dict=10,
                                batch=1, n_images=16, passes=1, precision="f32", seed=seed + g)
            cache[g] = synth.images(wl, range(16)).astype(np.float32)
        out.append(Request(i, float(a), g, cache[g][i % 16]))
    return out
