"""A CPU executor for the serving loop's tests: it runs each admitted
request with the oracle (small sizes only) and completes it after a
simulated duration on a virtual clock, so admission, batching and
back-pressure are testable without a GPU."""
import numpy as np

import oracle


class VirtualClock:
    def __init__(self, step=1e-4):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor:
    can_group = True

    def __init__(self, clock, per_flop_s=1e-9, fail_rids=(), bytes_per_elem=16):
        self.clock = clock
        self.per_flop_s = per_flop_s
        self.fail_rids = set(fail_rids)
        self.bpe = bytes_per_elem
        self.launched = []          # (batch rids, slot, t)
        self.inflight_slots = set()
        self.max_concurrent = 0

    def footprint(self, r):
        return self.bpe * r.n * r.n + self.bpe * r.n * max(r.nrhs, 1)

    def start(self):
        pass

    def stop(self):
        pass

    def launch(self, batch, slot):
        for r in batch:
            if r.rid in self.fail_rids:
                raise RuntimeError(f"injected failure for request {r.rid}")
        assert slot not in self.inflight_slots
        self.inflight_slots.add(slot)
        self.max_concurrent = max(self.max_concurrent, len(self.inflight_slots))
        t = self.clock.t
        dur = sum(2.0 * r.n ** 3 for r in batch) * self.per_flop_s
        self.launched.append(([r.rid for r in batch], slot, t))
        results = []
        for r in batch:
            if r.payload is not None:
                A, B = r.payload
                if r.kind == "gemm":
                    results.append(oracle.gemm(A, B, "block"))
                else:
                    LU, ipiv, _ = oracle.getrf(A, panel=8)
                    results.append(oracle.getrs(LU, ipiv, B))
            else:
                results.append(None)
        return {"t_end": t + dur, "results": results, "slot": slot}

    def done(self, h):
        return self.clock.t >= h["t_end"]

    def finish(self, h, batch):
        self.inflight_slots.discard(h["slot"])
        for r, res in zip(batch, h["results"]):
            r.result = res
        return h["t_end"]
