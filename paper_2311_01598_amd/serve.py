"""Serving loop: continuous batching of key-switch requests on one GPU.

* Keys (relinearisation + rotation keys) stay resident in HBM per ring
  degree, either full ([dnum][2][L+1+K][N]) or compressed (the b halves plus
  the seed of the a halves, Sec. IV-D: half the resident bytes).  A request
  names a key, a ring degree and a level and is either a key switch of its
  input polynomial, or a rotation of a ciphertext (c0, c1) by a Galois
  element with a full rotation key (the automorphism applied inside the
  key switch).
* Admission by memory: every batch needs workspace (from a preallocated HBM
  pool, first-fit) plus output buffers; requests wait while the bytes in
  flight plus theirs would exceed the budget, and a request that could never
  fit is rejected.
* Launch configuration: each plan's own.  A plan tuned for its batch shapes
  (tune.Tuner) runs with schedule AUTO, so every batch takes the autotuner's
  choice for its largest level and size; an untuned plan runs its starting
  configuration (OC, two targets per conversion tile).
* Continuous batching: whenever one of `streams` slots is free, the queued
  requests of one ring degree and kind (key switch with a full or a
  compressed key, or rotation) form a batch: the oldest request, then the
  others with its key, then the rest in arrival order.  The batch is launched
  with ks_keyswitch_batch, ks_keyswitch_batch_seeded or ks_rotate_batch on
  that slot's stream; completions are polled with
  events, so requests arriving while others run are admitted as slots and
  memory free up, and batches on different streams overlap on the device.
* Metrics: per-request latency (arrival to observed completion), p50/p99,
  key switches per second, bytes in flight high-water mark, queue depth.
"""
import collections
import gc
import time

import numpy as np


class HbmPool:
    """First-fit allocator over one preallocated device buffer (bytes)."""

    ALIGN = 256

    def __init__(self, nbytes, device="cuda"):
        import torch
        self.nbytes = (nbytes // self.ALIGN) * self.ALIGN
        self.buf = torch.empty(self.nbytes // 4, dtype=torch.int32, device=device)
        self.free = [(0, self.nbytes)]  # sorted (offset, size)

    def alloc(self, size):
        size = -(-size // self.ALIGN) * self.ALIGN
        for i, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + size, sz - size)
                return off, size
        return None

    def release(self, off, size):
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def view(self, off, size):
        return self.buf[off // 4:(off + size) // 4]


class Request:
    """A key switch of `d` with key `key`, or (galois and c0 given) the
    rotation of the ciphertext (c0, d) by that Galois element."""
    __slots__ = ("rid", "key", "log_n", "level", "d", "t_arrive", "t_start", "t_done", "out", "status", "ready",
                 "c0", "galois")

    def __init__(self, rid, key, log_n, level, d, t_arrive, c0=None, galois=None):
        self.rid, self.key, self.log_n, self.level, self.d = rid, key, log_n, level, d
        self.t_arrive, self.t_start, self.t_done = t_arrive, None, None
        self.out, self.status, self.ready = None, "queued", None
        self.c0, self.galois = c0, galois


class Server:
    def __init__(self, plans, keys, budget_bytes, streams=2, max_batch=16, keep_outputs=True):
        """plans: {log_n: Plan}; keys: {log_n: [key]} (resident), a key being
        a full evk tensor or a compressed key (b-half tensor, a_seed).
        keep_outputs=False drops each request's output once it has completed
        (a long measurement run that only needs the latencies)."""
        import torch
        self.torch = torch
        self.plans, self.keys = plans, keys
        self.budget = budget_bytes
        self.pool = HbmPool(budget_bytes)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.busy = [None] * streams  # per slot: (event, requests, pool block, bytes)
        self.max_batch = max_batch
        self.keep_outputs = keep_outputs
        self.queue = collections.deque()
        self.in_flight = 0
        self.high_water = 0
        self.done, self.failed, self.rejected = [], [], []
        self.batches = 0

    # ---------------------------------------------------------------- admission
    def _compressed(self, r):
        return isinstance(self.keys[r.log_n][r.key], tuple)

    def _kind(self, r):
        return "rotation" if r.galois is not None else ("compressed" if self._compressed(r) else "full")

    def _out_bytes(self, r):
        return 2 * (r.level + 1) * self.plans[r.log_n].n * 4

    def _need(self, batch):
        p = self.plans[batch[0].log_n]
        ws = p.workspace_bytes([r.level for r in batch])
        return ws, ws + sum(self._out_bytes(r) for r in batch)

    def submit(self, r):
        """Queue a request; rejects one that could never fit the budget."""
        if (r.log_n not in self.plans or not 0 <= r.key < len(self.keys[r.log_n])
                or not 0 <= r.level < self.plans[r.log_n].num_q
                or (r.galois is not None and (r.c0 is None or self._compressed(r)))):
            r.status = "rejected: invalid request"
            self.rejected.append(r)
            return False
        if self._need([r])[1] > self.budget:
            r.status = "rejected: over budget"
            self.rejected.append(r)
            return False
        r.ready = self.torch.cuda.Event()
        r.ready.record()  # the input is ready on the submitting stream
        self.queue.append(r)
        return True

    def _form_batch(self):
        if not self.queue:
            return None
        head = self.queue[0]
        n0, k0 = head.log_n, self._kind(head)
        # the oldest request, then the queued ones that share its key (the
        # jobs of a batch that share a key read it from L2 after the first),
        # then the rest of its degree and kind; arrival order within each
        same = [r for r in self.queue if r.log_n == n0 and self._kind(r) == k0]
        same.sort(key=lambda r: r.key != head.key)  # stable
        batch = []
        for r in same[:self.max_batch]:
            ws, need = self._need(batch + [r])
            if self.in_flight + need > self.budget:
                break
            batch.append(r)
        return batch or None

    # ---------------------------------------------------------------- loop
    def _launch(self, slot, batch):
        torch = self.torch
        ws_bytes, need = self._need(batch)
        blk = self.pool.alloc(ws_bytes)
        if blk is None:
            return False
        for r in batch:
            self.queue.remove(r)
        st = self.streams[slot]
        plan = self.plans[batch[0].log_n]
        now = time.perf_counter()
        with torch.cuda.stream(st):
            for r in batch:
                st.wait_event(r.ready)
                r.d.record_stream(st)
                if r.c0 is not None:
                    r.c0.record_stream(st)
                r.out = torch.empty((2, r.level + 1, plan.n), dtype=torch.int32, device="cuda")
                r.t_start = now
                r.status = "running"
            try:
                if self._kind(batch[0]) == "rotation":
                    from . import ks_rotate_batch
                    jobs = [(self.keys[r.log_n][r.key], r.galois, r.level, r.c0, r.d, r.out) for r in batch]
                    ks_rotate_batch(plan.handle, jobs, self.pool.view(*blk), stream=st)
                elif self._compressed(batch[0]):
                    jobs = [self.keys[r.log_n][r.key] + (r.level, r.d, r.out) for r in batch]
                    plan.keyswitch_batch_seeded(jobs, workspace=self.pool.view(*blk), stream=st)
                else:
                    jobs = [(self.keys[r.log_n][r.key], r.level, r.d, r.out) for r in batch]
                    plan.keyswitch_batch(jobs, workspace=self.pool.view(*blk), stream=st)
            except Exception as e:  # a failed launch fails only this batch
                for r in batch:
                    r.status = f"failed: {e}"
                    r.t_done = time.perf_counter()
                    self.failed.append(r)
                self.pool.release(*blk)
                return True
            ev = torch.cuda.Event()
            ev.record(st)
        self.in_flight += need
        self.high_water = max(self.high_water, self.in_flight)
        self.busy[slot] = (ev, batch, blk, need)
        self.batches += 1
        return True

    def _poll(self):
        progressed = False
        for i, b in enumerate(self.busy):
            if b is not None and b[0].query():
                ev, batch, blk, need = b
                t = time.perf_counter()
                for r in batch:
                    r.t_done = t
                    r.status = "done"
                    if not self.keep_outputs:
                        r.out = None
                    self.done.append(r)
                self.pool.release(*blk)
                self.in_flight -= need
                self.busy[i] = None
                progressed = True
        return progressed

    def step(self):
        progressed = self._poll()
        for i in range(len(self.busy)):
            if self.busy[i] is None:
                batch = self._form_batch()
                if batch and self._launch(i, batch):
                    progressed = True
        return progressed

    def idle(self):
        return not self.queue and all(b is None for b in self.busy)

    def run(self, arrivals, max_seconds=600.0, pause_gc=True):
        """arrivals: list of (t_offset_s, Request) sorted by time; drives the
        loop in real time until every request has finished.  pause_gc: the
        loop allocates many short-lived objects, and a full cyclic garbage
        collection in the middle of it stalls every request in flight, so
        it collects once before and suspends the cyclic collector until the
        run ends (reference counting still frees everything)."""
        was_enabled = gc.isenabled()
        if pause_gc:
            gc.collect()
            gc.disable()
        try:
            t0 = time.perf_counter()
            i = 0
            while i < len(arrivals) or not self.idle():
                now = time.perf_counter() - t0
                while i < len(arrivals) and arrivals[i][0] <= now:
                    r = arrivals[i][1]
                    r.t_arrive = t0 + arrivals[i][0]
                    self.submit(r)
                    i += 1
                if not self.step():
                    time.sleep(20e-6)
                if now > max_seconds:
                    raise TimeoutError("serving loop exceeded its time limit")
            self.torch.cuda.synchronize()
            return self.stats(time.perf_counter() - t0)
        finally:
            if pause_gc and was_enabled:
                gc.enable()

    def stats(self, wall):
        lat = np.array([r.t_done - r.t_arrive for r in self.done]) * 1e3
        out = {"completed": len(self.done), "failed": len(self.failed), "rejected": len(self.rejected),
               "batches": self.batches, "wall_s": wall, "ks_per_s": len(self.done) / wall if wall else 0.0,
               "high_water_bytes": self.high_water, "budget_bytes": self.budget}
        if len(lat):
            out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                        "mean_ms": float(lat.mean())})
        return out


def poisson_arrivals(rate, count, seed):
    """Arrival offsets (seconds) of a Poisson process with `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))
