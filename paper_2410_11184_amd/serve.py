"""Serving loop for encrypted Softmax requests: continuous batching.

A request is V Softmax vectors of one dimension n (logits in [-M, 0]).  It is
packed as one job of m ciphertexts (Section 4.2: the smallest power of two m
with m N0 / n >= V, vectors beyond V padded with zeros), and requests with the
same (n, m, M) run as the jobs of one lockstep ``hs_softmax_jobs`` call, whose
outputs are bit for bit those of each job alone.

Each worker has a context and its own HIP stream: worker 0 generates the
keys, the others are clones of its context (``hs_ctx_clone``) that read the
same key memory, so one key set sits in HBM and every worker computes the
same ciphertexts; batches of different workers overlap on the device.  A worker admits pending requests
(oldest first, same shape) while the estimated device memory of everything in
flight stays within the HBM budget, so requests that arrive while others run
are taken as soon as a worker and memory are free.

The client side (packing, encryption, decryption) runs inside the worker with
per-request seeds, standing in for a remote client; it is timed separately.
"""
import math
import threading
import time

import numpy as np

from . import hs
from .softmax import decrypt_outputs, encrypt_logits


class Request:
    def __init__(self, rid, logits, M, t_arrival):
        self.rid = rid
        self.logits = np.asarray(logits, dtype=np.float64)
        self.V, self.n = self.logits.shape
        self.M = float(M)
        self.t_arrival = t_arrival
        self.t_start = None
        self.t_done = None
        self.result = None
        self.error = None
        self.batch_jobs = 0
        self.worker = -1
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


def job_shape(V, n, slots):
    """(m, L): ciphertexts per job and Softmax slots per job for V vectors."""
    if n < 2 or n & (n - 1) or n > slots:
        raise ValueError("dimension must be a power of two in [2, N/2]")
    need = max(1, math.ceil(V * n / slots))
    m = 1 << (need - 1).bit_length()
    if m > n:
        raise ValueError("too many vectors for one job of dimension %d" % n)
    return m, m * slots // n


class SoftmaxServer:
    """Continuous-batching server over `workers` contexts on one GPU."""

    def __init__(self, params, workers=2, hbm_budget_gb=64.0, key_seed=2024, variant=1, max_jobs=64,
                 bytes_per_ct=None, device=0, softmax_kw=None, warm_dims=()):
        self.params = params
        self.slots = params["slots"]
        self.variant = variant
        self.softmax_kw = dict(softmax_kw or {})
        self.max_jobs = max_jobs
        self.budget = hbm_budget_gb * 1e9
        # peak working memory per ciphertext of a Softmax job (key-switching
        # buffers dominate): about 12 ciphertexts' worth at the top user level
        # for version B; 3 times that when the main ciphertexts are bootstrapped
        self.bytes_per_ct = bytes_per_ct or 12 * 2 * (params["user_top"] + 1) * params["N"] * 8
        self.lock = threading.Condition()
        self.pending = []
        self.in_flight = 0.0
        self.exclusive = 0          # batches waiting to run alone after running out of memory
        self.finished = []
        self.closed = False
        self.device, self.key_seed = device, key_seed
        self.contexts, self.streams = [], []
        for w in range(workers):
            self.streams.append(hs.stream_create(device))
            # worker 0 holds the key set, the others share it (one copy in HBM)
            self.contexts.append(self._make_context(w) if w == 0 else self.contexts[0].clone(self.streams[w]))
        # one small Softmax per worker and warm dimension builds the bootstrap
        # tables and keys before the first request
        for w, ctx in enumerate(self.contexts):
            for n in warm_dims:
                r = Request(-1, np.zeros((1, n)), 8.0, time.perf_counter())
                self._run(ctx, [r], w)
        self.threads = [threading.Thread(target=self._worker, args=(w,), daemon=True) for w in range(workers)]
        for t in self.threads:
            t.start()

    def _make_context(self, w):
        ctx = hs.Context(self.params, device=self.device, stream=self.streams[w])
        ctx.keygen(self.key_seed)
        # every power-of-two stride (both directions): no key generation while serving
        ctx.add_rotation_keys([s * (1 << t) for t in range(int(math.log2(self.slots))) for s in (1, -1)])
        return ctx

    # ------------------------------------------------------------ clients
    def submit(self, rid, logits, M, t_arrival=None):
        r = Request(rid, logits, M, time.perf_counter() if t_arrival is None else t_arrival)
        job_shape(r.V, r.n, self.slots)        # validate now
        with self.lock:
            self.pending.append(r)
            self.lock.notify_all()
        return r

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for t in self.threads:
            t.join()
        for ctx in self.contexts:
            ctx.sync()
        self.contexts = []
        import gc
        gc.collect()
        for st in self.streams:
            hs.stream_destroy(st)
        self.streams = []

    # ------------------------------------------------------------ workers
    def _admit(self):
        """Oldest pending request and every pending request of its shape,
        within the memory budget (at least one request when nothing runs)."""
        if not self.pending:
            return [], 0.0
        first = self.pending[0]
        m, _ = job_shape(first.V, first.n, self.slots)
        key = (first.n, m, first.M)
        batch, cost = [], 0.0
        for r in list(self.pending):
            rm, _ = job_shape(r.V, r.n, self.slots)
            if (r.n, rm, r.M) != key:
                continue
            c = rm * self.bytes_per_ct * (1 if self._variant(r.n, r.M) == 1 else 3)
            if batch and (self.in_flight + cost + c > self.budget or len(batch) >= self.max_jobs):
                break
            if not batch and self.in_flight > 0 and self.in_flight + c > self.budget:
                return [], 0.0                  # wait for memory
            batch.append(r)
            cost += c
        for r in batch:
            self.pending.remove(r)
        return batch, cost

    def _worker(self, w):
        while True:
            with self.lock:
                while True:
                    batch, cost = self._admit() if not self.exclusive else ([], 0.0)
                    if batch or (self.closed and not self.pending):
                        break
                    self.lock.wait(0.05)
                if not batch:
                    return
                self.in_flight += cost
            try:
                self._run_with_retry(w, batch, cost)
            except Exception as e:          # a failed batch fails its requests, not the server
                for r in batch:
                    r.error = e
                    r.t_done = time.perf_counter()
            with self.lock:
                self.in_flight -= cost
                for r in batch:
                    self.finished.append(r)
                    r.done.set()
                self.lock.notify_all()

    def _run_with_retry(self, w, batch, cost):
        try:
            self._run(self.contexts[w], batch, w)
        except hs.HSError as e:
            if e.name != "HS_E_OOM":
                raise
            # retry once with the GPU to ourselves, on a fresh context (the
            # failed call may have left blocks of its own allocated)
            with self.lock:
                self.exclusive += 1
                while self.in_flight > cost + 1.0:
                    self.lock.wait(0.05)
            try:
                self.contexts[w].sync()
                if w > 0:
                    # a fresh clone (the failed call may have left blocks of its own allocated)
                    self.contexts[w] = None
                    import gc
                    gc.collect()
                    self.contexts[w] = self.contexts[0].clone(self.streams[w])
                else:
                    self.contexts[0].trim()   # its clones share its keys: kept, trimmed
                self._run(self.contexts[w], batch, w)
            finally:
                with self.lock:
                    self.exclusive -= 1
                    self.lock.notify_all()
        finally:
            # return this worker's free memory to the device, so the other
            # workers' batches can grow into it
            if len(self.contexts) > 1 and self.contexts[w] is not None:
                self.contexts[w].trim()

    def _variant(self, n, M):
        # version B needs k + 2 main-thread levels after the exponential
        # (k <= 5 with twelve user levels; k as the library takes it: the
        # Theorem's, plus one from n = 4096); above n = 16384 its
        # intermediate normalisations cannot hold the intervals, and
        # Algorithm SM with Newton's steps is the more precise
        k = self.softmax_kw.get("k") or (max(1, math.ceil(math.log2(M) - math.log2(math.log(n))))
                                         + (1 if n >= 4096 else 0))
        return self.variant if (n <= 16384 and k <= 5) else 0

    def _run(self, ctx, batch, w):
        n, M = batch[0].n, batch[0].M
        m, L = job_shape(batch[0].V, n, self.slots)
        t0 = time.perf_counter()
        cts = []
        for r in batch:
            r.t_start = t0
            x = np.zeros((L, n))
            x[:r.V] = r.logits
            cts += encrypt_logits(ctx, x, M, seed=100003 * (r.rid + 1))
        out = ctx.softmax(cts, n, M, variant=self._variant(n, M), jobs=len(batch), **self.softmax_kw)
        del cts
        for i, r in enumerate(batch):
            y = decrypt_outputs(ctx, out[i * m:(i + 1) * m], n)
            r.result = y[:r.V]
            r.batch_jobs = len(batch)
            r.worker = w
            r.t_done = time.perf_counter()
        del out


def latency_stats(requests):
    lat = np.array([r.latency for r in requests if r.latency is not None])
    if lat.size == 0:
        return {}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}
