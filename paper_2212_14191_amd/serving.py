"""Continuous-batching request loop for HMULT / HROTATE (the API layer of
Sec. IV-E: requests are collected, decomposed into batched kernel workflows
and dispatched; keys and ciphertexts stay resident in HBM).

A scheduler thread keeps up to `slots` batches in flight, each on its own
HIP stream.  Pending requests are grouped by (op, N) when the backend runs
batches of mixed levels (operation-level batching across levels, Sec. IV-D;
the GPU backend does, through tfhe_hmult_levels / tfhe_rotate_levels), else
by (op, N, level); rotations by different amounts share a batch (each
ciphertext with its own Galois element and key, one batched launch
sequence);
whenever a slot is free, the oldest pending request and up to max_batch - 1
compatible ones form a batch, provided its device memory (staged inputs,
outputs, workspace) fits the remaining budget; otherwise admission waits
(back-pressure).  Requests that arrive while other batches run are admitted
as soon as a slot and memory free up, so their work overlaps on the device.
Each result depends only on its own inputs: batching never changes bits.

The backend does the device work (GpuBackend below); tests drive the same
scheduler with a CPU backend.
"""
import collections
import concurrent.futures
import heapq
import threading
import time

import numpy as np

HMULT, ROTATE = 0, 1


class Request:
    __slots__ = ("op", "log_n", "level", "galois", "ct_a", "ct_b", "future", "t_submit", "t_done",
                 "deadline", "ready")

    def __init__(self, op, log_n, level, galois, ct_a, ct_b, timeout_s):
        self.op, self.log_n, self.level, self.galois = op, log_n, level, galois
        self.ct_a, self.ct_b = ct_a, ct_b
        self.future = concurrent.futures.Future()
        self.t_submit = time.perf_counter()
        self.t_done = None
        self.deadline = None if timeout_s is None else self.t_submit + timeout_s
        self.ready = None  # backend-specific readiness marker of the inputs

    def key(self, mix_levels):
        """Batching key: rotations by different amounts batch together, and
        levels too where the backend mixes them."""
        return (self.op, self.log_n) if mix_levels else (self.op, self.log_n, self.level)


class Server:
    def __init__(self, backend, mem_budget_bytes, slots=4, max_batch=16, poll_s=1e-5, max_batch_by_n=None):
        self.backend = backend
        self.budget = int(mem_budget_bytes)
        self.slots = int(slots)
        # a backend may cap the batch (the GPU backend: TFHE_ROTATE_MULTI_MAX)
        cap = getattr(backend, "max_batch", int(max_batch))
        self.max_batch = min(int(max_batch), cap)
        # per-N limits (the autotuner's choice, autotune.serving_batches)
        self.max_batch_by_n = {int(k): max(1, min(int(v), cap)) for k, v in (max_batch_by_n or {}).items()}
        # a backend that runs batches of mixed levels says so and sizes them
        # with batch_nbytes(requests)
        self.mix = bool(getattr(backend, "mixes_levels", False))
        self.poll_s = poll_s
        self._pending = collections.OrderedDict()  # id -> Request (FIFO)
        self._by_key = {}                           # batching key -> deque of ids (FIFO)
        self._deadlines = []                        # heap of (deadline, id)
        self._inflight = []                         # (handle, requests, nbytes, slot)
        self._free_slots = list(range(self.slots))
        self._used = 0
        self._peak_used = 0
        self._lock = threading.Condition()
        self._done = []                             # (t_submit, t_done) of completed requests
        self._stop = False
        self._next_id = 0
        self._t0 = None
        self._thread = threading.Thread(target=self._run, name="tfhe-serving", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------------ API
    def submit(self, op, log_n, level, ct_a, ct_b=None, galois=None, timeout_s=None):
        """Queue an HMULT (ct_a * ct_b) or a rotation of ct_a by the Galois
        element `galois`.  Returns a Future resolving to the output."""
        if op == HMULT and ct_b is None:
            raise ValueError("HMULT needs two ciphertexts")
        if op == ROTATE and galois is None:
            raise ValueError("rotation needs a Galois element")
        req = Request(op, log_n, level, galois, ct_a, ct_b, timeout_s)
        need = self.backend.nbytes(op, log_n, level, 1)
        if need > self.budget:
            req.future.set_exception(MemoryError(f"request needs {need} B > budget {self.budget} B"))
            return req.future
        prepare = getattr(self.backend, "prepare", None)
        if prepare is not None:  # e.g. mark when the inputs are ready (caller's thread)
            prepare(req)
        with self._lock:
            if self._t0 is None:
                self._t0 = req.t_submit
            self._pending[self._next_id] = req
            self._by_key.setdefault(req.key(self.mix), collections.deque()).append(self._next_id)
            if req.deadline is not None:
                heapq.heappush(self._deadlines, (req.deadline, self._next_id))
            self._next_id += 1
            self._lock.notify()
        return req.future

    def submit_many(self, reqs, timeout_s=None):
        """Queue several requests at once: reqs is a list of (op, log_n,
        level, ct_a, ct_b, galois) tuples (ct_b None for a rotation, galois
        None for HMULT).  One lock acquisition and, on the GPU backend, one
        readiness event for the whole group.  Returns their Futures, in
        order; a request that fails its checks gets a failed Future and the
        others are queued."""
        out, ok = [], []
        for op, log_n, level, ct_a, ct_b, galois in reqs:
            req = Request(op, log_n, level, galois, ct_a, ct_b, timeout_s)
            out.append(req.future)
            if op == HMULT and ct_b is None:
                req.future.set_exception(ValueError("HMULT needs two ciphertexts"))
                continue
            if op == ROTATE and galois is None:
                req.future.set_exception(ValueError("rotation needs a Galois element"))
                continue
            need = self.backend.nbytes(op, log_n, level, 1)
            if need > self.budget:
                req.future.set_exception(MemoryError(f"request needs {need} B > budget {self.budget} B"))
                continue
            ok.append(req)
        prepare_many = getattr(self.backend, "prepare_many", None)
        prepare = getattr(self.backend, "prepare", None)
        if prepare_many is not None:
            bad = prepare_many(ok)
        else:
            bad = set()
            for i, r in enumerate(ok):
                try:
                    if prepare is not None:
                        prepare(r)
                except Exception as e:  # noqa: BLE001 - surfaced on the request's future
                    r.future.set_exception(e)
                    bad.add(i)
        with self._lock:
            for i, req in enumerate(ok):
                if i in bad:
                    continue
                if self._t0 is None:
                    self._t0 = req.t_submit
                self._pending[self._next_id] = req
                self._by_key.setdefault(req.key(self.mix), collections.deque()).append(self._next_id)
                if req.deadline is not None:
                    heapq.heappush(self._deadlines, (req.deadline, self._next_id))
                self._next_id += 1
            self._lock.notify()
        return out

    def stats(self):
        with self._lock:
            lat = np.array([t1 - t0 for t0, t1 in self._done])
            n = len(lat)
            span = (max(t1 for _, t1 in self._done) - self._t0) if n else 0.0
            return {
                "completed": n,
                "throughput_per_s": n / span if span > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if n else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if n else None,
                "mean_batch": (n / self._batches) if getattr(self, "_batches", 0) else None,
                "peak_mem_bytes": self._peak_used,
            }

    def reset_stats(self):
        with self._lock:
            self._done = []
            self._t0 = None
            self._batches = 0
            self._peak_used = self._used

    def drain(self, timeout_s=None):
        t_end = None if timeout_s is None else time.perf_counter() + timeout_s
        while True:
            with self._lock:
                if not self._pending and not self._inflight:
                    return True
            if t_end is not None and time.perf_counter() > t_end:
                return False
            time.sleep(self.poll_s)

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify()
        self._thread.join()

    # ------------------------------------------------------------ scheduler
    def _expired(self, r, now):
        return r.future.cancelled() or (r.deadline is not None and now > r.deadline)

    def _drop(self, rid):
        """Remove a cancelled or timed-out request from the queue."""
        r = self._pending.pop(rid)
        k = r.key(self.mix)
        q = self._by_key[k]
        q.remove(rid)
        if not q:
            del self._by_key[k]
        if not r.future.cancelled():
            r.future.set_exception(TimeoutError("request timed out in the queue"))

    def _form_batch(self):
        """Oldest pending request plus compatible ones, within the budget.
        Cost O(batch): requests are indexed by batching key, time-outs come
        off a deadline heap, and cancellations are dropped when a candidate
        is taken."""
        now = time.perf_counter()
        while self._deadlines and self._deadlines[0][0] < now:
            _, rid = heapq.heappop(self._deadlines)
            if rid in self._pending:
                self._drop(rid)
        while self._pending:
            hid, head = next(iter(self._pending.items()))
            if not self._expired(head, now):
                break
            self._drop(hid)
        if not self._pending:
            return None
        ids = []
        limit = self.max_batch_by_n.get(head.log_n, self.max_batch)
        # the oldest request, then the others of its level, then the rest
        # (each in arrival order): fewer level groups per mixed batch
        for same in ((True, False) if self.mix else (True,)):
            for rid in self._by_key[head.key(self.mix)]:
                if len(ids) == limit:
                    break
                r = self._pending[rid]
                if (r.level == head.level) == same and not self._expired(r, now):
                    ids.append(rid)
        while ids:
            if self.mix:
                need = self.backend.batch_nbytes([self._pending[i] for i in ids])
            else:
                need = self.backend.nbytes(head.op, head.log_n, head.level, len(ids))
            if self._used + need <= self.budget:
                return ids, need
            if len(ids) == 1:
                return None  # wait for memory
            ids = ids[: len(ids) // 2]
        return None

    def _run(self):
        self._batches = 0
        while True:
            with self._lock:
                if self._stop:
                    return
                # completions
                still = []
                for h, reqs, nbytes, slot in self._inflight:
                    if self.backend.done(h):
                        outs = self.backend.results(h)
                        t = time.perf_counter()
                        for r, o in zip(reqs, outs):
                            r.t_done = t
                            # the scheduler keeps only the timing: inputs
                            # and outputs belong to the callers from here on
                            r.ct_a = r.ct_b = r.ready = None
                            if not r.future.cancelled():
                                r.future.set_result(o)
                            self._done.append((r.t_submit, t))
                        self._used -= nbytes
                        self._free_slots.append(slot)
                    else:
                        still.append((h, reqs, nbytes, slot))
                self._inflight = still
                # admissions
                while self._free_slots:
                    fb = self._form_batch()
                    if fb is None:
                        break
                    ids, nbytes = fb
                    reqs = [self._pending.pop(rid) for rid in ids]
                    k = reqs[0].key(self.mix)
                    q = self._by_key[k]
                    for rid in ids:
                        q.remove(rid)
                    if not q:
                        del self._by_key[k]
                    for r in reqs:
                        r.future.set_running_or_notify_cancel()
                    slot = self._free_slots.pop()
                    self._used += nbytes
                    self._peak_used = max(self._peak_used, self._used)
                    try:
                        h = self.backend.launch(slot, reqs)
                    except Exception as e:  # surface to the callers, free the slot
                        for r in reqs:
                            r.future.set_exception(e)
                        self._used -= nbytes
                        self._free_slots.append(slot)
                        continue
                    self._batches += 1
                    self._inflight.append((h, reqs, nbytes, slot))
                idle = not self._pending and not self._inflight
                if idle:
                    self._lock.wait(timeout=0.05)
            if not idle:
                time.sleep(self.poll_s)


class GpuBackend:
    """Device backend: one CkksContext per N, resident keys, one HIP stream
    per slot.  A request alone runs in place (tfhe_hmult / tfhe_rotate at
    batch 1); a batch of several, whatever their levels, runs as one
    mixed-level launch sequence (tfhe_hmult_levels / tfhe_rotate_levels) that
    reads every input where it is and writes each request's own output
    tensor.  Each slot keeps one workspace, grown to the largest batch it has
    run."""

    mixes_levels = True
    max_batch = 64  # TFHE_HMULT_LEVELS_MAX

    def __init__(self, contexts, relin_keys, rot_keys, slots=4):
        import torch
        from . import tfhe
        self.tfhe = tfhe
        self.torch = torch
        self.ctx = contexts          # log_n -> CkksContext
        self.evk = relin_keys        # log_n -> tensor
        self.rk = rot_keys           # (log_n, galois) -> tensor
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self._sptr = [s.cuda_stream for s in self.streams]  # raw HIP stream handles
        # completion events, one per slot (a slot runs one batch at a time)
        self.events = [torch.cuda.Event() for _ in range(slots)]
        self._wsb = {}  # (log_n, level, batch) -> workspace bytes
        # one workspace per slot, grown to the largest batch it has run (a
        # slot's next batch starts only after its previous one completed)
        self.ws = [None] * slots

    def prepare(self, req):
        """Called in the submitting thread: checks the inputs (so that the
        scheduler can pass raw pointers) and records an event on the
        submitter's current stream that marks when they are ready."""
        self._check(req)
        st = self.torch.cuda.current_stream()
        ev = self.torch.cuda.Event()
        ev.record(st)
        req.ready = (st.cuda_stream, ev, st)

    def _check(self, req):
        ctx = self.ctx.get(req.log_n)
        if ctx is None:
            raise ValueError(f"no context for N = 2^{req.log_n}")
        shape = (2, req.level, 1, ctx.n)
        for t in ((req.ct_a, req.ct_b) if req.op == HMULT else (req.ct_a,)):
            if (t.dtype != self.torch.int32 or not t.is_cuda or not t.is_contiguous()
                    or t.numel() != 2 * req.level * ctx.n):
                raise ValueError(f"ciphertexts must be contiguous int32 device tensors of {shape} elements")
        if req.op == ROTATE and (req.log_n, req.galois) not in self.rk:
            raise ValueError(f"no rotation key for Galois element {req.galois}")

    def prepare_many(self, reqs):
        """prepare() for a group submitted together: every request is
        checked and all share one readiness event, recorded once on the
        submitter's current stream.  Returns the indices of the requests
        that failed their checks (their futures carry the error)."""
        bad = set()
        st = self.torch.cuda.current_stream()
        ev = None
        for i, req in enumerate(reqs):
            try:
                self._check(req)
            except Exception as e:  # noqa: BLE001 - surfaced on the request's future
                req.future.set_exception(e)
                bad.add(i)
                continue
            if ev is None:
                ev = self.torch.cuda.Event()
                ev.record(st)
            req.ready = (st.cuda_stream, ev, st)
        return bad

    def _ws_bytes(self, log_n, level, batch):
        k = (log_n, level, batch)
        b = self._wsb.get(k)
        if b is None:
            b = self._wsb[k] = max(self.ctx[log_n].workspace_bytes(level, batch), 256)
        return b

    def nbytes(self, op, log_n, level, batch):
        """Device memory of a same-level batch of `batch` requests."""
        n = 1 << log_n
        ct = 2 * level * batch * n * 4
        if batch == 1:  # in place: the output and the workspace
            return ct + self._ws_bytes(log_n, level, 1)
        return ct + max(self.ctx[log_n].levels_workspace_bytes([level] * batch), 256)

    def batch_nbytes(self, reqs):
        """Device memory of a batch of these requests (levels may differ):
        their outputs and the workspace."""
        r0 = reqs[0]
        if len(reqs) == 1:
            return self.nbytes(r0.op, r0.log_n, r0.level, 1)
        levels = [r.level for r in reqs]
        out = sum(2 * lv * (1 << r0.log_n) * 4 for lv in levels)
        return out + max(self.ctx[r0.log_n].levels_workspace_bytes(levels), 256)

    def _slot_ws(self, slot, need):
        w = self.ws[slot]
        if w is None or w.numel() < need:
            w = self.torch.empty(need, dtype=self.torch.uint8, device="cuda")
            self.ws[slot] = w
        return w

    def launch(self, slot, reqs):
        torch = self.torch
        r0 = reqs[0]
        ctx = self.ctx[r0.log_n]
        B, n = len(reqs), 1 << r0.log_n
        s = self.streams[slot]
        # inputs ready: the latest submission event of each submitting stream
        # (events on one stream complete in order)
        latest = {}
        for r in reqs:
            if r.ready is not None:
                latest[r.ready[0]] = r.ready[1]
            else:
                latest[None] = None
        for key, ev in latest.items():
            if ev is None:
                s.wait_stream(torch.cuda.current_stream())
            else:
                s.wait_event(ev)
        # this thread only launches batches: allocations below belong to s
        torch.cuda.set_stream(s)
        outs = [torch.empty((2, r.level, 1, n), dtype=torch.int32, device="cuda") for r in reqs]
        sp = self._sptr[slot]
        tfhe = self.tfhe
        # inputs were checked in prepare(): raw pointers into the C ABI
        if B == 1:
            level = r0.level
            ws = self._slot_ws(slot, self._ws_bytes(r0.log_n, level, 1))
            if r0.op == HMULT:
                tfhe._call("tfhe_hmult", ctx.handle, r0.ct_a.data_ptr(), r0.ct_b.data_ptr(), outs[0].data_ptr(),
                           self.evk[r0.log_n].data_ptr(), level, 1, ws.data_ptr(), ws.numel(), sp)
            else:
                tfhe._call("tfhe_rotate", ctx.handle, r0.ct_a.data_ptr(), outs[0].data_ptr(),
                           self.rk[(r0.log_n, r0.galois)].data_ptr(), r0.galois, level, 1, ws.data_ptr(),
                           ws.numel(), sp)
        else:
            levels = [r.level for r in reqs]
            ws = self._slot_ws(slot, max(ctx.levels_workspace_bytes(levels), 256))
            view = lambda t, r: t.view(2, r.level, n)
            if r0.op == HMULT:
                ctx.hmult_levels([view(r.ct_a, r) for r in reqs], [view(r.ct_b, r) for r in reqs],
                                 self.evk[r0.log_n], outs=[view(o, r) for o, r in zip(outs, reqs)], ws=ws, stream=s)
            else:
                ctx.rotate_levels([view(r.ct_a, r) for r in reqs], [self.rk[(r0.log_n, r.galois)] for r in reqs],
                                  [r.galois for r in reqs], outs=[view(o, r) for o, r in zip(outs, reqs)], ws=ws,
                                  stream=s)
        ev = self.events[slot]
        ev.record(s)
        # the result tensors are allocated on s but read by the submitters on
        # their streams: the caching allocator must not hand them out again
        # on s before their work on them has finished
        users = {r.ready[0]: r.ready[2] for r in reqs if r.ready is not None}
        for st in users.values():
            for o in outs:
                o.record_stream(st)
        return {"event": ev, "outs": outs, "keep": (ws, [(r.ct_a, r.ct_b) for r in reqs])}

    def done(self, h):
        return h["event"].query()

    def results(self, h):
        """Each request's own output [2][level][1][N]; the futures resolve
        after the batch's device work has completed."""
        return h["outs"]
