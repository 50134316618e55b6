"""Scheduler of the serving loop, driven on the CPU by a backend that runs
the oracle: admission by memory, back-pressure, continuous batching,
alone-vs-mix equality, time-outs and cancellation."""
import threading
import time

import numpy as np
import pytest

from oracle import ckks
from paper_2212_14191_amd import inputs
from paper_2212_14191_amd.serving import HMULT, ROTATE, Server


class OracleBackend:
    """Same interface as GpuBackend; work runs on a worker thread."""

    def __init__(self, pr, evk, rks, delay_s=0.0):
        self.pr, self.evk, self.rks, self.delay = pr, evk, rks, delay_s
        self.lock = threading.Lock()
        self.inflight_bytes = 0
        self.peak = 0
        self.launch_log = []   # (t_start, t_end, batch size, key)

    def nbytes(self, op, log_n, level, batch):
        return (3 if op == HMULT else 2) * 2 * level * batch * (1 << log_n) * 4 + 1000 * batch

    def launch(self, slot, reqs):
        r0 = reqs[0]
        nb = self.nbytes(r0.op, r0.log_n, r0.level, len(reqs))
        with self.lock:
            self.inflight_bytes += nb
            self.peak = max(self.peak, self.inflight_bytes)
        h = {"done": False, "out": None}

        def work():
            t0 = time.perf_counter()
            time.sleep(self.delay)
            a = np.concatenate([r.ct_a for r in reqs], axis=2)
            if r0.op == HMULT:
                b = np.concatenate([r.ct_b for r in reqs], axis=2)
                out = ckks.hmult(self.pr, a, b, self.evk, r0.level)
            else:  # a batch may mix rotation amounts
                out = np.concatenate([ckks.rotate(self.pr, r.ct_a, self.rks[r.galois], r.galois, r.level)
                                      for r in reqs], axis=2)
            h["out"] = [out[:, :, i:i + 1] for i in range(len(reqs))]
            with self.lock:
                self.inflight_bytes -= nb
                self.launch_log.append((t0, time.perf_counter(), len(reqs), [r.level for r in reqs]))
            h["done"] = True

        threading.Thread(target=work, daemon=True).start()
        return h

    def done(self, h):
        return h["done"]

    def results(self, h):
        return h["out"]


@pytest.fixture(scope="module")
def world():
    n = 64
    pr = ckks.Params(n, L=6, K=2, dnum=3)
    s = inputs.ternary_secret(1, n, 16)
    a = inputs.uniform_residues(1, pr.moduli, (3, n), stream=1).transpose(1, 0, 2)
    e = inputs.gaussian_error(2, (3, n), stream=1)
    evk = ckks.relin_key(pr, s, a, e)
    gal = [ckks.galois_element(r, n) for r in (1, 2)]
    rks = {k: ckks.rotation_key(pr, s, k, a, e) for k in gal}
    cts = {}
    for level in (2, 4, 6):
        for i in range(3):
            m = inputs.small_messages(i, (1, n))
            c1 = inputs.uniform_residues(10 + i, pr.mods(range(level)), (1, n), stream=5)
            cts[(level, i)] = ckks.encrypt(pr, s, m, c1, inputs.gaussian_error(2, (1, n), stream=i), level)
    return pr, evk, rks, gal, cts


def mix(world, count=24, seed=0):
    pr, evk, rks, gal, cts = world
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        level = int(rng.choice([2, 4, 6]))
        i, j = int(rng.integers(3)), int(rng.integers(3))
        if rng.random() < 0.5:
            out.append((HMULT, level, cts[(level, i)], cts[(level, j)], None))
        else:
            out.append((ROTATE, level, cts[(level, i)], None, gal[int(rng.integers(2))]))
    return out


def run(server, reqs):
    futs = [server.submit(op, 6, lv, a, b, g) for op, lv, a, b, g in reqs]
    return [f.result(timeout=60) for f in futs]


def test_alone_equals_mix(world):
    pr, evk, rks, _, _ = world
    reqs = mix(world)
    alone = []
    for r in reqs:
        srv = Server(OracleBackend(pr, evk, rks), mem_budget_bytes=1 << 30, slots=1, max_batch=1)
        alone.append(run(srv, [r])[0])
        srv.close()
    be = OracleBackend(pr, evk, rks, delay_s=0.01)
    srv = Server(be, mem_budget_bytes=1 << 30, slots=3, max_batch=8)
    mixed = run(srv, reqs)
    st = srv.stats()
    srv.close()
    for x, y in zip(alone, mixed):
        assert np.array_equal(x, y)
    assert st["completed"] == len(reqs)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    assert max(b for _, _, b, _ in be.launch_log) > 1   # some batching happened


def test_submit_many_equals_submit(world):
    """A group submitted in one call gives each request the result it gets
    when submitted alone; a request that fails its checks gets a failed
    future while the rest of the group is served."""
    pr, evk, rks, _, cts = world
    reqs = mix(world, count=12, seed=3)
    srv = Server(OracleBackend(pr, evk, rks), mem_budget_bytes=1 << 30, slots=1, max_batch=1)
    one = run(srv, reqs)
    srv.close()
    be = OracleBackend(pr, evk, rks, delay_s=0.005)
    srv = Server(be, mem_budget_bytes=1 << 30, slots=2, max_batch=8)
    group = [(op, 6, lv, a, b, g) for op, lv, a, b, g in reqs]
    group.insert(5, (HMULT, 6, 4, cts[(4, 0)], None, None))   # no second ciphertext
    futs = srv.submit_many(group)
    with pytest.raises(ValueError):
        futs[5].result(timeout=60)
    got = [f.result(timeout=60) for i, f in enumerate(futs) if i != 5]
    srv.close()
    for x, y in zip(one, got):
        assert np.array_equal(x, y)
    assert max(b for _, _, b, _ in be.launch_log) > 1


class MixingOracleBackend(OracleBackend):
    """A backend that runs batches of mixed levels (as GpuBackend does):
    each request of a batch at its own level."""

    mixes_levels = True

    def batch_nbytes(self, reqs):
        return sum(self.nbytes(r.op, r.log_n, r.level, 1) for r in reqs)

    def launch(self, slot, reqs):
        nb = self.batch_nbytes(reqs)
        with self.lock:
            self.inflight_bytes += nb
            self.peak = max(self.peak, self.inflight_bytes)
        h = {"done": False, "out": None}

        def work():
            t0 = time.perf_counter()
            time.sleep(self.delay)
            h["out"] = [ckks.hmult(self.pr, r.ct_a, r.ct_b, self.evk, r.level) if r.op == HMULT
                        else ckks.rotate(self.pr, r.ct_a, self.rks[r.galois], r.galois, r.level) for r in reqs]
            with self.lock:
                self.inflight_bytes -= nb
                self.launch_log.append((t0, time.perf_counter(), len(reqs), [r.level for r in reqs]))
            h["done"] = True

        threading.Thread(target=work, daemon=True).start()
        return h


def test_mixed_level_batches(world):
    """With a backend that mixes levels, requests batch on (op, N) alone:
    batches hold several levels, every result equals the request alone, and
    the memory budget (sized by the batch's own levels) holds."""
    pr, evk, rks, _, _ = world
    reqs = mix(world, count=30, seed=3)
    alone = []
    for r in reqs:
        srv = Server(OracleBackend(pr, evk, rks), mem_budget_bytes=1 << 30, slots=1, max_batch=1)
        alone.append(run(srv, [r])[0])
        srv.close()
    be = MixingOracleBackend(pr, evk, rks, delay_s=0.01)
    budget = 6 * be.nbytes(HMULT, 6, 6, 1)
    srv = Server(be, mem_budget_bytes=budget, slots=2, max_batch=8)
    mixed = run(srv, reqs)
    srv.close()
    for x, y in zip(alone, mixed):
        assert np.array_equal(x, y)
    assert any(len(set(levels)) > 1 for _, _, _, levels in be.launch_log)
    assert be.peak <= budget


def test_budget_is_never_exceeded(world):
    pr, evk, rks, _, _ = world
    be = OracleBackend(pr, evk, rks, delay_s=0.005)
    budget = be.nbytes(HMULT, 6, 6, 2) + 10   # room for about two small requests
    srv = Server(be, mem_budget_bytes=budget, slots=4, max_batch=8)
    out = run(srv, mix(world, 30, seed=1))
    srv.close()
    assert len(out) == 30
    assert be.peak <= budget


def test_request_larger_than_budget_fails(world):
    pr, evk, rks, _, cts = world
    srv = Server(OracleBackend(pr, evk, rks), mem_budget_bytes=100, slots=1)
    f = srv.submit(HMULT, 6, 6, cts[(6, 0)], cts[(6, 1)])
    with pytest.raises(MemoryError):
        f.result(timeout=5)
    srv.close()


def test_continuous_batching_overlaps(world):
    """A request arriving while a batch runs is dispatched before that
    batch finishes (another slot), not after."""
    pr, evk, rks, _, cts = world
    be = OracleBackend(pr, evk, rks, delay_s=0.3)
    srv = Server(be, mem_budget_bytes=1 << 30, slots=2, max_batch=4)
    f1 = srv.submit(HMULT, 6, 6, cts[(6, 0)], cts[(6, 1)])
    time.sleep(0.05)
    f2 = srv.submit(HMULT, 6, 4, cts[(4, 0)], cts[(4, 1)])
    f1.result(timeout=10)
    f2.result(timeout=10)
    srv.close()
    (s1, e1, _, _), (s2, e2, _, _) = sorted(be.launch_log)
    assert s2 < e1   # overlapped


def test_timeout_and_cancel(world):
    pr, evk, rks, _, cts = world
    be = OracleBackend(pr, evk, rks, delay_s=0.3)
    srv = Server(be, mem_budget_bytes=1 << 30, slots=1, max_batch=1)
    f1 = srv.submit(HMULT, 6, 6, cts[(6, 0)], cts[(6, 1)])
    time.sleep(0.05)
    f2 = srv.submit(HMULT, 6, 4, cts[(4, 0)], cts[(4, 1)], timeout_s=0.01)
    f3 = srv.submit(HMULT, 6, 2, cts[(2, 0)], cts[(2, 1)])
    assert f3.cancel()
    f1.result(timeout=10)
    with pytest.raises(TimeoutError):
        f2.result(timeout=10)
    srv.drain(5)
    srv.close()
    assert len(be.launch_log) == 1


def test_rotations_by_different_amounts_share_a_batch(world):
    """Rotations of one (N, level) batch together whatever their amounts;
    each result still equals that rotation alone."""
    pr, evk, rks, gal, cts = world
    be = OracleBackend(pr, evk, rks, delay_s=0.2)
    srv = Server(be, mem_budget_bytes=1 << 30, slots=1, max_batch=8)
    blocker = srv.submit(HMULT, 6, 2, cts[(2, 0)], cts[(2, 1)])   # occupies the only slot
    time.sleep(0.05)
    reqs = [(ROTATE, 4, cts[(4, i % 3)], None, gal[i % 2]) for i in range(4)]
    futs = [srv.submit(op, 6, lv, a, b, g) for op, lv, a, b, g in reqs]
    blocker.result(timeout=10)
    got = [f.result(timeout=10) for f in futs]
    srv.close()
    sizes = sorted(b for _, _, b, _ in be.launch_log)
    assert sizes == [1, 4]
    for (op, lv, a, b, g), out in zip(reqs, got):
        assert np.array_equal(out, ckks.rotate(pr, a, rks[g], g, lv))


class FailingBackend(OracleBackend):
    """Raises on every launch at level 4."""

    def launch(self, slot, reqs):
        if reqs[0].level == 4:
            raise RuntimeError("launch failed")
        return super().launch(slot, reqs)


def test_launch_failure_surfaces_and_frees_the_slot(world):
    pr, evk, rks, _, cts = world
    srv = Server(FailingBackend(pr, evk, rks), mem_budget_bytes=1 << 30, slots=1, max_batch=4)
    bad = srv.submit(HMULT, 6, 4, cts[(4, 0)], cts[(4, 1)])
    good = srv.submit(HMULT, 6, 2, cts[(2, 0)], cts[(2, 1)])
    with pytest.raises(RuntimeError):
        bad.result(timeout=10)
    out = good.result(timeout=10)   # the slot was freed and reused
    srv.close()
    assert np.array_equal(out, ckks.hmult(pr, cts[(2, 0)], cts[(2, 1)], evk, 2))


def test_served_requests_release_their_inputs(world):
    """After completion the scheduler keeps only timings: the callers'
    ciphertexts are no longer referenced by it (a long-running server does
    not grow outside its memory budget)."""
    import gc
    import weakref
    pr, evk, rks, gal, cts = world
    srv = Server(OracleBackend(pr, evk, rks, delay_s=0.002), mem_budget_bytes=1 << 30, slots=2, max_batch=4)
    refs, futs = [], []
    for i in range(12):
        a, b = cts[(4, i % 3)].copy(), cts[(4, (i + 1) % 3)].copy()
        refs += [weakref.ref(a), weakref.ref(b)]
        futs.append(srv.submit(HMULT, 6, 4, a, b))
        del a, b
    outs = [f.result(timeout=30) for f in futs]
    assert srv.drain(10)
    gc.collect()
    assert all(r() is None for r in refs)
    assert srv.stats()["completed"] == 12
    srv.close()
    assert len(outs) == 12
