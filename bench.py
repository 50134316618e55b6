#!/usr/bin/env python
"""Benchmark of the NTT / HMULT hot path on one MI355X.

One step = forward NTT then inverse NTT of a batch of N = 2^16 polynomials:
44 limbs (31-bit primes, q = 1 mod 2^17) x 128 polynomials, uniform residues,
computed with the four-step INT8-MFMA transform.  `value` is that transform's
throughput in KOPS (10^3 limb-transforms per second; one limb-transform is
one N-point NTT or INTT over one prime).  Measured beside it on the same data:
the radix-2 butterfly transform, the vector-ALU GEMM variant of the four-step
transform, the batched HMULT (N=2^16, L=24, K=8, dnum=3, 64 ciphertext
pairs) and RESCALE, the serving mix, and the plain CPU oracle on a bounded
sample.

Prints one JSON line.  Inputs are resident in HBM before timing starts.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LOG_N, LIMBS, BATCH = 16, 44, 128
HM_L, HM_K, HM_DNUM, HM_BATCH = 24, 8, 3, 64
METRIC = "NTT KOPS & HMULT ops/s at N=2^16, MFMA vs butterfly; p99 request latency"
HBM_PEAK_GBS = 8000.0
MFMA_I8_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak of the part
# int8 matrix-core work of one four-step pass at N = 2^16 (a 256-point stage
# split 16 x 16): per 256 coefficients, 8 v_mfma_i32_16x16x64_i8 (two
# 16-point levels x 4 twiddle digit planes) of 16 x 16 x 64 multiply-adds
I8_OPS_PER_COEFF_PASS = 8 * 16 * 16 * 64 * 2 // 256


# Sources that determine the four-step kernels' memory traffic; the profile
# summary records their hash next to the hardware byte counts.
# (and the tune table, which sets the launch shape the benchmark uses)
TRAFFIC_SOURCES = ("csrc/ntt_fourstep.hip", "csrc/fourstep_dev.hpp", "csrc/internal.hpp", "csrc/modarith.hpp",
                   "csrc/plan.cpp", "tune_mi355x.json")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ntt_mfma_n16_44x128.md")
# the HMULT benchmark's kernels: the transforms plus the key-switching code,
# and the rules that set its context's launch shape
HMULT_SOURCES = TRAFFIC_SOURCES + ("csrc/ckks.cpp", "csrc/ckks_kernels.hip", "csrc/ckks_internal.hpp",
                                   "autotune.py")
HMULT_PROFILE = os.path.join(ROOT, "profiles", "hmult_n16_l24_b64.md")


def _code_only(text):
    """Source text without comments and blank lines (so that comment edits
    do not invalidate a profile record)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", l).rstrip() for l in text.splitlines())
    return "\n".join(l for l in lines if l.strip())


def kernel_source_hash(sources=TRAFFIC_SOURCES):
    h = hashlib.sha256()
    for rel in sources:
        path = os.path.join(ROOT, "paper_2212_14191_amd", rel)
        if os.path.exists(path):
            with open(path) as f:
                h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def profile_record(key, path=TRAFFIC_PROFILE, sources=TRAFFIC_SOURCES):
    """The JSON record `key: {...}` of a committed rocprofv3 summary, or
    None when it is missing or was taken from different kernel sources."""
    try:
        with open(path) as f:
            m = re.search(r"^" + key + r": (\{.*\})$", f.read(), re.M)
        d = json.loads(m.group(1)) if m else None
    except (OSError, ValueError):
        return None
    if not d or d.get("source_sha256") != kernel_source_hash(sources):
        return None
    return d


def hmult_roofline(ops_per_s, n, L, K, dnum, batch):
    """HMULT against the 8 TB/s HBM peak, two ways: with the algorithmic
    bytes of one HMULT (the two input ciphertexts and the output, [2][L][N]
    words each, and a 1/batch share of the key, [dnum][2][L+K][N]), and with
    the bytes its kernels move, as the committed counter summary records
    them (None when missing or stale)."""
    alg = 4 * n * (6 * L) + 4 * n * 2 * dnum * (L + K) / batch
    rec = profile_record("hmult_traffic", HMULT_PROFILE, HMULT_SOURCES)
    meas = rec.get("bytes_per_hmult") if rec else None
    out = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "algorithmic_bytes_per_op": round(alg),
           "achieved_algorithmic": round(ops_per_s * alg / 1e9, 1),
           "frac_algorithmic": round(ops_per_s * alg / 1e9 / HBM_PEAK_GBS, 4),
           "measured_bytes_per_op": meas, "achieved_measured": None, "frac_measured": None}
    if meas:
        out["achieved_measured"] = round(ops_per_s * meas / 1e9, 1)
        out["frac_measured"] = round(ops_per_s * meas / 1e9 / HBM_PEAK_GBS, 4)
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when the summary is missing or stale."""
    d = profile_record("traffic")
    return d.get("bytes_per_launch", {}).get(kernel) if d else None


def measured_mfma(kernel):
    """Matrix-core counters per launch of `kernel` from the committed
    summary (SQ_INSTS_VALU_MFMA_MOPS_I8, SQ_VALU_MFMA_BUSY_CYCLES,
    GRBM_GUI_ACTIVE, and what they imply), or None when missing or stale."""
    d = profile_record("mfma")
    return d.get("per_launch", {}).get(kernel) if d else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return time.perf_counter() - t0


def host_cpu():
    """CPU model name and the number of cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_ntt_rate(qs, psis, budget_s, threads):
    """Forward + inverse radix-2 oracle transforms of whole N = 2^16
    limb-polynomials on `threads` host threads (0 = all), sized from a warm
    probe over every limb to take about budget_s."""
    import oracle
    from paper_2212_14191_amd import inputs
    n = 1 << LOG_N
    # probe on every limb (per-limb tables are built once per call and
    # amortised over the polynomials, as in the sample itself)
    probe_batch = 8 if threads != 1 else 1
    probe_units = LIMBS * probe_batch
    x = inputs.uniform_residues(0, qs[:LIMBS], (probe_batch, n))
    oracle.ntt(x, qs[:LIMBS], psis[:LIMBS], threads=threads)  # loads the library, starts the thread pool
    t0 = time.perf_counter()
    X, used = oracle.ntt(x, qs[:LIMBS], psis[:LIMBS], threads=threads)
    oracle.ntt(X, qs[:LIMBS], psis[:LIMBS], inverse=True, threads=threads)
    dt = time.perf_counter() - t0
    per_unit = dt / probe_units
    units = int(max(probe_units, min(LIMBS * BATCH, budget_s / max(per_unit, 1e-6))))
    limbs = min(LIMBS, units)
    batch = max(1, units // limbs)
    x = inputs.uniform_residues(0, qs[:limbs], (batch, n))
    t0 = time.perf_counter()
    X, used = oracle.ntt(x, qs[:limbs], psis[:limbs], threads=threads)
    back, _ = oracle.ntt(X, qs[:limbs], psis[:limbs], inverse=True, threads=threads)
    dt = time.perf_counter() - t0
    assert np.array_equal(back, x)
    transforms = 2 * limbs * batch
    return (transforms / dt / 1e3, int(used),
            f"{limbs} limbs x {batch} polys of N=2^16, forward+inverse radix-2 ({transforms} limb-transforms, "
            f"{dt:.1f} s)")


def _oracle_hmult_time():
    """The oracle's HMULT of one ciphertext pair at the HMULT benchmark
    shape (N = 2^16, L = 24, K = 8, dnum = 3, level 24); keys and
    encryption are set-up, outside the clock."""
    from oracle import ckks
    from paper_2212_14191_amd import inputs
    n = 1 << LOG_N
    pr = ckks.Params(n, L=HM_L, K=HM_K, dnum=HM_DNUM)
    s = inputs.ternary_secret(1, n, 192)
    a = inputs.uniform_residues(1, pr.moduli, (HM_DNUM, n), stream=1).transpose(1, 0, 2)
    e = inputs.gaussian_error(2, (HM_DNUM, n), stream=1)
    evk = ckks.relin_key(pr, s, a, e)
    cts = []
    for k in range(2):
        m = inputs.small_messages(0, (1, n), stream=k)
        c1 = inputs.uniform_residues(10 + k, pr.mods(range(HM_L)), (1, n), stream=5)
        cts.append(ckks.encrypt(pr, s, m, c1, inputs.gaussian_error(2, (1, n), stream=20 + k), HM_L))
    t0 = time.perf_counter()
    ckks.hmult(pr, cts[0], cts[1], evk, HM_L)
    return time.perf_counter() - t0


def cpu_baseline(qs, psis, budget_s=10.0):
    """The oracle as it stands, on the host: its radix-2 NTT+INTT on a
    bounded sample of the same workload (whole limb-polynomials of
    N = 2^16) on all host cores and on one core, and its HMULT of one pair
    at the HMULT benchmark shape."""
    model, nproc = host_cpu()
    kops, used, sample = _oracle_ntt_rate(qs, psis, budget_s, 0)
    kops1, _, sample1 = _oracle_ntt_rate(qs, psis, budget_s / 3, 1)
    hm_s = _oracle_hmult_time()
    return {"value": kops, "unit": "KOPS (10^3 limb-transforms/s)", "cores": used, "kind": "oracle",
            "sample": sample, "cpu_model": model, "nproc": nproc,
            "single_core": {"value": kops1, "unit": "KOPS", "cores": 1, "sample": sample1},
            "hmult": {"ms_per_op": round(1e3 * hm_s, 1), "ops_per_s": round(1 / hm_s, 3), "cores": used,
                      "sample": "1 ciphertext pair, N=2^16, L=24, K=8, dnum=3, level 24 "
                                "(numpy element-wise steps, C transforms on all cores)"}}


P99_BOUND_MS = 5.0


def sustainable_rate(fn, saturated, n_req, probes=7, keep_up=0.95):
    """Highest Poisson arrival rate (requests/s) whose p99 submit-to-done
    latency stays at or below P99_BOUND_MS while the measured throughput
    keeps up with it (at least keep_up x the rate: a backlog that grows, or
    a submitting loop that falls behind the schedule, is not sustained), by
    bisection on the fraction of the saturated rate (each probe serves
    min(n_req, 4000) requests of the same mix; the arrivals' seed differs
    from the load points')."""
    count = min(n_req, 4000)
    lo, hi, best = 0.0, 1.0, None
    for _ in range(probes):
        frac = (lo + hi) / 2
        st = fn(count, 4, frac * saturated)
        rec = {"rate_per_s": round(frac * saturated, 1), "throughput_per_s": round(st["throughput_per_s"], 1),
               "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3)}
        if st["p99_ms"] <= P99_BOUND_MS and st["throughput_per_s"] >= keep_up * frac * saturated:
            lo, best = frac, rec
        else:
            hi = frac
    return {"p99_bound_ms": P99_BOUND_MS, "keep_up": keep_up, "requests_per_probe": count, "probes": probes,
            "rate_per_s": best["rate_per_s"] if best else 0.0, "at_rate": best}


def serving_leg(n_sat, n_req, fracs, torch, tfhe, inputs, engines=("python", "native"), native_slots=8,
                table=None, batch_ms=None):
    """Config 5: Poisson HMULT / rotate requests, N in {2^13..2^16}, levels
    uniform in 1..24, 8 rotation keys per N, keys and ciphertexts resident,
    memory-gated continuous batching.  Returns throughput and p50/p99."""
    from paper_2212_14191_amd import autotune
    from paper_2212_14191_amd.scheme import Scheme
    from paper_2212_14191_amd.serving import GpuBackend, Server
    L, K, dnum = HM_L, HM_K, HM_DNUM
    log_ns, rots = (13, 14, 15, 16), (1, 2, 4, 8, 16, 32, 64, 128)
    ctxs, evks, rks, pool = {}, {}, {}, {}
    for ln in log_ns:
        n = 1 << ln
        ctx = tfhe.CkksContext(ln, L, K, dnum)
        sch = Scheme(ctx)
        s = inputs.ternary_secret(1, n, 192)
        a = inputs.uniform_residues(1, ctx.moduli, (dnum, n), stream=1).transpose(1, 0, 2)
        e = inputs.gaussian_error(2, (dnum, n), stream=1)
        ctxs[ln], evks[ln] = ctx, sch.relin_key(s, a, e)
        if table is not None:
            autotune.apply_ckks(ctx, table, L, 64, L)
        for r in rots:
            g = pow(5, r, 2 * n)
            rks[(ln, g)] = sch.rotation_key(s, g, a, e)
        full = []
        for i in range(2):
            m = inputs.small_messages(i, (1, n))
            c1 = inputs.uniform_residues(30 + i, ctx.moduli[:L], (1, n), stream=5)
            full.append(sch.encrypt(s, m, c1, inputs.gaussian_error(2, (1, n), stream=40 + i), L))
        for level in range(1, L + 1):  # dropping top limbs keeps a valid ciphertext
            pool[(ln, level)] = [c[:, :level].contiguous() for c in full]
    torch.cuda.synchronize()
    slots, budget = 4, 48 << 30

    # per-N batch limits from the autotuner's HMULT timings at level 24 (the
    # largest batch within batch_ms, else its throughput choice), else 16
    by_n = autotune.serving_batches(table, log_ns, L, batch_ms) if table is not None else {}

    # one long-lived backend: its streams, events and per-slot workspaces stay
    # warm across the runs, as in a running server
    backend = GpuBackend(ctxs, evks, rks, slots=slots)

    def run(count, seed, rate):
        mix = inputs.request_mix(seed, count, log_ns=log_ns, max_level=L, rotations=rots)
        arrivals = inputs.poisson_arrivals(seed, rate, count) if rate else np.zeros(count)
        srv = Server(backend, budget, slots=slots, max_batch=16, max_batch_by_n=by_n)
        futs = []
        t0 = time.perf_counter()
        for i in range(count):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            ln, lv = int(mix["log_n"][i]), int(mix["level"][i])
            c = pool[(ln, lv)]
            if mix["op"][i] == 0:
                futs.append(srv.submit(0, ln, lv, c[0], c[1]))
            else:
                futs.append(srv.submit(1, ln, lv, c[0], galois=pow(5, int(mix["rot"][i]), 2 << ln)))
        for f in futs:
            f.result(timeout=300)
        st = srv.stats()
        srv.close()
        return st

    # the library's own dispatcher (tfhe_server_*), same mix, same keys
    native = tfhe.NativeServer(slots=native_slots, max_batch=16, pool_bytes=native_slots * (3 << 30))
    for ln in log_ns:
        native.add_context(ctxs[ln], evks[ln], {g: k for (l2, g), k in rks.items() if l2 == ln})
        if ln in by_n:
            native.set_max_batch(ln, by_n[ln])

    def run_native(count, seed, rate):
        # The client prepares every request (inputs resident, outputs
        # allocated, the tfhe_server_request array filled) before the clock
        # starts, then submits whatever has arrived in one call and polls,
        # through the C ABI directly: the measured rates are the server's,
        # not the cost of building requests in Python.
        import ctypes
        mix = inputs.request_mix(seed, count, log_ns=log_ns, max_level=L, rotations=rots)
        arrivals = inputs.poisson_arrivals(seed, rate, count) if rate else np.zeros(count)
        arr = (tfhe.ServerRequest * count)()
        outs = []
        for k, (op, ln, lv, rt) in enumerate(zip(*(mix[f].tolist() for f in ("op", "log_n", "level", "rot")))):
            c = pool[(ln, lv)]
            out_t = torch.empty_like(c[0])
            outs.append(out_t)
            r = arr[k]
            r.op, r.log_n, r.level = op, ln, lv
            r.galois_elt = pow(5, rt, 2 << ln) if op == 1 else 0
            r.ct_a, r.ct_b = c[0].data_ptr(), c[1].data_ptr() if op == 0 else 0
            r.ct_out, r.tag = out_t.data_ptr(), k
        torch.cuda.synchronize()
        lib, h, stream = tfhe.load(), native.handle, tfhe._stream(None)
        base, size = ctypes.addressof(arr), ctypes.sizeof(tfhe.ServerRequest)
        cap = 4096
        tags = np.zeros(cap, dtype=np.uint64)
        status = np.zeros(cap, dtype=np.int32)
        tags_p = tags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        status_p = status.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        t_sub, t_done = np.zeros(count), np.full(count, np.nan)
        i, completed = 0, 0
        t0 = time.perf_counter()
        while completed < count:
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arrivals, now, side="right")) if rate else count
            if j > i:
                st = lib.tfhe_server_submit_many(h, ctypes.cast(base + i * size, ctypes.POINTER(tfhe.ServerRequest)),
                                                 j - i, stream, None)
                tfhe.check(st, "tfhe_server_submit_many")
                t_sub[i:j] = time.perf_counter() - t0
                i = j
            k = lib.tfhe_server_poll(h, tags_p, status_p, cap)
            if k:
                if status[:k].any():
                    raise RuntimeError(f"a request failed: {tfhe.status_name(int(status[:k][status[:k] != 0][0]))}")
                t_done[tags[:k].astype(np.int64)] = time.perf_counter() - t0
                completed += k
            if now > 300:
                raise RuntimeError("native serving run did not finish")
        del outs
        lat = t_done - t_sub
        by_n = {str(ln): round(float(np.percentile(lat[mix["log_n"] == ln], 99) * 1e3), 3)
                for ln in log_ns if (mix["log_n"] == ln).any()}
        return {"throughput_per_s": count / (np.max(t_done) - t_sub[0]),
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "p99_ms_by_log_n": by_n}

    out = {"requests": n_req, "max_batch": 16, "max_batch_by_n": {str(k): v for k, v in by_n.items()},
           "batch_ms": batch_ms, "p99_bound_ms": P99_BOUND_MS}
    for name, fn in (("python", run), ("native", run_native)):
        if name not in engines:
            continue
        fn(min(500, n_sat), 99, 0)  # warm-up
        sat = fn(n_sat, 98, 0)
        res = {"slots": native_slots if name == "native" else slots,
               "saturated_ops_per_s": round(sat["throughput_per_s"], 1), "runs": []}
        for frac in fracs:
            rate = frac * sat["throughput_per_s"]
            st = fn(n_req, 3, rate)
            rec = {"load": frac, "rate_per_s": round(rate, 1), "throughput_per_s": round(st["throughput_per_s"], 1),
                   "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3)}
            if "p99_ms_by_log_n" in st:
                rec["p99_ms_by_log_n"] = st["p99_ms_by_log_n"]
            res["runs"].append(rec)
        res["sustainable"] = sustainable_rate(fn, sat["throughput_per_s"], n_req)
        out[name] = res
    native.close()
    return out


def onepass_leg(args, torch, tfhe, inputs, sync, log_n=14, limbs=24, batch=64):
    """Profiling leg: forward + inverse on the one-pass kernel (each
    polynomial crosses HBM once per transform) at one serving shape; the
    algorithmic bytes of a launch are one read and one write of every
    residue."""
    n = 1 << log_n
    qs = tfhe.tfhe_find_primes(31, 1 << 17, limbs)
    plan = tfhe.NttPlan(log_n, qs)
    plan.set_param("fs_passes", 1)
    x = torch.from_numpy(inputs.uniform_residues(0, qs, (batch, n)).view(np.int32)).cuda()
    y, z = torch.empty_like(x), torch.empty_like(x)
    ws = plan.workspace(limbs, batch, "mfma")

    def step():
        plan.fwd(x, out=y, algo="mfma", ws=ws)
        plan.inv(y, out=z, algo="mfma", ws=ws)
    for _ in range(args.warmup):
        step()
    sync()
    assert torch.equal(z, x), "one-pass INTT(NTT(x)) != x"
    tfhe.tfhe_timing_enable(True)
    dt = timed(step, args.steps, sync)
    cnt, ms = tfhe.tfhe_timing_read("ntt_mfma_onepass")
    tfhe.tfhe_timing_enable(False)
    units = limbs * batch
    per_launch = ms / max(cnt, 1)
    nbytes = 2 * units * n * 4
    return {"log_n": log_n, "limbs": limbs, "batch": batch, "kops": 2 * units * args.steps / dt / 1e3,
            "launches": cnt, "avg_launch_ms": round(per_launch, 4), "algorithmic_bytes_per_launch": nbytes,
            "achieved_gbs": round(nbytes / (per_launch * 1e-3) / 1e9, 1)}


# 16 requests at 16 different levels (mean 12.5) against 16 at level 12
MIXED_LEVELS = (2, 3, 5, 6, 8, 9, 11, 12, 13, 14, 16, 17, 19, 20, 22, 23)


def levels_leg(args, torch, tfhe, inputs, sync, log_ns=(16, 14), L=24, K=8, dnum=3):
    """Profiling leg: one HMULT batch of 16 requests at 16 different levels
    (one request per level group, as the serving mix forms them) against a
    batch of 16 at one level, at the serving shapes (tfhe_hmult_levels;
    the key switch's launches are shared by every group either way)."""
    out = {}
    for ln in log_ns:
        n = 1 << ln
        ctx = tfhe.CkksContext(ln, L, K, dnum)
        ev = inputs.uniform_residues(ln, ctx.moduli, (dnum, 2, n)).transpose(1, 2, 0, 3)
        evk = torch.from_numpy(np.ascontiguousarray(ev).view(np.int32)).cuda()
        res = {}
        for name, levels in (("single_level", (12,) * 16), ("mixed_levels", MIXED_LEVELS)):
            def ct(seed, lv):
                c = inputs.uniform_residues(seed, ctx.moduli[:lv], (2, n)).transpose(1, 0, 2)
                return torch.from_numpy(np.ascontiguousarray(c).view(np.int32)).cuda()
            A = [ct(2 * k, lv) for k, lv in enumerate(levels)]
            B = [ct(2 * k + 1, lv) for k, lv in enumerate(levels)]
            outs = [torch.empty_like(a) for a in A]
            ws = ctx.levels_workspace(list(levels))

            def step():
                ctx.hmult_levels(A, B, evk, outs=outs, ws=ws)
            for _ in range(args.warmup):
                step()
            sync()
            k = len(levels) - 1
            one = ctx.hmult(A[k][:, :, None], B[k][:, :, None], evk, levels[k])  # [2][level][1][N]
            assert torch.equal(outs[k], one[:, :, 0]), "batched HMULT != single call"
            dt = timed(step, args.steps, sync)
            res[name] = {"levels": list(levels), "ms_per_batch": round(dt / args.steps * 1e3, 4)}
        res["mixed_over_single"] = round(res["mixed_levels"]["ms_per_batch"] / res["single_level"]["ms_per_batch"], 3)
        out[str(ln)] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed steps per leg (the clocks ramp up over the first tens of ms)")
    ap.add_argument("--hmult-steps", type=int, default=20)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-hmult", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--serving-engine", choices=["both", "python", "native"], default="both")
    ap.add_argument("--serving-batch-ms", type=float, default=P99_BOUND_MS / 4,
                    help="cap each N's serving batch at the largest whose measured HMULT time fits (0: no cap)")
    ap.add_argument("--native-slots", type=int, default=8,
                    help="worker threads (one stream each) of the native dispatcher")
    ap.add_argument("--only", choices=["mfma", "butterfly", "co", "hmult", "serving", "onepass", "levels"], default=None,
                    help="time one leg only (for profiling runs; onepass: the one-HBM-round-trip "
                         "transform at N = 2^14, 24 limbs x 64 polynomials, the serving shape; levels: "
                         "an HMULT batch of 16 levels against one of a single level, N = 2^16 and 2^14)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain device copy of the input batch (a known-size "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the NTT/HMULT "
              "path shards by ciphertext with no collective between GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_14191_amd import inputs, tfhe
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    if args.only == "onepass":
        print(json.dumps({"onepass": onepass_leg(args, torch, tfhe, inputs, sync)}), flush=True)
        return
    if args.only == "levels":
        print(json.dumps({"levels": levels_leg(args, torch, tfhe, inputs, sync)}), flush=True)
        return
    n = 1 << LOG_N

    qs = tfhe.tfhe_find_primes(31, 1 << 17, LIMBS)
    t_setup = time.perf_counter()
    plan = tfhe.NttPlan(LOG_N, qs)  # host-side tables for 44 primes, uploaded once (synchronous)
    setup = {"ntt_plan_s": round(time.perf_counter() - t_setup, 3)}
    units = LIMBS * BATCH
    results = {}
    algos = (["mfma", "butterfly", "co"] if args.only is None else
             [] if args.only in ("hmult", "serving") else [args.only])
    x = y = z = ws = None
    if algos:
        log(f"generating {LIMBS}x{BATCH}x{n} uniform residues")
        x_host = inputs.uniform_residues(0, qs, (BATCH, n))
        x = torch.from_numpy(x_host.view(np.int32)).cuda()
        del x_host
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        ws = plan.workspace(LIMBS, BATCH, "mfma")
        if args.copy_calib:
            y.copy_(x)
            sync()
    # measured bandwidth ceiling: a plain device copy of the same batch
    # (reads and writes the algorithmic bytes of one pass launch)
    copy_gbs = None
    if algos:
        for _ in range(args.warmup):
            y.copy_(x)
        copy_gbs = 2 * x.numel() * 4 * 10 / timed(lambda: y.copy_(x), 10, sync) / 1e9
    # the autotuner's persisted choices (written on the GPU by
    # `python -m paper_2212_14191_amd.autotune`); absent entries keep the
    # library defaults
    from paper_2212_14191_amd import autotune
    table = autotune.load_default()
    tuning = {"table": os.path.relpath(autotune.TABLE_PATH, ROOT) if table.entries else None}
    for algo in algos:
        if algo == "mfma":
            tuning["ntt"] = autotune.apply(plan, table, LIMBS, BATCH)
        else:
            for name in autotune.PLAN_PARAMS:
                plan.set_param(name, 0)

        def step(algo=algo):
            plan.fwd(x, out=y, algo=algo, ws=ws)
            plan.inv(y, out=z, algo=algo, ws=ws)
        for _ in range(args.warmup):
            step()
        sync()
        assert torch.equal(z, x), f"{algo}: INTT(NTT(x)) != x"
        steps = args.steps if algo == "mfma" else max(3, args.steps // 2)
        tfhe.tfhe_timing_enable(True)
        dt = timed(step, steps, sync)
        kern = {}
        names = {"mfma": ("ntt_mfma_pass1", "ntt_mfma_pass2"), "co": ("ntt_co_pass1", "ntt_co_pass2"),
                 "butterfly": ("ntt_bf_cols", "ntt_bf_rows")}[algo]
        for name in names:
            cnt, ms = tfhe.tfhe_timing_read(name)
            kern[name] = {"launches": cnt, "avg_ms": ms / max(cnt, 1)}
        tfhe.tfhe_timing_enable(False)
        # untimed check of forward output: both algorithms must agree bit for bit
        results[algo] = {"kops": 2 * units * steps / dt / 1e3, "ms_per_step": 1e3 * dt / steps,
                         "steps": steps, "kernels": kern}
        log(algo, json.dumps(results[algo]))
    if args.only is None:
        ym = torch.empty_like(x)
        plan.fwd(x, out=ym, algo="mfma", ws=ws)
        plan.fwd(x, out=y, algo="butterfly", ws=ws)
        sync()
        assert torch.equal(ym, y), "MFMA and butterfly forward outputs differ"
        del ym
    del y, z, ws

    hmult = None
    if not args.skip_hmult and args.only in (None, "hmult"):
        from paper_2212_14191_amd.scheme import Scheme
        t_setup = time.perf_counter()
        ctx = tfhe.CkksContext(LOG_N, HM_L, HM_K, HM_DNUM)
        setup["ckks_context_s"] = round(time.perf_counter() - t_setup, 3)
        tuning["hmult_ntt"] = autotune.apply_ckks(ctx, table, HM_L, HM_BATCH, HM_L)
        sch = Scheme(ctx)
        s = inputs.ternary_secret(1, n, 192)
        a = inputs.uniform_residues(1, ctx.moduli, (HM_DNUM, n), stream=1).transpose(1, 0, 2)
        e = inputs.gaussian_error(2, (HM_DNUM, n), stream=1)
        evk = sch.relin_key(s, a, e)
        level = HM_L
        qsl = ctx.moduli[:level]
        cts = []
        for k in range(2):
            m = inputs.small_messages(0, (HM_BATCH, n), stream=k)
            c1 = inputs.uniform_residues(10 + k, qsl, (HM_BATCH, n), stream=5)
            ee = inputs.gaussian_error(2, (HM_BATCH, n), stream=20 + k)
            cts.append(sch.encrypt(s, m, c1, ee, level))
        out = torch.empty_like(cts[0])
        hws = ctx.workspace(level, HM_BATCH)
        hstep = lambda: ctx.hmult(cts[0], cts[1], evk, level, out=out, ws=hws)
        for _ in range(max(2, args.warmup)):
            hstep()
        tfhe.tfhe_timing_enable(True)
        dt = timed(hstep, args.hmult_steps, sync)
        kern = {}
        for name in ("ntt_mfma_pass1", "ntt_mfma_pass2", "ntt_mfma_pass2_inner", "ckks_tensor", "ckks_modup",
                     "ckks_inner", "ckks_moddown_conv", "ckks_moddown_final"):
            cnt, ms = tfhe.tfhe_timing_read(name)
            kern[name] = {"launches": cnt, "total_ms": ms}
        tfhe.tfhe_timing_enable(False)
        hmult = {"ops_per_s": HM_BATCH * args.hmult_steps / dt, "ms_per_batch": 1e3 * dt / args.hmult_steps,
                 "batch": HM_BATCH, "level": level, "kernels": kern}
        hmult["roofline"] = hmult_roofline(hmult["ops_per_s"], n, HM_L, HM_K, HM_DNUM, HM_BATCH)
        log("hmult", json.dumps(hmult))
        # RESCALE of the HMULT results (level 24 -> 23), same batch
        rs_out = torch.empty((2, level - 1, HM_BATCH, n), dtype=torch.int32, device="cuda")
        rws = ctx.rescale_workspace(level, HM_BATCH)
        rstep = lambda: ctx.rescale(out, level, out=rs_out, ws=rws)
        for _ in range(max(1, args.warmup)):
            rstep()
        tfhe.tfhe_timing_enable(True)
        dt = timed(rstep, args.hmult_steps, sync)
        rk = {}
        for name in ("ntt_mfma_pass1", "ntt_mfma_pass2", "ckks_rescale_bcast", "ckks_rescale_final"):
            cnt, ms = tfhe.tfhe_timing_read(name)
            rk[name] = {"launches": cnt, "total_ms": ms}
        tfhe.tfhe_timing_enable(False)
        hmult["rescale"] = {"ops_per_s": HM_BATCH * args.hmult_steps / dt,
                            "ms_per_batch": 1e3 * dt / args.hmult_steps, "kernels": rk}
        log("rescale", json.dumps(hmult["rescale"]))
        # CMULT (plaintext = the first ciphertext's c0, in the NTT domain) and
        # HADD at the same shape: element-wise, HBM-bound; algorithmic bytes:
        # CMULT reads the ciphertext and the plaintext once and writes the
        # result (2.5 ciphertexts), HADD reads two and writes one (3)
        pt = cts[0][0].contiguous()
        ew_out = torch.empty_like(out)
        ct_bytes = cts[0].numel() * 4
        for name, fn, nbytes in (("cmult", lambda: ctx.cmult(cts[0], pt, level, out=ew_out), 2.5 * ct_bytes),
                                 ("hadd", lambda: ctx.hadd(cts[0], cts[1], level, out=ew_out), 3 * ct_bytes)):
            for _ in range(max(1, args.warmup)):
                fn()
            dt = timed(fn, args.hmult_steps, sync)
            hmult[name] = {"ops_per_s": HM_BATCH * args.hmult_steps / dt,
                           "gb_per_s": nbytes * args.hmult_steps / dt / 1e9}
            log(name, json.dumps(hmult[name]))
        del cts, out, hws, evk, ctx, rs_out, rws, pt, ew_out
        if args.only is None:
            # the serving mix's batches hold one request per level group:
            # such a batch against one of a single level (same size)
            hmult["levels"] = levels_leg(argparse.Namespace(steps=min(args.steps, 20), warmup=min(args.warmup, 5)),
                                         torch, tfhe, inputs, sync)
            log("levels", json.dumps({k: v["mixed_over_single"] for k, v in hmult["levels"].items()}))

    serving = None
    if not args.skip_serving and args.only in (None, "serving"):
        engines = ("python", "native") if args.serving_engine == "both" else (args.serving_engine,)
        serving = serving_leg(args.serving_requests, args.serving_requests, (0.25, 0.5, 0.75, 0.9), torch, tfhe,
                              inputs, engines, args.native_slots, table,
                              args.serving_batch_ms if args.serving_batch_ms > 0 else None)
        tuning["serving_max_batch"] = serving.get("max_batch_by_n")
        log("serving", json.dumps(serving))

    cpu = None
    if not args.skip_cpu and args.only is None:
        cpu = cpu_baseline(qs, plan.psi)
        log("cpu", json.dumps(cpu))

    head = results.get("mfma") or results.get("butterfly") or results.get("co")
    if head is None:  # --only hmult / serving (profiling runs)
        print(json.dumps({"hmult": hmult, "serving": serving}), flush=True)
        return
    kname, kstat = max(head["kernels"].items(), key=lambda kv: kv[1]["avg_ms"] * kv[1]["launches"])
    bytes_per_launch = 2 * units * n * 4  # one read and one write of every residue
    achieved = bytes_per_launch / (kstat["avg_ms"] * 1e-3) / 1e9
    mfma_line = None
    if "mfma" in results:
        # the same launch against the int8 matrix-core peak (the kernel is
        # HBM-bound; this is the second roofline, its matrix-core share)
        ops = units * n * I8_OPS_PER_COEFF_PASS
        tops = ops / (kstat["avg_ms"] * 1e-3) / 1e12
        mfma_line = {"kernel": kname, "bound": "hbm", "achieved": round(tops, 1), "peak": MFMA_I8_PEAK_TOPS,
                     "unit": "TOPS (int8)", "frac": round(tops / MFMA_I8_PEAK_TOPS, 4),
                     "algorithmic_ops_per_launch": ops, "counters": measured_mfma(kname)}
    line = {
        "metric": METRIC,
        "value": round(head["kops"], 1),
        "unit": "KOPS (10^3 limb-NTT/INTT per s, N=2^16)",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "negacyclic NTT+INTT, N=2^16, 44 limbs x 128 polys, " +
                   ("four-step INT8 MFMA" if "mfma" in results else
                    "butterfly" if "butterfly" in results else "four-step vector-ALU GEMM"),
                   "log_n": LOG_N, "limbs": LIMBS, "batch": BATCH, "primes": "31-bit, q = 1 mod 2^17"},
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kname) if "mfma" in results else None,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": round(kstat["avg_ms"], 4),
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "roofline_mfma": mfma_line,
        "tuning": tuning,
        "cpu_baseline": cpu,
    }
    if "butterfly" in results and "mfma" in results:
        line["butterfly_kops"] = round(results["butterfly"]["kops"], 1)
        line["mfma_over_butterfly"] = round(results["mfma"]["kops"] / results["butterfly"]["kops"], 3)
    if "co" in results:
        line["valu_gemm_kops"] = round(results["co"]["kops"], 1)
    line["kernels"] = {k: v for r in results.values() for k, v in r["kernels"].items()}
    if hmult:
        line["hmult_ops_per_s"] = round(hmult["ops_per_s"], 1)
        line["rescale_ops_per_s"] = round(hmult["rescale"]["ops_per_s"], 1)
        line["cmult_ops_per_s"] = round(hmult["cmult"]["ops_per_s"], 1)
        line["hadd_ops_per_s"] = round(hmult["hadd"]["ops_per_s"], 1)
        line["hmult"] = hmult
    if serving:
        if "native" in serving:
            line["p99_ms"] = next(r["p99_ms"] for r in serving["native"]["runs"] if r["load"] == 0.5)
            line["sustainable_requests_per_s"] = serving["native"]["sustainable"]["rate_per_s"]
        line["serving"] = serving
    line["setup"] = setup  # plan and context creation (host tables + upload), outside every timed region
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
