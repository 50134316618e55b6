"""Self-written autotuner (the API layer "generates the best batch size for
the different involved kernels according to the hardware resources",
Sec. IV-E; the best batch differs per kernel, Sec. VI-E).

* NTT: for a (log N, limbs, batch) shape, times forward + inverse for each
  candidate (algorithm x HBM round trips of the four-step transform, one or
  two x 256-point item width x persistent four-step workgroups per CU),
  re-times the fastest few against the library default in interleaved
  rounds and keeps the best (its entry records the default's rate beside
  its own).  Every candidate's round trip must be the identity.
* HMULT: sweeps the batch size at a (log N, level) and keeps the smallest
  batch within `slack` of the best throughput (small batches keep latency
  low in the serving loop).

Results persist as JSON (TuneTable).  `apply` writes a tuned NTT choice into
a plan; `serving_batches` turns the HMULT entries into per-N batch limits
for both serving engines (Server(max_batch_by_n=...),
NativeServer.set_max_batch).  The table shipped with the package
(TABLE_PATH) is written on the GPU by

    python -m paper_2212_14191_amd.autotune --out paper_2212_14191_amd/tune_mi355x.json

Knobs the search does not cover: the LDS ring depth of the two-pass kernel
(a compile-time constant) and the N1 x 256 split itself (fixed by the
operand tables; the one-pass kernel is the structural alternative).
"""
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tune_mi355x.json")

NTT_WG_CANDIDATES = (0, 1, 2, 3, 4, 6, 8)
NTT_WIDE_CANDIDATES = (1, 2)   # narrow / wide 256-point items (0 = library default)
NTT_RING_CANDIDATES = (2, 3)   # LDS ring stages of the wide-item passes
HMULT_BATCHES = (1, 2, 4, 8, 16, 32, 64)


def ntt_key(log_n, limbs, batch):
    return f"ntt:{log_n}:{limbs}:{batch}"


def hmult_key(log_n, level):
    return f"hmult:{log_n}:{level}"


def pick_best(results, higher_is_better=True):
    """results: list of (config dict, score).  Returns the best pair."""
    key = (lambda r: r[1]) if higher_is_better else (lambda r: -r[1])
    return max(results, key=key)


def pick_batch(throughput_by_batch, slack=0.05):
    """Smallest batch whose throughput is within `slack` of the maximum."""
    best = max(throughput_by_batch.values())
    for b in sorted(throughput_by_batch):
        if throughput_by_batch[b] >= (1.0 - slack) * best:
            return b
    return max(throughput_by_batch)


class TuneTable:
    def __init__(self, path=None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key):
        return self.entries.get(key)

    def put(self, key, value):
        self.entries[key] = value

    def save(self, path=None):
        path = path or self.path
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def load_default():
    """The table shipped with the package (empty when absent)."""
    return TuneTable(TABLE_PATH)


PLAN_PARAMS = ("fs_passes", "fs_wide", "fs_wg_per_cu", "fs_ring")


def apply(plan, table, limbs, batch):
    """Set a plan's tuned parameters for this shape, if the table has them.
    Returns the applied entry (or None)."""
    e = table.get(ntt_key(plan.log_n, limbs, batch))
    if not e:
        return None
    plan.set_param("auto_algo", {"butterfly": 1, "mfma": 2}[e["algo"]])
    for name in PLAN_PARAMS:
        plan.set_param(name, e.get(name, 0))
    return e


KS_INNER_MARGIN = 1.02


def ks_inner_choice(entry):
    """The key-switching variant an HMULT entry selects: the fused inner
    product (1, the library default, with less HBM traffic) unless the
    separate kernels (2) measured more than KS_INNER_MARGIN faster (the two
    are within a few per cent of each other at N >= 2^15, so a smaller
    difference is taken as noise)."""
    ops = entry.get("ks_inner_ops_per_s")
    if ops and "1" in ops and "2" in ops:
        return 2 if ops["2"] > KS_INNER_MARGIN * ops["1"] else 1
    return int(entry["ks_inner"]) if "ks_inner" in entry else None


def apply_ckks(ctx, table, limbs=24, batch=64, level=24):
    """Tuned plan parameters of a CKKS context's transforms and its key
    switching variant (the inner product fused into the transforms or not).
    A one-pass choice becomes the library default (fs_passes 0) here: the
    key switch's plain transforms (the INTT of d2 and of the special limbs)
    then take one pass for launches with at least two polynomials per CU,
    which measured 2-8 % faster HMULT at N = 2^12..2^14 and batch 8-64,
    and two below, where one pass would leave CUs idle (10-20 % slower at
    batch 1-4).  The persistent grid stays the library's (fs_wg_per_cu 0):
    the transform-tuned 4 workgroups per CU measured 0.6-2.4 % slower for
    HMULT at N = 2^15 and 2^16 (levels 12 and 24), whose many launches of
    other shapes balance better on the resident-count grid.  Returns the
    applied entries."""
    e = apply(ctx.plan, table, limbs, batch)
    if e is not None:
        e = dict(e)  # the parameters as applied to this context
        if e.get("fs_passes") == 1:
            e["fs_passes"] = 0
        e["fs_wg_per_cu"] = 0
        for name in ("fs_passes", "fs_wg_per_cu"):
            ctx.plan.set_param(name, e[name])
    h = table.get(hmult_key(ctx.log_n, level))
    choice = ks_inner_choice(h) if h else None
    if choice is not None:
        ctx.plan.set_param("ks_inner", choice)
    return {"ntt": e, "ks_inner": choice}


def serving_batches(table, log_ns, level, batch_ms=None):
    """{log_n: HMULT batch limit at `level`} for the N the table covers: the
    tuned (throughput) batch, or with `batch_ms` the largest measured batch
    whose time (batch / measured ops per second) stays within batch_ms, when
    that is smaller (a request waits for at most about one batch ahead of it
    and its own, so this bounds the latency a batch adds)."""
    out = {}
    for ln in log_ns:
        e = table.get(hmult_key(ln, level))
        if not e or "batch" not in e:
            continue
        b = int(e["batch"])
        if batch_ms is not None and e.get("ops_per_s"):
            fit = [int(k) for k, v in e["ops_per_s"].items() if v > 0 and int(k) / v * 1e3 <= batch_ms]
            b = min(b, max(fit)) if fit else 1
        out[ln] = b
    return out


def ntt_candidates(log_n, mfma):
    """(algo, fs_passes, fs_wide, fs_wg_per_cu, fs_ring) tuples to time: the
    LDS ring depth is searched where the 256-point stage takes wide items
    (fs_wide 2 at N >= 2^13); narrow items have one depth."""
    cands = [("butterfly", 0, 0, 0, 0)]
    if mfma:
        for wide in NTT_WIDE_CANDIDATES:
            rings = NTT_RING_CANDIDATES if wide == 2 and log_n >= 13 else (0,)
            cands += [("mfma", 2, wide, w, ring) for w in NTT_WG_CANDIDATES for ring in rings]
        if 12 <= log_n <= 15:
            cands += [("mfma", 1, 0, 0, 0)]
    return cands


def _time_candidate(plan, cand, x, y, z, ws, reps, trials):
    """Median over `trials` of the forward + inverse time of `reps` rounds
    (seconds per round), with the candidate's parameters set; checks that
    the round trip is the identity."""
    import statistics
    import torch
    algo, passes, wide, w, ring = cand
    plan.set_param("fs_passes", passes)
    plan.set_param("fs_wide", wide)
    plan.set_param("fs_wg_per_cu", w)
    plan.set_param("fs_ring", ring)
    for _ in range(2):
        plan.fwd(x, out=y, algo=algo, ws=ws)
        plan.inv(y, out=z, algo=algo, ws=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(trials):
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.fwd(x, out=y, algo=algo, ws=ws)
            plan.inv(y, out=z, algo=algo, ws=ws)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) / reps)
    if not torch.equal(z, x):
        raise RuntimeError(f"autotune: {algo}/{passes}/{wide}/{w}/{ring} failed the round trip")
    return statistics.median(times)


def tune_ntt(plan, x, reps=5, trials=3, finalists=3, rounds=3):
    """x: int32 [limbs][batch][N] on the device.  Every candidate is timed
    (median of `trials`); the best `finalists` and the library default are
    then timed again in `rounds` interleaved rounds (so that clock and
    thermal drift hit them alike) and the best median wins.  Returns (best,
    all)."""
    import statistics
    import torch
    from . import tfhe
    limbs, batch, _ = x.shape
    y, z = torch.empty_like(x), torch.empty_like(x)
    mfma = plan.get_param("auto_algo") == tfhe.FOURSTEP_MFMA or _has_mfma(plan)
    cands = ntt_candidates(plan.log_n, mfma)
    ws = plan.workspace(limbs, batch, "mfma" if mfma else "butterfly")
    old = {name: plan.get_param(name) for name in PLAN_PARAMS}
    first = [(c, _time_candidate(plan, c, x, y, z, ws, reps, trials)) for c in cands]
    default = ("mfma", 0, 0, 0, 0) if mfma else ("butterfly", 0, 0, 0, 0)
    top = [c for c, _ in sorted(first, key=lambda r: r[1])[:finalists]]
    if default not in top:
        top.append(default)
    final = {c: [] for c in top}
    for _ in range(rounds):
        for c in top:
            final[c].append(_time_candidate(plan, c, x, y, z, ws, reps, 1))
    for name, v in old.items():
        plan.set_param(name, v)
    units = 2 * limbs * batch
    kops = lambda t: units / t / 1e3
    scored = {c: statistics.median(ts) for c, ts in final.items()}
    best_c = min(scored, key=scored.get)
    as_cfg = lambda c: {"algo": c[0], "fs_passes": c[1], "fs_wide": c[2], "fs_wg_per_cu": c[3], "fs_ring": c[4]}
    best = dict(as_cfg(best_c), kops=kops(scored[best_c]), default_kops=kops(scored[default]))
    return best, [dict(as_cfg(c), kops=kops(t)) for c, t in first]


def _has_mfma(plan):
    try:
        plan.workspace_bytes(1, 1, "mfma")
        return True
    except Exception:
        return False


def tune_hmult_batch(ctx, make_inputs, level, batches=HMULT_BATCHES, reps=3, slack=0.05):
    """make_inputs(batch) -> (ct_a, ct_b, evk) on the device.  Returns
    (chosen batch, {batch: HMULT/s})."""
    import torch
    tput = {}
    for b in batches:
        a, bb, evk = make_inputs(b)
        out = torch.empty_like(a)
        ws = ctx.workspace(level, b)
        ctx.hmult(a, bb, evk, level, out=out, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.hmult(a, bb, evk, level, out=out, ws=ws)
        torch.cuda.synchronize()
        tput[b] = b * reps / (time.perf_counter() - t0)
        del a, bb, out, ws
    return pick_batch(tput, slack), tput


def _random_residues(torch, moduli, batch, n):
    """Uniform residues [len(moduli)][batch][n] drawn on the device (tuning
    inputs: timing does not depend on the values)."""
    t = torch.empty((len(moduli), batch, n), dtype=torch.int64, device="cuda")
    for l, q in enumerate(moduli):
        t[l].random_(0, q)
    return t.to(torch.int32)


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the NTT plans and HMULT batch sizes on this GPU")
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    import torch
    from . import tfhe
    tfhe.load()
    torch.cuda.set_device(0)
    table = TuneTable()
    table.put("device", {"name": torch.cuda.get_device_name(0),
                         "cus": torch.cuda.get_device_properties(0).multi_processor_count})
    # NTT shapes: the transform benchmark (44 limbs x 128) and the serving
    # shapes (24 limbs x 64) at every N of the four-step range
    shapes = [(16, 44, 128)] + [(ln, 24, 64) for ln in (12, 13, 14, 15, 16)]
    for ln, limbs, batch in shapes:
        qs = tfhe.tfhe_find_primes(31, 1 << 17, limbs)
        plan = tfhe.NttPlan(ln, qs)
        x = _random_residues(torch, qs, batch, 1 << ln)
        best, allr = tune_ntt(plan, x, reps=args.reps)
        table.put(ntt_key(ln, limbs, batch), best)
        print("ntt", ln, limbs, batch, json.dumps(best), flush=True)
        del x, plan
    # HMULT batch per N at the serving shapes (L = 24, K = 8, dnum = 3),
    # level 24 and a middle level
    for ln in (13, 14, 15, 16):
        ctx = tfhe.CkksContext(ln, 24, 8, 3)
        n = 1 << ln
        evk = torch.cat([_random_residues(torch, ctx.moduli, 2, n).permute(1, 0, 2).reshape(1, 2, 32, n)
                         for _ in range(3)])
        for level in (24, 12):
            def make(b, level=level):
                qs = ctx.moduli[:level]
                a = torch.stack([_random_residues(torch, qs, b, n) for _ in range(2)])
                c = torch.stack([_random_residues(torch, qs, b, n) for _ in range(2)])
                return a, c, evk.contiguous()
            b, tput = tune_hmult_batch(ctx, make, level)
            entry = {"batch": b, "ops_per_s": {str(k): round(v, 1) for k, v in tput.items()}}
            # key-switching variant at the chosen batch: separate inner
            # product (2) or fused into the transforms (1), interleaved rounds
            inner = {}
            for _ in range(3):
                for mode in (2, 1):
                    ctx.plan.set_param("ks_inner", mode)
                    _, t = tune_hmult_batch(ctx, make, level, batches=(b,))
                    inner.setdefault(mode, []).append(t[b])
            ctx.plan.set_param("ks_inner", 0)
            med = {m: sorted(v)[1] for m, v in inner.items()}
            entry["ks_inner_ops_per_s"] = {str(m): round(v, 1) for m, v in med.items()}
            entry["ks_inner"] = ks_inner_choice(entry)
            table.put(hmult_key(ln, level), entry)
            print("hmult", ln, level, b, entry["ks_inner"], flush=True)
        ctx.close()
    table.save(args.out)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
