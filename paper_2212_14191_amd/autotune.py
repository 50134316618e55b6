"""Self-written autotuner (the API layer "generates the best batch size for
the different involved kernels according to the hardware resources",
Sec. IV-E; the best batch differs per kernel, Sec. VI).

* NTT: for a (log N, limbs, batch) shape, times forward + inverse for each
  candidate (algorithm x 256-point item width x persistent four-step
  workgroups per CU) and keeps the fastest.
* HMULT: sweeps the batch size at a (log N, level) and keeps the smallest
  batch within `slack` of the best throughput (small batches keep latency
  low in the serving loop).
Results persist as JSON; `apply` writes the NTT choice into a plan.
"""
import json
import os
import time

NTT_WG_CANDIDATES = (0, 1, 2, 3, 4, 6, 8)
NTT_WIDE_CANDIDATES = (1, 2)   # narrow / wide 256-point items (0 = library default)


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


def apply(plan, table, limbs, batch):
    """Set a plan's tuned parameters for this shape, if the table has them."""
    e = table.get(ntt_key(plan.log_n, limbs, batch))
    if not e:
        return False
    plan.set_param("auto_algo", {"butterfly": 1, "mfma": 2}[e["algo"]])
    plan.set_param("fs_wg_per_cu", e.get("fs_wg_per_cu", 0))
    plan.set_param("fs_wide", e.get("fs_wide", 0))
    return True


def tune_ntt(plan, x, reps=5, warmup=1):
    """x: int32 [limbs][batch][N] on the device.  Returns (best, all)."""
    import torch
    from . import tfhe
    limbs, batch, _ = x.shape
    y, z = torch.empty_like(x), torch.empty_like(x)
    cands = [("butterfly", 0, 0)]
    if plan.get_param("auto_algo") == tfhe.FOURSTEP_MFMA or _has_mfma(plan):
        cands += [("mfma", wide, w) for wide in NTT_WIDE_CANDIDATES for w in NTT_WG_CANDIDATES]
    ws = plan.workspace(limbs, batch, "mfma" if len(cands) > 1 else "butterfly")
    results = []
    old = (plan.get_param("fs_wg_per_cu"), plan.get_param("fs_wide"))
    for algo, wide, w in cands:
        plan.set_param("fs_wg_per_cu", w)
        plan.set_param("fs_wide", wide)
        for _ in range(warmup):
            plan.fwd(x, out=y, algo=algo, ws=ws)
            plan.inv(y, out=z, algo=algo, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.fwd(x, out=y, algo=algo, ws=ws)
            plan.inv(y, out=z, algo=algo, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if not torch.equal(z, x):
            raise RuntimeError(f"autotune: {algo}/{wide}/{w} failed the round trip")
        results.append(({"algo": algo, "fs_wide": wide, "fs_wg_per_cu": w}, 2 * limbs * batch * reps / dt / 1e3))
    plan.set_param("fs_wg_per_cu", old[0])
    plan.set_param("fs_wide", old[1])
    cfg, kops = pick_best(results)
    best = dict(cfg, kops=kops)
    return best, [dict(c, kops=k) for c, k in results]


def _has_mfma(plan):
    try:
        plan.workspace_bytes(1, 1, "mfma")
        return True
    except Exception:
        return False


def tune_hmult_batch(ctx, make_inputs, level, batches=(1, 2, 4, 8, 16, 32, 64), reps=3, slack=0.05):
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
