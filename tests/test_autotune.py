"""Autotuner: selection logic, persistence and application (CPU, with a
stand-in plan), and on the GPU a tuning run whose chosen plan is checked
against the oracle, plus an HMULT batch sweep whose chosen batch gives the
oracle's results."""
import numpy as np
import pytest

from paper_2212_14191_amd import autotune


def test_pick_best_and_batch():
    res = [({"a": 1}, 3.0), ({"a": 2}, 5.0), ({"a": 3}, 4.0)]
    assert autotune.pick_best(res)[0] == {"a": 2}
    assert autotune.pick_best(res, higher_is_better=False)[0] == {"a": 1}
    tp = {1: 100.0, 2: 180.0, 4: 300.0, 8: 320.0, 16: 330.0}
    assert autotune.pick_batch(tp, slack=0.05) == 8
    assert autotune.pick_batch(tp, slack=0.5) == 2
    assert autotune.pick_batch({4: 1.0}) == 4


def test_table_roundtrip(tmp_path):
    p = str(tmp_path / "tune.json")
    t = autotune.TuneTable(p)
    t.put(autotune.ntt_key(16, 44, 128), {"algo": "mfma", "fs_wg_per_cu": 3, "kops": 1.0})
    t.put(autotune.hmult_key(16, 24), {"batch": 16})
    t.save()
    t2 = autotune.TuneTable(p)
    assert t2.get("ntt:16:44:128")["fs_wg_per_cu"] == 3
    assert t2.get("hmult:16:24") == {"batch": 16}
    assert t2.get("missing") is None


class FakePlan:
    def __init__(self, log_n):
        self.log_n = log_n
        self.params = {}

    def set_param(self, name, value):
        self.params[name] = value


def test_apply_and_serving_batches():
    t = autotune.TuneTable()
    t.put(autotune.ntt_key(14, 24, 64), {"algo": "mfma", "fs_passes": 1, "fs_wide": 0, "fs_wg_per_cu": 0})
    t.put(autotune.hmult_key(14, 24), {"batch": 8})
    t.put(autotune.hmult_key(16, 24), {"batch": 32})
    plan = FakePlan(14)
    e = autotune.apply(plan, t, 24, 64)
    assert e["fs_passes"] == 1
    assert plan.params == {"auto_algo": 2, "fs_passes": 1, "fs_wide": 0, "fs_wg_per_cu": 0, "fs_ring": 0}
    assert autotune.apply(FakePlan(15), t, 24, 64) is None
    assert autotune.serving_batches(t, (13, 14, 15, 16), 24) == {14: 8, 16: 32}
    # with a time budget per batch: the largest measured batch that fits
    t.put(autotune.hmult_key(16, 24), {"batch": 32, "ops_per_s": {"8": 12000.0, "16": 13600.0, "32": 14400.0}})
    assert autotune.serving_batches(t, (16,), 24, batch_ms=1.25) == {16: 16}
    assert autotune.serving_batches(t, (16,), 24, batch_ms=0.1) == {16: 1}
    assert autotune.serving_batches(t, (16,), 24, batch_ms=10.0) == {16: 32}


class FakeCtx:
    def __init__(self, log_n):
        self.log_n = log_n
        self.plan = FakePlan(log_n)


def test_apply_ckks_takes_tuned_shape():
    """A context's key switch takes the tuned item width, ring depth and
    inner-product variant; a one-pass choice becomes the library default,
    which takes one pass only for launches that fill the CUs, and the
    persistent grid stays the library's."""
    t = autotune.TuneTable()
    t.put(autotune.ntt_key(14, 24, 64), {"algo": "mfma", "fs_passes": 1, "fs_wide": 1, "fs_wg_per_cu": 2})
    t.put(autotune.hmult_key(14, 24), {"batch": 32, "ks_inner": 1})
    ctx = FakeCtx(14)
    got = autotune.apply_ckks(ctx, t)
    # the returned entry is what the context got
    assert got["ks_inner"] == 1 and got["ntt"]["fs_passes"] == 0 and got["ntt"]["fs_wg_per_cu"] == 0
    assert t.get(autotune.ntt_key(14, 24, 64))["fs_passes"] == 1  # the table itself is unchanged
    assert ctx.plan.params["fs_passes"] == 0 and ctx.plan.params["fs_wide"] == 1
    assert ctx.plan.params["fs_wg_per_cu"] == 0  # the library's grid for HMULT's launches
    assert ctx.plan.params["ks_inner"] == 1


def test_ks_inner_choice_margin():
    """The fused inner product stays unless the separate kernels measured
    more than 2 % faster."""
    assert autotune.ks_inner_choice({"ks_inner_ops_per_s": {"1": 100.0, "2": 101.5}, "ks_inner": 2}) == 1
    assert autotune.ks_inner_choice({"ks_inner_ops_per_s": {"1": 100.0, "2": 103.0}}) == 2
    assert autotune.ks_inner_choice({"ks_inner_ops_per_s": {"1": 104.0, "2": 100.0}}) == 1
    assert autotune.ks_inner_choice({"ks_inner": 2}) == 2
    assert autotune.ks_inner_choice({"batch": 4}) is None


def test_search_space_covers_passes_and_ring_depth():
    c14 = autotune.ntt_candidates(14, True)
    assert ("mfma", 1, 0, 0, 0) in c14 and ("butterfly", 0, 0, 0, 0) in c14
    assert ("mfma", 2, 2, 0, 2) in c14 and ("mfma", 2, 2, 0, 3) in c14 and ("mfma", 2, 1, 0, 0) in c14
    assert all(p == 2 for a, p, _, _, _ in autotune.ntt_candidates(16, True) if a == "mfma")
    # ring depth only where the 256-point stage can take wide items
    assert {c[4] for c in autotune.ntt_candidates(12, True)} == {0}
    assert autotune.ntt_candidates(10, False) == [("butterfly", 0, 0, 0, 0)]


def test_shipped_table_is_well_formed():
    t = autotune.load_default()
    if not t.entries:
        pytest.skip("no tune table shipped")
    for k, v in t.entries.items():
        if k.startswith("ntt:"):
            assert v["algo"] in ("mfma", "butterfly") and v.get("fs_passes", 0) in (0, 1, 2)
        elif k.startswith("hmult:"):
            assert 1 <= v["batch"] <= 64


@pytest.mark.gpu
def test_tuned_plan_matches_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2212_14191_amd import inputs, tfhe
    qs = oracle.ntt_primes(4, 31, 1 << 17)
    plan = tfhe.NttPlan(14, qs)
    x_host = inputs.uniform_residues(0, qs, (8, 1 << 14))
    x = torch.from_numpy(x_host.view(np.int32)).cuda()
    best, table = autotune.tune_ntt(plan, x, reps=2)
    assert len(table) >= 16 and best["kops"] > 0
    assert any(c["fs_passes"] == 1 for c in table)
    t = autotune.TuneTable()
    t.put(autotune.ntt_key(14, 4, 8), best)
    assert autotune.apply(plan, t, 4, 8) == best
    got = plan.fwd(x).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.ntt_fwd(x_host, qs, plan.psi))


@pytest.mark.gpu
def test_tune_hmult_batch_and_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import ckks
    from paper_2212_14191_amd import inputs, tfhe
    n, L, K, dnum, level = 1 << 12, 8, 4, 2, 6
    pr = ckks.Params(n, L=L, K=K, dnum=dnum)
    s = inputs.ternary_secret(1, n, 64)
    a = inputs.uniform_residues(1, pr.moduli, (dnum, n), stream=1).transpose(1, 0, 2)
    evk = ckks.relin_key(pr, s, a, inputs.gaussian_error(2, (dnum, n), stream=1))
    ctx = tfhe.CkksContext(12, L, K, dnum, moduli=pr.moduli)
    to_dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).view(np.int32)).cuda()
    evk_d = to_dev(evk)
    made = {}

    def make(b):
        cts = []
        for k in range(2):
            m = inputs.small_messages(k, (b, n))
            c1 = inputs.uniform_residues(5 + k, pr.mods(range(level)), (b, n), stream=5)
            cts.append(ckks.encrypt(pr, s, m, c1, inputs.gaussian_error(2, (b, n), stream=9 + k), level))
        made[b] = cts
        return to_dev(cts[0]), to_dev(cts[1]), evk_d

    batch, tput = autotune.tune_hmult_batch(ctx, make, level, batches=(1, 2, 4), reps=2)
    assert batch in (1, 2, 4) and set(tput) == {1, 2, 4} and all(v > 0 for v in tput.values())
    ca, cb = made[batch]
    got = ctx.hmult(to_dev(ca), to_dev(cb), evk_d, level).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ckks.hmult(pr, ca, cb, evk, level))
