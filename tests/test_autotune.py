"""Autotuner selection logic and persistence (CPU), and a GPU tuning run
whose chosen configuration gives the same bits as the default."""
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


@pytest.mark.gpu
def test_tuned_plan_is_bit_identical():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2212_14191_amd import inputs, tfhe
    qs = oracle.ntt_primes(4, 31, 1 << 17)
    plan = tfhe.NttPlan(16, qs)
    x_host = inputs.uniform_residues(0, qs, (8, 1 << 16))
    x = torch.from_numpy(x_host.view(np.int32)).cuda()
    ref = plan.fwd(x).clone()
    best, table = autotune.tune_ntt(plan, x, reps=2)
    assert len(table) >= 2 and best["kops"] > 0
    t = autotune.TuneTable()
    t.put(autotune.ntt_key(16, 4, 8), best)
    assert autotune.apply(plan, t, 4, 8)
    assert torch.equal(plan.fwd(x), ref)
