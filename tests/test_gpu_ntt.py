"""GPU parity of the NTT / INTT / element-wise kernels against the oracle,
bit-exact (integer work), called through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2212_14191_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_14191_amd import tfhe
    tfhe.load()
    return tfhe


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).cuda()


def to_host(t):
    return t.cpu().numpy().view(np.uint32)


PRIMES31 = oracle.ntt_primes(6, 31, 1 << 17)


@pytest.mark.parametrize("log_n", [4, 5, 8, 11, 12, 13, 14, 15, 16])
def test_butterfly_matches_oracle(tf, log_n):
    n = 1 << log_n
    qs = PRIMES31[:3]
    plan = tf.NttPlan(log_n, qs, algo="butterfly")
    psis = plan.psi
    assert psis == [oracle.psi(q, n) for q in qs]
    x = inputs.uniform_residues(log_n, qs, (3, n))
    X = plan.fwd(to_dev(x))
    ref = oracle.ntt_fwd(x, qs, psis)
    assert np.array_equal(to_host(X), ref)
    back = plan.inv(to_dev(ref))
    assert np.array_equal(to_host(back), x)


@pytest.mark.parametrize("log_n,batch", [(16, 1), (16, 3), (15, 3), (14, 5), (13, 3), (12, 1), (12, 7)])
def test_mfma_matches_oracle(tf, log_n, batch):
    """Four-step MFMA transform (N = N1 x 256, N1 = 16 .. 256) against the
    oracle, forward and inverse, on three limbs."""
    n = 1 << log_n
    qs = PRIMES31[:3]
    plan = tf.NttPlan(log_n, qs, algo="mfma")
    assert plan.algo == tf.FOURSTEP_MFMA
    x = inputs.uniform_residues(100 + batch + log_n, qs, (batch, n))
    ref = oracle.ntt_fwd(x, qs, plan.psi)
    X = plan.fwd(to_dev(x), algo="mfma")
    assert np.array_equal(to_host(X), ref)
    back = plan.inv(to_dev(ref), algo="mfma")
    assert np.array_equal(to_host(back), x)


# One prime from each window the four-step kernel treats differently: above
# 0x7F7F7F7F (the digit window of a centered residue needs the correction),
# a 31-bit prime at or below it (the correction-free body, which every
# default CKKS q-limb takes), and a 30-bit prime.
WINDOWS = {
    "q31_above_window": [q for q in PRIMES31 if q > 0x7F7F7F7F][:1],
    "q31_in_window": [q for q in oracle.ntt_primes(40, 31, 1 << 17) if q <= 0x7F7F7F7F][:1],
    "q30": oracle.ntt_primes(1, 30, 1 << 17),
}


@pytest.mark.parametrize("window", sorted(WINDOWS))
@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_mfma_matches_oracle_per_prime_window(tf, log_n, window):
    """The MFMA transform at every N = 2^12..2^16 for a prime of each window,
    forward and inverse against the oracle (ragged batch of 3, plus edge
    values 0, q - 1 and residues straddling 0x7F7F7F7F)."""
    n = 1 << log_n
    qs = WINDOWS[window]
    assert len(qs) == 1
    q = qs[0]
    plan = tf.NttPlan(log_n, qs, algo="mfma")
    assert plan.algo == tf.FOURSTEP_MFMA
    x = inputs.uniform_residues(200 + log_n, qs, (3, n))
    x[0, 1, : n // 2] = q - 1
    x[0, 1, n // 2:] = np.minimum(np.uint32(0x7F7F7F70) + np.arange(n // 2, dtype=np.uint32) % 32, q - 1)
    x[0, 2, :7] = 0
    ref = oracle.ntt_fwd(x, qs, plan.psi)
    assert np.array_equal(to_host(plan.fwd(to_dev(x), algo="mfma")), ref)
    assert np.array_equal(to_host(plan.inv(to_dev(ref), algo="mfma")), x)
    assert np.array_equal(to_host(plan.inv(to_dev(x), algo="mfma")), oracle.ntt_inv(x, qs, plan.psi))


@pytest.mark.parametrize("log_n,wide,ring", [(12, 0, 0), (13, 0, 0), (14, 0, 0), (15, 0, 0), (13, 2, 0),
                                              (14, 2, 0), (15, 1, 0), (16, 1, 0), (16, 2, 0), (13, 2, 3),
                                              (15, 0, 3), (16, 2, 3), (16, 1, 2)])
def test_mfma_equals_butterfly_ragged(tf, log_n, wide, ring):
    """Batches whose polynomial count is not a multiple of the workgroup
    grouping (5 limbs x 37 polynomials), with the default, narrow (1) and
    wide (2) items of the 256-point stage and the two LDS ring depths of the
    wide items (0 = default 2, 3; narrow items ignore it): MFMA == butterfly
    bit for bit, and the MFMA round trip is the identity."""
    n = 1 << log_n
    qs = PRIMES31[:5]
    plan = tf.NttPlan(log_n, qs)
    plan.set_param("fs_wide", wide)
    plan.set_param("fs_ring", ring)
    assert plan.get_param("fs_wide") == wide and plan.get_param("fs_ring") == ring
    x = to_dev(inputs.uniform_residues(7 * log_n, qs, (37, n)))
    f_m = plan.fwd(x, algo="mfma")
    f_b = plan.fwd(x, algo="butterfly")
    assert torch.equal(f_m, f_b)
    assert torch.equal(plan.inv(f_m, algo="mfma"), x)


def test_mfma_small_primes_config1(tf):
    """N = 2^12 with the four largest primes below 2^30 (q = 1 mod 2^13)."""
    n = 1 << 12
    qs = oracle.ntt_primes(4, 30, 1 << 13)
    plan = tf.NttPlan(12, qs, algo="mfma")
    x = inputs.uniform_residues(12, qs, (8, n))
    ref = oracle.ntt_fwd(x, qs, plan.psi)
    X = plan.fwd(to_dev(x), algo="mfma")
    assert np.array_equal(to_host(X), ref)
    assert np.array_equal(to_host(plan.inv(X, algo="mfma")), x)


def test_mfma_edge_values(tf):
    """All-zero, all q-1, single spikes and values near 0x7F7F7F7F."""
    n = 1 << 16
    qs = [PRIMES31[0], oracle.ntt_primes(1, 30, 1 << 17)[0]]
    plan = tf.NttPlan(16, qs)
    x = np.zeros((2, 4, n), np.uint32)
    for l, q in enumerate(qs):
        x[l, 1] = q - 1
        x[l, 2, 0] = q - 1
        x[l, 2, n - 1] = 1
        x[l, 3] = np.minimum(np.uint32(0x7F7F7F7F) + np.arange(n, dtype=np.uint32) % 64, q - 1)
    ref = oracle.ntt_fwd(x, qs, plan.psi)
    for algo in ("mfma", "butterfly"):
        got = to_host(plan.fwd(to_dev(x), algo=algo))
        assert np.array_equal(got, ref), algo
        assert np.array_equal(to_host(plan.inv(to_dev(ref), algo=algo)), x), algo


def test_in_place_and_limb_offset(tf):
    n = 1 << 16
    qs = PRIMES31[:5]
    plan = tf.NttPlan(16, qs)
    x = inputs.uniform_residues(9, qs[2:4], (2, n))
    ref = oracle.ntt_fwd(x, qs[2:4], plan.psi[2:4])
    for algo in ("mfma", "butterfly"):
        t = to_dev(x)
        plan.fwd(t, out=t, algo=algo, limb_begin=2)
        assert np.array_equal(to_host(t), ref), algo
        plan.inv(t, out=t, algo=algo, limb_begin=2)
        assert np.array_equal(to_host(t), x), algo


def test_config1_negacyclic_product(tf):
    """N=2^12, 4 limbs of 30-bit primes, 8 pairs: INTT(NTT(a) o NTT(b)) equals
    the schoolbook negacyclic product, bit for bit."""
    n = 1 << 12
    qs = oracle.ntt_primes(4, 30, 2 * n)
    plan = tf.NttPlan(12, qs)
    a = inputs.uniform_residues(0, qs, (8, n))
    b = inputs.uniform_residues(0, qs, (8, n), stream=1)
    A = plan.fwd(to_dev(a))
    B = plan.fwd(to_dev(b))
    c = plan.inv(plan.mul(A, B))
    ref, _ = oracle.negacyclic_mul(a, b, qs)
    assert np.array_equal(to_host(c), ref)


def test_elementwise_ops(tf):
    n = 1 << 12
    qs = PRIMES31[:3]
    plan = tf.NttPlan(12, qs)
    a = inputs.uniform_residues(1, qs, (5, n))
    b = inputs.uniform_residues(2, qs, (5, n))
    bb = inputs.uniform_residues(3, qs, n)
    A, B = to_dev(a), to_dev(b)
    assert np.array_equal(to_host(plan.mul(A, B)), oracle.mul(a, b, qs))
    assert np.array_equal(to_host(plan.add(A, B)), oracle.add(a, b, qs))
    assert np.array_equal(to_host(plan.sub(A, B)), oracle.sub(a, b, qs))
    want = oracle.mul(a, np.broadcast_to(bb[:, None, :], a.shape), qs)
    assert np.array_equal(to_host(plan.mul_bcast(A, to_dev(bb))), want)
    # extremes: (q-1)^2 and 0
    e = np.stack([np.full((2, n), q - 1, np.uint32) for q in qs])
    E = to_dev(e)
    assert np.array_equal(to_host(plan.mul(E, E)), oracle.mul(e, e, qs))


def test_frobenius_map(tf):
    from oracle import ckks
    n = 1 << 12
    qs = PRIMES31[:2]
    plan = tf.NttPlan(12, qs)
    x = inputs.uniform_residues(4, qs, (2, n))
    for r in (1, 3, 100):
        k = ckks.galois_element(r, n)
        want = oracle.ntt_fwd(ckks.automorphism_coeff(oracle.ntt_inv(x, qs, plan.psi), k, qs), qs, plan.psi)
        assert np.array_equal(to_host(plan.frobenius(to_dev(x), k)), want)


def test_empty_batch_and_errors(tf):
    n = 1 << 16
    qs = PRIMES31[:2]
    plan = tf.NttPlan(16, qs)
    empty = torch.empty((2, 0, n), dtype=torch.int32, device="cuda")
    plan.fwd(empty, out=torch.empty_like(empty))
    x = to_dev(inputs.uniform_residues(5, qs, (1, n)))
    small_ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(tf.TfheError) as ei:
        plan.fwd(x, ws=small_ws)
    assert ei.value.status == tf.TFHE_EINVAL
    with pytest.raises(tf.TfheError) as ei:
        plan.fwd(x, limb_begin=1)       # limbs [1, 3) exceed the plan
    assert ei.value.status == tf.TFHE_EINVAL


def test_deterministic(tf):
    n = 1 << 16
    qs = PRIMES31[:2]
    plan = tf.NttPlan(16, qs)
    x = to_dev(inputs.uniform_residues(6, qs, (4, n)))
    for algo in ("mfma", "butterfly"):
        a = plan.fwd(x, algo=algo)
        b = plan.fwd(x, algo=algo)
        assert torch.equal(a, b)


@pytest.mark.slow
@pytest.mark.parametrize("launch", ["tuned", "default"])
def test_full_size_44x128_sampled(tf, launch):
    """Config 2/3 shape (N=2^16, 44 limbs, 128 polynomials) in the launch
    configuration the benchmark times (the shipped tune table applied to the
    plan, as bench.py does) and in the library default: MFMA == butterfly
    everywhere, round trip everywhere, and sampled (limb, poly) units equal
    the oracle."""
    from paper_2212_14191_amd import autotune
    n = 1 << 16
    qs = oracle.ntt_primes(44, 31, 1 << 17)
    assert list(qs) == list(tf.tfhe_find_primes(31, 1 << 17, 44))  # bench.py's primes
    plan = tf.NttPlan(16, qs)
    if launch == "tuned":
        table = autotune.load_default()
        if autotune.apply(plan, table, 44, 128) is None:
            pytest.skip("no tune table entry for this shape")
    x_host = inputs.uniform_residues(0, qs, (128, n))
    x = to_dev(x_host)
    ws = plan.workspace(44, 128, "mfma")
    f_m = plan.fwd(x, algo="mfma", ws=ws)
    f_b = plan.fwd(x, algo="butterfly", ws=ws)
    assert torch.equal(f_m, f_b)
    del f_b
    back = plan.inv(f_m, algo="mfma", ws=ws)
    assert torch.equal(back, x)
    rng = np.random.default_rng(1)
    got = to_host(f_m)
    for _ in range(12):
        l, b = int(rng.integers(44)), int(rng.integers(128))
        ref = oracle.ntt_fwd(x_host[l, b], [qs[l]], [plan.psi[l]])
        assert np.array_equal(got[l, b], ref), (l, b)


def test_fused_batch_mixed_sizes_and_directions(tf):
    """Operation-level batching: one fused launch per pass covers transforms
    of different N, limb ranges and directions (butterfly), and of different
    directions and batches (MFMA, N = 2^13 and 2^16)."""
    plans = {ln: tf.NttPlan(ln, PRIMES31[:3]) for ln in (10, 13, 16)}
    specs = [(10, False, 3), (13, True, 2), (16, False, 1), (16, True, 2), (13, False, 1), (10, True, 4)]
    items, refs = [], []
    for ln, inv, b in specs:
        n = 1 << ln
        plan = plans[ln]
        x = inputs.uniform_residues(ln * 10 + b, plan.q[1:3], (b, n))
        X = to_dev(x)
        items.append((plan, X, torch.empty_like(X), inv, 1))
        refs.append(oracle.ntt(x, plan.q[1:3], plan.psi[1:3], inverse=inv)[0])
    for o, r in zip(tf.ntt_batch(items, algo="butterfly"), refs):
        assert np.array_equal(to_host(o), r)
    mf = [(i, r) for (i, r), (ln, _, _) in zip(zip(items, refs), specs) if ln >= 12]
    outs = tf.ntt_batch([i for i, _ in mf], algo="mfma")
    for o, (_, r) in zip(outs, mf):
        assert np.array_equal(to_host(o), r)
    first16 = next(k for k, (ln, inv, _) in enumerate(specs) if ln == 16 and not inv)
    X = items[first16][1].clone()
    tf.ntt_batch([(plans[16], X, X, False, 1)], algo="mfma")   # in place
    assert np.array_equal(to_host(X), refs[first16])


def test_valu_gemm_variant_matches_oracle(tf):
    """The vector-ALU GEMM four-step variant (N = 2^16): forward and inverse
    equal the oracle; on a ragged 4 x 21 batch it equals the MFMA transform
    and round-trips; other N and the fused-batch API refuse it."""
    n = 1 << 16
    qs = PRIMES31[:4]
    plan = tf.NttPlan(16, qs)
    x = inputs.uniform_residues(321, qs[:2], (2, n))
    ref = oracle.ntt_fwd(x, qs[:2], plan.psi[:2])
    X = plan.fwd(to_dev(x), algo="co")
    assert np.array_equal(to_host(X), ref)
    assert np.array_equal(to_host(plan.inv(to_dev(ref), algo="co")), x)
    y = to_dev(inputs.uniform_residues(322, qs, (21, n)))
    f_co = plan.fwd(y, algo="co")
    assert torch.equal(f_co, plan.fwd(y, algo="mfma"))
    assert torch.equal(plan.inv(f_co, algo="co"), y)
    small = tf.NttPlan(15, qs[:1])
    with pytest.raises(tf.TfheError):
        small.fwd(to_dev(inputs.uniform_residues(1, qs[:1], (1, 1 << 15))), algo="co")
    with pytest.raises(tf.TfheError):
        tf.ntt_batch([(plan, y, torch.empty_like(y), False, 0)], algo="co")


def test_fused_batch_beyond_one_launch_table(tf):
    """More units than one launch's descriptor table holds (40 for the
    four-step passes, 32 for the butterfly): 83 transforms of N = 2^12 with
    different limb offsets, batches and directions, each equal to the oracle."""
    plan = tf.NttPlan(12, PRIMES31[:4])
    n = 1 << 12
    items, refs = [], []
    for k in range(83):
        lb, limbs, b, inv = k % 3, 1 + (k % 2), 1 + (k % 3), bool(k % 2)
        x = inputs.uniform_residues(900 + k, plan.q[lb:lb + limbs], (b, n))
        X = to_dev(x)
        items.append((plan, X, torch.empty_like(X), inv, lb))
        refs.append(oracle.ntt(x, plan.q[lb:lb + limbs], plan.psi[lb:lb + limbs], inverse=inv)[0])
    for algo in ("mfma", "butterfly"):
        outs = tf.ntt_batch(items, algo=algo)
        for k, (o, r) in enumerate(zip(outs, refs)):
            assert np.array_equal(to_host(o), r), (algo, k)


@pytest.mark.parametrize("passes", [1, 2])
@pytest.mark.parametrize("log_n", [12, 13, 14, 15])
def test_mfma_one_and_two_passes_match_oracle(tf, log_n, passes):
    """The four-step transform with one HBM round trip (polynomial resident
    in LDS) and with two, at N = 2^12..2^15: forward and inverse against the
    oracle for limbs from all three prime windows, on a ragged batch of 7
    polynomials (workgroups end on partial polynomial ranges), in place."""
    n = 1 << log_n
    qs = [WINDOWS[w][0] for w in sorted(WINDOWS)] + PRIMES31[1:3]
    plan = tf.NttPlan(log_n, qs, algo="mfma")
    plan.set_param("fs_passes", passes)
    assert plan.get_param("fs_passes") == passes
    x = inputs.uniform_residues(300 + log_n, qs, (7, n))
    x[0, 0, :5] = [0, qs[0] - 1, 1, qs[0] - 2, 0x7F7F7F7F % qs[0]]
    ref = oracle.ntt_fwd(x, qs, plan.psi)
    X = to_dev(x)
    plan.fwd(X, out=X, algo="mfma")
    assert np.array_equal(to_host(X), ref)
    plan.inv(X, out=X, algo="mfma")
    assert np.array_equal(to_host(X), x)
    assert np.array_equal(to_host(plan.inv(to_dev(x), algo="mfma")), oracle.ntt_inv(x, qs, plan.psi))


@pytest.mark.parametrize("log_n", [12, 13, 14, 15])
def test_mfma_one_pass_large_batch_equals_two_pass(tf, log_n):
    """A batch of 8 limbs x 129 polynomials (more polynomials than
    workgroups, ranges crossing limbs): one pass == two passes bit for bit,
    both directions; sampled polynomials against the oracle."""
    n = 1 << log_n
    qs = PRIMES31[:4] + [WINDOWS["q31_in_window"][0]] + oracle.ntt_primes(3, 30, 1 << 17)
    plan = tf.NttPlan(log_n, qs, algo="mfma")
    x = to_dev(inputs.uniform_residues(400 + log_n, qs, (129, n)))
    plan.set_param("fs_passes", 2)
    f2, i2 = plan.fwd(x, algo="mfma"), plan.inv(x, algo="mfma")
    plan.set_param("fs_passes", 1)
    f1, i1 = plan.fwd(x, algo="mfma"), plan.inv(x, algo="mfma")
    assert torch.equal(f1, f2)
    assert torch.equal(i1, i2)
    # the library default (one pass at N <= 2^14 for launches this large)
    plan.set_param("fs_passes", 0)
    assert torch.equal(plan.fwd(x, algo="mfma"), f2)
    assert torch.equal(plan.inv(x, algo="mfma"), i2)
    xs = to_host(x)
    for l, b in ((0, 0), (3, 128), (7, 64)):
        got = to_host(f1)[l:l + 1, b:b + 1]
        assert np.array_equal(got, oracle.ntt_fwd(xs[l:l + 1, b:b + 1], qs[l:l + 1], plan.psi[l:l + 1]))
