"""GPU parity of HMULT, HROTATE, RESCALE, CMULT and HADD against the oracle
(bit-exact), plus decryption of the GPU results, through the C ABI."""
import numpy as np
import pytest

import oracle
from oracle import ckks
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


def setup(n, L, K, dnum, h=None):
    pr = ckks.Params(n, L=L, K=K, dnum=dnum)
    s = inputs.ternary_secret(1, n, h or min(192, n // 2))
    a = inputs.uniform_residues(1, pr.moduli, (dnum, n), stream=1).transpose(1, 0, 2)
    e = inputs.gaussian_error(2, (dnum, n), stream=1)
    evk = ckks.relin_key(pr, s, a, e)
    return pr, s, evk, (a, e)


def encrypt(pr, s, m, level, seed):
    b = m.shape[0]
    c1 = inputs.uniform_residues(seed, pr.mods(range(level)), (b, pr.n), stream=5)
    e = inputs.gaussian_error(2, (b, pr.n), stream=seed + 10)
    return ckks.encrypt(pr, s, m, c1, e, level)


@pytest.mark.parametrize("log_n,L,K,dnum,level", [
    (10, 6, 2, 3, 6), (10, 6, 2, 3, 5), (10, 6, 2, 3, 1), (12, 8, 4, 2, 8), (12, 8, 4, 2, 3),
    (13, 24, 8, 3, 24), (13, 24, 8, 3, 17), (5, 6, 2, 3, 6), (10, 12, 2, 12, 12), (10, 12, 2, 12, 9),
    (10, 40, 4, 10, 40), (10, 40, 4, 10, 37)])
def test_hmult_matches_oracle(tf, log_n, L, K, dnum, level):
    """Bit-exact HMULT.  The basis conversions run on the matrix cores,
    except at N = 2^5 (3 x 32-word planes are not whole 64-word chunks),
    which takes the VALU conversion; dnum = 12 runs the inner product in
    two digit groups; L = 40 gives conversions of more than 32 targets
    (ModUp 40 and 37-40, ModDown 40 and 37), each split over two
    descriptors."""
    n = 1 << log_n
    pr, s, evk, _ = setup(n, L, K, dnum)
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    assert ctx.moduli == pr.moduli and ctx.plan.psi == pr.psi
    m1 = inputs.small_messages(0, (3, n))
    m2 = inputs.small_messages(0, (3, n), stream=1)
    ca, cb = encrypt(pr, s, m1, level, 1), encrypt(pr, s, m2, level, 2)
    want = ckks.hmult(pr, ca, cb, evk, level)
    got = to_host(ctx.hmult(to_dev(ca), to_dev(cb), to_dev(evk), level))
    assert np.array_equal(got, want)


def test_hmult_output_aliases_input(tf):
    n = 1 << 10
    pr, s, evk, _ = setup(n, 6, 2, 3)
    ctx = tf.CkksContext(10, 6, 2, 3, moduli=pr.moduli)
    m = inputs.small_messages(0, (2, n))
    ca, cb = encrypt(pr, s, m, 6, 1), encrypt(pr, s, m, 6, 2)
    want = ckks.hmult(pr, ca, cb, evk, 6)
    A = to_dev(ca)
    ctx.hmult(A, to_dev(cb), to_dev(evk), 6, out=A)
    assert np.array_equal(to_host(A), want)


@pytest.mark.parametrize("log_n,r", [(10, 1), (10, 7), (10, "conj"), (13, 5)])
def test_rotate_matches_oracle(tf, log_n, r):
    """HROTATE by 5^r, and conjugation (galois element 2N - 1 with its own
    key), bit-exact vs the oracle; N = 2^13 runs the MFMA transform."""
    n = 1 << log_n
    L, K, dnum, level = 6, 2, 3, 5
    pr, s, _, (a, e) = setup(n, L, K, dnum)
    k = 2 * n - 1 if r == "conj" else ckks.galois_element(r, n)
    rk = ckks.rotation_key(pr, s, k, a, e)
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    m = inputs.small_messages(0, (2, n))
    ct = encrypt(pr, s, m, level, 1)
    want = ckks.rotate(pr, ct, rk, k, level)
    got = to_host(ctx.rotate(to_dev(ct), to_dev(rk), k, level))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("log_n", [10, 13])
def test_rotate_multi_matches_oracle(tf, log_n):
    """Rotations by different amounts in one batch (repeated amounts,
    conjugation, partial last digit at level 5): each ciphertext equals the
    oracle's rotation of it alone and the single-amount entry point."""
    n = 1 << log_n
    L, K, dnum, level = 6, 2, 3, 5
    pr, s, _, (a, e) = setup(n, L, K, dnum)
    gal = [ckks.galois_element(1, n), ckks.galois_element(3, n), 2 * n - 1, ckks.galois_element(1, n),
           ckks.galois_element(7, n)]
    rks = {k: ckks.rotation_key(pr, s, k, a, e) for k in set(gal)}
    drk = {k: to_dev(v) for k, v in rks.items()}
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    m = inputs.small_messages(3, (len(gal), n))
    ct = encrypt(pr, s, m, level, 4)
    got = to_host(ctx.rotate_multi(to_dev(ct), [drk[k] for k in gal], gal, level))
    for b, k in enumerate(gal):
        one = np.ascontiguousarray(ct[:, :, b:b + 1])
        want = ckks.rotate(pr, one, rks[k], k, level)
        assert np.array_equal(got[:, :, b:b + 1], want), f"element {b}, galois {k}"
        alone = to_host(ctx.rotate(to_dev(one), drk[k], k, level))
        assert np.array_equal(alone, want)


def test_rotate_multi_errors(tf):
    n = 1 << 10
    L, K, dnum, level = 6, 2, 3, 5
    pr, s, _, (a, e) = setup(n, L, K, dnum)
    k = ckks.galois_element(1, n)
    rk = to_dev(ckks.rotation_key(pr, s, k, a, e))
    ctx = tf.CkksContext(10, L, K, dnum, moduli=pr.moduli)
    ct = to_dev(encrypt(pr, s, inputs.small_messages(0, (2, n)), level, 1))
    with pytest.raises(tf.TfheError):
        ctx.rotate_multi(ct, [rk, rk], [k, 2 * k], level)          # even Galois element
    with pytest.raises(tf.TfheError):
        ctx.rotate_multi(ct, [rk, rk], [k, 2 * n + 1], level)      # not below 2N
    with pytest.raises(ValueError):
        ctx.rotate_multi(ct, [rk], [k], level)                     # one key per ciphertext
    big = torch.zeros((2, level, 65, n), dtype=torch.int32, device="cuda")
    with pytest.raises(tf.TfheError):
        ctx.rotate_multi(big, [rk] * 65, [k] * 65, level)          # above TFHE_ROTATE_MULTI_MAX
    with pytest.raises(tf.TfheError):
        ctx.rotate_multi(ct, [rk, rk], [k, k], level, out=ct)      # output aliases the input


_KEYS = {}


def serving_setup(log_n):
    """Keys of the serving shapes (L = 24, K = 8, dnum = 3, default moduli:
    every q-limb lies at or below 0x7F7F7F7F), cached per N."""
    if log_n not in _KEYS:
        n = 1 << log_n
        pr, s, evk, (a, e) = setup(n, 24, 8, 3)
        k = ckks.galois_element(5, n)
        _KEYS[log_n] = (pr, s, evk, k, ckks.rotation_key(pr, s, k, a, e))
    return _KEYS[log_n]


_ROT_KEYS = {}


def serving_rotation_key(log_n, r):
    """A second rotation key of the serving shapes (slots rotated by r)."""
    if (log_n, r) not in _ROT_KEYS:
        n = 1 << log_n
        pr = ckks.Params(n, L=24, K=8, dnum=3)
        s = inputs.ternary_secret(1, n, min(192, n // 2))
        a = inputs.uniform_residues(1, pr.moduli, (3, n), stream=1).transpose(1, 0, 2)
        e = inputs.gaussian_error(2, (3, n), stream=1)
        k = ckks.galois_element(r, n)
        _ROT_KEYS[(log_n, r)] = (k, ckks.rotation_key(pr, s, k, a, e))
    return _ROT_KEYS[(log_n, r)]


@pytest.mark.parametrize("level", [1, 9, 17, 24])
@pytest.mark.parametrize("log_n", [14, 15])
def test_hmult_rotate_serving_shapes_match_oracle(tf, log_n, level):
    """HMULT and HROTATE at the serving mix's N = 2^14 and 2^15 (L = 24,
    K = 8, dnum = 3) at levels with one partial digit (1, 9, 17) and three
    full digits (24), bit-exact against the oracle; from level 9 on the
    HMULT result of the first ciphertext also decrypts to m1 * m2."""
    n = 1 << log_n
    pr, s, evk, k, rk = serving_setup(log_n)
    assert max(pr.q) <= 0x7F7F7F7F
    ctx = tf.CkksContext(log_n, 24, 8, 3, moduli=pr.moduli)
    m1 = inputs.small_messages(log_n, (2, n))
    m2 = inputs.small_messages(log_n, (2, n), stream=1)
    ca, cb = encrypt(pr, s, m1, level, 11), encrypt(pr, s, m2, level, 12)
    got = to_host(ctx.hmult(to_dev(ca), to_dev(cb), to_dev(evk), level))
    assert np.array_equal(got, ckks.hmult(pr, ca, cb, evk, level))
    if level >= 3:      # the decryption bound needs Q_l > 2^60 * N * 16^2 * 2
        dec = ckks.decrypt(pr, s, got[:, :, :1], level)[0]
        d2 = 1 << 60
        prod = ckks.negacyclic_int(m1[0], m2[0])
        assert np.array_equal(np.array([(int(v) + d2 // 2) // d2 for v in dec]), prod)
    got_r = to_host(ctx.rotate(to_dev(ca), to_dev(rk), k, level))
    assert np.array_equal(got_r, ckks.rotate(pr, ca, rk, k, level))


@pytest.mark.parametrize("level", [9, 24])
def test_ring_depth_three_matches_oracle(tf, level):
    """HMULT, HROTATE and RESCALE at N = 2^15 (wide items) with the
    three-stage LDS ring instead of the default two: bit-exact against the
    oracle (the key switch's fused and epilogue passes included)."""
    log_n = 15
    n = 1 << log_n
    pr, s, evk, k, rk = serving_setup(log_n)
    ctx = tf.CkksContext(log_n, 24, 8, 3, moduli=pr.moduli)
    ctx.plan.set_param("fs_ring", 3)
    assert ctx.plan.get_param("fs_ring") == 3
    m1 = inputs.small_messages(log_n, (2, n))
    m2 = inputs.small_messages(log_n, (2, n), stream=1)
    ca, cb = encrypt(pr, s, m1, level, 11), encrypt(pr, s, m2, level, 12)
    got = to_host(ctx.hmult(to_dev(ca), to_dev(cb), to_dev(evk), level))
    assert np.array_equal(got, ckks.hmult(pr, ca, cb, evk, level))
    got_r = to_host(ctx.rotate(to_dev(ca), to_dev(rk), k, level))
    assert np.array_equal(got_r, ckks.rotate(pr, ca, rk, k, level))
    assert np.array_equal(to_host(ctx.rescale(to_dev(ca), level)), ckks.rescale(pr, ca, level))


@pytest.mark.slow
def test_rotate_full_size_level24(tf):
    """HROTATE at N = 2^16, level 24 (L = 24, K = 8, dnum = 3) on a batch of
    three, bit-exact against the oracle."""
    pr, s, _, k, rk = serving_setup(16)
    n = 1 << 16
    ctx = tf.CkksContext(16, 24, 8, 3, moduli=pr.moduli)
    ct = encrypt(pr, s, inputs.small_messages(16, (3, n)), 24, 13)
    got = to_host(ctx.rotate(to_dev(ct), to_dev(rk), k, 24))
    assert np.array_equal(got, ckks.rotate(pr, ct, rk, k, 24))


@pytest.mark.slow
def test_hmult_config4_full_size_sampled(tf):
    """N=2^16, L=24, K=8, dnum=3, h=192, 64 pairs on the GPU (MFMA NTT) in
    the launch configuration the benchmark times (the shipped tune table
    applied to the context, as bench.py does); sampled pairs (the first,
    both sides of the middle, an interior one and the last) equal the oracle
    bit for bit and decrypt to m1*m2."""
    from paper_2212_14191_amd import autotune
    n, L, K, dnum, level, B = 1 << 16, 24, 8, 3, 24, 64
    pr, s, evk, _ = setup(n, L, K, dnum)
    ctx = tf.CkksContext(16, L, K, dnum, moduli=pr.moduli)
    autotune.apply_ckks(ctx, autotune.load_default())
    m1 = inputs.small_messages(0, (B, n))
    m2 = inputs.small_messages(0, (B, n), stream=1)
    ca, cb = encrypt(pr, s, m1, level, 1), encrypt(pr, s, m2, level, 2)
    got = to_host(ctx.hmult(to_dev(ca), to_dev(cb), to_dev(evk), level))
    for b in (0, 31, 32, 37, 63):
        want = ckks.hmult(pr, ca[:, :, b:b + 1], cb[:, :, b:b + 1], evk, level)
        assert np.array_equal(got[:, :, b:b + 1], want), b
        dec = ckks.decrypt(pr, s, got[:, :, b:b + 1], level)[0]
        prod = ckks.negacyclic_int(m1[b], m2[b])
        d2 = 1 << 60
        assert np.array_equal(np.array([(int(v) + d2 // 2) // d2 for v in dec]), prod)


def test_device_keygen_and_encryption_match_oracle(tf):
    """The library-side key generation / encryption (paper_2212_14191_amd.scheme)
    produce the oracle's keys and ciphertexts from the same random draws."""
    from paper_2212_14191_amd.scheme import Scheme
    n = 1 << 10
    pr, s, evk, (a, e) = setup(n, 6, 2, 3)
    ctx = tf.CkksContext(10, 6, 2, 3, moduli=pr.moduli)
    sch = Scheme(ctx)
    assert np.array_equal(to_host(sch.relin_key(s, a, e)), evk)
    k = ckks.galois_element(3, n)
    assert np.array_equal(to_host(sch.rotation_key(s, k, a, e)), ckks.rotation_key(pr, s, k, a, e))
    m = inputs.small_messages(0, (3, n))
    c1 = inputs.uniform_residues(4, pr.mods(range(5)), (3, n), stream=5)
    ee = inputs.gaussian_error(2, (3, n), stream=9)
    got = to_host(sch.encrypt(s, m, c1, ee, 5))
    assert np.array_equal(got, ckks.encrypt(pr, s, m, c1, ee, 5))


def test_graph_replay_matches_eager(tf):
    """HMULT and HROTATE captured once as a HIP graph and replayed with new
    inputs, with eager work and synchronisation between replays: every replay
    equals the eager result bit for bit."""
    from paper_2212_14191_amd.graphs import CapturedOp
    n = 1 << 12
    L, K, dnum, level, B = 6, 2, 3, 5, 3
    pr, s, evk, (a, e) = setup(n, L, K, dnum)
    ctx = tf.CkksContext(12, L, K, dnum, moduli=pr.moduli)
    k = ckks.galois_element(3, n)
    rk = to_dev(ckks.rotation_key(pr, s, k, a, e))
    evk_d = to_dev(evk)
    g_mul = CapturedOp(ctx, evk_d, level, B, op=0)
    g_rot = CapturedOp(ctx, rk, level, B, op=1, galois=k)
    for rep in range(3):
        m1 = inputs.small_messages(rep, (B, n))
        m2 = inputs.small_messages(rep + 10, (B, n))
        ca, cb = to_dev(encrypt(pr, s, m1, level, 1 + rep)), to_dev(encrypt(pr, s, m2, level, 5 + rep))
        eager_mul = ctx.hmult(ca, cb, evk_d, level)
        eager_rot = ctx.rotate(ca, rk, k, level)
        torch.cuda.synchronize()
        got_mul = g_mul.run(ca, cb).clone()
        got_rot = g_rot.run(ca).clone()
        torch.cuda.synchronize()
        assert torch.equal(got_mul, eager_mul), rep
        assert torch.equal(got_rot, eager_rot), rep
        if rep == 0:
            want = ckks.hmult(pr, to_host(ca), to_host(cb), evk, level)
            assert np.array_equal(to_host(got_mul), want)


@pytest.mark.parametrize("log_n,L,K,dnum,level", [
    (10, 6, 2, 3, 6), (10, 6, 2, 3, 2), (12, 8, 4, 2, 5), (13, 24, 8, 3, 24), (14, 6, 2, 3, 3)])
def test_rescale_matches_oracle(tf, log_n, L, K, dnum, level):
    """RESCALE on the GPU (butterfly below N = 2^12, MFMA from 2^12) equals
    the oracle bit for bit and decrypts to Dec(ct) / q_{level-1} within 1 + h."""
    n = 1 << log_n
    pr, s, _, _ = setup(n, L, K, dnum)
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    m = inputs.small_messages(3, (3, n))
    ct = encrypt(pr, s, m, level, 7)
    got = to_host(ctx.rescale(to_dev(ct), level))
    want = ckks.rescale(pr, ct, level)
    assert np.array_equal(got, want)
    h = int(np.count_nonzero(s))
    qt = pr.q[level - 1]
    dec = ckks.decrypt(pr, s, ct[:, :, :1], level)
    dec2 = ckks.decrypt(pr, s, got[:, :, :1], level - 1)
    assert max(abs(int(b) * qt - int(a)) for a, b in zip(dec.ravel(), dec2.ravel())) <= (1 + h) * qt


def test_rescale_errors(tf):
    n = 1 << 10
    ctx = tf.CkksContext(10, 6, 2, 3)
    ct = torch.zeros((2, 1, 2, n), dtype=torch.int32, device="cuda")
    with pytest.raises(tf.TfheError):
        ctx.rescale(ct, 1)
    ct = torch.zeros((2, 3, 2, n), dtype=torch.int32, device="cuda")
    with pytest.raises(tf.TfheError):   # output overlapping the input
        ctx.rescale(ct, 3, out=ct.view(-1)[: 8 * n].view(2, 2, 2, n))


@pytest.mark.slow
def test_rescale_config4_full_size_sampled(tf):
    """N = 2^16, L = 24, 64 ciphertexts at level 24 (the HMULT benchmark
    shape, with the tuned launch configuration the benchmark applies): two
    sampled ciphertexts equal the oracle bit for bit."""
    from paper_2212_14191_amd import autotune
    n, L, K, dnum, level, B = 1 << 16, 24, 8, 3, 24, 64
    pr = ckks.Params(n, L=L, K=K, dnum=dnum)
    ctx = tf.CkksContext(16, L, K, dnum, moduli=pr.moduli)
    autotune.apply_ckks(ctx, autotune.load_default())
    qs = pr.mods(range(level))
    ct = np.stack([inputs.uniform_residues(60 + c, qs, (B, n)) for c in range(2)])
    got = to_host(ctx.rescale(to_dev(ct), level))
    for b in (0, 41):
        assert np.array_equal(got[:, :, b:b + 1], ckks.rescale(pr, ct[:, :, b:b + 1], level)), b


def test_cmult_hadd_match_oracle(tf):
    n = 1 << 12
    pr, s, _, _ = setup(n, 8, 4, 2)
    ctx = tf.CkksContext(12, 8, 4, 2, moduli=pr.moduli)
    level = 6
    qs, ps = pr.mods(range(level)), pr.psis(range(level))
    c1 = encrypt(pr, s, inputs.small_messages(1, (3, n)), level, 1)
    c2 = encrypt(pr, s, inputs.small_messages(2, (3, n)), level, 2)
    pt = oracle.ntt_fwd(oracle.to_residues(inputs.small_messages(3, (3, n)), qs), qs, ps)
    assert np.array_equal(to_host(ctx.cmult(to_dev(c1), to_dev(pt), level)), ckks.cmult(pr, c1, pt, level))
    assert np.array_equal(to_host(ctx.hadd(to_dev(c1), to_dev(c2), level)), ckks.hadd(pr, c1, c2, level))
    a = to_dev(c1)
    ctx.hadd(a, to_dev(c2), level, out=a)   # in place
    assert np.array_equal(to_host(a), ckks.hadd(pr, c1, c2, level))


def test_rotate_multi_at_the_batch_limit(tf):
    """TFHE_ROTATE_MULTI_MAX (64) ciphertexts, three rotation amounts and
    conjugation interleaved: each equals its rotation alone (one also
    against the oracle)."""
    n = 1 << 10
    L, K, dnum, level = 6, 2, 3, 4
    pr, s, _, (a, e) = setup(n, L, K, dnum)
    kinds = [ckks.galois_element(1, n), ckks.galois_element(2, n), ckks.galois_element(5, n), 2 * n - 1]
    B = tf.CkksContext.ROTATE_MULTI_MAX
    gal = [kinds[b % 4] for b in range(B)]
    rks = {k: ckks.rotation_key(pr, s, k, a, e) for k in kinds}
    drk = {k: to_dev(v) for k, v in rks.items()}
    ctx = tf.CkksContext(10, L, K, dnum, moduli=pr.moduli)
    m = inputs.small_messages(5, (B, n))
    ct = encrypt(pr, s, m, level, 6)
    got = to_host(ctx.rotate_multi(to_dev(ct), [drk[k] for k in gal], gal, level))
    for b in range(B):
        one = to_dev(np.ascontiguousarray(ct[:, :, b:b + 1]))
        alone = to_host(ctx.rotate(one, drk[gal[b]], gal[b], level))
        assert np.array_equal(got[:, :, b:b + 1], alone), b
    want = ckks.rotate(pr, np.ascontiguousarray(ct[:, :, 41:42]), rks[gal[41]], gal[41], level)
    assert np.array_equal(got[:, :, 41:42], want)


@pytest.mark.parametrize("log_n,L,K,dnum,level,B", [
    (12, 8, 4, 2, 8, 3), (13, 24, 8, 3, 17, 2), (14, 12, 2, 6, 11, 2), (16, 24, 8, 3, 24, 3), (12, 8, 1, 1, 8, 2)])
def test_fused_inner_product_equals_separate(tf, log_n, L, K, dnum, level, B):
    """Key switching with the ModUp transforms' second pass fused with the
    inner product (the default; wide items from N = 2^13, and narrow ones
    when the plan asks for them) and with the separate kernels: HMULT and a
    mixed-amount HROTATE batch give the same bits, and the fused HMULT equals
    the oracle (including K < alpha, where digits outnumber special primes)."""
    n = 1 << log_n
    pr, s, evk, (a, e) = setup(n, L, K, dnum)
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    m1 = inputs.small_messages(log_n, (B, n))
    m2 = inputs.small_messages(log_n, (B, n), stream=2)
    ca, cb = encrypt(pr, s, m1, level, 21), encrypt(pr, s, m2, level, 22)
    A, Bt, E = to_dev(ca), to_dev(cb), to_dev(evk)
    gal = [ckks.galois_element(1 + b, n) for b in range(B)]
    rks = [to_dev(ckks.rotation_key(pr, s, k, a, e)) for k in gal]
    got = {}
    for mode, wide in ((1, 0), (2, 0), (1, 1)):
        ctx.plan.set_param("ks_inner", mode)
        ctx.plan.set_param("fs_wide", wide)
        got[mode, wide] = (ctx.hmult(A, Bt, E, level).clone(), ctx.rotate_multi(A, rks, gal, level).clone())
    for k in ((2, 0), (1, 1)):
        assert torch.equal(got[1, 0][0], got[k][0]), k
        assert torch.equal(got[1, 0][1], got[k][1]), k
    got[1] = got[1, 0]
    b0 = 0 if log_n < 16 else B - 1
    want = ckks.hmult(pr, ca[:, :, b0:b0 + 1], cb[:, :, b0:b0 + 1], evk, level)
    assert np.array_equal(to_host(got[1][0])[:, :, b0:b0 + 1], want)


@pytest.mark.parametrize("log_n,ks_inner", [(13, 2), (13, 1), (14, 2), (14, 1), (15, 1)])
def test_levels_batch_equals_single_calls_and_oracle(tf, log_n, ks_inner):
    """tfhe_hmult_levels / tfhe_rotate_levels at the serving shapes (L = 24,
    K = 8, dnum = 3): one batch of eight ciphertexts at levels 24, 1, 9, 17,
    9, 24, 3, 24 (unsorted, groups of one to three) gives, for each, exactly
    what tfhe_hmult / tfhe_rotate gives for it alone, and the oracle's
    result; both inner-product kernels.  An output may alias its input."""
    n = 1 << log_n
    pr, s, evk, k, rk = serving_setup(log_n)
    ctx = tf.CkksContext(log_n, 24, 8, 3, moduli=pr.moduli)
    ctx.plan.set_param("ks_inner", ks_inner)
    levels = [24, 1, 9, 17, 9, 24, 3, 24]
    host_a, host_b = [], []
    for i, lv in enumerate(levels):
        m1 = inputs.small_messages(40 + i, (1, n))
        m2 = inputs.small_messages(40 + i, (1, n), stream=1)
        host_a.append(encrypt(pr, s, m1, lv, 50 + i)[:, :, 0])
        host_b.append(encrypt(pr, s, m2, lv, 70 + i)[:, :, 0])
    A = [to_dev(x) for x in host_a]
    B = [to_dev(x) for x in host_b]
    E, RK = to_dev(evk), to_dev(rk)
    got = [to_host(o) for o in ctx.hmult_levels(A, B, E)]
    rot = [to_host(o) for o in ctx.rotate_levels(A, [RK] * len(A), [k] * len(A))]
    # rotations by two amounts in one batch (one key per ciphertext)
    k2, rk2 = serving_rotation_key(log_n, 3)
    RK2 = to_dev(rk2)
    alt_k = [k if i % 2 else k2 for i in range(len(levels))]
    alt = [to_host(o) for o in ctx.rotate_levels(A, [RK if i % 2 else RK2 for i in range(len(levels))], alt_k)]
    for i in (1, 2):    # one of each amount
        want_r = ckks.rotate(pr, host_a[i][:, :, None], rk if i % 2 else rk2, alt_k[i], levels[i])[:, :, 0]
        assert np.array_equal(alt[i], want_r), (i, levels[i])
    for i, lv in enumerate(levels):
        single_r = to_host(ctx.rotate(A[i][:, :, None].contiguous(), RK if i % 2 else RK2, alt_k[i], lv))[:, :, 0]
        assert np.array_equal(alt[i], single_r), (i, lv)
    for i, lv in enumerate(levels):
        single = to_host(ctx.hmult(A[i][:, :, None].contiguous(), B[i][:, :, None].contiguous(), E, lv))[:, :, 0]
        assert np.array_equal(got[i], single), (i, lv)
        single_r = to_host(ctx.rotate(A[i][:, :, None].contiguous(), RK, k, lv))[:, :, 0]
        assert np.array_equal(rot[i], single_r), (i, lv)
    for i in (0, 1, 2, 6):   # one per distinct level class (full, partial digits)
        lv = levels[i]
        want = ckks.hmult(pr, host_a[i][:, :, None], host_b[i][:, :, None], evk, lv)[:, :, 0]
        assert np.array_equal(got[i], want), (i, lv)
        want_r = ckks.rotate(pr, host_a[i][:, :, None], rk, k, lv)[:, :, 0]
        assert np.array_equal(rot[i], want_r), (i, lv)
    # results written over the first operands
    outs = ctx.hmult_levels(A, B, E, outs=A)
    for i in range(len(levels)):
        assert np.array_equal(to_host(outs[i]), got[i])


def test_levels_batch_errors(tf):
    n = 1 << 10
    pr, s, evk, _ = setup(n, 6, 2, 3)
    ctx = tf.CkksContext(10, 6, 2, 3, moduli=pr.moduli)
    E = to_dev(evk)
    a = [torch.zeros((2, lv, n), dtype=torch.int32, device="cuda") for lv in (6, 3)]
    shared = torch.zeros((2, 6, n), dtype=torch.int32, device="cuda")
    with pytest.raises(tf.TfheError):      # two results in one buffer
        ctx.hmult_levels(a, a, E, outs=[shared, shared.view(-1)[:2 * 3 * n].view(2, 3, n)])
    with pytest.raises(tf.TfheError):      # workspace too small
        ctx.hmult_levels(a, a, E, ws=torch.empty(256, dtype=torch.uint8, device="cuda"))
    with pytest.raises(tf.TfheError):      # level above L
        ctx.levels_workspace_bytes([7])
    with pytest.raises(tf.TfheError):      # even Galois element
        ctx.rotate_levels(a, [E, E], [4, 5])
    assert ctx.hmult_levels([], [], E) == []


@pytest.mark.slow
def test_levels_batch_full_size(tf):
    """N = 2^16, L = 24: a batch at levels 24, 12, 24 equals the single calls,
    and the level-12 result equals the oracle."""
    log_n, n = 16, 1 << 16
    pr, s, evk, _ = setup(n, 24, 8, 3)
    ctx = tf.CkksContext(log_n, 24, 8, 3, moduli=pr.moduli)
    levels = [24, 12, 24]
    ha = [encrypt(pr, s, inputs.small_messages(i, (1, n)), lv, 90 + i)[:, :, 0] for i, lv in enumerate(levels)]
    hb = [encrypt(pr, s, inputs.small_messages(i, (1, n), stream=1), lv, 95 + i)[:, :, 0]
          for i, lv in enumerate(levels)]
    A, B, E = [to_dev(x) for x in ha], [to_dev(x) for x in hb], to_dev(evk)
    got = [to_host(o) for o in ctx.hmult_levels(A, B, E)]
    for i, lv in enumerate(levels):
        single = to_host(ctx.hmult(A[i][:, :, None].contiguous(), B[i][:, :, None].contiguous(), E, lv))[:, :, 0]
        assert np.array_equal(got[i], single), (i, lv)
    want = ckks.hmult(pr, ha[1][:, :, None], hb[1][:, :, None], evk, 12)[:, :, 0]
    assert np.array_equal(got[1], want)


@pytest.mark.parametrize("log_n", [13, 14])
def test_hmult_default_one_pass_at_large_batch(tf, log_n):
    """HMULT at a batch large enough (24 limbs x 24 ciphertexts, at least two
    polynomials per CU) for the library default to put the key switch's plain
    transforms on the one-pass kernel: equal to the all-two-pass HMULT, and
    the first and last ciphertexts equal the oracle."""
    n, level, B = 1 << log_n, 24, 24
    pr, s, evk, _ = setup(n, 24, 8, 3)
    ctx = tf.CkksContext(log_n, 24, 8, 3, moduli=pr.moduli)
    m1 = inputs.small_messages(log_n, (B, n))
    m2 = inputs.small_messages(log_n, (B, n), stream=5)
    ca, cb = encrypt(pr, s, m1, level, 71), encrypt(pr, s, m2, level, 72)
    A, Bt, E = to_dev(ca), to_dev(cb), to_dev(evk)
    assert ctx.plan.get_param("fs_passes") == 0
    auto = to_host(ctx.hmult(A, Bt, E, level))
    ctx.plan.set_param("fs_passes", 2)
    assert np.array_equal(auto, to_host(ctx.hmult(A, Bt, E, level)))
    for b in (0, B - 1):
        want = ckks.hmult(pr, ca[:, :, b:b + 1], cb[:, :, b:b + 1], evk, level)
        assert np.array_equal(auto[:, :, b:b + 1], want), b


@pytest.mark.parametrize("log_n,level,B", [(12, 8, 3), (13, 17, 3), (14, 24, 2), (15, 9, 2)])
def test_hmult_one_pass_transforms_match_oracle(tf, log_n, level, B):
    """HMULT with every transform of the key switch that can take it on the
    one-pass kernel (TFHE_PARAM_FS_PASSES = 1; the ModUp transforms fused
    with the inner product and ModDown's final transform keep their two
    passes) equals the two-pass HMULT and the oracle."""
    n = 1 << log_n
    L = 8 if log_n == 12 else 24
    K, dnum = (4, 2) if log_n == 12 else (8, 3)
    pr, s, evk, _ = setup(n, L, K, dnum)
    ctx = tf.CkksContext(log_n, L, K, dnum, moduli=pr.moduli)
    m1 = inputs.small_messages(log_n, (B, n))
    m2 = inputs.small_messages(log_n, (B, n), stream=3)
    ca, cb = encrypt(pr, s, m1, level, 61), encrypt(pr, s, m2, level, 62)
    A, Bt, E = to_dev(ca), to_dev(cb), to_dev(evk)
    got = {}
    for passes in (1, 2):
        ctx.plan.set_param("fs_passes", passes)
        got[passes] = to_host(ctx.hmult(A, Bt, E, level))
    assert np.array_equal(got[1], got[2])
    assert np.array_equal(got[1], ckks.hmult(pr, ca, cb, evk, level))
