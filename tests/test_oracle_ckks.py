"""Pins of the RNS CKKS oracle (key switching, HMULT, rotation) against
invariants and exact decryption (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import ckks, tiny
from paper_2212_14191_amd import inputs


def small_params(n=64):
    return ckks.Params(n, L=6, K=2, dnum=3)


def make_keys(pr, h=None):
    n = pr.n
    s = inputs.ternary_secret(1, n, h or min(192, n // 2))
    a = inputs.uniform_residues(1, pr.moduli, (pr.dnum, n), stream=1).transpose(1, 0, 2)
    e = inputs.gaussian_error(2, (pr.dnum, n), stream=1)
    return s, a, e


def enc(pr, s, m, level, seed):
    b = m.shape[0]
    c1 = inputs.uniform_residues(seed, pr.mods(range(level)), (b, pr.n), stream=5)
    e = inputs.gaussian_error(2, (b, pr.n), stream=seed + 10)
    return ckks.encrypt(pr, s, m, c1, e, level)


def test_digits_and_prime_order():
    pr = ckks.Params(64, L=24, K=8, dnum=3)
    assert pr.alpha == 8
    assert pr.digits(24) == [list(range(0, 8)), list(range(8, 16)), list(range(16, 24))]
    assert pr.digits(9) == [list(range(0, 8)), [8]]
    assert min(pr.p) > max(pr.q)
    for j in range(3):
        Qj = 1
        for i in range(8 * j, 8 * j + 8):
            Qj *= pr.q[i]
        assert pr.P > Qj


def test_mod_up_is_lift_plus_small_multiple():
    """ModUp gives lift([x]_{Q_j}) + u*Q_j on every target, one u in [0, |D_j|)."""
    pr = small_params(16)
    level = 5
    x = inputs.uniform_residues(0, pr.mods(range(level)), (2, pr.n))
    ext = pr.ext_limbs(level)
    for digit in pr.digits(level):
        up = ckks.mod_up(pr, x, digit, level)
        Qj = 1
        for i in digit:
            Qj *= pr.q[i]
        for b in range(2):
            for c in range(pr.n):
                lift = tiny.crt([int(x[i, b, c]) for i in digit], [pr.q[i] for i in digit])
                us = set()
                for pos, t in enumerate(ext):
                    m = pr.moduli[t]
                    r = int(up[pos, b, c])
                    if t in digit:
                        assert r == int(x[t, b, c])
                        continue
                    u = next(u for u in range(len(digit)) if (lift + u * Qj) % m == r)
                    us.add(u)
                assert len(us) == 1


def test_mod_down_divides_by_p():
    """ModDown(P*x + r) = x - u with u in [0, K) for 0 <= r < P."""
    pr = small_params(16)
    level = 4
    ext = pr.ext_limbs(level)
    rng = np.random.default_rng(3)
    xs = [[int(v) for v in rng.integers(0, 2 ** 62, size=pr.n)] for _ in range(2)]
    rs = [[int(v) % pr.P for v in rng.integers(0, 2 ** 62, size=pr.n)] for _ in range(2)]
    a = np.empty((len(ext), 2, pr.n), np.uint32)
    for pos, t in enumerate(ext):
        m = pr.moduli[t]
        for b in range(2):
            a[pos, b] = [(pr.P * xs[b][c] + rs[b][c]) % m for c in range(pr.n)]
    a_ntt = oracle.ntt_fwd(a, pr.mods(ext), pr.psis(ext))
    out = oracle.ntt_inv(ckks.mod_down(pr, a_ntt, level), pr.mods(range(level)),
                         pr.psis(range(level)))
    Q = 1
    for i in range(level):
        Q *= pr.q[i]
    for b in range(2):
        for c in range(pr.n):
            v = tiny.crt([int(out[i, b, c]) for i in range(level)], pr.q[:level])
            assert (xs[b][c] - v) % Q in range(pr.K)


def test_gadget_identity():
    """sum_j ModUp(d)_j * g_j = P*d over Q_l*P (g_j = P on the digit, else 0)."""
    pr = small_params(16)
    level = 5
    ext = pr.ext_limbs(level)
    d = inputs.uniform_residues(4, pr.mods(range(level)), (1, pr.n))
    total = np.zeros((len(ext), 1, pr.n), np.uint64)
    for digit in pr.digits(level):
        up = ckks.mod_up(pr, d, digit, level)
        for pos, t in enumerate(ext):
            if t in digit:
                m = pr.moduli[t]
                total[pos] = (total[pos] + up[pos].astype(np.uint64) * (pr.P % m)) % m
    for pos, t in enumerate(ext):
        m = pr.moduli[t]
        want = (d[t].astype(np.uint64) * (pr.P % m)) % m if t < level else np.zeros_like(total[pos])
        assert np.array_equal(total[pos], want)


def test_switch_key_hides_small_error():
    pr = small_params(64)
    s, a, e = make_keys(pr)
    evk = ckks.relin_key(pr, s, a, e)
    idx = list(range(pr.L + pr.K))
    s_ntt = ckks.secret_ntt(pr, s)
    s2 = oracle.mul(s_ntt, s_ntt, pr.moduli)
    for j in range(pr.dnum):
        g = np.zeros((len(idx), 1), np.uint32)
        for i in range(2 * j, 2 * j + 2):
            g[i] = pr.P % pr.q[i]
        lhs = oracle.add(evk[j, 0], oracle.mul(evk[j, 1], s_ntt, pr.moduli), pr.moduli)
        lhs = oracle.sub(lhs, oracle.mul(np.broadcast_to(g, s2.shape), s2, pr.moduli), pr.moduli)
        coef = oracle.ntt_inv(lhs, pr.moduli, pr.psi)
        assert np.array_equal(coef, oracle.to_residues(e[j], pr.moduli))


def test_encrypt_decrypt_exact():
    pr = small_params(64)
    s, _, _ = make_keys(pr)
    m = inputs.small_messages(0, (2, pr.n))
    ct = enc(pr, s, m, 4, 1)
    dec = ckks.decrypt(pr, s, ct, 4)
    e = inputs.gaussian_error(2, (2, pr.n), stream=11)
    assert np.array_equal(dec.astype(np.int64), (1 << 30) * m.astype(np.int64) + e)


def test_hmult_trivial_ciphertexts_exact():
    """c1 = c1' = 0 gives KeySwitch(0) = 0 and (c0 * c0', 0) exactly."""
    pr = small_params(64)
    s, a, e = make_keys(pr)
    evk = ckks.relin_key(pr, s, a, e)
    level = 5
    qs = pr.mods(range(level))
    ps = pr.psis(range(level))
    x = inputs.uniform_residues(0, qs, (2, pr.n))
    y = inputs.uniform_residues(1, qs, (2, pr.n))
    zero = np.zeros_like(x)
    cta = np.stack([oracle.ntt_fwd(x, qs, ps), zero])
    ctb = np.stack([oracle.ntt_fwd(y, qs, ps), zero])
    out = ckks.hmult(pr, cta, ctb, evk, level)
    assert np.all(out[1] == 0)
    got = oracle.ntt_inv(out[0], qs, ps)
    for i in range(level):
        for b in range(2):
            want = tiny.negacyclic_schoolbook([int(v) for v in x[i, b]], [int(v) for v in y[i, b]],
                                              qs[i])
            assert list(got[i, b]) == want


def _check_hmult_decrypts(pr, level, batch=2):
    s, a, e = make_keys(pr)
    evk = ckks.relin_key(pr, s, a, e)
    m1 = inputs.small_messages(0, (batch, pr.n))
    m2 = inputs.small_messages(0, (batch, pr.n), stream=1)
    out = ckks.hmult(pr, enc(pr, s, m1, level, 1), enc(pr, s, m2, level, 2), evk, level)
    dec = ckks.decrypt(pr, s, out, level)
    delta2 = 1 << 60
    for b in range(batch):
        want = ckks.negacyclic_int(m1[b], m2[b])
        got = np.array([(int(v) + delta2 // 2) // delta2 for v in dec[b]], dtype=np.int64)
        assert np.array_equal(got, want)
        noise = max(abs(int(v) - delta2 * int(w)) for v, w in zip(dec[b], want))
        assert noise < delta2 // 2 ** 4


@pytest.mark.parametrize("level", [6, 5, 3])
def test_hmult_decrypts_to_product(level):
    _check_hmult_decrypts(small_params(1024), level)


@pytest.mark.slow
def test_hmult_decrypts_to_product_full_size():
    """N = 2^16, L = 24, K = 8, dnum = 3, h = 192, one pair, level 24."""
    _check_hmult_decrypts(ckks.Params(1 << 16, L=24, K=8, dnum=3), 24, batch=1)


def test_automorphism_is_ntt_permutation():
    """sigma_k in the coefficient domain = index map pi(j) = ((2j+1)k mod 2N - 1)/2
    on the evaluation points psi^{2j+1}."""
    pr = small_params(64)
    n = pr.n
    k = ckks.galois_element(3, n)
    qs = pr.mods(range(2))
    ps = pr.psis(range(2))
    x = inputs.uniform_residues(0, qs, (1, n))
    lhs = oracle.ntt_fwd(ckks.automorphism_coeff(x, k, qs), qs, ps)
    j = np.arange(n)
    pi = (((2 * j + 1) * k) % (2 * n) - 1) // 2
    assert np.array_equal(lhs, oracle.ntt_fwd(x, qs, ps)[..., pi])
    # definition check on integers: X^i -> X^{ik}, X^N = -1
    si = np.arange(n) - n // 2
    got = ckks.automorphism_int(si, k)
    want = [0] * n
    for i in range(n):
        e = i * k % (2 * n)
        want[e % n] = si[i] if e < n else -si[i]
    assert list(got) == want


@pytest.mark.parametrize("which", ["rot5", "conj"])
def test_rotate_decrypts_to_rotated_message(which):
    """Rotation by 5^5 and conjugation (X -> X^{2N-1}, i.e. X^i -> -X^{N-i})
    decrypt to the automorphism of the message."""
    pr = small_params(1024)
    level = 4
    s, a, e = make_keys(pr)
    k = ckks.galois_element(5, pr.n) if which == "rot5" else 2 * pr.n - 1
    rk = ckks.rotation_key(pr, s, k, a, e)
    m = inputs.small_messages(0, (2, pr.n))
    out = ckks.rotate(pr, enc(pr, s, m, level, 1), rk, k, level)
    dec = ckks.decrypt(pr, s, out, level)
    delta = 1 << 30
    for b in range(2):
        got = np.array([(int(v) + delta // 2) // delta for v in dec[b]], dtype=np.int64)
        assert np.array_equal(got, ckks.automorphism_int(m[b], k))
        if which == "conj":  # closed form of X -> X^{-1} on Z[X]/(X^N + 1)
            want = np.concatenate([m[b][:1], -m[b][:0:-1]])
            assert np.array_equal(got, want)


# ------------------------------------------------------------------ RESCALE
@pytest.mark.parametrize("level", [2, 4, 6])
def test_rescale_is_floor_division_by_top_modulus(level):
    """Coefficient-wise, RESCALE is floor(C / q_{l-1}) of the CRT value C in
    [0, Q_l) (Garner CRT in Python integers), reduced mod each q_i, i < l-1."""
    pr = small_params(32)
    idx = list(range(level))
    qs, ps = pr.mods(idx), pr.psis(idx)
    ct = np.stack([inputs.uniform_residues(40 + c, qs, (2, pr.n)) for c in range(2)])
    got = ckks.rescale(pr, ct, level)
    assert got.shape == (2, level - 1, 2, pr.n)
    qt = qs[-1]
    for c in range(2):
        coef = oracle.ntt_inv(ct[c], qs, ps)
        got_coef = oracle.ntt_inv(got[c], qs[:-1], ps[:-1])
        for b in range(2):
            for k in range(pr.n):
                C = tiny.crt([int(coef[i, b, k]) for i in range(level)], qs)
                want = C // qt
                assert [int(got_coef[i, b, k]) for i in range(level - 1)] == [want % q for q in qs[:-1]]


@pytest.mark.parametrize("level", [6, 3])
def test_rescale_decrypts_to_scaled_message(level):
    """Dec(RESCALE(ct)) = Dec(ct) / q_{l-1} up to |r0 + r1 s| / q_{l-1} <= 1 + h
    (r0, r1 in [0, q_{l-1}) are the dropped residues, h the secret's weight)."""
    pr = small_params(256)
    s, _, _ = make_keys(pr)
    h = int(np.count_nonzero(s))
    m = inputs.small_messages(0, (2, pr.n))
    ct = enc(pr, s, m, level, 3)
    dec = ckks.decrypt(pr, s, ct, level)
    dec2 = ckks.decrypt(pr, s, ckks.rescale(pr, ct, level), level - 1)
    qt = pr.q[level - 1]
    err = max(abs(int(d2) * qt - int(d)) for d, d2 in zip(dec.ravel(), dec2.ravel()))
    assert err <= (1 + h) * qt
    assert err > 0  # the division is not exact for these inputs


def test_rescale_after_hmult_recovers_product():
    """HMULT then RESCALE: Delta^2 m1 m2 / q_{l-1} rounds back to m1*m2 at the
    new scale Delta^2 / q_{l-1}."""
    pr = small_params(256)
    s, a, e = make_keys(pr)
    evk = ckks.relin_key(pr, s, a, e)
    level = 6
    m1 = inputs.small_messages(0, (1, pr.n))
    m2 = inputs.small_messages(0, (1, pr.n), stream=1)
    out = ckks.hmult(pr, enc(pr, s, m1, level, 1), enc(pr, s, m2, level, 2), evk, level)
    dec = ckks.decrypt(pr, s, ckks.rescale(pr, out, level), level - 1)
    scale = (1 << 60) / pr.q[level - 1]
    want = ckks.negacyclic_int(m1[0], m2[0])
    got = np.array([round(int(v) / scale) for v in dec[0]], dtype=np.int64)
    assert np.array_equal(got, want)


def test_cmult_and_hadd_decrypt_exactly():
    """CMULT by a plaintext p (NTT of a small integer polynomial) decrypts to
    p * (Delta m + e) exactly; HADD to the sum of the two decryptions."""
    pr = small_params(64)
    s, _, _ = make_keys(pr)
    level = 4
    idx = list(range(level))
    qs, ps = pr.mods(idx), pr.psis(idx)
    m1 = inputs.small_messages(0, (2, pr.n))
    m2 = inputs.small_messages(0, (2, pr.n), stream=1)
    c1, c2 = enc(pr, s, m1, level, 1), enc(pr, s, m2, level, 2)
    d1, d2 = ckks.decrypt(pr, s, c1, level), ckks.decrypt(pr, s, c2, level)
    dsum = ckks.decrypt(pr, s, ckks.hadd(pr, c1, c2, level), level)
    assert np.array_equal(dsum.astype(np.int64), d1.astype(np.int64) + d2.astype(np.int64))
    p = inputs.small_messages(7, (2, pr.n))
    pt = oracle.ntt_fwd(oracle.to_residues(p, qs), qs, ps)
    dprod = ckks.decrypt(pr, s, ckks.cmult(pr, c1, pt, level), level)
    for b in range(2):
        want = [sum(int(d1[b, i]) * int(p[b, (k - i) % pr.n]) * (1 if i <= k else -1) for i in range(pr.n))
                for k in range(pr.n)]
        assert [int(v) for v in dprod[b]] == want
