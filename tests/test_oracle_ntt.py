"""Pins of the oracle's primes, roots and NTT against what the paper and the
mathematics fix (CPU only)."""
import os
import random

import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_2212_14191_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_pairs(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            out.append([int(x) for x in line.split()])
    return out


def _read_kv(name):
    d = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            k, *v = line.split()
            d[k] = [int(x) for x in v]
    return d


# ------------------------------------------------------------------ primes
def test_is_prime_matches_miller_rabin():
    rnd = random.Random(5)
    cands = list(range(0, 2000)) + [561, 1105, 1729, 2465, 2821, 6601, 8911, 41041,
                                    2147483647, 2147483649, 4294967291, 4294967295]
    cands += [rnd.randrange(2 ** 29, 2 ** 32) for _ in range(300)]
    for n in cands:
        assert oracle.is_prime(n) == tiny.is_prime_mr(n), n


@pytest.mark.parametrize("q,g", [tuple(p) for p in _read_pairs("primitive_roots.txt")])
def test_primitive_root_published(q, g):
    assert oracle.primitive_root(q) == g


@pytest.mark.parametrize("q", [17, 97, 257, 7681, 12289, 40961, 65537])
def test_primitive_root_bruteforce(q):
    g = oracle.primitive_root(q)
    assert tiny.multiplicative_order(g, q) == q - 1
    for h in range(2, g):
        assert tiny.multiplicative_order(h, q) < q - 1


@pytest.mark.parametrize("q,n", [(17, 8), (97, 16), (7681, 256), (12289, 1024), (65537, 4096)])
def test_psi_is_primitive_2n_root(q, n):
    s = oracle.psi(q, n)
    assert tiny.multiplicative_order(s, q) == 2 * n
    assert pow(s, n, q) == q - 1


def test_psi_rejects_bad_modulus():
    with pytest.raises(ValueError):
        oracle.psi(7681, 8192)          # 2N does not divide q-1
    with pytest.raises(ValueError):
        oracle.psi(7681 * 3, 16)        # not prime


def test_ntt_primes_rule():
    two_n = 1 << 17
    ps = oracle.ntt_primes(44, 31, two_n)
    assert len(set(ps)) == 44 and ps == sorted(ps, reverse=True)
    # every candidate = 1 mod 2^17 between 2^31 and the last one is listed iff prime
    cand = ((1 << 31) - 1) // two_n * two_n + 1
    listed = []
    while cand >= ps[-1]:
        if tiny.is_prime_mr(cand):
            listed.append(cand)
        cand -= two_n
    assert listed == ps
    for q in ps:
        assert q < 2 ** 31 and q % two_n == 1


# --------------------------------------------------------------------- NTT
def test_hand_worked_example():
    d = _read_kv("ntt_q17_n4.txt")
    q, psi = d["q"][0], d["psi"][0]
    assert oracle.psi(q, d["n"][0]) == psi
    a = np.array(d["a"], dtype=np.uint32)
    assert list(oracle.ntt_direct(a, q, psi)) == d["A"]
    assert list(oracle.ntt_radix2_single(a, q, psi)) == d["A"]
    assert list(oracle.ntt_radix2_single(np.array(d["A"], np.uint32), q, psi, True)) == d["a"]


SMALL = [(17, 4), (97, 8), (7681, 16), (12289, 32), (2147352577, 64)]


@pytest.mark.parametrize("q,n", SMALL)
def test_direct_matches_python_eq4(q, n):
    s = oracle.psi(q, n)
    a = inputs.uniform_residues(0, [q], n)[0]
    assert list(oracle.ntt_direct(a, q, s)) == tiny.ntt_eq4([int(x) for x in a], q, s)
    A = inputs.uniform_residues(1, [q], n)[0]
    assert list(oracle.ntt_direct(A, q, s, True)) == tiny.intt_eq4([int(x) for x in A], q, s)


@pytest.mark.parametrize("logn", range(1, 11))
def test_radix2_matches_direct(logn):
    n = 1 << logn
    for q in (oracle.ntt_primes(1, 30, 1 << 13)[0], oracle.ntt_primes(1, 31, 1 << 17)[0]):
        s = oracle.psi(q, n)
        a = inputs.uniform_residues(logn, [q], n)[0]
        assert np.array_equal(oracle.ntt_radix2_single(a, q, s), oracle.ntt_direct(a, q, s))
        assert np.array_equal(oracle.ntt_radix2_single(a, q, s, True),
                              oracle.ntt_direct(a, q, s, True))


@pytest.mark.parametrize("logn", [12, 16])
def test_horner_evaluation_points(logn):
    """A_k = a(psi^{2k+1}) at sampled k (Eq. 4 read as evaluation)."""
    n = 1 << logn
    qs = oracle.ntt_primes(3, 31, 1 << 17)
    psis = [oracle.psi(q, n) for q in qs]
    a = inputs.uniform_residues(7, qs, (2, n))
    A = oracle.ntt_fwd(a, qs, psis)
    rnd = random.Random(logn)
    for l, q in enumerate(qs):
        for b in range(2):
            coeffs = [int(x) for x in a[l, b]]
            for k in [0, n - 1] + [rnd.randrange(n) for _ in range(6)]:
                x = pow(psis[l], 2 * k + 1, q)
                assert int(A[l, b, k]) == tiny.horner(coeffs, x, q)


@pytest.mark.parametrize("logn", [4, 12, 16])
def test_closed_forms(logn):
    n = 1 << logn
    q = oracle.ntt_primes(1, 31, 1 << 17)[0]
    s = oracle.psi(q, n)
    k = np.arange(n, dtype=object)
    delta0 = np.zeros(n, np.uint32)
    delta0[0] = 1
    assert np.all(oracle.ntt_fwd(delta0, [q], [s]) == 1)
    for m, c in [(1, 1), (3, 12345), (n - 1, q - 1)]:
        x = np.zeros(n, np.uint32)
        x[m] = c
        want = [c * pow(s, (2 * kk + 1) * m, q) % q for kk in range(n)]
        assert list(oracle.ntt_fwd(x, [q], [s])) == want
    # X^{N-1} * X = X^N = -1 in Z_q[X]/(X^N+1)
    x1 = np.zeros(n, np.uint32)
    x1[1] = 1
    xn1 = np.zeros(n, np.uint32)
    xn1[n - 1] = 1
    prod = oracle.mul(oracle.ntt_fwd(x1, [q], [s]), oracle.ntt_fwd(xn1, [q], [s]), [q])
    c = oracle.ntt_inv(prod, [q], [s])
    assert c[0] == q - 1 and np.all(c[1:] == 0)
    del k


def test_round_trip_and_linearity():
    """INTT(NTT(x)) = x, the paper's own correctness check (Sec. VI-A)."""
    n = 1 << 16
    qs = oracle.ntt_primes(4, 31, 1 << 17)
    psis = [oracle.psi(q, n) for q in qs]
    x = inputs.uniform_residues(0, qs, (3, n))
    y = inputs.uniform_residues(1, qs, (3, n))
    X, used = oracle.ntt(x, qs, psis)
    assert used >= 1
    assert np.array_equal(oracle.ntt_inv(X, qs, psis), x)
    Y = oracle.ntt_fwd(y, qs, psis)
    assert np.array_equal(oracle.ntt_fwd(oracle.add(x, y, qs), qs, psis), oracle.add(X, Y, qs))


def test_batch_equals_single():
    n = 256
    qs = oracle.ntt_primes(3, 30, 1 << 13)
    psis = [oracle.psi(q, n) for q in qs]
    x = inputs.uniform_residues(3, qs, (4, n))
    X = oracle.ntt_fwd(x, qs, psis)
    for l in range(3):
        for b in range(4):
            assert np.array_equal(X[l, b], oracle.ntt_direct(x[l, b], qs[l], psis[l]))


@pytest.mark.parametrize("n", [4, 16, 64])
def test_schoolbook_matches_python(n):
    q = 7681 if n <= 256 else 12289
    a = inputs.uniform_residues(0, [q], n)[0]
    b = inputs.uniform_residues(1, [q], n)[0]
    c, _ = oracle.negacyclic_mul(a, b, [q])
    assert list(c) == tiny.negacyclic_schoolbook([int(x) for x in a], [int(x) for x in b], q)


def test_convolution_theorem_config1_shape():
    """Eq. (3): INTT(NTT(a) o NTT(b)) is the negacyclic product (N=2^12,
    4 limbs of 30-bit primes, 8 polynomial pairs)."""
    n = 1 << 12
    qs = oracle.ntt_primes(4, 30, 2 * n)
    psis = [oracle.psi(q, n) for q in qs]
    a = inputs.uniform_residues(0, qs, (8, n))
    b = inputs.uniform_residues(0, qs, (8, n), stream=1)
    c = oracle.ntt_inv(oracle.mul(oracle.ntt_fwd(a, qs, psis), oracle.ntt_fwd(b, qs, psis), qs),
                       qs, psis)
    ref, _ = oracle.negacyclic_mul(a, b, qs)
    assert np.array_equal(c, ref)
