"""RNS CKKS oracle: keys, secret-key encryption, decryption, HMULT and
HROTATE with hybrid (generalised) key switching.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes the operations (Sec. II-B: HMULT, HROTATE; Sec. IV-A,
Table 2: their kernels) and the hybrid key switching it adopts (Sec. II-B,
"Generalized Key-Switching": Q split into dnum slices Q_j of alpha limbs, a
special modulus P larger than every Q_j).  Its algorithm listings are images
that did not survive, so the steps below follow the standard hybrid key
switching the paper cites, in the order the text names them (Sec. IV-A:
Dcomp, ModUp, Inner-product, ModDown), with these readings:

* ct = (c0, c1) with Dec(ct) = c0 + c1*s (mod Q_l); encryption of m is
  c0 = -c1*s + e + Delta*m, c1 uniform.
* L counts the q-limbs, K the p-limbs, alpha = L/dnum; at level l the digits
  are D_j = [alpha*j, min(alpha*(j+1), l)) for j < ceil(l/alpha).
* Dcomp selects the limbs of D_j (no arithmetic).
* ModUp is the fast basis conversion without the Q_j-overflow correction:
  y_i = x_i * [(Q_j/q_i)^{-1}]_{q_i};  x_t = sum_i y_i * [Q_j/q_i]_t  (mod t)
  for each target limb t outside D_j; the D_j limbs keep their own residues.
* The key for s' (s' = s^2 for relinearisation, s' = sigma_k(s) for rotation)
  is evk_j = (b_j, a_j) over all L+K limbs, b_j = -a_j*s + e_j + g_j*s' with
  g_j = [P]_{q_i} on the q-limbs of the full digit D_j and 0 elsewhere.
* Inner product: acc_c = sum_j d~_j o evk_j[c] over the l+K limbs in use.
* ModDown: y_k = [acc_k * (P/p_k)^{-1}]_{p_k} (coefficient domain),
  conv_i = sum_k y_k [P/p_k]_{q_i}, out_i = (acc_i - NTT(conv)_i) * P^{-1},
  with no rounding offset.
* HMULT(ct, ct') = (d0, d1) + KS(d2), d0 = c0c0', d1 = c0c1' + c1c0',
  d2 = c1c1' (NTT domain); no rescale.
* HROTATE(ct, k) = (sigma_k(c0), 0) + KS_k(sigma_k(c1)), the automorphism
  X -> X^k applied here in the coefficient domain.
* RESCALE (Sec. II-B; Table 2: NTT and Ele-Sub) divides by the top modulus
  q_t = q_{l-1} and drops its limb: t = INTT(c_t) taken in [0, q_t), then
  c'_i = (c_i - NTT_i(t mod q_i)) * q_t^{-1} mod q_i for i < l-1, i.e. the
  exact floor(C / q_t) of the CRT value C in [0, Q_l) (no rounding offset).
* CMULT(ct, p) = (c0 o p, c1 o p) and HADD(ct, ct') = (c0 + c0', c1 + c1'),
  element-wise in the NTT domain (Sec. II-B).

Arrays: ciphertexts uint32 [2][level][batch][N] in the NTT domain; keys
uint32 [dnum][2][L+K][N] in the NTT domain, q-limbs first, then p-limbs.
"""
from functools import reduce

import numpy as np

from . import add, mul, ntt_fwd, ntt_inv, ntt_primes, psi as _psi, sub, to_residues


class Params:
    """Moduli and roots.  Default moduli: the L+K largest primes below 2^31
    that are 1 mod 2^17; the K largest are the special primes p_k, the next
    L (descending) are q_0..q_{L-1}."""

    def __init__(self, n, L, K, dnum, moduli=None, prime_two_n=1 << 17):
        if L % dnum:
            raise ValueError("L must be a multiple of dnum")
        self.n, self.L, self.K, self.dnum = n, L, K, dnum
        self.alpha = L // dnum
        if moduli is None:
            primes = ntt_primes(L + K, 31, prime_two_n)
            moduli = primes[K:K + L] + primes[:K]
        self.moduli = [int(m) for m in moduli]
        self.q = self.moduli[:L]
        self.p = self.moduli[L:]
        self.psi = [_psi(m, n) for m in self.moduli]
        self.P = reduce(lambda a, b: a * b, self.p, 1)

    def digits(self, level):
        """Digit limb ranges D_j at this level."""
        out = []
        j = 0
        while self.alpha * j < level:
            out.append(list(range(self.alpha * j, min(self.alpha * (j + 1), level))))
            j += 1
        return out

    def ext_limbs(self, level):
        """Limb indices of the extended basis Q_l * P: q_0..q_{l-1}, p_0..p_{K-1}."""
        return list(range(level)) + list(range(self.L, self.L + self.K))

    def mods(self, idx):
        return [self.moduli[i] for i in idx]

    def psis(self, idx):
        return [self.psi[i] for i in idx]


def _prod(xs):
    return reduce(lambda a, b: a * b, xs, 1)


def _ntt(pr, x, idx):
    return ntt_fwd(x, pr.mods(idx), pr.psis(idx))


def _intt(pr, x, idx):
    return ntt_inv(x, pr.mods(idx), pr.psis(idx))


# --------------------------------------------------------------- automorphism
def automorphism_coeff(x, k, qs):
    """sigma_k on coefficient-domain residues [limbs][...][N]:
    X^i -> X^{i*k mod 2N}, negated when i*k mod 2N >= N."""
    x = np.asarray(x, dtype=np.uint32)
    n = x.shape[-1]
    i = np.arange(n, dtype=np.int64)
    e = (i * k) % (2 * n)
    dest = e % n
    neg = e >= n
    q = np.asarray(qs, dtype=np.uint64).reshape((-1,) + (1,) * (x.ndim - 1))
    xv = x.astype(np.uint64)
    val = np.where(neg, (q - xv) % q, xv)
    out = np.empty_like(xv)
    out[..., dest] = val
    return out.astype(np.uint32)


def automorphism_int(s, k):
    """sigma_k on a signed integer polynomial [N]."""
    s = np.asarray(s, dtype=np.int64)
    n = s.shape[-1]
    i = np.arange(n, dtype=np.int64)
    e = (i * k) % (2 * n)
    out = np.empty_like(s)
    out[..., e % n] = np.where(e >= n, -s, s)
    return out


def galois_element(r, n):
    """Galois element 5^r mod 2N of a slot rotation by r (FrobeniusMap, Sec. IV-A)."""
    return pow(5, r % (n // 2), 2 * n)


# ------------------------------------------------------------------------ keys
def secret_ntt(pr, s, idx=None):
    """NTT of the ternary secret over the limbs idx (default: all L+K)."""
    if idx is None:
        idx = list(range(pr.L + pr.K))
    return _ntt(pr, to_residues(s, pr.mods(idx)), idx)


def switch_key(pr, s, sp_ntt, a_draw, e_draw):
    """Key-switching key from s' (given in the NTT domain over all L+K limbs)
    to s.  a_draw: uniform residues [dnum][L+K][N] (used as NTT-domain
    values); e_draw: small integers [dnum][N].  Returns [dnum][2][L+K][N]."""
    idx = list(range(pr.L + pr.K))
    mods = pr.mods(idx)
    s_ntt = secret_ntt(pr, s)
    key = np.empty((pr.dnum, 2) + s_ntt.shape, dtype=np.uint32)
    for j in range(pr.dnum):
        g = np.zeros((pr.L + pr.K, 1), dtype=np.uint64)
        for i in range(pr.alpha * j, pr.alpha * (j + 1)):
            g[i, 0] = pr.P % pr.q[i]
        a = np.asarray(a_draw[j], dtype=np.uint32)
        e = _ntt(pr, to_residues(e_draw[j], mods), idx)
        gs = mul(np.broadcast_to(g, sp_ntt.shape).astype(np.uint32), sp_ntt, mods)
        b = add(sub(e, mul(a, s_ntt, mods), mods), gs, mods)
        key[j, 0] = b
        key[j, 1] = a
    return key


def relin_key(pr, s, a_draw, e_draw):
    s_ntt = secret_ntt(pr, s)
    s2 = mul(s_ntt, s_ntt, pr.moduli)
    return switch_key(pr, s, s2, a_draw, e_draw)


def rotation_key(pr, s, k, a_draw, e_draw):
    return switch_key(pr, s, secret_ntt(pr, automorphism_int(s, k)), a_draw, e_draw)


# ------------------------------------------------------------ encrypt/decrypt
def encrypt(pr, s, m, c1_draw, e_draw, level, delta=1 << 30):
    """Secret-key encryption of integer messages m [B][N] at `level`;
    c1_draw: uniform residues [level][B][N]; e_draw: small ints [B][N]."""
    idx = list(range(level))
    qs = pr.mods(idx)
    s_ntt = secret_ntt(pr, s, idx)[:, None, :]
    pt = np.asarray(e_draw, np.int64) + delta * np.asarray(m, np.int64)
    pt_ntt = _ntt(pr, to_residues(pt, qs), idx)
    c1 = np.asarray(c1_draw, dtype=np.uint32)
    c0 = sub(pt_ntt, mul(c1, np.broadcast_to(s_ntt, c1.shape), qs), qs)
    return np.stack([c0, c1])


def crt_centered(res, qs):
    """Residues [limbs][...] -> centered integers (object array) mod prod(qs)."""
    Q = _prod(qs)
    acc = np.zeros(res.shape[1:], dtype=object)
    for i, qi in enumerate(qs):
        Qi = Q // qi
        t = (res[i].astype(np.uint64) * np.uint64(pow(Qi % qi, -1, qi))) % np.uint64(qi)
        acc = acc + t.astype(object) * Qi
    acc = acc % Q
    return np.where(acc > Q // 2, acc - Q, acc)


def decrypt(pr, s, ct, level):
    """Centered integer coefficients of c0 + c1*s mod Q_level, [B][N] objects."""
    idx = list(range(level))
    qs = pr.mods(idx)
    s_ntt = secret_ntt(pr, s, idx)[:, None, :]
    c0, c1 = ct[0], ct[1]
    m_ntt = add(c0, mul(c1, np.broadcast_to(s_ntt, c1.shape), qs), qs)
    return crt_centered(_intt(pr, m_ntt, idx), qs)


# ------------------------------------------------------------- key switching
def mod_up(pr, x, digit, level):
    """Fast basis conversion of the coefficient-domain digit limbs x[i], i in
    `digit`, to every limb of Q_level*P outside the digit.  x: [level][B][N].
    Returns coefficient-domain residues over the extended basis with the
    digit's own limbs copied through: [level+K][B][N]."""
    ext = pr.ext_limbs(level)
    Qj = _prod(pr.q[i] for i in digit)
    y = {}
    for i in digit:
        qi = pr.q[i]
        inv = pow((Qj // qi) % qi, -1, qi)
        y[i] = (x[i].astype(np.uint64) * np.uint64(inv)) % np.uint64(qi)
    out = np.empty((len(ext),) + x.shape[1:], dtype=np.uint32)
    for pos, t in enumerate(ext):
        if t in digit:
            out[pos] = x[t]
            continue
        m = pr.moduli[t]
        acc = np.zeros(x.shape[1:], dtype=np.uint64)
        for i in digit:
            c = np.uint64((Qj // pr.q[i]) % m)
            acc = (acc + (y[i] % np.uint64(m)) * c % np.uint64(m)) % np.uint64(m)
        out[pos] = acc.astype(np.uint32)
    return out


def mod_down(pr, acc_ntt, level):
    """(acc - ModUp_P->Q(acc mod P)) * P^{-1} on the q-limbs.
    acc_ntt: NTT domain [level+K][B][N] over Q_level*P.  Returns [level][B][N]."""
    pidx = list(range(pr.L, pr.L + pr.K))
    qidx = list(range(level))
    a_p = _intt(pr, acc_ntt[level:], pidx)
    y = []
    for k, pk in enumerate(pr.p):
        inv = pow((pr.P // pk) % pk, -1, pk)
        y.append((a_p[k].astype(np.uint64) * np.uint64(inv)) % np.uint64(pk))
    conv = np.empty((level,) + acc_ntt.shape[1:], dtype=np.uint32)
    for i in qidx:
        qi = pr.q[i]
        s = np.zeros(acc_ntt.shape[1:], dtype=np.uint64)
        for k, pk in enumerate(pr.p):
            c = np.uint64((pr.P // pk) % qi)
            s = (s + (y[k] % np.uint64(qi)) * c % np.uint64(qi)) % np.uint64(qi)
        conv[i] = s.astype(np.uint32)
    conv_ntt = _ntt(pr, conv, qidx)
    qs = pr.mods(qidx)
    pinv = np.array([pow(pr.P % qi, -1, qi) for qi in qs], dtype=np.uint32)
    diff = sub(acc_ntt[:level], conv_ntt, qs)
    return mul(diff, np.broadcast_to(pinv.reshape(-1, 1, 1), diff.shape), qs)


def key_switch(pr, d_ntt, key, level):
    """Hybrid key switching of d (NTT domain, [level][B][N]) with key
    [dnum][2][L+K][N].  Returns (out0, out1), each [level][B][N]."""
    ext = pr.ext_limbs(level)
    mods_ext = pr.mods(ext)
    x = _intt(pr, d_ntt, list(range(level)))
    acc = [np.zeros((len(ext),) + d_ntt.shape[1:], dtype=np.uint32) for _ in range(2)]
    for j, digit in enumerate(pr.digits(level)):
        up = mod_up(pr, x, digit, level)
        others = [pos for pos, t in enumerate(ext) if t not in digit]
        up_ntt = np.empty_like(up)
        up_ntt[others] = _ntt(pr, up[others], [ext[p] for p in others])
        for i in digit:
            up_ntt[i] = d_ntt[i]
        for c in range(2):
            k = key[j, c][ext][:, None, :]
            acc[c] = add(acc[c], mul(up_ntt, np.broadcast_to(k, up_ntt.shape), mods_ext),
                         mods_ext)
    return mod_down(pr, acc[0], level), mod_down(pr, acc[1], level)


def tensor(pr, ct_a, ct_b, level):
    qs = pr.mods(range(level))
    c0, c1 = ct_a[0], ct_a[1]
    e0, e1 = ct_b[0], ct_b[1]
    d0 = mul(c0, e0, qs)
    d1 = add(mul(c0, e1, qs), mul(c1, e0, qs), qs)
    d2 = mul(c1, e1, qs)
    return d0, d1, d2


def hmult(pr, ct_a, ct_b, evk, level):
    """HMULT (Sec. II-B): (d0, d1) + KeySwitch(d2)."""
    qs = pr.mods(range(level))
    d0, d1, d2 = tensor(pr, ct_a, ct_b, level)
    o0, o1 = key_switch(pr, d2, evk, level)
    return np.stack([add(d0, o0, qs), add(d1, o1, qs)])


def rotate(pr, ct, rk, k, level):
    """HROTATE (Sec. II-B): (sigma_k(c0), 0) + KeySwitch_k(sigma_k(c1))."""
    idx = list(range(level))
    qs = pr.mods(idx)
    r0 = _ntt(pr, automorphism_coeff(_intt(pr, ct[0], idx), k, qs), idx)
    r1 = _ntt(pr, automorphism_coeff(_intt(pr, ct[1], idx), k, qs), idx)
    o0, o1 = key_switch(pr, r1, rk, level)
    return np.stack([add(r0, o0, qs), o1])


def rescale(pr, ct, level):
    """RESCALE (Sec. II-B, Table 2): ct [2][level][B][N] (NTT domain) at
    `level` >= 2 -> [2][level-1][B][N], dividing by q_{level-1}."""
    if level < 2:
        raise ValueError("rescale needs level >= 2")
    top = level - 1
    qt = pr.q[top]
    idx = list(range(top))
    qs = pr.mods(idx)
    out = np.empty((2, top) + ct.shape[2:], dtype=np.uint32)
    for c in range(2):
        t = _intt(pr, ct[c][top:top + 1], [top])[0].astype(np.uint64)  # [B][N] in [0, q_t)
        t_mod = np.stack([(t % np.uint64(qi)).astype(np.uint32) for qi in qs])
        diff = sub(ct[c][:top], _ntt(pr, t_mod, idx), qs)
        qinv = np.array([pow(qt % qi, -1, qi) for qi in qs], dtype=np.uint32).reshape(-1, 1, 1)
        out[c] = mul(diff, np.broadcast_to(qinv, diff.shape), qs)
    return out


def cmult(pr, ct, pt, level):
    """CMULT (Sec. II-B): (c0 o p, c1 o p); pt [level][B][N], NTT domain."""
    qs = pr.mods(range(level))
    return np.stack([mul(ct[0], pt, qs), mul(ct[1], pt, qs)])


def hadd(pr, ct_a, ct_b, level):
    """HADD (Sec. II-B): component-wise addition."""
    qs = pr.mods(range(level))
    return np.stack([add(ct_a[0], ct_b[0], qs), add(ct_a[1], ct_b[1], qs)])


def negacyclic_int(a, b):
    """Exact negacyclic product of integer polynomials [..., N] via
    numpy.convolve (int64) folded with X^N = -1."""
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    n = a.shape[-1]
    full = np.convolve(a, b)
    out = full[:n].copy()
    out[: n - 1] -= full[n:]
    return out
