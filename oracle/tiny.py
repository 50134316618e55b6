"""Pure-Python (arbitrary-precision int) references for tiny sizes.

TEST INFRASTRUCTURE ONLY.  These share no code with oracle.c: they exist to
pin it.  Each evaluates a definition directly with Python integers.
"""


def is_prime_mr(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (bases 2..41)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def multiplicative_order(g, q):
    """Order of g mod q by walking its powers (small q only)."""
    x, k = g % q, 1
    while x != 1:
        x = x * g % q
        k += 1
    return k


def horner(a, x, q):
    """a(x) mod q by Horner's rule."""
    acc = 0
    for c in reversed(a):
        acc = (acc * x + c) % q
    return acc


def ntt_eq4(a, q, psi):
    """Eq. (4): A_k = sum_n a_n psi^{2nk+n} mod q, each power from pow()."""
    n = len(a)
    return [sum(a[j] * pow(psi, 2 * j * k + j, q) for j in range(n)) % q for k in range(n)]


def intt_eq4(A, q, psi):
    """Inverse of Eq. (4): a_n = N^{-1} psi^{-n} sum_k A_k psi^{-2nk} mod q
    (Eq. (2) with the psi^{-n} post-twist of Eq. (3))."""
    n = len(A)
    ninv = pow(n, -1, q)
    pinv = pow(psi, -1, q)
    return [ninv * pow(pinv, j, q) * sum(A[k] * pow(pinv, 2 * j * k, q) for k in range(n)) % q
            for j in range(n)]


def negacyclic_schoolbook(a, b, q=None):
    """Product in Z[X]/(X^N+1) (reduced mod q when q is given)."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    if q is not None:
        c = [x % q for x in c]
    return c


def crt(residues, moduli):
    """The unique x in [0, prod(moduli)) with x = r_i mod m_i, by Garner's
    mixed-radix recurrence (not the CRT-basis sum the oracle uses)."""
    x, m = 0, 1
    for r, mi in zip(residues, moduli):
        v = ((r - x) % mi) * pow(m % mi, -1, mi) % mi
        x += v * m
        m *= mi
    return x
