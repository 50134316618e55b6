"""Plain CPU oracle for the TensorFHE (arXiv 2212.14191) NTT / HMULT path.

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
CPU-baseline leg of the benchmark are the only callers.  The product library
never imports, links or calls anything in this package, and this package
imports nothing from the product: the two share no code, tables or constants.
Random draws (uniform residues, secrets, errors, messages) come in as inputs.

Layout conventions (the (L, B, N) batching layout of Sec. IV-D):
  a residue array is uint32 [limbs][batch][N], canonical in [0, q).

Modules:
  oracle          (this file)  ctypes binding of oracle.c: primes, roots,
                  direct O(N^2) NTT (Eq. 4), radix-2 NTT (Sec. II-A, Fig. 2),
                  schoolbook negacyclic product; numpy element-wise ops.
  oracle.ckks     RNS CKKS: keys, encryption, decryption, HMULT, rotation
                  (Sec. II-B, Sec. IV-A), hybrid key switching.
  oracle.tiny     pure-Python (big-int) references for tiny sizes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile oracle.c with gcc into liboracle.so (next to this file)."""
    import subprocess
    src = os.path.join(_HERE, "oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, _LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        p = ctypes.c_void_p
        L.or_is_prime.argtypes = [u64]
        L.or_is_prime.restype = i32
        L.or_primitive_root.argtypes = [u64, ctypes.POINTER(u64)]
        L.or_primitive_root.restype = i32
        L.or_psi.argtypes = [u64, u32, ctypes.POINTER(u64)]
        L.or_psi.restype = i32
        L.or_ntt_direct.argtypes = [u32, u64, u64, p, p, i32]
        L.or_ntt_direct.restype = None
        L.or_ntt_radix2.argtypes = [u32, u64, u64, p, p, i32]
        L.or_ntt_radix2.restype = None
        L.or_ntt_batch.argtypes = [u32, u32, u32, p, p, p, p, i32, i32]
        L.or_ntt_batch.restype = i32
        L.or_negacyclic_schoolbook.argtypes = [u32, u64, p, p, p]
        L.or_negacyclic_schoolbook.restype = None
        L.or_negacyclic_batch.argtypes = [u32, u32, u32, p, p, p, p, i32]
        L.or_negacyclic_batch.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- primes / roots
def is_prime(q):
    return bool(lib().or_is_prime(int(q)))


def primitive_root(q):
    """Smallest primitive root of the prime q (Sec. II-A)."""
    g = ctypes.c_uint64()
    if lib().or_primitive_root(int(q), ctypes.byref(g)) != 0:
        raise ValueError(f"{q} is not a prime below 2^32")
    return g.value


def psi(q, n):
    """psi = g^{(q-1)/2N} for the smallest primitive root g (Sec. II-A)."""
    r = ctypes.c_uint64()
    if lib().or_psi(int(q), int(n), ctypes.byref(r)) != 0:
        raise ValueError(f"no primitive 2N-th root: q={q}, N={n}")
    return r.value


def ntt_primes(count, bits, two_n):
    """The `count` largest primes q < 2^bits with q = 1 (mod two_n), in
    descending order (the prime-selection reading adopted for the paper's
    unspecified moduli)."""
    out = []
    q = ((1 << bits) - 1) // two_n * two_n + 1
    if q >= (1 << bits):
        q -= two_n
    while len(out) < count and q > two_n:
        if is_prime(q):
            out.append(q)
        q -= two_n
    if len(out) < count:
        raise ValueError("not enough primes")
    return out


# ------------------------------------------------------------------------- NTT
def _as_limb_array(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.ndim == 1:
        x = x.reshape(1, 1, -1)
    elif x.ndim == 2:
        x = x.reshape(x.shape[0], 1, x.shape[1])
    return x


def ntt(x, qs, psis, inverse=False, threads=0):
    """Radix-2 negacyclic NTT (Eq. 4) or its inverse over [limbs][batch][N],
    natural order in and out.  Returns (result, threads_used)."""
    shape = np.shape(x)
    a = _as_limb_array(x)
    limbs, batch, n = a.shape
    q = np.ascontiguousarray(np.asarray(qs, dtype=np.uint64).reshape(-1)[:limbs])
    s = np.ascontiguousarray(np.asarray(psis, dtype=np.uint64).reshape(-1)[:limbs])
    assert q.size == limbs and s.size == limbs
    out = np.empty_like(a)
    used = lib().or_ntt_batch(n, limbs, batch, _ptr(q), _ptr(s), _ptr(a), _ptr(out),
                              1 if inverse else 0, int(threads))
    return out.reshape(shape), used


def ntt_fwd(x, qs, psis, threads=0):
    return ntt(x, qs, psis, False, threads)[0]


def ntt_inv(x, qs, psis, threads=0):
    return ntt(x, qs, psis, True, threads)[0]


def ntt_direct(a, q, psi_, inverse=False):
    """O(N^2) evaluation of Eq. (4) (or the inverse sum) for one polynomial."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    out = np.empty_like(a)
    lib().or_ntt_direct(a.size, int(q), int(psi_), _ptr(a), _ptr(out), 1 if inverse else 0)
    return out


def ntt_radix2_single(a, q, psi_, inverse=False):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    out = np.empty_like(a)
    lib().or_ntt_radix2(a.size, int(q), int(psi_), _ptr(a), _ptr(out), 1 if inverse else 0)
    return out


def negacyclic_mul(a, b, qs, threads=0):
    """Schoolbook product in Z_q[X]/(X^N+1) over [limbs][batch][N]."""
    shape = np.shape(a)
    A = _as_limb_array(a)
    B = _as_limb_array(b)
    limbs, batch, n = A.shape
    q = np.ascontiguousarray(np.asarray(qs, dtype=np.uint64).reshape(-1)[:limbs])
    out = np.empty_like(A)
    used = lib().or_negacyclic_batch(n, limbs, batch, _ptr(q), _ptr(A), _ptr(B), _ptr(out),
                                     int(threads))
    return out.reshape(shape), used


# ---------------------------------------------------------- element-wise (numpy)
def _qcol(qs, ndim):
    q = np.asarray(qs, dtype=np.uint64).reshape(-1)
    return q.reshape((-1,) + (1,) * (ndim - 1))


def mul(a, b, qs):
    """Hada-Mult: (a o b) mod q per limb (Sec. IV-A)."""
    q = _qcol(qs, np.ndim(a))
    return ((np.asarray(a, np.uint64) * np.asarray(b, np.uint64)) % q).astype(np.uint32)


def add(a, b, qs):
    """Ele-Add: (a + b) mod q per limb."""
    q = _qcol(qs, np.ndim(a))
    return ((np.asarray(a, np.uint64) + np.asarray(b, np.uint64)) % q).astype(np.uint32)


def sub(a, b, qs):
    """Ele-Sub: (a - b) mod q per limb."""
    q = _qcol(qs, np.ndim(a))
    return ((np.asarray(a, np.uint64) + q - np.asarray(b, np.uint64)) % q).astype(np.uint32)


def to_residues(x, qs):
    """Signed integers (any int array) -> canonical residues [limbs][...]."""
    x = np.asarray(x, dtype=np.int64)
    q = np.asarray(qs, dtype=np.int64).reshape((-1,) + (1,) * x.ndim)
    return np.mod(x[None, ...], q).astype(np.uint32)
