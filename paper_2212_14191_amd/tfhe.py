"""Thin ctypes binding of libtfhe.so (include/tfhe.h).

Every compute step runs in the library's HIP kernels; this module only
marshals arguments.  Device memory and streams come from PyTorch: residue
arrays are torch tensors of dtype int32 (bit-identical to the uint32 the ABI
takes) on the current HIP device, in the (limb, batch, N) layout.

The functions named like the C entry points (tfhe_ntt_fwd, ...) take raw
pointers; the classes NttPlan and CkksContext wrap them for tensors.  Loading
fails loudly when the library has not been built: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtfhe.so")

TFHE_OK, TFHE_EINVAL, TFHE_ENOTNTT, TFHE_ENOMEM, TFHE_EHIP, TFHE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
AUTO, BUTTERFLY, FOURSTEP_MFMA, FOURSTEP_VALU = 0, 1, 2, 3
ALGOS = {"auto": AUTO, "butterfly": BUTTERFLY, "mfma": FOURSTEP_MFMA, "co": FOURSTEP_VALU}

_lib = None


class ServerRequest(ctypes.Structure):
    """tfhe_server_request."""
    _fields_ = [("op", ctypes.c_uint32), ("log_n", ctypes.c_uint32), ("level", ctypes.c_uint32),
                ("galois_elt", ctypes.c_uint32), ("ct_a", ctypes.c_void_p), ("ct_b", ctypes.c_void_p),
                ("ct_out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class NttDesc(ctypes.Structure):
    """tfhe_ntt_desc: one transform of a fused batch."""
    _fields_ = [("plan", ctypes.c_void_p), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("limb_begin", ctypes.c_uint32), ("limb_count", ctypes.c_uint32),
                ("batch", ctypes.c_uint32), ("inverse", ctypes.c_int32)]


class TfheError(RuntimeError):
    def __init__(self, status, func, detail):
        self.status = status
        super().__init__(f"{func} -> {status_name(status)}: {detail}")


def load():
    """Load libtfhe.so and declare its signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2212_14191_amd.build` (no CPU fallback exists)")
    # The library and PyTorch must share one HIP runtime: with torch loaded
    # first, the library's libamdhip64 dependency resolves to torch's copy.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    u32, u64, i32, vp, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    pu32 = ctypes.POINTER(u32)
    sig = {
        "tfhe_status_string": ([i32], ctypes.c_char_p),
        "tfhe_last_error": ([], ctypes.c_char_p),
        "tfhe_find_primes": ([u32, u64, u32, pu32], i32),
        "tfhe_default_psi": ([u32, u32, pu32], i32),
        "tfhe_ntt_plan_create": ([ctypes.POINTER(vp), u32, u32, pu32, pu32, i32], i32),
        "tfhe_ntt_plan_destroy": ([vp], i32),
        "tfhe_ntt_plan_info": ([vp, pu32, pu32, ctypes.POINTER(i32)], i32),
        "tfhe_ntt_plan_modulus": ([vp, u32, pu32, pu32], i32),
        "tfhe_ntt_workspace_size": ([vp, i32, u32, u32, ctypes.POINTER(sz)], i32),
        "tfhe_ntt_fwd": ([vp, i32, vp, vp, u32, u32, u32, vp, sz, vp], i32),
        "tfhe_ntt_inv": ([vp, i32, vp, vp, u32, u32, u32, vp, sz, vp], i32),
        "tfhe_pointwise_mul": ([vp, vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_pointwise_add": ([vp, vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_pointwise_sub": ([vp, vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_pointwise_mul_bcast": ([vp, vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_frobenius_map": ([vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_load_small": ([vp, vp, vp, u32, u32, u32, vp], i32),
        "tfhe_ntt_plan_set_param": ([vp, i32, ctypes.c_int64], i32),
        "tfhe_ntt_plan_get_param": ([vp, i32, ctypes.POINTER(ctypes.c_int64)], i32),
        "tfhe_ntt_batch_workspace_size": ([ctypes.POINTER(NttDesc), u32, i32, ctypes.POINTER(sz)], i32),
        "tfhe_ntt_batch": ([ctypes.POINTER(NttDesc), u32, i32, vp, sz, vp], i32),
        "tfhe_timing_enable": ([i32], i32),
        "tfhe_timing_read": ([ctypes.c_char_p, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)], i32),
        "tfhe_ckks_ctx_create": ([ctypes.POINTER(vp), u32, u32, u32, u32, pu32, pu32, i32], i32),
        "tfhe_ckks_ctx_destroy": ([vp], i32),
        "tfhe_ckks_ctx_plan": ([vp, ctypes.POINTER(vp)], i32),
        "tfhe_hmult_workspace_size": ([vp, u32, u32, ctypes.POINTER(sz)], i32),
        "tfhe_hmult": ([vp, vp, vp, vp, vp, u32, u32, vp, sz, vp], i32),
        "tfhe_hmult_noalloc": ([vp, vp, vp, vp, vp, u32, u32, vp], i32),
        "tfhe_hmult_levels_workspace_size": ([vp, pu32, u32, ctypes.POINTER(sz)], i32),
        "tfhe_hmult_levels": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), pu32, u32, vp, vp, sz,
                               vp], i32),
        "tfhe_rotate_levels": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), pu32, pu32, u32, vp,
                                sz, vp], i32),
        "tfhe_rotate": ([vp, vp, vp, vp, u32, u32, u32, vp, sz, vp], i32),
        "tfhe_rotate_multi": ([vp, vp, vp, ctypes.POINTER(vp), pu32, u32, u32, vp, sz, vp], i32),
        "tfhe_rescale_workspace_size": ([vp, u32, u32, ctypes.POINTER(sz)], i32),
        "tfhe_rescale": ([vp, vp, vp, u32, u32, vp, sz, vp], i32),
        "tfhe_cmult": ([vp, vp, vp, vp, u32, u32, vp], i32),
        "tfhe_hadd": ([vp, vp, vp, vp, u32, u32, vp], i32),
        "tfhe_server_create": ([ctypes.POINTER(vp), u32, u32, vp, sz], i32),
        "tfhe_server_add_context": ([vp, vp, vp], i32),
        "tfhe_server_add_rotation_key": ([vp, u32, u32, vp], i32),
        "tfhe_server_set_max_batch": ([vp, u32, u32], i32),
        "tfhe_server_submit": ([vp, u32, u32, u32, vp, vp, u32, vp, u64, vp], i32),
        "tfhe_server_submit_many": ([vp, ctypes.POINTER(ServerRequest), u32, vp, ctypes.POINTER(u32)], i32),
        "tfhe_server_poll": ([vp, ctypes.POINTER(u64), ctypes.POINTER(i32), u32], u32),
        "tfhe_server_destroy": ([vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def status_name(s):
    return load().tfhe_status_string(int(s)).decode()


def check(status, func):
    if status != TFHE_OK:
        detail = load().tfhe_last_error().decode()
        raise TfheError(status, func, detail)


def _call(name, *args):
    st = getattr(load(), name)(*args)
    check(st, name)
    return st


def _u32_array(values):
    if values is None:
        return None
    vals = [int(v) for v in values]
    return (ctypes.c_uint32 * len(vals))(*vals)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------ raw entry points
def tfhe_find_primes(bits, two_n, count):
    out = (ctypes.c_uint32 * count)()
    _call("tfhe_find_primes", bits, two_n, count, out)
    return list(out)


def tfhe_default_psi(q, log_n):
    r = ctypes.c_uint32()
    _call("tfhe_default_psi", q, log_n, ctypes.byref(r))
    return r.value


def _check_residues(t, name, shape=None):
    import torch
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous int32 CUDA/HIP tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")


class NttPlan:
    """Owns a tfhe_ntt_plan: N = 2^log_n over the given primes."""

    def __init__(self, log_n, q, psi=None, algo="auto", handle=None):
        self.log_n = int(log_n)
        self.n = 1 << self.log_n
        self._owned = handle is None
        if handle is None:
            h = ctypes.c_void_p()
            _call("tfhe_ntt_plan_create", ctypes.byref(h), self.log_n, len(q), _u32_array(q),
                  _u32_array(psi), ALGOS.get(algo, algo))
            self.handle = h
        else:
            self.handle = handle
        ln, nl, al = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
        _call("tfhe_ntt_plan_info", self.handle, ctypes.byref(ln), ctypes.byref(nl), ctypes.byref(al))
        self.n_limbs, self.algo = nl.value, al.value
        self.q, self.psi = [], []
        for l in range(self.n_limbs):
            a, b = ctypes.c_uint32(), ctypes.c_uint32()
            _call("tfhe_ntt_plan_modulus", self.handle, l, ctypes.byref(a), ctypes.byref(b))
            self.q.append(a.value)
            self.psi.append(b.value)

    PARAMS = {"fs_wg_per_cu": 1, "auto_algo": 2, "fs_wide": 3, "fs_passes": 4, "ks_inner": 5, "fs_ring": 6}

    def set_param(self, name, value):
        _call("tfhe_ntt_plan_set_param", self.handle, self.PARAMS[name], int(value))
        if name == "auto_algo":
            self.algo = self.get_param("auto_algo")

    def get_param(self, name):
        v = ctypes.c_int64()
        _call("tfhe_ntt_plan_get_param", self.handle, self.PARAMS[name], ctypes.byref(v))
        return v.value

    def close(self):
        if self._owned and self.handle:
            load().tfhe_ntt_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, limb_count, batch, algo="auto"):
        b = ctypes.c_size_t()
        _call("tfhe_ntt_workspace_size", self.handle, ALGOS.get(algo, algo), limb_count, batch,
              ctypes.byref(b))
        return b.value

    def workspace(self, limb_count, batch, algo="auto"):
        import torch
        nbytes = self.workspace_bytes(limb_count, batch, algo)
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda") if nbytes else None

    def _transform(self, name, x, out, algo, limb_begin, ws, stream):
        limbs, batch, n = x.shape
        if n != self.n:
            raise ValueError(f"last dimension {n} != N = {self.n}")
        _check_residues(x, "x")
        if out is None:
            out = torch_empty_like(x)
        _check_residues(out, "out", x.shape)
        if ws is None:
            ws = self.workspace(limbs, batch, algo)
        _call(name, self.handle, ALGOS.get(algo, algo), _ptr(x), _ptr(out), limb_begin, limbs, batch,
              _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream))
        return out

    def fwd(self, x, out=None, algo="auto", limb_begin=0, ws=None, stream=None):
        """Forward NTT (Eq. 4) of x: int32 [limbs][batch][N]."""
        return self._transform("tfhe_ntt_fwd", x, out, algo, limb_begin, ws, stream)

    def inv(self, x, out=None, algo="auto", limb_begin=0, ws=None, stream=None):
        """Inverse NTT of x: int32 [limbs][batch][N]."""
        return self._transform("tfhe_ntt_inv", x, out, algo, limb_begin, ws, stream)

    def _ew(self, name, a, b, out, limb_begin, stream):
        limbs, batch, n = a.shape
        _check_residues(a, "a")
        _check_residues(b, "b")
        if out is None:
            out = torch_empty_like(a)
        _call(name, self.handle, _ptr(a), _ptr(b), _ptr(out), limb_begin, limbs, batch, _stream(stream))
        return out

    def mul(self, a, b, out=None, limb_begin=0, stream=None):
        return self._ew("tfhe_pointwise_mul", a, b, out, limb_begin, stream)

    def add(self, a, b, out=None, limb_begin=0, stream=None):
        return self._ew("tfhe_pointwise_add", a, b, out, limb_begin, stream)

    def sub(self, a, b, out=None, limb_begin=0, stream=None):
        return self._ew("tfhe_pointwise_sub", a, b, out, limb_begin, stream)

    def mul_bcast(self, a, b, out=None, limb_begin=0, stream=None):
        """a [limbs][batch][N] times b [limbs][N] broadcast over the batch."""
        return self._ew("tfhe_pointwise_mul_bcast", a, b, out, limb_begin, stream)

    def load_small(self, x, limb_begin=0, limb_count=None, out=None, stream=None):
        """Residues of small signed ints x (int32 [batch][N]) on limbs
        [limb_begin, limb_begin + limb_count): int32 [limb_count][batch][N]."""
        import torch
        if x.dtype != torch.int32 or not x.is_cuda or x.dim() != 2 or x.shape[1] != self.n:
            raise ValueError("x: expected an int32 CUDA tensor [batch][N]")
        x = x.contiguous()
        if limb_count is None:
            limb_count = self.n_limbs - limb_begin
        if out is None:
            out = torch.empty((limb_count, x.shape[0], self.n), dtype=torch.int32, device=x.device)
        _call("tfhe_load_small", self.handle, _ptr(x), _ptr(out), limb_begin, limb_count, x.shape[0],
              _stream(stream))
        return out

    def frobenius(self, x, galois, out=None, stream=None):
        limbs, batch, n = x.shape
        _check_residues(x, "x")
        if out is None:
            out = torch_empty_like(x)
        _call("tfhe_frobenius_map", self.handle, _ptr(x), _ptr(out), galois, limbs, batch, _stream(stream))
        return out


def tfhe_timing_enable(enable=True):
    _call("tfhe_timing_enable", 1 if enable else 0)


def tfhe_timing_read(kernel):
    """(launches, total_ms) of a kernel since timing was enabled."""
    n, ms = ctypes.c_uint64(), ctypes.c_double()
    _call("tfhe_timing_read", kernel.encode(), ctypes.byref(n), ctypes.byref(ms))
    return n.value, ms.value


def ntt_batch(items, algo="auto", ws=None, stream=None):
    """Fused transforms (operation-level batching).  items: list of
    (plan, x, out, inverse, limb_begin); x/out int32 [limbs][batch][N]."""
    import torch
    descs = (NttDesc * len(items))()
    keep = []
    for d, (plan, x, out, inverse, limb_begin) in zip(descs, items):
        _check_residues(x, "x")
        _check_residues(out, "out", x.shape)
        limbs, batch, n = x.shape
        if n != plan.n:
            raise ValueError("last dimension != plan N")
        d.plan, d.in_, d.out = plan.handle.value, x.data_ptr(), out.data_ptr()
        d.limb_begin, d.limb_count, d.batch, d.inverse = limb_begin, limbs, batch, 1 if inverse else 0
        keep.append((x, out))
    a = ALGOS.get(algo, algo)
    if ws is None:
        nb = ctypes.c_size_t()
        _call("tfhe_ntt_batch_workspace_size", descs, len(items), a, ctypes.byref(nb))
        ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
    _call("tfhe_ntt_batch", descs, len(items), a, _ptr(ws), ws.numel(), _stream(stream))
    return [o for _, o in keep]


def torch_empty_like(x):
    import torch
    return torch.empty_like(x, memory_format=torch.contiguous_format)


class CkksContext:
    """Owns a tfhe_ckks_ctx (RNS-CKKS with hybrid key switching)."""

    def __init__(self, log_n, L, K, dnum, moduli=None, psi=None, algo="auto"):
        h = ctypes.c_void_p()
        _call("tfhe_ckks_ctx_create", ctypes.byref(h), log_n, L, K, dnum, _u32_array(moduli),
              _u32_array(psi), ALGOS.get(algo, algo))
        self.handle = h
        self.log_n, self.n, self.L, self.K, self.dnum = log_n, 1 << log_n, L, K, dnum
        ph = ctypes.c_void_p()
        _call("tfhe_ckks_ctx_plan", self.handle, ctypes.byref(ph))
        self.plan = NttPlan(log_n, None, handle=ph)
        self.moduli = self.plan.q

    def close(self):
        if getattr(self, "handle", None):
            self.plan.handle = None
            load().tfhe_ckks_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, level, batch):
        b = ctypes.c_size_t()
        _call("tfhe_hmult_workspace_size", self.handle, level, batch, ctypes.byref(b))
        return b.value

    def workspace(self, level, batch):
        import torch
        return torch.empty(max(self.workspace_bytes(level, batch), 256), dtype=torch.uint8, device="cuda")

    NOALLOC_MAX_BYTES = 128 << 20  # TFHE_HMULT_NOALLOC_MAX_BYTES

    def hmult_noalloc(self, ct_a, ct_b, evk, level, out, stream=None):
        """tfhe_hmult_noalloc: HMULT with the library's fixed per-GPU scratch
        array instead of a workspace; allocates nothing (`out` is required).
        Calls that overlap on one GPU race."""
        _, lv, batch, n = ct_a.shape
        if lv != level:
            raise ValueError("ciphertext level mismatch")
        for t, nm in ((ct_a, "ct_a"), (ct_b, "ct_b"), (out, "out")):
            _check_residues(t, nm, (2, level, batch, self.n))
        _check_residues(evk, "evk", (self.dnum, 2, self.L + self.K, self.n))
        _call("tfhe_hmult_noalloc", self.handle, _ptr(ct_a), _ptr(ct_b), _ptr(out), _ptr(evk), level, batch,
              _stream(stream))
        return out

    def hmult(self, ct_a, ct_b, evk, level, out=None, ws=None, stream=None):
        """HMULT of ct_a, ct_b: int32 [2][level][batch][N] (NTT domain)."""
        _, lv, batch, n = ct_a.shape
        if lv != level:
            raise ValueError("ciphertext level mismatch")
        for t, nm in ((ct_a, "ct_a"), (ct_b, "ct_b")):
            _check_residues(t, nm, (2, level, batch, self.n))
        _check_residues(evk, "evk", (self.dnum, 2, self.L + self.K, self.n))
        if out is None:
            out = torch_empty_like(ct_a)
        if ws is None:
            ws = self.workspace(level, batch)
        _call("tfhe_hmult", self.handle, _ptr(ct_a), _ptr(ct_b), _ptr(out), _ptr(evk), level, batch,
              _ptr(ws), ws.numel(), _stream(stream))
        return out

    LEVELS_MAX = 64  # TFHE_HMULT_LEVELS_MAX

    def levels_workspace_bytes(self, levels):
        """Workspace of a mixed-level batch (tfhe_hmult_levels_workspace_size)."""
        b = ctypes.c_size_t()
        _call("tfhe_hmult_levels_workspace_size", self.handle, _u32_array(levels), len(levels), ctypes.byref(b))
        return b.value

    def levels_workspace(self, levels):
        import torch
        return torch.empty(max(self.levels_workspace_bytes(levels), 256), dtype=torch.uint8, device="cuda")

    def hmult_levels(self, cts_a, cts_b, evk, outs=None, ws=None, stream=None):
        """HMULT of pairs of different levels in one batched launch sequence
        (tfhe_hmult_levels): cts_a[i], cts_b[i] are single ciphertexts, int32
        [2][level_i][N]; returns the results (outs[i], same shapes)."""
        if len(cts_a) != len(cts_b):
            raise ValueError("one second operand per first operand")
        levels = []
        for a, b in zip(cts_a, cts_b):
            if a.dim() != 3:
                raise ValueError("hmult_levels takes single ciphertexts [2][level][N]")
            lv = a.shape[1]
            _check_residues(a, "ct_a", (2, lv, self.n))
            _check_residues(b, "ct_b", (2, lv, self.n))
            levels.append(lv)
        _check_residues(evk, "evk", (self.dnum, 2, self.L + self.K, self.n))
        if outs is None:
            outs = [torch_empty_like(a) for a in cts_a]
        for o, lv in zip(outs, levels):
            _check_residues(o, "out", (2, lv, self.n))
        if ws is None:
            ws = self.levels_workspace(levels)
        cnt = len(levels)
        arr = lambda ts: (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in ts])
        _call("tfhe_hmult_levels", self.handle, arr(cts_a), arr(cts_b), arr(outs), _u32_array(levels), cnt,
              _ptr(evk), _ptr(ws), ws.numel(), _stream(stream))
        return outs

    def rotate_levels(self, cts, rotkeys, galois, outs=None, ws=None, stream=None):
        """Ciphertext i (int32 [2][level_i][N]) rotated by galois[i] with
        rotkeys[i], all in one batched launch sequence (tfhe_rotate_levels)."""
        if len(rotkeys) != len(cts) or len(galois) != len(cts):
            raise ValueError("one rotation key and one Galois element per ciphertext")
        levels = []
        for c in cts:
            if c.dim() != 3:
                raise ValueError("rotate_levels takes single ciphertexts [2][level][N]")
            _check_residues(c, "ct", (2, c.shape[1], self.n))
            levels.append(c.shape[1])
        for k in rotkeys:
            _check_residues(k, "rotkey", (self.dnum, 2, self.L + self.K, self.n))
        if outs is None:
            outs = [torch_empty_like(c) for c in cts]
        for o, lv in zip(outs, levels):
            _check_residues(o, "out", (2, lv, self.n))
        if ws is None:
            ws = self.levels_workspace(levels)
        cnt = len(levels)
        arr = lambda ts: (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in ts])
        _call("tfhe_rotate_levels", self.handle, arr(cts), arr(outs), arr(rotkeys), _u32_array(galois),
              _u32_array(levels), cnt, _ptr(ws), ws.numel(), _stream(stream))
        return outs

    def rotate(self, ct, rotkey, galois, level, out=None, ws=None, stream=None):
        _, lv, batch, n = ct.shape
        _check_residues(ct, "ct", (2, level, batch, self.n))
        _check_residues(rotkey, "rotkey", (self.dnum, 2, self.L + self.K, self.n))
        if out is None:
            out = torch_empty_like(ct)
        if ws is None:
            ws = self.workspace(level, batch)
        _call("tfhe_rotate", self.handle, _ptr(ct), _ptr(out), _ptr(rotkey), galois, level, batch,
              _ptr(ws), ws.numel(), _stream(stream))
        return out

    ROTATE_MULTI_MAX = 64

    def rotate_multi(self, ct, rotkeys, galois, level, out=None, ws=None, stream=None):
        """Ciphertext b of ct rotated by galois[b] with rotkeys[b] (one
        batched launch sequence; tfhe_rotate_multi)."""
        _, lv, batch, n = ct.shape
        _check_residues(ct, "ct", (2, level, batch, self.n))
        if len(rotkeys) != batch or len(galois) != batch:
            raise ValueError("one rotation key and one Galois element per ciphertext")
        for k in rotkeys:
            _check_residues(k, "rotkey", (self.dnum, 2, self.L + self.K, self.n))
        if out is None:
            out = torch_empty_like(ct)
        if ws is None:
            ws = self.workspace(level, batch)
        keys = (ctypes.c_void_p * batch)(*[k.data_ptr() for k in rotkeys])
        _call("tfhe_rotate_multi", self.handle, _ptr(ct), _ptr(out), keys, _u32_array(galois), level, batch,
              _ptr(ws), ws.numel(), _stream(stream))
        return out

    def rescale_workspace(self, level, batch):
        import torch
        b = ctypes.c_size_t()
        _call("tfhe_rescale_workspace_size", self.handle, level, batch, ctypes.byref(b))
        return torch.empty(max(b.value, 256), dtype=torch.uint8, device="cuda")

    def rescale(self, ct, level, out=None, ws=None, stream=None):
        """RESCALE of ct: int32 [2][level][batch][N] -> [2][level-1][batch][N]."""
        _, lv, batch, n = ct.shape
        _check_residues(ct, "ct", (2, level, batch, self.n))
        if out is None:
            import torch
            out = torch.empty((2, level - 1, batch, self.n), dtype=torch.int32, device=ct.device)
        _check_residues(out, "out", (2, level - 1, batch, self.n))
        if ws is None:
            ws = self.rescale_workspace(level, batch)
        _call("tfhe_rescale", self.handle, _ptr(ct), _ptr(out), level, batch, _ptr(ws), ws.numel(),
              _stream(stream))
        return out

    def cmult(self, ct, pt, level, out=None, stream=None):
        """CMULT: ct [2][level][batch][N] times plaintext pt [level][batch][N]."""
        _, lv, batch, n = ct.shape
        _check_residues(ct, "ct", (2, level, batch, self.n))
        _check_residues(pt, "pt", (level, batch, self.n))
        if out is None:
            out = torch_empty_like(ct)
        _call("tfhe_cmult", self.handle, _ptr(ct), _ptr(pt), _ptr(out), level, batch, _stream(stream))
        return out

    def hadd(self, ct_a, ct_b, level, out=None, stream=None):
        """HADD of two ciphertexts [2][level][batch][N]."""
        _, lv, batch, n = ct_a.shape
        for t, nm in ((ct_a, "ct_a"), (ct_b, "ct_b")):
            _check_residues(t, nm, (2, level, batch, self.n))
        if out is None:
            out = torch_empty_like(ct_a)
        _call("tfhe_hadd", self.handle, _ptr(ct_a), _ptr(ct_b), _ptr(out), level, batch, _stream(stream))
        return out


class NativeServer:
    """The library's request dispatcher (tfhe_server_*): single-ciphertext
    HMULT / HROTATE requests in, batched launches on `slots` streams, tagged
    completions out.  Holds references to each request's tensors until its
    completion has been polled."""

    HMULT, ROTATE = 0, 1

    def __init__(self, slots=2, max_batch=16, pool_bytes=1 << 30):
        import torch
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _call("tfhe_server_create", ctypes.byref(h), slots, max_batch, _ptr(self.pool), pool_bytes)
        self.handle = h
        self._ctx = {}       # log_n -> (CkksContext, evk, {galois: rotkey})
        self._keep = []      # every context and key ever registered (queued
                             # requests hold raw pointers to them until close())
        self._live = {}      # tag -> tensors the request reads or writes
        self._next = 0
        cap = 4096
        self._tags = (ctypes.c_uint64 * cap)()
        self._status = (ctypes.c_int * cap)()
        self._cap = cap

    def add_context(self, ctx, evk, rotkeys=None):
        """Registers ctx (CkksContext), its relinearisation key and a dict
        {galois element: rotation key}.  Registering the same context again
        adds rotation keys to those it has; a different context for the same
        N starts from none (the dispatcher drops the earlier ones).  Every
        context and key stays referenced until close()."""
        _check_residues(evk, "evk", (ctx.dnum, 2, ctx.L + ctx.K, ctx.n))
        for k in (rotkeys or {}).values():
            _check_residues(k, "rotkey", (ctx.dnum, 2, ctx.L + ctx.K, ctx.n))
        _call("tfhe_server_add_context", self.handle, ctx.handle, _ptr(evk))
        self._keep.append((ctx, evk))
        prev = self._ctx.get(ctx.log_n)
        keys = dict(prev[2]) if prev is not None and prev[0] is ctx else {}
        self._ctx[ctx.log_n] = (ctx, evk, keys)
        for g, k in (rotkeys or {}).items():
            _call("tfhe_server_add_rotation_key", self.handle, ctx.log_n, int(g), _ptr(k))
            self._keep.append(k)
            keys[int(g)] = k

    def set_max_batch(self, log_n, max_batch):
        """tfhe_server_set_max_batch: the batch limit of one N (0 = the
        server's)."""
        _call("tfhe_server_set_max_batch", self.handle, log_n, int(max_batch))

    def submit(self, op, ct_a, ct_b=None, galois=0, out=None, stream=None):
        """Queues one request on ciphertext(s) of shape [2][level][N] (or
        [2][level][1][N]); returns (tag, out)."""
        level, n = ct_a.shape[1], ct_a.shape[-1]
        if ct_a.numel() != 2 * level * n:
            raise ValueError("one ciphertext [2][level][N] per request")
        log_n = n.bit_length() - 1
        if log_n not in self._ctx:
            raise ValueError(f"no context registered for N = {n}")
        _check_residues(ct_a, "ct_a")
        if op == self.HMULT:
            _check_residues(ct_b, "ct_b", ct_a.shape)
        if out is None:
            out = torch_empty_like(ct_a)
        _check_residues(out, "out", ct_a.shape)
        tag = self._next
        self._next += 1
        _call("tfhe_server_submit", self.handle, op, log_n, level, _ptr(ct_a), _ptr(ct_b), galois, _ptr(out),
              tag, _stream(stream))
        self._live[tag] = (ct_a, ct_b, out)
        return tag, out

    def submit_many(self, reqs, stream=None):
        """Queues several requests in one call (one readiness event for all):
        reqs is a list of (op, ct_a, ct_b or None, galois, out or None).
        Returns [(tag, out)]; nothing is queued if one request is rejected."""
        arr = (ServerRequest * len(reqs))()
        res, live = [], []
        for i, (op, a, b, g, out) in enumerate(reqs):
            level, n = a.shape[1], a.shape[-1]
            if a.numel() != 2 * level * n:
                raise ValueError("one ciphertext [2][level][N] per request")
            _check_residues(a, "ct_a")
            if op == self.HMULT:
                _check_residues(b, "ct_b", a.shape)
            if out is None:
                out = torch_empty_like(a)
            _check_residues(out, "out", a.shape)
            tag = self._next + i
            r = arr[i]
            r.op, r.log_n, r.level, r.galois_elt = op, n.bit_length() - 1, level, int(g or 0)
            r.ct_a, r.ct_b, r.ct_out, r.tag = a.data_ptr(), b.data_ptr() if b is not None else 0, out.data_ptr(), tag
            res.append((tag, out))
            live.append((a, b, out))
        bad = ctypes.c_uint32()
        _call("tfhe_server_submit_many", self.handle, arr, len(reqs), _stream(stream), ctypes.byref(bad))
        self._next += len(reqs)
        for (tag, _), t in zip(res, live):
            self._live[tag] = t
        return res

    def hmult(self, ct_a, ct_b, out=None, stream=None):
        return self.submit(self.HMULT, ct_a, ct_b, 0, out, stream)

    def rotate(self, ct, galois, out=None, stream=None):
        return self.submit(self.ROTATE, ct, None, galois, out, stream)

    def poll(self):
        """Completed requests as a list of (tag, status name or None)."""
        k = load().tfhe_server_poll(self.handle, self._tags, self._status, self._cap)
        res = []
        for i in range(k):
            t, st = self._tags[i], self._status[i]
            self._live.pop(t, None)
            res.append((t, None if st == TFHE_OK else status_name(st)))
        return res

    def pending(self):
        return len(self._live)

    def close(self):
        if getattr(self, "handle", None):
            load().tfhe_server_destroy(self.handle)
            self.handle = None
            self._live.clear()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
