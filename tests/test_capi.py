"""The C-ABI library loads, exports every declared entry point, and its host
logic (prime search, default root, argument validation) agrees with the
oracle.  CPU only: no call here launches a kernel."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfhe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfhe_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def tf():
    from paper_2212_14191_amd import tfhe
    tfhe.load()
    return tfhe


def test_every_declared_symbol_is_exported(tf):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(tf.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(tf):
    assert tf.status_name(0) == "TFHE_OK"
    assert tf.status_name(-2) == "TFHE_ENOTNTT"


@pytest.mark.parametrize("bits,two_n,count", [(31, 1 << 17, 44), (30, 1 << 13, 4), (31, 1 << 14, 8)])
def test_find_primes_matches_oracle(tf, bits, two_n, count):
    assert tf.tfhe_find_primes(bits, two_n, count) == oracle.ntt_primes(count, bits, two_n)


@pytest.mark.parametrize("log_n", [4, 8, 12, 13, 16])
def test_default_psi_matches_oracle(tf, log_n):
    for q in oracle.ntt_primes(6, 31, 1 << 17):
        assert tf.tfhe_default_psi(q, log_n) == oracle.psi(q, 1 << log_n)


def test_plan_rejects_bad_moduli(tf):
    q_ok = oracle.ntt_primes(1, 31, 1 << 17)[0]
    bad = [
        [q_ok + 2],                       # not prime
        [oracle.ntt_primes(1, 31, 1 << 9)[0]] if oracle.ntt_primes(1, 31, 1 << 9)[0] % (1 << 17) != 1 else [7681],
        [12289],                          # below 2^29
    ]
    for qs in bad:
        with pytest.raises(tf.TfheError) as ei:
            tf.NttPlan(16, qs)
        assert ei.value.status == tf.TFHE_ENOTNTT
    with pytest.raises(tf.TfheError) as ei:
        tf.NttPlan(16, [q_ok], psi=[3])   # not a primitive 2N-th root
    assert ei.value.status == tf.TFHE_ENOTNTT
    with pytest.raises(tf.TfheError) as ei:
        tf.NttPlan(20, [q_ok])
    assert ei.value.status == tf.TFHE_EINVAL


def test_ckks_ctx_rejects_bad_shape(tf):
    with pytest.raises(tf.TfheError) as ei:
        tf.CkksContext(16, 24, 8, 5)      # dnum does not divide L
    assert ei.value.status == tf.TFHE_EINVAL
    with pytest.raises(tf.TfheError) as ei:
        tf.CkksContext(16, 24, 8, 2)      # alpha = 12 > 8
    assert ei.value.status == tf.TFHE_EUNSUPPORTED


def test_server_rejects_bad_arguments(tf):
    """tfhe_server_* argument checks that precede any HIP call."""
    lib = tf.load()
    h = ctypes.c_void_p()
    fake_pool = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails first
    assert lib.tfhe_server_create(None, 1, 1, fake_pool, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 0, 1, fake_pool, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 17, 1, fake_pool, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 1, 0, fake_pool, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 1, 65, fake_pool, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 1, 4, None, 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 1, 4, ctypes.c_void_p((1 << 20) + 16), 1 << 20) == tf.TFHE_EINVAL
    assert lib.tfhe_server_create(ctypes.byref(h), 4, 4, fake_pool, 512) == tf.TFHE_EINVAL
    assert h.value is None
    assert lib.tfhe_server_submit(None, 0, 10, 1, None, None, 0, None, 0, None) == tf.TFHE_EINVAL
    assert lib.tfhe_server_add_context(None, None, None) == tf.TFHE_EINVAL
    tags, status = (ctypes.c_uint64 * 4)(), (ctypes.c_int * 4)()
    assert lib.tfhe_server_poll(None, tags, status, 4) == 0
    assert lib.tfhe_server_destroy(None) == tf.TFHE_OK


def test_server_request_struct_and_batched_submit_checks(tf):
    assert ctypes.sizeof(tf.ServerRequest) == 48  # uint32 x 4, three pointers, uint64
    lib = tf.load()
    arr = (tf.ServerRequest * 2)()
    bad = ctypes.c_uint32(7)
    assert lib.tfhe_server_submit_many(None, arr, 2, None, ctypes.byref(bad)) == tf.TFHE_EINVAL
    assert bad.value == 7


def test_header_is_plain_c(tmp_path):
    """include/tfhe.h compiles as strict C99 (no C++ or HIP types cross the
    ABI) and its request struct has the layout the binding declares."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "h.c"
    src.write_text('#include "tfhe.h"\n'
                   "int main(void) { return (int)sizeof(tfhe_server_request) != 48; }\n")
    exe = tmp_path / "h"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    assert subprocess.run([str(exe)]).returncode == 0
