"""Planted mistakes in the oracle must fail its pins (CPU only).  Each
mutant is a plausible slip in one step of RESCALE (a swapped operand, a
wrong constant, an off-by-one limb, the rounding reading in place of the
floor) or of key switching, the tensor product and the automorphism (a
dropped inverse in ModUp, a flipped sign in ModDown, exchanged tensor
operands, a missing negation, ModDown with a rounding offset); the pin
tests run with the mutant in place of the oracle's function and must
fail."""
import numpy as np
import pytest

import oracle
from oracle import ckks

import test_oracle_bigint as bigint
import test_oracle_ckks as pins


def _rescale_mutant(kind):
    def rescale(pr, ct, level):
        top = level - 1
        qt = pr.q[top]
        idx = list(range(top))
        qs = pr.mods(idx)
        out = np.empty((2, top) + ct.shape[2:], dtype=np.uint32)
        for c in range(2):
            src = top if kind != "limb" else top - 1
            t = oracle.ntt_inv(ct[c][src:src + 1], [pr.q[src]], [pr.psi[src]])[0].astype(np.uint64)
            if kind == "centered":  # the rounding reading instead of the floor
                ti = t.astype(np.int64)
                ti = np.where(ti > qt // 2, ti - qt, ti)
                t_mod = np.stack([(ti % qi).astype(np.uint32) for qi in qs])
            else:
                t_mod = np.stack([(t % np.uint64(qi)).astype(np.uint32) for qi in qs])
            u = oracle.ntt_fwd(t_mod, qs, pr.psis(idx))
            diff = oracle.sub(u, ct[c][:top], qs) if kind == "order" else oracle.sub(ct[c][:top], u, qs)
            if kind == "constant":
                k = np.array([qt % qi for qi in qs], dtype=np.uint32).reshape(-1, 1, 1)
            else:
                k = np.array([pow(qt % qi, -1, qi) for qi in qs], dtype=np.uint32).reshape(-1, 1, 1)
            out[c] = oracle.mul(diff, np.broadcast_to(k, diff.shape), qs)
        return out
    return rescale


@pytest.mark.parametrize("kind", ["order", "constant", "limb", "centered"])
def test_rescale_mutants_fail_pins(kind, monkeypatch):
    monkeypatch.setattr(ckks, "rescale", _rescale_mutant(kind))
    failed = 0
    for pin in (lambda: pins.test_rescale_is_floor_division_by_top_modulus(4),
                lambda: pins.test_rescale_decrypts_to_scaled_message(6)):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1, f"mutant {kind} passed every RESCALE pin"


def test_rescale_unmutated_passes_pins():
    pins.test_rescale_is_floor_division_by_top_modulus(4)
    pins.test_rescale_decrypts_to_scaled_message(6)


# ------------------------------------------------------------ key switching
# Five slips in the key switch and the operations around it, each planted
# in place of one oracle function: ModUp without the (Q_j/q_i)^{-1} factor,
# ModDown with the subtraction's sign flipped, the tensor product with the
# second ciphertext's components exchanged in d1, the automorphism without
# the negation of wrapped coefficients (X^N = -1), and ModDown with the
# rounding offset P/2 that another reading adds (a result that still
# decrypts correctly: the decryption pins miss it).

def _mod_up_without_inverse(pr, x, digit, level):
    ext = pr.ext_limbs(level)
    Qj = 1
    for i in digit:
        Qj *= pr.q[i]
    out = np.empty((len(ext),) + x.shape[1:], dtype=np.uint32)
    for pos, t in enumerate(ext):
        if t in digit:
            out[pos] = x[t]
            continue
        m = pr.moduli[t]
        acc = np.zeros(x.shape[1:], dtype=np.uint64)
        for i in digit:
            c = np.uint64((Qj // pr.q[i]) % m)
            acc = (acc + (x[i].astype(np.uint64) % np.uint64(m)) * c % np.uint64(m)) % np.uint64(m)
        out[pos] = acc.astype(np.uint32)
    return out


def _mod_down_sign_flipped(pr, acc_ntt, level):
    # (conv - acc) P^{-1} instead of (acc - conv) P^{-1}
    good = _ORIG["mod_down"](pr, acc_ntt, level)
    qs = pr.mods(range(level))
    return oracle.sub(np.zeros_like(good), good, qs)


def _tensor_exchanged(pr, ct_a, ct_b, level):
    qs = pr.mods(range(level))
    c0, c1 = ct_a[0], ct_a[1]
    e0, e1 = ct_b[0], ct_b[1]
    d0 = oracle.mul(c0, e0, qs)
    d1 = oracle.add(oracle.mul(c0, e0, qs), oracle.mul(c1, e1, qs), qs)
    d2 = oracle.mul(c1, e1, qs)
    return d0, d1, d2


def _automorphism_without_negation(x, k, qs):
    x = np.asarray(x, dtype=np.uint32)
    n = x.shape[-1]
    dest = (np.arange(n, dtype=np.int64) * k) % (2 * n) % n
    out = np.empty_like(x)
    out[..., dest] = x
    return out


def _mod_down_rounded(pr, acc_ntt, level):
    # ModDown(acc + floor(P/2)) instead of ModDown(acc)
    ext = pr.ext_limbs(level)
    mods = pr.mods(ext)
    half = np.array([(pr.P // 2) % m for m in mods], dtype=np.uint32).reshape(-1, 1, 1)
    h = np.ascontiguousarray(np.broadcast_to(half, acc_ntt.shape))
    h_ntt = oracle.ntt_fwd(h, mods, pr.psis(ext))
    return _ORIG["mod_down"](pr, oracle.add(acc_ntt, h_ntt, mods), level)


_ORIG = {"mod_down": ckks.mod_down}

KS_PINS = {
    "mod_up": lambda: pins.test_mod_up_is_lift_plus_small_multiple(),
    "gadget": lambda: pins.test_gadget_identity(),
    "mod_down": lambda: pins.test_mod_down_divides_by_p(),
    "trivial": lambda: pins.test_hmult_trivial_ciphertexts_exact(),
    "hmult_dec": lambda: pins.test_hmult_decrypts_to_product(5),
    "automorphism": lambda: pins.test_automorphism_is_ntt_permutation(),
    "rotate_dec": lambda: pins.test_rotate_decrypts_to_rotated_message("rot5"),
    "hmult_bigint": lambda: bigint.check_hmult("l5"),
    "rotate_bigint": lambda: bigint.check_rotate(5, "l5"),
}

KS_MUTANTS = {
    # mutant: (oracle function replaced, replacement, pins it must fail)
    "modup_inverse": ("mod_up", _mod_up_without_inverse,
                      {"mod_up", "hmult_dec", "rotate_dec", "hmult_bigint", "rotate_bigint"}),
    "moddown_sign": ("mod_down", _mod_down_sign_flipped,
                     {"mod_down", "hmult_dec", "rotate_dec", "hmult_bigint", "rotate_bigint"}),
    "tensor_exchanged": ("tensor", _tensor_exchanged, {"trivial", "hmult_dec", "hmult_bigint"}),
    "automorphism_sign": ("automorphism_coeff", _automorphism_without_negation,
                          {"automorphism", "rotate_dec", "rotate_bigint"}),
    "moddown_rounded": ("mod_down", _mod_down_rounded, {"hmult_bigint", "rotate_bigint"}),
}


def _failing_pins():
    """Names of the pins that fail (an assertion, or an error such as a
    decrypted value too large for the pin's int64 rounding)."""
    failed = set()
    for name, pin in KS_PINS.items():
        try:
            pin()
        except Exception:
            failed.add(name)
    return failed


@pytest.mark.parametrize("kind", sorted(KS_MUTANTS))
def test_key_switch_mutants_fail_pins(kind, monkeypatch):
    fn, repl, must = KS_MUTANTS[kind]
    monkeypatch.setattr(ckks, fn, repl)
    failed = _failing_pins()
    assert must <= failed, f"mutant {kind}: pins {sorted(must - failed)} still pass"


def test_key_switch_unmutated_passes_pins():
    assert _failing_pins() == set()
