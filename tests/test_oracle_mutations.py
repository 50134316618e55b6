"""Planted mistakes in the oracle must fail its pins (CPU only).  Each
mutant is a plausible slip in one step of RESCALE (a swapped operand, a
wrong constant, an off-by-one limb, the rounding reading in place of the
floor); the pin tests run with the mutant in
place of the oracle's function and must fail."""
import numpy as np
import pytest

import oracle
from oracle import ckks

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
