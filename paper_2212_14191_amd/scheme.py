"""RNS-CKKS key generation and secret-key encryption on the device, built on
the library's kernels (NTT, Hada-Mult, Ele-Add/Sub, FrobeniusMap, small-
integer loading).  These produce the resident keys and ciphertexts that
HMULT / HROTATE consume (Sec. II-B); they are set-up work, not the hot path.

Conventions (the same as the library's HMULT): ct = (c0, c1) in the NTT
domain with Dec = c0 + c1*s; a switching key from s' to s is
evk_j = (b_j, a_j) over all L+K limbs, b_j = -a_j*s + e_j + g_j*s', with
g_j = [P]_{q_i} on the q-limbs of digit j and 0 elsewhere.  Random draws
come in as arguments (see paper_2212_14191_amd.inputs).
"""
import numpy as np
import torch

from . import tfhe


def _dev_i32(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x)).view(np.int32)).cuda()


class Scheme:
    def __init__(self, ctx: "tfhe.CkksContext"):
        self.ctx = ctx
        self.plan = ctx.plan
        self.n, self.L, self.K, self.dnum = ctx.n, ctx.L, ctx.K, ctx.dnum
        self.alpha = self.L // self.dnum
        self.moduli = list(ctx.moduli)
        P = 1
        for p in self.moduli[self.L:]:
            P *= p
        self.P = P

    # ---------------------------------------------------------------- secrets
    def secret_ntt(self, s, limbs=None):
        """NTT of a small-integer secret s (int8/int32 [N]) over plan limbs
        [0, limbs): int32 [limbs][N]."""
        limbs = self.L + self.K if limbs is None else limbs
        x = _dev_i32(np.asarray(s, np.int32).reshape(1, self.n))
        res = self.plan.load_small(x, 0, limbs)
        return self.plan.fwd(res).reshape(limbs, self.n)

    def _gadget(self, j):
        """[L+K][1][N] int32 tensor: [P]_{q_i} on digit j's q-limbs, else 0."""
        g = torch.zeros((self.L + self.K, 1, self.n), dtype=torch.int32, device="cuda")
        for i in range(self.alpha * j, self.alpha * (j + 1)):
            g[i].fill_(int(self.P % self.moduli[i]))
        return g

    def switch_key(self, s, sp_ntt, a_draw, e_draw):
        """a_draw: uint32 [dnum][L+K][N] uniform residues (NTT domain);
        e_draw: int32 [dnum][N].  Returns int32 [dnum][2][L+K][N]."""
        LK = self.L + self.K
        s_ntt = self.secret_ntt(s).reshape(LK, 1, self.n)
        sp = sp_ntt.reshape(LK, 1, self.n)
        key = torch.empty((self.dnum, 2, LK, 1, self.n), dtype=torch.int32, device="cuda")
        for j in range(self.dnum):
            a = _dev_i32(np.asarray(a_draw[j], np.uint32)).reshape(LK, 1, self.n)
            e = self.plan.fwd(self.plan.load_small(_dev_i32(np.asarray(e_draw[j], np.int32).reshape(1, self.n))))
            b = self.plan.sub(e, self.plan.mul(a, s_ntt))
            b = self.plan.add(b, self.plan.mul(self._gadget(j), sp))
            key[j, 0] = b
            key[j, 1] = a
        return key.reshape(self.dnum, 2, LK, self.n)

    def relin_key(self, s, a_draw, e_draw):
        s_ntt = self.secret_ntt(s).reshape(self.L + self.K, 1, self.n)
        return self.switch_key(s, self.plan.mul(s_ntt, s_ntt), a_draw, e_draw)

    def rotation_key(self, s, galois, a_draw, e_draw):
        s_ntt = self.secret_ntt(s).reshape(self.L + self.K, 1, self.n)
        return self.switch_key(s, self.plan.frobenius(s_ntt, galois), a_draw, e_draw)

    # -------------------------------------------------------------- encryption
    def encrypt(self, s, m, c1_draw, e_draw, level, delta=1 << 30):
        """Secret-key encryption of integer messages m (int32 [B][N]) at
        `level`: c0 = -c1*s + NTT(e + delta*m).  c1_draw: uint32
        [level][B][N] uniform residues; e_draw: int32 [B][N].  Returns int32
        [2][level][B][N]."""
        B = np.asarray(m).shape[0]
        s_ntt = self.secret_ntt(s, level)
        mres = self.plan.load_small(_dev_i32(np.asarray(m, np.int32)), 0, level)
        dl = torch.empty((level, self.n), dtype=torch.int32, device="cuda")
        for i in range(level):
            dl[i].fill_(delta % self.moduli[i])
        pt = self.plan.mul_bcast(mres, dl)
        pt = self.plan.add(pt, self.plan.load_small(_dev_i32(np.asarray(e_draw, np.int32)), 0, level))
        pt = self.plan.fwd(pt)
        c1 = _dev_i32(np.asarray(c1_draw, np.uint32))
        c0 = self.plan.sub(pt, self.plan.mul_bcast(c1, s_ntt))
        out = torch.empty((2, level, B, self.n), dtype=torch.int32, device="cuda")
        out[0] = c0
        out[1] = c1
        return out
