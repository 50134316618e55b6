"""Serving loop on the GPU: every result is bit-identical alone and in a
concurrent mix of HMULT / rotation requests of different N and level."""
import numpy as np
import pytest

from paper_2212_14191_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def world():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_14191_amd import tfhe
    from paper_2212_14191_amd.scheme import Scheme
    L, K, dnum = 6, 2, 3
    ctxs, evks, rks, cts = {}, {}, {}, {}
    for ln in (10, 12):
        n = 1 << ln
        ctx = tfhe.CkksContext(ln, L, K, dnum)
        sch = Scheme(ctx)
        s = inputs.ternary_secret(1, n, 64)
        a = inputs.uniform_residues(1, ctx.moduli, (dnum, n), stream=1).transpose(1, 0, 2)
        e = inputs.gaussian_error(2, (dnum, n), stream=1)
        ctxs[ln], evks[ln] = ctx, sch.relin_key(s, a, e)
        for r in (1, 3):
            g = pow(5, r, 2 * n)
            rks[(ln, g)] = sch.rotation_key(s, g, a, e)
        for level in (2, 5, 6):
            for i in range(2):
                m = inputs.small_messages(i, (1, n))
                c1 = inputs.uniform_residues(7 + i, ctx.moduli[:level], (1, n), stream=5)
                cts[(ln, level, i)] = sch.encrypt(s, m, c1, inputs.gaussian_error(2, (1, n), stream=i), level)
    return ctxs, evks, rks, cts


def requests(world, count, seed):
    _, _, rks, cts = world
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ln = int(rng.choice([10, 12]))
        level = int(rng.choice([2, 5, 6]))
        if rng.random() < 0.5:
            out.append((0, ln, level, cts[(ln, level, 0)], cts[(ln, level, 1)], None))
        else:
            g = pow(5, int(rng.choice([1, 3])), 2 << ln)
            out.append((1, ln, level, cts[(ln, level, int(rng.integers(2)))], None, g))
    return out


def test_alone_equals_mix_on_gpu(world):
    from paper_2212_14191_amd.serving import GpuBackend, Server
    ctxs, evks, rks, _ = world
    reqs = requests(world, 40, 0)
    alone = []
    be = GpuBackend(ctxs, evks, rks, slots=1)
    srv = Server(be, mem_budget_bytes=1 << 32, slots=1, max_batch=1)
    for op, ln, lv, a, b, g in reqs:
        alone.append(srv.submit(op, ln, lv, a, b, g).result(timeout=60).clone())
    srv.close()
    be = GpuBackend(ctxs, evks, rks, slots=4)
    srv = Server(be, mem_budget_bytes=1 << 32, slots=4, max_batch=8)
    futs = [srv.submit(op, ln, lv, a, b, g) for op, ln, lv, a, b, g in reqs]
    mixed = [f.result(timeout=60) for f in futs]
    st = srv.stats()
    srv.close()
    for x, y in zip(alone, mixed):
        assert torch.equal(x, y)
    assert st["completed"] == len(reqs) and st["p99_ms"] is not None
