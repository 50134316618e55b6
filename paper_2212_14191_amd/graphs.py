"""Graph capture of batched operations (operation-level batching with fixed
shapes, Sec. IV-D): one HMULT or HROTATE of a (N, level, batch) shape is
recorded once as a HIP graph on static buffers and replayed, which removes the
per-kernel launch cost of the ~20-launch key-switching sequence.

The library records no memset and no event inside these sequences, so the
captured graph holds kernel nodes only.  Per-kernel timing must be off while
capturing.
"""
import torch


class CapturedOp:
    """A captured HMULT (op=0) or HROTATE (op=1) on static device buffers.

    run(ct_a, ct_b=None) copies the inputs into the static buffers, replays
    the graph on the current stream and returns the static output tensor
    (overwritten by the next run)."""

    def __init__(self, ctx, key, level, batch, op=0, galois=None):
        n = ctx.n
        self.ctx, self.key, self.level, self.batch, self.op, self.galois = ctx, key, level, batch, op, galois
        self.a = torch.zeros((2, level, batch, n), dtype=torch.int32, device="cuda")
        self.b = torch.zeros_like(self.a) if op == 0 else None
        self.out = torch.empty_like(self.a)
        self.ws = ctx.workspace(level, batch)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._launch(side)          # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            self._launch(torch.cuda.current_stream())
        torch.cuda.synchronize()

    def _launch(self, stream):
        if self.op == 0:
            self.ctx.hmult(self.a, self.b, self.key, self.level, out=self.out, ws=self.ws, stream=stream)
        else:
            self.ctx.rotate(self.a, self.key, self.galois, self.level, out=self.out, ws=self.ws,
                            stream=stream)

    def run(self, ct_a, ct_b=None):
        self.a.copy_(ct_a)
        if self.op == 0:
            self.b.copy_(ct_b)
        self.graph.replay()
        return self.out
