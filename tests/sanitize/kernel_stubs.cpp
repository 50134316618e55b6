// Host-side stand-ins for the functions defined in the library's .hip
// sources (kernel launchers), so that its host code links in a sanitizer
// build against the HIP stand-in runtime.  The size queries follow the
// library's rules.  Each launcher computes nothing; it touches (reads or
// writes) the first and the last word of every range the real kernel reads
// or writes, so that under AddressSanitizer a workspace, output or input
// smaller than what the launch uses fails at once (the workspace audit
// driver sizes every buffer exactly).  The transform units' workspace
// slices follow the real layout rules (fs_run_units: one rounded slice per
// unit in unit order, none for first-pass-only units, whose intermediate is
// their output; bf_run_units: a slice per unit above N = 2^12).  Test
// infrastructure only.
#include "../../paper_2212_14191_amd/csrc/ckks_internal.hpp"

namespace tfhe {

bool fs_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 16; }

size_t bf_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  if (p->log_n <= 12) return 0;
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

size_t unit_ws_bytes(const NttUnit& u, bool mfma) {
  if (mfma) return (size_t)u.limb_count * u.batch * u.plan->n * sizeof(uint32_t);
  return bf_workspace_bytes(u.plan, u.limb_count, u.batch);
}

static volatile uint32_t g_sink;
static void rd(const uint32_t* p, uint64_t words) {
  if (words) g_sink = g_sink + p[0] + p[words - 1];
}
static void wr(uint32_t* p, uint64_t words) {
  if (words) p[0] = p[words - 1] = 0;
}
static uint64_t words_of(const NttUnit& u) { return (uint64_t)u.limb_count * u.batch * u.plan->n; }
static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static void unit_io(const NttUnit& u, uint32_t* mid, uint64_t mid_words) {
  rd(u.in, u.in_bcast ? (uint64_t)u.batch * u.plan->n : words_of(u));
  if (u.pass1_only) {
    wr(u.out, (uint64_t)(unit_ws_bytes(u, true) / 4));
    return;
  }
  wr(mid, mid_words);
  if (u.acc) rd(u.acc, words_of(u));
  if (u.epi_add) rd(u.out, words_of(u));
  wr(u.out, words_of(u));
}

hipError_t fs_run_units(const NttUnit* units, uint32_t count, void* ws, hipStream_t) {
  unsigned char* w = (unsigned char*)ws;
  for (uint32_t k = 0; k < count; ++k) {
    if (units[k].pass1_only) {
      unit_io(units[k], nullptr, 0);
      continue;
    }
    const size_t b = unit_ws_bytes(units[k], true);
    unit_io(units[k], (uint32_t*)w, b / 4);
    w += round256(b);
  }
  return hipSuccess;
}

hipError_t bf_run_units(const NttUnit* units, uint32_t count, void* ws, hipStream_t) {
  unsigned char* w = (unsigned char*)ws;
  for (uint32_t k = 0; k < count; ++k) {
    const NttUnit& u = units[k];
    if (u.limb_count * u.batch == 0) continue;
    if (u.plan->log_n <= 12) {
      unit_io(u, nullptr, 0);
      continue;
    }
    const size_t b = bf_workspace_bytes(u.plan, u.limb_count, u.batch);
    unit_io(u, (uint32_t*)w, b / 4);
    w += round256(b);
  }
  return hipSuccess;
}

hipError_t bf_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws, uint32_t lb,
                      uint32_t lc, uint32_t batch, hipStream_t s) {
  NttUnit u{p, false, in, out, lb, lc, batch};
  return bf_run_units(&u, 1, ws, s);
}
hipError_t bf_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws, uint32_t lb,
                      uint32_t lc, uint32_t batch, hipStream_t s) {
  NttUnit u{p, true, in, out, lb, lc, batch};
  return bf_run_units(&u, 1, ws, s);
}
hipError_t fs_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws, uint32_t lb,
                      uint32_t lc, uint32_t batch, hipStream_t s) {
  NttUnit u{p, false, in, out, lb, lc, batch};
  return fs_run_units(&u, 1, ws, s);
}
hipError_t fs_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws, uint32_t lb,
                      uint32_t lc, uint32_t batch, hipStream_t s) {
  NttUnit u{p, true, in, out, lb, lc, batch};
  return fs_run_units(&u, 1, ws, s);
}
hipError_t co_transform(const tfhe_ntt_plan_s* p, bool inverse, const uint32_t* in, uint32_t* out, void* ws,
                        uint32_t lb, uint32_t lc, uint32_t batch, hipStream_t s) {
  NttUnit u{p, inverse, in, out, lb, lc, batch};
  return fs_run_units(&u, 1, ws, s);
}
hipError_t ew_launch(EwOp op, const ModConst*, const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t limbs,
                     uint32_t batch, uint32_t n, hipStream_t) {
  const uint64_t w = (uint64_t)limbs * batch * n;
  rd(a, w);
  rd(b, op == EW_MUL_BCAST ? (uint64_t)limbs * n : w);
  wr(out, w);
  return hipSuccess;
}
hipError_t frobenius_launch(const uint32_t* in, uint32_t* out, uint32_t, uint32_t rows, uint32_t log_n,
                            hipStream_t) {
  rd(in, (uint64_t)rows << log_n);
  wr(out, (uint64_t)rows << log_n);
  return hipSuccess;
}
hipError_t load_small_launch(const ModConst*, const int32_t* in, uint32_t* out, uint32_t limbs, uint32_t batch,
                             uint32_t n, hipStream_t) {
  rd((const uint32_t*)in, (uint64_t)batch * n);
  wr(out, (uint64_t)limbs * batch * n);
  return hipSuccess;
}
hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2, const ModConst*,
                         uint32_t level, uint32_t batch, uint32_t n, hipStream_t) {
  const uint64_t P = (uint64_t)level * batch * n;
  rd(a, 2 * P);
  rd(b, 2 * P);
  wr(out, 2 * P);
  wr(d2, P);
  return hipSuccess;
}
// element idx of a level group's [level][B][N] planes: its first and last rows
static void group_rows(uint32_t* base, uint32_t level, uint32_t B, uint32_t idx, uint32_t n) {
  wr(base + (uint64_t)idx * n, n);
  wr(base + ((uint64_t)(level - 1) * B + idx) * n, n);
}
hipError_t launch_tensor_multi(const CtDescSet& set, const ModConst*, uint32_t log_n, hipStream_t) {
  const uint32_t n = 1u << log_n;
  for (uint32_t r = 0; r < set.count; ++r) {
    const CtDesc& c = set.c[r];
    rd(c.a, 2ull * c.level * n);
    rd(c.b, 2ull * c.level * n);
    group_rows(c.out, c.level, c.B, c.idx, n);
    group_rows(c.out + (uint64_t)c.level * c.B * n, c.level, c.B, c.idx, n);
    group_rows(c.d, c.level, c.B, c.idx, n);
  }
  return hipSuccess;
}
hipError_t launch_frobenius_multi(const CtDescSet& set, uint32_t log_n, hipStream_t) {
  const uint32_t n = 1u << log_n;
  for (uint32_t r = 0; r < set.count; ++r) {
    const CtDesc& c = set.c[r];
    rd(c.a, 2ull * c.level * n);
    group_rows(c.out, c.level, c.B, c.idx, n);
    group_rows(c.d, c.level, c.B, c.idx, n);
  }
  return hipSuccess;
}
hipError_t launch_modup(const uint32_t* x, uint32_t* up, const ModConst*, const uint2*, const uint2*, uint32_t d0,
                        uint32_t nd, uint32_t level, uint32_t, uint32_t K, uint32_t batch, uint32_t n, hipStream_t) {
  const uint64_t plane = (uint64_t)batch * n;
  rd(x + d0 * plane, nd * plane);
  wr(up, (level + K) * plane);
  return hipSuccess;
}
static void ip_io(const IpSet& set, uint32_t log_n) {
  const uint64_t n = 1ull << log_n;
  for (uint32_t g = 0; g < set.count; ++g) {
    const IpGroup& G = set.g[g];
    const uint64_t plane = G.batch * n, ext = G.level + set.K;
    rd(G.d2, G.level * plane);
    rd(G.src, G.digits * ext * plane);
    wr(G.acc, 2 * ext * plane);
    for (uint32_t b = 0; b < (set.keys.count == 1 ? 1u : G.batch); ++b)
      rd(set.keys.k[set.keys.count == 1 ? 0 : G.key0 + b], (uint64_t)G.digits * 2 * (set.L + set.K) * n);
  }
}
hipError_t launch_inner_product(const IpSet& set, const ModConst*, uint32_t log_n, hipStream_t) {
  ip_io(set, log_n);
  return hipSuccess;
}
hipError_t ip_run(const tfhe_ntt_plan_s* p, IpSet& set, hipStream_t) {
  ip_io(set, p->log_n);
  return hipSuccess;
}
hipError_t launch_moddown_conv(const uint32_t* a, uint32_t* conv, const ModConst*, const uint2*, const uint2*,
                               uint32_t level, uint32_t, uint32_t K, uint32_t batch, uint32_t n, hipStream_t) {
  const uint64_t plane = (uint64_t)batch * n;
  rd(a, K * plane);
  wr(conv, level * plane);
  return hipSuccess;
}
hipError_t launch_moddown_final(const uint32_t* acc, const uint32_t* conv, uint32_t* out, const ModConst*,
                                const uint2*, uint32_t level, uint32_t batch, uint32_t n, bool accumulate,
                                hipStream_t, KernelId) {
  const uint64_t w = (uint64_t)level * batch * n;
  rd(acc, w);
  rd(conv, w);
  if (accumulate) rd(out, w);
  wr(out, w);
  return hipSuccess;
}
hipError_t launch_frobenius_pair(const uint32_t* in0, uint32_t* out0, const uint32_t* in1, uint32_t* out1,
                                 const GaloisSet&, uint32_t rows, uint32_t log_n, hipStream_t) {
  const uint64_t w = (uint64_t)rows << log_n;
  rd(in0, w);
  rd(in1, w);
  wr(out0, w);
  wr(out1, w);
  return hipSuccess;
}
hipError_t launch_rescale_bcast(const uint32_t* t, uint32_t* u, const ModConst*, uint32_t top, uint32_t batch,
                                uint32_t n, hipStream_t) {
  const uint64_t plane = (uint64_t)batch * n;
  rd(t, 2 * plane);
  wr(u, 2 * top * plane);
  return hipSuccess;
}
hipError_t ConvQueue::flush(uint32_t, KernelId, hipStream_t) {
  for (const ConvDesc& a : q) {
    rd(a.in, a.nin * a.plane);
    for (uint32_t t = 0; t < a.nout; ++t) wr(a.out + conv_pos(a, a.first + t) * a.plane, a.plane);
  }
  q.clear();
  return hipSuccess;
}
hipError_t launch_scatter(const ScatterSet& e, uint32_t count, uint32_t log_n, hipStream_t) {
  const uint64_t n = 1ull << log_n;
  for (uint32_t r = 0; r < count; ++r) {
    rd(e.src[r] + (uint64_t)e.b[r] * n, n);
    rd(e.src[r] + ((uint64_t)(e.rows[r] - 1) * e.batch[r] + e.b[r]) * n, n);
    wr(e.dst[r], e.rows[r] * n);
  }
  return hipSuccess;
}

}  // namespace tfhe
