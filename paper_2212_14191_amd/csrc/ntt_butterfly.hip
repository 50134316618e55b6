// Radix-2 butterfly NTT / INTT on the vector ALUs: the plain baseline the
// paper compares against (Sec. II-A, Fig. 2; "TensorFHE-NT" in Sec. V).
//
// Forward: Cooley-Tukey butterflies with the negacyclic twist merged into the
// twiddles (psi^{bitrev(m+i)} for group i of stage m), natural-order input,
// bit-reversed intermediate; the final store gathers through the bit
// reversal so the output is in natural order (index k = evaluation at
// psi^{2k+1}, Eq. 4).  Inverse: Gentleman-Sande butterflies with
// psi^{-bitrev(h+i)}, reading the natural-order input through the bit
// reversal, then N^{-1}.
//
// N <= 2^12: one workgroup owns a polynomial, all stages in LDS.
// N  > 2^12: two passes over an R x 256 view (R = N/256): the stages with
// butterfly stride >= 256 act within columns (pass A), the rest within rows
// of 256 (pass B); the intermediate goes through the caller's workspace.
//
// Every kernel walks a descriptor table, so one launch can cover transforms
// of different N, moduli and direction (operation-level batching, Sec. III-D).
#include <algorithm>

#include "internal.hpp"

namespace tfhe {
namespace {

constexpr int kThreads = 256;
constexpr int kRow = 256;   // row length of the two-pass view
constexpr int kBlk = 16;    // columns (pass A) or rows (pass B) per workgroup
constexpr int kMaxUnits = 32;

struct BfUnit {
  const uint32_t* in;
  uint32_t* out;
  const uint2* tw;       // twiddles of the unit's first limb, [limb][N]
  const uint2* ninv;     // [limb]
  const ModConst* mods;  // [limb]
  uint32_t log_n, batch, inverse, item_begin;
};
struct BfTable {
  uint32_t count, total;
  BfUnit u[kMaxUnits];
};

__device__ __forceinline__ uint32_t find_unit(const BfTable& t, uint32_t i) {
  uint32_t k = 0;
  while (k + 1 < t.count && i >= t.u[k + 1].item_begin) ++k;
  return k;
}

__device__ __forceinline__ uint32_t brev(uint32_t x, uint32_t bits) {
  return __builtin_bitreverse32(x) >> (32 - bits);
}

__device__ __forceinline__ void ct_bfly(uint32_t* lds, uint32_t j, uint32_t t, uint2 w, uint32_t q) {
  uint32_t u = lds[j];
  uint32_t v = mul_shoup(lds[j + t], w.x, w.y, q);
  lds[j] = add_mod(u, v, q);
  lds[j + t] = sub_mod(u, v, q);
}

__device__ __forceinline__ void gs_bfly(uint32_t* lds, uint32_t j, uint32_t t, uint2 w, uint32_t q) {
  uint32_t u = lds[j];
  uint32_t v = lds[j + t];
  lds[j] = add_mod(u, v, q);
  lds[j + t] = mul_shoup(sub_mod(u, v, q), w.x, w.y, q);
}

// ---------------------------------------------------------- single pass
// item = polynomial of the unit
__global__ void __launch_bounds__(kThreads) bf_single(const BfTable tab) {
  extern __shared__ uint32_t lds[];
  const uint32_t k = find_unit(tab, blockIdx.x);
  const BfUnit U = tab.u[k];
  const uint32_t poly = blockIdx.x - U.item_begin, limb = poly / U.batch;
  const uint32_t log_n = U.log_n, n = 1u << log_n;
  const uint32_t q = U.mods[limb].q;
  const uint2* w = U.tw + (size_t)limb * n;
  const uint32_t* src = U.in + (size_t)poly * n;
  uint32_t* dst = U.out + (size_t)poly * n;
  if (!U.inverse) {
    for (uint32_t i = threadIdx.x; i < n; i += kThreads) lds[i] = src[i];
    __syncthreads();
    for (uint32_t m = 1, t = n >> 1; m < n; m <<= 1, t >>= 1) {
      for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) {
        uint32_t i = b / t, j = 2 * i * t + (b % t);
        ct_bfly(lds, j, t, w[m + i], q);
      }
      __syncthreads();
    }
    for (uint32_t kk = threadIdx.x; kk < n; kk += kThreads) dst[kk] = lds[brev(kk, log_n)];
  } else {
    for (uint32_t kk = threadIdx.x; kk < n; kk += kThreads) lds[brev(kk, log_n)] = src[kk];
    __syncthreads();
    for (uint32_t h = n >> 1, t = 1; h >= 1; h >>= 1, t <<= 1) {
      for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) {
        uint32_t i = b / t, j = 2 * i * t + (b % t);
        gs_bfly(lds, j, t, w[h + i], q);
      }
      __syncthreads();
    }
    const uint2 ni = U.ninv[limb];
    for (uint32_t kk = threadIdx.x; kk < n; kk += kThreads) dst[kk] = mul_shoup(lds[kk], ni.x, ni.y, q);
  }
}

// ------------------------------------------------------------ two passes
// Column pass: item = (polynomial, block of kBlk consecutive columns), tile
// lds[r][c] (R x kBlk).  Forward runs stages m = 1 .. R/2; inverse runs
// h = R/2 .. 1 then scales by N^{-1}.
__global__ void __launch_bounds__(kThreads) bf_cols(const BfTable tab) {
  __shared__ uint32_t lds[kRow * kBlk];
  const uint32_t k = find_unit(tab, blockIdx.x);
  const BfUnit U = tab.u[k];
  const uint32_t local = blockIdx.x - U.item_begin;
  const uint32_t n = 1u << U.log_n, R = n / kRow;
  // column blocks 2b and 2b+1 share 128-byte lines: place them 8 items
  // apart so both land on the same XCD (workgroups go round-robin over 8)
  const uint32_t slot = local % (kRow / kBlk), poly = local / (kRow / kBlk);
  const uint32_t cb = 2 * (slot % 8) + slot / 8;
  const uint32_t limb = poly / U.batch;
  const uint32_t q = U.mods[limb].q;
  const uint2* w = U.tw + (size_t)limb * n;
  const uint32_t* src = U.in + (size_t)poly * n + cb * kBlk;
  for (uint32_t e = threadIdx.x; e < R * kBlk; e += kThreads) {
    uint32_t r = e / kBlk, c = e % kBlk;
    lds[e] = src[r * kRow + c];
  }
  __syncthreads();
  const uint32_t nb = (R / 2) * kBlk;  // butterflies per stage
  if (!U.inverse) {
    for (uint32_t m = 1, tr = R / 2; m < R; m <<= 1, tr >>= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t c = b % kBlk, rb = b / kBlk;
        uint32_t i = rb / tr, r = 2 * i * tr + (rb % tr);
        ct_bfly(lds, r * kBlk + c, tr * kBlk, w[m + i], q);
      }
      __syncthreads();
    }
  } else {
    for (uint32_t h = R / 2, tr = 1; h >= 1; h >>= 1, tr <<= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t c = b % kBlk, rb = b / kBlk;
        uint32_t i = rb / tr, r = 2 * i * tr + (rb % tr);
        gs_bfly(lds, r * kBlk + c, tr * kBlk, w[h + i], q);
      }
      __syncthreads();
    }
  }
  uint32_t* dst = U.out + (size_t)poly * n + cb * kBlk;
  const uint2 ni = U.ninv[limb];
  for (uint32_t e = threadIdx.x; e < R * kBlk; e += kThreads) {
    uint32_t r = e / kBlk, c = e % kBlk;
    uint32_t v = lds[e];
    if (U.inverse) v = mul_shoup(v, ni.x, ni.y, q);
    dst[r * kRow + c] = v;
  }
}

// Row pass: item = (polynomial, block of the kBlk rows whose bit-reversed
// indices are consecutive, {row = bitrev(kBlk*rb + i)}), tile lds[i][col].
// Position row*256 + col of the bit-reversed order holds the natural-order
// index bitrev8(col)*R + kBlk*rb + i, so the natural-order side is accessed
// in runs of kBlk consecutive words.
// Forward: input = pass-A result (natural rows), stages m = R .. N/2, store
// gathered to natural order.  Inverse: load gathered from the natural-order
// input, stages h = N/2 .. R, store natural rows.
__global__ void __launch_bounds__(kThreads) bf_rows(const BfTable tab) {
  __shared__ uint32_t lds[kBlk * kRow];
  const uint32_t k = find_unit(tab, blockIdx.x);
  const BfUnit U = tab.u[k];
  const uint32_t local = blockIdx.x - U.item_begin;
  const uint32_t n = 1u << U.log_n, R = n / kRow, log_r = U.log_n - 8;
  const uint32_t rb = local % (R / kBlk), poly = local / (R / kBlk);
  const uint32_t limb = poly / U.batch;
  const uint32_t q = U.mods[limb].q;
  const uint2* w = U.tw + (size_t)limb * n;
  const uint32_t* src = U.in + (size_t)poly * n;
  const bool inv = U.inverse != 0;
  for (uint32_t e = threadIdx.x; e < kBlk * kRow; e += kThreads) {
    if (!inv) {
      uint32_t i = e / kRow, col = e % kRow;
      lds[e] = src[brev(kBlk * rb + i, log_r) * kRow + col];
    } else {
      uint32_t i = e % kBlk, cn = e / kBlk;  // natural index cn*R + kBlk*rb + i
      lds[i * kRow + brev(cn, 8)] = src[cn * R + kBlk * rb + i];
    }
  }
  __syncthreads();
  const uint32_t nb = kBlk * kRow / 2;
  if (!inv) {
    for (uint32_t m = R, t = kRow / 2; m < n; m <<= 1, t >>= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t i = b / (kRow / 2), bb = b % (kRow / 2);
        uint32_t row = brev(kBlk * rb + i, log_r);
        uint32_t g = bb / t, j = 2 * g * t + (bb % t);
        uint32_t grp = (row * kRow + j) / (2 * t);
        ct_bfly(lds, i * kRow + j, t, w[m + grp], q);
      }
      __syncthreads();
    }
  } else {
    for (uint32_t h = n / 2, t = 1; h >= R; h >>= 1, t <<= 1) {
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        uint32_t i = b / (kRow / 2), bb = b % (kRow / 2);
        uint32_t row = brev(kBlk * rb + i, log_r);
        uint32_t g = bb / t, j = 2 * g * t + (bb % t);
        uint32_t grp = (row * kRow + j) / (2 * t);
        gs_bfly(lds, i * kRow + j, t, w[h + grp], q);
      }
      __syncthreads();
    }
  }
  uint32_t* dst = U.out + (size_t)poly * n;
  for (uint32_t e = threadIdx.x; e < kBlk * kRow; e += kThreads) {
    if (!inv) {
      uint32_t i = e % kBlk, cn = e / kBlk;
      dst[cn * R + kBlk * rb + i] = lds[i * kRow + brev(cn, 8)];
    } else {
      uint32_t i = e / kRow, col = e % kRow;
      dst[brev(kBlk * rb + i, log_r) * kRow + col] = lds[e];
    }
  }
}

BfUnit make_unit(const NttUnit& u, const uint32_t* in, uint32_t* out) {
  const tfhe_ntt_plan_s* p = u.plan;
  BfUnit b;
  b.in = in;
  b.out = out;
  b.tw = (u.inverse ? p->d_bf_inv : p->d_bf_fwd) + (size_t)u.limb_begin * p->n;
  b.ninv = p->d_ninv + u.limb_begin;
  b.mods = p->d_mod + u.limb_begin;
  b.log_n = p->log_n;
  b.batch = u.batch;
  b.inverse = u.inverse ? 1 : 0;
  b.item_begin = 0;
  return b;
}

// Append a unit of `items` work items to a table.
void push(BfTable& t, BfUnit b, uint32_t items) {
  b.item_begin = t.total;
  t.u[t.count++] = b;
  t.total += items;
}

}  // namespace

size_t bf_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  if (p->log_n <= 12) return 0;
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

// Fused launches: every single-pass unit in one launch; every two-pass unit
// in one column-pass launch and one row-pass launch (ordered so each unit's
// first pass writes its workspace slice and its second pass reads it:
// forward = columns then rows, inverse = rows then columns).
hipError_t bf_run_units(const NttUnit* units, uint32_t count, void* ws, hipStream_t s) {
  unsigned char* w = (unsigned char*)ws;
  for (uint32_t first = 0; first < count; first += kMaxUnits) {
    const uint32_t n = std::min<uint32_t>(kMaxUnits, count - first);
    BfTable single{}, cols1{}, rows1{}, rows2{}, cols2{};
    uint32_t max_n = 0;
    for (uint32_t k = 0; k < n; ++k) {
      const NttUnit& u = units[first + k];
      const uint32_t polys = u.limb_count * u.batch;
      if (polys == 0) continue;
      const uint32_t N = u.plan->n, R = N / kRow;
      if (u.plan->log_n <= 12) {
        push(single, make_unit(u, u.in, u.out), polys);
        max_n = std::max(max_n, N);
        continue;
      }
      uint32_t* mid = (uint32_t*)w;
      w += (bf_workspace_bytes(u.plan, u.limb_count, u.batch) + 255) & ~(size_t)255;
      if (!u.inverse) {
        push(cols1, make_unit(u, u.in, mid), polys * (kRow / kBlk));
        push(rows2, make_unit(u, mid, u.out), polys * (R / kBlk));
      } else {
        push(rows1, make_unit(u, u.in, mid), polys * (R / kBlk));
        push(cols2, make_unit(u, mid, u.out), polys * (kRow / kBlk));
      }
    }
    if (single.total)
      TFHE_TIMED(K_BF_SINGLE, s, hipLaunchKernelGGL(bf_single, dim3(single.total), dim3(kThreads),
                                                    max_n * sizeof(uint32_t), s, single));
    if (cols1.total)
      TFHE_TIMED(K_BF_COLS, s, hipLaunchKernelGGL(bf_cols, dim3(cols1.total), dim3(kThreads), 0, s, cols1));
    if (rows1.total)
      TFHE_TIMED(K_BF_ROWS, s, hipLaunchKernelGGL(bf_rows, dim3(rows1.total), dim3(kThreads), 0, s, rows1));
    if (rows2.total)
      TFHE_TIMED(K_BF_ROWS, s, hipLaunchKernelGGL(bf_rows, dim3(rows2.total), dim3(kThreads), 0, s, rows2));
    if (cols2.total)
      TFHE_TIMED(K_BF_COLS, s, hipLaunchKernelGGL(bf_cols, dim3(cols2.total), dim3(kThreads), 0, s, cols2));
  }
  return hipGetLastError();
}

hipError_t bf_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  NttUnit u{p, false, in, out, limb_begin, limb_count, batch};
  return bf_run_units(&u, 1, ws, s);
}

hipError_t bf_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  NttUnit u{p, true, in, out, limb_begin, limb_count, batch};
  return bf_run_units(&u, 1, ws, s);
}

}  // namespace tfhe
