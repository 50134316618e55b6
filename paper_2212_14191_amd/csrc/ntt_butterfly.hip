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
// Stages run in pairs: each thread takes four elements through two radix-2
// stages in registers between LDS round trips (a radix-4 step); an odd stage
// count ends with one single stage.
//
// Every kernel walks a descriptor table, so one launch can cover transforms
// of different N, moduli and direction (operation-level batching, Sec. IV-D).
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

// Two consecutive stages per LDS round trip (radix-4 step) on the four
// elements p, p + d, p + 2d, p + 3d (d in words).
// Cooley-Tukey stages of strides 2d and d: (0,2), (1,3) with wa, then (0,1)
// with wb0 and (2,3) with wb1.
__device__ __forceinline__ void ct_bfly4(uint32_t* lds, uint32_t p, uint32_t d, uint2 wa, uint2 wb0, uint2 wb1,
                                         uint32_t q) {
  uint32_t x0 = lds[p], x1 = lds[p + d], x2 = lds[p + 2 * d], x3 = lds[p + 3 * d];
  uint32_t v = mul_shoup(x2, wa.x, wa.y, q);
  x2 = sub_mod(x0, v, q);
  x0 = add_mod(x0, v, q);
  v = mul_shoup(x3, wa.x, wa.y, q);
  x3 = sub_mod(x1, v, q);
  x1 = add_mod(x1, v, q);
  v = mul_shoup(x1, wb0.x, wb0.y, q);
  x1 = sub_mod(x0, v, q);
  x0 = add_mod(x0, v, q);
  v = mul_shoup(x3, wb1.x, wb1.y, q);
  x3 = sub_mod(x2, v, q);
  x2 = add_mod(x2, v, q);
  lds[p] = x0;
  lds[p + d] = x1;
  lds[p + 2 * d] = x2;
  lds[p + 3 * d] = x3;
}

// Gentleman-Sande stages of strides d and 2d: (0,1) with wa0 and (2,3) with
// wa1, then (0,2), (1,3) with wb.
__device__ __forceinline__ void gs_bfly4(uint32_t* lds, uint32_t p, uint32_t d, uint2 wa0, uint2 wa1, uint2 wb,
                                         uint32_t q) {
  uint32_t x0 = lds[p], x1 = lds[p + d], x2 = lds[p + 2 * d], x3 = lds[p + 3 * d];
  uint32_t u = x0;
  x0 = add_mod(u, x1, q);
  x1 = mul_shoup(sub_mod(u, x1, q), wa0.x, wa0.y, q);
  u = x2;
  x2 = add_mod(u, x3, q);
  x3 = mul_shoup(sub_mod(u, x3, q), wa1.x, wa1.y, q);
  u = x0;
  x0 = add_mod(u, x2, q);
  x2 = mul_shoup(sub_mod(u, x2, q), wb.x, wb.y, q);
  u = x1;
  x1 = add_mod(u, x3, q);
  x3 = mul_shoup(sub_mod(u, x3, q), wb.x, wb.y, q);
  lds[p] = x0;
  lds[p + d] = x1;
  lds[p + 2 * d] = x2;
  lds[p + 3 * d] = x3;
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
    uint32_t m = 1, t = n >> 1;
    for (; t >= 2; m <<= 2, t >>= 2) {  // stages (m, t) and (2m, t/2)
      for (uint32_t b = threadIdx.x; b < (n >> 2); b += kThreads) {
        const uint32_t g = b / (t >> 1), e0 = 2 * g * t + b % (t >> 1);
        ct_bfly4(lds, e0, t >> 1, w[m + g], w[2 * m + 2 * g], w[2 * m + 2 * g + 1], q);
      }
      __syncthreads();
    }
    if (t == 1) {  // odd stage count: the last stage alone
      for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) ct_bfly(lds, 2 * b, 1, w[m + b], q);
      __syncthreads();
    }
    for (uint32_t kk = threadIdx.x; kk < n; kk += kThreads) dst[kk] = lds[brev(kk, log_n)];
  } else {
    for (uint32_t kk = threadIdx.x; kk < n; kk += kThreads) lds[brev(kk, log_n)] = src[kk];
    __syncthreads();
    uint32_t h = n >> 1, t = 1;
    for (; 4 * t <= n; h >>= 2, t <<= 2) {  // stages (h, t) and (h/2, 2t)
      for (uint32_t b = threadIdx.x; b < (n >> 2); b += kThreads) {
        const uint32_t I = b / t, e0 = 4 * I * t + b % t;
        gs_bfly4(lds, e0, t, w[h + 2 * I], w[h + 2 * I + 1], w[(h >> 1) + I], q);
      }
      __syncthreads();
    }
    if (t < n) {  // odd stage count: the last stage alone
      for (uint32_t b = threadIdx.x; b < (n >> 1); b += kThreads) {
        const uint32_t i = b / t, j = 2 * i * t + (b % t);
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
  const uint32_t nu = (R / 4) * kBlk;  // radix-4 units per pair of stages
  if (!U.inverse) {
    uint32_t m = 1, tr = R / 2;
    for (; tr >= 2; m <<= 2, tr >>= 2) {  // stages (m, tr) and (2m, tr/2)
      for (uint32_t b = threadIdx.x; b < nu; b += kThreads) {
        const uint32_t c = b % kBlk, u = b / kBlk;
        const uint32_t g = u / (tr >> 1), e0 = 2 * g * tr + u % (tr >> 1);
        ct_bfly4(lds, e0 * kBlk + c, (tr >> 1) * kBlk, w[m + g], w[2 * m + 2 * g], w[2 * m + 2 * g + 1], q);
      }
      __syncthreads();
    }
    if (tr == 1) {  // odd stage count: the last stage alone
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        const uint32_t c = b % kBlk, rb = b / kBlk;
        ct_bfly(lds, 2 * rb * kBlk + c, kBlk, w[m + rb], q);
      }
      __syncthreads();
    }
  } else {
    uint32_t h = R / 2, tr = 1;
    for (; 4 * tr <= R; h >>= 2, tr <<= 2) {  // stages (h, tr) and (h/2, 2tr)
      for (uint32_t b = threadIdx.x; b < nu; b += kThreads) {
        const uint32_t c = b % kBlk, u = b / kBlk;
        const uint32_t I = u / tr, e0 = 4 * I * tr + u % tr;
        gs_bfly4(lds, e0 * kBlk + c, tr * kBlk, w[h + 2 * I], w[h + 2 * I + 1], w[(h >> 1) + I], q);
      }
      __syncthreads();
    }
    if (tr < R) {  // odd stage count: the last stage alone
      for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        const uint32_t c = b % kBlk, rb = b / kBlk;
        const uint32_t i = rb / tr, r = 2 * i * tr + (rb % tr);
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
  // the 8 stages of a row of 256 run as 4 radix-4 steps; group g of stage
  // (m, t) in row `row` uses twiddle m + row 256 / (2t) + g
  const uint32_t nu = kBlk * kRow / 4;
  if (!inv) {
    for (uint32_t m = R, t = kRow / 2; t >= 2; m <<= 2, t >>= 2) {  // stages (m, t) and (2m, t/2)
      for (uint32_t b = threadIdx.x; b < nu; b += kThreads) {
        const uint32_t i = b / (kRow / 4), u = b % (kRow / 4);
        const uint32_t row = brev(kBlk * rb + i, log_r);
        const uint32_t g = u / (t >> 1), e0 = 2 * g * t + u % (t >> 1);
        const uint32_t oa = m + row * (kRow / (2 * t)) + g, ob = 2 * m + row * (kRow / t) + 2 * g;
        ct_bfly4(lds, i * kRow + e0, t >> 1, w[oa], w[ob], w[ob + 1], q);
      }
      __syncthreads();
    }
  } else {
    for (uint32_t h = n / 2, t = 1; 4 * t <= kRow; h >>= 2, t <<= 2) {  // stages (h, t) and (h/2, 2t)
      for (uint32_t b = threadIdx.x; b < nu; b += kThreads) {
        const uint32_t i = b / (kRow / 4), u = b % (kRow / 4);
        const uint32_t row = brev(kBlk * rb + i, log_r);
        const uint32_t I = u / t, e0 = 4 * I * t + u % t;
        const uint32_t oa = h + row * (kRow / (2 * t)) + 2 * I, ob = (h >> 1) + row * (kRow / (4 * t)) + I;
        gs_bfly4(lds, i * kRow + e0, t, w[oa], w[oa + 1], w[ob], q);
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
