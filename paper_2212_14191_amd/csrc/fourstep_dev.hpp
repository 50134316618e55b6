// Device building blocks shared by the four-step transform kernels (the
// two-pass kernels and the one-pass kernel): the descriptor table of a fused
// launch, the INT8 matrix-core contraction with its digit-plane fusion and
// Montgomery step, the twist-and-re-slice, the radix-r level B, work-item
// location and the LDS / memory-counter waits.  See ntt_fourstep.hip for the
// arithmetic (balanced byte digits, exactness bounds).
#pragma once
#include <type_traits>

#include "internal.hpp"

namespace tfhe {

// Descriptor table of a fused launch (passed by value as a kernel argument):
// unit k covers global polynomials [item_begin[k], item_begin[k+1]).  Every
// unit of a launch has the same N and direction.
constexpr int kMaxUnits = 40;
struct FsUnit {
  const uint32_t* in;
  uint32_t* out;
  const FourStepLimb* limbs;  // tables of the unit's first limb
  uint32_t batch;
  uint32_t item_begin;
  // second-pass epilogue (forward transforms): out = (acc - y) m_l, or
  // out += (acc - y) m_l, with m_l the Shoup pair of the unit's limb l
  const uint32_t* acc;
  const uint2* mult;
  uint32_t accumulate;
  // first pass: every limb reads polynomial b of the one plane `in`
  uint32_t in_bcast;
};
struct FsTable {
  uint32_t count, total;  // units, polynomials
  uint32_t log_n;
  uint32_t cols;          // S = N / P: columns of this pass (row stride in natural order)
  uint32_t ipp_log;       // log2 of the items per polynomial (N / item words)
  FsUnit u[kMaxUnits];
};
// One-pass kernel (ntt_onepass.hip): N = 2^12..2^15, no epilogue; one
// launch over every unit of `t` (same N and direction).
bool op_supported(uint32_t log_n);
hipError_t op_run(const tfhe_ntt_plan_s* p, bool inverse, const FsTable& t, hipStream_t s);

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// 64-bit a b + c as one v_mad_u64_u32 (the carry-out is discarded).  Used
// where only the low word is needed, which the compiler would otherwise
// split into a 32-bit multiply and an add.
__device__ __forceinline__ uint64_t mad_u64(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t d, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=&v"(d), "=s"(carry) : "v"(a), "v"(b), "v"(c));
  return d;
}

// a b 2^{-32} mod q as (V + m q) / 2^32, V = a b, m = -V q^{-1} mod 2^32:
// below 2^32 for any a, b < 2^32, and below 2q for a, b < q (not reduced).
__device__ __forceinline__ uint32_t mont_mul_lazy(uint32_t a, uint32_t b, uint32_t q, uint32_t qneg) {
  const uint64_t V = mad_u64(a, b, 0);
  const uint32_t m = (uint32_t)V * qneg;
  return (uint32_t)(mad_u64(m, q, V) >> 32);
}

// Fusion and one Montgomery step: V 2^{-32} mod q, in [0, q + 2^17).
// (V + m q) is a multiple of 2^32 below 2^64, so its high word is exact
// (one v_mad_u64_u32).
__device__ __forceinline__ uint32_t fuse_redc(int c0, int c1, int c2, int c3, uint32_t q,
                                              uint32_t qneg) {
  const uint32_t lo = (uint32_t)c0 + ((uint32_t)c1 << 8);
  const uint32_t hi = (uint32_t)c2 + ((uint32_t)c3 << 8);
  const uint64_t V = mad_u64(hi, 0x10000u, lo);
  const uint32_t m = (uint32_t)V * qneg;
  return (uint32_t)(((uint64_t)m * q + V) >> 32);
}

// Twist (Shoup, t = {w, companion}) and re-slice into digits; r < 2^32.
// z - q lies in [-q, q), inside the digit window unless q > 0x7F7F7F7F.
// For such q the digits of z - q are ((r w - h q) + (0x80808080 - q)) ^
// 0x80808080 with h = floor(r w' / 2^32): two multiply-adds on the low word
// (nq = -q, cq = 0x80808080 - q, both mod 2^32).
template <bool kBigQ>
__device__ __forceinline__ uint32_t twist_digits(uint32_t r, uint2 t, uint32_t q, uint32_t nq, uint64_t cq) {
  if (!kBigQ) {
    const uint32_t h = __umulhi(r, t.y);
    return (uint32_t)mad_u64(h, nq, mad_u64(r, t.x, cq)) ^ 0x80808080u;
  }
  const uint32_t z = mul_shoup_lazy(r, t.x, t.y, q);  // [0, 2q)
  int32_t zz = (int32_t)(z - q);                      // [-q, q)
  zz = zz > 0x7F7F7F7F ? zz - (int32_t)q : zz;
  return balanced_digits(zz);
}

// After level A, lane (s, g) register j holds MFMA row i = 4g + j, i.e.
// vector m = i / kR, element v = i % kR.  After level B register j holds
// output t of vector m (the output index is s + 16 t).
template <int kR>
__device__ __forceinline__ void lane_out(int g, int j, int& m, int& t) {
  if (kR == 16) { m = 0; t = 4 * g + j; }
  else if (kR == 8) { m = g >> 1; t = 2 * j + (g & 1); }
  else if (kR == 4) { m = g; t = j; }
  else if (kR == 2) { m = 2 * g + (j >> 1); t = j & 1; }
  else { m = 4 * g + j; t = 0; }
}

// Radix-4 DFT y_t = sum_v x_v w4^{vt} (w4 of order 4) on residues in [0, q).
__device__ __forceinline__ void dft4(uint32_t* x, uint2 w4, uint32_t q) {
  const uint32_t a0 = add_mod(x[0], x[2], q), a1 = sub_mod(x[0], x[2], q);
  const uint32_t b0 = add_mod(x[1], x[3], q);
  const uint32_t b1 = mul_shoup(sub_mod(x[1], x[3], q), w4.x, w4.y, q);
  x[0] = add_mod(a0, b0, q);
  x[1] = add_mod(a1, b1, q);
  x[2] = sub_mod(a0, b0, q);
  x[3] = sub_mod(a1, b1, q);
}

// Level B for kR < 16: the kR-point cyclic DFT over v of y (residues in
// [0, q)), with lb[x] = rho^x for the root rho of order kR.  For kR = 8 the
// eight inputs of a vector sit in lanes g and g ^ 1 (four each): lane
// parity h computes the outputs t = 2 j + h from e_j = z_j + z_{j+4} (h = 0)
// or o_j = (z_j - z_{j+4}) rho^j (h = 1) with a radix-4 DFT by rho^2.
template <int kR>
__device__ __forceinline__ void level_b(uint32_t* y, const uint2* lb, const uint2* rj, int g,
                                        uint32_t q) {
  if (kR == 2) {
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
      const uint32_t a = y[j], b = y[j + 1];
      y[j] = add_mod(a, b, q);
      y[j + 1] = sub_mod(a, b, q);
    }
  } else if (kR == 4) {
    dft4(y, lb[1], q);
  } else if (kR == 8) {
    const bool h = g & 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t other = (uint32_t)__shfl_xor((int)y[j], 16);
      const uint32_t lo = h ? other : y[j], hi = h ? y[j] : other;  // z_j, z_{j+4}
      const uint32_t d = h ? sub_mod(lo, hi, q) : add_mod(lo, hi, q);
      y[j] = mul_shoup(d, rj[j].x, rj[j].y, q);
    }
    dft4(y, lb[2], q);
  }
}
struct Item {
  uint32_t unit, limb;
  size_t poly_base;  // word offset of the polynomial within the unit's arrays
  size_t in_base;    // its input's offset (the batch element's, for a broadcast input)
};
// Global polynomial p -> (unit, limb, offset); `k` is a running unit index
// (p only increases along a walk).
__device__ __forceinline__ Item locate(const FsTable& t, uint32_t p, uint32_t& k) {
  while (k + 1 < t.count && p >= t.u[k + 1].item_begin) ++k;
  const uint32_t local = p - t.u[k].item_begin;
  Item it;
  it.unit = k;
  it.limb = local / t.u[k].batch;
  it.poly_base = (size_t)local << t.log_n;
  it.in_base = t.u[k].in_bcast ? (size_t)(local % t.u[k].batch) << t.log_n : it.poly_base;
  return it;
}

typedef __attribute__((address_space(3))) void lds_void_t;

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding load): LDS accesses of this wave are completed
// first; the direct-to-LDS loads are covered by wait_item.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
}

}  // namespace
}  // namespace tfhe
