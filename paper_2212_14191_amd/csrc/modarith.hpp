// Modular arithmetic on 32-bit residues (q < 2^31), shared by every kernel
// of the library and by its host-side table construction.
//
//   Shoup multiplication by a fixed operand w (w' = floor(w 2^32 / q)):
//     a*w mod q for any a < 2^32 with one high and two low products.
//   Montgomery reduction (R = 2^32) for products of two variable residues.
//   Balanced base-256 digits: z in [-0x80808080, 0x7F7F7F7F] has a unique
//     expansion z = sum_d 2^{8d} c_d with c_d in [-128, 127], and the bytes of
//     (z + 0x80808080) ^ 0x80808080 are exactly c_0..c_3 as int8.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TFHE_HD __host__ __device__ __forceinline__

namespace tfhe {

TFHE_HD uint32_t mulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}

// Shoup companion of w (w < q).
TFHE_HD uint32_t shoup_companion(uint32_t w, uint32_t q) {
  return (uint32_t)(((uint64_t)w << 32) / q);
}

// a*w mod q in [0, 2q), any a < 2^32.
TFHE_HD uint32_t mul_shoup_lazy(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
  uint32_t t = mulhi32(a, wp);
  return a * w - t * q;
}

// x in [0, 2q) -> [0, q) (unsigned min trick: x - q wraps above x when x < q).
TFHE_HD uint32_t reduce_once(uint32_t x, uint32_t q) {
  uint32_t y = x - q;
  return y < x ? y : x;
}

TFHE_HD uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
  return reduce_once(mul_shoup_lazy(a, w, wp, q), q);
}

TFHE_HD uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q) { return reduce_once(a + b, q); }

TFHE_HD uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) {
  uint32_t d = a - b;
  uint32_t e = d + q;
  return e < d ? e : d;
}

// Montgomery: returns a*b*2^{-32} mod q in [0, q) for a, b < q < 2^31;
// qneg = -q^{-1} mod 2^32.
TFHE_HD uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t q, uint32_t qneg) {
  uint64_t x = (uint64_t)a * b;
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  uint32_t m = lo * qneg;
  uint32_t t = hi + mulhi32(m, q) + (lo != 0u);
  return reduce_once(t, q);
}

// Per-modulus constants for variable*variable products: a*b mod q =
// Shoup(REDC(a*b), 2^32 mod q).
struct ModConst {
  uint32_t q, qneg, r, rp;  // r = 2^32 mod q, rp its Shoup companion
};

TFHE_HD uint32_t mul_mod(uint32_t a, uint32_t b, const ModConst& c) {
  return mul_shoup(mont_mul(a, b, c.q, c.qneg), c.r, c.rp, c.q);
}

// Sums of products of residues (a, b < q < 2^31) kept as 64-bit values
// below q 2^32: s + a b < q 2^32 + q^2 < 2^64, and when the high word
// reaches q (it is then below 2q) taking q off it restores the bound.
TFHE_HD uint64_t mac_lazy(uint64_t s, uint32_t a, uint32_t b, uint32_t q) {
  const uint64_t v = (uint64_t)a * b + s;
  const uint32_t hi = (uint32_t)(v >> 32);
  const uint32_t h2 = hi - q;
  return ((uint64_t)(h2 < hi ? h2 : hi) << 32) | (uint32_t)v;
}

// s mod q for s < q 2^32: one Montgomery step (s + m q < 2q 2^32 is a
// multiple of 2^32), then the factor 2^32 restored by Shoup.
TFHE_HD uint32_t reduce_lazy(uint64_t s, const ModConst& c) {
  const uint32_t m = (uint32_t)s * c.qneg;
  const uint32_t t = (uint32_t)(((uint64_t)m * c.q + s) >> 32);
  return mul_shoup(reduce_once(t, c.q), c.r, c.rp, c.q);
}

// Balanced digits of z in [-0x80808080, 0x7F7F7F7F], packed as 4 int8.
TFHE_HD uint32_t balanced_digits(int32_t z) {
  return ((uint32_t)z + 0x80808080u) ^ 0x80808080u;
}

// canonical x in [0, q) -> representative in the balanced-digit window
TFHE_HD int32_t to_window(uint32_t x, uint32_t q) {
  return x > 0x7F7F7F7Fu ? (int32_t)(x - q) : (int32_t)x;
}

}  // namespace tfhe
