// NTT plan construction: modulus and root validation, and the twiddle tables
// of both transform algorithms, built once per (N, prime set) on the host and
// copied to the device (Sec. IV-B: the twiddle matrices are fixed by N and q,
// pre-computed at initialisation and reused by every NTT).
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace tfhe {

uint32_t pow_mod(uint32_t b, uint64_t e, uint32_t q) {
  uint64_t r = 1 % q, x = b % q;
  while (e) {
    if (e & 1) r = r * x % q;
    x = x * x % q;
    e >>= 1;
  }
  return (uint32_t)r;
}

uint32_t inv_mod(uint32_t x, uint32_t q) { return pow_mod(x, q - 2, q); }

static uint32_t mulm(uint32_t a, uint32_t b, uint32_t q) { return (uint32_t)((uint64_t)a * b % q); }

// Deterministic Miller-Rabin for 32-bit integers (bases 2, 7, 61).
bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u, 17u, 19u, 23u, 29u, 31u, 37u, 61u})
    if (n % p == 0) return n == p;
  uint32_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; ++r; }
  for (uint32_t a : {2u, 7u, 61u}) {
    uint32_t x = pow_mod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = mulm(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// psi = g^{(q-1)/2N}, g the smallest primitive root of q; 0 if q unsuitable.
uint32_t default_psi(uint32_t q, uint32_t log_n) {
  uint64_t two_n = 2ull << log_n;
  if (!is_prime_u32(q) || (q - 1) % two_n != 0) return 0;
  std::vector<uint32_t> fac;
  uint32_t m = q - 1;
  for (uint32_t d = 2; (uint64_t)d * d <= m; ++d)
    if (m % d == 0) {
      fac.push_back(d);
      while (m % d == 0) m /= d;
    }
  if (m > 1) fac.push_back(m);
  for (uint32_t g = 2; g < q; ++g) {
    bool ok = true;
    for (uint32_t f : fac)
      if (pow_mod(g, (q - 1) / f, q) == 1) { ok = false; break; }
    if (ok) return pow_mod(g, (q - 1) / two_n, q);
  }
  return 0;
}

static uint32_t bit_reverse(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

ModConst make_modconst(uint32_t q) {
  ModConst c;
  c.q = q;
  uint32_t inv = 1;  // q^{-1} mod 2^32 by Newton iteration
  for (int i = 0; i < 5; ++i) inv *= 2u - q * inv;
  c.qneg = 0u - inv;
  c.r = (uint32_t)((1ull << 32) % q);
  c.rp = shoup_companion(c.r, q);
  return c;
}

// ---------------------------------------------------------------- four-step
// Byte j of the balanced digit expansion of the window representative of w.
static int8_t digit(uint32_t w, uint32_t q, int j) {
  uint32_t packed = balanced_digits(to_window(w, q));
  return (int8_t)(packed >> (8 * j));
}

typedef uint32_t Mat16[16][16];

// Level-A data row of MFMA row i is (column m, element v) with i = m r + v;
// after level A lane (s, g) register j holds row i = 4g + j.  After level B
// register j holds output t of column m:
//   r = 16: m = 0, t = 4g + j      r = 8: m = g / 2, t = 2j + g % 2
//   r = 4:  m = g, t = j           r = 2: m = 2g + j / 2, t = j % 2
//   r = 1:  m = 4g + j, t = 0
static void lane_output(int r, int lane, int j, int* m, int* t) {
  const int g = lane / 16;
  switch (r) {
    case 16: *m = 0; *t = 4 * g + j; break;
    case 8: *m = g / 2; *t = 2 * j + g % 2; break;
    case 4: *m = g; *t = j; break;
    case 2: *m = 2 * g + j / 2; *t = j % 2; break;
    default: *m = 4 * g + j; *t = 0; break;
  }
}

// Lay out one pass (WA[u][s], T[s][v], WB[t][v] (r = 16), lb) as MFMA
// operands.  Level A contracts over u with the data as MFMA A operand: lane
// (i, g) holds u = 4g + c, byte 4c + d pairs data digit d with digit j of
// 2^{8d} WA[u][s].  Level B (r = 16) contracts over v with the twiddle as MFMA
// A operand: lane (t, g) holds v = 4g + c.  The twist carries the factor 2^32
// that cancels the Montgomery reduction of the level-A fusion; wb_scale
// multiplies WB (2^32 when level B is the transform's last).
// ua selects the level-A index of lane (i, g), dword c: u = 4g + c (false)
// or u = g + 4c (true; the one-pass kernel's second pass).  tw_scale is the
// twist's factor (2^32 by default).
static void build_pass(PassTables& pt, int r, const Mat16& WA, const Mat16& T, const Mat16& WB,
                       uint32_t q, uint32_t wb_scale, const uint32_t* lb, bool ua = false,
                       uint32_t tw_scale = 0) {
  memset(&pt, 0, sizeof(pt));
  uint32_t p2[4];
  for (int d = 0; d < 4; ++d) p2[d] = pow_mod(2, 8 * d, q);
  for (int j = 0; j < 4; ++j)
    for (int lane = 0; lane < 64; ++lane) {
      int col = lane % 16, g = lane / 16;
      for (int c = 0; c < 4; ++c) {
        uint32_t a = 0, b = 0;
        const int u = ua ? g + 4 * c : 4 * g + c;
        for (int d = 0; d < 4; ++d) {
          a |= (uint32_t)(uint8_t)digit(mulm(p2[d], WA[u][col], q), q, j) << (8 * d);
          if (r == 16) {
            uint32_t wb = mulm(WB[col][4 * g + c], wb_scale, q);
            b |= (uint32_t)(uint8_t)digit(mulm(p2[d], wb, q), q, j) << (8 * d);
          }
        }
        pt.opA[j][lane][c] = a;
        pt.opB[j][lane][c] = b;
      }
    }
  uint32_t r32 = (uint32_t)((1ull << 32) % q);
  if (!tw_scale) tw_scale = r32;
  for (int lane = 0; lane < 64; ++lane)
    for (int j = 0; j < 4; ++j) {
      const int v = (4 * (lane / 16) + j) % r;
      uint32_t w = mulm(T[lane % 16][v], tw_scale, q);
      pt.twist[lane][j] = make_uint2(w, shoup_companion(w, q));
    }
  for (int i = 0; i < 16; ++i) {
    uint32_t w = lb ? lb[i] % q : 0;
    pt.lb[i] = make_uint2(w, shoup_companion(w, q));
  }
}

// post[b][lane][j]: the post-twist P(column, output) of the value lane `lane`
// holds in register j after level B, for the set of columns b + 4 m (m as in
// lane_output; output = s + 16 t).  `scale` is 2^32 when the value still
// carries the Montgomery factor (r = 16), else 1.
template <typename F>
static void build_post(uint2* post, int r, int ncols, uint32_t q, uint32_t scale, F P) {
  for (int b = 0; b < 256; ++b)
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < 4; ++j) {
        int m, t;
        lane_output(r, lane, j, &m, &t);
        const int col = b + 4 * m, k = lane % 16 + 16 * t;
        uint32_t w = col < ncols ? mulm(P(col, k), scale, q) : 0;
        post[(b * 64 + lane) * 4 + j] = make_uint2(w, shoup_companion(w, q));
      }
}

// One-pass kernel: the first pass's post-twist P(col, out) split into a
// per-lane factor and a per-step factor (see OnePassTables).
template <typename F>
static void build_onepass_post(OnePassTables& op, int r1, int ncols, uint32_t q, uint32_t scale, F P) {
  const uint32_t r32 = (uint32_t)((1ull << 32) % q);
  const int mt = 16 / r1, steps = ncols / (4 * mt);
  memset(op.post_a, 0, sizeof(op.post_a));
  for (int lane = 0; lane < 64; ++lane)
    for (int j = 0; j < 4; ++j) {
      int m, t;
      lane_output(r1, lane, j, &m, &t);
      const int out = lane % 16 + 16 * t;
      for (int sg = 0; sg < 4; ++sg) {
        const uint32_t w = mulm(P(4 * m + sg, out), scale, q);
        op.post_b[lane][j][sg] = make_uint2(w, shoup_companion(w, q));
      }
      const uint32_t base_inv = inv_mod(P(4 * m, out), q);
      for (int st = 0; st < steps; ++st)
        op.post_a[st][lane][j] = mulm(mulm(P(4 * st * mt + 4 * m, out), base_inv, q), r32, q);
    }
}

struct FsHostLimb {
  PassTables p1, p2;
  OnePassTables op;
  std::vector<uint2> post;
  CoPass c1, c2;               // N = 2^16: plain matrices for the vector-ALU variant
  std::vector<uint2> co_post;  // [column][output]
};

static void co_pass(CoPass& c, const Mat16& WA, const Mat16& T, const Mat16& WB, uint32_t q) {
  const uint32_t r32 = (uint32_t)((1ull << 32) % q), r64 = mulm(r32, r32, q);
  for (int a = 0; a < 16; ++a)
    for (int b = 0; b < 16; ++b) {
      c.WA[b][a] = mulm(WA[a][b], r64, q);  // WA is [u][s]: stored [s][u]
      c.T[a][b] = make_uint2(T[a][b], shoup_companion(T[a][b], q));
      c.WB[a][b] = mulm(WB[a][b], r64, q);  // [t][v]
    }
}

// Four-step tables for N = N1 x 256 (N1 = 16 r), n = 256 n1 + n2,
// k = k1 + N1 k2:
//   A_k = sum_{n2} w^{k2 n2} psi^{(2k1+1) n2} sum_{n1} phi^{(2k1+1) n1} a[n1][n2]
// with phi = psi^256 (order 2 N1) and w = psi^{2 N1} (order 256).  The
// N1-point stage splits as n1 = r u + v, k1 = s + 16 t; the 256-point stage
// as n2 = 16 u + v, k2 = s + 16 t.  Forward: pass 1 = N1-point over columns
// (+ psi^{(2k1+1) n2}), pass 2 = 256-point.  Inverse: pass 1 = 256-point with
// w^{-1} (+ psi^{-(2k1+1) n2}), pass 2 = N1-point
//   a[s + 16t] = N^{-1} phi^{-s} phi^{-16t} sum_v phi^{-32vt} phi^{-2vs}
//                sum_u phi^{-2rus} Y[ru + v].
static void build_fourstep_limb(FsHostLimb& L, uint32_t log_n, uint32_t q, uint32_t psi, int dir) {
  const uint32_t N = 1u << log_n, N1 = N / 256;
  const int r = (int)(N1 / 16);
  const uint64_t twoN = 2ull * N;
  const uint32_t phi = pow_mod(psi, 256, q), om = pow_mod(psi, 2 * N1, q);
  const uint32_t phii = inv_mod(phi, q), omi = inv_mod(om, q), psii = inv_mod(psi, q);
  const uint32_t ninv = inv_mod(N % q, q), r32 = (uint32_t)((1ull << 32) % q);
  Mat16 WA, T, WB;
  uint32_t lb[16];
  auto cyc256 = [&](PassTables& pt, uint32_t root, uint32_t scale) {
    for (int a = 0; a < 16; ++a)
      for (int b = 0; b < 16; ++b) {
        WA[a][b] = pow_mod(root, 16ull * a * b, q);
        T[a][b] = pow_mod(root, (uint64_t)a * b, q);
        WB[a][b] = pow_mod(root, 16ull * a * b, q);
      }
    build_pass(pt, 16, WA, T, WB, q, scale, nullptr);
    if (r == 16) co_pass(&pt == &L.p1 ? L.c1 : L.c2, WA, T, WB, q);
  };
  // natural-order post-twist table of the vector-ALU variant
  auto co_post = [&](auto P) {
    L.co_post.resize(256 * 256);
    for (int col = 0; col < 256; ++col)
      for (int k = 0; k < 256; ++k) {
        const uint32_t w = P(col, k);
        L.co_post[col * 256 + k] = make_uint2(w, shoup_companion(w, q));
      }
  };
  L.post.resize(256 * 64 * 4);
  if (dir == 0) {
    for (int a = 0; a < 16; ++a)
      for (int b = 0; b < 16; ++b) {
        WA[a][b] = pow_mod(phi, (uint64_t)r * (2 * b + 1) * a, q);  // [u][s]
        T[a][b] = pow_mod(phi, (uint64_t)(2 * a + 1) * b, q);       // [s][v]
        WB[a][b] = pow_mod(phi, 32ull * a * b, q);                  // [t][v]
      }
    const uint32_t rho = pow_mod(phi, 32, q);
    for (int i = 0; i < 16; ++i) lb[i] = i < 8 ? pow_mod(rho, i, q) : 1;
    build_pass(L.p1, r, WA, T, WB, q, 1, lb);
    if (r == 16) co_pass(L.c1, WA, T, WB, q);
    cyc256(L.p2, om, r32);
    // column n2, output k1: psi^{(2 k1 + 1) n2}
    auto P = [&](int n2, int k1) { return pow_mod(psi, (uint64_t)(2 * k1 + 1) * n2 % twoN, q); };
    build_post(L.post.data(), r, 256, q, r == 16 ? r32 : 1, P);
    if (r == 16) co_post(P);
    if (r < 16) {
      // one-pass second pass: the 256-point stage with unscaled level-B
      // twiddles and the twist carrying 2^64
      for (int a = 0; a < 16; ++a)
        for (int b = 0; b < 16; ++b) {
          WA[a][b] = pow_mod(om, 16ull * a * b, q);
          T[a][b] = mulm(pow_mod(om, (uint64_t)a * b, q), r32, q);
          WB[a][b] = WA[a][b];
        }
      build_pass(L.op.p2, 16, WA, T, WB, q, 1, nullptr);
      build_onepass_post(L.op, r, 256, q, 1, P);
    }
  } else {
    cyc256(L.p1, omi, 1);
    if (r == 16) {
      for (int a = 0; a < 16; ++a)
        for (int b = 0; b < 16; ++b) {
          WA[a][b] = pow_mod(phii, 32ull * a * b, q);                               // [u][s]
          T[a][b] = pow_mod(phii, (uint64_t)(2 * b + 1) * a, q);                    // [s][v]
          WB[a][b] = mulm(pow_mod(phii, (uint64_t)(32 * b + 16) * a, q), ninv, q);  // [t][v]
        }
      build_pass(L.p2, 16, WA, T, WB, q, r32, nullptr);
      co_pass(L.c2, WA, T, WB, q);
    } else {
      for (int a = 0; a < 16; ++a)
        for (int b = 0; b < 16; ++b) {
          WA[a][b] = pow_mod(phii, 2ull * r * a * b, q);                             // [u][s]
          T[a][b] = mulm(pow_mod(phii, (uint64_t)(2 * b + 1) * a, q), ninv, q);     // [s][v]
          WB[a][b] = 0;
        }
      const uint32_t rho = pow_mod(phii, 32, q);
      for (int i = 0; i < 16; ++i) lb[i] = i < 8 ? pow_mod(rho, i, q) : pow_mod(phii, 16ull * (i - 8), q);
      build_pass(L.p2, r, WA, T, WB, q, 1, lb);
      build_pass(L.op.p2, r, WA, T, WB, q, 1, lb, true);
    }
    // column k1, output n2: psi^{-(2 k1 + 1) n2}
    auto P = [&](int k1, int n2) { return pow_mod(psii, (uint64_t)(2 * k1 + 1) * n2 % twoN, q); };
    build_post(L.post.data(), 16, (int)N1, q, r32, P);
    if (r == 16) co_post(P);
    if (r < 16) build_onepass_post(L.op, 16, (int)N1, q, r32, P);
  }
}

template <typename T>
static hipError_t upload(T** dst, const T* src, size_t count, std::vector<void*>& owned) {
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(count, 1));
  if (e != hipSuccess) return e;
  owned.push_back(*dst);
  return hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice);
}

tfhe_status plan_build(tfhe_ntt_plan_s* p) {
  const uint32_t N = p->n, L = p->n_limbs;
  std::vector<ModConst> mods(L);
  std::vector<uint2> fwd((size_t)L * N), inv((size_t)L * N), ninv(L);
  for (uint32_t l = 0; l < L; ++l) {
    uint32_t q = p->q[l], psi = p->psi[l], psii = inv_mod(psi, q);
    mods[l] = make_modconst(q);
    for (uint32_t i = 0; i < N; ++i) {
      uint32_t b = bit_reverse(i, p->log_n);
      uint32_t w = pow_mod(psi, b, q), wi = pow_mod(psii, b, q);
      fwd[(size_t)l * N + i] = make_uint2(w, shoup_companion(w, q));
      inv[(size_t)l * N + i] = make_uint2(wi, shoup_companion(wi, q));
    }
    uint32_t ni = inv_mod(N % q, q);
    ninv[l] = make_uint2(ni, shoup_companion(ni, q));
  }
  if (hipGetDevice(&p->device) != hipSuccess) return fail(TFHE_EHIP, "hipGetDevice failed");
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
    p->num_cus = (uint32_t)cus;
  hipError_t e;
  if ((e = upload(&p->d_mod, mods.data(), L, p->owned)) != hipSuccess ||
      (e = upload(&p->d_bf_fwd, fwd.data(), fwd.size(), p->owned)) != hipSuccess ||
      (e = upload(&p->d_bf_inv, inv.data(), inv.size(), p->owned)) != hipSuccess ||
      (e = upload(&p->d_ninv, ninv.data(), L, p->owned)) != hipSuccess)
    return e == hipErrorOutOfMemory ? fail(TFHE_ENOMEM, "plan tables: out of device memory")
                                    : hip_check(e, "plan tables");

  p->has_mfma = fs_supported(p->log_n);
  for (uint32_t l = 0; l < L && p->has_mfma; ++l)
    if (p->q[l] < (1u << 29)) p->has_mfma = false;  // digit bounds need q > 2^29
  p->has_co = p->has_mfma && p->log_n == 16;
  if (p->has_mfma) {
    // blob: per limb and direction {PassTables p1, p2, post[256*64*4]} and,
    // for N = 2^16, {CoPass c1, c2, co_post[256*256]}
    const size_t post_elems = 256 * 64 * 4;
    const bool co = p->log_n == 16;
    const size_t co_bytes = co ? 2 * sizeof(CoPass) + 256 * 256 * sizeof(uint2) : 0;
    const bool one = p->log_n <= 15;  // one-pass kernel tables
    const size_t op_bytes = one ? sizeof(OnePassTables) : 0;
    const size_t per = 2 * sizeof(PassTables) + post_elems * sizeof(uint2) + co_bytes + op_bytes;
    const size_t total = per * 2 * L;
    std::vector<unsigned char> blob(total);
    std::vector<FourStepLimb> hf(L), hi(L);
    e = hipMalloc(&p->d_fs_blob, total);
    if (e != hipSuccess) return fail(TFHE_ENOMEM, "four-step tables: out of device memory");
    p->owned.push_back(p->d_fs_blob);
    unsigned char* dbase = (unsigned char*)p->d_fs_blob;
    for (uint32_t l = 0; l < L; ++l)
      for (int dir = 0; dir < 2; ++dir) {
        FsHostLimb H;
        build_fourstep_limb(H, p->log_n, p->q[l], p->psi[l], dir);
        size_t off = per * (2 * l + dir);
        memcpy(&blob[off], &H.p1, sizeof(PassTables));
        memcpy(&blob[off + sizeof(PassTables)], &H.p2, sizeof(PassTables));
        memcpy(&blob[off + 2 * sizeof(PassTables)], H.post.data(), post_elems * sizeof(uint2));
        FourStepLimb& f = dir == 0 ? hf[l] : hi[l];
        f.pass1 = (const PassTables*)(dbase + off);
        f.pass2 = (const PassTables*)(dbase + off + sizeof(PassTables));
        f.post1 = (const uint2*)(dbase + off + 2 * sizeof(PassTables));
        f.co1 = f.co2 = nullptr;
        f.co_post = nullptr;
        f.op = nullptr;
        if (one) {
          const size_t o3 = off + 2 * sizeof(PassTables) + post_elems * sizeof(uint2) + co_bytes;
          memcpy(&blob[o3], &H.op, sizeof(OnePassTables));
          f.op = (const OnePassTables*)(dbase + o3);
        }
        if (co) {
          const size_t o2 = off + 2 * sizeof(PassTables) + post_elems * sizeof(uint2);
          memcpy(&blob[o2], &H.c1, sizeof(CoPass));
          memcpy(&blob[o2 + sizeof(CoPass)], &H.c2, sizeof(CoPass));
          memcpy(&blob[o2 + 2 * sizeof(CoPass)], H.co_post.data(), 256 * 256 * sizeof(uint2));
          f.co1 = (const CoPass*)(dbase + o2);
          f.co2 = (const CoPass*)(dbase + o2 + sizeof(CoPass));
          f.co_post = (const uint2*)(dbase + o2 + 2 * sizeof(CoPass));
        }
        f.q = p->q[l];
        f.qneg = mods[l].qneg;
      }
    if ((e = hipMemcpy(p->d_fs_blob, blob.data(), total, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = upload(&p->d_fs_fwd, hf.data(), L, p->owned)) != hipSuccess ||
        (e = upload(&p->d_fs_inv, hi.data(), L, p->owned)) != hipSuccess)
      return hip_check(e, "four-step tables");
  }
  return TFHE_OK;
}

void plan_free(tfhe_ntt_plan_s* p) {
  for (void* ptr : p->owned) (void)hipFree(ptr);
  p->owned.clear();
}

}  // namespace tfhe
