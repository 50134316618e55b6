// Four-step NTT on INT8 matrix cores (Sec. IV-B/IV-C, Eq. 9 and Eq. 10),
// re-designed for gfx950, for N = N1 x 256 with N1 = 16 r, r in {1,..,16}.
//
// With n = 256 n1 + n2 and k = k1 + N1 k2 (phi = psi^256 of order 2 N1,
// w = psi^{2 N1} of order 256):
//   A_k = sum_{n2} w^{k2 n2} psi^{(2k1+1) n2} sum_{n1} phi^{(2k1+1) n1} a[n1][n2].
// Forward: pass 1 transforms the 256 columns (N1 points each, negacyclic) and
// applies the twist psi^{(2k1+1) n2}; pass 2 transforms the N1 rows of the
// result (256 points, cyclic).  The inverse runs the mirror image: pass 1 the
// 256-point inverse over k2 with the twist psi^{-(2k1+1) n2}, pass 2 the
// N1-point inverse over k1 with N^{-1} folded in.
//
// A P-point stage (P = 16 r) splits as n = r u + v, k = s + 16 t: level A is
// a 16-point contraction over u on the matrix cores, then a twist by
// T[s][v], then level B, an r-point transform over v: on the matrix cores
// when r = 16, as VALU butterflies when r < 16.
//
// Exactness (the segment-fusion idea of Sec. IV-C, Fig. 4): every operand
// enters the matrix core as four balanced signed byte digits.  A data word x
// (taken in [-0x80808080, 0x7F7F7F7F]) is x = sum_d 2^{8d} x_d; a twiddle w
// is supplied as the digits j of W^(d) = 2^{8d} w mod q for d = 0..3.  With
// the four data digits of a coefficient packed into four consecutive K
// bytes, one v_mfma_i32_16x16x64_i8 per twiddle digit plane j yields
//   C_j = sum_u sum_d x_d[u] * digit_j(W^(d)[u])   (|C_j| <= 2^20, exact)
// and V = sum_j 2^{8j} C_j = sum_u x[u] w[u] (mod q).  The "fusion" step
// forms V = (C_0 + 2^8 C_1) + 2^16 (C_2 + 2^8 C_3) (C_0 and C_2 start at q
// so both halves are positive), reduces it by one Montgomery step to
// V 2^{-32} mod q, and multiplies by the next twist (stored as t 2^32, Shoup
// form), or, after a last matrix-core level whose twiddles carry the 2^32,
// leaves the canonical residue.  Twisted results are re-sliced into digits
// for the next contraction with two VALU operations.
//
// Data movement.  A work item is P rows x W columns (vectors) of one
// polynomial, 1024 words per wave (4 waves, or 8 for the wide items of the
// 256-point stage).  Items are staged through an LDS ring of three stages
// (two by default for the wide items, a plan parameter) by direct-to-LDS
// loads issued two (one) items ahead.  Each wave transforms four
// sets of vectors; a set fills the 16 rows of one MFMA tile with 16 / r
// vectors.  The intermediate array between the passes is tiled: block kb of
// 16 consecutive pass-1 outputs holds, for every pass-1 column c, the 16
// words (kb, c) contiguously, so pass 1 writes runs of whole lines (the wide
// first pass gathers each wave's results in a private LDS buffer and stores
// 256-byte runs) and pass 2 reads each item as one contiguous block.  The
// fusion's Montgomery step, the twist and the digit offset use 64-bit
// multiply-adds (v_mad_u64_u32 issues at the full VALU rate on gfx950), which
// keeps the passes close to the memory-only rate.  Pass 2 writes its canonical
// results back in natural order through the LDS stage it has just consumed;
// for forward transforms it can instead finish a ModDown / RESCALE step in
// that store (out (+)= (acc - y) m).
#include <algorithm>
#include <type_traits>

#include "ckks_internal.hpp"
#include "fourstep_dev.hpp"

namespace tfhe {
namespace {

// Geometry of a pass with P = 16 kR points.  A work item is P rows x W
// vectors (columns) of one polynomial, 1024 words per wave; each wave
// transforms four sets of vectors per item.  Its LDS tile is a sequence of
// 1 KiB slabs; slab k holds rows Rs k .. Rs k + Rs - 1 of every column of the
// item, slot L (16 bytes) row Rs k + L % Rs, columns 4 (L / Rs) .. + 3 (a
// "quad"), so one direct-to-LDS load covers Rs rows x W columns.  Narrow
// items (W = 16 for kR = 16) use 4 waves and Rs = 16: 64-byte row segments.
// Wide items (kR = 16 with at least 32 columns) use 8 waves and Rs = 8, so
// every load and store moves whole 128-byte lines.  For kR < 16, Rs = kR and
// W = 256 / kR >= 32.  Slabs are padded where 16 lanes of an LDS access
// would otherwise hit the same banks in several slabs.
template <bool kFirst, int kR, bool kWide>
struct Geo {
  static constexpr int waves = kWide ? 8 : 4;
  static constexpr int threads = 64 * waves;
  static constexpr int item = 1024 * waves;      // words per work item
  static constexpr int slabs = item / 256;
  static constexpr int P = 16 * kR;
  static constexpr int W = item / P;             // vectors per item
  static constexpr int Mt = 16 / kR;             // vectors per MFMA tile (quads per wave)
  static constexpr int Rs = kWide ? 8 : kR;      // rows per slab
  static constexpr int pitch = kWide ? 256 + 32 : (kFirst || kR == 16) ? 256 : 256 + 4 * kR;
  static constexpr int tile = slabs * pitch;
  static_assert(!kWide || kR == 16, "wide items are for the 256-point stage");
};

// Work distribution.  The grid is a multiple of 16.  Workgroup w belongs to
// group w / 16, which owns a contiguous range of polynomials; within the
// group, slot j = 2 (c % 8) + c / 8 of workgroup c = w % 16 selects its item
// column block (j mod items-per-polynomial) and its offset into the range
// (the group walks 16 / items-per-polynomial polynomials side by side).  A
// workgroup keeps its column block, so it reloads the limb's tables only when
// the limb changes.  Workgroups are dispatched round-robin over the 8 XCDs,
// each with its own L2: c and c + 8 own column blocks 2b and 2b + 1, which
// share the 128-byte lines of 64-byte row segments, on the same XCD.
struct Walk {
  uint32_t blk, p, step, p_end;
};
__device__ __forceinline__ Walk make_walk(uint32_t total_polys, uint32_t ipp_log) {
  const uint32_t groups = gridDim.x / 16, a = blockIdx.x / 16, c = blockIdx.x % 16;
  const uint32_t j = 2 * (c % 8) + c / 8;
  Walk w;
  w.blk = j & ((1u << ipp_log) - 1);
  w.step = 16u >> ipp_log;
  w.p = (uint32_t)((uint64_t)a * total_polys / groups) + (j >> ipp_log);
  w.p_end = (uint32_t)((uint64_t)(a + 1) * total_polys / groups);
  return w;
}

// Each wave loads slabs 4 wave .. 4 wave + 3 of an item: one 16-byte
// direct-to-LDS load per lane per slab (streaming hint: every byte is read
// once; a broadcast input, read once per limb, is loaded without it, which
// measured 3 % faster for RESCALE); lane L's bytes land at the slab base +
// 16 L.  Issued as inline assembly so that the compiler does not serialise
// later LDS reads on these loads: the pipeline waits for them explicitly
// (wait_item) before a barrier.
template <int kPitch>
__device__ __forceinline__ void issue_tile(const uint32_t* src, const uint32_t* off, uint32_t* stage,
                                           int wave, bool cached = false) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t* g = src + off[j];
    const uint32_t lds_addr = (uint32_t)(uintptr_t)(lds_void_t*)(stage + (4 * wave + j) * kPitch);
    if (cached)
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "global_load_lds_dwordx4 %1, off"
          :
          : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
          : "memory", "m0");
    else
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "global_load_lds_dwordx4 %1, off nt"
          :
          : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
          : "memory", "m0");
  }
}

// Wait until this wave's loads of the current item have landed.  Vector
// memory operations of a wave complete in issue order, so it suffices that at
// most as many operations remain outstanding as were issued after those
// loads.  With a ring of kRing stages the loads of item n are issued kRing - 1
// items ahead; each item then issues, in order, its epilogue loads (kE: 8
// with the store epilogue, else 0), the 4 ring loads of the item kRing - 1
// ahead and its kSt stores (16 in the narrow first passes, 4 otherwise).  In
// steady state that leaves the stores of item n - kRing + 1 and everything of
// the kRing - 2 items after it; near the start, the prologue's later loads
// and the first items' operations.  Without a next item everything is
// awaited.  Table loads issued in between only make the wait stricter.
template <int kRing, int kSt, int kE>
__device__ __forceinline__ void wait_item(uint32_t n, bool has_next) {
  static_assert(kRing == 2 || kRing == 3, "ring depth");
  constexpr int per = kE + 4 + kSt;  // operations of one item
  if (!has_next) wait_vmcnt<0>();
  else if (kRing == 2) {
    if (n == 0) wait_vmcnt<0>();
    else wait_vmcnt<kSt>();
  } else {
    if (n == 0) wait_vmcnt<4>();
    else if (n == 1) wait_vmcnt<per>();
    else wait_vmcnt<kSt + per>();
  }
}

template <bool kFirst, int kR, bool kWide, bool kEpi = false, int kRing = 3>
__global__ void __launch_bounds__(kWide ? 512 : 256, (kWide || kEpi) ? 2 : 3)
fs_pass(const FsTable tab) {
  static_assert(!kEpi || (!kFirst && kR == 16), "the epilogue belongs to the forward second pass");
  using G = Geo<kFirst, kR, kWide>;
  // The wide first pass gathers each wave's results in a private LDS buffer
  // (1024 words: 16 runs of 64 words, one per output block t, each a
  // contiguous 256-byte run of the tiled array) and stores them with
  // 16-byte stores; the narrow first passes store 64-byte runs directly.
  constexpr bool kGather = kFirst && kWide;
  __shared__ __attribute__((aligned(16))) uint32_t ring[kRing * G::tile + (kGather ? G::waves * 1024 : 0)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* const gather = kGather ? ring + kRing * G::tile + wave * 1024 : ring;
  const int i16 = lane & 15, g = lane >> 4;
  const Walk walk = make_walk(tab.total, tab.ipp_log);
  if (walk.p >= walk.p_end) return;
  const uint32_t S = tab.cols, c0 = walk.blk * G::W;

  // Per-lane word offsets within a polynomial.  Slab k = 4 wave + j, slot
  // L = lane: row Rs k + L % Rs, item column 4 (L / Rs).
  uint32_t ld_off[4], st_off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t row = G::Rs * (4 * wave + j) + lane % G::Rs, col = 4 * (lane / G::Rs);
    const uint32_t natural = row * S + c0 + col;
    const uint32_t tiled = ((c0 + col) >> 4) * (16 * G::P) + 16 * row + (col & 15);
    ld_off[j] = kFirst ? natural : tiled;
    if (kGather) {
      // 16 bytes of the run of output block t = 4 j + g: words 4 i16 ..
      st_off[j] = (4 * j + g) * 16 * S + (c0 + 4 * wave) * 16 + 4 * i16;
    } else if (kFirst) {
      // tiled store of output s + 16 t of column c0 + 4 (wave Mt + m) (+ set)
      int m, t;
      lane_out<kR>(g, j, m, t);
      st_off[j] = t * 16 * S + (c0 + 4 * (wave * G::Mt + m)) * 16 + i16;
    } else {
      st_off[j] = natural;
    }
  }

  uint32_t kf = 0, kc = 0;  // running unit indices of the load and compute walks
  auto issue = [&](uint32_t p, int stage) {
    const Item it = locate(tab, p, kf);
    issue_tile<G::pitch>(tab.u[it.unit].in + it.in_base, ld_off, ring + stage * G::tile, wave,
                         kFirst && tab.u[it.unit].in_bcast);
  };
#pragma unroll
  for (int j = 0; j < kRing - 1; ++j)
    if (walk.p + j * walk.step < walk.p_end) issue(walk.p + j * walk.step, j);

  const FourStepLimb* cur_limb = nullptr;
  uint32_t q = 0, qneg = 0, nq = 0;
  uint64_t cq = 0;  // 0x80808080 - q mod 2^32 (zero-extended), the twist's digit offset
  v4i opA[4], opB[4];
  uint2 tw[4];
  uint2 pt[4][4];  // pass 1: post-twist per set and register
  uint2 lb[4];     // kR < 16: rho^0..rho^3
  uint2 rj[4];     // kR = 8: multiplier of register j (rho^j or 1)
  uint2 pf[4];     // kR < 16, pass 2: per-output factor
  int st = 0;
  uint32_t n = 0;
  for (uint32_t p = walk.p; p < walk.p_end; p += walk.step, ++n, st = (st + 1 == kRing) ? 0 : st + 1) {
    const Item it = locate(tab, p, kc);
    const FourStepLimb* limb = tab.u[it.unit].limbs + it.limb;
    if (limb != cur_limb) {
      // rare (a few times per workgroup): completed here, so that the
      // steady-state path carries no wait on these loads
      const FourStepLimb L = *limb;
      const PassTables* P = kFirst ? L.pass1 : L.pass2;
      q = L.q;
      qneg = L.qneg;
      nq = 0u - q;
      cq = (uint32_t)(0x80808080u - q);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        opA[j] = *(const v4i*)&P->opA[j][lane][0];
        if (kR == 16) opB[j] = *(const v4i*)&P->opB[j][lane][0];
        tw[j] = P->twist[lane][j];
        if (kR < 16) {
          lb[j] = P->lb[j];
          int m, t;
          lane_out<kR>(g, j, m, t);
          pf[j] = P->lb[8 + t];
        }
      }
      if (kR == 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j) rj[j] = (g & 1) ? lb[j] : lb[0];
      }
      if (kFirst) {
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
          const uint2* pp = L.post1 + ((size_t)(c0 + 4 * wave * G::Mt + sg) * 64 + lane) * 4;
#pragma unroll
          for (int j = 0; j < 4; ++j) pt[sg][j] = pp[j];
        }
      }
      wait_vmcnt<0>();
      cur_limb = limb;
    }
    const bool has_next = p + walk.step < walk.p_end;
    wait_item<kRing, kFirst && !kWide ? 16 : 4, kEpi ? 8 : 0>(n, has_next);
    lds_barrier();  // the item's tile is complete; the oldest stage is free
    uint4 e_acc[4], e_out[4];  // epilogue operands at the item's store positions
    if (kEpi) {
      // a unit that overwrites its output (RESCALE, the second component of
      // a rotation) has no use for the old values: its second load re-reads
      // the lines the first has just fetched, so the count of loads that the
      // waits assume stays 8 per item without the output crossing HBM
      const FsUnit& U = tab.u[it.unit];
      const uint32_t* const eo = U.accumulate ? U.out : U.acc;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        e_acc[j] = *(const uint4*)(U.acc + it.poly_base + st_off[j]);
        e_out[j] = *(const uint4*)(eo + it.poly_base + st_off[j]);
      }
    }
    const bool issued = p + (kRing - 1) * walk.step < walk.p_end;
    if (issued) issue(p + (kRing - 1) * walk.step, (st + kRing - 1) % kRing);

    // lane (i, g) of wave w reads row kR (4g + c) + i % kR of the quad
    // w Mt + i / kR (four vectors, one per set): for 16 lanes either 256
    // contiguous bytes of one slab, or (wide) 128 bytes of two slabs
    uint32_t* const tile = ring + st * G::tile;
    uint4 rows[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int row = kR * (4 * g + c) + i16 % kR, quad = wave * G::Mt + i16 / kR;
      rows[c] = *(const uint4*)(tile + (row / G::Rs) * G::pitch + (quad * G::Rs + row % G::Rs) * 4);
    }

    uint32_t* const out = tab.u[it.unit].out + it.poly_base;
    uint4 res[4];  // pass 2: res[j] = the four sets' outputs of register j
    // The digit window needs a correction only for q > 0x7F7F7F7F; q is
    // uniform, so the item body is instantiated for both cases.
    auto body = [&](auto big_q) {
      constexpr bool kBigQ = decltype(big_q)::value;
#pragma unroll
      for (int sg = 0; sg < 4; ++sg) {
        v4i x;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t w = sg == 0 ? rows[c].x : sg == 1 ? rows[c].y : sg == 2 ? rows[c].z : rows[c].w;
          x[c] = kFirst ? (int)balanced_digits(kBigQ ? to_window(w, q) : (int32_t)w) : (int)w;
        }
        const v4i bias = {(int)q, (int)q, (int)q, (int)q};
        const v4i zero = {0, 0, 0, 0};
        const v4i a0 = mfma(x, opA[0], bias);
        const v4i a1 = mfma(x, opA[1], zero);
        const v4i a2 = mfma(x, opA[2], bias);
        const v4i a3 = mfma(x, opA[3], zero);
        uint32_t y[4];
        if (kR == 16) {
          v4i z;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            z[j] = (int)twist_digits<kBigQ>(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw[j], q, nq, cq);
          const v4i b0 = mfma(opB[0], z, bias);
          const v4i b1 = mfma(opB[1], z, zero);
          const v4i b2 = mfma(opB[2], z, bias);
          const v4i b3 = mfma(opB[3], z, zero);
#pragma unroll
          for (int j = 0; j < 4; ++j) y[j] = fuse_redc(b0[j], b1[j], b2[j], b3[j], q, qneg);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            y[j] = reduce_once(mul_shoup_lazy(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw[j].x, tw[j].y, q), q);
          level_b<kR>(y, lb, rj, g, q);
        }
        if (kGather) {
          // output 16 t + i16 (t = 4 g + j) of column 4 wave + sg: word
          // 16 sg + i16 of run t, with bits 4-5 XOR g (= t / 4) so that the
          // four lane groups write disjoint banks
#pragma unroll
          for (int j = 0; j < 4; ++j)
            gather[(4 * g + j) * 64 + 16 * (sg ^ g) + i16] = twist_digits<kBigQ>(y[j], pt[sg][j], q, nq, cq);
        } else if (kFirst) {
#pragma unroll
          for (int j = 0; j < 4; ++j) out[st_off[j] + 16 * sg] = twist_digits<kBigQ>(y[j], pt[sg][j], q, nq, cq);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t r = kR == 16 ? reduce_once(y[j], q) : mul_shoup(y[j], pf[j].x, pf[j].y, q);
            if (sg == 0) res[j].x = r;
            else if (sg == 1) res[j].y = r;
            else if (sg == 2) res[j].z = r;
            else res[j].w = r;
          }
        }
      }
    };
    // (the narrow first pass of the 256-point stage keeps one body: two
    // would not fit its register budget without spilling).  A broadcast
    // input (below 2^31, not reduced by this limb's modulus) takes the body
    // that maps its values into the digit window.
    constexpr bool kDual = !(kFirst && kR == 16 && !kWide);
    if (!kDual || q > 0x7F7F7F7Fu || (kFirst && tab.u[it.unit].in_bcast)) body(std::true_type{});
    else body(std::false_type{});

    if (kGather) {
      // this wave's runs t = 4 j + g, words 4 i16 .. 4 i16 + 3 (unswizzled).
      // A wave's LDS accesses complete in order; the compiler fence keeps the
      // 16-byte reads after the 4-byte writes (different access types).
      asm volatile("" ::: "memory");
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = 4 * j + g;
        __builtin_nontemporal_store(*(const v4u*)(gather + t * 64 + 16 * ((i16 >> 2) ^ j) + 4 * (i16 & 3)),
                                    (v4u*)(out + st_off[j]));
      }
    }
    if (!kFirst) {
      // results into the consumed stage in the slab layout, then 16-byte
      // streaming stores with the load's lane mapping (whole lines; the
      // first pass keeps cached stores, whose 64-byte halves merge in L2)
      lds_barrier();  // every wave has read the stage
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int m, t;
        lane_out<kR>(g, j, m, t);
        const int row = i16 + 16 * t;
        *(uint4*)(tile + (row / G::Rs) * G::pitch + ((wave * G::Mt + m) * G::Rs + row % G::Rs) * 4) = res[j];
      }
      lds_barrier();
      if (kEpi) {
        // only the ring loads of item n + 2 were issued after the epilogue loads
        if (issued) wait_vmcnt<4>();
        else wait_vmcnt<0>();
        const FsUnit& U = tab.u[it.unit];
        const uint2 m = U.mult[it.limb];
        const bool add = U.accumulate != 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint4 y = *(const uint4*)(tile + (4 * wave + j) * G::pitch + lane * 4);
          uint4 r;
          r.x = mul_shoup(sub_mod(e_acc[j].x, y.x, q), m.x, m.y, q);
          r.y = mul_shoup(sub_mod(e_acc[j].y, y.y, q), m.x, m.y, q);
          r.z = mul_shoup(sub_mod(e_acc[j].z, y.z, q), m.x, m.y, q);
          r.w = mul_shoup(sub_mod(e_acc[j].w, y.w, q), m.x, m.y, q);
          if (add) {
            r.x = add_mod(r.x, e_out[j].x, q);
            r.y = add_mod(r.y, e_out[j].y, q);
            r.z = add_mod(r.z, e_out[j].z, q);
            r.w = add_mod(r.w, e_out[j].w, q);
          }
          __builtin_nontemporal_store(*(const v4u*)&r, (v4u*)(out + st_off[j]));
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          __builtin_nontemporal_store(*(const v4u*)(tile + (4 * wave + j) * G::pitch + lane * 4), (v4u*)(out + st_off[j]));
      }
    }
  }
}

// Resident workgroups per CU of a pass kernel (queried once per process).
template <bool kFirst, int kR, bool kWide, bool kEpi, int kRing>
uint32_t occupancy() {
  static std::atomic<int> occ{0};
  return (uint32_t)occupancy_cached(occ, fs_pass<kFirst, kR, kWide, kEpi, kRing>, Geo<kFirst, kR, kWide>::threads);
}

// Persistent grid: a multiple of 16 workgroups, no more than the items need.
template <bool kFirst, int kR, bool kWide, bool kEpi, int kRing>
uint32_t grid_size(const tfhe_ntt_plan_s* p, uint32_t items) {
  // default: the resident count; twice that for the wide kernels (one or
  // two resident workgroups per CU), whose tail balances better with the
  // second half of the grid scheduled as the first half drains (measured)
  const uint32_t w =
      p->fs_wg_per_cu ? p->fs_wg_per_cu : occupancy<kFirst, kR, kWide, kEpi, kRing>() * (kWide ? 2 : 1);
  const uint32_t g = std::max(16u, (p->num_cus * w) / 16 * 16);
  return std::min(g, (items + 15) / 16 * 16);
}

template <bool kFirst, int kR, bool kWide, bool kEpi, int kRing>
void launch_ring(const tfhe_ntt_plan_s* p, FsTable t, hipStream_t s) {
  using G = Geo<kFirst, kR, kWide>;
  t.ipp_log = t.log_n - (kWide ? 13 : 12);  // items per polynomial: N / item words
  const uint32_t grid = grid_size<kFirst, kR, kWide, kEpi, kRing>(p, t.total << t.ipp_log);
  TFHE_TIMED(kFirst ? K_FS_PASS1 : K_FS_PASS2, s,
             hipLaunchKernelGGL((fs_pass<kFirst, kR, kWide, kEpi, kRing>), dim3(grid), dim3(G::threads), 0, s, t));
}

// LDS ring depth of a pass: for the wide items of the 256-point stage the
// plan's fs_ring, by default 2 (measured 1-2 % faster than 3 at N = 2^15
// and 2^16); narrow items keep 3 (2 measured 5-20 % slower at N = 2^12..
// 2^14, and the narrow first passes would spill registers).
template <bool kFirst, int kR, bool kWide, bool kEpi = false>
void launch_pass(const tfhe_ntt_plan_s* p, FsTable t, hipStream_t s) {
  if constexpr (kWide) {
    if (p->fs_ring != 3) {
      launch_ring<kFirst, kR, kWide, kEpi, 2>(p, t, s);
      return;
    }
  }
  launch_ring<kFirst, kR, kWide, kEpi, 3>(p, t, s);
}

// The 256-point stage uses wide items by default when the pass has >= 128
// columns (N >= 2^15); below that the narrow items leave more work items per
// polynomial, which measured faster.  The plan's fs_wide overrides this.
static bool use_wide(const tfhe_ntt_plan_s* p, uint32_t cols) {
  return p->fs_wide == 1 ? false : cols >= (p->fs_wide == 2 ? 32u : 128u);
}

template <bool kFirst>
void launch_pass_r(const tfhe_ntt_plan_s* p, uint32_t r, const FsTable& t, hipStream_t s) {
  switch (r) {
    case 1: launch_pass<kFirst, 1, false>(p, t, s); break;
    case 2: launch_pass<kFirst, 2, false>(p, t, s); break;
    case 4: launch_pass<kFirst, 4, false>(p, t, s); break;
    case 8: launch_pass<kFirst, 8, false>(p, t, s); break;
    default:
      if (use_wide(p, t.cols))
        launch_pass<kFirst, 16, true>(p, t, s);
      else launch_pass<kFirst, 16, false>(p, t, s);
      break;
  }
}


// ---------------------------------------------------------------------------
// Second pass of the ModUp forward transforms fused with the key inner
// product (Sec. IV-A, Table 2: NTT, then Inner-product): a workgroup takes
// one level group's extended-basis position t, batch element b and column
// block (an "item"), and for every digit j (a "task") either runs the second
// pass (the 256-point stage) on digit j's tiled intermediate of t, or, for
// the digit that holds t, takes d2[t] as it is;
// it multiplies the result by evk_j[c][t] at its natural positions and, after
// the last digit, writes acc_0 and acc_1 once.  The transformed limbs are
// never written: the separate transform store and the inner product's re-read
// of them disappear.  Products are summed as 64-bit values kept below
// q 2^32 and reduced once per output; every quantity is exact, so the
// result equals the unfused sequence bit for bit.  Items of all level groups
// form one sequence (group g from item0): one launch for a mixed-level batch.
// Pipelining: the task's source (tile or d2) and its two key blocks arrive
// by direct-to-LDS loads; the next task's source is issued into the other
// buffer as soon as this task's has landed, so one load is always in flight
// behind the arithmetic.  Keys and d2 are loaded into each wave's own slots
// of the output layout (slot (4 wave + j, lane) = natural positions st_off).
// Items are the wide ones of the 256-point stage (8 waves, 32 vectors: every
// load and store a whole 128-byte line, 144 KiB of LDS, one workgroup per
// CU) wherever N >= 2^13, else the narrow ones (4 waves, 16 vectors, two
// workgroups per CU); wide measured 2 % faster for this kernel at 2^16.
template <bool kWide>
__global__ void __launch_bounds__(kWide ? 512 : 256, kWide ? 1 : 2)
ip_pass(const IpSet set, const FourStepLimb* __restrict__ limbs, const ModConst* __restrict__ mods,
        uint32_t log_n, uint32_t ipp, uint32_t items) {
  using G = Geo<false, 16, kWide>;
  // two source buffers, then the key blocks of components 0 and 1
  __shared__ __attribute__((aligned(16))) uint32_t lds[4 * G::tile];
  uint32_t* const kbuf = lds + 2 * G::tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const uint64_t N = 1ull << log_n;
  const uint32_t S = (uint32_t)(N >> 8);  // second-pass columns (rows of the first)
  const uint64_t kplane = (uint64_t)(set.L + set.K) * N;  // one key component
  // per-lane offsets within a polynomial for column block blk
  auto offsets = [&](uint32_t blk, uint32_t* ld, uint32_t* st) {
    const uint32_t c0 = blk * G::W;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t row = G::Rs * (4 * wave + j) + lane % G::Rs, col = 4 * (lane / G::Rs);
      st[j] = row * S + c0 + col;
      ld[j] = ((c0 + col) >> 4) * (16 * G::P) + 16 * row + (col & 15);
    }
  };
  struct Pos {
    uint32_t grp, b, blk, t, pl, own;
  };
  auto pos_of = [&](uint32_t w) {
    Pos p;
    p.grp = 0;
    while (p.grp + 1 < set.count && set.g[p.grp + 1].item0 <= w) ++p.grp;
    const IpGroup& Gr = set.g[p.grp];
    const uint32_t l = w - Gr.item0;
    p.b = l % Gr.batch;
    const uint32_t tb = l / Gr.batch;
    p.blk = tb % ipp;
    p.t = tb / ipp;
    p.pl = p.t < Gr.level ? p.t : set.L + (p.t - Gr.level);  // plan limb
    p.own = p.t < Gr.level ? p.t / set.alpha : 0xFFFFFFFFu;
    return p;
  };
  // 16 bytes per lane into this wave's slot (4 wave + j) of `dst` (output layout)
  auto load_slots = [&](const uint32_t* src, const uint32_t* st, uint32_t* dst) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t lds_addr = (uint32_t)(uintptr_t)(lds_void_t*)(dst + (4 * wave + j) * G::pitch);
      asm volatile(
          "s_mov_b32 m0, %0\n\t"
          "global_load_lds_dwordx4 %1, off"
          :
          : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(src + st[j])
          : "memory", "m0");
    }
  };
  // the source of task (position p, digit jd) into buffer buf: 4 loads per lane
  auto issue_source = [&](const Pos& p, uint32_t jd, int buf) {
    const IpGroup& Gr = set.g[p.grp];
    const uint32_t ext = Gr.level + set.K;
    uint32_t ld[4], st[4];
    offsets(p.blk, ld, st);
    if (jd == p.own)
      load_slots(Gr.d2 + ((uint64_t)p.t * Gr.batch + p.b) * N, st, lds + buf * G::tile);
    else
      issue_tile<G::pitch>(Gr.src + ((uint64_t)(jd * ext + p.t) * Gr.batch + p.b) * N, ld, lds + buf * G::tile,
                           wave);
  };

  uint32_t w = blockIdx.x, jd = 0;
  if (w >= items) return;
  Pos p = pos_of(w);

  const FourStepLimb* cur = nullptr;
  v4i opA[4], opB[4];
  uint2 tw[4];
  uint32_t q = 0, qneg = 0, nq = 0;
  uint64_t cq = 0;
  ModConst m{};
  uint64_t s0[4][4], s1[4][4];  // sums of products, kept below q 2^32
  issue_source(p, 0, 0);
  bool stored_after = false;  // the previous task ended its item (8 stores after this source)
  for (int cb = 0;; cb ^= 1) {
    uint32_t* const src = lds + cb * G::tile;
    const IpGroup& Gr = set.g[p.grp];
    // the task after this one: the next digit, else the next item
    uint32_t nw = w, njd = jd + 1;
    if (njd == Gr.digits) {
      nw = w + gridDim.x;
      njd = 0;
    }
    const bool next = nw < items;
    uint32_t ld[4], st[4];
    offsets(p.blk, ld, st);
    // this task's source: issued before the previous task's stores (if any)
    if (stored_after) wait_vmcnt<8>();
    else wait_vmcnt<0>();
    if (jd == 0 && limbs + p.pl != cur) {
      // rare: completed here, so that the pipeline carries no wait on these
      cur = limbs + p.pl;
      const FourStepLimb L = *cur;
      q = L.q;
      qneg = L.qneg;
      nq = 0u - q;
      cq = (uint32_t)(0x80808080u - q);
      m = mods[p.pl];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        opA[j] = *(const v4i*)&L.pass2->opA[j][lane][0];
        opB[j] = *(const v4i*)&L.pass2->opB[j][lane][0];
        tw[j] = L.pass2->twist[lane][j];
      }
      // the builtin (unlike an asm wait) tells the compiler these registers
      // are ready, so it adds no vmcnt(0) at their first use downstream
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    }
    lds_barrier();  // the source is in LDS; every wave is done with the other buffer and the keys
    // this task's keys, then the next task's source
    const uint32_t* key = set.keys.k[set.keys.count == 1 ? 0 : Gr.key0 + p.b];
    const uint32_t* krow = key + (uint64_t)jd * 2 * kplane + (uint64_t)p.pl * N;
    load_slots(krow, st, kbuf);
    load_slots(krow + kplane, st, kbuf + G::tile);
    Pos np = p;
    if (next) {
      if (nw != w) np = pos_of(nw);
      issue_source(np, njd, cb ^ 1);
    }
    if (jd == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) s0[j][e] = s1[j][e] = 0;
    }
    if (jd != p.own) {
      uint4 rows[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int row = 16 * (4 * g + c) + i16;
        rows[c] = *(const uint4*)(src + (row / G::Rs) * G::pitch + (wave * G::Rs + row % G::Rs) * 4);
      }
      uint4 res[4];
      auto body = [&](auto big_q) {
        constexpr bool kBigQ = decltype(big_q)::value;
        const v4i bias = {(int)q, (int)q, (int)q, (int)q};
        const v4i zero = {0, 0, 0, 0};
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
          v4i x;
#pragma unroll
          for (int c = 0; c < 4; ++c)
            x[c] = (int)(sg == 0 ? rows[c].x : sg == 1 ? rows[c].y : sg == 2 ? rows[c].z : rows[c].w);
          const v4i a0 = mfma(x, opA[0], bias);
          const v4i a1 = mfma(x, opA[1], zero);
          const v4i a2 = mfma(x, opA[2], bias);
          const v4i a3 = mfma(x, opA[3], zero);
          v4i z;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            z[j] = (int)twist_digits<kBigQ>(fuse_redc(a0[j], a1[j], a2[j], a3[j], q, qneg), tw[j], q, nq, cq);
          const v4i b0 = mfma(opB[0], z, bias);
          const v4i b1 = mfma(opB[1], z, zero);
          const v4i b2 = mfma(opB[2], z, bias);
          const v4i b3 = mfma(opB[3], z, zero);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t r = reduce_once(fuse_redc(b0[j], b1[j], b2[j], b3[j], q, qneg), q);
            if (sg == 0) res[j].x = r;
            else if (sg == 1) res[j].y = r;
            else if (sg == 2) res[j].z = r;
            else res[j].w = r;
          }
        }
      };
      if (q > 0x7F7F7F7Fu) body(std::true_type{});
      else body(std::false_type{});
      lds_barrier();  // every wave has read the source
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = i16 + 16 * (4 * g + j);
        *(uint4*)(src + (row / G::Rs) * G::pitch + (wave * G::Rs + row % G::Rs) * 4) = res[j];
      }
    }
    // the keys (issued before the next source) have landed; the results in
    // the output layout are complete in every wave
    if (next) wait_vmcnt<4>();
    else wait_vmcnt<0>();
    lds_barrier();
    // s += y k as one 64-bit multiply-add; with y, k < q < 2^31 the sum
    // stays below q 2^32 + q^2 < 2^64, and taking q off its high word when
    // that reaches q keeps s below q 2^32.  Whole-vector 16-byte reads:
    // through uint4 the compiler splits the key reads into dword pairs,
    // which conflict four ways across the wave.
    auto mac = [&](uint64_t* acc, const v4u& y, const v4u& kk) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t v = mad_u64(y[e], kk[e], acc[e]);
        const uint32_t hi = (uint32_t)(v >> 32);
        acc[e] = ((uint64_t)min(hi, hi - q) << 32) | (uint32_t)v;
      }
    };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int slot = (4 * wave + j) * G::pitch + lane * 4;
      const v4u y = *(const v4u*)(src + slot);
      mac(s0[j], y, *(const v4u*)(kbuf + slot));
      mac(s1[j], y, *(const v4u*)(kbuf + G::tile + slot));
    }
    stored_after = jd + 1 == Gr.digits;
    if (stored_after) {
      // s mod q: one Montgomery step (s + m q < 2q 2^32), then times 2^32
      auto fin = [&](uint64_t v) {
        const uint32_t mm = (uint32_t)v * qneg;
        return mul_shoup(reduce_once((uint32_t)(mad_u64(mm, q, v) >> 32), q), m.r, m.rp, q);
      };
      const uint32_t ext = Gr.level + set.K;
      uint32_t* o0 = Gr.acc + ((uint64_t)p.t * Gr.batch + p.b) * N;
      uint32_t* o1 = Gr.acc + ((uint64_t)(ext + p.t) * Gr.batch + p.b) * N;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const v4u r0 = {fin(s0[j][0]), fin(s0[j][1]), fin(s0[j][2]), fin(s0[j][3])};
        const v4u r1 = {fin(s1[j][0]), fin(s1[j][1]), fin(s1[j][2]), fin(s1[j][3])};
        __builtin_nontemporal_store(r0, (v4u*)(o0 + st[j]));
        __builtin_nontemporal_store(r1, (v4u*)(o1 + st[j]));
      }
    }
    if (!next) break;
    w = nw;
    jd = njd;
    p = np;
  }
}

// ---------------------------------------------------------------------------
// Vector-ALU GEMM variant ("CO", Sec. IV-B: the NTT as matrix products on
// the general-purpose cores, one modular reduction per output), N = 2^16.
// Same passes, tables, work items and data movement as the matrix-core
// kernel (narrow items); each 16-point level is a 16 x 16 matrix product in
// which a thread forms one output from 16 full products of canonical
// residues summed in 96 bits and reduced once by two Montgomery steps
// against matrices stored as W 2^64 mod q ("reduce every 16").
//   level A: thread (v, col) computes Y[s][v] = T[s][v] sum_u WA[u][s] x[16u+v]
//   level B: thread (s, col) computes out[s+16t] = sum_v WB[t][v] Y[s][v]
// Level-A results go through LDS at (col 16 + s) 17 + v, conflict-free for
// both access patterns.
// One multiply-accumulate step of a 96-bit sum: acc + a b as one
// v_mad_u64_u32 whose carry-out (through VCC) is added into k.
__device__ __forceinline__ uint64_t mac96(uint32_t a, uint32_t b, uint64_t acc, uint32_t& k) {
  uint64_t d;
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %4\n\tv_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
      : "=&v"(d), "+v"(k)
      : "v"(a), "v"(b), "v"(acc)
      : "vcc");
  return d;
}

// S 2^{-64} mod q in [0, q) for S = k 2^64 + acc < 2^67 (sixteen products of
// residues below 2^31): two Montgomery steps.  The first leaves
// T = (S + m1 q) / 2^32 < 2^36, the second (T + m2 q) / 2^32 < q + 16.
__device__ __forceinline__ uint32_t redc96(uint64_t acc, uint32_t k, uint32_t q, uint32_t qneg) {
  const uint32_t m1 = (uint32_t)acc * qneg;
  const uint64_t t = mac96(m1, q, acc, k);  // low word 0
  const uint32_t th = (uint32_t)(t >> 32);
  const uint32_t m2 = th * qneg;
  const uint32_t u = (uint32_t)(mad_u64(m2, q, ((uint64_t)k << 32) | th) >> 32);
  return reduce_once(u, q);
}

template <bool kFirst>
__global__ void __launch_bounds__(256)
co_pass(const FsTable tab) {
  using G = Geo<kFirst, 16, false>;
  constexpr int kCoStages = 2;  // one item ahead: leaves LDS for three workgroups per CU
  __shared__ __attribute__((aligned(16))) uint32_t ring[kCoStages * G::tile];
  __shared__ uint32_t ybuf[16 * 16 * 17];
  __shared__ __attribute__((aligned(16))) uint32_t mats[512];  // WA[s][u] then WB[t][v] (broadcast reads)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo16 = tid & 15, col = tid >> 4;  // level A: v = lo16; level B: s = lo16
  const Walk walk = make_walk(tab.total, tab.ipp_log);
  if (walk.p >= walk.p_end) return;
  const uint32_t S = tab.cols, c0 = walk.blk * G::W;

  uint32_t ld_off[4], st_off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t row = 16 * (4 * wave + j) + lane % 16, c4 = 4 * (lane / 16);
    const uint32_t natural = row * S + c0 + c4;
    const uint32_t tiled = ((c0 + c4) >> 4) * (16 * G::P) + 16 * row + (c4 & 15);
    ld_off[j] = kFirst ? natural : tiled;
    st_off[j] = natural;
  }
  uint32_t kf = 0, kc = 0;
  auto issue = [&](uint32_t p, int stage) {
    const Item it = locate(tab, p, kf);
    issue_tile<G::pitch>(tab.u[it.unit].in + it.poly_base, ld_off, ring + stage * G::tile, wave);
  };
  issue(walk.p, 0);

  const FourStepLimb* cur_limb = nullptr;
  const CoPass* M = nullptr;
  uint32_t q = 0, qneg = 0;
  uint2 tv[16], post[16];  // T[s][v] of this thread's v; post-twist of (col, s + 16 t)
  int st = 0;
  uint32_t n = 0;
  for (uint32_t p = walk.p; p < walk.p_end; p += walk.step, ++n, st ^= 1) {
    const Item it = locate(tab, p, kc);
    const FourStepLimb* limb = tab.u[it.unit].limbs + it.limb;
    if (limb != cur_limb) {
      const FourStepLimb L = *limb;
      M = kFirst ? L.co1 : L.co2;
      q = L.q;
      qneg = L.qneg;
      lds_barrier();  // every wave is done with the previous limb's matrices
      mats[tid] = M->WA[tid >> 4][tid & 15];
      mats[256 + tid] = M->WB[tid >> 4][tid & 15];
#pragma unroll
      for (int s2 = 0; s2 < 16; ++s2) tv[s2] = M->T[s2][lo16];
      if (kFirst) {
#pragma unroll
        for (int t = 0; t < 16; ++t) post[t] = L.co_post[(c0 + col) * 256 + lo16 + 16 * t];
      }
      wait_vmcnt<0>();
      cur_limb = limb;
    }
    // this item's loads were followed only by the previous item's stores
    if (n == 0) wait_vmcnt<0>();
    else if (kFirst) wait_vmcnt<16>();
    else wait_vmcnt<4>();
    lds_barrier();  // also publishes a new limb's matrices; the other stage is free
    if (p + walk.step < walk.p_end) issue(p + walk.step, st ^ 1);
    uint32_t* const tile = ring + st * G::tile;
    // level A
    uint32_t x[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = tile[u * G::pitch + ((col >> 2) * 16 + lo16) * 4 + (col & 3)];
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
      uint64_t acc = 0;
      uint32_t k = 0;
#pragma unroll
      for (int u4 = 0; u4 < 4; ++u4) {
        const uint4 w = *(const uint4*)(mats + s2 * 16 + 4 * u4);
        acc = mac96(x[4 * u4], w.x, acc, k);
        acc = mac96(x[4 * u4 + 1], w.y, acc, k);
        acc = mac96(x[4 * u4 + 2], w.z, acc, k);
        acc = mac96(x[4 * u4 + 3], w.w, acc, k);
      }
      ybuf[(col * 16 + s2) * 17 + lo16] = mul_shoup(redc96(acc, k, q, qneg), tv[s2].x, tv[s2].y, q);
    }
    lds_barrier();
    // level B
    uint32_t y[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) y[v] = ybuf[(col * 16 + lo16) * 17 + v];
    uint32_t* const out = tab.u[it.unit].out + it.poly_base;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      uint64_t acc = 0;
      uint32_t k = 0;
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const uint4 w = *(const uint4*)(mats + 256 + t * 16 + 4 * v4);
        acc = mac96(y[4 * v4], w.x, acc, k);
        acc = mac96(y[4 * v4 + 1], w.y, acc, k);
        acc = mac96(y[4 * v4 + 2], w.z, acc, k);
        acc = mac96(y[4 * v4 + 3], w.w, acc, k);
      }
      const uint32_t r = redc96(acc, k, q, qneg);
      if (kFirst) {
        // post-twist, tiled store: block t, column c0 + col, word s
        out[t * 16 * S + (c0 + col) * 16 + lo16] = mul_shoup(r, post[t].x, post[t].y, q);
      } else {
        // into the consumed stage: row s + 16 t, column col, slab layout
        tile[t * G::pitch + ((col >> 2) * 16 + lo16) * 4 + (col & 3)] = r;
      }
    }
    if (!kFirst) {
      lds_barrier();
#pragma unroll
      for (int j = 0; j < 4; ++j)
        __builtin_nontemporal_store(*(const v4u*)(tile + (4 * wave + j) * G::pitch + lane * 4), (v4u*)(out + st_off[j]));
    }
  }
}

template <bool kFirst>
void co_launch(const tfhe_ntt_plan_s* p, FsTable t, hipStream_t s) {
  t.ipp_log = t.log_n - 12;
  static std::atomic<int> occ{0};
  const uint32_t w = p->fs_wg_per_cu ? p->fs_wg_per_cu : (uint32_t)occupancy_cached(occ, co_pass<kFirst>, 256);
  const uint32_t items = t.total << t.ipp_log;
  const uint32_t grid = std::min(std::max(16u, (p->num_cus * w) / 16 * 16), (items + 15) / 16 * 16);
  TFHE_TIMED(kFirst ? K_CO_PASS1 : K_CO_PASS2, s,
             hipLaunchKernelGGL((co_pass<kFirst>), dim3(grid), dim3(256), 0, s, t));
}

}  // namespace

bool fs_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 16; }

size_t unit_ws_bytes(const NttUnit& u, bool mfma) {
  if (mfma) return (size_t)u.limb_count * u.batch * u.plan->n * sizeof(uint32_t);
  return bf_workspace_bytes(u.plan, u.limb_count, u.batch);
}

size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

// Whether a launch of `polys` four-step transforms of this plan takes the
// one-pass kernel: always with fs_passes 1, never with 2; by default at
// N = 2^12..2^14 when the launch gives every CU at least two polynomials
// (one workgroup holds one whole polynomial, so a smaller launch leaves CUs
// idle: HMULT at N = 2^14, batch 1-4, ran 10-20 % slower with every
// transform on it; with the rule HMULT at batch 8-64 is 2-8 % faster at
// 2^12..2^14 and unchanged below; at 2^15 the kernel is slower).
static bool use_onepass(const tfhe_ntt_plan_s* p, uint64_t polys) {
  if (!op_supported(p->log_n) || p->fs_passes == 2) return false;
  if (p->fs_passes == 1) return true;
  return p->log_n <= 14 && polys >= 2ull * p->num_cus;
}

// Fused launches: units are grouped by (N, direction), in order of first
// appearance; per group, pass 1 of every unit (in -> unit workspace), then
// pass 2 of every unit (workspace -> out), kMaxUnits units per launch pair.
// Units are independent, so the grouping does not change any result.
hipError_t fs_run_units(const NttUnit* units, uint32_t count, void* ws, hipStream_t s) {
  // workspace slices in unit order
  std::vector<uint32_t*> mids(count);
  {
    unsigned char* w = (unsigned char*)ws;
    for (uint32_t k = 0; k < count; ++k) {
      if (units[k].pass1_only) {  // the caller's intermediate
        mids[k] = units[k].out;
        continue;
      }
      mids[k] = (uint32_t*)w;
      w += (unit_ws_bytes(units[k], true) + 255) & ~(size_t)255;
    }
  }
  std::vector<bool> done(count, false);
  for (uint32_t lead = 0; lead < count; ++lead) {
    if (done[lead]) continue;
    const uint32_t log_n = units[lead].plan->log_n;
    const bool inverse = units[lead].inverse;
    const bool epi = units[lead].acc != nullptr;
    const bool p1only = units[lead].pass1_only;
    const bool bcast = units[lead].in_bcast;
    if ((epi || p1only || bcast) && inverse) return hipErrorInvalidValue;
    const tfhe_ntt_plan_s* p0 = units[lead].plan;
    const uint32_t N = 1u << log_n, N1 = N >> 8, r = N1 / 16;
    FsTable t1, t2;
    t1.log_n = t2.log_n = log_n;
    t1.cols = inverse ? N1 : 256;  // N / P of pass 1
    t2.cols = inverse ? 256 : N1;
    const uint32_t r1 = inverse ? 16 : r, r2 = inverse ? r : 16;
    // one HBM round trip where the one-pass kernel covers the shape and
    // the group's polynomials fill the CUs
    uint64_t group_polys = 0;
    for (uint32_t k = lead; k < count; ++k) {
      const NttUnit& u = units[k];
      if (!done[k] && u.plan->log_n == log_n && u.inverse == inverse && (u.acc != nullptr) == epi &&
          u.pass1_only == p1only && u.in_bcast == bcast)
        group_polys += (uint64_t)u.limb_count * u.batch;
    }
    const bool one = !epi && !p1only && !bcast && use_onepass(p0, group_polys);
    auto flush = [&]() {
      if (t1.total == 0) return;
      if (one) {
        (void)op_run(p0, inverse, t1, s);
        return;
      }
      launch_pass_r<true>(p0, r1, t1, s);
      if (p1only) return;
      if (!epi) launch_pass_r<false>(p0, r2, t2, s);
      else if (use_wide(p0, t2.cols)) launch_pass<false, 16, true, true>(p0, t2, s);
      else launch_pass<false, 16, false, true>(p0, t2, s);
    };
    t1.count = t2.count = 0;
    t1.total = t2.total = 0;
    for (uint32_t k = lead; k < count; ++k) {
      const NttUnit& u = units[k];
      if (done[k] || u.plan->log_n != log_n || u.inverse != inverse || (u.acc != nullptr) != epi ||
          u.pass1_only != p1only || u.in_bcast != bcast)
        continue;
      done[k] = true;
      const uint32_t polys = u.limb_count * u.batch;
      if (polys == 0) continue;
      if (t1.count == kMaxUnits) {
        flush();
        t1.count = t2.count = 0;
        t1.total = t2.total = 0;
      }
      const FourStepLimb* tabs = (u.inverse ? u.plan->d_fs_inv : u.plan->d_fs_fwd) + u.limb_begin;
      t1.u[t1.count++] = FsUnit{u.in, one ? u.out : mids[k], tabs, u.batch, t1.total, nullptr, nullptr, 0,
                                u.in_bcast ? 1u : 0u};
      t2.u[t2.count++] = FsUnit{mids[k], u.out, tabs, u.batch, t2.total, u.acc, u.epi_mult, u.epi_add ? 1u : 0u, 0};
      t1.total += polys;
      t2.total += polys;
    }
    flush();
  }
  return hipGetLastError();
}

template <bool kWide>
static hipError_t ip_launch(const tfhe_ntt_plan_s* p, IpSet& set, hipStream_t s) {
  using G = Geo<false, 16, kWide>;
  const uint32_t ipp = p->n / G::item;  // second-pass items per polynomial (>= 1)
  static std::atomic<int> occ{0};
  const int resident = occupancy_cached(occ, ip_pass<kWide>, G::threads);
  uint64_t items = 0;
  for (uint32_t g = 0; g < set.count; ++g) {
    set.g[g].item0 = (uint32_t)items;
    items += (uint64_t)(set.g[g].level + set.K) * ipp * set.g[g].batch;
  }
  if (items == 0) return hipSuccess;
  if (items >= (1ull << 32)) return hipErrorInvalidValue;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(items, (uint64_t)p->num_cus * resident);
  TFHE_TIMED(K_IP, s,
             hipLaunchKernelGGL(ip_pass<kWide>, dim3(grid), dim3(G::threads), 0, s, set, p->d_fs_fwd, p->d_mod,
                                p->log_n, ipp, (uint32_t)items));
  return hipGetLastError();
}

hipError_t ip_run(const tfhe_ntt_plan_s* p, IpSet& set, hipStream_t s) {
  if (set.count == 0) return hipSuccess;
  if (!p->has_mfma) return hipErrorInvalidValue;
  // wide items need 32 columns of the 256-point stage (N >= 2^13); a plan
  // that asks for narrow items (fs_wide 1) keeps them here too
  if (p->fs_wide != 1 && (p->n >> 8) >= 32) return ip_launch<true>(p, set, s);
  return ip_launch<false>(p, set, s);
}

hipError_t co_transform(const tfhe_ntt_plan_s* p, bool inverse, const uint32_t* in, uint32_t* out,
                        void* ws, uint32_t limb_begin, uint32_t limb_count, uint32_t batch,
                        hipStream_t s) {
  if (!p->has_co) return hipErrorInvalidValue;
  const FourStepLimb* tabs = (inverse ? p->d_fs_inv : p->d_fs_fwd) + limb_begin;
  FsTable t1, t2;
  t1.count = t2.count = 1;
  t1.total = t2.total = limb_count * batch;
  t1.log_n = t2.log_n = p->log_n;
  t1.cols = t2.cols = 256;  // N = 2^16: both passes are 256 x 256
  t1.u[0] = FsUnit{in, (uint32_t*)ws, tabs, batch, 0, nullptr, nullptr, 0, 0};
  t2.u[0] = FsUnit{(const uint32_t*)ws, out, tabs, batch, 0, nullptr, nullptr, 0, 0};
  co_launch<true>(p, t1, s);
  co_launch<false>(p, t2, s);
  return hipGetLastError();
}

hipError_t fs_forward(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  NttUnit u{p, false, in, out, limb_begin, limb_count, batch};
  return fs_run_units(&u, 1, ws, s);
}

hipError_t fs_inverse(const tfhe_ntt_plan_s* p, const uint32_t* in, uint32_t* out, void* ws,
                      uint32_t limb_begin, uint32_t limb_count, uint32_t batch, hipStream_t s) {
  NttUnit u{p, true, in, out, limb_begin, limb_count, batch};
  return fs_run_units(&u, 1, ws, s);
}

}  // namespace tfhe
