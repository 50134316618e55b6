// Four-step NTT on INT8 matrix cores (Sec. III-B/III-C, Eq. 8 and Eq. 9),
// re-designed for gfx950.
//
// N = 2^16 is viewed as a 256 x 256 matrix (n = 256 n1 + n2, k = k1 + 256 k2):
//   pass 1, per column n2:  Y[k1] = sum_{n1} phi^{(2k1+1) n1} a[n1][n2],
//                           Z[k1][n2] = Y[k1] * psi^{(2k1+1) n2}   (the W2 twist)
//   pass 2, per row k1:     A[k1 + 256 k2] = sum_{n2} w^{k2 n2} Z[k1][n2]
// (phi = psi^256, w = psi^512).  Each 256-point stage runs as two radix-16
// levels (n = 16u + v, k = s + 16t): a dense 16 x 16 contraction on the
// matrix cores, an element-wise twist, a second 16 x 16 contraction.
//
// Exactness (the segment-fusion idea of Sec. III-C, Fig. 4): every operand
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
// form), or, after the last level, whose twiddles carry the 2^32, leaves the
// canonical residue.  Twisted results are re-sliced into digits for the next
// contraction with two VALU operations.
//
// Data movement: persistent workgroups stride over the work items (16
// vectors = 16 columns of the 256 x 256 matrix of one polynomial) with a
// stride that is a multiple of 16, so a workgroup keeps the same columns and
// reloads the limb's tables and the pass-1 post-twist only when the limb
// changes.  Each item is staged through LDS; the global loads of the next item
// are issued before the current one is computed.  Each wave transforms four vectors, one per
// 16 x 16 tile with four coefficients per lane.  Pass 1 writes its digit-form
// result row-wise to the workspace (the transpose), pass 2 writes canonical
// residues back as a column block through LDS.  The inverse runs the same
// kernels with the inverse tables (w^{-1}, phi^{-2}, psi^{-(2k1+1) n2}, N^{-1}
// folded into the last level).
#include <algorithm>

#include "internal.hpp"

namespace tfhe {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kCols = 16;     // vectors per workgroup
constexpr int kStride = 324;  // LDS words per vector: 256 + 64 pad, = 4 (mod 64)

__device__ __forceinline__ int lds_pos(int col, int n) { return col * kStride + n + 16 * (n >> 6); }

// Descriptor table of a fused launch (passed by value as a kernel argument):
// unit k covers work items [item_begin[k], item_begin[k+1]).
constexpr int kMaxUnits = 40;
struct FsUnit {
  const uint32_t* in;
  uint32_t* out;
  const FourStepLimb* limbs;  // tables of the unit's first limb
  uint32_t batch;
  uint32_t item_begin;
};
struct FsTable {
  uint32_t count, total;
  FsUnit u[kMaxUnits];
};

__device__ __forceinline__ v4i mfma(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Fusion and one Montgomery step: V 2^{-32} mod q, in [0, q + 2^17).
__device__ __forceinline__ uint32_t fuse_redc(int c0, int c1, int c2, int c3, uint32_t q,
                                              uint32_t qneg) {
  const uint32_t lo = (uint32_t)c0 + ((uint32_t)c1 << 8);
  const uint32_t hi = (uint32_t)c2 + ((uint32_t)c3 << 8);
  const uint64_t V = ((uint64_t)hi << 16) + lo;
  const uint32_t vlo = (uint32_t)V, vhi = (uint32_t)(V >> 32);
  const uint32_t m = vlo * qneg;
  return vhi + __umulhi(m, q) + (vlo != 0u);
}

// Twist (Shoup, t = {w 2^32, companion}) and re-slice into digits.
__device__ __forceinline__ uint32_t twist_digits(uint32_t r, uint2 t, uint32_t q) {
  const uint32_t z = mul_shoup_lazy(r, t.x, t.y, q);  // [0, 2q)
  int32_t zz = (int32_t)(z - q);                      // [-q, q)
  zz = zz > 0x7F7F7F7F ? zz - (int32_t)q : zz;        // only when q > 0x7F7F7F7F
  return balanced_digits(zz);
}

// One 256-point stage of one vector: level A, twist, level B.  x holds the
// lane's four input words as digits (lane (v, g), word c: element 64g+16c+v);
// on return acc[j][r] is plane j of output s + 16 (4g + r) for lane (s, g).
__device__ __forceinline__ void stage256(v4i x, const v4i* opA, const v4i* opB, const uint2* tw,
                                         uint32_t q, uint32_t qneg, v4i* acc) {
  const v4i bias = {(int)q, (int)q, (int)q, (int)q};
  const v4i zero = {0, 0, 0, 0};
  v4i c0 = mfma(x, opA[0], bias);
  v4i c1 = mfma(x, opA[1], zero);
  v4i c2 = mfma(x, opA[2], bias);
  v4i c3 = mfma(x, opA[3], zero);
  v4i z;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    z[r] = (int)twist_digits(fuse_redc(c0[r], c1[r], c2[r], c3[r], q, qneg), tw[r], q);
  acc[0] = mfma(opB[0], z, bias);
  acc[1] = mfma(opB[1], z, zero);
  acc[2] = mfma(opB[2], z, bias);
  acc[3] = mfma(opB[3], z, zero);
}

// Work distribution.  The grid is a multiple of 16; workgroup w belongs to
// group w / 16 and owns column block blk(w % 16) of every polynomial in its
// group's contiguous range, so it changes limb (and reloads the limb's
// tables and its post-twist slice) at most a few times.  Workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2: the two
// 64-byte halves of a 128-byte line are column blocks 2b and 2b+1, owned by
// workgroups c and c + 8 of a group, i.e. on the same XCD at the same time,
// so each line is fetched from memory once.
struct Walk {
  uint32_t blk, p, p_end;  // column block; current and end polynomial (global index)
};
__device__ __forceinline__ Walk make_walk(uint32_t total_polys) {
  const uint32_t groups = gridDim.x / 16, a = blockIdx.x / 16, c = blockIdx.x % 16;
  Walk w;
  w.blk = 2 * (c % 8) + c / 8;
  w.p = (uint32_t)((uint64_t)a * total_polys / groups);
  w.p_end = (uint32_t)((uint64_t)(a + 1) * total_polys / groups);
  return w;
}

struct Item {
  uint32_t unit, limb;
  size_t poly_base;  // word offset of the polynomial within the unit's arrays
};
// Global polynomial p -> (unit, limb, offset); `k` is a running unit index
// (p only increases along a walk).
__device__ __forceinline__ Item locate(const FsTable& t, uint32_t p, uint32_t& k) {
  while (k + 1 < t.count && p >= t.u[k + 1].item_begin) ++k;
  const uint32_t local = p - t.u[k].item_begin;
  Item it;
  it.unit = k;
  it.limb = local / t.u[k].batch;
  it.poly_base = (size_t)local << 16;
  return it;
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Item tile in LDS, as the direct-to-LDS loads deposit it: region k (1 KiB)
// holds rows 16k .. 16k+15 of the item's 16 columns; its 16-byte slot L holds
// row 16k + L % 16, columns 4 (L / 16) .. 4 (L / 16) + 3.
constexpr int kTile = 256 * kCols;  // words
constexpr int kStages = 3;           // input ring depth (items in LDS)

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Each wave loads regions 4 wave .. 4 wave + 3 of an item: one 16-byte
// direct-to-LDS load per lane per region (a 64-byte segment of 16 rows);
// lane L's bytes land at the region base + 16 L.  Issued as inline assembly so
// that the compiler does not serialise later LDS reads on these loads: the
// pipeline waits for them explicitly (wait_item) before a barrier.
__device__ __forceinline__ void issue_tile(const uint32_t* src, uint32_t* stage, int wave, int lane) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * wave + j;
    const uint32_t* g = src + (16 * k + (lane & 15)) * 256 + 4 * (lane >> 4);
    const uint32_t lds_addr = (uint32_t)(uintptr_t)(lds_void_t*)(stage + k * 256);
    asm volatile(
        "s_mov_b32 m0, %0\n\t"
        "global_load_lds_dwordx4 %1, off"
        :
        : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
        : "memory", "m0");
  }
}

// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding load): LDS writes of this wave are completed
// first; the direct-to-LDS loads are covered by wait_item.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
}

// Wait until this wave's loads of the current item have landed.  Vector
// memory operations of a wave complete in issue order, so it suffices that at
// most as many operations remain outstanding as were issued after those
// loads: in steady state the stores of the two previous items (16 each in
// pass 1, 4 in pass 2) and the loads of the next item (4); fewer near the
// start; without a next item everything is awaited.  Table loads issued in
// between only make the wait stricter.
template <bool kFirst>
__device__ __forceinline__ void wait_item(uint32_t n, bool has_next) {
  constexpr int st = kFirst ? 16 : 4;
  if (!has_next) wait_vmcnt<0>();
  else if (n == 0) wait_vmcnt<4>();
  else if (n == 1) wait_vmcnt<4 + st>();
  else wait_vmcnt<4 + 2 * st>();
}

template <bool kFirst>
__global__ void __launch_bounds__(kThreads)
fs_pass(const FsTable tab) {
  __shared__ __attribute__((aligned(16))) uint32_t ring[(kStages + (kFirst ? 0 : 1)) * kTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int v = lane & 15, g = lane >> 4;
  const Walk walk = make_walk(tab.total);
  const uint32_t blk = walk.blk, p_begin = walk.p, p_end = walk.p_end;
  if (p_begin >= p_end) return;

  uint32_t kf = 0, kc = 0;  // running unit indices of the load and compute walks
  auto issue = [&](uint32_t p, int st) {
    const Item it = locate(tab, p, kf);
    issue_tile(tab.u[it.unit].in + it.poly_base + blk * kCols, ring + st * kTile, wave, lane);
  };
#pragma unroll
  for (int j = 0; j < kStages - 1; ++j)
    if (p_begin + j < p_end) issue(p_begin + j, j);

  const FourStepLimb* cur_limb = nullptr;
  uint32_t q = 0, qneg = 0;
  v4i opA[4], opB[4];
  uint2 tw[4];
  uint2 pt[4][4];
  int st = 0;
  for (uint32_t p = p_begin; p < p_end; ++p, st = (st + 1 == kStages) ? 0 : st + 1) {
    const uint32_t n = p - p_begin;
    const Item it = locate(tab, p, kc);
    const FourStepLimb* limb = tab.u[it.unit].limbs + it.limb;
    if (limb != cur_limb) {
      // rare (a few times per workgroup): completed here, so that the
      // steady-state path carries no wait on these loads
      const FourStepLimb L = *limb;
      const PassTables* P = kFirst ? L.pass1 : L.pass2;
      q = L.q;
      qneg = L.qneg;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        opA[j] = *(const v4i*)&P->opA[j][lane][0];
        opB[j] = *(const v4i*)&P->opB[j][lane][0];
        tw[j] = P->twist[lane][j];
      }
      if (kFirst) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const uint2* pp = L.post1 + ((size_t)(blk * kCols + 4 * wave + cc) * 64 + lane) * 4;
#pragma unroll
          for (int r = 0; r < 4; ++r) pt[cc][r] = pp[r];
        }
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      cur_limb = limb;
    }
    wait_item<kFirst>(n, p + 1 < p_end);
    lds_barrier();  // the item's tile is complete; the oldest stage is free
    if (p + kStages - 1 < p_end) issue(p + kStages - 1, (st + kStages - 1) % kStages);

    // lane (v, g): rows 64g + 16c + v of the wave's four columns 4 wave .. +3
    const uint32_t* tile = ring + st * kTile;
    uint4 rows[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rows[c] = *(const uint4*)(tile + (4 * g + c) * 256 + (v + 16 * wave) * 4);

    const size_t base = it.poly_base;
    uint32_t* const out = tab.u[it.unit].out;
    uint4 res[4];  // pass 2: res[r] = the four columns' outputs for row s + 64g + 16r
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      v4i x;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t w = cc == 0 ? rows[c].x : cc == 1 ? rows[c].y : cc == 2 ? rows[c].z : rows[c].w;
        x[c] = kFirst ? (int)balanced_digits(to_window(w, q)) : (int)w;
      }
      v4i acc[4];
      stage256(x, opA, opB, tw, q, qneg, acc);
      if (kFirst) {
        // post twist and row store: output k = s + 64g + 16r of vector col
        const int col = 4 * wave + cc;
        uint32_t* dst = out + base + (blk * kCols + col) * 256 + v + 64 * g;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[16 * r] = twist_digits(fuse_redc(acc[0][r], acc[1][r], acc[2][r], acc[3][r], q, qneg),
                                     pt[cc][r], q);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t y = reduce_once(fuse_redc(acc[0][r], acc[1][r], acc[2][r], acc[3][r], q, qneg), q);
          if (cc == 0) res[r].x = y;
          else if (cc == 1) res[r].y = y;
          else if (cc == 2) res[r].z = y;
          else res[r].w = y;
        }
      }
    }

    if (!kFirst) {
      // output tile in the input layout, then 16-byte row-segment stores
      uint32_t* otile = ring + kStages * kTile;
#pragma unroll
      for (int r = 0; r < 4; ++r) *(uint4*)(otile + (4 * g + r) * 256 + (v + 16 * wave) * 4) = res[r];
      lds_barrier();
      uint32_t* dst = out + base + blk * kCols;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * wave + j;
        *(uint4*)(dst + (16 * k + (lane & 15)) * 256 + 4 * (lane >> 4)) =
            *(const uint4*)(otile + k * 256 + lane * 4);
      }
    }
  }
}

// Resident workgroups per CU of each pass kernel (queried once per process).
static uint32_t occupancy(bool first) {
  static int occ[2] = {0, 0};
  int& o = occ[first ? 1 : 0];
  if (o == 0) {
    int n = 0;
    hipError_t e = first ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fs_pass<true>, kThreads, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fs_pass<false>, kThreads, 0);
    o = (e == hipSuccess && n > 0) ? n : 2;
  }
  return (uint32_t)o;
}

// Persistent grid: resident workgroups of the whole device, rounded down to a
// multiple of 16 (one workgroup per column block in each group), and at most
// 16 per polynomial.
static uint32_t grid_size(const tfhe_ntt_plan_s* p, bool first, uint32_t polys) {
  const uint32_t w = p->fs_wg_per_cu ? p->fs_wg_per_cu : occupancy(first);
  uint32_t g = std::max(16u, (p->num_cus * w) / 16 * 16);
  return std::min(g, 16 * polys);
}

}  // namespace

bool fs_supported(uint32_t log_n) { return log_n == 16; }

size_t unit_ws_bytes(const NttUnit& u, bool mfma) {
  if (mfma) return (size_t)u.limb_count * u.batch * u.plan->n * sizeof(uint32_t);
  return bf_workspace_bytes(u.plan, u.limb_count, u.batch);
}

size_t fs_workspace_bytes(const tfhe_ntt_plan_s* p, uint32_t limb_count, uint32_t batch) {
  return (size_t)limb_count * batch * p->n * sizeof(uint32_t);
}

// Fused launch: pass 1 of every unit (in -> unit workspace), then pass 2 of
// every unit (workspace -> out), kMaxUnits units per launch pair.
hipError_t fs_run_units(const NttUnit* units, uint32_t count, void* ws, hipStream_t s) {
  unsigned char* w = (unsigned char*)ws;
  for (uint32_t first = 0; first < count; first += kMaxUnits) {
    const uint32_t n = std::min<uint32_t>(kMaxUnits, count - first);
    FsTable t1, t2;
    t1.count = t2.count = 0;
    uint32_t total = 0;
    const tfhe_ntt_plan_s* p0 = nullptr;
    for (uint32_t k = 0; k < n; ++k) {
      const NttUnit& u = units[first + k];
      const uint32_t items = u.limb_count * u.batch;  // polynomials
      if (items == 0) continue;
      p0 = u.plan;
      const FourStepLimb* tabs = (u.inverse ? u.plan->d_fs_inv : u.plan->d_fs_fwd) + u.limb_begin;
      uint32_t* mid = (uint32_t*)w;
      w += (unit_ws_bytes(u, true) + 255) & ~(size_t)255;
      t1.u[t1.count++] = FsUnit{u.in, mid, tabs, u.batch, total};
      t2.u[t2.count++] = FsUnit{mid, u.out, tabs, u.batch, total};
      total += items;
    }
    if (total == 0) continue;
    t1.total = t2.total = total;
    TFHE_TIMED(K_FS_PASS1, s,
               hipLaunchKernelGGL(fs_pass<true>, dim3(grid_size(p0, true, total)), dim3(kThreads), 0, s, t1));
    TFHE_TIMED(K_FS_PASS2, s,
               hipLaunchKernelGGL(fs_pass<false>, dim3(grid_size(p0, false, total)), dim3(kThreads), 0, s, t2));
  }
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
