// HIP kernels (gfx950) for batched affine-gap DP alignment of reads against
// reference windows: the DP phase of MICA (Methods, "Highly parallel dynamic
// programming").
//
// Mapping (a CDNA4 redesign of the paper's anti-diagonal fill):
//  * A group of P lanes (16 or 64) aligns one pair per 16-bit half of each
//    32-bit register (two pairs per group, packed int16 with saturating
//    v_pk_* arithmetic), or one pair with 32-bit scores.
//  * Lane k holds R consecutive read rows in registers.  Window columns stream
//    through the lanes: at step t lane k computes column t-k+1 for its R rows
//    top to bottom, so the cells a step computes lie on an anti-diagonal band
//    and every dependency is either in-lane or one lane up one step earlier.
//    The bottom row's T = H - o - e and I move one lane down per step by DPP
//    (row_shr:1 for 16-lane groups, wave_shr:1 for 64).
//  * The read occupies the bottom m of the P*R row slots; the slots above are
//    dummy rows whose substitution score is -1.  With the top boundary H = 0
//    they hold H = -d (d = depth), so the last dummy row is the read's row 0
//    shifted by -D0 (D0 = number of dummy rows).  Every value below is the
//    true value shifted by the constant -D0 (max and + commute with a shift);
//    the local floor 0 becomes -D0.  Row m is always the last register of the
//    last lane.
//  * The substitution score is one v_perm_b32 lookup: selector bytes come from
//    XOR of a per-row read code and a per-column window code, the table holds
//    the match and mismatch scores; a dummy row's code selects 0xFF bytes (-1).
//  * Per cell and per direction kind one sign bit is kept (diagonal / deletion
//    loses, deletion / insertion extends).  One v_perm_b32 turns the signs of
//    two kinds' differences into 0x00/0xFF bytes and one v_and_or_b32 keeps
//    the row's bit of each byte: word 2*(r/8) + kind/2, byte 2*(kind%2) + half,
//    bit r%8.  A lane stores two words per step (four when R > 8) to the
//    wave's scratch slot; after the fill one lane per pair walks them back to
//    the start cell and writes the CIGAR.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "dp_common.h"

namespace mica {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 as_s(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
__device__ __forceinline__ uint32_t as_u(s16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t as_u(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), in order
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int clamp16(int v) { return v < -32768 ? -32768 : (v > 32767 ? 32767 : v); }
__device__ __forceinline__ uint32_t bfi(uint32_t mask, uint32_t x, uint32_t y) {
  return (mask & x) | (~mask & y);
}

// One v_bfi_b32 (mask & x | ~mask & y).  Written out because the compiler
// would otherwise split a chain of them into and/or trees of twice the length.
__device__ __forceinline__ uint32_t bfi_op(uint32_t mask, uint32_t x, uint32_t y) {
  uint32_t d;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(d) : "s"(mask), "v"(x), "v"(y));
  return d;
}

// Packed 16-bit scores: half h of every register belongs to pair h of the group.
struct V16 {
  static constexpr int kPairs = 2;
  typedef uint32_t T;
  static constexpr uint32_t kNeg = 0x80008000u;
  static constexpr uint32_t kQDummy = 0xF0F0F0F0u;
  __device__ static T add(T a, T b) { return as_u(__builtin_elementwise_add_sat(as_s(a), as_s(b))); }
  __device__ static T sub(T a, T b) { return as_u(__builtin_elementwise_sub_sat(as_s(a), as_s(b))); }
  __device__ static T vmax(T a, T b) { return as_u(__builtin_elementwise_max(as_s(a), as_s(b))); }
  __device__ static T vmin(T a, T b) { return as_u(__builtin_elementwise_min(as_s(a), as_s(b))); }
  __device__ static T max3(T a, T b, T c) { return vmax(vmax(a, b), c); }
  // v_perm_b32 selector that turns the signs of two difference registers
  // (a, b) into four 0x00/0xFF bytes: b.lo, b.hi, a.lo, a.hi
  static constexpr uint32_t kSignSel = 0x0B0A0908u;
  // 0xFFFF in each half where d < 0 (one v_perm_b32 on the sign bits; an
  // arithmetic shift is folded by the compiler into per-half compares and
  // selects of three times the length)
  __device__ static T negmask(T d) { return __builtin_amdgcn_perm(d, d, 0x09090808u); }
  __device__ static T make2(int lo, int hi) {
    return (uint32_t)(uint16_t)clamp16(lo) | ((uint32_t)(uint16_t)clamp16(hi) << 16);
  }
  __device__ static T splat(int v) { return make2(v, v); }
  __device__ static int get(T x, int h) { return (int)(int16_t)(uint16_t)(x >> (16 * h)); }
  __device__ static uint32_t getu(T x, int h) { return (x >> (16 * h)) & 0xFFFFu; }
  // selector byte pattern of a read base q in half h, and of a window base r
  __device__ static uint32_t qcode(int q, int h) {
    return ((uint32_t)(2 * q) | ((uint32_t)(2 * q + 1) << 8)) << (16 * h);
  }
  __device__ static uint32_t qdummy(int h) { return 0xF0F0u << (16 * h); }
  __device__ static uint32_t rcode(int r, int h) { return ((uint32_t)r * 0x0202u) << (16 * h); }
};

// 32-bit scores, one pair per group.
struct V32 {
  static constexpr int kPairs = 1;
  typedef int32_t T;
  static constexpr int32_t kNeg = -(1 << 29);
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static T sub(T a, T b) { return a - b; }
  __device__ static T vmax(T a, T b) { return a > b ? a : b; }
  __device__ static T vmin(T a, T b) { return a < b ? a : b; }
  __device__ static T max3(T a, T b, T c) { return vmax(vmax(a, b), c); }
  // sign bytes b, b, a, a (the byte layout of the 16-bit variant, half 1 a copy of half 0)
  static constexpr uint32_t kSignSel = 0x0B0B0909u;
  __device__ static T splat(int v) { return v; }
  __device__ static int get(T x, int) { return x; }
  // bytes: 2q, 2q+1 pick a 16-bit table entry, 8+q replicate its sign
  __device__ static uint32_t qcode(int q, int) {
    return (uint32_t)(2 * q) | ((uint32_t)(2 * q + 1) << 8) | ((uint32_t)(8 + q) << 16) |
           ((uint32_t)(8 + q) << 24);
  }
  __device__ static uint32_t qdummy(int) { return 0xF0F0F0F0u; }
  __device__ static uint32_t rcode(int r, int) { return (uint32_t)r * 0x01010202u; }
};

template <int P>
__device__ __forceinline__ uint32_t shift_down(uint32_t src, uint32_t old) {
  // value of the lane above; the first lane of each group keeps `old`
  if constexpr (P == 16)
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x111, 0xF, 0xF, false);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xF, 0xF, false);
}

// Data pointers reach the kernels through the parameter block, so the
// compiler sees them as generic; casting them to the global address space
// gives global_load/store (flat instructions would also count against the
// LDS wait counter and stall every step).
#define MICA_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MICA_GLOBAL T* G(T* p) {
  return (MICA_GLOBAL T*)p;
}

// Values the compiler cannot prove wave-uniform (anything derived from the
// wave index threadIdx.x >> 6) are made uniform explicitly, so they live in
// SGPRs and the step loops are scalar loops.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
template <class T>
__device__ __forceinline__ T* uni(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int base_at(const MICA_GLOBAL uint32_t* __restrict__ seq, uint64_t pos) {
  return (int)((seq[pos >> 4] >> (2 * (uint32_t)(pos & 15))) & 3u);
}

// Resident waves per SIMD each fill kernel is compiled for (its VGPR budget
// is 512 / waves: 5 waves <= 102 VGPRs, 4 <= 128, 3 <= 170, 2 <= 256).
// Most variants get the most waves that their register need fits without
// spilling.  The packed 16-bit traceback variants of the semi-global mode
// with 6-16 rows and of the local and extension modes with 7-15 rows get
// one wave more: their step loops still do not spill, their set-up and walk
// do, and the extra wave hides more latency than those spills cost
// (measured on the 10-row kernels: +1.8% semi-global, +0.8% local).
__host__ __device__ constexpr int fill_waves(int kind, int cls, int mode, int tb) {
  // the banded traceback's fill keeps no direction bits: the score-only budget
  const bool dir = tb == 2;
  const int r = class_rows(cls);
  if (class_lanes(cls) == 64 && r == 16) return 2;
  if (kind == kK32) {
    if (mode == 0) return r <= 8 ? 5 : (r <= 11 ? 4 : 3);
    return dir ? (r <= 5 ? 5 : (r <= 8 ? 4 : (r <= 12 ? 3 : 2))) : (r <= 6 ? 5 : (r <= 10 ? 4 : (r <= 13 || mode == 1 ? 3 : 2)));
  }
  const int sat = kind == kK16Sat ? 1 : 0;
  if (mode == 0) {
    if (dir) return sat ? (r <= 3 ? 5 : (r <= 7 ? 4 : (r <= 12 ? 3 : 2))) : (r <= 10 ? 5 : (r <= 15 ? 4 : 3));
    return r <= 6 - sat ? 5 : (r <= 12 - 3 * sat ? 4 : (r <= 16 - 2 * sat ? 3 : 2));
  }
  if (dir) return sat ? (r <= 2 ? 5 : (r <= 5 ? 4 : (r <= 8 ? 3 : (r <= 15 ? 2 : 1)))) : (r <= 3 ? 5 : (r <= 10 ? 4 : (r <= 15 ? 3 : 2)));
  const int ext = mode == 2 ? 1 : 0;  // the extension also tracks its top boundary
  return r <= 4 - sat ? 5 : (r <= 8 - sat ? 4 : (r <= 12 - sat - ext ? 3 : 2));
}
#ifdef MICA_FILL_WAVES
#define MICA_BUCKET_WAVES(kind, cls, mode, dir) MICA_FILL_WAVES
#else
#define MICA_BUCKET_WAVES(kind, cls, mode, dir) fill_waves(kind, cls, mode, dir)
#endif
#ifndef MICA_ROW_SCHED_BARRIER
#define MICA_ROW_SCHED_BARRIER 1
#endif
// Resident waves per SIMD of a persistent kernel (all classes of its part
// share one register budget).  The traceback kernels run one wave more than
// their set-up and walk fit without spilling (the step loops spill at most
// a few reloads per step, in a few of the longest classes): the extra wave
// hides more of the latency of set-up and walk than the spills cost
// (measured: +4% on 10^6 seed extensions, +4-5% on the mixed-length batch,
// against the lower budgets).
__host__ __device__ constexpr int persist_waves(int tb, int mode, int part) {
#if defined(MICA_PERSIST_WAVES0) && defined(MICA_PERSIST_WAVES1)
  if (tb == 1) return part == 0 ? MICA_PERSIST_WAVES0 : MICA_PERSIST_WAVES1;
#endif
  return tb == 2 ? (mode == 0 ? 4 : (part == 0 ? 4 : 3))
                 : (tb ? (part == 0 ? 4 : 3) : (mode == 0 ? 3 : (part == 0 ? 4 : 3)));
}

// Lanes of one wave exchange values through LDS: LDS operations of a wave
// complete in order, and the wave-scope fences keep the compiler from moving
// a lane's LDS accesses across the exchange point.
__device__ __forceinline__ void lds_wait() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace mica

#include "band.h"

namespace mica {

// Traceback kinds of a fill kernel: none (score and end cell only), banded
// (score-only fill, then the band refill and walk of band.h), full
// (direction bits of every cell stored during the fill; the fallback for
// pairs whose band is too wide, and the 32-bit re-run), or the band refill
// alone of the pairs a banded fill passed on (bands of 17-64 diagonals), or
// the band refill of a wave's pending pairs (see band_route).
enum Traceback : int { kTbNone = 0, kTbBand = 1, kTbFull = 2, kTbDefer = 3, kTbPend = 4 };

// One wave-sized work item: G = 64/P groups, each aligning kPairs pairs.
// pend: the count of the wave's pending list (banded fills of 16-lane
// classes; unused otherwise).
template <class V, int P, int R, int MODE, int TB, bool SAT>
__device__ __forceinline__ void process_item(const Params* __restrict__ prm,
                                          const uint32_t* __restrict__ pairs, int npairs,
                                          uint32_t* lds, uint8_t* slot, int bucket, int* pend = nullptr) {
  typedef typename V::T T;
  constexpr bool DIR = (TB == kTbFull);
  constexpr int NP = V::kPairs;
  constexpr int PR = P * R;
  constexpr bool LOCAL = (MODE == 1);
  // Extension: the read occupies the top m row slots (rows below it compute
  // values nothing reads), the top boundary is the anchor's leading-deletion
  // row h0 - (o + j*e), values are not shifted (d0 = 0); the best cell is
  // tracked per row as in local mode.
  constexpr bool EXT = (MODE == 2);
  constexpr bool TRACK = (MODE != 0);
  const int lane = threadIdx.x & 63;
  const int g = lane / P;
  const int k = lane % P;
  const int sa = prm->sa, sb = prm->sb, so = prm->so, se = prm->se;
  const int oe = so + se;
  const MICA_GLOBAL uint32_t* __restrict__ ref2b = G(prm->ref2b);
  const MICA_GLOBAL uint32_t* __restrict__ reads2b = G(prm->reads2b);
  const MICA_GLOBAL uint32_t* __restrict__ gpairs = G(uni(pairs));
  npairs = uni(npairs);

  if constexpr (TB == kTbDefer || TB == kTbPend) {
    // the fill's results (shifted score, i*, j*) come back from the outputs
    // the banded fill wrote; none of these pairs saturated.  Pending pairs
    // (bands of up to 16 diagonals) are refilled as right after a fill.
    uint32_t* red = lds + kRedOff;
    if (lane < npairs) {
      const int p = (int)gpairs[lane];
      const int d0_ = EXT ? 0 : PR - G(prm->read_len)[p];
      red[lane * 4 + 0] = (uint32_t)(G(prm->score)[p] - d0_);
      red[lane * 4 + 1] = (uint32_t)G(prm->read_end)[p];
      red[lane * 4 + 2] = (uint32_t)G(prm->ref_end)[p];
    }
    lds_wait();
    bool none[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) none[h] = false;
    band_traceback<V, P, R, MODE, TB == kTbDefer>(prm, gpairs, npairs, lds, slot, none, bucket);
    return;
  }

  // ---- the pairs of this lane's group --------------------------------------
  int pid[NP], m[NP], n[NP], d0[NP], h0[NP];
  uint64_t woff[NP], roff[NP];
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    const int idx = g * NP + h;
    pid[h] = -1;
    h0[h] = 0;
    m[h] = PR;
    n[h] = 0;
    woff[h] = 0;
    roff[h] = 0;
    if (idx < npairs) {
      const int p = (int)gpairs[idx];
      pid[h] = p;
      m[h] = G(prm->read_len)[p];
      n[h] = G(prm->win_len)[p];
      woff[h] = G(prm->win_off)[p];
      roff[h] = G(prm->read_off)[p];
      if constexpr (EXT) h0[h] = prm->ext_h0 ? G(prm->ext_h0)[p] : prm->ext_default_h0;
    }
    d0[h] = EXT ? 0 : PR - m[h];
  }
  // column range of the item (uniform loop, scalar loads)
  int nmin = 1 << 30, nmax = 0;
  for (int s = 0; s < npairs; ++s) {
    const int nn = G(prm->win_len)[gpairs[s]];
    nmin = nn < nmin ? nn : nmin;
    nmax = nn > nmax ? nn : nmax;
  }
  nmin = uni(nmin);
  nmax = uni(nmax);

  // ---- read profile: selector code per row register -------------------------
  uint32_t Q[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = k * R + r;
    uint32_t q = 0;
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      if ((EXT ? u >= m[h] : u < d0[h]) || pid[h] < 0) {
        q |= V::qdummy(h);
      } else {
        q |= V::qcode(base_at(reads2b, roff[h] + (uint64_t)(u - d0[h])), h);
      }
    }
    Q[r] = q;
  }
  const uint32_t tab_lo = ((uint32_t)sa & 0xFFFFu) | ((uint32_t)sb << 16);
  const uint32_t tab_hi = ((uint32_t)sb & 0xFFFFu) | ((uint32_t)sb << 16);
  // the table's low half as the lookup's register operand, set once (the
  // compiler would otherwise copy it from a scalar register every step)
  uint32_t tab_lo_v;
  asm("v_mov_b32 %0, %1" : "=v"(tab_lo_v) : "s"(tab_lo));

  // ---- column 0 ---------------------------------------------------------------
  // per row: H, and E = the next column's deletion candidate
  // max(D - e, H - o - e) (D and T = H - o - e are not kept)
  T H[R], E[R];
  T bb[TRACK ? R : 1], cc[TRACK ? R : 1];
  int hv[NP];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = k * R + r;
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      if constexpr (EXT) {
        // leading insertion at the anchor (rows below the read continue it)
        hv[h] = h0[h] - (so + (u + 1) * se);
      } else if (u < d0[h]) {
        hv[h] = -(u + 1);
      } else {
        const int i = u - d0[h] + 1;
        hv[h] = (LOCAL ? 0 : -(so + i * se)) - d0[h];
      }
    }
    if constexpr (NP == 2) {
      H[r] = V::make2(hv[0], hv[1]);
      E[r] = V::make2(hv[0] - oe, hv[1] - oe);  // D(i,0) is -inf
    } else {
      H[r] = (T)hv[0];
      E[r] = (T)(hv[0] - oe);
    }
  }
  T floor_v = (T)0;
  if constexpr (LOCAL) {
    if constexpr (NP == 2)
      floor_v = V::make2(-d0[0], -d0[1]);
    else
      floor_v = (T)(-d0[0]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bb[r] = floor_v;
      cc[r] = (T)0;
    }
  }
  if constexpr (EXT) {
    // every row's best starts at its column 0 (the end-to-end candidate of
    // row m covers j = 0; elsewhere column 0 is below h0 and never wins)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bb[r] = H[r];
      cc[r] = (T)0;
    }
  }
  T hmax = (T)0, tmin = (T)0;
  if constexpr (SAT) {
    hmax = V::splat(-32768);
    tmin = V::splat(32767);
#pragma unroll
    for (int r = 0; r < R; ++r) tmin = V::vmin(tmin, E[r]);
  }
  // semi-global best over row m: key (score << 16 | 0xFFFF - j), or (score, j)
  int32_t best_key[NP];
  int32_t best_h32 = 0, best_j32 = 0;
  if constexpr (MODE == 0) {
    if constexpr (NP == 2) {
      best_key[0] = (int32_t)((H[R - 1] << 16) | 0xFFFFu);
      best_key[1] = (int32_t)((H[R - 1] & 0xFFFF0000u) | 0xFFFFu);
    } else {
      best_h32 = (int32_t)H[R - 1];
      best_j32 = 0;
    }
  }

  uint32_t* ring = lds + g * kRing;
  uint32_t* red = lds + kRedOff;     // final (score, i*, j*) per pair
  // direction words per lane and step
  constexpr int NW = R <= 8 ? 2 : 4;
  MICA_GLOBAL u32x4* dir4 = (MICA_GLOBAL u32x4*)slot;
  MICA_GLOBAL u32x2* dir2 = (MICA_GLOBAL u32x2*)slot;

  const T ev = V::splat(se);
  const T oev = V::splat(oe);
  // T and I of the row above each lane's top row.  The first lane of a group
  // gets the top boundary: T is 0 above the dummy rows (for an extension the
  // anchor row h0 - (o + j*e), which moves down by e per step), I is -inf.
  // The DPP move of each step writes the other lanes only, so the first
  // lane's boundary stays in tsh / ish without a copy per step.
  T tsh = V::splat(-oe);
  const T negv = (T)V::kNeg;
  T ish = negv;
  T t_last = E[R - 1];  // T of the bottom row, column 0
  T i_last = negv;
  T hdiag_next = (T)0;
  if constexpr (EXT) {
    if constexpr (NP == 2) {
      tsh = V::make2(h0[0] - so - se - oe, h0[1] - so - se - oe);
      hdiag_next = V::make2(h0[0], h0[1]);
    } else {
      tsh = (T)(h0[0] - so - se - oe);
      hdiag_next = (T)h0[0];
    }
  }
  T nn_v = (T)0;
  if constexpr (NP == 2) nn_v = V::make2(n[0], n[1]);
  const uint32_t kk16 = (uint32_t)k * 0x10001u;

  auto fill_ring = [&](int c0) {
    // an empty volatile statement keeps the address arithmetic below inside
    // the (rarely taken) branch: hoisted, it costs a few instructions per step
    asm volatile("" : "+s"(c0));
    for (int x = k; x < kRing / 2; x += P) {
      const int c = c0 + x;
      uint32_t sel = 0;
#pragma unroll
      for (int h = 0; h < NP; ++h)
        if (c < n[h]) sel |= V::rcode(base_at(ref2b, woff[h] + (uint64_t)c), h);
      ring[c & (kRing - 1)] = sel;
    }
    lds_wait();
  };

  // window selectors are read two steps ahead of their use
  fill_ring(0);
  uint32_t rs_a = ring[(0 - k) & (kRing - 1)];
  uint32_t rs_b = ring[(1 - k) & (kRing - 1)];

  auto step = [&](int t, auto checks) {
    constexpr bool CHECK = decltype(checks)::value;
    const uint32_t rsel = rs_a;
    rs_a = rs_b;
    tsh = (T)shift_down<P>((uint32_t)t_last, (uint32_t)tsh);
    ish = (T)shift_down<P>((uint32_t)i_last, (uint32_t)ish);
    T tup = tsh;
    T iup = ish;
    T hdiag = hdiag_next;
    hdiag_next = V::add(tup, oev);
    const int j = t - k + 1;
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    if (!CHECK || j >= 1) {
      T jj = (T)0, vmask = (T)0;
      if constexpr (TRACK) {
        if constexpr (NP == 2) {
          jj = (uint32_t)(t + 1) * 0x10001u - kk16;
          if constexpr (CHECK) vmask = ~V::negmask(V::sub(nn_v, jj));
        } else {
          jj = (T)j;
        }
      }
      static_for<R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        const T s = (T)__builtin_amdgcn_perm(tab_hi, tab_lo_v, Q[r] ^ rsel);
        const T x = V::add(hdiag, s);
        const T dn = E[r];
        const T in = V::vmax(V::sub(iup, ev), tup);
        T h = V::max3(x, dn, in);
        if constexpr (LOCAL) h = V::vmax(h, floor_v);
        const T tn = V::sub(h, oev);
        const T en = V::vmax(V::sub(dn, ev), tn);
        if constexpr (DIR) {
          // sign set: kind 0 diagonal loses, 1 deletion loses, 2 deletion
          // extends into the NEXT column (read by the walker one step back),
          // 3 insertion extends
          // the first row of a word takes the whole sign bytes, each later
          // row keeps the bits below it and overwrites the rest (bits above
          // the word's last row are copies of that row and never read)
          const uint32_t s01 = __builtin_amdgcn_perm((uint32_t)V::sub(dn, h), (uint32_t)V::sub(x, h), V::kSignSel);
          const uint32_t s23 = __builtin_amdgcn_perm((uint32_t)V::sub(tup, in), (uint32_t)V::sub(tn, en), V::kSignSel);
          constexpr int w = (r >> 3) * 2;
          if constexpr ((r & 7) == 0) {
            acc[w] = s01;
            acc[w + 1] = s23;
          } else {
            constexpr uint32_t low = ((1u << (r & 7)) - 1u) * 0x01010101u;
            acc[w] = bfi_op(low, acc[w], s01);
            acc[w + 1] = bfi_op(low, acc[w + 1], s23);
          }
        }
        if constexpr (TRACK) {
          if constexpr (NP == 2) {
            // a strictly better value moves the row's best and its column
            uint32_t msk = V::negmask(V::sub(bb[r], h));
            if constexpr (CHECK) {
              msk &= vmask;
              bb[r] = bfi(msk, h, bb[r]);
            } else {
              bb[r] = V::vmax(bb[r], h);
            }
            cc[r] = bfi(msk, jj, cc[r]);
          } else {
            const bool ok = (h > bb[r]) && (!CHECK || j <= n[0]);
            bb[r] = ok ? h : bb[r];
            cc[r] = ok ? jj : cc[r];
          }
        }
        if constexpr (SAT) {
          hmax = V::vmax(hmax, h);
          tmin = V::vmin(tmin, tn);
        }
        hdiag = H[r];
        H[r] = h;
        E[r] = en;
        tup = tn;
        iup = in;
#if MICA_ROW_SCHED_BARRIER
        // rows in order: keeps the live set to one row's temporaries
        __builtin_amdgcn_sched_barrier(0);
#endif
      });
      i_last = iup;
      t_last = tup;
    }
    if constexpr (EXT) {
      // (the other lanes of tsh hold T values of this step, already counted)
      if constexpr (SAT) tmin = V::vmin(tmin, tsh);
      tsh = V::sub(tsh, ev);
    }
    if (((t + 2) & (kRing / 2 - 1)) == 0) fill_ring(t + 2);
    rs_b = ring[(t + 2 - k) & (kRing - 1)];
    if constexpr (DIR) {
      if constexpr (NW == 4)
        dir4[t * 64 + lane] = (u32x4){acc[0], acc[1], acc[2], acc[3]};
      else
        dir2[t * 64 + lane] = (u32x2){acc[0], acc[1]};
    }
    if constexpr (MODE == 0) {
      // row m sits in the last register of the last lane: column t - P + 2
      const int jl = t - P + 2;
      if (jl >= 1) {
        if constexpr (NP == 2) {
          const uint32_t hm = (uint32_t)H[R - 1];
          const uint32_t jk = 0xFFFFu - (uint32_t)jl;
          int32_t k0 = (int32_t)((hm << 16) | jk);
          int32_t k1 = (int32_t)((hm & 0xFFFF0000u) | jk);
          if constexpr (CHECK) {
            k0 = jl <= n[0] ? k0 : INT32_MIN;
            k1 = jl <= n[1] ? k1 : INT32_MIN;
          }
          best_key[0] = k0 > best_key[0] ? k0 : best_key[0];
          best_key[1] = k1 > best_key[1] ? k1 : best_key[1];
        } else {
          const int32_t hm = (int32_t)H[R - 1];
          const bool ok = (hm > best_h32) && (!CHECK || jl <= n[0]);
          best_h32 = ok ? hm : best_h32;
          best_j32 = ok ? jl : best_j32;
        }
      }
    }
  };

  const int t_end = nmax + P - 1;
  int t = 0;
  for (; t < (P - 1 < t_end ? P - 1 : t_end); ++t) step(t, std::true_type{});
  // two steps per iteration: each step's new H goes to the registers the
  // step before freed, so the loop needs no copies at its back edge
  for (; t + 1 < nmin; t += 2) {
    step(t, std::false_type{});
    step(t + 1, std::false_type{});
  }
  for (; t < nmin; ++t) step(t, std::false_type{});
  for (; t < t_end; ++t) step(t, std::true_type{});

  // ---- result cell ------------------------------------------------------------
  // red[(g*NP + h)*4 + {0,1,2}] = shifted score, i*, j*
  if constexpr (MODE == 0) {
    if (k == P - 1) {
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        int sc, jj;
        if constexpr (NP == 2) {
          sc = best_key[h] >> 16;
          jj = 0xFFFF - (best_key[h] & 0xFFFF);
        } else {
          sc = best_h32;
          jj = best_j32;
        }
        red[(g * NP + h) * 4 + 0] = (uint32_t)sc;
        red[(g * NP + h) * 4 + 1] = (uint32_t)m[h];
        red[(g * NP + h) * 4 + 2] = (uint32_t)jj;
      }
    }
  } else {
    // per lane: best over its real rows, order (score desc, j asc, i asc);
    // the start cell (0,0) is worth 0 (local, shifted by -d0) or h0
    // (extension).  An extension's lane holding row m also leaves that row's
    // best (the end-to-end candidate) in gsl.
    uint32_t* gsl = lds + kGslOff;
    int fb[NP], fc[NP], fi[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      int b0 = EXT ? h0[h] : -d0[h], c0 = 0, i0 = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int u = k * R + r;
        if (EXT ? u < m[h] : u >= d0[h]) {
          int bv, cv;
          if constexpr (NP == 2) {
            bv = V::get(bb[r], h);
            cv = (int)((uint32_t)cc[r] >> (16 * h) & 0xFFFFu);
          } else {
            bv = bb[r];
            cv = cc[r];
          }
          const int iv = u - d0[h] + 1;
          if (bv > b0 || (bv == b0 && (cv < c0 || (cv == c0 && iv < i0)))) {
            b0 = bv;
            c0 = cv;
            i0 = iv;
          }
          if (EXT && u == m[h] - 1) {
            gsl[(g * NP + h) * 2 + 0] = (uint32_t)bv;
            gsl[(g * NP + h) * 2 + 1] = (uint32_t)cv;
          }
        }
      }
      // the group's best: the largest score over its lanes, then among the
      // lanes that hold it the smallest (j, i) (j < 2^13, i < 2^11)
      int smax = b0;
#pragma unroll
      for (int d = 1; d < P; d <<= 1) {
        const int o = __shfl_xor(smax, d, 64);
        smax = o > smax ? o : smax;
      }
      int key = b0 == smax ? (c0 << 11) | i0 : 0x7FFFFFFF;
#pragma unroll
      for (int d = 1; d < P; d <<= 1) {
        const int o = __shfl_xor(key, d, 64);
        key = o < key ? o : key;
      }
      fb[h] = smax;
      fc[h] = key >> 11;
      fi[h] = key & 2047;
    }
    lds_wait();
    if (k == P - 1) {
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        if constexpr (EXT) {
          // end to end when that is within the clipping penalty of the early end
          const int gv = m[h] > 0 ? (int)gsl[(g * NP + h) * 2 + 0] : h0[h];
          const int gc = m[h] > 0 ? (int)gsl[(g * NP + h) * 2 + 1] : 0;
          if ((long)gv >= (long)fb[h] - (long)prm->ext_clip) {
            fb[h] = gv;
            fc[h] = gc;
            fi[h] = m[h];
          }
        }
      }
    }
    lds_wait();
    if (k == P - 1) {
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        red[(g * NP + h) * 4 + 0] = (uint32_t)fb[h];
        red[(g * NP + h) * 4 + 1] = (uint32_t)fi[h];
        red[(g * NP + h) * 4 + 2] = (uint32_t)fc[h];
      }
    }
  }
  // saturation: any lane of the group flags the pair
  bool sat_h[NP];
#pragma unroll
  for (int h = 0; h < NP; ++h) sat_h[h] = false;
  if constexpr (SAT) {
    const int gd = (sa > -sb ? sa : -sb) > oe ? (sa > -sb ? sa : -sb) : oe;
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      const bool mine = V::get(hmax, h) >= 32767 - gd || V::get(tmin, h) <= -32768 + gd;
      const uint64_t bal = __ballot(mine);
      uint64_t gm = ~0ull;
      if constexpr (P < 64) gm = ((1ull << (P < 64 ? P : 0)) - 1) << (g * P);
      sat_h[h] = (bal & gm) != 0;
    }
  }
  lds_wait();
  if constexpr (TB == kTbBand) {
    if constexpr (P == 16) {
      // the caller refills the pending pairs (pending_take)
      band_route<V, P, R, MODE>(prm, gpairs, npairs, lds, sat_h, bucket, pending_list(prm, slot), pend);
    } else {
      band_traceback<V, P, R, MODE, false>(prm, gpairs, npairs, lds, slot, sat_h, bucket);
    }
    return;
  }
  if constexpr (DIR) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");

  // ---- outputs and traceback ---------------------------------------------------
  // The X = P / NP lanes h*X .. h*X + X - 1 of a group serve its pair h.  In
  // the walk, lane x of them examines cells x, x + X, ... ahead, so one
  // iteration consumes a run of diagonal moves of up to 64 cells, or of
  // deletion or insertion moves of up to X cells (a ballot finds where the
  // run stops).  The walk's state is the same in
  // all X lanes; lane x = 0 writes the outputs.
  constexpr int X = P / NP;
  const int h = k / X;
  const int x = k - h * X;
  if (g * NP + h < npairs) {
    // the pair's parameters are read again here rather than kept in
    // registers across the fill loop
    const int p_ = (int)gpairs[g * NP + h];
    const int m_ = G(prm->read_len)[p_];
    const int n_ = G(prm->win_len)[p_];
    const uint64_t wo_ = G(prm->win_off)[p_];
    const uint64_t ro_ = G(prm->read_off)[p_];
    const int d0_ = EXT ? 0 : PR - m_;
    bool sat_;
    if constexpr (NP == 2) sat_ = h ? sat_h[1] : sat_h[0];
    else sat_ = sat_h[0];
    if (sat_) {
      if (x == 0) {
        const uint32_t pos = atomicAdd(&prm->counters[kCtrRerun], 1u);
        G(prm->rerun)[pos] = (uint32_t)p_;
      }
    } else {
      const int score = (int)red[(g * NP + h) * 4 + 0] + d0_;
      const int ie = (int)red[(g * NP + h) * 4 + 1];
      const int je = (int)red[(g * NP + h) * 4 + 2];
      if (x == 0) {
        G(prm->score)[p_] = score;
        G(prm->read_end)[p_] = ie;
        G(prm->ref_end)[p_] = je;
      }
      uint32_t st = 0;
      if constexpr (DIR) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        MICA_GLOBAL uint32_t* stg = (MICA_GLOBAL uint32_t*)(slot + prm->dir_bytes) +
                                    (size_t)(g * NP + h) * (size_t)prm->stage_stride;
        const MICA_GLOBAL uint32_t* dirw = (const MICA_GLOBAL uint32_t*)slot;  // NW words per (step, lane)
        int i = ie, j = je;
        int hval = score;  // true H of the current cell (local zero test)
        int state = 0;     // 0: H, 1: D, 2: I
        int nruns = 0, cur_op = -1, cur_len = 0;
        // The walk only consumes cells 1 <= i <= m, 1 <= j <= n and lowers i
        // or j with every cell, so it emits at most ie + je ops.  A cell
        // outside the matrix can only come from inconsistent direction bits:
        // the walk then stops and the pair is flagged instead of reading out
        // of range.
        bool bad = ie < 0 || ie > m_ || je < 0 || je > n_;
        const int lane0 = lane - x;
        constexpr uint64_t xmask = X == 64 ? ~0ull : ((1ull << (X == 64 ? 0 : X)) - 1);
        auto sub = [&](bool pr) -> uint64_t { return (__ballot(pr) >> lane0) & xmask; };
        // index of the first clear bit of a sub-group mask (X when all are set)
        auto first_clear = [&](uint64_t msk) -> int {
          const uint64_t z = ~msk & xmask;
          return z ? (int)__builtin_ctzll(z) : X;
        };
        // a diagonal run is examined C cells per lane, X*C <= 64 at a time
        // (measured: 64 cells pay off on the long diagonals of semi-global
        // reads and, by 1%, of extensions; local walks, with more turns and
        // a prefix sum per cell for the zero test, do as well with 32 or
        // fewer)
        constexpr int C = MODE != 1 ? 64 / X : (X <= 16 ? 4 : (X == 32 ? 2 : 1));
        constexpr int XC = X * C;
        constexpr uint64_t xcmask = XC == 64 ? ~0ull : ((1ull << (XC == 64 ? 0 : XC)) - 1);
        auto first_clear_xc = [&](uint64_t msk) -> int {
          const uint64_t z = ~msk & xcmask;
          return z ? (int)__builtin_ctzll(z) : XC;
        };
        // direction word `which` (0: kinds 0 and 1, 1: kinds 2 and 3) of cell
        // (ii, jj), taken from step offset dt; *bit receives the bit of kinds 0
        // and 2 (kinds 1 and 3 sit 16 bits higher)
        auto dir_word = [&](int ii, int jj, int dt, int which, int* bit) -> uint32_t {
          const int u = d0_ + ii - 1;
          const int kk = u / R;
          const int rr = u - kk * R;
          const int ts = jj + kk - 1 + dt;
          *bit = 8 * h + (rr & 7);
          const int wsel = (NW == 4 && rr >= 8 ? 2 : 0) + which;
          return dirw[((size_t)ts * 64 + (size_t)(g * P + kk)) * NW + (size_t)wsel];
        };
        auto emit = [&](int op, int len) {
          if (op == cur_op) {
            cur_len += len;
          } else {
            if (cur_len > 0) {
              if (x == 0) stg[nruns] = ((uint32_t)cur_len << 4) | (uint32_t)cur_op;
              ++nruns;
            }
            cur_op = op;
            cur_len = len;
          }
        };
        while (!bad) {
          if (state == 0) {
            if (LOCAL && hval == 0) break;
            if (i == 0) {
              if (EXT && j > 0) {  // an extension starts at the anchor: a leading deletion
                emit(2, j);
                j = 0;
              }
              break;
            }
            if (!LOCAL && j == 0) {  // a leading insertion (semi-global, extension)
              emit(1, i);
              i = 0;
              break;
            }
            if (i < 1 || j < 1 || i > m_ || j > n_) {
              bad = true;
              break;
            }
            // lane x: the diagonal cells c = x + X*cc, cc < C, that is
            // (i - c, j - c); all their loads are in flight at once
            bool in[C], diag[C], dlose[C];
            int sc[C], incl[C];
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
              const int c = x + X * cc;
              const int ic = i - c, jc = j - c;
              in[cc] = ic >= 1 && jc >= 1;
              diag[cc] = false;
              dlose[cc] = false;
              sc[cc] = 0;
              if (in[cc]) {
                int bit;
                const uint32_t w = dir_word(ic, jc, 0, 0, &bit);
                diag[cc] = ((w >> bit) & 1u) == 0;
                dlose[cc] = ((w >> (bit + 16)) & 1u) != 0;
                if constexpr (LOCAL) {
                  const uint64_t qp = ro_ + (uint64_t)(ic - 1), rp = wo_ + (uint64_t)(jc - 1);
                  const uint32_t qb = (reads2b[qp >> 4] >> (2 * (uint32_t)(qp & 15))) & 3u;
                  const uint32_t rb = (ref2b[rp >> 4] >> (2 * (uint32_t)(rp & 15))) & 3u;
                  sc[cc] = qb == rb ? sa : sb;
                }
              }
            }
            // local: the H of cell c is hval less the scores of cells 0..c-1
            // (incl[cc]: the scores of cells 0..c), and the walk stops before
            // a cell whose H is 0
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
              incl[cc] = sc[cc];
              if constexpr (LOCAL) {
#pragma unroll
                for (int d = 1; d < X; d *= 2) {
                  const int t = __shfl_up(incl[cc], d, X);
                  if (x >= d) incl[cc] += t;
                }
                if (cc > 0) incl[cc] += __shfl(incl[cc - 1], X - 1, X);
              }
            }
            uint64_t good = 0, turn = 0, dl = 0;
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
              const bool zero = LOCAL && hval - (incl[cc] - sc[cc]) == 0;
              good |= sub(in[cc] && diag[cc] && !zero) << (X * cc);
              turn |= sub(in[cc] && !diag[cc] && !zero) << (X * cc);
              dl |= sub(dlose[cc]) << (X * cc);
            }
            const int L = first_clear_xc(good);
            if (L > 0) {
              emit(0, L);
              if constexpr (LOCAL) {
                int used = 0;
#pragma unroll
                for (int cc = 0; cc < C; ++cc)
                  if ((L - 1) / X == cc) used = __shfl(incl[cc], (L - 1) % X, X);
                hval -= used;
              }
              i -= L;
              j -= L;
            }
            // a cell that turns into a gap sets the state here; boundaries,
            // range and the zero stop are left to the next iteration
            if (L < XC && ((turn >> L) & 1u)) state = ((dl >> L) & 1u) ? 2 : 1;
            continue;
          }
          if (i < 1 || j < 1 || i > m_ || j > n_) {
            bad = true;
            break;
          }
          if (state == 1) {
            // a deletion along row i: the extend bit of (i, j - x) was stored
            // with column j - x - 1; at column 1 a deletion can only open
            const int jc = j - x;
            bool ext = false;
            if (jc >= 2) {
              int bit;
              const uint32_t w = dir_word(i, jc, -1, 1, &bit);
              ext = ((w >> bit) & 1u) != 0;
            }
            const int ones = first_clear(sub(ext));
            if (ones < X) {  // cells 0..ones-1 extend, cell `ones` opens
              const int L = ones + 1;
              emit(2, L);
              hval += oe + (L - 1) * se;
              j -= L;
              state = 0;
            } else {
              emit(2, X);
              hval += X * se;
              j -= X;
            }
          } else {
            // an insertion up column j: the extend bit of (i - x, j)
            const int ic = i - x;
            const bool in = ic >= 1;
            bool ext = false;
            if (in) {
              int bit;
              const uint32_t w = dir_word(ic, j, 0, 1, &bit);
              ext = ((w >> (bit + 16)) & 1u) != 0;
            }
            const int ones = first_clear(sub(ext));
            const uint64_t inm = sub(in);
            if (ones < X && ((inm >> ones) & 1u)) {
              const int L = ones + 1;
              emit(1, L);
              hval += oe + (L - 1) * se;
              i -= L;
              state = 0;
            } else {
              // X extensions, or a run that would leave the matrix (flagged
              // by the range check of the next iteration)
              emit(1, ones);
              hval += ones * se;
              i -= ones;
            }
          }
        }
        if (cur_len > 0) {
          if (x == 0) stg[nruns] = ((uint32_t)cur_len << 4) | (uint32_t)cur_op;
          ++nruns;
        }
        if (bad) {
          st |= kStInternal;
          i = j = 0;
          nruns = 0;
        }
        if (x == 0) {
          if (prm->flags & (kOutStart | kOutCigar)) {
            G(prm->read_start)[p_] = i;
            G(prm->ref_start)[p_] = j;
          }
          if (prm->flags & kOutCigar) {
            const int cap = prm->cigar_cap;
            MICA_GLOBAL uint32_t* out = G(prm->cigar) + (size_t)p_ * (size_t)cap;
            const int ncopy = nruns < cap ? nruns : cap;
            for (int y = 0; y < ncopy; ++y) out[y] = stg[nruns - 1 - y];
            if (nruns > cap) {
              st |= kStCigarTrunc;
              G(prm->n_cigar)[p_] = -nruns;
            } else {
              G(prm->n_cigar)[p_] = nruns;
            }
          }
        }
      }
      if (x == 0) G(prm->status)[p_] = st;
    }
  }
  lds_wait();
}

// ----------------------------------------------------------------------------
// dispatch of (kind, class, mode) to the specialised item function

template <int TB, int CLS, int KIND, int MODE>
__device__ __forceinline__ void run_one(const Params* prm, const uint32_t* pairs, int np,
                                        uint32_t* lds, uint8_t* slot, int bucket, int* pend = nullptr) {
  constexpr int P = class_lanes(CLS);
  constexpr int R = class_rows(CLS);
  if constexpr (KIND == kK32)
    process_item<V32, P, R, MODE, TB, false>(prm, pairs, np, lds, slot, bucket, pend);
  else
    process_item<V16, P, R, MODE, TB, KIND == kK16Sat>(prm, pairs, np, lds, slot, bucket, pend);
}

template <int TB, int MODE, int CLS, int CHI>
__device__ __forceinline__ void dispatch(int bucket, const Params* prm, const uint32_t* pairs, int np,
                                         uint32_t* lds, uint8_t* slot, int* pend = nullptr) {
  if constexpr (CLS <= CHI) {
    if (bucket_class(bucket) == CLS) run_one<TB, CLS, kK16, MODE>(prm, pairs, np, lds, slot, bucket, pend);
    else dispatch<TB, MODE, CLS + 1, CHI>(bucket, prm, pairs, np, lds, slot, pend);
  }
}

// the full traceback of a bucket's wide-band pairs, in its fallback class
template <int MODE, int CLS, int CHI>
__device__ __forceinline__ void dispatch_fallback(int bucket, const Params* prm, const uint32_t* pairs, int np,
                                                  uint32_t* lds, uint8_t* slot) {
  if constexpr (CLS <= CHI) {
    if (bucket_class(bucket) == CLS) run_one<kTbFull, fallback_class(CLS), kK16, MODE>(prm, pairs, np, lds, slot, bucket);
    else dispatch_fallback<MODE, CLS + 1, CHI>(bucket, prm, pairs, np, lds, slot);
  }
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// How many of a wave's pending pairs to refill next (at most an item's
// worth): an item's worth once there are that many, and the rest too when
// the wave's work ends or moves to another bucket.  Refilled before each
// fill item, the list never holds more than two items' worth less one
// (within its kPendWords words).
__device__ __forceinline__ int pending_take(int pend, int ppi, bool all) {
  return pend >= ppi ? ppi : (all ? pend : 0);
}
// After n of the pending pairs were refilled: the rest to the front.
__device__ __forceinline__ int pending_drop(MICA_GLOBAL uint32_t* pl, int pend, int n) {
  const int rest = pend - n;  // <= n: the two ranges do not overlap
  const int lane = threadIdx.x & 63;
  if (rest > 0) {
    uint32_t v = 0;
    if (lane < rest) v = pl[n + lane];
    if (lane < rest) pl[lane] = v;
  }
  return rest;
}
// The pending pairs' stores are read back by the same wave.
__device__ __forceinline__ void pending_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Deferred band item idx of a bucket: the items of the pairs with 33-64
// diagonals first (stored from the end of the bucket's range down), then
// those of 17-32 (from its start up).  Returns the item's pairs and count.
__device__ __forceinline__ const uint32_t* deferred_item(const Params* __restrict__ prm, int bucket, uint32_t idx,
                                                         int ppi, int* np) {
  const uint32_t nw = G(prm->dbwide)[bucket], nn = G(prm->dbcount)[bucket];
  const uint32_t iw = (nw + (uint32_t)ppi - 1) / (uint32_t)ppi;
  const uint32_t bs = G(prm->bstart)[bucket];
  const bool wide = idx < iw;
  const uint32_t first = (wide ? idx : idx - iw) * (uint32_t)ppi;
  const uint32_t cnt = wide ? nw : nn;
  const uint32_t base = wide ? bs + G(prm->bcount)[bucket] - nw : bs;
  *np = (int)((cnt - first) < (uint32_t)ppi ? (cnt - first) : (uint32_t)ppi);
  return prm->dbsorted + base + first;
}

// Persistent launch (one per mode and class part): every resident wave takes
// work items from its part of the queue (buckets in descending cost order)
// until it is empty.
template <int TB, int MODE, int PART>
__global__ __launch_bounds__(256, persist_waves(TB, MODE, PART)) void
k_fill_persistent(const Params* __restrict__ prm) {
  constexpr int QP = persist_queue_part(MODE, PART);
  constexpr int CLO = PART == 0 ? 0 : kPersistSmallMax + 1;
  constexpr int CHI = PART == 0 ? kPersistSmallMax : kPersistMaxClass;
  extern __shared__ uint32_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int slot_id = blockIdx.x * kWavesPerBlock + wave;
  if (slot_id >= prm->n_slots) return;
  uint32_t* lds = smem + wave * kLdsWaveWords;
  uint8_t* slot = prm->scratch + (size_t)slot_id * prm->slot_bytes;
  const int q0 = (int)prm->persist_q[QP], q1 = (int)prm->persist_q[QP + 1];
  const uint32_t base_item = G(prm->qstart)[q0];
  const uint32_t total = G(prm->qstart)[q1];
  // waves beyond the part's item count leave at once (see k_fill_bucket)
  if ((uint32_t)slot_id >= total - base_item) return;
  // the wave's pending pairs (banded fills) all belong to pend_bucket
  int pend = 0, pend_bucket = -1;
  for (;;) {
    uint32_t v = 0;
    if (lane == 0) v = atomicAdd(&prm->counters[kCtrQueueHead + QP], 1u);
    const uint32_t item = base_item + wave_uniform(v);
    const bool done = item >= total;
    int bucket = -1, np = 0;
    const uint32_t* pairs = nullptr;
    if (!done) {
      // queue position: last q with qstart[q] <= item
      int lo = q0, hi = q1 - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G(prm->qstart)[mid] <= item) lo = mid;
        else hi = mid - 1;
      }
      bucket = (int)G(prm->qorder)[lo];
      const uint32_t idx = item - G(prm->qstart)[lo];
      const int ppi = pairs_per_item(bucket_kind(bucket), bucket_class(bucket));
      const uint32_t first = idx * (uint32_t)ppi;
      const uint32_t cnt = G(prm->bcount)[bucket];
      np = (int)((cnt - first) < (uint32_t)ppi ? (cnt - first) : (uint32_t)ppi);
      pairs = prm->sorted + G(prm->bstart)[bucket] + first;
    }
    if constexpr (TB == kTbBand) {
      // the one refill site: an item's worth of pending pairs, and all of
      // them when the wave moves to another bucket or its work ends (at
      // most two passes: each takes at least one pair)
      for (;;) {
        const int nf = pending_take(pend, 8, done || bucket != pend_bucket);
        if (nf == 0) break;
        MICA_GLOBAL uint32_t* pl = pending_list(prm, slot);
        pending_fence();
        dispatch<kTbPend, MODE, CLO, CHI>(pend_bucket, prm, (const uint32_t*)pl, nf, lds, slot);
        pend = pending_drop(pl, pend, nf);
      }
      pend_bucket = bucket;
    }
    if (done) break;
    dispatch<TB, MODE, CLO, CHI>(bucket, prm, pairs, np, lds, slot, &pend);
  }
}

// Persistent launch over the side lists of the persistent buckets (one per
// mode and class part): one queue that holds first the items of the pairs
// whose band was too wide (full traceback: the longest items, so they start
// first and their latency overlaps the rest), then the items of the pairs
// with bands of 17-64 diagonals (band refill).
template <int MODE, int PART>
__global__ __launch_bounds__(256, persist_waves(kTbFull, MODE, PART)) void
k_side_persistent(const Params* __restrict__ prm) {
  constexpr int QP = persist_queue_part(MODE, PART);
  constexpr int CLO = PART == 0 ? 0 : kPersistSmallMax + 1;
  constexpr int CHI = PART == 0 ? kPersistSmallMax : kPersistMaxClass;
  extern __shared__ uint32_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int slot_id = blockIdx.x * kWavesPerBlock + wave;
  if (slot_id >= prm->n_slots) return;
  uint32_t* lds = smem + wave * kLdsWaveWords;
  uint8_t* slot = prm->scratch + (size_t)slot_id * prm->slot_bytes;
  const int q0 = (int)prm->persist_q[QP], q1 = (int)prm->persist_q[QP + 1];
  const uint32_t fb0 = G(prm->fbqstart)[q0];
  const uint32_t nfb = G(prm->fbqstart)[q1] - fb0;
  const uint32_t db0 = G(prm->dbqstart)[q0];
  const uint32_t total = nfb + (G(prm->dbqstart)[q1] - db0);
  if ((uint32_t)slot_id >= total) return;
  for (;;) {
    uint32_t v = 0;
    if (lane == 0) v = atomicAdd(&prm->counters[kCtrSideHead + QP], 1u);
    const uint32_t k = wave_uniform(v);
    if (k >= total) break;
    const bool full = k < nfb;
    const uint32_t* qstart = full ? prm->fbqstart : prm->dbqstart;
    const uint32_t item = full ? fb0 + k : db0 + (k - nfb);
    int lo = q0, hi = q1 - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (G(qstart)[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const int bucket = (int)G(prm->qorder)[lo];
    const uint32_t idx = item - G(qstart)[lo];
    const int cls = bucket_class(bucket);
    if (full) {
      const int ppi = pairs_per_item(bucket_kind(bucket), fallback_class(cls));
      const uint32_t first = idx * (uint32_t)ppi;
      const uint32_t cnt = G(prm->fbcount)[bucket];
      const int np = (int)((cnt - first) < (uint32_t)ppi ? (cnt - first) : (uint32_t)ppi);
      dispatch_fallback<MODE, CLO, CHI>(bucket, prm, prm->fbsorted + G(prm->bstart)[bucket] + first, np, lds, slot);
    } else {
      int np;
      const uint32_t* list = deferred_item(prm, bucket, idx, pairs_per_item(bucket_kind(bucket), cls), &np);
      dispatch<kTbDefer, MODE, CLO, CHI>(bucket, prm, list, np, lds, slot);
    }
  }
}

// Waves of a plain launch take the items of one bucket from a queue head (items
// differ in cost: window lengths and traceback paths vary).  Any number of
// waves drains the queue, so waves beyond the item count leave at once
// rather than contend for the head (an empty list then costs its launch only).
template <int TB, int KIND, int CLS, int MODE>
__device__ __forceinline__ void drain_list(const Params* __restrict__ prm, const uint32_t* base, uint32_t cnt,
                                           uint32_t* head) {
  extern __shared__ uint32_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int slot_id = blockIdx.x * kWavesPerBlock + wave;
  if (slot_id >= prm->n_slots) return;
  uint32_t* lds = smem + wave * kLdsWaveWords;
  uint8_t* slot = prm->scratch + (size_t)slot_id * prm->slot_bytes;
  constexpr int bucket = bucket_id(KIND, CLS, MODE);
  constexpr int ppi = pairs_per_item(KIND, CLS);
  const uint32_t items = (cnt + ppi - 1) / ppi;
  if ((uint32_t)slot_id >= items) return;
  int pend = 0;  // the wave's pending pairs (banded fills of 16-lane classes)
  for (;;) {
    uint32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(head, 1u);
    const uint32_t it = wave_uniform(v);
    if constexpr (TB == kTbBand && class_lanes(CLS) == 16) {
      // one refill site: an item's worth of pending pairs, and at the end
      // the rest (at most two passes: each takes at least one pair)
      for (;;) {
        const int nf = pending_take(pend, ppi, it >= items);
        if (nf == 0) break;
        MICA_GLOBAL uint32_t* pl = pending_list(prm, slot);
        pending_fence();
        run_one<kTbPend, CLS, KIND, MODE>(prm, (const uint32_t*)pl, nf, lds, slot, bucket);
        pend = pending_drop(pl, pend, nf);
      }
    }
    if (it >= items) break;
    const uint32_t first = it * ppi;
    const int np = (int)((cnt - first) < (uint32_t)ppi ? (cnt - first) : (uint32_t)ppi);
    run_one<TB, CLS, KIND, MODE>(prm, base + first, np, lds, slot, bucket, &pend);
  }
}

// Plain launch: one bucket per kernel.
template <int TB, int KIND, int CLS, int MODE>
__global__ __launch_bounds__(256, MICA_BUCKET_WAVES(KIND, CLS, MODE, TB)) void k_fill_bucket(const Params* __restrict__ prm) {
  constexpr int bucket = bucket_id(KIND, CLS, MODE);
  drain_list<TB, KIND, CLS, MODE>(prm, prm->sorted + G(prm->bstart)[bucket], G(prm->bcount)[bucket],
                                  &prm->bhead[bucket]);
}

// The side lists of one bucket after its banded fill: the full traceback of
// the pairs whose band was too wide (first: the longest items), then the
// band refill of the pairs with bands of 17-64 diagonals, from one queue.
template <int KIND, int CLS, int MODE>
__global__ __launch_bounds__(256, MICA_BUCKET_WAVES(KIND, CLS, MODE, kTbFull)) void k_side_bucket(const Params* __restrict__ prm) {
  constexpr int bucket = bucket_id(KIND, CLS, MODE);
  constexpr int ppi = pairs_per_item(KIND, CLS);
  constexpr int FBC = fallback_class(CLS);
  constexpr int ppf = pairs_per_item(KIND, FBC);
  extern __shared__ uint32_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int slot_id = blockIdx.x * kWavesPerBlock + wave;
  if (slot_id >= prm->n_slots) return;
  uint32_t* lds = smem + wave * kLdsWaveWords;
  uint8_t* slot = prm->scratch + (size_t)slot_id * prm->slot_bytes;
  const uint32_t nfb = G(prm->fbcount)[bucket];
  const uint32_t idb = (G(prm->dbwide)[bucket] + ppi - 1) / ppi + (G(prm->dbcount)[bucket] + ppi - 1) / ppi;
  // a list that fills every resident wave several times over is bound by
  // work, not by the latency of its last items: it stays in the pair's own
  // class (no extra dummy rows)
  const bool alt = FBC != CLS && 4u * ((nfb + ppi - 1) / ppi) <= (uint32_t)prm->n_slots;
  const uint32_t ifb = alt ? (nfb + ppf - 1) / ppf : (nfb + ppi - 1) / ppi;
  const uint32_t items = ifb + idb;
  if ((uint32_t)slot_id >= items) return;
  const uint32_t bs = G(prm->bstart)[bucket];
  for (;;) {
    uint32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(&prm->sidehead[bucket], 1u);
    const uint32_t it = wave_uniform(v);
    if (it >= items) break;
    if (it < ifb) {
      const uint32_t per = alt ? ppf : ppi;
      const uint32_t first = it * per;
      const int np = (int)((nfb - first) < per ? (nfb - first) : per);
      if constexpr (FBC != CLS) {
        if (alt) run_one<kTbFull, FBC, KIND, MODE>(prm, prm->fbsorted + bs + first, np, lds, slot, bucket);
        else run_one<kTbFull, CLS, KIND, MODE>(prm, prm->fbsorted + bs + first, np, lds, slot, bucket);
      } else {
        run_one<kTbFull, CLS, KIND, MODE>(prm, prm->fbsorted + bs + first, np, lds, slot, bucket);
      }
    } else {
      int np;
      const uint32_t* list = deferred_item(prm, bucket, it - ifb, ppi, &np);
      run_one<kTbDefer, CLS, KIND, MODE>(prm, list, np, lds, slot, bucket);
    }
  }
}

template <int TB, int KIND, int MODE, int... CLS>
void fill_bucket_table(KernelFn* out, std::integer_sequence<int, CLS...>) {
  ((out[bucket_id(KIND, CLS, MODE)] = &k_fill_bucket<TB, KIND, CLS, MODE>), ...);
}
template <int KIND, int MODE, int... CLS>
void side_bucket_table(KernelFn* out, std::integer_sequence<int, CLS...>) {
  ((out[bucket_id(KIND, CLS, MODE)] = &k_side_bucket<KIND, CLS, MODE>), ...);
}
using ClassSeq = std::make_integer_sequence<int, kNumClasses>;

}  // namespace mica
