// Banded traceback (included by dp_fill.h after the value types and helpers).
//
// The fill computes every cell of the DP (the paper's full table, Methods,
// "Highly parallel dynamic programming") but keeps only scores: the result
// cell (i*, j*) and its score S.  The traceback then refills, with direction
// bits, only a band of diagonals delta = j - i that provably holds the
// alignment the traceback rules pick, and walks back through those bits.
//
// Why a band holds the path.  Every path ending at (i*, j*) with Ld deleted
// and Li inserted bases scores at most a * (#diagonal moves) minus one gap
// open and the extension costs; the number of diagonal moves is at most
// min(i*, j*) and at most i* - Li.  Against the path's score (S, or S - h0
// for an extension) that bounds Ld <= (a min(i*, j*) - S - o) / e and
// Li <= (a i* - S - o) / (a + e), so the path stays on diagonals
// [j* - i* - Ld, j* - i* + Li].
//
// Why the refill decides as the full table does.  The band DP takes the best
// over in-band paths only, so each of its H, D and I values is at most the
// full value; on the canonical path (all in the band) every prefix is
// optimal, so there the values are equal.  The traceback at a path cell
// tests the higher-priority options first: one that failed against the full
// values (smaller than the cell's value) fails against values that are no
// larger, and the one the full table takes holds with equal values.  16-bit
// values that saturate at -32768 stay below every full value (the fill
// proved the full values inside the guard band), which keeps both facts.
//
// Layout.  A band group of 16 lanes (one DPP row) holds two pairs packed in
// 16-bit halves (one pair with 32-bit values); lane l of strip s holds
// diagonal delta_lo + 16 s + l, up to 4 strips (64 diagonals).  Bands of up
// to 16 diagonals (one strip) are refilled by the fill kernel itself; a pair
// with a wider band gets its score and end cell written and is passed on to
// a later launch whose items hold only such pairs, so that one wide band
// does not make the item's other pairs pay for its extra strips.  In the
// 16-lane classes a band of one diagonal that meets row 0 where the
// alignment may start needs no refill at all (band_route writes it out),
// and the other narrow bands wait in the wave's pending list until an
// item's worth of them is refilled at once.  Row by row:
// the diagonal predecessor is in the lane, the insertion comes from the next
// diagonal one row up (a DPP shift), and the deletion, which runs along the
// row across lanes, is a max-plus prefix scan (max over the cells to the
// left of H' - o - (distance) e, with H' = max(diagonal, insertion): a cell
// whose H came from a deletion never starts a better one).  Five sign bits
// per cell and pair are kept: diagonal loses, deletion loses, the deletion
// of the cell to the right extends, the insertion of the cell below extends,
// and (local) H is zero; two rows per 32-bit word per lane.
#pragma once

namespace mica {

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return uni(v);
}

// DPP moves within a 16-lane row; lanes without a source keep `old`
#define MICA_DPP(old, src, ctrl) \
  ((T)__builtin_amdgcn_update_dpp((int)(old), (int)(src), (ctrl), 0xF, 0xF, false))
// the same move writing 0 to lanes without a source (no copy of an old value)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_zero(uint32_t src) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)src, CTRL, 0xF, 0xF, true);
}
// a | (p & m) in one instruction (the compiler splits it into and/or trees)
__device__ __forceinline__ uint32_t and_or(uint32_t p, uint32_t m, uint32_t a) {
  uint32_t d;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(d) : "v"(p), "s"(m), "v"(a));
  return d;
}
constexpr int kDppShl1 = 0x101, kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppRor15 = 0x12F, kDppBcast15 = 0x15F;  // row_ror:15, row_newbcast:15

// Per band group (or per wave for the 64-lane classes): read selectors per
// row, then the window codes.  Window entry e holds, for each pair, the code
// of column e + delta_lo (one byte per pair), so that lane l of strip s reads
// entry i + 16 s + l at row i whatever the pair's band.
template <int P, int R, int NP>
struct BandLds {
  static constexpr int kGroupWords = P == 64 ? kBandWords : kBandWords / 4;
  static constexpr int kRows = P * R;
  static constexpr int kEntries = kRows + kBandMaxW;
  static_assert(kRows * 4 + kEntries * 2 <= kGroupWords * 4, "window codes of the widest band fit");
};

// The band of a pair whose end cell (ie, je) is off row and column 0, from
// its fill result (shifted score scs, dummy rows d0, anchor score h0): the
// lowest diagonal, the width (the bounds above), and whether the refill
// cannot take it: wider than kBandMaxW diagonals, or in packed 16 bits
// values that could reach the upper clamp (the deletion scan's lane
// offsets add up to o + 16 e to values up to the pair's bound).
struct Band {
  int lo, w;
  bool wide;
};
template <int NP, bool EXT>
__device__ __forceinline__ Band band_of(const Params* __restrict__ prm, int m, int n, int d0, int h0, int scs, int ie,
                                        int je) {
  const int sa = prm->sa, so = prm->so, se = prm->se;
  const int gain = scs + d0 - h0;  // score gained over the start
  const int ad = sa * (ie < je ? ie : je) - gain - so;
  const int ai = sa * ie - gain - so;
  const int ld = ad >= 0 ? ad / se : 0;
  const int li = ai >= 0 ? ai / (sa + se) : 0;
  const int ds = je - ie;
  int lo = ds - ld, hi = ds + li;
  lo = lo < -ie ? -ie : lo;
  hi = hi > je ? je : hi;
  const long hib = EXT ? (long)h0 + (long)sa * (m < n ? m : n) : (long)sa * (m < n ? m : n) - d0;
  const int w = hi - lo + 1;
  return Band{lo, w, w > kBandMaxW || (NP == 2 && (hib + 16L * se + so > 32767 || 16L * se + so > 32767))};
}

// The pending list of a slot: after the direction-bit (or band record)
// area and the CIGAR staging of 8 pairs.
__device__ __forceinline__ MICA_GLOBAL uint32_t* pending_list(const Params* __restrict__ prm, uint8_t* slot) {
  return (MICA_GLOBAL uint32_t*)(slot + prm->dir_bytes) + (size_t)8 * (size_t)prm->stage_stride;
}

// Right after a banded fill of 16-lane groups, one lane per pair: the
// saturated pairs go to the 32-bit re-run, pairs whose band is too wide for
// the refill to the full traceback, pairs with bands of 17-64 diagonals to
// the deferred lists of the bucket (score and end cell written now).
// Outside local mode a band of one diagonal that meets row 0 where the
// alignment may start (column 0 for an extension) holds no gap: the
// alignment is that diagonal, written out at once.  Every other pair (score
// and end cell written now) joins the wave's pending list pend_list[0,
// *pend), in lane order; the caller refills the list's pairs an item at a
// time, so that a refill runs on a full item rather than on each fill
// item's few narrow bands.  The band is the one band_traceback computes.
template <class V, int P, int R, int MODE>
__device__ __forceinline__ void band_route(const Params* __restrict__ prm,
                                           const MICA_GLOBAL uint32_t* __restrict__ gpairs, int npairs,
                                           const uint32_t* lds, const bool* sat_h, int bucket,
                                           MICA_GLOBAL uint32_t* pend_list, int* pend) {
  static_assert(P == 16, "pending lists serve the 16-lane classes");
  constexpr int NP = V::kPairs;
  constexpr int PR = P * R;
  constexpr bool LOCAL = (MODE == 1);
  constexpr bool EXT = (MODE == 2);
  constexpr int X = 16 / NP;
  const int lane = threadIdx.x & 63;
  const int l = lane & 15;
  const int h = l / X;
  const int q = (lane >> 4) * NP + h;
  const uint32_t* red = lds + kRedOff;
  bool join = false;
  uint32_t pj = 0;
  if (q < npairs && l == h * X) {
    bool sat;
    if constexpr (NP == 2) sat = h ? sat_h[1] : sat_h[0];
    else sat = sat_h[0];
    const int p = (int)gpairs[q];
    if (sat) {  // the 32-bit re-run recomputes the pair
      const uint32_t pos = atomicAdd(&prm->counters[kCtrRerun], 1u);
      G(prm->rerun)[pos] = (uint32_t)p;
    } else {
      const int m = G(prm->read_len)[p];
      const int n = G(prm->win_len)[p];
      const int d0 = EXT ? 0 : PR - m;
      const int h0 = EXT ? (prm->ext_h0 ? G(prm->ext_h0)[p] : prm->ext_default_h0) : 0;
      const int scs = (int)red[q * 4 + 0];
      const int ie = (int)red[q * 4 + 1], je = (int)red[q * 4 + 2];
      // the band of the traceback
      int W = 0;
      bool wide = false;
      if (ie >= 1 && je >= 1) {
        const Band bd = band_of<NP, EXT>(prm, m, n, d0, h0, scs, ie, je);
        W = bd.w;
        wide = bd.wide;
      }
      const uint32_t bs = G(prm->bstart)[bucket];
      if (wide) {  // the full traceback after the fills
        const uint32_t pos = atomicAdd(&prm->fbcount[bucket], 1u);
        G(prm->fbsorted)[bs + pos] = (uint32_t)p;
      } else {
        G(prm->score)[p] = scs + d0;
        G(prm->read_end)[p] = ie;
        G(prm->ref_end)[p] = je;
        if (!LOCAL && W == 1 && (EXT ? je == ie : je >= ie)) {
          if (prm->flags & (kOutStart | kOutCigar)) {
            G(prm->read_start)[p] = 0;
            G(prm->ref_start)[p] = je - ie;
          }
          uint32_t st = 0;
          if (prm->flags & kOutCigar) {
            if (prm->cigar_cap >= 1) {
              G(prm->cigar)[(size_t)p * (size_t)prm->cigar_cap] = (uint32_t)ie << 4;  // ie matches/mismatches
              G(prm->n_cigar)[p] = 1;
            } else {
              st = kStCigarTrunc;
              G(prm->n_cigar)[p] = -1;
            }
          }
          G(prm->status)[p] = st;
        } else if (W > kBandInlineW) {
          // two lists in the bucket's range, so that an item of the later
          // refill runs the strips its own pairs need: up to 32 diagonals
          // from the start, wider from the end
          if (W <= 32) {
            const uint32_t pos = atomicAdd(&prm->dbcount[bucket], 1u);
            G(prm->dbsorted)[bs + pos] = (uint32_t)p;
          } else {
            const uint32_t pos = atomicAdd(&prm->dbwide[bucket], 1u);
            G(prm->dbsorted)[bs + G(prm->bcount)[bucket] - 1u - pos] = (uint32_t)p;
          }
        } else {
          join = true;
          pj = (uint32_t)p;
        }
      }
    }
  }
  const uint64_t bal = __ballot(join);
  if (join) {
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    pend_list[*pend + (int)rank] = pj;
  }
  *pend += __builtin_popcountll(bal);
}

// The banded traceback and the outputs of one work item (all lanes of the
// wave take part).  red[] holds the fill's result per pair; sat_h[h] whether
// pair h of this lane's fill group saturated.  DEFER false: right after the
// fill (bands over 16 diagonals passed on); true: the passed-on pairs.
template <class V, int P, int R, int MODE, bool DEFER>
__device__ __forceinline__ void band_traceback(const Params* __restrict__ prm,
                                               const MICA_GLOBAL uint32_t* __restrict__ gpairs, int npairs,
                                               uint32_t* lds, uint8_t* slot, const bool* sat_h, int bucket) {
  typedef typename V::T T;
  constexpr int NP = V::kPairs;
  constexpr int PR = P * R;
  constexpr bool LOCAL = (MODE == 1);
  constexpr bool EXT = (MODE == 2);
  typedef BandLds<P, R, NP> L;
  constexpr int NS = DEFER ? kBandMaxW / 16 : kBandInlineW / 16;  // strips of the refill
  const int lane = threadIdx.x & 63;
  const int bg = lane >> 4;
  const int l = lane & 15;
  const bool bg_ok = P == 16 || bg == 0;
  const int sa = prm->sa, sb = prm->sb, so = prm->so, se = prm->se;
  const int oe = so + se;
  const MICA_GLOBAL uint32_t* __restrict__ ref2b = G(prm->ref2b);
  const MICA_GLOBAL uint32_t* __restrict__ reads2b = G(prm->reads2b);
  const uint32_t* red = lds + kRedOff;

  // ---- per pair: result cell and band ----------------------------------------
  int pid[NP], mm[NP], nn[NP], d0[NP], ie[NP], je[NP], scs[NP], dlo[NP], W[NP], h0[NP];
  uint64_t wo[NP], ro[NP];
  bool valid[NP], act[NP], fb[NP], sat[NP], dfr[NP];
  int rows_l = 0, ns_l = 0, mr_l = 0;
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    const int q = bg * NP + h;
    valid[h] = bg_ok && q < npairs;
    act[h] = fb[h] = sat[h] = dfr[h] = false;
    pid[h] = -1;
    mm[h] = nn[h] = d0[h] = ie[h] = je[h] = scs[h] = h0[h] = 0;
    dlo[h] = 0;
    W[h] = 1;
    wo[h] = ro[h] = 0;
    if (valid[h]) {
      const int p = (int)gpairs[q];
      pid[h] = p;
      mm[h] = G(prm->read_len)[p];
      nn[h] = G(prm->win_len)[p];
      wo[h] = G(prm->win_off)[p];
      ro[h] = G(prm->read_off)[p];
      if constexpr (EXT) h0[h] = prm->ext_h0 ? G(prm->ext_h0)[p] : prm->ext_default_h0;
      d0[h] = EXT ? 0 : PR - mm[h];
      scs[h] = (int)red[q * 4 + 0];
      ie[h] = (int)red[q * 4 + 1];
      je[h] = (int)red[q * 4 + 2];
      sat[h] = sat_h[h];
      if (!sat[h] && ie[h] >= 1 && je[h] >= 1) {
        const Band bd = band_of<NP, EXT>(prm, mm[h], nn[h], d0[h], h0[h], scs[h], ie[h], je[h]);
        dlo[h] = bd.lo;
        W[h] = bd.w;
        fb[h] = bd.wide;
        dfr[h] = !DEFER && !fb[h] && W[h] > kBandInlineW;
        act[h] = !fb[h] && !dfr[h];
        if (act[h]) {
          rows_l = ie[h] > rows_l ? ie[h] : rows_l;
          const int ns = (W[h] + 15) >> 4;
          ns_l = ns > ns_l ? ns : ns_l;
          mr_l = -bd.lo > mr_l ? -bd.lo : mr_l;
        }
      }
    }
  }
  // the band and the pair's state travel to the walk through LDS (word 3 of
  // the pair's result), so none of the values above stays live across the
  // refill: diagonal offset + 32768 (bits 0-15), width (16-23), band (24),
  // wide band (25), saturated (26), passed on (27)
#pragma unroll
  for (int h = 0; h < NP; ++h)
    if (valid[h])
      lds[kRedOff + (bg * NP + h) * 4 + 3] = (uint32_t)(dlo[h] + 32768) |
                                             ((uint32_t)(act[h] || dfr[h] ? W[h] : 0) << 16) |
                                             (act[h] ? 1u << 24 : 0u) | (fb[h] ? 1u << 25 : 0u) |
                                             (sat[h] ? 1u << 26 : 0u) | (dfr[h] ? 1u << 27 : 0u);
  const int rows_u = wave_max_int(rows_l);
  const int ns_u = wave_max_int(ns_l);
  const int mr_u = wave_max_int(mr_l);

  // ---- codes in LDS: read selector per row, window codes per band entry -------
  uint32_t* gq = lds + (P == 64 ? 0 : bg * L::kGroupWords);
  uint16_t* gw = (uint16_t*)(gq + L::kRows);
  if (bg_ok && rows_u > 0) {
    for (int i0 = l; i0 < rows_u; i0 += 16) {
      uint32_t qs = 0;
#pragma unroll
      for (int h = 0; h < NP; ++h)
        qs |= (act[h] && i0 < ie[h]) ? V::qcode(base_at(reads2b, ro[h] + (uint64_t)i0), h) : V::qdummy(h);
      gq[i0] = qs;
    }
    // entry e, pair h: column e + delta_lo (codes outside the window are
    // never used: those cells are masked or off the band)
    const int ne = rows_u + 16 * ns_u;
    for (int e = l; e < ne; e += 16) {
      uint32_t w = 0;
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        const int j = e + dlo[h];
        if (act[h] && j >= 1 && j <= nn[h])
          w |= (uint32_t)base_at(ref2b, wo[h] + (uint64_t)(j - 1)) << (8 * h + (NP == 2 ? 1 : 0));
      }
      gw[e] = (uint16_t)w;
    }
  }
  lds_wait();

  // ---- band refill with direction bits -----------------------------------------
  MICA_GLOBAL uint32_t* rec = (MICA_GLOBAL uint32_t*)slot;
  const int ns64 = ns_u * 64;
  if (rows_u > 0) {
    const uint32_t tab_lo = ((uint32_t)sa & 0xFFFFu) | ((uint32_t)sb << 16);
    const uint32_t tab_hi = ((uint32_t)sb & 0xFFFFu) | ((uint32_t)sb << 16);
    const T negv = (T)V::kNeg;
    const T ev = V::splat(se);
    const T oev = V::splat(oe);
    const T cg = V::splat(l * se);
    const T og = V::splat(so + l * se);
    const T e16 = V::splat(16 * se);
    T floor_v = (T)0, floor1 = (T)0;
    if constexpr (LOCAL) {
      if constexpr (NP == 2) {
        floor_v = V::make2(-d0[0], -d0[1]);
        floor1 = V::make2(1 - d0[0], 1 - d0[1]);
      } else {
        floor_v = (T)(-d0[0]);
        floor1 = (T)(1 - d0[0]);
      }
    }
    // row 0: H(0, j) (nothing for j < 0); the insertion candidate of the row
    // below is H - o - e there (I(0, j) is -inf); lanes past a pair's band
    // hold -inf so they never feed it
    T Hd[NS], Ic[NS], msk[NS];
    uint32_t acc[NS];
    const uint16_t* gwl = gw + l;
    // the score table's low half as a register operand of the lookup
    uint32_t tab_lo_v;
    asm("v_mov_b32 %0, %1" : "=v"(tab_lo_v) : "s"(tab_lo));
    constexpr uint32_t kFlip = 0x80008000u;  // signed <-> offset binary (16-bit halves)
    auto pack = [&](int v0, int v1) -> T {
      if constexpr (NP == 2) return V::make2(v0, v1);
      else return (T)v0;
    };
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      int hv[2] = {0, 0}, iv[2] = {0, 0};
      bool mk[2] = {false, false}, neg[2] = {false, false};
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        const int gl = 16 * s + l;
        const int j = dlo[h] + gl;
        hv[h] = EXT ? (j == 0 ? h0[h] : h0[h] - (so + j * se)) : -d0[h];
        iv[h] = hv[h] - oe;
        neg[h] = j < 0;
        mk[h] = act[h] && gl < W[h];
      }
      uint32_t nm = 0;
      if constexpr (NP == 2) {
        Hd[s] = V::make2(hv[0], hv[1]);
        Ic[s] = V::make2(iv[0], iv[1]);
        msk[s] = (mk[0] ? 0xFFFFu : 0u) | (mk[1] ? 0xFFFF0000u : 0u);
        nm = (neg[0] ? 0xFFFFu : 0u) | (neg[1] ? 0xFFFF0000u : 0u);
      } else {
        Hd[s] = (T)hv[0];
        Ic[s] = (T)iv[0];
        msk[s] = mk[0] ? ~0u : 0u;
        nm = neg[0] ? ~0u : 0u;
      }
      Hd[s] = (T)bfi(nm, (uint32_t)negv, (uint32_t)Hd[s]);
      Ic[s] = (T)bfi(msk[s] & ~nm, (uint32_t)Ic[s], (uint32_t)negv);
      acc[s] = 0;
    }

    auto row = [&](int i, auto par_c, auto masked_c) {
      constexpr int PAR = decltype(par_c)::value;
      constexpr bool MASKED = decltype(masked_c)::value;
      const uint32_t qs = gq[i - 1];
      T carry = negv;
      T bnd = (T)0;
      if constexpr (MASKED) {
        // H(i, 0): the column-0 boundary
        int bv[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < NP; ++h) bv[h] = LOCAL ? -d0[h] : (EXT ? h0[h] : -d0[h]) - (so + i * se);
        bnd = pack(bv[0], bv[1]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s >= ns_u) break;
        // window selector of column i + delta_lo + 16 s + l (each half its own pair)
        uint32_t rsel;
        {
          const uint32_t w = gwl[i + 16 * s];
          if constexpr (NP == 2) rsel = __builtin_amdgcn_perm(w, w, 0x01010000u);
          else rsel = w * 0x01010202u;
        }
        const T sc = (T)__builtin_amdgcn_perm(tab_hi, tab_lo_v, qs ^ rsel);
        const T x = V::add(Hd[s], sc);
        // insertion from the next diagonal one row up
        T old = negv;
        if (s + 1 < NS && s + 1 < ns_u) old = MICA_DPP(negv, Ic[s + 1 < NS ? s + 1 : s], kDppRor15);
        const T Iv = MICA_DPP(old, Ic[s], kDppShl1);
        T Hp = V::vmax(x, Iv);
        if constexpr (LOCAL) Hp = V::vmax(Hp, floor_v);
        if constexpr (MASKED) {
          // cells left of column 0 do not exist; column 0 is the boundary
          uint32_t zm = 0, nm = 0;
#pragma unroll
          for (int h = 0; h < NP; ++h) {
            const int j = i + dlo[h] + 16 * s + l;
            const uint32_t half = NP == 2 ? (0xFFFFu << (16 * h)) : ~0u;
            zm |= j == 0 ? half : 0u;
            nm |= j < 0 ? half : 0u;
          }
          Hp = (T)bfi(zm, (uint32_t)bnd, (uint32_t)Hp);
          Hp = (T)bfi(nm, (uint32_t)negv, (uint32_t)Hp);
        }
        // deletion: exclusive max-plus prefix over the row (strip-relative
        // offsets; `carry` brings the strips to the left)
        T Dv;
        if constexpr (NP == 2) {
          // in offset binary (sign bit flipped) -inf is 0, which the DPP
          // moves write into lanes without a source: no copies of -inf
          typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
          auto umax = [](uint32_t a, uint32_t b) -> uint32_t {
            return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                          __builtin_bit_cast(u16x2, b)));
          };
          uint32_t g = (uint32_t)V::add(Hp, cg) ^ kFlip;
          g = umax(g, dpp_zero<kDppShr1>(g));
          g = umax(g, dpp_zero<kDppShr2>(g));
          g = umax(g, dpp_zero<kDppShr4>(g));
          g = umax(g, dpp_zero<kDppShr8>(g));
          if (s > 0) g = umax(g, (uint32_t)carry);
          uint32_t excl = dpp_zero<kDppShr1>(g);
          if (s > 0) excl = umax(excl, (uint32_t)carry);
          Dv = V::sub((T)(excl ^ kFlip), og);
          if (s + 1 < NS && s + 1 < ns_u) carry = (T)((uint32_t)V::sub((T)(dpp_zero<kDppBcast15>(g) ^ kFlip), e16) ^ kFlip);
        } else {
          T g = V::add(Hp, cg);
          g = V::vmax(g, MICA_DPP(negv, g, kDppShr1));
          g = V::vmax(g, MICA_DPP(negv, g, kDppShr2));
          g = V::vmax(g, MICA_DPP(negv, g, kDppShr4));
          g = V::vmax(g, MICA_DPP(negv, g, kDppShr8));
          if (s > 0) g = V::vmax(g, carry);
          const T excl = MICA_DPP(carry, g, kDppShr1);
          Dv = V::sub(excl, og);
          if (s + 1 < NS && s + 1 < ns_u) carry = V::sub(MICA_DPP(negv, g, kDppBcast15), e16);
        }
        const T Hv = V::vmax(Hp, Dv);
        const T Tv = V::sub(Hv, oev);
        const T Icn = V::vmax(V::sub(Iv, ev), Tv);
        // sign bits: diagonal loses, deletion loses | deletion of the right
        // cell extends, insertion of the cell below extends | H is zero
        const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)V::sub(Dv, Hv), (uint32_t)V::sub(x, Hv), V::kSignSel);
        const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)V::sub(Tv, Icn), (uint32_t)V::sub(Tv, V::sub(Dv, ev)),
                                                   V::kSignSel);
        constexpr uint32_t M0 = 0x01010101u << (4 * PAR), M1 = 0x02020202u << (4 * PAR),
                           M2 = 0x04040404u << (4 * PAR);
        uint32_t a = acc[s];
        a = and_or(p01, M0, a);
        a = and_or(p23, M1, a);
        if constexpr (LOCAL) {
          const uint32_t zr = (uint32_t)V::sub(Hv, floor1);
          a = and_or(__builtin_amdgcn_perm(zr, zr, V::kSignSel), M2, a);
        }
        acc[s] = a;
        Hd[s] = Hv;
        Ic[s] = (T)bfi(msk[s], (uint32_t)Icn, (uint32_t)negv);
      }
    };
    auto flush = [&](int i) {  // rows i and i + 1 (1-based i odd)
      const size_t base = (size_t)((i - 1) >> 1) * (size_t)ns64 + (size_t)lane;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s >= ns_u) break;
        rec[base + (size_t)(s * 64)] = acc[s];
        acc[s] = 0;
      }
    };
    int i = 1;
    for (; i <= rows_u && i <= mr_u; i += 2) {
      row(i, std::integral_constant<int, 0>{}, std::true_type{});
      if (i + 1 <= rows_u) row(i + 1, std::integral_constant<int, 1>{}, std::true_type{});
      flush(i);
    }
    for (; i + 1 <= rows_u; i += 2) {
      row(i, std::integral_constant<int, 0>{}, std::false_type{});
      row(i + 1, std::integral_constant<int, 1>{}, std::false_type{});
      flush(i);
    }
    if (i <= rows_u) {
      row(i, std::integral_constant<int, 0>{}, std::false_type{});
      flush(i);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  lds_wait();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- outputs and the walk -------------------------------------------------------
  // X = 16 / NP lanes of a band group walk pair h together (see the walk of
  // the full traceback); every lane holds the walk state.  The pair's values
  // are read again here (global arrays, LDS results) rather than kept.
  constexpr int X = 16 / NP;
  const int h = l / X;
  const int x = l - h * X;
  const int q = bg * NP + h;
  if (bg_ok && q < npairs) {
    const int p_ = (int)gpairs[q];
    const int m_ = G(prm->read_len)[p_];
    const int n_ = G(prm->win_len)[p_];
    const int d0_ = EXT ? 0 : PR - m_;
    const uint32_t w3 = red[q * 4 + 3];
    if ((w3 >> 26) & 1u) {  // saturated: the 32-bit re-run recomputes the pair
      if (x == 0) {
        const uint32_t pos = atomicAdd(&prm->counters[kCtrRerun], 1u);
        G(prm->rerun)[pos] = (uint32_t)p_;
      }
    } else if ((w3 >> 25) & 1u) {  // band too wide: the full traceback after this launch
      if (x == 0) {
        const uint32_t pos = atomicAdd(&prm->fbcount[bucket], 1u);
        G(prm->fbsorted)[G(prm->bstart)[bucket] + pos] = (uint32_t)p_;
      }
    } else if ((w3 >> 27) & 1u) {  // band over 16 diagonals: the score now, the refill later
      if (x == 0) {
        G(prm->score)[p_] = (int)red[q * 4 + 0] + d0_;
        G(prm->read_end)[p_] = (int)red[q * 4 + 1];
        G(prm->ref_end)[p_] = (int)red[q * 4 + 2];
        // two lists in the bucket's range, so that an item of the later
        // refill runs the strips its own pairs need: up to 32 diagonals
        // from the start, wider from the end
        if (((w3 >> 16) & 0xFFu) <= 32u) {
          const uint32_t pos = atomicAdd(&prm->dbcount[bucket], 1u);
          G(prm->dbsorted)[G(prm->bstart)[bucket] + pos] = (uint32_t)p_;
        } else {
          const uint32_t pos = atomicAdd(&prm->dbwide[bucket], 1u);
          G(prm->dbsorted)[G(prm->bstart)[bucket] + G(prm->bcount)[bucket] - 1u - pos] = (uint32_t)p_;
        }
      }
    } else {
      const int score = (int)red[q * 4 + 0] + d0_;
      const int ie_ = (int)red[q * 4 + 1], je_ = (int)red[q * 4 + 2];
      const int dlo_ = (int)(w3 & 0xFFFFu) - 32768, W_ = (int)((w3 >> 16) & 0xFFu);
      if (!DEFER && x == 0) {
        G(prm->score)[p_] = score;
        G(prm->read_end)[p_] = ie_;
        G(prm->ref_end)[p_] = je_;
      }
      uint32_t st = 0;
      MICA_GLOBAL uint32_t* stg =
          (MICA_GLOBAL uint32_t*)(slot + prm->dir_bytes) + (size_t)q * (size_t)prm->stage_stride;
      int i = ie_, j = je_;
      int state = 0;  // 0: H, 1: D, 2: I
      int nruns = 0, cur_op = -1, cur_len = 0;
      bool bad = ie_ < 0 || ie_ > m_ || je_ < 0 || je_ > n_;
      const int lane0 = lane - x;
      constexpr uint64_t xmask = (1ull << X) - 1;
      auto sub = [&](bool pr) -> uint64_t { return (__ballot(pr) >> lane0) & xmask; };
      auto first_clear = [&](uint64_t msk) -> int {
        const uint64_t z = ~msk & xmask;
        return z ? (int)__builtin_ctzll(z) : X;
      };
      constexpr int C = 64 / X;
      constexpr int XC = X * C;
      auto first_clear_xc = [&](uint64_t msk) -> int {
        const uint64_t z = ~msk;
        return z ? (int)__builtin_ctzll(z) : XC;
      };
      // the record word of cell (ii, jj) (1 <= ii, inside the band) and the
      // bit offset of its row and pair half; kinds: +0 diagonal loses
      // (second half-word: deletion loses), +1 deletion of the right cell
      // extends (second: insertion of the cell below extends), +2 zero
      auto in_band = [&](int ii, int jj) -> bool {
        const int gl = jj - ii - dlo_;
        return ii >= 1 && gl >= 0 && gl < W_;
      };
      auto word = [&](int ii, int jj, int* bit) -> uint32_t {
        const int gl = jj - ii - dlo_;
        *bit = 8 * h + 4 * ((ii - 1) & 1);
        return rec[(size_t)((ii - 1) >> 1) * (size_t)ns64 + (size_t)((gl >> 4) * 64 + bg * 16 + (gl & 15))];
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
          if (i == 0) {
            if (EXT && j > 0) {  // an extension starts at the anchor: a leading deletion
              emit(2, j);
              j = 0;
            }
            break;
          }
          if (j == 0) {
            if (LOCAL) break;
            emit(1, i);  // a leading insertion (semi-global, extension)
            i = 0;
            break;
          }
          if (i > m_ || j > n_ || !in_band(i, j)) {
            bad = true;
            break;
          }
          if (LOCAL) {
            int bit;
            const uint32_t w = word(i, j, &bit);
            if ((w >> (bit + 2)) & 1u) break;  // H = 0: the local alignment starts here
          }
          // lane x: the diagonal cells c = x + X * cc, (i - c, j - c), all on
          // this lane's diagonal of the band
          uint64_t good = 0, turn = 0, dl = 0;
#pragma unroll
          for (int cc = 0; cc < C; ++cc) {
            const int c = x + X * cc;
            const int ic = i - c, jc = j - c;
            const bool in = ic >= 1 && jc >= 1;
            bool diag = false, dlose = false, zero = false;
            if (in) {
              int bit;
              const uint32_t w = word(ic, jc, &bit);
              diag = ((w >> bit) & 1u) == 0;
              dlose = ((w >> (bit + 16)) & 1u) != 0;
              zero = LOCAL && ((w >> (bit + 2)) & 1u) != 0;
            }
            good |= sub(in && diag && !zero) << (X * cc);
            turn |= sub(in && !diag && !zero) << (X * cc);
            dl |= sub(dlose) << (X * cc);
          }
          const int Lr = first_clear_xc(good);
          if (Lr > 0) {
            emit(0, Lr);
            i -= Lr;
            j -= Lr;
          }
          // a cell that turns into a gap sets the state here; boundaries,
          // range and the zero stop are left to the next iteration
          if (Lr < XC && ((turn >> Lr) & 1u)) state = ((dl >> Lr) & 1u) ? 2 : 1;
          continue;
        }
        if (i < 1 || j < 1 || i > m_ || j > n_) {
          bad = true;
          break;
        }
        if (state == 1) {
          // a deletion along row i: cell (i, j - x) extends when the bit its
          // left neighbour keeps says so; at column 1 a deletion can only open
          const int jc = j - x;
          bool ext = false;
          if (jc >= 2 && in_band(i, jc - 1)) {
            int bit;
            const uint32_t w = word(i, jc - 1, &bit);
            ext = ((w >> (bit + 1)) & 1u) != 0;
          }
          const int ones = first_clear(sub(ext));
          if (ones < X) {  // cells 0..ones-1 extend, cell `ones` opens
            emit(2, ones + 1);
            j -= ones + 1;
            state = 0;
          } else {
            emit(2, X);
            j -= X;
          }
        } else {
          // an insertion up column j: cell (i - x, j) extends when the bit of
          // the cell above says so; at row 1 an insertion can only open
          const int ic = i - x;
          const bool in = ic >= 1;
          bool ext = false;
          if (ic >= 2 && in_band(ic - 1, j)) {
            int bit;
            const uint32_t w = word(ic - 1, j, &bit);
            ext = ((w >> (bit + 17)) & 1u) != 0;
          }
          const int ones = first_clear(sub(ext));
          const uint64_t inm = sub(in);
          if (ones < X && ((inm >> ones) & 1u)) {
            emit(1, ones + 1);
            i -= ones + 1;
            state = 0;
          } else {
            // X extensions, or a run that would leave the matrix (flagged
            // by the range check of the next iteration)
            emit(1, ones);
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
        G(prm->status)[p_] = st;
      }
    }
  }
  lds_wait();
}

}  // namespace mica
