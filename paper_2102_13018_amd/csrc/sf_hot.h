// sf_hot.h -- DPP wavefront helpers and the hot-root phase of the
// partitioned path.
//
// A pass-A tile holds kPassATile consecutive leaves (in leaf order).  Its
// leaves of hot roots are listed in hx_pos grouped by root ("groups"), in
// leaf order inside a group, each entry a tile offset with bit 15 set at a
// group's first entry.  Both phases below run one block-wide segmented scan
// over these entries (segments = groups, combining in entry order):
//  * HOT_TOTALS (pass A): the value at a group's last entry is the group's
//    total, stored to gval[group] (groups numbered tile-major);
//  * HOT_FETCH (pass C of FetchAndOp): every entry gets the root's value just
//    before that leaf in leaf order: its group's base gval[group] (the root's
//    value before the tile) combined with the group's exclusive prefix.  The
//    base is folded into the first entry of its group, so the scan carries it.
// Thread t takes the K = ceil(entries / threads) consecutive entries from
// t * K: it folds them (phase 1), one DPP segmented scan per wavefront and a
// fold over the wavefronts' totals give its carry-in, and it walks them again
// (phase 2).
#pragma once

#include <type_traits>

#include "sf_device.h"

namespace sfi {

// v from the lane that the DPP control CTRL selects, for every 32-bit word
// of V (a pair's padding word is not moved).
template <int CTRL, typename V>
__device__ __forceinline__ V dpp_mov(V v) {
  constexpr int N = std::is_same<V, Pair>::value ? 3 : (int)(sizeof(V) / 4);
  static_assert(sizeof(V) % 4 == 0, "32-bit words");
  int w[sizeof(V) / 4];
  __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
  for (int k = 0; k < N; k++) w[k] = __builtin_amdgcn_mov_dpp(w[k], CTRL, 0xf, 0xf, false);
  V r;
  __builtin_memcpy(&r, w, sizeof(V));
  return r;
}
template <typename V>
__device__ __forceinline__ V read_lane(V v, int l) {
  int w[sizeof(V) / 4];
  __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
  for (int k = 0; k < (int)(sizeof(V) / 4); k++) w[k] = __builtin_amdgcn_readlane(w[k], l);
  V r;
  __builtin_memcpy(&r, w, sizeof(V));
  return r;
}
// Reduction of one value per lane over the whole wavefront (all lanes
// active), for an order-free op: every lane of a 16-lane row first holds the
// row's reduction (quad swaps, then the half-row and row mirrors), then the
// four rows are combined.
template <int OP, typename V>
__device__ __forceinline__ V wave_reduce_free(V v) {
  v = Op<OP, V>::apply(v, dpp_mov<0xB1>(v));   // quad_perm [1,0,3,2]
  v = Op<OP, V>::apply(v, dpp_mov<0x4E>(v));   // quad_perm [2,3,0,1]
  v = Op<OP, V>::apply(v, dpp_mov<0x141>(v));  // row_half_mirror
  v = Op<OP, V>::apply(v, dpp_mov<0x140>(v));  // row_mirror
  return Op<OP, V>::apply(Op<OP, V>::apply(read_lane(v, 0), read_lane(v, 16)),
                          Op<OP, V>::apply(read_lane(v, 32), read_lane(v, 48)));
}

// v from the lane that the DPP control CTRL selects, in the rows ROWMASK
// enables; a lane without a source lane, or in a disabled row, gets old.
template <int CTRL, int ROWMASK, typename V>
__device__ __forceinline__ V dpp_upd(V old, V v) {
  static_assert(sizeof(V) % 4 == 0, "32-bit words");
  int wo[sizeof(V) / 4], wv[sizeof(V) / 4];
  __builtin_memcpy(wo, &old, sizeof(V));
  __builtin_memcpy(wv, &v, sizeof(V));
#pragma unroll
  for (int k = 0; k < (int)(sizeof(V) / 4); k++) wo[k] = __builtin_amdgcn_update_dpp(wo[k], wv[k], CTRL, ROWMASK, 0xf, false);
  V r;
  __builtin_memcpy(&r, wo, sizeof(V));
  return r;
}
// Inclusive sum over the wavefront (all lanes active), and the exclusive one
// beside it: shifts by 1, 2, 4, 8 inside each 16-lane row, then the last lane
// of rows 0 and 2 added to rows 1 and 3, then lane 31 added to rows 2 and 3;
// the exclusive value is the inclusive one shifted by a lane.  The sums are
// associated differently from a lane-order fold: exact for integers, any
// order is allowed where this is used on floating point (atomic mode).
template <typename T>
__device__ __forceinline__ T wave_scan_sum(T v, T &excl) {
  const T z = T(0);
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x111, 0xf>(z, v));  // row_shr:1
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x112, 0xf>(z, v));  // row_shr:2
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x114, 0xf>(z, v));  // row_shr:4
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x118, 0xf>(z, v));  // row_shr:8
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x142, 0xa>(z, v));  // row_bcast:15 into rows 1, 3
  v = Op<OP_SUM, T>::apply(v, dpp_upd<0x143, 0xc>(z, v));  // row_bcast:31 into rows 2, 3
  excl = dpp_upd<0x138, 0xf>(z, v);                        // wave_shr:1
  return v;
}


// Segmented inclusive scan of one wavefront (all lanes active) by DPP moves:
// x is the lane's value, f whether a segment starts at or before the lane
// within what it holds (updated to: any start in [0, lane]).  Shifts by 1, 2,
// 4, 8 inside 16-lane rows, then the last lane of rows 0 and 2 into rows 1
// and 3, then lane 31 into rows 2 and 3; a lane combines with its source
// only while no segment has started between them.
template <int OP, typename T>
__device__ __forceinline__ T wave_seg_scan_dpp(T x, int &f, int lane) {
#define SF_SEG_STEP(CTRL, ROWMASK, HAS)                 \
  {                                                     \
    const T y = dpp_upd<CTRL, ROWMASK>(x, x);           \
    const int fy = dpp_upd<CTRL, ROWMASK>(0, f);        \
    if (HAS) {                                          \
      if (!f) x = Op<OP, T>::apply(y, x);               \
      f |= fy;                                          \
    }                                                   \
  }
  SF_SEG_STEP(0x111, 0xf, (lane & 15) >= 1)  // row_shr:1
  SF_SEG_STEP(0x112, 0xf, (lane & 15) >= 2)  // row_shr:2
  SF_SEG_STEP(0x114, 0xf, (lane & 15) >= 4)  // row_shr:4
  SF_SEG_STEP(0x118, 0xf, (lane & 15) >= 8)  // row_shr:8
  SF_SEG_STEP(0x142, 0xa, (lane >> 4) & 1)   // row_bcast:15 into rows 1, 3
  SF_SEG_STEP(0x143, 0xc, lane >= 32)        // row_bcast:31 into rows 2, 3
#undef SF_SEG_STEP
  return x;
}

constexpr int HOT_NONE = 0;
constexpr int HOT_TOTALS = 1;  // pass A of Reduce: group totals
constexpr int HOT_PREFIX = 2;  // pass A of FetchAndOp (SUM): group totals and every entry's exclusive prefix
constexpr int HOT_APPLY = 3;   // pass C of FetchAndOp: every entry's group base + its prefix
constexpr int kHotPer = 8;     // most entries per thread (kPassATile / kStageThreads)

template <typename T, int OP, int MODE>
struct HotSpec {
  using type = T;
  static constexpr int op = OP;
  static constexpr int mode = MODE;
};
struct HotNone {
  using type = int32_t;
  static constexpr int op = OP_SUM;
  static constexpr int mode = HOT_NONE;
};

struct HotArgs {
  const uint16_t *hx_pos, *hx_tg;
  const int32_t *hx_e0, *hx_grp0, *hx_rpos;
  void *gval;   // group totals (out, HOT_TOTALS / HOT_PREFIX) or bases (in, HOT_APPLY): [groups][bs], root-major
  void *gpre;   // every hot entry's exclusive prefix in its group, [entries][bs], tile-major
};

// The hot phase of one tile.  Thread t takes the K = ceil(entries / threads)
// consecutive entries from t * K.
//  HOT_TOTALS / HOT_PREFIX: values are read from the tile's units in LDS
//    (lds_units, at the tile offset; when the tile's slots are not
//    contiguous, leaf0 < 0, the hot units are first staged there from
//    leaf_units through pa_slot).  The thread folds its entries, one DPP
//    segmented scan per wavefront and a fold over the wavefronts' totals give
//    it the value carried in from earlier entries of its first group, and it
//    walks its entries again: a group's last entry stores the group's total,
//    and HOT_PREFIX stores every entry's exclusive prefix.
//  HOT_APPLY: every entry's result is its group's base combined with its
//    prefix, written over the tile in LDS (or to leaf_units at the slot).
// Group indices start from the plan's count of the groups started before a
// thread's first entry.
template <typename HS>
__device__ __forceinline__ void hot_phase(const HotArgs &ha, int tile, int64_t p0, int bs, int32_t leaf0,
                                          const int32_t *__restrict__ pa_slot,
                                          typename HS::type *lds_units, typename HS::type *leaf_units) {
  using T = typename HS::type;
  constexpr int OP = HS::op;
  constexpr int MODE = HS::mode;
  constexpr int WAVES = kStageThreads / 64;
  static_assert(kPassATile <= kHotPer * kStageThreads, "entries per thread");
  static_assert(MODE != HOT_PREFIX || OP == OP_SUM, "prefixes of sums");
  __shared__ T wtot[WAVES];       // a wavefront's scan total (its last lane's)
  __shared__ int32_t wfl[WAVES];  // whether a group starts in the wavefront's entries
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e0 = ha.hx_e0[tile], nh = ha.hx_e0[tile + 1] - e0;
  if (nh == 0) return;
  const int g0 = ha.hx_grp0[tile];
  T *gval = reinterpret_cast<T *>(ha.gval);
  T *gpre = reinterpret_cast<T *>(ha.gpre);
  const int K = (nh + kStageThreads - 1) / kStageThreads;
  const int b0 = min(threadIdx.x * K, nh), b1 = min(b0 + K, nh);
  int pos[kHotPer];
#pragma unroll
  for (int j = 0; j < kHotPer; j++) pos[j] = b0 + j < b1 ? (int)ha.hx_pos[e0 + b0 + j] : 0;
  auto slot_of = [&](int q) -> int64_t { return leaf0 >= 0 ? (int64_t)leaf0 + q : (int64_t)pa_slot[p0 + q]; };
  if (MODE != HOT_APPLY && leaf0 < 0) {  // stage this thread's units
#pragma unroll
    for (int j = 0; j < kHotPer; j++)
      if (b0 + j < b1) {
        const int q = pos[j] & 0x1fff;
        const int64_t sl = slot_of(q);
        for (int c = 0; c < bs; c++) st(lds_units + (int64_t)q * bs + c, ld(leaf_units + sl * bs + c));
      }
  }
  // groups started before the thread's first entry (from the plan)
  const int gfirst = ha.hx_tg[(int64_t)tile * kStageThreads + threadIdx.x];
  if (MODE != HOT_APPLY && leaf0 < 0) __syncthreads();  // the staged units
  if constexpr (MODE == HOT_APPLY) {
    for (int c = 0; c < bs; c++) {
      int g = gfirst - 1;
      T base{};
      if (b0 < b1 && !(pos[0] & 0x8000)) base = ld(gval + (int64_t)ha.hx_rpos[g0 + g] * bs + c);
#pragma unroll
      for (int j = 0; j < kHotPer; j++)
        if (b0 + j < b1) {
          if (pos[j] & 0x8000) {
            g++;
            base = ld(gval + (int64_t)ha.hx_rpos[g0 + g] * bs + c);
          }
          const T out = Op<OP, T>::apply(base, ld(gpre + (int64_t)(e0 + b0 + j) * bs + c));
          const int q = pos[j] & 0x1fff;
          if (leaf0 >= 0) st(lds_units + (int64_t)q * bs + c, out);
          else st(leaf_units + slot_of(q) * bs + c, out);
        }
    }
    return;
  } else {
    // is the entry after this thread's last one a group start (or the end)?
    const bool next_head = b1 >= nh || (ha.hx_pos[e0 + b1] & 0x8000);
    for (int c = 0; c < bs; c++) {
      T v[kHotPer];
      // phase 1: fold the thread's entries (the trailing group's part)
      int f = 0;
      T x{};
#pragma unroll
      for (int j = 0; j < kHotPer; j++)
        if (b0 + j < b1) {
          const bool head = pos[j] & 0x8000;
          v[j] = ld(lds_units + (int64_t)(pos[j] & 0x1fff) * bs + c);
          x = (head || j == 0) ? v[j] : Op<OP, T>::apply(x, v[j]);
          f |= head;
        }
      // carry-in: the scan over the threads before, inside and across wavefronts
      int fi = f;
      const T xi = wave_seg_scan_dpp<OP, T>(x, fi, lane);
      if (lane == 63) {
        wtot[wv] = xi;
        wfl[wv] = fi;
      }
      __syncthreads();
      T cw{};  // carry into the wavefront
      for (int w = 0; w < wv; w++) cw = (w == 0 || wfl[w]) ? wtot[w] : Op<OP, T>::apply(cw, wtot[w]);
      const T full = (fi || wv == 0) ? xi : Op<OP, T>::apply(cw, xi);
      T r = dpp_upd<0x138, 0xf>(cw, full);  // wave_shr:1: the previous thread's value (lane 0: cw)
      // phase 2: walk the entries again
      int g = gfirst - 1;
#pragma unroll
      for (int j = 0; j < kHotPer; j++)
        if (b0 + j < b1) {
          const bool head = pos[j] & 0x8000;
          if (head) g++;
          if constexpr (MODE == HOT_PREFIX) st(gpre + (int64_t)(e0 + b0 + j) * bs + c, head ? T{} : r);
          // (HOT_PREFIX reads the value again rather than keeping it across the scan: registers)
          const T vj = MODE == HOT_PREFIX ? ld(lds_units + (int64_t)(pos[j] & 0x1fff) * bs + c) : v[j];
          r = head ? vj : Op<OP, T>::apply(r, vj);
          const bool last = j + 1 < b1 - b0 ? (pos[j + 1] & 0x8000) != 0 : next_head;
          if (last) st(gval + (int64_t)ha.hx_rpos[g0 + g] * bs + c, r);
        }
      __syncthreads();
    }
  }
}

// Combine the groups of every hot root (stored root-major, in tile = leaf
// order inside a root): one wavefront per (hot root, unit element), 64 x
// kHotLoads groups per round with all their loads in flight.
//  HOT_TOTALS: root = root op (its groups combined, any order);
//  HOT_APPLY (SUM): the base of every group = root + the sum of the root's
//  earlier groups; root += the sum of all.
constexpr int kHotLoads = 16;
template <typename T, int OP, int MODE>
__global__ __launch_bounds__(256) void k_hot_combine(const int32_t *__restrict__ hx_root,
                                                     const int32_t *__restrict__ hx_rfirst, int H,
                                                     const T *__restrict__ gsum, T *__restrict__ gbase,
                                                     T *__restrict__ root, int bs) {
  const int64_t wid = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wid >= (int64_t)H * bs) return;
  const int h = (int)(wid / bs), c = (int)(wid % bs);
  const int64_t r = hx_root[h];
  T acc = ld(root + r * bs + c);
  const int i0 = hx_rfirst[h], i1 = hx_rfirst[h + 1];
  for (int a = i0; a < i1; a += 64 * kHotLoads) {
    T v[kHotLoads];
#pragma unroll
    for (int j = 0; j < kHotLoads; j++) {
      const int i = a + j * 64 + lane;
      v[j] = i < i1 ? ld(gsum + (int64_t)i * bs + c) : T{};
    }
    if constexpr (MODE == HOT_TOTALS) {
      // any combination order; lanes past the end take lane 0's first value
      // (idempotent ops) or zero (SUM)
      const T v00 = read_lane(v[0], 0);
      T x = v[0];
#pragma unroll
      for (int j = 1; j < kHotLoads; j++)
        if (a + j * 64 + lane < i1) x = Op<OP, T>::apply(x, v[j]);
      if (a + lane >= i1) x = OP == OP_SUM ? T{} : v00;
      acc = Op<OP, T>::apply(acc, wave_reduce_free<OP>(x));
    } else {
#pragma unroll
      for (int j = 0; j < kHotLoads; j++) {
        const int i = a + j * 64 + lane;
        T ex;
        const T inc = wave_scan_sum<T>(v[j], ex);
        if (i < i1) st(gbase + (int64_t)i * bs + c, Op<OP, T>::apply(acc, ex));
        acc = Op<OP, T>::apply(acc, read_lane(inc, 63));
      }
    }
  }
  if (lane == 0) st(root + r * bs + c, acc);
}

}  // namespace sfi
