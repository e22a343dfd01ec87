// sf_partition.hip -- the partitioned path of SFReduce and SFFetchAndOp for
// large star forests, in both reduce modes.
//
// The root-sorted order that the deterministic reduction needs visits the
// leaves at random; on a large leaf array every leaf read is then a request
// of its own.  Here the leaves are moved instead, in two passes that are
// coalesced on both sides:
//   pass A  takes a tile of consecutive processed leaves (contiguous leaf
//           units when the SF's slots are), stages it in LDS, and writes it
//           to a window-major scratch copy in increasing slot order: one
//           contiguous run per window;
//   pass B  loads one window -- whole small roots and aligned kChunk-leaf
//           chunks of large roots -- from its contiguous scratch range into
//           LDS, putting every leaf at its root-sorted place, and evaluates
//           the canonical pairwise trees from there.
// Deterministic floating-point sums take the same trees as the direct
// kernels, so results are bit-identical to them (and to the oracle); ops
// whose result does not depend on the order (MAX, MIN, MAXLOC, integer
// sums), and every op in atomic mode, combine in whatever order is fastest.
// FetchAndOp writes the fetched values back into the window (pass B) and
// moves them to leafupdate with the reverse of pass A (pass C).
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "sf_det_kernels.h"
#include "sf_hot.h"

namespace sfi {

// ------------------------------------------------------------ pass A / C
// A tile's positions are in increasing scratch-slot order, in runs of
// consecutive slots.  Position jj of a tile lies in run r = (run starts at
// or before jj) - 1 and goes to slot pa_run[r] + jj.  Thread t takes the
// positions t + k * kStageThreads (k < P): it loads all their offsets
// first; each wavefront counts the run starts of its 64 positions with a
// ballot; one wavefront turns the group counts into exclusive prefixes; the
// moves follow.  The tile's run offsets are staged in LDS after the tile's
// units (byte offset run_off) when the tile has at most run_cap runs.
constexpr int kMoveTile = 0x2000;          // most positions in a tile (13-bit offsets in pa_loc)
constexpr int kMoveGroups = kMoveTile / 64;  // most groups of 64 positions in a tile
// dynamic LDS of a pass-A/C block when two / one of them share a CU (a CU
// has 160 KB; the static group counts take the rest)
constexpr size_t kMoveLdsTwo = 80 * 1024 - kMoveGroups * 4;
constexpr size_t kMoveLdsOne = 160 * 1024 - kMoveGroups * 4;

// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD
// b % 8), each XCD with its own L2.  Neighbouring tiles write and read the
// two halves of the same cache lines of a window (their runs are adjacent),
// so every XCD takes a contiguous share of the tiles: workgroup b gets tile
// b / 8 of XCD b % 8's share.  A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n % X;
  const int x = b % X, i = b / X;
  return x * q + min(x, r) + i;
}

// Pass C of the deterministic FetchAndOp adds, to every element of a slot
// in a run of a root that spans windows (0x2000 in the slot's pa_loc), that
// run's base: rbase[(2 * window + which) * W + element], which = bit 14 of
// pa_loc, window = the window of the slot's pass-C run (staged in LDS beside
// the run offsets).  FIX is the element size (4 or 8 bytes, integer units;
// one Word per element) or 0 for a plain move.
template <int FIX, typename Word>
__device__ __forceinline__ Word add_word(Word v, Word b) {
  if constexpr (FIX == 4) {
    return (Word)((uint32_t)v + (uint32_t)b);
  } else {
    const uint64_t r = (((uint64_t)v.y << 32) | v.x) + (((uint64_t)b.y << 32) | b.x);
    Word o;
    o.x = (uint32_t)r;
    o.y = (uint32_t)(r >> 32);
    return o;
  }
}
template <int FIX, typename Word>
__device__ __forceinline__ Word add_base(Word v, const void *rbase, int64_t e) {
  return add_word<FIX>(v, reinterpret_cast<const Word *>(rbase)[e]);
}

struct MoveFix {
  const int32_t *pa_runw;
  const void *rbase;
};

// The 12 bytes of a (value, index) pair that a reduction reads: the
// window-major scratch of the pair ops holds these instead of whole 16-byte
// units, a quarter less written by pass A and read by pass B.
struct alignas(4) P12 {
  uint32_t x, y, z;
};
__device__ __forceinline__ P12 pair12(uint4 u) { return P12{u.x, u.y, u.z}; }
__device__ __forceinline__ Pair unpair12(P12 v) {
  Pair r;
  r.v = __longlong_as_double((long long)(((uint64_t)v.y << 32) | v.x));
  r.i = (int32_t)v.z;
  r.pad = 0;
  return r;
}

#define SP_MOVE_ARGS                                                                                      \
  const uint16_t *__restrict__ pa_loc, const int32_t *__restrict__ pa_run0, const int32_t *__restrict__ pa_run, \
      const int32_t *__restrict__ tile_leaf0, const int32_t *__restrict__ pa_slot, int64_t L, int ta,           \
      Word *__restrict__ leaf, Word *__restrict__ scratch, int W, int run_off, int run_cap, MoveFix fx,      \
      HotArgs ha, int bs
// HS: the hot-root phase (HotNone: none).  With one, the leaves of hot
// roots (0x4000 alone in pa_loc) are not moved: pass A combines them per
// group (HOT_TOTALS, HOT_PREFIX), pass C writes their fetched values
// (HOT_APPLY).
// PAIR12 (pass A of the pair ops, Word uint4): scratch holds 12-byte P12
// units (one per Word).
template <typename Word, int DIR, int P, int FIX, typename HS, bool PAIR12>
__device__ __forceinline__ void sp_move_body(SP_MOVE_ARGS) {
  static_assert(!PAIR12 || (DIR == 0 && FIX == 0 && std::is_same<Word, uint4>::value), "pair scratch: pass A");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t grp[kMoveGroups];
  Word *lds = reinterpret_cast<Word *>(smem);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t p0 = (int64_t)tile * ta;
  const int n = (int)min((int64_t)ta, L - p0);
  const uint16_t *loc = pa_loc + p0;
  const int32_t *run = pa_run + pa_run0[tile];
  const int nrun = pa_run0[tile + 1] - pa_run0[tile];
  const int32_t leaf0 = tile_leaf0[tile];
  const int64_t l0 = (int64_t)leaf0 * W;
  const int items = n * W;
  int lv[P];
#pragma unroll
  for (int k = 0; k < P; k++) {
    const int jj = k * kStageThreads + threadIdx.x;
    lv[k] = jj < n ? (int)loc[jj] : 0;
  }
  int32_t *rl = reinterpret_cast<int32_t *>(smem + run_off);
  int32_t *rw = rl + run_cap;  // FIX: the runs' windows
  const bool use_rl = nrun <= run_cap;
  if (use_rl) {
    for (int i = threadIdx.x; i < nrun; i += kStageThreads) rl[i] = run[i];
    if constexpr (FIX != 0)
      for (int i = threadIdx.x; i < nrun; i += kStageThreads) rw[i] = fx.pa_runw[pa_run0[tile] + i];
  }
  if (DIR == 0 && leaf0 >= 0) {  // leaf units are read once: streaming loads
#pragma unroll 8
    for (int q = threadIdx.x; q < items; q += kStageThreads) lds[q] = ld_stream(leaf + l0 + q);
  }
  // run starts per group of 64 positions (group of position jj: jj >> 6)
#pragma unroll
  for (int k = 0; k < P; k++) {
    const uint64_t b = __ballot(lv[k] & 0x8000);
    if (lane == 0) grp[k * (kStageThreads / 64) + wv] = __popcll(b);
  }
  __syncthreads();
  const int ngrp = P * (kStageThreads / 64);
  if (threadIdx.x < 64) {
    constexpr int E = kMoveGroups / 64;
    int v[E];
    int sum = 0;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int g = lane * E + e;
      v[e] = g < ngrp ? grp[g] : 0;
      sum += v[e];
    }
    int inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
      const int o = __shfl_up(inc, d);
      if (lane >= d) inc += o;
    }
    int acc = inc - sum;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int g = lane * E + e;
      if (g < ngrp) grp[g] = acc;
      acc += v[e];
    }
  }
  __syncthreads();
  // slots: the run index is kept inside the tile's runs and the slot inside
  // [0, L), so that a plan that broke its invariants could not make the move
  // leave its buffers
  int32_t sl[P];
  int32_t rr[FIX ? P : 1];
#pragma unroll
  for (int k = 0; k < P; k++) {
    const int jj = k * kStageThreads + threadIdx.x;
    const uint64_t b = __ballot(lv[k] & 0x8000);
    const int r = min(max(grp[jj >> 6] + __popcll(b & ((2ull << lane) - 1)) - 1, 0), nrun - 1);
    sl[k] = jj < n ? (use_rl ? rl[r] : run[r]) + jj : -1;
    if constexpr (FIX != 0) rr[k] = r;
  }
  // FIX: the first rbase element of each slot's run (-1: none), and for
  // one-word units the base itself, loaded together ahead of the moves
  int32_t fes[FIX ? P : 1];  // < 2 * windows * W
  Word fb[FIX ? P : 1];
  if constexpr (FIX != 0) {
#pragma unroll
    for (int k = 0; k < P; k++) {
      fes[k] = -1;
      if (sl[k] >= 0 && (lv[k] & 0x2000)) {
        const int w = use_rl ? rw[rr[k]] : fx.pa_runw[pa_run0[tile] + rr[k]];
        fes[k] = (2 * w + ((lv[k] >> 14) & 1)) * W;
      }
    }
    if (W == 1) {
#pragma unroll
      for (int k = 0; k < P; k++)
        if (fes[k] >= 0) fb[k] = reinterpret_cast<const Word *>(fx.rbase)[fes[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < P; k++) {
    const int64_t slot = sl[k];
    if (slot < 0 || slot >= L) continue;
    if constexpr (HS::mode != HOT_NONE)
      if ((lv[k] & 0x6000) == 0x4000) continue;  // a hot root's leaf: the hot phase takes it
    const int64_t s = slot * W;
    const int src = (lv[k] & 0x1fff);
    int64_t fe = -1;  // FIX: first rbase element of the slot's run, if it has one
    if constexpr (FIX != 0) fe = fes[k];
    if constexpr (FIX != 0) {
      if (W == 1 && leaf0 >= 0) {  // one-word units: the base is already loaded
        Word v = scratch[s];
        if (fe >= 0) v = add_word<FIX>(v, fb[k]);
        lds[src] = v;
        continue;
      }
    }
    if (leaf0 >= 0) {
      for (int c = 0; c < W; c++) {
        if (DIR == 0) {
          if constexpr (PAIR12)
            reinterpret_cast<P12 *>(scratch)[s + c] = pair12(lds[src * W + c]);
          else
            scratch[s + c] = lds[src * W + c];
        } else {
          Word v = scratch[s + c];
          if constexpr (FIX != 0)
            if (fe >= 0) v = add_base<FIX>(v, fx.rbase, fe + c);
          lds[src * W + c] = v;
        }
      }
    } else {  // slots not contiguous: the leaf side is gathered / scattered
      const int64_t l = (int64_t)pa_slot[p0 + src] * W;
      for (int c = 0; c < W; c++) {
        if (DIR == 0) {
          if constexpr (PAIR12)
            reinterpret_cast<P12 *>(scratch)[s + c] = pair12(leaf[l + c]);
          else
            scratch[s + c] = leaf[l + c];
        } else {
          Word v = scratch[s + c];
          if constexpr (FIX != 0)
            if (fe >= 0) v = add_base<FIX>(v, fx.rbase, fe + c);
          leaf[l + c] = v;
        }
      }
    }
  }
  if constexpr (HS::mode != HOT_NONE) {
    using HT = typename HS::type;
    static_assert(DIR == 0 ? HS::mode != HOT_APPLY : HS::mode == HOT_APPLY, "hot phase of the pass");
    // (pass A: the tile in LDS is complete since the barriers before the
    // moves, which only read it; pass C writes positions no move writes)
    hot_phase<HS>(ha, tile, p0, bs, leaf0, pa_slot, reinterpret_cast<HT *>(smem), reinterpret_cast<HT *>(leaf));
  }
  if (DIR == 1 && leaf0 >= 0) {  // leaf units are written once: streaming stores
    __syncthreads();
#pragma unroll 8
    for (int q = threadIdx.x; q < items; q += kStageThreads) st_stream(leaf + l0 + q, lds[q]);
  }
}

// Tiles of units up to 8 bytes take 64 KB of LDS; two blocks share a CU
// when the kernel also stays within 64 VGPRs (8 waves per SIMD).
template <typename Word, int DIR, int P, int FIX, typename HS, bool PAIR12 = false>
__global__ __launch_bounds__(kStageThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_sp_move2(SP_MOVE_ARGS) {
  sp_move_body<Word, DIR, P, FIX, HS, PAIR12>(pa_loc, pa_run0, pa_run, tile_leaf0, pa_slot, L, ta, leaf, scratch, W,
                                              run_off, run_cap, fx, ha, bs);
}
template <typename Word, int DIR, int P, int FIX, typename HS, bool PAIR12 = false>
__global__ __launch_bounds__(kStageThreads) void k_sp_move(SP_MOVE_ARGS) {
  sp_move_body<Word, DIR, P, FIX, HS, PAIR12>(pa_loc, pa_run0, pa_run, tile_leaf0, pa_slot, L, ta, leaf, scratch, W,
                                              run_off, run_cap, fx, ha, bs);
}
#undef SP_MOVE_ARGS

// Load one window from scratch into LDS in root-sorted order (LDS offset =
// sorted position - window start, the low 14 bits of lpos), and store it
// back.  Global accesses are
// coalesced; the permutation happens in LDS.
template <typename T>
__device__ __forceinline__ void win_load(T *lds, const T *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                         const DevSWin &w, int bs) {
  const T *src = scr + (int64_t)w.base * bs;  // read once: streaming loads
  if (bs == 1) {
#pragma unroll 8
    for (int q = threadIdx.x; q < w.n; q += kStageThreads) lds[lpos[w.base + q] & 0x3fff] = ld_stream(src + q);
  } else {
    const int items = w.n * bs;
#pragma unroll 4
    for (int q = threadIdx.x; q < items; q += kStageThreads) {
      const int k = q / bs;
      lds[(int)(lpos[w.base + k] & 0x3fff) * bs + (q - k * bs)] = ld_stream(src + q);
    }
  }
}
template <typename T>
__device__ __forceinline__ void win_store(const T *lds, T *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                          const DevSWin &w, int bs) {
  T *dst = scr + (int64_t)w.base * bs;
  if (bs == 1) {
#pragma unroll 8
    for (int q = threadIdx.x; q < w.n; q += kStageThreads) dst[q] = lds[lpos[w.base + q] & 0x3fff];
    return;
  }
  const int items = w.n * bs;
#pragma unroll 4
  for (int q = threadIdx.x; q < items; q += kStageThreads) {
    const int k = q / bs;
    dst[q] = lds[(int)(lpos[w.base + k] & 0x3fff) * bs + (q - k * bs)];
  }
}

// Pairwise tree over the n <= D consecutive (sorted) values at LDS offset o.
template <typename T, int OP, int D>
__device__ __forceinline__ T lds_tree(const T *lds, int o, int n, int bs, int c) {
  T x[D];
#pragma unroll
  for (int p = 0; p < D; p++)
    if (p < n) x[p] = ld(lds + (o + p) * bs + c);
#pragma unroll
  for (int d = 1; d < D; d *= 2)
#pragma unroll
    for (int p = 0; p + d < D; p += 2 * d)
      if (p + d < n) x[p] = Op<OP, T>::apply(x[p], x[p + d]);
  return x[0];
}

// Window-relative offset and degree of a whole root; offset, length and
// first / last-of-root flags of a chunk.
__device__ __forceinline__ int sr_off(int32_t on) { return on & 0xffff; }
__device__ __forceinline__ int sr_n(int32_t on) { return on >> 16; }
__device__ __forceinline__ int wc_off(int32_t onf) { return onf & 0xffff; }
__device__ __forceinline__ int wc_n(int32_t onf) { return ((onf >> 16) & 0xff) + 1; }
__device__ __forceinline__ bool wc_first(int32_t onf) { return (onf >> 24) & 1; }
__device__ __forceinline__ bool wc_last(int32_t onf) { return (onf >> 25) & 1; }

// Pass-B blocks are bound by chains of dependent global loads rather than
// by bandwidth, so every block first issues the loads that do not depend on
// the window (its first whole roots' descriptors and root values, its chunk
// descriptors), then loads the window; the LDS after the window's values
// holds the chunk descriptors (byte offset cd_off) and per-chunk values
// (byte offset cv_off).
constexpr int kSmallU = 2;  // whole-root elements per thread in flight

// Canonical pairwise tree of n <= kSmallMaxDeg sorted values.  Its lowest
// three levels stay inside aligned blocks of 8 (a short last block keeps its
// own tree), so it is evaluated as the trees of those blocks followed by the
// tree of the (at most 4) block values -- a third of the registers of one
// 32-wide tree.
template <typename T, int OP>
__device__ __forceinline__ T small_tree(const T *lds, int o, int n, int bs, int c) {
  static_assert(kSmallMaxDeg <= 32, "two levels above blocks of 8");
  if (n <= 1) return ld(lds + o * bs + c);
  if (n <= 2) return lds_tree<T, OP, 2>(lds, o, n, bs, c);
  if (n <= 4) return lds_tree<T, OP, 4>(lds, o, n, bs, c);
  if (n <= 8) return lds_tree<T, OP, 8>(lds, o, n, bs, c);
  const int nblk = (n + 7) >> 3;
  T b[4];
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (k < nblk) b[k] = lds_tree<T, OP, 8>(lds, o + 8 * k, min(8, n - 8 * k), bs, c);
  if (nblk > 3) b[2] = Op<OP, T>::apply(b[2], b[3]);
  b[0] = Op<OP, T>::apply(b[0], b[1]);
  if (nblk > 2) b[0] = Op<OP, T>::apply(b[0], b[2]);
  return b[0];
}

// The kSmallU whole-root elements q0 + u * kStageThreads of a window: their
// descriptors and root values.
template <typename T>
__device__ __forceinline__ void small_fetch(const DevSRoot *__restrict__ sroot, const T *__restrict__ root,
                                            const DevSWin &win, int q0, int nsmall, int bs, DevSRoot (&sd)[kSmallU],
                                            T (&rv)[kSmallU]) {
#pragma unroll
  for (int u = 0; u < kSmallU; u++) {
    const int q = q0 + u * kStageThreads;
    if (q < nsmall) sd[u] = sroot[win.small0 + q / bs];
  }
#pragma unroll
  for (int u = 0; u < kSmallU; u++) {
    const int q = q0 + u * kStageThreads;
    if (q < nsmall) rv[u] = ld(root + (int64_t)sd[u].root * bs + (q % bs));
  }
}

// ------------------------------------------------------------- pass B reduce
// Whole roots: one thread per (root, element) evaluates its tree from LDS.
// Chunks of large roots: one wavefront per chunk computes the chunk's tree
// into LDS; then one thread per chunk writes it on -- to its root when the
// chunk is the root's only one, else to the next chunk level (lvl_out).
// ATOM: the chunks of a root that lie in this window are combined in chunk
// order; a root whose chunks all lie in this window is then updated plainly,
// one that spans windows through one native atomic per window, in arrival
// order, in place of the chunk-level trees.
// Floating-point MAX / MIN hold the window in LDS as fkey keys, so that the
// trees compare unsigned integers once per pair instead of re-deriving the
// order of both operands (the keys order the values totally, -0 < +0).
template <typename T, int OP>
struct LdsKey {
  static constexpr bool on = false;
  using V = T;
};
template <int OP>
struct LdsKey<double, OP> {
  static constexpr bool on = OP == OP_MAX || OP == OP_MIN;
  using V = typename std::conditional<on, uint64_t, double>::type;
};
template <int OP>
struct LdsKey<float, OP> {
  static constexpr bool on = OP == OP_MAX || OP == OP_MIN;
  using V = typename std::conditional<on, uint32_t, float>::type;
};
template <typename K, typename V>
__device__ __forceinline__ auto lds_value(V v) {
  if constexpr (K::on)
    return fkey_inv(v);
  else
    return v;
}
// A window of pairs from their 12-byte scratch units.
__device__ __forceinline__ void win_load_pair12(Pair *lds, const P12 *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                                const DevSWin &w, int bs) {
  const P12 *src = scr + (int64_t)w.base * bs;
  const int items = w.n * bs;
#pragma unroll 4
  for (int q = threadIdx.x; q < items; q += kStageThreads) {
    const int k = bs == 1 ? q : q / bs;
    lds[(int)(lpos[w.base + k] & 0x3fff) * bs + (q - k * bs)] = unpair12(src[q]);
  }
}
template <typename T, typename V>
__device__ __forceinline__ void win_load_key(V *lds, const T *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                             const DevSWin &w, int bs) {
  const T *src = scr + (int64_t)w.base * bs;
  if (bs == 1) {
#pragma unroll 8
    for (int q = threadIdx.x; q < w.n; q += kStageThreads) lds[lpos[w.base + q] & 0x3fff] = fkey(src[q]);
  } else {
    const int items = w.n * bs;
#pragma unroll 4
    for (int q = threadIdx.x; q < items; q += kStageThreads) {
      const int k = q / bs;
      lds[(int)(lpos[w.base + k] & 0x3fff) * bs + (q - k * bs)] = fkey(src[q]);
    }
  }
}

// Ops whose result does not depend on the order in which the elements are
// combined: a maximum or minimum under a total order (MAXLOC breaks ties by
// the smaller index, so it is one too) and wrapping integer addition.  Their
// chunk reductions (and those of every op in atomic mode, which fixes no
// order) read the elements interleaved across the lanes (no LDS bank
// conflicts) and combine lanes with DPP row moves instead of LDS permutes;
// deterministic floating-point sums keep the canonical pairwise tree.
template <typename V, int OP>
struct OrderFree {
  static constexpr bool value = OP == OP_MAX || OP == OP_MIN || OP == OP_MAXLOC || OP == OP_MINLOC ||
                                ((OP == OP_SUM || OP == OP_PROD) && std::is_integral<V>::value);
  static constexpr bool idempotent = OP != OP_SUM && OP != OP_PROD;
};
// What fills the positions past the end of a run of elements whose first
// element is e0: e0 itself for an idempotent op, else the op's neutral
// element (0 for the sum, 1 for the product).
template <typename V, int OP>
__device__ __forceinline__ V free_pad(V e0) {
  if constexpr (OrderFree<V, OP>::idempotent)
    return e0;
  else if constexpr (OP == OP_PROD)
    return V(1);
  else
    return V{};
}

// Lane steps of the canonical chunk tree (lane l holds the tree of its LPT
// leaves; lanes combine at distances 1, 2, ..., 32 while the partner's block
// starts below n), with the same operands in the same order as a shuffle
// tree: DPP moves inside 16-lane rows (quad swaps, row shifts by 4 and 8),
// then the four row results read from lanes 0, 16, 32, 48.
template <int OP, typename V>
__device__ __forceinline__ V wave_tree(V v, int lane, int n) {
  constexpr int LPT = kChunkLPT;
  V o = dpp_upd<0xB1, 0xf>(v, v);  // quad_perm [1,0,3,2]
  if ((lane & 1) == 0 && (lane + 1) * LPT < n) v = Op<OP, V>::apply(v, o);
  o = dpp_upd<0x4E, 0xf>(v, v);  // quad_perm [2,3,0,1]
  if ((lane & 3) == 0 && (lane + 2) * LPT < n) v = Op<OP, V>::apply(v, o);
  o = dpp_upd<0x104, 0xf>(v, v);  // row_shl:4
  if ((lane & 7) == 0 && (lane + 4) * LPT < n) v = Op<OP, V>::apply(v, o);
  o = dpp_upd<0x108, 0xf>(v, v);  // row_shl:8
  if ((lane & 15) == 0 && (lane + 8) * LPT < n) v = Op<OP, V>::apply(v, o);
  const V r0 = read_lane(v, 0), r16 = read_lane(v, 16), r32 = read_lane(v, 32), r48 = read_lane(v, 48);
  const V a = 16 * LPT < n ? Op<OP, V>::apply(r0, r16) : r0;
  const V b = 48 * LPT < n ? Op<OP, V>::apply(r32, r48) : r32;
  return 32 * LPT < n ? Op<OP, V>::apply(a, b) : a;
}

// A whole root of an order-free op (or of any op in atomic mode): its n
// elements four at a time (loads in flight, one accumulator); positions past
// n take free_pad.
template <typename V, int OP>
__device__ __forceinline__ V small_free(const V *lds, int o, int n, int bs, int c) {
  const V e0 = ld(lds + o * bs + c);
  const V pad = free_pad<V, OP>(e0);
  V a = e0;
  for (int e = 1; e < n; e += 4) {
    V x[4];
#pragma unroll
    for (int k = 0; k < 4; k++) x[k] = e + k < n ? ld(lds + (o + e + k) * bs + c) : pad;
    a = Op<OP, V>::apply(a, Op<OP, V>::apply(Op<OP, V>::apply(x[0], x[1]), Op<OP, V>::apply(x[2], x[3])));
  }
  return a;
}

template <typename T, int OP, bool ATOM>
__device__ __forceinline__ void sp_reduce_body(const DevSWin *__restrict__ wins, const DevSRoot *__restrict__ sroot,
                                               const DevWChunk *__restrict__ wchunk,
                                               const uint16_t *__restrict__ lpos, const T *__restrict__ scr,
                                               T *__restrict__ lvl_out, T *__restrict__ root, int bs, int cd_off,
                                               int cv_off) {
  using K = LdsKey<T, OP>;
  using V = typename K::V;  // what the LDS holds: the values, or their keys
  // order-free evaluation: order-free ops, and any op in atomic mode (which
  // fixes no order)
  constexpr bool kFree = OrderFree<V, OP>::value || ATOM;
  extern __shared__ __align__(16) unsigned char smem[];
  V *lds = reinterpret_cast<V *>(smem);
  DevWChunk *cd = reinterpret_cast<DevWChunk *>(smem + cd_off);
  T *cv = reinterpret_cast<T *>(smem + cv_off);
  const DevSWin win = wins[blockIdx.x];
  const int nsmall = (win.small1 - win.small0) * bs;
  const int nb = win.big1 - win.big0;
  DevSRoot sd[kSmallU];
  T rv[kSmallU];
  small_fetch(sroot, root, win, threadIdx.x, nsmall, bs, sd, rv);
  for (int j = threadIdx.x; j < nb; j += kStageThreads) cd[j] = wchunk[win.big0 + j];
  if constexpr (K::on)
    win_load_key(lds, scr, lpos, win, bs);
  else if constexpr (std::is_same<T, Pair>::value)
    win_load_pair12(lds, reinterpret_cast<const P12 *>(scr), lpos, win, bs);
  else
    win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  for (int q0 = threadIdx.x;;) {
#pragma unroll
    for (int u = 0; u < kSmallU; u++) {
      const int q = q0 + u * kStageThreads;
      if (q >= nsmall) continue;
      const int c = q % bs;
      const V v = kFree ? small_free<V, OP>(lds, sr_off(sd[u].on), sr_n(sd[u].on), bs, c)
                        : small_tree<V, OP>(lds, sr_off(sd[u].on), sr_n(sd[u].on), bs, c);
      st(root + (int64_t)sd[u].root * bs + c, Op<OP, T>::apply(rv[u], lds_value<K>(v)));
      __builtin_amdgcn_sched_barrier(0);  // one tree's registers at a time
    }
    q0 += kSmallU * kStageThreads;
    if (q0 >= nsmall) break;
    small_fetch(sroot, root, win, q0, nsmall, bs, sd, rv);
  }
  if (nb == 0) return;
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < nb; j += kStageThreads / 64) {
    const int32_t onf = cd[j].onf;
    const int n = wc_n(onf);
    if constexpr (kFree) {
      const int o0 = wc_off(onf);
      for (int c = 0; c < bs; c++) {
        // lanes past the chunk's end take free_pad of its first element
        V a = lane < n ? ld(lds + (o0 + lane) * bs + c) : free_pad<V, OP>(ld(lds + o0 * bs + c));
#pragma unroll
        for (int s = 1; s < LPT; s++)
          if (s * 64 + lane < n) a = Op<OP, V>::apply(a, ld(lds + (o0 + s * 64 + lane) * bs + c));
        const V v = wave_reduce_free<OP>(a);
        if (lane == 0) st(cv + j * bs + c, (T)lds_value<K>(v));
      }
      continue;
    }
    const int o = wc_off(onf) + lane * LPT;
    const int m = n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      V x[LPT];
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (s < m) x[s] = ld(lds + (o + s) * bs + c);
#pragma unroll
      for (int d = 1; d < LPT; d *= 2)
#pragma unroll
        for (int p = 0; p + d < LPT; p += 2 * d)
          if (p + d < m) x[p] = Op<OP, V>::apply(x[p], x[p + d]);
      const V v = wave_tree<OP>(x[0], lane, n);
      if (lane == 0) st(cv + j * bs + c, (T)lds_value<K>(v));
    }
  }
  __syncthreads();
  if constexpr (ATOM) {
    // per run (the chunks of one root in this window): the combination of
    // its chunk results by a segmented scan, one wavefront per unit
    // component, 64 chunks at a time; the run's last lane updates the root,
    // plainly when the window holds the whole root, else atomically
    for (int c = wv; c < bs; c += kStageThreads / 64) {
      T carry{};   // running result of a run continuing from the previous group
      int jh = 0;  // head chunk of that run
      for (int g = 0; g < nb; g += 64) {
        const int j = g + lane;
        const bool in = j < nb;
        const int32_t r = in ? cd[j].root : -1;
        const bool head = in && (j == 0 || cd[j - 1].root != r);
        const bool tail = in && (j == nb - 1 || cd[j + 1].root != r);
        T v = in ? ld(cv + j * bs + c) : T{};
        const uint64_t hm = __ballot(head);
        const uint64_t hle = hm & (lane == 63 ? ~0ull : (2ull << lane) - 1);
        const int s0 = hle ? 63 - __clzll(hle) : -1;  // this lane's run head lane, -1: earlier group
#pragma unroll
        for (int d = 1; d < 64; d *= 2) {
          const T y = shfl_up(v, d);
          if (lane - d >= (s0 < 0 ? 0 : s0)) v = Op<OP, T>::apply(y, v);
        }
        if (s0 < 0) v = Op<OP, T>::apply(carry, v);
        if (tail) {
          const int j0 = s0 < 0 ? jh : g + s0;
          T *rp = root + (int64_t)r * bs + c;
          if (wc_first(cd[j0].onf) && wc_last(cd[j].onf))
            st(rp, Op<OP, T>::apply(ld(rp), v));
          else
            AtomicG<OP, T>::run(rp, v);
        }
        carry = shfl_idx(v, 63);
        const int s63 = __shfl(s0, 63);
        jh = s63 < 0 ? jh : g + s63;
      }
    }
  } else {
    for (int q = threadIdx.x; q < nb * bs; q += kStageThreads) {
      const int j = q / bs, c = q - j * bs;
      const int32_t dst = cd[j].dst;
      if (dst < 0) {
        T *rp = root + (int64_t)(-dst - 1) * bs + c;
        st(rp, Op<OP, T>::apply(ld(rp), ld(cv + q)));
      } else {
        st(lvl_out + (int64_t)dst * bs + c, ld(cv + q));
      }
    }
  }
}

// A window of up to 80 KB of LDS (with its chunk tables) lets two blocks
// share a CU when the kernel stays within 64 VGPRs (8 waves per SIMD); a
// larger one (a capacity raised for tuning) runs one block per CU.
constexpr size_t kPassBLdsTwo = 80 * 1024;
#define SP_REDUCE_ARGS                                                                                             \
  const DevSWin *__restrict__ wins, const DevSRoot *__restrict__ sroot, const DevWChunk *__restrict__ wchunk,     \
      const uint16_t *__restrict__ lpos, const T *__restrict__ scr, T *__restrict__ lvl_out, T *__restrict__ root, \
      int bs, int cd_off, int cv_off
template <typename T, int OP, bool ATOM>
__global__ __launch_bounds__(kStageThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_sp_reduce2(SP_REDUCE_ARGS) {
  sp_reduce_body<T, OP, ATOM>(wins, sroot, wchunk, lpos, scr, lvl_out, root, bs, cd_off, cv_off);
}
template <typename T, int OP, bool ATOM>
__global__ __launch_bounds__(kStageThreads) void k_sp_reduce(SP_REDUCE_ARGS) {
  sp_reduce_body<T, OP, ATOM>(wins, sroot, wchunk, lpos, scr, lvl_out, root, bs, cd_off, cv_off);
}
#undef SP_REDUCE_ARGS

// ------------------------------------------------------- pass B FetchAndOp
// Whole roots (all kernels below): one thread per (root, element) scans the
// root's leaves sequentially in leaf order; the fetched values replace the
// leaf values in the window.
template <typename T>
__device__ __forceinline__ void small_scan(T *lds, const DevSRoot *__restrict__ sroot, T *__restrict__ root,
                                           const DevSWin &win, int nsmall, int bs, DevSRoot (&sd)[kSmallU],
                                           T (&rv)[kSmallU]) {
  for (int q0 = threadIdx.x;;) {
#pragma unroll
    for (int u = 0; u < kSmallU; u++) {
      const int q = q0 + u * kStageThreads;
      if (q >= nsmall) continue;
      const int c = q % bs;
      const int o0 = sr_off(sd[u].on), o1 = o0 + sr_n(sd[u].on);
      T a = rv[u];
      for (int o = o0; o < o1; o++) {
        T *e = lds + o * bs + c;
        const T v = *e;
        *e = a;
        a = Op<OP_SUM, T>::apply(a, v);
      }
      root[(int64_t)sd[u].root * bs + c] = a;
    }
    q0 += kSmallU * kStageThreads;
    if (q0 >= nsmall) break;
    small_fetch(sroot, (const T *)root, win, q0, nsmall, bs, sd, rv);
  }
}

// Exclusive prefix inside chunk j of the window plus the chunk's base
// (from LDS), written over the chunk's values.
template <typename T>
__device__ __forceinline__ void chunk_apply(T *lds, const DevWChunk *cd, const T *base, int nb, int bs) {
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < nb; j += kStageThreads / 64) {
    const int32_t onf = cd[j].onf;
    const int o = wc_off(onf) + lane * LPT;
    const int m = wc_n(onf) - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
      T lane_sum = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        x[s] = s < m ? lds[(o + s) * bs + c] : T(0);
        lane_sum = Op<OP_SUM, T>::apply(lane_sum, x[s]);
      }
      T excl;
      wave_scan_sum(lane_sum, excl);
      T a = Op<OP_SUM, T>::apply(base[j * bs + c], excl);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        if (s < m) lds[(o + s) * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[s]);
      }
    }
  }
}

// One pass over a window.  Whole roots scan sequentially in leaf order.  The
// chunks of a large root that lie in this window form a run: their totals
// give every chunk its offset inside the run, and the leaves inside a chunk
// take the chunk's offset plus their exclusive prefix.  A run that is the
// whole root takes its base from the root plainly.  A run of a root that
// spans windows takes, in atomic mode (ATOM), its base from one native
// returning atomic add, so the windows of such a root are applied in
// arrival order; in deterministic mode it takes base 0 and leaves its total
// in rtot[2 * window + which] (which 0: the run continues a root from the
// previous window, 1: it continues into the next), for the scan over the
// root's windows and the base that pass C adds.
template <typename T, bool ATOM>
__global__ __launch_bounds__(kStageThreads) void k_sp_fop(const DevSWin *__restrict__ wins,
                                                          const DevSRoot *__restrict__ sroot,
                                                          const DevWChunk *__restrict__ wchunk,
                                                          const uint16_t *__restrict__ lpos, T *__restrict__ scr,
                                                          T *__restrict__ root, T *__restrict__ rtot, int bs,
                                                          int cd_off, int cv_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  DevWChunk *cd = reinterpret_cast<DevWChunk *>(smem + cd_off);
  T *cv = reinterpret_cast<T *>(smem + cv_off);
  const DevSWin win = wins[blockIdx.x];
  const int nsmall = (win.small1 - win.small0) * bs;
  const int nb = win.big1 - win.big0;
  DevSRoot sd[kSmallU];
  T rv[kSmallU];
  small_fetch(sroot, (const T *)root, win, threadIdx.x, nsmall, bs, sd, rv);
  for (int j = threadIdx.x; j < nb; j += kStageThreads) cd[j] = wchunk[win.big0 + j];
  win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  if (nsmall > 0) small_scan(lds, sroot, root, win, nsmall, bs, sd, rv);
  if (nb > 0) {
    constexpr int LPT = kChunkLPT;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // 1: chunk totals
    for (int j = wv; j < nb; j += kStageThreads / 64) {
      const int32_t onf = cd[j].onf;
      const int n = wc_n(onf);
      if constexpr (ATOM || std::is_integral<T>::value) {
        // integer sums are exact in any order, and atomic mode fixes no
        // order: interleaved reads and a DPP reduction
        const int o0 = wc_off(onf);
        for (int c = 0; c < bs; c++) {
          T a = lane < n ? lds[(o0 + lane) * bs + c] : T(0);
#pragma unroll
          for (int s = 1; s < LPT; s++)
            if (s * 64 + lane < n) a = Op<OP_SUM, T>::apply(a, lds[(o0 + s * 64 + lane) * bs + c]);
          a = wave_reduce_free<OP_SUM>(a);
          if (lane == 0) cv[j * bs + c] = a;
        }
        continue;
      }
      const int o = wc_off(onf) + lane * LPT;
      for (int c = 0; c < bs; c++) {
        T a = T(0);
#pragma unroll
        for (int s = 0; s < LPT; s++)
          if (lane * LPT + s < n) a = Op<OP_SUM, T>::apply(a, lds[(o + s) * bs + c]);
#pragma unroll
        for (int d = 32; d >= 1; d /= 2) a = Op<OP_SUM, T>::apply(a, shfl_down(a, d));
        if (lane == 0) cv[j * bs + c] = a;
      }
    }
    __syncthreads();
    // 2: per run (the chunks of one root in this window), each chunk's
    // offset inside the run and the run's base: a segmented scan over the
    // chunk totals, one wavefront per unit component, 64 chunks at a time.
    // The last lane of a run takes its base (the root value when the window
    // holds the whole root, else a returning atomic add, or in deterministic
    // mode 0 with the run total left for the cross-window scan) and the base
    // is broadcast to the run's chunks; chunks of a run that began in an
    // earlier group get it once the run ends.
    for (int c = wv; c < bs; c += kStageThreads / 64) {
      T carry = T(0);  // running total of a run continuing from the previous group
      int jh = 0;      // head chunk of that run
      for (int g = 0; g < nb; g += 64) {
        const int j = g + lane;
        const bool in = j < nb;
        const int32_t r = in ? cd[j].root : -1;
        const bool head = in && (j == 0 || cd[j - 1].root != r);
        const bool tail = in && (j == nb - 1 || cd[j + 1].root != r);
        const T t = in ? cv[j * bs + c] : T(0);
        const uint64_t hm = __ballot(head), tm = __ballot(tail);
        const uint64_t le = lane == 63 ? ~0ull : (2ull << lane) - 1;
        const uint64_t hle = hm & le;
        const int s0 = hle ? 63 - __clzll(hle) : -1;  // this lane's run head lane, -1: earlier group
        T v = t;
#pragma unroll
        for (int d = 1; d < 64; d *= 2) {
          const T y = shfl_up(v, d);
          if (lane - d >= (s0 < 0 ? 0 : s0)) v = Op<OP_SUM, T>::apply(y, v);
        }
        if (s0 < 0) v = Op<OP_SUM, T>::apply(carry, v);
        const T vprev = shfl_up(v, 1);
        const T ex = head ? T(0) : lane > 0 ? vprev : carry;
        const int j0 = s0 < 0 ? jh : g + s0;
        T base = T(0);
        if (tail) {
          T *rp = root + (int64_t)r * bs + c;
          if (wc_first(cd[j0].onf) && wc_last(cd[j].onf)) {
            base = *rp;
            *rp = Op<OP_SUM, T>::apply(base, v);
          } else if constexpr (ATOM) {
            base = fetch_add_g(rp, v);
          } else {
            const int which = wc_off(cd[j0].onf) == 0 ? 0 : 1;
            rtot[(int64_t)(2 * blockIdx.x + which) * bs + c] = v;
          }
        }
        const uint64_t tge = tm & ~((1ull << lane) - 1);  // tails at or above this lane
        const int tl = tge ? __ffsll((unsigned long long)tge) - 1 : 64;
        const T b = shfl_idx(base, tl & 63);
        if (in) cv[j * bs + c] = tl < 64 ? Op<OP_SUM, T>::apply(b, ex) : ex;
        if (g > 0 && !(hm & 1) && tm) {  // a run from earlier groups ends here
          const T b0 = shfl_idx(base, __ffsll((unsigned long long)tm) - 1);
          for (int jj = jh + lane; jj < g; jj += 64) cv[jj * bs + c] = Op<OP_SUM, T>::apply(b0, cv[jj * bs + c]);
        }
        carry = shfl_idx(v, 63);
        const int s63 = __shfl(s0, 63);
        jh = s63 < 0 ? jh : g + s63;
      }
    }
    __syncthreads();
    // 3: exclusive prefix inside each chunk plus the chunk's base
    chunk_apply(lds, cd, cv, nb, bs);
  }
  __syncthreads();
  win_store(lds, scr, lpos, win, bs);
}

// Deterministic FetchAndOp across windows: one wavefront per root that
// spans windows turns its runs' totals (in window order, i.e. leaf order)
// into their bases, starting from the root's value, and leaves the root's
// final value.  Each step takes 64 * kScanPer runs, kScanPer consecutive
// ones per lane (all their loads in flight), so the longest root -- a few
// hundred runs -- takes one or two steps.  Integer units only (exact sums).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sp_span_scan(const int32_t *__restrict__ span_first,
                                                         const int32_t *__restrict__ span_slot,
                                                         const int32_t *__restrict__ span_root, int nspan,
                                                         const T *__restrict__ rtot, T *__restrict__ rbase,
                                                         T *__restrict__ root, int bs) {
  const int lane = threadIdx.x & 63;
  const int i = (int)((blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6);
  if (i >= nspan) return;
  const int a = span_first[i], b = span_first[i + 1];
  T *rp = root + (int64_t)span_root[i] * bs;
  for (int c = 0; c < bs; c++) {
    T carry = rp[c];
    for (int k0 = a; k0 < b; k0 += 64 * kScanPer) {
      int64_t e[kScanPer];
      T x[kScanPer];
      T s = T(0);
#pragma unroll
      for (int j = 0; j < kScanPer; j++) {
        const int k = k0 + lane * kScanPer + j;
        e[j] = k < b ? (int64_t)span_slot[k] * bs + c : -1;
      }
#pragma unroll
      for (int j = 0; j < kScanPer; j++) {
        x[j] = e[j] >= 0 ? rtot[e[j]] : T(0);
        s = Op<OP_SUM, T>::apply(s, x[j]);
      }
      T inc = s;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o);
      }
      T acc = Op<OP_SUM, T>::apply(carry, wrap_sub(inc, s));
#pragma unroll
      for (int j = 0; j < kScanPer; j++) {
        if (e[j] >= 0) rbase[e[j]] = acc;
        acc = Op<OP_SUM, T>::apply(acc, x[j]);
      }
      carry = Op<OP_SUM, T>::apply(carry, shfl_idx(inc, 63));
    }
    if (lane == 0) rp[c] = carry;
  }
}

// ================================================================ launchers
static int sp_check() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

// Allow a kernel more than the default 64 KB of dynamic LDS.  The largest
// size granted so far is remembered per kernel and device, so the attribute
// is set once rather than on every launch.
static int allow_lds(const void *fn, size_t bytes) {
  if (bytes <= 65536) return SF_OK;
  // a fixed table, so that no call allocates host memory either (a full
  // table only means the attribute is set again on each launch)
  struct Grant {
    const void *fn;
    int dev;
    size_t bytes;
  };
  static std::mutex mu;
  static Grant granted[256];
  static int ngranted = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_hip_error(e);
  std::lock_guard<std::mutex> g(mu);
  for (int k = 0; k < ngranted; k++)
    if (granted[k].fn == fn && granted[k].dev == dev && granted[k].bytes >= bytes) return SF_OK;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return set_hip_error(e);
  if (ngranted < 256) granted[ngranted++] = {fn, dev, bytes};
  return SF_OK;
}

int stage_class(int64_t unit_bytes) { return unit_bytes <= 8 ? 0 : (unit_bytes <= 16 ? 1 : -1); }

// Move whole units between the leaf buffer and scratch (pass A / pass C),
// with the hot-root phase HS when the plan has hot roots and the op takes
// them (ha, bs: its arguments).
template <typename Word, int DIR, int P, int FIX, typename HS, bool PAIR12>
static int sp_move_p(sf_s *sf, int cls, void *leaf, void *scratch, int W, hipStream_t st, MoveFix fx,
                     const HotArgs &ha, int bs) {
  const HostPlan::Stage &hs = sf->hp.sp[cls];
  const DevPlan::Stage &ds = sf->dp.sp[cls];
  const unsigned g = (unsigned)hs.tile_leaf0.size();
  const size_t tile = ((size_t)hs.ta * W * sizeof(Word) + 15) / 16 * 16;
  const size_t runs = (size_t)hs.maxrun * sizeof(int32_t) * (FIX ? 2 : 1);  // offsets (and windows)
  // static LDS of the hot phase: a value and a count per block of 64 entries
  const size_t hot_static =
      HS::mode == HOT_NONE ? 0 : (size_t)(kMoveTile / 64) * (sizeof(typename HS::type) + sizeof(int32_t));
  // The run tables go to LDS beside the tile when they fit: in half of a
  // CU's LDS (less the static group counts) two blocks share the CU (the
  // 64-VGPR build), else in all of it; otherwise they are read from memory.
  if (tile + runs + hot_static <= kMoveLdsTwo) {
    const size_t lds = tile + runs;
    int rc = allow_lds((const void *)&k_sp_move2<Word, DIR, P, FIX, HS, PAIR12>, lds);
    if (rc) return rc;
    hipLaunchKernelGGL((k_sp_move2<Word, DIR, P, FIX, HS, PAIR12>), dim3(g), dim3(kStageThreads), lds, st, ds.pa_loc,
                       ds.pa_run0, ds.pa_run, ds.tile_leaf0, ds.pa_slot, (int64_t)sf->nleaves, hs.ta, (Word *)leaf,
                       (Word *)scratch, W, (int)tile, hs.maxrun, fx, ha, bs);
    return SF_OK;
  }
  const int run_cap = tile + runs + hot_static <= kMoveLdsOne ? hs.maxrun : 0;
  const size_t lds = tile + (run_cap ? runs : 0);
  int rc = allow_lds((const void *)&k_sp_move<Word, DIR, P, FIX, HS, PAIR12>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_sp_move<Word, DIR, P, FIX, HS, PAIR12>), dim3(g), dim3(kStageThreads), lds, st, ds.pa_loc,
                     ds.pa_run0, ds.pa_run, ds.tile_leaf0, ds.pa_slot, (int64_t)sf->nleaves, hs.ta, (Word *)leaf,
                     (Word *)scratch, W, (int)tile, run_cap, fx, ha, bs);
  return SF_OK;
}
template <typename Word, int DIR, int FIX = 0, typename HS = HotNone, bool PAIR12 = false>
static int sp_move_w(sf_s *sf, int cls, void *leaf, void *scratch, int W, hipStream_t st, MoveFix fx = MoveFix{},
                     const HotArgs &ha = HotArgs{}, int bs = 1) {
  static_assert(kMoveTile == 8 * kStageThreads, "positions per thread");
  if (sf->hp.sp[cls].ta > kMoveTile) return SF_ERR_ARG;
  return sp_move_p<Word, DIR, kMoveTile / kStageThreads, FIX, HS, PAIR12>(sf, cls, leaf, scratch, W, st, fx, ha, bs);
}

static int sp_move(sf_s *sf, int cls, int dir, void *leaf, void *scratch, int64_t ub, hipStream_t st) {
  const uintptr_t a = (uintptr_t)leaf | (uintptr_t)scratch;
  if (ub % 16 == 0 && a % 16 == 0)
    return dir == 0 ? sp_move_w<uint4, 0>(sf, cls, leaf, scratch, (int)(ub / 16), st)
                    : sp_move_w<uint4, 1>(sf, cls, leaf, scratch, (int)(ub / 16), st);
  if (ub % 8 == 0 && a % 8 == 0)
    return dir == 0 ? sp_move_w<uint2, 0>(sf, cls, leaf, scratch, (int)(ub / 8), st)
                    : sp_move_w<uint2, 1>(sf, cls, leaf, scratch, (int)(ub / 8), st);
  return dir == 0 ? sp_move_w<uint32_t, 0>(sf, cls, leaf, scratch, (int)(ub / 4), st)
                  : sp_move_w<uint32_t, 1>(sf, cls, leaf, scratch, (int)(ub / 4), st);
}

// The word a hot-phase move kernel moves: one element of the unit type (the
// typed LDS view of the tile then lines up with it).
template <typename T>
using ElemWord = typename std::conditional<sizeof(T) == 4, uint32_t,
                                           typename std::conditional<sizeof(T) == 8, uint2, uint4>::type>::type;

// Pass A with a hot phase (HOT_TOTALS of op OP for Reduce, HOT_PREFIX for
// FetchAndOp): cold leaves to scratch, hot roots' group totals to gsum (and
// every hot leaf's exclusive prefix in its group to gpre).
template <typename T, int OP, int MODE>
static int sp_move_hot_a(sf_s *sf, int cls, const T *leaf, T *scratch, int bs, T *gsum, T *gpre, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HotArgs ha{d.hx_pos, d.hx_tg, d.hx_e0, d.hx_grp0, d.hx_rpos, gsum, gpre};
  return sp_move_w<ElemWord<T>, 0, 0, HotSpec<T, OP, MODE>>(sf, cls, (void *)leaf, scratch, bs, st, MoveFix{}, ha,
                                                            bs);
}

// Pass C of FetchAndOp with the hot phase: cold leaves' fetched values from
// scratch (plus the spanning runs' bases when FIX), hot leaves' from their
// group bases and prefixes.
template <typename T, int FIX>
static int sp_move_hot_c(sf_s *sf, int cls, T *upd, T *scratch, int bs, const T *gbase, const T *gpre, MoveFix fx,
                         hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HotArgs ha{d.hx_pos, d.hx_tg, d.hx_e0, d.hx_grp0, d.hx_rpos, (void *)gbase, (void *)gpre};
  return sp_move_w<ElemWord<T>, 1, FIX, HotSpec<T, OP_SUM, HOT_APPLY>>(sf, cls, (void *)upd, scratch, bs, st, fx, ha,
                                                                      bs);
}

// Combine the hot roots' groups (one wavefront per hot root and element).
template <typename T, int OP, int MODE>
static void hot_combine(sf_s *sf, const T *gsum, T *gbase, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const int H = (int)sf->hp.hx_root.size();
  const int64_t waves = (int64_t)H * bs;
  hipLaunchKernelGGL((k_hot_combine<T, OP, MODE>), dim3((unsigned)((waves * 64 + 255) / 256)), dim3(256), 0, st,
                     d.hx_root, d.hx_rfirst, H, gsum, gbase, root, bs);
}

// LDS of a pass-B block: the window's values (cap units), then the chunk
// descriptors and one value per chunk (at most maxbig chunks per window).
struct PassBLds {
  int cd_off, cv_off;
  size_t bytes;
};
static PassBLds passb_lds(const HostPlan::Stage &hs, size_t ub) {
  const size_t cd = ((size_t)hs.cap * ub + 15) / 16 * 16;
  const size_t cv = cd + (size_t)hs.maxbig * sizeof(DevWChunk);
  return {(int)cd, (int)cv, cv + (size_t)hs.maxbig * ub};
}

// Bytes of one value per hot group, and per hot leaf (0 without hot
// roots), 256-aligned.
static size_t hot_group_bytes(const sf_s *sf, size_t ub) {
  const HostPlan &h = sf->hp;
  if (!h.hot) return 0;
  return ((size_t)h.hx_grp0.back() * ub + 255) / 256 * 256;
}
static size_t hot_prefix_bytes(const sf_s *sf, size_t ub) {
  const HostPlan &h = sf->hp;
  if (!h.hot) return 0;
  return ((size_t)h.hx_e0.back() * ub + 255) / 256 * 256;
}

// Whether a partitioned Reduce of op OP on T takes the hot path: the ops
// with a native atomic for pass B (SUM, MAX, MIN) in atomic mode, and in
// deterministic mode those whose result does not depend on the order of
// combination.  The location pairs and the product (no native atomic) and
// the deterministic floating-point sum (its canonical pairwise trees) keep
// their hot roots in the windows.
template <typename T, int OP>
static bool reduce_takes_hot(const sf_s *sf, bool atomic) {
  if (!sf->hp.hot || !kHasAtomic<OP>) return false;
  return atomic || OP == OP_MAX || OP == OP_MIN || std::is_integral<T>::value;
}

// Scratch bytes the partitioned Reduce / FetchAndOp of this SF need for a
// unit of ub bytes (0 when the SF does not take that path).
size_t part_scratch_need(const sf_s *sf, size_t ub) {
  const HostPlan &h = sf->hp;
  const int cls = stage_class((int64_t)ub);
  if (!h.part || cls < 0) return 0;
  const size_t main_bytes = ((size_t)sf->nleaves * ub + 255) / 256 * 256;
  const size_t lvl = (size_t)std::max<int64_t>(h.scratch_len, 1) * ub;
  const size_t runs = ((size_t)2 * h.sp[cls].win.size() * ub + 255) / 256 * 256;
  return main_bytes + std::max(2 * lvl, 2 * runs + 2 * hot_group_bytes(sf, ub) + hot_prefix_bytes(sf, ub));
}

template <typename T, int OP, bool ATOM>
static int sp_reduce_launch(unsigned gw, const PassBLds &pl, hipStream_t st, const DevSWin *win,
                            const DevSRoot *sroot, const DevWChunk *wchunk, const uint16_t *lpos, const T *scr,
                            T *lvl_out, T *root, int bs) {
  if (pl.bytes <= kPassBLdsTwo) {
    int rc = allow_lds((const void *)&k_sp_reduce2<T, OP, ATOM>, pl.bytes);
    if (rc) return rc;
    hipLaunchKernelGGL((k_sp_reduce2<T, OP, ATOM>), dim3(gw), dim3(kStageThreads), pl.bytes, st, win, sroot, wchunk,
                       lpos, scr, lvl_out, root, bs, pl.cd_off, pl.cv_off);
    return SF_OK;
  }
  int rc = allow_lds((const void *)&k_sp_reduce<T, OP, ATOM>, pl.bytes);
  if (rc) return rc;
  hipLaunchKernelGGL((k_sp_reduce<T, OP, ATOM>), dim3(gw), dim3(kStageThreads), pl.bytes, st, win, sroot, wchunk, lpos,
                     scr, lvl_out, root, bs, pl.cd_off, pl.cv_off);
  return SF_OK;
}

template <typename T, int OP>
int launch_reduce_part(sf_s *sf, const T *leaf, T *root, int bs, bool atomic, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int64_t L = sf->nleaves;
  const size_t ub = sizeof(T) * (size_t)bs;
  const int cls = stage_class((int64_t)ub);
  const HostPlan::Stage &hs = h.sp[cls];
  const DevPlan::Stage &ds = d.sp[cls];
  const size_t lvl = (size_t)std::max<int64_t>(h.scratch_len, 1) * ub;
  const size_t main_bytes = ((size_t)L * ub + 255) / 256 * 256;
  const bool hot = reduce_takes_hot<T, OP>(sf, atomic);
  void *s = nullptr;
  int rc = acquire_scratch(sf, main_bytes + (hot ? hot_group_bytes(sf, ub) : 2 * lvl), &s);
  if (rc) return rc;
  T *scr = (T *)s;
  T *buf[2] = {(T *)((char *)s + main_bytes), (T *)((char *)s + main_bytes + lvl)};
  const PassBLds pl = passb_lds(hs, ub);
  if constexpr (kHasAtomic<OP>) {
    if (hot) {
      // cold roots through their windows (root updates as in atomic mode:
      // exact for the ops that take this path in deterministic mode), hot
      // roots from their group totals
      T *gsum = (T *)((char *)s + main_bytes);
      rc = sp_move_hot_a<T, OP, HOT_TOTALS>(sf, cls, leaf, scr, bs, gsum, nullptr, st);
      if (rc) return rc;
      if (hs.wcold > 0) {
        rc = sp_reduce_launch<T, OP, true>((unsigned)hs.wcold, pl, st, ds.win, ds.sroot, ds.wchunk, ds.lpos,
                                           (const T *)scr, buf[0], root, bs);
        if (rc) return rc;
      }
      hot_combine<T, OP, HOT_TOTALS>(sf, gsum, nullptr, root, bs, st);
      return sp_check();
    }
  }
  if constexpr (std::is_same<T, Pair>::value)  // pairs: 12-byte scratch units (16-byte aligned leaves)
    rc = sp_move_w<uint4, 0, 0, HotNone, true>(sf, cls, (void *)leaf, scr, bs, st);
  else
    rc = sp_move(sf, cls, 0, (void *)leaf, scr, (int64_t)ub, st);
  if (rc) return rc;
  const unsigned gw = (unsigned)hs.win.size();
  if constexpr (kHasAtomic<OP>) {
    if (atomic) {
      rc = sp_reduce_launch<T, OP, true>(gw, pl, st, ds.win, ds.sroot, ds.wchunk, ds.lpos, (const T *)scr,
                                         buf[0], root, bs);
      if (rc) return rc;
      return sp_check();
    }
  }
  rc = sp_reduce_launch<T, OP, false>(gw, pl, st, ds.win, ds.sroot, ds.wchunk, ds.lpos, (const T *)scr, buf[0],
                                      root, bs);
  if (rc) return rc;
  for (size_t k = 1; k < h.levels.size(); k++) {
    const int nch = (int)h.levels[k].chunks.size();
    hipLaunchKernelGGL((k_det_chunk<T, OP>), dim3((unsigned)((nch * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       d.levels[k], nch, (const int32_t *)nullptr, (const T *)buf[(k - 1) % 2], buf[k % 2], root, bs);
  }
  return sp_check();
}

template <typename T>
int launch_fop_part(sf_s *sf, T *root, const T *leaf, T *upd, int bs, bool atomic, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int64_t L = sf->nleaves;
  const size_t ub = sizeof(T) * (size_t)bs;
  const int cls = stage_class((int64_t)ub);
  const HostPlan::Stage &hs = h.sp[cls];
  const DevPlan::Stage &ds = d.sp[cls];
  const bool hot = h.hot;
  // pass B runs over the windows of cold roots only when hot roots take their own path
  const unsigned gw = (unsigned)(hot ? hs.wcold : (int32_t)hs.win.size());
  const int nspan = hot ? hs.nspan_cold : (int)hs.span_root.size();
  const bool det = !atomic && std::is_integral<T>::value;  // floating point: atomic only
  if (det && (int64_t)2 * hs.win.size() * bs >= INT32_MAX) return SF_ERR_UNSUPPORTED;  // 32-bit run-base index
  // scratch: window-major leaf units, then run totals and run bases (2 per
  // window), then the hot groups' totals and bases
  const size_t main_bytes = ((size_t)L * ub + 255) / 256 * 256;
  const size_t runs_bytes = ((size_t)2 * hs.win.size() * ub + 255) / 256 * 256;
  const size_t grp_bytes = hot_group_bytes(sf, ub);
  const size_t pre_bytes = hot_prefix_bytes(sf, ub);
  void *s = nullptr;
  int rc = acquire_scratch(sf, main_bytes + (det ? 2 * runs_bytes : 0) + 2 * grp_bytes + pre_bytes, &s);
  if (rc) return rc;
  T *scr = (T *)s;
  T *rtot = (T *)((char *)s + main_bytes);
  T *rbase = (T *)((char *)s + main_bytes + runs_bytes);
  T *gsum = (T *)((char *)s + main_bytes + (det ? 2 * runs_bytes : 0));
  T *gbase = (T *)((char *)gsum + grp_bytes);
  T *gpre = (T *)((char *)gbase + grp_bytes);
  const PassBLds pl = passb_lds(hs, ub);
  rc = hot ? sp_move_hot_a<T, OP_SUM, HOT_PREFIX>(sf, cls, leaf, scr, bs, gsum, gpre, st)
           : sp_move(sf, cls, 0, (void *)leaf, scr, (int64_t)ub, st);
  if (rc) return rc;
  if (!det) {
    if (gw > 0) {
      if ((rc = allow_lds((const void *)&k_sp_fop<T, true>, pl.bytes))) return rc;
      hipLaunchKernelGGL((k_sp_fop<T, true>), dim3(gw), dim3(kStageThreads), pl.bytes, st, ds.win, ds.sroot,
                         ds.wchunk, ds.lpos, scr, root, rtot, bs, pl.cd_off, pl.cv_off);
    }
    if (hot) {
      hot_combine<T, OP_SUM, HOT_APPLY>(sf, gsum, gbase, root, bs, st);
      rc = sp_move_hot_c<T, 0>(sf, cls, upd, scr, bs, gbase, gpre, MoveFix{}, st);
    } else {
      rc = sp_move(sf, cls, 1, (void *)upd, scr, (int64_t)ub, st);
    }
    if (rc) return rc;
    return sp_check();
  }
  if constexpr (std::is_integral<T>::value) {
    if (gw > 0) {
      if ((rc = allow_lds((const void *)&k_sp_fop<T, false>, pl.bytes))) return rc;
      hipLaunchKernelGGL((k_sp_fop<T, false>), dim3(gw), dim3(kStageThreads), pl.bytes, st, ds.win, ds.sroot,
                         ds.wchunk, ds.lpos, scr, root, rtot, bs, pl.cd_off, pl.cv_off);
    }
    if (nspan)
      hipLaunchKernelGGL((k_sp_span_scan<T>), dim3((unsigned)((nspan * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                         st, ds.span_first, ds.span_slot, ds.span_root, nspan, (const T *)rtot, rbase, root, bs);
    // pass C with the run bases added: one word per element
    const MoveFix fx{ds.pa_runw, rbase};
    if (hot) {
      hot_combine<T, OP_SUM, HOT_APPLY>(sf, gsum, gbase, root, bs, st);
      rc = sp_move_hot_c<T, (int)sizeof(T)>(sf, cls, upd, scr, bs, gbase, gpre, fx, st);
    } else {
      using EW = typename std::conditional<sizeof(T) == 4, uint32_t, uint2>::type;
      rc = sp_move_w<EW, 1, (int)sizeof(T)>(sf, cls, (void *)upd, scr, bs, st, fx);
    }
    if (rc) return rc;
    return sp_check();
  }
  return SF_ERR_UNSUPPORTED;
}

template int launch_reduce_part<double, OP_SUM>(sf_s *, const double *, double *, int, bool, hipStream_t);
template int launch_reduce_part<double, OP_MAX>(sf_s *, const double *, double *, int, bool, hipStream_t);
template int launch_reduce_part<double, OP_MIN>(sf_s *, const double *, double *, int, bool, hipStream_t);
template int launch_reduce_part<float, OP_SUM>(sf_s *, const float *, float *, int, bool, hipStream_t);
template int launch_reduce_part<float, OP_MAX>(sf_s *, const float *, float *, int, bool, hipStream_t);
template int launch_reduce_part<float, OP_MIN>(sf_s *, const float *, float *, int, bool, hipStream_t);
template int launch_reduce_part<int32_t, OP_SUM>(sf_s *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_reduce_part<int32_t, OP_MAX>(sf_s *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_reduce_part<int32_t, OP_MIN>(sf_s *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_reduce_part<int64_t, OP_SUM>(sf_s *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_reduce_part<int64_t, OP_MAX>(sf_s *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_reduce_part<int64_t, OP_MIN>(sf_s *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_reduce_part<double, OP_PROD>(sf_s *, const double *, double *, int, bool, hipStream_t);
template int launch_reduce_part<float, OP_PROD>(sf_s *, const float *, float *, int, bool, hipStream_t);
template int launch_reduce_part<int32_t, OP_PROD>(sf_s *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_reduce_part<int64_t, OP_PROD>(sf_s *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_reduce_part<Pair, OP_MAXLOC>(sf_s *, const Pair *, Pair *, int, bool, hipStream_t);
template int launch_reduce_part<Pair, OP_MINLOC>(sf_s *, const Pair *, Pair *, int, bool, hipStream_t);
template int launch_fop_part<int32_t>(sf_s *, int32_t *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_fop_part<int64_t>(sf_s *, int64_t *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_fop_part<double>(sf_s *, double *, const double *, double *, int, bool, hipStream_t);
template int launch_fop_part<float>(sf_s *, float *, const float *, float *, int, bool, hipStream_t);

}  // namespace sfi
