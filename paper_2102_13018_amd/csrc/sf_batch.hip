// sf_batch.hip -- many star-forest operations in ONE kernel launch.
//
// Section 5.4 of the paper shows why this matters: each kernel launch costs
// microseconds, comparable to or larger than the work of one small pack or
// unpack, and a host synchronisation between launches exposes that cost.
// Here a batch of independent SF operations (uneven sizes, units and kinds)
// becomes one table of equal-sized work tiles, longest first, and one launch
// gives every tile a block of its own: the hardware dispatcher then balances
// tiles of uneven cost across the CUs (measured faster than persistent grids
// of 2048 or 4096 blocks walking the table, and far faster than blocks that
// take tiles from a device counter, which serialises on one address).  The
// launch can be captured into a HIP graph, and an autotuner picks leaves per
// thread and tile size by timing.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sf_device.h"

namespace sfi {

enum BatchWork : int32_t {
  BW_MOVE16 = 0,  // Bcast REPLACE, 16-byte words
  BW_MOVE8 = 1,   // Bcast REPLACE, 8-byte words
  BW_MOVE4 = 2,   // Bcast REPLACE, 4-byte words
  BW_RED_ATOMIC = 3,  // Reduce SUM with atomics (or plain when no duplicate roots)
  BW_RED_DET = 4,     // Reduce SUM, deterministic, one degree class
  BW_RED_WAVE = 5,    // Reduce SUM, deterministic, one wavefront per root (degree <= kChunk)
  BW_FOP_ATOMIC = 6,  // FetchAndOp SUM with returning atomics (plain without duplicate roots)
  BW_FOP_DET = 7,     // FetchAndOp SUM in leaf order, one degree class, a thread per (root, element)
  BW_FOP_WAVE = 8,    // FetchAndOp SUM in leaf order, one wavefront per root of degree > kSmallMaxDeg
};

struct BatchItemDev {
  const DevSegment *segs;
  const int32_t *ridx, *lidx;
  const int32_t *troot, *toff, *sl;
  const int32_t *cls[kNumClasses];
  const int32_t *large;
  void *root;
  void *leaf;
  void *upd;                 // FetchAndOp: leafupdate
  int32_t dtype, bs, words;  // words: W of the move kinds
  int32_t plain;             // reduce without duplicate roots
  int32_t nv;                // elements per vector access of the deterministic reduce
  int32_t pad;
  uint64_t magic_words, magic_bs, magic_nvg;  // divisions by words, bs, bs / nv
};

struct BatchTile {
  int32_t item, work, seg, t0, t1, cls, pad0, pad1;
};

// q / d for q < 2^24 and d < 2^16 as (q * ceil(2^40 / d)) >> 40.
__host__ __device__ inline uint64_t magic_of(uint32_t d) { return ((1ull << 40) + d - 1) / d; }
__device__ __forceinline__ int fdiv(int q, uint64_t m) { return (int)(((uint64_t)(uint32_t)q * m) >> 40); }

template <typename Word, int LPT>
__device__ __forceinline__ void bw_move(const BatchItemDev &it, const BatchTile &bt) {
  const DevSegment sg = it.segs[bt.seg];
  const int w = it.words;
  const int items = (bt.t1 - bt.t0) * w;
  const Word *root = (const Word *)it.root;
  Word *leaf = (Word *)it.leaf;
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * LPT) {
    Word v[LPT];
    int64_t dst[LPT];
#pragma unroll
    for (int u = 0; u < LPT; u++) {
      const int q = q0 + u * kBlock;
      dst[u] = -1;
      if (q < items) {
        const int lt = fdiv(q, it.magic_words);
        const int c = q - lt * w;
        const int t = bt.t0 + lt;
        const int32_t r = seg_root_s(sg, it.ridx, t);  // indices and leaf writes stream
        const int32_t l = seg_leaf_s(sg, it.lidx, t);
        v[u] = root[(int64_t)r * w + c];
        dst[u] = (int64_t)l * w + c;
      }
    }
#pragma unroll
    for (int u = 0; u < LPT; u++)
      if (dst[u] >= 0) st_stream(leaf + dst[u], v[u]);
  }
}

template <typename T, int LPT>
__device__ __forceinline__ void bw_red_atomic(const BatchItemDev &it, const BatchTile &bt) {
  const DevSegment sg = it.segs[bt.seg];
  const int bs = it.bs;
  const int items = (bt.t1 - bt.t0) * bs;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * LPT) {
    T v[LPT];
    int64_t dst[LPT];
#pragma unroll
    for (int u = 0; u < LPT; u++) {
      const int q = q0 + u * kBlock;
      dst[u] = -1;
      if (q < items) {
        const int lt = fdiv(q, it.magic_bs);
        const int c = q - lt * bs;
        const int t = bt.t0 + lt;
        const int32_t r = seg_root_s(sg, it.ridx, t);  // indices and leaf reads stream
        const int32_t l = seg_leaf_s(sg, it.lidx, t);
        v[u] = ld_stream(leaf + (int64_t)l * bs + c);
        dst[u] = (int64_t)r * bs + c;
      }
    }
#pragma unroll
    for (int u = 0; u < LPT; u++) {
      if (dst[u] < 0) continue;
      if (it.plain)
        root[dst[u]] = Op<OP_SUM, T>::apply(root[dst[u]], v[u]);
      else
        AtomicG<OP_SUM, T>::run(root + dst[u], v[u]);
    }
  }
}

// Deterministic SUM of one degree class: the same register tree as the
// single-SF kernel (canonical pairwise order, root added last), NV
// consecutive elements per thread.
template <typename T, int D, int NV>
__device__ __forceinline__ void bw_det_class(const BatchItemDev &it, const BatchTile &bt) {
  const int bs = it.bs;
  const int ng = bs / NV;
  const int items = (bt.t1 - bt.t0) * ng;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  const int32_t *cls = it.cls[bt.cls];
  for (int q = threadIdx.x; q < items; q += kBlock) {
    const int kk = fdiv(q, it.magic_nvg);
    const int c = (q - kk * ng) * NV;
    const int t = cls[bt.t0 + kk];
    const int g0 = it.toff[t];
    const int n = it.toff[t + 1] - g0;
    const Vec<T, NV> v = pw_tree<D, Vec<T, NV>>(
        n,
        [&](int p) {
          return ld_stream(reinterpret_cast<const Vec<T, NV> *>(leaf + (int64_t)ld_stream(it.sl + g0 + p) * bs + c));
        },
        [](const Vec<T, NV> &a, const Vec<T, NV> &b) { return vop<OP_SUM, T, NV>(a, b); });
    T *rp = root + (int64_t)it.troot[t] * bs + c;
    vst<T, NV>(rp, vop<OP_SUM, T, NV>(vld<T, NV>(rp), v));
  }
}

template <typename T, int D>
__device__ __forceinline__ void bw_det_class_nv(const BatchItemDev &it, const BatchTile &bt) {
  if (it.nv == 4)
    bw_det_class<T, D, (sizeof(T) <= 4 ? 4 : 1)>(it, bt);
  else if (it.nv == 2)
    bw_det_class<T, D, (sizeof(T) <= 8 ? 2 : 1)>(it, bt);
  else
    bw_det_class<T, D, 1>(it, bt);
}

// Deterministic SUM of roots with kSmallMaxDeg < degree <= kChunk: one
// wavefront per root, lanes hold kChunkLPT consecutive leaves.
template <typename T>
__device__ __forceinline__ void bw_det_wave(const BatchItemDev &it, const BatchTile &bt) {
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63;
  const int bs = it.bs;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  for (int k = bt.t0 + (threadIdx.x >> 6); k < bt.t1; k += kBlock / 64) {
    const int t = it.large[k];
    const int g0 = it.toff[t];
    const int n = it.toff[t + 1] - g0;
    const int m = n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (s < m) x[s] = ld_stream(leaf + (int64_t)ld_stream(it.sl + g0 + lane * LPT + s) * bs + c);
#pragma unroll
      for (int d = 1; d < LPT; d *= 2)
#pragma unroll
        for (int p = 0; p + d < LPT; p += 2 * d)
          if (p + d < m) x[p] = Op<OP_SUM, T>::apply(x[p], x[p + d]);
      T v = x[0];
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_down(v, d);
        if ((lane & (2 * d - 1)) == 0 && (lane + d) * LPT < n) v = Op<OP_SUM, T>::apply(v, o);
      }
      if (lane == 0) {
        T *rp = root + (int64_t)it.troot[t] * bs + c;
        *rp = Op<OP_SUM, T>::apply(*rp, v);
      }
    }
  }
}

// FetchAndOp SUM with returning atomics: each leaf fetches the partial
// value its root has when its add arrives (some per-root order).
template <typename T, int LPT>
__device__ __forceinline__ void bw_fop_atomic(const BatchItemDev &it, const BatchTile &bt) {
  const DevSegment sg = it.segs[bt.seg];
  const int bs = it.bs;
  const int items = (bt.t1 - bt.t0) * bs;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  T *upd = (T *)it.upd;
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * LPT) {
    T v[LPT];
    int64_t rp[LPT], lp[LPT];
#pragma unroll
    for (int u = 0; u < LPT; u++) {
      const int q = q0 + u * kBlock;
      rp[u] = -1;
      if (q < items) {
        const int lt = fdiv(q, it.magic_bs);
        const int c = q - lt * bs;
        const int t = bt.t0 + lt;
        const int32_t r = seg_root_s(sg, it.ridx, t);
        const int32_t l = seg_leaf_s(sg, it.lidx, t);
        lp[u] = (int64_t)l * bs + c;
        v[u] = ld_stream(leaf + lp[u]);
        rp[u] = (int64_t)r * bs + c;
      }
    }
#pragma unroll
    for (int u = 0; u < LPT; u++) {
      if (rp[u] < 0) continue;
      T old;
      if (it.plain) {
        old = root[rp[u]];
        root[rp[u]] = Op<OP_SUM, T>::apply(old, v[u]);
      } else {
        old = fetch_add_g(root + rp[u], v[u]);
      }
      st_stream(upd + lp[u], old);
    }
  }
}

// FetchAndOp SUM in leaf order for the roots of one degree class (<= 32
// leaves): a thread per (root, element) loads the root's leaves (sorted
// list, leaf order), then hands out the running value.
template <typename T, int D>
__device__ __forceinline__ void bw_fop_det_class(const BatchItemDev &it, const BatchTile &bt) {
  const int bs = it.bs;
  const int items = (bt.t1 - bt.t0) * bs;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  T *upd = (T *)it.upd;
  const int32_t *cls = it.cls[bt.cls];
  for (int q = threadIdx.x; q < items; q += kBlock) {
    const int kk = fdiv(q, it.magic_bs);
    const int c = q - kk * bs;
    const int t = cls[bt.t0 + kk];
    const int g0 = it.toff[t];
    const int n = it.toff[t + 1] - g0;
    T *rp = root + (int64_t)it.troot[t] * bs + c;
    T acc = *rp;
    // blocks of 8 leaves, one at a time (registers for 8 slots and values)
    constexpr int B = D < 8 ? D : 8;
#pragma unroll
    for (int k = 0; k < D / B; k++) {
      const int m = n - k * B;
      if (m > 0) {
        int64_t sl[B];
        T x[B];
#pragma unroll
        for (int p = 0; p < B; p++)
          if (p < m) sl[p] = (int64_t)ld_stream(it.sl + g0 + k * B + p) * bs + c;
#pragma unroll
        for (int p = 0; p < B; p++)
          if (p < m) x[p] = ld_stream(leaf + sl[p]);
#pragma unroll
        for (int p = 0; p < B; p++)
          if (p < m) {
            st_stream(upd + sl[p], acc);
            acc = Op<OP_SUM, T>::apply(acc, x[p]);
          }
      }
      if constexpr (D > B) __builtin_amdgcn_sched_barrier(0);
    }
    *rp = acc;
  }
}

// FetchAndOp SUM in leaf order for a root of degree > kSmallMaxDeg: one
// wavefront per root walks its sorted leaf list 64 leaves at a time, an
// exclusive wavefront scan giving each leaf the root's value before it.
template <typename T>
__device__ __forceinline__ void bw_fop_wave(const BatchItemDev &it, const BatchTile &bt) {
  const int lane = threadIdx.x & 63;
  const int bs = it.bs;
  const T *leaf = (const T *)it.leaf;
  T *root = (T *)it.root;
  T *upd = (T *)it.upd;
  for (int k = bt.t0 + (threadIdx.x >> 6); k < bt.t1; k += kBlock / 64) {
    const int t = it.large[k];
    const int g0 = it.toff[t];
    const int n = it.toff[t + 1] - g0;
    for (int c = 0; c < bs; c++) {
      T *rp = root + (int64_t)it.troot[t] * bs + c;
      T acc = *rp;
      for (int a = 0; a < n; a += 64) {
        const bool ok = a + lane < n;
        const int64_t l = ok ? (int64_t)ld_stream(it.sl + g0 + a + lane) * bs + c : -1;
        const T v = ok ? ld_stream(leaf + l) : T(0);
        T inc = v;
#pragma unroll
        for (int d = 1; d < 64; d *= 2) {
          const T o = shfl_up(inc, d);
          if (lane >= d) inc = Op<OP_SUM, T>::apply(o, inc);
        }
        const T ex = shfl_up(inc, 1);
        if (ok) st_stream(upd + l, lane == 0 ? acc : Op<OP_SUM, T>::apply(acc, ex));
        acc = Op<OP_SUM, T>::apply(acc, shfl_idx(inc, 63));
      }
      if (lane == 0) *rp = acc;
    }
  }
}

template <typename T, int LPT>
__device__ __forceinline__ void bw_fop(const BatchItemDev &it, const BatchTile &bt) {
  if (bt.work == BW_FOP_ATOMIC) {
    bw_fop_atomic<T, LPT>(it, bt);
  } else if (bt.work == BW_FOP_WAVE) {
    bw_fop_wave<T>(it, bt);
  } else {
    switch (bt.cls) {
      case 0: bw_fop_det_class<T, 1>(it, bt); break;
      case 1: bw_fop_det_class<T, 2>(it, bt); break;
      case 2: bw_fop_det_class<T, 4>(it, bt); break;
      case 3: bw_fop_det_class<T, 8>(it, bt); break;
      case 4: bw_fop_det_class<T, 16>(it, bt); break;
      default: bw_fop_det_class<T, 32>(it, bt); break;
    }
  }
}

template <typename T, int LPT>
__device__ __forceinline__ void bw_reduce(const BatchItemDev &it, const BatchTile &bt) {
  if (bt.work == BW_RED_ATOMIC) {
    bw_red_atomic<T, LPT>(it, bt);
  } else if (bt.work == BW_RED_WAVE) {
    bw_det_wave<T>(it, bt);
  } else {
    switch (bt.cls) {
      case 0: bw_det_class_nv<T, 1>(it, bt); break;
      case 1: bw_det_class_nv<T, 2>(it, bt); break;
      case 2: bw_det_class_nv<T, 4>(it, bt); break;
      case 3: bw_det_class_nv<T, 8>(it, bt); break;
      case 4: bw_det_class_nv<T, 16>(it, bt); break;
      default: bw_det_class_nv<T, 32>(it, bt); break;
    }
  }
}

// One block per tile (a grid smaller than the table walks it in strides).
template <int LPT>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchItemDev *__restrict__ items,
                                                  const BatchTile *__restrict__ tiles, int ntiles) {
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const BatchTile bt = tiles[w];
    const BatchItemDev &it = items[bt.item];
    switch (bt.work) {
      case BW_MOVE16: bw_move<uint4, LPT>(it, bt); break;
      case BW_MOVE8: bw_move<uint2, LPT>(it, bt); break;
      case BW_MOVE4: bw_move<uint32_t, LPT>(it, bt); break;
      case BW_FOP_ATOMIC:
      case BW_FOP_DET:
      case BW_FOP_WAVE:
        switch (it.dtype) {
          case SF_F64: bw_fop<double, LPT>(it, bt); break;
          case SF_F32: bw_fop<float, LPT>(it, bt); break;
          case SF_I32: bw_fop<int32_t, LPT>(it, bt); break;
          default: bw_fop<int64_t, LPT>(it, bt); break;
        }
        break;
      default:
        switch (it.dtype) {
          case SF_F64: bw_reduce<double, LPT>(it, bt); break;
          case SF_F32: bw_reduce<float, LPT>(it, bt); break;
          case SF_I32: bw_reduce<int32_t, LPT>(it, bt); break;
          default: bw_reduce<int64_t, LPT>(it, bt); break;
        }
    }
  }
}

}  // namespace sfi

using namespace sfi;

struct sf_batch_s {
  std::vector<sf_batch_item> items;
  std::vector<uint64_t> gen;  // each item's SF generation when the batch was created
  std::vector<BatchItemDev> hitems;
  std::vector<BatchTile> htiles;
  BatchItemDev *ditems = nullptr;
  BatchTile *dtiles = nullptr;
  size_t dtiles_cap = 0;
  int32_t lpt = 4, tile = kTileLeaves;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static int batch_build_tiles(sf_batch_s *b) {
  b->htiles.clear();
  for (size_t k = 0; k < b->items.size(); k++) {
    const sf_batch_item &it = b->items[k];
    const BatchItemDev &d = b->hitems[k];
    sf_s *sf = it.sf;
    if (it.kind == SF_KIND_BCAST) {
      const int es = elem_size(it.unit.dtype);
      const int64_t ub = (int64_t)es * it.unit.bs;
      const int work = d.words * 16 == ub ? BW_MOVE16 : (d.words * 8 == ub ? BW_MOVE8 : BW_MOVE4);
      for (size_t s = 0; s < sf->hp.dsegs.size(); s++) {
        const int n = sf->hp.dsegs[s].n;
        for (int t0 = 0; t0 < n; t0 += b->tile)
          b->htiles.push_back({(int32_t)k, work, (int32_t)s, t0, std::min(n, t0 + b->tile), 0, 0, 0});
      }
      continue;
    }
    if (it.kind == SF_KIND_FETCH_AND_OP) {
      // integer units with repeated roots: in leaf order (bit-exact) unless
      // the SF asks for atomics; floating point: atomics
      const bool is_int = it.unit.dtype == SF_I32 || it.unit.dtype == SF_I64;
      if (!sf->has_dup_roots || !is_int || sf->reduce_mode == SF_REDUCE_ATOMIC) {
        for (size_t s = 0; s < sf->hp.dsegs.size(); s++) {
          const int n = sf->hp.dsegs[s].n;
          for (int t0 = 0; t0 < n; t0 += b->tile)
            b->htiles.push_back({(int32_t)k, BW_FOP_ATOMIC, (int32_t)s, t0, std::min(n, t0 + b->tile), 0, 0, 0});
        }
        continue;
      }
      for (int c = 0; c < kNumClasses; c++) {
        const int n = (int)sf->hp.cls[c].size();
        const int per = std::max(1, b->tile >> c);
        for (int t0 = 0; t0 < n; t0 += per)
          b->htiles.push_back({(int32_t)k, BW_FOP_DET, 0, t0, std::min(n, t0 + per), c, 0, 0});
      }
      // larger roots: a wavefront each, four per tile; a tile's weight for
      // the ordering below is its leaves
      const int nl = (int)sf->hp.large.size();
      for (int t0 = 0; t0 < nl; t0 += kBlock / 64)
        b->htiles.push_back({(int32_t)k, BW_FOP_WAVE, 0, t0, std::min(nl, t0 + kBlock / 64), 0, 0, 0});
      continue;
    }
    // duplicate roots: deterministic unless the SF asks for atomics (no
    // atomics at all, and the sum is bit-reproducible)
    const bool det = sf->has_dup_roots && sf->reduce_mode != SF_REDUCE_ATOMIC && sf->max_degree <= kChunk;
    if (!det) {
      for (size_t s = 0; s < sf->hp.dsegs.size(); s++) {
        const int n = sf->hp.dsegs[s].n;
        for (int t0 = 0; t0 < n; t0 += b->tile)
          b->htiles.push_back({(int32_t)k, BW_RED_ATOMIC, (int32_t)s, t0, std::min(n, t0 + b->tile), 0, 0, 0});
      }
      continue;
    }
    // deterministic: tiles of roots per degree class, sized so that a tile
    // carries about a quarter of b->tile leaves (their random gathers want
    // more, smaller blocks than the streams: measured best at a quarter)
    for (int c = 0; c < kNumClasses; c++) {
      const int n = (int)sf->hp.cls[c].size();
      const int per = std::max(1, (b->tile / 4) >> c);
      for (int t0 = 0; t0 < n; t0 += per)
        b->htiles.push_back({(int32_t)k, BW_RED_DET, 0, t0, std::min(n, t0 + per), c, 0, 0});
    }
    const int nl = (int)sf->hp.large.size();
    const int per = std::max(1, b->tile / kChunk);
    for (int t0 = 0; t0 < nl; t0 += per)
      b->htiles.push_back({(int32_t)k, BW_RED_WAVE, 0, t0, std::min(nl, t0 + per), 0, 0, 0});
  }
  // largest work first across items (the dispatcher starts it first), by
  // the bytes a tile moves: its leaves x unit bytes, a degree-class-c tile of
  // roots counting 2^c leaves per root and a wavefront tile kChunk per root
  {
    std::vector<int64_t> w(b->htiles.size());
    for (size_t i = 0; i < w.size(); i++) {
      const BatchTile &t = b->htiles[i];
      const sf_batch_item &it = b->items[t.item];
      int64_t n = t.t1 - t.t0;
      if (t.work == BW_RED_DET || t.work == BW_FOP_DET)
        n <<= t.cls;
      else if (t.work == BW_RED_WAVE || t.work == BW_FOP_WAVE)
        n *= kChunk;
      w[i] = n * elem_size(it.unit.dtype) * it.unit.bs;
    }
    std::vector<size_t> ord(w.size());
    for (size_t i = 0; i < ord.size(); i++) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return w[x] > w[y]; });
    std::vector<BatchTile> sorted(ord.size());
    for (size_t i = 0; i < ord.size(); i++) sorted[i] = b->htiles[ord[i]];
    b->htiles.swap(sorted);
  }
  const size_t bytes = std::max<size_t>(b->htiles.size(), 1) * sizeof(BatchTile);
  if (bytes > b->dtiles_cap) {
    if (b->dtiles) (void)hipFree(b->dtiles);  // a new, larger table replaces it
    b->dtiles = nullptr;
    b->dtiles_cap = 0;
    hipError_t e = hipMalloc(&b->dtiles, bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
    b->dtiles_cap = bytes;
  }
  if (!b->htiles.empty()) {
    hipError_t e = hipMemcpy(b->dtiles, b->htiles.data(), b->htiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return set_hip_error(e);
  }
  return SF_OK;
}

// A batch holds device addresses of its SFs' plans (and graph mode 1 their
// scratch): an item whose SF was set up again (or is no longer set up) since
// the batch was created makes every use of the batch fail instead of reading
// freed memory.
static int batch_check(const sf_batch_s *b) {
  for (size_t k = 0; k < b->items.size(); k++) {
    const sf_s *sf = b->items[k].sf;
    if (!sf->setup || sf->generation != b->gen[k]) return SF_ERR_NOT_SETUP;
  }
  return SF_OK;
}

static void batch_free_graph(sf_batch_s *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

extern "C" int sf_batch_create(int32_t n, const sf_batch_item *items, sf_batch_t *out) {
  if (!out) return SF_ERR_ARG;
  *out = nullptr;
  if (n < 0 || (n > 0 && !items)) return SF_ERR_ARG;
  auto *b = new (std::nothrow) sf_batch_s();
  if (!b) return SF_ERR_OOM;
  for (int k = 0; k < n; k++) {
    const sf_batch_item &it = items[k];
    sf_s *sf = it.sf;
    if (!sf || !sf->setup) {
      delete b;
      return sf ? SF_ERR_NOT_SETUP : SF_ERR_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != sf->device) {  // every plan must live on this device
      delete b;
      return SF_ERR_ARG;
    }
    const int es = elem_size(it.unit.dtype);
    if (es <= 0 || it.unit.bs < 1 || it.unit.dtype == SF_F64_I32 || it.unit.dtype == SF_F16 ||
        it.unit.dtype == SF_BF16 || es * (int64_t)it.unit.bs > 4096) {
      delete b;
      return es <= 0 || it.unit.bs < 1 ? SF_ERR_ARG : SF_ERR_UNSUPPORTED;
    }
    if ((it.kind == SF_KIND_BCAST && it.op != SF_REPLACE) || (it.kind == SF_KIND_REDUCE && it.op != SF_SUM) ||
        (it.kind == SF_KIND_FETCH_AND_OP && it.op != SF_SUM) ||
        (it.kind != SF_KIND_BCAST && it.kind != SF_KIND_REDUCE && it.kind != SF_KIND_FETCH_AND_OP)) {
      delete b;
      return SF_ERR_UNSUPPORTED;
    }
    if (sf->nleaves > 0 && (!it.rootdata || !it.leafdata ||
                            (it.kind == SF_KIND_FETCH_AND_OP && (!it.leafupdate || it.leafupdate == it.leafdata)))) {
      delete b;
      return SF_ERR_ARG;
    }
    if (it.kind == SF_KIND_REDUCE && sf->has_dup_roots && sf->reduce_mode == SF_REDUCE_DETERMINISTIC &&
        sf->max_degree > kChunk) {  // AUTO falls back to atomics there
      delete b;
      return SF_ERR_UNSUPPORTED;
    }
    BatchItemDev d{};
    const DevPlan &p = sf->dp;
    d.segs = p.segs;
    d.ridx = p.ridx;
    d.lidx = p.lidx;
    d.troot = p.troot;
    d.toff = p.toff;
    d.sl = p.sl;
    for (int c = 0; c < kNumClasses; c++) d.cls[c] = p.cls[c];
    d.large = p.large;
    d.root = it.rootdata;
    d.leaf = it.leafdata;
    d.upd = it.kind == SF_KIND_FETCH_AND_OP ? it.leafupdate : nullptr;
    d.dtype = it.unit.dtype;
    d.bs = it.unit.bs;
    d.plain = sf->has_dup_roots ? 0 : 1;
    const int64_t ub = (int64_t)es * it.unit.bs;
    const uintptr_t a = (uintptr_t)it.rootdata | (uintptr_t)it.leafdata | (uintptr_t)d.upd;
    d.words = (int32_t)(ub % 16 == 0 && a % 16 == 0 ? ub / 16 : (ub % 8 == 0 && a % 8 == 0 ? ub / 8 : ub / 4));
    d.magic_words = magic_of((uint32_t)d.words);
    d.magic_bs = magic_of((uint32_t)d.bs);
    {
      const uintptr_t al = (uintptr_t)it.rootdata | (uintptr_t)it.leafdata;
      d.nv = 1;
      if (es * 4 <= 16 && d.bs % 4 == 0 && al % (size_t)(es * 4) == 0) d.nv = 4;
      else if (es * 2 <= 16 && d.bs % 2 == 0 && al % (size_t)(es * 2) == 0) d.nv = 2;
      d.magic_nvg = magic_of((uint32_t)(d.bs / d.nv));
    }
    b->items.push_back(it);
    b->gen.push_back(sf->generation);
    b->hitems.push_back(d);
  }
  if (n > 0) {
    hipError_t e = hipMalloc(&b->ditems, sizeof(BatchItemDev) * n);
    if (e != hipSuccess) {
      delete b;
      return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
    }
    e = hipMemcpy(b->ditems, b->hitems.data(), sizeof(BatchItemDev) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(b->ditems);
      delete b;
      return set_hip_error(e);
    }
  }
  int rc = batch_build_tiles(b);
  if (rc) {
    sf_batch_t bb = b;
    sf_batch_destroy(&bb);
    return rc;
  }
  *out = b;
  return SF_OK;
}

static int batch_launch_lpt(sf_batch_s *b, hipStream_t st) {
  const int nt = (int)b->htiles.size();
  if (nt == 0) return SF_OK;
  const unsigned g = (unsigned)nt;  // a block per tile
  switch (b->lpt) {
    case 1: hipLaunchKernelGGL((k_batch<1>), dim3(g), dim3(kBlock), 0, st, b->ditems, b->dtiles, nt); break;
    case 2: hipLaunchKernelGGL((k_batch<2>), dim3(g), dim3(kBlock), 0, st, b->ditems, b->dtiles, nt); break;
    case 8: hipLaunchKernelGGL((k_batch<8>), dim3(g), dim3(kBlock), 0, st, b->ditems, b->dtiles, nt); break;
    default: hipLaunchKernelGGL((k_batch<4>), dim3(g), dim3(kBlock), 0, st, b->ditems, b->dtiles, nt); break;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

extern "C" int sf_batch_launch(sf_batch_t b, hipStream_t stream) {
  if (!b) return SF_ERR_ARG;
  if (int rc = batch_check(b)) return rc;
  return batch_launch_lpt(b, stream);
}

extern "C" int sf_batch_launch_separate(sf_batch_t b, hipStream_t stream) {
  if (!b) return SF_ERR_ARG;
  if (int rc = batch_check(b)) return rc;
  for (const sf_batch_item &it : b->items) {
    std::lock_guard<std::mutex> g(it.sf->mu);
    int rc = it.kind == SF_KIND_BCAST    ? launch_bcast(it.sf, it.unit, it.rootdata, it.leafdata, it.op, stream)
             : it.kind == SF_KIND_REDUCE ? launch_reduce(it.sf, it.unit, it.leafdata, it.rootdata, it.op, stream)
                                         : launch_fetch_and_op(it.sf, it.unit, it.rootdata, it.leafdata,
                                                               it.leafupdate, it.op, stream, true);
    if (rc) return rc;
  }
  return SF_OK;
}

extern "C" int sf_batch_graph_capture(sf_batch_t b, int32_t mode, hipStream_t stream) {
  if (!b || !stream || (mode != 0 && mode != 1)) return SF_ERR_ARG;
  if (int rc = batch_check(b)) return rc;
  batch_free_graph(b);
  if (mode == 1) {
    // the per-item path may grow scratch memory (chunk levels, FetchAndOp
    // chunk sums, or the partitioned path of large SFs): do that before
    // capturing
    for (const sf_batch_item &it : b->items) {
      if (it.kind == SF_KIND_BCAST || !it.sf->has_dup_roots) continue;
      const size_t ub = (size_t)it.unit.bs * elem_size(it.unit.dtype);
      const size_t need = std::max({2 * (size_t)std::max<int64_t>(it.sf->hp.scratch_len, 1) * ub,
                                    it.sf->hp.fo_chunks.size() * ub, part_scratch_need(it.sf, ub)});
      int rc = ensure_scratch(it.sf, need);
      if (rc) return rc;
    }
  }
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return set_hip_error(e);
  int rc = mode == 0 ? sf_batch_launch(b, stream) : sf_batch_launch_separate(b, stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return set_hip_error(e);
  b->graph = graph;
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    batch_free_graph(b);
    return set_hip_error(e);
  }
  return SF_OK;
}

extern "C" int sf_batch_graph_launch(sf_batch_t b, hipStream_t stream) {
  if (!b) return SF_ERR_ARG;
  if (!b->exec) return SF_ERR_NOT_SETUP;
  if (int rc = batch_check(b)) return rc;
  hipError_t e = hipGraphLaunch(b->exec, stream);
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

extern "C" int sf_batch_get_config(sf_batch_t b, int32_t *lpt, int32_t *tile, int64_t *ntiles) {
  if (!b) return SF_ERR_ARG;
  if (lpt) *lpt = b->lpt;
  if (tile) *tile = b->tile;
  if (ntiles) *ntiles = (int64_t)b->htiles.size();
  return SF_OK;
}

extern "C" int sf_batch_set_config(sf_batch_t b, int32_t lpt, int32_t tile) {
  if (!b) return SF_ERR_ARG;
  if (!(lpt == 1 || lpt == 2 || lpt == 4 || lpt == 8)) return SF_ERR_ARG;
  if (tile < 256 || tile > (1 << 16) || (tile & (tile - 1))) return SF_ERR_ARG;
  if (int rc = batch_check(b)) return rc;
  b->lpt = lpt;
  b->tile = tile;
  batch_free_graph(b);
  return batch_build_tiles(b);
}

// Key of a batch for the tuning cache: FNV-1a over the items' shapes.
static std::string batch_key(const sf_batch_s *b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; i++) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const sf_batch_item &it : b->items) {
    mix(it.sf->nleaves);
    mix(it.sf->nroots);
    mix(it.unit.dtype);
    mix(it.unit.bs);
    mix(it.kind);
    mix(it.sf->reduce_mode);
  }
  char buf[64];
  snprintf(buf, sizeof buf, "b%zu-%016llx", b->items.size(), (unsigned long long)h);
  return buf;
}

extern "C" int sf_batch_autotune(sf_batch_t b, const char *cache_path, hipStream_t stream) {
  if (!b) return SF_ERR_ARG;
  if (int rc = batch_check(b)) return rc;
  const std::string key = batch_key(b);
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char k[128];
      int lpt, tile;
      while (fscanf(f, "%127s %d %d", k, &lpt, &tile) == 3) {
        if (key == k) {
          fclose(f);
          return sf_batch_set_config(b, lpt, tile);
        }
      }
      fclose(f);
    }
  }
  const int lpts[] = {1, 2, 4, 8};
  const int tiles[] = {256, 512, 1024, 2048, 4096};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SF_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SF_ERR_HIP;
  }
  float best = 1e30f;
  int best_lpt = b->lpt, best_tile = b->tile;
  int rc = SF_OK;
  for (int tile : tiles) {
    for (int lpt : lpts) {
      rc = sf_batch_set_config(b, lpt, tile);
      if (rc) break;
      rc = sf_batch_launch(b, stream);  // warm-up
      if (rc) break;
      float tot = 0.f;
      const int reps = 5;
      for (int r = 0; r < reps && !rc; r++) {
        hipError_t e = hipEventRecord(e0, stream);
        if (e == hipSuccess) rc = sf_batch_launch(b, stream);
        if (e == hipSuccess && !rc) e = hipEventRecord(e1, stream);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess && !rc) rc = set_hip_error(e);
        tot += ms;
      }
      if (rc) break;
      if (tot < best) {
        best = tot;
        best_lpt = lpt;
        best_tile = tile;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = sf_batch_set_config(b, best_lpt, best_tile);
  if (rc) return rc;
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d\n", key.c_str(), best_lpt, best_tile);
      fclose(f);
    }
  }
  return SF_OK;
}

extern "C" int sf_batch_destroy(sf_batch_t *pb) {
  if (!pb) return SF_ERR_ARG;
  sf_batch_s *b = *pb;
  if (!b) return SF_OK;
  batch_free_graph(b);
  if (b->ditems) (void)hipFree(b->ditems);
  if (b->dtiles) (void)hipFree(b->dtiles);
  delete b;
  *pb = nullptr;
  return SF_OK;
}
