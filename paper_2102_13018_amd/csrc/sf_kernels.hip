// sf_kernels.hip -- gfx950 kernels of SFBcast, SFReduce and SFFetchAndOp on
// one device's share of a star forest, and their launchers.
//
// The work is HBM bound (index streams, root gathers, leaf streams, root
// read-modify-writes); no matrix cores are involved.  Three families:
//  * stream kernels walk the leaves tile by tile in processing order
//    (segment by segment), reading each side's index from an int32 array
//    or computing it from a detected pattern (Section 5.2), and move /
//    combine whole units with the widest aligned word (Bcast REPLACE is a
//    bitwise move keyed on unit bytes);
//  * atomic kernels add leaves onto roots with device-scope atomics
//    (Section 5.3), the roots of highest degree first aggregated per block
//    in LDS so that no single address takes millions of atomics;
//  * deterministic kernels walk the root-sorted leaf lists: per-thread
//    register trees for small degrees, one wavefront per aligned chunk of
//    kChunk leaves for large ones, chunk results combined level by level.
//    Every tree node is a node of the canonical pairwise tree of the root's
//    leaves in leaf order, so the result is the same for any launch shape.
#include <algorithm>

#include "sf_det_kernels.h"

namespace sfi {

// ===================================================================== Bcast
// leaf[l] = root[r] as W words of type Word per unit.  2^sh blocks per
// tile, each taking its share of the tile's leaves: on SFs with full-size
// tiles the random root gathers want more, smaller blocks than the plan's
// tiles (measured on the 16M-leaf Zipf SF: 106 us with a block per 1024-leaf
// tile, 102 with a block per half; the halo's small tiles stay whole).
template <typename Word, int W>
__global__ __launch_bounds__(kBlock) void k_bcast_move(const DevSegment *__restrict__ segs,
                                                       const DevTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ ridx,
                                                       const int32_t *__restrict__ lidx,
                                                       const Word *__restrict__ root, Word *__restrict__ leaf,
                                                       int wrt, int sh) {
  DevTile tl = tiles[blockIdx.x >> sh];
  if (sh) {  // tiles hold at most kTileLeaves leaves: no overflow
    const int part = (int)(blockIdx.x & ((1u << sh) - 1)), len = tl.t1 - tl.t0;
    tl.t1 = tl.t0 + ((len * (part + 1)) >> sh);
    tl.t0 = tl.t0 + ((len * part) >> sh);
  }
  const DevSegment sg = segs[tl.seg];
  const int w = W > 0 ? W : wrt;
  const int items = (tl.t1 - tl.t0) * w;
  constexpr int U = 4;  // loads in flight per thread (more, smaller blocks measured faster)
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
    Word v[U];
    int64_t dst[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int q = q0 + u * kBlock;
      dst[u] = -1;
      if (q < items) {
        const int t = tl.t0 + q / w;
        const int c = q % w;
        // indices and leaf writes stream (used once); root reads stay cached
        const int32_t r = seg_root_s(sg, ridx, t);
        const int32_t l = seg_leaf_s(sg, lidx, t);
        v[u] = root[(int64_t)r * w + c];
        dst[u] = (int64_t)l * w + c;
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (dst[u] >= 0) st_stream(leaf + dst[u], v[u]);
  }
}

// leaf[l][c] = op(leaf[l][c], root[r][c]) element-wise.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_bcast_op(const DevSegment *__restrict__ segs,
                                                     const DevTile *__restrict__ tiles,
                                                     const int32_t *__restrict__ ridx,
                                                     const int32_t *__restrict__ lidx, const T *__restrict__ root,
                                                     T *__restrict__ leaf, int bs) {
  const DevTile tl = tiles[blockIdx.x];
  const DevSegment sg = segs[tl.seg];
  const int items = (tl.t1 - tl.t0) * bs;
  for (int q = threadIdx.x; q < items; q += kBlock) {
    const int t = tl.t0 + q / bs;
    const int c = q % bs;
    const int32_t r = seg_root(sg, ridx, t);
    const int32_t l = seg_leaf(sg, lidx, t);
    T *p = leaf + (int64_t)l * bs + c;
    st(p, Op<OP, T>::apply(ld(p), ld(root + (int64_t)r * bs + c)));
  }
}

// ===================================================== Reduce: stream kinds
// root[r][c] = op(root[r][c], leaf[l][c]) without atomics: every root has at
// most one leaf (no duplicate roots), or the op is REPLACE on such an SF.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_reduce_plain(const DevSegment *__restrict__ segs,
                                                         const DevTile *__restrict__ tiles,
                                                         const int32_t *__restrict__ ridx,
                                                         const int32_t *__restrict__ lidx,
                                                         const T *__restrict__ leaf, T *__restrict__ root, int bs) {
  const DevTile tl = tiles[blockIdx.x];
  const DevSegment sg = segs[tl.seg];
  const int items = (tl.t1 - tl.t0) * bs;
  constexpr int U = 4;  // elements per thread with all their loads in flight
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
    int64_t rq[U], lq[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int q = q0 + u * kBlock;
      rq[u] = -1;
      if (q < items) {
        const int lt = bs == 1 ? q : q / bs;
        const int t = tl.t0 + lt;
        const int c = q - lt * bs;
        rq[u] = (int64_t)seg_root_s(sg, ridx, t) * bs + c;
        lq[u] = (int64_t)seg_leaf_s(sg, lidx, t) * bs + c;
      }
    }
    T lv[U], rv[U];
#pragma unroll
    for (int u = 0; u < U; u++)
      if (rq[u] >= 0) {
        lv[u] = ld_stream(leaf + lq[u]);
        rv[u] = ld(root + rq[u]);
      }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (rq[u] >= 0) st(root + rq[u], Op<OP, T>::apply(rv[u], lv[u]));
  }
}

// Atomic reduction over a persistent grid.  Roots encoded as -(h+1) in
// ridx_hot with h < nhot_lds are combined in this block's LDS first and
// written with one device atomic per touched root when the block is done.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_reduce_atomic(const DevSegment *__restrict__ segs,
                                                          const DevTile *__restrict__ tiles, int ntiles,
                                                          const int32_t *__restrict__ ridx,
                                                          const int32_t *__restrict__ lidx,
                                                          const int32_t *__restrict__ hot_roots, int nhot_lds,
                                                          const T *__restrict__ leaf, T *__restrict__ root, int bs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *acc = reinterpret_cast<T *>(smem);
  int32_t *touched = reinterpret_cast<int32_t *>(smem + (size_t)nhot_lds * bs * sizeof(T));
  for (int k = threadIdx.x; k < nhot_lds * bs; k += kBlock) acc[k] = op_identity<OP, T>();
  for (int k = threadIdx.x; k < nhot_lds; k += kBlock) touched[k] = 0;
  __syncthreads();
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const DevTile tl = tiles[tile];
    const DevSegment sg = segs[tl.seg];
    const int items = (tl.t1 - tl.t0) * bs;
    constexpr int U = 4;
    for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
      T v[U];
      int32_t rr[U];
      int cc[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int q = q0 + u * kBlock;
        rr[u] = INT32_MIN;
        if (q < items) {
          const int t = tl.t0 + q / bs;
          cc[u] = q % bs;
          rr[u] = seg_root(sg, ridx, t);
          const int32_t l = seg_leaf(sg, lidx, t);
          v[u] = leaf[(int64_t)l * bs + cc[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (rr[u] == INT32_MIN) continue;
        if (rr[u] >= 0) {
          AtomicG<OP, T>::run(root + (int64_t)rr[u] * bs + cc[u], v[u]);
        } else {
          const int h = -rr[u] - 1;
          if (h < nhot_lds) {
            AtomicL<OP, T>::run(acc + h * bs + cc[u], v[u]);
            touched[h] = 1;
          } else {
            AtomicG<OP, T>::run(root + (int64_t)hot_roots[h] * bs + cc[u], v[u]);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nhot_lds * bs; k += kBlock) {
    const int h = k / bs, c = k % bs;
    if (touched[h]) AtomicG<OP, T>::run(root + (int64_t)hot_roots[h] * bs + c, acc[k]);
  }
}

// MAXLOC on the atomic path, in passes over the leaf stream:
//  (1) save each touched root's value,  (2) atomic max of the value,
//  (3) reset the index of roots whose value changed, (4) atomic min of the
//  index over the leaves whose value equals the root's final value.
__global__ __launch_bounds__(kBlock) void k_maxloc_save(const int32_t *__restrict__ troot, int ntouched,
                                                        const Pair *__restrict__ root, double *__restrict__ saved,
                                                        int bs) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)ntouched * bs) return;
  const int t = (int)(q / bs), c = (int)(q % bs);
  saved[q] = root[(int64_t)troot[t] * bs + c].v;
}
__global__ __launch_bounds__(kBlock) void k_maxloc_fix(const int32_t *__restrict__ troot, int ntouched,
                                                       Pair *__restrict__ root, const double *__restrict__ saved,
                                                       int bs) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)ntouched * bs) return;
  const int t = (int)(q / bs), c = (int)(q % bs);
  Pair *p = root + (int64_t)troot[t] * bs + c;
  if (__double_as_longlong(p->v) != __double_as_longlong(saved[q])) p->i = INT32_MAX;
}
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_maxloc_stream(const DevSegment *__restrict__ segs,
                                                          const DevTile *__restrict__ tiles,
                                                          const int32_t *__restrict__ ridx,
                                                          const int32_t *__restrict__ lidx,
                                                          const Pair *__restrict__ leaf, Pair *__restrict__ root,
                                                          int bs) {
  const DevTile tl = tiles[blockIdx.x];
  const DevSegment sg = segs[tl.seg];
  const int items = (tl.t1 - tl.t0) * bs;
  for (int q = threadIdx.x; q < items; q += kBlock) {
    const int t = tl.t0 + q / bs;
    const int c = q % bs;
    const int32_t r = seg_root(sg, ridx, t);
    const int32_t l = seg_leaf(sg, lidx, t);
    const Pair *s = leaf + (int64_t)l * bs + c;
    Pair *d = root + (int64_t)r * bs + c;
    if (PASS == 0) {
      AtomicG<OP_MAX, double>::run(&d->v, s->v);
    } else {
      const double rv = __hip_atomic_load(&d->v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__double_as_longlong(rv) == __double_as_longlong(s->v))
        __hip_atomic_fetch_min(&d->i, s->i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ============================================== Reduce: deterministic kinds
// All roots of degree <= kSmallMaxDeg in one launch (the classes
// concatenated, so a wavefront mostly sees one class): one thread per (root,
// group of NV consecutive elements), the leaves loaded in leaf order into
// registers with vector loads and combined bottom-up -- the canonical
// pairwise tree, element by element.  The root is combined last.
template <typename T, int OP, int NV, int D>
__device__ __forceinline__ Vec<T, NV> small_tree_v(const int32_t *__restrict__ sl, const T *__restrict__ leaf, int g0,
                                                   int n, int bs, int c) {
  return pw_tree<D, Vec<T, NV>>(
      n, [&](int p) { return vld<T, NV>(leaf + (int64_t)sl[g0 + p] * bs + c); },
      [](const Vec<T, NV> &a, const Vec<T, NV> &b) { return vop<OP, T, NV>(a, b); });
}

template <typename T, int OP, int NV>
__global__ __launch_bounds__(kBlock) void k_det_small_all(const int32_t *__restrict__ list, int count,
                                                          const int32_t *__restrict__ troot,
                                                          const int32_t *__restrict__ toff,
                                                          const int32_t *__restrict__ sl, const T *__restrict__ leaf,
                                                          T *__restrict__ root, int bs) {
  const int nv = bs / NV;
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)count * nv) return;
  const int k = (int)(q / nv), c = (int)(q - (int64_t)k * nv) * NV;
  const int t = list[k];
  const int g0 = toff[t];
  const int n = toff[t + 1] - g0;
  Vec<T, NV> v;
  if (n <= 1)
    v = small_tree_v<T, OP, NV, 1>(sl, leaf, g0, n, bs, c);
  else if (n <= 2)
    v = small_tree_v<T, OP, NV, 2>(sl, leaf, g0, n, bs, c);
  else if (n <= 4)
    v = small_tree_v<T, OP, NV, 4>(sl, leaf, g0, n, bs, c);
  else if (n <= 8)
    v = small_tree_v<T, OP, NV, 8>(sl, leaf, g0, n, bs, c);
  else if (n <= 16)
    v = small_tree_v<T, OP, NV, 16>(sl, leaf, g0, n, bs, c);
  else
    v = small_tree_v<T, OP, NV, 32>(sl, leaf, g0, n, bs, c);
  T *rp = root + (int64_t)troot[t] * bs + c;
  vst<T, NV>(rp, vop<OP, T, NV>(vld<T, NV>(rp), v));
}

// The Reduce split (one launch): blocks [0, ntiles) stream the leaves of the
// single-leaf roots tile by tile (index or pattern addressing; a leaf whose
// processing position is marked in rep_bits belongs to a repeated root and
// is skipped) and update those roots plainly; the remaining blocks give each
// (repeated root, element) its register tree over the root's sorted leaves,
// exactly as k_det_small_all.  The two parts write disjoint roots.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_reduce_split(const DevSegment *__restrict__ segs,
                                                         const DevTile *__restrict__ tiles, int ntiles,
                                                         const int32_t *__restrict__ ridx,
                                                         const int32_t *__restrict__ lidx,
                                                         const uint32_t *__restrict__ rep_bits,
                                                         const int32_t *__restrict__ rep_list, int nrep,
                                                         const int32_t *__restrict__ troot,
                                                         const int32_t *__restrict__ toff,
                                                         const int32_t *__restrict__ sl, const T *__restrict__ leaf,
                                                         T *__restrict__ root, int bs) {
  if ((int)blockIdx.x < ntiles) {
    const DevTile tl = tiles[blockIdx.x];
    const DevSegment sg = segs[tl.seg];
    const int items = (tl.t1 - tl.t0) * bs;
    constexpr int U = 4;  // elements per thread with all their loads in flight
    for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
      int64_t rq[U], lq[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int q = q0 + u * kBlock;
        rq[u] = -1;
        if (q < items) {
          const int lt = bs == 1 ? q : q / bs;
          const int t = tl.t0 + lt;
          const int c = q - lt * bs;
          const int p = sg.pbase + t;
          if (!((rep_bits[p >> 5] >> (p & 31)) & 1u)) {
            rq[u] = (int64_t)seg_root_s(sg, ridx, t) * bs + c;
            lq[u] = (int64_t)seg_leaf_s(sg, lidx, t) * bs + c;
          }
        }
      }
      T lv[U], rv[U];
#pragma unroll
      for (int u = 0; u < U; u++)
        if (rq[u] >= 0) {
          lv[u] = ld_stream(leaf + lq[u]);
          rv[u] = ld(root + rq[u]);
        }
#pragma unroll
      for (int u = 0; u < U; u++)
        if (rq[u] >= 0) st(root + rq[u], Op<OP, T>::apply(rv[u], lv[u]));
    }
    return;
  }
  const int64_t q = (int64_t)(blockIdx.x - ntiles) * kBlock + threadIdx.x;
  if (q >= (int64_t)nrep * bs) return;
  const int k = (int)(q / bs), c = (int)(q - (int64_t)k * bs);
  const int t = rep_list[k];
  const int g0 = toff[t];
  const int n = toff[t + 1] - g0;
  Vec<T, 1> v;
  if (n <= 2)
    v = small_tree_v<T, OP, 1, 2>(sl, leaf, g0, n, bs, c);
  else if (n <= 4)
    v = small_tree_v<T, OP, 1, 4>(sl, leaf, g0, n, bs, c);
  else if (n <= 8)
    v = small_tree_v<T, OP, 1, 8>(sl, leaf, g0, n, bs, c);
  else if (n <= 16)
    v = small_tree_v<T, OP, 1, 16>(sl, leaf, g0, n, bs, c);
  else
    v = small_tree_v<T, OP, 1, 32>(sl, leaf, g0, n, bs, c);
  T *rp = root + (int64_t)troot[t] * bs + c;
  vst<T, 1>(rp, vop<OP, T, 1>(vld<T, 1>(rp), v));
}

// Reduce REPLACE with duplicate roots: the last leaf in leaf order wins.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_det_replace(const int32_t *__restrict__ troot, int ntouched,
                                                        const int32_t *__restrict__ toff,
                                                        const int32_t *__restrict__ sl, const T *__restrict__ leaf,
                                                        T *__restrict__ root, int bs) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)ntouched * bs) return;
  const int t = (int)(q / bs), c = (int)(q % bs);
  st(root + (int64_t)troot[t] * bs + c, ld(leaf + (int64_t)sl[toff[t + 1] - 1] * bs + c));
}

// ================================================================ FetchAndOp
// Atomic path: every leaf element fetches and adds in one device atomic.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_atomic(const DevSegment *__restrict__ segs,
                                                       const DevTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ ridx,
                                                       const int32_t *__restrict__ lidx, T *__restrict__ root,
                                                       const T *__restrict__ leaf, T *__restrict__ upd, int bs) {
  const DevTile tl = tiles[blockIdx.x];
  const DevSegment sg = segs[tl.seg];
  const int items = (tl.t1 - tl.t0) * bs;
  for (int q = threadIdx.x; q < items; q += kBlock) {
    const int t = tl.t0 + q / bs;
    const int c = q % bs;
    const int32_t r = seg_root(sg, ridx, t);
    const int64_t l = (int64_t)seg_leaf(sg, lidx, t) * bs + c;
    upd[l] = fetch_add_g(root + (int64_t)r * bs + c, leaf[l]);
  }
}

// Atomic path with block aggregation of hot roots, over a persistent grid.
// Pass 1 over the block's tiles: ordinary leaves fetch-and-add on the
// device; leaves of hot roots only add into an LDS total.  The block then
// reserves each total with ONE device fetch-and-add, which returns the base
// of the block's run of partial values.  Pass 2 over the same tiles: the hot
// leaves fetch-and-add on that LDS base, obtaining consecutive partial
// values of the root (a valid per-root order of the reductions).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_atomic_hot(const DevSegment *__restrict__ segs,
                                                           const DevTile *__restrict__ tiles, int ntiles,
                                                           const int32_t *__restrict__ ridx_hot,
                                                           const int32_t *__restrict__ lidx,
                                                           const int32_t *__restrict__ hot_roots, int nhot_lds,
                                                           T *__restrict__ root, const T *__restrict__ leaf,
                                                           T *__restrict__ upd, int bs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *acc = reinterpret_cast<T *>(smem);
  int32_t *touched = reinterpret_cast<int32_t *>(smem + (size_t)nhot_lds * bs * sizeof(T));
  for (int k = threadIdx.x; k < nhot_lds * bs; k += kBlock) acc[k] = T(0);
  for (int k = threadIdx.x; k < nhot_lds; k += kBlock) touched[k] = 0;
  __syncthreads();
  constexpr int U = 4;  // returning atomics in flight per thread
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const DevTile tl = tiles[tile];
    const DevSegment sg = segs[tl.seg];
    const int items = (tl.t1 - tl.t0) * bs;
    for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
      T v[U], got[U];
      int64_t ro[U];
      int ldso[U];
      int64_t l[U];
      int32_t kind[U];  // 0 none, 1 device atomic, 2 LDS
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int q = q0 + u * kBlock;
        kind[u] = 0;
        if (q < items) {
          const int t = tl.t0 + q / bs;
          const int c = q % bs;
          const int32_t r = seg_root(sg, ridx_hot, t);
          l[u] = (int64_t)seg_leaf(sg, lidx, t) * bs + c;
          v[u] = leaf[l[u]];
          if (r >= 0 || -r - 1 >= nhot_lds) {
            kind[u] = 1;
            ro[u] = (int64_t)(r >= 0 ? r : hot_roots[-r - 1]) * bs + c;
          } else {
            kind[u] = 2;
            ldso[u] = (-r - 1) * bs + c;
            touched[-r - 1] = 1;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (kind[u] == 1)
          got[u] = fetch_add_g(root + ro[u], v[u]);
        else if (kind[u] == 2)
          __hip_atomic_fetch_add(acc + ldso[u], v[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
#pragma unroll
      for (int u = 0; u < U; u++)
        if (kind[u] == 1) upd[l[u]] = got[u];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nhot_lds * bs; k += kBlock)
    if (touched[k / bs]) acc[k] = fetch_add_g(root + (int64_t)hot_roots[k / bs] * bs + k % bs, acc[k]);
  __syncthreads();
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const DevTile tl = tiles[tile];
    const DevSegment sg = segs[tl.seg];
    const int items = (tl.t1 - tl.t0) * bs;
    for (int q = threadIdx.x; q < items; q += kBlock) {
      const int t = tl.t0 + q / bs;
      const int32_t r = seg_root(sg, ridx_hot, t);
      if (r >= 0 || -r - 1 >= nhot_lds) continue;
      const int c = q % bs;
      const int64_t l = (int64_t)seg_leaf(sg, lidx, t) * bs + c;
      upd[l] = __hip_atomic_fetch_add(acc + (-r - 1) * bs + c, leaf[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Deterministic path (integer units): roots of degree <= kSmallMaxDeg, one
// thread per (root, element), leaves applied in leaf order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_small(const int32_t *__restrict__ cls, int count,
                                                      const int32_t *__restrict__ troot,
                                                      const int32_t *__restrict__ toff,
                                                      const int32_t *__restrict__ sl, T *__restrict__ root,
                                                      const T *__restrict__ leaf, T *__restrict__ upd, int bs) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)count * bs) return;
  const int k = (int)(q / bs), c = (int)(q % bs);
  const int t = cls[k];
  const int g0 = toff[t], g1 = toff[t + 1];
  T *rp = root + (int64_t)troot[t] * bs + c;
  T a = *rp;
  for (int g = g0; g < g1; g++) {
    const int64_t l = (int64_t)sl[g] * bs + c;
    upd[l] = a;
    a = Op<OP_SUM, T>::apply(a, leaf[l]);
  }
  *rp = a;
}

// Large roots, pass 1: sum of every chunk (order-free for integers).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_chunk_sum(const DevChunk *__restrict__ chunks, int nchunks,
                                                          const int32_t *__restrict__ sl, const T *__restrict__ leaf,
                                                          T *__restrict__ sums, int bs) {
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63;
  const int wid = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
  if (wid >= nchunks) return;
  const DevChunk ch = chunks[wid];
  for (int c = 0; c < bs; c++) {
    T a = T(0);
#pragma unroll
    for (int s = 0; s < LPT; s++) {
      const int e = lane * LPT + s;
      if (e < ch.n) a = Op<OP_SUM, T>::apply(a, leaf[(int64_t)sl[ch.src + e] * bs + c]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d /= 2) a = Op<OP_SUM, T>::apply(a, shfl_down(a, d));
    if (lane == 0) sums[(int64_t)wid * bs + c] = a;
  }
}

// Large roots, pass 3: exclusive prefix inside every chunk, plus its base.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_chunk_apply(const DevChunk *__restrict__ chunks, int nchunks,
                                                            const int32_t *__restrict__ sl,
                                                            const T *__restrict__ leaf, const T *__restrict__ sums,
                                                            T *__restrict__ upd, int bs) {
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63;
  const int wid = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
  if (wid >= nchunks) return;
  const DevChunk ch = chunks[wid];
  int64_t li[LPT];
#pragma unroll
  for (int s = 0; s < LPT; s++) {
    const int e = lane * LPT + s;
    li[s] = e < ch.n ? (int64_t)sl[ch.src + e] : -1;
  }
  for (int c = 0; c < bs; c++) {
    T x[LPT];
    T lane_sum = T(0);
#pragma unroll
    for (int s = 0; s < LPT; s++) {
      x[s] = li[s] >= 0 ? leaf[li[s] * bs + c] : T(0);
      lane_sum = Op<OP_SUM, T>::apply(lane_sum, x[s]);
    }
    T inc = lane_sum;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
      const T o = shfl_up(inc, d);
      if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o);
    }
    T a = Op<OP_SUM, T>::apply(sums[(int64_t)wid * bs + c], wrap_sub(inc, lane_sum));
#pragma unroll
    for (int s = 0; s < LPT; s++) {
      if (li[s] >= 0) upd[li[s] * bs + c] = a;
      a = Op<OP_SUM, T>::apply(a, x[s]);
    }
  }
}

// ================================================================ launchers
static inline unsigned nblocks(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

static int check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

template <typename Word>
static void bcast_move_w(sf_s *sf, int W, const void *root, void *leaf, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const int sh = sf->hp.tile_leaves >= kTileLeaves ? 1 : 0;  // two blocks per full-size tile
  const unsigned g = (unsigned)sf->hp.tiles.size() << sh;
  const Word *r = (const Word *)root;
  Word *l = (Word *)leaf;
#define SF_MOVE(WW)                                                                                             \
  hipLaunchKernelGGL((k_bcast_move<Word, WW>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx, d.lidx, r, l, \
                     W, sh)
  switch (W) {
    case 1: SF_MOVE(1); break;
    case 2: SF_MOVE(2); break;
    case 3: SF_MOVE(3); break;
    case 4: SF_MOVE(4); break;
    case 5: SF_MOVE(5); break;
    case 6: SF_MOVE(6); break;
    case 7: SF_MOVE(7); break;
    case 8: SF_MOVE(8); break;
    default: SF_MOVE(0); break;
  }
#undef SF_MOVE
}

template <typename T>
static int bcast_op_t(sf_s *sf, int bs, int op, const void *root, void *leaf, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const unsigned g = (unsigned)sf->hp.tiles.size();
  const T *r = (const T *)root;
  T *l = (T *)leaf;
#define SF_BOP(OPV) \
  hipLaunchKernelGGL((k_bcast_op<T, OPV>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx, d.lidx, r, l, bs)
  switch (op) {
    case SF_SUM: SF_BOP(OP_SUM); break;
    case SF_MAX: SF_BOP(OP_MAX); break;
    case SF_MIN: SF_BOP(OP_MIN); break;
    case SF_PROD: SF_BOP(OP_PROD); break;
    default: return SF_ERR_UNSUPPORTED;
  }
#undef SF_BOP
  return SF_OK;
}

// Contiguous roots and contiguous leaves in every segment (Section 5.2: no
// pack needed): a REPLACE is one device-to-device copy per segment.
// dir 0: root -> leaf (Bcast), dir 1: leaf -> root (Reduce without
// duplicate roots).
static int copy_segments(sf_s *sf, int64_t ub, const void *root, void *leafv, int dir, hipStream_t st) {
  for (const DevSegment &d : sf->hp.dsegs) {
    char *r = (char *)root + (int64_t)d.root.start * ub;
    char *l = (char *)leafv + (int64_t)d.leaf.start * ub;
    hipError_t e = dir == 0 ? hipMemcpyAsync(l, r, (size_t)d.n * ub, hipMemcpyDeviceToDevice, st)
                            : hipMemcpyAsync(r, l, (size_t)d.n * ub, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return set_hip_error(e);
  }
  return SF_OK;
}

int launch_bcast(sf_s *sf, sf_unit unit, const void *root, void *leaf, int op, hipStream_t st) {
  if (sf->hp.tiles.empty()) return SF_OK;
  const int es = elem_size(unit.dtype);
  if (op == SF_REPLACE && unit.dtype != SF_F64_I32 && sf->hp.all_contig)
    return copy_segments(sf, (int64_t)es * unit.bs, root, leaf, 0, st);
  if (op == SF_REPLACE && unit.dtype != SF_F64_I32) {
    const int64_t ub = (int64_t)es * unit.bs;
    const uintptr_t a = (uintptr_t)root | (uintptr_t)leaf;
    if (ub % 16 == 0 && a % 16 == 0)
      bcast_move_w<uint4>(sf, (int)(ub / 16), root, leaf, st);
    else if (ub % 8 == 0 && a % 8 == 0)
      bcast_move_w<uint2>(sf, (int)(ub / 8), root, leaf, st);
    else if (ub % 4 == 0 && a % 4 == 0)
      bcast_move_w<uint32_t>(sf, (int)(ub / 4), root, leaf, st);
    else  // 16-bit units of an odd count
      bcast_move_w<uint16_t>(sf, (int)(ub / 2), root, leaf, st);
    return check_launch();
  }
  int rc;
  switch (unit.dtype) {
    case SF_F64: rc = bcast_op_t<double>(sf, unit.bs, op, root, leaf, st); break;
    case SF_F32: rc = bcast_op_t<float>(sf, unit.bs, op, root, leaf, st); break;
    case SF_I32: rc = bcast_op_t<int32_t>(sf, unit.bs, op, root, leaf, st); break;
    case SF_I64: rc = bcast_op_t<int64_t>(sf, unit.bs, op, root, leaf, st); break;
    case SF_F16: rc = bcast_op_t<H16>(sf, unit.bs, op, root, leaf, st); break;
    case SF_BF16: rc = bcast_op_t<BF16>(sf, unit.bs, op, root, leaf, st); break;
    case SF_F64_I32: {
      const DevPlan &d = sf->dp;
      const unsigned g = (unsigned)sf->hp.tiles.size();
      if (op == SF_MAXLOC)
        hipLaunchKernelGGL((k_bcast_op<Pair, OP_MAXLOC>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx,
                           d.lidx, (const Pair *)root, (Pair *)leaf, unit.bs);
      else if (op == SF_MINLOC)
        hipLaunchKernelGGL((k_bcast_op<Pair, OP_MINLOC>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx,
                           d.lidx, (const Pair *)root, (Pair *)leaf, unit.bs);
      else if (op == SF_REPLACE)
        hipLaunchKernelGGL((k_bcast_op<Pair, OP_REPLACE>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx,
                           d.lidx, (const Pair *)root, (Pair *)leaf, unit.bs);
      else
        return SF_ERR_UNSUPPORTED;
      rc = SF_OK;
      break;
    }
    default: return SF_ERR_UNSUPPORTED;
  }
  if (rc) return rc;
  return check_launch();
}

// -------------------------------------------------------------- Reduce
template <typename T, int OP>
static int reduce_split_t(sf_s *sf, const T *leaf, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int ntiles = (int)h.tiles.size(), nrep = (int)h.rep_list.size();
  const unsigned g = (unsigned)ntiles + nblocks((int64_t)nrep * bs);
  hipLaunchKernelGGL((k_reduce_split<T, OP>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, ntiles, d.ridx, d.lidx,
                     d.rep_bits, d.rep_list, nrep, d.troot, d.toff, d.sl, leaf, root, bs);
  return check_launch();
}

template <typename T, int OP>
static int reduce_det_t(sf_s *sf, const T *leaf, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const size_t ub = sizeof(T) * (size_t)bs;
  if constexpr (!kIsHalf<T>) {  // 16-bit units are not partitioned
    if (OP != OP_REPLACE && h.part_red_det && stage_class((int64_t)ub) >= 0 &&
        scratch_fits(sf, part_scratch_need(sf, ub)))
      return launch_reduce_part<T, OP>(sf, leaf, root, bs, false, st);
  }
  if (OP != OP_REPLACE && h.split && ub > kSplitMinUnit) return reduce_split_t<T, OP>(sf, leaf, root, bs, st);
  if (OP == OP_REPLACE) {
    const int64_t T_ = (int64_t)h.troot.size();
    if (T_)
      hipLaunchKernelGGL((k_det_replace<T>), dim3(nblocks(T_ * bs)), dim3(kBlock), 0, st, d.troot, (int)T_, d.toff,
                         d.sl, leaf, root, bs);
    return check_launch();
  }
  // scratch of the chunk levels first, so that nothing is enqueued when it
  // cannot be had
  T *buf[2] = {nullptr, nullptr};
  if (!h.levels.empty()) {
    const size_t len = (size_t)std::max<int64_t>(h.scratch_len, 1) * bs;
    void *s = nullptr;
    int rc = acquire_scratch(sf, 2 * len * sizeof(T), &s);
    if (rc) return rc;
    buf[0] = (T *)s;
    buf[1] = (T *)s + len;
  }
  // all small classes in one launch, NV elements per thread when the unit
  // and the buffers allow vector accesses
  if (!h.small_all.empty()) {
    const uintptr_t al = (uintptr_t)leaf | (uintptr_t)root;
    const int cnt = (int)h.small_all.size();
    int nv = 1;
    if (sizeof(T) * 4 <= 16 && bs % 4 == 0 && al % (sizeof(T) * 4) == 0) nv = 4;
    else if (sizeof(T) * 2 <= 16 && bs % 2 == 0 && al % (sizeof(T) * 2) == 0) nv = 2;
    if (nv == 4)
      hipLaunchKernelGGL((k_det_small_all<T, OP, (sizeof(T) <= 4 ? 4 : 1)>), dim3(nblocks((int64_t)cnt * (bs / 4))),
                         dim3(kBlock), 0, st, d.small_all, cnt, d.troot, d.toff, d.sl, leaf, root, bs);
    else if (nv == 2)
      hipLaunchKernelGGL((k_det_small_all<T, OP, (sizeof(T) <= 8 ? 2 : 1)>), dim3(nblocks((int64_t)cnt * (bs / 2))),
                         dim3(kBlock), 0, st, d.small_all, cnt, d.troot, d.toff, d.sl, leaf, root, bs);
    else
      hipLaunchKernelGGL((k_det_small_all<T, OP, 1>), dim3(nblocks((int64_t)cnt * bs)), dim3(kBlock), 0, st,
                         d.small_all, cnt, d.troot, d.toff, d.sl, leaf, root, bs);
  }
  // chunk levels
  if (!h.levels.empty()) {
    for (size_t k = 0; k < h.levels.size(); k++) {
      const int nch = (int)h.levels[k].chunks.size();
      const T *src = k == 0 ? leaf : buf[(k - 1) % 2];
      const int32_t *sl = k == 0 ? d.sl : nullptr;
      hipLaunchKernelGGL((k_det_chunk<T, OP>), dim3(nblocks((int64_t)nch * 64)), dim3(kBlock), 0, st, d.levels[k], nch,
                         sl, src, buf[k % 2], root, bs);
    }
  }
  return check_launch();
}

template <typename T, int OP>
static int reduce_plain_t(sf_s *sf, const T *leaf, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  hipLaunchKernelGGL((k_reduce_plain<T, OP>), dim3((unsigned)sf->hp.tiles.size()), dim3(kBlock), 0, st, d.segs,
                     d.tiles, d.ridx, d.lidx, leaf, root, bs);
  return check_launch();
}

template <typename T, int OP>
static int reduce_atomic_t(sf_s *sf, const T *leaf, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const size_t ub = sizeof(T) * (size_t)bs;
  if (h.part_red_atomic && stage_class((int64_t)ub) >= 0 && scratch_fits(sf, part_scratch_need(sf, ub)))
    return launch_reduce_part<T, OP>(sf, leaf, root, bs, true, st);
  if (h.split && ub > kSplitMinUnit) return reduce_split_t<T, OP>(sf, leaf, root, bs, st);  // no atomics at all
  const int ntiles = (int)h.tiles.size();
  const AtomicShape sh = atomic_shape(sf, ntiles, bs * sizeof(T) + 4, kReduceGrid);
  const int32_t *ri = h.hot_roots.empty() ? d.ridx : d.ridx_hot;
  hipLaunchKernelGGL((k_reduce_atomic<T, OP>), dim3((unsigned)sh.grid), dim3(kBlock), sh.lds_bytes, st, d.segs,
                     d.tiles, ntiles, ri, d.lidx, d.hot_roots, sh.nhot_lds, leaf, root, bs);
  return check_launch();
}

static int reduce_maxloc_atomic(sf_s *sf, const Pair *leaf, Pair *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int T_ = (int)h.troot.size();
  void *s = nullptr;
  int rc = acquire_scratch(sf, (size_t)std::max(T_, 1) * bs * sizeof(double), &s);
  if (rc) return rc;
  double *saved = (double *)s;
  const unsigned g = (unsigned)h.tiles.size();
  hipLaunchKernelGGL(k_maxloc_save, dim3(nblocks((int64_t)T_ * bs)), dim3(kBlock), 0, st, d.troot, T_, root, saved, bs);
  hipLaunchKernelGGL((k_maxloc_stream<0>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx, d.lidx, leaf, root, bs);
  hipLaunchKernelGGL(k_maxloc_fix, dim3(nblocks((int64_t)T_ * bs)), dim3(kBlock), 0, st, d.troot, T_, root, saved, bs);
  hipLaunchKernelGGL((k_maxloc_stream<1>), dim3(g), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx, d.lidx, leaf, root, bs);
  return check_launch();
}

template <typename T>
static int reduce_t(sf_s *sf, int op, int mode, const void *leafv, void *rootv, int bs, hipStream_t st) {
  const T *leaf = (const T *)leafv;
  T *root = (T *)rootv;
  const bool dup = sf->has_dup_roots;
  if (op == SF_REPLACE) {
    if (!dup) return reduce_plain_t<T, OP_REPLACE>(sf, leaf, root, bs, st);
    return reduce_det_t<T, OP_REPLACE>(sf, leaf, root, bs, st);
  }
#define SF_RED(OPV)                                                        \
  do {                                                                     \
    if (!dup) return reduce_plain_t<T, OPV>(sf, leaf, root, bs, st);       \
    if (mode != SF_REDUCE_ATOMIC) return reduce_det_t<T, OPV>(sf, leaf, root, bs, st); \
    return reduce_atomic_t<T, OPV>(sf, leaf, root, bs, st);                \
  } while (0)
  switch (op) {
    case SF_SUM: SF_RED(OP_SUM);
    case SF_MAX: SF_RED(OP_MAX);
    case SF_MIN: SF_RED(OP_MIN);
    case SF_PROD:  // no native atomic multiply: deterministic in every mode
      if (!dup) return reduce_plain_t<T, OP_PROD>(sf, leaf, root, bs, st);
      return reduce_det_t<T, OP_PROD>(sf, leaf, root, bs, st);
    default: return SF_ERR_UNSUPPORTED;
  }
#undef SF_RED
}

// 16-bit floating-point units: no per-element 16-bit atomics, so every
// reduce mode takes the deterministic kernels.
template <typename T>
static int reduce_half_t(sf_s *sf, int op, const void *leafv, void *rootv, int bs, hipStream_t st) {
  const T *leaf = (const T *)leafv;
  T *root = (T *)rootv;
  const bool dup = sf->has_dup_roots;
#define SF_RED(OPV)                                                  \
  do {                                                               \
    if (!dup) return reduce_plain_t<T, OPV>(sf, leaf, root, bs, st); \
    return reduce_det_t<T, OPV>(sf, leaf, root, bs, st);             \
  } while (0)
  switch (op) {
    case SF_REPLACE: SF_RED(OP_REPLACE);
    case SF_SUM: SF_RED(OP_SUM);
    case SF_MAX: SF_RED(OP_MAX);
    case SF_MIN: SF_RED(OP_MIN);
    case SF_PROD: SF_RED(OP_PROD);
    default: return SF_ERR_UNSUPPORTED;
  }
#undef SF_RED
}

int launch_reduce(sf_s *sf, sf_unit unit, const void *leaf, void *root, int op, hipStream_t st) {
  if (sf->nleaves == 0) return SF_OK;
  if (op == SF_REPLACE && unit.dtype != SF_F64_I32 && sf->hp.all_contig && !sf->has_dup_roots)
    return copy_segments(sf, (int64_t)elem_size(unit.dtype) * unit.bs, root, (void *)leaf, 1, st);
  const int mode = sf->reduce_mode;
  switch (unit.dtype) {
    case SF_F64: return reduce_t<double>(sf, op, mode, leaf, root, unit.bs, st);
    case SF_F32: return reduce_t<float>(sf, op, mode, leaf, root, unit.bs, st);
    case SF_I32: return reduce_t<int32_t>(sf, op, mode, leaf, root, unit.bs, st);
    case SF_I64: return reduce_t<int64_t>(sf, op, mode, leaf, root, unit.bs, st);
    case SF_F16: return reduce_half_t<H16>(sf, op, leaf, root, unit.bs, st);
    case SF_BF16: return reduce_half_t<BF16>(sf, op, leaf, root, unit.bs, st);
    case SF_F64_I32: {
      const Pair *l = (const Pair *)leaf;
      Pair *r = (Pair *)root;
      if (op == SF_REPLACE) {
        if (!sf->has_dup_roots) return reduce_plain_t<Pair, OP_REPLACE>(sf, l, r, unit.bs, st);
        return reduce_det_t<Pair, OP_REPLACE>(sf, l, r, unit.bs, st);
      }
      if (op == SF_MINLOC) {  // no atomic form: deterministic in every mode
        if (!sf->has_dup_roots) return reduce_plain_t<Pair, OP_MINLOC>(sf, l, r, unit.bs, st);
        return reduce_det_t<Pair, OP_MINLOC>(sf, l, r, unit.bs, st);
      }
      if (op != SF_MAXLOC) return SF_ERR_UNSUPPORTED;
      if (!sf->has_dup_roots) return reduce_plain_t<Pair, OP_MAXLOC>(sf, l, r, unit.bs, st);
      if (mode == SF_REDUCE_ATOMIC && !(sf->hp.split && 16 * (size_t)unit.bs > kSplitMinUnit))
        return reduce_maxloc_atomic(sf, l, r, unit.bs, st);
      return reduce_det_t<Pair, OP_MAXLOC>(sf, l, r, unit.bs, st);
    }
    default: return SF_ERR_UNSUPPORTED;
  }
}

// ---------------------------------------------------------- FetchAndOp
template <typename T>
static int fop_atomic_t(sf_s *sf, T *root, const T *leaf, T *upd, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  if (h.part_fop_atomic && stage_class((int64_t)sizeof(T) * bs) >= 0) return launch_fop_part<T>(sf, root, leaf, upd, bs, true, st);
  const int ntiles = (int)h.tiles.size();
  if (!h.hot_roots.empty()) {
    const AtomicShape sh = atomic_shape(sf, ntiles, bs * sizeof(T) + 4, kFetchGrid);
    hipLaunchKernelGGL((k_fop_atomic_hot<T>), dim3((unsigned)sh.grid), dim3(kBlock), sh.lds_bytes, st, d.segs, d.tiles,
                       ntiles, d.ridx_hot, d.lidx, d.hot_roots, sh.nhot_lds, root, leaf, upd, bs);
  } else {
    hipLaunchKernelGGL((k_fop_atomic<T>), dim3((unsigned)ntiles), dim3(kBlock), 0, st, d.segs, d.tiles, d.ridx, d.lidx,
                       root, leaf, upd, bs);
  }
  return check_launch();
}

template <typename T>
static int fop_det_t(sf_s *sf, T *root, const T *leaf, T *upd, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  if (h.part && stage_class((int64_t)sizeof(T) * bs) >= 0) return launch_fop_part<T>(sf, root, leaf, upd, bs, false, st);
  // roots of degree <= kSmallMaxDeg: one launch over the degree classes
  // (concatenated class by class, so a wavefront's threads mostly share one)
  if (!h.small_all.empty())
    hipLaunchKernelGGL((k_fop_small<T>), dim3(nblocks((int64_t)h.small_all.size() * bs)), dim3(kBlock), 0, st,
                       d.small_all, (int)h.small_all.size(), d.troot, d.toff, d.sl, root, leaf, upd, bs);
  const int nch = (int)h.fo_chunks.size();
  const int nlarge = (int)h.large.size();
  if (nch) {
    void *s = nullptr;
    int rc = acquire_scratch(sf, (size_t)nch * bs * sizeof(T), &s);
    if (rc) return rc;
    T *sums = (T *)s;
    hipLaunchKernelGGL((k_fop_chunk_sum<T>), dim3(nblocks((int64_t)nch * 64)), dim3(kBlock), 0, st, d.fo_chunks, nch,
                       d.sl, leaf, sums, bs);
    hipLaunchKernelGGL((k_fop_root_scan<T>), dim3((unsigned)((nlarge * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       d.fo_root_first, nlarge, d.fo_chunks, sums, root, bs);
    hipLaunchKernelGGL((k_fop_chunk_apply<T>), dim3(nblocks((int64_t)nch * 64)), dim3(kBlock), 0, st, d.fo_chunks, nch,
                       d.sl, leaf, sums, upd, bs);
  }
  return check_launch();
}

int launch_fetch_and_op(sf_s *sf, sf_unit unit, void *root, const void *leaf, void *upd, int op, hipStream_t st,
                        bool fp_atomic) {
  if (op != SF_SUM) return SF_ERR_UNSUPPORTED;
  if (sf->nleaves == 0) return SF_OK;
  const bool is_int = unit.dtype == SF_I32 || unit.dtype == SF_I64;
  int mode = sf->reduce_mode;
  if (mode == SF_REDUCE_AUTO || (fp_atomic && !is_int)) mode = is_int ? SF_REDUCE_DETERMINISTIC : SF_REDUCE_ATOMIC;
  if (mode == SF_REDUCE_DETERMINISTIC && !is_int) return SF_ERR_UNSUPPORTED;
  switch (unit.dtype) {
    case SF_I32:
      return mode == SF_REDUCE_DETERMINISTIC
                 ? fop_det_t<int32_t>(sf, (int32_t *)root, (const int32_t *)leaf, (int32_t *)upd, unit.bs, st)
                 : fop_atomic_t<int32_t>(sf, (int32_t *)root, (const int32_t *)leaf, (int32_t *)upd, unit.bs, st);
    case SF_I64:
      return mode == SF_REDUCE_DETERMINISTIC
                 ? fop_det_t<int64_t>(sf, (int64_t *)root, (const int64_t *)leaf, (int64_t *)upd, unit.bs, st)
                 : fop_atomic_t<int64_t>(sf, (int64_t *)root, (const int64_t *)leaf, (int64_t *)upd, unit.bs, st);
    case SF_F64:
      return fop_atomic_t<double>(sf, (double *)root, (const double *)leaf, (double *)upd, unit.bs, st);
    case SF_F32:
      return fop_atomic_t<float>(sf, (float *)root, (const float *)leaf, (float *)upd, unit.bs, st);
    default: return SF_ERR_UNSUPPORTED;
  }
}

}  // namespace sfi
