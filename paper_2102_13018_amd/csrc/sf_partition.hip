// sf_partition.hip -- the partitioned deterministic path of SFReduce and
// SFFetchAndOp for large star forests.
//
// The root-sorted order that the deterministic reduction needs visits the
// leaves at random; on a large leaf array every 8-byte leaf read then costs
// a whole cache line from the memory fabric.  Here the leaves are moved once
// into that order's neighbourhood instead:
//   pass A  moves every leaf unit into scratch; scratch is bucket-major and
//           inside a bucket keeps processing order, so one work tile owns
//           one contiguous run per bucket, which it writes with
//           consecutive lanes (its leaf reads stay inside the tile);
//   pass B  walks windows of the root-sorted order (whole small roots and
//           aligned kChunk-leaf chunks of large roots), reading the g-th
//           sorted leaf from scratch slot pp_src[g].  All slots of a window
//           lie in its bucket, and the windows of bucket b run on XCD
//           b % kXcd (work-group i is placed on XCD i % kXcd), so the reads
//           hit that XCD's L2.
// The trees are the same canonical pairwise trees as in the direct kernels,
// so results are bit-identical to them (and to the oracle).
// FetchAndOp adds: pass B leaves the fetched values in scratch (in place),
// and pass C streams them back to leafupdate in processing order.
#include <algorithm>

#include "sf_det_kernels.h"

namespace sfi {

// ---------------------------------------------------------------- pass A / C
// A work tile's leaves are visited in increasing scratch slot (pa_dst), so
// consecutive lanes write (pass A) or read (pass C) consecutive slots of a
// bucket run; the leaf side is addressed through the tile-local offset
// pa_loc, inside the tile's own leaf range.
// DIR 0 (pass A): scratch[slot] = leaf[l];  DIR 1 (pass C): leaf[l] = scratch[slot].
template <typename Word, int DIR>
__global__ __launch_bounds__(kBlock) void k_pp_move(const DevSegment *__restrict__ segs,
                                                    const DevTile *__restrict__ tiles,
                                                    const int32_t *__restrict__ lidx,
                                                    const int32_t *__restrict__ pa_dst,
                                                    const uint16_t *__restrict__ pa_loc, Word *__restrict__ leaf,
                                                    Word *__restrict__ scratch, int W, int stage) {
  extern __shared__ __align__(16) unsigned char smem[];
  Word *lds = reinterpret_cast<Word *>(smem);
  const DevTile tl = tiles[blockIdx.x];
  const DevSegment sg = segs[tl.seg];
  const int items = (tl.t1 - tl.t0) * W;
  const int64_t jbase = (int64_t)sg.pbase + tl.t0;
  if (stage && sg.leaf.kind == SF_PATTERN_CONTIGUOUS) {
    // the tile's leaf units are contiguous: move them whole through LDS,
    // so both the leaf side and the scratch side are coalesced
    const int64_t l0 = (int64_t)(sg.leaf.start + tl.t0) * W;
    if (DIR == 0) {
#pragma unroll 4
      for (int q = threadIdx.x; q < items; q += kBlock) lds[q] = leaf[l0 + q];
      __syncthreads();
#pragma unroll 4
      for (int q = threadIdx.x; q < items; q += kBlock) {
        const int jj = q / W;
        const int c = q - jj * W;
        scratch[(int64_t)pa_dst[jbase + jj] * W + c] = lds[(int)pa_loc[jbase + jj] * W + c];
      }
    } else {
#pragma unroll 4
      for (int q = threadIdx.x; q < items; q += kBlock) {
        const int jj = q / W;
        const int c = q - jj * W;
        lds[(int)pa_loc[jbase + jj] * W + c] = scratch[(int64_t)pa_dst[jbase + jj] * W + c];
      }
      __syncthreads();
#pragma unroll 4
      for (int q = threadIdx.x; q < items; q += kBlock) leaf[l0 + q] = lds[q];
    }
    return;
  }
  constexpr int U = 4;
  for (int q0 = threadIdx.x; q0 < items; q0 += kBlock * U) {
    Word v[U];
    int64_t to[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int q = q0 + u * kBlock;
      to[u] = -1;
      if (q < items) {
        const int jj = q / W;
        const int c = q - jj * W;
        const int64_t s = (int64_t)pa_dst[jbase + jj] * W + c;
        const int t = tl.t0 + (int)pa_loc[jbase + jj];
        const int64_t l = (int64_t)seg_leaf(sg, lidx, t) * W + c;
        if (DIR == 0) {
          v[u] = leaf[l];
          to[u] = s;
        } else {
          v[u] = scratch[s];
          to[u] = l;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (to[u] < 0) continue;
      if (DIR == 0)
        scratch[to[u]] = v[u];
      else
        leaf[to[u]] = v[u];
    }
  }
}

// Window of this work-group under the XCD schedule, or -1.
__device__ __forceinline__ int pp_window(const int32_t *__restrict__ sched, int jmax) {
  const int x = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  return j < jmax ? sched[x * jmax + j] : -1;
}

// Pairwise tree over n <= D values of one root (register array, unrolled).
template <typename T, int OP, int D>
__device__ __forceinline__ T small_tree(const T *__restrict__ scr, const int32_t *__restrict__ src, int g0, int n,
                                        int bs, int c) {
  T x[D];
#pragma unroll
  for (int p = 0; p < D; p++)
    if (p < n) x[p] = ld(scr + (int64_t)src[g0 + p] * bs + c);
#pragma unroll
  for (int d = 1; d < D; d *= 2)
#pragma unroll
    for (int p = 0; p + d < D; p += 2 * d)
      if (p + d < n) x[p] = Op<OP, T>::apply(x[p], x[p + d]);
  return x[0];
}

// ------------------------------------------------------------- pass B reduce
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_pp_reduce(const int32_t *__restrict__ sched, int jmax,
                                                      const DevWindow *__restrict__ wins,
                                                      const int32_t *__restrict__ small,
                                                      const int32_t *__restrict__ big,
                                                      const DevChunk *__restrict__ chunks0,
                                                      const int32_t *__restrict__ troot,
                                                      const int32_t *__restrict__ toff,
                                                      const int32_t *__restrict__ src, const T *__restrict__ scr,
                                                      T *__restrict__ lvl_out, T *__restrict__ root, int bs) {
  const int w = pp_window(sched, jmax);
  if (w < 0) return;
  const DevWindow win = wins[w];
  // whole roots of degree <= kSmallMaxDeg: one thread per (root, element)
  const int nsmall = (win.small1 - win.small0) * bs;
  for (int q = threadIdx.x; q < nsmall; q += kBlock) {
    const int k = q / bs, c = q % bs;
    const int t = small[win.small0 + k];
    const int g0 = toff[t];
    const int n = toff[t + 1] - g0;
    T v;
    if (n <= 1)
      v = small_tree<T, OP, 1>(scr, src, g0, n, bs, c);
    else if (n <= 2)
      v = small_tree<T, OP, 2>(scr, src, g0, n, bs, c);
    else if (n <= 4)
      v = small_tree<T, OP, 4>(scr, src, g0, n, bs, c);
    else if (n <= 8)
      v = small_tree<T, OP, 8>(scr, src, g0, n, bs, c);
    else if (n <= 16)
      v = small_tree<T, OP, 16>(scr, src, g0, n, bs, c);
    else
      v = small_tree<T, OP, 32>(scr, src, g0, n, bs, c);
    T *rp = root + (int64_t)troot[t] * bs + c;
    st(rp, Op<OP, T>::apply(ld(rp), v));
  }
  // aligned chunks of larger roots: one wavefront per chunk
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kBlock / 64) {
    const DevChunk ch = chunks0[big[ci]];
    int32_t idx[LPT];
#pragma unroll
    for (int s = 0; s < LPT; s++) {
      const int e = lane * LPT + s;
      idx[s] = e < ch.n ? src[ch.src + e] : 0;
    }
    const int m = ch.n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (s < m) x[s] = ld(scr + (int64_t)idx[s] * bs + c);
#pragma unroll
      for (int d = 1; d < LPT; d *= 2)
#pragma unroll
        for (int p = 0; p + d < LPT; p += 2 * d)
          if (p + d < m) x[p] = Op<OP, T>::apply(x[p], x[p + d]);
      T v = x[0];
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_down(v, d);
        if ((lane & (2 * d - 1)) == 0 && (lane + d) * LPT < ch.n) v = Op<OP, T>::apply(v, o);
      }
      if (lane == 0) {
        if (ch.dst < 0) {
          T *rp = root + (int64_t)(-ch.dst - 1) * bs + c;
          st(rp, Op<OP, T>::apply(ld(rp), v));
        } else {
          st(lvl_out + (int64_t)ch.dst * bs + c, v);
        }
      }
    }
  }
}

// ------------------------------------------------------- pass B FetchAndOp
// B1: small roots scan sequentially in leaf order, leaving the fetched
// values in scratch; chunks of large roots write their sums.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pp_fop_b1(const int32_t *__restrict__ sched, int jmax,
                                                      const DevWindow *__restrict__ wins,
                                                      const int32_t *__restrict__ small,
                                                      const int32_t *__restrict__ big,
                                                      const DevChunk *__restrict__ fo_chunks,
                                                      const int32_t *__restrict__ troot,
                                                      const int32_t *__restrict__ toff,
                                                      const int32_t *__restrict__ src, T *__restrict__ scr,
                                                      T *__restrict__ sums, T *__restrict__ root, int bs) {
  const int w = pp_window(sched, jmax);
  if (w < 0) return;
  const DevWindow win = wins[w];
  const int nsmall = (win.small1 - win.small0) * bs;
  for (int q = threadIdx.x; q < nsmall; q += kBlock) {
    const int k = q / bs, c = q % bs;
    const int t = small[win.small0 + k];
    const int g0 = toff[t], g1 = toff[t + 1];
    T *rp = root + (int64_t)troot[t] * bs + c;
    T a = *rp;
    for (int g = g0; g < g1; g++) {
      T *e = scr + (int64_t)src[g] * bs + c;
      const T v = *e;
      *e = a;
      a = Op<OP_SUM, T>::apply(a, v);
    }
    *rp = a;
  }
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kBlock / 64) {
    const int k = big[ci];
    const DevChunk ch = fo_chunks[k];
    for (int c = 0; c < bs; c++) {
      T a = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        const int e = lane * LPT + s;
        if (e < ch.n) a = Op<OP_SUM, T>::apply(a, scr[(int64_t)src[ch.src + e] * bs + c]);
      }
#pragma unroll
      for (int d = 32; d >= 1; d /= 2) a = Op<OP_SUM, T>::apply(a, shfl_down(a, d));
      if (lane == 0) sums[(int64_t)k * bs + c] = a;
    }
  }
}

// B3: chunks of large roots: exclusive prefix inside the chunk plus the
// chunk's base (from the root scan), written in place into scratch.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pp_fop_b3(const int32_t *__restrict__ sched, int jmax,
                                                      const DevWindow *__restrict__ wins,
                                                      const int32_t *__restrict__ big,
                                                      const DevChunk *__restrict__ fo_chunks,
                                                      const int32_t *__restrict__ src, T *__restrict__ scr,
                                                      const T *__restrict__ sums, int bs) {
  const int w = pp_window(sched, jmax);
  if (w < 0) return;
  const DevWindow win = wins[w];
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kBlock / 64) {
    const int k = big[ci];
    const DevChunk ch = fo_chunks[k];
    int64_t li[LPT];
#pragma unroll
    for (int s = 0; s < LPT; s++) {
      const int e = lane * LPT + s;
      li[s] = e < ch.n ? (int64_t)src[ch.src + e] : -1;
    }
    for (int c = 0; c < bs; c++) {
      T x[LPT];
      T lane_sum = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        x[s] = li[s] >= 0 ? scr[li[s] * bs + c] : T(0);
        lane_sum = Op<OP_SUM, T>::apply(lane_sum, x[s]);
      }
      T inc = lane_sum;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o);
      }
      T a = Op<OP_SUM, T>::apply(sums[(int64_t)k * bs + c], wrap_sub(inc, lane_sum));
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        if (li[s] >= 0) scr[li[s] * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[s]);
      }
    }
  }
}

// ================================================================ launchers
static int pp_check() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

// Move whole units between the leaf buffer and scratch (pass A / pass C).
static void pp_move(sf_s *sf, int dir, void *leaf, void *scratch, int64_t ub, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const unsigned g = (unsigned)sf->hp.tiles.size();
  const uintptr_t a = (uintptr_t)leaf | (uintptr_t)scratch;
  const size_t stage_bytes = (size_t)sf->hp.tile_leaves * (size_t)ub;
  const int stage = stage_bytes <= (size_t)kStageBytes ? 1 : 0;
  const size_t lds = stage ? stage_bytes : 0;
#define SF_PPM(WORD, WW)                                                                                         \
  do {                                                                                                           \
    if (dir == 0)                                                                                                \
      hipLaunchKernelGGL((k_pp_move<WORD, 0>), dim3(g), dim3(kBlock), lds, st, d.segs, d.tiles, d.lidx, d.pa_dst, \
                         d.pa_loc, (WORD *)leaf, (WORD *)scratch, (int)(WW), stage);                             \
    else                                                                                                         \
      hipLaunchKernelGGL((k_pp_move<WORD, 1>), dim3(g), dim3(kBlock), lds, st, d.segs, d.tiles, d.lidx, d.pa_dst, \
                         d.pa_loc, (WORD *)leaf, (WORD *)scratch, (int)(WW), stage);                             \
  } while (0)
  if (ub % 16 == 0 && a % 16 == 0)
    SF_PPM(uint4, ub / 16);
  else if (ub % 8 == 0 && a % 8 == 0)
    SF_PPM(uint2, ub / 8);
  else
    SF_PPM(uint32_t, ub / 4);
#undef SF_PPM
}

template <typename T, int OP>
int launch_reduce_part(sf_s *sf, const T *leaf, T *root, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int64_t L = sf->nleaves;
  const size_t ub = sizeof(T) * (size_t)bs;
  const size_t lvl = (size_t)std::max<int64_t>(h.scratch_len, 1) * ub;
  const size_t main_bytes = ((size_t)L * ub + 255) / 256 * 256;
  int rc = ensure_scratch(sf, main_bytes + 2 * lvl);
  if (rc) return rc;
  T *scr = (T *)sf->scratch;
  T *buf[2] = {(T *)((char *)sf->scratch + main_bytes), (T *)((char *)sf->scratch + main_bytes + lvl)};
  pp_move(sf, 0, (void *)leaf, scr, (int64_t)ub, st);
  const DevChunk *c0 = h.levels.empty() ? nullptr : d.levels[0];
  hipLaunchKernelGGL((k_pp_reduce<T, OP>), dim3((unsigned)(kXcd * h.pp_jmax)), dim3(kBlock), 0, st, d.pp_sched,
                     h.pp_jmax, d.pp_win, d.pp_small, d.pp_big, c0, d.troot, d.toff, d.pp_src, scr, buf[0], root, bs);
  for (size_t k = 1; k < h.levels.size(); k++) {
    const int nch = (int)h.levels[k].chunks.size();
    hipLaunchKernelGGL((k_det_chunk<T, OP>), dim3((unsigned)((nch * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, d.levels[k], nch, (const int32_t *)nullptr, (const T *)buf[(k - 1) % 2], buf[k % 2], root,
                       bs);
  }
  return pp_check();
}

template <typename T>
int launch_fop_part(sf_s *sf, T *root, const T *leaf, T *upd, int bs, hipStream_t st) {
  const DevPlan &d = sf->dp;
  const HostPlan &h = sf->hp;
  const int64_t L = sf->nleaves;
  const size_t ub = sizeof(T) * (size_t)bs;
  const int nch = (int)h.fo_chunks.size();
  const int nlarge = (int)h.large.size();
  const size_t main_bytes = ((size_t)L * ub + 255) / 256 * 256;
  int rc = ensure_scratch(sf, main_bytes + (size_t)std::max(nch, 1) * ub);
  if (rc) return rc;
  T *scr = (T *)sf->scratch;
  T *sums = (T *)((char *)sf->scratch + main_bytes);
  const unsigned gw = (unsigned)(kXcd * h.pp_jmax);
  pp_move(sf, 0, (void *)leaf, scr, (int64_t)ub, st);
  hipLaunchKernelGGL((k_pp_fop_b1<T>), dim3(gw), dim3(kBlock), 0, st, d.pp_sched, h.pp_jmax, d.pp_win, d.pp_small,
                     d.pp_big, d.fo_chunks, d.troot, d.toff, d.pp_src, scr, sums, root, bs);
  if (nch) {
    hipLaunchKernelGGL((k_fop_root_scan<T>), dim3(nlarge), dim3(kBlock), 0, st, d.fo_root_first, nlarge,
                       d.fo_chunks, sums, root, bs);
    hipLaunchKernelGGL((k_pp_fop_b3<T>), dim3(gw), dim3(kBlock), 0, st, d.pp_sched, h.pp_jmax, d.pp_win, d.pp_big,
                       d.fo_chunks, d.pp_src, scr, (const T *)sums, bs);
  }
  pp_move(sf, 1, (void *)upd, scr, (int64_t)ub, st);
  return pp_check();
}

template int launch_reduce_part<double, OP_SUM>(sf_s *, const double *, double *, int, hipStream_t);
template int launch_reduce_part<double, OP_MAX>(sf_s *, const double *, double *, int, hipStream_t);
template int launch_reduce_part<double, OP_MIN>(sf_s *, const double *, double *, int, hipStream_t);
template int launch_reduce_part<float, OP_SUM>(sf_s *, const float *, float *, int, hipStream_t);
template int launch_reduce_part<float, OP_MAX>(sf_s *, const float *, float *, int, hipStream_t);
template int launch_reduce_part<float, OP_MIN>(sf_s *, const float *, float *, int, hipStream_t);
template int launch_reduce_part<int32_t, OP_SUM>(sf_s *, const int32_t *, int32_t *, int, hipStream_t);
template int launch_reduce_part<int32_t, OP_MAX>(sf_s *, const int32_t *, int32_t *, int, hipStream_t);
template int launch_reduce_part<int32_t, OP_MIN>(sf_s *, const int32_t *, int32_t *, int, hipStream_t);
template int launch_reduce_part<int64_t, OP_SUM>(sf_s *, const int64_t *, int64_t *, int, hipStream_t);
template int launch_reduce_part<int64_t, OP_MAX>(sf_s *, const int64_t *, int64_t *, int, hipStream_t);
template int launch_reduce_part<int64_t, OP_MIN>(sf_s *, const int64_t *, int64_t *, int, hipStream_t);
template int launch_reduce_part<Pair, OP_MAXLOC>(sf_s *, const Pair *, Pair *, int, hipStream_t);
template int launch_fop_part<int32_t>(sf_s *, int32_t *, const int32_t *, int32_t *, int, hipStream_t);
template int launch_fop_part<int64_t>(sf_s *, int64_t *, const int64_t *, int64_t *, int, hipStream_t);

}  // namespace sfi
