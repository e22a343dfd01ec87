// sf_partition.hip -- the partitioned deterministic path of SFReduce and
// SFFetchAndOp for large star forests.
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
// The trees are the same as those of the direct kernels, so results are
// bit-identical to them (and to the oracle).  FetchAndOp writes the fetched
// values back into the window (pass B) and moves them to leafupdate with
// the reverse of pass A (pass C).
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "sf_det_kernels.h"

namespace sfi {

// ------------------------------------------------------------ pass A / C
// DIR 0 (pass A): scratch[slot] = leaf[l];  DIR 1 (pass C): leaf[l] = scratch[slot].
template <typename Word, int DIR>
__global__ __launch_bounds__(kStageThreads) void k_sp_move(const int32_t *__restrict__ pa_dst,
                                                           const uint16_t *__restrict__ pa_loc,
                                                           const int32_t *__restrict__ tile_leaf0,
                                                           const int32_t *__restrict__ pa_slot, int64_t L, int ta,
                                                           Word *__restrict__ leaf, Word *__restrict__ scratch,
                                                           int W) {
  extern __shared__ __align__(16) unsigned char smem[];
  Word *lds = reinterpret_cast<Word *>(smem);
  const int64_t p0 = (int64_t)blockIdx.x * ta;
  const int n = (int)min((int64_t)ta, L - p0);
  const int items = n * W;
  const int32_t leaf0 = tile_leaf0[blockIdx.x];
  if (leaf0 >= 0) {
    const int64_t l0 = (int64_t)leaf0 * W;
    if (DIR == 0) {
#pragma unroll 8
      for (int q = threadIdx.x; q < items; q += kStageThreads) lds[q] = leaf[l0 + q];
      __syncthreads();
#pragma unroll 8
      for (int q = threadIdx.x; q < items; q += kStageThreads) {
        const int jj = q / W;
        const int c = q - jj * W;
        scratch[(int64_t)pa_dst[p0 + jj] * W + c] = lds[(int)pa_loc[p0 + jj] * W + c];
      }
    } else {
#pragma unroll 8
      for (int q = threadIdx.x; q < items; q += kStageThreads) {
        const int jj = q / W;
        const int c = q - jj * W;
        lds[(int)pa_loc[p0 + jj] * W + c] = scratch[(int64_t)pa_dst[p0 + jj] * W + c];
      }
      __syncthreads();
#pragma unroll 8
      for (int q = threadIdx.x; q < items; q += kStageThreads) leaf[l0 + q] = lds[q];
    }
    return;
  }
  // slots not contiguous: the leaf side is gathered / scattered
#pragma unroll 4
  for (int q = threadIdx.x; q < items; q += kStageThreads) {
    const int jj = q / W;
    const int c = q - jj * W;
    const int64_t s = (int64_t)pa_dst[p0 + jj] * W + c;
    const int64_t l = (int64_t)pa_slot[p0 + pa_loc[p0 + jj]] * W + c;
    if (DIR == 0)
      scratch[s] = leaf[l];
    else
      leaf[l] = scratch[s];
  }
}

// Load one window from scratch into LDS in root-sorted order (LDS offset =
// sorted position - window start), and store it back.  Global accesses are
// coalesced; the permutation happens in LDS.
template <typename T>
__device__ __forceinline__ void win_load(T *lds, const T *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                         const DevSWin &w, int bs) {
  const T *src = scr + (int64_t)w.base * bs;
  if (bs == 1) {
#pragma unroll 8
    for (int q = threadIdx.x; q < w.n; q += kStageThreads) lds[lpos[w.base + q]] = src[q];
  } else {
    const int items = w.n * bs;
#pragma unroll 4
    for (int q = threadIdx.x; q < items; q += kStageThreads) {
      const int k = q / bs;
      lds[(int)lpos[w.base + k] * bs + (q - k * bs)] = src[q];
    }
  }
}
template <typename T>
__device__ __forceinline__ void win_store(const T *lds, T *__restrict__ scr, const uint16_t *__restrict__ lpos,
                                          const DevSWin &w, int bs) {
  T *dst = scr + (int64_t)w.base * bs;
  const int items = w.n * bs;
#pragma unroll 4
  for (int q = threadIdx.x; q < items; q += kStageThreads) {
    const int k = q / bs;
    dst[q] = lds[(int)lpos[w.base + k] * bs + (q - k * bs)];
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

// Root of level-0 chunk k and whether k is its root's first (bit 0) and
// last (bit 1) chunk, for the per-window runs of the atomic mode.
__device__ __forceinline__ void chunk_info(const DevChunk *__restrict__ fo, int k, int nfo, int32_t *cr,
                                           int32_t *cf) {
  const int32_t r = fo[k].dst;
  const int32_t prev = k > 0 ? fo[k - 1].dst : -1;
  const int32_t next = k + 1 < nfo ? fo[k + 1].dst : -1;
  *cr = r;
  *cf = (prev != r ? 1 : 0) | (next != r ? 2 : 0);
}

// ------------------------------------------------------------- pass B reduce
// ATOM: the chunk values of a root are combined per window (in chunk order,
// in LDS after the window's values, at element offset ctot_off, followed by
// each chunk's root and first/last flags); a root whose
// chunks all lie in this window is then updated plainly, one that spans
// windows through one native atomic per window, in arrival order, instead of
// the chunk-level trees.  fo (nfo chunks) gives each chunk's root.
template <typename T, int OP, bool ATOM>
__global__ __launch_bounds__(kStageThreads) void k_sp_reduce(const DevSWin *__restrict__ wins,
                                                             const int32_t *__restrict__ small,
                                                             const int32_t *__restrict__ big,
                                                             const DevChunk *__restrict__ chunks0,
                                                             const DevChunk *__restrict__ fo,
                                                             const int32_t *__restrict__ troot,
                                                             const int32_t *__restrict__ toff,
                                                             const uint16_t *__restrict__ lpos,
                                                             const T *__restrict__ scr, T *__restrict__ lvl_out,
                                                             T *__restrict__ root, int bs, int ctot_off, int nfo) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const DevSWin win = wins[blockIdx.x];
  win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  // whole roots of degree <= kSmallMaxDeg: one thread per (root, element),
  // U of them at a time so that their dependent index and root loads overlap
  const int nsmall = (win.small1 - win.small0) * bs;
  constexpr int U = 4;
  for (int q0 = threadIdx.x; q0 < nsmall; q0 += kStageThreads * U) {
    int t[U], o[U], n[U];
    int64_t rp[U];
    T rv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int q = q0 + u * kStageThreads;
      n[u] = 0;
      if (q < nsmall) {
        const int k = q / bs;
        t[u] = small[win.small0 + k];
        rp[u] = q - k * bs;  // element, completed below
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (q0 + u * kStageThreads < nsmall) {
        const int g0 = toff[t[u]];
        n[u] = toff[t[u] + 1] - g0;
        o[u] = g0 - win.g0;
        rp[u] += (int64_t)troot[t[u]] * bs;
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++)
      if (n[u] > 0) rv[u] = ld(root + rp[u]);
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (n[u] == 0) continue;
      const int c = (int)(rp[u] % bs);
      T v;
      if (n[u] <= 1)
        v = lds_tree<T, OP, 1>(lds, o[u], n[u], bs, c);
      else if (n[u] <= 2)
        v = lds_tree<T, OP, 2>(lds, o[u], n[u], bs, c);
      else if (n[u] <= 4)
        v = lds_tree<T, OP, 4>(lds, o[u], n[u], bs, c);
      else if (n[u] <= 8)
        v = lds_tree<T, OP, 8>(lds, o[u], n[u], bs, c);
      else if (n[u] <= 16)
        v = lds_tree<T, OP, 16>(lds, o[u], n[u], bs, c);
      else
        v = lds_tree<T, OP, 32>(lds, o[u], n[u], bs, c);
      st(root + rp[u], Op<OP, T>::apply(rv[u], v));
    }
  }
  // aligned chunks of larger roots: one wavefront per chunk, kChunkLPT per lane
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kStageThreads / 64) {
    const int k = big[ci];
    const DevChunk ch = chunks0[k];
    const int o = ch.src - win.g0 + lane * LPT;
    const int m = ch.n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (s < m) x[s] = ld(lds + (o + s) * bs + c);
#pragma unroll
      for (int d = 1; d < LPT; d *= 2)
#pragma unroll
        for (int p = 0; p + d < LPT; p += 2 * d)
          if (p + d < m) x[p] = Op<OP, T>::apply(x[p], x[p + d]);
      T v = x[0];
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o2 = shfl_down(v, d);
        if ((lane & (2 * d - 1)) == 0 && (lane + d) * LPT < ch.n) v = Op<OP, T>::apply(v, o2);
      }
      if (lane == 0) {
        if constexpr (ATOM) {
          lds[ctot_off + (ci - win.big0) * bs + c] = v;
          if (c == 0) {
            int32_t *cr = reinterpret_cast<int32_t *>(lds + ctot_off + (win.big1 - win.big0) * bs);
            chunk_info(fo, k, nfo, cr + (ci - win.big0), cr + (win.big1 - win.big0) + (ci - win.big0));
          }
        } else if (ch.dst < 0) {
          T *rp = root + (int64_t)(-ch.dst - 1) * bs + c;
          st(rp, Op<OP, T>::apply(ld(rp), v));
        } else {
          st(lvl_out + (int64_t)ch.dst * bs + c, v);
        }
      }
    }
  }
  if constexpr (ATOM) {
    __syncthreads();
    const T *ctot = lds + ctot_off;
    const int nb = win.big1 - win.big0;
    const int32_t *cr = reinterpret_cast<const int32_t *>(ctot + nb * bs);
    const int32_t *cf = cr + nb;
    for (int q = threadIdx.x; q < nb * bs; q += kStageThreads) {
      const int j = q / bs, c = q - j * bs;
      const int32_t r = cr[j];
      if (j > 0 && cr[j - 1] == r) continue;  // not the first chunk of its run
      T acc = ctot[j * bs + c];
      int j1 = j + 1;
      for (; j1 < nb && cr[j1] == r; j1++) acc = Op<OP, T>::apply(acc, ctot[j1 * bs + c]);
      const bool whole = (cf[j] & 1) && (cf[j1 - 1] & 2);
      T *rp = root + (int64_t)r * bs + c;
      if (whole)
        st(rp, Op<OP, T>::apply(ld(rp), acc));
      else
        AtomicG<OP, T>::run(rp, acc);
    }
  }
}

// ------------------------------------------------------- pass B FetchAndOp
// B1: small roots scan sequentially in leaf order (fetched values replace
// the leaf values in the window); chunks of large roots write their sums.
template <typename T>
__global__ __launch_bounds__(kStageThreads) void k_sp_fop_b1(const DevSWin *__restrict__ wins,
                                                             const int32_t *__restrict__ small,
                                                             const int32_t *__restrict__ big,
                                                             const DevChunk *__restrict__ fo_chunks,
                                                             const int32_t *__restrict__ troot,
                                                             const int32_t *__restrict__ toff,
                                                             const uint16_t *__restrict__ lpos, T *__restrict__ scr,
                                                             T *__restrict__ sums, T *__restrict__ root, int bs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const DevSWin win = wins[blockIdx.x];
  win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  const int nsmall = (win.small1 - win.small0) * bs;
  for (int q = threadIdx.x; q < nsmall; q += kStageThreads) {
    const int k = q / bs, c = q - (q / bs) * bs;
    const int t = small[win.small0 + k];
    const int o0 = toff[t] - win.g0, o1 = toff[t + 1] - win.g0;
    T *rp = root + (int64_t)troot[t] * bs + c;
    T a = *rp;
    for (int o = o0; o < o1; o++) {
      T *e = lds + o * bs + c;
      const T v = *e;
      *e = a;
      a = Op<OP_SUM, T>::apply(a, v);
    }
    *rp = a;
  }
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kStageThreads / 64) {
    const int k = big[ci];
    const DevChunk ch = fo_chunks[k];
    const int o = ch.src - win.g0 + lane * LPT;
    for (int c = 0; c < bs; c++) {
      T a = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (lane * LPT + s < ch.n) a = Op<OP_SUM, T>::apply(a, lds[(o + s) * bs + c]);
#pragma unroll
      for (int d = 32; d >= 1; d /= 2) a = Op<OP_SUM, T>::apply(a, shfl_down(a, d));
      if (lane == 0) sums[(int64_t)k * bs + c] = a;
    }
  }
  __syncthreads();
  if (win.small1 > win.small0) win_store(lds, scr, lpos, win, bs);
}

// B3: chunks of large roots: exclusive prefix inside the chunk plus the
// chunk's base (from the root scan), in the window, written back.
template <typename T>
__global__ __launch_bounds__(kStageThreads) void k_sp_fop_b3(const DevSWin *__restrict__ wins,
                                                             const int32_t *__restrict__ big,
                                                             const DevChunk *__restrict__ fo_chunks,
                                                             const uint16_t *__restrict__ lpos, T *__restrict__ scr,
                                                             const T *__restrict__ sums, int bs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  const DevSWin win = wins[blockIdx.x];
  if (win.big1 == win.big0) return;
  win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int ci = win.big0 + wv; ci < win.big1; ci += kStageThreads / 64) {
    const int k = big[ci];
    const DevChunk ch = fo_chunks[k];
    const int o = ch.src - win.g0 + lane * LPT;
    const int m = ch.n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
      T lane_sum = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        x[s] = s < m ? lds[(o + s) * bs + c] : T(0);
        lane_sum = Op<OP_SUM, T>::apply(lane_sum, x[s]);
      }
      T inc = lane_sum;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o2 = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o2);
      }
      T a = Op<OP_SUM, T>::apply(sums[(int64_t)k * bs + c], wrap_sub(inc, lane_sum));
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        if (s < m) lds[(o + s) * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[s]);
      }
    }
  }
  __syncthreads();
  win_store(lds, scr, lpos, win, bs);
}

// ------------------------------------------------- pass B FetchAndOp, atomic
// One pass: small roots scan in leaf order as in B1.  The chunks of a large
// root that lie in this window form a run: their totals (in LDS after the
// window's values, at element offset ctot_off, followed by each chunk's root
// and first/last flags) give every chunk its offset
// inside the run, and the run takes its base from the root -- plainly when
// the run is the whole root, else with one native returning atomic add, so
// the windows of a spanning root are applied in arrival order while the
// leaves inside a window keep leaf order.
template <typename T>
__global__ __launch_bounds__(kStageThreads) void k_sp_fop_atomic(const DevSWin *__restrict__ wins,
                                                                 const int32_t *__restrict__ small,
                                                                 const int32_t *__restrict__ big,
                                                                 const DevChunk *__restrict__ fo_chunks,
                                                                 const int32_t *__restrict__ troot,
                                                                 const int32_t *__restrict__ toff,
                                                                 const uint16_t *__restrict__ lpos,
                                                                 T *__restrict__ scr, T *__restrict__ root, int bs,
                                                                 int ctot_off, int nfo) {
  extern __shared__ __align__(16) unsigned char smem[];
  T *lds = reinterpret_cast<T *>(smem);
  T *ctot = lds + ctot_off;
  const DevSWin win = wins[blockIdx.x];
  win_load(lds, scr, lpos, win, bs);
  __syncthreads();
  const int nsmall = (win.small1 - win.small0) * bs;
  for (int q = threadIdx.x; q < nsmall; q += kStageThreads) {
    const int k = q / bs, c = q - (q / bs) * bs;
    const int t = small[win.small0 + k];
    const int o0 = toff[t] - win.g0, o1 = toff[t + 1] - win.g0;
    T *rp = root + (int64_t)troot[t] * bs + c;
    T a = *rp;
    for (int o = o0; o < o1; o++) {
      T *e = lds + o * bs + c;
      const T v = *e;
      *e = a;
      a = Op<OP_SUM, T>::apply(a, v);
    }
    *rp = a;
  }
  const int nb = win.big1 - win.big0;
  if (nb == 0) {
    __syncthreads();
    win_store(lds, scr, lpos, win, bs);
    return;
  }
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t *cr = reinterpret_cast<int32_t *>(ctot + nb * bs);
  int32_t *cf = cr + nb;
  // 1: chunk totals
  for (int j = wv; j < nb; j += kStageThreads / 64) {
    const int kk = big[win.big0 + j];
    const DevChunk ch = fo_chunks[kk];
    if (lane == 0) chunk_info(fo_chunks, kk, nfo, cr + j, cf + j);
    const int o = ch.src - win.g0 + lane * LPT;
    for (int c = 0; c < bs; c++) {
      T a = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++)
        if (lane * LPT + s < ch.n) a = Op<OP_SUM, T>::apply(a, lds[(o + s) * bs + c]);
#pragma unroll
      for (int d = 32; d >= 1; d /= 2) a = Op<OP_SUM, T>::apply(a, shfl_down(a, d));
      if (lane == 0) ctot[j * bs + c] = a;
    }
  }
  __syncthreads();
  // 2: per run, chunk offsets inside the run and the run's base from the root
  for (int q = threadIdx.x; q < nb * bs; q += kStageThreads) {
    const int j = q / bs, c = q - j * bs;
    const int32_t r = cr[j];
    if (j > 0 && cr[j - 1] == r) continue;  // not the first chunk of its run
    int j1 = j;
    T run = T(0);
    for (; j1 < nb && cr[j1] == r; j1++) {
      const T t = ctot[j1 * bs + c];
      ctot[j1 * bs + c] = run;
      run = Op<OP_SUM, T>::apply(run, t);
    }
    const bool whole = (cf[j] & 1) && (cf[j1 - 1] & 2);
    T *rp = root + (int64_t)r * bs + c;
    T base;
    if (whole) {
      base = *rp;
      *rp = Op<OP_SUM, T>::apply(base, run);
    } else {
      base = fetch_add_g(rp, run);
    }
    for (int jj = j; jj < j1; jj++) ctot[jj * bs + c] = Op<OP_SUM, T>::apply(base, ctot[jj * bs + c]);
  }
  __syncthreads();
  // 3: exclusive prefix inside each chunk plus the chunk's base
  for (int j = wv; j < nb; j += kStageThreads / 64) {
    const DevChunk ch = fo_chunks[big[win.big0 + j]];
    const int o = ch.src - win.g0 + lane * LPT;
    const int m = ch.n - lane * LPT;
    for (int c = 0; c < bs; c++) {
      T x[LPT];
      T lane_sum = T(0);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        x[s] = s < m ? lds[(o + s) * bs + c] : T(0);
        lane_sum = Op<OP_SUM, T>::apply(lane_sum, x[s]);
      }
      T inc = lane_sum;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o2 = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o2);
      }
      T excl = shfl_up(inc, 1);
      if (lane == 0) excl = T(0);
      T a = Op<OP_SUM, T>::apply(ctot[j * bs + c], excl);
#pragma unroll
      for (int s = 0; s < LPT; s++) {
        if (s < m) lds[(o + s) * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[s]);
      }
    }
  }
  __syncthreads();
  win_store(lds, scr, lpos, win, bs);
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
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void *, int>, size_t>> granted;
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(mu);
  for (auto &x : granted)
    if (x.first.first == fn && x.first.second == dev && x.second >= bytes) return SF_OK;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return set_hip_error(e);
  granted.push_back({{fn, dev}, bytes});
  return SF_OK;
}

int stage_class(int64_t unit_bytes) { return unit_bytes <= 8 ? 0 : (unit_bytes <= 16 ? 1 : -1); }

// Move whole units between the leaf buffer and scratch (pass A / pass C).
template <typename Word, int DIR>
static int sp_move_w(sf_s *sf, int cls, void *leaf, void *scratch, int W, hipStream_t st) {
  const HostPlan::Stage &hs = sf->hp.sp[cls];
  const DevPlan::Stage &ds = sf->dp.sp[cls];
  const unsigned g = (unsigned)hs.tile_leaf0.size();
  const size_t lds = (size_t)hs.ta * W * sizeof(Word);
  int rc = allow_lds((const void *)&k_sp_move<Word, DIR>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_sp_move<Word, DIR>), dim3(g), dim3(kStageThreads), lds, st, ds.pa_dst, ds.pa_loc,
                     ds.tile_leaf0, ds.pa_slot, (int64_t)sf->nleaves, hs.ta, (Word *)leaf, (Word *)scratch, W);
  return SF_OK;
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
  int rc = ensure_scratch(sf, main_bytes + 2 * lvl);
  if (rc) return rc;
  T *scr = (T *)sf->scratch;
  T *buf[2] = {(T *)((char *)sf->scratch + main_bytes), (T *)((char *)sf->scratch + main_bytes + lvl)};
  rc = sp_move(sf, cls, 0, (void *)leaf, scr, (int64_t)ub, st);
  if (rc) return rc;
  const size_t lds = (size_t)hs.cap * ub;
  const DevChunk *c0 = h.levels.empty() ? nullptr : d.levels[0];
  const int nfo = (int)h.fo_chunks.size();
  if constexpr (OP != OP_MAXLOC) {
    if (atomic) {
      const size_t lds_a = lds + (size_t)hs.maxbig * (ub + 8);
      rc = allow_lds((const void *)&k_sp_reduce<T, OP, true>, lds_a);
      if (rc) return rc;
      hipLaunchKernelGGL((k_sp_reduce<T, OP, true>), dim3((unsigned)hs.win.size()), dim3(kStageThreads), lds_a, st,
                         ds.win, ds.small, ds.big, c0, d.fo_chunks, d.troot, d.toff, ds.lpos, (const T *)scr, buf[0],
                         root, bs, hs.cap * bs, nfo);
      return sp_check();
    }
  }
  rc = allow_lds((const void *)&k_sp_reduce<T, OP, false>, lds);
  if (rc) return rc;
  hipLaunchKernelGGL((k_sp_reduce<T, OP, false>), dim3((unsigned)hs.win.size()), dim3(kStageThreads), lds, st, ds.win,
                     ds.small, ds.big, c0, d.fo_chunks, d.troot, d.toff, ds.lpos, (const T *)scr, buf[0], root, bs,
                     hs.cap * bs, nfo);
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
  const int nch = (int)h.fo_chunks.size();
  const int nlarge = (int)h.large.size();
  const size_t main_bytes = ((size_t)L * ub + 255) / 256 * 256;
  int rc = ensure_scratch(sf, main_bytes + (size_t)std::max(nch, 1) * ub);
  if (rc) return rc;
  T *scr = (T *)sf->scratch;
  T *sums = (T *)((char *)sf->scratch + main_bytes);
  const unsigned gw = (unsigned)hs.win.size();
  const size_t lds = (size_t)hs.cap * ub;
  rc = sp_move(sf, cls, 0, (void *)leaf, scr, (int64_t)ub, st);
  if (rc) return rc;
  if (atomic || !std::is_integral<T>::value) {  // floating point: atomic only
    const size_t lds_a = lds + (size_t)hs.maxbig * (ub + 8);
    if ((rc = allow_lds((const void *)&k_sp_fop_atomic<T>, lds_a))) return rc;
    hipLaunchKernelGGL((k_sp_fop_atomic<T>), dim3(gw), dim3(kStageThreads), lds_a, st, ds.win, ds.small, ds.big,
                       d.fo_chunks, d.troot, d.toff, ds.lpos, scr, root, bs, hs.cap * bs, nch);
    rc = sp_move(sf, cls, 1, (void *)upd, scr, (int64_t)ub, st);
    if (rc) return rc;
    return sp_check();
  }
  if constexpr (std::is_integral<T>::value) {
    if ((rc = allow_lds((const void *)&k_sp_fop_b1<T>, lds))) return rc;
    if ((rc = allow_lds((const void *)&k_sp_fop_b3<T>, lds))) return rc;
    hipLaunchKernelGGL((k_sp_fop_b1<T>), dim3(gw), dim3(kStageThreads), lds, st, ds.win, ds.small, ds.big,
                       d.fo_chunks, d.troot, d.toff, ds.lpos, scr, sums, root, bs);
    if (nch) {
      hipLaunchKernelGGL((k_fop_root_scan<T>), dim3((unsigned)((nlarge * 64 + kBlock - 1) / kBlock)), dim3(kBlock),
                         0, st, d.fo_root_first, nlarge, d.fo_chunks, sums, root, bs);
      hipLaunchKernelGGL((k_sp_fop_b3<T>), dim3(gw), dim3(kStageThreads), lds, st, ds.win, ds.big, d.fo_chunks,
                         ds.lpos, scr, (const T *)sums, bs);
    }
    rc = sp_move(sf, cls, 1, (void *)upd, scr, (int64_t)ub, st);
    if (rc) return rc;
    return sp_check();
  }
  return SF_ERR_UNSUPPORTED;  // deterministic FetchAndOp is defined for integers only
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
template int launch_reduce_part<Pair, OP_MAXLOC>(sf_s *, const Pair *, Pair *, int, bool, hipStream_t);
template int launch_fop_part<int32_t>(sf_s *, int32_t *, const int32_t *, int32_t *, int, bool, hipStream_t);
template int launch_fop_part<int64_t>(sf_s *, int64_t *, const int64_t *, int64_t *, int, bool, hipStream_t);
template int launch_fop_part<double>(sf_s *, double *, const double *, double *, int, bool, hipStream_t);
template int launch_fop_part<float>(sf_s *, float *, const float *, float *, int, bool, hipStream_t);

}  // namespace sfi
