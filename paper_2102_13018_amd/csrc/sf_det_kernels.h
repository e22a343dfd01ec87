// sf_det_kernels.h -- device kernels of the deterministic path used by
// both the direct and the partitioned launchers (templates: each
// translation unit instantiates what it launches).
#pragma once

#include "sf_device.h"

namespace sfi {

// One wavefront per aligned chunk of at most kChunk elements.  Lane l holds
// elements [l*LPT, (l+1)*LPT) of the chunk; the lane's block is reduced in
// registers, then lanes combine at distances 1, 2, ..., 32 -- all nodes of
// the canonical pairwise tree of the chunk.  Level 0 reads leaves through
// the sorted slot list; later levels read the previous level's results.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_det_chunk(const DevChunk *__restrict__ chunks, int nchunks,
                                                      const int32_t *__restrict__ sl, const T *__restrict__ src,
                                                      T *__restrict__ dst_seq, T *__restrict__ root, int bs) {
  constexpr int LPT = kChunkLPT;
  const int lane = threadIdx.x & 63;
  const int wid = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
  if (wid >= nchunks) return;
  const DevChunk ch = chunks[wid];
  int32_t idx[LPT];
#pragma unroll
  for (int s = 0; s < LPT; s++) {
    const int e = lane * LPT + s;
    idx[s] = e < ch.n ? (sl ? sl[ch.src + e] : ch.src + e) : 0;
  }
  const int m = ch.n - lane * LPT;  // valid elements of this lane (may be <= 0)
  for (int c = 0; c < bs; c++) {
    T x[LPT];
#pragma unroll
    for (int s = 0; s < LPT; s++)
      if (s < m) x[s] = ld(src + (int64_t)idx[s] * bs + c);
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
        st(dst_seq + (int64_t)ch.dst * bs + c, v);
      }
    }
  }
}

// Large roots, pass 2: one block per large root turns its chunk sums into
// chunk bases (root value + exclusive prefix) and writes the final root.
// Each iteration scans kBlock*4 chunk sums: 4 per thread in registers, the
// threads' totals across the wavefront with shuffles, the 4 wavefront totals
// through LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_root_scan(const int32_t *__restrict__ first, int nlarge,
                                                          const DevChunk *__restrict__ chunks, T *__restrict__ sums,
                                                          T *__restrict__ root, int bs) {
  __shared__ T wtot[kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x;
  if (k >= nlarge) return;
  const int c0 = first[k], c1 = first[k + 1];
  const int32_t r = chunks[c0].dst;
  for (int c = 0; c < bs; c++) {
    T carry = root[(int64_t)r * bs + c];
    for (int base = c0; base < c1; base += kBlock * 4) {
      T x[4];
      T s = T(0);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int i = base + threadIdx.x * 4 + j;
        x[j] = i < c1 ? sums[(int64_t)i * bs + c] : T(0);
        s = Op<OP_SUM, T>::apply(s, x[j]);
      }
      T inc = s;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o);
      }
      if (lane == 63) wtot[wv] = inc;
      __syncthreads();
      T before = carry;
      for (int w = 0; w < wv; w++) before = Op<OP_SUM, T>::apply(before, wtot[w]);
      T total = carry;
      for (int w = 0; w < kBlock / 64; w++) total = Op<OP_SUM, T>::apply(total, wtot[w]);
      T a = Op<OP_SUM, T>::apply(before, wrap_sub(inc, s));
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int i = base + threadIdx.x * 4 + j;
        if (i < c1) sums[(int64_t)i * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[j]);
      }
      carry = total;
      __syncthreads();
    }
    if (threadIdx.x == 0) root[(int64_t)r * bs + c] = carry;
  }
}

}  // namespace sfi
