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

// Large roots, pass 2: one wavefront per large root turns its chunk sums
// into chunk bases (root value + exclusive prefix) and writes the final
// root.  Each iteration scans 64*kScanPer chunk sums: kScanPer consecutive
// ones per lane in registers, the lane totals with shuffles.
constexpr int kScanPer = 8;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fop_root_scan(const int32_t *__restrict__ first, int nlarge,
                                                          const DevChunk *__restrict__ chunks, T *__restrict__ sums,
                                                          T *__restrict__ root, int bs) {
  const int lane = threadIdx.x & 63;
  const int k = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
  if (k >= nlarge) return;
  const int c0 = first[k], c1 = first[k + 1];
  const int32_t r = chunks[c0].dst;
  for (int c = 0; c < bs; c++) {
    T carry = root[(int64_t)r * bs + c];
    for (int base = c0; base < c1; base += 64 * kScanPer) {
      T x[kScanPer];
      T s = T(0);
#pragma unroll
      for (int j = 0; j < kScanPer; j++) {
        const int i = base + lane * kScanPer + j;
        x[j] = i < c1 ? sums[(int64_t)i * bs + c] : T(0);
        s = Op<OP_SUM, T>::apply(s, x[j]);
      }
      T inc = s;
#pragma unroll
      for (int d = 1; d < 64; d *= 2) {
        const T o = shfl_up(inc, d);
        if (lane >= d) inc = Op<OP_SUM, T>::apply(inc, o);
      }
      T a = Op<OP_SUM, T>::apply(carry, wrap_sub(inc, s));
#pragma unroll
      for (int j = 0; j < kScanPer; j++) {
        const int i = base + lane * kScanPer + j;
        if (i < c1) sums[(int64_t)i * bs + c] = a;
        a = Op<OP_SUM, T>::apply(a, x[j]);
      }
      carry = Op<OP_SUM, T>::apply(carry, __shfl(inc, 63));
    }
    if (lane == 0) root[(int64_t)r * bs + c] = carry;
  }
}

}  // namespace sfi
