// sf_multi.hip -- the multi-SF and the Gather / Scatter operations of
// Section 3.2, item 2.
//
// The multi-SF splits every root r of an SF into deg(r) new roots, one per
// leaf, and connects the leaves to them one by one.  It is built on the
// device as the paper describes: the degrees are a Reduce SUM of ones, the
// new roots of r start at the exclusive prefix of the degrees (a scan
// kernel), and a FetchAndOp SUM in leaf order with the roots starting there
// and every leaf adding 1 hands each leaf its new root.  The new graph is
// then set up like any SF (copied to the host: setup is host work).  Gather
// is a Reduce REPLACE on the multi-SF (each new root has exactly one leaf),
// Scatter a Bcast REPLACE.
#include <vector>

#include "sf_internal.h"

namespace sfi {

constexpr int kScanBlock = 1024;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kScanBlock * kScanPerThread;

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Exclusive prefix sum of x[0..n) in tiles of kScanTile: each block scans its
// tile (in[] -> out[]) and writes the tile's total to tot[block].
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                           int64_t n, int32_t *__restrict__ tot) {
  __shared__ int32_t wsum[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
  int32_t v[kScanPerThread];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPerThread; k++) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = s;
#pragma unroll
  for (int d = 1; d < 64; d *= 2) {
    const int o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wv; w++) before += wsum[w];
  int acc = before + inc - s;
#pragma unroll
  for (int k = 0; k < kScanPerThread; k++) {
    if (base + k < n) out[base + k] = acc;
    acc += v[k];
  }
  if (threadIdx.x == kScanBlock - 1) tot[blockIdx.x] = before + inc;
}

// Add the exclusive prefix of the tile totals to every tile (one block scans
// the at most kScanTile totals first).
__global__ __launch_bounds__(kScanBlock) void k_scan_add(int32_t *__restrict__ out, int64_t n,
                                                         const int32_t *__restrict__ tot, int ntiles) {
  __shared__ int32_t off;
  if (threadIdx.x == 0) {
    int32_t a = 0;
    for (int t = 0; t < (int)blockIdx.x && t < ntiles; t++) a += tot[t];
    off = a;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanBlock)
    if (base + k < n) out[base + k] += off;
}

static int hip_rc(hipError_t e) { return e == hipSuccess ? SF_OK : (e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e)); }

// Build sf->multi (the SF's lock is held).
static int build_multi(sf_s *sf) {
  const int64_t R = sf->nroots, L = sf->nleaves, LS = sf->leafspace;
  const int64_t ntiles = (R + kScanTile - 1) / kScanTile;
  if (ntiles > kScanTile) return SF_ERR_UNSUPPORTED;  // > 16M * 1024 roots
  int32_t *ones = nullptr, *deg = nullptr, *off = nullptr, *upd = nullptr, *tot = nullptr;
  const size_t ls = (size_t)std::max<int64_t>(LS, 1), rs = (size_t)std::max<int64_t>(R, 1);
  int rc = hip_rc(hipMalloc(&ones, ls * 4));
  if (!rc) rc = hip_rc(hipMalloc(&upd, ls * 4));
  if (!rc) rc = hip_rc(hipMalloc(&deg, rs * 4));
  if (!rc) rc = hip_rc(hipMalloc(&off, rs * 4));
  if (!rc) rc = hip_rc(hipMalloc(&tot, (size_t)std::max<int64_t>(ntiles, 1) * 4));
  std::vector<int32_t> h_upd;
  const hipStream_t st = nullptr;
  const sf_unit u{SF_I32, 1};
  if (!rc && L > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((LS + 255) / 256)), dim3(256), 0, st, ones, LS, 1);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, deg, R, 0);
    // degrees: Reduce SUM of ones (integer sums: exact in every mode)
    rc = launch_reduce(sf, u, ones, deg, SF_SUM, st);
    if (!rc && R > 0) {
      hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, deg, off, R, tot);
      hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, off, R, tot, (int)ntiles);
    }
    // new roots: FetchAndOp SUM in leaf order, roots from their offsets, leaves 1
    if (!rc) {
      const int32_t mode = sf->reduce_mode;
      sf->reduce_mode = SF_REDUCE_DETERMINISTIC;
      rc = launch_fetch_and_op(sf, u, off, ones, upd, SF_SUM, st);
      sf->reduce_mode = mode;
    }
    if (!rc) rc = hip_rc(hipGetLastError());
    if (!rc) {
      h_upd.resize((size_t)LS);
      rc = hip_rc(hipMemcpy(h_upd.data(), upd, (size_t)LS * 4, hipMemcpyDeviceToHost));
    }
  }
  (void)hipFree(ones);
  (void)hipFree(upd);
  (void)hipFree(deg);
  (void)hipFree(off);
  (void)hipFree(tot);
  if (rc) return rc;
  // the new graph: leaf i (slot l_i, same segment label) -> new root h_upd[l_i]
  std::vector<sf_node> nodes((size_t)L);
  std::vector<uint8_t> seen((size_t)L, 0);
  for (int64_t i = 0; i < L; i++) {
    const int64_t slot = sf->ilocal ? sf->ilocal[i] : i;
    const int64_t m = h_upd[(size_t)slot];
    if (m < 0 || m >= L || seen[(size_t)m]) return SF_ERR_HIP;  // not a permutation: the device work failed
    seen[(size_t)m] = 1;
    nodes[(size_t)i] = {sf->iremote[i].rank, m};
  }
  sf_t multi = nullptr;
  rc = sf_create(L, L, sf->ilocal, SF_COPY_VALUES, nodes.data(), SF_COPY_VALUES, &multi);
  if (rc) return rc;
  sf_setup_opts o{};
  o.reduce_mode = SF_REDUCE_AUTO;
  o.use_patterns = sf->opts.use_patterns;
  rc = sf_setup(multi, &o);
  if (rc) {
    sf_destroy(&multi);
    return rc;
  }
  sf->multi = multi;
  return SF_OK;
}

}  // namespace sfi

using namespace sfi;

extern "C" int sf_get_multi_sf(sf_t sf, sf_t *multi) {
  if (!sf || !multi) return SF_ERR_ARG;
  *multi = nullptr;
  std::lock_guard<std::mutex> g(sf->mu);
  if (!sf->setup) return SF_ERR_NOT_SETUP;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != sf->device) return SF_ERR_ARG;
  if (!sf->multi) {
    int rc = build_multi(sf);
    if (rc) return rc;
  }
  *multi = sf->multi;
  return SF_OK;
}
