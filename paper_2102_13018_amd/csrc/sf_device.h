// sf_device.h -- device-side element types, operations and index helpers
// shared by the star-forest kernels (single and batched).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "sf_internal.h"

namespace sfi {

// MAXLOC unit {double v; int32 i; int32 pad}: only v and i are touched.
struct Pair {
  double v;
  int32_t i;
  int32_t pad;
};

// binary16 and bfloat16 elements, held as their 16-bit patterns.  SUM and
// PROD compute in binary32 and round once to the format (round to nearest,
// ties to even): binary32's 24 bits are at least 2p + 2 for p = 11 and 8,
// so the binary32 rounding never changes the final one and the result is
// the exact one rounded once.  MAX / MIN compare 16-bit order keys.
struct H16 {
  uint16_t b;
};
struct BF16 {
  uint16_t b;
};
template <typename T>
constexpr bool kIsHalf = std::is_same<T, H16>::value || std::is_same<T, BF16>::value;

__device__ __forceinline__ float to_f32(H16 h) { return (float)__builtin_bit_cast(_Float16, h.b); }
__device__ __forceinline__ float to_f32(BF16 h) { return __uint_as_float((uint32_t)h.b << 16); }
// binary32 -> binary16 by the hardware conversion (round to nearest even)
__device__ __forceinline__ H16 from_f32(float x, H16) { return H16{__builtin_bit_cast(uint16_t, (_Float16)x)}; }
// binary32 -> bfloat16: add half an ulp of the kept part, minus one when the
// kept part is even, and truncate (round to nearest, ties to even; no NaN)
__device__ __forceinline__ BF16 from_f32(float x, BF16) {
  const uint32_t u = __float_as_uint(x);
  return BF16{(uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16)};
}
// order key of a sign-magnitude 16-bit pattern: -0 < +0
__device__ __forceinline__ uint32_t hkey(uint16_t b) { return b & 0x8000u ? (uint32_t)(uint16_t)~b : (uint32_t)b | 0x8000u; }

// Total-order key of a float / double: unsigned compare of the key orders
// the values with -0 < +0 (no NaN in the inputs).
__device__ __forceinline__ uint64_t fkey(double x) {
  const int64_t b = __double_as_longlong(x);
  return b < 0 ? ~(uint64_t)b : ((uint64_t)b | 0x8000000000000000ull);
}
__device__ __forceinline__ uint32_t fkey(float x) {
  const int32_t b = __float_as_int(x);
  return b < 0 ? ~(uint32_t)b : ((uint32_t)b | 0x80000000u);
}

// Inverse of fkey.
__device__ __forceinline__ double fkey_inv(uint64_t k) {
  return __longlong_as_double((long long)(k & 0x8000000000000000ull ? k & 0x7fffffffffffffffull : ~k));
}
__device__ __forceinline__ float fkey_inv(uint32_t k) {
  return __int_as_float((int)(k & 0x80000000u ? k & 0x7fffffffu : ~k));
}

enum OpCode {
  OP_REPLACE = SF_REPLACE,
  OP_SUM = SF_SUM,
  OP_MAX = SF_MAX,
  OP_MIN = SF_MIN,
  OP_MAXLOC = SF_MAXLOC,
  OP_MINLOC = SF_MINLOC,
  OP_PROD = SF_PROD
};
// Ops with a native device atomic on the scalar types (the others -- the
// location pairs and the product -- always combine through the
// deterministic kernels).
template <int OP>
constexpr bool kHasAtomic = OP == OP_SUM || OP == OP_MAX || OP == OP_MIN;

// a (left operand) op b
template <int OP, typename T>
struct Op;

template <int OP>
struct Op<OP, double> {
  static __device__ __forceinline__ double apply(double a, double b) {
    if (OP == OP_SUM) return a + b;
    if (OP == OP_PROD) return a * b;
    if (OP == OP_MAX) return fkey(a) < fkey(b) ? b : a;
    if (OP == OP_MIN) return fkey(b) < fkey(a) ? b : a;
    return b;
  }
};
template <int OP>
struct Op<OP, float> {
  static __device__ __forceinline__ float apply(float a, float b) {
    if (OP == OP_SUM) return a + b;
    if (OP == OP_PROD) return a * b;
    if (OP == OP_MAX) return fkey(a) < fkey(b) ? b : a;
    if (OP == OP_MIN) return fkey(b) < fkey(a) ? b : a;
    return b;
  }
};
template <int OP>
struct Op<OP, int32_t> {
  static __device__ __forceinline__ int32_t apply(int32_t a, int32_t b) {
    if (OP == OP_SUM) return (int32_t)((uint32_t)a + (uint32_t)b);
    if (OP == OP_PROD) return (int32_t)((uint32_t)a * (uint32_t)b);
    if (OP == OP_MAX) return a < b ? b : a;
    if (OP == OP_MIN) return b < a ? b : a;
    return b;
  }
};
template <int OP>
struct Op<OP, int64_t> {
  static __device__ __forceinline__ int64_t apply(int64_t a, int64_t b) {
    if (OP == OP_SUM) return (int64_t)((uint64_t)a + (uint64_t)b);
    if (OP == OP_PROD) return (int64_t)((uint64_t)a * (uint64_t)b);
    if (OP == OP_MAX) return a < b ? b : a;
    if (OP == OP_MIN) return b < a ? b : a;
    return b;
  }
};
// Unsigned keys (fkey of floating-point values): MAX / MIN only.
template <int OP>
struct Op<OP, uint64_t> {
  static __device__ __forceinline__ uint64_t apply(uint64_t a, uint64_t b) {
    if (OP == OP_MAX) return a < b ? b : a;
    return b < a ? b : a;
  }
};
template <int OP>
struct Op<OP, uint32_t> {
  static __device__ __forceinline__ uint32_t apply(uint32_t a, uint32_t b) {
    if (OP == OP_MAX) return a < b ? b : a;
    return b < a ? b : a;
  }
};
template <int OP, typename T>
struct OpHalf {
  static __device__ __forceinline__ T apply(T a, T b) {
    if (OP == OP_SUM) return from_f32(to_f32(a) + to_f32(b), T{});
    if (OP == OP_PROD) return from_f32(to_f32(a) * to_f32(b), T{});
    if (OP == OP_MAX) return hkey(a.b) < hkey(b.b) ? b : a;
    if (OP == OP_MIN) return hkey(b.b) < hkey(a.b) ? b : a;
    return b;
  }
};
template <int OP>
struct Op<OP, H16> : OpHalf<OP, H16> {};
template <int OP>
struct Op<OP, BF16> : OpHalf<OP, BF16> {};
template <int OP>
struct Op<OP, Pair> {
  static __device__ __forceinline__ Pair apply(Pair a, Pair b) {
    if (OP == OP_MAXLOC || OP == OP_MINLOC) {
      const uint64_t ka = fkey(a.v), kb = fkey(b.v);
      const bool better = (OP == OP_MAXLOC ? kb > ka : kb < ka) || (kb == ka && b.i < a.i);
      return better ? b : a;
    }
    return b;
  }
};

// Element loads / stores.  Pair stores never write the padding word.
template <typename T>
__device__ __forceinline__ T ld(const T *p) {
  return *p;
}
template <typename T>
__device__ __forceinline__ void st(T *p, T v) {
  *p = v;
}
template <>
__device__ __forceinline__ Pair ld<Pair>(const Pair *p) {
  Pair r;
  r.v = p->v;
  r.i = p->i;
  r.pad = 0;
  return r;
}
template <>
__device__ __forceinline__ void st<Pair>(Pair *p, Pair v) {
  p->v = v.v;
  p->i = v.i;
}

// Cross-lane move of an element (ds_bpermute based shuffles).
__device__ __forceinline__ double shfl_down(double v, int d) { return __shfl_down(v, d); }
__device__ __forceinline__ float shfl_down(float v, int d) { return __shfl_down(v, d); }
__device__ __forceinline__ int32_t shfl_down(int32_t v, int d) { return __shfl_down(v, d); }
__device__ __forceinline__ int64_t shfl_down(int64_t v, int d) {
  return (int64_t)__shfl_down((long long)v, d);
}
__device__ __forceinline__ Pair shfl_down(Pair v, int d) {
  Pair r;
  r.v = __shfl_down(v.v, d);
  r.i = __shfl_down(v.i, d);
  r.pad = 0;
  return r;
}
__device__ __forceinline__ H16 shfl_down(H16 v, int d) { return H16{(uint16_t)__shfl_down((int)v.b, d)}; }
__device__ __forceinline__ BF16 shfl_down(BF16 v, int d) { return BF16{(uint16_t)__shfl_down((int)v.b, d)}; }
__device__ __forceinline__ uint32_t shfl_down(uint32_t v, int d) { return (uint32_t)__shfl_down((int)v, d); }
__device__ __forceinline__ uint64_t shfl_down(uint64_t v, int d) {
  return (uint64_t)__shfl_down((long long)v, d);
}
__device__ __forceinline__ int32_t shfl_up(int32_t v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ int64_t shfl_up(int64_t v, int d) { return (int64_t)__shfl_up((long long)v, d); }
__device__ __forceinline__ double shfl_up(double v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ float shfl_up(float v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ int32_t shfl_idx(int32_t v, int l) { return __shfl(v, l); }
__device__ __forceinline__ int64_t shfl_idx(int64_t v, int l) { return (int64_t)__shfl((long long)v, l); }
__device__ __forceinline__ double shfl_idx(double v, int l) { return __shfl(v, l); }
__device__ __forceinline__ float shfl_idx(float v, int l) { return __shfl(v, l); }

// Streaming (non-temporal) accesses for data used once, so that it does not
// displace reused lines from the caches.  Values of 4, 8 and 16 bytes go
// through the native integer vector of that size (aligned to it in the
// buffers they stream), 2-byte values as one short.
template <int BYTES>
struct NtBytes;
template <>
struct NtBytes<2> {
  typedef unsigned short type;
};
template <>
struct NtBytes<4> {
  typedef unsigned int type;
};
template <>
struct NtBytes<8> {
  typedef unsigned int type __attribute__((ext_vector_type(2)));
};
template <>
struct NtBytes<16> {
  typedef unsigned int type __attribute__((ext_vector_type(4)));
};
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  using N = typename NtBytes<sizeof(T)>::type;
  const N v = __builtin_nontemporal_load(reinterpret_cast<const N *>(p));
  T r;
  __builtin_memcpy(&r, &v, sizeof(T));
  return r;
}
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) {
  using N = typename NtBytes<sizeof(T)>::type;
  N w;
  __builtin_memcpy(&w, &v, sizeof(T));
  __builtin_nontemporal_store(w, reinterpret_cast<N *>(p));
}

// Index of the t-th leaf of a segment side with a pattern (Section 5.2).
__device__ __forceinline__ int32_t pat_index(const DevPattern &p, int32_t t) {
  if (p.kind == SF_PATTERN_CONTIGUOUS) return p.start + t;
  // divisions by dx and dy as multiplications (magic numbers from the plan)
  const uint32_t ut = (uint32_t)t;
  const uint32_t q = p.mdx ? (uint32_t)__umul64hi(p.mdx, (uint64_t)ut) : ut;
  const uint32_t i = ut - q * (uint32_t)p.dx;
  const uint32_t k = p.mdy ? (uint32_t)__umul64hi(p.mdy, (uint64_t)q) : q;
  const uint32_t j = q - k * (uint32_t)p.dy;
  return p.start + (int32_t)i + p.sy * (int32_t)j + p.sz * (int32_t)k;
}

__device__ __forceinline__ int32_t seg_root(const DevSegment &s, const int32_t *__restrict__ ridx, int32_t t) {
  return s.root.kind == SF_PATTERN_GENERIC ? ridx[s.roff + t] : pat_index(s.root, t);
}
__device__ __forceinline__ int32_t seg_leaf(const DevSegment &s, const int32_t *__restrict__ lidx, int32_t t) {
  return s.leaf.kind == SF_PATTERN_GENERIC ? lidx[s.loff + t] : pat_index(s.leaf, t);
}
// The same, for index arrays read once per operation (streaming loads).
__device__ __forceinline__ int32_t seg_root_s(const DevSegment &s, const int32_t *__restrict__ ridx, int32_t t) {
  return s.root.kind == SF_PATTERN_GENERIC ? ld_stream(ridx + s.roff + t) : pat_index(s.root, t);
}
__device__ __forceinline__ int32_t seg_leaf_s(const DevSegment &s, const int32_t *__restrict__ lidx, int32_t t) {
  return s.leaf.kind == SF_PATTERN_GENERIC ? ld_stream(lidx + s.loff + t) : pat_index(s.leaf, t);
}

// ------------------------------------------------------------- atomics
// root (global memory) op= v, atomically, device scope.
template <int OP, typename T>
struct AtomicG;

template <int OP>
struct AtomicG<OP, double> {
  static __device__ __forceinline__ void run(double *p, double v) {
    if (OP == OP_SUM) {
      unsafeAtomicAdd(p, v);
    } else {
      // MAX/MIN under the total order through integer atomics on the bits:
      // for a non-negative v the signed order of the bit patterns is the
      // value order, for a negative v the unsigned order is reversed.
      // MIN mirrors it: signed min for v >= 0, unsigned max for v < 0.
      const int64_t b = __double_as_longlong(v);
      if (OP == OP_MAX) {
        if (b >= 0)
          __hip_atomic_fetch_max(reinterpret_cast<long long *>(p), (long long)b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(p), (unsigned long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (b >= 0)
          __hip_atomic_fetch_min(reinterpret_cast<long long *>(p), (long long)b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned long long *>(p), (unsigned long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
};
template <int OP>
struct AtomicG<OP, float> {
  static __device__ __forceinline__ void run(float *p, float v) {
    if (OP == OP_SUM) {
      unsafeAtomicAdd(p, v);
    } else {
      const int32_t b = __float_as_int(v);
      if (OP == OP_MAX) {
        if (b >= 0)
          __hip_atomic_fetch_max(reinterpret_cast<int *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned int *>(p), (unsigned int)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (b >= 0)
          __hip_atomic_fetch_min(reinterpret_cast<int *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned int *>(p), (unsigned int)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
};
template <int OP>
struct AtomicG<OP, int32_t> {
  static __device__ __forceinline__ void run(int32_t *p, int32_t v) {
    if (OP == OP_SUM)
      __hip_atomic_fetch_add(reinterpret_cast<unsigned int *>(p), (unsigned int)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (OP == OP_MAX)
      __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
template <int OP>
struct AtomicG<OP, int64_t> {
  static __device__ __forceinline__ void run(int64_t *p, int64_t v) {
    if (OP == OP_SUM)
      __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    else if (OP == OP_MAX)
      __hip_atomic_fetch_max(reinterpret_cast<long long *>(p), (long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_min(reinterpret_cast<long long *>(p), (long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Same operations on LDS (workgroup scope).
template <int OP, typename T>
struct AtomicL;

template <int OP>
struct AtomicL<OP, double> {
  static __device__ __forceinline__ void run(double *p, double v) {
    if (OP == OP_SUM) {
      __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      const int64_t b = __double_as_longlong(v);
      if (OP == OP_MAX) {
        if (b >= 0)
          __hip_atomic_fetch_max(reinterpret_cast<long long *>(p), (long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(p), (unsigned long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        if (b >= 0)
          __hip_atomic_fetch_min(reinterpret_cast<long long *>(p), (long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned long long *>(p), (unsigned long long)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
};
template <int OP>
struct AtomicL<OP, float> {
  static __device__ __forceinline__ void run(float *p, float v) {
    if (OP == OP_SUM) {
      __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      const int32_t b = __float_as_int(v);
      if (OP == OP_MAX) {
        if (b >= 0)
          __hip_atomic_fetch_max(reinterpret_cast<int *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_min(reinterpret_cast<unsigned int *>(p), (unsigned int)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        if (b >= 0)
          __hip_atomic_fetch_min(reinterpret_cast<int *>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          __hip_atomic_fetch_max(reinterpret_cast<unsigned int *>(p), (unsigned int)b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
};
template <int OP>
struct AtomicL<OP, int32_t> {
  static __device__ __forceinline__ void run(int32_t *p, int32_t v) {
    if (OP == OP_SUM)
      __hip_atomic_fetch_add(reinterpret_cast<unsigned int *>(p), (unsigned int)v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    else if (OP == OP_MAX)
      __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
template <int OP>
struct AtomicL<OP, int64_t> {
  static __device__ __forceinline__ void run(int64_t *p, int64_t v) {
    if (OP == OP_SUM)
      __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    else if (OP == OP_MAX)
      __hip_atomic_fetch_max(reinterpret_cast<long long *>(p), (long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      __hip_atomic_fetch_min(reinterpret_cast<long long *>(p), (long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Identity of an op on type T (start value of the LDS accumulators).
template <int OP, typename T>
__device__ __forceinline__ T op_identity() {
  if (OP == OP_SUM) return T(0);
  return T(0);
}
template <>
__device__ __forceinline__ double op_identity<OP_MAX, double>() {
  return -__builtin_huge_val();
}
template <>
__device__ __forceinline__ double op_identity<OP_MIN, double>() {
  return __builtin_huge_val();
}
template <>
__device__ __forceinline__ float op_identity<OP_MAX, float>() {
  return -__builtin_huge_valf();
}
template <>
__device__ __forceinline__ float op_identity<OP_MIN, float>() {
  return __builtin_huge_valf();
}
template <>
__device__ __forceinline__ int32_t op_identity<OP_MAX, int32_t>() {
  return INT32_MIN;
}
template <>
__device__ __forceinline__ int32_t op_identity<OP_MIN, int32_t>() {
  return INT32_MAX;
}
template <>
__device__ __forceinline__ int64_t op_identity<OP_MAX, int64_t>() {
  return INT64_MIN;
}
template <>
__device__ __forceinline__ int64_t op_identity<OP_MIN, int64_t>() {
  return INT64_MAX;
}

// Fetch-and-add returning the previous value (device scope).
__device__ __forceinline__ int32_t fetch_add_g(int32_t *p, int32_t v) {
  return (int32_t)__hip_atomic_fetch_add(reinterpret_cast<unsigned int *>(p), (unsigned int)v, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t fetch_add_g(int64_t *p, int64_t v) {
  return (int64_t)__hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch_add_g(double *p, double v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float fetch_add_g(float *p, float v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sfi

namespace sfi {
// a - b with two's-complement wrap-around.
__device__ __forceinline__ int32_t wrap_sub(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }
__device__ __forceinline__ int64_t wrap_sub(int64_t a, int64_t b) { return (int64_t)((uint64_t)a - (uint64_t)b); }
}  // namespace sfi

namespace sfi {
// Launchers of the partitioned path (sf_partition.hip), deterministic or
// with native atomics where chunks of one root meet, and
// its unit-size class (0: <= 8 bytes, 1: <= 16 bytes, -1: not staged).
int stage_class(int64_t unit_bytes);
size_t part_scratch_need(const sf_s *sf, size_t unit_bytes);
template <typename T, int OP>
int launch_reduce_part(sf_s *sf, const T *leaf, T *root, int bs, bool atomic, hipStream_t st);
template <typename T>
int launch_fop_part(sf_s *sf, T *root, const T *leaf, T *upd, int bs, bool atomic, hipStream_t st);
}  // namespace sfi

namespace sfi {
// NV consecutive elements of one unit, moved with one vector access.
template <typename T, int NV>
struct alignas(sizeof(T) * NV) Vec {
  T x[NV];
};
template <int OP, typename T, int NV>
__device__ __forceinline__ Vec<T, NV> vop(const Vec<T, NV> &a, const Vec<T, NV> &b) {
  Vec<T, NV> r;
#pragma unroll
  for (int i = 0; i < NV; i++) r.x[i] = Op<OP, T>::apply(a.x[i], b.x[i]);
  return r;
}
// The canonical pairwise tree (bottom-up form) of the n <= D values load(p),
// p = 0 .. n-1, combined by comb.  At most 8 values are live at once: a
// block of 8 consecutive positions is reduced by the levels at distance 1,
// 2 and 4 (whose pairs never leave the block), and the block results are
// combined at distances 8, 16, ... -- the same operands in the same order as
// the tree over all D positions, with a fraction of its registers (which
// keeps kernels with a 32-leaf class at a useful occupancy).
template <int D, typename V, typename Load, typename Comb>
__device__ __forceinline__ V pw_tree(int n, Load load, Comb comb) {
  constexpr int BMAX = sizeof(V) >= 16 ? 4 : 8;
  constexpr int B = D < BMAX ? D : BMAX;
  constexpr int NB = D / B;
  V blk[NB];
#pragma unroll
  for (int k = 0; k < NB; k++) {
    const int m = n - k * B;
    if (m > 0) {
      V x[B];
#pragma unroll
      for (int p = 0; p < B; p++)
        if (p < m) x[p] = load(k * B + p);
#pragma unroll
      for (int d = 1; d < B; d *= 2)
#pragma unroll
        for (int p = 0; p + d < B; p += 2 * d)
          if (p + d < m) x[p] = comb(x[p], x[p + d]);
      blk[k] = x[0];
    }
    if constexpr (NB > 1) __builtin_amdgcn_sched_barrier(0);  // one block's loads live at a time
  }
#pragma unroll
  for (int d = 1; d < NB; d *= 2)
#pragma unroll
    for (int p = 0; p + d < NB; p += 2 * d)
      if ((p + d) * B < n) blk[p] = comb(blk[p], blk[p + d]);
  return blk[0];
}

template <typename T, int NV>
__device__ __forceinline__ Vec<T, NV> vld(const T *p) {
  if constexpr (NV == 1) {
    Vec<T, 1> r;
    r.x[0] = ld(p);
    return r;
  } else {
    return *reinterpret_cast<const Vec<T, NV> *>(p);
  }
}
template <typename T, int NV>
__device__ __forceinline__ void vst(T *p, const Vec<T, NV> &v) {
  if constexpr (NV == 1)
    st(p, v.x[0]);
  else
    *reinterpret_cast<Vec<T, NV> *>(p) = v;
}
}  // namespace sfi
