// sf_api.cpp -- the C ABI of the star-forest library: creation and
// validation (PetscSFCreate + PetscSFSetGraph, Section 3.1), setup
// (PetscSFSetUp), begin/end pairs of Bcast / Reduce / FetchAndOp with their
// argument bookkeeping (Section 3.2), inspection and error strings.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>

#include "sf_internal.h"

using namespace sfi;

static bool valid_unit(sf_unit u) { return elem_size(u.dtype) > 0 && u.bs >= 1 && u.bs <= (1 << 20); }

static bool aligned(const void *p, int es) { return ((uintptr_t)p % (uintptr_t)std::min(es, 8)) == 0; }

extern "C" int sf_create(int64_t nroots, int64_t nleaves, const int64_t *ilocal, int32_t localmode,
                         const sf_node *iremote, int32_t remotemode, sf_t *out) {
  if (!out) return SF_ERR_ARG;
  *out = nullptr;
  if (localmode == SF_OWN_POINTER || remotemode == SF_OWN_POINTER) return SF_ERR_UNSUPPORTED;
  if ((localmode != SF_COPY_VALUES && localmode != SF_USE_POINTER) ||
      (remotemode != SF_COPY_VALUES && remotemode != SF_USE_POINTER))
    return SF_ERR_ARG;
  if (nroots < 0 || nleaves < 0 || nroots > INT32_MAX || nleaves > INT32_MAX) return SF_ERR_ARG;
  if (nleaves > 0 && !iremote) return SF_ERR_ARG;
  int64_t leafspace = nleaves;
  for (int64_t i = 0; i < nleaves; i++) {
    if (iremote[i].index < 0 || iremote[i].index >= nroots) return SF_ERR_ARG;
    if (ilocal) {
      if (ilocal[i] < 0 || ilocal[i] >= INT32_MAX) return SF_ERR_ARG;
      leafspace = std::max(leafspace, ilocal[i] + 1);
    }
  }
  if (ilocal) {
    leafspace = 0;
    for (int64_t i = 0; i < nleaves; i++) leafspace = std::max(leafspace, ilocal[i] + 1);
    // stars are disjoint: no two leaves may share a slot
    std::vector<uint8_t> seen((size_t)leafspace, 0);
    for (int64_t i = 0; i < nleaves; i++) {
      if (seen[ilocal[i]]) return SF_ERR_DUP_LEAF;
      seen[ilocal[i]] = 1;
    }
  }
  sf_s *sf = new (std::nothrow) sf_s();
  if (!sf) return SF_ERR_OOM;
  try {
    sf->nroots = nroots;
    sf->nleaves = nleaves;
    sf->leafspace = leafspace;
    if (ilocal) {
      if (localmode == SF_COPY_VALUES) {
        sf->ilocal_copy.assign(ilocal, ilocal + nleaves);
        sf->ilocal = sf->ilocal_copy.data();
      } else {
        sf->ilocal = ilocal;
      }
    }
    if (remotemode == SF_COPY_VALUES) {
      sf->iremote_copy.assign(iremote, iremote + nleaves);
      sf->iremote = sf->iremote_copy.data();
    } else {
      sf->iremote = iremote;
    }
  } catch (const std::bad_alloc &) {
    delete sf;
    return SF_ERR_OOM;
  }
  sf->opts.reduce_mode = SF_REDUCE_AUTO;
  sf->opts.use_patterns = 1;
  try {
    sf->pending.reserve(kMaxPending);
  } catch (const std::bad_alloc &) {
    delete sf;
    return SF_ERR_OOM;
  }
  *out = sf;
  return SF_OK;
}

extern "C" int sf_setup(sf_t sf, const sf_setup_opts *opts) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  sf_setup_opts o{};
  o.reduce_mode = SF_REDUCE_AUTO;
  o.use_patterns = 1;
  if (opts) o = *opts;
  if (o.reduce_mode < SF_REDUCE_AUTO || o.reduce_mode > SF_REDUCE_DETERMINISTIC) return SF_ERR_ARG;
  if (o.partition < 0 || o.partition > 2 || o.hot_path < 0 || o.hot_path > 2) return SF_ERR_ARG;
  sf->opts = o;
  sf->reduce_mode = o.reduce_mode;
  sf->setup = false;
  sf->generation++;
  if (sf->multi) sf_destroy(&sf->multi);  // built from the old plan
  sf->pending.clear();
  try {
    int rc = analyze(sf);
    if (rc) return rc;
  } catch (const std::bad_alloc &) {
    return SF_ERR_OOM;
  }
  if (o.analyze_only) {
    free_device(sf);
    return SF_OK;
  }
  int rc = upload(sf);
  if (rc) return rc;
  sf->setup = true;
  return SF_OK;
}

extern "C" int sf_set_reduce_mode(sf_t sf, int32_t mode) {
  if (!sf || mode < SF_REDUCE_AUTO || mode > SF_REDUCE_DETERMINISTIC) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  sf->reduce_mode = mode;
  return SF_OK;
}

// ---------------------------------------------------------- begin / end
static int begin_common(sf_t sf, int kind, sf_unit unit, int32_t op, const void *a, const void *b, const void *c) {
  if (!sf) return SF_ERR_ARG;
  if (!sf->setup) return SF_ERR_NOT_SETUP;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != sf->device) return SF_ERR_ARG;  // plan lives on sf->device
  if (!valid_unit(unit)) return SF_ERR_ARG;
  if (op < SF_REPLACE || op > SF_PROD) return SF_ERR_ARG;
  const bool loc = op == SF_MAXLOC || op == SF_MINLOC;
  if (loc && unit.dtype != SF_F64_I32) return SF_ERR_UNSUPPORTED;
  if (unit.dtype == SF_F64_I32 && !loc && op != SF_REPLACE) return SF_ERR_UNSUPPORTED;
  const int es = elem_size(unit.dtype);
  if (sf->nleaves > 0) {
    if (!a || !b || (kind == 2 && !c)) return SF_ERR_ARG;
    if (!aligned(a, es) || !aligned(b, es) || (c && !aligned(c, es))) return SF_ERR_ARG;
  }
  for (const Pending &p : sf->pending)
    if (p.kind == kind && p.a == a && p.b == b && p.c == c) return SF_ERR_BUSY;
  // SF_DEBUG=1: reject host memory (one pointer query per buffer; the
  // paper's Section 5.3 notes such a query costs about 0.3 us, so it is off
  // by default and the caller is trusted to pass device pointers)
  static const bool debug = getenv("SF_DEBUG") && atoi(getenv("SF_DEBUG")) > 0;
  if (debug && sf->nleaves > 0) {
    for (const void *ptr : {a, b, c}) {
      if (!ptr) continue;
      hipPointerAttribute_t at;
      if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return SF_ERR_ARG;
      }
    }
  }
  return SF_OK;
}

static int end_common(sf_t sf, int kind, sf_unit unit, int32_t op, const void *a, const void *b, const void *c) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  for (size_t k = 0; k < sf->pending.size(); k++) {
    const Pending &p = sf->pending[k];
    if (p.kind == kind && p.a == a && p.b == b && p.c == c) {
      if (p.dtype != unit.dtype || p.bs != unit.bs || p.op != op) return SF_ERR_MISMATCH;
      sf->pending.erase(sf->pending.begin() + (long)k);
      return SF_OK;
    }
  }
  return SF_ERR_MISMATCH;
}

static void push_pending(sf_t sf, int kind, sf_unit unit, int32_t op, const void *a, const void *b, const void *c) {
  sf->pending.push_back({kind, unit.dtype, unit.bs, op, a, b, c});
}

extern "C" int sf_bcast_begin(sf_t sf, sf_unit unit, const void *rootdata, void *leafdata, int32_t op,
                              hipStream_t stream) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  int rc = begin_common(sf, 0, unit, op, rootdata, leafdata, nullptr);
  if (rc) return rc;
  rc = launch_bcast(sf, unit, rootdata, leafdata, op, stream);
  if (rc) return rc;
  push_pending(sf, 0, unit, op, rootdata, leafdata, nullptr);
  return SF_OK;
}

extern "C" int sf_bcast_end(sf_t sf, sf_unit unit, const void *rootdata, void *leafdata, int32_t op,
                            hipStream_t stream) {
  (void)stream;
  return end_common(sf, 0, unit, op, rootdata, leafdata, nullptr);
}

extern "C" int sf_reduce_begin(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                               hipStream_t stream) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  int rc = begin_common(sf, 1, unit, op, rootdata, leafdata, nullptr);
  if (rc) return rc;
  rc = launch_reduce(sf, unit, leafdata, rootdata, op, stream);
  if (rc) return rc;
  push_pending(sf, 1, unit, op, rootdata, leafdata, nullptr);
  return SF_OK;
}

extern "C" int sf_reduce_begin_noalloc(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                                       hipStream_t stream) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  int rc = begin_common(sf, 1, unit, op, rootdata, leafdata, nullptr);
  if (rc) return rc;
  // the pending list has room reserved at creation: no host allocation
  if (sf->pending.size() >= sf->pending.capacity()) return SF_ERR_BUSY;
  void *p = nullptr;
  size_t cap = 0;
  rc = fixed_scratch(&p, &cap);
  if (rc) return rc;
  sf->fixed_scratch = p;
  sf->fixed_scratch_bytes = cap;
  rc = launch_reduce(sf, unit, leafdata, rootdata, op, stream);
  sf->fixed_scratch = nullptr;
  sf->fixed_scratch_bytes = 0;
  if (rc) return rc;
  push_pending(sf, 1, unit, op, rootdata, leafdata, nullptr);
  return SF_OK;
}

extern "C" int sf_reduce_end(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                             hipStream_t stream) {
  (void)stream;
  return end_common(sf, 1, unit, op, rootdata, leafdata, nullptr);
}

extern "C" int sf_fetch_and_op_begin(sf_t sf, sf_unit unit, void *rootdata, const void *leafdata, void *leafupdate,
                                     int32_t op, hipStream_t stream) {
  if (!sf) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  int rc = begin_common(sf, 2, unit, op, rootdata, leafdata, leafupdate);
  if (rc) return rc;
  if (unit.dtype == SF_F64_I32 || unit.dtype == SF_F16 || unit.dtype == SF_BF16 || op != SF_SUM)
    return SF_ERR_UNSUPPORTED;
  if (sf->nleaves > 0 && leafupdate == leafdata) return SF_ERR_ARG;
  rc = launch_fetch_and_op(sf, unit, rootdata, leafdata, leafupdate, op, stream);
  if (rc) return rc;
  push_pending(sf, 2, unit, op, rootdata, leafdata, leafupdate);
  return SF_OK;
}

extern "C" int sf_fetch_and_op_end(sf_t sf, sf_unit unit, void *rootdata, const void *leafdata, void *leafupdate,
                                   int32_t op, hipStream_t stream) {
  (void)stream;
  return end_common(sf, 2, unit, op, rootdata, leafdata, leafupdate);
}

// --------------------------------------------------- Gather / Scatter
// On the multi-SF (built on first use by sf_get_multi_sf): Gather is a
// Reduce REPLACE onto the new roots (one leaf each), Scatter a Bcast REPLACE.
// The pending pair is kept on the SF itself (kinds 3 and 4).
extern "C" int sf_gather_begin(sf_t sf, sf_unit unit, const void *leafdata, void *multirootdata,
                               hipStream_t stream) {
  sf_t m = nullptr;
  int rc = sf_get_multi_sf(sf, &m);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(sf->mu);
  rc = begin_common(sf, 3, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> gm(m->mu);
    rc = launch_reduce(m, unit, leafdata, multirootdata, SF_REPLACE, stream);
  }
  if (rc) return rc;
  push_pending(sf, 3, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
  return SF_OK;
}

extern "C" int sf_gather_end(sf_t sf, sf_unit unit, const void *leafdata, void *multirootdata, hipStream_t stream) {
  (void)stream;
  return end_common(sf, 3, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
}

extern "C" int sf_scatter_begin(sf_t sf, sf_unit unit, const void *multirootdata, void *leafdata,
                                hipStream_t stream) {
  sf_t m = nullptr;
  int rc = sf_get_multi_sf(sf, &m);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(sf->mu);
  rc = begin_common(sf, 4, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> gm(m->mu);
    rc = launch_bcast(m, unit, multirootdata, leafdata, SF_REPLACE, stream);
  }
  if (rc) return rc;
  push_pending(sf, 4, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
  return SF_OK;
}

extern "C" int sf_scatter_end(sf_t sf, sf_unit unit, const void *multirootdata, void *leafdata, hipStream_t stream) {
  (void)stream;
  return end_common(sf, 4, unit, SF_REPLACE, multirootdata, leafdata, nullptr);
}

// ------------------------------------------------------------ inspection
extern "C" int sf_get_info(sf_t sf, sf_info *info) {
  if (!sf || !info) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  std::memset(info, 0, sizeof(*info));
  info->nroots = sf->nroots;
  info->nleaves = sf->nleaves;
  info->leafspace = sf->leafspace;
  info->reduce_mode = sf->reduce_mode;
  if (!sf->analyzed) return SF_ERR_NOT_SETUP;
  info->nsegments = (int64_t)sf->segments.size();
  info->nroots_touched = (int64_t)sf->hp.troot.size();
  info->max_degree = sf->max_degree;
  info->has_dup_roots = sf->has_dup_roots ? 1 : 0;
  info->nhot = (int64_t)sf->hp.hot_roots.size();
  info->device_bytes = (int64_t)sf->dp.bytes;
  info->hot_roots = sf->hp.hot ? (int64_t)sf->hp.hx_root.size() : 0;
  return SF_OK;
}

extern "C" int sf_get_segment(sf_t sf, int64_t s, sf_segment_info *seg) {
  if (!sf || !seg) return SF_ERR_ARG;
  std::lock_guard<std::mutex> g(sf->mu);
  if (!sf->analyzed) return SF_ERR_NOT_SETUP;
  if (s < 0 || s >= (int64_t)sf->segments.size()) return SF_ERR_ARG;
  const Segment &S = sf->segments[(size_t)s];
  seg->rank = S.rank;
  seg->nleaves = (int64_t)S.members.size();
  seg->root = S.root;
  seg->leaf = S.leaf;
  return SF_OK;
}

extern "C" const char *sf_error_string(int code) {
  switch (code) {
    case SF_OK: return "success";
    case SF_ERR_ARG: return "invalid argument";
    case SF_ERR_DUP_LEAF: return "duplicate leaf slot (stars must be disjoint)";
    case SF_ERR_NOT_SETUP: return "star forest is not set up";
    case SF_ERR_UNSUPPORTED: return "unsupported unit / operation / mode";
    case SF_ERR_HIP: return "HIP runtime error";
    case SF_ERR_OOM: return "out of memory";
    case SF_ERR_MISMATCH: return "end does not match a pending begin";
    case SF_ERR_BUSY: return "the same operation on the same buffers is already pending";
    case SF_ERR_SCRATCH: return "the operation needs more scratch than the fixed buffer of the allocation-free call";
    default: return "unknown error";
  }
}

extern "C" int sf_destroy(sf_t *psf) {
  if (!psf) return SF_ERR_ARG;
  if (!*psf) return SF_OK;
  if ((*psf)->multi) sf_destroy(&(*psf)->multi);
  free_device(*psf);
  delete *psf;
  *psf = nullptr;
  return SF_OK;
}
