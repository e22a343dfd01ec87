// sf_internal.h -- plan structures shared by the host runtime and the
// device kernels of the star-forest library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sf.h"

namespace sfi {

// ------------------------------------------------------------------ limits
constexpr int kBlock = 256;          // threads per block of the stream kernels
constexpr int kTileLeaves = 1024;    // largest work tile of the stream kernels (leaves)
constexpr int kTileMin = 256;        // smallest work tile
constexpr int kChunkLPT = 4;         // leaves per lane of the wave-chunk reduction
constexpr int kChunk = 64 * kChunkLPT;  // leaves per aligned chunk (power of two)
constexpr int kSmallMaxDeg = 32;     // largest degree of the per-thread classes
constexpr int kNumClasses = 6;       // degree classes 1, 2, 4, 8, 16, 32
constexpr int kHotMax = 8192;        // candidate roots for LDS aggregation on the atomic path
constexpr int kHotMinDeg = 64;       // smallest degree of such a candidate
constexpr int kHotLdsBytes = 32768;  // LDS budget for the accumulators, default
constexpr int kReduceGrid = 512;     // grid of the persistent atomic Reduce (measured best)
constexpr int kFetchGrid = 1024;     // grid of the persistent atomic FetchAndOp (measured best)
constexpr size_t kMaxPending = 64;   // pending begin/end pairs reserved per SF
constexpr size_t kSplitMinUnit = 8;  // the Reduce split is taken for larger units only (measured)
// Partitioned deterministic path for large SFs (two fully coalesced passes
// through a window-major scratch copy of the leaves):
constexpr int kStageThreads = 1024;      // threads per block of the staged kernels
constexpr int kStageMaxLds = 131072;     // LDS of one staged block (bytes)
// Automatic partitioning (SFs with repeated roots), from the crossovers
// measured on Zipf and uniform SFs: the plans are built from kPartitionPlan
// leaves, where the deterministic FetchAndOp already gains from them; the
// atomic Reduce uses them from kPartitionMid leaves, the deterministic Reduce
// from there when some root has chunk levels (degree > kSmallMaxDeg) and
// from kPartitionBig leaves otherwise, the atomic FetchAndOp from
// kPartitionBig leaves.
constexpr int64_t kPartitionPlan = 1 << 16;
constexpr int64_t kPartitionMid = 1 << 19;
constexpr int64_t kPartitionBig = 1 << 20;
// Hot roots of the partitioned path: at least this many leaves per pass-A
// tile on average (fewer and a group costs about what the windows cost),
// and at most kHotRootsMax of them.
constexpr int kHotPerTile = 2;
constexpr int kHotRootsMax = 4096;
constexpr int kPassATile = 8192;     // pass-A tile (processing positions), both unit-size classes

// --------------------------------------------------------- device structs
// Pattern of one side of a segment: index(t) = start + i + sy*j + sz*k with
// t = i + dx*(j + dy*k).  kind: SF_PATTERN_GENERIC / CONTIGUOUS / 3D.
struct DevPattern {
  int32_t kind, start, dx, dy, sy, sz;
  uint64_t mdx, mdy;  // ceil(2^64 / dx), ceil(2^64 / dy) (0 for 1): t / d = mulhi64(m, t) for t < 2^32
};

struct DevSegment {
  int32_t n;        // leaves in the segment
  int32_t roff;     // offset of the segment in the root-index array (generic root side)
  int32_t loff;     // offset of the segment in the leaf-slot array (generic leaf side)
  int32_t pbase;    // processing position of the segment's first leaf
  DevPattern root;
  DevPattern leaf;
};

struct DevTile {  // leaves [t0, t1) of segment seg
  int32_t seg, t0, t1, pad;
};

struct DevSWin {  // one window of the partitioned path
  int32_t base, n;         // its units in scratch: [base, base + n)
  int32_t small0, small1;  // range in the small-root item list
  int32_t big0, big1;      // range in the chunk item list
  int32_t g0;              // its first position in the root-sorted order
  int32_t pad;
};

struct DevChunk {  // one aligned chunk of a root's (sorted) value list
  int32_t src;  // first element in the level's input sequence
  int32_t n;    // elements, 1..kChunk
  int32_t dst;  // >= 0: slot in the next level's sequence; < 0: final, root = -dst-1
  int32_t pad;
};

struct DevSRoot {  // a whole root of a window of the partitioned path
  int32_t root;     // its index
  int32_t on;       // window-relative offset of its first sorted leaf | degree << 16
};

struct DevWChunk {  // a level-0 chunk of a large root, as placed in a window
  int32_t onf;      // window-relative offset | (n - 1) << 16 | first-of-root << 24 | last-of-root << 25
  int32_t dst;      // level-0 destination: >= 0 next-level slot; < 0 final, root = -dst-1
  int32_t root;     // the chunk's root
  int32_t k;        // level-0 chunk ordinal (FetchAndOp chunk sums)
};

// ------------------------------------------------------------- host plan
struct Segment {
  int64_t rank;
  std::vector<int64_t> members;  // leaf indices, ascending
  sf_pattern root{}, leaf{};
};

struct ChunkLevel {
  std::vector<DevChunk> chunks;
  int64_t out_len = 0;  // length of the sequence this level writes
};

struct HostPlan {
  // segments and tiles of the stream kernels
  std::vector<DevSegment> dsegs;
  std::vector<DevTile> tiles;
  int32_t tile_leaves = kTileLeaves;  // leaves per tile of this SF
  bool all_contig = false;            // every segment contiguous on both sides (few segments)
  std::vector<int32_t> ridx;      // root index per processed leaf (generic root sides)
  std::vector<int32_t> ridx_hot;  // same, hot roots encoded as -(h+1)
  std::vector<int32_t> lidx;      // leaf slot per processed leaf (generic leaf sides)
  std::vector<int32_t> hot_roots; // root id of hot slot h, by decreasing degree
  std::vector<int64_t> hot_deg;   // degree of hot slot h
  // root-sorted lists
  std::vector<int32_t> troot;     // touched roots, ascending
  std::vector<int32_t> toff;      // [ntouched+1] offsets into sl
  std::vector<int32_t> sl;        // leaf slot of the g-th leaf in (root, leaf) order
  std::vector<int32_t> cls[kNumClasses];  // touched-root ordinals per degree class
  std::vector<int32_t> large;     // touched-root ordinals with degree > kSmallMaxDeg
  std::vector<int32_t> small_all; // the degree classes concatenated, class by class
  std::vector<ChunkLevel> levels; // chunk levels of the large roots
  int64_t scratch_len = 0;        // max sequence length written by a chunk level
  // Reduce split for SFs whose repeated roots all have at most kSmallMaxDeg
  // leaves and hold under half of the leaves: the leaves of single-leaf roots
  // stream (index or pattern) and update their roots plainly, the repeated
  // roots take the register trees -- in one launch
  // (taken for units of more than kSplitMinUnit bytes: on the 256^3 halo the
  // leaf-order root updates of 8-byte units were slower than the root-sorted
  // trees, 10.1 vs 7.4 us, and faster for 24-byte units, 11.6 vs 12.1 us)
  bool split = false;
  std::vector<uint32_t> rep_bits;  // [ceil(L / 32)] bit p: processing position p has a repeated root
  std::vector<int32_t> rep_list;   // touched-root ordinals of the repeated roots, degree class by class
  // FetchAndOp on large roots: level-0 chunks, and per large root its chunk range
  std::vector<DevChunk> fo_chunks;
  std::vector<int32_t> fo_root_first;  // [nlarge+1] first chunk of each large root
  // Hot roots of the partitioned path: roots with at least kHotPerTile leaves
  // per pass-A tile on average.  Their leaves stay in leaf order: pass A
  // combines each tile's leaves of one hot root (a "group": one per tile and
  // hot root present) into one value, a scan kernel combines the groups of a
  // root in tile order, and FetchAndOp's pass C gives every hot leaf its
  // group's base plus its exclusive prefix inside the group.  Cold roots take
  // the windows, which are packed cold roots first: windows [0, wcold) of a
  // stage hold no hot root.
  bool hot = false;                 // the hot path is planned
  std::vector<int32_t> hx_root;     // [H] root id of hot root h
  std::vector<uint16_t> hx_pos;     // per hot entry, tile-major, grouped by hot root, in leaf order inside a
                                    //   group: tile offset (13 bits) | 0x8000 at a group's first entry
  std::vector<int32_t> hx_e0;       // [ntiles + 1] first hot entry of each pass-A tile
  std::vector<int32_t> hx_grp0;     // [ntiles + 1] first group of each pass-A tile
  std::vector<int32_t> hx_rfirst;   // [H + 1] first group of each hot root in root-major order
  std::vector<int32_t> hx_rpos;     // per group (tile-major): its index in root-major order (tile order
                                    //   inside a root); group values are stored root-major
  std::vector<uint16_t> hx_tg;      // [ntiles * kStageThreads] groups that start before the first entry of each
                                    //   thread of a tile's hot phase (thread t takes K = ceil(entries /
                                    //   kStageThreads) consecutive entries from t * K)
  int32_t hx_maxgrp = 0;            // most groups of a hot root
  // partitioned deterministic path: one plan per unit-size class
  // (class 0: units of <= 8 bytes, class 1: units of 9..16 bytes)
  bool part = false;  // the partition plans are built (the deterministic FetchAndOp uses them)
  bool part_red_det = false, part_red_atomic = false, part_fop_atomic = false;  // ... these ops too
  struct Stage {
    int32_t ta = 0, cap = 0;          // pass-A tile and window capacity, in units
    int32_t maxbig = 0;               // most level-0 chunks in one window
    int32_t maxrun = 0;               // most slot runs in one pass-A tile
    int32_t wcold = 0;                // windows [0, wcold) hold only cold roots (all, without a hot path)
    int32_t nspan_cold = 0;           // spanning roots in those windows (listed first)
    std::vector<DevSWin> win;
    std::vector<DevSRoot> sroot;      // whole roots, window-major (by degree class inside a window)
    std::vector<DevWChunk> wchunk;    // chunks of large roots, window-major, in chunk order
    std::vector<uint16_t> lpos;       // [L] by scratch slot: sorted position minus window start (< 2^14)
    std::vector<uint16_t> pa_loc;     // [L] pass-A tile-major, by increasing scratch slot in a tile: the
                                      //     tile-local processing offset of that leaf (13 bits) | 0x8000 at
                                      //     a run start | 0x2000 if the slot lies in a run of a cold root that
                                      //     spans windows | 0x4000 if that run continues into the next;
                                      //     0x4000 without 0x2000: the leaf of a hot root
    std::vector<int32_t> pa_run;      // per run of consecutive slots: first slot minus its tile position
    std::vector<int32_t> pa_run0;     // [ntiles + 1] first run of each tile
    std::vector<int32_t> pa_runw;     // per run: its window
    // roots whose chunks span windows: their runs (2 * window + which) in window order
    std::vector<int32_t> span_first;  // [nspan + 1]
    std::vector<int32_t> span_slot;
    std::vector<int32_t> span_root;   // [nspan]
    std::vector<int32_t> tile_leaf0;  // [ntiles] first slot if the tile's slots are contiguous, else -1
    std::vector<int32_t> pa_slot;     // [L] slot per processing position (only if some tile is not contiguous)
  } sp[2];
};

// Device copy of the plan: one allocation, typed views into it.
struct DevPlan {
  void *blob = nullptr;
  size_t bytes = 0;
  DevSegment *segs = nullptr;
  DevTile *tiles = nullptr;
  int32_t *ridx = nullptr, *ridx_hot = nullptr, *lidx = nullptr, *hot_roots = nullptr;
  int32_t *troot = nullptr, *toff = nullptr, *sl = nullptr;
  int32_t *cls[kNumClasses] = {};
  int32_t *large = nullptr;
  int32_t *small_all = nullptr;
  std::vector<DevChunk *> levels;
  DevChunk *fo_chunks = nullptr;
  int32_t *fo_root_first = nullptr;
  struct Stage {
    DevSWin *win = nullptr;
    DevSRoot *sroot = nullptr;
    DevWChunk *wchunk = nullptr;
    int32_t *pa_run = nullptr, *pa_run0 = nullptr, *tile_leaf0 = nullptr, *pa_slot = nullptr;
    int32_t *pa_runw = nullptr, *span_first = nullptr, *span_slot = nullptr, *span_root = nullptr;
    uint16_t *lpos = nullptr, *pa_loc = nullptr;
  } sp[2];
  uint32_t *rep_bits = nullptr;
  int32_t *rep_list = nullptr;
  int32_t *hx_root = nullptr, *hx_e0 = nullptr, *hx_grp0 = nullptr, *hx_rfirst = nullptr, *hx_rpos = nullptr;
  uint16_t *hx_pos = nullptr, *hx_tg = nullptr;
};

struct Pending {
  int kind;  // 0 bcast, 1 reduce, 2 fetch-and-op
  int32_t dtype, bs, op;
  const void *a, *b, *c;
};

}  // namespace sfi

struct sf_s {
  int64_t nroots = 0, nleaves = 0, leafspace = 0;
  const int64_t *ilocal = nullptr;  // borrowed or owned copy (may be null)
  const sf_node *iremote = nullptr;
  std::vector<int64_t> ilocal_copy;
  std::vector<sf_node> iremote_copy;
  bool setup = false;
  bool analyzed = false;
  uint64_t generation = 0;  // incremented by every sf_setup (device plans of earlier ones are freed)
  sf_s *multi = nullptr;    // the multi-SF (Section 3.2, item 2), built on first use; owned
  sf_setup_opts opts{};
  int32_t reduce_mode = SF_REDUCE_AUTO;
  // analysis results
  std::vector<sfi::Segment> segments;
  sfi::HostPlan hp;
  int64_t max_degree = 0;
  bool has_dup_roots = false;
  int device = -1;
  sfi::DevPlan dp;
  // scratch for chunk levels / MAXLOC passes / the partitioned path, grown on
  // demand; outgrown buffers are kept (retired) until the device plan is
  // freed, so that work already enqueued or captured into a graph that uses
  // them stays valid
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  std::vector<void *> retired;
  // set only for the duration of an allocation-free call: scratch comes from
  // this fixed device buffer (one per device) and nothing is allocated
  void *fixed_scratch = nullptr;
  size_t fixed_scratch_bytes = 0;
  std::vector<sfi::Pending> pending;
  std::mutex mu;
};

namespace sfi {
// helpers implemented in sf_plan.cpp
int analyze(sf_s *sf);
sf_pattern detect_pattern(const int64_t *idx, int64_t n);
int upload(sf_s *sf);
void free_device(sf_s *sf);
int set_hip_error(hipError_t e);
int ensure_scratch(sf_s *sf, size_t bytes);
// Scratch of at least `bytes` for the operation being enqueued: the fixed
// buffer during an allocation-free call (SF_ERR_SCRATCH when it is too
// small), else the SF's own buffer, grown with ensure_scratch.
int acquire_scratch(sf_s *sf, size_t bytes, void **out);
// Whether `bytes` of scratch can be had without failing: always, unless an
// allocation-free call is in progress and the fixed buffer is smaller.
inline bool scratch_fits(const sf_s *sf, size_t bytes) {
  return sf->fixed_scratch == nullptr || bytes <= sf->fixed_scratch_bytes;
}
// Device address and size of the calling device's fixed scratch buffer
// (implemented in sf_noalloc.hip).
int fixed_scratch(void **ptr, size_t *bytes);

// kernel launchers implemented in sf_kernels.hip
int launch_bcast(sf_s *sf, sf_unit unit, const void *root, void *leaf, int op, hipStream_t st);
int launch_reduce(sf_s *sf, sf_unit unit, const void *leaf, void *root, int op, hipStream_t st);
// fp_atomic: floating-point units take atomics even in DETERMINISTIC mode
// (as batch items do) instead of SF_ERR_UNSUPPORTED
int launch_fetch_and_op(sf_s *sf, sf_unit unit, void *root, const void *leaf, void *upd, int op,
                        hipStream_t st, bool fp_atomic = false);
int elem_size(int32_t dtype);
// launch shape of the persistent atomic kernels: grid size and the number of
// hot roots (a prefix of hot_roots) that a block aggregates in LDS
struct AtomicShape {
  int grid;
  int nhot_lds;
  size_t lds_bytes;
};
AtomicShape atomic_shape(const sf_s *sf, int ntiles, size_t per_root_bytes, int grid);
}  // namespace sfi
