// sf_plan.cpp -- host-side analysis of a star forest (PetscSFSetUp,
// Section 3.1: "sets up internal data structures ... and checks for all
// possible optimizations") and the upload of the resulting index plan.
//
// What the analysis builds:
//  * segments: leaves grouped by their rank label, stable in leaf order
//    (the per-neighbour leaf lists of Section 5.1);
//  * per segment and side, an index pattern when one exists: contiguous, or
//    the multi-strided 3-D sub-block start + X*Y*k + X*j + i (Section 5.2);
//  * the work tiles of the stream kernels and the index arrays they read;
//  * duplicate-root detection (Section 5.3) and, for the atomic reduction,
//    the roots of highest degree that a block aggregates in LDS;
//  * the root-sorted leaf lists (CSR, stable in leaf index) with degree
//    classes and aligned chunk levels for the deterministic reduction.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "sf_internal.h"

namespace sfi {

static thread_local int g_last_hip = 0;

int set_hip_error(hipError_t e) {
  g_last_hip = (int)e;
  return SF_ERR_HIP;
}
}  // namespace sfi

extern "C" int sf_last_hip_error(void) { return sfi::g_last_hip; }

namespace sfi {

int elem_size(int32_t dtype) {
  switch (dtype) {
    case SF_F64: return 8;
    case SF_F32: return 4;
    case SF_I32: return 4;
    case SF_I64: return 8;
    case SF_F64_I32: return 16;
    default: return 0;
  }
}

// Pattern of a sequence of indices (Section 5.2).  The sequence is
// contiguous when idx[t] = idx[0] + t.  Otherwise it is tried as a 3-D
// sub-block: dx = length of the first unit-step run, sy = the jump to the
// next row, dy = number of rows that follow that stride, sz = the jump to the
// next plane, dz = n / (dx*dy); the formula is then verified on every
// element, so a near miss falls back to generic.
sf_pattern detect_pattern(const int64_t *idx, int64_t n) {
  sf_pattern p{};
  p.kind = SF_PATTERN_GENERIC;
  if (n <= 0) {
    p.kind = SF_PATTERN_CONTIGUOUS;
    p.dx = p.dy = p.dz = 1;
    return p;
  }
  const int64_t s0 = idx[0];
  int64_t dx = 1;
  while (dx < n && idx[dx] == s0 + dx) dx++;
  if (dx == n) {
    p.kind = SF_PATTERN_CONTIGUOUS;
    p.start = (int32_t)s0;
    p.dx = (int32_t)n;
    p.dy = p.dz = 1;
    p.sy = (int32_t)n;
    p.sz = (int32_t)n;
    return p;
  }
  const int64_t sy = idx[dx] - s0;
  int64_t dy = 1;
  while (dy * dx < n && idx[dy * dx] == s0 + sy * dy) dy++;
  const int64_t plane = dx * dy;
  int64_t sz = plane < n ? idx[plane] - s0 : sy * dy;
  if (n % plane) return p;
  const int64_t dz = n / plane;
  for (int64_t k = 0, t = 0; k < dz; k++)
    for (int64_t j = 0; j < dy; j++)
      for (int64_t i = 0; i < dx; i++, t++)
        if (idx[t] != s0 + i + sy * j + sz * k) return p;
  const int64_t lim = INT32_MAX;
  if (std::llabs(sy) > lim || std::llabs(sz) > lim || dx > lim || dy > lim || dz > lim) return p;
  p.kind = SF_PATTERN_3D;
  p.start = (int32_t)s0;
  p.dx = (int32_t)dx;
  p.dy = (int32_t)dy;
  p.dz = (int32_t)dz;
  p.sy = (int32_t)sy;
  p.sz = (int32_t)sz;
  return p;
}

static DevPattern to_dev(const sf_pattern &p) {
  DevPattern d{};
  d.kind = p.kind;
  d.start = p.start;
  d.dx = p.dx;
  d.dy = p.dy;
  d.sy = p.sy;
  d.sz = p.sz;
  return d;
}

int analyze(sf_s *sf) {
  const int64_t L = sf->nleaves, R = sf->nroots;
  const bool use_patterns = sf->opts.use_patterns != 0;
  HostPlan hp;
  auto slot = [&](int64_t i) -> int64_t { return sf->ilocal ? sf->ilocal[i] : i; };

  // ---- segments: stable group-by on the rank label
  std::vector<Segment> segs;
  bool runs = true;
  for (int64_t i = 1; i < L && runs; i++)
    if (sf->iremote[i].rank < sf->iremote[i - 1].rank) runs = false;
  if (runs) {
    for (int64_t i = 0; i < L; i++) {
      if (segs.empty() || segs.back().rank != sf->iremote[i].rank) {
        segs.emplace_back();
        segs.back().rank = sf->iremote[i].rank;
      }
      segs.back().members.push_back(i);
    }
  } else {
    std::vector<int64_t> order(L);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return sf->iremote[a].rank < sf->iremote[b].rank;
    });
    for (int64_t i : order) {
      if (segs.empty() || segs.back().rank != sf->iremote[i].rank) {
        segs.emplace_back();
        segs.back().rank = sf->iremote[i].rank;
      }
      segs.back().members.push_back(i);
    }
  }
  std::vector<int64_t> tmp;
  for (auto &s : segs) {
    const int64_t n = (int64_t)s.members.size();
    tmp.resize(n);
    for (int64_t t = 0; t < n; t++) tmp[t] = sf->iremote[s.members[t]].index;
    s.root = detect_pattern(tmp.data(), n);
    for (int64_t t = 0; t < n; t++) tmp[t] = slot(s.members[t]);
    s.leaf = detect_pattern(tmp.data(), n);
  }

  // ---- processing layout of the stream kernels.  Per-segment layout when
  // patterns are wanted and segments are not tiny; otherwise one segment in
  // leaf order whose only possible "pattern" is the contiguous leaf space
  // of ilocal == NULL.
  struct Lay {
    std::vector<int64_t> members;  // empty => all leaves in order
    sf_pattern root, leaf;
  };
  std::vector<Lay> lay;
  const bool per_segment = use_patterns && !segs.empty() && (int64_t)segs.size() * 256 <= std::max<int64_t>(L, 256);
  if (per_segment) {
    for (auto &s : segs) lay.push_back({s.members, s.root, s.leaf});
  } else if (L > 0) {
    Lay one;
    one.root.kind = SF_PATTERN_GENERIC;
    one.leaf.kind = SF_PATTERN_GENERIC;
    if (use_patterns) {
      tmp.resize(L);
      for (int64_t i = 0; i < L; i++) tmp[i] = sf->iremote[i].index;
      one.root = detect_pattern(tmp.data(), L);
      for (int64_t i = 0; i < L; i++) tmp[i] = slot(i);
      one.leaf = detect_pattern(tmp.data(), L);
    } else if (!sf->ilocal) {
      one.leaf.kind = SF_PATTERN_CONTIGUOUS;
      one.leaf.start = 0;
      one.leaf.dx = (int32_t)L;
    }
    lay.push_back(std::move(one));
  }

  // ---- degrees, duplicate detection, hot roots
  std::vector<int64_t> deg(R, 0);
  for (int64_t i = 0; i < L; i++) deg[sf->iremote[i].index]++;
  int64_t maxdeg = 0;
  for (int64_t r = 0; r < R; r++) maxdeg = std::max(maxdeg, deg[r]);
  sf->max_degree = maxdeg;
  sf->has_dup_roots = maxdeg > 1;

  std::vector<int32_t> hot_of(R > 0 ? R : 1, -1);
  if (L >= 65536 && sf->has_dup_roots) {
    const int64_t hot_min = kPersistBlocks / 2;
    std::vector<int32_t> cand;
    for (int64_t r = 0; r < R; r++)
      if (deg[r] >= hot_min) cand.push_back((int32_t)r);
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    if ((int64_t)cand.size() > kHotMax) cand.resize(kHotMax);
    hp.hot_roots = cand;
    for (size_t h = 0; h < cand.size(); h++) hot_of[cand[h]] = (int32_t)h;
  }

  // ---- index arrays and tiles.  Tiles shrink for small SFs so that the
  // grid still has about four blocks per compute unit.
  int32_t tl = kTileLeaves;
  while (tl > kTileMin && L / tl < 1024) tl /= 2;
  hp.tile_leaves = tl;
  const bool want_hot = !hp.hot_roots.empty();
  for (size_t s = 0; s < lay.size(); s++) {
    const Lay &ly = lay[s];
    const int64_t n = ly.members.empty() ? L : (int64_t)ly.members.size();
    DevSegment d{};
    d.n = (int32_t)n;
    d.root = to_dev(ly.root);
    d.leaf = to_dev(ly.leaf);
    d.roff = d.loff = -1;
    auto member = [&](int64_t t) { return ly.members.empty() ? t : ly.members[t]; };
    if (ly.root.kind == SF_PATTERN_GENERIC) {
      d.roff = (int32_t)hp.ridx.size();
      for (int64_t t = 0; t < n; t++) {
        const int64_t r = sf->iremote[member(t)].index;
        hp.ridx.push_back((int32_t)r);
        if (want_hot) hp.ridx_hot.push_back(hot_of[r] >= 0 ? -(hot_of[r] + 1) : (int32_t)r);
      }
    }
    if (ly.leaf.kind == SF_PATTERN_GENERIC) {
      d.loff = (int32_t)hp.lidx.size();
      for (int64_t t = 0; t < n; t++) hp.lidx.push_back((int32_t)slot(member(t)));
    }
    hp.dsegs.push_back(d);
    for (int64_t t0 = 0; t0 < n; t0 += tl)
      hp.tiles.push_back({(int32_t)s, (int32_t)t0, (int32_t)std::min<int64_t>(n, t0 + tl), 0});
  }
  if (want_hot && hp.ridx_hot.empty()) hp.hot_roots.clear();

  // ---- root-sorted leaf lists (stable in leaf index)
  std::vector<int32_t> tord(R > 0 ? R : 1, -1);
  for (int64_t r = 0; r < R; r++)
    if (deg[r] > 0) {
      tord[r] = (int32_t)hp.troot.size();
      hp.troot.push_back((int32_t)r);
    }
  const int64_t T = (int64_t)hp.troot.size();
  hp.toff.assign(T + 1, 0);
  for (int64_t t = 0; t < T; t++) hp.toff[t + 1] = hp.toff[t] + (int32_t)deg[hp.troot[t]];
  hp.sl.resize(L);
  {
    std::vector<int32_t> fill(hp.toff.begin(), hp.toff.end() - 1);
    for (int64_t i = 0; i < L; i++) hp.sl[fill[tord[sf->iremote[i].index]]++] = (int32_t)slot(i);
  }
  // degree classes: 1, 2, (2,4], (4,8], (8,16], (16,32]; larger -> chunks
  for (int64_t t = 0; t < T; t++) {
    const int64_t d = hp.toff[t + 1] - hp.toff[t];
    if (d > kSmallMaxDeg) {
      hp.large.push_back((int32_t)t);
      continue;
    }
    int c = 0;
    while ((1 << c) < d) c++;
    hp.cls[c].push_back((int32_t)t);
  }
  // chunk levels of the large roots: level 0 reads leaves through sl, level
  // k > 0 reads the chunk results of level k-1.  Chunks are aligned at
  // multiples of kChunk of the root's own list, so every chunk result is a
  // node of the root's pairwise tree.
  struct Pend {
    int32_t root, src, n;
  };
  std::vector<Pend> cur;
  for (int32_t t : hp.large) cur.push_back({hp.troot[t], hp.toff[t], hp.toff[t + 1] - hp.toff[t]});
  while (!cur.empty()) {
    ChunkLevel lv;
    std::vector<Pend> next;
    for (const Pend &p : cur) {
      const int32_t nc = (p.n + kChunk - 1) / kChunk;
      if (nc == 1) {
        lv.chunks.push_back({p.src, p.n, -(p.root + 1), 0});
        continue;
      }
      const int32_t base = (int32_t)lv.out_len;
      for (int32_t c = 0; c < nc; c++)
        lv.chunks.push_back({p.src + c * kChunk, std::min(kChunk, p.n - c * kChunk), base + c, 0});
      lv.out_len += nc;
      next.push_back({p.root, base, nc});
    }
    hp.scratch_len = std::max(hp.scratch_len, lv.out_len);
    hp.levels.push_back(std::move(lv));
    cur.swap(next);
  }
  // FetchAndOp on large roots: all level-0 chunks, grouped per root
  hp.fo_root_first.push_back(0);
  for (int32_t t : hp.large) {
    const int32_t n = hp.toff[t + 1] - hp.toff[t];
    const int32_t nc = (n + kChunk - 1) / kChunk;
    for (int32_t c = 0; c < nc; c++)
      hp.fo_chunks.push_back({hp.toff[t] + c * kChunk, std::min(kChunk, n - c * kChunk), hp.troot[t], 0});
    hp.fo_root_first.push_back((int32_t)hp.fo_chunks.size());
  }

  sf->segments = std::move(segs);
  sf->hp = std::move(hp);
  sf->analyzed = true;
  return SF_OK;
}

void free_device(sf_s *sf) {
  if (sf->dp.blob) hipFree(sf->dp.blob);
  if (sf->scratch) hipFree(sf->scratch);
  sf->dp = DevPlan{};
  sf->scratch = nullptr;
  sf->scratch_bytes = 0;
}

int ensure_scratch(sf_s *sf, size_t bytes) {
  if (bytes <= sf->scratch_bytes) return SF_OK;
  if (sf->scratch) {
    hipError_t e = hipFree(sf->scratch);
    sf->scratch = nullptr;
    sf->scratch_bytes = 0;
    if (e != hipSuccess) return set_hip_error(e);
  }
  hipError_t e = hipMalloc(&sf->scratch, bytes);
  if (e != hipSuccess) {
    sf->scratch = nullptr;
    return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
  }
  sf->scratch_bytes = bytes;
  return SF_OK;
}

int upload(sf_s *sf) {
  free_device(sf);
  HostPlan &hp = sf->hp;
  struct Part {
    const void *src;
    size_t bytes;
    void **dst;
  };
  std::vector<Part> parts;
  DevPlan &dp = sf->dp;
  auto add = [&](const void *src, size_t bytes, void **dst) { parts.push_back({src, bytes, dst}); };
  add(hp.dsegs.data(), hp.dsegs.size() * sizeof(DevSegment), (void **)&dp.segs);
  add(hp.tiles.data(), hp.tiles.size() * sizeof(DevTile), (void **)&dp.tiles);
  add(hp.ridx.data(), hp.ridx.size() * 4, (void **)&dp.ridx);
  add(hp.ridx_hot.data(), hp.ridx_hot.size() * 4, (void **)&dp.ridx_hot);
  add(hp.lidx.data(), hp.lidx.size() * 4, (void **)&dp.lidx);
  add(hp.hot_roots.data(), hp.hot_roots.size() * 4, (void **)&dp.hot_roots);
  add(hp.troot.data(), hp.troot.size() * 4, (void **)&dp.troot);
  add(hp.toff.data(), hp.toff.size() * 4, (void **)&dp.toff);
  add(hp.sl.data(), hp.sl.size() * 4, (void **)&dp.sl);
  for (int c = 0; c < kNumClasses; c++) add(hp.cls[c].data(), hp.cls[c].size() * 4, (void **)&dp.cls[c]);
  add(hp.large.data(), hp.large.size() * 4, (void **)&dp.large);
  dp.levels.assign(hp.levels.size(), nullptr);
  for (size_t k = 0; k < hp.levels.size(); k++)
    add(hp.levels[k].chunks.data(), hp.levels[k].chunks.size() * sizeof(DevChunk), (void **)&dp.levels[k]);
  add(hp.fo_chunks.data(), hp.fo_chunks.size() * sizeof(DevChunk), (void **)&dp.fo_chunks);
  add(hp.fo_root_first.data(), hp.fo_root_first.size() * 4, (void **)&dp.fo_root_first);

  size_t total = 0;
  for (auto &p : parts) total += (p.bytes + 255) / 256 * 256;
  total = std::max<size_t>(total, 256);
  hipError_t e = hipGetDevice(&sf->device);
  if (e != hipSuccess) return set_hip_error(e);
  e = hipMalloc(&dp.blob, total);
  if (e != hipSuccess) {
    dp.blob = nullptr;
    return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
  }
  dp.bytes = total;
  size_t off = 0;
  for (auto &p : parts) {
    if (p.bytes == 0) {
      *p.dst = nullptr;
      continue;
    }
    *p.dst = (char *)dp.blob + off;
    e = hipMemcpy(*p.dst, p.src, p.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_device(sf);
      return set_hip_error(e);
    }
    off += (p.bytes + 255) / 256 * 256;
  }
  return SF_OK;
}

}  // namespace sfi
