// sf_plan.cpp -- host-side analysis of a star forest (PetscSFSetUp of
// Section 3.1, which builds the internal structures once and looks for every
// optimisation it can apply) and the upload of the resulting index plan.
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
#include <system_error>
#include <thread>

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
    case SF_F16: return 2;
    case SF_BF16: return 2;
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

// ceil(2^64 / d) for d >= 2 (0 for d <= 1): with it, t / d = the high 64
// bits of m * t for every t < 2^32 (Lemire, Kaser and Kurz, "Faster
// remainder by direct computation", 2019).
static uint64_t magic_div(int32_t d) { return d <= 1 ? 0 : ~0ull / (uint64_t)d + 1; }

static DevPattern to_dev(const sf_pattern &p) {
  DevPattern d{};
  d.mdx = magic_div(p.dx);
  d.mdy = magic_div(p.dy);
  d.kind = p.kind;
  d.start = p.start;
  d.dx = p.dx;
  d.dy = p.dy;
  d.sy = p.sy;
  d.sz = p.sz;
  return d;
}

// The partitioned plan of one unit-size class.  Items -- a whole root of
// degree <= kSmallMaxDeg, or one level-0 chunk of a larger root -- are
// packed greedily into windows of at most `cap` sorted leaves, cold roots
// first (in root order), then hot roots (is_hot), so that windows
// [0, wcold) hold no hot root.  Every sorted leaf g gets its window win_g[g]
// and its offset loc_g[g] inside the window; a root's leaves, and a chunk's,
// have consecutive offsets.  Scratch is window-major and, inside a window,
// in processing order, so:
//  * pass A, which moves the leaves of `ta` consecutive processing positions
//    (one pass-A tile) into scratch, writes one contiguous run per window,
//    in increasing slot order (pa_loc with run starts, pa_run);
//  * pass B loads one window's contiguous scratch range into LDS, moving
//    scratch slot s to LDS offset lpos[s] (the leaf's offset in the window).
static int build_stage(HostPlan &hp, HostPlan::Stage &sp, const std::vector<int32_t> &perm,
                       const std::vector<int64_t> &proc_leaf, const std::vector<int32_t> &proc_slot,
                       const std::vector<uint8_t> &is_hot, int64_t L, int32_t ta, int32_t cap) {
  const int64_t T = (int64_t)hp.troot.size();
  sp = HostPlan::Stage();
  sp.ta = ta;
  sp.cap = cap;
  std::vector<int32_t> win_g(L), loc_g(L);  // window of the g-th sorted leaf, its offset there
  std::vector<int32_t> small, big;  // touched-root ordinals / level-0 chunk ordinals, window-major
  DevSWin cur{};
  int64_t cur_n = 0;
  std::vector<std::pair<int32_t, int32_t>> small_in_win;  // (class, t)
  auto close_window = [&]() {
    std::stable_sort(small_in_win.begin(), small_in_win.end(),
                     [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
                       return x.first < y.first;
                     });
    cur.small0 = (int32_t)small.size();
    for (auto &x : small_in_win) small.push_back(x.second);
    cur.small1 = (int32_t)small.size();
    cur.big1 = (int32_t)big.size();
    sp.maxbig = std::max(sp.maxbig, cur.big1 - cur.big0);
    cur.n = (int32_t)cur_n;
    sp.win.push_back(cur);
    small_in_win.clear();
    cur = DevSWin{};
    cur.big0 = (int32_t)big.size();
    cur_n = 0;
  };
  static const std::vector<DevChunk> none;
  const std::vector<DevChunk> &lv0 = hp.levels.empty() ? none : hp.levels[0].chunks;
  // first level-0 chunk of every large root (its chunks are consecutive in lv0)
  std::vector<int32_t> chunk_first(T, -1);
  {
    int32_t c = 0;
    for (int64_t t = 0; t < T; t++) {
      const int32_t n = hp.toff[t + 1] - hp.toff[t];
      if (n > kSmallMaxDeg) {
        chunk_first[t] = c;
        c += (n + kChunk - 1) / kChunk;
      }
    }
    if (c != (int32_t)lv0.size()) return SF_ERR_ARG;
  }
  int64_t placed_chunks = 0;
  for (int pass = 0; pass < 2; pass++) {
    if (pass == 1) {
      if (cur_n > 0) close_window();
      sp.wcold = (int32_t)sp.win.size();
    }
    for (int64_t t = 0; t < T; t++) {
      if ((int)is_hot[t] != pass) continue;
      const int32_t g0 = hp.toff[t], n = hp.toff[t + 1] - g0;
      if (n <= kSmallMaxDeg) {
        if (cur_n + n > cap) close_window();
        int c = 0;
        while ((1 << c) < n) c++;
        small_in_win.push_back({c, (int32_t)t});
        for (int32_t g = g0; g < g0 + n; g++) {
          win_g[g] = (int32_t)sp.win.size();
          loc_g[g] = (int32_t)(cur_n + (g - g0));
        }
        cur_n += n;
      } else {
        int32_t left = n;  // this root's level-0 chunks are consecutive in lv0
        for (int32_t chunk = chunk_first[t]; left > 0; chunk++) {
          const DevChunk &ch = lv0[chunk];
          if (cur_n + ch.n > cap) close_window();
          big.push_back(chunk);
          for (int32_t g = ch.src; g < ch.src + ch.n; g++) {
            win_g[g] = (int32_t)sp.win.size();
            loc_g[g] = (int32_t)(cur_n + (g - ch.src));
          }
          cur_n += ch.n;
          left -= ch.n;
          placed_chunks++;
        }
      }
    }
  }
  if (cur_n > 0 || sp.win.empty()) close_window();
  const int64_t W = (int64_t)sp.win.size();
  int64_t base = 0;
  for (int64_t w = 0; w < W; w++) {
    sp.win[w].base = (int32_t)base;
    sp.win[w].g0 = -1;  // windows are not ranges of the sorted order: offsets come from loc_g
    base += sp.win[w].n;
  }
  if (base != L || placed_chunks != (int64_t)lv0.size() || lv0.size() != hp.fo_chunks.size()) return SF_ERR_ARG;
  // per-window descriptors: offsets inside the window
  const int64_t nfo = (int64_t)hp.fo_chunks.size();
  for (int64_t w = 0; w < W; w++) {
    const DevSWin &win = sp.win[w];
    for (int32_t i = win.small0; i < win.small1; i++) {
      const int32_t t = small[i];
      const int64_t n = hp.toff[t + 1] - hp.toff[t];
      const int64_t o = loc_g[hp.toff[t]];
      if (win_g[hp.toff[t]] != w || o + n > win.n || o > 0xffff || n > kSmallMaxDeg) return SF_ERR_ARG;
      sp.sroot.push_back({hp.troot[t], (int32_t)(o | (n << 16))});
    }
    for (int32_t i = win.big0; i < win.big1; i++) {
      const int32_t k = big[i];
      const DevChunk &ch = lv0[k];
      const int32_t r = hp.fo_chunks[k].dst;
      const int64_t o = loc_g[ch.src];
      if (win_g[ch.src] != w || o + ch.n > win.n || o > 0xffff || ch.n < 1 || ch.n > kChunk ||
          hp.fo_chunks[k].src != ch.src)
        return SF_ERR_ARG;
      const int32_t first = (k == 0 || hp.fo_chunks[k - 1].dst != r) ? 1 : 0;
      const int32_t last = (k + 1 == nfo || hp.fo_chunks[k + 1].dst != r) ? 1 : 0;
      sp.wchunk.push_back({(int32_t)(o | ((int64_t)(ch.n - 1) << 16) | (first << 24) | (last << 25)), ch.dst, r, k});
    }
  }
  // scratch slot of every processed leaf: window base + rank in processing order
  std::vector<int32_t> pos(L);
  for (int64_t g = 0; g < L; g++) pos[perm[g]] = (int32_t)g;
  std::vector<int32_t> dst(L), cursor(W);
  for (int64_t w = 0; w < W; w++) cursor[w] = sp.win[w].base;
  std::vector<int32_t> proc_of_leaf(L);
  for (int64_t p = 0; p < L; p++) {
    const int64_t i = proc_leaf[p];
    proc_of_leaf[i] = (int32_t)p;
    dst[p] = cursor[win_g[pos[i]]]++;
  }
  sp.lpos.assign(L, 0);
  std::vector<int32_t> slot_of_g(L);
  for (int64_t g = 0; g < L; g++) {
    const DevSWin &w = sp.win[win_g[g]];
    const int64_t s = dst[proc_of_leaf[perm[g]]];
    if (s < w.base || s >= (int64_t)w.base + w.n || loc_g[g] > 0x3fff) return SF_ERR_ARG;
    sp.lpos[s] = (uint16_t)loc_g[g];
    slot_of_g[g] = (int32_t)s;
  }
  // Runs of a large root's chunks inside a window that are not the whole root
  // span windows.  Such a run starts at the window's first offset (it
  // continues one from the previous window; "which" 0) or ends at its last
  // (it continues into the next; which 1).  The slots of cold roots' runs are
  // marked (sflag: 1 | which << 1, carried into pa_loc below), and every
  // spanning root lists its runs (2 * window + which) in window order; the
  // leaves of hot roots are marked 2 (0x4000 alone in pa_loc).
  std::vector<uint8_t> sflag(L, 0);
  sp.span_first.assign(1, 0);
  for (int64_t w = 0; w < W; w++) {
    const DevSWin &win = sp.win[w];
    const bool hot_win = w >= sp.wcold;
    bool have0 = false;
    for (int32_t i = win.big0; i < win.big1;) {
      const DevWChunk &c0 = sp.wchunk[i];
      int32_t j = i + 1;
      while (j < win.big1 && sp.wchunk[j].root == c0.root) j++;
      const DevWChunk &c1 = sp.wchunk[j - 1];
      const bool whole = ((c0.onf >> 24) & 1) && ((c1.onf >> 25) & 1);
      if (!whole) {
        const int32_t o0 = c0.onf & 0xffff, o1 = (c1.onf & 0xffff) + ((c1.onf >> 16) & 0xff) + 1;
        const int32_t which = o0 == 0 ? 0 : 1;
        if ((which == 0 && have0) || (which == 1 && o1 != win.n)) return SF_ERR_ARG;
        have0 = have0 || which == 0;
        if (!hot_win) {
          for (int32_t q = i; q < j; q++) {
            const DevChunk &ch = lv0[sp.wchunk[q].k];
            for (int32_t g = ch.src; g < ch.src + ch.n; g++) sflag[slot_of_g[g]] = (uint8_t)(1 | (which << 1));
          }
        }
        if (sp.span_root.empty() || sp.span_root.back() != c0.root) {
          if (!sp.span_root.empty()) sp.span_first.push_back((int32_t)sp.span_slot.size());
          sp.span_root.push_back(c0.root);
          if (!hot_win) sp.nspan_cold = (int32_t)sp.span_root.size();
        }
        sp.span_slot.push_back((int32_t)(2 * w + which));
      }
      i = j;
    }
  }
  if (!sp.span_root.empty()) sp.span_first.push_back((int32_t)sp.span_slot.size());
  if (sp.wcold < W) {
    for (int64_t s2 = sp.win[sp.wcold].base; s2 < L; s2++) sflag[s2] = 2;
  }
  // pass-A tiles: increasing scratch slot inside each tile
  const int64_t ntiles = (L + ta - 1) / ta;
  if (ta > 0x2000) return SF_ERR_ARG;  // tile offsets take 13 bits
  sp.pa_loc.resize(L);
  sp.pa_run0.assign(ntiles + 1, 0);
  sp.tile_leaf0.assign(ntiles, -1);
  std::vector<int32_t> tdst(ta);
  bool gather = false;
  // inside a window, slots increase with processing position, so ordering a
  // tile by slot is a stable counting sort of its leaves by window
  std::vector<int32_t> wofp(L);
  for (int64_t p = 0; p < L; p++) wofp[p] = win_g[pos[proc_leaf[p]]];
  std::vector<int32_t> cnt(W + 1, 0);
  for (int64_t k = 0; k < ntiles; k++) {
    const int64_t p0 = k * ta, n = std::min<int64_t>(ta, L - p0);
    int32_t wlo = INT32_MAX, whi = -1;
    bool contiguous = true;
    for (int64_t q = 0; q < n; q++) {
      wlo = std::min(wlo, wofp[p0 + q]);
      whi = std::max(whi, wofp[p0 + q]);
      if (proc_slot[p0 + q] != proc_slot[p0] + q) contiguous = false;
    }
    std::fill(cnt.begin() + wlo, cnt.begin() + whi + 2, 0);
    for (int64_t q = 0; q < n; q++) cnt[wofp[p0 + q] + 1]++;
    for (int32_t w = wlo; w <= whi; w++) cnt[w + 1] += cnt[w];
    for (int64_t q = 0; q < n; q++) {
      const int32_t at = cnt[wofp[p0 + q]]++;
      tdst[at] = dst[p0 + q];
      sp.pa_loc[p0 + at] = (uint16_t)q;
    }
    for (int64_t at = 0; at < n; at++) {
      if (at > 0 && tdst[at] <= tdst[at - 1]) return SF_ERR_ARG;
      sp.pa_loc[p0 + at] |= (uint16_t)(sflag[tdst[at]] << 13);  // spanning run, which
      // a new run of consecutive slots, also where the window changes
      const int32_t w_at = wofp[p0 + (sp.pa_loc[p0 + at] & 0x1fff)];
      if (at == 0 || tdst[at] != tdst[at - 1] + 1 || w_at != sp.pa_runw.back()) {
        sp.pa_loc[p0 + at] |= 0x8000;
        sp.pa_run.push_back(tdst[at] - (int32_t)at);
        sp.pa_runw.push_back(w_at);
      }
    }
    sp.pa_run0[k + 1] = (int32_t)sp.pa_run.size();
    sp.maxrun = std::max(sp.maxrun, sp.pa_run0[k + 1] - sp.pa_run0[k]);
    if (contiguous) sp.tile_leaf0[k] = proc_slot[p0];
    else gather = true;
  }
  if (gather) sp.pa_slot = proc_slot;
  // self-check: dst is a permutation of the scratch slots
  std::vector<uint8_t> seen(L, 0);
  for (int64_t p = 0; p < L; p++) {
    if (dst[p] < 0 || dst[p] >= L || seen[dst[p]]) return SF_ERR_ARG;
    seen[dst[p]] = 1;
  }
  return SF_OK;
}

// Window and tile sizes per unit-size class.  Pass-A tiles of 8192 units
// (two 64 KB tiles of units <= 8 B share a CU; at most 8192 positions:
// 13-bit offsets in pa_loc).  Windows of 64 KB, so that two pass-B blocks
// share a CU: 8192 units <= 8 B (4096 and 16384 measured slower on the
// 16M-leaf Zipf SF), 4096 units of 9..16 B (MAXLOC 222 -> 207 us against
// one 128 KB window per CU).
static void stage_sizes(int cls, int32_t *ta, int32_t *cap) {
  *ta = kPassATile;
  *cap = cls == 0 ? 8192 : 4096;
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
    std::vector<int32_t> cand;
    for (int64_t r = 0; r < R; r++)
      if (deg[r] >= kHotMinDeg) cand.push_back((int32_t)r);
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
    if ((int64_t)cand.size() > kHotMax) cand.resize(kHotMax);
    hp.hot_roots = cand;
    for (int32_t r : cand) hp.hot_deg.push_back(deg[r]);
    for (size_t h = 0; h < cand.size(); h++) hot_of[cand[h]] = (int32_t)h;
  }

  std::vector<int64_t> proc_leaf;  // leaf index of the p-th processed leaf
  proc_leaf.reserve(L);
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
    d.pbase = (int32_t)proc_leaf.size();
    auto member = [&](int64_t t) { return ly.members.empty() ? t : ly.members[t]; };
    for (int64_t t = 0; t < n; t++) proc_leaf.push_back(member(t));
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
  // contiguous on both sides in every segment: a REPLACE is a plain copy
  hp.all_contig = !hp.dsegs.empty() && hp.dsegs.size() <= 64;
  for (const DevSegment &d : hp.dsegs)
    if (d.root.kind != SF_PATTERN_CONTIGUOUS || d.leaf.kind != SF_PATTERN_CONTIGUOUS) hp.all_contig = false;
  if (want_hot && hp.ridx_hot.empty()) {
    hp.hot_roots.clear();
    hp.hot_deg.clear();
  }

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
  std::vector<int32_t> perm(L);  // leaf index of the g-th sorted leaf
  {
    std::vector<int32_t> fill(hp.toff.begin(), hp.toff.end() - 1);
    for (int64_t i = 0; i < L; i++) {
      const int32_t g = fill[tord[sf->iremote[i].index]]++;
      hp.sl[g] = (int32_t)slot(i);
      perm[g] = (int32_t)i;
    }
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
  for (int c = 0; c < kNumClasses; c++) hp.small_all.insert(hp.small_all.end(), hp.cls[c].begin(), hp.cls[c].end());
  // the Reduce split: repeated roots of at most kSmallMaxDeg leaves that hold
  // under half of the leaves
  if (sf->has_dup_roots && maxdeg <= kSmallMaxDeg) {
    int64_t single = (int64_t)hp.cls[0].size();
    if (2 * single >= L) {
      hp.split = true;
      for (int c = 1; c < kNumClasses; c++) hp.rep_list.insert(hp.rep_list.end(), hp.cls[c].begin(), hp.cls[c].end());
      hp.rep_bits.assign((size_t)((L + 31) / 32), 0u);
      for (int64_t p = 0; p < L; p++)
        if (deg[sf->iremote[proc_leaf[p]].index] > 1) hp.rep_bits[(size_t)(p >> 5)] |= 1u << (p & 31);
    }
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

  // ---- partitioned deterministic path
  const int pmode = sf->opts.partition;  // 0 auto, 1 on, 2 off
  if (sf->has_dup_roots && (pmode == 1 || (pmode == 0 && L >= kPartitionPlan))) {
    std::vector<int32_t> proc_slot(L);
    for (int64_t p = 0; p < L; p++) proc_slot[p] = (int32_t)slot(proc_leaf[p]);
    // hot roots (they need tiles in leaf order: processing order must be
    // leaf order, as it is when segment labels do not decrease)
    std::vector<uint8_t> is_hot(T, 0);
    bool leaf_order = true;
    for (int64_t p = 0; p < L && leaf_order; p++) leaf_order = proc_leaf[p] == p;
    if (sf->opts.hot_path == 1 && leaf_order) {
      const int64_t ntiles = (L + kPassATile - 1) / kPassATile;
      const int64_t dmin = std::max<int64_t>(64, kHotPerTile * ntiles);
      std::vector<int32_t> cand;  // touched-root ordinals
      for (int64_t t = 0; t < T; t++)
        if (hp.toff[t + 1] - hp.toff[t] >= dmin) cand.push_back((int32_t)t);
      std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
        return hp.toff[a + 1] - hp.toff[a] > hp.toff[b + 1] - hp.toff[b];
      });
      if ((int64_t)cand.size() > kHotRootsMax) cand.resize(kHotRootsMax);
      if (!cand.empty()) {
        std::vector<int32_t> hid(R, -1);
        for (size_t h = 0; h < cand.size(); h++) {
          is_hot[cand[h]] = 1;
          hp.hx_root.push_back(hp.troot[cand[h]]);
          hid[hp.troot[cand[h]]] = (int32_t)h;
        }
        const int64_t H = (int64_t)cand.size();
        // per tile, the entries grouped by hot root (h ascending), in leaf
        // order inside a group: walk every hot root's leaves in leaf order
        // (processing position = leaf index here)
        std::vector<int32_t> cnt(ntiles + 1, 0);
        for (int64_t h = 0; h < H; h++) {
          const int32_t t = cand[h];
          for (int32_t g = hp.toff[t]; g < hp.toff[t + 1]; g++) cnt[perm[g] / kPassATile + 1]++;
        }
        for (int64_t k = 0; k < ntiles; k++) cnt[k + 1] += cnt[k];
        hp.hx_e0.assign(cnt.begin(), cnt.end());
        hp.hx_pos.resize(cnt[ntiles]);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1), last_h(ntiles, -1), ngrp(ntiles, 0);
        for (int64_t h = 0; h < H; h++) {
          const int32_t t = cand[h];
          for (int32_t g = hp.toff[t]; g < hp.toff[t + 1]; g++) {
            const int64_t k = perm[g] / kPassATile;
            const bool head = last_h[k] != (int32_t)h;
            if (head) {
              last_h[k] = (int32_t)h;
              ngrp[k]++;
            }
            hp.hx_pos[fill[k]++] = (uint16_t)((perm[g] - k * kPassATile) | (head ? 0x8000 : 0));
          }
        }
        hp.hx_grp0.assign(ntiles + 1, 0);
        for (int64_t k = 0; k < ntiles; k++) hp.hx_grp0[k + 1] = hp.hx_grp0[k] + ngrp[k];
        // per tile and hot-phase thread: the groups started before its first entry
        hp.hx_tg.assign((size_t)ntiles * kStageThreads, 0);
        for (int64_t k = 0; k < ntiles; k++) {
          const int32_t e0 = hp.hx_e0[k], nh = hp.hx_e0[k + 1] - e0;
          const int32_t K = (nh + kStageThreads - 1) / kStageThreads;
          int32_t heads = 0, e = 0;
          for (int32_t t = 0; t < kStageThreads; t++) {
            const int32_t b0 = std::min(t * K, nh);
            for (; e < b0; e++) heads += (hp.hx_pos[e0 + e] >> 15) & 1;
            hp.hx_tg[(size_t)k * kStageThreads + t] = (uint16_t)heads;
          }
        }
        std::vector<int32_t> gh(hp.hx_grp0[ntiles]);  // hot root of every group
        for (int64_t k = 0; k < ntiles; k++) {
          int32_t g = hp.hx_grp0[k];
          for (int32_t e = hp.hx_e0[k]; e < hp.hx_e0[k + 1]; e++)
            if (hp.hx_pos[e] & 0x8000) gh[g++] = hid[sf->iremote[k * kPassATile + (hp.hx_pos[e] & 0x1fff)].index];
        }
        // groups per hot root, in tile order: root-major positions
        hp.hx_rfirst.assign(H + 1, 0);
        for (int32_t h : gh) hp.hx_rfirst[h + 1]++;
        for (int64_t h = 0; h < H; h++) {
          hp.hx_maxgrp = std::max(hp.hx_maxgrp, hp.hx_rfirst[h + 1]);
          hp.hx_rfirst[h + 1] += hp.hx_rfirst[h];
        }
        hp.hx_rpos.resize(gh.size());
        std::vector<int32_t> rfill(hp.hx_rfirst.begin(), hp.hx_rfirst.end() - 1);
        for (size_t g = 0; g < gh.size(); g++) hp.hx_rpos[g] = rfill[gh[g]]++;
        hp.hot = true;
      }
    }
    // the two unit-size classes read the shared plan and write only their
    // own stage: built side by side
    int rcs[2] = {SF_OK, SF_OK};
    auto work = [&](int cls) {
      try {
        int32_t ta, cap;
        stage_sizes(cls, &ta, &cap);
        rcs[cls] = build_stage(hp, hp.sp[cls], perm, proc_leaf, proc_slot, is_hot, L, ta, cap);
      } catch (const std::bad_alloc &) {
        rcs[cls] = SF_ERR_OOM;
      }
    };
    try {
      std::thread other(work, 1);
      work(0);
      other.join();
    } catch (const std::system_error &) {  // no thread: one after the other
      work(0);
      work(1);
    }
    for (int rc : rcs)
      if (rc) return rc;
    hp.part = true;
    const bool levels = maxdeg > kSmallMaxDeg;
    hp.part_red_atomic = pmode == 1 || L >= kPartitionMid;
    hp.part_red_det = pmode == 1 || L >= (levels ? kPartitionMid : kPartitionBig);
    hp.part_fop_atomic = pmode == 1 || L >= kPartitionBig;
  }

  sf->segments = std::move(segs);
  sf->hp = std::move(hp);
  sf->analyzed = true;
  return SF_OK;
}

void free_device(sf_s *sf) {
  if (sf->dp.blob) (void)hipFree(sf->dp.blob);
  if (sf->scratch) (void)hipFree(sf->scratch);
  for (void *p : sf->retired) (void)hipFree(p);
  sf->retired.clear();
  sf->dp = DevPlan{};
  sf->scratch = nullptr;
  sf->scratch_bytes = 0;
}

// A block of the persistent atomic kernels sees about L / grid leaves; a
// root is worth an LDS slot when it has at least half a hit per block
// (otherwise flushing the slot costs as many atomics as it saves).
AtomicShape atomic_shape(const sf_s *sf, int ntiles, size_t per_root_bytes, int grid) {
  const size_t budget = kHotLdsBytes;
  grid = std::max(1, std::min(grid, ntiles));
  const HostPlan &h = sf->hp;
  int n = 0;
  const int64_t min_deg = std::max<int64_t>(kHotMinDeg, grid / 2);
  while (n < (int)h.hot_deg.size() && h.hot_deg[n] >= min_deg) n++;
  n = (int)std::min<size_t>((size_t)n, budget / per_root_bytes);
  return {grid, n, (size_t)n * per_root_bytes + 16};
}

int ensure_scratch(sf_s *sf, size_t bytes) {
  if (bytes <= sf->scratch_bytes) return SF_OK;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
  // the outgrown buffer may still be in use by enqueued or captured work
  if (sf->scratch) sf->retired.push_back(sf->scratch);
  sf->scratch = p;
  sf->scratch_bytes = bytes;
  return SF_OK;
}

int acquire_scratch(sf_s *sf, size_t bytes, void **out) {
  if (sf->fixed_scratch) {
    if (bytes > sf->fixed_scratch_bytes) return SF_ERR_SCRATCH;
    *out = sf->fixed_scratch;
    return SF_OK;
  }
  int rc = ensure_scratch(sf, bytes);
  if (rc) return rc;
  *out = sf->scratch;
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
  add(hp.small_all.data(), hp.small_all.size() * 4, (void **)&dp.small_all);
  dp.levels.assign(hp.levels.size(), nullptr);
  for (size_t k = 0; k < hp.levels.size(); k++)
    add(hp.levels[k].chunks.data(), hp.levels[k].chunks.size() * sizeof(DevChunk), (void **)&dp.levels[k]);
  add(hp.fo_chunks.data(), hp.fo_chunks.size() * sizeof(DevChunk), (void **)&dp.fo_chunks);
  add(hp.fo_root_first.data(), hp.fo_root_first.size() * 4, (void **)&dp.fo_root_first);
  for (int c = 0; c < 2; c++) {
    HostPlan::Stage &sp = hp.sp[c];
    DevPlan::Stage &ds = dp.sp[c];
    add(sp.win.data(), sp.win.size() * sizeof(DevSWin), (void **)&ds.win);
    add(sp.sroot.data(), sp.sroot.size() * sizeof(DevSRoot), (void **)&ds.sroot);
    add(sp.wchunk.data(), sp.wchunk.size() * sizeof(DevWChunk), (void **)&ds.wchunk);
    add(sp.lpos.data(), sp.lpos.size() * 2, (void **)&ds.lpos);
    add(sp.pa_run.data(), sp.pa_run.size() * 4, (void **)&ds.pa_run);
    add(sp.pa_runw.data(), sp.pa_runw.size() * 4, (void **)&ds.pa_runw);
    add(sp.span_first.data(), sp.span_first.size() * 4, (void **)&ds.span_first);
    add(sp.span_slot.data(), sp.span_slot.size() * 4, (void **)&ds.span_slot);
    add(sp.span_root.data(), sp.span_root.size() * 4, (void **)&ds.span_root);
    add(sp.pa_run0.data(), sp.pa_run0.size() * 4, (void **)&ds.pa_run0);
    add(sp.pa_loc.data(), sp.pa_loc.size() * 2, (void **)&ds.pa_loc);
    add(sp.tile_leaf0.data(), sp.tile_leaf0.size() * 4, (void **)&ds.tile_leaf0);
    add(sp.pa_slot.data(), sp.pa_slot.size() * 4, (void **)&ds.pa_slot);
  }

  add(hp.rep_bits.data(), hp.rep_bits.size() * 4, (void **)&dp.rep_bits);
  add(hp.rep_list.data(), hp.rep_list.size() * 4, (void **)&dp.rep_list);
  add(hp.hx_root.data(), hp.hx_root.size() * 4, (void **)&dp.hx_root);
  add(hp.hx_pos.data(), hp.hx_pos.size() * 2, (void **)&dp.hx_pos);
  add(hp.hx_e0.data(), hp.hx_e0.size() * 4, (void **)&dp.hx_e0);
  add(hp.hx_grp0.data(), hp.hx_grp0.size() * 4, (void **)&dp.hx_grp0);
  add(hp.hx_rfirst.data(), hp.hx_rfirst.size() * 4, (void **)&dp.hx_rfirst);
  add(hp.hx_rpos.data(), hp.hx_rpos.size() * 4, (void **)&dp.hx_rpos);
  add(hp.hx_tg.data(), hp.hx_tg.size() * 2, (void **)&dp.hx_tg);

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
