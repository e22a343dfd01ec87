// sf_compose.cpp -- making new star forests from existing ones (Section 3.3):
// concatenation (PetscSFCompose, PetscSFComposeInverse) and embedding
// (PetscSFCreateEmbeddedRootSF / LeafSF).  Host graph algebra on the graphs
// given to sf_create; the results are new SFs, created but not set up.
#include <algorithm>
#include <new>
#include <vector>

#include "sf_internal.h"

namespace {

int64_t slot_of(const sf_s *sf, int64_t i) { return sf->ilocal ? sf->ilocal[i] : i; }

// A new SF from the kept edges (leaf slots, root nodes), copied.
int make(int64_t nroots, const std::vector<int64_t> &slots, const std::vector<sf_node> &nodes, bool contiguous,
         sf_t *out) {
  const int64_t n = (int64_t)nodes.size();
  return sf_create(nroots, n, contiguous ? nullptr : slots.data(), SF_COPY_VALUES, nodes.data(), SF_COPY_VALUES, out);
}

// The root of every leaf slot of sf (-1: no leaf there), and that leaf's label.
void slot_table(const sf_s *sf, std::vector<int64_t> &root, std::vector<int64_t> &label) {
  root.assign((size_t)std::max<int64_t>(sf->leafspace, 0), -1);
  label.assign(root.size(), 0);
  for (int64_t i = 0; i < sf->nleaves; i++) {
    const int64_t s = slot_of(sf, i);
    root[(size_t)s] = sf->iremote[i].index;
    label[(size_t)s] = sf->iremote[i].rank;
  }
}

}  // namespace

extern "C" int sf_get_graph(sf_t sf, int64_t *ilocal, sf_node *iremote) {
  if (!sf) return SF_ERR_ARG;
  for (int64_t i = 0; i < sf->nleaves; i++) {
    if (ilocal) ilocal[i] = slot_of(sf, i);
    if (iremote) iremote[i] = sf->iremote[i];
  }
  return SF_OK;
}

extern "C" int sf_create_embedded_root_sf(sf_t sf, int64_t n, const int64_t *selected_roots, sf_t *out) {
  if (!sf || !out || n < 0 || (n > 0 && !selected_roots)) return SF_ERR_ARG;
  *out = nullptr;
  try {
    std::vector<uint8_t> keep((size_t)std::max<int64_t>(sf->nroots, 1), 0);
    for (int64_t k = 0; k < n; k++) {
      if (selected_roots[k] < 0 || selected_roots[k] >= sf->nroots) return SF_ERR_ARG;
      keep[(size_t)selected_roots[k]] = 1;
    }
    std::vector<int64_t> slots;
    std::vector<sf_node> nodes;
    for (int64_t i = 0; i < sf->nleaves; i++)
      if (keep[(size_t)sf->iremote[i].index]) {
        slots.push_back(slot_of(sf, i));
        nodes.push_back(sf->iremote[i]);
      }
    return make(sf->nroots, slots, nodes, false, out);
  } catch (const std::bad_alloc &) {
    return SF_ERR_OOM;
  }
}

extern "C" int sf_create_embedded_leaf_sf(sf_t sf, int64_t n, const int64_t *selected_leaves, sf_t *out) {
  if (!sf || !out || n < 0 || (n > 0 && !selected_leaves)) return SF_ERR_ARG;
  *out = nullptr;
  try {
    std::vector<uint8_t> keep((size_t)std::max<int64_t>(sf->leafspace, 1), 0);
    for (int64_t k = 0; k < n; k++) {
      if (selected_leaves[k] < 0) return SF_ERR_ARG;
      if (selected_leaves[k] < sf->leafspace) keep[(size_t)selected_leaves[k]] = 1;  // beyond: no leaf there
    }
    std::vector<int64_t> slots;
    std::vector<sf_node> nodes;
    for (int64_t i = 0; i < sf->nleaves; i++)
      if (keep[(size_t)slot_of(sf, i)]) {
        slots.push_back(slot_of(sf, i));
        nodes.push_back(sf->iremote[i]);
      }
    return make(sf->nroots, slots, nodes, false, out);
  } catch (const std::bad_alloc &) {
    return SF_ERR_OOM;
  }
}

extern "C" int sf_compose(sf_t a, sf_t b, sf_t *out) {
  if (!a || !b || !out) return SF_ERR_ARG;
  *out = nullptr;
  if (a->leafspace > b->nroots) return SF_ERR_ARG;  // a's leaves must lie among b's roots
  try {
    std::vector<int64_t> aroot, alabel;
    slot_table(a, aroot, alabel);
    std::vector<int64_t> slots;
    std::vector<sf_node> nodes;
    for (int64_t i = 0; i < b->nleaves; i++) {  // b's leaves in b's leaf order
      const int64_t mid = b->iremote[i].index;  // b's root = a's leaf slot
      if (mid >= (int64_t)aroot.size() || aroot[(size_t)mid] < 0) continue;
      slots.push_back(slot_of(b, i));
      nodes.push_back({b->iremote[i].rank, aroot[(size_t)mid]});
    }
    return make(a->nroots, slots, nodes, false, out);
  } catch (const std::bad_alloc &) {
    return SF_ERR_OOM;
  }
}

extern "C" int sf_compose_inverse(sf_t a, sf_t b, sf_t *out) {
  if (!a || !b || !out) return SF_ERR_ARG;
  *out = nullptr;
  try {
    // b's roots must have degree <= 1: each b root maps to its leaf's slot
    std::vector<int64_t> bslot((size_t)std::max<int64_t>(b->nroots, 1), -1);
    for (int64_t i = 0; i < b->nleaves; i++) {
      const int64_t r = b->iremote[i].index;
      if (bslot[(size_t)r] >= 0) return SF_ERR_ARG;
      bslot[(size_t)r] = slot_of(b, i);
    }
    std::vector<int64_t> aroot, alabel;
    slot_table(a, aroot, alabel);
    std::vector<int64_t> slots;
    std::vector<sf_node> nodes;
    for (int64_t r = 0; r < b->nroots; r++) {  // the new leaves: b's roots, in order
      const int64_t s = bslot[(size_t)r];
      if (s < 0 || s >= (int64_t)aroot.size() || aroot[(size_t)s] < 0) continue;
      slots.push_back(r);
      nodes.push_back({alabel[(size_t)s], aroot[(size_t)s]});
    }
    return make(a->nroots, slots, nodes, false, out);
  } catch (const std::bad_alloc &) {
    return SF_ERR_OOM;
  }
}
