// Host-side neighbour table of an octree leaf list (paper Sec. IV-C: a
// properly nested octree of 8^3 sub-grids, each refinable into 8 children).
//
// For every leaf and each of the 27 directions (dx,dy,dz) in {-1,0,1}^3 the
// table names where the ghost cells on that side come from: a leaf at the
// same level, a refined node at the same level (its children are one level
// finer), or the leaf one level coarser that contains the neighbour block.
// Periodic wrap is folded in.  This is setup work, run once per tree.
#include <cstdint>
#include <cstdio>
#include <string>
#include <unordered_map>

#include "octohydro.h"
#include "octohydro_internal.h"

namespace {

inline uint64_t pack(int32_t level, int32_t x, int32_t y, int32_t z) {
  return (uint64_t(uint32_t(level)) << 60) | (uint64_t(uint32_t(z)) << 40) |
         (uint64_t(uint32_t(y)) << 20) | uint64_t(uint32_t(x));
}

inline int32_t pmod(int32_t a, int32_t m) { return ((a % m) + m) % m; }

}  // namespace

extern "C" int hydro_build_table(int32_t n_leaves, int32_t base, const int32_t* leaf_coord,
                                 int32_t* nbr, uint8_t* kind, int32_t* children,
                                 int32_t max_nodes, int32_t* n_nodes_out) {
  octohydro::clear_error();
  if (n_leaves <= 0 || base <= 0 || !leaf_coord || !nbr || !kind || !children || !n_nodes_out ||
      max_nodes < 0)
    return octohydro::fail(HYDRO_E_ARG, "hydro_build_table: bad argument");
  std::unordered_map<uint64_t, int32_t> leaves;
  leaves.reserve(size_t(n_leaves) * 2);
  for (int32_t i = 0; i < n_leaves; ++i) {
    const int32_t* c = leaf_coord + 4 * i;
    const int32_t blocks = base << c[0];
    if (c[0] < 0 || c[0] > 12 || c[1] < 0 || c[2] < 0 || c[3] < 0 || c[1] >= blocks ||
        c[2] >= blocks || c[3] >= blocks)
      return octohydro::fail(HYDRO_E_ARG, "hydro_build_table: leaf %d out of range", i);
    if (!leaves.emplace(pack(c[0], c[1], c[2], c[3]), i).second)
      return octohydro::fail(HYDRO_E_TABLE, "hydro_build_table: duplicate leaf %d", i);
  }
  auto leaf_at = [&](int32_t L, int32_t x, int32_t y, int32_t z) -> int32_t {
    auto it = leaves.find(pack(L, x, y, z));
    return it == leaves.end() ? -1 : it->second;
  };

  std::unordered_map<uint64_t, int32_t> nodes;
  int32_t n_nodes = 0;
  for (int32_t i = 0; i < n_leaves; ++i) {
    const int32_t L = leaf_coord[4 * i];
    const int32_t blocks = base << L;
    for (int32_t s = 0; s < 27; ++s) {
      const int32_t d[3] = {s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1};
      int32_t b[3];
      for (int k = 0; k < 3; ++k) b[k] = pmod(leaf_coord[4 * i + 1 + k] + d[k], blocks);
      int32_t id = leaf_at(L, b[0], b[1], b[2]);
      if (id >= 0) {
        nbr[27 * i + s] = id;
        kind[27 * i + s] = HYDRO_SAME_LEAF;
        continue;
      }
      if (L > 0 && (id = leaf_at(L - 1, b[0] >> 1, b[1] >> 1, b[2] >> 1)) >= 0) {
        nbr[27 * i + s] = id;
        kind[27 * i + s] = HYDRO_COARSER_LEAF;
        continue;
      }
      // refined neighbour block: its children are the source cells
      const uint64_t key = pack(L, b[0], b[1], b[2]);
      auto it = nodes.find(key);
      int32_t node;
      if (it == nodes.end()) {
        if (n_nodes >= max_nodes)
          return octohydro::fail(HYDRO_E_TABLE, "hydro_build_table: more than %d refined nodes",
                                 max_nodes);
        node = n_nodes++;
        nodes.emplace(key, node);
        for (int32_t c = 0; c < 8; ++c)
          children[8 * node + c] =
              leaf_at(L + 1, 2 * b[0] + (c & 1), 2 * b[1] + ((c >> 1) & 1), 2 * b[2] + (c >> 2));
      } else {
        node = it->second;
      }
      // The halo is 3 cells deep: it only touches the children on the near
      // side of the node (child bit 1 when the node lies below, 0 above).
      for (int32_t c = 0; c < 8; ++c) {
        const int32_t bit[3] = {c & 1, (c >> 1) & 1, c >> 2};
        bool touched = true;
        for (int k = 0; k < 3; ++k)
          if (d[k] != 0 && bit[k] != (d[k] < 0 ? 1 : 0)) touched = false;
        if (touched && children[8 * node + c] < 0)
          return octohydro::fail(HYDRO_E_TABLE,
                                 "hydro_build_table: leaf %d slot %d: tree is not 2:1 balanced", i,
                                 s);
      }
      nbr[27 * i + s] = node;
      kind[27 * i + s] = HYDRO_SAME_REFINED;
    }
  }
  *n_nodes_out = n_nodes;
  return HYDRO_OK;
}

// Flux-register tables for the coarse-fine flux correction.  Face
// orientation o = 2*d + side (d = axis, side 0 = low face, 1 = high face).
// A coarse leaf whose face o borders a refined block owns one register slot
// for that face; slots are numbered orientation by orientation, leaves
// ascending within one orientation.  A fine leaf whose face o borders a
// coarser leaf writes its fluxes into the coarse leaf's slot for the
// opposite face, in the quadrant given by its coordinate parities along the
// face's two axes (u, v in increasing axis order).
extern "C" int hydro_build_reflux(int32_t n_leaves, const int32_t* leaf_coord,
                                  const int32_t* nbr, const uint8_t* kind,
                                  int32_t* face_slot, int32_t* fine_slot, int32_t* slot_leaf,
                                  int32_t max_slots, int32_t* orient_begin,
                                  int32_t* n_slots_out) {
  octohydro::clear_error();
  if (n_leaves <= 0 || !leaf_coord || !nbr || !kind || !face_slot || !fine_slot || !slot_leaf ||
      !orient_begin || !n_slots_out || max_slots < 0)
    return octohydro::fail(HYDRO_E_ARG, "hydro_build_reflux: bad argument");
  // face orientation o -> slot of the face neighbour in the 27-slot table
  auto nslot = [](int o) {
    const int d = o >> 1, s = (o & 1) ? 1 : -1;
    int r[3] = {0, 0, 0};
    r[d] = s;
    return (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
  };
  int32_t n_slots = 0;
  for (int o = 0; o < 6; ++o) {
    orient_begin[o] = n_slots;
    for (int32_t i = 0; i < n_leaves; ++i) {
      face_slot[6 * i + o] = -1;
      if (kind[27 * i + nslot(o)] == HYDRO_SAME_REFINED) {
        if (n_slots >= max_slots)
          return octohydro::fail(HYDRO_E_ARG, "hydro_build_reflux: more than %d slots",
                                 max_slots);
        slot_leaf[n_slots] = i;
        face_slot[6 * i + o] = n_slots++;
      }
    }
  }
  orient_begin[6] = n_slots;
  for (int32_t i = 0; i < n_leaves; ++i)
    for (int o = 0; o < 6; ++o) {
      fine_slot[6 * i + o] = -1;
      if (kind[27 * i + nslot(o)] != HYDRO_COARSER_LEAF) continue;
      const int32_t c = nbr[27 * i + nslot(o)];
      const int32_t cs = (c >= 0 && c < n_leaves) ? face_slot[6 * c + (o ^ 1)] : -1;
      if (cs < 0)
        return octohydro::fail(HYDRO_E_TABLE,
                               "hydro_build_reflux: leaf %d face %d has no matching coarse face",
                               i, o);
      const int d = o >> 1;
      const int au = d == 0 ? 1 : 0, av = d == 2 ? 1 : 2;  // axes u < v other than d
      const int qu = leaf_coord[4 * i + 1 + au] & 1, qv = leaf_coord[4 * i + 1 + av] & 1;
      fine_slot[6 * i + o] = (cs << 2) | (qu + 2 * qv);
    }
  *n_slots_out = n_slots;
  return HYDRO_OK;
}

// Inverse of the children table: the node and octant of every child leaf.
extern "C" int hydro_build_leaf_node(int32_t n_leaves, int32_t n_nodes, const int32_t* children,
                                     int32_t* leaf_node) {
  octohydro::clear_error();
  if (n_leaves <= 0 || n_nodes < 0 || !leaf_node || (n_nodes > 0 && !children))
    return octohydro::fail(HYDRO_E_ARG, "hydro_build_leaf_node: bad arguments");
  for (int32_t i = 0; i < n_leaves; ++i) leaf_node[i] = -1;
  for (int32_t n = 0; n < n_nodes; ++n)
    for (int o = 0; o < 8; ++o) {
      const int32_t c = children[8 * n + o];
      if (c < 0) continue;
      if (c >= n_leaves)
        return octohydro::fail(HYDRO_E_TABLE, "hydro_build_leaf_node: child %d out of range", c);
      if (leaf_node[c] >= 0)
        return octohydro::fail(HYDRO_E_TABLE, "hydro_build_leaf_node: leaf %d listed twice", c);
      leaf_node[c] = 8 * n + o;
    }
  return HYDRO_OK;
}
