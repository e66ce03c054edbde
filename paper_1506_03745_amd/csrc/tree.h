// Host-side octree of one surface and treecode interaction lists.
#pragma once

#include <cstdint>
#include <vector>

namespace pbt {

struct TreeBox {
  double c[3] = {0, 0, 0};   // expansion centre (Gauss points)
  double r = 0.0;            // radius about c of the Gauss points
  double tc[3] = {0, 0, 0};  // centre of the collocation points
  double tr = 0.0;           // radius about tc of the collocation points
  int32_t pbeg = 0, pend = 0;          // panel range (surface-local internal order)
  int32_t child_beg = 0, child_end = 0; // range in child_list
  int32_t parent = -1;
  int32_t level = 0;
  bool leaf = true;
};

struct SurfTree {
  std::vector<TreeBox> boxes;    // boxes[0] is the root
  std::vector<int32_t> child_list;
  std::vector<int32_t> perm;     // internal position -> original panel index
};

// Builds the tree from panel centroids given in the original order.
SurfTree build_tree(const double* cen, int64_t nt, int ncrit);

// Sets centres and radii; tgt_local: nt x 3 collocation points and
// src_local: (nt*K) x 3 Gauss points, both in the tree's internal order.
void tree_geometry(SurfTree& t, const double* tgt_local, const double* src_local, int K);

// Source boxes of tree `src` that the targets of `tleaf` (a target group:
// its collocation-point sphere tc, tr) evaluate directly (leaves) or
// through their expansions.
void interaction_lists(const SurfTree& src, const TreeBox& tleaf, double theta,
                       std::vector<int>& p2p_boxes, std::vector<int>& m2p_boxes);

}  // namespace pbt
