// Octree over the panels of one surface and the treecode interaction lists
// (Section 3.2: boxes of at most N_crit elements, Taylor far field accepted
// by a multipole-acceptance criterion theta, direct sums otherwise).
//
// Boxes are cubes split into octants while they hold more than N_crit
// panels; panels are reordered so that every box owns a contiguous range,
// and inside a leaf by finer octants (its 32-panel runs are compact).
// Expansion centre of a box: centre of the bounding box of its Gauss points;
// radius: the largest distance from that centre to one of them.  A target
// group T (a run of at most 32 collocation points of one leaf) accepts a
// source box B for the far field when
//     r_B < theta * (|c_T - c_B| - r_T),
// r_T being the radius of T's collocation points about their own centre, so
// that every target x in T satisfies r_B / |x - c_B| < theta.
#include "tree.h"

#include <algorithm>
#include <cmath>

namespace pbt {

namespace {

// Orders idx[beg, end) by recursive octants of the cube (c, half) down to
// groups of at most 8 points, so that consecutive runs of a leaf's panels
// (the 32-target groups the work is cut into) are spatially compact.
void order_octants(const double* cen, std::vector<int32_t>& idx, int beg, int end, const double c[3], double half,
                   int depth) {
  if (end - beg <= 8 || depth >= 20) return;
  int cnt[8] = {0};
  std::vector<int8_t> oct(end - beg);
  for (int i = beg; i < end; ++i) {
    const double* p = cen + 3 * (int64_t)idx[i];
    const int o = (p[0] > c[0] ? 1 : 0) | (p[1] > c[1] ? 2 : 0) | (p[2] > c[2] ? 4 : 0);
    oct[i - beg] = (int8_t)o;
    ++cnt[o];
  }
  int start[8], pos[8];
  start[0] = beg;
  for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
  for (int o = 0; o < 8; ++o) pos[o] = start[o] - beg;
  std::vector<int32_t> tmp(end - beg);
  for (int i = beg; i < end; ++i) tmp[pos[oct[i - beg]]++] = idx[i];
  std::copy(tmp.begin(), tmp.end(), idx.begin() + beg);
  for (int o = 0; o < 8; ++o) {
    if (cnt[o] == 0) continue;
    const double h2 = half * 0.5;
    const double cc[3] = {c[0] + ((o & 1) ? h2 : -h2), c[1] + ((o & 2) ? h2 : -h2), c[2] + ((o & 4) ? h2 : -h2)};
    order_octants(cen, idx, start[o], start[o] + cnt[o], cc, h2, depth + 1);
  }
}

void build_rec(SurfTree& t, const double* cen, std::vector<int32_t>& idx, int box, int beg, int end,
               const double c[3], double half, int level, int ncrit) {
  TreeBox& b = t.boxes[box];
  b.pbeg = beg;
  b.pend = end;
  b.level = level;
  if (end - beg <= ncrit || level >= 40) {
    b.leaf = true;
    order_octants(cen, idx, beg, end, c, half, 0);
    return;
  }
  // Counting partition into octants.
  int cnt[8] = {0};
  std::vector<int8_t> oct(end - beg);
  for (int i = beg; i < end; ++i) {
    const double* p = cen + 3 * (int64_t)idx[i];
    const int o = (p[0] > c[0] ? 1 : 0) | (p[1] > c[1] ? 2 : 0) | (p[2] > c[2] ? 4 : 0);
    oct[i - beg] = (int8_t)o;
    ++cnt[o];
  }
  int start[8];
  start[0] = beg;
  for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
  std::vector<int32_t> tmp(end - beg);
  int pos[8];
  for (int o = 0; o < 8; ++o) pos[o] = start[o] - beg;
  for (int i = beg; i < end; ++i) tmp[pos[oct[i - beg]]++] = idx[i];
  std::copy(tmp.begin(), tmp.end(), idx.begin() + beg);
  b.leaf = false;
  b.child_beg = (int32_t)t.child_list.size();
  std::vector<int> kids;
  for (int o = 0; o < 8; ++o) {
    if (cnt[o] == 0) continue;
    TreeBox nb;
    nb.parent = box;
    t.boxes.push_back(nb);
    kids.push_back((int)t.boxes.size() - 1);
  }
  for (int k : kids) t.child_list.push_back(k);
  t.boxes[box].child_end = (int32_t)t.child_list.size();
  int ki = 0;
  for (int o = 0; o < 8; ++o) {
    if (cnt[o] == 0) continue;
    const double h2 = half * 0.5;
    const double cc[3] = {c[0] + ((o & 1) ? h2 : -h2), c[1] + ((o & 2) ? h2 : -h2),
                          c[2] + ((o & 4) ? h2 : -h2)};
    build_rec(t, cen, idx, kids[ki++], start[o], start[o] + cnt[o], cc, h2, level + 1, ncrit);
  }
}

void sphere_of(const double* pts, int64_t beg, int64_t end, double c[3], double* r) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = beg; i < end; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], pts[3 * i + d]);
      hi[d] = std::max(hi[d], pts[3 * i + d]);
    }
  for (int d = 0; d < 3; ++d) c[d] = 0.5 * (lo[d] + hi[d]);
  double r2 = 0.0;
  for (int64_t i = beg; i < end; ++i) {
    const double dx = pts[3 * i] - c[0], dy = pts[3 * i + 1] - c[1], dz = pts[3 * i + 2] - c[2];
    r2 = std::max(r2, dx * dx + dy * dy + dz * dz);
  }
  *r = std::sqrt(r2) * (1.0 + 1e-12);
}

}  // namespace

SurfTree build_tree(const double* cen, int64_t nt, int ncrit) {
  SurfTree t;
  std::vector<int32_t> idx(nt);
  for (int64_t i = 0; i < nt; ++i) idx[i] = (int32_t)i;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < nt; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], cen[3 * i + d]);
      hi[d] = std::max(hi[d], cen[3 * i + d]);
    }
  double c[3], half = 0.0;
  for (int d = 0; d < 3; ++d) {
    c[d] = 0.5 * (lo[d] + hi[d]);
    half = std::max(half, 0.5 * (hi[d] - lo[d]));
  }
  half = half * (1.0 + 1e-9) + 1e-12;
  t.boxes.push_back(TreeBox{});
  t.boxes[0].parent = -1;
  build_rec(t, cen, idx, 0, 0, (int)nt, c, half, 0, ncrit);
  t.perm = std::move(idx);
  return t;
}

void tree_geometry(SurfTree& t, const double* tgt_local, const double* src_local, int K) {
  for (TreeBox& b : t.boxes) {
    sphere_of(src_local, (int64_t)b.pbeg * K, (int64_t)b.pend * K, b.c, &b.r);
    sphere_of(tgt_local, b.pbeg, b.pend, b.tc, &b.tr);
  }
}

void interaction_lists(const SurfTree& src, const TreeBox& tleaf, double theta,
                       std::vector<int>& p2p_boxes, std::vector<int>& m2p_boxes) {
  std::vector<int> stack{0};
  while (!stack.empty()) {
    const int bi = stack.back();
    stack.pop_back();
    const TreeBox& b = src.boxes[bi];
    const double dx = tleaf.tc[0] - b.c[0], dy = tleaf.tc[1] - b.c[1], dz = tleaf.tc[2] - b.c[2];
    const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (b.r < theta * (d - tleaf.tr)) {
      m2p_boxes.push_back(bi);
    } else if (b.leaf) {
      p2p_boxes.push_back(bi);
    } else {
      for (int k = b.child_end - 1; k >= b.child_beg; --k) stack.push_back(src.child_list[k]);
    }
  }
}

}  // namespace pbt
