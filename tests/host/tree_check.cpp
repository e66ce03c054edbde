// Host-side check of the octree and the interaction lists, built with the
// address and undefined-behaviour sanitizers by tests/test_tree_sanitized.py.
// For seeded point sets (uniform cube, sphere shell, a flat plate, repeated
// points) and several leaf sizes it checks:
//  * the panel permutation is a permutation, every box owns a contiguous
//    range that its children partition, and leaves hold at most ncrit panels
//    unless their panels cannot be separated (all at one point);
//  * every collocation and Gauss point lies inside its box's spheres;
//  * for target groups taken from the leaves, the P2P leaves and M2P boxes
//    of every source tree cover each source panel exactly once, and every
//    M2P box passes the acceptance test for every target of the group.
// Prints one line per failure and exits non-zero if there was any.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1506_03745_amd/csrc/tree.h"

using pbt::SurfTree;
using pbt::TreeBox;

static int failures = 0;
#define CHECK(c, ...)                        \
  do {                                       \
    if (!(c)) {                              \
      ++failures;                            \
      std::printf("FAIL %s: ", #c);          \
      std::printf(__VA_ARGS__);              \
      std::printf("\n");                     \
    }                                        \
  } while (0)

static std::vector<double> points(int kind, int n, uint32_t seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> p(3 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    double* q = &p[3 * (size_t)i];
    if (kind == 0) {          // uniform cube
      for (int d = 0; d < 3; ++d) q[d] = 10.0 * u(g);
    } else if (kind == 1) {   // sphere shell of radius 4
      double a = nd(g), b = nd(g), c = nd(g), s = std::sqrt(a * a + b * b + c * c);
      q[0] = 4.0 * a / s;
      q[1] = 4.0 * b / s;
      q[2] = 4.0 * c / s;
    } else if (kind == 2) {   // flat plate
      q[0] = 40.0 * u(g);
      q[1] = 40.0 * u(g);
      q[2] = 0.0;
    } else {                  // a few repeated points
      const int k = i % 3;
      q[0] = k;
      q[1] = 2.0 * k;
      q[2] = -k;
    }
  }
  return p;
}

static void check_tree(const SurfTree& t, const std::vector<double>& cen, const std::vector<double>& src, int nt,
                       int K, int ncrit, const char* name) {
  std::vector<int> seen(nt, 0);
  CHECK((int)t.perm.size() == nt, "%s perm size", name);
  for (int32_t o : t.perm) {
    CHECK(o >= 0 && o < nt, "%s perm entry %d", name, o);
    if (o >= 0 && o < nt) ++seen[o];
  }
  for (int i = 0; i < nt; ++i) CHECK(seen[i] == 1, "%s panel %d appears %d times", name, i, seen[i]);
  CHECK(!t.boxes.empty() && t.boxes[0].pbeg == 0 && t.boxes[0].pend == nt, "%s root range", name);
  for (size_t bi = 0; bi < t.boxes.size(); ++bi) {
    const TreeBox& b = t.boxes[bi];
    CHECK(0 <= b.pbeg && b.pbeg <= b.pend && b.pend <= nt, "%s box %zu range", name, bi);
    if (b.leaf) {
      bool same = true;
      for (int k = b.pbeg + 1; k < b.pend; ++k)
        for (int d = 0; d < 3; ++d) same = same && cen[3 * (size_t)k + d] == cen[3 * (size_t)b.pbeg + d];
      CHECK(b.pend - b.pbeg <= ncrit || same, "%s leaf %zu holds %d > %d", name, bi, b.pend - b.pbeg, ncrit);
    } else {
      int32_t at = b.pbeg;
      CHECK(b.child_beg < b.child_end, "%s inner box %zu without children", name, bi);
      for (int c = b.child_beg; c < b.child_end; ++c) {
        const TreeBox& ch = t.boxes[t.child_list[c]];
        CHECK(ch.pbeg == at && ch.parent == (int32_t)bi, "%s child of %zu out of order", name, bi);
        at = ch.pend;
      }
      CHECK(at == b.pend, "%s children of %zu do not cover it", name, bi);
    }
    for (int k = b.pbeg; k < b.pend; ++k) {
      const double* x = &cen[3 * (size_t)k];
      const double dt = std::sqrt((x[0] - b.tc[0]) * (x[0] - b.tc[0]) + (x[1] - b.tc[1]) * (x[1] - b.tc[1]) +
                                  (x[2] - b.tc[2]) * (x[2] - b.tc[2]));
      CHECK(dt <= b.tr * (1 + 1e-12) + 1e-12, "%s target %d outside box %zu", name, k, bi);
      for (int q = 0; q < K; ++q) {
        const double* y = &src[3 * ((size_t)k * K + q)];
        const double ds = std::sqrt((y[0] - b.c[0]) * (y[0] - b.c[0]) + (y[1] - b.c[1]) * (y[1] - b.c[1]) +
                                    (y[2] - b.c[2]) * (y[2] - b.c[2]));
        CHECK(ds <= b.r * (1 + 1e-12) + 1e-12, "%s source %d.%d outside box %zu", name, k, q, bi);
      }
    }
  }
}

int main() {
  const int K = 3;
  int cases = 0;
  for (int kind = 0; kind < 4; ++kind)
    for (int nt : {1, 7, 300, 301, 4000})
      for (int ncrit : {1, 8, 300}) {
        char name[64];
        std::snprintf(name, sizeof name, "kind %d n %d ncrit %d", kind, nt, ncrit);
        const std::vector<double> c0 = points(kind, nt, 17u + 31u * kind + (uint32_t)nt);
        SurfTree t = pbt::build_tree(c0.data(), nt, ncrit);
        // centroids and Gauss points in the internal order (points offset
        // by a small fixed triangle around each centroid)
        std::vector<double> cen(3 * (size_t)nt), src(3 * (size_t)nt * K);
        const double off[3][3] = {{0.05, 0, 0}, {0, 0.05, 0}, {-0.03, -0.03, 0.01}};
        for (int i = 0; i < nt; ++i)
          for (int d = 0; d < 3; ++d) {
            cen[3 * (size_t)i + d] = c0[3 * (size_t)t.perm[i] + d];
            for (int q = 0; q < K; ++q) src[3 * ((size_t)i * K + q) + d] = cen[3 * (size_t)i + d] + off[q][d];
          }
        pbt::tree_geometry(t, cen.data(), src.data(), K);
        check_tree(t, cen, src, nt, K, ncrit, name);
        // interaction lists of every leaf of a second tree against this one
        const std::vector<double> c1 = points((kind + 1) % 3, 600, 99u + (uint32_t)kind);
        SurfTree tt = pbt::build_tree(c1.data(), 600, 40);
        std::vector<double> tcen(3 * 600), tsrc(3 * 600 * K);
        for (int i = 0; i < 600; ++i)
          for (int d = 0; d < 3; ++d) {
            tcen[3 * (size_t)i + d] = c1[3 * (size_t)tt.perm[i] + d];
            for (int q = 0; q < K; ++q) tsrc[3 * ((size_t)i * K + q) + d] = tcen[3 * (size_t)i + d] + off[q][d];
          }
        pbt::tree_geometry(tt, tcen.data(), tsrc.data(), K);
        for (double theta : {0.3, 0.5, 0.8})
          for (const TreeBox& tl : tt.boxes) {
            if (!tl.leaf) continue;
            std::vector<int> pb, mb;
            pbt::interaction_lists(t, tl, theta, pb, mb);
            std::vector<int> cover(nt, 0);
            for (int b : pb) {
              CHECK(t.boxes[b].leaf, "%s P2P box %d is not a leaf", name, b);
              for (int k = t.boxes[b].pbeg; k < t.boxes[b].pend; ++k) ++cover[k];
            }
            for (int b : mb) {
              const TreeBox& B = t.boxes[b];
              for (int k = B.pbeg; k < B.pend; ++k) ++cover[k];
              for (int k = tl.pbeg; k < tl.pend; ++k) {
                const double* x = &tcen[3 * (size_t)k];
                const double d = std::sqrt((x[0] - B.c[0]) * (x[0] - B.c[0]) + (x[1] - B.c[1]) * (x[1] - B.c[1]) +
                                           (x[2] - B.c[2]) * (x[2] - B.c[2]));
                CHECK(B.r < theta * d, "%s M2P box %d fails the acceptance test for target %d", name, b, k);
              }
            }
            for (int k = 0; k < nt; ++k) CHECK(cover[k] == 1, "%s source panel %d covered %d times", name, k, cover[k]);
          }
        ++cases;
      }
  std::printf("%d cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
