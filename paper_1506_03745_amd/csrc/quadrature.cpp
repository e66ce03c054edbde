// Quadrature tables of the library (Section 3.1): symmetric triangle rules
// for the far (1, 3, 4, 7 points) and near (19 points) regimes, and
// Gauss-Legendre rules along the edges of the self panel.
//
// Triangle rules are the published symmetric rules: centroid (degree 1);
// the interior 3-point rule (2/3, 1/6, 1/6) (degree 2); Strang & Fix's
// 4-point rule (degree 3); Radon's 7-point rule (degree 5); Dunavant's
// 19-point rule (degree 9).  Gauss-Legendre nodes are found by Newton's
// method on the three-term recurrence of the Legendre polynomials.
#include "quadrature.h"

#include <cmath>
#include <stdexcept>

namespace pbt {

namespace {

void add_s3(std::vector<double>& b, std::vector<double>& w, double wt) {
  b.insert(b.end(), {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0});
  w.push_back(wt);
}

// (1-2a, a, a) and its rotations
void add_s21(std::vector<double>& b, std::vector<double>& w, double a, double wt) {
  const double c = 1.0 - 2.0 * a;
  b.insert(b.end(), {c, a, a, a, c, a, a, a, c});
  w.insert(w.end(), {wt, wt, wt});
}

// the six permutations of (a, b, 1-a-b)
void add_s111(std::vector<double>& bb, std::vector<double>& w, double a, double b, double wt) {
  const double c = 1.0 - a - b;
  bb.insert(bb.end(), {a, b, c, b, c, a, c, a, b, a, c, b, c, b, a, b, a, c});
  w.insert(w.end(), {wt, wt, wt, wt, wt, wt});
}

}  // namespace

bool triangle_rule(int npts, std::vector<double>& bary, std::vector<double>& w) {
  bary.clear();
  w.clear();
  switch (npts) {
    case 1:
      add_s3(bary, w, 1.0);
      break;
    case 3:
      add_s21(bary, w, 1.0 / 6.0, 1.0 / 3.0);
      break;
    case 4:
      add_s3(bary, w, -27.0 / 48.0);
      add_s21(bary, w, 0.2, 25.0 / 48.0);
      break;
    case 7: {
      const double r = std::sqrt(15.0);
      add_s3(bary, w, 9.0 / 40.0);
      add_s21(bary, w, (6.0 - r) / 21.0, (155.0 - r) / 1200.0);
      add_s21(bary, w, (6.0 + r) / 21.0, (155.0 + r) / 1200.0);
      break;
    }
    case 19:
      add_s3(bary, w, 0.097135796282799);
      add_s21(bary, w, 0.489682519198738, 0.031334700227139);
      add_s21(bary, w, 0.437089591492937, 0.077827541004774);
      add_s21(bary, w, 0.188203535619033, 0.079647738927210);
      add_s21(bary, w, 0.044729513394453, 0.025577675658698);
      add_s111(bary, w, 0.036838412054736, 0.221962989160766, 0.043283539377289);
      break;
    default:
      return false;
  }
  return true;
}

void gauss_legendre01(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(pi * (i + 0.75) / (n + 0.5));  // initial guess for the i-th root
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 0 ? 1.0 : p1;
      const double pm = n == 1 ? 1.0 : p0;
      dp = n * (x * pn - pm) / (x * x - 1.0);
      const double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = 0.5 * (1.0 - x);                         // map [-1, 1] -> [0, 1]
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);         // 2/((1-x^2) P_n'^2) scaled by 1/2
  }
}

}  // namespace pbt
