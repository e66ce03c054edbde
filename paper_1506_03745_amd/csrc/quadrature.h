#pragma once
#include <vector>

namespace pbt {
// Barycentric coordinates (3 per point) and weights summing to 1; false if
// there is no rule with npts points.
bool triangle_rule(int npts, std::vector<double>& bary, std::vector<double>& w);
// n-point Gauss-Legendre nodes and weights on [0, 1].
void gauss_legendre01(int n, std::vector<double>& t, std::vector<double>& w);
}  // namespace pbt
