// Setup kernels: panel geometry, Gauss-point sources, the near/far decision
// and the near-field and self-panel corrections (Section 3.1).
//
// The near test |x - c_j| < 2 L_j, L_j = sqrt(2 A_j), decides an integer
// outcome from floating point, so it is evaluated as a fixed sequence of
// correctly rounded FP64 operations with contraction disabled:
//   d2 = (dx*dx + dy*dy) + dz*dz,  near  <=>  d2*d2 < 16 |e1 x e2|^2
// (|e1 x e2| = 2 A_j, so 4 L_j^2 = 4 |e1 x e2|).
#include "pbt_internal.h"

#include <algorithm>

namespace pbt {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

__global__ void k_panel_geometry(int64_t np, const double* __restrict__ tri9, double* cen,
                                 double* nrm, double* area, double* cross2) {
#pragma clang fp contract(off)
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double* v = tri9 + 9 * i;
  const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
  const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
  const double cx = e1y * e2z - e1z * e2y;
  const double cy = e1z * e2x - e1x * e2z;
  const double cz = e1x * e2y - e1y * e2x;
  const double c2 = (cx * cx + cy * cy) + cz * cz;
  const double cn = sqrt(c2);
  cross2[i] = c2;
  area[i] = 0.5 * cn;
  nrm[3 * i + 0] = cx / cn;
  nrm[3 * i + 1] = cy / cn;
  nrm[3 * i + 2] = cz / cn;
  const double third = 1.0 / 3.0;
  cen[3 * i + 0] = ((v[0] + v[3]) + v[6]) * third;
  cen[3 * i + 1] = ((v[1] + v[4]) + v[7]) * third;
  cen[3 * i + 2] = ((v[2] + v[5]) + v[8]) * third;
}

// A Gauss point at the barycentre is computed exactly as the collocation
// point (k_panel_geometry), so that the self pair of the rules that contain
// it has r = 0 bit for bit and is skipped by the interaction kernels.
__device__ __forceinline__ void rule_point(const double* v, double b0, double b1, double b2,
                                           double* p) {
#pragma clang fp contract(off)
  const double third = 1.0 / 3.0;
  if (b0 == third && b1 == third && b2 == third) {
    for (int d = 0; d < 3; ++d) p[d] = ((v[d] + v[3 + d]) + v[6 + d]) * third;
  } else {
    for (int d = 0; d < 3; ++d) p[d] = (b0 * v[d] + b1 * v[3 + d]) + b2 * v[6 + d];
  }
}

__global__ void k_sources(int64_t np, int K, const double* __restrict__ tri9,
                          const double* __restrict__ area, const double* __restrict__ bary,
                          const double* __restrict__ w, double* src_pos, double* src_wa) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= np * K) return;
  const int64_t p = j / K;
  const int q = (int)(j - p * K);
  const double* v = tri9 + 9 * p;
  rule_point(v, bary[3 * q], bary[3 * q + 1], bary[3 * q + 2], src_pos + 3 * j);
  src_wa[j] = w[q] * area[p];
}

// |x - c| < f L with L = sqrt(2 A) = sqrt(|e1 x e2|), i.e. d^4 < f^4 |e1 x e2|^2
// (f4 = (f f)(f f), 16 for the paper's 2L), in one fixed sequence of
// correctly rounded FP64 operations.
__device__ __forceinline__ bool is_near(double tx, double ty, double tz, double cx, double cy,
                                        double cz, double c2, double f4) {
#pragma clang fp contract(off)
  const double dx = tx - cx, dy = ty - cy, dz = tz - cz;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  return (d2 * d2) < f4 * c2;
}

// One wavefront per target, lanes over panels.  The fill pass writes the
// hits of each 64-panel chunk in panel order (ballot + popcount), so the
// lists come out sorted exactly as a serial scan would produce them.  A
// target scans either every panel [0, np) (tleaf null) or the candidate
// panel ranges of its leaf, lrange[2r] .. lrange[2r+1] for r in
// lptr[tleaf[i]] .. lptr[tleaf[i]+1] (increasing and disjoint): the panels
// left out lie provably farther than the near distance, so both give the
// same lists.
template <bool FILL>
__global__ __launch_bounds__(256) void k_near(int64_t nt, const double* __restrict__ tx, int64_t np,
                                              const double* __restrict__ cen,
                                              const double* __restrict__ cross2,
                                              const int32_t* __restrict__ tleaf,
                                              const int64_t* __restrict__ lptr,
                                              const int64_t* __restrict__ lrange, double f4, int32_t* count,
                                              const int64_t* __restrict__ rowptr, int32_t* col) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= nt) return;  // uniform across the wavefront
  const double x = tx[3 * i], y = tx[3 * i + 1], z = tx[3 * i + 2];
  int64_t out = FILL ? rowptr[i] : 0;
  int32_t cnt = 0;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t r0 = tleaf ? lptr[tleaf[i]] : 0, r1 = tleaf ? lptr[tleaf[i] + 1] : 1;
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t jb = tleaf ? lrange[2 * r] : 0, je = tleaf ? lrange[2 * r + 1] : np;
    for (int64_t j0 = jb; j0 < je; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool hit = j < je && is_near(x, y, z, cen[3 * j], cen[3 * j + 1], cen[3 * j + 2], cross2[j], f4);
      const uint64_t m = __ballot(hit);
      if (FILL) {
        if (hit) col[out + __popcll(m & below)] = (int32_t)j;
        out += __popcll(m);
      } else {
        cnt += __popcll(m);
      }
    }
  }
  if (!FILL && lane == 0) count[i] = cnt;
}

// Target and source records from the device geometry: targets (x, y, z, 0),
// sources (x, y, z, 0, 0, 0, 0, 0) in FP64 and FP32 (strengths are written
// per product).
__global__ void k_pack_points(int64_t np, int64_t ns, const double* __restrict__ cen,
                              const double* __restrict__ src_pos, double* t64, float* t32, double* s64,
                              float* s32) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < np) {
    for (int d = 0; d < 3; ++d) {
      t64[4 * i + d] = cen[3 * i + d];
      t32[4 * i + d] = (float)cen[3 * i + d];
    }
    t64[4 * i + 3] = 0.0;
    t32[4 * i + 3] = 0.0f;
  }
  if (i < ns) {
    for (int d = 0; d < 8; ++d) {
      const double v = d < 3 ? src_pos[3 * i + d] : 0.0;
      s64[8 * i + d] = v;
      s32[8 * i + d] = (float)v;
    }
  }
}

struct K4 {
  double vl, kl, vy, ky;
};

// The K-point (or any) rule on panel j seen from x, exactly as the direct
// FP64 interaction kernel sums it (points at distance 0 contribute 0).
__device__ K4 rule_on_panel(double x, double y, double z, const double* v, const double* n,
                            double area, int npts, const double* bary, const double* w,
                            double kappa) {
  K4 r{0, 0, 0, 0};
  for (int q = 0; q < npts; ++q) {
    double sp[3];
    rule_point(v, bary[3 * q], bary[3 * q + 1], bary[3 * q + 2], sp);
    const double dx = x - sp[0], dy = y - sp[1], dz = z - sp[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0)) continue;
    const double rinv = rsqrt(r2);
    const double rr = r2 * rinv;
    const double wa = w[q] * area;
    const double nd = n[0] * dx + n[1] * dy + n[2] * dz;
    const double gl = rinv;
    const double kl = nd * rinv * rinv * rinv;
    const double e = exp(-kappa * rr);
    r.vl += wa * gl;
    r.kl += wa * kl;
    r.vy += wa * gl * e;
    r.ky += wa * kl * (1.0 + kappa * rr) * e;
  }
  r.vl *= kInv4Pi; r.kl *= kInv4Pi; r.vy *= kInv4Pi; r.ky *= kInv4Pi;
  return r;
}

// Single-layer integrals over panel j at a point x inside it: polar
// coordinates about x, radial integral of G rho in closed form,
// g_L(rho) = rho/(4 pi), g_Y(rho) = (1 - exp(-kappa rho))/(4 pi kappa), and the
// angle element along each edge h l dt / rho^2 by Gauss-Legendre in t.
__device__ void self_single_layer(double x, double y, double z, const double* v, int nedge,
                                  const double* gt, const double* gw, double kappa, double* vl,
                                  double* vy) {
  double sl = 0.0, sy = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3;
    const double px = v[3 * a], py = v[3 * a + 1], pz = v[3 * a + 2];
    const double ex = v[3 * b] - px, ey = v[3 * b + 1] - py, ez = v[3 * b + 2] - pz;
    const double ell = sqrt(ex * ex + ey * ey + ez * ez);
    const double ax = px - x, ay = py - y, az = pz - z;
    const double cx = ay * ez - az * ey, cy = az * ex - ax * ez, cz = ax * ey - ay * ex;
    const double h = sqrt(cx * cx + cy * cy + cz * cz) / ell;
    for (int q = 0; q < nedge; ++q) {
      const double t = gt[q];
      const double rx = ax + t * ex, ry = ay + t * ey, rz = az + t * ez;
      const double rho = sqrt(rx * rx + ry * ry + rz * rz);
      const double ang = gw[q] * h * ell / (rho * rho);
      sl += ang * rho;
      sy += ang * (kappa > 0.0 ? -expm1(-kappa * rho) / kappa : rho);
    }
  }
  *vl = sl * kInv4Pi;
  *vy = sy * kInv4Pi;
}

__global__ void k_near_values(int64_t nt, const double* __restrict__ tx,
                              const int32_t* __restrict__ tgt_self, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, const double* __restrict__ tri9,
                              const double* __restrict__ nrm, const double* __restrict__ area,
                              NearParams p, double* vals, const int32_t* __restrict__ skip) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nt || (skip && skip[i] >= 0)) return;
  const double x = tx[3 * i], y = tx[3 * i + 1], z = tx[3 * i + 2];
  const int32_t self = tgt_self ? tgt_self[i] : -1;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int32_t j = col[e];
    const double* v = tri9 + 9 * (int64_t)j;
    const double* n = nrm + 3 * (int64_t)j;
    const K4 coarse = rule_on_panel(x, y, z, v, n, area[j], p.K, p.bary_far, p.w_far, p.kappa);
    K4 fine;
    if (j == self) {
      self_single_layer(x, y, z, v, p.Nedge, p.gl_t, p.gl_w, p.kappa, &fine.vl, &fine.vy);
      fine.kl = 0.0;
      fine.ky = 0.0;
    } else {
      fine = rule_on_panel(x, y, z, v, n, area[j], p.Knear, p.bary_near, p.w_near, p.kappa);
    }
    vals[4 * e + 0] = fine.vl - coarse.vl;
    vals[4 * e + 1] = fine.kl - coarse.kl;
    vals[4 * e + 2] = fine.vy - coarse.vy;
    vals[4 * e + 3] = fine.ky - coarse.ky;
  }
}

__global__ void k_coulomb_rhs(int64_t n, const double* __restrict__ tx, const int32_t* __restrict__ rows,
                              int64_t nq, const double* __restrict__ qxyz, const double* __restrict__ q,
                              double inv_eps, double* b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = tx[3 * i], y = tx[3 * i + 1], z = tx[3 * i + 2];
  double s = 0.0;
  for (int64_t k = 0; k < nq; ++k) {
    const double dx = x - qxyz[3 * k], dy = y - qxyz[3 * k + 1], dz = z - qxyz[3 * k + 2];
    s += q[k] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  b[rows[i]] = s * kInv4Pi * inv_eps;
}

// Fold the per-row factors into the corrections.  forms[t * nsurf + s]
// says in which form target surface t's two rows (bits 0-1: interior row,
// bits 2-3: outside row) see source surface s: 0 not at all, 1 from inside
// (Laplace, factors -(eps_outside/eps_s) on the single layer and -1 on the
// double layer), 2 from outside with the Yukawa kernel (the raw Yukawa
// values), 3 from outside with the Laplace kernel (the raw Laplace values).
// Without Stern layers the interior row sees its own molecule from inside
// and the outside row sees every surface with the Yukawa kernel.
__device__ __forceinline__ void fold_pair(int f, double vl, double kl, double vy, double ky, double rhoinv,
                                          double* a) {
  a[0] = f == 1 ? -rhoinv * vl : f == 2 ? vy : f == 3 ? vl : 0.0;
  a[1] = f == 1 ? -kl : f == 2 ? ky : f == 3 ? kl : 0.0;
}

// A copy's near rows from the master rows (rep[i] >= 0): columns shifted by
// the copy's panel offset, then values copied.  One wavefront per row, lanes
// over its entries (coalesced).
__global__ void k_near_copy_cols(int64_t nt, const int32_t* __restrict__ rep, const int64_t* __restrict__ rowptr,
                                 int32_t* col) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= nt) return;
  const int32_t m = rep[i];
  if (m < 0) return;
  const int64_t a = rowptr[i], b = rowptr[m], n = rowptr[i + 1] - a;
  for (int64_t k = lane; k < n; k += 64) col[a + k] = col[b + k] + (int32_t)(i - m);
}

__global__ void k_near_copy_vals(int64_t nt, const int32_t* __restrict__ rep, const int64_t* __restrict__ rowptr,
                                 double* vals) {
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= nt) return;
  const int32_t m = rep[i];
  if (m < 0) return;
  const int64_t a = rowptr[i], b = rowptr[m], n = rowptr[i + 1] - a;
  for (int64_t k = lane; k < 4 * n; k += 64) vals[4 * a + k] = vals[4 * b + k];
}

__global__ void k_fold_near(int64_t nt, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ col, const int32_t* __restrict__ tgt_surf, int32_t tsurf,
                            const int32_t* __restrict__ panel_surf, const uint8_t* __restrict__ forms, int nsurf,
                            const double* __restrict__ surf_rhoinv, double* vals, const int32_t* __restrict__ skip) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nt || (skip && skip[i] >= 0)) return;
  const int32_t t = tgt_surf ? tgt_surf[i] : tsurf;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int32_t s = panel_surf[col[e]];
    const int f = forms[(int64_t)t * nsurf + s];
    double* v = vals + 4 * e;
    const double vl = v[0], kl = v[1], vy = v[2], ky = v[3];
    fold_pair(f & 3, vl, kl, vy, ky, surf_rhoinv[s], v);
    fold_pair((f >> 2) & 3, vl, kl, vy, ky, surf_rhoinv[s], v + 2);
  }
}

// Inverse of each panel's self block of the operator (the right block-Jacobi
// preconditioner of GMRES).  A panel's rows (interior, outside) against its
// unknowns (phi, dphi/dn) hold the jump 1/2 on phi in both rows (the double
// layer vanishes on the flat self panel) and the self single layers on
// dphi/dn, folded with the same row factors as the near corrections and
// scaled by the unknown's density factor: B = [[1/2, s_in], [1/2, s_out]].  A
// charged panel has B = [1/2] (its outside row on phi), a potential panel
// B = [s_out] (on dphi/dn).  m = (m00, m01, m10, m11) with
// z_phi = m00 v_int + m01 v_out, z_psi = m10 v_int + m11 v_out.
__global__ void k_self_blocks(int64_t np, const double* __restrict__ tri9, const double* __restrict__ cen,
                              const int32_t* __restrict__ panel_surf, const uint8_t* __restrict__ forms, int nsurf,
                              const double* __restrict__ surf_rhoinv, const double* __restrict__ dens_scale,
                              const int32_t* __restrict__ col_phi, const int32_t* __restrict__ col_psi,
                              NearParams p, double* __restrict__ m) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= np) return;
  double vl = 0.0, vy = 0.0;
  self_single_layer(cen[3 * i], cen[3 * i + 1], cen[3 * i + 2], tri9 + 9 * i, p.Nedge, p.gl_t, p.gl_w, p.kappa, &vl,
                    &vy);
  const int32_t t = panel_surf[i];
  const int f = forms[(int64_t)t * nsurf + t];
  double a_in[2], a_out[2];
  fold_pair(f & 3, vl, 0.0, vy, 0.0, surf_rhoinv[t], a_in);
  fold_pair((f >> 2) & 3, vl, 0.0, vy, 0.0, surf_rhoinv[t], a_out);
  const double ds = dens_scale[i];
  double* o = m + 4 * i;
  o[0] = o[1] = o[2] = o[3] = 0.0;
  if (col_phi[i] >= 0 && col_psi[i] >= 0) {
    const double s_in = a_in[0] * ds, s_out = a_out[0] * ds;
    const double det = 0.5 * s_out - 0.5 * s_in;
    o[0] = s_out / det;
    o[1] = -s_in / det;
    o[2] = -0.5 / det;
    o[3] = 0.5 / det;
  } else if (col_phi[i] >= 0) {
    o[1] = 2.0;
  } else {
    o[3] = 1.0 / (a_out[0] * ds);
  }
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_self_blocks(int64_t np, const double* tri9, const double* cen, const int32_t* panel_surf,
                        const uint8_t* forms, int nsurf, const double* surf_rhoinv, const double* dens_scale,
                        const int32_t* col_phi, const int32_t* col_psi, const NearParams& p, double* m,
                        hipStream_t s) {
  if (np <= 0) return;
  k_self_blocks<<<nblocks(np, 256), 256, 0, s>>>(np, tri9, cen, panel_surf, forms, nsurf, surf_rhoinv, dens_scale,
                                                  col_phi, col_psi, p, m);
  PBT_HIP(hipGetLastError());
}

void launch_fold_near(int64_t nt, const int64_t* rowptr, const int32_t* col, const int32_t* tgt_surf,
                      const int32_t* panel_surf, const uint8_t* forms, int nsurf, const double* surf_rhoinv,
                      double* vals, hipStream_t s, int32_t tsurf, const int32_t* skip) {
  if (nt <= 0) return;
  k_fold_near<<<nblocks(nt, 256), 256, 0, s>>>(nt, rowptr, col, tgt_surf, tsurf, panel_surf, forms, nsurf,
                                                surf_rhoinv, vals, skip);
  PBT_HIP(hipGetLastError());
}

void launch_panel_geometry(int64_t np, const double* tri9, double* cen, double* nrm, double* area,
                           double* cross2, hipStream_t s) {
  if (np <= 0) return;
  k_panel_geometry<<<nblocks(np, 256), 256, 0, s>>>(np, tri9, cen, nrm, area, cross2);
  PBT_HIP(hipGetLastError());
}

void launch_sources(int64_t np, int K, const double* tri9, const double* nrm, const double* area,
                    const double* bary, const double* w, double* src_pos, double* src_wa,
                    hipStream_t s) {
  (void)nrm;
  if (np <= 0) return;
  k_sources<<<nblocks(np * K, 256), 256, 0, s>>>(np, K, tri9, area, bary, w, src_pos, src_wa);
  PBT_HIP(hipGetLastError());
}

void launch_near_count(int64_t nt, const double* tx, int64_t np, const double* cen,
                       const double* cross2, const int32_t* tleaf, const int64_t* lptr,
                       const int64_t* lrange, double f4, int32_t* count, hipStream_t s) {
  if (nt <= 0) return;
  k_near<false><<<nblocks(64 * nt, 256), 256, 0, s>>>(nt, tx, np, cen, cross2, tleaf, lptr, lrange, f4, count,
                                                        nullptr, nullptr);
  PBT_HIP(hipGetLastError());
}

void launch_near_fill(int64_t nt, const double* tx, int64_t np, const double* cen,
                      const double* cross2, const int32_t* tleaf, const int64_t* lptr,
                      const int64_t* lrange, double f4, const int64_t* rowptr, int32_t* col, hipStream_t s) {
  if (nt <= 0) return;
  k_near<true><<<nblocks(64 * nt, 256), 256, 0, s>>>(nt, tx, np, cen, cross2, tleaf, lptr, lrange, f4, nullptr,
                                                       rowptr, col);
  PBT_HIP(hipGetLastError());
}

void launch_pack_points(int64_t np, int64_t ns, const double* cen, const double* src_pos, double* t64, float* t32,
                        double* s64, float* s32, hipStream_t s) {
  const int64_t n = std::max(np, ns);
  if (n <= 0) return;
  k_pack_points<<<nblocks(n, 256), 256, 0, s>>>(np, ns, cen, src_pos, t64, t32, s64, s32);
  PBT_HIP(hipGetLastError());
}

void launch_near_values(int64_t nt, const double* tx, const int32_t* tgt_self, const int64_t* rowptr,
                        const int32_t* col, const double* tri9, const double* nrm,
                        const double* area, const NearParams& p, double* vals, hipStream_t s,
                        const int32_t* skip) {
  if (nt <= 0) return;
  k_near_values<<<nblocks(nt, 128), 128, 0, s>>>(nt, tx, tgt_self, rowptr, col, tri9, nrm, area, p,
                                                  vals, skip);
  PBT_HIP(hipGetLastError());
}
void launch_near_copy_cols(int64_t nt, const int32_t* rep, const int64_t* rowptr, int32_t* col, hipStream_t s) {
  if (nt <= 0) return;
  k_near_copy_cols<<<nblocks(64 * nt, 256), 256, 0, s>>>(nt, rep, rowptr, col);
  PBT_HIP(hipGetLastError());
}
void launch_near_copy_vals(int64_t nt, const int32_t* rep, const int64_t* rowptr, double* vals, hipStream_t s) {
  if (nt <= 0) return;
  k_near_copy_vals<<<nblocks(64 * nt, 256), 256, 0, s>>>(nt, rep, rowptr, vals);
  PBT_HIP(hipGetLastError());
}

void launch_coulomb_rhs(int64_t n, const double* tx, const int32_t* rows, int64_t nq,
                        const double* qxyz, const double* q, double inv_eps, double* b,
                        hipStream_t s) {
  if (n <= 0) return;
  k_coulomb_rhs<<<nblocks(n, 256), 256, 0, s>>>(n, tx, rows, nq, qxyz, q, inv_eps, b);
  PBT_HIP(hipGetLastError());
}

}  // namespace pbt
