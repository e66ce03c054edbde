// FP64 vector kernels of the GMRES solver (Section 3.2 names GMRES for the
// discretised system; here restarted GMRES with classical Gram-Schmidt
// applied twice, or once with the norm by Pythagoras).  Every kernel works on G independent systems at once:
// the unknown vector is split into consecutive group ranges gu[2g] ..
// gu[2g+1] and each group has its own Krylov space, Hessenberg matrix,
// Givens rotations and residual estimate (one system is the case G = 1).
// All sums are taken in a fixed order, so results do not depend on timing.
#include "pbt_internal.h"

#include <algorithm>

namespace pbt {

namespace {

constexpr int kBS = 256;

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// out[i] = sum_b part[i * nbj + b] for i < nrows, by a block of kBS
// threads: eight lanes per row, each adding a strided eighth of the row in
// increasing b, then a fixed butterfly.  The loads of a lane are issued in
// batches of kRowBatch before any of them is added (one memory round trip
// per batch instead of one per few loads); out-of-range slots add an exact
// zero.  The order of the additions is fixed, so every block that calls
// this gets bitwise the same sums.
constexpr int kRowBatch = 32;
static_assert(8 * kRowBatch == kSumBatch, "one batch of loads per lane covers kSumBatch partials");
__device__ __forceinline__ void reduce_rows(const double* __restrict__ part, int nrows, int nbj, double* out) {
  const int sub = threadIdx.x & 7;
  for (int r0 = 0; r0 < nrows; r0 += kBS / 8) {
    const int i = r0 + (int)(threadIdx.x >> 3);
    double sq = 0;
    if (i < nrows) {
      const double* row = part + (int64_t)i * nbj;
      for (int b0 = 0; b0 < nbj; b0 += 8 * kRowBatch) {
        double t[kRowBatch];
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q) {
          const int b = b0 + sub + 8 * q;
          t[q] = b < nbj ? row[b] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q) sq += t[q];
      }
    }
    sq += __shfl_xor(sq, 4, 8);
    sq += __shfl_xor(sq, 2, 8);
    sq += __shfl_xor(sq, 1, 8);
    if (sub == 0 && i < nrows) out[i] = sq;
  }
}

// Block-partial dot products of one Gram-Schmidt pass.  Grid (nbj, nci, G):
// blockIdx.x strides over the elements of group blockIdx.z, blockIdx.y picks
// 8 consecutive outputs i0..i0+7 of V_0..V_{m-1} (and w.w as output m when
// self_dot).  Partials of group g go to part + g * R * nbj (row stride nbj).
// UPDATE: the block first adds up the partials of the previous pass (m rows
// of nbh at hpart + g * R * nbh, fixed order, so every block of the group gets the
// same h bitwise) and dots with w' = w - sum_i h_i V_i formed in registers
// (w is not written); block (0, 0) of the group stores that h at hout + g * R.
template <bool UPDATE>
__global__ __launch_bounds__(kBS) void k_gs_dots(const int64_t* __restrict__ gu, int m, int R,
                                                 const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, const double* __restrict__ hpart,
                                                 int nbh, double* __restrict__ hout, int self_dot,
                                                 double* __restrict__ part) {
  extern __shared__ double hs[];   // [m] (UPDATE)
  __shared__ double red[kBS / 64][8];
  const int nbj = gridDim.x;
  const int g = blockIdx.z;
  const int64_t u0 = gu[2 * g], u1 = gu[2 * g + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i0 = blockIdx.y * 8;
  const int mq = m + (self_dot ? 1 : 0);
  const int64_t j0 = u0 + blockIdx.x * (int64_t)kBS + threadIdx.x;
  // UPDATE: the thread's first element and its first kPre basis entries are
  // loaded before the partials of the previous pass are added up, so those
  // memory round trips overlap
  constexpr int kPre = UPDATE ? 32 : 1;
  double vpre[kPre];
  double wpre = 0.0;
  if (UPDATE && j0 < u1) {
    wpre = w[j0];
#pragma unroll
    for (int q = 0; q < kPre; ++q) vpre[q] = q < m ? V[(int64_t)q * ldv + j0] : 0.0;
  }
  if (UPDATE) {
    reduce_rows(hpart + (int64_t)g * R * nbh, m, nbh, hs);
    __syncthreads();
    if (blockIdx.x == 0 && blockIdx.y == 0)
      for (int i = threadIdx.x; i < m; i += kBS) hout[(int64_t)g * R + i] = hs[i];
  }
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = j0; j < u1; j += (int64_t)nbj * kBS) {
    // the rows of this block's dots (the same rows as some of the update's:
    // cache hits), issued before the update's chain of products
    double vd[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) vd[q] = i0 + q < m ? V[(int64_t)(i0 + q) * ldv + j] : 0.0;
    double wj;
    if (UPDATE) {
      int i = 0;
      if (j == j0) {
        wj = wpre;
#pragma unroll
        for (int q = 0; q < kPre; ++q)
          if (q < m) wj -= hs[q] * vpre[q];
        i = kPre;
      } else {
        wj = w[j];
      }
#pragma unroll 8
      for (; i < m; ++i) wj -= hs[i] * V[(int64_t)i * ldv + j];
    } else {
      wj = w[j];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q;
      if (i < mq) acc[q] += (i < m ? vd[q] : wj) * wj;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double sq = wave_sum(acc[q]);
    if (lane == 0) red[wid][q] = sq;
  }
  __syncthreads();
  if (threadIdx.x < 8 && i0 + (int)threadIdx.x < mq) {
    double sq = 0;
    for (int k = 0; k < kBS / 64; ++k) sq += red[k][threadIdx.x];
    part[((int64_t)g * R + i0 + threadIdx.x) * nbj + blockIdx.x] = sq;
  }
}

// The same partials for large groups (every thread several elements):
// grid (nbj, 1, G), every block forms all mq outputs, kDotRows at a time, so
// each element's basis entries are read about twice per pass instead of once
// per group of 8 outputs (the y-split above reads the m rows of the update
// ceil(mq / 8) times, which for long Krylov spaces dominates the traffic).
// Per output the per-thread sums, wave sums and block sum are formed exactly
// as in k_gs_dots, so both kernels give bitwise the same partials.
constexpr int kDotRows = 32;
template <bool UPDATE>
__global__ __launch_bounds__(kBS) void k_gs_dots_rows(const int64_t* __restrict__ gu, int m, int R,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ hpart, int nbh,
                                                      double* __restrict__ hout, int self_dot,
                                                      double* __restrict__ part) {
  extern __shared__ double hs[];   // [m] (UPDATE)
  __shared__ double red[kBS / 64][kDotRows];
  const int nbj = gridDim.x;
  const int g = blockIdx.z;
  const int64_t u0 = gu[2 * g], u1 = gu[2 * g + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int mq = m + (self_dot ? 1 : 0);
  const int64_t j0 = u0 + blockIdx.x * (int64_t)kBS + threadIdx.x;
  if (UPDATE) {
    reduce_rows(hpart + (int64_t)g * R * nbh, m, nbh, hs);
    __syncthreads();
    if (blockIdx.x == 0)
      for (int i = threadIdx.x; i < m; i += kBS) hout[(int64_t)g * R + i] = hs[i];
  }
  for (int i0 = 0; i0 < mq; i0 += kDotRows) {
    double acc[kDotRows];
#pragma unroll
    for (int q = 0; q < kDotRows; ++q) acc[q] = 0.0;
    for (int64_t j = j0; j < u1; j += (int64_t)nbj * kBS) {
      double wj = w[j];
      if (UPDATE) {
#pragma unroll 8
        for (int i = 0; i < m; ++i) wj -= hs[i] * V[(int64_t)i * ldv + j];
      }
#pragma unroll
      for (int q = 0; q < kDotRows; ++q) {
        const int i = i0 + q;
        if (i < mq) acc[q] += (i < m ? V[(int64_t)i * ldv + j] : wj) * wj;
      }
    }
#pragma unroll
    for (int q = 0; q < kDotRows; ++q) {
      const double sq = wave_sum(acc[q]);
      if (lane == 0) red[wid][q] = sq;
    }
    __syncthreads();
    if (threadIdx.x < kDotRows && i0 + (int)threadIdx.x < mq) {
      double sq = 0;
      for (int k = 0; k < kBS / 64; ++k) sq += red[k][threadIdx.x];
      part[((int64_t)g * R + i0 + threadIdx.x) * nbj + blockIdx.x] = sq;
    }
    __syncthreads();
  }
}

// The rest of Arnoldi step j after the second Gram-Schmidt pass, grid
// (blocks over the largest group, G).  Every block adds up its group's
// partials of that pass (h2 and |w'|^2, j + 2 rows of nbj, in a fixed
// order, so all blocks of the group hold the same values), forms
// h = h1 + h2 and |w''|^2 = |w'|^2 - |h2|^2 (w'' = w' - V h2 with V
// orthonormal), and updates its elements: w = (w - V h) / |w''|.  Block 0
// of each group also builds that group's Hessenberg column j: the previous
// Givens rotations applied, the new one computed, and the residual estimate
// |g_{j+1}| stored in resid[j].  Per group g: part + g R nbj, h1 + g R,
// H + g (m + 1) m, cs/sn/resid + g m, gv + g (m + 1).  With h1 = null the
// partials are those of a single pass (h and |w|^2) and the same formulas
// give classical Gram-Schmidt once, |w'|^2 = |w|^2 - |h|^2 by Pythagoras
// (Smoktunowicz, Barlow and Langou, Numer. Math. 105, 2006, bound its loss
// of orthogonality like that of the pass itself).  With SRC the threads
// run over the group's panels instead of its unknowns and also write the
// panel densities and the source records (type T) of the new basis vector,
// which the next operator application then takes as they are.
template <typename T, bool SRC>
__global__ __launch_bounds__(kBS) void k_arnoldi_update(const int64_t* __restrict__ gu, int j, int m, int R,
                                                        int nbj, const double* __restrict__ part,
                                                        const double* __restrict__ h1,
                                                        const double* __restrict__ V, int64_t ldv,
                                                        double* __restrict__ w, double* H, double* cs,
                                                        double* sn, double* gv, double* resid, NextSrc ns) {
  extern __shared__ double sh[];   // h[m], h2[m + 1], col[m + 1], c[m], s[m]
  __shared__ double nn_s;
  __shared__ int shaky_s;
  double* h = sh;
  double* h2 = h + m;
  double* col = h2 + (m + 1);
  double* c = col + (m + 1);
  double* sv = c + m;
  const int g = blockIdx.y;
  const int64_t u0 = gu[2 * g], u1 = gu[2 * g + 1];
  double* Hg = H + (size_t)g * (m + 1) * m;
  double* csg = cs + (size_t)g * m;
  double* sng = sn + (size_t)g * m;
  double* gg = gv + (size_t)g * (m + 1);
  // SRC: eight lanes per panel (below); the panel's unknowns, w and first
  // basis entries are loaded before the partials are added up, so the memory
  // round trips overlap
  const int sub = threadIdx.x & 7, qi = sub & 3;
  const int64_t p = SRC ? ns.gp[2 * g] + (blockIdx.x * (int64_t)kBS + threadIdx.x) / 8 : 0;
  const bool on = SRC && p < ns.gp[2 * g + 1];
  int32_t cphi = -1, cpsi = -1;
  if (on) {
    cphi = ns.m.col_phi[p];
    cpsi = ns.m.col_psi[p];
  }
  // the panel's geometry for the source records (independent of the
  // unknowns, so issued with them)
  double wa0 = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0, rl = 0.0, dsc = 0.0;
  if (on) {
    if (sub < ns.K) wa0 = ns.wa[p * ns.K + sub];
    n0 = ns.nrm[3 * p];
    n1 = ns.nrm[3 * p + 1];
    n2 = ns.nrm[3 * p + 2];
    rl = ns.rlap[p];
    dsc = ns.m.dens_scale[p];
  }
  const double h1v = h1 && (int)threadIdx.x <= j ? h1[(int64_t)g * R + threadIdx.x] : 0.0;
  const int32_t e = sub < 4 ? cphi : cpsi;
  constexpr int kPre = 8;
  double vr[kPre];
  double we = 0.0;
  if (SRC && e >= 0) {
    we = w[e];
#pragma unroll
    for (int k = 0; k < kPre; ++k) vr[k] = qi + 4 * k <= j ? V[(int64_t)(qi + 4 * k) * ldv + e] : 0.0;
  }
  reduce_rows(part + (int64_t)g * R * nbj, j + 2, nbj, h2);
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < j; i += kBS) {
      c[i] = csg[i];
      sv[i] = sng[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kBS) {
    h[i] = (i == (int)threadIdx.x ? h1v : h1 ? h1[(int64_t)g * R + i] : 0.0) + h2[i];
    col[i] = h[i];
  }
  if (threadIdx.x < 64) {
    // |h2|^2 by the first wavefront (lanes over i, fixed butterfly)
    double h2s = 0.0;
    for (int i = threadIdx.x; i <= j; i += 64) h2s += h2[i] * h2[i];
    h2s = wave_sum(h2s);
    if (threadIdx.x == 0) {
      // |w'|^2 = |w|^2 - |h|^2 cancels when w lies almost in the Krylov
      // space: below 64 rounding units of |w|^2 the norm (and the residual
      // estimate it gives) is not to be trusted
      nn_s = fmax(h2[j + 1] - h2s, 0.0);
      shaky_s = nn_s <= 64.0 * 2.220446049250313e-16 * h2[j + 1];
    }
  }
  __syncthreads();
  const double nn = nn_s;
  auto update = [&](int64_t e) {
    double se = w[e];
#pragma unroll 8
    for (int i = 0; i <= j; ++i) se -= h[i] * V[(int64_t)i * ldv + e];
    const double v = nn > 0.0 ? se / sqrt(nn) : 0.0;
    w[e] = v;
    return v;
  };
  if (!SRC) {
    const int64_t e = u0 + blockIdx.x * (int64_t)kBS + threadIdx.x;
    if (e < u1) update(e);
  } else {
    // eight lanes per panel of the group (the unknowns follow the panels'
    // order, so the V and w accesses are coalesced): lanes 0-3 form the
    // phi unknown, lanes 4-7 the psi unknown, each lane over every fourth
    // basis vector, added by a fixed butterfly; then the panel's densities
    // and source records for the next product, as the strengths kernel
    // would write them from the updated unknowns -- or, with the right
    // preconditioner, from z = M^-1 v (the panel's inverse self block on its
    // interior and outside rows, which share the indices of phi and psi),
    // z also stored for the product's jump terms
    double acc = 0.0;
    if (e >= 0) {
#pragma unroll
      for (int k = 0; k < kPre; ++k)
        if (qi + 4 * k <= j) acc += h[qi + 4 * k] * vr[k];
      for (int i = qi + 4 * kPre; i <= j; i += 4) acc += h[i] * V[(int64_t)i * ldv + e];
    }
    acc += __shfl_xor(acc, 1, 8);
    acc += __shfl_xor(acc, 2, 8);
    double v = 0.0;
    if (e >= 0) {
      v = nn > 0.0 ? (we - acc) / sqrt(nn) : 0.0;
      if (qi == 0) w[e] = v;
    }
    const double vo = __shfl_xor(v, 4, 8);
    double vphi = sub < 4 ? v : vo, vpsi = sub < 4 ? vo : v;
    if (on && ns.pinv) {
      const double* mb = ns.pinv + 4 * p;
      const double vin = cphi >= 0 && cpsi >= 0 ? vphi : 0.0;   // interior row (index of phi)
      const double vout = cpsi >= 0 ? vpsi : vphi;                // outside row
      const double zphi = mb[0] * vin + mb[1] * vout, zpsi = mb[2] * vin + mb[3] * vout;
      vphi = zphi;
      vpsi = zpsi;
      if (qi == 0 && e >= 0) ns.zout[e] = sub < 4 ? zphi : zpsi;
    }
    if (on) {
      const double sg = cpsi >= 0 ? dsc * vpsi : 0.0;
      const double mv = cphi >= 0 ? -vphi : 0.0;
      if (sub == 0) {
        ns.sig[p] = sg;
        ns.mu[p] = mv;
      }
      T* src = reinterpret_cast<T*>(ns.src);
      for (int k = sub; k < ns.K; k += 8) {
        const int64_t jj = p * ns.K + k;
        const double wa = k == sub ? wa0 : ns.wa[jj];
        const double mm = wa * mv;
        const double sval = wa * sg;
        T* o = src + kSrcStride * jj;
        o[3] = (T)sval;
        o[4] = (T)(mm * n0);
        o[5] = (T)(mm * n1);
        o[6] = (T)(mm * n2);
        o[7] = (T)(rl * sval);
      }
    }
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
    const double hn = sqrt(nn);
    // previous rotations: only the carried entry is sequential
    double a = col[0];
    for (int i = 0; i < j; ++i) {
      const double b = col[i + 1], ci = c[i], si = sv[i];
      col[i] = ci * a + si * b;
      a = -si * a + ci * b;
    }
    const double b = hn;
    const double den = hypot(a, b);
    const double cj = den > 0 ? a / den : 1.0, sj = den > 0 ? b / den : 0.0;
    csg[j] = cj;
    sng[j] = sj;
    col[j] = den;
    col[j + 1] = 0.0;
    const double gj = gg[j];
    gg[j + 1] = -sj * gj;
    gg[j] = cj * gj;
    // a step whose norm cancelled reports -1: the host restarts from the
    // true residual instead of reading a converged estimate
    resid[(size_t)g * m + j] = shaky_s ? -1.0 : hn > 0 ? fabs(sj * gj) : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += kBS) Hg[(size_t)i * m + j] = col[i];
}

// z = M^-1 v (or M^-T v) for the right block-Jacobi preconditioner, per
// panel: its inverse self block m on its interior and outside rows (the
// indices of its phi and psi unknowns); with add, z is added to out.
__global__ void k_precond(int64_t np, const int32_t* __restrict__ col_phi, const int32_t* __restrict__ col_psi,
                          const double* __restrict__ pinv, const double* __restrict__ v, double* out, int transpose,
                          int add) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int32_t cphi = col_phi[p], cpsi = col_psi[p];
  const double* mb = pinv + 4 * p;
  if (cphi >= 0 && cpsi >= 0) {
    const double vin = v[cphi], vout = v[cpsi];
    double zphi, zpsi;
    if (transpose) {
      zphi = mb[0] * vin + mb[2] * vout;   // (in, out) rows <- M^T (phi, psi)
      zpsi = mb[1] * vin + mb[3] * vout;
    } else {
      zphi = mb[0] * vin + mb[1] * vout;
      zpsi = mb[2] * vin + mb[3] * vout;
    }
    out[cphi] = add ? out[cphi] + zphi : zphi;
    out[cpsi] = add ? out[cpsi] + zpsi : zpsi;
  } else if (cphi >= 0) {
    const double z = mb[1] * v[cphi];
    out[cphi] = add ? out[cphi] + z : z;
  } else {
    const double z = mb[3] * v[cpsi];
    out[cpsi] = add ? out[cpsi] + z : z;
  }
}

// out[g] = sum_b part[g * R * nbj + b]: row 0 of each group's partials
// (one wavefront per group, fixed order).
__global__ void k_group_row0(int R, int nbj, const double* __restrict__ part, double* out) {
  const int g = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nbj; b += 64) s += part[(int64_t)g * R * nbj + b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[g] = s;
}

// out[g R + i] = sum_b part[(g R + i) nbh + b], i < nrows: the rows of a
// pass added up once, for the update to read as rows of one partial (with
// many chunk partials per row, so that every block of the update does not
// add them all up again).  Grid (ceil(nrows / 32), G); the sums are formed
// by reduce_rows, in its fixed order.
__global__ __launch_bounds__(kBS) void k_reduce_partials(int nrows, int R, int nbh,
                                                         const double* __restrict__ part, double* out) {
  const int g = blockIdx.y, r0 = blockIdx.x * (kBS / 8);
  reduce_rows(part + ((int64_t)g * R + r0) * nbh, std::min(kBS / 8, nrows - r0), nbh, out + (int64_t)g * R + r0);
}

// Per group g: x += sum_{i < m} y[g ystride + i] V_i (y is zero past the
// steps the group uses); grid (blocks over the largest group, G).
__global__ void k_lincomb(const int64_t* __restrict__ gu, int m, int ystride, const double* __restrict__ V,
                          int64_t ldv, const double* __restrict__ y, double* x) {
  const int g = blockIdx.y;
  const int64_t e = gu[2 * g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= gu[2 * g + 1]) return;
  double s = x[e];
  for (int i = 0; i < m; ++i) s += y[(int64_t)g * ystride + i] * V[(int64_t)i * ldv + e];
  x[e] = s;
}

// Per group g: V_0 = r * inv_beta[g] and g-vector = beta[g] e_1 (m + 1
// entries); grid (blocks over the largest group, G).
__global__ void k_start_cycle(const int64_t* __restrict__ gu, int m, const double* __restrict__ beta,
                              const double* __restrict__ inv_beta, const double* __restrict__ r, double* v0,
                              double* gv) {
  const int g = blockIdx.y;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= m; i += blockDim.x) gv[(size_t)g * (m + 1) + i] = i == 0 ? beta[g] : 0.0;
  const int64_t e = gu[2 * g] + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= gu[2 * g + 1]) return;
  v0[e] = r[e] * inv_beta[g];
}

__global__ void k_permute(int64_t n, const int32_t* __restrict__ u2i, const double* __restrict__ in, double* out,
                          int to_internal) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (to_internal) out[u2i[k]] = in[k];
  else out[k] = in[u2i[k]];
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

}  // namespace

int gs_blocks(int64_t n) { return (int)std::min<int64_t>(240, std::max<int64_t>(1, (n + kBS - 1) / kBS)); }

void launch_gs_dots(const int64_t* gu, int G, int m, int R, const double* V, int64_t ldv, const double* w,
                    const double* hpart, int nbh, double* hout, int self_dot, double* part, int nbj,
                    hipStream_t s, bool all_rows) {
  const int mq = m + (self_dot ? 1 : 0);
  if (G <= 0 || mq <= 0) return;
  if (all_rows && mq > 8) {
    const dim3 grid(nbj, 1, G);
    if (hpart)
      k_gs_dots_rows<true><<<grid, kBS, (size_t)m * sizeof(double), s>>>(gu, m, R, V, ldv, w, hpart, nbh, hout,
                                                                         self_dot, part);
    else
      k_gs_dots_rows<false><<<grid, kBS, 0, s>>>(gu, m, R, V, ldv, w, nullptr, 0, nullptr, self_dot, part);
    PBT_HIP(hipGetLastError());
    return;
  }
  const dim3 grid(nbj, (mq + 7) / 8, G);
  if (hpart)
    k_gs_dots<true><<<grid, kBS, (size_t)m * sizeof(double), s>>>(gu, m, R, V, ldv, w, hpart, nbh, hout,
                                                                  self_dot, part);
  else
    k_gs_dots<false><<<grid, kBS, 0, s>>>(gu, m, R, V, ldv, w, nullptr, 0, nullptr, self_dot, part);
  PBT_HIP(hipGetLastError());
}

void launch_arnoldi_update(const int64_t* gu, int G, int64_t nmax, int j, int m, int R, int nbj,
                           const double* part, const double* h1, const double* V, int64_t ldv, double* w,
                           double* H, double* cs, double* sn, double* gv, double* resid, const NextSrc* ns,
                           hipStream_t s) {
  if (G <= 0) return;
  const size_t lds = (size_t)(5 * m + 2) * sizeof(double);
  if (!ns) {
    const dim3 grid(nmax > 0 ? nblocks(nmax, kBS) : 1u, G);
    k_arnoldi_update<double, false><<<grid, kBS, lds, s>>>(gu, j, m, R, nbj, part, h1, V, ldv, w, H, cs, sn, gv,
                                                           resid, NextSrc{});
  } else {
    const dim3 grid(ns->pmax > 0 ? nblocks(8 * ns->pmax, kBS) : 1u, G);
    if (ns->fp32)
      k_arnoldi_update<float, true><<<grid, kBS, lds, s>>>(gu, j, m, R, nbj, part, h1, V, ldv, w, H, cs, sn, gv,
                                                           resid, *ns);
    else
      k_arnoldi_update<double, true><<<grid, kBS, lds, s>>>(gu, j, m, R, nbj, part, h1, V, ldv, w, H, cs, sn, gv,
                                                            resid, *ns);
  }
  PBT_HIP(hipGetLastError());
}

void launch_precond(int64_t np, const int32_t* col_phi, const int32_t* col_psi, const double* pinv, const double* v,
                    double* out, bool transpose, bool add, hipStream_t s) {
  if (np <= 0) return;
  k_precond<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(np, col_phi, col_psi, pinv, v, out, transpose ? 1 : 0,
                                                          add ? 1 : 0);
  PBT_HIP(hipGetLastError());
}

void launch_group_row0(int G, int R, int nbj, const double* part, double* out, hipStream_t s) {
  if (G <= 0) return;
  k_group_row0<<<G, 64, 0, s>>>(R, nbj, part, out);
  PBT_HIP(hipGetLastError());
}

void launch_reduce_partials(int G, int nrows, int R, int nbh, const double* part, double* out, hipStream_t s) {
  if (G <= 0 || nrows <= 0) return;
  k_reduce_partials<<<dim3((unsigned)((nrows + kBS / 8 - 1) / (kBS / 8)), G), kBS, 0, s>>>(nrows, R, nbh, part, out);
  PBT_HIP(hipGetLastError());
}

void launch_lincomb(const int64_t* gu, int G, int64_t nmax, int m, int ystride, const double* V, int64_t ldv,
                    const double* y, double* x, hipStream_t s) {
  if (G <= 0 || nmax <= 0 || m <= 0) return;
  k_lincomb<<<dim3(nblocks(nmax, 256), G), 256, 0, s>>>(gu, m, ystride, V, ldv, y, x);
  PBT_HIP(hipGetLastError());
}

void launch_start_cycle(const int64_t* gu, int G, int64_t nmax, int m, const double* beta, const double* inv_beta,
                        const double* r, double* v0, double* gv, hipStream_t s) {
  if (G <= 0) return;
  const unsigned nb = std::max(1u, nblocks(nmax, 256));
  k_start_cycle<<<dim3(nb, G), 256, 0, s>>>(gu, m, beta, inv_beta, r, v0, gv);
  PBT_HIP(hipGetLastError());
}

void launch_permute(int64_t n, const int32_t* u2i, const double* in, double* out, bool to_internal,
                    hipStream_t s) {
  if (n <= 0) return;
  k_permute<<<nblocks(n, 256), 256, 0, s>>>(n, u2i, in, out, to_internal ? 1 : 0);
  PBT_HIP(hipGetLastError());
}

void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n <= 0) return;
  k_axpby<<<nblocks(n, 256), 256, 0, s>>>(n, a, x, b, y);
  PBT_HIP(hipGetLastError());
}

}  // namespace pbt
