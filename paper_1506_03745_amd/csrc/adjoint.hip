// Exact transpose of the treecode boundary-element operator (the adjoint
// product A^T lambda used by the gradient of the free energy).
//
// The forward product maps panel densities (sigma, mu) to Gauss-point
// strengths s_j = w A sigma, D_j = w A mu n, then to target sums L, Y through
// P2P pairs, Taylor far fields (P2M -> M2M -> M2P) and sparse near/self
// corrections.  Its transpose takes target weights (l_i, u_i) =
// (lambda[interior row], lambda[solvent row]) and returns, per Gauss point,
//   sbar_j = d(lambda^T y)/d s_j,   Dbar_j = d(lambda^T y)/d D_j,
// through the same pairs, lists and expansions in reverse:
//   reverse P2P (lanes over sources, targets streamed), M2P^T (per box,
//   sum over targets of u_i a^Y_k(x_i - c) and l_i a^L_k(x_i - c)),
//   M2M^T (shift parents' sums down to children), P2M^T (evaluate the box
//   polynomial and its gradient at each Gauss point), and the transposed
//   near corrections; finally sigmabar_p = sum_j w A sbar_j and
//   mubar_p = sum_j w A n . Dbar_j, and the density maps in reverse.
// Every reduction is a fixed-order sum: the result is deterministic.
#include "pbt_internal.h"

namespace pbt {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;

__host__ __device__ constexpr int tidx(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
struct AMath;
template <>
struct AMath<float> {
  static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float expm(float x) { return __builtin_amdgcn_exp2f(-x * 1.4426950408889634f); }
};
template <>
struct AMath<double> {
  static __device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
  static __device__ __forceinline__ double expm(double x) { return exp(-x); }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Target records for the transpose: (x, y, z, l, u, pad, pad, pad).
template <typename T>
__global__ void k_adj_targets(int64_t np, const double* __restrict__ cen, const int32_t* __restrict__ row_int,
                              const int32_t* __restrict__ row_sol, const double* __restrict__ lam,
                              T* __restrict__ trec) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= np) return;
  T* o = trec + 8 * i;
  o[0] = (T)cen[3 * i];
  o[1] = (T)cen[3 * i + 1];
  o[2] = (T)cen[3 * i + 2];
  o[3] = row_int[i] >= 0 ? (T)lam[row_int[i]] : T(0);
  o[4] = (T)lam[row_sol[i]];
  o[5] = o[6] = o[7] = T(0);
}

// Reverse P2P: one wavefront per task = 64 sources (lanes) x a segment of
// target ranges (streamed with scalar loads).  Writes (sbar, Dbar) partials.
template <typename T, bool GUARD>
__global__ __launch_bounds__(256) void k_p2p_t(const Task* __restrict__ tasks, int ntasks,
                                               const int32_t* __restrict__ ranges,
                                               const T* __restrict__ src, const T* __restrict__ trec,
                                               T kappa, T* __restrict__ partial) {
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= ntasks) return;
  const int lane = threadIdx.x & 63;
  const int sbeg = tasks[wv].tbeg, scount = tasks[wv].tcount;
  const int lbeg = tasks[wv].lbeg, lend = tasks[wv].lend;
  const int fused = tasks[wv].fused;
  // form bits of the forward task: kappa = 0 for its outside sum, the two
  // sums stored in swapped rows, the outside sum dropped; the weights of the
  // sums are the multipliers of the rows they went to
  const int form = tasks[wv].form;
  if (form & kFormKz) kappa = T(0);
  const bool swap = (form & kFormSwap) != 0, drop = (form & kFormDropOut) != 0;
  const T ri = sizeof(T) == 4 ? (T)tasks[wv].rho_inv_f : (T)tasks[wv].rho_inv;
  const int sj = sbeg + (lane < scount ? lane : 0);
  const T sx = src[kSrcStride * (int64_t)sj], sy = src[kSrcStride * (int64_t)sj + 1],
          sz = src[kSrcStride * (int64_t)sj + 2];
  T sb = 0, dbx = 0, dby = 0, dbz = 0;
  for (int r = lbeg; r < lend; ++r) {
    const int i0 = ranges[2 * r], i1 = ranges[2 * r + 1];
#pragma unroll 2
    for (int i = i0; i < i1; ++i) {
      const T* t = trec + 8 * (int64_t)i;
      const T dx = t[0] - sx, dy = t[1] - sy, dz = t[2] - sz;   // x_target - y_source
      const T r2 = dx * dx + dy * dy + dz * dz;
      T rinv = AMath<T>::rsq(r2);
      if (GUARD) rinv = r2 > T(0) ? rinv : T(0);
      const T rr = r2 * rinv;
      const T e = AMath<T>::expm(kappa * rr);
      const T rinv3 = rinv * rinv * rinv;
      const T u = drop ? T(0) : swap ? t[3] : t[4];
      T c = u * (kappa * rr + T(1)) * e * rinv3;
      T g = u * e * rinv;
      if (fused) {
        const T l = swap ? t[4] : t[3];
        c -= l * rinv3;
        g -= ri * l * rinv;
      }
      sb += g;
      dbx += c * dx;
      dby += c * dy;
      dbz += c * dz;
    }
  }
  if (lane < scount) {
    T* o = partial + 4 * ((int64_t)tasks[wv].slot * 64 + lane);
    o[0] = sb;
    o[1] = dbx;
    o[2] = dby;
    o[3] = dbz;
  }
}

// M2P^T: one wavefront per (box, 64-target chunk).  Each lane computes the
// Taylor coefficients of its target about the box centre; then, kBatch
// coefficients at a time, the lanes store them weighted in LDS and lane k
// adds up coefficient k over the 64 targets in lane order (four interleaved
// partial sums, combined in a fixed order).  The reduction costs a few LDS
// reads per lane and coefficient instead of a chain of cross-lane shuffles
// per coefficient, and the batches keep the LDS per wave small enough not to
// limit occupancy.
constexpr int kLdsStride = 65;   // 64 targets + 1: lanes reading one column hit distinct banks
constexpr int kBatch = 32;

template <typename T, int P>
__device__ __forceinline__ void taylor_reduce(T Rx, T Ry, T Rz, T kappa, T w, bool yuk,
                                              T* __restrict__ out, int lane, T* lds) {
  constexpr int NC = ncoef(P);
  T A[NC];
  T B[NC];
  const T R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const T Rinv = R2 > T(0) ? AMath<T>::rsq(R2) : T(0);
  const T invR2 = Rinv * Rinv;
  const T kap = yuk ? kappa : T(0);
  const T e = yuk ? AMath<T>::expm(kappa * (R2 * Rinv)) : T(1);
  A[0] = e * Rinv;
  B[0] = e;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    const T c1 = T(2 * n - 1) / T(n) * invR2;
    const T c2 = T(n - 1) / T(n) * invR2;
    const T c3 = kap / T(n) * invR2;
    const T c4 = kap / T(n);
#pragma unroll
    for (int a = n; a >= 0; --a) {
#pragma unroll
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        const int k = tidx(a, b, c);
        T S1 = 0, S2 = 0, T1 = 0, T2 = 0;
        if (a >= 1) { S1 += Rx * A[tidx(a - 1, b, c)]; T1 += Rx * B[tidx(a - 1, b, c)]; }
        if (b >= 1) { S1 += Ry * A[tidx(a, b - 1, c)]; T1 += Ry * B[tidx(a, b - 1, c)]; }
        if (c >= 1) { S1 += Rz * A[tidx(a, b, c - 1)]; T1 += Rz * B[tidx(a, b, c - 1)]; }
        if (a >= 2) { S2 += A[tidx(a - 2, b, c)]; T2 += B[tidx(a - 2, b, c)]; }
        if (b >= 2) { S2 += A[tidx(a, b - 2, c)]; T2 += B[tidx(a, b - 2, c)]; }
        if (c >= 2) { S2 += A[tidx(a, b, c - 2)]; T2 += B[tidx(a, b, c - 2)]; }
        A[k] = c1 * S1 - c2 * S2 + c3 * (T1 - T2);
        B[k] = c4 * (S1 - S2);
      }
    }
  }
#pragma unroll
  for (int kb = 0; kb < NC; kb += kBatch) {
#pragma unroll
    for (int k = kb; k < kb + kBatch && k < NC; ++k) lds[(k - kb) * kLdsStride + lane] = w * A[k];
    __syncthreads();
    if (lane < kBatch && kb + lane < NC) {
      const T* row = lds + lane * kLdsStride;
      T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
      for (int j = 0; j < 64; j += 4) {
        s0 += row[j];
        s1 += row[j + 1];
        s2 += row[j + 2];
        s3 += row[j + 3];
      }
      out[kb + lane] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
}

template <typename T, int P>
__global__ __launch_bounds__(64) void k_m2p_t(const Task* __restrict__ tasks, int ntasks,
                                              const T* __restrict__ trec,
                                              const double* __restrict__ bcen, T kappa,
                                              T* __restrict__ mpart) {
  constexpr int NC = ncoef(P);
  __shared__ T lds[kBatch * kLdsStride];
  const int wv = blockIdx.x;
  if (wv >= ntasks) return;
  const int lane = threadIdx.x;
  const int tbeg = tasks[wv].tbeg, tcount = tasks[wv].tcount;
  const int b = tasks[wv].lbeg;
  const int slot = tasks[wv].slot;
  const bool act = lane < tcount;
  const int ti = tbeg + (act ? lane : 0);
  const T* t = trec + 8 * (int64_t)ti;
  const T Rx = t[0] - (T)bcen[3 * b], Ry = t[1] - (T)bcen[3 * b + 1], Rz = t[2] - (T)bcen[3 * b + 2];
  T* out = mpart + (int64_t)slot * 2 * NC;
  // form bits as in the reverse P2P
  const int form = tasks[wv].form;
  const bool swap = (form & kFormSwap) != 0, drop = (form & kFormDropOut) != 0;
  const T ku = (form & kFormKz) ? T(0) : kappa;
  const T wu = act && !drop ? (swap ? t[3] : t[4]) : T(0);
  const T wl = act ? (swap ? t[4] : t[3]) : T(0);
  taylor_reduce<T, P>(Rx, Ry, Rz, ku, wu, true, out, lane, lds);
  if (tasks[wv].fused) {
    taylor_reduce<T, P>(Rx, Ry, Rz, kappa, wl, false, out + NC, lane, lds);
  } else {
    for (int k = lane; k < NC; k += 64) out[NC + k] = T(0);
  }
}

// Per box: sum its M2P^T partial slots into Mbar[box][2][NC].  Block (box,
// 64 coefficients): thread (k, p) adds every kParts-th slot from p on, then
// the kParts partial sums are added in order; the order is fixed, and boxes
// with thousands of slots no longer wait on one thread's chain of loads.
constexpr int kParts = 16;
template <typename T>
__global__ __launch_bounds__(64 * kParts) void k_mbar_reduce(int nbox, int NC, const int32_t* __restrict__ sbeg,
                                                             const int32_t* __restrict__ send,
                                                             const T* __restrict__ mpart, T* __restrict__ mbar) {
  __shared__ T red[kParts][64];
  const int b = blockIdx.x;
  const int kk = threadIdx.x & 63, p = threadIdx.x >> 6;
  const int rk = blockIdx.y * 64 + kk;
  T s = 0;
  if (rk < 2 * NC) {
#pragma unroll 4
    for (int q = sbeg[b] + p; q < send[b]; q += kParts) s += mpart[(int64_t)q * 2 * NC + rk];
  }
  red[p][kk] = s;
  __syncthreads();
  if (p == 0 && rk < 2 * NC) {
    T t = 0;
    for (int i = 0; i < kParts; ++i) t += red[i][kk];
    mbar[(int64_t)b * 2 * NC + rk] = t;
  }
}

struct MidxT {
  int8_t a, b, c, n;
};
__constant__ MidxT c_midx_t[ncoef(kMaxP)];
__constant__ int8_t c_binom_t[kMaxP + 1][kMaxP + 1];

// M2M^T: one wavefront per (child box, coefficient m) at one level;
//   Mbar_m(child) += sum_{k >= m} C(k, m) delta^(k-m) Mbar_k(parent),
// delta = c_child - c_parent.
template <typename T>
__global__ __launch_bounds__(64) void k_m2m_t(int P, const int32_t* __restrict__ boxes,
                                              const int32_t* __restrict__ parent,
                                              const double* __restrict__ bcen, T* __restrict__ mbar) {
  const int NC = ncoef(P);
  const int c = boxes[blockIdx.x];
  const int m = blockIdx.y;
  const int lane = threadIdx.x;
  const int p = parent[c];
  const MidxT mm = c_midx_t[m];
  const T dx = (T)(bcen[3 * c] - bcen[3 * p]), dy = (T)(bcen[3 * c + 1] - bcen[3 * p + 1]),
          dz = (T)(bcen[3 * c + 2] - bcen[3 * p + 2]);
  T a0 = 0, a1 = 0;
  for (int k = lane; k < NC; k += 64) {
    const MidxT kk = c_midx_t[k];
    if (kk.a < mm.a || kk.b < mm.b || kk.c < mm.c) continue;
    T coef = (T)(c_binom_t[kk.a][mm.a] * c_binom_t[kk.b][mm.b] * c_binom_t[kk.c][mm.c]);
    for (int q = mm.a; q < kk.a; ++q) coef *= dx;
    for (int q = mm.b; q < kk.b; ++q) coef *= dy;
    for (int q = mm.c; q < kk.c; ++q) coef *= dz;
    a0 += coef * mbar[(int64_t)(2 * p) * NC + k];
    a1 += coef * mbar[(int64_t)(2 * p + 1) * NC + k];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    mbar[(int64_t)(2 * c) * NC + m] += a0;
    mbar[(int64_t)(2 * c + 1) * NC + m] += a1;
  }
}

// P2M^T at the leaves: evaluate sum_k (Mbar_Y - rho Mbar_L)_k h^k and the
// gradient sum_k (Mbar_Y - Mbar_L)_k grad h^k at each Gauss point.
template <typename T>
__global__ __launch_bounds__(256) void k_l2p_t(int P, const int32_t* __restrict__ leaves, BoxDev bd,
                                               const T* __restrict__ src, const T* __restrict__ mbar,
                                               T* __restrict__ far) {
  const int NC = ncoef(P);
  const int b = leaves[blockIdx.x];
  const T cx = (T)bd.center[3 * b], cy = (T)bd.center[3 * b + 1], cz = (T)bd.center[3 * b + 2];
  const T rho = (T)bd.rho_inv[b];
  const T* MY = mbar + (int64_t)(2 * b) * NC;
  const T* ML = MY + NC;
  for (int j = bd.sbeg[b] + threadIdx.x; j < bd.send[b]; j += blockDim.x) {
    const T* s = src + (int64_t)kSrcStride * j;
    const T hx = s[0] - cx, hy = s[1] - cy, hz = s[2] - cz;
    T sb = 0, gx = 0, gy = 0, gz = 0;
    for (int k = 0; k < NC; ++k) {
      const MidxT mi = c_midx_t[k];
      T px = 1, py = 1, pz = 1, qx = 0, qy = 0, qz = 0;
      for (int t = 0; t < mi.a; ++t) { qx = qx * hx + px; px *= hx; }
      for (int t = 0; t < mi.b; ++t) { qy = qy * hy + py; py *= hy; }
      for (int t = 0; t < mi.c; ++t) { qz = qz * hz + pz; pz *= hz; }
      const T wy = MY[k], wl = ML[k];
      sb += (wy - rho * wl) * (px * py * pz);
      const T wd = wy - wl;
      gx += wd * (qx * py * pz);
      gy += wd * (px * qy * pz);
      gz += wd * (px * py * qz);
    }
    T* o = far + 4 * (int64_t)j;
    o[0] = sb;
    o[1] = gx;
    o[2] = gy;
    o[3] = gz;
  }
}

// Per panel: gather its Gauss points' (sbar, Dbar) from the reverse-P2P slots
// and the far field, scale by 1/(4 pi), project onto (sigmabar, mubar), add
// the transposed near corrections (CSR by source panel), and apply the
// density maps and jump terms in reverse.
template <typename T>
__global__ void k_combine_t(AdjCombineArgs a, const T* __restrict__ partial, const T* __restrict__ far,
                            double* __restrict__ z, double* __restrict__ sigbar) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= a.np) return;
  double sg = a.add_sig ? a.add_sig[p] : 0.0, mu = a.add_mu ? a.add_mu[p] : 0.0;
  const double nx = a.nrm[3 * p], ny = a.nrm[3 * p + 1], nz = a.nrm[3 * p + 2];
  for (int q = 0; q < a.K; ++q) {
    const int64_t j = p * a.K + q;
    double sb = 0, dx = 0, dy = 0, dz = 0;
    if (a.chunks) {
      const ChunkSlots cs = a.chunks[a.chunk_of[j]];
      const int lane = (int)(j - cs.tbeg);
      for (int s = cs.sbeg; s < cs.send; ++s) {
        const T* v = partial + 4 * ((int64_t)s * 64 + lane);
        sb += (double)v[0];
        dx += (double)v[1];
        dy += (double)v[2];
        dz += (double)v[3];
      }
    }
    if (far) {
      const T* v = far + 4 * j;
      sb += (double)v[0];
      dx += (double)v[1];
      dy += (double)v[2];
      dz += (double)v[3];
    }
    const double w = a.wa[j] * kInv4Pi;
    sg += w * sb;
    mu += w * (nx * dx + ny * dy + nz * dz);
  }
  for (int64_t e = a.tptr ? a.tptr[p] : 0; a.tptr && e < a.tptr[p + 1]; ++e) {
    const int32_t i = a.trow[e];
    const double* v = a.tval + 4 * e;
    const double l = a.maps.row_int[i] >= 0 ? a.lam[a.maps.row_int[i]] : 0.0;
    const double u = a.lam[a.maps.row_sol[i]];
    sg += v[0] * l + v[2] * u;
    mu += v[1] * l + v[3] * u;
  }
  if (sigbar) sigbar[p] = sg;
  const int32_t cpsi = a.maps.col_psi[p], cphi = a.maps.col_phi[p];
  if (cpsi >= 0) z[cpsi] = a.maps.dens_scale[p] * sg;
  if (cphi >= 0) {
    double jump = 0.0;
    if (a.lam) {
      const double l = a.maps.row_int[p] >= 0 ? a.lam[a.maps.row_int[p]] : 0.0;
      jump = 0.5 * (l + a.lam[a.maps.row_sol[p]]);
    }
    z[cphi] = -mu + jump;
  }
}

// Transposed reaction-potential evaluator (phi_reac = -L at the charges):
// for each Gauss point of the molecule, the weights q_k of the charges give
//   sbar_j = sum_k q_k rho_inv / r,  Dbar_j = sum_k q_k (r_k - y_j) / r^3.
__global__ void k_reac_t(int64_t s0, int64_t s1, const double* __restrict__ src, int64_t nq,
                         const double* __restrict__ qxyz, const double* __restrict__ q,
                         double rho_inv, double dsign, double* __restrict__ far) {
  const int64_t j = s0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= s1) return;
  const double* s = src + (int64_t)kSrcStride * j;
  double sb = 0, gx = 0, gy = 0, gz = 0;
  for (int64_t k = 0; k < nq; ++k) {
    const double dx = qxyz[3 * k] - s[0], dy = qxyz[3 * k + 1] - s[1], dz = qxyz[3 * k + 2] - s[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double c = dsign * q[k] * rinv * rinv * rinv;
    sb += q[k] * rho_inv * rinv;
    gx += c * dx;
    gy += c * dy;
    gz += c * dz;
  }
  double* o = far + 4 * (j - s0);
  o[0] = sb;
  o[1] = gx;
  o[2] = gy;
  o[3] = gz;
}

// (B_q^T lambda)_k = sum_i lambda[row_int(i)] / (4 pi eps_in |x_i - r_k|);
// one block per charge, threads over panels.
__global__ __launch_bounds__(256) void k_coulomb_t(int64_t nq, const double* __restrict__ qxyz, int64_t n,
                                                   const double* __restrict__ tx,
                                                   const int32_t* __restrict__ rows,
                                                   const double* __restrict__ lam, double inv_eps,
                                                   double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  const double x = qxyz[3 * k], y = qxyz[3 * k + 1], z = qxyz[3 * k + 2];
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double dx = tx[3 * i] - x, dy = tx[3 * i + 1] - y, dz = tx[3 * i + 2] - z;
    s += lam[rows[i]] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[k] = (red[0] + red[1] + red[2] + red[3]) * kInv4Pi * inv_eps;
}

bool g_adj_tables[64] = {false};
void upload_adj_tables() {
  int dev = 0;
  PBT_HIP(hipGetDevice(&dev));
  if (dev < 64 && g_adj_tables[dev]) return;
  MidxT h[ncoef(kMaxP)];
  for (int n = 0; n <= kMaxP; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        h[tidx(a, b, c)] = MidxT{(int8_t)a, (int8_t)b, (int8_t)c, (int8_t)n};
      }
  int8_t bin[kMaxP + 1][kMaxP + 1] = {};
  for (int n = 0; n <= kMaxP; ++n) {
    bin[n][0] = 1;
    for (int k = 1; k <= n; ++k) bin[n][k] = (int8_t)(bin[n - 1][k - 1] + (k <= n - 1 ? bin[n - 1][k] : 0));
  }
  PBT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_midx_t), h, sizeof(h)));
  PBT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom_t), bin, sizeof(bin)));
  if (dev < 64) g_adj_tables[dev] = true;
}

template <typename T, int P>
void m2p_t_p(const Task* tasks, int ntasks, const T* trec, const double* bcen, T kappa, T* mpart,
             hipStream_t s) {
  k_m2p_t<T, P><<<ntasks, 64, 0, s>>>(tasks, ntasks, trec, bcen, kappa, mpart);
}

}  // namespace

template <typename T>
void launch_adj_targets(int64_t np, const double* cen, const int32_t* row_int, const int32_t* row_sol,
                        const double* lam, T* trec, hipStream_t s) {
  if (np <= 0) return;
  k_adj_targets<T><<<nblocks(np, 256), 256, 0, s>>>(np, cen, row_int, row_sol, lam, trec);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_p2p_t(const Task* tasks, int ntasks, const int32_t* ranges, const T* src, const T* trec,
                  T kappa, bool guard, T* partial, hipStream_t s) {
  if (ntasks <= 0) return;
  const int blocks = ((ntasks + 3) / 4 + 7) / 8 * 8;
  if (guard)
    k_p2p_t<T, true><<<blocks, 256, 0, s>>>(tasks, ntasks, ranges, src, trec, kappa, partial);
  else
    k_p2p_t<T, false><<<blocks, 256, 0, s>>>(tasks, ntasks, ranges, src, trec, kappa, partial);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_m2p_t(int P, const Task* tasks, int ntasks, const T* trec, const double* bcen, T kappa,
                  T* mpart, hipStream_t s) {
  if (ntasks <= 0) return;
  switch (P) {
    case 0: m2p_t_p<T, 0>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 1: m2p_t_p<T, 1>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 2: m2p_t_p<T, 2>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 3: m2p_t_p<T, 3>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 4: m2p_t_p<T, 4>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 5: m2p_t_p<T, 5>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 6: m2p_t_p<T, 6>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 7: m2p_t_p<T, 7>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    case 8: m2p_t_p<T, 8>(tasks, ntasks, trec, bcen, kappa, mpart, s); break;
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_mbar_reduce(int nbox, int P, const int32_t* sbeg, const int32_t* send, const T* mpart,
                        T* mbar, hipStream_t s) {
  if (nbox <= 0) return;
  const dim3 grid((unsigned)nbox, (unsigned)((2 * ncoef(P) + 63) / 64));
  k_mbar_reduce<T><<<grid, 64 * kParts, 0, s>>>(nbox, ncoef(P), sbeg, send, mpart, mbar);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_m2m_t(int P, int nbox, const int32_t* boxes, const int32_t* parent, const double* bcen,
                  T* mbar, hipStream_t s) {
  if (nbox <= 0) return;
  upload_adj_tables();
  k_m2m_t<T><<<dim3(nbox, ncoef(P)), 64, 0, s>>>(P, boxes, parent, bcen, mbar);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_l2p_t(int P, int nleaf, const int32_t* leaves, const BoxDev& bd, const T* src,
                  const T* mbar, T* far, hipStream_t s) {
  if (nleaf <= 0) return;
  upload_adj_tables();
  k_l2p_t<T><<<nleaf, 256, 0, s>>>(P, leaves, bd, src, mbar, far);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_combine_t(const AdjCombineArgs& a, const T* partial, const T* far, double* z, double* sigbar,
                      hipStream_t s) {
  if (a.np <= 0) return;
  k_combine_t<T><<<nblocks(a.np, 256), 256, 0, s>>>(a, partial, far, z, sigbar);
  PBT_HIP(hipGetLastError());
}

void launch_reac_t(int64_t s0, int64_t s1, const double* src, int64_t nq, const double* qxyz,
                   const double* q, double rho_inv, double* far, double dsign, hipStream_t s) {
  if (s1 <= s0) return;
  k_reac_t<<<nblocks(s1 - s0, 128), 128, 0, s>>>(s0, s1, src, nq, qxyz, q, rho_inv, dsign, far);
  PBT_HIP(hipGetLastError());
}

void launch_coulomb_t(int64_t nq, const double* qxyz, int64_t n, const double* tx, const int32_t* rows,
                      const double* lam, double inv_eps, double* out, hipStream_t s) {
  if (nq <= 0) return;
  k_coulomb_t<<<(unsigned)nq, 256, 0, s>>>(nq, qxyz, n, tx, rows, lam, inv_eps, out);
  PBT_HIP(hipGetLastError());
}

#define INST(T)                                                                                       \
  template void launch_adj_targets<T>(int64_t, const double*, const int32_t*, const int32_t*,         \
                                      const double*, T*, hipStream_t);                                \
  template void launch_p2p_t<T>(const Task*, int, const int32_t*, const T*, const T*, T, bool, T*,    \
                                hipStream_t);                                                         \
  template void launch_m2p_t<T>(int, const Task*, int, const T*, const double*, T, T*, hipStream_t);  \
  template void launch_mbar_reduce<T>(int, int, const int32_t*, const int32_t*, const T*, T*,         \
                                      hipStream_t);                                                   \
  template void launch_m2m_t<T>(int, int, const int32_t*, const int32_t*, const double*, T*,          \
                                hipStream_t);                                                         \
  template void launch_l2p_t<T>(int, int, const int32_t*, const BoxDev&, const T*, const T*, T*,      \
                                hipStream_t);                                                         \
  template void launch_combine_t<T>(const AdjCombineArgs&, const T*, const T*, double*, double*,      \
                                    hipStream_t);
INST(float)
INST(double)

}  // namespace pbt
