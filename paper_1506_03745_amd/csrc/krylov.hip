// FP64 vector kernels of the GMRES solver (Section 3.2): block-partial dot
// products against several basis vectors at once (classical Gram-Schmidt,
// applied twice), multi-vector updates and linear combinations.
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

// part[i * nblk + blockIdx.x] = sum over this block's strided range of V_i . w
__global__ __launch_bounds__(kBS) void k_multidot(int64_t n, int m, const double* __restrict__ V,
                                                  int64_t ldv, const double* __restrict__ w,
                                                  double* __restrict__ part) {
  __shared__ double red[kBS / 64][4];
  const int nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i0 = 0; i0 < m; i0 += 4) {
    double acc[4] = {0, 0, 0, 0};
    for (int64_t j = blockIdx.x * (int64_t)kBS + threadIdx.x; j < n; j += (int64_t)nblk * kBS) {
      const double wj = w[j];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + q < m) acc[q] += V[(int64_t)(i0 + q) * ldv + j] * wj;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double s = wave_sum(acc[q]);
      if (lane == 0) red[wid][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4 && i0 + (int)threadIdx.x < m) {
      double s = 0;
      for (int k = 0; k < kBS / 64; ++k) s += red[k][threadIdx.x];
      part[(int64_t)(i0 + threadIdx.x) * nblk + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// Block-partial dot products of one Gram-Schmidt pass.  Grid (nbj, nci):
// blockIdx.x strides over the elements, blockIdx.y picks 8 consecutive
// outputs i0..i0+7 of V_0..V_{m-1} (and w.w as output m when self_dot).
// UPDATE: the block first adds up the partials of the previous pass, hpart
// (m rows of nbj, fixed order, so every block gets the same h bitwise), and
// dots with w' = w - sum_i h_i V_i formed in registers (w is not written);
// block (0, 0) stores that h in hout.
template <bool UPDATE>
__global__ __launch_bounds__(kBS) void k_gs_dots(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, const double* __restrict__ hpart,
                                                 double* __restrict__ hout, int self_dot,
                                                 double* __restrict__ part) {
  extern __shared__ double hs[];   // [m] (UPDATE)
  __shared__ double red[kBS / 64][8];
  const int nbj = gridDim.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (UPDATE) {
    for (int i = wid; i < m; i += kBS / 64) {
      double sq = 0;
      for (int b = lane; b < nbj; b += 64) sq += hpart[(int64_t)i * nbj + b];
      sq = wave_sum(sq);
      if (lane == 0) {
        hs[i] = sq;
        if (blockIdx.x == 0 && blockIdx.y == 0) hout[i] = sq;
      }
    }
    __syncthreads();
  }
  const int i0 = blockIdx.y * 8;
  const int mq = m + (self_dot ? 1 : 0);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = blockIdx.x * (int64_t)kBS + threadIdx.x; j < n; j += (int64_t)nbj * kBS) {
    double wj = w[j];
    if (UPDATE) {
#pragma unroll 8
      for (int i = 0; i < m; ++i) wj -= hs[i] * V[(int64_t)i * ldv + j];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q;
      if (i < mq) acc[q] += (i < m ? V[(int64_t)i * ldv + j] : wj) * wj;
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
    part[(int64_t)(i0 + threadIdx.x) * nbj + blockIdx.x] = sq;
  }
}

// Arnoldi column j of the Hessenberg matrix: adds up the second pass's
// partials (h2 and |w'|^2, j + 2 rows of nbj), forms h = h1 + h2 and
// |w''|^2 = |w'|^2 - |h2|^2 (w'' = w' - V h2 with V orthonormal), applies
// the previous Givens rotations, computes the new one and stores the
// residual estimate |g_{j+1}| in resid[j].  Also writes h (hsum) and
// |w''|^2 (nrm2) for the update and normalisation of w.
__global__ __launch_bounds__(kBS) void k_arnoldi_col(int j, int m, int nbj, const double* __restrict__ part,
                                                     const double* __restrict__ h1, double* H, double* cs,
                                                     double* sn, double* g, double* resid,
                                                     double* __restrict__ hsum, double* __restrict__ nrm2) {
  extern __shared__ double sh[];   // col[m + 1], h2[m + 1], c[m], s[m]
  double* col = sh;
  double* h2 = sh + (m + 1);
  double* c = h2 + (m + 1);
  double* sv = c + m;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i <= j + 1; i += kBS / 64) {
    double sq = 0;
    for (int b = lane; b < nbj; b += 64) sq += part[(int64_t)i * nbj + b];
    sq = wave_sum(sq);
    if (lane == 0) h2[i] = sq;
  }
  for (int i = threadIdx.x; i < j; i += kBS) {
    c[i] = cs[i];
    sv[i] = sn[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kBS) {
    col[i] = h1[i] + h2[i];
    hsum[i] = col[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double h2s = 0.0;
    for (int i = 0; i <= j; ++i) h2s += h2[i] * h2[i];
    const double nn = fmax(h2[j + 1] - h2s, 0.0);
    *nrm2 = nn;
    const double hn = sqrt(nn);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = c[i] * a + sv[i] * b;
      col[i + 1] = -sv[i] * a + c[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double cj = den > 0 ? a / den : 1.0, sj = den > 0 ? b / den : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    col[j] = den;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    resid[j] = hn > 0 ? fabs(sj * gj) : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += kBS) H[(size_t)i * m + j] = col[i];
}

// w = (w - sum_i h_i V_i) / sqrt(*nrm2)  (the second Gram-Schmidt update
// fused with the normalisation)
__global__ void k_update_normalize(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                                   const double* __restrict__ h, const double* __restrict__ nrm2,
                                   double* __restrict__ w) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double sj = w[j];
#pragma unroll 8
  for (int i = 0; i < m; ++i) sj -= h[i] * V[(int64_t)i * ldv + j];
  const double v = *nrm2;
  w[j] = v > 0.0 ? sj / sqrt(v) : 0.0;
}

__global__ void k_reduce_cols(int m, int nblk, const double* __restrict__ part, double* out) {
  const int i = blockIdx.x;
  double s = 0;
  for (int k = threadIdx.x; k < nblk; k += 64) s += part[(int64_t)i * nblk + k];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[i] = s;
}

// w -= sum_i h_i V_i
__global__ void k_multi_axpy(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                             const double* __restrict__ h, double* w) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = w[j];
  for (int i = 0; i < m; ++i) s -= h[i] * V[(int64_t)i * ldv + j];
  w[j] = s;
}

// y += sum_i c_i V_i
__global__ void k_lincomb(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                          const double* __restrict__ c, double* y) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = y[j];
  for (int i = 0; i < m; ++i) s += c[i] * V[(int64_t)i * ldv + j];
  y[j] = s;
}

// y = x / sqrt(*nrm2) (in place allowed)
__global__ void k_normalize(int64_t n, const double* __restrict__ nrm2, const double* x, double* y) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double v = *nrm2;
  y[j] = v > 0.0 ? x[j] / sqrt(v) : 0.0;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* y) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  y[j] = a * x[j] + b * y[j];
}

__global__ void k_first_unit(int n, double beta, double* g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = i == 0 ? beta : 0.0;
}

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* y) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  y[j] = a * x[j];
}

}  // namespace

int multidot_blocks(int64_t n) {
  int64_t b = (n + 63) / 64;
  if (b < 1) b = 1;
  if (b > 960) b = 960;
  return (int)b;
}

void launch_multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* part,
                     int nblk, hipStream_t s) {
  k_multidot<<<nblk, kBS, 0, s>>>(n, m, V, ldv, w, part);
  PBT_HIP(hipGetLastError());
}

void launch_reduce_cols(int m, int nblk, const double* part, double* out, hipStream_t s) {
  k_reduce_cols<<<m, 64, 0, s>>>(m, nblk, part, out);
  PBT_HIP(hipGetLastError());
}

void launch_multi_axpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w,
                       hipStream_t s) {
  if (n <= 0 || m <= 0) return;
  k_multi_axpy<<<nblocks(n, 256), 256, 0, s>>>(n, m, V, ldv, h, w);
  PBT_HIP(hipGetLastError());
}

void launch_lincomb(int64_t n, int m, const double* V, int64_t ldv, const double* c, double* y,
                    hipStream_t s) {
  if (n <= 0 || m <= 0) return;
  k_lincomb<<<nblocks(n, 256), 256, 0, s>>>(n, m, V, ldv, c, y);
  PBT_HIP(hipGetLastError());
}

int gs_blocks(int64_t n) { return (int)std::min<int64_t>(240, std::max<int64_t>(1, (n + kBS - 1) / kBS)); }

void launch_gs_dots(int64_t n, int m, const double* V, int64_t ldv, const double* w, const double* hpart,
                    double* hout, int self_dot, double* part, int nbj, hipStream_t s) {
  const int mq = m + (self_dot ? 1 : 0);
  const dim3 grid(nbj, (mq + 7) / 8);
  if (hpart)
    k_gs_dots<true><<<grid, kBS, (size_t)m * sizeof(double), s>>>(n, m, V, ldv, w, hpart, hout, self_dot, part);
  else
    k_gs_dots<false><<<grid, kBS, 0, s>>>(n, m, V, ldv, w, nullptr, nullptr, self_dot, part);
  PBT_HIP(hipGetLastError());
}

void launch_arnoldi_col(int j, int m, int nbj, const double* part, const double* h1, double* H, double* cs,
                        double* sn, double* g, double* resid, double* hsum, double* nrm2, hipStream_t s) {
  k_arnoldi_col<<<1, kBS, (size_t)(4 * m + 2) * sizeof(double), s>>>(j, m, nbj, part, h1, H, cs, sn, g, resid,
                                                                     hsum, nrm2);
  PBT_HIP(hipGetLastError());
}

void launch_update_normalize(int64_t n, int m, const double* V, int64_t ldv, const double* h,
                             const double* nrm2, double* w, hipStream_t s) {
  if (n <= 0) return;
  k_update_normalize<<<nblocks(n, 256), 256, 0, s>>>(n, m, V, ldv, h, nrm2, w);
  PBT_HIP(hipGetLastError());
}

void launch_normalize(int64_t n, const double* nrm2, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  k_normalize<<<nblocks(n, 256), 256, 0, s>>>(n, nrm2, x, y);
  PBT_HIP(hipGetLastError());
}

void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n <= 0) return;
  k_axpby<<<nblocks(n, 256), 256, 0, s>>>(n, a, x, b, y);
  PBT_HIP(hipGetLastError());
}

void launch_first_unit(int n, double beta, double* g, hipStream_t s) {
  if (n <= 0) return;
  k_first_unit<<<nblocks(n, 256), 256, 0, s>>>(n, beta, g);
  PBT_HIP(hipGetLastError());
}

void launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  k_scale_copy<<<nblocks(n, 256), 256, 0, s>>>(n, a, x, y);
  PBT_HIP(hipGetLastError());
}

}  // namespace pbt
