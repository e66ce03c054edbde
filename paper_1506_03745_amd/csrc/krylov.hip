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

// out[i] = sum_b part[i * nbj + b] for i < nrows, by a block of kBS
// threads: eight lanes per row, each adding a strided eighth of the row
// (independent loads), then a fixed butterfly; the order of the additions
// is fixed, so every block that calls this gets bitwise the same sums.
__device__ __forceinline__ void reduce_rows(const double* __restrict__ part, int nrows, int nbj, double* out) {
  const int sub = threadIdx.x & 7;
  for (int r0 = 0; r0 < nrows; r0 += kBS / 8) {
    const int i = r0 + (int)(threadIdx.x >> 3);
    double sq = 0;
    if (i < nrows) {
#pragma unroll 8
      for (int b = sub; b < nbj; b += 8) sq += part[(int64_t)i * nbj + b];
    }
    sq += __shfl_xor(sq, 4, 8);
    sq += __shfl_xor(sq, 2, 8);
    sq += __shfl_xor(sq, 1, 8);
    if (sub == 0 && i < nrows) out[i] = sq;
  }
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
    reduce_rows(hpart, m, nbj, hs);
    __syncthreads();
    if (blockIdx.x == 0 && blockIdx.y == 0)
      for (int i = threadIdx.x; i < m; i += kBS) hout[i] = hs[i];
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

// The rest of Arnoldi step j after the second Gram-Schmidt pass.  Every
// block adds up that pass's partials (h2 and |w'|^2, j + 2 rows of nbj, in
// a fixed order, so all blocks hold the same values), forms h = h1 + h2 and
// |w''|^2 = |w'|^2 - |h2|^2 (w'' = w' - V h2 with V orthonormal), and
// updates its elements: w = (w - V h) / |w''|.  Block 0 also builds the
// Hessenberg column j: the previous Givens rotations applied, the new one
// computed, and the residual estimate |g_{j+1}| stored in resid[j].
__global__ __launch_bounds__(kBS) void k_arnoldi_update(int64_t n, int j, int m, int nbj,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ h1,
                                                        const double* __restrict__ V, int64_t ldv,
                                                        double* __restrict__ w, double* H, double* cs,
                                                        double* sn, double* g, double* resid) {
  extern __shared__ double sh[];   // h[m], h2[m + 1], col[m + 1], c[m], s[m]
  __shared__ double nn_s;
  double* h = sh;
  double* h2 = h + m;
  double* col = h2 + (m + 1);
  double* c = col + (m + 1);
  double* sv = c + m;
  reduce_rows(part, j + 2, nbj, h2);
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < j; i += kBS) {
      c[i] = cs[i];
      sv[i] = sn[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kBS) {
    h[i] = h1[i] + h2[i];
    col[i] = h[i];
  }
  if (threadIdx.x == 0) {
    double h2s = 0.0;
    for (int i = 0; i <= j; ++i) h2s += h2[i] * h2[i];
    nn_s = fmax(h2[j + 1] - h2s, 0.0);
  }
  __syncthreads();
  const double nn = nn_s;
  const int64_t e = blockIdx.x * (int64_t)kBS + threadIdx.x;
  if (e < n) {
    double se = w[e];
#pragma unroll 8
    for (int i = 0; i <= j; ++i) se -= h[i] * V[(int64_t)i * ldv + e];
    w[e] = nn > 0.0 ? se / sqrt(nn) : 0.0;
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
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

void launch_arnoldi_update(int64_t n, int j, int m, int nbj, const double* part, const double* h1,
                           const double* V, int64_t ldv, double* w, double* H, double* cs, double* sn, double* g,
                           double* resid, hipStream_t s) {
  const unsigned blocks = n > 0 ? nblocks(n, kBS) : 1u;
  k_arnoldi_update<<<blocks, kBS, (size_t)(5 * m + 2) * sizeof(double), s>>>(n, j, m, nbj, part, h1, V, ldv, w,
                                                                              H, cs, sn, g, resid);
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
