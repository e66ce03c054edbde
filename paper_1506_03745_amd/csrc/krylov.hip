// FP64 vector kernels of the GMRES solver (Section 3.2): block-partial dot
// products against several basis vectors at once (classical Gram-Schmidt,
// applied twice), multi-vector updates and linear combinations.
#include "pbt_internal.h"

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

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* y) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  y[j] = a * x[j];
}

}  // namespace

int multidot_blocks(int64_t n) {
  int64_t b = (n + kBS - 1) / kBS;
  if (b < 1) b = 1;
  if (b > 480) b = 480;
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

void launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  k_scale_copy<<<nblocks(n, 256), 256, 0, s>>>(n, a, x, y);
  PBT_HIP(hipGetLastError());
}

}  // namespace pbt
