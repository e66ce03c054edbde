// Cartesian Taylor-series far field of the treecode (Section 3.2; the
// treecode of Barnes & Hut with the Taylor expansions of Li, Johnston &
// Krasny, both cited there).
//
// For a source box with expansion centre c and a target x, with h = y - c and
// R = x - c, a kernel G(x, y) = f(|R - h|) is expanded as
//     G = sum_{|k| <= P} a_k(R) h^k,   a_k = (1/k!) d^k G / dh^k at h = 0,
// so the box acts on x through its moments
//     M_k = sum_j  s_j h_j^k  +  D_j . grad_h (h_j^k)
// (single-layer strength s and double-layer moment D of each Gauss point).
//
// Recurrences (derived from rho^2 (h . grad) f = ..., rho = |R - h|, by
// comparing coefficients of h^k), with n = |k| and e_i the unit multi-indices:
//  Laplace  f = 1/rho:
//     n |R|^2 a_k = (2n-1) sum_i R_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i}
//  Yukawa   f = exp(-kappa rho)/rho, with b_k the coefficients of exp(-kappa rho):
//     n |R|^2 a_k = (2n-1) sum_i R_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i}
//                   + kappa ( sum_i R_i b_{k-e_i} - sum_i b_{k-2e_i} )
//     n b_k = kappa ( sum_i R_i a_{k-e_i} - sum_i a_{k-2e_i} )
//  starting from a_0 = f(|R|), b_0 = exp(-kappa |R|).
//
// Moments are kept per box in two rows: row 0 for the solvent (Yukawa) row,
// M_Y = M_s + M_D, and row 1 for a molecule's interior (Laplace) row,
// M_L = -(eps_out/eps_s) M_s - M_D, so that both rows are a plain sum a_k M_k.
#include "pbt_internal.h"

namespace pbt {

namespace {

// Index of the multi-index (a, b, c): ordered by n = a+b+c, then a
// descending, then b descending.
__host__ __device__ constexpr int tidx(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

struct MultiIdx {
  int8_t a, b, c, n;
};

__constant__ MultiIdx c_midx[ncoef(kMaxP)];
__constant__ int8_t c_binom[kMaxP + 1][kMaxP + 1];

template <typename T>
struct TMath;
template <>
struct TMath<float> {
  static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float expm(float x) { return __builtin_amdgcn_exp2f(-x * 1.4426950408889634f); }
};
template <>
struct TMath<double> {
  static __device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
  static __device__ __forceinline__ double expm(double x) { return exp(-x); }
};

#include "near_field.h"

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// ---- P2M: one wavefront per (leaf box, coefficient k), four coefficients
// per block; lanes over sources.  The exponents of k are uniform across the
// wavefront, so the power loops do not diverge.
template <typename T>
__global__ __launch_bounds__(256) void k_p2m(int P, const int32_t* __restrict__ boxes, BoxDev bd,
                                             const T* __restrict__ src, T* __restrict__ mom) {
  const int NC = ncoef(P);
  const int b = boxes[blockIdx.x];
  const int k = blockIdx.y * 4 + (int)(threadIdx.x >> 6);
  if (k >= NC) return;
  const int lane = threadIdx.x & 63;
  const MultiIdx mi = c_midx[k];
  const T cx = (T)bd.center[3 * b], cy = (T)bd.center[3 * b + 1], cz = (T)bd.center[3 * b + 2];
  T ms = 0, md = 0;
#pragma unroll 4
  for (int j = bd.sbeg[b] + lane; j < bd.send[b]; j += 64) {
    const T* s = src + (int64_t)kSrcStride * j;
    const T hx = s[0] - cx, hy = s[1] - cy, hz = s[2] - cz;
    T px = 1, py = 1, pz = 1, qx = 0, qy = 0, qz = 0;  // h^a and a h^(a-1)
    for (int t = 0; t < mi.a; ++t) { qx = qx * hx + px; px *= hx; }
    for (int t = 0; t < mi.b; ++t) { qy = qy * hy + py; py *= hy; }
    for (int t = 0; t < mi.c; ++t) { qz = qz * hz + pz; pz *= hz; }
    ms += s[3] * (px * py * pz);
    md += s[4] * (qx * py * pz) + s[5] * (px * qy * pz) + s[6] * (px * py * qz);
  }
  ms = wave_sum(ms);
  md = wave_sum(md);
  if (lane == 0) {
    const T ri = (T)bd.rho_inv[b];
    mom[(int64_t)(2 * b) * NC + k] = ms + md;
    mom[(int64_t)(2 * b + 1) * NC + k] = -ri * ms - md;
  }
}

// ---- M2M: one block per (box, coefficient k); threads over the terms
// (descendant, m <= k) of
//   M_k(box) = sum_desc sum_{m <= k} C(k, m) delta^(k-m) M_m(desc),
// delta = c_desc - c_box (h = y - c_box = (y - c_desc) + delta).  The
// descendants are the box's leaves, whose moments come from P2M, so every
// box is done in the same launch.
constexpr int kM2MThreads = 256;
template <typename T>
__global__ __launch_bounds__(kM2MThreads) void k_m2m(int P, const int32_t* __restrict__ boxes, BoxDev bd,
                                                     T* __restrict__ mom) {
  __shared__ T red[kM2MThreads / 64][2];
  const int NC = ncoef(P);
  const int b = boxes[blockIdx.x];
  const int k = blockIdx.y;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const MultiIdx mk = c_midx[k];
  const int nb = mk.b + 1, nc = mk.c + 1;
  const int nterm = (mk.a + 1) * nb * nc;
  const int c0 = bd.child_beg[b], nchild = bd.child_end[b] - c0;
  const double pcx = bd.center[3 * b], pcy = bd.center[3 * b + 1], pcz = bd.center[3 * b + 2];
  T acc0 = 0, acc1 = 0;
#pragma unroll 2
  for (int t = threadIdx.x; t < nchild * nterm; t += kM2MThreads) {
    const int ci = t / nterm, r = t - ci * nterm;
    const int ma = r / (nb * nc), mb = (r / nc) % nb, mc = r % nc;
    const int c = bd.child_list[c0 + ci];
    const T dx = (T)(bd.center[3 * c] - pcx), dy = (T)(bd.center[3 * c + 1] - pcy),
            dz = (T)(bd.center[3 * c + 2] - pcz);
    T coef = (T)(c_binom[mk.a][ma] * c_binom[mk.b][mb] * c_binom[mk.c][mc]);
    for (int q = ma; q < mk.a; ++q) coef *= dx;
    for (int q = mb; q < mk.b; ++q) coef *= dy;
    for (int q = mc; q < mk.c; ++q) coef *= dz;
    const int m = tidx(ma, mb, mc);
    acc0 += coef * mom[(int64_t)(2 * c) * NC + m];
    acc1 += coef * mom[(int64_t)(2 * c + 1) * NC + m];
  }
  acc0 = wave_sum(acc0);
  acc1 = wave_sum(acc1);
  if (lane == 0) {
    red[wid][0] = acc0;
    red[wid][1] = acc1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T s0 = 0, s1 = 0;
    for (int w = 0; w < kM2MThreads / 64; ++w) {
      s0 += red[w][0];
      s1 += red[w][1];
    }
    mom[(int64_t)(2 * b) * NC + k] = s0;
    mom[(int64_t)(2 * b + 1) * NC + k] = s1;
  }
}

// ---- M2P -------------------------------------------------------------------
template <typename T, int P, bool YUK>
__device__ __forceinline__ T taylor_dot(T Rx, T Ry, T Rz, T kappa, const T* __restrict__ M) {
  constexpr int NC = ncoef(P);
  T A[NC];
  T B[YUK ? NC : 1];
  const T R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const T Rinv = TMath<T>::rsq(R2);
  const T invR2 = Rinv * Rinv;
  if (YUK) {
    const T e = TMath<T>::expm(kappa * (R2 * Rinv));
    A[0] = e * Rinv;
    B[0] = e;
  } else {
    A[0] = Rinv;
  }
  T acc = A[0] * M[0];
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    const T c1 = T(2 * n - 1) / T(n) * invR2;
    const T c2 = T(n - 1) / T(n) * invR2;
    const T c3 = kappa / T(n) * invR2;
    const T c4 = kappa / T(n);
#pragma unroll
    for (int a = n; a >= 0; --a) {
#pragma unroll
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        const int k = tidx(a, b, c);
        T S1 = 0, S2 = 0, T1 = 0, T2 = 0;
        if (a >= 1) { S1 += Rx * A[tidx(a - 1, b, c)]; if (YUK) T1 += Rx * B[tidx(a - 1, b, c)]; }
        if (b >= 1) { S1 += Ry * A[tidx(a, b - 1, c)]; if (YUK) T1 += Ry * B[tidx(a, b - 1, c)]; }
        if (c >= 1) { S1 += Rz * A[tidx(a, b, c - 1)]; if (YUK) T1 += Rz * B[tidx(a, b, c - 1)]; }
        if (a >= 2) { S2 += A[tidx(a - 2, b, c)]; if (YUK) T2 += B[tidx(a - 2, b, c)]; }
        if (b >= 2) { S2 += A[tidx(a, b - 2, c)]; if (YUK) T2 += B[tidx(a, b - 2, c)]; }
        if (c >= 2) { S2 += A[tidx(a, b, c - 2)]; if (YUK) T2 += B[tidx(a, b, c - 2)]; }
        if (YUK) {
          A[k] = c1 * S1 - c2 * S2 + c3 * (T1 - T2);
          B[k] = c4 * (S1 - S2);
        } else {
          A[k] = c1 * S1 - c2 * S2;
        }
        acc += A[k] * M[k];
      }
    }
  }
  return acc;
}

// One M2P task (64 targets x a list of boxes) on one wavefront, one target
// per lane.
template <typename T, int P>
__device__ __forceinline__ void m2p_task(const Task& task, const int32_t* __restrict__ blist,
                                         const T* __restrict__ tgt, const double* __restrict__ bcen,
                                         const T* __restrict__ mom, T kappa, T* __restrict__ partial) {
  constexpr int NC = ncoef(P);
  const int lane = threadIdx.x & 63;
  const int tbeg = task.tbeg, tcount = task.tcount;
  const int lbeg = task.lbeg, lend = task.lend;
  const int fused = task.fused;
  const int ti = tbeg + (lane < tcount ? lane : 0);
  const T tx = tgt[kTgtStride * ti], ty = tgt[kTgtStride * ti + 1], tz = tgt[kTgtStride * ti + 2];
  T l = 0, yy = 0;
  for (int r = lbeg; r < lend; ++r) {
    const int b = blist[r];
    const T Rx = tx - (T)bcen[3 * b], Ry = ty - (T)bcen[3 * b + 1], Rz = tz - (T)bcen[3 * b + 2];
    const T* M = mom + (int64_t)(2 * b) * NC;
    yy += taylor_dot<T, P, true>(Rx, Ry, Rz, kappa, M);
    if (fused) l += taylor_dot<T, P, false>(Rx, Ry, Rz, kappa, M + NC);
  }
  if (lane < tcount) {
    partial[2 * ((int64_t)task.slot * 64 + lane) + 0] = l;
    partial[2 * ((int64_t)task.slot * 64 + lane) + 1] = yy;
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_m2p(const Task* __restrict__ tasks, int ntasks,
                                             const int32_t* __restrict__ blist,
                                             const T* __restrict__ tgt,
                                             const double* __restrict__ bcen,
                                             const T* __restrict__ mom, T kappa,
                                             T* __restrict__ partial) {
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= ntasks) return;
  m2p_task<T, P>(tasks[wv], blist, tgt, bcen, mom, kappa, partial);
}

// M2P tasks and P2P task pairs in one launch (M2P first): the far field's wavefronts
// and the near field's share the machine instead of running one after the
// other.
template <typename T, int P, bool GUARD>
__global__ __launch_bounds__(256) void k_m2p_p2p(const Task* __restrict__ m2p, int nm2p,
                                                 const int32_t* __restrict__ blist,
                                                 const double* __restrict__ bcen, const T* __restrict__ mom,
                                                 const Task* __restrict__ p2p, int np2p,
                                                 const int32_t* __restrict__ ranges, const T* __restrict__ src,
                                                 const T* __restrict__ tgt, T kappa, T* __restrict__ partial,
                                                 T* __restrict__ ppartial) {
  __shared__ SrcRec<T> tiles[4][64];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv < nm2p) m2p_task<T, P>(m2p[wv], blist, tgt, bcen, mom, kappa, partial);
  else if (wv < nm2p + np2p)
    p2p_task_pair<T, GUARD>(p2p + 2 * (wv - nm2p), tiles[threadIdx.x >> 6], ranges, tgt, src, kappa, ppartial);
}

bool g_tables_ready[64] = {false};

void upload_tables() {
  int dev = 0;
  PBT_HIP(hipGetDevice(&dev));
  if (dev < 64 && g_tables_ready[dev]) return;
  MultiIdx h[ncoef(kMaxP)];
  for (int n = 0; n <= kMaxP; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        h[tidx(a, b, c)] = MultiIdx{(int8_t)a, (int8_t)b, (int8_t)c, (int8_t)n};
      }
  int8_t bin[kMaxP + 1][kMaxP + 1] = {};
  for (int n = 0; n <= kMaxP; ++n) {
    bin[n][0] = 1;
    for (int k = 1; k <= n; ++k) bin[n][k] = (int8_t)(bin[n - 1][k - 1] + (k <= n - 1 ? bin[n - 1][k] : 0));
  }
  PBT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_midx), h, sizeof(h)));
  PBT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), bin, sizeof(bin)));
  if (dev < 64) g_tables_ready[dev] = true;
}

}  // namespace

template <typename T>
void launch_p2m(int P, int nbox, const int32_t* boxes, const BoxDev& b, const T* src, T* mom,
                hipStream_t s) {
  if (nbox <= 0) return;
  upload_tables();
  k_p2m<T><<<dim3(nbox, (ncoef(P) + 3) / 4), 256, 0, s>>>(P, boxes, b, src, mom);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_m2m(int P, int nbox, const int32_t* boxes, const BoxDev& b, T* mom, hipStream_t s) {
  if (nbox <= 0) return;
  upload_tables();
  k_m2m<T><<<dim3(nbox, ncoef(P)), kM2MThreads, 0, s>>>(P, boxes, b, mom);
  PBT_HIP(hipGetLastError());
}

template <typename T, int P>
static void m2p_p(const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                  const double* bcen, const T* mom, T kappa, T* partial, hipStream_t s) {
  const int blocks = ((ntasks + 3) / 4 + 7) / 8 * 8;
  k_m2p<T, P><<<blocks, 256, 0, s>>>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial);
}

template <typename T>
void launch_m2p(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                const double* bcen, const T* mom, T kappa, T* partial, hipStream_t s) {
  if (ntasks <= 0) return;
  switch (P) {
    case 0: m2p_p<T, 0>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 1: m2p_p<T, 1>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 2: m2p_p<T, 2>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 3: m2p_p<T, 3>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 4: m2p_p<T, 4>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 5: m2p_p<T, 5>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 6: m2p_p<T, 6>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 7: m2p_p<T, 7>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 8: m2p_p<T, 8>(tasks, ntasks, blist, tgt, bcen, mom, kappa, partial, s); break;
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template <typename T, int P>
static void m2p_p2p_p(const Task* m2p, int nm2p, const int32_t* blist, const double* bcen, const T* mom,
                      const Task* p2p, int np2p, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                      bool guard, T* partial, T* ppartial, hipStream_t s) {
  const int blocks = ((nm2p + np2p + 3) / 4 + 7) / 8 * 8;
  if (guard)
    k_m2p_p2p<T, P, true><<<blocks, 256, 0, s>>>(m2p, nm2p, blist, bcen, mom, p2p, np2p, ranges, src, tgt,
                                                 kappa, partial, ppartial);
  else
    k_m2p_p2p<T, P, false><<<blocks, 256, 0, s>>>(m2p, nm2p, blist, bcen, mom, p2p, np2p, ranges, src, tgt,
                                                  kappa, partial, ppartial);
}

template <typename T>
void launch_m2p_p2p(int P, const Task* m2p, int nm2p, const int32_t* blist, const double* bcen, const T* mom,
                    const Task* p2p, int np2p, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                    bool guard, T* partial, T* ppartial, hipStream_t s) {
  if (nm2p + np2p <= 0) return;
  switch (P) {
#define PBT_CASE(PP)                                                                                      \
  case PP:                                                                                                \
    m2p_p2p_p<T, PP>(m2p, nm2p, blist, bcen, mom, p2p, np2p, ranges, src, tgt, kappa, guard, partial, ppartial, \
                     s);                                                                                  \
    break;
    PBT_CASE(0) PBT_CASE(1) PBT_CASE(2) PBT_CASE(3) PBT_CASE(4) PBT_CASE(5) PBT_CASE(6) PBT_CASE(7) PBT_CASE(8)
#undef PBT_CASE
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template void launch_p2m<float>(int, int, const int32_t*, const BoxDev&, const float*, float*, hipStream_t);
template void launch_p2m<double>(int, int, const int32_t*, const BoxDev&, const double*, double*, hipStream_t);
template void launch_m2m<float>(int, int, const int32_t*, const BoxDev&, float*, hipStream_t);
template void launch_m2m<double>(int, int, const int32_t*, const BoxDev&, double*, hipStream_t);
template void launch_m2p_p2p<float>(int, const Task*, int, const int32_t*, const double*, const float*,
                                    const Task*, int, const int32_t*, const float*, const float*, float, bool,
                                    float*, float*, hipStream_t);
template void launch_m2p_p2p<double>(int, const Task*, int, const int32_t*, const double*, const double*,
                                     const Task*, int, const int32_t*, const double*, const double*, double, bool,
                                     double*, double*, hipStream_t);
template void launch_m2p<float>(int, const Task*, int, const int32_t*, const float*, const double*,
                                const float*, float, float*, hipStream_t);
template void launch_m2p<double>(int, const Task*, int, const int32_t*, const double*, const double*,
                                 const double*, double, double*, hipStream_t);

}  // namespace pbt
