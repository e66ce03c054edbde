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
#include <type_traits>

#include "pbt_internal.h"

namespace pbt {

namespace {

// Index of the multi-index (a, b, c): ordered by n = a+b+c, then a
// descending, then b descending.
__host__ __device__ constexpr int tidx(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

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

// ---- Moments (P2M) -----------------------------------------------------------
// The leaves' moments (and those of any box given to P2M) straight from
// their sources (a box's sources are contiguous in tree order).  Large boxes
// are cut into chunks of at most kMomChunk sources; one wavefront per (chunk,
// group of kMomGroup coefficients), lanes over the chunk's sources, each lane
// accumulating the group's coefficients of both rows in registers:
//   row 0: sum_j s_j h^k + D_j . grad h^k,   row 1: -rho_inv s_j h^k - D_j . grad h^k
// with grad h^k = (a h^(k-e_x), b h^(k-e_y), c h^(k-e_z)).  The wavefront adds
// its lanes' sums up by a fixed butterfly (no LDS, no barrier).  A box of
// several chunks has its chunk sums written to partial slots, which a second
// launch adds in chunk order, so results do not depend on scheduling.
constexpr int kMomThreads = 256;

__host__ __device__ constexpr int midx_n(int k) {
  int n = 0;
  while (tidx(n + 1, 0, 0) <= k) ++n;
  return n;
}
__host__ __device__ constexpr int midx_m(int k) {  // b + c
  const int r = k - tidx(midx_n(k), 0, 0);
  int m = 0;
  while ((m + 1) * (m + 2) / 2 <= r) ++m;
  return m;
}
__host__ __device__ constexpr int midx_c(int k) { return k - tidx(midx_n(k), 0, 0) - midx_m(k) * (midx_m(k) + 1) / 2; }
__host__ __device__ constexpr int midx_b(int k) { return midx_m(k) - midx_c(k); }
__host__ __device__ constexpr int midx_a(int k) { return midx_n(k) - midx_m(k); }

template <typename T, int P, int K0, int K1>
__device__ __forceinline__ void moments_group(const MomChunk& ch, const double* __restrict__ bcen,
                                              const double* __restrict__ brho, const T* __restrict__ src,
                                              T* __restrict__ mom, T* __restrict__ mpart) {
  constexpr int NC = ncoef(P);
  constexpr int NG = K1 - K0;
  const int lane = threadIdx.x & 63;
  const int b = ch.box;
  const T cx = (T)bcen[3 * b], cy = (T)bcen[3 * b + 1], cz = (T)bcen[3 * b + 2];
  const T ri = (T)brho[b];
  T acc[2 * NG];
#pragma unroll
  for (int q = 0; q < 2 * NG; ++q) acc[q] = 0;
  const SrcRec<T>* srec = reinterpret_cast<const SrcRec<T>*>(src);
  for (int j = ch.sbeg + lane; j < ch.send; j += 64) {
    const SrcRec<T> r = load_rec(srec + j);
    const T hx = r.v[0] - cx, hy = r.v[1] - cy, hz = r.v[2] - cz;
    const T s = r.v[3], sl = -ri * r.v[3];
    T px[P + 1], py[P + 1], pz[P + 1], dx[P + 1], dy[P + 1], dz[P + 1];
    px[0] = py[0] = pz[0] = T(1);
    dx[0] = dy[0] = dz[0] = T(0);
#pragma unroll
    for (int e = 1; e <= P; ++e) {
      // d*[e] = e D h^(e-1): the derivative factor of the e-th power
      dx[e] = r.v[4] * (T(e) * px[e - 1]);
      dy[e] = r.v[5] * (T(e) * py[e - 1]);
      dz[e] = r.v[6] * (T(e) * pz[e - 1]);
      px[e] = px[e - 1] * hx;
      py[e] = py[e - 1] * hy;
      pz[e] = pz[e - 1] * hz;
    }
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      const int a = midx_a(k), bb = midx_b(k), c = midx_c(k);
      const T pyz = py[bb] * pz[c];
      const T hk = px[a] * pyz;
      T d = 0;
      if (a) d += dx[a] * pyz;
      if (bb) d += dy[bb] * (px[a] * pz[c]);
      if (c) d += dz[c] * (px[a] * py[bb]);
      acc[2 * (k - K0)] += s * hk + d;
      acc[2 * (k - K0) + 1] += sl * hk - d;
    }
  }
  // the wavefront's sums by a fixed xor butterfly; lane q keeps sum q
  // (coefficient K0 + q/2, row q%2) and writes it
  T out = 0;
#pragma unroll
  for (int q = 0; q < 2 * NG; ++q) {
    T v = acc[q];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == q) out = v;
  }
  if (lane < 2 * NG) {
    const int k = K0 + (lane >> 1), row = lane & 1;
    if (ch.nparts == 1) mom[(int64_t)(2 * b + row) * NC + k] = out;
    else mpart[((int64_t)(ch.slot0 + ch.idx) * NC + k) * 2 + row] = out;
  }
}

template <typename T, int P, int GS, int G>
__device__ __forceinline__ void moments_dispatch(const MomChunk& ch, int gi, const double* bcen, const double* brho,
                                                 const T* src, T* mom, T* mpart) {
  constexpr int K0 = G * GS;
  if constexpr (K0 < ncoef(P)) {
    constexpr int K1 = K0 + GS < ncoef(P) ? K0 + GS : ncoef(P);
    if (gi == G) {
      moments_group<T, P, K0, K1>(ch, bcen, brho, src, mom, mpart);
      return;
    }
    moments_dispatch<T, P, GS, G + 1>(ch, gi, bcen, brho, src, mom, mpart);
  }
}

// One moments item on one wavefront: entry b of the item list is (chunk,
// coefficient group); a chunk marked fine takes groups of kMomGroupFine
// coefficients (a large box done by one chunk, its work spread over more
// wavefronts), otherwise kMomGroup.
template <typename T, int P>
__device__ __forceinline__ void moments_item(int b, const int32_t* __restrict__ mblocks,
                                             const MomChunk* __restrict__ chunks, const double* bcen,
                                             const double* brho, const T* src, T* mom, T* mpart) {
  const MomChunk ch = chunks[mblocks[2 * b]];
  const int gi = mblocks[2 * b + 1];
  if (ch.fine) moments_dispatch<T, P, kMomGroupFine, 0>(ch, gi, bcen, brho, src, mom, mpart);
  else moments_dispatch<T, P, kMomGroup, 0>(ch, gi, bcen, brho, src, mom, mpart);
}

// Four moments items a block, one a wavefront.
template <typename T, int P>
__global__ __launch_bounds__(kMomThreads) void k_moments(int nitems, const int32_t* __restrict__ mblocks,
                                                         const MomChunk* __restrict__ chunks,
                                                         const double* __restrict__ bcen,
                                                         const double* __restrict__ brho,
                                                         const T* __restrict__ src, T* __restrict__ mom,
                                                         T* __restrict__ mpart) {
  const int it = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  if (it >= nitems) return;
  moments_item<T, P>(it, mblocks, chunks, bcen, brho, src, mom, mpart);
}

// Boxes of several chunks: their moments are the chunk sums added in chunk
// order.  One block per box, threads over the 2 ncoef(P) values.
template <typename T>
__global__ __launch_bounds__(256) void k_moments_sum(const MomChunk* __restrict__ heads, int NC,
                                                     const T* __restrict__ mpart, T* __restrict__ mom) {
  const MomChunk h = heads[blockIdx.x];
  for (int t = threadIdx.x; t < 2 * NC; t += 256) {
    const int k = t >> 1, row = t & 1;
    T v = 0;
    for (int i = 0; i < h.nparts; ++i) v += mpart[((int64_t)(h.slot0 + i) * NC + k) * 2 + row];
    mom[(int64_t)(2 * h.box + row) * NC + k] = v;
  }
}

// ---- M2M -------------------------------------------------------------------
// A box's moments about its centre c from a leaf's about its own, c': with
// d = c' - c, (y - c)^k = sum_{l <= k} C(k, l) (y - c')^l d^(k - l)
// (multi-index binomials), and grad_y commutes with the shift, so for both
// rows   M_k(c) = sum_leaves sum_{l <= k} C(k, l) d^(k - l) M_l(c').
// Every leaf under a box is shifted straight to the box (no level-by-level
// chain, so all shifts run in one launch); the multi-index sum factorises
// into three one-dimensional Taylor shifts, along x, y and z in turn: on each
// line of coefficients that differ only in that component (e = 0..L),
// new(t) = sum_{e <= t} C(t, e) d^(t - e) old(e), done in place for t from L
// down.  One thread per (pair, row) holds the row's coefficients in
// registers (every index a compile-time constant); the result goes to the
// pair's slot, and a second launch adds each box's slots in leaf order.
__host__ __device__ constexpr int binom(int n, int k) {
  int v = 1;
  for (int q = 1; q <= k; ++q) v = v * (n - k + q) / q;
  return v;
}

template <int D>
__host__ __device__ constexpr int line_idx(int e, int u, int v) {
  return D == 0 ? tidx(e, u, v) : D == 1 ? tidx(u, e, v) : tidx(u, v, e);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <typename T, int P, int D>
__device__ __forceinline__ void shift_pass(T* m, T d) {
  T pw[P + 1];
  pw[0] = T(1);
#pragma unroll
  for (int e = 1; e <= P; ++e) pw[e] = pw[e - 1] * d;
  static_for<0, P + 1>([&](auto U) {
    constexpr int u = decltype(U)::value;
    static_for<0, P + 1 - u>([&](auto V) {
      constexpr int v = decltype(V)::value;
      constexpr int L = P - u - v;
      // t from L down to 1
      static_for<0, L>([&](auto Q) {
        constexpr int t = L - decltype(Q)::value;
        T acc = m[line_idx<D>(t, u, v)];
        static_for<0, t>([&](auto E) {
          constexpr int e = decltype(E)::value;
          acc += (T(binom(t, e)) * pw[t - e]) * m[line_idx<D>(e, u, v)];
        });
        m[line_idx<D>(t, u, v)] = acc;
      });
    });
  });
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_m2m_shift(int npairs, const int32_t* __restrict__ pairs,
                                                   const double* __restrict__ bcen,
                                                   const T* __restrict__ mom, T* __restrict__ slots) {
  constexpr int NC = ncoef(P);
  const int t = blockIdx.x * 256 + (int)threadIdx.x;
  if (t >= 2 * npairs) return;
  const int pr = t >> 1, row = t & 1;
  const int b = pairs[3 * pr], leaf = pairs[3 * pr + 1], slot = pairs[3 * pr + 2];
  const T* in = mom + (int64_t)(2 * leaf + row) * NC;
  T m[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) m[k] = in[k];
  shift_pass<T, P, 0>(m, (T)(bcen[3 * leaf] - bcen[3 * b]));
  shift_pass<T, P, 1>(m, (T)(bcen[3 * leaf + 1] - bcen[3 * b + 1]));
  shift_pass<T, P, 2>(m, (T)(bcen[3 * leaf + 2] - bcen[3 * b + 2]));
  T* out = slots + ((int64_t)slot * 2 + row) * NC;
#pragma unroll
  for (int k = 0; k < NC; ++k) out[k] = m[k];
}

// Per box, its n slots added up.  Boxes of at most kM2MSmall leaves (heads
// listed first): one block per box, a thread per output value, its slots
// loaded in batches of 8 so that the loads are in flight together, and
// added in slot order.  The others: a wavefront per output value, lane l
// adding slots l, l + 64, ... (in batches of 8 loads), then a fixed xor
// butterfly over the 64 lanes.
template <typename T>
__global__ __launch_bounds__(256) void k_m2m_sum_small(int NO, const int32_t* __restrict__ heads,
                                                       const T* __restrict__ slots, T* __restrict__ mom) {
  const int b = heads[3 * blockIdx.x], s0 = heads[3 * blockIdx.x + 1], n = heads[3 * blockIdx.x + 2];
  for (int o = threadIdx.x; o < NO; o += 256) {
    const T* p = slots + (int64_t)s0 * NO + o;
    T acc = T(0);
    for (int i0 = 0; i0 < n; i0 += 8) {
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = i0 + q < n ? p[(int64_t)(i0 + q) * NO] : T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += v[q];
    }
    mom[(int64_t)b * NO + o] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_m2m_sum(int NO, const int32_t* __restrict__ heads,
                                                 const T* __restrict__ slots, T* __restrict__ mom) {
  const int b = heads[3 * blockIdx.x], s0 = heads[3 * blockIdx.x + 1], n = heads[3 * blockIdx.x + 2];
  const int o = blockIdx.y * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= NO) return;   // whole wavefronts
  const T* p = slots + (int64_t)s0 * NO + o;
  T acc = T(0);
  for (int i0 = lane; i0 < n; i0 += 8 * 64) {
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = i0 + 64 * q < n ? p[(int64_t)(i0 + 64 * q) * NO] : T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += v[q];
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) mom[(int64_t)b * NO + o] = acc;
}

// ---- M2P -------------------------------------------------------------------
// The recurrences above, evaluated with the first-neighbour sums taken
// against pre-scaled R: with u = (2n-1)/(n|R|^2) R and v = kappa/(n|R|^2) R,
//   Laplace  a_k = sum_i u_i a_{k-e_i} - (n-1)/(n|R|^2) sum_i a_{k-2e_i}
//   Yukawa   a_k = sum_i u_i a_{k-e_i} + sum_i v_i b_{k-e_i}
//                  - (n-1)/(n|R|^2) sum_i a_{k-2e_i} - kappa/(n|R|^2) sum_i b_{k-2e_i}
//            b_k = kappa |R|^2/(2n-1) sum_i u_i a_{k-e_i} - kappa/n sum_i a_{k-2e_i}
// (the same quantities, one multiplication fewer per coefficient).
// A wave-uniform zero that the compiler cannot see through, produced after
// v (orders a computation after v's).
template <typename T>
__device__ __forceinline__ int zero_after(T v) {
  int z;
  __asm__ volatile("s_mov_b32 %0, 0" : "=s"(z) : "v"(v));
  return z;
}

// The Taylor coefficients of the kernel (Yukawa, or Laplace), degree by
// degree: pre(n) runs at the start of degree n >= 1, between scheduling
// barriers (reads that the degree's use of its coefficients waits for are
// issued there, so that the recurrence hides their latency), and post(n, A)
// once A holds the coefficients of degrees 0..n.
template <typename T, int P, bool YUK, typename Pre, typename Post>
__device__ __forceinline__ void taylor_series(T Rx, T Ry, T Rz, T kappa, Pre&& pre, Post&& post) {
  constexpr int NC = ncoef(P);
  T A[NC];
  T B[YUK ? NC : 1];
  const T R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const T Rinv = TMath<T>::rsq(R2);
  const T invR2 = Rinv * Rinv;
  const T kR2 = kappa * R2;
  if (YUK) {
    const T e = TMath<T>::expm(kappa * (R2 * Rinv));
    A[0] = e * Rinv;
    B[0] = e;
  } else {
    A[0] = Rinv;
  }
  post(std::integral_constant<int, 0>{}, A);
  static_for<1, P + 1>([&](auto N) {
    constexpr int n = decltype(N)::value;
    __builtin_amdgcn_sched_barrier(0);
    pre(N);
    __builtin_amdgcn_sched_barrier(0);
    const T c1 = T(2 * n - 1) / T(n) * invR2;
    const T c2 = T(n - 1) / T(n) * invR2;
    const T c3 = kappa * (T(1) / T(n)) * invR2;
    const T c4 = kappa * (T(1) / T(n));
    const T e4 = kR2 * (T(1) / T(2 * n - 1));
    const T ux = c1 * Rx, uy = c1 * Ry, uz = c1 * Rz;
    T vx = 0, vy = 0, vz = 0;
    if (YUK) { vx = c3 * Rx; vy = c3 * Ry; vz = c3 * Rz; }
#pragma unroll
    for (int a = n; a >= 0; --a) {
#pragma unroll
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        const int k = tidx(a, b, c);
        // each sum starts from its first term (no zero start: x * y + 0 is
        // an instruction of its own unless the compiler may drop the +0)
        T S1, S2, T1, T2;
        bool h1 = false, h2 = false;
        auto first = [&](T u, T v, int i) {
          if (!h1) { S1 = u * A[i]; if (YUK) T1 = v * B[i]; }
          else { S1 += u * A[i]; if (YUK) T1 += v * B[i]; }
          h1 = true;
        };
        auto second = [&](int i) {
          if (!h2) { S2 = A[i]; if (YUK) T2 = B[i]; }
          else { S2 += A[i]; if (YUK) T2 += B[i]; }
          h2 = true;
        };
        if (a >= 1) first(ux, vx, tidx(a - 1, b, c));
        if (b >= 1) first(uy, vy, tidx(a, b - 1, c));
        if (c >= 1) first(uz, vz, tidx(a, b, c - 1));
        if (a >= 2) second(tidx(a - 2, b, c));
        if (b >= 2) second(tidx(a, b - 2, c));
        if (c >= 2) second(tidx(a, b, c - 2));
        if (YUK) {
          A[k] = h2 ? (S1 + T1) - c2 * S2 - c3 * T2 : S1 + T1;
          if (n < P) B[k] = h2 ? e4 * S1 - c4 * S2 : e4 * S1;
        } else {
          A[k] = h2 ? S1 - c2 * S2 : S1;
        }
      }
    }
    post(N, A);
  });
}

// sum_k a_k M_k with the moments M in LDS (a per-lane address): each
// degree's are read at its start, kept there by scheduling barriers, so
// that the degree's recurrence hides their latency and one degree of them
// is live at a time.
template <typename T, int P, bool YUK>
__device__ __forceinline__ T taylor_dot(T Rx, T Ry, T Rz, T kappa, const T* M) {
  T acc = T(0);
  T mo[(P + 1) * (P + 2) / 2];
  taylor_series<T, P, YUK>(
      Rx, Ry, Rz, kappa,
      [&](auto N) {
        constexpr int n = decltype(N)::value;
#pragma unroll
        for (int k = tidx(n, 0, 0); k < tidx(n + 1, 0, 0); ++k) mo[k - tidx(n, 0, 0)] = M[k];
      },
      [&](auto N, const T* A) {
        constexpr int n = decltype(N)::value;
        if constexpr (n == 0) {
          acc = A[0] * M[0];
        } else {
#pragma unroll
          for (int k = tidx(n, 0, 0); k < tidx(n + 1, 0, 0); ++k) acc += A[k] * mo[k - tidx(n, 0, 0)];
        }
      });
  return acc;
}

// Salt-free solvent (kappa = 0): both rows use the Laplace coefficients, so
// they are formed once and dotted with both moment rows.
template <typename T, int P>
__device__ __forceinline__ void taylor_dot_two(T Rx, T Ry, T Rz, const T* __restrict__ M, T& yy, T& l) {
  constexpr int NC = ncoef(P);
  T A[NC];
  const T R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const T Rinv = TMath<T>::rsq(R2);
  const T invR2 = Rinv * Rinv;
  A[0] = Rinv;
  T a0 = A[0] * M[0], a1 = A[0] * M[NC];
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    // both rows' moments of the degree (as in taylor_dot)
    T m0[(P + 1) * (P + 2) / 2], m1[(P + 1) * (P + 2) / 2];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = tidx(n, 0, 0); k < tidx(n + 1, 0, 0); ++k) {
      m0[k - tidx(n, 0, 0)] = M[k];
      m1[k - tidx(n, 0, 0)] = M[NC + k];
    }
    __builtin_amdgcn_sched_barrier(0);
    const T c1 = T(2 * n - 1) / T(n) * invR2;
    const T c2 = T(n - 1) / T(n) * invR2;
    const T ux = c1 * Rx, uy = c1 * Ry, uz = c1 * Rz;
#pragma unroll
    for (int a = n; a >= 0; --a) {
#pragma unroll
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        const int k = tidx(a, b, c);
        T S1, S2;
        bool h1 = false, h2 = false;
        auto first = [&](T u, int i) {
          S1 = h1 ? S1 + u * A[i] : u * A[i];
          h1 = true;
        };
        auto second = [&](int i) {
          S2 = h2 ? S2 + A[i] : A[i];
          h2 = true;
        };
        if (a >= 1) first(ux, tidx(a - 1, b, c));
        if (b >= 1) first(uy, tidx(a, b - 1, c));
        if (c >= 1) first(uz, tidx(a, b, c - 1));
        if (a >= 2) second(tidx(a - 2, b, c));
        if (b >= 2) second(tidx(a, b - 2, c));
        if (c >= 2) second(tidx(a, b, c - 2));
        A[k] = h2 ? S1 - c2 * S2 : S1;
      }
    }
#pragma unroll
    for (int k = tidx(n, 0, 0); k < tidx(n + 1, 0, 0); ++k) {
      a0 += A[k] * m0[k - tidx(n, 0, 0)];
      a1 += A[k] * m1[k - tidx(n, 0, 0)];
    }
  }
  yy += a0;
  l += a1;
}

// A pair of M2P tasks on one wavefront: lanes 0..31 serve tp[0], lanes
// 32..63 tp[1], each up to 32 targets (one a lane) against its own list of
// boxes; both have the same `fused` and kFormKz.  Box by box, each half
// copies its box's moments (both rows with `fused`, the Yukawa row
// otherwise) from registers into its part of the wave's LDS region, and the
// lanes read them back as LDS broadcasts, so the dot products take their
// moments from vector registers; the next box's moments are loaded into
// registers while the current box is evaluated.  A half with fewer boxes
// idles (masked) while the other finishes.  Partials [slot][32][2].
template <typename T, int P, bool SALTFREE>
__device__ __forceinline__ void m2p_task_pair(const Task* __restrict__ tp, T* __restrict__ mlds,
                                              const int32_t* __restrict__ blist, const T* __restrict__ tgt,
                                              const double* __restrict__ bcen, const T* __restrict__ mom, T kappa,
                                              T* __restrict__ partial) {
  constexpr int NC = ncoef(P), NM = 2 * NC, PER = (NM + 31) / 32;
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const Task t = tp[half];
  // both halves agree on these: wave-uniform
  const int fused = __builtin_amdgcn_readfirstlane(tp[0].fused);
  // an outside sum inside a salt-free Stern layer: kappa = 0 (the Yukawa
  // recurrence then reduces to the Laplace one)
  if (__builtin_amdgcn_readfirstlane(tp[0].form) & kFormKz) kappa = T(0);
  const int nm = fused ? NM : NC;
  const int n = t.lend - t.lbeg;
  const int nmax = __builtin_amdgcn_readfirstlane(max(tp[0].lend - tp[0].lbeg, tp[1].lend - tp[1].lbeg));
  const int ti = t.tbeg + (hl < t.tcount ? hl : 0);
  const T tx = tgt[kTgtStride * ti], ty = tgt[kTgtStride * ti + 1], tz = tgt[kTgtStride * ti + 2];
  T* mine = mlds + half * NM;
  // every lane evaluates a box of its half's list each round (the last one
  // again once its list is done, entry 0 of the list array for an empty
  // half) and keeps the result only while its list lasts: no divergence.
  // Box indices, centres and moments are loaded a round ahead, so a round
  // waits on no memory latency but the LDS reads of its own moments.
  const int last = t.lbeg + max(n - 1, 0);
  auto box = [&](int r) { return blist[min(t.lbeg + r, last)]; };
  T pre[PER];
  auto fetch = [&](int b) {
    const T* M = mom + (int64_t)(2 * b) * NC;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = hl + 32 * q;
      pre[q] = i < nm ? M[i] : T(0);
    }
  };
  int b = box(0);
  fetch(b);
  double cx = bcen[3 * b], cy = bcen[3 * b + 1], cz = bcen[3 * b + 2];
  int bn = box(1);
  T l = 0, yy = 0;
  for (int r = 0; r < nmax; ++r) {
    wave_lds_sync();   // the previous box's reads are done
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = hl + 32 * q;
      if (i < nm) mine[i] = pre[q];
    }
    wave_lds_sync();
    const T Rx = tx - (T)cx, Ry = ty - (T)cy, Rz = tz - (T)cz;
    if (r + 1 < nmax) {
      fetch(bn);
      cx = bcen[3 * bn];
      cy = bcen[3 * bn + 1];
      cz = bcen[3 * bn + 2];
      bn = box(r + 2);
    }
    T dy = 0, dl = 0;
    if (SALTFREE) {
      if (fused) taylor_dot_two<T, P>(Rx, Ry, Rz, mine, dy, dl);
      else dy = taylor_dot<T, P, false>(Rx, Ry, Rz, kappa, mine);
    } else {
      dy = taylor_dot<T, P, true>(Rx, Ry, Rz, kappa, mine);
      if (fused) {
        // the Laplace expansion after the Yukawa one (an opaque zero taken
        // from its result): interleaving the two would hold both sets of
        // coefficients in registers at once
        const T z = (T)zero_after(dy);
        dl = taylor_dot<T, P, false>(Rx + z, Ry + z, Rz + z, kappa, mine + NC);
      }
    }
    const bool on = r < n;
    yy += on ? dy : T(0);
    l += on ? dl : T(0);
  }
  if (hl < t.tcount) {
    T o0 = l, o1 = yy;
    if (t.form & kFormDropOut) o1 = T(0);
    if (t.form & kFormSwap) {
      const T sw = o0;
      o0 = o1;
      o1 = sw;
    }
    partial[2 * ((int64_t)t.slot * 32 + hl) + 0] = o0;
    partial[2 * ((int64_t)t.slot * 32 + hl) + 1] = o1;
  }
}

// One wavefront per pair of M2P tasks (four per block).
template <typename T, int P, bool SALTFREE>
__global__ __launch_bounds__(256) void k_m2p(const Task* __restrict__ tasks, int npairs,
                                             const int32_t* __restrict__ blist,
                                             const T* __restrict__ tgt,
                                             const double* __restrict__ bcen,
                                             const T* __restrict__ mom, T kappa,
                                             T* __restrict__ partial) {
  __shared__ T mlds[4][4 * ncoef(P)];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= npairs) return;
  m2p_task_pair<T, P, SALTFREE>(tasks + 2 * wv, mlds[threadIdx.x >> 6], blist, tgt, bcen, mom, kappa, partial);
}

// ---- M2P between surfaces shared by every group of a batch ------------------
// A target and a box of two surfaces that every group holds unmoved have the
// same R = x - c in every group, so the coefficients a_k(R) are formed once
// and dotted with the moments of the box's copy in kMultiPass groups at a
// time.  The moments of a pass are staged in LDS as rows of coefficients,
// one column per group (row stride kMultiRow, 16-byte aligned).
constexpr int kMultiPass = 8, kMultiRow = 12;

template <typename T, int P, bool YUK>
__device__ __forceinline__ void taylor_dot_multi(T Rx, T Ry, T Rz, T kappa, const T* __restrict__ M,
                                                 T (&d)[kMultiPass]) {
  taylor_series<T, P, YUK>(
      Rx, Ry, Rz, kappa, [&](auto) {},
      [&](auto N, const T* A) {
        constexpr int n = decltype(N)::value;
#pragma unroll
        for (int k = tidx(n, 0, 0); k < tidx(n + 1, 0, 0); ++k)
#pragma unroll
          for (int g = 0; g < kMultiPass; ++g) {
            if (n == 0) d[g] = A[k] * M[k * kMultiRow + g];
            else d[g] += A[k] * M[k * kMultiRow + g];
          }
      });
}

// A pair of shared-surface M2P tasks on one wavefront (lanes 0..31: tp[0],
// 32..63: tp[1], one target a lane, Yukawa-only rows, both serving groups
// split .. split + kMultiBlock - 1; nsrc is the row of boxoff that holds, per
// group, the offset of its copy's box numbers from group 0's).  Box by box
// and pass by pass, each half stages the moments of the box's copies in the
// pass's groups (row 0) and every lane adds sum_k a_k M_k per group; a half
// with fewer boxes evaluates its last box again and discards it.
template <typename T, int P, bool SALTFREE>
__device__ __forceinline__ void m2p_multi_pair(const Task* __restrict__ tp, T* __restrict__ mlds,
                                               const int32_t* __restrict__ blist, const T* __restrict__ tgt,
                                               const double* __restrict__ bcen, const T* __restrict__ mom,
                                               const int32_t* __restrict__ boxoff, const int32_t* __restrict__ mslot,
                                               int G, T kappa, T* __restrict__ partial) {
  constexpr int NC = ncoef(P), PER = (NC + 31) / 32;
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const Task t = tp[half];
  const int n = t.lend - t.lbeg;
  const int nmax = __builtin_amdgcn_readfirstlane(max(tp[0].lend - tp[0].lbeg, tp[1].lend - tp[1].lbeg));
  const int ti = t.tbeg + (hl < t.tcount ? hl : 0);
  const T tx = tgt[kTgtStride * ti], ty = tgt[kTgtStride * ti + 1], tz = tgt[kTgtStride * ti + 2];
  const int g0 = tp[0].split, g1 = min(G, g0 + kMultiBlock);
  const int32_t* off = boxoff + (int64_t)t.nsrc * G;
  const int last = t.lbeg + max(n - 1, 0);
  T* mine = mlds + half * (NC * kMultiRow);
  for (int gb = g0; gb < g1; gb += kMultiPass) {
    const int nb = min(kMultiPass, g1 - gb);
    T acc[kMultiPass];
#pragma unroll
    for (int g = 0; g < kMultiPass; ++g) acc[g] = T(0);
    for (int r = 0; r < nmax; ++r) {
      const int b = blist[min(t.lbeg + r, last)];
      // stage: coefficient i of group gb + g at mine[i * kMultiRow + g]
      // (groups past the block's last read its last group's and are
      // never used)
      T v[PER][kMultiPass];
#pragma unroll
      for (int g = 0; g < kMultiPass; ++g) {
        const T* M = mom + (int64_t)(2 * (b + off[min(gb + g, g1 - 1)])) * NC;
#pragma unroll
        for (int q = 0; q < PER; ++q) v[q][g] = M[min(hl + 32 * q, NC - 1)];
      }
      wave_lds_sync();   // the previous box's reads are done
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (hl + 32 * q < NC)
#pragma unroll
          for (int g = 0; g < kMultiPass; ++g) mine[(hl + 32 * q) * kMultiRow + g] = v[q][g];
      wave_lds_sync();
      const T Rx = tx - (T)bcen[3 * b], Ry = ty - (T)bcen[3 * b + 1], Rz = tz - (T)bcen[3 * b + 2];
      T d[kMultiPass];
      taylor_dot_multi<T, P, !SALTFREE>(Rx, Ry, Rz, kappa, mine, d);
      const bool on = r < n;
#pragma unroll
      for (int g = 0; g < kMultiPass; ++g) acc[g] += on ? d[g] : T(0);
    }
    if (hl < t.tcount) {
#pragma unroll
      for (int g = 0; g < kMultiPass; ++g) {
        if (g >= nb) break;
        T o0 = T(0), o1 = acc[g];
        if (t.form & kFormDropOut) o1 = T(0);
        if (t.form & kFormSwap) {
          const T sw = o0;
          o0 = o1;
          o1 = sw;
        }
        const int64_t slot = mslot[(int64_t)t.slot * G + gb + g];
        partial[2 * (slot * 32 + hl) + 0] = o0;
        partial[2 * (slot * 32 + hl) + 1] = o1;
      }
    }
  }
}

// One wavefront per pair of shared-surface M2P tasks (four per block).
template <typename T, int P, bool SALTFREE>
__global__ __launch_bounds__(256) void k_m2p_multi(const Task* __restrict__ tasks, int npairs,
                                                   const int32_t* __restrict__ blist, const T* __restrict__ tgt,
                                                   const double* __restrict__ bcen, const T* __restrict__ mom,
                                                   const int32_t* __restrict__ boxoff,
                                                   const int32_t* __restrict__ mslot, int G, T kappa,
                                                   T* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) T mlds[4][2 * ncoef(P) * kMultiRow];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= npairs) return;
  m2p_multi_pair<T, P, SALTFREE>(tasks + 2 * wv, mlds[threadIdx.x >> 6], blist, tgt, bcen, mom, boxoff, mslot, G,
                                 kappa, partial);
}

// M2P task pairs and P2P task pairs in one launch (M2P first): the far
// field's wavefronts and the near field's share the machine instead of
// running one after the other.  Both write the half-wave partials.
template <typename T, int P, bool GUARD, bool SALTFREE>
__global__ __launch_bounds__(256) void k_m2p_p2p(const Task* __restrict__ m2p, int nm2p,
                                                 const int32_t* __restrict__ blist,
                                                 const double* __restrict__ bcen, const T* __restrict__ mom,
                                                 const Task* __restrict__ p2p, int np2p,
                                                 const int32_t* __restrict__ ranges, const T* __restrict__ src,
                                                 const T* __restrict__ tgt, T kappa, T* __restrict__ ppartial) {
  __shared__ SrcRec<T> tiles[4][64];
  __shared__ T mlds[4][4 * ncoef(P)];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv < nm2p)
    m2p_task_pair<T, P, SALTFREE>(m2p + 2 * wv, mlds[threadIdx.x >> 6], blist, tgt, bcen, mom, kappa, ppartial);
  else if (wv < nm2p + np2p)
    p2p_task_pair<T, GUARD>(p2p + 2 * (wv - nm2p), tiles[threadIdx.x >> 6], ranges, tgt, src, kappa, ppartial);
}

// Moments blocks and P2P task pairs in one launch (moments first, so the
// short moment blocks start at once and P2P fills the machine around them):
// nmb moment blocks (the block list, padded to a multiple of 8), then the P2P blocks, whose
// logical order is made XCD-aware on their own range (nmb is a multiple of 8).
template <typename T, int P, bool GUARD>
__global__ __launch_bounds__(256) void k_p2p_mom(int nmreal, int nmb, const int32_t* __restrict__ mblocks,
                                                 const MomChunk* __restrict__ chunks,
                                                 const double* __restrict__ bcen,
                                                 const double* __restrict__ brho, T* __restrict__ mom,
                                                 T* __restrict__ mpart, const Task* __restrict__ p2p, int npairs,
                                                 const int32_t* __restrict__ ranges, const T* __restrict__ src,
                                                 const T* __restrict__ tgt, T kappa, T* __restrict__ ppartial) {
  __shared__ SrcRec<T> tiles[4][64];
  if ((int)blockIdx.x < nmb) {
    // moments items, one a wavefront
    const int it = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    if (it >= nmreal) return;
    moments_item<T, P>(it, mblocks, chunks, bcen, brho, src, mom, mpart);
    return;
  }
  const int l = (int)blockIdx.x - nmb, per = ((int)gridDim.x - nmb) >> 3;
  const int wv = __builtin_amdgcn_readfirstlane(((l & 7) * per + (l >> 3)) * 4 + (int)(threadIdx.x >> 6));
  if (wv >= npairs) return;
  p2p_task_pair<T, GUARD>(p2p + 2 * wv, tiles[threadIdx.x >> 6], ranges, tgt, src, kappa, ppartial);
}

}  // namespace

template <typename T, int P>
static void moments_p(int nitems, const int32_t* mblocks, const MomChunk* chunks, const double* bcen,
                      const double* brho, const T* src, T* mom, T* mpart, hipStream_t s) {
  k_moments<T, P><<<(nitems + 3) / 4, kMomThreads, 0, s>>>(nitems, mblocks, chunks, bcen, brho, src, mom, mpart);
}

template <typename T>
void launch_moments(int P, int nblocks, const int32_t* mblocks, const MomChunk* chunks, int nheads,
                    const MomChunk* heads, const double* bcen, const double* brho, const T* src, T* mom, T* mpart,
                    hipStream_t s) {
  if (nblocks <= 0) return;
  switch (P) {
#define PBT_CASE(PP) \
  case PP: moments_p<T, PP>(nblocks, mblocks, chunks, bcen, brho, src, mom, mpart, s); break;
    PBT_CASE(0) PBT_CASE(1) PBT_CASE(2) PBT_CASE(3) PBT_CASE(4) PBT_CASE(5) PBT_CASE(6) PBT_CASE(7) PBT_CASE(8)
#undef PBT_CASE
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
  if (nheads > 0) {
    k_moments_sum<T><<<nheads, 256, 0, s>>>(heads, ncoef(P), mpart, mom);
    PBT_HIP(hipGetLastError());
  }
}

template <typename T, int P>
static void p2p_mom_p(int nmreal, const int32_t* mblocks, const MomChunk* chunks, const double* bcen,
                      const double* brho, T* mom, T* mpart, const Task* p2p, int npairs, const int32_t* ranges,
                      const T* src, const T* tgt, T kappa, bool guard, T* ppartial, hipStream_t s) {
  const int nmb = ((nmreal + 3) / 4 + 7) / 8 * 8;   // blocks of four moments items
  const int blocks = nmb + ((npairs + 3) / 4 + 7) / 8 * 8;
  if (guard)
    k_p2p_mom<T, P, true><<<blocks, 256, 0, s>>>(nmreal, nmb, mblocks, chunks, bcen, brho, mom, mpart, p2p, npairs,
                                                 ranges, src, tgt, kappa, ppartial);
  else
    k_p2p_mom<T, P, false><<<blocks, 256, 0, s>>>(nmreal, nmb, mblocks, chunks, bcen, brho, mom, mpart, p2p,
                                                  npairs, ranges, src, tgt, kappa, ppartial);
}

template <typename T>
void launch_p2p_moments(int P, int nblocks, const int32_t* mblocks, const MomChunk* chunks, int nheads,
                        const MomChunk* heads, const double* bcen, const double* brho, T* mom, T* mpart,
                        const Task* p2p, int npairs, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                        bool guard, T* ppartial, hipStream_t s) {
  if (nblocks + npairs <= 0) return;
  switch (P) {
#define PBT_CASE(PP)                                                                                               \
  case PP:                                                                                                         \
    p2p_mom_p<T, PP>(nblocks, mblocks, chunks, bcen, brho, mom, mpart, p2p, npairs, ranges, src, tgt, kappa, guard, \
                     ppartial, s);                                                                                 \
    break;
    PBT_CASE(0) PBT_CASE(1) PBT_CASE(2) PBT_CASE(3) PBT_CASE(4) PBT_CASE(5) PBT_CASE(6) PBT_CASE(7) PBT_CASE(8)
#undef PBT_CASE
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
  if (nheads > 0) {
    k_moments_sum<T><<<nheads, 256, 0, s>>>(heads, ncoef(P), mpart, mom);
    PBT_HIP(hipGetLastError());
  }
}

template <typename T>
void launch_m2m(int P, int npairs, const int32_t* pairs, int nheads, int nsmall, const int32_t* heads,
                const double* bcen, T* slots, T* mom, hipStream_t s) {
  if (nheads <= 0) return;
  const unsigned blocks = (unsigned)((2 * (int64_t)npairs + 255) / 256);
  switch (P) {
#define PBT_CASE(PP) \
  case PP: k_m2m_shift<T, PP><<<blocks, 256, 0, s>>>(npairs, pairs, bcen, mom, slots); break;
    PBT_CASE(0) PBT_CASE(1) PBT_CASE(2) PBT_CASE(3) PBT_CASE(4) PBT_CASE(5) PBT_CASE(6) PBT_CASE(7) PBT_CASE(8)
#undef PBT_CASE
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
  const int NO = 2 * ncoef(P);
  if (nsmall > 0) {
    k_m2m_sum_small<T><<<nsmall, 256, 0, s>>>(NO, heads, slots, mom);
    PBT_HIP(hipGetLastError());
  }
  if (nheads > nsmall) {
    k_m2m_sum<T><<<dim3(nheads - nsmall, (NO + 3) / 4), 256, 0, s>>>(NO, heads + 3 * (int64_t)nsmall, slots, mom);
    PBT_HIP(hipGetLastError());
  }
}

template <typename T, int P>
static void m2p_p(const Task* tasks, int npairs, const int32_t* blist, const T* tgt,
                  const double* bcen, const T* mom, T kappa, T* partial, hipStream_t s) {
  const int blocks = ((npairs + 3) / 4 + 7) / 8 * 8;
  if (kappa == T(0))
    k_m2p<T, P, true><<<blocks, 256, 0, s>>>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial);
  else
    k_m2p<T, P, false><<<blocks, 256, 0, s>>>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial);
}

template <typename T>
void launch_m2p(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                const double* bcen, const T* mom, T kappa, T* partial, hipStream_t s) {
  if (ntasks <= 0) return;
  if (ntasks % 2) throw Error(1, "M2P half tasks come in pairs");
  const int npairs = ntasks / 2;
  switch (P) {
    case 0: m2p_p<T, 0>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 1: m2p_p<T, 1>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 2: m2p_p<T, 2>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 3: m2p_p<T, 3>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 4: m2p_p<T, 4>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 5: m2p_p<T, 5>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 6: m2p_p<T, 6>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 7: m2p_p<T, 7>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    case 8: m2p_p<T, 8>(tasks, npairs, blist, tgt, bcen, mom, kappa, partial, s); break;
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template <typename T, int P>
static void m2p_multi_p(const Task* tasks, int npairs, const int32_t* blist, const T* tgt, const double* bcen,
                        const T* mom, const int32_t* boxoff, const int32_t* mslot, int G, T kappa, T* partial,
                        hipStream_t s) {
  const int blocks = ((npairs + 3) / 4 + 7) / 8 * 8;
  if (kappa == T(0))
    k_m2p_multi<T, P, true><<<blocks, 256, 0, s>>>(tasks, npairs, blist, tgt, bcen, mom, boxoff, mslot, G, kappa,
                                                   partial);
  else
    k_m2p_multi<T, P, false><<<blocks, 256, 0, s>>>(tasks, npairs, blist, tgt, bcen, mom, boxoff, mslot, G, kappa,
                                                    partial);
}

template <typename T>
void launch_m2p_multi(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt, const double* bcen,
                      const T* mom, const int32_t* boxoff, const int32_t* mslot, int G, T kappa, T* partial,
                      hipStream_t s) {
  if (ntasks <= 0 || G <= 0) return;
  if (ntasks % 2) throw Error(1, "M2P half tasks come in pairs");
  const int npairs = ntasks / 2;
  switch (P) {
#define PBT_MM(Q) \
  case Q: m2p_multi_p<T, Q>(tasks, npairs, blist, tgt, bcen, mom, boxoff, mslot, G, kappa, partial, s); break;
    PBT_MM(0) PBT_MM(1) PBT_MM(2) PBT_MM(3) PBT_MM(4) PBT_MM(5) PBT_MM(6) PBT_MM(7) PBT_MM(8)
#undef PBT_MM
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template <typename T, int P>
static void m2p_p2p_p(const Task* m2p, int nm2p, const int32_t* blist, const double* bcen, const T* mom,
                      const Task* p2p, int np2p, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                      bool guard, T* ppartial, hipStream_t s) {
  const int blocks = ((nm2p + np2p + 3) / 4 + 7) / 8 * 8;
#define PBT_LAUNCH(G, SF)                                                                                  \
  k_m2p_p2p<T, P, G, SF><<<blocks, 256, 0, s>>>(m2p, nm2p, blist, bcen, mom, p2p, np2p, ranges, src, tgt, kappa, \
                                                ppartial)
  const bool sf = kappa == T(0);
  if (guard) {
    if (sf) PBT_LAUNCH(true, true);
    else PBT_LAUNCH(true, false);
  } else {
    if (sf) PBT_LAUNCH(false, true);
    else PBT_LAUNCH(false, false);
  }
#undef PBT_LAUNCH
}

template <typename T>
void launch_m2p_p2p(int P, const Task* m2p, int nm2p, const int32_t* blist, const double* bcen, const T* mom,
                    const Task* p2p, int np2p, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                    bool guard, T* ppartial, hipStream_t s) {
  if (nm2p % 2) throw Error(1, "M2P half tasks come in pairs");
  nm2p /= 2;   // wavefronts
  if (nm2p + np2p <= 0) return;
  switch (P) {
#define PBT_CASE(PP)                                                                                      \
  case PP:                                                                                                \
    m2p_p2p_p<T, PP>(m2p, nm2p, blist, bcen, mom, p2p, np2p, ranges, src, tgt, kappa, guard, ppartial, s);   \
    break;
    PBT_CASE(0) PBT_CASE(1) PBT_CASE(2) PBT_CASE(3) PBT_CASE(4) PBT_CASE(5) PBT_CASE(6) PBT_CASE(7) PBT_CASE(8)
#undef PBT_CASE
    default: throw Error(1, "Taylor order P must be 0..8");
  }
  PBT_HIP(hipGetLastError());
}

template void launch_p2p_moments<float>(int, int, const int32_t*, const MomChunk*, int, const MomChunk*,
                                        const double*, const double*, float*, float*, const Task*, int,
                                        const int32_t*, const float*, const float*, float, bool, float*, hipStream_t);
template void launch_p2p_moments<double>(int, int, const int32_t*, const MomChunk*, int, const MomChunk*,
                                         const double*, const double*, double*, double*, const Task*, int,
                                         const int32_t*, const double*, const double*, double, bool, double*,
                                         hipStream_t);
template void launch_moments<float>(int, int, const int32_t*, const MomChunk*, int, const MomChunk*, const double*,
                                    const double*, const float*, float*, float*, hipStream_t);
template void launch_moments<double>(int, int, const int32_t*, const MomChunk*, int, const MomChunk*,
                                     const double*, const double*, const double*, double*, double*, hipStream_t);
template void launch_m2p_p2p<float>(int, const Task*, int, const int32_t*, const double*, const float*,
                                    const Task*, int, const int32_t*, const float*, const float*, float, bool,
                                    float*, hipStream_t);
template void launch_m2p_p2p<double>(int, const Task*, int, const int32_t*, const double*, const double*,
                                     const Task*, int, const int32_t*, const double*, const double*, double, bool,
                                     double*, hipStream_t);
template void launch_m2m<float>(int, int, const int32_t*, int, int, const int32_t*, const double*, float*, float*,
                                hipStream_t);
template void launch_m2m<double>(int, int, const int32_t*, int, int, const int32_t*, const double*, double*, double*,
                                 hipStream_t);
template void launch_m2p_multi<float>(int, const Task*, int, const int32_t*, const float*, const double*,
                                      const float*, const int32_t*, const int32_t*, int, float, float*, hipStream_t);
template void launch_m2p_multi<double>(int, const Task*, int, const int32_t*, const double*, const double*,
                                       const double*, const int32_t*, const int32_t*, int, double, double*,
                                       hipStream_t);
template void launch_m2p<float>(int, const Task*, int, const int32_t*, const float*, const double*,
                                const float*, float, float*, hipStream_t);
template void launch_m2p<double>(int, const Task*, int, const int32_t*, const double*, const double*,
                                 const double*, double, double*, hipStream_t);

}  // namespace pbt
