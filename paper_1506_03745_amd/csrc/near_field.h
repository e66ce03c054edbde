// Device code shared by the near-field (P2P) kernels: source records staged
// in per-wavefront LDS tiles and the pairwise interaction of Section 3.2.
// Included inside namespace pbt { namespace { ... } } of a kernel file.
#pragma once

template <typename T>
struct KMath;
template <>
struct KMath<float> {
  static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
  // exp(-kappa r) = 2^(r * c) with c = -kappa log2(e)
  static __device__ __forceinline__ float expk(float r, float c) { return __builtin_amdgcn_exp2f(r * c); }
  static __host__ __device__ float expk_const(float kappa) { return -kappa * 1.4426950408889634f; }
};
template <>
struct KMath<double> {
  static __device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
  static __device__ __forceinline__ double expk(double r, double c) { return exp(r * c); }
  static __host__ __device__ double expk_const(double kappa) { return -kappa; }
};

// Map the hardware block index to a logical one so that consecutive logical
// blocks (tasks that share source ranges) land on the same XCD, whose L2
// then serves their common sources.  Workgroups are dispatched round-robin
// over the 8 XCDs; gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// One source record (x y z s Dx Dy Dz s_L), aligned so that LDS reads of a
// record are full-width.
template <typename T>
struct alignas(8 * sizeof(T)) SrcRec {
  T v[8];
};

// A record read back from LDS in 16-byte pieces (two for FP32, four for
// FP64), whatever the compiler knows about the base pointer's alignment.
typedef float pbt_f4 __attribute__((ext_vector_type(4)));
typedef double pbt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ SrcRec<float> load_rec(const SrcRec<float>* p) {
  const pbt_f4* q = reinterpret_cast<const pbt_f4*>(p);
  const pbt_f4 a = q[0], b = q[1];
  SrcRec<float> r;
  r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
  r.v[4] = b.x; r.v[5] = b.y; r.v[6] = b.z; r.v[7] = b.w;
  return r;
}
__device__ __forceinline__ SrcRec<double> load_rec(const SrcRec<double>* p) {
  const pbt_d2* q = reinterpret_cast<const pbt_d2*>(p);
  SrcRec<double> r;
  for (int k = 0; k < 4; ++k) {
    const pbt_d2 a = q[k];
    r.v[2 * k] = a.x;
    r.v[2 * k + 1] = a.y;
  }
  return r;
}

// Wave-scope ordering of LDS writes and reads between the lanes of one
// wavefront (no workgroup barrier: the waves of a block run independent
// tasks with different trip counts).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Interaction of one target with one source record (eqs. bem_interior and
// bem_exterior, discrete forms): l accumulates s_L/r - D.(x-y)/r^3, yy
// accumulates s e^{-kappa r}/r + D.grad_y(e^{-kappa r}/r)
//   = e^{-kappa r} (s/r + D.(x-y) (1 + kappa r)/r^3).
// With a = D.(x-y)/r the double-layer factors are a (1/r + kappa) for the
// Yukawa row and a/r for the Laplace row (r^2 (1/r)^2 = 1 taken exactly),
// one multiplication fewer than forming D.(x-y)/r^2 and 1 + kappa r.
// KIND bit 0: also the Laplace row (target and source on one molecule);
// bit 1: kappa = 0 (salt-free solvent), where the solvent row is the Laplace
// kernel too and the exponential drops out.
template <typename T, bool GUARD, int KIND>
__device__ __forceinline__ void p2p_pair(const SrcRec<T>& s, T tx, T ty, T tz, T kappa, T ck, T& l, T& yy) {
  constexpr bool FUSED = KIND & 1, SALTFREE = KIND & 2;
  const T dx = tx - s.v[0], dy = ty - s.v[1], dz = tz - s.v[2];
  const T r2 = dx * dx + dy * dy + dz * dz;
  T rinv = KMath<T>::rsq(r2);
  if (GUARD) rinv = r2 > T(0) ? rinv : T(0);
  const T dd = s.v[4] * dx + s.v[5] * dy + s.v[6] * dz;
  const T a = dd * rinv;                           // D.(x-y)/r
  if (SALTFREE) {
    const T t = a * rinv;                          // D.(x-y)/r^2
    if (FUSED) l += (s.v[7] - t) * rinv;
    yy += (t + s.v[3]) * rinv;
    return;
  }
  if (FUSED) l += (s.v[7] - a * rinv) * rinv;      // s_L/r - D.(x-y)/r^3
  const T rr = r2 * rinv;
  const T gy = KMath<T>::expk(rr, ck) * rinv;
  yy += gy * (a * (rinv + kappa) + s.v[3]);        // s G_Y + D.grad_y G_Y
}

// The records j = grp, grp + F, ... of a 32-record tile (F lane groups per
// half-wavefront share its targets).
template <typename T, bool GUARD, int KIND, int F>
__device__ __forceinline__ void p2p_tile(const SrcRec<T>* tile, int grp, T tx, T ty, T tz, T kappa, T ck, T& l,
                                         T& yy) {
  if (F == 1) {
    // the shape that keeps the fewest records in flight for the compiler:
    // eight FP32 (two FP64) records per unrolled step
    constexpr int UF = sizeof(T) == 4 ? 8 : 2;
    int j = 0;
    for (; j + UF <= 32; j += UF) {
#pragma unroll
      for (int q = 0; q < UF; ++q) p2p_pair<T, GUARD, KIND>(load_rec(tile + j + q), tx, ty, tz, kappa, ck, l, yy);
    }
    return;
  }
  constexpr int N = 32 / F;
  constexpr int U0 = sizeof(T) == 4 ? 8 : 4;
  constexpr int U = N < U0 ? N : U0;
  const SrcRec<T>* t0 = tile + grp;
  for (int q0 = 0; q0 < N; q0 += U) {
#pragma unroll
    for (int q = 0; q < U; ++q) p2p_pair<T, GUARD, KIND>(load_rec(t0 + F * (q0 + q)), tx, ty, tz, kappa, ck, l, yy);
  }
}

// A pair of P2P tasks on one wavefront: lanes 0..31 serve tasks[0], lanes
// 32..63 tasks[1] (each up to 32 targets with its own source ranges; both
// have the same `fused` and the same split F).  Each round, each half stages
// its next 32 source records into its half of the wave's LDS tile with one
// coalesced load per lane, padding with zero-strength records far away (they
// add exactly zero); the half's lanes form F groups of 32/F, each group
// holding the half's targets (one per lane) and reading every F-th record of
// the tile (LDS broadcasts), so a half with few targets keeps its lanes busy
// and needs 1/F of the time per round.  The groups' sums are added by a
// fixed butterfly.  Partials [slot][32][2].
template <typename T, bool GUARD, int KIND, int F>
__device__ __forceinline__ void p2p_task_pair_f(const Task* __restrict__ tp, SrcRec<T>* tile,
                                                const int32_t* __restrict__ ranges, const T* __restrict__ tgt,
                                                const T* __restrict__ src, T kappa, T* __restrict__ partial) {
  constexpr int TW = 32 / F;   // targets per half
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const int grp = hl / TW, tl = hl - grp * TW;
  const SrcRec<T>* srec = reinterpret_cast<const SrcRec<T>*>(src);
  const Task t = tp[half];
  const int rounds = (max(tp[0].nsrc, tp[1].nsrc) + 31) >> 5;
  const int ti = t.tbeg + (tl < t.tcount ? tl : 0);
  const T tx = tgt[kTgtStride * ti], ty = tgt[kTgtStride * ti + 1], tz = tgt[kTgtStride * ti + 2];
  const T ck = KMath<T>::expk_const(kappa);
  SrcRec<T> pad;
  for (int d = 0; d < 8; ++d) pad.v[d] = d < 3 ? T(1e18) : T(0);
  SrcRec<T>* mine = tile + 32 * half;
  T l = 0, yy = 0;
  int r = t.lbeg;
  int cur = r < t.lend ? ranges[2 * r] : 0;
  for (int round = 0; round < rounds; ++round) {
    // fill: up to 32 records of this half's remaining ranges, in order
    int cnt = 0;
    while (r < t.lend && cnt < 32) {
      const int end = ranges[2 * r + 1];
      const int take = min(end - cur, 32 - cnt);
      if (hl >= cnt && hl < cnt + take) mine[hl] = srec[cur + (hl - cnt)];
      cnt += take;
      cur += take;
      if (cur == end && ++r < t.lend) cur = ranges[2 * r];
    }
    if (hl >= cnt) mine[hl] = pad;
    wave_lds_sync();
    p2p_tile<T, GUARD, KIND, F>(mine, grp, tx, ty, tz, kappa, ck, l, yy);
    wave_lds_sync();
  }
  if (F >= 4) {
    l += __shfl_xor(l, 8, 32);
    yy += __shfl_xor(yy, 8, 32);
  }
  if (F >= 2) {
    l += __shfl_xor(l, 16, 32);
    yy += __shfl_xor(yy, 16, 32);
  }
  if (grp == 0 && tl < t.tcount) {
    T o0 = l, o1 = yy;
    if (t.form & kFormDropOut) o1 = T(0);
    if (t.form & kFormSwap) {
      const T sw = o0;
      o0 = o1;
      o1 = sw;
    }
    partial[2 * ((int64_t)t.slot * 32 + tl) + 0] = o0;
    partial[2 * ((int64_t)t.slot * 32 + tl) + 1] = o1;
  }
}

template <typename T, bool GUARD, int KIND>
__device__ __forceinline__ void p2p_task_pair_k(int split, const Task* __restrict__ tp, SrcRec<T>* tile,
                                                const int32_t* __restrict__ ranges, const T* __restrict__ tgt,
                                                const T* __restrict__ src, T kappa, T* __restrict__ partial) {
  if (split == 4) p2p_task_pair_f<T, GUARD, KIND, 4>(tp, tile, ranges, tgt, src, kappa, partial);
  else if (split == 2) p2p_task_pair_f<T, GUARD, KIND, 2>(tp, tile, ranges, tgt, src, kappa, partial);
  else p2p_task_pair_f<T, GUARD, KIND, 1>(tp, tile, ranges, tgt, src, kappa, partial);
}

template <typename T, bool GUARD>
__device__ __forceinline__ void p2p_task_pair(const Task* __restrict__ tp, SrcRec<T>* tile,
                                              const int32_t* __restrict__ ranges, const T* __restrict__ tgt,
                                              const T* __restrict__ src, T kappa, T* __restrict__ partial) {
  // both halves agree on fused, split and kFormKz (an outside sum inside a
  // salt-free layer takes kappa = 0)
  if (tp[0].form & kFormKz) kappa = T(0);
  const int kind = (tp[0].fused ? 1 : 0) | (kappa == T(0) ? 2 : 0), split = tp[0].split;
  switch (kind) {
    case 0: p2p_task_pair_k<T, GUARD, 0>(split, tp, tile, ranges, tgt, src, kappa, partial); break;
    case 1: p2p_task_pair_k<T, GUARD, 1>(split, tp, tile, ranges, tgt, src, kappa, partial); break;
    case 2: p2p_task_pair_k<T, GUARD, 2>(split, tp, tile, ranges, tgt, src, kappa, partial); break;
    default: p2p_task_pair_k<T, GUARD, 3>(split, tp, tile, ranges, tgt, src, kappa, partial); break;
  }
}
