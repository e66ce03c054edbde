// Near-field (P2P) kernels of the operator (Section 3.2): Gauss points as
// sources, collocation points as targets, direct sums over the source ranges
// of each target group's near list.  The pair interaction and the task
// layout of the per-group kernel are in near_field.h (shared with the joint
// launches in taylor.hip); this file launches it and holds the kernel for the
// pairs between surfaces that every group of a batch holds unmoved.
#include "pbt_internal.h"

namespace pbt {

namespace {

#include "near_field.h"

// One wavefront per pair of P2P tasks (four per block).
template <typename T, bool GUARD>
__global__ __launch_bounds__(256) void k_p2p(const Task* __restrict__ tasks, int npairs,
                                             const int32_t* __restrict__ ranges,
                                             const T* __restrict__ tgt, const T* __restrict__ src,
                                             T kappa, T* __restrict__ partial) {
  __shared__ SrcRec<T> tiles[4][64];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= npairs) return;
  p2p_task_pair<T, GUARD>(tasks + 2 * wv, tiles[threadIdx.x >> 6], ranges, tgt, src, kappa, partial);
}

// ---- P2P between surfaces shared by every group of a batch ------------------
// The geometry of a pair (target on one shared surface, Gauss point on
// another) is the same in every group; only the source strengths differ.
// With n the source panel's unit normal and d = D . n its double-layer
// density (D = d n in the record), the solvent row's pair term is
//   e^{-kappa r}/r (s + d q),   q = n.(x - y)/r (1/r + kappa)
// (salt-free: 1/r (s + d q) with q = n.(x - y)/r^2), the same sum as
// p2p_pair's outside row.  Per pair the kernel forms g = e^{-kappa r}/r
// and q once and applies them to NB groups' (s, d), staged in LDS.
// (s, d) of the groups in LDS as 16-byte chunks, eight a source: FP32 two
// groups a chunk (16 groups a pass), FP64 one (8 groups a pass).
template <typename T>
struct MultiChunk;
template <>
struct MultiChunk<float> {
  typedef pbt_f4 type;
  static constexpr int per = 2;
};
template <>
struct MultiChunk<double> {
  typedef pbt_d2 type;
  static constexpr int per = 1;
};

// s and D (entries 3..6) of a source record.
typedef float pbt_f4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ void load_sD(const float* r, float o[4]) {
  const pbt_f4u a = *reinterpret_cast<const pbt_f4u*>(r + 3);
  o[0] = a.x;
  o[1] = a.y;
  o[2] = a.z;
  o[3] = a.w;
}
__device__ __forceinline__ void load_sD(const double* r, double o[4]) {
  const pbt_d2 a = *reinterpret_cast<const pbt_d2*>(r + 2), b = *reinterpret_cast<const pbt_d2*>(r + 4);
  o[0] = a.y;
  o[1] = b.x;
  o[2] = b.y;
  o[3] = r[6];
}

// A pair of shared-surface tasks on one wavefront (lanes 0..31: tp[0],
// 32..63: tp[1], one target a lane, both non-fused, both serving groups
// split .. split + kMultiBlock - 1).  For each pass over NB of those
// groups, each half walks its source ranges in rounds of 32 records: lane
// hl stages the geometry of the round's hl-th source (position and normal)
// and its (s, d) in each of the pass's groups; every lane then adds the 32
// sources' terms for its target into NB sums.  Pad entries are far away with
// zero strengths (they add exactly zero).  Source q's chunk c is stored at
// position c ^ (q & 7) of its row (writes by 32 lanes at a 128-byte stride
// spread over the banks; reads are broadcasts with a compile-time position).
template <typename T, bool GUARD, bool SALTFREE>
__device__ __forceinline__ void p2p_multi_pair(const Task* __restrict__ tp, SrcRec<T>* geo,
                                               typename MultiChunk<T>::type* sd,
                                               const int32_t* __restrict__ ranges, const T* __restrict__ tgt,
                                               const T* __restrict__ src, const double* __restrict__ nrm, int K,
                                               const int32_t* __restrict__ goff, const int32_t* __restrict__ mslot,
                                               int G, T kappa, T* __restrict__ partial) {
  typedef typename MultiChunk<T>::type C;
  constexpr int PER = MultiChunk<T>::per, NB = 8 * PER;
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const Task t = tp[half];
  const int rounds = (max(tp[0].nsrc, tp[1].nsrc) + 31) >> 5;
  const int ti = t.tbeg + (hl < t.tcount ? hl : 0);
  const T tx = tgt[kTgtStride * ti], ty = tgt[kTgtStride * ti + 1], tz = tgt[kTgtStride * ti + 2];
  const T ck = KMath<T>::expk_const(kappa);
  SrcRec<T>* mine = geo + 32 * half;
  C* mc = sd + half * (32 * 8);
  // this task's block of groups (the same for both halves)
  const int g0 = tp[0].split, g1 = min(G, g0 + kMultiBlock);
  for (int gb = g0; gb < g1; gb += NB) {
    const int nb = min(NB, g1 - gb);
    T acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = T(0);
    int r = t.lbeg;
    int cur = r < t.lend ? ranges[2 * r] : 0;
    for (int round = 0; round < rounds; ++round) {
      // the source this lane stages this round (-1: a pad entry)
      int j = -1, cnt = 0;
      while (r < t.lend && cnt < 32) {
        const int end = ranges[2 * r + 1];
        const int take = min(end - cur, 32 - cnt);
        if (hl >= cnt && hl < cnt + take) j = cur + (hl - cnt);
        cnt += take;
        cur += take;
        if (cur == end && ++r < t.lend) cur = ranges[2 * r];
      }
      SrcRec<T> g;
#pragma unroll
      for (int d = 0; d < 8; ++d) g.v[d] = T(0);
      if (j >= 0) {
        const T* s0 = src + (int64_t)kSrcStride * j;
        const double* n = nrm + 3 * (int64_t)(j / K);
        g.v[0] = s0[0];
        g.v[1] = s0[1];
        g.v[2] = s0[2];
        g.v[4] = (T)n[0];
        g.v[5] = (T)n[1];
        g.v[6] = (T)n[2];
      } else {
        g.v[0] = g.v[1] = g.v[2] = T(1e18);
      }
      mine[hl] = g;
      // every lane loads all NB records (a pad entry or a group past the
      // last reads a valid record and discards it), so that the loads are
      // in flight together
      T sv[NB], dv[NB];
      const int64_t js = j >= 0 ? j : 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int gc = min(gb + b, g1 - 1);
        T sD[4];
        load_sD(src + (int64_t)kSrcStride * (js + (int64_t)goff[gc] * K), sD);
        const bool ok = j >= 0 && b < nb;
        sv[b] = ok ? sD[0] : T(0);
        dv[b] = ok ? sD[1] * g.v[4] + sD[2] * g.v[5] + sD[3] * g.v[6] : T(0);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        C v;
        if constexpr (PER == 2) {
          v.x = sv[2 * c];
          v.y = dv[2 * c];
          v.z = sv[2 * c + 1];
          v.w = dv[2 * c + 1];
        } else {
          v.x = sv[c];
          v.y = dv[c];
        }
        mc[hl * 8 + (c ^ (hl & 7))] = v;
      }
      wave_lds_sync();
      for (int q0 = 0; q0 < 32; q0 += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = q0 + k;
          const SrcRec<T> s = load_rec(mine + q);
          const T dx = tx - s.v[0], dy = ty - s.v[1], dz = tz - s.v[2];
          const T r2 = dx * dx + dy * dy + dz * dz;
          T rinv = KMath<T>::rsq(r2);
          if (GUARD) rinv = r2 > T(0) ? rinv : T(0);
          const T nd = (s.v[4] * dx + s.v[5] * dy + s.v[6] * dz) * rinv;
          T gk, qk;
          if (SALTFREE) {
            gk = rinv;
            qk = nd * rinv;
          } else {
            gk = KMath<T>::expk(r2 * rinv, ck) * rinv;
            qk = nd * (rinv + kappa);
          }
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const C v = mc[q * 8 + (c ^ k)];
            if constexpr (PER == 2) {
              acc[2 * c] += gk * (v.x + v.y * qk);
              acc[2 * c + 1] += gk * (v.z + v.w * qk);
            } else {
              acc[c] += gk * (v.x + v.y * qk);
            }
          }
        }
      }
      wave_lds_sync();
    }
    if (hl < t.tcount) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
        T o0 = T(0), o1 = acc[b];
        if (t.form & kFormDropOut) o1 = T(0);
        if (t.form & kFormSwap) {
          const T sw = o0;
          o0 = o1;
          o1 = sw;
        }
        const int64_t slot = mslot[(int64_t)t.slot * G + gb + b];
        partial[2 * (slot * 32 + hl) + 0] = o0;
        partial[2 * (slot * 32 + hl) + 1] = o1;
      }
    }
  }
}

// One wavefront per pair of shared-surface tasks (four per block).
template <typename T, bool GUARD, bool SALTFREE>
__global__ __launch_bounds__(256) void k_p2p_multi(const Task* __restrict__ tasks, int npairs,
                                                   const int32_t* __restrict__ ranges, const T* __restrict__ tgt,
                                                   const T* __restrict__ src, const double* __restrict__ nrm, int K,
                                                   const int32_t* __restrict__ goff,
                                                   const int32_t* __restrict__ mslot, int G, T kappa,
                                                   T* __restrict__ partial) {
  __shared__ SrcRec<T> geo[4][64];
  __shared__ typename MultiChunk<T>::type sd[4][2 * 32 * 8];
  const int wv = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (wv >= npairs) return;
  const int w = threadIdx.x >> 6;
  p2p_multi_pair<T, GUARD, SALTFREE>(tasks + 2 * wv, geo[w], sd[w], ranges, tgt, src, nrm, K, goff, mslot, G, kappa,
                                     partial);
}

}  // namespace

template <typename T>
void launch_p2p_multi(const Task* tasks, int npairs, const int32_t* ranges, const T* tgt, const T* src,
                      const double* nrm, int K, const int32_t* goff, const int32_t* mslot, int G, T kappa,
                      bool guard, T* partial, hipStream_t s) {
  if (npairs <= 0 || G <= 0) return;
  const int blocks = ((npairs + 3) / 4 + 7) / 8 * 8;
  const bool sf = kappa == T(0);
#define PBT_MULTI(GD, SF)                                                                                   \
  k_p2p_multi<T, GD, SF><<<blocks, 256, 0, s>>>(tasks, npairs, ranges, tgt, src, nrm, K, goff, mslot, G, kappa, \
                                                 partial)
  if (guard) {
    if (sf) PBT_MULTI(true, true);
    else PBT_MULTI(true, false);
  } else {
    if (sf) PBT_MULTI(false, true);
    else PBT_MULTI(false, false);
  }
#undef PBT_MULTI
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_p2p(const Task* tasks, int npairs, const int32_t* ranges, const T* tgt, const T* src,
                T kappa, bool guard, T* partial, hipStream_t s) {
  if (npairs <= 0) return;
  const int blocks = ((npairs + 3) / 4 + 7) / 8 * 8;
  if (guard)
    k_p2p<T, true><<<blocks, 256, 0, s>>>(tasks, npairs, ranges, tgt, src, kappa, partial);
  else
    k_p2p<T, false><<<blocks, 256, 0, s>>>(tasks, npairs, ranges, tgt, src, kappa, partial);
  PBT_HIP(hipGetLastError());
}

template void launch_p2p<float>(const Task*, int, const int32_t*, const float*, const float*, float,
                                bool, float*, hipStream_t);
template void launch_p2p<double>(const Task*, int, const int32_t*, const double*, const double*,
                                 double, bool, double*, hipStream_t);
template void launch_p2p_multi<float>(const Task*, int, const int32_t*, const float*, const float*,
                                      const double*, int, const int32_t*, const int32_t*, int, float, bool, float*,
                                      hipStream_t);
template void launch_p2p_multi<double>(const Task*, int, const int32_t*, const double*, const double*,
                                       const double*, int, const int32_t*, const int32_t*, int, double, bool,
                                       double*, hipStream_t);
}  // namespace pbt
