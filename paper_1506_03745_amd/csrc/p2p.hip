// Near-field (P2P) kernel of the operator (Section 3.2): Gauss points as
// sources, collocation points as targets, direct sums over the source ranges
// of each target leaf's near list.  The pair interaction and the task layout
// are in near_field.h; this file only launches them, so that its profile
// stays tied to these two files.
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

}  // namespace

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
}  // namespace pbt
