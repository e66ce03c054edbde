// Per-product kernels of the boundary-element operator (Sections 3.1-3.2).
//
// The product treats Gauss points as sources and collocation points as
// targets (Section 3.2, the N-body analogy).  Each source carries a
// single-layer strength s = w A sigma and a double-layer moment
// D = w A mu n, where sigma and mu are the panel densities of the solvent
// (Yukawa) row:
//   molecule   sigma = (eps_s/eps_out) dphi/dn,  mu = -phi
//   charged    sigma = 0 (known part moved to the rhs),  mu = -phi
//   potential  sigma = dphi/dn,  mu = 0 (known phi0 moved to the rhs)
// With G_L = 1/(4 pi r) and G_Y = exp(-kappa r)/(4 pi r) a target x receives
//   Y(x) = sum s G_Y + D.(x-y) (1 + kappa r) exp(-kappa r) / (4 pi r^3)
// and, from sources on its own molecule, the interior row
//   L(x) = -(eps_out/eps_s) sum s G_L - sum D.(x-y) / (4 pi r^3),
// which is K_L phi - V_L dphi/dn of eq. integral_eq.
#include <algorithm>

#include "pbt_internal.h"

namespace pbt {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_densities(int64_t np, PanelMaps m, const double* __restrict__ x, double* sig,
                            double* mu) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int32_t cphi = m.col_phi[p], cpsi = m.col_psi[p];
  sig[p] = cpsi >= 0 ? m.dens_scale[p] * x[cpsi] : 0.0;
  mu[p] = cphi >= 0 ? -x[cphi] : 0.0;
}

__global__ void k_known_densities(int64_t np, const double* __restrict__ ks,
                                  const double* __restrict__ km, double* sig, double* mu) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  sig[p] = ks[p];
  mu[p] = km[p];
}

// Solvent rows of the right-hand side: b = -(A k) - half, with A k the
// operator applied to the known densities and half the imposed potential's
// 1/2 jump (zero except on potential surfaces).
__global__ void k_rhs_solvent(int64_t np, const int32_t* __restrict__ row_sol, const double* __restrict__ ak,
                              const double* __restrict__ half, double* b) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int32_t r = row_sol[p];
  b[r] = -ak[r] - half[p];
}

// Source record: (x, y, z, s, Dx, Dy, Dz, s_L) with s_L = -(eps_out/eps_s) s,
// the single-layer strength of the interior (Laplace) row; rlap[p] holds
// -(eps_out/eps_s) for molecule panels and 0 otherwise.
template <typename T>
__global__ void k_strengths(int64_t ns, int K, const double* __restrict__ sig,
                            const double* __restrict__ mu, const double* __restrict__ wa,
                            const double* __restrict__ nrm, const double* __restrict__ rlap, T* src) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const int64_t p = j / K;
  const double w = wa[j];
  const double m = w * mu[p];
  const double sv = w * sig[p];
  T* o = src + kSrcStride * j;
  o[3] = (T)sv;
  o[4] = (T)(m * nrm[3 * p]);
  o[5] = (T)(m * nrm[3 * p + 1]);
  o[6] = (T)(m * nrm[3 * p + 2]);
  o[7] = (T)(rlap[p] * sv);
}

// Same, with the panel densities read straight from the unknowns (and also
// stored for the near-field combine by the first Gauss point of each panel).
template <typename T>
__global__ void k_strengths_x(int64_t ns, int K, PanelMaps m, const double* __restrict__ x,
                              const double* __restrict__ wa, const double* __restrict__ nrm,
                              const double* __restrict__ rlap, double* sig, double* mu, T* src) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const int64_t p = j / K;
  const int32_t cphi = m.col_phi[p], cpsi = m.col_psi[p];
  const double sg = cpsi >= 0 ? m.dens_scale[p] * x[cpsi] : 0.0;
  const double mv = cphi >= 0 ? -x[cphi] : 0.0;
  if (j == p * K) {
    sig[p] = sg;
    mu[p] = mv;
  }
  const double w = wa[j];
  const double mm = w * mv;
  const double sv = w * sg;
  T* o = src + kSrcStride * j;
  o[3] = (T)sv;
  o[4] = (T)(mm * nrm[3 * p]);
  o[5] = (T)(mm * nrm[3 * p + 1]);
  o[6] = (T)(mm * nrm[3 * p + 2]);
  o[7] = (T)(rlap[p] * sv);
}

// Sum the partial slots of every target, scale by 1/(4 pi), add the near and
// self corrections (sparse, FP64) and the 1/2 jump terms, and scatter into
// the unknown layout; optionally also the chunk's share of the first
// Gram-Schmidt pass over the result (CombineArgs::ndots).  One block per target chunk: lane = target within the
// chunk (coalesced slot reads), the kCombineWaves waves split the chunk's
// slots and each target's near entries, and add up through LDS.
constexpr int kCombineWaves = 16;
template <typename T>
__global__ __launch_bounds__(64 * kCombineWaves) void k_combine(CombineArgs a, const T* __restrict__ partial,
                                                              const T* __restrict__ ppartial, double* y) {
  __shared__ double red[kCombineWaves][4][64];
  const ChunkSlots cs = a.chunks[blockIdx.x];
  // the wave index is uniform: held in a scalar register, so the slot and
  // row addresses below are scalar bases plus the lane's offset
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool act = lane < cs.tcount;
  const int64_t i = cs.tbeg + lane;
  // the output rows and jump terms are read up front (wave 0 writes), so
  // their latency overlaps the sums instead of following them
  int32_t ri = -1, rs = 0;
  double xj = 0.0;
  if (act) {
    ri = a.maps.row_int[i];
    rs = a.maps.row_sol[i];
    if (w == 0) {
      const int32_t cphi = a.maps.col_phi[i];
      if (a.add_jump && cphi >= 0) xj = 0.5 * a.x[cphi];
    }
  }
  // the basis entries of this wave's first two Gram-Schmidt rows (below),
  // also loaded up front
  double vp[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  if (act) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = w + t * kCombineWaves;
      if (k < a.ndots) {
        const double* Vk = a.V + (int64_t)k * a.ldv;
        if (ri >= 0) vp[t][0] = Vk[ri];
        vp[t][1] = Vk[rs];
      }
    }
  }
  double l = 0.0, yy = 0.0, nl = 0.0, ny = 0.0;
  if (act) {
#pragma unroll 4
    for (int s = cs.sbeg + w; s < cs.send; s += kCombineWaves) {
      l += (double)partial[2 * ((int64_t)s * 64 + lane) + 0];
      yy += (double)partial[2 * ((int64_t)s * 64 + lane) + 1];
    }
    const int hl = lane & 31;
    const int pb = lane < 32 ? cs.hbeg0 : cs.hbeg1, pe = lane < 32 ? cs.hend0 : cs.hend1;
#pragma unroll 4
    for (int s = pb + w; s < pe; s += kCombineWaves) {
      l += (double)ppartial[2 * ((int64_t)s * 32 + hl) + 0];
      yy += (double)ppartial[2 * ((int64_t)s * 32 + hl) + 1];
    }
#pragma unroll 2
    for (int64_t e = a.near_ptr[i] + w; e < a.near_ptr[i + 1]; e += kCombineWaves) {
      const int32_t j = a.near_col[e];
      const double sj = a.sig[j], mj = a.mu[j];
      if (sizeof(T) == 4) {
        // FP32 interactions: the corrections in FP32 too (one 16-byte load)
        const float4 v = reinterpret_cast<const float4*>(a.near_val32)[e];
        nl += (double)v.x * sj + (double)v.y * mj;
        ny += (double)v.z * sj + (double)v.w * mj;
      } else {
        const double* v = a.near_val + 4 * e;
        nl += v[0] * sj + v[1] * mj;
        ny += v[2] * sj + v[3] * mj;
      }
    }
  }
  red[w][0][lane] = l;
  red[w][1][lane] = yy;
  red[w][2][lane] = nl;
  red[w][3][lane] = ny;
  __syncthreads();
  // wave q < 4 adds up sum q over the waves (in wave order) into red[0][q]
  if (w < 4) {
    double t = 0.0;
    for (int k = 0; k < kCombineWaves; ++k) t += red[k][w][lane];
    red[0][w][lane] = t;
  }
  __syncthreads();
  __shared__ double yv[2][64];
  if (w == 0) {
    double yi = 0.0, ys = 0.0;
    if (act) {
      l = red[0][0][lane];
      yy = red[0][1][lane];
      nl = red[0][2][lane];
      ny = red[0][3][lane];
      yi = xj + (l * kInv4Pi + nl);
      ys = xj + (yy * kInv4Pi + ny);
      if (ri >= 0) y[ri] = yi;
      else yi = 0.0;
      y[rs] = ys;
    }
    yv[0][lane] = yi;
    yv[1][lane] = ys;
  }
  if (a.ndots <= 0) return;
  // first Gram-Schmidt pass: this chunk's rows of V_i . y, a wave per i
  // (and y . y as row ndots when asked for)
  __syncthreads();
  const int nd = a.ndots + (a.self_dot ? 1 : 0);
  for (int k = w, t = 0; k < nd; k += kCombineWaves, ++t) {
    double pr = 0.0;
    if (act && k == a.ndots) {
      pr = yv[0][lane] * yv[0][lane] + yv[1][lane] * yv[1][lane];
    } else if (act) {
      const double* Vk = a.V + (int64_t)k * a.ldv;
      const double v0 = t == 0 ? vp[0][0] : t == 1 ? vp[1][0] : (ri >= 0 ? Vk[ri] : 0.0);
      const double v1 = t == 0 ? vp[0][1] : t == 1 ? vp[1][1] : Vk[rs];
      if (ri >= 0) pr = v0 * yv[0][lane];
      pr += v1 * yv[1][lane];
    }
    for (int o = 32; o > 0; o >>= 1) pr += __shfl_down(pr, o, 64);
    if (lane == 0) a.dpart[((int64_t)cs.grp * a.R + k) * a.nbh + cs.lchunk] = pr;
  }
}

// Reaction potential at the charges of one molecule (eq. phi_reac_bem):
// phi_reac = -K_L(phi) + V_L(dphi/dn) = -L with the interior-row sums L,
// direct FP64 sums over the molecule's Gauss points plus the near
// corrections of each charge.  One block per charge, threads over sources.
__global__ void k_to_f32(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// The reaction potential's far part in tiles: a wavefront holds 64 charges
// (one per lane) and runs over one segment of the molecule's sources, read
// with wave-uniform loads; part[seg nq + k] = -rho_inv sum s/r - sum D.(x-y)/r^3
// over the segment.  k_reac_sum adds the segments in order, the near
// corrections and the sign.
__global__ __launch_bounds__(64) void k_reac_part(int64_t nq, const double* __restrict__ qxyz, int64_t s0,
                                                  int64_t s1, int nseg, const double* __restrict__ src,
                                                  double rho_inv, double* __restrict__ part) {
  const int64_t k = blockIdx.x * (int64_t)64 + threadIdx.x;
  const int seg = blockIdx.y;
  const int64_t len = (s1 - s0 + nseg - 1) / nseg;
  const int64_t j0 = s0 + seg * len, j1 = min(s1, j0 + len);
  const int64_t kk = k < nq ? k : nq - 1;
  const double x = qxyz[3 * kk], y = qxyz[3 * kk + 1], z = qxyz[3 * kk + 2];
  double a1 = 0.0, a2 = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const double* s = src + (int64_t)kSrcStride * j;
    const double dx = x - s[0], dy = y - s[1], dz = z - s[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double dd = s[4] * dx + s[5] * dy + s[6] * dz;
    a1 += s[3] * rinv;
    a2 += dd * rinv * rinv * rinv;
  }
  if (k < nq) part[(int64_t)seg * nq + k] = -rho_inv * a1 - a2;
}

__global__ __launch_bounds__(256) void k_reac_sum(int64_t nq, int nseg, const double* __restrict__ part,
                                                  const int64_t* __restrict__ near_ptr,
                                                  const int32_t* __restrict__ near_col,
                                                  const double* __restrict__ near_val,
                                                  const double* __restrict__ sig, const double* __restrict__ mu,
                                                  double* phi) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nq) return;
  double f = 0.0;
  for (int g = 0; g < nseg; ++g) f += part[(int64_t)g * nq + k];
  double l = f * kInv4Pi;
  for (int64_t e = near_ptr[k]; e < near_ptr[k + 1]; ++e) {
    const int32_t j = near_col[e];
    l += near_val[4 * e] * sig[j] + near_val[4 * e + 1] * mu[j];
  }
  phi[k] = -l;
}

// A cavity's part of the reaction potential at the charges of its molecule:
// the cavity is seen from outside with the Laplace kernel (its sources'
// single-layer strengths already carry eps_cavity / eps_in), i.e. minus the
// outside-form sum sum_j (s_j / r + D_j . (x - y_j) / r^3) / (4 pi) plus its
// near corrections, added to phi.  One block per charge.
__global__ __launch_bounds__(256) void k_reac_cavity(int64_t nq, const double* __restrict__ qxyz, int64_t s0,
                                                     int64_t s1, const double* __restrict__ src,
                                                     const int64_t* __restrict__ near_ptr,
                                                     const int32_t* __restrict__ near_col,
                                                     const double* __restrict__ near_val,
                                                     const double* __restrict__ sig,
                                                     const double* __restrict__ mu, double* phi) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  const double x = qxyz[3 * k], y = qxyz[3 * k + 1], z = qxyz[3 * k + 2];
  double a1 = 0.0, a2 = 0.0;
  for (int64_t j = s0 + threadIdx.x; j < s1; j += blockDim.x) {
    const double* s = src + (int64_t)kSrcStride * j;
    const double dx = x - s[0], dy = y - s[1], dz = z - s[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double dd = s[4] * dx + s[5] * dy + s[6] * dz;
    a1 += s[3] * rinv;
    a2 += dd * rinv * rinv * rinv;
  }
  double l = (a1 + a2) * kInv4Pi;
  for (int64_t e = near_ptr[k] + threadIdx.x; e < near_ptr[k + 1]; e += blockDim.x) {
    const int32_t j = near_col[e];
    l += near_val[4 * e] * sig[j] + near_val[4 * e + 1] * mu[j];
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) phi[k] -= red[0] + red[1] + red[2] + red[3];
}

}  // namespace

void launch_reac_cavity(int64_t nq, const double* qxyz, int64_t s0, int64_t s1, const double* src,
                        const int64_t* near_ptr, const int32_t* near_col, const double* near_val,
                        const double* sig, const double* mu, double* phi, hipStream_t s) {
  if (nq <= 0) return;
  k_reac_cavity<<<(unsigned)nq, 256, 0, s>>>(nq, qxyz, s0, s1, src, near_ptr, near_col, near_val, sig, mu, phi);
  PBT_HIP(hipGetLastError());
}

void launch_reac(int64_t nq, const double* qxyz, int64_t s0, int64_t s1, const double* src,
                 double rho_inv, const int64_t* near_ptr, const int32_t* near_col,
                 const double* near_val, const double* sig, const double* mu, double* phi,
                 double* part, hipStream_t s) {
  if (nq <= 0) return;
  // enough wavefronts to fill the machine, segments of at least 256 sources
  const int64_t ntile = (nq + 63) / 64;
  const int64_t want = std::max<int64_t>(1, 4096 / ntile);
  const int nseg = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kReacMaxSeg, want, (s1 - s0 + 255) / 256}));
  k_reac_part<<<dim3((unsigned)ntile, (unsigned)nseg), 64, 0, s>>>(nq, qxyz, s0, s1, nseg, src, rho_inv, part);
  PBT_HIP(hipGetLastError());
  k_reac_sum<<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(nq, nseg, part, near_ptr, near_col, near_val, sig, mu,
                                                            phi);
  PBT_HIP(hipGetLastError());
}

void launch_densities(int64_t np, const PanelMaps& m, const double* x, double* sig, double* mu,
                      hipStream_t s) {
  if (np <= 0) return;
  k_densities<<<nblocks(np, 256), 256, 0, s>>>(np, m, x, sig, mu);
  PBT_HIP(hipGetLastError());
}

void launch_rhs_solvent(int64_t np, const int32_t* row_sol, const double* ak, const double* half, double* b,
                        hipStream_t s) {
  if (np <= 0) return;
  k_rhs_solvent<<<nblocks(np, 256), 256, 0, s>>>(np, row_sol, ak, half, b);
  PBT_HIP(hipGetLastError());
}

void launch_known_densities(int64_t np, const double* ks, const double* km, double* sig, double* mu,
                            hipStream_t s) {
  if (np <= 0) return;
  k_known_densities<<<nblocks(np, 256), 256, 0, s>>>(np, ks, km, sig, mu);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_strengths(int64_t ns, int K, const double* sig, const double* mu, const double* src_wa,
                      const double* nrm, const double* rlap, T* src, hipStream_t s) {
  if (ns <= 0) return;
  k_strengths<T><<<nblocks(ns, 256), 256, 0, s>>>(ns, K, sig, mu, src_wa, nrm, rlap, src);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_strengths_x(int64_t ns, int K, const PanelMaps& m, const double* x, const double* src_wa,
                        const double* nrm, const double* rlap, double* sig, double* mu, T* src,
                        hipStream_t s) {
  if (ns <= 0) return;
  k_strengths_x<T><<<nblocks(ns, 256), 256, 0, s>>>(ns, K, m, x, src_wa, nrm, rlap, sig, mu, src);
  PBT_HIP(hipGetLastError());
}

void launch_to_f32(int64_t n, const double* in, float* out, hipStream_t s) {
  if (n <= 0) return;
  k_to_f32<<<nblocks(n, 256), 256, 0, s>>>(n, in, out);
  PBT_HIP(hipGetLastError());
}

template <typename T>
void launch_combine(const CombineArgs& a, const T* partial, const T* ppartial, double* y, hipStream_t s) {
  if (a.np <= 0 || a.nchunks <= 0) return;
  k_combine<T><<<a.nchunks, 64 * kCombineWaves, 0, s>>>(a, partial, ppartial, y);
  PBT_HIP(hipGetLastError());
}

template void launch_strengths<float>(int64_t, int, const double*, const double*, const double*,
                                      const double*, const double*, float*, hipStream_t);
template void launch_strengths<double>(int64_t, int, const double*, const double*, const double*,
                                       const double*, const double*, double*, hipStream_t);
template void launch_strengths_x<float>(int64_t, int, const PanelMaps&, const double*, const double*,
                                        const double*, const double*, double*, double*, float*, hipStream_t);
template void launch_strengths_x<double>(int64_t, int, const PanelMaps&, const double*, const double*,
                                         const double*, const double*, double*, double*, double*, hipStream_t);
template void launch_combine<float>(const CombineArgs&, const float*, const float*, double*, hipStream_t);
template void launch_combine<double>(const CombineArgs&, const double*, const double*, double*, hipStream_t);

}  // namespace pbt
