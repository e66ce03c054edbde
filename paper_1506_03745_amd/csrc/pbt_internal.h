// Internal declarations of the pbt library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace pbt {

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define PBT_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::pbt::Error(3, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

// ---------------------------------------------------------------------------
// Work items shared by the P2P and M2P kernels.  One wavefront processes one
// task: up to 64 consecutive targets (one per lane) against a list segment
// [lbeg, lend) of source ranges (P2P) or source boxes (M2P), and writes its
// partial (L, Y) sums for its lanes into partial slot `slot`.
// ---------------------------------------------------------------------------
struct Task {
  int32_t tbeg;    // first target (internal order)
  int32_t tcount;  // 1..64
  int32_t lbeg, lend;
  int32_t slot;    // partial-sum slot
  int32_t fused;   // 1: Laplace interior row + Yukawa row; 0: Yukawa row only
  float rho_inv_f; // eps_out / eps_source, used by the Laplace row
  int32_t pad;
  double rho_inv;
};

// Per-target bookkeeping for the combine step.
struct ChunkSlots {
  int32_t tbeg, tcount, sbeg, send;
};

constexpr int kSrcStride = 8;  // x y z s Dx Dy Dz pad
constexpr int kTgtStride = 4;  // x y z pad

// Number of Taylor coefficients with |k| <= P.
constexpr int ncoef(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }
constexpr int kMaxP = 8;

// --- setup kernels (setup_kernels.hip) -------------------------------------
void launch_panel_geometry(int64_t np, const double* tri9, double* cen, double* nrm, double* area,
                           double* cross2, hipStream_t s);
void launch_sources(int64_t np, int K, const double* tri9, const double* nrm, const double* area,
                    const double* bary, const double* w, double* src_pos, double* src_wa,
                    hipStream_t s);
void launch_near_count(int64_t nt, const double* tx, int64_t np, const double* cen,
                       const double* cross2, int32_t* count, hipStream_t s);
void launch_near_fill(int64_t nt, const double* tx, int64_t np, const double* cen,
                      const double* cross2, const int64_t* rowptr, int32_t* col, hipStream_t s);
struct NearParams {
  int K, Knear, Nedge;
  double kappa;
  const double* bary_far; const double* w_far;
  const double* bary_near; const double* w_near;
  const double* gl_t; const double* gl_w;
};
// vals[4*e] = (V_L, K_L, V_Y, K_Y) corrections: fine (or self) minus the K-point rule.
void launch_near_values(int64_t nt, const double* tx, const int32_t* tgt_self, const int64_t* rowptr,
                        const int32_t* col, const double* tri9, const double* nrm,
                        const double* area, const NearParams& p, double* vals, hipStream_t s);
void launch_fold_near(int64_t nt, const int64_t* rowptr, const int32_t* col, const int32_t* tgt_surf,
                      const int32_t* panel_surf, const int32_t* surf_mol, const double* surf_rhoinv,
                      double* vals, hipStream_t s);
void launch_reac(int64_t nq, const double* qxyz, int64_t s0, int64_t s1, const double* src,
                 double rho_inv, const int64_t* near_ptr, const int32_t* near_col,
                 const double* near_val, const double* sig, const double* mu, double* phi,
                 hipStream_t s);
void launch_coulomb_rhs(int64_t n, const double* tx, const int32_t* rows, int64_t nq,
                        const double* qxyz, const double* q, double inv_eps, double* b,
                        hipStream_t s);

// --- per-matvec kernels (matvec_kernels.hip) -------------------------------
struct PanelMaps {
  const int32_t* col_phi;  // unknown index of phi or -1
  const int32_t* col_psi;  // unknown index of dphi/dn or -1
  const int32_t* row_int;  // interior row or -1
  const int32_t* row_sol;  // solvent row
  const double* dens_scale; // eps_s/eps_out for molecules, 1 otherwise (scales psi into sigma)
};
void launch_densities(int64_t np, const PanelMaps& m, const double* x, double* sig, double* mu,
                      hipStream_t s);
void launch_known_densities(int64_t np, const double* known_sig, const double* known_mu, double* sig,
                            double* mu, hipStream_t s);
template <typename T>
void launch_strengths(int64_t ns, int K, const double* sig, const double* mu, const double* src_wa,
                      const double* nrm, T* src, hipStream_t s);
template <typename T>
void launch_p2p(const Task* tasks, int ntasks, const int32_t* ranges, const T* tgt, const T* src,
                T kappa, bool guard, T* partial, hipStream_t s);
struct CombineArgs {
  int64_t np;
  const ChunkSlots* chunks; int nchunks;
  const int32_t* chunk_of;       // per target
  const int64_t* near_ptr; const int32_t* near_col; const double* near_val;  // (cLs, cLm, cYs, cYm)
  const double* sig; const double* mu;
  const double* x;               // unknowns (jump terms); may be null when add_jump = 0
  PanelMaps maps;
  int add_jump;
};
template <typename T>
void launch_combine(const CombineArgs& a, const T* partial, double* y, hipStream_t s);

// --- Taylor-series far field (taylor.hip) ----------------------------------
struct BoxDev {
  const double* center;   // [nbox][3]
  const int32_t* sbeg;    // source range per box
  const int32_t* send;
  const int32_t* child_beg; // children indices [child_beg, child_end) in child_list
  const int32_t* child_end;
  const int32_t* child_list;
  const double* rho_inv;  // per box: eps_out/eps_s of its surface (molecule) or 0
};
template <typename T>
void launch_p2m(int P, int nbox, const int32_t* boxes, const BoxDev& b, const T* src, T* mom,
                hipStream_t s);
template <typename T>
void launch_m2m(int P, int nbox, const int32_t* boxes, const BoxDev& b, T* mom, hipStream_t s);
template <typename T>
void launch_m2p(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                const double* box_center, const T* mom, T kappa, T* partial, hipStream_t s);

// --- Krylov BLAS-1 (krylov.hip) ---------------------------------------------
void launch_multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* part,
                     int nblk, hipStream_t s);
void launch_reduce_cols(int m, int nblk, const double* part, double* out, hipStream_t s);
void launch_multi_axpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w,
                       hipStream_t s);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
void launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s);
void launch_lincomb(int64_t n, int m, const double* V, int64_t ldv, const double* c, double* y,
                    hipStream_t s);
int multidot_blocks(int64_t n);

}  // namespace pbt
