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
// A work item of the interaction kernels: targets tbeg .. tbeg+tcount-1
// against the source ranges (P2P) or boxes (M2P) lbeg .. lend-1.  A task
// holds up to 32 targets, half a wavefront: tasks come in pairs, one per
// half, each writing slot `slot` of the half-wave partials [slot][32][2].
struct Task {
  int32_t tbeg;    // first target (internal order)
  int32_t tcount;  // 0..64 (M2P), 0..32 (P2P; 0 = an empty half)
  int32_t lbeg, lend;
  int32_t slot;    // partial-sum slot
  int32_t fused;   // 1: Laplace interior row + Yukawa row; 0: Yukawa row only
  float rho_inv_f; // eps_out / eps_source, used by the Laplace row
  int32_t nsrc;    // P2P: number of sources in the ranges
  double rho_inv;
  int32_t split;   // P2P: 1, 2 or 4 lane groups share the half's targets (tcount <= 32 / split),
                   // each taking every split-th source; both halves of a wavefront agree
  int16_t known;   // 1: the sources lie on a charged or potential surface (the only sources
                   // with known densities, which the right-hand side sums over)
  int16_t form;    // kForm* bits: how the two sums map to the two rows (Stern layers)
};

// Task::form bits.  A target row gets a source surface's sum in one of three
// forms: as seen from inside the surface (the Laplace sum of the interior
// row), as seen from outside it with the Yukawa kernel, or as seen from
// outside with the Laplace kernel (inside a salt-free Stern layer).  The
// task computes its usual pair (Laplace sum, outside sum); kFormKz takes
// kappa = 0 for the outside sum, kFormDropOut discards it, and kFormSwap
// stores the pair in the opposite rows (outside sum to the interior row).
constexpr int kFormKz = 1, kFormSwap = 2, kFormDropOut = 4;

// Per 64-target chunk: per half (targets 0..31 and 32..63), the half-wave
// slots [hbeg, hend) of its P2P and M2P tasks; [sbeg, send), slots of 64
// lanes, is empty in the forward plan (the transpose plan uses it).
struct ChunkSlots {
  int32_t tbeg, tcount, sbeg, send;
  int32_t hbeg0, hend0, hbeg1, hend1;
  int32_t grp, lchunk;   // the targets' group and the chunk's index within it
};

// Units: lengths in A, charges in e, potentials in e/(eps0 A), energies in
// e^2/(eps0 A).  CODATA-2018 exact constants for the conversions at the ABI.
constexpr double kFourPi = 12.566370614359172;
constexpr double kE = 1.602176634e-19, kEps0 = 8.8541878128e-12, kNA = 6.02214076e23;
constexpr double kVoltPerUnit = kE / (kEps0 * 1e-10);              // e/(eps0 A) in V
constexpr double kKcalPerUnit = kE * kE / (kEps0 * 1e-10) * kNA / 4184.0;
constexpr double kSigmaSI = 1e-20 / kE;                            // C/m^2 -> e/A^2

constexpr int kSrcStride = 8;  // x y z s Dx Dy Dz s_L
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
// Near lists (panels closer than f L, f = near_factor, 2 in the paper):
// every target scans all np panels (tleaf null) or the candidate ranges of
// its leaf (CSR lptr / lrange); f4 = (f f)(f f).
inline double near_f4(double f) { return (f * f) * (f * f); }
void launch_near_count(int64_t nt, const double* tx, int64_t np, const double* cen,
                       const double* cross2, const int32_t* tleaf, const int64_t* lptr,
                       const int64_t* lrange, double f4, int32_t* count, hipStream_t s);
void launch_near_fill(int64_t nt, const double* tx, int64_t np, const double* cen,
                      const double* cross2, const int32_t* tleaf, const int64_t* lptr,
                      const int64_t* lrange, double f4, const int64_t* rowptr, int32_t* col, hipStream_t s);
void launch_pack_points(int64_t np, int64_t ns, const double* cen, const double* src_pos, double* t64, float* t32,
                        double* s64, float* s32, hipStream_t s);
struct NearParams {
  int K, Knear, Nedge;
  double kappa;
  const double* bary_far; const double* w_far;
  const double* bary_near; const double* w_near;
  const double* gl_t; const double* gl_w;
};
// vals[4*e] = (V_L, K_L, V_Y, K_Y) corrections: fine (or self) minus the K-point rule.
// Rows i with skip[i] >= 0 (skip nullable) are left alone.
void launch_near_values(int64_t nt, const double* tx, const int32_t* tgt_self, const int64_t* rowptr,
                        const int32_t* col, const double* tri9, const double* nrm,
                        const double* area, const NearParams& p, double* vals, hipStream_t s,
                        const int32_t* skip = nullptr);
// Rows of targets i with rep[i] >= 0 taken from row rep[i] (the same length):
// columns shifted by i - rep[i] (a copy of a surface, its panels at that
// offset), then, after the values, the values copied.
void launch_near_copy_cols(int64_t nt, const int32_t* rep, const int64_t* rowptr, int32_t* col, hipStream_t s);
void launch_near_copy_vals(int64_t nt, const int32_t* rep, const int64_t* rowptr, double* vals, hipStream_t s);
// Inverse self blocks of every panel (m[4 np]: z_phi = m0 v_int + m1 v_out,
// z_psi = m2 v_int + m3 v_out), the right block-Jacobi preconditioner.
void launch_self_blocks(int64_t np, const double* tri9, const double* cen, const int32_t* panel_surf,
                        const uint8_t* forms, int nsurf, const double* surf_rhoinv, const double* dens_scale,
                        const int32_t* col_phi, const int32_t* col_psi, const NearParams& p, double* m,
                        hipStream_t s);
// tgt_surf null: every target belongs to surface tsurf.
void launch_fold_near(int64_t nt, const int64_t* rowptr, const int32_t* col, const int32_t* tgt_surf,
                      const int32_t* panel_surf, const uint8_t* forms, int nsurf, const double* surf_rhoinv,
                      double* vals, hipStream_t s, int32_t tsurf = 0, const int32_t* skip = nullptr);
void launch_reac_cavity(int64_t nq, const double* qxyz, int64_t s0, int64_t s1, const double* src,
                        const int64_t* near_ptr, const int32_t* near_col, const double* near_val,
                        const double* sig, const double* mu, double* phi, hipStream_t s);
// part: scratch of kReacMaxSeg nq doubles.
constexpr int kReacMaxSeg = 64;
void launch_reac(int64_t nq, const double* qxyz, int64_t s0, int64_t s1, const double* src,
                 double rho_inv, const int64_t* near_ptr, const int32_t* near_col,
                 const double* near_val, const double* sig, const double* mu, double* phi,
                 double* part, hipStream_t s);
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
                      const double* nrm, const double* rlap, T* src, hipStream_t s);
template <typename T>
void launch_strengths_x(int64_t ns, int K, const PanelMaps& m, const double* x, const double* src_wa,
                        const double* nrm, const double* rlap, double* sig, double* mu, T* src,
                        hipStream_t s);
template <typename T>
// P2P over npairs pairs of tasks (tasks[2w], tasks[2w+1] share wavefront w);
// partials [slot][32][2].
void launch_p2p(const Task* tasks, int npairs, const int32_t* ranges, const T* tgt, const T* src,
                T kappa, bool guard, T* partial, hipStream_t s);
// P2P tasks between surfaces shared by G groups: each task (group 0's
// targets and source ranges) is evaluated for every group g, with group g's
// source strengths (group 0's sources shifted by goff[g] panels of K points)
// and written to partial slot mslot[task.slot * G + g]; nrm holds the
// panels' unit normals (FP64).
// Groups served by one shared-surface task (Task::split = its first group).
constexpr int kMultiBlock = 16;
template <typename T>
void launch_p2p_multi(const Task* tasks, int npairs, const int32_t* ranges, const T* tgt, const T* src,
                      const double* nrm, int K, const int32_t* goff, const int32_t* mslot, int G, T kappa,
                      bool guard, T* partial, hipStream_t s);
struct CombineArgs {
  int64_t np;
  const ChunkSlots* chunks; int nchunks;
  const int32_t* chunk_of;       // per target
  const int64_t* near_ptr; const int32_t* near_col; const double* near_val;  // (cLs, cLm, cYs, cYm)
  const float* near_val32;       // the same values rounded to FP32 (read by the FP32 combine)
  const double* sig; const double* mu;
  const double* x;               // unknowns (jump terms); may be null when add_jump = 0
  PanelMaps maps;
  int add_jump;
  // When ndots > 0, also the first Gram-Schmidt pass of the product: the
  // chunk's part of V_i . y for i < ndots goes to dpart[(grp R + i) nbh + lchunk],
  // and with self_dot that of y . y to row ndots.
  int ndots;
  const double* V; int64_t ldv;
  double* dpart; int R; int nbh;
  int self_dot;
};
template <typename T>
void launch_combine(const CombineArgs& a, const T* partial, const T* ppartial, double* y, hipStream_t s);
// out[i] = (float)in[i], i < n.
void launch_to_f32(int64_t n, const double* in, float* out, hipStream_t s);

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
// Moments of the boxes M2P reads, straight from their sources (taylor.hip).
// A box's sources [sbeg, send) are one chunk (groups of kMomGroup
// coefficients a block, or of kMomGroupFine when `fine`: a larger box, its
// work spread over more blocks) or, for the largest boxes, several chunks:
// chunk idx of nparts writes partial slot slot0 + idx, and `heads` (the idx 0
// chunk of every such box) drives the sum of the slots.  The launch runs one
// block per entry (chunk, coefficient group) of the block list.
struct MomChunk {
  int32_t box, sbeg, send;
  int32_t slot0, nparts, idx;
  int32_t fine, pad_;
};
constexpr int kMomChunk = 1024;     // sources of a plain chunk (16 a lane)
constexpr int kMomFineMax = 16384;  // largest box done as one fine chunk
constexpr int kMomGroup = 12;       // coefficients per block
constexpr int kMomGroupFine = 4;
constexpr int mom_groups(int P, int gs = kMomGroup) { return (ncoef(P) + gs - 1) / gs; }
// The same moments in one launch with the P2P task pairs (then the chunk sums).
template <typename T>
void launch_p2p_moments(int P, int nblocks, const int32_t* mblocks, const MomChunk* chunks, int nheads,
                        const MomChunk* heads, const double* bcen, const double* brho, T* mom, T* mpart,
                        const Task* p2p, int npairs, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                        bool guard, T* ppartial, hipStream_t s);
template <typename T>
void launch_moments(int P, int nblocks, const int32_t* mblocks, const MomChunk* chunks, int nheads,
                    const MomChunk* heads, const double* bcen, const double* brho, const T* src, T* mom, T* mpart,
                    hipStream_t s);
// Moments of boxes from their leaves' (M2M): pairs[3 i] = (box, leaf,
// slot) shift the leaf's moments to the box's centre into slot (2 ncoef(P)
// values each), then heads[3 h] = (box, first slot, count) add a box's slots
// in order into its moments; the first nsmall heads have count <= kM2MSmall.
constexpr int kM2MSmall = 32;
template <typename T>
void launch_m2m(int P, int npairs, const int32_t* pairs, int nheads, int nsmall, const int32_t* heads,
                const double* bcen, T* slots, T* mom, hipStream_t s);
// M2P half tasks (ntasks / nm2p of them, consecutive pairs sharing a
// wavefront) write the half-wave partials [slot][32][2], like P2P.
// M2P and P2P tasks in one launch (taylor.hip).
template <typename T>
void launch_m2p_p2p(int P, const Task* m2p, int nm2p, const int32_t* blist, const double* bcen, const T* mom,
                    const Task* p2p, int np2p, const int32_t* ranges, const T* src, const T* tgt, T kappa,
                    bool guard, T* ppartial, hipStream_t s);
template <typename T>
void launch_m2p(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                const double* box_center, const T* mom, T kappa, T* partial, hipStream_t s);
// M2P tasks between surfaces shared by G groups (like launch_p2p_multi):
// group g's copy of box b is b + boxoff[task.nsrc * G + g]; each task
// serves groups split .. split + kMultiBlock - 1.
template <typename T>
void launch_m2p_multi(int P, const Task* tasks, int ntasks, const int32_t* blist, const T* tgt,
                      const double* box_center, const T* mom, const int32_t* boxoff, const int32_t* mslot, int G,
                      T kappa, T* partial, hipStream_t s);

// --- transpose operator (adjoint.hip) ---------------------------------------
struct AdjCombineArgs {
  int64_t np;
  int K;
  const ChunkSlots* chunks;   // reverse-P2P slots per 64-source chunk (nullable)
  const int32_t* chunk_of;    // per source
  const double* wa;           // per source: w A
  const double* nrm;          // per panel
  const int64_t* tptr;        // near corrections by source panel (nullable)
  const int32_t* trow;        // target panel of each entry
  const double* tval;         // (cLs, cLm, cYs, cYm)
  const double* lam;          // row weights (nullable: no near or jump terms)
  const double* add_sig;      // extra per-panel sigmabar / mubar (nullable)
  const double* add_mu;
  PanelMaps maps;
};
template <typename T>
void launch_adj_targets(int64_t np, const double* cen, const int32_t* row_int, const int32_t* row_sol,
                        const double* lam, T* trec, hipStream_t s);
template <typename T>
void launch_p2p_t(const Task* tasks, int ntasks, const int32_t* ranges, const T* src, const T* trec,
                  T kappa, bool guard, T* partial, hipStream_t s);
template <typename T>
void launch_m2p_t(int P, const Task* tasks, int ntasks, const T* trec, const double* bcen, T kappa,
                  T* mpart, hipStream_t s);
template <typename T>
void launch_mbar_reduce(int nbox, int P, const int32_t* sbeg, const int32_t* send, const T* mpart,
                        T* mbar, hipStream_t s);
template <typename T>
void launch_m2m_t(int P, int nbox, const int32_t* boxes, const int32_t* parent, const double* bcen,
                  T* mbar, hipStream_t s);
template <typename T>
void launch_l2p_t(int P, int nleaf, const int32_t* leaves, const BoxDev& bd, const T* src,
                  const T* mbar, T* far, hipStream_t s);
template <typename T>
void launch_combine_t(const AdjCombineArgs& a, const T* partial, const T* far, double* z, double* sigbar,
                      hipStream_t s);
void launch_reac_t(int64_t s0, int64_t s1, const double* src, int64_t nq, const double* qxyz,
                   const double* q, double rho_inv, double* far, double dsign, hipStream_t s);
void launch_coulomb_t(int64_t nq, const double* qxyz, int64_t n, const double* tx, const int32_t* rows,
                      const double* lam, double inv_eps, double* out, hipStream_t s);

// --- Krylov (krylov.hip) ----------------------------------------------------
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
// Krylov kernels (krylov.hip), for G independent systems at once: group g
// owns the unknowns gu[2g] .. gu[2g+1] (device array) and its own Krylov
// space.  One Arnoldi step = two Gram-Schmidt passes of partial dots (pass
// 1: hpart = null; pass 2: reduces pass 1's partials into hout and dots with
// w - V h1), then w = (w - V (h1 + h2)) / |w''| together with each group's
// Hessenberg column and Givens rotation.  R = rows reserved per group in
// the partial and h buffers (restart + 1).
int gs_blocks(int64_t n);
// hpart rows have stride nbh (the previous pass's block count).
void launch_gs_dots(const int64_t* gu, int G, int m, int R, const double* V, int64_t ldv, const double* w,
                    const double* hpart, int nbh, double* hout, int self_dot, double* part, int nbj,
                    hipStream_t s, bool all_rows = false);
// Source records of the next Krylov vector, written by the Arnoldi update
// (the strengths of launch_strengths_x, from the updated unknowns): panels
// of group g are gp[2g] .. gp[2g+1], pmax is the largest group's panel
// count; records are float (fp32) or double.
struct NextSrc {
  const int64_t* gp;
  int64_t pmax;
  int fp32;
  PanelMaps m;
  int K;
  const double* wa;
  const double* nrm;
  const double* rlap;
  double* sig;
  double* mu;
  void* src;
  const double* pinv;   // inverse self blocks (right preconditioner), or null
  double* zout;         // with pinv: z = M^-1 v of the new basis vector
};
void launch_arnoldi_update(const int64_t* gu, int G, int64_t nmax, int j, int m, int R, int nbj,
                           const double* part, const double* h1, const double* V, int64_t ldv, double* w,
                           double* H, double* cs, double* sn, double* gv, double* resid, const NextSrc* ns,
                           hipStream_t s);
void launch_group_row0(int G, int R, int nbj, const double* part, double* out, hipStream_t s);
// out = M^-1 v (M^-T v with transpose; out += with add), per panel from its
// inverse self block pinv[4 p] (right block-Jacobi preconditioner).
void launch_precond(int64_t np, const int32_t* col_phi, const int32_t* col_psi, const double* pinv, const double* v,
                    double* out, bool transpose, bool add, hipStream_t s);
// out[g R + i] = sum of the nbh partials of row i of group g, i < nrows
// (rows of R per group in both), in a fixed order.  Rows of up to
// kSumBatch partials are added with one batch of loads per lane.
constexpr int kSumBatch = 256;
void launch_reduce_partials(int G, int nrows, int R, int nbh, const double* part, double* out, hipStream_t s);
// out[u2i[k]] = in[k] (to_internal) or out[k] = in[u2i[k]] (otherwise), k < n.
void launch_permute(int64_t n, const int32_t* u2i, const double* in, double* out, bool to_internal,
                    hipStream_t s);
void launch_lincomb(const int64_t* gu, int G, int64_t nmax, int m, int ystride, const double* V, int64_t ldv,
                    const double* y, double* x, hipStream_t s);
void launch_start_cycle(const int64_t* gu, int G, int64_t nmax, int m, const double* beta, const double* inv_beta,
                        const double* r, double* v0, double* gv, hipStream_t s);
void launch_rhs_solvent(int64_t np, const int32_t* row_sol, const double* ak, const double* half, double* b,
                        hipStream_t s);

}  // namespace pbt
