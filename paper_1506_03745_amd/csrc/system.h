// A prepared boundary-element system: geometry, near-field corrections,
// octrees, interaction lists and work decomposition for one set of enabled
// surfaces, plus the operator, right-hand side, GMRES and energies.
#pragma once

#include <array>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pbt.h"
#include "pbt_internal.h"
#include "tree.h"

namespace pbt {

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t m) {
    if (m == n && p) return;
    release();
    if (m) {
      hipError_t e = hipMalloc(&p, m * sizeof(T));
      if (e != hipSuccess) throw Error(2, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    n = m;
  }
  // Synchronous with respect to the host vector: it may be released on return.
  void upload(const T* v, size_t m, hipStream_t s) {
    alloc(m);
    if (m) {
      PBT_HIP(hipMemcpyAsync(p, v, m * sizeof(T), hipMemcpyHostToDevice, s));
      PBT_HIP(hipStreamSynchronize(s));
    }
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size());
    if (!v.empty()) {
      PBT_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
      PBT_HIP(hipStreamSynchronize(s));
    }
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> v(n);
    if (n) {
      PBT_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      PBT_HIP(hipStreamSynchronize(s));
    }
    return v;
  }
};

// Pinned host memory, for readbacks that the host waits on.
template <typename T>
struct HBuf {
  T* p = nullptr;
  size_t n = 0;
  HBuf() = default;
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  ~HBuf() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t m) {
    if (m <= n && p) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc((void**)&p, m * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) throw Error(2, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    n = m;
  }
};

struct SurfIn {
  uint64_t version = 0;  // bumped whenever bc or the charges change
  int kind = 0;
  int64_t nv = 0, nt = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tri;
  std::vector<double> bc;  // SI: sigma [C/m^2] or phi0 [V]
  double eps_in = 1.0;
  std::vector<double> qxyz, q;
  bool enabled = true;
  int group = 0;  // surfaces of different groups belong to independent systems
  const SurfIn* parent = nullptr;  // Stern surface: the molecule it encloses; cavity: the molecule around it
  int shared = -1;  // >= 0: a copy, in every group, of one surface that the groups share unmoved
};

struct NearCSR {
  DBuf<int64_t> ptr;
  DBuf<int32_t> col;
  DBuf<double> val;
  DBuf<float> val32;   // FP32 copy for FP32-interaction products (collocation corrections only)
  int64_t nnz = 0;
};

// Work decomposition of one target set against all source surfaces.
struct Plan {
  std::vector<Task> p2p, m2p;
  std::vector<Task> p2p_known, m2p_known;   // right-hand side: only known-density sources do work
  std::vector<int32_t> ranges, blist;
  std::vector<ChunkSlots> chunks;
  std::vector<int32_t> chunk_of;
  int nslots = 0;    // M2P partial slots (64 lanes)
  int nbh = 1;       // most target chunks of one group
  int npslots = 0;   // P2P partial slots (32 lanes)
  int64_t p2p_pairs = 0, m2p_pairs = 0, p2p_fused_pairs = 0, m2p_fused_pairs = 0;
  // P2P between surfaces that every group holds unmoved: tasks on group 0's
  // copies (pairs of half tasks), each evaluated for all mgroups groups at
  // once; task.slot is a row of mslot, whose entry g is the partial slot of
  // group g, and group g's sources are group 0's shifted by goff[g] panels
  std::vector<Task> p2pm;
  std::vector<int32_t> mslot, goff;
  int mgroups = 0;
  // M2P between them likewise (m2pm, rows of mslot too): task.nsrc is a row
  // of mboxoff, whose entry g is the offset of group g's box numbers of the
  // source surface from group 0's
  std::vector<Task> m2pm;
  std::vector<int32_t> mboxoff;
};

struct Timing {
  double total = 0, p2p = 0, m2p = 0, moments = 0, rest = 0;
};

class System {
 public:
  System(const std::vector<const SurfIn*>& surfs, const pbt_params& prm, double eps_out,
         double kappa, hipStream_t stream);
  ~System();

  int64_t n() const { return n_; }
  int64_t np() const { return np_; }
  // Target x Gauss-point pairs a dense product evaluates: every target
  // against every source of its own group (independent systems do not pair).
  int64_t dense_pairs() const { return dense_pairs_; }
  const Plan& plan() const { return plan_; }

  // y = A x on device buffers (n doubles each), FP64 or FP32 interactions;
  // `timed` records the per-phase events read by timing().
  // Unknown vectors between the boundary's layout (panels of each surface in
  // their original order) and the internal one (the octree's order).
  void to_internal(const double* xu, double* xi, hipStream_t s) const;
  void to_boundary(const double* xi, double* xu, hipStream_t s) const;
  // src_ready: the source records, sig and mu of x are already in place;
  // dots: also the first Gram-Schmidt pass V_i . y, i < ndots, as per-chunk
  // partials (dpart rows of plan().nbh, R rows per group), and y . y as row
  // ndots with self_dot.
  struct DotReq {
    int ndots;
    const double* V;
    int64_t ldv;
    double* dpart;
    int R;
    int self_dot = 0;
  };
  // Caller-owned buffers for the P2P and M2P partial sums of a product
  // (instead of the system's own), of part_need() / ppart_need() bytes.
  struct ExtParts {
    void* part;
    void* ppart;
  };
  size_t part_need(bool fp32) const { return fp32 ? part_bytes<float>() : part_bytes<double>(); }
  size_t ppart_need(bool fp32) const { return fp32 ? ppart_bytes<float>() : ppart_bytes<double>(); }
  void matvec(const double* x, double* y, bool fp32, hipStream_t s, bool timed = false, bool src_ready = false,
              const DotReq* dots = nullptr, const ExtParts* ext = nullptr);
  // FP64 right-hand side for the current charges and boundary values.
  void rhs(double* b_dev, hipStream_t s);
  // Solves A x = b (b, x device); returns result fields (iters, outer,
  // rel_resid, matvecs) and whether it converged.  The surface groups are
  // independent systems: each is solved to its own relative tolerance and
  // rel_resid is the largest group's (group_rel() lists them).
  bool solve(const double* b, double* x, bool x0_given, pbt_result* res, hipStream_t s);
  const std::vector<double>& group_rel() const { return group_rel_; }
  // Energies (kcal/mol) of solution x (device).
  void energies(const double* x, pbt_result* res, hipStream_t s);
  // Energies per group (index = group id), same units.
  std::vector<pbt_result> energies_by_group(const double* x, int ngroups, hipStream_t s);
  // Host copy of a surface's solution in caller order.
  void unpack(const std::vector<double>& xh, int local_surface, double* phi, double* dphidn) const;
  int local_index(int surface_id) const;

  // z = A^T lam (device buffers), the exact transpose of matvec; sigbar
  // (nullable, np doubles) receives d(lam^T y)/d sigma per panel.
  void matvec_t(const double* lam, double* z, bool fp32, double* sigbar, hipStream_t s);
  // Adjoint right-hand side g = dF_total/du at the solution x (device, FP64).
  void adjoint_rhs(const double* x, double* g, hipStream_t s);
  // Solves A^T lam = g like solve() does for A.
  bool solve_t(const double* g, double* lam, pbt_result* res, hipStream_t s);
  // Gradient of F_total (reduced units) w.r.t. each molecule's charges and
  // each charged surface's sigma, from the solution x and the adjoint lam.
  void gradient_terms(const double* x, const double* lam, std::vector<std::vector<double>>& dq,
                      std::vector<std::vector<double>>& dsig, hipStream_t s);
  const SurfIn* surface(int e) const { return surfs_[e]; }
  // Whether some enabled surface is a Stern layer or a cavity (the
  // transpose, gradient and batched paths do not take them).
  bool has_nested() const { return has_nested_; }

  // Launch shape of the P2P / M2P tasks: Gauss points per P2P segment and
  // boxes per M2P segment (0 = size-based default).  Rebuilds the work lists.
  void set_segments(int64_t seg_src, int64_t seg_box, hipStream_t s);
  int64_t seg_src() const { return seg_src_used_; }
  int64_t seg_box() const { return seg_box_used_; }
  // Average milliseconds of `reps` operator applications (after one warm-up).
  double time_products(bool fp32, int reps, hipStream_t s);
  int n_surfaces() const { return (int)surfs_.size(); }

  // Milliseconds of the last operator application: total, P2P, M2P,
  // moments (P2M, M2M), and strengths + combine; P2P and the far field
  // (moments, M2P) run concurrently on two streams.
  void timing(double out[5]);
  // Operator applications since construction (every matvec and rhs pass),
  // not counting speculative Arnoldi steps discarded after convergence.
  int64_t applications() const { return napply_ - nwasted_; }
  // How the far field (moments, M2P) and P2P are scheduled:
  //   0: P2P, then the far field, on the caller's stream;
  //   1: the moments, then M2P on a second stream concurrently with P2P;
  //   2: moments first, then M2P and P2P tasks in one launch;
  //   3: moments inside the P2P launch, then M2P;
  //   4, 5, 6: moments inside a launch with 7/8, 3/4 or 1/2 of the P2P
  //      pairs, then M2P and the remaining P2P pairs in one launch.
  void set_far_mode(int mode) { far_mode_ = mode; }
  // Gram-Schmidt passes per Arnoldi step: 2 (classical, twice), 1 (once,
  // the new vector's norm by Pythagoras from the same reduction) or 0
  // (one pass for GMRES targets of at least 1e-7 relative, else two).
  void set_gs_passes(int n) { gs_passes_ = n; }
  int gs_passes() const { return gs_passes_; }
  int far_mode() const { return far_mode_; }

  // Per-kernel timing of every full product (off by default): HIP events on
  // the stream of each launch, read back in batches.  Totals by slot =
  // 4 * (0 FP32 | 1 FP64) + kind, kinds 0 the launch holding P2P, 1 the
  // launch of M2P (when separate), 2 moments (when separate), 3 combine.
  // set_profile(true) also clears the totals.
  void set_profile(bool on);
  // Adds this system's totals: out[2 * slot] ms, out[2 * slot + 1] launches.
  void add_profile(double out[16]);
  // Exact dense-equivalent target x Gauss-point pairs of the applications
  // made so far: a full product counts dense_pairs(), the right-hand side's
  // product (known densities only) its targets times the known sources;
  // speculative Arnoldi steps discarded after convergence do not count.
  int64_t pairs_done() const { return pairs_done_ - nwasted_ * dense_pairs_; }

 private:
  bool prof_ = false;
  std::vector<hipEvent_t> pev_;
  int pev_used_ = 0;
  struct PMark { int slot, e0, e1; };
  std::vector<PMark> pmarks_;
  double ptot_[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t pcnt_[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int prof_begin(hipStream_t s);
  void prof_end(int slot, int e0, hipStream_t s);
  void prof_flush();
  int64_t pairs_done_ = 0, known_pairs_ = 0;

  void build(hipStream_t s);
  void build_plan();
  void apply(bool fp32, bool add_jump, const double* x, double* y, hipStream_t s, bool from_x = false,
             bool timed = false, bool src_ready = false, const DotReq* dots = nullptr, bool known_only = false,
             const ExtParts* ext = nullptr);
  template <typename T>
  void interactions(hipStream_t s, const double* x, bool timed, bool src_ready, bool known_only,
                    const ExtParts* ext);
  // bytes of the M2P / P2P partial-slot buffers in precision T
  template <typename T>
  size_t part_bytes() const { return (size_t)std::max(plan_.nslots, 1) * 128 * sizeof(T); }
  template <typename T>
  size_t ppart_bytes() const { return (size_t)std::max(plan_.npslots, 1) * 64 * sizeof(T); }
  int gmres(bool fp32, const double* b, double* x, bool x_zero, const std::vector<double>& tol_abs,
            int restart, int maxit, std::vector<double>& resid_out, hipStream_t s,
            const std::vector<double>* b_norms = nullptr);
  void ensure_groups(hipStream_t s);
  std::vector<double> group_norms(const double* v, hipStream_t s);
  void true_residual(const double* b, const double* x, double* r, hipStream_t s);
  void op(const double* x, double* y, bool fp32, hipStream_t s, bool src_ready = false,
          const DotReq* dots = nullptr) {
    if (transpose_) matvec_t(x, y, fp32, nullptr, s);
    else matvec(x, y, fp32, s, false, src_ready, dots);
  }
  bool solve_any(const double* b, double* x, bool x0_given, pbt_result* res, hipStream_t s);
  void build_tplan(hipStream_t s);
  template <typename T>
  void apply_t(const double* lam, double* z, double* sigbar, hipStream_t s);
  // near corrections of nq points (charges of molecule t_surf) against the
  // panels of surface e, folded as surface t_surf's interior row sees e
  void charge_near(int e, int t_surf, const double* qx, int64_t nq, NearCSR& out, hipStream_t s);
  // Per-surface (F_coul, F_solv, F_surf) in reduced units.
  std::vector<std::array<double, 3>> surface_energies(const double* x, hipStream_t s);
  std::vector<double> reaction_potential(int e, hipStream_t s);  // densities already set

  // Device copies of what the right-hand side and the energies need from
  // the surfaces' inputs, rebuilt when a surface's version changes.
  struct ChargeData {
    uint64_t version = ~0ull;
    DBuf<double> qx, q, phi;
    DBuf<double> reac_part;   // per-segment partial sums of the reaction potential
    NearCSR qn;           // near corrections charge <- molecule panel
    std::vector<int> cav;                            // the molecule's cavities
    std::vector<std::unique_ptr<NearCSR>> cav_qn;    // near corrections charge <- cavity panel
    double coulomb = 0;   // sum over pairs k < l of q_k q_l / r_kl
  };
  std::vector<std::unique_ptr<ChargeData>> qdata_;
  ChargeData& charges(int e, hipStream_t s);
  std::vector<uint64_t> known_ver_;
  DBuf<double> known_ks_, known_km_, known_half_, rhs_y_;
  void ensure_known(hipStream_t s);
  HBuf<double> hbuf_;          // pinned: Hessenberg rows, g, y, residual estimates
  HBuf<double> hnorm_;         // pinned: norm readback
  hipEvent_t evg_[2];          // GMRES group readbacks

  std::vector<const SurfIn*> surfs_;
  pbt_params prm_;
  double eps_out_, kappa_;
  // Regions: every surface separates the region inside it from the one
  // outside, which is the solvent, the salt-free layer of the Stern surface
  // enclosing it, or (for a cavity) the interior of its molecule (outer_[e]
  // = that surface, or -1 for the solvent); eps_o_[e] is the outside
  // region's permittivity.  forms_[t * ns + s]: how the rows of
  // surface t see surface s (bits 0-1 interior row, 2-3 outside row; 0 not
  // at all, 1 from inside, 2 from outside with the Yukawa kernel, 3 from
  // outside with the Laplace kernel).
  std::vector<int> outer_;
  std::vector<double> eps_o_;
  std::vector<uint8_t> h_forms_;
  DBuf<uint8_t> forms_;
  bool has_nested_ = false;
  bool two_rows(int e) const {
    return surfs_[e]->kind == PBT_MOLECULE || surfs_[e]->kind == PBT_STERN || surfs_[e]->kind == PBT_CAVITY;
  }
  int form(int t, int s) const { return h_forms_[(size_t)t * surfs_.size() + s]; }
  void task_form(int t, int src, int32_t& fused, int16_t& tform) const;
  void build_regions();
  int K_ = 3;
  int64_t n_ = 0, np_ = 0, ns_ = 0;
  std::vector<int64_t> poff_, col_off_, row_off_;
  std::vector<SurfTree> trees_;
  std::vector<int64_t> boff_;

  // geometry (internal order)
  DBuf<double> tri9_, cen_, nrm_, area_, cross2_, src_pos_, src_wa_;
  std::vector<double> h_cen_, h_area_;
  DBuf<double> tgt64_;
  DBuf<float> tgt32_;
  DBuf<double> src64_;
  DBuf<float> src32_;
  DBuf<int32_t> col_phi_, col_psi_, row_int_, row_sol_;
  DBuf<double> dens_scale_, rlap_;
  DBuf<double> sig_, mu_;
  NearCSR near_;
  DBuf<int32_t> panel_surf_;
  DBuf<int32_t> surf_mol_;
  DBuf<double> surf_rhoinv_;
  std::vector<int32_t> h_panel_orig_;  // internal global -> original index within its surface
  std::vector<int32_t> h_pinv_;        // poff + original index -> internal global index
  DBuf<int32_t> u2i_;                  // boundary (original-order) unknown index -> internal one
  DBuf<double> qtab_[6];               // far rule (bary, w), near rule (bary, w), edge rule (t, w)

  // tree (global box numbering)
  int nbox_ = 0;
  DBuf<double> bcen_, brho_;
  DBuf<int32_t> bsbeg_, bsend_, bcbeg_, bcend_, bclist_;
  DBuf<int32_t> leaf_boxes_;
  int nmblocks_ = 0;              // moments blocks: (chunk, coefficient group) pairs
  DBuf<int32_t> mblocks_;
  DBuf<MomChunk> mchunks_;        // source chunks of the boxes whose moments M2P reads
  DBuf<float> msum32_;            // chunk sums of boxes of several chunks
  DBuf<double> msum64_;
  int nmheads_ = 0;               // boxes of several chunks (their first chunks)
  DBuf<MomChunk> mheads_;
  int nmblocks_known_ = 0, nmheads_known_ = 0;   // the same for boxes of charged / potential surfaces
  DBuf<int32_t> mblocks_known_;
  DBuf<MomChunk> mchunks_known_, mheads_known_;
  int nleaf_ = 0;
  // M2M: (box, leaf under it, slot) pairs and (box, first slot, leaves) per
  // box; the same for the boxes of charged / potential surfaces; slots of
  // 2 ncoef(P) shifted moments
  int npair_ = 0, nhead_ = 0, npair_known_ = 0, nhead_known_ = 0;
  int nhead_small_ = 0, nhead_small_known_ = 0;   // heads of at most kM2MSmall leaves (listed first)
  DBuf<int32_t> m2m_pairs_, m2m_heads_, m2m_pairs_known_, m2m_heads_known_;
  DBuf<float> mslot32_;
  DBuf<double> mslot64_;
  DBuf<float> mom32_;
  DBuf<double> mom64_;

  // plan
  Plan plan_;
  DBuf<Task> dp2p_, dm2p_;
  DBuf<Task> dp2p_known_, dm2p_known_;   // the same with tasks of unknown-density sources emptied
  DBuf<int32_t> dranges_, dblist_;
  DBuf<Task> dp2pm_, dm2pm_;
  DBuf<int32_t> dmslot_, dgoff_, dmboxoff_;
  DBuf<ChunkSlots> dchunks_;
  DBuf<int32_t> dchunk_of_;
  DBuf<float> part32_, ppart32_;
  DBuf<double> part64_, ppart64_;

  // Krylov workspace
  int restart_alloc_ = 0;
  DBuf<double> V_, r_, tmp_, hdev_, part_, y_, gm_, nrm_part_;
  DBuf<double> pinv_;         // [np][4] inverse self blocks (right block-Jacobi preconditioner)
  DBuf<double> zbuf_, ztmp_;  // z = M^-1 v of the current step; M^-1 (V y)
  int pdb_ = 1;
  // groups of surfaces = independent systems solved side by side
  int G_ = 1;
  int64_t dense_pairs_ = 0;
  int64_t gmax_ = 0;                 // unknowns of the largest group
  int64_t gpmax_ = 0;                // panels of the largest group
  std::vector<int64_t> gu_;          // [2G] unknown range of each group
  DBuf<int64_t> dgu_;
  DBuf<int64_t> dgp_;                // panel range [2g, 2g + 1) of each group
  std::vector<double> group_rel_;    // last solve: relative residual per group

  hipEvent_t ev_[6];
  hipStream_t s2_ = nullptr;   // far-field stream (moments, M2P), overlaps P2P
  hipEvent_t evm_[3];          // on s2_: moments start, M2P start, M2P end
  int64_t napply_ = 0, nwasted_ = 0;
  int far_mode_ = 0;
  int gs_passes_ = 0;
  bool transpose_ = false;
  bool far_timed_ = false;
  int64_t seg_src_ = 0, seg_box_ = 0, seg_src_used_ = 0, seg_box_used_ = 0;
  void upload_plan(hipStream_t s);
  void check_plan() const;

  // forward interaction lists per (target group, k-th source surface of the
  // group's surfaces in group_surfs_), for the transpose; a target group is
  // a run of at most 64 panels of leaf b of surface e, [g0, g1) globally
  struct LeafInfo { int e; int b; int64_t g0, g1; };
  std::vector<LeafInfo> leaves_;
  std::vector<std::vector<int>> group_surfs_;   // surfaces of each group, in order
  std::vector<std::vector<std::vector<int>>> lp2p_, lm2p_;
  // transpose plan
  bool tplan_ready_ = false;
  int ntp2p_ = 0, ntm2p_ = 0;
  DBuf<Task> dtp2p_, dtm2p_;
  DBuf<int32_t> dtranges_;
  DBuf<ChunkSlots> dtchunks_;
  DBuf<int32_t> dtchunk_of_;
  DBuf<int32_t> dmslot_beg_, dmslot_end_, bparent_, m2mt_boxes_;
  std::vector<std::pair<int, int>> m2mt_levels_;
  NearCSR tnear_;
  DBuf<float> tpart32_, mpart32_, mbar32_, far32_, trec32_;
  DBuf<double> tpart64_, mpart64_, mbar64_, far64_, trec64_;
};

}  // namespace pbt
