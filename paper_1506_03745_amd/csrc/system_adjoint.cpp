// Reaction potential at the charges, the exact transpose of the operator,
// the adjoint right-hand side and the gradient terms of the free energy.
//
// For fixed geometry the discrete system is A u = B p + b0 with p = (q, sigma)
// and every energy of Section 2 is F = 1/2 g(p)^T u + F_coul(q) with
// g = C p + g0 (solvation: C_q = R^T with R the phi_reac evaluator of
// eq. phi_reac_bem; set charge: C_sigma = diag(A) on phi; set potential: the
// constant eps_out phi0 A on dphi/dn).  Hence
//   dF/dp = 1/2 (C^T u + B^T lam) + dF_coul/dp,   A^T lam = g.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "quadrature.h"
#include "system.h"

namespace pbt {

void System::charge_near(int e, int t_surf, const double* qx, int64_t nq, NearCSR& qn, hipStream_t s) {
  const SurfIn& S = *surfs_[e];
  const int64_t p0 = poff_[e];
  NearParams npr{K_, prm_.k_near, prm_.k_self_edge, kappa_, qtab_[0].p, qtab_[1].p, qtab_[2].p, qtab_[3].p,
                 qtab_[4].p, qtab_[5].p};
  DBuf<int32_t> cnt;
  cnt.alloc(nq);
  launch_near_count(nq, qx, S.nt, cen_.p + 3 * p0, cross2_.p + p0, nullptr, nullptr, nullptr,
                    near_f4(prm_.near_factor), cnt.p, s);
  std::vector<int32_t> hc = cnt.download(s);
  std::vector<int64_t> ptr(nq + 1, 0);
  for (int64_t k = 0; k < nq; ++k) ptr[k + 1] = ptr[k] + hc[k];
  qn.nnz = ptr[nq];
  qn.ptr.upload(ptr, s);
  qn.col.alloc(std::max<int64_t>(ptr[nq], 1));
  qn.val.alloc(4 * std::max<int64_t>(ptr[nq], 1));
  launch_near_fill(nq, qx, S.nt, cen_.p + 3 * p0, cross2_.p + p0, nullptr, nullptr, nullptr,
                   near_f4(prm_.near_factor), qn.ptr.p, qn.col.p, s);
  launch_near_values(nq, qx, nullptr, qn.ptr.p, qn.col.p, tri9_.p + 9 * p0, nrm_.p + 3 * p0,
                     area_.p + p0, npr, qn.val.p, s);
  // the charges count as targets of surface t_surf (columns are local to
  // the panels of e)
  launch_fold_near(nq, qn.ptr.p, qn.col.p, nullptr, panel_surf_.p + p0, forms_.p, (int)surfs_.size(),
                   surf_rhoinv_.p, qn.val.p, s, t_surf);
  PBT_HIP(hipStreamSynchronize(s));
}

std::vector<double> System::reaction_potential(int e, hipStream_t s) {
  const SurfIn& S = *surfs_[e];
  const int64_t nq = (int64_t)S.q.size();
  if (nq == 0) return {};
  const int64_t p0 = poff_[e];
  ChargeData& d = charges(e, s);
  launch_reac(nq, d.qx.p, p0 * K_, (p0 + S.nt) * K_, src64_.p, eps_o_[e] / S.eps_in, d.qn.ptr.p, d.qn.col.p,
              d.qn.val.p, sig_.p + p0, mu_.p + p0, d.phi.p, d.reac_part.p, s);
  for (size_t k = 0; k < d.cav.size(); ++k) {
    const int c = d.cav[k];
    const NearCSR& cq = *d.cav_qn[k];
    launch_reac_cavity(nq, d.qx.p, poff_[c] * K_, (poff_[c] + surfs_[c]->nt) * K_, src64_.p, cq.ptr.p, cq.col.p,
                       cq.val.p, sig_.p + poff_[c], mu_.p + poff_[c], d.phi.p, s);
  }
  return d.phi.download(s);
}

// Transposed work lists built from the forward interaction lists:
// reverse P2P tasks = (64 sources of a source leaf) x (segment of target
// ranges that list that leaf), M2P^T tasks = (box, 64-target chunk) grouped
// by box, the near corrections re-indexed by source panel, and the M2M^T
// schedule (levels from the root down).
void System::build_tplan(hipStream_t s) {
  if (tplan_ready_) return;
  const int ns = (int)surfs_.size();
  // (surface, source leaf) -> target ranges (g0, g1, key); key = the forward
  // task's fused flag | its form bits << 1
  std::map<std::pair<int, int>, std::vector<std::tuple<int64_t, int64_t, int>>> lists;
  int64_t work = 0;
  for (size_t li = 0; li < leaves_.size(); ++li) {
    const LeafInfo& L = leaves_[li];
    const std::vector<int>& gsf = group_surfs_[surfs_[L.e]->group];
    for (size_t k2 = 0; k2 < gsf.size(); ++k2)
      for (int b2 : lp2p_[li][k2]) {
        const int e2 = gsf[k2];
        int32_t fu = 0;
        int16_t fm = 0;
        task_form(L.e, e2, fu, fm);
        lists[{e2, b2}].push_back({L.g0, L.g1, fu | (fm << 1)});
        const TreeBox& sb = trees_[e2].boxes[b2];
        work += (L.g1 - L.g0) * (int64_t)((sb.pend - sb.pbeg) * K_ + 63) / 64;
      }
  }
  const int64_t seg_t = std::min<int64_t>(16384, std::max<int64_t>(128, work / 16384));
  std::vector<Task> tasks;
  std::vector<int32_t> ranges;
  std::vector<ChunkSlots> chunks;
  std::vector<int32_t> chunk_of(ns_, 0);
  int slot = 0;
  for (auto& kv : lists) {
    const int e2 = kv.first.first;
    const TreeBox& sb = trees_[e2].boxes[kv.first.second];
    const int64_t s0 = (poff_[e2] + sb.pbeg) * K_, s1 = (poff_[e2] + sb.pend) * K_;
    auto tl = kv.second;
    std::sort(tl.begin(), tl.end(), [](const auto& a, const auto& b) {
      return std::get<2>(a) != std::get<2>(b) ? std::get<2>(a) < std::get<2>(b) : std::get<0>(a) < std::get<0>(b);
    });
    // segments: (lbeg, lend, key), one run per key
    std::vector<std::tuple<int32_t, int32_t, int>> segs;
    for (int f = 0; f < 16; ++f) {
      int64_t acc = 0;
      int32_t start = (int32_t)(ranges.size() / 2);
      for (auto& t : tl) {
        if (std::get<2>(t) != f) continue;
        for (int64_t a = std::get<0>(t); a < std::get<1>(t);) {
          const int64_t b = std::min<int64_t>(std::get<1>(t), a + (seg_t - acc));
          if (!ranges.empty() && (int32_t)(ranges.size() / 2) > start && ranges.back() == a) ranges.back() = (int32_t)b;
          else { ranges.push_back((int32_t)a); ranges.push_back((int32_t)b); }
          acc += b - a;
          a = b;
          if (acc >= seg_t) {
            segs.push_back({start, (int32_t)(ranges.size() / 2), f});
            start = (int32_t)(ranges.size() / 2);
            acc = 0;
          }
        }
      }
      if ((int32_t)(ranges.size() / 2) > start) segs.push_back({start, (int32_t)(ranges.size() / 2), f});
    }
    const double rho = two_rows(e2) ? eps_o_[e2] / surfs_[e2]->eps_in : 0.0;
    for (int64_t c0 = s0; c0 < s1; c0 += 64) {
      ChunkSlots cs{(int32_t)c0, (int32_t)std::min<int64_t>(64, s1 - c0), slot, slot + (int32_t)segs.size()};
      for (int64_t j = c0; j < c0 + cs.tcount; ++j) chunk_of[j] = (int32_t)chunks.size();
      for (size_t si = 0; si < segs.size(); ++si) {
        Task t{};
        t.tbeg = cs.tbeg;
        t.tcount = cs.tcount;
        t.lbeg = std::get<0>(segs[si]);
        t.lend = std::get<1>(segs[si]);
        t.slot = slot + (int)si;
        t.fused = std::get<2>(segs[si]) & 1;
        t.form = (int16_t)(std::get<2>(segs[si]) >> 1);
        t.rho_inv = rho;
        t.rho_inv_f = (float)rho;
        tasks.push_back(t);
      }
      slot += (int)segs.size();
      chunks.push_back(cs);
    }
  }
  // sources that no target lists (cannot happen for a consistent plan) keep chunk 0's slots
  ntp2p_ = (int)tasks.size();
  dtp2p_.upload(tasks.empty() ? std::vector<Task>(1) : tasks, s);
  dtranges_.upload(ranges.empty() ? std::vector<int32_t>{0, 0} : ranges, s);
  dtchunks_.upload(chunks.empty() ? std::vector<ChunkSlots>(1) : chunks, s);
  dtchunk_of_.upload(chunk_of, s);
  tpart32_.alloc((size_t)std::max(slot, 1) * 256);
  tpart64_.alloc((size_t)std::max(slot, 1) * 256);

  // M2P^T tasks grouped by box: per box, the target ranges of the groups
  // that list it, contiguous ranges of one kind merged (the forward groups
  // are runs of 32 targets), in chunks of 64
  std::vector<std::vector<std::tuple<int, int64_t, int64_t>>> ranges_of(nbox_);   // (key, t0, t1)
  for (size_t li = 0; li < leaves_.size(); ++li) {
    const LeafInfo& L = leaves_[li];
    const std::vector<int>& gsf = group_surfs_[surfs_[L.e]->group];
    for (size_t k2 = 0; k2 < gsf.size(); ++k2)
      for (int b : lm2p_[li][k2]) {
        const int e2 = gsf[k2];
        int32_t fu = 0;
        int16_t fm = 0;
        task_form(L.e, e2, fu, fm);
        ranges_of[boff_[e2] + b].push_back({fu | (fm << 1), L.g0, L.g1});
      }
  }
  std::vector<std::vector<Task>> bybox(nbox_);
  for (int gb = 0; gb < nbox_; ++gb) {
    auto& rl = ranges_of[gb];
    std::sort(rl.begin(), rl.end());
    for (size_t k = 0; k < rl.size();) {
      const int key = std::get<0>(rl[k]);
      const int64_t a = std::get<1>(rl[k]);
      int64_t e = std::get<2>(rl[k]);
      size_t q = k + 1;
      while (q < rl.size() && std::get<0>(rl[q]) == key && std::get<1>(rl[q]) == e) e = std::get<2>(rl[q++]);
      for (int64_t t0 = a; t0 < e; t0 += 64) {
        Task t{};
        t.tbeg = (int32_t)t0;
        t.tcount = (int32_t)std::min<int64_t>(64, e - t0);
        t.lbeg = gb;
        t.lend = gb + 1;
        t.fused = key & 1;
        t.form = (int16_t)(key >> 1);
        bybox[gb].push_back(t);
      }
      k = q;
    }
  }
  std::vector<Task> mt;
  std::vector<int32_t> mb(nbox_), me(nbox_);
  for (int b = 0; b < nbox_; ++b) {
    mb[b] = (int32_t)mt.size();
    for (Task t : bybox[b]) {
      t.slot = (int32_t)mt.size();
      mt.push_back(t);
    }
    me[b] = (int32_t)mt.size();
  }
  ntm2p_ = (int)mt.size();
  dtm2p_.upload(mt.empty() ? std::vector<Task>(1) : mt, s);
  dmslot_beg_.upload(mb.empty() ? std::vector<int32_t>(1) : mb, s);
  dmslot_end_.upload(me.empty() ? std::vector<int32_t>(1) : me, s);
  const int NC = ncoef(prm_.taylor_p);
  if (ntm2p_ > 0) {
    mpart32_.alloc((size_t)ntm2p_ * 2 * NC);
    mpart64_.alloc((size_t)ntm2p_ * 2 * NC);
    mbar32_.alloc((size_t)nbox_ * 2 * NC);
    mbar64_.alloc((size_t)nbox_ * 2 * NC);
    far32_.alloc((size_t)ns_ * 4);
    far64_.alloc((size_t)ns_ * 4);
  }
  // parents and M2M^T levels (children of each level, from the top)
  std::vector<int32_t> par(nbox_, -1);
  int maxlev = 0;
  for (int e = 0; e < ns; ++e)
    for (size_t b = 0; b < trees_[e].boxes.size(); ++b) {
      const TreeBox& tb = trees_[e].boxes[b];
      if (tb.parent >= 0) par[boff_[e] + b] = (int32_t)(boff_[e] + tb.parent);
      maxlev = std::max(maxlev, tb.level);
    }
  std::vector<std::vector<int32_t>> bylev(maxlev + 1);
  for (int e = 0; e < ns; ++e)
    for (size_t b = 0; b < trees_[e].boxes.size(); ++b)
      if (trees_[e].boxes[b].parent >= 0) bylev[trees_[e].boxes[b].level].push_back((int32_t)(boff_[e] + b));
  std::vector<int32_t> lb;
  m2mt_levels_.clear();
  for (int lv = 1; lv <= maxlev; ++lv) {
    if (bylev[lv].empty()) continue;
    m2mt_levels_.push_back({(int)lb.size(), (int)bylev[lv].size()});
    lb.insert(lb.end(), bylev[lv].begin(), bylev[lv].end());
  }
  if (lb.empty()) lb.push_back(0);
  m2mt_boxes_.upload(lb, s);
  bparent_.upload(par.empty() ? std::vector<int32_t>(1, 0) : par, s);

  // near corrections by source panel
  {
    std::vector<int64_t> ptr = near_.ptr.download(s);
    std::vector<int32_t> col = near_.col.download(s);
    std::vector<double> val = near_.val.download(s);
    std::vector<int64_t> tp(np_ + 1, 0);
    for (int64_t e = 0; e < near_.nnz; ++e) ++tp[col[e] + 1];
    for (int64_t p = 0; p < np_; ++p) tp[p + 1] += tp[p];
    std::vector<int32_t> trow(std::max<int64_t>(near_.nnz, 1));
    std::vector<double> tv(4 * std::max<int64_t>(near_.nnz, 1));
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < np_; ++i)
      for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int64_t d = fill[col[e]]++;
        trow[d] = (int32_t)i;
        for (int k = 0; k < 4; ++k) tv[4 * d + k] = val[4 * e + k];
      }
    tnear_.nnz = near_.nnz;
    tnear_.ptr.upload(tp, s);
    tnear_.col.upload(trow, s);
    tnear_.val.upload(tv, s);
  }
  trec32_.alloc((size_t)np_ * 8);
  trec64_.alloc((size_t)np_ * 8);
  PBT_HIP(hipStreamSynchronize(s));
  tplan_ready_ = true;
}

template <typename T>
void System::apply_t(const double* lam, double* z, double* sigbar, hipStream_t s) {
  const bool f32 = std::is_same<T, float>::value;
  T* src = f32 ? (T*)src32_.p : (T*)src64_.p;
  T* trec = f32 ? (T*)trec32_.p : (T*)trec64_.p;
  T* tpart = f32 ? (T*)tpart32_.p : (T*)tpart64_.p;
  ++napply_;
  pairs_done_ += dense_pairs_;
  PBT_HIP(hipEventRecord(ev_[0], s));
  launch_adj_targets<T>(np_, cen_.p, row_int_.p, row_sol_.p, lam, trec, s);
  PBT_HIP(hipEventRecord(ev_[1], s));
  PBT_HIP(hipEventRecord(ev_[2], s));
  const bool guard = K_ == 1 || K_ == 4 || K_ == 7;
  launch_p2p_t<T>(dtp2p_.p, ntp2p_, dtranges_.p, src, trec, (T)kappa_, guard, tpart, s);
  PBT_HIP(hipEventRecord(ev_[3], s));
  T* far = nullptr;
  if (ntm2p_ > 0) {
    T* mpart = f32 ? (T*)mpart32_.p : (T*)mpart64_.p;
    T* mbar = f32 ? (T*)mbar32_.p : (T*)mbar64_.p;
    far = f32 ? (T*)far32_.p : (T*)far64_.p;
    const int P = prm_.taylor_p;
    launch_m2p_t<T>(P, dtm2p_.p, ntm2p_, trec, bcen_.p, (T)kappa_, mpart, s);
    launch_mbar_reduce<T>(nbox_, P, dmslot_beg_.p, dmslot_end_.p, mpart, mbar, s);
    for (auto lv : m2mt_levels_) launch_m2m_t<T>(P, lv.second, m2mt_boxes_.p + lv.first, bparent_.p, bcen_.p, mbar, s);
    BoxDev bd{bcen_.p, bsbeg_.p, bsend_.p, bcbeg_.p, bcend_.p, bclist_.p, brho_.p};
    launch_l2p_t<T>(P, nleaf_, leaf_boxes_.p, bd, src, mbar, far, s);
  }
  PBT_HIP(hipEventRecord(ev_[4], s));
  AdjCombineArgs a{};
  a.np = np_;
  a.K = K_;
  a.chunks = dtchunks_.p;
  a.chunk_of = dtchunk_of_.p;
  a.wa = src_wa_.p;
  a.nrm = nrm_.p;
  a.tptr = tnear_.ptr.p;
  a.trow = tnear_.col.p;
  a.tval = tnear_.val.p;
  a.lam = lam;
  a.maps = PanelMaps{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
  launch_combine_t<T>(a, tpart, far, z, sigbar, s);
  PBT_HIP(hipEventRecord(ev_[5], s));
}

void System::matvec_t(const double* lam, double* z, bool fp32, double* sigbar, hipStream_t s) {
  build_tplan(s);
  if (fp32) apply_t<float>(lam, z, sigbar, s);
  else apply_t<double>(lam, z, sigbar, s);
}

void System::adjoint_rhs(const double* x, double* g, hipStream_t s) {
  const int ns = (int)surfs_.size();
  PBT_HIP(hipMemsetAsync(g, 0, n_ * sizeof(double), s));
  PanelMaps m{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
  // R^T q over the panels of surface e2 (the molecule itself, or one of its
  // cavities seen from outside: far part with the opposite sign and unit
  // single-layer factor), plus the near part qn
  auto rt_q = [&](const SurfIn& S, ChargeData& d, int e2, const NearCSR& qn, double rho, double dsign) {
    const int64_t nq = (int64_t)S.q.size(), p0 = poff_[e2], nt = surfs_[e2]->nt;
    DBuf<double> far;
    far.alloc((size_t)nt * K_ * 4);
    launch_reac_t(p0 * K_, (p0 + nt) * K_, src64_.p, nq, d.qx.p, d.q.p, rho, far.p, dsign, s);
    // near part: phi_reac holds -(corrections), so d(q . phi_reac)/d(sigma, mu) = -q (c_s, c_m)
    std::vector<int64_t> ptr = qn.ptr.download(s);
    std::vector<int32_t> col = qn.col.download(s);
    std::vector<double> val = qn.val.download(s);
    std::vector<double> asg(nt, 0.0), amu(nt, 0.0);
    for (int64_t k = 0; k < nq; ++k)
      for (int64_t e3 = ptr[k]; e3 < ptr[k + 1]; ++e3) {
        asg[col[e3]] -= S.q[k] * val[4 * e3];
        amu[col[e3]] -= S.q[k] * val[4 * e3 + 1];
      }
    DBuf<double> das, dam;
    das.upload(asg, s);
    dam.upload(amu, s);
    AdjCombineArgs a{};
    a.np = nt;
    a.K = K_;
    a.wa = src_wa_.p + p0 * K_;
    a.nrm = nrm_.p + 3 * p0;
    a.add_sig = das.p;
    a.add_mu = dam.p;
    a.maps = PanelMaps{col_phi_.p + p0, col_psi_.p + p0, row_int_.p + p0, row_sol_.p + p0, dens_scale_.p + p0};
    launch_combine_t<double>(a, nullptr, far.p, g, nullptr, s);
    PBT_HIP(hipStreamSynchronize(s));
  };
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind != PBT_MOLECULE || S.q.empty()) continue;
    ChargeData& d = charges(e, s);
    rt_q(S, d, e, d.qn, eps_o_[e] / S.eps_in, 1.0);
    for (size_t k = 0; k < d.cav.size(); ++k) rt_q(S, d, d.cav[k], *d.cav_qn[k], -1.0, -1.0);
  }
  (void)m;
  std::vector<double> hg(n_);
  PBT_HIP(hipMemcpyAsync(hg.data(), g, n_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PBT_HIP(hipStreamSynchronize(s));
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind != PBT_CHARGED && S.kind != PBT_POTENTIAL) continue;
    for (int64_t li = 0; li < S.nt; ++li) {
      const int64_t gi = poff_[e] + li;
      const int32_t o = h_panel_orig_[gi];
      if (S.kind == PBT_CHARGED) hg[col_off_[e] + li] += S.bc[o] * kSigmaSI * h_area_[gi];
      else hg[col_off_[e] + li] += eps_out_ * (S.bc[o] / kVoltPerUnit) * h_area_[gi];
    }
  }
  PBT_HIP(hipMemcpyAsync(g, hg.data(), n_ * sizeof(double), hipMemcpyHostToDevice, s));
  PBT_HIP(hipStreamSynchronize(s));
}

void System::gradient_terms(const double* x, const double* lam, std::vector<std::vector<double>>& dq,
                            std::vector<std::vector<double>>& dsig, hipStream_t s) {
  const int ns = (int)surfs_.size();
  dq.assign(ns, {});
  dsig.assign(ns, {});
  DBuf<double> z, sbar;
  z.alloc(n_);
  sbar.alloc(np_);
  matvec_t(lam, z.p, false, sbar.p, s);
  std::vector<double> hsb = sbar.download(s);
  std::vector<double> xh(n_);
  PBT_HIP(hipMemcpyAsync(xh.data(), x, n_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PanelMaps m{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
  launch_densities(np_, m, x, sig_.p, mu_.p, s);
  launch_strengths<double>(ns_, K_, sig_.p, mu_.p, src_wa_.p, nrm_.p, rlap_.p, src64_.p, s);
  PBT_HIP(hipStreamSynchronize(s));
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind == PBT_MOLECULE) {
      const int64_t nq = (int64_t)S.q.size();
      if (nq == 0) continue;
      std::vector<double> phi = reaction_potential(e, s);
      DBuf<double> qx, bt;
      qx.upload(S.qxyz, s);
      bt.alloc(nq);
      launch_coulomb_t(nq, qx.p, S.nt, cen_.p + 3 * poff_[e], row_int_.p + poff_[e], lam, 1.0 / S.eps_in,
                       bt.p, s);
      std::vector<double> hb = bt.download(s);
      // the charges' Coulomb sum is also on the outside rows of the cavities
      for (int c = 0; c < ns; ++c) {
        if (surfs_[c]->kind != PBT_CAVITY || outer_[c] != e) continue;
        launch_coulomb_t(nq, qx.p, surfs_[c]->nt, cen_.p + 3 * poff_[c], row_sol_.p + poff_[c], lam,
                         1.0 / S.eps_in, bt.p, s);
        const std::vector<double> hc = bt.download(s);
        for (int64_t k = 0; k < nq; ++k) hb[k] += hc[k];
      }
      dq[e].resize(nq);
      for (int64_t k = 0; k < nq; ++k) dq[e][k] = 0.5 * (phi[k] + hb[k]);
    } else if (S.kind == PBT_CHARGED) {
      dsig[e].resize(S.nt);
      for (int64_t li = 0; li < S.nt; ++li) {
        const int64_t gi = poff_[e] + li;
        const int32_t o = h_panel_orig_[gi];
        dsig[e][o] = 0.5 * (h_area_[gi] * xh[col_off_[e] + li] + hsb[gi] / eps_out_);
      }
    }
  }
}

}  // namespace pbt
