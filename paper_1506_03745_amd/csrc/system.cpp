// Boundary-element system for one set of enabled surfaces (Sections 2-3).
//
// Unknowns per surface: a molecule has [phi, dphi/dn inside], a charged
// surface [phi], a potential surface [dphi/dn] (eq. matrix_phi /
// eq. matrix_dphi generalised to any number of surfaces).  Rows: a molecule's
// interior row (first line of eq. integral_eq) then every surface's solvent
// row (second and third lines).
#include "system.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <map>

#include "parallel.h"
#include "quadrature.h"

namespace pbt {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Host staging arrays of the set-up (triangles, Gauss points), kept per
// thread and reused by later set-ups: for the largest systems, mapping a few
// hundred MB of fresh pages costs more than filling them.
double* host_stage(int which, size_t n) {
  thread_local std::vector<double> buf[2];
  if (buf[which].size() < n) buf[which].resize(n);
  return buf[which].data();
}

// Wall time of the set-up phases, printed to stderr when PBT_SETUP_TIMES is
// set in the environment (the stream is drained at each mark so that device
// work is charged to its own phase).
struct PhaseClock {
  bool on = std::getenv("PBT_SETUP_TIMES") != nullptr;
  double t = now_s();
  void mark(const char* what, hipStream_t s) {
    if (!on) return;
    PBT_HIP(hipStreamSynchronize(s));
    mark_host(what);
  }
  void mark_host(const char* what) {
    if (!on) return;
    const double u = now_s();
    std::fprintf(stderr, "[setup] %-16s %8.2f ms\n", what, 1e3 * (u - t));
    t = u;
  }
};

}  // namespace

System::System(const std::vector<const SurfIn*>& surfs, const pbt_params& prm, double eps_out,
               double kappa, hipStream_t stream)
    : surfs_(surfs), prm_(prm), eps_out_(eps_out), kappa_(kappa), K_(prm.k_far) {
  for (auto& e : ev_) PBT_HIP(hipEventCreate(&e));
  for (auto& e : evm_) PBT_HIP(hipEventCreate(&e));
  for (auto& e : evg_) PBT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  PBT_HIP(hipStreamCreate(&s2_));
  build(stream);
}

System::~System() {
  if (s2_) (void)hipStreamSynchronize(s2_);
  for (auto& e : pev_) (void)hipEventDestroy(e);
  for (auto& e : ev_) (void)hipEventDestroy(e);
  for (auto& e : evm_) (void)hipEventDestroy(e);
  for (auto& e : evg_) (void)hipEventDestroy(e);
  if (s2_) (void)hipStreamDestroy(s2_);
}

int System::local_index(int surface_id) const { return surface_id; }

// Regions and forms (Section 2's representation formula per region, with
// the extra interfaces of a Stern layer: a salt-free layer of its own
// permittivity between one molecule and the solvent).  The row of region R
// on a surface sees the surface whose inside is R from inside and every
// surface with R outside it from outside, with R's kernel.
void System::build_regions() {
  const int ns = (int)surfs_.size();
  outer_.assign(ns, -1);
  has_nested_ = false;
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind != PBT_STERN && S.kind != PBT_CAVITY) continue;
    has_nested_ = true;
    int par = -1;
    for (int k = 0; k < ns; ++k)
      if (surfs_[k] == S.parent) par = k;
    if (par < 0) throw Error(PBT_E_STATE, "a Stern surface or cavity is enabled without its molecule");
    if (surfs_[par]->group != S.group)
      throw Error(PBT_E_STATE, "a Stern surface or cavity and its molecule in different groups");
    if (S.kind == PBT_CAVITY) {
      outer_[e] = par;   // the cavity lies in the molecule's interior
      continue;
    }
    if (outer_[par] >= 0) throw Error(PBT_E_STATE, "a molecule with two Stern surfaces");
    outer_[par] = e;
  }
  eps_o_.assign(ns, eps_out_);
  for (int e = 0; e < ns; ++e)
    if (outer_[e] >= 0) eps_o_[e] = surfs_[outer_[e]]->eps_in;
  // forms: the interior row of t is the region t; its outside row the region
  // outer_[t] (-1: the solvent, Yukawa; a Stern surface's layer or a
  // molecule's interior: Laplace)
  h_forms_.assign((size_t)ns * ns, 0);
  // (the solvent's form is the Yukawa one also when kappa = 0: the kernels
  // then take their kappa = 0 path themselves)
  auto seen = [&](int R, int src) -> int {
    if (R >= 0 && R == src) return 1;          // R is the inside of src
    if (outer_[src] == R) return R < 0 ? 2 : 3;  // src seen from outside
    return 0;
  };
  for (int t = 0; t < ns; ++t)
    for (int src = 0; src < ns; ++src) {
      if (surfs_[t]->group != surfs_[src]->group) continue;
      const int fi = two_rows(t) ? seen(t, src) : 0;
      const int fo = seen(outer_[t], src);
      h_forms_[(size_t)t * ns + src] = (uint8_t)(fi | (fo << 2));
    }
}

// The task flags for targets on surface t and sources on surface src: the
// usual pair is (inside, Yukawa) = fused; the others occur with nested
// interfaces.
void System::task_form(int t, int src, int32_t& fused, int16_t& tform) const {
  const int f = form(t, src), fi = f & 3, fo = f >> 2;
  fused = fi == 1 ? 1 : 0;
  tform = 0;
  if (fi == 1 && fo == 3) tform = kFormKz;                          // seen from inside and from outside in a layer
  else if (fi == 0 && fo == 1) {                                    // seen from inside by the outside row
    fused = 1;
    tform = kFormKz | kFormDropOut | kFormSwap;
  } else if (fi == 3 && fo == 0) tform = kFormKz | kFormSwap;       // seen from outside by the interior row
  else if (!((fi == 1 && fo == 2) || (fi == 0 && fo == 2) || (fi == 0 && fo == 3)))
    throw Error(PBT_E_STATE, "unsupported arrangement of surfaces");
  if (fi == 0 && fo == 3) tform = kFormKz;                          // seen from outside in a layer only
}

void System::build(hipStream_t s) {
  const int ns = (int)surfs_.size();
  PhaseClock clk;
  build_regions();
  // ---- offsets, trees ------------------------------------------------------
  poff_.assign(ns + 1, 0);
  col_off_.assign(ns + 1, 0);
  row_off_.assign(ns + 1, 0);
  trees_.resize(ns);
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    const int64_t w = two_rows(e) ? 2 * S.nt : S.nt;
    poff_[e + 1] = poff_[e] + S.nt;
    col_off_[e + 1] = col_off_[e] + w;
    row_off_[e + 1] = row_off_[e] + w;
  }
  parallel_for(ns, [&](int64_t e) {
    const SurfIn& S = *surfs_[e];
    std::vector<double> hc(3 * S.nt);
    for (int64_t i = 0; i < S.nt; ++i)
      for (int d = 0; d < 3; ++d) {
        const int32_t* t = &S.tri[3 * i];
        hc[3 * i + d] = (S.xyz[3 * t[0] + d] + S.xyz[3 * t[1] + d] + S.xyz[3 * t[2] + d]) / 3.0;
      }
    trees_[e] = build_tree(hc.data(), S.nt, prm_.treecode ? prm_.ncrit : (int)std::max<int64_t>(S.nt, 1));
  });
  np_ = poff_[ns];
  n_ = col_off_[ns];
  ns_ = np_ * K_;
  clk.mark("trees", s);
  {
    std::map<int, int64_t> gp;   // panels per group
    for (int e = 0; e < ns; ++e) gp[surfs_[e]->group] += surfs_[e]->nt;
    std::map<int, int64_t> gk;   // Gauss points with known densities per group
    for (int e = 0; e < ns; ++e)
      if (surfs_[e]->kind == PBT_CHARGED || surfs_[e]->kind == PBT_POTENTIAL) gk[surfs_[e]->group] += surfs_[e]->nt * K_;
    dense_pairs_ = 0;
    known_pairs_ = 0;
    for (const auto& kv : gp) {
      dense_pairs_ += kv.second * kv.second * K_;
      known_pairs_ += kv.second * gk[kv.first];
    }
  }

  // ---- internal-order triangles ---------------------------------------------
  clk.mark("counts", s);
  std::vector<double> bf, wf, bn, wn, gt, gw;
  if (!triangle_rule(prm_.k_far, bf, wf)) throw Error(1, "k_far must be 1, 3, 4 or 7");
  if (!triangle_rule(prm_.k_near, bn, wn)) throw Error(1, "k_near must be 19 (or 1, 3, 4, 7)");
  gauss_legendre01(prm_.k_self_edge, gt, gw);
  // Host copies of the centroids, areas and Gauss points, in the same
  // sequence of correctly rounded operations as the device's geometry
  // kernels (so they agree bit for bit), formed while the triangles are
  // gathered instead of read back.
  double* tri9 = host_stage(0, 9 * (size_t)np_);
  double* hsrc = host_stage(1, 3 * (size_t)ns_);
  h_cen_.resize(3 * np_);
  h_area_.resize(np_);
  const double third = 1.0 / 3.0;
  auto host_geometry = [&](int64_t g) {
    const double* v = &tri9[9 * g];
    const double e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
    const double e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
    const double cx = e1y * e2z - e1z * e2y;
    const double cy = e1z * e2x - e1x * e2z;
    const double cz = e1x * e2y - e1y * e2x;
    h_area_[g] = 0.5 * std::sqrt((cx * cx + cy * cy) + cz * cz);
    for (int d = 0; d < 3; ++d) h_cen_[3 * g + d] = ((v[d] + v[3 + d]) + v[6 + d]) * third;
    for (int q = 0; q < K_; ++q) {
      const double b0 = bf[3 * q], b1 = bf[3 * q + 1], b2 = bf[3 * q + 2];
      double* p = &hsrc[3 * (g * K_ + q)];
      if (b0 == third && b1 == third && b2 == third)
        for (int d = 0; d < 3; ++d) p[d] = ((v[d] + v[3 + d]) + v[6 + d]) * third;
      else
        for (int d = 0; d < 3; ++d) p[d] = (b0 * v[d] + b1 * v[3 + d]) + b2 * v[6 + d];
    }
  };
  // A copy of a surface that the groups share unmoved (a batch's plate: the
  // same vertices, triangles and octree as group 0's copy) takes its
  // triangles from group 0's on the device and its host geometry from
  // group 0's on the host, instead of gathering them again.
  std::vector<int> twin(ns, -1);
  {
    std::map<int, int> first;   // shared id -> group 0's surface
    for (int e = 0; e < ns; ++e)
      if (surfs_[e]->shared >= 0 && surfs_[e]->group == 0) first.emplace(surfs_[e]->shared, e);
    parallel_for(ns, [&](int64_t e) {
      const SurfIn& S = *surfs_[e];
      if (S.shared < 0 || S.group == 0) return;
      auto it = first.find(S.shared);
      if (it == first.end()) return;
      const SurfIn& S0 = *surfs_[it->second];
      if (S.nt == S0.nt && S.xyz == S0.xyz && S.tri == S0.tri && trees_[e].perm == trees_[it->second].perm)
        twin[e] = it->second;
    });
  }
  h_panel_orig_.resize(np_);
  std::vector<int32_t> col_phi(np_), col_psi(np_), row_int(np_), row_sol(np_), psurf(np_);
  std::vector<double> dscale(np_);
  parallel_for(ns, [&](int64_t e) {
    const SurfIn& S = *surfs_[e];
    for (int64_t li = 0; li < S.nt; ++li) {
      const int64_t g = poff_[e] + li;
      const int32_t o = trees_[e].perm[li];
      h_panel_orig_[g] = o;
      if (twin[e] < 0) {
        for (int v = 0; v < 3; ++v)
          for (int d = 0; d < 3; ++d) tri9[9 * g + 3 * v + d] = S.xyz[3 * S.tri[3 * o + v] + d];
        host_geometry(g);
      }
      psurf[g] = e;
      switch (S.kind) {
        case PBT_MOLECULE:
        case PBT_STERN:
        case PBT_CAVITY:
          col_phi[g] = (int32_t)(col_off_[e] + li);
          col_psi[g] = (int32_t)(col_off_[e] + S.nt + li);
          row_int[g] = (int32_t)(row_off_[e] + li);
          row_sol[g] = (int32_t)(row_off_[e] + S.nt + li);
          dscale[g] = S.eps_in / eps_o_[e];
          break;
        case PBT_CHARGED:
          col_phi[g] = (int32_t)(col_off_[e] + li);
          col_psi[g] = -1;
          row_int[g] = -1;
          row_sol[g] = (int32_t)(row_off_[e] + li);
          dscale[g] = 1.0;
          break;
        default:
          col_phi[g] = -1;
          col_psi[g] = (int32_t)(col_off_[e] + li);
          row_int[g] = -1;
          row_sol[g] = (int32_t)(row_off_[e] + li);
          dscale[g] = 1.0;
      }
    }
  });
  // the twins' host geometry from group 0's copies (formed above)
  parallel_for(ns, [&](int64_t e) {
    const int e0 = twin[e];
    if (e0 < 0) return;
    const int64_t nt = surfs_[e]->nt, g = poff_[e], g0 = poff_[e0];
    std::memcpy(&h_cen_[3 * g], &h_cen_[3 * g0], 3 * nt * sizeof(double));
    std::memcpy(&h_area_[g], &h_area_[g0], nt * sizeof(double));
    std::memcpy(&hsrc[3 * g * K_], &hsrc[3 * g0 * K_], 3 * nt * K_ * sizeof(double));
  });
  clk.mark("tri9", s);
  {
    // The unknowns (and rows) of a surface follow its panels' internal order;
    // the boundary's layout follows the original order: u2i maps a boundary
    // index to the internal one.
    std::vector<int32_t> u2i(n_);
    h_pinv_.assign(np_, 0);
    for (int64_t g = 0; g < np_; ++g) {
      const int e = psurf[g];
      const int64_t li = g - poff_[e], o = h_panel_orig_[g], nt = surfs_[e]->nt;
      h_pinv_[poff_[e] + o] = (int32_t)g;
      u2i[col_off_[e] + o] = (int32_t)(col_off_[e] + li);
      if (col_off_[e + 1] - col_off_[e] == 2 * nt) u2i[col_off_[e] + nt + o] = (int32_t)(col_off_[e] + nt + li);
    }
    u2i_.upload(u2i, s);
  }
  // triangles: each surface's own from the host, a twin's copied from group
  // 0's on the device
  tri9_.alloc(9 * (size_t)np_);
  for (int e = 0; e < ns; ++e)
    if (twin[e] < 0 && surfs_[e]->nt > 0)
      PBT_HIP(hipMemcpyAsync(tri9_.p + 9 * poff_[e], &tri9[9 * poff_[e]], 9 * surfs_[e]->nt * sizeof(double),
                             hipMemcpyHostToDevice, s));
  for (int e = 0; e < ns; ++e)
    if (twin[e] >= 0 && surfs_[e]->nt > 0)
      PBT_HIP(hipMemcpyAsync(tri9_.p + 9 * poff_[e], tri9_.p + 9 * poff_[twin[e]], 9 * surfs_[e]->nt * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  PBT_HIP(hipStreamSynchronize(s));
  col_phi_.upload(col_phi, s);
  col_psi_.upload(col_psi, s);
  row_int_.upload(row_int, s);
  row_sol_.upload(row_sol, s);
  dens_scale_.upload(dscale, s);
  {
    std::vector<double> rl(np_, 0.0);
    for (int64_t g = 0; g < np_; ++g)
      if (two_rows(psurf[g])) rl[g] = -eps_o_[psurf[g]] / surfs_[psurf[g]]->eps_in;
    rlap_.upload(rl, s);
  }
  panel_surf_.upload(psurf, s);
  std::vector<int32_t> smol(ns);
  std::vector<double> srho(ns);
  for (int e = 0; e < ns; ++e) {
    smol[e] = two_rows(e);
    srho[e] = smol[e] ? eps_o_[e] / surfs_[e]->eps_in : 0.0;
  }
  surf_mol_.upload(smol, s);
  surf_rhoinv_.upload(srho, s);
  forms_.upload(h_forms_, s);
  clk.mark("maps upload", s);

  // ---- geometry and sources on the device ------------------------------------
  cen_.alloc(3 * np_);
  nrm_.alloc(3 * np_);
  area_.alloc(np_);
  cross2_.alloc(np_);
  launch_panel_geometry(np_, tri9_.p, cen_.p, nrm_.p, area_.p, cross2_.p, s);
  // the rules on the device, kept for later near-correction tables
  qtab_[0].upload(bf, s);
  qtab_[1].upload(wf, s);
  qtab_[2].upload(bn, s);
  qtab_[3].upload(wn, s);
  qtab_[4].upload(gt, s);
  qtab_[5].upload(gw, s);
  DBuf<double>&dbf = qtab_[0], &dwf = qtab_[1], &dbn = qtab_[2], &dwn = qtab_[3], &dgt = qtab_[4], &dgw = qtab_[5];
  src_pos_.alloc(3 * ns_);
  src_wa_.alloc(ns_);
  launch_sources(np_, K_, tri9_.p, nrm_.p, area_.p, dbf.p, dwf.p, src_pos_.p, src_wa_.p, s);
  clk.mark("geom kernels", s);
  if (std::getenv("PBT_CHECK_HOST_GEOMETRY")) {
    // the host's centroids, areas and Gauss points against the device's
    const std::vector<double> dc = cen_.download(s), da = area_.download(s), ds = src_pos_.download(s);
    if (std::memcmp(dc.data(), h_cen_.data(), dc.size() * sizeof(double)) != 0 ||
        std::memcmp(da.data(), h_area_.data(), da.size() * sizeof(double)) != 0 ||
        std::memcmp(ds.data(), hsrc, ds.size() * sizeof(double)) != 0)
      throw Error(PBT_E_STATE, "host and device panel geometry differ");
  }
  tgt64_.alloc(4 * np_);
  tgt32_.alloc(4 * np_);
  src64_.alloc(kSrcStride * ns_);
  src32_.alloc(kSrcStride * ns_);
  launch_pack_points(np_, ns_, cen_.p, src_pos_.p, tgt64_.p, tgt32_.p, src64_.p, src32_.p, s);
  sig_.alloc(np_);
  mu_.alloc(np_);

  clk.mark("geometry", s);
  // ---- tree geometry (global box numbering) --------------------------------
  boff_.assign(ns + 1, 0);
  parallel_for(ns, [&](int64_t e) {
    const int64_t p0 = poff_[e];
    tree_geometry(trees_[e], &h_cen_[3 * p0], &hsrc[3 * p0 * K_], K_);
  });
  for (int e = 0; e < ns; ++e) boff_[e + 1] = boff_[e] + (int64_t)trees_[e].boxes.size();
  nbox_ = (int)boff_[ns];
  {
    std::vector<double> bc(3 * nbox_), brho(nbox_);
    std::vector<int32_t> sb(nbox_), se(nbox_), cb(nbox_), ce(nbox_), cl, leaves;
    for (int e = 0; e < ns; ++e) {
      const SurfTree& T = trees_[e];
      for (size_t bi = 0; bi < T.boxes.size(); ++bi) {
        const TreeBox& b = T.boxes[bi];
        const int g = (int)(boff_[e] + bi);
        for (int d = 0; d < 3; ++d) bc[3 * g + d] = b.c[d];
        brho[g] = two_rows(e) ? eps_o_[e] / surfs_[e]->eps_in : 0.0;
        sb[g] = (int32_t)((poff_[e] + b.pbeg) * K_);
        se[g] = (int32_t)((poff_[e] + b.pend) * K_);
        cb[g] = (int32_t)cl.size();
        if (b.child_end - b.child_beg > 8) throw Error(PBT_E_STATE, "an octree box with more than 8 children");
        for (int k = b.child_beg; k < b.child_end; ++k) cl.push_back((int32_t)(boff_[e] + T.child_list[k]));
        ce[g] = (int32_t)cl.size();
        if (b.leaf) leaves.push_back(g);
      }
    }
    if (cl.empty()) cl.push_back(0);
    bcen_.upload(bc, s);
    brho_.upload(brho, s);
    bsbeg_.upload(sb, s);
    bsend_.upload(se, s);
    bcbeg_.upload(cb, s);
    bcend_.upload(ce, s);
    bclist_.upload(cl, s);
    leaf_boxes_.upload(leaves, s);
    nleaf_ = (int)leaves.size();
  }
  clk.mark("tree geometry", s);
  // ---- near / self corrections for the collocation points ------------------
  {
    // candidate panel ranges per target leaf: boxes of the same group whose
    // centroid sphere comes within 2 L_max (with a rounding margin) of the
    // leaf's; no panel outside them can pass the near test
    std::vector<int32_t> tleaf(np_, 0);
    std::vector<int64_t> lptr{0}, lrange;
    std::vector<double> lmax(ns, 0.0);
    for (int e = 0; e < ns; ++e)
      for (int64_t li = 0; li < surfs_[e]->nt; ++li)
        lmax[e] = std::max(lmax[e], prm_.near_factor * std::sqrt(2.0 * h_area_[poff_[e] + li]));
    struct TL { int e; const TreeBox* T; };
    std::vector<TL> tls;
    std::vector<int64_t> tls_first(ns + 1, 0);   // first target leaf of each surface
    for (int e = 0; e < ns; ++e) {
      tls_first[e] = (int64_t)tls.size();
      for (const TreeBox& T : trees_[e].boxes)
        if (T.leaf) tls.push_back({e, &T});
    }
    tls_first[ns] = (int64_t)tls.size();
    // A leaf of a shared surface's copy (twin) takes the near rows of group
    // 0's leaf, shifted by the copy's panel offset, when nothing of its own
    // group but its own surface comes near it and group 0's leaf's near
    // panels all lie on group 0's copy (its own surface is not searched).
    const bool replicate = !std::getenv("PBT_NO_SHARED");
    std::vector<int64_t> mleaf(tls.size(), -1);
    if (replicate)
      for (size_t k = 0; k < tls.size(); ++k) {
        const int e = tls[k].e;
        if (twin[e] >= 0) mleaf[k] = tls_first[twin[e]] + ((int64_t)k - tls_first[e]);
      }
    // candidate ranges of leaf k on the surfaces of its group (only >= 0:
    // that surface alone; skip >= 0: all but that surface)
    auto search = [&](int64_t k, int only, int skip, std::vector<std::pair<int64_t, int64_t>>& rg) {
      const int e = tls[k].e;
      const TreeBox& T = *tls[k].T;
      for (int e2 = 0; e2 < ns; ++e2) {
        if (surfs_[e2]->group != surfs_[e]->group || (only >= 0 && e2 != only) || e2 == skip) continue;
        const SurfTree& S2 = trees_[e2];
        std::vector<int> stack{0};
        while (!stack.empty()) {
          const TreeBox& B = S2.boxes[stack.back()];
          stack.pop_back();
          const double dx = T.tc[0] - B.tc[0], dy = T.tc[1] - B.tc[1], dz = T.tc[2] - B.tc[2];
          const double reach = (T.tr + B.tr + lmax[e2]) * (1.0 + 1e-9) + 1e-9;
          if (dx * dx + dy * dy + dz * dz >= reach * reach) continue;
          if (B.leaf) rg.push_back({poff_[e2] + B.pbeg, poff_[e2] + B.pend});
          else
            for (int c = B.child_end - 1; c >= B.child_beg; --c) stack.push_back(S2.child_list[c]);
        }
      }
      std::sort(rg.begin(), rg.end());
    };
    std::vector<std::vector<std::pair<int64_t, int64_t>>> cand(tls.size());
    parallel_for((int64_t)tls.size(), [&](int64_t k) {
      const int e = tls[k].e;
      const TreeBox& T = *tls[k].T;
      for (int64_t g = poff_[e] + T.pbeg; g < poff_[e] + T.pend; ++g) tleaf[g] = (int32_t)k;
      search(k, -1, mleaf[k] >= 0 ? e : -1, cand[k]);
    });
    std::vector<int32_t> rep_tgt(np_, -1);
    parallel_for((int64_t)tls.size(), [&](int64_t k) {
      if (mleaf[k] < 0) return;
      const int e = tls[k].e, e0 = twin[e];
      bool ok = cand[k].empty();
      for (const auto& r : cand[mleaf[k]]) ok = ok && r.first >= poff_[e0] && r.second <= poff_[e0 + 1];
      const TreeBox& T = *tls[k].T;
      if (ok) {
        for (int64_t g = poff_[e] + T.pbeg; g < poff_[e] + T.pend; ++g) rep_tgt[g] = (int32_t)(g - poff_[e] + poff_[e0]);
      } else {
        mleaf[k] = -1;
        search(k, e, -1, cand[k]);   // its own surface too
      }
    });
    bool any_rep = false;
    for (int32_t r : rep_tgt) any_rep = any_rep || r >= 0;
    for (const auto& rg : cand) {
      for (const auto& r : rg) {
        if (!lrange.empty() && (int64_t)lrange.size() / 2 > lptr.back() && lrange.back() == r.first)
          lrange.back() = r.second;
        else {
          lrange.push_back(r.first);
          lrange.push_back(r.second);
        }
      }
      lptr.push_back((int64_t)lrange.size() / 2);
    }
    if (lrange.empty()) lrange = {0, 0};
    clk.mark("near candidates", s);
    DBuf<int32_t> dtleaf;
    DBuf<int64_t> dlptr, dlrange;
    dtleaf.upload(tleaf, s);
    dlptr.upload(lptr, s);
    dlrange.upload(lrange, s);
    DBuf<int32_t> cnt;
    cnt.alloc(np_);
    launch_near_count(np_, cen_.p, np_, cen_.p, cross2_.p, dtleaf.p, dlptr.p, dlrange.p, near_f4(prm_.near_factor),
                      cnt.p, s);
    std::vector<int32_t> hc = cnt.download(s);
    clk.mark(" near count", s);
    for (int64_t i = 0; i < np_; ++i)
      if (rep_tgt[i] >= 0) hc[i] = hc[rep_tgt[i]];   // (its own count was 0: no candidates)
    std::vector<int64_t> ptr(np_ + 1, 0);
    for (int64_t i = 0; i < np_; ++i) ptr[i + 1] = ptr[i] + hc[i];
    near_.nnz = ptr[np_];
    near_.ptr.upload(ptr, s);
    near_.col.alloc(std::max<int64_t>(near_.nnz, 1));
    near_.val.alloc(4 * std::max<int64_t>(near_.nnz, 1));
    launch_near_fill(np_, cen_.p, np_, cen_.p, cross2_.p, dtleaf.p, dlptr.p, dlrange.p, near_f4(prm_.near_factor),
                     near_.ptr.p, near_.col.p, s);
    DBuf<int32_t> drep;
    if (any_rep) {
      drep.upload(rep_tgt, s);
      launch_near_copy_cols(np_, drep.p, near_.ptr.p, near_.col.p, s);
    }
    clk.mark(" near fill", s);
    std::vector<int32_t> self(np_);
    for (int64_t i = 0; i < np_; ++i) self[i] = (int32_t)i;
    DBuf<int32_t> dself;
    dself.upload(self, s);
    NearParams np{K_, prm_.k_near, prm_.k_self_edge, kappa_, dbf.p, dwf.p, dbn.p, dwn.p, dgt.p, dgw.p};
    launch_near_values(np_, cen_.p, dself.p, near_.ptr.p, near_.col.p, tri9_.p, nrm_.p, area_.p, np,
                       near_.val.p, s, drep.p);
    launch_fold_near(np_, near_.ptr.p, near_.col.p, panel_surf_.p, panel_surf_.p, forms_.p, ns,
                     surf_rhoinv_.p, near_.val.p, s, 0, drep.p);
    if (any_rep) launch_near_copy_vals(np_, drep.p, near_.ptr.p, near_.val.p, s);
    if (any_rep && std::getenv("PBT_CHECK_NEAR")) {
      // every target's rows searched and evaluated again, without copies,
      // and compared bit for bit
      std::vector<int64_t> lp2{0}, lr2;
      for (size_t k = 0; k < tls.size(); ++k) {
        std::vector<std::pair<int64_t, int64_t>> rg;
        search((int64_t)k, -1, -1, rg);
        for (const auto& r : rg) {
          if (!lr2.empty() && (int64_t)lr2.size() / 2 > lp2.back() && lr2.back() == r.first) {
            lr2.back() = r.second;
          } else {
            lr2.push_back(r.first);
            lr2.push_back(r.second);
          }
        }
        lp2.push_back((int64_t)lr2.size() / 2);
      }
      if (lr2.empty()) lr2 = {0, 0};
      DBuf<int64_t> dlp2, dlr2;
      dlp2.upload(lp2, s);
      dlr2.upload(lr2, s);
      DBuf<int32_t> c2, col2;
      c2.alloc(np_);
      launch_near_count(np_, cen_.p, np_, cen_.p, cross2_.p, dtleaf.p, dlp2.p, dlr2.p, near_f4(prm_.near_factor),
                        c2.p, s);
      const std::vector<int32_t> h2 = c2.download(s);
      std::vector<int64_t> p2(np_ + 1, 0);
      for (int64_t i = 0; i < np_; ++i) p2[i + 1] = p2[i] + h2[i];
      if (p2 != ptr) throw Error(PBT_E_STATE, "copied near rows differ in length from searched ones");
      DBuf<double> val2;
      col2.alloc(std::max<int64_t>(near_.nnz, 1));
      val2.alloc(4 * std::max<int64_t>(near_.nnz, 1));
      launch_near_fill(np_, cen_.p, np_, cen_.p, cross2_.p, dtleaf.p, dlp2.p, dlr2.p, near_f4(prm_.near_factor),
                       near_.ptr.p, col2.p, s);
      launch_near_values(np_, cen_.p, dself.p, near_.ptr.p, col2.p, tri9_.p, nrm_.p, area_.p, np, val2.p, s);
      launch_fold_near(np_, near_.ptr.p, col2.p, panel_surf_.p, panel_surf_.p, forms_.p, ns, surf_rhoinv_.p,
                       val2.p, s);
      const std::vector<int32_t> ca = near_.col.download(s), cb = col2.download(s);
      const std::vector<double> va = near_.val.download(s), vb = val2.download(s);
      if (ca != cb || std::memcmp(va.data(), vb.data(), va.size() * sizeof(double)) != 0)
        throw Error(PBT_E_STATE, "copied near rows differ from searched ones");
    }
    clk.mark(" near values", s);
    near_.val32.alloc(near_.val.n);
    launch_to_f32((int64_t)near_.val.n, near_.val.p, near_.val32.p, s);
    // inverse self blocks: the right block-Jacobi preconditioner of GMRES
    pinv_.alloc(4 * (size_t)np_);
    launch_self_blocks(np_, tri9_.p, cen_.p, panel_surf_.p, forms_.p, ns, surf_rhoinv_.p, dens_scale_.p, col_phi_.p,
                       col_psi_.p, np, pinv_.p, s);
    PBT_HIP(hipStreamSynchronize(s));
    clk.mark("near values", s);
  }

  build_plan();
  clk.mark("plan", s);
  upload_plan(s);
  clk.mark("plan upload", s);
  // Moments of every box that some M2P task reads and of all its
  // descendants: the leaves from their own sources (P2M), in chunks of at
  // most kMomChunk sources; every other box from its leaves' moments, each
  // shifted to the box's centre on its own (M2M by (box, leaf) pairs, all in
  // one launch) and added per box in leaf order.
  {
    std::vector<char> used(nbox_, 0), need(nbox_, 0), leaf(nbox_, 0);
    std::vector<int32_t> par(nbox_, -1), lev(nbox_, 0);
    int maxlev = 0;
    for (int e = 0; e < ns; ++e)
      for (size_t bi = 0; bi < trees_[e].boxes.size(); ++bi) {
        const TreeBox& tb = trees_[e].boxes[bi];
        const int g = (int)(boff_[e] + bi);
        par[g] = tb.parent >= 0 ? (int32_t)(boff_[e] + tb.parent) : -1;
        lev[g] = tb.level;
        leaf[g] = tb.leaf ? 1 : 0;
        maxlev = std::max(maxlev, tb.level);
      }
    for (int32_t b : plan_.blist) used[b] = 1;
    // the boxes that shared-surface M2P tasks read in every group
    for (const Task& t : plan_.m2pm)
      for (int32_t r = t.lbeg; r < t.lend; ++r)
        for (int g = t.split; g < std::min(plan_.mgroups, t.split + kMultiBlock); ++g)
          used[plan_.blist[r] + plan_.mboxoff[(size_t)t.nsrc * plan_.mgroups + g]] = 1;
    // a box's parent precedes it in the numbering of its tree
    for (int b = 0; b < nbox_; ++b) need[b] = used[b] || (par[b] >= 0 && need[par[b]]);
    std::vector<MomChunk> ch, heads;
    int32_t slots = 0;
    std::vector<int32_t> sb = bsbeg_.download(s), se = bsend_.download(s);
    std::vector<char> known_box(nbox_, 0);
    for (int e = 0; e < ns; ++e)
      for (int64_t b = boff_[e]; b < boff_[e + 1]; ++b) known_box[b] = !two_rows(e);
    // M2M pairs (box, leaf under it, slot) and per box (box, first slot,
    // leaves), all boxes and those of known surfaces; the leaves under a box
    // are the leaves of its surface whose panels start inside its range
    (void)maxlev;
    std::vector<int32_t> pr, hd, prk, hdk;
    int32_t nslot = 0;
    for (int e = 0; e < ns; ++e) {
      const SurfTree& T = trees_[e];
      std::vector<std::pair<int32_t, int32_t>> lv;   // (first panel, global leaf id)
      for (size_t bi = 0; bi < T.boxes.size(); ++bi)
        if (T.boxes[bi].leaf) lv.push_back({T.boxes[bi].pbeg, (int32_t)(boff_[e] + bi)});
      std::sort(lv.begin(), lv.end());
      for (size_t bi = 0; bi < T.boxes.size(); ++bi) {
        const int32_t g = (int32_t)(boff_[e] + bi);
        if (!need[g] || leaf[g]) continue;
        const TreeBox& tb = T.boxes[bi];
        auto lo = std::lower_bound(lv.begin(), lv.end(), std::make_pair(tb.pbeg, (int32_t)-1));
        auto hi = std::lower_bound(lv.begin(), lv.end(), std::make_pair(tb.pend, (int32_t)-1));
        const int32_t s0 = nslot, n = (int32_t)(hi - lo);
        for (auto it = lo; it != hi; ++it) {
          pr.insert(pr.end(), {g, it->second, nslot});
          if (known_box[g]) prk.insert(prk.end(), {g, it->second, nslot});
          ++nslot;
        }
        hd.insert(hd.end(), {g, s0, n});
        if (known_box[g]) hdk.insert(hdk.end(), {g, s0, n});
      }
    }
    npair_ = (int)pr.size() / 3;
    nhead_ = (int)hd.size() / 3;
    npair_known_ = (int)prk.size() / 3;
    nhead_known_ = (int)hdk.size() / 3;
    // heads of at most kM2MSmall leaves first (the sum takes them a thread
    // per value), keeping the box order within each class
    auto small_first = [](std::vector<int32_t>& h) {
      std::vector<int32_t> a, b;
      for (size_t i = 0; i < h.size(); i += 3) {
        std::vector<int32_t>& to = h[i + 2] <= kM2MSmall ? a : b;
        to.insert(to.end(), {h[i], h[i + 1], h[i + 2]});
      }
      const int ns = (int)a.size() / 3;
      a.insert(a.end(), b.begin(), b.end());
      h.swap(a);
      return ns;
    };
    nhead_small_ = small_first(hd);
    nhead_small_known_ = small_first(hdk);
    for (auto* v : {&pr, &hd, &prk, &hdk})
      if (v->empty()) v->assign(3, 0);
    m2m_pairs_.upload(pr, s);
    m2m_heads_.upload(hd, s);
    m2m_pairs_known_.upload(prk, s);
    m2m_heads_known_.upload(hdk, s);
    {
      const size_t NC2 = 2 * (size_t)ncoef(prm_.taylor_p);
      mslot32_.alloc(std::max<size_t>(nslot, 1) * NC2);
      mslot64_.alloc(std::max<size_t>(nslot, 1) * NC2);
    }
    for (int b = 0; b < nbox_; ++b) {
      if (!need[b] || !leaf[b] || se[b] <= sb[b]) continue;
      const int32_t n = se[b] - sb[b];
      if (n <= kMomFineMax) {
        // one chunk; a box above kMomChunk sources spreads over finer
        // coefficient groups instead of needing a second launch for sums
        ch.push_back(MomChunk{b, sb[b], se[b], 0, 1, 0, n > kMomChunk ? 1 : 0, 0});
        continue;
      }
      const int32_t np = (n + kMomChunk - 1) / kMomChunk;
      for (int32_t i = 0; i < np; ++i) {
        const int32_t a0 = sb[b] + (int32_t)((int64_t)n * i / np), a1 = sb[b] + (int32_t)((int64_t)n * (i + 1) / np);
        ch.push_back(MomChunk{b, a0, a1, slots, np, i, 0, 0});
      }
      heads.push_back(MomChunk{b, sb[b], se[b], slots, np, 0, 0, 0});
      slots += np;
    }
    // the right-hand side's product needs the moments of known boxes only
    std::vector<MomChunk> chk, headsk;
    for (const MomChunk& c : ch)
      if (known_box[c.box]) chk.push_back(c);
    for (const MomChunk& c : heads)
      if (known_box[c.box]) headsk.push_back(c);
    // block lists: (chunk, coefficient group) per block
    auto blocks_of = [&](const std::vector<MomChunk>& cs) {
      std::vector<int32_t> bl;
      for (size_t c = 0; c < cs.size(); ++c) {
        const int ng = cs[c].fine ? mom_groups(prm_.taylor_p, kMomGroupFine) : mom_groups(prm_.taylor_p);
        for (int g = 0; g < ng; ++g) {
          bl.push_back((int32_t)c);
          bl.push_back(g);
        }
      }
      return bl;
    };
    std::vector<int32_t> bl = blocks_of(ch), blk = blocks_of(chk);
    nmblocks_ = (int)bl.size() / 2;
    nmblocks_known_ = (int)blk.size() / 2;
    nmheads_ = (int)heads.size();
    nmheads_known_ = (int)headsk.size();
    for (auto* v : {&ch, &heads, &chk, &headsk})
      if (v->empty()) v->push_back(MomChunk{0, 0, 0, 0, 1, 0, 0, 0});
    for (auto* v : {&bl, &blk})
      if (v->empty()) v->assign(2, 0);
    mchunks_.upload(ch, s);
    mheads_.upload(heads, s);
    mchunks_known_.upload(chk, s);
    mheads_known_.upload(headsk, s);
    mblocks_.upload(bl, s);
    mblocks_known_.upload(blk, s);
    const size_t NC = (size_t)ncoef(prm_.taylor_p);
    msum32_.alloc(std::max<size_t>(slots, 1) * 2 * NC);
    msum64_.alloc(std::max<size_t>(slots, 1) * 2 * NC);
  }
  clk.mark("moment lists", s);
}

// Host-side bounds check of the work lists before any kernel reads them:
// every task's targets, source ranges, boxes and partial slot lie inside
// their arrays, the two halves of a P2P or M2P wavefront agree on their
// kind, and every partial slot a chunk's combine reads is written by exactly
// one task (so no product reads a slot that it did not write).  Throws on
// violation.
void System::check_plan() const {
  const Plan& P = plan_;
  auto bad = [](const std::string& m) { throw Error(PBT_E_STATE, "work list check: " + m); };
  const int64_t nr = (int64_t)P.ranges.size() / 2, nbl = (int64_t)P.blist.size();
  for (int64_t r = 0; r < nr; ++r)
    if (!(0 <= P.ranges[2 * r] && P.ranges[2 * r] <= P.ranges[2 * r + 1] && P.ranges[2 * r + 1] <= ns_))
      bad("source range out of bounds");
  for (int32_t b : P.blist)
    if (b < 0 || b >= nbox_) bad("box index out of bounds");
  // every half-wave slot is written by exactly one task, P2P or M2P
  std::vector<int32_t> written(std::max(P.npslots, 0), 0);
  auto check_p2p = [&](const std::vector<Task>& L, bool cover) {
    if (L.size() % 2) bad("odd number of P2P half tasks");
    for (size_t w = 0; w < L.size(); ++w) {
      const Task& t = L[w];
      const Task& o = L[w ^ 1];
      if (t.fused != o.fused || t.split != o.split || ((t.form ^ o.form) & kFormKz)) bad("P2P halves of one wave differ");
      if (!(t.split == 1 || t.split == 2 || t.split == 4)) bad("P2P split");
      if (t.tcount < 0 || t.tcount > 32 / t.split) bad("P2P target count");
      if (!(0 <= t.lbeg && t.lbeg <= t.lend && t.lend <= nr)) bad("P2P range list out of bounds");
      int64_t ns = 0;
      for (int32_t r = t.lbeg; r < t.lend; ++r) ns += P.ranges[2 * r + 1] - P.ranges[2 * r];
      if (ns != t.nsrc) bad("P2P source count");
      if (t.tcount == 0) continue;
      if (t.tbeg < 0 || (int64_t)t.tbeg + t.tcount > np_) bad("P2P targets out of bounds");
      if (t.slot < 0 || t.slot >= P.npslots) bad("P2P slot out of bounds");
      if (cover && ++written[t.slot] != 1) bad("P2P slot written twice");
    }
  };
  auto check_m2p = [&](const std::vector<Task>& L, bool cover) {
    if (L.size() % 2) bad("odd number of M2P half tasks");
    for (size_t w = 0; w < L.size(); ++w) {
      const Task& t = L[w];
      const Task& o = L[w ^ 1];
      if (t.fused != o.fused || ((t.form ^ o.form) & kFormKz)) bad("M2P halves of one wave differ");
      if (t.tcount < 0 || t.tcount > 32) bad("M2P target count");
      if (!(0 <= t.lbeg && t.lbeg <= t.lend && t.lend <= nbl)) bad("M2P box list out of bounds");
      if (t.tcount == 0) continue;
      if (t.tbeg < 0 || (int64_t)t.tbeg + t.tcount > np_) bad("M2P targets out of bounds");
      if (t.slot < 0 || t.slot >= P.npslots) bad("M2P slot out of bounds");
      if (cover && ++written[t.slot] != 1) bad("M2P slot written twice");
    }
  };
  check_p2p(P.p2p, true);
  check_m2p(P.m2p, true);
  if (!P.p2pm.empty()) {
    const int G = P.mgroups;
    if (G < 1 || (int)P.goff.size() != G) bad("shared-surface groups");
    if (P.p2pm.size() % 2) bad("odd number of shared-surface half tasks");
    const int64_t rows = (int64_t)P.mslot.size() / G;
    if ((int64_t)P.mslot.size() != rows * G) bad("shared-surface slot table");
    for (size_t w = 0; w < P.p2pm.size(); ++w) {
      const Task& t = P.p2pm[w];
      if (t.split != P.p2pm[w ^ 1].split) bad("shared-surface halves of one wave differ");
      if (t.fused || (t.form & kFormKz) || !t.known) bad("shared-surface task kind");
      if (t.tcount < 0 || t.tcount > 32) bad("shared-surface target count");
      if (!(0 <= t.lbeg && t.lbeg <= t.lend && t.lend <= nr)) bad("shared-surface range list out of bounds");
      int64_t nsrc = 0;
      for (int32_t r = t.lbeg; r < t.lend; ++r) nsrc += P.ranges[2 * r + 1] - P.ranges[2 * r];
      if (nsrc != t.nsrc) bad("shared-surface source count");
      if (t.tcount == 0) continue;
      if (t.tbeg < 0 || (int64_t)t.tbeg + t.tcount > np_) bad("shared-surface targets out of bounds");
      if (t.slot < 0 || t.slot >= rows) bad("shared-surface slot row out of bounds");
      if (t.split < 0 || t.split >= G || t.split % kMultiBlock) bad("shared-surface group block");
      for (int g = t.split; g < std::min(G, t.split + kMultiBlock); ++g) {
        const int64_t off = (int64_t)P.goff[g] * K_;
        for (int32_t r = t.lbeg; r < t.lend; ++r)
          if (P.ranges[2 * r] + off < 0 || P.ranges[2 * r + 1] + off > ns_) bad("shared-surface sources out of bounds");
        const int32_t sl = P.mslot[(int64_t)t.slot * G + g];
        if (sl < 0 || sl >= P.npslots) bad("shared-surface slot out of bounds");
        if (++written[sl] != 1) bad("shared-surface slot written twice");
      }
    }
  }
  if (!P.m2pm.empty()) {
    const int G = P.mgroups;
    if (G < 1 || P.mboxoff.empty() || P.mboxoff.size() % G) bad("shared-surface box offsets");
    if (P.m2pm.size() % 2) bad("odd number of shared-surface M2P half tasks");
    const int64_t rows = (int64_t)P.mslot.size() / G, orows = (int64_t)P.mboxoff.size() / G;
    for (size_t w = 0; w < P.m2pm.size(); ++w) {
      const Task& t = P.m2pm[w];
      if (t.split != P.m2pm[w ^ 1].split || t.nsrc != P.m2pm[w ^ 1].nsrc) bad("shared-surface M2P halves differ");
      if (t.fused || (t.form & kFormKz) || !t.known) bad("shared-surface M2P task kind");
      if (t.tcount < 0 || t.tcount > 32) bad("shared-surface M2P target count");
      if (!(0 <= t.lbeg && t.lbeg <= t.lend && t.lend <= nbl)) bad("shared-surface M2P box list out of bounds");
      if (t.nsrc < 0 || t.nsrc >= orows) bad("shared-surface M2P offset row");
      if (t.split < 0 || t.split >= G || t.split % kMultiBlock) bad("shared-surface M2P group block");
      // every half reads its boxes (an empty one too) in the groups of its block
      if (t.lend <= t.lbeg && (t.tcount > 0 || P.m2pm[w ^ 1].lend > P.m2pm[w ^ 1].lbeg))
        bad("shared-surface M2P half without boxes");
      for (int g = t.split; g < std::min(G, t.split + kMultiBlock); ++g) {
        const int32_t off = P.mboxoff[(size_t)t.nsrc * G + g];
        for (int32_t r = t.lbeg; r < t.lend; ++r)
          if (P.blist[r] + (int64_t)off < 0 || P.blist[r] + (int64_t)off >= nbox_) bad("shared-surface box out of bounds");
      }
      if (t.tcount == 0) continue;
      if (t.tbeg < 0 || (int64_t)t.tbeg + t.tcount > np_) bad("shared-surface M2P targets out of bounds");
      if (t.slot < 0 || t.slot >= rows) bad("shared-surface M2P slot row out of bounds");
      for (int g = t.split; g < std::min(G, t.split + kMultiBlock); ++g) {
        const int32_t sl = P.mslot[(int64_t)t.slot * G + g];
        if (sl < 0 || sl >= P.npslots) bad("shared-surface M2P slot out of bounds");
        if (++written[sl] != 1) bad("shared-surface M2P slot written twice");
      }
    }
  }
  for (int32_t v : written)
    if (v != 1) bad("partial slot never written");
  check_p2p(P.p2p_known, false);
  check_m2p(P.m2p_known, false);
  if ((int64_t)P.chunk_of.size() != np_) bad("chunk map size");
  for (int32_t c : P.chunk_of)
    if (c < 0 || c >= (int)P.chunks.size()) bad("chunk index out of bounds");
  for (const ChunkSlots& c : P.chunks) {
    if (c.tbeg < 0 || c.tcount < 1 || c.tcount > 64 || (int64_t)c.tbeg + c.tcount > np_) bad("chunk targets");
    if (c.sbeg != c.send) bad("chunk with 64-lane slots");
    if (!(0 <= c.hbeg0 && c.hbeg0 <= c.hend0 && c.hend0 <= P.npslots)) bad("chunk P2P slots (first half)");
    if (!(0 <= c.hbeg1 && c.hbeg1 <= c.hend1 && c.hend1 <= P.npslots)) bad("chunk P2P slots (second half)");
    if (c.tcount <= 32 && c.hend1 != c.hbeg1) bad("chunk without a second half has its slots");
    if (c.lchunk < 0 || c.lchunk >= P.nbh) bad("chunk index within its group");
  }
}

void System::upload_plan(hipStream_t s) {
  check_plan();
  dp2p_.upload(plan_.p2p.empty() ? std::vector<Task>(1) : plan_.p2p, s);
  dm2p_.upload(plan_.m2p.empty() ? std::vector<Task>(1) : plan_.m2p, s);
  dp2p_known_.upload(plan_.p2p_known.empty() ? std::vector<Task>(1) : plan_.p2p_known, s);
  dm2p_known_.upload(plan_.m2p_known.empty() ? std::vector<Task>(1) : plan_.m2p_known, s);
  dranges_.upload(plan_.ranges.empty() ? std::vector<int32_t>{0, 0} : plan_.ranges, s);
  dp2pm_.upload(plan_.p2pm.empty() ? std::vector<Task>(1) : plan_.p2pm, s);
  dm2pm_.upload(plan_.m2pm.empty() ? std::vector<Task>(1) : plan_.m2pm, s);
  dmboxoff_.upload(plan_.mboxoff.empty() ? std::vector<int32_t>{0} : plan_.mboxoff, s);
  dmslot_.upload(plan_.mslot.empty() ? std::vector<int32_t>{0} : plan_.mslot, s);
  dgoff_.upload(plan_.goff.empty() ? std::vector<int32_t>{0} : plan_.goff, s);
  dblist_.upload(plan_.blist.empty() ? std::vector<int32_t>{0} : plan_.blist, s);
  dchunks_.upload(plan_.chunks, s);
  dchunk_of_.upload(plan_.chunk_of, s);
  const int NC = ncoef(prm_.taylor_p);
  if (!plan_.m2p.empty() || !plan_.m2pm.empty()) {
    mom32_.alloc((size_t)nbox_ * 2 * NC);
    mom64_.alloc((size_t)nbox_ * 2 * NC);
  }
  part32_.alloc((size_t)std::max(plan_.nslots, 1) * 128);
  part64_.alloc((size_t)std::max(plan_.nslots, 1) * 128);
  ppart32_.alloc((size_t)std::max(plan_.npslots, 1) * 64);
  ppart64_.alloc((size_t)std::max(plan_.npslots, 1) * 64);
  PBT_HIP(hipStreamSynchronize(s));
}

void System::set_segments(int64_t seg_src, int64_t seg_box, hipStream_t s) {
  PBT_HIP(hipStreamSynchronize(s));
  seg_src_ = seg_src;
  seg_box_ = seg_box;
  build_plan();
  upload_plan(s);
}

// Average operator time over `reps` back-to-back applications, the best of
// three such runs (the autotuner compares launch shapes with it).
double System::time_products(bool fp32, int reps, hipStream_t s) {
  DBuf<double> x, y;
  x.alloc(n_);
  y.alloc(n_);
  PBT_HIP(hipMemsetAsync(x.p, 0, n_ * sizeof(double), s));
  matvec(x.p, y.p, fp32, s);
  hipEvent_t a, b;
  PBT_HIP(hipEventCreate(&a));
  PBT_HIP(hipEventCreate(&b));
  double best = 1e30;
  for (int trial = 0; trial < 3; ++trial) {
    PBT_HIP(hipEventRecord(a, s));
    for (int r = 0; r < reps; ++r) matvec(x.p, y.p, fp32, s);
    PBT_HIP(hipEventRecord(b, s));
    PBT_HIP(hipEventSynchronize(b));
    float ms = 0;
    PBT_HIP(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, (double)ms / reps);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

// Work decomposition: targets in chunks of 64 within tree leaves; for every
// leaf and source surface, the P2P source ranges and M2P boxes of the
// interaction lists are cut into segments; one task = (chunk, segment).
void System::build_plan() {
  Plan& P = plan_;
  P = Plan{};
  const int ns = (int)surfs_.size();
  PhaseClock clk;
  // Target groups: each leaf's panels in runs of at most kGroup = 32 (half a
  // wavefront; spatially compact in the leaf's octant order), every group
  // with the sphere of its own collocation points, so the acceptance test is
  // taken per 32 targets rather than per leaf (Section 3.2 states it per
  // target).  Two consecutive groups of a leaf form a 64-target chunk of the
  // combine, one per half.
  constexpr int kGroup = 32;
  struct LeafRef { int e; int b; TreeBox tb; };
  std::vector<LeafRef> leaves;
  for (int e = 0; e < ns; ++e)
    for (size_t b = 0; b < trees_[e].boxes.size(); ++b) {
      const TreeBox& lb = trees_[e].boxes[b];
      if (!lb.leaf) continue;
      for (int32_t t0 = lb.pbeg; t0 < lb.pend; t0 += kGroup) {
        TreeBox g = lb;
        g.pbeg = t0;
        g.pend = std::min<int32_t>(lb.pend, t0 + kGroup);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int32_t k = g.pbeg; k < g.pend; ++k)
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], h_cen_[3 * (poff_[e] + k) + d]);
            hi[d] = std::max(hi[d], h_cen_[3 * (poff_[e] + k) + d]);
          }
        for (int d = 0; d < 3; ++d) g.tc[d] = 0.5 * (lo[d] + hi[d]);
        double r2 = 0.0;
        for (int32_t k = g.pbeg; k < g.pend; ++k) {
          const double* x = &h_cen_[3 * (poff_[e] + k)];
          r2 = std::max(r2, (x[0] - g.tc[0]) * (x[0] - g.tc[0]) + (x[1] - g.tc[1]) * (x[1] - g.tc[1]) +
                                (x[2] - g.tc[2]) * (x[2] - g.tc[2]));
        }
        g.tr = std::sqrt(r2) * (1.0 + 1e-12);
        leaves.push_back({e, (int)b, g});
      }
    }
  clk.mark_host(" groups");
  leaves_.clear();
  for (const LeafRef& l : leaves) leaves_.push_back({l.e, l.b, poff_[l.e] + l.tb.pbeg, poff_[l.e] + l.tb.pend});
  // the surfaces of each group (a leaf only interacts with its own group's)
  group_surfs_.clear();
  for (int e = 0; e < ns; ++e) {
    const int g = surfs_[e]->group;
    if ((int)group_surfs_.size() <= g) group_surfs_.resize(g + 1);
    group_surfs_[g].push_back(e);
  }
  lp2p_.assign(leaves.size(), {});
  lm2p_.assign(leaves.size(), {});

  // Surfaces that every group holds unmoved (copies with one `shared` id, in
  // the same place in each group's panel layout, without an interior row):
  // the P2P pairs between them are the same in every group up to the source
  // strengths, so they go to tasks on group 0's copies that serve all groups
  // at once (P.p2pm).  Anything that does not fit leaves them to the usual
  // per-group tasks.
  const int ngroups = (int)group_surfs_.size();
  std::vector<int32_t> lfirst(ns + 1, 0);   // first target group of each surface
  for (const LeafRef& l : leaves) ++lfirst[l.e + 1];
  for (int e = 0; e < ns; ++e) lfirst[e + 1] += lfirst[e];
  std::vector<char> mshared(ns, 0);
  std::vector<std::map<int, int>> copy_in(ngroups);   // per group: shared id -> surface
  std::vector<int32_t> goff(ngroups, 0);
  bool multi = false;
  // (PBT_NO_SHARED in the environment keeps them in per-group tasks: the
  // reference the shared-surface kernels are tested against)
  if (ngroups >= 2 && !std::getenv("PBT_NO_SHARED")) {
    multi = true;
    for (int e = 0; e < ns; ++e)
      if (surfs_[e]->shared >= 0 && !two_rows(e)) {
        auto& m = copy_in[surfs_[e]->group];
        if (m.count(surfs_[e]->shared)) multi = false;   // one copy per group
        m[surfs_[e]->shared] = e;
      }
    if (copy_in[0].empty()) multi = false;
    for (int g = 0; multi && g < ngroups; ++g) {
      if (copy_in[g].size() != copy_in[0].size()) multi = false;
      bool first = true;
      for (const auto& kv : copy_in[0]) {
        auto it = copy_in[g].find(kv.first);
        if (it == copy_in[g].end()) { multi = false; break; }
        const int e0 = kv.second, e = it->second;
        const int64_t d = poff_[e] - poff_[e0];
        if (first) goff[g] = (int32_t)d;
        first = false;
        const SurfTree& A = trees_[e0];
        const SurfTree& B = trees_[e];
        bool same = d == goff[g] && surfs_[e]->nt == surfs_[e0]->nt && surfs_[e]->kind == surfs_[e0]->kind &&
                    A.boxes.size() == B.boxes.size() && lfirst[e + 1] - lfirst[e] == lfirst[e0 + 1] - lfirst[e0];
        for (size_t k = 0; same && k < A.boxes.size(); ++k)
          same = A.boxes[k].pbeg == B.boxes[k].pbeg && A.boxes[k].pend == B.boxes[k].pend &&
                 A.boxes[k].leaf == B.boxes[k].leaf;
        for (int64_t k = 0; same && k < surfs_[e]->nt; ++k) same = trees_[e].perm[k] == trees_[e0].perm[k];
        if (!same) multi = false;
      }
    }
    for (int g = 0; multi && g < ngroups; ++g)
      for (const auto& kv : copy_in[g]) {
        mshared[kv.second] = 1;
        for (const auto& kw : copy_in[g]) {
          int32_t fu = 0;
          int16_t tf = 0;
          task_form(kv.second, kw.second, fu, tf);
          if (fu || (tf & kFormKz)) multi = false;
        }
      }
    if (!multi) std::fill(mshared.begin(), mshared.end(), 0);
  }

  // A target group on a shared surface in a group other than 0 is a replica
  // of group 0's: its lists against shared surfaces are group 0's (the same
  // trees), so they are neither searched nor cut into ranges again; such
  // pairs only reserve the replica's partial slots, one per segment of
  // group 0's (rep: group 0's target group, -1 for the others).  kshared:
  // per source surface, the index of group 0's copy in group 0's surfaces.
  std::vector<int64_t> rep(leaves.size(), -1);
  std::vector<int> kshared(ns, -1);
  if (multi) {
    const std::vector<int>& gs0 = group_surfs_[0];
    for (int e = 0; e < ns; ++e)
      if (mshared[e]) {
        const int e0 = copy_in[0].at(surfs_[e]->shared);
        for (size_t k = 0; k < gs0.size(); ++k)
          if (gs0[k] == e0) kshared[e] = (int)k;
      }
    for (size_t li = 0; li < leaves.size(); ++li) {
      const int e = leaves[li].e;
      if (!mshared[e] || surfs_[e]->group == 0) continue;
      const int e0 = copy_in[0].at(surfs_[e]->shared);
      const int64_t l0 = lfirst[e0] + ((int64_t)li - lfirst[e]);
      if (leaves[l0].e != e0 || leaves[l0].tb.pbeg != leaves[li].tb.pbeg || leaves[l0].tb.pend != leaves[li].tb.pend)
        throw Error(PBT_E_STATE, "shared surfaces: target groups differ between groups");
      rep[li] = l0;
    }
  }
  auto replica_pair = [&](size_t li, int e2) { return rep[li] >= 0 && mshared[e2]; };

  // Per target group and source surface of its group of surfaces (k-th of
  // group_surfs_): merged P2P source ranges and M2P boxes.
  struct Lists { std::vector<std::pair<int32_t, int32_t>> rng; std::vector<int32_t> box; };
  std::vector<std::vector<Lists>> L(leaves.size());
  // (per target group in parallel; the counts are added up afterwards)
  std::vector<std::array<int64_t, 8>> cnt(leaves.size(), {0, 0, 0, 0, 0, 0, 0, 0});
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    const TreeBox& tl = leaves[li].tb;
    const int64_t nt = tl.pend - tl.pbeg;
    // tot_src and tot_box (pairs of shared surfaces left out), p2p, m2p,
    // fused p2p, fused m2p, group 0's sources and boxes of shared-surface
    // pairs
    std::array<int64_t, 8>& c = cnt[li];
    const bool g0 = surfs_[leaves[li].e]->group == 0;
    const std::vector<int>& gsf = group_surfs_[surfs_[leaves[li].e]->group];
    L[li].resize(gsf.size());
    lp2p_[li].resize(gsf.size());
    lm2p_[li].resize(gsf.size());
    for (size_t k2 = 0; k2 < gsf.size(); ++k2) {
      const int e2 = gsf[k2];
      const int f = form(leaves[li].e, e2);
      if (f == 0) continue;   // neither row of the leaf's surface sees e2
      if (replica_pair(li, e2)) continue;   // group 0's lists (below)
      const bool fused_pair = (f & 3) != 0 && (f >> 2) != 0;
      std::vector<int> pb, mb;
      if (prm_.treecode) interaction_lists(trees_[e2], tl, prm_.theta, pb, mb);
      else pb.push_back(0);
      std::sort(pb.begin(), pb.end(), [&](int a, int b) {
        return trees_[e2].boxes[a].pbeg < trees_[e2].boxes[b].pbeg;
      });
      Lists& o = L[li][k2];
      for (int b : pb) {
        const TreeBox& sb = trees_[e2].boxes[b];
        const int32_t j0 = (int32_t)((poff_[e2] + sb.pbeg) * K_), j1 = (int32_t)((poff_[e2] + sb.pend) * K_);
        if (!o.rng.empty() && o.rng.back().second == j0) o.rng.back().second = j1;
        else o.rng.push_back({j0, j1});
        if (!(mshared[leaves[li].e] && mshared[e2])) c[0] += (int64_t)(j1 - j0);
        else if (g0) c[6] += (int64_t)(j1 - j0);
        c[2] += (int64_t)(j1 - j0) * nt;
        if (fused_pair) c[4] += (int64_t)(j1 - j0) * nt;
      }
      for (int b : mb) o.box.push_back((int32_t)(boff_[e2] + b));
      if (!(mshared[leaves[li].e] && mshared[e2])) c[1] += (int64_t)mb.size();
      else if (g0) c[7] += (int64_t)mb.size();
      c[3] += (int64_t)mb.size() * nt;
      {
        int32_t fu = 0;
        int16_t tf = 0;
        task_form(leaves[li].e, e2, fu, tf);
        if (fu) c[5] += (int64_t)mb.size() * nt;
      }
      lp2p_[li][k2] = std::move(pb);
      lm2p_[li][k2] = std::move(mb);
    }
  });
  // the replicas' lists against shared surfaces (box numbers are local to
  // the source tree, the same in every group) and their pair counts
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    if (rep[li] < 0) return;
    const int64_t nt = leaves[li].tb.pend - leaves[li].tb.pbeg;
    const std::vector<int>& gsf = group_surfs_[surfs_[leaves[li].e]->group];
    for (size_t k2 = 0; k2 < gsf.size(); ++k2) {
      const int e2 = gsf[k2];
      if (!replica_pair(li, e2) || form(leaves[li].e, e2) == 0) continue;
      const int k0 = kshared[e2];
      lp2p_[li][k2] = lp2p_[rep[li]][k0];
      lm2p_[li][k2] = lm2p_[rep[li]][k0];
      std::array<int64_t, 8>& c = cnt[li];
      for (int b : lp2p_[li][k2]) c[2] += (int64_t)(trees_[e2].boxes[b].pend - trees_[e2].boxes[b].pbeg) * K_ * nt;
      c[3] += (int64_t)lm2p_[li][k2].size() * nt;
    }
  });
  clk.mark_host(" lists");
  int64_t tot_src = 0, tot_box = 0, tot_shared = 0, tot_shared_box = 0;
  for (const auto& c : cnt) {
    tot_src += c[0];
    tot_shared += c[6];
    tot_shared_box += c[7];
    tot_box += c[1];
    P.p2p_pairs += c[2];
    P.m2p_pairs += c[3];
    P.p2p_fused_pairs += c[4];
    P.m2p_fused_pairs += c[5];
  }
  // Segment sizes: aim at several thousand wavefront tasks (two half tasks
  // each) in each launch.
  const int64_t want = 2 * 16384;
  const int64_t seg_src = seg_src_ > 0 ? seg_src_ : std::min<int64_t>(16384, std::max<int64_t>(256, tot_src / want));
  const int64_t seg_box = seg_box_ > 0 ? seg_box_ : std::min<int64_t>(64, std::max<int64_t>(2, tot_box / want));
  seg_src_used_ = seg_src;
  seg_box_used_ = seg_box;
  // shared-surface segments: each serves kMultiBlock groups of every task,
  // so as many half tasks again from group 0's sources alone
  const int64_t mblocks = multi ? (ngroups + kMultiBlock - 1) / kMultiBlock : 1;
  const int64_t seg_m = std::min<int64_t>(16384, std::max<int64_t>(128, tot_shared * mblocks / want));
  const int64_t seg_box_m = std::min<int64_t>(64, std::max<int64_t>(2, tot_shared_box * mblocks / want));

  // Chunks (numbered per group of surfaces too, for the Gram-Schmidt
  // partials): a group that starts a 64-target run of its leaf opens a chunk
  // (its first half), the next group of the same leaf is the second half.
  std::vector<int> chunk_of_leaf(leaves.size()), half_of_leaf(leaves.size());
  P.chunk_of.assign(np_, 0);
  std::map<int, int32_t> gchunks;
  for (size_t li = 0; li < leaves.size(); ++li) {
    const TreeBox& tl = leaves[li].tb;
    const TreeBox& lb = trees_[leaves[li].e].boxes[leaves[li].b];
    const int64_t g0 = poff_[leaves[li].e] + tl.pbeg, g1 = poff_[leaves[li].e] + tl.pend;
    if ((tl.pbeg - lb.pbeg) % 64 == 0) {
      const int grp = surfs_[leaves[li].e]->group;
      P.chunks.push_back(ChunkSlots{(int32_t)g0, 0, 0, 0, 0, 0, 0, 0, grp, gchunks[grp]++});
      half_of_leaf[li] = 0;
    } else {
      half_of_leaf[li] = 1;
    }
    chunk_of_leaf[li] = (int)P.chunks.size() - 1;
    ChunkSlots& c = P.chunks.back();
    c.tcount += (int32_t)(g1 - g0);
    for (int64_t k = g0; k < g1; ++k) P.chunk_of[k] = (int32_t)(P.chunks.size() - 1);
  }
  P.nbh = 1;
  for (const auto& kv : gchunks) P.nbh = std::max(P.nbh, (int)kv.second);
  // Full chunks: both groups of 32 targets.
  std::vector<char> full_first(leaves.size(), 0);
  for (size_t li = 0; li + 1 < leaves.size(); ++li)
    if (half_of_leaf[li] == 0 && half_of_leaf[li + 1] == 1 && leaves[li].tb.pend - leaves[li].tb.pbeg == 32 &&
        leaves[li + 1].tb.pend - leaves[li + 1].tb.pbeg == 32)
      full_first[li] = 1;
  // Segments per (leaf, source surface): each group's ranges and boxes cut
  // into its own arrays in parallel, then laid end to end in group order.
  // e2: the source surface; a replica segment only reserves a slot
  struct Seg { int32_t lbeg, lend; int e2; bool m2p; bool shared = false; bool replica = false; };
  std::vector<std::vector<Seg>> segs(leaves.size());
  std::vector<std::vector<int32_t>> lranges(leaves.size()), lblist(leaves.size());
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    const std::vector<int>& gsf = group_surfs_[surfs_[leaves[li].e]->group];
    std::vector<int32_t>& rg_out = lranges[li];
    std::vector<int32_t>& bl_out = lblist[li];
    for (size_t k2 = 0; k2 < gsf.size(); ++k2) {
      const int e2 = gsf[k2];
      if (replica_pair(li, e2)) continue;   // placeholders below
      const Lists& o = L[li][k2];
      const bool shp = mshared[leaves[li].e] && mshared[e2];
      const int64_t seg = shp ? seg_m : seg_src;
      int64_t acc = 0;
      int32_t start = (int32_t)(rg_out.size() / 2);
      for (auto rg : o.rng) {
        for (int32_t a = rg.first; a < rg.second;) {
          const int32_t b = (int32_t)std::min<int64_t>(rg.second, a + (seg - acc));
          rg_out.push_back(a);
          rg_out.push_back(b);
          acc += b - a;
          a = b;
          if (acc >= seg) {
            segs[li].push_back({start, (int32_t)(rg_out.size() / 2), e2, false});
            start = (int32_t)(rg_out.size() / 2);
            acc = 0;
          }
        }
      }
      if ((int32_t)(rg_out.size() / 2) > start) segs[li].push_back({start, (int32_t)(rg_out.size() / 2), e2, false});
      const int64_t sbox = shp ? seg_box_m : seg_box;
      for (size_t k = 0; k < o.box.size(); k += sbox) {
        const int32_t b0 = (int32_t)bl_out.size();
        for (size_t q = k; q < std::min(o.box.size(), (size_t)(k + sbox)); ++q) bl_out.push_back(o.box[q]);
        segs[li].push_back({b0, (int32_t)bl_out.size(), e2, true});
      }
      if (shp)
        for (Seg& sg : segs[li])
          if (sg.e2 == e2) sg.shared = true;
    }
  });
  // a replica's shared segments: one placeholder per segment of group 0's
  // target group, in the same order (after the replica's own segments)
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    if (rep[li] < 0) return;
    const std::vector<int>& gsf = group_surfs_[surfs_[leaves[li].e]->group];
    for (int e2 : gsf) {
      if (!replica_pair(li, e2)) continue;
      const int e20 = group_surfs_[0][kshared[e2]];
      for (const Seg& s0 : segs[rep[li]])
        if (s0.shared && s0.e2 == e20) segs[li].push_back({0, 0, e2, s0.m2p, true, true});
    }
  });
  {
    std::vector<int64_t> roff(leaves.size() + 1, 0), boff(leaves.size() + 1, 0);
    for (size_t li = 0; li < leaves.size(); ++li) {
      roff[li + 1] = roff[li] + (int64_t)lranges[li].size();
      boff[li + 1] = boff[li] + (int64_t)lblist[li].size();
    }
    if (roff.back() / 2 > INT32_MAX || boff.back() > INT32_MAX)
      throw Error(PBT_E_NOMEM, "interaction lists exceed 32-bit indexing");
    P.ranges.resize(roff.back());
    P.blist.resize(boff.back());
    parallel_for((int64_t)leaves.size(), [&](int64_t li) {
      std::copy(lranges[li].begin(), lranges[li].end(), P.ranges.begin() + roff[li]);
      std::copy(lblist[li].begin(), lblist[li].end(), P.blist.begin() + boff[li]);
      for (Seg& sg : segs[li]) {
        if (sg.replica) continue;
        const int32_t d = (int32_t)(sg.m2p ? boff[li] : roff[li] / 2);
        sg.lbeg += d;
        sg.lend += d;
      }
    });
  }
  clk.mark_host(" segments");
  // Slots: every task of a group writes one half-wave partial slot
  // [slot][32][2]; per chunk half, the group's P2P slots then its M2P slots
  // (a chunk's combine reads hbeg0..hend0 for its first 32 targets,
  // hbeg1..hend1 for the others).  No 64-lane slots.
  int pslot = 0;
  std::vector<int> slot0(leaves.size(), 0);
  for (size_t li = 0; li < leaves.size(); ++li) {
    ChunkSlots& cs = P.chunks[chunk_of_leaf[li]];
    slot0[li] = pslot;
    pslot += (int)segs[li].size();
    if (half_of_leaf[li] == 0) {
      cs.hbeg0 = slot0[li];
      cs.hend0 = pslot;
      cs.hbeg1 = cs.hend1 = pslot;
    } else {
      cs.hbeg1 = slot0[li];
      cs.hend1 = pslot;
    }
  }
  P.nslots = 0;
  P.npslots = pslot;
  // Half tasks of every group and segment, P2P and M2P alike.  The two
  // halves of a full chunk (both groups of 32 targets) are put on one
  // wavefront segment by segment for each source surface (their lists are
  // nearly the same: same sources, balanced work); every other half is
  // paired below with a half of the same kind.
  auto make_task = [&](size_t li, const Seg& sg, int slot) {
    const int e = leaves[li].e;
    const bool mol = two_rows(e);
    Task t{};
    t.tbeg = (int32_t)(poff_[e] + leaves[li].tb.pbeg);
    t.tcount = leaves[li].tb.pend - leaves[li].tb.pbeg;
    t.lbeg = sg.lbeg;
    t.lend = sg.lend;
    t.slot = slot;
    task_form(e, sg.e2, t.fused, t.form);
    t.known = two_rows(sg.e2) ? 0 : 1;
    t.rho_inv = mol ? eps_o_[e] / surfs_[e]->eps_in : 0.0;
    t.rho_inv_f = (float)t.rho_inv;
    t.split = 1;
    t.nsrc = 0;
    if (!sg.m2p)
      for (int32_t r = sg.lbeg; r < sg.lend; ++r) t.nsrc += P.ranges[2 * r + 1] - P.ranges[2 * r];
    return t;
  };
  // (per chunk in parallel, then laid end to end in chunk order)
  struct ChunkTasks { std::vector<Task> p2p, m2p, spare, mspare; };
  std::vector<ChunkTasks> ct(leaves.size());
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    if (half_of_leaf[li] != 0) return;
    ChunkTasks& c = ct[li];
    const bool pair = full_first[li] != 0;
    if (!pair) {
      for (int h = 0; h < 2; ++h) {
        const size_t lj = li + h;
        if (h == 1 && !(lj < leaves.size() && half_of_leaf[lj] == 1)) break;
        for (size_t si = 0; si < segs[lj].size(); ++si)
          if (!segs[lj][si].shared)
            (segs[lj][si].m2p ? c.mspare : c.spare).push_back(make_task(lj, segs[lj][si], slot0[lj] + (int)si));
      }
      return;
    }
    // per source surface and kind, the k-th segment of each half together
    const std::vector<int>& gsf = group_surfs_[surfs_[leaves[li].e]->group];
    for (int e2 : gsf)
      for (int m = 0; m < 2; ++m) {
        std::vector<std::pair<size_t, int>> sa, sb;   // (segment index, slot)
        for (size_t si = 0; si < segs[li].size(); ++si)
          if (segs[li][si].e2 == e2 && segs[li][si].m2p == (m == 1) && !segs[li][si].shared)
            sa.push_back({si, slot0[li] + (int)si});
        for (size_t si = 0; si < segs[li + 1].size(); ++si)
          if (segs[li + 1][si].e2 == e2 && segs[li + 1][si].m2p == (m == 1) && !segs[li + 1][si].shared)
            sb.push_back({si, slot0[li + 1] + (int)si});
        std::vector<Task>& out = m ? c.m2p : c.p2p;
        std::vector<Task>& rest = m ? c.mspare : c.spare;
        const size_t k2 = std::min(sa.size(), sb.size());
        for (size_t k = 0; k < k2; ++k) {
          out.push_back(make_task(li, segs[li][sa[k].first], sa[k].second));
          out.push_back(make_task(li + 1, segs[li + 1][sb[k].first], sb[k].second));
        }
        for (size_t k = k2; k < sa.size(); ++k) rest.push_back(make_task(li, segs[li][sa[k].first], sa[k].second));
        for (size_t k = k2; k < sb.size(); ++k)
          rest.push_back(make_task(li + 1, segs[li + 1][sb[k].first], sb[k].second));
      }
  });
  std::vector<Task> spare, mspare;
  for (size_t li = 0; li < leaves.size(); ++li) {
    ChunkTasks& c = ct[li];
    P.p2p.insert(P.p2p.end(), c.p2p.begin(), c.p2p.end());
    P.m2p.insert(P.m2p.end(), c.m2p.begin(), c.m2p.end());
    spare.insert(spare.end(), c.spare.begin(), c.spare.end());
    mspare.insert(mspare.end(), c.mspare.begin(), c.mspare.end());
  }
  parallel_for((int64_t)leaves.size(), [&](int64_t li) { ct[li] = ChunkTasks(); });
  // The other halves, paired with halves of the same kind (both halves of a
  // wavefront agree on fused and kFormKz, for P2P also on the split; a half
  // of at most 8 (16) targets has its lanes in 4 (2) groups that split the
  // sources), similar work next to each other; an odd one out gets an empty
  // partner (no targets, no sources).
  auto kz = [](const Task& t) { return (t.form & kFormKz) ? 1 : 0; };
  auto pair_up = [&](std::vector<Task>& sp, std::vector<Task>& out, bool p2p) {
    if (p2p)
      for (Task& t : sp) t.split = t.tcount <= 8 ? 4 : t.tcount <= 16 ? 2 : 1;
    std::stable_sort(sp.begin(), sp.end(), [&](const Task& a, const Task& b) {
      if (a.fused != b.fused) return a.fused < b.fused;
      if (kz(a) != kz(b)) return kz(a) < kz(b);
      if (a.split != b.split) return a.split < b.split;
      return p2p ? a.nsrc > b.nsrc : a.lend - a.lbeg > b.lend - b.lbeg;
    });
    for (size_t k = 0; k < sp.size();) {
      out.push_back(sp[k]);
      if (k + 1 < sp.size() && sp[k + 1].fused == sp[k].fused && kz(sp[k + 1]) == kz(sp[k]) &&
          sp[k + 1].split == sp[k].split) {
        out.push_back(sp[k + 1]);
        k += 2;
      } else {
        Task empty = sp[k];
        empty.tcount = 0;
        empty.lbeg = empty.lend = 0;
        empty.nsrc = 0;
        empty.slot = 0;
        out.push_back(empty);
        k += 1;
      }
    }
  };
  clk.mark_host(" tasks");
  pair_up(spare, P.p2p, true);
  pair_up(mspare, P.m2p, false);
  clk.mark_host(" pairing");
  if (multi) {
    // shared-surface tasks on group 0's target groups; row r of mslot holds
    // the slot of the same segment in every group (the k-th shared segment
    // of group g's copy of the target group, whose ranges are group 0's
    // shifted by goff[g] panels)
    P.mgroups = ngroups;
    P.goff = goff;
    // per group-0 target group in parallel (its rows of mslot and tasks,
    // rows numbered locally), then laid end to end
    std::vector<int64_t> mleaves;
    for (size_t li = 0; li < leaves.size(); ++li)
      if (mshared[leaves[li].e] && surfs_[leaves[li].e]->group == 0) mleaves.push_back((int64_t)li);
    // box-number offsets of each shared surface's copies (row per shared id)
    std::map<int, int> sid_index;
    std::vector<int32_t> boxoff;
    for (const auto& kv : copy_in[0]) {
      sid_index[kv.first] = (int)sid_index.size();
      for (int g = 0; g < ngroups; ++g)
        boxoff.push_back((int32_t)(boff_[copy_in[g].at(kv.first)] - boff_[kv.second]));
    }
    P.mboxoff = boxoff;
    std::vector<std::vector<int32_t>> lrows(mleaves.size());
    std::vector<std::vector<Task>> ltasks(mleaves.size()), ltasksm(mleaves.size());
    std::vector<const char*> lerr(mleaves.size(), nullptr);
    parallel_for((int64_t)mleaves.size(), [&](int64_t m) {
      const size_t li = (size_t)mleaves[m];
      const int e0 = leaves[li].e;
      std::vector<int> s0;
      for (size_t si = 0; si < segs[li].size(); ++si)
        if (segs[li][si].shared) s0.push_back((int)si);
      if (s0.empty()) return;
      std::vector<size_t> lg(ngroups);
      std::vector<std::vector<int>> sg(ngroups);
      for (int g = 0; g < ngroups; ++g) {
        const int e = copy_in[g].at(surfs_[e0]->shared);
        lg[g] = (size_t)(lfirst[e] + ((int64_t)li - lfirst[e0]));
        if (lg[g] >= leaves.size() || leaves[lg[g]].e != e || leaves[lg[g]].tb.pbeg != leaves[li].tb.pbeg ||
            leaves[lg[g]].tb.pend != leaves[li].tb.pend) {
          lerr[m] = "shared surfaces: target groups differ between groups";
          return;
        }
        for (size_t si = 0; si < segs[lg[g]].size(); ++si)
          if (segs[lg[g]][si].shared) sg[g].push_back((int)si);
        if (sg[g].size() != s0.size()) {
          lerr[m] = "shared surfaces: lists differ between groups";
          return;
        }
      }
      for (size_t k = 0; k < s0.size(); ++k) {
        const Seg& a0 = segs[li][s0[k]];
        const int row = (int)(lrows[m].size() / ngroups);
        const int sidx = sid_index.at(surfs_[a0.e2]->shared);
        for (int g = 0; g < ngroups; ++g) {
          const Seg& ag = segs[lg[g]][sg[g][k]];
          bool same = ag.m2p == a0.m2p && mshared[ag.e2] && surfs_[ag.e2]->shared == surfs_[a0.e2]->shared;
          if (ag.replica) {
            // (group 0's lists by construction)
          } else if (ag.lend - ag.lbeg != a0.lend - a0.lbeg) {
            same = false;
          } else if (a0.m2p) {
            const int32_t off = boxoff[(size_t)sidx * ngroups + g];
            for (int32_t q = 0; same && q < a0.lend - a0.lbeg; ++q)
              same = P.blist[ag.lbeg + q] == P.blist[a0.lbeg + q] + off;
          } else {
            const int64_t off = (int64_t)goff[g] * K_;
            for (int32_t q = 0; same && q < a0.lend - a0.lbeg; ++q)
              same = P.ranges[2 * (ag.lbeg + q)] == P.ranges[2 * (a0.lbeg + q)] + off &&
                     P.ranges[2 * (ag.lbeg + q) + 1] == P.ranges[2 * (a0.lbeg + q) + 1] + off;
          }
          if (!same) {
            lerr[m] = "shared surfaces: interaction lists differ between groups";
            return;
          }
          lrows[m].push_back(slot0[lg[g]] + sg[g][k]);
        }
        // one task per block of kMultiBlock groups (split = its first group)
        for (int gb = 0; gb < ngroups; gb += kMultiBlock) {
          Task t = make_task(li, a0, row);
          t.split = gb;
          if (a0.m2p) t.nsrc = sidx;
          (a0.m2p ? ltasksm : ltasks)[m].push_back(t);
        }
      }
    });
    std::vector<Task> mt, mtm;
    for (size_t m = 0; m < mleaves.size(); ++m) {
      if (lerr[m]) throw Error(PBT_E_STATE, lerr[m]);
      const int base = (int)(P.mslot.size() / ngroups);
      P.mslot.insert(P.mslot.end(), lrows[m].begin(), lrows[m].end());
      for (Task t : ltasks[m]) {
        t.slot += base;
        mt.push_back(t);
      }
      for (Task t : ltasksm[m]) {
        t.slot += base;
        mtm.push_back(t);
      }
    }
    // the two halves of a wavefront serve the same block of groups (and,
    // for M2P, the same source surface); similar work side by side
    auto pair_blocks = [](std::vector<Task>& v, std::vector<Task>& out, bool m2p) {
      auto work = [m2p](const Task& t) { return m2p ? t.lend - t.lbeg : t.nsrc; };
      std::stable_sort(v.begin(), v.end(), [&](const Task& a, const Task& b) {
        if (a.split != b.split) return a.split < b.split;
        if (m2p && a.nsrc != b.nsrc) return a.nsrc < b.nsrc;
        return work(a) > work(b);
      });
      for (size_t k = 0; k < v.size();) {
        out.push_back(v[k]);
        if (k + 1 < v.size() && v[k + 1].split == v[k].split && (!m2p || v[k + 1].nsrc == v[k].nsrc)) {
          out.push_back(v[k + 1]);
          k += 2;
        } else {
          // an empty partner: same group block; an M2P one also keeps the
          // boxes (valid in every group of the block, evaluated and thrown
          // away), a P2P one has no sources
          Task empty = v[k];
          empty.tcount = 0;
          if (!m2p) {
            empty.lbeg = empty.lend = 0;
            empty.nsrc = 0;
          }
          empty.slot = 0;
          out.push_back(empty);
          k += 1;
        }
      }
    };
    pair_blocks(mt, P.p2pm, false);
    pair_blocks(mtm, P.m2pm, true);
  }
  clk.mark_host(" shared tasks");
  // The right-hand side's product: only the tasks whose sources carry known
  // densities (a wavefront pair stays together, its other half emptied); the
  // partial slots of the others are cleared before that product.
  auto known_only = [](const std::vector<Task>& all, std::vector<Task>& out) {
    out.clear();
    for (size_t w = 0; w + 1 < all.size(); w += 2) {
      Task a = all[w], b = all[w + 1];
      if (!a.known && !b.known) continue;
      for (Task* t : {&a, &b})
        if (!t->known) {
          t->lbeg = t->lend = 0;
          t->nsrc = 0;
        }
      out.push_back(a);
      out.push_back(b);
    }
  };
  known_only(P.p2p, P.p2p_known);
  known_only(P.m2p, P.m2p_known);
  clk.mark_host(" known lists");
  if (std::getenv("PBT_PLAN_STATS")) {
    // lane utilisation of the P2P wavefronts: pair evaluations issued (64
    // lanes x records per round x rounds) against useful target x source pairs
    double issued = 0, useful = 0;
    int64_t nsplit[5] = {0, 0, 0, 0, 0}, empty = 0;
    for (size_t w = 0; w + 1 < P.p2p.size(); w += 2) {
      const Task& a = P.p2p[w];
      const Task& b = P.p2p[w + 1];
      const int rounds = (std::max(a.nsrc, b.nsrc) + 31) / 32;
      const int f = std::max(1, a.split);
      issued += 64.0 * (32 / f) * rounds;
      useful += (double)a.tcount * a.nsrc + (double)b.tcount * b.nsrc;
      nsplit[f] += 2;
      empty += (a.tcount == 0) + (b.tcount == 0);
    }
    double missued = 0;
    for (size_t w = 0; w + 1 < P.m2p.size(); w += 2)
      missued += 64.0 * std::max(P.m2p[w].lend - P.m2p[w].lbeg, P.m2p[w + 1].lend - P.m2p[w + 1].lbeg);
    // (target, box) M2P pairs by the box's number of sources
    std::vector<int64_t> bsrc(nbox_, 0);
    for (int e = 0; e < ns; ++e)
      for (size_t bi = 0; bi < trees_[e].boxes.size(); ++bi)
        bsrc[boff_[e] + bi] = (int64_t)(trees_[e].boxes[bi].pend - trees_[e].boxes[bi].pbeg) * K_;
    int64_t hist[6] = {0, 0, 0, 0, 0, 0};
    for (size_t w = 0; w < P.m2p.size(); ++w) {
      const Task& t = P.m2p[w];
      for (int32_t r = t.lbeg; r < t.lend; ++r) {
        const int64_t n = bsrc[P.blist[r]];
        hist[n < 16 ? 0 : n < 32 ? 1 : n < 64 ? 2 : n < 128 ? 3 : n < 256 ? 4 : 5] += t.tcount;
      }
    }
    // pairs whose target and source surfaces both lack an interior row
    // (plates: the same in every placement of a batch)
    std::vector<char> known_panel(np_, 0);
    for (int e = 0; e < ns; ++e)
      for (int64_t k = poff_[e]; k < poff_[e + 1]; ++k) known_panel[k] = !two_rows(e);
    int64_t kk_p2p = 0, kk_m2p = 0;
    for (const Task& t : P.p2p)
      if (t.tcount > 0 && known_panel[t.tbeg] && t.known) kk_p2p += (int64_t)t.tcount * t.nsrc;
    for (const Task& t : P.m2p)
      if (t.tcount > 0 && known_panel[t.tbeg] && t.known) kk_m2p += (int64_t)t.tcount * (t.lend - t.lbeg);
    std::fprintf(stderr, "[plan] segments: p2p %lld, m2p %lld, shared p2p %lld, shared m2p %lld\n", (long long)seg_src,
                 (long long)seg_box, (long long)seg_m, (long long)seg_box_m);
    std::fprintf(stderr, "[plan] pairs between surfaces without interior rows: p2p %lld, m2p %lld; "
                 "shared-surface P2P / M2P tasks %zu / %zu for %d groups\n",
                 (long long)kk_p2p, (long long)kk_m2p, P.p2pm.size(), P.m2pm.size(), P.mgroups);
    std::fprintf(stderr, "[plan] m2p pairs by box sources <16 / <32 / <64 / <128 / <256 / more: "
                 "%lld / %lld / %lld / %lld / %lld / %lld\n", (long long)hist[0], (long long)hist[1],
                 (long long)hist[2], (long long)hist[3], (long long)hist[4], (long long)hist[5]);
    std::fprintf(stderr, "[plan] p2p pairs %lld (fused %lld), waves %zu, halves split 1/2/4: %lld/%lld/%lld, "
                 "empty halves %lld, lane utilisation %.3f; m2p pairs %lld, tasks %zu, lane utilisation %.3f\n",
                 (long long)P.p2p_pairs, (long long)P.p2p_fused_pairs, P.p2p.size() / 2, (long long)nsplit[1],
                 (long long)nsplit[2], (long long)nsplit[4], (long long)empty, useful / std::max(issued, 1.0),
                 (long long)P.m2p_pairs, P.m2p.size(), (double)P.m2p_pairs / std::max(missued, 1.0));
  }
  clk.mark_host(" statistics");
  // the per-group work vectors, released in parallel (most were allocated
  // by the worker threads)
  parallel_for((int64_t)leaves.size(), [&](int64_t li) {
    std::vector<Lists>().swap(L[li]);
    std::vector<Seg>().swap(segs[li]);
    std::vector<int32_t>().swap(lranges[li]);
    std::vector<int32_t>().swap(lblist[li]);
  });
  clk.mark_host(" release");
}

// Strengths, then P2P on the caller's stream while the far field (P2M,
// M2M, M2P) runs on the system's second stream; the two write disjoint
// partial slots and join before the combine.
template <typename T>
void System::interactions(hipStream_t s, const double* x, bool timed, bool src_ready, bool known_only,
                          const ExtParts* ext) {
  const bool f32 = std::is_same<T, float>::value;
  T* src = f32 ? (T*)src32_.p : (T*)src64_.p;
  const T* tgt = f32 ? (const T*)tgt32_.p : (const T*)tgt64_.p;
  T* part = ext ? (T*)ext->part : f32 ? (T*)part32_.p : (T*)part64_.p;
  T* ppart = ext ? (T*)ext->ppart : f32 ? (T*)ppart32_.p : (T*)ppart64_.p;
  const int npairs = (int)((known_only ? plan_.p2p_known.size() : plan_.p2p.size()) / 2);
  T* mom = f32 ? (T*)mom32_.p : (T*)mom64_.p;
  if (src_ready) {
    // records, sig and mu of x already written (by the Arnoldi update)
  } else if (x) {
    PanelMaps m{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
    launch_strengths_x<T>(ns_, K_, m, x, src_wa_.p, nrm_.p, rlap_.p, sig_.p, mu_.p, src, s);
  } else {
    launch_strengths<T>(ns_, K_, sig_.p, mu_.p, src_wa_.p, nrm_.p, rlap_.p, src, s);
  }
  // task lists and moment chunks: all sources, or those with known densities
  const Task* p2p_tasks = known_only ? dp2p_known_.p : dp2p_.p;
  const Task* m2p_tasks = known_only ? dm2p_known_.p : dm2p_.p;
  const int nm2p = (int)(known_only ? plan_.m2p_known.size() : plan_.m2p.size());
  if (known_only) {
    // slots of the tasks left out must read as zero in the combine
    PBT_HIP(hipMemsetAsync(part, 0, part_bytes<T>(), s));
    PBT_HIP(hipMemsetAsync(ppart, 0, ppart_bytes<T>(), s));
  }
  const int nmb = known_only ? nmblocks_known_ : nmblocks_, nmh = known_only ? nmheads_known_ : nmheads_;
  const int32_t* mbl = known_only ? mblocks_known_.p : mblocks_.p;
  const MomChunk* mch = known_only ? mchunks_known_.p : mchunks_.p;
  const MomChunk* mhd = known_only ? mheads_known_.p : mheads_.p;
  const bool far = !plan_.m2p.empty() || !plan_.m2pm.empty();
  const bool two = far && far_mode_ == 1;
  const bool fused = far && far_mode_ == 2;
  const bool with_mom = far && far_mode_ == 3;
  // 4..6: moments inside a launch with part of the P2P tasks, then M2P with
  // the rest of them in one launch (P2P fills the M2P launch's tail); the
  // share of the P2P pairs in the second launch is 1/8, 1/4 or 1/2
  const bool split = far && far_mode_ >= 4 && far_mode_ <= 6;
  if (timed) PBT_HIP(hipEventRecord(ev_[1], s));
  const bool guard = K_ == 1 || K_ == 4 || K_ == 7;
  T* msum = f32 ? (T*)msum32_.p : (T*)msum64_.p;
  // per-kernel profile marks (full products only)
  const bool pf = prof_ && !known_only && !ext;   // (caller-owned buffers: no bookkeeping)
  const int pbase = f32 ? 0 : 4;
  auto pb = [&](hipStream_t st) { return pf ? prof_begin(st) : -1; };
  auto pe = [&](int kind, int e0, hipStream_t st) {
    if (e0 >= 0) prof_end(pbase + kind, e0, st);
  };
  // P2P between surfaces shared by every group: launched right after the
  // usual P2P tasks on the same stream, inside their timing marks
  const int nmp = (int)(plan_.p2pm.size() / 2);
  auto multi = [&](hipStream_t st) {
    launch_p2p_multi<T>(dp2pm_.p, nmp, dranges_.p, tgt, src, nrm_.p, K_, dgoff_.p, dmslot_.p, plan_.mgroups,
                        (T)kappa_, guard, ppart, st);
  };
  // M2P between them, right after the usual M2P tasks (the moments are done)
  auto mmulti = [&](hipStream_t st) {
    launch_m2p_multi<T>(prm_.taylor_p, dm2pm_.p, (int)plan_.m2pm.size(), dblist_.p, tgt, bcen_.p, mom,
                        dmboxoff_.p, dmslot_.p, plan_.mgroups, (T)kappa_, ppart, st);
  };
  // M2M after the leaves' moments (P2M): every (box, leaf) shift, then the
  // sums per box
  const int npr = known_only ? npair_known_ : npair_, nhd = known_only ? nhead_known_ : nhead_;
  const int nhs = known_only ? nhead_small_known_ : nhead_small_;
  const int32_t* m2m_pr = known_only ? m2m_pairs_known_.p : m2m_pairs_.p;
  const int32_t* m2m_hd = known_only ? m2m_heads_known_.p : m2m_heads_.p;
  T* mslot = f32 ? (T*)mslot32_.p : (T*)mslot64_.p;
  auto m2m = [&](hipStream_t fs) {
    launch_m2m<T>(prm_.taylor_p, npr, m2m_pr, nhd, nhs, m2m_hd, bcen_.p, mslot, mom, fs);
  };
  auto moments = [&](hipStream_t fs) {
    const int e0 = pb(fs);
    launch_moments<T>(prm_.taylor_p, nmb, mbl, mch, nmh, mhd, bcen_.p, brho_.p, src, mom, msum, fs);
    m2m(fs);
    pe(2, e0, fs);
  };
  // after a launch that computed the leaves' moments with P2P
  auto m2m_marked = [&](hipStream_t fs) {
    if (nhd == 0) return;
    const int e0 = pb(fs);
    m2m(fs);
    pe(2, e0, fs);
  };
  auto far_field = [&](hipStream_t fs) {
    if (timed) PBT_HIP(hipEventRecord(evm_[0], fs));
    moments(fs);
    if (timed) PBT_HIP(hipEventRecord(evm_[1], fs));
    const int e0 = pb(fs);
    launch_m2p<T>(prm_.taylor_p, m2p_tasks, nm2p, dblist_.p, tgt, bcen_.p, mom, (T)kappa_, ppart, fs);
    mmulti(fs);
    pe(1, e0, fs);
    if (timed || two) PBT_HIP(hipEventRecord(evm_[2], fs));
  };
  if (fused) {
    // moments, then one launch of M2P and P2P tasks; timing reports the
    // moments as such and the joint launch under P2P
    if (timed) PBT_HIP(hipEventRecord(evm_[0], s));
    moments(s);
    if (timed) {
      PBT_HIP(hipEventRecord(evm_[1], s));
      PBT_HIP(hipEventRecord(evm_[2], s));
      PBT_HIP(hipEventRecord(ev_[2], s));
    }
    const int e0 = pb(s);
    launch_m2p_p2p<T>(prm_.taylor_p, m2p_tasks, nm2p, dblist_.p, bcen_.p, mom, p2p_tasks, npairs,
                      dranges_.p, src, tgt, (T)kappa_, guard, ppart, s);
    mmulti(s);
    multi(s);
    pe(0, e0, s);
    if (timed) {
      PBT_HIP(hipEventRecord(ev_[3], s));
      PBT_HIP(hipEventRecord(ev_[4], s));
    }
    far_timed_ = timed;
    return;
  }
  if (split) {
    const int nb = (int)((int64_t)npairs >> (7 - far_mode_)), na = npairs - nb;
    if (timed) PBT_HIP(hipEventRecord(ev_[2], s));
    int e0 = pb(s);
    launch_p2p_moments<T>(prm_.taylor_p, nmb, mbl, mch, nmh, mhd, bcen_.p, brho_.p, mom, msum, p2p_tasks, na,
                          dranges_.p, src, tgt, (T)kappa_, guard, ppart, s);
    multi(s);
    pe(0, e0, s);
    if (timed) {
      PBT_HIP(hipEventRecord(ev_[3], s));
      PBT_HIP(hipEventRecord(evm_[0], s));
    }
    m2m_marked(s);
    if (timed) PBT_HIP(hipEventRecord(evm_[1], s));
    e0 = pb(s);
    launch_m2p_p2p<T>(prm_.taylor_p, m2p_tasks, nm2p, dblist_.p, bcen_.p, mom, p2p_tasks + 2 * (int64_t)na, nb,
                      dranges_.p, src, tgt, (T)kappa_, guard, ppart, s);
    mmulti(s);
    pe(1, e0, s);
    if (timed) {
      PBT_HIP(hipEventRecord(evm_[2], s));
      PBT_HIP(hipEventRecord(ev_[4], s));
    }
    far_timed_ = timed;
    return;
  }
  if (with_mom) {
    // moments inside the P2P launch (and its timing), then M2P
    if (timed) PBT_HIP(hipEventRecord(ev_[2], s));
    int e0 = pb(s);
    launch_p2p_moments<T>(prm_.taylor_p, nmb, mbl, mch, nmh, mhd, bcen_.p, brho_.p, mom, msum, p2p_tasks, npairs,
                          dranges_.p, src, tgt, (T)kappa_, guard, ppart, s);
    multi(s);
    pe(0, e0, s);
    if (timed) {
      PBT_HIP(hipEventRecord(ev_[3], s));
      PBT_HIP(hipEventRecord(evm_[0], s));
    }
    m2m_marked(s);
    if (timed) PBT_HIP(hipEventRecord(evm_[1], s));
    e0 = pb(s);
    launch_m2p<T>(prm_.taylor_p, m2p_tasks, nm2p, dblist_.p, tgt, bcen_.p, mom, (T)kappa_, ppart, s);
    mmulti(s);
    pe(1, e0, s);
    if (timed) {
      PBT_HIP(hipEventRecord(evm_[2], s));
      PBT_HIP(hipEventRecord(ev_[4], s));
    }
    far_timed_ = timed;
    return;
  }
  if (two) {
    // the moments first (short launches, one tree level each, with the
    // whole machine), then M2P on the second stream concurrently with P2P
    if (timed) PBT_HIP(hipEventRecord(evm_[0], s));
    moments(s);
    PBT_HIP(hipEventRecord(evm_[1], s));
    PBT_HIP(hipStreamWaitEvent(s2_, evm_[1], 0));
    const int e1 = pb(s2_);
    launch_m2p<T>(prm_.taylor_p, m2p_tasks, nm2p, dblist_.p, tgt, bcen_.p, mom, (T)kappa_, ppart, s2_);
    mmulti(s2_);
    pe(1, e1, s2_);
    PBT_HIP(hipEventRecord(evm_[2], s2_));
  }
  if (timed) PBT_HIP(hipEventRecord(ev_[2], s));
  const int e0 = pb(s);
  launch_p2p<T>(p2p_tasks, npairs, dranges_.p, tgt, src, (T)kappa_, guard, ppart, s);
  multi(s);
  pe(0, e0, s);
  if (timed) PBT_HIP(hipEventRecord(ev_[3], s));
  if (two) {
    PBT_HIP(hipStreamWaitEvent(s, evm_[2], 0));
  } else if (far) {
    far_field(s);
  }
  if (timed) PBT_HIP(hipEventRecord(ev_[4], s));
  far_timed_ = far && timed;
}

void System::apply(bool fp32, bool add_jump, const double* x, double* y, hipStream_t s, bool from_x,
                   bool timed, bool src_ready, const DotReq* dots, bool known_only, const ExtParts* ext) {
  ++napply_;
  pairs_done_ += known_only ? known_pairs_ : dense_pairs_;
  if (timed) PBT_HIP(hipEventRecord(ev_[0], s));
  if (fp32) interactions<float>(s, from_x ? x : nullptr, timed, src_ready, known_only, ext);
  else interactions<double>(s, from_x ? x : nullptr, timed, src_ready, known_only, ext);
  CombineArgs a{};
  a.np = np_;
  a.chunks = dchunks_.p;
  a.nchunks = (int)plan_.chunks.size();
  a.chunk_of = dchunk_of_.p;
  a.near_ptr = near_.ptr.p;
  a.near_col = near_.col.p;
  a.near_val = near_.val.p;
  a.near_val32 = near_.val32.p;
  a.sig = sig_.p;
  a.mu = mu_.p;
  a.x = x;
  a.maps = PanelMaps{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
  a.add_jump = add_jump ? 1 : 0;
  if (dots) {
    a.ndots = dots->ndots;
    a.V = dots->V;
    a.ldv = dots->ldv;
    a.dpart = dots->dpart;
    a.R = dots->R;
    a.nbh = plan_.nbh;
    a.self_dot = dots->self_dot;
  }
  const int e0 = prof_ && !known_only && !ext ? prof_begin(s) : -1;
  if (fp32)
    launch_combine<float>(a, ext ? (const float*)ext->part : part32_.p, ext ? (const float*)ext->ppart : ppart32_.p,
                          y, s);
  else
    launch_combine<double>(a, ext ? (const double*)ext->part : part64_.p,
                           ext ? (const double*)ext->ppart : ppart64_.p, y, s);
  if (e0 >= 0) prof_end((fp32 ? 0 : 4) + 3, e0, s);
  if (timed) PBT_HIP(hipEventRecord(ev_[5], s));
}

void System::set_profile(bool on) {
  prof_flush();
  prof_ = on;
  for (int k = 0; k < 8; ++k) {
    ptot_[k] = 0;
    pcnt_[k] = 0;
  }
}

int System::prof_begin(hipStream_t s) {
  constexpr int kPool = 4096;
  if (pev_.empty()) {
    pev_.resize(kPool);
    for (auto& e : pev_) PBT_HIP(hipEventCreate(&e));
  }
  if (pev_used_ + 2 > (int)pev_.size()) prof_flush();
  const int e0 = pev_used_++;
  PBT_HIP(hipEventRecord(pev_[e0], s));
  return e0;
}

void System::prof_end(int slot, int e0, hipStream_t s) {
  const int e1 = pev_used_++;
  PBT_HIP(hipEventRecord(pev_[e1], s));
  pmarks_.push_back({slot, e0, e1});
}

void System::prof_flush() {
  for (const PMark& m : pmarks_) {
    PBT_HIP(hipEventSynchronize(pev_[m.e1]));
    float ms = 0;
    PBT_HIP(hipEventElapsedTime(&ms, pev_[m.e0], pev_[m.e1]));
    ptot_[m.slot] += ms;
    pcnt_[m.slot] += 1;
  }
  pmarks_.clear();
  pev_used_ = 0;
}

void System::add_profile(double out[16]) {
  prof_flush();
  for (int k = 0; k < 8; ++k) {
    out[2 * k] += ptot_[k];
    out[2 * k + 1] += (double)pcnt_[k];
  }
}

void System::timing(double out[5]) {
  PBT_HIP(hipEventSynchronize(ev_[5]));
  float t[5] = {0, 0, 0, 0, 0}, a = 0, b = 0;
  PBT_HIP(hipEventElapsedTime(&t[0], ev_[0], ev_[5]));
  PBT_HIP(hipEventElapsedTime(&t[1], ev_[2], ev_[3]));
  if (far_timed_) {
    PBT_HIP(hipEventSynchronize(evm_[2]));
    PBT_HIP(hipEventElapsedTime(&t[2], evm_[1], evm_[2]));
    PBT_HIP(hipEventElapsedTime(&t[3], evm_[0], evm_[1]));
  }
  PBT_HIP(hipEventElapsedTime(&a, ev_[0], ev_[1]));
  PBT_HIP(hipEventElapsedTime(&b, ev_[4], ev_[5]));
  out[0] = t[0];
  out[1] = t[1];
  out[2] = t[2];
  out[3] = t[3];
  out[4] = a + b;   // strengths + combine (P2P and the far field overlap)
}

void System::matvec(const double* x, double* y, bool fp32, hipStream_t s, bool timed, bool src_ready,
                    const DotReq* dots, const ExtParts* ext) {
  apply(fp32, true, x, y, s, true, timed, src_ready, dots, false, ext);
}

// Known densities of the charged (sigma) and potential (phi0) surfaces, in
// reduced units, and the 1/2 jump of the imposed potential.
void System::ensure_known(hipStream_t s) {
  const int ns = (int)surfs_.size();
  std::vector<uint64_t> ver(ns);
  for (int e = 0; e < ns; ++e) ver[e] = surfs_[e]->version;
  if (ver == known_ver_ && known_ks_.n == (size_t)np_) return;
  std::vector<double> ks(np_, 0.0), km(np_, 0.0), half(np_, 0.0);
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    for (int64_t li = 0; li < S.nt; ++li) {
      const int64_t g = poff_[e] + li;
      const int32_t o = h_panel_orig_[g];
      if (S.kind == PBT_CHARGED) ks[g] = -S.bc[o] * kSigmaSI / eps_out_;
      if (S.kind == PBT_POTENTIAL) {
        km[g] = -S.bc[o] / kVoltPerUnit;
        half[g] = 0.5 * S.bc[o] / kVoltPerUnit;
      }
    }
  }
  known_ks_.upload(ks, s);
  known_km_.upload(km, s);
  known_half_.upload(half, s);
  known_ver_ = ver;
}

// Charges of molecule e on the device, their near-field correction rows and
// the pairwise Coulomb sum, rebuilt when the charges change.
System::ChargeData& System::charges(int e, hipStream_t s) {
  if (qdata_.size() != surfs_.size()) {
    qdata_.clear();
    for (size_t k = 0; k < surfs_.size(); ++k) qdata_.push_back(std::make_unique<ChargeData>());
  }
  ChargeData& d = *qdata_[e];
  const SurfIn& S = *surfs_[e];
  if (d.version == S.version) return d;
  const int64_t nq = (int64_t)S.q.size();
  d.qx.upload(S.qxyz, s);
  d.q.upload(S.q, s);
  d.phi.alloc(nq);
  d.reac_part.alloc((size_t)nq * kReacMaxSeg);
  if (nq > 0) charge_near(e, e, d.qx.p, nq, d.qn, s);
  // near corrections of the charges against each cavity of the molecule
  d.cav.clear();
  d.cav_qn.clear();
  for (int c = 0; c < (int)surfs_.size(); ++c)
    if (surfs_[c]->kind == PBT_CAVITY && outer_[c] == e && nq > 0) {
      d.cav.push_back(c);
      d.cav_qn.push_back(std::make_unique<NearCSR>());
      charge_near(c, e, d.qx.p, nq, *d.cav_qn.back(), s);
    }
  double c = 0;
  for (int64_t k = 0; k < nq; ++k)
    for (int64_t l = k + 1; l < nq; ++l) {
      const double dx = S.qxyz[3 * k] - S.qxyz[3 * l], dy = S.qxyz[3 * k + 1] - S.qxyz[3 * l + 1],
                   dz = S.qxyz[3 * k + 2] - S.qxyz[3 * l + 2];
      c += S.q[k] * S.q[l] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  d.coulomb = c;
  d.version = S.version;
  return d;
}

// b = [interior rows: (1/eps_in) sum_k q_k G_L(x_i, x_k);  solvent rows:
// minus the operator applied to the known densities, minus the imposed
// potential's jump], all on the device.
void System::rhs(double* b, hipStream_t s) {
  ensure_known(s);
  rhs_y_.alloc(n_);
  launch_known_densities(np_, known_ks_.p, known_km_.p, sig_.p, mu_.p, s);
  // only sources on charged / potential surfaces carry known densities
  apply(false, false, nullptr, rhs_y_.p, s, false, false, false, nullptr, true);
  PBT_HIP(hipMemsetAsync(b, 0, n_ * sizeof(double), s));
  launch_rhs_solvent(np_, row_sol_.p, rhs_y_.p, known_half_.p, b, s);
  // rows of a molecule's interior (its own interior rows and its cavities'
  // outside rows): Coulomb sum with 1/eps_in (eq. green_identity)
  for (int e = 0; e < (int)surfs_.size(); ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind != PBT_MOLECULE || S.q.empty()) continue;
    ChargeData& d = charges(e, s);
    launch_coulomb_rhs(S.nt, cen_.p + 3 * poff_[e], row_int_.p + poff_[e], (int64_t)S.q.size(), d.qx.p,
                       d.q.p, 1.0 / S.eps_in, b, s);
    for (int c = 0; c < (int)surfs_.size(); ++c)
      if (surfs_[c]->kind == PBT_CAVITY && outer_[c] == e)
        launch_coulomb_rhs(surfs_[c]->nt, cen_.p + 3 * poff_[c], row_sol_.p + poff_[c], (int64_t)S.q.size(),
                           d.qx.p, d.q.p, 1.0 / S.eps_in, b, s);
  }
}

// Group layout of the unknowns: the surfaces of a group are consecutive, so
// each group owns one range of unknowns (rows and columns alike).
void System::ensure_groups(hipStream_t s) {
  if (!gu_.empty()) return;
  const int ns = (int)surfs_.size();
  int G = 1;
  for (int e = 0; e < ns; ++e) G = std::max(G, surfs_[e]->group + 1);
  std::vector<int64_t> gu(2 * G, -1), gp(2 * G, -1);
  for (int e = 0; e < ns; ++e) {
    const int g = surfs_[e]->group;
    if (gu[2 * g] < 0) {
      gu[2 * g] = col_off_[e];
      gp[2 * g] = poff_[e];
    } else if (gu[2 * g + 1] != col_off_[e]) {
      throw Error(PBT_E_INVALID, "the surfaces of a group must be consecutive");
    }
    gu[2 * g + 1] = col_off_[e + 1];
    gp[2 * g + 1] = poff_[e + 1];
  }
  gmax_ = 0;
  gpmax_ = 0;
  for (int g = 0; g < G; ++g) {
    if (gu[2 * g] < 0) gu[2 * g] = gu[2 * g + 1] = 0;
    if (gp[2 * g] < 0) gp[2 * g] = gp[2 * g + 1] = 0;
    gmax_ = std::max(gmax_, gu[2 * g + 1] - gu[2 * g]);
    gpmax_ = std::max(gpmax_, gp[2 * g + 1] - gp[2 * g]);
  }
  G_ = G;
  dgu_.upload(gu, s);
  dgp_.upload(gp, s);
  gu_ = gu;
}

// Euclidean norm of each group's part of v.
std::vector<double> System::group_norms(const double* v, hipStream_t s) {
  const int nbj = gs_blocks(gmax_);
  nrm_part_.alloc((size_t)G_ * nbj + G_);
  launch_gs_dots(dgu_.p, G_, 0, 1, nullptr, n_, v, nullptr, 0, nullptr, 1, nrm_part_.p, nbj, s);
  double* out = nrm_part_.p + (size_t)G_ * nbj;
  launch_group_row0(G_, 1, nbj, nrm_part_.p, out, s);
  hnorm_.alloc(G_);
  PBT_HIP(hipMemcpyAsync(hnorm_.p, out, G_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PBT_HIP(hipStreamSynchronize(s));
  std::vector<double> r(G_);
  for (int g = 0; g < G_; ++g) r[g] = std::sqrt(hnorm_.p[g]);
  return r;
}

void System::to_internal(const double* xu, double* xi, hipStream_t s) const {
  launch_permute(n_, u2i_.p, xu, xi, true, s);
}

void System::to_boundary(const double* xi, double* xu, hipStream_t s) const {
  launch_permute(n_, u2i_.p, xi, xu, false, s);
}

void System::true_residual(const double* b, const double* x, double* r, hipStream_t s) {
  op(x, r, false, s);
  launch_axpby(n_, 1.0, b, -1.0, r, s);  // r = b - A x
}

// Restarted GMRES with classical Gram-Schmidt (once or twice, below), for the G_
// independent systems of the groups at once (one Krylov space each; the
// operator is applied to all of them in one product).  Everything of an
// Arnoldi step runs on the device, including each group's Hessenberg column
// and Givens rotation, which store the residual estimates |g_{j+1}|
// straight into pinned host memory (no copy on the stream).  The host
// enqueues groups of steps, sized from the slowest group's observed
// convergence rate, and keeps up to two in flight: it reads the estimates
// of one group (after its event) while the next runs, so the GPU does not
// wait on the host between steps.  A group stops at its
// first estimate <= tol_abs[g]; steps taken after that (for it, or for all
// groups past the last one's) are discarded.  Returns the most iterations
// any group used.
int System::gmres(bool fp32, const double* b, double* x, bool x_zero, const std::vector<double>& tol_abs,
                  int restart, int maxit, std::vector<double>& resid_out, hipStream_t s,
                  const std::vector<double>* b_norms) {
  const int m = restart, G = G_, R = m + 1, nbj = pdb_;
  // pinned: H [G][m + 1][m], g [G][m + 1], y [G][m], rs [G][m], beta [G], 1/beta [G]
  const size_t HS = (size_t)(m + 1) * m;
  hbuf_.alloc((size_t)G * (HS + 3 * (size_t)m + 3));
  double* hH = hbuf_.p;
  double* hg = hH + G * HS;
  double* hy = hg + (size_t)G * (m + 1);
  double* rs = hy + (size_t)G * m;
  double* hb = rs + (size_t)G * m;
  double* dH = gm_.p;
  double* dcs = dH + G * HS;
  double* dsn = dcs + (size_t)G * m;
  double* dg = dsn + (size_t)G * m;
  double* dbeta = dg + (size_t)G * (m + 1) + (size_t)G * m;
  double* dy = dbeta + 2 * (size_t)G;
  double* h1 = hdev_.p;
  double* part1 = part_.p;                                            // [G][R][max(nbj, nbh)]
  double* part2 = part_.p + (size_t)G * R * std::max(nbj, plan_.nbh);  // [G][R][nbj]
  int iters = 0;
  if (x_zero) PBT_HIP(hipMemcpyAsync(r_.p, b, n_ * sizeof(double), hipMemcpyDeviceToDevice, s));
  else {
    op(x, r_.p, fp32, s);
    launch_axpby(n_, 1.0, b, -1.0, r_.p, s);
  }
  // with x = 0 the residual is b, whose norms the caller may already have
  std::vector<double> beta = (x_zero && b_norms) ? *b_norms : group_norms(r_.p, s);
  resid_out = beta;
  // Gram-Schmidt passes: automatic choice (0) takes one pass while every
  // group aims at a relative reduction of at least 1e-7 (the basis then
  // stays well enough conditioned for the loss of orthogonality of a single
  // classical pass, about the rounding unit times the square of its
  // condition, not to matter), two passes for tighter targets
  int passes = gs_passes_;
  if (passes == 0) {
    passes = 1;
    for (int g = 0; g < G; ++g)
      if (beta[g] > 0 && tol_abs[g] < 1e-7 * beta[g]) passes = 2;
  }
  auto pending = [&] {
    for (int g = 0; g < G; ++g)
      if (beta[g] > tol_abs[g]) return true;
    return false;
  };
  struct Group { int beg, cnt, ev; };
  // one Arnoldi step: w = A V_k, then pass 1 (partial V^T w), pass 2 (h1 =
  // sum of pass 1, partial V^T w' and |w'|^2 with w' = w - V h1), then
  // w = (w - V h) / |w''| with each group's Hessenberg column and rotation
  // The forward operator takes the new basis vector's source records from
  // the update that produced it (step k > 0); the transposed operator starts
  // from targets instead and does not use them.
  const bool fuse = !transpose_;
  // right preconditioning, A M^-1 u = b with x = M^-1 u (M the panels' self
  // blocks; A^T with M^-T): the product of step k acts on z = M^-1 v_k,
  // which the update forming v_k also forms (fused steps) or a kernel forms
  // before the product; GMRES still minimises the residual of A x = b
  const bool pre = prm_.precond != 0;
  const NextSrc nsrc{dgp_.p, gpmax_, fp32 ? 1 : 0,
                     PanelMaps{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p},
                     K_, src_wa_.p, nrm_.p, rlap_.p, sig_.p, mu_.p,
                     fp32 ? (void*)src32_.p : (void*)src64_.p, pre ? pinv_.p : nullptr, pre ? zbuf_.p : nullptr};
  // the vector a step's product acts on
  auto operand = [&](int k) -> const double* {
    const double* vk = V_.p + (size_t)k * n_;
    if (!pre) return vk;
    if (!fuse || k == 0) launch_precond(np_, col_phi_.p, col_psi_.p, pinv_.p, vk, zbuf_.p, transpose_, false, s);
    return zbuf_.p;
  };
  // The forward operator also forms the first Gram-Schmidt pass as it writes
  // its result (per-chunk partials, nbh per row).
  const int nbh = fuse ? plan_.nbh : nbj;
  // groups of more than one element per thread: all dot rows per block
  // (each basis entry read about twice per pass, not once per 8 rows)
  const bool big = gmax_ > (int64_t)nbj * 256;
  auto enqueue_step = [&](int k) {
    double* vj1 = V_.p + (size_t)(k + 1) * n_;
    if (passes == 1) {
      // one pass: h = V^T w and |w|^2 from one reduction, then the update
      if (fuse) {
        const DotReq dr{k + 1, V_.p, n_, part1, R, 1};
        op(operand(k), vj1, fp32, s, k > 0, &dr);
      } else {
        op(operand(k), vj1, fp32, s);
        launch_gs_dots(dgu_.p, G, k + 1, R, V_.p, n_, vj1, nullptr, 0, nullptr, 1, part1, nbj, s, big);
      }
      // more chunk partials per row than one batch of loads per lane of the
      // update's row sums: added up once, not again in every update block
      const double* up = part1;
      int ust = nbh;
      if (nbh > kSumBatch) {
        launch_reduce_partials(G, k + 2, R, nbh, part1, part2, s);
        up = part2;
        ust = 1;
      }
      launch_arnoldi_update(dgu_.p, G, gmax_, k, m, R, ust, up, nullptr, V_.p, n_, vj1, dH, dcs, dsn, dg, rs,
                            fuse ? &nsrc : nullptr, s);
      return;
    }
    if (fuse) {
      const DotReq dr{k + 1, V_.p, n_, part1, R};
      op(operand(k), vj1, fp32, s, k > 0, &dr);
    } else {
      op(operand(k), vj1, fp32, s);
      launch_gs_dots(dgu_.p, G, k + 1, R, V_.p, n_, vj1, nullptr, 0, nullptr, 0, part1, nbj, s, big);
    }
    launch_gs_dots(dgu_.p, G, k + 1, R, V_.p, n_, vj1, part1, nbh, h1, 1, part2, nbj, s, big);
    launch_arnoldi_update(dgu_.p, G, gmax_, k, m, R, nbj, part2, h1, V_.p, n_, vj1, dH, dcs, dsn, dg, rs,
                          fuse ? &nsrc : nullptr, s);
  };
  bool shaky = false;
  while (pending() && iters < maxit) {
    shaky = false;
    std::vector<int> used(G, 0);
    std::vector<char> done(G, 0);
    for (int g = 0; g < G; ++g) {
      done[g] = !(beta[g] > tol_abs[g]);
      hb[g] = beta[g];
      hb[G + g] = done[g] ? 0.0 : 1.0 / beta[g];
    }
    PBT_HIP(hipMemcpyAsync(dbeta, hb, 2 * G * sizeof(double), hipMemcpyHostToDevice, s));
    launch_start_cycle(dgu_.p, G, gmax_, m, dbeta, dbeta + G, r_.p, V_.p, dg, s);
    // steps still needed after the first `known` estimates: the largest
    // prediction over the groups still running, from the rate of their last
    // few estimates (a large number while there is no rate yet)
    auto remaining = [&](int known) -> int {
      if (known < 3) return 1 << 20;
      int need = 0;
      for (int g = 0; g < G; ++g) {
        if (done[g]) continue;
        const double* r = rs + (size_t)g * m;
        const int d = std::min(known - 1, 4);
        const double r1 = std::max(r[known - 1], 1e-300), r0 = std::max(r[known - 1 - d], 1e-300);
        const double rate = std::pow(r1 / r0, 1.0 / d);
        const int ng = !(rate < 0.999) ? 4
                     : (int)std::min(1e6, std::max(0.0, std::ceil(std::log(tol_abs[g] / r1) / std::log(rate))));
        need = std::max(need, ng);
      }
      return need;
    };
    int j = 0, known = 0, nev = 0;
    bool all_done = false;
    std::deque<Group> inflight;
    while (true) {
      while (inflight.size() < 2 && j < m && iters + j < maxit) {
        int want = remaining(known) - (j - known);
        if (!inflight.empty() && want <= 0) break;   // no speculation past the predicted end
        want = std::max(1, std::min(want, known < 3 ? (j == 0 ? 2 : 4) : 8));
        const int group = std::min({want, m - j, maxit - iters - j});
        for (int k = j; k < j + group; ++k) enqueue_step(k);
        const int ev = nev++ & 1;
        PBT_HIP(hipEventRecord(evg_[ev], s));
        inflight.push_back({j, group, ev});
        j += group;
      }
      if (inflight.empty()) break;
      const Group q = inflight.front();
      inflight.pop_front();
      PBT_HIP(hipEventSynchronize(evg_[q.ev]));
      all_done = true;
      for (int g = 0; g < G; ++g) {
        if (done[g]) continue;
        for (int k = q.beg; k < q.beg + q.cnt; ++k) {
          used[g] = k + 1;
          const double rk = rs[(size_t)g * m + k];
          if (rk < 0.0) {
            // the step's norm cancelled (its basis vector is unusable, the
            // steps up to it are fine): this cycle ends for the group, the
            // next starts from its true residual, with two passes
            done[g] = 1;
            shaky = true;
            break;
          }
          resid_out[g] = rk;
          if (rk <= tol_abs[g]) {
            done[g] = 1;
            break;
          }
        }
        all_done = all_done && done[g];
      }
      known = q.beg + q.cnt;
      if (all_done) break;
    }
    int umax = 0;
    for (int g = 0; g < G; ++g) umax = std::max(umax, used[g]);
    nwasted_ += j - umax;
    iters += umax;
    if (shaky) {
      passes = 2;
      all_done = false;
    }
    // per group: x += V y with H(0:used,0:used) y = g(0:used); the H rows
    // and g entries read were final before any later step was enqueued
    PBT_HIP(hipMemcpyAsync(hH, dH, G * HS * sizeof(double), hipMemcpyDeviceToHost, s));
    PBT_HIP(hipMemcpyAsync(hg, dg, (size_t)G * (m + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    PBT_HIP(hipStreamSynchronize(s));
    for (int g = 0; g < G; ++g) {
      const double* Hg = hH + g * HS;
      double* y = hy + (size_t)g * m;
      std::fill(y, y + m, 0.0);
      for (int i = used[g] - 1; i >= 0; --i) {
        double acc = hg[(size_t)g * (m + 1) + i];
        for (int k = i + 1; k < used[g]; ++k) acc -= Hg[(size_t)i * m + k] * y[k];
        y[i] = acc / Hg[(size_t)i * m + i];
      }
    }
    PBT_HIP(hipMemcpyAsync(dy, hy, (size_t)G * m * sizeof(double), hipMemcpyHostToDevice, s));
    if (pre) {
      // x += M^-1 (V y)
      PBT_HIP(hipMemsetAsync(ztmp_.p, 0, n_ * sizeof(double), s));
      launch_lincomb(dgu_.p, G, gmax_, umax, m, V_.p, n_, dy, ztmp_.p, s);
      launch_precond(np_, col_phi_.p, col_psi_.p, pinv_.p, ztmp_.p, x, transpose_, true, s);
    } else {
      launch_lincomb(dgu_.p, G, gmax_, umax, m, V_.p, n_, dy, x, s);
    }
    if (all_done || iters >= maxit) break;
    op(x, r_.p, fp32, s);
    launch_axpby(n_, 1.0, b, -1.0, r_.p, s);
    beta = group_norms(r_.p, s);
    resid_out = beta;
  }
  return iters;
}

bool System::solve(const double* b, double* x, bool x0_given, pbt_result* res, hipStream_t s) {
  transpose_ = false;
  return solve_any(b, x, x0_given, res, s);
}

bool System::solve_t(const double* g, double* lam, pbt_result* res, hipStream_t s) {
  build_tplan(s);
  transpose_ = true;
  const bool ok = solve_any(g, lam, false, res, s);
  transpose_ = false;
  return ok;
}

// Each group is solved to ||b_g - A_g x_g|| <= tol ||b_g||; res->rel_resid
// is the largest group's relative FP64 residual (group_rel() has them all).
bool System::solve_any(const double* b, double* x, bool x0_given, pbt_result* res, hipStream_t s) {
  ensure_groups(s);
  const int G = G_;
  const int m = std::max(1, std::min<int>(prm_.restart, (int)std::max<int64_t>(gmax_, 1)));
  if (restart_alloc_ != m || V_.n != (size_t)(m + 1) * n_) {
    V_.alloc((size_t)(m + 1) * n_);
    restart_alloc_ = m;
  }
  r_.alloc(n_);
  tmp_.alloc(n_);
  y_.alloc(n_);
  zbuf_.alloc(n_);
  ztmp_.alloc(n_);
  pdb_ = gs_blocks(gmax_);
  part_.alloc((size_t)G * (m + 1) * (pdb_ + std::max(pdb_, plan_.nbh)));
  // per-chunk partials of groups with fewer chunks than nbh stay zero
  PBT_HIP(hipMemsetAsync(part_.p, 0, part_.n * sizeof(double), s));
  hdev_.alloc((size_t)G * (m + 1));
  gm_.alloc((size_t)G * ((size_t)(m + 1) * m + 4 * (size_t)m + 3));
  if (!x0_given) PBT_HIP(hipMemsetAsync(x, 0, n_ * sizeof(double), s));
  const std::vector<double> bn = group_norms(b, s);
  res->iters = 0;
  res->outer = 0;
  res->matvecs = 0;
  res->fp64_fallback = 0;
  const double tol = prm_.tol;
  group_rel_.assign(G, 0.0);
  // the largest relative residual; a non-finite one (an overflowed norm or
  // product) wins, so that it is reported instead of read as converged
  auto relmax = [&](const std::vector<double>& rn) {
    double r = 0;
    bool finite = true;
    for (int g = 0; g < G; ++g) {
      group_rel_[g] = bn[g] > 0 || !std::isfinite(bn[g]) ? rn[g] / bn[g] : 0.0;
      if (!std::isfinite(group_rel_[g])) finite = false;
      else r = std::max(r, group_rel_[g]);
    }
    return finite ? r : std::numeric_limits<double>::quiet_NaN();
  };
  bool any_b = false;
  for (double v : bn) any_b = any_b || v > 0 || !std::isfinite(v);
  if (!any_b) {
    PBT_HIP(hipMemsetAsync(x, 0, n_ * sizeof(double), s));
    res->rel_resid = 0.0;
    return true;
  }
  std::vector<double> est(G), tabs(G);
  double rel = 0.0;
  if (prm_.prec == PBT_FP64) {
    for (int g = 0; g < G; ++g) tabs[g] = tol * bn[g];
    res->iters = gmres(false, b, x, !x0_given, tabs, m, prm_.max_iter, est, s, &bn);
    res->outer = 1;
    true_residual(b, x, tmp_.p, s);
    rel = relmax(group_norms(tmp_.p, s));
    // the estimates of the last cycle can undershoot the true residual
    // (rounding in the recurrences): continue from x while it misses
    for (int extra = 0; extra < 4 && rel > tol * (1.0 + 1e-12) && res->iters < prm_.max_iter; ++extra) {
      res->iters += gmres(false, b, x, false, tabs, m, prm_.max_iter - res->iters, est, s);
      res->outer += 1;
      true_residual(b, x, tmp_.p, s);
      rel = relmax(group_norms(tmp_.p, s));
    }
  } else {
    // Iterative refinement: FP32-interaction GMRES on the FP64 residual.
    if (x0_given) true_residual(b, x, tmp_.p, s);
    else PBT_HIP(hipMemcpyAsync(tmp_.p, b, n_ * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<double> rn = x0_given ? group_norms(tmp_.p, s) : bn;
    rel = relmax(rn);
    bool inner32 = true;
    for (int outer = 0; outer < 20 && rel > tol && res->iters < prm_.max_iter; ++outer) {
      // Each running group's inner solve aims straight at the requested
      // tolerance; the FP32 operator's relative error (~1e-7) bounds how far
      // that is meaningful.  Groups already converged stay at rest.
      for (int g = 0; g < G; ++g) {
        if (!(bn[g] > 0) || rn[g] <= tol * bn[g]) {
          tabs[g] = rn[g];
          continue;
        }
        tabs[g] = std::min(0.5, std::max(0.5 * tol * bn[g] / rn[g], inner32 ? 2e-7 : 0.0)) * rn[g];
      }
      PBT_HIP(hipMemsetAsync(y_.p, 0, n_ * sizeof(double), s));
      res->iters += gmres(inner32, tmp_.p, y_.p, true, tabs, m, prm_.max_iter - res->iters, est, s, &rn);
      launch_axpby(n_, 1.0, y_.p, 1.0, x, s);
      true_residual(b, x, tmp_.p, s);
      std::vector<double> rn2 = group_norms(tmp_.p, s);
      // refinement stagnates when a correction from the FP32 operator no
      // longer halves a running group's FP64 residual: the rest of the
      // solve takes FP64 inner solves
      bool stalled = false;
      for (int g = 0; g < G; ++g)
        if (bn[g] > 0 && rn[g] > tol * bn[g] && !(rn2[g] <= 0.5 * rn[g])) stalled = true;
      rn = rn2;
      rel = relmax(rn);
      res->outer = outer + 1;
      if (stalled && inner32 && rel > tol) {
        inner32 = false;
        res->fp64_fallback = 1;
      }
    }
  }
  res->rel_resid = rel;
  return rel <= tol * (1.0 + 1e-12);
}

std::vector<std::array<double, 3>> System::surface_energies(const double* x, hipStream_t s) {
  const int ns = (int)surfs_.size();
  std::vector<std::array<double, 3>> out(ns, {0.0, 0.0, 0.0});
  PanelMaps m{col_phi_.p, col_psi_.p, row_int_.p, row_sol_.p, dens_scale_.p};
  launch_densities(np_, m, x, sig_.p, mu_.p, s);
  launch_strengths<double>(ns_, K_, sig_.p, mu_.p, src_wa_.p, nrm_.p, rlap_.p, src64_.p, s);
  // reaction potential at every charge (eq. solv_energy), then one readback
  std::vector<std::vector<double>> phi(ns);
  bool surf_terms = false;
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind == PBT_STERN || S.kind == PBT_CAVITY) continue;   // no charges, no imposed values
    if (S.kind != PBT_MOLECULE) {
      surf_terms = true;
      continue;
    }
    const int64_t nq = (int64_t)S.q.size();
    if (nq == 0) continue;
    ChargeData& d = charges(e, s);
    launch_reac(nq, d.qx.p, poff_[e] * K_, (poff_[e] + S.nt) * K_, src64_.p, eps_o_[e] / S.eps_in, d.qn.ptr.p,
                d.qn.col.p, d.qn.val.p, sig_.p + poff_[e], mu_.p + poff_[e], d.phi.p, d.reac_part.p, s);
    for (size_t k = 0; k < d.cav.size(); ++k) {
      const int c = d.cav[k];
      const NearCSR& cq = *d.cav_qn[k];
      launch_reac_cavity(nq, d.qx.p, poff_[c] * K_, (poff_[c] + surfs_[c]->nt) * K_, src64_.p, cq.ptr.p, cq.col.p,
                         cq.val.p, sig_.p + poff_[c], mu_.p + poff_[c], d.phi.p, s);
    }
    phi[e].resize(nq);
    PBT_HIP(hipMemcpyAsync(phi[e].data(), d.phi.p, nq * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  std::vector<double> xh(surf_terms ? n_ : 0);
  if (surf_terms) PBT_HIP(hipMemcpyAsync(xh.data(), x, n_ * sizeof(double), hipMemcpyDeviceToHost, s));
  PBT_HIP(hipStreamSynchronize(s));
  for (int e = 0; e < ns; ++e) {
    const SurfIn& S = *surfs_[e];
    if (S.kind == PBT_STERN || S.kind == PBT_CAVITY) continue;
    if (S.kind == PBT_MOLECULE) {
      const int64_t nq = (int64_t)S.q.size();
      if (nq == 0) continue;
      // F_solv = 1/2 sum q phi_reac (eq. solv_energy, first line)
      double acc = 0;
      for (int64_t k = 0; k < nq; ++k) acc += S.q[k] * phi[e][k];
      out[e][1] = 0.5 * acc;
      out[e][0] = charges(e, s).coulomb / (kFourPi * S.eps_in);
    } else {
      double f = 0;
      for (int64_t li = 0; li < S.nt; ++li) {
        const int64_t g = poff_[e] + li;
        const int32_t o = h_panel_orig_[g];
        const double A = h_area_[g];
        if (S.kind == PBT_CHARGED) {
          // 1/2 sum phi_j sigma_j A_j (eq. energy_surf_disc, set charge)
          f += 0.5 * xh[col_off_[e] + li] * (S.bc[o] * kSigmaSI) * A;
        } else {
          // -1/2 sum phi0_j sigma_j A_j with sigma = -eps_out dphi/dn
          f += 0.5 * eps_out_ * (S.bc[o] / kVoltPerUnit) * xh[col_off_[e] + li] * A;
        }
      }
      out[e][2] = f;
    }
  }
  return out;
}

void System::energies(const double* x, pbt_result* res, hipStream_t s) {
  double fc = 0, fs = 0, fsu = 0;
  for (const auto& e : surface_energies(x, s)) {
    fc += e[0];
    fs += e[1];
    fsu += e[2];
  }
  res->F_coul = fc * kKcalPerUnit;
  res->F_solv = fs * kKcalPerUnit;
  res->F_surf = fsu * kKcalPerUnit;
  res->F_total = res->F_coul + res->F_solv + res->F_surf;
}

std::vector<pbt_result> System::energies_by_group(const double* x, int ngroups, hipStream_t s) {
  std::vector<pbt_result> out(ngroups);
  const auto se = surface_energies(x, s);
  for (size_t e = 0; e < se.size(); ++e) {
    pbt_result& r = out[surfs_[e]->group];
    r.F_coul += se[e][0] * kKcalPerUnit;
    r.F_solv += se[e][1] * kKcalPerUnit;
    r.F_surf += se[e][2] * kKcalPerUnit;
  }
  for (auto& r : out) r.F_total = r.F_coul + r.F_solv + r.F_surf;
  return out;
}

void System::unpack(const std::vector<double>& xh, int e, double* phi, double* dphidn) const {
  const SurfIn& S = *surfs_[e];
  for (int64_t o = 0; o < S.nt; ++o) {
    const int64_t li = h_pinv_[poff_[e] + o] - poff_[e];   // unknowns follow the internal order
    double p = 0, d = 0;
    switch (S.kind) {
      case PBT_MOLECULE:
      case PBT_STERN:
      case PBT_CAVITY:
        p = xh[col_off_[e] + li];
        d = xh[col_off_[e] + S.nt + li];
        break;
      case PBT_CHARGED:
        p = xh[col_off_[e] + li];
        d = -S.bc[o] * kSigmaSI / eps_out_;
        break;
      default:
        p = S.bc[o] / kVoltPerUnit;
        d = xh[col_off_[e] + li];
    }
    if (phi) phi[o] = p;
    if (dphidn) dphidn[o] = d;
  }
}

}  // namespace pbt
