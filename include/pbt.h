/*
 * pbt.h - treecode-accelerated boundary-element Poisson-Boltzmann solver for
 * molecules near surfaces with imposed charge or potential, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Cooper & Barba, "Poisson-Boltzmann model for protein-surface
 * electrostatic interactions and grid-convergence study using the PyGBe
 * code".  The problem (Section 2, eq. pde): a Poisson equation with point
 * charges inside each molecule (permittivity eps_in), the linearised
 * Poisson-Boltzmann equation in the solvent (eps_out, Debye parameter
 * kappa), continuity of phi and eps dphi/dn on every molecule boundary, and
 * phi = phi0 or -eps_out dphi/dn = sigma0 on every imposed-BC surface.  It is
 * solved as boundary integral equations (eq. integral_eq) discretised with
 * flat triangles carrying constant phi and dphi/dn, collocated at panel
 * centroids (Section 3.1, eq. layers_element), giving the block systems of
 * eq. matrix_phi / eq. matrix_dphi, solved by GMRES with a treecode
 * accelerated matrix-vector product (Section 3.2).
 *
 * Conventions for every call:
 *  - Every function returns pbt_status; nothing throws across the boundary.
 *    On any status other than PBT_OK or PBT_E_NOCONVERGE the outputs are left
 *    untouched and pbt_last_error() describes the failure.
 *  - Host pointers unless the name ends in _dev.  The caller owns every
 *    buffer; inputs are copied during the call; outputs are written to caller
 *    memory of the documented length.  The context owns all device memory.
 *  - One context per host thread, or external locking.
 *  - Units at the boundary: Angstrom, elementary charges e, sigma in C/m^2,
 *    phi0 in V, kappa in 1/Angstrom, relative permittivities, energies in
 *    kcal/mol.  Internally lengths are A, charges e and potentials
 *    e/(eps0 A); pbt_get_solution returns phi and dphi/dn in those reduced
 *    units (1 unit = 180.951 V and 180.951 V/A).
 *  - Surfaces are closed triangle meshes, triangles counter-clockwise seen
 *    from the solvent, so (v1-v0)x(v2-v0) is the outward normal.
 *
 * Unknown vector layout (pbt_matvec, pbt_rhs, pbt_solve x0): surfaces in the
 * order they were added, enabled surfaces only; a molecule contributes
 * [phi (nt), dphi/dn inside (nt)], a charged surface [phi (nt)], a potential
 * surface [dphi/dn (nt)], each in the caller's triangle order.  Rows follow
 * the same layout: a molecule's interior row block then its solvent row
 * block.
 */
#ifndef PBT_H
#define PBT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbt_ctx pbt_ctx;

typedef enum {
  PBT_OK = 0,
  PBT_E_INVALID = 1,     /* bad argument, mesh or parameter */
  PBT_E_NOMEM = 2,       /* device or host allocation failed */
  PBT_E_DEVICE = 3,      /* HIP runtime error */
  PBT_E_NOCONVERGE = 4,  /* GMRES hit max_iter; outputs hold the last iterate */
  PBT_E_NUMERIC = 5,     /* non-finite value produced */
  PBT_E_STATE = 6        /* call not valid in the current state */
} pbt_status;

typedef enum { PBT_FP64 = 0, PBT_MIXED = 1 } pbt_precision;

typedef enum { PBT_MOLECULE = 0, PBT_CHARGED = 1, PBT_POTENTIAL = 2, PBT_STERN = 3, PBT_CAVITY = 4 } pbt_kind;

/* Numerical parameters (Tables 1-3 of the paper list the same knobs). */
typedef struct {
  int32_t k_far;        /* Gauss points per panel beyond 2L: 1, 3, 4 or 7 (default 3) */
  int32_t k_near;       /* Gauss points per panel within 2L: 19 (default) */
  int32_t k_self_edge;  /* Gauss-Legendre points per edge on the self panel (default 9) */
  int32_t ncrit;        /* max panels per tree leaf (default 300) */
  int32_t taylor_p;     /* Taylor order P, terms |k| <= P (default 6; 0..8) */
  double theta;         /* multipole acceptance, 0 < theta < 1 (default 0.5) */
  double tol;           /* GMRES relative residual ||b-Ax||/||b|| (default 1e-6) */
  int32_t restart;      /* GMRES restart length, 1..1024 (default 100) */
  int32_t max_iter;     /* total GMRES iterations allowed (default 1000) */
  pbt_precision prec;   /* FP64 everywhere, or FP32 interactions + FP64 Krylov/refinement */
  int32_t treecode;     /* 1 = treecode matvec (default), 0 = direct sums over all pairs */
  double near_factor;   /* the near rule applies to panel j seen from x when |x - c_j| < near_factor * L_j,
                           L_j = sqrt(2 A_j), c_j its centroid (Section 3.1: 2); > 0 (default 2) */
  int32_t precond;      /* 1 (default): GMRES right-preconditioned by the inverses of the panels' own
                           2x2 (molecule, Stern, cavity) or 1x1 (charged, potential) self blocks of the
                           operator, so that it still minimises ||b - A x||; 0: none (Section 3.2 names
                           GMRES only) */
} pbt_params;

typedef struct {
  double F_coul, F_solv, F_surf, F_total;  /* kcal/mol */
  int32_t iters;          /* total inner GMRES iterations */
  int32_t outer;          /* refinement steps (1 for FP64) */
  double rel_resid;       /* final FP64 relative residual */
  double t_setup_s;       /* geometry, near integrals, tree, lists, RHS */
  double t_solve_s;       /* GMRES + energies */
  int64_t p2p_pairs;      /* target x Gauss-point pairs per matvec in P2P */
  int64_t m2p_pairs;      /* (target, box) pairs per matvec in M2P */
  int64_t dense_pairs;    /* targets x Gauss points (all pairs a dense product would need) */
  int64_t p2p_fused_pairs; /* P2P pairs evaluating both the Laplace and the Yukawa kernel */
  int32_t matvecs;        /* operator applications in this solve (incl. the rhs pass) */
  int32_t fp64_fallback;  /* PBT_MIXED: 1 if the iterative refinement stagnated (an FP32-interaction
                             correction no longer halved the FP64 residual) and FP64 inner solves
                             finished the solve, else 0 */
  int64_t m2p_fused_pairs; /* M2P (target, box) pairs evaluating both the Laplace and the Yukawa
                              expansion (a molecule's target and box) */
} pbt_result;

/* Fills *p with the defaults listed above.  Never fails for non-NULL p. */
void pbt_default_params(pbt_params* p);

/* Creates a context on HIP device `hip_device`.  `params` may be NULL for the
 * defaults.  Returns PBT_E_INVALID for out-of-range parameters, PBT_E_DEVICE
 * if the device cannot be selected.  The context owns its device memory. */
pbt_status pbt_create(pbt_ctx** out, int32_t hip_device, const pbt_params* params);

/* Releases all memory of the context.  NULL is allowed. */
void pbt_destroy(pbt_ctx* ctx);

/* Text of the last error on this context (never NULL). */
const char* pbt_last_error(const pbt_ctx* ctx);

/* Replaces the numerical parameters; drops prepared systems if tree or rule
 * parameters changed. */
pbt_status pbt_set_params(pbt_ctx* ctx, const pbt_params* params);

/* Solvent permittivity (eq. pde: eps_2) and Debye parameter kappa >= 0
 * (eq. free-space: G_Y = exp(-kappa r)/(4 pi r)). */
pbt_status pbt_set_solvent(pbt_ctx* ctx, double eps_out, double kappa_per_A);

/* Adds a closed surface (eq. pde: Gamma_1 for a molecule, Gamma_2 for an
 * imposed-BC surface; PBT_STERN: the outer interface of an ion-exclusion
 * layer around one molecule, which pbt_set_stern names; PBT_CAVITY: the
 * boundary of a solvent-filled cavity inside one molecule, which
 * pbt_set_cavity names).  xyz: nv*3 doubles (A); tri: nt*3 int32 vertex
 * indices; bc: nt doubles, sigma0 [C/m^2] for PBT_CHARGED, phi0 [V] for
 * PBT_POTENTIAL, ignored (may be NULL) for the other kinds.  Writes the new surface id.  Rejects
 * non-finite coordinates, indices out of range and panels of area < 1e-12
 * A^2.  Not allowed after a solve has prepared the geometry (PBT_E_STATE). */
pbt_status pbt_add_surface(pbt_ctx* ctx, pbt_kind kind, const double* xyz, int64_t nv,
                           const int32_t* tri, int64_t nt, const double* bc, int32_t* id);

/* Replaces the imposed sigma0 / phi0 of an imposed-BC surface (nt doubles,
 * same units as pbt_add_surface).  Allowed at any time. */
pbt_status pbt_set_bc(pbt_ctx* ctx, int32_t id, const double* bc);

/* Device variant of pbt_set_bc: bc_dev holds nt doubles in device memory of
 * the context's device, read in the order of `stream` (a hipStream_t, NULL
 * for the context's own stream: work queued there before the call is done
 * first); the call waits for the read and then behaves as pbt_set_bc.
 * PBT_E_INVALID for a pointer that is not device memory of that device. */
pbt_status pbt_set_bc_dev(pbt_ctx* ctx, int32_t id, const double* bc_dev, void* stream);

/* Interior permittivity and point charges of molecule `mol_id` (eq. pde:
 * eps_1 and q_k at r_k).  xyz: nq*3 doubles (A), q: nq doubles (e).
 * Allowed at any time; nq may be 0.  PBT_E_INVALID if a charge lies outside
 * the molecule's surface or inside one of its cavities (winding number of
 * the triangle mesh about the charge, tested whenever the positions
 * change). */
pbt_status pbt_set_charges(pbt_ctx* ctx, int32_t mol_id, double eps_in, const double* xyz,
                           const double* q, int64_t nq);

/* Device variant of pbt_set_charges: q_dev (nq doubles) and xyz_dev (nq*3
 * doubles, or NULL to keep the molecule's present positions, which needs
 * an unchanged nq) are device memory of the context's device, read in the
 * order of `stream` as for pbt_set_bc_dev; then as pbt_set_charges. */
pbt_status pbt_set_charges_dev(pbt_ctx* ctx, int32_t mol_id, double eps_in, const double* xyz_dev,
                               const double* q_dev, int64_t nq, void* stream);

/* Stern layer (the extra interfaces of Section 2's closing remarks): the
 * PBT_STERN surface `stern_id` encloses molecule `mol_id` and bounds a
 * salt-free layer of permittivity eps_layer between the molecule and the
 * ionic solvent.  In the layer the potential obeys the Laplace equation;
 * its Green's representation gives the molecule's outside row (Laplace
 * kernel, the molecule's psi scaled by eps_in / eps_layer, the Stern
 * surface seen from inside) and the Stern surface's inside row; the Stern
 * surface's outside row is the solvent's (Yukawa).  The Stern surface
 * carries phi and dphi/dn (layer side), like a molecule.  One Stern surface
 * per molecule; both must be enabled together in a solve (PBT_E_STATE
 * otherwise).  The transposed product and pbt_gradient take Stern surfaces
 * (the molecule is isolated together with its Stern surface), and so does
 * pbt_solve_batch (the Stern surface moves with its molecule).  Before the
 * geometry is frozen (PBT_E_STATE after). */
pbt_status pbt_set_stern(pbt_ctx* ctx, int32_t stern_id, int32_t mol_id, double eps_layer);

/* Solvent-filled cavity (the other nested interface of Section 2's closing
 * remarks): the PBT_CAVITY surface `cav_id` lies inside molecule `mol_id`
 * and encloses a salt-free, charge-free region of permittivity eps_cavity.
 * The molecule's interior equation then holds on both its own surface and
 * the cavity's (Laplace kernel, eps_in; the cavity seen from outside with
 * its psi scaled by eps_cavity / eps_in, the molecule's charges on the
 * right-hand side), and the cavity's inside row is the cavity's Laplace
 * equation; the reaction potential at the charges includes the cavity's
 * terms.  A molecule may hold several cavities; each must be enabled
 * with its molecule (PBT_E_STATE otherwise).  Like Stern surfaces, taken by
 * the transpose, pbt_gradient and pbt_solve_batch (cavities move with their
 * molecule).
 * PBT_E_INVALID if one of the molecule's charges lies inside the cavity.
 * Before the geometry is frozen (PBT_E_STATE after). */
pbt_status pbt_set_cavity(pbt_ctx* ctx, int32_t cav_id, int32_t mol_id, double eps_cavity);

/* Includes (on = 1) or excludes a surface from subsequent solves; excluded
 * surfaces are absent from the unknown layout.  Used for the isolated-body
 * solves of the interaction energy (eq. interaction_energy). */
pbt_status pbt_enable(pbt_ctx* ctx, int32_t id, int32_t on);

/* Prepares the enabled system now (geometry, near and self corrections,
 * octrees, interaction lists, work lists) instead of at the first solve or
 * product; freezes the geometry.  Host buffers are not needed afterwards. */
pbt_status pbt_prepare(pbt_ctx* ctx);

/* Number of unknowns of the currently enabled system. */
pbt_status pbt_num_unknowns(pbt_ctx* ctx, int64_t* n);

/* Solves the enabled system by GMRES to params.tol and computes the
 * energies of Section 2 (eqs. solv_energy, phi_reac_bem, energy_surf_disc,
 * total_energy).  x0: optional initial guess (n doubles, unknown layout) or
 * NULL for zero.  PBT_E_NOCONVERGE if max_iter is reached: the result and the
 * stored solution then hold the last iterate. */
pbt_status pbt_solve(pbt_ctx* ctx, const double* x0, pbt_result* res);

/* Solution of the last solve for surface `id`, in the caller's triangle
 * order: phi (nt) and dphi/dn (nt; interior side for molecules, Stern
 * surfaces and cavities, solvent side otherwise), reduced units.  Either pointer may be
 * NULL. */
pbt_status pbt_get_solution(pbt_ctx* ctx, int32_t id, double* phi, double* dphidn);

/* Device variant of pbt_get_solution: phi_dev and dphidn_dev (nt doubles
 * each, either NULL) are device memory of the context's device, written in
 * the order of `stream` (NULL: the context's stream); the call returns when
 * the writes are done. */
pbt_status pbt_get_solution_dev(pbt_ctx* ctx, int32_t id, double* phi_dev, double* dphidn_dev, void* stream);

/* Interaction free energy (eq. interaction_energy): one solve with every
 * surface enabled and one per component alone (a molecule together with
 * its Stern surface and cavities; each other surface by itself).  parts
 * (may be NULL) receives 1 + n_surfaces results: the assembly, then each
 * isolated component at its surface id (Stern and cavity entries stay
 * zero).
 * Restores the enable flags afterwards. */
pbt_status pbt_interaction_energy(pbt_ctx* ctx, double* F_int, pbt_result* parts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product y = A x of pbt_matvec_dev (forward operator) without any
 * allocation.  Its work vectors (2 n doubles) and the P2P / M2P partial
 * sums live in a static device array of 128 MiB that the library holds on
 * each device it runs on until the process ends; PBT_E_INVALID if the
 * enabled system needs more (the error states how much).  The system must
 * be prepared already (pbt_prepare or an earlier solve or product:
 * PBT_E_STATE otherwise, since preparing allocates).  x_dev, y_dev: n
 * doubles of device memory in the unknown layout; queued on `stream` (NULL
 * for the context's stream) without synchronising.  Every call on one
 * device shares that device's array: calls that overlap on one device
 * (other streams, other contexts, other threads) race.  pbt_profile does
 * not record its launches. */
pbt_status pbt_matvec_dev_static(pbt_ctx* ctx, const double* x_dev, double* y_dev, pbt_precision prec,
                                 void* stream);

/* y = A x for the enabled system (eq. matrix_phi / matrix_dphi generalised
 * to any number of surfaces), host buffers of n doubles.  transpose = 1
 * applies the exact transpose of the same discrete operator (same tree,
 * lists and expansions).  prec selects FP64 or FP32 interactions. */
pbt_status pbt_matvec(pbt_ctx* ctx, const double* x, double* y, int32_t transpose,
                      pbt_precision prec);

/* Device variant: x_dev, y_dev are device pointers of n doubles (same
 * layout); the work is queued on `stream` (a hipStream_t, NULL for the
 * context's own stream) and the call returns without synchronising.  It uses
 * the context's work buffers, so calls on one context must not overlap. */
pbt_status pbt_matvec_dev(pbt_ctx* ctx, const double* x_dev, double* y_dev, int32_t transpose,
                          pbt_precision prec, void* stream);

/* Right-hand side b of the enabled system (n doubles): the Coulomb term of
 * eq. matrix_dphi's first row (with the 1/eps_1 of eq. green_identity) and
 * the known-BC terms of the solvent rows, in FP64. */
pbt_status pbt_rhs(pbt_ctx* ctx, double* b);

/* Gradient of the interaction free energy with respect to the imposed charge
 * density of surface `sigma_id` (dF_dsigma: nt doubles, kcal/mol per C/m^2)
 * and to the charges of molecule `mol_id` (dF_dq: nq doubles, kcal/mol per
 * e), through the adjoint solves A^T lambda = g with the transpose treecode
 * operator.  Either id may be -1 (and its pointer NULL) to skip it. */
pbt_status pbt_gradient(pbt_ctx* ctx, int32_t sigma_id, double* dF_dsigma, int32_t mol_id,
                        double* dF_dq);

/* Device variant of pbt_gradient (the path of a torch.autograd.Function):
 * dF_dsigma_dev (nt doubles) and dF_dq_dev (nq doubles) are device memory
 * of the context's device, written in the order of `stream` (NULL: the
 * context's stream) once the adjoint solves are done; the call returns
 * when the writes are.  Both pointers are checked before any work
 * (PBT_E_INVALID leaves them untouched); with PBT_E_NOCONVERGE they hold
 * the gradient of the last iterates. */
pbt_status pbt_gradient_dev(pbt_ctx* ctx, int32_t sigma_id, double* dF_dsigma_dev, int32_t mol_id,
                            double* dF_dq_dev, void* stream);

/* Interaction free energies of molecule `mol_id` at nb rigid placements:
 * body-frame coordinates x map to R_b x + t_b with R_b = rot[9b..9b+8]
 * (row-major) and t_b = shift[3b..3b+2].  The isolated energies are computed
 * once; the nb assembly systems are solved together in lock-step batches.
 * The molecule's Stern surface and cavities move with it; every other
 * enabled surface stays.  F_int: nb doubles (kcal/mol).  The stored
 * geometry is left unchanged. */
pbt_status pbt_solve_batch(pbt_ctx* ctx, int32_t mol_id, const double* rot, const double* shift,
                           int32_t nb, double* F_int);

/* Chooses P2P / M2P launch shapes and the schedule of the far field against
 * P2P (the seven schedules of pbt_set_schedule) for the enabled system
 * by timing candidates; cached per (size, precision) in memory and, if
 * cache_path is not NULL, in that text file. */
pbt_status pbt_autotune(pbt_ctx* ctx, const char* cache_path);

/* Work of the last pbt_solve, pbt_interaction_energy, pbt_gradient or
 * pbt_solve_batch call, in a pbt_result whose energy fields are zero:
 * iters = most GMRES iterations of one solve, matvecs = operator
 * applications (forward and transposed, every system the call solved),
 * dense_pairs = the dense-equivalent target x Gauss-point pairs of all those
 * applications together (a right-hand side's product, which only the
 * sources of charged and potential surfaces enter, counts its targets times
 * those sources), t_setup_s = time spent building systems,
 * t_solve_s = wall time of the whole call.  Host-only. */
pbt_status pbt_last_stats(pbt_ctx* ctx, pbt_result* out);

/* Sets the schedule of the far field against P2P for the enabled system
 * (Section 3.2 splits every product into near-field P2P and far-field
 * P2M/M2M/M2P): 0 = P2P then the far field on the context's stream,
 * 1 = the moments, then M2P on a second stream concurrently with P2P, 2 = moments
 * first, then M2P and P2P tasks in one launch, 3 = moments and P2P tasks in
 * one launch, then M2P, 4 / 5 / 6 = moments with 7/8, 3/4 or 1/2 of the P2P
 * pairs in one launch, then M2P with the other P2P pairs in one launch.
 * All seven give bitwise the same products.  PBT_E_INVALID for another
 * mode. */
pbt_status pbt_set_schedule(pbt_ctx* ctx, int32_t mode);

/* The schedule the enabled system currently uses (0 to 6, as for
 * pbt_set_schedule; pbt_autotune may have chosen it) in *mode.  Host-only. */
pbt_status pbt_get_schedule(pbt_ctx* ctx, int32_t* mode);

/* Launch shape of the enabled system's products (pbt_autotune may have
 * chosen it): out[0] = Gauss points per P2P task segment, out[1] = boxes per
 * M2P task, out[2] = work-items of a stand-alone P2P launch (wavefronts of
 * two half-wave tasks, 256-thread blocks, a multiple of 8 blocks), out[3] =
 * work-items of a stand-alone M2P launch (likewise wavefronts of two half-wave
 * tasks, the same blocks).  out: 4 int64 (host).  Host-only. */
pbt_status pbt_get_launch_shape(pbt_ctx* ctx, int64_t* out);

/* Orthogonalisation of the GMRES solver (Section 3.2 solves with GMRES) for
 * every system of the context: passes = 2 applies classical Gram-Schmidt
 * twice per Arnoldi step; passes = 1 applies it once and takes the new basis
 * vector's norm from the same reduction by Pythagoras
 * (|w - V h|^2 = |w|^2 - |h|^2), one pass over the basis fewer per step;
 * passes = 0 (default) takes one pass for every GMRES run that aims at a
 * relative residual reduction of at least 1e-7 (the inner solves of
 * PBT_MIXED always do; PBT_FP64 solves with tol >= 1e-7 do) and two passes
 * otherwise.  Takes effect from the next solve.  PBT_E_INVALID for another
 * value.  Host-only. */
pbt_status pbt_set_gram_schmidt(pbt_ctx* ctx, int32_t passes);

/* Quadrature tables the library integrates with (Section 3.1): triangle rule
 * with npts points (1, 3, 4, 7 or 19) as barycentric coordinates
 * bary[3*npts] and weights w[npts] summing to 1, or, for npts < 0, the
 * Gauss-Legendre rule with -npts points on [0, 1] (bary receives the nodes).
 * Host-only; needs no context and no GPU. */
pbt_status pbt_quadrature_rule(int32_t npts, double* bary, double* w);

/* Timing of the last pbt_matvec / pbt_matvec_dev on the context's own
 * events, in milliseconds: out[0] total, out[1] P2P kernel, out[2] M2P
 * kernel, out[3] moments (P2M at the leaves, then M2M up the tree),
 * out[4] strengths, near field and combine.
 * Under schedule 2 out[1] is the joint M2P + P2P launch and out[2] is 0;
 * under schedule 3 out[1] is the launch of the leaves' moments and P2P and
 * out[3] the M2M launches; under schedules 4-6 out[1] is the launch of the
 * leaves' moments and part of P2P, out[3] the M2M launches and out[2] the
 * joint M2P + P2P launch. */
pbt_status pbt_last_matvec_timing(pbt_ctx* ctx, double out[5]);

/* Per-kernel timing of the operator (the measurement of Section 3.2's
 * matrix-vector product, whose near and far fields dominate the solve): with
 * on = 1 every full operator application of every system of the context
 * (solves, products, batches; not the right-hand side's known-density pass)
 * records HIP events on the stream of each launch; on = 0 stops.  Either
 * call clears the totals.  Events cost a marker packet per launch and a
 * host synchronisation per 2048 launches.  Host-only bookkeeping. */
pbt_status pbt_profile(pbt_ctx* ctx, int32_t on);

/* Totals since the last pbt_profile call: out[2 * slot] milliseconds and
 * out[2 * slot + 1] launches, slot = 4 * p + kind with p = 0 for FP32 and
 * 1 for FP64 interactions and kind 0 = the launch that holds the P2P tasks
 * (with the leaves' moments under schedules 3-6, with M2P under schedule
 * 2, the first of the two under schedules 4-6), 1 = the M2P launch (the
 * second, joint one under 4-6; none under 2), 2 = the moments launches
 * (P2M at the leaves and M2M up the tree under schedules 0-2, M2M alone
 * under 3-6), 3 = the combine (near-field corrections, jump terms,
 * scatter).  out: 16 doubles (host). */
pbt_status pbt_kernel_times(pbt_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif

#endif /* PBT_H */
