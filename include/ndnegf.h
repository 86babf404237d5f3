/*
 * ndnegf -- nested-dissection NEGF solver for MI355X (gfx950): C ABI.
 *
 * The library computes, for every energy E of a grid, the diagonals of the
 * retarded, lesser and greater Green's functions of an open device
 *
 *     A(E) G^r = I,   A(E) G^< = Sigma^< (G^r)^+,
 *     A(E) = (E + i eta) I - H - diag(V) - Sigma^r_L - Sigma^r_R
 *
 * (Section 1, equations defineGless1 and defineA, without the phonon term),
 * by the method of Section 3: a block LDL^T factorization of A over a
 * nested-dissection tree of point clusters (fold), the inversion of the root
 * separator block, and a top-down extraction (selected inversion) of every
 * diagonal block of G^r and G^<; diag G^> follows from G^> - G^< = G^r - G^r+.
 *
 * Conventions shared by every entry point
 *   - Complex numbers are ndg_c128 = {re, im} doubles, the layout of
 *     std::complex<double> and torch.complex128.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the plan's device.  The caller owns every buffer it
 *     passes; the library never keeps a caller pointer after a call returns.
 *   - No call throws.  Every call returns an ndg_status; on failure
 *     ndg_last_error() returns a message for the calling thread.
 *   - Argument and structural errors are reported synchronously.  Numerical
 *     faults inside kernels (a singular pivot, a non-finite value) are written
 *     to a device status word and read with ndg_plan_status() after the
 *     stream has been synchronised.
 *   - Sites are numbered 0..n-1 by the caller; all per-site inputs and outputs
 *     use the caller's numbering (the internal cluster ordering is hidden).
 */
#ifndef NDNEGF_H
#define NDNEGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ndg_symbolic ndg_symbolic; /* separator tree + symbolic analysis (host) */
typedef struct ndg_plan ndg_plan;         /* device workspace + launch schedule        */

typedef struct {
  double re, im;
} ndg_c128;

typedef enum {
  NDG_OK = 0,
  NDG_EINVAL = -1,     /* bad argument, size or layout                                  */
  NDG_ENOTSYM = -2,    /* H is not symmetric (the method needs a complex-symmetric A)   */
  NDG_ECONTACT = -3,   /* a contact cannot be kept inside one cluster                   */
  NDG_ESINGULAR = -4,  /* a zero pivot was met while inverting a cluster block          */
  NDG_ENOMEM = -5,     /* device allocation failed                                      */
  NDG_EHIP = -6,       /* a HIP runtime call failed                                     */
  NDG_ENONFINITE = -7, /* a non-finite value reached an output                          */
  NDG_ENOTSPD = -8     /* the Newton step's Jacobian was not positive definite along a
                          search direction (out of equilibrium, or a non-convex point)   */
} ndg_status;

typedef enum { NDG_FP64 = 0, NDG_MIXED = 1 } ndg_precision;

/* Tree options.  A zeroed struct (or NULL) selects the defaults. */
typedef struct {
  int32_t leaf_max;    /* regions of at most this many points become leaves (default 64)     */
  int32_t max_cluster; /* clusters larger than this are split into a chain (default/max 64)  */
  int32_t tree_kind;   /* 0 nested dissection (default); 1 layer chain, the partition that
                          reproduces RGF (Section 3.2, Fig. 6); 2 contacts merged into the top
                          of the tree (Section 3.2, Fig. 7); 3 open slab chain: separator
                          layers every slab + 1 transport layers, chained from the middle
                          layer (the root) towards both end layers, the slabs between them
                          dissected as in 0.  Every chain cluster's subtree then holds an end
                          layer (a contact), so no folded region is closed except the slabs,
                          whose levels lie far from the energy window when they are thin
                          (Section 3.2's rules hold for any of these trees)                  */
  int32_t slab;        /* kind 3: transport layers between consecutive separators; 0 selects
                          8, a negative value none (every layer a separator: the layer chain
                          with its root in the middle layer)                                */
  int32_t layer_max;   /* kind 3: separator and end layers of up to this many points stay one
                          cluster (0 selects 128, the largest the kernels take); a wider layer
                          is split into a parent-child chain of clusters                    */
  int32_t reserved;
  const int32_t* layer_of; /* kinds 1 and 3: host [n], the transport layer of every site
                          (H must couple only equal or consecutive layers), or NULL: the
                          sites of equal x coordinate form a layer (coords required)        */
} ndg_tree_opts;

/* Summary of a symbolic analysis.  Operation counts follow Section 4.1's
 * convention (an i x j by j x k product counts ijk, an i x i inversion i^3),
 * in complex multiply-adds per energy; flops = 8 real flops per complex
 * multiply-add. */
typedef struct {
  int64_t n;
  int32_t nclusters;
  int32_t max_height;     /* number of tree levels (leaves are height 1)                  */
  int32_t max_cluster;    /* largest cluster s_i                                          */
  int32_t max_boundary;   /* largest boundary b_i (ancestor points coupled after fill)    */
  int32_t ncontacts;
  int32_t reserved;
  int64_t nnz_boundary;   /* sum of b_i                                                   */
  double ops_fold_inv, ops_fold_psi, ops_fold_update; /* fold: pivot inverses, Psi, Schur updates */
  double ops_gr_off, ops_gr_diag;                      /* G^r extraction                          */
  double ops_gl_chain, ops_gl_off, ops_gl_diag;        /* G^< source terms and extraction         */
  double ops_total;
  double ops_rgf_equiv;   /* RGF count for a layered device of the same size (0 if unknown) */
  int64_t workspace_bytes_per_energy; /* device workspace a plan needs per energy in flight */
  int64_t scatter_bytes_per_energy;   /* extra workspace per energy once phonon scattering is
                                         enabled (0 before): the all-ancestor row blocks    */
} ndg_info;

/* ---------------------------------------------------------------------------
 * Symbolic analysis (host only, no device work).
 *
 * Builds the separator tree of Section 3.2 for the graph of H plus the dense
 * contact blocks, orders the points cluster by cluster with descendants
 * before ancestors, and computes for every cluster i the boundary B_i
 * (ancestor points coupled to the subtree of i after fill), the front
 * [i, B_i], and the level schedule (clusters of one height are independent,
 * rule 1 of Section 3.2).
 *
 *   n            number of sites
 *   rowptr, col, val   host CSR of the real symmetric H, 0-based, full
 *                pattern (both triangles and the diagonal), n+1 / nnz / nnz
 *                entries.  Copied.
 *   ncontacts    number of contacts (usually 2: left, right)
 *   contact_sites[c], contact_n[c]   host array of the sites of contact c;
 *                the contact self-energy blocks passed to ndg_solve are
 *                indexed in this order.  Each contact is kept inside one
 *                cluster (Section 3.1 takes Sigma^< block diagonal).
 *   coords       host n x 3 row-major site coordinates (any unit), or NULL
 *                for a purely graph-based dissection.
 *   opts         tree options or NULL.
 *   out          receives the analysis; free with ndg_symbolic_destroy.
 * Errors: NDG_EINVAL (bad sizes / indices), NDG_ENOTSYM (H not symmetric),
 * NDG_ECONTACT (overlapping contacts, or a contact larger than max_cluster).
 */
ndg_status ndg_analyze(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                       int32_t ncontacts, const int32_t* const* contact_sites,
                       const int32_t* contact_n, const double* coords,
                       const ndg_tree_opts* opts, ndg_symbolic** out);
void ndg_symbolic_destroy(ndg_symbolic* sy);
ndg_status ndg_symbolic_info(const ndg_symbolic* sy, ndg_info* out);

/* Copies the tree into caller-owned host arrays (any may be NULL):
 *   perm[n]              perm[k] = caller site at internal position k
 *   cl_off[nclusters+1]  cluster i owns internal positions [cl_off[i], cl_off[i+1])
 *   parent[nclusters]    parent cluster, -1 for a root
 *   height[nclusters]    leaves 1
 *   bptr[nclusters+1], bidx[nnz_boundary]   B_i as internal positions
 * Clusters are numbered in post-order (descendants before ancestors). */
ndg_status ndg_symbolic_arrays(const ndg_symbolic* sy, int32_t* perm, int32_t* cl_off,
                               int32_t* parent, int32_t* height, int64_t* bptr, int32_t* bidx);

/* ---------------------------------------------------------------------------
 * Plan: device workspace and launch schedule for up to max_batch energies in
 * flight at once (ndg_solve processes larger energy grids in batches).
 * Allocates all device memory a solve needs, so ndg_solve itself allocates
 * nothing.  The plan copies what it needs from `sy`; `sy` may be destroyed
 * afterwards.  device = HIP device ordinal.  A plan must not be used from two
 * streams at once.
 * Errors: NDG_EINVAL, NDG_ENOMEM, NDG_EHIP.
 */
ndg_status ndg_plan_create(const ndg_symbolic* sy, int32_t max_batch, int32_t device,
                           ndg_plan** out);
/* Waits for all work on the plan's device (solves still in flight use its
 * memory), then frees the plan.  NULL is a no-op. */
ndg_status ndg_plan_destroy(ndg_plan* plan);
ndg_status ndg_plan_info(const ndg_plan* plan, ndg_info* out);

/* ---------------------------------------------------------------------------
 * Solve: diagonals of G^r, G^<, G^> at nE energies (Section 3.2: fold, root
 * inversion, G^r extraction; G^< by its four steps), enqueued on `stream`
 * (a hipStream_t, NULL = default stream); returns once enqueued.
 *
 *   E[nE]            device, energies (real); the complex energy is E + i eta
 *   eta              broadening (>= 0), also the caller's choice for the leads
 *   V[n]             device, real on-site potential added to diag(H), or NULL
 *   sig_r[c]         host array of ncontacts device pointers; contact c's
 *                    retarded self-energy, [nE][nc][nc] row-major in the site
 *                    order given to ndg_analyze; complex symmetric
 *   sig_less[c]      same for the lesser self-energy (skew-Hermitian)
 *   diag_gr, diag_gless, diag_ggreater   device outputs [nE][n] in the
 *                    caller's site order; diag_ggreater may be NULL
 *   growth           device output [nE] or NULL: per energy, the largest
 *                    ||(A_ii^(fold))^{-1}||_inf ||A_{i,B_i}^(fold)||_inf over the
 *                    non-root clusters, an upper bound of ||Psi_i||_inf.  The
 *                    extraction forms G_{i,B} = Psi_i G_{B,B} and
 *                    G_ii = A_ii^{-1} + Psi_i G_{B,i}; when E nears an eigenvalue
 *                    of a closed cluster these terms grow like Psi while the sum
 *                    stays moderate, and rounding errors grow with it.  Values
 *                    near 1 mean a well-conditioned fold.
 *   prec             NDG_FP64: every step in double precision.
 *                    NDG_MIXED: the Schur-update products and the extraction
 *                    products of fronts larger than 64 points run in complex
 *                    FP32 on the matrix cores with FP32 accumulation (inputs
 *                    rounded from FP64, results stored in FP64); pivot-block
 *                    inverses, Psi, the contact clusters' factorization and all
 *                    fronts of at most 64 points stay FP64.
 * Errors (synchronous): NDG_EINVAL for null pointers, nE < 0, eta < 0 or a
 * precision the plan does not support; NDG_EHIP if a launch fails.
 * Numerical faults: see ndg_plan_status.
 */
ndg_status ndg_solve(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                     const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                     ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater,
                     double* growth, ndg_precision prec, void* stream);

/* ---------------------------------------------------------------------------
 * G^> in its own step, and the transmission (Section 2 computes G^> in a
 * separate step; Section 4.2 reports density and current).
 *
 * As ndg_solve in FP64 (diag_gr, diag_gless, growth as there), plus
 *   diag_ggreater   device [nE][n] or NULL: diag of G^> = G^r Sigma^> G^r+
 *                   with Sigma^> = Sigma^< + Sigma^r - Sigma^r+ on each
 *                   contact, formed by a further G^< pass over the same
 *                   factors with Sigma^> as its source (not the identity
 *                   G^< + G^r - G^r+ of ndg_solve, from which it differs by
 *                   2 i eta diag(G^r G^r+))
 *   transmission    device [nE] or NULL (two contacts): T(E) = Tr[Gamma_0
 *                   G_01 Gamma_1 G_01+], Gamma = i (Sigma^r - Sigma^r+), from
 *                   one more pass with source -i Gamma_1 (X = G Gamma_1 G+ on
 *                   contact 0's block, T = Tr[Gamma_0 X_00])
 * Each requested output costs one G^< source-and-extraction pass.  Not for
 * graph capture by ndg_batch_solve.  Errors: as ndg_solve; NDG_EINVAL for a
 * transmission with other than two contacts.
 */
ndg_status ndg_solve_transport(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                               const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                               ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater,
                               double* transmission, double* growth, void* stream);

/* ---------------------------------------------------------------------------
 * Solve with diagonal phonon self-energies (scattering).
 *
 * Equation defineA includes a phonon self-energy, which Section 1 takes
 * diagonal: A = zI - H - diag(V) - Sigma^r_L - Sigma^r_R - diag(Sigma^r_ph),
 * and Sigma^< = Sigma^<_L + Sigma^<_R + diag(Sigma^<_ph).  With Sigma^< on
 * every cluster, the G^< source is formed by the four steps of Section 3.2
 * "Computation of blocks for G^<" with P_i = all ancestors of cluster i:
 * the rows of G^(0) over every (cluster, ancestor) pair, N = Sigma^<
 * (G^(0))+, the fold of N, and D^{-1} N (the paper's most time-consuming
 * step); the contacts' part of the source comes from their chains as in
 * ndg_solve.  G^r, its extraction and the G^< extraction are those of
 * ndg_solve.
 *
 * ndg_plan_enable_scattering allocates, once per plan, max_batch times
 * ndg_info.scatter_bytes_per_energy of device memory (the all-ancestor
 * rows: sum over clusters of s_i (s_i + ancestor points)) and the launch
 * tables.  Errors: NDG_ENOMEM, NDG_EINVAL (a tree deeper than 63 levels).
 *
 * ndg_solve_scattering: the arguments of ndg_solve, FP64 only, plus
 *   sig_r_ph[nE][n]     device, Sigma^r_ph per energy and site (caller's
 *                       site order), or NULL for none
 *   sig_less_ph[nE][n]  device, Sigma^<_ph (anti-Hermitian: purely imaginary
 *                       for a physical model, any complex value accepted),
 *                       or NULL for none.  Non-NULL needs
 *                       ndg_plan_enable_scattering first.
 *   current[nE][ncontacts]   device output or NULL: per energy and contact the
 *                       current spectral density into the device,
 *                       i_c(E) = Tr[Sigma^<_c G^>_cc - Sigma^>_c G^<_cc] over the
 *                       contact block (Sigma^> = Sigma^< + Sigma^r - Sigma^r+,
 *                       G^> = G^< + G^r - G^r+); the terminal current is e/h
 *                       times its energy integral.  The contact block of G^r
 *                       and G^< is read from the clusters' stored rows, which
 *                       hold every pair of sites of one contact (its dense
 *                       self-energy couples them).
 * With both phonon pointers NULL it equals ndg_solve in FP64 (plus the
 * currents).  Runs on `stream` alone (no side streams).  Errors: as ndg_solve; NDG_EINVAL if sig_less_ph is given
 * and scattering was not enabled.
 */
ndg_status ndg_plan_enable_scattering(ndg_plan* plan);
ndg_status ndg_solve_scattering(ndg_plan* plan, int32_t nE, const double* E, double eta,
                                const double* V, const ndg_c128* const* sig_r,
                                const ndg_c128* const* sig_less, const ndg_c128* sig_r_ph,
                                const ndg_c128* sig_less_ph, ndg_c128* diag_gr, ndg_c128* diag_gless,
                                ndg_c128* diag_ggreater, double* growth, double* current, void* stream);

/* ---------------------------------------------------------------------------
 * Self-consistent Born loop for local elastic phonon scattering.
 *
 * The phonon self-energy of equation defineA depends on the Green's
 * functions; for local elastic (deformation-potential) scattering,
 *   Sigma^r_ph,k(E) = d0 G^r_kk(E),   Sigma^<_ph,k(E) = d0 G^<_kk(E).
 * ndg_scba iterates: solve with the current self-energies
 * (ndg_solve_scattering), S' = d0 diag G, residual = max|S' - S| / max|S'|
 * over both self-energies, all sites and energies, S <- (1 - mix) S + mix S';
 * it stops after the update once residual < tol, or after max_iter solves.
 *
 *   d0                coupling (energy^2), >= 0;  mix in (0, 1];  tol >= 0
 *   sig_r_ph, sig_less_ph   device [nE][n] (caller's site order): the
 *                     starting self-energies on entry (zero for a cold
 *                     start), the last update on return
 *   diag_*, current   device outputs of the last solve (diag_ggreater and
 *                     current may be NULL; current as in ndg_solve_scattering)
 *   iterations, residual   host outputs (may be NULL): solves run, last
 *                     residual
 * Needs ndg_plan_enable_scattering.  Synchronizes `stream` once per
 * iteration to read the residual, so it cannot be captured into a graph.  The other arguments are those of ndg_solve.
 * Errors: NDG_EINVAL (arguments, scattering not enabled), NDG_EHIP.
 */
ndg_status ndg_scba(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                    const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, double d0, double mix,
                    double tol, int32_t max_iter, ndg_c128* sig_r_ph, ndg_c128* sig_less_ph,
                    ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater, double* current,
                    int32_t* iterations, double* residual, void* stream);

/* ---------------------------------------------------------------------------
 * Electron density and its gradient with respect to the on-site potential.
 *
 * ndg_density: density[i] = sum_E cE[E] (-i G^<_ii(E)), the G^< of ndg_solve
 * (Section 1: the diagonal of G^< is the electron density per unit energy),
 * accumulated over the energies in order (deterministic).
 *   cE[nE]      device, quadrature weights (e.g. trapezoid dE / 2 pi)
 *   density[n]  device output in the caller's site order (overwritten)
 *
 * ndg_density_vjp: vbar = (d density / d V)^T nbar, the vector-Jacobian
 * product for a Newton step of the Schroedinger-Poisson loop.  With
 * A = zI - H - diag(V) - Sigma and Lambda = diag(nbar),
 *   vbar_k = sum_E cE[E] 2 Im[(G^< Lambda G^r)_kk],
 * evaluated (without phonon self-energies) as
 *   sum_c G_{k,c} Sigma^<_c X_c(k,:)^T,  X_c = A^{-1} Lambda conj(G_{:,c}),
 * with G_{:,c} and X_c obtained by solves with the fold's factors, which are
 * recomputed (not stored from a forward pass).  Needs
 * ndg_plan_enable_adjoint once per plan (allocates its workspace).
 *   nbar[n]     device, cotangent of density (caller order)
 *   vbar[n]     device output (caller order, overwritten)
 * Errors: as ndg_solve; NDG_EINVAL if the adjoint was not enabled.
 */
ndg_status ndg_density(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                       const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                       const double* cE, double* density, ndg_precision prec, void* stream);
ndg_status ndg_plan_enable_adjoint(ndg_plan* plan);
ndg_status ndg_density_vjp(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                           const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                           const double* cE, const double* nbar, double* vbar, ndg_precision prec,
                           void* stream);

/* ndg_density_vjp_noalloc: ndg_density_vjp for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, same kernels and same result; the
 * per-energy partials of a batch live in a file-scope device buffer of 4 Mi
 * doubles (32 MiB, one per GPU, held until the process ends) instead of the
 * plan's adjoint workspace, and the call allocates nothing (the plan and its
 * adjoint workspace, enabled beforehand, are inputs).  Calls that overlap on
 * one GPU race on that buffer.  Errors: as ndg_density_vjp; NDG_EINVAL when
 * n x min(nE, max_batch) exceeds 4 Mi, NDG_EHIP if the buffer's device
 * address cannot be obtained. */
ndg_status ndg_density_vjp_noalloc(ndg_plan* plan, int32_t nE, const double* E, double eta,
                                   const double* V, const ndg_c128* const* sig_r,
                                   const ndg_c128* const* sig_less, const double* cE,
                                   const double* nbar, double* vbar, ndg_precision prec,
                                   void* stream);

/* ---------------------------------------------------------------------------
 * Newton step of the Schroedinger-Poisson problem (self-consistency of the
 * potential with the density, the motivation for repeated solves in
 * Section 1), using the density's vector-Jacobian product.
 *
 * With a symmetric positive definite discrete Poisson operator K on the
 * sites, a coupling beta and a background density n_D:
 *   F(V) = K V - beta (n(V) - n_D),  J = dF/dV = K - beta chi,  chi = dn/dV,
 * ndg_poisson_newton_step returns delta with J delta = -F(V) by conjugate
 * gradients; each iteration applies chi through ndg_density_vjp's solves,
 * which is exact when chi is symmetric: in equilibrium (one chemical
 * potential for all contacts; exactly at eta = 0), where chi is the Hessian
 * of the grand potential and J is positive definite.  Out of equilibrium it
 * is a Newton-like step with the symmetrized response.
 *   E, eta, V, sig_r, sig_less, cE   as ndg_density (V: the current
 *                                      potential, device [n], not NULL)
 *   k_rowptr[n+1] (int64), k_col[k_nnz] (int32), k_val[k_nnz]   device CSR
 *                     of K in the caller's site order (row ranges outside
 *                     [0, k_nnz) and columns outside [0, n) are ignored)
 *   beta, nd[n]       coupling and device background density
 *   cg_tol, cg_max_iter   stop when ||r|| <= cg_tol ||F|| or after
 *                     cg_max_iter iterations (each one density VJP)
 *   delta[n]          device output (the caller updates V += delta)
 *   res_norm          host output or NULL: ||F(V)||_2
 *   cg_iterations, cg_residual   host outputs or NULL: iterations run,
 *                     final ||r|| / ||F||
 * Needs ndg_plan_enable_adjoint (its workspace holds the vectors).  Runs on
 * `stream` and synchronizes it once per iteration (dot products).
 * Errors: NDG_EINVAL, NDG_EHIP, NDG_ENOTSPD (see above).
 */
ndg_status ndg_poisson_newton_step(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                                   const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                                   const double* cE, const int64_t* k_rowptr, const int32_t* k_col,
                                   const double* k_val, int64_t k_nnz, double beta, const double* nd,
                                   double cg_tol, int32_t cg_max_iter, double* delta, double* res_norm,
                                   int32_t* cg_iterations, double* cg_residual, void* stream);

/* ---------------------------------------------------------------------------
 * Batched solve of several devices (plans) of uneven sizes in one launch.
 *
 * ndg_batch_solve captures, on its first call with a given argument set, one
 * batch of energies (each plan's max_batch) of every plan into one HIP graph
 * -- one branch per device, so the devices' level-by-level kernels run
 * concurrently -- whose first energies live in device memory and are
 * advanced by the graph's last node.  A second graph holds the resets of
 * those counters and then one copy of the batch graph per batch the longest
 * energy range needs, in sequence (each plan's workspace stays that of one
 * batch), so one call is one graph launch on `stream` (if that graph cannot
 * be built, the batch graph is launched once per batch instead; see
 * ndg_batch_launches).  Later calls with identical arguments relaunch the
 * instantiated graph.  Each args[i] holds the arguments ndg_solve
 * takes for plans[i] (device pointers; the growth pointer may be NULL).  The
 * plans must be distinct, on one device, and have profiling switched off.
 * The graph is re-captured whenever a pointer, nE, eta or the precision
 * differs from the cached set; the contents of the buffers may change
 * freely between calls.  Capturing allocates no device memory.  `stream`
 * must not be the legacy NULL stream (capture needs a created stream).
 * Errors: NDG_EINVAL (bad arguments), NDG_EHIP (capture or launch failed).
 */
typedef struct ndg_batch ndg_batch;
typedef struct {
  int32_t nE;
  const double* E;
  double eta;
  const double* V;
  const ndg_c128* const* sig_r;     /* host array of ncontacts device pointers */
  const ndg_c128* const* sig_less;
  ndg_c128* diag_gr;
  ndg_c128* diag_gless;
  ndg_c128* diag_ggreater;
  double* growth;
} ndg_solve_args;

ndg_status ndg_batch_create(int32_t nplans, ndg_plan* const* plans, ndg_batch** out);
/* Waits for all work on the batch's device (graph replays still in flight),
 * then frees the batch; the plans are the caller's and stay.  NULL is a no-op. */
ndg_status ndg_batch_destroy(ndg_batch* batch);
ndg_status ndg_batch_solve(ndg_batch* batch, const ndg_solve_args* args, ndg_precision prec,
                           void* stream);
/* Graph launches the last ndg_batch_solve on `batch` issued: 1 when the whole
 * energy range ran as one graph, else the number of batches (0 before the
 * first solve or for NULL). */
int32_t ndg_batch_launches(const ndg_batch* batch);

/* Status word of the last solves on this plan (call after synchronising the
 * stream).  *code = NDG_OK, NDG_ESINGULAR (a pivot of magnitude 0 in a
 * cluster inverse) or NDG_ENONFINITE; *energy and *cluster identify the first
 * fault recorded (-1 if none).  Reading clears the word. */
ndg_status ndg_plan_status(ndg_plan* plan, int32_t* code, int32_t* energy, int32_t* cluster);

/* Test access: copies one stored block of the most recent batch of energies
 * to host memory.  which: 0 = pivot inverse (s x s), 1 = Psi (s x b),
 * 2 = the cluster's rows of the G^r front over [i, B_i], i.e. [G_ii, G_{i,B}]
 * (s x f), 3 = the same for G^< (s x f); energy indexes the last batch
 * (0 .. batch-1).  Row-major, host `out` of s*s / s*b / s*f entries.  For a
 * leaf cluster (no children) with f <= 64 only the diagonal of G_ii is
 * stored (nothing reads the rest).  Synchronises the device. */
ndg_status ndg_plan_export_block(ndg_plan* plan, int32_t which, int32_t energy, int32_t cluster,
                                 ndg_c128* out);

/* Per-kernel timing.  With profiling enabled the plan records a HIP event
 * pair around every kernel launch of ndg_solve on the launch's stream; the
 * statistics hold, per launch group (kernel, tree level, size class), the
 * number of launches, the summed event time and the algorithmic work of
 * those launches: flops (8 real flops per complex multiply-add, Section
 * 4.1's counts) and bytes (each input block read once, each output block
 * written once).  Each launch is credited with its own group's work; the
 * flops of all groups of one phonon-free solve sum to 8 ndg_info.ops_total
 * per energy.  ndg_plan_set_profiling: mode 0 off, 1 on (the G^< extraction
 * and the contact chains run on side streams, overlapping the G^r
 * extraction, so event times include co-running kernels), 2 on with every
 * launch on the caller's stream (each event time is the kernel's own).
 * ndg_plan_profile synchronises the device, copies at most `capacity`
 * entries, sets *count and clears the statistics. */
typedef struct {
  char name[32];
  int32_t height;     /* tree level of the launches (0 for the epilogue)                  */
  int32_t size_class; /* 0-2: fronts of at most 32, 48, 64 points (whole on chip); 3-6:
                         larger fronts with clusters of at most 16, 32, 64, 128 points; the
                         phonon kernels' tile classes 0-2: clusters of at most 16, 32, 64 */
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} ndg_kernel_stat;

/* Algorithmic work per energy of every launch group of a phonon-free solve
 * on this tree (host only, no device): the entries of ndg_plan_profile with
 * launches = 1, ms = 0, flops and bytes per energy.  Returns NDG_EINVAL (and
 * the first `capacity` entries) if capacity is too small. */
ndg_status ndg_symbolic_costs(const ndg_symbolic* sy, int32_t capacity, ndg_kernel_stat* out,
                              int32_t* count);

ndg_status ndg_plan_set_profiling(ndg_plan* plan, int32_t enable);
ndg_status ndg_plan_profile(ndg_plan* plan, int32_t capacity, ndg_kernel_stat* out,
                            int32_t* count);

const char* ndg_status_string(int32_t status);
const char* ndg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NDNEGF_H */
