/*
 * fosb.h -- C ABI of the MI355X (gfx950) FOSB hot path.
 *
 * The library computes the second moment of the shape derivative of the
 * current on a perfectly conducting (PEC) scatterer with the first-order sparse
 * boundary element method (arXiv 2308.01457): dense Galerkin EFIE matrices on
 * RWG elements per mesh level, the two-sided solves Z_l1 Sigma Z_l2^H = C_l1l2
 * over the combination technique's level pairs, and the far-field variance.
 *
 * Conventions shared by every entry point
 *   - Complex arrays are interleaved (re, im) and row-major; complex128 unless
 *     stated.  Sizes and leading dimensions are int64_t, in elements.
 *   - "device" pointers are HIP device memory owned by the caller (typically
 *     torch tensors); they must stay valid until the context's stream has run
 *     the enqueued work.  "host" pointers are read during the call only.
 *   - Handles (context, mesh, level) are owned by the library until *_destroy.
 *     The library allocates its own O(N) tables (a MIXED level also keeps the
 *     inverses of the 256 x 256 diagonal blocks of its factors, 4 KiB per
 *     unknown) and work buffers (O(N*nrhs) for solves, up to 2 GiB for the
 *     assembly's two column bands) on the context's device; O(N^2) matrices are
 *     always caller buffers.  These device blocks come from a caching pool
 *     per context (and per stream the context creates): a released block is
 *     kept and handed out again, so once a pass has run, repeating it on
 *     shapes of the same sizes makes no device allocation and no hipFree
 *     (fosb_context_memory counts them; fosb_context_trim returns the cache
 *     to the device).  fosb_level_workspace_size gives a level's own bytes,
 *     and calls that build levels check, on the host and before any launch,
 *     that the device can still hold what they need (FOSB_E_OOM otherwise).
 *   - All work is enqueued on the context's stream.  Calls that must inspect a
 *     device result (pivot breakdown, refinement convergence) synchronise that
 *     stream before returning.
 *   - Errors: every call returns a fosb_status; nothing throws or aborts across
 *     the ABI.  Arguments are validated on the host before any launch.  On an
 *     error the outputs are unspecified (except FOSB_E_NOCONV, see below) and
 *     fosb_last_error() returns a message (thread-local).
 *
 * Mesh and basis conventions (paper: Galerkin section, planar triangulations):
 *   local edge a of triangle t is opposite vertex F[t][a]; edges are numbered in
 *   first-visit order scanning t = 0..nt-1, a = 0,1,2; the triangle that visits
 *   an edge first is T+, the other T-; the RWG function of an edge of length l
 *   is +l/(2A+) (x - p+) on T+ and -l/(2A-) (x - p-) on T- (p = free vertex).
 */
#ifndef FOSB_H
#define FOSB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fosb_context fosb_context;
typedef struct fosb_mesh fosb_mesh;
typedef struct fosb_level fosb_level;
typedef struct fosb_lowrank fosb_lowrank;

typedef enum fosb_status {
  FOSB_OK = 0,
  FOSB_E_INVALID = 1,     /* bad argument or invalid mesh                       */
  FOSB_E_SINGULAR = 2,    /* exactly zero pivot; fosb_last_error names its index */
  FOSB_E_NOCONV = 3,      /* refinement did not reach its tolerance; outputs hold
                             the last iterate and fosb_stats the achieved values  */
  FOSB_E_WORKSPACE = 4,   /* a caller buffer / leading dimension is too small    */
  FOSB_E_OOM = 5,         /* device allocation failed                            */
  FOSB_E_DEVICE = 6,      /* HIP runtime error                                   */
  FOSB_E_UNSUPPORTED = 7  /* valid request this build does not implement         */
} fosb_status;

typedef enum fosb_precision {
  FOSB_PREC_FP64 = 0,  /* complex128 LU and solves                                */
  FOSB_PREC_MIXED = 1  /* complex64 LU on FP32 MFMA + FP64 iterative refinement   */
} fosb_precision;

/* Covariance M2[v_r](x, y) of the scalar perturbation amplitude, r = |x - y|. */
typedef enum fosb_cov_kind {
  FOSB_COV_GAUSSIAN = 0,   /* sigma^2 exp(-r^2 / (2 ell^2))                        */
  FOSB_COV_MATERN32 = 1,   /* sigma^2 (1 + sqrt3 r/ell) exp(-sqrt3 r/ell)          */
  FOSB_COV_CONSTANT = 2,   /* sigma^2 (random change of scale)                     */
  FOSB_COV_NORMAL_DOT = 3  /* sigma^2 n(x).n(y) (rigid translation, c ~ N(0,s^2 I)) */
} fosb_cov_kind;

/* How the scalar amplitude v_r becomes the normal velocity v_n. */
typedef enum fosb_field {
  FOSB_FIELD_RADIAL = 0,   /* v = v_r x/|x|, v_n = v_r (x/|x|).n                   */
  FOSB_FIELD_NORMAL = 1,   /* v_n = v_r                                            */
  FOSB_SD_STREAMED = 16    /* flag for fosb_level_create_pmchwt: keep no shape-
                              derivative weights, recompute them by source bands
                              where the low-rank route needs them               */
} fosb_field;

/* Boundary integral equation of a level. */
typedef enum fosb_formulation {
  FOSB_FORM_EFIE = 0,    /* PEC: EFIE on RWG, N = number of edges                 */
  FOSB_FORM_PMCHWT = 1   /* dielectric: PMCHWT on RWG, N = 2 x edges, [J; M]      */
} fosb_formulation;

/* How a level's matrix was factored (fosb_level_factorization). */
typedef enum fosb_factorization {
  FOSB_FACTOR_LU = 0,    /* partial (tournament) pivoting at the level's precision */
  FOSB_FACTOR_SYM = 1    /* MIXED levels: the symmetric FP32 factorisation
                            without pivoting described for fosb_opts.lu_pivoting */
} fosb_factorization;

typedef struct fosb_cov {
  int32_t kind;   /* fosb_cov_kind                                                */
  int32_t pad;
  double sigma;   /* amplitude (standard deviation), >= 0                          */
  double ell;     /* correlation length, > 0 (ignored by CONSTANT, NORMAL_DOT)     */
} fosb_cov;

typedef struct fosb_opts {
  int32_t n_gauss_singular; /* Gauss-Legendre points per dimension of the
                               Sauter-Schwab rules on touching pairs (1..12; 5)   */
  int32_t ir_max_sweeps;    /* refinement sweeps of the MIXED path (0..50; 10)     */
  double ir_tol;            /* target relative error of refined solves (1e-10):
                               after corrections of relative size r_{k-1}, r_k
                               (r_0 = 1) the error is estimated as r_k^2/r_{k-1} */
  int32_t certify;          /* 0 (default) or 1: also report, in fosb_stats, the
                               backward error of every refined solve (one more
                               FP64 residual product per solve), a 1-norm
                               condition estimate and the growth factor of every
                               level built (a few extra solves per level)       */
  int32_t lu_pivoting;      /* MIXED levels' FP32 factorisation: 0 (default) uses
                               the matrix's symmetry when N >= 2048 and
                               max|Z - Z^T| <= 1e-5 max|Z| (the EFIE matrix is
                               complex symmetric up to quadrature; for PMCHWT the
                               test and the factorisation apply to S Z with
                               S = diag(I, -I) on the [J; M] halves, which is
                               symmetric, and the solves use Z^{-1} = (S Z)^{-1} S):
                               no pivoting, U = D L^T from the multipliers,
                               trailing updates of the lower triangle only (about
                               half the flops), and partial (tournament) pivoting
                               instead when a pivot vanishes or the growth factor
                               exceeds 1e3; 1: always partial pivoting.  FP64
                               levels always pivot.                              */
} fosb_opts;

/* Counters of a call; accumulate over calls (zero-initialise before the first).
 * The three certificate fields are filled only with opts.certify = 1 and
 * stay 0 otherwise. */
typedef struct fosb_stats {
  int32_t ir_sweeps;        /* largest number of refinement sweeps used            */
  int32_t n_solves;         /* level-pair solves performed                         */
  double ir_rel_correction; /* largest final ||dX||/||X||                          */
  double backward_error;    /* largest normwise backward error of a refined solve,
                               ||B - op(Z) X||_F / (||Z||_F ||X||_F + ||B||_F), with
                               the FP64 matrix Z and the returned iterate X (MIXED
                               levels; FP64 levels keep no copy of Z)            */
  double kappa1;            /* largest estimate of ||Z||_1 ||Z^{-1}||_1 of a level
                               built (Hager-Higham 1-norm estimator: a lower bound,
                               within a small factor of the true value)           */
  double growth;            /* largest max|U_ij| / max|Z_ij| of a level built
                               (U: the upper LU factor, in its stored precision)  */
} fosb_stats;

/* Thread-local message of the last failing call ("" if none). */
const char* fosb_last_error(void);
/* Fills *opts with the defaults listed in fosb_opts. */
fosb_status fosb_opts_default(fosb_opts* opts);

/* ---------------------------------------------------------------- context */
/* Binds HIP device `device` and stream `hip_stream` (a hipStream_t; NULL = the
 * null stream).  The stream is borrowed, not destroyed. */
fosb_status fosb_context_create(int32_t device, void* hip_stream, fosb_context** out);
/* Waits for the context's stream, then frees it.  Meshes and levels created on
 * it and not yet destroyed are detached: every call rejects them with
 * FOSB_E_INVALID, and their destroy only frees their device memory. */
fosb_status fosb_context_destroy(fosb_context* ctx);
fosb_status fosb_context_synchronize(fosb_context* ctx);
/* Device-memory counters of the context and the streams it created: the
 * number of device allocations made so far, the bytes held in its caching
 * pools for reuse, and the bytes handed out and not yet released (any output
 * pointer may be NULL). */
fosb_status fosb_context_memory(fosb_context* ctx, int64_t* n_device_allocs, int64_t* bytes_cached,
                                int64_t* bytes_in_use);
/* Waits for the context's streams and returns every cached (unused) block to
 * the device. */
fosb_status fosb_context_trim(fosb_context* ctx);

/* ---------------------------------------------------------------- mesh */
/* Host-only check (no device work): V (host, nv x 3 float64), F (host, nt x 3
 * int32).  The surface must be closed, 2-manifold, consistently oriented with
 * outward normals (positive enclosed volume) and free of degenerate triangles;
 * otherwise FOSB_E_INVALID.  *n_edges receives the RWG count (may be NULL). */
fosb_status fosb_mesh_validate(const double* V, int64_t nv, const int32_t* F, int64_t nt,
                               int64_t* n_edges);
/* Validates as above, builds the RWG, quadrature and touching-pair tables and
 * uploads them to the context's device. */
fosb_status fosb_mesh_create(fosb_context* ctx, const double* V, int64_t nv, const int32_t* F,
                             int64_t nt, fosb_mesh** out);
fosb_status fosb_mesh_info(const fosb_mesh* mesh, int64_t* n_triangles, int64_t* n_edges,
                           int64_t* n_touching_pairs);
/* The mesh must outlive every level built on it (levels read its geometry). */
fosb_status fosb_mesh_destroy(fosb_mesh* mesh);

/* ---------------------------------------------------------------- assembly */
/* Galerkin EFIE matrix (problem setting: EFIO T_k, EFIE T_k j = gamma_D E^inc;
 * Galerkin section: Z u = b):
 *   Z[m][n] = int int G_k(x,y) [ -i k phi_m(x).phi_n(y) + (i/k) div phi_m div phi_n ],
 *   G_k = exp(i k |x-y|) / (4 pi |x-y|),
 * with the symmetric 6-point degree-4 rule on both triangles of non-touching
 * triangle pairs and Sauter-Schwab rules (opts->n_gauss_singular points per
 * dimension) on identical, edge- and vertex-adjacent pairs.  FP64 throughout.
 * Z: device, N x N complex128, row stride ldz >= N (N = number of edges).
 * k > 0, and k times the diagonal of the mesh's bounding box at most 1e5 (the
 * range of the kernel's own sin/cos of the phase), else FOSB_E_INVALID.
 * opts may be NULL (defaults).  The whole-pass entry points assemble through
 * the same path. */
fosb_status fosb_assemble(fosb_context* ctx, const fosb_mesh* mesh, double k, const fosb_opts* opts,
                          void* Z, int64_t ldz);

/* Galerkin PMCHWT matrix of the dielectric problem (problem setting: the
 * transmission problem, the MFIO K_k, the multitrace operators A_k and their
 * eta-scaled interior form, the PMCHWT equation; Galerkin section, first
 * moments), for the exterior total traces J = n x H~ (H~ = eta0 H, eta0 = 1)
 * and M = -n x E on RWG, tested with RWG:
 *   Z = [ T0 + eta T1     K0 + K1        ]   (2N x 2N, N = number of edges)
 *       [ -(K0 + K1)      T0 + T1 / eta  ]
 *   T_i  the EFIE matrix of fosb_assemble at k_i,
 *   K_i[m][n] = int int phi_m(x) . (grad_x G_ki(x,y) x phi_n(y)) dx dy (principal value),
 *   k1 = k0 sqrt(eps_r mu_r), eta = sqrt(mu_r / eps_r).
 * Same quadrature as fosb_assemble (the MFIO blocks of identical flat
 * triangles vanish).  FP64 throughout.  Z: device, 2N x 2N complex128, row
 * stride ldz >= 2N.  eps_r, mu_r real and > 0; k0 > 0 with k1 times the mesh's
 * bounding-box diagonal at most 1e5, else FOSB_E_INVALID.  opts may be NULL. */
fosb_status fosb_assemble_pmchwt(fosb_context* ctx, const fosb_mesh* mesh, double k0, double eps_r, double mu_r,
                                 const fosb_opts* opts, void* Z, int64_t ldz);

/* ---------------------------------------------------------------- level */
/* A mesh level ready for the tensor solves: LU factorisation with partial
 * pivoting (tournament pivoting per 32-column panel), the first moment
 * u = Z^{-1} b for each plane wave E^inc = p exp(i k d.x)
 * (b[m] = -int E^inc . phi_m), and the shape-derivative right-hand-side weights
 *   b'_m = int v_n [ (i/k) div j div phi_m - i k j . phi_m ]   (FOA section)
 * of each first moment j.
 *   precision FP64 : Z (device complex128, assembled, ldz) is overwritten by
 *                    its LU factors; Zlow must be NULL.
 *   precision MIXED: Z is kept read-only for FP64 refinement residuals and
 *                    must outlive the level; Zlow (device complex64, N x N,
 *                    ldzlow) receives the FP32 LU factors, which the level's
 *                    solves apply through the inverses of their 256 x 256
 *                    diagonal blocks (kept by the level).
 *                    Z may be NULL: the level then assembles the matrix in FP64
 *                    column bands straight into Zlow (rounded to complex64) and
 *                    re-assembles FP64 bands of Z for every refinement residual
 *                    (R -= Z X band by band, each band discarded), so no
 *                    complex128 copy of Z is ever stored: about 2x the
 *                    assembly and 2x the residual product per residual, and
 *                    half the device memory.  Such a level supports no adjoint
 *                    solve (FOSB_E_UNSUPPORTED); its certificate normalises
 *                    by the norms of the complex64 rounding of Z.
 * dirs, pols: host, n_dirs x 3 float64 (unit incidence direction, real
 * polarisation).  field: fosb_field.  On an exactly zero pivot returns
 * FOSB_E_SINGULAR. */
fosb_status fosb_level_create(fosb_context* ctx, const fosb_mesh* mesh, double k, int32_t precision,
                              void* Z, int64_t ldz, void* Zlow, int64_t ldzlow, const double* dirs,
                              const double* pols, int64_t n_dirs, int32_t field,
                              const fosb_opts* opts, fosb_level** out);
/* A dielectric level: the PMCHWT matrix Z of fosb_assemble_pmchwt (2N x 2N)
 * factored as for fosb_level_create (FP64, or MIXED with Zlow 2N x 2N
 * complex64; Z may not be NULL), and the first moments u = Z^{-1} b for each
 * plane wave E^inc = p exp(i k0 d.x), H~^inc = (d x p) exp(i k0 d.x):
 *   b = [e; h],  e[m] = int phi_m . E^inc,  h[m] = int phi_m . H~^inc.
 * The level keeps b: fosb_rhs_correlation and fosb_correlation on dielectric
 * levels with cov = NULL form the rank-one right-hand side C = b_l1 b_l2^H of
 * the paper's sphere validation (a second moment with M2[f] = f (x) f, whose
 * solution is u_l1 u_l2^H).
 * field >= 0 (FOSB_FIELD_RADIAL or FOSB_FIELD_NORMAL; mu_r must be 1, else
 * FOSB_E_UNSUPPORTED) also builds the shape-derivative weights W (FOA section,
 * the DE shape-derivative equation), 2N x 6 nt per incidence, kept by the
 * level: the derivative's traces solve Z [J'; M'] = W v for the amplitude v at
 * the 6-point nodes, with the data derived from the transmission conditions
 * (non-magnetic interior): jumps a = n x [E'] = grad_G(v_n [E_n]) x n and
 * b = n x [H~'] = i k0 (1 - eps_r) v_n E_t, [E_n] = (1 - 1/eps_r) E_n^0, and
 *   r_E = -eta <E_k1 b> - <H_k1 a> + 1/2 <n x a>,  r_H = -<H_k1 b> + <E_k1 a>/eta + 1/2 <n x b>
 * (<X>[m] = int phi_m . X, principal values; 6-point rule on non-touching
 * pairs with the source at the nodes, Sauter-Schwab with the amplitude's
 * quadratic interpolant on touching ones).  fosb_rhs_correlation and
 * fosb_correlation with a covariance then form C = W_l1 K W_l2^H (K at the
 * nodes of both levels; v_n = v_r (x/|x|).n for the radial field).  field = -1
 * builds none.  field | FOSB_SD_STREAMED stores no weights (2N x 6 nt x 16
 * bytes per incidence, 121 GB at 2N = 61440): the low-rank route
 * (fosb_lowrank_*) then forms W_l L_l from weights recomputed in source-triangle
 * bands of at most 2 GiB, and the dense covariance route returns
 * FOSB_E_UNSUPPORTED.  fosb_level_solve,
 * fosb_level_solve_adjoint, fosb_level_first_moment, fosb_two_sided_solve,
 * fosb_far_field_matrix and fosb_far_field_moments accept dielectric levels;
 * the entry points that need the shape-derivative weights of the PEC
 * problem (low-rank, adjoint-route and backward variance, near field,
 * whole-pass and batch entry points) return FOSB_E_UNSUPPORTED for them. */
fosb_status fosb_level_create_pmchwt(fosb_context* ctx, const fosb_mesh* mesh, double k0, double eps_r,
                                     double mu_r, int32_t precision, void* Z, int64_t ldz, void* Zlow,
                                     int64_t ldzlow, const double* dirs, const double* pols, int64_t n_dirs,
                                     int32_t field, const fosb_opts* opts, fosb_level** out);
/* Copies the shape-derivative weights of incidence dir of a dielectric level
 * built with field >= 0 into W (device, 2N x 6 nt complex128, row stride
 * ldw >= 6 nt; column 6 t + q is node q of triangle t, the radial factor
 * included); a level with streamed weights computes them into W.
 * FOSB_E_INVALID for a level without them. */
fosb_status fosb_level_sd_weights(fosb_context* ctx, const fosb_level* level, int64_t dir, void* W, int64_t ldw);
/* The level's formulation (fosb_formulation) and, for FOSB_FORM_PMCHWT, its
 * eps_r and mu_r (1 for EFIE levels).  Any output pointer may be NULL. */
fosb_status fosb_level_formulation(const fosb_level* level, int32_t* form, double* eps_r, double* mu_r);
/* The factorisation the level's construction kept (fosb_factorization) in
 * *kind: FOSB_FACTOR_SYM when the symmetric attempt succeeded, FOSB_FACTOR_LU
 * otherwise (FP64 levels, N < 2048, lu_pivoting = 1, or the attempt fell
 * back).  Host-only. */
fosb_status fosb_level_factorization(const fosb_level* level, int32_t* kind);
fosb_status fosb_level_info(const fosb_level* level, int64_t* n, int32_t* precision, int64_t* n_dirs);
/* Device bytes a level built on mesh with this precision and n_dirs
 * incidences keeps for its lifetime (permutation, diagonal-block inverses,
 * first moments, RHS weights, quadrature nodes), and the largest work buffer
 * bytes its construction and a refined solve with nrhs right-hand sides take
 * from the context's pool (nrhs <= 0: n_dirs).  Host-only. */
fosb_status fosb_level_workspace_size(const fosb_mesh* mesh, int32_t precision, int64_t n_dirs, int64_t nrhs,
                                      int64_t* level_bytes, int64_t* work_bytes);
/* The level's certificate from construction with opts.certify = 1 (0 otherwise):
 * the 1-norm condition estimate of Z and the growth factor of its factors, as
 * described for fosb_stats. */
fosb_status fosb_level_certificate(const fosb_level* level, double* kappa1, double* growth);
/* B <- Z^{-1} B (device complex128, N x nrhs, row stride ldb >= nrhs).  MIXED
 * levels refine in FP64 against the kept Z.  stats may be NULL. */
fosb_status fosb_level_solve(fosb_context* ctx, const fosb_level* level, void* B, int64_t ldb,
                             int64_t nrhs, fosb_stats* stats);
/* B <- Z^{-H} B (device complex128, N x nrhs, row stride ldb >= nrhs): the
 * adjoint solve behind the gradient of the two-sided solve (P Z = L U gives
 * Z^{-H} = P^T L^{-H} U^{-H}).  MIXED levels refine in FP64 against the kept
 * Z (residual B - Z^H X).  stats may be NULL. */
fosb_status fosb_level_solve_adjoint(fosb_context* ctx, const fosb_level* level, void* B, int64_t ldb,
                                     int64_t nrhs, fosb_stats* stats);
/* Copies the first-moment coefficients of direction dir into u (device, N complex128). */
fosb_status fosb_level_first_moment(fosb_context* ctx, const fosb_level* level, int64_t dir, void* u);
fosb_status fosb_level_destroy(fosb_level* level);

/* ---------------------------------------------------------------- tensor equation */
/* RHS correlation C = E[b'_l1 b'_l2^H] = Wgt_l1 K Wgt_l2^H (FOA section,
 * second-moment tensor equation; combination-technique sub-systems), with K
 * the covariance of the amplitude at the quadrature nodes of both levels.
 * C: device, N1 x N2 complex128, row stride ldc >= N2.  dir selects the
 * incidence (first moment) of both levels.  Dielectric levels: with
 * cov = NULL the rank-one C = b_l1 b_l2^H of their right-hand sides (sphere
 * validation of the DE second moment, M2[f] = f (x) f); with a covariance
 * (levels built with shape-derivative weights) C = W_l1 K W_l2^H. */
fosb_status fosb_rhs_correlation(fosb_context* ctx, const fosb_level* l1, const fosb_level* l2,
                                 const fosb_cov* cov, int64_t dir, void* C, int64_t ldc);
/* In place: C (N1 x N2) <- Sigma with Z1 Sigma Z2^H = C, i.e. the sub-system
 * (Z_l1 (x) conj Z_l2) Sigma = C of the combination technique. */
fosb_status fosb_two_sided_solve(fosb_context* ctx, const fosb_level* l1, const fosb_level* l2,
                                 void* C, int64_t ldc, fosb_stats* stats);
/* Hermitian-reduced combination-technique index set Lambda_H(L0, L):
 * pairs (l1 >= l2) with l1 + l2 = L + L0 (sign +1) or L + L0 - 1 (sign -1),
 * mult = 2 when l1 != l2 (the transposed pair is the conjugate transpose).
 * Arrays (host) must hold L - L0 + 1 entries; *n_pairs receives the count.
 * Order: sign +1 first, then decreasing l1. */
fosb_status fosb_ct_pairs(int32_t L0, int32_t L, int32_t* l1, int32_t* l2, int32_t* sign,
                          int32_t* mult, int32_t* n_pairs);
/* All Sigma blocks of Lambda_H for direction dir.  levels[i] is level L0 + i
 * (n_levels = L - L0 + 1); blocks[p] (device, N_l1 x N_l2 complex128, row
 * stride ldb[p]) receives the block of pair p in fosb_ct_pairs order.
 * Dielectric levels take cov = NULL (rank-one right-hand sides) or, when built
 * with shape-derivative weights, a covariance. */
fosb_status fosb_correlation(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                             int32_t L0, int32_t L, const fosb_cov* cov, int64_t dir,
                             void* const* blocks, const int64_t* ldb, fosb_stats* stats);

/* ---------------------------------------------------------------- far field */
/* Far-field map of a level (problem setting, far-field expansion):
 *   F_c(x) = sum_m FF[c*n_a + i][m] u_m,  FF = -i k (I - x x^T) int phi_m(y) exp(-i k x.y) dy;
 * for a dielectric level (u = [J; M], exterior field E_k0 J - H_k0 M)
 *   FF = [ i k0 (I - x x^T) A_m  |  -i k0 x x A_m ],  A_m = int phi_m(y) exp(-i k0 x.y) dy.
 * xhat: host, n_a x 3 unit vectors.  FF: device, (3 n_a) x N complex128. */
fosb_status fosb_far_field_matrix(fosb_context* ctx, const fosb_level* level, const double* xhat,
                                  int64_t n_a, void* FF);
/* Combination-technique far-field variance (problem setting: far-field
 * expansion and RCS; combination-technique sub-systems)
 *   var[c*n_a + i] = sum_{Lambda_H} sign mult Re (FF_l1 Sigma FF_l2^H)[(c,i),(c,i)]
 * (device, 3 n_a float64), from the blocks of fosb_correlation.  cor (device,
 * 3 x n_a x n_a complex128, may be NULL) receives the far-field correlation
 * between angles, per component c:
 *   cor[c][i][j] = sum_{Lambda_H} sign P[i][j] (l1 = l2), sign (P + P^H)[i][j] (l1 != l2),
 *   P = (FF_l1 Sigma FF_l2^H) restricted to component c,
 * a Hermitian matrix whose diagonal has real part var (the transposed pair of
 * Lambda contributes P^H).  mean_F (device, 3 n_a complex128, may be NULL)
 * receives the first-moment far field of the finest level. */
fosb_status fosb_far_field_moments(fosb_context* ctx, const fosb_level* const* levels,
                                   int32_t n_levels, int32_t L0, int32_t L, void* const* blocks,
                                   const int64_t* ldb, const double* xhat, int64_t n_a, int64_t dir,
                                   double* var, void* cor, void* mean_F);

/* The same combination-technique variance (and optional mean field) by the
 * adjoint route, without any Sigma block or pair solve.  The variance is
 * linear in the right-hand-side correlation C = Wgt_l1 K Wgt_l2^H (FOA
 * section, second-moment tensor equation; combination-technique
 * sub-systems), so
 *   var[r] = sum_{Lambda_H} sign mult Re sum_{q,q'} P_l1[r][q] K(x_q, y_q') conj(P_l2[r][q']),
 *   P_l = FF_l Z_l^{-1} Wgt_l  (3 n_a x Q_l, Q_l = 6 triangles),
 * with P_l from one adjoint solve Z_l^{-H} FF_l^H (3 n_a right-hand sides) per
 * level.  For 3 n_a well below N this replaces the pair solves (N_l2 and N_l1
 * right-hand sides per pair) by per-level solves; the covariance is formed
 * in row chunks of at most 2^26 entries and contracted by FP64 GEMMs.
 * Arguments and layouts as for fosb_far_field_moments_backward (var: device,
 * 3 n_a float64; mean_F: device, 3 n_a complex128, may be NULL); the levels
 * must still hold their factors.  Equals fosb_correlation followed by
 * fosb_far_field_moments up to rounding. */
fosb_status fosb_far_field_variance_adjoint(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                            int32_t L0, int32_t L, const fosb_cov* cov, const double* xhat,
                                            int64_t n_a, int64_t dir, double* var, void* mean_F, fosb_stats* stats);

/* ---------------------------------------------------------------- low-rank covariance */
/* Low-rank factor K ~ L L^T of the covariance on the quadrature nodes of a
 * level ladder (levels[i] = level L0 + i, coarse to fine; the nodes of all
 * levels, in that order, are the candidate points), for a second moment
 * whose right-hand-side correlation factors as C_l1l2 = (Wgt_l1 L_l1)
 * (Wgt_l2 L_l2)^H, so that Sigma_l1l2 = Y_l1 Y_l2^H with Y_l = Z_l^{-1} Wgt_l L_l:
 * one solve with rank right-hand sides per level instead of N_l2 + N_l1 per
 * pair (the paper's future-work remarks on low-rank covariance
 * representations; the Fichera experiment's covariance is separable).
 * Greedy pivoted Cholesky: starting from d = diag K, each step takes as pivot
 * p the lowest candidate index with d_p >= (1 - 1e-9) max d, forms the column
 * L[:, j] = (K(X, x_p) - L[:, :j] L[p, :j]^T) / sqrt(d_p), subtracts its
 * squares from d and sets d_p = 0; it stops once max d <= tol max(diag K) or
 * at max_rank columns.  The factor is exact on the pivots and bounded by the
 * remaining diagonal elsewhere.  FP64 throughout; device memory about
 * 8 max_rank (number of nodes) bytes.  The levels must outlive the handle.
 * Dielectric levels built with shape-derivative weights (stored or streamed)
 * take Wgt_l = their W (2N x 6 nt).
 * E_INVALID for bad arguments (max_rank 1..min(8192, nodes), 0 <= tol < 1). */
fosb_status fosb_lowrank_create(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                const fosb_cov* cov, int32_t max_rank, double tol, fosb_lowrank** out);
/* rank reached, residual (largest remaining diagonal entry / largest initial
 * one) and the pivots (host, rank int64 candidate indices; may be NULL). */
fosb_status fosb_lowrank_info(const fosb_lowrank* lr, int32_t* rank, double* residual, int64_t* pivots);
/* Y (device, N x rank complex128, row stride ldy >= rank) = Z^{-1} Wgt_dir L_l
 * for ladder level level_index (refined in FP64 on MIXED levels). */
fosb_status fosb_lowrank_factor(fosb_context* ctx, const fosb_lowrank* lr, int32_t level_index, int64_t dir, void* Y,
                                int64_t ldy, fosb_stats* stats);
/* CT far-field variance with the low-rank covariance (var: device, 3 n_a
 * float64, layout as fosb_far_field_moments):
 *   var[r] = sum_{Lambda_H} sign mult Re sum_k G_l1[r][k] conj(G_l2[r][k]),  G_l = FF_l Y_l.
 * L - L0 + 1 must equal the ladder's length. */
fosb_status fosb_far_field_moments_lowrank(fosb_context* ctx, const fosb_lowrank* lr, int32_t L0, int32_t L,
                                           const double* xhat, int64_t n_a, int64_t dir, double* var,
                                           fosb_stats* stats);
fosb_status fosb_lowrank_destroy(fosb_lowrank* lr);

/* Bytes of the per-GPU work array of fosb_far_field_moments_noalloc. */
#define FOSB_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* Allocation-free variant of fosb_far_field_moments, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, hosts
 * that forbid hipMalloc).  Same arguments, layouts and results (var, and
 * mean_F if not NULL; no angular correlation), computed by the same kernels,
 * except that the complex GEMMs neither split K nor time tile shapes, so the
 * values may differ from fosb_far_field_moments in the last bits.  The call
 * makes no device allocation and frees nothing: its far-field maps, products
 * and the copies of xhat and of the first moment live in a file-scope device
 * array of FOSB_NOALLOC_SCRATCH_BYTES that each GPU holds from the first
 * fosb_context_create on it until the process ends.  The angles are processed
 * in chunks that fit that array; FOSB_E_WORKSPACE when a single angle does not
 * fit (3 (N_l1 + 2 N_l2) complex128 values of a pair, or 3 N_L + N_L for the
 * mean field, plus the 3 n_a angle coordinates).  Every call on one GPU uses
 * the same array and leaves its last contents there; var is cleared by a
 * kernel before it accumulates.  Calls that overlap on one GPU (other host
 * threads, other contexts or streams of the same device) race on the array
 * and must be serialised by the caller.  Synchronises the context's stream. */
fosb_status fosb_far_field_moments_noalloc(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                           int32_t L0, int32_t L, void* const* blocks, const int64_t* ldb,
                                           const double* xhat, int64_t n_a, int64_t dir, double* var, void* mean_F);

/* ---------------------------------------------------------------- near field */
/* Scattered field at field points off the surface (FOA section: the field's
 * shape derivative is E' = -E_k dj', the electric potential applied to the
 * trace's shape derivative; problem setting: E^sc = -E_k j):
 *   E^sc_c(x_p) = sum_m NF[c*n_p + p][m] u_m,
 *   E_k phi(x) = i k int G(x,y) phi(y) dy + (i/k) grad_x int G(x,y) div phi(y) dy,
 * 6-point rule on every triangle (accurate for points farther from the
 * surface than a few triangle sizes; points on the surface are singular).
 * points: host, n_p x 3 (1..65535).  NF: device, (3 n_p) x N complex128. */
fosb_status fosb_near_field_matrix(fosb_context* ctx, const fosb_level* level, const double* points, int64_t n_p,
                                   void* NF);
/* Combination-technique second moment of the field's shape derivative at the
 * field points:
 *   var[c*n_p + p] = sum_{Lambda_H} sign mult Re (NF_l1 Sigma NF_l2^H)[(c,p),(c,p)]
 * (device, 3 n_p float64), from the blocks of fosb_correlation, and mean_E
 * (device, 3 n_p complex128, may be NULL) the finest level's scattered field
 * there (the first moment).  Arguments otherwise as for fosb_far_field_moments. */
fosb_status fosb_near_field_moments(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels, int32_t L0,
                                    int32_t L, void* const* blocks, const int64_t* ldb, const double* points,
                                    int64_t n_p, int64_t dir, double* var, void* mean_E);

/* Adjoint of the combination-technique variance with respect to the
 * covariance parameters.  With upstream weights g = dvar (device, 3 n_a
 * float64, same layout as var) and S = sum_r g_r var_r:
 *   S = sum_{Lambda_H} sign mult sum_{q,q'} K(x_q, y_q') Re G[q][q'],
 *   G = P_l1^T diag(g) conj(P_l2),  P_l = FF_l Z_l^{-1} Wgt_l  (3 n_a x Q_l),
 * because var is linear in C = Wgt_l1 K Wgt_l2^H (FOA section, second-moment
 * tensor equation; combination-technique sub-systems).  P_l is formed from the
 * adjoint solve Z_l^{-H} FF_l^H, so one solve with 3 n_a right-hand sides per
 * level replaces the pair solves.  out (device, 3 float64) receives
 *   out[0] = dS/dsigma,  out[1] = dS/dell,  out[2] = S  (the adjoint-route value,
 * equal to sum_r g_r var_r of fosb_far_field_moments up to rounding).
 * levels and xhat (host, n_a x 3 unit vectors) as for fosb_far_field_moments;
 * the levels must still hold their factors.  Device scratch of about
 * 3 (Q_l1 + Q_l2) 3 n_a + min(Q_l1 Q_l2, 2^26) complex128 values per pair is
 * allocated by the context.  E_INVALID on bad arguments; E_NOCONV as for the
 * refined solves. */
fosb_status fosb_far_field_moments_backward(fosb_context* ctx, const fosb_level* const* levels,
                                            int32_t n_levels, int32_t L0, int32_t L, const fosb_cov* cov,
                                            const double* xhat, int64_t n_a, int64_t dir,
                                            const double* dvar, double* out, fosb_stats* stats);

/* ---------------------------------------------------------------- whole pipeline */
/* One pass of the hot path over a level ladder L0..L (levels[i] = level L0 + i,
 * coarse to fine): EFIE assembly into Z[i] (device, N_i x N_i complex128, row
 * stride ldz[i]; MIXED also needs Zlow[i], complex64, stride ldzlow[i], and
 * may pass Z[i] = NULL for levels that re-assemble, as for fosb_level_create),
 * factorisation, first moments and RHS weights of every level, the RHS
 * correlation and two-sided solve of every pair of fosb_ct_pairs(L0, L) into
 * blocks[p] (as fosb_correlation), and the far-field variance var (device,
 * 3 n_a float64, as fosb_far_field_moments) for incidence dir.  dir = -1
 * solves all n_dirs incidences together, their right-hand sides stacked:
 * blocks[p] is then N_l1 x (n_dirs N_l2) with incidence d in columns
 * d N_l2 .. (d+1) N_l2 (ldb[p] >= n_dirs N_l2), and var holds n_dirs
 * consecutive 3 n_a vectors.  The same
 * results as the step-by-step calls; the work is scheduled over two streams:
 * the finest level on the context's stream, the coarser levels and the pairs
 * among them concurrently on an auxiliary stream the context owns (a second
 * host thread drives it).  levels_out (may be NULL, else n_levels entries)
 * receives the level handles, owned by the caller; otherwise they are
 * destroyed.  Z buffers are overwritten (FP64: with the LU factors).  Errors
 * as for the step-by-step calls; outputs are unspecified on error. */
fosb_status fosb_second_moment(fosb_context* ctx, const fosb_mesh* const* meshes, int32_t n_levels,
                               int32_t L0, int32_t L, double k, int32_t precision, void* const* Z,
                               const int64_t* ldz, void* const* Zlow, const int64_t* ldzlow,
                               const double* dirs, const double* pols, int64_t n_dirs, int32_t field,
                               const fosb_cov* cov, int64_t dir, const double* xhat, int64_t n_a,
                               void* const* blocks, const int64_t* ldb, double* var,
                               const fosb_opts* opts, fosb_level** levels_out, fosb_stats* stats);

/* One shape of a batch: its level ladder (meshes[i] = level L0 + i, coarse to
 * fine, created on the batch's context), wavenumber, incidences (host, n_dirs
 * x 3 each), perturbation field, covariance and output: var (device, n_dirs
 * consecutive 3 n_a float64 vectors, as fosb_far_field_moments). */
typedef struct fosb_batch_shape {
  const fosb_mesh* const* meshes;
  int32_t n_levels, L0, L, field;
  double k;
  const double* dirs;
  const double* pols;
  int64_t n_dirs;
  fosb_cov cov;
  double* var;
} fosb_batch_shape;

/* The whole pass (as fosb_second_moment with every incidence stacked) for
 * many shapes of uneven sizes: n_workers host threads (1..16), each with its
 * own stream (created by the library, default priority), scratch and
 * grow-only Z / Zlow / block workspaces held by the context, take shapes in
 * order from a shared queue, so several shapes are in flight on the GPU at
 * once.  Per shape the results equal fosb_second_moment(dir = -1).  The
 * workspaces persist in the context (each worker holds its largest shape's
 * matrices).  Errors as for fosb_second_moment; on error the remaining shapes
 * are skipped and their var is unspecified. */
fosb_status fosb_second_moment_batch(fosb_context* ctx, const fosb_batch_shape* shapes, int64_t n_shapes,
                                     int32_t precision, const double* xhat, int64_t n_a,
                                     const fosb_opts* opts, int32_t n_workers, fosb_stats* stats);

/* ---------------------------------------------------------------- GEMM tile autotuner */
/* The complex GEMMs run one of several tile shapes (64x64, 64x32, 64x128,
 * 128x64 for complex64; 64x32, 64x64, 128x64 for complex128).  With tuning on
 * (the default) the first product of each size bucket (precision, operand
 * form, floor(log2) of M, N, K) times every shape on its real operands into
 * scratch output and keeps the fastest for the bucket; the table belongs to
 * the context and its auxiliary and worker streams.  The trailing update of
 * the blocked LU takes the 64x64 shape for its large complex64 products
 * without tuning.  All shapes give identical results, so tuning never changes
 * outputs.  mode: 0 off (built-in
 * shape: the first listed), 1 on, 2 on and forget the table, -1 query only.
 * n_entries (may be NULL) receives the number of tuned buckets. */
fosb_status fosb_autotune(fosb_context* ctx, int32_t mode, int32_t* n_entries);
/* Export of the tuned table, in increasing key order: up to capacity entries
 * into keys / variants (host arrays, may be NULL when capacity is 0);
 * *n_entries (required) receives the table's size.  A key packs the bucket:
 * bits 0-12 floor(log2 K), 13-25 floor(log2 N), 26-38 floor(log2 M), bit 39 set
 * for A^H products, bit 40 set for complex128.  A variant indexes the shape
 * list above for the key's precision. */
fosb_status fosb_autotune_table(fosb_context* ctx, int64_t* keys, int32_t* variants, int64_t capacity,
                                int64_t* n_entries);
/* Adds n entries (host arrays) to the table, replacing entries with equal
 * keys, so that a table exported from one run settles the same buckets in
 * another without timing.  A variant out of range for its key's precision,
 * or a key with bits above 40 set, gives FOSB_E_INVALID and loads nothing. */
fosb_status fosb_autotune_load(fosb_context* ctx, const int64_t* keys, const int32_t* variants, int64_t n);

/* ---------------------------------------------------------------- profiling */
/* Kernel classes timed by the profiler. */
typedef enum fosb_kernel_class {
  FOSB_K_GEMM_F64 = 0,      /* complex128 GEMM (LU updates, TRSM couplings, residuals) */
  FOSB_K_GEMM_F32 = 1,      /* complex64 GEMM (mixed-precision LU and solves)           */
  FOSB_K_ASSEMBLE = 2,      /* EFIE regular + singular pair integration and gather      */
  FOSB_K_PANEL = 3,         /* LU panel factorisation (tournament, swaps, L21)          */
  FOSB_K_TRSM_LEAF = 4,     /* diagonal-block inverse applications                      */
  FOSB_K_RHS = 5,           /* RHS correlation, weights, far-field kernels              */
  FOSB_K_GEMV = 6,          /* matrix times at most four columns (bandwidth-bound)      */
  FOSB_K_SPLITK_SUM = 7,    /* sum of the partial products of a split-K GEMM            */
  FOSB_K_COUNT = 8
} fosb_kernel_class;

/* on != 0: from now on every launch of an instrumented kernel on this context
 * is bracketed by HIP events (adds a few microseconds of host work per launch);
 * previous records are discarded.  on == 0: stop recording (records are kept). */
fosb_status fosb_profile_enable(fosb_context* ctx, int32_t on);
/* Synchronises the context's stream and returns, for kernel class `cls`, the
 * number of recorded launches, their summed device time (s) and the summed
 * algorithmic work of those launches: flops counts 8 per complex
 * multiply-add (GEMM) and bytes counts the operands each launch must move
 * at least once.  Any output pointer may be NULL. */
fosb_status fosb_profile_read(fosb_context* ctx, int32_t cls, int64_t* launches, double* seconds,
                              double* flops, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* FOSB_H */
