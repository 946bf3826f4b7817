/*
 * dgmg.h -- C ABI of libdgmg.so: matrix-free symmetric interior penalty (SIPG)
 * discontinuous Galerkin Laplacian on a uniform Cartesian mesh, the
 * overlapping vertex-patch Schwarz smoother by fast diagonalisation, and the
 * geometric multigrid V-cycle preconditioning CG, on one AMD MI355X (gfx950).
 *
 * Method: Cui & Kanschat, "Multilevel Interior Penalty Methods on GPUs".
 *
 * Problem (Sec. 2, eq. model): -kappa Laplace u = f on [0,1]^d, d = 2 or 3,
 * u = 0 on the boundary (imposed weakly by the Nitsche boundary terms of the
 * SIPG form).  Space (Sec. 2.1, Appendix A): discontinuous Q_k, Lagrange basis
 * on the k+1 Gauss-Lobatto points of each cell.  Bilinear form: eq.
 * (bilinear_form) with penalty gamma_F = sigma / h on every face (the paper's
 * gamma_e = k(k+1)(1/h+ + 1/h-) is sigma = 2k(k+1)), multiplied as a whole by
 * the coefficient kappa > 0.
 *
 * Mesh hierarchy (Sec. 3): level l = 0..L has N_l = 2^(l+1) cells per
 * direction (T_0 = one cell refined once); level operators are rediscretised.
 *
 * Vector layout (Sec. 4.1, cell-wise lexicographic numbering): every vector
 * argument is a contiguous device array of nrhs blocks of ndofs(l) = N_l^d (k+1)^d
 * entries; inside a block DoF = cell * (k+1)^d + local, cell = sum_i c_i N_l^i,
 * local = sum_i a_i (k+1)^i (x fastest in both).  Local node a in direction i
 * sits at the i-th coordinate c_i h + xi_a h, xi the Gauss-Lobatto points.
 *
 * Ownership: the caller owns every vector it passes (device memory, e.g. torch
 * tensors); the library owns its level vectors, Krylov workspace and tables,
 * allocated in dgmg_setup_levels and freed in dgmg_destroy.  Pointers must stay
 * valid until the enqueued work has completed.
 *
 * Streams: every call enqueues on the context stream (dgmg_set_stream; default
 * the null stream) and returns without waiting, except dgmg_pcg_solve, which
 * reads the residual norm back once per iteration and returns on completion,
 * and dgmg_node_coords, which is host-only.
 *
 * Errors: every entry point returns a dgmg_status; nothing throws across the
 * ABI.  Argument errors are reported before any device work; the message of
 * the last failure is available from dgmg_last_error.  One context per host
 * thread: a context is not safe for concurrent calls.
 */
#ifndef DGMG_H
#define DGMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgmg_ctx dgmg_ctx;

typedef enum {
  DGMG_OK = 0,
  DGMG_ERR_ARG = -1,           /* invalid argument (null pointer, bad size/level, NaN/Inf input) */
  DGMG_ERR_ALLOC = -2,         /* device allocation failed */
  DGMG_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
  DGMG_ERR_NOT_CONVERGED = -4, /* pcg reached maxit; iters/relres are still filled */
  DGMG_ERR_BREAKDOWN = -5,     /* pcg found p^T A p <= 0 or a non-finite scalar */
  DGMG_ERR_STATE = -6          /* call out of order (e.g. before dgmg_setup_levels) */
} dgmg_status;

enum { DGMG_FP64 = 64, DGMG_FP32 = 32 };

/* Local space and residual of the vertex-patch smoother (Sec. 3.1, Alg. 1).
 * Dirichlet kernel (V_j drops the patch-boundary nodes on interior faces):
 * EXACT uses (b - A x) restricted to V_j, i.e. it adds the coupling of V_j to
 *   the traces of the face-neighbour cells outside the patch; the smoother is
 *   then an exact multiplicative subspace correction and the V-cycle symmetric.
 * LOCAL is the paper's kernel with its inconsistent residual: only the patch
 *   cells are read and, on the patch's interior outer faces, the consistency
 *   term -[[u]].{grad v} of the form (which does not vanish on V_j) is left
 *   out altogether, so the residual is off by the jump of u there (not for
 *   CG: the smoother is not symmetric).
 * FULL is the Full kernel: V_j = every node of the patch cells.  Its domain of
 *   dependence reaches into face-neighbour cells that other patches of the
 *   same colour update, so the residual is taken once per colour (the global
 *   update of Sec. 3.1): every patch of a colour corrects from b - A x of the
 *   colour's entry state (additive inside a colour, multiplicative across
 *   colours; the V-cycle stays symmetric).  The library keeps a second copy of
 *   x per level for it.
 * CLAMPED is the clamped kernel: V_j = patch functions whose value and normal
 *   derivative vanish on the patch faces inside the domain (faces on the
 *   domain boundary stay free), (2k-2)^d unknowns for an interior patch.  The
 *   face terms coupling V_j to outside cells vanish on this space, so the
 *   exact local residual needs only the patch cells.  Needs degree >= 3 (for
 *   k = 2 the clamped spaces do not cover Q_k and the V-cycle is singular). */
enum { DGMG_SMOOTH_EXACT = 0, DGMG_SMOOTH_LOCAL = 1, DGMG_SMOOTH_FULL = 2, DGMG_SMOOTH_CLAMPED = 3 };

/* Create a context for the problem above.  dim in {2,3}; 1 <= degree <= 7;
 * 1 <= finest_level with ndofs(L) < 2^40; penalty_sigma > 0 (the operator is
 * SPD for sigma above a k-dependent threshold; sigma = 2(k+1)^2 and 2k(k+1) are
 * both safe); kappa > 0.  Builds the host tables (1-D matrices, patch
 * eigenpairs) in FP64; no device work.  *out receives the context. */
dgmg_status dgmg_setup_mesh(int dim, int degree, int finest_level, double penalty_sigma,
                            double kappa, dgmg_ctx** out);

/* Allocate device tables and workspaces.  vcycle_precision: DGMG_FP64, or
 * DGMG_FP32 for the mixed form (V-cycle in FP32 inside FP64 CG, Sec. 5.2).
 * smoother_variant: DGMG_SMOOTH_EXACT, DGMG_SMOOTH_LOCAL, DGMG_SMOOTH_FULL or
 * DGMG_SMOOTH_CLAMPED.
 * nrhs_max >= 1 bounds the nrhs of every later call.  hip_stream: hipStream_t
 * or NULL. */
dgmg_status dgmg_setup_levels(dgmg_ctx* ctx, int vcycle_precision, int smoother_variant,
                              int nrhs_max, void* hip_stream);

dgmg_status dgmg_set_stream(dgmg_ctx* ctx, void* hip_stream);

/* Change kappa (A(kappa) = kappa A_1).  Host-only; takes effect for work
 * enqueued afterwards. */
dgmg_status dgmg_set_kappa(dgmg_ctx* ctx, double kappa);

/* CG preconditioning by a captured HIP graph: on (default), dgmg_pcg_solve
 * captures its V-cycle (CG residual -> CG direction workspace, for the
 * given nrhs) on first use on a library-owned stream and replays it every
 * iteration on the context stream; off, every kernel is launched from the
 * host.  Both give bitwise identical results.  A new kappa drops the graphs. */
dgmg_status dgmg_use_graphs(dgmg_ctx* ctx, int enable);

/* The V-cycle's bottom as a dense operator.  Below a level m the V-cycle
 * (Sec. 3: smoothing, restriction, the exact solve on level 0, prolongation,
 * smoothing) maps the level-m right-hand side linearly to the level-m
 * correction.  For m = the finest level below L with at most 8192 DoFs (none
 * for L = 1), dgmg_setup_levels runs the cycle from
 * level m on that level's unit vectors and keeps the resulting nd x nd matrix
 * (context precision; 134 MB for 3-D Q3, nd = 4096, in FP64; 512 MB for 3-D
 * Q4, nd = 8000, in FP64) together with 8 x 16 x nd partial sums; a V-cycle
 * for at most 16 right-hand sides then applies it as one product with the
 * matrix, scaled by kappa_setup / kappa (one right-hand side: a
 * matrix-vector product on the vector units; 2..16: matrix-core tiles, the
 * matrix read once for all of them); more right-hand sides keep the
 * kernels, which run them side by side.  Same linear map as the kernels,
 * other rounding order.  If the matrix cannot be allocated the kernels stay
 * in use.  enable = 0 switches back to the kernels, 1 (default) to the
 * matrix; drops the captured graphs.  dgmg_dense_bottom_level returns m, or
 * -1 when no matrix was built. */
dgmg_status dgmg_use_dense_bottom(dgmg_ctx* ctx, int enable);
int dgmg_dense_bottom_level(const dgmg_ctx* ctx);

/* Sizes: cells per direction and DoFs per right-hand side of a level. */
long long dgmg_level_ndofs(const dgmg_ctx* ctx, int level);
int dgmg_level_cells(const dgmg_ctx* ctx, int level);
int dgmg_finest_level(const dgmg_ctx* ctx);

/* Host-only: physical coordinates of every DoF of a level, written to the host
 * array xyz[ndofs(level) * dim] as (x, y[, z]) per DoF in the layout above. */
dgmg_status dgmg_node_coords(const dgmg_ctx* ctx, int level, double* xyz);

/* y = A_l x (Sec. 2.2, patch-wise sum factorisation over the children of each
 * coarse cell; cell and face terms).  x, y: device [nrhs][ndofs(l)], must not
 * overlap.  0 <= level <= L. */
dgmg_status dgmg_apply_sipg(dgmg_ctx* ctx, int level, const double* x, double* y, int nrhs);
dgmg_status dgmg_apply_sipg_f32(dgmg_ctx* ctx, int level, const float* x, float* y, int nrhs);

/* y = M_l x, the mass matrix of the DG space (for load vectors b = M I_h f). */
dgmg_status dgmg_apply_mass(dgmg_ctx* ctx, int level, const double* x, double* y, int nrhs);

/* One step of the colourised multiplicative vertex-patch smoother S_l(x, b)
 * (Alg. 1) in place on x: for each of the 2^d colours (ascending, or
 * descending when reverse_colours != 0), every patch of the colour computes
 * its local residual on V_j and adds A[V_j,V_j]^{-1} r_j, the local inverse by
 * fast diagonalisation (Sec. 3.2, eqs. inverse2d/inverse3d/fast_inverse).
 * With the Dirichlet kernels V_j drops the patch-boundary nodes on interior
 * mesh faces and keeps those on the domain boundary; with the Full kernel it
 * is the whole patch (see DGMG_SMOOTH_FULL).  x, b: device [nrhs][ndofs(l)],
 * not overlapping.  1 <= level <= L. */
dgmg_status dgmg_smooth_patch(dgmg_ctx* ctx, int level, double* x, const double* b,
                              int reverse_colours, int nrhs);
dgmg_status dgmg_smooth_patch_f32(dgmg_ctx* ctx, int level, float* x, const float* b,
                                  int reverse_colours, int nrhs);

/* bc = P^T (b - A_l x): residual on level l restricted to level l-1 (Sec. 3;
 * P is the canonical embedding, P^T its transpose on dual vectors).
 * x, b: [nrhs][ndofs(l)], bc: [nrhs][ndofs(l-1)].  1 <= level <= L. */
dgmg_status dgmg_restrict_residual(dgmg_ctx* ctx, int level, const double* x, const double* b,
                                   double* bc, int nrhs);
dgmg_status dgmg_restrict_residual_f32(dgmg_ctx* ctx, int level, const float* x, const float* b,
                                       float* bc, int nrhs);

/* x += P xc: coarse correction from level l-1 prolongated into level l.
 * xc: [nrhs][ndofs(l-1)], x: [nrhs][ndofs(l)].  1 <= level <= L. */
dgmg_status dgmg_prolongate_add(dgmg_ctx* ctx, int level, const double* xc, double* x, int nrhs);
dgmg_status dgmg_prolongate_add_f32(dgmg_ctx* ctx, int level, const float* xc, float* x, int nrhs);

/* x = A_0^{-1} b on the coarsest level (Sec. 3): on T_0 the single interior
 * vertex patch covers the domain and keeps every node, so this is one exact
 * fast-diagonalisation solve.  b, x: [nrhs][ndofs(0)]. */
dgmg_status dgmg_coarse_solve(dgmg_ctx* ctx, const double* b, double* x, int nrhs);
dgmg_status dgmg_coarse_solve_f32(dgmg_ctx* ctx, const float* b, float* x, int nrhs);

/* x = P_L^{-1} b: one V-cycle on the finest level with zero initial guess, one
 * pre-smoothing step (colours ascending) and one post-smoothing step (colours
 * descending) per level (Sec. 3).  With vcycle_precision DGMG_FP32 the cycle
 * runs in FP32 (b rounded to nearest, x widened).  b, x: [nrhs][ndofs(L)]. */
dgmg_status dgmg_vcycle(dgmg_ctx* ctx, const double* b, double* x, int nrhs);
dgmg_status dgmg_vcycle_f32(dgmg_ctx* ctx, const float* b, float* x, int nrhs);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same V-cycle as dgmg_vcycle, same arguments, same kernels and the same
 * result, but the vectors it needs besides b and x -- b and x on levels
 * 0..L-1, for an FP32 V-cycle also the finest level's FP32 copies, for the
 * Full smoother the second copies of x on levels 1..L -- live in one
 * library-wide device array of 64 MiB per GPU (kept until the process ends)
 * instead of the context's own vectors.  No allocation, no graph.  Returns
 * DGMG_ERR_ARG (message from dgmg_last_error) when those vectors would not
 * fit in 64 MiB, e.g. a 3-D Q3 32^3 FP64 cycle holds at most 14 right-hand
 * sides.  Every call on one GPU shares that array: calls that overlap on one
 * GPU (two streams, two contexts, two threads) race and must be ordered by
 * the caller.  Nothing in the array needs to start at zero.  The dense bottom
 * operator (dgmg_use_dense_bottom), when in use, and its partial sums are the
 * context's own, allocated by dgmg_setup_levels. */
dgmg_status dgmg_vcycle_noalloc(dgmg_ctx* ctx, const double* b, double* x, int nrhs);

/* Solve A_L x = b by CG preconditioned with one V-cycle per iteration; FP64
 * outer iteration (residual, operator, inner products); beta by the flexible
 * (Polak-Ribiere) formula when the V-cycle runs in FP32.  Stops when
 * |r|_2 <= rtol |b|_2 for every right-hand side (per-RHS masks freeze the
 * converged ones).  use_initial_guess != 0 starts from x, else from 0.
 * iters[nrhs], relres[nrhs]: host arrays receiving the iteration count and
 * the final recursively updated relative residual of each right-hand side.
 * Blocks until done. */
dgmg_status dgmg_pcg_solve(dgmg_ctx* ctx, const double* b, double* x, int use_initial_guess,
                           double rtol, int maxit, int nrhs, int* iters, double* relres);

/* Solve A_L x = b (one right-hand side) by GMRES right-preconditioned with
 * one V-cycle per iteration, x0 = 0, no restart: the outer solver with which
 * the paper measures its fractional iteration counts (Sec. 3.3, Tables 1
 * and 2).  Flexible form (the preconditioned directions are stored), so the
 * FP32 V-cycle is allowed too; Arnoldi by classical Gram-Schmidt with one
 * re-orthogonalisation pass; Givens rotations on the host.  Stops when
 * |r_m|_2 <= rtol |b|_2 (the Arnoldi residual estimate) or after maxit
 * (1..1000) steps.  b, x: device [ndofs(L)].  *iters: steps taken;
 * hist: host [maxit + 1] receiving |r_i| / |b| for i = 0..*iters.  The
 * library keeps 2 maxit + 1 finest-level vectors for the Krylov basis (grown
 * on demand, freed in dgmg_destroy).  Blocks until done; returns
 * DGMG_ERR_NOT_CONVERGED (x, iters, hist filled) if maxit is reached. */
dgmg_status dgmg_gmres_solve(dgmg_ctx* ctx, const double* b, double* x, double rtol, int maxit,
                             int* iters, double* hist);

/* out[j] = a_j . b_j for each right-hand side j (deterministic two-stage
 * reduction); a, b: device [nrhs][ndofs(level)]; out: host [nrhs].  Blocks
 * until the result is on the host. */
dgmg_status dgmg_dot(dgmg_ctx* ctx, int level, const double* a, const double* b, int nrhs,
                     double* out);

/* Coefficient gradient of the differentiable solve u = A(kappa)^{-1} b with
 * A(kappa) = kappa A_1 (the adjoint method: for a loss L(u) and the adjoint
 * solution lambda = A(kappa)^{-1} dL/du, dL/dkappa = -lambda^T A_1 u, since
 * dA/dkappa = A_1 and the operator is symmetric).  lam, u: device
 * [nrhs][ndofs(L)] on the finest level.  per_rhs: host [nrhs] receiving
 * -lambda_j^T A_1 u_j for each right-hand side (may be NULL); total: host,
 * receiving their sum (in index order), the gradient with respect to the one
 * coefficient all right-hand sides share.  The operator apply (with kappa = 1),
 * the inner products, the sign and the sum run on the device; the library's
 * CG workspace holds A_1 u, so the call must not overlap a solve on the same
 * context.  Blocks until the values are on the host. */
dgmg_status dgmg_adjoint_dkappa(dgmg_ctx* ctx, const double* lam, const double* u, int nrhs,
                                double* per_rhs, double* total);

/* Host-only, no context: the reference (h = 1, kappa = 1) 1-D data of the
 * fast diagonalisation (Sec. 3.2, eq. fast_inverse) for patch type
 * t = 0 (interior), 1 (touches x = 0), 2 (touches x = 1), 3 (both; coarsest
 * level) of the local space of smoother_variant (Dirichlet for EXACT and
 * LOCAL, the whole patch for FULL, the clamped space for CLAMPED).  S: host
 * [(2k+2)*(2k+2)], S[p*(2k+2)+q] = value at patch node p of eigenvector q
 * (zero rows for dropped nodes, zero columns beyond dim V_j); lam: host [2k+2]
 * generalised eigenvalues, +inf in unused slots.  The eigenvectors satisfy
 * S^T M S = I. */
dgmg_status dgmg_patch_eigen(int degree, double sigma, int smoother_variant, int type, double* S,
                             double* lam);

/* Autotuner: for nrhs right-hand sides, time every workgroup shape (patches
 * per workgroup) and patch numbering (plain or XCD-aware) of the FP64
 * apply_sipg on the finest level, and of smooth_patch on every level 1..L in
 * the V-cycle's precision, where the shapes also choose whether a patch
 * fetches its b lines up front (fewer round trips, for latency-bound coarse
 * levels) or when needed (smaller cache footprint, for the finest level); use
 * the fastest from then on.  Timings run on the CG workspace and the level
 * vectors (their contents are overwritten).  cache_path (may be NULL) names a
 * JSON file of earlier results keyed by architecture, dim, degree, levels,
 * nrhs, precision, kernel and level; cached entries are used without timing
 * and new ones added.  report (may be NULL): host buffer receiving one line
 * per decision.  Drops captured V-cycle graphs. */
dgmg_status dgmg_autotune(dgmg_ctx* ctx, int nrhs, const char* cache_path, char* report,
                          int report_len);

const char* dgmg_last_error(const dgmg_ctx* ctx);
dgmg_status dgmg_destroy(dgmg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DGMG_H */
