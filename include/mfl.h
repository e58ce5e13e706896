/*
 * mfl.h -- C ABI of the matrix-free high-order Laplace library for AMD MI355X (gfx950).
 *
 * Method: Kronbichler & Wall, "A performance comparison of continuous and
 * discontinuous Galerkin methods with fast multigrid solvers" (arXiv 1611.03029).
 *   - operator: -div(kappa grad u) on hexahedra, continuous Q_k (Sec. 2.1, eq.
 *     poisson_fem) or symmetric interior penalty DG (Sec. 2.2, eq. poisson_dgsip with
 *     the boundary extension of eq. bc_dgsip), evaluated matrix-free by sum
 *     factorization with k+1 Gauss points per direction (Sec. 3, eq. mf_eval);
 *   - solver: conjugate gradients preconditioned by one geometric multigrid V-cycle
 *     with a Chebyshev-accelerated Jacobi smoother of degree 5 over
 *     [0.06, 1.2] * lambda_max, lambda_max from 15 CG iterations, embedding transfer,
 *     and a Chebyshev coarse solver with an a-priori error bound of 1e-3 (Sec. 4.1).
 *   - additions: the V-cycle may run in FP32 inside the FP64 outer CG; an adjoint
 *     solve and a per-cell gradient with respect to a cellwise kappa.
 *
 * Mesh: the cube [lo, lo + len]^3 (default the unit cube) with N_c^3 cells
 * (lexicographic, x fastest), either Cartesian or, on the unit cube, deformed by
 * x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1) through the isoparametric Q_k map at the
 * Gauss-Lobatto support points (Sec. 2).
 *
 * Boundary conditions: Dirichlet on all faces, Neumann on all faces (operator only), or
 * mixed as in the smooth-solution example of Sec. 4.3: Neumann on the faces x_e = lo and
 * Dirichlet on the faces x_e = lo + len.
 *
 * Vectors:
 *   - CG: full-length (k N_c + 1)^3 vector, lexicographic on the grid of per-cell
 *     Gauss-Lobatto positions, x fastest; boundary DoFs included.  The operator is the
 *     identity on the DoFs of Dirichlet faces and their columns are eliminated
 *     (symmetric positive definite on the whole space when some face is Dirichlet).
 *   - DG (SIPG): cell-major, N_c^3 (k+1)^3 values, local index i + n j + n^2 l
 *     (n = k+1), basis = Lagrange polynomials in the Gauss-Legendre points.
 *
 * Conventions:
 *   - every function returns MFL_OK (0) or a negative error code and never throws;
 *     mfl_last_error() describes the last failure of the calling thread;
 *   - all vector and field pointers are DEVICE pointers owned by the caller; the
 *     library never allocates device memory: its device state lives in a caller
 *     provided workspace (size from mfl_query), owned by the caller, which must
 *     stay valid and unmodified until mfl_destroy;
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work
 *     asynchronously on it, except where a function states that it synchronizes;
 *   - one handle must not be used from two host threads at the same time.
 */
#ifndef MFL_H
#define MFL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFL_OK 0
#define MFL_EINVAL (-1)        /* invalid argument (message in mfl_last_error) */
#define MFL_ENOCONV (-2)       /* iteration limit reached; outputs hold the last iterate */
#define MFL_EBREAKDOWN (-3)    /* CG breakdown: p^T A p <= 0, or NaN/Inf residual */
#define MFL_EHIP (-4)          /* a HIP runtime call failed */
#define MFL_EUNSUPPORTED (-5)  /* valid request outside the implemented combinations */

#define MFL_DISC_CG 0
#define MFL_DISC_SIPG 1
#define MFL_GEOM_CARTESIAN 0
#define MFL_GEOM_CURVED 1
#define MFL_BC_DIRICHLET 0
#define MFL_BC_NEUMANN 1
#define MFL_BC_MIXED 2        /* Neumann at x_e = lo, Dirichlet at x_e = lo + len (Sec. 4.3) */
#define MFL_F64 0
#define MFL_F32 1
#define MFL_DG_JACOBI_GAUSS 0  /* SIPG smoother: point Jacobi of the Gauss-point basis */
#define MFL_DG_JACOBI_GLL 1    /* ... point Jacobi of the GLL-Lagrange basis of each cell */
#define MFL_KAPPA_CELLWISE 0   /* kappa constant in each cell (the kappa_cells array, or 1) */
#define MFL_KAPPA_COSINE 1     /* ... times the position-dependent field of Sec. 4.3 (below) */

/* metric_mode */
#define MFL_METRIC_AUTO 0
#define MFL_METRIC_STORED 1
#define MFL_METRIC_ON_THE_FLY 2

typedef struct mfl_params {
  int degree;             /* polynomial degree k, 1..8 */
  int cells_per_dim;      /* N_c of the finest level, >= 1 */
  int min_level_cells;    /* cells per direction of the coarsest multigrid level (default 2) */
  int disc;               /* MFL_DISC_CG or MFL_DISC_SIPG */
  int geometry;           /* MFL_GEOM_CARTESIAN or MFL_GEOM_CURVED (CG only) */
  double curve_amp;       /* a of the deformation (default 0.1; ignored when Cartesian) */
  int bc;                 /* MFL_BC_DIRICHLET, MFL_BC_MIXED, or MFL_BC_NEUMANN (apply only) */
  double penalty_factor;  /* SIPG: sigma = penalty_factor (k+1)^2 / h (paper: 3 = d) */
  int cheb_degree;        /* smoother degree (Sec. 4.1: 5) */
  double cheb_lo;         /* lower end of the smoothing interval / lambda_max (0.06) */
  double cheb_hi;         /* upper end / lambda_max (1.2) */
  int eig_iters;          /* CG iterations of the lambda_max estimate (15) */
  double coarse_tol;      /* a-priori error bound of the coarse Chebyshev solver (1e-3) */
  int mg_precision;       /* MFL_F64 or MFL_F32: arithmetic of the V-cycle */
  int build_mg;           /* 0: finest-level operator only; 1: multigrid hierarchy */
  double domain_lo;       /* the mesh covers [domain_lo, domain_lo + domain_len]^3 (0) */
  double domain_len;      /* (1; curved meshes need the unit cube) */
  int dg_jacobi_basis;    /* SIPG multigrid: basis whose point Jacobi the Chebyshev smoother
                             uses.  MFL_DG_JACOBI_GLL (default): the Lagrange basis in the
                             Gauss-Lobatto points, applied to the Gauss-basis vectors as
                             T D'^{-1} T^T per cell (T = change of basis, D' = the operator's
                             diagonal in that basis); MFL_DG_JACOBI_GAUSS: diag(A)^{-1}. */
  int use_graphs;         /* 1 (default): the V-cycle is captured once as a HIP graph on an
                             internal stream and replayed on the caller's stream; 0: kernel
                             by kernel */
  int kappa_field;        /* MFL_KAPPA_CELLWISE (default) or MFL_KAPPA_COSINE: the cellwise
                             kappa is multiplied at every quadrature point x_q by the strongly
                             varying coefficient of Sec. 4.3, eq. (diffusivity_shell), read
                             with squared cosines so that it stays positive:
                               1 + kappa_field_amp prod_{e=1..3} cos^2(2 pi x_e + 0.1 e).
                             It is folded into the stored per-point metric, so it needs
                             geometry = MFL_GEOM_CURVED (curve_amp = 0 gives Cartesian cells
                             with a per-point metric) and the continuous discretization.
                             Every multigrid level evaluates it at its own quadrature points. */
  double kappa_field_amp; /* amplitude of that field (default 1e6, the paper's; >= 0) */
  int metric_mode;        /* curved CG meshes (Sec. 3: the geometry of non-affine cells):
                             MFL_METRIC_AUTO (default): on the fly with a cellwise kappa,
                             stored with the position-dependent kappa field;
                             MFL_METRIC_STORED: G_q = w_q det J_q J_q^{-1} J_q^{-T} per
                             quadrature point, computed at setup and read by every apply
                             (48 B per point in FP64 plus an FP32 copy);
                             MFL_METRIC_ON_THE_FLY: only the node displacement d of the
                             map x = X + d(X) (1,1,1) is stored (one value per DoF); every
                             apply forms grad d at the quadrature points by sum
                             factorization and G_q from J = h I + (1,1,1) (grad d)^T in
                             closed form.  Needs kappa_field = MFL_KAPPA_CELLWISE.
                             Ignored on Cartesian meshes. */
} mfl_params;

typedef struct mfl_context *mfl_handle;

/* Fill *p with the defaults above (k = 2, N_c = 8, CG, Cartesian, Dirichlet, MG in FP64,
 * cellwise kappa). */
int mfl_default_params(mfl_params *p);

/* Sizes for params p (host only, no GPU call): number of DoFs and cells of the finest
 * level, and the workspace size in bytes that mfl_setup needs.  Any output may be NULL.
 * Errors: MFL_EINVAL for an unsupported or inconsistent p (k outside 1..8, N_c not
 * reducible by halving to min_level_cells when build_mg = 1, SIPG with curved
 * geometry, multigrid with Neumann conditions on every face, a curved mesh off the unit
 * cube, a coarsest multigrid level with more than 20000 unknowns, the position-dependent
 * kappa field without curved CG geometry, an unknown metric_mode or the on-the-fly metric
 * with the position-dependent kappa field). */
int mfl_query(const mfl_params *p, int64_t *n_dofs, int64_t *n_cells, int64_t *workspace_bytes);

/* Build the level hierarchy in `workspace` (device memory, >= the queried size, 256-byte
 * aligned): geometry factors (Sec. 3: per-quadrature-point metric or node displacement
 * field on curved meshes, see metric_mode; one scalar per cell on Cartesian ones), Jacobi
 * diagonals, and for build_mg = 1 the
 * lambda_max estimates of every level (Sec. 4.1) and the coarse solver's eigenvalue range
 * (the extreme eigenvalues of the Jacobi-preconditioned coarsest operator, by Lanczos with
 * full reorthogonalization until both have converged to rounding).
 * kappa_cells: device array of n_cells doubles, each finite and > 0 (Sec. 2), or NULL for
 * kappa = 1.  Synchronizes `stream` (the kappa check and the eigenvalue estimates read
 * values back).  On success *out is a new handle.  Errors: MFL_EINVAL (params, NULL or
 * misaligned workspace, too small size, a kappa value that is not finite and positive, a
 * curved cell whose Jacobian determinant is not positive at some quadrature point),
 * MFL_EHIP. */
int mfl_setup(const mfl_params *p, void *workspace, int64_t workspace_bytes,
              const double *kappa_cells, void *stream, mfl_handle *out);

/* Replace the cellwise kappa (device, n_cells doubles, each finite and > 0) and rebuild
 * everything that depends on it: coarse-level kappa (mean of the 8 children), diagonals,
 * eigenvalue estimates.  A kappa equal bit for bit to the handle's current one (for example
 * the adjoint solve's call with the forward solve's kappa) is recognized on the device and
 * returns at once, without a rebuild.  Synchronizes `stream`.  Errors: MFL_EINVAL for a
 * NULL handle or array and for a kappa value that is not finite and positive (the handle is
 * then left unchanged), MFL_EHIP. */
int mfl_set_kappa(mfl_handle h, const double *kappa_cells, void *stream);

/* Number of levels (1 without multigrid); level 0 is the coarsest, num_levels-1 the finest. */
int mfl_num_levels(mfl_handle h);

/* Level description: cells per direction, DoFs, lambda_max estimate of D^{-1}A (0 on the
 * coarsest level), and for the coarsest level the eigenvalue range used by the coarse
 * solver and its number of Chebyshev steps (0 elsewhere).  Outputs may be NULL. */
int mfl_level_info(mfl_handle h, int level, int *cells_per_dim, int64_t *n_dofs,
                   double *lambda_max, double *coarse_lmin, double *coarse_lmax, int *coarse_steps);

/* dst = A src on `level` (-1 = finest) in precision dtype (MFL_F64: double vectors,
 * MFL_F32: float vectors with FP32 geometry factors).  Eq. (mf_eval) with sum
 * factorization; CG: identity on Dirichlet DoFs; SIPG: Sec. 2.2.  src and dst must not
 * overlap.  SIPG with an even number of points per direction (odd k) moves each cell's
 * lines in 16-byte accesses: src and dst must then be 16-byte aligned (MFL_EINVAL
 * otherwise; torch allocations are).  Asynchronous. */
int mfl_apply(mfl_handle h, int level, int dtype, const void *src, void *dst, void *stream);

/* out = diag(A) on `level` (-1 = finest), in dtype (CG: Dirichlet DoFs hold 1). */
int mfl_diagonal(mfl_handle h, int level, int dtype, void *out, void *stream);

/* Transfer between level l-1 (coarse) and l (fine), in the multigrid precision dtype:
 * direction 0: fine += P coarse (embedding, Sec. 4.1); direction 1: coarse = P^T fine.
 * CG: Dirichlet rows/columns of P are removed.  SIPG: the coarse cell's polynomial
 * evaluated at the Gauss points of its 8 children (block diagonal).  Asynchronous. */
int mfl_transfer(mfl_handle h, int level, int direction, int dtype, const void *src, void *dst,
                 void *stream);

/* z = one V(1,1)-cycle applied to r (finest level, FP64 in and out; the cycle itself runs
 * in the handle's mg_precision, the coarse solve always in FP64).  Asynchronous. */
int mfl_vcycle(mfl_handle h, const double *r, double *z, void *stream);

/* Solve A x = b by CG preconditioned with one V-cycle per iteration (Sec. 4.1), x_0 = 0,
 * until ||r||_2 <= rtol ||b||_2 or maxit iterations.  b, x: device, n_dofs doubles; x is
 * overwritten.  *iters and *final_rel_res (host pointers, may be NULL) receive the result.
 * Synchronizes once per iteration to test convergence.  Returns MFL_OK, MFL_ENOCONV (x,
 * iters and residual still valid) or MFL_EBREAKDOWN. */
int mfl_pcg_solve(mfl_handle h, const double *b, double *x, double rtol, int maxit, int *iters,
                  double *final_rel_res, void *stream);

/* b_i = int f phi_i with f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) (the right-hand side of the
 * manufactured solution sin sin sin), k+1 Gauss points, on the finest level (CG); zero on
 * Dirichlet DoFs.  Asynchronous. */
int mfl_rhs_sine(mfl_handle h, double *b, void *stream);

/* Right-hand side of the smooth-solution example (Sec. 4.3, eq. pois_analytic: a sum of
 * three Gaussians of width 1/5 centred at (-0.5,0.5,0.25), (-0.6,-0.5,-0.125),
 * (0.5,-0.5,0.5)) on the handle's Cartesian CG mesh and boundary conditions:
 *   b_i = int f phi_i + int_{Neumann faces} (grad u . n) phi_i - (A0 x0)_i  off the
 *         Dirichlet faces, b_i = x0_i on them,
 * f = -Laplace u with k+1 Gauss points per direction, x0 = u interpolated at the DoFs of
 * the Dirichlet faces (0 elsewhere), A0 = the operator without boundary conditions.  The
 * solution of A x = b then carries the Dirichlet data.  b: device, n_dofs doubles.
 * Uses the handle's work vectors (not concurrently with a solve on the same handle).
 * SIPG (Gauss-point basis): b_i = (f, psi_i) plus the data terms of the mirror extension
 * of eq. (bc_dgsip): int (2 sigma g_D psi_i - g_D n . grad psi_i) on Dirichlet faces and
 * int (grad u . n) psi_i on Neumann faces.
 * Errors: MFL_EUNSUPPORTED for curved meshes.  Asynchronous. */
int mfl_rhs_gaussians(mfl_handle h, double *b, void *stream);

/* Adjoint solve A lambda = dJdu with the same operator and preconditioner (A is symmetric);
 * the Dirichlet entries of the right-hand side are taken as zero.  Same outputs and errors
 * as mfl_pcg_solve. */
int mfl_adjoint_solve(mfl_handle h, const double *dJdu, double *lambda, double rtol, int maxit,
                      int *iters, double *final_rel_res, void *stream);

/* dJ/dkappa_c = -lambda_c^T A_c^{(kappa=1)} u_c for every cell c of the finest level (the
 * element operator of eq. mf_eval at unit kappa; Dirichlet entries of u and lambda are taken
 * as zero).  grad: device, n_cells doubles.  Asynchronous. */
int mfl_kappa_gradient(mfl_handle h, const double *u, const double *lambda, double *grad,
                       void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dst = A src for the continuous Q_k
 * operator on a Cartesian mesh (p->disc = MFL_DISC_CG, p->geometry = MFL_GEOM_CARTESIAN,
 * cellwise kappa), the same operator and kernels as mfl_apply, without a handle or a
 * workspace.  kappa_cells: device array of n_cells positive doubles (not checked), or NULL
 * for kappa = 1.  src, dst: device vectors of n_dofs values of dtype (must not overlap).
 * The work-group brick halo records (and kappa in FP32, or the unit kappa) live in a fixed
 * device array of MFL_NOALLOC_SCRATCH_BYTES per GPU that the library holds from its first
 * use on that GPU until the process ends; the call makes no allocation.  That array is
 * shared by every call on the GPU and keeps the last call's contents: calls that overlap on
 * one GPU (two streams, two host threads) race and must be serialized by the caller.  The
 * current device must be the stream's.  The first call on a device looks the array's
 * address up (hipGetSymbolAddress); make it outside graph capture.  Errors: MFL_EINVAL
 * (params, dtype, NULL or equal src/dst, a mesh whose halo records and kappa need more
 * than MFL_NOALLOC_SCRATCH_BYTES, e.g. Q6 on 64^3 cells), MFL_EUNSUPPORTED (SIPG, curved
 * geometry, the position-dependent kappa field), MFL_EHIP.  Asynchronous. */
#define MFL_NOALLOC_SCRATCH_BYTES (48ll << 20)
int mfl_apply_noalloc(const mfl_params *p, const double *kappa_cells, int dtype, const void *src, void *dst,
                      void *stream);

/* Timing of the operator's cell kernel (the dominant kernel of mfl_apply): enable = 1 starts
 * timing every cell-kernel launch that mfl_apply enqueues (up to 8192 launches) with a HIP
 * event pair that the launch's own dispatch records (hipExtLaunchKernelGGL: no packets are
 * added between kernels); enable = 0 stops, synchronizes on the recorded events and returns
 * the number of timed launches and their summed duration in milliseconds.  Outputs may be
 * NULL. */
int mfl_profile(mfl_handle h, int enable, int *launches, double *total_ms);

/* Release the handle (the workspace stays owned by the caller). */
int mfl_destroy(mfl_handle h);

/* Message of the last error on the calling thread ("" if none). */
const char *mfl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MFL_H */
