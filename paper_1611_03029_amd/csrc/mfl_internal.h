// Internal declarations of the matrix-free Laplace library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mfl.h"

namespace mfl {

constexpr int kMaxDegree = 8;
constexpr int kMaxN = kMaxDegree + 1;
constexpr int kMaxM = 2 * kMaxDegree + 1;   // fine points per coarse cell and direction
constexpr int kReduceBlocks = 1024;         // partial sums of the vector reductions

// One-dimensional tables of degree k (n = k+1 entries per direction), passed to the
// kernels by value so that fully unrolled loops read them through scalar loads.
//   S [q n + i] : GLL-Lagrange basis i at Gauss point q
//   Sd[q n + i] : derivative of GLL-Lagrange basis i at Gauss point q
//   D [q n + p] : derivative of Gauss-Lagrange basis p at Gauss point q (collocation)
//   M, K        : reference [0,1] mass and stiffness matrices of the GLL basis
//   Fv, Fd      : Gauss-Lagrange basis p and its derivative at xi = 0 (p) and xi = 1 (n + p)
//   w, gll, xg  : Gauss weights, GLL nodes, Gauss points on [0,1]
template <int N, typename T>
struct Tab {
  T S[N * N];
  T Sd[N * N];
  T D[N * N];
  T M[N * N];
  T K[N * N];
  T Fv[2 * N];
  T Fd[2 * N];
  T w[N];
  T gll[N];
  T xg[N];
};

// Even-odd form of an N x N matrix A that is centro-symmetric (A[N-1-q][N-1-i] = A[q][i])
// or centro-antisymmetric (= -A[q][i]), with H = N/2 and c = H the middle index (odd N):
//   ep[q][i] = (A[q][i] + A[q][N-1-i]) / 2,  op[q][i] = (A[q][i] - A[q][N-1-i]) / 2  (q, i < H)
//   ec[q] = A[q][c],  mid[i] = A[c][i] (i < H),  mid[H] = A[c][c].
// All 1D matrices of the Gauss/Gauss-Lobatto bases have this symmetry (the point sets
// are symmetric about 1/2), which halves the products of a 1D contraction (Sec. 3).
template <int N, typename T>
struct EO {
  static constexpr int H = N / 2;
  T ep[H * H];
  T op[H * H];
  T ec[H];
  T mid[H + 1];
};

template <int N, typename T>
struct EOTab {
  EO<N, T> M, K;   // reference mass and stiffness of the GLL basis (centro-symmetric)
  EO<N, T> S;      // GLL basis at the Gauss points (centro-symmetric)
  EO<N, T> D;      // Gauss-point collocation derivative (centro-antisymmetric)
};

template <int N, typename T>
EO<N, T> make_eo(const double *A) {   // A row-major N x N (row length N)
  EO<N, T> e{};
  constexpr int H = N / 2;
  for (int q = 0; q < H; ++q) {
    for (int i = 0; i < H; ++i) {
      e.ep[q * H + i] = T(0.5 * (A[q * N + i] + A[q * N + N - 1 - i]));
      e.op[q * H + i] = T(0.5 * (A[q * N + i] - A[q * N + N - 1 - i]));
    }
    e.ec[q] = (N % 2) ? T(A[q * N + H]) : T(0);
  }
  for (int i = 0; i <= H; ++i) e.mid[i] = (N % 2) ? T(A[H * N + i]) : T(0);
  return e;
}

// Embedding of the coarse GLL basis in the fine grid lines of one coarse cell:
// P[f (k+1) + i] = coarse basis i at the f-th of the 2k+1 fine points.  DG (Lagrange in
// the Gauss points): E[(s n + f) n + c] = coarse basis c at the f-th Gauss point of child
// s (the child covers [s/2, (s+1)/2] of the coarse cell).
struct TransferTab {
  double P[kMaxM * kMaxN];
  double E[2 * kMaxN * kMaxN];
};

struct Level {
  int Nc = 0;           // cells per direction
  int N1 = 0;           // CG grid lines per direction (k Nc + 1)
  int64_t ncells = 0;
  int64_t ndofs = 0;
  double h = 0.0;
  double *kappa64 = nullptr;
  float *kappa32 = nullptr;
  double *metric64 = nullptr;   // curved, stored metric: [cell][6][n^3], w_q det J J^{-1} J^{-T}
  float *metric32 = nullptr;
  double *disp64 = nullptr;     // curved, metric on the fly: node displacement d (x = X + d (1,1,1)),
  float *disp32 = nullptr;      // one value per CG DoF (lexicographic)
  double *diag64 = nullptr;
  double *dinv64 = nullptr;
  float *diag32 = nullptr;
  float *dinv32 = nullptr;
  void *halo = nullptr;         // CG apply: upper-face values of every brick (FP64 size)
  // multigrid vectors in the cycle's precision (FP64 on the coarsest level)
  void *b = nullptr, *x = nullptr, *ax = nullptr, *d = nullptr;
  void *x2 = nullptr;           // SIPG with the GLL Jacobi smoother: the fused step's second x
  void *tbuf = nullptr;         // CG multigrid, level >= 1: the restriction's per-cell
                                // contributions, (k+1)^3 values per cell of the next coarser
                                // level, FP64 size
  bool mg_f32 = false;          // vectors of this level are float
  double lambda_max = 0.0;
  double coarse_lmin = 0.0, coarse_lmax = 0.0;
  int coarse_steps = 0;
};

struct Context {
  mfl_params p{};
  int k = 0, n = 0;
  std::vector<Level> levels;
  Tab<kMaxN, double> tab64{};
  Tab<kMaxN, float> tab32{};
  TransferTab transfer{};
  // FP64 work vectors of the finest level (PCG and eigenvalue estimates)
  double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;
  double *partials = nullptr;   // reduction partials (at least kReduceBlocks doubles)
  double *scalars = nullptr;    // device scalars (see enum Scalar)
  double *eig_hist = nullptr;   // multigrid: p.A p, alpha, beta of each eigenvalue-estimate iteration
  int *flags = nullptr;         // device error flags of the setup checks (see enum Flag)
  double *host_scalars = nullptr;   // pinned host mirror
  double *host_coarse = nullptr;    // multigrid: pinned host staging of three coarsest-level vectors
  // the V-cycle on the work vectors r -> z, captured once as a HIP graph on an internal
  // stream and replayed on the caller's stream (use_graphs); rebuilt when the smoother or
  // coarse-solver parameters change
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t vcycle_graph = nullptr;
  // optional timing of the operator cell kernels of mfl_apply (HIP event pairs)
  bool profiling = false;
  int prof_used = 0;
  std::vector<hipEvent_t> prof_start, prof_stop;
};

// Whether the curved metric is formed on the fly (metric_mode AUTO resolves to it with a
// cellwise kappa).
inline bool metric_on_the_fly(const mfl_params &p) {
  return p.disc == MFL_DISC_CG && p.geometry == MFL_GEOM_CURVED && p.kappa_field == MFL_KAPPA_CELLWISE &&
         p.metric_mode != MFL_METRIC_STORED;
}

// Face mask of the Dirichlet conditions: bit 0 the lower faces (x_e = domain_lo), bit 1
// the upper faces (x_e = domain_lo + domain_len).
inline int dirichlet_mask(const mfl_params &p) {
  return p.bc == MFL_BC_DIRICHLET ? 3 : (p.bc == MFL_BC_MIXED ? 2 : 0);
}

enum Scalar { kRZ = 0, kPQ, kAlpha, kBeta, kRR, kBB, kRZnew, kNumScalars = 16 };

// Bits of flags[0], raised by setup kernels: a kappa value that is not finite and positive,
// a quadrature point of a curved cell with det J <= 0 (or not finite).
enum Flag { kFlagKappa = 1, kFlagDetJ = 2, kFlagChanged = 4, kNumFlags = 64 };

// ---- host-side tables -------------------------------------------------------
void gauss_legendre(int n, double *x, double *w);
void gauss_lobatto(int n, double *x, double *w);
void lagrange_eval(int n, const double *nodes, double x, double *val, double *der);
void build_tables(int k, Tab<kMaxN, double> &t64, Tab<kMaxN, float> &t32, TransferTab &tt);

// Optional timing of one kernel launch: the dispatch packet itself records start and stop
// (hipExtLaunchKernelGGL), so timing adds no packets between kernels.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// ---- kernel launchers (return hipError_t of the launch) -----------------------
hipError_t launch_boundary_init(const Context &c, const Level &L, int dtype, const void *src,
                                void *dst, hipStream_t s);
// CG operator: brick kernel (owned DoFs + halo records), then the halo addition
// (dmask < 0: the Dirichlet faces of the parameters; 0: the operator without boundary
// conditions, used for the lifting of Dirichlet data)
hipError_t launch_cg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                           hipStream_t s, int dmask = -1, const LaunchEvents *ev = nullptr);
hipError_t launch_cg_halo_add(const Context &c, const Level &L, int dtype, void *dst, hipStream_t s,
                              int dmask = -1);
int64_t cg_halo_elements(int k, int Nc, bool curved);
hipError_t launch_cg_kappa_grad(const Context &c, const Level &L, const double *u, const double *lam,
                                double *grad, hipStream_t s);
// per-point metric of curved cells (times the position-dependent kappa field when the
// parameters ask for it); raises kFlagDetJ in c.flags for a non-positive det J
hipError_t launch_metric_setup(const Context &c, const Level &L, hipStream_t s);
// raises `bit` in *flag for every value of v[0..n) that is not finite and positive
// flag |= bit if some v[i] is not finite and positive; with prev, flag |= change_bit if some
// v[i] differs bitwise from prev[i]
hipError_t launch_check_positive(const double *v, int64_t n, int *flag, int bit, hipStream_t s,
                                 const double *prev = nullptr, int change_bit = 0);
hipError_t launch_cg_diagonal(const Context &c, const Level &L, hipStream_t s);
hipError_t launch_rhs_sine(const Context &c, const Level &L, double *b, hipStream_t s);
// right-hand side of the three-Gaussian example: forcing and Neumann loads (b = 0 first)
hipError_t launch_rhs_gaussians(const Context &c, const Level &L, double *b, hipStream_t s);
// x0 = the solution of the three-Gaussian example on the Dirichlet DoFs, 0 elsewhere
hipError_t launch_gaussian_dirichlet(const Context &c, const Level &L, double *x0, hipStream_t s);
// b = x0 on Dirichlet DoFs, b - a0 elsewhere
hipError_t launch_lift(const Context &c, const Level &L, double *b, const double *x0, const double *a0,
                       hipStream_t s);
hipError_t launch_sipg_apply(const Context &c, const Level &L, int dtype, const void *src, void *dst,
                             hipStream_t s, const LaunchEvents *ev = nullptr);
// FP64 SIPG apply dst = A src that also writes the per-work-group partial sums of src . dst
// (in a fixed order) to partials[0 .. sipg_apply_blocks(k, Nc)); returns that count in *n.
hipError_t launch_sipg_apply_dot(const Context &c, const Level &L, const double *src, double *dst,
                                 double *partials, int *n, hipStream_t s);
int sipg_apply_blocks(int k, int Nc);
// SIPG: matrix diagonal (FP64, then inverse and FP32 copies), embedding transfers between
// level `coarse` and the next finer one, and the right-hand side of the three-Gaussian example
hipError_t launch_sipg_diagonal(const Context &c, const Level &L, hipStream_t s);
hipError_t launch_dg_prolongate_add(const Context &c, const Level &coarse, const void *xc, int c_dtype,
                                    void *xf, int f_dtype, hipStream_t s);
hipError_t launch_dg_restrict(const Context &c, const Level &coarse, const void *bf, const void *axf,
                              int f_dtype, void *bc, int c_dtype, hipStream_t s);
hipError_t launch_sipg_rhs_gaussians(const Context &c, const Level &L, double *b, hipStream_t s);
// SIPG smoother with the point Jacobi of the GLL basis: L.dinv64 / L.dinv32 receive D'^{-1}
// (cell-major, GLL index order) with D' = diag(T^T A T), T = S (x) S (x) S per cell
hipError_t launch_sipg_gll_jacobi_diag(const Context &c, const Level &L, hipStream_t s);
// the Chebyshev updates (cheb_first / cheb_step semantics) and the plain Jacobi step
// z = C r with C = T D'^{-1} T^T instead of the point Jacobi of the Gauss basis
hipError_t launch_dg_gll_cheb_first(const Context &c, const Level &L, const void *b_in, int in_dtype,
                                    void *b_store, void *d, void *x, int dtype, double inv_theta,
                                    hipStream_t s);
// One Chebyshev update of the SIPG smoother with the operator application fused in:
// d = c1 d + c2 C (b - A x), x_out = x + d (x_out must not alias x).
hipError_t launch_sipg_cheb(const Context &c, const Level &L, const void *x, const void *b, void *d, void *x_out,
                            double *x64_out, int dtype, double c1, double c2, hipStream_t s);
hipError_t launch_dg_gll_cheb_step(const Context &c, const Level &L, const void *b, const void *ax, void *d,
                                   void *x, double *x64_out, int dtype, double c1, double c2, hipStream_t s);
hipError_t launch_dg_gll_jacobi(const Context &c, const Level &L, const double *r, double *z, hipStream_t s);
hipError_t launch_diag_invert(const Level &L, hipStream_t s);

// multigrid and vector kernels
hipError_t launch_fill(void *dst, int dtype, int64_t n, double value, hipStream_t s);
hipError_t launch_cast(const void *src, int src_dtype, void *dst, int dst_dtype, int64_t n,
                       hipStream_t s);
hipError_t launch_coarsen_kappa(const Level &coarse, const Level &fine, hipStream_t s);
hipError_t launch_diag_finalize(const Context &c, const Level &L, hipStream_t s);
hipError_t launch_cheb_first(const void *b_in, int in_dtype, void *b_store, const void *dinv,
                             void *d, void *x, int dtype, int64_t n, double inv_theta, hipStream_t s);
hipError_t launch_cheb_step(const void *b, const void *ax, const void *dinv, void *d, void *x,
                            double *x64_out, int dtype, int64_t n, double c1, double c2,
                            hipStream_t s);
// The Chebyshev update fused with the halo addition of launch_cg_apply (continuous Q_k; ax
// as left by launch_cg_apply without launch_cg_halo_add).
// Coarse-grid Chebyshev solve from x = 0 in one launch (continuous Q_k, Cartesian, FP64
// level with at most 3 cells per direction that fits one work-group's LDS).
bool cg_coarse_cheb_supported(const Context &c, const Level &L);
hipError_t launch_cg_coarse_cheb(const Context &c, const Level &L, const double *b, double *x, double *x64_out,
                                 int steps, double theta, double delta, hipStream_t s);
hipError_t launch_cg_cheb_halo(const Context &c, const Level &L, const void *b, const void *ax,
                               const void *dinv, void *d, void *x, double *x64_out, int dtype, double c1,
                               double c2, hipStream_t s);
hipError_t launch_prolongate_add(const Context &c, const Level &coarse, const Level &fine,
                                 const void *xc, int c_dtype, void *xf, int f_dtype, hipStream_t s);
hipError_t launch_restrict_residual(const Context &c, const Level &coarse, const Level &fine,
                                    const void *bf, const void *axf, int f_dtype, void *bc,
                                    int c_dtype, hipStream_t s);
hipError_t launch_dot_partial(const double *a, const double *b, int64_t n, double *partials,
                              hipStream_t s);
hipError_t launch_finalize(const double *partials, double *scalars, int which, int op,
                           hipStream_t s, int n_partials = kReduceBlocks);
hipError_t launch_pcg_update_xr(double *x, double *r, const double *p, const double *q,
                                const double *scalars, int64_t n, double *partials, hipStream_t s);
hipError_t launch_pcg_update_p(double *p, const double *z, const double *scalars, int64_t n,
                               hipStream_t s);
hipError_t launch_random_start(double *v, const Level &L, uint64_t key, int dmask, hipStream_t s);
hipError_t launch_jacobi(const double *dinv, const double *r, double *z, int64_t n, hipStream_t s);
hipError_t launch_zero_boundary(double *v, const Level &L, int dmask, hipStream_t s);

// finalize ops
enum FinalizeOp { kFinSum = 0, kFinAlpha = 1, kFinBeta = 2 };

}  // namespace mfl
