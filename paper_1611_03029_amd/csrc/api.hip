// C ABI: parameter checks, workspace layout, setup, operator application, the multigrid
// V-cycle and the preconditioned conjugate gradient solver (Sec. 4.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "mfl_internal.h"

using namespace mfl;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(MFL_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Faces whose DoFs are identity rows of the operator: the Dirichlet faces for CG; none for
// SIPG, which imposes Dirichlet data weakly.
int row_mask(const mfl_params &p) { return p.disc == MFL_DISC_CG ? dirichlet_mask(p) : 0; }

// Unknowns of the coarsest multigrid level: CG without the DoFs of Dirichlet faces, SIPG all.
int64_t coarse_unknowns(const mfl_params &p) {
  const int64_t Nc = p.min_level_cells, n = p.degree + 1;
  if (p.disc != MFL_DISC_CG) return Nc * Nc * Nc * n * n * n;
  const int dm = row_mask(p);
  const int64_t m1 = p.degree * Nc + 1 - (dm & 1) - ((dm >> 1) & 1);
  return m1 * m1 * m1;
}

// The coarse solver's eigenvalue range comes from a Lanczos process whose basis is held on
// the host (see coarse_interval); this bounds its size.
constexpr int kMaxCoarseUnknowns = 20000;

int check_params(const mfl_params *p) {
  if (!p) return fail(MFL_EINVAL, "params is NULL");
  if (p->degree < 1 || p->degree > kMaxDegree)
    return fail(MFL_EINVAL, "degree %d outside 1..%d", p->degree, kMaxDegree);
  if (p->cells_per_dim < 1) return fail(MFL_EINVAL, "cells_per_dim must be >= 1");
  if (p->disc != MFL_DISC_CG && p->disc != MFL_DISC_SIPG) return fail(MFL_EINVAL, "unknown disc %d", p->disc);
  if (p->geometry != MFL_GEOM_CARTESIAN && p->geometry != MFL_GEOM_CURVED)
    return fail(MFL_EINVAL, "unknown geometry %d", p->geometry);
  if (p->bc != MFL_BC_DIRICHLET && p->bc != MFL_BC_NEUMANN && p->bc != MFL_BC_MIXED)
    return fail(MFL_EINVAL, "unknown bc %d", p->bc);
  if (!(std::isfinite(p->domain_lo) && p->domain_len > 0.0 && std::isfinite(p->domain_len)))
    return fail(MFL_EINVAL, "need a finite domain_lo and 0 < domain_len < inf");
  if (p->dg_jacobi_basis != MFL_DG_JACOBI_GAUSS && p->dg_jacobi_basis != MFL_DG_JACOBI_GLL)
    return fail(MFL_EINVAL, "unknown dg_jacobi_basis %d", p->dg_jacobi_basis);
  if (p->mg_precision != MFL_F64 && p->mg_precision != MFL_F32)
    return fail(MFL_EINVAL, "unknown mg_precision %d", p->mg_precision);
  if (p->disc == MFL_DISC_SIPG) {
    if (p->geometry != MFL_GEOM_CARTESIAN)
      return fail(MFL_EINVAL, "SIPG is implemented on Cartesian meshes only");
    if (!(p->penalty_factor > 0.0)) return fail(MFL_EINVAL, "penalty_factor must be > 0");
  }
  if (p->geometry == MFL_GEOM_CURVED) {
    // det J of the analytic map is 1 + a pi (c s s + s c s + s s c) >= 1 - 2 pi |a| / sqrt(3)
    // (the bracket's extremes are +-2/sqrt(3), on the diagonal), i.e. > 0.45 for |a| <= 0.15;
    // the interpolated map's det J is also checked at every quadrature point at setup.
    if (!(std::fabs(p->curve_amp) <= 0.15)) return fail(MFL_EINVAL, "|curve_amp| must be <= 0.15");
    if (p->domain_lo != 0.0 || p->domain_len != 1.0)
      return fail(MFL_EINVAL, "the curved map is defined on the unit cube (domain_lo 0, domain_len 1)");
  }
  if (p->kappa_field != MFL_KAPPA_CELLWISE && p->kappa_field != MFL_KAPPA_COSINE)
    return fail(MFL_EINVAL, "unknown kappa_field %d", p->kappa_field);
  if (p->metric_mode != MFL_METRIC_AUTO && p->metric_mode != MFL_METRIC_STORED &&
      p->metric_mode != MFL_METRIC_ON_THE_FLY)
    return fail(MFL_EINVAL, "unknown metric_mode %d", p->metric_mode);
  if (p->metric_mode == MFL_METRIC_ON_THE_FLY && p->kappa_field != MFL_KAPPA_CELLWISE)
    return fail(MFL_EINVAL, "the on-the-fly metric needs a cellwise kappa (kappa_field = MFL_KAPPA_CELLWISE)");
  if (p->kappa_field == MFL_KAPPA_COSINE) {
    if (p->disc != MFL_DISC_CG || p->geometry != MFL_GEOM_CURVED)
      return fail(MFL_EINVAL, "the position-dependent kappa field needs the continuous discretization on "
                              "curved geometry (it is folded into the per-point metric)");
    if (!(p->kappa_field_amp >= 0.0 && std::isfinite(p->kappa_field_amp)))
      return fail(MFL_EINVAL, "kappa_field_amp must be finite and >= 0");
  }
  if (p->build_mg) {
    if (p->bc == MFL_BC_NEUMANN) return fail(MFL_EINVAL, "multigrid requires Dirichlet conditions on some faces");
    if (p->min_level_cells < 1) return fail(MFL_EINVAL, "min_level_cells must be >= 1");
    int Nc = p->cells_per_dim;
    while (Nc > p->min_level_cells) {
      if (Nc % 2) return fail(MFL_EINVAL, "cells_per_dim %d does not halve down to min_level_cells %d",
                              p->cells_per_dim, p->min_level_cells);
      Nc /= 2;
    }
    if (Nc != p->min_level_cells)
      return fail(MFL_EINVAL, "cells_per_dim %d does not halve down to min_level_cells %d",
                  p->cells_per_dim, p->min_level_cells);
    const int64_t unknowns = coarse_unknowns(*p);
    if (unknowns > kMaxCoarseUnknowns)
      return fail(MFL_EINVAL, "the coarsest level has %lld unknowns; the coarse solver takes at most %d "
                              "(choose a smaller min_level_cells)", (long long)unknowns, kMaxCoarseUnknowns);
    if (p->cheb_degree < 1 || p->cheb_degree > 64) return fail(MFL_EINVAL, "cheb_degree outside 1..64");
    if (!(p->cheb_lo > 0.0 && p->cheb_hi > p->cheb_lo)) return fail(MFL_EINVAL, "need 0 < cheb_lo < cheb_hi");
    if (p->eig_iters < 1 || p->eig_iters > 1000) return fail(MFL_EINVAL, "eig_iters outside 1..1000");
    if (!(p->coarse_tol > 0.0 && p->coarse_tol < 1.0)) return fail(MFL_EINVAL, "coarse_tol outside (0,1)");
  }
  return MFL_OK;
}

std::vector<int> level_cells(const mfl_params &p) {
  std::vector<int> v;
  if (!p.build_mg) return {p.cells_per_dim};
  for (int Nc = p.min_level_cells; Nc <= p.cells_per_dim; Nc *= 2) v.push_back(Nc);
  return v;
}

struct Bump {
  char *base = nullptr;
  int64_t off = 0;
  template <typename T>
  T *take(int64_t count) {
    off = (off + 255) / 256 * 256;
    T *r = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * int64_t(sizeof(T));
    return r;
  }
};

// Lays out all device arrays of the context in the workspace (base == nullptr: sizes only).
int64_t layout(Context &c, char *base) {
  Bump b{base, 0};
  const mfl_params &p = c.p;
  const int n3 = c.n * c.n * c.n;
  const bool cg = p.disc == MFL_DISC_CG;
  for (size_t l = 0; l < c.levels.size(); ++l) {
    Level &L = c.levels[l];
    L.kappa64 = b.take<double>(L.ncells);
    L.kappa32 = b.take<float>(L.ncells);
    if (cg && p.geometry == MFL_GEOM_CURVED) {
      if (metric_on_the_fly(p)) {
        L.disp64 = b.take<double>(L.ndofs);
        L.disp32 = b.take<float>(L.ndofs);
      } else {
        L.metric64 = b.take<double>(L.ncells * 6 * n3);
        L.metric32 = b.take<float>(L.ncells * 6 * n3);
      }
    }
    if (cg) L.halo = b.take<double>(cg_halo_elements(c.k, L.Nc, p.geometry == MFL_GEOM_CURVED));
    {
      L.diag64 = b.take<double>(L.ndofs);
      L.dinv64 = b.take<double>(L.ndofs);
      L.diag32 = b.take<float>(L.ndofs);
      L.dinv32 = b.take<float>(L.ndofs);
    }
    if (p.build_mg) {
      L.mg_f32 = (p.mg_precision == MFL_F32) && l > 0;
      const int64_t es = L.mg_f32 ? 4 : 8;
      L.b = b.take<char>(L.ndofs * es);
      L.x = b.take<char>(L.ndofs * es);
      L.ax = b.take<char>(L.ndofs * es);
      L.d = b.take<char>(L.ndofs * es);
      if (p.disc == MFL_DISC_SIPG && p.dg_jacobi_basis == MFL_DG_JACOBI_GLL) L.x2 = b.take<char>(L.ndofs * es);
      if (cg && l > 0) L.tbuf = b.take<double>(c.levels[l - 1].ncells * n3);
    }
  }
  {
    const int64_t N = c.levels.back().ndofs;
    c.r = b.take<double>(N);
    c.z = b.take<double>(N);
    if (p.build_mg) {
      c.pv = b.take<double>(N);
      c.q = b.take<double>(N);
    }
  }
  // reduction partials: the vector kernels' fixed count, or the SIPG operator's work-groups
  // when the outer CG takes p . A p from the operator kernel
  const int64_t np = p.disc == MFL_DISC_SIPG && p.build_mg
                         ? std::max<int64_t>(kReduceBlocks, sipg_apply_blocks(p.degree, p.cells_per_dim))
                         : kReduceBlocks;
  c.partials = b.take<double>(np);
  c.scalars = b.take<double>(kNumScalars);
  if (p.build_mg) c.eig_hist = b.take<double>(3 * std::max(p.eig_iters, 1));
  c.flags = b.take<int>(kNumFlags);
  return b.off;
}

void init_context(Context &c, const mfl_params &p) {
  c.p = p;
  c.k = p.degree;
  c.n = p.degree + 1;
  c.levels.clear();
  for (int Nc : level_cells(p)) {
    Level L;
    L.Nc = Nc;
    L.N1 = c.k * Nc + 1;
    L.ncells = int64_t(Nc) * Nc * Nc;
    L.ndofs = p.disc == MFL_DISC_CG ? int64_t(L.N1) * L.N1 * L.N1 : L.ncells * c.n * c.n * c.n;
    L.h = p.domain_len / Nc;
    c.levels.push_back(L);
  }
}

int level_index(const Context &c, int level) {
  const int nl = int(c.levels.size());
  if (level == -1) return nl - 1;
  if (level < 0 || level >= nl) return -1;
  return level;
}

// Extreme eigenvalues of the symmetric tridiagonal matrix (a on the diagonal, b off it)
// by bisection on Sturm sequence counts.
void tridiag_extremes(const std::vector<double> &a, const std::vector<double> &b, double &lmin,
                      double &lmax) {
  const int m = int(a.size());
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::fmin(lo, a[i] - r);
    hi = std::fmax(hi, a[i] + r);
  }
  auto count_below = [&](double x) {   // number of eigenvalues < x
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  auto bisect = [&](int target) {   // smallest x with count_below(x) > target
    double l = lo, h = hi;
    for (int it = 0; it < 200 && h - l > 1e-16 * std::fmax(1.0, std::fabs(h)); ++it) {
      const double mid = 0.5 * (l + h);
      if (count_below(mid) > target) h = mid; else l = mid;
    }
    return 0.5 * (l + h);
  };
  lmin = bisect(0);
  lmax = bisect(m - 1);
}

constexpr int kMaxProfiled = 8192;

int apply_level(Context &c, int l, int dtype, const void *src, void *dst, hipStream_t s,
                bool timed = false, bool halo = true) {
  const Level &L = c.levels[l];
  const bool rec = timed && c.profiling && c.prof_used < kMaxProfiled;
  if (rec && c.prof_used == int(c.prof_start.size())) {
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    c.prof_start.push_back(a);
    c.prof_stop.push_back(b);
  }
  LaunchEvents ev;
  if (rec) {
    ev.start = c.prof_start[c.prof_used];
    ev.stop = c.prof_stop[c.prof_used++];
  }
  if (c.p.disc == MFL_DISC_SIPG) {
    HIP_TRY(launch_sipg_apply(c, L, dtype, src, dst, s, rec ? &ev : nullptr));
  } else {
    HIP_TRY(launch_cg_apply(c, L, dtype, src, dst, s, -1, rec ? &ev : nullptr));
  }
  if (c.p.disc == MFL_DISC_CG && halo) HIP_TRY(launch_cg_halo_add(c, L, dtype, dst, s));
  return MFL_OK;
}

int read_scalars(Context &c, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(c.host_scalars, c.scalars, kNumScalars * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MFL_OK;
}

// SIPG multigrid smoothed with the point Jacobi of the GLL-Lagrange basis (see
// launch_sipg_gll_jacobi_diag); otherwise point Jacobi of the vectors' own basis.
bool gll_jacobi(const Context &c) {
  return c.p.disc == MFL_DISC_SIPG && c.p.dg_jacobi_basis == MFL_DG_JACOBI_GLL;
}

hipError_t jacobi_step(const Context &c, const Level &L, const double *r, double *z, hipStream_t s) {
  if (gll_jacobi(c)) return launch_dg_gll_jacobi(c, L, r, z, s);
  return launch_jacobi(L.dinv64, r, z, L.ndofs, s);
}

int row_mask(const Context &c) { return row_mask(c.p); }

// Jacobi-preconditioned CG on level l from the SplitMix64 start vector (key = cells per
// direction, Dirichlet entries zero); records the Lanczos tridiagonal from alpha, beta.
// p.A p, alpha and beta of every iteration are copied to a device history and read once at
// the end; the recurrence stops at the first iteration whose p.A p is not finite and
// positive (a zero start residual gives p.A p = 0 at once).
int lanczos(Context &c, int l, int max_iters, std::vector<double> &diag, std::vector<double> &off,
            hipStream_t s) {
  Level &L = c.levels[l];
  const int64_t N = L.ndofs;
  double *r = c.r, *z = c.z, *p = c.pv, *q = c.q;
  int rc;
  max_iters = std::min(max_iters, std::max(c.p.eig_iters, 1));   // the history's length
  HIP_TRY(launch_random_start(r, L, uint64_t(L.Nc), row_mask(c), s));
  HIP_TRY(jacobi_step(c, L, r, z, s));
  HIP_TRY(hipMemcpyAsync(p, z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_dot_partial(r, z, N, c.partials, s));
  HIP_TRY(launch_finalize(c.partials, c.scalars, kRZ, kFinSum, s));
  static_assert(kAlpha == kPQ + 1 && kBeta == kPQ + 2, "p.A p, alpha, beta are consecutive scalars");
  for (int it = 0; it < max_iters; ++it) {
    if ((rc = apply_level(c, l, MFL_F64, p, q, s))) return rc;
    HIP_TRY(launch_dot_partial(p, q, N, c.partials, s));
    HIP_TRY(launch_finalize(c.partials, c.scalars, 0, kFinAlpha, s));
    // r -= alpha q (x is not needed: the z buffer takes the x update and is overwritten)
    HIP_TRY(launch_pcg_update_xr(z, r, p, q, c.scalars, N, c.partials, s));
    HIP_TRY(jacobi_step(c, L, r, z, s));
    HIP_TRY(launch_dot_partial(r, z, N, c.partials, s));
    HIP_TRY(launch_finalize(c.partials, c.scalars, 0, kFinBeta, s));
    HIP_TRY(launch_pcg_update_p(p, z, c.scalars, N, s));
    HIP_TRY(hipMemcpyAsync(c.eig_hist + 3 * it, c.scalars + kPQ, 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  std::vector<double> hist(3 * std::max(max_iters, 0));
  if (max_iters > 0)
    HIP_TRY(hipMemcpyAsync(hist.data(), c.eig_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<double> alphas, betas;
  for (int it = 0; it < max_iters; ++it) {
    const double pq = hist[3 * it];
    if (!(pq > 0.0) || !std::isfinite(pq)) break;
    alphas.push_back(hist[3 * it + 1]);
    betas.push_back(hist[3 * it + 2]);
  }
  const int m = int(alphas.size());
  if (m == 0) return fail(MFL_EBREAKDOWN, "eigenvalue estimate on level %d: no CG step possible", l);
  diag.assign(m, 0.0);
  off.assign(m > 1 ? m - 1 : 0, 0.0);
  for (int j = 0; j < m; ++j) {
    diag[j] = 1.0 / alphas[j] + (j > 0 ? betas[j - 1] / alphas[j - 1] : 0.0);
    if (j + 1 < m) off[j] = std::sqrt(betas[j]) / alphas[j];
  }
  return MFL_OK;
}

// Extreme eigenvalues of C A on the unknowns of level l, C the level's Jacobi step (the
// interval of the coarse-grid Chebyshev solver, Sec. 4.1).  Lanczos in the inner product of
// C (the recurrence behind preconditioned CG): q_1 = r / |r|_C from the SplitMix64 start
// vector, then w = A p_j - alpha_j q_j - beta_{j-1} q_{j-1} with p_j = C q_j, orthogonalized
// twice against the whole basis, q_{j+1} = w / beta_j with beta_j = (w^T C w)^{1/2}.  The
// basis vectors live on the host; the products with A run on the device, the point Jacobi
// step C on the host (SIPG's GLL-basis Jacobi on the device).  Full
// reorthogonalization keeps the tridiagonal's extreme eigenvalues from stalling below the
// operator's when the start vector is nearly deflated (a clustered spectrum), which plain
// CG-Lanczos run until its residual vanishes does not.  Stops when the Krylov space is
// invariant (beta_j <= 1e-12 lambda_max), when it spans all unknowns, or when both extreme
// Ritz values have moved by at most 1e-15 lambda_max over the last 8 steps.
int coarse_interval(Context &c, int l, hipStream_t s, double &lmin, double &lmax) {
  Level &L = c.levels[l];
  const int64_t N = L.ndofs;
  const int64_t unknowns = l == 0 ? coarse_unknowns(c.p) : N;
  const int max_steps = int(std::min<int64_t>(unknowns, 4000));
  // w, z and the staged p_j in pinned host memory (the coarsest level's length): each step
  // moves them with direct copies instead of through pageable staging
  if (!c.host_coarse || N > c.levels.front().ndofs) return fail(MFL_EINVAL, "coarse staging missing");
  double *w = c.host_coarse, *z = c.host_coarse + N, *pstage = c.host_coarse + 2 * N;
  std::vector<double> Q, P, alpha, beta;
  auto dot = [N](const double *a, const double *b) {
    double acc = 0.0;
    for (int64_t i = 0; i < N; ++i) acc += a[i] * b[i];
    return acc;
  };
  // z = C w: the point Jacobi step on the host from a copy of D^{-1} (the product of
  // jacobi_kernel), the GLL-basis Jacobi of SIPG on the device
  std::vector<double> dinv;
  if (!gll_jacobi(c)) {
    dinv.resize(N);
    HIP_TRY(hipMemcpyAsync(dinv.data(), L.dinv64, N * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  auto precondition = [&]() -> int {
    if (!dinv.empty()) {
      for (int64_t i = 0; i < N; ++i) z[i] = dinv[i] * w[i];
      return MFL_OK;
    }
    HIP_TRY(hipMemcpyAsync(c.r, w, N * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(jacobi_step(c, L, c.r, c.z, s));
    HIP_TRY(hipMemcpyAsync(z, c.z, N * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MFL_OK;
  };
  HIP_TRY(launch_random_start(c.r, L, uint64_t(L.Nc), row_mask(c), s));
  HIP_TRY(hipMemcpyAsync(w, c.r, N * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int rc = precondition();
  if (rc) return rc;
  double b0 = dot(w, z);
  if (!(b0 > 0.0) || !std::isfinite(b0))
    return fail(MFL_EBREAKDOWN, "coarse eigenvalue range on level %d: start vector has no C-norm", l);
  b0 = std::sqrt(b0);
  auto push = [&](double scale) {
    Q.resize(Q.size() + N);
    P.resize(P.size() + N);
    double *q = Q.data() + Q.size() - N, *p = P.data() + P.size() - N;
    for (int64_t i = 0; i < N; ++i) {
      q[i] = w[i] / scale;
      p[i] = z[i] / scale;
    }
  };
  push(b0);
  double last_min = 0.0, last_max = 0.0;
  lmin = lmax = 0.0;
  for (int j = 0; j < max_steps; ++j) {
    const double *qj = Q.data() + int64_t(j) * N, *pj = P.data() + int64_t(j) * N;
    std::copy(pj, pj + N, pstage);
    HIP_TRY(hipMemcpyAsync(c.pv, pstage, N * sizeof(double), hipMemcpyHostToDevice, s));
    if ((rc = apply_level(c, l, MFL_F64, c.pv, c.q, s))) return rc;
    HIP_TRY(hipMemcpyAsync(w, c.q, N * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double a = dot(pj, w);
    for (int64_t i = 0; i < N; ++i) w[i] -= a * qj[i];
    if (j > 0) {
      const double *qp = Q.data() + int64_t(j - 1) * N;
      for (int64_t i = 0; i < N; ++i) w[i] -= beta[j - 1] * qp[i];
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i <= j; ++i) {
        const double *qi = Q.data() + int64_t(i) * N, *pi = P.data() + int64_t(i) * N;
        const double h = dot(pi, w);
        for (int64_t e = 0; e < N; ++e) w[e] -= h * qi[e];
      }
    alpha.push_back(a);
    tridiag_extremes(alpha, beta, lmin, lmax);
    if (!std::isfinite(lmin) || !std::isfinite(lmax) || !(lmax > 0.0))
      return fail(MFL_EBREAKDOWN, "coarse eigenvalue range on level %d: Lanczos step %d is not finite", l, j);
    if (j + 1 == max_steps) break;
    if ((j + 1) % 8 == 0) {
      if (j + 1 > 8 && std::fabs(lmin - last_min) <= 1e-15 * lmax && std::fabs(lmax - last_max) <= 1e-15 * lmax)
        break;
      last_min = lmin;
      last_max = lmax;
    }
    if ((rc = precondition())) return rc;
    const double bb = dot(w, z);
    if (!(bb > 0.0) || std::sqrt(bb) <= 1e-12 * lmax) break;   // invariant Krylov space
    beta.push_back(std::sqrt(bb));
    push(beta.back());
  }
  if (!(lmin > 0.0))
    return fail(MFL_EBREAKDOWN, "coarse eigenvalue range on level %d: smallest eigenvalue %g is not positive",
                l, lmin);
  return MFL_OK;
}

int drop_vcycle_graph(Context &c) {
  if (c.vcycle_graph) {
    HIP_TRY(hipGraphExecDestroy(c.vcycle_graph));
    c.vcycle_graph = nullptr;
  }
  return MFL_OK;
}

// Everything that depends on kappa: coarse kappa, diagonals, eigenvalue estimates.
int rebuild_kappa_dependent(Context &c, hipStream_t s) {
  // the captured V-cycle holds the old smoother and coarse-solver coefficients
  HIP_TRY(hipStreamSynchronize(s));
  if (int rc = drop_vcycle_graph(c)) return rc;
  const int nl = int(c.levels.size());
  for (int l = nl - 2; l >= 0; --l) HIP_TRY(launch_coarsen_kappa(c.levels[l], c.levels[l + 1], s));
  for (int l = 0; l < nl; ++l) {
    if (c.p.disc == MFL_DISC_CG)
      HIP_TRY(launch_cg_diagonal(c, c.levels[l], s));
    else
    {
      HIP_TRY(launch_sipg_diagonal(c, c.levels[l], s));
      if (gll_jacobi(c)) HIP_TRY(launch_sipg_gll_jacobi_diag(c, c.levels[l], s));
    }
  }
  if (!c.p.build_mg) {
    HIP_TRY(hipStreamSynchronize(s));
    return MFL_OK;
  }
  std::vector<double> a, b;
  for (int l = 0; l < nl; ++l) {
    Level &L = c.levels[l];
    double lmin, lmax;
    int rc;
    if (l == 0) {
      if ((rc = coarse_interval(c, l, s, lmin, lmax))) return rc;
      L.coarse_lmin = lmin;
      L.coarse_lmax = lmax;
      const double cond = lmax / lmin;
      const double rate = (std::sqrt(cond) - 1.0) / (std::sqrt(cond) + 1.0);
      L.coarse_steps = rate <= 0.0 ? 1
                                   : int(std::ceil(std::log(2.0 / c.p.coarse_tol) / std::log(1.0 / rate)));
      if (L.coarse_steps < 1) L.coarse_steps = 1;
    } else {
      if ((rc = lanczos(c, l, c.p.eig_iters, a, b, s))) return rc;
      tridiag_extremes(a, b, lmin, lmax);
      L.lambda_max = lmax;
    }
  }
  return MFL_OK;
}

int dtype_of(const Level &L) { return L.mg_f32 ? MFL_F32 : MFL_F64; }
const void *dinv_of(const Level &L) { return L.mg_f32 ? (const void *)L.dinv32 : (const void *)L.dinv64; }

// d = c1 d + c2 C (b - A x); x += d with the level's Jacobi step C.
hipError_t cheb_step(const Context &c, Level &L, double *x64_out, int dt, double c1, double c2, hipStream_t s) {
  if (gll_jacobi(c)) return launch_dg_gll_cheb_step(c, L, L.b, L.ax, L.d, L.x, x64_out, dt, c1, c2, s);
  return launch_cheb_step(L.b, L.ax, dinv_of(L), L.d, L.x, x64_out, dt, L.ndofs, c1, c2, s);
}

// Continuous Q_k levels with 32-bit DoF indices take the halo addition of A x inside the
// Chebyshev update (one streaming pass instead of two).
bool fused_cheb(const Context &c, const Level &L) {
  return c.p.disc == MFL_DISC_CG && L.ndofs < (int64_t(1) << 31);
}

// x += d with d = c1 d + c2 C (b - A x): the operator application and the update.
int smoother_step(Context &c, int l, double *x64_out, int dt, double c1, double c2, hipStream_t s) {
  Level &L = c.levels[l];
  const bool fuse = fused_cheb(c, L);
  if (const int rc = apply_level(c, l, dt, L.x, L.ax, s, false, !fuse)) return rc;
  if (fuse) {
    HIP_TRY(launch_cg_cheb_halo(c, L, L.b, L.ax, dinv_of(L), L.d, L.x, x64_out, dt, c1, c2, s));
  } else {
    HIP_TRY(cheb_step(c, L, x64_out, dt, c1, c2, s));
  }
  return MFL_OK;
}

// Chebyshev iteration on level l with interval [lo, hi] and `updates` updates of x.
// zero_start: x = 0 initially and b is taken from b_in (stored into L.b when b_in != L.b).
// SIPG with the GLL Jacobi smoother fuses the operator into each update, which writes the
// new x into the level's other x buffer; the buffers alternate, and after an odd number of
// such updates L.x and L.x2 exchange roles.
int chebyshev(Context &c, int l, double lo, double hi, int updates, bool zero_start, const void *b_in,
              int b_dtype, double *x64_out, hipStream_t s) {
  Level &L = c.levels[l];
  const int dt = dtype_of(L);
  const int64_t N = L.ndofs;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  int rc;
  int done = 0;
  const bool last_writes = x64_out != nullptr;
  const bool dg_fused = gll_jacobi(c) && L.x2 != nullptr;
  void *cur = L.x, *other = L.x2;
  // the coarse-grid solve of a small Cartesian continuous level: all updates in one launch
  if (l == 0 && zero_start && b_dtype == MFL_F64 && dt == MFL_F64 && !dg_fused && cg_coarse_cheb_supported(c, L)) {
    HIP_TRY(launch_cg_coarse_cheb(c, L, static_cast<const double *>(b_in), static_cast<double *>(L.x), x64_out,
                                  updates, theta, delta, s));
    return MFL_OK;
  }
  auto step = [&](double *x64, double c1, double c2) -> int {
    if (!dg_fused) return smoother_step(c, l, x64, dt, c1, c2, s);
    HIP_TRY(launch_sipg_cheb(c, L, cur, L.b, L.d, other, x64, dt, c1, c2, s));
    std::swap(cur, other);
    return MFL_OK;
  };
  if (zero_start) {
    if (gll_jacobi(c))
      HIP_TRY(launch_dg_gll_cheb_first(c, L, b_in, b_dtype, b_in == L.b ? nullptr : L.b, L.d, L.x, dt,
                                       1.0 / theta, s));
    else
      HIP_TRY(launch_cheb_first(b_in, b_dtype, b_in == L.b ? nullptr : L.b, dinv_of(L), L.d, L.x, dt, N,
                                1.0 / theta, s));
    if (updates == 1 && last_writes) HIP_TRY(launch_cast(L.x, dt, x64_out, MFL_F64, N, s));
  } else {
    if ((rc = step((updates == 1) ? x64_out : nullptr, 0.0, 1.0 / theta))) return rc;
  }
  done = 1;
  double rho = delta > 0.0 ? delta / theta : 0.0;   // 1 / sigma_1
  for (; done < updates; ++done) {
    const double rho_new = 1.0 / (2.0 * theta / delta - rho);
    if ((rc = step(done + 1 == updates ? x64_out : nullptr, rho_new * rho, 2.0 * rho_new / delta))) return rc;
    rho = rho_new;
  }
  // after an odd number of fused updates the result is in the other buffer: the two buffers
  // trade roles (x is scratch of the cycle; a captured cycle replays the same sequence)
  if (cur != L.x) std::swap(L.x, L.x2);
  return MFL_OK;
}

// Transfers between level l-1 and level l of the discretization in use.
hipError_t restrict_to(Context &c, int l, const void *bf, const void *axf, int fd, void *bc, int cd,
                       hipStream_t s) {
  if (c.p.disc == MFL_DISC_CG)
    return launch_restrict_residual(c, c.levels[l - 1], c.levels[l], bf, axf, fd, bc, cd, s);
  return launch_dg_restrict(c, c.levels[l - 1], bf, axf, fd, bc, cd, s);
}

hipError_t prolongate_from(Context &c, int l, const void *xc, int cd, void *xf, int fd, hipStream_t s) {
  if (c.p.disc == MFL_DISC_CG) return launch_prolongate_add(c, c.levels[l - 1], c.levels[l], xc, cd, xf, fd, s);
  return launch_dg_prolongate_add(c, c.levels[l - 1], xc, cd, xf, fd, s);
}

// One V(1,1) cycle on level l; the right-hand side is b_in (level-0 and recursion: L.b).
int cycle(Context &c, int l, const void *b_in, int b_dtype, double *x64_out, hipStream_t s) {
  Level &L = c.levels[l];
  int rc;
  if (l == 0)
    return chebyshev(c, 0, L.coarse_lmin, L.coarse_lmax, L.coarse_steps, true, b_in, b_dtype, x64_out, s);
  const double lo = c.p.cheb_lo * L.lambda_max, hi = c.p.cheb_hi * L.lambda_max;
  const int updates = c.p.cheb_degree + 1;
  const int dt = dtype_of(L);
  Level &C = c.levels[l - 1];
  if ((rc = chebyshev(c, l, lo, hi, updates, true, b_in, b_dtype, nullptr, s))) return rc;
  if ((rc = apply_level(c, l, dt, L.x, L.ax, s))) return rc;
  HIP_TRY(restrict_to(c, l, L.b, L.ax, dt, C.b, dtype_of(C), s));
  if ((rc = cycle(c, l - 1, C.b, dtype_of(C), nullptr, s))) return rc;
  HIP_TRY(prolongate_from(c, l, C.x, dtype_of(C), L.x, dt, s));
  return chebyshev(c, l, lo, hi, updates, false, nullptr, dt, x64_out, s);
}

// Records one V-cycle c.r -> c.z on the internal capture stream (the caller's stream may
// be the legacy default stream, which cannot be captured) and instantiates it.
int capture_vcycle(Context &c) {
  if (!c.capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
  const int top = int(c.levels.size()) - 1;
  HIP_TRY(hipStreamBeginCapture(c.capture_stream, hipStreamCaptureModeThreadLocal));
  const int rc = cycle(c, top, c.r, MFL_F64, c.z, c.capture_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c.capture_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(MFL_EHIP, "capture of the V-cycle: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&c.vcycle_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c.vcycle_graph = nullptr;
    return fail(MFL_EHIP, "instantiation of the V-cycle graph: %s", hipGetErrorString(ei));
  }
  return MFL_OK;
}

// z = V-cycle(r).  With use_graphs the cycle on the work vectors runs as one graph launch
// (other vectors are staged through r and z); otherwise kernel by kernel.
int vcycle(Context &c, const double *r, double *z, hipStream_t s) {
  const int top = int(c.levels.size()) - 1;
  if (!c.p.use_graphs) return cycle(c, top, r, MFL_F64, z, s);
  const int64_t N = c.levels.back().ndofs;
  if (r != c.r) HIP_TRY(hipMemcpyAsync(c.r, r, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (!c.vcycle_graph) {
    int rc = capture_vcycle(c);
    if (rc) return rc;
  }
  HIP_TRY(hipGraphLaunch(c.vcycle_graph, s));
  if (z != c.z) HIP_TRY(hipMemcpyAsync(z, c.z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  return MFL_OK;
}

int pcg(Context &c, const double *b, double *x, double rtol, int maxit, int *iters, double *res,
        hipStream_t s) {
  const Level &F = c.levels.back();
  const int64_t N = F.ndofs;
  int rc;
  if (iters) *iters = 0;
  if (res) *res = 0.0;
  HIP_TRY(launch_fill(x, MFL_F64, N, 0.0, s));
  HIP_TRY(hipMemcpyAsync(c.r, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_dot_partial(b, b, N, c.partials, s));
  HIP_TRY(launch_finalize(c.partials, c.scalars, kBB, kFinSum, s));
  if ((rc = read_scalars(c, s))) return rc;
  const double bb = c.host_scalars[kBB];
  if (!std::isfinite(bb)) return fail(MFL_EBREAKDOWN, "right-hand side is not finite");
  if (bb == 0.0) return MFL_OK;
  const double nb = std::sqrt(bb);
  if ((rc = vcycle(c, c.r, c.z, s))) return rc;
  HIP_TRY(launch_dot_partial(c.r, c.z, N, c.partials, s));
  HIP_TRY(launch_finalize(c.partials, c.scalars, kRZ, kFinSum, s));
  HIP_TRY(hipMemcpyAsync(c.pv, c.z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  double rel = 1.0;
  for (int it = 1; it <= maxit; ++it) {
    if (c.p.disc == MFL_DISC_SIPG) {
      // q = A p with p . q from the operator kernel's work-group partials
      int np = 0;
      HIP_TRY(launch_sipg_apply_dot(c, F, c.pv, c.q, c.partials, &np, s));
      HIP_TRY(launch_finalize(c.partials, c.scalars, 0, kFinAlpha, s, np));
    } else {
      if ((rc = apply_level(c, int(c.levels.size()) - 1, MFL_F64, c.pv, c.q, s))) return rc;
      HIP_TRY(launch_dot_partial(c.pv, c.q, N, c.partials, s));
      HIP_TRY(launch_finalize(c.partials, c.scalars, 0, kFinAlpha, s));
    }
    HIP_TRY(launch_pcg_update_xr(x, c.r, c.pv, c.q, c.scalars, N, c.partials, s));
    HIP_TRY(launch_finalize(c.partials, c.scalars, kRR, kFinSum, s));
    if ((rc = read_scalars(c, s))) return rc;
    const double pq = c.host_scalars[kPQ], rz = c.host_scalars[kRZ], rr = c.host_scalars[kRR];
    if (iters) *iters = it;
    if (!(pq > 0.0) || !std::isfinite(pq) || !(rz > 0.0) || !std::isfinite(rr))
      return fail(MFL_EBREAKDOWN, "CG breakdown at iteration %d (p^T A p = %g, r^T z = %g)", it, pq, rz);
    rel = std::sqrt(rr) / nb;
    if (res) *res = rel;
    if (rel <= rtol) return MFL_OK;
    if ((rc = vcycle(c, c.r, c.z, s))) return rc;
    HIP_TRY(launch_dot_partial(c.r, c.z, N, c.partials, s));
    HIP_TRY(launch_finalize(c.partials, c.scalars, 0, kFinBeta, s));
    HIP_TRY(launch_pcg_update_p(c.pv, c.z, c.scalars, N, s));
  }
  return fail(MFL_ENOCONV, "no convergence in %d iterations (relative residual %g)", maxit, rel);
}

bool need_mg(const Context &c) { return c.p.build_mg != 0; }

// Reads the setup error flags (synchronizes s) and turns a raised flag into MFL_EINVAL.
int setup_flags(Context &c, hipStream_t s) {
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, c.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (f & kFlagKappa) return fail(MFL_EINVAL, "kappa holds a value that is not finite and positive");
  if (f & kFlagDetJ)
    return fail(MFL_EINVAL, "a curved cell has a Jacobian determinant that is not positive at a quadrature point");
  return MFL_OK;
}

}  // namespace

struct mfl_context : public Context {};

// ---- the allocation-free apply ---------------------------------------------------------
// Device memory of mfl_apply_noalloc: one fixed array per GPU, held from the library's
// first use on that GPU until the process ends.  Host code never names it except in
// hipGetSymbolAddress: its device address differs per GPU and is looked up once per device.
static __device__ __align__(256) char scratch[MFL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
int scratch_address(char **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MFL_EUNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MFL_EHIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return MFL_OK;
}

}  // namespace

extern "C" {

int mfl_default_params(mfl_params *p) {
  if (!p) return fail(MFL_EINVAL, "params is NULL");
  *p = mfl_params{};
  p->degree = 2;
  p->cells_per_dim = 8;
  p->min_level_cells = 2;
  p->disc = MFL_DISC_CG;
  p->geometry = MFL_GEOM_CARTESIAN;
  p->curve_amp = 0.1;
  p->bc = MFL_BC_DIRICHLET;
  p->penalty_factor = 1.0;
  p->cheb_degree = 5;
  p->cheb_lo = 0.06;
  p->cheb_hi = 1.2;
  p->eig_iters = 15;
  p->coarse_tol = 1e-3;
  p->mg_precision = MFL_F64;
  p->build_mg = 0;
  p->domain_lo = 0.0;
  p->domain_len = 1.0;
  p->dg_jacobi_basis = MFL_DG_JACOBI_GLL;
  p->use_graphs = 1;
  p->kappa_field = MFL_KAPPA_CELLWISE;
  p->kappa_field_amp = 1e6;
  p->metric_mode = MFL_METRIC_AUTO;
  return MFL_OK;
}

int mfl_query(const mfl_params *p, int64_t *n_dofs, int64_t *n_cells, int64_t *workspace_bytes) {
  int rc = check_params(p);
  if (rc) return rc;
  Context c;
  init_context(c, *p);
  const int64_t bytes = layout(c, nullptr);
  if (n_dofs) *n_dofs = c.levels.back().ndofs;
  if (n_cells) *n_cells = c.levels.back().ncells;
  if (workspace_bytes) *workspace_bytes = bytes;
  return MFL_OK;
}

int mfl_setup(const mfl_params *p, void *workspace, int64_t workspace_bytes, const double *kappa_cells,
              void *stream, mfl_handle *out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!out) return fail(MFL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!workspace) return fail(MFL_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(MFL_EINVAL, "workspace is not 256-byte aligned");
  mfl_context *c = new (std::nothrow) mfl_context();
  if (!c) return fail(MFL_EINVAL, "out of host memory");
  init_context(*c, *p);
  const int64_t need = layout(*c, nullptr);
  if (workspace_bytes < need) {
    delete c;
    return fail(MFL_EINVAL, "workspace too small: %lld < %lld bytes", (long long)workspace_bytes, (long long)need);
  }
  layout(*c, static_cast<char *>(workspace));
  build_tables(c->k, c->tab64, c->tab32, c->transfer);
  hipStream_t s = as_stream(stream);
  auto cleanup = [&](int code) {
    if (c->host_scalars) (void)hipHostFree(c->host_scalars);
    if (c->host_coarse) (void)hipHostFree(c->host_coarse);
    delete c;
    return code;
  };
  if (hipHostMalloc(reinterpret_cast<void **>(&c->host_scalars), kNumScalars * sizeof(double)) != hipSuccess)
    return cleanup(fail(MFL_EHIP, "hipHostMalloc of the scalar mirror failed"));
  if (p->build_mg && hipHostMalloc(reinterpret_cast<void **>(&c->host_coarse),
                                   3 * c->levels.front().ndofs * sizeof(double)) != hipSuccess)
    return cleanup(fail(MFL_EHIP, "hipHostMalloc of the coarse-level staging failed"));
  Level &F = c->levels.back();
  hipError_t e = hipMemsetAsync(c->flags, 0, kNumFlags * sizeof(int), s);
  if (e == hipSuccess) {
    if (kappa_cells)
      e = hipMemcpyAsync(F.kappa64, kappa_cells, F.ncells * sizeof(double), hipMemcpyDeviceToDevice, s);
    else
      e = launch_fill(F.kappa64, MFL_F64, F.ncells, 1.0, s);
  }
  if (e == hipSuccess) e = launch_check_positive(F.kappa64, F.ncells, c->flags, kFlagKappa, s);
  if (e == hipSuccess) e = launch_cast(F.kappa64, MFL_F64, F.kappa32, MFL_F32, F.ncells, s);
  if (e != hipSuccess) return cleanup(fail(MFL_EHIP, "kappa upload: %s", hipGetErrorString(e)));
  if (p->disc == MFL_DISC_CG && p->geometry == MFL_GEOM_CURVED)
    for (Level &L : c->levels)
      if ((e = launch_metric_setup(*c, L, s)) != hipSuccess)
        return cleanup(fail(MFL_EHIP, "metric setup: %s", hipGetErrorString(e)));
  if ((rc = setup_flags(*c, s))) return cleanup(rc);
  if ((rc = rebuild_kappa_dependent(*c, s))) return cleanup(rc);
  if ((e = hipStreamSynchronize(s)) != hipSuccess)
    return cleanup(fail(MFL_EHIP, "setup: %s", hipGetErrorString(e)));
  *out = c;
  return MFL_OK;
}

int mfl_set_kappa(mfl_handle h, const double *kappa_cells, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (!kappa_cells) return fail(MFL_EINVAL, "kappa_cells is NULL");
  hipStream_t s = as_stream(stream);
  Level &F = h->levels.back();
  HIP_TRY(hipMemsetAsync(h->flags, 0, kNumFlags * sizeof(int), s));
  HIP_TRY(launch_check_positive(kappa_cells, F.ncells, h->flags, kFlagKappa, s, F.kappa64, kFlagChanged));
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (f & kFlagKappa) return fail(MFL_EINVAL, "kappa holds a value that is not finite and positive");
  // the handle's kappa, bit for bit: everything that depends on it is current
  if (!(f & kFlagChanged)) return MFL_OK;
  HIP_TRY(hipMemcpyAsync(F.kappa64, kappa_cells, F.ncells * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_cast(F.kappa64, MFL_F64, F.kappa32, MFL_F32, F.ncells, s));
  int rc = rebuild_kappa_dependent(*h, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return MFL_OK;
}

int mfl_num_levels(mfl_handle h) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  return int(h->levels.size());
}

int mfl_level_info(mfl_handle h, int level, int *cells_per_dim, int64_t *n_dofs, double *lambda_max,
                   double *coarse_lmin, double *coarse_lmax, int *coarse_steps) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  const int l = level_index(*h, level);
  if (l < 0) return fail(MFL_EINVAL, "level %d out of range", level);
  const Level &L = h->levels[l];
  if (cells_per_dim) *cells_per_dim = L.Nc;
  if (n_dofs) *n_dofs = L.ndofs;
  if (lambda_max) *lambda_max = L.lambda_max;
  if (coarse_lmin) *coarse_lmin = L.coarse_lmin;
  if (coarse_lmax) *coarse_lmax = L.coarse_lmax;
  if (coarse_steps) *coarse_steps = L.coarse_steps;
  return MFL_OK;
}

int mfl_apply(mfl_handle h, int level, int dtype, const void *src, void *dst, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  const int l = level_index(*h, level);
  if (l < 0) return fail(MFL_EINVAL, "level %d out of range", level);
  if (dtype != MFL_F64 && dtype != MFL_F32) return fail(MFL_EINVAL, "unknown dtype %d", dtype);
  if (!src || !dst) return fail(MFL_EINVAL, "src/dst is NULL");
  if (src == dst) return fail(MFL_EINVAL, "src and dst must not overlap");
  if (h->p.disc == MFL_DISC_SIPG && (h->k + 1) % 2 == 0 &&
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return fail(MFL_EINVAL, "SIPG vectors with an even number of points per direction must be 16-byte aligned");
  return apply_level(*h, l, dtype, src, dst, as_stream(stream), true);
}

int mfl_apply_noalloc(const mfl_params *p, const double *kappa_cells, int dtype, const void *src, void *dst,
                      void *stream) {
  int rc = check_params(p);
  if (rc) return rc;
  if (p->disc != MFL_DISC_CG || p->geometry != MFL_GEOM_CARTESIAN || p->kappa_field != MFL_KAPPA_CELLWISE)
    return fail(MFL_EUNSUPPORTED, "mfl_apply_noalloc covers the continuous operator on Cartesian cells "
                                  "with a cellwise kappa");
  if (dtype != MFL_F64 && dtype != MFL_F32) return fail(MFL_EINVAL, "unknown dtype %d", dtype);
  if (!src || !dst) return fail(MFL_EINVAL, "src/dst is NULL");
  if (src == dst) return fail(MFL_EINVAL, "src and dst must not overlap");
  Context c;
  c.p = *p;
  c.p.build_mg = 0;
  c.k = p->degree;
  c.n = p->degree + 1;
  Level L;
  L.Nc = p->cells_per_dim;
  L.N1 = c.k * L.Nc + 1;
  L.ncells = int64_t(L.Nc) * L.Nc * L.Nc;
  L.ndofs = int64_t(L.N1) * L.N1 * L.N1;
  L.h = p->domain_len / L.Nc;
  // scratch layout: halo records, then kappa in the apply's precision (absent for FP64 with
  // a caller kappa), each 256-byte aligned
  const int64_t es = dtype == MFL_F64 ? 8 : 4;
  const int64_t halo_bytes = (cg_halo_elements(c.k, L.Nc, false) * es + 255) / 256 * 256;
  const bool own_kappa = !(dtype == MFL_F64 && kappa_cells);
  const int64_t need = halo_bytes + (own_kappa ? L.ncells * es : 0);
  if (need > MFL_NOALLOC_SCRATCH_BYTES)
    return fail(MFL_EINVAL, "this mesh needs %lld bytes of scratch; mfl_apply_noalloc has %lld",
                (long long)need, (long long)MFL_NOALLOC_SCRATCH_BYTES);
  char *ptr = nullptr;
  if ((rc = scratch_address(&ptr))) return rc;
  hipStream_t s = as_stream(stream);
  L.halo = ptr;
  if (dtype == MFL_F64) {
    L.kappa64 = own_kappa ? reinterpret_cast<double *>(ptr + halo_bytes) : const_cast<double *>(kappa_cells);
    if (own_kappa) HIP_TRY(launch_fill(L.kappa64, MFL_F64, L.ncells, 1.0, s));
  } else {
    L.kappa32 = reinterpret_cast<float *>(ptr + halo_bytes);
    if (kappa_cells)
      HIP_TRY(launch_cast(kappa_cells, MFL_F64, L.kappa32, MFL_F32, L.ncells, s));
    else
      HIP_TRY(launch_fill(L.kappa32, MFL_F32, L.ncells, 1.0, s));
  }
  HIP_TRY(launch_cg_apply(c, L, dtype, src, dst, s));
  HIP_TRY(launch_cg_halo_add(c, L, dtype, dst, s));
  return MFL_OK;
}

int mfl_profile(mfl_handle h, int enable, int *launches, double *total_ms) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (launches) *launches = 0;
  if (total_ms) *total_ms = 0.0;
  if (enable) {
    h->profiling = true;
    h->prof_used = 0;
    return MFL_OK;
  }
  double sum = 0.0;
  for (int i = 0; i < h->prof_used; ++i) {
    HIP_TRY(hipEventSynchronize(h->prof_stop[i]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, h->prof_start[i], h->prof_stop[i]));
    sum += ms;
  }
  if (launches) *launches = h->prof_used;
  if (total_ms) *total_ms = sum;
  h->profiling = false;
  h->prof_used = 0;
  return MFL_OK;
}

int mfl_diagonal(mfl_handle h, int level, int dtype, void *out, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  const int l = level_index(*h, level);
  if (l < 0) return fail(MFL_EINVAL, "level %d out of range", level);
  if (!out) return fail(MFL_EINVAL, "out is NULL");
  const Level &L = h->levels[l];
  hipStream_t s = as_stream(stream);
  if (dtype == MFL_F64)
    HIP_TRY(hipMemcpyAsync(out, L.diag64, L.ndofs * sizeof(double), hipMemcpyDeviceToDevice, s));
  else if (dtype == MFL_F32)
    HIP_TRY(hipMemcpyAsync(out, L.diag32, L.ndofs * sizeof(float), hipMemcpyDeviceToDevice, s));
  else
    return fail(MFL_EINVAL, "unknown dtype %d", dtype);
  return MFL_OK;
}

int mfl_transfer(mfl_handle h, int level, int direction, int dtype, const void *src, void *dst,
                 void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  const int l = level_index(*h, level);
  if (l < 1) return fail(MFL_EINVAL, "transfer needs a level >= 1 (got %d)", level);
  if (dtype != MFL_F64 && dtype != MFL_F32) return fail(MFL_EINVAL, "unknown dtype %d", dtype);
  if (!src || !dst) return fail(MFL_EINVAL, "src/dst is NULL");
  const int cdt = (l - 1 == 0) ? MFL_F64 : dtype;
  hipStream_t s = as_stream(stream);
  if (direction == 0)
    HIP_TRY(prolongate_from(*h, l, src, cdt, dst, dtype, s));
  else if (direction == 1)
    HIP_TRY(restrict_to(*h, l, src, nullptr, dtype, dst, cdt, s));
  else
    return fail(MFL_EINVAL, "direction must be 0 (prolongate) or 1 (restrict)");
  return MFL_OK;
}

int mfl_vcycle(mfl_handle h, const double *r, double *z, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (!need_mg(*h)) return fail(MFL_EINVAL, "handle was set up without multigrid (build_mg = 0)");
  if (!r || !z) return fail(MFL_EINVAL, "r/z is NULL");
  return vcycle(*h, r, z, as_stream(stream));
}

int mfl_pcg_solve(mfl_handle h, const double *b, double *x, double rtol, int maxit, int *iters,
                  double *final_rel_res, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (!need_mg(*h)) return fail(MFL_EINVAL, "handle was set up without multigrid (build_mg = 0)");
  if (!b || !x) return fail(MFL_EINVAL, "b/x is NULL");
  if (!(rtol > 0.0) || maxit < 1) return fail(MFL_EINVAL, "need rtol > 0 and maxit >= 1");
  return pcg(*h, b, x, rtol, maxit, iters, final_rel_res, as_stream(stream));
}

int mfl_rhs_sine(mfl_handle h, double *b, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (h->p.disc != MFL_DISC_CG) return fail(MFL_EUNSUPPORTED, "right-hand side helper is CG only");
  if (!b) return fail(MFL_EINVAL, "b is NULL");
  HIP_TRY(launch_rhs_sine(*h, h->levels.back(), b, as_stream(stream)));
  return MFL_OK;
}

int mfl_rhs_gaussians(mfl_handle h, double *b, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (h->p.geometry != MFL_GEOM_CARTESIAN)
    return fail(MFL_EUNSUPPORTED, "the three-Gaussian right-hand side needs a Cartesian mesh");
  if (!b) return fail(MFL_EINVAL, "b is NULL");
  hipStream_t s = as_stream(stream);
  const Level &F = h->levels.back();
  if (h->p.disc == MFL_DISC_SIPG) {
    HIP_TRY(launch_sipg_rhs_gaussians(*h, F, b, s));
    return MFL_OK;
  }
  // forcing and Neumann loads into b; x0 = Dirichlet data in r; z = A0 x0 (operator
  // without boundary conditions); then b = x0 on Dirichlet DoFs and b - z elsewhere
  HIP_TRY(launch_rhs_gaussians(*h, F, b, s));
  HIP_TRY(launch_gaussian_dirichlet(*h, F, h->r, s));
  HIP_TRY(launch_cg_apply(*h, F, MFL_F64, h->r, h->z, s, 0));
  HIP_TRY(launch_cg_halo_add(*h, F, MFL_F64, h->z, s, 0));
  HIP_TRY(launch_lift(*h, F, b, h->r, h->z, s));
  return MFL_OK;
}

int mfl_adjoint_solve(mfl_handle h, const double *dJdu, double *lambda, double rtol, int maxit,
                      int *iters, double *final_rel_res, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (!need_mg(*h)) return fail(MFL_EINVAL, "handle was set up without multigrid (build_mg = 0)");
  if (h->p.disc != MFL_DISC_CG) return fail(MFL_EUNSUPPORTED, "the adjoint solve is CG only");
  if (!dJdu || !lambda) return fail(MFL_EINVAL, "dJdu/lambda is NULL");
  if (!(rtol > 0.0) || maxit < 1) return fail(MFL_EINVAL, "need rtol > 0 and maxit >= 1");
  hipStream_t s = as_stream(stream);
  const Level &F = h->levels.back();
  // the right-hand side with zeroed Dirichlet entries is staged in the solution vector
  if (dJdu != lambda)
    HIP_TRY(hipMemcpyAsync(lambda, dJdu, F.ndofs * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_zero_boundary(lambda, F, dirichlet_mask(h->p), s));
  HIP_TRY(hipMemcpyAsync(h->q, lambda, F.ndofs * sizeof(double), hipMemcpyDeviceToDevice, s));
  // pcg() uses r, z, pv, q as work: move the staged right-hand side to the level's x-free slot
  double *rhs = h->q;
  // pcg copies b into r before q is first written, so q can carry b into the solve
  return pcg(*h, rhs, lambda, rtol, maxit, iters, final_rel_res, s);
}

int mfl_kappa_gradient(mfl_handle h, const double *u, const double *lambda, double *grad, void *stream) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (h->p.disc != MFL_DISC_CG) return fail(MFL_EUNSUPPORTED, "kappa gradient is CG only");
  if (!u || !lambda || !grad) return fail(MFL_EINVAL, "u/lambda/grad is NULL");
  HIP_TRY(launch_cg_kappa_grad(*h, h->levels.back(), u, lambda, grad, as_stream(stream)));
  return MFL_OK;
}

int mfl_destroy(mfl_handle h) {
  if (!h) return fail(MFL_EINVAL, "handle is NULL");
  if (h->vcycle_graph) (void)hipGraphExecDestroy(h->vcycle_graph);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->host_scalars) (void)hipHostFree(h->host_scalars);
  if (h->host_coarse) (void)hipHostFree(h->host_coarse);
  for (hipEvent_t e : h->prof_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->prof_stop) (void)hipEventDestroy(e);
  delete h;
  return MFL_OK;
}

const char *mfl_last_error(void) { return g_error.c_str(); }

}  // extern "C"
