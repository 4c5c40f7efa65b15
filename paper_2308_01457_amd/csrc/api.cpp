// C ABI of the library (declared in include/fosb.h): argument validation,
// object lifetimes, and the host-side orchestration of the kernels.
#include <algorithm>
#include <array>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <atomic>
#include <exception>
#include <map>
#include <thread>

#include "common.h"

namespace fosb {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(fosb_status s, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(s, buf);
}

static void check_opts(const fosb_opts& o) {
  if (o.n_gauss_singular < 1 || o.n_gauss_singular > 12) fail(FOSB_E_INVALID, "opts: n_gauss_singular must be 1..12");
  if (o.ir_max_sweeps < 0 || o.ir_max_sweeps > 50) fail(FOSB_E_INVALID, "opts: ir_max_sweeps must be 0..50");
  if (!(o.ir_tol > 0.0) || !std::isfinite(o.ir_tol)) fail(FOSB_E_INVALID, "opts: ir_tol must be positive");
  if (o.certify != 0 && o.certify != 1) fail(FOSB_E_INVALID, "opts: certify must be 0 or 1");
  if (o.lu_pivoting != 0 && o.lu_pivoting != 1) fail(FOSB_E_INVALID, "opts: lu_pivoting must be 0 or 1");
}

static fosb_opts opts_or_default(const fosb_opts* o) {
  fosb_opts r;
  r.n_gauss_singular = 5;
  r.ir_max_sweeps = 10;
  r.ir_tol = 1e-10;
  r.certify = 0;
  r.lu_pivoting = 0;
  if (o) r = *o;
  check_opts(r);
  return r;
}

// Makes ctx's device current and its caching pool the calling thread's pool.
static void bind(Context& ctx) {
  FOSB_HIP(hipSetDevice(ctx.device));
  bind_pool(ctx);
}

static void merge_stats(fosb_stats* dst, const fosb_stats& src) {
  if (!dst) return;
  dst->ir_sweeps = std::max(dst->ir_sweeps, src.ir_sweeps);
  dst->n_solves += src.n_solves;
  dst->ir_rel_correction = std::max(dst->ir_rel_correction, src.ir_rel_correction);
  dst->backward_error = std::max(dst->backward_error, src.backward_error);
  dst->kappa1 = std::max(dst->kappa1, src.kappa1);
  dst->growth = std::max(dst->growth, src.growth);
}

static void merge_level_certificate(fosb_stats* dst, const Level& L) {
  if (!dst) return;
  dst->kappa1 = std::max(dst->kappa1, L.kappa1);
  dst->growth = std::max(dst->growth, L.growth);
}

// ------------------------------------------------------------------ level solve
// B <- Z^{-1} B (or Z^{-H} B) for a factorised level; MIXED levels refine in FP64.
// With P Z = L U:  Z^{-1} = U^{-1} L^{-1} P  and  Z^{-H} = P^T L^{-H} U^{-H}.
void level_solve_inplace(Context& ctx, const Level& L, c128* B, int64_t ldb, int64_t nrhs, fosb_stats* st,
                         bool adjoint, int max_sweeps) {
  hipStream_t s = ctx.stream;
  const int64_t n = L.n;
  if (nrhs <= 0) return;
  const size_t bytes128 = (size_t)n * nrhs * sizeof(c128);
  const int32_t* perm = L.d_perm.as<int32_t>();
  ctx.scratch[1].reserve(bytes128);
  c128* T = ctx.scratch[1].as<c128>();
  if (L.precision == FOSB_PREC_FP64) {
    const c128* A = static_cast<const c128*>(L.Z);
    if (!adjoint) {
      permute_rows_gather(s, perm, B, ldb, T, nrhs, n, nrhs);
      trsm_lower_unit<double>(ctx, A, L.ldz, L.dinv_L.as<c128>(), 0, n, T, nrhs, nrhs);
      trsm_upper<double>(ctx, A, L.ldz, L.dinv_U.as<c128>(), 0, n, T, nrhs, nrhs);
      copy_c128(s, T, nrhs, B, ldb, n, nrhs);
    } else {
      copy_c128(s, B, ldb, T, nrhs, n, nrhs);
      trsm_upper_ch<double>(ctx, A, L.ldz, L.dinv_U.as<c128>(), 0, n, T, nrhs, nrhs);
      trsm_lower_unit_ch<double>(ctx, A, L.ldz, L.dinv_L.as<c128>(), 0, n, T, nrhs, nrhs);
      permute_rows_scatter(s, perm, T, nrhs, B, ldb, n, nrhs);
    }
    if (st) st->ir_sweeps = std::max(st->ir_sweeps, 0);
    return;
  }
  // mixed: FP32 LU solves + FP64 residuals against the kept complex128 Z, or
  // against Z re-assembled band by band when the level keeps no FP64 copy
  const int sweep_limit = max_sweeps >= 0 ? max_sweeps : L.opts.ir_max_sweeps;
  if (!L.Z && adjoint && sweep_limit > 0)
    fail(FOSB_E_UNSUPPORTED, "adjoint solves need the level's stored FP64 matrix (this level re-assembles it)");
  ctx.scratch[2].reserve(bytes128);
  ctx.scratch[3].reserve(bytes128);
  ctx.scratch[4].reserve((size_t)n * nrhs * sizeof(c64));
  ctx.scratch[5].reserve(bytes128);
  ctx.norms.reserve((2 + 2 * kNormBlocks) * sizeof(double));
  c128* Bo = ctx.scratch[2].as<c128>();
  c128* X = ctx.scratch[3].as<c128>();
  c64* R32 = ctx.scratch[4].as<c64>();
  c128* Rw = ctx.scratch[5].as<c128>();
  ctx.solve_tmp.reserve((size_t)n * nrhs * sizeof(c64));
  c64* Y32 = ctx.solve_tmp.as<c64>();  // L^{-1} P R between the two triangular solves
  const c64* A32 = static_cast<const c64*>(L.Zlow);
  const c128* Z64 = static_cast<const c128*>(L.Z);
  copy_c128(s, B, ldb, Bo, nrhs, n, nrhs);
  const c128* R = Bo;  // first residual is B itself
  // Each sweep contracts the error by about the FP32 solve's relative accuracy,
  // estimated by the ratio of consecutive corrections: after a correction of
  // relative size r_k following one of r_{k-1} (r_0 = 1, the first solve) the
  // iterate's error is about r_k^2 / r_{k-1}.  Refinement stops once that
  // estimate is below ir_tol.
  double prev = 1.0, rel = INFINITY, est = INFINITY;
  int sweeps = 0;
  for (int it = 0;; ++it) {
    c128* D;  // this sweep's correction
    if (!adjoint) {
      permute_rows_gather(s, perm, R, nrhs, T, nrhs, n, nrhs);
      copy_c128_to_c64(s, T, nrhs, R32, nrhs, n, nrhs);
      if (L.sym_sign) negate_rows_c64(s, R32, nrhs, n / 2, n, nrhs);   // (S Z)^{-1} S R
      trsm_lower_unit_inv<float>(ctx, A32, L.ldzlow, L.inv_L.as<c64>(), n, R32, nrhs, Y32, nrhs, nrhs);
      trsm_upper_inv<float>(ctx, A32, L.ldzlow, L.inv_U.as<c64>(), n, Y32, nrhs, R32, nrhs, nrhs);
      copy_c64_to_c128(s, R32, nrhs, T, nrhs, n, nrhs);
      D = T;
    } else {
      copy_c128_to_c64(s, R, nrhs, R32, nrhs, n, nrhs);
      trsm_upper_ch<float>(ctx, A32, L.ldzlow, L.dinv_U.as<c64>(), 0, n, R32, nrhs, nrhs);
      trsm_lower_unit_ch<float>(ctx, A32, L.ldzlow, L.dinv_L.as<c64>(), 0, n, R32, nrhs, nrhs);
      if (L.sym_sign) negate_rows_c64(s, R32, nrhs, n / 2, n, nrhs);   // Z^{-H} = S (S Z)^{-H}
      copy_c64_to_c128(s, R32, nrhs, T, nrhs, n, nrhs);
      permute_rows_scatter(s, perm, T, nrhs, Rw, nrhs, n, nrhs);  // R (if it was Rw) is consumed
      D = Rw;
    }
    if (it == 0) {
      copy_c128(s, D, nrhs, X, nrhs, n, nrhs);
    } else {
      axpy_c128(s, D, nrhs, X, nrhs, n, nrhs);
    }
    norms2_c128(s, D, nrhs, X, nrhs, n, nrhs, ctx.norms.as<double>());
    double nn[2];
    FOSB_HIP(hipMemcpyAsync(nn, ctx.norms.p, sizeof(nn), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    rel = nn[1] > 0 ? std::sqrt(nn[0] / nn[1]) : 0.0;
    est = it == 0 ? 1.0 : rel * rel / prev;
    if (it > 0) sweeps = it;
    if (est <= L.opts.ir_tol || it >= sweep_limit || (it > 1 && rel >= prev)) break;
    prev = rel;
    // residual R = Bo - op(Z64) X in FP64 (scratch[5])
    copy_c128(s, Bo, nrhs, Rw, nrhs, n, nrhs);
    if (!Z64)
      efie_residual(ctx, *L.mesh, L.k, L.opts.n_gauss_singular, X, nrhs, nrhs, Rw, nrhs);
    else if (!adjoint)
      gemm<double>(ctx, n, nrhs, n, -1.0, Z64, L.ldz, X, nrhs, 1.0, Rw, nrhs);
    else
      gemm_ch<double>(ctx, n, nrhs, n, -1.0, Z64, L.ldz, X, nrhs, 1.0, Rw, nrhs);
    R = Rw;
  }
  copy_c128(s, X, nrhs, B, ldb, n, nrhs);
  if (st && L.opts.certify && L.z_fro > 0) {
    // normwise backward error of the returned iterate: ||Bo - op(Z64) X|| / (||Z|| ||X|| + ||Bo||)
    copy_c128(s, Bo, nrhs, Rw, nrhs, n, nrhs);
    if (!Z64)
      efie_residual(ctx, *L.mesh, L.k, L.opts.n_gauss_singular, X, nrhs, nrhs, Rw, nrhs);
    else if (!adjoint)
      gemm<double>(ctx, n, nrhs, n, -1.0, Z64, L.ldz, X, nrhs, 1.0, Rw, nrhs);
    else
      gemm_ch<double>(ctx, n, nrhs, n, -1.0, Z64, L.ldz, X, nrhs, 1.0, Rw, nrhs);
    double rx[2], bb[2];
    norms2_c128(s, Rw, nrhs, X, nrhs, n, nrhs, ctx.norms.as<double>());
    FOSB_HIP(hipMemcpyAsync(rx, ctx.norms.p, sizeof(rx), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    norms2_c128(s, Bo, nrhs, Bo, nrhs, n, nrhs, ctx.norms.as<double>());
    FOSB_HIP(hipMemcpyAsync(bb, ctx.norms.p, sizeof(bb), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    const double den = L.z_fro * std::sqrt(rx[1]) + std::sqrt(bb[0]);
    if (den > 0) st->backward_error = std::max(st->backward_error, std::sqrt(rx[0]) / den);
  }
  if (st) {
    st->ir_sweeps = std::max(st->ir_sweeps, sweeps);
    st->ir_rel_correction = std::max(st->ir_rel_correction, rel);
  }
  if (est > L.opts.ir_tol && sweep_limit > 0) {
    FOSB_HIP(hipStreamSynchronize(s));
    fail(FOSB_E_NOCONV, "refinement stopped at estimated relative error %.3e after %d sweeps (tol %.1e)", est, sweeps,
         L.opts.ir_tol);
  }
}

// In place: C <- Sigma with Z1 Sigma Z2^H = C for nd incidences stacked side by
// side (C is N1 x nd*N2, direction d in columns d*N2 .. (d+1)*N2): one solve
// with nd*N2 right-hand sides, per-direction conjugate transposes into an
// N2 x nd*N1 slab, one solve with nd*N1 right-hand sides, and back.
static void two_sided(Context& ctx, const Level& l1, const Level& l2, c128* C, int64_t ldc, fosb_stats* st,
                      int64_t nd = 1) {
  const int64_t n1 = l1.n, n2 = l2.n;
  level_solve_inplace(ctx, l1, C, ldc, nd * n2, st);
  DevBuf& tb = ctx.scratch[0];
  tb.reserve((size_t)n1 * n2 * nd * sizeof(c128));
  c128* Tt = tb.as<c128>();
  for (int64_t d = 0; d < nd; ++d) conj_transpose_c128(ctx.stream, C + d * n2, ldc, Tt + d * n1, nd * n1, n1, n2);
  level_solve_inplace(ctx, l2, Tt, nd * n1, nd * n1, st);
  for (int64_t d = 0; d < nd; ++d) conj_transpose_c128(ctx.stream, Tt + d * n1, nd * n1, C + d * n2, ldc, n2, n1);
  if (st) st->n_solves += (int32_t)nd;
}

}  // namespace fosb

using namespace fosb;


// Every entry point drops the thread's pool binding when it returns, so a
// thread holds no reference to a context's pool between calls.
struct PoolRelease {
  ~PoolRelease() { fosb::thread_pool().reset(); }
};

#define API_BEGIN \
  PoolRelease pool_release_; \
  try {
#define API_END                                                   \
  }                                                               \
  catch (const fosb::Error& e) {                                  \
    set_last_error(e.what());                                     \
    return e.status;                                              \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    set_last_error("host allocation failed");                     \
    return FOSB_E_OOM;                                            \
  }                                                               \
  catch (const std::exception& e) {                               \
    set_last_error(e.what());                                     \
    return FOSB_E_DEVICE;                                         \
  }                                                               \
  catch (...) {                                                   \
    set_last_error("unknown error");                              \
    return FOSB_E_DEVICE;                                         \
  }                                                               \
  set_last_error("");                                             \
  return FOSB_OK;

#define REQUIRE(cond, ...) \
  do {                     \
    if (!(cond)) fail(FOSB_E_INVALID, __VA_ARGS__); \
  } while (0)


struct fosb_context : fosb::Context {};

// Low-rank covariance factor of a level ladder (fosb_lowrank_*).
struct fosb_lowrank {
  fosb::Context* ctx = nullptr;
  std::vector<const fosb::Level*> levels;   // the ladder, coarse to fine
  std::vector<int64_t> off;                 // first candidate row of each level
  fosb_cov cov{};
  int64_t nc = 0;
  int32_t rank = 0;
  double residual = 1.0;
  std::vector<int64_t> pivots;
  fosb::DevBuf L;                           // factor, column-major nc x rank (double)
};
struct fosb_mesh : fosb::Mesh {};
struct fosb_level : fosb::Level {};

namespace fosb {

static void check_physics(double k, int32_t precision, const double* dirs, const double* pols, int64_t n_dirs,
                          int32_t field) {
  REQUIRE(std::isfinite(k) && k > 0, "wavenumber must be positive and finite");
  REQUIRE(precision == FOSB_PREC_FP64 || precision == FOSB_PREC_MIXED, "unknown precision %d", precision);
  REQUIRE(field == FOSB_FIELD_RADIAL || field == FOSB_FIELD_NORMAL, "unknown field %d", field);
  REQUIRE(dirs && pols && n_dirs >= 1 && n_dirs <= 4096, "need 1..4096 incidence directions");
  for (int64_t d = 0; d < n_dirs; ++d) {
    double nd = 0, np = 0;
    for (int c = 0; c < 3; ++c) {
      REQUIRE(std::isfinite(dirs[3 * d + c]) && std::isfinite(pols[3 * d + c]), "non-finite direction/polarisation");
      nd += dirs[3 * d + c] * dirs[3 * d + c];
      np += pols[3 * d + c] * pols[3 * d + c];
    }
    REQUIRE(std::fabs(nd - 1.0) < 1e-9, "direction %lld is not a unit vector", (long long)d);
    REQUIRE(np > 0, "polarisation %lld is zero", (long long)d);
  }
}

static void check_level_args(const fosb_mesh* mesh, double k, int32_t precision, void* Z, int64_t ldz, void* Zlow,
                             int64_t ldzlow, const double* dirs, const double* pols, int64_t n_dirs, int32_t field) {
  check_physics(k, precision, dirs, pols, n_dirs, field);
  REQUIRE(Z || precision == FOSB_PREC_MIXED, "Z is NULL (only a MIXED level may re-assemble its FP64 matrix)");
  const int64_t n = mesh->h.ne;
  if (Z && ldz < n) fail(FOSB_E_WORKSPACE, "ldz < N");
  if (precision == FOSB_PREC_MIXED) {
    REQUIRE(Zlow, "MIXED precision needs the complex64 buffer Zlow");
    if (ldzlow < n) fail(FOSB_E_WORKSPACE, "ldzlow < N");
  } else {
    REQUIRE(!Zlow, "FP64 precision takes no Zlow buffer");
  }
}

// Estimate of ||Z^{-1}||_1 from a few solves with Z and Z^H: the 1-norm
// estimator of Hager (1984) in Higham's form (ACM TOMS 14, 1988), for complex
// matrices.  x starts uniform; each step solves y = Z^{-1} x, takes the
// complex signs xi of y, solves z = Z^{-H} xi and moves x to the unit vector of
// the largest |z_j|, until ||y||_1 stops growing or j repeats (at most five
// steps).  An alternating-sign test vector guards against the estimator's
// known bad cases.  The result is a lower bound of ||Z^{-1}||_1.
static double inverse_norm1_estimate(Context& c, const Level& L) {
  const int64_t n = L.n;
  hipStream_t s = c.stream;
  std::vector<c128> h(n);
  DevBuf v((size_t)n * sizeof(c128));
  // a level without a stored FP64 matrix estimates with its unrefined FP32 factors
  const int sweeps = L.Z ? -1 : 0;
  auto solve = [&](bool adjoint) {
    FOSB_HIP(hipMemcpyAsync(v.p, h.data(), n * sizeof(c128), hipMemcpyHostToDevice, s));
    level_solve_inplace(c, L, v.as<c128>(), 1, 1, nullptr, adjoint, sweeps);
    FOSB_HIP(hipMemcpyAsync(h.data(), v.p, n * sizeof(c128), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
  };
  auto norm1 = [&]() {
    double a = 0;
    for (const c128& z : h) a += std::hypot(z.re, z.im);
    return a;
  };
  for (auto& z : h) z = c128{1.0 / (double)n, 0.0};
  double est = 0;
  int64_t jlast = -1;
  for (int it = 0; it < 5; ++it) {
    solve(false);
    const double e = norm1();
    if (it > 0 && e <= est) break;
    est = e;
    for (auto& z : h) {
      const double m = std::hypot(z.re, z.im);
      z = m > 0 ? c128{z.re / m, z.im / m} : c128{1.0, 0.0};
    }
    solve(true);
    int64_t j = 0;
    double best = -1;
    for (int64_t i = 0; i < n; ++i) {
      const double m = std::hypot(h[i].re, h[i].im);
      if (m > best) {
        best = m;
        j = i;
      }
    }
    if (j == jlast) break;
    jlast = j;
    for (auto& z : h) z = c128{0.0, 0.0};
    h[j] = c128{1.0, 0.0};
  }
  for (int64_t i = 0; i < n; ++i)
    h[i] = c128{(i % 2 ? -1.0 : 1.0) * (1.0 + (n > 1 ? (double)i / (double)(n - 1) : 0.0)), 0.0};
  solve(false);
  return std::max(est, 2.0 * norm1() / (3.0 * (double)n));
}

// Factorisation, first moments and RHS weights of one level, on c's stream.
static std::unique_ptr<fosb_level> level_build(Context& c, const fosb_mesh* mesh, double k, int32_t precision,
                                               void* Z, int64_t ldz, void* Zlow, int64_t ldzlow, const double* dirs,
                                               const double* pols, int64_t n_dirs, int32_t field,
                                               const fosb_opts& o, int32_t form = FOSB_FORM_EFIE,
                                               double eps_r = 1.0, double mu_r = 1.0, int32_t sd_field = -1,
                                               bool sd_streamed = false, bool zlow_ready = false) {
  hipStream_t s = c.stream;
  const bool pm = form == FOSB_FORM_PMCHWT;
  const int64_t n = pm ? 2 * mesh->h.ne : mesh->h.ne;
  std::unique_ptr<fosb_level> L(new fosb_level());
  L->form = form;
  L->eps_r = eps_r;
  L->mu_r = mu_r;
  L->ctx = &c;
  L->mesh = mesh;
  L->k = k;
  L->precision = precision;
  L->n = n;
  L->Z = Z;
  L->ldz = ldz;
  L->Zlow = Zlow;
  L->ldzlow = ldzlow;
  L->n_dirs = n_dirs;
  L->field = field;
  L->opts = o;
  const int64_t nblk = (n + kPanel - 1) / kPanel;
  int64_t info = 0;
  DevBuf cert;
  // norms of the assembled matrix (certificates), taken before the factorisation
  // overwrites it: of Z, or of its complex64 rounding for a level that keeps no
  // FP64 copy (within 1e-7 of the FP64 norms)
  auto matrix_certificate = [&](bool fp32) {
    cert.alloc(6 * sizeof(double));
    if (fp32)
      matrix_norms<float>(c, static_cast<const c64*>(Zlow), n, ldzlow, false, cert.as<double>());
    else
      matrix_norms<double>(c, static_cast<const c128*>(Z), n, ldz, false, cert.as<double>());
    double zn[3];
    FOSB_HIP(hipMemcpyAsync(zn, cert.p, sizeof(zn), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    L->z_max = zn[0];
    L->z_fro = std::sqrt(zn[1]);
    L->z_one = zn[2];
  };
  if (o.certify && Z) matrix_certificate(false);
  if (precision == FOSB_PREC_FP64) {
    L->dinv_L.alloc((size_t)nblk * kPanel * kPanel * sizeof(c128));
    L->dinv_U.alloc((size_t)nblk * kPanel * kPanel * sizeof(c128));
    info = lu_factor<double>(c, static_cast<c128*>(Z), n, ldz, L->dinv_L.as<c128>(), L->dinv_U.as<c128>(), L->perm);
  } else {
    L->dinv_L.alloc((size_t)nblk * kPanel * kPanel * sizeof(c64));
    L->dinv_U.alloc((size_t)nblk * kPanel * kPanel * sizeof(c64));
    if (Z) {
      // zlow_ready: the assembly that wrote Z also stored it rounded to complex64
      if (!zlow_ready) copy_c128_to_c64(s, static_cast<const c128*>(Z), ldz, static_cast<c64*>(Zlow), ldzlow, n, n);
    } else {  // no FP64 copy: assemble in FP64 column bands straight into complex64
      assemble_efie_c64(c, *mesh, k, o.n_gauss_singular, static_cast<c64*>(Zlow), ldzlow);
      if (o.certify) matrix_certificate(true);
    }
    // the refined solves apply the factors through their diagonal-block inverses
    const size_t bytes = (size_t)((n + kInvBlock - 1) / kInvBlock) * kInvBlock * kInvBlock * sizeof(c64);
    L->inv_L.alloc(bytes);
    L->inv_U.alloc(bytes);
    bool factored = false;
    if (o.lu_pivoting == 0 && n >= 2048) {
      // symmetric matrix: no pivoting, half the trailing-update flops; kept when no
      // pivot vanished and the growth factor stays below 1e3.  The EFIE matrix is
      // symmetric; the PMCHWT matrix [[A, K], [-K, D]] (A, D, K symmetric) is not,
      // but S Z = [[A, K], [K, -D]] is, with S = diag(I, -I) on the [J; M] halves:
      // its factors serve Z^{-1} = (S Z)^{-1} S.
      if (pm) negate_rows_c64(s, static_cast<c64*>(Zlow), ldzlow, n / 2, n, n);
      double defect = 0.0, zmax = 0.0;
      sym_check<float>(c, static_cast<const c64*>(Zlow), n, ldzlow, &defect, &zmax);
      const bool symmetric = zmax > 0 && std::isfinite(zmax) && defect <= 1e-5 * zmax;
      if (symmetric) {
        info = lu_factor<float>(c, static_cast<c64*>(Zlow), n, ldzlow, L->dinv_L.as<c64>(), L->dinv_U.as<c64>(),
                                L->perm, L->inv_L.as<c64>(), true);
        const double growth = absmax_upper<float>(c, static_cast<const c64*>(Zlow), n, ldzlow) / zmax;
        factored = info == 0 && std::isfinite(growth) && growth <= 1e3;
        L->sym_lu = factored ? 1 : 0;
        L->sym_sign = factored && pm ? 1 : 0;
      }
      if (!factored && (symmetric || pm)) {  // start again from the assembled matrix with pivoting
        if (Z)
          copy_c128_to_c64(s, static_cast<const c128*>(Z), ldz, static_cast<c64*>(Zlow), ldzlow, n, n);
        else
          assemble_efie_c64(c, *mesh, k, o.n_gauss_singular, static_cast<c64*>(Zlow), ldzlow);
      }
    }
    if (!factored)
      info = lu_factor<float>(c, static_cast<c64*>(Zlow), n, ldzlow, L->dinv_L.as<c64>(), L->dinv_U.as<c64>(),
                              L->perm, L->inv_L.as<c64>());
    if (info == 0)
      upper_block_inverses<float>(c, static_cast<const c64*>(Zlow), n, ldzlow, L->dinv_U.as<c64>(),
                                  L->inv_U.as<c64>());
  }
  if (info != 0) fail(FOSB_E_SINGULAR, "exactly zero pivot at index %lld", (long long)(info - 1));
  upload(L->d_perm, L->perm, s);
  if (o.certify) {  // growth factor max|U| / max|Z| of the stored factors
    double un[3];
    if (precision == FOSB_PREC_FP64)
      matrix_norms<double>(c, static_cast<const c128*>(Z), n, ldz, true, cert.as<double>() + 3);
    else
      matrix_norms<float>(c, static_cast<const c64*>(Zlow), n, ldzlow, true, cert.as<double>() + 3);
    FOSB_HIP(hipMemcpyAsync(un, cert.as<double>() + 3, sizeof(un), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    L->growth = L->z_max > 0 ? un[0] / L->z_max : 0.0;
  }
  std::vector<double> dp(dirs, dirs + 3 * n_dirs), pp(pols, pols + 3 * n_dirs);
  DevBuf ddir, dpol;
  upload(ddir, dp, s);
  upload(dpol, pp, s);
  L->u.alloc((size_t)n * n_dirs * sizeof(c128));
  if (pm) {  // dielectric: keep the right-hand sides b = [e; h], first moments u = Z^{-1} b
    L->b.alloc((size_t)n * n_dirs * sizeof(c128));
    incident_rhs_pmchwt(s, *mesh, k, ddir.as<double>(), dpol.as<double>(), (int)n_dirs, L->b.as<c128>());
    copy_c128(s, L->b.as<c128>(), n_dirs, L->u.as<c128>(), n_dirs, n, n_dirs);
    level_solve_inplace(c, *L, L->u.as<c128>(), n_dirs, n_dirs, nullptr);
    if (sd_field >= 0) {  // shape-derivative weights per incidence, and the nodes for the covariance
      const int64_t Q = 6LL * mesh->h.nt;
      L->sd_field = sd_field;
      L->sd_streamed = sd_streamed ? 1 : 0;
      L->qx.alloc((size_t)3 * Q * sizeof(double));
      quad_nodes(s, *mesh, L->qx.as<double>());
      if (!sd_streamed) {
        L->Wsd.alloc((size_t)n_dirs * n * Q * sizeof(c128));
        ProfScope prof(c, FOSB_K_RHS, 0.0, 16.0 * (double)n_dirs * (double)n * (double)Q);
        for (int64_t d = 0; d < n_dirs; ++d)
          sd_weights(c, *mesh, k, eps_r, sd_field, L->u.as<c128>(), n_dirs, d, o.n_gauss_singular,
                     L->Wsd.as<c128>() + d * n * Q, Q);
      }
    }
    if (o.certify) L->kappa1 = L->z_one * inverse_norm1_estimate(c, *L);
    FOSB_HIP(hipStreamSynchronize(s));
    return L;
  }
  // quadrature nodes, first moments and RHS weights
  L->qx.alloc((size_t)3 * 6 * mesh->h.nt * sizeof(double));
  quad_nodes(s, *mesh, L->qx.as<double>());
  incident_rhs(s, *mesh, k, ddir.as<double>(), dpol.as<double>(), (int)n_dirs, L->u.as<c128>());
  level_solve_inplace(c, *L, L->u.as<c128>(), n_dirs, n_dirs, nullptr);
  L->W.alloc((size_t)n_dirs * mesh->h.nt * 18 * sizeof(c128));
  for (int64_t d = 0; d < n_dirs; ++d)
    rhs_weights(s, *mesh, k, field, L->u.as<c128>() + d, n_dirs, L->W.as<c128>() + d * mesh->h.nt * 18);
  if (o.certify) L->kappa1 = L->z_one * inverse_norm1_estimate(c, *L);
  FOSB_HIP(hipStreamSynchronize(s));
  return L;
}


// Hn (Q x R, R = 3 n_a) = (FF Z^{-1} Wgt_dir)^T: the rows of the map from the
// values of the perturbation amplitude at the level's quadrature nodes to the
// far field of the shape derivative, from one adjoint solve Z^{-H} FF^H with
// R right-hand sides.  dx: device angles (n_a x 3).
static void adjoint_node_rows(Context& c, const Level& l, const double* dx, int64_t n_a, int64_t dir, DevBuf& Hn,
                              fosb_stats* st) {
  hipStream_t s = c.stream;
  const int64_t R = 3 * n_a, N = l.n, Q = 6LL * l.mesh->h.nt;
  DevBuf FF((size_t)R * N * sizeof(c128)), Y((size_t)N * R * sizeof(c128));
  far_field_matrix_kernel(s, *l.mesh, l.k, dx, n_a, FF.as<c128>());
  conj_transpose_c128(s, FF.as<c128>(), N, Y.as<c128>(), R, R, N);   // Y = FF^H (N x R)
  level_solve_inplace(c, l, Y.as<c128>(), R, R, st, true);           // Y = Z^{-H} FF^H
  Hn.alloc((size_t)Q * R * sizeof(c128));
  adjoint_nodes(s, *l.mesh, l.W.as<c128>() + dir * l.mesh->h.nt * 18, Y.as<c128>(), R, Hn.as<c128>());
}

// Device bytes a level keeps for its lifetime.
static int64_t level_bytes(int64_t n, int64_t nt, int32_t precision, int64_t n_dirs) {
  const int64_t nblk = (n + kPanel - 1) / kPanel;
  const int64_t es = precision == FOSB_PREC_FP64 ? 16 : 8;
  int64_t b = 4 * n + 2 * nblk * kPanel * kPanel * es + 18 * nt * 8 + 16 * n * n_dirs + 18 * nt * n_dirs * 16;
  if (precision == FOSB_PREC_MIXED) b += 2 * ((n + kInvBlock - 1) / kInvBlock) * kInvBlock * kInvBlock * 8;
  return b;
}

// Largest work buffer bytes of a solve with nrhs right-hand sides (refined for MIXED).
static int64_t solve_work_bytes(int64_t n, int32_t precision, int64_t nrhs) {
  return precision == FOSB_PREC_FP64 ? 16 * n * nrhs : (4 * 16 + 2 * 8) * n * nrhs;
}

// Fails with FOSB_E_OOM, before any launch, when `need` bytes exceed the
// device's free memory plus what the context's pools hold for reuse.
static void check_device_memory(Context& ctx, int64_t need, const char* what) {
  size_t free_b = 0, total_b = 0;
  FOSB_HIP(hipMemGetInfo(&free_b, &total_b));
  int64_t n_alloc = 0, cached = 0, live = 0;
  pool_totals(ctx, n_alloc, cached, live);
  const int64_t avail = (int64_t)free_b + cached;
  if (need > avail)
    fail(FOSB_E_OOM, "%s needs about %.2f GB of device memory; %.2f GB are free (%.2f GB of it cached by the context)",
         what, need / 1e9, avail / 1e9, cached / 1e9);
}

static void check_pair(const fosb_context* ctx, const fosb_level* a, const fosb_level* b) {
  REQUIRE(a && b, "level is NULL");
  REQUIRE(a->ctx == ctx && b->ctx == ctx, "level belongs to another context");
  REQUIRE(a->k == b->k, "levels have different wavenumbers");
  REQUIRE(a->n_dirs == b->n_dirs, "levels have different incidence sets");
  REQUIRE(a->field == b->field, "levels use different perturbation fields");
  REQUIRE(a->form == b->form && a->eps_r == b->eps_r && a->mu_r == b->mu_r && a->sd_field == b->sd_field,
          "levels use different formulations, materials or perturbation fields");
}

// Entry points built on the PEC shape-derivative weights take EFIE levels only.
static void require_efie(const fosb_level* const* levels, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (levels[i] && levels[i]->form != FOSB_FORM_EFIE)
      fail(FOSB_E_UNSUPPORTED, "this entry point needs EFIE levels (the dielectric shape-derivative right-hand "
                               "side is not built)");
}

// Far-field map of a level of either formulation (rows 3 n_a, N columns).
static void level_far_field(hipStream_t s, const Level& l, const double* dx, int64_t n_a, c128* FF) {
  if (l.form == FOSB_FORM_PMCHWT)
    far_field_matrix_pmchwt(s, *l.mesh, l.k, dx, n_a, FF);
  else
    far_field_matrix_kernel(s, *l.mesh, l.k, dx, n_a, FF);
}

// C = Wsd_a K Wsd_b^H for dielectric levels with shape-derivative weights, K
// the amplitude covariance at the nodes of both levels, formed in row chunks
// of at most 2^26 entries: T = K_chunk Wsd_b^H, C += Wsd_a[:, chunk] T.
static void sd_correlation(Context& c, const Level& a, const Level& b, const fosb_cov& cov, int64_t dir, c128* C,
                           int64_t ldc) {
  hipStream_t s = c.stream;
  const int64_t Q1 = 6LL * a.mesh->h.nt, Q2 = 6LL * b.mesh->h.nt, n1 = a.n, n2 = b.n;
  const c128* W1 = a.Wsd.as<c128>() + dir * n1 * Q1;
  const c128* W2 = b.Wsd.as<c128>() + dir * n2 * Q2;
  DevBuf W2h((size_t)Q2 * n2 * sizeof(c128));
  conj_transpose_c128(s, W2, Q2, W2h.as<c128>(), n2, n2, Q2);
  const int64_t na = std::max<int64_t>(1, std::min<int64_t>(Q1, ((int64_t)1 << 26) / Q2));
  DevBuf Kc((size_t)na * Q2 * sizeof(c128)), T((size_t)na * n2 * sizeof(c128));
  for (int64_t a0 = 0; a0 < Q1; a0 += na) {
    const int64_t nr = std::min(na, Q1 - a0);
    cov_matrix(s, a, b, cov, a0, nr, Kc.as<c128>());
    gemm<double>(c, nr, n2, Q2, 1.0, Kc.as<c128>(), Q2, W2h.as<c128>(), n2, 0.0, T.as<c128>(), n2);
    gemm<double>(c, n1, n2, nr, 1.0, W1 + a0, Q1, T.as<c128>(), n2, a0 == 0 ? 0.0 : 1.0, C, ldc);
  }
  FOSB_HIP(hipStreamSynchronize(s));
}

// RHS correlation of a pair: the covariance form (EFIE, or dielectric levels
// with shape-derivative weights) or the rank-one b_l1 b_l2^H (dielectric, cov NULL).
static void pair_rhs(Context& c, const Level& a, const Level& b, const fosb_cov* cov, int64_t dir, c128* C,
                     int64_t ldc) {
  if (a.form == FOSB_FORM_PMCHWT && !cov)
    rank_one_correlation(c.stream, a.b.as<c128>(), a.n, b.b.as<c128>(), b.n, a.n_dirs, dir, C, ldc);
  else if (a.form == FOSB_FORM_PMCHWT)
    sd_correlation(c, a, b, *cov, dir, C, ldc);
  else
    rhs_correlation_kernel(c.stream, a, b, *cov, dir, C, ldc);
}

static void check_cov_for(const fosb_level* l, const fosb_cov* cov);

static void check_cov(const fosb_cov* cov) {
  REQUIRE(cov, "cov is NULL");
  REQUIRE(cov->kind >= FOSB_COV_GAUSSIAN && cov->kind <= FOSB_COV_NORMAL_DOT, "unknown covariance kind %d", cov->kind);
  REQUIRE(std::isfinite(cov->sigma) && cov->sigma >= 0, "sigma must be >= 0");
  if (cov->kind == FOSB_COV_GAUSSIAN || cov->kind == FOSB_COV_MATERN32)
    REQUIRE(std::isfinite(cov->ell) && cov->ell > 0, "ell must be > 0");
}

static void check_cov_for(const fosb_level* l, const fosb_cov* cov) {
  if (l->form == FOSB_FORM_PMCHWT && !cov) return;   // rank-one right-hand side
  if (l->form == FOSB_FORM_PMCHWT) {
    REQUIRE(l->sd_field >= 0, "a covariance right-hand side needs dielectric levels built with shape-derivative "
                              "weights (field >= 0)");
    if (l->sd_streamed)
      fail(FOSB_E_UNSUPPORTED, "levels with streamed shape-derivative weights take the low-rank route");
  }
  check_cov(cov);
}

static std::vector<std::array<int32_t, 4>> ct_pairs_vec(int32_t L0, int32_t L) {
  std::vector<std::array<int32_t, 4>> out;
  const int32_t tots[2] = {L + L0, L + L0 - 1};
  const int32_t sg[2] = {1, -1};
  for (int q = 0; q < 2; ++q)
    for (int32_t l1 = L; l1 >= L0; --l1) {
      const int32_t l2 = tots[q] - l1;
      if (l2 >= L0 && l2 <= l1) out.push_back({l1, l2, sg[q], l1 == l2 ? 1 : 2});
    }
  return out;
}

static void check_far_field_args(const double* xhat, int64_t n_a, int32_t L0, int32_t L,
                                 const fosb_level* const* levels, void* const* blocks, const int64_t* ldb) {
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  for (int64_t i = 0; i < n_a; ++i) {
    double nn = xhat[3 * i] * xhat[3 * i] + xhat[3 * i + 1] * xhat[3 * i + 1] + xhat[3 * i + 2] * xhat[3 * i + 2];
    REQUIRE(std::fabs(nn - 1.0) < 1e-9, "xhat[%lld] is not a unit vector", (long long)i);
  }
  auto v = ct_pairs_vec(L0, L);
  for (size_t p = 0; p < v.size(); ++p) {
    REQUIRE(blocks[p], "block %zu is NULL", p);
    if (ldb[p] < levels[v[p][1] - L0]->n) fail(FOSB_E_WORKSPACE, "ldb[%zu] < N_l2", p);
  }
}

// var = sum over Lambda_H of sign mult Re diag(FF_l1 Sigma FF_l2^H) for nd
// incidences dir0 .. dir0+nd-1 (blocks stacked side by side as in two_sided,
// var[d*3 n_a ..]); mean_F (optional) = FF_L u_L per direction.  The far-field
// maps are formed once.  Synchronises c's stream.
static void far_field_impl(Context& c, const fosb_level* const* levels, int32_t L0, int32_t L, void* const* blocks,
                           const int64_t* ldb, const double* xhat, int64_t n_a, int64_t dir0, int64_t nd, double* var,
                           void* mean_F, void* cor = nullptr, bool near = false) {
  const int32_t n_levels = L - L0 + 1;
  hipStream_t s = c.stream;
  std::vector<double> x(xhat, xhat + 3 * n_a);
  DevBuf dx;
  upload(dx, x, s);
  const int64_t rows = 3 * n_a;
  auto v = ct_pairs_vec(L0, L);
  std::vector<DevBuf> FF(n_levels);
  for (int32_t i = 0; i < n_levels; ++i) {
    FF[i].alloc((size_t)rows * levels[i]->n * sizeof(c128));
    if (near)  // scattered field at field points instead of the far field at directions
      near_field_matrix_kernel(s, *levels[i]->mesh, levels[i]->k, dx.as<double>(), n_a, FF[i].as<c128>());
    else
      level_far_field(s, *levels[i], dx.as<double>(), n_a, FF[i].as<c128>());
  }
  zero_f64(s, var, nd * rows);
  if (cor) {
    if (nd != 1) fail(FOSB_E_UNSUPPORTED, "the angular correlation is computed for one incidence at a time");
    zero_f64(s, static_cast<double*>(cor), 2 * 3 * n_a * n_a);
  }
  // one product FF_l1 [Sigma_0 | Sigma_1 | ...] per pair covers every incidence
  int64_t maxn2 = 0;
  for (auto& q : v) maxn2 = std::max(maxn2, levels[q[1] - L0]->n);
  DevBuf P((size_t)rows * nd * maxn2 * sizeof(c128));
  for (size_t p = 0; p < v.size(); ++p) {
    const int i1 = v[p][0] - L0, i2 = v[p][1] - L0;
    const int64_t n1 = levels[i1]->n, n2 = levels[i2]->n;
    gemm<double>(c, rows, nd * n2, n1, 1.0, FF[i1].as<c128>(), n1, static_cast<const c128*>(blocks[p]), ldb[p], 0.0,
                 P.as<c128>(), nd * n2);
    for (int64_t d = 0; d < nd; ++d)
      row_dot_re_accumulate(s, P.as<c128>() + d * n2, nd * n2, FF[i2].as<c128>(), rows, n2,
                            (double)(v[p][2] * v[p][3]), var + d * rows);
    if (cor) {  // per component c: (FF1 Sigma)_c FF2_c^H, with its conjugate transpose for l1 != l2
      DevBuf F2h((size_t)n2 * rows * sizeof(c128)), T((size_t)n_a * n_a * sizeof(c128));
      conj_transpose_c128(s, FF[i2].as<c128>(), n2, F2h.as<c128>(), rows, rows, n2);
      for (int cc = 0; cc < 3; ++cc) {
        gemm<double>(c, n_a, n_a, n2, 1.0, P.as<c128>() + cc * n_a * n2, n2, F2h.as<c128>() + cc * n_a, rows, 0.0,
                     T.as<c128>(), n_a);
        herm_accumulate(s, T.as<c128>(), n_a, n_a, (double)v[p][2], v[p][0] != v[p][1],
                        static_cast<c128*>(cor) + cc * n_a * n_a, n_a);
      }
    }
  }
  if (mean_F) {
    const int iL = n_levels - 1;
    c.scratch[1].reserve((size_t)levels[iL]->n * sizeof(c128));
    for (int64_t d = 0; d < nd; ++d) {
      copy_c128(s, levels[iL]->u.as<c128>() + dir0 + d, levels[iL]->n_dirs, c.scratch[1].as<c128>(), 1,
                levels[iL]->n, 1);
      matvec_rows(s, FF[iL].as<c128>(), rows, levels[iL]->n, c.scratch[1].as<c128>(),
                  static_cast<c128*>(mean_F) + d * rows);
    }
  }
  FOSB_HIP(hipStreamSynchronize(s));
}


// The whole pass for one ladder on c's stream alone, every incidence stacked,
// Z / Zlow / blocks from c's grow-only workspaces; var receives n_dirs
// consecutive 3 n_a vectors.  Used by the batch workers.
static void shape_pipeline(Context& c, const fosb_mesh* const* meshes, int32_t n_levels, int32_t L0, int32_t L,
                           double k, int32_t precision, const double* dirs, const double* pols, int64_t n_dirs,
                           int32_t field, const fosb_cov& cov, const double* xhat, int64_t n_a, double* var,
                           const fosb_opts& o, fosb_stats* st) {
  const bool mixed = precision == FOSB_PREC_MIXED;
  auto v = ct_pairs_vec(L0, L);
  if (c.ws_Z.size() < (size_t)n_levels) c.ws_Z.resize(n_levels);
  if (c.ws_Zlow.size() < (size_t)n_levels) c.ws_Zlow.resize(n_levels);
  if (c.ws_blocks.size() < v.size()) c.ws_blocks.resize(v.size());
  std::vector<std::unique_ptr<fosb_level>> lv(n_levels);
  for (int32_t i = 0; i < n_levels; ++i) {
    const int64_t n = meshes[i]->h.ne;
    c.ws_Z[i].reserve((size_t)n * n * sizeof(c128));
    if (mixed) c.ws_Zlow[i].reserve((size_t)n * n * sizeof(c64));
    {
      ProfScope prof(c, FOSB_K_ASSEMBLE, 0.0, (mixed ? 24.0 : 16.0) * (double)n * (double)n);
      assemble_efie(c, *meshes[i], k, o.n_gauss_singular, c.ws_Z[i].as<c128>(), n,
                    mixed ? c.ws_Zlow[i].as<c64>() : nullptr, mixed ? n : 0);
    }
    lv[i] = level_build(c, meshes[i], k, precision, c.ws_Z[i].p, n, mixed ? c.ws_Zlow[i].p : nullptr,
                        mixed ? n : 0, dirs, pols, n_dirs, field, o, FOSB_FORM_EFIE, 1.0, 1.0, -1, false, mixed);
  }
  std::vector<void*> bp(v.size());
  std::vector<int64_t> ldb(v.size());
  for (size_t p = 0; p < v.size(); ++p) {
    const fosb_level& a = *lv[v[p][0] - L0];
    const fosb_level& b = *lv[v[p][1] - L0];
    ldb[p] = n_dirs * b.n;
    c.ws_blocks[p].reserve((size_t)a.n * ldb[p] * sizeof(c128));
    bp[p] = c.ws_blocks[p].p;
    c128* C = c.ws_blocks[p].as<c128>();
    {
      ProfScope prof(c, FOSB_K_RHS, 0.0, 16.0 * (double)n_dirs * (double)a.n * (double)b.n);
      if (n_dirs == 1)
        rhs_correlation_kernel(c.stream, a, b, cov, 0, C, ldb[p]);
      else
        rhs_correlation_multi(c.stream, a, b, cov, 0, n_dirs, C, ldb[p], b.n);
    }
    two_sided(c, a, b, C, ldb[p], st, n_dirs);
  }
  std::vector<const fosb_level*> lp(n_levels);
  for (int32_t i = 0; i < n_levels; ++i) {
    lp[i] = lv[i].get();
    merge_level_certificate(st, *lv[i]);
  }
  far_field_impl(c, lp.data(), L0, L, bp.data(), ldb.data(), xhat, n_a, 0, n_dirs, var, nullptr);
}

}  // namespace fosb

extern "C" {

const char* fosb_last_error(void) { return g_last_error.c_str(); }

fosb_status fosb_opts_default(fosb_opts* opts) {
  API_BEGIN
  REQUIRE(opts, "opts is NULL");
  *opts = opts_or_default(nullptr);
  API_END
}

fosb_status fosb_context_create(int32_t device, void* hip_stream, fosb_context** out) {
  API_BEGIN
  REQUIRE(out, "out is NULL");
  *out = nullptr;
  int count = 0;
  FOSB_HIP(hipGetDeviceCount(&count));
  REQUIRE(device >= 0 && device < count, "device %d out of range (%d devices)", device, count);
  FOSB_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FOSB_HIP(hipGetDeviceProperties(&prop, device));
  std::unique_ptr<fosb_context> c(new fosb_context());
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->n_cu = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  noalloc_scratch_init(device);  // once per device: the allocation-free entry point's array
  *out = c.release();
  API_END
}

fosb_status fosb_context_destroy(fosb_context* ctx) {
  API_BEGIN
  if (!ctx) return FOSB_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    for (Level* l : ctx->live_levels) l->ctx = nullptr;
    for (Mesh* m : ctx->live_meshes) m->ctx = nullptr;
  }
  delete ctx;
  API_END
}

fosb_status fosb_context_synchronize(fosb_context* ctx) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  bind(*ctx);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  API_END
}

fosb_status fosb_context_memory(fosb_context* ctx, int64_t* n_device_allocs, int64_t* bytes_cached,
                                int64_t* bytes_in_use) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  int64_t a = 0, c = 0, l = 0;
  pool_totals(*ctx, a, c, l);
  if (n_device_allocs) *n_device_allocs = a;
  if (bytes_cached) *bytes_cached = c;
  if (bytes_in_use) *bytes_in_use = l;
  API_END
}

fosb_status fosb_context_trim(fosb_context* ctx) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  bind(*ctx);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->aux) FOSB_HIP(hipStreamSynchronize(ctx->aux->stream));
  if (ctx->la) FOSB_HIP(hipStreamSynchronize(ctx->la->stream));
  for (auto& w : ctx->workers) FOSB_HIP(hipStreamSynchronize(w->stream));
  pool_trim(*ctx);
  API_END
}

fosb_status fosb_mesh_validate(const double* V, int64_t nv, const int32_t* F, int64_t nt, int64_t* n_edges) {
  API_BEGIN
  MeshHost h;
  mesh_build_host(V, nv, F, nt, h);
  if (n_edges) *n_edges = h.ne;
  API_END
}

fosb_status fosb_mesh_create(fosb_context* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nt,
                             fosb_mesh** out) {
  API_BEGIN
  REQUIRE(ctx && out, "ctx/out is NULL");
  *out = nullptr;
  std::unique_ptr<fosb_mesh> m(new fosb_mesh());
  mesh_build_host(V, nv, F, nt, m->h);
  mesh_touching_pairs(m->h);
  bind(*ctx);
  m->ctx = ctx;
  mesh_upload(*m);
  {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    ctx->live_meshes.insert(m.get());
  }
  *out = m.release();
  API_END
}

fosb_status fosb_mesh_info(const fosb_mesh* mesh, int64_t* n_triangles, int64_t* n_edges, int64_t* n_touching) {
  API_BEGIN
  REQUIRE(mesh, "mesh is NULL");
  if (n_triangles) *n_triangles = mesh->h.nt;
  if (n_edges) *n_edges = mesh->h.ne;
  if (n_touching) *n_touching = (int64_t)mesh->h.tp_i.size();
  API_END
}

fosb_status fosb_mesh_destroy(fosb_mesh* mesh) {
  API_BEGIN
  if (!mesh) return FOSB_OK;
  if (mesh->ctx) {  // null once its context was destroyed
    (void)hipSetDevice(mesh->ctx->device);
    std::lock_guard<std::mutex> lock(mesh->ctx->reg_mu);
    mesh->ctx->live_meshes.erase(mesh);
  }
  delete mesh;
  API_END
}

fosb_status fosb_assemble(fosb_context* ctx, const fosb_mesh* mesh, double k, const fosb_opts* opts, void* Z,
                          int64_t ldz) {
  API_BEGIN
  REQUIRE(ctx && mesh, "ctx/mesh is NULL");
  REQUIRE(mesh->ctx == ctx, "mesh belongs to another context");
  REQUIRE(std::isfinite(k) && k > 0, "wavenumber must be positive and finite");
  REQUIRE(Z, "Z is NULL");
  if (ldz < mesh->h.ne) fail(FOSB_E_WORKSPACE, "ldz (%lld) < N (%lld)", (long long)ldz, (long long)mesh->h.ne);
  fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  {
    const double nt = (double)mesh->h.nt;
    ProfScope prof(*ctx, FOSB_K_ASSEMBLE, 0.0, 16.0 * (double)mesh->h.ne * (double)mesh->h.ne + 0.0 * nt);
    assemble_efie(*ctx, *mesh, k, o.n_gauss_singular, static_cast<c128*>(Z), ldz);
  }
  API_END
}

fosb_status fosb_level_create(fosb_context* ctx, const fosb_mesh* mesh, double k, int32_t precision, void* Z,
                              int64_t ldz, void* Zlow, int64_t ldzlow, const double* dirs, const double* pols,
                              int64_t n_dirs, int32_t field, const fosb_opts* opts, fosb_level** out) {
  API_BEGIN
  REQUIRE(ctx && mesh && out, "ctx/mesh/out is NULL");
  *out = nullptr;
  REQUIRE(mesh->ctx == ctx, "mesh belongs to another context");
  check_level_args(mesh, k, precision, Z, ldz, Zlow, ldzlow, dirs, pols, n_dirs, field);
  fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  check_device_memory(*ctx,
                      level_bytes(mesh->h.ne, mesh->h.nt, precision, n_dirs) +
                          solve_work_bytes(mesh->h.ne, precision, std::max<int64_t>(n_dirs, 256)),
                      "the level");
  auto L = level_build(*ctx, mesh, k, precision, Z, ldz, Zlow, ldzlow, dirs, pols, n_dirs, field, o);
  {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    ctx->live_levels.insert(L.get());
  }
  *out = L.release();
  API_END
}

static void check_material(double k0, double eps_r, double mu_r, const fosb_mesh* mesh) {
  REQUIRE(std::isfinite(k0) && k0 > 0, "wavenumber must be positive and finite");
  REQUIRE(std::isfinite(eps_r) && eps_r > 0 && std::isfinite(mu_r) && mu_r > 0, "eps_r and mu_r must be > 0");
  const MeshHost& h = mesh->h;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < h.nv; ++v)
    for (int q = 0; q < 3; ++q) {
      lo[q] = std::min(lo[q], h.V[3 * v + q]);
      hi[q] = std::max(hi[q], h.V[3 * v + q]);
    }
  const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                (hi[2] - lo[2]) * (hi[2] - lo[2]));
  const double k1 = k0 * std::sqrt(eps_r * mu_r);
  REQUIRE(std::max(k0, k1) * diag <= 1e5, "max(k0, k1) * (mesh bounding-box diagonal) = %g exceeds 1e5",
          std::max(k0, k1) * diag);
}

fosb_status fosb_assemble_pmchwt(fosb_context* ctx, const fosb_mesh* mesh, double k0, double eps_r, double mu_r,
                                 const fosb_opts* opts, void* Z, int64_t ldz) {
  API_BEGIN
  REQUIRE(ctx && mesh, "ctx/mesh is NULL");
  REQUIRE(mesh->ctx == ctx, "mesh belongs to another context");
  check_material(k0, eps_r, mu_r, mesh);
  REQUIRE(Z, "Z is NULL");
  const int64_t n = 2 * mesh->h.ne;
  if (ldz < n) fail(FOSB_E_WORKSPACE, "ldz (%lld) < 2N (%lld)", (long long)ldz, (long long)n);
  fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  {
    ProfScope prof(*ctx, FOSB_K_ASSEMBLE, 0.0, 2.0 * 16.0 * (double)n * (double)n);
    assemble_pmchwt(*ctx, *mesh, k0, eps_r, mu_r, o.n_gauss_singular, static_cast<c128*>(Z), ldz);
  }
  API_END
}

fosb_status fosb_level_create_pmchwt(fosb_context* ctx, const fosb_mesh* mesh, double k0, double eps_r,
                                     double mu_r, int32_t precision, void* Z, int64_t ldz, void* Zlow,
                                     int64_t ldzlow, const double* dirs, const double* pols, int64_t n_dirs,
                                     int32_t field, const fosb_opts* opts, fosb_level** out) {
  API_BEGIN
  REQUIRE(ctx && mesh && out, "ctx/mesh/out is NULL");
  *out = nullptr;
  REQUIRE(mesh->ctx == ctx, "mesh belongs to another context");
  check_material(k0, eps_r, mu_r, mesh);
  check_physics(k0, precision, dirs, pols, n_dirs, FOSB_FIELD_NORMAL);
  REQUIRE(Z, "Z is NULL (a dielectric level keeps its FP64 matrix)");
  const int64_t n = 2 * mesh->h.ne;
  if (ldz < n) fail(FOSB_E_WORKSPACE, "ldz < 2N");
  if (precision == FOSB_PREC_MIXED) {
    REQUIRE(Zlow, "MIXED precision needs the complex64 buffer Zlow");
    if (ldzlow < n) fail(FOSB_E_WORKSPACE, "ldzlow < 2N");
  } else {
    REQUIRE(!Zlow, "FP64 precision takes no Zlow buffer");
  }
  const bool streamed = field >= 0 && (field & FOSB_SD_STREAMED);
  if (field >= 0) field &= ~FOSB_SD_STREAMED;
  REQUIRE(field == -1 || field == FOSB_FIELD_RADIAL || field == FOSB_FIELD_NORMAL, "unknown field %d", field);
  if (field >= 0 && mu_r != 1.0)
    fail(FOSB_E_UNSUPPORTED, "the dielectric shape-derivative weights are built for mu_r = 1");
  fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  const int64_t sd_bytes = field >= 0 ? (streamed ? 0 : n_dirs * n * 6LL * mesh->h.nt * 16) + 24LL * mesh->h.nt : 0;
  check_device_memory(*ctx, level_bytes(n, 0, precision, n_dirs) + solve_work_bytes(n, precision, n_dirs) + sd_bytes,
                      "the level");
  auto L = level_build(*ctx, mesh, k0, precision, Z, ldz, Zlow, ldzlow, dirs, pols, n_dirs, FOSB_FIELD_NORMAL, o,
                       FOSB_FORM_PMCHWT, eps_r, mu_r, field, streamed);
  {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    ctx->live_levels.insert(L.get());
  }
  *out = L.release();
  API_END
}

fosb_status fosb_level_sd_weights(fosb_context* ctx, const fosb_level* level, int64_t dir, void* W, int64_t ldw) {
  API_BEGIN
  REQUIRE(ctx && level && W, "NULL argument");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  REQUIRE(level->form == FOSB_FORM_PMCHWT && level->sd_field >= 0, "the level has no shape-derivative weights");
  REQUIRE(dir >= 0 && dir < level->n_dirs, "dir out of range");
  const int64_t Q = 6LL * level->mesh->h.nt;
  if (ldw < Q) fail(FOSB_E_WORKSPACE, "ldw < 6 nt");
  bind(*ctx);
  if (level->sd_streamed)
    sd_weights(*ctx, *level->mesh, level->k, level->eps_r, level->sd_field, level->u.as<c128>(), level->n_dirs, dir,
               level->opts.n_gauss_singular, static_cast<c128*>(W), ldw);
  else
    copy_c128(ctx->stream, level->Wsd.as<c128>() + dir * level->n * Q, Q, static_cast<c128*>(W), ldw, level->n, Q);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  API_END
}

fosb_status fosb_level_formulation(const fosb_level* level, int32_t* form, double* eps_r, double* mu_r) {
  API_BEGIN
  REQUIRE(level, "level is NULL");
  if (form) *form = level->form;
  if (eps_r) *eps_r = level->eps_r;
  if (mu_r) *mu_r = level->mu_r;
  API_END
}

fosb_status fosb_level_factorization(const fosb_level* level, int32_t* kind) {
  API_BEGIN
  REQUIRE(level && kind, "level/kind is NULL");
  *kind = level->sym_lu ? FOSB_FACTOR_SYM : FOSB_FACTOR_LU;
  API_END
}

fosb_status fosb_level_info(const fosb_level* level, int64_t* n, int32_t* precision, int64_t* n_dirs) {
  API_BEGIN
  REQUIRE(level, "level is NULL");
  if (n) *n = level->n;
  if (precision) *precision = level->precision;
  if (n_dirs) *n_dirs = level->n_dirs;
  API_END
}

fosb_status fosb_level_workspace_size(const fosb_mesh* mesh, int32_t precision, int64_t n_dirs, int64_t nrhs,
                                      int64_t* level_b, int64_t* work_b) {
  API_BEGIN
  REQUIRE(mesh, "mesh is NULL");
  REQUIRE(precision == FOSB_PREC_FP64 || precision == FOSB_PREC_MIXED, "unknown precision %d", precision);
  REQUIRE(n_dirs >= 1 && n_dirs <= 4096, "need 1..4096 incidence directions");
  if (nrhs <= 0) nrhs = n_dirs;
  if (level_b) *level_b = level_bytes(mesh->h.ne, mesh->h.nt, precision, n_dirs);
  if (work_b) *work_b = std::max<int64_t>((int64_t)2 << 30, solve_work_bytes(mesh->h.ne, precision, nrhs));
  API_END
}

fosb_status fosb_level_certificate(const fosb_level* level, double* kappa1, double* growth) {
  API_BEGIN
  REQUIRE(level, "level is NULL");
  if (kappa1) *kappa1 = level->kappa1;
  if (growth) *growth = level->growth;
  API_END
}

fosb_status fosb_level_solve(fosb_context* ctx, const fosb_level* level, void* B, int64_t ldb, int64_t nrhs,
                             fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && level && B, "ctx/level/B is NULL");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  REQUIRE(nrhs >= 1, "nrhs must be >= 1");
  if (ldb < nrhs) fail(FOSB_E_WORKSPACE, "ldb < nrhs");
  bind(*ctx);
  level_solve_inplace(*ctx, *level, static_cast<c128*>(B), ldb, nrhs, stats);
  API_END
}

fosb_status fosb_level_solve_adjoint(fosb_context* ctx, const fosb_level* level, void* B, int64_t ldb, int64_t nrhs,
                                     fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && level && B, "ctx/level/B is NULL");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  REQUIRE(nrhs >= 1, "nrhs must be >= 1");
  if (ldb < nrhs) fail(FOSB_E_WORKSPACE, "ldb < nrhs");
  bind(*ctx);
  level_solve_inplace(*ctx, *level, static_cast<c128*>(B), ldb, nrhs, stats, true);
  API_END
}

fosb_status fosb_level_first_moment(fosb_context* ctx, const fosb_level* level, int64_t dir, void* u) {
  API_BEGIN
  REQUIRE(ctx && level && u, "ctx/level/u is NULL");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  REQUIRE(dir >= 0 && dir < level->n_dirs, "dir out of range");
  bind(*ctx);
  copy_c128(ctx->stream, level->u.as<c128>() + dir, level->n_dirs, static_cast<c128*>(u), 1, level->n, 1);
  API_END
}

fosb_status fosb_level_destroy(fosb_level* level) {
  API_BEGIN
  if (!level) return FOSB_OK;
  if (level->ctx) {  // null once its context was destroyed
    (void)hipSetDevice(level->ctx->device);
    (void)hipStreamSynchronize(level->ctx->stream);
    std::lock_guard<std::mutex> lock(level->ctx->reg_mu);
    level->ctx->live_levels.erase(level);
  }
  delete level;
  API_END
}

fosb_status fosb_rhs_correlation(fosb_context* ctx, const fosb_level* l1, const fosb_level* l2, const fosb_cov* cov,
                                 int64_t dir, void* C, int64_t ldc) {
  API_BEGIN
  REQUIRE(ctx && C, "ctx/C is NULL");
  check_pair(ctx, l1, l2);
  check_cov_for(l1, cov);
  REQUIRE(dir >= 0 && dir < l1->n_dirs, "dir out of range");
  if (ldc < l2->n) fail(FOSB_E_WORKSPACE, "ldc < N2");
  bind(*ctx);
  pair_rhs(*ctx, *l1, *l2, cov, dir, static_cast<c128*>(C), ldc);
  API_END
}

fosb_status fosb_two_sided_solve(fosb_context* ctx, const fosb_level* l1, const fosb_level* l2, void* C, int64_t ldc,
                                 fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && C, "ctx/C is NULL");
  check_pair(ctx, l1, l2);
  if (ldc < l2->n) fail(FOSB_E_WORKSPACE, "ldc < N2");
  bind(*ctx);
  two_sided(*ctx, *l1, *l2, static_cast<c128*>(C), ldc, stats);
  API_END
}

fosb_status fosb_ct_pairs(int32_t L0, int32_t L, int32_t* l1, int32_t* l2, int32_t* sign, int32_t* mult,
                          int32_t* n_pairs) {
  API_BEGIN
  REQUIRE(L0 >= 0 && L >= L0 && L - L0 < 64, "need 0 <= L0 <= L < L0 + 64");
  REQUIRE(n_pairs, "n_pairs is NULL");
  auto v = ct_pairs_vec(L0, L);
  *n_pairs = (int32_t)v.size();
  for (size_t p = 0; p < v.size(); ++p) {
    if (l1) l1[p] = v[p][0];
    if (l2) l2[p] = v[p][1];
    if (sign) sign[p] = v[p][2];
    if (mult) mult[p] = v[p][3];
  }
  API_END
}

fosb_status fosb_correlation(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels, int32_t L0,
                             int32_t L, const fosb_cov* cov, int64_t dir, void* const* blocks, const int64_t* ldb,
                             fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && levels && blocks && ldb, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  check_cov_for(levels[0], cov);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  auto v = ct_pairs_vec(L0, L);
  for (size_t p = 0; p < v.size(); ++p) {
    REQUIRE(blocks[p], "block %zu is NULL", p);
    if (ldb[p] < levels[v[p][1] - L0]->n) fail(FOSB_E_WORKSPACE, "ldb[%zu] < N_l2", p);
  }
  bind(*ctx);
  for (size_t p = 0; p < v.size(); ++p) {
    const fosb_level* a = levels[v[p][0] - L0];
    const fosb_level* b = levels[v[p][1] - L0];
    c128* C = static_cast<c128*>(blocks[p]);
    {
      ProfScope prof(*ctx, FOSB_K_RHS, 0.0, 16.0 * (double)a->n * (double)b->n);
      pair_rhs(*ctx, *a, *b, cov, dir, C, ldb[p]);
    }
    two_sided(*ctx, *a, *b, C, ldb[p], stats);
  }
  API_END
}

fosb_status fosb_far_field_matrix(fosb_context* ctx, const fosb_level* level, const double* xhat, int64_t n_a,
                                  void* FF) {
  API_BEGIN
  REQUIRE(ctx && level && xhat && FF, "NULL argument");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  bind(*ctx);
  std::vector<double> x(xhat, xhat + 3 * n_a);
  DevBuf dx;
  upload(dx, x, ctx->stream);
  level_far_field(ctx->stream, *level, dx.as<double>(), n_a, static_cast<c128*>(FF));
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  API_END
}

fosb_status fosb_far_field_moments(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels, int32_t L0,
                                   int32_t L, void* const* blocks, const int64_t* ldb, const double* xhat,
                                   int64_t n_a, int64_t dir, double* var, void* cor, void* mean_F) {
  API_BEGIN
  REQUIRE(ctx && levels && blocks && ldb && xhat && var, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  check_far_field_args(xhat, n_a, L0, L, levels, blocks, ldb);
  bind(*ctx);
  if (cor) REQUIRE(n_a <= 4096, "the angular correlation takes at most 4096 angles");
  far_field_impl(*ctx, levels, L0, L, blocks, ldb, xhat, n_a, dir, 1, var, mean_F, cor);
  API_END
}

fosb_status fosb_far_field_variance_adjoint(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                            int32_t L0, int32_t L, const fosb_cov* cov, const double* xhat,
                                            int64_t n_a, int64_t dir, double* var, void* mean_F, fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && levels && xhat && var, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  require_efie(levels, n_levels);
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  check_cov(cov);
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  for (int64_t i = 0; i < n_a; ++i) {
    double nn = xhat[3 * i] * xhat[3 * i] + xhat[3 * i + 1] * xhat[3 * i + 1] + xhat[3 * i + 2] * xhat[3 * i + 2];
    REQUIRE(std::fabs(nn - 1.0) < 1e-9, "xhat[%lld] is not a unit vector", (long long)i);
  }
  bind(*ctx);
  hipStream_t s = ctx->stream;
  std::vector<double> x(xhat, xhat + 3 * n_a);
  DevBuf dx;
  upload(dx, x, s);
  const int64_t R = 3 * n_a;
  std::vector<DevBuf> Hn(n_levels), Hc(n_levels);
  for (int32_t i = 0; i < n_levels; ++i) {
    const fosb_level& l = *levels[i];
    const int64_t Q = 6LL * l.mesh->h.nt;
    adjoint_node_rows(*ctx, l, dx.as<double>(), n_a, dir, Hn[i], stats);   // P_l^T
    Hc[i].alloc((size_t)Q * R * sizeof(c128));
    copy_c128(s, Hn[i].as<c128>(), R, Hc[i].as<c128>(), R, Q, R);
    conj_inplace_c128(s, Hc[i].as<c128>(), Q * R);                          // conj(P_l)^T
  }
  zero_f64(s, var, R);
  // V_r = sum sign mult Re sum_q1 P_l1[r][q1] T[q1][r],  T = K_l1l2 conj(P_l2)^T, in row chunks of K
  auto v = ct_pairs_vec(L0, L);
  const int64_t budget = (int64_t)1 << 26;
  DevBuf Kc, T, part;
  for (auto& q : v) {
    const fosb_level& l1 = *levels[q[0] - L0];
    const fosb_level& l2 = *levels[q[1] - L0];
    const int64_t Q1 = 6LL * l1.mesh->h.nt, Q2 = 6LL * l2.mesh->h.nt;
    const int64_t ch = std::min<int64_t>(Q1, std::max<int64_t>(256, budget / Q2) / 256 * 256);
    Kc.reserve((size_t)ch * Q2 * sizeof(c128));
    T.reserve((size_t)ch * R * sizeof(c128));
    part.reserve((size_t)((ch + 255) / 256) * R * sizeof(double));
    for (int64_t a0 = 0; a0 < Q1; a0 += ch) {
      const int64_t na = std::min(ch, Q1 - a0);
      cov_matrix(s, l1, l2, *cov, a0, na, Kc.as<c128>());
      gemm<double>(*ctx, na, R, Q2, 1.0, Kc.as<c128>(), Q2, Hc[q[1] - L0].as<c128>(), R, 0.0, T.as<c128>(), R);
      coldot_re_accumulate(s, Hn[q[0] - L0].as<c128>() + a0 * R, T.as<c128>(), na, R, (double)(q[2] * q[3]),
                           part.as<double>(), var);
    }
  }
  if (mean_F) {
    const fosb_level& lf = *levels[n_levels - 1];
    DevBuf FF((size_t)R * lf.n * sizeof(c128)), u((size_t)lf.n * sizeof(c128));
    far_field_matrix_kernel(s, *lf.mesh, lf.k, dx.as<double>(), n_a, FF.as<c128>());
    copy_c128(s, lf.u.as<c128>() + dir, lf.n_dirs, u.as<c128>(), 1, lf.n, 1);
    matvec_rows(s, FF.as<c128>(), R, lf.n, u.as<c128>(), static_cast<c128*>(mean_F));
  }
  FOSB_HIP(hipStreamSynchronize(s));
  API_END
}

fosb_status fosb_lowrank_create(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                const fosb_cov* cov, int32_t max_rank, double tol, fosb_lowrank** out) {
  API_BEGIN
  REQUIRE(ctx && levels && out, "NULL argument");
  *out = nullptr;
  REQUIRE(n_levels >= 1 && n_levels <= 64, "n_levels must be 1..64");
  for (int32_t i = 0; i < n_levels; ++i)
    REQUIRE(levels[i] && (levels[i]->form == FOSB_FORM_EFIE || levels[i]->sd_field >= 0),
            "dielectric levels need shape-derivative weights (field >= 0) for the low-rank route");
  check_cov(cov);
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(std::isfinite(tol) && tol >= 0.0 && tol < 1.0, "tol must be in [0, 1)");
  std::unique_ptr<fosb_lowrank> lr(new fosb_lowrank());
  lr->ctx = ctx;
  lr->cov = *cov;
  int64_t nc = 0;
  for (int32_t i = 0; i < n_levels; ++i) {
    lr->levels.push_back(levels[i]);
    lr->off.push_back(nc);
    nc += 6LL * levels[i]->mesh->h.nt;
  }
  lr->nc = nc;
  REQUIRE(max_rank >= 1 && max_rank <= 8192 && max_rank <= nc, "max_rank must be 1..min(8192, nodes)");
  bind(*ctx);
  check_device_memory(*ctx, (int64_t)max_rank * nc * 8 + 7 * nc * 8, "the low-rank factor");
  hipStream_t s = ctx->stream;
  DevBuf X((size_t)3 * nc * sizeof(double)), Nn((size_t)3 * nc * sizeof(double)), d((size_t)nc * sizeof(double));
  DevBuf pv(2 * sizeof(double));
  lr->L.alloc((size_t)max_rank * nc * sizeof(double));
  for (int32_t i = 0; i < n_levels; ++i)
    lr_candidates(s, *levels[i], lr->off[i], nc, X.as<double>(), Nn.as<double>());
  lr_diag(s, Nn.as<double>(), nc, *cov, d.as<double>());
  // Greedy pivoted Cholesky: the host reads each pivot (its remaining diagonal
  // entry decides termination) and launches the column update.
  constexpr double kTie = 1e-9;
  double dmax0 = -1.0, last = 0.0;
  for (int32_t j = 0; j < max_rank; ++j) {
    double h[2];
    lr_pivot(s, d.as<double>(), nc, kTie, pv.as<double>());
    FOSB_HIP(hipMemcpyAsync(h, pv.p, sizeof(h), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    if (j == 0) dmax0 = h[0];
    last = h[0];
    if (!(h[0] > tol * dmax0) || !(h[0] > 0.0)) break;
    const int64_t p = (int64_t)h[1];
    lr_column(s, X.as<double>(), Nn.as<double>(), nc, *cov, lr->L.as<double>(), j, p, h[0], d.as<double>());
    lr->pivots.push_back(p);
    lr->rank = j + 1;
  }
  if (lr->rank == max_rank) {  // the largest remaining diagonal entry after the last column
    double h[2];
    lr_pivot(s, d.as<double>(), nc, kTie, pv.as<double>());
    FOSB_HIP(hipMemcpyAsync(h, pv.p, sizeof(h), hipMemcpyDeviceToHost, s));
    FOSB_HIP(hipStreamSynchronize(s));
    last = h[0];
  }
  lr->residual = dmax0 > 0 ? last / dmax0 : 0.0;
  FOSB_HIP(hipStreamSynchronize(s));
  *out = lr.release();
  API_END
}

fosb_status fosb_lowrank_info(const fosb_lowrank* lr, int32_t* rank, double* residual, int64_t* pivots) {
  API_BEGIN
  REQUIRE(lr, "lowrank is NULL");
  if (rank) *rank = lr->rank;
  if (residual) *residual = lr->residual;
  if (pivots) std::copy(lr->pivots.begin(), lr->pivots.end(), pivots);
  API_END
}

fosb_status fosb_lowrank_destroy(fosb_lowrank* lr) {
  API_BEGIN
  if (!lr) return FOSB_OK;
  if (lr->ctx) {
    (void)hipSetDevice(lr->ctx->device);
    (void)hipStreamSynchronize(lr->ctx->stream);
  }
  delete lr;
  API_END
}

// Y (N x rank, row stride ldy) = Z^{-1} Wgt_dir L_l for ladder level i.
// M (N x r) = Wsd_dir L_l for a dielectric level: one product with the stored
// weights, or a sum over source-triangle bands of weights recomputed into a
// band buffer (at most 2 GiB) when the level stores none.
static void sd_times_factor(Context& c, const Level& l, int64_t dir, const double* Lr, int r, c128* M) {
  hipStream_t s = c.stream;
  const int64_t Q = 6LL * l.mesh->h.nt, n = l.n;
  DevBuf Lc((size_t)Q * r * sizeof(c128));
  real_to_c128(s, Lr, Q * r, Lc.as<c128>());
  if (!l.sd_streamed) {
    gemm<double>(c, n, r, Q, 1.0, l.Wsd.as<c128>() + dir * n * Q, Q, Lc.as<c128>(), r, 0.0, M, r);
    return;
  }
  const int nt = (int)l.mesh->h.nt;
  int w = (int)std::max<int64_t>(1, std::min<int64_t>(nt, ((int64_t)2 << 30) / (n * 6 * 16)));
  SdPlan P;
  sd_plan(c, *l.mesh, l.k, l.eps_r, l.u.as<c128>(), l.n_dirs, dir, P);
  DevBuf Wb((size_t)n * 6 * w * sizeof(c128));
  {
    ProfScope prof(c, FOSB_K_RHS, 0.0, 16.0 * (double)n * (double)Q);
    for (int j0 = 0; j0 < nt; j0 += w) {
      const int j1 = std::min(nt, j0 + w);
      const int64_t nb = 6LL * (j1 - j0);
      sd_band(c, *l.mesh, P, l.k, l.eps_r, l.sd_field, l.opts.n_gauss_singular, j0, j1, Wb.as<c128>(), nb);
      gemm<double>(c, n, r, nb, 1.0, Wb.as<c128>(), nb, Lc.as<c128>() + 6LL * j0 * r, r, j0 == 0 ? 0.0 : 1.0, M, r);
    }
  }
  FOSB_HIP(hipStreamSynchronize(s));
}

static void lowrank_factor_impl(Context& c, const fosb_lowrank& lr, int32_t i, int64_t dir, c128* Y, int64_t ldy,
                                fosb_stats* st) {
  const Level& l = *lr.levels[i];
  const int r = lr.rank;
  DevBuf Lr((size_t)6 * l.mesh->h.nt * r * sizeof(double));
  if (l.form == FOSB_FORM_PMCHWT) {
    DevBuf M((size_t)l.n * r * sizeof(c128));
    lr_rows(c.stream, l, lr.L.as<double>(), lr.nc, lr.off[i], r, Lr.as<double>());
    sd_times_factor(c, l, dir, Lr.as<double>(), r, M.as<c128>());
    level_solve_inplace(c, l, M.as<c128>(), r, r, st);
    copy_c128(c.stream, M.as<c128>(), r, Y, ldy, l.n, r);
    return;
  }
  if (ldy == r) {
    lr_rhs(c.stream, l, dir, lr.L.as<double>(), lr.nc, lr.off[i], r, Lr.as<double>(), Y);
    level_solve_inplace(c, l, Y, ldy, r, st);
  } else {
    DevBuf M((size_t)l.n * r * sizeof(c128));
    lr_rhs(c.stream, l, dir, lr.L.as<double>(), lr.nc, lr.off[i], r, Lr.as<double>(), M.as<c128>());
    level_solve_inplace(c, l, M.as<c128>(), r, r, st);
    copy_c128(c.stream, M.as<c128>(), r, Y, ldy, l.n, r);
  }
}

static void check_lowrank(const fosb_context* ctx, const fosb_lowrank* lr) {
  REQUIRE(lr, "lowrank is NULL");
  REQUIRE(lr->ctx == ctx, "lowrank belongs to another context");
  REQUIRE(lr->rank >= 1, "the low-rank factor is empty (rank 0)");
  for (const Level* l : lr->levels) REQUIRE(l->ctx == ctx, "a level of the low-rank factor was detached");
}

fosb_status fosb_lowrank_factor(fosb_context* ctx, const fosb_lowrank* lr, int32_t level_index, int64_t dir, void* Y,
                                int64_t ldy, fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && Y, "NULL argument");
  check_lowrank(ctx, lr);
  REQUIRE(level_index >= 0 && level_index < (int32_t)lr->levels.size(), "level_index out of range");
  REQUIRE(dir >= 0 && dir < lr->levels[0]->n_dirs, "dir out of range");
  if (ldy < lr->rank) fail(FOSB_E_WORKSPACE, "ldy < rank");
  bind(*ctx);
  lowrank_factor_impl(*ctx, *lr, level_index, dir, static_cast<c128*>(Y), ldy, stats);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  API_END
}

fosb_status fosb_far_field_moments_lowrank(fosb_context* ctx, const fosb_lowrank* lr, int32_t L0, int32_t L,
                                           const double* xhat, int64_t n_a, int64_t dir, double* var,
                                           fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && xhat && var, "NULL argument");
  check_lowrank(ctx, lr);
  REQUIRE(L0 >= 0 && L >= L0 && L - L0 + 1 == (int32_t)lr->levels.size(),
          "L - L0 + 1 must equal the low-rank factor's number of levels");
  REQUIRE(dir >= 0 && dir < lr->levels[0]->n_dirs, "dir out of range");
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  for (int64_t i = 0; i < n_a; ++i) {
    double nn = xhat[3 * i] * xhat[3 * i] + xhat[3 * i + 1] * xhat[3 * i + 1] + xhat[3 * i + 2] * xhat[3 * i + 2];
    REQUIRE(std::fabs(nn - 1.0) < 1e-9, "xhat[%lld] is not a unit vector", (long long)i);
  }
  bind(*ctx);
  hipStream_t s = ctx->stream;
  std::vector<double> x(xhat, xhat + 3 * n_a);
  DevBuf dx;
  upload(dx, x, s);
  const int64_t R = 3 * n_a;
  const int r = lr->rank;
  const int n_levels = (int)lr->levels.size();
  // per level: G_l = FF_l Z_l^{-1} Wgt_l L_l  (R x rank)
  std::vector<DevBuf> G(n_levels);
  for (int i = 0; i < n_levels; ++i) {
    const Level& l = *lr->levels[i];
    DevBuf Y((size_t)l.n * r * sizeof(c128)), FF((size_t)R * l.n * sizeof(c128));
    lowrank_factor_impl(*ctx, *lr, i, dir, Y.as<c128>(), r, stats);
    level_far_field(s, l, dx.as<double>(), n_a, FF.as<c128>());
    G[i].alloc((size_t)R * r * sizeof(c128));
    gemm<double>(*ctx, R, r, l.n, 1.0, FF.as<c128>(), l.n, Y.as<c128>(), r, 0.0, G[i].as<c128>(), r);
  }
  // Sigma_l1l2 = Y_l1 Y_l2^H, so (FF_l1 Sigma FF_l2^H)_rr = sum_k G_l1[r][k] conj(G_l2[r][k])
  zero_f64(s, var, R);
  for (auto& q : ct_pairs_vec(L0, L))
    row_dot_re_accumulate(s, G[q[0] - L0].as<c128>(), r, G[q[1] - L0].as<c128>(), R, r, (double)(q[2] * q[3]), var);
  FOSB_HIP(hipStreamSynchronize(s));
  API_END
}

fosb_status fosb_far_field_moments_noalloc(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                           int32_t L0, int32_t L, void* const* blocks, const int64_t* ldb,
                                           const double* xhat, int64_t n_a, int64_t dir, double* var, void* mean_F) {
  API_BEGIN
  REQUIRE(ctx && levels && blocks && ldb && xhat && var, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  require_efie(levels, n_levels);
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  check_far_field_args(xhat, n_a, L0, L, levels, blocks, ldb);
  bind(*ctx);
  // scratch layout: [xhat 3 n_a][first moment N_L (mean field only)][work]
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t total = (int64_t)FOSB_NOALLOC_SCRATCH_BYTES;
  const int64_t nL = levels[n_levels - 1]->n;
  const int64_t xb = up(3 * n_a * (int64_t)sizeof(double));
  const int64_t ub = mean_F ? up(nL * (int64_t)sizeof(c128)) : 0;
  const int64_t work = total - xb - ub;
  auto v = ct_pairs_vec(L0, L);
  int64_t per_angle = mean_F ? 3 * nL * (int64_t)sizeof(c128) : 0;
  for (auto& q : v)
    per_angle = std::max(per_angle, 3 * (levels[q[0] - L0]->n + 2 * levels[q[1] - L0]->n) * (int64_t)sizeof(c128));
  if (work < per_angle)
    fail(FOSB_E_WORKSPACE, "one angle needs %lld bytes of work memory; the allocation-free array leaves %lld",
         (long long)per_angle, (long long)std::max<int64_t>(work, 0));
  struct NoAlloc {  // no device allocation and no allocating GEMM mode while this call runs
    Context& c;
    explicit NoAlloc(Context& cc) : c(cc) { thread_no_alloc() = true; c.no_alloc = 1; }
    ~NoAlloc() { thread_no_alloc() = false; c.no_alloc = 0; }
  } guard(*ctx);
  hipStream_t s = ctx->stream;
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(ctx->device));
  double* dx = reinterpret_cast<double*>(base);
  c128* du = reinterpret_cast<c128*>(base + xb);
  c128* W = reinterpret_cast<c128*>(base + xb + ub);
  FOSB_HIP(hipMemcpyAsync(dx, xhat, 3 * n_a * sizeof(double), hipMemcpyHostToDevice, s));
  const int64_t rows = 3 * n_a;
  zero_f64(s, var, rows);
  for (auto& q : v) {
    const fosb_level& l1 = *levels[q[0] - L0];
    const fosb_level& l2 = *levels[q[1] - L0];
    const int64_t n1 = l1.n, n2 = l2.n;
    const int64_t c = std::min<int64_t>(n_a, work / (3 * (n1 + 2 * n2) * (int64_t)sizeof(c128)));
    const double scale = (double)(q[2] * q[3]);
    for (int64_t i0 = 0; i0 < n_a; i0 += c) {
      const int64_t cn = std::min(c, n_a - i0);
      c128* F1 = W;                       // 3 cn x n1, row comp * cn + i
      c128* F2 = F1 + 3 * cn * n1;        // 3 cn x n2
      c128* P = F2 + 3 * cn * n2;         // 3 cn x n2
      far_field_matrix_kernel(s, *l1.mesh, l1.k, dx + 3 * i0, cn, F1);
      far_field_matrix_kernel(s, *l2.mesh, l2.k, dx + 3 * i0, cn, F2);
      gemm<double>(*ctx, 3 * cn, n2, n1, 1.0, F1, n1, static_cast<const c128*>(blocks[&q - v.data()]),
                   ldb[&q - v.data()], 0.0, P, n2);
      for (int cc = 0; cc < 3; ++cc)
        row_dot_re_accumulate(s, P + cc * cn * n2, n2, F2 + cc * cn * n2, cn, n2, scale, var + cc * n_a + i0);
    }
  }
  if (mean_F) {
    const fosb_level& lf = *levels[n_levels - 1];
    copy_c128(s, lf.u.as<c128>() + dir, lf.n_dirs, du, 1, nL, 1);
    const int64_t c = std::min<int64_t>(n_a, work / (3 * nL * (int64_t)sizeof(c128)));
    for (int64_t i0 = 0; i0 < n_a; i0 += c) {
      const int64_t cn = std::min(c, n_a - i0);
      far_field_matrix_kernel(s, *lf.mesh, lf.k, dx + 3 * i0, cn, W);
      for (int cc = 0; cc < 3; ++cc)
        matvec_rows(s, W + cc * cn * nL, cn, nL, du, static_cast<c128*>(mean_F) + cc * n_a + i0);
    }
  }
  FOSB_HIP(hipStreamSynchronize(s));
  API_END
}

static void check_field_points(const double* xp, int64_t n_p) {
  REQUIRE(xp, "points is NULL");
  REQUIRE(n_p >= 1 && n_p <= 65535, "n_p must be 1..65535");
  for (int64_t i = 0; i < 3 * n_p; ++i) REQUIRE(std::isfinite(xp[i]), "non-finite field point coordinate");
}

fosb_status fosb_near_field_matrix(fosb_context* ctx, const fosb_level* level, const double* points, int64_t n_p,
                                   void* NF) {
  API_BEGIN
  REQUIRE(ctx && level && NF, "NULL argument");
  REQUIRE(level->ctx == ctx, "level belongs to another context");
  require_efie(&level, 1);
  check_field_points(points, n_p);
  bind(*ctx);
  std::vector<double> x(points, points + 3 * n_p);
  DevBuf dx;
  upload(dx, x, ctx->stream);
  near_field_matrix_kernel(ctx->stream, *level->mesh, level->k, dx.as<double>(), n_p, static_cast<c128*>(NF));
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  API_END
}

fosb_status fosb_near_field_moments(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels, int32_t L0,
                                    int32_t L, void* const* blocks, const int64_t* ldb, const double* points,
                                    int64_t n_p, int64_t dir, double* var, void* mean_E) {
  API_BEGIN
  REQUIRE(ctx && levels && blocks && ldb && var, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  require_efie(levels, n_levels);
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  check_field_points(points, n_p);
  auto v = ct_pairs_vec(L0, L);
  for (size_t p = 0; p < v.size(); ++p) {
    REQUIRE(blocks[p], "block %zu is NULL", p);
    if (ldb[p] < levels[v[p][1] - L0]->n) fail(FOSB_E_WORKSPACE, "ldb[%zu] < N_l2", p);
  }
  bind(*ctx);
  far_field_impl(*ctx, levels, L0, L, blocks, ldb, points, n_p, dir, 1, var, mean_E, nullptr, true);
  API_END
}

fosb_status fosb_far_field_moments_backward(fosb_context* ctx, const fosb_level* const* levels, int32_t n_levels,
                                            int32_t L0, int32_t L, const fosb_cov* cov, const double* xhat,
                                            int64_t n_a, int64_t dir, const double* dvar, double* out,
                                            fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && levels && xhat && dvar && out, "NULL argument");
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  require_efie(levels, n_levels);
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  check_cov(cov);
  for (int32_t i = 0; i < n_levels; ++i) check_pair(ctx, levels[0], levels[i]);
  REQUIRE(dir >= 0 && dir < levels[0]->n_dirs, "dir out of range");
  for (int64_t i = 0; i < n_a; ++i) {
    double nn = xhat[3 * i] * xhat[3 * i] + xhat[3 * i + 1] * xhat[3 * i + 1] + xhat[3 * i + 2] * xhat[3 * i + 2];
    REQUIRE(std::fabs(nn - 1.0) < 1e-9, "xhat[%lld] is not a unit vector", (long long)i);
  }
  bind(*ctx);
  hipStream_t s = ctx->stream;
  std::vector<double> x(xhat, xhat + 3 * n_a);
  DevBuf dx;
  upload(dx, x, s);
  const int64_t R = 3 * n_a;
  // per level: Hn = (FF Z^{-1} Wgt)^T (Q x R) and Bg = diag(g) conj(FF Z^{-1} Wgt) (R x Q)
  std::vector<DevBuf> Hn(n_levels), Bg(n_levels);
  for (int32_t i = 0; i < n_levels; ++i) {
    const fosb_level& l = *levels[i];
    const int64_t Q = 6LL * l.mesh->h.nt;
    adjoint_node_rows(*ctx, l, dx.as<double>(), n_a, dir, Hn[i], stats);
    Bg[i].alloc((size_t)R * Q * sizeof(c128));
    conj_transpose_c128(s, Hn[i].as<c128>(), R, Bg[i].as<c128>(), Q, Q, R, dvar);
  }
  FOSB_HIP(hipStreamSynchronize(s));
  // G = Hn_l1 Bg_l2 in row chunks of at most 2^26 entries, reduced against the covariance
  auto v = ct_pairs_vec(L0, L);
  const int64_t budget = (int64_t)1 << 26;
  auto chunk_rows = [&](int64_t Q1, int64_t Q2) {
    int64_t ch = std::max<int64_t>(16, budget / Q2) / 16 * 16;
    return std::min<int64_t>(ch, Q1);
  };
  int64_t n_part = 0, g_max = 0;
  for (auto& q : v) {
    const int64_t Q1 = 6LL * levels[q[0] - L0]->mesh->h.nt, Q2 = 6LL * levels[q[1] - L0]->mesh->h.nt;
    const int64_t ch = chunk_rows(Q1, Q2);
    g_max = std::max(g_max, ch * Q2);
    for (int64_t a0 = 0; a0 < Q1; a0 += ch) n_part += ((Q2 + 255) / 256) * ((std::min(ch, Q1 - a0) + 15) / 16);
  }
  DevBuf Gb((size_t)g_max * sizeof(c128));
  DevBuf part((size_t)2 * n_part * sizeof(double));
  int64_t off = 0;
  for (auto& q : v) {
    const fosb_level& l1 = *levels[q[0] - L0];
    const fosb_level& l2 = *levels[q[1] - L0];
    const int64_t Q1 = 6LL * l1.mesh->h.nt, Q2 = 6LL * l2.mesh->h.nt;
    const int64_t ch = chunk_rows(Q1, Q2);
    for (int64_t a0 = 0; a0 < Q1; a0 += ch) {
      const int64_t na = std::min(ch, Q1 - a0);
      gemm<double>(*ctx, na, Q2, R, 1.0, Hn[q[0] - L0].as<c128>() + a0 * R, R, Bg[q[1] - L0].as<c128>(), Q2, 0.0,
                   Gb.as<c128>(), Q2);
      off += cov_grad_partials(s, Gb.as<c128>(), a0, na, l1, l2, *cov, (double)(q[2] * q[3]),
                               part.as<double>() + 2 * off);
    }
  }
  if (off != n_part) fail(FOSB_E_DEVICE, "backward: partial count mismatch");
  cov_grad_finish(s, part.as<double>(), n_part, cov->sigma, out);
  FOSB_HIP(hipStreamSynchronize(s));
  API_END
}

fosb_status fosb_second_moment(fosb_context* ctx, const fosb_mesh* const* meshes, int32_t n_levels, int32_t L0,
                               int32_t L, double k, int32_t precision, void* const* Z, const int64_t* ldz,
                               void* const* Zlow, const int64_t* ldzlow, const double* dirs, const double* pols,
                               int64_t n_dirs, int32_t field, const fosb_cov* cov, int64_t dir, const double* xhat,
                               int64_t n_a, void* const* blocks, const int64_t* ldb, double* var,
                               const fosb_opts* opts, fosb_level** levels_out, fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && meshes && Z && ldz && blocks && ldb && xhat && var, "NULL argument");
  for (int32_t i = 0; i < n_levels; ++i)
    REQUIRE(Z[i] || precision == FOSB_PREC_MIXED, "Z[%d] is NULL (only MIXED levels may re-assemble)", i);
  REQUIRE(L0 >= 0 && L >= L0 && n_levels == L - L0 + 1, "n_levels must be L - L0 + 1");
  REQUIRE(precision == FOSB_PREC_FP64 || (Zlow && ldzlow), "MIXED precision needs Zlow and ldzlow");
  for (int32_t i = 0; i < n_levels; ++i) {
    REQUIRE(meshes[i] && meshes[i]->ctx == ctx, "mesh %d is NULL or belongs to another context", i);
    if (i > 0) REQUIRE(meshes[i]->h.ne > meshes[i - 1]->h.ne, "levels must be ordered coarse to fine");
    check_level_args(meshes[i], k, precision, Z[i], ldz[i], precision == FOSB_PREC_MIXED ? Zlow[i] : nullptr,
                     precision == FOSB_PREC_MIXED ? ldzlow[i] : 0, dirs, pols, n_dirs, field);
  }
  check_cov(cov);
  REQUIRE(dir >= -1 && dir < n_dirs, "dir out of range");
  const int64_t nd = dir < 0 ? n_dirs : 1;   // incidences solved together
  const int64_t d0 = dir < 0 ? 0 : dir;
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  auto v = ct_pairs_vec(L0, L);
  for (size_t p = 0; p < v.size(); ++p) {
    REQUIRE(blocks[p], "block %zu is NULL", p);
    if (ldb[p] < nd * meshes[v[p][1] - L0]->h.ne) fail(FOSB_E_WORKSPACE, "ldb[%zu] < n_dirs N_l2", p);
  }
  const fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  {
    int64_t need = (int64_t)2 << 30;  // the assembly's two band buffers
    for (int32_t i = 0; i < n_levels; ++i) {
      need += level_bytes(meshes[i]->h.ne, meshes[i]->h.nt, precision, n_dirs);
      if (!Z[i]) need += (int64_t)8 << 30;  // bands of the re-assembled residual
    }
    int64_t pair_max = 0;
    for (auto& q : v) {
      const int64_t n1 = meshes[q[0] - L0]->h.ne, n2 = meshes[q[1] - L0]->h.ne;
      pair_max = std::max(pair_max, 16 * n1 * n2 * nd + solve_work_bytes(n1, precision, nd * n2) +
                                        solve_work_bytes(n2, precision, nd * n1));
    }
    check_device_memory(*ctx, need + 2 * pair_max, "the pass");
  }
  Context& aux = ctx->aux_context();
  const int top = n_levels - 1;
  std::vector<std::unique_ptr<fosb_level>> lv(n_levels);
  fosb_stats st_main{}, st_aux{};

  const bool mixed = precision == FOSB_PREC_MIXED;
  auto build = [&](Context& c, int i) {
    if (Z[i]) {  // a MIXED level without Z assembles its complex64 copy itself
      const double ne = (double)meshes[i]->h.ne;
      ProfScope prof(c, FOSB_K_ASSEMBLE, 0.0, (mixed ? 24.0 : 16.0) * ne * ne);
      assemble_efie(c, *meshes[i], k, o.n_gauss_singular, static_cast<c128*>(Z[i]), ldz[i],
                    mixed ? static_cast<c64*>(Zlow[i]) : nullptr, mixed ? ldzlow[i] : 0);
    }
    lv[i] = level_build(c, meshes[i], k, precision, Z[i], ldz[i], mixed ? Zlow[i] : nullptr, mixed ? ldzlow[i] : 0,
                        dirs, pols, n_dirs, field, o, FOSB_FORM_EFIE, 1.0, 1.0, -1, false, mixed && Z[i] != nullptr);
  };
  auto pair = [&](Context& c, size_t p, fosb_stats* st) {
    const fosb_level& a = *lv[v[p][0] - L0];
    const fosb_level& b = *lv[v[p][1] - L0];
    c128* C = static_cast<c128*>(blocks[p]);
    {
      ProfScope prof(c, FOSB_K_RHS, 0.0, 16.0 * (double)nd * (double)a.n * (double)b.n);
      if (nd == 1)
        rhs_correlation_kernel(c.stream, a, b, *cov, d0, C, ldb[p]);
      else
        rhs_correlation_multi(c.stream, a, b, *cov, d0, nd, C, ldb[p], b.n);
    }
    two_sided(c, a, b, C, ldb[p], st, nd);
  };

  // The finest level (the bulk of the work) is built on the context's stream
  // while a worker thread builds the coarser levels and solves the pairs that
  // do not involve the finest level on the auxiliary stream; the pairs with
  // the finest level follow on the main stream once the coarse levels exist.
  // The auxiliary pairs wait on the GPU for the finest level's factorisation
  // to reach kAuxPairsAfter of its block steps: run beside its large trailing
  // updates they take compute units from them (the updates measured 76-131
  // instead of ~150 TFLOP/s), while its last block steps (bound by the panel
  // chain) and its first-moment solve leave the chip partly idle.  Measured on
  // the s = 2..5 sphere ladder: 0.585 s per mixed step without the wait,
  // 0.580-0.581 s at 0.6-0.9, 0.586-0.590 s at 0.95-0.99.
  constexpr double kAuxPairsAfter = 0.8;
  std::mutex mu;
  std::condition_variable cv;
  bool coarse_ready = false, mark_ready = false;
  // build_err is written before coarse_ready is published; pair_err only
  // before the worker ends, and read after the join
  std::exception_ptr build_err, pair_err;
  struct MarkEvent {
    hipEvent_t ev = nullptr;
    ~MarkEvent() {
      if (ev) (void)hipEventDestroy(ev);
    }
  } mark;
  FOSB_HIP(hipEventCreateWithFlags(&mark.ev, hipEventDisableTiming));
  std::thread worker([&] {
    PoolRelease pool_release;
    try {
      bind(aux);
      for (int i = top - 1; i >= 0; --i) build(aux, i);
    } catch (...) {
      build_err = std::current_exception();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      coarse_ready = true;
    }
    cv.notify_all();
    if (build_err) return;
    try {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return mark_ready; });
      }
      FOSB_HIP(hipStreamWaitEvent(aux.stream, mark.ev, 0));
      for (size_t p = 0; p < v.size(); ++p)
        if (v[p][0] != L) pair(aux, p, &st_aux);
      FOSB_HIP(hipStreamSynchronize(aux.stream));
    } catch (...) {
      pair_err = std::current_exception();
    }
  });
  struct Joiner {
    std::thread& t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } joiner{worker};
  auto release_aux = [&] {
    {
      std::lock_guard<std::mutex> lk(mu);
      mark_ready = true;
    }
    cv.notify_all();
  };
  // the mark is recorded by the finest level's blocked factorisation; a level
  // that factors without blocks (or fails) records it on the main stream here
  struct MarkGuard {
    Context& c;
    hipEvent_t ev;
    ~MarkGuard() {
      if (c.lu_mark_cb) {
        (void)hipEventRecord(ev, c.stream);
        std::function<void()> cb = std::move(c.lu_mark_cb);
        c.lu_mark_cb = nullptr;
        cb();
      }
      c.lu_mark_ev = nullptr;
    }
  };
  ctx->lu_mark_ev = mark.ev;
  ctx->lu_mark_frac = kAuxPairsAfter;
  ctx->lu_mark_cb = release_aux;
  {
    MarkGuard guard{*ctx, mark.ev};
    build(*ctx, top);
  }
  {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return coarse_ready; });
  }
  if (!build_err)
    for (size_t p = 0; p < v.size(); ++p)
      if (v[p][0] == L) pair(*ctx, p, &st_main);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  worker.join();
  if (build_err) std::rethrow_exception(build_err);
  if (pair_err) std::rethrow_exception(pair_err);

  std::vector<const fosb_level*> lp(n_levels);
  for (int i = 0; i < n_levels; ++i) {
    lv[i]->ctx = ctx;  // handles belong to the caller's context from here on
    lp[i] = lv[i].get();
  }
  far_field_impl(*ctx, lp.data(), L0, L, blocks, ldb, xhat, n_a, d0, nd, var, nullptr);
  merge_stats(stats, st_main);
  merge_stats(stats, st_aux);
  for (int i = 0; i < n_levels; ++i) merge_level_certificate(stats, *lv[i]);
  if (levels_out) {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    for (int i = 0; i < n_levels; ++i) {
      ctx->live_levels.insert(lv[i].get());
      levels_out[i] = lv[i].release();
    }
  }
  API_END
}

fosb_status fosb_second_moment_batch(fosb_context* ctx, const fosb_batch_shape* shapes, int64_t n_shapes,
                                     int32_t precision, const double* xhat, int64_t n_a, const fosb_opts* opts,
                                     int32_t n_workers, fosb_stats* stats) {
  API_BEGIN
  REQUIRE(ctx && shapes && xhat, "NULL argument");
  REQUIRE(n_shapes >= 1, "n_shapes must be >= 1");
  REQUIRE(n_workers >= 1 && n_workers <= 16, "n_workers must be 1..16");
  REQUIRE(n_a >= 1 && n_a <= 65535, "n_a must be 1..65535");
  for (int64_t i = 0; i < n_a; ++i) {
    double nn = xhat[3 * i] * xhat[3 * i] + xhat[3 * i + 1] * xhat[3 * i + 1] + xhat[3 * i + 2] * xhat[3 * i + 2];
    REQUIRE(std::fabs(nn - 1.0) < 1e-9, "xhat[%lld] is not a unit vector", (long long)i);
  }
  for (int64_t s = 0; s < n_shapes; ++s) {
    const fosb_batch_shape& b = shapes[s];
    REQUIRE(b.meshes && b.var, "shape %lld: meshes/var is NULL", (long long)s);
    REQUIRE(b.L0 >= 0 && b.L >= b.L0 && b.n_levels == b.L - b.L0 + 1, "shape %lld: n_levels must be L - L0 + 1",
            (long long)s);
    for (int32_t i = 0; i < b.n_levels; ++i) {
      REQUIRE(b.meshes[i] && b.meshes[i]->ctx == ctx, "shape %lld: mesh %d is NULL or foreign", (long long)s, i);
      if (i > 0) REQUIRE(b.meshes[i]->h.ne > b.meshes[i - 1]->h.ne, "shape %lld: levels must go coarse to fine",
                         (long long)s);
    }
    check_physics(b.k, precision, b.dirs, b.pols, b.n_dirs, b.field);
    check_cov(&b.cov);
  }
  const fosb_opts o = opts_or_default(opts);
  bind(*ctx);
  const int nw = (int)std::min<int64_t>(n_workers, n_shapes);
  for (int w = 0; w < nw; ++w) ctx->worker_context(w);
  std::atomic<int64_t> next(0);
  std::atomic<bool> stop(false);
  std::vector<std::exception_ptr> err(nw);
  std::vector<fosb_stats> st(nw);
  for (auto& x : st) x = fosb_stats{};
  std::vector<std::thread> pool;
  struct PoolJoiner {   // joins the started workers also when starting another one throws
    std::vector<std::thread>& p;
    std::atomic<bool>& stop;
    ~PoolJoiner() {
      stop.store(true);
      for (auto& t : p)
        if (t.joinable()) t.join();
    }
  } pool_joiner{pool, stop};
  for (int w = 0; w < nw; ++w)
    pool.emplace_back([&, w] {
      Context& c = *ctx->workers[w];
      PoolRelease pool_release;
      try {
        bind(c);
        for (;;) {
          if (stop.load()) break;
          const int64_t s = next.fetch_add(1);
          if (s >= n_shapes) break;
          const fosb_batch_shape& b = shapes[s];
          shape_pipeline(c, b.meshes, b.n_levels, b.L0, b.L, b.k, precision, b.dirs, b.pols, b.n_dirs, b.field,
                         b.cov, xhat, n_a, b.var, o, &st[w]);
        }
        FOSB_HIP(hipStreamSynchronize(c.stream));
      } catch (...) {
        err[w] = std::current_exception();
        stop.store(true);
      }
    });
  for (auto& t : pool) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  for (const fosb_stats& x : st) merge_stats(stats, x);
  API_END
}

fosb_status fosb_autotune(fosb_context* ctx, int32_t mode, int32_t* n_entries) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  REQUIRE(mode >= -1 && mode <= 2, "mode must be -1, 0, 1 or 2");
  std::lock_guard<std::mutex> lock(ctx->tune_mu);
  if (mode == 2) ctx->tune.clear();
  if (mode == 0) ctx->autotune = 0;
  if (mode >= 1) ctx->autotune = 1;
  if (n_entries) *n_entries = (int32_t)ctx->tune.size();
  API_END
}

fosb_status fosb_autotune_table(fosb_context* ctx, int64_t* keys, int32_t* variants, int64_t capacity,
                                int64_t* n_entries) {
  API_BEGIN
  REQUIRE(ctx && n_entries, "ctx/n_entries is NULL");
  REQUIRE(capacity >= 0, "capacity must be >= 0");
  REQUIRE(capacity == 0 || (keys && variants), "keys/variants is NULL");
  std::lock_guard<std::mutex> lock(ctx->tune_mu);
  int64_t i = 0;
  for (const auto& kv : ctx->tune) {  // std::map: increasing key order
    if (i >= capacity) break;
    keys[i] = kv.first;
    variants[i] = kv.second;
    ++i;
  }
  *n_entries = (int64_t)ctx->tune.size();
  API_END
}

fosb_status fosb_autotune_load(fosb_context* ctx, const int64_t* keys, const int32_t* variants, int64_t n) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  REQUIRE(n >= 0, "n must be >= 0");
  REQUIRE(n == 0 || (keys && variants), "keys/variants is NULL");
  for (int64_t i = 0; i < n; ++i) {
    REQUIRE(keys[i] >= 0 && (keys[i] >> 41) == 0, "entry %lld: key has bits above 40 set", (long long)i);
    const int nv = tile_variant_count((keys[i] >> 40) & 1);
    REQUIRE(variants[i] >= 0 && variants[i] < nv, "entry %lld: variant %d out of range 0..%d", (long long)i,
            (int)variants[i], nv - 1);
  }
  std::lock_guard<std::mutex> lock(ctx->tune_mu);
  for (int64_t i = 0; i < n; ++i) ctx->tune[keys[i]] = variants[i];
  API_END
}

fosb_status fosb_profile_enable(fosb_context* ctx, int32_t on) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  bind(*ctx);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->aux) FOSB_HIP(hipStreamSynchronize(ctx->aux->stream));
  for (auto& w : ctx->workers) FOSB_HIP(hipStreamSynchronize(w->stream));
  {
    std::lock_guard<std::mutex> lock(ctx->prof_mu);
    if (on) ctx->recs.clear();
    ctx->prof_on = on != 0;
  }
  API_END
}

fosb_status fosb_profile_read(fosb_context* ctx, int32_t cls, int64_t* launches, double* seconds, double* flops,
                              double* bytes) {
  API_BEGIN
  REQUIRE(ctx, "ctx is NULL");
  REQUIRE(cls >= 0 && cls < FOSB_K_COUNT, "unknown kernel class %d", cls);
  bind(*ctx);
  FOSB_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->aux) FOSB_HIP(hipStreamSynchronize(ctx->aux->stream));
  for (auto& w : ctx->workers) FOSB_HIP(hipStreamSynchronize(w->stream));
  std::lock_guard<std::mutex> lock(ctx->prof_mu);
  int64_t cnt = 0;
  double sec = 0, fl = 0, by = 0;
  for (const ProfRec& r : ctx->recs) {
    if (r.cls != cls) continue;
    float ms = 0.f;
    FOSB_HIP(hipEventElapsedTime(&ms, ctx->ev_pool[r.ev], ctx->ev_pool[r.ev + 1]));
    ++cnt;
    sec += 1e-3 * ms;
    fl += r.flops;
    by += r.bytes;
  }
  if (launches) *launches = cnt;
  if (seconds) *seconds = sec;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  API_END
}

}  // extern "C"
