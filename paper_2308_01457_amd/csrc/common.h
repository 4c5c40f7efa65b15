// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fosb.h"

namespace fosb {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  fosb_status status;
  Error(fosb_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void fail(fosb_status s, const char* fmt, ...);
void set_last_error(const std::string& msg);

#define FOSB_HIP(call)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      ::fosb::fail(e_ == hipErrorOutOfMemory ? FOSB_E_OOM : FOSB_E_DEVICE, "%s failed: %s (%s:%d)", \
                   #call, hipGetErrorString(e_), __FILE__, __LINE__);                          \
  } while (0)

#define FOSB_LAUNCH_CHECK() FOSB_HIP(hipGetLastError())

// ------------------------------------------------------------------ complex storage
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};
using c128 = cplx<double>;
using c64 = cplx<float>;

// ------------------------------------------------------------------ device buffers
// Caching device allocator of one context.  Every context runs its work on
// one stream, so a block returned to its pool may be handed out again at once:
// later work on that stream is ordered after the work that used it.  Blocks
// are only returned to the device (hipFree, which synchronises the device) by
// trim() or when the last owner of the pool goes away, so a pass repeated on
// the same shapes allocates nothing after its first run.
struct Pool {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;  // cached blocks by capacity
  size_t cached_bytes = 0;                   // capacity held in free_blocks
  size_t live_bytes = 0;                     // capacity handed out and not returned
  int64_t n_device_allocs = 0;               // hipMalloc calls made
  void* get(size_t n, size_t& cap);
  void put(void* p, size_t cap);
  void trim();
  ~Pool();
};

// The pool used by buffers that are not bound to one: that of the context
// whose work the calling thread is enqueueing (set by bind_pool).
std::shared_ptr<Pool>& thread_pool();
// Set while the calling thread runs the allocation-free entry point: any
// device buffer allocation then fails instead of reaching a pool or hipMalloc.
bool& thread_no_alloc();

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;                 // requested size
  size_t cap = 0;                   // capacity of the block
  std::shared_ptr<Pool> home;       // pool this buffer always draws from (context members)
  std::shared_ptr<Pool> from;       // pool the current block came from
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept
      : p(o.p), bytes(o.bytes), cap(o.cap), home(std::move(o.home)), from(std::move(o.from)) {
    o.p = nullptr; o.bytes = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; cap = o.cap; home = std::move(o.home); from = std::move(o.from);
      o.p = nullptr; o.bytes = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    if (thread_no_alloc()) fail(FOSB_E_DEVICE, "internal: device buffer of %zu bytes on the allocation-free path", n);
    std::shared_ptr<Pool> pool = home ? home : thread_pool();
    if (pool) {
      p = pool->get(n, cap);
      from = std::move(pool);
    } else {
      FOSB_HIP(hipMalloc(&p, n));
      cap = n;
    }
    bytes = n;
  }
  // grow-only (contents are not preserved when it grows past the block's capacity)
  void reserve(size_t n) {
    if (n <= bytes) return;
    if (p && n <= cap) { bytes = n; return; }
    alloc(n);
  }
  void release() {
    if (p) {
      if (from) from->put(p, cap);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = cap = 0;
    from.reset();
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

template <typename T>
inline void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  b.alloc(v.size() * sizeof(T));
  if (!v.empty()) FOSB_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------------------ profiling records
struct ProfRec {
  int cls;
  int ev;          // index of the start event in the pool (stop = ev + 1)
  double flops, bytes;
};

// ------------------------------------------------------------------ context
struct Context {
  std::shared_ptr<Pool> pool = std::make_shared<Pool>();   // declared first: destroyed last
  Context();
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  size_t max_lds = 65536;
  // reusable scratch (grow-only); each user documents which slot it uses
  DevBuf scratch[6];
  DevBuf solve_tmp;   // block-inverse solves: leaf products (LU block rows), intermediate (refined solves)
  DevBuf counters;    // int32 tree counters for panel factorisation
  DevBuf small;       // small per-panel buffers
  // Sauter-Schwab point tables per Gauss order n (1..12): 5 doubles per point,
  // kinds 0/1/2 concatenated; offsets and counts in points.
  DevBuf norms;       // refinement norms: 2 doubles + per-block partials
  DevBuf splitk;      // partial products of split-K GEMMs
  DevBuf tune_out;    // scratch output of autotuning runs
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  // handles created on this context and not yet destroyed: destroying the
  // context detaches them (their ctx becomes null), so a later destroy of a
  // handle never touches a freed context
  std::set<struct Level*> live_levels;
  std::set<struct Mesh*> live_meshes;
  std::mutex reg_mu;
  // GEMM tile autotuner (kept by the root context): size bucket -> variant
  int autotune = 1;
  // > 0: GEMMs launched on this context use the tile variant with the smallest
  // register and LDS footprint instead of the tuned one (set while this
  // context's kernels share the chip with a saturating GEMM on another stream)
  int lean_tiles = 0;
  // > 0: no GEMM on this context may allocate: split K and tile timing are off
  // (a tuned size bucket keeps its tile, others take the first tile)
  int no_alloc = 0;
  // > 0: this context runs the trailing update of a blocked LU; its large
  // complex64 GEMMs take the 64 x 64 tile instead of the tuned one
  int trailing_update = 0;
  std::map<int64_t, int> tune;
  std::mutex tune_mu;
  DevBuf ss[13];
  int ss_off[13][3] = {};
  int ss_cnt[13][3] = {};
  // profiler (fosb_profile_*): event pool and records of the current session,
  // kept by the root context for itself and its auxiliary context
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> recs;
  std::mutex prof_mu;
  // auxiliary context: own stream (created by the library, default priority)
  // and own scratch, used by the concurrent pipeline; its profiler root is the
  // owning context
  Context* prof_root = nullptr;
  bool owns_stream = false;
  std::unique_ptr<Context> aux;
  Context& aux_context();
  // LU update stream (blocked LU with lookahead) and its two events
  std::unique_ptr<Context> la;
  Context& la_context();
  hipEvent_t lu_ev[2] = {nullptr, nullptr};
  // Progress mark of the next blocked factorisation on this context, for a
  // caller that orders other streams' work behind part of it: with lu_mark_cb
  // set, the factorisation records lu_mark_ev on its update stream when it
  // starts block step floor(lu_mark_frac * blocks) (everything before that step
  // done), then calls lu_mark_cb once on the host and clears it.
  hipEvent_t lu_mark_ev = nullptr;
  double lu_mark_frac = 0.0;
  std::function<void()> lu_mark_cb;
  // batch workers: own streams, scratch and per-shape workspaces (Z, Zlow, blocks)
  std::vector<std::unique_ptr<Context>> workers;
  std::vector<DevBuf> ws_Z, ws_Zlow, ws_blocks;
  Context& worker_context(size_t i);
  ~Context();
};

// Makes ctx's pool the calling thread's pool (thread_pool()).
void bind_pool(Context& ctx);
// Sums of the pool counters of a context and its auxiliary, update and worker contexts.
void pool_totals(Context& ctx, int64_t& n_allocs, int64_t& cached, int64_t& live);
void pool_trim(Context& ctx);

// Brackets the launches issued during its lifetime with a pair of events when
// the context's profiler is on.
struct ProfScope {
  Context& ctx;      // records go to the root context ...
  hipStream_t stream;  // ... events are recorded on the launching context's stream
  int idx = -1;
  ProfScope(Context& c, int cls, double flops, double bytes);
  ~ProfScope();
};

// ------------------------------------------------------------------ mesh
struct MeshHost {
  int64_t nv = 0, nt = 0, ne = 0;
  std::vector<double> V;           // nv*3
  std::vector<int32_t> F;          // nt*3
  std::vector<double> area;        // nt
  std::vector<double> normal;      // nt*3
  std::vector<int32_t> tri_edge;   // nt*3
  std::vector<double> tri_sign;    // nt*3
  std::vector<double> edge_len;    // ne
  std::vector<int32_t> edge_tri;   // ne*2 (T+, T-)
  std::vector<int32_t> edge_loc;   // ne*2
  // touching ordered pairs (i, j), sorted by j then i
  std::vector<int32_t> tp_i, tp_j, tp_kind;   // kind: 0 identical, 1 edge, 2 vertex
  std::vector<int32_t> tp_ord;                // 6 per pair: local slots of (P0,P1,P2) in i, then in j
};

// Structure-of-arrays device view of a mesh (passed by value to kernels).
struct MeshDev {
  int nt, ne;
  const double* vtx;      // [9][nt]: component (v*3+c) of triangle t at vtx[(v*3+c)*nt + t]
  const double* area;     // [nt]
  const double* nrm;      // [3][nt]
  const double* alpha;    // [3][nt]: sign * edge length / area of local RWG a
  const int32_t* fv;      // [3][nt] vertex ids
  const int32_t* tri_edge;// [3][nt]
  const int32_t* edge_tri;// [2][ne]
  const int32_t* edge_loc;// [2][ne]
};

struct Mesh {
  Context* ctx = nullptr;
  MeshHost h;
  DevBuf vtx, area, nrm, alpha, fv, tri_edge, edge_tri, edge_loc;
  DevBuf tp_i, tp_j, tp_kind, tp_ord;
  MeshDev dev() const {
    return MeshDev{(int)h.nt, (int)h.ne, vtx.as<double>(), area.as<double>(), nrm.as<double>(),
                   alpha.as<double>(), fv.as<int32_t>(), tri_edge.as<int32_t>(),
                   edge_tri.as<int32_t>(), edge_loc.as<int32_t>()};
  }
};

void mesh_build_host(const double* V, int64_t nv, const int32_t* F, int64_t nt, MeshHost& out);
void mesh_touching_pairs(MeshHost& m);
void mesh_upload(Mesh& m);

// ------------------------------------------------------------------ quadrature (host-built tables)
// 6-point degree-4 rule: barycentric coordinates (6x3) and weights (6), per unit area.
void rule6(double bary[6][3], double w[6]);
// Gauss-Legendre on [0,1].
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
// Sauter-Schwab points for kind 0/1/2: xhat (2 per point), yhat (2 per point), weight.
void sauter_schwab_points(int kind, int n, std::vector<double>& pts /* 5 per point: x1,x2,y1,y2,w */);

// ------------------------------------------------------------------ level
struct Level {
  Context* ctx = nullptr;
  const Mesh* mesh = nullptr;
  double k = 1.0;
  int precision = FOSB_PREC_FP64;
  int64_t n = 0;
  void* Z = nullptr;        // FP64: LU factors; MIXED: the FP64 matrix (read-only)
  int64_t ldz = 0;
  void* Zlow = nullptr;     // MIXED: complex64 LU factors
  int64_t ldzlow = 0;
  int64_t n_dirs = 0;
  int field = FOSB_FIELD_RADIAL;
  fosb_opts opts{};
  std::vector<int32_t> perm;   // host: row permutation (position i holds original row perm[i])
  DevBuf d_perm;               // int32 [n]
  DevBuf dinv_L, dinv_U;       // inverted nb x nb diagonal blocks of L and U (LU precision)
  DevBuf inv_L, inv_U;         // MIXED: inverted kInvBlock x kInvBlock diagonal blocks of L and U (complex64)
  DevBuf u;                    // c128 [n_dirs][n]
  DevBuf W;                    // c128 [n_dirs][nt][3][6] RHS weights
  DevBuf qx;                   // double [3][6*nt] quadrature nodes (component-major)
  // certificate (opts.certify): norms of the assembled Z, condition estimate, growth factor
  double z_max = 0, z_fro = 0, z_one = 0, kappa1 = 0, growth = 0;
  // formulation: FOSB_FORM_EFIE (N = edges) or FOSB_FORM_PMCHWT (N = 2 edges,
  // unknowns [J; M], interior eps_r, mu_r; b keeps the right-hand sides)
  int form = FOSB_FORM_EFIE;
  double eps_r = 1.0, mu_r = 1.0;
  DevBuf b;                    // PMCHWT: c128 [n][n_dirs]
  int sd_field = -1;           // PMCHWT: field of the shape-derivative weights (-1: none built)
  int sd_streamed = 0;         // PMCHWT: weights recomputed by source bands when used, none stored
  int sym_lu = 0;              // MIXED: factored without pivoting (symmetric form)
  int sym_sign = 0;            // MIXED PMCHWT: the FP32 factors are of S Z, S = diag(I, -I) on [J; M]
  DevBuf Wsd;                  // PMCHWT: c128 [n_dirs][n][6 nt] shape-derivative weights (with nu)
  const void* lu() const { return precision == FOSB_PREC_FP64 ? Z : Zlow; }
};

constexpr int kPanel = 32;   // LU panel width / TRSM diagonal block size

// ------------------------------------------------------------------ kernels (host launchers)
// assemble.hip
// Zl (optional): also receives Z rounded to complex64, each entry written once it is final
void assemble_efie(Context& ctx, const Mesh& m, double k, int n_gauss, c128* Z, int64_t ldz, c64* Zl = nullptr,
                   int64_t ldl = 0);
// the same matrix assembled in FP64 and stored rounded to complex64 (no complex128 copy)
void assemble_efie_c64(Context& ctx, const Mesh& m, double k, int n_gauss, c64* Z, int64_t ldz);
// R (N x nrhs) -= Z X in FP64 with Z re-assembled band by band and discarded
void efie_residual(Context& ctx, const Mesh& m, double k, int n_gauss, const c128* X, int64_t ldx, int64_t nrhs,
                   c128* R, int64_t ldr);
// the 2N x 2N PMCHWT matrix [[T0 + eta T1, K0 + K1], [-(K0 + K1), T0 + T1/eta]] (EFIE blocks T, MFIO
// blocks K at k0 and k1 = k0 sqrt(eps_r mu_r), eta = sqrt(mu_r / eps_r)); synchronises the stream
void assemble_pmchwt(Context& ctx, const Mesh& m, double k0, double eps_r, double mu_r, int n_gauss, c128* Z,
                     int64_t ldz);
// W (2N x 6 nt, row stride ldw) of the dielectric shape derivative (mu_r = 1) for the first moment
// in column dir of u (2N x ldu): r = W v for the amplitude v at the 6-point nodes (field: radial or
// normal); synchronises the stream
void sd_weights(Context& ctx, const Mesh& m, double k0, double eps_r, int field, const c128* u, int64_t ldu,
                int64_t dir, int n_gauss, c128* W, int64_t ldw);
// The same weights by source-triangle bands: sd_plan once per (level, incidence) (per-triangle data
// and the touching (row, triangle) list sorted by triangle), then sd_band writes columns
// [6 j0, 6 j1) into W (2N x 6 (j1 - j0), row stride ldw), enqueued on the stream.
struct SdPlan {
  DevBuf td, dm, dj, dp;
  std::vector<int64_t> jbeg;
};
void sd_plan(Context& ctx, const Mesh& m, double k0, double eps_r, const c128* u, int64_t ldu, int64_t dir,
             SdPlan& P);
void sd_band(Context& ctx, const Mesh& m, const SdPlan& P, double k0, double eps_r, int field, int n_gauss, int j0,
             int j1, c128* W, int64_t ldw);
// gemm.hip: C = beta*C + alpha*A*B, complex, row-major.
template <typename T>
void gemm(Context& ctx, int64_t M, int64_t N, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
          const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc);
// number of GEMM tile variants (gemm.hip, Tiles<T>::n) for complex64 (fp64 = 0)
// or complex128 (fp64 = 1)
inline int tile_variant_count(int fp64) { return fp64 ? 3 : 4; }
// C = beta*C + alpha*A^H*B; A is stored K x M (row-major, leading dimension lda)
template <typename T>
void gemm_ch(Context& ctx, int64_t M, int64_t N, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
             const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc);
// lu.hip
// invL (optional, complex64 factors): receives the kInvBlock x kInvBlock
// diagonal-block inverses of L (layout as for upper_block_inverses); the
// blocked factorisation then also solves its block rows through them.
// sym: the matrix is (numerically) symmetric; for n >= 2048 it is factored
// without pivoting, A = L U with U = D L^T formed from the multipliers and the
// trailing updates restricted to the lower triangle (about half the flops).
// The caller judges the result (zero pivot through the return value, growth).
template <typename T>
int64_t lu_factor(Context& ctx, cplx<T>* A, int64_t n, int64_t lda, cplx<T>* dinvL, cplx<T>* dinvU,
                  std::vector<int32_t>& perm, cplx<T>* invL = nullptr, bool sym = false);
// *defect = max over i, j of |A[i][j] - A[j][i]|, *amax = max |A[i][j]|, in
// one pass (rounded to float; synchronises the stream)
template <typename T>
void sym_check(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, double* defect, double* amax);
// max |A[i][j]| over j >= i (rounded to float; synchronises the stream)
template <typename T>
double absmax_upper(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda);
template <typename T>
void trsm_lower_unit(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvL, int64_t k0,
                     int64_t n, cplx<T>* B, int64_t ldb, int64_t nrhs);
template <typename T>
void trsm_upper(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvU, int64_t k0, int64_t n,
                cplx<T>* B, int64_t ldb, int64_t nrhs);
// B <- U^{-H} B and B <- L^{-H} B with the same stored factors
template <typename T>
void trsm_upper_ch(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvU, int64_t k0, int64_t n,
                   cplx<T>* B, int64_t ldb, int64_t nrhs);
template <typename T>
void trsm_lower_unit_ch(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvL, int64_t k0, int64_t n,
                        cplx<T>* B, int64_t ldb, int64_t nrhs);
// Inverses of the kInvBlock x kInvBlock diagonal blocks of the upper factor
// (block b at inv + b kInvBlock^2, row-major, row stride kInvBlock; the last
// block's slot is the identity outside its corner; lu_factor makes L's), and
// out-of-place triangular solves of a whole factor that apply them at the
// leaves: X <- T^{-1} B, with B (n x nrhs) consumed as workspace.  Complex64
// factors only.
constexpr int kInvBlock = 256;
template <typename T>
void upper_block_inverses(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, const cplx<T>* dinvU,
                          cplx<T>* invU);
template <typename T>
void trsm_lower_unit_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* invL, int64_t n, cplx<T>* B,
                         int64_t ldb, cplx<T>* X, int64_t ldx, int64_t nrhs);
template <typename T>
void trsm_upper_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* invU, int64_t n, cplx<T>* B,
                    int64_t ldb, cplx<T>* X, int64_t ldx, int64_t nrhs);
void permute_rows_gather(hipStream_t s, const int32_t* perm, const c128* src, int64_t lds, c128* dst,
                         int64_t ldd, int64_t n, int64_t ncols);
// dst[perm[i]] = src[i]
void permute_rows_scatter(hipStream_t s, const int32_t* perm, const c128* src, int64_t lds, c128* dst,
                          int64_t ldd, int64_t n, int64_t ncols);
void copy_c128_to_c64(hipStream_t s, const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int64_t cols);
// rows [r0, r1) of a complex64 matrix (row stride ld, cols columns) <- their negatives
void negate_rows_c64(hipStream_t s, c64* p, int64_t ld, int64_t r0, int64_t r1, int64_t cols);
void copy_c64_to_c128(hipStream_t s, const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int64_t cols);
void copy_c128(hipStream_t s, const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int64_t cols);
// dst = diag(row_scale) src^H (row_scale: device, one per dst row, or nullptr)
void conj_transpose_c128(hipStream_t s, const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows,
                         int64_t cols, const double* row_scale = nullptr);
void conj_inplace_c128(hipStream_t s, c128* x, int64_t n);
void axpy_c128(hipStream_t s, const c128* x, int64_t ldx, c128* y, int64_t ldy, int64_t rows, int64_t cols);
// squared Frobenius norms of x and of y (two doubles written to out, device);
// out has room for 2 + 2 * kNormBlocks doubles (per-block partial sums follow
// the two results, reduced in a fixed order)
constexpr int kNormBlocks = 1024;
void norms2_c128(hipStream_t s, const c128* x, int64_t ldx, const c128* y, int64_t ldy, int64_t rows,
                 int64_t cols, double* out);
// uq.hip
// b[m * ndir + d] = -int p_d exp(i k d_d . x) . phi_m  (dirs/pols: device, ndir x 3)
void incident_rhs(hipStream_t s, const Mesh& m, double k, const double* dirs_dev, const double* pols_dev, int ndir,
                  c128* b);
void quad_nodes(hipStream_t s, const Mesh& m, double* qx);
// u: first-moment coefficients of one direction, u[e * ustride]
void rhs_weights(hipStream_t s, const Mesh& m, double k, int field, const c128* u, int64_t ustride, c128* W);
void rhs_correlation_kernel(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t dir,
                            c128* C, int64_t ldc);
// C_d = Wgt_l1(dir0 + d) K Wgt_l2(dir0 + d)^H for d < nd at C + d * dstride (row stride ldc)
void rhs_correlation_multi(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t dir0,
                           int64_t nd, c128* C, int64_t ldc, int64_t dstride);
// PMCHWT right-hand side b = [e; h] (2N x ndir, row stride ndir): e[m] = int phi_m . p e^{ik d.x},
// h[m] = int phi_m . (d x p) e^{ik d.x}
void incident_rhs_pmchwt(hipStream_t s, const Mesh& m, double k, const double* dirs_dev, const double* pols_dev,
                         int ndir, c128* b);
// PMCHWT far-field map (3 n_a x 2N): i k [(I - x x^T) A_m | -x x A_m], A_m = int phi_m e^{-ik x.y}
void far_field_matrix_pmchwt(hipStream_t s, const Mesh& m, double k, const double* xhat_dev, int64_t n_a, c128* FF);
// C[i][j] = b1[i] conj(b2[j]) (b1: n1 x nd, b2: n2 x nd, column dir)
void rank_one_correlation(hipStream_t s, const c128* b1, int64_t n1, const c128* b2, int64_t n2, int64_t nd,
                          int64_t dir, c128* C, int64_t ldc);
void far_field_matrix_kernel(hipStream_t s, const Mesh& m, double k, const double* xhat_dev, int64_t n_a,
                             c128* FF);
// NF[(c*n_p + p)][m]: scattered field at the field points x_p (device, n_p x 3) of each RWG
void near_field_matrix_kernel(hipStream_t s, const Mesh& m, double k, const double* xp_dev, int64_t n_p, c128* NF);
void row_dot_re_accumulate(hipStream_t s, const c128* P, int64_t ldp, const c128* FF2, int64_t rows, int64_t n,
                           double scale, double* var);
void matvec_rows(hipStream_t s, const c128* FF, int64_t rows, int64_t n, const c128* u, c128* out);
// adjoint of the variance: node rows Hn (Q x R) of FF Z^{-1} Wgt from B = Z^{-H} FF^H (N x R)
void adjoint_nodes(hipStream_t s, const Mesh& m, const c128* W, const c128* B, int64_t R, c128* Hn);
// partial sums of kappa Re G and dkappa/dell Re G over rows [a0, a0 + na) of G (Q1 x Q2 block
// of a pair); returns the number of partial pairs written
int64_t cov_grad_partials(hipStream_t s, const c128* G, int64_t a0, int64_t na, const Level& l1, const Level& l2,
                          const fosb_cov& cov, double scale, double* partial);
void cov_grad_finish(hipStream_t s, const double* partial, int64_t n, double sigma, double* out);
// rows [a0, a0 + na) of the covariance between the nodes of l1 and l2, as complex (row stride Q2)
void cov_matrix(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t a0, int64_t na,
                c128* Kc);
// out[r] += scale Re sum_{q < n} A[q][r] B[q][r] (row stride R); part: (n/256 + 1) R doubles of scratch
void coldot_re_accumulate(hipStream_t s, const c128* A, const c128* B, int64_t n, int64_t R, double scale,
                          double* part, double* out);

// out (device, 3 doubles): max |a_ij|, sum |a_ij|^2 and max_j sum_i |a_ij| of an
// n x n complex matrix, over its upper triangle only when upper is set
template <typename T>
void matrix_norms(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, bool upper, double* out);
// out (n x n) += scale * (T + T^H if both, else T), T n x n (row strides ldt, ldo)
void herm_accumulate(hipStream_t s, const c128* T, int64_t ldt, int64_t n, double scale, bool both, c128* out,
                     int64_t ldo);

// noalloc.hip: the allocation-free entry point's work memory (a file-scope
// device array per GPU, FOSB_NOALLOC_SCRATCH_BYTES), its per-device set-up
// (hipGetSymbolAddress, once per device, with that device current) and its
// device address; and a zero fill that needs no memset node.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
void noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
void zero_f64(hipStream_t s, double* p, int64_t n);

// lowrank.hip: pivoted Cholesky of the covariance on a ladder's quadrature nodes
// (candidates Xc, Nc: [3][nc]; factor L column-major, L[k * nc + i]).
void lr_candidates(hipStream_t s, const Level& l, int64_t off, int64_t nc, double* Xc, double* Nc);
void lr_diag(hipStream_t s, const double* Nc, int64_t nc, const fosb_cov& cov, double* d);
// out (device, 2 doubles) = {d[p], p}: p the lowest index with d[p] >= (1 - tie) max d
void lr_pivot(hipStream_t s, const double* d, int64_t nc, double tie, double* out);
void lr_column(hipStream_t s, const double* Xc, const double* Nc, int64_t nc, const fosb_cov& cov, double* L, int j,
               int64_t p, double dp, double* d);
// M (N x rank) = Wgt_dir L_l with L_l the factor's rows [off, off + 6 nt) (Lr: scratch, 6 nt x rank doubles)
// the level's rows of the factor, node-major (Q x rank); a real array widened to complex128
void lr_rows(hipStream_t s, const Level& l, const double* L, int64_t nc, int64_t off, int rank, double* Lr);
void real_to_c128(hipStream_t s, const double* a, int64_t n, c128* b);
void lr_rhs(hipStream_t s, const Level& l, int64_t dir, const double* L, int64_t nc, int64_t off, int rank,
            double* Lr, c128* M);

// level-wide solves (api.cpp helpers)
// B <- Z^{-1} B, or B <- Z^{-H} B (adjoint); max_sweeps >= 0 overrides the
// level's refinement sweep limit (0: the factors' solve alone)
void level_solve_inplace(Context& ctx, const Level& L, c128* B, int64_t ldb, int64_t nrhs, fosb_stats* st,
                         bool adjoint = false, int max_sweeps = -1);

}  // namespace fosb
