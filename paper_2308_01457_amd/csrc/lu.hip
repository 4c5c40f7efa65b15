// Dense complex LU with row pivoting, triangular solves and small helpers.
//
// LU (P Z = L U, L unit lower, row-major storage): recursive column splitting
// (left half, TRSM of the right half's top rows, GEMM update of the rest,
// right half) down to 32-column panels.  A panel is factorised with
// tournament pivoting: each 64-row block of the panel runs Gaussian
// elimination with partial pivoting in LDS and nominates 32 candidate rows,
// and the candidates are merged pairwise up a binary tree (the second
// workgroup to reach a tree node merges; a device-scope acquire/release
// counter per node orders the hand-over) until 32 pivot rows remain.  The
// pivot rows are swapped into place across the full matrix width, the panel
// below the diagonal block becomes A21 U11^{-1}, and the inverses of the
// 32x32 diagonal blocks of L and U are kept for the triangular solves.
//
// Triangular solves are recursive as well: halves are coupled by a GEMM and
// the 32-row leaves multiply by the stored diagonal-block inverse.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace fosb {

constexpr int NB = kPanel;   // panel width (32)
constexpr int RB = 64;       // rows per tournament leaf block
constexpr int SLD = NB + 1;  // LDS row pitch of a panel block

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cplx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cinv(cplx<T> a) {
  // 1/a with scaling to avoid overflow
  T s = fabs(a.re) + fabs(a.im);
  if (s == T(0)) return cplx<T>{T(0), T(0)};
  T ar = a.re / s, ai = a.im / s;
  T d = ar * ar + ai * ai;
  return cplx<T>{ar / (d * s), -ai / (d * s)};
}
template <typename T>
__device__ __forceinline__ T cabs1(cplx<T> a) {
  return fabs(a.re) + fabs(a.im);
}

// Gaussian elimination with partial pivoting on an nr x w block in LDS
// (nr <= 64, w <= 32), rows carrying their global index in idx[].  After the
// call rows 0..min(nr,w)-1 are the pivot rows in order, holding L (strictly
// below the diagonal, unit diagonal implied) and U.  Returns (to all threads)
// the first column with an exactly zero pivot, or -1.
template <typename T>
__device__ int gepp_lds(cplx<T> (*sa)[SLD], int* idx, int nr, int w, int* s_piv) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  int zero_col = -1;
  const int steps = min(nr, w);
  for (int j = 0; j < steps; ++j) {
    if (tid < 64) {
      T v = (lane >= j && lane < nr) ? cabs1(sa[lane][j]) : T(-1);
      int r = lane;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        T ov = __shfl_xor(v, off, 64);
        int orr = __shfl_xor(r, off, 64);
        if (ov > v || (ov == v && orr < r)) {
          v = ov;
          r = orr;
        }
      }
      if (lane == 0) *s_piv = r;
    }
    __syncthreads();
    const int p = *s_piv;
    if (p != j) {
      if (tid < w) {
        cplx<T> t = sa[j][tid];
        sa[j][tid] = sa[p][tid];
        sa[p][tid] = t;
      } else if (tid == w) {
        int t = idx[j];
        idx[j] = idx[p];
        idx[p] = t;
      }
    }
    __syncthreads();
    const cplx<T> piv = sa[j][j];
    if (piv.re == T(0) && piv.im == T(0) && zero_col < 0) zero_col = j;
    const cplx<T> inv = cinv(piv);
    for (int r = j + 1 + tid; r < nr; r += blockDim.x) sa[r][j] = cmul(sa[r][j], inv);
    __syncthreads();
    const int wc = w - j - 1;
    if (wc > 0) {
      const int tot = (nr - j - 1) * wc;
      for (int e = tid; e < tot; e += blockDim.x) {
        const int r = j + 1 + e / wc;
        const int c = j + 1 + e % wc;
        const cplx<T> l = sa[r][j], u = sa[j][c];
        cplx<T> a = sa[r][c];
        a.re -= l.re * u.re - l.im * u.im;
        a.im -= l.re * u.im + l.im * u.re;
        sa[r][c] = a;
      }
    }
    __syncthreads();
  }
  return zero_col;
}

struct PanelWork {
  int32_t* cand;      // candidate row indices, per tree level and node (NB each)
  int32_t* counters;  // one per tree node
  int32_t* lvl_cand;  // offset (in nodes) of each level in cand, [levels+1]
  int32_t* lvl_size;  // nodes per level
  int nlevels;
  int32_t* plist;     // [0] = count, then pairs (src, dst)
  int32_t* ipiv;      // global pivot positions (n)
  int32_t* info;      // first zero pivot (1-based), 0 if none
};

template <typename T>
__device__ void load_rows(const cplx<T>* A, int64_t lda, int64_t col0, int w, const int* rows, int nr,
                          cplx<T> (*sa)[SLD]) {
  for (int e = threadIdx.x; e < nr * w; e += blockDim.x) {
    const int r = e / w, c = e % w;
    sa[r][c] = A[(int64_t)rows[r] * lda + col0 + c];
  }
}

// Tournament pivoting of the panel rows [k, n) x columns [k, k + w).
template <typename T>
__global__ __launch_bounds__(256) void k_panel_tslu(const cplx<T>* __restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                    int w, PanelWork pw, cplx<T>* __restrict__ top,
                                                    cplx<T>* __restrict__ invL, cplx<T>* __restrict__ invU) {
  __shared__ cplx<T> sa[RB][SLD];
  __shared__ cplx<T> sinv[NB][SLD];
  __shared__ int idx[RB];
  __shared__ int s_piv, s_flag;
  const int tid = threadIdx.x;
  const int64_t m = n - k;
  int node = blockIdx.x;
  // leaf: GEPP on this block's rows
  int nr = (int)min<int64_t>(RB, m - (int64_t)node * RB);
  for (int r = tid; r < nr; r += blockDim.x) idx[r] = (int)(k + (int64_t)node * RB + r);
  __syncthreads();
  load_rows(A, lda, k, w, idx, nr, sa);
  __syncthreads();
  int zc = gepp_lds(sa, idx, nr, w, &s_piv);
  int ncand = min(nr, w);
  for (int level = 0; level < pw.nlevels - 1; ++level) {
    // publish this node's candidates
    int32_t* mine = pw.cand + (int64_t)(pw.lvl_cand[level] + node) * NB;
    for (int r = tid; r < NB; r += blockDim.x) mine[r] = r < ncand ? idx[r] : -1;
    const int parent = node >> 1;
    const int sib = node ^ 1;
    if (sib >= pw.lvl_size[level]) {  // no sibling: carry the candidates up unchanged
      node = parent;
      __syncthreads();
      continue;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      int old = __hip_atomic_fetch_add(pw.counters + pw.lvl_cand[level + 1] + parent, 1, __ATOMIC_ACQ_REL,
                                       __HIP_MEMORY_SCOPE_AGENT);
      s_flag = old;
      if (old == 1)
        __hip_atomic_store(pw.counters + pw.lvl_cand[level + 1] + parent, 0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_flag == 0) return;  // first to arrive: the sibling merges
    __threadfence();
    // merge: candidates of both children, original values
    const int32_t* c0 = pw.cand + (int64_t)(pw.lvl_cand[level] + 2 * parent) * NB;
    const int32_t* c1 = c0 + NB;
    if (tid == 0) {
      int cnt = 0;
      for (int r = 0; r < NB; ++r) {
        int v = __hip_atomic_load(c0 + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= 0) idx[cnt++] = v;
      }
      for (int r = 0; r < NB; ++r) {
        int v = __hip_atomic_load(c1 + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= 0) idx[cnt++] = v;
      }
      s_piv = cnt;
    }
    __syncthreads();
    nr = s_piv;
    __syncthreads();
    load_rows(A, lda, k, w, idx, nr, sa);
    __syncthreads();
    zc = gepp_lds(sa, idx, nr, w, &s_piv);
    ncand = min(nr, w);
    node = parent;
  }
  // root: rows 0..w-1 of sa hold L11 \ U11 of the chosen pivot rows
  const int wk = min(w, ncand);
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    top[e] = (r < wk && c < w) ? sa[r][c] : cplx<T>{T(0), T(0)};
  }
  if (zc >= 0 && tid == 0) atomicMin(pw.info, (int)(k + zc + 1));
  // inverse of the unit lower factor (column c per thread)
  if (tid < NB) {
    const int c = tid;
    for (int r = 0; r < NB; ++r) {
      cplx<T> x{r == c ? T(1) : T(0), T(0)};
      if (r < wk) {
        for (int t = c; t < r; ++t) {
          const cplx<T> l = sa[r][t], y = sinv[t][c];
          x.re -= l.re * y.re - l.im * y.im;
          x.im -= l.re * y.im + l.im * y.re;
        }
      }
      sinv[r][c] = (r < c) ? cplx<T>{T(0), T(0)} : x;
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += blockDim.x) invL[e] = sinv[e / NB][e % NB];
  __syncthreads();
  // inverse of the upper factor
  if (tid < NB) {
    const int c = tid;
    for (int r = NB - 1; r >= 0; --r) {
      cplx<T> x{r == c ? T(1) : T(0), T(0)};
      if (r < wk) {
        for (int t = r + 1; t <= c && t < wk; ++t) {
          const cplx<T> u = sa[r][t], y = sinv[t][c];
          x.re -= u.re * y.re - u.im * y.im;
          x.im -= u.re * y.im + u.im * y.re;
        }
        x = cmul(x, cinv(sa[r][r]));
      }
      sinv[r][c] = (r > c) ? cplx<T>{T(0), T(0)} : x;
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB; e += blockDim.x) invU[e] = sinv[e / NB][e % NB];
  // row interchanges: pivot r goes to position k + r (sequential swap semantics)
  if (tid == 0) {
    int pos[2 * NB], con[2 * NB];   // touched positions and their current original row
    int np = 0;
    auto find_pos = [&](int row) {  // current position of original row
      for (int q = 0; q < np; ++q)
        if (con[q] == row) return pos[q];
      return row;
    };
    auto slot = [&](int p) {
      for (int q = 0; q < np; ++q)
        if (pos[q] == p) return q;
      pos[np] = p;
      con[np] = p;
      return np++;
    };
    for (int r = 0; r < wk; ++r) {
      const int target = (int)(k + r);
      const int cur = find_pos(idx[r]);
      pw.ipiv[target] = cur;
      if (cur != target) {
        const int a = slot(target), b = slot(cur);
        const int t = con[a];
        con[a] = con[b];
        con[b] = t;
      }
    }
    int cnt = 0;
    for (int q = 0; q < np; ++q)
      if (con[q] != pos[q]) {
        pw.plist[1 + 2 * cnt] = con[q];  // source row (original content)
        pw.plist[2 + 2 * cnt] = pos[q];  // destination position
        ++cnt;
      }
    pw.plist[0] = cnt;
  }
}

// Apply the listed row moves to the full matrix width (column stripes of 64).
template <typename T>
__global__ __launch_bounds__(256) void k_permute_rows(cplx<T>* __restrict__ A, int64_t lda, int64_t ncols,
                                                      const int32_t* __restrict__ plist) {
  __shared__ cplx<T> buf[2 * NB][64];
  const int cnt = plist[0];
  const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  if (c < ncols)
    for (int e = g; e < cnt; e += 4) buf[e][threadIdx.x & 63] = A[(int64_t)plist[1 + 2 * e] * lda + c];
  __syncthreads();
  if (c < ncols)
    for (int e = g; e < cnt; e += 4) A[(int64_t)plist[2 + 2 * e] * lda + c] = buf[e][threadIdx.x & 63];
}

// Write L11\U11 into the diagonal block and form A21 U11^{-1} below it.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_finish(cplx<T>* __restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                      int w, const cplx<T>* __restrict__ top,
                                                      const cplx<T>* __restrict__ invU) {
  __shared__ cplx<T> su[NB][NB];
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) su[e / NB][e % NB] = invU[e];
  __syncthreads();
  const int64_t r = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  cplx<T>* row = A + r * lda + k;
  if (r < k + w) {
    const int rr = (int)(r - k);
    for (int c = 0; c < w; ++c) row[c] = top[rr * NB + c];
    return;
  }
  cplx<T> a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = c < w ? row[c] : cplx<T>{T(0), T(0)};
#pragma unroll
  for (int c = NB - 1; c >= 0; --c) {
    if (c < w) {
      T xr = 0, xi = 0;
#pragma unroll
      for (int t = 0; t <= c; ++t) {
        const cplx<T> u = su[t][c];
        xr += a[t].re * u.re - a[t].im * u.im;
        xi += a[t].re * u.im + a[t].im * u.re;
      }
      row[c] = cplx<T>{xr, xi};
    }
  }
}

// B (nr x nrhs, nr <= 32) <- Inv(nr x nr of a 32x32 block) * B.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_inv(const cplx<T>* __restrict__ inv, int nr, cplx<T>* __restrict__ B,
                                                   int64_t ldb, int64_t nrhs) {
  __shared__ cplx<T> si[NB][NB + 1];
  __shared__ cplx<T> sb[NB][65];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) si[e / NB][e % NB] = inv[e];
  for (int e = threadIdx.x; e < NB * 64; e += blockDim.x) {
    const int r = e / 64, c = e % 64;
    sb[r][c] = (r < nr && c0 + c < nrhs) ? B[(int64_t)r * ldb + c0 + c] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  const int c = threadIdx.x & 63;
  for (int r = threadIdx.x >> 6; r < nr; r += 4) {
    T xr = 0, xi = 0;
    for (int t = 0; t < nr; ++t) {
      const cplx<T> a = si[r][t], b = sb[t][c];
      xr += a.re * b.re - a.im * b.im;
      xi += a.re * b.im + a.im * b.re;
    }
    if (c0 + c < nrhs) B[(int64_t)r * ldb + c0 + c] = cplx<T>{xr, xi};
  }
}

// ------------------------------------------------------------------ host drivers
template <typename T>
struct LuRun {
  Context* ctx;
  cplx<T>* A;
  int64_t n, lda;
  cplx<T>* dinvL;
  cplx<T>* dinvU;
  PanelWork pw;
  cplx<T>* top;
  const int32_t* dmeta;          // per panel: 32 level offsets then 32 level sizes
  std::vector<int32_t> nlevels;  // per panel
};

constexpr int kMetaStride = 64;

static inline int64_t split_half(int64_t w) { return (int64_t)NB * (((w / NB) + 1) / 2); }

template <typename T>
static void panel(LuRun<T>& R, int64_t k, int w) {
  hipStream_t s = R.ctx->stream;
  const int64_t m = R.n - k;
  const int nblk = (int)((m + RB - 1) / RB);
  const int64_t blk = k / NB;
  ProfScope prof(*R.ctx, FOSB_K_PANEL, 0.0, (double)sizeof(cplx<T>) * (double)m * w * 3.0);
  PanelWork pw = R.pw;
  pw.lvl_cand = const_cast<int32_t*>(R.dmeta) + blk * kMetaStride;
  pw.lvl_size = pw.lvl_cand + kMetaStride / 2;
  pw.nlevels = R.nlevels[blk];
  hipLaunchKernelGGL(k_panel_tslu<T>, dim3(nblk), dim3(256), 0, s, R.A, R.lda, R.n, k, w, pw, R.top,
                     R.dinvL + blk * NB * NB, R.dinvU + blk * NB * NB);
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_permute_rows<T>, dim3((unsigned)((R.n + 63) / 64)), dim3(256), 0, s, R.A, R.lda, R.n,
                     pw.plist);
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_panel_finish<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, R.A, R.lda, R.n, k, w,
                     R.top, R.dinvU + blk * NB * NB);
  FOSB_LAUNCH_CHECK();
}

template <typename T>
static void rec_lu(LuRun<T>& R, int64_t k, int64_t w) {
  if (w <= NB) {
    panel(R, k, (int)w);
    return;
  }
  const int64_t w1 = split_half(w);
  rec_lu(R, k, w1);
  cplx<T>* A = R.A;
  const int64_t lda = R.lda;
  trsm_lower_unit<T>(*R.ctx, A, lda, R.dinvL, k, w1, A + k * lda + (k + w1), lda, w - w1);
  gemm<T>(*R.ctx, R.n - k - w1, w - w1, w1, -1.0, A + (k + w1) * lda + k, lda, A + k * lda + (k + w1), lda,
          1.0, A + (k + w1) * lda + (k + w1), lda);
  rec_lu(R, k + w1, w - w1);
}

template <typename T>
int64_t lu_factor(Context& ctx, cplx<T>* A, int64_t n, int64_t lda, cplx<T>* dinvL, cplx<T>* dinvU,
                  std::vector<int32_t>& perm) {
  hipStream_t s = ctx.stream;
  const int64_t maxblk = (n + RB - 1) / RB;
  const int64_t npanel = (n + NB - 1) / NB;
  // tournament-tree shape of every panel (rows n - k, k = p * NB)
  std::vector<int32_t> meta((size_t)npanel * kMetaStride, 0);
  std::vector<int32_t> nlev((size_t)npanel);
  for (int64_t p = 0; p < npanel; ++p) {
    const int64_t m = n - p * NB;
    std::vector<int32_t> sizes{(int32_t)((m + RB - 1) / RB)};
    while (sizes.back() > 1) sizes.push_back((sizes.back() + 1) / 2);
    if ((int)sizes.size() + 1 > kMetaStride / 2) fail(FOSB_E_UNSUPPORTED, "lu: matrix too large");
    int32_t off = 0;
    for (size_t l = 0; l < sizes.size(); ++l) {
      meta[p * kMetaStride + l] = off;
      meta[p * kMetaStride + kMetaStride / 2 + l] = sizes[l];
      off += sizes[l];
    }
    meta[p * kMetaStride + sizes.size()] = off;
    nlev[p] = (int32_t)sizes.size();
  }
  const int64_t nodes = 2 * maxblk + 8;
  ctx.counters.reserve(nodes * sizeof(int32_t));
  FOSB_HIP(hipMemsetAsync(ctx.counters.p, 0, nodes * sizeof(int32_t), s));
  const size_t n_i32 = (size_t)(nodes * NB + meta.size() + (1 + 4 * NB) + n + 1);
  const size_t top_off = (n_i32 * sizeof(int32_t) + 255) / 256 * 256;
  ctx.small.reserve(top_off + NB * NB * sizeof(cplx<T>));
  int32_t* base = ctx.small.as<int32_t>();
  LuRun<T> R;
  R.ctx = &ctx;
  R.A = A;
  R.n = n;
  R.lda = lda;
  R.dinvL = dinvL;
  R.dinvU = dinvU;
  R.pw.cand = base;
  R.pw.counters = ctx.counters.as<int32_t>();
  int32_t* dmeta = base + nodes * NB;
  R.dmeta = dmeta;
  R.nlevels = nlev;
  R.pw.plist = dmeta + meta.size();
  R.pw.ipiv = R.pw.plist + (1 + 4 * NB);
  R.pw.info = R.pw.ipiv + n;
  R.top = reinterpret_cast<cplx<T>*>(reinterpret_cast<char*>(base) + top_off);
  FOSB_HIP(hipMemcpyAsync(dmeta, meta.data(), meta.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  FOSB_HIP(hipMemsetAsync(R.pw.info, 0, sizeof(int32_t), s));
  rec_lu(R, 0, n);
  std::vector<int32_t> ipiv(n);
  int32_t info = 0;
  FOSB_HIP(hipMemcpyAsync(ipiv.data(), R.pw.ipiv, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipMemcpyAsync(&info, R.pw.info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipStreamSynchronize(s));
  perm.resize(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t r = 0; r < n; ++r) {
    const int32_t p = ipiv[r];
    if (p < 0 || p >= n) fail(FOSB_E_DEVICE, "lu: invalid pivot index %d at row %lld", p, (long long)r);
    std::swap(perm[r], perm[p]);
  }
  return info;  // 0, or 1-based index of the first exactly zero pivot
}

template <typename T>
void trsm_lower_unit(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvL, int64_t k0, int64_t n,
                     cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NB) {
    ProfScope prof(ctx, FOSB_K_TRSM_LEAF, 8.0 * n * n * nrhs, 2.0 * sizeof(cplx<T>) * n * nrhs);
    hipLaunchKernelGGL(k_apply_inv<T>, dim3((unsigned)((nrhs + 63) / 64)), dim3(256), 0, ctx.stream,
                       dinvL + (k0 / NB) * NB * NB, (int)n, B, ldb, nrhs);
    FOSB_LAUNCH_CHECK();
    return;
  }
  const int64_t n1 = split_half(n);
  trsm_lower_unit<T>(ctx, A, lda, dinvL, k0, n1, B, ldb, nrhs);
  gemm<T>(ctx, n - n1, nrhs, n1, -1.0, A + (k0 + n1) * lda + k0, lda, B, ldb, 1.0, B + n1 * ldb, ldb);
  trsm_lower_unit<T>(ctx, A, lda, dinvL, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
}

template <typename T>
void trsm_upper(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvU, int64_t k0, int64_t n,
                cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NB) {
    ProfScope prof(ctx, FOSB_K_TRSM_LEAF, 8.0 * n * n * nrhs, 2.0 * sizeof(cplx<T>) * n * nrhs);
    hipLaunchKernelGGL(k_apply_inv<T>, dim3((unsigned)((nrhs + 63) / 64)), dim3(256), 0, ctx.stream,
                       dinvU + (k0 / NB) * NB * NB, (int)n, B, ldb, nrhs);
    FOSB_LAUNCH_CHECK();
    return;
  }
  const int64_t n1 = split_half(n);
  trsm_upper<T>(ctx, A, lda, dinvU, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
  gemm<T>(ctx, n1, nrhs, n - n1, -1.0, A + k0 * lda + (k0 + n1), lda, B + n1 * ldb, ldb, 1.0, B, ldb);
  trsm_upper<T>(ctx, A, lda, dinvU, k0, n1, B, ldb, nrhs);
}

template int64_t lu_factor<double>(Context&, c128*, int64_t, int64_t, c128*, c128*, std::vector<int32_t>&);
template int64_t lu_factor<float>(Context&, c64*, int64_t, int64_t, c64*, c64*, std::vector<int32_t>&);
template void trsm_lower_unit<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*,
                                      int64_t, int64_t);
template void trsm_lower_unit<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
                                     int64_t);
template void trsm_upper<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*, int64_t,
                                 int64_t);
template void trsm_upper<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
                                int64_t);

// ------------------------------------------------------------------ element-wise helpers
template <typename S, typename D>
__global__ void k_copy2d(const cplx<S>* __restrict__ src, int64_t lds, cplx<D>* __restrict__ dst, int64_t ldd,
                         int64_t rows, int64_t cols) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  for (int64_t rr = r; rr < rows; rr += gridDim.y)
    if (c < cols) {
      const cplx<S> v = src[rr * lds + c];
      dst[rr * ldd + c] = cplx<D>{(D)v.re, (D)v.im};
    }
}

template <typename S, typename D>
static void copy2d(hipStream_t s, const cplx<S>* src, int64_t lds, cplx<D>* dst, int64_t ldd, int64_t rows,
                   int64_t cols) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g((unsigned)((cols + 255) / 256), (unsigned)std::min<int64_t>(rows, 65535));
  hipLaunchKernelGGL((k_copy2d<S, D>), g, dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  FOSB_LAUNCH_CHECK();
}

void copy_c128_to_c64(hipStream_t s, const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows,
                      int64_t cols) {
  copy2d<double, float>(s, src, lds, dst, ldd, rows, cols);
}
void copy_c64_to_c128(hipStream_t s, const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows,
                      int64_t cols) {
  copy2d<float, double>(s, src, lds, dst, ldd, rows, cols);
}
void copy_c128(hipStream_t s, const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int64_t cols) {
  copy2d<double, double>(s, src, lds, dst, ldd, rows, cols);
}

__global__ void k_gather_rows(const int32_t* __restrict__ perm, const c128* __restrict__ src, int64_t lds,
                              c128* __restrict__ dst, int64_t ldd, int64_t n, int64_t cols) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y)
    if (c < cols) dst[r * ldd + c] = src[(int64_t)perm[r] * lds + c];
}

void permute_rows_gather(hipStream_t s, const int32_t* perm, const c128* src, int64_t lds, c128* dst, int64_t ldd,
                         int64_t n, int64_t ncols) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g((unsigned)((ncols + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
  hipLaunchKernelGGL(k_gather_rows, g, dim3(256), 0, s, perm, src, lds, dst, ldd, n, ncols);
  FOSB_LAUNCH_CHECK();
}

// dst (cols x rows) = src^H (src rows x cols), 32x32 tiles through LDS
__global__ __launch_bounds__(256) void k_conj_transpose(const c128* __restrict__ src, int64_t lds,
                                                        c128* __restrict__ dst, int64_t ldd, int64_t rows,
                                                        int64_t cols) {
  __shared__ c128 t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int q = ty; q < 32; q += 8) {
    const int64_t r = r0 + q, c = c0 + tx;
    if (r < rows && c < cols) t[q][tx] = src[r * lds + c];
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int64_t r = c0 + q, c = r0 + tx;  // dst row = src col
    if (r < cols && c < rows) {
      const c128 v = t[tx][q];
      dst[r * ldd + c] = c128{v.re, -v.im};
    }
  }
}

void conj_transpose_c128(hipStream_t s, const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows,
                         int64_t cols) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_conj_transpose, g, dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  FOSB_LAUNCH_CHECK();
}

__global__ void k_axpy(const c128* __restrict__ x, int64_t ldx, c128* __restrict__ y, int64_t ldy, int64_t rows,
                       int64_t cols) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    if (c < cols) {
      const c128 a = x[r * ldx + c];
      c128 b = y[r * ldy + c];
      y[r * ldy + c] = c128{a.re + b.re, a.im + b.im};
    }
}

void axpy_c128(hipStream_t s, const c128* x, int64_t ldx, c128* y, int64_t ldy, int64_t rows, int64_t cols) {
  if (rows <= 0 || cols <= 0) return;
  dim3 g((unsigned)((cols + 255) / 256), (unsigned)std::min<int64_t>(rows, 65535));
  hipLaunchKernelGGL(k_axpy, g, dim3(256), 0, s, x, ldx, y, ldy, rows, cols);
  FOSB_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_norms2(const c128* __restrict__ x, int64_t ldx, const c128* __restrict__ y,
                                                int64_t ldy, int64_t rows, int64_t cols, double* out) {
  __shared__ double sx[256], sy[256];
  double ax = 0, ay = 0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    const c128 a = x[r * ldx + c], b = y[r * ldy + c];
    ax += a.re * a.re + a.im * a.im;
    ay += b.re * b.re + b.im * b.im;
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sx[threadIdx.x] += sx[threadIdx.x + o];
      sy[threadIdx.x] += sy[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(out, sx[0]);
    atomicAdd(out + 1, sy[0]);
  }
}

void norms2_c128(hipStream_t s, const c128* x, int64_t ldx, const c128* y, int64_t ldy, int64_t rows, int64_t cols,
                 double* out) {
  FOSB_HIP(hipMemsetAsync(out, 0, 2 * sizeof(double), s));
  if (rows <= 0 || cols <= 0) return;
  const int64_t total = rows * cols;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (total + 255) / 256);
  hipLaunchKernelGGL(k_norms2, dim3(blocks), dim3(256), 0, s, x, ldx, y, ldy, rows, cols, out);
  FOSB_LAUNCH_CHECK();
}

}  // namespace fosb
