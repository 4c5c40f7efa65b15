// Dense complex LU with row pivoting, triangular solves and small helpers.
//
// LU (P Z = L U, L unit lower, row-major storage): recursive column splitting
// (left half, TRSM of the right half's top rows, GEMM update of the rest,
// right half) down to 32-column panels.  A panel is factorised with
// tournament pivoting: each 256-row leaf of the panel runs Gaussian
// elimination with partial pivoting in registers and nominates 32 candidate
// rows; one launch per tree level then merges the candidates of up to eight
// children per node the same way, until a single root node chooses the 32
// pivot rows.  The pivot rows are moved into place across the panel's columns,
// the panel below the diagonal block becomes A21 U11^{-1}, and the inverses
// of the 32x32 diagonal blocks of L and U are kept for the triangular solves.
//
// Triangular solves are recursive as well: halves are coupled by a GEMM and
// the 256-row leaves solve with the stored 32x32 diagonal-block inverses.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace fosb {

constexpr int NB = kPanel;   // panel width (32)

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

// Tournament pivoting.  A tree node holds up to NODE candidate rows of the
// panel, one row per thread of a 4-wavefront workgroup, each row's w <= 32
// entries in registers.  Gaussian elimination with partial pivoting on the
// node picks, at step j, the largest |re|+|im| in column j among the rows not
// chosen yet, broadcasts that row through LDS and eliminates column j from the
// remaining rows; ties go to the lowest thread.  The step loop is unrolled,
// which keeps every register index constant; the row chosen at step j then
// holds row j of the node's L\U factors and writes it to lu[j][*] (LDS).
// Rows per tree node = threads per workgroup (one row per thread); a node
// merges NODE / NB children.  Wider nodes (512, 1024 rows: fewer tree levels)
// measured slower: the per-column barrier and key reduction grow with the
// number of waves; narrower ones (128 rows) too: one more tree level.
template <typename T> struct Node { static constexpr int size = 256; };

// The panel chain (tournament nodes, row moves, panel finish) and the
// triangular-solve leaves are latency-bound kernels that share compute units
// with the trailing update's GEMM waves.  They raise their waves' issue
// priority, so each SIMD issues their instructions ahead of the GEMM's.
__device__ __forceinline__ void raise_wave_priority() { __builtin_amdgcn_s_setprio(3); }

// Largest 32-bit value over the wavefront, returned to every lane: DPP
// exchanges within each row of 16 lanes (xor 1, xor 2, half-row mirror, row
// mirror), then the four row maxima through readlane.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));  // row_mirror
  unsigned m = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  m = max(m, (unsigned)__builtin_amdgcn_readlane((int)v, 16));
  m = max(m, (unsigned)__builtin_amdgcn_readlane((int)v, 32));
  m = max(m, (unsigned)__builtin_amdgcn_readlane((int)v, 48));
  return m;
}

// Pivot-search key of a candidate, a 32-bit value that orders like the
// modulus |re| + |im|: 1 for an exact zero, at least 2 for any nonzero entry,
// and 0 is left for rows that are not candidates.  Non-negative floating-point
// numbers order like their bit patterns.  FP32: the bits of the modulus plus
// one.  FP64: the upper 32 bits of the modulus (sign, exponent and 20 mantissa
// bits), so moduli that agree to 2^-20 tie (the lowest row wins, within that
// relative distance of the largest) and no nonzero modulus, however small or
// large, falls together with zero.
__device__ __forceinline__ unsigned pivot_key(cplx<float> v) {
  return (__float_as_uint(cabs1(v)) & 0x7fffffffu) + 1u;
}
__device__ __forceinline__ unsigned pivot_key(cplx<double> v) {
  const double m = cabs1(v);
  if (m == 0.0) return 1u;
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(m) >> 32) & 0x7fffffffu;
  return (hi < 1u ? 1u : hi) + 1u;
}

// 1/a for the panel's multipliers: FP32 through the hardware reciprocal with
// one Newton step (within an ulp or two of the exact quotient: partial
// pivoting needs no correctly rounded multipliers), FP64 by exact division.
__device__ __forceinline__ float rcp_nr(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return r * (2.0f - x * r);
}
__device__ __forceinline__ cplx<float> cinv_panel(cplx<float> a) {
  const float s = fabsf(a.re) + fabsf(a.im);
  if (s == 0.0f) return cplx<float>{0.0f, 0.0f};
  const float rs = rcp_nr(s);
  const float ar = a.re * rs, ai = a.im * rs;
  const float t = rcp_nr(ar * ar + ai * ai) * rs;
  return cplx<float>{ar * t, -ai * t};
}
__device__ __forceinline__ cplx<double> cinv_panel(cplx<double> a) { return cinv(a); }

// Partial-pivoting elimination of the node's rows (one row per thread, the
// row's NB columns in registers).  The step loop is unrolled, so column j is
// addressed statically and every row stays in place: a row chosen at step j
// then holds L[j][0..j) (its multipliers) followed by U[j][j..].  Per step:
// * every candidate forms its key and, speculatively, the reciprocal of its
//   entry in column j (off the critical path: it overlaps the reduction);
// * a wave maximum of the keys, and a ballot for the lowest lane holding it;
// * that lane publishes the key, its row and its reciprocal; one barrier;
// * every thread takes the largest of the wave keys (ties to the lowest
//   wave), reads that wave's row and reciprocal, and eliminates column j.
// Slots alternate between two buffers, so a wave entering step j+1 never
// overwrites a slot that another wave still reads at step j.
template <typename T, int NW>
__device__ __forceinline__ int gepp_node(cplx<T> (&a)[NB], bool valid, int nvalid, int w, int tid, int& step,
                                         cplx<T> (*prow)[NW][NB], cplx<T> (*pinv)[NW], cplx<T> (*lu)[NB + 1],
                                         unsigned (*skey)[NW]) {
  int zero_col = -1;
  const int steps = min(nvalid, w);
  const int lane = tid & 63, wave = tid >> 6;
  step = -1;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < steps) {  // uniform over the workgroup
      const int b = j & 1;
      const bool cand = valid && step < 0;
      const unsigned mine = cand ? pivot_key(a[j]) : 0u;
      const cplx<T> rinv = cinv_panel(a[j]);
      const unsigned wmax = wave_max_u32(mine);
      const unsigned long long hit = __ballot(mine != 0u && mine == wmax);
      const int wl = hit ? __ffsll((unsigned long long)hit) - 1 : -1;  // this wave's nominee
      if (lane == wl) {
        skey[b][wave] = wmax;
        pinv[b][wave] = rinv;
#pragma unroll
        for (int c = j & ~1; c < NB; ++c) prow[b][wave][c] = a[c];  // from an even column: 16-byte stores
      } else if (wl < 0 && lane == 0) {
        skey[b][wave] = 0u;
      }
      __syncthreads();
      unsigned key = 0u;
      int q = 0;
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const unsigned o = skey[b][v];
        if (o > key) {
          key = o;
          q = v;
        }
      }
      if (wave == q && lane == wl) step = j;
      const cplx<T> piv = prow[b][q][j];
      const cplx<T> pr = pinv[b][q];
      if (piv.re == T(0) && piv.im == T(0) && zero_col < 0) zero_col = j;
      if (cand && step < 0) {
        const cplx<T> l = cmul(a[j], pr);
        const T nlr = -l.re, nli = -l.im;
#pragma unroll
        for (int c = j + 1; c < NB; ++c) {
          const cplx<T> u = prow[b][q][c];
          a[c].re = fma(nlr, u.re, fma(l.im, u.im, a[c].re));  // a - (l.re u.re - l.im u.im)
          a[c].im = fma(nlr, u.im, fma(nli, u.re, a[c].im));   // a - (l.re u.im + l.im u.re)
        }
        a[j] = l;
      }
    }
  }
  if (step >= 0) {
#pragma unroll
    for (int c = 0; c < NB; ++c) lu[step][c] = a[c];
  }
  __syncthreads();
  return zero_col;
}

struct PanelOut {
  int32_t* moves;     // per panel: [0] = count, then pairs (src row, dst position), 1 + 4*NB ints
  int32_t* info;      // first zero pivot (1-based), 0 if none
};

template <typename T>
__device__ __forceinline__ void load_row(const cplx<T>* A, int64_t lda, int64_t col0, int w, int row,
                                         cplx<T> (&a)[NB]) {
#pragma unroll
  for (int c = 0; c < NB; ++c)
    a[c] = (row >= 0 && c < w) ? A[(int64_t)row * lda + col0 + c] : cplx<T>{T(0), T(0)};
}

// Root of the tournament: lu[][] holds L11 \ U11 of the chosen rows (in pivot
// order) and win[] their row indices.  Writes the top block, the inverses of
// both diagonal factors, the row moves and the first zero pivot.  Row moves: pivot r goes to position k + r; the
// rows that held positions k..k+wk-1 and are not pivots go, in increasing row
// order, to the positions the pivots below the block vacate (in increasing
// order).
template <typename T>
__device__ __forceinline__ void panel_root(cplx<T> (*tb)[NB + 1], const int* win, int wk, int w, int zc, int64_t k,
                                           int tid, int32_t* __restrict__ moves, int32_t* __restrict__ info,
                                           cplx<T>* __restrict__ top, cplx<T>* __restrict__ invL,
                                           cplx<T>* __restrict__ invU) {
  constexpr int NODE = Node<T>::size;
  __shared__ int inblk[NB];   // 1 if row k + r is itself a pivot
  __shared__ cplx<T> udinv[NB];   // 1 / U[i][i] for i < wk (FP32 back substitution)
  for (int e = tid; e < NB * NB; e += NODE) {
    const int r = e / NB, c = e % NB;
    if (r >= wk || c >= w) tb[r][c] = cplx<T>{T(0), T(0)};
  }
  if (tid < NB) inblk[tid] = 0;
  // the zero fill above leaves the diagonal entries i < wk (<= w) alone
  if (tid < NB) udinv[tid] = tid < wk ? cinv(tb[tid][tid]) : cplx<T>{T(0), T(0)};
  __syncthreads();
  if (tid < wk && win[tid] < k + wk) inblk[win[tid] - k] = 1;
  for (int e = tid; e < NB * NB; e += NODE) top[e] = tb[e / NB][e % NB];
  if (zc >= 0 && tid == 0) atomicMin(info, (int)(k + zc + 1));
  // Inverses of the diagonal factors (identity beyond wk; entries of U^{-1}
  // carry 1/U[i][i], zero for an exactly zero pivot).
  // FP32: one column per lane and no barrier.  Lane c of the first wavefront
  // solves L x = e_c by forward substitution while lane c of the second solves
  // U y = e_c by back substitution; the factor entries are broadcast reads of
  // the block in LDS.  FP64 keeps the Gauss-Jordan sweeps over the whole
  // workgroup below: its per-lane columns (128 registers of x alone) ran slower.
  static_assert(Node<T>::size >= 128, "the inverses take two wavefronts");
  if constexpr (sizeof(T) == 4) {
   if ((tid & 63) < NB && tid < 128) {
    const int c = tid & 63;
    const bool live = c < wk;
    cplx<T> x[NB];
    if (tid < 64) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        cplx<T> v{(i == c) ? T(1) : T(0), T(0)};
        if (live && i < wk) {
#pragma unroll
          for (int j = 0; j < i; ++j) {
            const cplx<T> l = tb[i][j];
            v.re -= l.re * x[j].re - l.im * x[j].im;
            v.im -= l.re * x[j].im + l.im * x[j].re;
          }
        }
        x[i] = v;
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) invL[i * NB + c] = x[i];
    } else {
#pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        cplx<T> v{(i == c) ? T(1) : T(0), T(0)};
        if (live && i < wk) {
#pragma unroll
          for (int j = i + 1; j < NB; ++j) {   // x[j] = 0 for j > c and for j >= wk
            const cplx<T> u = tb[i][j];
            v.re -= u.re * x[j].re - u.im * x[j].im;
            v.im -= u.re * x[j].im + u.im * x[j].re;
          }
          v = cmul(v, udinv[i]);
        }
        x[i] = v;
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) invU[i * NB + c] = x[i];
    }
  }
  } else {
  // Gauss-Jordan sweeps over the whole workgroup, one barrier per step: L X = I forward,
  // then U Y = I backward.  At backward step r every thread forms row r's
  // scaled entries Y[r][c] / U[r][r] (r <= c < wk) itself; the threads on row
  // r store them to invU (they are final), the others eliminate column r from
  // rows i < r with them.  Row r of Y is not read again after step r.
  __shared__ cplx<T> sx[NB][NB + 1];
  for (int e = tid; e < NB * NB; e += NODE) sx[e / NB][e % NB] = cplx<T>{(e / NB == e % NB) ? T(1) : T(0), T(0)};
  __syncthreads();
  for (int r = 0; r < wk; ++r) {
    // rows i > r: X[i][c] -= L[i][r] X[r][c], c <= r
    const int cols = r + 1, rows = wk - r - 1;
    for (int e = tid; e < rows * cols; e += NODE) {
      const int i = r + 1 + e / cols, c = e % cols;
      const cplx<T> l = tb[i][r], x = sx[r][c];
      sx[i][c].re -= l.re * x.re - l.im * x.im;
      sx[i][c].im -= l.re * x.im + l.im * x.re;
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += NODE) {  // each thread reads, then resets, its own entries
    invL[e] = sx[e / NB][e % NB];
    sx[e / NB][e % NB] = cplx<T>{(e / NB == e % NB) ? T(1) : T(0), T(0)};
  }
  __syncthreads();
  for (int r = wk - 1; r >= 0; --r) {
    // rows i < r: Y[i][c] -= U[i][r] (Y[r][c] / U[r][r]), c >= r
    const int cols = wk - r;
    const cplx<T> inv = cinv(tb[r][r]);
    for (int e = tid; e < (r + 1) * cols; e += NODE) {
      const int i = e / cols, c = r + e % cols;
      const cplx<T> x = cmul(sx[r][c], inv);
      if (i == r) {
        invU[r * NB + c] = x;
      } else {
        const cplx<T> u = tb[i][r];
        sx[i][c].re -= u.re * x.re - u.im * x.im;
        sx[i][c].im -= u.re * x.im + u.im * x.re;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += NODE) {
    const int r = e / NB, c = e % NB;
    if (r >= wk || c < r || c >= wk) invU[e] = cplx<T>{(r == c) ? T(1) : T(0), T(0)};  // the rest stored above
  }
  }
  // move list, built by the first wavefront (every thread reaches the barrier)
  __shared__ int vsorted[NB];
  const int lane = tid;  // meaningful for tid < 64 only
  bool vac = false;
  if (tid < 64) {
    vac = lane < wk && win[lane] >= k + wk;
    if (vac) {
      int rank_v = 0;
      for (int q = 0; q < wk; ++q)
        if (win[q] >= k + wk && win[q] < win[lane]) ++rank_v;
      vsorted[rank_v] = win[lane];
    }
  }
  __syncthreads();
  if (tid < 64) {
    // pivots: win[r] -> k + r
    const bool mv = lane < wk && win[lane] != k + lane;
    const unsigned long long m1 = __ballot(mv);
    const int n1 = __popcll(m1);
    if (mv) {
      const int b = __popcll(m1 & ((1ull << lane) - 1ull));
      moves[1 + 2 * b] = win[lane];
      moves[2 + 2 * b] = (int)(k + lane);
    }
    // displaced rows (positions k..k+wk-1 not holding a pivot), increasing order, to the vacated positions
    const bool disp = lane < wk && !inblk[lane];
    const unsigned long long md = __ballot(disp);
    if (disp) {
      const int rd = __popcll(md & ((1ull << lane) - 1ull));
      moves[1 + 2 * (n1 + rd)] = (int)(k + lane);
      moves[2 + 2 * (n1 + rd)] = vsorted[rd];
    }
    if (lane == 0) moves[0] = n1 + __popcll(md);
  }
}

// Tree node of the tournament over panel rows [k, n) x columns [k, k + w).
// Leaf nodes (cand_in == nullptr) take NODE consecutive rows; inner nodes take
// the candidates of up to FANIN children of the previous level.  Candidates
// of node p are written to cand_out[p*NB .. p*NB + NB) (-1 = none).
template <typename T, bool IS_ROOT>
__global__ __launch_bounds__(Node<T>::size) void k_tslu_node(const cplx<T>* __restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                    int w, const int32_t* __restrict__ cand_in, int n_in,
                                                    int32_t* __restrict__ cand_out,
                                                    int32_t* __restrict__ moves, int32_t* __restrict__ info,
                                                    cplx<T>* __restrict__ top, cplx<T>* __restrict__ invL,
                                                    cplx<T>* __restrict__ invU) {
  constexpr int NODE = Node<T>::size, NWAVE = NODE / 64, FANIN = NODE / NB;
  __shared__ __align__(16) cplx<T> prow[2][NWAVE][NB];
  __shared__ cplx<T> lu[NB][NB + 1];
  __shared__ int sidx[NODE];
  __shared__ int win[NB];
  __shared__ cplx<T> pinv[2][NWAVE];
  __shared__ unsigned skey[2][NWAVE];
  __shared__ int scnt[NWAVE];
  __shared__ int s_cnt;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  raise_wave_priority();
  int nvalid = 0;
  if (cand_in == nullptr) {
    nvalid = (int)min<int64_t>(NODE, n - k - (int64_t)p * NODE);
    if (tid < nvalid) sidx[tid] = (int)(k + (int64_t)p * NODE + tid);
  } else {
    // compact the children's candidate lists (ids >= 0) in order: ballot per wave, prefix over waves
    const int c0 = p * FANIN;
    const int nch = min(FANIN, n_in - c0);
    const int id = tid < nch * NB ? cand_in[(int64_t)c0 * NB + tid] : -1;
    const unsigned long long mask = __ballot(id >= 0);
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) scnt[wave] = __popcll(mask);
    __syncthreads();
    int off = 0;
    for (int q = 0; q < wave; ++q) off += scnt[q];
    if (id >= 0) sidx[off + __popcll(mask & ((1ull << lane) - 1ull))] = id;
    if (tid == 0) {
      int tot = 0;
      for (int q = 0; q < NWAVE; ++q) tot += scnt[q];
      s_cnt = tot;
    }
    __syncthreads();
    nvalid = s_cnt;
  }
  __syncthreads();
  const bool valid = tid < nvalid;
  const int row = valid ? sidx[tid] : -1;
  cplx<T> a[NB];
  load_row(A, lda, k, w, row, a);
  int step;
  const int zc = gepp_node(a, valid, nvalid, w, tid, step, prow, pinv, lu, skey);
  const int ncand = min(nvalid, w);
  if constexpr (IS_ROOT) {
    if (step >= 0) win[step] = row;
    __syncthreads();
    panel_root(lu, win, ncand, w, zc, k, tid, moves, info, top, invL, invU);
    return;
  }
  int32_t* out = cand_out + (int64_t)p * NB;
  if (step >= 0) out[step] = row;
  if (tid >= ncand && tid < NB) out[tid] = -1;
}

// Value of lane l of the wavefront (l uniform), through the scalar unit.
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Panel without pivoting (the symmetric factorisation below): LU of the
// panel's top w x w block with the pivots in place, and the same outputs as a
// tournament root (top block, inverses of both diagonal factors, an empty
// row-move list, the first exactly zero pivot).  The first wavefront factors
// the block in registers, lane r holding row r; at step j every lane takes
// row j's entries from lane j (row j is final once step j starts).
template <typename T>
__global__ __launch_bounds__(Node<T>::size) void k_nopiv_root(const cplx<T>* __restrict__ A, int64_t lda, int64_t k,
                                                              int w, int32_t* __restrict__ moves,
                                                              int32_t* __restrict__ info, cplx<T>* __restrict__ top,
                                                              cplx<T>* __restrict__ invL, cplx<T>* __restrict__ invU) {
  __shared__ cplx<T> lu[NB][NB + 1];
  __shared__ int win[NB];
  __shared__ int szc;
  const int tid = threadIdx.x;
  raise_wave_priority();
  if (tid < NB) win[tid] = (int)(k + tid);
  if (tid < 64) {
    const int r = tid;
    const bool row = r < w;
    cplx<T> a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) a[c] = (row && c < w) ? A[(k + r) * lda + k + c] : cplx<T>{T(0), T(0)};
    int zc = -1;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < w) {
        const cplx<T> p{lane_value(a[j].re, j), lane_value(a[j].im, j)};
        if (zc < 0 && p.re == T(0) && p.im == T(0)) zc = j;
        // the multiplier, zero on the rows at and above the pivot (their
        // entries then stay as they are); cinv_panel(0) = 0: an exactly zero
        // pivot is reported through info
        const bool below = row && r > j;
        const cplx<T> l = below ? cmul(a[j], cinv_panel(p)) : cplx<T>{T(0), T(0)};
        if (below) a[j] = l;
#pragma unroll
        for (int c = j + 1; c < NB; ++c) {
          const cplx<T> u{lane_value(a[c].re, j), lane_value(a[c].im, j)};
          a[c].re -= l.re * u.re - l.im * u.im;
          a[c].im -= l.re * u.im + l.im * u.re;
        }
      }
    }
    if (r < NB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) lu[r][c] = a[c];
    }
    if (tid == 0) szc = zc;
  }
  __syncthreads();
  const int zc = szc;
  panel_root(lu, win, w, w, zc, k, tid, moves, info, top, invL, invU);
}

// U12 = D L21^T for a symmetric factorisation without pivoting: rows
// kj .. kj + wj of columns c0 .. c0 + cn receive d_t A[c][kj + t], d_t the
// diagonal of U in the block's diagonal square (32 x 32 tiles through LDS).
template <typename T>
__global__ __launch_bounds__(256) void k_sym_u12(cplx<T>* __restrict__ A, int64_t lda, int64_t kj, int64_t wj,
                                                 int64_t c0, int64_t cn) {
  __shared__ cplx<T> tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t t0 = (int64_t)blockIdx.y * 32, cb = c0 + (int64_t)blockIdx.x * 32;
  for (int r = ty; r < 32; r += 8) {   // read rows c = cb + r, columns kj + t0 + tx (the multipliers)
    const int64_t c = cb + r, t = t0 + tx;
    tile[r][tx] = (c < c0 + cn && t < wj) ? A[c * lda + kj + t] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {   // write rows kj + t, t = t0 + r, columns cb + tx
    const int64_t t = t0 + r, c = cb + tx;
    if (t < wj && c < c0 + cn) {
      const cplx<T> d = A[(kj + t) * lda + kj + t];
      const cplx<T> l = tile[tx][r];
      A[(kj + t) * lda + c] = cplx<T>{d.re * l.re - d.im * l.im, d.re * l.im + d.im * l.re};
    }
  }
}

template <typename T>
static void sym_u12(hipStream_t s, cplx<T>* A, int64_t lda, int64_t kj, int64_t wj, int64_t c0, int64_t cn) {
  if (wj <= 0 || cn <= 0) return;
  dim3 g((unsigned)((cn + 31) / 32), (unsigned)((wj + 31) / 32));
  hipLaunchKernelGGL(k_sym_u12<T>, g, dim3(256), 0, s, A, lda, kj, wj, c0, cn);
  FOSB_LAUNCH_CHECK();
}

// |v| rounded to float; a non-finite magnitude (NaN included) becomes +inf, so
// that the maxima below report it
template <typename T>
__device__ __forceinline__ float mag_or_inf(T re, T im) {
  const float f = (float)sqrt((double)re * re + (double)im * im);
  return f <= 3.402823466e38f ? f : __builtin_inff();
}

// Symmetry check of a square matrix in one pass: out[0] receives the largest
// |A[i][j] - A[j][i]| and out[1] the largest |A[i][j]|, as float bits folded
// with atomicMax (non-negative floats order like their bit patterns, and a
// maximum does not depend on the order).  Workgroups stride over the 32 x 32
// tile pairs (bi >= bj) of the lower triangle; the mirrored tile goes through
// LDS, both tiles are read row-wise, and each workgroup reduces its maxima
// before one atomic per output.
template <typename T>
__global__ __launch_bounds__(256) void k_sym_check(const cplx<T>* __restrict__ A, int64_t lda, int64_t n,
                                                   unsigned* __restrict__ out) {
  __shared__ cplx<T> tile[32][33];
  __shared__ float red[2][4];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t nb = (n + 31) / 32, npairs = nb * (nb + 1) / 2;
  float md = 0.f, ma = 0.f;
  for (int64_t t = blockIdx.x; t < npairs; t += gridDim.x) {
    int64_t bi = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int64_t bj = t - bi * (bi + 1) / 2;
    __syncthreads();   // the previous pair's reads of the tile are done
    for (int r = ty; r < 32; r += 8) {
      const int64_t i = bj * 32 + r, j = bi * 32 + tx;   // the mirrored tile, row-major
      const cplx<T> v = (i < n && j < n) ? A[i * lda + j] : cplx<T>{T(0), T(0)};
      tile[r][tx] = v;
      ma = fmaxf(ma, mag_or_inf(v.re, v.im));
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t i = bi * 32 + r, j = bj * 32 + tx;
      if (i < n && j < n) {
        const cplx<T> a = A[i * lda + j], b = tile[tx][r];
        md = fmaxf(md, mag_or_inf((double)a.re - (double)b.re, (double)a.im - (double)b.im));
        ma = fmaxf(ma, mag_or_inf(a.re, a.im));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    md = fmaxf(md, __shfl_xor(md, o, 64));
    ma = fmaxf(ma, __shfl_xor(ma, o, 64));
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = md;
    red[1][wave] = ma;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const float m = fmaxf(fmaxf(red[threadIdx.x][0], red[threadIdx.x][1]), fmaxf(red[threadIdx.x][2], red[threadIdx.x][3]));
    atomicMax(out + threadIdx.x, __float_as_uint(m));
  }
}

// Largest |A[i][j]| over the upper triangle (j >= i) into *out (float bits,
// atomicMax): workgroups stride over the rows, their threads along a row.
template <typename T>
__global__ __launch_bounds__(256) void k_absmax_upper(const cplx<T>* __restrict__ A, int64_t lda, int64_t n,
                                                      unsigned* __restrict__ out) {
  __shared__ float red[4];
  float m = 0.f;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
    for (int64_t j = i + threadIdx.x; j < n; j += 256) {
      const cplx<T> v = A[i * lda + j];
      m = fmaxf(m, mag_or_inf(v.re, v.im));
    }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
}

// Apply npl consecutive row-move lists (list q at plist + q * kMoveStride, in
// order) to the columns of up to two ranges [c0[r], c1[r]), in stripes of 64.
struct ColRanges {
  int64_t c0[2], c1[2];
};
constexpr int kMoveStrideDev = 1 + 4 * NB;

template <typename T>
__global__ __launch_bounds__(256) void k_permute_rows(cplx<T>* __restrict__ A, int64_t lda, ColRanges cr,
                                                      const int32_t* __restrict__ plist, int npl) {
  __shared__ cplx<T> buf[2 * NB][64];
  raise_wave_priority();
  const int64_t w0 = cr.c1[0] - cr.c0[0];
  const int64_t x = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t c = x < w0 ? cr.c0[0] + x : cr.c0[1] + (x - w0);
  const bool live = x < w0 || (c < cr.c1[1]);
  const int g = threadIdx.x >> 6;
  for (int q = 0; q < npl; ++q) {
    const int32_t* pl = plist + (int64_t)q * kMoveStrideDev;
    const int cnt = pl[0];
    if (live)
      for (int e = g; e < cnt; e += 4) buf[e][threadIdx.x & 63] = A[(int64_t)pl[1 + 2 * e] * lda + c];
    __syncthreads();
    if (live)
      for (int e = g; e < cnt; e += 4) A[(int64_t)pl[2 + 2 * e] * lda + c] = buf[e][threadIdx.x & 63];
    __syncthreads();
  }
}

// Write L11\U11 into the diagonal block and form A21 U11^{-1} below it; four
// threads per row, each producing eight of the row's 32 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_finish(cplx<T>* __restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                      int w, const cplx<T>* __restrict__ top,
                                                      const cplx<T>* __restrict__ invU) {
  __shared__ cplx<T> su[NB][NB + 1];
  raise_wave_priority();
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) su[e / NB][e % NB] = invU[e];
  const int64_t r = k + (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2);
  const int q = threadIdx.x & 3;
  cplx<T>* row = A + r * lda + k;
  cplx<T> a[NB];
  const bool live = r < n && r >= k + w;
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = (live && c < w) ? row[c] : cplx<T>{T(0), T(0)};
  __syncthreads();  // every thread has read its row before any is overwritten
  if (r >= n) return;
  if (r < k + w) {
    const int rr = (int)(r - k);
    for (int c = q; c < w; c += 4) row[c] = top[rr * NB + c];
    return;
  }
#pragma unroll
  for (int cc = 0; cc < NB / 4; ++cc) {
    const int c = q + 4 * cc;
    T xr = 0, xi = 0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t <= c) {
        const cplx<T> u = su[t][c];
        xr += a[t].re * u.re - a[t].im * u.im;
        xi += a[t].re * u.im + a[t].im * u.re;
      }
    }
    if (c < w) row[c] = cplx<T>{xr, xi};
  }
}

// Triangular solve on a diagonal block of up to NL rows in one launch:
// rows [k0, k0 + n) of B <- op(T)^{-1} B.  Without CONJT, T is the unit lower
// (LOWER) or upper factor stored in A; with CONJT, op(T) is the conjugate
// transpose of the upper (LOWER: U^H is lower) or unit lower factor (L^H).
// The 32x32 diagonal blocks are applied through their stored inverses
// ((T^H)^{-1} = (T^{-1})^H).  Each workgroup owns a stripe of CS right-hand sides
// held in LDS; after each diagonal block the coupling to the remaining rows
// of the leaf is subtracted with the off-diagonal factor entries.
constexpr int NL = 256;
template <typename T> struct LeafCS { static constexpr int v = 16; };
template <> struct LeafCS<double> { static constexpr int v = 8; };

template <typename T, bool LOWER, int CS, bool CONJT>
__device__ __forceinline__ void trsm_leaf_body(const cplx<T>* __restrict__ A, int64_t lda,
                                               const cplx<T>* __restrict__ dinv, int64_t k0, int n,
                                               cplx<T>* __restrict__ B, int64_t ldb, int64_t nrhs, int64_t c0) {
  constexpr int XPT = (NB * CS + 255) / 256;
  raise_wave_priority();
  __shared__ cplx<T> sb[NL][CS + 1];
  __shared__ cplx<T> si[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < NL * CS; e += 256) {  // rows >= n are zero (they meet zero factor entries)
    const int r = e / CS, c = e % CS;
    sb[r][c] = (r < n && c0 + c < nrhs) ? B[(int64_t)r * ldb + c0 + c] : cplx<T>{T(0), T(0)};
  }
  const int nblk = (n + NB - 1) / NB;
  for (int bi = 0; bi < nblk; ++bi) {
    const int b = LOWER ? bi : nblk - 1 - bi;
    const int r0 = b * NB, rn = min(NB, n - r0);
    __syncthreads();
    const cplx<T>* inv = dinv + (k0 / NB + b) * NB * NB;
    for (int e = tid; e < NB * NB; e += 256) {
      if (CONJT) {
        const cplx<T> v = inv[(e % NB) * NB + e / NB];
        si[e / NB][e % NB] = cplx<T>{v.re, -v.im};
      } else {
        si[e / NB][e % NB] = inv[e];
      }
    }
    __syncthreads();
    cplx<T> xv[XPT];
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int e = tid + 256 * q;
      T xr = 0, xi = 0;
      if (e < rn * CS) {
        const int r = e / CS, c = e % CS;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          if (t < rn) {
            const cplx<T> u = si[r][t], v = sb[r0 + t][c];
            xr += u.re * v.re - u.im * v.im;
            xi += u.re * v.im + u.im * v.re;
          }
        }
      }
      xv[q] = cplx<T>{xr, xi};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int e = tid + 256 * q;
      if (e < rn * CS) sb[r0 + e / CS][e % CS] = xv[q];
    }
    __syncthreads();
    const int u0 = LOWER ? r0 + rn : 0;
    const int u1 = LOWER ? n : r0;
    if (tid >= u0 && tid < u1) {  // one thread per remaining row: its factor segment once, all CS columns
      cplx<T> l[NB];
      if (CONJT) {  // column tid of the stored factor, rows r0 .. r0 + rn: coalesced across the wave
        const cplx<T>* acol = A + (k0 + r0) * lda + k0 + tid;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const cplx<T> v = t < rn ? acol[(int64_t)t * lda] : cplx<T>{T(0), T(0)};
          l[t] = cplx<T>{v.re, -v.im};
        }
      } else {
        const cplx<T>* arow = A + (k0 + tid) * lda + k0 + r0;
#pragma unroll
        for (int t = 0; t < NB; ++t) l[t] = t < rn ? arow[t] : cplx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int c = 0; c < CS; ++c) {
        T xr = 0, xi = 0;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const cplx<T> v = sb[r0 + t][c];
          xr += l[t].re * v.re - l[t].im * v.im;
          xi += l[t].re * v.im + l[t].im * v.re;
        }
        sb[tid][c].re -= xr;
        sb[tid][c].im -= xi;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < n * CS; e += 256) {
    const int r = e / CS, c = e % CS;
    if (c0 + c < nrhs) B[(int64_t)r * ldb + c0 + c] = sb[r][c];
  }
}

template <typename T, bool LOWER, int CS, bool CONJT>
__global__ __launch_bounds__(256) void k_trsm_leaf(const cplx<T>* __restrict__ A, int64_t lda,
                                                   const cplx<T>* __restrict__ dinv, int64_t k0, int n,
                                                   cplx<T>* __restrict__ B, int64_t ldb, int64_t nrhs) {
  trsm_leaf_body<T, LOWER, CS, CONJT>(A, lda, dinv, k0, n, B, ldb, nrhs, (int64_t)blockIdx.x * CS);
}

// Inverses of NL x NL diagonal blocks of an n x n factor in one launch: block
// b = b0 + blockIdx.y (rows and columns b NL .. b NL + NL) is solved against
// its own identity block, W + b NL^2 (NL x NL, row stride NL), in stripes of CS
// columns.  The last block may be smaller; its slot keeps the identity outside
// its nb x nb corner.
template <typename T, bool LOWER, int CS>
__global__ __launch_bounds__(256) void k_trsm_leaf_blocks(const cplx<T>* __restrict__ A, int64_t lda,
                                                          const cplx<T>* __restrict__ dinv, int64_t n,
                                                          cplx<T>* __restrict__ W, int64_t b0) {
  const int64_t b = b0 + blockIdx.y, k0 = b * NL;
  const int nb = (int)min<int64_t>(NL, n - k0);
  trsm_leaf_body<T, LOWER, CS, false>(A, lda, dinv, k0, nb, W + b * NL * NL, NL, nb, (int64_t)blockIdx.x * CS);
}

template <typename T>
__global__ void k_identity_blocks(cplx<T>* __restrict__ W, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int r = (int)((i / NL) % NL), c = (int)(i % NL);
  W[i] = cplx<T>{r == c ? T(1) : T(0), T(0)};
}

// Inverses of diagonal blocks b0 .. b0 + nbk of the unit lower (LOWER) or
// upper factor into W (block b at W + b NL^2), on ctx's stream.
template <typename T, bool LOWER>
static void block_inverses(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, const cplx<T>* dinv,
                           cplx<T>* W, int64_t b0, int64_t nbk) {
  if (nbk <= 0) return;
  hipStream_t s = ctx.stream;
  constexpr int CS = LeafCS<T>::v;
  const int64_t count = nbk * NL * NL;
  hipLaunchKernelGGL(k_identity_blocks<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     W + b0 * NL * NL, count);
  FOSB_LAUNCH_CHECK();
  ProfScope prof(ctx, FOSB_K_TRSM_LEAF, 4.0 * NL * NL * (double)std::min(n, nbk * NL),
                 2.0 * sizeof(cplx<T>) * NL * (double)std::min(n, nbk * NL));
  hipLaunchKernelGGL((k_trsm_leaf_blocks<T, LOWER, CS>), dim3((unsigned)(NL / CS), (unsigned)nbk), dim3(256), 0, s,
                     A, lda, dinv, n, W, b0);
  FOSB_LAUNCH_CHECK();
}

// One right-hand side per workgroup (the stripe the launcher picks for narrow
// solves, e.g. a first moment or a pair with a coarse partner level): the same
// block steps as k_trsm_leaf, software-pipelined.
// Each step's loads of the next block's inverse and of the row's next factor
// segment are issued into registers before the step computes, so that the
// step's dependent global loads are off the critical chain.
template <typename T, bool LOWER, bool CONJT>
__global__ __launch_bounds__(256) void k_trsm_leaf1(const cplx<T>* __restrict__ A, int64_t lda,
                                                    const cplx<T>* __restrict__ dinv, int64_t k0, int n,
                                                    cplx<T>* __restrict__ B, int64_t ldb, int64_t nrhs) {
  static_assert(NL == 256, "one row per thread");
  constexpr int IPT = NB * NB / 256;  // inverse entries staged per thread
  raise_wave_priority();
  __shared__ cplx<T> sb[NL];
  __shared__ cplx<T> si[NB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x;
  sb[tid] = (tid < n && c < nrhs) ? B[(int64_t)tid * ldb + c] : cplx<T>{T(0), T(0)};
  const int nblk = (n + NB - 1) / NB;
  cplx<T> invn[IPT], ln[NB];
  auto fetch = [&](int bi) {  // the inverse and this row's factor segment for step bi
    const int b = LOWER ? bi : nblk - 1 - bi;
    const int r0 = b * NB, rn = min(NB, n - r0);
    const cplx<T>* inv = dinv + (k0 / NB + b) * NB * NB;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const int e = tid + 256 * q;
      if (CONJT) {
        const cplx<T> v = inv[(e % NB) * NB + e / NB];
        invn[q] = cplx<T>{v.re, -v.im};
      } else {
        invn[q] = inv[e];
      }
    }
    const int u0 = LOWER ? r0 + rn : 0, u1 = LOWER ? n : r0;
    if (tid >= u0 && tid < u1) {
      if (CONJT) {  // column tid of the stored factor
        const cplx<T>* acol = A + (k0 + r0) * lda + k0 + tid;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const cplx<T> v = t < rn ? acol[(int64_t)t * lda] : cplx<T>{T(0), T(0)};
          ln[t] = cplx<T>{v.re, -v.im};
        }
      } else {
        const cplx<T>* arow = A + (k0 + tid) * lda + k0 + r0;
#pragma unroll
        for (int t = 0; t < NB; ++t) ln[t] = t < rn ? arow[t] : cplx<T>{T(0), T(0)};
      }
    }
  };
  fetch(0);
  for (int bi = 0; bi < nblk; ++bi) {
    const int b = LOWER ? bi : nblk - 1 - bi;
    const int r0 = b * NB, rn = min(NB, n - r0);
    const int u0 = LOWER ? r0 + rn : 0, u1 = LOWER ? n : r0;
    const bool upd = tid >= u0 && tid < u1;
    cplx<T> l[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) l[t] = ln[t];
    // si was last read before the previous step's second barrier
#pragma unroll
    for (int q = 0; q < IPT; ++q) si[(tid + 256 * q) / NB][(tid + 256 * q) % NB] = invn[q];
    if (bi + 1 < nblk) fetch(bi + 1);
    __syncthreads();
    T xr = 0, xi = 0;
    if (tid < rn) {
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < rn) {
          const cplx<T> u = si[tid][t], v = sb[r0 + t];
          xr += u.re * v.re - u.im * v.im;
          xi += u.re * v.im + u.im * v.re;
        }
      }
    }
    __syncthreads();
    if (tid < rn) sb[r0 + tid] = cplx<T>{xr, xi};
    __syncthreads();
    if (upd) {
      T ur = 0, ui = 0;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const cplx<T> v = sb[r0 + t];
        ur += l[t].re * v.re - l[t].im * v.im;
        ui += l[t].re * v.im + l[t].im * v.re;
      }
      sb[tid].re -= ur;
      sb[tid].im -= ui;
    }
  }
  __syncthreads();
  if (tid < n && c < nrhs) B[(int64_t)tid * ldb + c] = sb[tid];
}

// ------------------------------------------------------------------ host drivers
template <typename T>
struct LuRun {
  Context* ctx;
  cplx<T>* A;
  int64_t n, lda;
  cplx<T>* dinvL;
  cplx<T>* dinvU;
  int32_t* moves;  // per panel: 1 + 4*NB ints
  int32_t* info;
  int32_t* cand;   // two candidate buffers (ping-pong), each cand_stride ints
  int64_t cand_stride;
  cplx<T>* top;
  int64_t pc0, pc1;  // columns a panel permutes at once (the rest is the update stream's)
  cplx<T>* invL = nullptr;  // optional: NL x NL diagonal-block inverses of L, filled per block
  bool sym = false;         // symmetric matrix, no pivoting: lower-triangle trailing updates, U12 = D L21^T
};

constexpr int kMoveStride = 1 + 4 * NB;
static_assert(kMoveStride == kMoveStrideDev, "row-move list stride");
constexpr int64_t kLookaheadMinN = 2048;  // smaller matrices: plain recursion on one stream
constexpr int64_t kTrailChunk = 16384;     // columns per trailing-update launch (measured: 2048..16384)
constexpr int64_t kSymChunk = 2048;        // symmetric form: its rows start at the chunk, so narrower chunks waste less

static inline int64_t split_half(int64_t w) { return (int64_t)NB * (((w / NB) + 1) / 2); }

template <typename T>
static void panel(LuRun<T>& R, int64_t k, int w) {
  hipStream_t s = R.ctx->stream;
  const int64_t m = R.n - k;
  const int64_t blk = k / NB;
  int32_t* moves = R.moves + blk * kMoveStride;
  ProfScope prof(*R.ctx, FOSB_K_PANEL, 0.0, (double)sizeof(cplx<T>) * (double)m * w * 3.0);
  if (R.sym) {  // pivots in place: factor the top block, then the multipliers below it
    hipLaunchKernelGGL(k_nopiv_root<T>, dim3(1), dim3(Node<T>::size), 0, s, R.A, R.lda, k, w, moves, R.info, R.top,
                       R.dinvL + blk * NB * NB, R.dinvU + blk * NB * NB);
    FOSB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_panel_finish<T>, dim3((unsigned)((m + 63) / 64)), dim3(256), 0, s, R.A, R.lda, R.n, k, w,
                       R.top, R.dinvU + blk * NB * NB);
    FOSB_LAUNCH_CHECK();
    return;
  }
  // leaf level over consecutive rows, then FANIN-way merges until one node remains
  constexpr int NODE = Node<T>::size, FANIN = NODE / NB;
  int nodes = (int)((m + NODE - 1) / NODE);
  int32_t* cin = R.cand;
  int32_t* cout = R.cand + R.cand_stride;
  bool root = nodes == 1;
  auto node = [&](int grid, const int32_t* in, int n_in, int32_t* out) {
    if (root)
      hipLaunchKernelGGL((k_tslu_node<T, true>), dim3(grid), dim3(NODE), 0, s, R.A, R.lda, R.n, k, w, in, n_in, out,
                         moves, R.info, R.top, R.dinvL + blk * NB * NB, R.dinvU + blk * NB * NB);
    else
      hipLaunchKernelGGL((k_tslu_node<T, false>), dim3(grid), dim3(NODE), 0, s, R.A, R.lda, R.n, k, w, in, n_in, out,
                         moves, R.info, R.top, R.dinvL + blk * NB * NB, R.dinvU + blk * NB * NB);
    FOSB_LAUNCH_CHECK();
  };
  node(nodes, nullptr, 0, cin);
  while (!root) {
    const int next = (nodes + FANIN - 1) / FANIN;
    root = next == 1;
    node(next, cin, nodes, cout);
    std::swap(cin, cout);
    nodes = next;
  }
  {
    ColRanges cr{{R.pc0, 0}, {R.pc1, 0}};
    hipLaunchKernelGGL(k_permute_rows<T>, dim3((unsigned)((R.pc1 - R.pc0 + 63) / 64)), dim3(256), 0, s, R.A, R.lda,
                       cr, moves, 1);
  }
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_panel_finish<T>, dim3((unsigned)((m + 63) / 64)), dim3(256), 0, s, R.A, R.lda, R.n, k, w,
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
  gemm<T>(*R.ctx, R.n - k - w1, w - w1, w1, -1.0, A + (k + w1) * lda + k, lda, A + k * lda + (k + w1), lda, 1.0,
          A + (k + w1) * lda + (k + w1), lda);
  rec_lu(R, k + w1, w - w1);
}

// Right-looking blocked LU with a lookahead of one block column, over two
// streams.  The panel stream (the context's) factors block column j with the
// recursion above, restricted to its own columns (its row moves touch only
// those columns).  The update stream (a child context with its own scratch)
// applies block j's row moves to every other column, solves and updates block
// column j+1 first, lets the panel stream start on it, and then updates the
// remaining columns while that panel is being factored.  The two streams never
// touch the same columns concurrently: the panel of block j+1 reads and writes
// only block j+1, the trailing update of step j only columns right of it, and
// block j's multipliers are permuted by the update stream after its last read.
template <typename T, bool LOWER>
static void trsm_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* inv, int64_t k0, int64_t n,
                     cplx<T>* B, int64_t ldb, int64_t nrhs, cplx<T>* tmp);

// B <- L_jj^{-1} B for the block row of block j (rows kj .. kj + wj): through
// the block inverses when the run keeps them (they are final once block j's
// panels are done), else with the leaf kernel.
template <typename T>
static void block_row_solve(LuRun<T>& R, Context& U, int64_t kj, int64_t wj, cplx<T>* B, int64_t ncols) {
  if (R.invL) {
    U.solve_tmp.reserve((size_t)NL * ncols * sizeof(cplx<T>));
    trsm_inv<T, true>(U, R.A, R.lda, R.invL, kj, wj, B, R.lda, ncols, U.solve_tmp.as<cplx<T>>());
  } else {
    trsm_lower_unit<T>(U, R.A, R.lda, R.dinvL, kj, wj, B, R.lda, ncols);
  }
}

template <typename T>
static void blocked_lu(LuRun<T>& R, Context& U, int64_t nb) {
  Context& P = *R.ctx;
  hipStream_t sa = P.stream, sb = U.stream;
  cplx<T>* A = R.A;
  const int64_t n = R.n, lda = R.lda;
  if (!P.lu_ev[0]) {
    FOSB_HIP(hipEventCreateWithFlags(&P.lu_ev[0], hipEventDisableTiming));
    FOSB_HIP(hipEventCreateWithFlags(&P.lu_ev[1], hipEventDisableTiming));
  }
  hipEvent_t ev_panel = P.lu_ev[0], ev_look = P.lu_ev[1];
  // the panel stream's GEMMs run beside the trailing update: small tiles, so a
  // workgroup fits where one of the update's workgroups has just retired
  struct Lean {
    Context& c;
    explicit Lean(Context& x) : c(x) { ++c.lean_tiles; }
    ~Lean() { --c.lean_tiles; }
  } lean(P);
  struct Update {
    Context& c;
    explicit Update(Context& x) : c(x) { ++c.trailing_update; }
    ~Update() { --c.trailing_update; }
  } update(U);
  auto panel_block = [&](int64_t k, int64_t w) {
    R.pc0 = k;
    R.pc1 = k + w;
    rec_lu(R, k, w);
    FOSB_HIP(hipEventRecord(ev_panel, sa));
  };
  panel_block(0, std::min(nb, n));
  const int64_t nblk = (n + nb - 1) / nb;
  const int64_t mark_blk = P.lu_mark_cb ? std::min<int64_t>(nblk - 1, (int64_t)(P.lu_mark_frac * (double)nblk)) : -1;
  for (int64_t j = 0; j < nblk; ++j) {
    const int64_t kj = j * nb, wj = std::min(nb, n - kj);
    if (j == mark_blk && P.lu_mark_cb) {
      FOSB_HIP(hipEventRecord(P.lu_mark_ev, sb));
      std::function<void()> cb = std::move(P.lu_mark_cb);
      P.lu_mark_cb = nullptr;
      cb();
    }
    FOSB_HIP(hipStreamWaitEvent(sb, ev_panel, 0));
    if (R.invL) block_inverses<T, true>(U, A, n, lda, R.dinvL, R.invL, kj / NL, (wj + NL - 1) / NL);
    if (!R.sym) {
      ColRanges cr{{0, kj + wj}, {kj, n}};
      const int64_t width = kj + (n - kj - wj);
      if (width > 0) {
        ProfScope prof(U, FOSB_K_PANEL, 0.0, 0.0);
        hipLaunchKernelGGL(k_permute_rows<T>, dim3((unsigned)((width + 63) / 64)), dim3(256), 0, sb, A, lda, cr,
                           R.moves + (kj / NB) * kMoveStride, (int)((wj + NB - 1) / NB));
        FOSB_LAUNCH_CHECK();
      }
    }
    if (j + 1 == nblk) break;
    const int64_t k1 = kj + wj, w1 = std::min(nb, n - k1);
    if (R.sym) {  // symmetric, no pivoting: U12 = D L21^T, trailing updates of the lower triangle only
      sym_u12<T>(sb, A, lda, kj, wj, k1, w1);
      gemm<T>(U, n - k1, w1, wj, -1.0, A + k1 * lda + kj, lda, A + kj * lda + k1, lda, 1.0, A + k1 * lda + k1, lda);
      FOSB_HIP(hipEventRecord(ev_look, sb));
      FOSB_HIP(hipStreamWaitEvent(sa, ev_look, 0));
      panel_block(k1, w1);
      // chunks of whole blocks (a block's diagonal square lies in one chunk, whose rows start at it)
      const int64_t chunk = std::max<int64_t>(nb, kSymChunk / nb * nb);
      for (int64_t c0 = k1 + w1; c0 < n; c0 += chunk) {
        const int64_t cn = std::min<int64_t>(chunk, n - c0);
        sym_u12<T>(sb, A, lda, kj, wj, c0, cn);
        gemm<T>(U, n - c0, cn, wj, -1.0, A + c0 * lda + kj, lda, A + kj * lda + c0, lda, 1.0, A + c0 * lda + c0, lda);
      }
      continue;
    }
    block_row_solve(R, U, kj, wj, A + kj * lda + k1, w1);
    gemm<T>(U, n - k1, w1, wj, -1.0, A + k1 * lda + kj, lda, A + kj * lda + k1, lda, 1.0, A + k1 * lda + k1, lda);
    FOSB_HIP(hipEventRecord(ev_look, sb));
    FOSB_HIP(hipStreamWaitEvent(sa, ev_look, 0));
    panel_block(k1, w1);
    if (k1 + w1 < n) {
      const int64_t kr = k1 + w1;
      // in column chunks: between two chunk launches the panel stream's small
      // kernels get workgroup slots instead of queueing behind one huge grid
      for (int64_t c0 = kr; c0 < n; c0 += kTrailChunk) {
        const int64_t cn = std::min<int64_t>(kTrailChunk, n - c0);
        block_row_solve(R, U, kj, wj, A + kj * lda + c0, cn);
        gemm<T>(U, n - k1, cn, wj, -1.0, A + k1 * lda + kj, lda, A + kj * lda + c0, lda, 1.0, A + k1 * lda + c0, lda);
      }
    }
  }
  FOSB_HIP(hipEventRecord(ev_look, sb));
  FOSB_HIP(hipStreamWaitEvent(sa, ev_look, 0));
}

__global__ void k_set_i32(int32_t* p, int32_t v) {
  if (threadIdx.x == 0) *p = v;
}

template <typename T>
int64_t lu_factor(Context& ctx, cplx<T>* A, int64_t n, int64_t lda, cplx<T>* dinvL, cplx<T>* dinvU,
                  std::vector<int32_t>& perm, cplx<T>* invL, bool sym) {
  hipStream_t s = ctx.stream;
  const int64_t maxnodes = (n + Node<T>::size - 1) / Node<T>::size;
  const int64_t npanel = (n + NB - 1) / NB;
  const size_t n_i32 = (size_t)(2 * maxnodes * NB + npanel * kMoveStride + 1);
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
  R.cand = base;
  R.cand_stride = maxnodes * NB;
  R.moves = base + 2 * maxnodes * NB;
  R.info = R.moves + npanel * kMoveStride;
  R.top = reinterpret_cast<cplx<T>*>(reinterpret_cast<char*>(base) + top_off);
  R.pc0 = 0;
  R.pc1 = n;
  R.invL = invL;
  R.sym = sym && n >= kLookaheadMinN;
  // first zero pivot, reduced with atomicMin: starts above every index (0x7f7f7f7f)
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, R.info, (int32_t)0x7f7f7f7f);
  FOSB_LAUNCH_CHECK();
  if (n >= kLookaheadMinN) {
    Context& U = ctx.la_context();
    // the update stream starts after everything already queued on the panel stream
    if (!ctx.lu_ev[0]) {
      FOSB_HIP(hipEventCreateWithFlags(&ctx.lu_ev[0], hipEventDisableTiming));
      FOSB_HIP(hipEventCreateWithFlags(&ctx.lu_ev[1], hipEventDisableTiming));
    }
    FOSB_HIP(hipEventRecord(ctx.lu_ev[1], s));
    FOSB_HIP(hipStreamWaitEvent(U.stream, ctx.lu_ev[1], 0));
    // block width: 768 from N = 16384 (measured at N = 30720: symmetric FP32
    // factorisation 0.325 -> 0.319 s, pivoted FP64 1.300 -> 1.293 s against 512;
    // 1024 gained nothing for the symmetric form)
    blocked_lu(R, U, n >= 16384 ? 768 : 256);
  } else {
    rec_lu(R, 0, n);
    if (invL) block_inverses<T, true>(ctx, A, n, lda, dinvL, invL, 0, (n + NL - 1) / NL);
  }
  std::vector<int32_t> mv((size_t)npanel * kMoveStride);
  int32_t info = 0;
  FOSB_HIP(hipMemcpyAsync(mv.data(), R.moves, mv.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipMemcpyAsync(&info, R.info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipStreamSynchronize(s));
  // replay the row moves of every panel: position i holds original row perm[i]
  perm.resize(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  std::vector<int32_t> src_rows;
  for (int64_t p = 0; p < npanel; ++p) {
    const int32_t* m = mv.data() + p * kMoveStride;
    const int cnt = m[0];
    if (cnt < 0 || cnt > 2 * NB) fail(FOSB_E_DEVICE, "lu: corrupt row-move list of panel %lld", (long long)p);
    src_rows.resize(cnt);
    for (int e = 0; e < cnt; ++e) {
      const int32_t a = m[1 + 2 * e], b = m[2 + 2 * e];
      if (a < 0 || a >= n || b < 0 || b >= n) fail(FOSB_E_DEVICE, "lu: invalid row move in panel %lld", (long long)p);
      src_rows[e] = perm[a];
    }
    for (int e = 0; e < cnt; ++e) perm[m[2 + 2 * e]] = src_rows[e];
  }
  if (info == 0x7f7f7f7f) info = 0;
  return info;  // 0, or 1-based index of the first exactly zero pivot
}

template <typename T, bool LOWER, int CS, bool CONJT>
static void trsm_leaf_go(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinv, int64_t k0, int64_t n,
                         cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if constexpr (CS == 1 && sizeof(T) == 4) {  // narrow solves: the pipelined one-column form
    hipLaunchKernelGGL((k_trsm_leaf1<T, LOWER, CONJT>), dim3((unsigned)nrhs), dim3(256), 0, ctx.stream, A, lda, dinv,
                       k0, (int)n, B, ldb, nrhs);
    FOSB_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL((k_trsm_leaf<T, LOWER, CS, CONJT>), dim3((unsigned)((nrhs + CS - 1) / CS)), dim3(256), 0,
                     ctx.stream, A, lda, dinv, k0, (int)n, B, ldb, nrhs);
  FOSB_LAUNCH_CHECK();
}

// The stripe of right-hand sides per workgroup is the widest that still gives
// about two workgroups per compute unit: a leaf is a chain of eight dependent
// block steps, so narrow right-hand sides are spread over more of the chip.
template <typename T, bool LOWER, bool CONJT>
static void trsm_leaf_launch(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinv, int64_t k0, int64_t n,
                             cplx<T>* B, int64_t ldb, int64_t nrhs) {
  ProfScope prof(ctx, FOSB_K_TRSM_LEAF, 4.0 * n * n * nrhs, sizeof(cplx<T>) * (0.5 * n * n + 2.0 * n * nrhs));
  const int64_t target = 2LL * ctx.n_cu;
  int cs = LeafCS<T>::v;
  while (cs > 1 && (nrhs + cs - 1) / cs < target) cs >>= 1;
  switch (cs) {
    case 16: return trsm_leaf_go<T, LOWER, (LeafCS<T>::v >= 16 ? 16 : 8), CONJT>(ctx, A, lda, dinv, k0, n, B, ldb, nrhs);
    case 8: return trsm_leaf_go<T, LOWER, 8, CONJT>(ctx, A, lda, dinv, k0, n, B, ldb, nrhs);
    case 4: return trsm_leaf_go<T, LOWER, 4, CONJT>(ctx, A, lda, dinv, k0, n, B, ldb, nrhs);
    case 2: return trsm_leaf_go<T, LOWER, 2, CONJT>(ctx, A, lda, dinv, k0, n, B, ldb, nrhs);
    default: return trsm_leaf_go<T, LOWER, 1, CONJT>(ctx, A, lda, dinv, k0, n, B, ldb, nrhs);
  }
}

template <typename T>
void trsm_lower_unit(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvL, int64_t k0, int64_t n,
                     cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) return trsm_leaf_launch<T, true, false>(ctx, A, lda, dinvL, k0, n, B, ldb, nrhs);
  const int64_t n1 = split_half(n);
  trsm_lower_unit<T>(ctx, A, lda, dinvL, k0, n1, B, ldb, nrhs);
  gemm<T>(ctx, n - n1, nrhs, n1, -1.0, A + (k0 + n1) * lda + k0, lda, B, ldb, 1.0, B + n1 * ldb, ldb);
  trsm_lower_unit<T>(ctx, A, lda, dinvL, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
}

template <typename T>
void trsm_upper(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvU, int64_t k0, int64_t n,
                cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) return trsm_leaf_launch<T, false, false>(ctx, A, lda, dinvU, k0, n, B, ldb, nrhs);
  const int64_t n1 = split_half(n);
  trsm_upper<T>(ctx, A, lda, dinvU, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
  gemm<T>(ctx, n1, nrhs, n - n1, -1.0, A + k0 * lda + (k0 + n1), lda, B + n1 * ldb, ldb, 1.0, B, ldb);
  trsm_upper<T>(ctx, A, lda, dinvU, k0, n1, B, ldb, nrhs);
}

// B <- U^{-H} B (U^H is lower triangular: forward substitution)
template <typename T>
void trsm_upper_ch(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvU, int64_t k0, int64_t n,
                   cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) return trsm_leaf_launch<T, true, true>(ctx, A, lda, dinvU, k0, n, B, ldb, nrhs);
  const int64_t n1 = split_half(n);
  trsm_upper_ch<T>(ctx, A, lda, dinvU, k0, n1, B, ldb, nrhs);
  // B2 -= (U12)^H B1, U12 = rows k0 .. k0+n1, columns k0+n1 .. k0+n
  gemm_ch<T>(ctx, n - n1, nrhs, n1, -1.0, A + k0 * lda + (k0 + n1), lda, B, ldb, 1.0, B + n1 * ldb, ldb);
  trsm_upper_ch<T>(ctx, A, lda, dinvU, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
}

// B <- L^{-H} B (L^H is unit upper triangular: backward substitution)
template <typename T>
void trsm_lower_unit_ch(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* dinvL, int64_t k0, int64_t n,
                        cplx<T>* B, int64_t ldb, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) return trsm_leaf_launch<T, false, true>(ctx, A, lda, dinvL, k0, n, B, ldb, nrhs);
  const int64_t n1 = split_half(n);
  trsm_lower_unit_ch<T>(ctx, A, lda, dinvL, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs);
  // B1 -= (L21)^H B2, L21 = rows k0+n1 .. k0+n, columns k0 .. k0+n1
  gemm_ch<T>(ctx, n1, nrhs, n - n1, -1.0, A + (k0 + n1) * lda + k0, lda, B + n1 * ldb, ldb, 1.0, B, ldb);
  trsm_lower_unit_ch<T>(ctx, A, lda, dinvL, k0, n1, B, ldb, nrhs);
}

template int64_t lu_factor<double>(Context&, c128*, int64_t, int64_t, c128*, c128*, std::vector<int32_t>&, c128*,
                                   bool);
template int64_t lu_factor<float>(Context&, c64*, int64_t, int64_t, c64*, c64*, std::vector<int32_t>&, c64*, bool);

__global__ void k_zero_u32(unsigned* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

static double float_bits(unsigned h) {
  float f;
  std::memcpy(&f, &h, sizeof(f));
  return (double)f;
}

template <typename T>
void sym_check(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, double* defect, double* amax) {
  hipStream_t s = ctx.stream;
  ctx.norms.reserve(64);
  unsigned* d = reinterpret_cast<unsigned*>(ctx.norms.p);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, d, 2);
  FOSB_LAUNCH_CHECK();
  const int64_t nb = (n + 31) / 32, npairs = nb * (nb + 1) / 2;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(npairs, 8LL * ctx.n_cu));
  hipLaunchKernelGGL(k_sym_check<T>, dim3(grid), dim3(256), 0, s, A, lda, n, d);
  FOSB_LAUNCH_CHECK();
  unsigned h[2] = {0u, 0u};
  FOSB_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipStreamSynchronize(s));
  *defect = float_bits(h[0]);
  *amax = float_bits(h[1]);
}
template void sym_check<float>(Context&, const c64*, int64_t, int64_t, double*, double*);
template void sym_check<double>(Context&, const c128*, int64_t, int64_t, double*, double*);

template <typename T>
double absmax_upper(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda) {
  hipStream_t s = ctx.stream;
  ctx.norms.reserve(64);
  unsigned* d = reinterpret_cast<unsigned*>(ctx.norms.p);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, d, 1);
  FOSB_LAUNCH_CHECK();
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 8LL * ctx.n_cu));
  hipLaunchKernelGGL(k_absmax_upper<T>, dim3(grid), dim3(256), 0, s, A, lda, n, d);
  FOSB_LAUNCH_CHECK();
  unsigned h = 0u;
  FOSB_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s));
  FOSB_HIP(hipStreamSynchronize(s));
  return float_bits(h);
}
template double absmax_upper<float>(Context&, const c64*, int64_t, int64_t);
template double absmax_upper<double>(Context&, const c128*, int64_t, int64_t);
template void trsm_lower_unit<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*,
                                      int64_t, int64_t);
template void trsm_lower_unit<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
                                     int64_t);
template void trsm_upper<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*, int64_t,
                                 int64_t);
template void trsm_upper<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
                                int64_t);
template void trsm_upper_ch<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*, int64_t,
                                    int64_t);
template void trsm_upper_ch<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
                                   int64_t);
template void trsm_lower_unit_ch<double>(Context&, const c128*, int64_t, const c128*, int64_t, int64_t, c128*,
                                         int64_t, int64_t);
template void trsm_lower_unit_ch<float>(Context&, const c64*, int64_t, const c64*, int64_t, int64_t, c64*, int64_t,
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

__global__ void k_negate_rows(c64* __restrict__ p, int64_t ld, int64_t r0, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    c64& v = p[(r0 + e / cols) * ld + e % cols];
    v = c64{-v.re, -v.im};
  }
}

void negate_rows_c64(hipStream_t s, c64* p, int64_t ld, int64_t r0, int64_t r1, int64_t cols) {
  const int64_t rows = r1 - r0;
  if (rows <= 0 || cols <= 0) return;
  const int64_t total = rows * cols;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_negate_rows, dim3(grid), dim3(256), 0, s, p, ld, r0, rows, cols);
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

__global__ void k_scatter_rows(const int32_t* __restrict__ perm, const c128* __restrict__ src, int64_t lds,
                               c128* __restrict__ dst, int64_t ldd, int64_t n, int64_t cols) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y)
    if (c < cols) dst[(int64_t)perm[r] * ldd + c] = src[r * lds + c];
}

void permute_rows_scatter(hipStream_t s, const int32_t* perm, const c128* src, int64_t lds, c128* dst, int64_t ldd,
                          int64_t n, int64_t ncols) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g((unsigned)((ncols + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
  hipLaunchKernelGGL(k_scatter_rows, g, dim3(256), 0, s, perm, src, lds, dst, ldd, n, ncols);
  FOSB_LAUNCH_CHECK();
}

// dst (cols x rows) = diag(scale) src^H (src rows x cols; scale optional), 32x32 tiles through LDS
__global__ __launch_bounds__(256) void k_conj_transpose(const c128* __restrict__ src, int64_t lds,
                                                        c128* __restrict__ dst, int64_t ldd, int64_t rows,
                                                        int64_t cols, const double* __restrict__ scale) {
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
      const double f = scale ? scale[r] : 1.0;
      dst[r * ldd + c] = c128{f * v.re, -f * v.im};
    }
  }
}

void conj_transpose_c128(hipStream_t s, const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows,
                         int64_t cols, const double* row_scale) {
  if (rows <= 0 || cols <= 0) return;
  if ((cols + 31) / 32 > INT32_MAX || (rows + 31) / 32 > 65535) fail(FOSB_E_UNSUPPORTED, "transpose of %lld rows", (long long)rows);
  dim3 g((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_conj_transpose, g, dim3(256), 0, s, src, lds, dst, ldd, rows, cols, row_scale);
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

__global__ void k_conj_inplace(c128* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i].im = -x[i].im;
}

void conj_inplace_c128(hipStream_t s, c128* x, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_conj_inplace, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
  FOSB_LAUNCH_CHECK();
}

// Squared Frobenius norms of x and y.  Each block writes its partial sums to
// its own slot and one block then adds the slots in a fixed order, so the
// result does not depend on the order in which blocks finish (the refinement
// takes its stopping decisions from these norms).
__global__ __launch_bounds__(256) void k_norms2(const c128* __restrict__ x, int64_t ldx, const c128* __restrict__ y,
                                                int64_t ldy, int64_t rows, int64_t cols, double* __restrict__ part) {
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
    part[2 * blockIdx.x] = sx[0];
    part[2 * blockIdx.x + 1] = sy[0];
  }
}

__global__ __launch_bounds__(256) void k_norms2_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sx[256], sy[256];
  double ax = 0, ay = 0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    ax += part[2 * b];
    ay += part[2 * b + 1];
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
    out[0] = sx[0];
    out[1] = sy[0];
  }
}

void norms2_c128(hipStream_t s, const c128* x, int64_t ldx, const c128* y, int64_t ldy, int64_t rows, int64_t cols,
                 double* out) {
  const int64_t total = std::max<int64_t>(rows, 0) * std::max<int64_t>(cols, 0);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kNormBlocks, (total + 255) / 256));
  double* part = out + 2;
  hipLaunchKernelGGL(k_norms2, dim3((unsigned)blocks), dim3(256), 0, s, x, ldx, y, ldy, std::max<int64_t>(rows, 0),
                     std::max<int64_t>(cols, 0), part);
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_norms2_finish, dim3(1), dim3(256), 0, s, (const double*)part, blocks, out);
  FOSB_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ matrix norms (certificates)
// Partial sums per (row chunk, column): thread = column (consecutive threads
// read consecutive entries of a row), block y = chunk of rows.  Column sums of
// |a| go to part1[chunk][col]; each block's sum of |a|^2 and max |a| go to
// part2 / partmax[chunk][column block].  The finish kernel reduces in a fixed
// order, so the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_norm_partials(const cplx<T>* __restrict__ A, int64_t lda, int64_t n,
                                                       int64_t rows_per_chunk, int upper, double* __restrict__ part1,
                                                       double* __restrict__ part2, double* __restrict__ partmax) {
  __shared__ double s2[256], sm[256];
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  double a1 = 0, a2 = 0, am = 0;
  if (c < n) {
    const int64_t rend = upper ? min(r1, c + 1) : r1;
    for (int64_t r = r0; r < rend; ++r) {
      const cplx<T> v = A[r * lda + c];
      const double re = (double)v.re, im = (double)v.im;
      const double m = sqrt(re * re + im * im);
      a1 += m;
      a2 += re * re + im * im;
      am = fmax(am, m);
    }
    part1[(int64_t)blockIdx.y * n + c] = a1;
  }
  s2[threadIdx.x] = a2;
  sm[threadIdx.x] = am;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s2[threadIdx.x] += s2[threadIdx.x + o];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part2[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s2[0];
    partmax[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sm[0];
  }
}

__global__ __launch_bounds__(256) void k_norm_finish(const double* __restrict__ part1, const double* __restrict__ part2,
                                                     const double* __restrict__ partmax, int64_t n, int nchunk,
                                                     int ncb, double* __restrict__ out) {
  __shared__ double s1[256], s2[256], sm[256];
  double one = 0, fro = 0, mx = 0;
  for (int64_t c = threadIdx.x; c < n; c += 256) {
    double col = 0;
    for (int k = 0; k < nchunk; ++k) col += part1[(int64_t)k * n + c];
    one = fmax(one, col);
  }
  for (int64_t b = threadIdx.x; b < (int64_t)nchunk * ncb; b += 256) {
    fro += part2[b];
    mx = fmax(mx, partmax[b]);
  }
  s1[threadIdx.x] = one;
  s2[threadIdx.x] = fro;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + o]);
      s2[threadIdx.x] += s2[threadIdx.x + o];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0];
    out[1] = s2[0];
    out[2] = s1[0];
  }
}

template <typename T>
void matrix_norms(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, bool upper, double* out) {
  if (n <= 0) fail(FOSB_E_INVALID, "matrix_norms: empty matrix");
  const int ncb = (int)((n + 255) / 256);
  const int nchunk = (int)std::min<int64_t>(32, n);
  const int64_t rpc = (n + nchunk - 1) / nchunk;
  DevBuf part((size_t)(n * nchunk + 2 * (int64_t)nchunk * ncb) * sizeof(double));
  double* p1 = part.as<double>();
  double* p2 = p1 + n * nchunk;
  double* pm = p2 + (int64_t)nchunk * ncb;
  hipLaunchKernelGGL(k_norm_partials<T>, dim3((unsigned)ncb, (unsigned)nchunk), dim3(256), 0, ctx.stream, A, lda, n,
                     rpc, upper ? 1 : 0, p1, p2, pm);
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(256), 0, ctx.stream, (const double*)p1, (const double*)p2,
                     (const double*)pm, n, nchunk, ncb, out);
  FOSB_LAUNCH_CHECK();
}

template void matrix_norms<float>(Context&, const c64*, int64_t, int64_t, bool, double*);
template void matrix_norms<double>(Context&, const c128*, int64_t, int64_t, bool, double*);

// ------------------------------------------------------------------ solves with block inverses
static_assert(NL == kInvBlock, "inverse block size");

template <typename T>
void upper_block_inverses(Context& ctx, const cplx<T>* A, int64_t n, int64_t lda, const cplx<T>* dinvU,
                          cplx<T>* invU) {
  if (n > 0) block_inverses<T, false>(ctx, A, n, lda, dinvU, invU, 0, (n + NL - 1) / NL);
}

// B <- T^{-1} B for rows k0 .. k0 + n of the unit lower (LOWER) or upper factor,
// k0 a multiple of NL: halves split at multiples of NL, coupled by a GEMM; a
// leaf block is X = inv_b B_b, a product into tmp (NL x nrhs) copied back.
template <typename T, bool LOWER>
static void trsm_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* inv, int64_t k0, int64_t n,
                     cplx<T>* B, int64_t ldb, int64_t nrhs, cplx<T>* tmp) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) {
    gemm<T>(ctx, n, nrhs, n, 1.0, inv + (k0 / NL) * NL * NL, NL, B, ldb, 0.0, tmp, nrhs);
    copy2d<T, T>(ctx.stream, tmp, nrhs, B, ldb, n, nrhs);
    return;
  }
  const int64_t n1 = NL * (((n + NL - 1) / NL + 1) / 2);
  if (LOWER) {
    trsm_inv<T, true>(ctx, A, lda, inv, k0, n1, B, ldb, nrhs, tmp);
    gemm<T>(ctx, n - n1, nrhs, n1, -1.0, A + (k0 + n1) * lda + k0, lda, B, ldb, 1.0, B + n1 * ldb, ldb);
    trsm_inv<T, true>(ctx, A, lda, inv, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs, tmp);
  } else {
    trsm_inv<T, false>(ctx, A, lda, inv, k0 + n1, n - n1, B + n1 * ldb, ldb, nrhs, tmp);
    gemm<T>(ctx, n1, nrhs, n - n1, -1.0, A + k0 * lda + (k0 + n1), lda, B + n1 * ldb, ldb, 1.0, B, ldb);
    trsm_inv<T, false>(ctx, A, lda, inv, k0, n1, B, ldb, nrhs, tmp);
  }
}

// X <- T^{-1} B out of place, same splits: B (rows k0 .. k0 + n) is consumed
// as workspace, each leaf product writes its block of X directly, and the
// coupling products read the solved part of X.  No copies.
template <typename T, bool LOWER>
static void trsm_inv_oop(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* inv, int64_t k0, int64_t n,
                         cplx<T>* B, int64_t ldb, cplx<T>* X, int64_t ldx, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  if (n <= NL) {
    gemm<T>(ctx, n, nrhs, n, 1.0, inv + (k0 / NL) * NL * NL, NL, B, ldb, 0.0, X, ldx);
    return;
  }
  const int64_t n1 = NL * (((n + NL - 1) / NL + 1) / 2);
  if (LOWER) {
    trsm_inv_oop<T, true>(ctx, A, lda, inv, k0, n1, B, ldb, X, ldx, nrhs);
    gemm<T>(ctx, n - n1, nrhs, n1, -1.0, A + (k0 + n1) * lda + k0, lda, X, ldx, 1.0, B + n1 * ldb, ldb);
    trsm_inv_oop<T, true>(ctx, A, lda, inv, k0 + n1, n - n1, B + n1 * ldb, ldb, X + n1 * ldx, ldx, nrhs);
  } else {
    trsm_inv_oop<T, false>(ctx, A, lda, inv, k0 + n1, n - n1, B + n1 * ldb, ldb, X + n1 * ldx, ldx, nrhs);
    gemm<T>(ctx, n1, nrhs, n - n1, -1.0, A + k0 * lda + (k0 + n1), lda, X + n1 * ldx, ldx, 1.0, B, ldb);
    trsm_inv_oop<T, false>(ctx, A, lda, inv, k0, n1, B, ldb, X, ldx, nrhs);
  }
}

template <typename T>
void trsm_lower_unit_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* invL, int64_t n, cplx<T>* B,
                         int64_t ldb, cplx<T>* X, int64_t ldx, int64_t nrhs) {
  trsm_inv_oop<T, true>(ctx, A, lda, invL, 0, n, B, ldb, X, ldx, nrhs);
}
template <typename T>
void trsm_upper_inv(Context& ctx, const cplx<T>* A, int64_t lda, const cplx<T>* invU, int64_t n, cplx<T>* B,
                    int64_t ldb, cplx<T>* X, int64_t ldx, int64_t nrhs) {
  trsm_inv_oop<T, false>(ctx, A, lda, invU, 0, n, B, ldb, X, ldx, nrhs);
}

template void upper_block_inverses<float>(Context&, const c64*, int64_t, int64_t, const c64*, c64*);
template void trsm_lower_unit_inv<float>(Context&, const c64*, int64_t, const c64*, int64_t, c64*, int64_t, c64*,
                                         int64_t, int64_t);
template void trsm_upper_inv<float>(Context&, const c64*, int64_t, const c64*, int64_t, c64*, int64_t, c64*, int64_t,
                                    int64_t);

}  // namespace fosb
