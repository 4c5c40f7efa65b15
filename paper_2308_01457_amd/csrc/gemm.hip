// Complex GEMM on CDNA matrix cores:  C = beta*C + alpha*op(A)*B  (row-major,
// interleaved complex, real alpha/beta; op(A) = A or its conjugate transpose).  FP64 uses v_mfma_f64_16x16x4f64,
// FP32 uses v_mfma_f32_16x16x4f32.  The complex product is formed with three
// real products (Higham's 3M form):
//   T1 = Ar Br,  T2 = Ai Bi,  T3 = (Ar + Ai)(Br + Bi),
//   Re C = T1 - T2,  Im C = T3 - T1 - T2,
// the operand sums being formed in registers from the staged tiles.
//
// Tiling: 256 threads (4 wave64) per workgroup, 128 x 64 output tile, each wave
// owns a 64 x 32 sub-tile = 4 x 2 MFMA 16x16 blocks; K is staged in slices
// through double-buffered LDS in planar (re/im) layout, A stored k-major so that a fragment
// load is 16 consecutive rows.  Operand fragments (16x16x4): lane l holds
// A[l%16][k0 + l/16] and B[k0 + l/16][l%16]; accumulator element v (0..3) of
// lane l is D[row][l%16] with row = 4*(l/16) + v for the FP32 instruction and
// row = l/16 + 4*v for the FP64 one.
#include <algorithm>
#include <map>

#include "common.h"

namespace fosb {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};

constexpr int NXCD = 8;  // accelerator complex dies; workgroups are dealt to them round-robin
constexpr int GM = 8;    // tile rows per group of the tile order
constexpr int PADA = 4, PADB = 4;
// K slice staged per LDS buffer: 16 (FP32) / 8 (FP64), two buffers, so one
// barrier per slice and the next slice's global loads overlap the MFMAs.
template <typename T> struct Slice { static constexpr int BK = 16; };
template <> struct Slice<double> { static constexpr int BK = 8; };

// Split K: workgroup z of gridDim.z covers K range [z*kc, min(K, (z+1)*kc)); with
// gridDim.z > 1 it writes its raw partial product to P + z*M*N (row stride N)
// and k_gemm_splitk_sum forms C = beta*C + alpha*sum_z P_z in fixed z order.
// Tile: 2 x 2 waves, each owning WM x WN blocks of 16 x 16, so the workgroup
// covers BM = 32 WM rows and BN = 32 WN columns.  Every variant accumulates an
// output element over K in the same order (same slices, same MFMA steps), so
// the tile choice does not change results.
template <typename T, bool CONJ_A, int WM, int WN>
__device__ __forceinline__ void gemm_tile(int64_t M, int64_t N, int64_t K, T alpha, const cplx<T>* __restrict__ A,
                                          int64_t lda, const cplx<T>* __restrict__ B, int64_t ldb, T beta,
                                          cplx<T>* __restrict__ C, int64_t ldc, int64_t kc, cplx<T>* __restrict__ P) {
  using V4 = typename Mfma<T>::v4;
  constexpr int BK = Slice<T>::BK;
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int AE = BM * BK / 256;  // A elements staged per thread
  constexpr int BE = BN * BK / 256;  // B elements staged per thread
  __shared__ T AsR[2][BK][BM + PADA];
  __shared__ T AsI[2][BK][BM + PADA];
  __shared__ T BsR[2][BK][BN + PADB];
  __shared__ T BsI[2][BK][BN + PADB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1;  // wave row (0..1): rows wr*16*WM ..
  const int wc = wave & 1;   // wave col (0..1): cols wc*16*WN ..
  // XCD-aware tile order: workgroup L runs on XCD L % 8, so XCD x is given the
  // contiguous tile range [start(x), start(x) + count(x)), walked in groups of
  // GM tile rows, column by column: the ~64 workgroups resident on one XCD then
  // cover an 8 x 8 block of tiles and share their A rows and B columns in that
  // XCD's L2.
  int64_t tm, tn;
  {
    const int64_t nN = gridDim.x, nM = gridDim.y, ntile = nN * nM;
    const int64_t L = (int64_t)blockIdx.y * nN + blockIdx.x;
    const int64_t x = L % NXCD, slot = L / NXCD;
    const int64_t t = x * (ntile / NXCD) + min(x, ntile % NXCD) + slot;
    const int64_t group = t / (GM * nN);
    const int64_t fm = group * GM;
    const int64_t gs = min<int64_t>(nM - fm, GM);
    const int64_t in = t - group * GM * nN;
    tm = fm + in % gs;
    tn = in / gs;
  }
  const int64_t m0 = tm * BM;
  const int64_t n0 = tn * BN;

  // global -> register staging assignment (op(A) = A^H: threads run along the
  // rows of op(A), which are contiguous in memory)
  const int a_row = CONJ_A ? tid % BM : tid / (BK / AE);
  const int a_k = CONJ_A ? (tid / BM) * AE : (tid % (BK / AE)) * AE;
  const int b_k = tid / (BN / BE);
  const int b_col = (tid % (BN / BE)) * BE;

  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke = min(K, kb + kc);
  cplx<T> ra[AE], rb[BE];
  const bool interior = m0 + BM <= M && n0 + BN <= N;  // no tile edge in M or N
  auto load_tiles = [&](int64_t k0) {
    const int64_t gr = m0 + a_row;
    if (interior && k0 + BK <= ke) {  // the whole slice is inside the operands: no edge checks
      // B's loads first: issued last, they would equal the checked path's
      // closing loads, and the compiler would merge the two tails and wait for
      // A's loads before issuing them.
      const cplx<T>* brow = B + (k0 + b_k) * ldb + n0 + b_col;
#pragma unroll
      for (int e = 0; e < BE; ++e) rb[e] = brow[e];
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int64_t gk = k0 + a_k + e;
        if (CONJ_A) {
          const cplx<T> v = A[gk * lda + gr];
          ra[e] = cplx<T>{v.re, -v.im};
        } else {
          ra[e] = A[gr * lda + gk];
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int64_t gk = k0 + a_k + e;
      if (CONJ_A) {
        const cplx<T> v = (gr < M && gk < ke) ? A[gk * lda + gr] : cplx<T>{T(0), T(0)};
        ra[e] = cplx<T>{v.re, -v.im};
      } else {
        ra[e] = (gr < M && gk < ke) ? A[gr * lda + gk] : cplx<T>{T(0), T(0)};
      }
    }
    const int64_t gk = k0 + b_k;
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int64_t gc = n0 + b_col + e;
      rb[e] = (gk < ke && gc < N) ? B[gk * ldb + gc] : cplx<T>{T(0), T(0)};
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      AsR[buf][a_k + e][a_row] = ra[e].re;
      AsI[buf][a_k + e][a_row] = ra[e].im;
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      BsR[buf][b_k][b_col + e] = rb[e].re;
      BsI[buf][b_k][b_col + e] = rb[e].im;
    }
  };

  V4 t1[WM][WN], t2[WM][WN], t3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      t1[i][j] = V4{0, 0, 0, 0};
      t2[i][j] = V4{0, 0, 0, 0};
      t3[i][j] = V4{0, 0, 0, 0};
    }

  const int r16 = lane & 15;
  const int kq = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T ar[WM], ai[WM], as[WM], br[WN], bi[WN], bs[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ar[i] = AsR[buf][kk + kq][wr * 16 * WM + i * 16 + r16];
        ai[i] = AsI[buf][kk + kq][wr * 16 * WM + i * 16 + r16];
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = BsR[buf][kk + kq][wc * 16 * WN + j * 16 + r16];
        bi[j] = BsI[buf][kk + kq][wc * 16 * WN + j * 16 + r16];
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          t1[i][j] = Mfma<T>::op(ar[i], br[j], t1[i][j]);
          t2[i][j] = Mfma<T>::op(ai[i], bi[j], t2[i][j]);
          t3[i][j] = Mfma<T>::op(as[i], bs[j], t3[i][j]);
        }
    }
  };

  if (ke > kb) {
    load_tiles(kb);
    store_tiles(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) load_tiles(k0 + BK);  // next slice in flight during the MFMAs
      compute(buf);
      if (more) store_tiles(buf ^ 1);  // the other buffer was last read before the previous barrier
      __syncthreads();
      buf ^= 1;
    }
  }

  // epilogue
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wr * 16 * WM + i * 16 + Mfma<T>::row(kq, v);
        const int64_t col = n0 + wc * 16 * WN + j * 16 + r16;
        if (row < M && col < N) {
          const T cr = t1[i][j][v] - t2[i][j][v];
          const T ci = t3[i][j][v] - t1[i][j][v] - t2[i][j][v];
          if (gridDim.z > 1) {
            P[(int64_t)blockIdx.z * M * N + row * N + col] = cplx<T>{cr, ci};
            continue;
          }
          cplx<T>* p = C + row * ldc + col;
          if (beta == T(0)) {
            *p = cplx<T>{alpha * cr, alpha * ci};
          } else {
            const cplx<T> o = *p;
            *p = cplx<T>{beta * o.re + alpha * cr, beta * o.im + alpha * ci};
          }
        }
      }
}

#define FOSB_GEMM_ARGS(T)                                                                                     \
  int64_t M, int64_t N, int64_t K, T alpha, const cplx<T>* __restrict__ A, int64_t lda,                       \
      const cplx<T>* __restrict__ B, int64_t ldb, T beta, cplx<T>* __restrict__ C, int64_t ldc, int64_t kc,    \
      cplx<T>* __restrict__ P

template <typename T, bool CONJ_A, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm(FOSB_GEMM_ARGS(T)) {
  gemm_tile<T, CONJ_A, WM, WN>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P);
}

// The FP64 64 x 32 tile asks for four waves per SIMD: the compiler then keeps its
// accumulators in VGPRs instead of AGPRs (113 registers, no spills) and the
// occupancy rises from 3 to 4, which measured 64 -> 78 TFLOP/s on a 30720 x 480
// x 30720 product.  The larger FP64 tiles would spill under that request.
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm<double, false, 2, 1>(
    FOSB_GEMM_ARGS(double)) {
  gemm_tile<double, false, 2, 1>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P);
}
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm<double, true, 2, 1>(
    FOSB_GEMM_ARGS(double)) {
  gemm_tile<double, true, 2, 1>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P);
}
#undef FOSB_GEMM_ARGS

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_splitk_sum(int64_t M, int64_t N, int nz, T alpha,
                                                         const cplx<T>* __restrict__ P, T beta,
                                                         cplx<T>* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t row = idx / N, col = idx % N;
  T sr = 0, si = 0;
  for (int z = 0; z < nz; ++z) {
    const cplx<T> v = P[(int64_t)z * M * N + idx];
    sr += v.re;
    si += v.im;
  }
  cplx<T>* p = C + row * ldc + col;
  if (beta == T(0)) {
    *p = cplx<T>{alpha * sr, alpha * si};
  } else {
    const cplx<T> o = *p;
    *p = cplx<T>{beta * o.re + alpha * sr, beta * o.im + alpha * si};
  }
}

// Narrow right-hand sides (N <= 4, e.g. one incidence): a bandwidth-bound
// product, one wave per row of A streaming it once with 16-byte loads; the N
// columns of B are read through the cache.  Row sums are reduced in the wave.
constexpr int GEMV_MAXN = 4;

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_gemv(int64_t M, int64_t K, T alpha, const cplx<T>* __restrict__ A,
                                              int64_t lda, const cplx<T>* __restrict__ B, int64_t ldb, T beta,
                                              cplx<T>* __restrict__ C, int64_t ldc) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= M) return;
  const cplx<T>* a = A + row * lda;
  T ar[NC], ai[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) ar[c] = ai[c] = T(0);
  int64_t k = lane;
  for (; k + 192 < K; k += 256) {
    cplx<T> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = a[k + 64 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const cplx<T> b = B[(k + 64 * u) * ldb + c];
        ar[c] += v[u].re * b.re - v[u].im * b.im;
        ai[c] += v[u].re * b.im + v[u].im * b.re;
      }
  }
  for (; k < K; k += 64) {
    const cplx<T> v = a[k];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cplx<T> b = B[k * ldb + c];
      ar[c] += v.re * b.re - v.im * b.im;
      ai[c] += v.re * b.im + v.im * b.re;
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ar[c] += __shfl_xor(ar[c], o);
      ai[c] += __shfl_xor(ai[c], o);
    }
  }
  if (lane < NC) {
    T sr = ar[0], si = ai[0];
#pragma unroll
    for (int c = 1; c < NC; ++c)
      if (lane == c) sr = ar[c], si = ai[c];
    cplx<T>* p = C + row * ldc + lane;
    if (beta == T(0)) {
      *p = cplx<T>{alpha * sr, alpha * si};
    } else {
      const cplx<T> o = *p;
      *p = cplx<T>{beta * o.re + alpha * sr, beta * o.im + alpha * si};
    }
  }
}

template <typename T, int NC>
static void gemv_launch(Context& ctx, int64_t M, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
                        const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc) {
  hipLaunchKernelGGL((k_gemv<T, NC>), dim3((unsigned)((M + 3) / 4)), dim3(256), 0, ctx.stream, M, K, (T)alpha, A,
                     lda, B, ldb, (T)beta, C, ldc);
  FOSB_LAUNCH_CHECK();
}

// Tile variants (WM, WN) offered to the autotuner, fastest-first by measurement
// on gfx950 (the first entry is the built-in choice when tuning is off).
template <typename T> struct Tiles;
// `lean` is the variant with the smallest register and LDS footprint.
template <> struct Tiles<float> {
  static constexpr int n = 4;
  static constexpr int wm[4] = {2, 2, 2, 4}, wn[4] = {2, 1, 4, 2};
  static constexpr int lean = 1;  // 64 x 32
};
template <> struct Tiles<double> {
  static constexpr int n = 3;
  static constexpr int wm[3] = {2, 2, 4}, wn[3] = {1, 2, 2};
  static constexpr int lean = 0;  // 64 x 32
};

template <typename T, bool CONJ_A, int WM, int WN>
static void launch_tile(hipStream_t s, int64_t M, int64_t N, int64_t K, T alpha, const cplx<T>* A, int64_t lda,
                        const cplx<T>* B, int64_t ldb, T beta, cplx<T>* C, int64_t ldc, int64_t kc, cplx<T>* P,
                        int64_t nz) {
  dim3 grid((unsigned)((N + 32 * WN - 1) / (32 * WN)), (unsigned)((M + 32 * WM - 1) / (32 * WM)), (unsigned)nz);
  hipLaunchKernelGGL((k_gemm<T, CONJ_A, WM, WN>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                     kc, P);
  FOSB_LAUNCH_CHECK();
}

template <typename T, bool CONJ_A>
static void launch_variant(int var, hipStream_t s, int64_t M, int64_t N, int64_t K, T alpha, const cplx<T>* A,
                           int64_t lda, const cplx<T>* B, int64_t ldb, T beta, cplx<T>* C, int64_t ldc, int64_t kc,
                           cplx<T>* P, int64_t nz) {
  if constexpr (sizeof(T) == 4) {
    switch (var) {
      case 1: return launch_tile<T, CONJ_A, 2, 1>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
      case 2: return launch_tile<T, CONJ_A, 2, 4>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
      case 3: return launch_tile<T, CONJ_A, 4, 2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
      default: return launch_tile<T, CONJ_A, 2, 2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
    }
  } else {
    switch (var) {
      case 1: return launch_tile<T, CONJ_A, 2, 2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
      case 2: return launch_tile<T, CONJ_A, 4, 2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
      default: return launch_tile<T, CONJ_A, 2, 1>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kc, P, nz);
    }
  }
}

static inline int log2_bucket(int64_t x) {
  int b = 0;
  while (x > 1) {
    x >>= 1;
    ++b;
  }
  return b;
}

// Tile variant for this product: the tuned choice of its size bucket (precision,
// A operand form, floor(log2) of M, N and K).  A bucket met for the first time
// with tuning on is settled by timing every variant on the real operands into
// scratch output (three interleaved rounds, each variant's fastest run counts);
// the choice is kept by the root context.  The variants give identical
// results, so tuning only affects speed.
template <typename T, bool CONJ_A>
static int pick_variant(Context& ctx, int64_t M, int64_t N, int64_t K, const cplx<T>* A, int64_t lda,
                        const cplx<T>* B, int64_t ldb) {
  Context& root = ctx.prof_root ? *ctx.prof_root : ctx;
  if (!root.autotune) return 0;
  const int64_t key = ((int64_t)(sizeof(T) == 8) << 40) | ((int64_t)CONJ_A << 39) | ((int64_t)log2_bucket(M) << 26) |
                      ((int64_t)log2_bucket(N) << 13) | (int64_t)log2_bucket(K);
  {
    std::lock_guard<std::mutex> lock(root.tune_mu);
    auto it = root.tune.find(key);
    if (it != root.tune.end()) return it->second;
  }
  if (ctx.no_alloc) return 0;  // no scratch output to time into
  ctx.tune_out.reserve((size_t)M * N * sizeof(cplx<T>));
  if (!ctx.tune_ev[0]) {
    FOSB_HIP(hipEventCreate(&ctx.tune_ev[0]));
    FOSB_HIP(hipEventCreate(&ctx.tune_ev[1]));
  }
  // three rounds over the variants, each variant keeping its fastest run: the
  // chip may be shared with other streams' work, which only ever adds time
  float t[Tiles<T>::n];
  for (int v = 0; v < Tiles<T>::n; ++v) t[v] = 1e30f;
  for (int rep = 0; rep < 3; ++rep)
    for (int v = 0; v < Tiles<T>::n; ++v) {
      FOSB_HIP(hipEventRecord(ctx.tune_ev[0], ctx.stream));
      launch_variant<T, CONJ_A>(v, ctx.stream, M, N, K, T(1), A, lda, B, ldb, T(0),
                                static_cast<cplx<T>*>(ctx.tune_out.p), N, K, nullptr, 1);
      FOSB_HIP(hipEventRecord(ctx.tune_ev[1], ctx.stream));
      FOSB_HIP(hipEventSynchronize(ctx.tune_ev[1]));
      float ms = 0.f;
      FOSB_HIP(hipEventElapsedTime(&ms, ctx.tune_ev[0], ctx.tune_ev[1]));
      t[v] = std::min(t[v], ms);
    }
  int best = 0;
  for (int v = 1; v < Tiles<T>::n; ++v)
    if (t[v] < t[best]) best = v;
  std::lock_guard<std::mutex> lock(root.tune_mu);
  root.tune[key] = best;
  return best;
}

template <typename T, bool CONJ_A>
static void gemm_launch(Context& ctx, int64_t M, int64_t N, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
                        const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return;
  if (K <= 0) {
    if (beta == 1.0) return;
  }
  // algorithmic work: 8 flop per complex multiply-add; A, B read and C read+written once
  const double flops = 8.0 * (double)M * (double)N * (double)std::max<int64_t>(K, 0);
  const double bytes = (double)sizeof(cplx<T>) * ((double)M * K + (double)K * N + (beta != 0.0 ? 2.0 : 1.0) * M * N);
  if (!CONJ_A && N <= GEMV_MAXN && K > 0 && (M + 3) / 4 <= INT32_MAX) {
    ProfScope prof(ctx, FOSB_K_GEMV, flops, bytes);
    switch (N) {
      case 1: return gemv_launch<T, 1>(ctx, M, K, alpha, A, lda, B, ldb, beta, C, ldc);
      case 2: return gemv_launch<T, 2>(ctx, M, K, alpha, A, lda, B, ldb, beta, C, ldc);
      case 3: return gemv_launch<T, 3>(ctx, M, K, alpha, A, lda, B, ldb, beta, C, ldc);
      default: return gemv_launch<T, 4>(ctx, M, K, alpha, A, lda, B, ldb, beta, C, ldc);
    }
  }
  const int64_t Kp = std::max<int64_t>(K, 0);
  // split K when the output has too few tiles to fill the chip and K is long:
  // about two workgroups per CU, each still streaming at least 256 of K.  The
  // decision uses a fixed 64 x 64 reference tile, so it (and the summation
  // order) does not depend on the tile variant chosen below.
  const int64_t tiles = ((N + 63) / 64) * ((M + 63) / 64);
  int64_t nz = 1;
  const int64_t want = 2LL * ctx.n_cu;
  if (tiles < want && Kp >= 512 && !ctx.no_alloc) nz = std::min<int64_t>({(want + tiles - 1) / tiles, Kp / 256, 64});
  int64_t kc = Kp;
  cplx<T>* P = nullptr;
  if (nz > 1) {
    kc = ((Kp + nz - 1) / nz + Slice<T>::BK - 1) / Slice<T>::BK * Slice<T>::BK;
    nz = (Kp + kc - 1) / kc;
    ctx.splitk.reserve((size_t)nz * M * N * sizeof(cplx<T>));
    P = static_cast<cplx<T>*>(ctx.splitk.p);
  }
  // The trailing update's large complex64 products (at least four 128 x 64
  // tiles per CU) take the 64 x 64 tile.  Timed beside the panel stream, the
  // tuner often prefers the 64 x 32 tile for them, whose five workgroups per
  // CU leave the panel stream's kernels no room: the step is then ~4% slower.
  const bool update_big =
      sizeof(T) == 4 && ctx.trailing_update > 0 && ((M + 127) / 128) * ((N + 63) / 64) >= 4LL * ctx.n_cu;
  const int var = (nz != 1 || Kp <= 0) ? 0
                  : ctx.lean_tiles > 0 ? Tiles<T>::lean
                  : update_big         ? 0
                                       : pick_variant<T, CONJ_A>(ctx, M, N, Kp, A, lda, B, ldb);
  {
    ProfScope prof(ctx, sizeof(T) == 8 ? FOSB_K_GEMM_F64 : FOSB_K_GEMM_F32, flops, bytes);
    launch_variant<T, CONJ_A>(var, ctx.stream, M, N, Kp, (T)alpha, A, lda, B, ldb, (T)beta, C, ldc, kc, P, nz);
  }
  if (nz > 1) {
    ProfScope prof(ctx, FOSB_K_SPLITK_SUM, 2.0 * (double)nz * M * N,
                   (double)sizeof(cplx<T>) * ((double)nz + 2.0) * M * N);
    hipLaunchKernelGGL((k_gemm_splitk_sum<T>), dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, ctx.stream, M, N,
                       (int)nz, (T)alpha, P, (T)beta, C, ldc);
    FOSB_LAUNCH_CHECK();
  }
}

template <typename T>
void gemm(Context& ctx, int64_t M, int64_t N, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
          const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc) {
  gemm_launch<T, false>(ctx, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

template <typename T>
void gemm_ch(Context& ctx, int64_t M, int64_t N, int64_t K, double alpha, const cplx<T>* A, int64_t lda,
             const cplx<T>* B, int64_t ldb, double beta, cplx<T>* C, int64_t ldc) {
  gemm_launch<T, true>(ctx, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

template void gemm<double>(Context&, int64_t, int64_t, int64_t, double, const c128*, int64_t, const c128*, int64_t,
                           double, c128*, int64_t);
template void gemm<float>(Context&, int64_t, int64_t, int64_t, double, const c64*, int64_t, const c64*, int64_t,
                          double, c64*, int64_t);
template void gemm_ch<double>(Context&, int64_t, int64_t, int64_t, double, const c128*, int64_t, const c128*, int64_t,
                              double, c128*, int64_t);
template void gemm_ch<float>(Context&, int64_t, int64_t, int64_t, double, const c64*, int64_t, const c64*, int64_t,
                             double, c64*, int64_t);

}  // namespace fosb
