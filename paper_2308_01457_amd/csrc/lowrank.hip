// Low-rank covariance: greedy pivoted Cholesky of the covariance on the
// quadrature nodes of a level ladder, and the right-hand sides Wgt_l L_l
// built from its rows.
#include "common.h"

namespace fosb {

struct LrCov {
  int kind;
  double s2, inv2l2, s3l;
};

__device__ __forceinline__ double lr_cov(const LrCov& c, double r2, double ndot) {
  switch (c.kind) {
    case FOSB_COV_GAUSSIAN: return c.s2 * exp(-r2 * c.inv2l2);
    case FOSB_COV_MATERN32: {
      const double a = sqrt(r2) * c.s3l;
      return c.s2 * (1.0 + a) * exp(-a);
    }
    case FOSB_COV_CONSTANT: return c.s2;
    default: return c.s2 * ndot;
  }
}

static LrCov lr_params(const fosb_cov& cov) {
  LrCov c;
  c.kind = cov.kind;
  c.s2 = cov.sigma * cov.sigma;
  c.inv2l2 = cov.ell > 0 ? 1.0 / (2.0 * cov.ell * cov.ell) : 0.0;
  c.s3l = cov.ell > 0 ? std::sqrt(3.0) / cov.ell : 0.0;
  return c;
}

// Candidate normals: Nc[c][off + q] = nrm[c][q / 6] for the Q = 6 nt nodes of one level.
__global__ void k_lr_node_normals(const double* __restrict__ nrm, int nt, int64_t off, int64_t nc,
                                  double* __restrict__ Nc) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 6LL * nt) return;
  const int t = (int)(q / 6);
  for (int c = 0; c < 3; ++c) Nc[c * nc + off + q] = nrm[(int64_t)c * nt + t];
}

void lr_candidates(hipStream_t s, const Level& l, int64_t off, int64_t nc, double* Xc, double* Nc) {
  const int64_t Q = 6LL * l.mesh->h.nt;
  for (int c = 0; c < 3; ++c)
    FOSB_HIP(hipMemcpyAsync(Xc + c * nc + off, l.qx.as<double>() + c * Q, Q * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_lr_node_normals, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, l.mesh->nrm.as<double>(),
                     (int)l.mesh->h.nt, off, nc, Nc);
  FOSB_LAUNCH_CHECK();
}

__global__ void k_lr_diag(const double* __restrict__ Nc, int64_t nc, LrCov cp, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double n0 = Nc[i], n1 = Nc[nc + i], n2 = Nc[2 * nc + i];
  d[i] = lr_cov(cp, 0.0, n0 * n0 + n1 * n1 + n2 * n2);
}

void lr_diag(hipStream_t s, const double* Nc, int64_t nc, const fosb_cov& cov, double* d) {
  hipLaunchKernelGGL(k_lr_diag, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, Nc, nc, lr_params(cov), d);
  FOSB_LAUNCH_CHECK();
}

// One workgroup: the largest d, then the lowest index i with d[i] >= (1 - tie) max,
// out = {d[i], i}.  The maximum and the first index are order-independent.
__global__ __launch_bounds__(1024) void k_lr_pivot(const double* __restrict__ d, int64_t nc, double tie,
                                                   double* __restrict__ out) {
  __shared__ double sm[1024];
  __shared__ long long si[1024];
  double m = -1.0;
  for (int64_t i = threadIdx.x; i < nc; i += 1024) m = fmax(m, d[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  const double thr = (1.0 - tie) * sm[0];
  __syncthreads();
  long long best = nc;
  for (int64_t i = threadIdx.x; i < nc; i += 1024)
    if (d[i] >= thr) {
      best = i;
      break;
    }
  si[threadIdx.x] = best;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) si[threadIdx.x] = min(si[threadIdx.x], si[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long long p = si[0] < nc ? si[0] : 0;
    out[0] = d[p];
    out[1] = (double)p;
  }
}

void lr_pivot(hipStream_t s, const double* d, int64_t nc, double tie, double* out) {
  hipLaunchKernelGGL(k_lr_pivot, dim3(1), dim3(1024), 0, s, d, nc, tie, out);
  FOSB_LAUNCH_CHECK();
}

// Column j of the factor (column-major, L[k * nc + i]):
//   L[j][i] = (K(x_i, x_p) - sum_{k<j} L[k][i] L[k][p]) / sqrt(dp),  d[i] -= L[j][i]^2,  d[p] = 0.
__global__ __launch_bounds__(256) void k_lr_column(const double* __restrict__ Xc, const double* __restrict__ Nc,
                                                   int64_t nc, LrCov cp, double* __restrict__ L, int j, int64_t p,
                                                   double dp, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double e0 = Xc[i] - Xc[p], e1 = Xc[nc + i] - Xc[nc + p], e2 = Xc[2 * nc + i] - Xc[2 * nc + p];
  const double nd = Nc[i] * Nc[p] + Nc[nc + i] * Nc[nc + p] + Nc[2 * nc + i] * Nc[2 * nc + p];
  double c = lr_cov(cp, e0 * e0 + e1 * e1 + e2 * e2, nd);
  for (int k = 0; k < j; ++k) c -= L[(int64_t)k * nc + i] * L[(int64_t)k * nc + p];
  const double v = c / sqrt(dp);
  L[(int64_t)j * nc + i] = v;
  d[i] = (i == p) ? 0.0 : d[i] - v * v;
}

void lr_column(hipStream_t s, const double* Xc, const double* Nc, int64_t nc, const fosb_cov& cov, double* L, int j,
               int64_t p, double dp, double* d) {
  hipLaunchKernelGGL(k_lr_column, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, Xc, Nc, nc, lr_params(cov),
                     L, j, p, dp, d);
  FOSB_LAUNCH_CHECK();
}

// Row-major copy of rows [off, off + n) of the column-major factor: Lr[i][k] = L[k][off + i].
__global__ __launch_bounds__(256) void k_lr_rows(const double* __restrict__ L, int64_t nc, int64_t off, int64_t n,
                                                 int rank, double* __restrict__ Lr) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t i0 = (int64_t)blockIdx.x * 32, k0 = (int64_t)blockIdx.y * 32;
  for (int r = ty; r < 32; r += 8) {
    const int64_t k = k0 + r, i = i0 + tx;
    tile[r][tx] = (k < rank && i < n) ? L[k * nc + off + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, k = k0 + tx;
    if (i < n && k < rank) Lr[i * rank + k] = tile[tx][r];
  }
}

// M[m][k] = sum over the 12 nodes q of RWG m of Wgt[m][q] Lr[q][k] (M: N x rank,
// row-major; Wgt: [nt][3][6] weights of one incidence; Lr: the level's rows of the factor).
__global__ __launch_bounds__(256) void k_lr_rhs(const int32_t* __restrict__ edge_tri, const int32_t* __restrict__ edge_loc,
                                                int ne, const c128* __restrict__ W, const double* __restrict__ Lr,
                                                int rank, c128* __restrict__ M) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)ne * rank) return;
  const int64_t m = id / rank;
  const int k = (int)(id % rank);
  double ar = 0, ai = 0;
  for (int side = 0; side < 2; ++side) {
    const int t = edge_tri[side * ne + m];
    const int a = edge_loc[side * ne + m];
    for (int q = 0; q < 6; ++q) {
      const c128 w = W[((int64_t)t * 3 + a) * 6 + q];
      const double v = Lr[(6LL * t + q) * rank + k];
      ar += w.re * v;
      ai += w.im * v;
    }
  }
  M[m * rank + k] = c128{ar, ai};
}

// Lc (n x rank, complex128) = Lr (real)
__global__ void k_real_to_c128(const double* __restrict__ a, int64_t n, c128* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = c128{a[i], 0.0};
}

void lr_rows(hipStream_t s, const Level& l, const double* L, int64_t nc, int64_t off, int rank, double* Lr) {
  const int64_t Q = 6LL * l.mesh->h.nt;
  dim3 g((unsigned)((Q + 31) / 32), (unsigned)((rank + 31) / 32));
  hipLaunchKernelGGL(k_lr_rows, g, dim3(256), 0, s, L, nc, off, Q, rank, Lr);
  FOSB_LAUNCH_CHECK();
}

void real_to_c128(hipStream_t s, const double* a, int64_t n, c128* b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_real_to_c128, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, b);
  FOSB_LAUNCH_CHECK();
}

void lr_rhs(hipStream_t s, const Level& l, int64_t dir, const double* L, int64_t nc, int64_t off, int rank,
            double* Lr, c128* M) {
  const Mesh& m = *l.mesh;
  const int64_t Q = 6LL * m.h.nt;
  dim3 g((unsigned)((Q + 31) / 32), (unsigned)((rank + 31) / 32));
  hipLaunchKernelGGL(k_lr_rows, g, dim3(256), 0, s, L, nc, off, Q, rank, Lr);
  FOSB_LAUNCH_CHECK();
  const int64_t total = (int64_t)m.h.ne * rank;
  hipLaunchKernelGGL(k_lr_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, m.edge_tri.as<int32_t>(),
                     m.edge_loc.as<int32_t>(), (int)m.h.ne, l.W.as<c128>() + dir * m.h.nt * 18, (const double*)Lr,
                     rank, M);
  FOSB_LAUNCH_CHECK();
}

}  // namespace fosb
