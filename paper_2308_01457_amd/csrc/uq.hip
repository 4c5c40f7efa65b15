// Right-hand sides, shape-derivative weights, RHS correlation and far-field
// kernels (FP64).
//
// On triangle t the RWG function of local edge a is phi = (alpha_a / 2)(x - P_a)
// with alpha_a = sign * length / area (sign +1 on T+, -1 on T-) and P_a the
// vertex opposite the edge; div phi = alpha_a.  All surface integrals use the
// symmetric 6-point rule.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace fosb {

struct Rule6Q {
  double l[6][3];
  double w[6];
};

static Rule6Q make_rule() {
  Rule6Q r;
  rule6(r.l, r.w);
  return r;
}

__device__ __forceinline__ void tri_vertices(const MeshDev& md, int t, double P[3][3]) {
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < 3; ++c) P[v][c] = md.vtx[(v * 3 + c) * md.nt + t];
}

// b[dir][m] = -int p exp(i k d.x) . phi_m(x) dx
__global__ void k_incident_rhs(MeshDev md, Rule6Q R, double k, const double* __restrict__ dirs,
                               const double* __restrict__ pols, int ndir, c128* __restrict__ b) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int dr = blockIdx.y;
  if (m >= md.ne || dr >= ndir) return;
  const double d0 = dirs[3 * dr], d1 = dirs[3 * dr + 1], d2 = dirs[3 * dr + 2];
  const double p0 = pols[3 * dr], p1 = pols[3 * dr + 1], p2 = pols[3 * dr + 2];
  double sr = 0, si = 0;
  for (int side = 0; side < 2; ++side) {
    const int t = md.edge_tri[side * md.ne + m];
    const int a = md.edge_loc[side * md.ne + m];
    double P[3][3];
    tri_vertices(md, t, P);
    const double half_alpha = 0.5 * md.alpha[a * md.nt + t];
    const double At = md.area[t];
    for (int q = 0; q < 6; ++q) {
      double x[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
      double sn, cs;
      sincos(k * (d0 * x[0] + d1 * x[1] + d2 * x[2]), &sn, &cs);
      const double pdot = p0 * (x[0] - P[a][0]) + p1 * (x[1] - P[a][1]) + p2 * (x[2] - P[a][2]);
      const double f = R.w[q] * At * half_alpha * pdot;
      sr += f * cs;
      si += f * sn;
    }
  }
  b[(int64_t)m * ndir + dr] = c128{-sr, -si};
}

void incident_rhs(hipStream_t s, const Mesh& m, double k, const double* dirs_dev, const double* pols_dev, int ndir,
                  c128* b) {
  dim3 g((unsigned)((m.h.ne + 255) / 256), (unsigned)ndir);
  hipLaunchKernelGGL(k_incident_rhs, g, dim3(256), 0, s, m.dev(), make_rule(), k, dirs_dev, pols_dev, ndir, b);
  FOSB_LAUNCH_CHECK();
}

// PMCHWT incident data: e[m] = int phi_m . p e^{ik d.x} (rows 0..N-1) and
// h[m] = int phi_m . (d x p) e^{ik d.x} (rows N..2N-1), 6-point rule.
__global__ void k_incident_rhs_pmchwt(MeshDev md, Rule6Q R, double k, const double* __restrict__ dirs,
                                      const double* __restrict__ pols, int ndir, c128* __restrict__ b) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int dr = blockIdx.y;
  if (m >= md.ne || dr >= ndir) return;
  const double d[3] = {dirs[3 * dr], dirs[3 * dr + 1], dirs[3 * dr + 2]};
  const double p[3] = {pols[3 * dr], pols[3 * dr + 1], pols[3 * dr + 2]};
  const double hp[3] = {d[1] * p[2] - d[2] * p[1], d[2] * p[0] - d[0] * p[2], d[0] * p[1] - d[1] * p[0]};
  double er = 0, ei = 0, hr = 0, hi = 0;
  for (int side = 0; side < 2; ++side) {
    const int t = md.edge_tri[side * md.ne + m];
    const int a = md.edge_loc[side * md.ne + m];
    double P[3][3];
    tri_vertices(md, t, P);
    const double half_alpha = 0.5 * md.alpha[a * md.nt + t];
    const double At = md.area[t];
    for (int q = 0; q < 6; ++q) {
      double x[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
      double sn, cs;
      sincos(k * (d[0] * x[0] + d[1] * x[1] + d[2] * x[2]), &sn, &cs);
      const double v0 = x[0] - P[a][0], v1 = x[1] - P[a][1], v2 = x[2] - P[a][2];
      const double f = R.w[q] * At * half_alpha;
      const double pe = f * (p[0] * v0 + p[1] * v1 + p[2] * v2);
      const double ph = f * (hp[0] * v0 + hp[1] * v1 + hp[2] * v2);
      er += pe * cs;
      ei += pe * sn;
      hr += ph * cs;
      hi += ph * sn;
    }
  }
  b[(int64_t)m * ndir + dr] = c128{er, ei};
  b[(int64_t)(md.ne + m) * ndir + dr] = c128{hr, hi};
}

void incident_rhs_pmchwt(hipStream_t s, const Mesh& m, double k, const double* dirs_dev, const double* pols_dev,
                         int ndir, c128* b) {
  dim3 g((unsigned)((m.h.ne + 255) / 256), (unsigned)ndir);
  hipLaunchKernelGGL(k_incident_rhs_pmchwt, g, dim3(256), 0, s, m.dev(), make_rule(), k, dirs_dev, pols_dev, ndir,
                     b);
  FOSB_LAUNCH_CHECK();
}

// C[i][j] = b1[i][dir] conj(b2[j][dir])
__global__ void k_rank_one(const c128* __restrict__ b1, int64_t n1, const c128* __restrict__ b2, int64_t n2,
                           int64_t nd, int64_t dir, c128* __restrict__ C, int64_t ldc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n2 || i >= n1) return;
  const c128 u = b1[i * nd + dir], v = b2[j * nd + dir];
  C[i * ldc + j] = c128{u.re * v.re + u.im * v.im, u.im * v.re - u.re * v.im};
}

void rank_one_correlation(hipStream_t s, const c128* b1, int64_t n1, const c128* b2, int64_t n2, int64_t nd,
                          int64_t dir, c128* C, int64_t ldc) {
  if (n1 <= 0 || n2 <= 0) return;
  dim3 g((unsigned)((n2 + 255) / 256), (unsigned)n1);
  hipLaunchKernelGGL(k_rank_one, g, dim3(256), 0, s, b1, n1, b2, n2, nd, dir, C, ldc);
  FOSB_LAUNCH_CHECK();
}

// qx[c][6t + q]: physical 6-point nodes
__global__ void k_quad_nodes(MeshDev md, Rule6Q R, double* __restrict__ qx) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= md.nt) return;
  double P[3][3];
  tri_vertices(md, t, P);
  const int64_t Q = 6LL * md.nt;
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      qx[c * Q + 6LL * t + q] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
}

void quad_nodes(hipStream_t s, const Mesh& m, double* qx) {
  hipLaunchKernelGGL(k_quad_nodes, dim3((unsigned)((m.h.nt + 255) / 256)), dim3(256), 0, s, m.dev(), make_rule(),
                     qx);
  FOSB_LAUNCH_CHECK();
}

// Shape-derivative RHS weights (FOA section, PEC shape derivative with
// E_n = (i/k) div j and gamma_T H = n x j):
//   W[t][a][q] = w_q A_t nu(x_q) [ (i/k) div j(t) div phi_a - i k j(x_q) . phi_a(x_q) ]
// nu = (x/|x|).n for the radial field, 1 for the normal field.
__global__ void k_rhs_weights(MeshDev md, Rule6Q R, double k, int field, const c128* __restrict__ u,
                              int64_t ustride, c128* __restrict__ W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= md.nt) return;
  const int nt = md.nt;
  double P[3][3];
  tri_vertices(md, t, P);
  double al[3];
  c128 ue[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    al[b] = md.alpha[b * nt + t];
    ue[b] = u[(int64_t)md.tri_edge[b * nt + t] * ustride];
  }
  double djr = 0, dji = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    djr += ue[b].re * al[b];
    dji += ue[b].im * al[b];
  }
  const double n0 = md.nrm[t], n1 = md.nrm[nt + t], n2 = md.nrm[2 * nt + t];
  const double At = md.area[t];
  for (int q = 0; q < 6; ++q) {
    double x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
    double nu = 1.0;
    if (field == FOSB_FIELD_RADIAL) {
      const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      nu = (x[0] * n0 + x[1] * n1 + x[2] * n2) / r;
    }
    // j(x) = sum_b u_b (alpha_b / 2)(x - P_b)
    double jr[3] = {0, 0, 0}, ji[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ph = 0.5 * al[b] * (x[c] - P[b][c]);
        jr[c] += ue[b].re * ph;
        ji[c] += ue[b].im * ph;
      }
    const double wq = R.w[q] * At * nu;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double dr = 0, di = 0;  // j . phi_a
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ph = 0.5 * al[a] * (x[c] - P[a][c]);
        dr += jr[c] * ph;
        di += ji[c] * ph;
      }
      // (i/k) divj alpha_a - i k (j.phi_a)
      const double re = -dji * al[a] / k + k * di;
      const double im = djr * al[a] / k - k * dr;
      W[((int64_t)t * 3 + a) * 6 + q] = c128{wq * re, wq * im};
    }
  }
}

void rhs_weights(hipStream_t s, const Mesh& m, double k, int field, const c128* u, int64_t ustride, c128* W) {
  hipLaunchKernelGGL(k_rhs_weights, dim3((unsigned)((m.h.nt + 255) / 256)), dim3(256), 0, s, m.dev(), make_rule(), k,
                     field, u, ustride, W);
  FOSB_LAUNCH_CHECK();
}

// C[m][n] = sum_{q in supp m} sum_{q' in supp n} W1[m,q] K(x_q, y_q') conj(W2[n,q'])
// one thread per entry; the 12 nodes and weights of each row/column RWG are
// staged in LDS (16 x 16 entries per block).
struct CovParams {
  int kind;
  double s2;       // sigma^2
  double inv2l2;   // 1 / (2 ell^2)
  double s3l;      // sqrt(3) / ell
};

__device__ __forceinline__ double cov_eval(const CovParams& cp, double r2, double ndot) {
  switch (cp.kind) {
    case FOSB_COV_GAUSSIAN: return cp.s2 * exp(-r2 * cp.inv2l2);
    case FOSB_COV_MATERN32: {
      const double a = sqrt(r2) * cp.s3l;
      return cp.s2 * (1.0 + a) * exp(-a);
    }
    case FOSB_COV_CONSTANT: return cp.s2;
    default: return cp.s2 * ndot;
  }
}

struct EdgeSide {
  const int32_t* edge_tri;
  const int32_t* edge_loc;
  const double* nrm;
  const double* qx;
  const c128* W;
  int ne, nt;
};

__device__ void stage_edge(const EdgeSide& L, int e, double (*x)[3], c128* w, double (*nn)[3]) {
  // 12 nodes: 6 on T+ then 6 on T-
  const int64_t Q = 6LL * L.nt;
  for (int side = 0; side < 2; ++side) {
    const int t = L.edge_tri[side * L.ne + e];
    const int a = L.edge_loc[side * L.ne + e];
    for (int q = 0; q < 6; ++q) {
      const int64_t id = 6LL * t + q;
      x[side * 6 + q][0] = L.qx[id];
      x[side * 6 + q][1] = L.qx[Q + id];
      x[side * 6 + q][2] = L.qx[2 * Q + id];
      w[side * 6 + q] = L.W[((int64_t)t * 3 + a) * 6 + q];
    }
    nn[side][0] = L.nrm[t];
    nn[side][1] = L.nrm[L.nt + t];
    nn[side][2] = L.nrm[2 * L.nt + t];
  }
}

// node coordinates and triangle normals of RWG e (no weights)
__device__ void stage_nodes(const EdgeSide& L, int e, double (*x)[3], double (*nn)[3]) {
  const int64_t Q = 6LL * L.nt;
  for (int side = 0; side < 2; ++side) {
    const int t = L.edge_tri[side * L.ne + e];
    for (int q = 0; q < 6; ++q) {
      const int64_t id = 6LL * t + q;
      x[side * 6 + q][0] = L.qx[id];
      x[side * 6 + q][1] = L.qx[Q + id];
      x[side * 6 + q][2] = L.qx[2 * Q + id];
    }
    nn[side][0] = L.nrm[t];
    nn[side][1] = L.nrm[L.nt + t];
    nn[side][2] = L.nrm[2 * L.nt + t];
  }
}

__global__ __launch_bounds__(256) void k_rhs_correlation(EdgeSide A, EdgeSide B, CovParams cp, c128* __restrict__ C,
                                                         int64_t ldc) {
  __shared__ double xa[16][12][3], xb[16][12][3];
  __shared__ c128 wa[16][12], wb[16][12];
  __shared__ double na[16][2][3], nb[16][2][3];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
  if (threadIdx.x < 16) {
    const int e = m0 + threadIdx.x;
    if (e < A.ne) stage_edge(A, e, xa[threadIdx.x], wa[threadIdx.x], na[threadIdx.x]);
  } else if (threadIdx.x < 32) {
    const int r = threadIdx.x - 16;
    const int e = n0 + r;
    if (e < B.ne) stage_edge(B, e, xb[r], wb[r], nb[r]);
  }
  __syncthreads();
  const int m = m0 + ty, n = n0 + tx;
  if (m >= A.ne || n >= B.ne) return;
  double cr = 0, ci = 0;
  for (int q = 0; q < 12; ++q) {
    const double x0 = xa[ty][q][0], x1 = xa[ty][q][1], x2 = xa[ty][q][2];
    const double* nx = na[ty][q / 6];
    double ar = 0, ai = 0;  // sum_q' K conj(W2)
#pragma unroll 4
    for (int p = 0; p < 12; ++p) {
      const double d0 = x0 - xb[tx][p][0], d1 = x1 - xb[tx][p][1], d2 = x2 - xb[tx][p][2];
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double* ny = nb[tx][p / 6];
      const double kv = cov_eval(cp, r2, nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2]);
      ar += kv * wb[tx][p].re;
      ai -= kv * wb[tx][p].im;
    }
    const c128 w = wa[ty][q];
    cr += w.re * ar - w.im * ai;
    ci += w.re * ai + w.im * ar;
  }
  C[(int64_t)m * ldc + n] = c128{cr, ci};
}

// Several incidences at once: the covariance between the 12 nodes of RWG m
// and those of RWG n does not depend on the incidence, so each block of
// kernel values is evaluated once per chunk of up to RC_DC incidences and
// applied to all of them.  C_d (incidence dir0 + d) is written at
// C + d * dstride with row stride ldc.
constexpr int RC_DC = 8;

__global__ __launch_bounds__(256) void k_rhs_correlation_multi(EdgeSide A, EdgeSide B, CovParams cp, int dc,
                                                               c128* __restrict__ C, int64_t ldc, int64_t dstride) {
  __shared__ double xa[16][12][3], xb[16][12][3];
  __shared__ c128 wa[16][12][RC_DC], wb[16][12][RC_DC];
  __shared__ double na[16][2][3], nb[16][2][3];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
  if (threadIdx.x < 16) {
    const int e = m0 + threadIdx.x;
    if (e < A.ne) stage_nodes(A, e, xa[threadIdx.x], na[threadIdx.x]);
  } else if (threadIdx.x < 32) {
    const int r = threadIdx.x - 16;
    const int e = n0 + r;
    if (e < B.ne) stage_nodes(B, e, xb[r], nb[r]);
  }
  // weights of every incidence of the chunk: wa[r][q][d], wb[r][q][d] (zero past dc)
  for (int e = threadIdx.x; e < 2 * 16 * 12 * RC_DC; e += 256) {
    const int side = e / (16 * 12 * RC_DC);
    const int rem = e % (16 * 12 * RC_DC);
    const int r = rem / (12 * RC_DC), q = (rem / RC_DC) % 12, d = rem % RC_DC;
    const EdgeSide& S = side ? B : A;
    const int eidx = (side ? n0 : m0) + r;
    c128 w = c128{0.0, 0.0};
    if (eidx < S.ne && d < dc) {
      const int t = S.edge_tri[(q / 6) * S.ne + eidx];
      const int a = S.edge_loc[(q / 6) * S.ne + eidx];
      w = S.W[(int64_t)d * S.nt * 18 + ((int64_t)t * 3 + a) * 6 + q % 6];  // incidences of a level: nt*18 apart
    }
    if (side)
      wb[r][q][d] = w;
    else
      wa[r][q][d] = w;
  }
  __syncthreads();
  const int m = m0 + ty, n = n0 + tx;
  if (m >= A.ne || n >= B.ne) return;
  double cr[RC_DC], ci[RC_DC];
#pragma unroll
  for (int d = 0; d < RC_DC; ++d) cr[d] = ci[d] = 0.0;
  for (int q = 0; q < 12; ++q) {
    const double x0 = xa[ty][q][0], x1 = xa[ty][q][1], x2 = xa[ty][q][2];
    const double* nx = na[ty][q / 6];
    double ar[RC_DC], ai[RC_DC];  // sum_p K(q, p) conj(W2_d[p])
#pragma unroll
    for (int d = 0; d < RC_DC; ++d) ar[d] = ai[d] = 0.0;
#pragma unroll 1
    for (int p = 0; p < 12; ++p) {
      const double d0 = x0 - xb[tx][p][0], d1 = x1 - xb[tx][p][1], d2 = x2 - xb[tx][p][2];
      const double* ny = nb[tx][p / 6];
      const double kv = cov_eval(cp, d0 * d0 + d1 * d1 + d2 * d2, nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2]);
#pragma unroll
      for (int d = 0; d < RC_DC; ++d) {
        const c128 w = wb[tx][p][d];
        ar[d] += kv * w.re;
        ai[d] -= kv * w.im;
      }
    }
#pragma unroll
    for (int d = 0; d < RC_DC; ++d) {
      const c128 w = wa[ty][q][d];
      cr[d] += w.re * ar[d] - w.im * ai[d];
      ci[d] += w.re * ai[d] + w.im * ar[d];
    }
  }
#pragma unroll
  for (int d = 0; d < RC_DC; ++d)
    if (d < dc) C[d * dstride + (int64_t)m * ldc + n] = c128{cr[d], ci[d]};
}

void rhs_correlation_multi(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t dir0,
                           int64_t nd, c128* C, int64_t ldc, int64_t dstride) {
  const Mesh& m1 = *l1.mesh;
  const Mesh& m2 = *l2.mesh;
  CovParams cp;
  cp.kind = cov.kind;
  cp.s2 = cov.sigma * cov.sigma;
  cp.inv2l2 = cov.ell > 0 ? 1.0 / (2.0 * cov.ell * cov.ell) : 0.0;
  cp.s3l = cov.ell > 0 ? std::sqrt(3.0) / cov.ell : 0.0;
  dim3 g((unsigned)((m2.h.ne + 15) / 16), (unsigned)((m1.h.ne + 15) / 16));
  for (int64_t c0 = 0; c0 < nd; c0 += RC_DC) {
    EdgeSide A{m1.edge_tri.as<int32_t>(), m1.edge_loc.as<int32_t>(), m1.nrm.as<double>(), l1.qx.as<double>(),
               l1.W.as<c128>() + (dir0 + c0) * m1.h.nt * 18, (int)m1.h.ne, (int)m1.h.nt};
    EdgeSide B{m2.edge_tri.as<int32_t>(), m2.edge_loc.as<int32_t>(), m2.nrm.as<double>(), l2.qx.as<double>(),
               l2.W.as<c128>() + (dir0 + c0) * m2.h.nt * 18, (int)m2.h.ne, (int)m2.h.nt};
    const int dc = (int)std::min<int64_t>(RC_DC, nd - c0);
    hipLaunchKernelGGL(k_rhs_correlation_multi, g, dim3(256), 0, s, A, B, cp, dc, C + c0 * dstride, ldc, dstride);
    FOSB_LAUNCH_CHECK();
  }
}

void rhs_correlation_kernel(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t dir,
                            c128* C, int64_t ldc) {
  const Mesh& m1 = *l1.mesh;
  const Mesh& m2 = *l2.mesh;
  EdgeSide A{m1.edge_tri.as<int32_t>(), m1.edge_loc.as<int32_t>(), m1.nrm.as<double>(), l1.qx.as<double>(),
             l1.W.as<c128>() + dir * m1.h.nt * 18, (int)m1.h.ne, (int)m1.h.nt};
  EdgeSide B{m2.edge_tri.as<int32_t>(), m2.edge_loc.as<int32_t>(), m2.nrm.as<double>(), l2.qx.as<double>(),
             l2.W.as<c128>() + dir * m2.h.nt * 18, (int)m2.h.ne, (int)m2.h.nt};
  CovParams cp;
  cp.kind = cov.kind;
  cp.s2 = cov.sigma * cov.sigma;
  cp.inv2l2 = cov.ell > 0 ? 1.0 / (2.0 * cov.ell * cov.ell) : 0.0;
  cp.s3l = cov.ell > 0 ? std::sqrt(3.0) / cov.ell : 0.0;
  dim3 g((unsigned)((m2.h.ne + 15) / 16), (unsigned)((m1.h.ne + 15) / 16));
  hipLaunchKernelGGL(k_rhs_correlation, g, dim3(256), 0, s, A, B, cp, C, ldc);
  FOSB_LAUNCH_CHECK();
}

// FF[(c*n_a + i)][m] = -i k [(I - x x^T) int phi_m(y) exp(-i k x.y) dy]_c
__global__ void k_far_field_matrix(MeshDev md, Rule6Q R, double k, const double* __restrict__ xh, int n_a,
                                   c128* __restrict__ FF) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (m >= md.ne || i >= n_a) return;
  const double x0 = xh[3 * i], x1 = xh[3 * i + 1], x2 = xh[3 * i + 2];
  double Jr[3] = {0, 0, 0}, Ji[3] = {0, 0, 0};
  for (int side = 0; side < 2; ++side) {
    const int t = md.edge_tri[side * md.ne + m];
    const int a = md.edge_loc[side * md.ne + m];
    double P[3][3];
    tri_vertices(md, t, P);
    const double ha = 0.5 * md.alpha[a * md.nt + t] * md.area[t];
    for (int q = 0; q < 6; ++q) {
      double y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
      double sn, cs;
      sincos(-k * (x0 * y[0] + x1 * y[1] + x2 * y[2]), &sn, &cs);
      const double f = R.w[q] * ha;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ph = f * (y[c] - P[a][c]);
        Jr[c] += ph * cs;
        Ji[c] += ph * sn;
      }
    }
  }
  const double dr = x0 * Jr[0] + x1 * Jr[1] + x2 * Jr[2];
  const double di = x0 * Ji[0] + x1 * Ji[1] + x2 * Ji[2];
  const double xv[3] = {x0, x1, x2};
  for (int c = 0; c < 3; ++c) {
    const double pr = Jr[c] - xv[c] * dr, pi = Ji[c] - xv[c] * di;
    // -i k (pr + i pi) = k pi - i k pr
    FF[((int64_t)c * n_a + i) * md.ne + m] = c128{k * pi, -k * pr};
  }
}

// PMCHWT far field: FF[(c n_a + i)][m] = i k ((I - x x^T) A_m)_c and
// FF[(c n_a + i)][N + m] = -i k (x x A_m)_c, A_m = int phi_m(y) e^{-ik x.y} dy.
__global__ void k_far_field_pmchwt(MeshDev md, Rule6Q R, double k, const double* __restrict__ xh, int n_a,
                                   c128* __restrict__ FF) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (m >= md.ne || i >= n_a) return;
  const double xv[3] = {xh[3 * i], xh[3 * i + 1], xh[3 * i + 2]};
  double Ar[3] = {0, 0, 0}, Ai[3] = {0, 0, 0};
  for (int side = 0; side < 2; ++side) {
    const int t = md.edge_tri[side * md.ne + m];
    const int a = md.edge_loc[side * md.ne + m];
    double P[3][3];
    tri_vertices(md, t, P);
    const double ha = 0.5 * md.alpha[a * md.nt + t] * md.area[t];
    for (int q = 0; q < 6; ++q) {
      double y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
      double sn, cs;
      sincos(-k * (xv[0] * y[0] + xv[1] * y[1] + xv[2] * y[2]), &sn, &cs);
      const double f = R.w[q] * ha;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ph = f * (y[c] - P[a][c]);
        Ar[c] += ph * cs;
        Ai[c] += ph * sn;
      }
    }
  }
  const double dr = xv[0] * Ar[0] + xv[1] * Ar[1] + xv[2] * Ar[2];
  const double di = xv[0] * Ai[0] + xv[1] * Ai[1] + xv[2] * Ai[2];
  const double xr[3] = {xv[1] * Ar[2] - xv[2] * Ar[1], xv[2] * Ar[0] - xv[0] * Ar[2], xv[0] * Ar[1] - xv[1] * Ar[0]};
  const double xi[3] = {xv[1] * Ai[2] - xv[2] * Ai[1], xv[2] * Ai[0] - xv[0] * Ai[2], xv[0] * Ai[1] - xv[1] * Ai[0]};
  const int64_t ld = 2LL * md.ne;
  for (int c = 0; c < 3; ++c) {
    const double pr = Ar[c] - xv[c] * dr, pi = Ai[c] - xv[c] * di;
    // i k (pr + i pi) = -k pi + i k pr;  -i k (xr + i xi) = k xi - i k xr
    FF[((int64_t)c * n_a + i) * ld + m] = c128{-k * pi, k * pr};
    FF[((int64_t)c * n_a + i) * ld + md.ne + m] = c128{k * xi[c], -k * xr[c]};
  }
}

void far_field_matrix_pmchwt(hipStream_t s, const Mesh& m, double k, const double* xhat_dev, int64_t n_a, c128* FF) {
  dim3 g((unsigned)((m.h.ne + 255) / 256), (unsigned)n_a);
  hipLaunchKernelGGL(k_far_field_pmchwt, g, dim3(256), 0, s, m.dev(), make_rule(), k, xhat_dev, (int)n_a, FF);
  FOSB_LAUNCH_CHECK();
}

void far_field_matrix_kernel(hipStream_t s, const Mesh& m, double k, const double* xhat_dev, int64_t n_a, c128* FF) {
  dim3 g((unsigned)((m.h.ne + 255) / 256), (unsigned)n_a);
  hipLaunchKernelGGL(k_far_field_matrix, g, dim3(256), 0, s, m.dev(), make_rule(), k, xhat_dev, (int)n_a, FF);
  FOSB_LAUNCH_CHECK();
}

// NF[(c*n_p + p)][m] = E^sc_c(x_p) of phi_m, E^sc = -E_k phi with
//   E_k phi(x) = i k int G phi + (i/k) grad_x int G div phi,
//   grad_x G(x, y) = (i k - 1/R) G (x - y)/R,  G = e^{ikR}/(4 pi R),
// 6-point rule on both triangles of the RWG (field points off the surface).
__global__ void k_near_field_matrix(MeshDev md, Rule6Q R, double k, const double* __restrict__ xp, int n_p,
                                    c128* __restrict__ NF) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int ip = blockIdx.y;
  if (m >= md.ne || ip >= n_p) return;
  const double x[3] = {xp[3 * ip], xp[3 * ip + 1], xp[3 * ip + 2]};
  double Ar[3] = {0, 0, 0}, Ai[3] = {0, 0, 0};   // int G phi
  double Br[3] = {0, 0, 0}, Bi[3] = {0, 0, 0};   // int grad_x G div phi
  const double inv4pi = 0.25 / M_PI;
  for (int side = 0; side < 2; ++side) {
    const int t = md.edge_tri[side * md.ne + m];
    const int a = md.edge_loc[side * md.ne + m];
    double P[3][3];
    tri_vertices(md, t, P);
    const double al = md.alpha[a * md.nt + t];
    const double ha = 0.5 * al * md.area[t];
    const double dv = al * md.area[t];
    for (int q = 0; q < 6; ++q) {
      double y[3], dx[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        y[c] = R.l[q][0] * P[0][c] + R.l[q][1] * P[1][c] + R.l[q][2] * P[2][c];
        dx[c] = x[c] - y[c];
      }
      const double r = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
      double sn, cs;
      sincos(k * r, &sn, &cs);
      const double g0 = inv4pi / r;                      // G = g0 (cs + i sn)
      const double gr = g0 * cs, gi = g0 * sn;
      // (i k - 1/r) G / r = ((-1/r) gr - k gi + i (k gr - (1/r) gi)) / r
      const double hr = (-gr / r - k * gi) / r, hi = (k * gr - gi / r) / r;
      const double f = R.w[q] * ha, fd = R.w[q] * dv;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ph = f * (y[c] - P[a][c]);
        Ar[c] += ph * gr;
        Ai[c] += ph * gi;
        Br[c] += fd * hr * dx[c];
        Bi[c] += fd * hi * dx[c];
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    // -(i k A + (i/k) B) = (k Ai + Bi/k) - i (k Ar + Br/k)
    NF[((int64_t)c * n_p + ip) * md.ne + m] = c128{k * Ai[c] + Bi[c] / k, -(k * Ar[c] + Br[c] / k)};
  }
}

void near_field_matrix_kernel(hipStream_t s, const Mesh& m, double k, const double* xp_dev, int64_t n_p, c128* NF) {
  dim3 g((unsigned)((m.h.ne + 255) / 256), (unsigned)n_p);
  hipLaunchKernelGGL(k_near_field_matrix, g, dim3(256), 0, s, m.dev(), make_rule(), k, xp_dev, (int)n_p, NF);
  FOSB_LAUNCH_CHECK();
}

// var[r] += scale * Re sum_n P[r][n] conj(F2[r][n]) (P row stride ldp); one
// block per row, fixed order.
__global__ __launch_bounds__(256) void k_row_dot_re(const c128* __restrict__ P, int64_t ldp,
                                                    const c128* __restrict__ F2, int64_t n, double scale,
                                                    double* __restrict__ var) {
  __shared__ double sm[256];
  const int64_t r = blockIdx.x;
  double acc = 0;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const c128 a = P[r * ldp + c], b = F2[r * n + c];
    acc += a.re * b.re + a.im * b.im;
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) var[r] += scale * sm[0];
}

void row_dot_re_accumulate(hipStream_t s, const c128* P, int64_t ldp, const c128* FF2, int64_t rows, int64_t n,
                           double scale, double* var) {
  hipLaunchKernelGGL(k_row_dot_re, dim3((unsigned)rows), dim3(256), 0, s, P, ldp, FF2, n, scale, var);
  FOSB_LAUNCH_CHECK();
}

// out[i][j] += scale * (T[i][j] + conj T[j][i] when both): the combination of
// a pair's angular correlation block with that of its transposed pair.
__global__ __launch_bounds__(256) void k_herm_accumulate(const c128* __restrict__ T, int64_t ldt, int64_t n,
                                                         double scale, int both, c128* __restrict__ out,
                                                         int64_t ldo) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  c128 a = T[i * ldt + j];
  if (both) {
    const c128 b = T[j * ldt + i];
    a.re += b.re;
    a.im -= b.im;
  }
  c128 o = out[i * ldo + j];
  o.re += scale * a.re;
  o.im += scale * a.im;
  out[i * ldo + j] = o;
}

void herm_accumulate(hipStream_t s, const c128* T, int64_t ldt, int64_t n, double scale, bool both, c128* out,
                     int64_t ldo) {
  if (n <= 0) return;
  if (n > 65535) fail(FOSB_E_UNSUPPORTED, "correlation of more than 65535 angles");
  hipLaunchKernelGGL(k_herm_accumulate, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, T, ldt, n,
                     scale, both ? 1 : 0, out, ldo);
  FOSB_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_matvec_rows(const c128* __restrict__ FF, int64_t n, const c128* __restrict__ u,
                                                     c128* __restrict__ out) {
  __shared__ double sr[256], si[256];
  const int64_t r = blockIdx.x;
  double ar = 0, ai = 0;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
    const c128 a = FF[r * n + c], b = u[c];
    ar += a.re * b.re - a.im * b.im;
    ai += a.re * b.im + a.im * b.re;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = c128{sr[0], si[0]};
}

void matvec_rows(hipStream_t s, const c128* FF, int64_t rows, int64_t n, const c128* u, c128* out) {
  hipLaunchKernelGGL(k_matvec_rows, dim3((unsigned)rows), dim3(256), 0, s, FF, n, u, out);
  FOSB_LAUNCH_CHECK();
}


// ------------------------------------------------------------------ adjoint of the variance
// Hn[q][r] = P[r][q] = sum_a conj(B[e(t,a)][r]) W[t][a][j] for node q = 6t + j,
// with B = Z^{-H} FF^H (N x R): the rows of FF Z^{-1} Wgt, one per node.
__global__ __launch_bounds__(256) void k_adjoint_nodes(const int32_t* __restrict__ tri_edge, int nt,
                                                       const c128* __restrict__ W, const c128* __restrict__ B,
                                                       int64_t R, c128* __restrict__ Hn) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int64_t Q = 6LL * nt;
  for (int64_t q = blockIdx.y; q < Q; q += gridDim.y) {
    const int t = (int)(q / 6), j = (int)(q % 6);
    double hr = 0, hi = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int e = tri_edge[a * nt + t];
      const c128 w = W[((int64_t)t * 3 + a) * 6 + j];
      const c128 b = B[(int64_t)e * R + r];
      // conj(b) * w
      hr += b.re * w.re + b.im * w.im;
      hi += b.re * w.im - b.im * w.re;
    }
    Hn[q * R + r] = c128{hr, hi};
  }
}

void adjoint_nodes(hipStream_t s, const Mesh& m, const c128* W, const c128* B, int64_t R, c128* Hn) {
  const int64_t Q = 6LL * m.h.nt;
  dim3 g((unsigned)((R + 255) / 256), (unsigned)std::min<int64_t>(Q, 65535));
  hipLaunchKernelGGL(k_adjoint_nodes, g, dim3(256), 0, s, m.tri_edge.as<int32_t>(), (int)m.h.nt, W, B, R, Hn);
  FOSB_LAUNCH_CHECK();
}

// Correlation function kappa = K / sigma^2 and d kappa / d ell at squared distance r2.
__device__ __forceinline__ void corr_and_dell(const CovParams& cp, double ell, double r2, double ndot, double& kv,
                                              double& dl) {
  switch (cp.kind) {
    case FOSB_COV_GAUSSIAN: {
      kv = exp(-r2 * cp.inv2l2);
      dl = kv * r2 / (ell * ell * ell);
      return;
    }
    case FOSB_COV_MATERN32: {
      const double a = sqrt(r2) * cp.s3l;
      const double ea = exp(-a);
      kv = (1.0 + a) * ea;
      dl = a * a * ea / ell;
      return;
    }
    case FOSB_COV_CONSTANT: kv = 1.0; dl = 0.0; return;
    default: kv = ndot; dl = 0.0; return;
  }
}

// For rows q1 in [a0, a0 + na) of G (row stride Q2) and all columns q2:
// partial[2 b] = scale sum kappa Re G, partial[2 b + 1] = scale sum dkappa/dell Re G,
// one pair of values per block b (16 rows x 256 columns), summed later in block order.
__global__ __launch_bounds__(256) void k_cov_grad_partials(const c128* __restrict__ G, int64_t a0, int64_t na,
                                                           int64_t Q2, const double* __restrict__ x1, int64_t Q1,
                                                           const double* __restrict__ n1, int nt1,
                                                           const double* __restrict__ x2,
                                                           const double* __restrict__ n2, int nt2, CovParams cp,
                                                           double ell, double scale, double* __restrict__ partial) {
  __shared__ double s0[256], s1[256];
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rb = (int64_t)blockIdx.y * 16;
  double acc0 = 0, acc1 = 0;
  if (c < Q2) {
    const double y0 = x2[c], y1 = x2[Q2 + c], y2 = x2[2 * Q2 + c];
    const int t2 = (int)(c / 6);
    const double m0 = n2[t2], m1 = n2[nt2 + t2], m2 = n2[2 * nt2 + t2];
    for (int i = 0; i < 16; ++i) {
      const int64_t rr = rb + i;
      if (rr >= na) break;
      const int64_t q1 = a0 + rr;
      const double d0 = x1[q1] - y0, d1 = x1[Q1 + q1] - y1, d2 = x1[2 * Q1 + q1] - y2;
      const int t1 = (int)(q1 / 6);
      const double nd = n1[t1] * m0 + n1[nt1 + t1] * m1 + n1[2 * nt1 + t1] * m2;
      double kv, dl;
      corr_and_dell(cp, ell, d0 * d0 + d1 * d1 + d2 * d2, nd, kv, dl);
      const double g = G[rr * Q2 + c].re;
      acc0 += kv * g;
      acc1 += dl * g;
    }
  }
  s0[threadIdx.x] = acc0;
  s1[threadIdx.x] = acc1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * b] = scale * s0[0];
    partial[2 * b + 1] = scale * s1[0];
  }
}

int64_t cov_grad_partials(hipStream_t s, const c128* G, int64_t a0, int64_t na, const Level& l1, const Level& l2,
                          const fosb_cov& cov, double scale, double* partial) {
  const Mesh& m1 = *l1.mesh;
  const Mesh& m2 = *l2.mesh;
  const int64_t Q1 = 6LL * m1.h.nt, Q2 = 6LL * m2.h.nt;
  CovParams cp;
  cp.kind = cov.kind;
  cp.s2 = 1.0;
  cp.inv2l2 = cov.ell > 0 ? 1.0 / (2.0 * cov.ell * cov.ell) : 0.0;
  cp.s3l = cov.ell > 0 ? std::sqrt(3.0) / cov.ell : 0.0;
  dim3 g((unsigned)((Q2 + 255) / 256), (unsigned)((na + 15) / 16));
  hipLaunchKernelGGL(k_cov_grad_partials, g, dim3(256), 0, s, G, a0, na, Q2, l1.qx.as<double>(), Q1,
                     m1.nrm.as<double>(), (int)m1.h.nt, l2.qx.as<double>(), m2.nrm.as<double>(), (int)m2.h.nt, cp,
                     cov.ell, scale, partial);
  FOSB_LAUNCH_CHECK();
  return (int64_t)g.x * g.y;
}

// ------------------------------------------------------------------ variance through the adjoint maps
// Kc[rr][c] = K(x1[a0 + rr], x2[c]) + 0i for rr < na (row stride Q2): a row
// chunk of the covariance between the quadrature nodes of two levels.
__global__ __launch_bounds__(256) void k_cov_matrix(int64_t a0, int64_t na, int64_t Q2, const double* __restrict__ x1,
                                                    int64_t Q1, const double* __restrict__ n1, int nt1,
                                                    const double* __restrict__ x2, const double* __restrict__ n2,
                                                    int nt2, CovParams cp, c128* __restrict__ Kc) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= Q2) return;
  const double y0 = x2[c], y1 = x2[Q2 + c], y2 = x2[2 * Q2 + c];
  const int t2 = (int)(c / 6);
  const double m0 = n2[t2], m1 = n2[nt2 + t2], m2 = n2[2 * nt2 + t2];
  for (int64_t rr = blockIdx.y; rr < na; rr += gridDim.y) {
    const int64_t q1 = a0 + rr;
    const double d0 = x1[q1] - y0, d1 = x1[Q1 + q1] - y1, d2 = x1[2 * Q1 + q1] - y2;
    const int t1 = (int)(q1 / 6);
    const double nd = n1[t1] * m0 + n1[nt1 + t1] * m1 + n1[2 * nt1 + t1] * m2;
    Kc[rr * Q2 + c] = c128{cov_eval(cp, d0 * d0 + d1 * d1 + d2 * d2, nd), 0.0};
  }
}

void cov_matrix(hipStream_t s, const Level& l1, const Level& l2, const fosb_cov& cov, int64_t a0, int64_t na,
                c128* Kc) {
  const Mesh& m1 = *l1.mesh;
  const Mesh& m2 = *l2.mesh;
  const int64_t Q1 = 6LL * m1.h.nt, Q2 = 6LL * m2.h.nt;
  CovParams cp;
  cp.kind = cov.kind;
  cp.s2 = cov.sigma * cov.sigma;
  cp.inv2l2 = cov.ell > 0 ? 1.0 / (2.0 * cov.ell * cov.ell) : 0.0;
  cp.s3l = cov.ell > 0 ? std::sqrt(3.0) / cov.ell : 0.0;
  dim3 g((unsigned)((Q2 + 255) / 256), (unsigned)std::min<int64_t>(na, 65535));
  hipLaunchKernelGGL(k_cov_matrix, g, dim3(256), 0, s, a0, na, Q2, l1.qx.as<double>(), Q1, m1.nrm.as<double>(),
                     (int)m1.h.nt, l2.qx.as<double>(), m2.nrm.as<double>(), (int)m2.h.nt, cp, Kc);
  FOSB_LAUNCH_CHECK();
}

// part[b][r] = Re sum over rows q of block b (256 rows of [0, n)) of A[q][r] B[q][r]
// (row stride R for both): 64 columns x 4 row lanes per block.
__global__ __launch_bounds__(256) void k_coldot_partials(const c128* __restrict__ A, const c128* __restrict__ B,
                                                         int64_t n, int64_t R, double* __restrict__ part) {
  __shared__ double sm[4][64];
  const int cl = threadIdx.x & 63, lane = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + cl;
  const int64_t q0 = (int64_t)blockIdx.y * 256;
  double acc = 0;
  if (r < R)
    for (int64_t q = q0 + lane; q < min(n, q0 + 256); q += 4) {
      const c128 a = A[q * R + r], b = B[q * R + r];
      acc += a.re * b.re - a.im * b.im;
    }
  sm[lane][cl] = acc;
  __syncthreads();
  if (lane == 0 && r < R) part[(int64_t)blockIdx.y * R + r] = ((sm[0][cl] + sm[1][cl]) + sm[2][cl]) + sm[3][cl];
}

__global__ __launch_bounds__(256) void k_coldot_finish(const double* __restrict__ part, int nb, int64_t R, double scale,
                                                       double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  double acc = 0;
  for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * R + r];
  out[r] += scale * acc;
}

void coldot_re_accumulate(hipStream_t s, const c128* A, const c128* B, int64_t n, int64_t R, double scale,
                          double* part, double* out) {
  if (n <= 0 || R <= 0) return;
  const int nb = (int)((n + 255) / 256);
  if (nb > 65535) fail(FOSB_E_UNSUPPORTED, "column dot over %lld rows", (long long)n);
  hipLaunchKernelGGL(k_coldot_partials, dim3((unsigned)((R + 63) / 64), (unsigned)nb), dim3(256), 0, s, A, B, n, R,
                     part);
  FOSB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_coldot_finish, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, (const double*)part, nb, R,
                     scale, out);
  FOSB_LAUNCH_CHECK();
}

// out[0] = 2 sigma A, out[1] = sigma^2 B, out[2] = sigma^2 A with (A, B) the
// partial pairs summed in order (one block, fixed reduction tree).
__global__ __launch_bounds__(256) void k_cov_grad_finish(const double* __restrict__ partial, int64_t n, double sigma,
                                                         double* __restrict__ out) {
  __shared__ double s0[256], s1[256];
  double a = 0, b = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = 2.0 * sigma * s0[0];
    out[1] = sigma * sigma * s1[0];
    out[2] = sigma * sigma * s0[0];
  }
}

void cov_grad_finish(hipStream_t s, const double* partial, int64_t n, double sigma, double* out) {
  hipLaunchKernelGGL(k_cov_grad_finish, dim3(1), dim3(256), 0, s, partial, n, sigma, out);
  FOSB_LAUNCH_CHECK();
}

}  // namespace fosb
