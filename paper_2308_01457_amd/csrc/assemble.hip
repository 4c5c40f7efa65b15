// EFIE Galerkin assembly on RWG elements (FP64).
//
//   Z[m][n] = sum over the triangle pairs (T, T') of the supports of phi_m, phi_n of
//     int_T int_T' G_k(x,y) [ -i k phi_m(x).phi_n(y) + (i/k) div phi_m div phi_n ]
//
// Every ordered triangle pair is integrated once ("unassembled" 3x3 block of the
// three local RWG functions of each triangle); the blocks of a band of column
// triangles are written to a scratch matrix Zc (3 nt rows x 3 band columns) and
// then gathered onto the RWG indices.  The gather writes each Z entry from a
// fixed-order sum (store on the band of the edge's T+, add on the band of its T-
// when that lies in a later band), so results are deterministic.
//
// Per triangle pair the integrand is reduced to eight moments (relative to the
// two centroids c, c'):
//   I0 = sum w w' G,  Ix = sum w w' G x~,  Iy = sum w w' G y~,  Ixy = sum w w' G x~.y~
// because phi_a(x).phi_b(y) = (alpha_a beta_b / 4) (x~ - P~_a).(y~ - Q~_b) and
// div phi_a = alpha_a, alpha_a = sign * length / area of local RWG a.
#include <algorithm>
#include <cmath>

#include <functional>
#include <array>
#include <map>

#include "common.h"

namespace fosb {

struct Rule6 {
  double l[6][3];
  double w[6];
};

static constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

// sin and cos of x for the Green's function phase k |x - y|.  Reduction by
// pi/2 in the manner of Cody and Waite (1980): n = rint(2x/pi),
// r = x - n (P1 + P2 + P3) with pi/2 split into three doubles and each product
// applied by one fused multiply-add; then the Taylor series of sin and cos on
// |r| <= pi/4 (about), cut where the first omitted term is below 1e-16 (sin:
// through r^17, cos: through r^16); the quadrant n mod 4 picks and signs the
// pair.  Accurate to about an ulp for |x| up to kTrigPhaseMax, which
// assemble_efie enforces (k times the mesh's bounding-box diagonal).
static constexpr double kTrigPhaseMax = 1.0e5;
__device__ __forceinline__ void sincos_phase(double x, double* sn, double* cs) {
  constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
  constexpr double P1 = 0x1.921fb54442d18p+0, P2 = 0x1.1a62633145c07p-54, P3 = -0x1.f1976b7ed8fbcp-110;
  const double n = rint(x * kTwoOverPi);
  double r = fma(-n, P1, x);
  r = fma(-n, P2, r);
  r = fma(-n, P3, r);
  const double r2 = r * r;
  // coefficients (-1)^j / (2j+1)! and (-1)^j / (2j)!
  double ps = 2.8114572543455206e-15;
  ps = fma(ps, r2, -7.647163731819816e-13);
  ps = fma(ps, r2, 1.6059043836821613e-10);
  ps = fma(ps, r2, -2.505210838544172e-08);
  ps = fma(ps, r2, 2.7557319223985893e-06);
  ps = fma(ps, r2, -0.0001984126984126984);
  ps = fma(ps, r2, 0.008333333333333333);
  ps = fma(ps, r2, -0.16666666666666666);
  ps = fma(ps * r2, r, r);
  double pc = 4.779477332387385e-14;
  pc = fma(pc, r2, -1.1470745597729725e-11);
  pc = fma(pc, r2, 2.08767569878681e-09);
  pc = fma(pc, r2, -2.755731922398589e-07);
  pc = fma(pc, r2, 2.48015873015873e-05);
  pc = fma(pc, r2, -0.001388888888888889);
  pc = fma(pc, r2, 0.041666666666666664);
  pc = fma(pc, r2, -0.5);
  pc = fma(pc, r2, 1.0);
  const int q = (int)n;  // two's complement: its low bits are n mod 4 also for n < 0
  const double s0 = (q & 1) ? pc : ps, c0 = (q & 1) ? ps : pc;
  // negation as a flip of the sign bit: sin for quadrants 2 and 3, cos for 1 and 2
  const unsigned long long fs = (unsigned long long)(q & 2) << 62, fc = (unsigned long long)((q + 1) & 2) << 62;
  *sn = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(s0) ^ fs));
  *cs = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(c0) ^ fc));
}

// 1 / sqrt(x) for a positive finite x (the distance of two points of
// non-touching triangles): the hardware estimate, then one step of the
// second-order Newton iteration for the reciprocal square root,
// y (1 + e/2 + 3e^2/8) with e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(y * -x, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ void write_local_block(const MeshDev& md, int i, int j, int jj, double k,
                                                  const double Li[3][3], const double Lj[3][3], double I0r,
                                                  double I0i, const double Ixr[3], const double Ixi[3],
                                                  const double Iyr[3], const double Iyi[3], double Ixyr,
                                                  double Ixyi, c128* __restrict__ Zc, int64_t ldc) {
  const int nt = md.nt;
  const double ik = 1.0 / k;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double al = md.alpha[a * nt + i];
    const double Pa0 = Li[a][0], Pa1 = Li[a][1], Pa2 = Li[a][2];
    const double PIyr = Pa0 * Iyr[0] + Pa1 * Iyr[1] + Pa2 * Iyr[2];
    const double PIyi = Pa0 * Iyi[0] + Pa1 * Iyi[1] + Pa2 * Iyi[2];
    c128* row = Zc + (int64_t)(3 * i + a) * ldc + 3 * jj;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double be = md.alpha[b * nt + j];
      const double Qb0 = Lj[b][0], Qb1 = Lj[b][1], Qb2 = Lj[b][2];
      const double PQ = Pa0 * Qb0 + Pa1 * Qb1 + Pa2 * Qb2;
      const double Mr = Ixyr - (Ixr[0] * Qb0 + Ixr[1] * Qb1 + Ixr[2] * Qb2) - PIyr + PQ * I0r;
      const double Mi = Ixyi - (Ixi[0] * Qb0 + Ixi[1] * Qb1 + Ixi[2] * Qb2) - PIyi + PQ * I0i;
      // -i k M / 4 + (i / k) I0
      const double zr = 0.25 * k * Mi - I0i * ik;
      const double zi = -0.25 * k * Mr + I0r * ik;
      const double sc = al * be;
      row[b] = c128{zr * sc, zi * sc};
    }
  }
}

__device__ __forceinline__ void load_tri(const MeshDev& md, int t, double P[3][3], double c[3]) {
  const int nt = md.nt;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < 3; ++q) P[v][q] = md.vtx[(v * 3 + q) * nt + t];
#pragma unroll
  for (int q = 0; q < 3; ++q) c[q] = (P[0][q] + P[1][q] + P[2][q]) * (1.0 / 3.0);
}

// One thread per ordered non-touching triangle pair (i, j0 + jj).
__global__ __launch_bounds__(256) void k_assemble_regular(MeshDev md, Rule6 R, double k, int j0, int jc,
                                                          c128* __restrict__ Zc, int64_t ldc) {
  const int jj = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (jj >= jc || i >= md.nt) return;
  const int j = j0 + jj;
  const int nt = md.nt;
  {
    const int a0 = md.fv[i], a1 = md.fv[nt + i], a2 = md.fv[2 * nt + i];
    const int b0 = md.fv[j], b1 = md.fv[nt + j], b2 = md.fv[2 * nt + j];
    if (a0 == b0 || a0 == b1 || a0 == b2 || a1 == b0 || a1 == b1 || a1 == b2 || a2 == b0 || a2 == b1 ||
        a2 == b2)
      return;  // touching pair: integrated by the singular kernel
  }
  double Pi[3][3], Pj[3][3], ci[3], cj[3];
  load_tri(md, i, Pi, ci);
  load_tri(md, j, Pj, cj);
  double Li[3][3], Lj[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Li[v][q] = Pi[v][q] - ci[q];
      Lj[v][q] = Pj[v][q] - cj[q];
    }
  const double Ai = md.area[i], Aj = md.area[j];
  double yq[6][3], wq[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int c = 0; c < 3; ++c) yq[q][c] = R.l[q][0] * Lj[0][c] + R.l[q][1] * Lj[1][c] + R.l[q][2] * Lj[2][c];
    wq[q] = R.w[q] * Aj * kInv4Pi;
  }
  const double dc0 = ci[0] - cj[0], dc1 = ci[1] - cj[1], dc2 = ci[2] - cj[2];
  double I0r = 0, I0i = 0, Ixyr = 0, Ixyi = 0;
  double Ixr[3] = {0, 0, 0}, Ixi[3] = {0, 0, 0}, Iyr[3] = {0, 0, 0}, Iyi[3] = {0, 0, 0};
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double xp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xp[c] = R.l[p][0] * Li[0][c] + R.l[p][1] * Li[1][c] + R.l[p][2] * Li[2][c];
    const double wp = R.w[p] * Ai;
    const double e0 = xp[0] + dc0, e1 = xp[1] + dc1, e2 = xp[2] + dc2;
    double Sr = 0, Si = 0, Syr[3] = {0, 0, 0}, Syi[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double d0 = e0 - yq[q][0], d1 = e1 - yq[q][1], d2 = e2 - yq[q][2];
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double ir = rsqrt_pos(r2);
      const double r = r2 * ir;
      double sn, cs;
      sincos_phase(k * r, &sn, &cs);
      const double g = wq[q] * ir;
      const double gr = cs * g, gi = sn * g;
      Sr += gr;
      Si += gi;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Syr[c] += gr * yq[q][c];
        Syi[c] += gi * yq[q][c];
      }
    }
    I0r += wp * Sr;
    I0i += wp * Si;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ixr[c] += wp * Sr * xp[c];
      Ixi[c] += wp * Si * xp[c];
      Iyr[c] += wp * Syr[c];
      Iyi[c] += wp * Syi[c];
    }
    Ixyr += wp * (xp[0] * Syr[0] + xp[1] * Syr[1] + xp[2] * Syr[2]);
    Ixyi += wp * (xp[0] * Syi[0] + xp[1] * Syi[1] + xp[2] * Syi[2]);
  }
  write_local_block(md, i, j, jj, k, Li, Lj, I0r, I0i, Ixr, Ixi, Iyr, Iyi, Ixyr, Ixyi, Zc, ldc);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wavefront per touching ordered pair; lanes stride over the Sauter-Schwab points.
__global__ __launch_bounds__(256) void k_assemble_singular(MeshDev md, const int32_t* __restrict__ tp_i,
                                                           const int32_t* __restrict__ tp_j,
                                                           const int32_t* __restrict__ tp_kind,
                                                           const int32_t* __restrict__ tp_ord, int pbeg, int pend,
                                                           const double* __restrict__ ss, int off0, int off1,
                                                           int off2, int cnt0, int cnt1, int cnt2, double k, int j0,
                                                           c128* __restrict__ Zc, int64_t ldc) {
  const int p = pbeg + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= pend) return;
  const int i = tp_i[p], j = tp_j[p], kind = tp_kind[p];
  const int* ord = tp_ord + 6 * p;
  double Pi[3][3], Pj[3][3], ci[3], cj[3];
  load_tri(md, i, Pi, ci);
  load_tri(md, j, Pj, cj);
  double Li[3][3], Lj[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Li[v][q] = Pi[v][q] - ci[q];
      Lj[v][q] = Pj[v][q] - cj[q];
    }
  // Sauter-Schwab vertex order (local coordinates)
  double S0[3], S1[3], S2[3], T0[3], T1[3], T2[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    S0[q] = Li[ord[0]][q]; S1[q] = Li[ord[1]][q] - Li[ord[0]][q]; S2[q] = Li[ord[2]][q] - Li[ord[1]][q];
    T0[q] = Lj[ord[3]][q]; T1[q] = Lj[ord[4]][q] - Lj[ord[3]][q]; T2[q] = Lj[ord[5]][q] - Lj[ord[4]][q];
  }
  const double jac = 4.0 * md.area[i] * md.area[j] * kInv4Pi;
  const double dc0 = ci[0] - cj[0], dc1 = ci[1] - cj[1], dc2 = ci[2] - cj[2];
  const int off = kind == 0 ? off0 : (kind == 1 ? off1 : off2);
  const int cnt = kind == 0 ? cnt0 : (kind == 1 ? cnt1 : cnt2);
  double I0r = 0, I0i = 0, Ixyr = 0, Ixyi = 0;
  double Ixr[3] = {0, 0, 0}, Ixi[3] = {0, 0, 0}, Iyr[3] = {0, 0, 0}, Iyi[3] = {0, 0, 0};
  for (int m = lane; m < cnt; m += 64) {
    const double* pt = ss + 5 * (int64_t)(off + m);
    const double x1 = pt[0], x2 = pt[1], y1 = pt[2], y2 = pt[3], w = pt[4];
    double x[3], y[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      x[q] = S0[q] + x1 * S1[q] + x2 * S2[q];
      y[q] = T0[q] + y1 * T1[q] + y2 * T2[q];
    }
    const double d0 = x[0] - y[0] + dc0, d1 = x[1] - y[1] + dc1, d2 = x[2] - y[2] + dc2;
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double g = w * jac * ir;
    const double gr = cs * g, gi = sn * g;
    I0r += gr;
    I0i += gi;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Ixr[q] += gr * x[q];
      Ixi[q] += gi * x[q];
      Iyr[q] += gr * y[q];
      Iyi[q] += gi * y[q];
    }
    const double xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    Ixyr += gr * xy;
    Ixyi += gi * xy;
  }
  I0r = wave_sum(I0r);
  I0i = wave_sum(I0i);
  Ixyr = wave_sum(Ixyr);
  Ixyi = wave_sum(Ixyi);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    Ixr[q] = wave_sum(Ixr[q]);
    Ixi[q] = wave_sum(Ixi[q]);
    Iyr[q] = wave_sum(Iyr[q]);
    Iyi[q] = wave_sum(Iyi[q]);
  }
  if (lane == 0) write_local_block(md, i, j, j - j0, k, Li, Lj, I0r, I0i, Ixr, Ixi, Iyr, Iyi, Ixyr, Ixyi, Zc, ldc);
}

// Z[m][n] for the columns n listed for this band: sum of the (up to) four local
// blocks of the band; store when the band holds T+ of n, add otherwise.  With
// Zl, the final entries are also stored rounded to complex64.
__global__ __launch_bounds__(256) void k_assemble_gather(int ne, const int32_t* __restrict__ edge_tri,
                                                         const int32_t* __restrict__ edge_loc, int j0, int j1,
                                                         const int32_t* __restrict__ cols, int ncols,
                                                         const c128* __restrict__ Zc, int64_t ldc,
                                                         c128* __restrict__ Z, int64_t ldz,
                                                         c64* __restrict__ Zl, int64_t ldl) {
  const int ci = blockIdx.x * 64 + (threadIdx.x & 63);
  const int m = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ci >= ncols || m >= ne) return;
  const int n = cols[ci];
  const int tp = edge_tri[n], tm = edge_tri[ne + n];
  const int64_t rp = 3 * (int64_t)edge_tri[m] + edge_loc[m];
  const int64_t rm = 3 * (int64_t)edge_tri[ne + m] + edge_loc[ne + m];
  double sr = 0.0, si = 0.0;
  const bool has_p = tp >= j0 && tp < j1;
  if (has_p) {
    const int64_t c = 3 * (int64_t)(tp - j0) + edge_loc[n];
    const c128 u = Zc[rp * ldc + c], v = Zc[rm * ldc + c];
    sr += u.re + v.re;
    si += u.im + v.im;
  }
  if (tm >= j0 && tm < j1) {
    const int64_t c = 3 * (int64_t)(tm - j0) + edge_loc[ne + n];
    const c128 u = Zc[rp * ldc + c], v = Zc[rm * ldc + c];
    sr += u.re + v.re;
    si += u.im + v.im;
  }
  c128* z = Z + (int64_t)m * ldz + n;
  c128 out{sr, si};
  if (!has_p) {
    const c128 o = *z;
    out = c128{o.re + sr, o.im + si};
  }
  *z = out;
  // the optional complex64 copy receives the entry once it is final: T- lies
  // in this band (T+ < T-, so an earlier band held T+ if this one does not)
  if (Zl && tm < j1) Zl[(int64_t)m * ldl + n] = c64{(float)out.re, (float)out.im};
}

static void ensure_ss_table(Context& ctx, int n) {
  if (ctx.ss[n].p) return;
  std::vector<double> all, part;
  for (int kind = 0; kind < 3; ++kind) {
    sauter_schwab_points(kind, n, part);
    ctx.ss_off[n][kind] = (int)(all.size() / 5);
    ctx.ss_cnt[n][kind] = (int)(part.size() / 5);
    all.insert(all.end(), part.begin(), part.end());
  }
  upload(ctx.ss[n], all, ctx.stream);
  FOSB_HIP(hipStreamSynchronize(ctx.stream));
}

// Row-gathered band: Zr[m][c] = Zc[r+(m)][c] + Zc[r-(m)][c] for the 3w local
// columns of the band (the edge rows of Z restricted to the band's triangle
// columns; each RWG row is the sum of its two triangles' local rows).
__global__ __launch_bounds__(256) void k_band_rows(int ne, const int32_t* __restrict__ edge_tri,
                                                   const int32_t* __restrict__ edge_loc, int ncol,
                                                   const c128* __restrict__ Zc, int64_t ldc, c128* __restrict__ Zr) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int m = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= ncol || m >= ne) return;
  const int64_t rp = 3 * (int64_t)edge_tri[m] + edge_loc[m];
  const int64_t rm = 3 * (int64_t)edge_tri[ne + m] + edge_loc[ne + m];
  const c128 u = Zc[rp * ldc + c], v = Zc[rm * ldc + c];
  Zr[(int64_t)m * ncol + c] = c128{u.re + v.re, u.im + v.im};
}

// Xt[3 (t - j0) + a][:] = X[edge(t, a)][:] for the band's triangles.
__global__ __launch_bounds__(256) void k_band_gather_x(int nt, const int32_t* __restrict__ tri_edge, int j0, int w,
                                                       const c128* __restrict__ X, int64_t ldx, int64_t nrhs,
                                                       c128* __restrict__ Xt) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;   // 0 .. 3w-1
  if (c >= nrhs || r >= 3 * w) return;
  const int t = j0 + r / 3, a = r % 3;
  const int e = tri_edge[a * nt + t];
  Xt[(int64_t)r * nrhs + c] = X[(int64_t)e * ldx + c];
}

// As k_assemble_gather, into a complex64 matrix: the first part of a column is
// rounded and stored, the second added to it in FP64 and rounded again.
__global__ __launch_bounds__(256) void k_assemble_gather_c64(int ne, const int32_t* __restrict__ edge_tri,
                                                             const int32_t* __restrict__ edge_loc, int j0, int j1,
                                                             const int32_t* __restrict__ cols, int ncols,
                                                             const c128* __restrict__ Zc, int64_t ldc,
                                                             c64* __restrict__ Z, int64_t ldz) {
  const int ci = blockIdx.x * 64 + (threadIdx.x & 63);
  const int m = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ci >= ncols || m >= ne) return;
  const int n = cols[ci];
  const int tp = edge_tri[n], tm = edge_tri[ne + n];
  const int64_t rp = 3 * (int64_t)edge_tri[m] + edge_loc[m];
  const int64_t rm = 3 * (int64_t)edge_tri[ne + m] + edge_loc[ne + m];
  double sr = 0.0, si = 0.0;
  const bool has_p = tp >= j0 && tp < j1;
  if (has_p) {
    const int64_t c = 3 * (int64_t)(tp - j0) + edge_loc[n];
    const c128 u = Zc[rp * ldc + c], v = Zc[rm * ldc + c];
    sr += u.re + v.re;
    si += u.im + v.im;
  }
  if (tm >= j0 && tm < j1) {
    const int64_t c = 3 * (int64_t)(tm - j0) + edge_loc[ne + n];
    const c128 u = Zc[rp * ldc + c], v = Zc[rm * ldc + c];
    sr += u.re + v.re;
    si += u.im + v.im;
  }
  c64* z = Z + (int64_t)m * ldz + n;
  if (has_p) {
    *z = c64{(float)sr, (float)si};
  } else {
    const c64 o = *z;
    *z = c64{(float)((double)o.re + sr), (float)((double)o.im + si)};
  }
}

namespace {
// Triangle-column bands of the local EFIE blocks.  For each band [j0, j1) of
// column triangles, the regular and touching-pair kernels fill Zc (3 nt x 3 w
// local blocks, row stride ldc) and sink(stream, j0, j1, Zc, ldc, cols, ncols)
// consumes it on the given stream; cols lists the RWG columns whose T+ or T-
// lies in the band.  The band buffer holds about `budget` bytes.  With a
// second context `sg`, two band buffers alternate and the sink runs on sg's
// stream: band b + 1 is integrated (VALU-bound) while band b is consumed
// (memory-bound), and a buffer is refilled only after its previous sink ran.
// The sinks still run in band order, on one stream.
template <typename Sink>
void assemble_bands(Context& ctx, const Mesh& m, double k, int n_gauss, int64_t budget, Sink&& sink,
                    Context* sg = nullptr) {
  hipStream_t s = ctx.stream;
  const MeshHost& h = m.h;
  const int nt = (int)h.nt, ne = (int)h.ne;
  {  // every phase k |x - y| stays within the range of sincos_phase
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < h.nv; ++v)
      for (int q = 0; q < 3; ++q) {
        lo[q] = std::min(lo[q], h.V[3 * v + q]);
        hi[q] = std::max(hi[q], h.V[3 * v + q]);
      }
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    if (!(k * diag <= kTrigPhaseMax))
      fail(FOSB_E_INVALID, "k * (mesh bounding-box diagonal) = %g exceeds %g", k * diag, kTrigPhaseMax);
  }
  ensure_ss_table(ctx, n_gauss);
  Rule6 R;
  rule6(R.l, R.w);
  int jc = (int)std::max<int64_t>(1, std::min<int64_t>(nt, budget / (9LL * nt * (int64_t)sizeof(c128))));
  if (jc < nt) jc = std::max(64, jc / 64 * 64);
  jc = std::min(jc, nt);
  const int64_t ldc = 3LL * jc;
  const size_t band_bytes = (size_t)(3LL * nt) * ldc * sizeof(c128);
  DevBuf band(band_bytes), band2;
  c128* Zbuf[2] = {band.as<c128>(), nullptr};
  struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;   // [0, 1]: band buffer filled; [2, 3]: band buffer consumed
  const bool two = sg != nullptr && nt > jc;
  if (two) {
    band2.alloc(band_bytes);
    Zbuf[1] = band2.as<c128>();
    for (hipEvent_t& x : ev.e) FOSB_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  }
  // column lists per band (host): edges whose T+ or T- lies in the band
  std::vector<int32_t> cols;
  std::vector<int64_t> cbeg;
  for (int j0 = 0; j0 < nt; j0 += jc) {
    const int j1 = std::min(nt, j0 + jc);
    cbeg.push_back((int64_t)cols.size());
    for (int e = 0; e < ne; ++e) {
      int tp = h.edge_tri[2 * e], tm = h.edge_tri[2 * e + 1];
      if ((tp >= j0 && tp < j1) || (tm >= j0 && tm < j1)) cols.push_back(e);
    }
  }
  cbeg.push_back((int64_t)cols.size());
  DevBuf dcols;
  upload(dcols, cols, s);
  const MeshDev md = m.dev();
  int bi = 0;
  for (int j0 = 0; j0 < nt; j0 += jc, ++bi) {
    const int j1 = std::min(nt, j0 + jc);
    const int w = j1 - j0;
    const int buf = two ? (bi & 1) : 0;
    c128* Zc = Zbuf[buf];
    if (two && bi >= 2) FOSB_HIP(hipStreamWaitEvent(s, ev.e[2 + buf], 0));   // band bi - 2 consumed
    dim3 g1((w + 63) / 64, (nt + 3) / 4);
    hipLaunchKernelGGL(k_assemble_regular, g1, dim3(256), 0, s, md, R, k, j0, w, Zc, ldc);
    FOSB_LAUNCH_CHECK();
    const int pb = (int)(std::lower_bound(h.tp_j.begin(), h.tp_j.end(), j0) - h.tp_j.begin());
    const int pe = (int)(std::lower_bound(h.tp_j.begin(), h.tp_j.end(), j1) - h.tp_j.begin());
    if (pe > pb) {
      dim3 g2((pe - pb + 3) / 4);
      hipLaunchKernelGGL(k_assemble_singular, g2, dim3(256), 0, s, md, m.tp_i.as<int32_t>(), m.tp_j.as<int32_t>(),
                         m.tp_kind.as<int32_t>(), m.tp_ord.as<int32_t>(), pb, pe, ctx.ss[n_gauss].as<double>(),
                         ctx.ss_off[n_gauss][0], ctx.ss_off[n_gauss][1], ctx.ss_off[n_gauss][2],
                         ctx.ss_cnt[n_gauss][0], ctx.ss_cnt[n_gauss][1], ctx.ss_cnt[n_gauss][2], k, j0, Zc, ldc);
      FOSB_LAUNCH_CHECK();
    }
    const int32_t* bc = dcols.as<int32_t>() + cbeg[bi];
    const int nbc = (int)(cbeg[bi + 1] - cbeg[bi]);
    if (two) {
      FOSB_HIP(hipEventRecord(ev.e[buf], s));
      FOSB_HIP(hipStreamWaitEvent(sg->stream, ev.e[buf], 0));
      sink(sg->stream, j0, j1, (const c128*)Zc, ldc, bc, nbc);
      FOSB_HIP(hipEventRecord(ev.e[2 + buf], sg->stream));
    } else {
      sink(s, j0, j1, (const c128*)Zc, ldc, bc, nbc);
    }
  }
  if (two) FOSB_HIP(hipStreamWaitEvent(s, ev.e[2 + ((bi - 1) & 1)], 0));   // the last band consumed
  // the band buffers and the column lists must live until the kernels ran
  FOSB_HIP(hipStreamSynchronize(s));
}
}  // namespace

void assemble_efie(Context& ctx, const Mesh& m, double k, int n_gauss, c128* Z, int64_t ldz, c64* Zl,
                   int64_t ldl) {
  // 1 GiB bands: at nt = 20480 these assembled faster than 256 and 512 MiB ones, and about as fast as 2 GiB
  const int ne = (int)m.h.ne;
  const MeshDev md = m.dev();
  assemble_bands(
      ctx, m, k, n_gauss, (int64_t)1024 << 20,
      [&](hipStream_t st, int j0, int j1, const c128* Zc, int64_t ldc, const int32_t* cols, int nc) {
        if (nc <= 0) return;
        dim3 g3((nc + 63) / 64, (ne + 3) / 4);
        hipLaunchKernelGGL(k_assemble_gather, g3, dim3(256), 0, st, ne, md.edge_tri, md.edge_loc, j0, j1, cols, nc,
                           Zc, ldc, Z, ldz, Zl, ldl);
        FOSB_LAUNCH_CHECK();
      },
      &ctx.la_context());
}

void assemble_efie_c64(Context& ctx, const Mesh& m, double k, int n_gauss, c64* Z, int64_t ldz) {
  const int ne = (int)m.h.ne;
  const MeshDev md = m.dev();
  assemble_bands(
      ctx, m, k, n_gauss, (int64_t)1024 << 20,
      [&](hipStream_t st, int j0, int j1, const c128* Zc, int64_t ldc, const int32_t* cols, int nc) {
        if (nc <= 0) return;
        dim3 g3((nc + 63) / 64, (ne + 3) / 4);
        hipLaunchKernelGGL(k_assemble_gather_c64, g3, dim3(256), 0, st, ne, md.edge_tri, md.edge_loc, j0, j1, cols,
                           nc, Zc, ldc, Z, ldz);
        FOSB_LAUNCH_CHECK();
      },
      &ctx.la_context());
}

// ------------------------------------------------------------------ PMCHWT (dielectric) blocks
//
// The MFIO pairing of two RWG functions,
//   K[m][n] = int int phi_m(x) . (grad_x G_k(x, y) x phi_n(y)) dx dy,
//   grad_x G_k = g (x - y),  g = (i k R - 1) exp(i k R) / (4 pi R^3),
// reduces per triangle pair to ten moments.  With phi_a(x) = (alpha_a / 2)(x - P_a),
// phi_b(y) = (beta_b / 2)(y - Q_b) and x - y = (x - P_a) - (y - Q_b) + (P_a - Q_b),
// the triple product (x - P_a) . ((x - y) x (y - Q_b)) equals
// (P_a - Q_b) . ((y - Q_b) x (x - P_a)); relative to the centroids
// (x = c + x~, y = c' + y~) it is linear in
//   K0 = sum g,  Kx = sum g x~,  Ky = sum g y~,  Kyx = sum g (y~ x x~):
//   blk[a][b] = (alpha_a beta_b / 4) (dc + P~_a - Q~_b) . (Kyx - Ky x P~_a - Q~_b x Kx + (Q~_b x P~_a) K0).
// On identical (flat) triangles all three vectors lie in the plane and the
// integrand vanishes, so those blocks are zero.

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void write_local_block_k(const MeshDev& md, int i, int j, int jj, const double Li[3][3],
                                                    const double Lj[3][3], const double dc[3], double K0r, double K0i,
                                                    const double Kxr[3], const double Kxi[3], const double Kyr[3],
                                                    const double Kyi[3], const double Kyxr[3], const double Kyxi[3],
                                                    c128* __restrict__ Kc, int64_t ldc) {
  const int nt = md.nt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double al = md.alpha[a * nt + i];
    const double Pa[3] = {Li[a][0], Li[a][1], Li[a][2]};
    double KyPr[3], KyPi[3];
    cross3(Kyr, Pa, KyPr);
    cross3(Kyi, Pa, KyPi);
    c128* row = Kc + (int64_t)(3 * i + a) * ldc + 3 * jj;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double be = md.alpha[b * nt + j];
      const double Qb[3] = {Lj[b][0], Lj[b][1], Lj[b][2]};
      double QKxr[3], QKxi[3], QP[3];
      cross3(Qb, Kxr, QKxr);
      cross3(Qb, Kxi, QKxi);
      cross3(Qb, Pa, QP);
      double vr = 0, vi = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double cab = dc[c] + Pa[c] - Qb[c];
        vr += cab * (Kyxr[c] - KyPr[c] - QKxr[c] + QP[c] * K0r);
        vi += cab * (Kyxi[c] - KyPi[c] - QKxi[c] + QP[c] * K0i);
      }
      const double sc = 0.25 * al * be;
      row[b] = c128{vr * sc, vi * sc};
    }
  }
}

// One thread per ordered non-touching triangle pair (i, j0 + jj): the EFIE
// block into Tc and the MFIO block into Kc, from the same point pairs.
__global__ __launch_bounds__(256) void k_pm_regular(MeshDev md, Rule6 R, double k, int j0, int jc,
                                                    c128* __restrict__ Tc, c128* __restrict__ Kc, int64_t ldc) {
  const int jj = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (jj >= jc || i >= md.nt) return;
  const int j = j0 + jj;
  const int nt = md.nt;
  {
    const int a0 = md.fv[i], a1 = md.fv[nt + i], a2 = md.fv[2 * nt + i];
    const int b0 = md.fv[j], b1 = md.fv[nt + j], b2 = md.fv[2 * nt + j];
    if (a0 == b0 || a0 == b1 || a0 == b2 || a1 == b0 || a1 == b1 || a1 == b2 || a2 == b0 || a2 == b1 ||
        a2 == b2)
      return;  // touching pair: integrated by k_pm_singular
  }
  double Pi[3][3], Pj[3][3], ci[3], cj[3];
  load_tri(md, i, Pi, ci);
  load_tri(md, j, Pj, cj);
  double Li[3][3], Lj[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Li[v][q] = Pi[v][q] - ci[q];
      Lj[v][q] = Pj[v][q] - cj[q];
    }
  const double Ai = md.area[i], Aj = md.area[j];
  double yq[6][3], wq[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
#pragma unroll
    for (int c = 0; c < 3; ++c) yq[q][c] = R.l[q][0] * Lj[0][c] + R.l[q][1] * Lj[1][c] + R.l[q][2] * Lj[2][c];
    wq[q] = R.w[q] * Aj * kInv4Pi;
  }
  const double dc[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
  double I0r = 0, I0i = 0, Ixyr = 0, Ixyi = 0;
  double Ixr[3] = {0, 0, 0}, Ixi[3] = {0, 0, 0}, Iyr[3] = {0, 0, 0}, Iyi[3] = {0, 0, 0};
  double K0r = 0, K0i = 0;
  double Kxr[3] = {0, 0, 0}, Kxi[3] = {0, 0, 0}, Kyr[3] = {0, 0, 0}, Kyi[3] = {0, 0, 0};
  double Kyxr[3] = {0, 0, 0}, Kyxi[3] = {0, 0, 0};
  for (int p = 0; p < 6; ++p) {
    double xp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xp[c] = R.l[p][0] * Li[0][c] + R.l[p][1] * Li[1][c] + R.l[p][2] * Li[2][c];
    const double wp = R.w[p] * Ai;
    const double e0 = xp[0] + dc[0], e1 = xp[1] + dc[1], e2 = xp[2] + dc[2];
    double Sr = 0, Si = 0, Syr[3] = {0, 0, 0}, Syi[3] = {0, 0, 0};
    double Tr = 0, Ti = 0, Tyr[3] = {0, 0, 0}, Tyi[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double d0 = e0 - yq[q][0], d1 = e1 - yq[q][1], d2 = e2 - yq[q][2];
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double ir = rsqrt_pos(r2);
      const double r = r2 * ir;
      double sn, cs;
      sincos_phase(k * r, &sn, &cs);
      const double g = wq[q] * ir;
      const double gr = cs * g, gi = sn * g;
      // (i k R - 1) / R^2 times G
      const double ir2 = ir * ir, kr = k * r;
      const double hr = (-gr - gi * kr) * ir2, hi = (gr * kr - gi) * ir2;
      Sr += gr;
      Si += gi;
      Tr += hr;
      Ti += hi;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Syr[c] += gr * yq[q][c];
        Syi[c] += gi * yq[q][c];
        Tyr[c] += hr * yq[q][c];
        Tyi[c] += hi * yq[q][c];
      }
    }
    I0r += wp * Sr;
    I0i += wp * Si;
    K0r += wp * Tr;
    K0i += wp * Ti;
    double cyr[3], cyi[3];
    cross3(Tyr, xp, cyr);
    cross3(Tyi, xp, cyi);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ixr[c] += wp * Sr * xp[c];
      Ixi[c] += wp * Si * xp[c];
      Iyr[c] += wp * Syr[c];
      Iyi[c] += wp * Syi[c];
      Kxr[c] += wp * Tr * xp[c];
      Kxi[c] += wp * Ti * xp[c];
      Kyr[c] += wp * Tyr[c];
      Kyi[c] += wp * Tyi[c];
      Kyxr[c] += wp * cyr[c];
      Kyxi[c] += wp * cyi[c];
    }
    Ixyr += wp * (xp[0] * Syr[0] + xp[1] * Syr[1] + xp[2] * Syr[2]);
    Ixyi += wp * (xp[0] * Syi[0] + xp[1] * Syi[1] + xp[2] * Syi[2]);
  }
  write_local_block(md, i, j, jj, k, Li, Lj, I0r, I0i, Ixr, Ixi, Iyr, Iyi, Ixyr, Ixyi, Tc, ldc);
  write_local_block_k(md, i, j, jj, Li, Lj, dc, K0r, K0i, Kxr, Kxi, Kyr, Kyi, Kyxr, Kyxi, Kc, ldc);
}

// One wavefront per touching ordered pair (Sauter-Schwab points over the lanes):
// EFIE block into Tc, MFIO block into Kc (zero for identical triangles).
__global__ __launch_bounds__(256) void k_pm_singular(MeshDev md, const int32_t* __restrict__ tp_i,
                                                     const int32_t* __restrict__ tp_j,
                                                     const int32_t* __restrict__ tp_kind,
                                                     const int32_t* __restrict__ tp_ord, int pbeg, int pend,
                                                     const double* __restrict__ ss, int off0, int off1, int off2,
                                                     int cnt0, int cnt1, int cnt2, double k, int j0,
                                                     c128* __restrict__ Tc, c128* __restrict__ Kc, int64_t ldc) {
  const int p = pbeg + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= pend) return;
  const int i = tp_i[p], j = tp_j[p], kind = tp_kind[p];
  const int* ord = tp_ord + 6 * p;
  double Pi[3][3], Pj[3][3], ci[3], cj[3];
  load_tri(md, i, Pi, ci);
  load_tri(md, j, Pj, cj);
  double Li[3][3], Lj[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Li[v][q] = Pi[v][q] - ci[q];
      Lj[v][q] = Pj[v][q] - cj[q];
    }
  double S0[3], S1[3], S2[3], T0[3], T1[3], T2[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    S0[q] = Li[ord[0]][q]; S1[q] = Li[ord[1]][q] - Li[ord[0]][q]; S2[q] = Li[ord[2]][q] - Li[ord[1]][q];
    T0[q] = Lj[ord[3]][q]; T1[q] = Lj[ord[4]][q] - Lj[ord[3]][q]; T2[q] = Lj[ord[5]][q] - Lj[ord[4]][q];
  }
  const double jac = 4.0 * md.area[i] * md.area[j] * kInv4Pi;
  const double dc[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
  const int off = kind == 0 ? off0 : (kind == 1 ? off1 : off2);
  const int cnt = kind == 0 ? cnt0 : (kind == 1 ? cnt1 : cnt2);
  const bool with_k = kind != 0;
  double I0r = 0, I0i = 0, Ixyr = 0, Ixyi = 0;
  double Ixr[3] = {0, 0, 0}, Ixi[3] = {0, 0, 0}, Iyr[3] = {0, 0, 0}, Iyi[3] = {0, 0, 0};
  double K0r = 0, K0i = 0;
  double Kxr[3] = {0, 0, 0}, Kxi[3] = {0, 0, 0}, Kyr[3] = {0, 0, 0}, Kyi[3] = {0, 0, 0};
  double Kyxr[3] = {0, 0, 0}, Kyxi[3] = {0, 0, 0};
  for (int m = lane; m < cnt; m += 64) {
    const double* pt = ss + 5 * (int64_t)(off + m);
    const double x1 = pt[0], x2 = pt[1], y1 = pt[2], y2 = pt[3], w = pt[4];
    double x[3], y[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      x[q] = S0[q] + x1 * S1[q] + x2 * S2[q];
      y[q] = T0[q] + y1 * T1[q] + y2 * T2[q];
    }
    const double d0 = x[0] - y[0] + dc[0], d1 = x[1] - y[1] + dc[1], d2 = x[2] - y[2] + dc[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double g = w * jac * ir;
    const double gr = cs * g, gi = sn * g;
    I0r += gr;
    I0i += gi;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Ixr[q] += gr * x[q];
      Ixi[q] += gi * x[q];
      Iyr[q] += gr * y[q];
      Iyi[q] += gi * y[q];
    }
    const double xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    Ixyr += gr * xy;
    Ixyi += gi * xy;
    if (with_k) {
      const double ir2 = ir * ir, kr = k * r;
      const double hr = (-gr - gi * kr) * ir2, hi = (gr * kr - gi) * ir2;
      double yx[3];
      cross3(y, x, yx);
      K0r += hr;
      K0i += hi;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        Kxr[q] += hr * x[q];
        Kxi[q] += hi * x[q];
        Kyr[q] += hr * y[q];
        Kyi[q] += hi * y[q];
        Kyxr[q] += hr * yx[q];
        Kyxi[q] += hi * yx[q];
      }
    }
  }
  I0r = wave_sum(I0r);
  I0i = wave_sum(I0i);
  Ixyr = wave_sum(Ixyr);
  Ixyi = wave_sum(Ixyi);
  K0r = wave_sum(K0r);
  K0i = wave_sum(K0i);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    Ixr[q] = wave_sum(Ixr[q]);
    Ixi[q] = wave_sum(Ixi[q]);
    Iyr[q] = wave_sum(Iyr[q]);
    Iyi[q] = wave_sum(Iyi[q]);
    Kxr[q] = wave_sum(Kxr[q]);
    Kxi[q] = wave_sum(Kxi[q]);
    Kyr[q] = wave_sum(Kyr[q]);
    Kyi[q] = wave_sum(Kyi[q]);
    Kyxr[q] = wave_sum(Kyxr[q]);
    Kyxi[q] = wave_sum(Kyxi[q]);
  }
  if (lane == 0) {
    write_local_block(md, i, j, j - j0, k, Li, Lj, I0r, I0i, Ixr, Ixi, Iyr, Iyi, Ixyr, Ixyi, Tc, ldc);
    write_local_block_k(md, i, j, j - j0, Li, Lj, dc, K0r, K0i, Kxr, Kxi, Kyr, Kyi, Kyxr, Kyxi, Kc, ldc);
  }
}

// The 2N x 2N PMCHWT matrix from one band of local blocks at both
// wavenumbers (EFIE T0, T1 and MFIO K0, K1, same layout):
//   Z[m][n] = T0 + eta T1,  Z[m][N+n] = K0 + K1,  Z[N+m][n] = -(K0 + K1),
//   Z[N+m][N+n] = T0 + T1/eta,
// each block the sum of the (up to) four local blocks of the band.  Stored
// when the band holds T+ of n, added otherwise (the band of T- when it comes
// later), so every entry is a fixed-order sum.
__global__ __launch_bounds__(256) void k_pm_gather(int ne, const int32_t* __restrict__ edge_tri,
                                                   const int32_t* __restrict__ edge_loc, int j0, int j1,
                                                   const int32_t* __restrict__ cols, int ncols,
                                                   const c128* __restrict__ T0c, const c128* __restrict__ K0c,
                                                   const c128* __restrict__ T1c, const c128* __restrict__ K1c,
                                                   int64_t ldc, double eta, c128* __restrict__ Z, int64_t ldz) {
  const int ci = blockIdx.x * 64 + (threadIdx.x & 63);
  const int m = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ci >= ncols || m >= ne) return;
  const int n = cols[ci];
  const int tp = edge_tri[n], tm = edge_tri[ne + n];
  const int64_t rp = 3 * (int64_t)edge_tri[m] + edge_loc[m];
  const int64_t rm = 3 * (int64_t)edge_tri[ne + m] + edge_loc[ne + m];
  double t0r = 0, t0i = 0, t1r = 0, t1i = 0, kr = 0, ki = 0;
  auto add = [&](int64_t c) {
    const c128 a = T0c[rp * ldc + c], b = T0c[rm * ldc + c];
    const c128 e = T1c[rp * ldc + c], f = T1c[rm * ldc + c];
    const c128 x = K0c[rp * ldc + c], y = K0c[rm * ldc + c];
    const c128 u = K1c[rp * ldc + c], v = K1c[rm * ldc + c];
    t0r += a.re + b.re;
    t0i += a.im + b.im;
    t1r += e.re + f.re;
    t1i += e.im + f.im;
    kr += (x.re + y.re) + (u.re + v.re);
    ki += (x.im + y.im) + (u.im + v.im);
  };
  const bool has_p = tp >= j0 && tp < j1;
  if (has_p) add(3 * (int64_t)(tp - j0) + edge_loc[n]);
  if (tm >= j0 && tm < j1) add(3 * (int64_t)(tm - j0) + edge_loc[ne + n]);
  const double ie = 1.0 / eta;
  const c128 v00{t0r + eta * t1r, t0i + eta * t1i}, v01{kr, ki}, v10{-kr, -ki}, v11{t0r + ie * t1r, t0i + ie * t1i};
  c128* z00 = Z + (int64_t)m * ldz + n;
  c128* z01 = z00 + ne;
  c128* z10 = Z + (int64_t)(ne + m) * ldz + n;
  c128* z11 = z10 + ne;
  if (has_p) {
    *z00 = v00;
    *z01 = v01;
    *z10 = v10;
    *z11 = v11;
  } else {
    c128 o = *z00;
    *z00 = c128{o.re + v00.re, o.im + v00.im};
    o = *z01;
    *z01 = c128{o.re + v01.re, o.im + v01.im};
    o = *z10;
    *z10 = c128{o.re + v10.re, o.im + v10.im};
    o = *z11;
    *z11 = c128{o.re + v11.re, o.im + v11.im};
  }
}

void assemble_pmchwt(Context& ctx, const Mesh& m, double k0, double eps_r, double mu_r, int n_gauss, c128* Z,
                     int64_t ldz) {
  hipStream_t s = ctx.stream;
  const MeshHost& h = m.h;
  const int nt = (int)h.nt, ne = (int)h.ne;
  const double k1 = k0 * std::sqrt(eps_r * mu_r), eta = std::sqrt(mu_r / eps_r);
  ensure_ss_table(ctx, n_gauss);
  Rule6 R;
  rule6(R.l, R.w);
  // four band buffers (EFIE and MFIO blocks at k0 and k1) of up to 256 MiB each
  const int64_t budget = (int64_t)256 << 20;
  int jc = (int)std::max<int64_t>(1, std::min<int64_t>(nt, budget / (9LL * nt * (int64_t)sizeof(c128))));
  if (jc < nt) jc = std::max(64, jc / 64 * 64);
  jc = std::min(jc, nt);
  const int64_t ldc = 3LL * jc;
  const size_t bb = (size_t)(3LL * nt) * ldc * sizeof(c128);
  DevBuf band[4] = {DevBuf(bb), DevBuf(bb), DevBuf(bb), DevBuf(bb)};   // T0, K0, T1, K1
  std::vector<int32_t> cols;
  std::vector<int64_t> cbeg;
  for (int j0 = 0; j0 < nt; j0 += jc) {
    const int j1 = std::min(nt, j0 + jc);
    cbeg.push_back((int64_t)cols.size());
    for (int e = 0; e < ne; ++e) {
      const int tp = h.edge_tri[2 * e], tm = h.edge_tri[2 * e + 1];
      if ((tp >= j0 && tp < j1) || (tm >= j0 && tm < j1)) cols.push_back(e);
    }
  }
  cbeg.push_back((int64_t)cols.size());
  DevBuf dcols;
  upload(dcols, cols, s);
  const MeshDev md = m.dev();
  const double kk[2] = {k0, k1};
  int bi = 0;
  for (int j0 = 0; j0 < nt; j0 += jc, ++bi) {
    const int j1 = std::min(nt, j0 + jc);
    const int w = j1 - j0;
    const int pb = (int)(std::lower_bound(h.tp_j.begin(), h.tp_j.end(), j0) - h.tp_j.begin());
    const int pe = (int)(std::lower_bound(h.tp_j.begin(), h.tp_j.end(), j1) - h.tp_j.begin());
    for (int q = 0; q < 2; ++q) {
      c128* Tc = band[2 * q].as<c128>();
      c128* Kc = band[2 * q + 1].as<c128>();
      dim3 g1((w + 63) / 64, (nt + 3) / 4);
      hipLaunchKernelGGL(k_pm_regular, g1, dim3(256), 0, s, md, R, kk[q], j0, w, Tc, Kc, ldc);
      FOSB_LAUNCH_CHECK();
      if (pe > pb) {
        dim3 g2((pe - pb + 3) / 4);
        hipLaunchKernelGGL(k_pm_singular, g2, dim3(256), 0, s, md, m.tp_i.as<int32_t>(), m.tp_j.as<int32_t>(),
                           m.tp_kind.as<int32_t>(), m.tp_ord.as<int32_t>(), pb, pe, ctx.ss[n_gauss].as<double>(),
                           ctx.ss_off[n_gauss][0], ctx.ss_off[n_gauss][1], ctx.ss_off[n_gauss][2],
                           ctx.ss_cnt[n_gauss][0], ctx.ss_cnt[n_gauss][1], ctx.ss_cnt[n_gauss][2], kk[q], j0, Tc,
                           Kc, ldc);
        FOSB_LAUNCH_CHECK();
      }
    }
    const int nc = (int)(cbeg[bi + 1] - cbeg[bi]);
    if (nc > 0) {
      dim3 g3((nc + 63) / 64, (ne + 3) / 4);
      hipLaunchKernelGGL(k_pm_gather, g3, dim3(256), 0, s, ne, md.edge_tri, md.edge_loc, j0, j1,
                         dcols.as<int32_t>() + cbeg[bi], nc, band[0].as<c128>(), band[1].as<c128>(),
                         band[2].as<c128>(), band[3].as<c128>(), ldc, eta, Z, ldz);
      FOSB_LAUNCH_CHECK();
    }
  }
  FOSB_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ dielectric shape-derivative right-hand side
//
// W (2N x 6 nt) maps the perturbation amplitude at the 6-point nodes to the
// PMCHWT right-hand side of the shape derivative (non-magnetic interior):
//   r_E = -eta <E_k1 b> - <H_k1 a> + 1/2 <n x a>,   r_H = -<H_k1 b> + <E_k1 a>/eta + 1/2 <n x b>,
// with the jumps a = curl_G psi, psi = v_n (1 - 1/eps_r) E^0_n, E^0_n = -(i/k0) div J, and
// b = i k0 (1 - eps_r) v_n E_t, E_t = n x M, and (by parts onto the kernel)
//   <E_k a> = i k int int phi_m . (grad_x G x n_y) psi,  <n x a> = -int psi div phi_m,
//   <H_k a> = k^2 int int G phi_m . n_y psi - int int div phi_m (grad_x G . n_y) psi,
//   <E_k b> = i k int int G phi_m . b - (i/k) int int div phi_m grad_x G . b,
//   <H_k b> = int int phi_m . (grad_x G x b).
// Non-touching triangle pairs: the 6-point rule in x, the source at the node;
// touching pairs: Sauter-Schwab points with the amplitude's quadratic
// interpolant through the source triangle's six nodes.

struct SdParams {
  double k0, k1, eta, cbi;   // cb = i k0 (1 - eps_r) = i cbi
  int field;                 // FOSB_FIELD_RADIAL or FOSB_FIELD_NORMAL
  double lag[6][6];          // ell_q(l1, l2) = sum_k mono_k(l1, l2) lag[k][q], mono = (1, l1, l2, l1^2, l1 l2, l2^2)
};

// Per triangle t: c_psi (re, im) and the M coefficients of its three local RWG functions.
__global__ void k_sd_tri_data(MeshDev md, const c128* __restrict__ u, int64_t ldu, int64_t dir, double k0,
                              double eps_r, double* __restrict__ td) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= md.nt) return;
  double dr = 0, di = 0;
  double* o = td + 8LL * t;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int e = md.tri_edge[a * md.nt + t];
    const c128 uj = u[(int64_t)e * ldu + dir], um = u[(int64_t)(md.ne + e) * ldu + dir];
    const double al = md.alpha[a * md.nt + t];
    dr += al * uj.re;
    di += al * uj.im;
    o[2 + 2 * a] = um.re;
    o[3 + 2 * a] = um.im;
  }
  // E_n = -(i/k0) div J;  c_psi = (1 - 1/eps_r) E_n
  const double f = (1.0 - 1.0 / eps_r) / k0;
  o[0] = f * di;
  o[1] = -f * dr;
}

__device__ __forceinline__ bool tri_touch(const MeshDev& md, int i, int j) {
  const int nt = md.nt;
  const int a0 = md.fv[i], a1 = md.fv[nt + i], a2 = md.fv[2 * nt + i];
  const int b0 = md.fv[j], b1 = md.fv[nt + j], b2 = md.fv[2 * nt + j];
  return a0 == b0 || a0 == b1 || a0 == b2 || a1 == b0 || a1 == b1 || a1 == b2 || a2 == b0 || a2 == b1 || a2 == b2;
}

// E_t(y) = n x sum_b uM_b (alpha_b / 2)(y - P_b) on triangle t, y and P relative to the same origin.
__device__ __forceinline__ void sd_et(const double* td, const double al[3], const double P[3][3], const double n[3],
                                      const double y[3], double er[3], double ei[3]) {
  double mr[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const double h = 0.5 * al[b];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = h * (y[c] - P[b][c]);
      mr[c] += td[2 + 2 * b] * v;
      mi[c] += td[3 + 2 * b] * v;
    }
  }
  cross3(n, mr, er);
  cross3(n, mi, ei);
}

// The four kernel sums of one point pair (x, y), weight folded into Gr/Gi:
// EA += h f.(d x n), HA += k^2 G f.n - alpha h d.n, EB += i k G f.E - (i/k) alpha h d.E,
// HB += h f.(d x E), with h = G (i k R - 1) / R^2, d = x - y.
struct SdAcc {
  double EAr = 0, EAi = 0, HAr = 0, HAi = 0, EBr = 0, EBi = 0, HBr = 0, HBi = 0;
};

__device__ __forceinline__ void sd_point(double k, const double f[3], double alpha, const double d[3], double r,
                                         double ir, double Gr, double Gi, const double n[3], const double er[3],
                                         const double ei[3], double s, SdAcc& A) {
  const double ir2 = ir * ir, kr = k * r;
  const double hr = (-Gr - Gi * kr) * ir2, hi = (Gr * kr - Gi) * ir2;
  double dn[3], dEr[3], dEi[3];
  cross3(d, n, dn);
  cross3(d, er, dEr);
  cross3(d, ei, dEi);
  const double fdn = f[0] * dn[0] + f[1] * dn[1] + f[2] * dn[2];
  const double fn = f[0] * n[0] + f[1] * n[1] + f[2] * n[2];
  const double ddn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
  const double fEr = f[0] * er[0] + f[1] * er[1] + f[2] * er[2], fEi = f[0] * ei[0] + f[1] * ei[1] + f[2] * ei[2];
  const double dEr_ = d[0] * er[0] + d[1] * er[1] + d[2] * er[2], dEi_ = d[0] * ei[0] + d[1] * ei[1] + d[2] * ei[2];
  const double fdEr = f[0] * dEr[0] + f[1] * dEr[1] + f[2] * dEr[2];
  const double fdEi = f[0] * dEi[0] + f[1] * dEi[1] + f[2] * dEi[2];
  A.EAr += s * hr * fdn;
  A.EAi += s * hi * fdn;
  A.HAr += s * (k * k * Gr * fn - alpha * hr * ddn);
  A.HAi += s * (k * k * Gi * fn - alpha * hi * ddn);
  // i k G (fEr + i fEi) = k (-Gi fEr - Gr fEi) + i k (Gr fEr - Gi fEi)
  // -(i/k) alpha h (dEr + i dEi) = (alpha/k) (hr dEi + hi dEr) + i (alpha/k) (hi dEi - hr dEr)
  A.EBr += s * (k * (-Gi * fEr - Gr * fEi) + alpha / k * (hr * dEi_ + hi * dEr_));
  A.EBi += s * (k * (Gr * fEr - Gi * fEi) + alpha / k * (hi * dEi_ - hr * dEr_));
  A.HBr += s * (hr * fdEr - hi * fdEi);
  A.HBi += s * (hr * fdEi + hi * fdEr);
}

// Combines the sums of one (row m, source node) into W[m][col], W[N+m][col]:
// WE = -eta cb EB - c_psi HA, WH = -cb HB + i k c_psi EA / eta, plus the identity parts.
__device__ __forceinline__ void sd_combine(const SdParams& sp, const SdAcc& A, double cpr, double cpi, double IEr,
                                           double IEi, double IHr, double IHi, double nu, double& WEr, double& WEi,
                                           double& WHr, double& WHi) {
  // cb X = i cbi (Xr + i Xi) = -cbi Xi + i cbi Xr
  const double cEBr = -sp.cbi * A.EBi, cEBi = sp.cbi * A.EBr;
  const double cHBr = -sp.cbi * A.HBi, cHBi = sp.cbi * A.HBr;
  const double pHAr = cpr * A.HAr - cpi * A.HAi, pHAi = cpr * A.HAi + cpi * A.HAr;
  const double pEAr = cpr * A.EAr - cpi * A.EAi, pEAi = cpr * A.EAi + cpi * A.EAr;
  // i k pEA / eta
  const double kEAr = -sp.k1 * pEAi / sp.eta, kEAi = sp.k1 * pEAr / sp.eta;
  WEr = nu * (-sp.eta * cEBr - pHAr + IEr);
  WEi = nu * (-sp.eta * cEBi - pHAi + IEi);
  WHr = nu * (-cHBr + kEAr + IHr);
  WHi = nu * (-cHBi + kEAi + IHi);
}

// One thread per (RWG row m, source node col = 6 j + q): the non-touching triangles of m
// with the 6-point rule, the identity parts; stores W[m][col] and W[N+m][col].
__global__ __launch_bounds__(256) void k_sd_regular(MeshDev md, Rule6 R, SdParams sp, const double* __restrict__ td,
                                                    int64_t col0, int64_t ncol, c128* __restrict__ W, int64_t ldw) {
  const int64_t lc = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y;
  if (lc >= ncol || m >= md.ne) return;
  const int64_t col = col0 + lc;
  const int j = (int)(col / 6), q = (int)(col % 6);
  const int nt = md.nt, ne = md.ne;
  double Pj[3][3], cj[3];
  load_tri(md, j, Pj, cj);
  const double nj[3] = {md.nrm[j], md.nrm[nt + j], md.nrm[2 * nt + j]};
  const double alj[3] = {md.alpha[j], md.alpha[nt + j], md.alpha[2 * nt + j]};
  double y[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) y[c] = R.l[q][0] * Pj[0][c] + R.l[q][1] * Pj[1][c] + R.l[q][2] * Pj[2][c];
  const double wq = R.w[q] * md.area[j];
  const double* tj = td + 8LL * j;
  double er[3], ei[3];
  sd_et(tj, alj, Pj, nj, y, er, ei);
  double nu = 1.0;
  if (sp.field == FOSB_FIELD_RADIAL) {
    const double iy = rsqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    nu = (y[0] * nj[0] + y[1] * nj[1] + y[2] * nj[2]) * iy;
  }
  SdAcc A;
  double IEr = 0, IEi = 0, IHr = 0, IHi = 0;
  for (int side = 0; side < 2; ++side) {
    const int i = md.edge_tri[side * ne + m];
    const int a = md.edge_loc[side * ne + m];
    double Pi[3][3], ci[3];
    load_tri(md, i, Pi, ci);
    const double ala = md.alpha[a * nt + i];
    if (i == j) {  // identity parts: -1/2 c_psi alpha_a w_q, 1/2 cb phi_a(y).(n x E_t) w_q
      double nE_r[3], nE_i[3];
      cross3(nj, er, nE_r);
      cross3(nj, ei, nE_i);
      double fr = 0, fi = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double fc = 0.5 * ala * (y[c] - Pi[a][c]);
        fr += fc * nE_r[c];
        fi += fc * nE_i[c];
      }
      IEr += -0.5 * tj[0] * ala * wq;
      IEi += -0.5 * tj[1] * ala * wq;
      // 1/2 i cbi (fr + i fi) wq
      IHr += -0.5 * sp.cbi * fi * wq;
      IHi += 0.5 * sp.cbi * fr * wq;
    }
    if (tri_touch(md, i, j)) continue;  // integrated by k_sd_singular
    for (int p = 0; p < 6; ++p) {
      double x[3], f[3], d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[c] = R.l[p][0] * Pi[0][c] + R.l[p][1] * Pi[1][c] + R.l[p][2] * Pi[2][c];
        f[c] = 0.5 * ala * (x[c] - Pi[a][c]);
        d[c] = x[c] - y[c];
      }
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double ir = rsqrt(r2);
      const double r = r2 * ir;
      double sn, cs;
      sincos_phase(sp.k1 * r, &sn, &cs);
      const double g = R.w[p] * md.area[i] * wq * kInv4Pi * ir;
      sd_point(sp.k1, f, ala, d, r, ir, cs * g, sn * g, nj, er, ei, 1.0, A);
    }
  }
  double WEr, WEi, WHr, WHi;
  sd_combine(sp, A, tj[0], tj[1], IEr, IEi, IHr, IHi, nu, WEr, WEi, WHr, WHi);
  W[(int64_t)m * ldw + lc] = c128{WEr, WEi};
  W[(int64_t)(ne + m) * ldw + lc] = c128{WHr, WHi};
}

// One wavefront per (RWG row m, source triangle j) with a triangle of m touching j:
// Sauter-Schwab points over the lanes, the amplitude's quadratic interpolant in j;
// adds to W[m][6 j + q] and W[N+m][6 j + q], q = 0..5.
__global__ __launch_bounds__(256) void k_sd_singular(MeshDev md, Rule6 R, SdParams sp, const double* __restrict__ td,
                                                     const int32_t* __restrict__ sm_m, const int32_t* __restrict__ sm_j,
                                                     const int32_t* __restrict__ sm_p, int e0, int nS, int64_t col0,
                                                     const int32_t* __restrict__ tp_kind,
                                                     const int32_t* __restrict__ tp_ord, const double* __restrict__ ss,
                                                     int off0, int off1, int off2, int cnt0, int cnt1, int cnt2,
                                                     c128* __restrict__ W, int64_t ldw) {
  const int e = e0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= e0 + nS) return;
  const int m = sm_m[e], j = sm_j[e];
  const int nt = md.nt, ne = md.ne;
  double Pj[3][3], cj[3];
  load_tri(md, j, Pj, cj);
  double Lj[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < 3; ++c) Lj[v][c] = Pj[v][c] - cj[c];
  const double nj[3] = {md.nrm[j], md.nrm[nt + j], md.nrm[2 * nt + j]};
  const double alj[3] = {md.alpha[j], md.alpha[nt + j], md.alpha[2 * nt + j]};
  const double* tj = td + 8LL * j;
  SdAcc A[6];
  for (int side = 0; side < 2; ++side) {
    const int p = sm_p[2 * e + side];
    if (p < 0) continue;
    const int i = md.edge_tri[side * ne + m];
    const int a = md.edge_loc[side * ne + m];
    const int kind = tp_kind[p];
    const int* ord = tp_ord + 6 * p;
    double Pi[3][3], ci[3], Li[3][3];
    load_tri(md, i, Pi, ci);
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) Li[v][c] = Pi[v][c] - ci[c];
    const double ala = md.alpha[a * nt + i];
    const double dc[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
    double S0[3], S1[3], S2[3], T0[3], T1[3], T2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S0[c] = Li[ord[0]][c]; S1[c] = Li[ord[1]][c] - Li[ord[0]][c]; S2[c] = Li[ord[2]][c] - Li[ord[1]][c];
      T0[c] = Lj[ord[3]][c]; T1[c] = Lj[ord[4]][c] - Lj[ord[3]][c]; T2[c] = Lj[ord[5]][c] - Lj[ord[4]][c];
    }
    const double jac = 4.0 * md.area[i] * md.area[j] * kInv4Pi;
    const int off = kind == 0 ? off0 : (kind == 1 ? off1 : off2);
    const int cnt = kind == 0 ? cnt0 : (kind == 1 ? cnt1 : cnt2);
    for (int mm = lane; mm < cnt; mm += 64) {
      const double* pt = ss + 5 * (int64_t)(off + mm);
      const double x1 = pt[0], x2 = pt[1], y1 = pt[2], y2 = pt[3], w = pt[4];
      double x[3], y[3], f[3], d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[c] = S0[c] + x1 * S1[c] + x2 * S2[c];
        y[c] = T0[c] + y1 * T1[c] + y2 * T2[c];
        f[c] = 0.5 * ala * (x[c] - Li[a][c]);
        d[c] = x[c] - y[c] + dc[c];
      }
      // barycentric coordinates of y in j's own vertex order
      double lam[3];
      lam[ord[3]] = 1.0 - y1;
      lam[ord[4]] = y1 - y2;
      lam[ord[5]] = y2;
      const double l1 = lam[1], l2 = lam[2];
      const double mono[6] = {1.0, l1, l2, l1 * l1, l1 * l2, l2 * l2};
      double er[3], ei[3];
      sd_et(tj, alj, Lj, nj, y, er, ei);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double ir = rsqrt(r2);
      const double r = r2 * ir;
      double sn, cs;
      sincos(sp.k1 * r, &sn, &cs);
      const double g = w * jac * ir;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        double ell = 0;
#pragma unroll
        for (int kk = 0; kk < 6; ++kk) ell += mono[kk] * sp.lag[kk][q];
        sd_point(sp.k1, f, ala, d, r, ir, cs * g, sn * g, nj, er, ei, ell, A[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    A[q].EAr = wave_sum(A[q].EAr);
    A[q].EAi = wave_sum(A[q].EAi);
    A[q].HAr = wave_sum(A[q].HAr);
    A[q].HAi = wave_sum(A[q].HAi);
    A[q].EBr = wave_sum(A[q].EBr);
    A[q].EBi = wave_sum(A[q].EBi);
    A[q].HBr = wave_sum(A[q].HBr);
    A[q].HBi = wave_sum(A[q].HBi);
  }
  if (lane < 6) {
    const int q = lane;
    SdAcc Aq;
#pragma unroll
    for (int qq = 0; qq < 6; ++qq)
      if (qq == q) Aq = A[qq];
    double nu = 1.0;
    if (sp.field == FOSB_FIELD_RADIAL) {  // (y_q / |y_q|) . n at node q of j
      double y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c] = R.l[q][0] * Pj[0][c] + R.l[q][1] * Pj[1][c] + R.l[q][2] * Pj[2][c];
      nu = (y[0] * nj[0] + y[1] * nj[1] + y[2] * nj[2]) * rsqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    }
    const int64_t col = 6LL * j + q - col0;
    double WEr, WEi, WHr, WHi;
    sd_combine(sp, Aq, tj[0], tj[1], 0.0, 0.0, 0.0, 0.0, nu, WEr, WEi, WHr, WHi);
    c128* w0 = W + (int64_t)m * ldw + col;
    c128* w1 = W + (int64_t)(ne + m) * ldw + col;
    const c128 o0 = *w0, o1 = *w1;
    *w0 = c128{o0.re + WEr, o0.im + WEi};
    *w1 = c128{o1.re + WHr, o1.im + WHi};
  }
}

// Inverse of the 6 x 6 matrix of the monomials (1, l1, l2, l1^2, l1 l2, l2^2) at
// the 6-point nodes (Gauss-Jordan with partial pivoting): the coefficients of
// the quadratic Lagrange basis through the nodes.
static void lagrange6(double out[6][6]) {
  double bary[6][3], w[6];
  rule6(bary, w);
  double A[6][12];
  for (int r = 0; r < 6; ++r) {
    const double l1 = bary[r][1], l2 = bary[r][2];
    const double mono[6] = {1.0, l1, l2, l1 * l1, l1 * l2, l2 * l2};
    for (int c = 0; c < 6; ++c) {
      A[r][c] = mono[c];
      A[r][6 + c] = r == c ? 1.0 : 0.0;
    }
  }
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int k = 0; k < 12; ++k) std::swap(A[c][k], A[piv][k]);
    const double d = A[c][c];
    for (int k = 0; k < 12; ++k) A[c][k] /= d;
    for (int r = 0; r < 6; ++r)
      if (r != c) {
        const double f = A[r][c];
        for (int k = 0; k < 12; ++k) A[r][k] -= f * A[c][k];
      }
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) out[r][c] = A[r][6 + c];
}

void sd_plan(Context& ctx, const Mesh& m, double k0, double eps_r, const c128* u, int64_t ldu, int64_t dir,
             SdPlan& P) {
  hipStream_t s = ctx.stream;
  const MeshHost& h = m.h;
  const int nt = (int)h.nt, ne = (int)h.ne;
  P.td.alloc((size_t)8 * nt * sizeof(double));
  hipLaunchKernelGGL(k_sd_tri_data, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, m.dev(), u, ldu, dir, k0,
                     eps_r, P.td.as<double>());
  FOSB_LAUNCH_CHECK();
  // (row m, source triangle j) with a triangle of m touching j, sorted by j, and the
  // touching-pair index of each side (-1: that side does not touch j)
  std::vector<std::vector<std::pair<int, int>>> by_i(nt);
  for (size_t p = 0; p < h.tp_i.size(); ++p) by_i[h.tp_i[p]].push_back({h.tp_j[p], (int)p});
  std::vector<std::vector<std::array<int32_t, 3>>> by_j(nt);   // j -> (m, p+, p-)
  for (int e = 0; e < ne; ++e) {
    const int ip = h.edge_tri[2 * e], im = h.edge_tri[2 * e + 1];
    std::map<int, std::pair<int, int>> js;
    for (auto& jp : by_i[ip]) js[jp.first].first = jp.second + 1;
    for (auto& jp : by_i[im]) js[jp.first].second = jp.second + 1;
    for (auto& kv : js) by_j[kv.first].push_back({e, kv.second.first - 1, kv.second.second - 1});
  }
  std::vector<int32_t> sm_m, sm_j, sm_p;
  P.jbeg.assign(nt + 1, 0);
  for (int j = 0; j < nt; ++j) {
    P.jbeg[j] = (int64_t)sm_m.size();
    for (auto& r : by_j[j]) {
      sm_m.push_back(r[0]);
      sm_j.push_back(j);
      sm_p.push_back(r[1]);
      sm_p.push_back(r[2]);
    }
  }
  P.jbeg[nt] = (int64_t)sm_m.size();
  upload(P.dm, sm_m, s);
  upload(P.dj, sm_j, s);
  upload(P.dp, sm_p, s);
  FOSB_HIP(hipStreamSynchronize(s));
}

void sd_band(Context& ctx, const Mesh& m, const SdPlan& P, double k0, double eps_r, int field, int n_gauss, int j0,
             int j1, c128* W, int64_t ldw) {
  hipStream_t s = ctx.stream;
  const int ne = (int)m.h.ne;
  if (j1 <= j0) return;
  ensure_ss_table(ctx, n_gauss);
  Rule6 R;
  rule6(R.l, R.w);
  SdParams sp;
  sp.k0 = k0;
  sp.k1 = k0 * std::sqrt(eps_r);
  sp.eta = 1.0 / std::sqrt(eps_r);
  sp.cbi = k0 * (1.0 - eps_r);
  sp.field = field;
  lagrange6(sp.lag);
  const int64_t col0 = 6LL * j0, ncol = 6LL * (j1 - j0);
  dim3 g1((unsigned)((ncol + 255) / 256), (unsigned)ne);
  hipLaunchKernelGGL(k_sd_regular, g1, dim3(256), 0, s, m.dev(), R, sp, P.td.as<double>(), col0, ncol, W, ldw);
  FOSB_LAUNCH_CHECK();
  const int e0 = (int)P.jbeg[j0], nS = (int)(P.jbeg[j1] - P.jbeg[j0]);
  if (nS > 0) {
    hipLaunchKernelGGL(k_sd_singular, dim3((unsigned)((nS + 3) / 4)), dim3(256), 0, s, m.dev(), R, sp,
                       P.td.as<double>(), P.dm.as<int32_t>(), P.dj.as<int32_t>(), P.dp.as<int32_t>(), e0, nS, col0,
                       m.tp_kind.as<int32_t>(), m.tp_ord.as<int32_t>(), ctx.ss[n_gauss].as<double>(),
                       ctx.ss_off[n_gauss][0], ctx.ss_off[n_gauss][1], ctx.ss_off[n_gauss][2], ctx.ss_cnt[n_gauss][0],
                       ctx.ss_cnt[n_gauss][1], ctx.ss_cnt[n_gauss][2], W, ldw);
    FOSB_LAUNCH_CHECK();
  }
}

void sd_weights(Context& ctx, const Mesh& m, double k0, double eps_r, int field, const c128* u, int64_t ldu,
                int64_t dir, int n_gauss, c128* W, int64_t ldw) {
  SdPlan P;
  sd_plan(ctx, m, k0, eps_r, u, ldu, dir, P);
  sd_band(ctx, m, P, k0, eps_r, field, n_gauss, 0, (int)m.h.nt, W, ldw);
  FOSB_HIP(hipStreamSynchronize(ctx.stream));
}

void efie_residual(Context& ctx, const Mesh& m, double k, int n_gauss, const c128* X, int64_t ldx, int64_t nrhs,
                   c128* R, int64_t ldr) {
  if (nrhs <= 0) return;
  const int ne = (int)m.h.ne, nt = (int)m.h.nt;
  const MeshDev md = m.dev();
  // R -= sum over bands (rows of Z on the band's local columns) x (X at the band's local columns)
  const int64_t budget = (int64_t)4096 << 20;
  int jc = (int)std::max<int64_t>(1, std::min<int64_t>(nt, budget / (9LL * nt * (int64_t)sizeof(c128))));
  if (jc < nt) jc = std::max(64, jc / 64 * 64);
  jc = std::min(jc, nt);
  DevBuf zr((size_t)ne * 3 * jc * sizeof(c128)), xt((size_t)3 * jc * nrhs * sizeof(c128));
  assemble_bands(ctx, m, k, n_gauss, budget,
                 [&](hipStream_t, int j0, int j1, const c128* Zc, int64_t ldc, const int32_t*, int) {
                   const int w = j1 - j0, ncol = 3 * w;
                   dim3 g1((ncol + 63) / 64, (ne + 3) / 4);
                   hipLaunchKernelGGL(k_band_rows, g1, dim3(256), 0, ctx.stream, ne, md.edge_tri, md.edge_loc,
                                      ncol, Zc, ldc, zr.as<c128>());
                   FOSB_LAUNCH_CHECK();
                   dim3 g2((unsigned)((nrhs + 255) / 256), (unsigned)ncol);
                   hipLaunchKernelGGL(k_band_gather_x, g2, dim3(256), 0, ctx.stream, nt, md.tri_edge, j0, w, X, ldx,
                                      nrhs, xt.as<c128>());
                   FOSB_LAUNCH_CHECK();
                   gemm<double>(ctx, ne, nrhs, ncol, -1.0, zr.as<c128>(), ncol, xt.as<c128>(), nrhs, 1.0, R, ldr);
                 });
}

}  // namespace fosb
