// Host-side mesh processing: validation, RWG tables, touching-pair lists and
// the quadrature tables that the kernels read.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "common.h"

namespace fosb {

static inline uint64_t edge_key(int32_t a, int32_t b) {
  uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
  return ((uint64_t)lo << 32) | hi;
}

void mesh_build_host(const double* V, int64_t nv, const int32_t* F, int64_t nt, MeshHost& m) {
  if (!V || !F) fail(FOSB_E_INVALID, "mesh: null vertex or triangle array");
  if (nv < 4 || nt < 4) fail(FOSB_E_INVALID, "mesh: need at least 4 vertices and 4 triangles");
  if (nt > (int64_t)1 << 27) fail(FOSB_E_INVALID, "mesh: too many triangles (%lld)", (long long)nt);
  m.nv = nv;
  m.nt = nt;
  m.V.assign(V, V + 3 * nv);
  m.F.assign(F, F + 3 * nt);
  double scale = 0.0;
  for (int64_t i = 0; i < 3 * nv; ++i) {
    if (!std::isfinite(V[i])) fail(FOSB_E_INVALID, "mesh: non-finite vertex coordinate at %lld", (long long)i);
    scale = std::max(scale, std::fabs(V[i]));
  }
  m.area.resize(nt);
  m.normal.resize(3 * nt);
  double vol6 = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    int32_t a = F[3 * t], b = F[3 * t + 1], c = F[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
      fail(FOSB_E_INVALID, "mesh: triangle %lld has a vertex index out of range", (long long)t);
    if (a == b || b == c || a == c) fail(FOSB_E_INVALID, "mesh: triangle %lld repeats a vertex", (long long)t);
    const double* p0 = V + 3 * a;
    const double* p1 = V + 3 * b;
    const double* p2 = V + 3 * c;
    double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(len > 1e-14 * scale * scale)) fail(FOSB_E_INVALID, "mesh: degenerate triangle %lld", (long long)t);
    m.area[t] = 0.5 * len;
    for (int k = 0; k < 3; ++k) m.normal[3 * t + k] = cr[k] / len;
    // p0 . (p1 x p2)
    vol6 += p0[0] * (p1[1] * p2[2] - p1[2] * p2[1]) + p0[1] * (p1[2] * p2[0] - p1[0] * p2[2]) +
            p0[2] * (p1[0] * p2[1] - p1[1] * p2[0]);
  }
  // edges in first-visit order
  std::unordered_map<uint64_t, int32_t> id;
  id.reserve((size_t)(2 * nt));
  m.tri_edge.assign(3 * nt, -1);
  m.tri_sign.assign(3 * nt, 0.0);
  m.edge_tri.clear();
  m.edge_loc.clear();
  std::vector<int32_t> first_from;  // directed start vertex of the first visit
  for (int64_t t = 0; t < nt; ++t) {
    for (int a = 0; a < 3; ++a) {
      int32_t u = F[3 * t + (a + 1) % 3], v = F[3 * t + (a + 2) % 3];
      uint64_t key = edge_key(u, v);
      auto it = id.find(key);
      if (it == id.end()) {
        int32_t e = (int32_t)(m.edge_tri.size() / 2);
        id.emplace(key, e);
        m.edge_tri.push_back((int32_t)t);
        m.edge_tri.push_back(-1);
        m.edge_loc.push_back(a);
        m.edge_loc.push_back(-1);
        first_from.push_back(u);
        m.tri_edge[3 * t + a] = e;
        m.tri_sign[3 * t + a] = 1.0;
      } else {
        int32_t e = it->second;
        if (m.edge_tri[2 * e + 1] != -1)
          fail(FOSB_E_INVALID, "mesh: non-manifold edge (%d,%d) shared by more than two triangles", u, v);
        if (first_from[e] != v)
          fail(FOSB_E_INVALID, "mesh: inconsistent orientation across edge (%d,%d)", u, v);
        m.edge_tri[2 * e + 1] = (int32_t)t;
        m.edge_loc[2 * e + 1] = a;
        m.tri_edge[3 * t + a] = e;
        m.tri_sign[3 * t + a] = -1.0;
      }
    }
  }
  m.ne = (int64_t)(m.edge_tri.size() / 2);
  for (int64_t e = 0; e < m.ne; ++e)
    if (m.edge_tri[2 * e + 1] < 0) fail(FOSB_E_INVALID, "mesh: open surface (edge %lld has one triangle)", (long long)e);
  if (!(vol6 > 0.0)) fail(FOSB_E_INVALID, "mesh: triangles are oriented inward (enclosed volume <= 0)");
  m.edge_len.resize(m.ne);
  for (int64_t e = 0; e < m.ne; ++e) {
    int32_t t = m.edge_tri[2 * e], a = m.edge_loc[2 * e];
    int32_t u = F[3 * t + (a + 1) % 3], v = F[3 * t + (a + 2) % 3];
    double d0 = V[3 * u] - V[3 * v], d1 = V[3 * u + 1] - V[3 * v + 1], d2 = V[3 * u + 2] - V[3 * v + 2];
    m.edge_len[e] = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  }
}

// Ordered pairs of triangles sharing at least one vertex, with the local vertex
// order used by the Sauter-Schwab parameterisation: shared vertices first (in
// triangle i's cyclic order from its vertex 0), then the remaining vertices of
// each triangle in their own cyclic order.
void mesh_touching_pairs(MeshHost& m) {
  std::vector<std::vector<int32_t>> v2t((size_t)m.nv);
  for (int64_t t = 0; t < m.nt; ++t)
    for (int a = 0; a < 3; ++a) v2t[(size_t)m.F[3 * t + a]].push_back((int32_t)t);
  struct P { int32_t i, j, kind, ord[6]; };
  std::vector<P> pairs;
  pairs.reserve((size_t)m.nt * 14);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < m.nt; ++i) {
    nb.clear();
    for (int a = 0; a < 3; ++a)
      for (int32_t t : v2t[(size_t)m.F[3 * i + a]]) nb.push_back(t);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    const int32_t* fi = &m.F[3 * i];
    for (int32_t j : nb) {
      const int32_t* fj = &m.F[3 * (size_t)j];
      int shared_i[3], ns = 0;   // local slots in i of shared vertices (i's order)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          if (fi[a] == fj[b]) shared_i[ns++] = a;
      P p{};
      p.i = (int32_t)i;
      p.j = j;
      auto slot_in_j = [&](int32_t v) { for (int b = 0; b < 3; ++b) if (fj[b] == v) return b; return -1; };
      if (ns == 3) {
        p.kind = 0;
        for (int a = 0; a < 3; ++a) { p.ord[a] = a; p.ord[3 + a] = slot_in_j(fi[a]); }
      } else if (ns == 2) {
        p.kind = 1;
        int oi = 3 - shared_i[0] - shared_i[1];
        int sj0 = slot_in_j(fi[shared_i[0]]), sj1 = slot_in_j(fi[shared_i[1]]);
        p.ord[0] = shared_i[0]; p.ord[1] = shared_i[1]; p.ord[2] = oi;
        p.ord[3] = sj0; p.ord[4] = sj1; p.ord[5] = 3 - sj0 - sj1;
      } else if (ns == 1) {
        p.kind = 2;
        int a0 = shared_i[0];
        int b0 = slot_in_j(fi[a0]);
        p.ord[0] = a0; p.ord[1] = (a0 + 1) % 3; p.ord[2] = (a0 + 2) % 3;
        p.ord[3] = b0; p.ord[4] = (b0 + 1) % 3; p.ord[5] = (b0 + 2) % 3;
      } else {
        continue;
      }
      pairs.push_back(p);
    }
  }
  std::sort(pairs.begin(), pairs.end(), [](const P& a, const P& b) { return a.j != b.j ? a.j < b.j : a.i < b.i; });
  size_t np = pairs.size();
  m.tp_i.resize(np); m.tp_j.resize(np); m.tp_kind.resize(np); m.tp_ord.resize(6 * np);
  for (size_t q = 0; q < np; ++q) {
    m.tp_i[q] = pairs[q].i; m.tp_j[q] = pairs[q].j; m.tp_kind[q] = pairs[q].kind;
    for (int r = 0; r < 6; ++r) m.tp_ord[6 * q + r] = pairs[q].ord[r];
  }
}

void mesh_upload(Mesh& mesh) {
  const MeshHost& m = mesh.h;
  hipStream_t s = mesh.ctx->stream;
  int64_t nt = m.nt, ne = m.ne;
  std::vector<double> vtx(9 * nt), nrm(3 * nt), alpha(3 * nt);
  std::vector<int32_t> fv(3 * nt), te(3 * nt), et(2 * ne), el(2 * ne);
  for (int64_t t = 0; t < nt; ++t) {
    for (int v = 0; v < 3; ++v) {
      int32_t id = m.F[3 * t + v];
      fv[v * nt + t] = id;
      for (int c = 0; c < 3; ++c) vtx[(v * 3 + c) * nt + t] = m.V[3 * id + c];
    }
    for (int c = 0; c < 3; ++c) nrm[c * nt + t] = m.normal[3 * t + c];
    for (int a = 0; a < 3; ++a) {
      int32_t e = m.tri_edge[3 * t + a];
      te[a * nt + t] = e;
      alpha[a * nt + t] = m.tri_sign[3 * t + a] * m.edge_len[e] / m.area[t];
    }
  }
  for (int64_t e = 0; e < ne; ++e) {
    et[e] = m.edge_tri[2 * e]; et[ne + e] = m.edge_tri[2 * e + 1];
    el[e] = m.edge_loc[2 * e]; el[ne + e] = m.edge_loc[2 * e + 1];
  }
  upload(mesh.vtx, vtx, s);
  upload(mesh.area, m.area, s);
  upload(mesh.nrm, nrm, s);
  upload(mesh.alpha, alpha, s);
  upload(mesh.fv, fv, s);
  upload(mesh.tri_edge, te, s);
  upload(mesh.edge_tri, et, s);
  upload(mesh.edge_loc, el, s);
  upload(mesh.tp_i, m.tp_i, s);
  upload(mesh.tp_j, m.tp_j, s);
  upload(mesh.tp_kind, m.tp_kind, s);
  upload(mesh.tp_ord, m.tp_ord, s);
  FOSB_HIP(hipStreamSynchronize(s));   // host vectors above are temporaries
}

// ------------------------------------------------------------------ quadrature tables
// Symmetric 6-point degree-4 triangle rule: orbits (1-2b, b, b) with
// b = (8 - sqrt10 +- sqrt(38 - 44 sqrt(2/5)))/18, weights (620 +- sqrt(213125 - 53320 sqrt10))/3720.
void rule6(double bary[6][3], double w[6]) {
  const double r10 = std::sqrt(10.0);
  const double root = std::sqrt(38.0 - 44.0 * std::sqrt(0.4));
  const double b[2] = {(8.0 - r10 + root) / 18.0, (8.0 - r10 - root) / 18.0};
  const double wr = std::sqrt(213125.0 - 53320.0 * r10);
  const double ww[2] = {(620.0 + wr) / 3720.0, (620.0 - wr) / 3720.0};
  int q = 0;
  for (int o = 0; o < 2; ++o) {
    double a = 1.0 - 2.0 * b[o];
    double orbit[3][3] = {{a, b[o], b[o]}, {b[o], a, b[o]}, {b[o], b[o], a}};
    for (int r = 0; r < 3; ++r, ++q) {
      for (int c = 0; c < 3; ++c) bary[q][c] = orbit[r][c];
      w[q] = ww[o];
    }
  }
}

// Gauss-Legendre nodes on [0,1] by Newton iteration on P_n from Chebyshev guesses.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // = (2/((1-z^2) P'^2)) / 2
  }
}

// Sauter-Schwab regularising transforms of [0,1]^4 (Sauter & Schwab, Boundary
// Element Methods, sec. 5.2) for the reference triangle {0 <= x2 <= x1 <= 1};
// kind 0: identical panels (6 regions), 1: common edge P0-P1 (5 regions),
// 2: common vertex P0 (2 regions).
void sauter_schwab_points(int kind, int n, std::vector<double>& pts) {
  std::vector<double> g, gw;
  gauss_legendre01(n, g, gw);
  pts.clear();
  auto push = [&](double x1, double x2, double y1, double y2, double w) {
    pts.push_back(x1); pts.push_back(x2); pts.push_back(y1); pts.push_back(y2); pts.push_back(w);
  };
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c)
        for (int d = 0; d < n; ++d) {
          const double xi = g[a], e1 = g[b], e2 = g[c], e3 = g[d];
          const double wc = gw[a] * gw[b] * gw[c] * gw[d];
          if (kind == 0) {
            const double j = wc * xi * xi * xi * e1 * e1 * e2;
            push(xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1), j);
            push(xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2), j);
            push(xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2), j);
            push(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3), j);
            push(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2), j);
            push(xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), j);
          } else if (kind == 1) {
            const double j1 = wc * xi * xi * xi * e1 * e1;
            const double j2 = j1 * e2;
            push(xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2), j1);
            push(xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), j2);
            push(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3, j2);
            push(xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1, j2);
            push(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2, j2);
          } else {
            const double j = wc * xi * xi * xi * e2;
            push(xi, xi * e1, xi * e2, xi * e2 * e3, j);
            push(xi * e2, xi * e2 * e3, xi, xi * e1, j);
          }
        }
}

}  // namespace fosb
