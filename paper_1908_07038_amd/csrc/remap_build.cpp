// Host set-up of grid-to-grid remapping (Section 4.3, Figures 4-6): the
// points of a target grid, the source triangle each one lies in, and the
// weights of linear interpolation over that triangle in 3-D on the sphere.
//
// Target grids: "F<M>" is the regular Gaussian grid (2M rows at the roots of
// P_2M, 4M points per row at longitude 2 pi j / 4M); "O<M>" is the
// octahedral grid of the source meshes.  Points are numbered row by row from
// north to south, west to east.
//
// Element and weights: a source triangle (a, b, c) (outward counter-
// clockwise, unit vectors) is the flat triangle through its nodes.  The ray
// from the centre through the target point p meets it when the triple
// products D_a = det(p, b, c), D_b = det(a, p, c), D_c = det(a, b, p) are all
// >= 0 with sum D > 0; the weights are (D_a, D_b, D_c) / D, the barycentric
// coordinates of the point where the ray crosses the triangle's plane.
//
// Location: a target point between source rows k and k+1 (by colatitude)
// lies in band k, or -- since the great circles through consecutive nodes
// of a row bow poleward of the row -- in band k - 1 or k + 1, or in a polar
// cap.  Each band's triangles are kept sorted by the longitude of their
// centroid; a point tests the triangles of those bands whose centroids are
// nearest its longitude (and all triangles of a polar cap).  A triangle
// contains the point when D > 0 and its smallest triple product is >= -1e-14
// (rounding of products of unit vectors; a bound on the normalised weights
// would have to grow as 1/h^2).  Among the containing triangles the one whose
// smallest weight is largest wins, the lowest triangle index on ties.  A
// point no candidate contains is searched over all triangles (counted in
// RemapHost::fallback).
#include <algorithm>
#include <array>
#include <cctype>
#include <cmath>
#include <cstdint>
#include <limits>
#include <stdexcept>
#include <string>
#include <vector>

#include "mesh.hpp"

namespace atlasnabla {

namespace {

using V3 = std::array<double, 3>;

inline V3 at(const std::vector<double>& xyz, int64_t i) { return {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]}; }
inline double det3(const V3& a, const V3& b, const V3& c) {
  // a . (b x c)
  return a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
}

constexpr double kDetTol = 1e-14;
constexpr int kWindow = 6;   // candidates on each side of the nearest centroid

struct Hit {
  double score = -std::numeric_limits<double>::infinity();
  int64_t tri = -1;
};

// Score of triangle t for point p: its smallest weight if it contains p,
// else -inf.
inline double score_of(const HostMesh& m, int64_t t, const V3& p) {
  const V3 a = at(m.xyz, m.tris[3 * t]), b = at(m.xyz, m.tris[3 * t + 1]), c = at(m.xyz, m.tris[3 * t + 2]);
  const double da = det3(p, b, c), db = det3(a, p, c), dc = det3(a, b, p);
  const double d = da + db + dc;
  const double lo = std::min(da, std::min(db, dc));
  if (!(d > 0.0) || !(lo >= -kDetTol)) return -std::numeric_limits<double>::infinity();
  return lo / d;
}

inline void consider(const HostMesh& m, int64_t t, const V3& p, Hit& h) {
  const double s = score_of(m, t, p);
  if (s > h.score || (s == h.score && t < h.tri)) {
    h.score = s;
    h.tri = t;
  }
}

}  // namespace

int parse_target_name(const std::string& name, char* kind) {
  size_t b = 0, e = name.size();
  while (b < e && std::isspace((unsigned char)name[b])) ++b;
  while (e > b && std::isspace((unsigned char)name[e - 1])) --e;
  if (e - b < 2) return -1;
  const char k = (char)std::toupper((unsigned char)name[b]);
  if (k != 'F' && k != 'O') return -1;
  long n = 0;
  for (size_t i = b + 1; i < e; ++i) {
    if (name[i] < '0' || name[i] > '9') return -1;
    n = n * 10 + (name[i] - '0');
    if (n > 100000) return -1;
  }
  if (n < 1) return -1;
  if (kind) *kind = k;
  return (int)n;
}

void build_remap(const HostMesh& m, const std::string& target, RemapHost& out) {
  char kind = 0;
  const int M = parse_target_name(target, &kind);
  if (M < 1) throw std::runtime_error("not a target grid name: '" + target + "'");
  out = RemapHost();
  out.target = std::string(1, kind) + std::to_string(M);

  // ---- target points ---------------------------------------------------------
  const int nrows = 2 * M;
  std::vector<double> th;
  gaussian_colatitudes(nrows, th);
  std::vector<int64_t> rsize(nrows);
  for (int k = 0; k < nrows; ++k) rsize[k] = kind == 'F' ? 4LL * M : 4LL * std::min(k + 1, nrows - k) + 16;
  int64_t P = 0;
  for (int k = 0; k < nrows; ++k) P += rsize[k];
  if (P > (int64_t)INT32_MAX) throw std::length_error("target grid too large");
  out.P = P;
  out.xyz.resize(3 * P);
  {
    int64_t g = 0;
    for (int k = 0; k < nrows; ++k) {
      const double sl = std::cos(th[k]), cl = std::sin(th[k]);
      for (int64_t j = 0; j < rsize[k]; ++j, ++g) {
        const double lon = (2.0 * M_PI * (double)j) / (double)rsize[k];
        out.xyz[3 * g] = cl * std::cos(lon);
        out.xyz[3 * g + 1] = cl * std::sin(lon);
        out.xyz[3 * g + 2] = sl;
      }
    }
  }

  // ---- triangles by band, sorted by centroid longitude ----------------------------
  const int n = m.nrows;
  // band b in 0..n-2 between rows b and b+1; index n-1: north cap, n: south cap
  std::vector<std::vector<std::pair<double, int64_t>>> band(n + 1);
  for (int64_t t = 0; t < m.T; ++t) {
    const int32_t* v = &m.tris[3 * t];
    const int r0 = m.node_row[v[0]], r1 = m.node_row[v[1]], r2 = m.node_row[v[2]];
    const int lo = std::min(r0, std::min(r1, r2)), hi = std::max(r0, std::max(r1, r2));
    int id;
    if (lo == hi) id = lo == 0 ? n - 1 : n;
    else id = lo;
    const double cx = m.xyz[3 * v[0]] + m.xyz[3 * v[1]] + m.xyz[3 * v[2]];
    const double cy = m.xyz[3 * v[0] + 1] + m.xyz[3 * v[1] + 1] + m.xyz[3 * v[2] + 1];
    double lam = std::atan2(cy, cx);
    if (lam < 0) lam += 2.0 * M_PI;
    band[id].push_back({lam, t});
  }
  for (auto& b : band) std::sort(b.begin(), b.end());

  auto search_band = [&](int id, double lam, const V3& p, Hit& h) {
    const auto& b = band[id];
    const int64_t nb = (int64_t)b.size();
    if (nb == 0) return;
    if (id >= n - 1 || nb <= 2 * kWindow + 1) {   // polar cap or a short band: every triangle
      for (const auto& e : b) consider(m, e.second, p, h);
      return;
    }
    const int64_t i0 = std::lower_bound(b.begin(), b.end(), std::make_pair(lam, (int64_t)-1)) - b.begin();
    for (int64_t d = -kWindow; d <= kWindow; ++d) consider(m, b[((i0 + d) % nb + nb) % nb].second, p, h);
  };

  out.nodes.assign(4 * P, 0);
  out.w.assign(4 * P, 0.0);
  for (int64_t g = 0; g < P; ++g) {
    const V3 p = at(out.xyz, g);
    double lam = std::atan2(p[1], p[0]);
    if (lam < 0) lam += 2.0 * M_PI;
    const double t = std::acos(std::max(-1.0, std::min(1.0, p[2])));
    // source row k with colat[k] <= t < colat[k+1] (k = -1 north of row 0)
    const int k = (int)(std::upper_bound(m.colat.begin(), m.colat.end(), t) - m.colat.begin()) - 1;
    Hit h;
    for (int b = k - 1; b <= k + 1; ++b)
      if (b >= 0 && b <= n - 2) search_band(b, lam, p, h);
    if (k <= 1) search_band(n - 1, lam, p, h);
    if (k >= n - 2) search_band(n, lam, p, h);
    if (h.tri < 0 || !std::isfinite(h.score)) {
      ++out.fallback;
      for (int64_t tt = 0; tt < m.T; ++tt) consider(m, tt, p, h);
      if (h.tri < 0 || !std::isfinite(h.score)) throw std::runtime_error("a target point lies in no source triangle");
    }
    const int32_t* v = &m.tris[3 * h.tri];
    const V3 a = at(m.xyz, v[0]), b = at(m.xyz, v[1]), c = at(m.xyz, v[2]);
    const double da = det3(p, b, c), db = det3(a, p, c), dc = det3(a, b, p);
    const double d = da + db + dc;
    for (int s = 0; s < 3; ++s) out.nodes[4 * g + s] = v[s];
    out.w[4 * g] = da / d;
    out.w[4 * g + 1] = db / d;
    out.w[4 * g + 2] = dc / d;
  }
  // transpose by source node (counting sort; targets stay ascending)
  out.adj_off.assign(m.V + 1, 0);
  for (int64_t g = 0; g < P; ++g)
    for (int s = 0; s < 3; ++s) ++out.adj_off[out.nodes[4 * g + s] + 1];
  for (int64_t i = 0; i < m.V; ++i) out.adj_off[i + 1] += out.adj_off[i];
  out.adj_t.resize(3 * P);
  out.adj_w.resize(3 * P);
  std::vector<int64_t> fill(out.adj_off.begin(), out.adj_off.end() - 1);
  for (int64_t g = 0; g < P; ++g)
    for (int s = 0; s < 3; ++s) {
      const int64_t e = fill[out.nodes[4 * g + s]]++;
      out.adj_t[e] = (int32_t)g;
      out.adj_w[e] = out.w[4 * g + s];
    }
}

}  // namespace atlasnabla