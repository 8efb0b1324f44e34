// Host FP64 construction of the O-grid, its triangulation, the median dual
// and the per-node operator tables.
//
// Definitions (the report names "O32"-type grids and meshes, Sections 2.3 and
// 4.3, and defers their construction to other documents):
//  * Row k of O<N> (2N rows, north to south) lies at the k-th Gaussian
//    colatitude t_k, a root of P_2N(cos t), found by Newton iteration in t;
//    it holds n_k = 4*min(k+1, 2N-k)+16 points at longitudes 2*pi*j/n_k.
//    sin(lat) = cos(t_k) and cos(lat) = sin(t_k) come from t_k directly.
//  * Bands between rows k and k+1 are zipped from the zero meridian east,
//    advancing the row whose next point comes first in longitude (exact
//    integer comparison (p+1)*n_b vs (q+1)*n_a; ties: the row with fewer
//    points, or the northern row if counts are equal).
//  * Each 20-point polar row is closed by a ladder of 18 triangles; its 17
//    chords are the pole edges.
//  * Median dual on the sphere: edge midpoints m_e and triangle centres c_T
//    are the normalised vertex sums; the dual face of an edge is the geodesic
//    path c_T1 -> m_e -> c_T2; S_e is its integrated conormal (pointing from
//    the edge's first node to its second); V_i is the spherical area of the
//    median cell.
//
// Evaluation order of positions (vertex sums, norms, divisions) is fixed and
// no fused multiply-add contraction is allowed in this file: dual normals are
// differences of nearby points, so an ulp of position error would become a
// relative error of order eps/h in S_e.
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cctype>
#include <cmath>
#include <cstring>
#include <stdexcept>

namespace atlasnabla {

namespace {

using V3 = std::array<double, 3>;

inline V3 load3(const std::vector<double>& a, int64_t i) {
  return {a[3 * i], a[3 * i + 1], a[3 * i + 2]};
}
inline V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
inline V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double dot(const V3& a, const V3& b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
inline V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline V3 normalized(const V3& s) {
  const double n = std::sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
  return {s[0] / n, s[1] / n, s[2] / n};
}

// Spherical triangle area on the unit sphere (Van Oosterom & Strackee 1983):
// tan(Omega/2) = |a.(b x c)| / (1 + a.b + b.c + c.a), with the triple
// product taken on differences to keep small triangles accurate.
inline double tri_solid_angle(const V3& a, const V3& b, const V3& c) {
  const double num = std::fabs(dot(a, cross(sub(b, a), sub(c, a))));
  const double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
  return 2.0 * std::atan2(num, den);
}

}  // namespace

// Roots of P_n(cos t), ascending in t.
void gaussian_colatitudes(int n, std::vector<double>& out) {
  const int half = n / 2;
  out.assign(n, 0.0);
  for (int k = 0; k < half; ++k) {
    double th = (M_PI * ((double)k + 0.75)) / ((double)n + 0.5);
    for (int it = 0; it < 100; ++it) {
      const double x = std::cos(th);
      const double s = std::sin(th);
      double p_prev = 1.0, p_cur = x;          // P_0, P_1
      for (int l = 2; l <= n; ++l) {
        const double p_next = ((double)(2 * l - 1) * x * p_cur - (double)(l - 1) * p_prev) / (double)l;
        p_prev = p_cur;
        p_cur = p_next;
      }
      const double d = (double)n * (p_prev - x * p_cur) / s;   // -dP_n/dt
      const double step = p_cur / d;
      const bool done = std::fabs(step) <= 1e-15 * th;
      th = th + step;
      if (done) break;
    }
    out[k] = th;
  }
  for (int k = 0; k < half; ++k) out[n - 1 - k] = M_PI - out[k];
}

namespace {

struct Tri {
  int32_t v[3];
};

inline Tri canonical(int32_t a, int32_t b, int32_t c) {
  // rotate so that the smallest index comes first, keeping the cyclic order
  if (a < b && a < c) return {{a, b, c}};
  if (b < a && b < c) return {{b, c, a}};
  return {{c, a, b}};
}

}  // namespace

int parse_grid_name(const std::string& name) {
  size_t b = 0, e = name.size();
  while (b < e && std::isspace((unsigned char)name[b])) ++b;
  while (e > b && std::isspace((unsigned char)name[e - 1])) --e;
  if (e - b < 2 || (name[b] != 'O' && name[b] != 'o')) return -1;
  long n = 0;
  for (size_t i = b + 1; i < e; ++i) {
    if (name[i] < '0' || name[i] > '9') return -1;
    n = n * 10 + (name[i] - '0');
    if (n > 1000000) return -1;
  }
  return n >= 1 ? (int)n : -1;
}

void build_host_mesh(int N, double radius, HostMesh& m) {
  if (N < 1) throw std::runtime_error("grid N must be >= 1");
  const int64_t Vexp = 4LL * N * N + 36LL * N;
  // slot and element offsets are kept in 32 bits per node table entry
  if (3 * Vexp > (int64_t)INT32_MAX) throw std::length_error("grid too large for 32-bit indices");
  m.N = N;
  m.radius = radius;
  const int n = 2 * N;
  m.nrows = n;

  // ---- grid ----------------------------------------------------------------
  m.row_size.resize(n);
  m.row_off.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    m.row_size[k] = 4 * std::min(k + 1, n - k) + 16;
    m.row_off[k + 1] = m.row_off[k] + m.row_size[k];
  }
  const int64_t V = m.row_off[n];
  m.V = V;
  gaussian_colatitudes(n, m.colat);

  m.node_row.resize(V);
  m.lon.resize(V);
  m.coslon.resize(V);
  m.sinlon.resize(V);
  m.sinlat.resize(V);
  m.coslat.resize(V);
  m.xyz.resize(3 * V);
  for (int k = 0; k < n; ++k) {
    const double sl = std::cos(m.colat[k]);
    const double cl = std::sin(m.colat[k]);
    const int nk = m.row_size[k];
    for (int j = 0; j < nk; ++j) {
      const int64_t g = m.row_off[k] + j;
      m.node_row[g] = k;
      m.lon[g] = (2.0 * M_PI * (double)j) / (double)nk;
      m.sinlat[g] = sl;
      m.coslat[g] = cl;
    }
  }
  for (int64_t g = 0; g < V; ++g) m.coslon[g] = std::cos(m.lon[g]);
  for (int64_t g = 0; g < V; ++g) m.sinlon[g] = std::sin(m.lon[g]);
  for (int64_t g = 0; g < V; ++g) {
    m.xyz[3 * g + 0] = m.coslat[g] * m.coslon[g];
    m.xyz[3 * g + 1] = m.coslat[g] * m.sinlon[g];
    m.xyz[3 * g + 2] = m.sinlat[g];
  }

  // ---- triangles ---------------------------------------------------------------
  std::vector<Tri> raw;
  raw.reserve(2 * V);
  for (int cap = 0; cap < 2; ++cap) {
    const int row = cap == 0 ? 0 : n - 1;
    const int32_t o = (int32_t)m.row_off[row];
    const int n0 = m.row_size[row];
    for (int j = 0; j < n0 / 2 - 1; ++j) {
      const int32_t p = o + j, q = o + j + 1, r = o + n0 - 1 - j, s = o + n0 - 2 - j;
      // longitude grows counter-clockwise seen from above the north pole and
      // clockwise seen from below the south pole
      if (cap == 0) {
        raw.push_back(canonical(p, q, r));
        raw.push_back(canonical(q, s, r));
      } else {
        raw.push_back(canonical(p, r, q));
        raw.push_back(canonical(q, r, s));
      }
    }
  }
  for (int k = 0; k + 1 < n; ++k) {
    const int64_t na = m.row_size[k], nb = m.row_size[k + 1];
    const int32_t oa = (int32_t)m.row_off[k], ob = (int32_t)m.row_off[k + 1];
    int64_t p = 0, q = 0;
    while (p < na || q < nb) {
      bool adv_a;
      if (q == nb) {
        adv_a = true;
      } else if (p == na) {
        adv_a = false;
      } else {
        const int64_t ka = (p + 1) * nb, kb = (q + 1) * na;
        adv_a = ka < kb || (ka == kb && na <= nb);
      }
      const int32_t ap = oa + (int32_t)(p % na), bq = ob + (int32_t)(q % nb);
      // with north up and east to the right, (a_p, b_q, x) is counter-clockwise
      if (adv_a) {
        raw.push_back(canonical(ap, bq, oa + (int32_t)((p + 1) % na)));
        ++p;
      } else {
        raw.push_back(canonical(ap, bq, ob + (int32_t)((q + 1) % nb)));
        ++q;
      }
    }
  }
  const int64_t T = (int64_t)raw.size();
  if (T != 2 * V - 4) throw std::runtime_error("triangle count mismatch");
  m.T = T;
  // counting sort by first vertex, then (second, third) within a bucket
  {
    std::vector<int64_t> start(V + 1, 0);
    for (const Tri& t : raw) ++start[t.v[0] + 1];
    for (int64_t i = 0; i < V; ++i) start[i + 1] += start[i];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    std::vector<Tri> sorted(T);
    for (const Tri& t : raw) sorted[fill[t.v[0]]++] = t;
    for (int64_t i = 0; i < V; ++i)
      std::sort(sorted.begin() + start[i], sorted.begin() + start[i + 1], [](const Tri& x, const Tri& y) {
        return x.v[1] != y.v[1] ? x.v[1] < y.v[1] : x.v[2] < y.v[2];
      });
    m.tris.resize(3 * T);
    for (int64_t t = 0; t < T; ++t)
      for (int s = 0; s < 3; ++s) m.tris[3 * t + s] = sorted[t].v[s];
  }

  // ---- edges -------------------------------------------------------------------
  // bucket each triangle side (lo, hi) by lo; a node has at most 7 higher
  // neighbours, each seen twice
  std::vector<int64_t> bstart(V + 1, 0);
  for (int64_t t = 0; t < T; ++t)
    for (int s = 0; s < 3; ++s) {
      const int32_t a = m.tris[3 * t + s], b = m.tris[3 * t + (s + 1) % 3];
      ++bstart[std::min(a, b) + 1];
    }
  for (int64_t i = 0; i < V; ++i) bstart[i + 1] += bstart[i];
  std::vector<int32_t> bhi(bstart[V]);
  {
    std::vector<int64_t> fill(bstart.begin(), bstart.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int s = 0; s < 3; ++s) {
        const int32_t a = m.tris[3 * t + s], b = m.tris[3 * t + (s + 1) % 3];
        bhi[fill[std::min(a, b)]++] = std::max(a, b);
      }
  }
  std::vector<int64_t> estart(V + 1, 0);   // first edge id whose lower end is i
  m.edges.clear();
  m.edges.reserve(2 * (3 * V - 6));
  for (int64_t i = 0; i < V; ++i) {
    estart[i] = (int64_t)m.edges.size() / 2;
    auto b0 = bhi.begin() + bstart[i], b1 = bhi.begin() + bstart[i + 1];
    std::sort(b0, b1);
    for (auto it = b0; it != b1; ++it) {
      if (it != b0 && *it == *(it - 1)) continue;
      m.edges.push_back((int32_t)i);
      m.edges.push_back(*it);
    }
  }
  const int64_t E = (int64_t)m.edges.size() / 2;
  estart[V] = E;
  if (E != 3 * V - 6) throw std::runtime_error("edge count mismatch");
  m.E = E;
  auto find_edge = [&](int32_t a, int32_t b) -> int32_t {
    const int32_t lo = std::min(a, b), hi = std::max(a, b);
    for (int64_t e = estart[lo]; e < estart[lo + 1]; ++e)
      if (m.edges[2 * e + 1] == hi) return (int32_t)e;
    throw std::runtime_error("edge lookup failed");
  };
  m.tri_edge.resize(3 * T);
  m.edge_tris.assign(2 * E, -1);
  {
    std::vector<uint8_t> cnt(E, 0);
    for (int64_t t = 0; t < T; ++t)
      for (int s = 0; s < 3; ++s) {
        const int32_t e = find_edge(m.tris[3 * t + s], m.tris[3 * t + (s + 1) % 3]);
        m.tri_edge[3 * t + s] = e;
        if (cnt[e] >= 2) throw std::runtime_error("edge shared by more than two triangles");
        m.edge_tris[2 * e + cnt[e]++] = (int32_t)t;
      }
    for (int64_t e = 0; e < E; ++e)
      if (cnt[e] != 2) throw std::runtime_error("open edge");
  }

  // ---- node -> slot CSR ------------------------------------------------------------
  m.csr_off.assign(V + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    ++m.csr_off[m.edges[2 * e] + 1];
    ++m.csr_off[m.edges[2 * e + 1] + 1];
  }
  for (int64_t i = 0; i < V; ++i) m.csr_off[i + 1] += m.csr_off[i];
  m.nbr.resize(2 * E);
  m.eid.resize(2 * E);
  m.sgn.resize(2 * E);
  m.rev.resize(2 * E);
  {
    // edges are sorted by (a, b): all (x, i) with x < i precede all (i, y),
    // so appending in edge order leaves every slot list sorted by neighbour
    std::vector<int64_t> fill(m.csr_off.begin(), m.csr_off.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t a = m.edges[2 * e], b = m.edges[2 * e + 1];
      int64_t s = fill[a]++;
      m.nbr[s] = b; m.eid[s] = (int32_t)e; m.sgn[s] = 1;
      s = fill[b]++;
      m.nbr[s] = a; m.eid[s] = (int32_t)e; m.sgn[s] = -1;
    }
  }
  m.max_degree = 0;
  for (int64_t i = 0; i < V; ++i) {
    const int deg = (int)(m.csr_off[i + 1] - m.csr_off[i]);
    if (deg > kEll - 1) throw std::runtime_error("node degree above 7");
    m.max_degree = std::max(m.max_degree, deg);
    for (int64_t s = m.csr_off[i]; s < m.csr_off[i + 1]; ++s) {
      const int32_t nb = m.nbr[s];
      int r = -1;
      for (int64_t t = m.csr_off[nb]; t < m.csr_off[nb + 1]; ++t)
        if (m.nbr[t] == (int32_t)i) { r = (int)(t - m.csr_off[nb]); break; }
      if (r < 0) throw std::runtime_error("reverse slot missing");
      m.rev[s] = (int8_t)r;
    }
  }
  m.is_pole.assign(E, 0);
  m.npole = 0;
  for (int64_t e = 0; e < E; ++e) {
    const int32_t a = m.edges[2 * e], b = m.edges[2 * e + 1];
    const int ra = m.node_row[a], rb = m.node_row[b];
    if (ra != rb || (ra != 0 && ra != n - 1)) continue;
    const int64_t dj = ((b - m.row_off[rb]) - (a - m.row_off[ra]) + kCapPoints) % kCapPoints;
    if (dj != 1 && dj != kCapPoints - 1) { m.is_pole[e] = 1; ++m.npole; }
  }

  // ---- median dual ---------------------------------------------------------------------
  std::vector<double> mid(3 * E), cen(3 * T);
  for (int64_t e = 0; e < E; ++e) {
    const V3 s = add(load3(m.xyz, m.edges[2 * e]), load3(m.xyz, m.edges[2 * e + 1]));
    const V3 u = normalized(s);
    for (int c = 0; c < 3; ++c) mid[3 * e + c] = u[c];
  }
  for (int64_t t = 0; t < T; ++t) {
    int32_t v[3] = {m.tris[3 * t], m.tris[3 * t + 1], m.tris[3 * t + 2]};
    std::sort(v, v + 3);
    const V3 s = add(add(load3(m.xyz, v[0]), load3(m.xyz, v[1])), load3(m.xyz, v[2]));
    const V3 u = normalized(s);
    for (int c = 0; c < 3; ++c) cen[3 * t + c] = u[c];
  }
  m.S.assign(3 * E, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    const V3 me = load3(mid, e);
    const V3 d = sub(load3(m.xyz, m.edges[2 * e + 1]), load3(m.xyz, m.edges[2 * e]));
    V3 acc = {0.0, 0.0, 0.0};
    for (int side = 0; side < 2; ++side) {
      const V3 c = load3(cen, m.edge_tris[2 * e + side]);
      // integrated conormal of the arc m_e -> c_T: R * angle * unit(m x c),
      // with m x c taken as m x (c - m)
      const V3 w = cross(me, sub(c, me));
      const double wn = std::sqrt(dot(w, w));
      const double ang = std::atan2(wn, dot(me, c));
      const double f = radius * ang / wn;
      V3 term = {f * w[0], f * w[1], f * w[2]};
      if (dot(term, d) < 0.0) term = {-term[0], -term[1], -term[2]};
      acc = add(acc, term);
    }
    for (int c = 0; c < 3; ++c) m.S[3 * e + c] = acc[c];
  }
  std::vector<double> area(V, 0.0);
  for (int r = 0; r < 3; ++r)
    for (int64_t t = 0; t < T; ++t) {
      const int32_t i = m.tris[3 * t + r];
      const V3 xi = load3(m.xyz, i);
      const V3 c = load3(cen, t);
      const V3 mij = load3(mid, m.tri_edge[3 * t + r]);
      const V3 mik = load3(mid, m.tri_edge[3 * t + (r + 2) % 3]);
      area[i] += tri_solid_angle(xi, mij, c) + tri_solid_angle(xi, c, mik);
    }
  m.vol.resize(V);
  for (int64_t i = 0; i < V; ++i) m.vol[i] = radius * radius * area[i];

  m.basis.resize(6 * V);
  for (int64_t i = 0; i < V; ++i) {
    double* b = &m.basis[6 * i];
    b[0] = -m.sinlon[i]; b[1] = m.coslon[i]; b[2] = 0.0;
    b[3] = -m.sinlat[i] * m.coslon[i]; b[4] = -m.sinlat[i] * m.sinlon[i]; b[5] = m.coslat[i];
  }
  m.C.assign(3 * V, 0.0);
  for (int64_t i = 0; i < V; ++i)
    for (int64_t s = m.csr_off[i]; s < m.csr_off[i + 1]; ++s) {
      const double sg = (double)m.sgn[s];
      for (int c = 0; c < 3; ++c) m.C[3 * i + c] += sg * m.S[3 * (int64_t)m.eid[s] + c];
    }
}

// Row-window metadata of node i (packed above the degree in the header slot):
// bits 0..7 the number cu of neighbours in the row above, bit 8 set when the
// node's slots, in neighbour order, read [row above (cu), left, right, row
// below] with the row-above and row-below neighbours consecutive in their
// rows without wrapping past the zero meridian.  Then a walk along the row
// can reuse the previous node's values: its self and right neighbour become
// this node's left and self, and the last neighbour above (below) of the
// previous node is this node's first neighbour above (below).  Polar rows
// (ladder chords) and nodes whose ranges wrap get 0.
int window_meta(const HostMesh& m, int64_t i, int deg) {
  const int k = m.node_row[i];
  if (k == 0 || k == m.nrows - 1) return 0;
  const int64_t s0 = m.csr_off[i];
  const int64_t rk = m.row_off[k], nk = m.row_size[k];
  const int64_t j = i - rk;
  if (j == 0 || j == nk - 1) return 0;
  int cu = 0;
  while (cu < deg && m.node_row[m.nbr[s0 + cu]] == k - 1) ++cu;
  const int cl = deg - cu - 2;
  if (cu < 1 || cl < 1 || cu > 3 || cl > 3) return 0;
  if (m.nbr[s0 + cu] != i - 1 || m.nbr[s0 + cu + 1] != i + 1) return 0;
  for (int t = 1; t < cu; ++t)
    if (m.nbr[s0 + t] != m.nbr[s0 + t - 1] + 1 || m.node_row[m.nbr[s0 + t]] != k - 1) return 0;
  for (int t = 0; t < cl; ++t) {
    const int32_t nb = m.nbr[s0 + cu + 2 + t];
    if (m.node_row[nb] != k + 1) return 0;
    if (t > 0 && nb != m.nbr[s0 + cu + 2 + t - 1] + 1) return 0;
  }
  return cu | (1 << 8);
}

// T_e = m_e x S_e, m_e the unit midpoint of edge e (normalised endpoint sum,
// evaluated as for the dual faces): the dual face conormal turned by a right
// angle about the local vertical, the tangential face flux of the curl.
static V3 face_tangent(const HostMesh& m, int64_t e, const V3& S) {
  const int64_t a = m.edges[2 * e], b = m.edges[2 * e + 1];
  const double x = m.xyz[3 * a] + m.xyz[3 * b], y = m.xyz[3 * a + 1] + m.xyz[3 * b + 1],
               z = m.xyz[3 * a + 2] + m.xyz[3 * b + 2];
  const double nrm = std::sqrt((x * x + y * y) + z * z);
  const double mx = x / nrm, my = y / nrm, mz = z / nrm;
  return {my * S[2] - mz * S[1], mz * S[0] - mx * S[2], mx * S[1] - my * S[0]};
}

// Per-slot coefficients (difference / gather form of the edge sums):
//   a_is = 0.5 sign (east_i . S_e) / V_i     b_is = 0.5 sign (north_i . S_e) / V_i
//   c_is = 0.5 sign (east_n . S_e) / V_i     d_is = 0.5 sign (north_n . S_e) / V_i
// with A_i = sum_s a_is, B_i = sum_s b_is.  Then
//   grad_i  = (sum_s a_is (f_n - f_i), sum_s b_is (f_n - f_i))
//   div_i   = A_i u_i + B_i v_i + sum_s (c_is u_n + d_is v_n)
//   gradT_m = -A_m wx_m - B_m wy_m + sum_s (a_{n,r} wx_n + b_{n,r} wy_n)
//   divT_m  = (A_m d_m + sum_s c_{n,r} d_n,  B_m d_m + sum_s d_{n,r} d_n)
// and curl, curlT as div, divT with T_e = m_e x S_e in place of S_e (A', B'
// the sums of the curl's own-basis terms).
// where r = rev(m, s) is m's slot in n's list.  The two-ring Laplacian weights
// W_im (m != i) satisfy lap_i = sum_m W_im (f_m - f_i) = div(grad f)_i.
void build_op_tables(const HostMesh& m, OpTables& t) {
  const int64_t V = m.V;
  t.nbr8.assign(kEll * V, 0);
  t.grad.assign(2 * kEll * V, 0.0);
  t.div.assign(2 * kEll * V, 0.0);
  t.gradT.assign(2 * kEll * V, 0.0);
  t.divT.assign(2 * kEll * V, 0.0);
  t.curl.assign(2 * kEll * V, 0.0);
  t.curlT.assign(2 * kEll * V, 0.0);
  for (int64_t i = 0; i < V; ++i) {
    const int64_t s0 = m.csr_off[i];
    const int deg = (int)(m.csr_off[i + 1] - s0);
    const V3 ei = {m.basis[6 * i], m.basis[6 * i + 1], m.basis[6 * i + 2]};
    const V3 ni = {m.basis[6 * i + 3], m.basis[6 * i + 4], m.basis[6 * i + 5]};
    double A = 0.0, B = 0.0, Ac = 0.0, Bc = 0.0;
    for (int s = 0; s < kEll - 1; ++s) t.nbr8[kEll * i + s] = (int32_t)i;
    for (int s = 0; s < deg; ++s) {
      const int32_t nb = m.nbr[s0 + s];
      const V3 Se = load3(m.S, m.eid[s0 + s]);
      const V3 en = {m.basis[6 * (int64_t)nb], m.basis[6 * (int64_t)nb + 1], m.basis[6 * (int64_t)nb + 2]};
      const V3 nn = {m.basis[6 * (int64_t)nb + 3], m.basis[6 * (int64_t)nb + 4], m.basis[6 * (int64_t)nb + 5]};
      const double h = 0.5 * (double)m.sgn[s0 + s] / m.vol[i];
      const double a = h * dot(ei, Se), b = h * dot(ni, Se);
      t.nbr8[kEll * i + s] = nb;
      t.grad[2 * (kEll * i + s)] = a;
      t.grad[2 * (kEll * i + s) + 1] = b;
      t.div[2 * (kEll * i + s)] = h * dot(en, Se);
      t.div[2 * (kEll * i + s) + 1] = h * dot(nn, Se);
      A += a;
      B += b;
      // curl: the face conormal turned about the unit edge midpoint
      const V3 Te = face_tangent(m, m.eid[s0 + s], Se);
      t.curl[2 * (kEll * i + s)] = h * dot(en, Te);
      t.curl[2 * (kEll * i + s) + 1] = h * dot(nn, Te);
      Ac += h * dot(ei, Te);
      Bc += h * dot(ni, Te);
    }
    t.nbr8[kEll * i + kEll - 1] = deg | (window_meta(m, i, deg) << 8);
    const int64_t dg = 2 * (kEll * i + kEll - 1);
    t.grad[dg] = A; t.grad[dg + 1] = B;
    t.div[dg] = A; t.div[dg + 1] = B;
    t.gradT[dg] = -A; t.gradT[dg + 1] = -B;
    t.divT[dg] = A; t.divT[dg + 1] = B;
    t.curl[dg] = Ac; t.curl[dg + 1] = Bc;
    t.curlT[dg] = Ac; t.curlT[dg + 1] = Bc;
  }
  for (int64_t i = 0; i < V; ++i) {
    const int64_t s0 = m.csr_off[i];
    const int deg = (int)(m.csr_off[i + 1] - s0);
    for (int s = 0; s < deg; ++s) {
      const int64_t nb = m.nbr[s0 + s];
      const int64_t src = 2 * (kEll * nb + m.rev[s0 + s]);
      const int64_t dst = 2 * (kEll * i + s);
      t.gradT[dst] = t.grad[src];
      t.gradT[dst + 1] = t.grad[src + 1];
      t.divT[dst] = t.div[src];
      t.divT[dst + 1] = t.div[src + 1];
      t.curlT[dst] = t.curl[src];
      t.curlT[dst + 1] = t.curl[src + 1];
    }
  }

  // two-ring Laplacian stencil
  struct Entry { int32_t node; double w; };
  std::vector<Entry> ring;
  int maxcnt = 0;
  std::vector<int32_t> cnt(V);
  std::vector<Entry> flat;
  flat.reserve(20 * V);
  std::vector<int64_t> fstart(V + 1, 0);
  for (int64_t i = 0; i < V; ++i) {
    ring.clear();
    auto add_w = [&](int32_t node, double w) {
      for (Entry& en : ring)
        if (en.node == node) { en.w += w; return; }
      ring.push_back({node, w});
    };
    const int deg_i = t.nbr8[kEll * i + kEll - 1] & 0xff;
    for (int s = -1; s < deg_i; ++s) {
      // s = -1: the node itself with the diagonal pair (A_i, B_i)
      const int64_t j = s < 0 ? i : t.nbr8[kEll * i + s];
      const int64_t cs = 2 * (kEll * i + (s < 0 ? kEll - 1 : s));
      const double alpha = t.div[cs], beta = t.div[cs + 1];
      const int deg_j = t.nbr8[kEll * j + kEll - 1] & 0xff;
      for (int u = 0; u < deg_j; ++u) {
        const int32_t mm = t.nbr8[kEll * j + u];
        const int64_t cu = 2 * (kEll * j + u);
        const double g = alpha * t.grad[cu] + beta * t.grad[cu + 1];
        if (mm != (int32_t)i) add_w(mm, g);
        if (j != i) add_w((int32_t)j, -g);
      }
    }
    // order: the 1-ring neighbours in slot order (so that a kernel can take
    // the gradient from the first deg_i differences), then the rest by index
    std::sort(ring.begin(), ring.end(), [](const Entry& x, const Entry& y) { return x.node < y.node; });
    {
      std::vector<Entry> ord;
      ord.reserve(ring.size());
      for (int s = 0; s < deg_i; ++s)
        for (const Entry& en : ring)
          if (en.node == t.nbr8[kEll * i + s]) ord.push_back(en);
      for (const Entry& en : ring) {
        bool nb = false;
        for (int s = 0; s < deg_i; ++s) nb = nb || en.node == t.nbr8[kEll * i + s];
        if (!nb) ord.push_back(en);
      }
      if (ord.size() != ring.size()) throw std::runtime_error("two-ring stencil misses a neighbour");
      ring.swap(ord);
    }
    cnt[i] = (int32_t)ring.size();
    maxcnt = std::max(maxcnt, (int)ring.size());
    flat.insert(flat.end(), ring.begin(), ring.end());
    fstart[i + 1] = (int64_t)flat.size();
  }
  if (maxcnt > kLapStride - 1) throw std::runtime_error("two-ring stencil wider than the kernel table");
  const int stride = kLapStride;
  t.lap_stride = stride;
  t.lap_nbr.assign((int64_t)stride * V, 0);
  t.lap_w.assign((int64_t)stride * V, 0.0);
  for (int64_t i = 0; i < V; ++i) {
    int32_t* nb = &t.lap_nbr[(int64_t)stride * i];
    double* w = &t.lap_w[(int64_t)stride * i];
    for (int s = 0; s < stride - 1; ++s) nb[s] = (int32_t)i;
    for (int64_t k = fstart[i]; k < fstart[i + 1]; ++k) {
      nb[k - fstart[i]] = flat[k].node;
      w[k - fstart[i]] = flat[k].w;
    }
    nb[stride - 1] = cnt[i];
  }
}

void build_band_runs(const HostMesh& m, int band_rows, int run_nodes, std::vector<int32_t>& runs_out) {
  if (band_rows < 1 || run_nodes < 1) throw std::runtime_error("band_rows and run_nodes must be >= 1");
  struct Run { int32_t j, n, row; };
  std::vector<Run> runs;
  runs_out.clear();
  for (int k0 = 0; k0 < m.nrows; k0 += band_rows) {
    const int k1 = std::min(m.nrows, k0 + band_rows);
    runs.clear();
    for (int k = k0; k < k1; ++k)
      for (int j = 0; j < m.row_size[k]; j += run_nodes) runs.push_back({j, m.row_size[k], k});
    std::sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) {
      const int64_t a = (int64_t)x.j * y.n, b = (int64_t)y.j * x.n;
      return a != b ? a < b : x.row < y.row;
    });
    for (const Run& r : runs) {
      runs_out.push_back((int32_t)(m.row_off[r.row] + r.j));
      runs_out.push_back(std::min(r.n, r.j + run_nodes) - r.j);
    }
  }
}

void build_band_order(const HostMesh& m, int band_rows, int run_nodes, std::vector<int32_t>& order) {
  if (band_rows < 1 || run_nodes < 1) throw std::runtime_error("band_rows and run_nodes must be >= 1");
  order.resize(m.V);
  struct Run { int32_t j, n, row; };
  std::vector<Run> runs;
  int64_t pos = 0;
  for (int k0 = 0; k0 < m.nrows; k0 += band_rows) {
    const int k1 = std::min(m.nrows, k0 + band_rows);
    runs.clear();
    for (int k = k0; k < k1; ++k)
      for (int j = 0; j < m.row_size[k]; j += run_nodes) runs.push_back({j, m.row_size[k], k});
    std::sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) {
      const int64_t a = (int64_t)x.j * y.n, b = (int64_t)y.j * x.n;
      return a != b ? a < b : x.row < y.row;
    });
    for (const Run& r : runs) {
      const int j1 = std::min(r.n, r.j + run_nodes);
      for (int j = r.j; j < j1; ++j) order[pos++] = (int32_t)(m.row_off[r.row] + j);
    }
  }
}

void build_halo_tiles(const HostMesh& m, const OpTables& t, int ring, int band_rows, int run_nodes,
                      int64_t col_bytes, int64_t row_bytes, int64_t budget_bytes, HaloTiles& out) {
  if (ring != 1 && ring != 2) throw std::runtime_error("ring must be 1 or 2");
  if (col_bytes <= 0 || row_bytes < 0 || budget_bytes <= 0) throw std::runtime_error("bad tile byte sizes");
  const int64_t V = m.V;
  const int stride = ring == 1 ? kEll : t.lap_stride;
  out = HaloTiles();
  out.ring = ring;
  out.stride = stride;
  out.loc.assign((size_t)V * stride, 0);
  if (band_rows < 1 || run_nodes < 1) throw std::runtime_error("tile rows and bands per sweep must be >= 1");

  // Candidate tiles: `band_rows` rows by one longitude sector.  Rows are
  // grouped into bands of band_rows rows and bands into sweeps of run_nodes
  // bands; a sweep is cut into S sectors of equal longitude, sector s of row
  // k holding nodes j in [ceil(s n_k / S), ceil((s + 1) n_k / S)).  S is set
  // so that a tile of the sweep's longest rows fits the budget.  Order:
  // sweep, sector, band -- tiles stacked in latitude follow each other, so
  // the halo rows they share are still in L2.
  std::vector<int32_t> gnodes;
  std::vector<int64_t> gstart;
  {
    const int h = band_rows, r = ring;
    for (int K0 = 0; K0 < m.nrows; K0 += h * run_nodes) {
      const int K1 = std::min(m.nrows, K0 + h * run_nodes);
      int64_t nmax = 1;
      for (int k = K0; k < K1; ++k) nmax = std::max<int64_t>(nmax, m.row_size[k]);
      const int64_t hh = h + 2 * r;
      int64_t w = (budget_bytes - hh * (2 + r) * col_bytes) / (hh * col_bytes + (int64_t)h * row_bytes);
      if (w < 1) w = 1;
      const int64_t S = (nmax + w - 1) / w;
      for (int64_t sct = 0; sct < S; ++sct)
        for (int b0 = K0; b0 < K1; b0 += h) {
          gstart.push_back((int64_t)gnodes.size());
          for (int k = b0; k < std::min(b0 + h, K1); ++k) {
            const int64_t n = m.row_size[k];
            const int64_t j0 = (sct * n + S - 1) / S, j1 = ((sct + 1) * n + S - 1) / S;
            for (int64_t j = j0; j < j1; ++j) gnodes.push_back((int32_t)(m.row_off[k] + j));
          }
          if ((int64_t)gnodes.size() == gstart.back()) gstart.pop_back();
        }
    }
    gstart.push_back((int64_t)gnodes.size());
  }

  // entries of node i (without i itself)
  auto entries = [&](int64_t i, int32_t* e) -> int {
    if (ring == 1) {
      const int deg = t.nbr8[kEll * i + kEll - 1] & 0xff;
      for (int s = 0; s < deg; ++s) e[s] = t.nbr8[kEll * i + s];
      return deg;
    }
    const int cnt = t.lap_nbr[(size_t)stride * i + stride - 1];
    for (int s = 0; s < cnt; ++s) e[s] = t.lap_nbr[(size_t)stride * i + s];
    return cnt;
  };

  std::vector<int64_t> stamp(V, -1);     // tile that already holds column v
  std::vector<int32_t> cols, nodes;      // current tile
  int64_t tile = 0;
  int32_t e[kLapStride];

  auto close_tile = [&]() {
    if (nodes.empty()) return;
    std::sort(cols.begin(), cols.end());
    const int32_t seg0 = (int32_t)(out.segs.size() / 2);
    out.info.push_back(seg0);
    out.info.push_back((int32_t)out.order.size());
    out.info.push_back((int32_t)cols.size());
    out.info.push_back((int32_t)nodes.size());
    out.run_off.push_back((int32_t)(out.runs.size() / 2));
    out.order.insert(out.order.end(), nodes.begin(), nodes.end());
    for (size_t c = 0; c < cols.size(); ++c) {
      if (c > 0 && cols[c] == cols[c - 1] + 1) {
        ++out.segs.back();
      } else {
        out.segs.push_back(cols[c]);
        out.segs.push_back(1);
      }
    }
    for (size_t q = 0; q < nodes.size(); ++q) {
      if (q > 0 && nodes[q] == nodes[q - 1] + 1) {
        ++out.runs.back();
      } else {
        out.runs.push_back(nodes[q]);
        out.runs.push_back(1);
      }
    }
    auto pos = [&](int32_t v) -> uint16_t {
      return (uint16_t)(std::lower_bound(cols.begin(), cols.end(), v) - cols.begin());
    };
    int32_t ce[kLapStride];
    for (int32_t i : nodes) {
      const int n = entries(i, ce);
      const uint16_t self = pos(i);
      uint16_t* l = &out.loc[(size_t)stride * i];
      for (int s = 0; s < stride - 1; ++s) l[s] = s < n ? pos(ce[s]) : self;
      l[stride - 1] = (uint16_t)(self | (n << kLocCountShift));
    }
    out.max_cols = std::max(out.max_cols, (int)cols.size());
    out.max_nodes = std::max(out.max_nodes, (int)nodes.size());
    cols.clear();
    nodes.clear();
    ++tile;
  };

  for (size_t g = 0; g + 1 < gstart.size(); ++g) {
    close_tile();   // a candidate tile never shares a tile with another
    for (int64_t q = gstart[g]; q < gstart[g + 1]; ++q) {
      const int32_t i = gnodes[q];
      const int n = entries(i, e);
      e[n] = i;
      int fresh = 0;
      for (int s = 0; s <= n; ++s) {
        bool dup = stamp[e[s]] == tile;
        for (int u = 0; u < s && !dup; ++u) dup = e[u] == e[s];
        fresh += !dup;
      }
      const int64_t need = (int64_t)(cols.size() + fresh) * col_bytes + (int64_t)(nodes.size() + 1) * row_bytes;
      if (!nodes.empty() && (need > budget_bytes || (int64_t)cols.size() + fresh > kMaxTileCols)) {
        close_tile();
        fresh = n + 1;   // every entry of a node is distinct
      }
      if ((int64_t)fresh * col_bytes + row_bytes > budget_bytes || fresh > kMaxTileCols)
        throw std::runtime_error("one node's stencil does not fit the LDS tile budget");
      for (int s = 0; s <= n; ++s)
        if (stamp[e[s]] != tile) {
          stamp[e[s]] = tile;
          cols.push_back(e[s]);
        }
      nodes.push_back(i);
    }
  }
  close_tile();
  out.ntiles = tile;
  // sentinel: one past the last tile
  out.info.push_back((int32_t)(out.segs.size() / 2));
  out.info.push_back((int32_t)out.order.size());
  out.info.push_back(0);
  out.info.push_back(0);
  out.run_off.push_back((int32_t)(out.runs.size() / 2));
}

}  // namespace atlasnabla
