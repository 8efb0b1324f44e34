// Host check of the LDS tile builder (build_halo_tiles): for a mesh and a
// tile geometry given on the command line it verifies that
//   - every node belongs to exactly one tile, listed in the tile-by-tile
//     node order at the tile's position,
//   - each tile's segments are in-range, sorted, disjoint runs of columns,
//   - each tile's footprint columns * col_bytes + nodes * row_bytes fits the
//     budget, and the column count fits the position field,
//   - every stored LDS position of a node names the right column (the
//     stencil entry in slot order, the node itself for padding and for the
//     own-position field) and the stored count equals the stencil size,
// and it emulates the tiled evaluation of the gradient (ring 1) or the
// two-ring Laplacian (ring 2) from the positions, which must equal a direct
// gather over the neighbour tables bit for bit.
// Usage: halo_tiles_check N nlev tile_rows sweep_bands ring col_bytes row_bytes budget
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <stdexcept>
#include <vector>

#include "mesh.hpp"

using namespace atlasnabla;

int main(int argc, char** argv) {
  if (argc != 9) {
    std::fprintf(stderr, "usage: %s N nlev tile_rows sweep_bands ring col_bytes row_bytes budget\n", argv[0]);
    return 2;
  }
  const int N = std::atoi(argv[1]), L = std::atoi(argv[2]), H = std::atoi(argv[3]), R = std::atoi(argv[4]);
  const int ring = std::atoi(argv[5]);
  const int64_t col_bytes = std::atoll(argv[6]), row_bytes = std::atoll(argv[7]), budget = std::atoll(argv[8]);
  HostMesh m;
  build_host_mesh(N, 6371220.0, m);
  OpTables t;
  build_op_tables(m, t);
  HaloTiles ht;
  try {
    build_halo_tiles(m, t, ring, H, R, col_bytes, row_bytes, budget, ht);
  } catch (const std::exception& e) {
    std::printf("REFUSED: %s\n", e.what());
    return 3;
  }
  const int stride = ht.stride;
  int bad = 0;
  auto err = [&](const char* what, int64_t a, int64_t b) {
    if (bad < 10) std::printf("FAIL %s (%lld, %lld)\n", what, (long long)a, (long long)b);
    ++bad;
  };
  if ((int64_t)ht.info.size() != 4 * (ht.ntiles + 1)) err("info size", (int64_t)ht.info.size(), ht.ntiles);
  if ((int64_t)ht.order.size() != m.V) err("order size", (int64_t)ht.order.size(), m.V);
  if ((int64_t)ht.run_off.size() != ht.ntiles + 1) err("run_off size", (int64_t)ht.run_off.size(), ht.ntiles);
  std::vector<int> seen(m.V, 0);
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  std::vector<double> f((size_t)m.V * L);
  for (double& x : f) x = nd(rng);
  const int oc = ring == 1 ? 2 : 1;
  std::vector<double> tiled((size_t)m.V * L * oc, NAN);
  double cols_total = 0;
  for (int64_t tl = 0; tl < ht.ntiles && bad < 10; ++tl) {
    const int32_t* in = &ht.info[4 * tl];
    const int seg0 = in[0], pos0 = in[1], ncols = in[2], nnodes = in[3], seg1 = in[4], pos1 = in[5];
    const int run0 = ht.run_off[tl], run1 = ht.run_off[tl + 1];
    if (pos1 - pos0 != nnodes) err("order span", tl, pos1 - pos0);
    if (ncols * col_bytes + nnodes * row_bytes > budget) err("over budget", tl, ncols);
    if (ncols > kMaxTileCols) err("too many columns", tl, ncols);
    std::vector<int32_t> col;
    for (int sg = seg0; sg < seg1; ++sg) {
      const int first = ht.segs[2 * sg], cnt = ht.segs[2 * sg + 1];
      if (first < 0 || cnt < 1 || first + cnt > m.V) err("segment range", first, cnt);
      if (!col.empty() && first <= col.back() + 1) err("segments not disjoint runs", first, col.back());
      for (int c = 0; c < cnt; ++c) col.push_back(first + c);
    }
    if ((int)col.size() != ncols) err("column count", (int64_t)col.size(), ncols);
    cols_total += ncols;
    int nn = 0;
    for (int r = run0; r < run1; ++r) {
      for (int q = 0; q < ht.runs[2 * r + 1]; ++q) {
        const int64_t i = ht.runs[2 * r] + q;
        if (i < 0 || i >= m.V) {
          err("run range", i, r);
          continue;
        }
        ++seen[i];
        if (pos0 + nn >= (int)ht.order.size() || ht.order[pos0 + nn] != i) err("order entry", tl, nn);
        ++nn;
        const uint16_t* l = &ht.loc[(size_t)stride * i];
        const int self = l[stride - 1] & kMaxTileCols, cnt = l[stride - 1] >> kLocCountShift;
        const int want_cnt = ring == 1 ? (t.nbr8[kEll * i + kEll - 1] & 0xff) : t.lap_nbr[(size_t)kLapStride * i + kLapStride - 1];
        if (cnt != want_cnt) err("entry count", i, cnt);
        if (self >= ncols || col[self] != i) err("own position", i, self);
        bool ok = self < ncols;
        for (int s = 0; s < stride - 1; ++s) {
          const int64_t want = s >= cnt ? i : (ring == 1 ? t.nbr8[kEll * i + s] : t.lap_nbr[(size_t)kLapStride * i + s]);
          if (l[s] >= ncols || col[l[s]] != want) {
            err("slot position", i, s);
            ok = false;
          }
        }
        if (!ok) continue;
        for (int k = 0; k < L; ++k) {
          const double x0 = f[(size_t)col[self] * L + k];
          if (ring == 1) {
            double ax = 0, ay = 0;
            for (int s = 0; s < cnt; ++s) {
              const double d = f[(size_t)col[l[s]] * L + k] - x0;
              ax = std::fma(t.grad[2 * (kEll * i + s)], d, ax);
              ay = std::fma(t.grad[2 * (kEll * i + s) + 1], d, ay);
            }
            tiled[2 * ((size_t)i * L + k)] = ax;
            tiled[2 * ((size_t)i * L + k) + 1] = ay;
          } else {
            double acc = 0;
            for (int s = 0; s < cnt; ++s)
              acc = std::fma(t.lap_w[(size_t)kLapStride * i + s], f[(size_t)col[l[s]] * L + k] - x0, acc);
            tiled[(size_t)i * L + k] = acc;
          }
        }
      }
    }
    if (nn != nnodes) err("node count", tl, nn);
  }
  for (int64_t i = 0; i < m.V && bad < 10; ++i)
    if (seen[i] != 1) err("node coverage", i, seen[i]);
  for (int64_t i = 0; i < m.V && bad < 10; ++i) {
    for (int k = 0; k < L; ++k) {
      const double x0 = f[(size_t)i * L + k];
      if (ring == 1) {
        const int deg = t.nbr8[kEll * i + kEll - 1] & 0xff;
        double ax = 0, ay = 0;
        for (int s = 0; s < deg; ++s) {
          const double d = f[(size_t)t.nbr8[kEll * i + s] * L + k] - x0;
          ax = std::fma(t.grad[2 * (kEll * i + s)], d, ax);
          ay = std::fma(t.grad[2 * (kEll * i + s) + 1], d, ay);
        }
        if (ax != tiled[2 * ((size_t)i * L + k)] || ay != tiled[2 * ((size_t)i * L + k) + 1]) err("tiled gradient", i, k);
      } else {
        const int cnt = t.lap_nbr[(size_t)kLapStride * i + kLapStride - 1];
        double acc = 0;
        for (int s = 0; s < cnt; ++s)
          acc = std::fma(t.lap_w[(size_t)kLapStride * i + s], f[(size_t)t.lap_nbr[(size_t)kLapStride * i + s] * L + k] - x0, acc);
        if (acc != tiled[(size_t)i * L + k]) err("tiled laplacian", i, k);
      }
    }
  }
  std::printf("O%d ring %d: %lld tiles, %.1f nodes and %.1f columns per tile, largest %d columns / %d nodes\n", N, ring,
              (long long)ht.ntiles, (double)m.V / ht.ntiles, cols_total / ht.ntiles, ht.max_cols, ht.max_nodes);
  std::printf(bad ? "FAILED\n" : "OK\n");
  return bad ? 1 : 0;
}
