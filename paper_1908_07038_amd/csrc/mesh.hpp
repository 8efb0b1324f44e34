// Host-side mesh of an octahedral reduced Gaussian grid with its median dual
// and the per-node operator tables the gfx950 kernels read.
//
// The Atlas report describes Grid -> Mesh -> FunctionSpace -> Field
// (Section 2.3, Figure 2) and leaves grid and mesh generation to other
// documents; the definitions implemented here are stated in
// include/atlas_nabla.h (atlas_mesh_build) and in mesh_build.cpp.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace atlasnabla {

constexpr int kCapPoints = 20;   // points of each polar row
constexpr int kEll = 8;          // slots per node record: 7 neighbours + 1 header
constexpr int kLapStride = 24;   // two-ring record: up to 23 entries + the count

struct HostMesh {
  int N = 0;
  double radius = 0.0;
  int nrows = 0;
  int64_t V = 0, E = 0, T = 0;

  std::vector<int32_t> row_size;   // [nrows]
  std::vector<int64_t> row_off;    // [nrows+1]
  std::vector<double> colat;       // [nrows]
  std::vector<int32_t> node_row;   // [V]
  std::vector<double> lon, coslon, sinlon, sinlat, coslat;  // [V]
  std::vector<double> xyz;         // [V][3]

  std::vector<int32_t> tris;       // [T][3]
  std::vector<int32_t> edges;      // [E][2]
  std::vector<int32_t> tri_edge;   // [T][3], side s = (t_s, t_s+1)
  std::vector<int32_t> edge_tris;  // [E][2], ascending
  std::vector<int64_t> csr_off;    // [V+1]
  std::vector<int32_t> nbr, eid;   // [2E]
  std::vector<int8_t> sgn, rev;    // [2E]
  std::vector<uint8_t> is_pole;    // [E]
  int64_t npole = 0;
  int max_degree = 0;

  std::vector<double> S;           // [E][3] dual normals (m)
  std::vector<double> vol;         // [V] dual areas (m^2)
  std::vector<double> basis;       // [V][2][3] east, north
  std::vector<double> C;           // [V][3] closure
};

// Per-node operator tables in FP64, later rounded to FP32 for the FP32 and
// BF16 kernels.  Record layout per node (kEll slots):
//   nbr8[i][s]   neighbour of slot s (s < deg), i itself for s >= deg,
//   nbr8[i][7]   deg | cu << 8 | window-eligible << 16 (see window_meta)
//   coef[i][s]   (x, y) coefficient pair of slot s, (0, 0) padding,
//   coef[i][7]   the diagonal pair of the operator.
struct OpTables {
  std::vector<int32_t> nbr8;        // [V][8]
  std::vector<double> grad;         // [V][8][2]  (a, b); diag (A, B)
  std::vector<double> div;          // [V][8][2]  (c, d); diag (A, B)
  std::vector<double> gradT;        // [V][8][2]  (a, b) of the reverse slot; diag (-A, -B)
  std::vector<double> divT;         // [V][8][2]  (c, d) of the reverse slot; diag (A, B)
  std::vector<double> curl;         // [V][8][2]  (c', d') with T_e = m_e x S_e for S_e; diag (A', B')
  std::vector<double> curlT;        // [V][8][2]  (c', d') of the reverse slot; diag (A', B')
  int lap_stride = kLapStride;      // entries per node in the two-ring table
  std::vector<int32_t> lap_nbr;     // [V][lap_stride]: neighbours (the 1-ring ones first, in
                                    // slot order, then the rest by index), then padding (i);
                                    // entry lap_stride-1 holds the count
  std::vector<double> lap_w;        // [V][lap_stride]
};

// Parse "O<N>"; returns N or -1.
int parse_grid_name(const std::string& name);

// Colatitudes (ascending) of the n roots of P_n(cos t), n even: Newton in t
// from pi (k + 0.75) / (n + 0.5), mirrored about the equator.
void gaussian_colatitudes(int n, std::vector<double>& out);

// Build grid, connectivity and dual geometry.  Throws std::runtime_error /
// std::bad_alloc on failure.
void build_host_mesh(int N, double radius, HostMesh& m);

// Build the per-node tables from the geometry.
void build_op_tables(const HostMesh& m, OpTables& t);

// Processing order of the nodes for cache reuse: the rows are cut into bands
// of `band_rows` rows and each row into runs of `run_nodes` consecutive
// nodes; within a band, runs are ordered by the longitude of their first node
// (exact rational comparison j/n_k), then by row.  Work walks this order, so
// the rows above and below a node are visited at the same longitude and stay
// in cache (only rows at band edges are fetched twice), while the nodes of a
// run, whose columns share cache lines, are processed together.
void build_band_order(const HostMesh& m, int band_rows, int run_nodes, std::vector<int32_t>& order);
// The same runs as pairs (first node, node count), in the same order.
void build_band_runs(const HostMesh& m, int band_rows, int run_nodes, std::vector<int32_t>& runs);
// Row-window metadata of a node (see mesh_build.cpp); packed in the header
// slot of the neighbour table above the degree: deg | meta << 8.
int window_meta(const HostMesh& m, int64_t i, int deg);

// LDS tiles.  A tile is a set of nodes (band_rows consecutive rows by one
// longitude sector; see mesh_build.cpp) together with every column its
// stencils read: the one-ring (ring 1) or two-ring (ring 2) entries of each
// node and the node itself.
// The sorted column set is stored as segments of consecutive nodes, so a
// workgroup copies it from HBM with contiguous loads; column c of the set
// (in ascending node order) sits at position c of the tile's LDS buffer.
// loc[i][s] is the LDS position of entry s of node i (padded with the
// node's own position), and the last entry packs the node's own position
// with its entry count: pos | count << kLocCountShift.
constexpr int kLocCountShift = 11;
constexpr int kMaxTileCols = (1 << kLocCountShift) - 1;

struct HaloTiles {
  int ring = 1;
  int stride = 8;                  // loc entries per node: 8 (ring 1) or kLapStride (ring 2)
  int64_t ntiles = 0;
  std::vector<int32_t> info;       // [ntiles + 1][4]: first segment, first position in order, columns, nodes
  std::vector<int32_t> segs;       // [nseg][2]: first node, count
  std::vector<int32_t> order;      // [V]: the nodes, tile by tile
  std::vector<int32_t> runs;       // [nrun][2]: first node, count (the tiles' nodes as runs)
  std::vector<int32_t> run_off;    // [ntiles + 1]: first run of each tile
  std::vector<uint16_t> loc;       // [V][stride]
  int max_cols = 0, max_nodes = 0; // largest tile
};

// Cut the mesh into tiles of band_rows rows by one longitude sector, swept
// run_nodes bands at a time, whose LDS footprint, columns * col_bytes +
// nodes * row_bytes, stays within budget_bytes (and at most kMaxTileCols
// columns); a sector tile that does not fit is split row-major.  Throws
// std::runtime_error when a single node does not fit.
void build_halo_tiles(const HostMesh& m, const OpTables& t, int ring, int band_rows, int run_nodes,
                      int64_t col_bytes, int64_t row_bytes, int64_t budget_bytes, HaloTiles& out);

// Remapping from an O-grid mesh to the points of a target grid by linear
// interpolation over the source triangles in 3-D on the sphere (see
// remap_build.cpp): per target point the three nodes of the triangle its ray
// meets and their barycentric weights.
struct RemapHost {
  std::string target;             // canonical target name, "F<M>" or "O<M>"
  int64_t P = 0;                  // target points
  std::vector<double> xyz;        // [P][3] unit vectors
  std::vector<int32_t> nodes;     // [P][4]: three source nodes, 0 padding
  std::vector<double> w;          // [P][4]: their weights, 0 padding
  int64_t fallback = 0;           // points located by the exhaustive search
  // transpose (adjoint) in compressed rows by source node: the entries
  // (target point, weight) of node n are adj_t/adj_w[adj_off[n] .. adj_off[n+1]),
  // in ascending target order
  std::vector<int64_t> adj_off;   // [V+1]
  std::vector<int32_t> adj_t;     // [3P]
  std::vector<double> adj_w;      // [3P]
};

// Parse "F<M>" or "O<M>"; returns M (kind in *kind) or -1.
int parse_target_name(const std::string& name, char* kind);

// Target points and their source triangles and weights.  Throws
// std::runtime_error when a point lies in no triangle (cannot happen on a
// closed mesh) and std::bad_alloc when memory runs out.
void build_remap(const HostMesh& src, const std::string& target, RemapHost& out);

}  // namespace atlasnabla
