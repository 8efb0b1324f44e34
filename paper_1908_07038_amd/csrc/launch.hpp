// Host-side interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace atlasnabla {

// OP_CURL and OP_CURLT run the divergence and divergence-adjoint kernels on
// their own coefficient tables (the curl is the divergence form with the
// tangential face vector).
enum Op : int { OP_GRAD = 0, OP_DIV = 1, OP_GRADT = 2, OP_DIVT = 3, OP_LAP = 4, OP_CURL = 5, OP_CURLT = 6,
                OP_COUNT = 7 };
// Gradient and two-ring Laplacian of one field in one pass over LDS tiles
// (one-tile form only): an internal kernel operator beyond the public ones.
constexpr int OP_GRADLAP = OP_COUNT;
// Divergence and curl of one vector field in one pass (one-tile form only).
constexpr int OP_DIVCURL = OP_COUNT + 1;
// Divergence and gradient adjoint of one vector field in one pass: the
// OP_DIVCURL kernel on records holding the divergence and gradient-adjoint
// coefficient rows (both operators combine a vector field's 1-ring values
// with a diagonal and one pair per slot, in slot order).
constexpr int OP_DIVGRADT = OP_COUNT + 2;
// Kernel template an operator runs with.
inline int kernel_op(int op) {
  return op == OP_CURL ? OP_DIV : op == OP_CURLT ? OP_DIVT : op == OP_DIVGRADT ? OP_DIVCURL : op;
}
enum Dtype : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Device tables of one mesh for one coefficient precision (FP64 for DT_F64,
// FP32 for DT_F32 and DT_BF16).
struct DevTables {
  const int32_t* nbr8 = nullptr;        // [V][8]
  const void* coef[OP_COUNT] = {};      // per Op (none for OP_LAP): [V][8] pairs
  const int32_t* lap_nbr = nullptr;     // [V][lap_stride]
  const void* lap_w = nullptr;          // [V][lap_stride]
  int lap_stride = 0;
};

struct Shape {
  int waves_per_block = 4;   // 64-lane waves per workgroup
  int nodes_per_wave = 1;    // node groups per wave per workgroup
  int blocks_per_cu = 4;     // persistent kernels only
  int xcd_remap = 1;         // contiguous slices of work per XCD
  int lanes_per_node = 0;    // 0: chosen from nlev; else 16, 32 or 64 (nlev > 32)
  int slices_per_iter = 0;   // 0: 3 (capped by the slice count); else 1..3
  int band_rows = 0;         // 0: kDefaultBandRows; rows per band of the node order
  int run_nodes = 0;         // 0: kDefaultRunNodes (kDefaultWindowRunNodes on the row-window walk)
  int nt_stores = 0;         // 0: default (off), 1: non-temporal output stores, 2: off
  int row_window = 0;        // 0: default (on), 1: on, 2: off -- row-window walk of 1-ring operators
  int lds_tiles = 0;         // 0: default (per operator and dtype, see resolve_shape), 1: on
                             // (persistent, double buffered), 2: off, 3: on (one tile per
                             // workgroup) -- LDS tile path (FP32/FP64, > 32 levels)
  int tile_kb = 0;           // 0: kDefaultTileKB; LDS budget of one tile in KiB (8..64)
  int tile_waves = 0;        // 0: 6; consumer waves per persistent tile workgroup
  int producer_waves = 0;    // 0: 2; producer (copy) waves per persistent tile workgroup
  int tile_wgs_per_cu = 0;   // 0: 1; persistent tile workgroups per CU
  int tile_levels = 0;       // 0: automatic; else levels per column chunk of a tile
  int batch_mode = 0;        // batched plans: 0 default (persistent), 1 persistent tiled, 2 field launches
  int batch_claim = 0;       // batched persistent form: tiles per work claim (0: kDefaultBatchClaim)
};

constexpr int kDefaultBandRows = 32;
constexpr int kDefaultRunNodes = 16;
constexpr int kDefaultWindowRunNodes = 64;
constexpr int kDefaultTileKB = 48;
constexpr int kDefaultTileRows = 4;    // LDS tiles: rows per tile (band_rows)
constexpr int kDefaultBatchClaim = 4;  // batched persistent form: tiles per work claim
constexpr int kDefaultTileSweep = 8;   // LDS tiles: bands swept together (run_nodes)
inline int band_rows_of(const Shape& s) { return s.band_rows > 0 ? s.band_rows : kDefaultBandRows; }
inline int run_nodes_of(const Shape& s) { return s.run_nodes > 0 ? s.run_nodes : kDefaultRunNodes; }
inline bool nt_of(const Shape& s) { return s.nt_stores == 1; }

// Device node order of a launch shape: the permutation of the nodes and the
// same order as runs of consecutive nodes (first node, count).
struct NodeOrder {
  const int32_t* order = nullptr;
  const int32_t* runs = nullptr;
  int64_t nruns = 0;
};

// Whether an operator walks rows with a register window (1-ring operators
// on columns of more than 32 levels, unless the shape turns it off).
bool uses_window(int op, int nlev, const Shape& sh);
// Lanes per node: nlev for columns of at most 32 levels (64 / nlev nodes per
// wave), else the width in {64, 32, 16} that wastes the fewest lanes.
int lanes_per_node(int nlev, const Shape& sh);
// Level slices per loop iteration of a lane (1..3), per-lane path.
int slices_per_iter(int nlev, const Shape& sh);
// Level slices (of 64) in flight per node step, row-window path (1..3).
int window_slices(int nlev, const Shape& sh);

// LDS tile path: device tiles of one tiling (see HaloTiles in mesh.hpp).
struct DevTiles {
  const int32_t* info = nullptr;
  const int32_t* segs = nullptr;
  const int32_t* order = nullptr;   // [V] nodes in tile order
  const uint16_t* loc = nullptr;    // [V][8 or 24] LDS positions (source of the records)
  int64_t ntiles = 0;
  int KL = 0, nchunks = 1;  // level chunk of the launch (set per call)
  uint32_t lds_bytes = 0;   // largest tile footprint
  int64_t col_bytes = 0, row_bytes = 0;   // LDS bytes per column chunk / node the tiling was cut for
};
// Geometry of a tiled launch: stencil ring, level chunking (KL levels per
// chunk), LDS bytes per column chunk and per node (table rows), budget.
struct TileGeom {
  int ring = 1, KL = 0, nchunks = 1;   // KL = 0: no geometry fits the budget
  int64_t col_bytes = 0, row_bytes = 0, budget = 0;
};
// The shape a launch runs with: lds_tiles = 0 picks the path (and tile
// parameters left at 0) from per-operator, per-dtype defaults.
Shape resolve_shape(int op, int dtype, int nlev, const Shape& sh);
bool uses_tiles(int op, int dtype, int nlev, const Shape& sh);
// Name of the kernel template instance a single-field launch with the
// resolved shape runs, e.g. "k_tile<float, 0, 3>".
void kernel_label(int op, int dtype, int nlev, const Shape& resolved, char* buf, int len);
TileGeom tile_geom(int op, int dtype, int nlev, const Shape& sh);
// Bytes of one node record of the tile path (LDS bytes per tile node).
int64_t tile_record_bytes(int op, int dtype);
// LDS bytes kept free behind a one-tile-per-workgroup buffer: lanes past a
// column's last level read (and drop) values beyond it, up to the next
// multiple of 64 U levels of a chunk (chunks of KL levels, the last one
// shorter; U slices per step).
int64_t tile_tail_bytes(int op, int dtype, int KL, int nlev, int U);
// Level slices per step of the one-tile form for chunks of KL levels: the
// whole 64-level slices (a remainder of 1..32 levels is evaluated in a packed
// pass, several nodes to a wave), at most 3 or slices_per_iter.
int tile_slices(int KL, const Shape& sh);
// Packs a tiling's node records for (op, dtype) into rec ([V] records in tile
// order: coefficients, LDS positions, node index).
hipError_t pack_tile_records(int op, int dtype, const DevTables& t, const int32_t* order, const uint16_t* loc,
                             int64_t V, void* rec, hipStream_t stream);
// out2: the gradient output of OP_GRADLAP (out: its Laplacian), the curl
// output of OP_DIVCURL and the gradient adjoint of OP_DIVGRADT (out: their
// divergence), else NULL.
hipError_t launch_tiles(int op, int dtype, const DevTiles& dt, const void* rec, int nlev, const void* in,
                        void* out, const Shape& shape, int num_cus, hipStream_t stream, void* out2 = nullptr);

// Single-field operator launch; in/out are device pointers of the dtype and
// `ord` the device node order work follows.
hipError_t launch_op(int op, int dtype, const DevTables& t, const NodeOrder& ord, int64_t V, int nlev,
                     const void* in, void* out, const Shape& shape, hipStream_t stream);

// Conservation sums: partial [nparts][nlev][2] doubles of scratch, then the
// final fixed-order pass into out_sum/out_abs.
int conservation_parts(int64_t V, int nlev);
hipError_t launch_conservation(int dtype, const double* vol, int64_t V, int nlev,
                               const void* div, double* scratch, double* out_sum,
                               double* out_abs, hipStream_t stream);

// Device array for the allocation-free conservation call's partial sums
// (conservation_parts(V, nlev) * nlev * 2 doubles must fit), one per GPU.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxScratchDevices = 64;
// Its device address on `device`, which must be the current device; looked
// up on the first call per device, then cached.
hipError_t scratch_address(int device, double** ptr);

// Remapping: out[t][k] = sum_j w[t][j] in[nodes[t][j]][k] over P target
// points; nodes [P][4] int32 (< V) and w [P][4] (FP64 for DT_F64, FP32
// otherwise), fourth entries unused; in is [V][nlev].
hipError_t launch_remap(int dtype, const int32_t* nodes, const void* w, int64_t V, int64_t P, int nlev,
                        const void* in, void* out, hipStream_t stream);
// Its transpose: out[n][k] = sum over e in [off[n], off[n+1]) of w[e] in[tt[e]][k]
// for the V source nodes (off [V+1] int64, tt int32 < P, w of the weight type;
// in is [P][nlev]); ht [V][2] and hw [V][2] repeat the first two entries of
// each node (zero past its count).
hipError_t launch_remap_adjoint(int dtype, const int64_t* off, const int32_t* tt, const void* w, const int32_t* ht,
                                const void* hw, int64_t V, int64_t P, int nlev, const void* in, void* out,
                                hipStream_t stream);

// Batched persistent launch: one kernel over many fields (tracers) of one
// operator on LDS tilings.  Per tracer: its fields, its tiling and records,
// its level chunk (at most the tiling's), chunks per column, slices per step
// and work items (tiles x chunks).
struct BatchTile {
  const void* in;
  void* out;
  void* out2;            // the gradient adjoint of a divergence pair (OP_DIVGRADT), else NULL
  const int32_t* info;   // the tracer's tiling (DevTiles::info, segs) and its node records
  const int32_t* segs;
  const char* rec;
  int64_t nitems;
  int32_t L, KL, nchunks, U;
};
// tr: device [ntr] descriptors; pre: device [8][ntr + 1] item counts of each
// XCD before each tracer (see k_tile_batched); ctr: device int32 work
// counters (kBatchCounterInts of them), zero before the first launch (each
// launch leaves them zero; two launches with the same counters must not
// overlap in time); claim: consecutive items per counter claim (1..64);
// lds: bytes per
// workgroup (the largest tile of the tracers' tilings plus the read-past
// tail of every tracer); grid: a multiple of 8 workgroups of `waves` waves;
// umax: the largest U of the descriptors (1..3), which picks the kernel
// instance.
hipError_t launch_tiles_batched(int op, int dtype, const BatchTile* tr, const int32_t* pre, int ntr, int32_t* ctr,
                                int32_t claim, uint32_t lds, int waves, int64_t grid, int umax,
                                hipStream_t stream);
// Work counters of the batched kernel: a claim counter and a finished count
// (kBatchCtrStride / 2 further on) per XCD share, each share on its own
// 256-byte span.
constexpr int kBatchCtrStride = 64;
constexpr int kBatchCounterInts = 8 * kBatchCtrStride;
// Workgroups of the batched kernel instance one CU holds at once (registers,
// waves and `lds` bytes of LDS), 0 if it does not launch.
int tiles_batched_per_cu(int op, int dtype, uint32_t lds, int waves, int umax);

}  // namespace atlasnabla
