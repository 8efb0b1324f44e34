// C ABI of the Nabla library (declared in include/atlas_nabla.h): argument
// checking, mesh ownership, device upload of the operator tables, and
// dispatch to the gfx950 kernels.  No C++ exception crosses this layer.
#include "atlas_nabla.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mesh.hpp"

using namespace atlasnabla;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(ATLAS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Current-device guard: operator calls run on the mesh's device and leave the
// caller's current device unchanged.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

size_t dtype_size(int dtype) {
  switch (dtype) {
    case ATLAS_F64: return 8;
    case ATLAS_F32: return 4;
    case ATLAS_BF16: return 2;
    default: return 0;
  }
}

}  // namespace

struct atlas_mesh_s {
  HostMesh host;
  int device = -1;
  int num_cus = 0;
  std::vector<void*> allocations;
  DevTables tab64, tab32;
  double* vol = nullptr;
  std::mutex scratch_mu;
  double* scratch = nullptr;
  size_t scratch_bytes = 0;
  Shape shape[OP_COUNT][3];
  std::mutex order_mu;
  std::map<std::pair<int, int>, NodeOrder> orders;   // (band rows, run) -> device node order
  OpTables host_nbr;                                   // neighbour tables only (tile building)
  std::map<std::vector<int64_t>, DevTiles> tilings;   // tiling key -> device tiles
  std::map<std::vector<int64_t>, void*> records;      // tiling key + (op, dtype) -> packed node records

  ~atlas_mesh_s() {
    if (device >= 0) {
      DeviceGuard g(device);
      for (void* p : allocations) (void)hipFree(p);
      if (scratch) (void)hipFree(scratch);
    }
  }

  template <class T>
  T* upload(const std::vector<T>& v) {
    void* p = nullptr;
    const size_t bytes = v.size() * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e != hipSuccess) throw std::bad_alloc();
    allocations.push_back(p);
    if (bytes) {
      e = hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) throw std::runtime_error(std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    return static_cast<T*>(p);
  }

  const DevTables& tables(int dtype) const { return dtype == ATLAS_F64 ? tab64 : tab32; }

  // Device node order for a launch shape, built and uploaded on first use.
  NodeOrder order(const Shape& sh) {
    const std::pair<int, int> key(band_rows_of(sh), run_nodes_of(sh));
    std::lock_guard<std::mutex> lk(order_mu);
    auto it = orders.find(key);
    if (it != orders.end()) return it->second;
    std::vector<int32_t> ord, runs;
    build_band_order(host, key.first, key.second, ord);
    build_band_runs(host, key.first, key.second, runs);
    NodeOrder no;
    no.order = upload(ord);
    no.runs = upload(runs);
    no.nruns = (int64_t)runs.size() / 2;
    orders[key] = no;
    return no;
  }

  // Device tiles of an LDS-tiled launch, built and uploaded on first use.
  DevTiles tiles(const TileGeom& g, const Shape& sh) {
    const int h = sh.band_rows > 0 ? sh.band_rows : kDefaultTileRows;
    const int sweep = sh.run_nodes > 0 ? sh.run_nodes : kDefaultTileSweep;
    const std::vector<int64_t> key = {g.ring, h, sweep, g.col_bytes, g.row_bytes, g.budget};
    std::lock_guard<std::mutex> lk(order_mu);
    auto it = tilings.find(key);
    if (it != tilings.end()) return it->second;
    HaloTiles ht;
    build_halo_tiles(host, host_nbr, g.ring, h, sweep, g.col_bytes, g.row_bytes, g.budget, ht);
    DevTiles dt;
    // eight pairs of padding: kernels fetch pairs eight at a time
    ht.segs.resize(ht.segs.size() + 16, 0);
    dt.info = upload(ht.info);
    dt.segs = upload(ht.segs);
    dt.order = upload(ht.order);
    dt.loc = upload(ht.loc);
    dt.ntiles = ht.ntiles;
    dt.col_bytes = g.col_bytes;
    dt.row_bytes = g.row_bytes;
    int64_t lds = 0;
    for (int64_t t = 0; t < ht.ntiles; ++t)
      lds = std::max(lds, ht.info[4 * t + 2] * g.col_bytes + ht.info[4 * t + 3] * g.row_bytes);
    dt.lds_bytes = (uint32_t)lds;
    tilings[key] = dt;
    return dt;
  }

  // Node records of a tiling for (op, dtype), packed on the device on first
  // use (one allocation of V records, kept until the mesh is freed).
  const void* tile_records(const TileGeom& g, const Shape& sh, const DevTiles& dt, int op, int dtype,
                           hipStream_t stream) {
    const int h = sh.band_rows > 0 ? sh.band_rows : kDefaultTileRows;
    const int sweep = sh.run_nodes > 0 ? sh.run_nodes : kDefaultTileSweep;
    const std::vector<int64_t> key = {g.ring, h, sweep, g.col_bytes, g.row_bytes, g.budget, op, dtype};
    std::lock_guard<std::mutex> lk(order_mu);
    auto it = records.find(key);
    if (it != records.end()) return it->second;
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)host.V * tile_record_bytes(op, dtype)) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    allocations.push_back(p);
    hipError_t e = pack_tile_records(op, dtype, tables(dtype), dt.order, dt.loc, host.V, p, stream);
    // finished before any stream may read the records
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) throw std::runtime_error(std::string("packing tile records: ") + hipGetErrorString(e));
    records[key] = p;
    return p;
  }
};

namespace {

std::vector<float> to_f32(const std::vector<double>& v) {
  std::vector<float> r(v.size());
  for (size_t i = 0; i < v.size(); ++i) r[i] = (float)v[i];
  return r;
}

void upload_tables(atlas_mesh_s& m) {
  OpTables t;
  build_op_tables(m.host, t);
  const int32_t* nbr8 = m.upload(t.nbr8);
  const int32_t* lap_nbr = m.upload(t.lap_nbr);
  m.tab64.nbr8 = m.tab32.nbr8 = nbr8;
  m.tab64.lap_nbr = m.tab32.lap_nbr = lap_nbr;
  m.tab64.lap_stride = m.tab32.lap_stride = t.lap_stride;
  const std::vector<double>* src[OP_COUNT] = {&t.grad, &t.div, &t.gradT, &t.divT, nullptr, &t.curl, &t.curlT};
  for (int o = 0; o < OP_COUNT; ++o) {
    if (!src[o]) continue;
    m.tab64.coef[o] = m.upload(*src[o]);
    m.tab32.coef[o] = m.upload(to_f32(*src[o]));
  }
  m.tab64.lap_w = m.upload(t.lap_w);
  m.tab32.lap_w = m.upload(to_f32(t.lap_w));
  m.vol = m.upload(m.host.vol);
  m.host_nbr.nbr8 = std::move(t.nbr8);
  m.host_nbr.lap_nbr = std::move(t.lap_nbr);
  m.host_nbr.lap_stride = t.lap_stride;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

int op_from_bit(uint32_t bit) {
  switch (bit) {
    case ATLAS_OP_GRADIENT: return OP_GRAD;
    case ATLAS_OP_DIVERGENCE: return OP_DIV;
    case ATLAS_OP_GRADIENT_ADJOINT: return OP_GRADT;
    case ATLAS_OP_DIVERGENCE_ADJOINT: return OP_DIVT;
    case ATLAS_OP_LAPLACIAN: return OP_LAP;
    case ATLAS_OP_CURL: return OP_CURL;
    case ATLAS_OP_CURL_ADJOINT: return OP_CURLT;
    default: return -1;
  }
}

// components of the input and output fields of each operator
const int kInComps[OP_COUNT] = {1, 2, 2, 1, 1, 2, 1};
const int kOutComps[OP_COUNT] = {2, 1, 1, 2, 1, 1, 2};
const char* kOpName[OP_COUNT] = {"gradient", "divergence", "gradient_adjoint", "divergence_adjoint", "laplacian",
                                 "curl", "curl_adjoint"};

int check_mesh_device(atlas_mesh_t mesh) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  if (mesh->device < 0) return fail(ATLAS_ENODEV, "mesh was built host-only (device = -1)");
  return ATLAS_OK;
}

int check_field(const void* p, size_t comps, size_t esize, const char* name) {
  if (!p) return fail(ATLAS_EINVAL, std::string(name) + " is NULL");
  if ((uintptr_t)p % (comps * esize) != 0)
    return fail(ATLAS_EINVAL, std::string(name) + " is not aligned to " + std::to_string(comps * esize) + " bytes");
  return ATLAS_OK;
}

void shape_out(const Shape& s, atlas_tune_t* t) {
  t->waves_per_block = s.waves_per_block;
  t->nodes_per_wave = s.nodes_per_wave;
  t->blocks_per_cu = s.blocks_per_cu;
  t->xcd_remap = s.xcd_remap ? 1 : 2;
  t->lanes_per_node = s.lanes_per_node;
  t->slices_per_iter = s.slices_per_iter;
  t->band_rows = s.band_rows;
  t->run_nodes = s.run_nodes;
  t->nt_stores = s.nt_stores;
  t->row_window = s.row_window;
  t->lds_tiles = s.lds_tiles;
  t->tile_kb = s.tile_kb;
  t->tile_waves = s.tile_waves;
  t->producer_waves = s.producer_waves;
  t->tile_wgs_per_cu = s.tile_wgs_per_cu;
  t->tile_levels = s.tile_levels;
  t->batch_mode = s.batch_mode;
  t->batch_claim = s.batch_claim;
}

int check_shape(Shape& s, const atlas_tune_t* t) {
  if (!t) return ATLAS_OK;
  if (t->waves_per_block) {
    const int w = t->waves_per_block;
    if (w != 1 && w != 2 && w != 4 && w != 8 && w != 16)
      return fail(ATLAS_EINVAL, "waves_per_block must be 1, 2, 4, 8 or 16");
    s.waves_per_block = w;
  }
  if (t->nodes_per_wave) {
    if (t->nodes_per_wave < 1 || t->nodes_per_wave > 64) return fail(ATLAS_EINVAL, "nodes_per_wave must be 1..64");
    s.nodes_per_wave = t->nodes_per_wave;
  }
  if (t->blocks_per_cu) {
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return fail(ATLAS_EINVAL, "blocks_per_cu must be 1..64");
    s.blocks_per_cu = t->blocks_per_cu;
  }
  if (t->xcd_remap < 0 || t->xcd_remap > 2) return fail(ATLAS_EINVAL, "xcd_remap must be 0, 1 or 2");
  if (t->xcd_remap) s.xcd_remap = t->xcd_remap == 1 ? 1 : 0;
  const int p = t->lanes_per_node;
  if (p != 0 && p != 16 && p != 32 && p != 64) return fail(ATLAS_EINVAL, "lanes_per_node must be 0, 16, 32 or 64");
  s.lanes_per_node = p;
  if (t->slices_per_iter < 0 || t->slices_per_iter > 3) return fail(ATLAS_EINVAL, "slices_per_iter must be 0..3");
  s.slices_per_iter = t->slices_per_iter;
  if (t->band_rows < 0 || t->band_rows > 65536) return fail(ATLAS_EINVAL, "band_rows must be 0..65536");
  s.band_rows = t->band_rows;
  if (t->run_nodes < 0 || t->run_nodes > 65536) return fail(ATLAS_EINVAL, "run_nodes must be 0..65536");
  s.run_nodes = t->run_nodes;
  if (t->nt_stores < 0 || t->nt_stores > 2) return fail(ATLAS_EINVAL, "nt_stores must be 0, 1 or 2");
  s.nt_stores = t->nt_stores;
  if (t->row_window < 0 || t->row_window > 2) return fail(ATLAS_EINVAL, "row_window must be 0, 1 or 2");
  s.row_window = t->row_window;
  if (t->lds_tiles < 0 || t->lds_tiles > 3) return fail(ATLAS_EINVAL, "lds_tiles must be 0..3");
  s.lds_tiles = t->lds_tiles;
  if (t->tile_kb != 0 && (t->tile_kb < 8 || t->tile_kb > 160)) return fail(ATLAS_EINVAL, "tile_kb must be 0 or 8..160");
  s.tile_kb = t->tile_kb;
  if (t->tile_waves < 0 || t->tile_waves > 15) return fail(ATLAS_EINVAL, "tile_waves must be 0..15");
  if (t->producer_waves < 0 || t->producer_waves > 8 || (t->producer_waves & (t->producer_waves - 1)))
    return fail(ATLAS_EINVAL, "producer_waves must be 0, 1, 2, 4 or 8");
  if ((t->tile_waves ? t->tile_waves : 6) + (t->producer_waves ? t->producer_waves : 2) > 16)
    return fail(ATLAS_EINVAL, "tile_waves + producer_waves must be at most 16 (8 for FP64 launches)");
  s.tile_waves = t->tile_waves;
  s.producer_waves = t->producer_waves;
  if (t->tile_wgs_per_cu < 0 || t->tile_wgs_per_cu > 4) return fail(ATLAS_EINVAL, "tile_wgs_per_cu must be 0..4");
  s.tile_wgs_per_cu = t->tile_wgs_per_cu;
  if (t->tile_levels < 0) return fail(ATLAS_EINVAL, "tile_levels must be >= 0");
  s.tile_levels = t->tile_levels;
  if (t->batch_mode < 0 || t->batch_mode > 2) return fail(ATLAS_EINVAL, "batch_mode must be 0, 1 or 2");
  s.batch_mode = t->batch_mode;
  if (t->batch_claim < 0 || t->batch_claim > 64) return fail(ATLAS_EINVAL, "batch_claim must be 0..64");
  s.batch_claim = t->batch_claim;

  return ATLAS_OK;
}

int run_op(atlas_mesh_t mesh, int op, int dtype, int32_t nlev, const void* in, void* out, void* stream,
           const Shape* shape_override = nullptr) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  const int64_t V = mesh->host.V;
  // node-level indices are 32-bit inside the kernels
  if ((int64_t)nlev * V > (int64_t)UINT32_MAX) return fail(ATLAS_ESHAPE, "nnodes * nlev exceeds 2^32 - 1");
  if ((rc = check_field(in, kInComps[op], es, "input"))) return rc;
  if ((rc = check_field(out, kOutComps[op], es, "output"))) return rc;
  const size_t nin = (size_t)V * nlev * kInComps[op] * es;
  const size_t nout = (size_t)V * nlev * kOutComps[op] * es;
  if (overlaps(in, nin, out, nout)) return fail(ATLAS_EINVAL, "output overlaps input");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  Shape sh = resolve_shape(op, dtype, nlev, shape_override ? *shape_override : mesh->shape[op][dtype]);
  TileGeom tg = uses_tiles(op, dtype, nlev, sh) ? tile_geom(op, dtype, nlev, sh) : TileGeom();
  // BF16 tiles copy whole dwords around each column segment: they need a
  // 4-byte aligned field (else the row-window walk or gather runs)
  if (dtype == ATLAS_BF16 && ((uintptr_t)in & 3u)) tg.KL = 0;
  if (tg.KL > 0) {   // tiles asked for and a tile geometry fits the budget
    DevTiles dt;
    const void* rec = nullptr;
    try {
      // tilings depend on the byte sizes only; the level chunk is the call's
      dt = mesh->tiles(tg, sh);
      dt.KL = tg.KL;
      dt.nchunks = tg.nchunks;
      rec = mesh->tile_records(tg, sh, dt, op, dtype, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
      return fail(ATLAS_ENOMEM, "cannot allocate the LDS tiles");
    } catch (const std::exception& ex) {
      return fail(ATLAS_EHIP, ex.what());
    }
    hipError_t e = launch_tiles(op, dtype, dt, rec, nlev, in, out, sh, mesh->num_cus, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, kOpName[op]);
    return ATLAS_OK;
  }
  // the row-window walk works best on long runs
  if (sh.run_nodes == 0 && uses_window(op, nlev, sh)) sh.run_nodes = kDefaultWindowRunNodes;
  NodeOrder order;
  try {
    order = mesh->order(sh);
  } catch (const std::bad_alloc&) {
    return fail(ATLAS_ENOMEM, "cannot allocate the node order");
  } catch (const std::exception& ex) {
    return fail(ATLAS_EHIP, ex.what());
  }
  hipError_t e = launch_op(op, dtype, mesh->tables(dtype), order, V, nlev, in, out, sh, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, kOpName[op]);
  return ATLAS_OK;
}

}  // namespace

extern "C" {

const char* atlas_version(void) { return "atlas-nabla 0.1.0 gfx950"; }

const char* atlas_last_error(void) { return g_err.c_str(); }

int atlas_device_count(int* count) {
  if (!count) return fail(ATLAS_EINVAL, "count is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    *count = 0;
    return fail(ATLAS_ENODEV, "no HIP device available");
  }
  *count = n;
  return ATLAS_OK;
}

int atlas_mesh_build(const char* grid, double radius, int device, atlas_mesh_t* out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid) return fail(ATLAS_EINVAL, "grid name is NULL");
  const int N = parse_grid_name(grid);
  if (N < 1) return fail(ATLAS_EINVAL, std::string("not an octahedral grid name: '") + grid + "'");
  if (!(radius > 0.0) || radius > 1e300) return fail(ATLAS_EINVAL, "radius must be positive and finite");
  if (device < -1) return fail(ATLAS_ENODEV, "bad device ordinal");
  int ndev = 0;
  if (device >= 0) {
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
      (void)hipGetLastError();
      return fail(ATLAS_ENODEV, "no HIP device available");
    }
    if (device >= ndev) return fail(ATLAS_ENODEV, "device ordinal out of range");
  }
  atlas_mesh_s* m = nullptr;
  try {
    m = new atlas_mesh_s();
    build_host_mesh(N, radius, m->host);
    if (device >= 0) {
      DeviceGuard g(device);
      if (!g.ok) {
        delete m;
        return fail(ATLAS_EHIP, "cannot select device");
      }
      m->device = device;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, device) == hipSuccess) m->num_cus = prop.multiProcessorCount;
      if (m->num_cus <= 0) m->num_cus = 256;
      upload_tables(*m);
    }
  } catch (const std::bad_alloc&) {
    delete m;
    return fail(ATLAS_ENOMEM, "out of memory building mesh " + std::string(grid));
  } catch (const std::length_error& e) {
    delete m;
    return fail(ATLAS_ESHAPE, e.what());
  } catch (const std::exception& e) {
    delete m;
    return fail(ATLAS_EHIP, e.what());
  }
  *out = m;
  return ATLAS_OK;
}

void atlas_mesh_free(atlas_mesh_t mesh) { delete mesh; }

int atlas_mesh_sizes(atlas_mesh_t mesh, int64_t* nnodes, int64_t* nedges, int64_t* ntris, int64_t* npole_edges,
                     int32_t* max_slots, int32_t* nrows) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  const HostMesh& h = mesh->host;
  if (nnodes) *nnodes = h.V;
  if (nedges) *nedges = h.E;
  if (ntris) *ntris = h.T;
  if (npole_edges) *npole_edges = h.npole;
  if (max_slots) *max_slots = h.max_degree;
  if (nrows) *nrows = h.nrows;
  return ATLAS_OK;
}

int atlas_mesh_export_grid(atlas_mesh_t mesh, int32_t* row_size, int64_t* row_off, double* colat, double* lonlat,
                           double* xyz) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  const HostMesh& h = mesh->host;
  if (row_size) std::memcpy(row_size, h.row_size.data(), h.row_size.size() * sizeof(int32_t));
  if (row_off) std::memcpy(row_off, h.row_off.data(), h.row_off.size() * sizeof(int64_t));
  if (colat) std::memcpy(colat, h.colat.data(), h.colat.size() * sizeof(double));
  if (lonlat)
    for (int64_t i = 0; i < h.V; ++i) {
      lonlat[2 * i] = h.lon[i];
      lonlat[2 * i + 1] = 0.5 * M_PI - h.colat[h.node_row[i]];
    }
  if (xyz) std::memcpy(xyz, h.xyz.data(), h.xyz.size() * sizeof(double));
  return ATLAS_OK;
}

int atlas_mesh_export_connectivity(atlas_mesh_t mesh, int32_t* tris, int32_t* edges, int64_t* csr_off, int32_t* nbr,
                                   int32_t* eid, int8_t* sgn, int8_t* rev, uint8_t* is_pole) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  const HostMesh& h = mesh->host;
  if (tris) std::memcpy(tris, h.tris.data(), h.tris.size() * sizeof(int32_t));
  if (edges) std::memcpy(edges, h.edges.data(), h.edges.size() * sizeof(int32_t));
  if (csr_off) std::memcpy(csr_off, h.csr_off.data(), h.csr_off.size() * sizeof(int64_t));
  if (nbr) std::memcpy(nbr, h.nbr.data(), h.nbr.size() * sizeof(int32_t));
  if (eid) std::memcpy(eid, h.eid.data(), h.eid.size() * sizeof(int32_t));
  if (sgn) std::memcpy(sgn, h.sgn.data(), h.sgn.size() * sizeof(int8_t));
  if (rev) std::memcpy(rev, h.rev.data(), h.rev.size() * sizeof(int8_t));
  if (is_pole) std::memcpy(is_pole, h.is_pole.data(), h.is_pole.size() * sizeof(uint8_t));
  return ATLAS_OK;
}

int atlas_mesh_export_geometry(atlas_mesh_t mesh, double* S, double* V, double* basis, double* C) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  const HostMesh& h = mesh->host;
  if (S) std::memcpy(S, h.S.data(), h.S.size() * sizeof(double));
  if (V) std::memcpy(V, h.vol.data(), h.vol.size() * sizeof(double));
  if (basis) std::memcpy(basis, h.basis.data(), h.basis.size() * sizeof(double));
  if (C) std::memcpy(C, h.C.data(), h.C.size() * sizeof(double));
  return ATLAS_OK;
}

int atlas_nabla_gradient(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* f, void* grad, void* stream) {
  return run_op(mesh, OP_GRAD, dtype, nlev, f, grad, stream);
}

int atlas_nabla_divergence(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* uv, void* div, void* stream) {
  return run_op(mesh, OP_DIV, dtype, nlev, uv, div, stream);
}

int atlas_nabla_gradient_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* w, void* fbar,
                                 void* stream) {
  return run_op(mesh, OP_GRADT, dtype, nlev, w, fbar, stream);
}

int atlas_nabla_divergence_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* d, void* uvbar,
                                   void* stream) {
  return run_op(mesh, OP_DIVT, dtype, nlev, d, uvbar, stream);
}

int atlas_nabla_curl(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* uv, void* zeta, void* stream) {
  return run_op(mesh, OP_CURL, dtype, nlev, uv, zeta, stream);
}

int atlas_nabla_curl_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* z, void* uvbar, void* stream) {
  return run_op(mesh, OP_CURLT, dtype, nlev, z, uvbar, stream);
}

int atlas_nabla_laplacian(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* f, void* lap, void* workspace,
                          void* stream) {
  if (!workspace) return run_op(mesh, OP_LAP, dtype, nlev, f, lap, stream);
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  const size_t n1 = (size_t)mesh->host.V * nlev * es;
  if ((rc = check_field(workspace, 2, es, "workspace"))) return rc;
  if (f && overlaps(workspace, 2 * n1, f, n1)) return fail(ATLAS_EINVAL, "workspace overlaps input");
  if (lap && overlaps(workspace, 2 * n1, lap, n1)) return fail(ATLAS_EINVAL, "workspace overlaps output");
  if (f && lap && overlaps(f, n1, lap, n1)) return fail(ATLAS_EINVAL, "output overlaps input");
  if ((rc = run_op(mesh, OP_GRAD, dtype, nlev, f, workspace, stream))) return rc;
  return run_op(mesh, OP_DIV, dtype, nlev, workspace, lap, stream);
}

int atlas_nabla_gradient_laplacian(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* f, void* grad, void* lap,
                                   void* stream) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  const int64_t V = mesh->host.V;
  if ((int64_t)nlev * V > (int64_t)UINT32_MAX) return fail(ATLAS_ESHAPE, "nnodes * nlev exceeds 2^32 - 1");
  if ((rc = check_field(f, 1, es, "f"))) return rc;
  if ((rc = check_field(grad, 2, es, "grad"))) return rc;
  if ((rc = check_field(lap, 1, es, "lap"))) return rc;
  const size_t n1 = (size_t)V * nlev * es;
  if (overlaps(f, n1, grad, 2 * n1) || overlaps(f, n1, lap, n1) || overlaps(grad, 2 * n1, lap, n1))
    return fail(ATLAS_EINVAL, "f, grad and lap must not overlap");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  // the fused pass runs on the Laplacian's launch shape when that is the
  // one-tile LDS form; otherwise the two operators run one after the other
  const Shape sh = resolve_shape(OP_GRADLAP, dtype, nlev, mesh->shape[OP_LAP][dtype]);
  TileGeom tg;
  if (sh.lds_tiles == 3 && uses_tiles(OP_GRADLAP, dtype, nlev, sh)) tg = tile_geom(OP_GRADLAP, dtype, nlev, sh);
  if (dtype == ATLAS_BF16 && ((uintptr_t)f & 3u)) tg.KL = 0;
  if (tg.KL > 0) {
    DevTiles dt;
    const void* rec = nullptr;
    try {
      dt = mesh->tiles(tg, sh);
      dt.KL = tg.KL;
      dt.nchunks = tg.nchunks;
      rec = mesh->tile_records(tg, sh, dt, OP_GRADLAP, dtype, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
      return fail(ATLAS_ENOMEM, "cannot allocate the LDS tiles");
    } catch (const std::exception& ex) {
      return fail(ATLAS_EHIP, ex.what());
    }
    hipError_t e = launch_tiles(OP_GRADLAP, dtype, dt, rec, nlev, f, lap, sh, mesh->num_cus, (hipStream_t)stream, grad);
    if (e != hipSuccess) return hip_fail(e, "gradient_laplacian");
    return ATLAS_OK;
  }
  if ((rc = run_op(mesh, OP_GRAD, dtype, nlev, f, grad, stream))) return rc;
  return run_op(mesh, OP_LAP, dtype, nlev, f, lap, stream);
}

namespace {

// The divergence and a second divergence-form operator (op2: OP_CURL or
// OP_GRADT) of one vector field: one pass of the dual kernel (fused op
// OP_DIVCURL or OP_DIVGRADT) on the divergence's launch shape when that is
// the one-tile LDS form, else the two operators one after the other.
int divergence_pair(atlas_mesh_t mesh, int fused, int op2, const char* name, int dtype, int32_t nlev,
                    const void* uv, void* div, void* out2, void* stream) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  const int64_t V = mesh->host.V;
  if ((int64_t)nlev * V > (int64_t)UINT32_MAX) return fail(ATLAS_ESHAPE, "nnodes * nlev exceeds 2^32 - 1");
  if ((rc = check_field(uv, 2, es, "uv"))) return rc;
  if ((rc = check_field(div, 1, es, "div"))) return rc;
  if ((rc = check_field(out2, 1, es, op2 == OP_CURL ? "zeta" : "fbar"))) return rc;
  const size_t n1 = (size_t)V * nlev * es;
  if (overlaps(uv, 2 * n1, div, n1) || overlaps(uv, 2 * n1, out2, n1) || overlaps(div, n1, out2, n1))
    return fail(ATLAS_EINVAL, std::string("uv, div and ") + (op2 == OP_CURL ? "zeta" : "fbar") +
                                  " must not overlap");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  const Shape sh = resolve_shape(fused, dtype, nlev, mesh->shape[OP_DIV][dtype]);
  TileGeom tg;
  if (sh.lds_tiles == 3 && uses_tiles(fused, dtype, nlev, sh)) tg = tile_geom(fused, dtype, nlev, sh);
  if (dtype == ATLAS_BF16 && ((uintptr_t)uv & 3u)) tg.KL = 0;
  if (tg.KL > 0) {
    DevTiles dt;
    const void* rec = nullptr;
    try {
      dt = mesh->tiles(tg, sh);
      dt.KL = tg.KL;
      dt.nchunks = tg.nchunks;
      rec = mesh->tile_records(tg, sh, dt, fused, dtype, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
      return fail(ATLAS_ENOMEM, "cannot allocate the LDS tiles");
    } catch (const std::exception& ex) {
      return fail(ATLAS_EHIP, ex.what());
    }
    hipError_t e = launch_tiles(fused, dtype, dt, rec, nlev, uv, div, sh, mesh->num_cus, (hipStream_t)stream, out2);
    if (e != hipSuccess) return hip_fail(e, name);
    return ATLAS_OK;
  }
  if ((rc = run_op(mesh, OP_DIV, dtype, nlev, uv, div, stream))) return rc;
  return run_op(mesh, op2, dtype, nlev, uv, out2, stream);
}

}  // namespace

int atlas_nabla_divergence_curl(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* uv, void* div, void* zeta,
                                void* stream) {
  return divergence_pair(mesh, OP_DIVCURL, OP_CURL, "divergence_curl", dtype, nlev, uv, div, zeta, stream);
}

int atlas_nabla_divergence_gradient_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* uv, void* div,
                                            void* fbar, void* stream) {
  return divergence_pair(mesh, OP_DIVGRADT, OP_GRADT, "divergence_gradient_adjoint", dtype, nlev, uv, div, fbar,
                         stream);
}

int atlas_nabla_conservation(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* div, double* out_sum,
                             double* out_abs, void* stream) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  if ((rc = check_field(div, 1, es, "div"))) return rc;
  if ((rc = check_field(out_sum, 1, 8, "out_sum"))) return rc;
  if ((rc = check_field(out_abs, 1, 8, "out_abs"))) return rc;
  if (overlaps(out_sum, 8 * (size_t)nlev, out_abs, 8 * (size_t)nlev))
    return fail(ATLAS_EINVAL, "out_sum overlaps out_abs");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  const int64_t V = mesh->host.V;
  const size_t need = (size_t)conservation_parts(V, nlev) * nlev * 2 * sizeof(double);
  double* scratch = nullptr;
  {
    std::lock_guard<std::mutex> lk(mesh->scratch_mu);
    if (mesh->scratch_bytes < need) {
      if (mesh->scratch) {
        // a previous call may still be using the smaller buffer
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "conservation");
        (void)hipFree(mesh->scratch);
        mesh->scratch = nullptr;
        mesh->scratch_bytes = 0;
      }
      void* p = nullptr;
      if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ATLAS_ENOMEM, "cannot allocate conservation partials");
      }
      mesh->scratch = static_cast<double*>(p);
      mesh->scratch_bytes = need;
    }
    scratch = mesh->scratch;
  }
  hipError_t e = launch_conservation(dtype, mesh->vol, V, nlev, div, scratch, out_sum, out_abs, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "conservation");
  return ATLAS_OK;
}

int atlas_nabla_conservation_noalloc(atlas_mesh_t mesh, int dtype, int32_t nlev, const void* div, double* out_sum,
                                     double* out_abs, void* stream) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  if ((rc = check_field(div, 1, es, "div"))) return rc;
  if ((rc = check_field(out_sum, 1, 8, "out_sum"))) return rc;
  if ((rc = check_field(out_abs, 1, 8, "out_abs"))) return rc;
  if (overlaps(out_sum, 8 * (size_t)nlev, out_abs, 8 * (size_t)nlev))
    return fail(ATLAS_EINVAL, "out_sum overlaps out_abs");
  const int64_t V = mesh->host.V;
  const size_t need = (size_t)conservation_parts(V, nlev) * (size_t)nlev * 2 * sizeof(double);
  if (need > kScratchBytes)
    return fail(ATLAS_ESHAPE, "nlev " + std::to_string(nlev) + " needs " + std::to_string(need) +
                                  " bytes of partial sums, more than the " + std::to_string(kScratchBytes) +
                                  "-byte static buffer (at most " +
                                  std::to_string(kScratchBytes / ((size_t)conservation_parts(V, 1) * 16)) +
                                  " levels on this mesh)");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  double* part = nullptr;
  hipError_t e = scratch_address(mesh->device, &part);
  if (e != hipSuccess) return hip_fail(e, "conservation_noalloc: scratch address");
  e = launch_conservation(dtype, mesh->vol, V, nlev, div, part, out_sum, out_abs, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "conservation_noalloc");
  return ATLAS_OK;
}

int atlas_nabla_set_tune(atlas_mesh_t mesh, int dtype, uint32_t op, const atlas_tune_t* tune) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  if (!dtype_size(dtype)) return fail(ATLAS_EDTYPE, "unknown dtype");
  const int o = op_from_bit(op);
  if (o < 0) return fail(ATLAS_EINVAL, "op must be one ATLAS_OP_* bit");
  Shape s;
  int rc = check_shape(s, tune);
  if (rc) return rc;
  mesh->shape[o][dtype] = s;
  return ATLAS_OK;
}

struct atlas_remap_s {
  atlas_mesh_t mesh = nullptr;
  RemapHost host;
  int32_t* nodes = nullptr;   // device [P][4]
  void* w64 = nullptr;        // device [P][4] FP64
  void* w32 = nullptr;        // device [P][4] FP32
  int64_t* adj_off = nullptr; // device transpose by source node: [V+1]
  int32_t* adj_t = nullptr;   // [3P]
  void* adj_w64 = nullptr;    // [3P] FP64
  void* adj_w32 = nullptr;    // [3P] FP32
  int32_t* head_t = nullptr;  // [V][2]: each node's first two entries (0 past its count)
  void* head_w64 = nullptr;   // [V][2] FP64
  void* head_w32 = nullptr;   // [V][2] FP32
  ~atlas_remap_s() {
    if (mesh && mesh->device >= 0) {
      DeviceGuard g(mesh->device);
      for (void* p : {(void*)nodes, w64, w32, (void*)adj_off, (void*)adj_t, adj_w64, adj_w32, (void*)head_t, head_w64,
                      head_w32})
        if (p) (void)hipFree(p);
    }
  }
};

namespace {

hipError_t upload_to(const void* data, size_t bytes, void** p) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return e;
  return hipMemcpy(*p, data, bytes, hipMemcpyHostToDevice);
}

}  // namespace

int atlas_remap_build(atlas_mesh_t mesh, const char* target, atlas_remap_t* out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  if (!target) return fail(ATLAS_EINVAL, "target grid name is NULL");
  if (parse_target_name(target, nullptr) < 1)
    return fail(ATLAS_EINVAL, std::string("not a target grid name: '") + target + "'");
  atlas_remap_s* r = nullptr;
  try {
    r = new atlas_remap_s();
    r->mesh = mesh;
    build_remap(mesh->host, target, r->host);
    if (mesh->device >= 0) {
      DeviceGuard g(mesh->device);
      if (!g.ok) {
        delete r;
        return fail(ATLAS_EHIP, "cannot select the mesh's device");
      }
      const std::vector<float> w32 = to_f32(r->host.w);
      hipError_t e = upload_to(r->host.nodes.data(), r->host.nodes.size() * sizeof(int32_t),
                               reinterpret_cast<void**>(&r->nodes));
      if (e == hipSuccess) e = upload_to(r->host.w.data(), r->host.w.size() * sizeof(double), &r->w64);
      if (e == hipSuccess) e = upload_to(w32.data(), w32.size() * sizeof(float), &r->w32);
      const std::vector<float> aw32 = to_f32(r->host.adj_w);
      if (e == hipSuccess)
        e = upload_to(r->host.adj_off.data(), r->host.adj_off.size() * sizeof(int64_t),
                      reinterpret_cast<void**>(&r->adj_off));
      if (e == hipSuccess)
        e = upload_to(r->host.adj_t.data(), r->host.adj_t.size() * sizeof(int32_t), reinterpret_cast<void**>(&r->adj_t));
      if (e == hipSuccess) e = upload_to(r->host.adj_w.data(), r->host.adj_w.size() * sizeof(double), &r->adj_w64);
      if (e == hipSuccess) e = upload_to(aw32.data(), aw32.size() * sizeof(float), &r->adj_w32);
      {
        // the first two entries of each node beside the compressed rows, so
        // the transpose reads them with the row bounds, not after them
        const RemapHost& h = r->host;
        const int64_t V = mesh->host.V;
        std::vector<int32_t> ht(2 * V, 0);
        std::vector<double> hw(2 * V, 0.0);
        for (int64_t n = 0; n < V; ++n)
          for (int64_t q = 0; q < 2 && h.adj_off[n] + q < h.adj_off[n + 1]; ++q) {
            ht[2 * n + q] = h.adj_t[h.adj_off[n] + q];
            hw[2 * n + q] = h.adj_w[h.adj_off[n] + q];
          }
        const std::vector<float> hw32 = to_f32(hw);
        if (e == hipSuccess) e = upload_to(ht.data(), ht.size() * sizeof(int32_t), reinterpret_cast<void**>(&r->head_t));
        if (e == hipSuccess) e = upload_to(hw.data(), hw.size() * sizeof(double), &r->head_w64);
        if (e == hipSuccess) e = upload_to(hw32.data(), hw32.size() * sizeof(float), &r->head_w32);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        delete r;
        return e == hipErrorOutOfMemory ? fail(ATLAS_ENOMEM, "out of device memory for the remap tables")
                                        : hip_fail(e, "remap tables");
      }
    }
  } catch (const std::bad_alloc&) {
    delete r;
    return fail(ATLAS_ENOMEM, "out of memory building the remap");
  } catch (const std::length_error& e) {
    delete r;
    return fail(ATLAS_ESHAPE, e.what());
  } catch (const std::exception& e) {
    delete r;
    return fail(ATLAS_EINVAL, e.what());
  }
  *out = r;
  return ATLAS_OK;
}

void atlas_remap_free(atlas_remap_t remap) { delete remap; }

int atlas_remap_sizes(atlas_remap_t remap, int64_t* npoints, int64_t* nfallback) {
  if (!remap) return fail(ATLAS_EINVAL, "remap is NULL");
  if (npoints) *npoints = remap->host.P;
  if (nfallback) *nfallback = remap->host.fallback;
  return ATLAS_OK;
}

int atlas_remap_export(atlas_remap_t remap, int32_t* nodes, double* weights, double* xyz) {
  if (!remap) return fail(ATLAS_EINVAL, "remap is NULL");
  const RemapHost& h = remap->host;
  for (int64_t t = 0; t < h.P; ++t)
    for (int j = 0; j < 3; ++j) {
      if (nodes) nodes[3 * t + j] = h.nodes[4 * t + j];
      if (weights) weights[3 * t + j] = h.w[4 * t + j];
    }
  if (xyz) std::memcpy(xyz, h.xyz.data(), h.xyz.size() * sizeof(double));
  return ATLAS_OK;
}

int atlas_remap_apply(atlas_remap_t remap, int dtype, int32_t nlev, const void* src, void* dst, void* stream) {
  if (!remap) return fail(ATLAS_EINVAL, "remap is NULL");
  int rc = check_mesh_device(remap->mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  if ((rc = check_field(src, 1, es, "src"))) return rc;
  if ((rc = check_field(dst, 1, es, "dst"))) return rc;
  const size_t nin = (size_t)remap->mesh->host.V * nlev * es, nout = (size_t)remap->host.P * nlev * es;
  if (overlaps(src, nin, dst, nout)) return fail(ATLAS_EINVAL, "dst overlaps src");
  DeviceGuard g(remap->mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  const void* w = dtype == ATLAS_F64 ? remap->w64 : remap->w32;
  hipError_t e = launch_remap(dtype, remap->nodes, w, remap->mesh->host.V, remap->host.P, nlev, src, dst,
                              (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "remap");
  return ATLAS_OK;
}

int atlas_remap_apply_adjoint(atlas_remap_t remap, int dtype, int32_t nlev, const void* ybar, void* fbar,
                              void* stream) {
  if (!remap) return fail(ATLAS_EINVAL, "remap is NULL");
  int rc = check_mesh_device(remap->mesh);
  if (rc) return rc;
  const size_t es = dtype_size(dtype);
  if (!es) return fail(ATLAS_EDTYPE, "unknown dtype " + std::to_string(dtype));
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  if ((rc = check_field(ybar, 1, es, "ybar"))) return rc;
  if ((rc = check_field(fbar, 1, es, "fbar"))) return rc;
  const size_t nin = (size_t)remap->host.P * nlev * es, nout = (size_t)remap->mesh->host.V * nlev * es;
  if (overlaps(ybar, nin, fbar, nout)) return fail(ATLAS_EINVAL, "fbar overlaps ybar");
  DeviceGuard g(remap->mesh->device);
  if (!g.ok) return fail(ATLAS_EHIP, "cannot select the mesh's device");
  const void* w = dtype == ATLAS_F64 ? remap->adj_w64 : remap->adj_w32;
  const void* hw = dtype == ATLAS_F64 ? remap->head_w64 : remap->head_w32;
  hipError_t e = launch_remap_adjoint(dtype, remap->adj_off, remap->adj_t, w, remap->head_t, hw, remap->mesh->host.V,
                                      remap->host.P, nlev, ybar, fbar, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "remap adjoint");
  return ATLAS_OK;
}

int atlas_nabla_describe(atlas_mesh_t mesh, int dtype, uint32_t op, int32_t nlev, atlas_tune_t* resolved, char* kernel,
                         int32_t len) {
  if (!mesh) return fail(ATLAS_EINVAL, "mesh is NULL");
  if (!dtype_size(dtype)) return fail(ATLAS_EDTYPE, "unknown dtype");
  // a one-pass call: its fused operator, on the shape entry it reads
  const int fused = op == ATLAS_OP_GRADIENT_LAPLACIAN ? OP_GRADLAP
                    : op == ATLAS_OP_DIVERGENCE_CURL ? OP_DIVCURL
                    : op == ATLAS_OP_DIVERGENCE_GRADIENT_ADJOINT ? OP_DIVGRADT
                                                                  : -1;
  const int o = fused >= 0 ? (fused == OP_GRADLAP ? OP_LAP : OP_DIV) : op_from_bit(op);
  if (o < 0) return fail(ATLAS_EINVAL, "op must be one ATLAS_OP_* bit or one-pass code");
  if (nlev <= 0) return fail(ATLAS_ESHAPE, "nlev must be >= 1");
  if (kernel && len <= 0) return fail(ATLAS_EINVAL, "len must be positive");
  const int k = fused >= 0 ? fused : o;
  const Shape sh = resolve_shape(k, dtype, nlev, mesh->shape[o][dtype]);
  if (resolved) shape_out(sh, resolved);
  if (kernel) {
    // the one-pass calls run their kernel on the one-tile form only
    if (fused >= 0 && !(sh.lds_tiles == 3 && uses_tiles(k, dtype, nlev, sh) && tile_geom(k, dtype, nlev, sh).KL > 0))
      snprintf(kernel, (size_t)len, "two calls");
    else
      kernel_label(k, dtype, nlev, sh, kernel, len);
  }
  return ATLAS_OK;
}

int atlas_nabla_tune(atlas_mesh_t mesh, int dtype, uint32_t op, int32_t nlev, const void* in, void* out, int32_t reps,
                     void* stream, atlas_tune_t* best, float* best_ms) {
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  const int o = op_from_bit(op);
  if (o < 0) return fail(ATLAS_EINVAL, "op must be one ATLAS_OP_* bit");
  if (reps < 1 || reps > 10000) return fail(ATLAS_EINVAL, "reps must be 1..10000");
  if (!best) return fail(ATLAS_EINVAL, "best is NULL");
  // argument check through a normal call with the current shape
  if ((rc = run_op(mesh, o, dtype, nlev, in, out, stream))) return rc;
  DeviceGuard g(mesh->device);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ATLAS_EHIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ATLAS_EHIP, "hipEventCreate");
  }
  float bestt = 1e30f;
  Shape bs = Shape();
  auto time_shape = [&](const Shape& s) -> int {
    int r = run_op(mesh, o, dtype, nlev, in, out, stream, &s);
    if (r) return r;
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i)
      if ((r = run_op(mesh, o, dtype, nlev, in, out, stream, &s))) return r;
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return fail(ATLAS_EHIP, "hipEventSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (ms < bestt) {
      bestt = ms;
      bs = s;
    }
    return ATLAS_OK;
  };
  // stage 1: the default, then each path -- row-window walk, gather with P
  // lanes per node, LDS tiles -- with its main parameters
  {
    if ((rc = time_shape(Shape()))) goto done;
    for (int u = 1; u <= 3; ++u) {
      Shape s;
      s.lds_tiles = 2;
      if (!uses_window(o, nlev, s)) break;
      s.slices_per_iter = u;
      if ((rc = time_shape(s))) goto done;
    }
    const int ps[] = {16, 32, 64};
    for (int p : ps) {
      if (nlev <= 32 && p != 16) continue;   // short columns always use nlev lanes
      for (int u = 1; u <= 3; ++u) {
        Shape s;
        s.lds_tiles = 2;
        s.row_window = 2;
        s.lanes_per_node = nlev <= 32 ? 0 : p;
        s.slices_per_iter = u;
        if ((rc = time_shape(s))) goto done;
      }
    }
    Shape probe;
    probe.lds_tiles = 3;
    if (uses_tiles(o, dtype, nlev, probe)) {
      const int kbs[] = {32, 48, 64};
      for (int kb : kbs)
        for (int h = 2; h <= 4; ++h) {
          Shape s;
          s.lds_tiles = 3;
          s.tile_kb = kb;
          s.band_rows = h;
          if ((rc = time_shape(s))) goto done;
        }
      const int splits[3][2] = {{6, 2}, {4, 4}, {12, 4}};   // computing, copying waves
      for (int kb = 48; kb <= 64; kb += 16)
        for (int h = 3; h <= 5; ++h)
          for (const auto& sp : splits) {
            if (dtype == ATLAS_F64 && sp[0] + sp[1] > 8) continue;
            Shape s;
            s.lds_tiles = 1;
            s.tile_kb = kb;
            s.band_rows = h;
            s.tile_waves = sp[0];
            s.producer_waves = sp[1];
            if ((rc = time_shape(s))) goto done;
          }
    }
  }
  if (bs.lds_tiles == 1 || bs.lds_tiles == 3 || (bs.lds_tiles == 0 && uses_tiles(o, dtype, nlev,
                                                                                 resolve_shape(o, dtype, nlev, bs)))) {
    // LDS tiles won: bands swept together
    const Shape base = resolve_shape(o, dtype, nlev, bs);
    const int sweeps[] = {4, 8, 16};
    for (int b : sweeps) {
      Shape s = base;
      s.run_nodes = b;
      if ((rc = time_shape(s))) goto done;
    }
    shape_out(bs, best);
    if (best_ms) *best_ms = bestt;
    goto done;
  }
  // stage 2: workgroup shape and XCD remapping around the best mapping
  {
    const Shape base = bs;
    const int wpbs[] = {1, 2, 4};
    const int npws[] = {1, 2, 4, 8};
    for (int w : wpbs)
      for (int n : npws)
        for (int x = 0; x < 2; ++x) {
          Shape s = base;
          s.waves_per_block = w;
          s.nodes_per_wave = n;
          s.xcd_remap = x;
          if ((rc = time_shape(s))) goto done;
        }
  }
  // stage 3: node order (band height, run length) and store kind
  {
    const Shape base = bs;
    const int hs[] = {8, 16, 32, 64};
    const int rs[] = {4, 16, 64};
    for (int h : hs)
      for (int r : rs)
        for (int nt = 1; nt <= 2; ++nt) {
          Shape s = base;
          s.band_rows = h;
          s.run_nodes = r;
          s.nt_stores = nt;
          if ((rc = time_shape(s))) goto done;
        }
  }
  shape_out(bs, best);
  if (best_ms) *best_ms = bestt;
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"

// ---- batched plans ------------------------------------------------------------

// Persistent tiled launch of one operator of a plan.
struct BatchOp {
  bool tiled = false;       // else the tracers' single-field launches
  BatchTile* tr = nullptr;  // device [ntracers]
  int32_t* pre = nullptr;   // device [8][ntracers + 1]
  int32_t* ctr = nullptr;   // device [kBatchCounterInts] work counters (zero between launches)
  uint32_t lds = 0;
  int waves = 0;
  int umax = 1;             // largest slice count of the tracers
  int32_t claim = kDefaultBatchClaim;   // tiles per work claim
  int64_t grid = 0;
};

struct atlas_batch_s {
  atlas_mesh_t mesh = nullptr;
  int dtype = 0;
  uint32_t mask = 0;
  Shape shape[4];           // launch shape of each operator
  std::vector<atlas_tracer_desc_t> descs;
  BatchOp ops[4];
  BatchOp pair;             // divergence and gradient adjoint in one launch (see plan_pairs)
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  void release_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  void release_tables() {
    auto release = [](BatchOp& bo) {
      if (bo.tr) (void)hipFree(bo.tr);
      if (bo.pre) (void)hipFree(bo.pre);
      if (bo.ctr) (void)hipFree(bo.ctr);
      bo = BatchOp();
    };
    for (BatchOp& bo : ops) release(bo);
    release(pair);
  }
  ~atlas_batch_s() {
    if (!mesh) return;
    DeviceGuard g(mesh->device);
    release_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    release_tables();
  }
};

namespace {

// Persistent form (batch_mode 0 or 1) unless field launches are asked for.
bool plan_persistent(const Shape& sh) { return sh.batch_mode != 2; }

// Level count whose tiling a tracer of L levels uses: L rounded up to a
// power of two, at most the plan's largest L.  Tracers of similar depth share
// a tiling; each tiling packs about as many columns as its single-field
// launch would, so short columns still fill the tile's waves.
int bucket_levels(int L, int Lmax) {
  int p = 1;
  while (p < L) p <<= 1;
  return std::min(p, Lmax);
}

// Sets up the persistent tiled launch of operator o: for each level bucket
// the tiling and node records of the single-field one-tile form, each
// tracer's chunk (at most its tiling's) and slices, the per-XCD item counts,
// the LDS size (largest tile plus read-past tail over the tracers) and the
// grid (as many workgroups as the CUs hold at once).  Leaves bo.tiled false
// when some tracer's tiles do not fit.  pair: the divergence (o = OP_DIV)
// with the gradient adjoint of the same fields in one pass (OP_DIVGRADT), on
// the divergence's shape.
int plan_op(atlas_batch_s* b, int o, BatchOp& bo, bool pair = false) {
  const int k = pair ? OP_DIVGRADT : o;   // the launch's operator
  int Lmax = 1;
  for (const atlas_tracer_desc_t& d : b->descs) Lmax = std::max(Lmax, d.nlev);
  // tile defaults of the long-column launch, also for batches of short columns
  const Shape sh = resolve_shape(k, b->dtype, std::max(Lmax, 33), b->shape[o]);
  if (sh.lds_tiles != 3) return ATLAS_OK;
  const int ntr = (int)b->descs.size();
  std::map<int, std::pair<DevTiles, const void*>> tilings;
  std::vector<BatchTile> tr(ntr);
  std::vector<int32_t> pre(8 * (size_t)(ntr + 1), 0);
  int64_t lds = 0;
  for (int t = 0; t < ntr; ++t) {
    BatchTile& d = tr[t];
    d.L = b->descs[t].nlev;
    const int Lb = bucket_levels(d.L, Lmax);
    auto it = tilings.find(Lb);
    if (it == tilings.end()) {
      const TileGeom tg = tile_geom(k, b->dtype, Lb, sh);
      if (tg.KL < 1) return ATLAS_OK;
      try {
        DevTiles dt = b->mesh->tiles(tg, sh);
        dt.KL = tg.KL;
        dt.nchunks = tg.nchunks;
        const void* rec = b->mesh->tile_records(tg, sh, dt, k, b->dtype, nullptr);
        it = tilings.emplace(Lb, std::make_pair(dt, rec)).first;
      } catch (const std::bad_alloc&) {
        return fail(ATLAS_ENOMEM, "cannot allocate the LDS tiles");
      } catch (const std::exception& ex) {
        return fail(ATLAS_EHIP, ex.what());
      }
    }
    const DevTiles& dt = it->second.first;
    d.in = b->descs[t].in[o];
    d.out = b->descs[t].out[o];
    d.out2 = pair ? b->descs[t].out[OP_GRADT] : nullptr;
    d.info = dt.info;
    d.segs = dt.segs;
    d.rec = static_cast<const char*>(it->second.second);
    d.KL = std::min(dt.KL, d.L);
    d.nchunks = (d.L + d.KL - 1) / d.KL;
    d.U = tile_slices(d.KL, sh);
    bo.umax = std::max(bo.umax, d.U);
    d.nitems = dt.ntiles * d.nchunks;
    lds = std::max(lds, (int64_t)dt.lds_bytes + tile_tail_bytes(k, b->dtype, d.KL, d.L, d.U));
    for (int x = 0; x < 8; ++x) {
      const int64_t share = (x + 1) * d.nitems / 8 - x * d.nitems / 8;
      const int64_t next = (int64_t)pre[x * (ntr + 1) + t] + share;
      if (next > INT32_MAX) return fail(ATLAS_ESHAPE, "too many batched work items");
      pre[x * (ntr + 1) + t + 1] = (int32_t)next;
    }
  }
  bo.waves = sh.waves_per_block;
  bo.claim = sh.batch_claim > 0 ? sh.batch_claim : kDefaultBatchClaim;
  const int n = lds <= (int64_t)160 * 1024 ? tiles_batched_per_cu(k, b->dtype, (uint32_t)lds, bo.waves, bo.umax) : 0;
  if (n < 1) return ATLAS_OK;   // does not launch with this shape: field launches
  const int per_cu = sh.tile_wgs_per_cu > 0 ? std::min(sh.tile_wgs_per_cu, n) : n;
  bo.grid = std::max<int64_t>(8, (int64_t)per_cu * b->mesh->num_cus / 8 * 8);
  bo.lds = (uint32_t)lds;
  void* p = nullptr;
  if (hipMalloc(&p, tr.size() * sizeof(BatchTile)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ATLAS_ENOMEM, "cannot allocate batch table");
  }
  bo.tr = static_cast<BatchTile*>(p);
  if (hipMalloc(&p, pre.size() * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ATLAS_ENOMEM, "cannot allocate batch table");
  }
  bo.pre = static_cast<int32_t*>(p);
  if (hipMalloc(&p, kBatchCounterInts * sizeof(int32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ATLAS_ENOMEM, "cannot allocate batch counters");
  }
  bo.ctr = static_cast<int32_t*>(p);
  hipError_t e = hipMemcpy(bo.tr, tr.data(), tr.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(bo.pre, pre.data(), pre.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  // zero once here, outside any capture; every launch leaves them zero
  if (e == hipSuccess) e = hipMemset(bo.ctr, 0, kBatchCounterInts * sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(e, "batch table upload");
  bo.tiled = true;
  return ATLAS_OK;
}

// Whether the plan's divergence and gradient adjoint can run as one pass:
// both asked for, on the same input field in every tracer, and no output of
// either overlapping an input of any tracer (run one after the other, the
// divergence of every tracer precedes every gradient adjoint; in one pass
// they interleave).
bool plan_pairs(const atlas_batch_s* b) {
  if ((b->mask & ((1u << OP_DIV) | (1u << OP_GRADT))) != ((1u << OP_DIV) | (1u << OP_GRADT))) return false;
  const size_t es = dtype_size(b->dtype);
  const int64_t V = b->mesh->host.V;
  for (const atlas_tracer_desc_t& d : b->descs)
    if (d.in[OP_DIV] != d.in[OP_GRADT]) return false;
  for (const atlas_tracer_desc_t& d : b->descs)
    for (const atlas_tracer_desc_t& e : b->descs) {
      const size_t nd = (size_t)V * d.nlev * es, ne = (size_t)V * e.nlev * es;
      if (overlaps(d.out[OP_DIV], nd, e.in[OP_DIV], 2 * ne) || overlaps(d.out[OP_GRADT], nd, e.in[OP_DIV], 2 * ne))
        return false;
    }
  return true;
}

// (Re)build the device work tables of a plan for its operators' shapes.
int plan_upload(atlas_batch_s* b) {
  b->release_tables();
  for (int o = 0; o < 4; ++o) {
    if (!(b->mask & (1u << o)) || !plan_persistent(b->shape[o])) continue;
    int rc = plan_op(b, o, b->ops[o]);
    if (rc) return rc;
  }
  // the divergence and the gradient adjoint of the same fields in one
  // persistent launch, on the divergence's shape, where it fits
  if (plan_persistent(b->shape[OP_DIV]) && plan_pairs(b)) {
    int rc = plan_op(b, OP_DIV, b->pair, true);
    if (rc) return rc;
  }
  return ATLAS_OK;
}

// One operator over every tracer: one persistent launch, or the tracers'
// single-field launches in order.
int plan_run_op(atlas_batch_s* b, int o, hipStream_t st) {
  const BatchOp& bo = b->ops[o];
  if (bo.tiled) {
    hipError_t e = launch_tiles_batched(o, b->dtype, bo.tr, bo.pre, (int)b->descs.size(), bo.ctr, bo.claim, bo.lds,
                                        bo.waves, bo.grid, bo.umax, st);
    return e != hipSuccess ? hip_fail(e, kOpName[o]) : ATLAS_OK;
  }
  for (const atlas_tracer_desc_t& d : b->descs) {
    int rc = run_op(b->mesh, o, b->dtype, d.nlev, d.in[o], d.out[o], st);
    if (rc) return rc;
  }
  return ATLAS_OK;
}

// Operators outermost, in the order of their bits; the divergence and
// gradient adjoint pair, where planned, in the divergence's place.
int plan_run(atlas_batch_s* b, hipStream_t st) {
  for (int o = 0; o < 4; ++o) {
    if (!(b->mask & (1u << o))) continue;
    if (b->pair.tiled && (o == OP_DIV || o == OP_GRADT)) {
      if (o == OP_GRADT) continue;
      const BatchOp& bo = b->pair;
      hipError_t e = launch_tiles_batched(OP_DIVGRADT, b->dtype, bo.tr, bo.pre, (int)b->descs.size(), bo.ctr, bo.claim,
                                          bo.lds, bo.waves, bo.grid, bo.umax, st);
      if (e != hipSuccess) return hip_fail(e, "divergence_gradient_adjoint");
      continue;
    }
    int rc = plan_run_op(b, o, st);
    if (rc) return rc;
  }
  return ATLAS_OK;
}

// Whether every operator of the plan runs as one persistent launch.
bool plan_all_tiled(const atlas_batch_s* b) {
  for (int o = 0; o < 4; ++o)
    if ((b->mask & (1u << o)) && !b->ops[o].tiled && !(b->pair.tiled && (o == OP_DIV || o == OP_GRADT)))
      return false;
  return true;
}

}  // namespace

extern "C" {

int atlas_batch_create(atlas_mesh_t mesh, int dtype, const atlas_tracer_desc_t* descs, int32_t ntracers,
                       uint32_t op_mask, const atlas_tune_t* tune, atlas_batch_t* out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_mesh_device(mesh);
  if (rc) return rc;
  if (dtype != ATLAS_F32 && dtype != ATLAS_F64) return fail(ATLAS_EDTYPE, "batched plans take ATLAS_F32 or ATLAS_F64");
  if (!descs || ntracers < 1) return fail(ATLAS_EINVAL, "need at least one tracer descriptor");
  if (op_mask == 0 || (op_mask & ~0xFu)) return fail(ATLAS_EINVAL, "op_mask must be a non-empty OR of the four operator bits");
  const size_t es = dtype_size(dtype);
  for (int32_t t = 0; t < ntracers; ++t) {
    const atlas_tracer_desc_t& d = descs[t];
    if (d.nlev < 1 || d.reserved != 0)
      return fail(ATLAS_ESHAPE, "tracer " + std::to_string(t) + ": nlev must be >= 1 and reserved 0");
    if ((int64_t)d.nlev * mesh->host.V > (int64_t)UINT32_MAX)
      return fail(ATLAS_ESHAPE, "tracer " + std::to_string(t) + ": nnodes * nlev exceeds 2^32 - 1");
    for (int o = 0; o < 4; ++o) {
      if (!(op_mask & (1u << o))) continue;
      const std::string nm = "tracer " + std::to_string(t) + " " + kOpName[o];
      if ((rc = check_field(d.in[o], kInComps[o], es, (nm + " input").c_str()))) return rc;
      if ((rc = check_field(d.out[o], kOutComps[o], es, (nm + " output").c_str()))) return rc;
      const size_t n = (size_t)mesh->host.V * d.nlev * es;
      if (overlaps(d.in[o], n * kInComps[o], d.out[o], n * kOutComps[o]))
        return fail(ATLAS_EINVAL, nm + ": output overlaps input");
    }
  }
  atlas_batch_s* b = nullptr;
  try {
    b = new atlas_batch_s();
  } catch (const std::bad_alloc&) {
    return fail(ATLAS_ENOMEM, "out of memory");
  }
  b->mesh = mesh;
  b->dtype = dtype;
  b->mask = op_mask;
  if ((rc = check_shape(b->shape[0], tune))) {
    delete b;
    return rc;
  }
  for (int o = 1; o < 4; ++o) b->shape[o] = b->shape[0];
  b->descs.assign(descs, descs + ntracers);
  DeviceGuard g(mesh->device);
  if ((rc = plan_upload(b))) {
    delete b;
    return rc;
  }
  *out = b;
  return ATLAS_OK;
}

int atlas_batch_run(atlas_batch_t plan, void* stream) {
  if (!plan) return fail(ATLAS_EINVAL, "plan is NULL");
  DeviceGuard g(plan->mesh->device);
  return plan_run(plan, (hipStream_t)stream);
}

int atlas_batch_graph_launch(atlas_batch_t plan, void* stream) {
  if (!plan) return fail(ATLAS_EINVAL, "plan is NULL");
  DeviceGuard g(plan->mesh->device);
  if (!plan->exec) {
    hipError_t e;
    if (!plan->capture_stream) {
      e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    if (!plan_all_tiled(plan)) {
      // one eager pass, in order on the caller's stream, builds every node
      // order, tiling and record table the field launches need (host work
      // and allocation cannot be captured)
      int rc0 = plan_run(plan, (hipStream_t)stream);
      if (rc0) return rc0;
      e = hipStreamSynchronize((hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = plan_run(plan, plan->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(plan->capture_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    plan->graph = graph;
    e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      plan->release_graph();
      return hip_fail(e, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ATLAS_OK;
}

void atlas_batch_free(atlas_batch_t plan) { delete plan; }

int atlas_batch_tune(atlas_batch_t plan, int32_t reps, void* stream, atlas_tune_t* best, float* best_ms) {
  if (!plan) return fail(ATLAS_EINVAL, "plan is NULL");
  if (reps < 1 || reps > 10000) return fail(ATLAS_EINVAL, "reps must be 1..10000");
  if (!best) return fail(ATLAS_EINVAL, "best is NULL");
  DeviceGuard g(plan->mesh->device);
  hipStream_t st = (hipStream_t)stream;
  plan->release_graph();
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ATLAS_EHIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ATLAS_EHIP, "hipEventCreate");
  }
  Shape orig[4], bs[4];
  float bestt[4];
  for (int o = 0; o < 4; ++o) {
    orig[o] = bs[o] = plan->shape[o];
    bestt[o] = 1e30f;
  }
  int rc = ATLAS_OK;
  // the field form first (its launches use the mesh's shapes), then the
  // persistent tiled form over the tile's LDS budget (0: each operator's
  // default), tiles per work claim and waves per workgroup; each operator's
  // launch is timed on its own and keeps its fastest shape
  const int kbs[] = {0, 64, 80};
  const int claims[] = {4, 8};
  const int wpbs[] = {8, 16};
  for (int k = -1; k < 3 * 2 * 2; ++k) {
    Shape s;
    if (k < 0) {
      s.batch_mode = 2;
    } else {
      s.batch_mode = 1;
      s.tile_kb = kbs[k / 4];
      s.batch_claim = claims[(k / 2) % 2];
      s.waves_per_block = wpbs[k % 2];
    }
    for (int o = 0; o < 4; ++o) plan->shape[o] = s;
    if (hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(ATLAS_EHIP, "hipStreamSynchronize");
      goto done;
    }
    if ((rc = plan_upload(plan))) goto done;
    for (int o = 0; o < 4; ++o) {
      if (!(plan->mask & (1u << o))) continue;
      if ((rc = plan_run_op(plan, o, st))) goto done;
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r)
        if ((rc = plan_run_op(plan, o, st))) goto done;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(ATLAS_EHIP, "hipEventSynchronize");
        goto done;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)reps;
      if (ms < bestt[o]) {
        bestt[o] = ms;
        bs[o] = s;
      }
    }
  }
  {
    float total = 0.f;
    for (int o = 0; o < 4; ++o) {
      if (!(plan->mask & (1u << o))) continue;
      shape_out(bs[o], best + o);
      total += bestt[o];
    }
    if (best_ms) *best_ms = total;
  }
done:
  // leave the plan with each operator's best shape (or the original ones on
  // error)
  for (int o = 0; o < 4; ++o) plan->shape[o] = rc ? orig[o] : bs[o];
  (void)hipStreamSynchronize(st);
  int rc2 = plan_upload(plan);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc ? rc : rc2;
}

}  // extern "C"
