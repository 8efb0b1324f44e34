// Host-side interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace atlasnabla {

enum Op : int { OP_GRAD = 0, OP_DIV = 1, OP_GRADT = 2, OP_DIVT = 3, OP_LAP = 4, OP_COUNT = 5 };
enum Dtype : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Device tables of one mesh for one coefficient precision (FP64 for DT_F64,
// FP32 for DT_F32 and DT_BF16).
struct DevTables {
  const int32_t* nbr8 = nullptr;        // [V][8]
  const void* coef[4] = {};             // grad, div, gradT, divT: [V][8] pairs
  const int32_t* lap_nbr = nullptr;     // [V][lap_stride]
  const void* lap_w = nullptr;          // [V][lap_stride]
  int lap_stride = 0;
};

struct Shape {
  int waves_per_block = 4;   // 64-lane waves per workgroup
  int nodes_per_wave = 2;    // nodes (or node groups) per wave per workgroup
  int blocks_per_cu = 4;     // persistent kernels only
  int xcd_remap = 1;         // contiguous slices of work per XCD
};

// Number of nodes handled together by one wave: 0 means one node per wave with
// its levels spread over the lanes (nlev > 32), otherwise floor(64 / nlev)
// nodes share a wave, one (node, level) per lane.
inline int pack_factor(int nlev) { return nlev > 32 ? 0 : 64 / nlev; }

// Single-field operator launch; in/out are device pointers of the dtype.
hipError_t launch_op(int op, int dtype, const DevTables& t, int64_t V, int nlev,
                     const void* in, void* out, const Shape& shape, hipStream_t stream);

// Conservation sums: partial [nparts][nlev][2] doubles of scratch, then the
// final fixed-order pass into out_sum/out_abs.
int conservation_parts(int64_t V, int nlev);
hipError_t launch_conservation(int dtype, const double* vol, int64_t V, int nlev,
                               const void* div, double* scratch, double* out_sum,
                               double* out_abs, hipStream_t stream);

// Batched persistent launch over a device table of work items.
struct BatchItem {
  const void* in;
  void* out;
  int32_t nlev;
  int32_t pack;          // pack_factor(nlev)
  int64_t tile_begin;    // first global tile of this tracer
};
int64_t tiles_for(int64_t V, int nlev, const Shape& shape);
hipError_t launch_batched(int op, int dtype, const DevTables& t, int64_t V,
                          const BatchItem* items, int nitems, int64_t total_tiles,
                          const Shape& shape, int num_cus, hipStream_t stream);

}  // namespace atlasnabla
