// gfx950 kernels of the median-dual Nabla operators.
//
// Every operator is a gather over a node's incident edges (the edge sums of
// the finite-volume operators listed in Section 2.3 of the report, evaluated
// node by node): the output element (node i, level k) is written by exactly
// one lane, neighbour values are read in a fixed slot order, and nothing is
// accumulated across lanes, so there are no atomics and reruns are bitwise
// identical.  The path is a sparse stencil whose dense dimension is the
// level column, so it is bound by HBM traffic and uses no matrix cores.
//
// Mapping.  Fields are [node][level] with levels innermost.  For columns of
// more than 32 levels one 64-lane wave owns one node and sweeps its column in
// slices of 64 consecutive levels: the node's table row (neighbour indices
// and coefficient pairs) is wave-uniform, so it is fetched once through the
// scalar cache and held in scalar registers, and each neighbour read is one
// contiguous 64-element vector load.  Short columns (<= 32 levels) pack
// floor(64 / nlev) nodes into one wave, one (node, level) per lane.
//
// XCD awareness.  Workgroups are dispatched round-robin over the eight XCDs;
// with remapping on, workgroup b works on logical block
// (b mod 8) * ceil(nblocks / 8) + b / 8, so each XCD walks a contiguous band
// of latitude rows and the rows above and below a band stay in its own L2.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace atlasnabla {

namespace {

using bf16_t = uint16_t;

constexpr int kLapMax = 24;   // two-ring table stride the kernels are built for

template <class S> struct Traits;
template <> struct Traits<double> { using C = double; using C2 = double2; };
template <> struct Traits<float> { using C = float; using C2 = float2; };
template <> struct Traits<bf16_t> { using C = float; using C2 = float2; };

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// round to nearest even; NaN stays a (quiet) NaN
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ double ld1(const double* p) { return *p; }
__device__ __forceinline__ float ld1(const float* p) { return *p; }
__device__ __forceinline__ float ld1(const bf16_t* p) { return bf16_to_f32(*p); }

__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ float2 ld2(const float* p) { return *reinterpret_cast<const float2*>(p); }
__device__ __forceinline__ float2 ld2(const bf16_t* p) {
  const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
  return make_float2(bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16));
}

__device__ __forceinline__ void st1(double* p, double v) { *p = v; }
__device__ __forceinline__ void st1(float* p, float v) { *p = v; }
__device__ __forceinline__ void st1(bf16_t* p, float v) { *p = (bf16_t)f32_to_bf16(v); }

__device__ __forceinline__ void st2(double* p, double x, double y) {
  *reinterpret_cast<double2*>(p) = make_double2(x, y);
}
__device__ __forceinline__ void st2(float* p, float x, float y) {
  *reinterpret_cast<float2*>(p) = make_float2(x, y);
}
__device__ __forceinline__ void st2(bf16_t* p, float x, float y) {
  *reinterpret_cast<uint32_t*>(p) = f32_to_bf16(x) | (f32_to_bf16(y) << 16);
}

// Read-only table data read through the constant address space: with a
// wave-uniform address the compiler fetches it with scalar loads into scalar
// registers.  Valid because no kernel writes the tables.
template <class T>
__device__ __forceinline__ T ld_const(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}
__device__ __forceinline__ int32_t ld_uniform(const int32_t* p) { return ld_const(p); }
__device__ __forceinline__ float ld_uniform(const float* p) { return ld_const(p); }
__device__ __forceinline__ double ld_uniform(const double* p) { return ld_const(p); }
__device__ __forceinline__ float2 ld_uniform(const float2* p) {
  const float* q = reinterpret_cast<const float*>(p);
  return make_float2(ld_const(q), ld_const(q + 1));
}
__device__ __forceinline__ double2 ld_uniform(const double2* p) {
  const double* q = reinterpret_cast<const double*>(p);
  return make_double2(ld_const(q), ld_const(q + 1));
}

struct Args {
  const int32_t* nbr;   // nbr8 or the two-ring neighbour table
  const void* coef;     // coefficient pairs or two-ring weights
  int stride;           // entries per node row of nbr/coef
  const void* in;
  void* out;
  int64_t V;
  int32_t L;            // levels
  int32_t pack;         // 0: one node per wave, else nodes per wave
  int32_t npw;          // nodes (or node groups) per wave per block
};

// ---- per-element arithmetic (shared by every launch form) -------------------
//
// NS is the number of table entries a node uses (its degree, or its two-ring
// size for the Laplacian), fixed at compile time so that all neighbour loads
// of an element are issued back to back before any arithmetic waits on them.
// Entries are consumed in slot order, which fixes the summation order.

// gradient, difference form: sum_s (a, b)_s (f_n - f_i)
template <class S, int NS>
__device__ __forceinline__ void elem_grad(const S* __restrict__ in, S* __restrict__ out, int64_t L,
                                          int64_t node, int k, const int32_t* nb,
                                          const typename Traits<S>::C2* cf) {
  using C = typename Traits<S>::C;
  C v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = ld1(in + (int64_t)nb[s] * L + k);
  const C fi = ld1(in + node * L + k);
  C ax = 0, ay = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const C d = v[s] - fi;
    ax = fma(cf[s].x, d, ax);
    ay = fma(cf[s].y, d, ay);
  }
  st2(out + 2 * (node * L + k), ax, ay);
}

// divergence adjoint: (A, B)_i d_i + sum_s (c, d)_{n,rev} d_n
template <class S, int NS>
__device__ __forceinline__ void elem_divT(const S* __restrict__ in, S* __restrict__ out, int64_t L,
                                          int64_t node, int k, const int32_t* nb,
                                          const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg) {
  using C = typename Traits<S>::C;
  C v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = ld1(in + (int64_t)nb[s] * L + k);
  const C di = ld1(in + node * L + k);
  C ax = dg.x * di, ay = dg.y * di;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    ax = fma(cf[s].x, v[s], ax);
    ay = fma(cf[s].y, v[s], ay);
  }
  st2(out + 2 * (node * L + k), ax, ay);
}

// divergence and gradient adjoint: (x, y)_diag . in_i + sum_s (x, y)_s . in_n
template <class S, int NS>
__device__ __forceinline__ void elem_v2s(const S* __restrict__ in, S* __restrict__ out, int64_t L,
                                         int64_t node, int k, const int32_t* nb,
                                         const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg) {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  C2 v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = ld2(in + 2 * ((int64_t)nb[s] * L + k));
  const C2 ui = ld2(in + 2 * (node * L + k));
  C acc = dg.x * ui.x;
  acc = fma(dg.y, ui.y, acc);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    acc = fma(cf[s].x, v[s].x, acc);
    acc = fma(cf[s].y, v[s].y, acc);
  }
  st1(out + node * L + k, acc);
}

// fused Laplacian over the two-ring: sum_m W_im (f_m - f_i)
template <class S, int NS>
__device__ __forceinline__ void elem_lap(const S* __restrict__ in, S* __restrict__ out, int64_t L,
                                         int64_t node, int k, const int32_t* nb,
                                         const typename Traits<S>::C* w) {
  using C = typename Traits<S>::C;
  C v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = ld1(in + (int64_t)nb[s] * L + k);
  const C fi = ld1(in + node * L + k);
  C acc = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) acc = fma(w[s], v[s] - fi, acc);
  st1(out + node * L + k, acc);
}

template <class S, int OP, int NS>
__device__ __forceinline__ void elem_1ring(const Args& a, int64_t node, int k, const int32_t* nb,
                                           const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg) {
  const S* in = static_cast<const S*>(a.in);
  S* out = static_cast<S*>(a.out);
  if constexpr (OP == OP_GRAD) elem_grad<S, NS>(in, out, a.L, node, k, nb, cf);
  else if constexpr (OP == OP_DIVT) elem_divT<S, NS>(in, out, a.L, node, k, nb, cf, dg);
  else elem_v2s<S, NS>(in, out, a.L, node, k, nb, cf, dg);
}

// ---- one node per wave (columns of more than 32 levels) ---------------------
//
// The node's table row is wave-uniform: it is read once, kept in registers,
// and reused for every 64-level slice of the column.

template <class S, int OP, int NS>
__device__ __forceinline__ void slab_1ring(const Args& a, int64_t node, int lane) {
  using C2 = typename Traits<S>::C2;
  const int32_t* nbp = a.nbr + node * 8;
  const C2* cfp = static_cast<const C2*>(a.coef) + node * 8;
  int nb[NS];
  C2 cf[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    nb[s] = ld_uniform(nbp + s);
    cf[s] = ld_uniform(cfp + s);
  }
  const C2 dg = ld_uniform(cfp + 7);
  for (int k0 = 0; k0 < a.L; k0 += 64) {
    const int k = k0 + lane;
    if (k < a.L) elem_1ring<S, OP, NS>(a, node, k, nb, cf, dg);
  }
}

template <class S, int NS>
__device__ __forceinline__ void slab_lap(const Args& a, int64_t node, int lane) {
  using C = typename Traits<S>::C;
  const int32_t* nbp = a.nbr + node * a.stride;
  const C* wp = static_cast<const C*>(a.coef) + node * a.stride;
  int nb[NS];
  C w[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    nb[s] = ld_uniform(nbp + s);
    w[s] = ld_uniform(wp + s);
  }
  for (int k0 = 0; k0 < a.L; k0 += 64) {
    const int k = k0 + lane;
    if (k < a.L) elem_lap<S, NS>(static_cast<const S*>(a.in), static_cast<S*>(a.out), a.L, node, k, nb, w);
  }
}

template <class S, int OP>
__device__ __forceinline__ void slab_node(const Args& a, int64_t node, int lane) {
  if constexpr (OP == OP_LAP) {
    // two-ring sizes on O-grids are 14..22; entries past the count are padding
    // (the node itself, weight 0), so a larger instance stays exact
    const int cnt = ld_uniform(a.nbr + node * a.stride + a.stride - 1);
    if (cnt == 18) slab_lap<S, 18>(a, node, lane);
    else if (cnt <= 16) slab_lap<S, 16>(a, node, lane);
    else if (cnt == 17) slab_lap<S, 17>(a, node, lane);
    else if (cnt <= 20) slab_lap<S, 20>(a, node, lane);
    else slab_lap<S, kLapMax - 1>(a, node, lane);
  } else {
    const int deg = ld_uniform(a.nbr + node * 8 + 7);
    if (deg == 6) slab_1ring<S, OP, 6>(a, node, lane);
    else if (deg == 5) slab_1ring<S, OP, 5>(a, node, lane);
    else slab_1ring<S, OP, 7>(a, node, lane);   // degree 7, or padding for degrees < 5
  }
}

// ---- several nodes per wave (columns of at most 32 levels) ------------------
//
// Lanes belong to different nodes, so every lane reads its own table row and
// uses the full padded width (padding adds exact zeros).

template <class S, int OP>
__device__ __forceinline__ void packed_elem(const Args& a, int64_t node, int k) {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  if constexpr (OP == OP_LAP) {
    const int32_t* nbp = a.nbr + node * a.stride;
    const C* wp = static_cast<const C*>(a.coef) + node * a.stride;
    int nb[kLapMax - 1];
    C w[kLapMax - 1];
#pragma unroll
    for (int s = 0; s < kLapMax - 1; ++s) {
      nb[s] = nbp[s];
      w[s] = wp[s];
    }
    elem_lap<S, kLapMax - 1>(static_cast<const S*>(a.in), static_cast<S*>(a.out), a.L, node, k, nb, w);
  } else {
    const int32_t* nbp = a.nbr + node * 8;
    const C2* cfp = static_cast<const C2*>(a.coef) + node * 8;
    int nb[7];
    C2 cf[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      nb[s] = nbp[s];
      cf[s] = cfp[s];
    }
    elem_1ring<S, OP, 7>(a, node, k, nb, cf, cfp[7]);
  }
}

// Work of logical block `lb`: waves_per_block * npw nodes (or node groups).
template <class S, int OP>
__device__ __forceinline__ void process_block(const Args& a, int64_t lb) {
  const int wpb = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a.pack == 0) {
    const int64_t base = lb * (int64_t)wpb * a.npw;
    for (int r = 0; r < a.npw; ++r) {
      const int64_t node = base + (int64_t)r * wpb + wave;
      if (node >= a.V) break;
      slab_node<S, OP>(a, node, lane);
    }
  } else {
    const int sub = lane / a.L;
    const int k = lane - sub * a.L;
    for (int r = 0; r < a.npw; ++r) {
      const int64_t group = (lb * a.npw + r) * wpb + wave;
      const int64_t node = group * a.pack + sub;
      if (sub < a.pack && node < a.V) packed_elem<S, OP>(a, node, k);
    }
  }
}

__device__ __forceinline__ int64_t logical_block(int64_t b, int64_t nblocks, int remap) {
  if (!remap) return b;
  const int64_t per = (nblocks + 7) / 8;
  return (b & 7) * per + (b >> 3);
}

template <class S, int OP>
__global__ __launch_bounds__(1024) void k_op(Args a, int64_t nblocks, int remap) {
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  process_block<S, OP>(a, lb);
}

// Persistent batched form: the global tile index space is the concatenation
// of each tracer's blocks; every workgroup walks a contiguous range of it.
template <class S, int OP>
__global__ __launch_bounds__(1024) void k_batched(Args base, const BatchItem* __restrict__ items, int nitems,
                                                  int64_t total, int remap) {
  const int64_t nb = gridDim.x;
  const int64_t lb = logical_block(blockIdx.x, nb, remap);   // grid is a multiple of 8 when remapping
  const int64_t per = (total + nb - 1) / nb;
  const int64_t t0 = lb * per;
  const int64_t t1 = t0 + per < total ? t0 + per : total;
  int item = 0;
  for (int64_t tile = t0; tile < t1; ++tile) {
    while (item + 1 < nitems && items[item + 1].tile_begin <= tile) ++item;
    // tiles are ascending, so the search from the first item only moves forward
    Args a = base;
    a.in = items[item].in;
    a.out = items[item].out;
    a.L = items[item].nlev;
    a.pack = items[item].pack;
    process_block<S, OP>(a, tile - items[item].tile_begin);
  }
}

// ---- conservation: fixed-order FP64 sums of V_i div_ik -------------------------

constexpr int kConsWaves = 4;

template <class S>
__global__ __launch_bounds__(256) void k_cons_partial(const S* __restrict__ div, const double* __restrict__ vol,
                                                      int64_t V, int L, int64_t chunk, double* __restrict__ part) {
  __shared__ double red[kConsWaves][64][2];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t n0 = (int64_t)blockIdx.x * chunk;
  const int64_t n1 = n0 + chunk < V ? n0 + chunk : V;
  for (int k0 = 0; k0 < L; k0 += 64) {
    const int k = k0 + lane;
    double s = 0.0, ab = 0.0;
    if (k < L) {
      for (int64_t i = n0 + wave; i < n1; i += kConsWaves) {
        const double p = vol[i] * (double)ld1(div + i * (int64_t)L + k);
        s += p;
        ab += fabs(p);
      }
    }
    red[wave][lane][0] = s;
    red[wave][lane][1] = ab;
    __syncthreads();
    if (wave == 0 && k < L) {
      double ts = red[0][lane][0], ta = red[0][lane][1];
      for (int w = 1; w < kConsWaves; ++w) {
        ts += red[w][lane][0];
        ta += red[w][lane][1];
      }
      part[((int64_t)blockIdx.x * L + k) * 2] = ts;
      part[((int64_t)blockIdx.x * L + k) * 2 + 1] = ta;
    }
    __syncthreads();
  }
}

__global__ void k_cons_final(const double* __restrict__ part, int nparts, int L, double* __restrict__ out_sum,
                             double* __restrict__ out_abs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  double s = 0.0, a = 0.0;
  for (int p = 0; p < nparts; ++p) {
    s += part[((int64_t)p * L + k) * 2];
    a += part[((int64_t)p * L + k) * 2 + 1];
  }
  out_sum[k] = s;
  out_abs[k] = a;
}

// ---- dispatch ---------------------------------------------------------------

Args make_args(int op, const DevTables& t, int64_t V, int nlev, const void* in, void* out, const Shape& sh) {
  Args a;
  if (op == OP_LAP) {
    a.nbr = t.lap_nbr;
    a.coef = t.lap_w;
    a.stride = t.lap_stride;
  } else {
    a.nbr = t.nbr8;
    a.coef = t.coef[op];
    a.stride = 8;
  }
  a.in = in;
  a.out = out;
  a.V = V;
  a.L = nlev;
  a.pack = pack_factor(nlev);
  a.npw = sh.nodes_per_wave;
  return a;
}

int64_t blocks_for(int64_t V, int nlev, const Shape& sh) {
  const int pack = pack_factor(nlev);
  const int64_t per_block = (int64_t)sh.waves_per_block * sh.nodes_per_wave * (pack ? pack : 1);
  return (V + per_block - 1) / per_block;
}

template <class S>
hipError_t launch_op_t(int op, const Args& a, int64_t nblocks, const Shape& sh, hipStream_t st) {
  const int64_t grid = sh.xcd_remap ? (nblocks + 7) / 8 * 8 : nblocks;
  const dim3 g((unsigned)grid), b((unsigned)(64 * sh.waves_per_block));
  switch (op) {
    case OP_GRAD: hipLaunchKernelGGL((k_op<S, OP_GRAD>), g, b, 0, st, a, nblocks, sh.xcd_remap); break;
    case OP_DIV: hipLaunchKernelGGL((k_op<S, OP_DIV>), g, b, 0, st, a, nblocks, sh.xcd_remap); break;
    case OP_GRADT: hipLaunchKernelGGL((k_op<S, OP_GRADT>), g, b, 0, st, a, nblocks, sh.xcd_remap); break;
    case OP_DIVT: hipLaunchKernelGGL((k_op<S, OP_DIVT>), g, b, 0, st, a, nblocks, sh.xcd_remap); break;
    case OP_LAP: hipLaunchKernelGGL((k_op<S, OP_LAP>), g, b, 0, st, a, nblocks, sh.xcd_remap); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_batched_t(int op, const Args& a, const BatchItem* items, int nitems, int64_t total,
                            const Shape& sh, int num_cus, hipStream_t st) {
  int64_t grid = (int64_t)sh.blocks_per_cu * num_cus;
  if (grid > total) grid = total;
  if (grid < 1) grid = 1;
  const int remap = (sh.xcd_remap && grid % 8 == 0) ? 1 : 0;
  const dim3 g((unsigned)grid), b((unsigned)(64 * sh.waves_per_block));
  switch (op) {
    case OP_GRAD: hipLaunchKernelGGL((k_batched<S, OP_GRAD>), g, b, 0, st, a, items, nitems, total, remap); break;
    case OP_DIV: hipLaunchKernelGGL((k_batched<S, OP_DIV>), g, b, 0, st, a, items, nitems, total, remap); break;
    case OP_GRADT: hipLaunchKernelGGL((k_batched<S, OP_GRADT>), g, b, 0, st, a, items, nitems, total, remap); break;
    case OP_DIVT: hipLaunchKernelGGL((k_batched<S, OP_DIVT>), g, b, 0, st, a, items, nitems, total, remap); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_op(int op, int dtype, const DevTables& t, int64_t V, int nlev, const void* in, void* out,
                     const Shape& shape, hipStream_t stream) {
  if (op == OP_LAP && t.lap_stride != kLapMax) return hipErrorInvalidValue;
  const Args a = make_args(op, t, V, nlev, in, out, shape);
  const int64_t nblocks = blocks_for(V, nlev, shape);
  switch (dtype) {
    case DT_F64: return launch_op_t<double>(op, a, nblocks, shape, stream);
    case DT_F32: return launch_op_t<float>(op, a, nblocks, shape, stream);
    case DT_BF16: return launch_op_t<bf16_t>(op, a, nblocks, shape, stream);
    default: return hipErrorInvalidValue;
  }
}

int conservation_parts(int64_t V, int nlev) {
  (void)nlev;
  int64_t p = (V + 255) / 256;
  return (int)(p < 1024 ? p : 1024);
}

hipError_t launch_conservation(int dtype, const double* vol, int64_t V, int nlev, const void* div, double* scratch,
                               double* out_sum, double* out_abs, hipStream_t stream) {
  const int parts = conservation_parts(V, nlev);
  const int64_t chunk = (V + parts - 1) / parts;
  switch (dtype) {
    case DT_F64:
      hipLaunchKernelGGL(k_cons_partial<double>, dim3(parts), dim3(256), 0, stream,
                         static_cast<const double*>(div), vol, V, nlev, chunk, scratch);
      break;
    case DT_F32:
      hipLaunchKernelGGL(k_cons_partial<float>, dim3(parts), dim3(256), 0, stream,
                         static_cast<const float*>(div), vol, V, nlev, chunk, scratch);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_cons_partial<bf16_t>, dim3(parts), dim3(256), 0, stream,
                         static_cast<const bf16_t*>(div), vol, V, nlev, chunk, scratch);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cons_final, dim3((nlev + 127) / 128), dim3(128), 0, stream, scratch, parts, nlev, out_sum,
                     out_abs);
  return hipGetLastError();
}

int64_t tiles_for(int64_t V, int nlev, const Shape& shape) { return blocks_for(V, nlev, shape); }

hipError_t launch_batched(int op, int dtype, const DevTables& t, int64_t V, const BatchItem* items, int nitems,
                          int64_t total_tiles, const Shape& shape, int num_cus, hipStream_t stream) {
  Args a = make_args(op, t, V, 1, nullptr, nullptr, shape);
  switch (dtype) {
    case DT_F64: return launch_batched_t<double>(op, a, items, nitems, total_tiles, shape, num_cus, stream);
    case DT_F32: return launch_batched_t<float>(op, a, items, nitems, total_tiles, shape, num_cus, stream);
    case DT_BF16: return launch_batched_t<bf16_t>(op, a, items, nitems, total_tiles, shape, num_cus, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace atlasnabla
