// gfx950 kernels of the median-dual Nabla operators.
//
// Every operator is a gather over a node's incident edges (the edge sums of
// the finite-volume operators listed in Section 2.3 of the report, evaluated
// node by node): the output element (node i, level k) is written by exactly
// one lane, neighbour values are read in a fixed slot order, and nothing is
// accumulated across lanes, so there are no atomics and reruns are bitwise
// identical.  The path is a sparse stencil whose dense dimension is the level
// column, so it is bound by memory traffic and uses no matrix cores.
//
// Mapping.  Fields are [node][level] with levels innermost.  A 64-lane wave
// owns G = 64 / P nodes at a time, P lanes per node; lane t of a node handles
// levels t, t + P, t + 2P, ... of its column.  P is chosen per level count so
// that the column fills the lanes well (P = nlev for columns of at most 32
// levels, else 64, 32 or 16, e.g. 16 lanes x 9 slices for 137 levels).  The
// lane -> node assignment is fixed, so each lane reads its node's table row
// (neighbour offsets and coefficient pairs) once and keeps it in registers for
// the whole column.  U level slices are processed per iteration with all
// neighbour loads issued before any arithmetic, which keeps many independent
// loads in flight per wave; loads of slices past the column end are clamped
// to the last level (cache hits) and their results are not stored.
//
// Cache reuse.  Each node value is read by the node and its ~6 neighbours,
// two of them in the row above and two in the row below; at 137 FP32 levels
// three rows of the O1280 grid already exceed an XCD's 4 MB L2.  Work
// therefore follows a node order built on the host: bands of rows, nodes of a
// band sorted by longitude, so the rows above and below are touched at the
// same longitude at about the same time.  Workgroups are dispatched
// round-robin over the eight XCDs; with remapping on, workgroup b works on
// logical block (b mod 8) * ceil(nblocks / 8) + b / 8, so each XCD walks a
// contiguous part of the order (whole bands) in its own L2.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <type_traits>

#include "launch.hpp"

namespace atlasnabla {

namespace {

using bf16_t = uint16_t;

constexpr int kLapStride = 24;   // two-ring record: up to 23 entries + the count

template <class S> struct Traits;
template <> struct Traits<double> { using C = double; using C2 = double2; };
template <> struct Traits<float> { using C = float; using C2 = float2; };
template <> struct Traits<bf16_t> { using C = float; using C2 = float2; };

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// FP32 to BF16, round to nearest even, a NaN kept as a quiet NaN with its
// payload's top bits: gfx950's v_cvt_pk_bf16_f32, one instruction for two
// values (checked equal, on all 2^32 inputs, to the rounding written out on
// the bits: add 0x7fff plus the lowest kept bit, keep the top half).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x, y}, bf16x2_t));
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

// Output stores: plain, or non-temporal (streamed past L2) when the launch
// asks for it.  Plain stores let L2 merge the partial cache lines shared by
// the columns of neighbouring nodes.
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <bool NT, class T>
__device__ __forceinline__ void st_raw(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <bool NT>
__device__ __forceinline__ void st1(double* p, double v) { st_raw<NT>(p, v); }
template <bool NT>
__device__ __forceinline__ void st1(float* p, float v) { st_raw<NT>(p, v); }
template <bool NT>
__device__ __forceinline__ void st1(bf16_t* p, float v) { st_raw<NT>(p, (bf16_t)f32_to_bf16(v)); }

template <bool NT>
__device__ __forceinline__ void st2(double* p, double x, double y) {
  st_raw<NT>(reinterpret_cast<f64x2*>(p), f64x2{x, y});
}
template <bool NT>
__device__ __forceinline__ void st2(float* p, float x, float y) {
  st_raw<NT>(reinterpret_cast<f32x2*>(p), f32x2{x, y});
}
template <bool NT>
__device__ __forceinline__ void st2(bf16_t* p, float x, float y) {
  st_raw<NT>(reinterpret_cast<uint32_t*>(p), f32x2_to_bf16x2(x, y));
}

// Read-only table data read through the constant address space: with a
// wave-uniform address the compiler fetches it with scalar loads into scalar
// registers.  Valid because no kernel writes the tables.
template <class T>
__device__ __forceinline__ T ld_const(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}
__device__ __forceinline__ int32_t ld_uniform(const int32_t* p) { return ld_const(p); }
__device__ __forceinline__ float2 ld_uniform(const float2* p) {
  const float* q = reinterpret_cast<const float*>(p);
  return make_float2(ld_const(q), ld_const(q + 1));
}
__device__ __forceinline__ double2 ld_uniform(const double2* p) {
  const double* q = reinterpret_cast<const double*>(p);
  return make_double2(ld_const(q), ld_const(q + 1));
}

struct Args {
  const int32_t* order; // [V] node processing order (a permutation)
  const int32_t* runs;  // [nruns][2] (first node, count): the same order as row runs
  int64_t nruns;
  const int32_t* nbr;   // [V][8] neighbour table or [V][24] two-ring table
  const void* coef;     // coefficient pairs or two-ring weights (same row layout)
  const void* in;
  void* out;
  int64_t V;
  int32_t L;            // levels
  int32_t P;            // lanes per node (64 / P nodes per wave)
  int32_t npw;          // node groups (or runs) per wave per workgroup
  int32_t nt;           // non-temporal output stores
};

// ---- one node group per wave --------------------------------------------------
//
// NS: table entries read per node (7 = every slot, padded with the node itself
// and zero coefficients; 6 when every node of the wave has degree 6; 23 or 18
// for the two-ring table).  Padding entries add exact zeros.  Entries are
// consumed in slot order, which fixes the summation order of every element.

template <class S, int OP, int NS, int U>
__device__ __forceinline__ void run_1ring(const Args& a, int64_t nd, bool ok, int t) {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  const int32_t* nbp = a.nbr + nd * 8;
  const C2* cfp = static_cast<const C2*>(a.coef) + nd * 8;
  const uint32_t L = (uint32_t)a.L;
  uint32_t off[NS];
  C2 cf[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    off[s] = (uint32_t)nbp[s] * L;
    cf[s] = cfp[s];
  }
  const C2 dg = cfp[7];
  const uint32_t self = (uint32_t)nd * L;
  const S* __restrict__ in = static_cast<const S*>(a.in);
  S* __restrict__ out = static_cast<S*>(a.out);
  const int P = a.P;
  const int nsl = (a.L + P - 1) / P;
  for (int r0 = 0; r0 < nsl; r0 += U) {
    uint32_t kc[U];
    bool st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t k = (uint32_t)(t + P * (r0 + u));
      st[u] = ok && k < L;
      kc[u] = k < L ? k : L - 1;
    }
    if constexpr (OP == OP_GRAD || OP == OP_DIVT) {
      C v[U][NS], x0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int s = 0; s < NS; ++s) v[u][s] = ld1(in + (size_t)(off[s] + kc[u]));
        x0[u] = ld1(in + (size_t)(self + kc[u]));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        C ax, ay;
        if constexpr (OP == OP_GRAD) {
          // difference form: sum_s (a, b)_s (f_n - f_i)
          ax = 0;
          ay = 0;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const C d = v[u][s] - x0[u];
            ax = fma(cf[s].x, d, ax);
            ay = fma(cf[s].y, d, ay);
          }
        } else {
          // divergence adjoint: (A, B)_i d_i + sum_s (c, d)_{n,rev} d_n
          ax = dg.x * x0[u];
          ay = dg.y * x0[u];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            ax = fma(cf[s].x, v[u][s], ax);
            ay = fma(cf[s].y, v[u][s], ay);
          }
        }
        if (st[u]) {
          if (a.nt) st2<true>(out + 2 * (size_t)(self + kc[u]), ax, ay);
          else st2<false>(out + 2 * (size_t)(self + kc[u]), ax, ay);
        }
      }
    } else {
      // divergence and gradient adjoint: diag . in_i + sum_s (x, y)_s . in_n
      C2 v[U][NS], x0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int s = 0; s < NS; ++s) v[u][s] = ld2(in + 2 * (size_t)(off[s] + kc[u]));
        x0[u] = ld2(in + 2 * (size_t)(self + kc[u]));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        C acc = dg.x * x0[u].x;
        acc = fma(dg.y, x0[u].y, acc);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          acc = fma(cf[s].x, v[u][s].x, acc);
          acc = fma(cf[s].y, v[u][s].y, acc);
        }
        if (st[u]) {
          if (a.nt) st1<true>(out + (size_t)(self + kc[u]), acc);
          else st1<false>(out + (size_t)(self + kc[u]), acc);
        }
      }
    }
  }
}

// fused Laplacian over the two-ring: sum_m W_im (f_m - f_i)
template <class S, int NS, int U>
__device__ __forceinline__ void run_lap(const Args& a, int64_t nd, bool ok, int t) {
  using C = typename Traits<S>::C;
  const int32_t* nbp = a.nbr + nd * kLapStride;
  const C* wp = static_cast<const C*>(a.coef) + nd * kLapStride;
  const uint32_t L = (uint32_t)a.L;
  uint32_t off[NS];
  C w[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    off[s] = (uint32_t)nbp[s] * L;
    w[s] = wp[s];
  }
  const uint32_t self = (uint32_t)nd * L;
  const S* __restrict__ in = static_cast<const S*>(a.in);
  S* __restrict__ out = static_cast<S*>(a.out);
  const int P = a.P;
  const int nsl = (a.L + P - 1) / P;
  for (int r0 = 0; r0 < nsl; r0 += U) {
    uint32_t kc[U];
    bool st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t k = (uint32_t)(t + P * (r0 + u));
      st[u] = ok && k < L;
      kc[u] = k < L ? k : L - 1;
    }
    C v[U][NS], x0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = ld1(in + (size_t)(off[s] + kc[u]));
      x0[u] = ld1(in + (size_t)(self + kc[u]));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      C acc = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = fma(w[s], v[u][s] - x0[u], acc);
      if (st[u]) {
        if (a.nt) st1<true>(out + (size_t)(self + kc[u]), acc);
        else st1<false>(out + (size_t)(self + kc[u]), acc);
      }
    }
  }
}

// gbase: first position (in the node order) of the wave's group of G nodes.
template <class S, int OP, int U>
__device__ __forceinline__ void run_group(const Args& a, int64_t gbase, int lane) {
  const int P = a.P;
  const int G = 64 / P;
  const int j = lane / P;
  const int t = lane - j * P;
  const int64_t q = gbase + j;
  const bool ok = j < G && q < a.V;
  const int64_t nd = a.order[ok ? q : gbase];   // gbase < V: a valid node for idle lanes
  // The padded wide variants serve the few waves that touch a node of
  // degree 5 or 7 (16 + 4 per mesh) or a wide two-ring; they run one slice
  // per iteration so that they do not set the register budget of the kernel.
  if constexpr (OP == OP_LAP) {
    const int cnt = a.nbr[nd * kLapStride + kLapStride - 1];
    if (__all(cnt <= 18)) run_lap<S, 18, U>(a, nd, ok, t);
    else run_lap<S, kLapStride - 1, 1>(a, nd, ok, t);
  } else {
    const int deg = a.nbr[nd * 8 + 7] & 0xff;
    if (__all(deg == 6)) run_1ring<S, OP, 6, U>(a, nd, ok, t);
    else run_1ring<S, OP, 7, 1>(a, nd, ok, t);
  }
}

// ---- row-window walk (1-ring operators, columns of more than 32 levels) ----
//
// A wave walks a run of consecutive nodes of one latitude row, 64 lanes =
// 64 levels, U slices of the column at once.  For a window-eligible node the
// slots in neighbour order are [row above (cu), left, right, row below (cl)],
// the previous node's self and right neighbour are this node's left and self,
// and the previous node's last neighbour above (below) is this node's first
// one above (below).  So a node needs only 1 + (cu - 1) + (cl - 1) new column
// loads (3 for the usual cu = cl = 2) instead of deg + 1.  Other nodes (run
// starts, polar rows, neighbours wrapping past the zero meridian) load every
// slot.  Either way the values are combined in slot order with the same fused
// multiply-adds as the per-lane path, so all paths give identical bits.

template <class S, int OP>
struct WinT {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  static constexpr bool kVecIn = (OP == OP_DIV || OP == OP_GRADT || OP == OP_DIVCURL);
  using X = typename std::conditional<kVecIn, C2, C>::type;
  static __device__ __forceinline__ X ld(const S* __restrict__ in, uint32_t idx) {
    if constexpr (kVecIn) return ld2(in + 2 * (size_t)idx);
    else return ld1(in + (size_t)idx);
  }
};

// Combine deg slot values (slot order) with the node's coefficients: r0 (and
// r1 for the two-component outputs of OP_GRAD and OP_DIVT).
template <class S, int OP, int DEG>
__device__ __forceinline__ void win_combine(const typename WinT<S, OP>::X x0, const typename WinT<S, OP>::X* v,
                                            const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg,
                                            typename Traits<S>::C& r0, typename Traits<S>::C& r1) {
  using C = typename Traits<S>::C;
  if constexpr (OP == OP_GRAD || OP == OP_DIVT) {
    C ax, ay;
    if constexpr (OP == OP_GRAD) {
      ax = 0;
      ay = 0;
#pragma unroll
      for (int s = 0; s < DEG; ++s) {
        const C d = v[s] - x0;
        ax = fma(cf[s].x, d, ax);
        ay = fma(cf[s].y, d, ay);
      }
    } else {
      ax = dg.x * x0;
      ay = dg.y * x0;
#pragma unroll
      for (int s = 0; s < DEG; ++s) {
        ax = fma(cf[s].x, v[s], ax);
        ay = fma(cf[s].y, v[s], ay);
      }
    }
    r0 = ax;
    r1 = ay;
  } else {
    C acc = dg.x * x0.x;
    acc = fma(dg.y, x0.y, acc);
#pragma unroll
    for (int s = 0; s < DEG; ++s) {
      acc = fma(cf[s].x, v[s].x, acc);
      acc = fma(cf[s].y, v[s].y, acc);
    }
    r0 = acc;
    r1 = 0;
  }
}

// Store of a combined value at node-level index o (two components for
// OP_GRAD and OP_DIVT).
template <class S, int OP>
__device__ __forceinline__ void win_store(S* __restrict__ out, uint32_t o, int nt, typename Traits<S>::C r0,
                                          typename Traits<S>::C r1) {
  if constexpr (OP == OP_GRAD || OP == OP_DIVT) {
    if (nt) st2<true>(out + 2 * (size_t)o, r0, r1);
    else st2<false>(out + 2 * (size_t)o, r0, r1);
  } else {
    if (nt) st1<true>(out + (size_t)o, r0);
    else st1<false>(out + (size_t)o, r0);
  }
}

// Combine and store (lanes with st set).
template <class S, int OP, int DEG>
__device__ __forceinline__ void win_emit(S* __restrict__ out, uint32_t o, bool st, int nt,
                                         const typename WinT<S, OP>::X x0, const typename WinT<S, OP>::X* v,
                                         const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg) {
  typename Traits<S>::C r0, r1;
  win_combine<S, OP, DEG>(x0, v, cf, dg, r0, r1);
  if (st) win_store<S, OP>(out, o, nt, r0, r1);
}

// Run-time choice among register values, written as element-wise selects so
// that no private array is indexed at run time.
__device__ __forceinline__ float pick3(int k, float a, float b, float c) { return k == 0 ? a : (k == 1 ? b : c); }
__device__ __forceinline__ double pick3(int k, double a, double b, double c) { return k == 0 ? a : (k == 1 ? b : c); }
__device__ __forceinline__ float2 pick3(int k, float2 a, float2 b, float2 c) {
  return make_float2(pick3(k, a.x, b.x, c.x), pick3(k, a.y, b.y, c.y));
}
__device__ __forceinline__ double2 pick3(int k, double2 a, double2 b, double2 c) {
  return make_double2(pick3(k, a.x, b.x, c.x), pick3(k, a.y, b.y, c.y));
}
template <class T>
__device__ __forceinline__ T pick4(int k, T a, T b, T c, T d) { return k == 3 ? d : pick3(k, a, b, c); }

template <class S, int OP, int U>
struct WinState {
  typename WinT<S, OP>::X self[U], right[U], up[U], lo[U];
};

// Full step: every slot loaded (slot order), one slice at a time.
template <class S, int OP, int U>
__device__ __forceinline__ void win_full(const Args& a, int32_t i, const int32_t* nbp, int deg, int cu, bool eligible,
                                         const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg,
                                         const uint32_t* kc, const bool* st, WinState<S, OP, U>& w) {
  using X = typename WinT<S, OP>::X;
  const S* __restrict__ in = static_cast<const S*>(a.in);
  const uint32_t L = (uint32_t)a.L;
  uint32_t off[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) off[s] = (uint32_t)ld_uniform(nbp + s) * L;   // padded with the node itself
  const uint32_t self = (uint32_t)i * L;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    X v[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) v[s] = WinT<S, OP>::ld(in, off[s] + kc[u]);
    const X x0 = WinT<S, OP>::ld(in, self + kc[u]);
    S* out = static_cast<S*>(a.out);
    switch (deg) {
      case 6: win_emit<S, OP, 6>(out, self + kc[u], st[u], a.nt, x0, v, cf, dg); break;
      case 5: win_emit<S, OP, 5>(out, self + kc[u], st[u], a.nt, x0, v, cf, dg); break;
      case 7: win_emit<S, OP, 7>(out, self + kc[u], st[u], a.nt, x0, v, cf, dg); break;
      case 4: win_emit<S, OP, 4>(out, self + kc[u], st[u], a.nt, x0, v, cf, dg); break;
      default: win_emit<S, OP, 3>(out, self + kc[u], st[u], a.nt, x0, v, cf, dg); break;
    }
    if (eligible) {
      // eligible nodes have cu in 1..3 and deg = cu + cl + 2 with cl in 1..3
      w.self[u] = x0;
      w.right[u] = pick3(cu - 1, v[2], v[3], v[4]);
      w.up[u] = pick3(cu - 1, v[0], v[1], v[2]);
      w.lo[u] = pick4(deg - 4, v[3], v[4], v[5], v[6]);
    }
  }
}

// Window step of a window-eligible node with CU neighbours above and CL
// below: loads only the columns that are new to the window (the right
// neighbour, above 2..CU, below 2..CL) and slides the window by one node.
template <class S, int OP, int U, int CU, int CL>
__device__ __forceinline__ void win_step(const Args& a, int32_t i, const int32_t* nbp,
                                         const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg,
                                         const uint32_t* kc, const bool* st, WinState<S, OP, U>& w) {
  using X = typename WinT<S, OP>::X;
  constexpr int DEG = CU + CL + 2;
  const S* __restrict__ in = static_cast<const S*>(a.in);
  const uint32_t L = (uint32_t)a.L;
  uint32_t offu[CU > 1 ? CU - 1 : 1], offl[CL > 1 ? CL - 1 : 1];
#pragma unroll
  for (int t = 1; t < CU; ++t) offu[t - 1] = (uint32_t)ld_uniform(nbp + t) * L;
#pragma unroll
  for (int t = 1; t < CL; ++t) offl[t - 1] = (uint32_t)ld_uniform(nbp + CU + 2 + t) * L;
  const uint32_t offr = (uint32_t)(i + 1) * L;
  X nu[U][CU > 1 ? CU - 1 : 1], nl[U][CL > 1 ? CL - 1 : 1], nr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    nr[u] = WinT<S, OP>::ld(in, offr + kc[u]);
#pragma unroll
    for (int t = 0; t < CU - 1; ++t) nu[u][t] = WinT<S, OP>::ld(in, offu[t] + kc[u]);
#pragma unroll
    for (int t = 0; t < CL - 1; ++t) nl[u][t] = WinT<S, OP>::ld(in, offl[t] + kc[u]);
  }
  const uint32_t self = (uint32_t)i * L;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    X v[DEG];
    v[0] = w.up[u];
#pragma unroll
    for (int t = 1; t < CU; ++t) v[t] = nu[u][t - 1];
    v[CU] = w.self[u];           // left neighbour = previous node
    v[CU + 1] = nr[u];           // right neighbour
    v[CU + 2] = w.lo[u];
#pragma unroll
    for (int t = 1; t < CL; ++t) v[CU + 2 + t] = nl[u][t - 1];
    const X x0 = w.right[u];     // this node = previous right neighbour
    win_emit<S, OP, DEG>(static_cast<S*>(a.out), self + kc[u], st[u], a.nt, x0, v, cf, dg);
    w.self[u] = x0;
    w.right[u] = nr[u];
    w.up[u] = v[CU - 1];
    w.lo[u] = v[DEG - 1];
  }
}

// One wave walks one run of consecutive nodes of a row, U level slices of 64
// at a time; the first node of a run, and any node outside the window pattern,
// takes a full step that reloads every slot.
template <class S, int OP, int U>
__device__ __forceinline__ void win_run(const Args& a, int32_t i0, int cnt, int lane) {
  using C2 = typename Traits<S>::C2;
  const uint32_t L = (uint32_t)a.L;
  for (uint32_t k0 = 0; k0 < L; k0 += 64u * U) {
    uint32_t kc[U];
    bool st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t k = k0 + 64u * u + (uint32_t)lane;
      st[u] = k < L;
      kc[u] = k < L ? k : L - 1;
    }
    WinState<S, OP, U> w;
    bool have = false;
    for (int n = 0; n < cnt; ++n) {
      const int32_t i = i0 + n;
      const int32_t* nbp = a.nbr + (int64_t)i * 8;
      const int meta = ld_uniform(nbp + 7);
      const int deg = meta & 0xff;
      const int cu = (meta >> 8) & 0xff;
      const bool eligible = (meta >> 16) & 1;
      const C2* cfp = static_cast<const C2*>(a.coef) + (int64_t)i * 8;
      C2 cf[7];
#pragma unroll
      for (int s = 0; s < 7; ++s) cf[s] = ld_uniform(cfp + s);
      const C2 dg = ld_uniform(cfp + 7);
      const int cl = deg - cu - 2;
      if (have && eligible && cu == 2 && cl == 2) win_step<S, OP, U, 2, 2>(a, i, nbp, cf, dg, kc, st, w);
      else if (have && eligible && cu == 1 && cl == 3) win_step<S, OP, U, 1, 3>(a, i, nbp, cf, dg, kc, st, w);
      else if (have && eligible && cu == 3 && cl == 1) win_step<S, OP, U, 3, 1>(a, i, nbp, cf, dg, kc, st, w);
      else if (have && eligible && cu == 1 && cl == 2) win_step<S, OP, U, 1, 2>(a, i, nbp, cf, dg, kc, st, w);
      else if (have && eligible && cu == 2 && cl == 1) win_step<S, OP, U, 2, 1>(a, i, nbp, cf, dg, kc, st, w);
      else win_full<S, OP, U>(a, i, nbp, deg, cu, eligible, cf, dg, kc, st, w);
      have = eligible;
    }
  }
}

// Work of logical block `lb` on the run list: waves_per_block * npw runs.
template <class S, int OP, int U>
__device__ __forceinline__ void process_runs(const Args& a, int64_t lb) {
  const int wpb = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int r = 0; r < a.npw; ++r) {
    const int64_t run = (lb * a.npw + r) * wpb + wave;
    if (run >= a.nruns) break;
    const int32_t i0 = ld_uniform(a.runs + 2 * run);
    const int32_t cnt = ld_uniform(a.runs + 2 * run + 1);
    win_run<S, OP, U>(a, i0, cnt, lane);
  }
}

// Work of logical block `lb`: waves_per_block * npw node groups.
template <class S, int OP, int U>
__device__ __forceinline__ void process_block(const Args& a, int64_t lb) {
  const int wpb = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int G = 64 / a.P;
  for (int r = 0; r < a.npw; ++r) {
    const int64_t gbase = ((lb * a.npw + r) * wpb + wave) * G;
    if (gbase >= a.V) break;
    run_group<S, OP, U>(a, gbase, lane);
  }
}

__device__ __forceinline__ int64_t logical_block(int64_t b, int64_t nblocks, int remap) {
  if (!remap) return b;
  const int64_t per = (nblocks + 7) / 8;
  return (b & 7) * per + (b >> 3);
}

template <class S, int OP, int U>
__global__ __launch_bounds__(256) void k_op(Args a, int64_t nblocks, int remap) {
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  process_block<S, OP, U>(a, lb);
}

template <class S, int OP, int U>
__global__ __launch_bounds__(256) void k_win(Args a, int64_t nblocks, int remap) {
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  process_runs<S, OP, U>(a, lb);
}

// ---- LDS tiles -------------------------------------------------------------------
//
// A workgroup takes one tile: a set of nodes (a few latitude rows by one
// longitude sector) and the sorted set of every column their stencils read,
// stored as segments of consecutive nodes.  Columns of consecutive nodes are
// contiguous in memory, so each segment is one contiguous block, which a wave
// copies with direct global->LDS loads (16 bytes per lane, no registers
// involved); the tile's node records (coefficients, LDS positions of the
// stencil entries, node index), packed in tile order when the tiling is set
// up, arrive in one more contiguous copy.  One wait and one barrier end the
// copy.  Each wave then takes nodes of the tile in turn, 64 lanes = 64
// levels, and reads its stencil and record from LDS; only the output goes
// back to memory.  No global load sits on a node's critical path, every wave
// keeps many independent loads in flight during the copy, and the
// workgroups sharing a CU overlap each other's copy and compute phases.
// Tiles stacked in latitude follow each other, so the halo columns they share
// are L2 hits.

struct TileArgs {
  const int32_t* info;   // [ntiles + 1][4]: first segment, first record, columns, nodes
  const int32_t* segs;   // [nseg (+ 8 padding)][2]: first node, count
  const char* rec;       // [V] node records in tile order (see tile_record_bytes)
  const void* in;
  void* out;
  void* out2;            // OP_GRADLAP: the gradient ([V][L][2]); out gets the Laplacian
  int64_t ntiles;
  int32_t L;             // levels
  int32_t KL;            // levels per chunk (L: whole columns)
  int32_t nchunks;
  int32_t nt;
};

// Node record of the tile path: coefficient row (8 pairs, ring 1, followed
// for OP_DIVCURL by the 8 pairs of the second operator, the curl's or, for
// OP_DIVGRADT, the gradient adjoint's; 24 weights, ring 2, followed for
// OP_GRADLAP by the gradient's 8 pairs), LDS
// position row (8 or 24 uint16), node index (int32), zero padding to 16
// bytes.
template <class S, int OP>
struct TileRec {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  static constexpr bool kRing2 = OP == OP_LAP || OP == OP_GRADLAP;
  static constexpr bool kGrad = OP == OP_GRADLAP;   // gradient pairs after the weights
  static constexpr bool kDual = OP == OP_DIVCURL;    // second pairs after the divergence pairs
  static constexpr int kEntries = kRing2 ? kLapStride : 8;
  static constexpr uint32_t kLapB = kEntries * sizeof(C);   // ring 2: the 24 weights
  static constexpr uint32_t kCoefB = kRing2 ? kLapB + (kGrad ? 8 * sizeof(C2) : 0)
                                            : 8 * sizeof(C2) * (kDual ? 2 : 1);
  static constexpr uint32_t kLocB = 2 * kEntries;
  static constexpr uint32_t kIdOff = kCoefB + kLocB;
  static constexpr uint32_t kBytes = (kIdOff + 4 + 15) & ~15u;
  static constexpr int kCin = (OP == OP_DIV || OP == OP_GRADT || OP == OP_DIVCURL) ? 2 : 1;
};

constexpr int kLocCountShift = 11;

typedef __attribute__((address_space(3))) void* lds_vptr;

// s_waitcnt immediate with lgkmcnt = 0 and vmcnt, expcnt left at their
// maxima (vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).  Issued
// through the builtin rather than inline assembly so that the compiler's own
// wait insertion accounts for it.
constexpr int kWaitLgkm0 = 0xC07F;

constexpr uint64_t kLdsPerCu = 160 * 1024;   // gfx950 LDS per CU
constexpr int64_t kBf16ColExtra = 12;        // BF16 tiles: LDS bytes per column beyond the data

// Direct loads of nbytes (a multiple of 4) from global src to LDS byte offset
// dst: 16 bytes per lane (lane l of instruction q moves bytes 16 (64 q + l)
// onwards; gfx950 accepts any 4-byte alignment on both sides), then the last
// 0..3 dwords one per lane.  Instruction q goes to wave (ctr + q) mod W (W a
// power of two), ctr counting the instructions of the workgroup's earlier
// copies, so that small copies spread over the waves.
__device__ __forceinline__ void dma_copy(const char* src, char* lds, uint32_t dst, uint32_t nbytes, int wave, int W,
                                         int lane, uint32_t& ctr) {
  const uint32_t n16 = nbytes >> 4;
  const uint32_t ninst = (n16 + 63) >> 6;
  const uint32_t wm = (uint32_t)W - 1;   // W is a power of two
  for (uint32_t q = ((uint32_t)wave - ctr) & wm; q < ninst; q += (uint32_t)W) {
    const uint32_t d = q * 64 + (uint32_t)lane;
    if (d < n16)
      __builtin_amdgcn_global_load_lds(src + 16 * (size_t)d, (lds_vptr)(lds + dst + 1024 * q), 16, 0, 0);
  }
  ctr += ninst;
  const uint32_t rem = (nbytes & 15u) >> 2;
  if (rem) {
    if ((uint32_t)wave == (ctr & wm) && (uint32_t)lane < rem)
      __builtin_amdgcn_global_load_lds(src + 16 * (size_t)n16 + 4 * lane, (lds_vptr)(lds + dst + 16 * n16), 4, 0, 0);
    ++ctr;
  }
}

// Direct loads of cnt column chunks of nb bytes each (nb a multiple of 4),
// chunk c at global src + c * gstride, packed back to back at LDS byte offset
// dst.  The LDS image is contiguous, so each instruction still fills 64
// consecutive units (16 bytes when nb allows, else 4); a lane finds its
// chunk by dividing its unit index by the units per chunk.
__device__ __forceinline__ void dma_copy_strided(const char* src, size_t gstride, uint32_t cnt, uint32_t nb,
                                                 char* lds, uint32_t dst, int wave, int W, int lane,
                                                 uint32_t& ctr) {
  const bool wide = (nb & 15u) == 0;
  const uint32_t ub = wide ? 16u : 4u;
  const uint32_t upc = nb / ub;                       // units per chunk
  const uint32_t total = cnt * upc;
  const uint32_t ninst = (total + 63) >> 6;
  const uint32_t wm = (uint32_t)W - 1;   // W is a power of two
  for (uint32_t q = ((uint32_t)wave - ctr) & wm; q < ninst; q += (uint32_t)W) {
    const uint32_t u = q * 64 + (uint32_t)lane;
    if (u < total) {
      const uint32_t c = u / upc, o = u - c * upc;
      const char* g = src + (size_t)c * gstride + (size_t)o * ub;
      if (wide) __builtin_amdgcn_global_load_lds(g, (lds_vptr)(lds + dst + 1024 * q), 16, 0, 0);
      else __builtin_amdgcn_global_load_lds(g, (lds_vptr)(lds + dst + 256 * q), 4, 0, 0);
    }
  }
  ctr += ninst;
}

// Calls f(first, count) for pairs [b, e) of a (first, count) table, in order.
// Pairs come eight at a time from independent scalar loads (one wait per
// eight); the tables carry eight pairs of padding so the loads stay in
// bounds.  Scalar loads leave the vector memory counter alone, so fetching
// the next pairs never waits for direct loads already in flight.
template <class F>
__device__ __forceinline__ void for_pairs(const int32_t* tab, int32_t b, int32_t e, F&& f) {
  for (int32_t base = b; base < e; base += 8) {
    int32_t v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = ld_uniform(tab + 2 * (size_t)base + j);
    const int32_t n = e - base;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < n) f(v[2 * q], v[2 * q + 1]);
  }
}

template <class T>
__device__ __forceinline__ T lds_ld(const char* lds, uint32_t off) {
  return *reinterpret_cast<const T*>(lds + off);
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// One stencil value from an LDS tile, in the arithmetic type X (BF16 columns
// widen to FP32).
template <class S, class X>
__device__ __forceinline__ X lds_elem(const char* lds, uint32_t off) {
  if constexpr (sizeof(S) != 2) {
    return lds_ld<X>(lds, off);
  } else if constexpr (sizeof(X) == 4) {
    return bf16_to_f32(lds_ld<uint16_t>(lds, off));
  } else {
    const uint32_t w = lds_ld<uint32_t>(lds, off);
    return make_float2(bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16));
  }
}

// LDS positions of a node's entries (wave-uniform): pos[s] for the stencil
// slots, own position and entry count from the last record entry.
template <int NREC>
__device__ __forceinline__ void tile_positions(const char* lds, uint32_t off, uint32_t* pos, uint32_t& self,
                                               int& cnt) {
  uint32_t w[NREC / 2];
#pragma unroll
  for (int q = 0; q < NREC / 8; ++q) {
    const uint4 r = lds_ld<uint4>(lds, off + 16 * q);
    w[4 * q] = uni(r.x);
    w[4 * q + 1] = uni(r.y);
    w[4 * q + 2] = uni(r.z);
    w[4 * q + 3] = uni(r.w);
  }
#pragma unroll
  for (int s = 0; s < NREC - 1; ++s) pos[s] = (s & 1) ? (w[s >> 1] >> 16) : (w[s >> 1] & 0xffffu);
  const uint32_t last = w[NREC / 2 - 1] >> 16;
  self = last & ((1u << kLocCountShift) - 1);
  cnt = (int)(last >> kLocCountShift);
}

// Marks a value as computed here: the compiler may not sink its computation
// (and the LDS reads feeding it) into the predicated store that follows, so
// the reads of all slices of a step issue together.
template <class T>
__device__ __forceinline__ void keep(T& v) {
  asm volatile("" : "+v"(v));
}

// One node of a 1-ring operator: DEG slots, U slices of 64 levels per step.
// Each lane's LDS address of a slot is formed once per node; the level slices
// of a step then sit at constant offsets from it.  Lanes past the chunk's
// last level read (and drop) values beyond their column, which stay inside
// the tile buffer's tail of 64 U levels (tile_tail_bytes).
template <class S, int OP, int U, int DEG>
__device__ __forceinline__ void tile_node1(const TileArgs& a, const char* lds, const uint32_t* so, uint32_t xo,
                                           const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg,
                                           uint32_t obase, int klc, int lane) {
  using X = typename WinT<S, OP>::X;
  using C = typename Traits<S>::C;
  using R = TileRec<S, OP>;
  constexpr uint32_t kEl = (uint32_t)sizeof(S) * R::kCin;   // bytes per level in LDS
  constexpr uint32_t kOut = (OP == OP_GRAD || OP == OP_DIVT) ? 2 : 1;
  // BF16: values are left to the compiler's placement, which keeps the
  // vector-input kernels within 64 VGPRs (four workgroups per CU)
  constexpr bool kKeep = sizeof(S) != 2;
  const uint32_t lo = (uint32_t)lane * kEl;
  uint32_t vb[DEG];
#pragma unroll
  for (int s = 0; s < DEG; ++s) vb[s] = so[s] + lo;
  const uint32_t vx = xo + lo;
  S* __restrict__ out = static_cast<S*>(a.out) + (size_t)kOut * (obase + (uint32_t)lane);
  auto step = [&](int kb) {
    const uint32_t ko = (uint32_t)kb * kEl;
    X v[U][DEG], x0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = 0; s < DEG; ++s) v[u][s] = lds_elem<S, X>(lds, vb[s] + ko + 64u * kEl * u);
      x0[u] = lds_elem<S, X>(lds, vx + ko + 64u * kEl * u);
    }
    C r0[U], r1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      win_combine<S, OP, DEG>(x0[u], v[u], cf, dg, r0[u], r1[u]);
      if constexpr (kKeep) {
        keep(r0[u]);
        if constexpr (kOut == 2) keep(r1[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (kb + 64 * u + lane < klc) win_store<S, OP>(out + (size_t)kOut * kb, 64u * u, a.nt, r0[u], r1[u]);
  };
  step(0);
  for (int kb = 64 * U; kb < klc; kb += 64 * U) step(kb);
}

// One node of the two-ring Laplacian: NS entries (padded with the node itself
// and zero weights, which add exact zeros), sum_m W_im (f_m - f_i).  Addresses
// as in tile_node1.
template <class S, int U, int NS>
__device__ __forceinline__ void tile_node2(const TileArgs& a, const char* lds, const uint32_t* so, uint32_t xo,
                                           const typename Traits<S>::C* w, uint32_t obase, int klc, int lane) {
  using C = typename Traits<S>::C;
  constexpr uint32_t kEl = (uint32_t)sizeof(S);
  const uint32_t lo = (uint32_t)lane * kEl;
  uint32_t vb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) vb[s] = so[s] + lo;
  const uint32_t vx = xo + lo;
  S* __restrict__ out = static_cast<S*>(a.out) + (size_t)(obase + (uint32_t)lane);
  auto step = [&](int kb) {
    const uint32_t ko = (uint32_t)kb * kEl;
    C v[U][NS], x0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = lds_elem<S, C>(lds, vb[s] + ko + 64u * kEl * u);
      x0[u] = lds_elem<S, C>(lds, vx + ko + 64u * kEl * u);
    }
    C acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[u] = fma(w[s], v[u][s] - x0[u], acc[u]);
      keep(acc[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (kb + 64 * u + lane < klc) {
        S* o = out + (size_t)(kb + 64 * u);
        if (a.nt) st1<true>(o, acc[u]);
        else st1<false>(o, acc[u]);
      }
    }
  };
  step(0);
  for (int kb = 64 * U; kb < klc; kb += 64 * U) step(kb);
}

// One node of the fused gradient and two-ring Laplacian (OP_GRADLAP): the
// differences f_m - f_i of the NS entries feed both sums; the first 7 entries
// are the node's 1-ring neighbours in slot order (the two-ring tables are
// ordered so), weighted by the gradient pairs (zero past the node's degree,
// which add exact zeros).  Same slot-order arithmetic as tile_node2 and the
// gradient's tile_node1.
template <class S, int U, int NS>
__device__ __forceinline__ void tile_node2g(const TileArgs& a, const char* lds, const uint32_t* so, uint32_t xo,
                                            const typename Traits<S>::C* w, const typename Traits<S>::C2* cf,
                                            uint32_t obase, int klc, int lane) {
  using C = typename Traits<S>::C;
  constexpr uint32_t kEl = (uint32_t)sizeof(S);
  const uint32_t lo = (uint32_t)lane * kEl;
  uint32_t vb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) vb[s] = so[s] + lo;
  const uint32_t vx = xo + lo;
  S* __restrict__ out = static_cast<S*>(a.out) + (size_t)(obase + (uint32_t)lane);
  S* __restrict__ og = static_cast<S*>(a.out2) + 2 * (size_t)(obase + (uint32_t)lane);
  auto step = [&](int kb) {
    const uint32_t ko = (uint32_t)kb * kEl;
    C v[U][NS], x0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = lds_elem<S, C>(lds, vb[s] + ko + 64u * kEl * u);
      x0[u] = lds_elem<S, C>(lds, vx + ko + 64u * kEl * u);
    }
    C acc[U], ax[U], ay[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = 0;
      ax[u] = 0;
      ay[u] = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const C d = v[u][s] - x0[u];
        acc[u] = fma(w[s], d, acc[u]);
        if (s < 7) {
          ax[u] = fma(cf[s].x, d, ax[u]);
          ay[u] = fma(cf[s].y, d, ay[u]);
        }
      }
      keep(acc[u]);
      keep(ax[u]);
      keep(ay[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (kb + 64 * u + lane < klc) {
        const size_t k = (size_t)(kb + 64 * u);
        if (a.nt) {
          st1<true>(out + k, acc[u]);
          st2<true>(og + 2 * k, ax[u], ay[u]);
        } else {
          st1<false>(out + k, acc[u]);
          st2<false>(og + 2 * k, ax[u], ay[u]);
        }
      }
    }
  };
  step(0);
  for (int kb = 64 * U; kb < klc; kb += 64 * U) step(kb);
}

// One node of the divergence and a second operator of one vector field
// (OP_DIVCURL: the curl, or the gradient adjoint on OP_DIVGRADT's records):
// the same loads feed the divergence-form sums with the divergence pairs
// (out) and with the second pairs (out2), each exactly as tile_node1
// computes it for that operator.
template <class S, int U, int DEG>
__device__ __forceinline__ void tile_node1d(const TileArgs& a, const char* lds, const uint32_t* so, uint32_t xo,
                                            const typename Traits<S>::C2* cf, typename Traits<S>::C2 dg,
                                            const typename Traits<S>::C2* cf2, typename Traits<S>::C2 dg2,
                                            uint32_t obase, int klc, int lane) {
  using X = typename WinT<S, OP_DIVCURL>::X;
  using C = typename Traits<S>::C;
  constexpr uint32_t kEl = (uint32_t)sizeof(S) * 2;
  const uint32_t lo = (uint32_t)lane * kEl;
  uint32_t vb[DEG];
#pragma unroll
  for (int s = 0; s < DEG; ++s) vb[s] = so[s] + lo;
  const uint32_t vx = xo + lo;
  S* __restrict__ out = static_cast<S*>(a.out) + (size_t)(obase + (uint32_t)lane);
  S* __restrict__ oz = static_cast<S*>(a.out2) + (size_t)(obase + (uint32_t)lane);
  auto step = [&](int kb) {
    const uint32_t ko = (uint32_t)kb * kEl;
    X v[U][DEG], x0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = 0; s < DEG; ++s) v[u][s] = lds_elem<S, X>(lds, vb[s] + ko + 64u * kEl * u);
      x0[u] = lds_elem<S, X>(lds, vx + ko + 64u * kEl * u);
    }
    C r0[U], z0[U], unused;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      win_combine<S, OP_DIVCURL, DEG>(x0[u], v[u], cf, dg, r0[u], unused);
      win_combine<S, OP_DIVCURL, DEG>(x0[u], v[u], cf2, dg2, z0[u], unused);
      keep(r0[u]);
      keep(z0[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (kb + 64 * u + lane < klc) {
        win_store<S, OP_DIVCURL>(out + kb, 64u * u, a.nt, r0[u], 0);
        win_store<S, OP_DIVCURL>(oz + kb, 64u * u, a.nt, z0[u], 0);
      }
  };
  step(0);
  for (int kb = 64 * U; kb < klc; kb += 64 * U) step(kb);
}

// Copy of one tile (chunk) into an LDS buffer by W waves: the records as one
// copy spread over the waves, then each column segment by one wave (segment
// i by wave i mod W), so each wave sets up only its own copies.
template <class S, int OP>
__device__ __forceinline__ void tile_copy(const TileArgs& a, int64_t tile, int k0, int klc, char* buf, int wave,
                                          int W, int lane) {
  using R = TileRec<S, OP>;
  const int32_t* inf = a.info + 4 * tile;
  const int32_t seg0 = ld_uniform(inf), rec0 = ld_uniform(inf + 1), ncols = ld_uniform(inf + 2),
                nnodes = ld_uniform(inf + 3);
  const int32_t seg1 = ld_uniform(inf + 4);
  const uint32_t colB = (uint32_t)klc * R::kCin * (uint32_t)sizeof(S);   // LDS column stride (this chunk)
  uint32_t ctr = 0;
  dma_copy(a.rec + (size_t)rec0 * R::kBytes, buf, 0, (uint32_t)nnodes * R::kBytes, wave, W, lane, ctr);
  const size_t gcol = (size_t)a.L * R::kCin * sizeof(S);                 // global column bytes
  const char* in = static_cast<const char*>(a.in);
  uint32_t p = 0, i = 0;
  if constexpr (sizeof(S) == 2) {
    // BF16 columns may start 2 bytes into a dword: each segment is copied as
    // the dword-aligned span around it, placed so that LDS and memory agree
    // mod 4, and its columns' LDS offsets go to a table after the records.
    const uint32_t tab = (uint32_t)nnodes * R::kBytes;
    uint32_t cur = tab + (((uint32_t)ncols * 4u + 15u) & ~15u);
    for_pairs(a.segs, seg0, seg1, [&](int32_t first, int32_t cnt) {
      const size_t g0 = (size_t)first * gcol;
      const uint32_t mis = (uint32_t)(g0 & 3u);
      const uint32_t nb = (uint32_t)((((g0 + (size_t)cnt * colB) + 3u) & ~(size_t)3u) - (g0 - mis));
      if ((i & (uint32_t)(W - 1)) == (uint32_t)wave) {
        uint32_t own = 0;
        dma_copy(in + (g0 - mis), buf, cur, nb, 0, 1, lane, own);
        for (int32_t c = lane; c < cnt; c += 64)
          *reinterpret_cast<uint32_t*>(buf + tab + 4 * (p + (uint32_t)c)) = cur + mis + (uint32_t)c * colB;
      }
      cur += nb;
      p += (uint32_t)cnt;
      ++i;
    });
  } else {
    const uint32_t data_off = (uint32_t)nnodes * R::kBytes;
    for_pairs(a.segs, seg0, seg1, [&](int32_t first, int32_t cnt) {
      if ((i & (uint32_t)(W - 1)) == (uint32_t)wave) {
        uint32_t own = 0;
        if (a.KL == a.L)
          dma_copy(in + (size_t)first * gcol, buf, data_off + p * colB, (uint32_t)cnt * colB, 0, 1, lane, own);
        else
          dma_copy_strided(in + (size_t)first * gcol + (size_t)k0 * R::kCin * sizeof(S), gcol, (uint32_t)cnt, colB,
                           buf, data_off + p * colB, 0, 1, lane, own);
      }
      p += (uint32_t)cnt;
      ++i;
    });
  }
}

// LDS offsets of a node's stencil columns from their tile positions: a
// fixed stride for FP32/FP64, the offset table for BF16.
template <class S, int N>
__device__ __forceinline__ void tile_offsets(const char* lds, uint32_t tab, uint32_t data_off, uint32_t colB,
                                             const uint32_t* pos, uint32_t self, uint32_t* so, uint32_t& xo) {
  if constexpr (sizeof(S) == 2) {
#pragma unroll
    for (int q = 0; q < N; ++q) so[q] = uni(lds_ld<uint32_t>(lds, tab + 4 * pos[q]));
    xo = uni(lds_ld<uint32_t>(lds, tab + 4 * self));
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) so[q] = data_off + pos[q] * colB;
    xo = data_off + self * colB;
  }
}

// One node of a tile (record tn) by one wave, 64 lanes over the levels of
// the chunk: positions and coefficients from the record, then the stencil.
template <class S, int OP, int U>
__device__ __forceinline__ void tile_eval(const TileArgs& a, const char* lds, int32_t tn, uint32_t data_off,
                                          uint32_t colB, int k0, int klc, int lane) {
  using R = TileRec<S, OP>;
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  const uint32_t ro = (uint32_t)tn * R::kBytes;
  const uint32_t obase = uni((uint32_t)lds_ld<int32_t>(lds, ro + R::kIdOff)) * (uint32_t)a.L + (uint32_t)k0;
  uint32_t pos[R::kEntries - 1], self;
  int ne;
  tile_positions<R::kEntries>(lds, ro + R::kCoefB, pos, self, ne);
  uint32_t so[R::kEntries - 1], xo;
  if constexpr (R::kRing2) {
    C w[R::kEntries - 1];
#pragma unroll
    for (int q = 0; q < R::kEntries - 1; ++q) w[q] = lds_ld<C>(lds, ro + q * (uint32_t)sizeof(C));
    if constexpr (R::kGrad) {
      C2 cf[7];
#pragma unroll
      for (int q = 0; q < 7; ++q) cf[q] = lds_ld<C2>(lds, ro + R::kLapB + q * (uint32_t)sizeof(C2));
      if (ne <= 18) {
        tile_offsets<S, 18>(lds, data_off, data_off, colB, pos, self, so, xo);
        tile_node2g<S, U, 18>(a, lds, so, xo, w, cf, obase, klc, lane);
      } else {
        tile_offsets<S, R::kEntries - 1>(lds, data_off, data_off, colB, pos, self, so, xo);
        tile_node2g<S, 1, R::kEntries - 1>(a, lds, so, xo, w, cf, obase, klc, lane);
      }
    } else if (ne <= 18) {
      tile_offsets<S, 18>(lds, data_off, data_off, colB, pos, self, so, xo);
      tile_node2<S, U, 18>(a, lds, so, xo, w, obase, klc, lane);
    } else {
      tile_offsets<S, R::kEntries - 1>(lds, data_off, data_off, colB, pos, self, so, xo);
      tile_node2<S, 1, R::kEntries - 1>(a, lds, so, xo, w, obase, klc, lane);
    }
  } else {
    C2 cf[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) cf[q] = lds_ld<C2>(lds, ro + q * (uint32_t)sizeof(C2));
    const C2 dg = lds_ld<C2>(lds, ro + 7 * (uint32_t)sizeof(C2));
    tile_offsets<S, 7>(lds, data_off, data_off, colB, pos, self, so, xo);
    if constexpr (R::kDual) {
      C2 cf2[7];
#pragma unroll
      for (int q = 0; q < 7; ++q) cf2[q] = lds_ld<C2>(lds, ro + (8 + q) * (uint32_t)sizeof(C2));
      const C2 dg2 = lds_ld<C2>(lds, ro + 15 * (uint32_t)sizeof(C2));
      switch (ne) {
        case 6: tile_node1d<S, U, 6>(a, lds, so, xo, cf, dg, cf2, dg2, obase, klc, lane); break;
        case 5: tile_node1d<S, 1, 5>(a, lds, so, xo, cf, dg, cf2, dg2, obase, klc, lane); break;
        case 7: tile_node1d<S, 1, 7>(a, lds, so, xo, cf, dg, cf2, dg2, obase, klc, lane); break;
        case 4: tile_node1d<S, 1, 4>(a, lds, so, xo, cf, dg, cf2, dg2, obase, klc, lane); break;
        default: tile_node1d<S, 1, 3>(a, lds, so, xo, cf, dg, cf2, dg2, obase, klc, lane); break;
      }
      return;
    }
    switch (ne) {
      case 6: tile_node1<S, OP, U, 6>(a, lds, so, xo, cf, dg, obase, klc, lane); break;
      case 5: tile_node1<S, OP, 1, 5>(a, lds, so, xo, cf, dg, obase, klc, lane); break;
      case 7: tile_node1<S, OP, 1, 7>(a, lds, so, xo, cf, dg, obase, klc, lane); break;
      case 4: tile_node1<S, OP, 1, 4>(a, lds, so, xo, cf, dg, obase, klc, lane); break;
      default: tile_node1<S, OP, 1, 3>(a, lds, so, xo, cf, dg, obase, klc, lane); break;
    }
  }
}

// Tail levels [kt, kt + rem) of all nodes of a tile, rem <= 32: G = 64 / rem
// nodes share a wave, lane = (node j, level t), each lane with its node's
// record (reads within a node group are broadcasts).  The same slot-order
// arithmetic as tile_eval; 1-ring nodes of another degree than 6 in a group
// take the padded seventh slot under a select, so every lane combines
// exactly its own stencil.
template <class S, int OP>
__device__ __forceinline__ void tile_tail(const TileArgs& a, const char* lds, int32_t nnodes, uint32_t data_off,
                                          uint32_t colB, int k0, int kt, int rem, int wave, int W, int lane) {
  using R = TileRec<S, OP>;
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  using X = typename WinT<S, OP>::X;
  constexpr uint32_t kEl = (uint32_t)sizeof(S) * R::kCin;
  constexpr int NE = R::kEntries - 1;
  const int G = 64 / rem;
  const int j = lane / rem, t = lane - j * rem;
  S* __restrict__ out = static_cast<S*>(a.out);
  for (int32_t g0 = wave * G; g0 < nnodes; g0 += W * G) {
    const int32_t tn = g0 + j;
    const bool ok = j < G && tn < nnodes;
    const uint32_t ro = (uint32_t)(ok ? tn : g0) * R::kBytes;
    uint32_t w32[R::kEntries / 2];
#pragma unroll
    for (int q = 0; q < R::kEntries / 8; ++q) {
      const uint4 r = lds_ld<uint4>(lds, ro + R::kCoefB + 16 * q);
      w32[4 * q] = r.x;
      w32[4 * q + 1] = r.y;
      w32[4 * q + 2] = r.z;
      w32[4 * q + 3] = r.w;
    }
    const uint32_t lev = (uint32_t)(kt + t) * kEl;
    auto off = [&](uint32_t pos) -> uint32_t {
      if constexpr (sizeof(S) == 2) return lds_ld<uint32_t>(lds, data_off + 4 * pos) + lev;   // BF16 table
      else return data_off + pos * colB + lev;
    };
    const uint32_t last = w32[R::kEntries / 2 - 1] >> 16;
    const X x0 = lds_elem<S, X>(lds, off(last & ((1u << kLocCountShift) - 1)));
    const int ne = (int)(last >> kLocCountShift);
    const uint32_t o = (uint32_t)lds_ld<int32_t>(lds, ro + R::kIdOff) * (uint32_t)a.L + (uint32_t)(k0 + kt + t);
    if constexpr (R::kRing2) {
      auto run = [&](auto ns) {
        constexpr int NS = decltype(ns)::value;
        C acc = 0, ax = 0, ay = 0;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const uint32_t pos = (q & 1) ? (w32[q >> 1] >> 16) : (w32[q >> 1] & 0xffffu);
          const C d = lds_elem<S, C>(lds, off(pos)) - x0;
          acc = fma(lds_ld<C>(lds, ro + q * (uint32_t)sizeof(C)), d, acc);
          if constexpr (R::kGrad) {
            if (q < 7) {
              const C2 cq = lds_ld<C2>(lds, ro + R::kLapB + q * (uint32_t)sizeof(C2));
              ax = fma(cq.x, d, ax);
              ay = fma(cq.y, d, ay);
            }
          }
        }
        if (ok) {
          if (a.nt) st1<true>(out + (size_t)o, acc);
          else st1<false>(out + (size_t)o, acc);
          if constexpr (R::kGrad) {
            S* og = static_cast<S*>(a.out2) + 2 * (size_t)o;
            if (a.nt) st2<true>(og, ax, ay);
            else st2<false>(og, ax, ay);
          }
        }
      };
      if (__all(!ok || ne <= 18)) run(std::integral_constant<int, 18>());
      else run(std::integral_constant<int, NE>());
    } else {
      X v[7];
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const uint32_t pos = (q & 1) ? (w32[q >> 1] >> 16) : (w32[q >> 1] & 0xffffu);
        v[q] = lds_elem<S, X>(lds, off(pos));
      }
      const bool six = __all(!ok || ne == 6);
      // the sums with the coefficient row at byte cb (8 pairs: 7 slots and
      // the diagonal); per-lane degree: slots past ne leave the sums unchanged
      auto combine = [&](uint32_t cb, C& r0, C& r1) {
        C2 cf[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) cf[q] = lds_ld<C2>(lds, ro + cb + q * (uint32_t)sizeof(C2));
        const C2 dg = lds_ld<C2>(lds, ro + cb + 7 * (uint32_t)sizeof(C2));
        if (six) {
          win_combine<S, OP, 6>(x0, v, cf, dg, r0, r1);
        } else {
          C a0, a1, b0, b1;
          win_combine<S, OP, 3>(x0, v, cf, dg, b0, b1);
#pragma unroll
          for (int d = 4; d <= 7; ++d) {
            if (d == 4) win_combine<S, OP, 4>(x0, v, cf, dg, a0, a1);
            if (d == 5) win_combine<S, OP, 5>(x0, v, cf, dg, a0, a1);
            if (d == 6) win_combine<S, OP, 6>(x0, v, cf, dg, a0, a1);
            if (d == 7) win_combine<S, OP, 7>(x0, v, cf, dg, a0, a1);
            if (ne >= d) {
              b0 = a0;
              b1 = a1;
            }
          }
          r0 = b0;
          r1 = b1;
        }
      };
      C r0, r1;
      combine(0, r0, r1);
      if constexpr (R::kDual) {
        C z0, z1;
        combine(8 * (uint32_t)sizeof(C2), z0, z1);
        if (ok) win_store<S, OP>(static_cast<S*>(a.out2), o, a.nt, z0, z1);
      }
      if (ok) win_store<S, OP>(out, o, a.nt, r0, r1);
    }
  }
}

// Up to 16 waves per workgroup (at most 128 registers per lane), 8 for the
// three-slice FP64 Laplacian and the FP64 one-pass pairs of more than one
// slice per step, which need more registers.
template <class S, int OP, int U>
constexpr int kTileThreads =
    (sizeof(S) == 8 && (((OP == OP_GRADLAP || OP == OP_DIVCURL) && U > 1) || (OP == OP_LAP && U == 3))) ? 512 : 1024;

// A device pointer read from a table, marked as global memory: accesses
// through it compile to global (not flat) instructions, which leave the LDS
// counter alone, so waits for LDS reads never wait for output stores.
template <class T>
__device__ __forceinline__ T* global_ptr(const void* slot) {
  using G = __attribute__((address_space(1))) T*;
  return (T*)(G)ld_const(reinterpret_cast<const uint64_t*>(slot));
}

// Workgroup barrier that orders LDS accesses only: each wave's LDS reads and
// writes are complete before it, and visible after it, but the wave's global
// stores stay in flight (a full __syncthreads() would wait for them too).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One (tile, level chunk) of a field by the W waves of a workgroup: copy into
// LDS, wait, run after_copy() (all waves are past the barrier), evaluate.
// The caller synchronises before the buffer is reused.
template <class S, int OP, int U, class F>
__device__ __forceinline__ void tile_work(const TileArgs& a, int64_t tile, int chunk, char* lds, int W, int wave,
                                          int lane, F&& after_copy) {
  using R = TileRec<S, OP>;
  const int k0 = chunk * a.KL;
  const int klc = a.L - k0 < a.KL ? a.L - k0 : a.KL;
  tile_copy<S, OP>(a, tile, k0, klc, lds, wave, W, lane);
  const int32_t nnodes = ld_uniform(a.info + 4 * tile + 3);
  const uint32_t colB = (uint32_t)klc * R::kCin * (uint32_t)sizeof(S);
  const uint32_t data_off = (uint32_t)nnodes * R::kBytes;   // BF16: the offset table starts here
  __builtin_amdgcn_s_waitcnt(0);   // all counters: the direct loads have landed
  __syncthreads();
  after_copy();
  // compute: node tn of the tile goes to wave tn mod W for whole 64-level
  // slices; a short remainder (1..32 levels) of all nodes is packed G = 64 /
  // rem nodes to a wave
  const int rem = klc & 63;
  const bool pack = rem != 0 && rem <= 32;
  const int kmain = pack ? klc - rem : klc;
  if (kmain > 0)
    for (int32_t tn = wave; tn < nnodes; tn += W) tile_eval<S, OP, U>(a, lds, tn, data_off, colB, k0, kmain, lane);
  if (pack) tile_tail<S, OP>(a, lds, nnodes, data_off, colB, k0, kmain, rem, wave, W, lane);
}

template <class S, int OP, int U>
__global__ __launch_bounds__((kTileThreads<S, OP, U>)) void k_tile(TileArgs a, int64_t nblocks, int remap) {
  extern __shared__ __align__(16) char lds[];
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  const int64_t tile = lb / a.nchunks;
  const int chunk = (int)(lb - tile * a.nchunks);
  const int W = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  tile_work<S, OP, U>(a, tile, chunk, lds, W, wave, lane, [] {});
}

// Persistent form over many fields (tracers) of one operator, each on its
// own tiling (tracers of similar level counts share one).  The work items of
// tracer t are its ntiles_t x nchunks_t (tile, chunk) pairs in tile order;
// XCD x takes the contiguous share [x n_t / 8, (x + 1) n_t / 8) of every
// tracer, so tiles stacked in latitude still meet in one L2, and every XCD
// gets the same mix of long and short columns.  pre[x][t] counts the items of
// share x before tracer t (pre[x][ntr] its total).  The workgroups b with
// b mod 8 = x (the ones the hardware places on XCD x) take the items of share
// x in order from a counter, `claim` consecutive items per claim (tiles
// stacked in latitude, whose shared halo rows the workgroup then finds in
// L2), as they become free, so the tiles in flight on an XCD stay a narrow
// window of the order (a fixed stride lets workgroups drift apart and the
// halo rows they share drop out of L2).  Claims are device-scope atomics,
// which the XCDs' counters serialise; claiming several items at once and
// giving each share's counters a cache line of their own keeps them off the
// critical path, and each workgroup claims once ahead, so a claim's latency
// hides behind a tile's copy.  The last workgroup of share x to finish sets
// both of its counters back to zero for the next launch, so a graph replays
// without a memset.  Each tracer's chunk is its own (at most its tiling's), with the
// slice count of the single-field launch (at most UMAX).  Every wave of a
// workgroup runs the same loop, so the barriers are reached by all.
// Workgroup size bound of the batched kernel: 1024 threads (16 waves), or
// 512 (8 waves, up to 256 registers a lane) for the FP64 divergence pair,
// whose two coefficient rows do not fit in 128 registers.
template <class S, int OP>
constexpr int kBatchedThreads = (sizeof(S) == 8 && OP == OP_DIVCURL) ? 512 : 1024;
inline int batched_max_waves(int kop, int dtype) { return (dtype == DT_F64 && kop == OP_DIVCURL) ? 8 : 16; }

template <class S, int OP, int UMAX>
__global__ __launch_bounds__((kBatchedThreads<S, OP>)) void k_tile_batched(TileArgs base, const BatchTile* __restrict__ tr,
                                                       const int32_t* __restrict__ pre, int ntr,
                                                       int32_t* __restrict__ ctr, int32_t claim) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t next_item;
  const int W = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int x = (int)(blockIdx.x & 7u);
  const int32_t gx = (int32_t)(gridDim.x >> 3);   // the grid is a multiple of 8
  const int32_t* px = pre + (size_t)x * (ntr + 1);
  const int32_t mx = ld_uniform(px + ntr);
  int32_t* cx = ctr + kBatchCtrStride * x;         // claim counter; cx[kBatchCtrStride / 2]: finished
  // Thread 0 holds the end of the current claim and the next claim (`ahead`):
  // a claim made during one claim's items is used only after a later copy has
  // been waited for, which has also waited for the claim, so no evaluation
  // stalls on it.
  int32_t cur_end = 0, ahead = 0;
  if (threadIdx.x == 0) {
    const int32_t c0 = __hip_atomic_fetch_add(cx, claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ahead = __hip_atomic_fetch_add(cx, claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    next_item = c0;
    cur_end = c0 + claim;
  }
  __syncthreads();
  // k is the same in every lane: read it into a scalar register, so the
  // loop and the table loads below stay scalar
  int32_t k = __builtin_amdgcn_readfirstlane(next_item);
  // the current tracer's fields stay in registers: they are loaded again
  // only when the item index moves past the tracer's items (k only grows)
  int t = -1;
  int32_t t_lo = 0, t_hi = 0;   // the tracer's items on this share: [t_lo, t_hi)
  int64_t first = 0;            // its first item index on this share
  int U = 1;
  TileArgs a = base;
  while (k < mx) {
    if (k >= t_hi) {
      do {
        ++t;
        t_hi = ld_uniform(px + t + 1);   // px[ntr] = mx > k ends the scan
      } while (t_hi <= k);
      t_lo = ld_uniform(px + t);
      const BatchTile* d = tr + t;
      a.in = global_ptr<const S>(&d->in);
      a.out = global_ptr<S>(&d->out);
      if constexpr (OP == OP_DIVCURL) a.out2 = global_ptr<S>(&d->out2);
      a.info = reinterpret_cast<const int32_t*>(ld_const(reinterpret_cast<const uint64_t*>(&d->info)));
      a.segs = reinterpret_cast<const int32_t*>(ld_const(reinterpret_cast<const uint64_t*>(&d->segs)));
      a.rec = reinterpret_cast<const char*>(ld_const(reinterpret_cast<const uint64_t*>(&d->rec)));
      a.L = ld_const(&d->L);
      a.KL = ld_const(&d->KL);
      a.nchunks = ld_const(&d->nchunks);
      U = ld_const(&d->U);
      first = (int64_t)x * ld_const(&d->nitems) / 8;
    }
    const int64_t item = first + (k - t_lo);
    const int64_t tile = a.nchunks == 1 ? item : item / a.nchunks;
    const int chunk = (int)(item - tile * a.nchunks);
    // after the copy's wait and barrier (every wave has read next_item):
    // publish the next item, the claim's next or the first of the claim
    // ahead (then claiming another)
    auto advance = [&] {
      if (threadIdx.x == 0) {
        if (k + 1 < cur_end) {
          next_item = k + 1;
        } else {
          next_item = ahead;
          cur_end = ahead + claim;
          ahead = __hip_atomic_fetch_add(cx, claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    };
    // UMAX: the largest slice count of the plan's tracers; only the paths
    // up to it are compiled in, which keeps the kernel's code small
    if (UMAX == 1 || U == 1) tile_work<S, OP, 1>(a, tile, chunk, lds, W, wave, lane, advance);
    else if (UMAX == 2 || U == 2) tile_work<S, OP, (UMAX < 2 ? UMAX : 2)>(a, tile, chunk, lds, W, wave, lane, advance);
    else tile_work<S, OP, UMAX>(a, tile, chunk, lds, W, wave, lane, advance);
    // every wave is done reading the buffer, and next_item is written; the
    // tile's output stores need not have landed
    lds_barrier();
    k = __builtin_amdgcn_readfirstlane(next_item);
  }
  if (threadIdx.x == 0) {
    // every claim of this workgroup (the one ahead included) is complete
    // before its count (release); the last workgroup of the share (acquire)
    // sets both counters back to zero
    int32_t* fin = cx + kBatchCtrStride / 2;
    if (__hip_atomic_fetch_add(fin, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gx - 1) {
      __hip_atomic_store(cx, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(fin, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Packs the node records of a tiling in tile order: record q is node
// order[q]; one thread per dword of the records.
template <class S, int OP>
__global__ __launch_bounds__(256) void k_pack_records(const int32_t* __restrict__ order,
                                                      const void* __restrict__ coef,
                                                      const void* __restrict__ coef2,
                                                      const uint16_t* __restrict__ loc, int64_t V,
                                                      uint32_t* __restrict__ rec) {
  using R = TileRec<S, OP>;
  constexpr uint32_t kDw = R::kBytes / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= V * kDw) return;
  const int64_t q = t / kDw;
  const uint32_t d = (uint32_t)(t - q * kDw);
  const int64_t i = order[q];
  uint32_t v = 0;
  constexpr uint32_t kC1 = R::kGrad ? R::kLapB / 4 : R::kDual ? R::kCoefB / 8 : R::kCoefB / 4;   // from coef
  constexpr uint32_t kC2 = R::kCoefB / 4 - kC1;                       // dwords from coef2
  if (d < kC1) v = static_cast<const uint32_t*>(coef)[i * kC1 + d];
  else if (d < R::kCoefB / 4) v = static_cast<const uint32_t*>(coef2)[i * kC2 + (d - kC1)];
  else if (d < R::kIdOff / 4) v = reinterpret_cast<const uint32_t*>(loc)[i * (R::kLocB / 4) + (d - R::kCoefB / 4)];
  else if (d == R::kIdOff / 4) v = (uint32_t)i;
  rec[t] = v;
}

// ---- persistent LDS tiles, double buffered ------------------------------------
//
// One or two workgroups per CU stay resident and walk their share of the
// tiles.  Producer waves copy tile n+1 into one LDS buffer (direct loads, then
// their own wait) while consumer waves evaluate tile n from the other; one
// barrier per tile swaps the buffers.  Consumers use the lane mapping of the
// gather path: P lanes per node, 64 / P nodes per wave step, lane t handling
// levels t, t + P, ...; each lane reads its node's record from LDS (broadcast
// reads).

// P-lane evaluation of 1-ring nodes from an LDS tile: NS slots (7 = padded
// with the node itself and zero coefficients).
template <class S, int OP, int NS, int U>
__device__ __forceinline__ void tile_lanes1(const TileArgs& a, const char* buf, uint32_t data_off, uint32_t colB,
                                            const uint32_t* so, uint32_t xo, const typename Traits<S>::C2* cf,
                                            typename Traits<S>::C2 dg, uint32_t obase, bool ok, int t, int P,
                                            int klc) {
  using C = typename Traits<S>::C;
  using X = typename WinT<S, OP>::X;
  S* __restrict__ out = static_cast<S*>(a.out);
  const int nsl = (klc + P - 1) / P;
  for (int r0 = 0; r0 < nsl; r0 += U) {
    X v[U][NS], x0[U];
    bool st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = t + P * (r0 + u);
      st[u] = ok && k < klc;
      const uint32_t kk = (uint32_t)(k < klc ? k : klc - 1) * (uint32_t)sizeof(X);
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = lds_ld<X>(buf, so[s] + kk);
      x0[u] = lds_ld<X>(buf, xo + kk);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      win_emit<S, OP, NS>(out, obase + (uint32_t)(t + P * (r0 + u)), st[u], a.nt, x0[u], v[u], cf, dg);
  }
}

template <class S, int NS, int U>
__device__ __forceinline__ void tile_lanes2(const TileArgs& a, const char* buf, const uint32_t* so, uint32_t xo,
                                            const typename Traits<S>::C* w, uint32_t obase, bool ok, int t, int P,
                                            int klc) {
  using C = typename Traits<S>::C;
  S* __restrict__ out = static_cast<S*>(a.out);
  const int nsl = (klc + P - 1) / P;
  for (int r0 = 0; r0 < nsl; r0 += U) {
    C v[U][NS], x0[U];
    bool st[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = t + P * (r0 + u);
      st[u] = ok && k < klc;
      const uint32_t kk = (uint32_t)(k < klc ? k : klc - 1) * (uint32_t)sizeof(C);
#pragma unroll
      for (int s = 0; s < NS; ++s) v[u][s] = lds_ld<C>(buf, so[s] + kk);
      x0[u] = lds_ld<C>(buf, xo + kk);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      C acc = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = fma(w[s], v[u][s] - x0[u], acc);
      if (st[u]) {
        const uint32_t o = obase + (uint32_t)(t + P * (r0 + u));
        if (a.nt) st1<true>(out + (size_t)o, acc);
        else st1<false>(out + (size_t)o, acc);
      }
    }
  }
}

template <class S, int OP, int U>
__device__ __forceinline__ void tile_consume(const TileArgs& a, int64_t lb, const char* buf, int cw, int NC, int P,
                                             int lane) {
  using R = TileRec<S, OP>;
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  const int64_t tile = lb / a.nchunks;
  const int chunk = (int)(lb - tile * a.nchunks);
  const int32_t nnodes = ld_uniform(a.info + 4 * tile + 3);
  const int k0 = chunk * a.KL;
  const int klc = a.L - k0 < a.KL ? a.L - k0 : a.KL;
  const uint32_t colB = (uint32_t)klc * R::kCin * (uint32_t)sizeof(S);   // LDS column stride (this chunk)
  const uint32_t data_off = (uint32_t)nnodes * R::kBytes;
  if (P == 64) {   // one node per wave, as in the one-tile form
    for (int32_t tn = cw; tn < nnodes; tn += NC) tile_eval<S, OP, U>(a, buf, tn, data_off, colB, k0, klc, lane);
    return;
  }
  const int G = 64 / P;
  const int j = lane / P, t = lane - (lane / P) * P;
  for (int32_t tn0 = cw * G; tn0 < nnodes; tn0 += NC * G) {
    const int32_t tn = tn0 + j;
    const bool ok = j < G && tn < nnodes;
    const uint32_t ro = (uint32_t)(ok ? tn : tn0) * R::kBytes;
    const int32_t i = lds_ld<int32_t>(buf, ro + R::kIdOff);
    const uint32_t obase = (uint32_t)i * (uint32_t)a.L + (uint32_t)k0;
    uint32_t w32[R::kEntries / 2];
#pragma unroll
    for (int q = 0; q < R::kEntries / 8; ++q) {
      const uint4 r = lds_ld<uint4>(buf, ro + R::kCoefB + 16 * q);
      w32[4 * q] = r.x;
      w32[4 * q + 1] = r.y;
      w32[4 * q + 2] = r.z;
      w32[4 * q + 3] = r.w;
    }
    uint32_t so[R::kEntries - 1];
#pragma unroll
    for (int q = 0; q < R::kEntries - 1; ++q)
      so[q] = data_off + ((q & 1) ? (w32[q >> 1] >> 16) : (w32[q >> 1] & 0xffffu)) * colB;
    const uint32_t last = w32[R::kEntries / 2 - 1] >> 16;
    const uint32_t xo = data_off + (last & ((1u << kLocCountShift) - 1)) * colB;
    const int ne = (int)(last >> kLocCountShift);
    if constexpr (R::kRing2) {
      C w[R::kEntries - 1];
#pragma unroll
      for (int q = 0; q < R::kEntries - 1; ++q) w[q] = lds_ld<C>(buf, ro + q * (uint32_t)sizeof(C));
      if (__all(ne <= 18)) tile_lanes2<S, 18, U>(a, buf, so, xo, w, obase, ok, t, P, klc);
      else tile_lanes2<S, R::kEntries - 1, 1>(a, buf, so, xo, w, obase, ok, t, P, klc);
    } else {
      C2 cf[7];
#pragma unroll
      for (int q = 0; q < 7; ++q) cf[q] = lds_ld<C2>(buf, ro + q * (uint32_t)sizeof(C2));
      const C2 dg = lds_ld<C2>(buf, ro + 7 * (uint32_t)sizeof(C2));
      if (__all(ne == 6)) tile_lanes1<S, OP, 6, U>(a, buf, data_off, colB, so, xo, cf, dg, obase, ok, t, P, klc);
      else tile_lanes1<S, OP, 7, 1>(a, buf, data_off, colB, so, xo, cf, dg, obase, ok, t, P, klc);
    }
  }
}

// Up to 16 waves per workgroup for 4-byte data (at most 128 registers per
// lane), 8 for FP64, whose two-ring variant needs more registers.
template <class S>
constexpr int kTile2Threads = sizeof(S) == 8 ? 512 : 1024;

// Copy of logical block lb (tile, level chunk) by the NP producer waves.
template <class S, int OP>
__device__ __forceinline__ void tile_issue(const TileArgs& a, int64_t lb, char* buf, int pw, int NP, int lane) {
  const int64_t tile = lb / a.nchunks;
  const int chunk = (int)(lb - tile * a.nchunks);
  const int k0 = chunk * a.KL;
  const int klc = a.L - k0 < a.KL ? a.L - k0 : a.KL;
  tile_copy<S, OP>(a, tile, k0, klc, buf, pw, NP, lane);
}

template <class S, int OP, int U>
__global__ __launch_bounds__(kTile2Threads<S>) void k_tile2(TileArgs a, int64_t nblocks, int remap, uint32_t buf_bytes, int nprod,
                                               int P) {
  extern __shared__ __align__(16) char lds[];
  const int W = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // this workgroup's tiles: with remapping, the workgroups of one XCD sweep
  // a contiguous eighth of the tile list together
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  int64_t lb, step, end;
  if (remap) {
    const int64_t per = (nblocks + 7) / 8;
    lb = (b % 8) * per + b / 8;
    step = nwg / 8;
    end = (b % 8 + 1) * per < nblocks ? (b % 8 + 1) * per : nblocks;
  } else {
    lb = b;
    step = nwg;
    end = nblocks;
  }
  const bool producer = wave < nprod;
  uint32_t cur = 0;
  if (producer && lb < end) {
    tile_issue<S, OP>(a, lb, lds, wave, nprod, lane);
    __builtin_amdgcn_s_waitcnt(0);   // all counters: the direct loads have landed
  }
  __syncthreads();
  while (lb < end) {
    const int64_t nx = lb + step;
    if (producer) {
      if (nx < end) {
        tile_issue<S, OP>(a, nx, lds + (cur ^ buf_bytes), wave, nprod, lane);
        __builtin_amdgcn_s_waitcnt(0);   // all counters: the direct loads have landed
      }
    } else {
      tile_consume<S, OP, U>(a, lb, lds + cur, wave - nprod, W - nprod, P, lane);
    }
    // LDS traffic of this step done (consumer reads, producer index stores;
    // the producers' direct loads were waited for above); consumers' global
    // stores may stay in flight across the barrier
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    lb = nx;
    cur ^= buf_bytes;
  }
}

// ---- remapping: out[t][k] = w0 f[n0][k] + w1 f[n1][k] + w2 f[n2][k] ---------------
//
// Linear interpolation over the source triangle of each target point
// (Section 4.3).  A wave serves 64 / P lane groups, P lanes each (P = nlev
// for columns of at most 32 levels, else 64), and each group TP consecutive
// target points, lane t of a group taking levels t, t + P, ...; the node
// indices and weights of the TP points and then U level slices of all their
// source columns are loaded before the arithmetic (more loads in flight for
// the 4- and 2-byte types).  Blocks are remapped so that each XCD walks a
// contiguous range of target points (whose source columns are neighbours, so
// they stay in that XCD's L2).  The sum is w0 f0, then + w1 f1, then + w2 f2,
// with fused multiply-adds.  With O32 the input is addressed by 32-bit byte
// offsets from its base (the launch checks that it is under 4 GiB); with
// EXACT (64 lanes, U = the column's 64-level slices) every slice but the
// last lies inside the column, at a constant offset from the first.
template <class S, int U, int TP, bool O32 = false, bool EXACT = false>
__global__ __launch_bounds__(256) void k_remap(const int32_t* __restrict__ nodes, const void* __restrict__ wv,
                                               const S* __restrict__ in, S* __restrict__ out, int64_t P, int L,
                                               int lanes, int64_t nblocks, int remap) {
  using C = typename Traits<S>::C;
  const C* __restrict__ w = static_cast<const C*>(wv);
  const char* __restrict__ inb = reinterpret_cast<const char*>(in);
  const uint32_t colB = (uint32_t)L * (uint32_t)sizeof(S);
  auto src = [&](int32_t node, int k) -> const S* {
    if constexpr (O32) return reinterpret_cast<const S*>(inb + ((uint32_t)node * colB + (uint32_t)k * (uint32_t)sizeof(S)));
    else return in + (size_t)node * (size_t)L + k;
  };
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  const int W = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int G = 64 / lanes;
  const int j = lane / lanes, tl = lane - j * lanes;
  if (j >= G) return;   // idle lanes; the kernel has no barrier
  const int64_t t0 = ((lb * W + wave) * G + j) * TP;
  if (t0 >= P) return;
  int4 nd[TP];
  C w0[TP], w1[TP], w2[TP];
#pragma unroll
  for (int q = 0; q < TP; ++q) {
    const int64_t t = t0 + q < P ? t0 + q : P - 1;   // past the last point: reload it, store nothing
    nd[q] = *reinterpret_cast<const int4*>(nodes + 4 * t);
    w0[q] = w[4 * t];
    w1[q] = w[4 * t + 1];
    w2[q] = w[4 * t + 2];
  }
  for (int k0 = tl; k0 < L; k0 += lanes * U) {
    C v0[TP][U], v1[TP][U], v2[TP][U];
#pragma unroll
    for (int q = 0; q < TP; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (EXACT && u < U - 1) {
          v0[q][u] = ld1(src(nd[q].x, k0) + 64 * u);
          v1[q][u] = ld1(src(nd[q].y, k0) + 64 * u);
          v2[q][u] = ld1(src(nd[q].z, k0) + 64 * u);
        } else {
          const int k = k0 + lanes * u;
          const int kc = k < L ? k : L - 1;
          v0[q][u] = ld1(src(nd[q].x, kc));
          v1[q][u] = ld1(src(nd[q].y, kc));
          v2[q][u] = ld1(src(nd[q].z, kc));
        }
      }
    // every sum is formed before the guarded stores (keep), so the compiler
    // cannot sink the loads of a partial last slice into the store's branch,
    // where they would issue late and wait for all loads in flight
    C r[TP][U];
#pragma unroll
    for (int q = 0; q < TP; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        C acc = w0[q] * v0[q][u];
        acc = fma(w1[q], v1[q][u], acc);
        r[q][u] = fma(w2[q], v2[q][u], acc);
        keep(r[q][u]);
      }
#pragma unroll
    for (int q = 0; q < TP; ++q)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + lanes * u;
        if (k < L && t0 + q < P) st1<false>(out + (size_t)(t0 + q) * (size_t)L + k, r[q][u]);
      }
  }
}

template <class S, int U, int TP>
void launch_remap_u(dim3 g, dim3 b, hipStream_t st, const int32_t* nodes, const void* w, const S* src, S* dst,
                    int64_t V, int64_t P, int nlev, int lanes, int64_t nblocks) {
  const bool o32 = (uint64_t)V * (uint64_t)nlev * sizeof(S) < (1ull << 32);
  const bool exact = lanes == 64 && (nlev + 63) / 64 == U;
  if (o32 && exact)
    hipLaunchKernelGGL((k_remap<S, U, TP, true, true>), g, b, 0, st, nodes, w, src, dst, P, nlev, lanes, nblocks, 1);
  else if (o32)
    hipLaunchKernelGGL((k_remap<S, U, TP, true, false>), g, b, 0, st, nodes, w, src, dst, P, nlev, lanes, nblocks, 1);
  else
    hipLaunchKernelGGL((k_remap<S, U, TP>), g, b, 0, st, nodes, w, src, dst, P, nlev, lanes, nblocks, 1);
}

template <class S, int TP>
hipError_t launch_remap_tp(const int32_t* nodes, const void* w, int64_t V, int64_t P, int nlev, const S* src,
                           S* dst, hipStream_t st) {
  const int lanes = nlev <= 32 ? nlev : 64;
  const int G = 64 / lanes;
  constexpr int W = 4;
  const int64_t groups = (P + (int64_t)G * TP - 1) / ((int64_t)G * TP);
  const int64_t nblocks = (groups + W - 1) / W;
  const int64_t grid = (nblocks + 7) / 8 * 8;
  const int nsl = (nlev + lanes - 1) / lanes;
  const int U = nsl < 3 ? nsl : 3;
  const dim3 g((unsigned)grid), b(64 * W);
  switch (U) {
    case 1: launch_remap_u<S, 1, TP>(g, b, st, nodes, w, src, dst, V, P, nlev, lanes, nblocks); break;
    case 2: launch_remap_u<S, 2, TP>(g, b, st, nodes, w, src, dst, V, P, nlev, lanes, nblocks); break;
    default: launch_remap_u<S, 3, TP>(g, b, st, nodes, w, src, dst, V, P, nlev, lanes, nblocks); break;
  }
  return hipGetLastError();
}

// Target points per lane group (measured at O1280 x 137 -> F640): one for
// FP64, two (columns of at most 32 levels) or four for 4- and 2-byte data.
template <class S>
hipError_t launch_remap_t(const int32_t* nodes, const void* w, int64_t V, int64_t P, int nlev, const void* in,
                          void* out, hipStream_t st) {
  const S* src = static_cast<const S*>(in);
  S* dst = static_cast<S*>(out);
  if constexpr (sizeof(S) == 8) return launch_remap_tp<S, 1>(nodes, w, V, P, nlev, src, dst, st);
  else if (nlev <= 32) return launch_remap_tp<S, 2>(nodes, w, V, P, nlev, src, dst, st);
  else return launch_remap_tp<S, 4>(nodes, w, V, P, nlev, src, dst, st);
}

// Transpose of the remapping: fbar[n][k] = the sum over the entries (t, w)
// of source node n, in ascending target order, of w ybar[t][k] (fused
// multiply-adds from zero; 0 for nodes no target point uses).  A group of P
// lanes serves one node (64 / P nodes per wave).  Lane tl keeps VEC
// consecutive levels of each of NS slices of P VEC levels in registers
// (levels kb + VEC tl + P VEC s + c), so each entry's target index and
// weight are read once per block of levels; with VEC = 2 (FP64) a column is
// read with 16-byte loads where the lane's two levels lie inside it (element
// loads at its end).  A node's row bounds and first two entries (kept beside
// the compressed rows) are read together; entries go two at a time: both
// target columns are loaded together and the next pair's indices and
// weights are requested before the multiply-adds of this pair, which are
// taken in entry order.  With O32 the input is addressed by 32-bit byte
// offsets from its base (the launch checks that it is smaller than 4 GiB).
// With STG (whole columns in one block) the wave's G consecutive output
// columns are staged in LDS and written as one contiguous run in units of
// `unit` bytes: measured 15-20 % faster than the groups' own 64-byte pieces.
typedef double f64x2_e __attribute__((ext_vector_type(2), aligned(8)));   // two levels, element-aligned
template <class S, int VEC>
struct VecOf {
  using T = S;
};
template <>
struct VecOf<double, 2> {
  using T = f64x2_e;
};

template <class S, int NS, int VEC, bool O32, bool STG, bool EXACT = false>
__global__ __launch_bounds__(256) void k_remap_adj(const int64_t* __restrict__ off, const int32_t* __restrict__ tt,
                                                   const void* __restrict__ wv, const int32_t* __restrict__ ht,
                                                   const void* __restrict__ hwv, const S* __restrict__ in,
                                                   S* __restrict__ out, int64_t V, int L, int lanes, int64_t nblocks,
                                                   int remap, int unit) {
  using C = typename Traits<S>::C;
  using C2 = typename Traits<S>::C2;
  using VT = typename VecOf<S, VEC>::T;
  constexpr int EB = 2;
  extern __shared__ __align__(16) char smem[];
  const C* __restrict__ w = static_cast<const C*>(wv);
  const C* __restrict__ hw = static_cast<const C*>(hwv);
  const int64_t lb = logical_block(blockIdx.x, nblocks, remap);
  if (lb >= nblocks) return;
  const int W = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int G = 64 / lanes;
  const int j = lane / lanes, tl = lane - j * lanes;
  const int64_t nw0 = (lb * W + wave) * G;   // the wave's first node
  const int64_t n = nw0 + j;
  // idle lanes (past the node groups or the nodes) stay to the end: with STG
  // every wave reaches the barrier
  const bool act = j < G && n < V;
  if (!STG && !act) return;
  const char* __restrict__ inb = reinterpret_cast<const char*>(in);
  const uint32_t colB = (uint32_t)L * (uint32_t)sizeof(S);
  int64_t e0 = 0, e1 = 0;
  int2 h2 = make_int2(0, 0);
  C2 hw2;
  hw2.x = 0;
  hw2.y = 0;
  if (act) {
    e0 = off[n];
    e1 = off[n + 1];
    h2 = *reinterpret_cast<const int2*>(ht + 2 * n);
    hw2 = *reinterpret_cast<const C2*>(hw + 2 * n);
  }
  S* __restrict__ o = out + (size_t)n * (size_t)L;
  S* __restrict__ sb = reinterpret_cast<S*>(smem) + (size_t)wave * G * L;
  for (int kb = VEC * tl; kb < L + VEC * tl; kb += lanes * VEC * NS) {
    int kl[NS];   // first level of the lane's VEC levels in slice s
#pragma unroll
    for (int s = 0; s < NS; ++s) kl[s] = kb + lanes * VEC * s;
    auto addr = [&](int32_t t, int k) -> const S* {
      if constexpr (O32) return reinterpret_cast<const S*>(inb + ((uint32_t)t * colB + (uint32_t)k * (uint32_t)sizeof(S)));
      else return reinterpret_cast<const S*>(inb + ((size_t)t * colB + (size_t)k * sizeof(S)));
    };
    // the lane's VEC levels of slice s of column t: one 16-byte load inside
    // the column, else element loads (past the column: its last level, not
    // stored)
    auto load = [&](int32_t t, int s, C* v) {
      const int k = kl[s];
      if (EXACT && s < NS - 1) {
        // EXACT: 16 lanes and NS = ceil(L / (16 VEC)), so every slice but the
        // last lies inside the column; its address is the first slice's plus
        // a constant (an immediate offset of the load)
        const S* p0 = addr(t, kb) + 16 * VEC * s;
        if constexpr (VEC == 1) {
          v[0] = ld1(p0);
        } else {
          const VT x = *reinterpret_cast<const VT*>(p0);
          v[0] = x.x;
          v[1] = x.y;
        }
      } else if (VEC == 1 || k + VEC <= L) {
        if constexpr (VEC == 1) {
          v[0] = ld1(addr(t, k < L ? k : L - 1));
        } else {
          const VT x = *reinterpret_cast<const VT*>(addr(t, k));
          v[0] = x.x;
          v[1] = x.y;
        }
      } else {
#pragma unroll
        for (int c = 0; c < VEC; ++c) v[c] = ld1(addr(t, k + c < L ? k + c : L - 1));
      }
    };
    C acc[NS][VEC];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[s][c] = 0;
    int32_t tn[EB] = {h2.x, h2.y};
    C wn[EB] = {hw2.x, hw2.y};
    for (int64_t e = e0; e < e1; e += EB) {
      int32_t t[EB];
      C wq[EB];
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        t[q] = tn[q];
        wq[q] = wn[q];
      }
      C v[EB][NS][VEC];
#pragma unroll
      for (int q = 0; q < EB; ++q)
        if (e + q < e1) {
#pragma unroll
          for (int s = 0; s < NS; ++s) load(t[q], s, v[q][s]);
        }
      if (e + EB < e1) {
#pragma unroll
        for (int q = 0; q < EB; ++q) {
          const int64_t eq = e + EB + q < e1 ? e + EB + q : e1 - 1;
          tn[q] = tt[eq];
          wn[q] = w[eq];
        }
      }
#pragma unroll
      for (int q = 0; q < EB; ++q)
        if (e + q < e1) {
#pragma unroll
          for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < VEC; ++c) acc[s][c] = fma(wq[q], v[q][s][c], acc[s][c]);
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        const int k = kl[s] + c;
        if constexpr (STG) {
          if (act && k < L) st1<false>(sb + j * L + k, acc[s][c]);
        } else {
          if (k < L) st1<false>(o + k, acc[s][c]);
        }
      }
  }
  if constexpr (STG) {
    __syncthreads();
    const int cnt = (V - nw0 < G ? (int)(V - nw0) : G) * L;   // elements of the wave's run
    S* __restrict__ ob = out + (size_t)nw0 * (size_t)L;
    // whole units of `unit` bytes (16, 8 or 4; both ends of every full run
    // and the output are aligned to it), then the elements past the last one
    auto copy = [&](auto tag) {
      using T = decltype(tag);
      const int nu = cnt * (int)sizeof(S) / (int)sizeof(T);
      T* __restrict__ d = reinterpret_cast<T*>(ob);
      const T* __restrict__ q = reinterpret_cast<const T*>(sb);
      for (int i = lane; i < nu; i += 64) d[i] = q[i];
      return nu * (int)sizeof(T) / (int)sizeof(S);
    };
    int done;
    if (unit == 16) done = copy(uint4());
    else if (unit == 8) done = copy(uint2());
    else if (unit == 4) done = copy(uint32_t());
    else done = copy(S());
    for (int i = done + lane; i < cnt; i += 64) ob[i] = sb[i];
  }
}

template <class S, int NS, int VEC>
hipError_t launch_remap_adj_ns(const int64_t* off, const int32_t* tt, const void* w, const int32_t* ht, const void* hw,
                               int64_t V, int64_t P, int nlev, int lanes, const S* src, S* dst, hipStream_t st) {
  const int G = 64 / lanes;
  constexpr int W = 4;
  const int64_t groups = (V + G - 1) / G;
  const int64_t nblocks = (groups + W - 1) / W;
  const int64_t grid = (nblocks + 7) / 8 * 8;
  const bool o32 = (uint64_t)P * (uint64_t)nlev * sizeof(S) < (1ull << 32);
  const size_t lds = (size_t)W * G * nlev * sizeof(S);
  const bool stage = nlev <= lanes * VEC * NS && lds <= 32768;
  // the widest store unit that divides a full run's bytes and the output's alignment
  const uint64_t run = (uint64_t)G * nlev * sizeof(S), addr = (uint64_t)(uintptr_t)dst;
  int unit = (int)sizeof(S);
  for (int u : {16, 8, 4})
    if (u > unit && run % u == 0 && addr % u == 0) {
      unit = u;
      break;
    }
  const dim3 g((unsigned)grid), b(64 * W);
  // 16 lanes with exactly the slices the column needs: constant slice
  // offsets (4- and 2-byte data; measured 3 % and 8 % faster at O1280 x 137
  // <- F640, but 6 % slower for the FP64 16-byte loads)
  const bool exact = VEC == 1 && lanes == 16 && (nlev + 15) / 16 == NS;
#define RADJ_LAUNCH(O, T)                                                                                             \
  hipLaunchKernelGGL((k_remap_adj<S, NS, VEC, O, T>), g, b, T ? lds : 0, st, off, tt, w, ht, hw, src, dst, V, nlev, \
                     lanes, nblocks, 1, unit)
  if (o32 && stage && exact) {
    hipLaunchKernelGGL((k_remap_adj<S, NS, VEC, true, true, true>), g, b, lds, st, off, tt, w, ht, hw, src, dst, V,
                       nlev, lanes, nblocks, 1, unit);
  } else if (o32) {
    if (stage) RADJ_LAUNCH(true, true);
    else RADJ_LAUNCH(true, false);
  } else {
    if (stage) RADJ_LAUNCH(false, true);
    else RADJ_LAUNCH(false, false);
  }
#undef RADJ_LAUNCH
  return hipGetLastError();
}

// One node per 16 lanes (fewer columns of at most 16 levels: one lane per
// level); FP64 columns of more than 32 levels are read two levels per lane
// (16-byte loads; FP32 columns, only 4-byte aligned, measured slower that
// way).  Measured at O1280 x 137 <- F640.
template <class S>
hipError_t launch_remap_adj_t(const int64_t* off, const int32_t* tt, const void* w, const int32_t* ht, const void* hw,
                              int64_t V, int64_t P, int nlev, const void* in, void* out, hipStream_t st) {
  const int lanes = nlev <= 16 ? nlev : 16;
  const S* src = static_cast<const S*>(in);
  S* dst = static_cast<S*>(out);
  if constexpr (sizeof(S) == 8) {
    if (nlev > 32) {
      const int ns = (nlev + 2 * lanes - 1) / (2 * lanes);
      if (ns <= 2) return launch_remap_adj_ns<S, 2, 2>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
      if (ns == 3) return launch_remap_adj_ns<S, 3, 2>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
      return launch_remap_adj_ns<S, 5, 2>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
    }
  }
  const int ns = (nlev + lanes - 1) / lanes;
  if (ns <= 1) return launch_remap_adj_ns<S, 1, 1>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
  if (ns == 2) return launch_remap_adj_ns<S, 2, 1>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
  if (ns == 3) return launch_remap_adj_ns<S, 3, 1>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
  if (ns <= 5) return launch_remap_adj_ns<S, 5, 1>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
  return launch_remap_adj_ns<S, 9, 1>(off, tt, w, ht, hw, V, P, nlev, lanes, src, dst, st);
}

// ---- conservation: fixed-order FP64 sums of V_i div_ik --------------------------
//
// Workgroup b reduces nodes [b*chunk, (b+1)*chunk) for every level.  Wave w
// takes nodes w, w + W, ... of the chunk and reads each node's column in one
// go (lane = level within a 256-level block, four 64-level slices), so every
// column is fetched once; waves are then combined in order through LDS and a
// second pass sums the workgroup partials in order.  Deterministic by
// construction.

constexpr int kConsWaves = 4;
constexpr int kConsBlockLevels = 256;

template <class S, int NSL>
__global__ __launch_bounds__(64 * kConsWaves) void k_cons_partial(const S* __restrict__ div,
                                                                  const double* __restrict__ vol, int64_t V,
                                                                  int L, int64_t chunk, double* __restrict__ part) {
  // NSL: 64-level slices of a 256-level block that hold levels (the last
  // block of a short column needs fewer); nodes are read four at a time and
  // added in node order, so every sum keeps its order
  constexpr int kNodes = 4;
  __shared__ double red[kConsWaves][kConsBlockLevels][2];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t n0 = (int64_t)blockIdx.x * chunk;
  const int64_t n1 = n0 + chunk < V ? n0 + chunk : V;
  for (int kb = 0; kb < L; kb += kConsBlockLevels) {
    double s[4] = {0.0, 0.0, 0.0, 0.0}, ab[4] = {0.0, 0.0, 0.0, 0.0};
    bool in[4];
    int kc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = kb + lane + 64 * r;
      in[r] = k < L;
      kc[r] = k < L ? k : L - 1;
    }
    // slices this block needs (all four unless it is the column's last)
    const int nsl = L - kb >= kConsBlockLevels ? 4 : NSL;
    int64_t i = n0 + wave;
    for (; i + (kNodes - 1) * kConsWaves < n1; i += kNodes * kConsWaves) {
      double p[kNodes][4];
#pragma unroll
      for (int q = 0; q < kNodes; ++q) {
        const int64_t nd = i + q * kConsWaves;
        const double v = vol[nd];
        const S* col = div + nd * (int64_t)L;
#pragma unroll
        for (int r = 0; r < 4; ++r) p[q][r] = r < nsl ? v * (double)ld1(col + kc[r]) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kNodes; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r < nsl && in[r]) {
            s[r] += p[q][r];
            ab[r] += fabs(p[q][r]);
          }
    }
    for (; i < n1; i += kConsWaves) {
      const double v = vol[i];
      const S* col = div + i * (int64_t)L;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r < nsl && in[r]) {
          const double p = v * (double)ld1(col + kc[r]);
          s[r] += p;
          ab[r] += fabs(p);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[wave][lane + 64 * r][0] = s[r];
      red[wave][lane + 64 * r][1] = ab[r];
    }
    __syncthreads();
    const int k = kb + (int)threadIdx.x;
    if (threadIdx.x < kConsBlockLevels && k < L) {
      double ts = red[0][threadIdx.x][0], ta = red[0][threadIdx.x][1];
      for (int w = 1; w < kConsWaves; ++w) {
        ts += red[w][threadIdx.x][0];
        ta += red[w][threadIdx.x][1];
      }
      part[((int64_t)blockIdx.x * L + k) * 2] = ts;
      part[((int64_t)blockIdx.x * L + k) * 2 + 1] = ta;
    }
    __syncthreads();
  }
}

// One workgroup per level: thread t sums partials t, t + 256, ... in order,
// then a fixed binary tree combines the 256 thread sums.
__global__ __launch_bounds__(256) void k_cons_final(const double* __restrict__ part, int nparts, int L,
                                                    double* __restrict__ out_sum, double* __restrict__ out_abs) {
  __shared__ double red[256][2];
  const int k = blockIdx.x;
  double s = 0.0, a = 0.0;
  for (int p = threadIdx.x; p < nparts; p += 256) {
    s += part[((int64_t)p * L + k) * 2];
    a += part[((int64_t)p * L + k) * 2 + 1];
  }
  red[threadIdx.x][0] = s;
  red[threadIdx.x][1] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x][0] += red[threadIdx.x + w][0];
      red[threadIdx.x][1] += red[threadIdx.x + w][1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out_sum[k] = red[0][0];
    out_abs[k] = red[0][1];
  }
}

// ---- dispatch ---------------------------------------------------------------

Args make_args(int op, const DevTables& t, const NodeOrder& ord, int64_t V, int nlev, const void* in, void* out,
               const Shape& sh) {
  Args a;
  a.order = ord.order;
  a.runs = ord.runs;
  a.nruns = ord.nruns;
  if (op == OP_LAP) {
    a.nbr = t.lap_nbr;
    a.coef = t.lap_w;
  } else {
    a.nbr = t.nbr8;
    a.coef = t.coef[op];
  }
  a.in = in;
  a.out = out;
  a.V = V;
  a.L = nlev;
  a.P = lanes_per_node(nlev, sh);
  a.npw = sh.nodes_per_wave;
  a.nt = nt_of(sh) ? 1 : 0;
  return a;
}

template <class S, int OP>
hipError_t launch_win(const Args& a, int U, dim3 g, dim3 b, int64_t nblocks, int remap, hipStream_t st) {
  switch (U) {
    case 1: hipLaunchKernelGGL((k_win<S, OP, 1>), g, b, 0, st, a, nblocks, remap); break;
    case 2: hipLaunchKernelGGL((k_win<S, OP, 2>), g, b, 0, st, a, nblocks, remap); break;
    default: hipLaunchKernelGGL((k_win<S, OP, 3>), g, b, 0, st, a, nblocks, remap); break;
  }
  return hipGetLastError();
}

template <class S, int OP>
hipError_t launch_u(const Args& a, int U, dim3 g, dim3 b, int64_t nblocks, int remap, hipStream_t st) {
  switch (U) {
    case 1: hipLaunchKernelGGL((k_op<S, OP, 1>), g, b, 0, st, a, nblocks, remap); break;
    case 2: hipLaunchKernelGGL((k_op<S, OP, 2>), g, b, 0, st, a, nblocks, remap); break;
    default: hipLaunchKernelGGL((k_op<S, OP, 3>), g, b, 0, st, a, nblocks, remap); break;
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_op_t(int op, const Args& a, int U, int64_t nblocks, bool window, const Shape& sh,
                       hipStream_t st) {
  const int64_t grid = sh.xcd_remap ? (nblocks + 7) / 8 * 8 : nblocks;
  const dim3 g((unsigned)grid), b((unsigned)(64 * sh.waves_per_block));
  if (window) {
    switch (op) {
      case OP_GRAD: return launch_win<S, OP_GRAD>(a, U, g, b, nblocks, sh.xcd_remap, st);
      case OP_DIV: return launch_win<S, OP_DIV>(a, U, g, b, nblocks, sh.xcd_remap, st);
      case OP_GRADT: return launch_win<S, OP_GRADT>(a, U, g, b, nblocks, sh.xcd_remap, st);
      case OP_DIVT: return launch_win<S, OP_DIVT>(a, U, g, b, nblocks, sh.xcd_remap, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (op) {
    case OP_GRAD: return launch_u<S, OP_GRAD>(a, U, g, b, nblocks, sh.xcd_remap, st);
    case OP_DIV: return launch_u<S, OP_DIV>(a, U, g, b, nblocks, sh.xcd_remap, st);
    case OP_GRADT: return launch_u<S, OP_GRADT>(a, U, g, b, nblocks, sh.xcd_remap, st);
    case OP_DIVT: return launch_u<S, OP_DIVT>(a, U, g, b, nblocks, sh.xcd_remap, st);
    case OP_LAP: return launch_u<S, OP_LAP>(a, U, g, b, nblocks, sh.xcd_remap, st);
    default: return hipErrorInvalidValue;
  }
}

template <class S, int OP>
hipError_t launch_tile_u(const TileArgs& a, int U, dim3 g, dim3 b, uint32_t lds, int64_t nblocks, int remap,
                         hipStream_t st) {
  const int maxt = U == 1 ? kTileThreads<S, OP, 1> : U == 2 ? kTileThreads<S, OP, 2> : kTileThreads<S, OP, 3>;
  if ((int)b.x > maxt) b.x = (unsigned)maxt;
  if (lds > 65536) {
    const void* fn = U == 1 ? reinterpret_cast<const void*>(&k_tile<S, OP, 1>)
                     : U == 2 ? reinterpret_cast<const void*>(&k_tile<S, OP, 2>)
                              : reinterpret_cast<const void*>(&k_tile<S, OP, 3>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  switch (U) {
    case 1: hipLaunchKernelGGL((k_tile<S, OP, 1>), g, b, lds, st, a, nblocks, remap); break;
    case 2: hipLaunchKernelGGL((k_tile<S, OP, 2>), g, b, lds, st, a, nblocks, remap); break;
    default: hipLaunchKernelGGL((k_tile<S, OP, 3>), g, b, lds, st, a, nblocks, remap); break;
  }
  return hipGetLastError();
}

template <class S, int OP>
hipError_t launch_tile2_u(const TileArgs& a, int U, dim3 g, dim3 b, uint32_t buf_bytes, uint32_t lds,
                          int64_t nblocks, int remap, int nprod, int P, hipStream_t st) {
  const void* fn = U == 1 ? reinterpret_cast<const void*>(&k_tile2<S, OP, 1>)
                   : U == 2 ? reinterpret_cast<const void*>(&k_tile2<S, OP, 2>)
                            : reinterpret_cast<const void*>(&k_tile2<S, OP, 3>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  switch (U) {
    case 1: hipLaunchKernelGGL((k_tile2<S, OP, 1>), g, b, lds, st, a, nblocks, remap, buf_bytes, nprod, P); break;
    case 2: hipLaunchKernelGGL((k_tile2<S, OP, 2>), g, b, lds, st, a, nblocks, remap, buf_bytes, nprod, P); break;
    default: hipLaunchKernelGGL((k_tile2<S, OP, 3>), g, b, lds, st, a, nblocks, remap, buf_bytes, nprod, P); break;
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_tiles2_t(int op, const TileArgs& a, int U, uint32_t buf_bytes, uint32_t lds, int nprod, int ncons,
                           int per_cu, int num_cus, int P, const Shape& sh, hipStream_t st) {
  const int64_t nblocks = a.ntiles * a.nchunks;
  int64_t grid = (int64_t)per_cu * num_cus;
  if (grid > nblocks) grid = nblocks;
  const int remap = (sh.xcd_remap && grid % 8 == 0) ? 1 : 0;
  const dim3 g((unsigned)grid), b((unsigned)(64 * (nprod + ncons)));
  switch (op) {
    case OP_GRAD: return launch_tile2_u<S, OP_GRAD>(a, U, g, b, buf_bytes, lds, nblocks, remap, nprod, P, st);
    case OP_DIV: return launch_tile2_u<S, OP_DIV>(a, U, g, b, buf_bytes, lds, nblocks, remap, nprod, P, st);
    case OP_GRADT: return launch_tile2_u<S, OP_GRADT>(a, U, g, b, buf_bytes, lds, nblocks, remap, nprod, P, st);
    case OP_DIVT: return launch_tile2_u<S, OP_DIVT>(a, U, g, b, buf_bytes, lds, nblocks, remap, nprod, P, st);
    case OP_LAP: return launch_tile2_u<S, OP_LAP>(a, U, g, b, buf_bytes, lds, nblocks, remap, nprod, P, st);
    default: return hipErrorInvalidValue;
  }
}

template <class S>
hipError_t launch_tiles_t(int op, const TileArgs& a, int U, uint32_t lds, const Shape& sh, hipStream_t st) {
  const int64_t nblocks = a.ntiles * a.nchunks;
  const int64_t grid = sh.xcd_remap ? (nblocks + 7) / 8 * 8 : nblocks;
  const dim3 g((unsigned)grid), b((unsigned)(64 * sh.waves_per_block));
  switch (op) {
    case OP_GRAD: return launch_tile_u<S, OP_GRAD>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_DIV: return launch_tile_u<S, OP_DIV>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_GRADT: return launch_tile_u<S, OP_GRADT>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_DIVT: return launch_tile_u<S, OP_DIVT>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_LAP: return launch_tile_u<S, OP_LAP>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_GRADLAP: return launch_tile_u<S, OP_GRADLAP>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    case OP_DIVCURL: return launch_tile_u<S, OP_DIVCURL>(a, U, g, b, lds, nblocks, sh.xcd_remap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool uses_window(int op, int nlev, const Shape& sh) {
  return op != OP_LAP && nlev > 32 && sh.row_window != 2;
}

int lanes_per_node(int nlev, const Shape& sh) {
  if (nlev <= 32) return nlev;
  if (sh.lanes_per_node > 0) return sh.lanes_per_node;
  // best lane utilisation nlev / (P * ceil(nlev / P)); ties go to the wider P
  int best = 64;
  double bu = -1.0;
  for (int p : {64, 32, 16}) {
    const int nsl = (nlev + p - 1) / p;
    const double u = (double)nlev / (double)(p * nsl);
    if (u > bu + 1e-12) {
      bu = u;
      best = p;
    }
  }
  return best;
}

int slices_per_iter(int nlev, const Shape& sh) {
  const int P = lanes_per_node(nlev, sh);
  const int nsl = (nlev + P - 1) / P;
  int U = sh.slices_per_iter > 0 ? sh.slices_per_iter : 3;
  if (U > 3) U = 3;
  return U < nsl ? U : nsl;
}

int64_t blocks_for(int op, const NodeOrder& ord, int64_t V, int nlev, const Shape& sh) {
  if (uses_window(op, nlev, sh)) {
    const int64_t per_block = (int64_t)sh.waves_per_block * sh.nodes_per_wave;
    return (ord.nruns + per_block - 1) / per_block;
  }
  const int G = 64 / lanes_per_node(nlev, sh);
  const int64_t per_block = (int64_t)sh.waves_per_block * sh.nodes_per_wave * G;
  return (V + per_block - 1) / per_block;
}

hipError_t launch_op(int op, int dtype, const DevTables& t, const NodeOrder& ord, int64_t V, int nlev,
                     const void* in, void* out, const Shape& shape_in, hipStream_t stream) {
  Shape shape = shape_in;
  if (shape.waves_per_block > 4) shape.waves_per_block = 4;   // 8 applies to LDS tiles only
  if (op == OP_LAP && t.lap_stride != kLapStride) return hipErrorInvalidValue;
  const Args a = make_args(op, t, ord, V, nlev, in, out, shape);
  const bool window = uses_window(op, nlev, shape);
  const int U = window ? window_slices(nlev, shape) : slices_per_iter(nlev, shape);
  const int64_t nblocks = blocks_for(op, ord, V, nlev, shape);
  switch (dtype) {
    case DT_F64: return launch_op_t<double>(kernel_op(op), a, U, nblocks, window, shape, stream);
    case DT_F32: return launch_op_t<float>(kernel_op(op), a, U, nblocks, window, shape, stream);
    case DT_BF16: return launch_op_t<bf16_t>(kernel_op(op), a, U, nblocks, window, shape, stream);
    default: return hipErrorInvalidValue;
  }
}

Shape resolve_shape(int op, int dtype, int nlev, const Shape& sh) {
  Shape e = sh;
  if (e.lds_tiles != 0) return e;
  if (nlev <= 32) {
    e.lds_tiles = 2;
    return e;
  }
  // Measured defaults at O1280 x 137 (rows: mode, KiB, tile rows, computing
  // and copying waves of the persistent form): scalar-input 1-ring operators,
  // vector-input ones, the two-ring Laplacian.
  // (mode, KiB, tile rows, computing waves, copying waves, lanes per node,
  // waves per workgroup of the one-tile form)
  struct Def { int mode, kb, rows, cw, pw, lanes, wpb; };
  const bool vec_in = kernel_op(op) == OP_DIV || kernel_op(op) == OP_GRADT || kernel_op(op) == OP_DIVCURL;
  const bool lap = op == OP_LAP || op == OP_GRADLAP;   // the fused form takes the Laplacian's
  // the divergence paired with the curl or the gradient adjoint in one pass
  // (its records hold two coefficient rows)
  const bool dual = kernel_op(op) == OP_DIVCURL;
  Def d;
  if (dtype == DT_F32)
    d = lap    ? Def{3, 80, 4, 0, 0, 0, 8}
        : dual ? Def{3, 80, 4, 0, 0, 0, 16}
        : vec_in ? Def{3, 64, 4, 0, 0, 0, 8}
                 : Def{3, 40, 4, 0, 0, 0, 8};
  else if (dtype == DT_BF16)
    d = lap ? Def{3, 53, 4, 0, 0, 0, 8} : vec_in ? Def{3, 80, 4, 0, 0, 0, 16} : Def{3, 64, 4, 0, 0, 0, 16};
  else
    d = lap    ? Def{3, 160, 4, 0, 0, 0, 16}
        : dual ? Def{3, 160, 4, 0, 0, 0, 8}
        : vec_in ? Def{3, 80, 4, 0, 0, 0, 8}
                 : Def{3, 64, 3, 0, 0, 0, 8};
  e.lds_tiles = d.mode;
  if (d.mode == 2) return e;
  if (!e.tile_kb) e.tile_kb = d.kb;
  if (!e.band_rows) e.band_rows = d.rows;
  if (!e.tile_waves) e.tile_waves = d.cw;
  if (!e.producer_waves) e.producer_waves = d.pw;
  if (!e.lanes_per_node) e.lanes_per_node = d.lanes;
  if (d.wpb && e.waves_per_block == Shape().waves_per_block) e.waves_per_block = d.wpb;
  // FP64 one-pass gradient and Laplacian: one slice per step fits 16 waves
  // in 128 registers (7.1 ms against 7.7 ms with two slices and 8 waves)
  if (op == OP_GRADLAP && dtype == DT_F64 && !e.slices_per_iter) e.slices_per_iter = 1;
  return e;
}

bool uses_tiles(int op, int dtype, int nlev, const Shape& sh) {
  (void)op;
  if (nlev <= 32) return false;
  if (dtype == DT_BF16) return sh.lds_tiles == 3;   // BF16: one-tile form only
  return (dtype == DT_F32 || dtype == DT_F64) && (sh.lds_tiles == 1 || sh.lds_tiles == 3);
}

TileGeom tile_geom(int op, int dtype, int nlev, const Shape& sh) {
  TileGeom g;
  const int64_t es = dtype == DT_F64 ? 8 : dtype == DT_BF16 ? 2 : 4;
  const int64_t cin = (kernel_op(op) == OP_DIV || kernel_op(op) == OP_GRADT || kernel_op(op) == OP_DIVCURL) ? 2 : 1;
  g.ring = (op == OP_LAP || op == OP_GRADLAP) ? 2 : 1;
  g.row_bytes = tile_record_bytes(op, dtype);
  g.budget = (int64_t)(sh.tile_kb > 0 ? sh.tile_kb : kDefaultTileKB) * 1024;
  // the read-past tail behind a workgroup's buffers (one, or two for the
  // persistent form) must not cost a workgroup per CU: with n = LDS / (nb
  // budget) workgroups per CU, the budget leaves room for the largest tail
  // (3 x 64 levels)
  if (sh.lds_tiles == 3 || sh.lds_tiles == 1) {
    const int64_t nb = sh.lds_tiles == 1 ? 2 : 1;
    const int64_t n = (int64_t)kLdsPerCu / (nb * g.budget) > 1 ? (int64_t)kLdsPerCu / (nb * g.budget) : 1;
    const int64_t cap = (((int64_t)kLdsPerCu / n - 3 * 64 * cin * es) / nb) & ~(int64_t)15;
    if (g.budget > cap) g.budget = cap;
  }
  if (dtype == DT_BF16) {
    // whole columns only; per column the data, its offset-table entry and up
    // to 8 bytes of alignment padding, plus 16 bytes of table alignment
    g.budget -= 16;
    const int64_t stencil = g.ring == 2 ? kLapStride : 8;
    g.col_bytes = (int64_t)nlev * cin * es + kBf16ColExtra;
    if (stencil * g.col_bytes + (stencil / 2) * g.row_bytes > g.budget) return g;   // KL = 0: no tiles
    g.KL = nlev;
    g.nchunks = 1;
    return g;
  }
  // Column chunk: whole columns if a tile of `want` columns (and half as many
  // nodes' table rows) fits, else the largest equal chunks that do; if even
  // that fails, fall back to the minimum of one node's stencil.
  const int64_t stencil = g.ring == 2 ? kLapStride : 8;
  const int64_t wants[2] = {g.ring == 2 ? 96 : 48, stencil};
  g.KL = 0;
  if (sh.tile_levels > 0) {
    // asked-for chunk, if one node's stencil fits with it
    const int64_t k = sh.tile_levels < nlev ? sh.tile_levels : nlev;
    if (stencil * k * cin * es + (stencil / 2) * g.row_bytes <= g.budget) {
      g.KL = (int)k;
      g.nchunks = (nlev + g.KL - 1) / g.KL;
      g.col_bytes = (int64_t)g.KL * cin * es;
      return g;
    }
  }
  for (int64_t want : wants) {
    const int64_t per_col = (g.budget - (want / 2) * g.row_bytes) / want;
    const int64_t kl = per_col / (cin * es);
    if (kl < 1) continue;
    // equal chunks, rounded up to whole 16-byte units when that still fits
    const int64_t nch = (nlev + kl - 1) / kl;
    const int64_t m = 16 / (cin * es) > 1 ? 16 / (cin * es) : 1;
    int64_t k = (nlev + nch - 1) / nch;
    if ((k + m - 1) / m * m <= kl) k = (k + m - 1) / m * m;
    g.KL = (int)(k < nlev ? k : nlev);
    break;
  }
  if (g.KL < 1) return g;   // no tile geometry fits the budget
  g.nchunks = (nlev + g.KL - 1) / g.KL;
  g.col_bytes = (int64_t)g.KL * cin * es;
  return g;
}

int tile_slices(int KL, const Shape& sh) {
  // whole 64-level slices of a chunk: a remainder of 1..32 levels goes to the
  // packed tail pass
  const int rem = KL & 63;
  const int kmain = rem != 0 && rem <= 32 ? KL - rem : KL;
  const int nsl = (kmain + 63) / 64 > 0 ? (kmain + 63) / 64 : 1;
  const int u = sh.slices_per_iter > 0 ? sh.slices_per_iter : 3;
  return u < nsl ? u : nsl;
}

int64_t tile_tail_bytes(int op, int dtype, int KL, int nlev, int U) {
  const int64_t es = dtype == DT_F64 ? 8 : dtype == DT_BF16 ? 2 : 4;
  const int64_t cin = (kernel_op(op) == OP_DIV || kernel_op(op) == OP_GRADT || kernel_op(op) == OP_DIVCURL) ? 2 : 1;
  // a step reads 64 U levels (64 on the single-slice paths) from level 0 on:
  // past a chunk of k levels up to round_up(k, 64 U) - k levels
  const int64_t step = 64 * (int64_t)U;
  const int64_t last = nlev - (int64_t)((nlev - 1) / KL) * KL;
  const int64_t t0 = (KL + step - 1) / step * step - KL, t1 = (last + step - 1) / step * step - last;
  return (t0 > t1 ? t0 : t1) * cin * es;
}

int64_t tile_record_bytes(int op, int dtype) {
  switch (op * 2 + (dtype == DT_F64 ? 1 : 0)) {
    case OP_LAP * 2: return TileRec<float, OP_LAP>::kBytes;
    case OP_LAP * 2 + 1: return TileRec<double, OP_LAP>::kBytes;
    case OP_GRADLAP * 2: return TileRec<float, OP_GRADLAP>::kBytes;
    case OP_GRADLAP * 2 + 1: return TileRec<double, OP_GRADLAP>::kBytes;
    case OP_DIVCURL * 2:
    case OP_DIVGRADT * 2: return TileRec<float, OP_DIVCURL>::kBytes;
    case OP_DIVCURL * 2 + 1:
    case OP_DIVGRADT * 2 + 1: return TileRec<double, OP_DIVCURL>::kBytes;
    default: return dtype == DT_F64 ? TileRec<double, OP_GRAD>::kBytes : TileRec<float, OP_GRAD>::kBytes;
  }
}

hipError_t pack_tile_records(int op, int dtype, const DevTables& t, const int32_t* order, const uint16_t* loc,
                             int64_t V, void* rec, hipStream_t stream) {
  const int64_t n = V * (tile_record_bytes(op, dtype) / 4);
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  const bool dual = op == OP_DIVCURL || op == OP_DIVGRADT;   // divergence rows, then the second operator's
  const void* coef = (op == OP_LAP || op == OP_GRADLAP) ? t.lap_w : dual ? t.coef[OP_DIV] : t.coef[op];
  const void* coef2 = op == OP_GRADLAP ? t.coef[OP_GRAD]
                      : op == OP_DIVCURL ? t.coef[OP_CURL]
                      : op == OP_DIVGRADT ? t.coef[OP_GRADT]
                                          : nullptr;
  uint32_t* r = static_cast<uint32_t*>(rec);
  const bool f64 = dtype == DT_F64;
  if (op == OP_LAP) {
    if (f64) hipLaunchKernelGGL((k_pack_records<double, OP_LAP>), g, b, 0, stream, order, coef, coef2, loc, V, r);
    else hipLaunchKernelGGL((k_pack_records<float, OP_LAP>), g, b, 0, stream, order, coef, coef2, loc, V, r);
  } else if (op == OP_GRADLAP) {
    if (f64) hipLaunchKernelGGL((k_pack_records<double, OP_GRADLAP>), g, b, 0, stream, order, coef, coef2, loc, V, r);
    else hipLaunchKernelGGL((k_pack_records<float, OP_GRADLAP>), g, b, 0, stream, order, coef, coef2, loc, V, r);
  } else if (dual) {
    if (f64) hipLaunchKernelGGL((k_pack_records<double, OP_DIVCURL>), g, b, 0, stream, order, coef, coef2, loc, V, r);
    else hipLaunchKernelGGL((k_pack_records<float, OP_DIVCURL>), g, b, 0, stream, order, coef, coef2, loc, V, r);
  } else {
    if (f64) hipLaunchKernelGGL((k_pack_records<double, OP_GRAD>), g, b, 0, stream, order, coef, coef2, loc, V, r);
    else hipLaunchKernelGGL((k_pack_records<float, OP_GRAD>), g, b, 0, stream, order, coef, coef2, loc, V, r);
  }
  return hipGetLastError();
}

hipError_t launch_tiles(int op, int dtype, const DevTiles& dt, const void* rec, int nlev, const void* in,
                        void* out, const Shape& shape, int num_cus, hipStream_t stream, void* out2) {
  // the tiling's LDS footprint must be the one the kernel lays out
  const bool bf = dtype == DT_BF16;
  const int64_t es = dtype == DT_F64 ? 8 : bf ? 2 : 4;
  const int64_t cin = (kernel_op(op) == OP_DIV || kernel_op(op) == OP_GRADT || kernel_op(op) == OP_DIVCURL) ? 2 : 1;
  const int64_t row = tile_record_bytes(op, dtype);
  const int64_t colb = (int64_t)dt.KL * cin * es + (bf ? kBf16ColExtra : 0);
  const int U3 = tile_slices(dt.KL, shape);
  // one tile per workgroup: lanes past a column's last level read into a
  // tail behind the buffer
  const uint32_t lds_need =
      dt.lds_bytes + (bf ? 16u : 0u) +
      (shape.lds_tiles == 3 && dt.KL >= 1 ? (uint32_t)tile_tail_bytes(op, dtype, dt.KL, nlev, U3) : 0u);
  if (dt.KL < 1 || dt.KL > nlev || dt.nchunks != (nlev + dt.KL - 1) / dt.KL || lds_need > kLdsPerCu ||
      dt.col_bytes != colb || dt.row_bytes != row || (bf && (dt.KL != nlev || shape.lds_tiles != 3)))
    return hipErrorInvalidValue;
  TileArgs a;
  a.info = dt.info;
  a.segs = dt.segs;
  a.rec = static_cast<const char*>(rec);
  a.in = in;
  a.out = out;
  a.out2 = out2;
  const bool two = op == OP_GRADLAP || kernel_op(op) == OP_DIVCURL;
  if (two != (out2 != nullptr) || (two && shape.lds_tiles != 3))
    return hipErrorInvalidValue;   // the one-pass forms: one-tile workgroups, both outputs
  a.ntiles = dt.ntiles;
  a.L = nlev;
  a.KL = dt.KL;
  a.nchunks = dt.nchunks;
  a.nt = nt_of(shape) ? 1 : 0;
  if (shape.lds_tiles == 3) {
    const int U = U3;
    switch (dtype) {
      case DT_F64: return launch_tiles_t<double>(kernel_op(op), a, U, lds_need, shape, stream);
      case DT_F32: return launch_tiles_t<float>(kernel_op(op), a, U, lds_need, shape, stream);
      case DT_BF16: return launch_tiles_t<bf16_t>(kernel_op(op), a, U, lds_need, shape, stream);
      default: return hipErrorInvalidValue;
    }
  }
  // persistent double-buffered form
  const int nprod = shape.producer_waves > 0 ? shape.producer_waves : 2;
  const int ncons = shape.tile_waves > 0 ? shape.tile_waves : 6;
  if (nprod + ncons > (dtype == DT_F64 ? 8 : 16) || (nprod & (nprod - 1))) return hipErrorInvalidValue;
  const uint32_t buf_bytes = (dt.lds_bytes + 15u) & ~15u;
  const int P = lanes_per_node(dt.KL, shape);
  const int nsl = (dt.KL + P - 1) / P;
  int U = shape.slices_per_iter > 0 ? shape.slices_per_iter : 3;
  if (U > nsl) U = nsl;
  // whole-wave nodes read past a column's last level, as in the one-tile form
  const uint32_t lds = 2 * buf_bytes + (P == 64 ? (uint32_t)tile_tail_bytes(op, dtype, dt.KL, nlev, U) : 0u);
  // workgroups per CU as asked, as far as their two buffers fit the CU's LDS
  int per_cu = shape.tile_wgs_per_cu > 0 ? shape.tile_wgs_per_cu : 1;
  while (per_cu > 1 && (uint64_t)lds * per_cu > kLdsPerCu) --per_cu;
  if (lds > kLdsPerCu) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_F64:
      return launch_tiles2_t<double>(kernel_op(op), a, U, buf_bytes, lds, nprod, ncons, per_cu, num_cus, P, shape,
                                     stream);
    case DT_F32:
      return launch_tiles2_t<float>(kernel_op(op), a, U, buf_bytes, lds, nprod, ncons, per_cu, num_cus, P, shape,
                                    stream);
    default: return hipErrorInvalidValue;
  }
}

void kernel_label(int op, int dtype, int nlev, const Shape& sh, char* buf, int len) {
  const char* ty = dtype == DT_F64 ? "double" : dtype == DT_F32 ? "float" : "unsigned short";
  const char* name = nullptr;
  int U = 1;
  if (uses_tiles(op, dtype, nlev, sh)) {
    const TileGeom g = tile_geom(op, dtype, nlev, sh);
    if (g.KL > 0) {
      if (sh.lds_tiles == 3) {
        U = tile_slices(g.KL, sh);
      } else {
        const int P = lanes_per_node(g.KL, sh);
        const int nsl = (g.KL + P - 1) / P;
        U = sh.slices_per_iter > 0 ? sh.slices_per_iter : 3;
        if (U > nsl) U = nsl;
      }
      name = sh.lds_tiles == 3 ? "k_tile" : "k_tile2";
    }
  }
  if (!name) {
    if (op != OP_LAP && uses_window(op, nlev, sh)) {
      name = "k_win";
      U = window_slices(nlev, sh);
    } else {
      name = "k_op";
      U = slices_per_iter(nlev, sh);
    }
  }
  snprintf(buf, (size_t)len, "%s<%s, %d, %d>", name, ty, kernel_op(op), U);
}

int window_slices(int nlev, const Shape& sh) {
  const int nsl = (nlev + 63) / 64;
  int U = sh.slices_per_iter > 0 ? sh.slices_per_iter : 3;
  if (U > 3) U = 3;
  return U < nsl ? U : nsl;
}

int conservation_parts(int64_t V, int nlev) {
  (void)nlev;
  const int64_t p = (V + 63) / 64;
  return (int)(p < 4096 ? p : 4096);
}

hipError_t launch_conservation(int dtype, const double* vol, int64_t V, int nlev, const void* div, double* scratch,
                               double* out_sum, double* out_abs, hipStream_t stream) {
  const int parts = conservation_parts(V, nlev);
  const int64_t chunk = (V + parts - 1) / parts;
  const dim3 g(parts), b(64 * kConsWaves);
  // slices of the column's last 256-level block
  const int rem = nlev % kConsBlockLevels;
  const int nsl = rem == 0 ? 4 : (rem + 63) / 64;
  switch (dtype * 4 + (nsl - 1)) {
#define ATLAS_CONS(DT, S, N)                                                                                   \
  case DT * 4 + (N - 1):                                                                                       \
    hipLaunchKernelGGL((k_cons_partial<S, N>), g, b, 0, stream, static_cast<const S*>(div), vol, V, nlev, chunk, \
                       scratch);                                                                               \
    break;
    ATLAS_CONS(DT_F64, double, 1) ATLAS_CONS(DT_F64, double, 2) ATLAS_CONS(DT_F64, double, 3)
    ATLAS_CONS(DT_F64, double, 4) ATLAS_CONS(DT_F32, float, 1) ATLAS_CONS(DT_F32, float, 2)
    ATLAS_CONS(DT_F32, float, 3) ATLAS_CONS(DT_F32, float, 4) ATLAS_CONS(DT_BF16, bf16_t, 1)
    ATLAS_CONS(DT_BF16, bf16_t, 2) ATLAS_CONS(DT_BF16, bf16_t, 3) ATLAS_CONS(DT_BF16, bf16_t, 4)
#undef ATLAS_CONS
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cons_final, dim3(nlev), dim3(256), 0, stream, scratch, parts, nlev, out_sum, out_abs);
  return hipGetLastError();
}

// Partial sums of the allocation-free conservation call: one array per GPU,
// held by the library until the process ends.  In host code `scratch` names
// a host-side stand-in, never the device memory: kernels and copies take the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t scratch_address(int device, double** ptr) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    // the caller has made `device` current
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

namespace {

template <class S, int OP, int UMAX>
hipError_t launch_tb(const TileArgs& a, const BatchTile* tr, const int32_t* pre, int ntr, int32_t* ctr, int32_t claim,
                     uint32_t lds, int waves, int64_t grid, hipStream_t st) {
  const void* fn = reinterpret_cast<const void*>(&k_tile_batched<S, OP, UMAX>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 g((unsigned)grid), b((unsigned)(64 * waves));
  hipLaunchKernelGGL((k_tile_batched<S, OP, UMAX>), g, b, lds, st, a, tr, pre, ntr, ctr, claim);
  return hipGetLastError();
}

template <class S, int OP>
const void* tb_fn_u(int umax) {
  return umax == 1   ? reinterpret_cast<const void*>(&k_tile_batched<S, OP, 1>)
         : umax == 2 ? reinterpret_cast<const void*>(&k_tile_batched<S, OP, 2>)
                     : reinterpret_cast<const void*>(&k_tile_batched<S, OP, 3>);
}

template <class S>
const void* tb_fn(int op, int umax) {
  switch (op) {
    case OP_GRAD: return tb_fn_u<S, OP_GRAD>(umax);
    case OP_DIV: return tb_fn_u<S, OP_DIV>(umax);
    case OP_GRADT: return tb_fn_u<S, OP_GRADT>(umax);
    case OP_DIVT: return tb_fn_u<S, OP_DIVT>(umax);
    case OP_DIVCURL: return tb_fn_u<S, OP_DIVCURL>(umax);
    default: return nullptr;
  }
}

template <class S, int OP>
hipError_t launch_tb_u(const TileArgs& a, const BatchTile* tr, const int32_t* pre, int ntr, int32_t* ctr,
                       int32_t claim, uint32_t lds, int waves, int64_t grid, int umax, hipStream_t st) {
  switch (umax) {
    case 1: return launch_tb<S, OP, 1>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, st);
    case 2: return launch_tb<S, OP, 2>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, st);
    default: return launch_tb<S, OP, 3>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, st);
  }
}

template <class S>
hipError_t launch_tb_t(int op, const TileArgs& a, const BatchTile* tr, const int32_t* pre, int ntr, int32_t* ctr,
                       int32_t claim, uint32_t lds, int waves, int64_t grid, int umax, hipStream_t st) {
  switch (op) {
    case OP_GRAD: return launch_tb_u<S, OP_GRAD>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, st);
    case OP_DIV: return launch_tb_u<S, OP_DIV>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, st);
    case OP_GRADT: return launch_tb_u<S, OP_GRADT>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, st);
    case OP_DIVT: return launch_tb_u<S, OP_DIVT>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, st);
    case OP_DIVCURL: return launch_tb_u<S, OP_DIVCURL>(a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int tiles_batched_per_cu(int op, int dtype, uint32_t lds, int waves, int umax) {
  const int kop = kernel_op(op);
  const void* fn = dtype == DT_F64 ? tb_fn<double>(kop, umax) : dtype == DT_F32 ? tb_fn<float>(kop, umax) : nullptr;
  if (!fn || waves < 1 || waves > batched_max_waves(kop, dtype) || lds > kLdsPerCu || umax < 1 || umax > 3) return 0;
  if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * waves, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

hipError_t launch_tiles_batched(int op, int dtype, const BatchTile* tr, const int32_t* pre, int ntr, int32_t* ctr,
                                int32_t claim, uint32_t lds, int waves, int64_t grid, int umax,
                                hipStream_t stream) {
  const int kop = kernel_op(op);
  // the four batchable operators and the divergence and gradient adjoint
  // pair (each tracer's out2 set)
  if (kop != OP_GRAD && kop != OP_DIV && kop != OP_GRADT && kop != OP_DIVT && op != OP_DIVGRADT)
    return hipErrorInvalidValue;
  // the grid is a multiple of 8 workgroups (one share per XCD)
  if (ntr < 1 || !ctr || claim < 1 || claim > 64 || grid < 8 || grid % 8 != 0 || grid > INT32_MAX || waves < 1 ||
      waves > batched_max_waves(kop, dtype) || lds > kLdsPerCu || umax < 1 || umax > 3)
    return hipErrorInvalidValue;
  TileArgs a;   // fields, tiling and level chunking per tracer in the kernel
  a.info = nullptr;
  a.segs = nullptr;
  a.rec = nullptr;
  a.in = nullptr;
  a.out = nullptr;
  a.out2 = nullptr;
  a.ntiles = 0;
  a.L = a.KL = a.nchunks = 1;
  a.nt = 0;
  switch (dtype) {
    case DT_F64: return launch_tb_t<double>(kop, a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, stream);
    case DT_F32: return launch_tb_t<float>(kop, a, tr, pre, ntr, ctr, claim, lds, waves, grid, umax, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_remap(int dtype, const int32_t* nodes, const void* w, int64_t V, int64_t P, int nlev,
                        const void* in, void* out, hipStream_t stream) {
  if (V < 1 || P < 1 || nlev < 1 || (P + 15) / 16 > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_F64: return launch_remap_t<double>(nodes, w, V, P, nlev, in, out, stream);
    case DT_F32: return launch_remap_t<float>(nodes, w, V, P, nlev, in, out, stream);
    case DT_BF16: return launch_remap_t<bf16_t>(nodes, w, V, P, nlev, in, out, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_remap_adjoint(int dtype, const int64_t* off, const int32_t* tt, const void* w, const int32_t* ht,
                                const void* hw, int64_t V, int64_t P, int nlev, const void* in, void* out,
                                hipStream_t stream) {
  if (V < 1 || P < 1 || nlev < 1 || (V + 15) / 16 > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_F64: return launch_remap_adj_t<double>(off, tt, w, ht, hw, V, P, nlev, in, out, stream);
    case DT_F32: return launch_remap_adj_t<float>(off, tt, w, ht, hw, V, P, nlev, in, out, stream);
    case DT_BF16: return launch_remap_adj_t<bf16_t>(off, tt, w, ht, hw, V, P, nlev, in, out, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace atlasnabla
