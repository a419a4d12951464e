// Device-side building blocks shared by the HIP kernels of the library:
// the D3Q19 velocity set, population storage formats and the pull-stream
// gather with periodic or halfway bounce-back boundaries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"
#include "lbmibm.h"

namespace lbmd {

// D3Q19 velocity set in the export order documented in lbmibm.h.
constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// Lattice weights: 1/3 rest, 1/18 axis links, 1/36 diagonal links.
__host__ __device__ constexpr float wgt(int i) {
  return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double wgt_d(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------------------
// Population storage.  Every format holds the offset f_i - t_i; arithmetic is
// FP32.  16-bit formats round to nearest even on store.
// ---------------------------------------------------------------------------
template <int S>
struct Store;

// load_nt / store_nt: the same access with a non-temporal (streaming) hint,
// for the stream-collide's lattice reads and writes.
template <>
struct Store<LBM_STORE_F32> {
  using T = float;
  static __device__ __forceinline__ float load(const T* p) { return *p; }
  static __device__ __forceinline__ float load_nt(const T* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void store(T* p, float v) { *p = v; }
  static __device__ __forceinline__ void store_nt(T* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<LBM_STORE_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float load(const T* p) { return (float)*p; }
  static __device__ __forceinline__ float load_nt(const T* p) {
    return (float)__builtin_nontemporal_load(p);
  }
  static __device__ __forceinline__ void store(T* p, float v) { *p = (_Float16)v; }
  static __device__ __forceinline__ void store_nt(T* p, float v) {
    __builtin_nontemporal_store((_Float16)v, p);
  }
  // load2_nt / store2_nt: two consecutive values at an even element offset
  // (4-byte aligned) in one access.
  typedef _Float16 V2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load2_nt(const T* p, float& a, float& b) {
    const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
    a = (float)v.x;
    b = (float)v.y;
  }
  static __device__ __forceinline__ void store2_nt(T* p, float a, float b) {
    V2 v;
    v.x = (_Float16)a;
    v.y = (_Float16)b;
    __builtin_nontemporal_store(v, reinterpret_cast<V2*>(p));
  }
  // the pair as one 32-bit word (a in the low half)
  static __device__ __forceinline__ uint32_t pack2(float a, float b) {
    V2 v;
    v.x = (_Float16)a;
    v.y = (_Float16)b;
    return __builtin_bit_cast(uint32_t, v);
  }
};

template <>
struct Store<LBM_STORE_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float load(const T* p) {
    return __uint_as_float(((uint32_t)*p) << 16);
  }
  static __device__ __forceinline__ float load_nt(const T* p) {
    return __uint_as_float(((uint32_t)__builtin_nontemporal_load(p)) << 16);
  }
  // gfx950 converts FP32 to BF16 in hardware, rounding to nearest even and
  // keeping NaN quiet; one instruction in place of the integer sequence.
  static __device__ __forceinline__ uint16_t bits(float v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
  }
  static __device__ __forceinline__ void store(T* p, float v) { *p = bits(v); }
  static __device__ __forceinline__ void store_nt(T* p, float v) {
    __builtin_nontemporal_store(bits(v), p);
  }
  static __device__ __forceinline__ void load2_nt(const T* p, float& a, float& b) {
    const uint32_t u = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
    a = __uint_as_float(u << 16);
    b = __uint_as_float(u & 0xffff0000u);
  }
  static __device__ __forceinline__ void store2_nt(T* p, float a, float b) {
    const uint32_t u = (uint32_t)bits(a) | ((uint32_t)bits(b) << 16);
    __builtin_nontemporal_store(u, reinterpret_cast<uint32_t*>(p));
  }
  // the pair as one 32-bit word (a in the low half)
  static __device__ __forceinline__ uint32_t pack2(float a, float b) {
    return (uint32_t)bits(a) | ((uint32_t)bits(b) << 16);
  }
};

// ---------------------------------------------------------------------------
// Lattice geometry passed by value to the lattice kernels.
// bb_add[a][face][i]: term added to population i when it is reflected at the
// wall of axis a (face 0 = low, 1 = high): 6 t_i rho_w e_i . u_w.
// ---------------------------------------------------------------------------
// Population layout of a lattice buffer: population i of cell (x, y, z) is
// element i spop + x + y srow + z splane.  Below 4 GB per lattice the 19
// populations of each x row of cells are interleaved ([z][y][i][x], rows
// padded to 128 bytes: spop = padded row, srow = 19 spop), so that a
// workgroup's accesses to one row of cells stay within one 19-row stretch;
// else one array per population ([i][z][y][x]: srow = nx, splane = nx ny).
// Offsets of a cell (x + y srow + z splane) fit in 32 bits in both forms.
struct LatticeGeom {
  int nx, ny, nz;
  int bc[3];
  int64_t ncell;
  int64_t spop;       // elements between a cell's consecutive populations
  int64_t srow;       // elements between rows (y) of cells
  int64_t splane;     // elements between planes (z) of cells
  int64_t lat_elems;  // elements of one lattice buffer
  float bb_add[3][2][Q];
  float tau, omega;   // omega = 1 / tau
  float g_ext[3];
  int fblk_x, fblk_y;  // grid of 4^3 force blocks (x, y extent) for flag lookups
};

// Element offset of population 0 of cell (x, y, z) in a lattice buffer.
__device__ __forceinline__ int64_t lat_cell(const LatticeGeom& g, int x, int y, int z) {
  return (int64_t)x + (int64_t)y * g.srow + (int64_t)z * g.splane;
}


// Pull-stream gather of the 19 post-stream offsets at cell (x, y, z) from the
// post-collision lattice `lat` (eq. (4) read backwards: f_i(X) = f*_i(X - e_i);
// at a wall the reflected population of the same cell, plus bb_add).
template <int S>
__device__ __forceinline__ void gather_pull(const typename Store<S>::T* __restrict__ lat,
                                            const LatticeGeom& g, int x, int y, int z,
                                            float f[Q]) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t here = lat_cell(g, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int sx = x - EX[i], sy = y - EY[i], sz = z - EZ[i];
    int wall_axis = -1, wall_face = 0;
    if (EX[i] != 0 && (sx < 0 || sx >= nx)) {
      if (g.bc[0] == LBM_BC_PERIODIC) {
        sx = sx < 0 ? sx + nx : sx - nx;
      } else {
        wall_axis = 0;
        wall_face = sx < 0 ? 0 : 1;
      }
    }
    if (EY[i] != 0 && (sy < 0 || sy >= ny)) {
      if (g.bc[1] == LBM_BC_PERIODIC) {
        sy = sy < 0 ? sy + ny : sy - ny;
      } else if (wall_axis < 0) {
        wall_axis = 1;
        wall_face = sy < 0 ? 0 : 1;
      }
    }
    if (EZ[i] != 0 && (sz < 0 || sz >= nz)) {
      if (g.bc[2] == LBM_BC_PERIODIC) {
        sz = sz < 0 ? sz + nz : sz - nz;
      } else if (wall_axis < 0) {
        wall_axis = 2;
        wall_face = sz < 0 ? 0 : 1;
      }
    }
    if (wall_axis < 0) {
      f[i] = Store<S>::load(lat + (int64_t)i * g.spop + lat_cell(g, sx, sy, sz));
    } else {
      f[i] = Store<S>::load(lat + (int64_t)OPP[i] * g.spop + here) +
             g.bb_add[wall_axis][wall_face][i];
    }
  }
}

// Source offsets of the pull stream at cell (x, y, z): for each axis the
// cell offsets of the sources X - e with e = -1, 0, +1 (periodic wrap);
// `fast` is false next to a wall, where gather_pull must be used.
struct PullIdx {
  uint32_t xs[3], ys[3], zs[3];
  bool fast;
};

__device__ __forceinline__ PullIdx pull_index(const LatticeGeom& g, int x, int y, int z) {
  PullIdx p;
  const int n[3] = {g.nx, g.ny, g.nz};
  const int c[3] = {x, y, z};
  const uint32_t mul[3] = {1u, (uint32_t)g.srow, (uint32_t)g.splane};
  uint32_t* out[3] = {p.xs, p.ys, p.zs};
  p.fast = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int lo = c[a] - 1, hi = c[a] + 1;  // sources for e = +1 and e = -1
    if (g.bc[a] == LBM_BC_PERIODIC) {
      lo = lo < 0 ? lo + n[a] : lo;
      hi = hi >= n[a] ? hi - n[a] : hi;
    } else {
      p.fast = p.fast && lo >= 0 && hi < n[a];
      lo = lo < 0 ? 0 : lo;
      hi = hi >= n[a] ? n[a] - 1 : hi;
    }
    out[a][0] = (uint32_t)hi * mul[a];    // e = -1
    out[a][1] = (uint32_t)c[a] * mul[a];  // e = 0
    out[a][2] = (uint32_t)lo * mul[a];    // e = +1
  }
  return p;
}

// Pull gather away from walls: 19 loads at uniform per-population bases plus
// 32-bit cell offsets.
template <int S, bool NT = false>
__device__ __forceinline__ void gather_fast(const typename Store<S>::T* __restrict__ lat,
                                            const LatticeGeom& g, const PullIdx& p, float f[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const typename Store<S>::T* q =
        lat + (int64_t)i * g.spop + (p.xs[EX[i] + 1] + p.ys[EY[i] + 1] + p.zs[EZ[i] + 1]);
    f[i] = NT ? Store<S>::load_nt(q) : Store<S>::load(q);
  }
}

// Pull gather away from walls through buffer resources (FP32 lattices of
// less than 4 GB): the lattice base sits in scalar registers, each load
// takes the cell's 32-bit byte offset and the population's byte offset as a
// scalar, so no 64-bit address is formed per load.  Streaming (nt) loads.
__device__ __forceinline__ void gather_fast_buf(__amdgpu_buffer_rsrc_t rs, const LatticeGeom& g,
                                                const PullIdx& p, float f[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t off = (p.xs[EX[i] + 1] + p.ys[EY[i] + 1] + p.zs[EZ[i] + 1]) * 4u;
    f[i] = __uint_as_float(
        __builtin_amdgcn_raw_buffer_load_b32(rs, off, (uint32_t)(i * g.spop * 4), 2));
  }
}

// Pull gather of two neighbouring cells x0 and x0 + 1 of one row for the
// 16-bit formats (x0 even, nx even, so that the pair is aligned).  Away from walls each population
// comes as one pair load at the source row's x0; a population with e_x = +1
// takes x0 - 1 for the first cell from a single load, one with e_x = -1 takes
// x0 + 2 for the second.  Next to a wall: the general gather of each cell.
template <int S>
__device__ __forceinline__ void gather_pair(const typename Store<S>::T* __restrict__ lat,
                                            const LatticeGeom& g, int x0, int y, int z,
                                            float f0[Q], float f1[Q]) {
  const PullIdx p = pull_index(g, x0, y, z);
  const bool periodic_x = g.bc[0] == LBM_BC_PERIODIC;
  if (!(p.fast && (periodic_x || x0 + 2 < g.nx))) {
    gather_pull<S>(lat, g, x0, y, z, f0);
    gather_pull<S>(lat, g, x0 + 1, y, z, f1);
    return;
  }
  const uint32_t xl = p.xs[2];                                   // x0 - 1, wrapped
  const uint32_t xr = (uint32_t)(x0 + 2 == g.nx ? 0 : x0 + 2);   // x0 + 2, wrapped
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const typename Store<S>::T* row =
        lat + (int64_t)i * g.spop + (p.ys[EY[i] + 1] + p.zs[EZ[i] + 1]);
    float a, b;
    Store<S>::load2_nt(row + x0, a, b);
    if (EX[i] == 0) {
      f0[i] = a;
      f1[i] = b;
    } else if (EX[i] == 1) {
      f0[i] = Store<S>::load_nt(row + xl);
      f1[i] = a;
    } else {
      f0[i] = b;
      f1[i] = Store<S>::load_nt(row + xr);
    }
  }
}

// The pair gather through a buffer resource (16-bit lattices of less than
// 4 GB): one 4-byte load per population pair, one 2-byte load for the outer
// value of an e_x = +-1 population; 32-bit byte offsets, the population's
// offset as a scalar.  Streaming (nt) loads.  Away from walls only.
template <int S>
__device__ __forceinline__ void gather_pair_buf(__amdgpu_buffer_rsrc_t rs, const LatticeGeom& g,
                                                const PullIdx& p, int x0, float f0[Q],
                                                float f1[Q]) {
  static_assert(S != LBM_STORE_F32, "16-bit storage");
  const uint32_t xl = p.xs[2];                                   // x0 - 1, wrapped
  const uint32_t xr = (uint32_t)(x0 + 2 == g.nx ? 0 : x0 + 2);   // x0 + 2, wrapped
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t row = p.ys[EY[i] + 1] + p.zs[EZ[i] + 1];
    const uint32_t soff = (uint32_t)(i * g.spop * 2);
    const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(rs, (row + (uint32_t)x0) * 2u, soff, 2);
    float a, b;
    if (S == LBM_STORE_F16) {
      const typename Store<LBM_STORE_F16>::V2 v =
          __builtin_bit_cast(typename Store<LBM_STORE_F16>::V2, u);
      a = (float)v.x;
      b = (float)v.y;
    } else {
      a = __uint_as_float(u << 16);
      b = __uint_as_float(u & 0xffff0000u);
    }
    if (EX[i] == 0) {
      f0[i] = a;
      f1[i] = b;
    } else {
      const uint32_t xo = EX[i] == 1 ? xl : xr;
      const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(rs, (row + xo) * 2u, soff, 2);
      const float o = S == LBM_STORE_F16 ? (float)__builtin_bit_cast(_Float16, h)
                                         : __uint_as_float(((uint32_t)h) << 16);
      if (EX[i] == 1) {
        f0[i] = o;
        f1[i] = a;
      } else {
        f0[i] = b;
        f1[i] = o;
      }
    }
  }
}

// Pull gather at any cell: the fast form away from walls, the general one
// next to them.  NT: streaming loads (the stream-collide reads each value
// once per step, from the L2 at most a few times).
template <int S, bool NT = false>
__device__ __forceinline__ void gather_any(const typename Store<S>::T* __restrict__ lat,
                                           const LatticeGeom& g, int x, int y, int z, float f[Q]) {
  const PullIdx p = pull_index(g, x, y, z);
  if (p.fast)
    gather_fast<S, NT>(lat, g, p, f);
  else
    gather_pull<S>(lat, g, x, y, z, f);
}

// Index of the 4^3 force block holding cell (x, y, z).
__device__ __forceinline__ int64_t fblock_of(const LatticeGeom& g, int x, int y, int z) {
  return (int64_t)(x >> FBLK_SHIFT) +
         (int64_t)g.fblk_x * ((int64_t)(y >> FBLK_SHIFT) + (int64_t)g.fblk_y * (z >> FBLK_SHIFT));
}

// 64-lane FP64 sum across a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace lbmd
