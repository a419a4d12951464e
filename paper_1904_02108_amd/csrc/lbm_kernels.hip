// Lattice kernels: fused pull stream-collide with forcing (§2, eqs. (1)-(4)
// and the six-step loop), initial state, checkpoint load, field export and
// the FP64 mass/momentum reduction.
#include "internal.h"

using namespace lbmd;

namespace {

// Cell coordinates of a linear cell index (x fastest).
__device__ __forceinline__ void cell_xyz(const LatticeGeom& g, int64_t cell, int& x, int& y,
                                         int& z) {
  const int64_t row = cell / g.nx;
  x = (int)(cell - row * g.nx);
  z = (int)(row / g.ny);
  y = (int)(row - (int64_t)z * g.ny);
}

// ---------------------------------------------------------------------------
// Fused stream-collide.  Per cell: gather the post-stream offsets (pull), form
// rho and U (eq. 1), add the force of flagged tiles and the uniform
// acceleration, relax towards the equilibrium (eqs. 2-3) with the
// velocity-shift or Guo forcing, store the post-collision offsets.  Each
// workgroup also writes FP64 partial sums of (rho - 1, rho U).
// ---------------------------------------------------------------------------

// e_i . (ax, ay, az) over the nonzero components of e_i (entries -1, 0, 1),
// added in x, y, z order: for finite operands the value of the full dot
// product, without its products by zero.
__device__ __forceinline__ float edot(int i, float ax, float ay, float az) {
  float r = 0.0f;
  bool any = false;
  if (EX[i]) {
    r = EX[i] > 0 ? ax : -ax;
    any = true;
  }
  if (EY[i]) {
    const float t = EY[i] > 0 ? ay : -ay;
    r = any ? r + t : t;
    any = true;
  }
  if (EZ[i]) {
    const float t = EZ[i] > 0 ? az : -az;
    r = any ? r + t : t;
  }
  return r;
}

// The D3Q19 table lists opposite directions in pairs: e_{i+1} = -e_i for odd i.
constexpr bool opposite_pairs() {
  for (int i = 1; i < Q; i += 2)
    if (OPP[i] != i + 1 || EX[i + 1] != -EX[i] || EY[i + 1] != -EY[i] || EZ[i + 1] != -EZ[i])
      return false;
  return true;
}
static_assert(opposite_pairs(), "opposite directions in consecutive pairs");

// Collision of one cell: f holds the post-stream offsets on entry and the
// post-collision ones on return; (gx, gy, gz) is the acceleration at the
// cell.  Returns rho - 1 and rho U before the force.
template <int FORCING>
__device__ __forceinline__ void collide_cell(const LatticeGeom& g, float f[Q], float gx, float gy,
                                             float gz, float& drho, float& jx, float& jy,
                                             float& jz) {
  drho = 0.f;
  jx = 0.f;
  jy = 0.f;
  jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += f[i];
    if (EX[i]) jx += EX[i] * f[i];
    if (EY[i]) jy += EY[i] * f[i];
    if (EZ[i]) jz += EZ[i] * f[i];
  }
  const float rho = 1.0f + drho;
  const float inv = 1.0f / rho;
  float ux, uy, uz;
  if (FORCING == LBM_FORCE_SHIFT) {
    ux = jx * inv + g.tau * gx;
    uy = jy * inv + g.tau * gy;
    uz = jz * inv + g.tau * gz;
  } else {
    ux = jx * inv + 0.5f * gx;
    uy = jy * inv + 0.5f * gy;
    uz = jz * inv + 0.5f * gz;
  }
  const float uu = ux * ux + uy * uy + uz * uz;
  const float om = g.omega;
  const float fx = rho * gx, fy = rho * gy, fz = rho * gz;
  const float uF = ux * fx + uy * fy + uz * fz;
  const float guo = 1.0f - 0.5f * om;
  // e_i . u and e_i . F: formed for the rest and the odd directions, negated
  // for the even ones (e_{i+1} = -e_i)
  float eu = 0.0f, eF = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    eu = (i & 1) || i == 0 ? edot(i, ux, uy, uz) : -eu;
    const float feq = wgt(i) * (drho + rho * (3.0f * eu + 4.5f * eu * eu - 1.5f * uu));
    float post = f[i] + om * (feq - f[i]);
    if (FORCING == LBM_FORCE_GUO) {
      eF = (i & 1) || i == 0 ? edot(i, fx, fy, fz) : -eF;
      post += guo * wgt(i) * (3.0f * (eF - uF) + 9.0f * eu * eF);
    }
    f[i] = post;
  }
}

// The workgroup's FP64 sums of part[0..3] into partials[blk]; a sum that is
// not finite (a NaN or infinite population, or an overflowing moment) also
// sets the sticky status word bad[0] (the non-finite check of lbm_step).
__device__ __forceinline__ void store_partials(double part[4], int tid, int64_t blk,
                                               double* __restrict__ partials,
                                               uint32_t* __restrict__ bad) {
  __shared__ double red[4][LBM_BLOCK / 64];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = wave_sum(part[k]);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (tid < 4) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < LBM_BLOCK / 64; ++w) s += red[tid][w];
    partials[blk * 4 + tid] = s;
    if (!(fabs(s) <= 1.7976931348623157e308)) bad[0] = 1u;
  }
}

// One thread per cell (FP32 storage, odd x extents).
#ifndef LBM_SC_ROWS
#define LBM_SC_ROWS 1
#endif
// BUF (FP32 lattices under 4 GB): buffer-resource loads and stores of the
// populations (see gather_fast_buf).
template <int S, int FORCING, bool FLAT, bool BUF = false>
__global__ __launch_bounds__(LBM_BLOCK) void k_stream_collide(
    const typename Store<S>::T* __restrict__ src, typename Store<S>::T* __restrict__ dst,
    const LatticeGeom g, const float* __restrict__ G, const uint8_t* __restrict__ flags,
    double* __restrict__ partials, uint32_t* __restrict__ bad) {
  static_assert(!BUF || S == LBM_STORE_F32, "buffer form for FP32 storage");
  const uint32_t lat_bytes = BUF ? (uint32_t)(g.lat_elems * 4) : 0u;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, lat_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, lat_bytes, 0x00020000);
  // 3-D launch: blockDim.x spans x, blockDim.y spans y, one z-plane per block
  // row; each workgroup takes LBM_SC_ROWS consecutive block rows along y.
  // FLAT (x extents that are not a multiple of the wavefront): 256 threads
  // over consecutive cells of an x-y plane, so that no lane idles at the
  // end of a row.
  int xf = blockIdx.x * blockDim.x + threadIdx.x, yf = 0;
  if (FLAT) {
    yf = xf / g.nx;
    xf -= yf * g.nx;
  }
  const int x = xf;
  const int z = blockIdx.z;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = 0; r < LBM_SC_ROWS; ++r) {
    const int y = FLAT ? yf : (blockIdx.y * LBM_SC_ROWS + r) * blockDim.y + threadIdx.y;
    if (x < g.nx && y < g.ny) {
      const uint32_t cell =
          (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
      // the cell's offset in the lattice buffers (32 bits in either layout)
      const uint32_t lc =
          (uint32_t)x + (uint32_t)g.srow * (uint32_t)y + (uint32_t)g.splane * (uint32_t)z;
      float f[Q];
      if constexpr (BUF) {
        const PullIdx pi = pull_index(g, x, y, z);
        if (pi.fast)
          gather_fast_buf(rsrc, g, pi, f);
        else
          gather_pull<S>(src, g, x, y, z, f);
      } else {
        gather_any<S, true>(src, g, x, y, z, f);
      }
      float gx = g.g_ext[0], gy = g.g_ext[1], gz = g.g_ext[2];
      if (flags[fblock_of(g, x, y, z)]) {
        gx += G[cell];
        gy += G[g.ncell + cell];
        gz += G[2 * g.ncell + cell];
      }
      float drho, jx, jy, jz;
      collide_cell<FORCING>(g, f, gx, gy, gz, drho, jx, jy, jz);
      if constexpr (BUF) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(f[i]), rdst, lc * 4u,
                                                (uint32_t)(i * g.spop * 4), 2);
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::store_nt(dst + (int64_t)i * g.spop + lc, f[i]);
      }
      part[0] += drho;
      part[1] += jx;
      part[2] += jy;
      part[3] += jz;
    }
  }
  const int64_t blk = (int64_t)blockIdx.x +
                      (int64_t)gridDim.x * ((int64_t)blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  store_partials(part, threadIdx.x + blockDim.x * threadIdx.y, blk, partials, bad);
}

// Two cells per thread (16-bit storage, even x extents): the pair (x0, x0 + 1)
// is read and written with one 4-byte access per population (see
// gather_pair); 256 threads over consecutive pairs of an x-y plane.
// BUF (16-bit lattices under 4 GB): buffer-resource loads and stores
// (gather_pair_buf).
template <int S, int FORCING, bool BUF = false>
__global__ __launch_bounds__(LBM_BLOCK) void k_stream_collide_pairs(
    const typename Store<S>::T* __restrict__ src, typename Store<S>::T* __restrict__ dst,
    const LatticeGeom g, const float* __restrict__ G, const uint8_t* __restrict__ flags,
    double* __restrict__ partials, uint32_t* __restrict__ bad) {
  static_assert(!BUF || S != LBM_STORE_F32, "buffer form for 16-bit storage");
  const uint32_t lat_bytes = BUF ? (uint32_t)(g.lat_elems * 2) : 0u;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, lat_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, lat_bytes, 0x00020000);
  const int px = g.nx >> 1;
  const int pf = blockIdx.x * LBM_BLOCK + threadIdx.x;
  const int y = pf / px;
  const int x0 = 2 * (pf - y * px);
  const int z = blockIdx.z;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  if (y < g.ny) {
    const uint32_t cell =
        (uint32_t)x0 + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
    const uint32_t lc =
        (uint32_t)x0 + (uint32_t)g.srow * (uint32_t)y + (uint32_t)g.splane * (uint32_t)z;
    float f0[Q], f1[Q];
    if constexpr (BUF) {
      const PullIdx pi = pull_index(g, x0, y, z);
      if (pi.fast && (g.bc[0] == LBM_BC_PERIODIC || x0 + 2 < g.nx))
        gather_pair_buf<S>(rsrc, g, pi, x0, f0, f1);
      else
        gather_pair<S>(src, g, x0, y, z, f0, f1);
    } else {
      gather_pair<S>(src, g, x0, y, z, f0, f1);
    }
    float ax[2] = {g.g_ext[0], g.g_ext[0]}, ay[2] = {g.g_ext[1], g.g_ext[1]},
          az[2] = {g.g_ext[2], g.g_ext[2]};
    if (flags[fblock_of(g, x0, y, z)]) {  // x0 and x0 + 1 share a force block
      const float2 gxv = *reinterpret_cast<const float2*>(G + cell);
      const float2 gyv = *reinterpret_cast<const float2*>(G + g.ncell + cell);
      const float2 gzv = *reinterpret_cast<const float2*>(G + 2 * g.ncell + cell);
      ax[0] += gxv.x;
      ax[1] += gxv.y;
      ay[0] += gyv.x;
      ay[1] += gyv.y;
      az[0] += gzv.x;
      az[1] += gzv.y;
    }
    float drho, jx, jy, jz;
    collide_cell<FORCING>(g, f0, ax[0], ay[0], az[0], drho, jx, jy, jz);
    part[0] += drho;
    part[1] += jx;
    part[2] += jy;
    part[3] += jz;
    collide_cell<FORCING>(g, f1, ax[1], ay[1], az[1], drho, jx, jy, jz);
    part[0] += drho;
    part[1] += jx;
    part[2] += jy;
    part[3] += jz;
    if constexpr (BUF) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        __builtin_amdgcn_raw_buffer_store_b32(Store<S>::pack2(f0[i], f1[i]), rdst, lc * 2u,
                                              (uint32_t)(i * g.spop * 2), 2);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        Store<S>::store2_nt(dst + (int64_t)i * g.spop + lc, f0[i], f1[i]);
    }
  }
  store_partials(part, threadIdx.x, (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.z,
                 partials, bad);
}

// Loads post-stream populations f (full values, float or double) as the
// state at the start of a step: the post-collision lattice is their inverse
// stream, f*_i(Y) = f_i(Y + e_i), or at a wall f*_i(Y) = f_opp(i)(Y) + bb_add.
struct SrcPops {
  const void* p;
  int f64;
  int64_t n;
  __device__ double get(int i, int64_t cell) const {
    const int64_t k = (int64_t)i * n + cell;
    return f64 ? ((const double*)p)[k] - wgt_d(i) : (double)((const float*)p)[k] - wgt_d(i);
  }
};
// Uniform equilibrium offsets Eq_i(rho0, u0) - t_i (eq. 3 with density).
struct SrcUniform {
  double feq[Q];
  __device__ double get(int i, int64_t) const { return feq[i]; }
};

template <int S, class Src>
__global__ __launch_bounds__(LBM_BLOCK) void k_unstream(typename Store<S>::T* __restrict__ dst,
                                                        const LatticeGeom g, const Src src) {
  const int64_t cell = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  if (cell >= g.ncell) return;
  int x, y, z;
  cell_xyz(g, cell, x, y, z);
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int d[3] = {x + EX[i], y + EY[i], z + EZ[i]};
    const int e[3] = {EX[i], EY[i], EZ[i]};
    int wall_axis = -1, wall_face = 0;
    for (int a = 0; a < 3; ++a) {
      if (e[a] != 0 && (d[a] < 0 || d[a] >= n[a])) {
        if (g.bc[a] == LBM_BC_PERIODIC) {
          d[a] = d[a] < 0 ? d[a] + n[a] : d[a] - n[a];
        } else if (wall_axis < 0) {
          wall_axis = a;
          wall_face = d[a] < 0 ? 0 : 1;
        }
      }
    }
    double v;
    if (wall_axis < 0)
      v = src.get(i, (int64_t)d[0] + (int64_t)g.nx * ((int64_t)d[1] + (int64_t)g.ny * d[2]));
    else
      v = src.get(OPP[i], cell) + (double)g.bb_add[wall_axis][wall_face][i];
    Store<S>::store(dst + (int64_t)i * g.spop + lat_cell(g, x, y, z), (float)v);
  }
}

// Export: density, velocity and post-stream populations of every cell.
template <int S>
__global__ __launch_bounds__(LBM_BLOCK) void k_readout(const typename Store<S>::T* __restrict__ lat,
                                                       const LatticeGeom g, float* rho_out,
                                                       float* vel_out, void* pops_out,
                                                       int pops_f64) {
  const int64_t cell = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  if (cell >= g.ncell) return;
  int x, y, z;
  cell_xyz(g, cell, x, y, z);
  float f[Q];
  gather_any<S>(lat, g, x, y, z, f);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += f[i];
    jx += EX[i] * f[i];
    jy += EY[i] * f[i];
    jz += EZ[i] * f[i];
  }
  const float rho = 1.0f + drho;
  if (rho_out) rho_out[cell] = rho;
  if (vel_out) {
    vel_out[cell] = jx / rho;
    vel_out[g.ncell + cell] = jy / rho;
    vel_out[2 * g.ncell + cell] = jz / rho;
  }
  if (pops_out) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (pops_f64)
        ((double*)pops_out)[(int64_t)i * g.ncell + cell] = wgt_d(i) + (double)f[i];
      else
        ((float*)pops_out)[(int64_t)i * g.ncell + cell] = wgt(i) + f[i];
    }
  }
}

// Sum of the per-workgroup partials (single workgroup, fixed order).
__global__ __launch_bounds__(LBM_BLOCK) void k_reduce_sums(const double* __restrict__ partials,
                                                           int64_t nblocks, double ncell,
                                                           double* out) {
  double s[4] = {0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += LBM_BLOCK)
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += partials[b * 4 + k];
  __shared__ double red[4][LBM_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v = wave_sum(s[k]);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < LBM_BLOCK / 64; ++w) v += red[threadIdx.x][w];
    out[threadIdx.x] = threadIdx.x == 0 ? ncell + v : v;
  }
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy_f32(float* __restrict__ d, const float* __restrict__ s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// G of flagged blocks, zero elsewhere (G is only maintained where supports reach).
__global__ __launch_bounds__(LBM_BLOCK) void k_export_force(const float* __restrict__ G,
                                                            const uint8_t* __restrict__ flags,
                                                            const LatticeGeom g, float* out) {
  const int64_t cell = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  if (cell >= g.ncell) return;
  int x, y, z;
  cell_xyz(g, cell, x, y, z);
  const bool on = flags[fblock_of(g, x, y, z)] != 0;
  for (int c = 0; c < 3; ++c) out[c * g.ncell + cell] = on ? G[c * g.ncell + cell] : 0.0f;
}

int64_t cell_blocks(const lbm_ctx* c) { return (c->ncell + LBM_BLOCK - 1) / LBM_BLOCK; }

}  // namespace

// Launch shape of the stream-collide.  16-bit storage with an even x extent:
// the pair kernel, 256 threads over consecutive cell pairs of an x-y plane
// (a 2-byte access per lane reaches far less of the HBM bandwidth than a
// 4-byte one; for FP32 the pair form measured slower than one cell per
// thread).  Otherwise 256 threads, blockDim.x = the x extent rounded to a
// wavefront (at most 256), the rest of the block along y; for an x extent
// that is not a multiple of the wavefront, 256 consecutive cells of an x-y
// plane.  No shape has more blocks than ceil(nx / bx) * ceil(ny / by) * nz,
// the count the partial sums are sized for.
static bool stream_collide_pairs(const lbm_ctx* c) {
  return c->p.storage != LBM_STORE_F32 && c->p.nx % 2 == 0;
}
static bool stream_collide_flat(const lbm_ctx* c) { return c->p.nx % 64 != 0; }

void stream_collide_shape(const lbm_ctx* c, dim3& grid, dim3& block) {
  if (stream_collide_pairs(c)) {
    block = dim3(LBM_BLOCK, 1, 1);
    grid = dim3((unsigned)(((int64_t)(c->p.nx / 2) * c->p.ny + LBM_BLOCK - 1) / LBM_BLOCK), 1,
                c->p.nz);
    return;
  }
  if (stream_collide_flat(c)) {
    block = dim3(LBM_BLOCK, 1, 1);
    grid = dim3((unsigned)(((int64_t)c->p.nx * c->p.ny + LBM_BLOCK - 1) / LBM_BLOCK), 1, c->p.nz);
    return;
  }
  int bx = ((c->p.nx + 63) / 64) * 64;
  if (bx > LBM_BLOCK) bx = LBM_BLOCK;
  const int by = LBM_BLOCK / bx;
  block = dim3(bx, by, 1);
  const int rows = (c->p.ny + by - 1) / by;
  grid = dim3((c->p.nx + bx - 1) / bx, (rows + LBM_SC_ROWS - 1) / LBM_SC_ROWS, c->p.nz);
}

namespace {

template <int S>
hipError_t stream_collide_s(lbm_ctx* c) {
  using T = typename Store<S>::T;
  const T* src = (const T*)c->lat[c->cur];
  T* dst = (T*)c->lat[c->cur ^ 1];
  dim3 grid, block;
  stream_collide_shape(c, grid, block);
  if constexpr (S != LBM_STORE_F32) {
    {
      if (stream_collide_pairs(c) && c->geom.lat_elems * 2 < ((int64_t)1 << 32)) {
        if (c->p.forcing == LBM_FORCE_SHIFT)
          k_stream_collide_pairs<S, LBM_FORCE_SHIFT, true><<<grid, block, 0, c->stream>>>(
              src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
        else
          k_stream_collide_pairs<S, LBM_FORCE_GUO, true><<<grid, block, 0, c->stream>>>(
              src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
        return hipGetLastError();
      }
    }
    if (stream_collide_pairs(c)) {
      if (c->p.forcing == LBM_FORCE_SHIFT)
        k_stream_collide_pairs<S, LBM_FORCE_SHIFT><<<grid, block, 0, c->stream>>>(
            src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
      else
        k_stream_collide_pairs<S, LBM_FORCE_GUO><<<grid, block, 0, c->stream>>>(
            src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
      return hipGetLastError();
    }
  }
  const bool flat = stream_collide_flat(c);
  if constexpr (S == LBM_STORE_F32) {
    if (!flat && c->geom.lat_elems * 4 < ((int64_t)1 << 32)) {
      if (c->p.forcing == LBM_FORCE_SHIFT)
        k_stream_collide<S, LBM_FORCE_SHIFT, false, true><<<grid, block, 0, c->stream>>>(
            src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
      else
        k_stream_collide<S, LBM_FORCE_GUO, false, true><<<grid, block, 0, c->stream>>>(
            src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
      return hipGetLastError();
    }
  }
  if (c->p.forcing == LBM_FORCE_SHIFT) {
    if (flat)
      k_stream_collide<S, LBM_FORCE_SHIFT, true><<<grid, block, 0, c->stream>>>(
          src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
    else
      k_stream_collide<S, LBM_FORCE_SHIFT, false><<<grid, block, 0, c->stream>>>(
          src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
  } else {
    if (flat)
      k_stream_collide<S, LBM_FORCE_GUO, true><<<grid, block, 0, c->stream>>>(
          src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
    else
      k_stream_collide<S, LBM_FORCE_GUO, false><<<grid, block, 0, c->stream>>>(
          src, dst, c->geom, c->G, c->bflag, c->sum_partials, c->status);
  }
  return hipGetLastError();
}

template <int S, class Src>
hipError_t unstream_s(lbm_ctx* c, const Src& src) {
  using T = typename Store<S>::T;
  k_unstream<S, Src><<<(unsigned)cell_blocks(c), LBM_BLOCK, 0, c->stream>>>(
      (T*)c->lat[c->cur], c->geom, src);
  return hipGetLastError();
}

template <class Src>
hipError_t unstream_any(lbm_ctx* c, const Src& src) {
  switch (c->p.storage) {
    case LBM_STORE_F16: return unstream_s<LBM_STORE_F16>(c, src);
    case LBM_STORE_BF16: return unstream_s<LBM_STORE_BF16>(c, src);
    default: return unstream_s<LBM_STORE_F32>(c, src);
  }
}

}  // namespace

hipError_t launch_stream_collide(lbm_ctx* c) {
  hipError_t e;
  switch (c->p.storage) {
    case LBM_STORE_F16: e = stream_collide_s<LBM_STORE_F16>(c); break;
    case LBM_STORE_BF16: e = stream_collide_s<LBM_STORE_BF16>(c); break;
    default: e = stream_collide_s<LBM_STORE_F32>(c); break;
  }
  if (e == hipSuccess) c->cur ^= 1;
  return e;
}

hipError_t launch_init_equilibrium(lbm_ctx* c) {
  SrcUniform s;
  const double rho = c->p.rho0;
  const double* u = c->p.u0;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    const double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
    s.feq[i] = wgt_d(i) * (rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu) - 1.0);
  }
  return unstream_any(c, s);
}

hipError_t launch_unstream_from(lbm_ctx* c, const void* pops, int f64) {
  SrcPops s{pops, f64, c->ncell};
  return unstream_any(c, s);
}

hipError_t launch_readout(lbm_ctx* c, float* rho, float* vel, void* pops, int pops_f64) {
  const unsigned nb = (unsigned)cell_blocks(c);
  switch (c->p.storage) {
    case LBM_STORE_F16:
      k_readout<LBM_STORE_F16><<<nb, LBM_BLOCK, 0, c->stream>>>(
          (const _Float16*)c->lat[c->cur], c->geom, rho, vel, pops, pops_f64);
      break;
    case LBM_STORE_BF16:
      k_readout<LBM_STORE_BF16><<<nb, LBM_BLOCK, 0, c->stream>>>(
          (const uint16_t*)c->lat[c->cur], c->geom, rho, vel, pops, pops_f64);
      break;
    default:
      k_readout<LBM_STORE_F32><<<nb, LBM_BLOCK, 0, c->stream>>>(
          (const float*)c->lat[c->cur], c->geom, rho, vel, pops, pops_f64);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_sums(lbm_ctx* c, double* out4) {
  dim3 grid, block;
  stream_collide_shape(c, grid, block);
  k_reduce_sums<<<1, LBM_BLOCK, 0, c->stream>>>(c->sum_partials,
                                                (int64_t)grid.x * grid.y * grid.z,
                                                (double)c->ncell, out4);
  return hipGetLastError();
}

hipError_t launch_fill_u8(lbm_ctx* c, uint8_t* p, uint8_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  k_fill<uint8_t><<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, c->stream>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(lbm_ctx* c, uint32_t* p, uint32_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  k_fill<uint32_t><<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, c->stream>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_copy_f32(lbm_ctx* c, float* dst, const float* src, int64_t n) {
  if (n <= 0) return hipSuccess;
  k_copy_f32<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, c->stream>>>(dst, src, n);
  return hipGetLastError();
}

hipError_t launch_export_force(lbm_ctx* c, float* out) {
  k_export_force<<<(unsigned)cell_blocks(c), LBM_BLOCK, 0, c->stream>>>(c->G, c->bflag, c->geom, out);
  return hipGetLastError();
}
