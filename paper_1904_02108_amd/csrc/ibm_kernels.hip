// Forcing kernels: rigid motion of the Lagrangian points (§4.2, Algorithm 1),
// binning of the points by 8^3 tile, velocity near the surface (§5: U is
// needed only close to the object), interpolation / deficit / correction
// (§3, Algorithm 1) and spreading (§3, Algorithm 2), repeated for the sweeps
// of the multi-direct forcing.
//
// Work decomposition (instead of the paper's thread-per-point gather and
// block-per-point atomicAdd scatter):
//   * points are counting-sorted by the tile of their base cell floor(x)
//     ("owner" tile) and, in addition, listed in every tile their 4x4x4
//     support touches;
//   * interpolation: one workgroup per owner tile stages U over the tile and
//     its support halo (11^3 cells) in LDS, one thread per point;
//   * spreading: one workgroup per touched tile accumulates the contributions
//     of its listed points in LDS (LDS float atomics) and then writes the tile
//     with plain stores: no global atomics, every cell has one writer.
#include "internal.h"

using namespace lbmd;

namespace {

constexpr int BOX = TILE + 3;             // interpolation box edge: tile + taps -1..+2
constexpr int BOX3 = BOX * BOX * BOX;
constexpr int TILE3 = TILE * TILE * TILE;
constexpr int WG = 256;                   // threads of the per-tile point kernels

struct PointGeom {
  int n[3];
  int bc[3];
  int tiles[3];
  int fblk[3];
  int64_t ncell;
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Cell coordinate of a tap: wrapped on periodic axes; clamped into the box on
// walled axes (the surface is validated to keep its supports inside, so the
// clamp only guards memory against rounding at the validation margin).
__device__ __forceinline__ int tap_coord(int v, int n, int bc) {
  return bc == LBM_BC_PERIODIC ? wrap(v, n) : min(max(v, 0), n - 1);
}

// Per-body rotation coefficients for step n (theta_n = theta0 + omega n) and
// their change since step n-1, in FP64.
__global__ void k_body_motion(const double* __restrict__ bodies, int nb, int64_t step,
                              BodyMotion* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double* B = bodies + 8 * b;
  const double len = sqrt(B[3] * B[3] + B[4] * B[4] + B[5] * B[5]);
  const double th = B[6] + B[7] * (double)step;
  const double thp = B[6] + B[7] * (double)(step - 1);
  double s, c, sp, cp;
  sincos(th, &s, &c);
  sincos(thp, &sp, &cp);
  BodyMotion m;
  for (int a = 0; a < 3; ++a) {
    m.center[a] = B[a];
    m.axis[a] = B[3 + a] / len;
  }
  m.c = c;
  m.s = s;
  m.dc = c - cp;
  m.ds = s - sp;
  out[b] = m;
}

// Position (base cell and fraction) and velocity of one point (FP64):
// x = c + R r (Rodrigues), u_b = (R_n - R_{n-1}) r.
struct PointState {
  int base[3];
  float frac[3];
  float ub[3];
};

__device__ __forceinline__ PointState move_point(const BodyMotion& m, float4 r4,
                                                 const PointGeom& pg) {
  const double r[3] = {(double)r4.x, (double)r4.y, (double)r4.z};
  const double* a = m.axis;
  const double adr = a[0] * r[0] + a[1] * r[1] + a[2] * r[2];
  const double axr[3] = {a[1] * r[2] - a[2] * r[1], a[2] * r[0] - a[0] * r[2],
                         a[0] * r[1] - a[1] * r[0]};
  PointState ps;
  for (int k = 0; k < 3; ++k) {
    const double x = m.center[k] + r[k] * m.c + axr[k] * m.s + a[k] * adr * (1.0 - m.c);
    const double fl = floor(x);
    int b = (int)fl;
    float fr = (float)(x - fl);
    if (fr >= 1.0f) {  // x - floor(x) rounded up to 1 in FP32
      fr = 0.0f;
      b += 1;
    }
    if (pg.bc[k] == LBM_BC_PERIODIC) {
      b %= pg.n[k];
      if (b < 0) b += pg.n[k];
    } else {
      b = min(max(b, 0), pg.n[k] - 1);
    }
    ps.base[k] = b;
    ps.frac[k] = fr;
    ps.ub[k] = (float)(r[k] * m.dc + axr[k] * m.ds - a[k] * adr * m.dc);
  }
  return ps;
}

__device__ __forceinline__ uint32_t tile_index(const PointGeom& pg, int tx, int ty, int tz) {
  return (uint32_t)tx + (uint32_t)pg.tiles[0] * ((uint32_t)ty + (uint32_t)pg.tiles[1] * (uint32_t)tz);
}

// Distinct blocks (edge 2^shift) holding the four support cells base-1 ..
// base+2 along one axis: up to three when a short last block is crossed.
struct Span1 {
  int t0, t1, t2, n;
  __device__ __forceinline__ int at(int j) const { return j == 0 ? t0 : (j == 1 ? t1 : t2); }
};

__device__ __forceinline__ Span1 span_axis(int base, int n, int bc, int shift) {
  Span1 sp;
  sp.t0 = tap_coord(base - 1, n, bc) >> shift;
  sp.t1 = sp.t0;
  sp.t2 = sp.t0;
  sp.n = 1;
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    const int v = tap_coord(base - 1 + j, n, bc) >> shift;
    const bool fresh = v != sp.t0 && (sp.n < 2 || v != sp.t1) && (sp.n < 3 || v != sp.t2);
    if (fresh) {
      if (sp.n == 1) sp.t1 = v;
      else if (sp.n == 2) sp.t2 = v;
      sp.n = sp.n < 3 ? sp.n + 1 : 3;
    }
  }
  return sp;
}

// Wave-aggregated counter increment: lanes adding to the same counter are
// merged into one atomic; returns each lane's slot (old value + rank).
// Must be called by every lane of the wave (valid = false lanes take part).
__device__ __forceinline__ uint32_t agg_increment(uint32_t* counters, uint32_t key, bool valid) {
  const unsigned lane = __lane_id();
  unsigned long long active = __ballot(valid);
  uint32_t slot = 0;
  while (active) {
    const int leader = __ffsll(active) - 1;
    const uint32_t k0 = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(valid && key == k0) & active;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(&counters[k0], (uint32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if (valid && key == k0) slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    active &= ~same;
  }
  return slot;
}

// Pass 1: owner tile and rank of each point; count of points per touched tile.
__global__ __launch_bounds__(LBM_BLOCK) void k_point_count(
    const float4* __restrict__ rest, const int32_t* __restrict__ body_of,
    const BodyMotion* __restrict__ motion, int64_t npts, PointGeom pg, uint32_t* __restrict__ key,
    uint32_t* __restrict__ rank, uint32_t* __restrict__ cnt_own, uint32_t* __restrict__ cnt_touch) {
  const int64_t k = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  const bool valid = k < npts;
  PointState ps{};
  if (valid) ps = move_point(motion[body_of[k]], rest[k], pg);
  const uint32_t own = valid ? tile_index(pg, ps.base[0] >> TILE_SHIFT, ps.base[1] >> TILE_SHIFT,
                                          ps.base[2] >> TILE_SHIFT)
                             : 0u;
  const uint32_t r = agg_increment(cnt_own, own, valid);
  if (valid) {
    key[k] = own;
    rank[k] = r;
  }
  Span1 sx{0, 0, 0, 0}, sy{0, 0, 0, 0}, sz{0, 0, 0, 0};
  if (valid) {
    sx = span_axis(ps.base[0], pg.n[0], pg.bc[0], TILE_SHIFT);
    sy = span_axis(ps.base[1], pg.n[1], pg.bc[1], TILE_SHIFT);
    sz = span_axis(ps.base[2], pg.n[2], pg.bc[2], TILE_SHIFT);
  }
  for (int j = 0; j < 27; ++j) {
    const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
    const bool v = valid && jx < sx.n && jy < sy.n && jz < sz.n;
    if (!__ballot(v)) continue;
    const uint32_t t = v ? tile_index(pg, sx.at(jx), sy.at(jy), sz.at(jz)) : 0u;
    agg_increment(cnt_touch, t, v);
  }
}

// Pass 2 (one workgroup): exclusive scans of the owner and touch counts, the
// compact lists of tiles that own points / are touched, and clearing of the
// counters and force-block flags for this step.  Tiles are taken in chunks
// of SCAN_THREADS * SCAN_PER; each thread owns SCAN_PER consecutive tiles,
// waves scan their thread totals with shuffles, one wave scans the wave
// totals, and a running carry joins the chunks.
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_PER = 16;
constexpr int SCAN_WAVES = SCAN_THREADS / 64;
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(
    uint32_t* __restrict__ cnt_own, uint32_t* __restrict__ cnt_touch, uint32_t* __restrict__ fill,
    uint32_t* __restrict__ start_own, uint32_t* __restrict__ start_touch,
    uint32_t* __restrict__ own_tiles, uint32_t* __restrict__ touch_tiles,
    uint32_t* __restrict__ meta, uint32_t* __restrict__ bflag_words, int64_t nbflag_words,
    int64_t ntiles) {
  __shared__ uint32_t wtot[4][SCAN_WAVES];
  __shared__ uint32_t carry[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 4) carry[tid] = 0u;
  __syncthreads();
  for (int64_t c0 = 0; c0 < ntiles; c0 += (int64_t)SCAN_THREADS * SCAN_PER) {
    const int64_t t0 = c0 + (int64_t)tid * SCAN_PER;
    uint32_t a[SCAN_PER], b[SCAN_PER];
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
      const bool in = t0 + j < ntiles;
      a[j] = in ? cnt_own[t0 + j] : 0u;
      b[j] = in ? cnt_touch[t0 + j] : 0u;
    }
    uint32_t s[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
      s[0] += a[j];
      s[1] += b[j];
      s[2] += a[j] ? 1u : 0u;
      s[3] += b[j] ? 1u : 0u;
    }
    uint32_t inc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t v = s[q];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
      }
      inc[q] = v;
      if (lane == 63) wtot[q][wv] = v;
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t v = lane < SCAN_WAVES ? wtot[q][lane] : 0u;
#pragma unroll
        for (int off = 1; off < SCAN_WAVES; off <<= 1) {
          const uint32_t u = __shfl_up(v, off, 64);
          if (lane >= off) v += u;
        }
        if (lane < SCAN_WAVES) wtot[q][lane] = v;  // inclusive over waves
      }
    }
    __syncthreads();
    uint32_t run[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      run[q] = carry[q] + (wv ? wtot[q][wv - 1] : 0u) + inc[q] - s[q];
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
      const int64_t t = t0 + j;
      if (t < ntiles) {
        start_own[t] = run[0];
        start_touch[t] = run[1];
        if (a[j]) own_tiles[run[2]++] = (uint32_t)t;
        if (b[j]) touch_tiles[run[3]++] = (uint32_t)t;
        run[0] += a[j];
        run[1] += b[j];
        cnt_own[t] = 0u;
        cnt_touch[t] = 0u;
        fill[t] = 0u;
      }
    }
    __syncthreads();
    if (tid < 4) carry[tid] += wtot[tid][SCAN_WAVES - 1];
    __syncthreads();
  }
  if (tid == 0) {
    start_own[ntiles] = carry[0];
    start_touch[ntiles] = carry[1];
    meta[0] = carry[2];
    meta[1] = carry[3];
  }
  for (int64_t w = tid; w < nbflag_words; w += SCAN_THREADS) bflag_words[w] = 0u;
}

// Pass 3: move every point again (same arithmetic), store it at its slot in
// owner-tile order, append its slot to the lists of the tiles it touches, and
// flag the 4^3 force blocks of its support.  FP64 partial sums of s and
// s |u_b|^2 per workgroup.
__global__ __launch_bounds__(LBM_BLOCK) void k_point_scatter(
    const float4* __restrict__ rest, const int32_t* __restrict__ body_of,
    const BodyMotion* __restrict__ motion, int64_t npts, PointGeom pg,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
    const uint32_t* __restrict__ start_own, const uint32_t* __restrict__ start_touch,
    uint32_t* __restrict__ fill, uint32_t* __restrict__ tlist, int4* __restrict__ sp_base,
    float4* __restrict__ sp_frac, float4* __restrict__ sp_ub, uint8_t* __restrict__ bflag,
    double* __restrict__ part_s, double* __restrict__ part_sub2) {
  const int64_t k = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  const bool valid = k < npts;
  double ps_s = 0.0, ps_ub2 = 0.0;
  PointState ps{};
  uint32_t slot = 0;
  if (valid) {
    const float4 r4 = rest[k];
    ps = move_point(motion[body_of[k]], r4, pg);
    slot = start_own[key[k]] + rank[k];
    sp_base[slot] = make_int4(ps.base[0], ps.base[1], ps.base[2], (int)k);
    sp_frac[slot] = make_float4(ps.frac[0], ps.frac[1], ps.frac[2], r4.w);
    sp_ub[slot] = make_float4(ps.ub[0], ps.ub[1], ps.ub[2], 0.0f);
    // flag the force blocks of the support (idempotent byte stores)
    const Span1 fx = span_axis(ps.base[0], pg.n[0], pg.bc[0], FBLK_SHIFT);
    const Span1 fy = span_axis(ps.base[1], pg.n[1], pg.bc[1], FBLK_SHIFT);
    const Span1 fz = span_axis(ps.base[2], pg.n[2], pg.bc[2], FBLK_SHIFT);
    for (int cz = 0; cz < fz.n; ++cz)
      for (int cy = 0; cy < fy.n; ++cy)
        for (int cx = 0; cx < fx.n; ++cx)
          bflag[(int64_t)fx.at(cx) +
                (int64_t)pg.fblk[0] * ((int64_t)fy.at(cy) + (int64_t)pg.fblk[1] * fz.at(cz))] = 1u;
    ps_s = r4.w;
    ps_ub2 = (double)r4.w * ((double)ps.ub[0] * ps.ub[0] + (double)ps.ub[1] * ps.ub[1] +
                             (double)ps.ub[2] * ps.ub[2]);
  }
  Span1 sx{0, 0, 0, 0}, sy{0, 0, 0, 0}, sz{0, 0, 0, 0};
  if (valid) {
    sx = span_axis(ps.base[0], pg.n[0], pg.bc[0], TILE_SHIFT);
    sy = span_axis(ps.base[1], pg.n[1], pg.bc[1], TILE_SHIFT);
    sz = span_axis(ps.base[2], pg.n[2], pg.bc[2], TILE_SHIFT);
  }
  for (int j = 0; j < 27; ++j) {
    const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
    const bool v = valid && jx < sx.n && jy < sy.n && jz < sz.n;
    if (!__ballot(v)) continue;
    const uint32_t t = v ? tile_index(pg, sx.at(jx), sy.at(jy), sz.at(jz)) : 0u;
    const uint32_t pos = agg_increment(fill, t, v);
    if (v) tlist[start_touch[t] + pos] = slot;
  }
  __shared__ double red[2][LBM_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double a = wave_sum(ps_s), b = wave_sum(ps_ub2);
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int w = 0; w < LBM_BLOCK / 64; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    part_s[blockIdx.x] = sa;
    part_sub2[blockIdx.x] = sb;
  }
}

// Workgroup -> entry of a compact tile list.  Workgroups are dealt to the 8
// XCDs round-robin; this mapping gives each XCD a contiguous run of the list
// so that neighbouring tiles (which share halo cells) meet in the same L2.
__device__ __forceinline__ int64_t list_entry(uint32_t n_active) {
  const uint32_t chunk = (n_active + 7u) / 8u;
  const uint32_t xcd = blockIdx.x & 7u, idx = blockIdx.x >> 3;
  if (idx >= chunk) return -1;
  const uint32_t e = xcd * chunk + idx;
  return e < n_active ? (int64_t)e : -1;
}

__device__ __forceinline__ void tile_origin(const PointGeom& pg, uint32_t t, int o[3]) {
  o[0] = (int)(t % (uint32_t)pg.tiles[0]) * TILE;
  o[1] = (int)((t / (uint32_t)pg.tiles[0]) % (uint32_t)pg.tiles[1]) * TILE;
  o[2] = (int)(t / ((uint32_t)pg.tiles[0] * (uint32_t)pg.tiles[1])) * TILE;
}

// Velocity U = sum e f / rho (eq. 1) of the post-stream populations on the
// flagged 4^3 blocks of every touched tile (the paper's lbm_u_start limited
// to the cells the supports reach).  512 threads: one wave per 8x8 z-plane.
template <int S>
__global__ __launch_bounds__(TILE3) void k_moments_blocks(
    const typename Store<S>::T* __restrict__ lat, const LatticeGeom g, PointGeom pg,
    const uint32_t* __restrict__ touch_tiles, const uint32_t* __restrict__ meta,
    const uint8_t* __restrict__ bflag, float* __restrict__ U) {
  const int64_t e = list_entry(meta[1]);
  if (e < 0) return;
  int o[3];
  tile_origin(pg, touch_tiles[e], o);
  const int x = o[0] + (threadIdx.x & (TILE - 1));
  const int y = o[1] + ((threadIdx.x >> TILE_SHIFT) & (TILE - 1));
  const int z = o[2] + (threadIdx.x >> (2 * TILE_SHIFT));
  if (x >= g.nx || y >= g.ny || z >= g.nz) return;
  if (!bflag[fblock_of(g, x, y, z)]) return;
  float f[Q];
  gather_pull<S>(lat, g, x, y, z, f);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += f[i];
    jx += EX[i] * f[i];
    jy += EY[i] * f[i];
    jz += EZ[i] * f[i];
  }
  const float inv = 1.0f / (1.0f + drho);
  const int64_t cell = (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
  U[cell] = jx * inv;
  U[g.ncell + cell] = jy * inv;
  U[2 * g.ncell + cell] = jz * inv;
}

// 1-D weights of Peskin's 4-point kernel (§3) for the taps floor(x)-1 ..
// floor(x)+2 at fraction r in [0, 1): with q = sqrt(1 + 4r - 4r^2) the four
// distances 1+r, r, 1-r, 2-r give (3-2r-q)/8, (3-2r+q)/8, (1+2r+q)/8,
// (1+2r-q)/8.
__device__ __forceinline__ void peskin4(float r, float w[4]) {
  const float q = sqrtf(fmaxf(1.0f + 4.0f * r - 4.0f * r * r, 0.0f));
  w[0] = (3.0f - 2.0f * r - q) * 0.125f;
  w[1] = (3.0f - 2.0f * r + q) * 0.125f;
  w[2] = (1.0f + 2.0f * r + q) * 0.125f;
  w[3] = (1.0f + 2.0f * r - q) * 0.125f;
}

// Interpolation, deficit and correction for one sweep (§3; Algorithm 1):
// u = sum_taps U W, g = u_b - u, du = (first ? 0 : du) + s g.  One workgroup
// per tile that owns points; U of the tile plus halo staged in LDS.  FP64
// partial sum of s |g|^2 per workgroup (0 for idle workgroups).
__global__ __launch_bounds__(WG) void k_interp_tiles(
    const uint32_t* __restrict__ own_tiles, const uint32_t* __restrict__ meta,
    const uint32_t* __restrict__ start_own, const int4* __restrict__ sp_base,
    const float4* __restrict__ sp_frac, const float4* __restrict__ sp_ub,
    float4* __restrict__ sp_g, float4* __restrict__ sp_du, const float* __restrict__ U,
    PointGeom pg, int first, double* __restrict__ part_res) {
  __shared__ float sUx[BOX3], sUy[BOX3], sUz[BOX3];
  __shared__ double red[WG / 64];
  double res = 0.0;
  const int64_t e = list_entry(meta[0]);
  if (e >= 0) {
    const uint32_t t = own_tiles[e];
    int o[3];
    tile_origin(pg, t, o);
#pragma unroll 2
    for (int i = threadIdx.x; i < BOX3; i += WG) {
      const int bx = i % BOX, by = (i / BOX) % BOX, bz = i / (BOX * BOX);
      const int cx = tap_coord(o[0] - 1 + bx, pg.n[0], pg.bc[0]);
      const int cy = tap_coord(o[1] - 1 + by, pg.n[1], pg.bc[1]);
      const int cz = tap_coord(o[2] - 1 + bz, pg.n[2], pg.bc[2]);
      const int64_t c = (int64_t)cx + (int64_t)pg.n[0] * ((int64_t)cy + (int64_t)pg.n[1] * cz);
      sUx[i] = U[c];
      sUy[i] = U[pg.ncell + c];
      sUz[i] = U[2 * pg.ncell + c];
    }
    __syncthreads();
    const uint32_t p0 = start_own[t], p1 = start_own[t + 1];
    for (uint32_t k = p0 + threadIdx.x; k < p1; k += WG) {
      const int4 b = sp_base[k];
      const float4 fr = sp_frac[k];
      float wx[4], wy[4], wz[4];
      peskin4(fr.x, wx);
      peskin4(fr.y, wy);
      peskin4(fr.z, wz);
      // box-local index of tap (-1, -1, -1): the box starts one cell before the tile
      const int l0 = (b.x - o[0]) + BOX * ((b.y - o[1]) + BOX * (b.z - o[2]));
      float u0 = 0.f, u1 = 0.f, u2 = 0.f;
#pragma unroll 1
      for (int cz = 0; cz < 4; ++cz) {
        const float wzc = cz == 0 ? wz[0] : (cz == 1 ? wz[1] : (cz == 2 ? wz[2] : wz[3]));
#pragma unroll
        for (int cy = 0; cy < 4; ++cy) {
          const float wyz = wzc * wy[cy];
          const int row = l0 + BOX * (cy + BOX * cz);
#pragma unroll
          for (int cx = 0; cx < 4; ++cx) {
            const float w = wyz * wx[cx];
            u0 += w * sUx[row + cx];
            u1 += w * sUy[row + cx];
            u2 += w * sUz[row + cx];
          }
        }
      }
      const float4 ub = sp_ub[k];
      const float g0 = ub.x - u0, g1 = ub.y - u1, g2 = ub.z - u2;
      float4 du = first ? make_float4(0.f, 0.f, 0.f, 0.f) : sp_du[k];
      du.x += fr.w * g0;
      du.y += fr.w * g1;
      du.z += fr.w * g2;
      sp_g[k] = make_float4(g0, g1, g2, 0.0f);
      sp_du[k] = du;
      res += (double)fr.w * ((double)g0 * g0 + (double)g1 * g1 + (double)g2 * g2);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double v = wave_sum(res);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < WG / 64; ++w) s += red[w];
    part_res[blockIdx.x] = s;
  }
}

// Spreading (§3; Algorithm 2) for one sweep: every touched tile sums
// v(k) W_k over its listed points in LDS, then
//   mode 0/1 (inner sweep, v = s g or g):  U += sum   on cells with a nonzero sum
//   mode 2   (final spread, v = du):       G  = sum   on every cell of the tile.
// The LDS sum is kept in 32-bit fixed point (integer LDS atomics are fast on
// CDNA; float ones are not) with a per-tile unit B / 2^30, where
// B = (1/8) sum_k max_c |v_k,c| bounds every cell's sum (a tap weight is at
// most 1/8), so it cannot overflow; integer addition also makes the result
// independent of the order of the atomics.
constexpr float FIX_ONE = 1073741824.0f;  // 2^30
__global__ __launch_bounds__(WG) void k_spread_tiles(
    const uint32_t* __restrict__ touch_tiles, const uint32_t* __restrict__ meta,
    const uint32_t* __restrict__ start_touch, const uint32_t* __restrict__ tlist,
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_frac,
    const float4* __restrict__ vsrc, float* __restrict__ target, PointGeom pg, int mode) {
  __shared__ int acc[3][TILE3];
  __shared__ float red[WG / 64];
  const int64_t e = list_entry(meta[1]);
  if (e < 0) return;
  const uint32_t t = touch_tiles[e];
  int o[3];
  tile_origin(pg, t, o);
  for (int i = threadIdx.x; i < 3 * TILE3; i += WG) (&acc[0][0])[i] = 0;
  const uint32_t q0 = start_touch[t], L = start_touch[t + 1] - q0;
  // bound of the cell sums
  float bsum = 0.0f;
  for (uint32_t i = threadIdx.x; i < L; i += WG) {
    const uint32_t k = tlist[q0 + i];
    const float4 v = vsrc[k];
    const float sc = mode == 0 ? sp_frac[k].w : 1.0f;
    bsum += sc * fmaxf(fabsf(v.x), fmaxf(fabsf(v.y), fabsf(v.z)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bsum;
  __syncthreads();
  float B = 0.0f;
#pragma unroll
  for (int w = 0; w < WG / 64; ++w) B += red[w];
  B *= 0.125f;
  const float scale = B > 0.0f ? FIX_ONE / B : 0.0f;
  // Neighbouring list entries are neighbouring points; a stride coprime to
  // the list length deals them to lanes in scattered order so that the lanes
  // of a wave rarely add into the same LDS word at once.
  const uint32_t P = (L % 97u) ? 97u : 89u;
  for (uint32_t i = threadIdx.x; i < L; i += WG) {
    const uint32_t k = tlist[q0 + (uint32_t)(((uint64_t)i * P) % L)];
    const int4 b = sp_base[k];
    const float4 fr = sp_frac[k];
    float4 v = vsrc[k];
    const float vs = (mode == 0 ? fr.w : 1.0f) * scale;
    v.x *= vs;
    v.y *= vs;
    v.z *= vs;
    float wx[4], wy[4], wz[4];
    peskin4(fr.x, wx);
    peskin4(fr.y, wy);
    peskin4(fr.z, wz);
    int lx[4], ly[4], lz[4];  // tile-local tap coordinates, -1 when outside the tile
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cx = tap_coord(b.x - 1 + j, pg.n[0], pg.bc[0]) - o[0];
      const int cy = tap_coord(b.y - 1 + j, pg.n[1], pg.bc[1]) - o[1];
      const int cz = tap_coord(b.z - 1 + j, pg.n[2], pg.bc[2]) - o[2];
      lx[j] = (cx >= 0 && cx < TILE) ? cx : -1;
      ly[j] = (cy >= 0 && cy < TILE) ? cy : -1;
      lz[j] = (cz >= 0 && cz < TILE) ? cz : -1;
    }
#pragma unroll
    for (int cz = 0; cz < 4; ++cz) {
#pragma unroll
      for (int cy = 0; cy < 4; ++cy) {
        const float wyz = wz[cz] * wy[cy];
        const int row = TILE * (ly[cy] + TILE * lz[cz]);
        const bool in_yz = (ly[cy] | lz[cz]) >= 0;
#pragma unroll
        for (int cx = 0; cx < 4; ++cx) {
          if (in_yz && lx[cx] >= 0) {
            const float w = wyz * wx[cx];
            const int idx = row + lx[cx];
            atomicAdd(&acc[0][idx], __float2int_rn(w * v.x));
            atomicAdd(&acc[1][idx], __float2int_rn(w * v.y));
            atomicAdd(&acc[2][idx], __float2int_rn(w * v.z));
          }
        }
      }
    }
  }
  __syncthreads();
  const float unit = B / FIX_ONE;
  for (int i = threadIdx.x; i < TILE3; i += WG) {
    const int x = o[0] + (i & (TILE - 1)), y = o[1] + ((i >> TILE_SHIFT) & (TILE - 1)),
              z = o[2] + (i >> (2 * TILE_SHIFT));
    if (x >= pg.n[0] || y >= pg.n[1] || z >= pg.n[2]) continue;
    const int64_t c = (int64_t)x + (int64_t)pg.n[0] * ((int64_t)y + (int64_t)pg.n[1] * z);
    const int a0 = acc[0][i], a1 = acc[1][i], a2 = acc[2][i];
    if (mode == 2) {
      target[c] = (float)a0 * unit;
      target[pg.ncell + c] = (float)a1 * unit;
      target[2 * pg.ncell + c] = (float)a2 * unit;
    } else if (a0 != 0 || a1 != 0 || a2 != 0) {
      target[c] += (float)a0 * unit;
      target[pg.ncell + c] += (float)a1 * unit;
      target[2 * pg.ncell + c] += (float)a2 * unit;
    }
  }
}

// Sum of per-workgroup partials: row r holds n_r doubles (rows 0-1: n_a,
// rows >= 2: n_b) at stride row_stride.
__global__ __launch_bounds__(LBM_BLOCK) void k_reduce_rows(const double* __restrict__ part,
                                                           int64_t n_a, int64_t n_b,
                                                           int64_t row_stride,
                                                           double* __restrict__ out) {
  const double* row = part + (int64_t)blockIdx.x * row_stride;
  const int64_t nblk = blockIdx.x < 2 ? n_a : n_b;
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += LBM_BLOCK) s += row[b];
  __shared__ double red[LBM_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double v = wave_sum(s);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < LBM_BLOCK / 64; ++w) t += red[w];
    out[blockIdx.x] = t;
  }
}

// Sorted point arrays back to the caller's order.
__global__ __launch_bounds__(LBM_BLOCK) void k_export_points(
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_frac,
    const float4* __restrict__ sp_ub, const float4* __restrict__ sp_g,
    const float4* __restrict__ sp_du, int64_t npts, double* x, float* ub, float* g, float* du) {
  const int64_t k = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  if (k >= npts) return;
  const int4 b = sp_base[k];
  const int64_t o = b.w;
  if (x) {
    const float4 fr = sp_frac[k];
    x[3 * o] = (double)b.x + (double)fr.x;
    x[3 * o + 1] = (double)b.y + (double)fr.y;
    x[3 * o + 2] = (double)b.z + (double)fr.z;
  }
  if (ub) {
    const float4 v = sp_ub[k];
    ub[3 * o] = v.x;
    ub[3 * o + 1] = v.y;
    ub[3 * o + 2] = v.z;
  }
  if (g) {
    const float4 v = sp_g[k];
    g[3 * o] = v.x;
    g[3 * o + 1] = v.y;
    g[3 * o + 2] = v.z;
  }
  if (du) {
    const float4 v = sp_du[k];
    du[3 * o] = v.x;
    du[3 * o + 1] = v.y;
    du[3 * o + 2] = v.z;
  }
}

PointGeom point_geom(const lbm_ctx* c) {
  PointGeom pg;
  pg.n[0] = c->p.nx;
  pg.n[1] = c->p.ny;
  pg.n[2] = c->p.nz;
  for (int a = 0; a < 3; ++a) {
    pg.bc[a] = c->p.bc[a];
    pg.tiles[a] = c->tiles[a];
    pg.fblk[a] = c->fblk[a];
  }
  pg.ncell = c->ncell;
  return pg;
}

#define LAUNCH_CHECK()                     \
  do {                                     \
    hipError_t e_ = hipGetLastError();     \
    if (e_ != hipSuccess) return e_;       \
  } while (0)

}  // namespace

// Grid of the compact-list kernels: a multiple of 8 workgroups (one per XCD
// slot) covering every tile.
int64_t forcing_list_grid(const lbm_ctx* c) { return (c->ntiles + 7) / 8 * 8; }

// The forcing of one time step: motion, binning, U near the surface,
// n_iter sweeps of interpolation + correction with n_iter - 1 intermediate
// spreads into U and the final spread of du into G.
hipError_t launch_forcing(lbm_ctx* c) {
  const PointGeom pg = point_geom(c);
  const int64_t n = c->npts;
  const unsigned nb = (unsigned)((n + LBM_BLOCK - 1) / LBM_BLOCK);
  const unsigned lg = (unsigned)forcing_list_grid(c);
  const int64_t rs = c->part_row;  // row stride of pt_partials
  hipStream_t st = c->stream;

  k_body_motion<<<(c->nbodies + 63) / 64, 64, 0, st>>>(c->bodies, c->nbodies, c->step, c->motion);
  LAUNCH_CHECK();
  k_point_count<<<nb, LBM_BLOCK, 0, st>>>(c->rest, c->body_of, c->motion, n, pg, c->key, c->rank,
                                          c->cnt_own, c->cnt_touch);
  LAUNCH_CHECK();
  k_scan_tiles<<<1, SCAN_THREADS, 0, st>>>(c->cnt_own, c->cnt_touch, c->fill, c->start_own,
                                           c->start_touch, c->own_tiles, c->touch_tiles, c->meta,
                                           (uint32_t*)c->bflag, c->nbflag_words, c->ntiles);
  LAUNCH_CHECK();
  k_point_scatter<<<nb, LBM_BLOCK, 0, st>>>(c->rest, c->body_of, c->motion, n, pg, c->key, c->rank,
                                            c->start_own, c->start_touch, c->fill, c->tlist,
                                            c->sp_base, c->sp_frac, c->sp_ub, c->bflag,
                                            c->pt_partials, c->pt_partials + rs);
  LAUNCH_CHECK();
  switch (c->p.storage) {
    case LBM_STORE_F16:
      k_moments_blocks<LBM_STORE_F16><<<lg, TILE3, 0, st>>>(
          (const _Float16*)c->lat[c->cur], c->geom, pg, c->touch_tiles, c->meta, c->bflag, c->U);
      break;
    case LBM_STORE_BF16:
      k_moments_blocks<LBM_STORE_BF16><<<lg, TILE3, 0, st>>>(
          (const uint16_t*)c->lat[c->cur], c->geom, pg, c->touch_tiles, c->meta, c->bflag, c->U);
      break;
    default:
      k_moments_blocks<LBM_STORE_F32><<<lg, TILE3, 0, st>>>(
          (const float*)c->lat[c->cur], c->geom, pg, c->touch_tiles, c->meta, c->bflag, c->U);
  }
  LAUNCH_CHECK();
  const int inner_mode = (c->flags & IBM_INNER_UNWEIGHTED) ? 1 : 0;
  for (int it = 0; it < c->n_iter; ++it) {
    k_interp_tiles<<<lg, WG, 0, st>>>(c->own_tiles, c->meta, c->start_own, c->sp_base, c->sp_frac,
                                      c->sp_ub, c->sp_g, c->sp_du, c->U, pg, it == 0,
                                      c->pt_partials + (2 + it) * rs);
    LAUNCH_CHECK();
    if (it < c->n_iter - 1)
      k_spread_tiles<<<lg, WG, 0, st>>>(c->touch_tiles, c->meta, c->start_touch, c->tlist,
                                        c->sp_base, c->sp_frac, c->sp_g, c->U, pg, inner_mode);
    else
      k_spread_tiles<<<lg, WG, 0, st>>>(c->touch_tiles, c->meta, c->start_touch, c->tlist,
                                        c->sp_base, c->sp_frac, c->sp_du, c->G, pg, 2);
    LAUNCH_CHECK();
  }
  return hipSuccess;
}

hipError_t launch_reduce_point_stats(lbm_ctx* c, double* out) {
  const int64_t na = (c->npts + LBM_BLOCK - 1) / LBM_BLOCK;
  k_reduce_rows<<<(unsigned)(2 + c->n_iter), LBM_BLOCK, 0, c->stream>>>(
      c->pt_partials, na, forcing_list_grid(c), c->part_row, out);
  return hipGetLastError();
}

hipError_t launch_export_points(lbm_ctx* c, double* x, float* ub, float* g, float* du) {
  const unsigned nb = (unsigned)((c->npts + LBM_BLOCK - 1) / LBM_BLOCK);
  if (nb == 0) return hipSuccess;
  k_export_points<<<nb, LBM_BLOCK, 0, c->stream>>>(c->sp_base, c->sp_frac, c->sp_ub, c->sp_g,
                                                   c->sp_du, c->npts, x, ub, g, du);
  return hipGetLastError();
}
