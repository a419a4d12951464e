// Forcing kernels: rigid motion of the Lagrangian points (§4.2, Algorithm 1),
// binning of the points by 8^3 tile, velocity near the surface (§5: U is
// needed only close to the object), interpolation / deficit / correction
// (§3, Algorithm 1) and spreading (§3, Algorithm 2), repeated for the sweeps
// of the multi-direct forcing.
//
// Work decomposition (instead of the paper's thread-per-point gather and
// block-per-point atomicAdd scatter):
//   * points are counting-sorted by the tile of their base cell floor(x)
//     (their "owner" tile); tiles whose cells a support reaches are listed
//     as "touched";
//   * one sweep = two kernels.  k_sweep_tiles: one workgroup per owner tile
//     stages U over the 11^3 box that holds every tap of its points (tile
//     plus taps -1..+2), interpolates (one thread per point), forms the
//     deficit and correction, and spreads the vector of this sweep into an
//     11^3 box accumulator in LDS (integer atomics on a fixed-point unit),
//     which it stores.  k_merge_tiles: one workgroup per touched tile adds,
//     for each of its cells in a fixed order, the stored boxes covering it
//     and updates U (inner sweeps) or writes G (last sweep).  No global
//     atomics; every cell has one writer; results do not depend on timing.
#include "internal.h"

using namespace lbmd;

namespace {

constexpr int BOX = TILE + 3;             // interpolation box edge: tile + taps -1..+2
constexpr int BOX3 = BOX * BOX * BOX;
// a point's first tap is box cell l0 = lx + BOX (ly + BOX lz) with its local
// cell (lx, ly, lz) in 0..TILE-1; its taps add 0..3 per axis: all in the box
static_assert((TILE - 1 + 3) * (1 + BOX + BOX * BOX) == BOX3 - 1, "taps inside the box");
constexpr int TILE3 = TILE * TILE * TILE;
constexpr int WG = 256;                   // threads of the per-tile point kernels

// The slot of an owner tile's spread box in boxbuf (BOX_SLOT_BYTES): the
// packed x/y sums of the 11^3 cells (64-bit, as accumulated), the z sums
// (32-bit), the support mask (bit i set when cell i of the box is a tap of
// some point of the tile; written once per forcing by k_tile_order), and the
// box's fixed-point unit B / 2^30 (FP32) in the slot's last word.
constexpr int BOX_Z_OFF = BOX3 * 8;
constexpr int BOX_MASK_WORDS = (BOX3 + 31) / 32;
constexpr int BOX_MASK_OFF = (BOX_Z_OFF + BOX3 * 4 + 7) / 8 * 8;
constexpr int BOX_UNIT_OFF = BOX_SLOT_BYTES - 4;
static_assert(BOX_MASK_OFF + BOX_MASK_WORDS * 4 <= BOX_UNIT_OFF, "box slot too small");

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
  if (bc == LBM_BC_PERIODIC) {
    if (v < 0 || v >= n) {  // any distance: boxes are wider than short axes
      v %= n;
      if (v < 0) v += n;
    }
    return v;
  }
  return min(max(v, 0), n - 1);
}

// Per-body rotation coefficients for step n (theta_n = theta0 + omega n) and
// their change since step n-1, in FP64, from the body's row (centre, axis,
// theta0, omega).
__device__ __forceinline__ BodyMotion body_motion(const double* __restrict__ B, int64_t step) {
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
  return m;
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

// Cell of a base position within its tile (x fastest).
__device__ __forceinline__ uint32_t local_cell(const int base[3]) {
  return (uint32_t)(base[0] & (TILE - 1)) +
         TILE * ((uint32_t)(base[1] & (TILE - 1)) + TILE * (uint32_t)(base[2] & (TILE - 1)));
}

// Pass 1: owner tile and rank of each point; flags of the touched tiles.
// The kernel also forms the bodies' motion for this step: into LDS for the
// bodies of the workgroup's points (a contiguous range, since every body owns
// a contiguous range of points; a thread computes its own body's when the
// range is longer than MOTION_LDS), and into `motion` for every body (body b
// by workgroup b mod the grid), for the later kernels of the forcing.
constexpr int MOTION_LDS = 32;
__global__ __launch_bounds__(LBM_BLOCK) void k_point_count(
    const float4* __restrict__ rest, const int32_t* __restrict__ body_of,
    const double* __restrict__ bodies, int nbodies, int64_t step,
    BodyMotion* __restrict__ motion, int64_t npts, PointGeom pg, uint32_t* __restrict__ key,
    uint32_t* __restrict__ rank, uint32_t* __restrict__ cnt_own, uint32_t* __restrict__ cnt_touch) {
  __shared__ BodyMotion sm[MOTION_LDS];
  for (int64_t b = blockIdx.x + (int64_t)threadIdx.x * gridDim.x; b < nbodies;
       b += (int64_t)LBM_BLOCK * gridDim.x)
    motion[b] = body_motion(bodies + 8 * b, step);
  const int64_t k0 = (int64_t)blockIdx.x * LBM_BLOCK;
  const int lo = body_of[k0], hi = body_of[min(k0 + LBM_BLOCK, npts) - 1];
  const bool in_lds = hi - lo < MOTION_LDS;
  if (in_lds && (int)threadIdx.x <= hi - lo)
    sm[threadIdx.x] = body_motion(bodies + 8 * (int64_t)(lo + (int)threadIdx.x), step);
  __syncthreads();
  const int64_t k = k0 + threadIdx.x;
  const bool valid = k < npts;
  PointState ps{};
  if (valid) {
    const int b = body_of[k];
    ps = move_point(in_lds ? sm[b - lo] : body_motion(bodies + 8 * (int64_t)b, step), rest[k],
                    pg);
  }
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
  // the tiles the support reaches are only flagged (the scan needs whether a
  // tile is touched, not how often): idempotent stores, no atomics
  if (valid)
    for (int jz = 0; jz < sz.n; ++jz)
      for (int jy = 0; jy < sy.n; ++jy)
        for (int jx = 0; jx < sx.n; ++jx) cnt_touch[tile_index(pg, sx.at(jx), sy.at(jy), sz.at(jz))] = 1u;
}

// Pass 2: exclusive scan of the owner counts and the compact lists of tiles
// that own points / are touched (with each owner tile's slot in its list;
// tiles with more points than a sweep workgroup has threads come first, so
// that their longer sweeps start first),
// in two launches: chunk totals, then the chunk rescans that write the
// outputs and clear the counters and this step's force-block flags, each
// workgroup scanning the (few) chunk totals itself (k_scan_write); in three
// when there are many chunks (a separate scan of the chunk totals,
// k_scan_chunks).  (One workgroup for the whole pass of a small tile grid
// was slower than two launches: a single CU issues every scattered load and
// store of the pass.)  The pass also writes the list lengths, to the device and
// to pinned host memory for the next forcing's grid sizes.  A chunk is
// SCAN_WG threads x SCAN_PER consecutive scan positions.
//
// The scan visits the tiles by 4 x 4 x 4 blocks of tiles (x fastest within a
// block, blocks x fastest): consecutive list entries, which the forcing
// kernels deal to one XCD in contiguous runs, are then neighbours in all
// three directions, and the U, box and lattice data the halos of a run
// share stay in that XCD's L2.  Positions of the padded block grid outside
// the tile grid hold no tile.
constexpr int SCAN_WG = 256, SCAN_PER = 8, SCAN_CHUNK = SCAN_WG * SCAN_PER;
constexpr int SB = 4;  // tiles per edge of a scan block

// Tile at scan position p, or -1.
__device__ __forceinline__ int64_t scan_tile(const PointGeom& pg, int64_t p) {
  const int64_t sb = p / (SB * SB * SB);
  const int w = (int)(p - sb * (SB * SB * SB));
  const int nbx = (pg.tiles[0] + SB - 1) / SB, nby = (pg.tiles[1] + SB - 1) / SB;
  const int64_t r = sb / nbx;
  const int x = SB * (int)(sb - r * nbx) + (w % SB);
  const int y = SB * (int)(r % nby) + ((w / SB) % SB);
  const int z = SB * (int)(r / nby) + (w / (SB * SB));
  if (x >= pg.tiles[0] || y >= pg.tiles[1] || z >= pg.tiles[2]) return -1;
  return (int64_t)x + (int64_t)pg.tiles[0] * ((int64_t)y + (int64_t)pg.tiles[1] * z);
}
constexpr int SCAN_WAVES = SCAN_WG / 64;
// scanned per tile: points owned, owner tile with more than HEAVY_TILE
// points, other owner tile, touched tile
constexpr int SCAN_NV = 4;
constexpr uint32_t HEAVY_TILE = WG;

template <int PER>
__device__ __forceinline__ void load_counts(const PointGeom& pg,
                                            const uint32_t* __restrict__ cnt_own,
                                            const uint32_t* __restrict__ cnt_touch, int64_t p0,
                                            int32_t tl[PER], uint32_t a[PER], uint32_t b[PER],
                                            uint32_t s[SCAN_NV]) {
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    tl[j] = (int32_t)scan_tile(pg, p0 + j);  // tile indices fit 31 bits
    a[j] = tl[j] >= 0 ? cnt_own[tl[j]] : 0u;
    b[j] = tl[j] >= 0 ? cnt_touch[tl[j]] : 0u;
  }
  s[0] = s[1] = s[2] = s[3] = 0u;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    s[0] += a[j];
    s[1] += a[j] > HEAVY_TILE ? 1u : 0u;
    s[2] += (a[j] && a[j] <= HEAVY_TILE) ? 1u : 0u;
    s[3] += b[j] ? 1u : 0u;
  }
}

// Workgroup-wide exclusive scan of SCAN_NV values per thread; tot: the sums.
template <int NW>
__device__ __forceinline__ void block_scan(const uint32_t s[SCAN_NV], uint32_t ex[SCAN_NV],
                                           uint32_t tot[SCAN_NV]) {
  __shared__ uint32_t wtot[SCAN_NV][NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc[SCAN_NV];
#pragma unroll
  for (int q = 0; q < SCAN_NV; ++q) {
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
#pragma unroll
  for (int q = 0; q < SCAN_NV; ++q) {
    uint32_t base = 0u, all = 0u;
    for (int w = 0; w < NW; ++w) {
      base += w < wv ? wtot[q][w] : 0u;
      all += wtot[q][w];
    }
    ex[q] = base + inc[q] - s[q];
    tot[q] = all;
  }
  __syncthreads();
}

// The outputs of a thread's PER scan positions, from its running offsets
// (run: points, heavy owner tiles, other owner tiles, touched tiles).
template <int PER>
__device__ __forceinline__ void write_scan(const int32_t tl[PER], const uint32_t a[PER],
                                           const uint32_t b[PER], uint32_t run[SCAN_NV],
                                           uint32_t* __restrict__ cnt_own,
                                           uint32_t* __restrict__ cnt_touch,
                                           uint32_t* __restrict__ start_own,
                                           uint32_t* __restrict__ end_own,
                                           int32_t* __restrict__ own_slot,
                                           uint32_t* __restrict__ own_tiles,
                                           uint32_t* __restrict__ touch_tiles) {
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int32_t t = tl[j];
    if (t >= 0) {
      start_own[t] = run[0];
      end_own[t] = run[0] + a[j];
      int32_t slot = -1;
      if (a[j]) slot = (int32_t)(a[j] > HEAVY_TILE ? run[1]++ : run[2]++);
      own_slot[t] = slot;
      if (slot >= 0) own_tiles[slot] = (uint32_t)t;
      if (b[j]) touch_tiles[run[3]++] = (uint32_t)t;
      run[0] += a[j];
      cnt_own[t] = 0u;
      cnt_touch[t] = 0u;
    }
  }
}

// List lengths from the scan totals: owner tiles, touched tiles, heavy owner
// tiles (listed first); the first two also to pinned host memory (nullable).
__device__ __forceinline__ void write_meta(const uint32_t tot[SCAN_NV], uint32_t* __restrict__ meta,
                                           uint32_t* __restrict__ meta_host) {
  meta[0] = tot[1] + tot[2];
  meta[1] = tot[3];
  meta[2] = tot[1];
  if (meta_host) {  // zero-copy: a plain (vector) store to pinned host memory
    meta_host[0] = tot[1] + tot[2];
    meta_host[1] = tot[3];
  }
}

__global__ __launch_bounds__(SCAN_WG) void k_scan_totals(PointGeom pg,
                                                         const uint32_t* __restrict__ cnt_own,
                                                         const uint32_t* __restrict__ cnt_touch,
                                                         uint32_t* __restrict__ chunk) {
  const int64_t p0 = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int32_t tl[SCAN_PER];
  uint32_t a[SCAN_PER], b[SCAN_PER], s[SCAN_NV], ex[SCAN_NV], tot[SCAN_NV];
  load_counts<SCAN_PER>(pg, cnt_own, cnt_touch, p0, tl, a, b, s);
  block_scan<SCAN_WAVES>(s, ex, tot);
  if (threadIdx.x < SCAN_NV) chunk[SCAN_NV * blockIdx.x + threadIdx.x] = tot[threadIdx.x];
}

// Scan of many chunk totals in one workgroup (in place: exclusive offsets);
// writes the list lengths.
constexpr int SCAN2_WG = 1024;
__global__ __launch_bounds__(SCAN2_WG) void k_scan_chunks(uint32_t* __restrict__ chunk, int64_t nch,
                                                          uint32_t* __restrict__ meta,
                                                          uint32_t* __restrict__ meta_host) {
  __shared__ uint32_t carry[SCAN_NV];
  if (threadIdx.x < SCAN_NV) carry[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nch; c0 += SCAN2_WG) {
    const int64_t c = c0 + threadIdx.x;
    uint32_t s[SCAN_NV], ex[SCAN_NV], tot[SCAN_NV];
#pragma unroll
    for (int q = 0; q < SCAN_NV; ++q) s[q] = c < nch ? chunk[SCAN_NV * c + q] : 0u;
    block_scan<SCAN2_WG / 64>(s, ex, tot);
    if (c < nch)
#pragma unroll
      for (int q = 0; q < SCAN_NV; ++q) chunk[SCAN_NV * c + q] = carry[q] + ex[q];
    __syncthreads();
    if (threadIdx.x < SCAN_NV) carry[threadIdx.x] += tot[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t tot[SCAN_NV] = {carry[0], carry[1], carry[2], carry[3]};
    write_meta(tot, meta, meta_host);
  }
}

// The chunk rescans.  FEW (at most SCAN_WG chunks): every workgroup scans the
// chunk totals itself and workgroup 0 writes the list lengths; otherwise the
// totals hold k_scan_chunks' offsets and meta its lengths.
#ifndef LBM_SCAN_FEW_CHUNKS
#define LBM_SCAN_FEW_CHUNKS 256
#endif
constexpr int64_t SCAN_FEW_CHUNKS = LBM_SCAN_FEW_CHUNKS;
static_assert(SCAN_FEW_CHUNKS <= SCAN_WG, "a thread per chunk total");
template <bool FEW>
__global__ __launch_bounds__(SCAN_WG) void k_scan_write(
    PointGeom pg, uint32_t* __restrict__ cnt_own, uint32_t* __restrict__ cnt_touch,
    const uint32_t* __restrict__ chunk, int64_t nch, uint32_t* __restrict__ start_own,
    uint32_t* __restrict__ end_own, int32_t* __restrict__ own_slot,
    uint32_t* __restrict__ own_tiles, uint32_t* __restrict__ touch_tiles,
    uint32_t* __restrict__ bflag_words, int64_t nbflag_words, uint32_t* __restrict__ meta,
    uint32_t* __restrict__ meta_host) {
  __shared__ uint32_t pre[SCAN_NV];
  uint32_t base[SCAN_NV], heavy;
  if constexpr (FEW) {
    uint32_t s[SCAN_NV], ex[SCAN_NV], tot[SCAN_NV];
#pragma unroll
    for (int q = 0; q < SCAN_NV; ++q)
      s[q] = (int64_t)threadIdx.x < nch ? chunk[SCAN_NV * threadIdx.x + q] : 0u;
    block_scan<SCAN_WAVES>(s, ex, tot);
    if (threadIdx.x == blockIdx.x)
#pragma unroll
      for (int q = 0; q < SCAN_NV; ++q) pre[q] = ex[q];
    if (blockIdx.x == 0 && threadIdx.x == 0) write_meta(tot, meta, meta_host);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SCAN_NV; ++q) base[q] = pre[q];
    heavy = tot[1];
  } else {
#pragma unroll
    for (int q = 0; q < SCAN_NV; ++q) base[q] = chunk[SCAN_NV * blockIdx.x + q];
    heavy = meta[2];
  }
  const int64_t p0 = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int32_t tl[SCAN_PER];
  uint32_t a[SCAN_PER], b[SCAN_PER], s[SCAN_NV], ex[SCAN_NV], tot[SCAN_NV];
  load_counts<SCAN_PER>(pg, cnt_own, cnt_touch, p0, tl, a, b, s);
  block_scan<SCAN_WAVES>(s, ex, tot);
  uint32_t run[SCAN_NV];
#pragma unroll
  for (int q = 0; q < SCAN_NV; ++q) run[q] = base[q] + ex[q];
  run[2] += heavy;  // the other owner tiles follow the heavy ones
  write_scan<SCAN_PER>(tl, a, b, run, cnt_own, cnt_touch, start_own, end_own, own_slot, own_tiles,
                       touch_tiles);
  // this chunk's share of the force-block flags
  const int64_t per = (nbflag_words + gridDim.x - 1) / gridDim.x;
  const int64_t w1 = min(nbflag_words, per * (blockIdx.x + 1));
  for (int64_t w = per * blockIdx.x + threadIdx.x; w < w1; w += SCAN_WG) bflag_words[w] = 0u;
}

// Pass 3: move every point again (same arithmetic), store it at its slot in
// owner-tile order (in the temporaries t_base, t_frac, t_ub; k_tile_order
// then orders each tile's points by cell) and flag the 4^3 force blocks of
// its support.  FP64 partial sums of s and s |u_b|^2 per workgroup.
__global__ __launch_bounds__(LBM_BLOCK) void k_point_scatter(
    const float4* __restrict__ rest, const int32_t* __restrict__ body_of,
    const BodyMotion* __restrict__ motion, int64_t npts, PointGeom pg,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
    const uint32_t* __restrict__ start_own, int4* __restrict__ t_base,
    float4* __restrict__ t_frac, float4* __restrict__ t_ub, uint8_t* __restrict__ bflag,
    double* __restrict__ part_s, double* __restrict__ part_sub2) {
  const int64_t k = (int64_t)blockIdx.x * LBM_BLOCK + threadIdx.x;
  double ps_s = 0.0, ps_ub2 = 0.0;
  if (k < npts) {
    const float4 r4 = rest[k];
    const PointState ps = move_point(motion[body_of[k]], r4, pg);
    const uint32_t slot = start_own[key[k]] + rank[k];
    t_base[slot] = make_int4(ps.base[0], ps.base[1], ps.base[2], (int)k);
    t_frac[slot] = make_float4(ps.frac[0], ps.frac[1], ps.frac[2], r4.w);
    t_ub[slot] = make_float4(ps.ub[0], ps.ub[1], ps.ub[2], 0.0f);
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

// Owner / touched tile entries of this workgroup in a launch of any
// multiple of 8 workgroups: XCD x takes the contiguous run
// [x chunk, (x + 1) chunk) of the list and its workgroups stride through it.
struct ListRange {
  uint32_t e, end, step;
};
__device__ __forceinline__ ListRange list_range(uint32_t n) {
  const uint32_t chunk = (n + 7u) / 8u, xcd = blockIdx.x & 7u;
  ListRange r;
  r.e = xcd * chunk + (blockIdx.x >> 3);
  r.end = min(n, (xcd + 1u) * chunk);
  r.step = gridDim.x >> 3;
  return r;
}

// Owner-tile entries of a sweep workgroup: the nh heavy tiles at the front
// of the list go one per workgroup to the first workgroups of the launch
// (dispatched first; each XCD takes a contiguous run of them); the others to
// the remaining workgroups as in list_range.  A grid too small for that
// interleaves every entry over all workgroups.
struct OwnOrder {
  uint32_t h, h_end, h_step;
  ListRange l;
  __device__ __forceinline__ bool next(uint32_t& e) {
    if (h < h_end) {
      e = h;
      h += h_step;
      return true;
    }
    if (l.e < l.end) {
      e = l.e;
      l.e += l.step;
      return true;
    }
    return false;
  }
};
__device__ __forceinline__ OwnOrder own_order(uint32_t n, uint32_t nh) {
  OwnOrder o;
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t H = (nh + 7u) / 8u * 8u;
  o.l.e = o.l.end = o.l.step = 0u;
  if (G < H + 8u) {
    o.h = b;
    o.h_end = n;
    o.h_step = G;
    return o;
  }
  // heavy entries, one per workgroup b < H, in contiguous runs per XCD
  // (workgroup b runs on XCD b mod 8)
  const uint32_t he = (b & 7u) * (H / 8u) + (b >> 3);
  o.h = he;
  o.h_end = (b < H && he < nh) ? he + 1u : he;
  o.h_step = 1u;
  if (b >= H) {
    const uint32_t m = n - nh, chunk = (m + 7u) / 8u, xcd = (b - H) & 7u;
    o.l.e = nh + xcd * chunk + ((b - H) >> 3);
    o.l.end = nh + min(m, (xcd + 1u) * chunk);
    o.l.step = (G - H) >> 3;
  }
  return o;
}

__device__ __forceinline__ void tile_origin(const PointGeom& pg, uint32_t t, int o[3]) {
  o[0] = (int)(t % (uint32_t)pg.tiles[0]) * TILE;
  o[1] = (int)((t / (uint32_t)pg.tiles[0]) % (uint32_t)pg.tiles[1]) * TILE;
  o[2] = (int)(t / ((uint32_t)pg.tiles[0] * (uint32_t)pg.tiles[1])) * TILE;
}

// Workgroup-wide exclusive scan of one value per thread (CELL_WG threads).
constexpr int CELL_WG = 256;
__device__ __forceinline__ uint32_t block_scan1(uint32_t v, uint32_t* __restrict__ wtot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  uint32_t base = 0u;
  for (int w = 0; w < wv; ++w) base += wtot[w];
  __syncthreads();
  return base + inc - v;
}

// Pass 4: the points of every owner tile ordered by their base cell (x
// fastest), from the temporaries into sp_base, sp_frac and sp_ub, with the
// LDS box index of the point's first tap in u_b's fourth word.  Lanes that
// interpolate neighbouring slots then read the same or neighbouring LDS
// words.  A counting sort in LDS: cell counts with the rank of each point
// within its cell (the order of equal cells is that of the LDS atomics), an
// exclusive scan over the 512 cells, the move.  The ranks of a thread's
// first ORDER_KEEP points stay in registers, further ones go through `rank`
// (free after the scatter).  Also the support mask of the tile's box (the
// cells its points' taps reach), in the box slot.
constexpr int ORDER_KEEP = 4;
static_assert(TILE3 == 2 * CELL_WG, "two cells per thread");
__global__ __launch_bounds__(CELL_WG) void k_tile_order(
    const uint32_t* __restrict__ own_tiles, const uint32_t* __restrict__ meta,
    const uint32_t* __restrict__ start_own, const uint32_t* __restrict__ end_own,
    const int4* __restrict__ t_base, const float4* __restrict__ t_frac,
    const float4* __restrict__ t_ub,
    uint32_t* __restrict__ rank, int4* __restrict__ sp_base, float4* __restrict__ sp_frac,
    float4* __restrict__ sp_ub, unsigned char* __restrict__ boxbuf) {
  __shared__ uint32_t hist[TILE3];
  __shared__ uint32_t wtot[CELL_WG / 64];
  __shared__ uint32_t smask[BOX_MASK_WORDS];
  __shared__ uint32_t drow[TILE * TILE];
  const ListRange lr = list_range(meta[0]);
  for (uint32_t e = lr.e; e < lr.end; e += lr.step) {
    const uint32_t t = own_tiles[e];
    const uint32_t p0 = start_own[t], P = end_own[t] - p0;
    hist[threadIdx.x] = 0u;
    hist[threadIdx.x + CELL_WG] = 0u;
    if (threadIdx.x < BOX_MASK_WORDS) smask[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t kr[ORDER_KEEP];
    uint32_t j = 0;
    for (uint32_t i = threadIdx.x; i < P; i += CELL_WG, ++j) {
      const int4 b = t_base[p0 + i];
      const int bb[3] = {b.x, b.y, b.z};
      const uint32_t c = local_cell(bb);
      const uint32_t r = atomicAdd(&hist[c], 1u);  // rank within the cell
      if (j < ORDER_KEEP) {
#pragma unroll
        for (int q = 0; q < ORDER_KEEP; ++q)
          if (q == (int)j) kr[q] = r;
      } else {
        rank[p0 + i] = r;
      }
    }
    __syncthreads();
    // the support mask: the tile's occupied cells dilated by the taps
    // -1 .. +2 per axis; in box coordinates a point at cell l reaches box
    // positions l .. l + 3.  Rows of 8 occupancy bits, dilated along x, then
    // the 4 x 4 rows around each box row.
    if (threadIdx.x < TILE * TILE) {
      uint32_t occ = 0u;
#pragma unroll
      for (int lx = 0; lx < TILE; ++lx) occ |= (hist[lx + TILE * threadIdx.x] ? 1u : 0u) << lx;
      drow[threadIdx.x] = occ | (occ << 1) | (occ << 2) | (occ << 3);
    }
    __syncthreads();
    if (threadIdx.x < BOX * BOX) {
      const int by = threadIdx.x % BOX, bz = threadIdx.x / BOX;
      uint32_t m = 0u;
#pragma unroll
      for (int cz = 0; cz < 4; ++cz)
#pragma unroll
        for (int cy = 0; cy < 4; ++cy) {
          const int ly = by - cy, lz = bz - cz;
          if (ly >= 0 && ly < TILE && lz >= 0 && lz < TILE) m |= drow[ly + TILE * lz];
        }
      const int bit = BOX * threadIdx.x;  // first cell of box row (by, bz)
      const int w = bit >> 5, sh = bit & 31;
      if (m) {
        atomicOr(&smask[w], m << sh);
        if (sh > 32 - BOX) atomicOr(&smask[w + 1], m >> (32 - sh));
      }
    }
    const uint32_t c0 = hist[2 * threadIdx.x], c1 = hist[2 * threadIdx.x + 1];
    const uint32_t ex = block_scan1(c0 + c1, wtot);  // (synchronises)
    hist[2 * threadIdx.x] = ex;
    hist[2 * threadIdx.x + 1] = ex + c0;
    __syncthreads();
    j = 0;
    for (uint32_t i = threadIdx.x; i < P; i += CELL_WG, ++j) {
      uint32_t r = 0u;
      if (j < ORDER_KEEP) {
#pragma unroll
        for (int q = 0; q < ORDER_KEEP; ++q)
          if (q == (int)j) r = kr[q];
      } else {
        r = rank[p0 + i];
      }
      const int4 b = t_base[p0 + i];
      const int bb[3] = {b.x, b.y, b.z};
      const uint32_t dst = p0 + hist[local_cell(bb)] + r;
      const float4 u = t_ub[p0 + i];
      // box index of the tap (-1, -1, -1): the box starts one cell before the tile
      const int l0 = (b.x & (TILE - 1)) + BOX * ((b.y & (TILE - 1)) + BOX * (b.z & (TILE - 1)));
      sp_base[dst] = b;
      sp_frac[dst] = t_frac[p0 + i];
      sp_ub[dst] = make_float4(u.x, u.y, u.z, __int_as_float(l0));
    }
    __syncthreads();  // the mask is complete; hist is cleared for the next tile
    if (threadIdx.x < BOX_MASK_WORDS)
      reinterpret_cast<uint32_t*>(boxbuf + (int64_t)e * BOX_SLOT_BYTES + BOX_MASK_OFF)[threadIdx.x] =
          smask[threadIdx.x];
  }
}

// U (the forcing's velocity scratch) is stored tile-major, one float4
// (x, y, z, 0) per cell: tile t holds its 512 cells (x fastest) as 8 KB of
// consecutive memory, so that a cell is one 16-byte access.
__device__ __forceinline__ int64_t u_index(uint32_t tile, int local) {
  return (int64_t)tile * TILE3 + local;
}
__device__ __forceinline__ int64_t u_index_cell(const PointGeom& pg, int x, int y, int z) {
  const uint32_t t = (uint32_t)(x >> TILE_SHIFT) +
                     (uint32_t)pg.tiles[0] * ((uint32_t)(y >> TILE_SHIFT) +
                                              (uint32_t)pg.tiles[1] * (uint32_t)(z >> TILE_SHIFT));
  const int l = (x & (TILE - 1)) + TILE * ((y & (TILE - 1)) + TILE * (z & (TILE - 1)));
  return u_index(t, l);
}

// Velocity U = sum e f / rho (eq. 1) of the post-stream populations at one
// cell, stored in the tile-major U array.  Every U pre-pass strategy uses
// this one function, so all of them give bit-identical values.
template <int S>
__device__ __forceinline__ void cell_velocity(const typename Store<S>::T* __restrict__ lat,
                                              const LatticeGeom& g, const PointGeom& pg, int x,
                                              int y, int z, float4* __restrict__ U) {
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
  const float inv = 1.0f / (1.0f + drho);
  U[u_index_cell(pg, x, y, z)] = make_float4(jx * inv, jy * inv, jz * inv, 0.0f);
}

// Boxes covering local coordinate l (0..7) of a tile along one axis when the
// tile and both neighbours are full tiles without a wrap: the own tile's box
// (position l + 1), the previous tile's when l <= 1 (position l + 9) and the
// next tile's when l == 7 (position 0).  nd: tile offset, nb: box position.
struct Cover1 {
  int nd[2], nb[2], n;
};
__device__ __forceinline__ Cover1 simple_cover(int l) {
  Cover1 c;
  c.nd[0] = 0;
  c.nb[0] = l + 1;
  c.n = 1;
  c.nd[1] = 0;
  c.nb[1] = 0;
  if (l <= 1) {
    c.nd[1] = -1;
    c.nb[1] = l + 9;
    c.n = 2;
  } else if (l == TILE - 1) {
    c.nd[1] = 1;
    c.n = 2;
  }
  return c;
}

// Whether tile coordinates tc and both neighbours on every axis are full
// tiles without a periodic wrap (the fast covering of simple_cover holds).
__device__ __forceinline__ bool simple_tile(const PointGeom& pg, const int tc[3]) {
  bool simple = true;
  for (int a = 0; a < 3; ++a) simple = simple && tc[a] >= 1 && (tc[a] + 2) * TILE <= pg.n[a];
  return simple;
}

// Owner-list slots and support masks of the 27 tiles around tile tc (slot
// -1 and an empty mask for a tile without points), into LDS; ends with a
// barrier.
template <int NT>
__device__ __forceinline__ void load_neighbour_masks(const PointGeom& pg, const int tc[3],
                                                     const int32_t* __restrict__ own_slot,
                                                     const unsigned char* __restrict__ boxbuf,
                                                     int32_t nslot[27],
                                                     uint32_t nmask[27][BOX_MASK_WORDS]) {
  if (threadIdx.x < 27) {
    const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
    nslot[threadIdx.x] = own_slot[tile_index(pg, tc[0] + dx, tc[1] + dy, tc[2] + dz)];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 27 * BOX_MASK_WORDS; i += NT) {
    const int nbr = i / BOX_MASK_WORDS, w = i - nbr * BOX_MASK_WORDS;
    const int32_t slot = nslot[nbr];
    nmask[nbr][w] = slot >= 0 ? reinterpret_cast<const uint32_t*>(
                                    boxbuf + (int64_t)slot * BOX_SLOT_BYTES + BOX_MASK_OFF)[w]
                              : 0u;
  }
  __syncthreads();
}

// U pre-pass, tile-mask strategy (default): the cells of the flagged 4^3
// blocks of every touched tile, i.e. the paper's lbm_u_start limited to the
// blocks the supports reach, and of those (away from seams and short axes)
// only the cells that are a tap of some point: the union of the support
// masks of the owner boxes covering the cell.  512 threads: one wave per 8x8
// z-plane.
template <int S>
__global__ __launch_bounds__(TILE3) void k_moments_blocks(
    const typename Store<S>::T* __restrict__ lat, const LatticeGeom g, PointGeom pg,
    const uint32_t* __restrict__ touch_tiles, const uint32_t* __restrict__ meta,
    const uint8_t* __restrict__ bflag, const int32_t* __restrict__ own_slot,
    const unsigned char* __restrict__ boxbuf, float4* __restrict__ U) {
  __shared__ int32_t nslot[27];
  __shared__ uint32_t nmask[27][BOX_MASK_WORDS];
  const ListRange lr = list_range(meta[1]);
  for (uint32_t e = lr.e; e < lr.end; e += lr.step) {
    int o[3], tc[3];
    tile_origin(pg, touch_tiles[e], o);
    for (int a = 0; a < 3; ++a) tc[a] = o[a] / TILE;
    const bool simple = simple_tile(pg, tc);
    __syncthreads();  // the previous tile's masks are no longer read
    if (simple) load_neighbour_masks<TILE3>(pg, tc, own_slot, boxbuf, nslot, nmask);
    const int lx = threadIdx.x & (TILE - 1), ly = (threadIdx.x >> TILE_SHIFT) & (TILE - 1),
              lz = threadIdx.x >> (2 * TILE_SHIFT);
    const int x = o[0] + lx, y = o[1] + ly, z = o[2] + lz;
    if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
    if (!bflag[fblock_of(g, x, y, z)]) continue;
    if (simple) {
      const Cover1 cx = simple_cover(lx), cy = simple_cover(ly), cz = simple_cover(lz);
      bool tap = false;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int jx = j & 1, jy = (j >> 1) & 1, jz = j >> 2;
        if (jx < cx.n && jy < cy.n && jz < cz.n) {
          const int ni = (cx.nd[jx] + 1) + 3 * (cy.nd[jy] + 1) + 9 * (cz.nd[jz] + 1);
          const int bi = cx.nb[jx] + BOX * (cy.nb[jy] + BOX * cz.nb[jz]);
          tap = tap || ((nmask[ni][bi >> 5] >> (bi & 31)) & 1u);
        }
      }
      if (!tap) continue;
    }
    cell_velocity<S>(lat, g, pg, x, y, z, U);
  }
}

// U pre-pass, box strategy (§5): for each body, the axis-aligned box of its
// rest-position bounding box (ubox: lo, hi relative to the centre) after the
// step's rotation, widened to the support cells floor(x)-1 .. floor(x)+2
// plus one cell.
// Workgroup blockIdx.x covers body blockIdx.x / sub^3 and the 8^3 sub-block
// blockIdx.x % sub^3 of a cube of edge 8 sub that bounds every rotation of
// the box; cells outside the moved box are skipped.  Cells of overlapping
// boxes are computed once per box (same value).
template <int S>
__global__ __launch_bounds__(TILE3) void k_moments_box(
    const typename Store<S>::T* __restrict__ lat, const LatticeGeom g, PointGeom pg,
    const BodyMotion* __restrict__ motion, const float* __restrict__ ubox, int sub,
    float4* __restrict__ U) {
  const int sub3 = sub * sub * sub;
  const int b = blockIdx.x / sub3, sblk = blockIdx.x - b * sub3;
  const BodyMotion m = motion[b];
  // moved box: the 8 corners of the rest box through the rotation
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  const double* a = m.axis;
  for (int corner = 0; corner < 8; ++corner) {
    const double r[3] = {(double)ubox[6 * b + ((corner & 1) ? 3 : 0)],
                         (double)ubox[6 * b + 1 + ((corner & 2) ? 3 : 0)],
                         (double)ubox[6 * b + 2 + ((corner & 4) ? 3 : 0)]};
    const double adr = a[0] * r[0] + a[1] * r[1] + a[2] * r[2];
    const double axr[3] = {a[1] * r[2] - a[2] * r[1], a[2] * r[0] - a[0] * r[2],
                           a[0] * r[1] - a[1] * r[0]};
    for (int k = 0; k < 3; ++k) {
      const double x = m.center[k] + r[k] * m.c + axr[k] * m.s + a[k] * adr * (1.0 - m.c);
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
  // support cells floor(x)-1 .. floor(x)+2, one more on each side so that a
  // point on the box's face cannot fall outside it by rounding
  int c0[3], c1[3];
  for (int k = 0; k < 3; ++k) {
    c0[k] = (int)floor(lo[k]) - 2;
    c1[k] = (int)floor(hi[k]) + 3;
  }
  const int sx = sblk % sub, sy = (sblk / sub) % sub, sz = sblk / (sub * sub);
  const int v[3] = {c0[0] + TILE * sx + (int)(threadIdx.x & (TILE - 1)),
                    c0[1] + TILE * sy + (int)((threadIdx.x >> TILE_SHIFT) & (TILE - 1)),
                    c0[2] + TILE * sz + (int)(threadIdx.x >> (2 * TILE_SHIFT))};
  int cxyz[3];
  for (int k = 0; k < 3; ++k) {
    if (v[k] > c1[k]) return;
    if (pg.bc[k] == LBM_BC_PERIODIC) {
      cxyz[k] = tap_coord(v[k], pg.n[k], LBM_BC_PERIODIC);
    } else {
      if (v[k] < 0 || v[k] >= pg.n[k]) return;
      cxyz[k] = v[k];
    }
  }
  cell_velocity<S>(lat, g, pg, cxyz[0], cxyz[1], cxyz[2], U);
}

// U pre-pass, kernel strategy (§5): one wave per point, one lane per cell of
// its 4^3 support (the paper uses a CUDA block per point's neighbourhood).
template <int S>
__global__ __launch_bounds__(WG) void k_moments_points(
    const typename Store<S>::T* __restrict__ lat, const LatticeGeom g, PointGeom pg,
    const int4* __restrict__ sp_base, int64_t npts, float4* __restrict__ U) {
  const int64_t k = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
  if (k >= npts) return;
  const int lane = threadIdx.x & 63;
  const int4 b = sp_base[k];
  const int x = tap_coord(b.x - 1 + (lane & 3), pg.n[0], pg.bc[0]);
  const int y = tap_coord(b.y - 1 + ((lane >> 2) & 3), pg.n[1], pg.bc[1]);
  const int z = tap_coord(b.z - 1 + (lane >> 4), pg.n[2], pg.bc[2]);
  cell_velocity<S>(lat, g, pg, x, y, z, U);
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

// One sweep of the multi-direct forcing for the points of one owner tile
// (§3; Algorithms 1 and 2), in parts chosen by the mode bits:
//   SW_INTERP:  u = sum_taps U W, g = u_b - u, du = (first ? 0 : du) + s g
//                                                                   (Alg. 1)
//   SW_SPREAD_G / SW_SPREAD_DU: the spread vector
//               v = s g (inner sweep), g (SW_UNWEIGHTED: paper-literal inner
//               sweep) or du (last sweep, or a predicted warm start), and
//               box(X) = sum_k v(k) W_k(X) over the tile's points     (Alg. 2)
// With neither spread bit only the interpolation runs; with SW_INTERP clear
// only the spread.  g_orig (nullable) receives g in the caller's order.
// U is staged over the 11^3 box [o-1, o+10)^3 that holds every tap of the
// tile's points (coordinates wrapped on periodic axes).  The box sum is
// accumulated in LDS in fixed point with the unit B / 2^30, where
// B = (1/8) sum_k max_c |v_k,c| bounds every box cell (a tap weight is at
// most 1/8; the sum is formed exactly in fixed point, bound_units): no
// overflow is possible and integer addition makes the box independent of the
// order of the atomics and of the points.  Components x and y share one
// 64-bit atomic (x sign-extended in the low word, y in the high word: the
// 64-bit sum is exactly sum_y 2^32 + sum_x, and |sum_x| < 2^31 recovers
// both), z has its own 32-bit one.  The box is stored as these integer sums
// with its unit in the tile's slot of boxbuf (box_slot layout); the merge
// converts them.
//
// Each workgroup takes a stride of the owner-tile list (contiguous per XCD;
// one tile per workgroup unless the list is longer than the grid).  A
// nonzero *gate (the forcing has converged) makes the launch a no-op.  Each
// workgroup writes its FP64 partial of s |g|^2 when interpolating.
constexpr float FIX_ONE = 1073741824.0f;  // 2^30


// Adds cell bi of a stored box to (s0, s1, s2): each sum times the unit.
__device__ __forceinline__ void add_box_cell(const unsigned char* __restrict__ slot, int bi,
                                             float& s0, float& s1, float& s2) {
  const float unit = *reinterpret_cast<const float*>(slot + BOX_UNIT_OFF);
  const unsigned long long xy = reinterpret_cast<const unsigned long long*>(slot)[bi];
  const int sx = (int)(uint32_t)xy;
  const int sy = (int)(uint32_t)((xy - (unsigned long long)(long long)sx) >> 32);
  const int sz = reinterpret_cast<const int*>(slot + BOX_Z_OFF)[bi];
  s0 += (float)sx * unit;
  s1 += (float)sy * unit;
  s2 += (float)sz * unit;
}

// A point's share of the box bound in units of 2^-32, rounded up, capped at
// SPREAD_CAP = 2^12 (far beyond any sound lattice velocity or correction):
// with up to 2^20 points per tile the 64-bit sum cannot overflow, and integer
// addition makes the bound independent of the order of the tile's points,
// which the binning does not fix.  The box bound B, and with it the promise
// that no fixed-point sum overflows, holds only while every point's
// max_c |v_c| is finite and at most the cap.  A larger or non-finite value
// (a diverging flow) would saturate the conversions, let the packed x sum
// carry into the y half and replace NaN by a finite number; spread_guard
// raises the sticky status word bad[1] for it instead of hiding it, and the
// forcing's results are then not valid.
constexpr float SPREAD_CAP = 4096.0f;
__device__ __forceinline__ unsigned long long bound_units(float m) {
  return (unsigned long long)ceilf(fminf(m, SPREAD_CAP) * 4294967296.0f);
}
// (each component on its own: fmaxf would drop a NaN operand)
__device__ __forceinline__ void spread_guard(float a, float b, float c, uint32_t* __restrict__ bad) {
  if (!(fabsf(a) <= SPREAD_CAP && fabsf(b) <= SPREAD_CAP && fabsf(c) <= SPREAD_CAP)) bad[1] = 1u;
}
enum : int {
  SW_INTERP = 1,
  SW_FIRST = 2,
  SW_SPREAD_G = 4,
  SW_SPREAD_DU = 8,
  SW_UNWEIGHTED = 16,
  SW_LOAD_PREV = 32,  // spreading du: take it from du_prev (caller order) into sp_du
  SW_SAVE_DU = 64,    // spreading du: also store it into du_prev (caller order)
  SW_STORE_G = 128,   // interpolating: store every point's g into sp_g
};

// The box's U as one float4 (x, y, z, 0) per cell, padded to whole waves of
// the staging (LDS direct loads write 64 consecutive cells per wave).
constexpr int BOX3P = (BOX3 + 63) / 64 * 64;
// Points whose spread vector a thread keeps in registers between the two
// passes (its first KEEP points of the tile; the fraction is read again);
// further points go through sp_g / sp_du.
constexpr int KEEP = 2;

struct KeptPoint {
  int l0;            // box index of the point's tap (-1, -1, -1)
  float v0, v1, v2;  // raw spread vector (g, or du when spreading du)
};

// w[c] for a lane-dependent c in 0..3, as two levels of selects (no branches).
__device__ __forceinline__ float sel4(const float w[4], int c) {
  const bool odd = c & 1;
  const float lo = odd ? w[1] : w[0], hi = odd ? w[3] : w[2];
  return (c & 2) ? hi : lo;
}

// The factor of a point's raw spread vector: s for the weighted inner sweep,
// 1 for the unweighted one and for du.
__device__ __forceinline__ float spread_weight(int mode, float s) {
  return ((mode & SW_SPREAD_DU) || (mode & SW_UNWEIGHTED)) ? 1.0f : s;
}

// Range check and bound term of the vector vs v that a point spreads.
__device__ __forceinline__ void spread_bound(const KeptPoint& kp, float vs,
                                             unsigned long long& bsum, uint32_t* __restrict__ bad) {
  const float a0 = vs * kp.v0, a1 = vs * kp.v1, a2 = vs * kp.v2;
  spread_guard(a0, a1, a2, bad);
  bsum += bound_units(fmaxf(fabsf(a0), fmaxf(fabsf(a1), fabsf(a2))));
}

// The interpolation pass of one point (§3; Algorithm 1): u = sum_taps U W
// from the staged box, g = u_b - u, du = (first ? 0 : du) + s g (stored);
// returns the raw spread vector and adds the residual and bound terms.
// The point's data as the interpolation reads them: fraction and s, u_b and
// box index, the du of the previous sweeps (zero in the first).
struct PointIn {
  float4 fr, ub, du;
};

__device__ __forceinline__ PointIn load_point_in(uint32_t k, const float4* __restrict__ sp_frac,
                                                 const float4* __restrict__ sp_ub,
                                                 const float4* __restrict__ sp_du, int mode) {
  PointIn pi;
  pi.fr = sp_frac[k];
  pi.ub = sp_ub[k];
  pi.du = (mode & SW_FIRST) ? make_float4(0.f, 0.f, 0.f, 0.f) : sp_du[k];
  return pi;
}

// PRE: the point's data come loaded in pin; else they are loaded here (du
// only after the taps, which keeps it out of the registers of the tap loop).
template <bool PRE>
__device__ __forceinline__ KeptPoint interp_point(
    uint32_t k, const PointIn& pin, const float4* __restrict__ sU,
    const float4* __restrict__ sp_frac, const float4* __restrict__ sp_ub,
    float4* __restrict__ sp_g, float4* __restrict__ sp_du, const int4* __restrict__ sp_base,
    float4* __restrict__ g_orig, int mode, bool store_g, double& res, unsigned long long& bsum,
    uint32_t* __restrict__ bad) {
  const float4 fr = PRE ? pin.fr : sp_frac[k];
  const float4 ub = PRE ? pin.ub : sp_ub[k];
  KeptPoint kp;
  kp.l0 = __float_as_int(ub.w);
  float wx[4], wy[4], wz[4];
  peskin4(fr.x, wx);
  peskin4(fr.y, wy);
  peskin4(fr.z, wz);
  float u0 = 0.f, u1 = 0.f, u2 = 0.f;
#pragma unroll 1
  for (int cz = 0; cz < 4; ++cz) {
    const float wzc = sel4(wz, cz);
#pragma unroll
    for (int cy = 0; cy < 4; ++cy) {
      const float wyz = wzc * wy[cy];
      const int row = kp.l0 + BOX * (cy + BOX * cz);
#pragma unroll
      for (int cx = 0; cx < 4; ++cx) {
        const float w = wyz * wx[cx];
        const float4 u = sU[row + cx];
        u0 += w * u.x;
        u1 += w * u.y;
        u2 += w * u.z;
      }
    }
  }
  const float g0 = ub.x - u0, g1 = ub.y - u1, g2 = ub.z - u2;
  const float s = fr.w;
  float4 du = PRE ? pin.du : ((mode & SW_FIRST) ? make_float4(0.f, 0.f, 0.f, 0.f) : sp_du[k]);
  du.x += s * g0;
  du.y += s * g1;
  du.z += s * g2;
  du.w = 0.0f;
  sp_du[k] = du;
  if (store_g) sp_g[k] = make_float4(g0, g1, g2, 0.0f);
  if (g_orig) g_orig[sp_base[k].w] = make_float4(g0, g1, g2, 0.0f);
  res += (double)s * ((double)g0 * g0 + (double)g1 * g1 + (double)g2 * g2);
  const bool spread_du = mode & SW_SPREAD_DU;
  kp.v0 = spread_du ? du.x : g0;
  kp.v1 = spread_du ? du.y : g1;
  kp.v2 = spread_du ? du.z : g2;
  const float vs = spread_weight(mode, s);
  const float a0 = vs * kp.v0, a1 = vs * kp.v1, a2 = vs * kp.v2;
  if (mode & (SW_SPREAD_G | SW_SPREAD_DU)) spread_guard(a0, a1, a2, bad);
  bsum += bound_units(fmaxf(fabsf(a0), fmaxf(fabsf(a1), fabsf(a2))));
  return kp;
}

// The raw spread vector of a point when no interpolation runs this sweep
// (spreading a predicted or previous du) or when the interpolation pass
// stored it: from sp_du or sp_g, or from du_prev in the caller's order (then
// also stored into sp_du).
__device__ __forceinline__ KeptPoint load_point(uint32_t k, const float4* __restrict__ sp_ub,
                                                const float4* __restrict__ sp_g,
                                                float4* __restrict__ sp_du,
                                                const int4* __restrict__ sp_base,
                                                const float4* __restrict__ du_prev, int mode) {
  KeptPoint kp;
  kp.l0 = __float_as_int(sp_ub[k].w);
  float4 v;
  if (mode & SW_SPREAD_DU) {
    if (mode & SW_LOAD_PREV) {
      v = du_prev[sp_base[k].w];
      sp_du[k] = v;  // read again only by later launches or this thread
    } else {
      v = sp_du[k];
    }
  } else {
    v = sp_g[k];
  }
  kp.v0 = v.x;
  kp.v1 = v.y;
  kp.v2 = v.z;
  return kp;
}

// Fixed-point spread of one point into the LDS accumulators: the raw vector
// times f (its weight times the box scale) times each tap weight, rounded to
// the fixed-point unit.  Lanes holding points of the same cell (the slots
// are in cell order) start at different rows of the 4 x 4 (y, z) tap rows,
// so that they rarely add into the same word at the same time.
__device__ __forceinline__ void spread_point(const KeptPoint& kp, float4 fr, float f,
                                             unsigned long long* __restrict__ accxy,
                                             int* __restrict__ accz, int rot) {
  float wx[4], wy[4], wz[4];
  peskin4(fr.x, wx);
  peskin4(fr.y, wy);
  peskin4(fr.z, wz);
  const float v0 = kp.v0 * f, v1 = kp.v1 * f, v2 = kp.v2 * f;
  // the x weights times the vector, once per point: a tap's value is then
  // one product per component, wz wy (wx v)
  float ax[4], ay[4], az[4];
#pragma unroll
  for (int cx = 0; cx < 4; ++cx) {
    ax[cx] = wx[cx] * v0;
    ay[cx] = wx[cx] * v1;
    az[cx] = wx[cx] * v2;
  }
#pragma unroll 1
  for (int j = 0; j < 16; ++j) {
    const int rr = (j + rot) & 15;
    const int cy = rr & 3, cz = rr >> 2;
    const float wyz = sel4(wz, cz) * sel4(wy, cy);
    const int row = kp.l0 + BOX * (cy + BOX * cz);
#pragma unroll
    for (int cx = 0; cx < 4; ++cx) {
      const int ix = __float2int_rn(wyz * ax[cx]), iy = __float2int_rn(wyz * ay[cx]);
      // x sign-extended in the low word, y added into the high word
      atomicAdd(&accxy[row + cx], (unsigned long long)(long long)ix +
                                      ((unsigned long long)(uint32_t)iy << 32));
      atomicAdd(&accz[row + cx], __float2int_rn(wyz * az[cx]));
    }
  }
}

// One sweep of the multi-direct forcing for the points of one owner tile
// (§3; Algorithms 1 and 2), in parts chosen by the mode bits:
//   SW_INTERP:  u = sum_taps U W, g = u_b - u, du = (first ? 0 : du) + s g
//                                                                   (Alg. 1)
//   SW_SPREAD_G / SW_SPREAD_DU: the spread vector
//               v = s g (inner sweep), g (SW_UNWEIGHTED: paper-literal inner
//               sweep) or du (last sweep, or a predicted warm start), and
//               box(X) = sum_k v(k) W_k(X) over the tile's points     (Alg. 2)
// With neither spread bit only the interpolation runs; with SW_INTERP clear
// only the spread.  g_orig (nullable) receives g in the caller's order.
// U is staged, by LDS direct loads, over the 11^3 box [o-1, o+10)^3 that
// holds every tap of the tile's points (coordinates wrapped on periodic
// axes).  The box sum is accumulated in LDS in fixed point with the unit
// B / 2^30, where B = (1/8) sum_k max_c |v_k,c| bounds every box cell (a tap
// weight is at most 1/8; the sum is formed exactly in fixed point,
// bound_units): no overflow is possible while every |v_k,c| is finite and at
// most SPREAD_CAP (else the status word is raised), and integer addition
// makes the box independent of the order of the atomics and of the points.
// Components x and y share one 64-bit atomic (x sign-extended in the low
// word, y in the high word: the 64-bit sum is exactly sum_y 2^32 + sum_x,
// and |sum_x| < 2^31 recovers both), z has its own 32-bit one.  The box is
// stored as these integer sums with its unit in the tile's slot of boxbuf
// (box_slot layout); the merge converts them.
//
// A thread handles the points i = threadIdx.x + WG j of the tile (in cell
// order, see k_tile_order) in both passes; the spread vectors of its first
// KEEP points stay in registers.  Each workgroup takes a stride of the
// owner-tile list (contiguous per XCD; one tile per workgroup unless the
// list is longer than the grid).  A nonzero *gate (the forcing has
// converged) makes the launch a no-op.  Each workgroup writes its FP64
// partial of s |g|^2 when interpolating.
//
// 21 KB of LDS per workgroup: 7 workgroups of 4 waves fit a CU.
//
// PREF (launches over few tiles, whose time is the chain of memory round
// trips of one workgroup): each thread's first point is loaded before the
// box is staged, the two loads overlapping, and its fraction is kept for the
// spread pass; more registers, so fewer waves per SIMD.
template <bool PREF>
__global__ __launch_bounds__(WG, PREF ? 4 : 7) void k_sweep_tiles(
    const uint32_t* __restrict__ own_tiles, const uint32_t* __restrict__ meta,
    const uint32_t* __restrict__ start_own, const uint32_t* __restrict__ end_own,
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_frac,
    const float4* __restrict__ sp_ub, float4* __restrict__ sp_g, float4* __restrict__ sp_du,
    const float4* __restrict__ U, unsigned char* __restrict__ boxbuf, PointGeom pg, int mode,
    double* __restrict__ part_res, const uint32_t* __restrict__ gate, float4* __restrict__ g_orig,
    float4* __restrict__ du_prev, uint32_t* __restrict__ bad) {
  // U of the box during the interpolation, then (same storage) the integer
  // accumulators of the spread: x and y packed in 64 bits, z in 32 bits
  __shared__ __align__(16) float4 sU[BOX3P];
  unsigned long long* accxy = reinterpret_cast<unsigned long long*>(sU);
  int* accz = reinterpret_cast<int*>(accxy + BOX3);
  static_assert(BOX3 * 12 <= BOX3P * 16, "accumulators fit the staged box");
  __shared__ unsigned long long bred[WG / 64];
  __shared__ double dred[WG / 64];
  // float4 index of the box's cells in the tile-major U: a sum of one term
  // per axis (the wrapped coordinate's tile times the tile stride plus its
  // position in the tile), tabulated once per tile
  __shared__ uint32_t uoff[3][BOX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (gate && *gate) return;  // the forcing has already converged
  const bool interp = mode & SW_INTERP;
  const bool spread = mode & (SW_SPREAD_G | SW_SPREAD_DU);
  const bool spread_du = mode & SW_SPREAD_DU;
  const bool save_du = spread_du && (mode & SW_SAVE_DU);
  const bool store_g = mode & SW_STORE_G;
  double res = 0.0;  // this thread's part of sum s |g|^2 over the workgroup's tiles
  OwnOrder order = own_order(meta[0], meta[2]);
  uint32_t e;
  while (order.next(e)) {
    const uint32_t t = own_tiles[e];
    // the point range is loaded before the box is staged (one memory round
    // trip fewer on the path of a lone tile)
    const uint32_t p0 = start_own[t], P = end_own[t] - p0;
    PointIn pf;
    if (PREF && interp && threadIdx.x < P)
      pf = load_point_in(p0 + threadIdx.x, sp_frac, sp_ub, sp_du, mode);
    int o[3];
    tile_origin(pg, t, o);
    __syncthreads();  // the previous tile's box has been stored
    if (interp && threadIdx.x < 3 * BOX) {
      const int a = threadIdx.x / BOX, b = threadIdx.x - a * BOX;
      const int v = tap_coord(o[a] - 1 + b, pg.n[a], pg.bc[a]);
      const uint32_t tstride = a == 0 ? 1u : (a == 1 ? (uint32_t)pg.tiles[0]
                                                     : (uint32_t)pg.tiles[0] * pg.tiles[1]);
      uoff[a][b] = (uint32_t)(v >> TILE_SHIFT) * tstride * TILE3 +
                   ((uint32_t)(v & (TILE - 1)) << (TILE_SHIFT * a));
    }
    __syncthreads();
    if (interp) {
      // wave w stages the 64-cell chunks w, w + 4, ...; the padding lanes of
      // the last chunk load cell 0 again into the unused tail
      for (int j = wave; j < BOX3P / 64; j += WG / 64) {
        const int i = j * 64 + lane;
        const int ii = i < BOX3 ? i : 0;
        const int bz = ii / (BOX * BOX), r = ii - bz * (BOX * BOX);
        const int by = r / BOX, bx = r - by * BOX;
        const float4* src = U + (uoff[0][bx] + uoff[1][by] + uoff[2][bz]);
        __builtin_amdgcn_global_load_lds(
            src, (__attribute__((address_space(3))) void*)(sU + __builtin_amdgcn_readfirstlane(j * 64)),
            16, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0): this wave's loads have landed in LDS
    }
    __syncthreads();
    // pass 1: interpolation, deficit, correction (or, spreading only, the
    // spread vectors); each thread keeps its first KEEP points
    unsigned long long bsum = 0ull;  // in units of 2^-32 (see bound_units)
    KeptPoint keep[KEEP];
#pragma unroll
    for (int q = 0; q < KEEP; ++q) {
      const uint32_t i = threadIdx.x + q * WG;
      keep[q].l0 = 0;
      if (i < P) {
        if (interp) {
          if (PREF && q == 0)
            keep[q] = interp_point<true>(p0 + i, pf, sU, sp_frac, sp_ub, sp_g, sp_du, sp_base,
                                         g_orig, mode, store_g, res, bsum, bad);
          else
            keep[q] = interp_point<false>(p0 + i, pf, sU, sp_frac, sp_ub, sp_g, sp_du, sp_base,
                                          g_orig, mode, store_g, res, bsum, bad);
        } else {
          keep[q] = load_point(p0 + i, sp_ub, sp_g, sp_du, sp_base, du_prev, mode);
          spread_bound(keep[q], spread_weight(mode, sp_frac[p0 + i].w), bsum, bad);
        }
      }
    }
    for (uint32_t i = threadIdx.x + KEEP * WG; i < P; i += WG) {
      if (interp) {
        // the spread pass reads this point's vector back from sp_g / sp_du
        (void)interp_point<false>(p0 + i, pf, sU, sp_frac, sp_ub, sp_g, sp_du, sp_base, g_orig,
                                  mode, store_g || (spread && !spread_du), res, bsum, bad);
      } else {
        const KeptPoint kp = load_point(p0 + i, sp_ub, sp_g, sp_du, sp_base, du_prev, mode);
        spread_bound(kp, spread_weight(mode, sp_frac[p0 + i].w), bsum, bad);
      }
    }
    if (!spread) continue;
    // block bound B: an exact integer sum, whatever the order of the points
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off, 64);
    if (lane == 0) bred[wave] = bsum;
    __syncthreads();  // also: the interpolation's reads of sU are done
    unsigned long long btot = 0ull;
#pragma unroll
    for (int w = 0; w < WG / 64; ++w) btot += bred[w];
    const float B = (float)((double)btot * 0x1p-32) * 0.125f;
    const float scale = B > 0.0f ? FIX_ONE / B : 0.0f;
    for (int i = threadIdx.x; i < BOX3; i += WG) {
      accxy[i] = 0ull;
      accz[i] = 0;
    }
    __syncthreads();
    // pass 2: spread into the box (every tap of an owned point is inside it)
    const int rot = lane & 15;
    auto spread_one = [&](const KeptPoint& kp, uint32_t k, bool prefetched) {
      const float4 fr = (PREF && prefetched) ? pf.fr : sp_frac[k];
      if (save_du) du_prev[sp_base[k].w] = make_float4(kp.v0, kp.v1, kp.v2, 0.f);
      spread_point(kp, fr, spread_weight(mode, fr.w) * scale, accxy, accz, rot);
    };
#pragma unroll
    for (int q = 0; q < KEEP; ++q) {
      const uint32_t i = threadIdx.x + q * WG;
      if (i < P) spread_one(keep[q], p0 + i, q == 0 && interp);
    }
    for (uint32_t i = threadIdx.x + KEEP * WG; i < P; i += WG)
      spread_one(load_point(p0 + i, sp_ub, sp_g, sp_du, sp_base, du_prev, mode & ~SW_LOAD_PREV),
                 p0 + i, false);
    __syncthreads();
    unsigned char* slot = boxbuf + (int64_t)e * BOX_SLOT_BYTES;
    unsigned long long* sxy = reinterpret_cast<unsigned long long*>(slot);
    int* sz = reinterpret_cast<int*>(slot + BOX_Z_OFF);
    for (int i = threadIdx.x; i < BOX3; i += WG) {
      sxy[i] = accxy[i];
      sz[i] = accz[i];
    }
    if (threadIdx.x == 0) *reinterpret_cast<float*>(slot + BOX_UNIT_OFF) = B / FIX_ONE;
  }
  if (interp) {  // this workgroup's residual partial (zero if it had no tile)
    const double rv = wave_sum(res);
    if (lane == 0) dred[wave] = rv;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sres = 0.0;
      for (int w = 0; w < WG / 64; ++w) sres += dred[w];
      part_res[blockIdx.x] = sres;
    }
  }
}

// Boxes covering one cell coordinate along one axis: the owner tiles A and
// box positions b with wrap(o_A - 1 + b) = x, b in [0, 11).  At most 11
// (only for axes shorter than the box); usually 1 or 2.
constexpr int MAXCOV = BOX;
__device__ __forceinline__ int covering(int x, int n, int bc, int ntiles_axis, int16_t* tt,
                                        int16_t* bb) {
  int cnt = 0;
  const int kmax = bc == LBM_BC_PERIODIC ? (BOX + n - 1) / n + 1 : 0;
  for (int k = -kmax; k <= kmax; ++k) {
    // origins o = 8 t with o + k n in [x - 9, x + 1]
    const int lo = x - 9 - k * n, hi = x + 1 - k * n;
    int t0 = lo <= 0 ? 0 : (lo + TILE - 1) / TILE;
    const int t1 = hi < 0 ? -1 : min(hi / TILE, ntiles_axis - 1);
    for (int tv = t0; tv <= t1 && cnt < MAXCOV; ++tv) {
      tt[cnt] = (int16_t)tv;
      bb[cnt] = (int16_t)(x - (TILE * tv + k * n) + 1);
      ++cnt;
    }
  }
  return cnt;
}

// Merge of the stored boxes into one touched tile: for every cell of a
// flagged force block, the sum over the boxes that cover it (fixed order):
//   mode 0: U += sum on cells with a nonzero sum;   mode 2: G = sum.
// (x + 0 = x exactly, so skipping zero sums changes no value of U.)
constexpr int MERGE_WG = 256;
__global__ __launch_bounds__(MERGE_WG) void k_merge_tiles(
    const uint32_t* __restrict__ touch_tiles, const uint32_t* __restrict__ meta,
    const int32_t* __restrict__ own_slot, const unsigned char* __restrict__ boxbuf,
    const uint8_t* __restrict__ bflag, float* __restrict__ G, float4* __restrict__ U,
    PointGeom pg, int mode, const uint32_t* __restrict__ gate) {
  __shared__ int16_t ct[3][TILE][MAXCOV], cb[3][TILE][MAXCOV];
  __shared__ int cn[3][TILE];
  __shared__ int32_t nslot[27];
  __shared__ uint8_t tflag[8];
  if (gate && *gate) return;  // the forcing has already converged
  const ListRange lr = list_range(meta[1]);
  for (uint32_t e = lr.e; e < lr.end; e += lr.step) {
    __syncthreads();  // the previous tile's covering tables are no longer read
    const uint32_t t = touch_tiles[e];
    int o[3], tc[3];
    tile_origin(pg, t, o);
    for (int a = 0; a < 3; ++a) tc[a] = o[a] / TILE;
    // Fast path: on every axis the tile and both neighbours are full tiles
    // without a wrap, so the boxes covering local coordinate l are the own
    // tile (position l + 1), the previous tile when l <= 1 (position l + 9)
    // and the next tile when l == 7 (position 0).
    bool simple = true;
    for (int a = 0; a < 3; ++a)
      simple = simple && tc[a] >= 1 && (tc[a] + 2) * TILE <= pg.n[a];
    if (simple) {
      // list slots of the 27 tiles around this one (the box units are
      // loaded with the box sums, one memory round trip fewer), and the
      // flags of the tile's eight force blocks
      if (threadIdx.x < 27) {
        const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
        nslot[threadIdx.x] = own_slot[tile_index(pg, tc[0] + dx, tc[1] + dy, tc[2] + dz)];
      } else if (threadIdx.x >= 64 && threadIdx.x < 72) {
        const int b = threadIdx.x - 64;
        const int bx = (o[0] >> FBLK_SHIFT) + (b & 1), by = (o[1] >> FBLK_SHIFT) + ((b >> 1) & 1),
                  bz = (o[2] >> FBLK_SHIFT) + (b >> 2);
        tflag[b] = bflag[(int64_t)bx + (int64_t)pg.fblk[0] * ((int64_t)by + (int64_t)pg.fblk[1] * bz)];
      }
      __syncthreads();
    } else {  // general covering tables (short axes, seams, short tiles)
      if (threadIdx.x < 3 * TILE) {
        const int a = threadIdx.x / TILE, l = threadIdx.x % TILE;
        const int x = o[a] + l;
        cn[a][l] = x < pg.n[a] ? covering(x, pg.n[a], pg.bc[a], pg.tiles[a], ct[a][l], cb[a][l]) : 0;
      }
      __syncthreads();
    }
    for (int cell = threadIdx.x; cell < TILE3; cell += MERGE_WG) {
      const int lx = cell & (TILE - 1), ly = (cell >> TILE_SHIFT) & (TILE - 1),
                lz = cell >> (2 * TILE_SHIFT);
      const int x = o[0] + lx, y = o[1] + ly, z = o[2] + lz;
      if (x >= pg.n[0] || y >= pg.n[1] || z >= pg.n[2]) continue;
      // only cells of flagged force blocks can receive a contribution, and
      // only there is G read by the stream-collide
      if (simple ? !tflag[(lx >> FBLK_SHIFT) + 2 * ((ly >> FBLK_SHIFT) + 2 * (lz >> FBLK_SHIFT))]
                 : !bflag[(int64_t)(x >> FBLK_SHIFT) +
                          (int64_t)pg.fblk[0] * ((int64_t)(y >> FBLK_SHIFT) +
                                                 (int64_t)pg.fblk[1] * (z >> FBLK_SHIFT))])
        continue;
      float4* uc = U + u_index(t, cell);
      // the old U is loaded with the boxes (latency overlapped)
      const float4 uold = mode == 2 ? make_float4(0.f, 0.f, 0.f, 0.f) : *uc;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
      if (simple) {
        const int l[3] = {lx, ly, lz};
        int nd[3][2], nb[3][2], nn[3];
  #pragma unroll
        for (int a = 0; a < 3; ++a) {
          nd[a][0] = 0;
          nb[a][0] = l[a] + 1;
          nn[a] = 1;
          nd[a][1] = 0;
          nb[a][1] = 0;
          if (l[a] <= 1) {
            nd[a][1] = -1;
            nb[a][1] = l[a] + 9;
            nn[a] = 2;
          } else if (l[a] == TILE - 1) {
            nd[a][1] = 1;
            nn[a] = 2;
          }
        }
        // every covering box's sums are loaded before any is added (all loads
        // in flight at once); absent boxes contribute exactly zero, which
        // leaves the sums bit-identical to skipping them
        unsigned long long xy[8];
        int zz[8];
        float un[8];
  #pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int jx = j & 1, jy = (j >> 1) & 1, jz = j >> 2;
          const bool in = jx < nn[0] && jy < nn[1] && jz < nn[2];
          const int ni = (nd[0][jx] + 1) + 3 * (nd[1][jy] + 1) + 9 * (nd[2][jz] + 1);
          const int32_t slot = in ? nslot[ni] : -1;
          xy[j] = 0ull;
          zz[j] = 0;
          un[j] = 0.0f;
          if (slot >= 0) {
            const unsigned char* sl = boxbuf + (int64_t)slot * BOX_SLOT_BYTES;
            const int bi = nb[0][jx] + BOX * (nb[1][jy] + BOX * nb[2][jz]);
            xy[j] = reinterpret_cast<const unsigned long long*>(sl)[bi];
            zz[j] = reinterpret_cast<const int*>(sl + BOX_Z_OFF)[bi];
            un[j] = *reinterpret_cast<const float*>(sl + BOX_UNIT_OFF);
          }
        }
  #pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int sx = (int)(uint32_t)xy[j];
          const int sy = (int)(uint32_t)((xy[j] - (unsigned long long)(long long)sx) >> 32);
          if (un[j] != 0.0f) {
            s0 += (float)sx * un[j];
            s1 += (float)sy * un[j];
            s2 += (float)zz[j] * un[j];
          }
        }
      } else {
        const int nx_ = cn[0][lx], ny_ = cn[1][ly], nz_ = cn[2][lz];
        for (int jz = 0; jz < nz_; ++jz)
          for (int jy = 0; jy < ny_; ++jy)
            for (int jx = 0; jx < nx_; ++jx) {
              const uint32_t A = tile_index(pg, ct[0][lx][jx], ct[1][ly][jy], ct[2][lz][jz]);
              const int32_t slot = own_slot[A];
              if (slot < 0) continue;
              const int bi = cb[0][lx][jx] + BOX * (cb[1][ly][jy] + BOX * cb[2][lz][jz]);
              add_box_cell(boxbuf + (int64_t)slot * BOX_SLOT_BYTES, bi, s0, s1, s2);
            }
      }
      if (mode == 2) {  // G, in the lattice layout read by the stream-collide
        const int64_t c = (int64_t)x + (int64_t)pg.n[0] * ((int64_t)y + (int64_t)pg.n[1] * z);
        G[c] = s0;
        G[pg.ncell + c] = s1;
        G[2 * pg.ncell + c] = s2;
      } else if (s0 != 0.0f || s1 != 0.0f || s2 != 0.0f) {  // U, tile-major
        *uc = make_float4(uold.x + s0, uold.y + s1, uold.z + s2, uold.w);
      }
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

// Residual-stopped forcing (ctl: [0] converged flag, [1] sweeps run).  After
// each sweep, unless already converged, R = sum_k s |g|^2 of the sweep is
// compared with thr = eps^2 sum_k s |u_b|^2 (both FP64, fixed order; thr is
// formed by the check of sweep 0); R <= thr, or the last allowed sweep, ends
// the forcing.  Comparing squared sums keeps a body at rest (both sums zero)
// converged without a division.  (A check inside the sweep by its last
// workgroup would need a device-scope release fence in every workgroup,
// which writes back the L2 and costs more than this launch.)
// One workgroup of RESID_WG threads sums the partials in a fixed order: each
// thread a strided subset (four loads in flight), then the waves.
constexpr int RESID_WG = 1024;
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int64_t n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t b = threadIdx.x;
  for (; b + 3 * RESID_WG < n; b += 4 * RESID_WG) {
    s0 += part[b];
    s1 += part[b + RESID_WG];
    s2 += part[b + 2 * RESID_WG];
    s3 += part[b + 3 * RESID_WG];
  }
  for (; b < n; b += RESID_WG) s0 += part[b];
  __shared__ double red[RESID_WG / 64];
  const double v = wave_sum((s0 + s1) + (s2 + s3));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < RESID_WG / 64; ++w) t += red[w];
  return t;  // the same on every thread
}

// Residual test after sweep `it`: sets ctl[1] = it + 1 and, once the sweep's
// sum s |g|^2 is within the threshold (or the sweep is the last), ctl[0] = 1,
// which gates off every later sweep and merge of the forcing.  The check of
// sweep 0 starts the forcing's control words and first forms the threshold
// eps^2 sum s |u_b|^2 from the binning's partials (part_sub2, na of them); a
// later check returns at once when ctl[0] is already set.
__global__ __launch_bounds__(RESID_WG) void k_resid_check(const double* __restrict__ part_res,
                                                          int64_t nblk,
                                                          const double* __restrict__ part_sub2,
                                                          int64_t na, double eps2,
                                                          double* __restrict__ thr, int it,
                                                          int last, int use_thr,
                                                          uint32_t* __restrict__ ctl) {
  double th;
  if (it == 0) {
    th = eps2 * sum_partials(part_sub2, na);
    if (threadIdx.x == 0) *thr = th;
  } else {
    if (ctl[0]) return;
    th = *thr;
  }
  const double t = sum_partials(part_res, nblk);
  if (threadIdx.x == 0) {
    ctl[1] = (uint32_t)(it + 1);
    ctl[0] = (last || (use_thr && t <= th)) ? 1u : 0u;
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
// Workgroups of the sweep, merge and U pre-pass launches over the owner
// (list 0) or touched (list 1) tiles: a multiple of 8, each XCD striding
// through its contiguous part of the list, so any size is correct.  The
// lists' lengths are known on the device only; the host sizes the grids from
// the lengths of a recent forcing (copied asynchronously to pinned memory at
// most every META_EVERY forcings, used once that copy has completed) with a
// quarter of headroom, so that
// idle or gated-off launches do not dispatch a workgroup per tile of the
// grid.  Without a previous length every tile gets a workgroup (up to
// LBM_TILE_GRID_MAX).
#ifndef LBM_TILE_GRID_MAX
#define LBM_TILE_GRID_MAX 32768
#endif
constexpr uint32_t META_EVERY = 8;
#ifndef SWEEP_PREF_TILES
#define SWEEP_PREF_TILES 1024
#endif

int64_t tile_grid(const lbm_ctx* c, int list) {
  const int64_t full = std::min<int64_t>((c->ntiles + 7) / 8 * 8, LBM_TILE_GRID_MAX);
  if (!c->prev_len_valid) return full;
  const int64_t want = (int64_t)c->prev_len[list] + c->prev_len[list] / 4 + 64;
  return std::min<int64_t>(full, (want + 7) / 8 * 8);
}

int64_t forcing_list_grid(const lbm_ctx* c) { return c->own_grid; }

// The U pre-pass of the strategy the surface was set with.
template <int S>
hipError_t launch_u_prepass(lbm_ctx* c, const typename Store<S>::T* lat, const PointGeom& pg,
                            unsigned tg) {
  hipStream_t st = c->stream;
  if (c->flags & IBM_U_BOX) {
    const int64_t sub = c->ubox_sub;
    const int64_t nblk = (int64_t)c->nbodies * sub * sub * sub;
    if (nblk > 0)
      k_moments_box<S><<<(unsigned)nblk, TILE3, 0, st>>>(lat, c->geom, pg, c->motion, c->ubox,
                                                         (int)sub, c->U);
  } else if (c->flags & IBM_U_KERNEL) {
    const int64_t nblk = (c->npts + WG / 64 - 1) / (WG / 64);
    if (nblk > 0)
      k_moments_points<S><<<(unsigned)nblk, WG, 0, st>>>(lat, c->geom, pg, c->sp_base, c->npts,
                                                         c->U);
  } else {
    k_moments_blocks<S><<<tg, TILE3, 0, st>>>(lat, c->geom, pg, c->touch_tiles, c->meta,
                                              c->bflag, c->own_slot,
                                              (const unsigned char*)c->boxbuf, c->U);
  }
  return hipGetLastError();
}

// Positions of the tile scan: the tile grid padded to whole 4 x 4 x 4 blocks.
int64_t scan_positions(const lbm_ctx* c) {
  int64_t n = 1;
  for (int a = 0; a < 3; ++a) n *= (c->tiles[a] + SB - 1) / SB * SB;
  return n;
}

// The forcing of one time step: motion, binning, U near the surface,
// n_iter sweeps of interpolation + correction with n_iter - 1 intermediate
// spreads into U and the final spread of du into G.
hipError_t launch_forcing(lbm_ctx* c) {
  const PointGeom pg = point_geom(c);
  const int64_t n = c->npts;
  const unsigned nb = (unsigned)((n + LBM_BLOCK - 1) / LBM_BLOCK);
  if (c->meta_pending && hipEventQuery(c->meta_event) == hipSuccess) {
    c->prev_len[0] = c->meta_host[0];
    c->prev_len[1] = c->meta_host[1];
    c->prev_len_valid = true;
    c->meta_pending = false;
  }
  const unsigned lg = (unsigned)tile_grid(c, 0);
  const unsigned tg = (unsigned)tile_grid(c, 1);
  c->own_grid = lg;
  const int64_t rs = c->part_row;  // row stride of pt_partials
  hipStream_t st = c->stream;

  k_point_count<<<nb, LBM_BLOCK, 0, st>>>(c->rest, c->body_of, c->bodies, c->nbodies, c->step,
                                          c->motion, n, pg, c->key, c->rank, c->cnt_own,
                                          c->cnt_touch);
  LAUNCH_CHECK();
  {
    const int64_t nch = (scan_positions(c) + SCAN_CHUNK - 1) / SCAN_CHUNK;
    // a pending host copy of the lengths is not overwritten before it is
    // read; the copy is refreshed every META_EVERY forcings (the event that
    // marks its arrival costs a few microseconds of queue time, and the
    // lengths only size the grids, with a margin)
    const bool refresh = !c->meta_pending && (!c->prev_len_valid || c->meta_age >= META_EVERY);
    uint32_t* mh = refresh ? c->meta_host_dev : nullptr;
    c->meta_age = refresh ? 0u : c->meta_age + 1u;
    k_scan_totals<<<(unsigned)nch, SCAN_WG, 0, st>>>(pg, c->cnt_own, c->cnt_touch, c->chunk_tot);
    LAUNCH_CHECK();
    const bool few = nch <= SCAN_FEW_CHUNKS;
    if (!few) {
      k_scan_chunks<<<1, SCAN2_WG, 0, st>>>(c->chunk_tot, nch, c->meta, mh);
      LAUNCH_CHECK();
    }
    auto kw = few ? k_scan_write<true> : k_scan_write<false>;
    kw<<<(unsigned)nch, SCAN_WG, 0, st>>>(pg, c->cnt_own, c->cnt_touch, c->chunk_tot, nch,
                                          c->start_own, c->end_own, c->own_slot, c->own_tiles,
                                          c->touch_tiles, (uint32_t*)c->bflag, c->nbflag_words,
                                          c->meta, few ? mh : nullptr);
    LAUNCH_CHECK();
    if (mh && hipEventRecord(c->meta_event, st) == hipSuccess) c->meta_pending = true;
  }
  // the scatter's temporaries: base in sp_tmp, fraction in sp_g, u_b in sp_du
  // (both written by sweep 0 before they are read)
  k_point_scatter<<<nb, LBM_BLOCK, 0, st>>>(c->rest, c->body_of, c->motion, n, pg, c->key, c->rank,
                                            c->start_own, c->sp_tmp, c->sp_g, c->sp_du, c->bflag,
                                            c->pt_partials, c->pt_partials + rs);
  LAUNCH_CHECK();
  k_tile_order<<<lg, CELL_WG, 0, st>>>(c->own_tiles, c->meta, c->start_own, c->end_own, c->sp_tmp,
                                       c->sp_g,
                                       c->sp_du, c->rank, c->sp_base, c->sp_frac, c->sp_ub,
                                       (unsigned char*)c->boxbuf);
  LAUNCH_CHECK();
  {
    hipError_t e = hipSuccess;
    switch (c->p.storage) {
      case LBM_STORE_F16:
        e = launch_u_prepass<LBM_STORE_F16>(c, (const _Float16*)c->lat[c->cur], pg, tg);
        break;
      case LBM_STORE_BF16:
        e = launch_u_prepass<LBM_STORE_BF16>(c, (const uint16_t*)c->lat[c->cur], pg, tg);
        break;
      default:
        e = launch_u_prepass<LBM_STORE_F32>(c, (const float*)c->lat[c->cur], pg, tg);
    }
    if (e != hipSuccess) return e;
  }
  const int uw = (c->flags & IBM_INNER_UNWEIGHTED) ? SW_UNWEIGHTED : 0;
  const bool feats = (c->flags & (IBM_WARM_START | IBM_KEEP_FEATURES)) != 0;
  if (feats && !c->nbr_valid) {
    hipError_t e = launch_neighbours(c);
    if (e != hipSuccess) return e;
    c->nbr_valid = true;
  }
  // few owner tiles (a recent forcing's count): the latency form of the sweep
  const bool pref = c->prev_len_valid && c->prev_len[0] <= SWEEP_PREF_TILES;
  auto sweep = [&](int it, int mode, const uint32_t* gate, float4* g_orig) {
    auto kern = pref ? k_sweep_tiles<true> : k_sweep_tiles<false>;
    kern<<<lg, WG, 0, st>>>(c->own_tiles, c->meta, c->start_own, c->end_own, c->sp_base,
                            c->sp_frac, c->sp_ub, c->sp_g, c->sp_du, c->U,
                            (unsigned char*)c->boxbuf, pg, mode | uw,
                            c->pt_partials + (2 + it) * rs, gate, g_orig, c->du_prev, c->status);
    return hipGetLastError();
  };
  auto merge = [&](bool final_, const uint32_t* gate) {
    k_merge_tiles<<<tg, MERGE_WG, 0, st>>>(c->touch_tiles, c->meta, c->own_slot,
                                        (const unsigned char*)c->boxbuf, c->bflag, c->G, c->U, pg,
                                        final_ ? 2 : 0, gate);
    return hipGetLastError();
  };
#define TRY(x)                               \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return e_;         \
  } while (0)
  const int N = c->n_iter;
  if (!(c->flags & (IBM_STOP_RESIDUAL | IBM_WARM_START | IBM_WARM_PREV))) {
    // fixed number of sweeps; the last one spreads du into G
    for (int it = 0; it < N; ++it) {
      const bool last = it == N - 1;
      // g is kept for the export (last sweep) and the warm-start features (sweep 0)
      const int mode = SW_INTERP | (it == 0 ? SW_FIRST : 0) | (last ? SW_SPREAD_DU : SW_SPREAD_G) |
                       ((last || (it == 0 && feats)) ? SW_STORE_G : 0);
      TRY(sweep(it, mode, nullptr, it == 0 && feats ? c->g0_orig : nullptr));
      if (it == 0 && feats) TRY(launch_features_warm(c));
      TRY(merge(last, nullptr));
    }
    return hipSuccess;
  }
  // Residual-stopped and/or warm-started: every launch after sweep 0 is
  // gated by the device flag ctl[0], so the sequence runs without host round
  // trips; the final spread of du into G always runs.
  const bool warm = (c->flags & IBM_WARM_START) != 0;
  const bool save_prev = (c->flags & IBM_WARM_PREV) != 0;
  const bool from_prev = save_prev && c->du_prev_valid;
  const int use_thr = (c->flags & IBM_STOP_RESIDUAL) ? 1 : 0;
  const int64_t na = (n + LBM_BLOCK - 1) / LBM_BLOCK;
  const double eps2 = (double)c->eps * (double)c->eps;
  for (int it = 0; it < N; ++it) {
    const bool last = it == N - 1;
    const uint32_t* gate = it == 0 ? nullptr : c->ctl;
    // sweep 0 under a warm start only interpolates: the predicted (or the
    // previous forcing's) du is spread in place of s g0
    const bool spread = !last && !((warm || from_prev) && it == 0);
    // any sweep may be the last one: g is always kept
    const int mode =
        SW_INTERP | SW_STORE_G | (it == 0 ? SW_FIRST : 0) | (spread ? SW_SPREAD_G : 0);
    TRY(sweep(it, mode, gate, it == 0 && feats ? c->g0_orig : nullptr));
    k_resid_check<<<1, RESID_WG, 0, st>>>(c->pt_partials + (2 + it) * rs, lg,
                                           c->pt_partials + rs, na, eps2, c->resid_thr, it,
                                           last ? 1 : 0, use_thr, c->ctl);
    TRY(hipGetLastError());
    if (it == 0 && feats) {
      // features stored for logging, else computed inside the warm-start
      // kernel (BF16 or FP32 operands on the matrix cores)
      const bool fp32 = (c->flags & IBM_MLP_FP32) != 0;
      const bool keep = (c->flags & IBM_KEEP_FEATURES) != 0;
      if (keep) TRY(launch_features_warm(c));
      if (warm) TRY(fp32 ? launch_warm_mfma32(c, keep) : launch_warm_mfma(c, keep));
    }
    if (it == 0 && warm && !last) {
      TRY(sweep(0, SW_SPREAD_DU, c->ctl, nullptr));
      TRY(merge(false, c->ctl));
    } else if (it == 0 && from_prev && !last) {
      TRY(sweep(0, SW_SPREAD_DU | SW_LOAD_PREV, c->ctl, nullptr));
      TRY(merge(false, c->ctl));
    } else if (spread) {
      TRY(merge(false, c->ctl));
    }
  }
  TRY(sweep(0, SW_SPREAD_DU | (save_prev ? SW_SAVE_DU : 0), nullptr, nullptr));
  TRY(merge(true, nullptr));
#undef TRY
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
