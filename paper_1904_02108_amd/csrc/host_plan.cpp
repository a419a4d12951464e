// Host-side planning of the C ABI (see host_plan.h): plain C++, no HIP.
#include "host_plan.h"

#include <algorithm>
#include <cmath>

namespace {

// Consecutive 256-byte aligned regions of one buffer.
struct Cursor {
  size_t at = 0;
  size_t take(size_t bytes) {
    size_t o = at;
    at = align_up(at + bytes);
    return o;
  }
};

}  // namespace

lbm_status check_params(const lbm_params* p, std::string& msg) {
  if (!p) {
    msg = "params is NULL";
    return LBM_ERR_ARG;
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
    msg = "lattice sizes must be >= 1";
    return LBM_ERR_ARG;
  }
  const int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
  if (ncell > ((int64_t)1 << 31) - 1) {
    msg = "lattice larger than 2^31 - 1 cells";
    return LBM_ERR_ARG;
  }
  // the forcing indexes cells of whole 8^3 tiles with 32-bit unsigned offsets
  const int64_t T = lbmd::TILE;
  const int64_t tile_cells =
      ((p->nx + T - 1) / T) * ((p->ny + T - 1) / T) * ((p->nz + T - 1) / T) * T * T * T;
  if (tile_cells > ((int64_t)1 << 32) - 1) {
    msg = "lattice padded to whole 8^3 tiles larger than 2^32 - 1 cells";
    return LBM_ERR_ARG;
  }
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != LBM_BC_PERIODIC && p->bc[a] != LBM_BC_BOUNCEBACK) {
      msg = "bc must be LBM_BC_PERIODIC or LBM_BC_BOUNCEBACK";
      return LBM_ERR_ARG;
    }
  if (p->storage < LBM_STORE_F32 || p->storage > LBM_STORE_BF16) {
    msg = "unknown storage";
    return LBM_ERR_ARG;
  }
  if (p->forcing != LBM_FORCE_GUO && p->forcing != LBM_FORCE_SHIFT) {
    msg = "unknown forcing";
    return LBM_ERR_ARG;
  }
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) {
    msg = "tau must be finite and > 0.5";
    return LBM_ERR_ARG;
  }
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0) || !std::isfinite(p->rho_wall)) {
    msg = "rho0 must be > 0 and rho_wall finite";
    return LBM_ERR_ARG;
  }
  const double* d = &p->wall_u[0][0][0];
  for (int k = 0; k < 18; ++k)
    if (!std::isfinite(d[k])) {
      msg = "wall_u must be finite";
      return LBM_ERR_ARG;
    }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->g_ext[a]) || !std::isfinite(p->u0[a])) {
      msg = "g_ext and u0 must be finite";
      return LBM_ERR_ARG;
    }
  if (p->max_points < 0 || p->max_points > ((int64_t)1 << 31) - 1) {
    msg = "max_points must be in [0, 2^31 - 1]";
    return LBM_ERR_ARG;
  }
  if (p->max_iter < 1 || p->max_iter > LBM_MAX_ITER) {
    msg = "max_iter must be in [1, 64]";
    return LBM_ERR_ARG;
  }
  if (p->reserved_ != 0) {
    msg = "reserved_ must be 0";
    return LBM_ERR_ARG;
  }
  return LBM_OK;
}

// lattices of fewer bytes than this get interleaved populations (at most
// 4 GB: the stream-collide's buffer descriptors take 32-bit offsets)
#ifndef LBM_INTERLEAVE_MAX_BYTES
#define LBM_INTERLEAVE_MAX_BYTES 4294967296ll
#endif
static_assert(LBM_INTERLEAVE_MAX_BYTES <= 4294967296ll, "32-bit lattice offsets");

void make_plan(const lbm_params* p, Plan& pl) {
  pl.ncell = (int64_t)p->nx * p->ny * p->nz;
  pl.elem = p->storage == LBM_STORE_F32 ? 4 : 2;
  // populations of each x row interleaved, rows padded to 128 bytes, when a
  // lattice stays below 4 GB (32-bit buffer offsets); else one array per
  // population
  const int64_t row_align = 128 / (int64_t)pl.elem;
  const int64_t nxp = ((int64_t)p->nx + row_align - 1) / row_align * row_align;
  const int64_t inter = (int64_t)lbmd::Q * nxp * p->ny * p->nz;
  if (inter * (int64_t)pl.elem < (int64_t)LBM_INTERLEAVE_MAX_BYTES) {
    pl.spop = nxp;
    pl.srow = (int64_t)lbmd::Q * nxp;
    pl.splane = pl.srow * p->ny;
    pl.lat_elems = inter;
  } else {
    pl.spop = (int64_t)(align_up((size_t)pl.ncell * pl.elem) / pl.elem);
    pl.srow = p->nx;
    pl.splane = (int64_t)p->nx * p->ny;
    pl.lat_elems = (int64_t)lbmd::Q * pl.spop;
  }
  pl.lat_bytes = align_up((size_t)pl.lat_elems * pl.elem);
  pl.size[LBM_BUF_LATTICE] = 2 * pl.lat_bytes;
  const size_t M = (size_t)std::max<int64_t>(p->max_points, 1);
  const int dims[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    pl.tiles[a] = (dims[a] + lbmd::TILE - 1) / lbmd::TILE;
    pl.fblk[a] = (dims[a] + lbmd::FBLK - 1) / lbmd::FBLK;
  }
  pl.ntiles = (int64_t)pl.tiles[0] * pl.tiles[1] * pl.tiles[2];
  // U (tile-major, whole tiles, one float4 per cell), G (lattice layout),
  // and the spread boxes of the tiles that own points (at most one per tile
  // and one per point)
  pl.o_G = align_up((size_t)pl.ntiles * lbmd::TILE * lbmd::TILE * lbmd::TILE * VEC4_BYTES);
  pl.size[LBM_BUF_FIELDS] = pl.o_G + align_up(3 * (size_t)pl.ncell * sizeof(float));
  pl.max_boxes = std::max<int64_t>(1, std::min<int64_t>(pl.ntiles, p->max_points));
  pl.o_box = pl.size[LBM_BUF_FIELDS];
  pl.size[LBM_BUF_FIELDS] += align_up((size_t)pl.max_boxes * BOX_SLOT_BYTES);
  pl.nblocks4 = (int64_t)pl.fblk[0] * pl.fblk[1] * pl.fblk[2];
  pl.nbflag_words = (pl.nblocks4 + 3) / 4;

  Cursor pc;
  pl.o_rest = pc.take(M * VEC4_BYTES);
  pl.o_body_of = pc.take(M * sizeof(int32_t));
  pl.o_key = pc.take(M * sizeof(uint32_t));
  pl.o_rank = pc.take(M * sizeof(uint32_t));
  pl.o_base = pc.take(M * VEC4_BYTES);
  pl.o_frac = pc.take(M * VEC4_BYTES);
  pl.o_ub = pc.take(M * VEC4_BYTES);
  pl.o_g = pc.take(M * VEC4_BYTES);
  pl.o_du = pc.take(M * VEC4_BYTES);
  pl.o_tmp = pc.take(M * VEC4_BYTES);
  pl.o_bodies = pc.take((size_t)LBM_MAX_BODIES * 8 * sizeof(double));
  pl.o_motion = pc.take((size_t)LBM_MAX_BODIES * BODY_MOTION_BYTES);
  pl.o_nbr = pc.take(M * IBM_MLP_NNBR * sizeof(int32_t));
  pl.o_g0 = pc.take(M * VEC4_BYTES);
  pl.o_duprev = pc.take(M * VEC4_BYTES);
  pl.o_feat = pc.take(M * IBM_MLP_NFEAT * sizeof(float));
  pl.o_vref = pc.take((size_t)LBM_MAX_BODIES * sizeof(float));
  pl.o_ubox = pc.take((size_t)LBM_MAX_BODIES * 6 * sizeof(float));
  pl.o_theta = pc.take((size_t)IBM_MLP_NPARAM * sizeof(float));
  pl.o_packed = pc.take(MLP_PACKED_BYTES);
  pl.size[LBM_BUF_POINTS] = pc.at;

  const size_t NT = (size_t)pl.ntiles;
  Cursor tc;
  // positions of the tile scan: the tile grid padded to whole 4^3 blocks of
  // tiles, in whole chunks of 2048
  size_t NP = 1;
  for (int a = 0; a < 3; ++a) NP *= (size_t)(pl.tiles[a] + 3) / 4 * 4;
  const size_t NPpad = (NP + 2047) / 2048 * 2048;
  pl.o_cnt_own = tc.take(NT * 4);
  pl.o_cnt_touch = tc.take(NT * 4);
  pl.o_start_own = tc.take(NT * 4);
  pl.o_end_own = tc.take(NT * 4);
  pl.o_own_slot = tc.take(NT * 4);
  pl.o_own_tiles = tc.take(NT * 4);
  pl.o_touch_tiles = tc.take(NT * 4);
  pl.o_meta = tc.take(4 * 4);
  pl.o_bflag = tc.take((size_t)pl.nbflag_words * 4);
  pl.o_chunk = tc.take((NPpad / 2048) * 4 * 4);  // totals of the scan chunks

  pl.size[LBM_BUF_TILES] = tc.at;

  {  // blocks of the stream-collide launch (see stream_collide_shape)
    int bx = ((p->nx + 63) / 64) * 64;
    if (bx > LBM_BLOCK) bx = LBM_BLOCK;
    const int by = LBM_BLOCK / bx;
    pl.n_cell_blocks = (int64_t)((p->nx + bx - 1) / bx) * ((p->ny + by - 1) / by) * p->nz;
    pl.n_cell_blocks = std::max<int64_t>(pl.n_cell_blocks, (pl.ncell + LBM_BLOCK - 1) / LBM_BLOCK);
  }
  pl.n_pt_blocks = ((int64_t)M + LBM_BLOCK - 1) / LBM_BLOCK;
  pl.part_row = std::max<int64_t>(pl.n_pt_blocks, (pl.ntiles + 7) / 8 * 8);
  Cursor sc;
  pl.o_sum_part = sc.take((size_t)pl.n_cell_blocks * 4 * sizeof(double));
  pl.o_pt_part = sc.take((size_t)(p->max_iter + 2) * pl.part_row * sizeof(double));
  pl.o_small = sc.take(256 * sizeof(double));
  pl.o_ctl = sc.take(4 * sizeof(uint32_t));
  pl.o_thr = sc.take(sizeof(double));
  pl.o_status = sc.take(4 * sizeof(uint32_t));
  pl.size[LBM_BUF_SCRATCH] = sc.at;
}


lbm_status prepare_surface(const lbm_params& p, int64_t n, const float* rest_xyz,
                           const float* area, const int64_t* body_off, int32_t nbodies,
                           const ibm_body* bodies, int32_t n_iter, uint32_t flags, float eps,
                           SurfaceHost& out, std::string& msg) {
  auto bad = [&](lbm_status st, const char* m) {
    msg = m;
    return st;
  };
  if (n < 1 || n > p.max_points) return bad(LBM_ERR_ARG, "n must be in [0, max_points]");
  if (!rest_xyz || !area || !body_off || !bodies) return bad(LBM_ERR_ARG, "NULL point array");
  if (nbodies < 1 || nbodies > LBM_MAX_BODIES)
    return bad(LBM_ERR_ARG, "nbodies must be in [1, 65536]");
  if (n_iter < 1 || n_iter > p.max_iter)
    return bad(LBM_ERR_ARG, "n_iter must be in [1, max_iter]");
  const uint32_t known = IBM_INNER_UNWEIGHTED | IBM_STOP_RESIDUAL | IBM_WARM_START |
                         IBM_KEEP_FEATURES | IBM_MLP_FP32 | IBM_WARM_PREV | IBM_U_BOX |
                         IBM_U_KERNEL;
  if (flags & ~known) return bad(LBM_ERR_ARG, "unknown flags");
  if ((flags & IBM_WARM_START) && (flags & IBM_WARM_PREV))
    return bad(LBM_ERR_ARG, "IBM_WARM_START and IBM_WARM_PREV exclude each other");
  if ((flags & IBM_U_BOX) && (flags & IBM_U_KERNEL))
    return bad(LBM_ERR_ARG, "IBM_U_BOX and IBM_U_KERNEL exclude each other");
  if ((flags & IBM_WARM_START) && (flags & IBM_INNER_UNWEIGHTED))
    return bad(LBM_ERR_ARG, "IBM_WARM_START needs the weighted inner sweep");
  if (flags & IBM_STOP_RESIDUAL) {
    if (!(eps >= 0.0f) || !std::isfinite(eps))
      return bad(LBM_ERR_ARG, "eps must be finite and >= 0");
  } else if (eps != 0.0f) {
    return bad(LBM_ERR_ARG, "eps must be 0 without IBM_STOP_RESIDUAL");
  }
  if (body_off[0] != 0 || body_off[nbodies] != n)
    return bad(LBM_ERR_ARG, "body_off must start at 0 and end at n");
  for (int b = 0; b < nbodies; ++b)
    if (body_off[b + 1] < body_off[b]) return bad(LBM_ERR_ARG, "body_off must not decrease");
  out.rest4.assign((size_t)n * 4, 0.0f);
  out.body_of.assign((size_t)n, 0);
  out.btab.assign((size_t)nbodies * 8, 0.0);
  out.vref.assign((size_t)nbodies, 1.0f);
  out.ubox.assign((size_t)nbodies * 6, 0.0f);
  double ubox_reach = 0.0;  // largest distance of a rest-box corner from its centre
  const int dims[3] = {p.nx, p.ny, p.nz};
  for (int b = 0; b < nbodies; ++b) {
    const ibm_body& B = bodies[b];
    const double al =
        std::sqrt(B.axis[0] * B.axis[0] + B.axis[1] * B.axis[1] + B.axis[2] * B.axis[2]);
    if (!(al > 0.0) || !std::isfinite(al) || !std::isfinite(B.theta0) || !std::isfinite(B.omega))
      return bad(LBM_ERR_ARG, "body axis must be nonzero and finite; theta0, omega finite");
    double rmax = 0.0;
    for (int64_t k = body_off[b]; k < body_off[b + 1]; ++k) {
      const float* r = rest_xyz + 3 * k;
      if (!std::isfinite(r[0]) || !std::isfinite(r[1]) || !std::isfinite(r[2]) ||
          !std::isfinite(area[k]) || area[k] < 0.0f)
        return bad(LBM_ERR_ARG, "rest positions must be finite and areas finite, >= 0");
      float* q = &out.rest4[4 * (size_t)k];
      q[0] = r[0];
      q[1] = r[1];
      q[2] = r[2];
      q[3] = area[k];
      out.body_of[(size_t)k] = b;
      rmax = std::max(rmax, std::sqrt((double)r[0] * r[0] + (double)r[1] * r[1] +
                                      (double)r[2] * r[2]));
    }
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(B.center[a])) return bad(LBM_ERR_ARG, "body centre must be finite");
      if (p.bc[a] == LBM_BC_BOUNCEBACK && body_off[b + 1] > body_off[b]) {
        // every support must stay inside: 1 <= x < n - 2 for all angles
        const double margin = 1e-6 * (1.0 + rmax + std::fabs(B.center[a]));
        if (B.center[a] - rmax < 1.0 + margin || B.center[a] + rmax >= dims[a] - 2.0 - margin)
          return bad(LBM_ERR_DOMAIN, "a body's kernel support can cross a wall");
      }
    }
    for (int a = 0; a < 3; ++a) {
      out.btab[8 * (size_t)b + a] = B.center[a];
      out.btab[8 * (size_t)b + 3 + a] = B.axis[a];
    }
    out.btab[8 * (size_t)b + 6] = B.theta0;
    out.btab[8 * (size_t)b + 7] = B.omega;
    // reference speed of the learned features: the fastest rest point's
    // speed bound |omega| max |r|, or 1 for a body at rest
    const double vr = std::fabs(B.omega) * rmax;
    out.vref[(size_t)b] = vr > 0.0 ? (float)vr : 1.0f;
    // rest-position bounding box of the body's points (box U pre-pass)
    if (body_off[b + 1] > body_off[b]) {
      const float* r0 = rest_xyz + 3 * body_off[b];
      float lo[3] = {r0[0], r0[1], r0[2]};
      float hi[3] = {lo[0], lo[1], lo[2]};
      for (int64_t k = body_off[b]; k < body_off[b + 1]; ++k)
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], rest_xyz[3 * k + a]);
          hi[a] = std::max(hi[a], rest_xyz[3 * k + a]);
        }
      double reach2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        out.ubox[6 * (size_t)b + a] = lo[a];
        out.ubox[6 * (size_t)b + 3 + a] = hi[a];
        const double m = std::max(std::fabs((double)lo[a]), std::fabs((double)hi[a]));
        reach2 += m * m;
      }
      ubox_reach = std::max(ubox_reach, std::sqrt(reach2));
    }
  }
  // a moved box lies in the cube of half-edge reach around the centre; the
  // pre-pass widens it to floor(lo) - 2 .. floor(hi) + 3, at most 2 reach + 7
  // cells per axis (one more for rounding)
  out.ubox_sub = (int)std::ceil((2.0 * ubox_reach + 8.0) / lbmd::TILE);
  return LBM_OK;
}
