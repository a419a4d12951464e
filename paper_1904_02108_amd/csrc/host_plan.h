// Host-side planning of the C ABI, in plain C++ (no HIP), so that it also
// builds for the CPU under sanitizers: parameter checks, the carving of the
// five caller buffers into arrays (byte offsets), and the validation and
// host layout of a Lagrangian surface given to ibm_set_points.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.h"
#include "lbmibm.h"

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of every array inside the caller buffers.
struct Plan {
  size_t size[LBM_NBUF];
  // lattice
  size_t elem, lat_bytes;
  int64_t spop, srow, splane, lat_elems;  // population layout (LatticeGeom)
  // points
  size_t o_rest, o_body_of, o_key, o_rank, o_base, o_frac, o_ub, o_g, o_du, o_tmp, o_bodies,
      o_motion;
  size_t o_nbr, o_g0, o_duprev, o_feat, o_vref, o_theta, o_packed, o_ubox;
  size_t o_box, o_G;
  int64_t max_boxes;
  // tiles
  size_t o_cnt_own, o_cnt_touch, o_start_own, o_end_own, o_own_slot, o_own_tiles, o_touch_tiles, o_meta,
      o_bflag, o_chunk;
  int64_t nblocks4, nbflag_words;
  int fblk[3];
  // scratch
  size_t o_sum_part, o_pt_part, o_small, o_ctl, o_thr, o_status;
  int64_t part_row;
  int64_t n_cell_blocks, n_pt_blocks;
  int64_t ncell, ntiles;
  int tiles[3];
};

// Checks lbm_params; on error returns the status and sets msg.
lbm_status check_params(const lbm_params* p, std::string& msg);

// Sizes and carves the caller buffers for valid parameters p.
void make_plan(const lbm_params* p, Plan& pl);

// A surface (ibm_set_points) validated and laid out as the device arrays
// hold it: per point (x, y, z, s) and its body; per body (centre, axis,
// theta0, omega), the reference speed of the learned features and the
// rest-position bounding box of the box U pre-pass (lo, hi); and the number
// of 8^3 sub-blocks per axis that bounds every rotation of the largest box.
struct SurfaceHost {
  std::vector<float> rest4;
  std::vector<int32_t> body_of;
  std::vector<double> btab;
  std::vector<float> vref;
  std::vector<float> ubox;
  int ubox_sub = 0;
};

// Validates a surface of n >= 1 points against the lattice parameters p and
// fills out; on error returns the status (LBM_ERR_ARG, or LBM_ERR_DOMAIN if
// a support could cross a wall) and sets msg.
lbm_status prepare_surface(const lbm_params& p, int64_t n, const float* rest_xyz,
                           const float* area, const int64_t* body_off, int32_t nbodies,
                           const ibm_body* bodies, int32_t n_iter, uint32_t flags, float eps,
                           SurfaceHost& out, std::string& msg);
