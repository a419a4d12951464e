// Host-side internals: the context and the kernel launchers that the C ABI
// in lbmibm.cpp drives.  Launchers enqueue on ctx->stream and return
// hipError_t from the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "device_common.h"
#include "lbmibm.h"


// Per-body motion coefficients computed on the device each step:
// normalised axis, centre, cos/sin of theta_n, and the differences of cos and
// sin between steps n and n-1.
struct BodyMotion {
  double center[3];
  double axis[3];
  double c, s, dc, ds;
};
static_assert(sizeof(BodyMotion) == BODY_MOTION_BYTES, "BodyMotion size");
static_assert(sizeof(float4) == VEC4_BYTES && sizeof(int4) == VEC4_BYTES, "vector sizes");

struct lbm_ctx {
  lbm_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  lbmd::LatticeGeom geom{};
  int64_t ncell = 0;
  int tiles[3] = {0, 0, 0};
  int64_t ntiles = 0;
  size_t elem = 4;  // bytes per stored population

  // caller buffers, carved
  void* lat[2] = {nullptr, nullptr};
  int cur = 0;  // lattice holding the post-collision state of the previous step
  float4* U = nullptr;  // [ntiles][512] velocity scratch of the forcing (tile-major, x y z 0)
  float* G = nullptr;  // [3][ncell] force
  // points (capacity max_points)
  float4* rest = nullptr;     // (x, y, z, s) relative to the body centre
  int32_t* body_of = nullptr;
  uint32_t* key = nullptr;
  uint32_t* rank = nullptr;
  int4* sp_base = nullptr;    // sorted: base cell (x, y, z), original index
  float4* sp_frac = nullptr;  // sorted: fractional position (x, y, z), s
  float4* sp_ub = nullptr;    // sorted: point velocity u_b
  float4* sp_g = nullptr;     // sorted: deficit g
  float4* sp_du = nullptr;    // sorted: accumulated correction du
  int4* sp_tmp = nullptr;     // binning temporary: base cells in tile order
  double* bodies = nullptr;   // [LBM_MAX_BODIES][8] as given
  BodyMotion* motion = nullptr;
  // tiles (8^3) and force blocks (4^3)
  int fblk[3] = {0, 0, 0};
  int64_t nblocks4 = 0;        // number of 4^3 force blocks
  int64_t nbflag_words = 0;    // bflag size in 32-bit words
  uint32_t* cnt_own = nullptr;     // [ntiles] points owned per tile (pass 1)
  uint32_t* cnt_touch = nullptr;   // [ntiles] 1 where a support reaches the tile (pass 1)
  uint32_t* start_own = nullptr;   // [ntiles] first slot of each tile's points
  uint32_t* end_own = nullptr;     // [ntiles] one past its last slot
  int32_t* own_slot = nullptr;     // [ntiles] index in own_tiles, or -1
  uint32_t* own_tiles = nullptr;   // compact list of tiles owning points
  uint32_t* touch_tiles = nullptr; // compact list of touched tiles
  uint32_t* meta = nullptr;        // [4]: list lengths
  uint32_t* chunk_tot = nullptr;   // [scan chunks][3] totals, then offsets
  uint8_t* bflag = nullptr;        // [nbflag_words * 4] force-block flags
  // learned warm start
  int32_t* nbr = nullptr;       // [max_points][16] neighbour lists (caller order)
  float4* g0_orig = nullptr;    // [max_points] first deficit (caller order)
  float4* du_prev = nullptr;    // [max_points] last forcing's du (caller order)
  float* ubox = nullptr;        // [LBM_MAX_BODIES][6] rest-position box (lo, hi) per body
  int ubox_sub = 0;             // 8^3 sub-blocks per axis bounding any moved box
  float* feat = nullptr;        // [max_points][12] features of the last forcing (sorted)
  float* vref = nullptr;        // [LBM_MAX_BODIES] reference speed per body
  float* theta = nullptr;       // [IBM_MLP_NPARAM] network parameters
  void* theta_packed = nullptr; // BF16 matrix-core operands of the network
  uint32_t* ctl = nullptr;      // [4] residual stop: converged flag, sweeps run
  double* resid_thr = nullptr;  // [1] eps^2 sum s |u_b|^2
  void* boxbuf = nullptr;           // [max_boxes] slots of BOX_SLOT_BYTES: spread boxes of owner tiles
  int64_t max_boxes = 0;
  // scratch
  double* sum_partials = nullptr;   // [n_cell_blocks][4]
  int64_t n_cell_blocks = 0;
  double* pt_partials = nullptr;    // [max_iter + 2][part_row]
  int64_t part_row = 0;
  double* small = nullptr;          // [256] reduced results
  uint32_t* status = nullptr;       // [4] sticky: [0] sums not finite, [1] spread out of range
  // device staging of host sources and destinations in lbm_read_fields /
  // lbm_write_fields: grown to the largest request, freed by lbm_destroy
  void* stage = nullptr;
  size_t stage_bytes = 0;

  // state
  int64_t npts = 0;
  int32_t nbodies = 0;
  int32_t n_iter = 5;
  uint32_t flags = 0;
  float eps = 0.0f;
  bool nbr_valid = false;   // neighbour lists match the current surface
  bool du_prev_valid = false;  // du_prev holds a forcing of the current surface
  bool theta_set = false;   // ibm_set_mlp has been called
  int64_t step = 0;
  int64_t g_valid_step = -1;
  bool g_prescribed = false;
  bool have_sums = false;  // a stream-collide has written the sum partials
  int32_t check_every = 0;  // lbm_set_check interval (0 = off)
  int64_t check_since = 0;  // steps since the last check

  // lengths of the owner / touched tile lists of a previous forcing, copied
  // asynchronously to pinned host memory, to size the tile grids
  uint32_t* meta_host = nullptr;      // pinned, mapped host memory
  uint32_t* meta_host_dev = nullptr;  // its device address
  hipEvent_t meta_event = nullptr;
  bool meta_pending = false;
  bool prev_len_valid = false;
  uint32_t prev_len[2] = {0, 0};
  uint32_t meta_age = 0;  // forcings since the lengths were last copied to the host
  int64_t own_grid = 8;  // workgroups of the last forcing's sweep launches

  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;  // per recorded event, the phase it opens: 0 forcing, 1 stream-collide, -1 none
  size_t ev_used = 0;
  double t_acc[4] = {0, 0, 0, 0};

  std::string err;
};

// message returned by lbm_last_error(NULL) on this thread (calls without a
// context: lbm_create, mlp_loss_grad_noalloc)
void set_noalloc_error(const std::string& msg);

// lattice kernels (lbm_kernels.hip)
hipError_t launch_init_equilibrium(lbm_ctx* c);
hipError_t launch_unstream_from(lbm_ctx* c, const void* pops, int f64);
hipError_t launch_stream_collide(lbm_ctx* c);
void stream_collide_shape(const lbm_ctx* c, dim3& grid, dim3& block);
hipError_t launch_readout(lbm_ctx* c, float* rho, float* vel, void* pops, int pops_f64);
hipError_t launch_reduce_sums(lbm_ctx* c, double* out4);
hipError_t launch_fill_u8(lbm_ctx* c, uint8_t* p, uint8_t v, int64_t n);
hipError_t launch_fill_u32(lbm_ctx* c, uint32_t* p, uint32_t v, int64_t n);
hipError_t launch_copy_f32(lbm_ctx* c, float* dst, const float* src, int64_t n);
hipError_t launch_export_force(lbm_ctx* c, float* out);

// forcing kernels (ibm_kernels.hip)
hipError_t launch_forcing(lbm_ctx* c);
int64_t forcing_list_grid(const lbm_ctx* c);
hipError_t launch_reduce_point_stats(lbm_ctx* c, double* out /* [n_iter + 2] */);
hipError_t launch_export_points(lbm_ctx* c, double* x, float* ub, float* g, float* du);

// learned warm start (mlp_kernels.hip)
hipError_t launch_neighbours(lbm_ctx* c);
hipError_t launch_features_warm(lbm_ctx* c);
hipError_t launch_export_pairs(lbm_ctx* c, float* feat, float* targets);
hipError_t launch_mlp_pack(lbm_ctx* c);
hipError_t launch_warm_mfma(lbm_ctx* c, bool from_stored_features);
hipError_t launch_warm_mfma32(lbm_ctx* c, bool from_stored_features);
