// C ABI of the LBM-IBM library (declared in include/lbmibm.h): argument
// checks, carving of the caller buffers, the per-step kernel sequence and
// field import/export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_plan.h"
#include "internal.h"

namespace {

thread_local std::string g_create_error;

}  // namespace

void set_noalloc_error(const std::string& msg) { g_create_error = msg; }

namespace {

lbm_status fail(lbm_ctx* c, lbm_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return LBM_ERR_HIP;
}

#define HIP_TRY(ctx, expr)                                    \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);  \
  } while (0)

void fill_geom(lbm_ctx* c, const Plan& pl) {
  lbmd::LatticeGeom& g = c->geom;
  const lbm_params& p = c->p;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  for (int a = 0; a < 3; ++a) g.bc[a] = p.bc[a];
  g.ncell = pl.ncell;
  g.spop = pl.spop;
  g.srow = pl.srow;
  g.splane = pl.splane;
  g.lat_elems = pl.lat_elems;
  for (int a = 0; a < 3; ++a)
    for (int f = 0; f < 2; ++f)
      for (int i = 0; i < lbmd::Q; ++i) {
        const double* u = p.wall_u[a][f];
        const double eu = lbmd::EX[i] * u[0] + lbmd::EY[i] * u[1] + lbmd::EZ[i] * u[2];
        g.bb_add[a][f][i] = (float)(6.0 * lbmd::wgt_d(i) * p.rho_wall * eu);
      }
  g.tau = (float)p.tau;
  g.omega = (float)(1.0 / p.tau);
  for (int a = 0; a < 3; ++a) g.g_ext[a] = (float)p.g_ext[a];
  g.fblk_x = pl.fblk[0];
  g.fblk_y = pl.fblk[1];
}

// Timing: events recorded on the stream at the boundaries of the phases.
// The interval from one event to the next is charged to the phase that
// began at the first (ev_kind: 0 forcing, 1 stream-collide, -1 none).  With
// `chain` (nothing enqueued since the last event, which closed a phase) that
// event also opens the new phase, so consecutive phases share a boundary
// and each costs one event record.
void ev_mark(lbm_ctx* c, int kind, bool chain) {
  if (!c->timing) return;
  if (chain && c->ev_used > 0 && c->ev_kind[c->ev_used - 1] < 0) {
    c->ev_kind[c->ev_used - 1] = kind;
    return;
  }
  if (c->ev_used >= c->ev_pool.size()) {
    size_t old = c->ev_pool.size();
    c->ev_pool.resize(std::max<size_t>(64, 2 * old));
    for (size_t k = old; k < c->ev_pool.size(); ++k) (void)hipEventCreate(&c->ev_pool[k]);
  }
  (void)hipEventRecord(c->ev_pool[c->ev_used++], c->stream);
  c->ev_kind.resize(c->ev_used);
  c->ev_kind[c->ev_used - 1] = kind;
}

void ev_collect(lbm_ctx* c) {
  if (c->ev_used == 0) return;
  (void)hipEventSynchronize(c->ev_pool[c->ev_used - 1]);
  for (size_t k = 0; k + 1 < c->ev_used; ++k) {
    const int kind = c->ev_kind[k];
    if (kind < 0) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]);
    c->t_acc[kind] += ms;
    c->t_acc[2 + kind] += 1.0;
  }
  c->ev_used = 0;
  c->ev_kind.clear();
}

// chain: see ev_mark.
lbm_status do_forcing(lbm_ctx* c, bool chain) {
  if ((c->flags & IBM_WARM_START) && !c->theta_set)
    return fail(c, LBM_ERR_STATE, "IBM_WARM_START needs ibm_set_mlp first");
  ev_mark(c, 0, chain);
  hipError_t e = launch_forcing(c);
  if (e != hipSuccess) return hip_fail(c, e, "forcing");
  ev_mark(c, -1, false);
  if (c->flags & IBM_WARM_PREV) c->du_prev_valid = true;
  c->g_valid_step = c->step;
  return LBM_OK;
}

// Statistics of the last forcing: FP64 sums of the point partials; with a
// residual stop, the sweeps run come from the device control block.
lbm_status read_stats(lbm_ctx* c, ibm_stats* stats) {
  hipError_t e = launch_reduce_point_stats(c, c->small);
  if (e != hipSuccess) return hip_fail(c, e, "reduce point stats");
  double h[2 + LBM_MAX_ITER];
  uint32_t ctl[4] = {0, 0, 0, 0};
  HIP_TRY(c, hipMemcpyAsync(h, c->small, sizeof(double) * (2 + c->n_iter), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(ctl, c->ctl, sizeof(ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const bool gated = (c->flags & (IBM_STOP_RESIDUAL | IBM_WARM_START | IBM_WARM_PREV)) != 0;
  const int ran = gated ? std::min<int>((int)ctl[1], c->n_iter) : c->n_iter;
  std::memset(stats, 0, sizeof(*stats));
  stats->n_iter = ran;
  stats->sum_s = h[0];
  stats->sum_s_ub2 = h[1];
  for (int it = 0; it < ran; ++it) stats->resid[it] = h[2 + it];
  return LBM_OK;
}

// The non-finite check: reads the sticky status words (synchronises) and
// turns a raised word into LBM_ERR_NONFINITE naming where it was raised.
lbm_status check_status(lbm_ctx* c, const char* where) {
  uint32_t* h = c->meta_host + 4;  // pinned words 4..7
  HIP_TRY(c, hipMemcpyAsync(h, c->status, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->check_since = 0;
  if (!h[0] && !h[1]) return LBM_OK;
  std::string m = std::string("non-finite state detected ") + where + " (step " +
                  std::to_string(c->step) + ", checked every " +
                  std::to_string(c->check_every) + " step(s)):";
  if (h[0]) m += " mass/momentum sums not finite;";
  if (h[1]) m += " a forcing spread value not finite or beyond 4096;";
  return fail(c, LBM_ERR_NONFINITE, m);
}

}  // namespace

extern "C" {

lbm_status lbm_buffer_sizes(const lbm_params* p, size_t sizes_out[LBM_NBUF]) {
  std::string msg;
  lbm_status st = check_params(p, msg);
  if (st != LBM_OK) {
    g_create_error = msg;
    return st;
  }
  if (!sizes_out) {
    g_create_error = "sizes_out is NULL";
    return LBM_ERR_ARG;
  }
  Plan pl;
  make_plan(p, pl);
  for (int b = 0; b < LBM_NBUF; ++b) sizes_out[b] = pl.size[b];
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, void* const bufs[LBM_NBUF], lbm_ctx** out) {
  std::string msg;
  lbm_status st = check_params(p, msg);
  if (st != LBM_OK) {
    g_create_error = msg;
    return st;
  }
  if (!out || !bufs) {
    g_create_error = "bufs or out is NULL";
    return LBM_ERR_ARG;
  }
  for (int b = 0; b < LBM_NBUF; ++b)
    if (!bufs[b] || ((uintptr_t)bufs[b] % ALIGN) != 0) {
      g_create_error = "buffer " + std::to_string(b) + " is NULL or not 256-byte aligned";
      return LBM_ERR_OOM;
    }
  Plan pl;
  make_plan(p, pl);
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->stream = (hipStream_t)p->stream;
  (void)hipGetDevice(&c->device);
  c->ncell = pl.ncell;
  for (int a = 0; a < 3; ++a) c->tiles[a] = pl.tiles[a];
  c->ntiles = pl.ntiles;
  c->elem = pl.elem;
  fill_geom(c, pl);

  char* L = (char*)bufs[LBM_BUF_LATTICE];
  c->lat[0] = L;
  c->lat[1] = L + pl.lat_bytes;
  char* F = (char*)bufs[LBM_BUF_FIELDS];
  c->U = (float4*)F;
  c->G = (float*)(F + pl.o_G);
  char* P = (char*)bufs[LBM_BUF_POINTS];
  c->rest = (float4*)(P + pl.o_rest);
  c->body_of = (int32_t*)(P + pl.o_body_of);
  c->key = (uint32_t*)(P + pl.o_key);
  c->rank = (uint32_t*)(P + pl.o_rank);
  c->sp_base = (int4*)(P + pl.o_base);
  c->sp_frac = (float4*)(P + pl.o_frac);
  c->sp_ub = (float4*)(P + pl.o_ub);
  c->sp_g = (float4*)(P + pl.o_g);
  c->sp_du = (float4*)(P + pl.o_du);
  c->sp_tmp = (int4*)(P + pl.o_tmp);
  c->bodies = (double*)(P + pl.o_bodies);
  c->motion = (BodyMotion*)(P + pl.o_motion);
  c->nbr = (int32_t*)(P + pl.o_nbr);
  c->g0_orig = (float4*)(P + pl.o_g0);
  c->du_prev = (float4*)(P + pl.o_duprev);
  c->feat = (float*)(P + pl.o_feat);
  c->vref = (float*)(P + pl.o_vref);
  c->ubox = (float*)(P + pl.o_ubox);
  c->theta = (float*)(P + pl.o_theta);
  c->theta_packed = (void*)(P + pl.o_packed);
  c->boxbuf = (void*)(F + pl.o_box);
  c->max_boxes = pl.max_boxes;
  char* T = (char*)bufs[LBM_BUF_TILES];
  for (int a = 0; a < 3; ++a) c->fblk[a] = pl.fblk[a];
  c->nblocks4 = pl.nblocks4;
  c->nbflag_words = pl.nbflag_words;
  c->cnt_own = (uint32_t*)(T + pl.o_cnt_own);
  c->cnt_touch = (uint32_t*)(T + pl.o_cnt_touch);
  c->start_own = (uint32_t*)(T + pl.o_start_own);
  c->end_own = (uint32_t*)(T + pl.o_end_own);
  c->own_slot = (int32_t*)(T + pl.o_own_slot);
  c->own_tiles = (uint32_t*)(T + pl.o_own_tiles);
  c->touch_tiles = (uint32_t*)(T + pl.o_touch_tiles);
  c->meta = (uint32_t*)(T + pl.o_meta);
  c->bflag = (uint8_t*)(T + pl.o_bflag);
  c->chunk_tot = (uint32_t*)(T + pl.o_chunk);
  char* S = (char*)bufs[LBM_BUF_SCRATCH];
  c->sum_partials = (double*)(S + pl.o_sum_part);
  c->n_cell_blocks = pl.n_cell_blocks;
  c->pt_partials = (double*)(S + pl.o_pt_part);
  c->part_row = pl.part_row;
  c->small = (double*)(S + pl.o_small);
  c->ctl = (uint32_t*)(S + pl.o_ctl);
  c->resid_thr = (double*)(S + pl.o_thr);
  c->status = (uint32_t*)(S + pl.o_status);

  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = launch_fill_u32(c, c->cnt_own, 0u, c->ntiles);
  if (e == hipSuccess) e = launch_fill_u32(c, c->cnt_touch, 0u, c->ntiles);
  if (e == hipSuccess) e = launch_fill_u32(c, c->meta, 0u, 4);
  if (e == hipSuccess) e = launch_fill_u32(c, c->ctl, 0u, 4);
  if (e == hipSuccess) e = launch_fill_u32(c, c->status, 0u, 4);
  if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t*)c->bflag, 0u, c->nbflag_words);
  if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t*)c->U, 0u, pl.o_G / sizeof(uint32_t));
  if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t*)c->G, 0u, 3 * c->ncell);
  if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t*)c->sum_partials, 0u, 8 * c->n_cell_blocks);
  if (e == hipSuccess) e = launch_init_equilibrium(c);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->meta_host, 8 * sizeof(uint32_t), hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->meta_host_dev, c->meta_host, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->meta_event, hipEventDisableTiming);
  if (e != hipSuccess) {
    g_create_error = std::string("initialisation: ") + hipGetErrorString(e);
    if (c->meta_host) (void)hipHostFree(c->meta_host);
    if (c->meta_event) (void)hipEventDestroy(c->meta_event);
    delete c;
    return LBM_ERR_HIP;
  }
  c->have_sums = false;
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  for (auto& ev : c->ev_pool) (void)hipEventDestroy(ev);
  if (c->meta_event) {
    (void)hipEventSynchronize(c->meta_event);
    (void)hipEventDestroy(c->meta_event);
  }
  if (c->meta_host) (void)hipHostFree(c->meta_host);
  if (c->stage) (void)hipFree(c->stage);
  delete c;
}

const char* lbm_last_error(const lbm_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

lbm_status ibm_set_points(lbm_ctx* c, int64_t n, const float* rest_xyz, const float* area,
                          const int64_t* body_off, int32_t nbodies, const ibm_body* bodies,
                          int32_t n_iter, uint32_t flags, float eps) {
  if (!c) return LBM_ERR_ARG;
  if (n < 0 || n > c->p.max_points)
    return fail(c, LBM_ERR_ARG, "n must be in [0, max_points]");
  if (n == 0) {
    c->npts = 0;
    c->nbodies = 0;
    c->g_valid_step = -1;
    c->g_prescribed = false;
    hipError_t e = launch_fill_u32(c, (uint32_t*)c->bflag, 0u, c->nbflag_words);
    if (e != hipSuccess) return hip_fail(c, e, "clear force-block flags");
    return LBM_OK;
  }
  SurfaceHost sh;
  std::string msg;
  const lbm_status vst =
      prepare_surface(c->p, n, rest_xyz, area, body_off, nbodies, bodies, n_iter, flags, eps, sh, msg);
  if (vst != LBM_OK) return fail(c, vst, msg);
  HIP_TRY(c, hipMemcpyAsync(c->rest, sh.rest4.data(), sh.rest4.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->body_of, sh.body_of.data(), sh.body_of.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->bodies, sh.btab.data(), sh.btab.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->vref, sh.vref.data(), sh.vref.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->ubox, sh.ubox.data(), sh.ubox.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->npts = n;
  c->nbodies = nbodies;
  c->n_iter = n_iter;
  c->flags = flags;
  c->eps = (flags & IBM_STOP_RESIDUAL) ? eps : 0.0f;
  c->nbr_valid = false;
  c->du_prev_valid = false;
  c->ubox_sub = sh.ubox_sub;
  c->meta_pending = false;  // the stream has been synchronised above
  c->prev_len_valid = false;
  c->g_valid_step = -1;
  c->g_prescribed = false;
  return LBM_OK;
}

lbm_status ibm_force_iterate(lbm_ctx* c, ibm_stats* stats) {
  if (!c) return LBM_ERR_ARG;
  if (c->npts == 0) return fail(c, LBM_ERR_STATE, "no Lagrangian points set");
  lbm_status st = do_forcing(c, false);
  if (st != LBM_OK) return st;
  if (c->check_every > 0) {
    st = check_status(c, "after the forcing");
    if (st != LBM_OK) return st;
  }
  return stats ? read_stats(c, stats) : LBM_OK;
}

lbm_status lbm_set_check(lbm_ctx* c, int32_t every) {
  if (!c) return LBM_ERR_ARG;
  if (every < 0) return fail(c, LBM_ERR_ARG, "every must be >= 0");
  hipError_t e = launch_fill_u32(c, c->status, 0u, 4);
  if (e != hipSuccess) return hip_fail(c, e, "clear status words");
  c->check_every = every;
  c->check_since = 0;
  return LBM_OK;
}

lbm_status ibm_last_stats(lbm_ctx* c, ibm_stats* stats) {
  if (!c) return LBM_ERR_ARG;
  if (!stats) return fail(c, LBM_ERR_ARG, "stats is NULL");
  if (c->npts == 0 || c->g_valid_step < 0)
    return fail(c, LBM_ERR_STATE, "no forcing has run for the current points");
  return read_stats(c, stats);
}

lbm_status ibm_set_mlp(lbm_ctx* c, const float* theta) {
  if (!c) return LBM_ERR_ARG;
  if (!theta) return fail(c, LBM_ERR_ARG, "theta is NULL");
  for (int i = 0; i < IBM_MLP_NPARAM; ++i)
    if (!std::isfinite(theta[i])) return fail(c, LBM_ERR_ARG, "theta must be finite");
  HIP_TRY(c, hipMemcpyAsync(c->theta, theta, sizeof(float) * IBM_MLP_NPARAM, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_mlp_pack(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->theta_set = true;
  return LBM_OK;
}

lbm_status ibm_log_pairs(lbm_ctx* c, float* features, float* targets) {
  if (!c) return LBM_ERR_ARG;
  if (!features || !targets) return fail(c, LBM_ERR_ARG, "NULL destination");
  if (!(c->flags & IBM_KEEP_FEATURES))
    return fail(c, LBM_ERR_STATE, "the surface was set without IBM_KEEP_FEATURES");
  if (c->npts == 0 || c->g_valid_step < 0)
    return fail(c, LBM_ERR_STATE, "no forcing has run for the current points");
  hipError_t e = launch_export_pairs(c, features, targets);
  if (e != hipSuccess) return hip_fail(c, e, "export pairs");
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int32_t n_steps) {
  if (!c) return LBM_ERR_ARG;
  if (n_steps < 0) return fail(c, LBM_ERR_ARG, "n_steps must be >= 0");
  // chain: the last timing event closed a phase of this call and nothing has
  // been enqueued since (see ev_mark)
  bool chain = false;
  for (int32_t s = 0; s < n_steps; ++s) {
    if (c->npts > 0 && c->g_valid_step != c->step) {
      lbm_status st = do_forcing(c, chain);
      if (st != LBM_OK) return st;
      chain = true;
    }
    ev_mark(c, 1, chain);
    hipError_t e = launch_stream_collide(c);
    if (e != hipSuccess) return hip_fail(c, e, "stream_collide");
    ev_mark(c, -1, false);
    chain = true;
    if (c->ev_used > 4000) ev_collect(c);
    c->have_sums = true;
    c->step += 1;
    if (c->check_every > 0 && ++c->check_since >= c->check_every) {
      lbm_status st = check_status(c, "after the stream-collide");
      if (st != LBM_OK) return st;
      chain = false;
    }
  }
  return LBM_OK;
}

}  // extern "C"

namespace {

// The context's device staging buffer for host destinations and sources,
// grown to at least `bytes`.  Each use ends with a synchronisation of the
// context's stream, so a buffer that is replaced is idle.
hipError_t stage_at_least(lbm_ctx* c, size_t bytes, void** p) {
  if (bytes > c->stage_bytes) {
    if (c->stage) {
      const hipError_t e = hipFree(c->stage);
      c->stage = nullptr;
      c->stage_bytes = 0;
      if (e != hipSuccess) return e;
    }
    const hipError_t e = hipMalloc(&c->stage, bytes);
    if (e != hipSuccess) {
      c->stage = nullptr;
      return e;
    }
    c->stage_bytes = bytes;
  }
  *p = c->stage;
  return hipSuccess;
}

}  // namespace

extern "C" {

lbm_status lbm_read_fields(lbm_ctx* c, uint32_t mask, const lbm_fields* dst) {
  if (!c) return LBM_ERR_ARG;
  if (!dst) return fail(c, LBM_ERR_ARG, "dst is NULL");
  const uint32_t known = LBM_F_RHO | LBM_F_VEL | LBM_F_FORCE | LBM_F_POPS | LBM_F_PT_X |
                         LBM_F_PT_UB | LBM_F_PT_G | LBM_F_PT_DU | LBM_F_SUMS | LBM_F_STEP;
  if (mask & ~known) return fail(c, LBM_ERR_ARG, "unknown field bits");
  const bool dev = dst->on_device != 0;
  const size_t nc = (size_t)c->ncell, np = (size_t)c->npts;
  const size_t pop_b = (dst->pops_f64 ? 8 : 4) * 19 * nc;
  if ((mask & LBM_F_RHO) && !dst->rho) return fail(c, LBM_ERR_ARG, "rho is NULL");
  if ((mask & LBM_F_VEL) && !dst->vel) return fail(c, LBM_ERR_ARG, "vel is NULL");
  if ((mask & LBM_F_FORCE) && !dst->force) return fail(c, LBM_ERR_ARG, "force is NULL");
  if ((mask & LBM_F_POPS) && !dst->pops) return fail(c, LBM_ERR_ARG, "pops is NULL");
  if ((mask & LBM_F_SUMS) && !dst->sums) return fail(c, LBM_ERR_ARG, "sums is NULL");
  if ((mask & LBM_F_STEP) && !dst->step) return fail(c, LBM_ERR_ARG, "step is NULL");
  if ((mask & LBM_F_SUMS) && !c->have_sums) return fail(c, LBM_ERR_STATE, "no step has run yet");
  const uint32_t ptm = LBM_F_PT_X | LBM_F_PT_UB | LBM_F_PT_G | LBM_F_PT_DU;
  if (mask & ptm) {
    if (c->g_valid_step < 0) return fail(c, LBM_ERR_STATE, "no forcing has run for the current points");
    if (((mask & LBM_F_PT_X) && !dst->pt_x) || ((mask & LBM_F_PT_UB) && !dst->pt_ub) ||
        ((mask & LBM_F_PT_G) && !dst->pt_g) || ((mask & LBM_F_PT_DU) && !dst->pt_du))
      return fail(c, LBM_ERR_ARG, "NULL point destination");
  }

  // Device destinations, or staging buffers for host ones.
  float *rho = dst->rho, *vel = dst->vel, *force = dst->force;
  void* pops = dst->pops;
  double* ptx = dst->pt_x;
  float *ptub = dst->pt_ub, *ptg = dst->pt_g, *ptdu = dst->pt_du;
  double* sums = dst->sums;
  if (!dev) {
    size_t bytes = 0;
    auto want = [&](uint32_t bit, size_t b) -> size_t {
      if (!(mask & bit)) return 0;
      size_t o = bytes;
      bytes = align_up(bytes + b);
      return o;
    };
    size_t o_rho = want(LBM_F_RHO, 4 * nc), o_vel = want(LBM_F_VEL, 12 * nc),
           o_f = want(LBM_F_FORCE, 12 * nc), o_p = want(LBM_F_POPS, pop_b),
           o_x = want(LBM_F_PT_X, 24 * np), o_ub = want(LBM_F_PT_UB, 12 * np),
           o_g = want(LBM_F_PT_G, 12 * np), o_du = want(LBM_F_PT_DU, 12 * np),
           o_s = want(LBM_F_SUMS, 32);
    void* stage = nullptr;
    if (bytes) HIP_TRY(c, stage_at_least(c, bytes, &stage));
    char* b = (char*)stage;
    rho = (mask & LBM_F_RHO) ? (float*)(b + o_rho) : nullptr;
    vel = (mask & LBM_F_VEL) ? (float*)(b + o_vel) : nullptr;
    force = (mask & LBM_F_FORCE) ? (float*)(b + o_f) : nullptr;
    pops = (mask & LBM_F_POPS) ? (void*)(b + o_p) : nullptr;
    ptx = (mask & LBM_F_PT_X) ? (double*)(b + o_x) : nullptr;
    ptub = (mask & LBM_F_PT_UB) ? (float*)(b + o_ub) : nullptr;
    ptg = (mask & LBM_F_PT_G) ? (float*)(b + o_g) : nullptr;
    ptdu = (mask & LBM_F_PT_DU) ? (float*)(b + o_du) : nullptr;
    sums = (mask & LBM_F_SUMS) ? (double*)(b + o_s) : nullptr;
  } else {
    if (!(mask & LBM_F_RHO)) rho = nullptr;
    if (!(mask & LBM_F_VEL)) vel = nullptr;
    if (!(mask & LBM_F_FORCE)) force = nullptr;
    if (!(mask & LBM_F_POPS)) pops = nullptr;
    if (!(mask & LBM_F_PT_X)) ptx = nullptr;
    if (!(mask & LBM_F_PT_UB)) ptub = nullptr;
    if (!(mask & LBM_F_PT_G)) ptg = nullptr;
    if (!(mask & LBM_F_PT_DU)) ptdu = nullptr;
    if (!(mask & LBM_F_SUMS)) sums = nullptr;
  }
  hipError_t e = hipSuccess;
  if (rho || vel || pops) e = launch_readout(c, rho, vel, pops, dst->pops_f64);
  if (e == hipSuccess && force) e = launch_export_force(c, force);
  if (e == hipSuccess && (ptx || ptub || ptg || ptdu)) e = launch_export_points(c, ptx, ptub, ptg, ptdu);
  if (e == hipSuccess && sums) e = launch_reduce_sums(c, sums);
  if (e != hipSuccess) return hip_fail(c, e, "read_fields");
  if (!dev) {
    auto back = [&](uint32_t bit, void* host, const void* devp, size_t b) -> hipError_t {
      if (!(mask & bit)) return hipSuccess;
      return hipMemcpyAsync(host, devp, b, hipMemcpyDeviceToHost, c->stream);
    };
    HIP_TRY(c, back(LBM_F_RHO, dst->rho, rho, 4 * nc));
    HIP_TRY(c, back(LBM_F_VEL, dst->vel, vel, 12 * nc));
    HIP_TRY(c, back(LBM_F_FORCE, dst->force, force, 12 * nc));
    HIP_TRY(c, back(LBM_F_POPS, dst->pops, pops, pop_b));
    HIP_TRY(c, back(LBM_F_PT_X, dst->pt_x, ptx, 24 * np));
    HIP_TRY(c, back(LBM_F_PT_UB, dst->pt_ub, ptub, 12 * np));
    HIP_TRY(c, back(LBM_F_PT_G, dst->pt_g, ptg, 12 * np));
    HIP_TRY(c, back(LBM_F_PT_DU, dst->pt_du, ptdu, 12 * np));
    HIP_TRY(c, back(LBM_F_SUMS, dst->sums, sums, 32));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (mask & LBM_F_STEP) *dst->step = c->step;
  } else if (mask & LBM_F_STEP) {
    HIP_TRY(c, hipMemcpyAsync(dst->step, &c->step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

lbm_status lbm_write_fields(lbm_ctx* c, uint32_t mask, const lbm_fields* src) {
  if (!c) return LBM_ERR_ARG;
  if (!src) return fail(c, LBM_ERR_ARG, "src is NULL");
  if (mask & ~(uint32_t)(LBM_F_POPS | LBM_F_FORCE | LBM_F_STEP))
    return fail(c, LBM_ERR_ARG, "only POPS, FORCE and STEP can be written");
  if ((mask & LBM_F_POPS) && !src->pops) return fail(c, LBM_ERR_ARG, "pops is NULL");
  if ((mask & LBM_F_FORCE) && !src->force) return fail(c, LBM_ERR_ARG, "force is NULL");
  if ((mask & LBM_F_STEP) && !src->step) return fail(c, LBM_ERR_ARG, "step is NULL");
  if ((mask & LBM_F_FORCE) && c->npts > 0)
    return fail(c, LBM_ERR_STATE, "a prescribed force needs a context without points");
  const bool dev = src->on_device != 0;
  const size_t nc = (size_t)c->ncell;
  if (mask & LBM_F_POPS) {
    const size_t b = (src->pops_f64 ? 8 : 4) * 19 * nc;
    const void* p = src->pops;
    if (!dev) {
      void* stage = nullptr;
      HIP_TRY(c, stage_at_least(c, b, &stage));
      HIP_TRY(c, hipMemcpyAsync(stage, src->pops, b, hipMemcpyHostToDevice, c->stream));
      p = stage;
    }
    hipError_t e = launch_unstream_from(c, p, src->pops_f64);
    if (e != hipSuccess) return hip_fail(c, e, "write pops");
    if (!dev) HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->g_valid_step = -1;
    c->du_prev_valid = false;
  }
  if (mask & LBM_F_FORCE) {
    const float* p = src->force;
    if (!dev) {
      void* stage = nullptr;
      HIP_TRY(c, stage_at_least(c, 12 * nc, &stage));
      HIP_TRY(c, hipMemcpyAsync(stage, src->force, 12 * nc, hipMemcpyHostToDevice, c->stream));
      p = (const float*)stage;
    }
    hipError_t e = launch_copy_f32(c, c->G, p, 3 * c->ncell);
    if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t*)c->bflag, 0x01010101u, c->nbflag_words);
    if (e != hipSuccess) return hip_fail(c, e, "write force");
    if (!dev) HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->g_prescribed = true;
  }
  if (mask & LBM_F_STEP) {
    int64_t s;
    if (dev) {
      HIP_TRY(c, hipMemcpyAsync(&s, src->step, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    } else {
      s = *src->step;
    }
    if (s < 0) return fail(c, LBM_ERR_ARG, "step must be >= 0");
    c->step = s;
    c->g_valid_step = -1;
  }
  return LBM_OK;
}

lbm_status lbm_set_timing(lbm_ctx* c, int32_t enable) {
  if (!c) return LBM_ERR_ARG;
  if (c->timing && !enable) ev_collect(c);
  c->timing = enable != 0;
  for (double& v : c->t_acc) v = 0.0;
  c->ev_used = 0;
  c->ev_kind.clear();
  return LBM_OK;
}

lbm_status lbm_get_timing(lbm_ctx* c, double out[4]) {
  if (!c || !out) return LBM_ERR_ARG;
  ev_collect(c);
  for (int k = 0; k < 4; ++k) out[k] = c->t_acc[k];
  return LBM_OK;
}

}  // extern "C"
