// CPU check of the library's host-side planning (host_plan.cpp, plain C++)
// under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// For many lattice shapes, storage formats, point capacities and sweep
// capacities it checks that the caller buffers are carved into 256-byte
// aligned, disjoint arrays, each large enough for what the kernels index in
// it (the sizes below restate the arrays the header and kernels describe),
// and that parameter checks reject what they should.  It then feeds
// prepare_surface valid and invalid surfaces (non-finite coordinates,
// negative areas, bad body ranges, flag conflicts, supports that cross a
// wall) and checks the statuses and the host layout.  Prints OK on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_plan.h"

namespace {

int fails = 0;
void expect(bool ok, const std::string& what) {
  if (!ok) {
    ++fails;
    if (fails < 20) std::printf("FAIL: %s\n", what.c_str());
  }
}

struct Region {
  int buf;
  size_t off, bytes;
  const char* name;
};

void check_plan(const lbm_params& p) {
  Plan pl;
  make_plan(&p, pl);
  const size_t M = (size_t)(p.max_points > 0 ? p.max_points : 1);
  const size_t nc = (size_t)p.nx * p.ny * p.nz;
  const size_t nt = (size_t)pl.ntiles;
  const size_t np4 = (size_t)((pl.tiles[0] + 3) / 4 * 4) * ((pl.tiles[1] + 3) / 4 * 4) *
                     ((pl.tiles[2] + 3) / 4 * 4);
  const size_t elem = p.storage == LBM_STORE_F32 ? 4 : 2;
  const size_t nb4 = (size_t)((p.nx + 3) / 4) * ((p.ny + 3) / 4) * ((p.nz + 3) / 4);
  std::vector<Region> r = {
      {LBM_BUF_LATTICE, 0, 2 * (size_t)pl.lat_elems * elem, "lattices"},
      {LBM_BUF_FIELDS, 0, nt * 512 * 16, "U"},
      {LBM_BUF_FIELDS, pl.o_G, 3 * nc * 4, "G"},
      {LBM_BUF_FIELDS, pl.o_box, (size_t)pl.max_boxes * BOX_SLOT_BYTES, "boxes"},
      {LBM_BUF_POINTS, pl.o_rest, M * 16, "rest"},
      {LBM_BUF_POINTS, pl.o_body_of, M * 4, "body_of"},
      {LBM_BUF_POINTS, pl.o_key, M * 4, "key"},
      {LBM_BUF_POINTS, pl.o_rank, M * 4, "rank"},
      {LBM_BUF_POINTS, pl.o_base, M * 16, "base"},
      {LBM_BUF_POINTS, pl.o_frac, M * 16, "frac"},
      {LBM_BUF_POINTS, pl.o_ub, M * 16, "ub"},
      {LBM_BUF_POINTS, pl.o_g, M * 16, "g"},
      {LBM_BUF_POINTS, pl.o_du, M * 16, "du"},
      {LBM_BUF_POINTS, pl.o_tmp, M * 16, "binning temporary"},
      {LBM_BUF_POINTS, pl.o_bodies, (size_t)LBM_MAX_BODIES * 64, "bodies"},
      {LBM_BUF_POINTS, pl.o_motion, (size_t)LBM_MAX_BODIES * BODY_MOTION_BYTES, "motion"},
      {LBM_BUF_POINTS, pl.o_nbr, M * 16 * 4, "nbr"},
      {LBM_BUF_POINTS, pl.o_g0, M * 16, "g0"},
      {LBM_BUF_POINTS, pl.o_duprev, M * 16, "du_prev"},
      {LBM_BUF_POINTS, pl.o_feat, M * 12 * 4, "feat"},
      {LBM_BUF_POINTS, pl.o_vref, (size_t)LBM_MAX_BODIES * 4, "vref"},
      {LBM_BUF_POINTS, pl.o_ubox, (size_t)LBM_MAX_BODIES * 24, "ubox"},
      {LBM_BUF_POINTS, pl.o_theta, (size_t)IBM_MLP_NPARAM * 4, "theta"},
      {LBM_BUF_POINTS, pl.o_packed, MLP_PACKED_BYTES, "packed"},
      {LBM_BUF_TILES, pl.o_cnt_own, nt * 4, "cnt_own"},
      {LBM_BUF_TILES, pl.o_cnt_touch, nt * 4, "cnt_touch"},
      {LBM_BUF_TILES, pl.o_start_own, nt * 4, "start_own"},
      {LBM_BUF_TILES, pl.o_end_own, nt * 4, "end_own"},
      {LBM_BUF_TILES, pl.o_own_slot, nt * 4, "own_slot"},
      {LBM_BUF_TILES, pl.o_own_tiles, nt * 4, "own_tiles"},
      {LBM_BUF_TILES, pl.o_touch_tiles, nt * 4, "touch_tiles"},
      {LBM_BUF_TILES, pl.o_meta, 16, "meta"},
      {LBM_BUF_TILES, pl.o_bflag, (nb4 + 3) / 4 * 4, "bflag"},
      // the tile scan: the tile grid padded to whole 4^3 blocks, in chunks of 2048 positions
      {LBM_BUF_TILES, pl.o_chunk, (np4 + 2047) / 2048 * 4 * 4, "chunk totals"},
      {LBM_BUF_SCRATCH, pl.o_sum_part, (size_t)pl.n_cell_blocks * 32, "sum partials"},
      {LBM_BUF_SCRATCH, pl.o_pt_part, (size_t)(p.max_iter + 2) * pl.part_row * 8, "pt partials"},
      {LBM_BUF_SCRATCH, pl.o_small, 256 * 8, "small"},
      {LBM_BUF_SCRATCH, pl.o_ctl, 16, "ctl"},
      {LBM_BUF_SCRATCH, pl.o_thr, 8, "thr"},
      {LBM_BUF_SCRATCH, pl.o_status, 16, "status"},
  };
  const std::string tag = std::to_string(p.nx) + "x" + std::to_string(p.ny) + "x" +
                          std::to_string(p.nz) + " s" + std::to_string(p.storage) + " M" +
                          std::to_string(p.max_points) + ": ";
  // the stream-collide writes one partial per workgroup of its launch
  expect((size_t)pl.n_cell_blocks >= (nc + LBM_BLOCK - 1) / LBM_BLOCK, tag + "cell blocks");
  // a sweep launch writes one residual partial per workgroup (at most one per tile, rounded to 8)
  expect((size_t)pl.part_row >= (nt + 7) / 8 * 8 && (size_t)pl.part_row >= (M + 255) / 256,
         tag + "partial row");
  expect(pl.max_boxes >= 1 && (size_t)pl.max_boxes >= std::min(nt, M), tag + "box count");
  // population layout: rows of interleaved populations, or one array per
  // population; every (population, cell) has its own element, inside the
  // buffer, and cell offsets fit in 32 bits
  const bool inter = pl.srow == 19 * pl.spop;
  if (inter)
    expect(pl.spop >= p.nx && pl.splane == (int64_t)p.ny * pl.srow &&
               (pl.spop * (int64_t)elem) % 128 == 0 && pl.lat_elems * (int64_t)elem < (1ll << 32),
           tag + "interleaved rows");
  else
    expect(pl.srow == p.nx && pl.splane == (int64_t)p.nx * p.ny && pl.spop >= (int64_t)nc &&
               (pl.spop * (int64_t)elem) % (int64_t)ALIGN == 0 && pl.lat_elems == 19 * pl.spop,
           tag + "population arrays");
  const int64_t last_cell = (p.nx - 1) + (int64_t)(p.ny - 1) * pl.srow + (int64_t)(p.nz - 1) * pl.splane;
  expect(last_cell < (1ll << 32) && 18 * pl.spop + last_cell < pl.lat_elems, tag + "layout extent");
  expect((size_t)pl.lat_elems * elem <= pl.lat_bytes && pl.lat_bytes % ALIGN == 0, tag + "lattice bytes");
  for (size_t i = 0; i < r.size(); ++i) {
    expect(r[i].off % ALIGN == 0, tag + r[i].name + " aligned");
    expect(r[i].off + r[i].bytes <= pl.size[r[i].buf], tag + r[i].name + " inside its buffer");
    for (size_t j = 0; j < i; ++j)
      if (r[j].buf == r[i].buf)
        expect(r[i].off >= r[j].off + r[j].bytes || r[j].off >= r[i].off + r[i].bytes,
               tag + r[i].name + " overlaps " + r[j].name);
  }
}

lbm_params base_params(int nx, int ny, int nz) {
  lbm_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.tau = 0.6;
  p.rho_wall = 1.0;
  p.rho0 = 1.0;
  p.max_points = 1000;
  p.max_iter = 8;
  return p;
}

void check_params_cases() {
  std::string msg;
  lbm_params p = base_params(8, 8, 8);
  expect(check_params(&p, msg) == LBM_OK, "valid params");
  expect(check_params(nullptr, msg) == LBM_ERR_ARG, "NULL params");
  lbm_params q = p;
  q.tau = 0.5;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "tau 0.5");
  q = p;
  q.tau = NAN;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "tau NaN");
  q = p;
  q.nx = 0;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "nx 0");
  q = p;
  q.nx = 2048;
  q.ny = 2048;
  q.nz = 1024;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "2^32 cells");
  q = p;
  q.storage = 3;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "storage 3");
  q = p;
  q.max_iter = 65;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "max_iter 65");
  q = p;
  q.wall_u[2][1][2] = INFINITY;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "wall_u inf");
  q = p;
  q.reserved_ = 1;
  expect(check_params(&q, msg) == LBM_ERR_ARG, "reserved");
}

void check_surfaces() {
  lbm_params p = base_params(20, 18, 16);
  p.bc[1] = LBM_BC_BOUNCEBACK;
  const int n = 30;
  std::vector<float> rest(3 * n), area(n);
  for (int k = 0; k < n; ++k) {
    rest[3 * k] = 0.1f * k - 1.5f;
    rest[3 * k + 1] = 0.05f * (k % 7) - 0.2f;
    rest[3 * k + 2] = 0.07f * (k % 5);
    area[k] = 0.3f + 0.01f * k;
  }
  std::vector<int64_t> off = {0, 10, 10, n};
  ibm_body b[3];
  for (int i = 0; i < 3; ++i) {
    b[i].center[0] = 10.0 + i;
    b[i].center[1] = 9.0;
    b[i].center[2] = 8.0;
    b[i].axis[0] = 0.0;
    b[i].axis[1] = 0.0;
    b[i].axis[2] = 1.0 + i;
    b[i].theta0 = 0.1 * i;
    b[i].omega = 0.01;
  }
  std::string msg;
  SurfaceHost sh;
  expect(prepare_surface(p, n, rest.data(), area.data(), off.data(), 3, b, 5, 0, 0.0f, sh, msg) ==
             LBM_OK, "valid surface: " + msg);
  expect(sh.rest4.size() == 4u * n && sh.rest4[4 * 7 + 3] == area[7] && sh.body_of[12] == 2 &&
             sh.btab.size() == 24 && sh.btab[8 * 2 + 5] == 3.0 && sh.ubox_sub >= 1,
         "surface layout");
  auto status = [&](int64_t nn, const float* r, const float* a, const int64_t* o, int nb,
                    const ibm_body* bb, int it, uint32_t fl, float eps) {
    SurfaceHost s2;
    std::string m;
    return prepare_surface(p, nn, r, a, o, nb, bb, it, fl, eps, s2, m);
  };
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 5, IBM_STOP_RESIDUAL, 0.1f) == LBM_OK,
         "residual stop");
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 5, 0, 0.1f) == LBM_ERR_ARG,
         "eps without stop");
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 9, 0, 0.0f) == LBM_ERR_ARG,
         "n_iter beyond max_iter");
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 5, IBM_WARM_START | IBM_WARM_PREV,
                0.0f) == LBM_ERR_ARG, "warm start flags");
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 5, IBM_U_BOX | IBM_U_KERNEL, 0.0f) ==
             LBM_ERR_ARG, "U strategies");
  expect(status(n, rest.data(), area.data(), off.data(), 3, b, 5, 1u << 20, 0.0f) == LBM_ERR_ARG,
         "unknown flag");
  expect(status(1001, rest.data(), area.data(), off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG,
         "n beyond max_points");
  std::vector<int64_t> bad_off = {0, 20, 10, n};
  expect(status(n, rest.data(), area.data(), bad_off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG,
         "decreasing body_off");
  std::vector<int64_t> short_off = {0, 10, 10, n - 1};
  expect(status(n, rest.data(), area.data(), short_off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG,
         "body_off end");
  std::vector<float> r2 = rest;
  r2[3 * 17 + 1] = NAN;
  expect(status(n, r2.data(), area.data(), off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG, "NaN point");
  std::vector<float> a2 = area;
  a2[29] = -1.0f;
  expect(status(n, rest.data(), a2.data(), off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG,
         "negative area");
  ibm_body b2[3] = {b[0], b[1], b[2]};
  b2[1].axis[2] = 0.0;  // body 1 is empty, but its axis is still checked
  expect(status(n, rest.data(), area.data(), off.data(), 3, b2, 5, 0, 0.0f) == LBM_ERR_ARG,
         "zero axis");
  b2[1] = b[1];
  b2[2].center[1] = 2.0;  // support reaches the wall at y = -1/2
  expect(status(n, rest.data(), area.data(), off.data(), 3, b2, 5, 0, 0.0f) == LBM_ERR_DOMAIN,
         "support across a wall");
  expect(status(n, nullptr, area.data(), off.data(), 3, b, 5, 0, 0.0f) == LBM_ERR_ARG, "NULL rest");
}

}  // namespace

int main() {
  check_params_cases();
  const int dims[][3] = {{1, 1, 1},    {2, 5, 4},     {8, 8, 8},       {13, 10, 9},
                         {32, 32, 32}, {130, 3, 2},   {160, 160, 320}, {256, 256, 256},
                         {17, 33, 65}, {255, 1, 257}, {64, 8, 1},      {9, 100, 7}};
  const int64_t caps[] = {0, 1, 295, 4096, 1596800};
  for (const auto& d : dims)
    for (int s = 0; s < 3; ++s)
      for (int64_t m : caps)
        for (int it : {1, 5, 64}) {
          lbm_params p = base_params(d[0], d[1], d[2]);
          p.storage = s;
          p.max_points = m;
          p.max_iter = it;
          std::string msg;
          expect(check_params(&p, msg) == LBM_OK, "params " + msg);
          check_plan(p);
        }
  check_surfaces();
  if (fails) {
    std::printf("FAILED %d\n", fails);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
