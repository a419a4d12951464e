// Sizes and constants shared by the host-side planning code (host_plan.cpp,
// which is plain C++ without HIP) and the HIP sources: the D3Q19 population
// count, the tile and force-block edges, workgroup and table sizes, and the
// byte sizes of the device structures the host carves room for.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace lbmd {
constexpr int Q = 19;         // D3Q19 populations
constexpr int TILE = 8;       // edge of the cubic tiles the forcing works on
constexpr int TILE_SHIFT = 3;
constexpr int FBLK = 4;       // edge of the cubic blocks flagged as touched by a support
constexpr int FBLK_SHIFT = 2;
}  // namespace lbmd

constexpr int LBM_MAX_BODIES = 65536;
constexpr int LBM_BLOCK = 256;  // threads per workgroup of the cell and point kernels
// bytes per stored spread box (11^3 cells: packed x/y sums, z sums, unit)
constexpr int BOX_SLOT_BYTES = 16384;
// matrix-core operands of the warm-start network: BF16 (22 operands x 64
// lanes x 8 values), then FP32 (144 operands x 64 lanes x 1 value)
constexpr size_t MLP_PACKED_BF16_BYTES = 22 * 64 * 16;
constexpr size_t MLP_PACKED_F32_BYTES = 144 * 64 * 4;
constexpr size_t MLP_PACKED_BYTES = MLP_PACKED_BF16_BYTES + MLP_PACKED_F32_BYTES;
static_assert(MLP_PACKED_BF16_BYTES % 256 == 0, "FP32 operands 256-byte aligned");
constexpr size_t BODY_MOTION_BYTES = 10 * sizeof(double);  // struct BodyMotion
constexpr size_t VEC4_BYTES = 16;                          // float4 / int4
