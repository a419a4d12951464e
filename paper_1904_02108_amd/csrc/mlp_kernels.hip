// Learned warm start of the multi-direct forcing (not part of the paper):
// per-point neighbour lists, features, the MLP 12 -> 64 -> 64 -> 64 -> 3
// (SiLU) forward pass, and its training (forward, backward, Adam) on
// batches of (features, converged correction) pairs.
//
// Parameter layout (row-major, out x in):
//   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
#include <mutex>
#include <string>

#include "internal.h"

using namespace lbmd;

namespace {

constexpr int NIN = IBM_MLP_NFEAT, NH = 64, NOUT = 3;
constexpr int NPARAM = IBM_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH,
              OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NOUT * NH;
static_assert(OFF_B4 + NOUT == NPARAM, "MLP parameter layout");
constexpr int NNBR = IBM_MLP_NNBR;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
// The same with the hardware reciprocal (about 1 ulp), for the matrix-core
// networks.
__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Whole forward pass of one sample with the parameters in LDS (FP32).
__device__ __forceinline__ void mlp_eval(const float* __restrict__ P, const float x[NIN],
                                         float y[NOUT]) {
  float a[NH], b[NH];
#pragma unroll 4
  for (int o = 0; o < NH; ++o) {
    float s = P[OFF_B1 + o];
#pragma unroll
    for (int i = 0; i < NIN; ++i) s += P[OFF_W1 + o * NIN + i] * x[i];
    a[o] = silu(s);
  }
#pragma unroll 2
  for (int o = 0; o < NH; ++o) {
    float s = P[OFF_B2 + o];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += P[OFF_W2 + o * NH + i] * a[i];
    b[o] = silu(s);
  }
#pragma unroll 2
  for (int o = 0; o < NH; ++o) {
    float s = P[OFF_B3 + o];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += P[OFF_W3 + o * NH + i] * b[i];
    a[o] = silu(s);
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float s = P[OFF_B4 + o];
#pragma unroll
    for (int i = 0; i < NH; ++i) s += P[OFF_W4 + o * NH + i] * a[i];
    y[o] = s;
  }
}

__device__ __forceinline__ void load_params(const float* __restrict__ theta, float* P) {
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) P[i] = theta[i];
  __syncthreads();
}

// y[n][3] = MLP(x[n][12]), one thread per sample.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ theta, int64_t n,
                                                     const float* __restrict__ x,
                                                     float* __restrict__ y) {
  __shared__ float P[NPARAM];
  load_params(theta, P);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float xi[NIN], yo[NOUT];
#pragma unroll
  for (int i = 0; i < NIN; ++i) xi[i] = x[k * NIN + i];
  mlp_eval(P, xi, yo);
#pragma unroll
  for (int c = 0; c < NOUT; ++c) y[k * NOUT + c] = yo[c];
}

// ---------------------------------------------------------------------------
// BF16 matrix-core form of the forward pass (FP32 accumulation), for batches
// of points: one wave evaluates 32 points with 22 MFMA 32x32x16 operations.
// Each layer is computed transposed, H_out^T[64 x 32] = W[64 x K] H_in^T[K x 32],
// so a lane's accumulator registers (one point, 16 hidden units per 32-unit
// block) are directly the B operand of the next layer once converted to
// BF16.  The K order inside a chunk is therefore the accumulator's row order;
// the packed weights (A operands) use the same order, so the sum over K is
// unchanged.  Accumulator register r of lane l (half h = l / 32) holds row
// 8 (r / 4) + 4 h + r % 4 of its 32-row block; the A and B operands hold K
// elements 8 h .. 8 h + 7 of a 16-wide chunk (row / column l % 32).
// Packed operand list (64 lanes x 8 BF16 each):
//   0-1: layer 1, output block b;       2-9: layer 2, (b_out, b_in, chunk);
//   10-17: layer 3, same;               18-21: layer 4 (rows 0-2), (b_in, chunk).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int N_MFMA = 22;

// Eight values as BF16 (round to nearest even; gfx950 converts two per
// instruction).
__device__ __forceinline__ bf16x8 pack8(const float* v) {
  bf16x8 w;
#pragma unroll
  for (int e = 0; e < 8; ++e) w[e] = (__bf16)v[e];
  return w;
}

// Hidden unit held by element e of the B operand of chunk c of input block b
// in lane half h (the accumulator row of register 8 c + e).
__device__ __forceinline__ int chunk_unit(int b, int c, int h, int e) {
  return 32 * b + 16 * c + 8 * (e >> 2) + 4 * h + (e & 3);
}

// theta (FP32 flat layout) -> packed[N_MFMA][64] A operands.
__global__ __launch_bounds__(64) void k_mlp_pack(const float* __restrict__ theta,
                                                 u32x4* __restrict__ packed) {
  const int m = blockIdx.x, l = threadIdx.x, i = l & 31, h = l >> 5;
  float w[8];
  for (int e = 0; e < 8; ++e) {
    float v = 0.0f;
    if (m < 2) {
      const int k = 8 * h + e;
      v = k < NIN ? theta[OFF_W1 + (32 * m + i) * NIN + k] : 0.0f;
    } else if (m < 18) {
      const int q = (m - 2) & 7, off = m < 10 ? OFF_W2 : OFF_W3;
      const int bo = q >> 2, bi = (q >> 1) & 1, c = q & 1;
      v = theta[off + (32 * bo + i) * NH + chunk_unit(bi, c, h, e)];
    } else {
      const int q = m - 18, bi = q >> 1, c = q & 1;
      v = i < NOUT ? theta[OFF_W4 + i * NH + chunk_unit(bi, c, h, e)] : 0.0f;
    }
    w[e] = v;
  }
  const bf16x8 a = pack8(w);
  packed[m * 64 + l] = __builtin_bit_cast(u32x4, a);
}

struct MfmaWeights {
  u32x4 A[N_MFMA * 64];
  float bias[3 * NH + NOUT];
};

__device__ __forceinline__ void load_mfma_weights(const u32x4* __restrict__ packed,
                                                  const float* __restrict__ theta, MfmaWeights& W) {
  for (int i = threadIdx.x; i < N_MFMA * 64; i += blockDim.x) W.A[i] = packed[i];
  for (int i = threadIdx.x; i < NH; i += blockDim.x) {
    W.bias[i] = theta[OFF_B1 + i];
    W.bias[NH + i] = theta[OFF_B2 + i];
    W.bias[2 * NH + i] = theta[OFF_B3 + i];
  }
  if (threadIdx.x < NOUT) W.bias[3 * NH + threadIdx.x] = theta[OFF_B4 + threadIdx.x];
  __syncthreads();
}

// Bias and SiLU on the two 32-row accumulator blocks of a hidden layer, then
// conversion to the four B operands of the next layer.
__device__ __forceinline__ void hidden_to_operands(const f32x16 acc[2], const float* bias, int h,
                                                   bf16x8 B[4]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    float a[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      a[r] = silu_fast(acc[b][r] + bias[32 * b + 8 * (r >> 2) + 4 * h + (r & 3)]);
    B[2 * b] = pack8(a);
    B[2 * b + 1] = pack8(a + 8);
  }
}

// Forward pass of the 32 points of one wave: x8 holds features 8 h .. 8 h + 7
// of point l % 32 (zeros beyond 12); on lanes 0-31 y receives the outputs.
__device__ __forceinline__ void mlp_group_mfma(const MfmaWeights& W, const float x8[8], float y[3]) {
  const int l = __lane_id(), h = l >> 5;
  const f32x16 zero = {};
  bf16x8 B[4];
  f32x16 acc[2];
  const bf16x8 X = pack8(x8);
#pragma unroll
  for (int b = 0; b < 2; ++b)
    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
        __builtin_bit_cast(bf16x8, W.A[b * 64 + l]), X, zero, 0, 0, 0);
  hidden_to_operands(acc, W.bias, h, B);
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int m0 = 2 + 8 * layer;
#pragma unroll
    for (int bo = 0; bo < 2; ++bo) {
      f32x16 a = zero;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, W.A[(m0 + 4 * bo + q) * 64 + l]), B[q], a, 0, 0, 0);
      acc[bo] = a;
    }
    hidden_to_operands(acc, W.bias + NH * (layer + 1), h, B);
  }
  f32x16 o = zero;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, W.A[(18 + q) * 64 + l]),
                                                B[q], o, 0, 0, 0);
  y[0] = o[0] + W.bias[3 * NH];
  y[1] = o[1] + W.bias[3 * NH + 1];
  y[2] = o[2] + W.bias[3 * NH + 2];
}

// Features of point k, elements 8 h .. 8 h + 7 (zeros past the 12th).
__device__ __forceinline__ void load_x8(const float* __restrict__ x, int64_t k, int64_t n, int h,
                                        float x8[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = 8 * h + e;
    x8[e] = (k < n && f < NIN) ? x[k * NIN + f] : 0.0f;
  }
}

constexpr int MFMA_WG = 256;  // 4 waves, 32 points each per group

__global__ __launch_bounds__(MFMA_WG) void k_mlp_forward_mfma(const u32x4* __restrict__ packed,
                                                              const float* __restrict__ theta,
                                                              int64_t n, const float* __restrict__ x,
                                                              float* __restrict__ y) {
  __shared__ MfmaWeights W;
  load_mfma_weights(packed, theta, W);
  const int l = __lane_id(), h = l >> 5, wave = threadIdx.x >> 6;
  const int64_t groups = (n + 31) / 32;
  for (int64_t g = (int64_t)blockIdx.x * (MFMA_WG / 64) + wave; g < groups;
       g += (int64_t)gridDim.x * (MFMA_WG / 64)) {
    // weights and biases are re-read from LDS for every group: kept in
    // registers across groups they would take most of the register file
    // and leave one wave per SIMD to hide the gathers' latency
    asm volatile("" ::: "memory");
    const int64_t k = 32 * g + (l & 31);
    float x8[8], yo[3];
    load_x8(x, k, n, h, x8);
    mlp_group_mfma(W, x8, yo);
    if (h == 0 && k < n) {
      y[k * NOUT] = yo[0];
      y[k * NOUT + 1] = yo[1];
      y[k * NOUT + 2] = yo[2];
    }
  }
}

// Sum, component-wise max and count of g0 over entries 8 half .. 8 half + 7
// of N(orig) (the list's -1 pads come last): two 16-byte loads of indices,
// then the eight deficits loaded together.  The features add the two halves'
// sums (half 0 + half 1), the same in both feature kernels.
__device__ __forceinline__ void nbr_half(const int32_t* __restrict__ nbr,
                                         const float4* __restrict__ g0_orig, int orig, int half,
                                         float s[3], float mx[3], int& cnt) {
  const int4* row = reinterpret_cast<const int4*>(nbr + (int64_t)orig * NNBR) + 2 * half;
  const int4 a = row[0], b = row[1];
  const int q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  float4 gq[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) gq[e] = q[e] >= 0 ? g0_orig[q[e]] : make_float4(0.f, 0.f, 0.f, 0.f);
  s[0] = s[1] = s[2] = 0.0f;
  mx[0] = mx[1] = mx[2] = -INFINITY;
  cnt = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if (q[e] < 0) continue;
    s[0] += gq[e].x;
    s[1] += gq[e].y;
    s[2] += gq[e].z;
    mx[0] = fmaxf(mx[0], gq[e].x);
    mx[1] = fmaxf(mx[1], gq[e].y);
    mx[2] = fmaxf(mx[2], gq[e].z);
    ++cnt;
  }
}

// Elements 8 h .. 8 h + 7 of the features of point k (sorted order; the same
// definition as k_features_warm): g0, u_b, mean and component-wise max of g0
// over N(k), divided by v_ref.  Each half-wave gathers half of the
// neighbours; the two halves of a point (lanes l and l ^ 32) exchange their
// partial sums, so every lane of the wave must call this.
__device__ __forceinline__ void features8(int64_t k, int64_t n, int h,
                                          const int4* __restrict__ sp_base,
                                          const float4* __restrict__ sp_g,
                                          const float4* __restrict__ sp_ub,
                                          const float4* __restrict__ g0_orig,
                                          const int32_t* __restrict__ nbr,
                                          const int32_t* __restrict__ body_of,
                                          const float* __restrict__ vref, float x8[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) x8[e] = 0.0f;
  const bool live = k < n;  // the same for both halves of a point
  const int orig = live ? sp_base[k].w : 0;
  float sh[3], mh[3];
  int ch;
  nbr_half(nbr, g0_orig, orig, h, sh, mh, ch);
  float m[3], mx[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float so = __shfl_xor(sh[c], 32, 64), mo = __shfl_xor(mh[c], 32, 64);
    m[c] = h == 0 ? sh[c] + so : so + sh[c];  // half 0 + half 1 on both
    mx[c] = fmaxf(mh[c], mo);
  }
  const int cnt = ch + __shfl_xor(ch, 32, 64);
  if (!live) return;
  const float inv = 1.0f / vref[body_of[orig]];
  const float mean[3] = {cnt ? m[0] / (float)cnt * inv : 0.0f, cnt ? m[1] / (float)cnt * inv : 0.0f,
                         cnt ? m[2] / (float)cnt * inv : 0.0f};
  if (h == 0) {
    const float4 g = sp_g[k], ub = sp_ub[k];
    x8[0] = g.x * inv;
    x8[1] = g.y * inv;
    x8[2] = g.z * inv;
    x8[3] = ub.x * inv;
    x8[4] = ub.y * inv;
    x8[5] = ub.z * inv;
    x8[6] = mean[0];
    x8[7] = mean[1];
  } else {
    x8[0] = mean[2];
    x8[1] = cnt ? mx[0] * inv : 0.0f;
    x8[2] = cnt ? mx[1] * inv : 0.0f;
    x8[3] = cnt ? mx[2] * inv : 0.0f;
  }
}

// Warm start: du = s v_ref y, unless the forcing has already converged
// (*gate).  Features from the stored array (feat != nullptr, sorted order) or
// computed here from the first deficit.
__global__ __launch_bounds__(MFMA_WG) void k_warm_mfma(
    const u32x4* __restrict__ packed, const float* __restrict__ theta, int64_t n,
    const float* __restrict__ feat, const int4* __restrict__ sp_base,
    const float4* __restrict__ sp_frac, const int32_t* __restrict__ body_of,
    const float* __restrict__ vref, const uint32_t* __restrict__ gate, float4* __restrict__ sp_du,
    const float4* __restrict__ sp_g, const float4* __restrict__ sp_ub,
    const float4* __restrict__ g0_orig, const int32_t* __restrict__ nbr) {
  __shared__ MfmaWeights W;
  if (*gate) return;
  load_mfma_weights(packed, theta, W);
  const int l = __lane_id(), h = l >> 5, wave = threadIdx.x >> 6;
  const int64_t groups = (n + 31) / 32;
  for (int64_t g = (int64_t)blockIdx.x * (MFMA_WG / 64) + wave; g < groups;
       g += (int64_t)gridDim.x * (MFMA_WG / 64)) {
    // weights and biases are re-read from LDS for every group: kept in
    // registers across groups they would take most of the register file
    // and leave one wave per SIMD to hide the gathers' latency
    asm volatile("" ::: "memory");
    const int64_t k = 32 * g + (l & 31);
    float x8[8], yo[3];
    if (feat)
      load_x8(feat, k, n, h, x8);
    else
      features8(k, n, h, sp_base, sp_g, sp_ub, g0_orig, nbr, body_of, vref, x8);
    mlp_group_mfma(W, x8, yo);
    if (h == 0 && k < n) {
      const float sv = sp_frac[k].w * vref[body_of[sp_base[k].w]];
      sp_du[k] = make_float4(yo[0] * sv, yo[1] * sv, yo[2] * sv, 0.0f);
    }
  }
}

// ---------------------------------------------------------------------------
// The same network with FP32 operands on the matrix cores
// (v_mfma_f32_32x32x2_f32: a 32 x 32 block, two K values per instruction,
// one operand value per lane).  Lane l holds row / column l % 32 and the K
// value of its half h = l / 32.  The K order of a contraction is free, so
// step s of a hidden layer's input block b takes, in half h, hidden unit
// 32 b + 8 (s / 4) + 4 h + s % 4: the accumulator row that the same lane
// holds in register s.  The activations then feed the next layer from the
// lane's own registers, with no exchange between lanes.  Step s of the
// first layer takes feature 8 h + s (zero past the 12th).  The output layer
// (3 rows) runs on the vector units: a matrix instruction would compute 29
// rows of zeros.
// Packed operand list (64 lanes x 1 FP32 each):
//   0-15: layer 1, (block, step);        16-79: layer 2, (b_out, b_in, step);
//   80-143: layer 3, same.
// ---------------------------------------------------------------------------
constexpr int N_MFMA32 = 144;
static_assert((size_t)N_MFMA32 * 64 * 4 == MLP_PACKED_F32_BYTES, "FP32 operand count");

__device__ __forceinline__ int step_unit(int b, int s, int h) {
  return 32 * b + 8 * (s >> 2) + 4 * h + (s & 3);
}

// theta (FP32 flat layout) -> packed32[N_MFMA32][64] A operands.
__global__ __launch_bounds__(64) void k_mlp_pack32(const float* __restrict__ theta,
                                                   float* __restrict__ packed32) {
  const int m = blockIdx.x, l = threadIdx.x, i = l & 31, h = l >> 5;
  float v = 0.0f;
  if (m < 16) {
    const int bo = m >> 3, k = 8 * h + (m & 7);
    v = k < NIN ? theta[OFF_W1 + (32 * bo + i) * NIN + k] : 0.0f;
  } else {
    const int q = (m - 16) & 63, off = m < 80 ? OFF_W2 : OFF_W3;
    const int bo = q >> 5, bi = (q >> 4) & 1, st = q & 15;
    v = theta[off + (32 * bo + i) * NH + step_unit(bi, st, h)];
  }
  packed32[m * 64 + l] = v;
}

struct MfmaWeights32 {
  float A[N_MFMA32 * 64];
  float W4[NOUT * NH];  // output layer, row-major
  float bias[3 * NH + NOUT];
};

__device__ __forceinline__ void load_mfma_weights32(const float* __restrict__ packed32,
                                                    const float* __restrict__ theta,
                                                    MfmaWeights32& W) {
  for (int i = threadIdx.x; i < N_MFMA32 * 64; i += blockDim.x) W.A[i] = packed32[i];
  for (int i = threadIdx.x; i < NOUT * NH; i += blockDim.x) W.W4[i] = theta[OFF_W4 + i];
  for (int i = threadIdx.x; i < NH; i += blockDim.x) {
    W.bias[i] = theta[OFF_B1 + i];
    W.bias[NH + i] = theta[OFF_B2 + i];
    W.bias[2 * NH + i] = theta[OFF_B3 + i];
  }
  if (threadIdx.x < NOUT) W.bias[3 * NH + threadIdx.x] = theta[OFF_B4 + threadIdx.x];
  __syncthreads();
}

// Bias and SiLU on the two 32-row accumulator blocks of a hidden layer, in
// place (the next layer's B operands); the reciprocal of the SiLU to about
// 1 ulp.
__device__ __forceinline__ void hidden_act32(f32x16 acc[2], const float* bias, int h) {
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = silu_fast(acc[b][r] + bias[step_unit(b, r, h)]);
}

// Forward pass of the 32 points of one wave in FP32 (x8 and y as in
// mlp_group_mfma).
__device__ __forceinline__ void mlp_group_mfma32(const MfmaWeights32& W, const float x8[8],
                                                 float y[3]) {
  const int l = __lane_id(), h = l >> 5;
  const f32x16 zero = {};
  f32x16 act[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    f32x16 a = zero;
#pragma unroll
    for (int st = 0; st < 8; ++st)
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(W.A[(8 * b + st) * 64 + l], x8[st], a, 0, 0, 0);
    act[b] = a;
  }
  hidden_act32(act, W.bias, h);
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int m0 = 16 + 64 * layer;
    f32x16 nxt[2];
#pragma unroll
    for (int bo = 0; bo < 2; ++bo) {
      f32x16 a = zero;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int st = 0; st < 16; ++st)
          a = __builtin_amdgcn_mfma_f32_32x32x2f32(W.A[(m0 + 32 * bo + 16 * bi + st) * 64 + l],
                                                   act[bi][st], a, 0, 0, 0);
      nxt[bo] = a;
    }
    act[0] = nxt[0];
    act[1] = nxt[1];
    hidden_act32(act, W.bias + NH * (layer + 1), h);
  }
  // output layer: each half-wave's 32 hidden units, then the halves added
  float p[NOUT] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int u = step_unit(bi, st, h);
#pragma unroll
      for (int j = 0; j < NOUT; ++j) p[j] = fmaf(W.W4[j * NH + u], act[bi][st], p[j]);
    }
#pragma unroll
  for (int j = 0; j < NOUT; ++j) y[j] = p[j] + __shfl_xor(p[j], 32, 64) + W.bias[3 * NH + j];
}

// Warm start with the FP32 network (as k_warm_mfma otherwise).
__global__ __launch_bounds__(MFMA_WG) void k_warm_mfma32(
    const float* __restrict__ packed32, const float* __restrict__ theta, int64_t n,
    const float* __restrict__ feat, const int4* __restrict__ sp_base,
    const float4* __restrict__ sp_frac, const int32_t* __restrict__ body_of,
    const float* __restrict__ vref, const uint32_t* __restrict__ gate, float4* __restrict__ sp_du,
    const float4* __restrict__ sp_g, const float4* __restrict__ sp_ub,
    const float4* __restrict__ g0_orig, const int32_t* __restrict__ nbr) {
  __shared__ MfmaWeights32 W;
  if (*gate) return;
  load_mfma_weights32(packed32, theta, W);
  const int l = __lane_id(), h = l >> 5, wave = threadIdx.x >> 6;
  const int64_t groups = (n + 31) / 32;
  for (int64_t g = (int64_t)blockIdx.x * (MFMA_WG / 64) + wave; g < groups;
       g += (int64_t)gridDim.x * (MFMA_WG / 64)) {
    asm volatile("" ::: "memory");  // weights re-read from LDS for every group
    const int64_t k = 32 * g + (l & 31);
    float x8[8], yo[3];
    if (feat)
      load_x8(feat, k, n, h, x8);
    else
      features8(k, n, h, sp_base, sp_g, sp_ub, g0_orig, nbr, body_of, vref, x8);
    mlp_group_mfma32(W, x8, yo);
    if (h == 0 && k < n) {
      const float sv = sp_frac[k].w * vref[body_of[sp_base[k].w]];
      sp_du[k] = make_float4(yo[0] * sv, yo[1] * sv, yo[2] * sv, 0.0f);
    }
  }
}

unsigned mfma_grid(int64_t n) {
  const int64_t groups = (n + 31) / 32;
  const int64_t wgs = (groups + MFMA_WG / 64 - 1) / (MFMA_WG / 64);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(wgs, 2048));
}

// ---------------------------------------------------------------------------
// Neighbour lists N(k): up to 16 points of k's body nearest to k, at
// Euclidean distance < 2, ordered by (distance, caller index), stored by
// caller index (-1 pads).  Distances are taken between the rest positions
// r (body frame), in FP64 as ((dx^2 + dy^2) + dz^2) with every operation
// rounded (no fused multiply-add), so the lists are exact and independent of
// the rotation.  Candidates come from the points binned by owner tile at the
// current step: a point within distance 2 has its base cell within 3 cells
// of k's on every axis (rounding of the lattice position included), hence in
// one of at most three distinct tiles per axis.
// ---------------------------------------------------------------------------
struct NbrGeom {
  int n[3], bc[3], tiles[3];
};

__device__ __forceinline__ int cell_coord(int v, int n, int bc) {
  if (bc == LBM_BC_PERIODIC) {
    v %= n;
    return v < 0 ? v + n : v;
  }
  return min(max(v, 0), n - 1);
}

// Distinct tiles of the cells base-3 .. base+3 along one axis.
__device__ __forceinline__ int tile_span(int base, int n, int bc, int out[3]) {
  int cnt = 0;
  for (int d = -3; d <= 3; ++d) {
    const int t = cell_coord(base + d, n, bc) >> TILE_SHIFT;
    bool fresh = true;
    for (int j = 0; j < cnt; ++j) fresh = fresh && out[j] != t;
    if (fresh && cnt < 3) out[cnt++] = t;
  }
  return cnt;
}

__device__ __forceinline__ double rest_dist2(float4 a, float4 b) {
#pragma clang fp contract(off)
  const double dx = (double)b.x - (double)a.x;
  const double dy = (double)b.y - (double)a.y;
  const double dz = (double)b.z - (double)a.z;
  return (dx * dx + dy * dy) + dz * dz;
}

// Lattice-frame separation of two binned points along one axis (nearest
// image on periodic axes).
__device__ __forceinline__ float lat_sep(int b0, float f0, int b1, float f1, int n, int bc) {
  float d = (float)(b1 - b0) + (f1 - f0);
  if (bc == LBM_BC_PERIODIC) {
    const float h = 0.5f * (float)n;
    if (d > h) d -= (float)n;
    else if (d < -h) d += (float)n;
  }
  return fabsf(d);
}

__global__ __launch_bounds__(256) void k_neighbours(
    const uint32_t* __restrict__ start_own, const uint32_t* __restrict__ end_own,
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_frac,
    const float4* __restrict__ rest, const int32_t* __restrict__ body_of, int64_t npts, NbrGeom ng,
    int32_t* __restrict__ nbr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npts) return;
  const int4 b = sp_base[k];
  const float4 fk = sp_frac[k];
  const int me = b.w;
  const float4 rk = rest[me];
  const int body = body_of[me];
  double bd[NNBR];
  int bi[NNBR];
#pragma unroll
  for (int j = 0; j < NNBR; ++j) {
    bd[j] = 4.0;  // squared distance bound (distance < 2)
    bi[j] = INT32_MAX;
  }
  int tx[3], ty[3], tz[3];
  const int nx = tile_span(b.x, ng.n[0], ng.bc[0], tx);
  const int ny = tile_span(b.y, ng.n[1], ng.bc[1], ty);
  const int nz = tile_span(b.z, ng.n[2], ng.bc[2], tz);
  for (int iz = 0; iz < nz; ++iz)
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        const uint32_t t = (uint32_t)tx[ix] +
                           (uint32_t)ng.tiles[0] * ((uint32_t)ty[iy] + (uint32_t)ng.tiles[1] * (uint32_t)tz[iz]);
        const uint32_t q1 = end_own[t];
#pragma unroll 4
        for (uint32_t q = start_own[t]; q < q1; ++q) {
          // cheap filter in the lattice frame (the rigid motion keeps
          // distances; 1e-3 covers the rounding of the FP32 fractions)
          const int4 qb = sp_base[q];
          const float4 qf = sp_frac[q];
          if (lat_sep(b.x, fk.x, qb.x, qf.x, ng.n[0], ng.bc[0]) >= 2.001f ||
              lat_sep(b.y, fk.y, qb.y, qf.y, ng.n[1], ng.bc[1]) >= 2.001f ||
              lat_sep(b.z, fk.z, qb.z, qf.z, ng.n[2], ng.bc[2]) >= 2.001f)
            continue;
          const int id = qb.w;
          if (id == me || body_of[id] != body) continue;
          const double d2 = rest_dist2(rk, rest[id]);
          // (the sentinel 4.0 must not admit points at distance exactly 2)
          if (d2 < 4.0 && (d2 < bd[NNBR - 1] || (d2 == bd[NNBR - 1] && id < bi[NNBR - 1]))) {
            // insertion into the list sorted by (distance, index)
            double cd = d2;
            int ci = id;
#pragma unroll
            for (int j = 0; j < NNBR; ++j) {
              const bool before = cd < bd[j] || (cd == bd[j] && ci < bi[j]);
              const double td = bd[j];
              const int ti = bi[j];
              bd[j] = before ? cd : td;
              bi[j] = before ? ci : ti;
              cd = before ? td : cd;
              ci = before ? ti : ci;
            }
          }
        }
      }
#pragma unroll
  for (int j = 0; j < NNBR; ++j) nbr[(int64_t)me * NNBR + j] = bi[j] == INT32_MAX ? -1 : bi[j];
}

// ---------------------------------------------------------------------------
// Features of every point after the first sweep (kept in sorted order for
// logging): g0 (3), u_b (3), mean and component-wise max of g0 over N(k)
// (3 + 3, zeros for an empty N(k)), all divided by v_ref of k's body.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_features_warm(
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_g,
    const float4* __restrict__ sp_ub, const float4* __restrict__ g0_orig,
    const int32_t* __restrict__ nbr, const int32_t* __restrict__ body_of,
    const float* __restrict__ vref, int64_t npts, float* __restrict__ feat) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npts) return;
  const int orig = sp_base[k].w;
  const float v = vref[body_of[orig]];
  const float inv = 1.0f / v;
  const float4 g = sp_g[k];
  const float4 ub = sp_ub[k];
  float s0[3], s1[3], x0[3], x1[3], m[3], mx[3];
  int c0, c1;
  nbr_half(nbr, g0_orig, orig, 0, s0, x0, c0);
  nbr_half(nbr, g0_orig, orig, 1, s1, x1, c1);
  for (int c = 0; c < 3; ++c) {
    m[c] = s0[c] + s1[c];
    mx[c] = fmaxf(x0[c], x1[c]);
  }
  const int cnt = c0 + c1;
  float x[NIN];
  x[0] = g.x * inv;
  x[1] = g.y * inv;
  x[2] = g.z * inv;
  x[3] = ub.x * inv;
  x[4] = ub.y * inv;
  x[5] = ub.z * inv;
  for (int c = 0; c < 3; ++c) {
    x[6 + c] = cnt ? m[c] / (float)cnt * inv : 0.0f;
    x[9 + c] = cnt ? mx[c] * inv : 0.0f;
  }
  for (int i = 0; i < NIN; ++i) feat[k * NIN + i] = x[i];
}

// Training pairs in caller order: the features and t = du / (s v_ref)
// (0 where s = 0).
__global__ __launch_bounds__(256) void k_export_pairs(
    const int4* __restrict__ sp_base, const float4* __restrict__ sp_frac,
    const float* __restrict__ feat, const float4* __restrict__ sp_du,
    const int32_t* __restrict__ body_of, const float* __restrict__ vref, int64_t npts,
    float* __restrict__ fout, float* __restrict__ tout) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npts) return;
  const int orig = sp_base[k].w;
  for (int i = 0; i < NIN; ++i) fout[(int64_t)orig * NIN + i] = feat[k * NIN + i];
  const float s = sp_frac[k].w;
  const float inv = s > 0.0f ? 1.0f / (s * vref[body_of[orig]]) : 0.0f;
  const float4 d = sp_du[k];
  tout[(int64_t)orig * 3] = d.x * inv;
  tout[(int64_t)orig * 3 + 1] = d.y * inv;
  tout[(int64_t)orig * 3 + 2] = d.z * inv;
}

// ---------------------------------------------------------------------------
// Training.  Activations of a batch live in the workspace:
//   Z1,H1,Z2,H2,Z3,H3: [B][64]; Y: [B][3]; dZ (reused per layer): [B][64]
// One thread per sample runs each dense layer (weights in LDS); the weight
// gradients sum outer products over the batch in per-workgroup partials that
// a second kernel reduces in a fixed order.
// ---------------------------------------------------------------------------
struct TrainWS {
  float *Z1, *H1, *Z2, *H2, *Z3, *H3, *Y, *D3, *D2, *D1;  // D4 is stored in Y's slot of dY
  float* dY;
  float* grad;      // [NPARAM]
  float* partials;  // [n_chunks][NPARAM]
  double* loss_part;  // [n_blocks]
  double* small;      // [4]
  int64_t B, n_chunks;
};

constexpr int CHUNK = 128;  // samples per weight-gradient workgroup

// Forward of layer l for every sample: Z = W A + b, H = silu(Z) (no SiLU on
// the output layer, which also writes dL/dy and the squared error).
template <int IN, int OUT, bool LAST>
__global__ __launch_bounds__(256) void k_layer_fwd(const float* __restrict__ theta, int offW,
                                                   int offB, int64_t n, const float* __restrict__ A,
                                                   float* __restrict__ Z, float* __restrict__ H,
                                                   const float* __restrict__ T, float* __restrict__ dY,
                                                   double inv3n, double* __restrict__ loss_part) {
  __shared__ float W[OUT * IN + OUT];
  for (int i = threadIdx.x; i < OUT * IN; i += blockDim.x) W[i] = theta[offW + i];
  for (int i = threadIdx.x; i < OUT; i += blockDim.x) W[OUT * IN + i] = theta[offB + i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (s < n) {
    float a[IN];
#pragma unroll
    for (int i = 0; i < IN; ++i) a[i] = A[s * IN + i];
    for (int o = 0; o < OUT; ++o) {
      float z = W[OUT * IN + o];
#pragma unroll
      for (int i = 0; i < IN; ++i) z += W[o * IN + i] * a[i];
      if (LAST) {
        const float r = z - T[s * OUT + o];
        sq += (double)r * r;
        dY[s * OUT + o] = (float)(2.0 * inv3n) * r;
      } else {
        Z[s * OUT + o] = z;
        H[s * OUT + o] = silu(z);
      }
    }
  }
  if (LAST) {
    __shared__ double red[4];
    const double v = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv3n;
  }
}

// Backward data of layer l: D_in = (W^T D_out) * silu'(Z_in).
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_layer_bwd(const float* __restrict__ theta, int offW,
                                                   int64_t n, const float* __restrict__ Dout,
                                                   const float* __restrict__ Zin,
                                                   float* __restrict__ Din) {
  __shared__ float W[OUT * IN];
  for (int i = threadIdx.x; i < OUT * IN; i += blockDim.x) W[i] = theta[offW + i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float d[OUT];
#pragma unroll
  for (int o = 0; o < OUT; ++o) d[o] = Dout[s * OUT + o];
  for (int i = 0; i < IN; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int o = 0; o < OUT; ++o) acc += W[o * IN + i] * d[o];
    Din[s * IN + i] = acc * silu_grad(Zin[s * IN + i]);
  }
}

// Weight and bias gradient partials of one layer: per chunk of CHUNK samples,
// gW[o][i] = sum_s D[s][o] A[s][i], gb[o] = sum_s D[s][o].
template <int IN, int OUT>
__global__ __launch_bounds__(256) void k_layer_wgrad(int64_t n, const float* __restrict__ D,
                                                     const float* __restrict__ A, int offW,
                                                     int offB, float* __restrict__ partials) {
  __shared__ float sD[CHUNK][OUT];
  __shared__ float sA[CHUNK][IN];
  const int64_t s0 = (int64_t)blockIdx.x * CHUNK;
  const int cnt = (int)min<int64_t>(CHUNK, n - s0);
  for (int i = threadIdx.x; i < CHUNK * OUT; i += blockDim.x) {
    const int s = i / OUT, o = i % OUT;
    sD[s][o] = s < cnt ? D[(s0 + s) * OUT + o] : 0.0f;
  }
  for (int i = threadIdx.x; i < CHUNK * IN; i += blockDim.x) {
    const int s = i / IN, c = i % IN;
    sA[s][c] = s < cnt ? A[(s0 + s) * IN + c] : 0.0f;
  }
  __syncthreads();
  float* part = partials + (int64_t)blockIdx.x * NPARAM;
  for (int w = threadIdx.x; w < OUT * IN + OUT; w += blockDim.x) {
    float acc = 0.f;
    if (w < OUT * IN) {
      const int o = w / IN, i = w % IN;
      for (int s = 0; s < CHUNK; ++s) acc += sD[s][o] * sA[s][i];
      part[offW + w] = acc;
    } else {
      const int o = w - OUT * IN;
      for (int s = 0; s < CHUNK; ++s) acc += sD[s][o];
      part[offB + o] = acc;
    }
  }
}

// Sum of the chunk partials (fixed order) into grad.
__global__ __launch_bounds__(256) void k_reduce_grad(const float* __restrict__ partials,
                                                     int64_t n_chunks, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  double s = 0.0;
  for (int64_t c = 0; c < n_chunks; ++c) s += partials[c * NPARAM + p];
  grad[p] = (float)s;
}

__global__ __launch_bounds__(256) void k_reduce_loss(const double* __restrict__ part, int64_t nb,
                                                     double* out) {
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  __shared__ double red[4];
  const double v = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// Adam with bias correction (c1 = 1 - beta1^t, c2 = 1 - beta2^t).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr,
                                              float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gp = g[p];
  const float mp = 0.9f * m[p] + 0.1f * gp;
  const float vp = 0.999f * v[p] + 0.001f * gp * gp;
  m[p] = mp;
  v[p] = vp;
  theta[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + 1e-8f);
}

constexpr size_t ws_align(size_t v) { return (v + 255) / 256 * 256; }

// Workspace bytes of a training batch of B samples (the carving of carve_ws).
constexpr size_t ws_bytes(int64_t batch) {
  const int64_t B = batch < 1 ? 1 : batch;
  const int64_t nch = (B + CHUNK - 1) / CHUNK;
  return 9 * ws_align((size_t)B * NH * 4) + ws_align((size_t)B * NOUT * 4) +
         ws_align((size_t)NPARAM * 4) + ws_align((size_t)nch * NPARAM * 4) +
         ws_align((size_t)((B + 255) / 256) * 8) + ws_align(4 * 8);
}

// Library-held workspace of mlp_loss_grad_noalloc, for callers that cannot
// allocate device memory: one copy per device, sized for batches of at most
// MLP_NOALLOC_MAX_BATCH samples (about 2.7 MB).  Every byte a batch reads is
// written earlier in the same call (activations, chunk partials, loss
// partials), so nothing needs clearing between calls; calls that overlap on
// one device share it and race.
constexpr size_t MLP_NOALLOC_BYTES = ws_bytes(MLP_NOALLOC_MAX_BATCH);
__device__ __align__(256) unsigned char scratch[MLP_NOALLOC_BYTES];

// Sum of an epoch's batch losses on the device, in batch order: s[1] =
// s[1] + s[0] (s[1] = s[0] for the first batch), read once per epoch.
__global__ void k_loss_acc(double* s, bool first) { s[1] = (first ? 0.0 : s[1]) + s[0]; }

TrainWS carve_ws(void* ws, int64_t B) {
  TrainWS w;
  char* p = (char*)ws;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    char* r = p + at;
    at = ws_align(at + bytes);
    return r;
  };
  w.B = B;
  w.n_chunks = (B + CHUNK - 1) / CHUNK;
  w.Z1 = (float*)take(B * NH * 4);
  w.H1 = (float*)take(B * NH * 4);
  w.Z2 = (float*)take(B * NH * 4);
  w.H2 = (float*)take(B * NH * 4);
  w.Z3 = (float*)take(B * NH * 4);
  w.H3 = (float*)take(B * NH * 4);
  w.D3 = (float*)take(B * NH * 4);
  w.D2 = (float*)take(B * NH * 4);
  w.D1 = (float*)take(B * NH * 4);
  w.dY = (float*)take(B * NOUT * 4);
  w.Y = nullptr;
  w.grad = (float*)take((size_t)NPARAM * 4);
  w.partials = (float*)take((size_t)w.n_chunks * NPARAM * 4);
  w.loss_part = (double*)take((size_t)((B + 255) / 256) * 8);
  w.small = (double*)take(4 * 8);
  return w;
}

// Loss and gradient of one batch [x, x + B).
hipError_t batch_grad(const float* theta, int64_t B, const float* x, const float* t, float* grad,
                      double* loss, const TrainWS& w, hipStream_t st) {
  const unsigned nb = (unsigned)((B + 255) / 256);
  const double inv3n = 1.0 / (3.0 * (double)B);
  k_layer_fwd<NIN, NH, false><<<nb, 256, 0, st>>>(theta, OFF_W1, OFF_B1, B, x, w.Z1, w.H1, nullptr,
                                                  nullptr, 0.0, nullptr);
  k_layer_fwd<NH, NH, false><<<nb, 256, 0, st>>>(theta, OFF_W2, OFF_B2, B, w.H1, w.Z2, w.H2, nullptr,
                                                 nullptr, 0.0, nullptr);
  k_layer_fwd<NH, NH, false><<<nb, 256, 0, st>>>(theta, OFF_W3, OFF_B3, B, w.H2, w.Z3, w.H3, nullptr,
                                                 nullptr, 0.0, nullptr);
  k_layer_fwd<NH, NOUT, true><<<nb, 256, 0, st>>>(theta, OFF_W4, OFF_B4, B, w.H3, nullptr, nullptr,
                                                  t, w.dY, inv3n, w.loss_part);
  k_layer_bwd<NH, NOUT><<<nb, 256, 0, st>>>(theta, OFF_W4, B, w.dY, w.Z3, w.D3);
  k_layer_bwd<NH, NH><<<nb, 256, 0, st>>>(theta, OFF_W3, B, w.D3, w.Z2, w.D2);
  k_layer_bwd<NH, NH><<<nb, 256, 0, st>>>(theta, OFF_W2, B, w.D2, w.Z1, w.D1);
  const unsigned nc = (unsigned)((B + CHUNK - 1) / CHUNK);
  k_layer_wgrad<NH, NOUT><<<nc, 256, 0, st>>>(B, w.dY, w.H3, OFF_W4, OFF_B4, w.partials);
  k_layer_wgrad<NH, NH><<<nc, 256, 0, st>>>(B, w.D3, w.H2, OFF_W3, OFF_B3, w.partials);
  k_layer_wgrad<NH, NH><<<nc, 256, 0, st>>>(B, w.D2, w.H1, OFF_W2, OFF_B2, w.partials);
  k_layer_wgrad<NIN, NH><<<nc, 256, 0, st>>>(B, w.D1, x, OFF_W1, OFF_B1, w.partials);
  k_reduce_grad<<<(NPARAM + 255) / 256, 256, 0, st>>>(w.partials, (int64_t)nc, grad);
  if (loss) k_reduce_loss<<<1, 256, 0, st>>>(w.loss_part, nb, loss);
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_neighbours(lbm_ctx* c) {
  NbrGeom ng;
  const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int a = 0; a < 3; ++a) {
    ng.n[a] = dims[a];
    ng.bc[a] = c->p.bc[a];
    ng.tiles[a] = c->tiles[a];
  }
  const unsigned nb = (unsigned)((c->npts + 255) / 256);
  if (nb == 0) return hipSuccess;
  k_neighbours<<<nb, 256, 0, c->stream>>>(c->start_own, c->end_own, c->sp_base, c->sp_frac, c->rest,
                                          c->body_of, c->npts, ng, c->nbr);
  return hipGetLastError();
}

hipError_t launch_features_warm(lbm_ctx* c) {
  const unsigned nb = (unsigned)((c->npts + 255) / 256);
  if (nb == 0) return hipSuccess;
  k_features_warm<<<nb, 256, 0, c->stream>>>(c->sp_base, c->sp_g, c->sp_ub, c->g0_orig, c->nbr,
                                             c->body_of, c->vref, c->npts, c->feat);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(lbm_ctx* c) {
  k_mlp_pack<<<N_MFMA, 64, 0, c->stream>>>(c->theta, (u32x4*)c->theta_packed);
  k_mlp_pack32<<<N_MFMA32, 64, 0, c->stream>>>(
      c->theta, (float*)((char*)c->theta_packed + MLP_PACKED_BF16_BYTES));
  return hipGetLastError();
}

hipError_t launch_warm_mfma(lbm_ctx* c, bool from_stored_features) {
  if (c->npts == 0) return hipSuccess;
  k_warm_mfma<<<mfma_grid(c->npts), MFMA_WG, 0, c->stream>>>(
      (const u32x4*)c->theta_packed, c->theta, c->npts, from_stored_features ? c->feat : nullptr,
      c->sp_base, c->sp_frac, c->body_of, c->vref, c->ctl, c->sp_du, c->sp_g, c->sp_ub, c->g0_orig,
      c->nbr);
  return hipGetLastError();
}

hipError_t launch_warm_mfma32(lbm_ctx* c, bool from_stored_features) {
  if (c->npts == 0) return hipSuccess;
  k_warm_mfma32<<<mfma_grid(c->npts), MFMA_WG, 0, c->stream>>>(
      (const float*)((const char*)c->theta_packed + MLP_PACKED_BF16_BYTES), c->theta, c->npts,
      from_stored_features ? c->feat : nullptr, c->sp_base, c->sp_frac, c->body_of, c->vref,
      c->ctl, c->sp_du, c->sp_g, c->sp_ub, c->g0_orig, c->nbr);
  return hipGetLastError();
}

hipError_t launch_export_pairs(lbm_ctx* c, float* feat, float* targets) {
  const unsigned nb = (unsigned)((c->npts + 255) / 256);
  if (nb == 0) return hipSuccess;
  k_export_pairs<<<nb, 256, 0, c->stream>>>(c->sp_base, c->sp_frac, c->feat, c->sp_du, c->body_of,
                                            c->vref, c->npts, feat, targets);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the array's name is only a host-side
// stand-in for it).
static lbm_status noalloc_workspace(void** out) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static void* addr[MAX_DEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEV) {
    set_noalloc_error(std::string("mlp_loss_grad_noalloc: no usable current device: ") +
                      hipGetErrorString(e));
    return LBM_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_noalloc_error(std::string("mlp_loss_grad_noalloc: hipGetSymbolAddress: ") +
                        hipGetErrorString(e));
      return LBM_ERR_HIP;
    }
    addr[dev] = p;
  }
  *out = addr[dev];
  return LBM_OK;
}

extern "C" {

size_t mlp_workspace_size(int64_t batch) { return ws_bytes(batch); }

lbm_status mlp_forward(const float* theta, int64_t n, const float* x, float* y, int32_t precision,
                       void* workspace, void* stream) {
  if (!theta || n < 0 || (n > 0 && (!x || !y))) return LBM_ERR_ARG;
  if (precision != MLP_FP32 && precision != MLP_BF16) return LBM_ERR_ARG;
  if (precision == MLP_BF16 && !workspace) return LBM_ERR_ARG;
  if (n == 0) return LBM_OK;
  hipStream_t st = (hipStream_t)stream;
  if (precision == MLP_FP32) {
    k_mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(theta, n, x, y);
  } else {
    u32x4* packed = (u32x4*)workspace;
    k_mlp_pack<<<N_MFMA, 64, 0, st>>>(theta, packed);
    k_mlp_forward_mfma<<<mfma_grid(n), MFMA_WG, 0, st>>>(packed, theta, n, x, y);
  }
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status mlp_loss_grad(const float* theta, int64_t n, const float* x, const float* t,
                         float* grad, double* loss_out, void* workspace, void* stream) {
  if (!theta || n < 1 || !x || !t || !grad || !workspace) return LBM_ERR_ARG;
  const TrainWS w = carve_ws(workspace, n);
  hipError_t e = batch_grad(theta, n, x, t, grad, loss_out, w, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status mlp_loss_grad_noalloc(const float* theta, int64_t n, const float* x, const float* t,
                                 float* grad, double* loss_out, void* stream) {
  if (!theta || n < 1 || !x || !t || !grad) {
    set_noalloc_error("mlp_loss_grad_noalloc: a pointer is NULL or n < 1");
    return LBM_ERR_ARG;
  }
  if (n > MLP_NOALLOC_MAX_BATCH) {
    set_noalloc_error("mlp_loss_grad_noalloc: n = " + std::to_string(n) +
                      " exceeds the library workspace's batch limit of " +
                      std::to_string(MLP_NOALLOC_MAX_BATCH) + " samples");
    return LBM_ERR_ARG;
  }
  void* ws = nullptr;
  const lbm_status st = noalloc_workspace(&ws);
  if (st != LBM_OK) return st;
  const TrainWS w = carve_ws(ws, n);
  hipError_t e = batch_grad(theta, n, x, t, grad, loss_out, w, (hipStream_t)stream);
  if (e != hipSuccess) {
    set_noalloc_error(std::string("mlp_loss_grad_noalloc: ") + hipGetErrorString(e));
    return LBM_ERR_HIP;
  }
  return LBM_OK;
}

lbm_status mlp_train(float* theta, float* m, float* v, int64_t* step_t, int64_t n, const float* x,
                     const float* t, int64_t batch, int32_t n_epochs, double lr,
                     double* loss_per_epoch, void* workspace, void* stream) {
  if (!theta || !m || !v || !step_t || n < 1 || !x || !t || batch < 1 || n_epochs < 0 ||
      !workspace || !(lr > 0.0))
    return LBM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const TrainWS w = carve_ws(workspace, batch);
  float* grad = w.grad;
  for (int ep = 0; ep < n_epochs; ++ep) {
    int64_t nbatches = 0;
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int64_t B = std::min<int64_t>(batch, n - b0);
      hipError_t e = batch_grad(theta, B, x + b0 * NIN, t + b0 * NOUT, grad, w.small, w, st);
      if (e != hipSuccess) return LBM_ERR_HIP;
      *step_t += 1;
      const float c1 = (float)(1.0 - std::pow(0.9, (double)*step_t));
      const float c2 = (float)(1.0 - std::pow(0.999, (double)*step_t));
      k_adam<<<(NPARAM + 255) / 256, 256, 0, st>>>(theta, grad, m, v, (float)lr, c1, c2);
      if (hipGetLastError() != hipSuccess) return LBM_ERR_HIP;
      if (loss_per_epoch) {
        k_loss_acc<<<1, 1, 0, st>>>(w.small, nbatches == 0);
        if (hipGetLastError() != hipSuccess) return LBM_ERR_HIP;
      }
      ++nbatches;
    }
    if (loss_per_epoch) {
      double acc = 0.0;
      if (hipMemcpyAsync(&acc, w.small + 1, sizeof(double), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return LBM_ERR_HIP;
      loss_per_epoch[ep] = nbatches ? acc / (double)nbatches : 0.0;
    }
  }
  return LBM_OK;
}

}  // extern "C"
