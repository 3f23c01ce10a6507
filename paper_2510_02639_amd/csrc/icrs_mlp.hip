// icrs_mlp.hip -- the learned-bounds network (10 -> 128 -> 128 -> 128 -> 4, GELU) on the
// gfx950 matrix cores: bfloat16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16).
//
// The network is not part of the paper's method; it predicts, for every point-source
// image, the polar box its limb images would span, so the learned path can skip most of
// the limb root solves of the sector step.  Inference, the backward pass of the mean
// squared error and AdamW are all here; the host only sequences calls.
//
// Tiling: a workgroup of four wave64s owns a tile of 64 rows, 16 rows per wave.  Every
// matrix product is a sequence of 16x16x32 MFMAs.  For a 16x32 A block and a 32x16 B
// block, lane l supplies A[l % 16][8 (l / 16) .. + 7] and B[8 (l / 16) .. + 7][l % 16]
// as eight bf16 each, and receives D[4 (l / 16) + i][l % 16], i = 0..3.  Activations live
// in LDS (row pitch padded by 8 halfs); weights are read from a packed bf16 blob that
// holds W and, for the backward products, W transposed, so every operand load is one
// 16-byte vector load.
//
// Determinism: weight gradients are accumulated per workgroup in a private FP32 slice
// (each element is owned by one lane for the whole kernel), then summed over the slices
// in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "icrs_launch.hpp"

namespace icrs {
namespace mlp {
namespace {

constexpr int kIn = 10, kInPad = 32, kHid = 128, kOut = 4, kOutPad = 16;
constexpr int kTile = 64, kThreads = 256;
constexpr int kPitchH = kHid + 8;     // LDS row pitch (halfs) of 128-wide activations
constexpr int kPitchX = kInPad + 8;   // LDS row pitch (halfs) of 32-wide blocks

// FP32 master parameters (padded): W1 [128][32], b1, W2 [128][128], b2, W3, b3, W4 [16][128], b4 [16]
constexpr int oW1 = 0, oB1 = oW1 + kHid * kInPad, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid * kHid, oW4 = oB3 + kHid, oB4 = oW4 + kOutPad * kHid, kParamFloats = oB4 + kOutPad;
// packed bf16: W1 [128][32], W2, W3 [128][128], W4 [16][128], W2t, W3t [128][128] (t[k][n] = W[n][k]),
// W4t [128][32] (rows of W4 beyond 16 are zero)
constexpr int pW1 = 0, pW2 = pW1 + kHid * kInPad, pW3 = pW2 + kHid * kHid, pW4 = pW3 + kHid * kHid,
              pW2t = pW4 + kOutPad * kHid, pW3t = pW2t + kHid * kHid, pW4t = pW3t + kHid * kHid,
              kPackedHalfs = pW4t + kHid * 32;
static_assert(kParamFloats == 39312, "parameter blob layout");
static_assert(kPackedHalfs == 75776, "packed blob layout");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma(u16x8 a, u16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// round to nearest bfloat16, ties to even, NaN stays NaN (gfx950's v_cvt_pk_bf16_f32)
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU, tanh form: x/2 (1 + tanh(c (x + a x^3))), c = sqrt(2/pi), a = 0.044715, evaluated
// as x sigmoid(2 c x (1 + a x^2)) with the hardware base-2 exponential and reciprocal (their
// rounding, a few FP32 units, is far below the bfloat16 the activations are stored in);
// e^{-z} overflowing to infinity gives the limit 0.
constexpr float kGc = 0.7978845608028654f, kGa = 0.044715f, kLog2e = 1.4426950408889634f;
__device__ inline float exp_hw(float u) { return __builtin_amdgcn_exp2f(u * kLog2e); }
__device__ inline float tanh_f(float u) { return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + exp_hw(2.0f * u)); }
__device__ inline float gelu(float x) {
  return x * __builtin_amdgcn_rcpf(1.0f + exp_hw(-2.0f * kGc * x * fmaf(kGa * x, x, 1.0f)));
}
__device__ inline float gelu_grad(float x) {
  const float t = tanh_f(kGc * (x + kGa * x * x * x));
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGc * (1.0f + 3.0f * kGa * x * x);
}

__device__ inline u16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }

// Eight bf16 values down a column of an LDS block (operands of the weight-gradient products).
__device__ inline u16x8 ld8_col(const uint16_t* base, int pitch) {
  u16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = base[j * pitch];
  return v;
}

struct Net {
  const uint16_t* wb;   // packed bf16 weights
  const float* prm;     // FP32 master blob (biases are read from it)
  const float* norm;    // in_mean[10], in_std[10], out_mean[4], out_std[4]
};

// Standardised inputs of rows [row0, row0 + 64) into XS (bf16, zero padding).
__device__ inline void load_inputs(const Net& net, const float* __restrict__ x, int64_t m_rows, int64_t row0,
                                   uint16_t* XS) {
  const int tid = threadIdx.x;
  const int r = tid >> 2, c0 = (tid & 3) * 8;
  const int64_t gm = row0 + r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = c0 + j;
    float v = 0.0f;
    if (c < kIn && gm < m_rows) v = (x[gm * kIn + c] - net.norm[c]) / net.norm[kIn + c];
    XS[r * kPitchX + c] = f2bf(v);
  }
}

// Hidden layer: Hout = bf16(gelu(Hin W^T + b)) for this wave's 16 rows (and G = bf16(gelu')).
template <int KCH, bool STORE_G>
__device__ inline void hidden_layer(const uint16_t* Hin, int pitch_in, const uint16_t* __restrict__ W, int ldw,
                                    const float* __restrict__ bias, uint16_t* Hout, uint16_t* G) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  u16x8 a[KCH];
#pragma unroll
  for (int kc = 0; kc < KCH; ++kc) a[kc] = ld8(Hin + (16 * w + lr) * pitch_in + kc * 32 + 8 * lq);
#pragma unroll 2
  for (int nt = 0; nt < kHid / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) acc = mfma(a[kc], ld8(W + (nt * 16 + lr) * ldw + kc * 32 + 8 * lq), acc);
    const int col = nt * 16 + lr;
    const float b = bias[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * w + 4 * lq + i;
      const float pre = acc[i] + b;
      Hout[row * kPitchH + col] = f2bf(gelu(pre));
      if constexpr (STORE_G) G[row * kPitchH + col] = f2bf(gelu_grad(pre));
    }
  }
}

// Output layer for this wave's rows: returns the standardised outputs of column lr (< 4 real)
// for rows 16 w + 4 lq + i.
__device__ inline f32x4 output_layer(const Net& net, const uint16_t* H3) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < 4; ++kc)
    acc = mfma(ld8(H3 + (16 * w + lr) * kPitchH + kc * 32 + 8 * lq), ld8(net.wb + pW4 + lr * kHid + kc * 32 + 8 * lq),
               acc);
  const float b = net.prm[oB4 + lr];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] += b;
  return acc;
}

// Inference: a workgroup of four waves owns 128 rows, 32 per wave as two 16-row tiles, so each
// 16-byte weight operand feeds two MFMAs (half the weight traffic per row of the 16-row
// tiling, which the vector L1 could not keep up with).  One activation buffer: a layer loads
// its wave's A operands into registers before it writes any output, and each wave reads and
// writes only its own rows, so layers update it in place (45 KB of LDS per workgroup).
constexpr int kFwdTile = 128, kFwdRowsPerWave = 32;

template <int KCH>
__device__ inline void fwd_layer(const uint16_t* Hin, int pitch_in, const uint16_t* __restrict__ W, int ldw,
                                 const float* __restrict__ bias, uint16_t* Hout) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int rw = kFwdRowsPerWave * w;
  // the previous layer's outputs (other lanes of this wave) are visible
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  u16x8 a0[KCH], a1[KCH];
#pragma unroll
  for (int kc = 0; kc < KCH; ++kc) {
    a0[kc] = ld8(Hin + (rw + lr) * pitch_in + kc * 32 + 8 * lq);
    a1[kc] = ld8(Hin + (rw + 16 + lr) * pitch_in + kc * 32 + 8 * lq);
  }
  // the wave's operands are in registers before any of its rows is overwritten
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 2
  for (int nt = 0; nt < kHid / 16; ++nt) {
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) {
      const u16x8 b = ld8(W + (nt * 16 + lr) * ldw + kc * 32 + 8 * lq);
      c0 = mfma(a0[kc], b, c0);
      c1 = mfma(a1[kc], b, c1);
    }
    const int col = nt * 16 + lr;
    const float bb = bias[col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = rw + 4 * lq + i;
      Hout[row * kPitchH + col] = f2bf(gelu(c0[i] + bb));
      Hout[(row + 16) * kPitchH + col] = f2bf(gelu(c1[i] + bb));
    }
  }
}

__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(Net net, const float* __restrict__ x, int64_t m_rows,
                                                               float* __restrict__ y) {
  __shared__ __align__(16) uint16_t XS[kFwdTile * kPitchX];
  __shared__ __align__(16) uint16_t H[kFwdTile * kPitchH];
  const int64_t row0 = (int64_t)blockIdx.x * kFwdTile;
  load_inputs(net, x, m_rows, row0, XS);
  load_inputs(net, x, m_rows, row0 + kTile, XS + kTile * kPitchX);
  __syncthreads();
  fwd_layer<1>(XS, kPitchX, net.wb + pW1, kInPad, net.prm + oB1, H);
  fwd_layer<4>(H, kPitchH, net.wb + pW2, kHid, net.prm + oB2, H);
  fwd_layer<4>(H, kPitchH, net.wb + pW3, kHid, net.prm + oB3, H);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int rw = kFwdRowsPerWave * w;
  f32x4 o0 = {0.f, 0.f, 0.f, 0.f}, o1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const u16x8 b = ld8(net.wb + pW4 + lr * kHid + kc * 32 + 8 * lq);
    o0 = mfma(ld8(H + (rw + lr) * kPitchH + kc * 32 + 8 * lq), b, o0);
    o1 = mfma(ld8(H + (rw + 16 + lr) * kPitchH + kc * 32 + 8 * lq), b, o1);
  }
  if (lr < kOut) {
    const float bb = net.prm[oB4 + lr];
    const float om = net.norm[2 * kIn + lr], os = net.norm[2 * kIn + kOut + lr];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t g0 = row0 + rw + 4 * lq + i, g1 = g0 + 16;
      if (g0 < m_rows) y[g0 * kOut + lr] = (o0[i] + bb) * os + om;
      if (g1 < m_rows) y[g1 * kOut + lr] = (o1[i] + bb) * os + om;
    }
  }
}

// dW[n][k] (+)= sum over the tile's 64 rows of A[m][n] B[m][k] for n-tiles [nt0, nt0 + nn) and
// k-tiles [kt0, kt0 + nk); A, B in LDS.  Each element is owned by one lane of one wave.
__device__ inline void weight_grad(const uint16_t* A, int pa, const uint16_t* B, int pb, int nt0, int nn, int kt0,
                                   int nk, float* __restrict__ dst, int ld, bool first) {
  const int l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  for (int nt = nt0; nt < nt0 + nn; ++nt) {
    const u16x8 a0 = ld8_col(A + (8 * lq) * pa + nt * 16 + lr, pa);
    const u16x8 a1 = ld8_col(A + (32 + 8 * lq) * pa + nt * 16 + lr, pa);
    for (int kt = kt0; kt < kt0 + nk; ++kt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(a0, ld8_col(B + (8 * lq) * pb + kt * 16 + lr, pb), acc);
      acc = mfma(a1, ld8_col(B + (32 + 8 * lq) * pb + kt * 16 + lr, pb), acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float* d = dst + (nt * 16 + 4 * lq + i) * ld + kt * 16 + lr;
        *d = first ? acc[i] : *d + acc[i];
      }
    }
  }
}

// db[n] (+)= sum over rows of bf16 error signal (threads n < width own column n)
__device__ inline void bias_grad(const uint16_t* D, int pitch, int width, float* __restrict__ dst, bool first) {
  const int n = threadIdx.x;
  if (n >= width) return;
  float s = 0.0f;
  for (int m = 0; m < kTile; ++m) s += bf2f(D[m * pitch + n]);
  dst[n] = first ? s : dst[n] + s;
}

// Backward of one hidden layer's input: Dout = bf16((Din W) * G) for this wave's rows,
// Din [rows][n] (K = 32 * KCH), W^T packed as Wt[k][n] with row length ldt.
template <int KCH>
__device__ inline void back_layer(const uint16_t* Din, int pitch_in, const uint16_t* __restrict__ Wt, int ldt,
                                  const uint16_t* G, uint16_t* Dout) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  u16x8 a[KCH];
#pragma unroll
  for (int kc = 0; kc < KCH; ++kc) a[kc] = ld8(Din + (16 * w + lr) * pitch_in + kc * 32 + 8 * lq);
#pragma unroll 2
  for (int kt = 0; kt < kHid / 16; ++kt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) acc = mfma(a[kc], ld8(Wt + (kt * 16 + lr) * ldt + kc * 32 + 8 * lq), acc);
    const int col = kt * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * w + 4 * lq + i;
      Dout[row * kPitchH + col] = f2bf(acc[i] * bf2f(G[row * kPitchH + col]));
    }
  }
}

// Loss and gradient of mean((y - t)^2) over rows and outputs (standardised targets);
// inv = 1 / (4 m_rows).  part: [gridDim.x][kParamFloats] slices, loss_part: [gridDim.x].
__global__ __launch_bounds__(kThreads) void mlp_train_kernel(Net net, const float* __restrict__ x,
                                                             const float* __restrict__ tgt, int64_t m_rows, float inv,
                                                             float* __restrict__ part, float* __restrict__ loss_part) {
  extern __shared__ __align__(16) uint16_t lds[];
  uint16_t* XS = lds;
  uint16_t* DY = XS + kTile * kPitchX;
  uint16_t* H1 = DY + kTile * kPitchX;
  uint16_t* H2 = H1 + kTile * kPitchH;
  uint16_t* H3 = H2 + kTile * kPitchH;
  uint16_t* G1 = H3 + kTile * kPitchH;
  uint16_t* G2 = G1 + kTile * kPitchH;
  uint16_t* G3 = G2 + kTile * kPitchH;
  uint16_t* D0 = G3 + kTile * kPitchH;
  uint16_t* D1 = D0 + kTile * kPitchH;
  __shared__ float red[kThreads / 64];

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lq = l >> 4;
  float* mine = part + (int64_t)blockIdx.x * kParamFloats;
  const int64_t n_tiles = (m_rows + kTile - 1) / kTile;
  float sq = 0.0f;
  bool first = true;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t row0 = tile * kTile;
    load_inputs(net, x, m_rows, row0, XS);
    for (int i = tid; i < kTile * kPitchX; i += kThreads) DY[i] = 0;
    __syncthreads();
    hidden_layer<1, true>(XS, kPitchX, net.wb + pW1, kInPad, net.prm + oB1, H1, G1);
    __syncthreads();
    hidden_layer<4, true>(H1, kPitchH, net.wb + pW2, kHid, net.prm + oB2, H2, G2);
    __syncthreads();
    hidden_layer<4, true>(H2, kPitchH, net.wb + pW3, kHid, net.prm + oB3, H3, G3);
    __syncthreads();
    const f32x4 o = output_layer(net, H3);
    if (lr < kOut) {
      const float om = net.norm[2 * kIn + lr], os = net.norm[2 * kIn + kOut + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * w + 4 * lq + i;
        const int64_t gm = row0 + row;
        if (gm < m_rows) {
          const float diff = o[i] - (tgt[gm * kOut + lr] - om) / os;
          sq += diff * diff;
          DY[row * kPitchX + lr] = f2bf(2.0f * diff * inv);
        }
      }
    }
    __syncthreads();
    // dW4 = DY^T H3 (k-tiles 2w, 2w+1), db4; dH3 = DY W4 -> D0
    weight_grad(DY, kPitchX, H3, kPitchH, 0, 1, 2 * w, 2, mine + oW4, kHid, first);
    bias_grad(DY, kPitchX, kOutPad, mine + oB4, first);
    back_layer<1>(DY, kPitchX, net.wb + pW4t, 32, G3, D0);
    __syncthreads();
    // dW3 = D0^T H2 (n-tiles 2w, 2w+1), db3; dH2 = D0 W3 -> D1
    weight_grad(D0, kPitchH, H2, kPitchH, 2 * w, 2, 0, 8, mine + oW3, kHid, first);
    bias_grad(D0, kPitchH, kHid, mine + oB3, first);
    back_layer<4>(D0, kPitchH, net.wb + pW3t, kHid, G2, D1);
    __syncthreads();
    // dW2 = D1^T H1, db2; dH1 = D1 W2 -> D0
    weight_grad(D1, kPitchH, H1, kPitchH, 2 * w, 2, 0, 8, mine + oW2, kHid, first);
    bias_grad(D1, kPitchH, kHid, mine + oB2, first);
    __syncthreads();
    back_layer<4>(D1, kPitchH, net.wb + pW2t, kHid, G1, D0);
    __syncthreads();
    // dW1 = D0^T X (n-tiles 2w, 2w+1; k-tiles 0, 1), db1
    weight_grad(D0, kPitchH, XS, kPitchX, 2 * w, 2, 0, 2, mine + oW1, kInPad, first);
    bias_grad(D0, kPitchH, kHid, mine + oB1, first);
    __syncthreads();
    first = false;
  }
  // loss partial: wave sums, then a fixed-order sum of the four waves
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off);
  if (l == 0) red[w] = sq;
  __syncthreads();
  if (tid == 0) loss_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void mlp_reduce_kernel(const float* __restrict__ part, int n_part, const float* __restrict__ loss_part,
                                  float inv, float* __restrict__ grad, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kParamFloats) {
    float s = 0.0f;
    for (int p = 0; p < n_part; ++p) s += part[(int64_t)p * kParamFloats + i];
    grad[i] = s;
  }
  if (i == 0 && loss) {
    double s = 0.0;
    for (int p = 0; p < n_part; ++p) s += loss_part[p];
    loss[0] = (float)(s * inv);
  }
}

__device__ inline bool is_weight(int i) {
  return (i >= oW1 && i < oB1) || (i >= oW2 && i < oB2) || (i >= oW3 && i < oB3) || (i >= oW4 && i < oB4);
}

__global__ void mlp_adamw_kernel(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m,
                                 float* __restrict__ v, float lr, float beta1, float beta2, float eps, float wd,
                                 float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParamFloats) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * g;
  const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  float p = prm[i];
  const float step = lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  if (is_weight(i)) p -= lr * wd * p;
  prm[i] = p - step;
}

__global__ void mlp_pack_kernel(const float* __restrict__ prm, uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPackedHalfs) return;
  float v;
  if (i < pW2) v = prm[oW1 + i];
  else if (i < pW3) v = prm[oW2 + (i - pW2)];
  else if (i < pW4) v = prm[oW3 + (i - pW3)];
  else if (i < pW2t) v = prm[oW4 + (i - pW4)];
  else if (i < pW3t) { const int j = i - pW2t, k = j / kHid, n = j % kHid; v = prm[oW2 + n * kHid + k]; }
  else if (i < pW4t) { const int j = i - pW3t, k = j / kHid, n = j % kHid; v = prm[oW3 + n * kHid + k]; }
  else { const int j = i - pW4t, k = j / 32, n = j % 32; v = n < kOutPad ? prm[oW4 + n * kHid + k] : 0.0f; }
  wb[i] = f2bf(v);
}

constexpr size_t kTrainLds = (size_t)(2 * kTile * kPitchX + 8 * kTile * kPitchH) * sizeof(uint16_t);
constexpr int kMaxTrainGroups = 512;

}  // namespace

int param_floats() { return kParamFloats; }
int packed_halfs() { return kPackedHalfs; }

int64_t train_groups(int64_t m_rows) {
  const int64_t tiles = (m_rows + kTile - 1) / kTile;
  return tiles < kMaxTrainGroups ? tiles : kMaxTrainGroups;
}

size_t train_workspace_bytes(int64_t m_rows) {
  const int64_t g = train_groups(m_rows);
  return (size_t)g * (kParamFloats + 1) * sizeof(float);
}

hipError_t launch_pack(const float* prm, uint16_t* wb, hipStream_t s) {
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((kPackedHalfs + 255) / 256), dim3(256), 0, s, prm, wb);
  return hipGetLastError();
}

hipError_t launch_forward(const uint16_t* wb, const float* prm, const float* norm, int64_t m_rows, const float* x,
                          float* y, hipStream_t s) {
  if (m_rows == 0) return hipSuccess;
  const int64_t tiles = (m_rows + kFwdTile - 1) / kFwdTile;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, s, Net{wb, prm, norm}, x, m_rows,
                     y);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const uint16_t* wb, const float* prm, const float* norm, int64_t m_rows, const float* x,
                            const float* tgt, float* grad, float* loss, void* ws, hipStream_t s) {
  const int64_t g = train_groups(m_rows);
  const float inv = (float)(1.0 / (4.0 * (double)m_rows));
  float* part = (float*)ws;
  float* loss_part = part + g * kParamFloats;
  hipError_t e = hipFuncSetAttribute((const void*)mlp_train_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kTrainLds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)g), dim3(kThreads), kTrainLds, s, Net{wb, prm, norm}, x, tgt,
                     m_rows, inv, part, loss_part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParamFloats + 255) / 256), dim3(256), 0, s, part, (int)g, loss_part,
                     inv, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adamw(float* prm, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                        float beta2, float eps, float wd, uint16_t* wb, hipStream_t s) {
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)step));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)step));
  hipLaunchKernelGGL(mlp_adamw_kernel, dim3((kParamFloats + 255) / 256), dim3(256), 0, s, prm, grad, m, v, lr, beta1,
                     beta2, eps, wd, (float)c1, (float)c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !wb) return e;
  return launch_pack(prm, wb, s);
}

}  // namespace mlp
}  // namespace icrs
