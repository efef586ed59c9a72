// gpe_learn.hip -- kernels of the learned coarse-grid correction
// (include/gpe_learn.h): restriction of fine states, network input, the
// three 3 x 3 convolutions forward and backward, loss, Adam, the
// mass-projected correction and the interface position.
//
// Convolutions: with bfloat16 operands the two layers with 32 output
// channels run as implicit GEMMs on the matrix cores (MFMA, FP32
// accumulation); the last layer (4 outputs), the FP32-operand variant and
// the backward passes are direct (per pixel, all output channels in
// registers, the layer's weights in LDS as FP32).  Every sum accumulates in
// FP32.  Weight gradients are an im2col product over
// chunks of 32 pixels staged in LDS; each work-group writes its partial sums
// and a second pass adds them in a fixed order, so a training step is
// bitwise reproducible.  Inference has a fused path (cnn_infer_kernel):
// network input, all three layers on the matrix cores and the tile sums of
// the phi output in one persistent kernel with the activations in LDS, then
// the correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "gpe.h"
#include "gpe_learn.h"

// Scratch of the allocation-free inference entry point: a file-scope device
// array, one copy on every GPU the library runs on, alive until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is a stand-in, not a device address): the address of each device's copy
// is looked up once per device with hipGetSymbolAddress (static_scratch).
static __device__ __align__(256) float scratch[GPE_CNN_INFER_STATIC_FLOATS];

namespace {

constexpr int C0 = 4, C1 = 32, C2 = 32, C3 = 4;
constexpr size_t NW1 = (size_t)C1 * 9 * C0, NW2 = (size_t)C2 * 9 * C1, NW3 = (size_t)C3 * 9 * C2;
constexpr size_t OFF_W1 = 0, OFF_B1 = OFF_W1 + NW1, OFF_W2 = OFF_B1 + C1, OFF_B2 = OFF_W2 + NW2;
constexpr size_t OFF_W3 = OFF_B2 + C2, OFF_B3 = OFF_W3 + NW3, NPARAM = OFF_B3 + C3;
constexpr int kBlock = 256;
constexpr int kPixPerBlockW = 2048;  // pixels per work-group of the weight-gradient pass
constexpr int kMaxPartials = (int)(C2 * 9 * C1 + C2);

// bfloat16 storage: the upper half of the FP32 bit pattern, rounded to
// nearest even (NaN kept NaN)
struct bf16 {
  uint16_t bits;
};
__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
__device__ __forceinline__ void store(float& d, float v) { d = v; }
__device__ __forceinline__ void store(bf16& d, float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    d.bits = (uint16_t)((u >> 16) | 0x40u);
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  d.bits = (uint16_t)(u >> 16);
}

__device__ __forceinline__ int wrap(int x, int W) { return x < 0 ? x + W : (x >= W ? x - W : x); }

unsigned blocks_for(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---- restriction ----------------------------------------------------------
__global__ __launch_bounds__(kBlock) void restrict_kernel(const float* const* fine, float* const* coarse, int B,
                                                          int ny, int nx, int f) {
  const int H = ny / f, W = nx / f;
  const long n = (long)B * H * W;
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int I = (int)(q % W);
  const long r = q / W;
  const int J = (int)(r % H);
  const int b = (int)(r / H);
  const float* fu = fine[4 * b + 0];
  const float* fv = fine[4 * b + 1];
  const float* fp = fine[4 * b + 2];
  const float* ff = fine[4 * b + 3];
  float sp = 0.f, sf = 0.f, su = 0.f, sv = 0.f;
  for (int a = 0; a < f; ++a) {
    const size_t row = (size_t)(f * J + a) * nx;
    for (int c = 0; c < f; ++c) {
      sp += fp[row + f * I + c];
      sf += ff[row + f * I + c];
    }
    su += fu[row + f * I];                         // x-face f*I on fine row f*J + a
    sv += fv[(size_t)(f * J) * nx + f * I + a];    // y-face f*J on fine column f*I + a
  }
  const size_t o = (size_t)J * W + I;
  coarse[4 * b + 0][o] = su / f;
  coarse[4 * b + 1][o] = sv / f;
  coarse[4 * b + 2][o] = sp / (f * f);
  coarse[4 * b + 3][o] = sf / (f * f);
}

// ---- network input ----------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(kBlock) void features_kernel(const float* const* fields, int B, int H, int W,
                                                          float s0, float s1, float s2, float s3, TA* x0) {
  const long n = (long)B * H * W;
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % W);
  const long r = q / W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  const float* u = fields[4 * b + 0];
  const float* v = fields[4 * b + 1];
  const float* p = fields[4 * b + 2];
  const float* ph = fields[4 * b + 3];
  const size_t o = (size_t)y * W + x;
  const float uc = 0.5f * (u[o] + u[(size_t)y * W + wrap(x + 1, W)]);
  const float vn = (y + 1 < H) ? v[o + W] : 0.f;  // the face above the top row is a wall face
  const float vc = 0.5f * (v[o] + vn);
  // scaled by the reciprocals of the scales (as the fused inference does)
  store(x0[q * 4 + 0], uc * (1.f / s0));
  store(x0[q * 4 + 1], vc * (1.f / s1));
  store(x0[q * 4 + 2], p[o] * (1.f / s2));
  store(x0[q * 4 + 3], ph[o] * (1.f / s3));
}

__global__ __launch_bounds__(kBlock) void target_kernel(const float* const* next, const float* const* pred, int B,
                                                        int H, int W, float s0, float s1, float s2, float s3,
                                                        float* target) {
  const long n = (long)B * H * W;
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int b = (int)(q / ((long)H * W));
  const size_t o = (size_t)(q - (long)b * H * W);
  const float sc[4] = {s0, s1, s2, s3};
#pragma unroll
  for (int c = 0; c < 4; ++c) target[q * 4 + c] = (next[4 * b + c][o] - pred[4 * b + c][o]) / sc[c];
}

template <typename TA>
__global__ __launch_bounds__(kBlock) void convert_kernel(const float* src, TA* dst, long n) {
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q < n) store(dst[q], src[q]);
}

// ---- convolutions -------------------------------------------------------------
// out[p][o] = bias[o] + sum over taps (dy, dx) and inputs i of
//   w[o][dy+1][dx+1][i] * x[(y+dy, (x+dx) mod W)][i]   (zero for y+dy outside)
template <int CI, int CO, typename TA, bool RELU, typename TO>
__global__ __launch_bounds__(kBlock) void conv_fwd_kernel(const TA* __restrict__ x, const TA* __restrict__ w,
                                                          const float* __restrict__ bias, TO* __restrict__ y,
                                                          int B, int H, int W) {
  __shared__ float sw[CO * 9 * CI];
  for (int q = threadIdx.x; q < CO * 9 * CI; q += kBlock) sw[q] = to_float(w[q]);
  __syncthreads();
  const long P = (long)B * H * W;
  const long p = (long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= P) return;
  const int xx = (int)(p % W);
  const long r = p / W;
  const int yy = (int)(r % H);
  const long b = r / H;
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = bias[o];
#pragma unroll 1
  for (int dy = -1; dy <= 1; ++dy) {
    const int y2 = yy + dy;
    if (y2 < 0 || y2 >= H) continue;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const TA* in = x + ((b * H + y2) * W + wrap(xx + dx, W)) * CI;
      float v[CI];
#pragma unroll
      for (int i = 0; i < CI; ++i) v[i] = to_float(in[i]);
      const float* wt = sw + ((dy + 1) * 3 + (dx + 1)) * CI;
#pragma unroll
      for (int o = 0; o < CO; ++o) {
#pragma unroll
        for (int i = 0; i < CI; ++i) acc[o] = fmaf(wt[o * 9 * CI + i], v[i], acc[o]);
      }
    }
  }
  TO* out = y + p * CO;
#pragma unroll
  for (int o = 0; o < CO; ++o) store(out[o], RELU ? fmaxf(acc[o], 0.f) : acc[o]);
}

// The same convolution on the matrix cores for bfloat16 operands and 32
// output channels: an implicit GEMM with M = pixels, N = 32 output channels
// and K = 9 CI (tap, input channel), one v_mfma_f32_32x32x8 bf16 per 8 values
// of K, FP32 accumulation.  A wave computes a tile of 32 consecutive pixels.
// Fragment layout of the instruction (lane l, element t of 4, output r of 16):
// A[l % 32][4 (l / 32) + t], B[4 (l / 32) + t][l % 32],
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  The weights sit in LDS as
// [K / 4][32][4], so the 32 lanes of a half-wave read 32 consecutive 8-byte
// chunks of B.  CI = 4 puts one tap in each half-wave's 4 values of K (ten
// taps with the last zero); CI a multiple of 8 keeps a K-step inside one tap.
typedef short mfma_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int mfma_u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));

template <int CI, bool RELU>
__global__ __launch_bounds__(kBlock) void conv_fwd_mfma_kernel(const bf16* __restrict__ x, const bf16* __restrict__ w,
                                                               const float* __restrict__ bias, bf16* __restrict__ y,
                                                               int B, int H, int W) {
  constexpr int CO = 32;
  constexpr int K = 9 * CI;
  static_assert(CI == 4 || CI % 8 == 0, "input channels: 4 or a multiple of 8");
  __shared__ uint2 sw[(K / 4) * CO];  // 4 bf16 per entry
  for (int q = threadIdx.x; q < (K / 4) * CO; q += kBlock) {
    const int kc = q / CO, o = q % CO;  // K chunk (tap, 4 input channels) and output channel
    const uint16_t* src = &w[(size_t)o * K + kc * 4].bits;
    uint2 v;
    v.x = (uint32_t)src[0] | ((uint32_t)src[1] << 16);
    v.y = (uint32_t)src[2] | ((uint32_t)src[3] << 16);
    sw[q] = v;
  }
  __syncthreads();
  const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
  const long P = (long)B * H * W;
  const long p0 = ((long)blockIdx.x * (kBlock / 64) + wave) * 32;
  if (p0 >= P) return;  // uniform per wave
  const int kg = lane / 32;           // which 4 of the 8 K values this lane holds
  const long pa = p0 + (lane % 32);   // the lane's A-row pixel
  const bool va = pa < P;
  const int xa = va ? (int)(pa % W) : 0;
  const long ra = pa / W;
  const int ya = va ? (int)(ra % H) : 0;
  const long ba = ra / H;
  // x at (y + dy, x + dx) of the lane's pixel, 4 channels from c0, or zeros
  auto load_a = [&](int tap, int c0) -> mfma_bf16x4 {
    mfma_bf16x4 a = {0, 0, 0, 0};
    const int y2 = ya + tap / 3 - 1;
    if (va && tap < 9 && y2 >= 0 && y2 < H) {
      const uint2 v = *reinterpret_cast<const uint2*>(x + ((ba * H + y2) * W + wrap(xa + tap % 3 - 1, W)) * CI + c0);
      a[0] = (short)(v.x & 0xffffu);
      a[1] = (short)(v.x >> 16);
      a[2] = (short)(v.y & 0xffffu);
      a[3] = (short)(v.y >> 16);
    }
    return a;
  };
  auto load_b = [&](int kc) -> mfma_bf16x4 {
    mfma_bf16x4 b = {0, 0, 0, 0};
    if (kc < K / 4) {
      const uint2 v = sw[kc * CO + (lane % 32)];
      b[0] = (short)(v.x & 0xffffu);
      b[1] = (short)(v.x >> 16);
      b[2] = (short)(v.y & 0xffffu);
      b[3] = (short)(v.y >> 16);
    }
    return b;
  };
  // the accumulators start at the bias of the lane's output channel (the
  // fused inference starts there too)
  const int o = lane % 32;
  const float bo = bias[o];
  mfma_f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = bo;
  if (CI == 4) {
#pragma unroll
    for (int s = 0; s < 5; ++s) {  // K values 8s .. 8s+7 = taps 2s and 2s+1
      const int tap = 2 * s + kg;
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(load_a(tap, 0), load_b(tap), acc, 0, 0, 0);
    }
  } else {
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
      for (int c = 0; c < CI; c += 8) {
        const int c0 = c + 4 * kg;
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(load_a(tap, c0), load_b((tap * CI + c0) / 4), acc, 0, 0,
                                                        0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long p = p0 + 8 * (r / 4) + 4 * kg + (r % 4);
    if (p < P) {
      const float v = acc[r];
      store(y[p * CO + o], RELU ? fmaxf(v, 0.f) : v);
    }
  }
}

// gin[q][i] = (sum over taps and outputs o of w[o][tap][i] gout[q - tap][o]) *
//             (ain[q][i] > 0): the gradient w.r.t. the pre-activation of the
// layer whose ReLU output ain is this layer's input
template <int CI, int CO, typename TA>
__global__ __launch_bounds__(kBlock) void conv_bwd_in_kernel(const float* __restrict__ gout,
                                                             const TA* __restrict__ w, const TA* __restrict__ ain,
                                                             float* __restrict__ gin, int B, int H, int W) {
  __shared__ float sw[CO * 9 * CI];
  for (int q = threadIdx.x; q < CO * 9 * CI; q += kBlock) sw[q] = to_float(w[q]);
  __syncthreads();
  const long P = (long)B * H * W;
  const long p = (long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= P) return;
  const int xx = (int)(p % W);
  const long r = p / W;
  const int yy = (int)(r % H);
  const long b = r / H;
  float acc[CI];
#pragma unroll
  for (int i = 0; i < CI; ++i) acc[i] = 0.f;
#pragma unroll 1
  for (int dy = -1; dy <= 1; ++dy) {
    const int yo = yy - dy;  // the output row that read this row through tap dy
    if (yo < 0 || yo >= H) continue;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const float* g = gout + ((b * H + yo) * W + wrap(xx - dx, W)) * CO;
      float gv[CO];
#pragma unroll
      for (int o = 0; o < CO; ++o) gv[o] = g[o];
      const float* wt = sw + ((dy + 1) * 3 + (dx + 1)) * CI;
#pragma unroll
      for (int o = 0; o < CO; ++o) {
#pragma unroll
        for (int i = 0; i < CI; ++i) acc[i] = fmaf(wt[o * 9 * CI + i], gv[o], acc[i]);
      }
    }
  }
  const TA* a = ain + p * CI;
  float* out = gin + p * CI;
#pragma unroll
  for (int i = 0; i < CI; ++i) out[i] = to_float(a[i]) > 0.f ? acc[i] : 0.f;
}

// partial[blk][o*9*CI + tap*CI + i] = sum over the block's pixels p of
//   gout[p][o] * x[p + tap][i];   partial[blk][CO*9*CI + o] = sum gout[p][o]
template <int CI, int CO, typename TA>
__global__ __launch_bounds__(kBlock) void conv_bwd_w_kernel(const float* __restrict__ gout,
                                                            const TA* __restrict__ ain, float* __restrict__ partial,
                                                            int B, int H, int W) {
  constexpr int K = 9 * CI;
  constexpr int E = CO * K;
  constexpr int NE = (E + kBlock - 1) / kBlock;
  constexpr int PC = 32;
  __shared__ float sg[PC][CO];
  __shared__ float sc[PC][K];
  float acc[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) acc[j] = 0.f;
  float bacc = 0.f;
  const long P = (long)B * H * W;
  const long p0 = (long)blockIdx.x * kPixPerBlockW;
  const long p1 = p0 + kPixPerBlockW < P ? p0 + kPixPerBlockW : P;
  for (long pc = p0; pc < p1; pc += PC) {
    __syncthreads();
    for (int q = threadIdx.x; q < PC * CO; q += kBlock) {
      const long p = pc + q / CO;
      sg[q / CO][q % CO] = p < p1 ? gout[p * CO + q % CO] : 0.f;
    }
    for (int q = threadIdx.x; q < PC * K; q += kBlock) {
      const int pp = q / K, k = q % K, tap = k / CI, i = k % CI;
      const long p = pc + pp;
      float v = 0.f;
      if (p < p1) {
        const int xx = (int)(p % W);
        const long r = p / W;
        const int yy = (int)(r % H);
        const long b = r / H;
        const int y2 = yy + tap / 3 - 1;
        if (y2 >= 0 && y2 < H) v = to_float(ain[((b * H + y2) * W + wrap(xx + tap % 3 - 1, W)) * CI + i]);
      }
      sc[pp][k] = v;
    }
    __syncthreads();
    for (int pp = 0; pp < PC; ++pp) {
#pragma unroll
      for (int j = 0; j < NE; ++j) {
        const int e = (int)threadIdx.x + j * kBlock;
        if (e < E) acc[j] = fmaf(sg[pp][e / K], sc[pp][e % K], acc[j]);
      }
      if ((int)threadIdx.x < CO) bacc += sg[pp][threadIdx.x];
    }
  }
  float* out = partial + (size_t)blockIdx.x * (E + CO);
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int e = (int)threadIdx.x + j * kBlock;
    if (e < E) out[e] = acc[j];
  }
  if ((int)threadIdx.x < CO) out[E + threadIdx.x] = bacc;
}

// The same weight and bias gradients on the matrix cores for bfloat16
// activations (BF16 path): an implicit GEMM with M = output channels o
// (padded to 32), N = 32 consecutive values of k = tap CI + i per tile and
// the reduction over pixels, one v_mfma_f32_32x32x2f32 per 2 pixels, FP32
// operands (the output gradient stays FP32; a BF16 activation converts to
// FP32 exactly) and FP32 accumulation.  Fragment layout (lane l): A[l % 32]
// [l / 32] = gout[p + l / 32][o = l % 32], B[l / 32][l % 32] = x(p + l / 32,
// k0 + l % 32), D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] as for the other
// 32 x 32 instructions.  A block of NW waves owns kPixPerBlockM pixels; wave
// w takes k-tiles w, w + NW, ...; wave 0 also sums the bias gradient.
constexpr int kPixPerBlockM = 512;

template <int CI, int CO>
struct BwdWTiles {
  static constexpr int K = 9 * CI, NKT = (K + 31) / 32;
  static constexpr int NW = NKT < 4 ? NKT : (NKT % 3 == 0 ? 3 : 4);  // waves per block
  static constexpr int TPW = (NKT + NW - 1) / NW;                     // k-tiles per wave
};

template <int CI, int CO>
__global__ __launch_bounds__((64 * BwdWTiles<CI, CO>::NW)) void conv_bwd_w_mfma_kernel(
    const float* __restrict__ gout, const bf16* __restrict__ ain, float* __restrict__ partial, int B, int H, int W) {
  using Tl = BwdWTiles<CI, CO>;
  constexpr int K = Tl::K, NKT = Tl::NKT, NW = Tl::NW, TPW = Tl::TPW, E = CO * K;
  static_assert(CO <= 32, "output channels");
  const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
  const int col = lane % 32, half = lane / 32;
  const long P = (long)B * H * W;
  const long p0 = (long)blockIdx.x * kPixPerBlockM;
  const long p1 = p0 + kPixPerBlockM < P ? p0 + kPixPerBlockM : P;
  // the lane's value of k in each of its tiles: tap and channel
  int tdy[TPW], tdx[TPW], tch[TPW];
  bool tok[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kt = wave + t * NW, k = kt * 32 + col;
    tok[t] = kt < NKT && k < K;
    const int tap = tok[t] ? k / CI : 4;
    tdy[t] = tap / 3 - 1;
    tdx[t] = tap % 3 - 1;
    tch[t] = tok[t] ? k % CI : 0;
  }
  mfma_f32x16 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  float bacc = 0.f;
  // pixel of this lane's half, (b, y, x), advanced by 2 per step
  long p = p0 + half;
  int xx = (int)(p % W);
  long rr = p / W;
  int yy = (int)(rr % H);
  long bb = rr / H;
  for (long pp = p0; pp < p1; pp += 2) {
    const bool vp = p < p1;
    const float a = (vp && col < CO) ? gout[p * CO + col] : 0.f;
    if (wave == 0) bacc += a;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      float b = 0.f;
      const int y2 = yy + tdy[t];
      if (vp && tok[t] && y2 >= 0 && y2 < H)
        b = to_float(ain[((bb * H + y2) * W + wrap(xx + tdx[t], W)) * CI + tch[t]]);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
    }
    p += 2;
    xx += 2;
    while (xx >= W) {
      xx -= W;
      if (++yy == H) {
        yy = 0;
        ++bb;
      }
    }
  }
  float* out = partial + (size_t)blockIdx.x * (E + CO);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kt = wave + t * NW, k = kt * 32 + col;
    if (kt >= NKT || k >= K) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = 8 * (r / 4) + 4 * half + (r % 4);
      if (o < CO) out[o * K + k] = acc[t][r];
    }
  }
  if (wave == 0) {
    const float other = __shfl_down(bacc, 32, 64);
    if (lane < CO) out[E + lane] = bacc + other;
  }
}

// grads_w[e] = sum over blocks of partial[blk][e] (blocks in order), and the
// bias entries likewise
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(const float* partial, int nblk, int E, int CO,
                                                                 float* gw, float* gb) {
  const int e = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (e >= E + CO) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += partial[(size_t)k * (E + CO) + e];
  if (e < E)
    gw[e] = s;
  else
    gb[e - E] = s;
}

// ---- loss ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void loss_kernel(const float* out, const float* t, float* gout, float* partial,
                                                      long n, float two_over_n) {
  __shared__ float red[kBlock];
  float s = 0.f;
  for (long q = (long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long)gridDim.x * kBlock) {
    const float d = out[q] - t[q];
    gout[q] = two_over_n * d;
    s = fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const float* partial, int nblk, float inv_n, float* loss) {
  if (threadIdx.x != 0) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += partial[k];
  loss[0] = s * inv_n;
}

// ---- Adam ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void adam_kernel(float* prm, float* m, float* v, const float* g, long n,
                                                      float lr, float b1, float b2, float eps, float c1, float c2) {
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  prm[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// ---- correction ---------------------------------------------------------------------
// sums[b] = sum over the cells of state b of out[.][3]
__global__ __launch_bounds__(kBlock) void phi_sum_kernel(const float* out, int HW, float* sums) {
  __shared__ float red[kBlock];
  const int b = (int)blockIdx.x;
  float s = 0.f;
  for (int q = (int)threadIdx.x; q < HW; q += kBlock) s += out[((size_t)b * HW + q) * 4 + 3];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[b] = red[0];
}

__global__ __launch_bounds__(kBlock) void apply_kernel(float* const* fields, const float* out, int B, int H, int W,
                                                       float s0, float s1, float s2, float s3, const float* sums) {
  const long n = (long)B * H * W;
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % W);
  const long r = q / W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  const size_t o = (size_t)y * W + x;
  const float* d = out + q * 4;
  const float mean = sums[b] / (float)(H * W);
  fields[4 * b + 0][o] += s0 * d[0];
  if (y > 0) fields[4 * b + 1][o] += s1 * d[1];  // the wall face of row 0 stays 0
  fields[4 * b + 2][o] += s2 * d[2];
  fields[4 * b + 3][o] += s3 * (d[3] - mean);
}

// apply_kernel with the case means taken from the per-tile sums of the phi
// output (tiles_per_case consecutive entries per case, in tile order) instead
// of per-case sums: a block's pixels lie in at most two cases (H W >= kBlock),
// whose tile sums (<= kBlock / 2 each) it loads into LDS together and adds in
// order in one lane per case, the same additions in the same order as
// case_sums_kernel, so the correction has the same bits and needs no launch
// of its own.
__global__ __launch_bounds__(kBlock) void apply_tiles_kernel(float* const* fields, const float* out, int B, int H,
                                                             int W, float s0, float s1, float s2, float s3,
                                                             const float* partial, int tiles_per_case) {
  __shared__ float part[kBlock];
  __shared__ float csum[2];
  const long n = (long)B * H * W, hw = (long)H * W;
  const long q0 = (long)blockIdx.x * kBlock;
  const int b0 = (int)(q0 / hw);
  const int nb = (int)(((q0 + kBlock < n ? q0 + kBlock : n) - 1) / hw) - b0 + 1;  // 1 or 2
  const int t = (int)threadIdx.x;
  if (t < nb * tiles_per_case) part[t] = partial[(size_t)b0 * tiles_per_case + t];
  __syncthreads();
  if (t < nb) {
    float sum = 0.f;
    for (int i = 0; i < tiles_per_case; ++i) sum += part[t * tiles_per_case + i];
    csum[t] = sum;
  }
  __syncthreads();
  const long q = q0 + t;
  if (q >= n) return;
  const int x = (int)(q % W);
  const long r = q / W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  const size_t o = (size_t)y * W + x;
  const float* d = out + q * 4;
  const float mean = csum[b - b0] / (float)(H * W);
  fields[4 * b + 0][o] += s0 * d[0];
  if (y > 0) fields[4 * b + 1][o] += s1 * d[1];  // the wall face of row 0 stays 0
  fields[4 * b + 2][o] += s2 * d[2];
  fields[4 * b + 3][o] += s3 * (d[3] - mean);
}

// ---- interface position -----------------------------------------------------------
__global__ __launch_bounds__(kBlock) void interface_kernel(const float* const* phi, int B, int H, int W,
                                                           float* out) {
  const long q = (long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (long)B * W) return;
  const int x = (int)(q % W);
  const int b = (int)(q / W);
  const float* c = phi[b];
  float top = NAN, bot = NAN;
  for (int j = H - 1; j > 0; --j) {
    const float a = c[(size_t)(j - 1) * W + x], e = c[(size_t)j * W + x];
    if ((a > 0.f) != (e > 0.f)) {
      top = (float)(j - 1) + 0.5f + a / (a - e);
      break;
    }
  }
  for (int j = 0; j < H - 1; ++j) {
    const float a = c[(size_t)j * W + x], e = c[(size_t)(j + 1) * W + x];
    if ((a > 0.f) != (e > 0.f)) {
      bot = (float)j + 0.5f + a / (a - e);
      break;
    }
  }
  out[q * 2 + 0] = top;
  out[q * 2 + 1] = bot;
}

// ---- fused inference ------------------------------------------------------------------
// Network input, the three convolutions and the per-tile sums of the phi
// output for one TW x TH tile of one state per iteration of a persistent
// work-group, with every activation in LDS: the input on the tile + 3 cells,
// layer 1 on the tile + 2, layer 2 on the tile + 1, the output on the tile.
// All three layers run on the matrix cores as products W x X (rows: output
// channels, columns: pixels) in the K order tap, then channel.  The weights
// are the A operand and stay in registers for the whole kernel (layers 1
// and 2) or in LDS (layer 3); the activations are the B operand, read from
// LDS.  Layers 1 and 2 use v_mfma_f32_32x32x16_bf16 (32 output channels x 32
// pixels); the 4-channel layer 3 uses v_mfma_f32_16x16x32_bf16 (16 rows, 4
// of them used, x 16 pixels).  A lane's result then holds consecutive output
// channels of one pixel, written to LDS as packed 8-byte words.
// Rows outside [0, H) are zero in every layer's input (zero padding in y);
// x is periodic.  A region pixel keeps its 32 channels at a 72-byte stride
// (36 bf16) so that the 32 lanes of a half-wave reading 8 bytes at
// consecutive pixels spread over the LDS banks.
constexpr int kTW = 32, kTH = 8;
constexpr int kR0W = kTW + 6, kR0H = kTH + 6, kR0N = kR0W * kR0H;
constexpr int kR1W = kTW + 4, kR1H = kTH + 4, kR1N = kR1W * kR1H;
constexpr int kR2W = kTW + 2, kR2H = kTH + 2, kR2N = kR2W * kR2H;
constexpr int kAS = 36;  // bf16 slots per pixel of a 32-channel region
constexpr int kN1 = (kR1N + 31) / 32, kN2 = (kR2N + 31) / 32;  // 32-pixel column blocks of layers 1 and 2

typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// two values rounded to nearest even and packed by one v_cvt_pk_bf16_f32 (lo
// in the low half); equal to two store(bf16&, float) except for the payload
// of a NaN
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
  const f32x2_t f = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}
// ReLU of two packed bf16 values in one packed 16-bit integer max against 0:
// a negative bf16 (-0 included) is a negative 16-bit integer.  Rounding
// first and then clamping gives the same bits as clamping first for every
// number (a NaN stays NaN).
typedef short s16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w) {
  const s16x2_t z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2_t, w), z));
}

__global__ __launch_bounds__(kBlock, 2) void cnn_infer_kernel(const float* const* __restrict__ fields,
                                                             const float* __restrict__ prm,
                                                             const bf16* __restrict__ wa, int B, int H, int W,
                                                             float s0, float s1, float s2, float s3,
                                                             float* __restrict__ out, float* __restrict__ partial) {
  __shared__ __align__(16) uint16_t a1[kR1N * kAS];
  __shared__ __align__(16) uint16_t a2x[kR2N * kAS];  // the input region (4 channels) until layer 1 is done, then layer 2
  __shared__ uint4 w3s[9 * 64];         // layer-3 A operand per K step and lane (rows 4-15 zero)
  __shared__ float4 bls[16];            // biases of layers 1 and 2, four channels per entry
  __shared__ float red[kBlock / 64];
  static_assert(kR0N * 4 <= kR2N * kAS, "input region fits the layer-2 buffer");

  const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
  const int kg = lane / 32, col = lane % 32;  // 32 x 32 x 16 fragments
  const int q16 = lane / 16, c16 = lane % 16;  // 16 x 16 x 32 fragments

  // 8 consecutive bf16 weights as one A fragment (4 words, element 0 low)
  auto w8 = [&](const bf16* src) -> uint4 {
    uint4 v;
    v.x = (uint32_t)src[0].bits | ((uint32_t)src[1].bits << 16);
    v.y = (uint32_t)src[2].bits | ((uint32_t)src[3].bits << 16);
    v.z = (uint32_t)src[4].bits | ((uint32_t)src[5].bits << 16);
    v.w = (uint32_t)src[6].bits | ((uint32_t)src[7].bits << 16);
    return v;
  };
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  // layer 1: K step s holds taps 4 s + 2 kg and 4 s + 2 kg + 1 (4 channels
  // each) of output channel col; taps 9-11 are zero
  uint4 w1r[3];
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const int ta = 4 * st + 2 * kg;
    if (ta + 1 < 9) {
      w1r[st] = w8(wa + OFF_W1 + (size_t)col * 36 + ta * 4);
    } else if (ta < 9) {
      const bf16* src = wa + OFF_W1 + (size_t)col * 36 + ta * 4;
      w1r[st] = make_uint4((uint32_t)src[0].bits | ((uint32_t)src[1].bits << 16),
                           (uint32_t)src[2].bits | ((uint32_t)src[3].bits << 16), 0u, 0u);
    } else {
      w1r[st] = z4;
    }
  }
  // layer 2: K step s holds tap s / 2, channels 16 (s % 2) + 8 kg .. + 7
  uint4 w2r[18];
#pragma unroll
  for (int st = 0; st < 18; ++st) w2r[st] = w8(wa + OFF_W2 + (size_t)col * 288 + 16 * st + 8 * kg);
  // layer 3 (16 x 16 x 32): K step s is tap s, channels 8 q16 .. + 7 of row c16
  for (int q = threadIdx.x; q < 9 * 64; q += kBlock) {
    const int st = q / 64, l = q % 64;
    w3s[q] = (l % 16) < 4 ? w8(wa + OFF_W3 + (size_t)(l % 16) * 288 + 32 * st + 8 * (l / 16)) : z4;
  }
  // biases: layers 1 and 2 in LDS (entry 8 l + c / 4 holds channels c .. c + 3
  // of layer l + 1), layer 3 in registers (rows 4 q16 + r, those of q16 = 0 used)
  if (threadIdx.x < 16) {
    const float* src = prm + (threadIdx.x < 8 ? OFF_B1 : OFF_B2) + 4 * (threadIdx.x % 8);
    bls[threadIdx.x] = make_float4(src[0], src[1], src[2], src[3]);
  }
  float b3r[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) b3r[r] = prm[OFF_B3 + r];

  const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
  const int ntiles = B * tiles_x * tiles_y;
  // input scales as reciprocals (as features_kernel)
  const float i0 = 1.f / s0, i1 = 1.f / s1, i2 = 1.f / s2, i3 = 1.f / s3;

  auto mfma32 = [&](uint4 a, uint2 b_lo, uint2 b_hi, mfma_f32x16 acc) {
    const mfma_u32x4 bv = {b_lo.x, b_lo.y, b_hi.x, b_hi.y};
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(mfma_bf16x8, a),
                                                    __builtin_bit_cast(mfma_bf16x8, bv), acc, 0, 0, 0);
  };
  auto mfma16 = [&](uint4 a, uint2 b_lo, uint2 b_hi, mfma_f32x4 acc) {
    const mfma_u32x4 bv = {b_lo.x, b_lo.y, b_hi.x, b_hi.y};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mfma_bf16x8, a),
                                                    __builtin_bit_cast(mfma_bf16x8, bv), acc, 0, 0, 0);
  };
  const uint2 z2 = make_uint2(0u, 0u);
  // accumulators of layer 1 or 2 start at the layer's bias: row 8 j + 4 kg
  // + i of the lane's 32 x 32 result is output channel 8 j + 4 kg + i
  auto bias_init = [&](mfma_f32x16& acc, int layer) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float4 bj = bls[8 * layer + 2 * j + kg];
      acc[4 * j + 0] = bj.x;
      acc[4 * j + 1] = bj.y;
      acc[4 * j + 2] = bj.z;
      acc[4 * j + 3] = bj.w;
    }
  };
  // the lane's result (16 rows = output channels 8 j + 4 kg + i of one
  // pixel, bias included) after ReLU, zero for pixels outside the image
  // rows, as four packed 8-byte words
  auto store_rows = [&](uint16_t* dst, const mfma_f32x16& acc, bool inside) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint2 v = z2;
      if (inside) {
        v.x = relu_bf16x2(bf16_pair(acc[4 * j + 0], acc[4 * j + 1]));
        v.y = relu_bf16x2(bf16_pair(acc[4 * j + 2], acc[4 * j + 3]));
      }
      *reinterpret_cast<uint2*>(dst + 8 * j + 4 * kg) = v;
    }
  };

  for (int t = (int)blockIdx.x; t < ntiles; t += (int)gridDim.x) {
    const int b = t / (tiles_x * tiles_y);
    const int tr = t % (tiles_x * tiles_y);
    const int y0 = (tr / tiles_x) * kTH, x0 = (tr % tiles_x) * kTW;
    const float* u = fields[4 * b + 0];
    const float* v = fields[4 * b + 1];
    const float* p = fields[4 * b + 2];
    const float* ph = fields[4 * b + 3];
    __syncthreads();  // layer-3 weights and biases staged / the previous tile's last layer done with a2x

    // network input on the tile + 3 (as features_kernel).  The loads of all
    // passes are issued first, unconditionally (rows outside the image read a
    // clamped row and are zeroed afterwards), at raised wave priority, so the
    // tile waits for one memory latency rather than one per pass.
    {
      constexpr int NPI = (kR0N + kBlock - 1) / kBlock;
      float ld[NPI][6];
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int it = 0; it < NPI; ++it) {
        const int q = min((int)threadIdx.x + it * kBlock, kR0N - 1);
        const int ry = q / kR0W, rx = q % kR0W;
        const int y = min(max(y0 - 3 + ry, 0), H - 1);
        // periodic x; x0 - 3 + rx lies in [-3, W + 33], one period when W >= 34
        const int xr = x0 - 3 + rx;
        const int x = W >= 34 ? wrap(xr, W) : (xr % W + W) % W;
        const size_t o = (size_t)y * W + x;
        ld[it][0] = u[o];
        ld[it][1] = u[(size_t)y * W + wrap(x + 1, W)];
        ld[it][2] = v[o];
        ld[it][3] = v[(size_t)min(y + 1, H - 1) * W + x];
        ld[it][4] = p[o];
        ld[it][5] = ph[o];
      }
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int it = 0; it < NPI; ++it) {
        const int q = (int)threadIdx.x + it * kBlock;
        if (q < kR0N) {
          const int y = y0 - 3 + q / kR0W;
          uint2 pk = z2;
          if (y >= 0 && y < H) {
            const float uc = 0.5f * (ld[it][0] + ld[it][1]);
            const float vn = (y + 1 < H) ? ld[it][3] : 0.f;
            const float vc = 0.5f * (ld[it][2] + vn);
            pk.x = bf16_pair(uc * i0, vc * i1);
            pk.y = bf16_pair(ld[it][4] * i2, ld[it][5] * i3);
          }
          *reinterpret_cast<uint2*>(&a2x[q * 4]) = pk;
        }
      }
    }
    __syncthreads();

    // layer 1 on the tile + 2: column blocks n = wave + 4 i, two at a time
    // with independent accumulators; the lane's pixel is column col
    {
      const int in_lo = max(0, 2 - y0) * kR1W, in_hi = min(kR1H, H - y0 + 2) * kR1W;
      for (int n0 = wave; n0 < kN1; n0 += 2 * (kBlock / 64)) {
        const int n1 = n0 + kBlock / 64;
        const int d0 = n0 * 32 + col, d1 = n1 * 32 + col;
        const bool v0 = d0 < kR1N, v1 = d1 < kR1N;
        const int ry0 = v0 ? d0 / kR1W : 0, rx0 = v0 ? d0 % kR1W : 0;
        const int ry1 = v1 ? d1 / kR1W : 0, rx1 = v1 ? d1 % kR1W : 0;
        mfma_f32x16 acc0, acc1;
        bias_init(acc0, 0);
        bias_init(acc1, 0);
#pragma unroll
        for (int st = 0; st < 3; ++st) {
          const int ta = 4 * st + 2 * kg, tb = ta + 1;
          auto xin = [&](int ry, int rx, int tap) -> uint2 {
            return tap < 9 ? *reinterpret_cast<const uint2*>(&a2x[((ry + tap / 3) * kR0W + rx + tap % 3) * 4]) : z2;
          };
          acc0 = mfma32(w1r[st], xin(ry0, rx0, ta), xin(ry0, rx0, tb), acc0);
          acc1 = mfma32(w1r[st], xin(ry1, rx1, ta), xin(ry1, rx1, tb), acc1);
        }
        if (v0) store_rows(&a1[d0 * kAS], acc0, d0 >= in_lo && d0 < in_hi);
        if (v1) store_rows(&a1[d1 * kAS], acc1, d1 >= in_lo && d1 < in_hi);
      }
    }
    __syncthreads();

    // layer 2 on the tile + 1: column blocks wave, wave + 4, wave + 8 with
    // three independent accumulators; K step s reads tap s / 2, channels
    // 16 (s % 2) + 8 kg .. + 7 of the source pixel (two 8-byte LDS reads)
    {
      const int in_lo = max(0, 1 - y0) * kR2W, in_hi = min(kR2H, H - y0 + 1) * kR2W;
      int dd[3];
      const uint16_t* sp[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        dd[i] = (wave + 4 * i) * 32 + col;
        const bool vi = dd[i] < kR2N;
        sp[i] = a1 + ((vi ? dd[i] / kR2W : 0) * kR1W + (vi ? dd[i] % kR2W : 0)) * kAS + 8 * kg;
      }
      mfma_f32x16 acc[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) bias_init(acc[i], 1);
#pragma unroll
      for (int st = 0; st < 18; ++st) {
        const int tap = st / 2, off = ((tap / 3) * kR1W + tap % 3) * kAS + 16 * (st % 2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          if (i == 2 && wave + 8 >= kN2) continue;  // wave-uniform: no third block
          const uint16_t* q = sp[i] + off;
          acc[i] = mfma32(w2r[st], *reinterpret_cast<const uint2*>(q), *reinterpret_cast<const uint2*>(q + 4), acc[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (dd[i] < kR2N) store_rows(&a2x[dd[i] * kAS], acc[i], dd[i] >= in_lo && dd[i] < in_hi);
    }
    __syncthreads();

    // layer 3 on the tile: 16-pixel blocks, tile rows 2 w and 2 w + 1 per
    // wave (two blocks each); K step s is tap s, channels 8 q16 .. + 7 of the
    // source pixel; lanes 0-15 hold the 4 output channels of their pixel
    float psum = 0.f;
    {
      static_assert(kTH == 2 * (kBlock / 64) && kTW == 32, "two tile rows of two 16-pixel blocks per wave");
      mfma_f32x4 acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = mfma_f32x4{0.f, 0.f, 0.f, 0.f};
      const uint16_t* sp[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ry = 2 * wave + i / 2, rx = 16 * (i % 2) + c16;
        sp[i] = a2x + (ry * kR2W + rx) * kAS + 8 * q16;
      }
#pragma unroll
      for (int st = 0; st < 9; ++st) {
        const uint4 a = w3s[st * 64 + lane];
        const int off = ((st / 3) * kR2W + st % 3) * kAS;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint16_t* q = sp[i] + off;
          acc[i] = mfma16(a, *reinterpret_cast<const uint2*>(q), *reinterpret_cast<const uint2*>(q + 4), acc[i]);
        }
      }
      if (q16 == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int y = y0 + 2 * wave + i / 2, xc = x0 + 16 * (i % 2) + c16;
          if (y < H && xc < W) {
            const float4 val = make_float4(acc[i][0] + b3r[0], acc[i][1] + b3r[1], acc[i][2] + b3r[2], acc[i][3] + b3r[3]);
            *reinterpret_cast<float4*>(&out[(((size_t)b * H + y) * W + xc) * 4]) = val;
            psum += val.w;
          }
        }
      }
    }
    // tile sum of the phi output: lanes 0-15 of each wave, then the waves
#pragma unroll
    for (int o = 8; o >= 1; o /= 2) psum += __shfl_xor(psum, o, 64);
    if (lane == 0) red[wave] = psum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float sum = 0.f;
      for (int w = 0; w < kBlock / 64; ++w) sum += red[w];
      partial[t] = sum;
    }
  }
}

// per-case sums of the phi output from the per-tile sums, in tile order: the
// block of case b loads kBlock of its partials into LDS at a time (one memory
// latency per chunk instead of one per tile), then one lane adds them in order
__global__ __launch_bounds__(kBlock) void case_sums_kernel(const float* partial, int tiles_per_case, float* sums) {
  __shared__ float part[kBlock];
  const int b = (int)blockIdx.x;
  const float* src = partial + (size_t)b * tiles_per_case;
  float s = 0.f;
  for (int t0 = 0; t0 < tiles_per_case; t0 += kBlock) {
    const int n = tiles_per_case - t0 < kBlock ? tiles_per_case - t0 : kBlock;
    if ((int)threadIdx.x < n) part[threadIdx.x] = src[t0 + (int)threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int t = 0; t < n; ++t) s += part[t];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[b] = s;
}

// ---- launch helpers ----------------------------------------------------------------
bool dims_ok(int B, int H, int W) { return B >= 1 && H >= 1 && W >= 1 && (long)B * H * W < (1L << 31); }

template <typename TA>
hipError_t forward_t(const float* prm, const TA* wa, const TA* x0, TA* a1, TA* a2, float* out, int B, int H, int W,
                     hipStream_t s) {
  const long P = (long)B * H * W;
  const unsigned g = blocks_for(P);
  if constexpr (std::is_same<TA, bf16>::value) {
    // layers with 32 output channels on the matrix cores
    const unsigned gm = (unsigned)((P + 4 * 32 - 1) / (4 * 32));
    hipLaunchKernelGGL((conv_fwd_mfma_kernel<C0, true>), dim3(gm), dim3(kBlock), 0, s, x0, wa + OFF_W1,
                       prm + OFF_B1, a1, B, H, W);
    hipLaunchKernelGGL((conv_fwd_mfma_kernel<C1, true>), dim3(gm), dim3(kBlock), 0, s, a1, wa + OFF_W2,
                       prm + OFF_B2, a2, B, H, W);
  } else {
    hipLaunchKernelGGL((conv_fwd_kernel<C0, C1, TA, true, TA>), dim3(g), dim3(kBlock), 0, s, x0, wa + OFF_W1,
                       prm + OFF_B1, a1, B, H, W);
    hipLaunchKernelGGL((conv_fwd_kernel<C1, C2, TA, true, TA>), dim3(g), dim3(kBlock), 0, s, a1, wa + OFF_W2,
                       prm + OFF_B2, a2, B, H, W);
  }
  hipLaunchKernelGGL((conv_fwd_kernel<C2, C3, TA, false, float>), dim3(g), dim3(kBlock), 0, s, a2, wa + OFF_W3,
                     prm + OFF_B3, out, B, H, W);
  return hipGetLastError();
}

// First pass of a two-level reduction of many blocks' partials: mid[c][e] =
// the sum of partial[k][e] over the kRedChunk consecutive blocks k of chunk c,
// in block order (the second pass sums the chunks in order: deterministic).
constexpr int kRedChunk = 32;
__global__ __launch_bounds__(kBlock) void reduce_chunks_kernel(const float* partial, int nblk, int EE, float* mid) {
  const int e = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (e >= EE) return;
  const int k0 = (int)blockIdx.y * kRedChunk;
  const int k1 = k0 + kRedChunk < nblk ? k0 + kRedChunk : nblk;
  float s = 0.f;
  for (int k = k0; k < k1; ++k) s += partial[(size_t)k * EE + e];
  mid[(size_t)blockIdx.y * EE + e] = s;
}

size_t gin_floats(int B, int H, int W) { return (size_t)B * H * W * C2; }
int wblocks(int B, int H, int W) { return (int)(((long)B * H * W + kPixPerBlockW - 1) / kPixPerBlockW); }
int wblocks_mfma(int B, int H, int W) { return (int)(((long)B * H * W + kPixPerBlockM - 1) / kPixPerBlockM); }

template <int CI, int CO, typename TA>
hipError_t weight_grads(const float* g, const TA* ain, float* partial, float* gw, float* gb, int B, int H, int W,
                        hipStream_t s) {
  int nb;
  if constexpr (std::is_same<TA, bf16>::value) {  // BF16 activations: on the matrix cores
    nb = wblocks_mfma(B, H, W);
    hipLaunchKernelGGL((conv_bwd_w_mfma_kernel<CI, CO>), dim3(nb), dim3(64 * BwdWTiles<CI, CO>::NW), 0, s, g, ain,
                       partial, B, H, W);
  } else {
    nb = wblocks(B, H, W);
    hipLaunchKernelGGL((conv_bwd_w_kernel<CI, CO, TA>), dim3(nb), dim3(kBlock), 0, s, g, ain, partial, B, H, W);
  }
  const int E = CO * 9 * CI;
  if (nb > 2 * kRedChunk) {  // two passes: chunks of kRedChunk blocks, then the chunks
    const int nc = (nb + kRedChunk - 1) / kRedChunk;
    float* mid = partial + (size_t)nb * (E + CO);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3(blocks_for(E + CO), nc), dim3(kBlock), 0, s, partial, nb, E + CO,
                       mid);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks_for(E + CO)), dim3(kBlock), 0, s, mid, nc, E, CO, gw, gb);
  } else {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks_for(E + CO)), dim3(kBlock), 0, s, partial, nb, E, CO, gw,
                       gb);
  }
  return hipGetLastError();
}

template <typename TA>
hipError_t backward_t(const TA* wa, const TA* x0, const TA* a1, const TA* a2, const float* gout, float* grads,
                      int B, int H, int W, float* scratch, hipStream_t s) {
  const size_t ng = gin_floats(B, H, W);
  float* g2 = scratch;
  float* g1 = scratch + ng;
  float* partial = scratch + 2 * ng;
  const unsigned g = blocks_for((long)B * H * W);
  hipError_t e = weight_grads<C2, C3, TA>(gout, a2, partial, grads + OFF_W3, grads + OFF_B3, B, H, W, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((conv_bwd_in_kernel<C2, C3, TA>), dim3(g), dim3(kBlock), 0, s, gout, wa + OFF_W3, a2, g2, B, H,
                     W);
  e = weight_grads<C1, C2, TA>(g2, a1, partial, grads + OFF_W2, grads + OFF_B2, B, H, W, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((conv_bwd_in_kernel<C1, C2, TA>), dim3(g), dim3(kBlock), 0, s, g2, wa + OFF_W2, a1, g1, B, H,
                     W);
  return weight_grads<C0, C1, TA>(g1, x0, partial, grads + OFF_W1, grads + OFF_B1, B, H, W, s);
}

// Fused inference of B states with the per-tile partial sums (and then the
// per-case sums) in `partial`, which holds infer_scratch_floats(B, H, W)
// floats; every entry is written before it is read, so it needs no clearing.
size_t infer_scratch_floats(int B, int H, int W) {
  return (size_t)B * ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH) + B;
}

int infer_launch(float* const* d_fields, const float* d_params, const void* d_params_bf16, int B, int H, int W,
                 const float in_scale[4], const float out_scale[4], float* d_out, float* partial, hipStream_t s) {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
  }
  const int tpc = ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
  const long ntiles = (long)B * tpc;
  const unsigned grid = (unsigned)std::min<long>(ntiles, 2L * ncu);
  hipLaunchKernelGGL(cnn_infer_kernel, dim3(grid), dim3(kBlock), 0, s, d_fields, d_params,
                     (const bf16*)d_params_bf16, B, H, W, in_scale[0], in_scale[1], in_scale[2], in_scale[3], d_out,
                     partial);
  if ((long)H * W >= kBlock && tpc <= kBlock / 2) {
    hipLaunchKernelGGL(apply_tiles_kernel, dim3(blocks_for((long)B * H * W)), dim3(kBlock), 0, s, d_fields, d_out, B,
                       H, W, out_scale[0], out_scale[1], out_scale[2], out_scale[3], (const float*)partial, tpc);
  } else {
    float* sums = partial + ntiles;
    hipLaunchKernelGGL(case_sums_kernel, dim3((unsigned)B), dim3(kBlock), 0, s, (const float*)partial, tpc, sums);
    hipLaunchKernelGGL(apply_kernel, dim3(blocks_for((long)B * H * W)), dim3(kBlock), 0, s, d_fields, d_out, B, H, W,
                       out_scale[0], out_scale[1], out_scale[2], out_scale[3], (const float*)sums);
  }
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

bool infer_args_ok(float* const* d_fields, const float* d_params, const void* d_params_bf16, int B, int H, int W,
                   const float in_scale[4], const float out_scale[4], const float* d_out) {
  if (!d_fields || !d_params || !d_params_bf16 || !in_scale || !out_scale || !d_out || !dims_ok(B, H, W))
    return false;
  for (int c = 0; c < 4; ++c)
    if (!(in_scale[c] > 0.f)) return false;
  return true;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, or nullptr.
float* static_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = (float*)ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t gpe_cnn_param_count(void) { return NPARAM; }

size_t gpe_cnn_act_bytes(int32_t act_type) {
  return act_type == GPE_ACT_BF16 ? 2 : (act_type == GPE_ACT_FP32 ? 4 : 0);
}

size_t gpe_cnn_scratch_bytes(int32_t B, int32_t H, int32_t W) {
  if (!dims_ok(B, H, W)) return 0;
  // per-block partials, then the chunk sums of the two-level reduction
  const size_t nb = (size_t)std::max(wblocks(B, H, W), wblocks_mfma(B, H, W));
  const size_t parts = (nb + (nb + kRedChunk - 1) / kRedChunk) * kMaxPartials;
  const size_t loss_parts = 1024;
  return (2 * gin_floats(B, H, W) + parts + loss_parts) * sizeof(float);
}

int gpe_restrict2d(const float* const* d_fine, float* const* d_coarse, int32_t B, int32_t ny, int32_t nx, int32_t f,
                   void* stream) {
  if (!d_fine || !d_coarse || f < 1 || ny % f || nx % f || !dims_ok(B, ny, nx)) return GPE_EINVAL;
  const long n = (long)B * (ny / f) * (nx / f);
  hipLaunchKernelGGL(restrict_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, (hipStream_t)stream, d_fine, d_coarse,
                     B, ny, nx, f);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_target(const float* const* d_next, const float* const* d_pred, int32_t B, int32_t H, int32_t W,
                   const float out_scale[4], float* d_target, void* stream) {
  if (!d_next || !d_pred || !out_scale || !d_target || !dims_ok(B, H, W)) return GPE_EINVAL;
  for (int c = 0; c < 4; ++c)
    if (!(out_scale[c] > 0.f)) return GPE_EINVAL;
  hipLaunchKernelGGL(target_kernel, dim3(blocks_for((long)B * H * W)), dim3(kBlock), 0, (hipStream_t)stream, d_next,
                     d_pred, B, H, W, out_scale[0], out_scale[1], out_scale[2], out_scale[3], d_target);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_features(const float* const* d_fields, int32_t B, int32_t H, int32_t W, const float in_scale[4],
                     int32_t act_type, void* d_x0, void* stream) {
  if (!d_fields || !in_scale || !d_x0 || !dims_ok(B, H, W)) return GPE_EINVAL;
  for (int c = 0; c < 4; ++c)
    if (!(in_scale[c] > 0.f)) return GPE_EINVAL;
  const unsigned g = blocks_for((long)B * H * W);
  hipStream_t s = (hipStream_t)stream;
  if (act_type == GPE_ACT_BF16)
    hipLaunchKernelGGL(features_kernel<bf16>, dim3(g), dim3(kBlock), 0, s, d_fields, B, H, W, in_scale[0],
                       in_scale[1], in_scale[2], in_scale[3], (bf16*)d_x0);
  else if (act_type == GPE_ACT_FP32)
    hipLaunchKernelGGL(features_kernel<float>, dim3(g), dim3(kBlock), 0, s, d_fields, B, H, W, in_scale[0],
                       in_scale[1], in_scale[2], in_scale[3], (float*)d_x0);
  else
    return GPE_EINVAL;
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_convert(const float* d_params, void* d_params_act, int32_t act_type, void* stream) {
  if (!d_params || !d_params_act) return GPE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = blocks_for((long)NPARAM);
  if (act_type == GPE_ACT_BF16)
    hipLaunchKernelGGL(convert_kernel<bf16>, dim3(g), dim3(kBlock), 0, s, d_params, (bf16*)d_params_act,
                       (long)NPARAM);
  else if (act_type == GPE_ACT_FP32)
    hipLaunchKernelGGL(convert_kernel<float>, dim3(g), dim3(kBlock), 0, s, d_params, (float*)d_params_act,
                       (long)NPARAM);
  else
    return GPE_EINVAL;
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_forward(const float* d_params, const void* d_params_act, const void* d_x0, void* d_a1, void* d_a2,
                    float* d_out, int32_t B, int32_t H, int32_t W, int32_t act_type, void* stream) {
  if (!d_params || !d_params_act || !d_x0 || !d_a1 || !d_a2 || !d_out || !dims_ok(B, H, W)) return GPE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (act_type == GPE_ACT_BF16)
    e = forward_t<bf16>(d_params, (const bf16*)d_params_act, (const bf16*)d_x0, (bf16*)d_a1, (bf16*)d_a2, d_out, B,
                        H, W, s);
  else if (act_type == GPE_ACT_FP32)
    e = forward_t<float>(d_params, (const float*)d_params_act, (const float*)d_x0, (float*)d_a1, (float*)d_a2,
                         d_out, B, H, W, s);
  else
    return GPE_EINVAL;
  return e == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_loss(const float* d_out, const float* d_target, float* d_gout, float* d_loss, int64_t n,
                 void* d_scratch, size_t scratch_bytes, void* stream) {
  if (!d_out || !d_target || !d_gout || !d_loss || !d_scratch || n < 1 || scratch_bytes < 1024 * sizeof(float))
    return GPE_EINVAL;
  const int nblk = 1024;
  hipStream_t s = (hipStream_t)stream;
  float* partial = (float*)d_scratch;
  hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(kBlock), 0, s, d_out, d_target, d_gout, partial, (long)n,
                     (float)(2.0 / (double)n));
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, partial, nblk, (float)(1.0 / (double)n), d_loss);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_backward(const float* d_params, const void* d_params_act, const void* d_x0, const void* d_a1,
                     const void* d_a2, const float* d_gout, float* d_grads, int32_t B, int32_t H, int32_t W,
                     int32_t act_type, void* d_scratch, size_t scratch_bytes, void* stream) {
  (void)d_params;
  if (!d_params_act || !d_x0 || !d_a1 || !d_a2 || !d_gout || !d_grads || !d_scratch || !dims_ok(B, H, W))
    return GPE_EINVAL;
  if (scratch_bytes < gpe_cnn_scratch_bytes(B, H, W)) return GPE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (act_type == GPE_ACT_BF16)
    e = backward_t<bf16>((const bf16*)d_params_act, (const bf16*)d_x0, (const bf16*)d_a1, (const bf16*)d_a2, d_gout,
                         d_grads, B, H, W, (float*)d_scratch, s);
  else if (act_type == GPE_ACT_FP32)
    e = backward_t<float>((const float*)d_params_act, (const float*)d_x0, (const float*)d_a1, (const float*)d_a2,
                          d_gout, d_grads, B, H, W, (float*)d_scratch, s);
  else
    return GPE_EINVAL;
  return e == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_adam(float* d_params, float* d_m, float* d_v, const float* d_grads, int64_t n, float lr, float beta1,
                 float beta2, float eps, int64_t t, void* stream) {
  if (!d_params || !d_m || !d_v || !d_grads || n < 1 || t < 1) return GPE_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, (hipStream_t)stream, d_params, d_m, d_v,
                     d_grads, (long)n, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

int gpe_cnn_apply(float* const* d_fields, const float* d_out, int32_t B, int32_t H, int32_t W,
                  const float out_scale[4], float* d_scratch, void* stream) {
  if (!d_fields || !d_out || !out_scale || !d_scratch || !dims_ok(B, H, W)) return GPE_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(phi_sum_kernel, dim3(B), dim3(kBlock), 0, s, d_out, H * W, d_scratch);
  hipLaunchKernelGGL(apply_kernel, dim3(blocks_for((long)B * H * W)), dim3(kBlock), 0, s, d_fields, d_out, B, H, W,
                     out_scale[0], out_scale[1], out_scale[2], out_scale[3], (const float*)d_scratch);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

size_t gpe_cnn_infer_scratch_bytes(int32_t B, int32_t H, int32_t W) {
  if (!dims_ok(B, H, W)) return 0;
  return infer_scratch_floats(B, H, W) * sizeof(float);
}

int gpe_cnn_infer(float* const* d_fields, const float* d_params, const void* d_params_bf16, int32_t B, int32_t H,
                  int32_t W, const float in_scale[4], const float out_scale[4], float* d_out, void* d_scratch,
                  size_t scratch_bytes, void* stream) {
  if (!d_scratch || !infer_args_ok(d_fields, d_params, d_params_bf16, B, H, W, in_scale, out_scale, d_out))
    return GPE_EINVAL;
  if (scratch_bytes < gpe_cnn_infer_scratch_bytes(B, H, W)) return GPE_EINVAL;
  return infer_launch(d_fields, d_params, d_params_bf16, B, H, W, in_scale, out_scale, d_out, (float*)d_scratch,
                      (hipStream_t)stream);
}

int gpe_cnn_infer_noalloc(float* const* d_fields, const float* d_params, const void* d_params_bf16, int32_t B,
                          int32_t H, int32_t W, const float in_scale[4], const float out_scale[4], float* d_out,
                          void* stream) {
  if (!infer_args_ok(d_fields, d_params, d_params_bf16, B, H, W, in_scale, out_scale, d_out)) return GPE_EINVAL;
  if (infer_scratch_floats(B, H, W) > (size_t)GPE_CNN_INFER_STATIC_FLOATS) return GPE_EWORKSPACE;
  float* ptr = static_scratch();
  if (!ptr) return GPE_EHIP;
  return infer_launch(d_fields, d_params, d_params_bf16, B, H, W, in_scale, out_scale, d_out, ptr,
                      (hipStream_t)stream);
}

int gpe_interface_position(const float* const* d_phi, int32_t B, int32_t H, int32_t W, float* d_out,
                           void* stream) {
  if (!d_phi || !d_out || !dims_ok(B, H, W)) return GPE_EINVAL;
  hipLaunchKernelGGL(interface_kernel, dim3(blocks_for((long)B * W)), dim3(kBlock), 0, (hipStream_t)stream, d_phi, B,
                     H, W, d_out);
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}

}  // extern "C"
