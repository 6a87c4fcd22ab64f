// Learned layer manager: a small CNN that predicts, from a 48 x 48 window
// centred on a lost block, the PSNR gain of IDL over BRL (g1) and of HQL over
// IDL (g2).  It replaces the profile rule of the paper's layer switching
// (Sec. "Layer switching and profile selection"), choosing the layer before
// any candidate is examined: BRL if g1 <= tau1, else HQL if g2 > tau2, else
// IDL.
//
// Network: input (2, 48, 48) = ((u - 128)/128 at known pixels, 1 at unknown
// pixels), rearranged without loss into (8, 24, 24) (channel 4 c + 2 dy + dx
// at (Y, X) is channel c at pixel (2 Y + dy, 2 X + dx)); three 3x3
// convolutions, stride 2, zero padding 1, 32 channels, ReLU (24 -> 12 -> 6 ->
// 3); global average pool; linear 32 -> 2.  Weights and the inputs of every
// convolution are bfloat16 values, accumulation is FP32.  Parameters live in
// one flat FP32 array (w1, b1, w2, b2, w3, b3, wh, bh); `wq` is the same array
// with the convolution weights rounded to bfloat16.
//
// Training kernels are batched over N samples in NCHW FP32 buffers; every
// reduction runs in a fixed order, so a training step is deterministic.
#include "skm_device.h"

namespace skm {

constexpr int kP = 48;          // input window
constexpr int kS = 24;          // its space-to-depth side
constexpr int kC0 = 8;          // space-to-depth channels
constexpr int kC = 32;          // channels
constexpr int kPool = 9;        // positions of the last layer (3 x 3)
constexpr int kOffW1 = 0, kOffB1 = 2304, kOffW2 = 2336, kOffB2 = 11552, kOffW3 = 11584,
              kOffB3 = 20800, kOffWh = 20832, kOffBh = 20896, kNParams = 20898;
static_assert(kNParams == kCnnParams, "parameter count");

static __device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}
static __device__ __forceinline__ float bf16_to_f(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
static __device__ __forceinline__ bool is_conv_weight(int k) {
  return (k >= kOffW1 && k < kOffB1) || (k >= kOffW2 && k < kOffB2) || (k >= kOffW3 && k < kOffB3);
}

// Input channels of one block from the value plane (known = value >= 0).
static __device__ __forceinline__ void input_pixel(const FrameArgs& a, const DevParams& p, int by,
                                                   int bx, int idx, float& c0, float& c1) {
  const int py = idx / kP, px = idx - py * kP;
  const int gy = by * p.B + p.B / 2 - kP / 2 + py, gx = bx * p.B + p.B / 2 - kP / 2 + px;
  int v = -1;
  if (gy >= 0 && gy < p.height && gx >= 0 && gx < p.width) v = a.val[(size_t)gy * p.width + gx];
  c0 = v >= 0 ? (float)(v - 128) * (1.0f / 128.0f) : 0.0f;
  c1 = v >= 0 ? 0.0f : 1.0f;
}

// inputs of every lost block (received frame), bf16 [n][8][24][24]
__global__ __launch_bounds__(kThreads) void k_cnn_inputs(FrameArgs a, DevParams p, uint16_t* out) {
  const int n_lost = a.st->n_lost;
  for (int i = blockIdx.x; i < n_lost; i += gridDim.x) {
    const int cell = a.blk[i];
    const int by = cell / p.gw, bx = cell - by * p.gw;
    for (int e = threadIdx.x; e < kC0 * kS * kS; e += kThreads) {
      const int ch = e / (kS * kS), q = e - ch * (kS * kS);
      const int Y = q / kS, X = q - Y * kS;
      const int dy = (ch >> 1) & 1, dx = ch & 1;
      float c0, c1;
      input_pixel(a, p, by, bx, (2 * Y + dy) * kP + 2 * X + dx, c0, c1);
      out[(size_t)i * kC0 * kS * kS + e] = (uint16_t)(__float_as_uint(ch < 4 ? c0 : c1) >> 16);
    }
  }
}

// ------------------------------------------------------------- training

// z = conv(in) + b, act = relu(z) (rounded to bf16 when round_act); one
// thread per output element.  The layer-1 input is bf16 (in16).
__global__ __launch_bounds__(kThreads) void k_conv_fwd(int N, int Cin, int H, const float* in,
                                                       const uint16_t* in16, const float* w,
                                                       const float* b, float* z, float* act,
                                                       int round_act) {
  const int Ho = H / 2;
  const long long total = (long long)N * kC * Ho * Ho;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kThreads) {
    const int ox = (int)(e % Ho), oy = (int)((e / Ho) % Ho);
    const int k = (int)((e / ((long long)Ho * Ho)) % kC);
    const long long n = e / ((long long)kC * Ho * Ho);
    float s = b[k];
    for (int c = 0; c < Cin; ++c) {
      const size_t ib = ((size_t)n * Cin + c) * H * H;
      const float* wk = w + ((size_t)k * Cin + c) * 9;
      for (int ky = 0; ky < 3; ++ky) {
        const int y = 2 * oy + ky - 1;
        if (y < 0 || y >= H) continue;
        for (int kx = 0; kx < 3; ++kx) {
          const int x = 2 * ox + kx - 1;
          if (x < 0 || x >= H) continue;
          const float v = in16 ? bf16_to_f(in16[ib + (size_t)y * H + x]) : in[ib + (size_t)y * H + x];
          s = fmaf(v, wk[ky * 3 + kx], s);
        }
      }
    }
    z[e] = s;
    const float r = fmaxf(s, 0.0f);
    act[e] = round_act ? bf16_round(r) : r;
  }
}

// global average pool and linear head, one thread per sample
__global__ __launch_bounds__(kThreads) void k_head_fwd(int N, const float* a3, const float* wq,
                                                       float* g, float* y) {
  const int n = blockIdx.x * kThreads + threadIdx.x;
  if (n >= N) return;
  float gv[kC];
  for (int c = 0; c < kC; ++c) {
    float s = 0.0f;
    for (int q = 0; q < kPool; ++q) s += a3[((size_t)n * kC + c) * kPool + q];
    gv[c] = s * (1.0f / kPool);
    g[(size_t)n * kC + c] = gv[c];
  }
  for (int o = 0; o < 2; ++o) {
    float s = wq[kOffBh + o];
    for (int c = 0; c < kC; ++c) s = fmaf(gv[c], wq[kOffWh + o * kC + c], s);
    y[(size_t)n * 2 + o] = s;
  }
}

// MSE over N x 2 outputs; gy = d loss / d y; loss to out[0] (single workgroup)
__global__ __launch_bounds__(kThreads) void k_loss(int N, const float* y, const float* t, float* gy,
                                                   float* out) {
  __shared__ double red[kThreads / 64];
  double s = 0.0;
  const float scale = 2.0f / (2.0f * (float)N);
  for (int e = threadIdx.x; e < 2 * N; e += kThreads) {
    const float d = y[e] - t[e];
    gy[e] = scale * d;
    s += (double)d * d;
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (float)((((red[0] + red[1]) + red[2]) + red[3]) / (2.0 * N));
}

// deterministic workgroup reduction of one float per thread (float64 partials)
static __device__ __forceinline__ float block_sum_f(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  const double t = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return (float)t;
}

// head gradients: workgroup per (o, c) weight, then per bias
__global__ __launch_bounds__(kThreads) void k_head_wgrad(int N, const float* gy, const float* g,
                                                         float* grad) {
  __shared__ double red[kThreads / 64];
  const int e = blockIdx.x;                // 0..63 weights, 64..65 biases
  const int o = e < 64 ? e / kC : e - 64, c = e < 64 ? e % kC : -1;
  double s = 0.0;
  for (int n = threadIdx.x; n < N; n += kThreads)
    s += (double)gy[(size_t)n * 2 + o] * (c >= 0 ? (double)g[(size_t)n * kC + c] : 1.0);
  const float v = block_sum_f(s, red);
  if (threadIdx.x == 0) grad[e < 64 ? kOffWh + e : kOffBh + o] = v;
}

// d loss / d z3 through the head, the pool and the last ReLU
__global__ __launch_bounds__(kThreads) void k_head_back(int N, const float* gy, const float* wq,
                                                        const float* z3, float* gz3) {
  const long long total = (long long)N * kC * kPool;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kThreads) {
    const long long n = e / (kC * kPool);
    const int c = (int)((e / kPool) % kC);
    const float gg = gy[n * 2] * wq[kOffWh + c] + gy[n * 2 + 1] * wq[kOffWh + kC + c];
    gz3[e] = z3[e] > 0.0f ? gg * (1.0f / kPool) : 0.0f;
  }
}

// input gradient of a convolution, times the ReLU mask of the layer below:
// gz_in[n][c][y][x] = (z_in > 0) * sum_k sum_taps gz[n][k][oy][ox] w[k][c][ky][kx]
__global__ __launch_bounds__(kThreads) void k_conv_dgrad(int N, int Cin, int H, const float* gz,
                                                         const float* w, const float* z_in,
                                                         float* gz_in) {
  const int Ho = H / 2;
  const long long total = (long long)N * Cin * H * H;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (long long)gridDim.x * kThreads) {
    if (!(z_in[e] > 0.0f)) { gz_in[e] = 0.0f; continue; }
    const int x = (int)(e % H), y = (int)((e / H) % H);
    const int c = (int)((e / ((long long)H * H)) % Cin);
    const long long n = e / ((long long)Cin * H * H);
    float s = 0.0f;
    for (int ky = 0; ky < 3; ++ky) {
      const int ty = y + 1 - ky;
      if (ty < 0 || (ty & 1) || ty / 2 >= Ho) continue;
      const int oy = ty / 2;
      for (int kx = 0; kx < 3; ++kx) {
        const int tx = x + 1 - kx;
        if (tx < 0 || (tx & 1) || tx / 2 >= Ho) continue;
        const int ox = tx / 2;
        for (int k = 0; k < kC; ++k)
          s = fmaf(gz[(((size_t)n * kC + k) * Ho + oy) * Ho + ox], w[((size_t)k * Cin + c) * 9 + ky * 3 + kx], s);
      }
    }
    gz_in[e] = s;
  }
}

// weight and bias gradients of a convolution: one workgroup per weight
// (K * Cin * 9 of them) followed by one per bias
__global__ __launch_bounds__(kThreads) void k_conv_wgrad(int N, int Cin, int H, const float* gz,
                                                         const float* in, const uint16_t* in16,
                                                         float* gw, float* gb) {
  __shared__ double red[kThreads / 64];
  const int Ho = H / 2;
  const int nw = kC * Cin * 9;
  const int e = blockIdx.x;
  double s = 0.0;
  const long long cnt = (long long)N * Ho * Ho;
  if (e < nw) {
    const int k = e / (Cin * 9), c = (e / 9) % Cin, ky = (e % 9) / 3, kx = e % 3;
    for (long long t = threadIdx.x; t < cnt; t += kThreads) {
      const int ox = (int)(t % Ho), oy = (int)((t / Ho) % Ho);
      const long long n = t / ((long long)Ho * Ho);
      const int y = 2 * oy + ky - 1, x = 2 * ox + kx - 1;
      if (y < 0 || y >= H || x < 0 || x >= H) continue;
      const size_t ii = (((size_t)n * Cin + c) * H + y) * H + x;
      const float v = in16 ? bf16_to_f(in16[ii]) : in[ii];
      s += (double)gz[(((size_t)n * kC + k) * Ho + oy) * Ho + ox] * v;
    }
  } else {
    const int k = e - nw;
    for (long long t = threadIdx.x; t < cnt; t += kThreads) {
      const long long n = t / ((long long)Ho * Ho);
      const int q = (int)(t % ((long long)Ho * Ho));
      s += gz[((size_t)n * kC + k) * Ho * Ho + q];
    }
  }
  const float v = block_sum_f(s, red);
  if (threadIdx.x == 0) {
    if (e < nw) gw[e] = v; else gb[e - nw] = v;
  }
}

// Adam on the FP32 master parameters; refreshes the bf16-rounded copy
__global__ __launch_bounds__(kThreads) void k_adam(float* prm, const float* grad, float* m, float* v,
                                                   float* wq, float lr, float b1, float b2, float eps,
                                                   float bc1, float bc2) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= kNParams) return;
  const float gk = grad[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float w = prm[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  prm[k] = w;
  wq[k] = is_conv_weight(k) ? bf16_round(w) : w;
}

__global__ __launch_bounds__(kThreads) void k_quantize(const float* prm, float* wq) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k < kNParams) wq[k] = is_conv_weight(k) ? bf16_round(prm[k]) : prm[k];
}

// He-uniform initialisation from a counter-based generator (splitmix64 of
// seed + index), zero biases
__global__ __launch_bounds__(kThreads) void k_cnn_init(float* prm, unsigned long long seed) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= kNParams) return;
  float lim = 0.0f;
  if (k < kOffB1) lim = sqrtf(6.0f / 72.0f);
  else if (k >= kOffW2 && k < kOffB2) lim = sqrtf(6.0f / 288.0f);
  else if (k >= kOffW3 && k < kOffB3) lim = sqrtf(6.0f / 288.0f);
  else if (k >= kOffWh && k < kOffBh) lim = sqrtf(6.0f / 32.0f);
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(k + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float u01 = (float)(z >> 40) * (1.0f / 16777216.0f);
  prm[k] = (2.0f * u01 - 1.0f) * lim;
}

// ------------------------------------------------------------------ gate
// Inference on MFMA: every convolution is a GEMM of 32 output channels by
// (3x3 taps x input channels) times (taps x channels) by (output positions),
// run as v_mfma_f32_16x16x32_bf16 tiles with FP32 accumulation: the weights
// are the A operand (rows = output channels), the im2col activations the B
// operand (columns = positions).
//
// A workgroup of two waves owns one block at a time, persistently over a
// range of blocks.  Wave w computes output channels 16 w .. 16 w + 15 of
// every layer over all its positions, so that it keeps one half of every
// layer's weights in registers for the workgroup's life, and a barrier
// separates the layers.  The block's input and both hidden activations stay
// in LDS in a position-major layout (one 80-byte slot of 32 bf16 channels per
// pixel, padded against bank conflicts) with a zero row and column in front
// for the convolutions' padding.  Small workgroups with 27 KB of LDS put five
// blocks in flight on every CU.
//
// Operand layout of the 16x16x32 MFMA: lane l supplies row (A) or column (B)
// l % 16 with the eight K values 8 (l / 16) .. 8 (l / 16) + 7; it receives
// D rows 4 (l / 16) .. + 3 of column l % 16, i.e. four consecutive output
// channels of one position, stored as one 8-byte LDS write of packed bf16
// (v_cvt_pk_bf16_f32, round to nearest even).  K index k = 8 g + e maps to
// input channel k in layers 2 and 3 (one tap per K step) and to (tap k / 2,
// channel k % 2) in layer 1 (taps 0..8, the rest zero).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kGateThreads = 128; // two waves per workgroup, one block at a time
constexpr int kIn = kS + 1;       // padded side of the space-to-depth input
constexpr int kS1 = 13;           // padded side of layer-1 output (12 + 1)
constexpr int kS2 = 7;            // padded side of layer-2 output (6 + 1)
constexpr int kPix = 40;          // bf16 slots per activation pixel (32 used)

struct __align__(16) GateLds {
  u32x4 in[kIn * kIn];                    // the 8 input channels of a pixel (16 B)
  uint16_t a1[kS1 * kS1 * kPix];
  uint16_t a2[kS2 * kS2 * kPix];
  float bias[5][kC];                      // per channel: b1, b2, b3 and the head weights wh0, wh1
  float hp[2][2];                         // head sums of the two waves
  int red[2][4];                          // ring statistics of the two waves
};
static_assert(offsetof(GateLds, a1) % 16 == 0 && offsetof(GateLds, a2) % 16 == 0,
              "activation images must be 16-byte aligned for 128-bit LDS reads");

// A wave's weights: output-channel tile mt = wave index; lane l holds row
// l % 16 of the A fragments.  The per-channel values (biases, head weights)
// are in LDS (GateLds::bias), where lane l reads those of its four D rows,
// channels 16 mt + 4 (l / 16) + j, when a layer needs them.
struct GateWeights {
  bf16x8 w1[3];                           // layer 1: K steps of 4 taps x 8 channels
  bf16x8 w2[9];                           // layer 2: per tap
  bf16x8 w3[9];                           // layer 3: per tap
  float bh0, bh1;                         // head biases
};

static __device__ __forceinline__ uint32_t bf16_bits(float x) {   // x already bf16-valued
  return __float_as_uint(x) >> 16;
}

// relu(v + b) of four accumulator rows, packed to bf16 (RNE): 8 bytes
static __device__ __forceinline__ uint2 relu_pack4(const f32x4& v, const float* b) {
  const bf16x2 lo = {(__bf16)fmaxf(v[0] + b[0], 0.0f), (__bf16)fmaxf(v[1] + b[1], 0.0f)};
  const bf16x2 hi = {(__bf16)fmaxf(v[2] + b[2], 0.0f), (__bf16)fmaxf(v[3] + b[3], 0.0f)};
  return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

// eight consecutive input channels c0 .. c0 + 7 of weight row n at one tap
static __device__ __forceinline__ bf16x8 weight_frag(const float* w, int cin, int n, int c0,
                                                     int tap) {
  uint32_t u[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    u[q] = bf16_bits(w[(n * cin + c0 + 2 * q) * 9 + tap]) |
           (bf16_bits(w[(n * cin + c0 + 2 * q + 1) * 9 + tap]) << 16);
  return __builtin_bit_cast(bf16x8, (u32x4){u[0], u[1], u[2], u[3]});
}

// The register image of one wave's weights, per lane: 21 bf16x8 MFMA
// fragments (layer 1: 3, layers 2 and 3: 9 each).  Packed once per weight
// update (k_gate_pack) into [role = wave][item][lane] order, so that a
// workgroup loads its weights with 16-byte coalesced reads.
constexpr int kPackItems = 3 + 9 + 9;

static __device__ __forceinline__ GateWeights gate_weights_from(const float* wq, int mt,
                                                                int lane) {
  const int row = lane & 15, g = lane >> 4;
  const int n = mt * 16 + row;
  const bf16x8 zero = __builtin_bit_cast(bf16x8, (u32x4){0u, 0u, 0u, 0u});
  GateWeights W;
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    const int tap = 4 * ks + g;                 // k = 32 ks + 8 g + channel
    W.w1[ks] = tap < 9 ? weight_frag(wq + kOffW1, kC0, n, 0, tap) : zero;
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) W.w2[tap] = weight_frag(wq + kOffW2, kC, n, 8 * g, tap);
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) W.w3[tap] = weight_frag(wq + kOffW3, kC, n, 8 * g, tap);
  W.bh0 = wq[kOffBh];
  W.bh1 = wq[kOffBh + 1];
  return W;
}

// one workgroup per role (wave index of the gate kernels), one thread per lane
__global__ __launch_bounds__(64) void k_gate_pack(const float* wq, uint4* pk) {
  const int role = blockIdx.x, lane = threadIdx.x;
  const GateWeights W = gate_weights_from(wq, role, lane);
  uint4* o = pk + (size_t)role * kPackItems * 64 + lane;
  int f = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) o[64 * f++] = __builtin_bit_cast(uint4, W.w1[k]);
#pragma unroll
  for (int k = 0; k < 9; ++k) o[64 * f++] = __builtin_bit_cast(uint4, W.w2[k]);
#pragma unroll
  for (int k = 0; k < 9; ++k) o[64 * f++] = __builtin_bit_cast(uint4, W.w3[k]);
}

static __device__ __forceinline__ GateWeights load_gate_weights(const uint4* pk, const float* wq) {
  const int lane = lane_id(), wave = wave_id();
  const uint4* src = pk + (size_t)wave * kPackItems * 64 + lane;
  uint4 v[kPackItems];
#pragma unroll
  for (int f = 0; f < kPackItems; ++f) v[f] = src[64 * f];
  GateWeights W;
  int f = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) W.w1[k] = __builtin_bit_cast(bf16x8, v[f++]);
#pragma unroll
  for (int k = 0; k < 9; ++k) W.w2[k] = __builtin_bit_cast(bf16x8, v[f++]);
#pragma unroll
  for (int k = 0; k < 9; ++k) W.w3[k] = __builtin_bit_cast(bf16x8, v[f++]);
  W.bh0 = wq[kOffBh];
  W.bh1 = wq[kOffBh + 1];
  return W;
}

// zero the padding row and column of every LDS image (never written later)
// and copy the per-channel values to LDS
static __device__ __forceinline__ void gate_lds_init(GateLds& G, const float* wq) {
  for (int e = threadIdx.x; e < 5 * kC; e += kGateThreads) {
    const int k = e / kC, c = e - k * kC;
    const int off = k == 0 ? kOffB1 : k == 1 ? kOffB2 : k == 2 ? kOffB3 : k == 3 ? kOffWh : kOffWh + kC;
    G.bias[k][c] = wq[off + c];
  }
  for (int e = threadIdx.x; e < 2 * kIn; e += kGateThreads) {
    const int k = e % kIn;
    G.in[e < kIn ? k : k * kIn] = (u32x4){0u, 0u, 0u, 0u};
  }
  for (int e = threadIdx.x; e < 2 * kS1 * kPix; e += kGateThreads) {
    const int pix = (e / kPix) % kS1, c = e % kPix;
    G.a1[(e < kS1 * kPix ? pix : pix * kS1) * kPix + c] = 0;
  }
  for (int e = threadIdx.x; e < 2 * kS2 * kPix; e += kGateThreads) {
    const int pix = (e / kPix) % kS2, c = e % kPix;
    G.a2[(e < kS2 * kPix ? pix : pix * kS2) * kPix + c] = 0;
  }
}

static __device__ __forceinline__ bf16x8 lds_frag(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

// The network on the input staged in G.in (the caller has synchronised the
// workgroup after staging); returns (y0, y1) in every thread.  Barriers
// inside; G.in is free again when it returns.
static __device__ __forceinline__ void gate_network(GateLds& G, const GateWeights& W, float& y0,
                                                    float& y1) {
  const int lane = lane_id(), mt = wave_id();
  const int col = lane & 15, g = lane >> 4;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const int ch = mt * 16 + 4 * g;        // channel of this lane's first D row
  auto bias4 = [&](int k, float* b) {
    const float4 v = *reinterpret_cast<const float4*>(&G.bias[k][ch]);
    b[0] = v.x; b[1] = v.y; b[2] = v.z; b[3] = v.w;
  };

  // layer 1: 144 positions = 9 column tiles; K = 9 taps x 8 channels in
  // three steps (lane group g takes tap 4 step + g; taps 9 .. 11 are zero).
  // The next tile's fragments are read while this tile's products run.
  {
    float b1[4];
    bias4(0, b1);
    u32x4 Xn[3];
    auto read_tile = [&](int nt) {
      const int m = nt * 16 + col;
      const int oy = m / 12, ox = m - oy * 12;
#pragma unroll
      for (int ks = 0; ks < 3; ++ks) {
        const int tap = 4 * ks + g;
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        Xn[ks] = tap < 9 ? G.in[(2 * oy + ky) * kIn + 2 * ox + kx] : (u32x4){0u, 0u, 0u, 0u};
      }
    };
    read_tile(0);
#pragma unroll 1
    for (int nt = 0; nt < 9; ++nt) {
      u32x4 X[3];
#pragma unroll
      for (int ks = 0; ks < 3; ++ks) X[ks] = Xn[ks];
      if (nt + 1 < 9) read_tile(nt + 1);
      f32x4 d = zero;
#pragma unroll
      for (int ks = 0; ks < 3; ++ks)
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w1[ks], __builtin_bit_cast(bf16x8, X[ks]), d,
                                                    0, 0, 0);
      const int m = nt * 16 + col;
      const int oy = m / 12, ox = m - oy * 12;
      *reinterpret_cast<uint2*>(&G.a1[((oy + 1) * kS1 + ox + 1) * kPix + mt * 16 + 4 * g]) =
          relu_pack4(d, b1);
    }
  }
  __syncthreads();

  // layer 2: 36 positions = 3 column tiles (the last 4 columns wide), the
  // three accumulation chains interleaved tap by tap
  {
    float b2[4];
    bias4(1, b2);
    f32x4 acc[3] = {zero, zero, zero};
    int base[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int m = min(t * 16 + col, 35);
      const int oy = m / 6, ox = m - oy * 6;
      base[t] = (2 * oy * kS1 + 2 * ox) * kPix + 8 * g;
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int off = ((tap / 3) * kS1 + tap % 3) * kPix;
      bf16x8 X[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) X[t] = lds_frag(&G.a1[base[t] + off]);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w2[tap], X[t], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int mv = t * 16 + col;
      if (mv < 36) {
        const int oy = mv / 6, ox = mv - oy * 6;
        *reinterpret_cast<uint2*>(&G.a2[((oy + 1) * kS2 + ox + 1) * kPix + mt * 16 + 4 * g]) =
            relu_pack4(acc[t], b2);
      }
    }
  }
  __syncthreads();

  // layer 3: 9 positions = one column tile (columns 9 .. 15 repeat position
  // 8 and are dropped); then the average pool of relu(conv + b3) and the
  // linear head over this wave's 16 channels
  {
    const int m = min(col, kPool - 1);
    const int oy = m / 3, ox = m - oy * 3;
    f32x4 acc = zero;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap % 3;
      const bf16x8 X = lds_frag(&G.a2[((2 * oy + ky) * kS2 + 2 * ox + kx) * kPix + 8 * g]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w3[tap], X, acc, 0, 0, 0);
    }
    float b3[4], wh0[4], wh1[4];
    bias4(2, b3);
    bias4(3, wh0);
    bias4(4, wh1);
    float h0 = 0.0f, h1 = 0.0f;
    if (col < kPool) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float r = fmaxf(acc[j] + b3[j], 0.0f);
        h0 += r * wh0[j];
        h1 += r * wh1[j];
      }
    }
    h0 = wave_sum(h0);
    h1 = wave_sum(h1);
    if (lane == 0) { G.hp[mt][0] = h0; G.hp[mt][1] = h1; }
  }
  __syncthreads();
  y0 = (G.hp[0][0] + G.hp[1][0]) * (1.0f / kPool) + W.bh0;
  y1 = (G.hp[0][1] + G.hp[1][1]) * (1.0f / kPool) + W.bh1;
}

// the 8 space-to-depth channels of input pixel (Y, X) from the four window
// pixels (2 Y + dy, 2 X + dx), dy, dx in {0, 1} (value -1 = unknown)
static __device__ __forceinline__ u32x4 s2d_pixel(const int* v) {
  uint32_t c0[4], c1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // (u - 128) / 128 is exact in bf16
    c0[q] = v[q] >= 0 ? bf16_bits((float)(v[q] - 128) * (1.0f / 128.0f)) : 0u;
    c1[q] = v[q] >= 0 ? 0u : 0x3f80u;                   // bf16 1.0
  }
  return (u32x4){c0[0] | (c0[1] << 16), c0[2] | (c0[3] << 16), c1[0] | (c1[1] << 16),
                 c1[2] | (c1[3] << 16)};
}

// Window staging of the gate kernels: thread t owns input pixels
// t + 128 k (four window pixels each).  The other workgroups on the CU
// (five are resident) cover the load latency.
constexpr int kGatePer = (kS * kS + kGateThreads - 1) / kGateThreads;

struct GateWindow {
  int v[kGatePer][4];

  // the window of the block in frame cell `cell`
  __device__ __forceinline__ void load(const FrameArgs& a, const DevParams& p, int cell) {
    // the per-thread index arithmetic is redone for every block rather than
    // kept live across the network (an empty asm hides that it repeats)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int by = cell / p.gw, bx = cell - by * p.gw;
    const int gy0 = by * p.B + p.B / 2 - kP / 2, gx0 = bx * p.B + p.B / 2 - kP / 2;
#pragma unroll
    for (int t = 0; t < kGatePer; ++t) {
      const int idx = tid + t * kGateThreads;
      const int Y = idx / kS, X = idx - Y * kS;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gy = gy0 + 2 * Y + (q >> 1), gx = gx0 + 2 * X + (q & 1);
        const bool in = idx < kS * kS && gy >= 0 && gy < p.height && gx >= 0 && gx < p.width;
        const int cy = min(max(gy, 0), p.height - 1), cx = min(max(gx, 0), p.width - 1);
        // 32-bit byte offsets (a value plane is far below 4 GiB): one register
        // per address
        const uint32_t off = 2u * (uint32_t)(cy * p.width + cx);
        const int val = *(const int16_t*)((const char*)a.val + off);
        v[t][q] = in ? val : -1;
      }
    }
  }

  // Writes the input image and returns the known context pixels of the
  // footprint (ring plus the block's own received pixels): count (own ones
  // again in bits 16..), sum, minimum, maximum, summed over the workgroup
  // (every thread gets them; one barrier inside).
  __device__ __forceinline__ void stage(GateLds& G, const DevParams& p, int& c, int& sum,
                                        int& vmin, int& vmax) const {
    const int lane = lane_id(), wave = wave_id();
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int b0 = kP / 2 - p.B / 2, b1 = b0 + p.B, f0 = b0 - p.r, f1 = b1 + p.r;
    c = 0; sum = 0; vmin = 255; vmax = 0;
#pragma unroll
    for (int t = 0; t < kGatePer; ++t) {
      const int idx = tid + t * kGateThreads;
      if (idx < kS * kS) {
        const int Y = idx / kS, X = idx - Y * kS;
        G.in[(Y + 1) * kIn + X + 1] = s2d_pixel(v[t]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int wy = 2 * Y + (q >> 1), wx = 2 * X + (q & 1);
          const bool ctx = wy >= f0 && wy < f1 && wx >= f0 && wx < f1;
          const bool own = wy >= b0 && wy < b1 && wx >= b0 && wx < b1;
          if (ctx && v[t][q] >= 0) {
            c += own ? 1 + (1 << 16) : 1;
            sum += v[t][q]; vmin = min(vmin, v[t][q]); vmax = max(vmax, v[t][q]);
          }
        }
      }
    }
    c = wave_sum(c); sum = wave_sum(sum); vmin = wave_min(vmin); vmax = wave_max(vmax);
    if (lane == 0) { G.red[wave][0] = c; G.red[wave][1] = sum; G.red[wave][2] = vmin; G.red[wave][3] = vmax; }
    __syncthreads();
    c = G.red[0][0] + G.red[1][0];
    sum = G.red[0][1] + G.red[1][1];
    vmin = min(G.red[0][2], G.red[1][2]);
    vmax = max(G.red[0][3], G.red[1][3]);
  }
};

// the statistics and the layer choice of block i (thread 0); a flat ring
// takes BRL without predictions
static __device__ __forceinline__ void gate_record(const FrameArgs& a, const DevParams& p, int i,
                                                   int c, int sum, int vmin, int vmax, bool flat,
                                                   float y0, float y1, float tau1, float tau2,
                                                   int& nq, int& mx) {
  const int nown = c >> 16;
  c &= 0xffff;
  a.m0cnt[i] = c | (nown > 0 ? kPartialBit : 0);
  a.ring[i] = make_int2(sum, vmin | (vmax << 16));
  nq += c >= p.r * p.B;
  mx = max(mx, c);
  a.gate[i] = (int8_t)(flat || y0 <= tau1 ? SKM_LAYER_BRL
                                          : (y1 > tau2 ? SKM_LAYER_HQL : SKM_LAYER_IDL));
  if (a.gate_pred) { a.gate_pred[2 * i] = y0; a.gate_pred[2 * i + 1] = y1; }
}

// The profile rule's flatness test on the staged ring statistics (phi =
// max - min of the known context pixels, 0 without any): a flat ring takes
// BRL, and the network is not run for it.
static __device__ __forceinline__ bool gate_flat(const DevParams& p, int c, int vmin, int vmax) {
  return (double)((c & 0xffff) > 0 ? vmax - vmin : 0) <= p.t_phi;
}

// In-pipeline gate, which also does the round preparation in CNN mode: one
// pass over the pending blocks of the round.  For each it records the
// known in-frame ring pixels (count, sum, minimum, maximum) from the window
// it has loaded anyway; a flat ring (phi <= t_phi) takes BRL as in the
// profile rule, any other block the network's choice, written to gate[i]
// (the predictions to gate_pred, NaN for flat rings).  Each workgroup adds its (blocks
// with |m0| >= r B, largest |m0|) to the round's context rule, as the prep
// kernel does.
__global__ __launch_bounds__(kGateThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_cnn_gate(FrameArgs a, DevParams p,
                                                           const uint4* pk, const float* wq,
                                                           float tau1, float tau2) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  GateLds& G = *reinterpret_cast<GateLds*>(lds_raw);
  RoundState* st = a.st;
  if (st->remaining == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->n_hql = 0;
  const int n_lost = st->n_lost;
  // XCD x (workgroups x, x + 8, ...) takes the x-th contiguous eighth of the
  // blocks, the same eighth as in the estimation kernel, so that the window
  // pixels read here are still in that XCD's L2 when the block is estimated;
  // its workgroups split the eighth evenly (the grid is a multiple of 8)
  const int per8 = (n_lost + 7) >> 3, xcd = blockIdx.x & 7;
  const int xend = min(n_lost, (xcd + 1) * per8);
  const int pw = (per8 + (int)(gridDim.x >> 3) - 1) / (int)(gridDim.x >> 3);
  const int i_begin = min(xend, xcd * per8 + (int)(blockIdx.x >> 3) * pw);
  const int i_end = min(xend, i_begin + pw);
  if (i_begin >= i_end) return;
  gate_lds_init(G, wq);
  const GateWeights W = load_gate_weights(pk, wq);
  // state and cell of the next block are read one block ahead
  int nx_state = a.bstate[i_begin], nx_cell = a.blk[i_begin];
  int wg_nq = 0, wg_max = 0;
  for (int i = i_begin; i < i_end; ++i) {
    const int state = nx_state, cell = nx_cell;
    if (i + 1 < i_end) { nx_state = a.bstate[i + 1]; nx_cell = a.blk[i + 1]; }
    if (state != 0) continue;            // not pending (uniform in the workgroup)
    GateWindow win;
    win.load(a, p, cell);
    int c, sum, vmin, vmax;
    win.stage(G, p, c, sum, vmin, vmax);
    if (gate_flat(p, c, vmin, vmax)) {    // uniform in the workgroup
      if (threadIdx.x == 0)
        gate_record(a, p, i, c, sum, vmin, vmax, true, NAN, NAN, tau1, tau2, wg_nq, wg_max);
      __syncthreads();                    // both waves have read G.red
      continue;
    }
    float y0, y1;
    gate_network(G, W, y0, y1);
    if (threadIdx.x == 0)
      gate_record(a, p, i, c, sum, vmin, vmax, false, y0, y1, tau1, tau2, wg_nq, wg_max);
  }
  if (threadIdx.x == 0) note_context_rule(st, wg_nq, wg_max);
}

// The gate over every frame of a batch (same block size and ring): as
// k_cnn_gate, with the items (frame, lost block) of all frames split among
// the workgroups by XCD eighths.  The weights are loaded once per workgroup
// for all its blocks.  Each workgroup adds its blocks to the context rule of
// their frame when it moves to the next frame.
__global__ __launch_bounds__(kGateThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_cnn_gate_b(BatchArgs b, DevParams p,
                                                             const uint4* pk, const float* wq,
                                                             float tau1, float tau2) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  GateLds& G = *reinterpret_cast<GateLds*>(lds_raw);
  if (b.bs->remaining == 0) return;
  if (blockIdx.x == 0)
    for (int f = threadIdx.x; f < b.nf; f += kGateThreads) b.a0.st[f].n_hql = 0;
  const int total = b.bs->total;
  const int per8 = (total + 7) >> 3, xcd = blockIdx.x & 7;
  const int xend = min(total, (xcd + 1) * per8);
  const int pw = (per8 + (int)(gridDim.x >> 3) - 1) / (int)(gridDim.x >> 3);
  const int g_begin = min(xend, xcd * per8 + (int)(blockIdx.x >> 3) * pw);
  const int g_end = min(xend, g_begin + pw);
  if (g_begin >= g_end) return;
  gate_lds_init(G, wq);
  const GateWeights W = load_gate_weights(pk, wq);
  int fc = -1;
  FrameArgs ac = batch_frame(b, 0);
  int wg_nq = 0, wg_max = 0;
  for (int g = g_begin; g < g_end; ++g) {
    if (fc < 0 || g >= b.cum[fc + 1]) {
      if (fc >= 0 && threadIdx.x == 0) note_context_rule(ac.st, wg_nq, wg_max);
      wg_nq = 0; wg_max = 0;
      fc = fc < 0 ? frame_of(b.cum, b.nf, g) : fc + 1;
      while (g >= b.cum[fc + 1]) ++fc;
      ac = batch_frame(b, fc);
    }
    const int i = g - b.cum[fc];
    if (ac.st->remaining == 0 || ac.bstate[i] != 0) continue;   // uniform in the workgroup
    GateWindow win;
    win.load(ac, p, ac.blk[i]);
    int c, sum, vmin, vmax;
    win.stage(G, p, c, sum, vmin, vmax);
    if (gate_flat(p, c, vmin, vmax)) {    // uniform in the workgroup
      if (threadIdx.x == 0)
        gate_record(ac, p, i, c, sum, vmin, vmax, true, NAN, NAN, tau1, tau2, wg_nq, wg_max);
      __syncthreads();                    // both waves have read G.red
      continue;
    }
    float y0, y1;
    gate_network(G, W, y0, y1);
    if (threadIdx.x == 0)
      gate_record(ac, p, i, c, sum, vmin, vmax, false, y0, y1, tau1, tau2, wg_nq, wg_max);
  }
  if (threadIdx.x == 0) note_context_rule(ac.st, wg_nq, wg_max);
}

// Batched inference on prepared inputs x (bf16 bits [n][8][24][24]).
__global__ __launch_bounds__(kGateThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_cnn_infer(const uint16_t* x, int n,
                                                            const uint4* pk, const float* wq,
                                                            float* y) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  GateLds& G = *reinterpret_cast<GateLds*>(lds_raw);
  gate_lds_init(G, wq);
  const GateWeights W = load_gate_weights(pk, wq);
  const int tid = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const uint16_t* xi = x + (size_t)i * kC0 * kS * kS;
    for (int idx = tid; idx < kS * kS; idx += kGateThreads) {
      uint32_t u[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        u[q] = (uint32_t)xi[(2 * q) * kS * kS + idx] | ((uint32_t)xi[(2 * q + 1) * kS * kS + idx] << 16);
      const int Y = idx / kS, X = idx - Y * kS;
      G.in[(Y + 1) * kIn + X + 1] = (u32x4){u[0], u[1], u[2], u[3]};
    }
    __syncthreads();
    float y0, y1;
    gate_network(G, W, y0, y1);
    if (tid == 0) { y[2 * (size_t)i] = y0; y[2 * (size_t)i + 1] = y1; }
  }
}

// -------------------------------------------------------------- launchers

static int cgrid(long long work) {
  long long g = (work + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_cnn_inputs(const FrameArgs& a, const DevParams& p, uint16_t* out, int max_blocks,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_inputs, dim3(max_blocks < 1 ? 1 : (max_blocks > 4096 ? 4096 : max_blocks)),
                     dim3(kThreads), 0, s, a, p, out);
  return hipGetLastError();
}

// upper bound of the gate's persistent grid (five workgroups per CU are
// resident: LDS; the caller picks the grid below this)
constexpr int kGateGrid = 4096;
constexpr int kInferGrid = 768;

// a multiple of 8 workgroups (the block ranges follow the XCD order)
int cnn_gate_grid(int requested) {
  const int g = requested < 1 ? 1 : (requested > kGateGrid ? kGateGrid : requested);
  return (g + 7) / 8 * 8;
}

hipError_t launch_cnn_gate(const FrameArgs& a, const DevParams& p, const uint4* pk,
                           const float* wq, float tau1, float tau2, int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_gate, dim3(cnn_gate_grid(max_blocks)), dim3(kGateThreads), sizeof(GateLds),
                     s, a, p, pk, wq, tau1, tau2);
  return hipGetLastError();
}

hipError_t launch_cnn_gate_b(const BatchArgs& b, const DevParams& p, const uint4* pk,
                             const float* wq, float tau1, float tau2, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_gate_b, dim3(cnn_gate_grid(grid)), dim3(kGateThreads), sizeof(GateLds), s,
                     b, p, pk, wq, tau1, tau2);
  return hipGetLastError();
}

hipError_t cnn_infer(const uint16_t* x, int n, const uint4* pk, const float* wq, float* y,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_infer, dim3(n > kInferGrid ? kInferGrid : n), dim3(kGateThreads),
                     sizeof(GateLds), s, x, n, pk, wq, y);
  return hipGetLastError();
}

hipError_t cnn_pack(const float* wq, uint4* pk, hipStream_t s) {
  hipLaunchKernelGGL(k_gate_pack, dim3(kGateThreads / 64), dim3(64), 0, s, wq, pk);
  return hipGetLastError();
}

size_t cnn_pack_bytes() { return sizeof(uint4) * (kGateThreads / 64) * kPackItems * 64; }

size_t cnn_gate_lds_bytes() { return sizeof(GateLds); }

hipError_t set_cnn_gate_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_cnn_gate,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_cnn_gate_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_cnn_infer, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t cnn_init(float* prm, float* wq, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_init, dim3(cgrid(kNParams)), dim3(kThreads), 0, s, prm, seed);
  hipLaunchKernelGGL(k_quantize, dim3(cgrid(kNParams)), dim3(kThreads), 0, s, prm, wq);
  return hipGetLastError();
}

hipError_t cnn_quantize(const float* prm, float* wq, hipStream_t s) {
  hipLaunchKernelGGL(k_quantize, dim3(cgrid(kNParams)), dim3(kThreads), 0, s, prm, wq);
  return hipGetLastError();
}

hipError_t cnn_forward(const CnnBuffers& b, const float* wq, const uint16_t* x, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_conv_fwd, dim3(cgrid((long long)N * kC * 144)), dim3(kThreads), 0, s, N, kC0,
                     kS, (const float*)nullptr, x, wq + kOffW1, wq + kOffB1, b.z1, b.a1, 1);
  hipLaunchKernelGGL(k_conv_fwd, dim3(cgrid((long long)N * kC * 36)), dim3(kThreads), 0, s, N, kC, 12,
                     (const float*)b.a1, (const uint16_t*)nullptr, wq + kOffW2, wq + kOffB2, b.z2, b.a2, 1);
  hipLaunchKernelGGL(k_conv_fwd, dim3(cgrid((long long)N * kC * kPool)), dim3(kThreads), 0, s, N, kC,
                     6, (const float*)b.a2, (const uint16_t*)nullptr, wq + kOffW3, wq + kOffB3, b.z3,
                     b.a3, 0);
  hipLaunchKernelGGL(k_head_fwd, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, s, N,
                     (const float*)b.a3, wq, b.g, b.y);
  return hipGetLastError();
}

hipError_t cnn_backward(const CnnBuffers& b, const float* wq, const uint16_t* x, const float* t,
                        int N, float* grad, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(kThreads), 0, s, N, (const float*)b.y, t, b.gy, loss);
  hipLaunchKernelGGL(k_head_wgrad, dim3(66), dim3(kThreads), 0, s, N, (const float*)b.gy,
                     (const float*)b.g, grad);
  hipLaunchKernelGGL(k_head_back, dim3(cgrid((long long)N * kC * kPool)), dim3(kThreads), 0, s, N,
                     (const float*)b.gy, wq, (const float*)b.z3, b.gz3);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(kC * kC * 9 + kC), dim3(kThreads), 0, s, N, kC, 6,
                     (const float*)b.gz3, (const float*)b.a2, (const uint16_t*)nullptr, grad + kOffW3,
                     grad + kOffB3);
  hipLaunchKernelGGL(k_conv_dgrad, dim3(cgrid((long long)N * kC * 36)), dim3(kThreads), 0, s, N, kC,
                     6, (const float*)b.gz3, wq + kOffW3, (const float*)b.z2, b.gz2);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(kC * kC * 9 + kC), dim3(kThreads), 0, s, N, kC, 12,
                     (const float*)b.gz2, (const float*)b.a1, (const uint16_t*)nullptr, grad + kOffW2,
                     grad + kOffB2);
  hipLaunchKernelGGL(k_conv_dgrad, dim3(cgrid((long long)N * kC * 144)), dim3(kThreads), 0, s, N, kC,
                     12, (const float*)b.gz2, wq + kOffW2, (const float*)b.z1, b.gz1);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(kC * kC0 * 9 + kC), dim3(kThreads), 0, s, N, kC0, kS,
                     (const float*)b.gz1, (const float*)nullptr, x, grad + kOffW1, grad + kOffB1);
  return hipGetLastError();
}

hipError_t cnn_adam(float* prm, const float* grad, float* m, float* v, float* wq, float lr, int step,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(cgrid(kNParams)), dim3(kThreads), 0, s, prm, grad, m, v, wq, lr,
                     b1, b2, 1e-8f, bc1, bc2);
  return hipGetLastError();
}

}  // namespace skm
