// Learned emission guide on gfx950.
//
// A 6-64-64-64-41 perceptron (position normalised to the scene box, unit
// normal) whose outputs parameterise a mixture of 8 von Mises-Fisher lobes
// folded onto the emitting hemisphere, mixed with the cosine density:
//   q(w) = alpha sum_k pi_k [v_k(w) + v_k(mirror(w))] + (1 - alpha) max(w.n, 0) / pi,
//   alpha = 0.9 sigmoid(o_40),  kappa_k = exp(clamp(o_5k+3, -3, 8)),
//   pi = softmax(o_5k+4),       mu_k = normalize(o_5k..5k+2).
// Products run on MFMA (v_mfma_f32_16x16x32_bf16): weights and layer inputs
// rounded to bfloat16 (nearest even), FP32 accumulation, FP32 bias and ReLU.
//
// Matrix layout.  A wave evaluates 64 items at once as four 16-item column
// tiles.  For D = A B (A 16x32, B 32x16) lane l holds A row l%16 and B column
// l%16 with k = 8(l/16) .. 8(l/16)+7, and D column l%16 with rows
// 4(l/16) .. 4(l/16)+3.  A layer computes out x items = W (out x in) times
// X (in x items), so its D registers, read as the next layer's B operand,
// carry input features in the order
//   k = 8g + i  ->  feature 32s + 16(i/4) + 4g + (i%4)     (g = l/16, K-step s);
// the packed weights use the same order, so activations never leave
// registers between layers.  Backward products dX = W^T dZ reuse it with
// W^T packed likewise; weight gradients dW = dZ X^T contract over the items
// and take both operands from LDS copies laid out [feature][item].
#include <hip/hip_runtime.h>
#define LT_NO_EVENT_COUNTERS
#include "lt_device.h"
#include "lt_launch.h"

namespace lt {
#ifdef LT_COUNTERS
inline namespace counted {
#endif

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kGIn = 6, kGH = 64, kGOut = 41, kGLobes = 8;
constexpr int kGW1 = 0, kGB1 = 384, kGW2 = 448, kGB2 = 4544, kGW3 = 4608, kGB3 = 8704, kGW4 = 8768,
              kGB4 = 11392, kGN = 11433;
static_assert(kGN == kGB4 + kGOut, "parameter layout");
// packed operand tiles, 16 bytes per lane, in u32x4 units
constexpr int kP1 = 0, kP2 = 256, kP3 = 768, kP4 = 1280, kPFwd = 1664;   // forward W
constexpr int kQ4 = 1664, kQ3 = 2176, kQ2 = 2688, kPAll = 3200;          // backward W^T
constexpr int kStage = 49;   // floats per item row of the output staging (odd: no bank aliasing)
constexpr int kHS = 72;      // bf16 per feature row of the [feature][item] copies
constexpr float kPiF = 3.14159265358979323846f, kInvPiF = 0.318309886183790672f;
constexpr float kLogKMin = -3.0f, kLogKMax = 8.0f, kAlphaMax = 0.9f;

__device__ __forceinline__ uint32_t bf16_bits(float x) {  // round to nearest, ties to even
  uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t pack2(float a, float b) { return bf16_bits(a) | (bf16_bits(b) << 16); }
__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int kperm(int s, int g, int i) { return 32 * s + 16 * (i >> 2) + 4 * g + (i & 3); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------ weight packing
__global__ void k_guide_pack(const float* __restrict__ w, u32x4* __restrict__ P) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kPAll) return;
  int lane = idx & 63, q = idx >> 6, g = lane >> 4, r = lane & 15;
  float v[8];
  for (int i = 0; i < 8; ++i) {
    float x = 0.f;
    if (idx < kP2) {  // layer 1, natural k order, inputs 6..31 zero
      int row = 16 * q + r, k = 8 * g + i;
      if (k < kGIn) x = w[kGW1 + row * kGIn + k];
    } else if (idx < kPFwd) {
      int base = idx < kP3 ? 4 : idx < kP4 ? 12 : 20;
      int off = idx < kP3 ? kGW2 : idx < kP4 ? kGW3 : kGW4;
      int n_out = idx < kP4 ? kGH : kGOut;
      int qq = q - base, m = qq >> 1, s = qq & 1;
      int row = 16 * m + r, in = kperm(s, g, i);
      if (row < n_out) x = w[off + row * kGH + in];
    } else {
      int base = idx < kQ3 ? 26 : idx < kQ2 ? 34 : 42;
      int off = idx < kQ3 ? kGW4 : idx < kQ2 ? kGW3 : kGW2;
      int n_out = idx < kQ3 ? kGOut : kGH;
      int qq = q - base, m = qq >> 1, s = qq & 1;
      int in = 16 * m + r, out = kperm(s, g, i);
      if (out < n_out) x = w[off + out * kGH + in];
    }
    v[i] = x;
  }
  P[idx] = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])};
}

// ------------------------------------------------------------ network
struct Fwd {
  f32x4 o[3][4];        // outputs, D layout (rows 16m + 4g + i, item 16t + l%16)
  uint64_t mask[3];     // ReLU masks of layers 1-3, bit (m*4 + t)*4 + i
};

__device__ __forceinline__ void features(const DevScene& sc, f3 x, f3 n, float f[kGIn]) {
  f[0] = (x.x - sc.gb_c[0]) * sc.gb_ih[0];
  f[1] = (x.y - sc.gb_c[1]) * sc.gb_ih[1];
  f[2] = (x.z - sc.gb_c[2]) * sc.gb_ih[2];
  f[3] = n.x; f[4] = n.y; f[5] = n.z;
}

// Layer-1 B operands from every lane's features.
__device__ __forceinline__ void input_tiles(const float f[kGIn], bf16x8 xb[4]) {
  const int lane = __lane_id(), g = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int src = 16 * t + (lane & 15);
    float v[kGIn];
#pragma unroll
    for (int k = 0; k < kGIn; ++k) v[k] = __shfl(f[k], src);
    u32x4 u = {0u, 0u, 0u, 0u};
    if (g == 0) u = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), 0u};
    xb[t] = as_bf(u);
  }
}

// bias + ReLU of a 64-row layer; returns the next layer's B operands and the
// mask; optionally stores the bf16 activations to LDS as [feature][item].
template <bool STORE>
__device__ __forceinline__ void relu_tiles(f32x4 (&d)[4][4], const float* __restrict__ bias, bf16x8 (&h)[2][4],
                                           uint64_t& mask, uint16_t* hs) {
  const int lane = __lane_id(), g = lane >> 4;
  mask = 0ull;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    float b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = bias[16 * m + 4 * g + i];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float z = d[m][t][i] + b[i];
        if (z > 0.f) mask |= 1ull << ((m * 4 + t) * 4 + i);
        d[m][t][i] = fmaxf(z, 0.f);
      }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u32x4 u = {pack2(d[2 * s][t][0], d[2 * s][t][1]), pack2(d[2 * s][t][2], d[2 * s][t][3]),
                 pack2(d[2 * s + 1][t][0], d[2 * s + 1][t][1]), pack2(d[2 * s + 1][t][2], d[2 * s + 1][t][3])};
      h[s][t] = as_bf(u);
      if (STORE) {
        int item = 16 * t + (lane & 15);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          uint32_t word = u[i >> 1];
          hs[kperm(s, g, i) * kHS + item] = (uint16_t)((i & 1) ? (word >> 16) : (word & 0xFFFFu));
        }
      }
    }
}

__device__ __forceinline__ void dense64(const u32x4* __restrict__ P, int base, const bf16x8 (&h)[2][4],
                                        f32x4 (&d)[4][4]) {
  const int lane = __lane_id();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x8 a0 = as_bf(P[base + (m * 2 + 0) * 64 + lane]);
    bf16x8 a1 = as_bf(P[base + (m * 2 + 1) * 64 + lane]);
#pragma unroll
    for (int t = 0; t < 4; ++t) d[m][t] = mfma(a1, h[1][t], mfma(a0, h[0][t], f32x4{0.f, 0.f, 0.f, 0.f}));
  }
}

// Full forward pass of the wave's 64 items.  P: packed forward weights
// (LDS or global); w: FP32 master parameters (biases).  STORE: keep the
// layer inputs in LDS ([feature][item], bf16) for the weight gradients.
template <bool STORE>
__device__ __forceinline__ void mlp_forward(const u32x4* __restrict__ P, const float* __restrict__ w,
                                            const float f[kGIn], Fwd& F, uint16_t* x1s, uint16_t* h1s,
                                            uint16_t* h2s, uint16_t* h3s) {
  const int lane = __lane_id(), g = lane >> 4;
  bf16x8 xb[4];
  input_tiles(f, xb);
  if (STORE) {
#pragma unroll
    for (int k = 0; k < kGIn; ++k) x1s[k * kHS + lane] = (uint16_t)bf16_bits(f[k]);
  }
  f32x4 d[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x8 a = as_bf(P[kP1 + m * 64 + lane]);
#pragma unroll
    for (int t = 0; t < 4; ++t) d[m][t] = mfma(a, xb[t], f32x4{0.f, 0.f, 0.f, 0.f});
  }
  bf16x8 h[2][4];
  relu_tiles<STORE>(d, w + kGB1, h, F.mask[0], h1s);
  dense64(P, kP2, h, d);
  relu_tiles<STORE>(d, w + kGB2, h, F.mask[1], h2s);
  dense64(P, kP3, h, d);
  relu_tiles<STORE>(d, w + kGB3, h, F.mask[2], h3s);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    bf16x8 a0 = as_bf(P[kP4 + (m * 2 + 0) * 64 + lane]);
    bf16x8 a1 = as_bf(P[kP4 + (m * 2 + 1) * 64 + lane]);
    float b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int row = 16 * m + 4 * g + i;
      b[i] = row < kGOut ? w[kGB4 + row] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 o = mfma(a1, h[1][t], mfma(a0, h[0][t], f32x4{0.f, 0.f, 0.f, 0.f}));
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] += b[i];
      F.o[m][t] = o;
    }
  }
}

// D-layout outputs -> this lane's own item row of 41 outputs (via LDS).
__device__ __forceinline__ void outputs_to_lane(const Fwd& F, float* stage, float o[kGOut]) {
  const int lane = __lane_id(), g = lane >> 4;
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) stage[(16 * t + (lane & 15)) * kStage + 16 * m + 4 * g + i] = F.o[m][t][i];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kGOut; ++k) o[k] = stage[lane * kStage + k];
  __syncthreads();
}

// ------------------------------------------------------------ mixture
struct GMix {
  f3 mu[kGLobes];
  float mlen[kGLobes], kap[kGLobes], pi[kGLobes];
  uint32_t kfree;   // bit k: log-concentration inside its clamp range
  float alpha, sig;
};

__device__ __forceinline__ GMix mixture_of(const float o[kGOut]) {
  GMix m;
  float lmax = o[4];
#pragma unroll
  for (int k = 1; k < kGLobes; ++k) lmax = fmaxf(lmax, o[5 * k + 4]);
  float z = 0.f;
  m.kfree = 0u;
#pragma unroll
  for (int k = 0; k < kGLobes; ++k) {
    f3 v = {o[5 * k], o[5 * k + 1], o[5 * k + 2]};
    float l = sqrtf(dot(v, v));
    m.mlen[k] = l;
    m.mu[k] = l > 0.f ? v * (1.0f / l) : mk(0.f, 0.f, 1.f);
    float lk = o[5 * k + 3];
    if (lk > kLogKMin && lk < kLogKMax) m.kfree |= 1u << k;
    m.kap[k] = expf(fminf(fmaxf(lk, kLogKMin), kLogKMax));
    m.pi[k] = expf(o[5 * k + 4] - lmax);
    z += m.pi[k];
  }
  float iz = 1.0f / z;
#pragma unroll
  for (int k = 0; k < kGLobes; ++k) m.pi[k] *= iz;
  m.sig = 1.0f / (1.0f + expf(-o[40]));
  m.alpha = kAlphaMax * m.sig;
  return m;
}

__device__ __forceinline__ float vmf(f3 mu, float kap, f3 w) {
  return kap / (2.0f * kPiF * -expm1f(-2.0f * kap)) * expf(kap * (dot(mu, w) - 1.0f));
}
__device__ __forceinline__ f3 mirror(f3 w, f3 n) { return w - n * (2.0f * dot(w, n)); }

__device__ __forceinline__ float mix_pdf(const GMix& m, f3 n, f3 w) {
  float c = dot(w, n);
  if (c < 0.f) return 0.f;
  f3 wm = mirror(w, n);
  float V = 0.f;
#pragma unroll
  for (int k = 0; k < kGLobes; ++k) V += m.pi[k] * (vmf(m.mu[k], m.kap[k], w) + vmf(m.mu[k], m.kap[k], wm));
  return m.alpha * V + (1.0f - m.alpha) * c * kInvPiF;
}

// Component by g0 (cosine part when g0 >= alpha, else the lobe whose
// cumulative weight first exceeds g0/alpha), direction by (g1, g2): the vMF
// cosine t by inverting its marginal (Wood 1994; Jakob 2012),
// t = 1 + log(xi + (1 - xi) e^{-2 kappa}) / kappa with xi = 1 - g1.
__device__ __forceinline__ f3 mix_sample(const GMix& m, f3 n, float g0, float g1, float g2, int& comp) {
  if (g0 >= m.alpha) {
    comp = 0;
    return cosine_dir(n, g1, g2);
  }
  float v = g0 / m.alpha, acc = 0.f;
  int k = kGLobes - 1;
  bool found = false;
#pragma unroll
  for (int i = 0; i < kGLobes; ++i) {
    acc += m.pi[i];
    if (!found && v < acc) { k = i; found = true; }
  }
  comp = k + 1;
  f3 mu = m.mu[0];
  float kap = m.kap[0];
#pragma unroll
  for (int i = 1; i < kGLobes; ++i)
    if (i == k) { mu = m.mu[i]; kap = m.kap[i]; }
  // 1 - t = -log(xi + (1 - xi) e^{-2 kappa}) / kappa = -log1p(-g1 (1 - e^{-2 kappa})) / kappa
  // (1 - xi = g1 exactly)
  f3 w = vmf_dir(mu, kap, -expm1f(-2.0f * kap), g1, g2);
  if (dot(w, n) < 0.f) w = mirror(w, n);
  return w;
}

// d(-c log q(w))/d(outputs); returns -c log q (0 when q <= 0 or c == 0).
__device__ __forceinline__ float mix_loss_grad(const float o[kGOut], f3 n, f3 w, float c, float go[kGOut]) {
#pragma unroll
  for (int k = 0; k < kGOut; ++k) go[k] = 0.f;
  if (c == 0.f) return 0.f;
  GMix m = mixture_of(o);
  float q = mix_pdf(m, n, w);
  if (!(q > 0.f)) return 0.f;
  float cosp = fmaxf(dot(w, n), 0.f) * kInvPiF;
  f3 wm = mirror(w, n);
  float Vk[kGLobes], V = 0.f;
#pragma unroll
  for (int k = 0; k < kGLobes; ++k) {
    Vk[k] = vmf(m.mu[k], m.kap[k], w) + vmf(m.mu[k], m.kap[k], wm);
    V += m.pi[k] * Vk[k];
  }
  float s = -c / q;
  go[40] = s * (V - cosp) * kAlphaMax * m.sig * (1.0f - m.sig);
#pragma unroll
  for (int k = 0; k < kGLobes; ++k) {
    float wk = s * m.alpha * m.pi[k];
    go[5 * k + 4] = wk * (Vk[k] - V);
    float kap = m.kap[k], dk = 0.f;
    f3 gm = {0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      f3 wr = r ? wm : w;
      float mw = dot(m.mu[k], wr);
      float v = vmf(m.mu[k], kap, wr);
      dk += v * (1.0f / kap - 2.0f / expm1f(2.0f * kap) + (mw - 1.0f));
      if (m.mlen[k] > 0.f) gm = gm + (wr - m.mu[k] * mw) * (v * kap / m.mlen[k]);
    }
    go[5 * k + 3] = ((m.kfree >> k) & 1u) ? wk * dk * kap : 0.f;
    go[5 * k + 0] = wk * gm.x; go[5 * k + 1] = wk * gm.y; go[5 * k + 2] = wk * gm.z;
  }
  return -c * logf(q);
}

// ------------------------------------------------------------ kernels
// Raw outputs [count][41] at positions x and normals n [count][3].
__global__ void __launch_bounds__(256) k_guide_eval(GuideArgs G) {
  extern __shared__ u32x4 gl_lds[];
  for (int i = threadIdx.x; i < kPFwd; i += blockDim.x) gl_lds[i] = G.packed[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = __lane_id();
  float* stage = reinterpret_cast<float*>(gl_lds + kPFwd) + wave * 64 * kStage;
  const int64_t n_tiles = (G.count + 63) / 64;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_tiles; base += (int64_t)gridDim.x * 4) {
    int64_t item = (base + wave) * 64 + lane;
    bool valid = item < G.count;
    int64_t ic = valid ? item : G.count - 1;
    f3 x = ld3(G.x + ic * 3), n = ld3(G.n + ic * 3);
    float f[kGIn];
    features(G.sc, x, n, f);
    Fwd F;
    mlp_forward<false>(gl_lds, G.w, f, F, nullptr, nullptr, nullptr, nullptr);
    float o[kGOut];
    outputs_to_lane(F, stage, o);
    if (valid)
      for (int k = 0; k < kGOut; ++k) G.out[item * kGOut + k] = o[k];
  }
}

// Guide table of the Lambertian texels: item i = 2 texel + side evaluates
// the network at the texel centre x[texel] with normal +n[texel] (side 0)
// or -n[texel] (side 1) and stores the folded mixture as a 16-float4 entry
// (layout of gtab_sample); a texel with n = 0 (no covering triangle) gets
// alpha = -1 (cosine sampling).
__global__ void __launch_bounds__(256) k_guide_table(GuideArgs G) {
  extern __shared__ u32x4 gl_lds[];
  for (int i = threadIdx.x; i < kPFwd; i += blockDim.x) gl_lds[i] = G.packed[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = __lane_id();
  float* stage = reinterpret_cast<float*>(gl_lds + kPFwd) + wave * 64 * kStage;
  const int64_t n_tiles = (G.count + 63) / 64;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_tiles; base += (int64_t)gridDim.x * 4) {
    int64_t item = (base + wave) * 64 + lane;
    bool valid = item < G.count;
    int64_t it = valid ? item : G.count - 1, tx = it >> 1;
    f3 x = ld3(G.x + tx * 3), n = ld3(G.n + tx * 3);
    if (it & 1) n = n * -1.0f;
    float f[kGIn];
    features(G.sc, x, n, f);
    Fwd F;
    mlp_forward<false>(gl_lds, G.w, f, F, nullptr, nullptr, nullptr, nullptr);
    float o[kGOut];
    outputs_to_lane(F, stage, o);
    if (!valid) continue;
    float4* e = G.table + item * kGTabF4;
    if (dot(n, n) == 0.f) {
      for (int k = 0; k < kGTabF4; ++k) e[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      e[1].w = -1.0f;
      continue;
    }
    GMix m = mixture_of(o);
    for (int k = 0; k < kGLobes; ++k) {
      float kap = m.kap[k], em = -expm1f(-2.0f * kap);
      e[2 * k] = make_float4(m.mu[k].x, m.mu[k].y, m.mu[k].z, kap);
      e[2 * k + 1] = make_float4(m.pi[k], kap / (2.0f * kPiF * em), em, k == 0 ? m.alpha : 0.f);
    }
  }
}

// Guided emission of paths [0, count): record (w, q) per path for the
// tracer and, optionally, the training sample (x, n, w, q, S, component).
__global__ void __launch_bounds__(256) k_guide_emit(GuideArgs G) {
  extern __shared__ u32x4 gl_lds[];
  for (int i = threadIdx.x; i < kPFwd; i += blockDim.x) gl_lds[i] = G.packed[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = __lane_id();
  float* stage = reinterpret_cast<float*>(gl_lds + kPFwd) + wave * 64 * kStage;
  const DevScene& sc = G.sc;
  const f3 o0 = ld3(sc.em_o), e1 = ld3(sc.em_e1), e2 = ld3(sc.em_e2), ne = ld3(sc.em_n);
  const int64_t n_tiles = (G.count + 63) / 64;
  const uint64_t seed = G.seed_ptr ? *G.seed_ptr : G.seed;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_tiles; base += (int64_t)gridDim.x * 4) {
    int64_t p = (base + wave) * 64 + lane;
    bool valid = p < G.count;
    uint32_t path = (uint32_t)(valid ? p : 0);
    u4f u = rng4(seed, path, 0u, 0u);
    f3 x = o0 + e1 * u.u0 + e2 * u.u1;
    float f[kGIn];
    features(sc, x, ne, f);
    Fwd F;
    mlp_forward<false>(gl_lds, G.w, f, F, nullptr, nullptr, nullptr, nullptr);
    float o[kGOut];
    outputs_to_lane(F, stage, o);
    GMix m = mixture_of(o);
    u4f gu = rng4(seed, path, 0u, 1u);
    int comp;
    f3 w = mix_sample(m, ne, gu.u0, gu.u1, gu.u2, comp);
    float q = mix_pdf(m, ne, w);
    if (!valid) continue;
    if (G.rec) G.rec[p] = make_float4(w.x, w.y, w.z, q);
    if (G.samples) {
      float* s = G.samples + p * 12;
      s[0] = x.x; s[1] = x.y; s[2] = x.z; s[3] = ne.x; s[4] = ne.y; s[5] = ne.z;
      s[6] = w.x; s[7] = w.y; s[8] = w.z; s[9] = q;
      s[10] = G.contrib ? G.contrib[p] : 0.f;
      s[11] = (float)comp;
    }
  }
}

// Weight-gradient products of one layer: acc[m][n] += dZ (rows 16m..) times
// X^T (columns 16n..), contracting over the 64 items, operands from LDS.
template <int M, int N>
__device__ __forceinline__ void dw_tiles(const uint16_t* zs, const uint16_t* xs, f32x4 (&acc)[M][N]) {
  const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bf16x8 b[N];
#pragma unroll
    for (int n = 0; n < N; ++n)
      b[n] = as_bf(*reinterpret_cast<const u32x4*>(xs + (16 * n + r) * kHS + 32 * s + 8 * g));
#pragma unroll
    for (int m = 0; m < M; ++m) {
      bf16x8 a = as_bf(*reinterpret_cast<const u32x4*>(zs + (16 * m + r) * kHS + 32 * s + 8 * g));
#pragma unroll
      for (int n = 0; n < N; ++n) acc[m][n] = mfma(a, b[n], acc[m][n]);
    }
  }
}

// dZ (D layout, 64 rows) -> next B operands (bf16) and the LDS copy.
__device__ __forceinline__ void dz_store(const f32x4 (&dz)[4][4], bf16x8 (&zb)[2][4], uint16_t* zs) {
  const int lane = __lane_id(), g = lane >> 4;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u32x4 u = {pack2(dz[2 * s][t][0], dz[2 * s][t][1]), pack2(dz[2 * s][t][2], dz[2 * s][t][3]),
                 pack2(dz[2 * s + 1][t][0], dz[2 * s + 1][t][1]), pack2(dz[2 * s + 1][t][2], dz[2 * s + 1][t][3])};
      zb[s][t] = as_bf(u);
      int item = 16 * t + (lane & 15);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        uint32_t word = u[i >> 1];
        zs[kperm(s, g, i) * kHS + item] = (uint16_t)((i & 1) ? (word >> 16) : (word & 0xFFFFu));
      }
    }
}

// dH = W^T dZ for a 64-input layer, masked by the layer's ReLU: dZ_prev.
__device__ __forceinline__ void back64(const u32x4* __restrict__ P, int base, const bf16x8 (&zb)[2][4],
                                       uint64_t mask, f32x4 (&dz)[4][4]) {
  const int lane = __lane_id();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x8 a0 = as_bf(P[base + (m * 2 + 0) * 64 + lane]);
    bf16x8 a1 = as_bf(P[base + (m * 2 + 1) * 64 + lane]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 d = mfma(a1, zb[1][t], mfma(a0, zb[0][t], f32x4{0.f, 0.f, 0.f, 0.f}));
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = ((mask >> ((m * 4 + t) * 4 + i)) & 1ull) ? d[i] : 0.f;
      dz[m][t] = d;
    }
  }
}

__device__ __forceinline__ void bias_acc(const f32x4 (&dz)[4][4], float (&db)[4][4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) db[m][i] += dz[m][0][i] + dz[m][1][i] + dz[m][2][i] + dz[m][3][i];
}

// Unnormalised loss -sum_b (S_b / q_b) log q(w_b | x_b, n_b), its gradient and
// Z = sum_b S_b / q_b: one wave per workgroup; each workgroup writes its
// partial gradient, loss (slot kGN) and Z (slot kGN + 1) to
// partial[blockIdx.x][kGN + 2]; the reduction divides by Z.
__global__ void __launch_bounds__(64) k_guide_grad(GuideArgs G) {
  extern __shared__ float gg_lds[];
  float* stage = gg_lds;                                              // [64][kStage]
  uint16_t* x1s = reinterpret_cast<uint16_t*>(stage + 64 * kStage);   // [16][kHS]
  uint16_t* h1s = x1s + 16 * kHS;                                     // [64][kHS] each
  uint16_t* h2s = h1s + 64 * kHS;
  uint16_t* h3s = h2s + 64 * kHS;
  uint16_t* zs = h3s + 64 * kHS;
  const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
  const u32x4* P = G.packed;
  for (int i = lane; i < 16 * kHS; i += 64) x1s[i] = 0;
  __syncthreads();
  f32x4 a1[4][1], a2[4][4], a3[4][4], a4[3][4];
  float db1[4][4], db2[4][4], db3[4][4];
  float db4 = 0.f;  // lane k < 41: output bias k
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    a1[m][0] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int n = 0; n < 4; ++n) { a2[m][n] = a1[m][0]; a3[m][n] = a1[m][0]; if (m < 3) a4[m][n] = a1[m][0]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) db1[m][i] = db2[m][i] = db3[m][i] = 0.f;
  }
  float loss = 0.f, zsum = 0.f;
  const int64_t n_tiles = (G.count + 63) / 64;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    int64_t b = tile * 64 + lane;
    bool valid = b < G.count;
    const float* smp = G.samples + (valid ? b : 0) * 12;
    f3 x = ld3(smp), n = ld3(smp + 3), w = ld3(smp + 6);
    float qs = smp[9], S = smp[10];
    float c = (valid && qs > 0.f && S != 0.f) ? S / qs : 0.f;
    zsum += c;
    float f[kGIn];
    features(G.sc, x, n, f);
    Fwd F;
    mlp_forward<true>(P, G.w, f, F, x1s, h1s, h2s, h3s);
    float o[kGOut], go[kGOut];
    outputs_to_lane(F, stage, o);
    loss += mix_loss_grad(o, n, w, c, go);
    // output adjoints: FP32 copy [item][output] for the bias sums, bf16 copy
    // [output][item] for the products
#pragma unroll
    for (int k = 0; k < kGOut; ++k) stage[lane * kStage + k] = go[k];
#pragma unroll
    for (int k = 0; k < 48; ++k) zs[k * kHS + lane] = k < kGOut ? (uint16_t)bf16_bits(go[k]) : (uint16_t)0;
    __syncthreads();
    if (lane < kGOut) {
      float sacc = 0.f;
      for (int it = 0; it < 64; ++it) sacc += stage[it * kStage + lane];
      db4 += sacc;
    }
    dw_tiles<3, 4>(zs, h3s, a4);
    // dH3 = W4^T dZ4, B operands gathered from the LDS copy in permuted order
    bf16x8 zb[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int item = 16 * t + r;
        uint32_t e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          int row = kperm(s, g, i);
          e[i] = row < 48 ? zs[row * kHS + item] : 0u;
        }
        zb[s][t] = as_bf(u32x4{e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16), e[6] | (e[7] << 16)});
      }
    f32x4 dz[4][4];
    back64(P, kQ4, zb, F.mask[2], dz);
    bias_acc(dz, db3);
    __syncthreads();
    dz_store(dz, zb, zs);
    __syncthreads();
    dw_tiles<4, 4>(zs, h2s, a3);
    back64(P, kQ3, zb, F.mask[1], dz);
    bias_acc(dz, db2);
    __syncthreads();
    dz_store(dz, zb, zs);
    __syncthreads();
    dw_tiles<4, 4>(zs, h1s, a2);
    back64(P, kQ2, zb, F.mask[0], dz);
    bias_acc(dz, db1);
    __syncthreads();
    dz_store(dz, zb, zs);
    __syncthreads();
    dw_tiles<4, 1>(zs, x1s, a1);
    __syncthreads();
  }
  // write this workgroup's partial gradient
  float* out = G.partial + (size_t)blockIdx.x * (kGN + 2);
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int row = 16 * m + 4 * g + i;
      if (r < kGIn) out[kGW1 + row * kGIn + r] = a1[m][0][i];
#pragma unroll
      for (int nn = 0; nn < 4; ++nn) {
        int col = 16 * nn + r;
        out[kGW2 + row * kGH + col] = a2[m][nn][i];
        out[kGW3 + row * kGH + col] = a3[m][nn][i];
        if (m < 3 && row < kGOut) out[kGW4 + row * kGH + col] = a4[m][nn][i];
      }
    }
  // bias sums: over the 16 lanes of a row group (hidden), over all lanes (output)
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v1 = db1[m][i], v2 = db2[m][i], v3 = db3[m][i];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        v1 += __shfl_xor(v1, off); v2 += __shfl_xor(v2, off); v3 += __shfl_xor(v3, off);
      }
      if (r == 0) {
        int row = 16 * m + 4 * g + i;
        out[kGB1 + row] = v1; out[kGB2 + row] = v2; out[kGB3 + row] = v3;
      }
    }
  if (lane < kGOut) out[kGB4 + lane] = db4;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    loss += __shfl_xor(loss, off);
    zsum += __shfl_xor(zsum, off);
  }
  if (lane == 0) { out[kGN] = loss; out[kGN + 1] = zsum; }
}

// grad[j] = (sum over workgroups of partial[.][j]) / Z, sums in fixed order;
// loss likewise; everything zero when Z is.
__global__ void k_guide_reduce(const float* __restrict__ partial, int n_part, float* __restrict__ grad,
                               float* __restrict__ loss) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > kGN) return;
  float s = 0.f, z = 0.f;
  for (int b = 0; b < n_part; ++b) {
    s += partial[(size_t)b * (kGN + 2) + j];
    z += partial[(size_t)b * (kGN + 2) + kGN + 1];
  }
  float r = z > 0.f ? s / z : 0.f;
  if (j < kGN) grad[j] = r;
  else if (loss) loss[0] = r;
}

// Adam (Kingma & Ba 2015); c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t).
__global__ void k_guide_adam(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ m,
                             float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                             float c2) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float gj = grad[j];
  float mj = b1 * m[j] + (1.0f - b1) * gj;
  float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
  m[j] = mj; v[j] = vj;
  w[j] -= lr * (mj * c1) / (sqrtf(vj * c2) + eps);
}

#ifdef LT_COUNTERS
}  // namespace counted
#endif

// ------------------------------------------------------------ launchers
size_t guide_packed_bytes() { return (size_t)kPAll * sizeof(u32x4); }
size_t guide_partial_floats() { return (size_t)kGN + 2; }
static size_t emit_lds() { return (size_t)kPFwd * sizeof(u32x4) + 4 * 64 * kStage * sizeof(float); }
static size_t grad_lds() { return 64 * kStage * sizeof(float) + (16 + 4 * 64) * kHS * sizeof(uint16_t); }

hipError_t guide_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_guide_emit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)emit_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_guide_eval, hipFuncAttributeMaxDynamicSharedMemorySize, (int)emit_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_guide_table, hipFuncAttributeMaxDynamicSharedMemorySize, (int)emit_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_guide_grad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_lds());
  return e;
}

hipError_t launch_guide_pack(const float* w, void* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_pack, dim3((kPAll + 255) / 256), dim3(256), 0, s, w, (u32x4*)packed);
  return hipGetLastError();
}
hipError_t launch_guide_eval(const GuideArgs& G, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_eval, dim3(grid), dim3(256), emit_lds(), s, G);
  return hipGetLastError();
}
hipError_t launch_guide_table(const GuideArgs& G, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_table, dim3(grid), dim3(256), emit_lds(), s, G);
  return hipGetLastError();
}
hipError_t launch_guide_emit(const GuideArgs& G, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_emit, dim3(grid), dim3(256), emit_lds(), s, G);
  return hipGetLastError();
}
hipError_t launch_guide_grad(const GuideArgs& G, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_grad, dim3(grid), dim3(64), grad_lds(), s, G);
  return hipGetLastError();
}
hipError_t launch_guide_reduce(const float* partial, int n_part, float* grad, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_reduce, dim3((kGN + 1 + 255) / 256), dim3(256), 0, s, partial, n_part, grad, loss);
  return hipGetLastError();
}
hipError_t launch_guide_adam(float* w, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                             float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, grad, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lt
