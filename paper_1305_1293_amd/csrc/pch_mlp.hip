// Learned selection cutoff: a small MLP that predicts the geodesic distance
// of every vertex from the source, trained on distance fields computed by the
// PCH kernels. Its predictions only decide how far each round's selection
// reaches; the distances stay exact whatever it predicts (processing order
// does not change the result: Section 4, "Correctness", and Remark 2).
//
// Network: features x (7) -> 64 -> 64 -> 1, ReLU. FP32 master weights;
// weights and activations are rounded to BF16 (round to nearest even) before
// every product and the products are accumulated in FP32. Output
// d = base * (1 + softplus(y)) with base the 3-D chord |v - s|, so a
// prediction never undercuts the chord. Loss mean(((d - target) / scale)^2).
//
// Mapping: one wavefront per stream of samples, lane j = hidden unit j; the
// 64-wide layers exchange activations with wavefront shuffles. Gradients are
// reduced per block in LDS and added to the global gradient with one atomic
// per parameter and block (training). Inference runs on the matrix cores
// (k_mlp_forward_mfma).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pch.h"
#include "pch_internal.h"

namespace {

pch_status mlp_err(pch_status s, const std::string& m) { return (pch_status)pch::set_error(s, m); }
#define MLP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return mlp_err(e_ == hipErrorOutOfMemory ? PCH_ENOMEM : PCH_EDEVICE,                  \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

constexpr int H = 64;   // hidden width
constexpr int NIN = 7;  // input features
// parameter layout (floats): W1[7][64], b1[64], W2[64][64], b2[64], W3[64], b3
constexpr int OW1 = 0, OB1 = OW1 + NIN * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int NP = OB3 + 1;
static_assert(NP == PCH_MLP_NPARAM, "parameter count");
constexpr int kMlpBlock = 256;

__device__ __forceinline__ float bf16r(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ float softplusf(float y) { return y > 20.f ? y : log1pf(expf(y)); }
__device__ __forceinline__ float sigmoidf(float y) { return 1.f / (1.f + expf(-y)); }

// Forward (and optionally backward) over samples [0, n). grads (NP floats)
// and loss (1 float) are accumulated; pred (optional) receives predictions.
__global__ void __launch_bounds__(kMlpBlock) k_mlp(const float* __restrict__ P, const float* __restrict__ X,
                                                   const float* __restrict__ base, const float* __restrict__ target,
                                                   const float* __restrict__ scale, int64_t n, float inv_n,
                                                   float* __restrict__ pred, float* __restrict__ grads,
                                                   float* __restrict__ loss, int backward) {
  __shared__ float red[NP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = lane;
  // this lane's weights, BF16-rounded
  float w1[NIN], w2c[H], w2r[H];
  for (int i = 0; i < NIN; ++i) w1[i] = bf16r(P[OW1 + i * H + j]);
  for (int i = 0; i < H; ++i) {
    w2c[i] = bf16r(P[OW2 + i * H + j]);  // column j: z2_j = sum_i a1_i W2[i][j]
    w2r[i] = bf16r(P[OW2 + j * H + i]);  // row j: da1_j = sum_i dz2_i W2[j][i]
  }
  const float b1 = P[OB1 + j], b2 = P[OB2 + j], w3 = bf16r(P[OW3 + j]), b3 = P[OB3];
  float gw1[NIN] = {0}, gw2[H], gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
  for (int i = 0; i < H; ++i) gw2[i] = 0.f;
  const int64_t wid = (int64_t)blockIdx.x * (kMlpBlock / 64) + wave;
  const int64_t nw = (int64_t)gridDim.x * (kMlpBlock / 64);
  for (int64_t s = wid; s < n; s += nw) {
    float x[NIN];
    for (int i = 0; i < NIN; ++i) x[i] = bf16r(X[s * NIN + i]);
    float z1 = b1;
    for (int i = 0; i < NIN; ++i) z1 += x[i] * w1[i];
    const float a1 = bf16r(z1 > 0.f ? z1 : 0.f);
    float z2 = b2;
    for (int i = 0; i < H; ++i) z2 += __shfl(a1, i, 64) * w2c[i];
    const float a2 = bf16r(z2 > 0.f ? z2 : 0.f);
    float y = a2 * w3;
    for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
    y += b3;
    const float bs = base[s];
    const float d = bs * (1.f + softplusf(y));
    if (pred && lane == 0) pred[s] = d;
    if (!backward) continue;
    const float sc = scale[s];
    const float r = (d - target[s]) / sc;
    if (lane == 0) lsum += r * r * inv_n;
    const float dd = 2.f * r / sc * inv_n;
    const float dy = dd * bs * sigmoidf(y);
    gw3 += a2 * dy;
    if (lane == 0) gb3 += dy;
    const float dz2 = z2 > 0.f ? dy * w3 : 0.f;
    gb2 += dz2;
    float da1 = 0.f;
    for (int i = 0; i < H; ++i) {
      gw2[i] += __shfl(a1, i, 64) * dz2;  // dW2[i][j] = a1_i dz2_j
      da1 += __shfl(dz2, i, 64) * w2r[i];  // da1_j = sum_i W2[j][i] dz2_i
    }
    const float dz1 = z1 > 0.f ? da1 : 0.f;
    gb1 += dz1;
    for (int i = 0; i < NIN; ++i) gw1[i] += x[i] * dz1;
  }
  if (!backward) return;
  // block reduction in LDS, then one atomic per parameter
  for (int i = threadIdx.x; i < NP; i += kMlpBlock) red[i] = 0.f;
  __syncthreads();
  for (int w = 0; w < kMlpBlock / 64; ++w) {
    if (wave == w) {
      for (int i = 0; i < NIN; ++i) red[OW1 + i * H + j] += gw1[i];
      red[OB1 + j] += gb1;
      for (int i = 0; i < H; ++i) red[OW2 + i * H + j] += gw2[i];
      red[OB2 + j] += gb2;
      red[OW3 + j] += gw3;
      if (lane == 0) {
        red[OB3] += gb3;
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < NP; i += kMlpBlock) atomicAdd(&grads[i], red[i]);
  if (lane == 0) atomicAdd(loss, lsum);
}

// AdamW (decoupled weight decay on the weights, not the biases).
__global__ void k_adamw(float* P, float* M, float* V, float* G, int t, float lr, float wd, float b1, float b2,
                        float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.f - b1) * g;
  const float v = b2 * V[i] + (1.f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  const float mh = m / (1.f - powf(b1, (float)t));
  const float vh = v / (1.f - powf(b2, (float)t));
  const bool is_bias = (i >= OB1 && i < OW2) || (i >= OB2 && i < OW3) || i == OB3;
  float w = P[i];
  if (!is_bias) w -= lr * wd * w;
  w -= lr * mh / (sqrtf(vh) + eps);
  P[i] = w;
  G[i] = 0.f;
}

__global__ void k_zero(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Inference on the matrix cores (v_mfma_f32_16x16x16_bf16): each wavefront
// takes tiles of 16 samples. Every layer computes the transposed product
// Z^T = W^T A^T (rows: units, columns: samples), with the bias, ReLU and the
// BF16 rounding of its output applied per element. In the 16 x 16 result
// tile lane l holds rows 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16,
// which is exactly where the next product's B operand wants them, so the
// activations never leave the registers. The same arithmetic as k_mlp (BF16
// operands, FP32 accumulation), in another summation order.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// bits of bf16r(x)
__device__ __forceinline__ short bf16bits(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__global__ void __launch_bounds__(kMlpBlock) k_mlp_forward_mfma(const float* __restrict__ P,
                                                                const float* __restrict__ X,
                                                                const float* __restrict__ base, int64_t n,
                                                                float* __restrict__ pred) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;  // A operand row; B, D column (the sample of the tile)
  const int q = lane >> 4;  // rows (A: k) 4 q .. 4 q + 3
  // W1^T in 4 row blocks (units 16 mb + r, inputs 4 q + i, zero past the 7th)
  bf16x4 a1[4];
  // W2^T in 4 x 4 blocks (output unit 16 mb + r, input unit 16 kb + 4 q + i)
  bf16x4 a2[4][4];
  // per D-layout row (unit 16 mb + 4 q + i): biases and the last layer
  float b1v[4][4], b2v[4][4], w3v[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * q + i;
      a1[mb][i] = k < NIN ? bf16bits(P[OW1 + k * H + 16 * mb + r]) : (short)0;
      const int u = 16 * mb + 4 * q + i;
      b1v[mb][i] = P[OB1 + u];
      b2v[mb][i] = P[OB2 + u];
      w3v[mb][i] = bf16r(P[OW3 + u]);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) a2[mb][kb][i] = bf16bits(P[OW2 + (16 * kb + 4 * q + i) * H + 16 * mb + r]);
    }
  }
  const float b3 = P[OB3];
  const int64_t tiles = (n + 15) / 16;
  const int64_t wid = (int64_t)blockIdx.x * (kMlpBlock / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kMlpBlock / 64);
  for (int64_t t = wid; t < tiles; t += nw) {
    const int64_t s = t * 16 + r;
    const bool ok = s < n;
    bf16x4 xb;  // X^T: inputs 4 q + i of sample s
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * q + i;
      xb[i] = (ok && k < NIN) ? bf16bits(X[s * NIN + k]) : (short)0;
    }
    bf16x4 h1[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[mb], xb, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float zz = z[i] + b1v[mb][i];
        h1[mb][i] = bf16bits(zz > 0.f ? zz : 0.f);
      }
    }
    float y = 0.f;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[mb][kb], h1[kb], z, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float zz = z[i] + b2v[mb][i];
        y += bf16r(zz > 0.f ? zz : 0.f) * w3v[mb][i];
      }
    }
    y += __shfl_xor(y, 16, 64);
    y += __shfl_xor(y, 32, 64);
    y += b3;
    if (ok && q == 0) pred[s] = base[s] * (1.f + softplusf(y));
  }
}

// Features of every vertex for a source s: [(v - c) / R, (s - c) / R,
// |v - s| / R] and the chord |v - s|.
__global__ void k_features(const double* xyz, int64_t nv, int32_t s, double cx, double cy, double cz, double R,
                           float* X, float* base) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double px = xyz[3 * v], py = xyz[3 * v + 1], pz = xyz[3 * v + 2];
  const double sx = xyz[3 * (int64_t)s], sy = xyz[3 * (int64_t)s + 1], sz = xyz[3 * (int64_t)s + 2];
  const double dx = px - sx, dy = py - sy, dz = pz - sz;
  const double ch = sqrt(dx * dx + dy * dy + dz * dz);
  float* x = X + v * NIN;
  x[0] = (float)((px - cx) / R);
  x[1] = (float)((py - cy) / R);
  x[2] = (float)((pz - cz) / R);
  x[3] = (float)((sx - cx) / R);
  x[4] = (float)((sy - cy) / R);
  x[5] = (float)((sz - cz) / R);
  x[6] = (float)(ch / R);
  base[v] = (float)ch;
}

}  // namespace

struct pch_mlp_s {
  float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr, *loss = nullptr;
  int t = 0;
};

extern "C" {

pch_status pch_mlp_create(uint64_t seed, pch_mlp* out) {
  if (!out) return mlp_err(PCH_EINVAL, "null pointer argument");
  *out = nullptr;
  pch_mlp_s* m = new (std::nothrow) pch_mlp_s();
  if (!m) return mlp_err(PCH_ENOMEM, "host allocation failed");
  // He-uniform initialisation from a 64-bit LCG (MMIX constants)
  std::vector<float> p(NP, 0.f);
  uint64_t st = seed * 2862933555777941757ull + 3037000493ull;
  auto uni = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return ((st >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
  };
  for (int i = 0; i < NIN * H; ++i) p[OW1 + i] = (float)(uni() * std::sqrt(6.0 / NIN));
  for (int i = 0; i < H * H; ++i) p[OW2 + i] = (float)(uni() * std::sqrt(6.0 / H));
  for (int i = 0; i < H; ++i) p[OW3 + i] = (float)(uni() * std::sqrt(6.0 / H) * 0.1);
  hipError_t e;
  if ((e = hipMalloc(&m->P, NP * 4)) || (e = hipMalloc(&m->M, NP * 4)) || (e = hipMalloc(&m->V, NP * 4)) ||
      (e = hipMalloc(&m->G, NP * 4)) || (e = hipMalloc(&m->loss, 4))) {
    pch_mlp_destroy(m);
    return mlp_err(PCH_ENOMEM, hipGetErrorString(e));
  }
  if ((e = hipMemcpy(m->P, p.data(), NP * 4, hipMemcpyHostToDevice)) || (e = hipMemset(m->M, 0, NP * 4)) ||
      (e = hipMemset(m->V, 0, NP * 4)) || (e = hipMemset(m->G, 0, NP * 4))) {
    pch_mlp_destroy(m);
    return mlp_err(PCH_EDEVICE, hipGetErrorString(e));
  }
  *out = m;
  return PCH_OK;
}

void pch_mlp_destroy(pch_mlp m) {
  if (!m) return;
  (void)hipFree(m->P);
  (void)hipFree(m->M);
  (void)hipFree(m->V);
  (void)hipFree(m->G);
  (void)hipFree(m->loss);
  delete m;
}

pch_status pch_mlp_get_params(pch_mlp m, float* host) {
  if (!m || !host) return mlp_err(PCH_EINVAL, "null pointer argument");
  MLP_TRY(hipMemcpy(host, m->P, NP * 4, hipMemcpyDeviceToHost));
  return PCH_OK;
}

pch_status pch_mlp_set_params(pch_mlp m, const float* host) {
  if (!m || !host) return mlp_err(PCH_EINVAL, "null pointer argument");
  MLP_TRY(hipMemcpy(m->P, host, NP * 4, hipMemcpyHostToDevice));
  MLP_TRY(hipMemset(m->M, 0, NP * 4));
  MLP_TRY(hipMemset(m->V, 0, NP * 4));
  m->t = 0;
  return PCH_OK;
}

pch_status pch_mlp_features(const double* xyz, int64_t nv, int32_t source, const double* center, double radius,
                            float* feats, float* base, void* hip_stream) {
  if (!xyz || !center || !feats || !base) return mlp_err(PCH_EINVAL, "null pointer argument");
  if (nv < 1 || source < 0 || source >= nv || !(radius > 0.0)) return mlp_err(PCH_EINVAL, "bad feature argument");
  hipStream_t st = (hipStream_t)hip_stream;
  k_features<<<(unsigned)((nv + 255) / 256), 256, 0, st>>>(xyz, nv, source, center[0], center[1], center[2], radius,
                                                           feats, base);
  MLP_TRY(hipGetLastError());
  return PCH_OK;
}

pch_status pch_mlp_forward(pch_mlp m, const float* feats, const float* base, int64_t n, float* pred,
                           void* hip_stream) {
  if (!m || !feats || !base || !pred || n < 1) return mlp_err(PCH_EINVAL, "bad forward argument");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t tiles = (n + 15) / 16;  // one wavefront per 16-sample tile
  const unsigned blocks = (unsigned)std::min<int64_t>(std::max<int64_t>((tiles + 3) / 4, 1), 4096);
  k_mlp_forward_mfma<<<blocks, kMlpBlock, 0, st>>>(m->P, feats, base, n, pred);
  MLP_TRY(hipGetLastError());
  return PCH_OK;
}

pch_status pch_mlp_gradients(pch_mlp m, const float* feats, const float* base, const float* target, const float* scale,
                             int64_t n, float* grads_host, float* loss_host, void* hip_stream) {
  if (!m || !feats || !base || !target || !scale || n < 1) return mlp_err(PCH_EINVAL, "bad gradient argument");
  hipStream_t st = (hipStream_t)hip_stream;
  k_zero<<<(NP + 255) / 256, 256, 0, st>>>(m->G, NP);
  k_zero<<<1, 1, 0, st>>>(m->loss, 1);
  k_mlp<<<64, kMlpBlock, 0, st>>>(m->P, feats, base, target, scale, n, 1.f / (float)n, nullptr, m->G, m->loss, 1);
  MLP_TRY(hipGetLastError());
  if (grads_host) MLP_TRY(hipMemcpyAsync(grads_host, m->G, NP * 4, hipMemcpyDeviceToHost, st));
  if (loss_host) MLP_TRY(hipMemcpyAsync(loss_host, m->loss, 4, hipMemcpyDeviceToHost, st));
  MLP_TRY(hipStreamSynchronize(st));
  return PCH_OK;
}

pch_status pch_mlp_train_step(pch_mlp m, const float* feats, const float* base, const float* target,
                              const float* scale, int64_t n, float lr, float weight_decay, float* loss_host,
                              void* hip_stream) {
  if (!m || !feats || !base || !target || !scale || n < 1) return mlp_err(PCH_EINVAL, "bad training argument");
  hipStream_t st = (hipStream_t)hip_stream;
  k_zero<<<(NP + 255) / 256, 256, 0, st>>>(m->G, NP);
  k_zero<<<1, 1, 0, st>>>(m->loss, 1);
  k_mlp<<<64, kMlpBlock, 0, st>>>(m->P, feats, base, target, scale, n, 1.f / (float)n, nullptr, m->G, m->loss, 1);
  m->t += 1;
  k_adamw<<<(NP + 255) / 256, 256, 0, st>>>(m->P, m->M, m->V, m->G, m->t, lr, weight_decay, 0.9f, 0.999f, 1e-8f);
  MLP_TRY(hipGetLastError());
  if (loss_host) {
    MLP_TRY(hipMemcpyAsync(loss_host, m->loss, 4, hipMemcpyDeviceToHost, st));
    MLP_TRY(hipStreamSynchronize(st));
  }
  return PCH_OK;
}

}  // extern "C"
