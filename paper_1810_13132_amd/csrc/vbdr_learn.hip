// Learned cardinality estimator beside the HyperLogLog estimate of Alg. 5:
// a 67 -> 64 -> 64 -> 1 GELU MLP over a host's register histogram, the pool's
// register histogram and ln(g/m), predicting ln(1 + n).
//   - inference: bf16 weights and inputs on the matrix cores
//     (v_mfma_f32_16x16x32_bf16, fp32 accumulation), 16 hosts per wave, with
//     the plain estimate as fallback outside the training envelope;
//   - training: fp32 per-sample backpropagation with the weights in LDS,
//     gradients reduced with atomics, then an Adam update.
// Parameter vector (fp32, 8577): W1 (64 x 67), b1, W2 (64 x 64), b2, w3, b3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "vbdr_internal.h"

using namespace vbdr;

namespace {

constexpr int kIn = 67, kHid = 64, kInPad = 96;
constexpr int kOffW1 = 0, kOffB1 = kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid, kParams = kOffB3 + 1;
static_assert(kParams == 8577, "parameter layout");

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct MlpDev {
  uint16_t w1[kHid * kInPad];  // bf16, K zero-padded to 96
  uint16_t w2p[kHid * kHid];   // bf16, W2 with its columns in layer 2's K order (l2_unit)
  float b1[kHid], b2[kHid], w3[kHid], b3;  // w3 holds bf16-rounded values
  float env_lo[kIn], env_hi[kIn];
  int has_env;
  float plain_above;  // hosts whose plain estimate is at least this keep it (+inf: none)
};

// float -> bf16 bits, round to nearest even (host and device).
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// GELU of the inference kernel: erf by Abramowitz & Stegun 7.1.26 (absolute
// error <= 1.5e-7, below one fp32 ulp of the GELU's 1 + erf term), without
// the branches of erff, so that a lane's 16 activations need few registers.
__device__ __forceinline__ float gelu_inf(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * z);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = 1.0f - poly * __expf(-z * z);  // erf(|x| / sqrt 2)
  return 0.5f * x * (1.0f + (x < 0.0f ? -e : e));
}

// ------------------------------------------------------------ features
// fp32 features of nh hosts from the histogram pass: [h][67].
__global__ __launch_bounds__(256) void k_features(uint32_t nh, uint32_t parts, const uint32_t* __restrict__ hws,
                                                  const unsigned long long* __restrict__ hist, uint32_t g, uint32_t m,
                                                  float* __restrict__ feats) {
  const uint32_t h = blockIdx.x * 256 + threadIdx.x;
  if (h >= nh) return;
  float* f = feats + (uint64_t)h * kIn;
  for (int r = 0; r < kBins; ++r) {
    uint32_t c = 0;
    for (uint32_t x = 0; x < parts; ++x) c += hws[((uint64_t)x * kLearnChunk + h) * kBins + r];
    f[r] = (float)((double)c / (double)g);
    f[kBins + r] = (float)((double)hist[r] / (double)m);
  }
  f[2 * kBins] = (float)log((double)g / (double)m);
}

// ----------------------------------------------------------- inference
// A wave estimates a tile of 16 hosts.  Both layers run transposed on the
// matrix cores, hidden units as rows and hosts as columns, so that the
// accumulator of layer 1 (lane l: units 16 nt + 4 (l/16) + i of host l%16) is
// already the B operand of layer 2 once the K order of layer 2 is permuted to
// match (W2's columns are stored permuted, w2p).  Layer 2's outputs meet w3 in
// the same lanes; three lane exchanges give the tile's 16 sums.  The plain
// estimate is computed (in parallel over the tile's hosts) only for hosts that
// fall back.
constexpr int kInfBlock = 256;
constexpr int kInfWaves = kInfBlock / 64;
constexpr int kHistStride = 36;  // words per histogram row (16-byte aligned rows)

// Unit of layer 1 held in K slot (ks, q, i) of layer 2's operands.
__host__ __device__ inline int l2_unit(int ks, int q, int i) { return 16 * (2 * ks + (i >> 2)) + 4 * q + (i & 3); }

// bf16x8 of eight fp32 values.
__device__ __forceinline__ bf16x8 pack8(const float* v) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (short)f2bf(v[i]);
  return r;
}

// DIRECT: each wave gathers its 16 hosts' registers itself (pools whose
// registers are cache resident) into an LDS histogram per host; otherwise
// the histograms come from a histogram pass (hws, summed over parts).  Five
// waves per SIMD (at most 102 registers) keep enough gathers in flight.
template <bool DIRECT>
__global__ __launch_bounds__(kInfBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_learned(uint32_t nh, uint32_t parts, const uint32_t* __restrict__ hws,
                                                       const uint32_t* __restrict__ hosts,
                                                       const uint32_t* __restrict__ s1g, const uint8_t* __restrict__ reg,
                                                       const unsigned long long* __restrict__ hist, uint32_t g,
                                                       uint32_t m, const MlpDev* __restrict__ mlp,
                                                       float* __restrict__ out, uint8_t* __restrict__ used_fallback) {
  extern __shared__ uint32_t s1_lds[];
  __shared__ __attribute__((aligned(16))) uint16_t sw1[kHid * kInPad];
  __shared__ __attribute__((aligned(16))) uint16_t sw2[kHid * kHid];
  __shared__ __attribute__((aligned(16))) uint32_t lh[kInfWaves][16 * kHistStride];
  __shared__ __attribute__((aligned(16))) uint16_t sconst[kInPad];  // bf16 features 33..95 (pool, ln(g/m), 0)
  __shared__ float sb1[kHid], sb2[kHid], sw3[kHid], senv_lo[kBins], senv_hi[kBins];
  __shared__ int spool_bad;
  __shared__ double sem;
  for (int i = threadIdx.x; i < kHid * kInPad / 8; i += kInfBlock)
    reinterpret_cast<uint4*>(sw1)[i] = reinterpret_cast<const uint4*>(mlp->w1)[i];
  for (int i = threadIdx.x; i < kHid * kHid / 8; i += kInfBlock)
    reinterpret_cast<uint4*>(sw2)[i] = reinterpret_cast<const uint4*>(mlp->w2p)[i];
  for (int i = threadIdx.x; i < kInfWaves * 16 * kHistStride; i += kInfBlock) (&lh[0][0])[i] = 0;
  if (threadIdx.x < kHid) {
    sb1[threadIdx.x] = mlp->b1[threadIdx.x];
    sb2[threadIdx.x] = mlp->b2[threadIdx.x];
    sw3[threadIdx.x] = mlp->w3[threadIdx.x];
  }
  if (threadIdx.x < kBins) {
    senv_lo[threadIdx.x] = mlp->has_env ? mlp->env_lo[threadIdx.x] : -INFINITY;
    senv_hi[threadIdx.x] = mlp->has_env ? mlp->env_hi[threadIdx.x] : INFINITY;
  }
  if (threadIdx.x == 0) {
    sem = pool_estimate(hist, (double)m);
    spool_bad = 0;
  }
  if constexpr (DIRECT)
    for (uint32_t i = threadIdx.x; i < g; i += kInfBlock) s1_lds[i] = s1g[i];
  __syncthreads();
  if (threadIdx.x < kInPad) {
    const int c = threadIdx.x;
    float v = 0.0f;
    if (c >= kBins && c < 2 * kBins) v = (float)((double)hist[c - kBins] / (double)m);
    if (c == 2 * kBins) v = (float)log((double)g / (double)m);
    sconst[c] = f2bf(v);
    if (c >= kBins && c < kIn && mlp->has_env && !(v >= mlp->env_lo[c] && v <= mlp->env_hi[c])) atomicOr(&spool_bad, 1);
  }
  __syncthreads();
  const double Em = sem;
  const int pool_bad = spool_bad;
  const float inv_g = 1.0f / (float)g;  // g is a power of two: c * inv_g == c / g exactly
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, q = lane >> 4;
  uint32_t* H = lh[wave];
  const uint32_t ntiles = (nh + 15) / 16;
  for (uint32_t tile = blockIdx.x * kInfWaves + wave; tile < ntiles; tile += gridDim.x * kInfWaves) {
    // An offset opaque to the compiler: the weights, biases and envelope are
    // read from LDS per tile instead of being pinned in ~150 registers across
    // the loop, which would cut the waves available to hide gather latency.
    uint32_t woff = 0;
    asm volatile("" : "+v"(woff));
    // 1. register histograms of the tile's hosts
    if constexpr (DIRECT) {
      for (int row = 0; row < 16; ++row) {
        const uint32_t h = tile * 16 + row;
        if (h >= nh) break;
        const uint32_t kmix = mm3_key(hosts[h]);
        uint32_t* my = H + row * kHistStride;
        for (uint32_t i0 = lane; i0 < g; i0 += 64 * 4) {
          uint32_t r[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + 64u * u;
            r[u] = i < g ? (uint32_t)reg[reduce_m(mm3_seeded(kmix, s1_lds[i]), m)] : 255u;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (r[u] != 255u) atomicAdd(&my[r[u]], 1u);
        }
      }
    } else {
      for (int e = lane; e < 16 * kBins; e += 64) {
        const int row = e / kBins, r = e - row * kBins;
        const uint32_t h = tile * 16 + row;
        uint32_t c = 0;
        if (h < nh)
          for (uint32_t x = 0; x < parts; ++x) c += hws[((uint64_t)x * kLearnChunk + h) * kBins + r];
        H[row * kHistStride + r] = c;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // 2. features of host `col`: this lane's bins 8q..8q+7 (and bin 32 for q = 0)
    uint32_t c8[8];
    {
      const uint4 lo = *reinterpret_cast<const uint4*>(H + col * kHistStride + 8 * q);
      const uint4 hi = *reinterpret_cast<const uint4*>(H + col * kHistStride + 8 * q + 4);
      c8[0] = lo.x, c8[1] = lo.y, c8[2] = lo.z, c8[3] = lo.w, c8[4] = hi.x, c8[5] = hi.y, c8[6] = hi.z, c8[7] = hi.w;
    }
    const uint32_t c32 = q == 0 ? H[col * kHistStride + 32] : 0u;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < 8; ++i) H[col * kHistStride + 8 * q + i] = 0;  // clean for the next tile
    if (q == 0) H[col * kHistStride + 32] = 0;
    float f[8];
    int bad = 0;
    uint64_t U = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = 8 * q + i;
      f[i] = (float)c8[i] * inv_g;
      bad |= !(f[i] >= senv_lo[woff + r] && f[i] <= senv_hi[woff + r]);
      U += (uint64_t)c8[i] << (32 - r);
    }
    const float f32 = (float)c32 * inv_g;
    if (q == 0) {
      bad |= !(f32 >= senv_lo[woff + 32] && f32 <= senv_hi[woff + 32]);
      U += (uint64_t)c32;
    }
    const bf16x8 x0 = pack8(f);
    bf16x8 x1 = *reinterpret_cast<const bf16x8*>(sconst + woff + 32 + 8 * q);
    if (q == 0) x1[0] = (short)f2bf(f32);
    const bf16x8 x2 = *reinterpret_cast<const bf16x8*>(sconst + woff + 64 + 8 * q);
    // 3. layer 1, transposed: Z1^T (64 x 16) = W1 (64 x 96) X^T
    f32x4 z1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* wr = sw1 + woff + (nt * 16 + col) * kInPad + 8 * q;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(wr), x0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(wr + 32), x1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(wr + 64), x2, acc, 0, 0, 0);
      z1[nt] = acc;
    }
    // 4. H1 = bf16(gelu(Z1 + b1)) in place as layer 2's B operand
    bf16x8 hb[2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) hb[nt >> 1][4 * (nt & 1) + i] = (short)f2bf(gelu_inf(z1[nt][i] + sb1[woff + 16 * nt + 4 * q + i]));
    // 5. layer 2, transposed, and the output unit
    float part = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const uint16_t* wr = sw2 + woff + (nt * 16 + col) * kHid + 8 * q;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(wr), hb[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(wr + 32), hb[1], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = woff + 16 * nt + 4 * q + i;
        part += gelu_inf(acc[i] + sb2[u]) * sw3[u];
      }
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    U += __shfl_xor(U, 16);
    U += __shfl_xor(U, 32);
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    // 6. outputs of the tile, lane col of the first row group
    const uint32_t h = tile * 16 + col;
    if (q == 0 && h < nh) {
      float est = expf(part + mlp->b3) - 1.0f;
      int fb = bad | pool_bad;
      if (!isfinite(est)) fb = 1;
      const float above = mlp->plain_above;
      if (fb || above < INFINITY) {
        const double Es = hll_estimate(U, c8[0], (double)g);
        const double n = noise_removed(Es, Em, (double)m, (double)g);
        const float plain = (float)(n > 0.0 ? n : 0.0);
        if (!fb && plain >= above) fb = 2;  // a large count: the plain estimate is kept
        if (fb) est = plain;
      }
      out[h] = est > 0.0f ? est : 0.0f;
      if (used_fallback) used_fallback[h] = (uint8_t)fb;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------ training
constexpr int kW2Pad = kHid + 1;  // padded LDS row of W2 (bank conflicts)

// One wave per block; lane j owns hidden unit j of both layers: its W1 row
// and gradient rows live in registers, W2 (read by rows forward and by
// columns backward) in LDS.  Each block runs spb samples, then adds its
// gradient of the batch-mean loss into grads with atomics.
__global__ __launch_bounds__(64) void k_train_grad(const float* __restrict__ params, const float* __restrict__ feats,
                                                   const float* __restrict__ targets, uint32_t B, uint32_t spb,
                                                   float* __restrict__ grads, float* __restrict__ loss) {
  __shared__ float w2[kHid * kW2Pad];
  __shared__ float xs[kIn], h1s[kHid], dz2s[kHid];
  const int j = threadIdx.x;
  float w1r[kIn], g1r[kIn], g2r[kHid];
#pragma unroll
  for (int k = 0; k < kIn; ++k) {
    w1r[k] = params[kOffW1 + j * kIn + k];
    g1r[k] = 0.f;
  }
#pragma unroll
  for (int k = 0; k < kHid; ++k) g2r[k] = 0.f;
  for (int i = j; i < kHid * kHid; i += 64) w2[(i / kHid) * kW2Pad + i % kHid] = params[kOffW2 + i];
  const float b1 = params[kOffB1 + j], b2 = params[kOffB2 + j], w3 = params[kOffW3 + j], b3 = params[kOffB3];
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
  __syncthreads();
  const uint32_t s0 = blockIdx.x * spb, s1 = min(B, s0 + spb);
  const float inv_b = 1.0f / (float)B;
  for (uint32_t s = s0; s < s1; ++s) {
    for (int i = j; i < kIn; i += 64) xs[i] = feats[(uint64_t)s * kIn + i];
    __syncthreads();
    float z1 = b1;
#pragma unroll
    for (int k = 0; k < kIn; ++k) z1 += w1r[k] * xs[k];
    h1s[j] = gelu(z1);
    __syncthreads();
    float z2 = b2;
#pragma unroll
    for (int k = 0; k < kHid; ++k) z2 += w2[j * kW2Pad + k] * h1s[k];
    const float h2 = gelu(z2);
    float y = w3 * h2;
    for (int off = 32; off > 0; off >>= 1) y += __shfl_xor(y, off);
    y += b3;
    const float r = y - targets[s];
    const float dy = 2.0f * r * inv_b;
    lsum += r * r * inv_b;
    gw3 += dy * h2;
    gb3 += dy;
    const float dz2 = dy * w3 * gelu_grad(z2);
    dz2s[j] = dz2;
    gb2 += dz2;
#pragma unroll
    for (int k = 0; k < kHid; ++k) g2r[k] += dz2 * h1s[k];
    __syncthreads();
    float dh1 = 0.f;
#pragma unroll
    for (int i = 0; i < kHid; ++i) dh1 += w2[i * kW2Pad + j] * dz2s[i];
    const float dz1 = dh1 * gelu_grad(z1);
    gb1 += dz1;
#pragma unroll
    for (int k = 0; k < kIn; ++k) g1r[k] += dz1 * xs[k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kIn; ++k) atomicAdd(&grads[kOffW1 + j * kIn + k], g1r[k]);
#pragma unroll
  for (int k = 0; k < kHid; ++k) atomicAdd(&grads[kOffW2 + j * kHid + k], g2r[k]);
  atomicAdd(&grads[kOffB1 + j], gb1);
  atomicAdd(&grads[kOffB2 + j], gb2);
  atomicAdd(&grads[kOffW3 + j], gw3);
  if (j == 0) {
    atomicAdd(&grads[kOffB3], gb3);
    if (loss) atomicAdd(loss, lsum);
  }
}

__global__ void k_adam(float* __restrict__ params, float* __restrict__ grads, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float beta1, float beta2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float gr = grads[i];
  const float a = beta1 * m1[i] + (1.0f - beta1) * gr;
  const float v = beta2 * m2[i] + (1.0f - beta2) * gr * gr;
  m1[i] = a;
  m2[i] = v;
  params[i] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
  grads[i] = 0.f;
}

__global__ void k_zero_f32(float* __restrict__ p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

struct vbdr_mlp {
  int device;
  MlpDev* dev;
};

struct vbdr_trainer {
  int device;
  float *params, *grads, *m1, *m2;
  uint64_t step;
  float lr, beta1, beta2, eps;
};

extern "C" {

int vbdr_mlp_create(const float* params_host, const float* env_lo, const float* env_hi, vbdr_mlp** out) {
  if (!params_host || !out) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if ((env_lo == nullptr) != (env_hi == nullptr)) return vbdr_fail(VBDR_EINVAL, "give both envelope bounds or none");
  *out = nullptr;
  std::vector<uint8_t> buf(sizeof(MlpDev), 0);
  MlpDev* h = reinterpret_cast<MlpDev*>(buf.data());
  for (int j = 0; j < kHid; ++j) {
    for (int k = 0; k < kIn; ++k) h->w1[j * kInPad + k] = f2bf(params_host[kOffW1 + j * kIn + k]);
    for (int ks = 0; ks < 2; ++ks)
      for (int q = 0; q < 4; ++q)
        for (int i = 0; i < 8; ++i)
          h->w2p[j * kHid + 32 * ks + 8 * q + i] = f2bf(params_host[kOffW2 + j * kHid + l2_unit(ks, q, i)]);
    h->b1[j] = params_host[kOffB1 + j];
    h->b2[j] = params_host[kOffB2 + j];
    h->w3[j] = bf2f(f2bf(params_host[kOffW3 + j]));
  }
  h->b3 = params_host[kOffB3];
  h->has_env = env_lo != nullptr;
  h->plain_above = INFINITY;
  for (int k = 0; k < kIn; ++k) {
    h->env_lo[k] = env_lo ? env_lo[k] : 0.f;
    h->env_hi[k] = env_hi ? env_hi[k] : 0.f;
  }
  vbdr_mlp* mlp = new (std::nothrow) vbdr_mlp();
  if (!mlp) return vbdr_fail(VBDR_ENOMEM, "host allocation failed");
  if (hipGetDevice(&mlp->device) != hipSuccess || vbdr_malloc(&mlp->dev, sizeof(MlpDev)) != hipSuccess) {
    delete mlp;
    return vbdr_fail(VBDR_ENOMEM, "device allocation of the MLP failed");
  }
  if (hipMemcpy(mlp->dev, h, sizeof(MlpDev), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(mlp->dev);
    delete mlp;
    return vbdr_fail(VBDR_EHIP, "upload of the MLP failed");
  }
  *out = mlp;
  return VBDR_OK;
}

int vbdr_mlp_set_plain_above(vbdr_mlp* mlp, float threshold) {
  if (!mlp) return vbdr_fail(VBDR_EINVAL, "mlp is NULL");
  if (!(threshold > 0.0f)) return vbdr_fail(VBDR_EINVAL, "threshold must be positive (INFINITY: never)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != mlp->device)
    return vbdr_fail(VBDR_EINVAL, "the network lives on device %d, not the current one", mlp->device);
  if (hipMemcpy(reinterpret_cast<uint8_t*>(mlp->dev) + offsetof(MlpDev, plain_above), &threshold, sizeof(float),
                hipMemcpyHostToDevice) != hipSuccess)
    return vbdr_fail(VBDR_EHIP, "upload of the threshold failed");
  return VBDR_OK;
}

void vbdr_mlp_destroy(vbdr_mlp* mlp) {
  if (!mlp) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(mlp->dev);
  delete mlp;
}

int vbdr_features(vbdr_sketch* sk, const uint32_t* hosts_dev, uint64_t n_hosts, float* feats_dev, void* stream) {
  if (!sk) return vbdr_fail(VBDR_EINVAL, "sketch is NULL");
  if (n_hosts == 0) return VBDR_OK;
  if (!hosts_dev || !feats_dev) return vbdr_fail(VBDR_EINVAL, "hosts_dev and feats_dev must not be NULL");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (uint64_t c = 0; c < n_hosts; c += kLearnChunk) {
    const uint32_t nh = (uint32_t)(n_hosts - c < kLearnChunk ? n_hosts - c : kLearnChunk);
    if (int rc = vbdr_hist_pass(sk, hosts_dev + c, nh, st)) return rc;
    hipLaunchKernelGGL(k_features, dim3((nh + 255) / 256), dim3(256), 0, st, nh, (uint32_t)sk->parts, sk->hist_ws,
                       sk->hist, sk->g, (uint32_t)sk->m, feats_dev + c * kIn);
    VBDR_LAUNCHED("k_features");
  }
  return VBDR_OK;
}

int vbdr_estimate_learned(vbdr_sketch* sk, const vbdr_mlp* mlp, const uint32_t* hosts_dev, uint64_t n_hosts,
                          float* out_dev, uint8_t* used_fallback_dev, void* stream) {
  if (!sk || !mlp) return vbdr_fail(VBDR_EINVAL, "sketch and mlp must not be NULL");
  if (n_hosts == 0) return VBDR_OK;
  if (!hosts_dev || !out_dev) return vbdr_fail(VBDR_EINVAL, "hosts_dev and out_dev must not be NULL");
  if (mlp->device != sk->device) return vbdr_fail(VBDR_EINVAL, "mlp and sketch live on different devices");
  if (int rc = vbdr_check_device(sk)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (sk->parts == 1 && sk->g <= kStageMaxG && n_hosts < (1ull << 32)) {
    // registers cache resident: one fused launch, gathers feed the MLP tile directly
    const uint32_t nh = (uint32_t)n_hosts;
    const uint32_t tiles = (uint32_t)((n_hosts + 15) / 16);
    const uint32_t want = (tiles + kInfWaves - 1) / kInfWaves;
    const uint32_t cap = (uint32_t)sk->n_cu * 8;
    hipLaunchKernelGGL(k_learned<true>, dim3(want < cap ? want : cap), dim3(kInfBlock), (size_t)sk->g * 4, st, nh, 1u,
                       (const uint32_t*)nullptr, hosts_dev, sk->s1, sk->reg, sk->hist, sk->g, (uint32_t)sk->m,
                       mlp->dev, out_dev, used_fallback_dev);
    VBDR_LAUNCHED("k_learned(direct)");
    return VBDR_OK;
  }
  for (uint64_t c = 0; c < n_hosts; c += kLearnChunk) {
    const uint32_t nh = (uint32_t)(n_hosts - c < kLearnChunk ? n_hosts - c : kLearnChunk);
    if (int rc = vbdr_hist_pass(sk, hosts_dev + c, nh, st)) return rc;
    const uint32_t tiles = (nh + 15) / 16;
    const uint32_t want = (tiles + kInfWaves - 1) / kInfWaves;
    const uint32_t cap = (uint32_t)sk->n_cu * 4;
    hipLaunchKernelGGL(k_learned<false>, dim3(want < cap ? want : cap), dim3(kInfBlock), 0, st, nh,
                       (uint32_t)sk->parts, sk->hist_ws, (const uint32_t*)nullptr, (const uint32_t*)nullptr,
                       (const uint8_t*)nullptr, sk->hist, sk->g, (uint32_t)sk->m, mlp->dev, out_dev + c,
                       used_fallback_dev ? used_fallback_dev + c : nullptr);
    VBDR_LAUNCHED("k_learned");
  }
  return VBDR_OK;
}

int vbdr_trainer_create(const float* params_host, float lr, vbdr_trainer** out) {
  if (!params_host || !out) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (!(lr > 0.f)) return vbdr_fail(VBDR_EINVAL, "learning rate must be positive");
  *out = nullptr;
  vbdr_trainer* tr = new (std::nothrow) vbdr_trainer();
  if (!tr) return vbdr_fail(VBDR_ENOMEM, "host allocation failed");
  std::memset(tr, 0, sizeof(*tr));
  tr->lr = lr, tr->beta1 = 0.9f, tr->beta2 = 0.999f, tr->eps = 1e-8f;
  const size_t bytes = kParams * sizeof(float);
  if (hipGetDevice(&tr->device) != hipSuccess || vbdr_malloc(&tr->params, bytes) != hipSuccess ||
      vbdr_malloc(&tr->grads, bytes) != hipSuccess || vbdr_malloc(&tr->m1, bytes) != hipSuccess ||
      vbdr_malloc(&tr->m2, bytes) != hipSuccess) {
    vbdr_trainer_destroy(tr);
    return vbdr_fail(VBDR_ENOMEM, "device allocation of the trainer failed");
  }
  const uint32_t grid = (kParams + 255) / 256;
  hipLaunchKernelGGL(k_zero_f32, dim3(grid), dim3(256), 0, nullptr, tr->grads, (uint32_t)kParams);
  hipLaunchKernelGGL(k_zero_f32, dim3(grid), dim3(256), 0, nullptr, tr->m1, (uint32_t)kParams);
  hipLaunchKernelGGL(k_zero_f32, dim3(grid), dim3(256), 0, nullptr, tr->m2, (uint32_t)kParams);
  if (hipGetLastError() != hipSuccess || hipMemcpy(tr->params, params_host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    vbdr_trainer_destroy(tr);
    return vbdr_fail(VBDR_EHIP, "trainer initialisation failed");
  }
  *out = tr;
  return VBDR_OK;
}

void vbdr_trainer_destroy(vbdr_trainer* tr) {
  if (!tr) return;
  (void)hipDeviceSynchronize();
  if (tr->params) (void)hipFree(tr->params);
  if (tr->grads) (void)hipFree(tr->grads);
  if (tr->m1) (void)hipFree(tr->m1);
  if (tr->m2) (void)hipFree(tr->m2);
  delete tr;
}

int vbdr_trainer_set_lr(vbdr_trainer* tr, float lr) {
  if (!tr || !(lr > 0.f)) return vbdr_fail(VBDR_EINVAL, "bad trainer or learning rate");
  tr->lr = lr;
  return VBDR_OK;
}

int vbdr_trainer_grad(vbdr_trainer* tr, const float* feats_dev, const float* targets_dev, uint64_t n, float* grads_out_dev,
                      float* loss_dev, void* stream) {
  if (!tr || !feats_dev || !targets_dev || !grads_out_dev) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  if (n == 0 || n >= (1ull << 31)) return vbdr_fail(VBDR_EINVAL, "batch size out of range");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint32_t spb = 32;
  const uint32_t grid = (uint32_t)((n + spb - 1) / spb);
  hipLaunchKernelGGL(k_train_grad, dim3(grid), dim3(64), 0, st, tr->params, feats_dev, targets_dev, (uint32_t)n, spb,
                     grads_out_dev, loss_dev);
  VBDR_LAUNCHED("k_train_grad");
  return VBDR_OK;
}

int vbdr_trainer_step(vbdr_trainer* tr, const float* feats_dev, const float* targets_dev, uint64_t n, float* loss_dev,
                      void* stream) {
  if (int rc = vbdr_trainer_grad(tr, feats_dev, targets_dev, n, tr ? tr->grads : nullptr, loss_dev, stream)) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  tr->step++;
  const float bc1 = 1.0f - powf(tr->beta1, (float)tr->step), bc2 = 1.0f - powf(tr->beta2, (float)tr->step);
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, tr->params, tr->grads, tr->m1, tr->m2,
                     tr->lr, tr->beta1, tr->beta2, tr->eps, bc1, bc2);
  VBDR_LAUNCHED("k_adam");
  return VBDR_OK;
}

int vbdr_trainer_params(vbdr_trainer* tr, float* params_host, void* stream) {
  if (!tr || !params_host) return vbdr_fail(VBDR_EINVAL, "NULL argument");
  VBDR_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  VBDR_HIP(hipMemcpy(params_host, tr->params, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return VBDR_OK;
}

}  // extern "C"
