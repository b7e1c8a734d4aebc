// Device helpers shared by the kernels of the six-layer softmax network
// (Section II-B, Neural Network Architecture) for 8-bit samples (256 output
// levels) and 12-bit ones (4096 levels, Section IV-C, Higher Bit Depth):
// the operand-order weight layout, the window gather, the table rule's last
// step, the stream header check and the grid barrier of the cooperative
// decoders.
#pragma once

#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

// Layer i of a k -> H x 5 -> nout net: inputs padded to 32 for layer 1.
__host__ __device__ constexpr int deep_in(int i, int H) { return i == 0 ? 32 : H; }
__host__ __device__ constexpr int deep_out(int i, int H, int nout) {
  return i == DEEP_LAYERS - 1 ? nout : H;
}
// bf16x8 operands (64 per (tile, k-step)) before layer i
__host__ __device__ constexpr long long deep_off(int i, int H, int nout) {
  long long o = 0;
  for (int l = 0; l < i; ++l) o += (long long)(deep_out(l, H, nout) / 16) * (deep_in(l, H) / 32) * 64;
  return o;
}

// Input index of slot e of lane group q in k-step s of layer i (-1: zero slot).
__device__ __forceinline__ int deep_slot_input(int i, int s, int q, int e, int k_in) {
  if (i == 0) return 4 * e + q < k_in ? 4 * e + q : -1;
  return 32 * s + 16 * (e >> 2) + 4 * q + (e & 3);
}

// F(v) = v + min(M', floor(C M')) with M' = 2^16 - (number of levels).
__device__ __forceinline__ uint32_t deep_F(int v, float C, uint32_t mp) {
  const float t = floorf(C * (float)mp);
  const uint32_t qv = t >= (float)mp ? mp : (uint32_t)t;
  return (uint32_t)v + qv;
}

// A sample as a level index: 12-bit samples above 4095 (invalid input, which
// the encoder reports) read the last entry instead of past the table.
__device__ __forceinline__ int deep_level(uint8_t v) { return v; }
__device__ __forceinline__ int deep_level(uint16_t v) { return v < 4096 ? (int)v : 4095; }

// Layer-1 operand of lane group q for pixel (z, y, x) (y, the row in slice z
// of the stacked image): slot e holds window value 4 e + q scaled to [-1, 1]
// by the table sc (one entry per level), 0 outside the slice (or below the
// first slice) and past the window.  Values 0..11 are the pixel's own slice,
// 12..20 the slice below, row by row.  Samples must be valid levels.
template <int KIN, typename PX>
__device__ __forceinline__ bf16x8 deep_features(const float* __restrict__ sc, const PX* img, int H,
                                                int W, int ws, int z, int y, int x, bool valid,
                                                int q) {
  const __bf16 zero = (__bf16)0.0f;
  bf16x8 o = {zero, zero, zero, zero, zero, zero, zero, zero};
  const PX* sl = img + (long long)z * H * W;
#pragma unroll
  for (int e = 0; e < (KIN + 3) / 4; ++e) {
    const int k = 4 * e + q;
    float f = 0.0f;
    if (k < K_IN) {
      const int yy = y + nb_dy(k), xx = x + nb_dx(k);
      if (valid && yy >= 0 && xx >= 0 && xx < W) f = sc[deep_level(sl[(long long)yy * W + xx])];
    } else if (k < KIN) {
      const int j = k - K_IN;
      const int yy = y + ws - 3 + j / 3, xx = x + j % 3 - 1;
      if (valid && z > 0 && yy >= 0 && yy < H && xx >= 0 && xx < W)
        f = sc[deep_level(sl[(long long)(yy - H) * W + xx])];
    }
    o[e] = (__bf16)f;
  }
  return o;
}

// The five hidden layers of one 16-pixel tile (one wave).  Lane l holds the
// layer-1 operand of pixel l % 16 (features 4 e + l / 16 in slot e) and gets
// the output layer's operand a[s] (slot e: neuron 32 s + 16 (e / 4) +
// 4 (l / 16) + e % 4 of that pixel, as BF16).  Bias-seeded FP32 accumulation,
// one chain of MFMAs per neuron tile in k order, ReLU, then BF16.
// w: the operand-order weights from layer 1 on; bias(l): layer l's biases
// (global memory, or copies in LDS).
template <int H, class Bias>
__device__ __forceinline__ void deep_hidden_at(const bf16x8* w, Bias bias, const bf16x8 x,
                                               bf16x8 (&a)[H / 32]) {
  constexpr int NT = H / 16, NK = H / 32;
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int q = lane >> 4;
  float h[NT][4];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const float* b = bias(0) + 16 * nt + 4 * q;
    f4 acc = {b[0], b[1], b[2], b[3]};
    acc = mfma_bf16(w[nt * 64 + lane], x, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) h[nt][r] = relu(acc[r]);
  }
  w += NT * 64;
#pragma unroll 1
  for (int li = 1; li < DEEP_LAYERS - 1; ++li) {
#pragma unroll
    for (int s = 0; s < NK; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) a[s][e] = (__bf16)h[2 * s + (e >> 2)][e & 3];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const float* b = bias(li) + 16 * nt + 4 * q;
      f4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
      for (int s = 0; s < NK; ++s) acc = mfma_bf16(w[(nt * NK + s) * 64 + lane], a[s], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) h[nt][r] = relu(acc[r]);
    }
    w += NT * NK * 64;
  }
#pragma unroll
  for (int s = 0; s < NK; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) a[s][e] = (__bf16)h[2 * s + (e >> 2)][e & 3];
}

template <int H>
__device__ __forceinline__ void deep_hidden(const DeepNetArgs& d, const bf16x8 x,
                                            bf16x8 (&a)[H / 32]) {
  deep_hidden_at<H>(reinterpret_cast<const bf16x8*>(d.wop), [&](int l) { return d.b[l]; }, x, a);
}

// Test hook: a seeded pause of up to max_cycles shader cycles (in 64-cycle
// sleeps) at one point of one wave, so that the decoder's hand-offs between
// workgroups meet in other orders.  No-op when max_cycles is 0.
__device__ __forceinline__ void deep_delay(uint32_t seed, uint32_t max_cycles, uint32_t site,
                                           uint32_t who, uint32_t step) {
  if (max_cycles == 0) return;
  uint32_t h = seed ^ (site * 0x9E3779B1u) ^ (who * 0x85EBCA77u) ^ (step * 0xC2B2AE3Du);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  const uint32_t n = (h % max_cycles) >> 6;
  for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(1);
}

__device__ __forceinline__ uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
__device__ __forceinline__ uint32_t rd16(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8);
}

// Grid barrier over a cooperative launch: a counter that only grows (barrier
// k completes when it reaches k * gridDim.x).  One thread per workgroup
// arrives with a release add and polls with plain (relaxed) loads, then takes
// one acquire fence: an acquire per poll would invalidate the cache the
// network's weights are read through on every spin.  The wait is bounded;
// giving up sets the abort flag, which ends every workgroup's walk.
__device__ __forceinline__ bool grid_sync(unsigned* bar, int* abort_flag, unsigned& k,
                                          uint32_t limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ++k;
    const unsigned target = k * gridDim.x;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > limit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  // uniform by construction, so loops that end on it keep their barriers whole
  return __builtin_amdgcn_readfirstlane(s_ok) != 0;
}

// 3: the stream does not fit the geometry (or is damaged); 4: another model.
__device__ __forceinline__ int deep_check_header(const DeepDecArgs& a) {
  const int GT = a.vg.Z * a.G;
  if (a.n_bytes < (unsigned long long)(HEADER_BYTES + 4LL * GT)) return 3;
  const uint8_t* b = a.bits;
  if (b[0] != 'D' || b[1] != 'L' || b[2] != 'I' || b[3] != 'C') return 3;
  if (rd16(b + 4) != 1u || rd16(b + 6) != (uint32_t)a.hf.flags) return 3;
  if (rd32(b + 8) != (uint32_t)(a.vg.Z * a.H) || rd32(b + 12) != (uint32_t)a.W) return 3;
  if (b[19] != SKEW || b[24] != PROB_BITS) return 3;
  if (b[25] != (uint8_t)a.L || rd16(b + 26) != (uint32_t)GT) return 3;
  const uint64_t fp = (uint64_t)rd32(b + 28) | ((uint64_t)rd32(b + 32) << 32);
  if (b[16] != (uint8_t)a.hf.k_in || b[17] != 0 || b[18] != (uint8_t)a.hf.dtype ||
      rd16(b + 20) != (uint32_t)a.hf.h1 || rd16(b + 22) != (uint32_t)a.hf.h2 ||
      fp != a.hf.fingerprint)
    return 4;
  return 0;
}

}  // namespace dlic
