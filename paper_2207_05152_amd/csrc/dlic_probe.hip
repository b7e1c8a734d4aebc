// Latencies of the primitive steps on the wavefront decoder's critical path
// (Section II-B, Preprocessor and rANS: each wavefront step waits for the one
// before it, so decode time is the number of steps times the chain of
// dependent operations one step needs).  Every probe runs a chain in which
// each operation takes the previous one's result, so the cycles per link are
// the operation's latency, not its throughput.  The decode bound the bench
// reports is built from these numbers.
//
// Probes (cycles per link of the chain, shader clock):
//   0  v_fma_f32                       6  DPP reduction over 16 lanes (4 steps)
//   1  v_mfma_f32_4x4x1f32 (C chain)   7  expf
//   2  v_mfma_f32_16x16x4f32 (C chain) 8  rANS decode update (one symbol)
//   3  LDS store then load, one wave   9  ballot + popcount
//   4  LDS load (address chase)        10 flag hand-off between two workgroups
//   5  LDS flag hand-off between two      through device memory (one way)
//      waves of a workgroup (one way)  11 v_readlane (VALU -> SGPR -> VALU)
// and at index 12 the shader clock in MHz (cycles against the 100 MHz
// real-time counter over probe 0).
#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

constexpr int PROBE_LINKS = 4096;   // links per chain
constexpr uint32_t PROBE_SPIN = 1u << 22;  // polls before a hand-off probe gives up

__device__ __forceinline__ unsigned long long probe_clock() {
  const unsigned long long c = clock64();
  asm volatile("" ::"s"(c));
  return c;
}

// One wave per probe (block of 64 threads) except the hand-offs.
__global__ __launch_bounds__(128) void latency_probe_kernel(int probe, float seed,
                                                            unsigned long long* out,
                                                            uint32_t* gflags) {
  __shared__ uint32_t s_buf[1024];
  __shared__ int s_flag[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) s_buf[i] = (uint32_t)((i * 37 + 11) & 1023);
  if (threadIdx.x < 2) s_flag[threadIdx.x] = -1;
  __syncthreads();
  unsigned long long c0 = 0, c1 = 0, r0 = 0, r1 = 0;
  float sink = 0.0f;
  uint32_t usink = 0;
  bool ok = true;
  if (probe == 0 && wave == 0) {
    float a = seed + lane * 1e-3f, w = 0.999f - lane * 1e-6f, b = 1e-4f;
    r0 = __builtin_amdgcn_s_memrealtime();
    c0 = probe_clock();
#pragma unroll 64
    for (int i = 0; i < PROBE_LINKS; ++i) a = __builtin_fmaf(w, a, b);
    asm volatile("" ::"v"(a));
    c1 = probe_clock();
    r1 = __builtin_amdgcn_s_memrealtime();
    sink = a;
  } else if (probe == 1 && wave == 0) {
    f4 acc = {seed, 0.0f, 0.0f, 0.0f};
    const float x = 1e-3f * lane, y = 0.5f;
    c0 = probe_clock();
#pragma unroll 32
    for (int i = 0; i < PROBE_LINKS; ++i) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(x, y, acc, 0, 0, 0);
    asm volatile("" ::"v"(acc));
    c1 = probe_clock();
    sink = acc[0] + acc[3];
  } else if (probe == 2 && wave == 0) {
    f4 acc = {seed, 0.0f, 0.0f, 0.0f};
    const float x = 1e-3f * lane, y = 0.5f;
    c0 = probe_clock();
#pragma unroll 32
    for (int i = 0; i < PROBE_LINKS / 4; ++i) acc = mfma_f32(x, y, acc);
    asm volatile("" ::"v"(acc));
    c1 = probe_clock();
    sink = acc[0] + acc[3];
  } else if (probe == 3 && wave == 0) {
    // store a value, load it back, the next store writes what was loaded
    uint32_t v = (uint32_t)lane;
    volatile uint32_t* p = s_buf + lane;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) {
      *p = v + 1u;
      v = *p;
    }
    c1 = probe_clock();
    usink = v;
  } else if (probe == 4 && wave == 0) {
    uint32_t idx = (uint32_t)lane;
    volatile uint32_t* p = s_buf;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) idx = p[idx & 1023u];
    c1 = probe_clock();
    usink = idx;
  } else if (probe == 5) {
    // wave 0 posts i, wave 1 answers i; a round trip is two hand-offs
    constexpr int N = PROBE_LINKS / 8;
    if (wave == 0) c0 = probe_clock();
    for (int i = 0; i < N && ok; ++i) {
      uint32_t spins = 0;
      if (wave == 0) {
        if (lane == 0) __hip_atomic_store(&s_flag[0], i, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        while (__hip_atomic_load(&s_flag[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != i)
          if (++spins > PROBE_SPIN) { ok = false; break; }
      } else {
        while (__hip_atomic_load(&s_flag[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != i)
          if (++spins > PROBE_SPIN) { ok = false; break; }
        if (lane == 0) __hip_atomic_store(&s_flag[1], i, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    if (wave == 0) c1 = probe_clock();
  } else if (probe == 6 && wave == 0) {
    uint32_t v = (uint32_t)(lane * 2654435761u);
    c0 = probe_clock();
#pragma unroll 8
    for (int i = 0; i < PROBE_LINKS / 16; ++i) {
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));
      v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));
      v += (uint32_t)lane;
    }
    c1 = probe_clock();
    usink = v;
  } else if (probe == 7 && wave == 0) {
    float a = seed * 1e-3f + lane * 1e-6f;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) a = expf(a) * 1e-3f;
    asm volatile("" ::"v"(a));
    c1 = probe_clock();
    sink = a;
  } else if (probe == 8 && wave == 0) {
    // x <- f * (x >> 16) + slot - c with slot = x & 0xFFFF and (c, f) taken
    // from the slot, renormalised as the decoder does
    uint32_t x = 0x12345678u + (uint32_t)lane;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) {
      const uint32_t slot = x & 0xFFFFu;
      const uint32_t c = slot & 0xFF00u, f = 256u;
      const uint32_t xd = __umul24(f, x >> 16) + slot - c;
      x = xd < RANS_L ? ((xd << 16) | (slot ^ 0x5A5Au)) : xd;
    }
    c1 = probe_clock();
    usink = x;
  } else if (probe == 9 && wave == 0) {
    uint32_t v = (uint32_t)lane;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) {
      const uint64_t m = __ballot((v & 1u) != 0u);
      v = v + (uint32_t)__popcll(m) + (uint32_t)lane;
    }
    c1 = probe_clock();
    usink = v;
  } else if (probe == 10 && wave == 0) {
    // block 0 posts i, block 1 answers i, through agent-scope atomics
    constexpr int N = PROBE_LINKS / 16;
    const int me = blockIdx.x;
    if (me == 0) c0 = probe_clock();
    for (int i = 1; i <= N && ok; ++i) {
      uint32_t spins = 0;
      if (me == 0) {
        if (lane == 0) __hip_atomic_store(&gflags[0], (uint32_t)i, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(&gflags[16], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != (uint32_t)i)
          if (++spins > PROBE_SPIN) { ok = false; break; }
      } else {
        while (__hip_atomic_load(&gflags[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != (uint32_t)i)
          if (++spins > PROBE_SPIN) { ok = false; break; }
        if (lane == 0) __hip_atomic_store(&gflags[16], (uint32_t)i, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (me == 0) c1 = probe_clock();
  } else if (probe == 11 && wave == 0) {
    float a = seed + lane;
    c0 = probe_clock();
#pragma unroll 16
    for (int i = 0; i < PROBE_LINKS / 4; ++i) {
      const float s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a), i & 63));
      a = a * 0.5f + s;
    }
    asm volatile("" ::"v"(a));
    c1 = probe_clock();
    sink = a;
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = c1 - c0;
    out[1] = r1 - r0;
    out[2] = ok ? 1ull : 0ull;
    out[3] = (unsigned long long)__float_as_uint(sink) ^ usink;  // keeps the chains live
  }
}

int probe_links(int probe) {
  switch (probe) {
    case 0: case 1: return PROBE_LINKS;
    case 2: case 3: case 4: case 7: case 8: case 9: case 11: return PROBE_LINKS / 4;
    case 5: return 2 * (PROBE_LINKS / 8);
    case 6: return PROBE_LINKS / 16;
    case 10: return 2 * (PROBE_LINKS / 16);
    default: return 1;
  }
}

void launch_latency_probe(int probe, unsigned long long* out, uint32_t* gflags, hipStream_t s) {
  const int blocks = probe == 10 ? 2 : 1;
  const int threads = probe == 5 ? 128 : 64;
  hipLaunchKernelGGL(latency_probe_kernel, dim3(blocks), dim3(threads), 0, s, probe, 0.25f, out,
                     gflags);
}

}  // namespace dlic
