// Wavefront decoder of the DLIC hot path (Section II-A, Fig. 2 right;
// Section II-B, Preprocessor and rANS; Fig. 1 right).
//
// One persistent workgroup per group of rows.  In wavefront step t every
// pixel (y, x) with x + 3y == t has all 12 window pixels decoded (the
// up-right neighbour (y-1, x+2) finished in step t-1), so the workgroup
//   1. receives the two rows above its strip from the upstream group,
//   2. runs the network on all its active pixels (16-pixel MFMA tiles over
//      the four waves) and the mixture head,
//   3. decodes the active pixels lane by lane in canonical order with wave 0
//      (slot -> symbol by halving search on the FP32 table rule -> state
//      update -> ballot renormalisation from an LDS ring of the stream),
//   4. publishes the values just decoded in its two bottom rows.
// Records carry data and validity in one 32-bit word (bit 31 valid, bits
// 8..15 row r1-2, bits 0..7 row r1-1), written and read with agent-scope
// atomics, so no fences are needed.  A workgroup only ever waits for the
// one before it, which the dispatcher started earlier, and every wait is
// bounded by a spin limit, so the grid always drains.
#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

constexpr int RING_MASK = DEC_RING - 1;
constexpr int RING_HALF = DEC_RING / 2;
constexpr int REFILL_PER_THREAD = RING_HALF / 256;

__device__ __forceinline__ int floordiv(int a, int b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__device__ __forceinline__ uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
__device__ __forceinline__ uint32_t rd_u16(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8);
}

// Header check; returns 0 or a status code.  Every workgroup computes the
// same answer, so a bad stream makes all of them stop before any wait.
__device__ int check_header(const DecArgs& a) {
  if (a.n_bytes < (unsigned long long)(HEADER_BYTES + 4LL * a.G)) return 3;
  const uint8_t* b = a.bits;
  if (b[0] != 'D' || b[1] != 'L' || b[2] != 'I' || b[3] != 'C') return 3;
  if (rd_u16(b + 4) != 1u) return 3;
  if (rd_u32(b + 8) != (uint32_t)a.H || rd_u32(b + 12) != (uint32_t)a.W) return 3;
  if (b[16] != K_IN || b[17] != N_MIX || b[19] != SKEW || b[24] != PROB_BITS) return 3;
  if (b[25] != (uint8_t)a.L || rd_u16(b + 26) != (uint32_t)a.G) return 3;
  if (a.check_model) {
    const uint64_t fp = (uint64_t)rd_u32(b + 28) | ((uint64_t)rd_u32(b + 32) << 32);
    if (b[18] != (uint8_t)a.hf.dtype || rd_u16(b + 20) != (uint32_t)a.hf.h1 ||
        rd_u16(b + 22) != (uint32_t)a.hf.h2 || fp != a.hf.fingerprint)
      return 4;
  }
  return 0;
}

template <int H1, int H2, bool TABLES>
__global__ __launch_bounds__(256) void wavefront_decode_kernel(const Consts* __restrict__ K,
                                                               DevModel m, DecArgs a) {
  __shared__ float2 s_sd[LUT_N];
  __shared__ float s_beta[257];
  __shared__ float s_scale[256];
  __shared__ __attribute__((aligned(16))) float s_par[DEC_RMAX * 16];
  __shared__ uint8_t s_ring[(DEC_RMAX + 2) * 16];
  __shared__ uint16_t s_words[DEC_RING];
  __shared__ unsigned long long s_total, s_before;
  __shared__ int s_err;
  __shared__ uint32_t s_P;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4;
  const int g = blockIdx.x;
  const int H = a.H, W = a.W, G = a.G, L = a.L;

  if (!TABLES) {
    for (int i = tid; i < LUT_N; i += 256) s_sd[i] = K->sd[i];
    for (int i = tid; i < 257; i += 256) s_beta[i] = K->beta[i];
    s_scale[tid] = K->scale[tid];
  }
  if (tid == 0) {
    s_err = check_header(a);
    s_total = 0;
    s_before = 0;
  }
  __syncthreads();
  if (s_err == 0) {
    for (int i = tid; i < G; i += 256) {
      const unsigned long long c = rd_u32(a.bits + HEADER_BYTES + 4 * i);
      atomicAdd(&s_total, c);
      if (i < g) atomicAdd(&s_before, c);
    }
  }
  __syncthreads();
  if (tid == 0 && s_err == 0 &&
      (unsigned long long)(HEADER_BYTES + 4LL * G) + 2ull * s_total != a.n_bytes)
    s_err = 3;
  __syncthreads();
  if (s_err != 0) {
    if (tid == 0) atomicMax(a.status, s_err);
    return;
  }

  const int r0 = group_row(g, H, G), r1 = group_row(g + 1, H, G);
  const int R = r1 - r0;
  const int J = (R + L - 1) / L;
  const int t_first = SKEW * r0, t_last = SKEW * (r1 - 1) + W - 1;
  const int up_last = (g > 0) ? SKEW * (r0 - 1) + W - 1 : -1;
  const int t_begin = (g > 0) ? t_first - 2 * SKEW + 1 : t_first;
  const uint32_t n_words = rd_u32(a.bits + HEADER_BYTES + 4 * g);
  const uint16_t* gw = reinterpret_cast<const uint16_t*>(
      a.bits + HEADER_BYTES + 4LL * G + 2ull * s_before);
  bool bad = n_words < 2u * (uint32_t)L;
  bool over = false, timeout = false;

  NetF32<H1, H2> net;
  if (!TABLES) net.load(m, lane);

  // stream ring: first DEC_RING words; lane states from the stream head
  uint32_t E = bad ? 0u : min(n_words, (uint32_t)DEC_RING);
  for (uint32_t i = tid; i < E; i += 256) s_words[i] = gw[i];
  uint32_t x = RANS_L;
  if (wave == 0 && lane < L && !bad) x = (uint32_t)gw[2 * lane] | ((uint32_t)gw[2 * lane + 1] << 16);
  if (tid == 0) s_P = 2u * (uint32_t)L;
  __syncthreads();

  uint32_t* up_rec = a.rec + (long long)(g - 1) * a.T;
  uint32_t* my_rec = a.rec + (long long)g * a.T;

  for (int t = t_begin; t <= t_last; ++t) {
    // (1) rows r0-2 and r0-1 from the upstream group (its step t-1)
    if (tid == 0 && g > 0 && t - 1 <= up_last && !timeout) {
      uint32_t v = __hip_atomic_load(up_rec + (t - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t spins = 0;
      while (!(v >> 31)) {
        if (++spins > a.spin_limit) {
          timeout = true;
          v = 0x80000000u;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(up_rec + (t - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const int c1 = (t - 1) - SKEW * (r0 - 1);  // row r0-1
      const int c2 = (t - 1) - SKEW * (r0 - 2);  // row r0-2
      if (c1 >= 0 && c1 < W) s_ring[1 * 16 + (c1 & 15)] = (uint8_t)(v & 0xFF);
      if (c2 >= 0 && c2 < W) s_ring[0 * 16 + (c2 & 15)] = (uint8_t)((v >> 8) & 0xFF);
    }
    __syncthreads();

    // stream refill: fetch the next half ring now, store it after the coder
    const uint32_t P0 = s_P;
    const bool refill = !bad && E < n_words && E - P0 <= (uint32_t)RING_HALF;
    uint16_t pre[REFILL_PER_THREAD];
    if (refill) {
#pragma unroll
      for (int i = 0; i < REFILL_PER_THREAD; ++i) {
        const uint32_t pos = E + (uint32_t)(i * 256 + tid);
        pre[i] = pos < n_words ? gw[pos] : (uint16_t)0;
      }
    }

    const int ylo = max(r0, floordiv(t - W, SKEW) + 1);
    const int yhi = min(r1 - 1, floordiv(t, SKEW));
    const int n_act = yhi - ylo + 1;

    if (!TABLES) {
      // (2) network on the active pixels, raw outputs to s_par
      for (int tile = wave; tile * 16 < n_act; tile += 4) {
        const int i = tile * 16 + (lane & 15);
        const int y = ylo + i;
        const bool valid = i < n_act;
        const int xc = t - SKEW * y;
        float fk[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int k = 4 * kk + q;
          const int yy = y + nb_dy(k), xx = xc + nb_dx(k);
          fk[kk] = (valid && yy >= 0 && xx >= 0 && xx < W)
                       ? s_scale[s_ring[(yy - r0 + 2) * 16 + (xx & 15)]]
                       : 0.0f;
        }
        const f4 o = net.run(fk[0], fk[1], fk[2]);
        if (valid) *reinterpret_cast<f4*>(&s_par[(y - r0) * 16 + 4 * q]) = o;
      }
      __syncthreads();
      for (int i = tid; i < n_act; i += 256) {
        float* pp = &s_par[(ylo + i - r0) * 16];
        float o[N_OUT];
#pragma unroll
        for (int k = 0; k < N_OUT; ++k) o[k] = pp[k];
        const Mix mix = mixture_head(o);
#pragma unroll
        for (int k = 0; k < N_MIX; ++k) {
          pp[k] = mix.pi[k];
          pp[N_MIX + k] = mix.mu[k];
          pp[2 * N_MIX + k] = mix.is[k];
        }
      }
      __syncthreads();
    }

    // (3) coder: one sub-round per block of L rows, canonical order
    if (wave == 0 && n_act > 0) {
      uint32_t P = P0;
      for (int j = 0; j < J; ++j) {
        const int rr = j * L + lane;
        const int y = r0 + rr;
        const bool act = lane < L && rr < R && y >= ylo && y <= yhi;
        const int xc = t - SKEW * y;
        const uint32_t slot = x & 0xFFFFu;
        int v = 0;
        uint32_t c = 0, f = 1;
        if (TABLES) {
          uint32_t ti = act ? a.tidx[(long long)y * W + xc] : 0u;
          if (ti >= (uint32_t)a.n_tables) {
            bad = bad || act;
            ti = 0;
          }
          const uint32_t* tab = a.tables + (long long)ti * 257;
          find_symbol(slot, [&](int lv) { return tab[lv]; }, v, c, f);
        } else {
          const float* pp = &s_par[(act ? rr : 0) * 16];
          Mix mix;
#pragma unroll
          for (int k = 0; k < N_MIX; ++k) {
            mix.pi[k] = pp[k];
            mix.mu[k] = pp[N_MIX + k];
            mix.is[k] = pp[2 * N_MIX + k];
          }
          find_symbol(slot, [&](int lv) { return cdf_F(lv, mix, s_sd, s_beta); }, v, c, f);
        }
        if (act) x = f * (x >> 16) + slot - c;
        P = rans_dec_renorm(x, act && !bad, P, n_words,
                            [&](uint32_t pos) { return (uint32_t)s_words[pos & RING_MASK]; }, over);
        if (act) {
          s_ring[(rr + 2) * 16 + (xc & 15)] = (uint8_t)v;
          a.img[(long long)y * W + xc] = (uint8_t)v;
        }
      }
      if (lane == 0) s_P = P;
    }
    // (4) publish this step's values of rows r1-2 and r1-1 for the next group
    if (tid == 0 && t >= t_first && g + 1 < G) {
      const int c1 = t - SKEW * (r1 - 1), c2 = t - SKEW * (r1 - 2);
      uint32_t rv = 0x80000000u;
      if (c1 >= 0 && c1 < W) rv |= (uint32_t)s_ring[(R - 1 + 2) * 16 + (c1 & 15)];
      if (c2 >= 0 && c2 < W) rv |= (uint32_t)s_ring[(R - 2 + 2) * 16 + (c2 & 15)] << 8;
      __hip_atomic_store(my_rec + t, rv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (refill) {
#pragma unroll
      for (int i = 0; i < REFILL_PER_THREAD; ++i)
        s_words[(E + (uint32_t)(i * 256 + tid)) & RING_MASK] = pre[i];
      E = min(n_words, E + (uint32_t)RING_HALF);
    }
  }

  // every lane back at the initial state and every word consumed
  if (wave == 0) {
    const bool lane_bad = (lane < L) && (x != RANS_L);
    const bool any_bad = __ballot(lane_bad || over || bad) != 0ull;
    if (lane == 0) {
      const uint32_t P = s_P;
      if (any_bad || P != n_words) atomicMax(a.status, 3);
    }
  }
  if (tid == 0 && timeout) atomicMax(a.status, 7);
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

template <int H1, int H2, bool TB>
static void launch_decode_t(const Consts* K, const DevModel& m, const DecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((wavefront_decode_kernel<H1, H2, TB>), dim3(a.G), dim3(256), 0, s, K, m, a);
}

bool launch_decode(int width, bool tables_mode, const Consts* K, const DevModel& m,
                   const DecArgs& a, hipStream_t s) {
  if (tables_mode) {
    launch_decode_t<32, 32, true>(K, m, a, s);
    return true;
  }
  switch (width) {
    case 32: launch_decode_t<32, 32, false>(K, m, a, s); return true;
    case 64: launch_decode_t<64, 64, false>(K, m, a, s); return true;
    default: return false;
  }
}

}  // namespace dlic
