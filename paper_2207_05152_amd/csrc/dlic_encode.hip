// Encoder kernels of the DLIC hot path (Section II-A, Fig. 2 left; Section II-B).
//
// Phase A, density_kernel: every pixel's window goes through the network as
// one big matrix (Section II-B, Preprocessor: one row per window), 16-pixel
// MFMA tiles, 64 pixels per wave; the head and the FP32 table rule then give
// the pixel's interval (c, f) in its table.  All pixels are independent.
//
// Phase B, rans_encode_kernel: rANS is last-in first-out, so each group's
// symbols are coded walking the canonical wavefront order backwards; one
// wave per group, one lane per coder instance (Section II-B, rANS), words
// placed by ballot rank so the stream reads forward in decoding order.
//
// pack_kernel: header, per-group word counts and the streams, concatenated.
#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

// Stride (floats) of one pixel's outputs in the per-wave LDS staging area.
constexpr int O_STRIDE = 16;

// LDS of the density kernels: logistic table, bin edges, scaled grey levels,
// per-wave output staging and the net's layer-2 weights when they live in LDS.
template <class Net>
struct DensityLds {
  float2 sd[LUT_N];
  float beta[257];
  float scale[256];
  __attribute__((aligned(16))) float o[4][64 * O_STRIDE];
  __attribute__((aligned(16))) char w2[Net::LDS_BYTES > 0 ? Net::LDS_BYTES : 16];
};

template <class Net>
__device__ __forceinline__ void density_prologue(const Consts* K, const DevModel& m,
                                                 DensityLds<Net>& S, Net& net) {
  const int tid = threadIdx.x;
  for (int i = tid; i < LUT_N; i += 256) S.sd[i] = K->sd[i];
  for (int i = tid; i < 257; i += 256) S.beta[i] = K->beta[i];
  S.scale[tid] = K->scale[tid];
  Net::stage(m, S.w2, tid, 256);
  __syncthreads();
  net.load(m, tid & 63);
}

// One block of 256 consecutive raster pixels of an image: four 16-pixel MFMA
// tiles per wave, then one lane per pixel for the head and the table rule.
template <class Net>
__device__ __forceinline__ void density_block(const Net& net, DensityLds<Net>& S,
                                              const uint8_t* __restrict__ img, int W, long long n,
                                              long long blk, uint32_t* __restrict__ cf,
                                              float* __restrict__ out15,
                                              uint32_t* __restrict__ tables) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4;
  const long long base = blk * 256 + wave * 64;
#pragma unroll 1
  for (int tile = 0; tile < 4; ++tile) {
    const long long p = base + tile * 16 + (lane & 15);
    float fk[3] = {0.0f, 0.0f, 0.0f};
    if (p < n) {
      const int y = (int)(p / W), x = (int)(p - (long long)y * W);
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const int k = 4 * kk + q;
        const int yy = y + nb_dy(k), xx = x + nb_dx(k);
        if (yy >= 0 && xx >= 0 && xx < W) fk[kk] = S.scale[img[(long long)yy * W + xx]];
      }
    }
    const f4 o = net.run(fk[0], fk[1], fk[2], S.w2);
    *reinterpret_cast<f4*>(&S.o[wave][(tile * 16 + (lane & 15)) * O_STRIDE + 4 * q]) = o;
  }
  __syncthreads();
  const long long p = base + lane;
  if (p < n) {
    float o[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const f4 v = *reinterpret_cast<const f4*>(&S.o[wave][lane * O_STRIDE + 4 * i]);
      o[4 * i] = v[0];
      o[4 * i + 1] = v[1];
      o[4 * i + 2] = v[2];
      o[4 * i + 3] = v[3];
    }
    const Mix mix = mixture_head(o);
    const int v = img[p];
    const uint32_t Flo = cdf_F(v, mix, S.sd, S.beta);
    const uint32_t Fhi = cdf_F(v + 1, mix, S.sd, S.beta);
    if (cf) cf[p] = Flo | ((Fhi - Flo - 1u) << 16);
    if (out15) {
#pragma unroll
      for (int k = 0; k < N_OUT; ++k) out15[p * N_OUT + k] = o[k];
    }
    if (tables) {
      for (int lv = 0; lv <= 256; ++lv) tables[p * 257 + lv] = cdf_F(lv, mix, S.sd, S.beta);
    }
  }
  __syncthreads();
}

template <class Net>
__global__ __launch_bounds__(256) void density_kernel(const Consts* __restrict__ K, DevModel m,
                                                      const uint8_t* __restrict__ img, int H,
                                                      int W, uint32_t* __restrict__ cf,
                                                      float* __restrict__ out15,
                                                      uint32_t* __restrict__ tables) {
  __shared__ DensityLds<Net> S;
  Net net;
  density_prologue(K, m, S, net);
  const long long n = (long long)H * W;
  const long long n_blk = (n + 255) / 256;
  for (long long blk = blockIdx.x; blk < n_blk; blk += gridDim.x)
    density_block(net, S, img, W, n, blk, cf, out15, tables);
}

// Batched form: blocks of all images in one grid-stride loop; block b belongs
// to the last image whose first block is <= b.
__device__ __forceinline__ int batch_image_of_block(const BatchArgs& b, int blk) {
  int lo = 0, hi = b.n_img - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.images[mid].blk_off <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class Net>
__global__ __launch_bounds__(256) void batch_density_kernel(const Consts* __restrict__ K,
                                                            DevModel m, BatchArgs b) {
  __shared__ DensityLds<Net> S;
  Net net;
  density_prologue(K, m, S, net);
  for (int blk = blockIdx.x; blk < b.n_blk; blk += gridDim.x) {
    const BatchImage im = b.images[batch_image_of_block(b, blk)];
    density_block(net, S, b.pix_in + im.px_off, im.W, (long long)im.H * im.W,
                  (long long)(blk - im.blk_off), b.cf + im.px_off, nullptr, nullptr);
  }
}

// Largest hidden activations of the FP32 net over every pixel of an image:
// amax[0] (layer 1) and amax[1] (layer 2), non-negative after ReLU, so their
// bit patterns order like unsigned integers.
template <int H>
__global__ __launch_bounds__(256) void activation_range_kernel(const Consts* __restrict__ K,
                                                               DevModel m,
                                                               const uint8_t* __restrict__ img,
                                                               int Hh, int W, float* amax) {
  using Net = NetF32<H, (H > 64)>;
  __shared__ DensityLds<Net> S;
  Net net;
  density_prologue(K, m, S, net);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4;
  const long long n = (long long)Hh * W;
  float mx1 = 0.0f, mx2 = 0.0f;
  for (long long blk = blockIdx.x; blk * 256 < n; blk += gridDim.x) {
#pragma unroll 1
    for (int tile = 0; tile < 4; ++tile) {
      const long long p = blk * 256 + wave * 64 + tile * 16 + (lane & 15);
      float fk[3] = {0.0f, 0.0f, 0.0f};
      if (p < n) {
        const int y = (int)(p / W), x = (int)(p - (long long)y * W);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int k = 4 * kk + q;
          const int yy = y + nb_dy(k), xx = x + nb_dx(k);
          if (yy >= 0 && xx >= 0 && xx < W) fk[kk] = S.scale[img[(long long)yy * W + xx]];
        }
      }
      float a1, a2;
      net.hidden_max(fk[0], fk[1], fk[2], S.w2, a1, a2);
      // lanes past the last pixel ran the all-dummy window: leave them out
      if (p < n) {
        mx1 = fmaxf(mx1, a1);
        mx2 = fmaxf(mx2, a2);
      }
    }
  }
  atomicMax((unsigned*)&amax[0], __float_as_uint(mx1));
  atomicMax((unsigned*)&amax[1], __float_as_uint(mx2));
}

bool launch_activation_range(int width, const Consts* K, const DevModel& m, const uint8_t* img,
                             int H, int W, float* amax, int grid, hipStream_t s) {
  switch (width) {
    case 32:
      hipLaunchKernelGGL(activation_range_kernel<32>, dim3(grid), dim3(256), 0, s, K, m, img, H, W, amax);
      return true;
    case 64:
      hipLaunchKernelGGL(activation_range_kernel<64>, dim3(grid), dim3(256), 0, s, K, m, img, H, W, amax);
      return true;
    case 128:
      hipLaunchKernelGGL(activation_range_kernel<128>, dim3(grid), dim3(256), 0, s, K, m, img, H, W, amax);
      return true;
    default: return false;
  }
}

// Test hook: the encoder's 16-pixel FP32 form of the 12-H-H-15 net (H = 64
// or 128) and the decoder's 4-pixel form (NetF32x4) on the same caller-given
// feature rows.  One wave per block, 16 rows per tile.  In the 4-pixel form,
// rows 4s + j with j >= lanes get all-zero features (the decoder's idle tile
// rows).
template <int H>
__global__ __launch_bounds__(64) void net_forms_kernel(DevModel m, const float* __restrict__ feats,
                                                      long long n, int lanes,
                                                      float* __restrict__ out16,
                                                      float* __restrict__ out4) {
  using Net16 = NetF32<H>;
  // the 4-pixel form with layer-2 weights in LDS, and at H = 64 also with them
  // in registers: out4 holds the LDS form's outputs, NaN where the two differ
  using Net4 = NetF32x4<H>;
  using Net4R = NetF32x4<H, (H == 64)>;
  __shared__ __attribute__((aligned(16))) char w16[Net16::LDS_BYTES > 0 ? Net16::LDS_BYTES : 16];
  __shared__ __attribute__((aligned(16))) char w4[Net4::LDS_BYTES > 0 ? Net4::LDS_BYTES : 16];
  __shared__ __attribute__((aligned(16))) float xs[Net4::SCRATCH_FLOATS];
  const int lane = threadIdx.x, q = lane >> 4, p = lane & 15;
  Net16::stage(m, w16, lane, 64);
  Net4::stage(m, w4, lane, 64);
  __syncthreads();
  Net16 a;
  a.load(m, lane);
  Net4 b;
  b.load(m, lane);
  b.xs = xs;
  Net4R br;
  br.load(m, lane);
  br.xs = xs;
  for (long long tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
    const long long r16 = tile * 16 + p;
    float f[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) f[kk] = feats[r16 * K_IN + 4 * kk + q];
    const f4 o = a.run(f[0], f[1], f[2], w16);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * q + r < N_OUT) out16[r16 * N_OUT + 4 * q + r] = o[r];
#pragma unroll 1
    for (int sub = 0; sub < 4; ++sub) {
      const long long r4 = tile * 16 + 4 * sub + (p & 3);
      const bool live = p < 4 && p < lanes;
      float g[3];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) g[kk] = live ? feats[r4 * K_IN + 4 * kk + q] : 0.0f;
      f4 o4 = b.run(g[0], g[1], g[2], w4);
      if constexpr (H == 64) {
        const f4 o4r = br.run(g[0], g[1], g[2], w4);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (__float_as_uint(o4r[r]) != __float_as_uint(o4[r])) o4[r] = __builtin_nanf("");
      }
      if (p < 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * q + r < N_OUT) out4[r4 * N_OUT + 4 * q + r] = o4[r];
      }
    }
  }
}

bool launch_net_forms(int width, const DevModel& m, const float* feats, long long n, int lanes,
                      float* out16, float* out4, hipStream_t s) {
  long long tiles = n / 16;
  const int grid = (int)(tiles < 1024 ? (tiles > 0 ? tiles : 1) : 1024);
  if (width == 64)
    hipLaunchKernelGGL(net_forms_kernel<64>, dim3(grid), dim3(64), 0, s, m, feats, n, lanes, out16,
                       out4);
  else if (width == 128)
    hipLaunchKernelGGL(net_forms_kernel<128>, dim3(grid), dim3(64), 0, s, m, feats, n, lanes,
                       out16, out4);
  else
    return false;
  return true;
}

constexpr int ENC_CHUNK = 32;   // wavefront steps staged in LDS per chunk
constexpr int ENC_BATCH = 8;    // sub-rounds read from LDS ahead of coding
constexpr int ENC_STAGERS = 192;  // threads of waves 1..3
constexpr int ENC_ROWS = DEC_RMAX + 64;  // J * L <= rows + L - 1 rows per step, padded
constexpr int ENC_SLOTS = ENC_CHUNK * ENC_ROWS;
constexpr int ENC_PER_STAGER = (ENC_SLOTS + ENC_STAGERS - 1) / ENC_STAGERS;

// One group's rANS walk (one workgroup of 4 waves).  Wave 0 codes; while it
// walks one chunk of 32 steps in reverse canonical order from LDS, waves 1..3
// stage the next chunk's intervals, all of a thread's loads issued before any
// LDS store so their latencies overlap.  They store them in the order the
// coder reads them: sub-round i of the chunk's reverse walk at [i * L, i * L
// + L), inactive slots (rows past the group, steps before its first) marked,
// so the coder's reads are one running index.  Words go below the top of the
// group's scratch slice (cap_g = R*W + 2L words, the worst case), so a stream
// is contiguous at [cap_g - count, cap_g).  With S strips per group the walk
// takes the group's strips from the last to the first, each from its last
// step back, the lanes' states carrying from strip to strip.
struct EncStrip {
  int r0, R, J, t_first, t_last, n_chunks;
};

__device__ __forceinline__ EncStrip enc_strip(int b, int H, int W, int GS, int L) {
  EncStrip st;
  st.r0 = group_row(b, H, GS);
  st.R = group_row(b + 1, H, GS) - st.r0;
  st.J = (st.R + L - 1) / L;
  st.t_first = SKEW * st.r0;
  st.t_last = SKEW * (st.r0 + st.R - 1) + W - 1;
  st.n_chunks = st.R > 0 ? (st.t_last - st.t_first + ENC_CHUNK) / ENC_CHUNK : 0;
  return st;
}

__device__ __forceinline__ void rans_encode_group(uint32_t (*s_cf)[ENC_SLOTS],
                                                  const uint32_t* __restrict__ cf, int H, int W,
                                                  int G, int L, int S, int g,
                                                  uint16_t* __restrict__ words,
                                                  uint32_t* __restrict__ counts) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int GS = G * S;
  int before, rows;
  group_span(g, H, G, S, before, rows);
  const long long cap = (long long)rows * W + 2LL * L;
  uint16_t* out = words + (long long)before * W + 2LL * L * g;
  int n_chunks = 0;
  for (int s = 0; s < S; ++s) n_chunks += enc_strip(s * G + g, H, W, GS, L).n_chunks;
  // chunk k of the walk: its strip and its index c within the strip
  auto locate = [&](int k, int& c) {
    EncStrip st{};
    for (int s = S - 1; s >= 0; --s) {
      st = enc_strip(s * G + g, H, W, GS, L);
      if (k < st.n_chunks) break;
      k -= st.n_chunks;
    }
    c = k;
    return st;
  };

  // chunk c of a strip holds steps [t_last - 32c - 31, t_last - 32c]; the
  // interval of step t_lo + k, row j * L + l of the strip goes to slot
  // i * L + l with i = (31 - k) * J + (J - 1 - j), its sub-round in the
  // reverse walk
  auto stage = [&](int kc, uint32_t* buf, int first, int stride) {
    int c;
    const EncStrip st = locate(kc, c);
    const int r0 = st.r0, R = st.R, J = st.J, t_first = st.t_first;
    const int JL = J * L;  // <= R + L - 1 <= ENC_ROWS - 1
    const int t_lo = st.t_last - ENC_CHUNK * c - (ENC_CHUNK - 1);
    uint32_t v[ENC_PER_STAGER];
#pragma unroll
    for (int i = 0; i < ENC_PER_STAGER; ++i) {
      const int idx = first + i * stride;
      const int rr = idx / ENC_CHUNK, k = idx - rr * ENC_CHUNK;
      const int y = r0 + rr, t = t_lo + k, x = t - SKEW * y;
      v[i] = (idx < JL * ENC_CHUNK && rr < R && t >= t_first && x >= 0 && x < W)
                 ? cf[(long long)y * W + x]
                 : INACTIVE;
    }
#pragma unroll
    for (int i = 0; i < ENC_PER_STAGER; ++i) {
      const int idx = first + i * stride;
      if (idx < JL * ENC_CHUNK) {
        const int rr = idx / ENC_CHUNK, k = idx - rr * ENC_CHUNK;
        const int jb = rr / L, l = rr - jb * L;
        buf[((ENC_CHUNK - 1 - k) * J + (J - 1 - jb)) * L + l] = v[i];
      }
    }
  };
  if (n_chunks > 0 && wave > 0) stage(0, s_cf[0], tid - 64, ENC_STAGERS);
  __syncthreads();

  uint32_t Q = (uint32_t)cap;
  uint32_t x = RANS_L;
  for (int c = 0; c < n_chunks; ++c) {
    if (wave > 0) {
      if (c + 1 < n_chunks) stage(c + 1, s_cf[(c + 1) & 1], tid - 64, ENC_STAGERS);
    } else {
      const uint32_t* buf = s_cf[c & 1];
      int cs;
      const int J = locate(c, cs).J;
      const int n_sub = ENC_CHUNK * J;  // a multiple of ENC_BATCH
      for (int s0 = 0; s0 < n_sub; s0 += ENC_BATCH) {
        uint32_t v[ENC_BATCH];
#pragma unroll
        for (int i = 0; i < ENC_BATCH; ++i) {
          // read an in-bounds slot unconditionally, then select
          const uint32_t w = buf[min((s0 + i) * L + lane, ENC_SLOTS - 1)];
          v[i] = lane < L ? w : INACTIVE;
        }
#pragma unroll
        for (int i = 0; i < ENC_BATCH; ++i) {
          const bool act = v[i] != INACTIVE;
          Q = rans_enc_subround(x, act, v[i] & 0xFFFFu, (v[i] >> 16) + 1u, out, Q);
        }
      }
    }
    __syncthreads();
  }
  if (wave == 0) {
    // flush: states as (low, high) pairs for lanes 0..L-1 at the stream head
    Q -= 2u * (uint32_t)L;
    if (lane < L) {
      out[Q + 2 * lane] = (uint16_t)(x & 0xFFFFu);
      out[Q + 2 * lane + 1] = (uint16_t)(x >> 16);
    }
    if (lane == 0) counts[g] = (uint32_t)cap - Q;
  }
}

__global__ __launch_bounds__(256) void rans_encode_kernel(const uint32_t* __restrict__ cf, int H,
                                                          int W, int G, int L, int S,
                                                          uint16_t* __restrict__ words,
                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_cf[2][ENC_SLOTS];
  rans_encode_group(s_cf, cf, H, W, G, L, S, blockIdx.x, words, counts);
}

// Batched form: workgroup i codes work item i (image, group).
__global__ __launch_bounds__(256) void batch_rans_encode_kernel(BatchArgs b) {
  __shared__ uint32_t s_cf[2][ENC_SLOTS];
  const BatchItem it = b.items[blockIdx.x];
  const BatchImage im = b.images[it.image];
  rans_encode_group(s_cf, b.cf + im.px_off, im.H, im.W, im.G, im.L, 1, it.group,
                    b.words + im.words_off, b.counts + im.counts_off);
}

__device__ __forceinline__ void put_u16(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
}
__device__ __forceinline__ void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

// Part `part` of `parts` of group g's stream copy; part 0 of group 0 also
// writes the header, the counts and the total length.
__device__ __forceinline__ void pack_group_part(const uint16_t* __restrict__ words,
                                                const uint32_t* __restrict__ counts, int H,
                                                int W, int G, int L, int S, const HeaderFields& hf,
                                                uint8_t* __restrict__ out,
                                                uint64_t* __restrict__ out_len, int g, int part,
                                                int parts) {
  __shared__ unsigned long long s_before, s_total;
  if (threadIdx.x == 0) {
    unsigned long long before = 0, total = 0;
    for (int i = 0; i < G; ++i) {
      total += counts[i];
      if (i < g) before += counts[i];
    }
    s_before = before;
    s_total = total;
  }
  __syncthreads();
  const long long hdr = HEADER_BYTES + 4LL * G;
  if (g == 0 && part == 0) {
    if (threadIdx.x == 0) {
      out[0] = 'D'; out[1] = 'L'; out[2] = 'I'; out[3] = 'C';
      put_u16(out + 4, 1u);
      put_u16(out + 6, (uint32_t)hf.flags);
      put_u32(out + 8, (uint32_t)H);
      put_u32(out + 12, (uint32_t)W);
      out[16] = (uint8_t)hf.k_in;
      out[17] = (uint8_t)hf.n_mix;
      out[18] = (uint8_t)hf.dtype;
      out[19] = (uint8_t)SKEW;
      put_u16(out + 20, (uint32_t)hf.h1);
      put_u16(out + 22, (uint32_t)hf.h2);
      out[24] = (uint8_t)PROB_BITS;
      out[25] = (uint8_t)L;
      put_u16(out + 26, (uint32_t)G);
      put_u32(out + 28, (uint32_t)hf.fingerprint);
      put_u32(out + 32, (uint32_t)(hf.fingerprint >> 32));
      *out_len = (uint64_t)(hdr + 2LL * (long long)s_total);
    }
    for (int i = threadIdx.x; i < G; i += blockDim.x) put_u32(out + HEADER_BYTES + 4 * i, counts[i]);
  }
  int before, rows;
  group_span(g, H, G, S, before, rows);
  const long long cap = (long long)rows * W + 2LL * L;
  const uint32_t cnt = counts[g];
  const uint16_t* src = words + (long long)before * W + 2LL * L * g + (cap - cnt);
  uint8_t* dst = out + hdr + 2LL * (long long)s_before;
  for (long long i = (long long)part * blockDim.x + threadIdx.x; i < cnt;
       i += (long long)parts * blockDim.x)
    put_u16(dst + 2 * i, src[i]);
}

// grid (chunks, G): block (c, g) copies part c of group g's stream.
__global__ __launch_bounds__(256) void pack_kernel(const uint16_t* __restrict__ words,
                                                   const uint32_t* __restrict__ counts, int H,
                                                   int W, int G, int L, int S, HeaderFields hf,
                                                   uint8_t* __restrict__ out,
                                                   uint64_t* __restrict__ out_len) {
  pack_group_part(words, counts, H, W, G, L, S, hf, out, out_len, blockIdx.y, blockIdx.x,
                  gridDim.x);
}

// Batched form, grid (parts, items).  The last block of an image to finish
// stamps the image's completion time.
__global__ __launch_bounds__(256) void batch_pack_kernel(BatchArgs b) {
  const BatchItem it = b.items[blockIdx.y];
  const BatchImage im = b.images[it.image];
  pack_group_part(b.words + im.words_off, b.counts + im.counts_off, im.H, im.W, im.G, im.L, 1, b.hf,
                  b.out + im.out_off, b.len + it.image, it.group, blockIdx.x, gridDim.x);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned need = (unsigned)(im.G * gridDim.x);
    if (atomicAdd(b.done + it.image, 1u) + 1u == need && b.t_done)
      b.t_done[it.image] = __builtin_amdgcn_s_memrealtime();
  }
}

// ---- host-side launchers -------------------------------------------------

template <class Net>
static void launch_density_t(const Consts* K, const DevModel& m, const uint8_t* img, int H,
                             int W, uint32_t* cf, float* out15, uint32_t* tables, int grid,
                             hipStream_t s) {
  hipLaunchKernelGGL((density_kernel<Net>), dim3(grid), dim3(256), 0, s, K, m, img, H, W, cf,
                     out15, tables);
}

template <int H>
static bool launch_density_h(int wtype, const Consts* K, const DevModel& m, const uint8_t* img,
                             int Hh, int W, uint32_t* cf, float* out15, uint32_t* tables,
                             int grid, hipStream_t s) {
  switch (wtype) {
    case WT_F32:
      launch_density_t<NetF32<H>>(K, m, img, Hh, W, cf, out15, tables, grid, s);
      return true;
    case WT_BF16:
      launch_density_t<NetBF16<H, WT_BF16, false>>(K, m, img, Hh, W, cf, out15, tables, grid, s);
      return true;
    case WT_FP8:
      launch_density_t<NetBF16<H, WT_FP8, false>>(K, m, img, Hh, W, cf, out15, tables, grid, s);
      return true;
    case WT_FP8A8:
      launch_density_t<NetFP8A<H, false>>(K, m, img, Hh, W, cf, out15, tables, grid, s);
      return true;
    default: return false;
  }
}

bool launch_density(int wtype, int width, const Consts* K, const DevModel& m, const uint8_t* img,
                    int H, int W, uint32_t* cf, float* out15, uint32_t* tables, int grid,
                    hipStream_t s) {
  switch (width) {
    case 32: return launch_density_h<32>(wtype, K, m, img, H, W, cf, out15, tables, grid, s);
    case 64: return launch_density_h<64>(wtype, K, m, img, H, W, cf, out15, tables, grid, s);
    case 128: return launch_density_h<128>(wtype, K, m, img, H, W, cf, out15, tables, grid, s);
    default: return false;
  }
}

template <class Net>
static void launch_batch_density_t(const Consts* K, const DevModel& m, const BatchArgs& b,
                                   int grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_density_kernel<Net>), dim3(grid), dim3(256), 0, s, K, m, b);
}

template <int H>
static bool launch_batch_density_h(int wtype, const Consts* K, const DevModel& m,
                                   const BatchArgs& b, int grid, hipStream_t s) {
  switch (wtype) {
    case WT_F32: launch_batch_density_t<NetF32<H>>(K, m, b, grid, s); return true;
    case WT_BF16: launch_batch_density_t<NetBF16<H, WT_BF16, false>>(K, m, b, grid, s); return true;
    case WT_FP8: launch_batch_density_t<NetBF16<H, WT_FP8, false>>(K, m, b, grid, s); return true;
    case WT_FP8A8: launch_batch_density_t<NetFP8A<H, false>>(K, m, b, grid, s); return true;
    default: return false;
  }
}

bool launch_batch_density(int wtype, int width, const Consts* K, const DevModel& m,
                          const BatchArgs& b, int grid, hipStream_t s) {
  switch (width) {
    case 32: return launch_batch_density_h<32>(wtype, K, m, b, grid, s);
    case 64: return launch_batch_density_h<64>(wtype, K, m, b, grid, s);
    case 128: return launch_batch_density_h<128>(wtype, K, m, b, grid, s);
    default: return false;
  }
}

void launch_batch_rans_encode(const BatchArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(batch_rans_encode_kernel, dim3(b.n_items), dim3(256), 0, s, b);
}

void launch_batch_pack(const BatchArgs& b, int parts, hipStream_t s) {
  hipLaunchKernelGGL(batch_pack_kernel, dim3(parts, b.n_items), dim3(256), 0, s, b);
}

void launch_rans_encode(const uint32_t* cf, int H, int W, int G, int L, int S, uint16_t* words,
                        uint32_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(rans_encode_kernel, dim3(G), dim3(256), 0, s, cf, H, W, G, L, S, words,
                     counts);
}

void launch_pack(const uint16_t* words, const uint32_t* counts, int H, int W, int G, int L, int S,
                 const HeaderFields& hf, uint8_t* out, uint64_t* out_len, int chunks,
                 hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(chunks, G), dim3(256), 0, s, words, counts, H, W, G, L, S,
                     hf, out, out_len);
}

}  // namespace dlic
