// 12-bit samples (Section IV-C, Higher Bit Depth): the six-layer network with
// 4096 output neurons and a softmax over the 4096 levels.
//
// Arithmetic (the format; encoder and decoder run these same functions):
//  * the hidden layers as for 8-bit samples (deep_hidden), inputs scaled by
//    (2v - 4095) / 4095;
//  * the output layer as one bias-seeded chain of NK BF16 MFMAs per tile of
//    16 output neurons, FP32 logits;
//  * the table rule of the 8-bit network over 64 blocks of 64 levels: m = max
//    logit, e_v = expf(o_v - m), S_b summed in level order, S = ((S_0 + S_1)
//    + ...) + S_63, r = 1 / S, p_v = e_v r, block totals T_b in level order,
//    offsets O_0 = 0, O_b+1 = O_b + T_b, running sum L inside a block, C_v =
//    O_b + L_v, F(v) = v + min(M', floor(C_v M')) with M' = 2^16 - 4096.
//
// The output layer holds 1 MB of weights at H = 128, too much to stream once
// per 16-pixel tile, so it runs as a GEMM: a unit is 256 levels (one chunk of
// weights, loaded once per wave) times 16 pixel tiles.  The rule runs one wave
// per pixel, lane b owning block b, so the per-block sums in level order are
// each one lane's sequential loop and the sums across blocks are sequential
// loops over the lanes.
//
// Encoding: three kernels per chunk of pixels (hidden layers, output GEMM,
// rule).  Decoding: one cooperative launch walking the 2-D or 3-D wavefront;
// per step the step's tiles through the hidden layers (one wave per tile),
// grid barrier, the output GEMM, grid barrier, the rule per row into the
// row's table, grid barrier, every group decodes its rows' pixels of the step
// (a three-level 16-ary search of the table), grid barrier.
#include "dlic_deep.hpp"

namespace dlic {

constexpr int N12 = DEEP_OUT12;
constexpr uint32_t MP12 = M_TOTAL - N12;  // 61440
constexpr int UNIT_LEVELS = 256;          // levels per GEMM unit
constexpr int UNIT_TILES = 16;            // pixel tiles per GEMM unit
constexpr int UNIT_CHUNKS = N12 / UNIT_LEVELS;

// ---- hidden layers ----------------------------------------------------------
template <int H, int KIN>
__global__ __launch_bounds__(256) void deep12_hidden_kernel(const float* __restrict__ sc,
                                                            DeepNetArgs net,
                                                            const uint16_t* __restrict__ img,
                                                            int Hh, int W, VolGeom vg,
                                                            long long px0, long long n,
                                                            bf16x8* __restrict__ h5, int* bad) {
  constexpr int NK = H / 32;
  const int lane = threadIdx.x & 63;
  const int p = lane & 15, q = lane >> 4;
  const long long n_tiles = (n + 15) / 16;
  const long long NW = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long tile = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
       tile < n_tiles; tile += NW) {
    const long long i = tile * 16 + p;
    const bool valid = i < n;
    const long long px = px0 + (valid ? i : 0);
    const int Y = (int)(px / W), x = (int)(px - (long long)Y * W);
    const int z = Y / Hh, y = Y - z * Hh;
    if (valid && q == 0 && img[px] >= N12) atomicOr(bad, 1);
    const bf16x8 xin = deep_features<KIN, uint16_t>(sc, img, Hh, W, vg.ws, z, y, x, valid, q);
    bf16x8 a[NK];
    deep_hidden<H>(net, xin, a);
#pragma unroll
    for (int s = 0; s < NK; ++s) h5[(tile * NK + s) * 64 + lane] = a[s];
  }
}

// ---- output layer -----------------------------------------------------------
// Unit (c, g): levels [256 c, 256 c + 256) of the pixel tiles [16 g, 16 g + 16).
// Wave w computes the neuron tiles nt = 16 c + w + 4 i (i < 4) with their
// weights and biases held across the unit's tiles.  Rows: the encoder's tile t
// holds pixels 16 t + p (p < 16, below n_px); the decoder's tile t the rows
// tile_rows[t].x + p for p < tile_rows[t].y.
template <int H, bool DEC>
__device__ __forceinline__ void deep12_unit(const DeepNetArgs& d, const bf16x8* __restrict__ h5,
                                            long long n_tiles, long long n_px,
                                            const int2* __restrict__ tile_rows, int c,
                                            long long g, float* __restrict__ logits) {
  constexpr int NK = H / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  const bf16x8* w =
      reinterpret_cast<const bf16x8*>(d.wop) + deep_off(DEEP_LAYERS - 1, H, N12);
  bf16x8 wr[4][NK];
  f4 bias[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int nt = 16 * c + wave + 4 * i;
#pragma unroll
    for (int s = 0; s < NK; ++s) wr[i][s] = w[(nt * NK + s) * 64 + lane];
    const float* b = d.b[DEEP_LAYERS - 1] + 16 * nt + 4 * q;
    bias[i] = f4{b[0], b[1], b[2], b[3]};
  }
  const long long t_end = n_tiles < UNIT_TILES * (g + 1) ? n_tiles : UNIT_TILES * (g + 1);
  for (long long t = UNIT_TILES * g; t < t_end; ++t) {
    bf16x8 a[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) a[s] = h5[(t * NK + s) * 64 + lane];
    long long row;
    bool ok;
    if (DEC) {
      const int2 tr = tile_rows[t];
      ok = p < tr.y;
      row = (long long)tr.x + p;
    } else {
      row = t * 16 + p;
      ok = row < n_px;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int nt = 16 * c + wave + 4 * i;
      f4 acc = bias[i];
#pragma unroll
      for (int s = 0; s < NK; ++s) acc = mfma_bf16(wr[i][s], a[s], acc);
      if (ok) *reinterpret_cast<f4*>(logits + row * N12 + 16 * nt + 4 * q) = acc;
    }
  }
}

template <int H>
__global__ __launch_bounds__(256) void deep12_logits_kernel(DeepNetArgs net,
                                                            const bf16x8* __restrict__ h5,
                                                            long long n_tiles, long long n_px,
                                                            float* __restrict__ logits) {
  const long long units = (n_tiles + UNIT_TILES - 1) / UNIT_TILES * UNIT_CHUNKS;
  for (long long u = blockIdx.x; u < units; u += gridDim.x)
    deep12_unit<H, false>(net, h5, n_tiles, n_px, nullptr, (int)(u % UNIT_CHUNKS),
                          u / UNIT_CHUNKS, logits);
}

// ---- table rule -------------------------------------------------------------
__device__ __forceinline__ float lane_value(float v, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
}

// Lane b's block of one pixel's logits: levels 64 b .. 64 b + 63.
__device__ __forceinline__ void deep12_load_block(const float* __restrict__ lg, float (&pv)[64]) {
  const f4* src = reinterpret_cast<const f4*>(lg + 64 * (threadIdx.x & 63));
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const f4 v = src[j];
#pragma unroll
    for (int r = 0; r < 4; ++r) pv[4 * j + r] = v[r];
  }
}

// The rule on one pixel's logits, lane b holding block b in pv (one wave):
// afterwards pv[k] = p_v of level 64 b + k and off = O_b.
__device__ __forceinline__ void deep12_rule_regs(float (&pv)[64], float& off) {
  const int b = threadIdx.x & 63;
  float m = pv[0];
#pragma unroll
  for (int k = 1; k < 64; ++k) m = fmaxf(m, pv[k]);
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) m = fmaxf(m, __shfl_xor(m, sh));
  float sb = 0.0f;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    pv[k] = expf(pv[k] - m);
    sb = sb + pv[k];
  }
  float S = lane_value(sb, 0);
  for (int j = 1; j < 64; ++j) S = S + lane_value(sb, j);
  const float r = 1.0f / S;
  float tb = 0.0f;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    pv[k] = pv[k] * r;
    tb = tb + pv[k];
  }
  float o = 0.0f;
  for (int j = 0; j < 63; ++j) {
    const float t = lane_value(tb, j);
    if (j < b) o = o + t;
  }
  off = o;
}

__device__ __forceinline__ void deep12_rule(const float* __restrict__ lg, float (&pv)[64],
                                            float& off) {
  deep12_load_block(lg, pv);
  deep12_rule_regs(pv, off);
}

// Table of one pixel: F(0..4095) as u16 (F(0) = 0), 8 levels per 16-byte store.
__device__ __forceinline__ void deep12_write_table(const float (&pv)[64], float off,
                                                   uint16_t* __restrict__ tab) {
  const int b = threadIdx.x & 63;
  float L = 0.0f;
  uint4* dst = reinterpret_cast<uint4*>(tab + 64 * b);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      uint32_t pair = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = 8 * j + 2 * h + e, v = 64 * b + k;
        const uint32_t Fv = v == 0 ? 0u : deep_F(v, off + L, MP12);
        pair |= Fv << (16 * e);
        L = L + pv[k];
      }
      w[h] = pair;
    }
    dst[j] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

__global__ __launch_bounds__(256) void deep12_softmax_kernel(const float* __restrict__ logits,
                                                             const uint16_t* __restrict__ img,
                                                             long long px0, long long n,
                                                             uint32_t* __restrict__ cf,
                                                             uint16_t* __restrict__ tables) {
  const int b = threadIdx.x & 63;
  const long long NW = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long i = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n;
       i += NW) {
    float pv[64], off;
    deep12_rule(logits + i * N12, pv, off);
    if (tables) deep12_write_table(pv, off, tables + i * N12);
    if (cf) {
      const int xv = deep_level(img[px0 + i]);
      if ((xv >> 6) == b) {
        float L = 0.0f;
        uint32_t c = 0, fn = 0;
#pragma unroll
        for (int k = 0; k < 64; ++k) {
          const int v = 64 * b + k;
          if (v == xv) c = v == 0 ? 0u : deep_F(v, off + L, MP12);
          L = L + pv[k];
          if (v == xv) fn = v == N12 - 1 ? M_TOTAL : deep_F(v + 1, off + L, MP12);
        }
        cf[px0 + i] = c | ((fn - c - 1u) << 16);
      }
    }
  }
}

__global__ void deep12_reject_kernel(const int* bad, uint64_t* out_len) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *bad != 0) *out_len = 0;
}

// ---- decoder ------------------------------------------------------------------
// The hidden layers' weights and biases and the input scale of the decoder,
// copied to LDS once: a grid barrier's acquire invalidates the cache every step.
template <int H>
struct Hidden12Lds {
  static constexpr long long N_OPS = deep_off(DEEP_LAYERS - 1, H, N12);  // bf16x8
  static constexpr int N_BIAS = (DEEP_LAYERS - 1) * H;
};

template <int H, int KIN>
__global__ __launch_bounds__(DEEP_WAVES * 64) void deep12_decode_kernel(DeepDecArgs a) {
  constexpr int NK = H / 32;
  __shared__ bf16x8 s_w[Hidden12Lds<H>::N_OPS];
  __shared__ float s_b[Hidden12Lds<H>::N_BIAS];
  __shared__ float s_scale[N12];
  __shared__ int s_err;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  if (threadIdx.x == 0) s_err = deep_check_header(a);
  {
    const bf16x8* w = reinterpret_cast<const bf16x8*>(a.net.wop);
    for (int i = threadIdx.x; i < Hidden12Lds<H>::N_OPS; i += blockDim.x) s_w[i] = w[i];
    for (int i = threadIdx.x; i < Hidden12Lds<H>::N_BIAS; i += blockDim.x)
      s_b[i] = a.net.b[i / H][i % H];
    for (int i = threadIdx.x; i < N12; i += blockDim.x) s_scale[i] = a.K->scale12[i];
  }
  __syncthreads();
  const int err = __builtin_amdgcn_readfirstlane(s_err);
  const int Z = a.vg.Z, lag = a.vg.lag;
  const int HT = Z * a.H, GT = Z * a.G;
  const long long T2 = (long long)a.W + SKEW * (a.H - 1);  // steps of one slice
  const int gw = blockIdx.x * DEEP_WAVES + wave;            // this wave in the grid
  const int NW = gridDim.x * DEEP_WAVES;
  uint16_t* img = reinterpret_cast<uint16_t*>(a.img);
  bf16x8* h5 = reinterpret_cast<bf16x8*>(a.h5);
  // the group this wave decodes, if any: its lanes' states live in registers
  const int g = gw;
  const bool coder = err == 0 && g < GT;
  int r0 = 0, R = 0, J = 0, zg = 0;
  uint32_t n_words = 0, Pw = 0, x = RANS_L;
  const uint16_t* gw16 = nullptr;
  bool bad = false;
  if (coder) {
    r0 = group_row(g, HT, GT);
    R = group_row(g + 1, HT, GT) - r0;
    J = (R + a.L - 1) / a.L;
    zg = r0 / a.H;
    unsigned long long before = 0, total = 0;
    for (int i = lane; i < GT; i += 64) {
      const uint32_t c = rd32(a.bits + HEADER_BYTES + 4 * i);
      total += c;
      if (i < g) before += c;
    }
    for (int sh = 32; sh >= 1; sh >>= 1) {
      total += __shfl_xor(total, sh);
      before += __shfl_xor(before, sh);
    }
    n_words = rd32(a.bits + HEADER_BYTES + 4 * g);
    bad = (unsigned long long)(HEADER_BYTES + 4LL * GT) + 2ull * total != a.n_bytes ||
          n_words < 2u * (uint32_t)a.L;
    gw16 = reinterpret_cast<const uint16_t*>(a.bits + HEADER_BYTES + 4LL * GT + 2ull * before);
    if (!bad && lane < a.L) x = (uint32_t)gw16[2 * lane] | ((uint32_t)gw16[2 * lane + 1] << 16);
    Pw = 2u * (uint32_t)a.L;
  }
  bool over = false;
  unsigned k_bar = 0;
  bool alive = err == 0;
  for (long long t = 0; t < a.T && alive; ++t) {
    // ---- hidden layers of the step's tiles (tile k: the k-th 16-row block of
    // the active rows, slice by slice), one wave per tile
    int z_lo = 0, z_hi = Z - 1;
    if (lag > 0) {
      z_hi = (int)(t / lag < Z - 1 ? t / lag : Z - 1);
      z_lo = (int)(t - T2 + 1 > 0 ? (t - T2 + lag) / lag : 0);
    }
    int k = gw, base = 0;
    for (int z = z_lo; z <= z_hi; ++z) {
      const long long tz = t - (long long)lag * z;
      const int y_lo = (int)(tz - a.W + 1 > 0 ? (tz - a.W + SKEW) / SKEW : 0);
      const int y_hi = (int)(tz / SKEW < a.H - 1 ? tz / SKEW : a.H - 1);
      const int n_act = y_hi - y_lo + 1;
      const int nt = n_act > 0 ? (n_act + 15) / 16 : 0;
      for (; k < base + nt; k += NW) {
        const int y0 = y_lo + 16 * (k - base);
        const int y = y0 + p;
        const bool valid = y <= y_hi;
        const int xx = valid ? (int)(tz - (long long)SKEW * y) : 0;
        const bf16x8 xin = deep_features<KIN, uint16_t>(s_scale, img, a.H, a.W, a.vg.ws, z,
                                                        valid ? y : 0, xx, valid, q);
        bf16x8 av[NK];
        deep_hidden_at<H>(s_w, [&](int l) { return s_b + l * H; }, xin, av);
#pragma unroll
        for (int s = 0; s < NK; ++s) h5[((long long)k * NK + s) * 64 + lane] = av[s];
        if (lane == 0) a.tile_rows[k] = make_int2(z * a.H + y0, y_hi - y0 + 1 < 16 ? y_hi - y0 + 1 : 16);
      }
      base += nt;
    }
    const int n_tiles = base;
    alive = grid_sync(a.bar, a.abort_flag, k_bar, a.spin_limit);
    if (!alive) break;
    // ---- the output layer of every row of the step
    const int units = (n_tiles + UNIT_TILES - 1) / UNIT_TILES * UNIT_CHUNKS;
    for (int u = blockIdx.x; u < units; u += gridDim.x)
      deep12_unit<H, true>(a.net, h5, n_tiles, 0, a.tile_rows, u % UNIT_CHUNKS, u / UNIT_CHUNKS,
                           a.logits);
    alive = grid_sync(a.bar, a.abort_flag, k_bar, a.spin_limit);
    if (!alive) break;
    // ---- the table rule, one wave per row
    for (int j = gw; j < n_tiles * 16; j += NW) {
      const int2 tr = a.tile_rows[j >> 4];
      if ((j & 15) >= tr.y) continue;
      const long long Y = (long long)tr.x + (j & 15);
      float pv[64], off;
      deep12_rule(a.logits + Y * N12, pv, off);
      deep12_write_table(pv, off, a.tables + Y * N12);
    }
    alive = grid_sync(a.bar, a.abort_flag, k_bar, a.spin_limit);
    if (!alive) break;
    // ---- each group decodes its rows' pixels of the step
    const long long tg = t - (long long)lag * zg;
    if (coder && !bad && tg >= 0 && tg < T2) {
      for (int j = 0; j < J; ++j) {
        const int rr = j * a.L + lane;
        const int Y = r0 + rr;
        const long long xc = tg - (long long)SKEW * (Y - zg * a.H);
        const bool act = lane < a.L && rr < R && xc >= 0 && xc < a.W;
        if (__ballot(act) == 0ull) continue;
        const uint32_t slot = x & 0xFFFFu;
        const uint16_t* tab = a.tables + (long long)(act ? Y : 0) * N12;
        // 256-level bucket, 16-level bucket, then the level
        int b1 = 0;
#pragma unroll
        for (int kk = 1; kk < 16; ++kk) b1 += ((uint32_t)tab[256 * kk] <= slot) ? 1 : 0;
        int b2 = 0;
#pragma unroll
        for (int kk = 1; kk < 16; ++kk) b2 += ((uint32_t)tab[256 * b1 + 16 * kk] <= slot) ? 1 : 0;
        const int base16 = 256 * b1 + 16 * b2;
        uint32_t Fl[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) Fl[i] = tab[base16 + i];
        int cnt = 0;
#pragma unroll
        for (int i = 1; i < 16; ++i) cnt += (Fl[i] <= slot) ? 1 : 0;
        const int v = base16 + cnt;
        uint32_t c = Fl[0];
        uint32_t fn = base16 + 16 < N12 ? (uint32_t)tab[base16 + 16] : M_TOTAL;
#pragma unroll
        for (int i = 1; i < 16; ++i) {
          if (i == cnt) c = Fl[i];
          if (i == cnt + 1) fn = Fl[i];
        }
        const uint32_t f = fn - c;
        const uint32_t xd = __umul24(f, x >> 16) + slot - c;
        const bool ren = act && xd < RANS_L;
        const uint64_t m = __ballot(ren);
        const uint32_t rk = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        const uint32_t pos = Pw + rk;
        uint32_t wv = 0;
        if (ren) {
          if (pos < n_words)
            wv = gw16[pos];
          else
            over = true;
        }
        if (act) x = ren ? ((xd << 16) | wv) : xd;
        Pw += (uint32_t)__popcll(m);
        if (act) img[(long long)Y * a.W + xc] = (uint16_t)v;
      }
    }
    alive = grid_sync(a.bar, a.abort_flag, k_bar, a.spin_limit);
  }
  if (err != 0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicMax(a.status, err);
    return;
  }
  if (!alive) {
    if (threadIdx.x == 0) atomicMax(a.status, 7);
    return;
  }
  if (coder) {
    const bool lane_bad = lane < a.L && x != RANS_L;
    if (__ballot(lane_bad || over || bad) != 0ull || Pw != n_words) {
      if (lane == 0) atomicMax(a.status, 3);
    }
  }
}

template <int H, int KIN>
static int decode12_residency() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, deep12_decode_kernel<H, KIN>,
                                                   DEEP_WAVES * 64, 0) != hipSuccess)
    return 0;
  return per_cu;
}

int deep12_decode_max_grid(int H, int k_in) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  int per_cu = 0;
  if (k_in == K_IN)
    per_cu = H == 64 ? decode12_residency<64, K_IN>() : decode12_residency<128, K_IN>();
  else
    per_cu = H == 64 ? decode12_residency<64, K_IN_3D>() : decode12_residency<128, K_IN_3D>();
  return cus * per_cu;
}

hipError_t launch_deep12_decode(const DeepDecArgs& a, int grid, hipStream_t s) {
  DeepDecArgs args = a;
  void* kargs[] = {&args};
  const void* fn = nullptr;
  if (a.net.k_in == K_IN)
    fn = a.net.H == 64 ? (const void*)deep12_decode_kernel<64, K_IN>
                       : (const void*)deep12_decode_kernel<128, K_IN>;
  else if (a.net.k_in == K_IN_3D)
    fn = a.net.H == 64 ? (const void*)deep12_decode_kernel<64, K_IN_3D>
                       : (const void*)deep12_decode_kernel<128, K_IN_3D>;
  if (!fn || (a.net.H != 64 && a.net.H != 128)) return hipErrorInvalidValue;
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(DEEP_WAVES * 64), kargs, 0, s);
}

// ---- launchers --------------------------------------------------------------
static unsigned grid_for(long long waves) {
  long long g = (waves + 3) / 4;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

bool launch_deep12_hidden(const Consts* K, const DeepNetArgs& net, const uint16_t* img, int H,
                          int W, const VolGeom& vg, long long px0, long long n, void* h5,
                          int* bad, hipStream_t s) {
  const unsigned grid = grid_for((n + 15) / 16);
  const float* sc = K->scale12;
  bf16x8* o = (bf16x8*)h5;
  if (net.H == 64 && net.k_in == K_IN)
    hipLaunchKernelGGL((deep12_hidden_kernel<64, K_IN>), dim3(grid), dim3(256), 0, s, sc, net,
                       img, H, W, vg, px0, n, o, bad);
  else if (net.H == 128 && net.k_in == K_IN)
    hipLaunchKernelGGL((deep12_hidden_kernel<128, K_IN>), dim3(grid), dim3(256), 0, s, sc, net,
                       img, H, W, vg, px0, n, o, bad);
  else if (net.H == 64 && net.k_in == K_IN_3D)
    hipLaunchKernelGGL((deep12_hidden_kernel<64, K_IN_3D>), dim3(grid), dim3(256), 0, s, sc,
                       net, img, H, W, vg, px0, n, o, bad);
  else if (net.H == 128 && net.k_in == K_IN_3D)
    hipLaunchKernelGGL((deep12_hidden_kernel<128, K_IN_3D>), dim3(grid), dim3(256), 0, s, sc,
                       net, img, H, W, vg, px0, n, o, bad);
  else
    return false;
  return true;
}

bool launch_deep12_logits(const DeepNetArgs& net, const void* h5, long long n_px,
                          float* logits, hipStream_t s) {
  const long long n_tiles = (n_px + 15) / 16;
  const long long units = (n_tiles + UNIT_TILES - 1) / UNIT_TILES * UNIT_CHUNKS;
  const unsigned grid = (unsigned)(units < 2048 ? (units > 0 ? units : 1) : 2048);
  if (net.H == 64)
    hipLaunchKernelGGL(deep12_logits_kernel<64>, dim3(grid), dim3(256), 0, s, net,
                       (const bf16x8*)h5, n_tiles, n_px, logits);
  else if (net.H == 128)
    hipLaunchKernelGGL(deep12_logits_kernel<128>, dim3(grid), dim3(256), 0, s, net,
                       (const bf16x8*)h5, n_tiles, n_px, logits);
  else
    return false;
  return true;
}

void launch_deep12_softmax(const float* logits, const uint16_t* img, long long px0, long long n,
                           uint32_t* cf, uint16_t* tables, hipStream_t s) {
  hipLaunchKernelGGL(deep12_softmax_kernel, dim3(grid_for(n)), dim3(256), 0, s, logits, img, px0,
                     n, cf, tables);
}

void launch_deep12_reject(const int* bad, uint64_t* out_len, hipStream_t s) {
  hipLaunchKernelGGL(deep12_reject_kernel, dim3(1), dim3(64), 0, s, bad, out_len);
}

}  // namespace dlic
