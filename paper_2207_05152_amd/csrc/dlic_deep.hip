// The paper's own density network and head (Section II-B, Neural Network
// Architecture): six dense layers, k -> H -> H -> H -> H -> H -> 256 with
// ReLU, and a softmax over the 256 grey levels; the PMF becomes the coder's
// cumulative table by a prefix sum (Section II-B, rANS).  k = 12 for images;
// for volumes (Section IV-C, 3D Dependencies and 3D Wavefront) k = 21: the
// 12-pixel window of the pixel's own slice and a 3 x 3 block of the slice
// below, rows y + WS - 3 .. y + WS - 1, columns x - 1 .. x + 1.
//
// Arithmetic (the format; encoder and decoder run these same functions):
//  * BF16 weights and layer inputs, FP32 accumulation on
//    v_mfma_f32_16x16x32_bf16 (16-pixel tiles, the layout of NetBF16: slot e
//    of lane group q of k-step s is input neuron 32 s + 16 (e / 4) + 4 q + e % 4,
//    layer 1 takes feature 4 e + q in slot e while 4 e + q < k); the bias seeds
//    the accumulator;
//  * table rule in FP32: m = max logit, e_v = expf(o_v - m), S = ((S0 + S1) +
//    S2) + S3 over four blocks of 64 levels each summed in level order,
//    r = 1 / S, p_v = e_v r, block totals T_b in level order, offsets O_0 = 0,
//    O_b+1 = O_b + T_b, running sum L inside a block, C_v = O_b + L_v,
//    F(v) = v + min(M', floor(C_v M')), F(0) = 0, F(256) = 2^16.
//
// Decoding follows the paper's GPU scheme (Section II-B, Preprocessor: all
// pixels of one wavefront step enter the network as one matrix): one
// cooperative launch walks the steps; in each, the grid evaluates the network
// for the step's pixels (one 16-pixel tile per workgroup, its layers split
// over the four waves) and writes their tables, then every group's wave
// decodes its rows' pixels of the step from those tables.  Instead of grid
// barriers between the phases, each row carries two progress counters: the
// step of its newest table and of its newest decoded pixel.  A tile waits for
// the pixels its windows read (rows above, its own rows' left neighbours, the
// slice below), a group for its rows' tables; every wait is for an event of an
// earlier step or phase, which every workgroup reaches in the same order, so
// with all workgroups resident the pipeline cannot deadlock.  Weights do not fit a CU's LDS (200 KB at H = 128), so every tile
// reads them from the L2 in operand order.  A volume is coded as its slices
// stacked into one image with G groups per slice; its decode walks the 3-D
// wavefront: global step t holds pixel (z, y, x) with x + 3 y + lag z = t, so
// every slice's pixels of a step are evaluated together (lag = 0: all slices
// in lock-step).
#include "dlic_deep.hpp"

namespace dlic {

constexpr int SM_ROW = DEEP_OUT + 4;  // floats per pixel row of the softmax scratch

size_t deep_wop_bytes(int H, int nout) { return (size_t)deep_off(DEEP_LAYERS, H, nout) * 16; }

struct DeepPackArgs {
  const uint16_t* w[DEEP_LAYERS];
};

__global__ __launch_bounds__(256) void deep_pack_kernel(int H, int k_in, int nout,
                                                       DeepPackArgs p, uint16_t* wop) {
  const long long total = deep_off(DEEP_LAYERS, H, nout);
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int i = 0;
    while (idx >= deep_off(i + 1, H, nout)) ++i;
    const long long r = idx - deep_off(i, H, nout);
    const int lane = (int)(r & 63), blk = (int)(r >> 6);
    const int NK = deep_in(i, H) / 32;
    const int nt = blk / NK, s = blk - nt * NK;
    const int row = 16 * nt + (lane & 15), q = lane >> 4;
    const int fan_in = i == 0 ? k_in : H;
    for (int e = 0; e < 8; ++e) {
      const int k = deep_slot_input(i, s, q, e, k_in);
      wop[idx * 8 + e] = k >= 0 ? p.w[i][(long long)row * fan_in + k] : (uint16_t)0;
    }
  }
}

void launch_deep_pack(int H, int k_in, int nout, const uint16_t* const* w, void* wop,
                      hipStream_t s) {
  DeepPackArgs p;
  for (int i = 0; i < DEEP_LAYERS; ++i) p.w[i] = w[i];
  const long long total = deep_off(DEEP_LAYERS, H, nout);
  const int grid = (int)((total + 255) / 256);
  hipLaunchKernelGGL(deep_pack_kernel, dim3(grid), dim3(256), 0, s, H, k_in, nout, p,
                     (uint16_t*)wop);
}

// One 16-pixel tile through the six layers.  Lane l holds the layer-1 operand
// of pixel l % 16 (features 4 e + l / 16 in slot e) and gets logits
// 16 nt + 4 (l / 16) + r of that pixel in o[nt][r].
template <int H>
__device__ __forceinline__ void deep_run(const DeepNetArgs& d, const bf16x8 x,
                                         float (&o)[DEEP_OUT / 16][4]) {
  constexpr int NK = H / 32;
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int q = lane >> 4;
  bf16x8 a[NK];
  deep_hidden<H>(d, x, a);
  const bf16x8* w = reinterpret_cast<const bf16x8*>(d.wop) + deep_off(DEEP_LAYERS - 1, H, DEEP_OUT);
#pragma unroll
  for (int nt = 0; nt < DEEP_OUT / 16; ++nt) {
    const float* b = d.b[DEEP_LAYERS - 1] + 16 * nt + 4 * q;
    f4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
    for (int s = 0; s < NK; ++s) acc = mfma_bf16(w[(nt * NK + s) * 64 + lane], a[s], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) o[nt][r] = acc[r];
  }
}

// The same network evaluated by the four waves of a workgroup on one tile:
// wave w computes the neuron tiles nt = w, w + 4, ... of every layer.  The
// decoder runs it once per wavefront step with a grid barrier in between,
// whose acquire invalidates the cache, so the wave keeps its quarter of the
// weights in registers for the whole launch (WgNet, loaded once) and the
// biases sit in LDS.  Layer outputs go through LDS as the next layer's BF16
// operands (act: two buffers of NK * 64 bf16x8); the logits land in sm[p][v].
// Each output tile's accumulation is the same chain of the same MFMAs as in
// deep_run, so the results are identical.
template <int H>
struct WgNet {
  static constexpr int NT = H / 16, NK = H / 32;
  static constexpr int TW = NT / DEEP_WAVES;            // hidden tiles per wave (1 or 2)
  static constexpr int TO = DEEP_OUT / 16 / DEEP_WAVES;  // output tiles per wave (4)
  static constexpr int NB = (DEEP_LAYERS - 1) * H + DEEP_OUT;  // biases
  bf16x8 w0[TW];
  bf16x8 wh[DEEP_LAYERS - 2][TW][NK];
  bf16x8 wo[TO][NK];

  __device__ __forceinline__ void load(const DeepNetArgs& d, int wave, int lane) {
    const bf16x8* w = reinterpret_cast<const bf16x8*>(d.wop);
#pragma unroll
    for (int i = 0; i < TW; ++i) w0[i] = w[(wave + DEEP_WAVES * i) * 64 + lane];
#pragma unroll
    for (int l = 0; l < DEEP_LAYERS - 2; ++l) {
      const bf16x8* wl = w + deep_off(l + 1, H, DEEP_OUT);
#pragma unroll
      for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int s = 0; s < NK; ++s) wh[l][i][s] = wl[((wave + DEEP_WAVES * i) * NK + s) * 64 + lane];
    }
    const bf16x8* wl = w + deep_off(DEEP_LAYERS - 1, H, DEEP_OUT);
#pragma unroll
    for (int i = 0; i < TO; ++i)
#pragma unroll
      for (int s = 0; s < NK; ++s) wo[i][s] = wl[((wave + DEEP_WAVES * i) * NK + s) * 64 + lane];
  }
  // biases of layer l start at bias_off(l) in the LDS copy
  static __device__ __forceinline__ int bias_off(int l) { return l * H; }
};

template <int H>
__device__ __forceinline__ void deep_stage_biases(const DeepNetArgs& d, float* s_bias) {
  for (int i = threadIdx.x; i < WgNet<H>::NB; i += blockDim.x) {
    const int l = i / H < DEEP_LAYERS - 1 ? i / H : DEEP_LAYERS - 1;
    s_bias[i] = d.b[l][i - l * H];
  }
}

template <int H>
__device__ __forceinline__ void deep_run_wg(const WgNet<H>& n, const float* s_bias,
                                            const bf16x8 x, bf16x8* act, float* sm) {
  constexpr int NK = WgNet<H>::NK, TW = WgNet<H>::TW, TO = WgNet<H>::TO;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, p = lane & 15;
  // layer 0
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int nt = wave + DEEP_WAVES * i;
    const float* b = s_bias + WgNet<H>::bias_off(0) + 16 * nt + 4 * q;
    f4 acc = {b[0], b[1], b[2], b[3]};
    acc = mfma_bf16(n.w0[i], x, acc);
    // neuron 16 nt + 4 q + r goes to slot e = 4 (nt % 2) + r of lane group q, k-step nt / 2
    __bf16* dst = reinterpret_cast<__bf16*>(&act[(nt >> 1) * 64 + 16 * q + p]) + 4 * (nt & 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[r] = (__bf16)relu(acc[r]);
  }
  __syncthreads();
  // hidden layers 1 .. 4
#pragma unroll
  for (int l = 0; l < DEEP_LAYERS - 2; ++l) {
    const int cur = l & 1;
    bf16x8 a[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) a[s] = act[cur * NK * 64 + s * 64 + lane];
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      const int nt = wave + DEEP_WAVES * i;
      const float* b = s_bias + WgNet<H>::bias_off(l + 1) + 16 * nt + 4 * q;
      f4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
      for (int s = 0; s < NK; ++s) acc = mfma_bf16(n.wh[l][i][s], a[s], acc);
      __bf16* dst = reinterpret_cast<__bf16*>(&act[(cur ^ 1) * NK * 64 + (nt >> 1) * 64 +
                                                   16 * q + p]) + 4 * (nt & 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[r] = (__bf16)relu(acc[r]);
    }
    __syncthreads();
  }
  // output layer (its input is buffer (DEEP_LAYERS - 2) & 1)
  {
    constexpr int cur = (DEEP_LAYERS - 2) & 1;
    bf16x8 a[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) a[s] = act[cur * NK * 64 + s * 64 + lane];
#pragma unroll
    for (int i = 0; i < TO; ++i) {
      const int nt = wave + DEEP_WAVES * i;
      const float* b = s_bias + WgNet<H>::bias_off(DEEP_LAYERS - 1) + 16 * nt + 4 * q;
      f4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
      for (int s = 0; s < NK; ++s) acc = mfma_bf16(n.wo[i][s], a[s], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) sm[p * SM_ROW + 16 * nt + 4 * q + r] = acc[r];
    }
    __syncthreads();
  }
}

// The table rule for the 16 pixels of a tile.  sm: the wave's [16][SM_ROW]
// scratch.  Afterwards lane (b, p) = (l / 16, l % 16) holds block b of pixel
// p: its offset O_b and, in sm[p][64 b + k], the probabilities p_v.
struct DeepBlock {
  float off;
};

__device__ __forceinline__ DeepBlock deep_softmax(float (&o)[DEEP_OUT / 16][4], float* sm) {
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int p = lane & 15, q = lane >> 4;
  float m = o[0][0];
#pragma unroll
  for (int nt = 0; nt < DEEP_OUT / 16; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) m = fmaxf(m, o[nt][r]);
  m = fmaxf(m, __shfl_xor(m, 16));
  m = fmaxf(m, __shfl_xor(m, 32));
#pragma unroll
  for (int nt = 0; nt < DEEP_OUT / 16; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) sm[p * SM_ROW + 16 * nt + 4 * q + r] = expf(o[nt][r] - m);
  wave_lds_handover();
  // block b = q of pixel p, in level order
  float* row = sm + p * SM_ROW + 64 * q;
  float sb = 0.0f;
#pragma unroll 8
  for (int k = 0; k < 64; ++k) sb = sb + row[k];
  const float s0 = __shfl(sb, p), s1 = __shfl(sb, p + 16), s2 = __shfl(sb, p + 32),
              s3 = __shfl(sb, p + 48);
  const float S = ((s0 + s1) + s2) + s3;
  const float rr = 1.0f / S;
  float tb = 0.0f;
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    const float pv = row[k] * rr;
    row[k] = pv;
    tb = tb + pv;
  }
  const float t0 = __shfl(tb, p), t1 = __shfl(tb, p + 16), t2 = __shfl(tb, p + 32);
  const float o1 = t0, o2 = o1 + t1, o3 = o2 + t2;
  DeepBlock blk;
  blk.off = q == 0 ? 0.0f : (q == 1 ? o1 : (q == 2 ? o2 : o3));
  return blk;
}

// The decoder's tables for the 16 pixels of a tile, by the four waves of a
// workgroup (logits in sm[p][v]; afterwards F(v) of pixel p in
// tab_lds[p][v]), with the operations and order of deep_softmax and the
// encoder's table loop, so the tables are the encoder's: the exponentials and
// the F evaluations, which no sum orders, are spread over all 256 threads;
// wave 0 keeps the order-fixed sums (lane (b, p): block b of pixel p) and
// leaves each level's C_v in sm.  part: 256 floats of scratch.
__device__ __forceinline__ void deep_tables_wg(float* sm, float* part, uint16_t* tab_lds) {
  const int tid = threadIdx.x;
  const int p = tid & 15, s16 = tid >> 4;  // pixel, 16-level slice
  {
    const f4* src = reinterpret_cast<const f4*>(sm + p * SM_ROW + 16 * s16);
    float m = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f4 v = src[j];
      m = fmaxf(fmaxf(m, v[0]), fmaxf(fmaxf(v[1], v[2]), v[3]));
    }
    part[s16 * 16 + p] = m;
  }
  __syncthreads();
  {
    float m = part[p];
#pragma unroll
    for (int j = 1; j < 16; ++j) m = fmaxf(m, part[j * 16 + p]);
    f4* row = reinterpret_cast<f4*>(sm + p * SM_ROW + 16 * s16);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      f4 v = row[j];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = expf(v[r] - m);
      row[j] = v;
    }
  }
  __syncthreads();
  if (tid < 64) {
    const int q = tid >> 4;  // block
    f4* row = reinterpret_cast<f4*>(sm + p * SM_ROW + 64 * q);
    float v[64];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const f4 t = row[j];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[4 * j + r] = t[r];
    }
    float sb = 0.0f;
#pragma unroll
    for (int k = 0; k < 64; ++k) sb = sb + v[k];
    const float s0 = __shfl(sb, p), s1 = __shfl(sb, p + 16), s2 = __shfl(sb, p + 32),
                s3 = __shfl(sb, p + 48);
    const float S = ((s0 + s1) + s2) + s3;
    const float rr = 1.0f / S;
    float tb = 0.0f;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      v[k] = v[k] * rr;
      tb = tb + v[k];
    }
    const float t0 = __shfl(tb, p), t1 = __shfl(tb, p + 16), t2 = __shfl(tb, p + 32);
    const float o1 = t0, o2 = o1 + t1, o3 = o2 + t2;
    const float off = q == 0 ? 0.0f : (q == 1 ? o1 : (q == 2 ? o2 : o3));
    float L = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      f4 c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        c[r] = off + L;
        L = L + v[4 * j + r];
      }
      row[j] = c;
    }
  }
  __syncthreads();
  {
    const f4* src = reinterpret_cast<const f4*>(sm + p * SM_ROW + 16 * s16);
    uint32_t w[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f4 c = src[j];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int l0 = 16 * s16 + 4 * j + 2 * h;
        const uint32_t F0 = l0 == 0 ? 0u : deep_F(l0, c[2 * h], M_PRIME);
        const uint32_t F1 = deep_F(l0 + 1, c[2 * h + 1], M_PRIME);
        w[2 * j + h] = F0 | (F1 << 16);
      }
    }
    uint4* dst = reinterpret_cast<uint4*>(tab_lds + p * DEEP_OUT + 16 * s16);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
  __syncthreads();
}

// Encoder side: every pixel's interval (and optionally logits / tables).
template <int H, int KIN>
__global__ __launch_bounds__(DEEP_WAVES * 64) void deep_density_kernel(
    const Consts* __restrict__ K, DeepNetArgs net, const uint8_t* __restrict__ img, int Hh, int W,
    VolGeom vg, uint32_t* __restrict__ cf, float* __restrict__ logits,
    uint16_t* __restrict__ tables) {
  __shared__ float s_sm[DEEP_WAVES][16 * SM_ROW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  float* sm = s_sm[wave];
  const long long n = (long long)vg.Z * Hh * W;
  const long long n_tiles = (n + 15) / 16;
  for (long long tile = (long long)blockIdx.x * DEEP_WAVES + wave; tile < n_tiles;
       tile += (long long)gridDim.x * DEEP_WAVES) {
    const long long px = tile * 16 + p;
    const bool valid = px < n;
    const int Y = valid ? (int)(px / W) : 0, x = valid ? (int)(px - (long long)Y * W) : 0;
    const int z = Y / Hh, y = Y - z * Hh;
    const bf16x8 xin = deep_features<KIN, uint8_t>(K->scale, img, Hh, W, vg.ws, z, y, x, valid, q);
    float o[DEEP_OUT / 16][4];
    deep_run<H>(net, xin, o);
    if (logits && valid) {
#pragma unroll
      for (int nt = 0; nt < DEEP_OUT / 16; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) logits[px * DEEP_OUT + 16 * nt + 4 * q + r] = o[nt][r];
    }
    const DeepBlock blk = deep_softmax(o, sm);
    const float* row = sm + p * SM_ROW + 64 * q;
    const int xv = valid ? (int)img[px] : 0;
    const bool mine = (xv >> 6) == q;  // this lane's block holds the pixel's level
    float L = 0.0f;
    uint32_t c = 0, fnext = 0;
#pragma unroll 4
    for (int k = 0; k < 64; ++k) {
      const int v = 64 * q + k;
      const uint32_t Fv = v == 0 ? 0u : deep_F(v, blk.off + L, M_PRIME);
      if (tables && valid) tables[px * DEEP_OUT + v] = (uint16_t)Fv;
      if (v == xv) c = Fv;
      L = L + row[k];
      if (v == xv) fnext = v == DEEP_OUT - 1 ? M_TOTAL : deep_F(v + 1, blk.off + L, M_PRIME);
    }
    if (valid && mine && cf) cf[px] = c | ((fnext - c - 1u) << 16);
    wave_lds_handover();
  }
}

template <int H, int KIN>
static void density_at(unsigned grid, hipStream_t s, const Consts* K, const DeepNetArgs& net,
                       const uint8_t* img, int Hh, int W, const VolGeom& vg, uint32_t* cf,
                       float* logits, uint16_t* tables) {
  hipLaunchKernelGGL((deep_density_kernel<H, KIN>), dim3(grid), dim3(DEEP_WAVES * 64), 0, s, K,
                     net, img, Hh, W, vg, cf, logits, tables);
}

bool launch_deep_density(const Consts* K, const DeepNetArgs& net, const uint8_t* img, int H,
                         int W, const VolGeom& vg, uint32_t* cf, float* logits, uint16_t* tables,
                         hipStream_t s) {
  const long long tiles = ((long long)vg.Z * H * W + 15) / 16;
  long long grid = (tiles + DEEP_WAVES - 1) / DEEP_WAVES;
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  const unsigned g = (unsigned)grid;
  if (net.k_in == K_IN && net.H == 64)
    density_at<64, K_IN>(g, s, K, net, img, H, W, vg, cf, logits, tables);
  else if (net.k_in == K_IN && net.H == 128)
    density_at<128, K_IN>(g, s, K, net, img, H, W, vg, cf, logits, tables);
  else if (net.k_in == K_IN_3D && net.H == 64)
    density_at<64, K_IN_3D>(g, s, K, net, img, H, W, vg, cf, logits, tables);
  else if (net.k_in == K_IN_3D && net.H == 128)
    density_at<128, K_IN_3D>(g, s, K, net, img, H, W, vg, cf, logits, tables);
  else
    return false;
  return true;
}

// ---- decoder ----------------------------------------------------------------

// Device real-time stamps of the last decode (a measurement hook): [0] the
// launch's start, [1 + z] the moment slice z's last pixel was published.
__device__ unsigned long long g_slice_stamps[1 + DEEP_MAX_SLICES];

template <int H, int KIN>
__global__ __launch_bounds__(DEEP_WAVES * 64) void deep_decode_kernel(DeepDecArgs a) {
  __shared__ float s_sm[16 * SM_ROW];
  __shared__ bf16x8 s_act[2 * (H / 32) * 64];
  __shared__ float s_bias[WgNet<H>::NB];
  __shared__ float s_scale[256];
  __shared__ float s_part[256];
  __shared__ __attribute__((aligned(16))) uint16_t s_tab[16 * DEEP_OUT];
  __shared__ int s_err;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  float* sm = s_sm;
  if (threadIdx.x == 0) s_err = deep_check_header(a);
  if (threadIdx.x == 0 && blockIdx.x == 0) g_slice_stamps[0] = __builtin_amdgcn_s_memrealtime();
  deep_stage_biases<H>(a.net, s_bias);
  for (int i = threadIdx.x; i < 256; i += blockDim.x) s_scale[i] = a.K->scale[i];
  WgNet<H> wnet;
  wnet.load(a.net, wave, lane);
  __syncthreads();
  const int err = __builtin_amdgcn_readfirstlane(s_err);
  const int Z = a.vg.Z, lag = a.vg.lag;
  const int HT = Z * a.H, GT = Z * a.G;
  const long long T2 = (long long)a.W + SKEW * (a.H - 1);  // steps of one slice
  // the group this wave decodes, if any: its lanes' states live in registers
  const int g = blockIdx.x * DEEP_WAVES + wave;
  const bool coder = err == 0 && g < GT;
  int r0 = 0, R = 0, J = 0, zg = 0;
  uint32_t n_words = 0, Pw = 0, x = RANS_L;
  const uint16_t* gw16 = nullptr;
  bool bad = false;
  if (coder) {
    r0 = group_row(g, HT, GT);
    R = group_row(g + 1, HT, GT) - r0;
    J = (R + a.L - 1) / a.L;
    zg = r0 / a.H;  // every group lies in one slice
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
  bool alive = err == 0;
  __shared__ int s_alive;
  for (long long t = 0; t < a.T && alive; ++t) {
    // every wave of the workgroup goes on or stops together: a wait that gave
    // up has set the abort flag
    __syncthreads();
    if (threadIdx.x == 0)
      s_alive = __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    alive = __builtin_amdgcn_readfirstlane(s_alive) != 0;
    if (!alive) break;
    // ---- the step's pixels through the network: tile k of the step is the
    // k-th 16-row block of the active rows, slice by slice; one tile per
    // workgroup, its layers split over the four waves
    int z_lo = 0, z_hi = Z - 1;
    if (lag > 0) {
      z_hi = (int)(t / lag < Z - 1 ? t / lag : Z - 1);
      z_lo = (int)(t - T2 + 1 > 0 ? (t - T2 + lag) / lag : 0);
    }
    int k = blockIdx.x, base = 0;
    for (int z = z_lo; z <= z_hi && alive; ++z) {
      const long long tz = t - (long long)lag * z;  // the slice's own step, 0 <= tz < T2
      const int y_lo = (int)(tz - a.W + 1 > 0 ? (tz - a.W + SKEW) / SKEW : 0);
      const int y_hi = (int)(tz / SKEW < a.H - 1 ? tz / SKEW : a.H - 1);
      const int n_act = y_hi - y_lo + 1;
      const int nt = n_act > 0 ? (n_act + 15) / 16 : 0;
      for (; k < base + nt && alive; k += gridDim.x) {
        const int y0 = y_lo + 16 * (k - base);
        // wait for the decoded pixels the tile's windows read: all pixels of
        // steps before this one in rows y0 - 2 .. y0 + 15 and, with the 3-D
        // window, in the slice below's rows the window reaches
        if (wave == 0) {
          deep_delay(a.delay_seed, a.delay_max, 1u, blockIdx.x, (uint32_t)t);
          int fy = -1;
          long long need = 0;
          if (lane < 18) {
            const int r = y0 - 2 + lane;
            const long long first = (long long)SKEW * r + (long long)lag * z;
            if (r >= 0 && r <= y_hi && first <= t - 1) {
              fy = z * a.H + r;
              const long long last = first + a.W - 1;
              need = t - 1 < last ? t - 1 : last;
            }
          } else if (KIN == K_IN_3D && lane >= 32 && lane < 50 && z > 0) {
            const int r = y0 + a.vg.ws - 3 + (lane - 32);
            const long long first = (long long)SKEW * r + (long long)lag * (z - 1);
            if (r >= 0 && r < a.H && first <= t - 1) {
              fy = (z - 1) * a.H + r;
              const long long last = first + a.W - 1;
              need = t - 1 < last ? t - 1 : last;
            }
          }
          uint32_t spins = 0;
          int ok = 1;
          for (;;) {
            const bool ready = fy < 0 || (long long)__hip_atomic_load(
                                             &a.pix_step[fy], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) >= need;
            if (__ballot(!ready) == 0ull) break;
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > a.spin_limit) {
              __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ok = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (lane == 0) s_alive = ok;
        }
        __syncthreads();
        alive = __builtin_amdgcn_readfirstlane(s_alive) != 0;
        if (!alive) break;
        const int y = y0 + p;
        const bool valid = y <= y_hi;
        const int xx = valid ? (int)(tz - (long long)SKEW * y) : 0;
        const bf16x8 xin =
            deep_features<KIN, uint8_t>(s_scale, (const uint8_t*)a.img, a.H, a.W, a.vg.ws, z,
                                        valid ? y : 0, xx, valid, q);
        deep_run_wg<H>(wnet, s_bias, xin, s_act, sm);
        deep_tables_wg(sm, s_part, s_tab);
        if (wave == 0) {
          // the tile's tables to device memory: lane (q, p) copies block q of
          // pixel p's 256 levels
          if (valid) {
            const uint4* src = reinterpret_cast<const uint4*>(s_tab + p * DEEP_OUT + 64 * q);
            uint4* dst = reinterpret_cast<uint4*>(a.tables + (long long)(z * a.H + y) * DEEP_OUT +
                                                  64 * q);
#pragma unroll
            for (int j = 0; j < 8; ++j) dst[j] = src[j];
          }
          deep_delay(a.delay_seed, a.delay_max, 2u, blockIdx.x, (uint32_t)t);
          // the tables out, then the rows' table counters
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (q == 0 && valid)
            __hip_atomic_store(&a.tab_step[z * a.H + y], (int)t, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
      }
      base += nt;
    }
    if (!alive) break;
    // ---- each group decodes its rows' pixels of the step, once their tables
    // are there, and then publishes them (a damaged stream is not decoded but
    // still published, so that nothing waits on it)
    const long long tg = t - (long long)lag * zg;  // the step within the group's slice
    if (coder && tg >= 0 && tg < T2) {
      bool waited = true;
      deep_delay(a.delay_seed, a.delay_max, 3u, (uint32_t)g, (uint32_t)t);
      if (!bad) {
        uint32_t spins = 0;
        for (;;) {
          bool ready = true;
          for (int j = 0; j < J; ++j) {
            const int rr = j * a.L + lane;
            const int Y = r0 + rr;
            const long long xc = tg - (long long)SKEW * (Y - zg * a.H);
            const bool act = lane < a.L && rr < R && xc >= 0 && xc < a.W;
            if (act && __hip_atomic_load(&a.tab_step[Y], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < (int)t)
              ready = false;
          }
          if (__ballot(!ready) == 0ull) break;
          if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
              ++spins > a.spin_limit) {
            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            waited = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      for (int j = 0; j < J && waited && !bad; ++j) {
        const int rr = j * a.L + lane;
        const int Y = r0 + rr;
        const long long xc = tg - (long long)SKEW * (Y - zg * a.H);
        const bool act = lane < a.L && rr < R && xc >= 0 && xc < a.W;
        if (__ballot(act) == 0ull) continue;
        const uint32_t slot = x & 0xFFFFu;
        const uint16_t* tab = a.tables + (long long)(act ? Y : 0) * DEEP_OUT;
        // bucket of 16 levels from the boundaries F(16 k), then the level in it
        int nb = 0;
#pragma unroll
        for (int kk = 1; kk < 16; ++kk) nb += ((uint32_t)tab[16 * kk] <= slot) ? 1 : 0;
        uint32_t Fl[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) Fl[i] = tab[16 * nb + i];
        int cnt = 0;
#pragma unroll
        for (int i = 1; i < 16; ++i) cnt += (Fl[i] <= slot) ? 1 : 0;
        const int v = 16 * nb + cnt;
        uint32_t c = Fl[0], fn = nb < 15 ? (uint32_t)tab[16 * (nb + 1)] : M_TOTAL;
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
        if (act) reinterpret_cast<uint8_t*>(a.img)[(long long)Y * a.W + xc] = (uint8_t)v;
      }
      deep_delay(a.delay_seed, a.delay_max, 4u, (uint32_t)g, (uint32_t)t);
      // the pixels out, then the rows' pixel counters
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (int j = 0; j < J; ++j) {
        const int rr = j * a.L + lane;
        const int Y = r0 + rr;
        const long long xc = tg - (long long)SKEW * (Y - zg * a.H);
        if (lane < a.L && rr < R && xc >= 0 && xc < a.W) {
          __hip_atomic_store(&a.pix_step[Y], (int)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // the slice's last pixel
          if (Y - zg * a.H == a.H - 1 && xc == a.W - 1)
            g_slice_stamps[1 + zg] = __builtin_amdgcn_s_memrealtime();
        }
      }
    }
  }
  if (err != 0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicMax(a.status, err);
    return;
  }
  if (!alive ||
      __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
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
static int decode_residency() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, deep_decode_kernel<H, KIN>,
                                                   DEEP_WAVES * 64, 0) != hipSuccess)
    return 0;
  return per_cu;
}

int deep_slice_stamps(unsigned long long* h_out, int n) {
  if (n < 1 || n > 1 + DEEP_MAX_SLICES) return -1;
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  return hipMemcpyFromSymbol(h_out, HIP_SYMBOL(g_slice_stamps), sizeof(unsigned long long) * n, 0,
                             hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
}

int deep_decode_max_grid(int H, int k_in) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  int per_cu = 0;
  if (k_in == K_IN)
    per_cu = H == 64 ? decode_residency<64, K_IN>() : decode_residency<128, K_IN>();
  else
    per_cu = H == 64 ? decode_residency<64, K_IN_3D>() : decode_residency<128, K_IN_3D>();
  return cus * per_cu;
}

hipError_t launch_deep_decode(const DeepDecArgs& a, int grid, hipStream_t s) {
  DeepDecArgs args = a;
  void* kargs[] = {&args};
  const void* fn = nullptr;
  if (a.net.k_in == K_IN)
    fn = a.net.H == 64 ? (const void*)deep_decode_kernel<64, K_IN>
                       : (const void*)deep_decode_kernel<128, K_IN>;
  else if (a.net.k_in == K_IN_3D)
    fn = a.net.H == 64 ? (const void*)deep_decode_kernel<64, K_IN_3D>
                       : (const void*)deep_decode_kernel<128, K_IN_3D>;
  if (!fn || (a.net.H != 64 && a.net.H != 128)) return hipErrorInvalidValue;
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(DEEP_WAVES * 64), kargs, 0, s);
}

}  // namespace dlic
