// Device-side building blocks of the DLIC hot path for gfx950 (CDNA4).
//
// Everything a pixel's density needs lives here exactly once: the causal
// window, the network tile on MFMA, the mixture head, the FP32 table rule and
// the rANS sub-round steps.  The encoder, the wavefront decoder and the test
// hooks all call these same functions, which is how the paper's requirement
// that encoder and decoder feed identical inputs through identical arithmetic
// (Section II-B, Preprocessor) is kept: every per-pixel value depends only on
// that pixel's own 12 inputs and the weights, through one fixed sequence of
// FP32 operations (no FMA contraction, fixed summation order), and an MFMA
// output column depends only on its own B column.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace dlic {

constexpr int K_IN = 12;
constexpr int N_MIX = 5;
constexpr int N_OUT = 15;
constexpr int SKEW = 3;               // wavefront step t = x + SKEW * y
constexpr uint32_t PROB_BITS = 16;
constexpr uint32_t M_TOTAL = 1u << PROB_BITS;
constexpr uint32_t M_PRIME = M_TOTAL - 256;  // spread over the 256 levels, +1 each
constexpr uint32_t RANS_L = 1u << 16;        // rANS state lives in [2^16, 2^32)
constexpr int LUT_N = 4097;                  // logistic table knots on [-16, 16], step 1/128
constexpr float LOG_SCALE_MIN = -7.0f;
constexpr int HEADER_BYTES = 36;
constexpr uint32_t INACTIVE = 0xFFFFFFFFu;   // cf sentinel: no symbol in this slot

// Format constants uploaded once per device (built on the host).
struct Consts {
  float2 sd[LUT_N];   // (S_j, D_j): knot value and exact slope to the next knot
  float beta[257];    // FP32 bin edges, beta[0] = -inf, beta[256] = +inf
  float scale[256];   // RN32((2v - 255) / 255)
  float scale12[4096];  // RN32((2v - 4095) / 4095), 12-bit samples
};

// Network weights as the kernels see them: row-major [out][in] matrices in
// the model's storage type (FP32, BF16 bit patterns, or FP8 e4m3 codes), FP32
// biases, and for FP8 one FP32 scale per layer (W = scale * code value).
struct DevModel {
  const void *w1, *w2, *w3;
  const float *b1, *b2, *b3;
  const float* wscale;
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// D(16x16) = A(16x4) B(4x16) + C with lane l holding A[l%16][l/16],
// B[l/16][l%16] and D[4*(l/16) + r][l%16] (r = 0..3).
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// D(16x16) = A(16x32) B(32x16) + C in BF16 with FP32 accumulation; lane l
// holds A[l%16][8*(l/16) + e] and B[8*(l/16) + e][l%16] (e = 0..7), and D as
// for mfma_f32.
__device__ __forceinline__ f4 mfma_bf16(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// The same shape with OCP e4m3 operands: byte e of a lane's 64-bit A and B
// is element 8*(l/16) + e, as for mfma_bf16.
__device__ __forceinline__ f4 mfma_fp8(long a, long b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// e4m3 codes of two FP32 values (nearest even, saturating at +-448) in the
// low two bytes.
__device__ __forceinline__ uint32_t cvt_e4m3x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

// Causal window offset of feature k (rows y-2, y-1 at dx -2..2, then (y, x-2), (y, x-1)).
__device__ __forceinline__ int nb_dy(int k) { return k < 5 ? -2 : (k < 10 ? -1 : 0); }
__device__ __forceinline__ int nb_dx(int k) { return k < 5 ? k - 2 : (k < 10 ? k - 7 : k - 12); }

__device__ __forceinline__ float relu(float v) { return v > 0.0f ? v : 0.0f; }

// Hand-over of LDS data between lanes of one wave: a wave-scope release and
// acquire keep the compiler from moving the reads above the writes (the
// hardware already serves one wave's LDS accesses in order; no wait is added).
__device__ __forceinline__ void wave_lds_handover() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Storage types of the weight matrices.
enum WeightType { WT_F32 = 0, WT_BF16 = 1, WT_FP8 = 2, WT_FP8A8 = 4 };

// OCP e4m3 (FN) code -> BF16 bit pattern: bias 7, 3 mantissa bits,
// subnormal step 2^-9; every code is exact in BF16 (exponent bias 127).
__device__ __forceinline__ uint32_t e4m3_bf16_bits(uint32_t b) {
  const uint32_t e = (b >> 3) & 15u, m = b & 7u;
  const uint32_t normal = ((e + 120u) << 7) | (m << 4);
  const uint32_t sub = __float_as_uint((float)m * 0.001953125f) >> 16;
  return (e ? normal : sub) | ((b & 0x80u) << 8);
}

// BF16 bit pattern of element idx of a weight matrix (exact for BF16 and
// FP8 storage), in the low half of the result.
template <int WT>
__device__ __forceinline__ uint32_t weight_bf16_bits(const void* p, long idx) {
  if constexpr (WT == WT_BF16) {
    return ((const uint16_t*)p)[idx];
  } else {
    return e4m3_bf16_bits(((const uint8_t*)p)[idx]);
  }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Eight BF16 bit patterns (element e in half e % 2 of word e / 2) as one operand.
__device__ __forceinline__ bf16x8 pack_bf16x8(const uint32_t* h) {
  const u32x4 w = {h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                   h[6] | (h[7] << 16)};
  return __builtin_bit_cast(bf16x8, w);
}

// -----------------------------------------------------------------------------
// Network tiles: 16 pixels through 12 -> H -> H -> 15 on MFMA.
//
// Activations are the B operand (K x 16 pixels) and weights the A operand
// (16 neurons x K), so a layer's D registers (neuron 16*nt + 4*(l/16) + r of
// pixel l%16) are directly the next layer's B operand: the weights are
// loaded with the matching permutation of their input index.  Every net has
// the same interface:
//   LDS_BYTES            workgroup LDS the net reads its layer-2 weights from
//                        (0 when they live in registers)
//   stage(m, lds, t, n)  thread t of n copies layer-2 weights into LDS
//   load(m, lane)        per-lane weights and biases into registers
//   run(f0, f1, f2, lds) features 4e + l/16 (e = 0, 1, 2) of pixel l%16 in,
//                        outputs 4*(l/16) .. 4*(l/16)+3 of that pixel out.
//   SCRATCH_FLOATS       LDS floats each decoder density wave lends the net
//                        (xs points there before run)
// -----------------------------------------------------------------------------

// FP32 weights, v_mfma_f32_16x16x4f32, biases seed the accumulators.
// Layer-2 weights sit in VGPRs up to H = 64 and in LDS above (64 KB at 128),
// or in LDS at any width with W2L.
template <int H, bool W2L = (H > 64)>
struct NetF32 {
  static constexpr int NT = H / 16;
  static constexpr bool W2_LDS = W2L;
  // few enough VGPRs for three decoder waves per SIMD
  static constexpr bool DEC_WIDE = H <= 32 || (H == 64 && W2L);
  static constexpr int LDS_BYTES = W2_LDS ? NT * NT * 64 * 16 : 0;
  static constexpr int SCRATCH_FLOATS = 0;  // per-wave LDS scratch of the decoder
  float a1[NT][3];
  float a2[W2_LDS ? 1 : NT][W2_LDS ? 1 : NT * 4];
  float a3[NT * 4];
  float c1[NT][4], c2[NT][4], c3[4];

  // LDS order: f4 index (n2 * NT + n1) * 64 + lane holds r = 0..3.
  __device__ __forceinline__ static void stage(const DevModel& m, void* lds, int t, int n) {
    if constexpr (W2_LDS) {
      const float* w2 = (const float*)m.w2;
      float* d = (float*)lds;
      for (int idx = t; idx < NT * NT * 256; idx += n) {
        const int r = idx & 3, lane = (idx >> 2) & 63, blk = idx >> 8;
        const int n2 = blk / NT, n1 = blk - n2 * NT;
        d[idx] = w2[(16 * n2 + (lane & 15)) * H + 16 * n1 + 4 * (lane >> 4) + r];
      }
    }
  }

  __device__ __forceinline__ void load(const DevModel& m, int lane) {
    const float* w1 = (const float*)m.w1;
    const float* w2 = (const float*)m.w2;
    const float* w3 = (const float*)m.w3;
    const int i = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) a1[nt][kk] = w1[(16 * nt + i) * K_IN + 4 * kk + q];
    if constexpr (!W2_LDS) {
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < NT; ++n1)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            a2[n2][n1 * 4 + r] = w2[(16 * n2 + i) * H + 16 * n1 + 4 * q + r];
    }
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        a3[n2 * 4 + r] = (i < N_OUT) ? w3[i * H + 16 * n2 + 4 * q + r] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        c1[nt][r] = m.b1[16 * nt + 4 * q + r];
        c2[nt][r] = m.b2[16 * nt + 4 * q + r];
      }
      c3[r] = (4 * q + r < N_OUT) ? m.b3[4 * q + r] : 0.0f;
    }
  }

  __device__ __forceinline__ f4 run(float f0, float f1, float f2, const void* lds) const {
    f4 h1[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      f4 acc = {c1[nt][0], c1[nt][1], c1[nt][2], c1[nt][3]};
      acc = mfma_f32(a1[nt][0], f0, acc);
      acc = mfma_f32(a1[nt][1], f1, acc);
      acc = mfma_f32(a1[nt][2], f2, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[nt][r] = relu(acc[r]);
    }
    f4 h2[NT];
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      f4 acc = {c2[n2][0], c2[n2][1], c2[n2][2], c2[n2][3]};
#pragma unroll
      for (int n1 = 0; n1 < NT; ++n1) {
        f4 w;
        if constexpr (W2_LDS) {
          w = ((const f4*)lds)[(n2 * NT + n1) * 64 + lane];
        } else {
          w = f4{a2[n2][n1 * 4], a2[n2][n1 * 4 + 1], a2[n2][n1 * 4 + 2], a2[n2][n1 * 4 + 3]};
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = mfma_f32(w[r], h1[n1][r], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[n2][r] = relu(acc[r]);
    }
    if constexpr (H >= 64) {
      // four K quarters (neuron tiles NT/4 g .. NT/4 g + NT/4 - 1), each its
      // own chain, the first seeded with the bias; summed as
      // ((q0 + q1) + q2) + q3
      constexpr int TQ = NT / 4;
      f4 oq[4] = {{c3[0], c3[1], c3[2], c3[3]}, {0.0f, 0.0f, 0.0f, 0.0f},
                  {0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          oq[n2 / TQ] = mfma_f32(a3[n2 * 4 + r], h2[n2][r], oq[n2 / TQ]);
      f4 o;
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = ((oq[0][e] + oq[1][e]) + oq[2][e]) + oq[3][e];
      return o;
    }
    f4 o = {c3[0], c3[1], c3[2], c3[3]};
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r) o = mfma_f32(a3[n2 * 4 + r], h2[n2][r], o);
    return o;
  }

  // Largest hidden activation of each layer among this lane's values (the
  // ranges that the FP8-activation net's multipliers are chosen from).
  __device__ __forceinline__ void hidden_max(float f0, float f1, float f2, const void* lds,
                                             float& mx1, float& mx2) const {
    f4 h1[NT];
    mx1 = 0.0f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      f4 acc = {c1[nt][0], c1[nt][1], c1[nt][2], c1[nt][3]};
      acc = mfma_f32(a1[nt][0], f0, acc);
      acc = mfma_f32(a1[nt][1], f1, acc);
      acc = mfma_f32(a1[nt][2], f2, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h1[nt][r] = relu(acc[r]);
        mx1 = fmaxf(mx1, h1[nt][r]);
      }
    }
    mx2 = 0.0f;
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      f4 acc = {c2[n2][0], c2[n2][1], c2[n2][2], c2[n2][3]};
#pragma unroll
      for (int n1 = 0; n1 < NT; ++n1) {
        f4 w;
        if constexpr (W2_LDS) {
          w = ((const f4*)lds)[(n2 * NT + n1) * 64 + lane];
        } else {
          w = f4{a2[n2][n1 * 4], a2[n2][n1 * 4 + 1], a2[n2][n1 * 4 + 2], a2[n2][n1 * 4 + 3]};
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = mfma_f32(w[r], h1[n1][r], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) mx2 = fmaxf(mx2, relu(acc[r]));
    }
  }
};

// The 12-H-H-15 FP32 net (H = 64 or 128) for decoder tiles of at most 4
// pixels, with results bit-identical to NetF32<H> (the encoder's form).
//
// The FP32 MFMAs compute each output as a chain of correctly rounded fused
// multiply-adds in K order: v_mfma_f32_16x16x4f32 takes its four K slots in
// order, v_mfma_f32_4x4x1f32 one product (checked on the MI355X for 512 000
// results of each form against scalar fma chains, operands from 2^-8 to 2^8
// with both signs).  All three layers therefore run as one-product steps of
// the 4x4 form in NetF32's K order, on the 4 pixels a tile has, where the
// 16x16 form computes 16 pixels: a quarter of the MFMA time.  The 16 blocks of
// the 4x4 form are 16 groups of 4 output neurons (lane 4b + i is neuron 4b + i
// of the A operand, lane 4b + j pixel j of the B operand and of D); one
// accumulator covers 64 neurons (two at H = 128).  Activations change layout
// through the wave's own LDS scratch (one row of ROW floats per pixel).
//
// NetF32's layer-2 order: MFMA (n1, r) takes slots q = 0..3, i.e. layer-1
// neurons 16 n1 + 4 q + r, so chain step c takes neuron kc(c).  Layer 3 (15
// outputs) is summed in four K quarters of H/4 neurons on both sides.
__device__ __forceinline__ f4 mfma_f32_4x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

template <int H_, bool W2R = false>
struct NetF32x4 {
  static_assert(H_ == 64 || H_ == 128, "4-pixel form for 64 or 128 neurons");
  static_assert(!W2R || H_ == 64, "layer-2 weights in registers at 64 neurons only");
  static constexpr int H = H_, NT = H / 16;
  static constexpr int HALVES = H / 64;               // accumulators of 64 neurons
  static constexpr int QS = H / 4;                    // chain steps of a layer-3 quarter
  static constexpr bool DEC_WIDE = false;             // 8 waves per decoder workgroup
  // W2 in chain order: in registers with W2R (64 per lane at H = 64; two waves
  // per SIMD leave room), else in LDS
  static constexpr bool W2_REG = W2R;
  static constexpr int LDS_BYTES = W2_REG ? 0 : H * H * 4;
  static constexpr int ROW = H + 4;                   // scratch floats per pixel row
  static constexpr int SCRATCH_FLOATS = 2 * 4 * ROW;  // layer-1 rows, then layer-2 rows
  float a1[HALVES][K_IN];  // W1[64 h + lane][k]
  float a2[W2_REG ? H : 1];  // W2[lane][kc(c)] along layer 2's chain (H = 64)
  float a3[QS];            // W3[lane % 16][k] along quarter lane / 16 of layer 3's chain
  float c1[HALVES][4], c2[HALVES][4], c3[4];
  float* xs = nullptr;

  __host__ __device__ static constexpr int kc(int c) {
    return 16 * (c / 16) + 4 * (c % 4) + (c % 16) / 4;
  }

  // H = 128: f4 index cp * 64 + lane holds, for steps c = 2 cp and 2 cp + 1
  // in turn, W2[lane][kc(c)] and W2[64 + lane][kc(c)].  H = 64: f4 index
  // cq * 64 + lane holds W2[lane][kc(c)] for steps c = 4 cq .. 4 cq + 3.
  __device__ __forceinline__ static void stage(const DevModel& m, void* lds, int t, int n) {
    if constexpr (W2_REG) return;
    const float* w2 = (const float*)m.w2;
    float* d = (float*)lds;
    for (int idx = t; idx < H * H; idx += n) {
      const int e = idx & 3, lane = (idx >> 2) & 63, cp = idx >> 8;
      if constexpr (HALVES == 2) {
        const int c = 2 * cp + (e >> 1), half = e & 1;
        d[idx] = w2[(64 * half + lane) * H + kc(c)];
      } else {
        d[idx] = w2[lane * H + kc(4 * cp + e)];
      }
    }
  }

  __device__ __forceinline__ void load(const DevModel& m, int lane) {
    const float* w1 = (const float*)m.w1;
    const float* w3 = (const float*)m.w3;
    const int i = lane & 15, q = lane >> 4;
#pragma unroll
    for (int h = 0; h < HALVES; ++h)
#pragma unroll
      for (int k = 0; k < K_IN; ++k) a1[h][k] = w1[(64 * h + lane) * K_IN + k];
    if constexpr (W2_REG) {
      const float* w2 = (const float*)m.w2;
#pragma unroll
      for (int c = 0; c < H; ++c) a2[c] = w2[lane * H + kc(c)];
    }
#pragma unroll
    for (int st = 0; st < QS; ++st)
      a3[st] = (i < N_OUT) ? w3[i * H + k3(q, st)] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int h = 0; h < HALVES; ++h) {
        c1[h][r] = m.b1[64 * h + 4 * (lane >> 2) + r];
        c2[h][r] = m.b2[64 * h + 4 * (lane >> 2) + r];
      }
      const int o3 = 4 * ((lane >> 2) & 3) + r;  // output of D register r
      c3[r] = (q == 0 && o3 < N_OUT) ? m.b3[o3] : 0.0f;
    }
  }

  // Layer 3 in NetF32<H>'s four K quarters: step st of quarter g takes neuron
  // k3(g, st) (MFMA (n2, r) of the 16x16 form, n2 in quarter g, takes slots
  // q = 0..3, neurons 16 n2 + 4 q + r), and l3pos is where neuron n sits in
  // the quarters' chains (QS g + st).
  __host__ __device__ static constexpr int k3(int g, int st) {
    return 16 * ((QS / 16) * g + st / 16) + 4 * (st & 3) + ((st >> 2) & 3);
  }
  __host__ __device__ static constexpr int l3pos(int n) {
    return 16 * (n >> 4) + 4 * (n & 3) + ((n >> 2) & 3);
  }

  // Layer 1 in two parts.  A decoder knows every feature of a pixel's window
  // one wavefront step early except 9 (up-right) and 11 (left): l1_pre takes
  // f0 and f1 of every lane group and f2 of groups 0 and 2 (features 8 and 10)
  // and runs steps 0..8 of layer 1's chain; finish adds f2 of groups 1 and 3
  // (features 9 and 11), runs steps 9..11 and the rest of the net.  The chain
  // order is run's, so are the results, bit for bit.
  struct L1 {
    f4 acc[HALVES];
  };

  __device__ __forceinline__ L1 l1_pre(float f0, float f1, float f2) const {
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int p = lane & 15, q = lane >> 4, j = lane & 3;
    // the 12 features of pixel j in every lane 4 b + j (K order 0..11, as the
    // 16x16 form's slots take them), through the layer-2 rows of the scratch
    // (free until layer 2 ends)
    float* ft = xs + 4 * ROW;
    if (p < 4) {
      ft[p * ROW + q] = f0;
      ft[p * ROW + 4 + q] = f1;
      if ((q & 1) == 0) ft[p * ROW + 8 + q] = f2;
    }
    wave_lds_handover();
    const f4 fa = *reinterpret_cast<const f4*>(&ft[j * ROW]);
    const f4 fb = *reinterpret_cast<const f4*>(&ft[j * ROW + 4]);
    const float f8 = ft[j * ROW + 8];
    const float fv[9] = {fa[0], fa[1], fa[2], fa[3], fb[0], fb[1], fb[2], fb[3], f8};
    L1 l;
#pragma unroll
    for (int h = 0; h < HALVES; ++h) l.acc[h] = f4{c1[h][0], c1[h][1], c1[h][2], c1[h][3]};
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int h = 0; h < HALVES; ++h) l.acc[h] = mfma_f32_4x4(a1[h][k], fv[k], l.acc[h]);
    return l;
  }

  // Features as NetF32::run; the outputs of pixels 0..3 (lanes l % 16 < 4)
  // are NetF32<H>'s, the other lanes' are unspecified.
  __device__ __forceinline__ f4 run(float f0, float f1, float f2, const void* lds) const {
    return finish(l1_pre(f0, f1, f2), f2, lds);
  }

  __device__ __forceinline__ f4 finish(L1 l, float f2, const void* lds) const {
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int p = lane & 15, q = lane >> 4, j = lane & 3;
    float* h1t = xs;            // [pixel][chain step]
    float* h2t = xs + 4 * ROW;  // [pixel][neuron]
    float* ft = h2t;
    if (p < 4 && (q & 1) != 0) ft[p * ROW + 8 + q] = f2;
    wave_lds_handover();
    {
      // steps 9..11, then neuron n = 16 n1 + 4 q + r goes to chain step
      // 16 n1 + 4 r + q of layer 2
      const f4 fc = *reinterpret_cast<const f4*>(&ft[j * ROW + 8]);
#pragma unroll
      for (int k = 9; k < K_IN; ++k)
#pragma unroll
        for (int h = 0; h < HALVES; ++h) l.acc[h] = mfma_f32_4x4(a1[h][k], fc[k - 8], l.acc[h]);
      // lane 4 b + j holds neurons 64 h + 4 b + i of pixel j
      const int b = lane >> 2;
      const int c0 = 16 * (b >> 2) + (b & 3);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int h = 0; h < HALVES; ++h) h1t[j * ROW + 64 * h + c0 + 4 * i] = relu(l.acc[h][i]);
    }
    wave_lds_handover();
    // layer 2: the chain of H steps, both neuron halves at H = 128
    const f4* w = reinterpret_cast<const f4*>(lds);
    f4 lo = {c2[0][0], c2[0][1], c2[0][2], c2[0][3]};
    f4 hi = {c2[HALVES - 1][0], c2[HALVES - 1][1], c2[HALVES - 1][2], c2[HALVES - 1][3]};
#pragma unroll
    for (int c4 = 0; c4 < H / 4; ++c4) {
      const f4 hv = *reinterpret_cast<const f4*>(&h1t[j * ROW + 4 * c4]);
      if constexpr (HALVES == 2) {
        const f4 wa = w[(2 * c4) * 64 + lane];
        const f4 wb = w[(2 * c4 + 1) * 64 + lane];
        lo = mfma_f32_4x4(wa[0], hv[0], lo);
        hi = mfma_f32_4x4(wa[1], hv[0], hi);
        lo = mfma_f32_4x4(wa[2], hv[1], lo);
        hi = mfma_f32_4x4(wa[3], hv[1], hi);
        lo = mfma_f32_4x4(wb[0], hv[2], lo);
        hi = mfma_f32_4x4(wb[1], hv[2], hi);
        lo = mfma_f32_4x4(wb[2], hv[3], lo);
        hi = mfma_f32_4x4(wb[3], hv[3], hi);
      } else {
        const f4 wa = W2_REG ? f4{a2[4 * c4], a2[4 * c4 + 1], a2[4 * c4 + 2], a2[4 * c4 + 3]}
                             : w[c4 * 64 + lane];
        lo = mfma_f32_4x4(wa[0], hv[0], lo);
        lo = mfma_f32_4x4(wa[1], hv[1], lo);
        lo = mfma_f32_4x4(wa[2], hv[2], lo);
        lo = mfma_f32_4x4(wa[3], hv[3], lo);
      }
    }
    // lane 4 b + j holds neurons 64 h + 4 b + i of pixel j; they go to their
    // places in layer 3's chains
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 4 * (lane >> 2) + i;
      h2t[j * ROW + l3pos(n)] = relu(lo[i]);
      if constexpr (HALVES == 2) h2t[j * ROW + l3pos(64 + n)] = relu(hi[i]);
    }
    wave_lds_handover();
    // layer 3 on the 4x4 form: block b = 4 g + og is quarter g of outputs
    // 4 og .. 4 og + 3, so lane 16 g + 4 og + j accumulates that quarter for
    // pixel j; the quarters then meet in the 16x16 layout
    f4 o3 = {c3[0], c3[1], c3[2], c3[3]};
#pragma unroll
    for (int s4 = 0; s4 < QS / 4; ++s4) {
      const f4 hv = *reinterpret_cast<const f4*>(&h2t[j * ROW + QS * q + 4 * s4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) o3 = mfma_f32_4x4(a3[4 * s4 + e], hv[e], o3);
    }
    float* part = h1t;  // free once layer 2 has read it
    *reinterpret_cast<f4*>(&part[4 * lane]) = o3;
    wave_lds_handover();
    f4 o = {0.0f, 0.0f, 0.0f, 0.0f};
    if (p < 4) {
      // outputs 4 q .. 4 q + 3 of pixel p: quarter g sits at lane 16 g + 4 q + p
      f4 v[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) v[g] = *reinterpret_cast<const f4*>(&part[4 * (16 * g + 4 * q + p)]);
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = ((v[0][e] + v[1][e]) + v[2][e]) + v[3][e];
    }
    return o;
  }
};

// BF16 operands with FP32 accumulation on v_mfma_f32_16x16x32_bf16.  Inputs
// and hidden activations are rounded to BF16 (round to nearest even) before
// each product; biases and accumulators stay FP32.
//
// WT_BF16: weights are BF16; the bias seeds the accumulator.
// WT_FP8:  weights are e4m3 codes, widened exactly to BF16; a layer's FP32
//          scale multiplies the finished accumulator, then the bias is added
//          (z = scale * (Q a) + b).
//
// K slots: a lane holds slots 8*(l/16) + e.  Layer 1 puts feature 4e + l/16
// in slot e < 3 (zero for e >= 3), so every lane gathers three features.
// Layers 2 and 3 take k-step s from the D registers of neuron tiles 2s
// (e = r) and 2s + 1 (e = 4 + r): slot e of lane group q is neuron
// 32s + 16*(e/4) + 4q + e%4.  Layer-2 weights sit in VGPRs by default; with
// W2_LDS they are read from LDS (32 KB at H = 128).
template <int H, int WT, bool W2_LDS_>
struct NetBF16 {
  static constexpr int NT = H / 16, NK = H / 32;
  static constexpr bool W2_LDS = W2_LDS_;
  static constexpr bool SCALED = WT == WT_FP8;
  static constexpr bool DEC_WIDE = H <= 64;
  static constexpr int LDS_BYTES = W2_LDS ? NT * NK * 64 * 16 : 0;
  static constexpr int SCRATCH_FLOATS = 0;  // per-wave LDS scratch of the decoder
  bf16x8 a1[NT];
  bf16x8 a2[W2_LDS ? 1 : NT][W2_LDS ? 1 : NK];
  bf16x8 a3[NK];
  float c1[NT][4], c2[NT][4], c3[4];
  float s1, s2, s3;

  __device__ __forceinline__ static int slot_neuron(int s, int q, int e) {
    return 32 * s + 16 * (e >> 2) + 4 * q + (e & 3);
  }

  // LDS order: bf16x8 index (n2 * NK + s) * 64 + lane.
  __device__ __forceinline__ static void stage(const DevModel& m, void* lds, int t, int n) {
    if constexpr (W2_LDS) {
      uint16_t* d = (uint16_t*)lds;
      for (int idx = t; idx < NT * NK * 512; idx += n) {
        const int e = idx & 7, lane = (idx >> 3) & 63, blk = idx >> 9;
        const int n2 = blk / NK, s = blk - n2 * NK;
        d[idx] = (uint16_t)weight_bf16_bits<WT>(
            m.w2, (16 * n2 + (lane & 15)) * H + slot_neuron(s, lane >> 4, e));
      }
    }
  }

  __device__ __forceinline__ void load(const DevModel& m, int lane) {
    const int i = lane & 15, q = lane >> 4;
    uint32_t h[8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        h[e] = e < 3 ? weight_bf16_bits<WT>(m.w1, (16 * nt + i) * K_IN + 4 * e + q) : 0u;
      a1[nt] = pack_bf16x8(h);
    }
    if constexpr (!W2_LDS) {
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int s = 0; s < NK; ++s) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            h[e] = weight_bf16_bits<WT>(m.w2, (16 * n2 + i) * H + slot_neuron(s, q, e));
          a2[n2][s] = pack_bf16x8(h);
        }
    }
#pragma unroll
    for (int s = 0; s < NK; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        h[e] = i < N_OUT ? weight_bf16_bits<WT>(m.w3, i * H + slot_neuron(s, q, e)) : 0u;
      a3[s] = pack_bf16x8(h);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        c1[nt][r] = m.b1[16 * nt + 4 * q + r];
        c2[nt][r] = m.b2[16 * nt + 4 * q + r];
      }
      c3[r] = (4 * q + r < N_OUT) ? m.b3[4 * q + r] : 0.0f;
    }
    if constexpr (SCALED) {
      s1 = m.wscale[0];
      s2 = m.wscale[1];
      s3 = m.wscale[2];
    } else {
      s1 = s2 = s3 = 1.0f;
    }
  }

  // Accumulator start and finished pre-activation of one layer.
  __device__ __forceinline__ static f4 seed(const float* c) {
    if constexpr (SCALED) return f4{0.0f, 0.0f, 0.0f, 0.0f};
    return f4{c[0], c[1], c[2], c[3]};
  }
  __device__ __forceinline__ static float finish(float acc, float scale, float bias) {
    if constexpr (SCALED) return acc * scale + bias;
    return acc;
  }

  __device__ __forceinline__ f4 run(float f0, float f1, float f2, const void* lds) const {
    const __bf16 zero = (__bf16)0.0f;
    const bf16x8 x = {(__bf16)f0, (__bf16)f1, (__bf16)f2, zero, zero, zero, zero, zero};
    float h1[NT][4];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      f4 acc = mfma_bf16(a1[nt], x, seed(c1[nt]));
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[nt][r] = relu(finish(acc[r], s1, c1[nt][r]));
    }
    bf16x8 b1[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) b1[s][e] = (__bf16)h1[2 * s + (e >> 2)][e & 3];
    float h2[NT][4];
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      f4 acc = seed(c2[n2]);
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        bf16x8 w;
        if constexpr (W2_LDS) {
          w = ((const bf16x8*)lds)[(n2 * NK + s) * 64 + lane];
        } else {
          w = a2[n2][s];
        }
        acc = mfma_bf16(w, b1[s], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[n2][r] = relu(finish(acc[r], s2, c2[n2][r]));
    }
    bf16x8 b2[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) b2[s][e] = (__bf16)h2[2 * s + (e >> 2)][e & 3];
    f4 acc = seed(c3);
#pragma unroll
    for (int s = 0; s < NK; ++s) acc = mfma_bf16(a3[s], b2[s], acc);
    f4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = finish(acc[r], s3, c3[r]);
    return o;
  }
};

// FP8 weights and FP8 activations (W8A8) on v_mfma_f32_16x16x32_fp8_fp8.
// Weights are e4m3 codes with one FP32 scale s_l per layer; the input of
// layer l is multiplied by a power of two m_l (exact) and rounded to e4m3, so
// z = (s_l / m_l) * (Q_l a_q) + b with s_l / m_l exact as well.  The K slots
// are those of NetBF16.  wscale holds s_1, s_2, s_3, m_1, m_2, m_3.
template <int H, bool W2_LDS_>
struct NetFP8A {
  static constexpr int NT = H / 16, NK = H / 32;
  static constexpr bool W2_LDS = W2_LDS_;
  static constexpr bool DEC_WIDE = H <= 64;
  static constexpr int LDS_BYTES = W2_LDS ? NT * NK * 64 * 8 : 0;
  static constexpr int SCRATCH_FLOATS = 0;  // per-wave LDS scratch of the decoder
  long a1[NT];
  long a2[W2_LDS ? 1 : NT][W2_LDS ? 1 : NK];
  long a3[NK];
  float c1[NT][4], c2[NT][4], c3[4];
  float d1, d2, d3, m1, m2, m3;

  __device__ __forceinline__ static int slot_neuron(int s, int q, int e) {
    return 32 * s + 16 * (e >> 2) + 4 * q + (e & 3);
  }
  __device__ __forceinline__ static long w8(const void* p, long idx) {
    return (long)((const uint8_t*)p)[idx];
  }

  // LDS order: 64-bit word (n2 * NK + s) * 64 + lane.
  __device__ __forceinline__ static void stage(const DevModel& m, void* lds, int t, int n) {
    if constexpr (W2_LDS) {
      uint8_t* d = (uint8_t*)lds;
      for (int idx = t; idx < NT * NK * 512; idx += n) {
        const int e = idx & 7, lane = (idx >> 3) & 63, blk = idx >> 9;
        const int n2 = blk / NK, s = blk - n2 * NK;
        d[idx] = ((const uint8_t*)m.w2)[(16 * n2 + (lane & 15)) * H + slot_neuron(s, lane >> 4, e)];
      }
    }
  }

  __device__ __forceinline__ void load(const DevModel& m, int lane) {
    const int i = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      long v = 0;
#pragma unroll
      for (int e = 0; e < 3; ++e) v |= w8(m.w1, (16 * nt + i) * K_IN + 4 * e + q) << (8 * e);
      a1[nt] = v;
    }
    if constexpr (!W2_LDS) {
#pragma unroll
      for (int n2 = 0; n2 < NT; ++n2)
#pragma unroll
        for (int s = 0; s < NK; ++s) {
          long v = 0;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            v |= w8(m.w2, (16 * n2 + i) * H + slot_neuron(s, q, e)) << (8 * e);
          a2[n2][s] = v;
        }
    }
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      long v = 0;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (i < N_OUT) v |= w8(m.w3, i * H + slot_neuron(s, q, e)) << (8 * e);
      a3[s] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        c1[nt][r] = m.b1[16 * nt + 4 * q + r];
        c2[nt][r] = m.b2[16 * nt + 4 * q + r];
      }
      c3[r] = (4 * q + r < N_OUT) ? m.b3[4 * q + r] : 0.0f;
    }
    m1 = m.wscale[3];
    m2 = m.wscale[4];
    m3 = m.wscale[5];
    d1 = m.wscale[0] / m1;  // exact: m is a power of two
    d2 = m.wscale[1] / m2;
    d3 = m.wscale[2] / m3;
  }

  // e4m3 codes of 8 activations (two tiles' D registers) times the layer's
  // power-of-two multiplier, in the K-slot order of slot_neuron.
  __device__ __forceinline__ static long pack8(const float* lo, const float* hi, float mul) {
    const uint32_t w0 = cvt_e4m3x2(lo[0] * mul, lo[1] * mul) | (cvt_e4m3x2(lo[2] * mul, lo[3] * mul) << 16);
    const uint32_t w1 = cvt_e4m3x2(hi[0] * mul, hi[1] * mul) | (cvt_e4m3x2(hi[2] * mul, hi[3] * mul) << 16);
    return (long)((uint64_t)w0 | ((uint64_t)w1 << 32));
  }

  __device__ __forceinline__ f4 run(float f0, float f1, float f2, const void* lds) const {
    const long x = (long)(cvt_e4m3x2(f0 * m1, f1 * m1) | (cvt_e4m3x2(f2 * m1, 0.0f) << 16));
    float h1[NT][4];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const f4 acc = mfma_fp8(a1[nt], x, f4{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[nt][r] = relu(acc[r] * d1 + c1[nt][r]);
    }
    long b1[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) b1[s] = pack8(h1[2 * s], h1[2 * s + 1], m2);
    float h2[NT][4];
    const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int n2 = 0; n2 < NT; ++n2) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        long w;
        if constexpr (W2_LDS) {
          w = ((const long*)lds)[(n2 * NK + s) * 64 + lane];
        } else {
          w = a2[n2][s];
        }
        acc = mfma_fp8(w, b1[s], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[n2][r] = relu(acc[r] * d2 + c2[n2][r]);
    }
    long b2[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) b2[s] = pack8(h2[2 * s], h2[2 * s + 1], m3);
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NK; ++s) acc = mfma_fp8(a3[s], b2[s], acc);
    f4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = acc[r] * d3 + c3[r];
    return o;
  }
};

// -----------------------------------------------------------------------------
// Mixture head and the FP32 table rule.
// -----------------------------------------------------------------------------
// Mixture of one pixel in the form the table rule consumes: weights pi and
// the affine map u = beta * A + B of each component's table coordinate
// (A = 128 inv_s, B = 2048 - mu A, so u = 128 (beta - mu) inv_s + 2048).
struct Mix {
  float pi[N_MIX], A[N_MIX], B[N_MIX];
};

// pi = softmax(o[0:5]) (one reciprocal of the sum, then products);
// mu = o[5:10]; inv_s = exp(-max(o[10:15], -7)).
__device__ __forceinline__ Mix mixture_head(const float* o) {
  Mix p;
  float m = o[0];
#pragma unroll
  for (int k = 1; k < N_MIX; ++k) m = fmaxf(m, o[k]);
  float e[N_MIX], s = 0.0f;
#pragma unroll
  for (int k = 0; k < N_MIX; ++k) {
    e[k] = expf(o[k] - m);
    s = s + e[k];
  }
  const float rs = 1.0f / s;
#pragma unroll
  for (int k = 0; k < N_MIX; ++k) {
    p.pi[k] = e[k] * rs;
    const float inv_s = expf(-fmaxf(o[2 * N_MIX + k], LOG_SCALE_MIN));
    p.A[k] = inv_s * 128.0f;
    p.B[k] = 2048.0f - o[N_MIX + k] * p.A[k];
  }
  return p;
}

// Table logistic at table coordinate u: piecewise linear through RN32(sigma)
// knots, monotone by construction (non-negative exact slopes, each segment
// ends on the next knot; the last knot has slope 0).
__device__ __forceinline__ float sigma_hat(float u, const float2* sd) {
  u = u > 0.0f ? u : 0.0f;
  u = fminf(u, 4096.0f);
  const int j = (int)u;
  const float w = __builtin_amdgcn_fractf(u);  // u - floor(u), exact for u >= 0
  const float2 e = sd[j];
  return e.x + w * e.y;
}

// Mixture CDF at bin edge b in the format's order: two partial sums, the
// first three components and the last two, each left to right, then their
// sum.  (The split lets a decoder evaluate the parts on two half-waves.)
__device__ __forceinline__ float cdf_part(float b, const float* pi, const float* A, const float* B,
                                          int n, const float2* sd) {
  float s = pi[0] * sigma_hat(b * A[0] + B[0], sd);
#pragma unroll
  for (int k = 1; k < n; ++k) s = s + pi[k] * sigma_hat(b * A[k] + B[k], sd);
  return s;
}

__device__ __forceinline__ float cdf_C(float b, const Mix& p, const float2* sd) {
  const float lo = cdf_part(b, p.pi, p.A, p.B, 3, sd);
  const float hi = cdf_part(b, p.pi + 3, p.A + 3, p.B + 3, 2, sd);
  return lo + hi;
}

// F(v) = v + min(M', floor(C * M')) from C = C(beta_v).
__device__ __forceinline__ uint32_t F_of_C(int v, float C) {
  uint32_t q = (uint32_t)(C * 65280.0f);
  q = min(q, M_PRIME);
  return (uint32_t)v + q;
}

// Cumulative frequency F(v) = v + min(M', floor(C(beta_v) * M')), F(0) = 0,
// F(256) = 2^16.
__device__ __forceinline__ uint32_t cdf_F(int v, const Mix& p, const float2* sd,
                                          const float* beta) {
  if (v <= 0) return 0u;
  if (v >= 256) return M_TOTAL;
  return F_of_C(v, cdf_C(beta[v], p, sd));
}

// F(v) for 0 < v < 256 with the bin edge beta_v already at hand.
__device__ __forceinline__ uint32_t cdf_F_at(int v, float b, const Mix& p, const float2* sd) {
  return F_of_C(v, cdf_C(b, p, sd));
}

// Largest v with F(v) <= slot, by 8 halvings of [0, 256); returns (v, c, f).
template <class Fn>
__device__ __forceinline__ void find_symbol(uint32_t slot, Fn F, int& v, uint32_t& c,
                                            uint32_t& f) {
  int lo = 0, hi = 256;
  uint32_t Flo = 0, Fhi = M_TOTAL;
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const int mid = (lo + hi) >> 1;
    const uint32_t Fm = F(mid);
    if (Fm <= slot) {
      lo = mid;
      Flo = Fm;
    } else {
      hi = mid;
      Fhi = Fm;
    }
  }
  v = lo;
  c = Flo;
  f = Fhi - Flo;
}

// -----------------------------------------------------------------------------
// rANS (32-bit state, 16-bit words), one sub-round = one wave ballot.
// -----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// x' = floor(x / f) * 2^16 + x mod f + c for x < f * 2^16.  The quotient
// (< 2^16) comes from an FP32 reciprocal estimate within 0.02 of x / f and
// one integer correction step, all by selects (no branches); q * f < 2^32
// with both factors below 2^24, so the 24-bit multiplier is exact.
__device__ __forceinline__ uint32_t rans_enc_update(uint32_t x, uint32_t c, uint32_t f) {
  const float rcp = __builtin_amdgcn_rcpf((float)f);
  uint32_t q = (uint32_t)((float)x * rcp);
  int32_t r = (int32_t)(x - __umul24(q, f));
  const bool below = r < 0;
  q = below ? q - 1u : q;
  r = below ? r + (int32_t)f : r;
  const bool above = r >= (int32_t)f;
  q = above ? q + 1u : q;
  r = above ? r - (int32_t)f : r;
  return (q << 16) + (uint32_t)r + c;
}

// Encoder sub-round (reverse walk).  Lanes with a symbol renormalise, then
// push their low words so that reading forward gives ascending lane order;
// words are written below write index Q, which is returned lowered.
__device__ __forceinline__ uint32_t rans_enc_subround(uint32_t& x, bool act, uint32_t c,
                                                      uint32_t f, uint16_t* out, uint32_t Q) {
  const bool ren = act && (x >= (f << 16));
  const uint64_t mask = __ballot(ren);
  const uint32_t cnt = (uint32_t)__popcll(mask);
  if (ren) out[Q - cnt + lane_rank(mask)] = (uint16_t)(x & 0xFFFFu);
  const uint32_t xs = ren ? (x >> 16) : x;
  const uint32_t xn = rans_enc_update(xs, c, f);
  x = act ? xn : xs;
  return Q - cnt;
}

// Decoder renormalisation for one sub-round: lanes whose state fell below
// 2^16 take the next words in ascending lane order.  word(pos) fetches the
// pos-th word of the group stream; reads at or past n_words set `over`.
template <class Word>
__device__ __forceinline__ uint32_t rans_dec_renorm(uint32_t& x, bool act, uint32_t P,
                                                    uint32_t n_words, Word word, bool& over) {
  const bool ren = act && (x < RANS_L);
  const uint64_t mask = __ballot(ren);
  if (ren) {
    const uint32_t pos = P + lane_rank(mask);
    uint32_t wd = 0;
    if (pos < n_words)
      wd = word(pos);
    else
      over = true;
    x = (x << 16) | wd;
  }
  return P + (uint32_t)__popcll(mask);
}

// Row strip of group g: [g*H/G, (g+1)*H/G).
__device__ __forceinline__ int group_row(int g, int H, int G) {
  return (int)(((long long)g * H) / G);
}

// With S strips per group the image is cut into S*G strips and group g codes
// strips g, G + g, ..., (S - 1) G + g in that order.  rows: the rows of those
// strips; before: the rows of the strips of groups 0 .. g-1 (a group's word
// scratch follows theirs).  S = 1 gives the contiguous strip of group_row.
__device__ __forceinline__ void group_span(int g, int H, int G, int S, int& before, int& rows) {
  const int GS = G * S;
  before = 0;
  rows = 0;
  for (int s = 0; s < S; ++s) {
    const int b = s * G + g;
    before += group_row(b, H, GS) - group_row(s * G, H, GS);
    rows += group_row(b + 1, H, GS) - group_row(b, H, GS);
  }
}

}  // namespace dlic
