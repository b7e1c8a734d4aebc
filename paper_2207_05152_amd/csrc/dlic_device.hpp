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
};

// Network weights as the kernels see them (FP32, row-major [out][in]).
struct DevModel {
  const float *w1, *b1, *w2, *b2, *w3, *b3;
};

typedef float f4 __attribute__((ext_vector_type(4)));

// D(16x16) = A(16x4) B(4x16) + C with lane l holding A[l%16][l/16],
// B[l/16][l%16] and D[4*(l/16) + r][l%16] (r = 0..3).
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Causal window offset of feature k (rows y-2, y-1 at dx -2..2, then (y, x-2), (y, x-1)).
__device__ __forceinline__ int nb_dy(int k) { return k < 5 ? -2 : (k < 10 ? -1 : 0); }
__device__ __forceinline__ int nb_dx(int k) { return k < 5 ? k - 2 : (k < 10 ? k - 7 : k - 12); }

__device__ __forceinline__ float relu(float v) { return v > 0.0f ? v : 0.0f; }

// -----------------------------------------------------------------------------
// Network tile: 16 pixels through 12 -> H1 -> H2 -> 15 on v_mfma_f32_16x16x4f32.
//
// Activations are the B operand (K x 16 pixels) and weights the A operand
// (16 neurons x K), so a layer's D registers (neuron 16*nt + 4*(l/16) + r of
// pixel l%16) are directly the next layer's B operand for the k-step (nt, r):
// the weights are loaded with the matching permutation of their input index.
// Biases seed the accumulators.  Weights stay resident in VGPRs.
// -----------------------------------------------------------------------------
template <int H1, int H2>
struct NetF32 {
  static constexpr int NT1 = H1 / 16, NT2 = H2 / 16;
  float a1[NT1][3];
  float a2[NT2][NT1 * 4];
  float a3[NT2 * 4];
  float c1[NT1][4], c2[NT2][4], c3[4];

  __device__ __forceinline__ void load(const DevModel& m, int lane) {
    const int i = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < NT1; ++nt)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) a1[nt][kk] = m.w1[(16 * nt + i) * K_IN + 4 * kk + q];
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
      for (int n1 = 0; n1 < NT1; ++n1)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          a2[n2][n1 * 4 + r] = m.w2[(16 * n2 + i) * H1 + 16 * n1 + 4 * q + r];
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        a3[n2 * 4 + r] = (i < N_OUT) ? m.w3[i * H2 + 16 * n2 + 4 * q + r] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int nt = 0; nt < NT1; ++nt) c1[nt][r] = m.b1[16 * nt + 4 * q + r];
#pragma unroll
      for (int nt = 0; nt < NT2; ++nt) c2[nt][r] = m.b2[16 * nt + 4 * q + r];
      c3[r] = (4 * q + r < N_OUT) ? m.b3[4 * q + r] : 0.0f;
    }
  }

  // f0, f1, f2: this lane's window features k = l/16, 4 + l/16, 8 + l/16 of
  // pixel l%16.  Returns outputs 4*(l/16) .. 4*(l/16)+3 of pixel l%16.
  __device__ __forceinline__ f4 run(float f0, float f1, float f2) const {
    f4 h1[NT1];
#pragma unroll
    for (int nt = 0; nt < NT1; ++nt) {
      f4 acc = {c1[nt][0], c1[nt][1], c1[nt][2], c1[nt][3]};
      acc = mfma_f32(a1[nt][0], f0, acc);
      acc = mfma_f32(a1[nt][1], f1, acc);
      acc = mfma_f32(a1[nt][2], f2, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[nt][r] = relu(acc[r]);
    }
    f4 h2[NT2];
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2) {
      f4 acc = {c2[n2][0], c2[n2][1], c2[n2][2], c2[n2][3]};
#pragma unroll
      for (int n1 = 0; n1 < NT1; ++n1)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = mfma_f32(a2[n2][n1 * 4 + r], h1[n1][r], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[n2][r] = relu(acc[r]);
    }
    f4 o = {c3[0], c3[1], c3[2], c3[3]};
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r) o = mfma_f32(a3[n2 * 4 + r], h2[n2][r], o);
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

// pi = softmax(o[0:5]); mu = o[5:10]; inv_s = exp(-max(o[10:15], -7)).
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
#pragma unroll
  for (int k = 0; k < N_MIX; ++k) {
    p.pi[k] = e[k] / s;
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

// Cumulative frequency F(v) = v + min(M', floor(C(beta_v) * M')), F(0) = 0,
// F(256) = 2^16; C summed over components in index order.
__device__ __forceinline__ uint32_t cdf_F(int v, const Mix& p, const float2* sd,
                                          const float* beta) {
  if (v <= 0) return 0u;
  if (v >= 256) return M_TOTAL;
  const float b = beta[v];
  float C = p.pi[0] * sigma_hat(b * p.A[0] + p.B[0], sd);
#pragma unroll
  for (int k = 1; k < N_MIX; ++k) C = C + p.pi[k] * sigma_hat(b * p.A[k] + p.B[k], sd);
  uint32_t q = (uint32_t)(C * 65280.0f);
  q = min(q, M_PRIME);
  return (uint32_t)v + q;
}

// F(v) for 0 < v < 256 with the bin edge beta_v already at hand.
__device__ __forceinline__ uint32_t cdf_F_at(int v, float b, const Mix& p, const float2* sd) {
  float C = p.pi[0] * sigma_hat(b * p.A[0] + p.B[0], sd);
#pragma unroll
  for (int k = 1; k < N_MIX; ++k) C = C + p.pi[k] * sigma_hat(b * p.A[k] + p.B[k], sd);
  uint32_t q = (uint32_t)(C * 65280.0f);
  q = min(q, M_PRIME);
  return (uint32_t)v + q;
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
// one integer correction step.
__device__ __forceinline__ uint32_t rans_enc_update(uint32_t x, uint32_t c, uint32_t f) {
  const float rcp = __builtin_amdgcn_rcpf((float)f);
  uint32_t q = (uint32_t)((float)x * rcp);
  int32_t r = (int32_t)(x - q * f);
  if (r < 0) {
    q -= 1u;
    r += (int32_t)f;
  } else if (r >= (int32_t)f) {
    q += 1u;
    r -= (int32_t)f;
  }
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
  if (ren) {
    out[Q - cnt + lane_rank(mask)] = (uint16_t)(x & 0xFFFFu);
    x >>= 16;
  }
  if (act) x = rans_enc_update(x, c, f);
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

}  // namespace dlic
