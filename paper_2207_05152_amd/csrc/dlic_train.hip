// Retraining kernels of the DLIC hot path: mean discretised-logistic-mixture
// NLL in bits over sampled pixels, its gradient with respect to every network
// weight by a hand-written backward pass, and Adam.
//
// The paper trains its density network with a cross-entropy loss whose value
// in bits per pixel indicates the rate (Section III-A) and retrains it on a
// domain (MRI, Section IV).  Here the loss for one sample with target level v
// and network output o is -log2 sum_k pi_k P_k(v), P_k the mass of bin v
// under logistic k, and its derivatives with respect to o are
//   d/d logit_k   = pi_k - r_k                      (r_k = posterior of k)
//   d/d mu_k      = r_k inv_s_k (dA_k + dB_k)
//   d/d logscale_k = r_k (A_k dA_k + B_k dB_k)      (0 where the -7 clamp binds)
// with A, B the standardised upper and lower bin edges and
//   interior: dA = sigma(-A) + 1/expm1(A-B),  dB = -sigma(B) - 1/expm1(A-B)
//   v = 0:    dA = sigma(-A), dB = 0;   v = 255: dA = 0, dB = -sigma(B),
// all divided by n ln 2 for the mean in bits.  The network's backward pass
// and the weight gradients (contractions over the sample dimension) run on
// MFMA, FP32 or FP64 (the FP64 instantiation serves the gradient check).
#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
// Row of the 16x16 result held in register r of lane group q (= lane / 16):
// FP32 16x16x4 keeps rows 4q .. 4q+3 in a lane; FP64 16x16x4 interleaves
// them as q, q+4, q+8, q+12.
template <>
struct Mma<float> {
  typedef f4 v;
  __device__ static __forceinline__ int row(int q, int r) { return 4 * q + r; }
  __device__ static __forceinline__ v op(float a, float b, v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ float exp_(float x) { return expf(x); }
  __device__ static __forceinline__ float log_(float x) { return logf(x); }
  __device__ static __forceinline__ float log1p_(float x) { return log1pf(x); }
  __device__ static __forceinline__ float expm1_(float x) { return expm1f(x); }
};
template <>
struct Mma<double> {
  typedef d4 v;
  __device__ static __forceinline__ int row(int q, int r) { return q + 4 * r; }
  __device__ static __forceinline__ v op(double a, double b, v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ double exp_(double x) { return exp(x); }
  __device__ static __forceinline__ double log_(double x) { return log(x); }
  __device__ static __forceinline__ double log1p_(double x) { return log1p(x); }
  __device__ static __forceinline__ double expm1_(double x) { return expm1(x); }
};

// softplus(x) = max(x, 0) + log1p(exp(-|x|)) and sigmoid(x) = 1 / (1 + exp(-x))
// (e / (1 + e) for x < 0), sharing the one exponential exp(-|x|).
template <typename T>
__device__ __forceinline__ void softplus_sigmoid(T x, T& sp, T& sg) {
  const T e = Mma<T>::exp_(x > T(0) ? -x : x);
  sp = (x > T(0) ? x : T(0)) + Mma<T>::log1p_(e);
  sg = x >= T(0) ? T(1) / (T(1) + e) : e / (T(1) + e);
}

// One mixture component of one sample: the log mass lp_k of bin v (before the
// mixture weight) and the factors of its mean and log-scale derivatives,
// u_mu = inv_s (dA + dB) and u_ls = A dA + B dB (0 where the clamp binds).
// hi, lo: the bin's upper and lower edges (0 where unused).
template <typename T>
struct CompTerms {
  T lpk, u_mu, u_ls;
};

template <typename T>
__device__ __forceinline__ CompTerms<T> component_terms(const T* o, int k, int v, T hi, T lo) {
  CompTerms<T> c;
  const T mu = o[N_MIX + k];
  const bool free_ls = o[2 * N_MIX + k] > T(LOG_SCALE_MIN);
  const T ls = free_ls ? o[2 * N_MIX + k] : T(LOG_SCALE_MIN);
  const T is = Mma<T>::exp_(-ls);
  const T A = (hi - mu) * is, B = (lo - mu) * is;
  T dA, dB;
  if (v == 0) {
    T sp, sg;
    softplus_sigmoid(-A, sp, sg);
    c.lpk = -sp;
    dA = sg;
    dB = T(0);
  } else if (v == 255) {
    T sp, sg;
    softplus_sigmoid(B, sp, sg);
    c.lpk = -sp;
    dA = T(0);
    dB = -sg;
  } else {
    T spa, sga, spb, sgb;
    softplus_sigmoid(-A, spa, sga);
    softplus_sigmoid(B, spb, sgb);
    const T em = Mma<T>::expm1_(A - B);  // > 0
    c.lpk = -spa - spb + Mma<T>::log_(-Mma<T>::expm1_(B - A));
    const T E = T(1) / em;
    dA = sga + E;
    dB = -sgb - E;
  }
  c.u_mu = is * (dA + dB);
  c.u_ls = free_ls ? A * dA + B * dB : T(0);
  return c;
}

template <typename T>
struct TrainArgs {
  const T *w1, *b1, *w2, *b2, *w3, *b3;
  const uint8_t* slices;
  int n_slices, sh, sw;
  const int32_t* idx;
  long long n;
  T* partials;   // [rows][P + 1]
  int want_grad;
  T scale;       // 1 / (n ln 2)
};

template <typename T, int H1, int H2, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void nll_fwd_bwd_kernel(TrainArgs<T> a) {
  typedef typename Mma<T>::v V;
  constexpr int NT1 = H1 / 16, NT2 = H2 / 16;
  constexpr int NP = 13 * H1 + H1 * H2 + 16 * H2 + 15;
  constexpr int O_W1 = 0, O_B1 = 12 * H1, O_W2 = 13 * H1, O_B2 = 13 * H1 + H1 * H2;
  constexpr int O_W3 = O_B2 + H2, O_B3 = O_W3 + 15 * H2;
  // weights as MFMA A operands, lane-contiguous
  __shared__ T s_a1[NT1 * 3 * 64];
  __shared__ T s_a2[NT2 * NT1 * 4 * 64];
  __shared__ T s_a3[NT2 * 4 * 64];
  __shared__ T s_w2t[NT1 * NT2 * 4 * 64];
  __shared__ T s_w3t[NT2 * 4 * 64];
  __shared__ T s_b1[H1], s_b2[H2], s_b3[16];
  __shared__ T s_f[WAVES][16 * 16];
  __shared__ T s_o[WAVES][16 * 16];
  __shared__ T s_h1[WAVES][H1 * 16];
  // s_h2 holds layer 2's outputs until the layer-3 weight gradient has read
  // them, then layer 1's input gradients (H1 == H2)
  __shared__ T s_h2[WAVES][H2 * 16];
  __shared__ T s_d2[WAVES][H2 * 16];
  static_assert(H1 == H2, "layer-1 gradients reuse layer 2's output buffer");

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, i16 = lane & 15;
  constexpr int NTH = WAVES * 64;
  for (int e = tid; e < NT1 * 3 * 64; e += NTH) {
    const int l = e & 63, kk = (e >> 6) % 3, nt = (e >> 6) / 3;
    s_a1[e] = a.w1[(16 * nt + (l & 15)) * K_IN + 4 * kk + (l >> 4)];
  }
  for (int e = tid; e < NT2 * NT1 * 4 * 64; e += NTH) {
    const int l = e & 63, ks = (e >> 6) % (NT1 * 4), n2 = (e >> 6) / (NT1 * 4);
    const int n1 = ks >> 2, r = ks & 3;
    s_a2[e] = a.w2[(16 * n2 + (l & 15)) * H1 + 16 * n1 + Mma<T>::row(l >> 4, r)];
  }
  for (int e = tid; e < NT2 * 4 * 64; e += NTH) {
    const int l = e & 63, ks = e >> 6, n2 = ks >> 2, r = ks & 3;
    s_a3[e] = ((l & 15) < N_OUT) ? a.w3[(l & 15) * H2 + 16 * n2 + Mma<T>::row(l >> 4, r)] : T(0);
  }
  for (int e = tid; e < NT1 * NT2 * 4 * 64; e += NTH) {
    const int l = e & 63, ks = (e >> 6) % (NT2 * 4), mt = (e >> 6) / (NT2 * 4);
    const int nt = ks >> 2, r = ks & 3;
    s_w2t[e] = a.w2[(16 * nt + Mma<T>::row(l >> 4, r)) * H1 + 16 * mt + (l & 15)];
  }
  for (int e = tid; e < NT2 * 4 * 64; e += NTH) {
    const int l = e & 63, kk = (e >> 6) & 3, n2 = e >> 8;
    const int out = 4 * kk + (l >> 4);
    s_w3t[e] = (out < N_OUT) ? a.w3[out * H2 + 16 * n2 + (l & 15)] : T(0);
  }
  for (int e = tid; e < H1; e += NTH) s_b1[e] = a.b1[e];
  for (int e = tid; e < H2; e += NTH) s_b2[e] = a.b2[e];
  for (int e = tid; e < 16; e += NTH) s_b3[e] = (e < N_OUT) ? a.b3[e] : T(0);
  for (int e = lane; e < 16 * 16; e += 64) s_f[wave][e] = T(0);
  __syncthreads();

  V g1[NT1], g2[NT2][NT1], g3[NT2];
#pragma unroll
  for (int x = 0; x < NT1; ++x) g1[x] = V{0, 0, 0, 0};
#pragma unroll
  for (int x = 0; x < NT2; ++x) {
    g3[x] = V{0, 0, 0, 0};
#pragma unroll
    for (int y = 0; y < NT1; ++y) g2[x][y] = V{0, 0, 0, 0};
  }
  T gb1[NT1][4], gb2[NT2][4], gb3[N_OUT], lsum = T(0);
#pragma unroll
  for (int x = 0; x < NT1; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) gb1[x][r] = T(0);
#pragma unroll
  for (int x = 0; x < NT2; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) gb2[x][r] = T(0);
#pragma unroll
  for (int k = 0; k < N_OUT; ++k) gb3[k] = T(0);

  T* sf = s_f[wave];
  T* so = s_o[wave];
  T* sh1 = s_h1[wave];
  T* sh2 = s_h2[wave];
  T* sd2 = s_d2[wave];
  T* sd1 = s_h2[wave];
  const long long row = (long long)blockIdx.x * WAVES + wave;
  const long long n_rows = (long long)gridDim.x * WAVES;
  const long long plane = (long long)a.sh * a.sw;

  for (long long base = row * 16; base < a.n; base += n_rows * 16) {
    // ---- forward, one 16-sample tile
    const long long p = base + i16;
    bool valid = p < a.n;
    int ps = 0, py = 0, px = 0;
    if (valid) {
      ps = a.idx[3 * p];
      py = a.idx[3 * p + 1];
      px = a.idx[3 * p + 2];
      // samples whose index lies outside the stack contribute nothing
      if (ps < 0 || ps >= a.n_slices || py < 0 || py >= a.sh || px < 0 || px >= a.sw) {
        valid = false;
        ps = py = px = 0;
      }
    }
    const uint8_t* sl = a.slices + (long long)ps * plane;
    T fk[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      const int k = 4 * kk + q;
      const int yy = py + nb_dy(k), xx = px + nb_dx(k);
      fk[kk] = (valid && yy >= 0 && xx >= 0 && xx < a.sw)
                   ? (T(2 * (int)sl[(long long)yy * a.sw + xx]) - T(255)) / T(255)
                   : T(0);
      sf[i16 * 16 + k] = fk[kk];
    }
    T h1[NT1][4], h2[NT2][4];
#pragma unroll
    for (int nt = 0; nt < NT1; ++nt) {
      V acc = {s_b1[16 * nt + Mma<T>::row(q, 0)], s_b1[16 * nt + Mma<T>::row(q, 1)],
               s_b1[16 * nt + Mma<T>::row(q, 2)], s_b1[16 * nt + Mma<T>::row(q, 3)]};
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) acc = Mma<T>::op(s_a1[(nt * 3 + kk) * 64 + lane], fk[kk], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h1[nt][r] = acc[r] > T(0) ? acc[r] : T(0);
        sh1[(16 * nt + Mma<T>::row(q, r)) * 16 + i16] = h1[nt][r];
      }
    }
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2) {
      V acc = {s_b2[16 * n2 + Mma<T>::row(q, 0)], s_b2[16 * n2 + Mma<T>::row(q, 1)],
               s_b2[16 * n2 + Mma<T>::row(q, 2)], s_b2[16 * n2 + Mma<T>::row(q, 3)]};
#pragma unroll
      for (int n1 = 0; n1 < NT1; ++n1)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = Mma<T>::op(s_a2[(n2 * NT1 * 4 + n1 * 4 + r) * 64 + lane], h1[n1][r], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h2[n2][r] = acc[r] > T(0) ? acc[r] : T(0);
        sh2[(16 * n2 + Mma<T>::row(q, r)) * 16 + i16] = h2[n2][r];
      }
    }
    {
      V acc = {s_b3[Mma<T>::row(q, 0)], s_b3[Mma<T>::row(q, 1)], s_b3[Mma<T>::row(q, 2)],
               s_b3[Mma<T>::row(q, 3)]};
#pragma unroll
      for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = Mma<T>::op(s_a3[(n2 * 4 + r) * 64 + lane], h2[n2][r], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) so[i16 * 16 + Mma<T>::row(q, r)] = acc[r];
    }
    // ---- loss and d loss / d o: lane group q of sample i16 takes mixture
    // component q (and group 0 component 4 as well); the five log masses meet
    // through shuffles, and every lane then has the sample's loss
    {
      T o[N_OUT];
#pragma unroll
      for (int k = 0; k < N_OUT; ++k) o[k] = so[i16 * 16 + k];
      const T LN2 = T(0.69314718055994530942);
      const int v = valid ? (int)sl[(long long)py * a.sw + px] : 0;
      T m = o[0];
#pragma unroll
      for (int k = 1; k < N_MIX; ++k) m = o[k] > m ? o[k] : m;
      T se = T(0);
#pragma unroll
      for (int k = 0; k < N_MIX; ++k) se += Mma<T>::exp_(o[k] - m);
      const T lse = m + Mma<T>::log_(se);
      const T hi = (v < 255) ? (T(2 * v + 1) / T(255) - T(1)) : T(0);
      const T lo = (v > 0) ? (T(2 * v - 1) / T(255) - T(1)) : T(0);
      const CompTerms<T> ca = component_terms(o, q, v, hi, lo);
      const CompTerms<T> cb = component_terms(o, N_MIX - 1, v, hi, lo);  // used by group 0
      const T lpa = (o[q] - lse) + ca.lpk;
      const T lpb = (o[N_MIX - 1] - lse) + cb.lpk;
      T lp[N_MIX];
#pragma unroll
      for (int k = 0; k < N_MIX - 1; ++k) lp[k] = __shfl(lpa, i16 + 16 * k);
      lp[N_MIX - 1] = __shfl(lpb, i16);
      T mx = lp[0];
#pragma unroll
      for (int k = 1; k < N_MIX; ++k) mx = lp[k] > mx ? lp[k] : mx;
      T ssum = T(0);
#pragma unroll
      for (int k = 0; k < N_MIX; ++k) ssum += Mma<T>::exp_(lp[k] - mx);
      const T LP = mx + Mma<T>::log_(ssum);
      const T sc = valid ? a.scale : T(0);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c == 1 && q != 0) break;
        const int k = c == 0 ? q : N_MIX - 1;
        const CompTerms<T>& t = c == 0 ? ca : cb;
        const T r = Mma<T>::exp_(lp[k] - LP);
        const T pi = Mma<T>::exp_(o[k] - lse);
        so[i16 * 16 + k] = (pi - r) * sc;
        so[i16 * 16 + N_MIX + k] = r * t.u_mu * sc;
        so[i16 * 16 + 2 * N_MIX + k] = r * t.u_ls * sc;
      }
      if (q == 0) {
        so[i16 * 16 + 15] = T(0);
        if (valid) lsum += -LP / LN2;
      }
      wave_lds_handover();
      if (q == 0) {
#pragma unroll
        for (int k = 0; k < N_OUT; ++k) gb3[k] += so[i16 * 16 + k];
      }
    }
    if (!a.want_grad) continue;
    wave_lds_handover();
    // ---- backward through the network
    T d2[NT2][4];
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2) {
      V acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = Mma<T>::op(s_w3t[(n2 * 4 + kk) * 64 + lane], so[i16 * 16 + 4 * kk + q], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T dv = h2[n2][r] > T(0) ? acc[r] : T(0);
        d2[n2][r] = dv;
        gb2[n2][r] += dv;
        sd2[(16 * n2 + Mma<T>::row(q, r)) * 16 + i16] = dv;
      }
    }
    // ---- weight gradients: contractions over the 16 samples of the tile.
    // Layer 3's first, which frees layer 2's outputs for layer 1's gradients.
    wave_lds_handover();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int s_ = 4 * kk + q;  // sample index of this k-step
      const T ao = so[s_ * 16 + i16];
#pragma unroll
      for (int n2 = 0; n2 < NT2; ++n2)
        g3[n2] = Mma<T>::op(ao, sh2[(16 * n2 + i16) * 16 + s_], g3[n2]);
    }
    wave_lds_handover();
#pragma unroll
    for (int mt = 0; mt < NT1; ++mt) {
      V acc = {0, 0, 0, 0};
#pragma unroll
      for (int nt = 0; nt < NT2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = Mma<T>::op(s_w2t[(mt * NT2 * 4 + nt * 4 + r) * 64 + lane], d2[nt][r], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T dv = h1[mt][r] > T(0) ? acc[r] : T(0);
        gb1[mt][r] += dv;
        sd1[(16 * mt + Mma<T>::row(q, r)) * 16 + i16] = dv;
      }
    }
    wave_lds_handover();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int s_ = 4 * kk + q;  // sample index of this k-step
      const T bf = sf[s_ * 16 + i16];
      T a2v[NT2], b1v[NT1], a1v[NT1];
#pragma unroll
      for (int n2 = 0; n2 < NT2; ++n2) a2v[n2] = sd2[(16 * n2 + i16) * 16 + s_];
#pragma unroll
      for (int mt = 0; mt < NT1; ++mt) {
        b1v[mt] = sh1[(16 * mt + i16) * 16 + s_];
        a1v[mt] = sd1[(16 * mt + i16) * 16 + s_];
      }
#pragma unroll
      for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
        for (int mt = 0; mt < NT1; ++mt) g2[n2][mt] = Mma<T>::op(a2v[n2], b1v[mt], g2[n2][mt]);
#pragma unroll
      for (int mt = 0; mt < NT1; ++mt) g1[mt] = Mma<T>::op(a1v[mt], bf, g1[mt]);
    }
    // the next tile's forward pass overwrites these buffers
    wave_lds_handover();
  }

  // ---- this wave's partial sums, one row of [P + 1]
  T* out = a.partials + row * (NP + 1);
  if (a.want_grad) {
#pragma unroll
    for (int mt = 0; mt < NT1; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (i16 < K_IN) out[O_W1 + (16 * mt + Mma<T>::row(q, r)) * K_IN + i16] = g1[mt][r];
#pragma unroll
        for (int n2 = 0; n2 < NT2; ++n2)
          out[O_W2 + (16 * n2 + Mma<T>::row(q, r)) * H1 + 16 * mt + i16] = g2[n2][mt][r];
      }
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (Mma<T>::row(q, r) < N_OUT) out[O_W3 + Mma<T>::row(q, r) * H2 + 16 * n2 + i16] = g3[n2][r];
    // biases: sum the 16 sample lanes of each lane group
#pragma unroll
    for (int mt = 0; mt < NT1; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = gb1[mt][r];
        for (int sft = 1; sft < 16; sft <<= 1) v += __shfl_xor(v, sft);
        if (i16 == 0) out[O_B1 + 16 * mt + Mma<T>::row(q, r)] = v;
      }
#pragma unroll
    for (int n2 = 0; n2 < NT2; ++n2)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = gb2[n2][r];
        for (int sft = 1; sft < 16; sft <<= 1) v += __shfl_xor(v, sft);
        if (i16 == 0) out[O_B2 + 16 * n2 + Mma<T>::row(q, r)] = v;
      }
#pragma unroll
    for (int k = 0; k < N_OUT; ++k) {
      T v = gb3[k];
      for (int sft = 1; sft < 16; sft <<= 1) v += __shfl_xor(v, sft);
      if (lane == 0) out[O_B3 + k] = v;
    }
  }
  for (int sft = 1; sft < 16; sft <<= 1) lsum += __shfl_xor(lsum, sft);
  if (lane == 0) out[NP] = lsum;
}

// Sum the partial rows in a fixed order: blocks of 32 rows, then the blocks.
// Stage 1 gives every block of 32 rows (and every 256 columns) its own
// workgroup, each thread summing one column's 32 rows in row order; stage 2
// sums the block sums of a column in block order.  The result is the same
// sequence of additions as one thread walking all rows block by block.
constexpr int RED_BLOCK = 32;

template <typename T>
__global__ __launch_bounds__(256) void nll_reduce_rows_kernel(const T* __restrict__ partials,
                                                              long long rows, int np,
                                                              T* __restrict__ blocks) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > np) return;
  const long long r0 = (long long)blockIdx.y * RED_BLOCK;
  const long long r1 = r0 + RED_BLOCK < rows ? r0 + RED_BLOCK : rows;
  T s = T(0);
  for (long long r = r0; r < r1; ++r) s += partials[r * (np + 1) + e];
  blocks[(long long)blockIdx.y * (np + 1) + e] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void nll_reduce_blocks_kernel(const T* __restrict__ blocks,
                                                                long long n_blocks, int np,
                                                                T* __restrict__ grad,
                                                                T* __restrict__ loss, long long n,
                                                                int want_grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > np) return;
  if (e < np && !want_grad) return;
  T total = T(0);
  for (long long b = 0; b < n_blocks; ++b) total += blocks[b * (np + 1) + e];
  if (e < np)
    grad[e] = total;
  else
    *loss = total / T(n);
}

template <typename T>
static void launch_reduce(const T* partials, long long rows, int np, T* grad, T* loss, long long n,
                          bool want_grad, hipStream_t s) {
  const unsigned cgrid = (unsigned)((np + 1 + 255) / 256);
  const long long n_blocks = (rows + RED_BLOCK - 1) / RED_BLOCK;
  T* blocks = const_cast<T*>(partials) + rows * (np + 1);  // after the partial rows
  hipLaunchKernelGGL(nll_reduce_rows_kernel<T>, dim3(cgrid, (unsigned)n_blocks), dim3(256), 0, s,
                     partials, rows, np, blocks);
  hipLaunchKernelGGL(nll_reduce_blocks_kernel<T>, dim3(cgrid), dim3(256), 0, s,
                     (const T*)blocks, n_blocks, np, grad, loss, n, want_grad ? 1 : 0);
}

// step_size = lr / (1 - b1^t) and bc2_sqrt = sqrt(1 - b2^t) come from the
// host in double precision (1 - b2^t cancels badly in FP32).
__global__ void adam_kernel(long long np, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float b1, float b2,
                            float eps, float step_size, float bc2_sqrt) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < np;
       e += (long long)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = m[e] + (1.0f - b1) * (gi - m[e]);
    const float vi = v[e] * b2 + (1.0f - b2) * (gi * gi);
    m[e] = mi;
    v[e] = vi;
    const float denom = sqrtf(vi) / bc2_sqrt + eps;
    p[e] = p[e] - step_size * (mi / denom);
  }
}

// ---- launchers -------------------------------------------------------------

int train_n_params(int h1, int h2) { return 13 * h1 + h1 * h2 + 16 * h2 + 15; }

template <typename T, int H, int WAVES>
static void launch_nll_t(const TrainArgs<T>& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((nll_fwd_bwd_kernel<T, H, H, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, a);
}

bool launch_nll(bool fp64, int width, const void* w1, const void* b1, const void* w2,
                const void* b2, const void* w3, const void* b3, const uint8_t* slices,
                int n_slices, int sh, int sw, const int32_t* idx, long long n, void* partials,
                int grid, bool want_grad, void* grad, void* loss, hipStream_t s) {
  const long long rows = (long long)grid * (fp64 ? TRAIN_WAVES_F64 : TRAIN_WAVES_F32);
  const int np = train_n_params(width, width);
  if (fp64) {
    TrainArgs<double> a{(const double*)w1, (const double*)b1, (const double*)w2, (const double*)b2,
                        (const double*)w3, (const double*)b3, slices, n_slices, sh, sw, idx, n,
                        (double*)partials, want_grad ? 1 : 0,
                        1.0 / ((double)n * 0.69314718055994530942)};
    switch (width) {
      case 32: launch_nll_t<double, 32, TRAIN_WAVES_F64>(a, grid, s); break;
      case 64: launch_nll_t<double, 64, TRAIN_WAVES_F64>(a, grid, s); break;
      default: return false;
    }
    launch_reduce((const double*)partials, rows, np, (double*)grad, (double*)loss, n, want_grad, s);
  } else {
    TrainArgs<float> a{(const float*)w1, (const float*)b1, (const float*)w2, (const float*)b2,
                       (const float*)w3, (const float*)b3, slices, n_slices, sh, sw, idx, n,
                       (float*)partials, want_grad ? 1 : 0,
                       (float)(1.0 / ((double)n * 0.69314718055994530942))};
    switch (width) {
      case 32: launch_nll_t<float, 32, TRAIN_WAVES_F32>(a, grid, s); break;
      case 64: launch_nll_t<float, 64, TRAIN_WAVES_F32>(a, grid, s); break;
      default: return false;
    }
    launch_reduce((const float*)partials, rows, np, (float*)grad, (float*)loss, n, want_grad, s);
  }
  return true;
}

void launch_adam(long long np, float* p, const float* g, float* m, float* v, int step, float lr,
                 float b1, float b2, float eps, hipStream_t s) {
  const double bc1 = 1.0 - pow((double)b1, (double)step);
  const double bc2 = 1.0 - pow((double)b2, (double)step);
  const float step_size = (float)((double)lr / bc1), bc2_sqrt = (float)sqrt(bc2);
  long long blocks = (np + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, np, p, g, m, v, b1, b2,
                     eps, step_size, bc2_sqrt);
}

}  // namespace dlic
