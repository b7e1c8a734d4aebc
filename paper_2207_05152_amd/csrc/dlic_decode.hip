// Wavefront decoder of the DLIC hot path (Section II-A, Fig. 2 right;
// Section II-B, Preprocessor and rANS; Fig. 1 right).
//
// One persistent workgroup per group of rows.  In wavefront step t every
// pixel (y, x) with x + 3y == t has its whole 12-pixel window decoded (the
// up-right neighbour (y-1, x+2) finished in step t-1).  A group's symbols
// are decoded in canonical order: step t, then block j of L rows, then lane.
// One block of one step is a sub-round q = (t - t_first) * J + j.
//
// Inside the workgroup the work is split by wave and synchronised through
// LDS counters instead of barriers:
//   * wave 0, the coder, walks the sub-rounds in order: for each active pixel
//     it locates the symbol from the slot of its state (16-level bucket from
//     precomputed boundaries, then the level inside the bucket on the FP32
//     table rule: 4 halvings with one or two lanes per pixel, or one level per
//     lane with 16 lanes per pixel when L <= 4), updates the state,
//     renormalises by ballot from an LDS ring of the stream, writes the pixel
//     to the ring, and publishes the sub-rounds done;
//   * wave 4, the publisher, hands each finished step's last two rows to the
//     next group and stores rows' last pixels to the image;
//   * the other waves compute densities ahead of the coder, one 16-pixel tile of
//     one sub-round at a time: gather from the LDS pixel ring, network on
//     MFMA, mixture head, and the table at the 15 bucket boundaries.  Sub-round
//     (t, j) only needs (t-1, j) and (t-1, j-1) decoded, so densities run up
//     to J-1 sub-rounds ahead of the coder.
// Rows r0-2 and r0-1 come from the group above through 32-bit records that
// carry validity and both pixels in one word (bit 31 valid, bits 8..15 row
// r1-2, bits 0..7 row r1-1), written and read with agent-scope atomics.  A
// group only waits for the one before it, whose workgroup took its ticket
// earlier and is running or done, and every wait is bounded, so the grid
// always drains.
#include <type_traits>

#include "dlic_device.hpp"
#include "dlic_kernels.h"

namespace dlic {

constexpr int RING_MASK = DEC_RING - 1;
constexpr int REFILL_WORDS = 1024;           // one coder-wave refill: 16 words per lane
// Waves per decoder workgroup: 12 where a density wave's registers allow
// three waves per SIMD (nets up to 64 wide, the FP32 net's layer-2 weights
// then in LDS), else 8.  Waves are placed on the four SIMDs round-robin, so
// waves 4, 8, ... share the coder's SIMD: wave 4 is the publisher (light and
// mostly asleep), wave 8 stays idle.  The others compute densities.
template <class Net>
constexpr int dec_waves() { return Net::DEC_WIDE ? 12 : 8; }
template <class Net>
constexpr int dec_workers() { return dec_waves<Net>() - dec_waves<Net>() / 4; }
constexpr int NSLOT = 8;                     // sub-round densities in flight
constexpr int SLOT_PX = 64;                  // lanes per group at most
constexpr int PAR_STRIDE = 16;               // floats per pixel: pi[5], A[5], B[5]
constexpr int N_BUCKET = 15;                 // F(16 m), m = 1..15
constexpr uint32_t LDS_SPIN_LIMIT = 1u << 24;
constexpr int PROF_SLOTS = 16;               // decode profile counters per group


__device__ __forceinline__ int floordiv(int a, int b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__device__ __forceinline__ uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
__device__ __forceinline__ uint32_t rd_u16(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8);
}

__device__ __forceinline__ int lds_acquire(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
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
  // an image's flags: strips per group - 1 in bits 12..15, nothing else
  if (rd_u16(b + 6) != ((uint32_t)(a.S - 1) << 12)) return 3;
  if (a.check_model) {
    const uint64_t fp = (uint64_t)rd_u32(b + 28) | ((uint64_t)rd_u32(b + 32) << 32);
    if (b[18] != (uint8_t)a.hf.dtype || rd_u16(b + 20) != (uint32_t)a.hf.h1 ||
        rd_u16(b + 22) != (uint32_t)a.hf.h2 || fp != a.hf.fingerprint)
      return 4;
  }
  return 0;
}

// Record of step s from the group above, spinning up to `limit` polls.
// Returns false on timeout (the caller then stops waiting for good).
__device__ bool receive_record(const uint32_t* up_rec, int s, uint32_t limit, uint32_t& v) {
  v = __hip_atomic_load(up_rec + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t spins = 0;
  while (!(v >> 31)) {
    if (++spins > limit) {
      v = 0x80000000u;
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(up_rec + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

// Test hook: a seeded pause of up to delay_max shader cycles (in 64-cycle
// sleeps) at one point of one wave, the same for every lane, so that the
// waves' hand-offs meet in other orders.  No-op when delay_max is 0.
__device__ __forceinline__ void inject_delay(const DecArgs& a, uint32_t site, uint32_t g,
                                             uint32_t step) {
  if (a.delay_max == 0) return;
  uint32_t h = a.delay_seed ^ (site * 0x9E3779B1u) ^ (g * 0x85EBCA77u) ^ (step * 0xC2B2AE3Du);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  const uint32_t n = (h % a.delay_max) >> 6;
  for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(1);
}

// The pixel ring keeps 16 columns per row, so step t overwrites step t - 16.
// Before step t the coder makes sure the publisher wave has taken every step
// up to t - PUB_LAG from the ring; pub caches the last value seen.  Returns
// false if the wait gives up.
constexpr int PUB_LAG = 13;
constexpr int RCV_AHEAD = 6;  // upstream records stored at most this many steps ahead
__device__ __forceinline__ bool wait_publisher(const int* s_pub, int t, int& pub) {
  uint32_t spins = 0;
  while (pub < t - PUB_LAG) {
    pub = __hip_atomic_load(s_pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (pub >= t - PUB_LAG) break;
    if (++spins > LDS_SPIN_LIMIT) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Put the two pixels of upstream record s into ring rows 0 (r0-2) and 1 (r0-1).
__device__ __forceinline__ void stash_record(uint8_t* ring, uint32_t v, int s, int r0, int W) {
  const int c1 = s - SKEW * (r0 - 1);
  const int c2 = s - SKEW * (r0 - 2);
  if (c1 >= 0 && c1 < W) ring[1 * 16 + (c1 & 15)] = (uint8_t)(v & 0xFF);
  if (c2 >= 0 && c2 < W) ring[0 * 16 + (c2 & 15)] = (uint8_t)((v >> 8) & 0xFF);
}

// Reductions over the 16 lanes of one row of the wave (lanes 16i .. 16i+15
// serve pixel i): four rotations inside the row.
__device__ __forceinline__ uint32_t row16_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));  // row_ror:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));  // row_ror:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));  // row_ror:2
  return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));  // row_ror:1
}
__device__ __forceinline__ uint32_t row16_min(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));
  return min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));
}

// Shader clock, waited for at once: a clock read left in flight would make
// later LDS waits wait for everything (the scalar read completes out of order).
__device__ __forceinline__ unsigned long long clk_now() {
  const unsigned long long c = clock64();
  asm volatile("" ::"s"(c));
  return c;
}

// RN(n / 255) for an integer n in [-256, 256] without a table: one product
// by RN(1/255) and two fused corrections give the correctly rounded quotient
// for every such n.  Bin edges beta_v = RN((2v - 256) / 255) and scaled grey
// levels RN((2v - 255) / 255) (the host's tables) are both of this form.
__device__ __forceinline__ float div255(int n) {
  const float xv = (float)n;
  const float r = 1.0f / 255.0f;
  const float q0 = xv * r;
  const float e = __builtin_fmaf(-q0, 255.0f, xv);
  return __builtin_fmaf(e, r, q0);
}
__device__ __forceinline__ float bin_edge(int v) { return div255(2 * v - 256); }

// Decode of group g of one stream by the whole workgroup.  LPP is
// coder_lpp(L): how many coder lanes share each pixel's symbol search.
// Layer 1's partial state of a net that splits layer 1 around the last
// step's pixels (the 4-pixel net), else an empty stand-in.
template <class Net, class = void>
struct NetL1 {
  struct type {};
};
template <class Net>
struct NetL1<Net, std::void_t<typename Net::L1>> {
  using type = typename Net::L1;
};

// The coder wave's end of a strip.  After the group's last strip every lane
// must be back at its initial state and every word consumed; after an earlier
// one the states and the word position go to LDS for the next strip, and a
// failure stops the group.
__device__ __forceinline__ void coder_strip_end(const DecArgs& a, int g, bool last_strip, int lane,
                                                bool in_use, uint32_t x, uint32_t Pw,
                                                uint32_t n_words, bool bad, bool stuck,
                                                bool timeout, uint32_t* s_x, uint32_t* s_pw,
                                                int* s_stop) {
  (void)g;
  const bool lane_bad = last_strip && in_use && x != RANS_L;
  const bool any_bad = __ballot(lane_bad || bad) != 0ull;
  if (!last_strip) s_x[lane] = x;
  if (lane == 0) {
    if (any_bad || stuck || (last_strip && Pw != n_words)) atomicMax(a.status, 3);
    if (timeout) atomicMax(a.status, 7);
    if (!last_strip) *s_pw = Pw;
    if (any_bad || stuck || timeout) *s_stop = 1;
  }
}

// STRIPS: the row strips per group this kernel form serves: 1 (one strip,
// no loop), 2 (two strips in straight-line code, the lightest on registers), or
// 0 (any number, a loop over them).
template <class Net, bool TABLES, int LPP, bool DELAY = false, int STRIPS = 1>
__device__ __forceinline__ void decode_group(const Consts* __restrict__ K, const DevModel& m,
                                             const DecArgs& a, const int g) {
  __shared__ float2 s_sd[LUT_N];
  __shared__ __attribute__((aligned(16))) float s_beta[260];
  // nets for tiles of at most 4 pixels run only with the 16-lane coder,
  // which serves at most 4 pixels per sub-round
  constexpr int SPX = Net::SCRATCH_FLOATS > 0 ? 4 : SLOT_PX;
  __shared__ __attribute__((aligned(16))) float s_par[NSLOT][SPX * PAR_STRIDE];
  __shared__ __attribute__((aligned(16))) uint16_t s_bk[NSLOT][SPX * 16];
  __shared__ uint8_t s_ring[(DEC_RMAX + 2) * 16];
  __shared__ uint16_t s_words[DEC_RING];
  __shared__ int s_done[NSLOT][4];
  __shared__ int s_pub;                 // last step handed on by the courier wave
  __shared__ int s_rcv;                 // last upstream step in the ring (courier)
  __shared__ int s_decoded;
  __shared__ uint32_t s_pw, s_end;  // words consumed by the coder / loaded into the ring
  __shared__ unsigned long long s_total, s_before;
  __shared__ int s_err, s_flag, s_stop;
  __shared__ uint32_t s_x[64];          // lane states carried from strip to strip
  __shared__ __attribute__((aligned(16))) char s_w2[Net::LDS_BYTES > 0 ? Net::LDS_BYTES : 16];
  __shared__ __attribute__((aligned(16)))
  float s_xs[Net::SCRATCH_FLOATS > 0 ? dec_workers<Net>() * Net::SCRATCH_FLOATS : 4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H = a.H, W = a.W, G = a.G, L = a.L;
  constexpr int NTH = dec_waves<Net>() * 64;

  if (!TABLES) {
    for (int i = tid; i < LUT_N; i += NTH) s_sd[i] = K->sd[i];
    for (int i = tid; i < 257; i += NTH) s_beta[i] = K->beta[i];
    Net::stage(m, s_w2, tid, NTH);
  }
  if (tid == 0) {
    s_err = check_header(a);
    s_total = 0;
    s_before = 0;
    s_stop = 0;
    s_pw = 0;
    s_end = 0;
  }
  __syncthreads();
  if (s_err == 0) {
    for (int i = tid; i < G; i += NTH) {
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

  const uint32_t n_words = rd_u32(a.bits + HEADER_BYTES + 4 * g);
  const uint16_t* gw = reinterpret_cast<const uint16_t*>(
      a.bits + HEADER_BYTES + 4LL * G + 2ull * s_before);
  const bool bad = n_words < 2u * (uint32_t)L;
  const uint32_t E0 = bad ? 0u : min(n_words, (uint32_t)DEC_RING);
  for (uint32_t i = tid; i < E0; i += NTH) s_words[i] = gw[i];
  if (tid == 0) s_end = E0;

  // The group's strips one after another (strip b = sG + g of the S*G strips,
  // its upstream neighbour strip b - 1, which for g = 0 is the last group's
  // previous strip); the coder's lane states, its word position and the word
  // ring carry over.  Every wave passes the barriers at the strip's start and
  // end, whatever its role.
  const int n_strips = STRIPS == 0 ? a.S : STRIPS;
  const int GS = G * n_strips;
  // one strip: a barrier, then every wave in its role; a wave may leave early
  auto strip = [&](const int sp) {
  const int b = sp * G + g;
  const bool first_strip = sp == 0, last_strip = sp == n_strips - 1;
  const int r0 = group_row(b, H, GS), r1 = group_row(b + 1, H, GS);
  const int R = r1 - r0;
  const int J = (R + L - 1) / L;
  const int NT = (L + 15) / 16;
  const int t_first = SKEW * r0, t_last = SKEW * (r1 - 1) + W - 1;
  const int P = (t_last - t_first + 1) * J;  // sub-rounds (host keeps this below 2^31)
  const int up_last = (b > 0) ? SKEW * (r0 - 1) + W - 1 : -1;
  const uint32_t* up_rec = a.rec + (long long)(b - 1) * a.T;
  uint32_t* my_rec = a.rec + (long long)b * a.T;

  if (tid < NSLOT * 4) s_done[tid / 4][tid % 4] = -1;
  if (tid == 0) {
    s_decoded = 0;
    s_flag = 0;
  }
  // upstream records of the steps before this strip's first one
  if (tid == 0 && b > 0) {
    bool ok = true;
    for (int s = t_first - 2 * SKEW; s <= t_first - 2 && ok; ++s) {
      uint32_t v;
      ok = receive_record(up_rec, s, a.spin_limit, v);
      stash_record(s_ring, v, s, r0, W);
    }
    if (!ok) s_flag = 7;
  }
  if (tid == 0) {
    s_pub = t_first - 1;
    s_rcv = t_first - 2;
  }
  __syncthreads();

  unsigned long long t_wait = 0, t_busy = 0, t_load = 0, t_search = 0, c_ld = 0, c_sr = 0;
  unsigned long long t_wait0 = 0;

  if (!TABLES && LPP == 16 && wave == 0) {
    // ------------------------------------------ coder, 16 lanes per pixel
    // L <= 4: row cl of the wave (lanes 16 cl + h, h = 0..15) serves pixel
    // cl, and every lane keeps its own copy of that pixel's state, so all take
    // the same decisions without a broadcast.  Lane h < 15 holds boundary
    // F(16 (h + 1)); one max and one min reduction over the row give the
    // bucket and its end points.  Lane h < 15 then evaluates the interior
    // level base + h + 1, and two more reductions give the symbol, F(v) and
    // F(v + 1).  F rises strictly with the level, so the levels at or below
    // the slot are a prefix of the row and the packed (count, F) key of the
    // last of them is the maximum.
    // A sub-round waits on few LDS round trips: the density flag and the
    // pixel's parameters and boundary are read in one batch (LDS serves a
    // wave's accesses in order, so data read after the flag was written
    // before it), and the batch of sub-round q + 1 is issued while sub-round q
    // waits for its table reads; bin edges are computed, not read; stream
    // words come from a 64-word register window (lane i holds word base + i);
    // the work is branch-free.
    const int cl = lane >> 4, h = lane & 15;
    uint32_t x = RANS_L;
    if (!first_strip)
      x = s_x[lane];
    else if (cl < L && !bad)
      x = (uint32_t)gw[2 * cl] | ((uint32_t)gw[2 * cl + 1] << 16);
    uint32_t Pw = first_strip ? 2u * (uint32_t)L : s_pw;
    bool over = false, stuck = false;
    const bool timeout = s_flag != 0;
    uint32_t E = first_strip
                     ? E0
                     : __hip_atomic_load(&s_end, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    int t = t_first, j = -1, pub = t_first - 1;
    const unsigned long long k0 = a.prof ? clk_now() : 0ull;
    const unsigned long long rt0 = a.prof ? __builtin_amdgcn_s_memrealtime() : 0ull;
    const uint64_t row_heads = 0x0001000100010001ull;
    // sub-rounds whose densities were not there yet (high half: of them at
    // block 0) and the cycles spent waiting for them
    unsigned long long n_late = 0, t_late = 0;
    const uint64_t below = (1ull << (16 * cl)) - 1ull;
    // stream words wbase .. wbase + 63, one per lane (the ring holds at least
    // min(n_words, 4096) words at the start; a later strip loads its window
    // in its first sub-round, once the ring is known to hold it)
    uint32_t wbase = Pw;
    uint32_t wwin = first_strip ? s_words[(wbase + (uint32_t)lane) & RING_MASK] : 0u;
    bool win_ok = first_strip;
    // the batch of sub-round pre_q, issued during the sub-round before it
    int pre_q = -1, nd = 0;
    f4 n0 = {0.0f, 0.0f, 0.0f, 0.0f}, n1 = n0, n2 = n0, n3 = n0;
    uint32_t nFb = 0;
    for (int q = 0; q < P; ++q) {
      if constexpr (DELAY) inject_delay(a, 2u, (uint32_t)g, (uint32_t)q);
      if (++j == J) {
        j = 0;
        ++t;
      }
      if (!bad && E < n_words && Pw + 64u > E && !stuck) {
        uint32_t spins = 0;
        while ((E = __hip_atomic_load(&s_end, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) <
                   min(n_words, Pw + 64u)) {
          if (++spins > LDS_SPIN_LIMIT) {
            stuck = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (j == 0 && !stuck) stuck = !wait_publisher(&s_pub, t, pub);
      if (Pw + 4u > wbase + 64u || !win_ok) {
        // the ring holds min(n_words, Pw + 64) words by now
        wbase = Pw;
        wwin = s_words[(wbase + (uint32_t)lane) & RING_MASK];
        win_ok = true;
      }
      const int rr = j * L + cl;
      const int y = r0 + rr;
      const int xc = t - SKEW * y;
      const bool act = cl < L && rr < R && xc >= 0 && xc < W;
      const int slot_i = q & (NSLOT - 1);
      const unsigned long long c0 = a.prof ? clk_now() : 0ull;
      unsigned long long c1 = c0;
      if (__ballot(act) != 0ull && !stuck) {
        const f4* pq = reinterpret_cast<const f4*>(&s_par[slot_i][cl * PAR_STRIDE]);
        const uint16_t* pb = &s_bk[slot_i][cl * 16 + h];
        int d;
        f4 p0, p1, p2, p3;
        uint32_t Fb;
        if (pre_q == q) {
          d = nd;
          p0 = n0;
          p1 = n1;
          p2 = n2;
          p3 = n3;
          Fb = nFb;
        } else {
          d = __hip_atomic_load(&s_done[slot_i][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          asm volatile("" ::: "memory");
          p0 = pq[0];
          p1 = pq[1];
          p2 = pq[2];
          p3 = pq[3];
          Fb = *pb;
        }
        // keep the batch together: one wait for all of it, no reload merged
        // into the rare path below
        asm volatile("" : "+v"(p0), "+v"(p1), "+v"(p2), "+v"(p3), "+v"(Fb), "+v"(d));
        // the flag is one LDS word read by every lane: decide on lane 0's copy
        if (__builtin_amdgcn_readfirstlane(d) != q) {
          n_late += j == 0 ? (1ull << 32) + 1ull : 1ull;
          const unsigned long long cw = a.prof ? clk_now() : 0ull;
          uint32_t spins = 0;
          while ((d = __hip_atomic_load(&s_done[slot_i][0], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP)) != q) {
            if (++spins > LDS_SPIN_LIMIT) {
              stuck = true;
              break;
            }
          }
          asm volatile("" ::: "memory");
          p0 = pq[0];
          p1 = pq[1];
          p2 = pq[2];
          p3 = pq[3];
          Fb = *pb;
          if (a.prof) t_late += clk_now() - cw;
        }
        if (a.prof) c1 = clk_now();
        const float pv[16] = {p0[0], p0[1], p0[2], p0[3], p1[0], p1[1], p1[2], p1[3],
                              p2[0], p2[1], p2[2], p2[3], p3[0], p3[1], p3[2], p3[3]};
        const uint32_t slot = x & 0xFFFFu;
        // slot 15 of a pixel's boundaries is padding: F(256) = 2^16 there
        Fb = h < N_BUCKET ? Fb : M_TOTAL;
        const bool le = Fb <= slot;
        const uint32_t klo = row16_max(le ? (((uint32_t)(h + 1) << 17) | Fb) : 0u);
        const uint32_t Fhi = row16_min(le ? M_TOTAL : Fb);
        if (a.prof) c_ld = clk_now();
        const int base = 16 * min((int)(klo >> 17), N_BUCKET);
        const int lv = base + h + 1;  // <= 256; lane 15's value is not used
        // C(beta_lv) in the format's order, the five table reads together
        const float bq = bin_edge(lv);
        int ji[N_MIX];
        float wf[N_MIX];
#pragma unroll
        for (int k = 0; k < N_MIX; ++k) {
          float u = bq * pv[N_MIX + k] + pv[2 * N_MIX + k];
          u = u > 0.0f ? u : 0.0f;
          u = fminf(u, 4096.0f);
          ji[k] = (int)u;
          wf[k] = __builtin_amdgcn_fractf(u);
        }
        float2 e[N_MIX];
#pragma unroll
        for (int k = 0; k < N_MIX; ++k) e[k] = s_sd[ji[k]];
        // the batch of the next sub-round goes out behind the table reads
        // (unconditionally, so that the wait for the table reads can leave it
        // in flight; past the last sub-round it is not used)
        {
          const int sn = (q + 1) & (NSLOT - 1);
          __builtin_amdgcn_sched_barrier(0);
          nd = __hip_atomic_load(&s_done[sn][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          asm volatile("" ::: "memory");
          __builtin_amdgcn_sched_barrier(0);
          const f4* nq = reinterpret_cast<const f4*>(&s_par[sn][cl * PAR_STRIDE]);
          n0 = nq[0];
          n1 = nq[1];
          n2 = nq[2];
          n3 = nq[3];
          nFb = s_bk[sn][cl * 16 + h];
          pre_q = q + 1;
        }
        // the table values are used only from here on, with the batch in flight
        __builtin_amdgcn_sched_barrier(0);
        float sg[N_MIX];
#pragma unroll
        for (int k = 0; k < N_MIX; ++k) sg[k] = e[k].x + wf[k] * e[k].y;
        float clo = pv[0] * sg[0];
        clo = clo + pv[1] * sg[1];
        clo = clo + pv[2] * sg[2];
        float chi = pv[3] * sg[3];
        chi = chi + pv[4] * sg[4];
        // every lane evaluates (lane 15's value is dropped), so that no
        // branch makes the wait for the table reads also wait for the batch
        uint32_t Fe = F_of_C(lv, clo + chi);
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t Fk = h < N_BUCKET ? Fe : Fhi;
        const bool le2 = Fk <= slot;
        const uint32_t k2 = row16_max(le2 ? (((uint32_t)(h + 1) << 17) | Fk) : 0u);
        const uint32_t F2 = row16_min(le2 ? M_TOTAL : Fk);
        const int cnt = min((int)(k2 >> 17), N_BUCKET);
        const int v = base + cnt;
        const uint32_t c = cnt > 0 ? (k2 & 0x1FFFFu) : (klo & 0x1FFFFu);
        const uint32_t f = F2 - c;
        if (a.prof) c_sr = clk_now();
        // f <= 2^16 - 255 and x >> 16 < 2^16: the 24-bit multiplier is exact
        const uint32_t xd = __umul24(f, x >> 16) + slot - c;
        const bool ren = act && !bad && xd < RANS_L;
        const uint64_t mr = __ballot(ren) & row_heads;
        const uint32_t rk = (uint32_t)__popcll(mr & below);
        const int wo = (int)(Pw - wbase);  // <= 60
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)wwin, wo);
        const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)wwin, wo + 1);
        const uint32_t w2 = (uint32_t)__builtin_amdgcn_readlane((int)wwin, wo + 2);
        const uint32_t w3 = (uint32_t)__builtin_amdgcn_readlane((int)wwin, wo + 3);
        uint32_t w = rk == 0 ? w0 : (rk == 1 ? w1 : (rk == 2 ? w2 : w3));
        const bool past = ren && Pw + rk >= n_words;
        over = over || past;
        w = past ? 0u : w;
        x = act ? (ren ? ((xd << 16) | w) : xd) : x;
        Pw += (uint32_t)__popcll(mr);
        if (act && h == 0) s_ring[(rr + 2) * 16 + (xc & 15)] = (uint8_t)v;
      }
      if (lane == 0) {
        // LDS performs this wave's ring store before these two stores
        asm volatile("" ::: "memory");
        __hip_atomic_store(&s_pw, Pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&s_decoded, q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (a.prof) {
        const unsigned long long c2 = clk_now();
        t_wait += c1 - c0;
        if (j == 0) t_wait0 += c1 - c0;
        t_busy += c2 - c1;
        if (c_sr) {
          t_load += c_ld - c1;
          t_search += c_sr - c_ld;
        }
        c_ld = c_sr = 0;
      }
    }
    coder_strip_end(a, g, last_strip, lane, cl < L, x, Pw, n_words, over || bad, stuck, timeout,
                    s_x, &s_pw, &s_stop);
    if (lane == 0 && a.prof) {
      // counters add up over the strips (the caller clears them)
      a.prof[g * PROF_SLOTS + 0] += t_wait;
      a.prof[g * PROF_SLOTS + 1] += t_busy;
      a.prof[g * PROF_SLOTS + 8] += t_load;
      a.prof[g * PROF_SLOTS + 9] += t_search;
      a.prof[g * PROF_SLOTS + 10] += (unsigned long long)P;
      a.prof[g * PROF_SLOTS + 12] += t_late;
      a.prof[g * PROF_SLOTS + 13] += clk_now() - k0;
      a.prof[g * PROF_SLOTS + 14] += __builtin_amdgcn_s_memrealtime() - rt0;
      a.prof[g * PROF_SLOTS + 15] += n_late;
    }
  } else if (!TABLES && wave == 4) {
    // --------------------------------------------------------------- courier
    // Carries rows between groups, both ways:
    //  * after each finished step, rows r1-2 and r1-1 go to the next group as
    //    one record, and a row whose last pixel was decoded in this step
    //    stores that pixel to the image (density waves store every other
    //    pixel one step later);
    //  * records of the group above are polled ahead of need, eight steps per
    //    vector load, and put into ring rows 0 and 1, up to RCV_AHEAD steps
    //    beyond the coder's step, so no density wave waits on global memory.
    // The ring keeps 16 columns: record s shares its columns with s + 16, and
    // a density wave of step t reads records t-8 .. t-1, so storing at most 7
    // steps ahead of the coder never overwrites a column still to be read.
    // The coder waits for this wave only to keep its own rows from being
    // overwritten before they are published.
    int pub_t = t_first;      // next own step to publish
    int rcv = t_first - 1;    // next upstream record to receive
    const int rcv_last = b > 0 ? up_last : rcv - 1;
    bool stuck = false, timeout = s_flag != 0;
    uint32_t idle = 0, rspins = 0;
    while ((pub_t <= t_last || (rcv <= rcv_last && !timeout)) && !stuck) {
      if constexpr (DELAY) inject_delay(a, 4u, (uint32_t)g, (uint32_t)(pub_t * 8 + rcv));
      bool progress = false;
      const int done_q = lds_acquire(&s_decoded);
      while (pub_t <= t_last && done_q >= (pub_t - t_first + 1) * J) {
        if (lane == 0 && b + 1 < GS) {
          const int d1 = pub_t - SKEW * (r1 - 1), d2 = pub_t - SKEW * (r1 - 2);
          uint32_t rv = 0x80000000u;
          if (d1 >= 0 && d1 < W) rv |= (uint32_t)s_ring[(R - 1 + 2) * 16 + (d1 & 15)];
          if (d2 >= 0 && d2 < W) rv |= (uint32_t)s_ring[(R - 2 + 2) * 16 + (d2 & 15)] << 8;
          __hip_atomic_store(my_rec + pub_t, rv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // row y ends in step pub_t when pub_t - SKEW y = W - 1
        const int ye = pub_t - (W - 1);
        if (lane == 1 && ye >= 0 && ye % SKEW == 0) {
          const int y = ye / SKEW;
          if (y >= r0 && y < r1)
            a.img[(long long)y * W + (W - 1)] = s_ring[(y - r0 + 2) * 16 + ((W - 1) & 15)];
        }
        if (lane == 0) {
          asm volatile("" ::: "memory");
          __hip_atomic_store(&s_pub, pub_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        ++pub_t;
        progress = true;
      }
      const int lim = min(rcv_last, t_first + done_q / J + RCV_AHEAD);
      if (rcv <= lim && !timeout) {
        const int sr = rcv + lane;
        uint32_t v = 0;
        if (lane < 8 && sr <= lim)
          v = __hip_atomic_load(up_rec + sr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t okm = __ballot((v >> 31) != 0u);
        const int n = (int)__builtin_ctzll(~okm);  // leading run of valid records
        if (lane < n) stash_record(s_ring, v, sr, r0, W);
        if (n > 0) {
          rcv += n;
          if (lane == 0) {
            asm volatile("" ::: "memory");
            __hip_atomic_store(&s_rcv, rcv - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
          progress = true;
          rspins = 0;
        } else if (++rspins > a.spin_limit) {
          timeout = true;
        }
      }
      if (progress) {
        idle = 0;
      } else {
        if (++idle > LDS_SPIN_LIMIT) stuck = true;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (lane == 0) {
      // density waves stop waiting for records that will not come
      if (timeout || stuck) {
        __hip_atomic_store(&s_rcv, 0x7FFFFFFF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        s_stop = 1;
      }
      if (stuck) atomicMax(a.status, 3);
      if (timeout) atomicMax(a.status, 7);
    }
  } else if (wave == 0) {
    // ------------------------------------------------------------------ coder
    const int cl = lane;  // the pixel (coder lane) this lane serves
    uint32_t x = RANS_L;
    if (!first_strip)
      x = s_x[lane];
    else if (cl < L && !bad)
      x = (uint32_t)gw[2 * cl] | ((uint32_t)gw[2 * cl + 1] << 16);
    uint32_t Pw = first_strip ? 2u * (uint32_t)L : s_pw;  // words consumed
    bool over = false, stuck = false, timeout = s_flag != 0;
    // words known to be in the ring
    uint32_t E = first_strip
                     ? E0
                     : __hip_atomic_load(&s_end, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    int t = t_first, j = -1, pub = t_first - 1;
    const unsigned long long k0 = a.prof ? clk_now() : 0ull;
    const unsigned long long rt0 = a.prof ? __builtin_amdgcn_s_memrealtime() : 0ull;
    for (int q = 0; q < P; ++q) {
      if constexpr (DELAY) inject_delay(a, 3u, (uint32_t)g, (uint32_t)q);
      if (++j == J) {
        j = 0;
        ++t;
      }
      if (TABLES) {
        // no density waves here: the coder keeps its own ring filled
        if (!bad && E < n_words && E - Pw <= (uint32_t)(DEC_RING - 2 * REFILL_WORDS)) {
          uint16_t pre[REFILL_WORDS / 64];
#pragma unroll
          for (int i = 0; i < REFILL_WORDS / 64; ++i) {
            const uint32_t pos = E + (uint32_t)(i * 64 + lane);
            pre[i] = pos < n_words ? gw[pos] : (uint16_t)0;
          }
#pragma unroll
          for (int i = 0; i < REFILL_WORDS / 64; ++i)
            s_words[(E + (uint32_t)(i * 64 + lane)) & RING_MASK] = pre[i];
          E = min(n_words, E + (uint32_t)REFILL_WORDS);
        }
      } else if (!bad && E < n_words && Pw + 64u > E && !stuck) {
        // a sub-round takes at most 64 words; the ring owner keeps ahead
        uint32_t spins = 0;
        while ((E = __hip_atomic_load(&s_end, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) <
                   min(n_words, Pw + 64u)) {
          if (++spins > LDS_SPIN_LIMIT) {
            stuck = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (!TABLES && j == 0 && !stuck) stuck = !wait_publisher(&s_pub, t, pub);
      const int rr = j * L + cl;
      const int y = r0 + rr;
      const int xc = t - SKEW * y;
      const bool act = cl < L && rr < R && xc >= 0 && xc < W;
      const bool any = __ballot(act) != 0ull;
      const int slot_i = q & (NSLOT - 1);
      const unsigned long long c0 = a.prof ? clk_now() : 0ull;
      if (!TABLES && any && !stuck) {
        // all tiles' flags in one round of relaxed loads, then one acquire
        uint32_t spins = 0;
        for (;;) {
          int n_ready = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int d = __hip_atomic_load(&s_done[slot_i][i], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
            n_ready += (i < NT && d == q) ? 1 : 0;
          }
          if (n_ready == NT) break;
          // no sleep: the coder has its SIMD to itself
          if (++spins > LDS_SPIN_LIMIT) {
            stuck = true;
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      const unsigned long long c1 = a.prof ? clk_now() : 0ull;
      if (any) {
        const uint32_t slot = x & 0xFFFFu;
        int v = 0;
        uint32_t c = 0, f = 1;
        if (TABLES) {
          uint32_t ti = act ? a.tidx[(long long)y * W + xc] : 0u;
          if (ti >= (uint32_t)a.n_tables) {
            over = over || act;
            ti = 0;
          }
          const uint32_t* tab = a.tables + (long long)ti * 257;
          find_symbol(slot, [&](int lv) { return tab[lv]; }, v, c, f);
        } else {
          // With L <= 32 the two half-waves share the work of each pixel:
          // lanes i and 32 + i both serve pixel i, the low half evaluating
          // mixture components 0..2 and the high half components 3..4 (plus
          // a zero-weight pad), joined by one cross-half swap.  With L > 32
          // every lane evaluates both parts.  Either way C is the format's
          // (part 0..2) + (part 3..4), so every lane takes the same decisions.
          constexpr bool split = LPP == 2;
          const int hlf = split ? (lane >> 5) : 0;
          uint32_t sl = slot;
          int px = act ? lane : 0;
          if (split) {
            const auto sx = __builtin_amdgcn_permlane32_swap(slot, slot, false, false);
            const auto sa = __builtin_amdgcn_permlane32_swap((uint32_t)px, (uint32_t)px, false, false);
            sl = sx[0];
            px = (int)sa[0];
          }
          const float* pp = &s_par[slot_i][px * PAR_STRIDE];
          // component slots of this lane: k0 .. k0+2 (k0 = 0 or 3); slot 2 of
          // the high half is the pad
          const int k0 = 3 * hlf;
          float cp[3], cA[3], cB[3], dp[2], dA[2], dB[2];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const bool pad = hlf == 1 && i == 2;
            cp[i] = pad ? 0.0f : pp[k0 + i];
            cA[i] = pad ? 0.0f : pp[N_MIX + k0 + i];
            cB[i] = pad ? 0.0f : pp[2 * N_MIX + k0 + i];
          }
          if (!split) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              dp[i] = pp[3 + i];
              dA[i] = pp[N_MIX + 3 + i];
              dB[i] = pp[2 * N_MIX + 3 + i];
            }
          }
          const uint16_t* bk = &s_bk[slot_i][px * 16];
          int nb = 0;
          if (split) {
            // low half counts boundaries 0..7, high half 8..14
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int bi = 8 * hlf + i;
              nb += (bi < N_BUCKET && (uint32_t)bk[bi] <= sl) ? 1 : 0;
            }
            const auto sn = __builtin_amdgcn_permlane32_swap((uint32_t)nb, (uint32_t)nb, false, false);
            nb = (int)(sn[0] + sn[1]);
          } else {
#pragma unroll
            for (int i = 0; i < N_BUCKET; ++i) nb += ((uint32_t)bk[i] <= sl) ? 1 : 0;
          }
          const int base = 16 * nb;
          uint32_t Flo = nb > 0 ? (uint32_t)bk[nb - 1] : 0u;
          uint32_t Fhi = nb < N_BUCKET ? (uint32_t)bk[nb] : M_TOTAL;
          // bin edges of the whole bucket in registers (levels base .. base+15)
          float be[16];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const f4 v4 = *reinterpret_cast<const f4*>(&s_beta[base + 4 * i]);
            be[4 * i] = v4[0];
            be[4 * i + 1] = v4[1];
            be[4 * i + 2] = v4[2];
            be[4 * i + 3] = v4[3];
          }
          if (a.prof) c_ld = clk_now();
          int off = 0;
#pragma unroll
          for (int it = 0; it < 4; ++it) {
            const int step = 8 >> it;
            // edge of level base + off + step, picked from registers
            float b = be[0];
#pragma unroll
            for (int c = 1; c < 16; ++c)
              if (c % step == 0) b = (off + step == c) ? be[c] : b;
            const int mid = base + off + step;
            const float part = cdf_part(b, cp, cA, cB, 3, s_sd);
            float C;
            if (split) {
              const auto pc = __builtin_amdgcn_permlane32_swap(__float_as_uint(part),
                                                               __float_as_uint(part), false, false);
              C = __uint_as_float(pc[0]) + __uint_as_float(pc[1]);
            } else {
              C = part + cdf_part(b, dp, dA, dB, 2, s_sd);
            }
            const uint32_t Fm = F_of_C(mid, C);
            if (Fm <= sl) {
              off += step;
              Flo = Fm;
            } else {
              Fhi = Fm;
            }
          }
          const int lo = base + off;
          v = lo;
          c = Flo;
          f = Fhi - Flo;
          if (a.prof) c_sr = clk_now();
        }
        // f <= 2^16 - 255 and x >> 16 < 2^16: the 24-bit multiplier is exact
        if (act) x = __umul24(f, x >> 16) + slot - c;
        Pw = rans_dec_renorm(x, act && !bad, Pw, n_words,
                             [&](uint32_t pos) { return (uint32_t)s_words[pos & RING_MASK]; }, over);
        if (act) {
          s_ring[(rr + 2) * 16 + (xc & 15)] = (uint8_t)v;
          // density waves store a pixel to the image one step later and the
          // publisher wave a row's last pixel
          if (TABLES) a.img[(long long)y * W + xc] = (uint8_t)v;
        }
      }
      if (lane == 0) {
        s_pw = Pw;
        lds_release(&s_decoded, q + 1);
      }
      if (a.prof) {
        const unsigned long long c2 = clk_now();
        t_wait += c1 - c0;
        if (j == 0) t_wait0 += c1 - c0;
        t_busy += c2 - c1;
        if (c_sr) {
          t_load += c_ld - c1;
          t_search += c_sr - c_ld;
        }
        c_ld = c_sr = 0;
      }
      // after the last block of step t, hand rows r1-2 and r1-1 to the next
      // group (with density waves the publisher wave does this)
      if (TABLES && j == J - 1 && lane == 0 && b + 1 < GS) {
        const int d1 = t - SKEW * (r1 - 1), d2 = t - SKEW * (r1 - 2);
        uint32_t rv = 0x80000000u;
        if (d1 >= 0 && d1 < W) rv |= (uint32_t)s_ring[(R - 1 + 2) * 16 + (d1 & 15)];
        if (d2 >= 0 && d2 < W) rv |= (uint32_t)s_ring[(R - 2 + 2) * 16 + (d2 & 15)] << 8;
        __hip_atomic_store(my_rec + t, rv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // the table coder keeps its own ring: its end carries to the next strip
    if (TABLES && lane == 0 && !last_strip) s_end = E;
    coder_strip_end(a, g, last_strip, lane, cl < L, x, Pw, n_words, over || bad, stuck, timeout,
                    s_x, &s_pw, &s_stop);
    if (lane == 0 && a.prof) {
      a.prof[g * PROF_SLOTS + 0] += t_wait;
      a.prof[g * PROF_SLOTS + 1] += t_busy;
      a.prof[g * PROF_SLOTS + 8] += t_load;
      a.prof[g * PROF_SLOTS + 9] += t_search;
      a.prof[g * PROF_SLOTS + 10] += (unsigned long long)P;
      a.prof[g * PROF_SLOTS + 12] += t_wait0;
      a.prof[g * PROF_SLOTS + 13] += clk_now() - k0;
      a.prof[g * PROF_SLOTS + 14] += __builtin_amdgcn_s_memrealtime() - rt0;
    }
  } else if (!TABLES) {
    // -------------------------------------------------------- density waves
    // waves 4, 8, ... share the coder's SIMD and compute no densities
    {
    if ((wave & 3) == 0) return;
    constexpr int nwork = dec_workers<Net>();
    const int w = wave - 1 - (wave >> 2);
    Net net;
    net.load(m, lane);
    if constexpr (Net::SCRATCH_FLOATS > 0) net.xs = &s_xs[w * Net::SCRATCH_FLOATS];
    const int q4 = lane >> 4;
    unsigned long long t_net = 0, t_head = 0, t_tab = 0, n_tiles = 0, c_net = 0, c_head = 0;
    bool timeout = s_flag != 0;
    bool stuck = false;
    // tile tau = NT * q + ti of sub-round q = (t - t_first) * J + j, every nwork-th
    int q = 0, ti = w, t = t_first, j = 0;
    while (ti >= NT) {
      ti -= NT;
      ++q;
    }
    j = q % J;
    t = t_first + q / J;
    for (;; ) {
      if (q >= P) break;
      const int slot_i = q & (NSLOT - 1);
      const int need = max(q - J + 1, q - NSLOT + 1);
      // With the 4-pixel net a tile starts once the step before last is
      // decoded (every window pixel but the up-right and the left one, which
      // come with the last step, J sub-rounds before this one) and runs layer
      // 1 that far; it then waits for the last step.
      constexpr bool SPLIT = Net::SCRATCH_FLOATS > 0;
      const int need_pre = SPLIT ? max(q - 2 * J + 1, q - NSLOT + 1) : need;
      if constexpr (DELAY) inject_delay(a, 8u + (uint32_t)wave, (uint32_t)g, (uint32_t)q);
      const unsigned long long c0 = a.prof ? clk_now() : 0ull;
      auto wait_decoded = [&](int n) {
        if (stuck) return;
        uint32_t spins = 0;
        while (lds_acquire(&s_decoded) < n) {
          if (++spins > LDS_SPIN_LIMIT) {
            stuck = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      };
      wait_decoded(need_pre);
      const unsigned long long c1 = a.prof ? clk_now() : 0ull;
      unsigned long long c_late = 0;  // cycles of the second wait
      // density wave 0 keeps the stream ring ahead of the coder
      if (w == 0 && !bad) {
        const uint32_t end = s_end;
        const uint32_t pw = __hip_atomic_load(&s_pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (end < n_words && end - pw <= (uint32_t)(DEC_RING - 2 * REFILL_WORDS)) {
          uint16_t pre[REFILL_WORDS / 64];
#pragma unroll
          for (int i = 0; i < REFILL_WORDS / 64; ++i) {
            const uint32_t pos = end + (uint32_t)(i * 64 + lane);
            pre[i] = pos < n_words ? gw[pos] : (uint16_t)0;
          }
#pragma unroll
          for (int i = 0; i < REFILL_WORDS / 64; ++i)
            s_words[(end + (uint32_t)(i * 64 + lane)) & RING_MASK] = pre[i];
          if (lane == 0)
            __hip_atomic_store(&s_end, min(n_words, end + (uint32_t)REFILL_WORDS), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      const int ln = 16 * ti + (lane & 15);  // coder lane of this pixel
      const int rr = j * L + ln;
      const int y = r0 + rr;
      const int xc = t - SKEW * y;
      const bool valid = ln < L && rr < R && xc >= 0 && xc < W;
      const bool any_valid = __ballot(valid) != 0ull;
      // the tile holding row r0 needs the group above's step s in the ring;
      // the courier has usually put it there already
      auto wait_record = [&](int s) {
        if (rr == 0 && valid && lane == 0 && b > 0 && s <= up_last && !stuck) {
          uint32_t spins = 0;
          while (lds_acquire(&s_rcv) < s) {
            if (++spins > LDS_SPIN_LIMIT) {
              stuck = true;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
      };
      // window pixel kk of this lane (feature 4 kk + q4; a neighbour outside
      // the image reads ring slot 0 and is replaced by 0), scaled
      // arithmetically to the table's value
      auto feature = [&](int kk) {
        const int k = 4 * kk + q4;
        const int yy = y + nb_dy(k), xx = xc + nb_dx(k);
        const bool inside = valid && yy >= 0 && xx >= 0 && xx < W;
        const uint32_t pv = s_ring[inside ? (yy - r0 + 2) * 16 + (xx & 15) : 0];
        const float sv = div255((int)(2 * pv) - 255);
        return inside ? sv : 0.0f;
      };
      float fk[3] = {0.0f, 0.0f, 0.0f};
      [[maybe_unused]] typename NetL1<Net>::type l1{};
      if constexpr (SPLIT) {
        if (any_valid) {
          wait_record(t - 2);
          // lane groups 1 and 3 hold features 9 and 11 in slot 2: read later
          fk[0] = feature(0);
          fk[1] = feature(1);
          if ((q4 & 1) == 0) fk[2] = feature(2);
          l1 = net.l1_pre(fk[0], fk[1], fk[2]);
        }
        const unsigned long long cl0 = a.prof ? clk_now() : 0ull;
        wait_decoded(need);
        if (a.prof) c_late = clk_now() - cl0;
      }
      if (any_valid) {
        wait_record(t - 1);
        if constexpr (SPLIT) {
          if ((q4 & 1) != 0) fk[2] = feature(2);
        } else {
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) fk[kk] = feature(kk);
        }
        // the left neighbour (decoded last step) goes to the image
        if (valid && q4 == 0 && xc >= 1)
          a.img[(long long)y * W + xc - 1] = s_ring[(rr + 2) * 16 + ((xc - 1) & 15)];
        f4 o;
        if constexpr (SPLIT)
          o = net.finish(l1, fk[2], s_w2);
        else
          o = net.run(fk[0], fk[1], fk[2], s_w2);
        float* par = &s_par[slot_i][0];
        if (a.prof) {
          c_net = clk_now();
          ++n_tiles;
        }
        if (valid) *reinterpret_cast<f4*>(&par[ln * PAR_STRIDE + 4 * q4]) = o;
        wave_lds_handover();
        if (SPX == 4 || L <= 4) {
          // At most 4 pixels: row p of the wave (lanes 16 p + k) serves pixel
          // p.  Lane k < 5 evaluates mixture component k (the head's two
          // exponentials), lane 0 the softmax sum in the head's order, and lane
          // h < 15 the boundary F(16 (h + 1)); every value equals the one
          // mixture_head and cdf_F give.  LDS serves the wave's reads and
          // writes in program order.
          const int p = lane >> 4, k = lane & 15;
          const int rp = j * L + p, yp = r0 + rp, xp = t - SKEW * yp;
          const bool pv = p < L && rp < R && xp >= 0 && xp < W;
          float* pp = &par[p * PAR_STRIDE];
          if (pv && k < N_MIX) {
            float lg[N_MIX];
#pragma unroll
            for (int i = 0; i < N_MIX; ++i) lg[i] = pp[i];
            const float mu = pp[N_MIX + k], ls = pp[2 * N_MIX + k], ok = pp[k];
            float m = lg[0];
#pragma unroll
            for (int i = 1; i < N_MIX; ++i) m = fmaxf(m, lg[i]);
            const float e = expf(ok - m);
            const float inv_s = expf(-fmaxf(ls, LOG_SCALE_MIN));
            const float A = inv_s * 128.0f;
            const float B = 2048.0f - mu * A;
            pp[k] = e;
            pp[N_MIX + k] = A;
            pp[2 * N_MIX + k] = B;
          }
          wave_lds_handover();
          if (pv && k < N_MIX) {
            float sm = 0.0f;
#pragma unroll
            for (int i = 0; i < N_MIX; ++i) sm = sm + pp[i];
            const float rs = 1.0f / sm;
            const float e = pp[k];
            pp[k] = e * rs;
          }
          wave_lds_handover();
          if (a.prof) c_head = clk_now();
          if (pv && k < N_BUCKET) {
            Mix mx;
#pragma unroll
            for (int i = 0; i < N_MIX; ++i) {
              mx.pi[i] = pp[i];
              mx.A[i] = pp[N_MIX + i];
              mx.B[i] = pp[2 * N_MIX + i];
            }
            s_bk[slot_i][p * 16 + k] = (uint16_t)cdf_F(16 * (k + 1), mx, s_sd, s_beta);
          }
        } else {
        // mixture head, one lane per pixel
        if (lane < 16 && valid) {
          float* pp = &par[ln * PAR_STRIDE];
          float ov[N_OUT];
#pragma unroll
          for (int k = 0; k < N_OUT; ++k) ov[k] = pp[k];
          const Mix mx = mixture_head(ov);
#pragma unroll
          for (int k = 0; k < N_MIX; ++k) {
            pp[k] = mx.pi[k];
            pp[N_MIX + k] = mx.A[k];
            pp[2 * N_MIX + k] = mx.B[k];
          }
        }
        wave_lds_handover();
        if (a.prof) c_head = clk_now();
        // table at the bucket boundaries 16, 32, ..., 240
        if (valid) {
          // four boundaries per lane
          const float* pp = &par[ln * PAR_STRIDE];
          Mix mx;
#pragma unroll
          for (int k = 0; k < N_MIX; ++k) {
            mx.pi[k] = pp[k];
            mx.A[k] = pp[N_MIX + k];
            mx.B[k] = pp[2 * N_MIX + k];
          }
          uint16_t* bk = &s_bk[slot_i][ln * 16];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int mb = q4 + 4 * i + 1;
            if (mb <= N_BUCKET) bk[mb - 1] = (uint16_t)cdf_F(16 * mb, mx, s_sd, s_beta);
          }
        }
        }
      }
      if constexpr (DELAY) inject_delay(a, 32u + (uint32_t)wave, (uint32_t)g, (uint32_t)q);
      if (lane == 0) lds_release(&s_done[slot_i][ti], q);
      if (a.prof) {
        const unsigned long long c2 = clk_now();
        t_wait += c1 - c0 + c_late;
        t_busy += c2 - c1 - c_late;
        if (c_net) {
          t_net += c_net - c1 - c_late;
          t_head += c_head - c_net;
          t_tab += c2 - c_head;
        }
        c_net = c_head = 0;
      }
      // next tile of this wave
      ti += nwork;
      while (ti >= NT) {
        ti -= NT;
        ++q;
        if (++j == J) {
          j = 0;
          ++t;
        }
      }
    }
    if (lane == 0) {
      if (stuck || timeout) s_stop = 1;
      if (stuck) atomicMax(a.status, 3);
      if (timeout) atomicMax(a.status, 7);
      if (a.prof) {
        atomicAdd(&a.prof[g * PROF_SLOTS + 2], t_wait);
        atomicAdd(&a.prof[g * PROF_SLOTS + 3], t_busy);
        atomicAdd(&a.prof[g * PROF_SLOTS + 4], t_net);
        atomicAdd(&a.prof[g * PROF_SLOTS + 5], t_head);
        atomicAdd(&a.prof[g * PROF_SLOTS + 6], t_tab);
        atomicAdd(&a.prof[g * PROF_SLOTS + 7], n_tiles);
      }
    }
    }
  }
  };
  if constexpr (STRIPS == 1) {
    strip(0);
  } else if constexpr (STRIPS == 2) {
    strip(0);
    // the strip is done on every wave; a failed strip ends the group
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_stop) == 0) strip(1);
  } else {
    for (int sp = 0; sp < n_strips; ++sp) {
      strip(sp);
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_stop) != 0) break;
    }
  }
}

// One image: each workgroup takes its group by ticket, so group g - 1 was
// taken by a workgroup that is running or done before group g waits on it,
// whatever order the dispatcher starts workgroups in.
template <class Net, bool TABLES, int LPP, bool DELAY = false, int STRIPS = 1>
__global__ __launch_bounds__(dec_waves<Net>() * 64) void wavefront_decode_kernel(
    const Consts* __restrict__ K, DevModel m, DecArgs a) {
  __shared__ int s_group;
  if (threadIdx.x == 0) s_group = (int)atomicAdd(a.ticket, 1u);
  __syncthreads();
  const int g = __builtin_amdgcn_readfirstlane(s_group);
  if (g >= a.G) return;
  decode_group<Net, TABLES, LPP, DELAY, STRIPS>(K, m, a, g);
}

// Batched decode, persistent: a grid of resident workgroups, each taking the
// next work item by ticket until the list is empty.  Items list the groups
// of an image in order, and a workgroup finishes its item before it takes
// another, so the group an item waits for was taken earlier by a workgroup
// that is running or done: the waits end.  The last group of an image to
// finish stamps the image's completion time.
template <class Net, int LPP, bool DELAY = false>
__global__ __launch_bounds__(dec_waves<Net>() * 64) void batch_decode_kernel(
    const Consts* __restrict__ K, DevModel m, BatchArgs b) {
  __shared__ int s_item;
  if (threadIdx.x == 0) s_item = (int)atomicAdd(b.ticket, 1u);
  __syncthreads();
  // The item is read as a wave-uniform value, so every wave leaves or repeats
  // the loop as a whole.  Read per lane, the loop's exit would be divergent,
  // and the compiler may then send lanes 1..63 of wave 0 back to the top
  // barrier ahead of lane 0, before it has taken the next ticket.
  int item = __builtin_amdgcn_readfirstlane(s_item);
  while (item < b.n_items) {
    const BatchItem it = b.items[item];
    const BatchImage im = b.images[it.image];
    DecArgs a;
    a.bits = b.bits + im.out_off;
    // a length beyond the region is corrupt; 0 makes the header check say so
    a.n_bytes = b.len[it.image] <= (unsigned long long)im.out_cap ? b.len[it.image] : 0ull;
    a.img = b.pix_out + im.px_off;
    a.H = im.H;
    a.W = im.W;
    a.G = im.G;
    a.L = im.L;
    a.S = 1;
    a.rec = b.rec + im.rec_off;
    a.ticket = nullptr;
    a.T = im.T;
    a.status = b.status + it.image;
    a.spin_limit = b.spin_limit;
    a.delay_seed = b.delay_seed;
    a.delay_max = b.delay_max;
    a.check_model = 1;
    a.hf = b.hf;
    a.tables = nullptr;
    a.n_tables = 0;
    a.tidx = nullptr;
    a.prof = nullptr;
    decode_group<Net, false, LPP, DELAY>(K, m, a, it.group);
    // every wave is done with the item (and with the LDS of decode_group)
    // before thread 0 counts it and takes the next ticket
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(b.done + it.image, 1u) + 1u == (unsigned)im.G && b.t_done)
        b.t_done[it.image] = __builtin_amdgcn_s_memrealtime();
      s_item = (int)atomicAdd(b.ticket, 1u);
    }
    __syncthreads();
    item = __builtin_amdgcn_readfirstlane(s_item);
  }
}

// Workgroups of a persistent batch decode: as many as stay resident at once,
// at most one per work item.
template <class Kern>
static int persistent_grid(Kern kern, int threads, int n_items) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess)
    per_cu = 0;
  long long g = (long long)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  if (g > n_items) g = n_items;
  return (int)(g > 0 ? g : 1);
}

template <class Net, int LPP, bool DELAY>
static void launch_batch_decode_d(const Consts* K, const DevModel& m, const BatchArgs& b,
                                  int grid_cap, hipStream_t s) {
  const int threads = dec_waves<Net>() * 64;
  int grid = persistent_grid(batch_decode_kernel<Net, LPP, DELAY>, threads, b.n_items);
  if (grid_cap > 0 && grid_cap < grid) grid = grid_cap;
  hipLaunchKernelGGL((batch_decode_kernel<Net, LPP, DELAY>), dim3(grid), dim3(threads), 0, s, K,
                     m, b);
}

// The delay-injecting form (a test hook) is a separate kernel, so that the
// production kernel carries no trace of it.
template <class Net, int LPP>
static void launch_batch_decode_k(const Consts* K, const DevModel& m, const BatchArgs& b,
                                  int grid_cap, hipStream_t s) {
  if (b.delay_max > 0)
    launch_batch_decode_d<Net, LPP, true>(K, m, b, grid_cap, s);
  else
    launch_batch_decode_d<Net, LPP, false>(K, m, b, grid_cap, s);
}

__global__ void stamp_kernel(unsigned long long* t) {
  if (threadIdx.x == 0) *t = __builtin_amdgcn_s_memrealtime();
}

void launch_stamp(unsigned long long* t, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, t);
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

template <class Net>
static void launch_batch_decode_t(const Consts* K, const DevModel& m, const BatchArgs& b,
                                  int lpp, int cap, hipStream_t s) {
  if (lpp == 16)
    launch_batch_decode_k<Net, 16>(K, m, b, cap, s);
  else if (lpp == 2)
    launch_batch_decode_k<Net, 2>(K, m, b, cap, s);
  else
    launch_batch_decode_k<Net, 1>(K, m, b, cap, s);
}

template <int H>
static bool launch_batch_decode_h(int wtype, const Consts* K, const DevModel& m,
                                  const BatchArgs& b, int lpp, int cap, hipStream_t s) {
  switch (wtype) {
    case WT_F32:
      // as for one image: nets of 64 or 128 neurons on tiles of at most 4 pixels
      if (H >= 64 && lpp == 16) {
        launch_batch_decode_k<NetF32x4<(H >= 64 ? H : 64), (H == 64)>, 16>(K, m, b, cap, s);
      } else {
        launch_batch_decode_t<NetF32<H, (H >= 64)>>(K, m, b, lpp, cap, s);
      }
      return true;
    case WT_BF16:
      launch_batch_decode_t<NetBF16<H, WT_BF16, (H > 64)>>(K, m, b, lpp, cap, s);
      return true;
    case WT_FP8:
      launch_batch_decode_t<NetBF16<H, WT_FP8, (H > 64)>>(K, m, b, lpp, cap, s);
      return true;
    case WT_FP8A8:
      launch_batch_decode_t<NetFP8A<H, (H > 64)>>(K, m, b, lpp, cap, s);
      return true;
    default: return false;
  }
}

bool launch_batch_decode(int wtype, int width, const Consts* K, const DevModel& m,
                         const BatchArgs& b, int lpp, int grid_cap, hipStream_t s) {
  switch (width) {
    case 32: return launch_batch_decode_h<32>(wtype, K, m, b, lpp, grid_cap, s);
    case 64: return launch_batch_decode_h<64>(wtype, K, m, b, lpp, grid_cap, s);
    case 128: return launch_batch_decode_h<128>(wtype, K, m, b, lpp, grid_cap, s);
    default: return false;
  }
}

template <class Net, bool TABLES, int LPP>
static bool launch_wavefront(const Consts* K, const DevModel& m, const DecArgs& a, hipStream_t s) {
  const dim3 grid(a.G), block(dec_waves<Net>() * 64);
  // the delay-injecting forms (a test hook) are separate kernels, so that the
  // production kernels carry no trace of it
  auto go = [&](auto kern, auto kern_delay) {
    // With several strips per group, group 0's second strip waits for the last
    // group's first: every group's workgroup must be resident at once.
    if (a.S > 1 && persistent_grid(kern, (int)block.x, a.G) < a.G) return false;
    const auto k = a.delay_max > 0 ? kern_delay : kern;
    hipLaunchKernelGGL(k, grid, block, 0, s, K, m, a);
    return true;
  };
  if (a.S == 1)
    return go(wavefront_decode_kernel<Net, TABLES, LPP, false, 1>,
              wavefront_decode_kernel<Net, TABLES, LPP, true, 1>);
  if (a.S == 2)
    return go(wavefront_decode_kernel<Net, TABLES, LPP, false, 2>,
              wavefront_decode_kernel<Net, TABLES, LPP, true, 2>);
  return go(wavefront_decode_kernel<Net, TABLES, LPP, false, 0>,
            wavefront_decode_kernel<Net, TABLES, LPP, true, 0>);
}

// The table-driven coder (no density waves) runs one lane per pixel.
template <class Net, bool TB>
static bool launch_decode_t(const Consts* K, const DevModel& m, const DecArgs& a, hipStream_t s) {
  if constexpr (TB) {
    return launch_wavefront<Net, true, 1>(K, m, a, s);
  } else {
    const int lpp = coder_lpp(a.L);
    if (lpp == 16) return launch_wavefront<Net, false, 16>(K, m, a, s);
    if (lpp == 2) return launch_wavefront<Net, false, 2>(K, m, a, s);
    return launch_wavefront<Net, false, 1>(K, m, a, s);
  }
}

// Nets for tiles of at most 4 pixels run only with the 16-lane coder (L <= 4).
template <class Net>
static bool launch_decode_lpp16(const Consts* K, const DevModel& m, const DecArgs& a,
                                hipStream_t s) {
  return launch_wavefront<Net, false, 16>(K, m, a, s);
}

// Layer-2 weights of the BF16 nets go to LDS at H = 128: six density waves
// share one copy instead of holding 128 VGPRs each.
template <int H>
static bool launch_decode_h(int wtype, const Consts* K, const DevModel& m, const DecArgs& a,
                            hipStream_t s) {
  switch (wtype) {
    case WT_F32:
      // layouts of at most 4 lanes (one tile of at most 4 pixels per
      // sub-round, latency-bound): the 4-pixel 4x4 MFMA form at H = 64 and
      // 128; wider layouts need the 9 density waves of the 12-wave form at
      // H = 64
      // at 64 neurons the layer-2 weights sit in registers for one strip per
      // group; the strip-looping kernels keep them in LDS, which measured faster
      if (H == 64 && a.L <= 4 && a.S == 1) return launch_decode_lpp16<NetF32x4<64, true>>(K, m, a, s);
      if (H >= 64 && a.L <= 4) return launch_decode_lpp16<NetF32x4<(H >= 64 ? H : 64)>>(K, m, a, s);
      return launch_decode_t<NetF32<H, (H >= 64)>, false>(K, m, a, s);
    case WT_BF16: return launch_decode_t<NetBF16<H, WT_BF16, (H > 64)>, false>(K, m, a, s);
    case WT_FP8: return launch_decode_t<NetBF16<H, WT_FP8, (H > 64)>, false>(K, m, a, s);
    case WT_FP8A8: return launch_decode_t<NetFP8A<H, (H > 64)>, false>(K, m, a, s);
    default: return false;
  }
}

// False for an unsupported model or layout (nothing launched then).
bool launch_decode(int wtype, int width, bool tables_mode, const Consts* K, const DevModel& m,
                   const DecArgs& a, hipStream_t s) {
  if (tables_mode) return launch_decode_t<NetF32<32>, true>(K, m, a, s);
  switch (width) {
    case 32: return launch_decode_h<32>(wtype, K, m, a, s);
    case 64: return launch_decode_h<64>(wtype, K, m, a, s);
    case 128: return launch_decode_h<128>(wtype, K, m, a, s);
    default: return false;
  }
}

}  // namespace dlic
