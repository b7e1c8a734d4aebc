// C ABI of the DLIC hot path (see include/dlic.h for the contract of every
// entry point).  This file validates arguments, carves caller workspace,
// builds the format's constant tables once per device and enqueues the
// kernels; all per-pixel work happens in the kernels.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dlic.h"
#include "dlic_kernels.h"

using namespace dlic;

namespace {

constexpr int MAX_DEVICES = 64;
constexpr int MAX_TIMED = 16;

struct DeviceState {
  bool ready = false;
  Consts* consts = nullptr;
  void* scratch = nullptr;  // this device's address of `scratch` below
};

// Decode workspace of dlic_decode_noalloc: a fixed array in the code
// object, one copy per device, reserved until the process ends.  Host code
// never passes this name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address that ensure_device looks up.
constexpr size_t NOALLOC_SCRATCH_BYTES = DLIC_DECODE_NOALLOC_BYTES;
__device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
DeviceState g_dev[MAX_DEVICES];
uint32_t g_spin_limit = 1u << 22;
int g_deep_grid = 0;       // decode grid of the deep decoder; 0: by the step's tiles
int g_deep_grid_used = 0;  // the grid of the last deep decode launch
uint32_t g_delay_seed = 0, g_delay_max = 0;  // decoder delay injection (test hook)
unsigned long long* g_prof = nullptr;

struct TimedLaunch {
  const char* name;
  hipEvent_t start, stop;
};
bool g_timing = false;
std::vector<TimedLaunch> g_events;  // pool, reused
int g_n_timed = 0;

void build_consts(Consts* c) {
  for (int j = 0; j < LUT_N; ++j) {
    const double t = -16.0 + (double)j / 128.0;
    double s;
    if (t >= 0) {
      s = 1.0 / (1.0 + exp(-t));
    } else {
      const double e = exp(t);
      s = e / (1.0 + e);
    }
    c->sd[j].x = (float)s;
  }
  for (int j = 0; j < LUT_N; ++j) c->sd[j].y = (j + 1 < LUT_N) ? c->sd[j + 1].x - c->sd[j].x : 0.0f;
  for (int v = 0; v <= 256; ++v) c->beta[v] = ((float)(2 * v) - 256.0f) / 255.0f;
  c->beta[0] = -INFINITY;
  c->beta[256] = INFINITY;
  for (int v = 0; v < 256; ++v) c->scale[v] = ((float)(2 * v) - 255.0f) / 255.0f;
  for (int v = 0; v < 4096; ++v) c->scale12[v] = ((float)(2 * v) - 4095.0f) / 4095.0f;
}

dlic_status ensure_device(int device, const Consts** out) {
  if (device < 0 || device >= MAX_DEVICES) return DLIC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& st = g_dev[device];
  if (!st.ready) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return DLIC_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DLIC_ERR_UNSUPPORTED;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return DLIC_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return DLIC_ERR_HIP;
    Consts host;
    build_consts(&host);
    Consts* d = nullptr;
    void* sp = nullptr;
    dlic_status rc = DLIC_OK;
    if (hipMalloc((void**)&d, sizeof(Consts)) != hipSuccess ||
        hipMemcpy(d, &host, sizeof(Consts), hipMemcpyHostToDevice) != hipSuccess)
      rc = DLIC_ERR_HIP;
    // the no-alloc decode's workspace on this device (device current here)
    if (rc == DLIC_OK &&
        (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || sp == nullptr))
      rc = DLIC_ERR_HIP;
    (void)hipSetDevice(prev);
    if (rc != DLIC_OK) return rc;
    st.consts = d;
    st.scratch = sp;
    st.ready = true;
  }
  if (out) *out = st.consts;
  return DLIC_OK;
}

dlic_status current_consts(const Consts** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DLIC_ERR_HIP;
  return ensure_device(dev, out);
}

// --- timing -----------------------------------------------------------------
void timing_reset() { g_n_timed = 0; }

// Timing stays off while one of these lives (calls that must not allocate).
bool g_timing_off = false;
struct NoTiming {
  bool prev;
  NoTiming() : prev(g_timing_off) { g_timing_off = true; }
  ~NoTiming() { g_timing_off = prev; }
};

void timing_begin(const char* name, hipStream_t s) {
  if (!g_timing || g_timing_off) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_n_timed >= MAX_TIMED) return;
  if ((int)g_events.size() <= g_n_timed) {
    TimedLaunch tl;
    (void)hipEventCreate(&tl.start);
    (void)hipEventCreate(&tl.stop);
    g_events.push_back(tl);
  }
  g_events[g_n_timed].name = name;
  (void)hipEventRecord(g_events[g_n_timed].start, s);
}

void timing_end(hipStream_t s) {
  if (!g_timing || g_timing_off) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_n_timed >= MAX_TIMED) return;
  (void)hipEventRecord(g_events[g_n_timed].stop, s);
  ++g_n_timed;
}

dlic_status launch_ok() {
  return hipGetLastError() == hipSuccess ? DLIC_OK : DLIC_ERR_HIP;
}

// --- validation -------------------------------------------------------------
int max_group_rows(int h, int G) {
  int m = 0;
  for (int g = 0; g < G; ++g) {
    const int r = (int)(((long long)(g + 1) * h) / G - ((long long)g * h) / G);
    if (r > m) m = r;
  }
  return m;
}

// Row strips per group: 0 and 1 both mean one contiguous strip; -1 for an
// out-of-range value.
int coder_strips(const dlic_coder* c) {
  if (c->strips < 0 || c->strips > DLIC_MAX_STRIPS) return -1;
  return c->strips > 1 ? c->strips : 1;
}

// Layouts this library writes and reads: 1..64 lanes, at most 1024 groups of
// 1..16 row strips each, every strip at least 2 rows (one strip in all aside)
// and at most 256 rows.
bool coder_ok(int h, const dlic_coder* c) {
  if (!c) return false;
  const int G = c->groups, L = c->lanes_per_group, S = coder_strips(c);
  if (L < 1 || L > 64 || G < 1 || G > 1024 || S < 1) return false;
  if (G * S > 1 && h < 2 * G * S) return false;
  if (max_group_rows(h, G * S) > DEC_RMAX) return false;
  return true;
}

// The deep network's codecs, the volumes and the batches code one strip per group.
bool flat_coder_ok(int h, const dlic_coder* c) { return coder_ok(h, c) && coder_strips(c) == 1; }

dlic_status model_ok(const dlic_model* m) {
  if (!m) return DLIC_ERR_ARG;
  if (m->k_in != K_IN || m->n_out != N_OUT || m->reserved != 0) return DLIC_ERR_ARG;
  if (!m->d_w1 || !m->d_w2 || !m->d_w3 || !m->d_b1 || !m->d_b2 || !m->d_b3) return DLIC_ERR_ARG;
  if (m->dtype != DLIC_FP32 && m->dtype != DLIC_BF16 && m->dtype != DLIC_FP8_E4M3 &&
      m->dtype != DLIC_FP8_W8A8)
    return DLIC_ERR_UNSUPPORTED;
  if ((m->dtype == DLIC_FP8_E4M3 || m->dtype == DLIC_FP8_W8A8) && !m->d_wscale)
    return DLIC_ERR_ARG;
  if (m->h1 != m->h2 || (m->h1 != 32 && m->h1 != 64 && m->h1 != 128))
    return DLIC_ERR_UNSUPPORTED;
  return DLIC_OK;
}

int weight_type(const dlic_model* m) {
  switch (m->dtype) {
    case DLIC_BF16: return WT_BF16;
    case DLIC_FP8_E4M3: return WT_FP8;
    case DLIC_FP8_W8A8: return WT_FP8A8;
    default: return WT_F32;
  }
}

DevModel dev_model(const dlic_model* m) {
  DevModel d;
  d.w1 = m->d_w1;
  d.w2 = m->d_w2;
  d.w3 = m->d_w3;
  d.b1 = m->d_b1;
  d.b2 = m->d_b2;
  d.b3 = m->d_b3;
  d.wscale = (m->dtype == DLIC_FP8_E4M3 || m->dtype == DLIC_FP8_W8A8) ? m->d_wscale : nullptr;
  return d;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct EncWs {
  uint32_t* cf;
  uint16_t* words;
  uint32_t* counts;
};

size_t enc_ws_layout(int h, int w, int G, int L, void* base, EncWs* out) {
  const size_t n = (size_t)h * w;
  const size_t o_cf = 0;
  const size_t o_words = align256(o_cf + 4 * n);
  const size_t o_counts = align256(o_words + 2 * (n + 2 * (size_t)L * G));
  const size_t total = align256(o_counts + 4 * (size_t)G);
  if (out && base) {
    char* b = (char*)base;
    out->cf = (uint32_t*)(b + o_cf);
    out->words = (uint16_t*)(b + o_words);
    out->counts = (uint32_t*)(b + o_counts);
  }
  return total;
}

long long n_steps(int h, int w) { return (long long)w + 3LL * h - 3; }

int density_grid(long long n) {
  long long blocks = (n + 255) / 256;
  if (blocks > 768) blocks = 768;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

int pack_chunks(long long n, int G) {
  long long per_group = (n / (G > 0 ? G : 1)) / 4096 + 1;
  if (per_group > 64) per_group = 64;
  return (int)per_group;
}

dlic_status run_rans_and_pack(int h, int w, const dlic_coder* coder, const uint32_t* cf,
                              const EncWs& ws, const HeaderFields& hf, uint8_t* d_out,
                              uint64_t* d_out_len, hipStream_t s) {
  const int G = coder->groups, L = coder->lanes_per_group, S = coder_strips(coder);
  timing_begin("rans_encode_kernel", s);
  launch_rans_encode(cf, h, w, G, L, S, ws.words, ws.counts, s);
  timing_end(s);
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  timing_begin("pack_kernel", s);
  launch_pack(ws.words, ws.counts, h, w, G, L, S, hf, d_out, d_out_len,
              pack_chunks((long long)h * w, G), s);
  timing_end(s);
  return launch_ok();
}

// ---- the six-layer softmax-256 network -----------------------------------
// volume: the model may take the slice below (k_in 21) or not (12); an image: 12
dlic_status deep_model_ok(const dlic_deep_model* m, bool volume) {
  if (!m) return DLIC_ERR_ARG;
  if (m->hidden != 64 && m->hidden != 128) return DLIC_ERR_UNSUPPORTED;
  if (m->depth != 8 && m->depth != 12) return DLIC_ERR_UNSUPPORTED;
  if (m->k_in != K_IN && !(volume && m->k_in == K_IN_3D)) return DLIC_ERR_UNSUPPORTED;
  for (int i = 0; i < DLIC_DEEP_LAYERS; ++i)
    if (!m->d_w[i] || !m->d_b[i]) return DLIC_ERR_ARG;
  return DLIC_OK;
}

DeepNetArgs deep_net(const dlic_deep_model* m, void* wop) {
  DeepNetArgs n;
  n.H = m->hidden;
  n.k_in = m->k_in;
  n.nout = m->depth == 12 ? DEEP_OUT12 : DEEP_OUT;
  n.wop = wop;
  for (int i = 0; i < DLIC_DEEP_LAYERS; ++i) n.b[i] = m->d_b[i];
  return n;
}

// Operand-order weights at the head of every deep workspace.
dlic_status deep_stage(const dlic_deep_model* m, void* wop, hipStream_t s) {
  launch_deep_pack(m->hidden, m->k_in, m->depth == 12 ? DEEP_OUT12 : DEEP_OUT, m->d_w, wop, s);
  return launch_ok();
}

// Volume geometry: z slices, window shift ws; nullptr geometry for images.
bool vol_geom(const dlic_deep_model* m, int z, int ws, VolGeom* vg) {
  if (z < 1 || z > DLIC_VOLUME_MAX_SLICES || ws < 0 || ws > DLIC_VOLUME_MAX_SHIFT) return false;
  if (m->k_in == K_IN && ws != 0) return false;  // no window in the slice below
  vg->Z = z;
  vg->ws = ws;
  vg->lag = m->k_in == K_IN_3D ? (3 * ws - 1 > 0 ? 3 * ws - 1 : 0) : 0;
  return true;
}

HeaderFields deep_header(const dlic_deep_model* m, const VolGeom* vg) {
  // the dtype byte's high nibble holds the bit depth above 8
  HeaderFields hf{DLIC_BF16 | ((m->depth - 8) << 4), m->hidden, m->hidden, m->fingerprint};
  hf.n_mix = 0;
  hf.k_in = m->k_in;
  hf.flags = vg ? (vg->Z | (vg->ws << 12)) : 0;
  return hf;
}

// The stacked image's coder: G groups in each of z slices.
dlic_coder stacked_coder(const dlic_coder* c, int z) {
  dlic_coder t = *c;
  t.groups = c->groups * z;
  return t;
}

bool vol_coder_ok(int z, int h, const dlic_coder* c) {
  if (!flat_coder_ok(h, c)) return false;
  const dlic_coder t = stacked_coder(c, z);
  return coder_ok(z * h, &t);
}

// Upper bound on the tiles of one decode step: every slice's active rows.
int deep_step_tiles(int z, int h, int w) {
  const int rows = h < (w + SKEW - 1) / SKEW ? h : (w + SKEW - 1) / SKEW;
  const long long t = (long long)z * ((rows + 15) / 16);
  return t > (1 << 20) ? (1 << 20) : (int)t;
}

// Pixels per pass of the 12-bit encoder's three stages (logits: 256 MB).
constexpr long long DEEP12_CHUNK = 16384;

// Workspace of the deep entry points, in order: operand-order weights, then
//  density / encode: 12-bit: h5 of a chunk, logits of a chunk, an error flag;
//                    encode: the rANS encoder's scratch;
//  decode: tables [Z H][levels] u16; 12-bit: logits [Z H][4096], h5 and rows
//          of a step's tiles; 256 bytes of barrier state.
struct DeepWs {
  size_t wop = 0, h5 = 0, logits = 0, bad = 0, enc = 0, tables = 0, steps = 0, rows = 0, ctl = 0,
         total = 0;
};

DeepWs deep_ws(int z, int h, int w, const dlic_coder* coder, int hidden, int depth, int decode) {
  DeepWs o;
  const int nout = depth == 12 ? DEEP_OUT12 : DEEP_OUT;
  size_t at = align256(deep_wop_bytes(hidden, nout));
  if (decode <= 0) {
    if (depth == 12) {
      const long long n = (long long)z * h * w;
      const long long ch = n < DEEP12_CHUNK ? n : DEEP12_CHUNK;
      o.h5 = at;
      at += align256((size_t)((ch + 15) / 16) * deep12_tile_bytes(hidden));
      o.logits = at;
      at += align256((size_t)ch * DEEP_OUT12 * 4);
      o.bad = at;
      at += 256;
    }
    if (decode == 0) {
      o.enc = at;
      at += enc_ws_layout(z * h, w, coder->groups * z, coder->lanes_per_group, nullptr, nullptr);
    }
  } else {
    o.tables = at;
    at += align256((size_t)z * h * nout * 2);
    o.steps = at;  // per row: newest pixel step, newest table step
    at += align256((size_t)z * h * 2 * sizeof(int));
    if (depth == 12) {
      const size_t tiles = (size_t)deep_step_tiles(z, h, w);
      o.logits = at;
      at += align256((size_t)z * h * DEEP_OUT12 * 4);
      o.h5 = at;
      at += align256(tiles * deep12_tile_bytes(hidden));
      o.rows = at;
      at += align256(tiles * sizeof(int2));
    }
    o.ctl = at;
    at += 256;
  }
  o.total = at;
  return o;
}

size_t deep_ws_bytes(int z, int h, int w, const dlic_coder* coder, int hidden, int depth,
                     int decode) {
  return deep_ws(z, h, w, coder, hidden, depth, decode).total;
}

// The 12-bit encoder's stages over every pixel, chunk by chunk: packed
// intervals into cf and, for the density hook, logits and tables.
dlic_status deep12_stages(const Consts* K, const DeepNetArgs& net, const uint16_t* img, int h,
                          int w, const VolGeom& vg, const DeepWs& L, uint8_t* base,
                          uint32_t* d_cf, float* d_logits, uint16_t* d_tables,
                          hipStream_t stream) {
  const long long n = (long long)vg.Z * h * w;
  int* bad = (int*)(base + L.bad);
  launch_fill_u32((uint32_t*)bad, 0u, 1, stream);
  // one timed span over every chunk's three kernels (the per-kernel split is in
  // a kernel trace)
  timing_begin("deep12_density", stream);
  for (long long px0 = 0; px0 < n; px0 += DEEP12_CHUNK) {
    const long long nn = n - px0 < DEEP12_CHUNK ? n - px0 : DEEP12_CHUNK;
    float* lg = d_logits ? d_logits + px0 * DEEP_OUT12 : (float*)(base + L.logits);
    if (!launch_deep12_hidden(K, net, img, h, w, vg, px0, nn, base + L.h5, bad, stream))
      return DLIC_ERR_UNSUPPORTED;
    if (!launch_deep12_logits(net, base + L.h5, nn, lg, stream)) return DLIC_ERR_UNSUPPORTED;
    launch_deep12_softmax(lg, img, px0, nn, d_cf, d_tables ? d_tables + px0 * DEEP_OUT12 : nullptr,
                          stream);
  }
  timing_end(stream);
  return launch_ok();
}

dlic_status deep_density_impl(const dlic_deep_model* model, const void* d_img, int h, int w,
                              const VolGeom& vg, float* d_logits, uint32_t* d_cf,
                              uint16_t* d_tables, void* d_ws, size_t ws_bytes,
                              hipStream_t stream) {
  const DeepWs L = deep_ws(vg.Z, h, w, nullptr, model->hidden, model->depth, -1);
  if (ws_bytes < L.total) return DLIC_ERR_CAPACITY;
  const Consts* K = nullptr;
  dlic_status rc = current_consts(&K);
  if (rc != DLIC_OK) return rc;
  if ((rc = deep_stage(model, d_ws, stream)) != DLIC_OK) return rc;
  if (model->depth == 12)
    return deep12_stages(K, deep_net(model, d_ws), (const uint16_t*)d_img, h, w, vg, L,
                         (uint8_t*)d_ws, d_cf, d_logits, d_tables, stream);
  timing_begin("deep_density_kernel", stream);
  if (!launch_deep_density(K, deep_net(model, d_ws), (const uint8_t*)d_img, h, w, vg, d_cf,
                           d_logits, d_tables, stream))
    return DLIC_ERR_UNSUPPORTED;
  timing_end(stream);
  return launch_ok();
}

dlic_status deep_encode_impl(const dlic_deep_model* model, const dlic_coder* coder,
                             const void* d_img, int h, int w, const VolGeom& vg,
                             const HeaderFields& hf, uint8_t* d_out, size_t out_cap,
                             uint64_t* d_out_len, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  const dlic_coder tc = stacked_coder(coder, vg.Z);
  const int HT = vg.Z * h;
  if (out_cap < dlic_encode_bound(HT, w, &tc)) return DLIC_ERR_CAPACITY;
  const DeepWs L = deep_ws(vg.Z, h, w, coder, model->hidden, model->depth, 0);
  if (ws_bytes < L.total) return DLIC_ERR_CAPACITY;
  const Consts* K = nullptr;
  dlic_status rc = current_consts(&K);
  if (rc != DLIC_OK) return rc;
  uint8_t* base = (uint8_t*)d_ws;
  EncWs ws;
  enc_ws_layout(HT, w, tc.groups, tc.lanes_per_group, base + L.enc, &ws);
  if ((rc = deep_stage(model, d_ws, stream)) != DLIC_OK) return rc;
  if (model->depth == 12) {
    if ((rc = deep12_stages(K, deep_net(model, d_ws), (const uint16_t*)d_img, h, w, vg, L, base,
                            ws.cf, nullptr, nullptr, stream)) != DLIC_OK)
      return rc;
  } else {
    timing_begin("deep_density_kernel", stream);
    if (!launch_deep_density(K, deep_net(model, d_ws), (const uint8_t*)d_img, h, w, vg, ws.cf,
                             nullptr, nullptr, stream))
      return DLIC_ERR_UNSUPPORTED;
    timing_end(stream);
  }
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  rc = run_rans_and_pack(HT, w, &tc, ws.cf, ws, hf, d_out, d_out_len, stream);
  if (rc == DLIC_OK && model->depth == 12) {
    launch_deep12_reject((const int*)(base + L.bad), d_out_len, stream);
    rc = launch_ok();
  }
  return rc;
}

dlic_status deep_decode_impl(const dlic_deep_model* model, const dlic_coder* coder,
                             const uint8_t* d_bits, size_t n_bytes, void* d_img, int h, int w,
                             const VolGeom& vg, const HeaderFields& hf, int32_t* d_status,
                             void* d_ws, size_t ws_bytes, hipStream_t stream) {
  const DeepWs L = deep_ws(vg.Z, h, w, coder, model->hidden, model->depth, 1);
  if (ws_bytes < L.total) return DLIC_ERR_CAPACITY;
  const Consts* K = nullptr;
  dlic_status rc = current_consts(&K);
  if (rc != DLIC_OK) return rc;
  // one wave per group, all workgroups resident (cooperative launch); as many
  // workgroups as a step has tiles, at least 64, at most 256 and the residency
  const int GT = coder->groups * vg.Z;
  const bool d12 = model->depth == 12;
  const int resident = d12 ? deep12_decode_max_grid(model->hidden, model->k_in)
                           : deep_decode_max_grid(model->hidden, model->k_in);
  if (resident <= 0) return DLIC_ERR_HIP;
  int grid = deep_step_tiles(vg.Z, h, w);
  if (grid > 256) grid = 256;
  if (grid < 64) grid = 64;
  if (g_deep_grid > 0) grid = g_deep_grid;
  if (grid < (GT + DEEP_WAVES - 1) / DEEP_WAVES) grid = (GT + DEEP_WAVES - 1) / DEEP_WAVES;
  if (grid > resident) grid = resident;
  if (GT > grid * DEEP_WAVES) return DLIC_ERR_UNSUPPORTED;
  uint8_t* base = (uint8_t*)d_ws;
  DeepDecArgs a;
  memset(&a, 0, sizeof(a));
  a.net = deep_net(model, d_ws);
  a.K = K;
  a.bits = d_bits;
  a.n_bytes = n_bytes;
  a.img = d_img;
  a.H = h;
  a.W = w;
  a.G = coder->groups;
  a.L = coder->lanes_per_group;
  a.vg = vg;
  a.T = n_steps(h, w) + (long long)vg.lag * (vg.Z - 1);
  a.tables = (uint16_t*)(base + L.tables);
  if (d12) {
    a.logits = (float*)(base + L.logits);
    a.h5 = base + L.h5;
    a.tile_rows = (int2*)(base + L.rows);
  }
  uint32_t* ctl = (uint32_t*)(base + L.ctl);
  a.pix_step = (int*)(base + L.steps);
  a.delay_seed = g_delay_seed;
  a.delay_max = g_delay_max;
  a.tab_step = a.pix_step + (size_t)vg.Z * h;
  a.bar = ctl;
  a.abort_flag = (int*)(ctl + 16);
  a.status = d_status;
  a.spin_limit = g_spin_limit;
  a.hf = hf;
  if ((rc = deep_stage(model, d_ws, stream)) != DLIC_OK) return rc;
  launch_fill_u32(ctl, 0u, 64, stream);
  launch_fill_u32((uint32_t*)a.pix_step, 0xFFFFFFFFu, 2LL * vg.Z * h, stream);
  launch_fill_u32((uint32_t*)d_status, 0u, 1, stream);
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  g_deep_grid_used = grid;
  timing_begin(d12 ? "deep12_decode_kernel" : "deep_decode_kernel", stream);
  if ((d12 ? launch_deep12_decode(a, grid, stream) : launch_deep_decode(a, grid, stream)) !=
      hipSuccess)
    return DLIC_ERR_HIP;
  timing_end(stream);
  return launch_ok();
}

}  // namespace

// A batch plan: per-image layout, the work items in longest-wavefront-first
// order, their device copies, and up to one captured graph per direction.
struct dlic_batch {
  int device = 0;
  dlic_model model{};
  int n_img = 0, n_blk = 0, density_grid = 0, pack_parts = 1;
  int widest = 1;       // largest lanes per group of any image
  int search_lpp = 0;   // coder lanes per pixel in decode; 0: coder_lpp(widest)
  int decode_grid = 0;  // cap on the persistent decode grid; 0: resident capacity
  std::vector<BatchImage> images;
  std::vector<BatchItem> items;
  BatchImage* d_images = nullptr;
  BatchItem* d_items = nullptr;
  size_t pixels = 0, out_bytes = 0;
  long long n_words = 0, n_rec = 0;
  int n_counts = 0;
  size_t off_words = 0, off_counts = 0, off_rec = 0, off_ctrl = 0, ws_bytes = 0;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

// Device-side arguments of a batch call on the plan's workspace.
BatchArgs batch_args(const dlic_batch* b, void* d_ws) {
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  uint8_t* ws = (uint8_t*)d_ws;
  a.images = b->d_images;
  a.items = b->d_items;
  a.n_img = b->n_img;
  a.n_items = (int)b->items.size();
  a.n_blk = b->n_blk;
  a.cf = (uint32_t*)ws;
  a.words = (uint16_t*)(ws + b->off_words);
  a.counts = (uint32_t*)(ws + b->off_counts);
  a.rec = (uint32_t*)(ws + b->off_rec);
  a.ticket = (unsigned*)(ws + b->off_ctrl);
  a.done = a.ticket + 1;
  a.hf = HeaderFields{b->model.dtype, b->model.h1, b->model.h2, b->model.fingerprint};
  a.spin_limit = g_spin_limit;
  a.delay_seed = g_delay_seed;
  a.delay_max = g_delay_max;
  return a;
}

dlic_status batch_enqueue(dlic_batch* b, bool decode, const uint8_t* in, uint8_t* out,
                          uint64_t* len, int32_t* status, uint64_t* t_done, void* ws,
                          hipStream_t s) {
  const Consts* K = nullptr;
  dlic_status rc = current_consts(&K);
  if (rc != DLIC_OK) return rc;
  BatchArgs a = batch_args(b, ws);
  a.len = len;
  a.t_done = (unsigned long long*)t_done;
  const DevModel dm = dev_model(&b->model);
  const int wtype = weight_type(&b->model);
  // control words: ticket, then one completion counter per image
  launch_fill_u32(a.ticket, 0u, 1 + b->n_img, s);
  if (t_done) launch_stamp(a.t_done + b->n_img, s);
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  if (!decode) {
    a.pix_in = in;
    a.out = out;
    timing_begin("batch_density_kernel", s);
    if (!launch_batch_density(wtype, b->model.h1, K, dm, a, b->density_grid, s))
      return DLIC_ERR_UNSUPPORTED;
    timing_end(s);
    timing_begin("batch_rans_encode_kernel", s);
    launch_batch_rans_encode(a, s);
    timing_end(s);
    timing_begin("batch_pack_kernel", s);
    launch_batch_pack(a, b->pack_parts, s);
    timing_end(s);
  } else {
    a.bits = in;
    a.pix_out = out;
    a.status = status;
    launch_fill_u32(a.rec, 0u, b->n_rec, s);
    launch_fill_u32((uint32_t*)status, 0u, b->n_img, s);
    if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
    timing_begin("batch_decode_kernel", s);
    const int lpp = b->search_lpp > 0 ? b->search_lpp : coder_lpp(b->widest);
    if (!launch_batch_decode(wtype, b->model.h1, K, dm, a, lpp, b->decode_grid, s))
      return DLIC_ERR_UNSUPPORTED;
    timing_end(s);
  }
  return launch_ok();
}

dlic_status batch_call_ok(const dlic_batch* b, const void* in, const void* out, const void* len,
                          const void* ws, size_t ws_bytes) {
  if (!b || !in || !out || !len || !ws) return DLIC_ERR_ARG;
  if (ws_bytes < b->ws_bytes) return DLIC_ERR_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DLIC_ERR_HIP;
  if (dev != b->device) return DLIC_ERR_ARG;
  return DLIC_OK;
}

}  // namespace

extern "C" {

const char* dlic_status_string(dlic_status s) {
  switch (s) {
    case DLIC_OK: return "ok";
    case DLIC_ERR_ARG: return "invalid argument";
    case DLIC_ERR_CAPACITY: return "buffer too small";
    case DLIC_ERR_CORRUPT: return "corrupt stream";
    case DLIC_ERR_MODEL_MISMATCH: return "stream coded with another model";
    case DLIC_ERR_UNSUPPORTED: return "unsupported parameters";
    case DLIC_ERR_HIP: return "HIP error or no usable device";
    case DLIC_ERR_TIMEOUT: return "decode wait timed out";
  }
  return "unknown status";
}

uint64_t dlic_fnv1a64(uint64_t h, const void* h_bytes, size_t n) {
  const uint8_t* p = (const uint8_t*)h_bytes;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

void dlic_host_constants(float* h_S, float* h_D, float* h_beta, float* h_scale) {
  Consts* c = new Consts;
  build_consts(c);
  for (int j = 0; j < LUT_N; ++j) {
    if (h_S) h_S[j] = c->sd[j].x;
    if (h_D) h_D[j] = c->sd[j].y;
  }
  if (h_beta) memcpy(h_beta, c->beta, sizeof(c->beta));
  if (h_scale) memcpy(h_scale, c->scale, sizeof(c->scale));
  delete c;
}

dlic_status dlic_host_scale(int32_t depth, float* h_out) {
  if (!h_out || (depth != 8 && depth != 12)) return DLIC_ERR_ARG;
  Consts* c = new Consts;
  build_consts(c);
  if (depth == 8)
    memcpy(h_out, c->scale, sizeof(c->scale));
  else
    memcpy(h_out, c->scale12, sizeof(c->scale12));
  delete c;
  return DLIC_OK;
}

dlic_status dlic_quantize_weights(int32_t dtype, const float* h_w, size_t n, void* h_out,
                                  float* h_scale) {
  if (!h_w || !h_out || n == 0) return DLIC_ERR_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(h_w[i])) return DLIC_ERR_ARG;
  if (dtype == DLIC_BF16) {
    uint16_t* out = (uint16_t*)h_out;
    for (size_t i = 0; i < n; ++i) {
      uint32_t u;
      memcpy(&u, &h_w[i], 4);
      u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
      out[i] = (uint16_t)(u >> 16);
    }
    if (h_scale) *h_scale = 1.0f;
    return DLIC_OK;
  }
  if (dtype != DLIC_FP8_E4M3 || !h_scale) return DLIC_ERR_ARG;
  float amax = 0.0f;
  for (size_t i = 0; i < n; ++i) amax = fmaxf(amax, fabsf(h_w[i]));
  const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
  uint8_t* out = (uint8_t*)h_out;
  for (size_t i = 0; i < n; ++i) {
    const float x = h_w[i] / scale;
    const double a = fabs((double)x);
    uint32_t code;
    if (a >= 448.0) {
      code = 0x7Eu;  // saturate at the largest finite e4m3 value
    } else if (a < 0.015625) {
      code = (uint32_t)nearbyint(a * 512.0);  // subnormal step 2^-9; 8 is 2^-6 itself
    } else {
      int e = (int)floor(log2(a));
      if (ldexp(1.0, e) > a) --e;
      if (ldexp(1.0, e + 1) <= a) ++e;
      uint32_t m = (uint32_t)nearbyint(ldexp(a, 3 - e)) - 8u;
      if (m == 8u) {
        m = 0;
        ++e;
      }
      code = ((uint32_t)(e + 7) << 3) | m;
      if (code > 0x7Eu) code = 0x7Eu;
    }
    out[i] = (uint8_t)(code | (signbit(x) && code != 0 ? 0x80u : 0u));
  }
  *h_scale = scale;
  return DLIC_OK;
}

dlic_status dlic_w8a8_multipliers(const float* h_amax, float* h_mult) {
  if (!h_amax || !h_mult) return DLIC_ERR_ARG;
  for (int l = 0; l < 3; ++l) {
    const float a = h_amax[l];
    if (!(a > 0.0f) || !isfinite(a)) {
      h_mult[l] = 1.0f;
      continue;
    }
    int k = (int)floor(log2(448.0 / (double)a));
    // floor(log2) of a quotient can land one off at exact powers of two
    while (ldexp((double)a, k) > 448.0) --k;
    while (ldexp((double)a, k + 1) <= 448.0) ++k;
    if (k > 100) k = 100;
    if (k < -100) k = -100;
    h_mult[l] = (float)ldexp(1.0, k);
  }
  return DLIC_OK;
}

size_t dlic_encode_bound(int32_t h, int32_t w, const dlic_coder* coder) {
  if (h <= 0 || w <= 0 || !coder_ok(h, coder)) return 0;
  const size_t G = coder->groups, L = coder->lanes_per_group;
  return HEADER_BYTES + 4 * G + 2 * ((size_t)h * w + 2 * L * G);
}

size_t dlic_encode_workspace(int32_t h, int32_t w, const dlic_coder* coder) {
  if (h <= 0 || w <= 0 || !coder_ok(h, coder)) return 0;
  return enc_ws_layout(h, w, coder->groups, coder->lanes_per_group, nullptr, nullptr);
}

size_t dlic_decode_workspace(int32_t h, int32_t w, const dlic_coder* coder) {
  if (h <= 0 || w <= 0 || !coder_ok(h, coder)) return 0;
  // records [S*G][T] (one row per strip), then the group ticket
  const size_t strips = (size_t)coder->groups * (size_t)coder_strips(coder);
  return align256(4 * (strips * (size_t)n_steps(h, w) + 1));
}

dlic_status dlic_peek_header(const uint8_t* b, size_t n, int32_t* h, int32_t* w,
                             dlic_coder* coder, uint64_t* fingerprint, int32_t* h1, int32_t* h2,
                             int32_t* dtype) {
  if (!b || n < (size_t)HEADER_BYTES) return DLIC_ERR_CORRUPT;
  if (memcmp(b, "DLIC", 4) != 0) return DLIC_ERR_CORRUPT;
  auto u16 = [&](int o) { return (uint32_t)b[o] | ((uint32_t)b[o + 1] << 8); };
  auto u32 = [&](int o) { return u16(o) | (u16(o + 2) << 16); };
  if (u16(4) != 1u) return DLIC_ERR_CORRUPT;
  const int G = (int)u16(26), L = b[25];
  if (h) *h = (int32_t)u32(8);
  if (w) *w = (int32_t)u32(12);
  if (dtype) *dtype = b[18];
  if (h1) *h1 = (int32_t)u16(20);
  if (h2) *h2 = (int32_t)u16(22);
  if (coder) {
    coder->groups = G;
    coder->lanes_per_group = L;
    // an image's flags hold its strips per group - 1 in bits 12..15
    const uint32_t flags = u16(6);
    coder->strips = (flags & 0xFFFu) == 0 ? (int32_t)(flags >> 12) + 1 : 1;
  }
  if (fingerprint) *fingerprint = (uint64_t)u32(28) | ((uint64_t)u32(32) << 32);
  return DLIC_OK;
}

dlic_status dlic_init(int device) { return ensure_device(device, nullptr); }

dlic_status dlic_encode(const dlic_model* model, const dlic_coder* coder, const uint8_t* d_img,
                        int32_t h, int32_t w, uint8_t* d_out, size_t out_cap,
                        uint64_t* d_out_len, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  if (!d_img || !d_out || !d_out_len || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  dlic_status rc = model_ok(model);
  if (rc != DLIC_OK) return rc;
  if (out_cap < dlic_encode_bound(h, w, coder)) return DLIC_ERR_CAPACITY;
  if (ws_bytes < dlic_encode_workspace(h, w, coder)) return DLIC_ERR_CAPACITY;
  const Consts* K = nullptr;
  if ((rc = current_consts(&K)) != DLIC_OK) return rc;
  EncWs ws;
  enc_ws_layout(h, w, coder->groups, coder->lanes_per_group, d_ws, &ws);
  const long long n = (long long)h * w;
  timing_begin("density_kernel", stream);
  launch_density(weight_type(model), model->h1, K, dev_model(model), d_img, h, w, ws.cf, nullptr, nullptr,
                 density_grid(n), stream);
  timing_end(stream);
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  HeaderFields hf{model->dtype, model->h1, model->h2, model->fingerprint};
  hf.flags = (coder_strips(coder) - 1) << 12;
  return run_rans_and_pack(h, w, coder, ws.cf, ws, hf, d_out, d_out_len, stream);
}

dlic_status dlic_activation_range(const dlic_model* model, const uint8_t* d_img, int32_t h,
                                  int32_t w, float* d_amax, hipStream_t stream) {
  timing_reset();
  if (!d_img || !d_amax || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  dlic_status rc = model_ok(model);
  if (rc != DLIC_OK) return rc;
  if (model->dtype != DLIC_FP32) return DLIC_ERR_ARG;
  const Consts* K = nullptr;
  if ((rc = current_consts(&K)) != DLIC_OK) return rc;
  timing_begin("activation_range_kernel", stream);
  if (!launch_activation_range(model->h1, K, dev_model(model), d_img, h, w, d_amax,
                               density_grid((long long)h * w), stream))
    return DLIC_ERR_UNSUPPORTED;
  timing_end(stream);
  return launch_ok();
}

dlic_status dlic_rans_encode_cf(const dlic_coder* coder, int32_t h, int32_t w,
                                const uint32_t* d_cf, uint8_t* d_out, size_t out_cap,
                                uint64_t* d_out_len, void* d_ws, size_t ws_bytes,
                                hipStream_t stream) {
  timing_reset();
  if (!d_cf || !d_out || !d_out_len || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  if (out_cap < dlic_encode_bound(h, w, coder)) return DLIC_ERR_CAPACITY;
  if (ws_bytes < dlic_encode_workspace(h, w, coder)) return DLIC_ERR_CAPACITY;
  dlic_status rc = current_consts(nullptr);
  if (rc != DLIC_OK) return rc;
  EncWs ws;
  enc_ws_layout(h, w, coder->groups, coder->lanes_per_group, d_ws, &ws);
  HeaderFields hf{0, 0, 0, 0ull};
  hf.flags = (coder_strips(coder) - 1) << 12;
  return run_rans_and_pack(h, w, coder, d_cf, ws, hf, d_out, d_out_len, stream);
}

static dlic_status decode_common(const dlic_model* model, bool tables_mode,
                                 const dlic_coder* coder, const uint32_t* d_tables,
                                 int32_t n_tables, const uint32_t* d_tidx, const uint8_t* d_bits,
                                 size_t n_bytes, uint8_t* d_img, int32_t h, int32_t w,
                                 int32_t* d_status, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
  timing_reset();
  if (!d_bits || !d_img || !d_status || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  // sub-round counters are 32-bit: (W + 3R) * ceil(R / L) < 2^31
  if (((long long)w + 3LL * DEC_RMAX) * DEC_RMAX >= (1LL << 31)) return DLIC_ERR_UNSUPPORTED;
  if (ws_bytes < dlic_decode_workspace(h, w, coder)) return DLIC_ERR_CAPACITY;
  dlic_status rc;
  const Consts* K = nullptr;
  if ((rc = current_consts(&K)) != DLIC_OK) return rc;
  DecArgs a;
  memset(&a, 0, sizeof(a));
  a.bits = d_bits;
  a.n_bytes = n_bytes;
  a.img = d_img;
  a.H = h;
  a.W = w;
  a.G = coder->groups;
  a.L = coder->lanes_per_group;
  a.S = coder_strips(coder);
  a.rec = (uint32_t*)d_ws;
  a.T = n_steps(h, w);
  a.ticket = (unsigned*)(a.rec + (long long)a.G * a.S * a.T);
  a.status = d_status;
  a.spin_limit = g_spin_limit;
  a.delay_seed = g_delay_seed;
  a.delay_max = g_delay_max;
  a.prof = tables_mode ? nullptr : g_prof;
  DevModel dm;
  memset(&dm, 0, sizeof(dm));
  int width = 32, wtype = WT_F32;
  if (tables_mode) {
    if (!d_tables || !d_tidx || n_tables < 1) return DLIC_ERR_ARG;
    a.tables = d_tables;
    a.n_tables = n_tables;
    a.tidx = d_tidx;
  } else {
    if ((rc = model_ok(model)) != DLIC_OK) return rc;
    a.check_model = 1;
    a.hf = HeaderFields{model->dtype, model->h1, model->h2, model->fingerprint};
    dm = dev_model(model);
    width = model->h1;
    wtype = weight_type(model);
  }
  timing_begin("fill_u32_kernel", stream);
  launch_fill_u32(a.rec, 0u, (long long)a.G * a.S * a.T + 1, stream);
  launch_fill_u32((uint32_t*)d_status, 0u, 1, stream);
  timing_end(stream);
  if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
  timing_begin(tables_mode ? "wavefront_decode_kernel<tables>" : "wavefront_decode_kernel",
               stream);
  if (!launch_decode(wtype, width, tables_mode, K, dm, a, stream)) return DLIC_ERR_UNSUPPORTED;
  timing_end(stream);
  return launch_ok();
}

dlic_status dlic_decode(const dlic_model* model, const dlic_coder* coder,
                        const uint8_t* d_bits, size_t n_bytes, uint8_t* d_img, int32_t h,
                        int32_t w, int32_t* d_status, void* d_ws, size_t ws_bytes,
                        hipStream_t stream) {
  return decode_common(model, false, coder, nullptr, 0, nullptr, d_bits, n_bytes, d_img, h, w,
                       d_status, d_ws, ws_bytes, stream);
}

dlic_status dlic_decode_noalloc(const dlic_model* model, const dlic_coder* coder,
                                const uint8_t* d_bits, size_t n_bytes, uint8_t* d_img, int32_t h,
                                int32_t w, int32_t* d_status, hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return DLIC_ERR_HIP;
  void* sp = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_dev[dev].ready) sp = g_dev[dev].scratch;
  }
  // set-up (constant tables, workspace address) allocates: dlic_init first
  if (sp == nullptr) return DLIC_ERR_ARG;
  if (!d_bits || !d_img || !d_status || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  if (dlic_decode_workspace(h, w, coder) > NOALLOC_SCRATCH_BYTES) return DLIC_ERR_CAPACITY;
  // no timing events either: creating one may allocate
  const NoTiming quiet;
  return decode_common(model, false, coder, nullptr, 0, nullptr, d_bits, n_bytes, d_img, h, w,
                       d_status, sp, NOALLOC_SCRATCH_BYTES, stream);
}

dlic_status dlic_rans_decode_tables(const dlic_coder* coder, int32_t h, int32_t w,
                                    const uint32_t* d_tables, int32_t n_tables,
                                    const uint32_t* d_tidx, const uint8_t* d_bits,
                                    size_t n_bytes, uint8_t* d_sym, int32_t* d_status,
                                    void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return decode_common(nullptr, true, coder, d_tables, n_tables, d_tidx, d_bits, n_bytes, d_sym,
                       h, w, d_status, d_ws, ws_bytes, stream);
}

dlic_status dlic_density(const dlic_model* model, const uint8_t* d_img, int32_t h, int32_t w,
                         float* d_out15, uint32_t* d_cf, uint32_t* d_tables, hipStream_t stream) {
  timing_reset();
  if (!d_img || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  dlic_status rc = model_ok(model);
  if (rc != DLIC_OK) return rc;
  const Consts* K = nullptr;
  if ((rc = current_consts(&K)) != DLIC_OK) return rc;
  timing_begin("density_kernel", stream);
  launch_density(weight_type(model), model->h1, K, dev_model(model), d_img, h, w, d_cf, d_out15, d_tables,
                 density_grid((long long)h * w), stream);
  timing_end(stream);
  return launch_ok();
}

dlic_status dlic_net_forms(const dlic_model* model, const float* d_feats, int64_t n,
                           int32_t lanes, float* d_out16, float* d_out4, hipStream_t stream) {
  timing_reset();
  if (!d_feats || !d_out16 || !d_out4 || n <= 0 || n % 16 != 0 || lanes < 1 || lanes > 4)
    return DLIC_ERR_ARG;
  dlic_status rc = model_ok(model);
  if (rc != DLIC_OK) return rc;
  if (model->dtype != DLIC_FP32 || (model->h1 != 64 && model->h1 != 128))
    return DLIC_ERR_UNSUPPORTED;
  if ((rc = current_consts(nullptr)) != DLIC_OK) return rc;
  timing_begin("net_forms_kernel", stream);
  launch_net_forms(model->h1, dev_model(model), d_feats, n, lanes, d_out16, d_out4, stream);
  timing_end(stream);
  return launch_ok();
}

size_t dlic_nll_workspace(int64_t n, const dlic_model* model) {
  if (!model || n <= 0) return 0;
  const bool f64 = model->dtype == DLIC_FP64;
  const size_t rows = (size_t)TRAIN_GRID * (f64 ? TRAIN_WAVES_F64 : TRAIN_WAVES_F32);
  // per-wave partial rows, then one sum row per block of 32 rows
  const size_t sums = rows + (rows + 31) / 32;
  return align256(sums * (size_t)(train_n_params(model->h1, model->h2) + 1) *
                  (f64 ? sizeof(double) : sizeof(float)));
}

dlic_status dlic_nll_fwd_bwd(const dlic_model* m, const uint8_t* d_slices, int32_t n_slices,
                             int32_t sh, int32_t sw, const int32_t* d_idx, int64_t n, void* d_loss,
                             void* d_grad, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  if (!m || !d_slices || !d_idx || !d_loss || !d_ws || n <= 0 || n_slices <= 0 || sh <= 0 ||
      sw <= 0)
    return DLIC_ERR_ARG;
  if (m->k_in != K_IN || m->n_out != N_OUT || !m->d_w1 || !m->d_w2 || !m->d_w3 || !m->d_b1 ||
      !m->d_b2 || !m->d_b3)
    return DLIC_ERR_ARG;
  if (m->dtype != DLIC_FP32 && m->dtype != DLIC_FP64) return DLIC_ERR_UNSUPPORTED;
  if (m->h1 != m->h2 || (m->h1 != 32 && m->h1 != 64)) return DLIC_ERR_UNSUPPORTED;
  if (ws_bytes < dlic_nll_workspace(n, m)) return DLIC_ERR_CAPACITY;
  dlic_status rc = current_consts(nullptr);
  if (rc != DLIC_OK) return rc;
  timing_begin("nll_fwd_bwd_kernel", stream);
  const bool ok = launch_nll(m->dtype == DLIC_FP64, m->h1, m->d_w1, m->d_b1, m->d_w2, m->d_b2,
                             m->d_w3, m->d_b3, d_slices, n_slices, sh, sw, d_idx, n, d_ws,
                             TRAIN_GRID, d_grad != nullptr, d_grad, d_loss, stream);
  timing_end(stream);
  if (!ok) return DLIC_ERR_UNSUPPORTED;
  return launch_ok();
}

dlic_status dlic_adam_step(int64_t n_params, float* d_params, const float* d_grad, float* d_m,
                           float* d_v, int32_t step, float lr, float b1, float b2, float eps,
                           hipStream_t stream) {
  if (n_params <= 0 || !d_params || !d_grad || !d_m || !d_v || step < 1) return DLIC_ERR_ARG;
  dlic_status rc = current_consts(nullptr);
  if (rc != DLIC_OK) return rc;
  timing_begin("adam_kernel", stream);
  launch_adam(n_params, d_params, d_grad, d_m, d_v, step, lr, b1, b2, eps, stream);
  timing_end(stream);
  return launch_ok();
}

void dlic_set_spin_limit(uint32_t polls) { g_spin_limit = polls ? polls : 1u; }

void dlic_set_decode_delays(uint32_t seed, uint32_t max_cycles) {
  g_delay_seed = seed;
  g_delay_max = max_cycles > (1u << 20) ? (1u << 20) : max_cycles;
}

void dlic_set_decode_profile(unsigned long long* d_counters) { g_prof = d_counters; }

void dlic_set_timing(int enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing = enable != 0;
}

int dlic_kernel_times(float* h_ms, const char** h_names, int max_n) {
  std::lock_guard<std::mutex> lk(g_mu);
  int n = g_n_timed < max_n ? g_n_timed : max_n;
  for (int i = 0; i < n; ++i) {
    float ms = -1.0f;
    if (hipEventSynchronize(g_events[i].stop) == hipSuccess)
      (void)hipEventElapsedTime(&ms, g_events[i].start, g_events[i].stop);
    if (h_ms) h_ms[i] = ms;
    if (h_names) h_names[i] = g_events[i].name;
  }
  return n;
}

// ---- batches -----------------------------------------------------------------

dlic_status dlic_batch_create(const dlic_model* model, int32_t n_img, const int32_t* h_hw,
                              const dlic_coder* h_coders, int32_t density_grid,
                              dlic_batch** out) {
  if (!out || !h_hw || n_img < 1 || n_img > (1 << 20) || density_grid < 0) return DLIC_ERR_ARG;
  *out = nullptr;
  dlic_status rc = model_ok(model);
  if (rc != DLIC_OK) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DLIC_ERR_HIP;
  if ((rc = ensure_device(dev, nullptr)) != DLIC_OK) return rc;
  dlic_batch* b = new dlic_batch;
  b->device = dev;
  b->model = *model;
  b->n_img = n_img;
  b->images.resize(n_img);
  long long px = 0, words = 0, rec = 0, outb = 0, blk = 0, maxper = 1;
  int counts = 0;
  for (int i = 0; i < n_img; ++i) {
    const int h = h_hw[2 * i], w = h_hw[2 * i + 1];
    dlic_coder c;
    if (h_coders) {
      c = h_coders[i];
    } else {
      c.groups = h > 192 ? (h + 191) / 192 : 1;
      c.lanes_per_group = 32;
      c.strips = 1;
    }
    if (h <= 0 || w <= 0 || !flat_coder_ok(h, &c) ||
        ((long long)w + 3LL * DEC_RMAX) * DEC_RMAX >= (1LL << 31)) {
      delete b;
      return h <= 0 || w <= 0 ? DLIC_ERR_ARG : DLIC_ERR_UNSUPPORTED;
    }
    BatchImage& im = b->images[i];
    const long long n = (long long)h * w;
    im.H = h;
    im.W = w;
    im.G = c.groups;
    im.L = c.lanes_per_group;
    im.T = n_steps(h, w);
    im.px_off = px;
    im.words_off = words;
    im.out_off = outb;
    im.out_cap = (long long)dlic_encode_bound(h, w, &c);
    im.rec_off = rec;
    im.counts_off = counts;
    im.blk_off = (int)blk;
    px += n;
    words += n + 2LL * im.L * im.G;
    outb += (im.out_cap + 255) & ~255LL;
    rec += (long long)im.G * im.T;
    counts += im.G;
    blk += (n + 255) / 256;
    if (n / im.G > maxper) maxper = n / im.G;
  }
  if (blk >= (1LL << 31) || counts > (1 << 24)) {
    delete b;
    return DLIC_ERR_UNSUPPORTED;
  }
  // longest wavefront first; an image's groups in order (the decode waits
  // only ever point to an earlier item)
  std::vector<int> order(n_img);
  for (int i = 0; i < n_img; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return b->images[x].T > b->images[y].T;
  });
  for (int i : order)
    for (int g = 0; g < b->images[i].G; ++g) b->items.push_back(BatchItem{i, g});
  for (const BatchImage& im : b->images) b->widest = std::max(b->widest, im.L);
  b->n_blk = (int)blk;
  b->density_grid = density_grid > 0 ? density_grid : (int)std::min<long long>(blk, 1024);
  b->pack_parts = (int)std::min<long long>(64, maxper / 4096 + 1);
  b->pixels = (size_t)px;
  b->out_bytes = (size_t)outb;
  b->n_words = words;
  b->n_rec = rec;
  b->n_counts = counts;
  b->off_words = align256(4 * (size_t)px);
  b->off_counts = align256(b->off_words + 2 * (size_t)words);
  b->off_rec = align256(b->off_counts + 4 * (size_t)counts);
  b->off_ctrl = align256(b->off_rec + 4 * (size_t)rec);
  b->ws_bytes = align256(b->off_ctrl + 4 * (size_t)(1 + n_img));
  if (hipMalloc((void**)&b->d_images, sizeof(BatchImage) * n_img) != hipSuccess ||
      hipMalloc((void**)&b->d_items, sizeof(BatchItem) * b->items.size()) != hipSuccess ||
      hipMemcpy(b->d_images, b->images.data(), sizeof(BatchImage) * n_img,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_items, b->items.data(), sizeof(BatchItem) * b->items.size(),
                hipMemcpyHostToDevice) != hipSuccess) {
    dlic_batch_destroy(b);
    return DLIC_ERR_HIP;
  }
  *out = b;
  return DLIC_OK;
}

dlic_status dlic_batch_tune(dlic_batch* b, int32_t search_lanes, int32_t decode_grid) {
  if (!b || decode_grid < 0) return DLIC_ERR_ARG;
  // 16 lanes per pixel serve at most 4 pixels per sub-round; the split
  // binary search at most 32
  if (search_lanes != 0 && search_lanes != 1 && search_lanes != 2 && search_lanes != 16)
    return DLIC_ERR_ARG;
  if ((search_lanes == 16 && b->widest > 4) || (search_lanes == 2 && b->widest > 32))
    return DLIC_ERR_UNSUPPORTED;
  b->search_lpp = search_lanes;
  b->decode_grid = decode_grid;
  return DLIC_OK;
}

void dlic_batch_destroy(dlic_batch* b) {
  if (!b) return;
  for (int d = 0; d < 2; ++d)
    if (b->exec[d]) (void)hipGraphExecDestroy(b->exec[d]);
  if (b->d_images) (void)hipFree(b->d_images);
  if (b->d_items) (void)hipFree(b->d_items);
  delete b;
}

dlic_status dlic_batch_sizes(const dlic_batch* b, size_t* pixels, size_t* out_bytes,
                             size_t* ws_bytes, int32_t* n_items) {
  if (!b) return DLIC_ERR_ARG;
  if (pixels) *pixels = b->pixels;
  if (out_bytes) *out_bytes = b->out_bytes;
  if (ws_bytes) *ws_bytes = b->ws_bytes;
  if (n_items) *n_items = (int32_t)b->items.size();
  return DLIC_OK;
}

dlic_status dlic_batch_layout(const dlic_batch* b, uint64_t* h_px_off, uint64_t* h_out_off,
                              int32_t* h_coders) {
  if (!b) return DLIC_ERR_ARG;
  for (int i = 0; i < b->n_img; ++i) {
    if (h_px_off) h_px_off[i] = (uint64_t)b->images[i].px_off;
    if (h_out_off) h_out_off[i] = (uint64_t)b->images[i].out_off;
    if (h_coders) {
      h_coders[2 * i] = b->images[i].G;
      h_coders[2 * i + 1] = b->images[i].L;
    }
  }
  return DLIC_OK;
}

dlic_status dlic_encode_batch(dlic_batch* b, const uint8_t* d_pixels, uint8_t* d_out,
                              uint64_t* d_out_len, uint64_t* d_t_done, void* d_ws,
                              size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  dlic_status rc = batch_call_ok(b, d_pixels, d_out, d_out_len, d_ws, ws_bytes);
  if (rc != DLIC_OK) return rc;
  return batch_enqueue(b, false, d_pixels, d_out, d_out_len, nullptr, d_t_done, d_ws, stream);
}

dlic_status dlic_decode_batch(dlic_batch* b, const uint8_t* d_bits, const uint64_t* d_len,
                              uint8_t* d_pixels, int32_t* d_status, uint64_t* d_t_done,
                              void* d_ws, size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  dlic_status rc = batch_call_ok(b, d_bits, d_pixels, d_len, d_ws, ws_bytes);
  if (rc != DLIC_OK) return rc;
  if (!d_status) return DLIC_ERR_ARG;
  return batch_enqueue(b, true, d_bits, d_pixels, (uint64_t*)d_len, d_status, d_t_done, d_ws,
                       stream);
}

dlic_status dlic_batch_capture(dlic_batch* b, int32_t decode, const uint8_t* d_in,
                               uint8_t* d_out, uint64_t* d_len, int32_t* d_status,
                               uint64_t* d_t_done, void* d_ws, size_t ws_bytes) {
  dlic_status rc = batch_call_ok(b, d_in, d_out, d_len, d_ws, ws_bytes);
  if (rc != DLIC_OK) return rc;
  if (decode && !d_status) return DLIC_ERR_ARG;
  const int d = decode ? 1 : 0;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DLIC_ERR_HIP;
  const bool timing = g_timing;
  g_timing = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rc = DLIC_ERR_HIP;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    const dlic_status er = batch_enqueue(b, decode != 0, d_in, d_out, d_len, d_status, d_t_done,
                                         d_ws, cs);
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (er != DLIC_OK) {
      rc = er;
    } else if (ec == hipSuccess && graph &&
               hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
      rc = DLIC_OK;
    }
  }
  g_timing = timing;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  (void)hipGetLastError();
  if (rc != DLIC_OK) return rc;
  if (b->exec[d]) (void)hipGraphExecDestroy(b->exec[d]);
  b->exec[d] = exec;
  return DLIC_OK;
}

dlic_status dlic_batch_replay(dlic_batch* b, int32_t decode, hipStream_t stream) {
  if (!b) return DLIC_ERR_ARG;
  const int d = decode ? 1 : 0;
  if (!b->exec[d]) return DLIC_ERR_ARG;
  timing_reset();
  timing_begin(decode ? "batch_decode_graph" : "batch_encode_graph", stream);
  const hipError_t e = hipGraphLaunch(b->exec[d], stream);
  timing_end(stream);
  return e == hipSuccess ? DLIC_OK : DLIC_ERR_HIP;
}

dlic_status dlic_latency_probe(double* h_out, int32_t n, void* d_ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (!h_out || n < DLIC_PROBE_COUNT || !d_ws || ws_bytes < 256) return DLIC_ERR_ARG;
  dlic_status rc = current_consts(nullptr);
  if (rc != DLIC_OK) return rc;
  unsigned long long* out = (unsigned long long*)d_ws;
  uint32_t* gflags = (uint32_t*)((uint8_t*)d_ws + 128);
  unsigned long long hv[4];
  bool all_ok = true;
  double mhz = 0.0;
  for (int p = 0; p + 1 < DLIC_PROBE_COUNT; ++p) {
    launch_fill_u32(gflags, 0u, 32, stream);
    launch_latency_probe(p, out, gflags, stream);
    if (launch_ok() != DLIC_OK) return DLIC_ERR_HIP;
    if (hipMemcpyAsync(hv, out, sizeof(hv), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return DLIC_ERR_HIP;
    all_ok = all_ok && hv[2] == 1ull;
    h_out[p] = (double)hv[0] / (double)probe_links(p);
    if (p == 0 && hv[1] > 0) mhz = (double)hv[0] / (double)hv[1] * 100.0;
  }
  h_out[DLIC_PROBE_COUNT - 1] = mhz;
  return all_ok ? DLIC_OK : DLIC_ERR_TIMEOUT;
}

size_t dlic_deep_workspace(const dlic_deep_model* model, int32_t h, int32_t w,
                           const dlic_coder* coder, int32_t decode) {
  if (!model || h <= 0 || w <= 0 || deep_model_ok(model, true) != DLIC_OK) return 0;
  if (decode >= 0 && !flat_coder_ok(h, coder)) return 0;
  return deep_ws_bytes(1, h, w, coder, model->hidden, model->depth, decode);
}

dlic_status dlic_deep_density(const dlic_deep_model* model, const void* d_img, int32_t h,
                              int32_t w, float* d_logits, uint32_t* d_cf, uint16_t* d_tables,
                              void* d_ws, size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  if (!d_img || !d_ws || h <= 0 || w <= 0 || (!d_logits && !d_cf && !d_tables))
    return DLIC_ERR_ARG;
  const dlic_status rc = deep_model_ok(model, false);
  if (rc != DLIC_OK) return rc;
  return deep_density_impl(model, d_img, h, w, VolGeom{}, d_logits, d_cf, d_tables, d_ws,
                           ws_bytes, stream);
}

dlic_status dlic_deep_encode(const dlic_deep_model* model, const dlic_coder* coder,
                             const void* d_img, int32_t h, int32_t w, uint8_t* d_out,
                             size_t out_cap, uint64_t* d_out_len, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  timing_reset();
  if (!d_img || !d_out || !d_out_len || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!flat_coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  const dlic_status rc = deep_model_ok(model, false);
  if (rc != DLIC_OK) return rc;
  return deep_encode_impl(model, coder, d_img, h, w, VolGeom{}, deep_header(model, nullptr),
                          d_out, out_cap, d_out_len, d_ws, ws_bytes, stream);
}

dlic_status dlic_deep_decode(const dlic_deep_model* model, const dlic_coder* coder,
                             const uint8_t* d_bits, size_t n_bytes, void* d_img, int32_t h,
                             int32_t w, int32_t* d_status, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  timing_reset();
  if (!d_bits || !d_img || !d_status || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  if (!flat_coder_ok(h, coder)) return DLIC_ERR_UNSUPPORTED;
  const dlic_status rc = deep_model_ok(model, false);
  if (rc != DLIC_OK) return rc;
  return deep_decode_impl(model, coder, d_bits, n_bytes, d_img, h, w, VolGeom{},
                          deep_header(model, nullptr), d_status, d_ws, ws_bytes, stream);
}

void dlic_set_deep_decode_grid(int32_t workgroups) { g_deep_grid = workgroups > 0 ? workgroups : 0; }

dlic_status dlic_deep_slice_stamps(uint64_t* h_out, int32_t n) {
  if (!h_out) return DLIC_ERR_ARG;
  return deep_slice_stamps((unsigned long long*)h_out, n) == 0 ? DLIC_OK : DLIC_ERR_ARG;
}

int32_t dlic_deep_decode_grid(void) { return g_deep_grid_used; }

size_t dlic_volume_encode_bound(int32_t z, int32_t h, int32_t w, const dlic_coder* coder) {
  if (z < 1 || z > DLIC_VOLUME_MAX_SLICES || h <= 0 || w <= 0 || !vol_coder_ok(z, h, coder))
    return 0;
  const dlic_coder tc = stacked_coder(coder, z);
  return dlic_encode_bound(z * h, w, &tc);
}

size_t dlic_volume_workspace(const dlic_deep_model* model, int32_t z, int32_t h, int32_t w,
                             const dlic_coder* coder, int32_t decode) {
  if (!model || z < 1 || z > DLIC_VOLUME_MAX_SLICES || h <= 0 || w <= 0 ||
      deep_model_ok(model, true) != DLIC_OK)
    return 0;
  if (decode >= 0 && !vol_coder_ok(z, h, coder)) return 0;
  return deep_ws_bytes(z, h, w, coder, model->hidden, model->depth, decode);
}

dlic_status dlic_volume_density(const dlic_deep_model* model, const void* d_vol, int32_t z,
                                int32_t h, int32_t w, int32_t ws, float* d_logits, uint32_t* d_cf,
                                uint16_t* d_tables, void* d_ws, size_t ws_bytes,
                                hipStream_t stream) {
  timing_reset();
  if (!d_vol || !d_ws || h <= 0 || w <= 0 || (!d_logits && !d_cf && !d_tables))
    return DLIC_ERR_ARG;
  const dlic_status rc = deep_model_ok(model, true);
  if (rc != DLIC_OK) return rc;
  VolGeom vg;
  if (!vol_geom(model, z, ws, &vg)) return DLIC_ERR_ARG;
  return deep_density_impl(model, d_vol, h, w, vg, d_logits, d_cf, d_tables, d_ws, ws_bytes,
                           stream);
}

dlic_status dlic_volume_encode(const dlic_deep_model* model, const dlic_coder* coder,
                               const void* d_vol, int32_t z, int32_t h, int32_t w, int32_t ws,
                               uint8_t* d_out, size_t out_cap, uint64_t* d_out_len, void* d_ws,
                               size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  if (!d_vol || !d_out || !d_out_len || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  const dlic_status rc = deep_model_ok(model, true);
  if (rc != DLIC_OK) return rc;
  VolGeom vg;
  if (!vol_geom(model, z, ws, &vg)) return DLIC_ERR_ARG;
  if (!vol_coder_ok(z, h, coder)) return DLIC_ERR_UNSUPPORTED;
  return deep_encode_impl(model, coder, d_vol, h, w, vg, deep_header(model, &vg), d_out, out_cap,
                          d_out_len, d_ws, ws_bytes, stream);
}

dlic_status dlic_volume_decode(const dlic_deep_model* model, const dlic_coder* coder,
                               const uint8_t* d_bits, size_t n_bytes, void* d_vol, int32_t z,
                               int32_t h, int32_t w, int32_t ws, int32_t* d_status, void* d_ws,
                               size_t ws_bytes, hipStream_t stream) {
  timing_reset();
  if (!d_bits || !d_vol || !d_status || !d_ws || h <= 0 || w <= 0) return DLIC_ERR_ARG;
  const dlic_status rc = deep_model_ok(model, true);
  if (rc != DLIC_OK) return rc;
  VolGeom vg;
  if (!vol_geom(model, z, ws, &vg)) return DLIC_ERR_ARG;
  if (!vol_coder_ok(z, h, coder)) return DLIC_ERR_UNSUPPORTED;
  return deep_decode_impl(model, coder, d_bits, n_bytes, d_vol, h, w, vg,
                          deep_header(model, &vg), d_status, d_ws, ws_bytes, stream);
}

dlic_status dlic_peek_volume(const uint8_t* b, size_t n, int32_t* z, int32_t* h, int32_t* ws,
                             int32_t* k_in, dlic_coder* coder) {
  if (!b || n < (size_t)HEADER_BYTES) return DLIC_ERR_CORRUPT;
  if (memcmp(b, "DLIC", 4) != 0) return DLIC_ERR_CORRUPT;
  auto u16 = [&](int o) { return (uint32_t)b[o] | ((uint32_t)b[o + 1] << 8); };
  auto u32 = [&](int o) { return u16(o) | (u16(o + 2) << 16); };
  if (u16(4) != 1u) return DLIC_ERR_CORRUPT;
  const int Z = (int)(u16(6) & 0xFFFu), S = (int)(u16(6) >> 12);
  const int HT = (int)u32(8), GT = (int)u16(26);
  if (Z < 1 || HT % Z != 0 || GT % Z != 0) return DLIC_ERR_CORRUPT;  // not a volume stream
  if (z) *z = Z;
  if (h) *h = HT / Z;
  if (ws) *ws = S;
  if (k_in) *k_in = b[16];
  if (coder) {
    coder->groups = GT / Z;
    coder->lanes_per_group = b[25];
  }
  return DLIC_OK;
}

double dlic_wallclock_hz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0.0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
  return 1000.0 * (double)khz;
}

}  // extern "C"
