// Launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dlic_device.hpp"

namespace dlic {

struct HeaderFields {
  int dtype, h1, h2;
  uint64_t fingerprint;
  int n_mix = N_MIX;  // 0: the six-layer softmax-256 network
  int k_in = K_IN;    // window size: 12, or 21 with the slice below (volumes)
  int flags = 0;      // volumes: slices in bits 0..11, window shift in bits 12..15;
                      // images: strips per group - 1 in bits 12..15
};

// Decoder limits: rows per group, and the per-group stream ring in LDS.
constexpr int DEC_RMAX = 256;
constexpr int DEC_RING = 4096;

struct DecArgs {
  const uint8_t* bits;
  unsigned long long n_bytes;
  uint8_t* img;
  int H, W, G, L;
  int S;                  // row strips per group (1: one contiguous strip)
  uint32_t* rec;          // [S*G][T] progress records (one row per strip), cleared before launch
  unsigned* ticket;       // one-image decode: next group to take, cleared before launch
  long long T;            // wavefront steps W + 3H - 3
  int* status;
  uint32_t spin_limit;
  uint32_t delay_seed, delay_max;  // injected wave delays (test hook), 0: none
  int check_model;        // compare header model fields with the ones below
  HeaderFields hf;
  const uint32_t* tables;  // table mode: [n_tables][257]
  int n_tables;
  const uint32_t* tidx;    // table mode: [H*W]
  unsigned long long* prof;  // optional per-group cycle counters (8 per group)
};

// wtype: WeightType of the model; width: h1 == h2.  False for an unsupported pair.
// ---- batches of images (one plan, work items = (image, group)) ----------
struct BatchImage {
  long long px_off;     // first pixel in the concatenated pixel buffers (also the cf index)
  long long words_off;  // first u16 of the image's word scratch
  long long out_off;    // first byte of the image's stream region
  long long out_cap;    // bytes of that region (dlic_encode_bound of the image)
  long long rec_off;    // first u32 of the image's decode records
  long long T;          // wavefront steps W + 3H - 3
  int H, W, G, L;
  int counts_off;       // first u32 of the image's per-group word counts
  int blk_off;          // first 256-pixel density block of the image
};

struct BatchItem {
  int image, group;
};

struct BatchArgs {
  const BatchImage* images;
  const BatchItem* items;  // longest wavefront first; groups of an image in order
  int n_img, n_items, n_blk;
  const uint8_t* pix_in;   // encode: the images
  uint8_t* pix_out;        // decode: the images
  uint32_t* cf;
  uint16_t* words;
  uint32_t* counts;
  uint8_t* out;            // encode: stream regions
  const uint8_t* bits;     // decode: stream regions
  uint64_t* len;           // encode writes / decode reads one length per image
  uint32_t* rec;
  int* status;             // decode: one per image
  unsigned* ticket;        // decode: next work item
  unsigned* done;          // per image: finished blocks (encode) or groups (decode)
  unsigned long long* t_done;  // optional per-image completion times (realtime counter)
  HeaderFields hf;
  uint32_t spin_limit;
  uint32_t delay_seed, delay_max;  // injected wave delays (test hook), 0: none
};

bool launch_density(int wtype, int width, const Consts* K, const DevModel& m, const uint8_t* img,
                    int H, int W, uint32_t* cf, float* out15, uint32_t* tables, int grid,
                    hipStream_t s);
// Largest layer-1 and layer-2 activations of the FP32 net over an image,
// folded into amax[0..1] (atomic maximum; the caller clears them).
bool launch_activation_range(int width, const Consts* K, const DevModel& m, const uint8_t* img,
                             int H, int W, float* amax, int grid, hipStream_t s);
// Test hook: both FP32 forms of the 12-H-H-15 net (H = width, 64 or 128) on n
// (a multiple of 16) feature rows; out16 / out4: [n][15].  False for another width.
bool launch_net_forms(int width, const DevModel& m, const float* feats, long long n, int lanes,
                      float* out16, float* out4, hipStream_t s);
// S: row strips per group (1: one contiguous strip)
void launch_rans_encode(const uint32_t* cf, int H, int W, int G, int L, int S, uint16_t* words,
                        uint32_t* counts, hipStream_t s);
void launch_pack(const uint16_t* words, const uint32_t* counts, int H, int W, int G, int L, int S,
                 const HeaderFields& hf, uint8_t* out, uint64_t* out_len, int chunks,
                 hipStream_t s);
bool launch_decode(int wtype, int width, bool tables_mode, const Consts* K, const DevModel& m,
                   const DecArgs& a, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t s);
// Stamps the realtime counter into *t (the start of a batch).
void launch_stamp(unsigned long long* t, hipStream_t s);

bool launch_batch_density(int wtype, int width, const Consts* K, const DevModel& m,
                          const BatchArgs& b, int grid, hipStream_t s);
void launch_batch_rans_encode(const BatchArgs& b, hipStream_t s);
void launch_batch_pack(const BatchArgs& b, int parts, hipStream_t s);
// Lanes of the decoder's coder wave that serve one pixel in its symbol
// search: 1 for L > 32, 2 for 4 < L <= 32 (two half-waves, mixture
// components 0..2 and 3..4), 16 for L <= 4 (one interior level of the bucket
// per lane).
__host__ __device__ constexpr int coder_lpp(int L) { return L <= 4 ? 16 : (L <= 32 ? 2 : 1); }

// lpp: coder lanes per pixel, coder_lpp(L) of the widest image of the batch
// or a smaller fan-out the plan asks for.  grid_cap > 0 caps the persistent
// grid below the number of workgroups that stay resident.
bool launch_batch_decode(int wtype, int width, const Consts* K, const DevModel& m,
                         const BatchArgs& b, int lpp, int grid_cap, hipStream_t s);

// Latency probes of the decode's critical path (one chain per probe; see
// dlic_probe.hip): out[0] shader cycles, out[1] real-time ticks, out[2] 1 if
// every hand-off completed.  gflags: 32 cleared words.
void launch_latency_probe(int probe, unsigned long long* out, uint32_t* gflags, hipStream_t s);
int probe_links(int probe);

// ---- six-layer softmax-256 network (the paper's own head) -----------------
constexpr int DEEP_LAYERS = 6;
constexpr int DEEP_OUT = 256;
constexpr int K_IN_3D = 21;   // the 12-pixel window plus 3 x 3 pixels of the slice below
constexpr int DEEP_OUT12 = 4096;  // output levels of 12-bit samples
struct DeepNetArgs {
  int H;                        // hidden width (64 or 128)
  int k_in;                     // K_IN, or K_IN_3D for volumes
  int nout;                     // DEEP_OUT, or DEEP_OUT12 for 12-bit samples
  const void* wop;              // weights in MFMA operand order (deep_pack_weights)
  const float* b[DEEP_LAYERS];  // FP32 biases
};
// Geometry of what the deep kernels code: Z slices of H x W stacked into one
// image of Z H rows (an image: Z = 1).  Slice z trails z - 1 by lag wavefront
// steps; the window reaches rows y + ws - 3 .. y + ws - 1 of the slice below.
struct VolGeom {
  int Z = 1, ws = 0, lag = 0;
};
// Bytes of the operand-order weights of a k_in -> H x 5 -> nout net (k_in <= 32).
size_t deep_wop_bytes(int H, int nout);
// Rearrange row-major BF16 weights (w[i]: [out][in]) into operand order at wop.
void launch_deep_pack(int H, int k_in, int nout, const uint16_t* const* w, void* wop,
                      hipStream_t s);
// Encoder density: packed interval c | (f - 1) << 16 of every pixel (raster
// order of the stacked image) by the softmax table rule; optionally the FP32
// logits [n][256] and the tables F(0..255) [n][256] (u16).  H: rows per slice.
// False for an unsupported width or window.
bool launch_deep_density(const Consts* K, const DeepNetArgs& net, const uint8_t* img, int H,
                         int W, const VolGeom& vg, uint32_t* cf, float* logits,
                         uint16_t* tables, hipStream_t s);
struct DeepDecArgs {
  DeepNetArgs net;
  const Consts* K;
  const uint8_t* bits;
  unsigned long long n_bytes;
  void* img;          // u8 samples, or u16 for 12-bit ones
  int H, W, G, L;     // H: rows per slice; G: groups per slice
  VolGeom vg;
  long long T;        // W + 3 (H - 1) + lag (Z - 1)
  uint16_t* tables;   // [Z H][levels]: F(0..levels-1) of each row's pixel of the current step
  // 12-bit decoder: the step's tiles (last hidden layer as operands, first row
  // and row count) and each row's logits [Z H][4096]
  void* h5;
  int2* tile_rows;
  float* logits;
  unsigned* bar;      // grid barrier counter, cleared before launch (12-bit decoder)
  int* pix_step;      // [Z H]: step of each row's newest decoded pixel, -1 before launch
  int* tab_step;      // [Z H]: step of each row's newest table, -1 before launch
  uint32_t delay_seed, delay_max;  // injected wave delays (test hook), 0: none
  int* abort_flag;    // cleared before launch
  int* status;
  uint32_t spin_limit;
  HeaderFields hf;
};
// Cooperative launch of the per-step decoder; returns the hipError of the launch.
hipError_t launch_deep_decode(const DeepDecArgs& a, int grid, hipStream_t s);
int deep_decode_max_grid(int H, int k_in);
constexpr int DEEP_MAX_SLICES = 4095;
// Host copy of the last 8-bit deep decode's real-time stamps (start, then each
// slice's completion); -1 on a bad count or a HIP error.
int deep_slice_stamps(unsigned long long* h_out, int n);

// ---- 12-bit samples: 4096 output levels ----------------------------------
// Encoder stages over pixels [px0, px0 + n) of the stacked image (u16
// samples): hidden layers of every 16-pixel tile into h5 (operand order,
// NK * 64 bf16x8 per tile); the output layer as a GEMM into logits [n][4096]
// FP32; the table rule per pixel into packed intervals cf[px] (and optionally
// tables [n][4096] u16).  bad: set to 1 where a sample exceeds 4095.
bool launch_deep12_hidden(const Consts* K, const DeepNetArgs& net, const uint16_t* img, int H,
                          int W, const VolGeom& vg, long long px0, long long n, void* h5,
                          int* bad, hipStream_t s);
bool launch_deep12_logits(const DeepNetArgs& net, const void* h5, long long n_px,
                          float* logits, hipStream_t s);
void launch_deep12_softmax(const float* logits, const uint16_t* img, long long px0, long long n,
                           uint32_t* cf, uint16_t* tables, hipStream_t s);
// Zero *out_len when bad is set (the stream of an invalid image is empty).
void launch_deep12_reject(const int* bad, uint64_t* out_len, hipStream_t s);
// Cooperative per-step decoder of 12-bit streams (four grid barriers a step).
hipError_t launch_deep12_decode(const DeepDecArgs& a, int grid, hipStream_t s);
int deep12_decode_max_grid(int H, int k_in);
// h5 bytes of one 16-pixel tile
inline size_t deep12_tile_bytes(int H) { return (size_t)H * 16 * 2; }
constexpr int DEEP_WAVES = 4;  // waves per workgroup of the deep kernels

// Training: waves per workgroup of the FP32 / FP64 loss-and-gradient kernel.
constexpr int TRAIN_WAVES_F32 = 8;
constexpr int TRAIN_WAVES_F64 = 1;
constexpr int TRAIN_GRID = 256;
int train_n_params(int h1, int h2);
bool launch_nll(bool fp64, int width, const void* w1, const void* b1, const void* w2,
                const void* b2, const void* w3, const void* b3, const uint8_t* slices,
                int n_slices, int sh, int sw, const int32_t* idx, long long n, void* partials,
                int grid, bool want_grad, void* grad, void* loss, hipStream_t s);
void launch_adam(long long np, float* p, const float* g, float* m, float* v, int step, float lr,
                 float b1, float b2, float eps, hipStream_t s);

}  // namespace dlic
