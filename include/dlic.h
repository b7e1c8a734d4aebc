/*
 * dlic.h -- C ABI of the DLIC hot path on AMD Instinct MI355X (gfx950).
 *
 * Deep Lossless Image Coding (Barzen, Glazov, Geistert, Sikora, arXiv
 * 2207.05152) codes an 8-bit greyscale image pixel by pixel: a small fully
 * connected network turns each pixel's causal neighbourhood into a PDF over
 * the 256 grey levels (Section II-A, Fig. 2), and an rANS coder codes the
 * pixel with it (Section II-B, rANS).  Pixels whose neighbourhood is already
 * coded are processed together in wavefront order (Section II-B,
 * Preprocessor; Fig. 1 right), and everything stays on the GPU with one
 * upload and one download (Section II-B, Preprocessor, last paragraph).
 *
 * Conventions for every entry point:
 *   - d_ pointers are device memory owned by the caller; h_ pointers are
 *     host memory owned by the caller.  The library never frees caller
 *     memory.  Scratch space is passed in as d_ws of the size the matching
 *     *_workspace function returns.
 *   - Work is enqueued on the caller's stream and the call returns without
 *     synchronising.  Argument errors found on the host are returned
 *     directly; failures found by kernels (corrupt stream, timeout) are
 *     written to a device status word that the caller reads after
 *     synchronising.
 *   - No call throws or exits.  The library has no CPU fallback: without a
 *     usable gfx950 device every GPU entry point returns DLIC_ERR_HIP.
 *   - Results are deterministic: the same inputs give the same bytes.
 *
 * Format constants (all fixed by this library): 12-neighbour causal window
 * (rows y-2, y-1 at dx -2..+2, then (y, x-2), (y, x-1)), values scaled by
 * (2v-255)/255, dummy 0 outside the image; network 12 -> h1 -> h2 -> 15 with
 * ReLU; outputs [5 logits, 5 means, 5 log-scales >= -7]; frequency tables of
 * total 2^16 with every symbol >= 1; 32-bit rANS state, 16-bit words;
 * wavefront step t = x + 3y.
 */
#ifndef DLIC_H
#define DLIC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DLIC_OK = 0,
  DLIC_ERR_ARG = 1,            /* bad pointer, size or parameter                 */
  DLIC_ERR_CAPACITY = 2,       /* output or workspace buffer too small           */
  DLIC_ERR_CORRUPT = 3,        /* stream malformed or inconsistent (device)      */
  DLIC_ERR_MODEL_MISMATCH = 4, /* stream coded with another model (device)       */
  DLIC_ERR_UNSUPPORTED = 5,    /* dims, dtype or layout the library does not run */
  DLIC_ERR_HIP = 6,            /* HIP runtime error or no usable device          */
  DLIC_ERR_TIMEOUT = 7         /* a decode wait exceeded its spin limit (device) */
} dlic_status;

typedef enum {
  DLIC_FP32 = 0,
  DLIC_BF16 = 1,
  DLIC_FP8_E4M3 = 2, /* e4m3 weights, BF16 activations (W8A16)              */
  DLIC_FP64 = 3,     /* training entry points only (gradient checks)       */
  DLIC_FP8_W8A8 = 4  /* e4m3 weights and activations on the FP8 MFMA       */
} dlic_dtype;

/* Network weights (Section II-B, Neural Network Architecture; the mixture
 * head of Section I / IV-C).  Matrices are row-major [out][in] in the given
 * dtype (FP32 values, BF16 bit patterns or e4m3 codes, as
 * dlic_quantize_weights writes them); biases are FP32.  Supported widths:
 * h1 == h2 in {32, 64, 128} for FP32, BF16 and FP8 inference; {32, 64} for
 * training (FP32, FP64). */
typedef struct dlic_model {
  int32_t k_in;          /* must be 12                                      */
  int32_t h1, h2;        /* hidden widths                                   */
  int32_t n_out;         /* must be 15                                      */
  int32_t dtype;         /* dlic_dtype of d_w1, d_w2, d_w3                  */
  int32_t reserved;      /* must be 0                                       */
  const void *d_w1;      /* [h1][12]                                        */
  const void *d_w2;      /* [h2][h1]                                        */
  const void *d_w3;      /* [15][h2]                                        */
  const float *d_b1, *d_b2, *d_b3;
  const float *d_wscale; /* FP8_E4M3: 3 per-layer weight scales; FP8_W8A8:
                            those 3, then the 3 activation multipliers
                            (device); otherwise NULL                        */
  uint64_t fingerprint;  /* dlic_fnv1a64 over W1,b1,W2,b2,W3,b3 bytes (then
                            the 3 scales for FP8)                          */
} dlic_model;

/* Coder instances (Section II-B, rANS: several coder instances and
 * bitstreams).  G groups, each one stream shared by lanes_per_group
 * interleaved 32-bit rANS states.  With S = strips (0 or 1: S = 1) the image
 * is cut into S*G row strips, strip b owning rows [b*H/(SG), (b+1)*H/(SG)),
 * and group g codes strips g, G + g, ..., (S-1)G + g one after another, its
 * lanes' states carrying from strip to strip; row y of a strip starting at
 * row r is lane (y - r) % L.  Spread strips let a group's decode work in
 * fewer wavefront steps at once when a strip is shorter than the band of
 * rows the wavefront keeps active (about W/3 rows).  An image stream stores
 * S - 1 in bits 12..15 of its header flags.
 * Constraints: 1 <= L <= 64; G <= 1024; S <= DLIC_MAX_STRIPS; S*G == 1 or
 * H >= 2*S*G; at most 256 rows per strip (the decoder keeps a strip's pixel
 * ring in LDS).  S > 1: the mixture-network image codec only (dlic_encode,
 * dlic_decode, dlic_rans_encode_cf, dlic_rans_decode_tables), with all G
 * decoder workgroups resident at once (DLIC_ERR_UNSUPPORTED otherwise). */
#define DLIC_MAX_STRIPS 16
typedef struct dlic_coder {
  int32_t groups;
  int32_t lanes_per_group;
  int32_t strips;
} dlic_coder;

/* ---- host-only helpers (no device needed) ----------------------------- */

/* Human-readable name of a status code.  Never NULL. */
const char *dlic_status_string(dlic_status s);

/* 64-bit FNV-1a of n bytes continuing from hash h (start with
 * 0xcbf29ce484222325).  Used for the model fingerprint that the stream
 * header carries, so a decoder refuses weights other than the encoder's
 * (Section II-B, Preprocessor: both sides must evaluate the same network). */
uint64_t dlic_fnv1a64(uint64_t h, const void *h_bytes, size_t n);

/* The format's FP32 constant tables, as the kernels use them: the table
 * logistic knots S[4097] and slopes D[4097] on [-16, 16] (step 2^-7), the
 * bin edges beta[257] (beta[0] = -inf, beta[256] = +inf) and the scaled grey
 * levels scale[256].  Any pointer may be NULL. */
void dlic_host_constants(float *h_S, float *h_D, float *h_beta, float *h_scale);

/* The network's input scale of each level as the kernels use it,
 * RN32((2v - m) / m) with m = 2^depth - 1: 256 floats for depth 8, 4096 for
 * depth 12 (DLIC_ERR_ARG for another depth). */
dlic_status dlic_host_scale(int32_t depth, float *h_out);

/* Weight storage of the reduced-precision networks (the network of Section
 * II-B run with BF16 or FP8 operands and FP32 accumulation).  Converts one
 * FP32 matrix of n finite elements, host to host:
 *   DLIC_BF16      h_out: n uint16 BF16 bit patterns, round to nearest even;
 *                  *h_scale (if not NULL) = 1.
 *   DLIC_FP8_E4M3  *h_scale = max|W| / 448 in FP32 (1 for an all-zero
 *                  matrix); h_out: n OCP e4m3 codes (bias 7, no infinities)
 *                  of W / scale computed in FP32, rounded to nearest even and
 *                  saturated at +-448.  The net computes scale * (Q a) + b.
 * Returns DLIC_ERR_ARG for NULL pointers, n == 0, a non-finite weight or
 * another dtype.  A model's fingerprint covers the converted bytes of W1,
 * b1, W2, b2, W3, b3 in that order, then for FP8 the three scales. */
dlic_status dlic_quantize_weights(int32_t dtype, const float *h_w, size_t n, void *h_out,
                                  float *h_scale);

/* Activation multipliers of the W8A8 net: m_l = 2^floor(log2(448 / amax_l))
 * for each of the 3 layer inputs (1 where amax_l <= 0), so that the largest
 * input times m_l fits the e4m3 range exactly; the net rounds m_l * a to
 * e4m3 and rescales the layer's accumulator by s_l / m_l (exact).  The
 * inputs of layer 1 are the scaled grey levels, amax_1 = 1; amax_2 and
 * amax_3 come from dlic_activation_range on calibration images.  Host only. */
dlic_status dlic_w8a8_multipliers(const float *h_amax, float *h_mult);

/* Worst-case stream size in bytes for an h x w image: header, word counts,
 * at most one 16-bit word per pixel and the flushed states. */
size_t dlic_encode_bound(int32_t h, int32_t w, const dlic_coder *coder);

/* Scratch bytes dlic_encode / dlic_rans_encode_cf need (d_ws). */
size_t dlic_encode_workspace(int32_t h, int32_t w, const dlic_coder *coder);

/* Scratch bytes dlic_decode / dlic_rans_decode_tables need (d_ws). */
size_t dlic_decode_workspace(int32_t h, int32_t w, const dlic_coder *coder);

/* Parse the 36-byte stream header from host bytes.  Any out pointer may be
 * NULL.  coder receives groups, lanes and strips (1 for a volume stream).
 * Returns DLIC_ERR_CORRUPT for a bad magic, version or length. */
dlic_status dlic_peek_header(const uint8_t *h_bits, size_t n, int32_t *h, int32_t *w,
                             dlic_coder *coder, uint64_t *fingerprint,
                             int32_t *h1, int32_t *h2, int32_t *dtype);

/* ---- device entry points ------------------------------------------------ */

/* Select and prepare a device: uploads the constant tables once per device.
 * Idempotent; every other device entry point calls it for the current
 * device.  Returns DLIC_ERR_HIP if no gfx950 device is usable. */
dlic_status dlic_init(int device);

/* Encode an 8-bit image (Section II-A, Fig. 2 left; Section II-B).
 * d_img: [h][w] uint8 row-major.  Phase one computes every pixel's mixture
 * and frequency interval in parallel (the network on the matrix of all
 * windows); phase two runs each group's rANS walk in reverse wavefront
 * order; a pack kernel writes header, word counts and streams to d_out.
 * out_cap must be >= dlic_encode_bound.  *d_out_len (device, u64) receives
 * the stream length in bytes. */
dlic_status dlic_encode(const dlic_model *model, const dlic_coder *coder,
                        const uint8_t *d_img, int32_t h, int32_t w,
                        uint8_t *d_out, size_t out_cap, uint64_t *d_out_len,
                        void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Decode a stream (Section II-A, Fig. 2 right): one persistent workgroup per
 * group walks the wavefront, evaluating the same network on already decoded
 * windows and decoding every active pixel from its lane's state.  h, w and
 * the coder layout are the header's (dlic_peek_header on the host copy of
 * the first bytes); the kernel re-validates the header against them, the
 * model and the stream length.  d_img: [h][w] uint8.  *d_status (device,
 * int32) receives DLIC_OK, or DLIC_ERR_CORRUPT / DLIC_ERR_MODEL_MISMATCH /
 * DLIC_ERR_TIMEOUT.  A corrupt stream never faults or hangs: every read is
 * bounds-checked and every wait is bounded. */
dlic_status dlic_decode(const dlic_model *model, const dlic_coder *coder,
                        const uint8_t *d_bits, size_t n_bytes, uint8_t *d_img,
                        int32_t h, int32_t w, int32_t *d_status,
                        void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of the fixed workspace array of dlic_decode_noalloc. */
#define DLIC_DECODE_NOALLOC_BYTES ((size_t)8 << 20)

/* dlic_decode for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same stream format, kernels, results and device status as dlic_decode,
 * without d_ws: the decode's progress records and group ticket live in a
 * fixed array of DLIC_DECODE_NOALLOC_BYTES (8 MiB) that the library keeps on
 * every device it runs on until the process ends.  The call makes
 * no allocation, creates no timing events, and clears the part of the array
 * it uses with a kernel before its decode kernel runs.  Needs dlic_init on
 * the current device first (DLIC_ERR_ARG otherwise: set-up allocates).
 * Returns DLIC_ERR_CAPACITY when dlic_decode_workspace(h, w, coder) exceeds
 * the limit (G * (W + 3H - 3) + 1 four-byte words; 2048x1536 with 64 groups
 * takes 1.7 MB).  Every call on one device shares its array: calls whose
 * kernels overlap on one GPU (several streams, several host threads) race
 * and must be serialised by the caller. */
dlic_status dlic_decode_noalloc(const dlic_model *model, const dlic_coder *coder,
                                const uint8_t *d_bits, size_t n_bytes, uint8_t *d_img,
                                int32_t h, int32_t w, int32_t *d_status, hipStream_t stream);


/* Test hook for the decoder's synchronisation (Section II-B, Preprocessor:
 * decode follows the wavefront, so every wave waits for the ones producing
 * its inputs).  With max_cycles > 0 every later decode (single images and
 * batches) pauses each wave at fixed points (the coder before each
 * sub-round, the density waves before each tile and before publishing it,
 * the courier in each round of its loop) for a seeded pseudo-random time
 * below max_cycles shader cycles (at most 2^20), so that the waves' hand-offs
 * meet in other orders; decoded pixels must not change.  0 turns it off
 * (the default).  Host-side setting, not thread-safe. */
void dlic_set_decode_delays(uint32_t seed, uint32_t max_cycles);

/* Spin limit of one decode wait (polls of an upstream record, each followed
 * by a short sleep); a wait that exceeds it reports DLIC_ERR_TIMEOUT and the
 * workgroup continues without waiting again.  Default 2^22.  For tests of the
 * timeout path. */
void dlic_set_spin_limit(uint32_t polls);

/* Density of every pixel of a known image with the same device code the
 * encoder and decoder run (Equation 1; Section II-A).  Outputs, each
 * optional (NULL to skip), raster order:
 *   d_out15  [h*w][15] FP32 raw network outputs (logits, means, log-scales)
 *   d_cf     [h*w] u32: c | (f - 1) << 16 of the pixel's own value
 *   d_tables [h*w][257] u32 cumulative tables F(0..256) (small images) */
dlic_status dlic_density(const dlic_model *model, const uint8_t *d_img, int32_t h, int32_t w,
                         float *d_out15, uint32_t *d_cf, uint32_t *d_tables,
                         hipStream_t stream);

/* Test hook for the rule that encoder and decoder evaluate the network
 * identically (Section II-B, Preprocessor: the same arithmetic on both sides
 * makes the rounding errors equal).  At 12-H-H-15 in FP32 with H = 64 or 128
 * the encoder's density kernel runs 16-pixel tiles on the 16x16x4 MFMA and
 * the decoder (with at most 4 lanes per group) 4-pixel tiles on the 4x4x1
 * MFMA in the same summation order.  This runs both forms on n caller-given
 * feature rows (d_feats: [n][12] FP32, n a multiple of 16) and writes their
 * outputs to d_out16 and d_out4 ([n][15] FP32).  In the 4-pixel form, rows
 * 4s + j with j >= lanes (1..4) are replaced by zero features, as the
 * decoder's unused tile rows; their d_out4 entries are unspecified.  At H = 64
 * the 4-pixel form runs twice, with its layer-2 weights in LDS and in
 * registers (the decoder uses both); an output where the two differ is NaN.
 * model: FP32, h1 = h2 = 64 or 128 (DLIC_ERR_UNSUPPORTED otherwise). */
dlic_status dlic_net_forms(const dlic_model *model, const float *d_feats, int64_t n,
                           int32_t lanes, float *d_out16, float *d_out4, hipStream_t stream);

/* Calibration for the W8A8 net: runs the FP32 network (model->dtype must be
 * DLIC_FP32) on every pixel of an image and folds the largest layer-1 and
 * layer-2 activations into d_amax[0], d_amax[1] (device FP32, atomic
 * maximum: clear them before the first image). */
dlic_status dlic_activation_range(const dlic_model *model, const uint8_t *d_img, int32_t h,
                                  int32_t w, float *d_amax, hipStream_t stream);

/* rANS-only encode (Section II-B, rANS) of caller-given intervals:
 * d_cf [h][w] u32 holds c | (f - 1) << 16 for each pixel (c + f <= 2^16,
 * f >= 1).  Runs the same rANS and pack kernels as dlic_encode; the header
 * carries zeros for the model fields.  Same buffers as dlic_encode. */
dlic_status dlic_rans_encode_cf(const dlic_coder *coder, int32_t h, int32_t w,
                                const uint32_t *d_cf, uint8_t *d_out, size_t out_cap,
                                uint64_t *d_out_len, void *d_ws, size_t ws_bytes,
                                hipStream_t stream);

/* rANS-only decode with caller-given tables: pixel i uses the cumulative
 * table d_tables[d_tidx[i]][0..256] (strictly increasing from 0 to 2^16).
 * Runs the decoder's rANS code in wavefront order without the network.
 * d_sym [h][w] uint8 receives the symbols; *d_status as for dlic_decode. */
dlic_status dlic_rans_decode_tables(const dlic_coder *coder, int32_t h, int32_t w,
                                    const uint32_t *d_tables, int32_t n_tables,
                                    const uint32_t *d_tidx, const uint8_t *d_bits,
                                    size_t n_bytes, uint8_t *d_sym, int32_t *d_status,
                                    void *d_ws, size_t ws_bytes, hipStream_t stream);

/* ---- batches of images --------------------------------------------------- */

/* Many images of any sizes coded with one model in one launch per direction
 * (the wavefront decode of Section II-B, Preprocessor, applied to every
 * group of every image at once).  A plan fixes the images' sizes and coder
 * layouts; work items are (image, group) pairs ordered longest wavefront
 * first, an image's groups in order.  Decode workgroups take items by
 * ticket, so every group an item waits for was taken earlier by a resident
 * or finished workgroup, and all waits end.  Encode = density over all
 * pixels, rANS per item, pack per item: three kernels, one graph. */
typedef struct dlic_batch dlic_batch;

/* Plan for n_img images; h_hw: [n_img][2] (h, w).  h_coders: one layout per
 * image, or NULL for G = ceil(h / 192) groups of 32 lanes.  density_grid:
 * workgroups of the density kernel, 0 for the default.  The plan owns a
 * small device table on the current device until dlic_batch_destroy; its
 * model's weights must stay valid while it is used.  DLIC_ERR_UNSUPPORTED
 * for a layout dlic_encode would refuse. */
dlic_status dlic_batch_create(const dlic_model *model, int32_t n_img, const int32_t *h_hw,
                              const dlic_coder *h_coders, int32_t density_grid,
                              dlic_batch **out);
void dlic_batch_destroy(dlic_batch *b);

/* Decode knobs of a plan, for the autotuner (Section II-B, Preprocessor: the
 * wavefront's work per step spread over the GPU).  search_lanes: coder lanes
 * that share one pixel's symbol search: 16 (one level of a 16-level bucket
 * per lane; every image at most 4 lanes per group), 2 (binary halvings with
 * the mixture split over two half-waves; at most 32 lanes per group), 1 (one
 * lane per pixel), or 0 for the default (16 / 2 / 1 by the widest layout).
 * decode_grid: workgroups of the persistent decode kernel, 0 for as many as
 * stay resident on the device (capped at the number of work items).
 * DLIC_ERR_UNSUPPORTED when a layout of the plan is too wide for the fan-out.
 * The streams and decoded pixels do not depend on either knob. */
dlic_status dlic_batch_tune(dlic_batch *b, int32_t search_lanes, int32_t decode_grid);

/* Bytes of the concatenated pixel buffer (images back to back, raster
 * order), of the stream regions (one per image, dlic_encode_bound bytes,
 * 256-aligned), of the workspace both directions need, and the number of
 * work items.  Any out pointer may be NULL. */
dlic_status dlic_batch_sizes(const dlic_batch *b, size_t *pixels, size_t *out_bytes,
                             size_t *ws_bytes, int32_t *n_items);

/* Per image: first pixel, first byte of its stream region, and (G, L) into
 * h_coders[2i], h_coders[2i+1].  Any out pointer may be NULL. */
dlic_status dlic_batch_layout(const dlic_batch *b, uint64_t *h_px_off, uint64_t *h_out_off,
                              int32_t *h_coders);

/* Encode every image: image i's stream (the same bytes dlic_encode writes
 * for it) goes to its region of d_out, its length to d_out_len[i].  After
 * the call, and until the workspace is used again, its first 4 * pixels
 * bytes hold every pixel's packed interval c | (f - 1) << 16 (u32, at the
 * pixel's index in the concatenated buffer) that the streams code.
 * d_t_done, if not NULL, has n_img + 1 entries: the device realtime counter
 * when image i's stream was complete, and at [n_img] the start of the call
 * (dlic_wallclock_hz gives the counter's rate). */
dlic_status dlic_encode_batch(dlic_batch *b, const uint8_t *d_pixels, uint8_t *d_out,
                              uint64_t *d_out_len, uint64_t *d_t_done, void *d_ws,
                              size_t ws_bytes, hipStream_t stream);

/* Decode every image from its region of d_bits (d_len[i] bytes) into its
 * place in d_pixels; d_status[i] as dlic_decode's status; d_t_done as for
 * dlic_encode_batch.  One launch of a persistent grid: each workgroup takes
 * (image, group) items by ticket until none is left. */
dlic_status dlic_decode_batch(dlic_batch *b, const uint8_t *d_bits, const uint64_t *d_len,
                              uint8_t *d_pixels, int32_t *d_status, uint64_t *d_t_done,
                              void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Capture one direction's kernels (decode = 0: dlic_encode_batch with
 * d_in = pixels, d_out = streams, d_len = lengths; decode = 1:
 * dlic_decode_batch with d_in = streams, d_out = pixels) into a hipGraph
 * kept by the plan, replacing an earlier one.  Counters are cleared by
 * kernels, not memset nodes, so replays start clean.  Buffers are baked in:
 * they must stay valid while the graph is replayed. */
dlic_status dlic_batch_capture(dlic_batch *b, int32_t decode, const uint8_t *d_in,
                               uint8_t *d_out, uint64_t *d_len, int32_t *d_status,
                               uint64_t *d_t_done, void *d_ws, size_t ws_bytes);

/* Launch the captured graph of one direction on a stream. */
dlic_status dlic_batch_replay(dlic_batch *b, int32_t decode, hipStream_t stream);

/* Rate (Hz) of the device realtime counter behind the d_t_done stamps. */
double dlic_wallclock_hz(void);

/* ---- The paper's own network and head (Section II-B, Neural Network
 * Architecture: six dense layers, the output layer 256 neurons with a
 * softmax, one probability per grey level). -------------------------------
 * Layers 12 -> H -> H -> H -> H -> H -> 256 (H = 64 or 128), ReLU after the
 * first five; BF16 weights and layer inputs with FP32 accumulation on the
 * BF16 MFMA, FP32 biases.  The coder's table is the format's FP32 rule on
 * the logits: e_v = expf(o_v - max), the sum over four blocks of 64 levels
 * (each in level order, the blocks added left to right), p_v = e_v / sum,
 * the cumulative sum C_v by blocks (running sums inside a block, offsets the
 * running sum of block totals), F(v) = v + min(65280, floor(C_v 65280)),
 * F(0) = 0, F(256) = 2^16.  Streams use the container, rANS layout and
 * wavefront order of dlic_encode; the header's mixture count is 0 and its
 * dtype DLIC_BF16, h1 = h2 = H.
 *
 * Decoding follows the paper's GPU scheme (Section II-B, Preprocessor: the
 * pixels of one wavefront step enter the network together as a matrix): one
 * cooperative launch walks the W + 3H - 3 steps, the grid evaluating the
 * step's pixels, then every group decoding its rows' pixels of the step
 * (8-bit samples: the phases hand over through per-row step counters; 12-bit
 * samples: a grid barrier after each phase).  It needs every group's wave
 * resident (DLIC_ERR_UNSUPPORTED otherwise): at least 256 groups fit.
 *
 * k_in is 12 for images; volumes (below) also take 21: the 12-pixel window
 * and a 3 x 3 block of the slice below.
 *
 * 12-bit samples (Section IV-C, Higher Bit Depth: 4096 output neurons):
 * depth = 12, an output layer of 4096 neurons, samples as u16 below 4096
 * (d_img / d_vol point to u16 then, u8 for depth 8).  Inputs are scaled by
 * (2v - 4095) / 4095; the table rule is the one above over 64 blocks of 64
 * levels with 65536 - 4096 in place of 65280; the header's dtype byte holds
 * the depth above 8 in its high nibble (0x41).  The encoder writes a stream
 * length of 0 if a sample exceeds 4095. */
#define DLIC_DEEP_LAYERS 6
typedef struct {
  int32_t hidden;                          /* H: 64 or 128 */
  int32_t k_in;                            /* inputs of layer 1: 12, or 21 (volumes) */
  const uint16_t *d_w[DLIC_DEEP_LAYERS];   /* BF16 bit patterns, row-major [out][in] */
  const float *d_b[DLIC_DEEP_LAYERS];      /* FP32 biases */
  uint64_t fingerprint; /* FNV-1a 64 over W1, b1, ..., W6, b6 as stored (BF16 / FP32) */
  int32_t depth;        /* bits per sample: 8 (256 outputs) or 12 (4096 outputs) */
} dlic_deep_model;

/* Device workspace bytes for the model (host struct): decode = 0 for
 * dlic_deep_encode, 1 for dlic_deep_decode, -1 for dlic_deep_density (coder
 * may be NULL then).  0 for an unsupported model, size or layout.  At depth 12
 * encoding takes about 260 MB (the logits of 16384 pixels at a time) and
 * decoding 24 KB per row. */
size_t dlic_deep_workspace(const dlic_deep_model *model, int32_t h, int32_t w,
                           const dlic_coder *coder, int32_t decode);

/* Encode one image with the softmax network: as dlic_encode (same bound,
 * output and length conventions). */
dlic_status dlic_deep_encode(const dlic_deep_model *model, const dlic_coder *coder,
                             const void *d_img, int32_t h, int32_t w, uint8_t *d_out,
                             size_t out_cap, uint64_t *d_out_len, void *d_ws, size_t ws_bytes,
                             hipStream_t stream);

/* Decode a stream of dlic_deep_encode: as dlic_decode (d_status 0, 3 corrupt,
 * 4 other model, 7 a bounded wait gave up). */
dlic_status dlic_deep_decode(const dlic_deep_model *model, const dlic_coder *coder,
                             const uint8_t *d_bits, size_t n_bytes, void *d_img, int32_t h,
                             int32_t w, int32_t *d_status, void *d_ws, size_t ws_bytes,
                             hipStream_t stream);

/* Test hook: the encoder's network and table rule on every pixel of an image
 * (raster order): FP32 logits [n][levels], packed intervals c | (f - 1) << 16
 * [n] of each pixel's own value, tables F(0..levels-1) [n][levels] (u16);
 * each output optional (NULL), at least one. */
dlic_status dlic_deep_density(const dlic_deep_model *model, const void *d_img, int32_t h,
                              int32_t w, float *d_logits, uint32_t *d_cf, uint16_t *d_tables,
                              void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Grid of the deep decoders (dlic_deep_decode, dlic_volume_decode): the
 * number of workgroups of the cooperative launch, clamped to what is resident
 * and raised to fit every group; 0 restores the default (a step's tiles,
 * 64..256).  Process-wide; dlic_deep_decode_grid gives the last launch's. */
void dlic_set_deep_decode_grid(int32_t workgroups);
int32_t dlic_deep_decode_grid(void);

/* Measurement hook for the paper's first-slice and complete-scan times
 * (Section IV-D, Table III): device real-time stamps (dlic_wallclock_hz ticks)
 * of the last 8-bit dlic_deep_decode / dlic_volume_decode on the current
 * device, h_out[0] its start and h_out[1 + s] the moment slice s's last pixel
 * was published (an image is slice 0).  Waits for the device; n is 1 + the
 * number of slices wanted (at most 4096).  Concurrent decodes overwrite each
 * other's stamps. */
dlic_status dlic_deep_slice_stamps(uint64_t *h_out, int32_t n);

/* ---- volumes: the 3-D window and the 3-D wavefront (Section IV-C, 3D
 * Dependencies and 3D Wavefront, Fig. 6) -------------------------------------
 * A volume is z slices of h x w pixels, slice-major in device memory
 * (d_vol[(s h + y) w + x]).  With a model of k_in = 21 a pixel's window is
 * the 12 causal pixels of its own slice, then the 3 x 3 pixels of the slice
 * below at rows y + ws - 3 .. y + ws - 1 and columns x - 1 .. x + 1, row by
 * row, 0 outside the slice (and for the first slice); ws is the paper's
 * window shift.  A model of k_in = 12 codes each slice on its own (ws = 0).
 * The stream is the container of dlic_encode for the z h x w image of the
 * stacked slices with coder->groups groups per slice (so every group lies in
 * one slice): header H = z h, G = z coder->groups, window size k_in, and the
 * header's flags hold z in bits 0..11 and ws in bits 12..15.
 *
 * The decoder walks the 3-D wavefront: pixel (s, y, x) is decoded in step
 * x + 3 y + lag s, lag = max(0, 3 ws - 1) for k_in = 21 (else 0), the least
 * lag that puts every lower-window pixel in an earlier step.  At ws = 0 all
 * slices decode together; the first slice is complete after w + 3 h - 3
 * steps, the volume after lag (z - 1) more.  Limits: 1 <= z <= 4095,
 * 0 <= ws <= 15; coder valid for h (per slice) and z h (stacked), z groups at
 * most 1024 and every group's wave resident. */
#define DLIC_VOLUME_MAX_SLICES 4095
#define DLIC_VOLUME_MAX_SHIFT 15

/* Bytes of the largest stream of a volume (0 for an unsupported layout). */
size_t dlic_volume_encode_bound(int32_t z, int32_t h, int32_t w, const dlic_coder *coder);

/* Device workspace bytes for the model: decode = 0 encode, 1 decode, -1
 * density hook. */
size_t dlic_volume_workspace(const dlic_deep_model *model, int32_t z, int32_t h, int32_t w,
                             const dlic_coder *coder, int32_t decode);

/* Encode a volume (d_vol: z h w samples); as dlic_deep_encode otherwise.
 * DLIC_ERR_ARG for z, ws out of range or ws != 0 with k_in = 12. */
dlic_status dlic_volume_encode(const dlic_deep_model *model, const dlic_coder *coder,
                               const void *d_vol, int32_t z, int32_t h, int32_t w, int32_t ws,
                               uint8_t *d_out, size_t out_cap, uint64_t *d_out_len, void *d_ws,
                               size_t ws_bytes, hipStream_t stream);

/* Decode a stream of dlic_volume_encode into d_vol (z h w samples); z, h, ws
 * and the coder as dlic_peek_volume gives them.  d_status as dlic_deep_decode
 * (3 also when z, h, ws or the coder do not match the stream). */
dlic_status dlic_volume_decode(const dlic_deep_model *model, const dlic_coder *coder,
                               const uint8_t *d_bits, size_t n_bytes, void *d_vol, int32_t z,
                               int32_t h, int32_t w, int32_t ws, int32_t *d_status, void *d_ws,
                               size_t ws_bytes, hipStream_t stream);

/* Test hook: the encoder's network and table rule on every pixel of a volume,
 * outputs as dlic_deep_density in slice-major raster order. */
dlic_status dlic_volume_density(const dlic_deep_model *model, const void *d_vol, int32_t z,
                                int32_t h, int32_t w, int32_t ws, float *d_logits, uint32_t *d_cf,
                                uint16_t *d_tables, void *d_ws, size_t ws_bytes,
                                hipStream_t stream);

/* Volume fields of a stream's header (host memory): slices, rows per slice,
 * window shift, window size and the per-slice coder (any output may be NULL).
 * DLIC_ERR_CORRUPT for a short or foreign header or one that is not a
 * volume's (no slice count, or H or G not a multiple of it). */
dlic_status dlic_peek_volume(const uint8_t *b, size_t n, int32_t *z, int32_t *h, int32_t *ws,
                             int32_t *k_in, dlic_coder *coder);

/* Measurement hook for the decode bound (Section II-B, Preprocessor and rANS:
 * each wavefront step waits for the previous one, so the decode takes at least
 * the steps times the latency of the dependent operations one step needs).
 * Runs one dependent chain per primitive on the current device and writes
 * shader cycles per link to h_out[0..11]:
 *   0 v_fma_f32, 1 4x4x1 FP32 MFMA, 2 16x16x4 FP32 MFMA (accumulator chains),
 *   3 LDS store then load by one wave, 4 LDS load (address chase),
 *   5 LDS flag hand-off between two waves (one way), 6 DPP reduction over 16
 *   lanes, 7 expf, 8 one rANS decode update, 9 ballot + popcount,
 *   10 flag hand-off between two workgroups through device memory (one way),
 *   11 v_readlane;
 * and h_out[12] = the shader clock in MHz over probe 0.  n >= DLIC_PROBE_COUNT.
 * d_ws: at least 256 bytes of device memory.  Synchronous: returns after the
 * probes ran (DLIC_ERR_TIMEOUT if a hand-off probe's bounded wait gave up). */
#define DLIC_PROBE_COUNT 13
dlic_status dlic_latency_probe(double *h_out, int32_t n, void *d_ws, size_t ws_bytes,
                               hipStream_t stream);

/* ---- retraining ------------------------------------------------------------ */

/* Scratch bytes of dlic_nll_fwd_bwd for n samples (d_ws). */
size_t dlic_nll_workspace(int64_t n, const dlic_model *model);

/* Mean discretised-logistic-mixture NLL in bits over n sampled pixels and its
 * gradient with respect to every weight (Section III-A: cross-entropy loss
 * in bits; Section IV: retraining on domain data).  d_slices: [n_slices][sh]
 * [sw] uint8 stack; d_idx: [n][3] int32 (slice, y, x), windows taken inside
 * the slice with the coding rule (dummy 0 outside); samples whose index lies
 * outside the stack contribute nothing.  model->dtype is DLIC_FP32 or
 * DLIC_FP64 (weights AND biases in that type; h1 == h2 in {32, 64}).
 * d_loss: one scalar of that type; d_grad: NULL for the loss only, else the
 * gradient in the concatenated layout W1, b1, W2, b2, W3, b3 (row-major).
 * The reduction over samples has a fixed order, so results are
 * deterministic. */
dlic_status dlic_nll_fwd_bwd(const dlic_model *model, const uint8_t *d_slices,
                             int32_t n_slices, int32_t sh, int32_t sw, const int32_t *d_idx,
                             int64_t n, void *d_loss, void *d_grad, void *d_ws,
                             size_t ws_bytes, hipStream_t stream);

/* One Adam step (Kingma and Ba) on n_params FP32 parameters in place:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr / (1 - b1^step) * m / (sqrt(v) / sqrt(1 - b2^step) + eps), with the
 * bias corrections evaluated in double on the host.  step >= 1. */
dlic_status dlic_adam_step(int64_t n_params, float *d_params, const float *d_grad, float *d_m,
                           float *d_v, int32_t step, float lr, float b1, float b2, float eps,
                           hipStream_t stream);

/* ---- measurement ---------------------------------------------------------- */

/* When enabled, every kernel launch of the library is bracketed by HIP
 * events on the stream it runs on.  dlic_kernel_times copies the durations
 * (ms) of the most recent call's launches, in launch order, and their
 * kernel names; it synchronises on those events.  Returns the count. */
void dlic_set_timing(int enable);
int dlic_kernel_times(float *h_ms, const char **h_names, int max_n);

/* When d_counters is non-NULL, later dlic_decode calls add shader-clock
 * cycle counts per group g to d_counters[16g .. 16g+15] (device, zeroed by
 * the caller): [0] coder waiting for densities, [1] coder busy, [2] density
 * waves waiting for decoded pixels (sum over waves), [3] density waves busy
 * (sum), and of that busy time [4] gather + network, [5] mixture head,
 * [6] bucket boundaries + publish, then [7] the number of tiles; of the
 * coder's busy time [8] from the densities' arrival to the start of the
 * symbol search, [9] the search itself, and [10] the group's sub-rounds;
 * [11] unused (0), [12] the coder's
 * wait at the first block of each step (with 16 lanes per pixel: its cycles
 * waiting for densities not ready when first read), [13] the coder loop's
 * shader-clock cycles and [14] its duration in 100 MHz real-time ticks, [15]
 * (16 lanes per pixel) the sub-rounds whose densities were not ready when
 * first read, low 32 bits, and of them those at block 0, high 32 bits.  NULL
 * turns it off. */
void dlic_set_decode_profile(unsigned long long *d_counters);

#ifdef __cplusplus
}
#endif

#endif /* DLIC_H */
