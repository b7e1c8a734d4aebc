// Launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dlic_device.hpp"

namespace dlic {

struct HeaderFields {
  int dtype, h1, h2;
  uint64_t fingerprint;
};

// Decoder limits: rows per group, and the per-group stream ring in LDS.
constexpr int DEC_RMAX = 256;
constexpr int DEC_RING = 4096;
constexpr int DEC_WAVES = 8;  // wave 0 codes, six of waves 1..7 compute densities

struct DecArgs {
  const uint8_t* bits;
  unsigned long long n_bytes;
  uint8_t* img;
  int H, W, G, L;
  uint32_t* rec;          // [G][T] progress records, cleared before launch
  long long T;            // wavefront steps W + 3H - 3
  int* status;
  uint32_t spin_limit;
  int check_model;        // compare header model fields with the ones below
  HeaderFields hf;
  const uint32_t* tables;  // table mode: [n_tables][257]
  int n_tables;
  const uint32_t* tidx;    // table mode: [H*W]
  unsigned long long* prof;  // optional per-group cycle counters (8 per group)
};

// wtype: WeightType of the model; width: h1 == h2.  False for an unsupported pair.
bool launch_density(int wtype, int width, const Consts* K, const DevModel& m, const uint8_t* img,
                    int H, int W, uint32_t* cf, float* out15, uint32_t* tables, int grid,
                    hipStream_t s);
void launch_rans_encode(const uint32_t* cf, int H, int W, int G, int L, uint16_t* words,
                        uint32_t* counts, hipStream_t s);
void launch_pack(const uint16_t* words, const uint32_t* counts, int H, int W, int G, int L,
                 const HeaderFields& hf, uint8_t* out, uint64_t* out_len, int chunks,
                 hipStream_t s);
bool launch_decode(int wtype, int width, bool tables_mode, const Consts* K, const DevModel& m,
                   const DecArgs& a, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t s);

// Training: waves per workgroup of the FP32 / FP64 loss-and-gradient kernel.
constexpr int TRAIN_WAVES_F32 = 4;
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
