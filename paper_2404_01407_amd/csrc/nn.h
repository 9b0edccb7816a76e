// Learned preconditioner: device layouts and kernel launchers (nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

namespace fnlh {

// Padded layer shapes (in x out); the packed FP32 master order is W1..W5, each
// row-major [in][out] with the unpadded sizes below.
constexpr int kNnLayers = 5;
constexpr int kNnIn[kNnLayers] = {60, 88, 128, 128, 64};
constexpr int kNnOut[kNnLayers] = {64, 64, 64, 64, 12};
constexpr int kNnInPad[kNnLayers] = {64, 96, 128, 128, 64};
constexpr int kNnOutPad[kNnLayers] = {64, 64, 64, 64, 32};
constexpr int kNnParams = 60 * 64 + 88 * 64 + 128 * 64 + 128 * 64 + 64 * 12;  // 26624
constexpr int kNnPadded = 64 * 64 + 96 * 64 + 128 * 64 + 128 * 64 + 64 * 32;  // 28672
constexpr int kNnU = 32;  // node feature stride (24 used)

// offsets (in elements) of layer l in the packed and in the padded arrays
__host__ __device__ inline int nn_packed_off(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += kNnIn[k] * kNnOut[k];
  return o;
}
__host__ __device__ inline int nn_padded_off(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += kNnInPad[k] * kNnOutPad[k];
  return o;
}

// Device scalars of one feature pass.
struct NnScalars {
  double sumsq;  // sum |r|^2
  double sigma;  // RMS scale
  double den;    // sum |e / sigma|^2 (training)
  double loss;   // sum |d - e / sigma|^2 (training)
};

struct NnBufs {
  const uint16_t* wt = nullptr;  // bf16 transposed weights, [out_pad][in_pad] per layer
  const uint16_t* w = nullptr;   // bf16 weights, [in_pad][out_pad] per layer
  uint16_t* u = nullptr;         // node features [NP][32] bf16
  uint16_t* h = nullptr;         // layer-1 output [NP][64] bf16
  float* d = nullptr;            // decoder output [NP][16]
  float* ehat = nullptr;         // training target e / sigma [NP][16]
  float* dc = nullptr;           // d loss / d c (layer-2 aggregate) [NP][64]
  float* dh = nullptr;           // d loss / d h [NP][64]
  double* part = nullptr;        // per-tile partial sums [n_tiles]
  NnScalars* sc = nullptr;
  float* gpart = nullptr;        // weight-gradient partials [G][kNnPadded]
  double* lpart = nullptr;       // loss partials [G]
};

// A complex vector of one system: FP64 user order [N][12] (iperm maps internal rows to
// user cells), or internal [NP][ns][12] at slot vs in FP64 or BF16 (bit patterns).
struct NnVec {
  const double* d64 = nullptr;
  const uint16_t* b16 = nullptr;
  const int32_t* iperm = nullptr;
  int ns = 1, vs = 0;
};
// Output sigma * d: user order [N][12] when iperm is set, else internal [NP][ns][12] at
// slot vs; base (internal only, may be null) is added.
struct NnOut {
  double* out = nullptr;
  const double* base = nullptr;
  const int32_t* iperm = nullptr;
  int ns = 1, vs = 0;
};

void nn_launch_cast(const float* master, uint16_t* wt, uint16_t* w, hipStream_t s);
// sigma, node features u (and ehat, den when e is given and B.ehat is set)
void nn_launch_features(int storage, const DevPattern& p, const void* diag, int orow, const NnVec& r,
                        const NnVec* e, int64_t N, const NnBufs& B, bool pivot, hipStream_t s);
void nn_launch_forward(int storage, const DevPattern& p, const void* offd, const NnBufs& B, hipStream_t s);
void nn_launch_forward_l1(int storage, const DevPattern& p, const void* offd, const NnBufs& B, hipStream_t s);
void nn_launch_output(const DevPattern& p, const NnBufs& B, const NnOut& o, hipStream_t s);
// backward of one sample of a batch-mean loss (scale = 1 / batch): accumulates into
// B.gpart / B.lpart, which the caller clears once per batch.  Needs B.h from
// nn_launch_forward_l1 of the same sample.
void nn_launch_backward(int storage, const DevPattern& p, const void* offd, const NnBufs& B, int G, double scale,
                        hipStream_t s);
void nn_launch_grad_reduce(const NnBufs& B, int G, float* grad_packed, double* loss_out, hipStream_t s);
void nn_launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                    int t, hipStream_t s);
// sign x FP64 user-order vector -> BF16 internal [NP][12] (training pairs), and back to FP64
void nn_launch_pack16(const DevPattern& p, const int32_t* iperm, const double* user, double sign, uint16_t* out,
                      hipStream_t s);
void nn_launch_unpack16(const DevPattern& p, const int32_t* iperm, const uint16_t* in, double* user, hipStream_t s);
// Random starts of generated pairs: x[v] = 2 u - 1 with u = (mix(key + v) >> 11) 2^-53,
// key = nn_start_key(seed, start) = mix(seed + 0x9E3779B97F4A7C15 (start + 1)), mix the
// splitmix64 finaliser.
uint64_t nn_start_key(uint64_t seed, int64_t start);
void nn_launch_uniform(int64_t n, uint64_t key, double* x, hipStream_t s);
// learned step, per system slot vs: y = r - rn; alpha = <y, r> / <y, y> if that lowers
// ||r||^2 by at least the fraction accept and the system is active, else 0;
// x <- x + alpha (xt - x), r <- r - alpha y
void nn_launch_step(const DevPattern& p, double* x, const double* xt, double* r, const double* rn, int ns, int vs,
                    const SysState* st, double* part4, double* alpha, int* counts, double accept, hipStream_t s);
// MFMA self-check: C = A B for 64x64 bf16 operands held in device memory, one tile
void nn_launch_selftest(const uint16_t* a, const uint16_t* bt, float* c, hipStream_t s);

}  // namespace fnlh
