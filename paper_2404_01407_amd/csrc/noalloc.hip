// fnlh_residual_noalloc: the residual r = b - K_s x of fnlh_residual, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops).
// Its staging vectors, per-tile norm partials and reduction state live in one file-scope
// device array instead of context buffers allocated at first use; the kernels are
// fnlh_residual's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;

// The device array.  In host code `scratch` names a host-side stand-in, not device
// memory: only the address hipGetSymbolAddress returns for the current device is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

__global__ void k_copy_norm(const fnlh::SysState* __restrict__ st, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = st->last_n2;
}

}  // namespace

namespace fnlh {

// Device address of the scratch array on the context's device, looked up once per
// device with that device current (fnlh_create calls this after hipSetDevice).
int noalloc_init(fnlh_ctx c) {
  if (c->dev < 0 || c->dev >= kMaxDevices) return set_err(c, FNLH_E_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[c->dev]) return FNLH_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
  g_scratch[c->dev] = p;
  return FNLH_OK;
}

size_t noalloc_residual_bytes(const Layout& L, bool with_r) {
  const size_t vec = round256((size_t)L.NP * 12 * sizeof(double));
  return (with_r ? 3 : 2) * vec + round256((size_t)L.n_tiles * sizeof(double)) + round256(sizeof(SysState));
}

}  // namespace fnlh

using namespace fnlh;

extern "C" {

size_t fnlh_noalloc_scratch_bytes(void) { return kScratchBytes; }

int fnlh_residual_noalloc(fnlh_ctx c, int32_t sys, const double* x, const double* b, double* r, double* norm2,
                          void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "residual_noalloc: matrix and harmonics first");
  if (sys < 0 || sys >= c->n_sys) return set_err(c, FNLH_E_ARG, "residual_noalloc: system out of range");
  if (!x || !b) return set_err(c, FNLH_E_ARG, "residual_noalloc: null vector");
  const Layout& L = c->L;
  const size_t need = noalloc_residual_bytes(L, r != nullptr);
  if (need > kScratchBytes)
    return set_err(c, FNLH_E_ARG,
                   "residual_noalloc: mesh needs " + std::to_string(need) + " bytes of scratch, more than the " +
                       std::to_string(kScratchBytes) + " the library holds per device (at most about 233,000 cells)");
  unsigned char* base = (unsigned char*)g_scratch[c->dev];
  if (!base) return set_err(c, FNLH_E_ORDER, "residual_noalloc: scratch not set up for this device");
  hipStream_t s = (hipStream_t)stream;
  const size_t vec = round256((size_t)L.NP * 12 * sizeof(double));
  double* xi = (double*)base;
  double* bi = (double*)(base + vec);
  double* ri = r ? (double*)(base + 2 * vec) : nullptr;
  unsigned char* tail = base + (r ? 3 : 2) * vec;
  double* part = (double*)tail;
  SysState* st = (SysState*)(tail + round256((size_t)L.n_tiles * sizeof(double)));
  // every row of xi and bi is written (padding rows with 0), every tile's partial is
  // written by the residual kernel and the reduction sets last_n2: nothing left from an
  // earlier call is read
  DevPattern p = c->pat();
  launch_to_internal(p, (const int32_t*)c->iperm.p, x, xi, 12, 1, 0, s);
  launch_to_internal(p, (const int32_t*)c->iperm.p, b, bi, 12, 1, 0, s);
  if (c->is_frozen(sys)) launch_zero_sixth(L.NP, xi, 1, 0, s);
  SysBatch sb;
  sb.n = 1;
  sb.orow[0] = sys;
  sb.dslot[0] = 0;
  sb.vslot[0] = 0;
  outer_residual_of(c, 1, sb, xi, bi, ri, s, part);
  launch_reduce(sb, part, L.n_tiles, 0, L.n_tiles, 1, st, kReduceFinal, 0, 0, 0, s);
  if (r) launch_to_user(p, (const int32_t*)c->iperm.p, ri, r, 12, 1, 0, s);
  if (norm2) hipLaunchKernelGGL(k_copy_norm, dim3(1), dim3(64), 0, s, st, norm2);
  return check_launch(c, "residual_noalloc launch");
}

}  // extern "C"
