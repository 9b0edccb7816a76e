// Vector kernels of the restarted flexible GMRES (the Krylov solve of include/fnlh.h):
// block inner products of one vector against several basis vectors, the matching
// multi-axpy, per-system scaling and the sweep-state set-up of a preconditioner call.
// Vectors are interleaved complex FP64 in the internal layout [NP][ns][12] (system slot
// vs); only the valid rows of each 64-row tile take part.  All of it is HBM-bound
// streaming work: each launch reads every vector it touches once, coalesced in 16-byte
// pieces, and reduces in a fixed order (deterministic results).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fnlh {
namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline bool row_valid(const int32_t* __restrict__ tile_nrows, int64_t row) {
  return (int)(row & 63) < tile_nrows[row >> 6];
}

// Thread mapping of every kernel here: work item (row, kk) with the system index kk of sb
// fastest, so consecutive lanes read consecutive 96-byte records of the interleaved rows
// (the systems of sb are usually all or most of the row's ns) and each vector is streamed
// from HBM once per launch, whatever the number of systems.

// partial[(blk * nq + (i0 + i) * nk + kk) * 2 + {0,1}] = sum over the block's rows of
// conj(V_{i0+i}) . w  for system kk of sb, i < cnt (cnt <= kMdot).  A block holds
// R = 256 / nk rows per step (threads t < R nk: kk = t % nk, row offset t / nk) and
// strides over the rows; the per-system sums are reduced through LDS in a fixed order.
__global__ void __launch_bounds__(256) k_mdot(int64_t NP, const int32_t* __restrict__ tile_nrows, int ns,
                                              const double* __restrict__ V, int64_t vstride, int i0, int cnt,
                                              const double* __restrict__ w, SysBatch sb, int nq,
                                              double* __restrict__ partial) {
  const int nk = sb.n;
  const int R = 256 / nk;
  const int t = threadIdx.x;
  const bool act = t < R * nk;
  const int kk = act ? t % nk : 0;
  const int vs = sb.vslot[kk];
  double ar[kMdot], ai[kMdot];
#pragma unroll
  for (int i = 0; i < kMdot; ++i) ar[i] = ai[i] = 0.0;
  if (act) {
    for (int64_t row = (int64_t)blockIdx.x * R + t / nk; row < NP; row += (int64_t)gridDim.x * R) {
      if (!row_valid(tile_nrows, row)) continue;
      const int64_t o = (row * ns + vs) * 12;
      double2 wv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) wv[c] = ((const double2*)(w + o))[c];
#pragma unroll
      for (int i = 0; i < kMdot; ++i) {
        if (i >= cnt) break;
        const double2* vp = (const double2*)(V + (int64_t)(i0 + i) * vstride + o);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double2 v = vp[c];
          ar[i] += v.x * wv[c].x + v.y * wv[c].y;
          ai[i] += v.x * wv[c].y - v.y * wv[c].x;
        }
      }
    }
  }
  __shared__ double sh[2 * kMdot][256];
#pragma unroll
  for (int i = 0; i < kMdot; ++i) {
    sh[2 * i][t] = ar[i];
    sh[2 * i + 1][t] = ai[i];
  }
  __syncthreads();
  // thread q < 2 cnt nk sums value (i, part) of system kk over the block's R rows
  if (t < 2 * cnt * nk) {
    const int kq = t % nk, v = t / nk;  // v = 2 i + part
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc += sh[v][r * nk + kq];
    const int i = v >> 1, part = v & 1;
    partial[((int64_t)blockIdx.x * nq + (int64_t)(i0 + i) * nk + kq) * 2 + part] = acc;
  }
}

// out[q] = sum over blocks of partial[blk][q] (complex, q < nq), blocks in order
__global__ void __launch_bounds__(256) k_mreduce(const double* __restrict__ partial, int nblk, int nq,
                                                 double* __restrict__ out) {
  const int q = blockIdx.x;
  double r = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    r += partial[((int64_t)b * nq + q) * 2];
    im += partial[((int64_t)b * nq + q) * 2 + 1];
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = r;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sr[threadIdx.x] += sr[threadIdx.x + o];
      si[threadIdx.x] += si[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * q] = sr[0];
    out[2 * q + 1] = si[0];
  }
}

// w = w + sgn * sum_{i < cnt} coef[i * nk + kk] V_i  (complex coefficients, system kk of sb)
__global__ void __launch_bounds__(256) k_maxpy(int64_t NP, const int32_t* __restrict__ tile_nrows, int ns,
                                               double* __restrict__ w, const double* __restrict__ V, int64_t vstride,
                                               int cnt, const double* __restrict__ coef, double sgn, SysBatch sb) {
  const int nk = sb.n;
  const int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = item / nk;
  const int kk = (int)(item - row * nk);
  if (row >= NP || !row_valid(tile_nrows, row)) return;
  const int vs = sb.vslot[kk];
  const int64_t o = (row * ns + vs) * 12;
  double2 acc[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = ((const double2*)(w + o))[c];
  for (int i = 0; i < cnt; ++i) {
    const double cr = sgn * coef[2 * (i * nk + kk)], ci = sgn * coef[2 * (i * nk + kk) + 1];
    const double2* vp = (const double2*)(V + (int64_t)i * vstride + o);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double2 v = vp[c];
      acc[c].x += cr * v.x - ci * v.y;
      acc[c].y += cr * v.y + ci * v.x;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) ((double2*)(w + o))[c] = acc[c];
}

// dst = scale[kk] * src for system kk of sb (dst may be src)
__global__ void __launch_bounds__(256) k_mscale(int64_t NP, const int32_t* __restrict__ tile_nrows, int ns,
                                                double* dst, const double* src, KScale sc, SysBatch sb) {
  const int nk = sb.n;
  const int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = item / nk;
  const int kk = (int)(item - row * nk);
  if (row >= NP || !row_valid(tile_nrows, row)) return;
  const int vs = sb.vslot[kk];
  const int64_t o = (row * ns + vs) * 12;
  const double a = sc.s[kk];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double2 v = ((const double2*)(src + o))[c];
    v.x *= a;
    v.y *= a;
    ((double2*)(dst + o))[c] = v;
  }
}

// sweep states of a preconditioner application: active, ||r0||^2 = n2, `limit` sweeps
__global__ void k_kstate(SysBatch sb, SysState* __restrict__ st, double n2, int limit) {
  const int k = threadIdx.x;
  if (k >= sb.n) return;
  SysState S;
  S.norm0sq = n2;
  S.last_n2 = n2;
  S.active = limit > 0 ? 1 : 0;
  S.pending = 0;
  S.sweeps = 0;
  S.status = 1;  // not converged
  S.limit = limit;
  S.outer_iters = 0;
  S.hist = nullptr;  // preconditioner sweeps keep no residual history
  S.hist_len = 0;
  S.hist_off = 0;
  st[sb.vslot[k]] = S;
}

inline unsigned item_blocks(int64_t NP, int nk) { return (unsigned)((NP * nk + 255) / 256); }

}  // namespace

int mdot_blocks(int64_t NP) {
  const int64_t b = (NP + 15) / 16;  // at least 16 rows per block (16 systems fill it)
  return (int)(b < kMdotBlocks ? b : kMdotBlocks);
}

void launch_mdot(const DevPattern& p, int ns, const double* V, int64_t vstride, int nv, const double* w,
                 const SysBatch& sb, int nq, double* partial, double* out, hipStream_t s) {
  if (sb.n <= 0 || nv <= 0) return;
  const int nb = mdot_blocks(p.NP);
  for (int i0 = 0; i0 < nv; i0 += kMdot) {
    const int cnt = nv - i0 < kMdot ? nv - i0 : kMdot;
    hipLaunchKernelGGL(k_mdot, dim3((unsigned)nb), dim3(256), 0, s, p.NP, p.tile_nrows, ns, V,
                       vstride, i0, cnt, w, sb, nq, partial);
  }
  hipLaunchKernelGGL(k_mreduce, dim3((unsigned)(nv * sb.n)), dim3(256), 0, s, partial, nb, nq, out);
}

void launch_maxpy(const DevPattern& p, int ns, double* w, const double* V, int64_t vstride, int nv,
                  const double* coef, double sgn, const SysBatch& sb, hipStream_t s) {
  if (sb.n <= 0 || nv <= 0) return;
  hipLaunchKernelGGL(k_maxpy, dim3(item_blocks(p.NP, sb.n)), dim3(256), 0, s, p.NP, p.tile_nrows, ns, w, V,
                     vstride, nv, coef, sgn, sb);
}

void launch_mscale(const DevPattern& p, int ns, double* dst, const double* src, const KScale& sc, const SysBatch& sb,
                   hipStream_t s) {
  if (sb.n <= 0) return;
  hipLaunchKernelGGL(k_mscale, dim3(item_blocks(p.NP, sb.n)), dim3(256), 0, s, p.NP, p.tile_nrows, ns, dst,
                     src, sc, sb);
}

void launch_kstate(const SysBatch& sb, SysState* st, double n2, int limit, hipStream_t s) {
  if (sb.n <= 0) return;
  hipLaunchKernelGGL(k_kstate, dim3(1), dim3(64), 0, s, sb, st, n2, limit);
}

}  // namespace fnlh
