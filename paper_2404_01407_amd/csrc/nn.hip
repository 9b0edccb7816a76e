// Learned preconditioner on gfx950: a two-layer per-edge message-passing network with
// BF16 weights and activations and FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16).  Forward, backward (by recomputation) and Adam; no
// floating-point atomics: weight gradients are per-workgroup partials summed in a fixed
// order.
//
// Network (per cell i, coupling i <- j; complex values as (re, im) pairs):
//   u_i = [r_i, z_i] / sigma (24),  z_i = (K_ii + i w_i I)^-1 r_i,  g_ij = K_ij z_j / sigma
//   m_ij = relu(W1^T [u_i; u_j; g_ij]),  a_i = sum_j m_ij,  h_i = relu(W2^T [u_i; a_i])
//   p_ij = relu(W3^T [h_i; h_j]),        c_i = sum_j p_ij,  q_i = relu(W4^T [h_i; c_i])
//   d_i = W5^T q_i (12),  dx_i = sigma d_i
//
// Tiles are the sweep kernels' 64-row tiles; a workgroup of four waves handles one tile,
// wave w owning rows 16w..16w+15 of every 64 x N product.  Matrix-core operand layout
// (16x16x32): lane l supplies A[l % 16][8 (l / 16) + t] and B[8 (l / 16) + t][l % 16],
// t = 0..7, and receives D[4 (l / 16) + i][l % 16], i = 0..3.
#include "device.h"
#include "nn.h"

namespace fnlh {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline f32x4 mfma(const u16x8 a, const u16x8 b, const f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

__device__ inline int ln() { return threadIdx.x & 63; }
__device__ inline int wv() { return threadIdx.x >> 6; }
// element (row, col) of output tile nt held by this lane, item i
__device__ inline int orow(int i) { return 16 * wv() + 4 * (ln() >> 4) + i; }
__device__ inline int ocol(int nt) { return nt * 16 + (ln() & 15); }

// acc[nt] += A[rows of this wave][0..K) x B[0..K)[16 (nt0 + nt) ..], with Bt[n][k] = B[k][n]
template <int K, int NT>
__device__ inline void mm_rows(const uint16_t* A, int lda, const uint16_t* Bt, int ldb, int nt0, f32x4 (&acc)[NT]) {
  const int l = ln();
#pragma unroll
  for (int kk = 0; kk < K; kk += 32) {
    const u16x8 a = *(const u16x8*)(A + (16 * wv() + (l & 15)) * lda + kk + 8 * (l >> 4));
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const u16x8 b = *(const u16x8*)(Bt + ((nt0 + nt) * 16 + (l & 15)) * ldb + kk + 8 * (l >> 4));
      acc[nt] = mfma(a, b, acc[nt]);
    }
  }
}

// acc[nt] += sum over the 64 tile rows r of X[r][16 mt + m] * D[r][16 nt + n]  (weight
// gradient X^T D), with Dt[n][r] = D[r][n]
template <int NT>
__device__ inline void mm_wgrad(const uint16_t* X, int ldx, int mt, const uint16_t* Dt, int ldd, f32x4 (&acc)[NT]) {
  const int l = ln();
#pragma unroll
  for (int kk = 0; kk < 64; kk += 32) {
    u16x8 a;
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] = X[(kk + 8 * (l >> 4) + t) * ldx + 16 * mt + (l & 15)];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const u16x8 b = *(const u16x8*)(Dt + (nt * 16 + (l & 15)) * ldd + kk + 8 * (l >> 4));
      acc[nt] = mfma(a, b, acc[nt]);
    }
  }
}

template <int NT> __device__ inline void zero(f32x4 (&a)[NT]) {
#pragma unroll
  for (int k = 0; k < NT; ++k) a[k] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// cooperative 16-byte copy global -> LDS (n uint16, multiple of 8)
__device__ inline void copy_lds(uint16_t* dst, const uint16_t* src, int n) {
  for (int i = threadIdx.x; i < n / 8; i += blockDim.x) ((uint4*)dst)[i] = ((const uint4*)src)[i];
}

// LDS row strides (uint16) of the 32-, 64-, 96- and 128-wide tiles: 16 bytes more than
// the row, so the 16 rows that one 16-byte operand read of mm_rows / mm_wgrad touches
// start 4 banks apart and cover the 64 banks once (a stride of 128 or 256 bytes puts
// them all on the same banks)
constexpr int kL32 = 40, kL64 = 72, kL96 = 104, kL128 = 136;

// copy a [rows][cols] matrix (cols a multiple of 8, row-contiguous in global memory)
// into LDS rows of stride ld
__device__ inline void copy_lds_rows(uint16_t* dst, int ld, const uint16_t* src, int rows, int cols) {
  const int cpr = cols / 8;
  for (int i = threadIdx.x; i < rows * cpr; i += blockDim.x) {
    const int r = i / cpr, c = (i - r * cpr) * 8;
    *(uint4*)(dst + r * ld + c) = *(const uint4*)(src + (int64_t)r * cols + c);
  }
}

// store an MFMA output (64 x 16 NT) to LDS as bf16, optionally transposed ([col][row])
template <int NT>
__device__ inline void put(uint16_t* S, int ld, int col0, const f32x4 (&v)[NT], bool transposed) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = orow(i), c = col0 + ocol(nt);
      if (transposed)
        S[c * ld + r] = f2bf(v[nt][i]);
      else
        S[r * ld + c] = f2bf(v[nt][i]);
    }
}

// ---------------------------------------------------------------- weights
__global__ void k_nn_cast(const float* __restrict__ master, uint16_t* __restrict__ wt, uint16_t* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNnPadded) return;
  int l = 0, o = t;
  while (o >= kNnInPad[l] * kNnOutPad[l]) {
    o -= kNnInPad[l] * kNnOutPad[l];
    ++l;
  }
  const int i = o / kNnOutPad[l], j = o % kNnOutPad[l];  // W[i][j] in [in_pad][out_pad]
  float v = 0.f;
  if (i < kNnIn[l] && j < kNnOut[l]) v = master[nn_packed_off(l) + i * kNnOut[l] + j];
  const uint16_t b = f2bf(v);
  w[nn_padded_off(l) + i * kNnOutPad[l] + j] = b;
  wt[nn_padded_off(l) + j * kNnInPad[l] + i] = b;
}

// ---------------------------------------------------------------- features
__device__ inline double nv_get(const NnVec& v, int64_t row, int c) {
  if (v.iperm) {
    const int32_t u = v.iperm[row];
    return u < 0 ? 0.0 : v.d64[(int64_t)u * 12 + c];
  }
  const int64_t o = (row * v.ns + v.vs) * 12 + c;
  return v.d64 ? v.d64[o] : (double)bf2f(v.b16[o]);
}

// sum |r|^2 per tile
__global__ void k_nn_sumsq(DevPattern p, NnVec r, double* __restrict__ part) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = tile * 64 + lane;
  double s = 0.0;
  if (lane < p.tile_nrows[tile])
    for (int c = 0; c < 12; ++c) {
      const double v = nv_get(r, row, c);
      s += v * v;
    }
  s = wave_sum(s);
  if (lane == 0) part[tile] = s;
}

// which = 0: sigma from sum |r|^2; which = 1: den from the ehat partials
__global__ void k_nn_finalize(const double* __restrict__ part, int64_t n, int64_t N, NnScalars* sc, int which) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x) return;
  if (which == 0) {
    sc->sumsq = sh[0];
    const double sg = sqrt(sh[0] / (12.0 * (double)N));
    sc->sigma = sg > 0.0 ? sg : 1.0;
    sc->loss = 0.0;
  } else {
    sc->den = sh[0] > 0.0 ? sh[0] : 1.0;
  }
}

template <typename TB>
__global__ void k_nn_feat(DevPattern p, const TB* __restrict__ diag, int orow_sys, NnVec rv, NnVec ev, int has_e,
                          NnBufs B, bool pivot) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = tile * 64 + lane;
  const bool valid = lane < p.tile_nrows[tile];
  const double is = 1.0 / B.sc->sigma;
  float r[12], z[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    r[c] = valid ? (float)(nv_get(rv, row, c) * is) : 0.f;
    z[c] = r[c];
  }
  float d[36];
  load_block(diag + tile * slot_elems<TB>(), lane, d);
  const float w = (float)(p.omega[(int64_t)orow_sys * p.n_zones + p.zone[row]] * p.vol[row]);
  if (valid) {
    // z = (K_ii + i w I)^-1 r: complex elimination with partial pivoting
    float mr[36], mi[36];
#pragma unroll
    for (int c2 = 0; c2 < 36; ++c2) {
      mr[c2] = d[c2];
      mi[c2] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) mi[7 * k] = w;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float best = mr[7 * k] * mr[7 * k] + mi[7 * k] * mi[7 * k];
      int pv = k;
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const float m = mr[6 * i + k] * mr[6 * i + k] + mi[6 * i + k] * mi[6 * i + k];
        if (pivot && m > best) {
          best = m;
          pv = i;
        }
      }
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const bool sw = pv == i;
#pragma unroll
        for (int c2 = k; c2 < 6; ++c2) {
          const float ar = mr[6 * k + c2], ai = mi[6 * k + c2], br = mr[6 * i + c2], bi = mi[6 * i + c2];
          mr[6 * k + c2] = sw ? br : ar;
          mi[6 * k + c2] = sw ? bi : ai;
          mr[6 * i + c2] = sw ? ar : br;
          mi[6 * i + c2] = sw ? ai : bi;
        }
        const float xr = z[2 * k], xi = z[2 * k + 1], yr = z[2 * i], yi = z[2 * i + 1];
        z[2 * k] = sw ? yr : xr;
        z[2 * k + 1] = sw ? yi : xi;
        z[2 * i] = sw ? xr : yr;
        z[2 * i + 1] = sw ? xi : yi;
      }
      const float pr = mr[7 * k], pim = mi[7 * k];
      const float rd = 1.f / (pr * pr + pim * pim);
      const float ivr = pr * rd, ivi = -pim * rd;
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const float ar = mr[6 * i + k], ai = mi[6 * i + k];
        const float fr = ar * ivr - ai * ivi, fi = ar * ivi + ai * ivr;
#pragma unroll
        for (int c2 = k + 1; c2 < 6; ++c2) {
          mr[6 * i + c2] -= fr * mr[6 * k + c2] - fi * mi[6 * k + c2];
          mi[6 * i + c2] -= fr * mi[6 * k + c2] + fi * mr[6 * k + c2];
        }
        z[2 * i] -= fr * z[2 * k] - fi * z[2 * k + 1];
        z[2 * i + 1] -= fr * z[2 * k + 1] + fi * z[2 * k];
      }
      mr[7 * k] = ivr;  // keep the pivot inverse on the diagonal
      mi[7 * k] = ivi;
    }
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      float sr = z[2 * k], si = z[2 * k + 1];
#pragma unroll
      for (int c2 = k + 1; c2 < 6; ++c2) {
        sr -= mr[6 * k + c2] * z[2 * c2] - mi[6 * k + c2] * z[2 * c2 + 1];
        si -= mr[6 * k + c2] * z[2 * c2 + 1] + mi[6 * k + c2] * z[2 * c2];
      }
      z[2 * k] = sr * mr[7 * k] - si * mi[7 * k];
      z[2 * k + 1] = sr * mi[7 * k] + si * mr[7 * k];
    }
  }
  uint16_t* u = B.u + row * kNnU;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    u[c] = f2bf(r[c]);
    u[12 + c] = f2bf(z[c]);
  }
#pragma unroll
  for (int c = 24; c < 32; ++c) u[c] = 0;
  if (has_e) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const float e = valid ? (float)(nv_get(ev, row, c) * is) : 0.f;
      B.ehat[row * 16 + c] = e;
      s += (double)e * e;
    }
#pragma unroll
    for (int c = 12; c < 16; ++c) B.ehat[row * 16 + c] = 0.f;
    s = wave_sum(s);
    if (lane == 0) B.part[tile] = s;
  }
}

// ---------------------------------------------------------------- forward pieces
// edge input row of layer 1 for (tile row t, slot q): [u_i; u_j; K_ij z_j/sigma; 0],
// zeros where row t has no edge in this slot (one thread per row)
template <typename TB>
__device__ inline void l1_row(const DevPattern& p, const TB* __restrict__ offd, const uint16_t* __restrict__ u,
                              int64_t tile, int q, int t, uint16_t* X) {
  const int64_t s0 = p.tile_slot0[tile];
  const int64_t f = (s0 + q) * 64 + t;
  uint16_t* x = X + t * kL64;
  if (t >= p.tile_nrows[tile] || p.ent_edge[f] == 0) {
#pragma unroll
    for (int c = 0; c < 64; c += 8) *(uint4*)(x + c) = make_uint4(0, 0, 0, 0);
    return;
  }
  const int64_t row = tile * 64 + t;
  const int nb = p.ent_nbr[f];
  const uint16_t* ui = u + row * kNnU;
  const uint16_t* uj = u + (int64_t)nb * kNnU;
#pragma unroll
  for (int c = 0; c < 24; c += 8) {
    *(uint4*)(x + c) = *(const uint4*)(ui + c);
    *(uint4*)(x + 24 + c) = *(const uint4*)(uj + c);
  }
  float kb[36];
  load_block(offd + (s0 + q) * slot_elems<TB>(), t, kb);
  float zj[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) zj[c] = bf2f(uj[12 + c]);
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    float gr = 0.f, gi = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      gr += kb[6 * r + c] * zj[2 * c];
      gi += kb[6 * r + c] * zj[2 * c + 1];
    }
    x[48 + 2 * r] = f2bf(gr);
    x[49 + 2 * r] = f2bf(gi);
  }
#pragma unroll
  for (int c = 60; c < 64; ++c) x[c] = 0;
}

// layer-2 edge input row, built by the whole workgroup (256 threads), four threads per
// tile row (t = threadIdx.x / 4, part = threadIdx.x % 4), each copying 32 of the 128
// values: [h_i; h_j] (self_first) or [h_j; h_i], zeros where row t has no edge in this slot
__device__ inline void l2_row(const DevPattern& p, const uint16_t* __restrict__ h, int64_t tile, int q, uint16_t* X,
                              bool self_first) {
  const int t = threadIdx.x >> 2, part = threadIdx.x & 3;
  const int64_t f = (p.tile_slot0[tile] + q) * 64 + t;
  uint16_t* x = X + t * kL128 + 32 * part;
  if (t >= p.tile_nrows[tile] || p.ent_edge[f] == 0) {
#pragma unroll
    for (int c = 0; c < 32; c += 8) *(uint4*)(x + c) = make_uint4(0, 0, 0, 0);
    return;
  }
  const int64_t src = ((part < 2) == self_first) ? tile * 64 + t : (int64_t)p.ent_nbr[f];
  const uint16_t* hs = h + src * 64 + 32 * (part & 1);
#pragma unroll
  for (int c = 0; c < 32; c += 8) *(uint4*)(x + c) = *(const uint4*)(hs + c);
}

// layer 1 of one tile: returns pre-activation of h (pre1) and leaves Y1 = [u; a] in sY
template <typename TB>
__device__ inline void l1_tile(const DevPattern& p, const TB* __restrict__ offd, const uint16_t* __restrict__ u,
                               const uint16_t* W1t, int ldw1, const uint16_t* W2t, int ldw2, int64_t tile,
                               uint16_t* sX, uint16_t* sY,
                               f32x4 (&pre1)[4], f32x4* pre_m_slot = nullptr) {
  f32x4 agg[4];
  zero(agg);
  const int wd = p.tile_width[tile];
  for (int q = 0; q < wd; ++q) {
    __syncthreads();
    if (threadIdx.x < 64) l1_row<TB>(p, offd, u, tile, q, threadIdx.x, sX);
    __syncthreads();
    f32x4 acc[4];
    zero(acc);
    mm_rows<64, 4>(sX, kL64, W1t, ldw1, 0, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) agg[nt][i] += fmaxf(acc[nt][i], 0.f);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint16_t* ui = u + (tile * 64 + threadIdx.x) * kNnU;
    uint16_t* y = sY + threadIdx.x * kL96;
#pragma unroll
    for (int c = 0; c < 24; c += 8) *(uint4*)(y + c) = *(const uint4*)(ui + c);
#pragma unroll
    for (int c = 88; c < 96; ++c) y[c] = 0;
  }
  put<4>(sY, kL96, 24, agg, false);
  __syncthreads();
  zero(pre1);
  mm_rows<96, 4>(sY, kL96, W2t, ldw2, 0, pre1);
}

// layer 2 + decoder of one tile: returns pre2 (pre-activation of q); on exit sX holds
// Y2 = [h_i; c] and sQ holds q.  d (decoder, 16 columns) in dout.
__device__ inline void l2_tile(const DevPattern& p, const uint16_t* __restrict__ h, const uint16_t* W3t, int ldw3,
                               const uint16_t* W4t, int ldw4, const uint16_t* W5t, int ldw5, int64_t tile,
                               uint16_t* sX, uint16_t* sQ,
                               f32x4 (&pre2)[4], f32x4 (&dout)[1]) {
  f32x4 agg[4];
  zero(agg);
  const int wd = p.tile_width[tile];
  for (int q = 0; q < wd; ++q) {
    __syncthreads();
    l2_row(p, h, tile, q, sX, true);
    __syncthreads();
    f32x4 acc[4];
    zero(acc);
    mm_rows<128, 4>(sX, kL128, W3t, ldw3, 0, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) agg[nt][i] += fmaxf(acc[nt][i], 0.f);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint16_t* hs = h + (tile * 64 + threadIdx.x) * 64;
    uint16_t* x = sX + threadIdx.x * kL128;
#pragma unroll
    for (int c = 0; c < 64; c += 8) *(uint4*)(x + c) = *(const uint4*)(hs + c);
  }
  put<4>(sX, kL128, 64, agg, false);
  __syncthreads();
  zero(pre2);
  mm_rows<128, 4>(sX, kL128, W4t, ldw4, 0, pre2);
  f32x4 qv[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) qv[nt][i] = fmaxf(pre2[nt][i], 0.f);
  put<4>(sQ, kL64, 0, qv, false);
  __syncthreads();
  zero(dout);
  mm_rows<64, 1>(sQ, kL64, W5t, ldw5, 0, dout);
}

// weight pointers inside the padded layouts
__device__ inline const uint16_t* WT(const NnBufs& B, int l) { return B.wt + nn_padded_off(l); }
__device__ inline const uint16_t* WW(const NnBufs& B, int l) { return B.w + nn_padded_off(l); }

template <typename TB>
__global__ void __launch_bounds__(256) k_nn_l1_fwd(DevPattern p, const TB* __restrict__ offd, NnBufs B) {
  __shared__ __attribute__((aligned(16))) uint16_t sW1[64 * kL64], sW2[64 * kL96], sX[64 * kL64], sY[64 * kL96];
  copy_lds_rows(sW1, kL64, WT(B, 0), 64, 64);
  copy_lds_rows(sW2, kL96, WT(B, 1), 64, 96);
  const int64_t tile = blockIdx.x;
  f32x4 pre1[4];
  l1_tile<TB>(p, offd, B.u, sW1, kL64, sW2, kL96, tile, sX, sY, pre1);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      B.h[(tile * 64 + orow(i)) * 64 + ocol(nt)] = f2bf(fmaxf(pre1[nt][i], 0.f));
}

__global__ void __launch_bounds__(256) k_nn_l2_fwd(DevPattern p, NnBufs B) {
  // W3 (read once per slot) and W5 in LDS; W4 (once per tile) from the cache, which
  // leaves room for three workgroups per CU
  __shared__ __attribute__((aligned(16))) uint16_t sW3[64 * kL128], sW5[16 * kL64], sX[64 * kL128],
      sQ[64 * kL64];
  copy_lds_rows(sW3, kL128, WT(B, 2), 64, 128);
  copy_lds_rows(sW5, kL64, WT(B, 4), 16, 64);  // the 16 (12 used) decoder outputs
  const int64_t tile = blockIdx.x;
  f32x4 pre2[4], dout[1];
  l2_tile(p, B.h, sW3, kL128, WT(B, 3), 128, sW5, kL64, tile, sX, sQ, pre2, dout);
#pragma unroll
  for (int i = 0; i < 4; ++i) B.d[(tile * 64 + orow(i)) * 16 + ocol(0)] = dout[0][i];
}

__global__ void k_nn_output(int64_t NP, NnBufs B, NnOut o) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * 12) return;
  const int64_t row = t / 12;
  const int c = (int)(t % 12);
  const double v = B.sc->sigma * (double)B.d[row * 16 + c];
  if (o.iperm) {
    const int32_t u = o.iperm[row];
    if (u >= 0) o.out[(int64_t)u * 12 + c] = v;
  } else {
    const int64_t k = (row * o.ns + o.vs) * 12 + c;
    o.out[k] = (o.base ? o.base[k] : 0.0) + v;
  }
}

// BF16 keeps the exponent range of FP32, so pairs need no scaling (the loss is
// scale-free as long as r and e share one factor)
__global__ void k_nn_pack16(int64_t NP, const int32_t* __restrict__ iperm, const double* __restrict__ user,
                            double sign, uint16_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * 12) return;
  const int32_t u = iperm[t / 12];
  out[t] = u < 0 ? (uint16_t)0 : f2bf((float)(sign * user[(int64_t)u * 12 + t % 12]));
}

// stored BF16 pair vector (internal order) -> FP64 user order
__global__ void k_nn_unpack16(int64_t NP, const int32_t* __restrict__ iperm, const uint16_t* __restrict__ in,
                              double* __restrict__ user) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * 12) return;
  const int32_t u = iperm[t / 12];
  if (u >= 0) user[(int64_t)u * 12 + t % 12] = (double)bf2f(in[t]);
}

// splitmix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014)
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// x[v] = 2 u - 1, u = (mix64(key + v) >> 11) 2^-53 uniform on [0, 1): counter-based, so
// any value can be recomputed on its own
__global__ void k_nn_uniform(int64_t n, uint64_t key, double* __restrict__ x) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double u = (double)(mix64(key + (uint64_t)v) >> 11) * 0x1.0p-53;
  x[v] = 2.0 * u - 1.0;
}

// learned step: partial sums per tile of <y, r> (re, im), |y|^2, |r|^2 with y = r - rn
__global__ void k_nn_dots(DevPattern p, const double* __restrict__ r, const double* __restrict__ rn, int ns, int vs,
                          double* __restrict__ part) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = tile * 64 + lane;
  double are = 0.0, aim = 0.0, yy = 0.0, rr = 0.0;
  if (lane < p.tile_nrows[tile]) {
    const double* a = r + (row * ns + vs) * 12;
    const double* b = rn + (row * ns + vs) * 12;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double xr = a[2 * k], xi = a[2 * k + 1];
      const double yr = xr - b[2 * k], yi = xi - b[2 * k + 1];
      are += yr * xr + yi * xi;  // conj(y) r
      aim += yr * xi - yi * xr;
      yy += yr * yr + yi * yi;
      rr += xr * xr + xi * xi;
    }
  }
  are = wave_sum(are);
  aim = wave_sum(aim);
  yy = wave_sum(yy);
  rr = wave_sum(rr);
  if (lane == 0) {
    part[tile * 4 + 0] = are;
    part[tile * 4 + 1] = aim;
    part[tile * 4 + 2] = yy;
    part[tile * 4 + 3] = rr;
  }
}

__global__ void k_nn_alpha(const double* __restrict__ part, int64_t n_tiles, const SysState* st, int vs,
                           double* __restrict__ alpha, int* __restrict__ counts, double accept) {
  __shared__ double sh[4][256];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t = threadIdx.x; t < n_tiles; t += 256)
    for (int k = 0; k < 4; ++k) a[k] += part[t * 4 + k];
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x) return;
  double ar = 0.0, ai = 0.0;
  if (st[vs].active) {
    const double are = sh[0][0], aim = sh[1][0], yy = sh[2][0], rr = sh[3][0];
    // ||r - alpha y||^2 = rr - |<y, r>|^2 / yy at the optimum
    const double gain = (yy > 0.0 && rr > 0.0) ? (are * are + aim * aim) / (yy * rr) : 0.0;
    const bool ok = isfinite(are) && isfinite(aim) && isfinite(yy) && gain >= accept;
    if (ok) {
      ar = are / yy;
      ai = aim / yy;
      counts[2 * vs] += 1;
    } else {
      counts[2 * vs + 1] += 1;
    }
  }
  alpha[2 * vs] = ar;
  alpha[2 * vs + 1] = ai;
}

__global__ void k_nn_update(int64_t NP, double* __restrict__ x, const double* __restrict__ xt, double* __restrict__ r,
                            const double* __restrict__ rn, int ns, int vs, const double* __restrict__ alpha) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * 6) return;
  const double ar = alpha[2 * vs], ai = alpha[2 * vs + 1];
  if (ar == 0.0 && ai == 0.0) return;
  const int64_t k = ((t / 6) * ns + vs) * 12 + 2 * (t % 6);
  const double dr = xt[k] - x[k], di = xt[k + 1] - x[k + 1];
  x[k] += ar * dr - ai * di;
  x[k + 1] += ar * di + ai * dr;
  if (r) {
    const double yr = r[k] - rn[k], yi = r[k + 1] - rn[k + 1];
    r[k] -= ar * yr - ai * yi;
    r[k + 1] -= ar * yi + ai * yr;
  }
}

// ---------------------------------------------------------------- backward
// Layer 2 (receiver side) + decoder: dW5, dW4, dW3 (receiver rows), dc, dh (part)
__global__ void __launch_bounds__(256) k_nn_l2_bwd(DevPattern p, NnBufs B, int G, float scale) {
  __shared__ __attribute__((aligned(16))) uint16_t sX[64 * kL128], sQ[64 * kL64], sDD[64 * kL32],
      sDDt[16 * kL64], sDP[64 * kL64], sDPt[64 * kL64];
  const int w = wv();
  f32x4 g5[1], g4[2][4], g3[2][4];
  zero(g5);
  for (int k = 0; k < 2; ++k) {
    zero(g4[k]);
    zero(g3[k]);
  }
  double lsum = 0.0;
  const float den = (float)B.sc->den;
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += G) {
    f32x4 pre2[4], dout[1];
    l2_tile(p, B.h, WT(B, 2), 128, WT(B, 3), 128, WT(B, 4), 64, tile, sX, sQ, pre2, dout);
    // loss and dd = 2 (d - ehat) scale / den on the 12 used columns
    f32x4 dd[1];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = tile * 64 + orow(i);
      const int c = ocol(0);
      float v = 0.f;
      if (c < 12 && orow(i) < p.tile_nrows[tile]) {
        const float diff = dout[0][i] - B.ehat[row * 16 + c];
        lsum += (double)diff * diff;
        v = 2.f * diff * scale / den;
      }
      dd[0][i] = v;
    }
    __syncthreads();
    // sDD [64][32]: dd in columns 0..15, zeros in 16..31
    for (int k = threadIdx.x; k < 64 * kL32; k += 256) sDD[k] = 0;
    __syncthreads();
    put<1>(sDD, kL32, 0, dd, false);
    put<1>(sDDt, kL64, 0, dd, true);
    __syncthreads();
    mm_wgrad<1>(sQ, kL64, w, sDDt, kL64, g5);  // dW5[m][n], m = 16 w + .., n = 0..15
    f32x4 dq[4];
    zero(dq);
    mm_rows<32, 4>(sDD, kL32, WW(B, 4), 32, 0, dq);  // dq = dd W5^T
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) dq[nt][i] = pre2[nt][i] > 0.f ? dq[nt][i] : 0.f;
    put<4>(sDP, kL64, 0, dq, false);
    put<4>(sDPt, kL64, 0, dq, true);
    __syncthreads();
    mm_wgrad<4>(sX, kL128, w, sDPt, kL64, g4[0]);  // dW4 rows 16w.. (h part)
    mm_wgrad<4>(sX, kL128, w + 4, sDPt, kL64, g4[1]);  // dW4 rows 64 + 16w.. (c part)
    f32x4 dy2[8];
    zero(dy2);
    mm_rows<64, 8>(sDP, kL64, WW(B, 3), 64, 0, dy2);  // dY2 = dp2 W4^T: [dh_A | dc]
    f32x4 dh[4], dc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      dh[nt] = dy2[nt];
      dc[nt] = dy2[4 + nt];
#pragma unroll
      for (int i = 0; i < 4; ++i) B.dc[(tile * 64 + orow(i)) * 64 + ocol(nt)] = dc[nt][i];
    }
    // edges where this row receives
    const int wd = p.tile_width[tile];
    for (int q = 0; q < wd; ++q) {
      __syncthreads();
      l2_row(p, B.h, tile, q, sX, true);
      __syncthreads();
      f32x4 pre[4];
      zero(pre);
      mm_rows<128, 4>(sX, kL128, WT(B, 2), 128, 0, pre);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) pre[nt][i] = pre[nt][i] > 0.f ? dc[nt][i] : 0.f;  // dpp
      put<4>(sDP, kL64, 0, pre, false);
      put<4>(sDPt, kL64, 0, pre, true);
      __syncthreads();
      mm_wgrad<4>(sX, kL128, w, sDPt, kL64, g3[0]);
      mm_wgrad<4>(sX, kL128, w + 4, sDPt, kL64, g3[1]);
      mm_rows<64, 4>(sDP, kL64, WW(B, 2), 64, 0, dh);  // receiver half of dX2 = dpp W3^T
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) B.dh[(tile * 64 + orow(i)) * 64 + ocol(nt)] = dh[nt][i];
    __syncthreads();
  }
  // partials (padded layout of dW): W5 [64][32] at off(4), W4 [128][64] at off(3), W3 at off(2)
  float* gp = B.gpart + (int64_t)blockIdx.x * kNnPadded;
  const int l = ln();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = 16 * w + 4 * (l >> 4) + i;
    gp[nn_padded_off(4) + m * 32 + (l & 15)] += g5[0][i];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int mm = m + 64 * half;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        gp[nn_padded_off(3) + mm * 64 + nt * 16 + (l & 15)] += g4[half][nt][i];
        gp[nn_padded_off(2) + mm * 64 + nt * 16 + (l & 15)] += g3[half][nt][i];
      }
    }
  }
  lsum = wave_sum(lsum);
  __shared__ double sl[4];
  if (l == 0) sl[w] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) B.lpart[blockIdx.x] += (sl[0] + sl[1] + sl[2] + sl[3]) * (double)scale / B.sc->den;
}

// Layer 2, sender side: dh_j += sum over i in N(j) of the sender half of dpp_ij W3^T,
// dpp_ij = dc_i * [p_ij > 0] recomputed from [h_i; h_j].
__global__ void __launch_bounds__(256) k_nn_l2_bwd_send(DevPattern p, NnBufs B, int G) {
  __shared__ __attribute__((aligned(16))) uint16_t sX[64 * kL128], sDP[64 * kL64];
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += G) {
    f32x4 dh[4];
    zero(dh);
    const int wd = p.tile_width[tile];
    const int64_t s0 = p.tile_slot0[tile];
    for (int q = 0; q < wd; ++q) {
      __syncthreads();
      l2_row(p, B.h, tile, q, sX, false);  // [h_nbr; h_self]
      __syncthreads();
      f32x4 pre[4];
      zero(pre);
      mm_rows<128, 4>(sX, kL128, WT(B, 2), 128, 0, pre);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = orow(i);
        const int nb = p.ent_nbr[(s0 + q) * 64 + r];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
          pre[nt][i] = pre[nt][i] > 0.f ? B.dc[(int64_t)nb * 64 + ocol(nt)] : 0.f;
      }
      put<4>(sDP, kL64, 0, pre, false);
      __syncthreads();
      mm_rows<64, 4>(sDP, kL64, WW(B, 2) + 64 * 64, 64, 0, dh);  // sender half: rows 64..127 of W3
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) B.dh[(tile * 64 + orow(i)) * 64 + ocol(nt)] += dh[nt][i];
    __syncthreads();
  }
}

// Layer 1: dW2, dW1 from dh.
template <typename TB>
__global__ void __launch_bounds__(256) k_nn_l1_bwd(DevPattern p, const TB* __restrict__ offd, NnBufs B, int G) {
  __shared__ __attribute__((aligned(16))) uint16_t sX[64 * kL64], sY[64 * kL96], sDP[64 * kL64],
      sDPt[64 * kL64], sDA[64 * kL96];
  const int w = wv();
  f32x4 g1[4], g2[2][4];
  zero(g1);
  zero(g2[0]);
  zero(g2[1]);
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += G) {
    f32x4 pre1[4];
    l1_tile<TB>(p, offd, B.u, WT(B, 0), 64, WT(B, 1), 96, tile, sX, sY, pre1);
    f32x4 dp1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        dp1[nt][i] = pre1[nt][i] > 0.f ? B.dh[(tile * 64 + orow(i)) * 64 + ocol(nt)] : 0.f;
    __syncthreads();
    put<4>(sDP, kL64, 0, dp1, false);
    put<4>(sDPt, kL64, 0, dp1, true);
    __syncthreads();
    mm_wgrad<4>(sY, kL96, w, sDPt, kL64, g2[0]);  // dW2 rows 16 w ..
    if (w < 2) mm_wgrad<4>(sY, kL96, w + 4, sDPt, kL64, g2[1]);  // rows 64 + 16 w .. (96 rows)
    f32x4 dy1[6];
    zero(dy1);
    mm_rows<64, 6>(sDP, kL64, WW(B, 1), 64, 0, dy1);  // dY1 = dp1 W2^T  [64 x 96]
    put<6>(sDA, kL96, 0, dy1, false);
    __syncthreads();
    const int wd = p.tile_width[tile];
    for (int q = 0; q < wd; ++q) {
      __syncthreads();
      if (threadIdx.x < 64) l1_row<TB>(p, offd, B.u, tile, q, threadIdx.x, sX);
      __syncthreads();
      f32x4 pre[4];
      zero(pre);
      mm_rows<64, 4>(sX, kL64, WT(B, 0), 64, 0, pre);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) pre[nt][i] = pre[nt][i] > 0.f ? bf2f(sDA[orow(i) * kL96 + 24 + ocol(nt)]) : 0.f;
      __syncthreads();
      put<4>(sDPt, kL64, 0, pre, true);
      __syncthreads();
      mm_wgrad<4>(sX, kL64, w, sDPt, kL64, g1);
    }
    __syncthreads();
  }
  float* gp = B.gpart + (int64_t)blockIdx.x * kNnPadded;
  const int l = ln();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = 16 * w + 4 * (l >> 4) + i;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      gp[nn_padded_off(0) + m * 64 + nt * 16 + (l & 15)] += g1[nt][i];
      gp[nn_padded_off(1) + m * 64 + nt * 16 + (l & 15)] += g2[0][nt][i];
      if (w < 2) gp[nn_padded_off(1) + (m + 64) * 64 + nt * 16 + (l & 15)] += g2[1][nt][i];
    }
  }
}

// fixed-order sum of the per-workgroup partials -> packed gradient; loss
__global__ void k_nn_grad_reduce(NnBufs B, int G, float* __restrict__ grad, double* __restrict__ loss) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0 && loss) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += B.lpart[g];
    *loss = s;
  }
  if (t >= kNnPadded) return;
  int l = 0, o = t;
  while (o >= kNnInPad[l] * kNnOutPad[l]) {
    o -= kNnInPad[l] * kNnOutPad[l];
    ++l;
  }
  const int i = o / kNnOutPad[l], j = o % kNnOutPad[l];
  if (i >= kNnIn[l] || j >= kNnOut[l]) return;
  float s = 0.f;
  for (int g = 0; g < G; ++g) s += B.gpart[(int64_t)g * kNnPadded + t];
  grad[nn_packed_off(l) + i * kNnOut[l] + j] = s;
}

__global__ void k_nn_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                          const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                          float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gg = g[t];
  const float mm = b1 * m[t] + (1.f - b1) * gg;
  const float vv = b2 * v[t] + (1.f - b2) * gg * gg;
  m[t] = mm;
  v[t] = vv;
  w[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_nn_selftest(const uint16_t* a, const uint16_t* bt, float* c) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[64 * 64], sB[64 * 64];
  copy_lds(sA, a, 64 * 64);
  copy_lds(sB, bt, 64 * 64);
  __syncthreads();
  f32x4 acc[4];
  zero(acc);
  mm_rows<64, 4>(sA, 64, sB, 64, 0, acc);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) c[orow(i) * 64 + ocol(nt)] = acc[nt][i];
}

}  // namespace

#define FNLH_NN_STORE(storage, BODY) \
  do {                               \
    if ((storage) == kF64) {         \
      using TB = double;             \
      BODY;                          \
    } else if ((storage) == kF32) {  \
      using TB = float;              \
      BODY;                          \
    } else {                         \
      using TB = bf16s;              \
      BODY;                          \
    }                                \
  } while (0)

void nn_launch_cast(const float* master, uint16_t* wt, uint16_t* w, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_cast, dim3((kNnPadded + 255) / 256), dim3(256), 0, s, master, wt, w);
}

void nn_launch_features(int storage, const DevPattern& p, const void* diag, int orow_sys, const NnVec& r,
                        const NnVec* e, int64_t N, const NnBufs& B, bool pivot, hipStream_t s) {
  const unsigned nt = (unsigned)p.n_tiles;
  hipLaunchKernelGGL(k_nn_sumsq, dim3(nt), dim3(64), 0, s, p, r, B.part);
  hipLaunchKernelGGL(k_nn_finalize, dim3(1), dim3(256), 0, s, B.part, p.n_tiles, N, B.sc, 0);
  const int has_e = (e && B.ehat) ? 1 : 0;
  const NnVec ev = has_e ? *e : NnVec{};
  FNLH_NN_STORE(storage, {
    hipLaunchKernelGGL((k_nn_feat<TB>), dim3(nt), dim3(64), 0, s, p, (const TB*)diag, orow_sys, r, ev, has_e, B,
                       pivot);
  });
  if (has_e) hipLaunchKernelGGL(k_nn_finalize, dim3(1), dim3(256), 0, s, B.part, p.n_tiles, N, B.sc, 1);
}

void nn_launch_forward_l1(int storage, const DevPattern& p, const void* offd, const NnBufs& B, hipStream_t s) {
  FNLH_NN_STORE(storage, {
    hipLaunchKernelGGL((k_nn_l1_fwd<TB>), dim3((unsigned)p.n_tiles), dim3(256), 0, s, p, (const TB*)offd, B);
  });
}

void nn_launch_forward(int storage, const DevPattern& p, const void* offd, const NnBufs& B, hipStream_t s) {
  nn_launch_forward_l1(storage, p, offd, B, s);
  hipLaunchKernelGGL(k_nn_l2_fwd, dim3((unsigned)p.n_tiles), dim3(256), 0, s, p, B);
}

void nn_launch_output(const DevPattern& p, const NnBufs& B, const NnOut& o, hipStream_t s) {
  const int64_t n = p.NP * 12;
  hipLaunchKernelGGL(k_nn_output, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, B, o);
}

void nn_launch_pack16(const DevPattern& p, const int32_t* iperm, const double* user, double sign, uint16_t* out,
                      hipStream_t s) {
  const int64_t n = p.NP * 12;
  hipLaunchKernelGGL(k_nn_pack16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, iperm, user, sign, out);
}

void nn_launch_unpack16(const DevPattern& p, const int32_t* iperm, const uint16_t* in, double* user, hipStream_t s) {
  const int64_t n = p.NP * 12;
  hipLaunchKernelGGL(k_nn_unpack16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, iperm, in, user);
}

uint64_t nn_start_key(uint64_t seed, int64_t start) {
  uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(start + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

void nn_launch_uniform(int64_t n, uint64_t key, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_uniform, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, key, x);
}

void nn_launch_step(const DevPattern& p, double* x, const double* xt, double* r, const double* rn, int ns, int vs,
                    const SysState* st, double* part4, double* alpha, int* counts, double accept, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_dots, dim3((unsigned)p.n_tiles), dim3(64), 0, s, p, r, rn, ns, vs, part4);
  hipLaunchKernelGGL(k_nn_alpha, dim3(1), dim3(256), 0, s, part4, p.n_tiles, st, vs, alpha, counts, accept);
  const int64_t n = p.NP * 6;
  hipLaunchKernelGGL(k_nn_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, x, xt, r, rn, ns, vs,
                     alpha);
}

void nn_launch_backward(int storage, const DevPattern& p, const void* offd, const NnBufs& B, int G, double scale,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_nn_l2_bwd, dim3(G), dim3(256), 0, s, p, B, G, (float)scale);
  hipLaunchKernelGGL(k_nn_l2_bwd_send, dim3(G), dim3(256), 0, s, p, B, G);
  FNLH_NN_STORE(storage, {
    hipLaunchKernelGGL((k_nn_l1_bwd<TB>), dim3(G), dim3(256), 0, s, p, (const TB*)offd, B, G);
  });
}

void nn_launch_grad_reduce(const NnBufs& B, int G, float* grad_packed, double* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_grad_reduce, dim3((kNnPadded + 255) / 256), dim3(256), 0, s, B, G, grad_packed, loss_out);
}

void nn_launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                    int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_nn_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
}

void nn_launch_selftest(const uint16_t* a, const uint16_t* bt, float* c, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_selftest, dim3(1), dim3(256), 0, s, a, bt, c);
}

}  // namespace fnlh
