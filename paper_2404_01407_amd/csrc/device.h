// Device-side helpers shared by the gfx950 kernels: storage formats and their
// SELL-64 access, the Euler + SA flux Jacobian, complex 6x6 inversion.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fnlh {

constexpr int kLanes = 64;

// ---------------------------------------------------------------- storage formats
// A 6x6 block of one row is stored as 16-byte vectors of V entries; vector v of all 64
// rows of a tile is contiguous, so one dwordx4 load per lane reads 1 KiB per wave:
//   element (q, lane) of a slot at ((q / V) * 64 + lane) * V + q % V.
struct bf16s {
  uint16_t v;
};

template <typename T> struct Fmt;
template <> struct Fmt<double> {
  static constexpr int V = 2;
  static constexpr int NV = 18;
  using A = double;  // arithmetic type of the sweep
};
template <> struct Fmt<float> {
  static constexpr int V = 4;
  static constexpr int NV = 9;
  using A = float;
};
template <> struct Fmt<bf16s> {
  static constexpr int V = 8;
  static constexpr int NV = 5;  // 40 entries, the last 4 unused
  using A = float;
};
template <typename T> constexpr int64_t slot_elems() { return (int64_t)Fmt<T>::NV * kLanes * Fmt<T>::V; }

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __uint_as_float((uint32_t)h << 16);
#else
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
#endif
}

// FP64 -> BF16, round to nearest, ties to even, directly from the double (8 significant
// bits).  Normal BF16 range assumed (no subnormals / overflow in Jacobian entries).
__device__ inline uint16_t f64_to_bf16_rne(double x) {
  uint64_t u = (uint64_t)__double_as_longlong(x);
  uint32_t sign = (uint32_t)(u >> 63);
  int32_t ex = (int32_t)((u >> 52) & 0x7ff);
  uint64_t man = u & ((1ull << 52) - 1);
  if (ex == 0) return (uint16_t)(sign << 15);  // zero (and double subnormals) -> signed zero
  uint64_t keep = man >> 45;
  uint64_t rest = man & ((1ull << 45) - 1);
  const uint64_t half = 1ull << 44;
  if (rest > half || (rest == half && (keep & 1ull))) ++keep;
  if (keep == 128) {
    keep = 0;
    ++ex;
  }
  int32_t fe = ex - 1023 + 127;
  return (uint16_t)((sign << 15) | ((uint32_t)fe << 7) | (uint32_t)keep);
}

template <typename T> __device__ inline void store_entry(T* slot, int q, int lane, double v);
template <> __device__ inline void store_entry<double>(double* s, int q, int lane, double v) {
  s[((q >> 1) * kLanes + lane) * 2 + (q & 1)] = v;
}
template <> __device__ inline void store_entry<float>(float* s, int q, int lane, double v) {
  s[((q >> 2) * kLanes + lane) * 4 + (q & 3)] = (float)v;  // RNE
}
template <> __device__ inline void store_entry<bf16s>(bf16s* s, int q, int lane, double v) {
  s[((q >> 3) * kLanes + lane) * 8 + (q & 7)].v = f64_to_bf16_rne(v);
}

template <typename T> __device__ inline double load_entry_f64(const T* slot, int q, int lane);
template <> __device__ inline double load_entry_f64<double>(const double* s, int q, int lane) {
  return s[((q >> 1) * kLanes + lane) * 2 + (q & 1)];
}
template <> __device__ inline double load_entry_f64<float>(const float* s, int q, int lane) {
  return (double)s[((q >> 2) * kLanes + lane) * 4 + (q & 3)];
}
template <> __device__ inline double load_entry_f64<bf16s>(const bf16s* s, int q, int lane) {
  return (double)bf16_to_f32(s[((q >> 3) * kLanes + lane) * 8 + (q & 7)].v);
}

// Read-once streams (blocks, factors) use non-temporal loads so they do not displace
// the neighbour vectors that other rows read again from the cache.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
__device__ inline nt_f4 ld_stream(const float4* p) { return __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p)); }
__device__ inline nt_d2 ld_stream(const double2* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
}
__device__ inline nt_u4 ld_stream(const uint4* p) { return __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p)); }

// Whole block of one lane, 16-byte vector loads, converted to the arithmetic type A.
template <typename T, typename A> __device__ inline void load_block(const T* __restrict__ slot, int lane, A (&k)[36]);
template <typename A> __device__ inline void load_block(const double* __restrict__ s, int lane, A (&k)[36]) {
  const double2* p = reinterpret_cast<const double2*>(s) + lane;
#pragma unroll
  for (int v = 0; v < 18; ++v) {
    const nt_d2 d = ld_stream(p + v * kLanes);
    k[2 * v] = (A)d.x;
    k[2 * v + 1] = (A)d.y;
  }
}
template <typename A> __device__ inline void load_block(const float* __restrict__ s, int lane, A (&k)[36]) {
  const float4* p = reinterpret_cast<const float4*>(s) + lane;
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    const nt_f4 d = ld_stream(p + v * kLanes);
    k[4 * v] = (A)d.x;
    k[4 * v + 1] = (A)d.y;
    k[4 * v + 2] = (A)d.z;
    k[4 * v + 3] = (A)d.w;
  }
}
template <typename A> __device__ inline void load_block(const bf16s* __restrict__ s, int lane, A (&k)[36]) {
  const uint4* p = reinterpret_cast<const uint4*>(s) + lane;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const nt_u4 d = ld_stream(p + v * kLanes);
    uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      int q = 8 * v + 2 * h;
      if (q < 36) k[q] = (A)__uint_as_float(w[h] << 16);
      if (q + 1 < 36) k[q + 1] = (A)__uint_as_float(w[h] & 0xffff0000u);
    }
  }
}

// ---------------------------------------------------------------- D~^-1 slots
// Complex 6x6 inverse per row, 36 complex entries (row-major), stored per tile as
// [v][lane][VD]: FP64 one complex per double2, FP32 two complex per float4.
template <typename TD> struct DFmt;
template <> struct DFmt<double> {
  static constexpr int NV = 36;
};
template <> struct DFmt<float> {
  static constexpr int NV = 18;
};
// Reduced-precision factors: FP16 entries with a power-of-two scale per row.  A tile is
// [9][lane][8 halves] (four complex entries per 16-byte vector, row-major) followed by
// one float scale per lane: 74 * 64 two-byte elements.
struct hfac {
  uint16_t v;
};
template <typename TD> struct DinvTile;  // elements of TD per tile (dinv_tile_elems on the host)
template <> struct DinvTile<double> {
  static constexpr int64_t N = 72 * kLanes;
};
template <> struct DinvTile<float> {
  static constexpr int64_t N = 72 * kLanes;
};
template <> struct DinvTile<hfac> {
  static constexpr int64_t N = 74 * kLanes;
};

// Store a row's D~^-1 (re, im: 36 complex entries, row-major, of the arithmetic type F).
template <typename F> __device__ inline void store_dinv(double* t, int lane, const F (&re)[36], const F (&im)[36]) {
  double2* p = reinterpret_cast<double2*>(t) + lane;
#pragma unroll
  for (int c = 0; c < 36; ++c) p[c * kLanes] = make_double2((double)re[c], (double)im[c]);
}
template <typename F> __device__ inline void store_dinv(float* t, int lane, const F (&re)[36], const F (&im)[36]) {
  float4* p = reinterpret_cast<float4*>(t) + lane;
#pragma unroll
  for (int v = 0; v < 18; ++v)
    p[v * kLanes] = make_float4((float)re[2 * v], (float)im[2 * v], (float)re[2 * v + 1], (float)im[2 * v + 1]);
}

template <typename F> __device__ inline void store_dinv(hfac* t, int lane, const F (&re)[36], const F (&im)[36]) {
  double m = 0.0;
#pragma unroll
  for (int c = 0; c < 36; ++c) m = fmax(m, fmax(fabs((double)re[c]), fabs((double)im[c])));
  // entries scaled by 2^(14 - e) with m in [2^e, 2^(e+1)) stay below 2^15 (FP16 max 65504)
  int e = 0;
  if (m > 0.0 && isfinite(m)) e = ilogb(m);
  const double up = ldexp(1.0, 14 - e);
  uint4* p = reinterpret_cast<uint4*>(t) + lane;
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = 4 * v + h;
      const uint16_t a = __builtin_bit_cast(uint16_t, (_Float16)(float)((double)re[c] * up));
      const uint16_t b = __builtin_bit_cast(uint16_t, (_Float16)(float)((double)im[c] * up));
      w[h] = (uint32_t)a | ((uint32_t)b << 16);
    }
    p[v * kLanes] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  reinterpret_cast<float*>(t + 72 * kLanes)[lane] = (float)ldexp(1.0, e - 14);
}

// y = Dinv a, complex; Dinv streamed from memory row by row.
template <typename TD, typename A>
__device__ inline void apply_dinv(const TD* __restrict__ t, int lane, const A (&a)[12], A (&y)[12]);
template <typename A>
__device__ inline void apply_dinv(const double* __restrict__ t, int lane, const A (&a)[12], A (&y)[12]) {
  const double2* p = reinterpret_cast<const double2*>(t) + lane;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    A yr = 0, yi = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const nt_d2 d = ld_stream(p + (6 * r + c) * kLanes);
      yr += (A)d.x * a[2 * c] - (A)d.y * a[2 * c + 1];
      yi += (A)d.x * a[2 * c + 1] + (A)d.y * a[2 * c];
    }
    y[2 * r] = yr;
    y[2 * r + 1] = yi;
  }
}
template <typename A>
__device__ inline void apply_dinv(const float* __restrict__ t, int lane, const A (&a)[12], A (&y)[12]) {
  const float4* p = reinterpret_cast<const float4*>(t) + lane;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    A yr = 0, yi = 0;
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      const nt_f4 d = ld_stream(p + (3 * r + h) * kLanes);
      const int c0 = 2 * h, c1 = 2 * h + 1;
      yr += (A)d.x * a[2 * c0] - (A)d.y * a[2 * c0 + 1] + (A)d.z * a[2 * c1] - (A)d.w * a[2 * c1 + 1];
      yi += (A)d.x * a[2 * c0 + 1] + (A)d.y * a[2 * c0] + (A)d.z * a[2 * c1 + 1] + (A)d.w * a[2 * c1];
    }
    y[2 * r] = yr;
    y[2 * r + 1] = yi;
  }
}
__device__ inline float h2f(uint32_t bits) { return (float)__builtin_bit_cast(_Float16, (uint16_t)bits); }
// A row's FP16 D~^-1 held in registers: load() issues the reads, apply() uses them, so a
// caller can have the next row's (or system's) factor in flight while it works.
struct HfacInv {
  uint32_t w[36];  // complex entry (r, c) at 6r + c: low half re, high half im
  float sc;
  __device__ inline void load(const hfac* __restrict__ t, int lane) {
    const uint4* p = reinterpret_cast<const uint4*>(t) + lane;
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const nt_u4 d = ld_stream(p + v * kLanes);
      w[4 * v] = d.x;
      w[4 * v + 1] = d.y;
      w[4 * v + 2] = d.z;
      w[4 * v + 3] = d.w;
    }
    sc = reinterpret_cast<const float*>(t + 72 * kLanes)[lane];
  }
  template <typename A> __device__ inline void apply(const A (&a)[12], A (&y)[12]) const {
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      A yr = 0, yi = 0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const uint32_t q = w[6 * r + c];
        const A dr = (A)h2f(q & 0xffffu), di = (A)h2f(q >> 16);
        yr += dr * a[2 * c] - di * a[2 * c + 1];
        yi += dr * a[2 * c + 1] + di * a[2 * c];
      }
      y[2 * r] = yr * (A)sc;
      y[2 * r + 1] = yi * (A)sc;
    }
  }
};
template <typename A>
__device__ inline void apply_dinv(const hfac* __restrict__ t, int lane, const A (&a)[12], A (&y)[12]) {
  HfacInv f;
  f.load(t, lane);
  f.apply(a, y);
}

template <typename TD> __device__ inline void load_dinv_entry(const TD* t, int lane, int c, double& re, double& im);
template <> __device__ inline void load_dinv_entry<double>(const double* t, int lane, int c, double& re, double& im) {
  double2 d = reinterpret_cast<const double2*>(t)[c * kLanes + lane];
  re = d.x;
  im = d.y;
}
template <> __device__ inline void load_dinv_entry<hfac>(const hfac* t, int lane, int c, double& re, double& im) {
  const uint32_t q = reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint4*>(t) + (c >> 2) * kLanes + lane)[c & 3];
  const double sc = (double)reinterpret_cast<const float*>(t + 72 * kLanes)[lane];
  re = (double)h2f(q & 0xffffu) * sc;
  im = (double)h2f(q >> 16) * sc;
}
template <> __device__ inline void load_dinv_entry<float>(const float* t, int lane, int c, double& re, double& im) {
  float4 d = reinterpret_cast<const float4*>(t)[(c >> 1) * kLanes + lane];
  re = (c & 1) ? d.z : d.x;
  im = (c & 1) ? d.w : d.y;
}

// ---------------------------------------------------------------- vectors
// Internal vectors: [system][row][12] (interleaved complex), 96 B (FP64) / 48 B (FP32).
template <typename T> __device__ inline void load_vec(const T* __restrict__ p, T (&v)[12]);
template <> __device__ inline void load_vec<double>(const double* __restrict__ p, double (&v)[12]) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double2 d = q[i];
    v[2 * i] = d.x;
    v[2 * i + 1] = d.y;
  }
}
template <> __device__ inline void load_vec<float>(const float* __restrict__ p, float (&v)[12]) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float4 d = q[i];
    v[4 * i] = d.x;
    v[4 * i + 1] = d.y;
    v[4 * i + 2] = d.z;
    v[4 * i + 3] = d.w;
  }
}
template <typename T> __device__ inline void store_vec(T* __restrict__ p, const T (&v)[12]);
template <> __device__ inline void store_vec<double>(double* __restrict__ p, const double (&v)[12]) {
  double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
  for (int i = 0; i < 6; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
}
template <> __device__ inline void store_vec<float>(float* __restrict__ p, const float (&v)[12]) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
}

// acc -= K x  (K real 6x6, x complex 6)
template <typename A> __device__ inline void sub_kx(A (&acc)[12], const A (&k)[36], const A (&x)[12]) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    A sr = 0, si = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      sr += k[6 * r + c] * x[2 * c];
      si += k[6 * r + c] * x[2 * c + 1];
    }
    acc[2 * r] -= sr;
    acc[2 * r + 1] -= si;
  }
}

// ---------------------------------------------------------------- wave reduction
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- tile mapping
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Give
// every XCD a contiguous range of tiles (neighbouring cells, overlapping gathers), and
// keep the system groups of one tile on the same XCD, adjacent in dispatch order.
// The grid is 8 * ceil(nt*ng / 8) workgroups; returns false for the spare ones.
// b: the workgroup's index among the tile workgroups (blockIdx.x unless a kernel puts other
// work first); the grid holds 8 * ceil(nt * ng / 8) of them.
__device__ inline bool map_tile_b(int64_t nt, int ng, int64_t b, int64_t& tile, int& group) {
  const int64_t total = nt * ng;
  const int64_t per = (total + 7) / 8;
  if (b >= 8 * per) return false;
  const int64_t k = (b & 7) * per + (b >> 3);
  if (k >= total) return false;
  tile = k / ng;
  group = (int)(k % ng);
  return true;
}
__device__ inline bool map_tile(int64_t nt, int ng, int64_t& tile, int& group) {
  return map_tile_b(nt, ng, blockIdx.x, tile, group);
}

// ---------------------------------------------------------------- flux Jacobian
constexpr double kGamma = 1.4;

// A(Q;S) = dF/dQ of the Euler + convected-SA flux, row-major 6x6.
__device__ inline void flux_jacobian(const double (&Q)[6], const double (&S)[3], double (&A)[36]) {
  const double g1 = kGamma - 1.0;
  const double ir = 1.0 / Q[0];
  const double u0 = Q[1] * ir, u1 = Q[2] * ir, u2 = Q[3] * ir;
  const double q2 = u0 * u0 + u1 * u1 + u2 * u2;
  const double p = g1 * (Q[4] - 0.5 * Q[0] * q2);
  const double H = (Q[4] + p) * ir;
  const double nut = Q[5] * ir;
  const double U = u0 * S[0] + u1 * S[1] + u2 * S[2];
  const double phi = 0.5 * g1 * q2;
  const double u[3] = {u0, u1, u2};
  A[0] = 0.0;
  A[1] = S[0];
  A[2] = S[1];
  A[3] = S[2];
  A[4] = 0.0;
  A[5] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double* row = A + 6 * (1 + a);
    row[0] = -u[a] * U + phi * S[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) row[1 + b] = u[a] * S[b] - g1 * S[a] * u[b] + (a == b ? U : 0.0);
    row[4] = g1 * S[a];
    row[5] = 0.0;
  }
  A[24] = U * (phi - H);
  A[25] = H * S[0] - g1 * U * u0;
  A[26] = H * S[1] - g1 * U * u1;
  A[27] = H * S[2] - g1 * U * u2;
  A[28] = kGamma * U;
  A[29] = 0.0;
  A[30] = -nut * U;
  A[31] = nut * S[0];
  A[32] = nut * S[1];
  A[33] = nut * S[2];
  A[34] = 0.0;
  A[35] = U;
}

// |u.S| + a|S|
__device__ inline double spectral_radius(const double (&Q)[6], const double (&S)[3]) {
  const double ir = 1.0 / Q[0];
  const double u0 = Q[1] * ir, u1 = Q[2] * ir, u2 = Q[3] * ir;
  const double p = (kGamma - 1.0) * (Q[4] - 0.5 * Q[0] * (u0 * u0 + u1 * u1 + u2 * u2));
  const double a = sqrt(kGamma * p * ir);
  return fabs(u0 * S[0] + u1 * S[1] + u2 * S[2]) + a * sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
}

// ---------------------------------------------------------------- complex 6x6 inverse
// In-place Gauss-Jordan with partial (row) pivoting; row interchanges are undone as
// column interchanges at the end.  All indexing is static (selects), so the matrix
// stays in registers.  ok <- false for a zero or non-finite pivot.
template <typename F> __device__ inline void cinv6(F (&ar)[36], F (&ai)[36], bool& ok) {
  int piv[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    F best = ar[6 * k + k] * ar[6 * k + k] + ai[6 * k + k] * ai[6 * k + k];
    int p = k;
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      F m = ar[6 * i + k] * ar[6 * i + k] + ai[6 * i + k] * ai[6 * i + k];
      if (m > best) {
        best = m;
        p = i;
      }
    }
    piv[k] = p;
    if (!(best > (F)0) || !isfinite(best)) ok = false;
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      const bool sw = (p == i);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        F tr = ar[6 * k + c], ti = ai[6 * k + c];
        F vr = ar[6 * i + c], vi = ai[6 * i + c];
        ar[6 * k + c] = sw ? vr : tr;
        ai[6 * k + c] = sw ? vi : ti;
        ar[6 * i + c] = sw ? tr : vr;
        ai[6 * i + c] = sw ? ti : vi;
      }
    }
    // pivot reciprocal
    const F pr = ar[6 * k + k], pi = ai[6 * k + k];
    const F den = pr * pr + pi * pi;
    const F ivr = pr / den, ivi = -pi / den;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (c == k) continue;
      F r = ar[6 * k + c], i = ai[6 * k + c];
      ar[6 * k + c] = r * ivr - i * ivi;
      ai[6 * k + c] = r * ivi + i * ivr;
    }
    ar[6 * k + k] = ivr;
    ai[6 * k + k] = ivi;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i == k) continue;
      const F fr = ar[6 * i + k], fi = ai[6 * i + k];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (c == k) continue;
        const F br = ar[6 * k + c], bi = ai[6 * k + c];
        ar[6 * i + c] -= fr * br - fi * bi;
        ai[6 * i + c] -= fr * bi + fi * br;
      }
      ar[6 * i + k] = -(fr * ivr - fi * ivi);
      ai[6 * i + k] = -(fr * ivi + fi * ivr);
    }
  }
#pragma unroll
  for (int k = 5; k >= 0; --k) {
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      const bool sw = (piv[k] == i);
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        F tr = ar[6 * r + k], ti = ai[6 * r + k];
        F vr = ar[6 * r + i], vi = ai[6 * r + i];
        ar[6 * r + k] = sw ? vr : tr;
        ai[6 * r + k] = sw ? vi : ti;
        ar[6 * r + i] = sw ? tr : vr;
        ai[6 * r + i] = sw ? ti : vi;
      }
    }
  }
}

}  // namespace fnlh
