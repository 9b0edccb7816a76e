// gfx950 kernels of the shared-Jacobian, frequency-shifted block solve.
//
// Work decomposition: a tile is 64 consecutive internal rows of one colour (one row per
// lane of a wave).  A workgroup handles one tile for `spw` systems, one wave per system:
// the waves of a workgroup read the same off-diagonal blocks (sliced-ELL, coalesced
// 16-byte loads, served once from HBM and then from L2/L1), each applies them to its own
// system's vectors, whose only difference is the diagonal shift i omega V (section
// "Generalized RK Scheme for Time-Linearized Harmonic Flows": the harmonic LHS differs
// from the mean-flow LHS by that diagonal term and keeps its pattern).
//
// No floating-point atomics: norms are reduced per wave with shuffles, written per
// (system, tile), then summed in a fixed order by one workgroup per system, so results
// are bitwise reproducible run to run.
#include <cfloat>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace fnlh {

namespace {

constexpr int kOK = 0, kNotConverged = 1, kDiverged = 2;

inline dim3 tile_grid(int64_t nt, int ng) {
  const int64_t total = nt * ng;
  const int64_t per = (total + 7) / 8;
  return dim3((unsigned)(8 * per));
}

template <typename TB> struct TV_of {
  using T = typename Fmt<TB>::A;
};
// factor storage: FP64 with FP64 blocks, scaled FP16 with FP32 / BF16 blocks
template <typename TB> struct DF_of {
  using T = hfac;
};
template <> struct DF_of<double> {
  using T = double;
};

__device__ inline double shift_w(const DevPattern& p, int orow, int64_t row) {
  return p.omega[(int64_t)orow * p.n_zones + p.zone[row]] * p.vol[row];
}

// Phase-lagged periodic coupling (entry fe, system omega row orow): the neighbour is the
// image one pitch over, its value v times e^{i s sigma}, s = +-1 from the entry.
template <typename A> __device__ inline void apply_phase(const DevPattern& p, int64_t fe, int orow, A (&v)[12]) {
  const int sg = p.ent_phase[fe];
  if (sg == 0) return;
  const A c = (A)p.phase_cs[2 * orow], sn = (A)(sg * p.phase_cs[2 * orow + 1]);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const A re = v[2 * k], im = v[2 * k + 1];
    v[2 * k] = c * re - sn * im;
    v[2 * k + 1] = sn * re + c * im;
  }
}

// Frozen turbulence (system omega row orow): only the leading 5x5 sub-system is solved,
// so the sixth equation's residual is dropped (it never reaches the factors, whose sixth
// row and column are zero, and does not count in the norm).
template <typename A> __device__ inline void mask_frozen(const DevPattern& p, int orow, A (&v)[12]) {
  if (p.sys_frozen && p.sys_frozen[orow]) {
    v[10] = (A)0;
    v[11] = (A)0;
  }
}

// acc -= (K_ii + i w I) x_i
template <typename A>
__device__ inline void sub_diag_shift(A (&acc)[12], const A (&d)[36], A w, const A (&xi)[12]) {
  sub_kx(acc, d, xi);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    acc[2 * c] += w * xi[2 * c + 1];
    acc[2 * c + 1] -= w * xi[2 * c];
  }
}

template <typename A> __device__ inline double norm2_12(const A (&v)[12]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 12; ++i) s += (double)v[i] * (double)v[i];
  return s;
}

// ================================================================ sweeps
// Internal vectors interleave the systems of a solve per row, [row][ns][12], so the P
// systems a lane carries sit in one contiguous run of P*12 values: a lane loads each
// block once and applies it to all P systems.  A workgroup handles one tile (64 rows)
// with ceil(nb / P) waves.

// The systems of one wave: batch entries w*P .. w*P+P-1.
template <int P> struct WaveSys {
  int vs[P];
  int orow[P];
  int ds[P];
  bool run[P];
};

// norm_pass selects the flag test: a pass that accumulates the residual norm runs
// only for systems not yet pending; the other passes run for every active system.
template <int P>
__device__ inline bool wave_systems(const SysBatch& sb, const SysState* __restrict__ st, int w, bool norm_pass,
                                    WaveSys<P>& W) {
  bool any = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int k = w * P + j;
    W.run[j] = false;
    W.vs[j] = 0;
    W.orow[j] = 0;
    W.ds[j] = 0;
    if (k < sb.n) {
      W.vs[j] = sb.vslot[k];
      W.orow[j] = sb.orow[k];
      W.ds[j] = sb.dslot[k];
      const int act = st[W.vs[j]].active, pen = st[W.vs[j]].pending;
      W.run[j] = norm_pass ? (act && !pen) : (act != 0);
      any |= W.run[j];
    }
  }
  return any;
}

// acc[j] -= sum over the tile's slots of K_ik x_k (x of system j), blocks loaded once
template <typename TB, typename A, int P>
__device__ inline void gather_offd(const DevPattern& p, const TB* __restrict__ offd, const A* __restrict__ x, int ns,
                                   int64_t tile, int lane, const WaveSys<P>& W, A (&acc)[P][12]) {
  const int w = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  auto body = [&](int q) {
    const int64_t slot = s0 + q;
    const int nb = p.ent_nbr[slot * kLanes + lane];
    A kb[36];
    load_block(offd + slot * slot_elems<TB>(), lane, kb);
    const A* xr = x + (int64_t)nb * ns * 12;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      A xn[12];
      load_vec(xr + W.vs[j] * 12, xn);
      if (p.ent_phase) apply_phase(p, slot * kLanes + lane, W.orow[j], xn);
      sub_kx(acc[j], kb, xn);
    }
  };
  if (w == 6) {
#pragma unroll
    for (int q = 0; q < 6; ++q) body(q);
  } else {
    for (int q = 0; q < w; ++q) body(q);
  }
}

// Solve (Kd + i w I) y = r in place (r -> y) for a real 6x6 Kd: complex Gaussian
// elimination, static indexing (registers only).  PIVOT: partial pivoting; without it
// the caller guarantees Kd is strictly diagonally dominant by rows, which the shift
// preserves and elimination keeps (Schur complements stay dominant, pivots nonzero).
template <bool PIVOT, typename A>
__device__ inline void csolve6_shift(const A (&kd)[36], A w, A (&r)[12]) {
  A mr[36], mi[36], ivr[6], ivi[6];
#pragma unroll
  for (int c = 0; c < 36; ++c) {
    mr[c] = kd[c];
    mi[c] = 0;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) mi[7 * i] = w;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (PIVOT) {
      A best = mr[7 * k] * mr[7 * k] + mi[7 * k] * mi[7 * k];
      int pv = k;
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const A m = mr[6 * i + k] * mr[6 * i + k] + mi[6 * i + k] * mi[6 * i + k];
        if (m > best) {
          best = m;
          pv = i;
        }
      }
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        const bool sw = pv == i;
#pragma unroll
        for (int c = k; c < 6; ++c) {
          const A ar = mr[6 * k + c], ai = mi[6 * k + c], br = mr[6 * i + c], bi = mi[6 * i + c];
          mr[6 * k + c] = sw ? br : ar;
          mi[6 * k + c] = sw ? bi : ai;
          mr[6 * i + c] = sw ? ar : br;
          mi[6 * i + c] = sw ? ai : bi;
        }
        const A xr = r[2 * k], xi = r[2 * k + 1], yr = r[2 * i], yi = r[2 * i + 1];
        r[2 * k] = sw ? yr : xr;
        r[2 * k + 1] = sw ? yi : xi;
        r[2 * i] = sw ? xr : yr;
        r[2 * i + 1] = sw ? xi : yi;
      }
    }
    const A pr = mr[7 * k], pi = mi[7 * k];
    const A rden = (A)1 / (pr * pr + pi * pi);
    ivr[k] = pr * rden;
    ivi[k] = -pi * rden;
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      const A ar = mr[6 * i + k], ai = mi[6 * i + k];
      const A fr = ar * ivr[k] - ai * ivi[k], fi = ar * ivi[k] + ai * ivr[k];
#pragma unroll
      for (int c = k + 1; c < 6; ++c) {
        const A br = mr[6 * k + c], bi = mi[6 * k + c];
        mr[6 * i + c] -= fr * br - fi * bi;
        mi[6 * i + c] -= fr * bi + fi * br;
      }
      r[2 * i] -= fr * r[2 * k] - fi * r[2 * k + 1];
      r[2 * i + 1] -= fr * r[2 * k + 1] + fi * r[2 * k];
    }
  }
#pragma unroll
  for (int k = 5; k >= 0; --k) {
    A sr = r[2 * k], si = r[2 * k + 1];
#pragma unroll
    for (int c = k + 1; c < 6; ++c) {
      sr -= mr[6 * k + c] * r[2 * c] - mi[6 * k + c] * r[2 * c + 1];
      si -= mr[6 * k + c] * r[2 * c + 1] + mi[6 * k + c] * r[2 * c];
    }
    r[2 * k] = sr * ivr[k] - si * ivi[k];
    r[2 * k + 1] = sr * ivi[k] + si * ivr[k];
  }
}

// Strict row diagonal dominance of every stored diagonal block (valid rows); clears
// *flag (vector store) when a block is not dominant.
template <typename TB>
__global__ void k_check_dominance(DevPattern p, const TB* __restrict__ diag, int* __restrict__ flag) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane >= p.tile_nrows[tile]) return;
  const TB* d = diag + tile * slot_elems<TB>();
  bool ok = true;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double off = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (c != r) off += fabs(load_entry_f64<TB>(d, 6 * r + c, lane));
    ok &= fabs(load_entry_f64<TB>(d, 7 * r, lane)) > off;
  }
  if (!ok) *flag = 0;
}

// Two-colour fused pass.  With colours C0 (first) and C1, the DILU-Richardson step
//   forward:  y = Dt^-1 (r - L y),  backward: z = y - Dt^-1 U z,  x += z
// satisfies, row by row,
//   C0 rows:  x_i <- (K_ii + i w_i I)^-1 (b_i - sum_k K_ik x_k)          (Dt_i = D_i on C0)
//   C1 rows:  x_k <- x_k + Dt_k^-1 (b_k - (K_kk + i w_k I) x_k - sum_i K_ki x_i)
// so one step = [C1 pass, C0 pass] after an initial C0 pass, each block read once per
// step, and the C1 pass accumulates ||b - K_s x||^2 of the previous iterate (its C0
// residual is zero).  The C0 pass solves with the shifted diagonal block directly
// (no per-system factor read); the C1 pass applies the stored Dt^-1.
//
// Lane mapping: SW lanes share a row (lane = row_in_wave * SW + s), each carrying P
// systems (batch entries s, s+SW, ...).  The SW lanes of a row load the same block
// address (one fetch per instruction), and their vector records are adjacent in the
// interleaved layout.  A tile of 64 rows takes SW waves of 64/SW rows each.
// Sum of a system's per-tile norm partials (tiles [t0, t0 + nt), `slots` each) in one
// canonical order whatever the workgroup size (64 or 256 threads): 256 accumulators,
// accumulator v taking tiles v, v + 256, ... with their slots in order, then a fixed
// binary tree.  Every reduction of sweep norms uses it, so fused and separate reductions
// give the same bits.  All threads of the workgroup call it; the result is valid in
// thread 0.
__device__ inline double canonical_sum(const double* __restrict__ pp, int64_t nt, int slots) {
  __shared__ double sh[256];
  for (int v = threadIdx.x; v < 256; v += blockDim.x) {
    double s = 0.0;
    for (int64_t t = v; t < nt; t += 256)
      for (int q = 0; q < slots; ++q) s += pp[t * kPartialSlots + q];
    sh[v] = s;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    for (int v = threadIdx.x; v < o; v += blockDim.x) sh[v] += sh[v + o];
    __syncthreads();
  }
  return sh[0];
}

// The stop logic after one sweep (the norm is that of the sweep's residual, taken before
// its update; NoNorm: the first sweep, no norm yet).  A system that meets a criterion is
// marked pending and retires after the next sweep's reduction.
__device__ inline void sweep_state(SysState& S, double n2, int mode, double rtol2, double div2) {
  if (!S.active) return;
  if (S.pending) {
    S.active = 0;
    return;
  }
  S.sweeps += 1;
  if (mode == kReduceSweep) {
    // the norm is that of the iterate before this sweep, after sweeps - 1 of them (the
    // first sweep's is the initial norm, recorded at set-up)
    if (S.hist && S.sweeps >= 2 && S.hist_off + S.sweeps - 1 < S.hist_len) S.hist[S.hist_off + S.sweeps - 1] = n2;
    S.last_n2 = n2;
    if (n2 <= rtol2 * S.norm0sq) {
      S.status = kOK;
      S.pending = 1;
    } else if (!isfinite(n2) || n2 > div2 * S.norm0sq) {
      S.status = kDiverged;
      S.pending = 1;
    }
  }
  if (S.sweeps >= S.limit) S.pending = 1;
}

// The reduction of the update pass's per-tile norms for one system, done by one workgroup
// of the first-colour pass that follows it (one launch fewer per sweep), in the canonical
// order.
__device__ inline void fused_sweep_reduce(const FusedReduce& fr, const SysBatch& sb, const double* __restrict__ partial,
                                          int64_t n_tiles, SysState* __restrict__ st, int k) {
  const int vs = sb.vslot[k];
  const double* pp = partial + ((int64_t)vs * n_tiles + fr.t0) * kPartialSlots;
  const double n2 = canonical_sum(pp, fr.mode != kReduceSweepNoNorm ? fr.nt : 0, fr.slots);
  if (threadIdx.x != 0) return;
  SysState S = st[vs];
  sweep_state(S, n2, fr.mode, fr.rtol2, fr.div2);
  st[vs] = S;
}

// LDS staging of the blocks of one coupling slot for the R = 64 / SW rows of a wave whose
// SW lanes share a row: the wave loads the slot's R blocks once (distinct 16-byte chunks,
// U per lane) into its LDS buffer, then every lane reads its row's block from there (a
// broadcast among the row's lanes), instead of each lane fetching its row's whole block.
// Item t = v * R + i is 16-byte chunk v of row rowbase + i (NV chunks per block: FP64 18,
// FP32 9, BF16 5).
template <typename TB, int SW> struct BlockStage {
  static constexpr int R = kLanes / SW;
  static constexpr int NV = Fmt<TB>::NV;
  static constexpr int N = NV * R;           // chunks per slot
  static constexpr int U = (N + 63) / 64;    // loads per lane
  uint4 pre[U];
  // keep(i): whether row rowbase + i needs this slot's block (others are not fetched)
  template <typename Keep> __device__ void gload(const TB* base, int rowbase, int lane, Keep keep) {
    const uint4* src = reinterpret_cast<const uint4*>(base);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = lane + 64 * u;
      if (t < N && keep(t % R)) {
        const nt_u4 d = ld_stream(src + (t / R) * kLanes + rowbase + (t % R));
        pre[u] = make_uint4(d.x, d.y, d.z, d.w);
      }
    }
  }
  __device__ void lstore(uint4* buf, int lane) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = lane + 64 * u;
      if (t < N) buf[t] = pre[u];
    }
  }
  template <typename A> __device__ static void lload(const uint4* buf, int ir, A (&k)[36]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const uint4 d = buf[v * R + ir];
      if constexpr (std::is_same<TB, double>::value) {
        k[2 * v] = (A)__hiloint2double((int)d.y, (int)d.x);
        k[2 * v + 1] = (A)__hiloint2double((int)d.w, (int)d.z);
      } else if constexpr (std::is_same<TB, float>::value) {
        k[4 * v] = (A)__uint_as_float(d.x);
        k[4 * v + 1] = (A)__uint_as_float(d.y);
        k[4 * v + 2] = (A)__uint_as_float(d.z);
        k[4 * v + 3] = (A)__uint_as_float(d.w);
      } else {
        const uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int q = 8 * v + 2 * h;
          if (q < 36) k[q] = (A)__uint_as_float(w[h] << 16);
          if (q + 1 < 36) k[q + 1] = (A)__uint_as_float(w[h] & 0xffff0000u);
        }
      }
    }
  }
};
struct KeepAll {
  __device__ bool operator()(int) const { return true; }
};

// The general-colouring passes with four lanes per row stage their coupling blocks through
// LDS (two slot buffers of 16 blocks per wave), for any block precision and systems per lane.
template <typename TB, int SW> constexpr bool gen_lds_path() { return SW == 4; }

// Both two-colour passes with four lanes per row stage their diagonal and coupling blocks
// through LDS (two slot buffers of 16 blocks per wave), for any block precision.
template <typename TB, int SW, int P, bool UPDATE, bool PH> constexpr bool rb_lds_path() { return SW == 4; }
// 16-byte LDS chunks per wave of the staged passes (four lanes per row, two slot buffers)
constexpr int lds_chunks_per_wave(int storage) {
  return 2 * (kLanes / 4) * (storage == kF64 ? Fmt<double>::NV : storage == kF32 ? Fmt<float>::NV : Fmt<bf16s>::NV);
}
// The first-colour pass with FP32 or BF16 blocks parks its diagonal block in a third slot
// buffer until the elimination that follows the couplings, instead of holding it in 36
// registers through the coupling loop (the register count sets the waves per SIMD).
// FP64 keeps it in registers.
template <typename TB, bool UPDATE> constexpr bool rb_diag_in_lds() { return !UPDATE && !std::is_same<TB, double>::value; }
template <typename TB, bool UPDATE> constexpr int rb_lds_chunks_t() {
  return (rb_diag_in_lds<TB, UPDATE>() ? 3 : 2) * (kLanes / 4) * Fmt<TB>::NV;
}
constexpr int rb_lds_chunks(int storage, bool update) {
  return (!update && storage != kF64 ? 3 : 2) * (kLanes / 4) *
         (storage == kF64 ? Fmt<double>::NV : storage == kF32 ? Fmt<float>::NV : Fmt<bf16s>::NV);
}

// PH = false: no phase-lagged couplings (p.ent_phase is null); the FP32 four-lanes-per-row
// passes then stage their blocks through LDS (rb_lds_path).
template <typename TB, int SW, int P, bool UPDATE, bool PIVOT, bool PH = true>
__device__ inline void rb_tile(const DevPattern& p, const TB* __restrict__ offd, const TB* __restrict__ diag,
                               const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride,
                               typename TV_of<TB>::T* __restrict__ x, const typename TV_of<TB>::T* __restrict__ b,
                               int ns, const SysBatch& sb, const SysState* __restrict__ st,
                               double* __restrict__ partial, int64_t tile, int w, uint4* lds = nullptr) {
  using A = typename TV_of<TB>::T;
  const int lane = threadIdx.x & 63;
  const int sidx = lane % SW;
  const int rl = w * (kLanes / SW) + lane / SW;  // row within the tile
  const int64_t row = tile * kLanes + rl;
  const bool valid = rl < p.tile_nrows[tile];
  int vs[P], orow[P], ds[P];
  bool run[P];
  bool any = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int k = j * SW + sidx;
    run[j] = false;
    vs[j] = orow[j] = ds[j] = 0;
    if (k < sb.n) {
      vs[j] = sb.vslot[k];
      orow[j] = sb.orow[k];
      ds[j] = sb.dslot[k];
      const int act = st[vs[j]].active, pen = st[vs[j]].pending;
      run[j] = UPDATE ? (act && !pen) : (act != 0);
      any |= run[j];
    }
  }
  if (!__any(any)) return;
  const int64_t rb = row * ns * 12;
  A acc[P][12];
#pragma unroll
  for (int j = 0; j < P; ++j) {
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[j][i] = 0;
    if (run[j]) load_vec(b + rb + vs[j] * 12, acc[j]);
  }
  // update pass, FP32/BF16: every system's own x is requested together, before the
  // diagonal block is staged (one latency for all of them)
  constexpr bool kXFirst = UPDATE && !std::is_same<TB, double>::value;
  A xo[kXFirst ? P : 1][12];
  if constexpr (kXFirst) {
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (run[j]) load_vec(x + rb + vs[j] * 12, xo[j]);
  }
  // LDS staging of the blocks (rb_lds_path): see BlockStage
  const int rowbase = w * (kLanes / SW);
  BlockStage<TB, SW> stg;
  constexpr int SN = BlockStage<TB, SW>::N;
  constexpr bool kDiagLds = rb_lds_path<TB, SW, P, UPDATE, PH>() && rb_diag_in_lds<TB, UPDATE>();
  A d[36];
  if constexpr (kDiagLds) {
    // read back after the couplings (third slot buffer, untouched by their staging)
    stg.gload(diag + tile * slot_elems<TB>(), rowbase, lane, KeepAll());
    stg.lstore(lds + 2 * SN, lane);
  } else if constexpr (rb_lds_path<TB, SW, P, UPDATE, PH>()) {
    stg.gload(diag + tile * slot_elems<TB>(), rowbase, lane, KeepAll());
    stg.lstore(lds + SN, lane);
    __builtin_amdgcn_wave_barrier();
    BlockStage<TB, SW>::lload(lds + SN, lane / SW, d);
    __builtin_amdgcn_wave_barrier();
  } else {
    load_block(diag + tile * slot_elems<TB>(), rl, d);
  }
  if constexpr (kXFirst) {
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (run[j]) sub_diag_shift(acc[j], d, (A)shift_w(p, orow[j], row), xo[j]);
  } else if (UPDATE) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!run[j]) continue;
      A xi[12];
      load_vec(x + rb + vs[j] * 12, xi);
      sub_diag_shift(acc[j], d, (A)shift_w(p, orow[j], row), xi);
    }
  }
  {
    const int wd = p.tile_width[tile];
    const int64_t s0 = p.tile_slot0[tile];
    auto body = [&](int q) {
      const int64_t slot = s0 + q;
      const int nb = p.ent_nbr[slot * kLanes + rl];
      A kb[36];
      load_block(offd + slot * slot_elems<TB>(), rl, kb);
      const A* xr = x + (int64_t)nb * ns * 12;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        if (!run[j]) continue;
        A xn[12];
        load_vec(xr + vs[j] * 12, xn);
        if (PH && p.ent_phase) apply_phase(p, slot * kLanes + rl, orow[j], xn);
        sub_kx(acc[j], kb, xn);
      }
    };
    if constexpr (rb_lds_path<TB, SW, P, UPDATE, PH>()) {
      // two buffers: slot q + 1 is loaded while slot q is applied
      if (wd > 0) {
        stg.gload(offd + s0 * slot_elems<TB>(), rowbase, lane, KeepAll());
        stg.lstore(lds, lane);
      }
      // the neighbour index of slot q + 1 is requested while slot q is applied
      int nb_next = wd > 0 ? p.ent_nbr[s0 * kLanes + rl] : 0;
      for (int q = 0; q < wd; ++q) {
        const int nb = nb_next;
        if (q + 1 < wd) {
          stg.gload(offd + (s0 + q + 1) * slot_elems<TB>(), rowbase, lane, KeepAll());
          nb_next = p.ent_nbr[(s0 + q + 1) * kLanes + rl];
        }
        const int64_t slot = s0 + q;
        const A* xr = x + (int64_t)nb * ns * 12;
        if constexpr (P == 1) {
          // one system: its neighbour vector is fetched before the block is read back
          A xn[12];
          if (run[0]) load_vec(xr + vs[0] * 12, xn);
          if (PH && run[0] && p.ent_phase) apply_phase(p, slot * kLanes + rl, orow[0], xn);
          __builtin_amdgcn_wave_barrier();
          A kb[36];
          BlockStage<TB, SW>::lload(lds + (q & 1) * SN, lane / SW, kb);
          if (run[0]) sub_kx(acc[0], kb, xn);
        } else if constexpr (!std::is_same<TB, double>::value) {
          // every system's neighbour vector is requested before the block is read back and
          // before any of them is used: one gather latency per slot, not one per system
          A xn[P][12];
#pragma unroll
          for (int j = 0; j < P; ++j)
            if (run[j]) load_vec(xr + vs[j] * 12, xn[j]);
          __builtin_amdgcn_wave_barrier();
          A kb[36];
          BlockStage<TB, SW>::lload(lds + (q & 1) * SN, lane / SW, kb);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!run[j]) continue;
            if (PH && p.ent_phase) apply_phase(p, slot * kLanes + rl, orow[j], xn[j]);
            sub_kx(acc[j], kb, xn[j]);
          }
        } else {
          __builtin_amdgcn_wave_barrier();
          A kb[36];
          BlockStage<TB, SW>::lload(lds + (q & 1) * SN, lane / SW, kb);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!run[j]) continue;
            A xn[12];
            load_vec(xr + vs[j] * 12, xn);
            if (PH && p.ent_phase) apply_phase(p, slot * kLanes + rl, orow[j], xn);
            sub_kx(acc[j], kb, xn);
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (q + 1 < wd) stg.lstore(lds + ((q + 1) & 1) * SN, lane);
      }
    } else if (wd == 6) {
#pragma unroll
      for (int q = 0; q < 6; ++q) body(q);
    } else {
      for (int q = 0; q < wd; ++q) body(q);
    }
  }
  if constexpr (kDiagLds) {
    __builtin_amdgcn_wave_barrier();
    BlockStage<TB, SW>::lload(lds + 2 * SN, lane / SW, d);
  }
  if constexpr (UPDATE && !std::is_same<TB, double>::value) {
    // FP16 factor inverses: system j + 1's factor row is requested before system j's
    // norm reduction and update, so its latency overlaps j's work; j's own x is requested
    // before j's factor solve
    HfacInv f[2];
    auto request = [&](int j) {
      if (run[j]) f[j & 1].load(dinv + (int64_t)ds[j] * dstride + tile * DinvTile<hfac>::N, rl);
    };
    request(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      double n2 = (valid && run[j]) ? norm2_12(acc[j]) : 0.0;
#pragma unroll
      for (int o = 32; o >= SW; o >>= 1) n2 += __shfl_xor(n2, o, 64);
      if (lane < SW && j * SW + lane < sb.n && run[j])
        partial[((int64_t)vs[j] * p.n_tiles + tile) * kPartialSlots + w] = n2;
      if (j + 1 < P) request(j + 1);
      if (!run[j]) continue;
      A xo[12];
      if (valid) load_vec(x + rb + vs[j] * 12, xo);
      A y[12];
      f[j & 1].apply(acc[j], y);
      if (valid) {
#pragma unroll
        for (int i = 0; i < 12; ++i) y[i] += xo[i];
        store_vec(x + rb + vs[j] * 12, y);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (UPDATE) {
      double n2 = (valid && run[j]) ? norm2_12(acc[j]) : 0.0;
#pragma unroll
      for (int o = 32; o >= SW; o >>= 1) n2 += __shfl_xor(n2, o, 64);
      if (lane < SW && j * SW + lane < sb.n && run[j])
        partial[((int64_t)vs[j] * p.n_tiles + tile) * kPartialSlots + w] = n2;
    }
    if (!run[j]) continue;
    if (UPDATE) {
      A y[12];
      apply_dinv(dinv + (int64_t)ds[j] * dstride + tile * DinvTile<typename DF_of<TB>::T>::N, rl, acc[j], y);
      if (valid) {
        A xi[12];
        load_vec(x + rb + vs[j] * 12, xi);
#pragma unroll
        for (int i = 0; i < 12; ++i) y[i] += xi[i];
        store_vec(x + rb + vs[j] * 12, y);
      }
    } else {
      if (valid) {
        csolve6_shift<PIVOT>(d, (A)shift_w(p, orow[j], row), acc[j]);
        store_vec(x + rb + vs[j] * 12, acc[j]);
      }
    }
  }
}



template <typename TB, int SW, int P, bool UPDATE, bool PIVOT, bool PH>
__global__ void __launch_bounds__(256)
k_rb_pass(DevPattern p, const TB* __restrict__ offd, const TB* __restrict__ diag,
          const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride, typename TV_of<TB>::T* __restrict__ x,
          const typename TV_of<TB>::T* __restrict__ b, int ns, SysBatch sb, SysState* st,
          double* __restrict__ partial, int64_t t0, int64_t nt, int wave_groups, FusedReduce fr) {
  // first-colour pass: the first fr.n workgroups reduce the preceding update pass's norms
  // (one system each) while the others sweep.  The sweeping workgroups read each
  // system's `active` flag while a reducing workgroup may be rewriting that state: a
  // system the reduction retires (it was pending) may or may not be swept here, and both
  // are right, because its update pass did not run this sweep (pending systems skip
  // it), so this pass would recompute exactly the x it computed last sweep.  The flags
  // the sweeping workgroups act on are otherwise unchanged by the reduction (it only
  // turns pending systems off and running ones pending).
  int64_t blk = blockIdx.x;
  if (!UPDATE && fr.n > 0) {
    if (blk < fr.n) {
      fused_sweep_reduce(fr, sb, partial, p.n_tiles, st, (int)blk);
      return;
    }
    blk -= fr.n;
  }
  // a tile's SW waves in one workgroup, or (wave_groups) one workgroup per wave: finer
  // dispatch granularity, the tile's waves still adjacent on one XCD
  int64_t tile;
  int grp;
  if (!map_tile_b(nt, wave_groups ? SW : 1, blk, tile, grp)) return;
  const int w = wave_groups ? grp : (int)(threadIdx.x >> 6);
  uint4* lds = nullptr;
  if constexpr (rb_lds_path<TB, SW, P, UPDATE, PH>()) {
    extern __shared__ uint4 rb_lds[];
    lds = rb_lds + (threadIdx.x >> 6) * rb_lds_chunks_t<TB, UPDATE>();
  }
  rb_tile<TB, SW, P, UPDATE, PIVOT, PH>(p, offd, diag, dinv, dstride, x, b, ns, sb, st, partial, t0 + tile, w, lds);
}

// Batched form: one launch over the concatenated (instance, tile) work list of many
// independent instances; each workgroup reads its instance's descriptor.
template <typename TB, int SW, int P, bool UPDATE, bool PIVOT>
__global__ void __launch_bounds__(256) k_rb_batched(const InstDesc* __restrict__ inst,
                                                    const WorkItem* __restrict__ work, int64_t n_work,
                                                    int wave_groups, const WorkItem* __restrict__ red, int n_red,
                                                    int red_mode, double rtol2, double div2) {
  using A = typename TV_of<TB>::T;
  int64_t blk = blockIdx.x;
  if (!UPDATE && n_red > 0) {
    // the preceding update pass's norm reductions, one (instance, system) per workgroup
    if (blk < n_red) {
      const WorkItem it = red[blk];
      const InstDesc& D = inst[it.inst];
      FusedReduce fr;
      fr.n = 1;
      fr.slots = D.slots;
      fr.mode = red_mode;
      fr.t0 = D.c1_t0;
      fr.nt = D.c1_nt;
      fr.rtol2 = rtol2;
      fr.div2 = div2;
      fused_sweep_reduce(fr, D.sb, D.partial, D.p.n_tiles, D.st, it.tile);
      return;
    }
    blk -= n_red;
  }
  int64_t k;
  int grp;
  if (!map_tile_b(n_work, wave_groups ? SW : 1, blk, k, grp)) return;
  const int w = wave_groups ? grp : (int)(threadIdx.x >> 6);
  const WorkItem wi = work[k];
  const InstDesc& D = inst[wi.inst];
  const bool pivot = D.pivot;
  uint4* lds = nullptr;
  if constexpr (rb_lds_path<TB, SW, P, UPDATE, true>()) {
    extern __shared__ uint4 rbb_lds[];
    lds = rbb_lds + (threadIdx.x >> 6) * rb_lds_chunks_t<TB, UPDATE>();
  }
  if (!UPDATE && !pivot)
    rb_tile<TB, SW, P, UPDATE, false>(D.p, (const TB*)D.offd, (const TB*)D.diag, (const typename DF_of<TB>::T*)D.dinv, D.dstride,
                                      (A*)D.x, (const A*)D.b, D.ns, D.sb, D.st, D.partial, wi.tile, w, lds);
  else
    rb_tile<TB, SW, P, UPDATE, true>(D.p, (const TB*)D.offd, (const TB*)D.diag, (const typename DF_of<TB>::T*)D.dinv, D.dstride,
                                     (A*)D.x, (const A*)D.b, D.ns, D.sb, D.st, D.partial, wi.tile, w, lds);
}

// Systems of one lane when SW lanes share a row: batch entries k = j * SW + sidx.
template <int SW, int P>
__device__ inline bool row_systems(const SysBatch& sb, const SysState* __restrict__ st, int sidx, bool norm_pass,
                                   WaveSys<P>& W) {
  bool any = false;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int k = j * SW + sidx;
    W.run[j] = false;
    W.vs[j] = 0;
    W.orow[j] = 0;
    W.ds[j] = 0;
    if (k < sb.n) {
      W.vs[j] = sb.vslot[k];
      W.orow[j] = sb.orow[k];
      W.ds[j] = sb.dslot[k];
      const int act = st[W.vs[j]].active, pen = st[W.vs[j]].pending;
      W.run[j] = norm_pass ? (act && !pen) : (act != 0);
      any |= W.run[j];
    }
  }
  return any;
}

// General colouring, forward pass of colour c (rows of lower colours are < cstart):
//   r_i = b_i - (K_ii + i w) x_i - sum_k K_ik x_k      (accumulated into ||r||^2)
//   y_i = Dt_i^-1 (r_i - sum_{k lower} K_ik y_k);  LAST colour: x_i += y_i (z = y there)
// Lane mapping as in the two-colour pass: SW lanes share a row (one block fetch serves
// all of them), each carrying P systems; a 64-row tile takes SW waves; the norm of
// system k over the rows of wave w goes to partial slot w.
//
// Two further modes serve the two-colours-plus-remainder sweep (see one_sweep), where
// x is updated in place colour by colour, so that b - K x already holds the lower
// colours' corrections (the forward substitution of the DILU step):
//   kFwdHybrid: y_i = Dt_i^-1 (b - K x)_i, stored, and x_i += y_i; no norm.
//   kFwdNorm:   only ||(b - K x)_i||^2 into the partials (the rows' residual at the
//               iterate the sweep starts from); nothing is written.
template <typename TB, int SW, int P, int MODE>
__global__ void __launch_bounds__(256) k_fwd(DevPattern p, const TB* __restrict__ offd, const TB* __restrict__ diag,
                                             const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride,
                                             typename TV_of<TB>::T* __restrict__ x,
                                             const typename TV_of<TB>::T* __restrict__ b,
                                             typename TV_of<TB>::T* __restrict__ y, int ns, SysBatch sb,
                                             const SysState* __restrict__ st, double* __restrict__ partial,
                                             int64_t t0, int64_t nt, int64_t cstart, int wave_groups) {
  using A = typename TV_of<TB>::T;
  // a tile's SW waves in one workgroup, or (wave_groups) one workgroup per wave
  int64_t tile;
  int grp;
  if (!map_tile(nt, wave_groups ? SW : 1, tile, grp)) return;
  tile += t0;
  const int lane = threadIdx.x & 63;
  const int w = wave_groups ? grp : (int)(threadIdx.x >> 6);
  const int sidx = lane % SW;
  const int rl = w * (kLanes / SW) + lane / SW;
  WaveSys<P> W;
  const bool any = row_systems<SW, P>(sb, st, sidx, true, W);
  if (!__any(any)) return;
  const int64_t row = tile * kLanes + rl;
  const bool valid = rl < p.tile_nrows[tile];
  const int64_t rb = row * ns * 12;
  constexpr bool kLowerY = MODE == kFwdGeneral || MODE == kFwdLast;
  // FP32/BF16 blocks: each step's loads for all of a lane's systems are requested
  // before any of them is used (one latency per step, not one per system)
  constexpr bool kBatch = !std::is_same<TB, double>::value;
  A r[P][12], t[P][kLowerY ? 12 : 1];
  if constexpr (kBatch) {
    A xi[P][12];
#pragma unroll
    for (int j = 0; j < P; ++j) {
#pragma unroll
      for (int i = 0; i < 12; ++i) r[j][i] = 0;
#pragma unroll
      for (int i = 0; i < (kLowerY ? 12 : 1); ++i) t[j][i] = 0;
      if (!W.run[j]) continue;
      load_vec(b + rb + W.vs[j] * 12, r[j]);
      load_vec(x + rb + W.vs[j] * 12, xi[j]);
    }
    A d[36];
    load_block(diag + tile * slot_elems<TB>(), rl, d);
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (W.run[j]) sub_diag_shift(r[j], d, (A)shift_w(p, W.orow[j], row), xi[j]);
  } else {
    A d[36];
    load_block(diag + tile * slot_elems<TB>(), rl, d);
#pragma unroll
    for (int j = 0; j < P; ++j) {
#pragma unroll
      for (int i = 0; i < 12; ++i) r[j][i] = 0;
#pragma unroll
      for (int i = 0; i < (kLowerY ? 12 : 1); ++i) t[j][i] = 0;
      if (!W.run[j]) continue;
      A xi[12];
      load_vec(b + rb + W.vs[j] * 12, r[j]);
      load_vec(x + rb + W.vs[j] * 12, xi);
      sub_diag_shift(r[j], d, (A)shift_w(p, W.orow[j], row), xi);
    }
  }
  const int wd = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  auto body = [&](int64_t slot, int nb, const A(&kb)[36]) {
    const int64_t nbo = (int64_t)nb * ns * 12;
    const bool lower = nb < cstart;
    if constexpr (kBatch) {
      A v[P][12];
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (W.run[j]) load_vec(x + nbo + W.vs[j] * 12, v[j]);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        if (!W.run[j]) continue;
        if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v[j]);
        sub_kx(r[j], kb, v[j]);
      }
      if constexpr (kLowerY) {
        if (lower) {
#pragma unroll
          for (int j = 0; j < P; ++j)
            if (W.run[j]) load_vec(y + nbo + W.vs[j] * 12, v[j]);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!W.run[j]) continue;
            if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v[j]);
            sub_kx(t[j], kb, v[j]);
          }
        }
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      A v[12];
      load_vec(x + nbo + W.vs[j] * 12, v);
      if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v);
      sub_kx(r[j], kb, v);
      if constexpr (kLowerY) {
        if (lower) {
          load_vec(y + nbo + W.vs[j] * 12, v);
          if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v);
          sub_kx(t[j], kb, v);
        }
      }
    }
  };
  if constexpr (gen_lds_path<TB, SW>()) {
    // blocks staged through LDS (see BlockStage), two buffers
    extern __shared__ uint4 gen_lds[];
    constexpr int SN = BlockStage<TB, SW>::N;
    uint4* lds = gen_lds + (threadIdx.x >> 6) * 2 * SN;  // this workgroup's wave slot
    const int rowbase = w * (kLanes / SW);
    BlockStage<TB, SW> stg;
    if (wd > 0) {
      stg.gload(offd + s0 * slot_elems<TB>(), rowbase, lane, KeepAll());
      stg.lstore(lds, lane);
    }
    int nb_next = wd > 0 ? p.ent_nbr[s0 * kLanes + rl] : 0;  // one slot ahead
    for (int q = 0; q < wd; ++q) {
      const int nb = nb_next;
      if (q + 1 < wd) {
        stg.gload(offd + (s0 + q + 1) * slot_elems<TB>(), rowbase, lane, KeepAll());
        nb_next = p.ent_nbr[(s0 + q + 1) * kLanes + rl];
      }
      const int64_t slot = s0 + q;
      __builtin_amdgcn_wave_barrier();
      A kb[36];
      BlockStage<TB, SW>::lload(lds + (q & 1) * SN, lane / SW, kb);
      body(slot, nb, kb);
      __builtin_amdgcn_wave_barrier();
      if (q + 1 < wd) stg.lstore(lds + ((q + 1) & 1) * SN, lane);
    }
  } else {
    for (int q = 0; q < wd; ++q) {
      const int64_t slot = s0 + q;
      const int nb = p.ent_nbr[slot * kLanes + rl];
      A kb[36];
      load_block(offd + slot * slot_elems<TB>(), rl, kb);
      body(slot, nb, kb);
    }
  }
  if constexpr (kBatch && MODE != kFwdNorm) {
    // system j + 1's factor row is requested before system j's reduction and solve
    HfacInv f[2];
    auto request = [&](int j) {
      if (W.run[j]) f[j & 1].load(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<hfac>::N, rl);
    };
    request(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (W.run[j]) mask_frozen(p, W.orow[j], r[j]);
      if constexpr (MODE != kFwdHybrid) {
        double n2 = (valid && W.run[j]) ? norm2_12(r[j]) : 0.0;
#pragma unroll
        for (int o = 32; o >= SW; o >>= 1) n2 += __shfl_xor(n2, o, 64);
        if (lane < SW && j * SW + lane < sb.n && W.run[j])
          partial[((int64_t)W.vs[j] * p.n_tiles + tile) * kPartialSlots + w] = n2;
      }
      if (j + 1 < P) request(j + 1);
      if (!W.run[j]) continue;
      constexpr bool kAddX = MODE == kFwdLast || MODE == kFwdHybrid;
      A xi[12];
      if (kAddX && valid) load_vec(x + rb + W.vs[j] * 12, xi);
      A yi[12];
      if constexpr (kLowerY) {
#pragma unroll
        for (int i = 0; i < 12; ++i) t[j][i] += r[j][i];
        f[j & 1].apply(t[j], yi);
      } else {
        f[j & 1].apply(r[j], yi);
      }
      if (valid) {
        store_vec(y + rb + W.vs[j] * 12, yi);
        if (kAddX) {
#pragma unroll
          for (int i = 0; i < 12; ++i) xi[i] += yi[i];
          store_vec(x + rb + W.vs[j] * 12, xi);
        }
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (W.run[j]) mask_frozen(p, W.orow[j], r[j]);
    if constexpr (MODE != kFwdHybrid) {
      double n2 = (valid && W.run[j]) ? norm2_12(r[j]) : 0.0;
#pragma unroll
      for (int o = 32; o >= SW; o >>= 1) n2 += __shfl_xor(n2, o, 64);
      if (lane < SW && j * SW + lane < sb.n && W.run[j])
        partial[((int64_t)W.vs[j] * p.n_tiles + tile) * kPartialSlots + w] = n2;
    }
    if (MODE == kFwdNorm || !W.run[j]) continue;
    A yi[12];
    if constexpr (kLowerY) {
#pragma unroll
      for (int i = 0; i < 12; ++i) t[j][i] += r[j][i];
      apply_dinv(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<typename DF_of<TB>::T>::N, rl, t[j], yi);
    } else {
      apply_dinv(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<typename DF_of<TB>::T>::N, rl, r[j], yi);
    }
    if (valid) {
      store_vec(y + rb + W.vs[j] * 12, yi);
      if (MODE == kFwdLast || MODE == kFwdHybrid) {
        A xi[12];
        load_vec(x + rb + W.vs[j] * 12, xi);
#pragma unroll
        for (int i = 0; i < 12; ++i) xi[i] += yi[i];
        store_vec(x + rb + W.vs[j] * 12, xi);
      }
    }
  }
}

// General colouring, backward pass of colour c (rows of higher colours are >= cend and
// already hold z in y):  z_i = y_i - Dt_i^-1 sum_{k upper} K_ik z_k;  x_i += z_i; y_i <- z_i
// In the two-colours-plus-remainder sweep x already holds x + y (kFwdHybrid), so
//   kBwdHybrid:  d_i = -Dt_i^-1 sum_{k upper} K_ik z_k;  x_i += d_i;  y_i += d_i (= z_i)
// and, with no reduction since the update pass, it runs for the systems that pass ran.
template <typename TB, int SW, int P, int MODE>
__global__ void __launch_bounds__(256) k_bwd(DevPattern p, const TB* __restrict__ offd,
                                             const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride,
                                             typename TV_of<TB>::T* __restrict__ x,
                                             typename TV_of<TB>::T* __restrict__ y, int ns, SysBatch sb,
                                             const SysState* __restrict__ st, int64_t t0, int64_t nt, int64_t cend,
                                             int wave_groups) {
  using A = typename TV_of<TB>::T;
  int64_t tile;
  int grp;
  if (!map_tile(nt, wave_groups ? SW : 1, tile, grp)) return;
  tile += t0;
  const int lane = threadIdx.x & 63;
  const int w = wave_groups ? grp : (int)(threadIdx.x >> 6);
  const int sidx = lane % SW;
  const int rl = w * (kLanes / SW) + lane / SW;
  WaveSys<P> W;
  const bool any = row_systems<SW, P>(sb, st, sidx, MODE != kBwdGeneral, W);
  if (!__any(any)) return;
  const int64_t row = tile * kLanes + rl;
  const bool valid = rl < p.tile_nrows[tile];
  const int64_t rb = row * ns * 12;
  A t[P][12];
#pragma unroll
  for (int j = 0; j < P; ++j)
#pragma unroll
    for (int i = 0; i < 12; ++i) t[j][i] = 0;
  const int wd = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  // FP32/BF16 blocks: each step's loads for all of a lane's systems are requested
  // before any of them is used (one latency per step, not one per system)
  constexpr bool kBatch = !std::is_same<TB, double>::value;
  auto body = [&](int64_t slot, int nb, const A(&kb)[36]) {
    const int64_t nbo = (int64_t)nb * ns * 12;
    if constexpr (kBatch) {
      A v[P][12];
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (W.run[j]) load_vec(y + nbo + W.vs[j] * 12, v[j]);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        if (!W.run[j]) continue;
        if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v[j]);
        sub_kx(t[j], kb, v[j]);
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      A v[12];
      load_vec(y + nbo + W.vs[j] * 12, v);
      if (p.ent_phase) apply_phase(p, slot * kLanes + rl, W.orow[j], v);
      sub_kx(t[j], kb, v);
    }
  };
  if constexpr (gen_lds_path<TB, SW>()) {
    // blocks staged through LDS (see BlockStage), two buffers; only the rows whose
    // coupling goes to a higher colour fetch theirs
    extern __shared__ uint4 gen_lds[];
    constexpr int SN = BlockStage<TB, SW>::N;
    uint4* lds = gen_lds + (threadIdx.x >> 6) * 2 * SN;  // this workgroup's wave slot
    const int rowbase = w * (kLanes / SW);
    BlockStage<TB, SW> stg;
    auto upper = [&](int64_t slot) {
      return [=](int i) { return p.ent_nbr[slot * kLanes + rowbase + i] >= cend; };
    };
    if (wd > 0) {
      stg.gload(offd + s0 * slot_elems<TB>(), rowbase, lane, upper(s0));
      stg.lstore(lds, lane);
    }
    int nb_next = wd > 0 ? p.ent_nbr[s0 * kLanes + rl] : 0;  // one slot ahead
    for (int q = 0; q < wd; ++q) {
      const int nb = nb_next;
      if (q + 1 < wd) {
        stg.gload(offd + (s0 + q + 1) * slot_elems<TB>(), rowbase, lane, upper(s0 + q + 1));
        nb_next = p.ent_nbr[(s0 + q + 1) * kLanes + rl];
      }
      const int64_t slot = s0 + q;
      __builtin_amdgcn_wave_barrier();
      if (nb >= cend) {
        A kb[36];
        BlockStage<TB, SW>::lload(lds + (q & 1) * SN, lane / SW, kb);
        body(slot, nb, kb);
      }
      __builtin_amdgcn_wave_barrier();
      if (q + 1 < wd) stg.lstore(lds + ((q + 1) & 1) * SN, lane);
    }
  } else {
    for (int q = 0; q < wd; ++q) {
      const int64_t slot = s0 + q;
      const int nb = p.ent_nbr[slot * kLanes + rl];
      if (nb >= cend) {
        A kb[36];
        load_block(offd + slot * slot_elems<TB>(), rl, kb);
        body(slot, nb, kb);
      }
    }
  }
  HfacInv f[kBatch ? 2 : 1];
  auto request = [&](int j) {
    if constexpr (kBatch)
      if (W.run[j]) f[j & 1].load(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<hfac>::N, rl);
  };
  request(0);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (j + 1 < P) request(j + 1);  // the next system's factor row while this one is solved
    if (!W.run[j]) continue;
    A z[12], yi[12], xi[12];
    if (valid) {
      load_vec(y + rb + W.vs[j] * 12, yi);
      load_vec(x + rb + W.vs[j] * 12, xi);
    }
    if constexpr (kBatch)
      f[j & 1].apply(t[j], z);
    else
      apply_dinv(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<typename DF_of<TB>::T>::N, rl, t[j], z);
    if (valid) {
      if constexpr (MODE == kBwdGeneral) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          z[i] += yi[i];
          xi[i] += z[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          xi[i] += z[i];
          if constexpr (MODE == kBwdHybrid) z[i] += yi[i];
        }
      }
      store_vec(y + rb + W.vs[j] * 12, z);
      store_vec(x + rb + W.vs[j] * 12, xi);
    }
  }
}

// The correction of the two-colours-plus-remainder sweep: every second-colour row coupled
// to a higher colour gets x_i += -Dt_i^-1 sum_{k upper} K_ik z_k (z of the remainder in
// y), the same update as the backward step without z.  The rows are packed 64 to a group
// with their upward couplings (flat entries of the SELL layout, in slot order), one wave
// per group and P systems, so the launch touches only those rows (about one in
// seventy of the second colour on a three-row sector).
template <typename TB, int P>
__global__ void __launch_bounds__(64) k_correct(DevPattern p, CorrDev q, const TB* __restrict__ offd,
                                                const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride,
                                                typename TV_of<TB>::T* __restrict__ x,
                                                const typename TV_of<TB>::T* __restrict__ y, int ns, SysBatch sb,
                                                const SysState* __restrict__ st) {
  using A = typename TV_of<TB>::T;
  const int64_t g = blockIdx.x;
  const int lane = threadIdx.x;
  WaveSys<P> W;
  if (!wave_systems<P>(sb, st, (int)blockIdx.y, true, W)) return;
  const int32_t row = q.row[g * kLanes + lane];
  if (row < 0) return;
  A t[P][12];
#pragma unroll
  for (int j = 0; j < P; ++j)
#pragma unroll
    for (int i = 0; i < 12; ++i) t[j][i] = 0;
  const int wd = q.width[g];
  const int64_t s0 = q.slot0[g];
  // The latency chain of a wave is the launch time (a few hundred waves): the entry and
  // neighbour indices of up to eight couplings are requested in two rounds, then each
  // coupling's block and its neighbour's z for every system in one.
  constexpr int kIdx = 8;
  bool more = true;
  for (int k0 = 0; k0 < wd && more; k0 += kIdx) {
    int32_t fe[kIdx], nb[kIdx];
#pragma unroll
    for (int u = 0; u < kIdx; ++u) fe[u] = k0 + u < wd ? q.fe[(s0 + k0 + u) * kLanes + lane] : -1;
#pragma unroll
    for (int u = 0; u < kIdx; ++u) nb[u] = fe[u] >= 0 ? p.ent_nbr[fe[u]] : 0;
#pragma unroll
    for (int u = 0; u < kIdx; ++u) {
      if (fe[u] < 0) {
        more = false;
        break;
      }
      const int64_t nbo = (int64_t)nb[u] * ns * 12;
      A v[P][12];
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (W.run[j]) load_vec(y + nbo + W.vs[j] * 12, v[j]);
      A kb[36];
      load_block(offd + (int64_t)(fe[u] >> 6) * slot_elems<TB>(), fe[u] & 63, kb);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        if (!W.run[j]) continue;
        if (p.ent_phase) apply_phase(p, fe[u], W.orow[j], v[j]);
        sub_kx(t[j], kb, v[j]);
      }
    }
  }
  const int64_t rb = (int64_t)row * ns * 12;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (!W.run[j]) continue;
    A z[12], xi[12];
    load_vec(x + rb + W.vs[j] * 12, xi);
    apply_dinv(dinv + (int64_t)W.ds[j] * dstride + (int64_t)(row >> 6) * DinvTile<typename DF_of<TB>::T>::N, row & 63,
               t[j], z);
#pragma unroll
    for (int i = 0; i < 12; ++i) xi[i] += z[i];
    store_vec(x + rb + W.vs[j] * 12, xi);
  }
}

// Block Jacobi (the paper's explicit, point-by-point inversion): y = D_s^-1 (b - K_s x)
// over all rows, then x += y.
template <typename TB, int P>
__global__ void __launch_bounds__(256) k_jacobi(DevPattern p, const TB* __restrict__ offd,
                                                const TB* __restrict__ diag,
                                                const typename DF_of<TB>::T* __restrict__ dinv, int64_t dstride,
                                                const typename TV_of<TB>::T* __restrict__ x,
                                                const typename TV_of<TB>::T* __restrict__ b,
                                                typename TV_of<TB>::T* __restrict__ y, int ns, SysBatch sb,
                                                const SysState* __restrict__ st, double* __restrict__ partial) {
  using A = typename TV_of<TB>::T;
  int64_t tile;
  int grp;
  if (!map_tile(p.n_tiles, 1, tile, grp)) return;
  const int lane = threadIdx.x & 63;
  WaveSys<P> W;
  if (!wave_systems<P>(sb, st, threadIdx.x >> 6, true, W)) return;
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  const int64_t rb = row * ns * 12;
  A r[P][12];
  {
    A d[36];
    load_block(diag + tile * slot_elems<TB>(), lane, d);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      A xi[12];
      load_vec(b + rb + W.vs[j] * 12, r[j]);
      load_vec(x + rb + W.vs[j] * 12, xi);
      sub_diag_shift(r[j], d, (A)shift_w(p, W.orow[j], row), xi);
    }
  }
  gather_offd<TB, A, P>(p, offd, x, ns, tile, lane, W, r);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (!W.run[j]) continue;
    mask_frozen(p, W.orow[j], r[j]);
    const double n2 = wave_sum(valid ? norm2_12(r[j]) : 0.0);
    if (lane == 0) partial[((int64_t)W.vs[j] * p.n_tiles + tile) * kPartialSlots] = n2;
    A yi[12];
    apply_dinv(dinv + (int64_t)W.ds[j] * dstride + tile * DinvTile<typename DF_of<TB>::T>::N, lane, r[j], yi);
    if (valid) store_vec(y + rb + W.vs[j] * 12, yi);
  }
}

// x += y for the active systems (interleaved layout), also used for the FP64 update.
template <typename A>
__global__ void k_axpy_y(int64_t NP, int ns, A* __restrict__ x, const A* __restrict__ y, SysBatch sb,
                         const SysState* __restrict__ st) {
  const int k = blockIdx.y;
  const int vs = sb.vslot[k];
  if (!st[vs].active) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP * 12) return;
  const int64_t o = (i / 12) * ns * 12 + vs * 12 + (i % 12);
  x[o] += y[o];
}

// ================================================================ norm reduction
// Sum the norm partials of one system in a fixed order and advance its state.
__device__ inline void reduce_one(const double* __restrict__ partial, int64_t n_tiles, int64_t t0, int64_t nt,
                                  int slots, SysState* __restrict__ st, int vs, int mode, double rtol2, double div2,
                                  int max_sweeps) {
  const double* pp = partial + ((int64_t)vs * n_tiles + t0) * kPartialSlots;
  const double n2 = canonical_sum(pp, mode != kReduceSweepNoNorm ? nt : 0, slots);
  if (threadIdx.x != 0) return;
  SysState S = st[vs];
  switch (mode) {
    case kReduceInit:
      S.norm0sq = n2;
      S.last_n2 = n2;
      S.hist = nullptr;
      S.hist_len = 0;
      S.hist_off = 0;
      S.sweeps = 0;
      S.pending = 0;
      S.outer_iters = 0;
      S.limit = max_sweeps;
      if (!isfinite(n2)) {
        S.status = kDiverged;
        S.active = 0;
      } else {
        S.status = n2 > 0.0 ? kNotConverged : kOK;
        S.active = (n2 > 0.0 && max_sweeps > 0) ? 1 : 0;
      }
      break;
    case kReduceSweep:
    case kReduceSweepNoNorm:
      sweep_state(S, n2, mode, rtol2, div2);
      break;
    case kReduceFinal:
      S.last_n2 = n2;
      break;
    case kReduceOuter:
      S.last_n2 = n2;
      if (!S.active) break;
      if (S.hist && S.sweeps < S.hist_len) S.hist[S.sweeps] = n2;  // the FP64 norm after a correction
      if (n2 <= rtol2 * S.norm0sq) {
        S.status = kOK;
        S.active = 0;
      } else if (!isfinite(n2) || n2 > div2 * S.norm0sq) {
        S.status = kDiverged;
        S.active = 0;
      } else if (S.sweeps >= S.limit) {
        S.status = kNotConverged;
        S.active = 0;
      }
      break;
  }
  st[vs] = S;
}

__global__ void __launch_bounds__(256) k_reduce(SysBatch sb, const double* __restrict__ partial, int64_t n_tiles,
                                                int64_t t0, int64_t nt, int slots, SysState* __restrict__ st,
                                                int mode, double rtol2, double div2, int max_sweeps) {
  reduce_one(partial, n_tiles, t0, nt, slots, st, sb.vslot[blockIdx.x], mode, rtol2, div2, max_sweeps);
}

// Batched reduction: one workgroup per (instance, system) item, over the instance's
// second-colour tiles.
__global__ void __launch_bounds__(256) k_reduce_batched(const InstDesc* __restrict__ inst,
                                                        const WorkItem* __restrict__ items, int mode, double rtol2,
                                                        double div2) {
  const WorkItem it = items[blockIdx.x];
  const InstDesc& D = inst[it.inst];
  reduce_one(D.partial, D.p.n_tiles, D.c1_t0, D.c1_nt, D.slots, D.st, D.sb.vslot[it.tile], mode, rtol2, div2, 0);
}

__global__ void k_inner_init(SysBatch sb, const SysState* __restrict__ outer, SysState* __restrict__ inner,
                             int max_inner) {
  const int k = threadIdx.x;
  if (k >= sb.n) return;
  const int vs = sb.vslot[k];
  const SysState O = outer[vs];
  SysState I;
  I.norm0sq = O.last_n2;
  I.last_n2 = O.last_n2;
  I.pending = 0;
  I.sweeps = 0;
  I.outer_iters = 0;
  I.status = kNotConverged;
  I.hist = O.hist;
  I.hist_len = O.hist_len;
  I.hist_off = O.sweeps;
  int lim = O.limit - O.sweeps;
  if (lim > max_inner) lim = max_inner;
  I.limit = lim;
  I.active = (O.active && lim > 0 && O.last_n2 > 0.0) ? 1 : 0;
  inner[vs] = I;
}

__global__ void k_set_history(SysBatch sb, SysState* __restrict__ st, double* __restrict__ hist, int len) {
  const int k = threadIdx.x;
  if (k >= sb.n) return;
  const int vs = sb.vslot[k];
  SysState S = st[vs];
  S.hist = hist ? hist + (int64_t)vs * len : nullptr;
  S.hist_len = hist ? len : 0;
  S.hist_off = 0;
  if (S.hist && len > 0) S.hist[0] = S.norm0sq;
  st[vs] = S;
}

__global__ void k_outer_update(SysBatch sb, const SysState* __restrict__ inner, SysState* __restrict__ outer) {
  const int k = threadIdx.x;
  if (k >= sb.n) return;
  const int vs = sb.vslot[k];
  if (!outer[vs].active) return;
  outer[vs].sweeps += inner[vs].sweeps;
  outer[vs].outer_iters += 1;
}

// ================================================================ assembly
// First-order Rusanov Jacobian (frozen spectral radius), section "Generalized RK Scheme
// for The Mean Flow": for row i and neighbour k with area S_ik (outward from i),
//   K_ik = 1/2 A(Q_k; S_ik) - 1/2 lam_ik I,  lam_ik = max(rho(Q_i,S), rho(Q_k,S))
//   J_ii = sum over faces [1/2 A(Q_i; S) + 1/2 lam I] = 1/2 A(Q_i; sum S) + 1/2 (sum lam) I
// (A is linear in S), boundary faces against the frozen far-field state, and
// K_ii = (1 + 1/(eps sigma)) J_ii (implicit) / J_ii with no off-diagonal (explicit).
__device__ inline void load_state(const double* __restrict__ q, double (&Q)[6]) {
  const double2* p = reinterpret_cast<const double2*>(q);
  double2 a = p[0], b = p[1], c = p[2];
  Q[0] = a.x;
  Q[1] = a.y;
  Q[2] = b.x;
  Q[3] = b.y;
  Q[4] = c.x;
  Q[5] = c.y;
}

__device__ inline void entry_area(const DevFlow& f, int32_t e, double (&S)[3]) {
  const int64_t id = (e > 0 ? e : -e) - 1;
  const double sg = e > 0 ? 1.0 : -1.0;
  S[0] = sg * f.area[3 * id];
  S[1] = sg * f.area[3 * id + 1];
  S[2] = sg * f.area[3 * id + 2];
}

template <typename TB>
__global__ void __launch_bounds__(64) k_assemble(DevPattern p, DevFlow f, TB* __restrict__ offd,
                                                 TB* __restrict__ diag) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  double Qi[6] = {1, 0, 0, 0, 2.5, 0};
  if (valid) load_state(f.state + row * 6, Qi);
  double sumS[3] = {0, 0, 0}, lam_sum = 0.0;
  const int w = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  for (int q = 0; q < w; ++q) {
    const int64_t slot = s0 + q;
    const int64_t fe = slot * kLanes + lane;
    const int32_t e = p.ent_edge[fe];
    TB* dst = offd + slot * slot_elems<TB>();
    if (e == 0) {
#pragma unroll
      for (int c = 0; c < 36; ++c) store_entry<TB>(dst, c, lane, 0.0);
      continue;
    }
    double S[3], Qk[6], Ak[36];
    entry_area(f, e, S);
    load_state(f.state + (int64_t)p.ent_nbr[fe] * 6, Qk);
    const double lam = fmax(spectral_radius(Qi, S), spectral_radius(Qk, S));
    flux_jacobian(Qk, S, Ak);
    sumS[0] += S[0];
    sumS[1] += S[1];
    sumS[2] += S[2];
    lam_sum += lam;
#pragma unroll
    for (int c = 0; c < 36; ++c) {
      double v = 0.5 * Ak[c] - ((c % 7 == 0) ? 0.5 * lam : 0.0);
      store_entry<TB>(dst, c, lane, f.offdiag ? v : 0.0);
    }
  }
  if (valid) {
    for (int32_t j = f.bf_ptr[row]; j < f.bf_ptr[row + 1]; ++j) {
      const int32_t face = f.bf_idx[j];
      double S[3] = {f.bface_area[3 * face], f.bface_area[3 * face + 1], f.bface_area[3 * face + 2]};
      double Qf[6];
      if (f.bstate) {
        load_state(f.bstate + (int64_t)face * 6, Qf);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) Qf[c] = Qi[c];
      }
      lam_sum += fmax(spectral_radius(Qi, S), spectral_radius(Qf, S));
      sumS[0] += S[0];
      sumS[1] += S[1];
      sumS[2] += S[2];
    }
  }
  double Ai[36];
  flux_jacobian(Qi, sumS, Ai);
  TB* dst = diag + tile * slot_elems<TB>();
#pragma unroll
  for (int c = 0; c < 36; ++c) {
    double v = f.diag_scale * (0.5 * Ai[c] + ((c % 7 == 0) ? 0.5 * lam_sum : 0.0));
    store_entry<TB>(dst, c, lane, valid ? v : 0.0);
  }
}

// raw blocks: thread per (directed coupling | cell, entry)
template <typename TB>
__global__ void k_set_offd(int64_t E, const int64_t* __restrict__ edge_ent, const double* __restrict__ offd_user,
                           TB* __restrict__ offd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * E * 36) return;
  const int64_t d = t / 36;
  const int c = (int)(t % 36);
  const int64_t f = edge_ent[d];
  store_entry<TB>(offd + (f >> 6) * slot_elems<TB>(), c, (int)(f & 63), offd_user[t]);
}
template <typename TB>
__global__ void k_set_diag(int64_t N, const int32_t* __restrict__ perm, const double* __restrict__ diag_user,
                           TB* __restrict__ diag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * 36) return;
  const int64_t u = t / 36;
  const int c = (int)(t % 36);
  const int64_t row = perm[u];
  store_entry<TB>(diag + (row >> 6) * slot_elems<TB>(), c, (int)(row & 63), diag_user[t]);
}
template <typename TB>
__global__ void k_get_offd(int64_t E, const int64_t* __restrict__ edge_ent, const TB* __restrict__ offd,
                           double* __restrict__ offd_user) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * E * 36) return;
  const int64_t d = t / 36;
  const int c = (int)(t % 36);
  const int64_t f = edge_ent[d];
  offd_user[t] = load_entry_f64<TB>(offd + (f >> 6) * slot_elems<TB>(), c, (int)(f & 63));
}
template <typename TB>
__global__ void k_get_diag(int64_t N, const int32_t* __restrict__ perm, const TB* __restrict__ diag,
                           double* __restrict__ diag_user) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * 36) return;
  const int64_t u = t / 36;
  const int c = (int)(t % 36);
  const int64_t row = perm[u];
  diag_user[t] = load_entry_f64<TB>(diag + (row >> 6) * slot_elems<TB>(), c, (int)(row & 63));
}

// ================================================================ factorisation
// Colour c, one wave per (tile, system):
//   Dt_i = K_ii + i w_i I - sum_{k in N(i), col k < c} K_ik Dt_k^-1 K_ki   (DILU)
//   Dt_i = K_ii + i w_i I                                                (SGS / Jacobi)
// inverted by Gauss-Jordan with partial pivoting.  Arithmetic type F: FP64 with FP64
// blocks; FP32 with FP32/BF16 blocks, whose factor inverses are stored in FP16 (the FP64
// defect correction makes the factor's precision irrelevant to the converged result).
// Per lower neighbour k the two blocks are loaded whole, and T = Dt_k^-1 K_ki is formed
// row by row (one row of Dt_k^-1 per step) and folded into Dt_i as the rank-one update
// K_ik[:, r] T[r, :].
template <typename TB> struct Fact_of {
  using T = float;
};
template <> struct Fact_of<double> {
  using T = double;
};
// row r of Dt^-1 (six complex entries) of one lane's factor tile
template <typename TD, typename F>
__device__ inline void dinv_row_entries(const TD* __restrict__ t, int lane, int r, F (&dr)[6], F (&di)[6]);
template <typename F>
__device__ inline void dinv_row_entries(const double* __restrict__ t, int lane, int r, F (&dr)[6], F (&di)[6]) {
  const double2* p = reinterpret_cast<const double2*>(t) + lane;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double2 d = p[(6 * r + c) * kLanes];
    dr[c] = (F)d.x;
    di[c] = (F)d.y;
  }
}
template <typename F>
__device__ inline void dinv_row_entries(const hfac* __restrict__ t, int lane, int r, F (&dr)[6], F (&di)[6]) {
  const uint4* p = reinterpret_cast<const uint4*>(t) + lane;
  const int v0 = (6 * r) >> 2;
  const uint4 d0 = p[v0 * kLanes];
  const uint4 d1 = p[(v0 + 1) * kLanes];
  const uint32_t w[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
  const int o = 6 * r - 4 * v0;  // 0 or 2
  const F sc = (F)reinterpret_cast<const float*>(t + 72 * kLanes)[lane];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const uint32_t q = o ? w[c + 2] : w[c];
    dr[c] = (F)h2f(q & 0xffffu) * sc;
    di[c] = (F)h2f(q >> 16) * sc;
  }
}
template <typename TB, typename TD, bool DILU>
__global__ void __launch_bounds__(64) k_factor(DevPattern p, const TB* __restrict__ offd,
                                               const TB* __restrict__ diag, TD* __restrict__ dinv,
                                               int64_t dstride, SysBatch sb, int64_t t0, int64_t nt, int64_t cstart,
                                               int* __restrict__ err) {
  using F = typename Fact_of<TB>::T;
  // the systems of one tile are adjacent in dispatch order on one XCD, so the tile's
  // coupling blocks, read by every system, come from that XCD's L2 after the first
  int64_t tile;
  int k;
  if (!map_tile(nt, sb.n, tile, k)) return;
  tile += t0;
  const int lane = threadIdx.x;
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  F mr[36], mi[36];
  load_block(diag + tile * slot_elems<TB>(), lane, mr);
#pragma unroll
  for (int c = 0; c < 36; ++c) mi[c] = (F)0;
  const F wv = (F)shift_w(p, sb.orow[k], row);
#pragma unroll
  for (int c = 0; c < 6; ++c) mi[7 * c] += wv;
  TD* dbase = dinv + (int64_t)sb.dslot[k] * dstride;
  if (DILU) {
    const int w = p.tile_width[tile];
    const int64_t s0 = p.tile_slot0[tile];
    for (int q = 0; q < w; ++q) {
      const int64_t fe = (s0 + q) * kLanes + lane;
      const int nb = p.ent_nbr[fe];
      if (p.ent_edge[fe] == 0 || nb >= cstart) continue;
      F kij[36], kji[36];
      load_block(offd + (s0 + q) * slot_elems<TB>(), lane, kij);
      const int32_t rv = p.ent_rev[fe];
      load_block(offd + (int64_t)(rv >> 6) * slot_elems<TB>(), rv & 63, kji);
      const TD* dn = dbase + (int64_t)(nb >> 6) * DinvTile<TD>::N;
      const int nl = nb & 63;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        F dr[6], di[6];
        dinv_row_entries(dn, nl, r, dr, di);
        F tr[6], ti[6];  // row r of Dt_k^-1 K_ki
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          F sr = 0, si = 0;
#pragma unroll
          for (int q2 = 0; q2 < 6; ++q2) {
            sr += dr[q2] * kji[6 * q2 + c];
            si += di[q2] * kji[6 * q2 + c];
          }
          tr[c] = sr;
          ti[c] = si;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const F a = kij[6 * i + r];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            mr[6 * i + c] -= a * tr[c];
            mi[6 * i + c] -= a * ti[c];
          }
        }
      }
    }
  }
  // frozen turbulence: the inverse of the leading 5x5 block, sixth row and column zero
  const bool frz = p.sys_frozen && p.sys_frozen[sb.orow[k]];
  if (frz) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      mr[30 + c] = mi[30 + c] = (F)0;
      mr[6 * c + 5] = mi[6 * c + 5] = (F)0;
    }
    mr[35] = (F)1;
  }
  bool ok = true;
  cinv6(mr, mi, ok);
  if (frz) mr[35] = (F)0;
  if (valid && !ok) atomicOr(err, 1);
  if (!valid) {
#pragma unroll
    for (int c = 0; c < 36; ++c) {
      mr[c] = (F)0;
      mi[c] = (F)0;
    }
  }
  store_dinv(dbase + tile * DinvTile<TD>::N, lane, mr, mi);
}

// ================================================================ partition-local ILU(0)
// Section "Parallel Implementation": every partition runs ILU(0) on its own block of the
// LHS, the couplings to other partitions left out.  Inside a partition the order is the
// natural one (cell ids), processed level by level (cells of one level are never
// coupled): one workgroup per (work unit, systems), a unit being one or more whole
// partitions whose levels are merged (cells of different partitions are never coupled
// either), the unit's y vector in LDS.
// Blocks are read from packed copies in position order (PiluLayout), so the lanes of a
// wave, which take consecutive positions of one level, load coalesced 16-byte vectors.

// packed couplings and diagonal blocks: one thread per (entry or position, 16-byte chunk)
template <typename TB>
__global__ void k_pilu_pack(PiluDev q, const TB* __restrict__ offd, const TB* __restrict__ diag, TB* __restrict__ coup,
                            TB* __restrict__ pdiag) {
  constexpr int NV = Fmt<TB>::NV;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_ent = q.n_slots * kLanes, n_pos = q.n_groups * kLanes;
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  if (t < n_ent * NV) {
    const int64_t e = t / NV;
    const int v = (int)(t % NV);
    const int32_t src = q.e_src[e];
    const uint4 val =
        src < 0 ? zero : reinterpret_cast<const uint4*>(offd)[((int64_t)(src >> 6) * NV + v) * kLanes + (src & 63)];
    reinterpret_cast<uint4*>(coup)[((e >> 6) * NV + v) * kLanes + (e & 63)] = val;
  } else if (t < (n_ent + n_pos) * NV) {
    const int64_t k = t - n_ent * NV;
    const int64_t pos = k / NV;
    const int v = (int)(k % NV);
    const int32_t row = q.pos_row[pos];
    const uint4 val =
        row < 0 ? zero : reinterpret_cast<const uint4*>(diag)[((int64_t)(row >> 6) * NV + v) * kLanes + (row & 63)];
    reinterpret_cast<uint4*>(pdiag)[((pos >> 6) * NV + v) * kLanes + (pos & 63)] = val;
  }
}

// Dt_i = K_ii + i w_i I - sum_{j lower, same partition} K_ij Dt_j^-1 K_ji, level by level
// (one wave per (unit, system)); the inverses go to the factor slot in position
// order (tile g = position / 64).  The inverses of lower levels are read back from global
// memory after the workgroup barrier that ends their level: the wave wrote them itself.
template <typename TB, typename TD>
__global__ void __launch_bounds__(64) k_pilu_factor(DevPattern p, PiluDev q, const TB* __restrict__ coup,
                                                    const TB* __restrict__ pdiag, TD* dinv, int64_t dstride,
                                                    SysBatch sb, int* __restrict__ err) {
  const int64_t unit = blockIdx.x;
  const int k = blockIdx.y;
  const int lane = threadIdx.x;
  TD* dbase = dinv + (int64_t)sb.dslot[k] * dstride;
  const bool frz = p.sys_frozen && p.sys_frozen[sb.orow[k]];
  const int l0 = q.unit_lev[unit], l1 = q.unit_lev[unit + 1];
  for (int l = l0; l < l1; ++l) {
    const int a = q.lev_ptr[l], e = q.lev_ptr[l + 1];
    for (int qq = a + lane; qq < e; qq += kLanes) {
      const int64_t g = qq >> 6;
      const int ln = qq & 63;
      const int64_t row = q.pos_row[qq];
      double mr[36], mi[36];
      const TB* ds = pdiag + g * slot_elems<TB>();
#pragma unroll
      for (int c = 0; c < 36; ++c) {
        mr[c] = load_entry_f64<TB>(ds, c, ln);
        mi[c] = 0.0;
      }
      const double wv = shift_w(p, sb.orow[k], row);
#pragma unroll
      for (int c = 0; c < 6; ++c) mi[7 * c] += wv;
      const int wd = q.g_width[g];
      const int64_t s0 = q.g_slot0[g];
      for (int kk = 0; kk < wd; ++kk) {
        const int64_t fe = (s0 + kk) * kLanes + ln;
        const int nb = q.e_pos[fe];
        if (nb < 0 || nb > qq) break;  // lower neighbours come first
        const TB* ks = coup + (s0 + kk) * slot_elems<TB>();
        double kij[36];
#pragma unroll
        for (int c = 0; c < 36; ++c) kij[c] = load_entry_f64<TB>(ks, c, ln);
        const int32_t rv = q.e_rev[fe];
        const TB* rs = coup + (int64_t)(rv >> 6) * slot_elems<TB>();
        const int rl = rv & 63;
        const TD* dn = dbase + (int64_t)(nb >> 6) * DinvTile<TD>::N;
        const int nl = nb & 63;
        for (int c = 0; c < 6; ++c) {
          double kc[6];
#pragma unroll
          for (int q2 = 0; q2 < 6; ++q2) kc[q2] = load_entry_f64<TB>(rs, 6 * q2 + c, rl);
          double tr[6], ti[6];
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < 6; ++q2) {
              double dr, di;
              load_dinv_entry<TD>(dn, nl, 6 * r + q2, dr, di);
              sr += dr * kc[q2];
              si += di * kc[q2];
            }
            tr[r] = sr;
            ti[r] = si;
          }
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < 6; ++q2) {
              sr += kij[6 * r + q2] * tr[q2];
              si += kij[6 * r + q2] * ti[q2];
            }
            mr[6 * r + c] -= sr;
            mi[6 * r + c] -= si;
          }
        }
      }
      if (frz) {  // the inverse of the leading 5x5 block, sixth row and column zero
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          mr[30 + c] = mi[30 + c] = 0.0;
          mr[6 * c + 5] = mi[6 * c + 5] = 0.0;
        }
        mr[35] = 1.0;
      }
      bool ok = true;
      cinv6(mr, mi, ok);
      if (frz) mr[35] = 0.0;
      if (!ok) atomicOr(err, 1);
      store_dinv(dbase + g * DinvTile<TD>::N, ln, mr, mi);
    }
    __syncthreads();
  }
}

// Row r of y = Dinv a (complex 6x6 times complex 6) for one position's factor, in two
// steps: load() fetches the row (its address does not depend on the data it multiplies,
// so a sweep issues it before its other loads), apply() forms the row's product.  The
// products are accumulated with explicit fused multiply-adds in a fixed order, so the
// result does not depend on how the compiler contracts the kernel it is inlined in (the
// same for every number of systems a workgroup carries).
__device__ inline float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename A> __device__ inline void cmac(A dr, A di, A ar, A ai, A& yr, A& yi) {
  yr = fmad(dr, ar, yr);
  yr = fmad(-di, ai, yr);
  yi = fmad(dr, ai, yi);
  yi = fmad(di, ar, yi);
}
template <typename TD> struct DinvRow;
template <> struct DinvRow<double> {
  double2 d[6];
  __device__ inline void load(const double* __restrict__ t, int lane, int r) {
    const double2* p = reinterpret_cast<const double2*>(t) + lane;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const nt_d2 v = ld_stream(p + (6 * r + c) * kLanes);
      d[c] = make_double2(v.x, v.y);
    }
  }
  template <typename A> __device__ inline void apply(const A (&a)[12], A& yr, A& yi) const {
    yr = 0;
    yi = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) cmac((A)d[c].x, (A)d[c].y, a[2 * c], a[2 * c + 1], yr, yi);
  }
};
template <> struct DinvRow<hfac> {
  // entries 6r .. 6r+5 lie in the 16-byte vectors (6r)/4 and (6r)/4 + 1 (four per vector)
  uint4 d0, d1;
  float sc;
  int o;  // 0 or 2: the row's first entry within d0
  __device__ inline void load(const hfac* __restrict__ t, int lane, int r) {
    const uint4* p = reinterpret_cast<const uint4*>(t) + lane;
    const int v0 = (6 * r) >> 2;
    const nt_u4 a = ld_stream(p + v0 * kLanes);
    const nt_u4 b = ld_stream(p + (v0 + 1) * kLanes);
    d0 = make_uint4(a.x, a.y, a.z, a.w);
    d1 = make_uint4(b.x, b.y, b.z, b.w);
    sc = reinterpret_cast<const float*>(t + 72 * kLanes)[lane];
    o = 6 * r - 4 * v0;
  }
  template <typename A> __device__ inline void apply(const A (&a)[12], A& yr, A& yi) const {
    const uint32_t w[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    A sr = 0, si = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const uint32_t q = o ? w[c + 2] : w[c];
      cmac((A)h2f(q & 0xffffu), (A)h2f(q >> 16), a[2 * c], a[2 * c + 1], sr, si);
    }
    yr = sr * (A)sc;
    yi = si * (A)sc;
  }
};

// One preconditioned Richardson sweep of each unit for P systems:
//   forward, levels ascending:   r_i = b_i - (K_ii + i w) x_i - sum_j K_ij x_j   (||r||^2)
//                                y_i = Dt_i^-1 (r_i - sum_{j lower} K_ij y_j)
//   backward, levels descending: z_i = y_i - Dt_i^-1 sum_{j upper} K_ij z_j
//   x_i += z_i.
// y (then z) of the unit's rows lives in LDS, [row in unit][P][12]; x and b are the
// interleaved vectors [NP][ns][12].  A level's rows are taken NT/4 at a time by the
// workgroup's NT lanes (64, 128 or 256, after the units' level widths), four lanes per
// row: the row's blocks (its diagonal block and
// couplings) are dealt out to the four lanes in turn, their partial sums combined by
// shuffles within the quad, and each lane forms rows {s, s+4} of the factor solve.
// Cutting the work of a row four ways shortens the chain of dependent steps that every
// level adds to the sweep.
template <typename TB, int P, int NT>
__global__ void __launch_bounds__(NT) k_pilu_sweep(DevPattern p, PiluDev q, const TB* __restrict__ coup,
                                                             const TB* __restrict__ pdiag,
                                                             const typename DF_of<TB>::T* __restrict__ dinv,
                                                             int64_t dstride, typename TV_of<TB>::T* __restrict__ x,
                                                             const typename TV_of<TB>::T* __restrict__ b, int ns,
                                                             SysBatch sb, const SysState* __restrict__ st,
                                                             double* __restrict__ partial) {
  using A = typename TV_of<TB>::T;
  using TD = typename DF_of<TB>::T;
  extern __shared__ uint4 pilu_lds[];
  __shared__ double wsum[NT / kLanes][P];
  A* ys = reinterpret_cast<A*>(pilu_lds);
  const int64_t unit = blockIdx.x;
  const int sl = threadIdx.x & 3;    // lane within the row's quad
  const int slot = threadIdx.x >> 2;  // row slot, 64 per pass
  constexpr int kSlots = NT / 4;
  WaveSys<P> W;
  if (!wave_systems<P>(sb, st, (int)blockIdx.y, true, W)) return;
  const int q0 = q.unit_ptr[unit], q1 = q.unit_ptr[unit + 1];
  const int l0 = q.unit_lev[unit], l1 = q.unit_lev[unit + 1];
  double n2[P];
#pragma unroll
  for (int j = 0; j < P; ++j) n2[j] = 0.0;
  for (int l = l0; l < l1; ++l) {
    const int a = q.lev_ptr[l], e = q.lev_ptr[l + 1];
    for (int base = a; base < e; base += kSlots) {
      const int qq = base + slot;
      const bool act = qq < e;
      const int64_t g = qq >> 6;
      const int ln = qq & 63;
      A r[P][12], t[P][12];
#pragma unroll
      for (int j = 0; j < P; ++j)
#pragma unroll
        for (int i = 0; i < 12; ++i) r[j][i] = t[j][i] = 0;
      // the lane's rows of the factor solve (rows sl and sl + 4 of each system's factor)
      DinvRow<TD> fr[P][2];
      if (act) {
        const int64_t row = q.pos_row[qq];
        const int wd = q.g_width[g];
        const int64_t s0 = q.g_slot0[g];
        // loads in three rounds: the factor rows (their address is the position's), the
        // indices of items sl and sl + 4 (item 0 the diagonal block, item i > 0 coupling
        // i - 1) with b, then their blocks and vectors
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!W.run[j]) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (sl + 4 * h < 6) fr[j][h].load(dinv + (int64_t)W.ds[j] * dstride + g * DinvTile<TD>::N, ln, sl + 4 * h);
        }
        int nbv[2], srcv[2];
        int64_t vrowv[2];
        bool on[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = sl + 4 * h;
          on[h] = i <= wd;
          nbv[h] = qq;
          srcv[h] = -1;
          vrowv[h] = row;
          if (on[h] && i > 0) {
            const int64_t fe = (s0 + i - 1) * kLanes + ln;
            nbv[h] = q.e_pos[fe];
            vrowv[h] = q.e_row[fe];
            srcv[h] = q.e_src[fe];
            on[h] = nbv[h] >= 0;
          }
        }
        A bv[P][12];
#pragma unroll
        for (int j = 0; j < P; ++j)
          if (sl == 0 && W.run[j]) load_vec(b + row * ns * 12 + W.vs[j] * 12, bv[j]);
        auto item = [&](int i, int nb, int src, int64_t vrow) {
          const TB* blk = i == 0 ? pdiag + g * slot_elems<TB>() : coup + (s0 + i - 1) * slot_elems<TB>();
          A kb[36];
          load_block(blk, ln, kb);
          const int64_t vo = vrow * ns * 12;
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!W.run[j]) continue;
            A v[12];
            load_vec(x + vo + W.vs[j] * 12, v);
            if (src >= 0 && p.ent_phase) apply_phase(p, src, W.orow[j], v);
            sub_kx(r[j], kb, v);
            if (i == 0) {  // the shift i w of the diagonal block
              const A w = (A)shift_w(p, W.orow[j], row);
#pragma unroll
              for (int c = 0; c < 6; ++c) {
                r[j][2 * c] = fmad(w, v[2 * c + 1], r[j][2 * c]);
                r[j][2 * c + 1] = fmad(-w, v[2 * c], r[j][2 * c + 1]);
              }
            } else if (nb < qq) {
              load_vec(ys + ((int64_t)(nb - q0) * P + j) * 12, v);
              if (p.ent_phase) apply_phase(p, src, W.orow[j], v);
              sub_kx(t[j], kb, v);
            }
          }
        };
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (on[h]) item(sl + 4 * h, nbv[h], srcv[h], vrowv[h]);
        // rows with more than seven couplings (general meshes)
        if (on[1]) {
          for (int i = sl + 8; i <= wd; i += 4) {
            const int64_t fe = (s0 + i - 1) * kLanes + ln;
            const int nb = q.e_pos[fe];
            if (nb < 0) break;
            item(i, nb, q.e_src[fe], q.e_row[fe]);
          }
        }
        if (sl == 0) {
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!W.run[j]) continue;
#pragma unroll
            for (int i = 0; i < 12; ++i) r[j][i] += bv[j][i];
          }
        }
      }
      // the quad's partial sums (every lane takes part in the shuffles)
#pragma unroll
      for (int j = 0; j < P; ++j)
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          r[j][i] += __shfl_xor(r[j][i], 1, kLanes);
          r[j][i] += __shfl_xor(r[j][i], 2, kLanes);
          t[j][i] += __shfl_xor(t[j][i], 1, kLanes);
          t[j][i] += __shfl_xor(t[j][i], 2, kLanes);
        }
      if (act) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!W.run[j]) continue;
          mask_frozen(p, W.orow[j], r[j]);
          if (sl == 0) n2[j] += norm2_12(r[j]);
#pragma unroll
          for (int i = 0; i < 12; ++i) t[j][i] += r[j][i];
          A* yp = ys + ((int64_t)(qq - q0) * P + j) * 12;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int rr = sl + 4 * h;
            if (rr >= 6) continue;
            A yr, yi;
            fr[j][h].apply(t[j], yr, yi);
            yp[2 * rr] = yr;
            yp[2 * rr + 1] = yi;
          }
        }
      }
    }
    __syncthreads();
  }
  // the top level has no upper neighbours: z = y there
  for (int l = l1 - 2; l >= l0; --l) {
    const int a = q.lev_ptr[l], e = q.lev_ptr[l + 1];
    for (int base = a; base < e; base += kSlots) {
      const int qq = base + slot;
      const bool act = qq < e;
      const int64_t g = qq >> 6;
      const int ln = qq & 63;
      A u[P][12];
#pragma unroll
      for (int j = 0; j < P; ++j)
#pragma unroll
        for (int i = 0; i < 12; ++i) u[j][i] = 0;
      int any = 0;
      DinvRow<TD> fr[P][2];
      if (act) {
        const int wd = q.g_width[g];
        const int64_t s0 = q.g_slot0[g];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!W.run[j]) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (sl + 4 * h < 6) fr[j][h].load(dinv + (int64_t)W.ds[j] * dstride + g * DinvTile<TD>::N, ln, sl + 4 * h);
        }
        auto coupling = [&](int k, int nb, int src) {
          any = 1;
          A kb[36];
          load_block(coup + (s0 + k) * slot_elems<TB>(), ln, kb);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (!W.run[j]) continue;
            A v[12];
            load_vec(ys + ((int64_t)(nb - q0) * P + j) * 12, v);
            if (p.ent_phase) apply_phase(p, src, W.orow[j], v);
            sub_kx(u[j], kb, v);
          }
        };
        // couplings sl and sl + 4: indices first, then the upper ones' blocks
        int nbv[2], srcv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = sl + 4 * h;
          nbv[h] = -1;
          srcv[h] = 0;
          if (k < wd) {
            const int64_t fe = (s0 + k) * kLanes + ln;
            nbv[h] = q.e_pos[fe];
            srcv[h] = q.e_src[fe];
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (nbv[h] > qq) coupling(sl + 4 * h, nbv[h], srcv[h]);  // upper only (lower and padding skipped)
        for (int k = sl + 8; k < wd; k += 4) {
          const int64_t fe = (s0 + k) * kLanes + ln;
          const int nb = q.e_pos[fe];
          if (nb > qq) coupling(k, nb, q.e_src[fe]);
        }
      }
      any |= __shfl_xor(any, 1, kLanes);
      any |= __shfl_xor(any, 2, kLanes);
#pragma unroll
      for (int j = 0; j < P; ++j)
#pragma unroll
        for (int i = 0; i < 12; ++i) {
          u[j][i] += __shfl_xor(u[j][i], 1, kLanes);
          u[j][i] += __shfl_xor(u[j][i], 2, kLanes);
        }
      if (act && any) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!W.run[j]) continue;
          A* yp = ys + ((int64_t)(qq - q0) * P + j) * 12;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int rr = sl + 4 * h;
            if (rr >= 6) continue;
            A dr, di;
            fr[j][h].apply(u[j], dr, di);
            yp[2 * rr] += dr;
            yp[2 * rr + 1] += di;
          }
        }
      }
    }
    __syncthreads();
  }
  // x += z, three of the twelve values of a row per lane
  for (int qq = q0 + slot; qq < q1; qq += kSlots) {
    const int64_t rb = (int64_t)q.pos_row[qq] * ns * 12;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      A* xp = x + rb + W.vs[j] * 12 + 3 * sl;
      const A* zp = ys + ((int64_t)(qq - q0) * P + j) * 12 + 3 * sl;
#pragma unroll
      for (int i = 0; i < 3; ++i) xp[i] += zp[i];
    }
  }
  // norms: per wave, then the workgroup's waves in order
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const double sum = wave_sum(n2[j]);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6][j] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!W.run[j]) continue;
      double tot = 0.0;
      for (int w = 0; w < NT / kLanes; ++w) tot += wsum[w][j];
      partial[(int64_t)W.vs[j] * q.pt * kPartialSlots + unit] = tot;
    }
  }
}

// ================================================================ FP64 residuals
// One wave per (tile, system), FP64 vectors in the interleaved layout.
template <typename TB>
__global__ void __launch_bounds__(256) k_resid_stored(DevPattern p, const TB* __restrict__ offd,
                                                      const TB* __restrict__ diag, const double* __restrict__ x,
                                                      const double* __restrict__ b, double* __restrict__ r, int ns,
                                                      SysBatch sb, double* __restrict__ partial, int spw) {
  int64_t tile;
  int grp;
  const int ng = (sb.n + spw - 1) / spw;
  if (!map_tile(p.n_tiles, ng, tile, grp)) return;
  const int lane = threadIdx.x & 63;
  const int k = grp * spw + (int)(threadIdx.x >> 6);
  if (k >= sb.n) return;
  const int vs = sb.vslot[k];
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  const int64_t ro = (row * ns + vs) * 12;
  double acc[12], xi[12];
  load_vec(b + ro, acc);
  load_vec(x + ro, xi);
  {
    double d[36];
    load_block(diag + tile * slot_elems<TB>(), lane, d);
    sub_diag_shift(acc, d, shift_w(p, sb.orow[k], row), xi);
  }
  const int w = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  for (int q = 0; q < w; ++q) {
    const int64_t slot = s0 + q;
    const int nb = p.ent_nbr[slot * kLanes + lane];
    double kb[36], v[12];
    load_block(offd + slot * slot_elems<TB>(), lane, kb);
    load_vec(x + ((int64_t)nb * ns + vs) * 12, v);
    if (p.ent_phase) apply_phase(p, slot * kLanes + lane, sb.orow[k], v);
    sub_kx(acc, kb, v);
  }
  mask_frozen(p, sb.orow[k], acc);
  double n2 = wave_sum(valid ? norm2_12(acc) : 0.0);
  if (lane == 0) partial[((int64_t)vs * p.n_tiles + tile) * kPartialSlots] = n2;
  if (r && valid) store_vec(r + ro, acc);
}

// The matrix-free FP64 operator: each coupling's Rusanov Jacobian is rebuilt from the
// FP64 state (the ALU-bound part) once per lane and applied to the P systems the lane
// carries; one wave per (tile, P systems).
template <int P>
__global__ void __launch_bounds__(64) k_resid_mfree(DevPattern p, DevFlow f, const double* __restrict__ x,
                                                    const double* __restrict__ b, double* __restrict__ r, int ns,
                                                    SysBatch sb, double* __restrict__ partial) {
  int64_t tile;
  int grp;
  const int ng = (sb.n + P - 1) / P;
  if (!map_tile(p.n_tiles, ng, tile, grp)) return;
  const int lane = threadIdx.x;
  int vs[P], orow[P];
  bool on[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int k = grp * P + j;
    on[j] = k < sb.n;
    vs[j] = on[j] ? sb.vslot[k] : 0;
    orow[j] = on[j] ? sb.orow[k] : 0;
  }
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  double Qi[6] = {1, 0, 0, 0, 2.5, 0};
  if (valid) load_state(f.state + row * 6, Qi);
  double acc[P][12];
#pragma unroll
  for (int j = 0; j < P; ++j) {
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[j][i] = 0.0;
    if (on[j]) load_vec(b + (row * ns + vs[j]) * 12, acc[j]);
  }
  double sumS[3] = {0, 0, 0}, lam_sum = 0.0;
  const int w = p.tile_width[tile];
  const int64_t s0 = p.tile_slot0[tile];
  for (int q = 0; q < w; ++q) {
    const int64_t fe = (s0 + q) * kLanes + lane;
    const int32_t e = p.ent_edge[fe];
    if (e == 0) continue;
    const int nb = p.ent_nbr[fe];
    double S[3], Qk[6], Ak[36];
    entry_area(f, e, S);
    load_state(f.state + (int64_t)nb * 6, Qk);
    const double lam = fmax(spectral_radius(Qi, S), spectral_radius(Qk, S));
    sumS[0] += S[0];
    sumS[1] += S[1];
    sumS[2] += S[2];
    lam_sum += lam;
    if (!f.offdiag) continue;
    if (f.ent_drop && f.ent_drop[fe]) continue;  // coupling between partitions: left out
    flux_jacobian(Qk, S, Ak);
#pragma unroll
    for (int c = 0; c < 36; ++c) Ak[c] = 0.5 * Ak[c] - ((c % 7 == 0) ? 0.5 * lam : 0.0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      if (!on[j]) continue;
      double v[12];
      load_vec(x + ((int64_t)nb * ns + vs[j]) * 12, v);
      if (p.ent_phase) apply_phase(p, fe, orow[j], v);
      sub_kx(acc[j], Ak, v);
    }
  }
  if (valid) {
    for (int32_t j = f.bf_ptr[row]; j < f.bf_ptr[row + 1]; ++j) {
      const int32_t face = f.bf_idx[j];
      double S[3] = {f.bface_area[3 * face], f.bface_area[3 * face + 1], f.bface_area[3 * face + 2]};
      double Qf[6];
      if (f.bstate) {
        load_state(f.bstate + (int64_t)face * 6, Qf);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) Qf[c] = Qi[c];
      }
      lam_sum += fmax(spectral_radius(Qi, S), spectral_radius(Qf, S));
      sumS[0] += S[0];
      sumS[1] += S[1];
      sumS[2] += S[2];
    }
  }
  double Ai[36];
  flux_jacobian(Qi, sumS, Ai);
#pragma unroll
  for (int c = 0; c < 36; ++c) Ai[c] = f.diag_scale * (0.5 * Ai[c] + ((c % 7 == 0) ? 0.5 * lam_sum : 0.0));
#pragma unroll
  for (int j = 0; j < P; ++j) {
    double xi[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) xi[i] = 0.0;
    if (on[j]) {
      load_vec(x + (row * ns + vs[j]) * 12, xi);
      sub_diag_shift(acc[j], Ai, shift_w(p, orow[j], row), xi);
      mask_frozen(p, orow[j], acc[j]);
    }
    const double n2 = wave_sum(valid && on[j] ? norm2_12(acc[j]) : 0.0);
    if (!on[j]) continue;
    if (lane == 0) partial[((int64_t)vs[j] * p.n_tiles + tile) * kPartialSlots] = n2;
    if (r && valid) store_vec(r + (row * ns + vs[j]) * 12, acc[j]);
  }
}

// ================================================================ nonlinear residual
// Rusanov residual of the state q (internal [NP][6]) with the dissipation coefficients
// and far field taken from q itself:
//   R_i = sum_k [1/2 (F(q_i; S_ik) + F(q_k; S_ik)) - 1/2 lam_ik (q_k - q_i)]
//       + sum_f [1/2 (F(q_i; S_f) + F(q_f; S_f)) - 1/2 lam_f (q_f - q_i)],
// lam = larger end spectral radius, F(q; S) = A(q; S) q (the flux is homogeneous of
// degree one).  R goes to user order; part[tile] = sum |R|^2 over the tile.
__device__ inline void add_rusanov(const double (&Qa)[6], const double (&Qb)[6], const double (&S)[3],
                                   double (&acc)[6]) {
  double Aa[36], Ab[36];
  flux_jacobian(Qa, S, Aa);
  flux_jacobian(Qb, S, Ab);
  const double lam = fmax(spectral_radius(Qa, S), spectral_radius(Qb, S));
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double fa = 0.0, fb = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      fa += Aa[6 * r + c] * Qa[c];
      fb += Ab[6 * r + c] * Qb[c];
    }
    acc[r] += 0.5 * (fa + fb) - 0.5 * lam * (Qb[r] - Qa[r]);
  }
}

__global__ void __launch_bounds__(64) k_rusanov_residual(DevPattern p, DevFlow f, const int32_t* __restrict__ iperm,
                                                         double* __restrict__ R, double* __restrict__ part) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t row = tile * kLanes + lane;
  const bool valid = lane < p.tile_nrows[tile];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    double Qi[6];
    load_state(f.state + row * 6, Qi);
    const int w = p.tile_width[tile];
    const int64_t s0 = p.tile_slot0[tile];
    for (int q = 0; q < w; ++q) {
      const int64_t fe = (s0 + q) * kLanes + lane;
      const int32_t e = p.ent_edge[fe];
      if (e == 0) continue;
      double S[3], Qk[6];
      entry_area(f, e, S);
      load_state(f.state + (int64_t)p.ent_nbr[fe] * 6, Qk);
      add_rusanov(Qi, Qk, S, acc);
    }
    for (int32_t j = f.bf_ptr[row]; j < f.bf_ptr[row + 1]; ++j) {
      const int32_t face = f.bf_idx[j];
      const double S[3] = {f.bface_area[3 * face], f.bface_area[3 * face + 1], f.bface_area[3 * face + 2]};
      double Qf[6];
      if (f.bstate) {
        load_state(f.bstate + (int64_t)face * 6, Qf);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) Qf[c] = Qi[c];
      }
      add_rusanov(Qi, Qf, S, acc);
    }
    const int64_t u = iperm[row];
#pragma unroll
    for (int c = 0; c < 6; ++c) R[u * 6 + c] = acc[c];
  }
  double n2 = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) n2 += acc[c] * acc[c];
  n2 = wave_sum(n2);
  if (lane == 0) part[tile] = n2;
}

// RK stage helpers on user-order vectors: b = scale * R (real R -> complex b),
// q = q0 + Re x (real state), q = q0 + x (complex), y = scale * y (complex)
__global__ void k_rk_rhs_real(int64_t n, const double* __restrict__ R, double scale, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  b[2 * i] = scale * R[i];
  b[2 * i + 1] = 0.0;
}
__global__ void k_rk_update_real(int64_t n, const double* __restrict__ q0, const double* __restrict__ x,
                                 double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  q[i] = q0[i] + x[2 * i];
}
__global__ void k_rk_update_complex(int64_t n, const double* __restrict__ q0, const double* __restrict__ x,
                                    double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  q[i] = q0[i] + x[i];
}
__global__ void k_scale(int64_t n, double* __restrict__ y, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] *= scale;
}

// ================================================================ vectors
// user [N][width] (one system)  <->  internal [NP][ns][width], slot vs
__global__ void k_to_internal(int64_t NP, const int32_t* __restrict__ iperm, const double* __restrict__ user,
                              double* __restrict__ internal, int width, int ns, int vs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * width) return;
  const int64_t row = t / width;
  const int c = (int)(t % width);
  const int32_t u = iperm[row];
  internal[(row * ns + vs) * width + c] = u >= 0 ? user[(int64_t)u * width + c] : 0.0;
}
__global__ void k_to_user(int64_t NP, const int32_t* __restrict__ iperm, const double* __restrict__ internal,
                          double* __restrict__ user, int width, int ns, int vs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * width) return;
  const int64_t row = t / width;
  const int c = (int)(t % width);
  const int32_t u = iperm[row];
  if (u >= 0) user[(int64_t)u * width + c] = internal[(row * ns + vs) * width + c];
}
// Several systems' complex vectors at once: item (internal row, system j, component),
// component fastest, so the interleaved rows [row][ns][12] are written (read) as one
// stream while each user vector is gathered (scattered) by rows.
__global__ void k_to_internal_n(int64_t NP, const int32_t* __restrict__ iperm, VecPtrs users,
                                double* __restrict__ internal, int ns, int vs0, int n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * n * 12) return;
  const int64_t row = t / (n * 12);
  const int rem = (int)(t % (n * 12));
  const int j = rem / 12, c = rem % 12;
  const int32_t u = iperm[row];
  internal[(row * ns + vs0 + j) * 12 + c] = u >= 0 ? users.p[j][(int64_t)u * 12 + c] : 0.0;
}
__global__ void k_to_user_n(int64_t NP, const int32_t* __restrict__ iperm, const double* __restrict__ internal,
                            VecPtrsOut users, int ns, int vs0, int n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NP * n * 12) return;
  const int64_t row = t / (n * 12);
  const int rem = (int)(t % (n * 12));
  const int j = rem / 12, c = rem % 12;
  const int32_t u = iperm[row];
  if (u >= 0) users.p[j][(int64_t)u * 12 + c] = internal[(row * ns + vs0 + j) * 12 + c];
}
// defect-correction conversions, item (row, system kk of sb, component) with the component
// fastest, then the system: consecutive lanes touch consecutive entries of the
// interleaved rows, so each vector is streamed once whatever the number of systems
__global__ void k_to_f32(int64_t NP, int ns, const double* __restrict__ r64, float* __restrict__ rhs32,
                         float* __restrict__ d32, SysBatch sb, const SysState* __restrict__ outer) {
  const int nk = sb.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP * nk * 12) return;
  const int64_t rk = i / 12;
  const int64_t row = rk / nk;
  const int kk = (int)(rk - row * nk);
  const int vs = sb.vslot[kk];
  if (!outer[vs].active) return;
  const int64_t o = (row * ns + vs) * 12 + (i - rk * 12);
  rhs32[o] = (float)r64[o];
  d32[o] = 0.0f;
}
__global__ void k_add_f32(int64_t NP, int ns, double* __restrict__ x64, const float* __restrict__ d32, SysBatch sb,
                          const SysState* __restrict__ outer) {
  const int nk = sb.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP * nk * 12) return;
  const int64_t rk = i / 12;
  const int64_t row = rk / nk;
  const int kk = (int)(rk - row * nk);
  const int vs = sb.vslot[kk];
  if (!outer[vs].active) return;
  const int64_t o = (row * ns + vs) * 12 + (i - rk * 12);
  x64[o] += (double)d32[o];
}
template <typename TB>
__global__ void k_drop_blocks(int64_t n_ent, const int8_t* __restrict__ ent_drop, TB* __restrict__ offd) {
  const int64_t fe = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (fe >= n_ent || !ent_drop[fe]) return;
  TB* dst = offd + (fe / kLanes) * slot_elems<TB>();
  const int lane = (int)(fe % kLanes);
#pragma unroll
  for (int c = 0; c < 36; ++c) store_entry<TB>(dst, c, lane, 0.0);
}
__global__ void k_zero_sixth(int64_t NP, int ns, int vs, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP) return;
  v[(i * ns + vs) * 12 + 10] = 0.0;
  v[(i * ns + vs) * 12 + 11] = 0.0;
}
__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline int ng_of(const SysBatch& sb, int spw) { return (sb.n + spw - 1) / spw; }

}  // namespace

// ================================================================ launchers
#define FNLH_DISPATCH_STORE(storage, BODY)    \
  do {                                        \
    if ((storage) == kF64) {                  \
      using TB = double;                      \
      BODY;                                   \
    } else if ((storage) == kF32) {           \
      using TB = float;                       \
      BODY;                                   \
    } else {                                  \
      using TB = bf16s;                       \
      BODY;                                   \
    }                                         \
  } while (0)

void launch_assemble(int storage, const DevPattern& p, const DevFlow& f, void* offd, void* diag, hipStream_t s) {
  FNLH_DISPATCH_STORE(storage, {
    hipLaunchKernelGGL((k_assemble<TB>), dim3((unsigned)p.n_tiles), dim3(64), 0, s, p, f, (TB*)offd, (TB*)diag);
  });
}

void launch_check_dominance(int storage, const DevPattern& p, const void* diag, int* flag, hipStream_t s) {
  FNLH_DISPATCH_STORE(storage, {
    hipLaunchKernelGGL((k_check_dominance<TB>), dim3((unsigned)p.n_tiles), dim3(64), 0, s, p, (const TB*)diag, flag);
  });
}

void launch_set_blocks(int storage, const DevPattern& p, int64_t N, int64_t E, const int32_t* perm,
                       const int64_t* edge_ent, const double* diag_user, const double* offd_user, void* offd,
                       void* diag, hipStream_t s) {
  FNLH_DISPATCH_STORE(storage, {
    if (E > 0)
      hipLaunchKernelGGL((k_set_offd<TB>), dim3((unsigned)((2 * E * 36 + 255) / 256)), dim3(256), 0, s, E, edge_ent,
                         offd_user, (TB*)offd);
    hipLaunchKernelGGL((k_set_diag<TB>), dim3((unsigned)((N * 36 + 255) / 256)), dim3(256), 0, s, N, perm, diag_user,
                       (TB*)diag);
  });
}

void launch_get_blocks(int storage, const DevPattern& p, int64_t N, int64_t E, const int32_t* perm,
                       const int64_t* edge_ent, const void* offd, const void* diag, double* diag_user,
                       double* offd_user, hipStream_t s) {
  FNLH_DISPATCH_STORE(storage, {
    if (E > 0)
      hipLaunchKernelGGL((k_get_offd<TB>), dim3((unsigned)((2 * E * 36 + 255) / 256)), dim3(256), 0, s, E, edge_ent,
                         (const TB*)offd, offd_user);
    hipLaunchKernelGGL((k_get_diag<TB>), dim3((unsigned)((N * 36 + 255) / 256)), dim3(256), 0, s, N, perm,
                       (const TB*)diag, diag_user);
  });
}

void launch_factor(int storage, bool dilu, const DevPattern& p, const void* offd, const void* diag, void* dinv,
                   int64_t dinv_stride, const SysBatch& sb, int64_t t0, int64_t nt, int64_t cstart, int* err,
                   hipStream_t s) {
  if (nt <= 0 || sb.n <= 0) return;
  const dim3 grid = tile_grid(nt, sb.n);
  FNLH_DISPATCH_STORE(storage, {
    using TD = typename DF_of<TB>::T;
    if (dilu)
      hipLaunchKernelGGL((k_factor<TB, TD, true>), grid, dim3(64), 0, s, p, (const TB*)offd, (const TB*)diag,
                         (TD*)dinv, dinv_stride, sb, t0, nt, cstart, err);
    else
      hipLaunchKernelGGL((k_factor<TB, TD, false>), grid, dim3(64), 0, s, p, (const TB*)offd, (const TB*)diag,
                         (TD*)dinv, dinv_stride, sb, t0, nt, cstart, err);
  });
}

// systems per lane for the one-row-per-lane kernels (general colouring, Jacobi): the
// requested value, or automatic; never fewer than ceil(n / 4) so that at most four
// waves per tile cover all n <= 16 systems.
inline int lanes_p(const SweepCfg& c, int n) {
  int P = c.spw > 0 ? c.spw : (c.storage == kF64 ? 2 : 4);
  if (P >= 4 && n <= 3) P = n <= 2 ? n : 4;
  const int need = (n + 3) / 4;
  if (P < need) P = need;
  return P <= 1 ? 1 : (P <= 2 ? 2 : 4);
}
inline dim3 block_for(int n, int P) {
  int nw = (n + P - 1) / P;
  if (nw > 4) nw = 4;
  return dim3(64 * nw);
}

#define FNLH_DISPATCH_P(P, BODY)                         \
  do {                                                   \
    if ((P) == 1) {                                      \
      constexpr int PP = 1;                              \
      BODY;                                              \
    } else if ((P) == 2) {                               \
      constexpr int PP = 2;                              \
      BODY;                                              \
    } else if ((P) == 3) {                               \
      constexpr int PP = 3;                              \
      BODY;                                              \
    } else {                                             \
      constexpr int PP = 4;                              \
      BODY;                                              \
    }                                                    \
  } while (0)

// lanes per row (SW) and systems per lane (P) of the two-colour pass
void rb_shape(const SweepCfg& c, int n, int& SW, int& P) {
  SW = c.lanes_per_row;
  if (SW <= 0) SW = n >= 4 ? 4 : (n >= 2 ? 2 : 1);
  if (SW != 1 && SW != 2 && SW != 4) SW = 4;
  // SW * P must cover the n <= 16 systems with P <= 4
  const int sw_need = n <= 4 ? 1 : (n <= 8 ? 2 : 4);
  if (SW < sw_need) SW = sw_need;
  P = (n + SW - 1) / SW;
  if (c.spw > 0 && c.spw > P) P = c.spw;
  if (P > 4) P = 4;
}
int rb_slots(const SweepCfg& c, int n) {
  int SW, P;
  rb_shape(c, n, SW, P);
  return SW;
}

void launch_rb_pass(const SweepCfg& c, bool update, const DevPattern& p, const void* offd, const void* diag,
                    const void* dinv, int64_t dinv_stride, void* x, const void* b, int ns, const SysBatch& sb,
                    const SysState* st, double* partial, int64_t t0, int64_t nt, hipStream_t s,
                    const FusedReduce* fused) {
  if (nt <= 0 || sb.n <= 0) return;
  int SW, P;
  rb_shape(c, sb.n, SW, P);
  const int wg = c.wave_groups ? 1 : 0;
  FusedReduce fr;
  if (!update && fused) fr = *fused;
  dim3 grid = tile_grid(nt, wg ? SW : 1);
  grid.x += (unsigned)fr.n;
  dim3 block(wg ? 64 : 64 * SW);
  // LDS of the staged update pass (other instantiations do not touch it)
  const bool ph = p.ent_phase != nullptr;
  const unsigned lds_bytes = (SW == 4)
                                 ? (unsigned)(block.x / 64) * rb_lds_chunks(c.storage, update) * 16u
                                 : 0u;
#define FNLH_RB_LAUNCH(SWV)                                                                                     \
  FNLH_DISPATCH_P(P, {                                                                                          \
    if (update && ph)                                                                                           \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, true, true, true>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                                         \
    else if (update)                                                                                            \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, true, true, false>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                                \
    else if (c.pivot && ph)                                                                                     \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, false, true, true>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                                        \
    else if (c.pivot)                                                                                           \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, false, true, false>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                               \
    else if (ph)                                                                                                \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, false, false, true>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                                       \
    else                                                                                                        \
      hipLaunchKernelGGL((k_rb_pass<TB, SWV, PP, false, false, false>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                         (SysState*)st, partial, t0, nt, wg, fr);                                              \
  })
FNLH_DISPATCH_STORE(c.storage, {
    using A = typename Fmt<TB>::A;
    if (SW == 1)
      FNLH_RB_LAUNCH(1);
    else if (SW == 2)
      FNLH_RB_LAUNCH(2);
    else
      FNLH_RB_LAUNCH(4);
  });
#undef FNLH_RB_LAUNCH
}

void launch_rb_batched(int storage, int SW, int P, bool update, const InstDesc* inst, const WorkItem* work,
                       int64_t n_work, hipStream_t s, bool wave_groups, const WorkItem* red, int n_red, int red_mode,
                       double rtol, double div_factor) {
  if (update) n_red = 0;
  if (n_work <= 0 && n_red <= 0) return;
  const int wg = wave_groups ? 1 : 0;
  dim3 grid(n_work > 0 ? tile_grid(n_work, wg ? SW : 1).x : 0u);
  grid.x += (unsigned)n_red;
  dim3 block(wg ? 64 : 64 * SW);
  const unsigned lds_bytes =
      (SW == 4) ? (unsigned)(block.x / 64) * rb_lds_chunks(storage, update) * 16u : 0u;
  const double rtol2 = rtol * rtol, div2 = div_factor * div_factor;
#define FNLH_RBB_LAUNCH(SWV)                                                                                   \
  FNLH_DISPATCH_P(P, {                                                                                         \
    if (update)                                                                                                \
      hipLaunchKernelGGL((k_rb_batched<TB, SWV, PP, true, true>), grid, block, lds_bytes, s, inst, work, n_work,   \
                         wg, red, n_red, red_mode, rtol2, div2);                                              \
    else                                                                                                       \
      hipLaunchKernelGGL((k_rb_batched<TB, SWV, PP, false, true>), grid, block, lds_bytes, s, inst, work, n_work,  \
                         wg, red, n_red, red_mode, rtol2, div2);                                              \
  })
  FNLH_DISPATCH_STORE(storage, {
    if (SW == 1)
      FNLH_RBB_LAUNCH(1);
    else if (SW == 2)
      FNLH_RBB_LAUNCH(2);
    else
      FNLH_RBB_LAUNCH(4);
  });
#undef FNLH_RBB_LAUNCH
}

void launch_reduce_batched(const InstDesc* inst, const WorkItem* items, int n_items, int mode, double rtol,
                           double div_factor, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(k_reduce_batched, dim3((unsigned)n_items), dim3(256), 0, s, inst, items, mode, rtol * rtol,
                     div_factor * div_factor);
}

void launch_fwd(const SweepCfg& c, int mode, const DevPattern& p, const void* offd, const void* diag,
                const void* dinv, int64_t dinv_stride, void* x, const void* b, void* y, int ns, const SysBatch& sb,
                const SysState* st, double* partial, int64_t t0, int64_t nt, int64_t cstart, hipStream_t s) {
  if (nt <= 0 || sb.n <= 0) return;
  int SW, P;
  rb_shape(c, sb.n, SW, P);
  const int wg = c.wave_groups ? 1 : 0;
  dim3 grid = tile_grid(nt, wg ? SW : 1);
  dim3 block(wg ? 64 : 64 * SW);
  const unsigned lds_bytes = (SW == 4) ? (unsigned)(block.x / 64) * lds_chunks_per_wave(c.storage) * 16u : 0u;
#define FNLH_FWD_ONE(SWV, MD)                                                                                     \
  hipLaunchKernelGGL((k_fwd<TB, SWV, PP, MD>), grid, block, lds_bytes, s, p, (const TB*)offd, (const TB*)diag,        \
                     (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, (A*)y, ns, sb, st, partial, t0,  \
                     nt, cstart, wg)
#define FNLH_FWD_LAUNCH(SWV)                                                                                      \
  FNLH_DISPATCH_P(P, {                                                                                            \
    if (mode == kFwdLast)                                                                                         \
      FNLH_FWD_ONE(SWV, kFwdLast);                                                                                \
    else if (mode == kFwdHybrid)                                                                                  \
      FNLH_FWD_ONE(SWV, kFwdHybrid);                                                                              \
    else if (mode == kFwdNorm)                                                                                    \
      FNLH_FWD_ONE(SWV, kFwdNorm);                                                                                \
    else                                                                                                          \
      FNLH_FWD_ONE(SWV, kFwdGeneral);                                                                             \
  })
  FNLH_DISPATCH_STORE(c.storage, {
    using A = typename Fmt<TB>::A;
    if (SW == 1)
      FNLH_FWD_LAUNCH(1);
    else if (SW == 2)
      FNLH_FWD_LAUNCH(2);
    else
      FNLH_FWD_LAUNCH(4);
  });
#undef FNLH_FWD_LAUNCH
#undef FNLH_FWD_ONE
}

void launch_bwd(const SweepCfg& c, int mode, const DevPattern& p, const void* offd, const void* dinv,
                int64_t dinv_stride, void* x, void* y, int ns, const SysBatch& sb, const SysState* st, int64_t t0,
                int64_t nt, int64_t cend, hipStream_t s) {
  if (nt <= 0 || sb.n <= 0) return;
  int SW, P;
  rb_shape(c, sb.n, SW, P);
  const int wg = c.wave_groups ? 1 : 0;
  dim3 grid = tile_grid(nt, wg ? SW : 1);
  dim3 block(wg ? 64 : 64 * SW);
  const unsigned lds_bytes = (SW == 4) ? (unsigned)(block.x / 64) * lds_chunks_per_wave(c.storage) * 16u : 0u;
#define FNLH_BWD_ONE(SWV, MD)                                                                                 \
  hipLaunchKernelGGL((k_bwd<TB, SWV, PP, MD>), grid, block, lds_bytes, s, p, (const TB*)offd,                   \
                     (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (A*)y, ns, sb, st, t0, nt, cend, wg)
#define FNLH_BWD_LAUNCH(SWV)                                                                                  \
  FNLH_DISPATCH_P(P, {                                                                                        \
    if (mode == kBwdHybrid)                                                                                   \
      FNLH_BWD_ONE(SWV, kBwdHybrid);                                                                          \
    else                                                                                                      \
      FNLH_BWD_ONE(SWV, kBwdGeneral);                                                                         \
  })
  FNLH_DISPATCH_STORE(c.storage, {
    using A = typename Fmt<TB>::A;
    if (SW == 1)
      FNLH_BWD_LAUNCH(1);
    else if (SW == 2)
      FNLH_BWD_LAUNCH(2);
    else
      FNLH_BWD_LAUNCH(4);
  });
#undef FNLH_BWD_LAUNCH
#undef FNLH_BWD_ONE
}
void launch_correct(int storage, const DevPattern& p, const CorrDev& q, const void* offd, const void* dinv,
                    int64_t dinv_stride, void* x, const void* y, int ns, const SysBatch& sb, const SysState* st,
                    hipStream_t s) {
  if (q.n_groups <= 0 || sb.n <= 0) return;
  const int P = sb.n < 4 ? sb.n : 4;
  dim3 grid((unsigned)q.n_groups, (unsigned)((sb.n + P - 1) / P));
  FNLH_DISPATCH_STORE(storage, {
    using A = typename Fmt<TB>::A;
    FNLH_DISPATCH_P(P, {
      hipLaunchKernelGGL((k_correct<TB, PP>), grid, dim3(64), 0, s, p, q, (const TB*)offd,
                         (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)y, ns, sb, st);
    });
  });
}

void launch_jacobi(const SweepCfg& c, const DevPattern& p, const void* offd, const void* diag, const void* dinv,
                   int64_t dinv_stride, const void* x, const void* b, void* y, int ns, const SysBatch& sb,
                   const SysState* st, double* partial, hipStream_t s) {
  if (sb.n <= 0) return;
  const int P = lanes_p(c, sb.n);
  dim3 grid = tile_grid(p.n_tiles, 1);
  dim3 block = block_for(sb.n, P);
  FNLH_DISPATCH_STORE(c.storage, {
    using A = typename Fmt<TB>::A;
    FNLH_DISPATCH_P(P, {
      hipLaunchKernelGGL((k_jacobi<TB, PP>), grid, block, 0, s, p, (const TB*)offd, (const TB*)diag,
                         (const typename DF_of<TB>::T*)dinv, dinv_stride, (const A*)x, (const A*)b, (A*)y, ns, sb, st, partial);
    });
  });
}

void launch_axpy_y(int storage, const DevPattern& p, void* x, const void* y, int ns, const SysBatch& sb,
                   const SysState* st, hipStream_t s) {
  if (sb.n <= 0) return;
  dim3 grid((unsigned)((p.NP * 12 + 255) / 256), (unsigned)sb.n);
  if (storage == kF64)
    hipLaunchKernelGGL((k_axpy_y<double>), grid, dim3(256), 0, s, p.NP, ns, (double*)x, (const double*)y, sb, st);
  else
    hipLaunchKernelGGL((k_axpy_y<float>), grid, dim3(256), 0, s, p.NP, ns, (float*)x, (const float*)y, sb, st);
}

void launch_reduce(const SysBatch& sb, const double* partial, int64_t n_tiles, int64_t t0, int64_t nt, int slots,
                   SysState* st, int mode, double rtol, double div_factor, int max_sweeps, hipStream_t s) {
  if (sb.n <= 0) return;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)sb.n), dim3(256), 0, s, sb, partial, n_tiles, t0, nt, slots, st, mode,
                     rtol * rtol, div_factor * div_factor, max_sweeps);
}

void launch_resid_stored(int storage, const DevPattern& p, const void* offd, const void* diag, const double* x,
                         const double* b, double* r, int ns, const SysBatch& sb, double* partial, hipStream_t s) {
  if (sb.n <= 0) return;
  const int spw = 4 < sb.n ? 4 : sb.n;
  dim3 grid = tile_grid(p.n_tiles, ng_of(sb, spw));
  FNLH_DISPATCH_STORE(storage, {
    hipLaunchKernelGGL((k_resid_stored<TB>), grid, dim3(64 * spw), 0, s, p, (const TB*)offd, (const TB*)diag, x, b,
                       r, ns, sb, partial, spw);
  });
}

void launch_resid_mfree(const DevPattern& p, const DevFlow& f, const double* x, const double* b, double* r, int ns,
                        const SysBatch& sb, double* partial, hipStream_t s) {
  if (sb.n <= 0) return;
  // at most three systems a lane (four would leave one wave per SIMD), spread evenly
  const int groups = (sb.n + 2) / 3;
  const int P = (sb.n + groups - 1) / groups;
  dim3 grid = tile_grid(p.n_tiles, ng_of(sb, P));
  FNLH_DISPATCH_P(P, {
    hipLaunchKernelGGL((k_resid_mfree<PP>), grid, dim3(64), 0, s, p, f, x, b, r, ns, sb, partial);
  });
}

void launch_to_internal(const DevPattern& p, const int32_t* iperm, const double* user, double* internal, int width,
                        int ns, int vs, hipStream_t s) {
  const int64_t n = p.NP * width;
  hipLaunchKernelGGL(k_to_internal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, iperm, user, internal,
                     width, ns, vs);
}
void launch_to_user(const DevPattern& p, const int32_t* iperm, const double* internal, double* user, int width,
                    int ns, int vs, hipStream_t s) {
  const int64_t n = p.NP * width;
  hipLaunchKernelGGL(k_to_user, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.NP, iperm, internal, user,
                     width, ns, vs);
}
void launch_to_internal_n(const DevPattern& p, const int32_t* iperm, const double* const* users, int n,
                          double* internal, int ns, int vs0, hipStream_t s) {
  for (int j0 = 0; j0 < n; j0 += kMaxBatch) {
    const int m = n - j0 < kMaxBatch ? n - j0 : kMaxBatch;
    VecPtrs v;
    for (int j = 0; j < m; ++j) v.p[j] = users[j0 + j];
    const int64_t items = p.NP * m * 12;
    hipLaunchKernelGGL(k_to_internal_n, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, p.NP, iperm, v,
                       internal, ns, vs0 + j0, m);
  }
}
void launch_to_user_n(const DevPattern& p, const int32_t* iperm, const double* internal, double* const* users, int n,
                      int ns, int vs0, hipStream_t s) {
  for (int j0 = 0; j0 < n; j0 += kMaxBatch) {
    const int m = n - j0 < kMaxBatch ? n - j0 : kMaxBatch;
    VecPtrsOut v;
    for (int j = 0; j < m; ++j) v.p[j] = users[j0 + j];
    const int64_t items = p.NP * m * 12;
    hipLaunchKernelGGL(k_to_user_n, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, p.NP, iperm, internal,
                       v, ns, vs0 + j0, m);
  }
}
void launch_to_f32(const DevPattern& p, const double* r64, float* rhs32, float* d32, int ns, const SysBatch& sb,
                   const SysState* outer, hipStream_t s) {
  if (sb.n <= 0) return;
  dim3 grid((unsigned)((p.NP * sb.n * 12 + 255) / 256));
  hipLaunchKernelGGL(k_to_f32, grid, dim3(256), 0, s, p.NP, ns, r64, rhs32, d32, sb, outer);
}
void launch_add_f32(const DevPattern& p, double* x64, const float* d32, int ns, const SysBatch& sb,
                    const SysState* outer, hipStream_t s) {
  if (sb.n <= 0) return;
  dim3 grid((unsigned)((p.NP * sb.n * 12 + 255) / 256));
  hipLaunchKernelGGL(k_add_f32, grid, dim3(256), 0, s, p.NP, ns, x64, d32, sb, outer);
}
void launch_inner_init(const SysBatch& sb, const SysState* outer, SysState* inner, int max_sweeps, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_init, dim3(1), dim3(64), 0, s, sb, outer, inner, max_sweeps);
}
void launch_outer_update(const SysBatch& sb, const SysState* inner, SysState* outer, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_update, dim3(1), dim3(64), 0, s, sb, inner, outer);
}
void launch_rusanov_residual(const DevPattern& p, const DevFlow& f, const int32_t* iperm, double* R_user,
                             double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_rusanov_residual, dim3((unsigned)p.n_tiles), dim3(64), 0, s, p, f, iperm, R_user, part);
}
void launch_rk_rhs_real(int64_t n, const double* R, double scale, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_rk_rhs_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, R, scale, b);
}
void launch_rk_update(bool complex_state, int64_t n, const double* q0, const double* x, double* q, hipStream_t s) {
  if (complex_state)
    hipLaunchKernelGGL(k_rk_update_complex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, q0, x, q);
  else
    hipLaunchKernelGGL(k_rk_update_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, q0, x, q);
}
void launch_scale(int64_t n, double* y, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, y, scale);
}
void launch_drop_blocks(int storage, const DevPattern& p, int64_t n_slots, const int8_t* ent_drop, void* offd,
                        hipStream_t s) {
  const int64_t n = n_slots * kLanes;
  if (n <= 0 || !ent_drop) return;
  (void)p;
  FNLH_DISPATCH_STORE(storage, {
    hipLaunchKernelGGL((k_drop_blocks<TB>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ent_drop,
                       (TB*)offd);
  });
}
void launch_zero_sixth(int64_t rows, double* v, int ns, int vs, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_zero_sixth, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows, ns, vs, v);
}
void launch_set_history(const SysBatch& sb, SysState* st, double* hist, int len, hipStream_t s) {
  if (sb.n <= 0) return;
  hipLaunchKernelGGL(k_set_history, dim3(1), dim3(64), 0, s, sb, st, hist, len);
}
void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, n);
}

void launch_pilu_pack(int storage, const PiluDev& q, const void* offd, const void* diag, void* coup, void* pdiag,
                      hipStream_t s) {
  FNLH_DISPATCH_STORE(storage, {
    const int64_t n = (q.n_slots + q.n_groups) * kLanes * Fmt<TB>::NV;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_pilu_pack<TB>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, (const TB*)offd,
                       (const TB*)diag, (TB*)coup, (TB*)pdiag);
  });
}
void launch_pilu_factor(int storage, const DevPattern& p, const PiluDev& q, const void* coup, const void* pdiag,
                        void* dinv, int64_t dinv_stride, const SysBatch& sb, int* err, hipStream_t s) {
  if (q.n_units <= 0 || sb.n <= 0) return;
  dim3 grid((unsigned)q.n_units, (unsigned)sb.n);
  FNLH_DISPATCH_STORE(storage, {
    using TD = typename DF_of<TB>::T;
    hipLaunchKernelGGL((k_pilu_factor<TB, TD>), grid, dim3(64), 0, s, p, q, (const TB*)coup, (const TB*)pdiag,
                       (TD*)dinv, dinv_stride, sb, err);
  });
}
int pilu_lds_row_bytes(int storage) { return 12 * (storage == kF64 ? 8 : 4); }
#define FNLH_PILU_ATTR(PV, NTV)                                                                                      \
  ok = ok && hipFuncSetAttribute((const void*)k_pilu_sweep<TB, PV, NTV>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                 lds) == hipSuccess
bool pilu_allow_lds(int storage, int lds) {
  bool ok = true;
  FNLH_DISPATCH_STORE(storage, {
    FNLH_PILU_ATTR(1, 64);
    FNLH_PILU_ATTR(2, 64);
    FNLH_PILU_ATTR(1, 128);
    FNLH_PILU_ATTR(2, 128);
    FNLH_PILU_ATTR(1, 256);
    FNLH_PILU_ATTR(2, 256);
  });
  (void)hipGetLastError();
  return ok;
}
#undef FNLH_PILU_ATTR
int pilu_threads(int avg_width) { return avg_width <= 16 ? 64 : avg_width <= 32 ? 128 : 256; }
int pilu_systems_per_group(int storage, int nb, int max_rows, int lds_max) {
  // at most two systems a workgroup: the sweep keeps each lane's factor rows, item
  // indices and b in registers, and more workgroups hide the level chain's latency
  int P = nb < 2 ? nb : 2;
  while (P > 0 && (int64_t)max_rows * P * pilu_lds_row_bytes(storage) > lds_max) --P;
  return P;
}
#define FNLH_PILU_LAUNCH(NTV)                                                                                  \
  hipLaunchKernelGGL((k_pilu_sweep<TB, PP, NTV>), grid, dim3(NTV), lds, s, p, q, (const TB*)coup,              \
                     (const TB*)pdiag, (const typename DF_of<TB>::T*)dinv, dinv_stride, (A*)x, (const A*)b, ns, sb, \
                     st, partial)
void launch_pilu_sweep(int storage, const DevPattern& p, const PiluDev& q, const void* coup, const void* pdiag,
                       const void* dinv, int64_t dinv_stride, void* x, const void* b, int ns, const SysBatch& sb,
                       const SysState* st, double* partial, int lds_max, hipStream_t s) {
  if (q.n_units <= 0 || sb.n <= 0) return;
  const int P = pilu_systems_per_group(storage, sb.n, q.max_rows, lds_max);
  if (P <= 0) return;  // the caller checks that a unit fits
  dim3 grid((unsigned)q.n_units, (unsigned)((sb.n + P - 1) / P));
  const unsigned lds = (unsigned)q.max_rows * P * pilu_lds_row_bytes(storage);
  const int nt = q.threads;
  FNLH_DISPATCH_STORE(storage, {
    using A = typename Fmt<TB>::A;
    if (P == 1) {
      constexpr int PP = 1;
      if (nt == 64)
        FNLH_PILU_LAUNCH(64);
      else if (nt == 128)
        FNLH_PILU_LAUNCH(128);
      else
        FNLH_PILU_LAUNCH(256);
    } else {
      constexpr int PP = 2;
      if (nt == 64)
        FNLH_PILU_LAUNCH(64);
      else if (nt == 128)
        FNLH_PILU_LAUNCH(128);
      else
        FNLH_PILU_LAUNCH(256);
    }
  });
}
#undef FNLH_PILU_LAUNCH

}  // namespace fnlh
