// C ABI of libfnlh (include/fnlh.h): context lifecycle, assembly, factorisation and
// the relaxation driver.  Stop decisions are taken on the device (SysState); the host
// reads the few per-system states back every `check_every` sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

using namespace fnlh;

namespace {

thread_local std::string g_create_error;

}  // namespace

namespace fnlh {

int set_err(fnlh_ctx c, int code, const std::string& m) {
  if (c) c->err = m; else g_create_error = m;
  return code;
}

int hip_fail(fnlh_ctx c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_err(c, e == hipErrorOutOfMemory ? FNLH_E_OOM : FNLH_E_HIP, m);
}

int dalloc(fnlh_ctx c, DevBuf& b, size_t bytes, const char* what) {
  if (c) c->buf_gen++;
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return FNLH_OK;
  HIPC(c, hipMalloc(&b.p, bytes), what);
  b.bytes = bytes;
  return FNLH_OK;
}

void dfree(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

int check_launch(fnlh_ctx c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, what);
  return FNLH_OK;
}

void outer_residual_of(fnlh_ctx c, int ns, const SysBatch& sb, const double* x, const double* b, double* r,
                       hipStream_t s, double* part) {
  DevPattern p = c->pat();
  if (!part) part = (double*)c->partial.p;
  if (c->storage == FNLH_F64) {
    launch_resid_stored(kF64, p, c->offd.p, c->diag.p, x, b, r, ns, sb, part, s);
  } else if (c->outer == FNLH_OUTER_STORED) {
    launch_resid_stored(c->storage, p, c->offd.p, c->diag.p, x, b, r, ns, sb, part, s);
  } else if (c->assembled) {
    launch_resid_mfree(p, c->flow(), x, b, r, ns, sb, part, s);
  } else {
    launch_resid_stored(kF64, p, c->offd64.p, c->diag64.p, x, b, r, ns, sb, part, s);
  }
}

}  // namespace fnlh

namespace {

template <typename T> int dupload(fnlh_ctx c, DevBuf& b, const std::vector<T>& v, const char* what) {
  int rc = dalloc(c, b, v.size() * sizeof(T), what);
  if (rc) return rc;
  if (!v.empty()) HIPC(c, hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
  return FNLH_OK;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

int ensure_vectors(fnlh_ctx c, int n) {
  if (n <= c->vec_cap) return FNLH_OK;
  const size_t v64 = (size_t)n * c->L.NP * 12 * sizeof(double);
  const size_t v32 = (size_t)n * c->L.NP * 12 * sizeof(float);
  int rc;
  if ((rc = dalloc(c, c->x64, v64, "alloc x"))) return rc;
  if ((rc = dalloc(c, c->b64, v64, "alloc b"))) return rc;
  if ((rc = dalloc(c, c->y, v64, "alloc y"))) return rc;
  if ((rc = dalloc(c, c->partial, (size_t)n * c->L.n_tiles * kPartialSlots * sizeof(double), "alloc partial")))
    return rc;
  if ((rc = dalloc(c, c->st, (size_t)n * sizeof(SysState), "alloc state"))) return rc;
  if ((rc = dalloc(c, c->st_outer, (size_t)n * sizeof(SysState), "alloc state"))) return rc;
  if (c->storage != FNLH_F64) {
    if ((rc = dalloc(c, c->r64, v64, "alloc r"))) return rc;
    if ((rc = dalloc(c, c->rhs32, v32, "alloc rhs32"))) return rc;
    if ((rc = dalloc(c, c->d32, v32, "alloc d32"))) return rc;
  }
  if (c->h_st) (void)hipHostFree(c->h_st);
  c->h_st = nullptr;
  HIPC(c, hipHostMalloc((void**)&c->h_st, 2 * (size_t)n * sizeof(SysState), hipHostMallocDefault), "host state");
  // vectors start at zero so padding rows stay zero
  HIPC(c, hipMemset(c->x64.p, 0, v64), "zero");
  HIPC(c, hipMemset(c->b64.p, 0, v64), "zero");
  HIPC(c, hipMemset(c->y.p, 0, v64), "zero");
  if (c->storage != FNLH_F64) {
    HIPC(c, hipMemset(c->r64.p, 0, v64), "zero");
    HIPC(c, hipMemset(c->rhs32.p, 0, v32), "zero");
    HIPC(c, hipMemset(c->d32.p, 0, v32), "zero");
  }
  c->vec_cap = n;
  return FNLH_OK;
}

int ensure_slots(fnlh_ctx c, int slots) {
  if (slots <= c->n_slots) return FNLH_OK;
  const size_t per = (size_t)c->L.n_tiles * dinv_tile_elems(c->storage) * dinv_elem_bytes(c->storage);
  int rc = dalloc(c, c->dinv, per * slots, "alloc factor slots");
  if (rc) return rc;
  HIPC(c, hipMemset(c->dinv.p, 0, per * slots), "zero factors");
  c->n_slots = slots;
  c->slot_sys.assign(slots, -1);
  c->slot_kind.assign(slots, -1);
  return FNLH_OK;
}

int64_t dinv_stride(fnlh_ctx c) { return c->L.n_tiles * dinv_tile_elems(c->storage); }

void invalidate_factors(fnlh_ctx c) {
  std::fill(c->slot_sys.begin(), c->slot_sys.end(), -1);
  std::fill(c->slot_kind.begin(), c->slot_kind.end(), -1);
  c->pl_packed = false;
}

// outer FP64 operator residual of the systems of sb (x64, b64 -> r, partial)
void outer_residual(fnlh_ctx c, int ns, const SysBatch& sb, double* r, hipStream_t s) {
  outer_residual_of(c, ns, sb, (const double*)c->x64.p, (const double*)c->b64.p, r, s);
}

// fkind: 0 DILU on the colour ordering, 1 the shifted diagonal blocks (SGS, Jacobi),
// 2 partition-local ILU(0) (blocks packed into position order first if stale)
int factor_batch(fnlh_ctx c, const SysBatch& sb, int fkind, hipStream_t s) {
  DevPattern p = c->pat();
  HIPC(c, hipMemsetAsync(c->d_err.p, 0, sizeof(int), s), "clear error flag");
  if (fkind == 2) {
    const PiluDev q = c->pilu();
    if (!c->pl_packed) {
      launch_pilu_pack(c->storage, q, c->offd.p, c->diag.p, c->pl_coup.p, c->pl_diag.p, s);
      c->pl_packed = true;
    }
    launch_pilu_factor(c->storage, p, q, c->pl_coup.p, c->pl_diag.p, c->dinv.p, dinv_stride(c), sb,
                       (int*)c->d_err.p, s);
  } else {
    for (int col = 0; col < c->L.n_colours; ++col)
      launch_factor(c->storage, fkind == 0, p, c->offd.p, c->diag.p, c->dinv.p, dinv_stride(c), sb,
                    c->L.ctile[col], c->L.ctile[col + 1] - c->L.ctile[col], c->L.cstart[col], (int*)c->d_err.p, s);
  }
  int rc = check_launch(c, "factor launch");
  if (rc) return rc;
  HIPC(c, hipMemcpyAsync(c->h_err, c->d_err.p, sizeof(int), hipMemcpyDeviceToHost, s), "read error flag");
  HIPC(c, hipStreamSynchronize(s), "factor sync");
  if (*c->h_err) return set_err(c, FNLH_E_SINGULAR, "factorisation: singular or non-finite diagonal block");
  return FNLH_OK;
}

// kPathHybrid: the two-colours-plus-remainder sweep of a colouring whose first two
// colours hold almost every row (see one_sweep)
// kPathPilu: the partition-local ILU(0) sweep (one launch per sweep)
enum Path { kPathRB, kPathGeneral, kPathJacobi, kPathHybrid, kPathPilu };

// The passes of the hybrid sweep's remainder, for their byte model.
enum RemPass { kRemNorm = 1, kRemFwd = 2, kRemBwd = 3, kRemCorrect = 4 };

// One timed launch: kernel kind, colour, sweep index (0 = the initial pass), events,
// and the remainder pass (RemPass, 0 otherwise).
struct LaunchRec {
  int kind, colour, sweep;
  hipEvent_t a, b;
  double ms;
  int mode;
};

struct Timer {
  fnlh_ctx c;
  hipStream_t s;
  std::vector<LaunchRec> recs;
  size_t harvested = 0;
  bool pooled = true;                 // events come from (and return to) the context pool
  std::vector<hipEvent_t>* own = nullptr;  // graph capture: events owned by the graph
  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pooled) {
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      own->push_back(e);
      return e;
    }
    if (c->evpool.empty()) {
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    e = c->evpool.back();
    c->evpool.pop_back();
    return e;
  }
  bool open = false;
  void begin(int kind, int colour, int sweep, int mode = 0) {
    open = c->stats_on && sweep % c->stats_period == 0;
    if (!open) return;
    LaunchRec r{kind, colour, sweep, get(), get(), 0.0, mode};
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end() {
    if (!open) return;
    (void)hipEventRecord(recs.back().b, s);
    open = false;
  }
  // after a stream synchronisation: read durations, recycle pooled events
  void harvest() {
    for (; harvested < recs.size(); ++harvested) {
      LaunchRec& r = recs[harvested];
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      r.ms = ms;
      if (pooled) {
        c->evpool.push_back(r.a);
        c->evpool.push_back(r.b);
      }
    }
  }
};

}  // namespace

// A captured run of `K` sweeps (all after the first), replayed with hipGraphLaunch.
struct GraphEntry {
  // key
  int path, storage, spw, lpr, pivot, wg, ns, K;
  SysBatch sb;
  const void *x, *b, *y, *st;
  double rtol, divf;
  bool stats;
  uint64_t gen = 0;  // buffer generation at capture
  // value
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> events;
  std::vector<LaunchRec> tmpl;  // timed launches inside, sweep = offset within the graph
  uint64_t last_use = 0;
};

namespace {

// Algorithmic bytes of one launch (compulsory traffic: each block, vector entry and
// factor entry touched once), for `na` active systems.
double alg_bytes(fnlh_ctx c, int kind, int col, int na, int mode = 0) {
  const Layout& L = c->L;
  const double sA = (double)c->block_bytes();
  const double sv = (double)c->tv_bytes();
  const double blk = 36.0 * sA;
  const double dv = dinv_row_bytes(c->storage);  // one row's factor inverse
  auto nrows = [&](int cc) { return (double)L.ccount[cc]; };
  double shared = 0.0, per = 0.0;
  switch (kind) {
    case FNLH_KSTAT_SWEEP_UPDATE:
      shared = L.c_deg[col] * (blk + 4) + nrows(col) * (blk + 12);
      per = nrows(col) * (3 * 12 * sv + dv) + L.c_nbr[col] * 12 * sv;
      break;
    case FNLH_KSTAT_SWEEP_SET:  // solves with the shifted diagonal block, no factor read
      shared = L.c_deg[col] * (blk + 4) + nrows(col) * (blk + 12);
      per = nrows(col) * (2 * 12) * sv + L.c_nbr[col] * 12 * sv;
      break;
    case FNLH_KSTAT_FWD:
    case FNLH_KSTAT_FWD_LAST: {
      const bool last = col == L.n_colours - 1;
      shared = L.c_deg[col] * (blk + 4) + nrows(col) * (blk + 12);
      per = nrows(col) * ((last ? 4 : 3) * 12 * sv + dv) + (L.c_nbr[col] + L.c_nbr_lower[col]) * 12 * sv;
      break;
    }
    case FNLH_KSTAT_REMAINDER:
      if (mode == kRemNorm) {  // every colour from col on: b and x read, neighbours' x
        for (int cc = col; cc < L.n_colours; ++cc) {
          shared += L.c_deg[cc] * (blk + 4) + nrows(cc) * (blk + 12);
          per += nrows(cc) * 2 * 12 * sv + L.c_nbr[cc] * 12 * sv;
        }
      } else if (mode == kRemFwd) {  // b, x read; x, y written; the factor
        shared = L.c_deg[col] * (blk + 4) + nrows(col) * (blk + 12);
        per = nrows(col) * (4 * 12 * sv + dv) + L.c_nbr[col] * 12 * sv;
      } else if (mode == kRemBwd) {  // upper couplings; x, y read and written; the factor
        shared = L.c_deg_upper[col] * blk + L.c_deg[col] * 4;
        per = nrows(col) * (4 * 12 * sv + dv) + L.c_nbr_upper[col] * 12 * sv;
      } else {  // kRemCorrect: the second colour's rows coupled upwards, their upward couplings
        shared = (double)c->hyb_ents * (blk + 8) + (double)c->hyb_rows * 4;
        per = (double)c->hyb_rows * (2 * 12 * sv + dv) + L.c_nbr_upper[col] * 12 * sv;
      }
      break;
    case FNLH_KSTAT_BWD:
      shared = L.c_deg_upper[col] * blk + L.c_deg[col] * 4;
      per = nrows(col) * (4 * 12 * sv + dv) + L.c_nbr_upper[col] * 12 * sv;
      break;
    case FNLH_KSTAT_PILU: {  // in-partition couplings, diagonal blocks and tables; per
                             // system b read, x read and written, the factor
      const PiluLayout& Q = c->pl;
      shared = (double)Q.n_coup * (blk + 12) + (double)L.N * (blk + 4);
      per = (double)L.N * (3 * 12 * sv + dv);
      break;
    }
    case FNLH_KSTAT_JACOBI: {
      double deg = 0;
      for (int cc = 0; cc < L.n_colours; ++cc) deg += L.c_deg[cc];
      shared = deg * (blk + 4) + (double)L.N * (blk + 12);
      per = (double)L.N * (3 * 12 * sv + dv);
      break;
    }
  }
  return shared + na * per;
}

// Fold a finished loop's launches into the context totals; S_j = final sweeps.
void account(fnlh_ctx c, Timer& t, const SysBatch& sb, const SysState* h) {
  if (!c->stats_on) return;
  for (const LaunchRec& r : t.recs) {
    int na = 0;
    for (int k = 0; k < sb.n; ++k) {
      const int S = h[sb.vslot[k]].sweeps;
      na += (r.sweep == 0 ? S >= 1 : S >= r.sweep) ? 1 : 0;
    }
    c->st_ms[r.kind] += r.ms;
    c->st_n[r.kind] += 1;
    c->st_bytes[r.kind] += alg_bytes(c, r.kind, r.colour, na, r.mode);
  }
  t.recs.clear();
  t.harvested = 0;
}

// One preconditioned sweep for the systems of sb (vectors x, b, y of type TV).
void one_sweep(fnlh_ctx c, Path path, const SweepCfg& cfg, int ns, const SysBatch& sb, void* x, const void* b,
               void* y, SysState* st, int k, double rtol, double divf, hipStream_t s, Timer& T) {
  const bool first = k == 1;
  DevPattern p = c->pat();
  const Layout& L = c->L;
  const int64_t ds = dinv_stride(c);
  double* part = (double*)c->partial.p;
  if (path == kPathRB) {
    T.begin(FNLH_KSTAT_SWEEP_UPDATE, 1, k);
    launch_rb_pass(cfg, true, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, ns, sb, st, part, L.ctile[1],
                   L.ctile[2] - L.ctile[1], s);
    T.end();
    // the update pass's norms are reduced by the first workgroups of the pass that follows
    FusedReduce fr;
    fr.n = sb.n;
    fr.slots = rb_slots(cfg, sb.n);
    fr.mode = first ? kReduceSweepNoNorm : kReduceSweep;
    fr.t0 = L.ctile[1];
    fr.nt = L.ctile[2] - L.ctile[1];
    fr.rtol2 = rtol * rtol;
    fr.div2 = divf * divf;
    const bool fuse = L.ctile[1] > L.ctile[0];
    if (!fuse)
      launch_reduce(sb, part, L.n_tiles, fr.t0, fr.nt, fr.slots, st, fr.mode, rtol, divf, 0, s);
    T.begin(FNLH_KSTAT_SWEEP_SET, 0, k);
    launch_rb_pass(cfg, false, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, ns, sb, st, part, L.ctile[0],
                   L.ctile[1] - L.ctile[0], s, fuse ? &fr : nullptr);
    T.end();
  } else if (path == kPathHybrid) {
    // Colours C0, C1 hold almost every row; C2 .. C(m-1) are a small remainder (e.g. the
    // rows at blade-row interfaces).  With x updated in place, the DILU step is
    //   forward, colours ascending:  x_c += y_c,  y_c = Dt_c^-1 (b - K x)_c
    //   backward, colours descending: x_c += -Dt_c^-1 sum_{upper} K z (z_c = y_c + that)
    // and, as in the two-colour pass, the C0 residual is zero on entry (y_C0 = 0) and C0's
    // backward step is x_C0 = (K_ii + i w)^-1 (b - sum K x): so a sweep is the C1 update
    // pass, forward and backward passes over the remainder colours, the correction of the
    // C1 rows coupled to the remainder, and the first-colour pass, which reduces the
    // norms.  Blocks of C0 and C1 are read once per sweep (the general passes read them
    // 1.5 times).  The norm is that of the iterate the sweep starts from: C1's in the
    // update pass, the remainder's in a first pass that only reads (C0's is zero).
    const int m = L.n_colours;
    T.begin(FNLH_KSTAT_REMAINDER, 2, k, kRemNorm);
    launch_fwd(cfg, kFwdNorm, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, y, ns, sb, st, part, L.ctile[2],
               L.ctile[m] - L.ctile[2], L.cstart[2], s);
    T.end();
    T.begin(FNLH_KSTAT_SWEEP_UPDATE, 1, k);
    launch_rb_pass(cfg, true, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, ns, sb, st, part, L.ctile[1],
                   L.ctile[2] - L.ctile[1], s);
    T.end();
    for (int col = 2; col < m; ++col) {
      T.begin(FNLH_KSTAT_REMAINDER, col, k, kRemFwd);
      launch_fwd(cfg, kFwdHybrid, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, y, ns, sb, st, part, L.ctile[col],
                 L.ctile[col + 1] - L.ctile[col], L.cstart[col], s);
      T.end();
    }
    for (int col = m - 2; col >= 2; --col) {
      T.begin(FNLH_KSTAT_REMAINDER, col, k, kRemBwd);
      launch_bwd(cfg, kBwdHybrid, p, c->offd.p, c->dinv.p, ds, x, y, ns, sb, st, L.ctile[col],
                 L.ctile[col + 1] - L.ctile[col], L.cstart[col + 1], s);
      T.end();
    }
    if (c->hyb_groups > 0) {
      T.begin(FNLH_KSTAT_REMAINDER, 1, k, kRemCorrect);
      launch_correct(cfg.storage, p, c->corr(), c->offd.p, c->dinv.p, ds, x, y, ns, sb, st, s);
      T.end();
    }
    FusedReduce fr;
    fr.n = sb.n;
    fr.slots = rb_slots(cfg, sb.n);
    fr.mode = first ? kReduceSweepNoNorm : kReduceSweep;
    fr.t0 = L.ctile[1];
    fr.nt = L.ctile[m] - L.ctile[1];
    fr.rtol2 = rtol * rtol;
    fr.div2 = divf * divf;
    T.begin(FNLH_KSTAT_SWEEP_SET, 0, k);
    launch_rb_pass(cfg, false, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, ns, sb, st, part, L.ctile[0],
                   L.ctile[1] - L.ctile[0], s, &fr);
    T.end();
  } else if (path == kPathPilu) {
    const PiluDev q = c->pilu();
    double* pp = (double*)c->pl_partial.p;
    T.begin(FNLH_KSTAT_PILU, 0, k);
    launch_pilu_sweep(cfg.storage, p, q, c->pl_coup.p, c->pl_diag.p, c->dinv.p, ds, x, b, ns, sb, st, pp,
                      c->pl_lds_max, s);
    T.end();
    launch_reduce(sb, pp, q.pt, 0, q.pt, kPartialSlots, st, kReduceSweep, rtol, divf, 0, s);
  } else if (path == kPathGeneral) {
    const int m = L.n_colours;
    for (int col = 0; col < m; ++col) {
      const bool last = col == m - 1;
      T.begin(last ? FNLH_KSTAT_FWD_LAST : FNLH_KSTAT_FWD, col, k);
      launch_fwd(cfg, last ? kFwdLast : kFwdGeneral, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, y, ns, sb, st,
                 part, L.ctile[col], L.ctile[col + 1] - L.ctile[col], L.cstart[col], s);
      T.end();
    }
    launch_reduce(sb, part, L.n_tiles, 0, L.n_tiles, rb_slots(cfg, sb.n), st, kReduceSweep, rtol, divf, 0, s);
    for (int col = m - 2; col >= 0; --col) {
      T.begin(FNLH_KSTAT_BWD, col, k);
      launch_bwd(cfg, kBwdGeneral, p, c->offd.p, c->dinv.p, ds, x, y, ns, sb, st, L.ctile[col],
                 L.ctile[col + 1] - L.ctile[col], L.cstart[col + 1], s);
      T.end();
    }
  } else {
    T.begin(FNLH_KSTAT_JACOBI, 0, k);
    launch_jacobi(cfg, p, c->offd.p, c->diag.p, c->dinv.p, ds, x, b, y, ns, sb, st, part, s);
    T.end();
    launch_reduce(sb, part, L.n_tiles, 0, L.n_tiles, 1, st, kReduceSweep, rtol, divf, 0, s);
    launch_axpy_y(cfg.storage, p, x, y, ns, sb, st, s);
  }
}

bool same_key(const GraphEntry* g, uint64_t gen, int path, const SweepCfg& cfg, int ns, int K, const SysBatch& sb,
              const void* x, const void* b, const void* y, const void* st, double rtol, double divf, bool stats) {
  if (g->gen != gen || g->path != path || g->storage != cfg.storage || g->spw != cfg.spw || g->lpr != cfg.lanes_per_row ||
      g->pivot != (int)cfg.pivot || g->wg != (int)cfg.wave_groups || g->ns != ns || g->K != K || g->x != x || g->b != b || g->y != y ||
      g->st != st || g->rtol != rtol || g->divf != divf || g->stats != stats || g->sb.n != sb.n)
    return false;
  for (int k = 0; k < sb.n; ++k)
    if (g->sb.orow[k] != sb.orow[k] || g->sb.dslot[k] != sb.dslot[k] || g->sb.vslot[k] != sb.vslot[k]) return false;
  return true;
}

void destroy_graph(GraphEntry* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  for (auto e : g->events) (void)hipEventDestroy(e);
  delete g;
}

// Find or capture the graph of K sweeps for this configuration (nullptr: capture failed).
GraphEntry* get_graph(fnlh_ctx c, Path path, const SweepCfg& cfg, int ns, int K, const SysBatch& sb, void* x,
                      const void* b, void* y, SysState* st, double rtol, double divf) {
  static uint64_t tick = 0;
  // graphs captured before a buffer was (re)allocated may point at freed memory
  for (size_t i = 0; i < c->graphs.size();) {
    if (c->graphs[i]->gen != c->buf_gen) {
      destroy_graph(c->graphs[i]);
      c->graphs.erase(c->graphs.begin() + i);
    } else {
      ++i;
    }
  }
  for (GraphEntry* g : c->graphs)
    if (same_key(g, c->buf_gen, path, cfg, ns, K, sb, x, b, y, st, rtol, divf, c->stats_on)) {
      g->last_use = ++tick;
      return g;
    }
  if (c->graph_broken) return nullptr;
  if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->graph_broken = true;
    return nullptr;
  }
  GraphEntry* g = new GraphEntry();
  g->gen = c->buf_gen;
  g->path = path;
  g->storage = cfg.storage;
  g->spw = cfg.spw;
  g->lpr = cfg.lanes_per_row;
  g->wg = (int)cfg.wave_groups;
  g->pivot = cfg.pivot;
  g->ns = ns;
  g->K = K;
  g->sb = sb;
  g->x = x;
  g->b = b;
  g->y = y;
  g->st = st;
  g->rtol = rtol;
  g->divf = divf;
  g->stats = c->stats_on;
  Timer T{c, c->cap, {}, 0, false, &g->events};
  hipGraph_t graph = nullptr;
  bool ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (int i = 0; i < K; ++i) one_sweep(c, path, cfg, ns, sb, x, b, y, st, 2 + i, rtol, divf, c->cap, T);
    ok = hipStreamEndCapture(c->cap, &graph) == hipSuccess && graph;
  }
  (void)hipGetLastError();
  if (ok) ok = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (!ok) {
    c->graph_broken = true;
    destroy_graph(g);
    return nullptr;
  }
  for (auto& r : T.recs) r.sweep -= 2;
  g->tmpl = T.recs;
  g->last_use = ++tick;
  if (c->graphs.size() >= 8) {
    auto it = std::min_element(c->graphs.begin(), c->graphs.end(),
                               [](GraphEntry* a, GraphEntry* b2) { return a->last_use < b2->last_use; });
    destroy_graph(*it);
    c->graphs.erase(it);
  }
  c->graphs.push_back(g);
  return g;
}

// Iterate until every system of sb is inactive.  States must be initialised.  Sweeps
// after the first are replayed from a captured graph of check_every sweeps when
// use_graph is set (direct launches otherwise, or if capture is unavailable).
// chunk: launch about max_sweeps sweeps (whole graph replays) and return with the states
// read back; otherwise run until every system has stopped (max_sweeps plus one to retire).
int sweep_loop(fnlh_ctx c, Path path, const SweepCfg& cfg, int ns, const SysBatch& sb, void* x, const void* b,
               void* y, SysState* st, double rtol, double divf, int max_sweeps, int check_every, bool use_graph,
               hipStream_t s, bool chunk = false) {
  const int limit = chunk ? max_sweeps : max_sweeps + 2;
  Timer T{c, s, {}, 0, true, nullptr};
  if (path == kPathRB || path == kPathHybrid) {
    DevPattern p = c->pat();
    T.begin(FNLH_KSTAT_SWEEP_SET, 0, 0);
    launch_rb_pass(cfg, false, p, c->offd.p, c->diag.p, c->dinv.p, dinv_stride(c), x, b, ns, sb, st,
                   (double*)c->partial.p, c->L.ctile[0], c->L.ctile[1] - c->L.ctile[0], s);
    T.end();
  }
  int launched = 0;
  SysState* h = c->h_st;
  GraphEntry* g = nullptr;
  // each system needs at most max_sweeps sweeps plus one to retire
  while (launched < limit) {
    if (launched == 0) {
      one_sweep(c, path, cfg, ns, sb, x, b, y, st, 1, rtol, divf, s, T);
      launched = 1;
      // per-kernel timing needs events around every launch; events recorded by graph
      // nodes cannot be queried for elapsed time here, so timing runs launch directly
      if (use_graph && !c->stats_on) g = get_graph(c, path, cfg, ns, check_every, sb, x, b, y, st, rtol, divf);
      if (!g) {
        for (int i = 1; i < check_every && launched < limit; ++i, ++launched)
          one_sweep(c, path, cfg, ns, sb, x, b, y, st, launched + 1, rtol, divf, s, T);
      }
    } else if (g) {
      HIPC(c, hipGraphLaunch(g->exec, s), "graph launch");
      if (c->stats_on)
        for (const LaunchRec& r : g->tmpl) T.recs.push_back(LaunchRec{r.kind, r.colour, launched + 1 + r.sweep,
                                                                       r.a, r.b, 0.0, r.mode});
      launched += check_every;
    } else {
      for (int i = 0; i < check_every && launched < limit; ++i, ++launched)
        one_sweep(c, path, cfg, ns, sb, x, b, y, st, launched + 1, rtol, divf, s, T);
    }
    int rc = check_launch(c, "sweep launch");
    if (rc) return rc;
    HIPC(c, hipMemcpyAsync(h, st, sizeof(SysState) * (sb.vslot[sb.n - 1] + 1), hipMemcpyDeviceToHost, s),
         "read states");
    HIPC(c, hipStreamSynchronize(s), "sweep sync");
    // graph events are re-recorded on every replay: read them now, never recycle them
    for (; T.harvested < T.recs.size(); ++T.harvested) {
      LaunchRec& r = T.recs[T.harvested];
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      r.ms = ms;
      bool from_graph = false;
      if (g)
        for (auto e : g->events)
          if (e == r.a) {
            from_graph = true;
            break;
          }
      if (!from_graph) {
        c->evpool.push_back(r.a);
        c->evpool.push_back(r.b);
      }
    }
    bool any = false;
    for (int k = 0; k < sb.n; ++k) any |= h[sb.vslot[k]].active != 0;
    if (!any) break;
  }
  account(c, T, sb, h);
  return FNLH_OK;
}

// Dominance of the diagonal blocks (decides the first-colour solve), once per matrix.
// The two-colours-plus-remainder sweep (kPathHybrid) pays when the colours past the
// second are a small remainder: it reads C0 and C1 once per sweep but adds a few small
// launches.
constexpr double kHybridMaxRemainder = 0.25;  // largest fraction of rows past C1
bool hybrid_ok(fnlh_ctx c) {
  const Layout& L = c->L;
  if (!c->hybrid || L.n_colours < 3) return false;
  if (c->hybrid == 2) return true;
  int64_t rest = 0;
  for (int k = 2; k < L.n_colours; ++k) rest += L.ccount[k];
  return (double)rest <= kHybridMaxRemainder * (double)L.N;
}

// The second-colour rows coupled to a higher colour (the rows the hybrid sweep corrects
// after the remainder's backward passes), packed 64 to a group with their upward
// couplings in slot order; counts of rows and entries for the byte model.
int setup_hybrid(fnlh_ctx c) {
  const Layout& L = c->L;
  c->hyb_groups = c->hyb_rows = c->hyb_ents = 0;
  if (L.n_colours < 3) return FNLH_OK;
  std::vector<int32_t> rows;
  std::vector<std::vector<int32_t>> ents;
  for (int64_t t = L.ctile[1]; t < L.ctile[2]; ++t) {
    for (int lane = 0; lane < L.tile_nrows[t]; ++lane) {
      std::vector<int32_t> up;
      for (int q = 0; q < L.tile_width[t]; ++q) {
        const int64_t fe = (L.tile_slot0[t] + q) * kTile + lane;
        if (L.ent_edge[fe] != 0 && L.ent_nbr[fe] >= L.cstart[2]) up.push_back((int32_t)fe);
      }
      if (!up.empty()) {
        rows.push_back((int32_t)(t * kTile + lane));
        ents.push_back(up);
      }
    }
  }
  if (rows.empty()) return FNLH_OK;
  const int64_t ng = ((int64_t)rows.size() + kTile - 1) / kTile;
  std::vector<int32_t> row(ng * kTile, -1), width(ng, 0);
  std::vector<int64_t> slot0(ng, 0);
  int64_t slots = 0;
  for (int64_t g = 0; g < ng; ++g) {
    int32_t w = 0;
    for (int lane = 0; lane < kTile && g * kTile + lane < (int64_t)rows.size(); ++lane)
      w = std::max<int32_t>(w, (int32_t)ents[g * kTile + lane].size());
    width[g] = w;
    slot0[g] = slots;
    slots += w;
  }
  std::vector<int32_t> fe(slots * kTile, -1);
  for (int64_t i = 0; i < (int64_t)rows.size(); ++i) {
    const int64_t g = i / kTile;
    const int lane = (int)(i % kTile);
    row[i] = rows[i];
    for (size_t k = 0; k < ents[i].size(); ++k) fe[(slot0[g] + (int64_t)k) * kTile + lane] = ents[i][k];
    c->hyb_ents += (int64_t)ents[i].size();
  }
  c->hyb_rows = (int64_t)rows.size();
  c->hyb_groups = ng;
  int rc;
  if ((rc = dupload(c, c->corr_row, row, "pattern")) || (rc = dupload(c, c->corr_width, width, "pattern")) ||
      (rc = dupload(c, c->corr_slot0, slot0, "pattern")) || (rc = dupload(c, c->corr_fe, fe, "pattern")))
    return rc;
  return FNLH_OK;
}

int ensure_dominance(fnlh_ctx c, hipStream_t s) {
  if (c->dom_known) return FNLH_OK;
  int rc;
  if (!c->d_dom.p && (rc = dalloc(c, c->d_dom, sizeof(int), "alloc flag"))) return rc;
  if (!c->h_dom) HIPC(c, hipHostMalloc((void**)&c->h_dom, sizeof(int), hipHostMallocDefault), "host flag");
  const int one = 1;
  HIPC(c, hipMemcpyAsync(c->d_dom.p, &one, sizeof(int), hipMemcpyHostToDevice, s), "set flag");
  launch_check_dominance(c->storage, c->pat(), c->diag.p, (int*)c->d_dom.p, s);
  if ((rc = check_launch(c, "dominance launch"))) return rc;
  HIPC(c, hipMemcpyAsync(c->h_dom, c->d_dom.p, sizeof(int), hipMemcpyDeviceToHost, s), "read flag");
  HIPC(c, hipStreamSynchronize(s), "dominance sync");
  c->dom = *c->h_dom != 0;
  c->dom_known = true;
  return FNLH_OK;
}

// The partition-local ILU(0) tables for the current partitions (built on first use),
// its packed-block buffers, and norm partials for n systems.
int ensure_pilu(fnlh_ctx c, int n, hipStream_t s) {
  if (c->part_host.empty())
    return set_err(c, FNLH_E_ORDER, "partition-local ILU: no partitions (fnlh_set_partitions first)");
  int rc;
  if (!c->pl_built) {
    // the largest LDS a workgroup's y vector may take: the device's less a reserve for the
    // sweep's static LDS, once the sweep kernels allow it
    int dev_lds = 0;
    constexpr int kStaticReserve = 1024;
    if (hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->dev) == hipSuccess &&
        dev_lds - kStaticReserve > c->pl_lds_max && pilu_allow_lds(c->storage, dev_lds - kStaticReserve))
      c->pl_lds_max = dev_lds - kStaticReserve;
    (void)hipGetLastError();
    const int64_t N = c->L.N;
    const int32_t fit = c->pl_lds_max / pilu_lds_row_bytes(c->storage);
    int32_t unit = c->pl_unit_rows > 0 ? c->pl_unit_rows : (int32_t)std::min<int64_t>(1024, std::max<int64_t>(64, N / 2048));
    unit = std::min(unit, fit);
    std::string e;
    if ((rc = build_pilu(c->L, c->part_host, unit, c->pl, e))) return set_err(c, rc, e);
    const PiluLayout& Q = c->pl;
    if (Q.n_groups > c->L.n_tiles) return set_err(c, FNLH_E_ARG, "partition-local ILU: factor slots too small");
    const size_t slot_bytes = (size_t)c->slot_elems_storage() * c->block_bytes();
    if ((rc = dupload(c, c->pl_unit_ptr, Q.unit_ptr, "partition tables")) ||
        (rc = dupload(c, c->pl_unit_lev, Q.unit_lev, "partition tables")) ||
        (rc = dupload(c, c->pl_lev_ptr, Q.lev_ptr, "partition tables")) ||
        (rc = dupload(c, c->pl_pos_row, Q.pos_row, "partition tables")) ||
        (rc = dupload(c, c->pl_gwidth, Q.g_width, "partition tables")) ||
        (rc = dupload(c, c->pl_gslot0, Q.g_slot0, "partition tables")))
      return rc;
    if (Q.n_slots > 0 && ((rc = dupload(c, c->pl_epos, Q.e_pos, "partition tables")) ||
                          (rc = dupload(c, c->pl_erow, Q.e_row, "partition tables")) ||
                          (rc = dupload(c, c->pl_esrc, Q.e_src, "partition tables")) ||
                          (rc = dupload(c, c->pl_erev, Q.e_rev, "partition tables")) ||
                          (rc = dalloc(c, c->pl_coup, (size_t)Q.n_slots * slot_bytes, "alloc packed blocks"))))
      return rc;
    if ((rc = dalloc(c, c->pl_diag, (size_t)Q.n_groups * slot_bytes, "alloc packed blocks"))) return rc;
    dfree(c->pl_partial);
    c->pl_cap = 0;
    c->pl_built = true;
    c->pl_packed = false;
    c->buf_gen++;  // captured sweeps hold the tables' addresses
  }
  if (pilu_systems_per_group(c->storage, 1, c->pl.max_rows, c->pl_lds_max) < 1)
    return set_err(c, FNLH_E_ARG,
                   "partition-local ILU: the largest partition has " + std::to_string(c->pl.max_part) +
                       " cells; at most " + std::to_string(c->pl_lds_max / pilu_lds_row_bytes(c->storage)) +
                       " fit in a workgroup's LDS");
  if (n > c->pl_cap) {
    const size_t bytes = (size_t)n * c->pilu().pt * kPartialSlots * sizeof(double);
    if ((rc = dalloc(c, c->pl_partial, bytes, "alloc partition partials"))) return rc;
    HIPC(c, hipMemsetAsync(c->pl_partial.p, 0, bytes, s), "zero partition partials");  // entries past n_units
    c->pl_cap = n;
    c->buf_gen++;
  }
  return FNLH_OK;
}

// ---------------------------------------------------------------- relax phases
struct RelaxPlan {
  Path path = kPathRB;
  SweepCfg cfg;
  bool reduced = false, use_graph = false, learned = false;
  int learn_every = 16;
  double inner_rtol = 1e-4, divf = 1e3;
  int inner_max = 1, check_every = 8, fkind = 0, G = 1;
  std::vector<double> tf, ts;
};

// Validate, size the scratch, move x and b into the internal layout, pick the path.
int relax_prepare(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b,
                  const fnlh_relax_opts* o, hipStream_t s, RelaxPlan& P) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "relax: matrix and harmonics first");
  if (n < 1 || !sys || !x || !b || !o) return set_err(c, FNLH_E_ARG, "relax: bad arguments");
  for (int j = 0; j < n; ++j) {
    if (sys[j] < 0 || sys[j] >= c->n_sys) return set_err(c, FNLH_E_ARG, "relax: system out of range");
    if (!x[j] || !b[j]) return set_err(c, FNLH_E_ARG, "relax: null vector");
  }
  if (o->kind != FNLH_DILU && o->kind != FNLH_SGS && o->kind != FNLH_JACOBI && o->kind != FNLH_LEARNED &&
      o->kind != FNLH_PILU)
    return set_err(c, FNLH_E_ARG, "relax: unsupported preconditioner kind");
  if (o->learn_every < 0) return set_err(c, FNLH_E_ARG, "relax: learn_every >= 0");
  if (o->max_sweeps < 0 || !(o->rtol >= 0.0)) return set_err(c, FNLH_E_ARG, "relax: need max_sweeps >= 0, rtol >= 0");
  P.check_every = o->check_every > 0 ? o->check_every : 8;
  P.divf = o->div_factor > 0 ? o->div_factor : 1e3;
  P.reduced = c->storage != FNLH_F64;
  P.inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : (c->storage == FNLH_F32 ? 1e-4 : 1e-2);
  P.inner_max = o->inner_sweeps > 0 ? o->inner_sweeps : std::max(1, o->max_sweeps);
  P.use_graph = o->use_graph != 0;
  P.learned = o->kind == FNLH_LEARNED;
  if (P.learned)
    for (int j = 0; j < n; ++j)
      if (c->is_frozen(sys[j])) return set_err(c, FNLH_E_ARG, "relax: the learned kind does not take frozen-turbulence systems");
  P.learn_every = o->learn_every > 0 ? o->learn_every : 16;
  int rc;
  if ((rc = ensure_vectors(c, n))) return rc;
  if (P.learned && (rc = nn_relax_begin(c, n, s))) return rc;
  if (o->kind == FNLH_PILU && (rc = ensure_pilu(c, n, s))) return rc;
  const int want_slots = c->factor_slots_opt > 0 ? c->factor_slots_opt : std::min<int>(c->n_sys, 64);
  if ((rc = ensure_slots(c, want_slots))) return rc;
  if ((rc = ensure_dominance(c, s))) return rc;
  DevPattern p = c->pat();
  launch_to_internal_n(p, (const int32_t*)c->iperm.p, x, n, (double*)c->x64.p, n, 0, s);
  launch_to_internal_n(p, (const int32_t*)c->iperm.p, b, n, (double*)c->b64.p, n, 0, s);
  P.path = o->kind == FNLH_JACOBI ? kPathJacobi
           : o->kind == FNLH_PILU ? kPathPilu
                                  : (c->L.n_colours == 2 ? kPathRB : (hybrid_ok(c) ? kPathHybrid : kPathGeneral));
  // frozen-turbulence systems run on the stored-factor kernels (the two-colour pass solves
  // the first colour's full 6x6 diagonal block in place); their sixth unknown starts at 0
  bool frozen = false;
  for (int j = 0; j < n; ++j)
    if (c->is_frozen(sys[j])) {
      frozen = true;
      launch_zero_sixth(c->L.NP, (double*)c->x64.p, n, j, s);
    }
  if (frozen && (P.path == kPathRB || P.path == kPathHybrid)) P.path = kPathGeneral;
  P.fkind = (o->kind == FNLH_DILU || o->kind == FNLH_LEARNED) ? 0 : o->kind == FNLH_PILU ? 2 : 1;
  P.cfg.storage = c->storage;
  P.cfg.spw = c->lanes_per_sys;
  P.cfg.lanes_per_row = c->lanes_per_row;
  P.cfg.wave_groups = c->wave_groups != 0;
  P.cfg.pivot = !c->dom;
  P.G = std::min({n, kMaxBatch, c->n_slots});
  P.tf.assign(n, 0.0);
  P.ts.assign(n, 0.0);
  return FNLH_OK;
}

// Assign factor slots to the systems of sb (reusing cached factors) and factor the rest.
int relax_factor(fnlh_ctx c, SysBatch& sb, int fkind, hipStream_t s) {
  std::vector<int> used(c->n_slots, 0);
  SysBatch need;
  need.n = 0;
  for (int k = 0; k < sb.n; ++k) {
    sb.dslot[k] = -1;
    for (int q = 0; q < c->n_slots; ++q)
      if (!used[q] && c->slot_sys[q] == sb.orow[k] && c->slot_kind[q] == fkind) {
        sb.dslot[k] = q;
        used[q] = 1;
        break;
      }
  }
  for (int k = 0; k < sb.n; ++k) {
    if (sb.dslot[k] >= 0) continue;
    int q = 0;
    while (used[q]) ++q;
    used[q] = 1;
    sb.dslot[k] = q;
    need.orow[need.n] = sb.orow[k];
    need.dslot[need.n] = q;
    need.vslot[need.n] = sb.vslot[k];
    need.n++;
  }
  if (!need.n) return FNLH_OK;
  for (int k = 0; k < need.n; ++k) {
    c->slot_sys[need.dslot[k]] = -1;
    c->slot_kind[need.dslot[k]] = -1;
  }
  int rc = factor_batch(c, need, fkind, s);
  if (rc) return rc;
  for (int k = 0; k < need.n; ++k) {
    c->slot_sys[need.dslot[k]] = need.orow[k];
    c->slot_kind[need.dslot[k]] = fkind;
  }
  return FNLH_OK;
}

// Defect correction: FP64 residual (in r64) -> FP32 inner right-hand side, inner states.
void outer_to_inner(fnlh_ctx c, int ns, const SysBatch& sb, const SysState* so, SysState* st, int inner_max,
                    hipStream_t s) {
  launch_to_f32(c->pat(), (const double*)c->r64.p, (float*)c->rhs32.p, (float*)c->d32.p, ns, sb, so, s);
  launch_inner_init(sb, so, st, inner_max, s);
}
// x64 += d32, new FP64 residual, outer stop test.
void inner_to_outer(fnlh_ctx c, int ns, const SysBatch& sb, const SysState* st, SysState* so, double rtol,
                    double divf, hipStream_t s) {
  launch_outer_update(sb, st, so, s);
  launch_add_f32(c->pat(), (double*)c->x64.p, (const float*)c->d32.p, ns, sb, so, s);
  outer_residual(c, ns, sb, (double*)c->r64.p, s);
  launch_reduce(sb, (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, so, kReduceOuter, rtol, divf, 0,
                s);
}

// Outer residual of the returned iterates (into fin), x back to user order.
int relax_finish_launch(fnlh_ctx c, int n, const int32_t* sys, double* const* x, SysState* fin, hipStream_t s) {
  for (int g0 = 0; g0 < n; g0 += kMaxBatch) {
    SysBatch sb;
    sb.n = std::min(kMaxBatch, n - g0);
    for (int k = 0; k < sb.n; ++k) {
      sb.orow[k] = sys[g0 + k];
      sb.vslot[k] = g0 + k;
      sb.dslot[k] = 0;
    }
    outer_residual(c, n, sb, nullptr, s);
    launch_reduce(sb, (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, fin, kReduceFinal, 0, 0, 0, s);
  }
  DevPattern p = c->pat();
  launch_to_user_n(p, (const int32_t*)c->iperm.p, (const double*)c->x64.p, x, n, n, 0, s);
  return check_launch(c, "final launch");
}

// Severity order of the per-system outcomes: OK < FELL_BACK < NOT_CONVERGED < DIVERGED.
int status_rank(int st) {
  return st == FNLH_OK ? 0 : st == FNLH_FELL_BACK ? 1 : st == FNLH_NOT_CONVERGED ? 2 : 3;
}
int worse_status(int a, int b) { return status_rank(b) > status_rank(a) ? b : a; }

// c: the context whose network's controller reports systems switched off (learned kind)
int relax_reports(const SysState* h, int n, const RelaxPlan& P, const fnlh_relax_opts* o, fnlh_sys_report* rep,
                  const int* counts = nullptr, fnlh_ctx c = nullptr) {
  int worst = FNLH_OK;
  for (int j = 0; j < n; ++j) {
    const SysState& S0 = h[j];
    fnlh_sys_report R;
    std::memset(&R, 0, sizeof(R));
    R.sweeps = S0.sweeps;
    R.outer = P.reduced ? S0.outer_iters : 0;
    R.res0 = std::sqrt(S0.norm0sq);
    R.rel_res = S0.norm0sq > 0 ? std::sqrt(S0.last_n2 / S0.norm0sq) : 0.0;
    int status = S0.status;
    if (status != FNLH_DIVERGED) status = (R.rel_res <= o->rtol) ? FNLH_OK : FNLH_NOT_CONVERGED;
    if (!std::isfinite(R.rel_res)) status = FNLH_DIVERGED;
    if (status == FNLH_OK && counts && c && nn_system_off(c, j)) status = FNLH_FELL_BACK;
    R.status = status;
    R.t_factor_ms = P.tf.empty() ? 0.0 : P.tf[j];
    R.t_sweep_ms = P.ts.empty() ? 0.0 : P.ts[j];
    if (counts) {
      R.learned = counts[2 * j];
      R.fallbacks = counts[2 * j + 1];
    }
    if (rep) rep[j] = R;
    worst = worse_status(worst, status);
  }
  return worst;
}


// ---------------------------------------------------------------- batching
struct BatchGroup {
  int SW = 4, P = 1;
  int64_t w0_off = 0, w0_n = 0, w1_off = 0, w1_n = 0;  // into the C0 / C1 work lists
};

}  // namespace

struct fnlh_batch_s {
  std::vector<fnlh_ctx> inst;
  std::string err;
  DevBuf desc, work0, work1, items, st, sto;
  SysState* h_st = nullptr;
  size_t h_cap = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_K = -1, g_storage = -1;
  double g_rtol = -1, g_divf = -1;
  std::vector<BatchGroup> groups;
  int n_items = 0;
  // full lists (all batched instances) and the per-instance state ranges, for compaction
  std::vector<WorkItem> all_w0, all_w1, all_items;
  std::vector<std::pair<int, int>> group_key;  // (SW, P) per group
  std::vector<int> inst_group, inst_base, inst_ns;  // per descriptor
  // instances of at least this many cells are iterated alone (0: none); 80k cells (about
  // 100 MB of FP32 blocks) measured best on the uneven 64-instance workload
  int64_t loop_cells = 80000;
};

namespace {

int bset_err(fnlh_batch b, int code, const std::string& m) {
  b->err = m;
  return code;
}

int bdalloc(fnlh_batch b, DevBuf& d, size_t bytes) {
  if (d.bytes >= bytes && d.p) return FNLH_OK;
  if (d.p) (void)hipFree(d.p);
  d.p = nullptr;
  d.bytes = 0;
  if (hipMalloc(&d.p, bytes) != hipSuccess) return bset_err(b, FNLH_E_OOM, "batch: device allocation failed");
  d.bytes = bytes;
  if (b->exec) {  // graphs hold buffer addresses
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  return FNLH_OK;
}

// Rebuild the device work lists keeping only the instances flagged live.
int compact_lists(fnlh_batch B, const std::vector<char>& live, hipStream_t s) {
  std::vector<WorkItem> w0, w1, it;
  for (size_t g = 0; g < B->groups.size(); ++g) {
    BatchGroup& G = B->groups[g];
    G.w0_off = (int64_t)w0.size();
    G.w1_off = (int64_t)w1.size();
    for (const WorkItem& w : B->all_w0)
      if (live[w.inst] && B->inst_group[w.inst] == (int)g) w0.push_back(w);
    for (const WorkItem& w : B->all_w1)
      if (live[w.inst] && B->inst_group[w.inst] == (int)g) w1.push_back(w);
    G.w0_n = (int64_t)w0.size() - G.w0_off;
    G.w1_n = (int64_t)w1.size() - G.w1_off;
  }
  for (const WorkItem& w : B->all_items)
    if (live[w.inst]) it.push_back(w);
  B->n_items = (int)it.size();
  if (!w0.empty() &&
      hipMemcpyAsync(B->work0.p, w0.data(), sizeof(WorkItem) * w0.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return bset_err(B, FNLH_E_HIP, "batch: upload failed");
  if (!w1.empty() &&
      hipMemcpyAsync(B->work1.p, w1.data(), sizeof(WorkItem) * w1.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return bset_err(B, FNLH_E_HIP, "batch: upload failed");
  if (!it.empty() &&
      hipMemcpyAsync(B->items.p, it.data(), sizeof(WorkItem) * it.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return bset_err(B, FNLH_E_HIP, "batch: upload failed");
  if (B->exec) {  // the graph holds the old list lengths
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  return FNLH_OK;
}

void batched_sweep(fnlh_batch B, int storage, bool first, double rtol, double divf, hipStream_t s) {
  const InstDesc* d = (const InstDesc*)B->desc.p;
  const WorkItem* w0 = (const WorkItem*)B->work0.p;
  const WorkItem* w1 = (const WorkItem*)B->work1.p;
  for (const BatchGroup& g : B->groups)
    launch_rb_batched(storage, g.SW, g.P, true, d, w1 + g.w1_off, g.w1_n, s, true);
  // the update passes' norm reductions ride in the first first-colour launch
  const int mode = first ? kReduceSweepNoNorm : kReduceSweep;
  const WorkItem* red = (const WorkItem*)B->items.p;
  bool reduced = false;
  for (const BatchGroup& g : B->groups) {
    const bool here = !reduced;
    launch_rb_batched(storage, g.SW, g.P, false, d, w0 + g.w0_off, g.w0_n, s, true, here ? red : nullptr,
                      here ? B->n_items : 0, mode, rtol, divf);
    reduced = true;
  }
  if (!reduced) launch_reduce_batched(d, red, B->n_items, mode, rtol, divf, s);
}

// All systems of the batch to their stop criteria (states in B->st, initialised).  At
// every check the work lists are compacted to the instances that still iterate.
int batched_loop(fnlh_batch B, int storage, double rtol, double divf, int max_sweeps, int check_every, bool use_graph,
                 int total, hipStream_t s, bool chunk = false) {
  const int limit = chunk ? max_sweeps : max_sweeps + 2;
  const int nd = (int)B->inst_group.size();
  std::vector<char> live(nd, 1);
  int rc = compact_lists(B, live, s);
  if (rc) return rc;
  const InstDesc* d = (const InstDesc*)B->desc.p;
  const WorkItem* w0 = (const WorkItem*)B->work0.p;
  for (const BatchGroup& g : B->groups)
    launch_rb_batched(storage, g.SW, g.P, false, d, w0 + g.w0_off, g.w0_n, s, true);
  int launched = 0;
  while (launched < limit) {
    bool graph = false;
    if (launched == 0) {
      batched_sweep(B, storage, true, rtol, divf, s);
      launched = 1;
    }
    if (use_graph) {
      if (B->exec && (B->g_K != check_every || B->g_storage != storage || B->g_rtol != rtol || B->g_divf != divf)) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
      }
      if (!B->exec) {
        if (!B->cap) (void)hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
        hipGraph_t gr = nullptr;
        bool ok = B->cap && hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
          for (int i = 0; i < check_every; ++i) batched_sweep(B, storage, false, rtol, divf, B->cap);
          ok = hipStreamEndCapture(B->cap, &gr) == hipSuccess && gr;
        }
        if (ok) ok = hipGraphInstantiate(&B->exec, gr, nullptr, nullptr, 0) == hipSuccess;
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        if (ok) {
          B->g_K = check_every;
          B->g_storage = storage;
          B->g_rtol = rtol;
          B->g_divf = divf;
        } else {
          B->exec = nullptr;
        }
      }
      graph = B->exec != nullptr;
    }
    if (graph) {
      if (hipGraphLaunch(B->exec, s) != hipSuccess) return bset_err(B, FNLH_E_HIP, "batch: graph launch failed");
      launched += check_every;
    } else {
      for (int i = 0; i < check_every && launched < limit; ++i, ++launched)
        batched_sweep(B, storage, false, rtol, divf, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bset_err(B, FNLH_E_HIP, std::string("batch: launch: ") + hipGetErrorString(e));
    if (hipMemcpyAsync(B->h_st, B->st.p, sizeof(SysState) * total, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bset_err(B, FNLH_E_HIP, "batch: state read-back failed");
    bool any = false, changed = false;
    for (int i = 0; i < nd; ++i) {
      if (!live[i]) continue;
      bool a = false;
      for (int k = 0; k < B->inst_ns[i]; ++k) a |= B->h_st[B->inst_base[i] + k].active != 0;
      if (!a) {
        live[i] = 0;
        changed = true;
      }
      any |= a;
    }
    if (!any) break;
    if (changed && (rc = compact_lists(B, live, s))) return rc;
  }
  return FNLH_OK;
}

}  // namespace

extern "C" {

const char* fnlh_version(void) { return "fnlh 0.1 gfx950"; }

const char* fnlh_last_error(fnlh_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int fnlh_order_mesh(const fnlh_mesh* mesh, const fnlh_options* opts, int32_t* colour, int32_t* perm,
                    int32_t* n_colours) {
  if (!mesh || !opts) return set_err(nullptr, FNLH_E_ARG, "null mesh or options");
  Layout L;
  std::string e;
  int rc = build_layout(*mesh, *opts, L, e);
  if (rc) return set_err(nullptr, rc, e);
  if (colour) std::copy(L.colour_user.begin(), L.colour_user.end(), colour);
  if (perm) std::copy(L.perm.begin(), L.perm.end(), perm);
  if (n_colours) *n_colours = L.n_colours;
  return FNLH_OK;
}

int fnlh_create(fnlh_ctx* out, const fnlh_mesh* mesh, const fnlh_options* opts) {
  if (!out) return set_err(nullptr, FNLH_E_ARG, "null output pointer");
  *out = nullptr;
  if (!mesh || !opts) return set_err(nullptr, FNLH_E_ARG, "null mesh or options");
  fnlh_ctx c = new fnlh_ctx_s();
  std::string e;
  int rc = build_layout(*mesh, *opts, c->L, e);
  if (rc) {
    delete c;
    return set_err(nullptr, rc, e);
  }
  c->dev = opts->device;
  c->storage = opts->storage;
  c->outer = opts->outer;
  c->factor_slots_opt = opts->factor_slots;
  auto fail = [&](int code) {
    g_create_error = c->err;
    fnlh_destroy(c);
    return code;
  };
  hipError_t he = hipSetDevice(c->dev);
  if (he != hipSuccess) {
    hip_fail(c, he, "hipSetDevice");
    return fail(FNLH_E_HIP);
  }
  if ((rc = noalloc_init(c))) return fail(rc);
  const Layout& L = c->L;
  if ((rc = dupload(c, c->tile_nrows, L.tile_nrows, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->tile_width, L.tile_width, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->tile_slot0, L.tile_slot0, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->ent_nbr, L.ent_nbr, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->ent_edge, L.ent_edge, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->ent_rev, L.ent_rev, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->vol, L.vol, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->zone, L.zone, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->iperm, L.iperm, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->perm, L.perm, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->edge_ent, L.edge_ent, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->bf_ptr, L.bf_ptr, "pattern"))) return fail(rc);
  if ((rc = dupload(c, c->bf_idx, L.bf_idx, "pattern"))) return fail(rc);
  if ((rc = setup_hybrid(c))) return fail(rc);
  {
    std::vector<double> a(mesh->area, mesh->area + 3 * mesh->n_edges);
    if ((rc = dupload(c, c->area, a, "geometry"))) return fail(rc);
    std::vector<double> ba(mesh->bface_area, mesh->bface_area + 3 * mesh->n_bfaces);
    if ((rc = dupload(c, c->bface_area, ba, "geometry"))) return fail(rc);
  }
  const size_t be = c->block_bytes();
  if ((rc = dalloc(c, c->offd, (size_t)L.n_slots * c->slot_elems_storage() * be, "alloc blocks"))) return fail(rc);
  if ((rc = dalloc(c, c->diag, (size_t)L.n_tiles * c->slot_elems_storage() * be, "alloc blocks"))) return fail(rc);
  if (c->offd.p && hipMemset(c->offd.p, 0, c->offd.bytes) != hipSuccess) return fail(FNLH_E_HIP);
  if (hipMemset(c->diag.p, 0, c->diag.bytes) != hipSuccess) return fail(FNLH_E_HIP);
  if ((rc = dalloc(c, c->d_err, sizeof(int), "alloc flag"))) return fail(rc);
  if (hipHostMalloc((void**)&c->h_err, sizeof(int), hipHostMallocDefault) != hipSuccess) return fail(FNLH_E_HIP);
  for (auto& ev : c->ev)
    if (hipEventCreate(&ev) != hipSuccess) return fail(FNLH_E_HIP);
  *out = c;
  return FNLH_OK;
}

int fnlh_destroy(fnlh_ctx c) {
  if (!c) return FNLH_E_ARG;
  nn_release(c);
  DevBuf* bufs[] = {&c->tile_nrows, &c->tile_width, &c->tile_slot0, &c->ent_nbr, &c->ent_edge, &c->ent_rev,
                    &c->vol, &c->zone, &c->iperm, &c->perm, &c->edge_ent, &c->bf_ptr, &c->bf_idx, &c->area,
                    &c->bface_area, &c->offd, &c->diag, &c->offd64, &c->diag64, &c->state, &c->bstate,
                    &c->d_omega, &c->dinv, &c->x64, &c->b64, &c->r64, &c->y, &c->rhs32, &c->d32, &c->partial,
                    &c->st, &c->st_outer, &c->d_err, &c->ent_phase, &c->phase_cs, &c->sys_frozen, &c->ent_drop,
                    &c->corr_row, &c->corr_width, &c->corr_slot0, &c->corr_fe, &c->pl_unit_ptr,
                    &c->pl_unit_lev, &c->pl_lev_ptr, &c->pl_pos_row, &c->pl_gwidth, &c->pl_gslot0, &c->pl_epos, &c->pl_erow, &c->pl_esrc, &c->pl_erev, &c->pl_coup,
                    &c->pl_diag, &c->pl_partial};
  for (DevBuf* b : bufs) dfree(*b);
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_err) (void)hipHostFree(c->h_err);
  for (auto& ev : c->ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : c->evpool) (void)hipEventDestroy(ev);
  for (auto g : c->graphs) destroy_graph(g);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->h_dom) (void)hipHostFree(c->h_dom);
  dfree(c->d_dom);
  delete c;
  return FNLH_OK;
}

int fnlh_assemble_jacobian(fnlh_ctx c, const double* state, const double* bstate, double eps, double sigma,
                           int32_t scheme, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!state) return set_err(c, FNLH_E_ARG, "assemble: null state");
  if (scheme != FNLH_IMPLICIT && scheme != FNLH_EXPLICIT) return set_err(c, FNLH_E_ARG, "assemble: bad scheme");
  if (scheme == FNLH_IMPLICIT && !(eps * sigma > 0.0 && std::isfinite(eps * sigma)))
    return set_err(c, FNLH_E_ARG, "assemble: need eps * sigma > 0");
  hipStream_t s = S(stream);
  int rc;
  if (!c->state.p && (rc = dalloc(c, c->state, (size_t)c->L.NP * 6 * sizeof(double), "alloc state"))) return rc;
  DevPattern p = c->pat();
  launch_to_internal(p, (const int32_t*)c->iperm.p, state, (double*)c->state.p, 6, 1, 0, s);
  if (bstate && c->L.B > 0) {
    if (!c->bstate.p && (rc = dalloc(c, c->bstate, (size_t)c->L.B * 6 * sizeof(double), "alloc bstate"))) return rc;
    HIPC(c, hipMemcpyAsync(c->bstate.p, bstate, (size_t)c->L.B * 6 * sizeof(double), hipMemcpyDeviceToDevice, s),
         "copy bstate");
  } else {
    dfree(c->bstate);
  }
  c->eps = eps;
  c->sigma = sigma;
  c->scheme = scheme;
  launch_assemble(c->storage, p, c->flow(), c->offd.p, c->diag.p, s);
  launch_drop_blocks(c->storage, p, c->L.n_slots, (const int8_t*)c->ent_drop.p, c->offd.p, s);
  if ((rc = check_launch(c, "assemble launch"))) return rc;
  dfree(c->offd64);
  dfree(c->diag64);
  c->have_shadow = false;
  c->have_matrix = true;
  c->assembled = true;
  c->dom_known = false;
  invalidate_factors(c);
  return FNLH_OK;
}

int fnlh_set_blocks(fnlh_ctx c, const double* diag, const double* offd, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!diag || (c->L.E > 0 && !offd)) return set_err(c, FNLH_E_ARG, "set_blocks: null blocks");
  hipStream_t s = S(stream);
  DevPattern p = c->pat();
  launch_set_blocks(c->storage, p, c->L.N, c->L.E, (const int32_t*)c->perm.p, (const int64_t*)c->edge_ent.p, diag,
                    offd, c->offd.p, c->diag.p, s);
  int rc;
  if (c->storage != FNLH_F64 && c->outer == FNLH_OUTER_EXACT) {
    if (!c->offd64.p && (rc = dalloc(c, c->offd64, (size_t)c->L.n_slots * 18 * 64 * 2 * 8, "alloc shadow")))
      return rc;
    if (!c->diag64.p && (rc = dalloc(c, c->diag64, (size_t)c->L.n_tiles * 18 * 64 * 2 * 8, "alloc shadow")))
      return rc;
    if (c->offd64.p) HIPC(c, hipMemsetAsync(c->offd64.p, 0, c->offd64.bytes, s), "zero shadow");
    HIPC(c, hipMemsetAsync(c->diag64.p, 0, c->diag64.bytes, s), "zero shadow");
    launch_set_blocks(kF64, p, c->L.N, c->L.E, (const int32_t*)c->perm.p, (const int64_t*)c->edge_ent.p, diag, offd,
                      c->offd64.p, c->diag64.p, s);
    launch_drop_blocks(kF64, p, c->L.n_slots, (const int8_t*)c->ent_drop.p, c->offd64.p, s);
    c->have_shadow = true;
  }
  launch_drop_blocks(c->storage, p, c->L.n_slots, (const int8_t*)c->ent_drop.p, c->offd.p, s);
  if ((rc = check_launch(c, "set_blocks launch"))) return rc;
  c->have_matrix = true;
  c->assembled = false;
  c->dom_known = false;
  invalidate_factors(c);
  return FNLH_OK;
}

int fnlh_get_blocks(fnlh_ctx c, double* diag, double* offd, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix) return set_err(c, FNLH_E_ORDER, "get_blocks: no matrix yet");
  if (!diag || (c->L.E > 0 && !offd)) return set_err(c, FNLH_E_ARG, "get_blocks: null output");
  hipStream_t s = S(stream);
  launch_get_blocks(c->storage, c->pat(), c->L.N, c->L.E, (const int32_t*)c->perm.p, (const int64_t*)c->edge_ent.p,
                    c->offd.p, c->diag.p, diag, offd, s);
  return check_launch(c, "get_blocks launch");
}

int fnlh_set_harmonics(fnlh_ctx c, int32_t n_sys, const double* omega, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix) return set_err(c, FNLH_E_ORDER, "set_harmonics: assemble or set blocks first");
  if (n_sys < 1 || n_sys > 4096 || !omega) return set_err(c, FNLH_E_ARG, "set_harmonics: need 1 <= n_sys <= 4096");
  const size_t n = (size_t)n_sys * c->L.n_zones;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(omega[i])) return set_err(c, FNLH_E_ARG, "set_harmonics: non-finite omega");
  c->omega.assign(omega, omega + n);
  int rc;
  // the table keeps its buffer while it fits (captured sweep graphs hold its address)
  if (n * sizeof(double) > c->d_omega.bytes && (rc = dalloc(c, c->d_omega, n * sizeof(double), "alloc omega")))
    return rc;
  HIPC(c, hipMemcpy(c->d_omega.p, omega, n * sizeof(double), hipMemcpyHostToDevice), "copy omega");
  c->n_sys = n_sys;
  invalidate_factors(c);
  if (c->sys_frozen.p) {  // no system frozen (fnlh_set_frozen_turbulence sets them)
    dfree(c->sys_frozen);
    c->buf_gen++;
  }
  c->frozen.clear();
  if (c->ent_phase.p) {  // every system's phase back to 0 (fnlh_set_phase_lag sets them)
    c->ibpa.assign(n_sys, 0.0);
    std::vector<double> cs(2 * (size_t)n_sys);
    for (int s = 0; s < n_sys; ++s) {
      cs[2 * s] = 1.0;
      cs[2 * s + 1] = 0.0;
    }
    if (c->phase_cs.bytes == cs.size() * sizeof(double)) {
      HIPC(c, hipMemcpy(c->phase_cs.p, cs.data(), c->phase_cs.bytes, hipMemcpyHostToDevice), "phase table");
    } else if ((rc = dupload(c, c->phase_cs, cs, "phase table"))) {
      return rc;
    }
  }
  (void)stream;
  return FNLH_OK;
}

int fnlh_set_phase_lag(fnlh_ctx c, const int8_t* edge_phase, int32_t n_sys, const double* sigma) {
  if (!c) return FNLH_E_ARG;
  if (c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "set_phase_lag: set the harmonics first");
  int rc;
  if (!edge_phase) {  // no periodic couplings
    dfree(c->ent_phase);
    dfree(c->phase_cs);
    c->ibpa.clear();
    c->edge_phase_host.clear();
    c->buf_gen++;
    return FNLH_OK;
  }
  if (n_sys != c->n_sys || !sigma)
    return set_err(c, FNLH_E_ARG, "set_phase_lag: one phase per system of set_harmonics");
  const Layout& L = c->L;
  for (int64_t e = 0; e < L.E; ++e)
    if (edge_phase[e] < -1 || edge_phase[e] > 1) return set_err(c, FNLH_E_ARG, "set_phase_lag: edge signs are -1, 0, +1");
  for (int s = 0; s < n_sys; ++s)
    if (!std::isfinite(sigma[s])) return set_err(c, FNLH_E_ARG, "set_phase_lag: non-finite phase");
  const bool same = c->ent_phase.p && c->edge_phase_host.size() == (size_t)L.E &&
                    std::equal(edge_phase, edge_phase + L.E, c->edge_phase_host.begin());
  if (!same) {
    // per entry: the edge's sign seen from its first cell, negated from its second
    std::vector<int8_t> ph(L.ent_edge.size(), 0);
    for (size_t f = 0; f < L.ent_edge.size(); ++f) {
      const int32_t e = L.ent_edge[f];
      if (e == 0) continue;
      const int8_t sg = edge_phase[std::abs(e) - 1];
      ph[f] = (int8_t)(e > 0 ? sg : -sg);
    }
    if ((rc = dupload(c, c->ent_phase, ph, "periodic couplings"))) return rc;
    c->edge_phase_host.assign(edge_phase, edge_phase + L.E);
  }
  std::vector<double> cs(2 * (size_t)n_sys);
  for (int s = 0; s < n_sys; ++s) {
    cs[2 * s] = std::cos(sigma[s]);
    cs[2 * s + 1] = std::sin(sigma[s]);
  }
  if (c->phase_cs.bytes == cs.size() * sizeof(double)) {  // same buffer: graphs stay valid
    HIPC(c, hipMemcpy(c->phase_cs.p, cs.data(), c->phase_cs.bytes, hipMemcpyHostToDevice), "phase table");
  } else if ((rc = dupload(c, c->phase_cs, cs, "phase table"))) {
    return rc;
  }
  c->ibpa.assign(sigma, sigma + n_sys);
  return FNLH_OK;
}

int fnlh_set_partitions(fnlh_ctx c, const int32_t* part, void* stream) {
  if (!c) return FNLH_E_ARG;
  const Layout& L = c->L;
  std::vector<int8_t> drop;
  std::vector<int32_t> ph;
  bool any = false;
  if (part) {
    ph.assign(part, part + L.N);
    drop.assign(L.ent_nbr.size(), 0);
    for (int64_t e = 0; e < L.E; ++e) {
      const int64_t f0 = L.edge_ent[2 * e], f1 = L.edge_ent[2 * e + 1];
      // entry f0 is (a -> b): its neighbour is b; entry f1 (b -> a) has neighbour a
      const int32_t ua = L.iperm[L.ent_nbr[f1]], ub = L.iperm[L.ent_nbr[f0]];
      if (part[ua] != part[ub]) {
        drop[f0] = drop[f1] = 1;
        any = true;
      }
    }
  }
  if (!any) ph.clear();
  if (ph == c->part_host) return FNLH_OK;  // same couplings dropped as before
  const bool had = c->ent_drop.p != nullptr;
  int rc;
  if (!any) {
    dfree(c->ent_drop);
  } else if ((rc = dupload(c, c->ent_drop, drop, "partition couplings"))) {
    return rc;
  }
  c->part_host = ph;
  c->pl_built = false;  // the partition-local ILU tables follow the partitions
  c->pl_packed = false;
  c->buf_gen++;  // captured sweeps hold the flag table's address
  if (c->have_matrix) {
    if (had) {
      // blocks dropped by the previous partitions are gone: the matrix must be set again
      c->have_matrix = false;
      c->assembled = false;
    } else {
      hipStream_t s = S(stream);
      const DevPattern p = c->pat();
      launch_drop_blocks(c->storage, p, L.n_slots, (const int8_t*)c->ent_drop.p, c->offd.p, s);
      if (c->have_shadow) launch_drop_blocks(kF64, p, L.n_slots, (const int8_t*)c->ent_drop.p, c->offd64.p, s);
      if ((rc = check_launch(c, "partition launch"))) return rc;
    }
    invalidate_factors(c);
  }
  return FNLH_OK;
}

int fnlh_set_frozen_turbulence(fnlh_ctx c, int32_t n_sys, const int8_t* flags) {
  if (!c) return FNLH_E_ARG;
  if (c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "set_frozen_turbulence: set the harmonics first");
  bool any = false;
  if (flags) {
    if (n_sys != c->n_sys) return set_err(c, FNLH_E_ARG, "set_frozen_turbulence: one flag per system of set_harmonics");
    for (int s = 0; s < n_sys; ++s) {
      if (flags[s] != 0 && flags[s] != 1) return set_err(c, FNLH_E_ARG, "set_frozen_turbulence: flags are 0 or 1");
      any |= flags[s] == 1;
    }
  }
  std::vector<uint8_t> f;
  if (any) f.assign(flags, flags + n_sys);
  if (f == c->frozen) return FNLH_OK;
  int rc;
  if (!any) {
    dfree(c->sys_frozen);
  } else if ((rc = dupload(c, c->sys_frozen, f, "frozen flags"))) {
    return rc;
  }
  c->frozen = f;
  c->buf_gen++;  // captured sweeps hold the flag table's address
  invalidate_factors(c);
  return FNLH_OK;
}

int fnlh_residual(fnlh_ctx c, int32_t sys, const double* x, const double* b, double* r, double* norm2,
                  void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "residual: matrix and harmonics first");
  if (sys < 0 || sys >= c->n_sys) return set_err(c, FNLH_E_ARG, "residual: system out of range");
  if (!x || !b) return set_err(c, FNLH_E_ARG, "residual: null vector");
  hipStream_t s = S(stream);
  int rc;
  if ((rc = ensure_vectors(c, 1))) return rc;
  DevPattern p = c->pat();
  launch_to_internal(p, (const int32_t*)c->iperm.p, x, (double*)c->x64.p, 12, 1, 0, s);
  launch_to_internal(p, (const int32_t*)c->iperm.p, b, (double*)c->b64.p, 12, 1, 0, s);
  if (c->is_frozen(sys)) launch_zero_sixth(c->L.NP, (double*)c->x64.p, 1, 0, s);
  SysBatch sb;
  sb.n = 1;
  sb.orow[0] = sys;
  sb.dslot[0] = 0;
  sb.vslot[0] = 0;
  double* rint = r ? (double*)c->y.p : nullptr;
  outer_residual(c, 1, sb, rint, s);
  launch_reduce(sb, (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, (SysState*)c->st.p, kReduceFinal, 0,
                0, 0, s);
  if (r) launch_to_user(p, (const int32_t*)c->iperm.p, rint, r, 12, 1, 0, s);
  if ((rc = check_launch(c, "residual launch"))) return rc;
  HIPC(c, hipMemcpyAsync(c->h_st, c->st.p, sizeof(SysState), hipMemcpyDeviceToHost, s), "read state");
  HIPC(c, hipStreamSynchronize(s), "residual sync");
  if (norm2) *norm2 = c->h_st[0].last_n2;
  return FNLH_OK;
}

}  // extern "C"

namespace fnlh {

int precond_prepare(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b, int kind,
                    int inner, bool use_graph, hipStream_t s, PrecondPlan& out) {
  if (!c) return FNLH_E_ARG;
  if (kind != FNLH_DILU && kind != FNLH_SGS && kind != FNLH_JACOBI && kind != FNLH_LEARNED && kind != FNLH_PILU)
    return set_err(c, FNLH_E_ARG, "preconditioner kind must be DILU, SGS, JACOBI, LEARNED or PILU");
  if (inner < 1) return set_err(c, FNLH_E_ARG, "inner sweeps >= 1");
  fnlh_relax_opts o{};
  o.kind = kind;
  o.max_sweeps = inner;
  o.rtol = 0.0;
  o.check_every = inner + 2;
  o.inner_sweeps = inner;
  o.use_graph = use_graph ? 1 : 0;
  RelaxPlan P;
  int rc = relax_prepare(c, n, sys, x, b, &o, s, P);
  if (rc) return rc;
  if (P.G < n) return set_err(c, FNLH_E_ARG, "more systems than factor slots (fnlh_options.factor_slots)");
  SysBatch sb;
  sb.n = n;
  for (int k = 0; k < n; ++k) {
    sb.orow[k] = sys[k];
    sb.vslot[k] = k;
  }
  if ((rc = relax_factor(c, sb, P.fkind, s))) return rc;
  out.path = P.path;
  out.fkind = P.fkind;
  out.inner = inner;
  out.reduced = P.reduced;
  out.use_graph = use_graph;
  out.learned = P.learned;
  out.cfg = P.cfg;
  return FNLH_OK;
}

int precond_apply(fnlh_ctx c, const PrecondPlan& pp, int ns, const SysBatch& sb, const double* v, double* z,
                  hipStream_t s) {
  if (sb.n <= 0) return FNLH_OK;
  // the factor slots of these systems (cached: no refactorisation)
  SysBatch fb = sb;
  int rc;
  if ((rc = relax_factor(c, fb, pp.fkind, s))) return rc;
  const DevPattern p = c->pat();
  SysState* st = (SysState*)c->st.p;
  const size_t zb = (size_t)c->L.NP * ns * 12 * sizeof(double);
  // exactly `inner` sweeps from zero: launched directly, no host synchronisation (the
  // states retire every system after its last sweep; with per-kernel timing on, or graph
  // replay asked for, the sweep loop of fnlh_relax runs them instead)
  auto run = [&](void* xz, const void* bb) -> int {
    if (c->stats_on || pp.use_graph)
      return sweep_loop(c, (Path)pp.path, pp.cfg, ns, fb, xz, bb, c->y.p, st, 0.0, 1e30, pp.inner, pp.inner + 2,
                        pp.use_graph, s);
    Timer T{c, s, {}, 0, true, nullptr};
    if (pp.path == kPathRB || pp.path == kPathHybrid)
      launch_rb_pass(pp.cfg, false, p, c->offd.p, c->diag.p, c->dinv.p, dinv_stride(c), xz, bb, ns, fb, st,
                     (double*)c->partial.p, c->L.ctile[0], c->L.ctile[1] - c->L.ctile[0], s);
    for (int k = 1; k <= pp.inner; ++k)
      one_sweep(c, (Path)pp.path, pp.cfg, ns, fb, xz, bb, c->y.p, st, k, 0.0, 1e30, s, T);
    return FNLH_OK;
  };
  if (!pp.reduced) {
    launch_fill_zero(z, zb, s);
    launch_kstate(fb, st, 1.0, pp.inner, s);
    // the learned step moves z off zero (its residual there is v itself); the sweeps
    // continue from there on K z = v
    if (pp.learned) {
      HIPC(c, hipMemcpyAsync(nn_step_residual(c), v, zb, hipMemcpyDeviceToDevice, s), "learned residual");
      if ((rc = nn_learned_step(c, ns, fb, z, v, nn_step_residual(c), st, s))) return rc;
    }
    if ((rc = run(z, v))) return rc;
  } else {
    SysState* so = (SysState*)c->st_outer.p;
    launch_kstate(fb, so, 1.0, 1 << 30, s);
    launch_fill_zero(z, zb, s);
    const double* rv = v;
    if (pp.learned) {  // z = alpha d; the inner sweeps correct the FP64 residual v - K z
      rv = nn_step_residual(c);
      HIPC(c, hipMemcpyAsync((void*)rv, v, zb, hipMemcpyDeviceToDevice, s), "learned residual");
      if ((rc = nn_learned_step(c, ns, fb, z, v, (double*)rv, so, s))) return rc;
    }
    launch_to_f32(p, rv, (float*)c->rhs32.p, (float*)c->d32.p, ns, fb, so, s);
    launch_inner_init(fb, so, st, pp.inner, s);
    if ((rc = run(c->d32.p, c->rhs32.p))) return rc;
    launch_add_f32(p, z, (const float*)c->d32.p, ns, fb, so, s);
  }
  return check_launch(c, "preconditioner launch");
}

}  // namespace fnlh

extern "C" {

int fnlh_relax(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b,
               const fnlh_relax_opts* o, fnlh_sys_report* rep, void* stream) {
  RelaxPlan P;
  hipStream_t s = S(stream);
  int rc = relax_prepare(c, n, sys, x, b, o, s, P);
  if (rc) return rc;
  SysState* st = (SysState*)c->st.p;
  SysState* so = (SysState*)c->st_outer.p;
  // residual history: norm^2 per sweep on the device, [n][len]
  const int hlen = (o->history && o->history_len > 0) ? o->history_len : 0;
  DevBuf hist;
  struct FreeOnExit {
    DevBuf* b;
    ~FreeOnExit() { dfree(*b); }
  } hist_guard{&hist};
  if (hlen) {
    if ((rc = dalloc(c, hist, (size_t)n * hlen * sizeof(double), "alloc history"))) return rc;
    launch_fill_zero(hist.p, hist.bytes, s);
  }
  for (int g0 = 0; g0 < n; g0 += P.G) {
    SysBatch sb;
    sb.n = std::min(P.G, n - g0);
    for (int k = 0; k < sb.n; ++k) {
      sb.orow[k] = sys[g0 + k];
      sb.vslot[k] = g0 + k;
    }
    HIPC(c, hipEventRecord(c->ev[0], s), "event");
    if ((rc = relax_factor(c, sb, P.fkind, s))) return rc;
    HIPC(c, hipEventRecord(c->ev[1], s), "event");
    if (!P.reduced) {
      outer_residual(c, n, sb, nullptr, s);
      launch_reduce(sb, (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, st, kReduceInit, 0, 0,
                    o->max_sweeps, s);
      if (hlen) launch_set_history(sb, st, (double*)hist.p, hlen, s);
      if (!P.learned) {
        if ((rc = sweep_loop(c, P.path, P.cfg, n, sb, c->x64.p, c->b64.p, c->y.p, st, o->rtol, P.divf,
                             o->max_sweeps, P.check_every, P.use_graph, s)))
          return rc;
      } else {
        // chunks of sweeps, each followed by a learned correction of the active systems
        for (int done = 0;;) {
          const int chunk = std::min(P.learn_every, o->max_sweeps + 1 - done);
          if ((rc = sweep_loop(c, P.path, P.cfg, n, sb, c->x64.p, c->b64.p, c->y.p, st, o->rtol, P.divf,
                               std::max(chunk, 1), P.check_every, P.use_graph, s, true)))
            return rc;
          done += std::max(chunk, 1);
          bool any = false;
          for (int k = 0; k < sb.n; ++k) any |= c->h_st[sb.vslot[k]].active != 0;
          if (!any || done > o->max_sweeps) break;
          if ((rc = nn_learned_step(c, n, sb, (double*)c->x64.p, (const double*)c->b64.p, nullptr, st, s)))
            return rc;
        }
      }
    } else {
      outer_residual(c, n, sb, (double*)c->r64.p, s);
      launch_reduce(sb, (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, so, kReduceInit, 0, 0,
                    o->max_sweeps, s);
      if (hlen) launch_set_history(sb, so, (double*)hist.p, hlen, s);
      for (int it = 0; it < 100000; ++it) {
        if ((rc = check_launch(c, "outer launch"))) return rc;
        HIPC(c, hipMemcpyAsync(c->h_st, so, sizeof(SysState) * (sb.vslot[sb.n - 1] + 1), hipMemcpyDeviceToHost, s),
             "read states");
        HIPC(c, hipStreamSynchronize(s), "outer sync");
        bool any = false;
        for (int k = 0; k < sb.n; ++k) any |= c->h_st[sb.vslot[k]].active != 0;
        if (!any) break;
        outer_to_inner(c, n, sb, so, st, P.inner_max, s);
        if ((rc = sweep_loop(c, P.path, P.cfg, n, sb, c->d32.p, c->rhs32.p, c->y.p, st, P.inner_rtol, 1e30,
                             P.inner_max, P.check_every, P.use_graph, s)))
          return rc;
        inner_to_outer(c, n, sb, st, so, o->rtol, P.divf, s);
        if (P.learned &&
            (rc = nn_learned_step(c, n, sb, (double*)c->x64.p, (const double*)c->b64.p, (double*)c->r64.p, so, s)))
          return rc;
      }
    }
    HIPC(c, hipEventRecord(c->ev[2], s), "event");
    HIPC(c, hipEventSynchronize(c->ev[2]), "event sync");
    float fa = 0.f, fb = 0.f;
    (void)hipEventElapsedTime(&fa, c->ev[0], c->ev[1]);
    (void)hipEventElapsedTime(&fb, c->ev[1], c->ev[2]);
    for (int k = 0; k < sb.n; ++k) {
      P.tf[g0 + k] = fa;
      P.ts[g0 + k] = fb;
    }
  }
  SysState* fin = P.reduced ? so : st;
  if ((rc = relax_finish_launch(c, n, sys, x, fin, s))) return rc;
  HIPC(c, hipMemcpyAsync(c->h_st, fin, sizeof(SysState) * n, hipMemcpyDeviceToHost, s), "read states");
  HIPC(c, hipStreamSynchronize(s), "final sync");
  std::vector<int> counts;
  if (P.learned) {
    counts.assign(2 * n, 0);
    if ((rc = nn_relax_counts(c, n, counts.data(), s))) return rc;
  }
  std::vector<fnlh_sys_report> reps(n);
  const int worst = relax_reports(c->h_st, n, P, o, reps.data(), P.learned ? counts.data() : nullptr, c);
  if (rep) std::copy(reps.begin(), reps.end(), rep);
  if (hlen) {
    std::vector<double> h((size_t)n * hlen);
    HIPC(c, hipMemcpyAsync(h.data(), hist.p, hist.bytes, hipMemcpyDeviceToHost, s), "read history");
    HIPC(c, hipStreamSynchronize(s), "history sync");
    for (int j = 0; j < n; ++j) {
      double* out = o->history + (size_t)j * hlen;
      const int sw = reps[j].sweeps;
      for (int m = 0; m < hlen; ++m) {
        if (m < sw) out[m] = std::sqrt(std::max(h[(size_t)j * hlen + m], 0.0));
        else if (m == sw) out[m] = reps[j].rel_res * reps[j].res0;
        else out[m] = std::nan("");
      }
    }
  }
  return worst;
}


int fnlh_batch_create(fnlh_batch* out, int32_t n, const fnlh_ctx* inst) {
  if (!out) return set_err(nullptr, FNLH_E_ARG, "batch: null output");
  *out = nullptr;
  if (n < 1 || !inst) return set_err(nullptr, FNLH_E_ARG, "batch: need n >= 1 instances");
  for (int i = 0; i < n; ++i) {
    if (!inst[i]) return set_err(nullptr, FNLH_E_ARG, "batch: null instance");
    if (inst[i]->storage != inst[0]->storage || inst[i]->dev != inst[0]->dev)
      return set_err(nullptr, FNLH_E_ARG, "batch: instances differ in storage precision or device");
  }
  fnlh_batch b = new fnlh_batch_s();
  b->inst.assign(inst, inst + n);
  *out = b;
  return FNLH_OK;
}

int fnlh_batch_destroy(fnlh_batch b) {
  if (!b) return FNLH_E_ARG;
  DevBuf* bufs[] = {&b->desc, &b->work0, &b->work1, &b->items, &b->st, &b->sto};
  for (DevBuf* d : bufs) dfree(*d);
  if (b->h_st) (void)hipHostFree(b->h_st);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return FNLH_OK;
}

const char* fnlh_batch_last_error(fnlh_batch b) { return b ? b->err.c_str() : g_create_error.c_str(); }

int fnlh_batch_set_loop_cells(fnlh_batch B, int64_t loop_cells) {
  if (!B) return FNLH_E_ARG;
  B->loop_cells = loop_cells > 0 ? loop_cells : 0;
  return FNLH_OK;
}

int fnlh_batch_autotune(fnlh_batch B, const int32_t* n_sys, const int32_t* const* sys, double* const* const* x,
                        const double* const* const* bvec, const fnlh_relax_opts* o, int32_t n_cand,
                        const int64_t* cand, int64_t* pick, double* ms, void* stream) {
  if (!B) return FNLH_E_ARG;
  if (!n_sys || !sys || !x || !bvec || !o || n_cand < 1 || n_cand > 64 || !cand) {
    B->err = "batch autotune: bad arguments";
    return FNLH_E_ARG;
  }
  hipStream_t s = S(stream);
  const int n = (int)B->inst.size();
  auto zero_x = [&]() {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n_sys[i]; ++j)
        if (x[i] && x[i][j]) launch_fill_zero(x[i][j], (size_t)B->inst[i]->L.N * 12 * sizeof(double), s);
  };
  fnlh_ctx c0 = B->inst[0];
  const int64_t save = B->loop_cells;
  double best = 1e300;
  int64_t best_lc = save;
  for (int k = 0; k < n_cand; ++k) {
    B->loop_cells = cand[k] > 0 ? cand[k] : 0;
    float f = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // a warm-up (factors, graphs), then one timed solve
      zero_x();
      if (hipEventRecord(c0->ev[0], s) != hipSuccess) return hip_fail(c0, hipGetLastError(), "event");
      const int rc = fnlh_batch_relax(B, n_sys, sys, x, bvec, o, nullptr, stream);
      if (rc < 0) {
        B->loop_cells = save;
        return rc;
      }
      if (hipEventRecord(c0->ev[1], s) != hipSuccess || hipEventSynchronize(c0->ev[1]) != hipSuccess)
        return hip_fail(c0, hipGetLastError(), "event");
      (void)hipEventElapsedTime(&f, c0->ev[0], c0->ev[1]);
    }
    if (ms) ms[k] = f;
    if (f < best) {
      best = f;
      best_lc = B->loop_cells;
    }
  }
  B->loop_cells = best_lc;
  if (pick) *pick = best_lc;
  zero_x();
  return fnlh_batch_relax(B, n_sys, sys, x, bvec, o, nullptr, stream);
}

int fnlh_batch_relax(fnlh_batch B, const int32_t* n_sys, const int32_t* const* sys, double* const* const* x,
                     const double* const* const* bvec, const fnlh_relax_opts* o, fnlh_sys_report* rep, void* stream) {
  if (!B) return FNLH_E_ARG;
  if (!n_sys || !sys || !x || !bvec || !o) return bset_err(B, FNLH_E_ARG, "batch_relax: bad arguments");
  if (o->kind != FNLH_DILU && o->kind != FNLH_SGS && o->kind != FNLH_LEARNED)
    return bset_err(B, FNLH_E_ARG, "batch_relax: kind must be DILU, SGS or LEARNED");
  hipStream_t s = S(stream);
  const int n = (int)B->inst.size();
  std::vector<int> base(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if (n_sys[i] < 1) return bset_err(B, FNLH_E_ARG, "batch_relax: every instance needs >= 1 system");
    base[i + 1] = base[i] + n_sys[i];
  }
  const int total = base[n];
  int rc;
  if ((rc = bdalloc(B, B->st, sizeof(SysState) * total)) || (rc = bdalloc(B, B->sto, sizeof(SysState) * total)))
    return rc;
  if (B->h_cap < (size_t)total) {
    if (B->h_st) (void)hipHostFree(B->h_st);
    B->h_st = nullptr;
    if (hipHostMalloc((void**)&B->h_st, sizeof(SysState) * total, hipHostMallocDefault) != hipSuccess)
      return bset_err(B, FNLH_E_OOM, "batch: host allocation failed");
    B->h_cap = total;
  }
  SysState* dst = (SysState*)B->st.p;
  SysState* dso = (SysState*)B->sto.p;
  const int storage = B->inst[0]->storage;
  const bool reduced = storage != FNLH_F64;
  std::vector<RelaxPlan> plans(n);
  std::vector<SysBatch> sbs(n);
  std::vector<char> batched(n, 0);
  std::vector<InstDesc> desc;
  std::vector<int> di(n, -1);
  // prepare and factor every instance
  for (int i = 0; i < n; ++i) {
    fnlh_ctx c = B->inst[i];
    if ((rc = relax_prepare(c, n_sys[i], sys[i], x[i], bvec[i], o, s, plans[i]))) {
      B->err = c->err;
      return rc;
    }
    if (plans[i].path != kPathRB || plans[i].G < n_sys[i]) continue;  // solved one by one below
    if (B->loop_cells > 0 && c->L.N >= B->loop_cells) continue;      // iterated alone (cache-resident)
    SysBatch& sb = sbs[i];
    sb.n = n_sys[i];
    for (int k = 0; k < sb.n; ++k) {
      sb.orow[k] = sys[i][k];
      sb.vslot[k] = k;
    }
    if ((rc = relax_factor(c, sb, plans[i].fkind, s))) {
      B->err = c->err;
      return rc;
    }
    batched[i] = 1;
    InstDesc D;
    D.p = c->pat();
    D.offd = c->offd.p;
    D.diag = c->diag.p;
    D.dinv = c->dinv.p;
    D.dstride = dinv_stride(c);
    D.ns = n_sys[i];
    D.pivot = plans[i].cfg.pivot ? 1 : 0;
    D.sb = sb;
    D.st = dst + base[i];
    D.partial = (double*)c->partial.p;
    D.c1_t0 = c->L.ctile[1];
    D.c1_nt = c->L.ctile[2] - c->L.ctile[1];
    int SW, P;
    rb_shape(plans[i].cfg, sb.n, SW, P);
    D.slots = SW;
    di[i] = (int)desc.size();
    desc.push_back(D);
  }
  // groups of equal (SW, P); work lists and reduction items
  std::vector<WorkItem> w0, w1, items;
  B->groups.clear();
  {
    std::vector<std::pair<int, int>> keys;
    for (int i = 0; i < n; ++i)
      if (batched[i]) {
        int SW, P;
        rb_shape(plans[i].cfg, sbs[i].n, SW, P);
        if (std::find(keys.begin(), keys.end(), std::make_pair(SW, P)) == keys.end()) keys.emplace_back(SW, P);
      }
    for (auto& kp : keys) {
      BatchGroup g;
      g.SW = kp.first;
      g.P = kp.second;
      g.w0_off = (int64_t)w0.size();
      g.w1_off = (int64_t)w1.size();
      for (int i = 0; i < n; ++i) {
        if (!batched[i]) continue;
        int SW, P;
        rb_shape(plans[i].cfg, sbs[i].n, SW, P);
        if (SW != g.SW || P != g.P) continue;
        const Layout& L = B->inst[i]->L;
        for (int64_t t = L.ctile[0]; t < L.ctile[1]; ++t) w0.push_back(WorkItem{di[i], (int32_t)t});
        for (int64_t t = L.ctile[1]; t < L.ctile[2]; ++t) w1.push_back(WorkItem{di[i], (int32_t)t});
      }
      g.w0_n = (int64_t)w0.size() - g.w0_off;
      g.w1_n = (int64_t)w1.size() - g.w1_off;
      B->groups.push_back(g);
    }
    for (int i = 0; i < n; ++i)
      if (batched[i])
        for (int k = 0; k < sbs[i].n; ++k) items.push_back(WorkItem{di[i], k});
  }
  B->n_items = (int)items.size();
  B->all_w0 = w0;
  B->all_w1 = w1;
  B->all_items = items;
  B->inst_group.assign(desc.size(), 0);
  B->inst_base.assign(desc.size(), 0);
  B->inst_ns.assign(desc.size(), 0);
  for (int i = 0; i < n; ++i) {
    if (!batched[i]) continue;
    int SW, P;
    rb_shape(plans[i].cfg, sbs[i].n, SW, P);
    for (size_t g = 0; g < B->groups.size(); ++g)
      if (B->groups[g].SW == SW && B->groups[g].P == P) B->inst_group[di[i]] = (int)g;
    B->inst_base[di[i]] = base[i];
    B->inst_ns[di[i]] = n_sys[i];
  }
  if (!desc.empty()) {
    if ((rc = bdalloc(B, B->desc, sizeof(InstDesc) * desc.size())) ||
        (rc = bdalloc(B, B->work0, sizeof(WorkItem) * std::max<size_t>(1, w0.size()))) ||
        (rc = bdalloc(B, B->work1, sizeof(WorkItem) * std::max<size_t>(1, w1.size()))) ||
        (rc = bdalloc(B, B->items, sizeof(WorkItem) * std::max<size_t>(1, items.size()))))
      return rc;
    const RelaxPlan& P0 = plans[std::find(batched.begin(), batched.end(), 1) - batched.begin()];
    if (!reduced) {
      for (int i = 0; i < n; ++i) {
        if (!batched[i]) continue;
        fnlh_ctx c = B->inst[i];
        desc[di[i]].x = c->x64.p;
        desc[di[i]].b = c->b64.p;
        outer_residual(c, n_sys[i], sbs[i], nullptr, s);
        launch_reduce(sbs[i], (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, dst + base[i],
                      kReduceInit, 0, 0, o->max_sweeps, s);
      }
      HIPC(nullptr, hipMemcpyAsync(B->desc.p, desc.data(), sizeof(InstDesc) * desc.size(), hipMemcpyHostToDevice, s),
           "upload");
      if (!P0.learned) {
        if ((rc = batched_loop(B, storage, o->rtol, P0.divf, o->max_sweeps, P0.check_every, P0.use_graph, total, s)))
          return rc;
      } else {
        // batched chunks of sweeps, each followed by the learned correction of every
        // instance that still iterates
        for (int done = 0;;) {
          const int chunk = std::max(1, std::min(P0.learn_every, o->max_sweeps + 1 - done));
          if ((rc = batched_loop(B, storage, o->rtol, P0.divf, chunk, P0.check_every, P0.use_graph, total, s, true)))
            return rc;
          done += chunk;
          bool any = false;
          std::vector<char> act(n, 0);
          for (int i = 0; i < n; ++i)
            if (batched[i])
              for (int k = 0; k < n_sys[i]; ++k) act[i] |= B->h_st[base[i] + k].active != 0;
          for (int i = 0; i < n; ++i) any |= act[i] != 0;
          if (!any || done > o->max_sweeps) break;
          for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            fnlh_ctx c = B->inst[i];
            if ((rc = nn_learned_step(c, n_sys[i], sbs[i], (double*)c->x64.p, (const double*)c->b64.p, nullptr,
                                      dst + base[i], s))) {
              B->err = c->err;
              return rc;
            }
          }
        }
      }
    } else {
      for (int i = 0; i < n; ++i) {
        if (!batched[i]) continue;
        fnlh_ctx c = B->inst[i];
        desc[di[i]].x = c->d32.p;
        desc[di[i]].b = c->rhs32.p;
        outer_residual(c, n_sys[i], sbs[i], (double*)c->r64.p, s);
        launch_reduce(sbs[i], (const double*)c->partial.p, c->L.n_tiles, 0, c->L.n_tiles, 1, dso + base[i],
                      kReduceInit, 0, 0, o->max_sweeps, s);
      }
      HIPC(nullptr, hipMemcpyAsync(B->desc.p, desc.data(), sizeof(InstDesc) * desc.size(), hipMemcpyHostToDevice, s),
           "upload");
      for (int it = 0; it < 100000; ++it) {
        if (hipMemcpyAsync(B->h_st, dso, sizeof(SysState) * total, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return bset_err(B, FNLH_E_HIP, "batch: state read-back failed");
        bool any = false;
        for (int i = 0; i < n; ++i)
          if (batched[i])
            for (int k = 0; k < n_sys[i]; ++k) any |= B->h_st[base[i] + k].active != 0;
        if (!any) break;
        for (int i = 0; i < n; ++i)
          if (batched[i]) outer_to_inner(B->inst[i], n_sys[i], sbs[i], dso + base[i], dst + base[i], P0.inner_max, s);
        if ((rc = batched_loop(B, storage, P0.inner_rtol, 1e30, P0.inner_max, P0.check_every, P0.use_graph, total,
                               s)))
          return rc;
        for (int i = 0; i < n; ++i)
          if (batched[i])
            inner_to_outer(B->inst[i], n_sys[i], sbs[i], dst + base[i], dso + base[i], o->rtol, P0.divf, s);
        if (P0.learned)
          for (int i = 0; i < n; ++i) {
            if (!batched[i]) continue;
            fnlh_ctx c = B->inst[i];
            if ((rc = nn_learned_step(c, n_sys[i], sbs[i], (double*)c->x64.p, (const double*)c->b64.p,
                                      (double*)c->r64.p, dso + base[i], s))) {
              B->err = c->err;
              return rc;
            }
          }
      }
    }
  }
  // finish the batched instances
  SysState* fin = reduced ? dso : dst;
  for (int i = 0; i < n; ++i) {
    if (!batched[i]) continue;
    if ((rc = relax_finish_launch(B->inst[i], n_sys[i], sys[i], x[i], fin + base[i], s))) {
      B->err = B->inst[i]->err;
      return rc;
    }
  }
  if (hipMemcpyAsync(B->h_st, fin, sizeof(SysState) * total, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bset_err(B, FNLH_E_HIP, "batch: state read-back failed");
  int worst = FNLH_OK;
  auto fold = [&](int r) {
    if (r < 0) return;
    worst = worse_status(worst, r);
  };
  for (int i = 0; i < n; ++i) {
    if (!batched[i]) continue;
    std::vector<int> counts;
    if (plans[i].learned) {
      counts.assign(2 * n_sys[i], 0);
      if ((rc = nn_relax_counts(B->inst[i], n_sys[i], counts.data(), s))) {
        B->err = B->inst[i]->err;
        return rc;
      }
    }
    fold(relax_reports(B->h_st + base[i], n_sys[i], plans[i], o, rep ? rep + base[i] : nullptr,
                       plans[i].learned ? counts.data() : nullptr, B->inst[i]));
  }
  // the rest one by one
  for (int i = 0; i < n; ++i) {
    if (batched[i]) continue;
    rc = fnlh_relax(B->inst[i], n_sys[i], sys[i], x[i], bvec[i], o, rep ? rep + base[i] : nullptr, stream);
    if (rc < 0) {
      B->err = B->inst[i]->err;
      return rc;
    }
    fold(rc);
  }
  return worst;
}

int fnlh_autotune(fnlh_ctx c, int32_t n_sys, double rtol, int32_t max_sweeps, fnlh_tune_result* out,
                  void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "autotune: matrix and harmonics first");
  if (n_sys < 1 || n_sys > c->n_sys || n_sys > kMaxBatch || max_sweeps < 2 || !(rtol >= 0.0))
    return set_err(c, FNLH_E_ARG, "autotune: need 1 <= n_sys <= min(harmonics, 16), max_sweeps >= 2, rtol >= 0");
  hipStream_t s = S(stream);
  const size_t vb = (size_t)c->L.N * 12 * sizeof(double);
  DevBuf xb, bb;
  struct FreeOnExit {
    DevBuf* a;
    DevBuf* b;
    ~FreeOnExit() {
      dfree(*a);
      dfree(*b);
    }
  } guard{&xb, &bb};
  int rc;
  if ((rc = dalloc(c, xb, vb * n_sys, "autotune alloc")) || (rc = dalloc(c, bb, vb * n_sys, "autotune alloc")))
    return rc;
  std::vector<double> ones(c->L.N * 12, 1.0);
  std::vector<double*> xs(n_sys), bs(n_sys);
  std::vector<int32_t> sys(n_sys);
  for (int j = 0; j < n_sys; ++j) {
    xs[j] = (double*)xb.p + (size_t)j * c->L.N * 12;
    bs[j] = (double*)bb.p + (size_t)j * c->L.N * 12;
    sys[j] = j;
    HIPC(c, hipMemcpyAsync(bs[j], ones.data(), vb, hipMemcpyHostToDevice, s), "autotune rhs");
  }
  // the objective: wall time of a whole solve (factorisation cached after the warm-up,
  // graph-replayed sweeps, FP64 outer corrections) to rtol, or of max_sweeps sweeps
  fnlh_relax_opts o;
  std::memset(&o, 0, sizeof(o));
  o.kind = FNLH_DILU;
  o.max_sweeps = max_sweeps;
  o.rtol = rtol;
  o.check_every = 16;
  o.use_graph = 1;
  if (rtol == 0.0) {
    o.inner_sweeps = max_sweeps;
    o.inner_rtol = 1e-30;
  }
  struct Cand {
    int hybrid, lpr, spw, wg;
  };
  const int save_spw = c->lanes_per_sys, save_lpr = c->lanes_per_row, save_wg = c->wave_groups,
            save_hyb = c->hybrid;
  const bool save_stats = c->stats_on;
  c->stats_on = false;
  std::vector<Cand> cands;
  std::vector<int> paths = {save_hyb};
  if (c->L.n_colours >= 3) paths = {1, 0};
  for (int hy : paths) {
    cands.push_back({hy, 0, 0, 1});
    for (int lpr : {1, 2, 4})
      for (int spw : {1, 2, 4})
        if (lpr <= std::max(1, n_sys)) cands.push_back({hy, lpr, spw, 1});
    cands.push_back({hy, 0, 0, 0});  // a 64-row tile per workgroup
  }
  double best = 1e300, dflt = 0.0;
  int best_sweeps = 0;
  Cand pick = cands[0];
  int tried = 0;
  for (const Cand& cd : cands) {
    c->hybrid = cd.hybrid;
    c->lanes_per_sys = cd.spw;
    c->lanes_per_row = cd.lpr;
    c->wave_groups = cd.wg;
    double ms[2] = {0.0, 0.0};
    int sweeps = 0;
    for (int rep = 0; rep < 3 && rc >= 0; ++rep) {  // a warm-up (factors, graphs), then two timed solves
      launch_fill_zero(xb.p, vb * n_sys, s);
      HIPC(c, hipEventRecord(c->ev[0], s), "event");
      std::vector<fnlh_sys_report> reps(n_sys);
      rc = fnlh_relax(c, n_sys, sys.data(), xs.data(), (const double* const*)bs.data(), &o, reps.data(), stream);
      if (rc < 0) break;
      HIPC(c, hipEventRecord(c->ev[1], s), "event");
      HIPC(c, hipEventSynchronize(c->ev[1]), "event sync");
      float f = 0.f;
      (void)hipEventElapsedTime(&f, c->ev[0], c->ev[1]);
      if (rep > 0) ms[rep - 1] = f;
      sweeps = 0;
      for (const auto& r : reps) sweeps += r.sweeps;
    }
    if (rc < 0) break;
    const double t = std::min(ms[0], ms[1]);
    ++tried;
    if (tried == 1) dflt = t;
    if (t < best) {
      best = t;
      pick = cd;
      best_sweeps = sweeps;
    }
  }
  c->stats_on = save_stats;
  if (rc < 0) {
    c->lanes_per_sys = save_spw;
    c->lanes_per_row = save_lpr;
    c->wave_groups = save_wg;
    c->hybrid = save_hyb;
    return rc;
  }
  c->hybrid = pick.hybrid;
  c->lanes_per_sys = pick.spw;
  c->lanes_per_row = pick.lpr;
  c->wave_groups = pick.wg;
  if (out) {
    out->lanes_per_row = pick.lpr;
    out->sys_per_lane = pick.spw;
    out->wave_groups = pick.wg;
    out->hybrid = pick.hybrid;
    out->ms_best = best;
    out->ms_default = dflt;
    out->sweeps = best_sweeps;
    out->candidates = tried;
  }
  return FNLH_OK;
}

int fnlh_tune(fnlh_ctx c, int32_t param, int32_t value) {
  if (!c) return FNLH_E_ARG;
  if (param == FNLH_TUNE_SYS_PER_LANE) {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return set_err(c, FNLH_E_ARG, "tune: systems per lane must be 0, 1, 2 or 4");
    c->lanes_per_sys = value;
    return FNLH_OK;
  }
  if (param == FNLH_TUNE_LANES_PER_ROW) {
    if (value != 0 && value != 1 && value != 2 && value != 4)
      return set_err(c, FNLH_E_ARG, "tune: lanes per row must be 0, 1, 2 or 4");
    c->lanes_per_row = value;
    return FNLH_OK;
  }
  if (param == FNLH_TUNE_WAVE_GROUPS) {
    if (value != 0 && value != 1) return set_err(c, FNLH_E_ARG, "tune: wave groups must be 0 or 1");
    c->wave_groups = value;
    return FNLH_OK;
  }
  if (param == FNLH_TUNE_HYBRID) {
    if (value < 0 || value > 2) return set_err(c, FNLH_E_ARG, "tune: hybrid must be 0, 1 or 2");
    c->hybrid = value;
    return FNLH_OK;
  }
  if (param == FNLH_TUNE_PILU_THREADS) {
    if (value != 0 && value != 64 && value != 128 && value != 256)
      return set_err(c, FNLH_E_ARG, "tune: sweep workgroup size must be 0, 64, 128 or 256");
    if (value != c->pl_threads) c->buf_gen++;  // captured sweeps hold the launch shape
    c->pl_threads = value;
    return FNLH_OK;
  }
  if (param == FNLH_TUNE_PILU_UNIT) {
    if (value < 0) return set_err(c, FNLH_E_ARG, "tune: cells per work unit must be >= 0");
    if (value != c->pl_unit_rows) {
      c->pl_unit_rows = value;
      c->pl_built = false;  // new units: new tables (the factors follow the positions)
      invalidate_factors(c);
    }
    return FNLH_OK;
  }
  return set_err(c, FNLH_E_ARG, "tune: unknown parameter");
}

int fnlh_stats_enable(fnlh_ctx c, int32_t on) {
  if (!c) return FNLH_E_ARG;
  if (on) {
    for (int k = 0; k < FNLH_KSTAT_N; ++k) {
      c->st_ms[k] = 0.0;
      c->st_bytes[k] = 0.0;
      c->st_n[k] = 0;
    }
  }
  if (on < 0) return set_err(c, FNLH_E_ARG, "stats_enable: period must be >= 0");
  c->stats_on = on != 0;
  c->stats_period = on > 0 ? on : 1;
  return FNLH_OK;
}

int fnlh_stats_get(fnlh_ctx c, int32_t which, fnlh_kernel_stats* out) {
  if (!c || !out || which < 0 || which >= FNLH_KSTAT_N) return set_err(c, FNLH_E_ARG, "stats_get: bad arguments");
  out->launches = c->st_n[which];
  out->total_ms = c->st_ms[which];
  out->alg_bytes = c->st_bytes[which];
  return FNLH_OK;
}

int fnlh_get_ordering(fnlh_ctx c, int32_t* colour_of_cell, int32_t* n_colours) {
  if (!c) return FNLH_E_ARG;
  if (colour_of_cell) std::copy(c->L.colour_user.begin(), c->L.colour_user.end(), colour_of_cell);
  if (n_colours) *n_colours = c->L.n_colours;
  return FNLH_OK;
}

int fnlh_memory(fnlh_ctx c, size_t* matrix_bytes, size_t* factor_bytes, size_t* vector_bytes) {
  if (!c) return FNLH_E_ARG;
  const DevBuf* mat[] = {&c->ent_phase, &c->ent_drop, &c->tile_nrows, &c->tile_width, &c->tile_slot0, &c->ent_nbr, &c->ent_edge, &c->ent_rev,
                         &c->vol, &c->zone, &c->iperm, &c->perm, &c->edge_ent, &c->bf_ptr, &c->bf_idx, &c->area,
                         &c->bface_area, &c->offd, &c->diag, &c->offd64, &c->diag64, &c->state, &c->bstate,
                         &c->corr_row, &c->corr_width, &c->corr_slot0, &c->corr_fe, &c->pl_unit_ptr,
                         &c->pl_unit_lev, &c->pl_lev_ptr, &c->pl_pos_row,
                         &c->pl_gwidth, &c->pl_gslot0, &c->pl_epos, &c->pl_erow, &c->pl_esrc, &c->pl_erev,
                         &c->pl_coup, &c->pl_diag};
  const DevBuf* vec[] = {&c->x64, &c->b64,     &c->r64,     &c->y,  &c->rhs32,   &c->d32,
                         &c->partial, &c->st, &c->st_outer, &c->d_omega, &c->phase_cs, &c->sys_frozen,
                         &c->pl_partial};
  size_t m = 0, v = 0;
  for (auto* b : mat) m += b->bytes;
  for (auto* b : vec) v += b->bytes;
  if (matrix_bytes) *matrix_bytes = m;
  if (factor_bytes) *factor_bytes = c->dinv.bytes;
  if (vector_bytes) *vector_bytes = v;
  return FNLH_OK;
}

}  // extern "C"
