// Launchers of the gfx950 kernels (kernels.hip).  All work is stream-ordered.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fnlh {

constexpr int kMaxBatch = 16;  // systems handled by one launch
// One tile of complex 6x6 factor inverses: FP64 with FP64 blocks (72 * 64 doubles), else
// FP16 entries with a power-of-two scale per row (74 * 64 two-byte elements).
inline int64_t dinv_tile_elems(int storage) { return storage == 0 ? 72 * 64 : 74 * 64; }
inline size_t dinv_elem_bytes(int storage) { return storage == 0 ? 8 : 2; }
inline double dinv_row_bytes(int storage) { return storage == 0 ? 72.0 * 8 : 72.0 * 2 + 4; }
constexpr int kPartialSlots = 4;             // norm partials per (system, tile): one per wave

// Per-system solver state kept on the device so stop decisions need no host round trip.
struct SysState {
  double norm0sq;       // ||r0||^2
  double last_n2;       // latest residual norm^2
  int32_t active;       // still iterating
  int32_t pending;      // met a stop criterion; finish the current sweep, then stop
  int32_t sweeps;       // sweeps done
  int32_t status;       // FNLH_OK / NOT_CONVERGED / DIVERGED
  int32_t limit;        // max sweeps
  int32_t outer_iters;  // FP64 corrections (reduced precision)
  // optional residual history, norm^2 of the iterate after m sweeps at hist[m]
  // (m < hist_len); hist_off: sweeps of the outer solve before this inner one
  // (default: none, so a state built field by field never carries a stale pointer)
  double* hist = nullptr;
  int32_t hist_len = 0;
  int32_t hist_off = 0;
};

struct DevPattern {
  int64_t NP = 0;
  int64_t n_tiles = 0;
  const int32_t* tile_nrows = nullptr;
  const int32_t* tile_width = nullptr;
  const int64_t* tile_slot0 = nullptr;
  const int32_t* ent_nbr = nullptr;
  const int32_t* ent_edge = nullptr;
  const int32_t* ent_rev = nullptr;
  const double* vol = nullptr;
  const int32_t* zone = nullptr;
  const double* omega = nullptr;  // [n_sys][n_zones]
  int32_t n_zones = 1;
  // phase-lagged periodic couplings: per entry 0 or +-1 (null: none), and per system
  // (cos sigma, sin sigma) of its inter-blade phase angle
  const int8_t* ent_phase = nullptr;
  const double* phase_cs = nullptr;  // [n_sys][2]
  // frozen turbulence: per system 1 = the leading 5x5 sub-system only, sixth unknown
  // held at zero (null: no system frozen)
  const uint8_t* sys_frozen = nullptr;
};

struct SysBatch {
  int32_t n = 0;
  int32_t orow[kMaxBatch];   // omega row (system id)
  int32_t dslot[kMaxBatch];  // factor slot
  int32_t vslot[kMaxBatch];  // internal vector / state slot
};

enum Store { kF64 = 0, kF32 = 1, kBF16 = 2 };

// Rusanov geometry + state for assembly and the matrix-free FP64 operator.
struct DevFlow {
  const double* state = nullptr;       // [NP][6] internal order
  const double* area = nullptr;        // [E][3] user edge order
  const int32_t* bf_ptr = nullptr;     // [NP+1]
  const int32_t* bf_idx = nullptr;     // [B]
  const double* bface_area = nullptr;  // [B][3]
  const double* bstate = nullptr;      // [B][6] far field or null
  double diag_scale = 1.0;             // 1 + 1/(eps sigma) (implicit) or 1 (explicit)
  int32_t offdiag = 1;                 // 0 for the explicit scheme (K = P)
  // per entry 1 = coupling between two partitions, left out of the operator (null: none)
  const int8_t* ent_drop = nullptr;
};

// One instance of a batched solve: its pattern, matrix, factors, vectors and states.
struct InstDesc {
  DevPattern p;
  const void* offd = nullptr;
  const void* diag = nullptr;
  const void* dinv = nullptr;
  int64_t dstride = 0;
  void* x = nullptr;        // inner vectors (TV) of the solve, [NP][ns][12]
  const void* b = nullptr;
  int32_t ns = 0;
  int32_t pivot = 1;        // first-colour solve pivots
  SysBatch sb;              // the instance's systems (vslot indexes st and the vectors)
  SysState* st = nullptr;   // states, indexed by vslot
  double* partial = nullptr;
  int64_t c1_t0 = 0, c1_nt = 0;  // second-colour tile range
  int32_t slots = 1;        // norm partial slots per tile
  int32_t pad_ = 0;
};
struct WorkItem {
  int32_t inst;
  int32_t tile;  // tile (work lists) or batch entry (reduction items)
};

struct SweepCfg {
  int storage = kF64;
  int spw = 0;            // systems per lane (1, 2, 4); 0 = automatic
  int lanes_per_row = 0;  // two-colour pass: lanes sharing a row (1, 2, 4); 0 = automatic
  bool pivot = true;      // first-colour solve pivots (false: diagonal blocks are dominant)
  bool wave_groups = false;  // two-colour pass: one wave per workgroup (else a whole tile)
};
int rb_slots(const SweepCfg& c, int n);  // norm partial slots per tile of the two-colour pass
void rb_shape(const SweepCfg& c, int n, int& SW, int& P);  // lanes per row, systems per lane

// assembly / raw blocks
void launch_assemble(int storage, const DevPattern& p, const DevFlow& f, void* offd, void* diag, hipStream_t s);
void launch_set_blocks(int storage, const DevPattern& p, int64_t N, int64_t E, const int32_t* perm,
                       const int64_t* edge_ent, const double* diag_user, const double* offd_user, void* offd,
                       void* diag, hipStream_t s);
void launch_get_blocks(int storage, const DevPattern& p, int64_t N, int64_t E, const int32_t* perm,
                       const int64_t* edge_ent, const void* offd, const void* diag, double* diag_user,
                       double* offd_user, hipStream_t s);

// *flag = 0 if some diagonal block is not strictly diagonally dominant by rows
void launch_check_dominance(int storage, const DevPattern& p, const void* diag, int* flag, hipStream_t s);

// factorisation of one colour (tiles [t0, t0+nt), rows below cstart are lower)
void launch_factor(int storage, bool dilu, const DevPattern& p, const void* offd, const void* diag, void* dinv,
                   int64_t dinv_stride, const SysBatch& sb, int64_t t0, int64_t nt, int64_t cstart, int* err,
                   hipStream_t s);

// sweeps; TV = double for F64 storage, float otherwise
// Vectors: internal layout [NP][ns][12], ns = systems of the solve, slot = vslot.
// The reduction of an update pass's norms folded into the first-colour pass that follows
// (same stop logic as launch_reduce with mode kReduceSweep / kReduceSweepNoNorm).
struct FusedReduce {
  int n = 0;  // systems of sb to reduce (0: none)
  int slots = 0;
  int mode = 0;
  int64_t t0 = 0, nt = 0;  // the update pass's tile range
  double rtol2 = 0.0, div2 = 0.0;
};
void launch_rb_pass(const SweepCfg& c, bool update, const DevPattern& p, const void* offd, const void* diag,
                    const void* dinv, int64_t dinv_stride, void* x, const void* b, int ns, const SysBatch& sb,
                    const SysState* st, double* partial, int64_t t0, int64_t nt, hipStream_t s,
                    const FusedReduce* fused = nullptr);
// General-colouring passes (k_fwd / k_bwd).  Forward modes: kFwdGeneral / kFwdLast (the
// textbook forward substitution with the lower colours' y, x += y on the last colour),
// kFwdHybrid (x updated in place colour by colour, y = Dt^-1 (b - K x), x += y),
// kFwdNorm (norm partials of b - K x only).  Backward modes: kBwdGeneral, kBwdHybrid
// (x and y += -Dt^-1 sum_upper K z).
enum { kFwdGeneral = 0, kFwdLast = 1, kFwdHybrid = 2, kFwdNorm = 3 };
enum { kBwdGeneral = 0, kBwdHybrid = 1 };
void launch_fwd(const SweepCfg& c, int mode, const DevPattern& p, const void* offd, const void* diag,
                const void* dinv, int64_t dinv_stride, void* x, const void* b, void* y, int ns, const SysBatch& sb,
                const SysState* st, double* partial, int64_t t0, int64_t nt, int64_t cstart, hipStream_t s);
void launch_bwd(const SweepCfg& c, int mode, const DevPattern& p, const void* offd, const void* dinv,
                int64_t dinv_stride, void* x, void* y, int ns, const SysBatch& sb, const SysState* st, int64_t t0,
                int64_t nt, int64_t cend, hipStream_t s);
// The second-colour rows coupled to higher colours (two colours plus remainder), packed
// 64 to a group with their upward couplings: row[g * 64 + lane] (internal row, -1
// padding), width[g], slot0[g], fe[(slot0[g] + k) * 64 + lane] (flat SELL entry, -1
// padding, in slot order).
struct CorrDev {
  const int32_t* row = nullptr;
  const int32_t* width = nullptr;
  const int64_t* slot0 = nullptr;
  const int32_t* fe = nullptr;
  int64_t n_groups = 0;
};
// x_i += -Dt_i^-1 sum_{k upper} K_ik y_k for those rows (systems not pending)
void launch_correct(int storage, const DevPattern& p, const CorrDev& q, const void* offd, const void* dinv,
                    int64_t dinv_stride, void* x, const void* y, int ns, const SysBatch& sb, const SysState* st,
                    hipStream_t s);
void launch_jacobi(const SweepCfg& c, const DevPattern& p, const void* offd, const void* diag, const void* dinv,
                   int64_t dinv_stride, const void* x, const void* b, void* y, int ns, const SysBatch& sb,
                   const SysState* st, double* partial, hipStream_t s);
void launch_axpy_y(int storage, const DevPattern& p, void* x, const void* y, int ns, const SysBatch& sb,
                   const SysState* st, hipStream_t s);

// Partition-local natural-order ILU(0) (layout.h, PiluLayout): device copies of the
// work-unit, level, position and packed-coupling tables.  Norm partials of system slot
// vs, unit k at partial[vs * pt * kPartialSlots + k] (pt = ceil(n_units / kPartialSlots);
// the entries past n_units stay zero), so launch_reduce sums them with n_tiles = nt = pt
// and slots = kPartialSlots.
struct PiluDev {
  const int32_t* unit_ptr = nullptr;
  const int32_t* unit_lev = nullptr;
  const int32_t* lev_ptr = nullptr;
  const int32_t* pos_row = nullptr;
  const int32_t* g_width = nullptr;
  const int64_t* g_slot0 = nullptr;
  const int32_t* e_pos = nullptr;
  const int32_t* e_row = nullptr;
  const int32_t* e_src = nullptr;
  const int32_t* e_rev = nullptr;
  int64_t n_units = 0, n_groups = 0, n_slots = 0, pt = 0;
  int32_t max_rows = 0;
  int32_t threads = 256;  // sweep workgroup size (pilu_threads)
};
// copy the in-partition couplings and the diagonal blocks into the position layout
void launch_pilu_pack(int storage, const PiluDev& q, const void* offd, const void* diag, void* coup, void* pdiag,
                      hipStream_t s);
// Dt^-1 of every position for the systems of sb (slot dslot, group-major tiles)
void launch_pilu_factor(int storage, const DevPattern& p, const PiluDev& q, const void* coup, const void* pdiag,
                        void* dinv, int64_t dinv_stride, const SysBatch& sb, int* err, hipStream_t s);
// LDS bytes per unit row and system of the sweep (the y vector held there)
int pilu_lds_row_bytes(int storage);
// systems per workgroup of the sweep for nb systems within lds_max bytes (0: a unit does
// not fit)
int pilu_systems_per_group(int storage, int nb, int max_rows, int lds_max);
// allow the sweep kernels of this storage lds bytes of dynamic LDS (above the 64 KiB
// default); false if the runtime refuses
bool pilu_allow_lds(int storage, int lds);
// sweep workgroup size for units whose levels hold avg_width rows on average (four
// lanes per row): 64, 128 or 256
int pilu_threads(int avg_width);
// one sweep x <- x + M^-1 (b - K x) for every unit and system of sb, norms of
// b - K x (before the update) into the partials; systems pending or inactive are skipped
void launch_pilu_sweep(int storage, const DevPattern& p, const PiluDev& q, const void* coup, const void* pdiag,
                       const void* dinv, int64_t dinv_stride, void* x, const void* b, int ns, const SysBatch& sb,
                       const SysState* st, double* partial, int lds_max, hipStream_t s);

// batched two-colour pass over a work list (instances grouped so SW, P are uniform)
// Batched two-colour pass over the (instance, tile) work list of one shape group.
// wave_groups: one wave per workgroup.  red (first-colour pass only): the reduction items
// (instance, system) of the preceding update pass, done by the first n_red workgroups
// (mode kReduceSweep / kReduceSweepNoNorm, squared tolerances).
void launch_rb_batched(int storage, int SW, int P, bool update, const InstDesc* inst, const WorkItem* work,
                       int64_t n_work, hipStream_t s, bool wave_groups = false, const WorkItem* red = nullptr,
                       int n_red = 0, int red_mode = 0, double rtol = 0.0, double div_factor = 0.0);
void launch_reduce_batched(const InstDesc* inst, const WorkItem* items, int n_items, int mode, double rtol,
                           double div_factor, hipStream_t s);

// residual norms -> state.  modes: 0 init (limit = max_sweeps), 1 sweep with a valid
// norm, 2 sweep without a norm, 3 final (record only), 4 outer FP64 correction test
enum { kReduceInit = 0, kReduceSweep = 1, kReduceSweepNoNorm = 2, kReduceFinal = 3, kReduceOuter = 4 };
void launch_reduce(const SysBatch& sb, const double* partial, int64_t n_tiles, int64_t t0, int64_t nt, int slots,
                   SysState* st, int mode, double rtol, double div_factor, int max_sweeps, hipStream_t s);

// FP64 residual r = b - K_s x.  stored: blocks of the given storage upcast; mfree: Rusanov
// recomputed from the FP64 state.  r may be null.
void launch_resid_stored(int storage, const DevPattern& p, const void* offd, const void* diag, const double* x,
                         const double* b, double* r, int ns, const SysBatch& sb, double* partial, hipStream_t s);
void launch_resid_mfree(const DevPattern& p, const DevFlow& f, const double* x, const double* b, double* r, int ns,
                        const SysBatch& sb, double* partial, hipStream_t s);

// vectors: user [N][width] of one system <-> internal [NP][ns][width] slot vs
void launch_to_internal(const DevPattern& p, const int32_t* iperm, const double* user, double* internal, int width,
                        int ns, int vs, hipStream_t s);
void launch_to_user(const DevPattern& p, const int32_t* iperm, const double* internal, double* user, int width,
                    int ns, int vs, hipStream_t s);
// n systems' complex vectors (user [N][6], host array of device pointers) <-> internal
// slots vs0 .. vs0 + n - 1, in launches of up to kMaxBatch systems
struct VecPtrs {
  const double* p[kMaxBatch];
};
struct VecPtrsOut {
  double* p[kMaxBatch];
};
void launch_to_internal_n(const DevPattern& p, const int32_t* iperm, const double* const* users, int n,
                          double* internal, int ns, int vs0, hipStream_t s);
void launch_to_user_n(const DevPattern& p, const int32_t* iperm, const double* internal, double* const* users, int n,
                      int ns, int vs0, hipStream_t s);
void launch_to_f32(const DevPattern& p, const double* r64, float* rhs32, float* d32, int ns, const SysBatch& sb,
                   const SysState* outer, hipStream_t s);
void launch_add_f32(const DevPattern& p, double* x64, const float* d32, int ns, const SysBatch& sb,
                    const SysState* outer, hipStream_t s);
void launch_inner_init(const SysBatch& sb, const SysState* outer, SysState* inner, int max_sweeps, hipStream_t s);
void launch_outer_update(const SysBatch& sb, const SysState* inner, SysState* outer, hipStream_t s);
// zero the stored off-diagonal blocks of the entries flagged in ent_drop (flat entries)
void launch_drop_blocks(int storage, const DevPattern& p, int64_t n_slots, const int8_t* ent_drop, void* offd,
                        hipStream_t s);
// zero the sixth unknown of slot vs of an interleaved complex vector [rows][ns][6]
// (frozen-turbulence systems)
void launch_zero_sixth(int64_t rows, double* v, int ns, int vs, hipStream_t s);
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// attach a residual history of len entries per system slot to the states of sb
// (hist + vslot * len; null detaches) and record the initial norm^2 at entry 0
void launch_set_history(const SysBatch& sb, SysState* st, double* hist, int len, hipStream_t s);

// ---- restarted flexible GMRES vector kernels (krylov.hip); vectors [NP][ns][12] FP64
constexpr int kMdot = 8;          // basis vectors per inner-product launch
constexpr int kMdotBlocks = 1024;  // workgroups of an inner-product launch (partials per product)
struct KScale {
  double s[kMaxBatch];
};
int mdot_blocks(int64_t NP);
// out[(i * sb.n + kk) * 2 + {re, im}] = (V_i, w) = sum conj(V_i) w over the valid rows, i < nv,
// for system kk of sb; partial: mdot_blocks(NP) * nq * 2 doubles with nq >= nv * sb.n
void launch_mdot(const DevPattern& p, int ns, const double* V, int64_t vstride, int nv, const double* w,
                 const SysBatch& sb, int nq, double* partial, double* out, hipStream_t s);
// w += sgn * sum_{i < nv} coef[i * sb.n + kk] V_i  (complex coef)
void launch_maxpy(const DevPattern& p, int ns, double* w, const double* V, int64_t vstride, int nv,
                  const double* coef, double sgn, const SysBatch& sb, hipStream_t s);
// dst = sc.s[kk] * src for system kk of sb
void launch_mscale(const DevPattern& p, int ns, double* dst, const double* src, const KScale& sc, const SysBatch& sb,
                   hipStream_t s);
// sweep states of sb: active, ||r0||^2 = n2, limit sweeps
void launch_kstate(const SysBatch& sb, SysState* st, double n2, int limit, hipStream_t s);

// RK driver: Rusanov residual of f.state (internal [NP][6]) into user order R [N][6]
// (part[tile]: sum |R|^2); stage helpers on user-order vectors of n reals
void launch_rusanov_residual(const DevPattern& p, const DevFlow& f, const int32_t* iperm, double* R_user,
                             double* part, hipStream_t s);
void launch_rk_rhs_real(int64_t n, const double* R, double scale, double* b, hipStream_t s);
void launch_rk_update(bool complex_state, int64_t n, const double* q0, const double* x, double* q, hipStream_t s);
void launch_scale(int64_t n, double* y, double scale, hipStream_t s);

}  // namespace fnlh
