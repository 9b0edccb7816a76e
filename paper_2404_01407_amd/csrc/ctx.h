// Private host-side state of a context, shared by the C ABI (api.cpp) and the learned
// preconditioner (nn.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/fnlh.h"
#include "kernels.h"
#include "layout.h"

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GraphEntry;
struct fnlh_nn_s;

using fnlh::DevPattern;
using fnlh::Layout;
using fnlh::SysState;
using fnlh::DevFlow;

struct fnlh_ctx_s {
  Layout L;
  int dev = 0;
  int storage = FNLH_F64;
  int outer = FNLH_OUTER_EXACT;
  int factor_slots_opt = 0;
  int lanes_per_sys = 0;  // systems per lane of the sweep kernels (0 = automatic)
  int lanes_per_row = 0;  // lanes sharing a row in the two-colour pass (0 = automatic)
  int wave_groups = 1;    // two-colour pass: 1 = one wave per workgroup (default), 0 = a tile per workgroup
  int hybrid = 1;         // colourings with a small remainder past two colours: two-colour passes + remainder
  // second-colour rows coupled to a higher colour, packed for the correction (CorrDev)
  DevBuf corr_row, corr_width, corr_slot0, corr_fe;
  int64_t hyb_groups = 0, hyb_rows = 0, hyb_ents = 0;
  std::string err;

  // pattern (device)
  DevBuf tile_nrows, tile_width, tile_slot0, ent_nbr, ent_edge, ent_rev, vol, zone, iperm, perm, edge_ent, bf_ptr,
      bf_idx, area, bface_area;
  // matrix
  DevBuf offd, diag, offd64, diag64;  // *64: FP64 shadow of raw blocks in reduced precision
  DevBuf state, bstate;
  bool have_matrix = false, assembled = false, have_shadow = false;
  double eps = 0.6, sigma = 50.0;
  int scheme = FNLH_IMPLICIT;
  // systems
  int n_sys = 0;
  std::vector<double> omega;
  DevBuf d_omega;
  // phase-lagged periodic couplings: per-entry sign, per-system phase (cos, sin)
  DevBuf ent_phase, phase_cs;
  std::vector<double> ibpa;  // inter-blade phase angle per system
  std::vector<int8_t> edge_phase_host;  // the signs behind ent_phase (repeat calls skip the rebuild)
  // frozen turbulence: per system 1 = its sixth unknown is held at zero (null: none)
  DevBuf sys_frozen;
  std::vector<uint8_t> frozen;
  // partition-dropped couplings: per entry 1 = between two partitions (null: none), and
  // the partition of each user cell behind it
  DevBuf ent_drop;
  std::vector<int32_t> part_host;
  // partition-local natural-order ILU(0) (FNLH_PILU): the position layout of the
  // partitions above, its device tables, the blocks packed in position order (stale
  // after new blocks), norm partials for pl_cap systems, and the LDS a workgroup may use
  fnlh::PiluLayout pl;
  bool pl_built = false, pl_packed = false;
  int pl_cap = 0;
  int pl_lds_max = 65536 - 1024;  // dynamic LDS of a sweep workgroup; raised to the device's at first use
  int pl_unit_rows = 0;     // cells per work unit (0: automatic)
  int pl_threads = 0;       // sweep workgroup size (0: automatic)
  DevBuf pl_unit_ptr, pl_unit_lev, pl_lev_ptr, pl_pos_row, pl_gwidth, pl_gslot0, pl_epos, pl_erow, pl_esrc, pl_erev,
      pl_coup, pl_diag, pl_partial;
  // factors
  int n_slots = 0;
  DevBuf dinv;
  std::vector<int> slot_sys, slot_kind;
  // scratch
  int vec_cap = 0;
  DevBuf x64, b64, r64, y, rhs32, d32, partial, st, st_outer;
  SysState* h_st = nullptr;
  DevBuf d_err;
  int* h_err = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // diagonal blocks strictly diagonally dominant (first-colour solve without pivoting)
  bool dom_known = false, dom = false;
  DevBuf d_dom;
  int* h_dom = nullptr;
  // captured sweep graphs; their kernel nodes hold device pointers (factors, omega,
  // partial sums, vectors), so every (re)allocation bumps buf_gen and graphs captured
  // under an older generation are discarded
  uint64_t buf_gen = 0;
  hipStream_t cap = nullptr;
  std::vector<GraphEntry*> graphs;
  bool graph_broken = false;
  // learned preconditioner attached to this context (nn.cpp)
  fnlh_nn_s* nn = nullptr;
  // kernel statistics
  bool stats_on = false;
  int stats_period = 1;  // time the launches of every stats_period-th sweep
  std::vector<hipEvent_t> evpool;
  double st_ms[FNLH_KSTAT_N] = {0};
  double st_bytes[FNLH_KSTAT_N] = {0};
  int64_t st_n[FNLH_KSTAT_N] = {0};

  bool is_frozen(int s) const { return !frozen.empty() && frozen[(size_t)s] != 0; }
  DevPattern pat() const {
    DevPattern p;
    p.NP = L.NP;
    p.n_tiles = L.n_tiles;
    p.tile_nrows = (const int32_t*)tile_nrows.p;
    p.tile_width = (const int32_t*)tile_width.p;
    p.tile_slot0 = (const int64_t*)tile_slot0.p;
    p.ent_nbr = (const int32_t*)ent_nbr.p;
    p.ent_edge = (const int32_t*)ent_edge.p;
    p.ent_rev = (const int32_t*)ent_rev.p;
    p.vol = (const double*)vol.p;
    p.zone = (const int32_t*)zone.p;
    p.omega = (const double*)d_omega.p;
    p.n_zones = L.n_zones;
    p.ent_phase = (const int8_t*)ent_phase.p;
    p.phase_cs = (const double*)phase_cs.p;
    p.sys_frozen = (const uint8_t*)sys_frozen.p;
    return p;
  }
  fnlh::CorrDev corr() const {
    fnlh::CorrDev q;
    q.row = (const int32_t*)corr_row.p;
    q.width = (const int32_t*)corr_width.p;
    q.slot0 = (const int64_t*)corr_slot0.p;
    q.fe = (const int32_t*)corr_fe.p;
    q.n_groups = hyb_groups;
    return q;
  }
  fnlh::PiluDev pilu() const {
    fnlh::PiluDev q;
    q.unit_ptr = (const int32_t*)pl_unit_ptr.p;
    q.unit_lev = (const int32_t*)pl_unit_lev.p;
    q.lev_ptr = (const int32_t*)pl_lev_ptr.p;
    q.pos_row = (const int32_t*)pl_pos_row.p;
    q.g_width = (const int32_t*)pl_gwidth.p;
    q.g_slot0 = (const int64_t*)pl_gslot0.p;
    q.e_pos = (const int32_t*)pl_epos.p;
    q.e_row = (const int32_t*)pl_erow.p;
    q.e_src = (const int32_t*)pl_esrc.p;
    q.e_rev = (const int32_t*)pl_erev.p;
    q.n_units = pl.n_units;
    q.n_groups = pl.n_groups;
    q.n_slots = pl.n_slots;
    q.pt = (pl.n_units + fnlh::kPartialSlots - 1) / fnlh::kPartialSlots;
    q.max_rows = pl.max_rows;
    const int64_t levels = pl.lev_ptr.empty() ? 1 : (int64_t)pl.lev_ptr.size() - 1;
    q.threads = pl_threads > 0 ? pl_threads
                               : fnlh::pilu_threads((int)((pl.n_groups * 64 + levels - 1) / std::max<int64_t>(levels, 1)));
    return q;
  }
  DevFlow flow() const {
    DevFlow f;
    f.state = (const double*)state.p;
    f.area = (const double*)area.p;
    f.bf_ptr = (const int32_t*)bf_ptr.p;
    f.bf_idx = (const int32_t*)bf_idx.p;
    f.bface_area = (const double*)bface_area.p;
    f.bstate = (const double*)bstate.p;
    f.diag_scale = scheme == FNLH_IMPLICIT ? 1.0 + 1.0 / (eps * sigma) : 1.0;
    f.offdiag = scheme == FNLH_IMPLICIT ? 1 : 0;
    f.ent_drop = (const int8_t*)ent_drop.p;
    return f;
  }
  size_t block_bytes() const { return storage == FNLH_F64 ? 8 : storage == FNLH_F32 ? 4 : 2; }
  int64_t slot_elems_storage() const {
    return storage == FNLH_F64 ? 18 * 64 * 2 : storage == FNLH_F32 ? 9 * 64 * 4 : 5 * 64 * 8;
  }
  size_t tv_bytes() const { return storage == FNLH_F64 ? 8 : 4; }
};

namespace fnlh {

// helpers of the ABI layer (api.cpp)
int set_err(fnlh_ctx c, int code, const std::string& m);
int hip_fail(fnlh_ctx c, hipError_t e, const char* what);
int dalloc(fnlh_ctx c, DevBuf& b, size_t bytes, const char* what);
void dfree(DevBuf& b);
int check_launch(fnlh_ctx c, const char* what);
// outer FP64 operator residual of the systems of sb (x, b internal -> r, c->partial)
// (per-tile norm partials into part, c->partial when null)
void outer_residual_of(fnlh_ctx c, int ns, const SysBatch& sb, const double* x, const double* b, double* r,
                       hipStream_t s, double* part = nullptr);
// The no-allocation residual (noalloc.hip): device address of its scratch array on the
// context's device, looked up once per device at context creation; the scratch bytes a
// mesh needs.
int noalloc_init(fnlh_ctx c);
size_t noalloc_residual_bytes(const Layout& L, bool with_r);

// Learned preconditioner inside fnlh_relax (nn.cpp).  nn_relax_begin checks that a
// network with weights is attached, sizes its scratch for ns systems and clears the
// per-system step counters.  nn_learned_step corrects the systems of sb that are still
// active in st: x <- x + alpha dx, r <- r - alpha K dx, with dx the network's output for
// the FP64 residual r (computed from x and b into scratch when r is null) and alpha the
// complex step minimising ||r - alpha K dx||; a step that is not finite or lowers
// ||r||^2 by less than the acceptance fraction is rejected (x, r unchanged).
// nn_relax_counts copies [ns][2] (accepted, rejected) to the host.
int nn_relax_begin(fnlh_ctx c, int ns, hipStream_t s);
int nn_learned_step(fnlh_ctx c, int ns, const SysBatch& sb, double* x, const double* b, double* r,
                    const SysState* st, hipStream_t s);
int nn_relax_counts(fnlh_ctx c, int ns, int* host_counts, hipStream_t s);
// true when system slot vs had its learned corrections switched off in this call
// (rejected three times in a row): the plain sweeps carried it on
bool nn_system_off(fnlh_ctx c, int vs);
// the learned step's residual scratch, [NP][ns][12] FP64: where nn_learned_step is
// called with r null it computes b - K x there, and either way it leaves b - K x of the
// corrected x in the r it was given
double* nn_step_residual(fnlh_ctx c);
void nn_release(fnlh_ctx c);  // context destroyed: detach its network

// Preconditioner access for the Krylov solve (api.cpp).  precond_prepare does what
// fnlh_relax does before its sweeps (validation, x and b into the internal vectors x64
// and b64 as slots 0..n-1, the frozen systems' sixth unknown zeroed, factors of all n
// systems, the sweep path) for preconditioner `kind`; precond_apply sets z = M^-1 v for
// the systems of sb, M^-1 being `inner` preconditioned Richardson sweeps from z = 0 (one
// sweep is exactly the DILU, SGS or Jacobi M^-1), in the storage precision (FP32/BF16
// sweeps on the rounded v for reduced storage); v and z internal [NP][ns][12] FP64.
// FNLH_LEARNED: z = alpha d from one learned step at z = 0 (nn_learned_step), then the
// DILU sweeps on the remaining residual v - K z, added to z.
struct PrecondPlan {
  int path = 0, fkind = 0, inner = 1;
  bool reduced = false, use_graph = false, learned = false;
  SweepCfg cfg;
};
int precond_prepare(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b, int kind,
                    int inner, bool use_graph, hipStream_t s, PrecondPlan& out);
int precond_apply(fnlh_ctx c, const PrecondPlan& pp, int ns, const SysBatch& sb, const double* v, double* z,
                  hipStream_t s);

}  // namespace fnlh

#define HIPC(c, expr, what)                              \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_fail(c, _e, what);  \
  } while (0)
