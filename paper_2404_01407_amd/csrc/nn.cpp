// C ABI of the learned preconditioner (include/fnlh.h, "learned preconditioner") and
// its use inside fnlh_relax.  The network, its FP32 master weights, Adam moments and the
// training pairs live on the device; every step (features, forward, backward, gradient
// reduction, Adam, the corrected update) is a kernel of nn.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "nn.h"

using namespace fnlh;

struct fnlh_nn_s {
  fnlh_ctx c = nullptr;
  DevBuf master, mom1, mom2, grad, wt, w;  // FP32 master/moments/gradient [kNnParams], bf16 padded weights
  DevBuf u, h, d, sc, part;                // inference
  DevBuf ehat, dc, dh, gpart, lpart, loss;  // training
  DevBuf pool;                             // pairs: [cap][2][NP][12] BF16 (r, e), internal order
  std::vector<int32_t> pair_sys;
  int64_t n_pairs = 0, cap_pairs = 0;
  DevBuf rr, xt, rn, part4, alpha, counts;  // learned step scratch
  int step_cap = 0;
  int G = 0;
  int adam_t = 0;
  int hidden = 64;
  bool weights_set = false;
  // per call of relax / gmres: counts seen after the last step, rejections in a row,
  // and the systems whose corrections are switched off for the rest of the call
  std::vector<int> prev_acc, prev_rej, consec, off;
  std::vector<int> hcounts;
};

namespace {

constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;
constexpr double kAccept = 1e-3;  // minimum fractional drop of ||r||^2 for a learned step
constexpr int kMaxG = 512;        // workgroups of the backward kernels (gradient partials)
constexpr int kOffAfter = 3;      // rejected learned corrections in a row that switch a system's off
constexpr char kMagic[8] = {'F', 'N', 'L', 'H', 'N', 'N', '0', '1'};  // checkpoint file tag

inline hipStream_t S(void* s) { return (hipStream_t)s; }

int nn_err(fnlh_nn nn, int code, const char* m) { return nn->c ? set_err(nn->c, code, m) : code; }

NnBufs bufs(fnlh_nn nn) {
  NnBufs B;
  B.wt = (const uint16_t*)nn->wt.p;
  B.w = (const uint16_t*)nn->w.p;
  B.u = (uint16_t*)nn->u.p;
  B.h = (uint16_t*)nn->h.p;
  B.d = (float*)nn->d.p;
  B.ehat = (float*)nn->ehat.p;
  B.dc = (float*)nn->dc.p;
  B.dh = (float*)nn->dh.p;
  B.part = (double*)nn->part.p;
  B.sc = (NnScalars*)nn->sc.p;
  B.gpart = (float*)nn->gpart.p;
  B.lpart = (double*)nn->lpart.p;
  return B;
}

void free_all(fnlh_nn nn) {
  DevBuf* b[] = {&nn->master, &nn->mom1, &nn->mom2, &nn->grad, &nn->wt, &nn->w, &nn->u, &nn->h, &nn->d,
                 &nn->sc, &nn->part, &nn->ehat, &nn->dc, &nn->dh, &nn->gpart, &nn->lpart, &nn->loss,
                 &nn->pool, &nn->rr, &nn->xt, &nn->rn, &nn->part4, &nn->alpha, &nn->counts};
  for (DevBuf* x : b) dfree(*x);
  nn->n_pairs = nn->cap_pairs = 0;
  nn->pair_sys.clear();
  nn->step_cap = 0;
}

int ready(fnlh_nn nn) {
  if (!nn) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "network: matrix and harmonics first");
  if (!nn->weights_set) return set_err(c, FNLH_E_ORDER, "network: weights not set");
  return FNLH_OK;
}

int ensure_train(fnlh_nn nn) {
  fnlh_ctx c = nn->c;
  int rc;
  if (!nn->ehat.p) {
    const size_t NP = (size_t)c->L.NP;
    if ((rc = dalloc(c, nn->ehat, NP * 16 * sizeof(float), "alloc network"))) return rc;
    if ((rc = dalloc(c, nn->dc, NP * 64 * sizeof(float), "alloc network"))) return rc;
    if ((rc = dalloc(c, nn->dh, NP * 64 * sizeof(float), "alloc network"))) return rc;
    HIPC(c, hipMemset(nn->ehat.p, 0, nn->ehat.bytes), "zero");
  }
  // gradient partials: one row per backward workgroup (their count G may be changed)
  if (nn->gpart.bytes != (size_t)nn->G * kNnPadded * sizeof(float)) {
    dfree(nn->gpart);
    dfree(nn->lpart);
    if ((rc = dalloc(c, nn->gpart, (size_t)nn->G * kNnPadded * sizeof(float), "alloc network"))) return rc;
    if ((rc = dalloc(c, nn->lpart, (size_t)nn->G * sizeof(double), "alloc network"))) return rc;
  }
  return FNLH_OK;
}

int auto_groups(fnlh_ctx c) { return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxG, c->L.n_tiles)); }

// features + forward of one residual (and the training target when e is given)
void features(fnlh_nn nn, int sys, const NnVec& r, const NnVec* e, hipStream_t s) {
  fnlh_ctx c = nn->c;
  NnBufs B = bufs(nn);
  if (!e) B.ehat = nullptr;
  nn_launch_features(c->storage, c->pat(), c->diag.p, sys, r, e, c->L.N, B, true, s);
}

NnVec user_vec(fnlh_ctx c, const double* v) {
  NnVec x;
  x.d64 = v;
  x.iperm = (const int32_t*)c->iperm.p;
  return x;
}

// gradient of the batch-mean loss of n samples into nn->grad (device) and the loss
// into *loss_dev; samples given by a callback filling (sys, r, e)
template <typename F> int batch_grad(fnlh_nn nn, int n, F sample, double* loss_dev, hipStream_t s) {
  fnlh_ctx c = nn->c;
  int rc;
  if ((rc = ensure_train(nn))) return rc;
  launch_fill_zero(nn->gpart.p, nn->gpart.bytes, s);
  launch_fill_zero(nn->lpart.p, nn->lpart.bytes, s);
  const DevPattern p = c->pat();
  const NnBufs B = bufs(nn);
  for (int k = 0; k < n; ++k) {
    int sys = 0;
    NnVec r, e;
    sample(k, sys, r, e);
    features(nn, sys, r, &e, s);
    nn_launch_forward_l1(c->storage, p, c->offd.p, B, s);
    nn_launch_backward(c->storage, p, c->offd.p, B, nn->G, 1.0 / n, s);
  }
  nn_launch_grad_reduce(B, nn->G, (float*)nn->grad.p, loss_dev, s);
  return check_launch(c, "network gradient launch");
}

// pair pool to cap pairs, keeping the stored ones
int grow_pairs(fnlh_nn nn, int64_t cap, hipStream_t s) {
  fnlh_ctx c = nn->c;
  const size_t bytes = (size_t)2 * c->L.NP * 12 * sizeof(uint16_t);
  DevBuf nb;
  int rc = dalloc(c, nb, (size_t)cap * bytes, "alloc training pairs");
  if (rc) return rc;
  if (nn->n_pairs)
    HIPC(c, hipMemcpyAsync(nb.p, nn->pool.p, (size_t)nn->n_pairs * bytes, hipMemcpyDeviceToDevice, s), "grow pairs");
  HIPC(c, hipStreamSynchronize(s), "grow pairs");
  dfree(nn->pool);
  nn->pool = nb;
  nn->cap_pairs = cap;
  return FNLH_OK;
}

}  // namespace

namespace fnlh {

void nn_release(fnlh_ctx c) {
  if (!c || !c->nn) return;
  free_all(c->nn);
  c->nn->c = nullptr;
  c->nn = nullptr;
}

int nn_relax_begin(fnlh_ctx c, int ns, hipStream_t s) {
  fnlh_nn nn = c->nn;
  if (!nn) return set_err(c, FNLH_E_ORDER, "relax: FNLH_LEARNED needs a network (fnlh_nn_create)");
  int rc = ready(nn);
  if (rc) return rc;
  if (ns > nn->step_cap) {
    const size_t v = (size_t)ns * c->L.NP * 12 * sizeof(double);
    if ((rc = dalloc(c, nn->rr, v, "alloc learned step"))) return rc;
    if ((rc = dalloc(c, nn->xt, v, "alloc learned step"))) return rc;
    if ((rc = dalloc(c, nn->rn, v, "alloc learned step"))) return rc;
    if ((rc = dalloc(c, nn->alpha, (size_t)ns * 2 * sizeof(double), "alloc learned step"))) return rc;
    if ((rc = dalloc(c, nn->counts, (size_t)ns * 2 * sizeof(int), "alloc learned step"))) return rc;
    HIPC(c, hipMemset(nn->rr.p, 0, v), "zero");
    HIPC(c, hipMemset(nn->xt.p, 0, v), "zero");
    HIPC(c, hipMemset(nn->rn.p, 0, v), "zero");
    nn->step_cap = ns;
  }
  if (!nn->part4.p && (rc = dalloc(c, nn->part4, (size_t)c->L.n_tiles * 4 * sizeof(double), "alloc learned step")))
    return rc;
  launch_fill_zero(nn->counts.p, (size_t)ns * 2 * sizeof(int), s);
  nn->prev_acc.assign(ns, 0);
  nn->prev_rej.assign(ns, 0);
  nn->consec.assign(ns, 0);
  nn->off.assign(ns, 0);
  nn->hcounts.assign(2 * ns, 0);
  return check_launch(c, "learned step setup");
}

bool nn_system_off(fnlh_ctx c, int vs) {
  fnlh_nn nn = c->nn;
  return nn && vs >= 0 && vs < (int)nn->off.size() && nn->off[vs] != 0;
}

int nn_learned_step(fnlh_ctx c, int ns, const SysBatch& sb0, double* x, const double* b, double* r,
                    const SysState* st, hipStream_t s) {
  fnlh_nn nn = c->nn;
  const DevPattern p = c->pat();
  if ((int)nn->off.size() < ns) {  // first step of a call that did not clear the controller
    nn->prev_acc.resize(ns, 0);
    nn->prev_rej.resize(ns, 0);
    nn->consec.resize(ns, 0);
    nn->off.resize(ns, 0);
    nn->hcounts.resize(2 * ns, 0);
  }
  // systems whose corrections were rejected kOffAfter times in a row get none
  SysBatch sb = sb0;
  sb.n = 0;
  for (int k = 0; k < sb0.n; ++k) {
    if (nn->off[sb0.vslot[k]]) continue;
    sb.orow[sb.n] = sb0.orow[k];
    sb.vslot[sb.n] = sb0.vslot[k];
    sb.dslot[sb.n] = sb0.dslot[k];
    sb.n++;
  }
  if (sb.n == 0) return FNLH_OK;
  double* res = r;
  if (!res) {
    res = (double*)nn->rr.p;
    outer_residual_of(c, ns, sb, x, b, res, s);
  }
  const NnBufs B = bufs(nn);
  for (int k = 0; k < sb.n; ++k) {
    NnVec rv;
    rv.d64 = res;
    rv.ns = ns;
    rv.vs = sb.vslot[k];
    features(nn, sb.orow[k], rv, nullptr, s);
    nn_launch_forward(c->storage, p, c->offd.p, B, s);
    NnOut o;
    o.out = (double*)nn->xt.p;
    o.base = x;
    o.ns = ns;
    o.vs = sb.vslot[k];
    nn_launch_output(p, B, o, s);
  }
  outer_residual_of(c, ns, sb, (const double*)nn->xt.p, b, (double*)nn->rn.p, s);
  for (int k = 0; k < sb.n; ++k)
    nn_launch_step(p, x, (const double*)nn->xt.p, res, (const double*)nn->rn.p, ns, sb.vslot[k], st,
                   (double*)nn->part4.p, (double*)nn->alpha.p, (int*)nn->counts.p, kAccept, s);
  int rc = check_launch(c, "learned step launch");
  if (rc) return rc;
  // the controller: a rejection extends a system's run of rejections, an acceptance ends it
  HIPC(c, hipMemcpyAsync(nn->hcounts.data(), nn->counts.p, (size_t)ns * 2 * sizeof(int), hipMemcpyDeviceToHost, s),
       "read counts");
  HIPC(c, hipStreamSynchronize(s), "counts sync");
  for (int k = 0; k < sb.n; ++k) {
    const int vs = sb.vslot[k];
    const int acc = nn->hcounts[2 * vs], rej = nn->hcounts[2 * vs + 1];
    if (rej > nn->prev_rej[vs]) {
      if (++nn->consec[vs] >= kOffAfter) nn->off[vs] = 1;
    } else if (acc > nn->prev_acc[vs]) {
      nn->consec[vs] = 0;
    }
    nn->prev_acc[vs] = acc;
    nn->prev_rej[vs] = rej;
  }
  return FNLH_OK;
}

double* nn_step_residual(fnlh_ctx c) { return (double*)c->nn->rr.p; }

int nn_relax_counts(fnlh_ctx c, int ns, int* host_counts, hipStream_t s) {
  HIPC(c, hipMemcpyAsync(host_counts, c->nn->counts.p, (size_t)ns * 2 * sizeof(int), hipMemcpyDeviceToHost, s),
       "read counts");
  HIPC(c, hipStreamSynchronize(s), "counts sync");
  return FNLH_OK;
}

}  // namespace fnlh

extern "C" {

int fnlh_nn_create(fnlh_nn* out, fnlh_ctx c, int32_t hidden) {
  if (!out || !c) return FNLH_E_ARG;
  *out = nullptr;
  if (hidden != 0 && hidden != 64)
    return set_err(c, FNLH_E_ARG, "network: hidden width 64 only (the matrix-core tiles are built for it)");
  if (c->nn) return set_err(c, FNLH_E_ORDER, "network: context already has one");
  fnlh_nn nn = new fnlh_nn_s();
  nn->c = c;
  const size_t NP = (size_t)c->L.NP;
  nn->G = auto_groups(c);
  int rc = 0;
  auto fail = [&](int code) {
    free_all(nn);
    delete nn;
    return code;
  };
  if ((rc = dalloc(c, nn->master, kNnParams * sizeof(float), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->mom1, kNnParams * sizeof(float), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->mom2, kNnParams * sizeof(float), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->grad, kNnParams * sizeof(float), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->wt, kNnPadded * sizeof(uint16_t), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->w, kNnPadded * sizeof(uint16_t), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->u, NP * kNnU * sizeof(uint16_t), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->h, NP * 64 * sizeof(uint16_t), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->d, NP * 16 * sizeof(float), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->sc, sizeof(NnScalars), "alloc network"))) return fail(rc);
  if ((rc = dalloc(c, nn->part, (size_t)c->L.n_tiles * sizeof(double), "alloc network"))) return fail(rc);
  if (hipMemset(nn->d.p, 0, nn->d.bytes) != hipSuccess) return fail(FNLH_E_HIP);
  c->nn = nn;
  *out = nn;
  return FNLH_OK;
}

int fnlh_nn_set_grad_groups(fnlh_nn nn, int32_t groups) {
  if (!nn) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  if (groups < 0 || groups > kMaxG) return set_err(nn->c, FNLH_E_ARG, "network: gradient workgroups in 0..512");
  nn->G = groups == 0 ? auto_groups(nn->c) : groups;
  return FNLH_OK;
}

int fnlh_nn_destroy(fnlh_nn nn) {
  if (!nn) return FNLH_E_ARG;
  if (nn->c) nn->c->nn = nullptr;
  free_all(nn);
  delete nn;
  return FNLH_OK;
}

int fnlh_nn_set_weights(fnlh_nn nn, const float* w) {
  if (!nn || !w) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  for (int i = 0; i < kNnParams; ++i)
    if (!std::isfinite(w[i])) return set_err(c, FNLH_E_ARG, "network: weights must be finite");
  HIPC(c, hipMemcpy(nn->master.p, w, kNnParams * sizeof(float), hipMemcpyHostToDevice), "upload weights");
  HIPC(c, hipMemset(nn->mom1.p, 0, nn->mom1.bytes), "zero");
  HIPC(c, hipMemset(nn->mom2.p, 0, nn->mom2.bytes), "zero");
  nn_launch_cast((const float*)nn->master.p, (uint16_t*)nn->wt.p, (uint16_t*)nn->w.p, nullptr);
  HIPC(c, hipDeviceSynchronize(), "cast weights");
  nn->adam_t = 0;
  nn->weights_set = true;
  return check_launch(c, "cast weights");
}

int fnlh_nn_get_weights(fnlh_nn nn, float* w) {
  if (!nn || !w) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  HIPC(nn->c, hipMemcpy(w, nn->master.p, kNnParams * sizeof(float), hipMemcpyDeviceToHost), "read weights");
  return FNLH_OK;
}

int fnlh_nn_apply(fnlh_nn nn, int32_t sys, const double* r, double* dx, void* stream) {
  int rc = ready(nn);
  if (rc) return rc;
  fnlh_ctx c = nn->c;
  if (sys < 0 || sys >= c->n_sys) return set_err(c, FNLH_E_ARG, "network: system out of range");
  if (!r || !dx) return set_err(c, FNLH_E_ARG, "network: null vector");
  hipStream_t s = S(stream);
  features(nn, sys, user_vec(c, r), nullptr, s);
  nn_launch_forward(c->storage, c->pat(), c->offd.p, bufs(nn), s);
  NnOut o;
  o.out = dx;
  o.iperm = (const int32_t*)c->iperm.p;
  nn_launch_output(c->pat(), bufs(nn), o, s);
  return check_launch(c, "network apply launch");
}

int fnlh_nn_loss_grad(fnlh_nn nn, int32_t n, const int32_t* sys, const double* const* r, const double* const* e,
                      float* grad, double* loss, void* stream) {
  int rc = ready(nn);
  if (rc) return rc;
  fnlh_ctx c = nn->c;
  if (n < 1 || !sys || !r || !e) return set_err(c, FNLH_E_ARG, "network: bad arguments");
  for (int k = 0; k < n; ++k) {
    if (sys[k] < 0 || sys[k] >= c->n_sys) return set_err(c, FNLH_E_ARG, "network: system out of range");
    if (!r[k] || !e[k]) return set_err(c, FNLH_E_ARG, "network: null vector");
  }
  hipStream_t s = S(stream);
  if (!nn->loss.p && (rc = dalloc(c, nn->loss, sizeof(double), "alloc network"))) return rc;
  rc = batch_grad(
      nn, n,
      [&](int k, int& sy, NnVec& rv, NnVec& ev) {
        sy = sys[k];
        rv = user_vec(c, r[k]);
        ev = user_vec(c, e[k]);
      },
      (double*)nn->loss.p, s);
  if (rc) return rc;
  if (grad) HIPC(c, hipMemcpyAsync(grad, nn->grad.p, kNnParams * sizeof(float), hipMemcpyDeviceToHost, s), "read");
  double l = 0.0;
  HIPC(c, hipMemcpyAsync(&l, nn->loss.p, sizeof(double), hipMemcpyDeviceToHost, s), "read");
  HIPC(c, hipStreamSynchronize(s), "gradient sync");
  if (loss) *loss = l;
  return FNLH_OK;
}

int fnlh_nn_add_pairs(fnlh_nn nn, int32_t n, const int32_t* sys, const double* const* r, const double* const* e,
                      void* stream) {
  if (!nn) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  if (c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "network: harmonics first");
  if (n < 1 || !sys || !r || !e) return set_err(c, FNLH_E_ARG, "network: bad arguments");
  for (int k = 0; k < n; ++k) {
    if (sys[k] < 0 || sys[k] >= c->n_sys) return set_err(c, FNLH_E_ARG, "network: system out of range");
    if (!r[k] || !e[k]) return set_err(c, FNLH_E_ARG, "network: null vector");
  }
  hipStream_t s = S(stream);
  int rc;
  if (nn->n_pairs + n > nn->cap_pairs &&
      (rc = grow_pairs(nn, std::max<int64_t>(nn->n_pairs + n, 2 * nn->cap_pairs), s)))
    return rc;
  const size_t pair = (size_t)2 * c->L.NP * 12;  // BF16 values
  const DevPattern p = c->pat();
  for (int k = 0; k < n; ++k) {
    uint16_t* dst = (uint16_t*)nn->pool.p + (size_t)(nn->n_pairs + k) * pair;
    nn_launch_pack16(p, (const int32_t*)c->iperm.p, r[k], 1.0, dst, s);
    nn_launch_pack16(p, (const int32_t*)c->iperm.p, e[k], 1.0, dst + pair / 2, s);
    nn->pair_sys.push_back(sys[k]);
  }
  nn->n_pairs += n;
  return check_launch(c, "store pairs");
}

int fnlh_nn_reserve_pairs(fnlh_nn nn, int64_t n_pairs, void* stream) {
  if (!nn || n_pairs < 0) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  if (n_pairs <= nn->cap_pairs) return FNLH_OK;
  return grow_pairs(nn, n_pairs, S(stream));
}

int fnlh_nn_clear_pairs(fnlh_nn nn) {
  if (!nn) return FNLH_E_ARG;
  nn->n_pairs = 0;
  nn->pair_sys.clear();
  return FNLH_OK;
}

int fnlh_nn_pairs(fnlh_nn nn, int64_t* n_pairs) {
  if (!nn || !n_pairs) return FNLH_E_ARG;
  *n_pairs = nn->n_pairs;
  return FNLH_OK;
}

int fnlh_nn_train(fnlh_nn nn, int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss, void* stream) {
  int rc = ready(nn);
  if (rc) return rc;
  fnlh_ctx c = nn->c;
  if (steps < 0 || batch < 1 || !(lr > 0.f)) return set_err(c, FNLH_E_ARG, "train: need steps >= 0, batch >= 1, lr > 0");
  if (nn->n_pairs == 0) return set_err(c, FNLH_E_ORDER, "train: no training pairs");
  if (steps == 0) return FNLH_OK;
  hipStream_t s = S(stream);
  DevBuf hist;
  if ((rc = dalloc(c, hist, (size_t)steps * sizeof(double), "alloc loss history"))) return rc;
  const size_t pair = (size_t)2 * c->L.NP * 12;  // BF16 values
  uint64_t z = seed;
  auto next = [&]() {  // splitmix64
    z += 0x9e3779b97f4a7c15ull;
    uint64_t q = z;
    q = (q ^ (q >> 30)) * 0xbf58476d1ce4e5b9ull;
    q = (q ^ (q >> 27)) * 0x94d049bb133111ebull;
    return q ^ (q >> 31);
  };
  for (int t = 0; t < steps && !rc; ++t) {
    rc = batch_grad(
        nn, batch,
        [&](int, int& sy, NnVec& rv, NnVec& ev) {
          const int64_t i = (int64_t)(next() % (uint64_t)nn->n_pairs);
          const uint16_t* base = (const uint16_t*)nn->pool.p + (size_t)i * pair;
          sy = nn->pair_sys[i];
          rv = NnVec{};
          rv.b16 = base;
          ev = NnVec{};
          ev.b16 = base + pair / 2;
        },
        (double*)hist.p + t, s);
    if (rc) break;
    nn->adam_t++;
    nn_launch_adam((float*)nn->master.p, (float*)nn->mom1.p, (float*)nn->mom2.p, (const float*)nn->grad.p,
                   kNnParams, lr, kB1, kB2, kEps, nn->adam_t, s);
    nn_launch_cast((const float*)nn->master.p, (uint16_t*)nn->wt.p, (uint16_t*)nn->w.p, s);
    rc = check_launch(c, "train launch");
  }
  if (!rc && loss) {
    std::vector<double> h(steps);
    hipError_t e = hipMemcpyAsync(h.data(), hist.p, (size_t)steps * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(c, e, "read loss history");
    for (int t = 0; t < steps; ++t) loss[t] = (float)h[t];
  }
  if (!rc) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(c, e, "train sync");
  }
  dfree(hist);
  return rc;
}

int fnlh_nn_generate(fnlh_nn nn, int32_t n, const int32_t* sys, int32_t starts, int32_t snapshots, int32_t every,
                     uint64_t seed, void* stream) {
  if (!nn) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  if (!c->have_matrix || c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "generate: matrix and harmonics first");
  if (n < 1 || n > 16 || !sys || starts < 1 || snapshots < 1 || every < 1)
    return set_err(c, FNLH_E_ARG, "generate: need 1..16 systems and starts, snapshots, every >= 1");
  for (int j = 0; j < n; ++j)
    if (sys[j] < 0 || sys[j] >= c->n_sys) return set_err(c, FNLH_E_ARG, "generate: system out of range");
  hipStream_t s = S(stream);
  const int64_t N = c->L.N;
  const size_t vb = (size_t)N * 12 * sizeof(double);
  const int64_t add = (int64_t)n * starts * snapshots;
  int rc;
  if (nn->n_pairs + add > nn->cap_pairs && (rc = grow_pairs(nn, nn->n_pairs + add, s))) return rc;
  DevBuf X, Z, R;
  if ((rc = dalloc(c, X, (size_t)n * vb, "alloc generate"))) return rc;
  if ((rc = dalloc(c, Z, vb, "alloc generate")) || (rc = dalloc(c, R, vb, "alloc generate"))) {
    dfree(X);
    dfree(Z);
    return rc;
  }
  launch_fill_zero(Z.p, vb, s);
  std::vector<double*> xp(n);
  std::vector<const double*> zp(n, (const double*)Z.p);
  for (int j = 0; j < n; ++j) xp[j] = (double*)X.p + (size_t)j * N * 12;
  fnlh_relax_opts o;
  std::memset(&o, 0, sizeof(o));
  o.kind = FNLH_DILU;
  o.max_sweeps = every;
  o.rtol = 0.0;
  o.check_every = 16;
  o.use_graph = 1;
  const DevPattern p = c->pat();
  const size_t pair = (size_t)2 * c->L.NP * 12;  // BF16 values
  rc = FNLH_OK;
  for (int k = 0; k < starts && rc >= 0; ++k) {
    for (int j = 0; j < n; ++j) nn_launch_uniform(N * 12, nn_start_key(seed, (int64_t)j * starts + k), xp[j], s);
    for (int t = 0; t < snapshots && rc >= 0; ++t) {
      rc = fnlh_relax(c, n, sys, xp.data(), zp.data(), &o, nullptr, s);
      for (int j = 0; j < n && rc >= 0; ++j) {
        rc = fnlh_residual(c, sys[j], xp[j], (const double*)Z.p, (double*)R.p, nullptr, s);
        if (rc < 0) break;
        uint16_t* dst = (uint16_t*)nn->pool.p + (size_t)nn->n_pairs * pair;
        nn_launch_pack16(p, (const int32_t*)c->iperm.p, (const double*)R.p, 1.0, dst, s);
        nn_launch_pack16(p, (const int32_t*)c->iperm.p, xp[j], -1.0, dst + pair / 2, s);  // e = x* - x = -x
        nn->pair_sys.push_back(sys[j]);
        nn->n_pairs++;
      }
    }
  }
  if (rc >= 0) rc = check_launch(c, "generate launch");
  const hipError_t e = hipStreamSynchronize(s);
  dfree(X);
  dfree(Z);
  dfree(R);
  if (rc < 0) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "generate sync");
  return FNLH_OK;
}

int fnlh_nn_get_pair(fnlh_nn nn, int64_t k, int32_t* sys, double* r, double* e, void* stream) {
  if (!nn) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  if (k < 0 || k >= nn->n_pairs) return set_err(c, FNLH_E_ARG, "get_pair: index out of range");
  if (sys) *sys = nn->pair_sys[k];
  const size_t pair = (size_t)2 * c->L.NP * 12;
  const uint16_t* base = (const uint16_t*)nn->pool.p + (size_t)k * pair;
  const DevPattern p = c->pat();
  hipStream_t s = S(stream);
  if (r) nn_launch_unpack16(p, (const int32_t*)c->iperm.p, base, r, s);
  if (e) nn_launch_unpack16(p, (const int32_t*)c->iperm.p, base + pair / 2, e, s);
  return check_launch(c, "get_pair launch");
}

int fnlh_nn_copy_state(fnlh_nn dst, fnlh_nn src) {
  if (!dst || !src) return FNLH_E_ARG;
  if (!dst->c || !src->c) return FNLH_E_ORDER;
  fnlh_ctx c = dst->c;
  if (!src->weights_set) return set_err(c, FNLH_E_ORDER, "copy_state: source has no weights");
  if (src->c->dev != c->dev) return set_err(c, FNLH_E_ARG, "copy_state: networks on different devices");
  HIPC(c, hipDeviceSynchronize(), "copy sync");
  HIPC(c, hipMemcpy(dst->master.p, src->master.p, kNnParams * sizeof(float), hipMemcpyDeviceToDevice), "copy");
  HIPC(c, hipMemcpy(dst->mom1.p, src->mom1.p, kNnParams * sizeof(float), hipMemcpyDeviceToDevice), "copy");
  HIPC(c, hipMemcpy(dst->mom2.p, src->mom2.p, kNnParams * sizeof(float), hipMemcpyDeviceToDevice), "copy");
  nn_launch_cast((const float*)dst->master.p, (uint16_t*)dst->wt.p, (uint16_t*)dst->w.p, nullptr);
  HIPC(c, hipDeviceSynchronize(), "cast weights");
  dst->adam_t = src->adam_t;
  dst->weights_set = true;
  return check_launch(c, "cast weights");
}

namespace {
struct CkptHead {
  char magic[8];
  int32_t hidden, n_params;
  int64_t adam_t;
};
}  // namespace

int fnlh_nn_save(fnlh_nn nn, const char* path) {
  if (!nn || !path) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  if (!nn->weights_set) return set_err(c, FNLH_E_ORDER, "save: weights not set");
  std::vector<float> buf(3 * (size_t)kNnParams);
  HIPC(c, hipDeviceSynchronize(), "save sync");
  HIPC(c, hipMemcpy(buf.data(), nn->master.p, kNnParams * sizeof(float), hipMemcpyDeviceToHost), "read master");
  HIPC(c, hipMemcpy(buf.data() + kNnParams, nn->mom1.p, kNnParams * sizeof(float), hipMemcpyDeviceToHost), "read m");
  HIPC(c, hipMemcpy(buf.data() + 2 * kNnParams, nn->mom2.p, kNnParams * sizeof(float), hipMemcpyDeviceToHost),
       "read v");
  CkptHead h;
  std::memcpy(h.magic, kMagic, 8);
  h.hidden = nn->hidden;
  h.n_params = kNnParams;
  h.adam_t = nn->adam_t;
  FILE* f = std::fopen(path, "wb");
  if (!f) return set_err(c, FNLH_E_ARG, "save: cannot open the file for writing");
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? FNLH_OK : set_err(c, FNLH_E_ARG, "save: write failed");
}

int fnlh_nn_load(fnlh_nn nn, const char* path) {
  if (!nn || !path) return FNLH_E_ARG;
  if (!nn->c) return FNLH_E_ORDER;
  fnlh_ctx c = nn->c;
  FILE* f = std::fopen(path, "rb");
  if (!f) return set_err(c, FNLH_E_ARG, "load: cannot open the file");
  CkptHead h;
  std::vector<float> buf(3 * (size_t)kNnParams);
  bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
  ok = ok && std::memcmp(h.magic, kMagic, 8) == 0 && h.hidden == nn->hidden && h.n_params == kNnParams &&
       h.adam_t >= 0 && h.adam_t < (int64_t)1 << 30;
  ok = ok && std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the moments
  std::fclose(f);
  if (!ok) return set_err(c, FNLH_E_ARG, "load: not a checkpoint of this network (tag, sizes or length)");
  for (float v : buf)
    if (!std::isfinite(v)) return set_err(c, FNLH_E_ARG, "load: non-finite values");
  HIPC(c, hipMemcpy(nn->master.p, buf.data(), kNnParams * sizeof(float), hipMemcpyHostToDevice), "upload");
  HIPC(c, hipMemcpy(nn->mom1.p, buf.data() + kNnParams, kNnParams * sizeof(float), hipMemcpyHostToDevice), "upload");
  HIPC(c, hipMemcpy(nn->mom2.p, buf.data() + 2 * kNnParams, kNnParams * sizeof(float), hipMemcpyHostToDevice),
       "upload");
  nn_launch_cast((const float*)nn->master.p, (uint16_t*)nn->wt.p, (uint16_t*)nn->w.p, nullptr);
  HIPC(c, hipDeviceSynchronize(), "cast weights");
  nn->adam_t = (int)h.adam_t;
  nn->weights_set = true;
  return check_launch(c, "cast weights");
}

int fnlh_nn_selftest(fnlh_ctx c, const uint16_t* a, const uint16_t* bt, float* out) {
  if (!c || !a || !bt || !out) return FNLH_E_ARG;
  DevBuf da, db, dc;
  int rc = 0;
  if ((rc = dalloc(c, da, 64 * 64 * 2, "selftest"))) return rc;
  if ((rc = dalloc(c, db, 64 * 64 * 2, "selftest"))) return rc;
  if ((rc = dalloc(c, dc, 64 * 64 * 4, "selftest"))) return rc;
  hipError_t e = hipMemcpy(da.p, a, 64 * 64 * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db.p, bt, 64 * 64 * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    nn_launch_selftest((const uint16_t*)da.p, (const uint16_t*)db.p, (float*)dc.p, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dc.p, 64 * 64 * 4, hipMemcpyDeviceToHost);
  dfree(da);
  dfree(db);
  dfree(dc);
  if (e != hipSuccess) return hip_fail(c, e, "selftest");
  return FNLH_OK;
}

}  // extern "C"
