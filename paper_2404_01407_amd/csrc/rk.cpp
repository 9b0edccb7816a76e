// RK(5,3) pseudo-time driver around the linear solve (include/fnlh.h, "pseudo-time
// driver"): section "Generalized RK Scheme for The Mean Flow" (eqn:rk with the hybrid
// RK(5,3) coefficient table), section "Generalized RK Scheme for Time-Linearized Harmonic
// Flows" (eqn:rk_lin) and section "Solution Update" (each stage solves
// K x = -Gamma alpha_k R^(k) inexactly).  K is assembled once per pseudo-time step; the
// stage residuals are kernels (Rusanov residual, matrix-free linearised residual), the
// stage solves go through fnlh_relax.
#include <cmath>
#include <vector>

#include "ctx.h"

using namespace fnlh;

namespace {

constexpr double kAlpha[5] = {0.25, 1.0 / 6.0, 0.375, 0.5, 1.0};

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// sum of slot `stride`-spaced partials on the host
int host_sum(fnlh_ctx c, const DevBuf& part, int64_t n, int64_t stride, hipStream_t s, double& out) {
  std::vector<double> h((size_t)(n * stride));
  HIPC(c, hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s), "read norm");
  HIPC(c, hipStreamSynchronize(s), "norm sync");
  double t = 0.0;
  for (int64_t i = 0; i < n; ++i) t += h[(size_t)(i * stride)];
  out = t;
  return FNLH_OK;
}

struct Bufs {
  std::vector<DevBuf*> all;
  ~Bufs() {
    for (DevBuf* b : all) dfree(*b);
  }
};

int worse(int a, int b) {
  if (a < 0 || b < 0) return a < b ? a : b;
  if (a == FNLH_DIVERGED || b == FNLH_DIVERGED) return FNLH_DIVERGED;
  return a > b ? a : b;
}

}  // namespace

extern "C" {

int fnlh_rusanov_residual(fnlh_ctx c, const double* state, const double* bstate, double* R, double* norm2,
                          void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!state || !R) return set_err(c, FNLH_E_ARG, "rusanov_residual: null vector");
  hipStream_t s = S(stream);
  DevBuf q, part;
  Bufs keep{{&q, &part}};
  int rc;
  if ((rc = dalloc(c, q, (size_t)c->L.NP * 6 * sizeof(double), "alloc residual state")) ||
      (rc = dalloc(c, part, (size_t)c->L.n_tiles * sizeof(double), "alloc residual norm")))
    return rc;
  HIPC(c, hipMemsetAsync(q.p, 0, q.bytes, s), "zero");
  const DevPattern p = c->pat();
  launch_to_internal(p, (const int32_t*)c->iperm.p, state, (double*)q.p, 6, 1, 0, s);
  DevFlow f = c->flow();
  f.state = (const double*)q.p;
  f.bstate = bstate;
  launch_rusanov_residual(p, f, (const int32_t*)c->iperm.p, R, (double*)part.p, s);
  if ((rc = check_launch(c, "residual launch"))) return rc;
  double n2 = 0.0;
  if ((rc = host_sum(c, part, c->L.n_tiles, 1, s, n2))) return rc;
  if (norm2) *norm2 = n2;
  return FNLH_OK;
}

int fnlh_rk_mean(fnlh_ctx c, int32_t sys, double* state, const double* bstate, int32_t n_steps, double eps,
                 double sigma, int32_t scheme, const fnlh_relax_opts* lin, double* res_norm, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!state || !lin || n_steps < 0) return set_err(c, FNLH_E_ARG, "rk_mean: bad arguments");
  if (c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "rk_mean: set the harmonics first");
  if (sys < 0 || sys >= c->n_sys) return set_err(c, FNLH_E_ARG, "rk_mean: system out of range");
  for (int z = 0; z < c->L.n_zones; ++z)
    if (c->omega[(size_t)sys * c->L.n_zones + z] != 0.0)
      return set_err(c, FNLH_E_ARG, "rk_mean: the mean-flow system needs omega = 0");
  if (lin->kind == FNLH_LEARNED) return set_err(c, FNLH_E_ARG, "rk_mean: stage solves are DILU, SGS or Jacobi");
  hipStream_t s = S(stream);
  const int64_t N = c->L.N;
  const double G = scheme == FNLH_IMPLICIT ? 1.0 / eps : sigma;
  DevBuf q0, R, x, b, q, part;
  Bufs keep{{&q0, &R, &x, &b, &q, &part}};
  int rc;
  if ((rc = dalloc(c, q0, (size_t)N * 6 * sizeof(double), "alloc rk")) ||
      (rc = dalloc(c, R, (size_t)N * 6 * sizeof(double), "alloc rk")) ||
      (rc = dalloc(c, x, (size_t)N * 12 * sizeof(double), "alloc rk")) ||
      (rc = dalloc(c, b, (size_t)N * 12 * sizeof(double), "alloc rk")) ||
      (rc = dalloc(c, q, (size_t)c->L.NP * 6 * sizeof(double), "alloc rk")) ||
      (rc = dalloc(c, part, (size_t)c->L.n_tiles * sizeof(double), "alloc rk")))
    return rc;
  HIPC(c, hipMemsetAsync(q.p, 0, q.bytes, s), "zero");
  const int32_t* iperm = (const int32_t*)c->iperm.p;
  int worst = FNLH_OK;
  for (int n = 0; n < n_steps; ++n) {
    // K at Q^n, kept through the five stages
    if ((rc = fnlh_assemble_jacobian(c, state, bstate, eps, sigma, scheme, stream))) return rc;
    HIPC(c, hipMemcpyAsync(q0.p, state, q0.bytes, hipMemcpyDeviceToDevice, s), "copy state");
    const DevPattern p = c->pat();
    DevFlow f = c->flow();
    f.state = (const double*)q.p;
    f.bstate = bstate;
    for (int k = 0; k < 5; ++k) {
      launch_to_internal(p, iperm, state, (double*)q.p, 6, 1, 0, s);
      launch_rusanov_residual(p, f, iperm, (double*)R.p, (double*)part.p, s);
      if ((rc = check_launch(c, "rk residual"))) return rc;
      if (k == 0 && res_norm) {
        double n2 = 0.0;
        if ((rc = host_sum(c, part, c->L.n_tiles, 1, s, n2))) return rc;
        res_norm[n] = std::sqrt(n2);
      }
      launch_rk_rhs_real(N * 6, (const double*)R.p, -G * kAlpha[k], (double*)b.p, s);
      launch_fill_zero(x.p, x.bytes, s);
      double* xp = (double*)x.p;
      const double* bp = (const double*)b.p;
      rc = fnlh_relax(c, 1, &sys, &xp, &bp, lin, nullptr, stream);
      if (rc < 0) return rc;
      worst = worse(worst, rc);
      launch_rk_update(false, N * 6, (const double*)q0.p, (const double*)x.p, state, s);
    }
  }
  if ((rc = check_launch(c, "rk update"))) return rc;
  HIPC(c, hipStreamSynchronize(s), "rk sync");
  return worst;
}

int fnlh_rk_harmonic(fnlh_ctx c, int32_t sys, double* qhat, const double* fhat, int32_t n_steps,
                     const fnlh_relax_opts* lin, double* res_norm, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!qhat || !fhat || !lin || n_steps < 0) return set_err(c, FNLH_E_ARG, "rk_harmonic: bad arguments");
  if (!c->assembled) return set_err(c, FNLH_E_ORDER, "rk_harmonic: assemble the Jacobian first");
  if (c->n_sys == 0) return set_err(c, FNLH_E_ORDER, "rk_harmonic: set the harmonics first");
  if (sys < 0 || sys >= c->n_sys) return set_err(c, FNLH_E_ARG, "rk_harmonic: system out of range");
  if (lin->kind == FNLH_LEARNED) return set_err(c, FNLH_E_ARG, "rk_harmonic: stage solves are DILU, SGS or Jacobi");
  hipStream_t s = S(stream);
  const int64_t N = c->L.N, NP = c->L.NP;
  const double G = c->scheme == FNLH_IMPLICIT ? 1.0 / c->eps : c->sigma;
  DevBuf q0, xi, bi, ri, xu, bu, part;
  Bufs keep{{&q0, &xi, &bi, &ri, &xu, &bu, &part}};
  int rc;
  const size_t vu = (size_t)N * 12 * sizeof(double), vi = (size_t)NP * 12 * sizeof(double);
  if ((rc = dalloc(c, q0, vu, "alloc rk")) || (rc = dalloc(c, xi, vi, "alloc rk")) ||
      (rc = dalloc(c, bi, vi, "alloc rk")) || (rc = dalloc(c, ri, vi, "alloc rk")) ||
      (rc = dalloc(c, xu, vu, "alloc rk")) || (rc = dalloc(c, bu, vu, "alloc rk")) ||
      (rc = dalloc(c, part, (size_t)c->L.n_tiles * kPartialSlots * sizeof(double), "alloc rk")))
    return rc;
  HIPC(c, hipMemsetAsync(xi.p, 0, vi, s), "zero");
  HIPC(c, hipMemsetAsync(bi.p, 0, vi, s), "zero");
  const DevPattern p = c->pat();
  const int32_t* iperm = (const int32_t*)c->iperm.p;
  DevFlow fJ = c->flow();  // the residual Jacobian J itself (K without the CFL term)
  fJ.diag_scale = 1.0;
  fJ.offdiag = 1;
  fJ.ent_drop = nullptr;  // the residual keeps every coupling (only K is partitioned)
  SysBatch sb;
  sb.n = 1;
  sb.orow[0] = sys;
  sb.dslot[0] = 0;
  sb.vslot[0] = 0;
  launch_to_internal(p, iperm, fhat, (double*)bi.p, 12, 1, 0, s);
  if (c->is_frozen(sys)) launch_zero_sixth(N, qhat, 1, 0, s);  // the sixth unknown is held at 0
  int worst = FNLH_OK;
  for (int n = 0; n < n_steps; ++n) {
    HIPC(c, hipMemcpyAsync(q0.p, qhat, vu, hipMemcpyDeviceToDevice, s), "copy state");
    for (int k = 0; k < 5; ++k) {
      // r = f^ - (J + i omega V) q^ = -R_l
      launch_to_internal(p, iperm, qhat, (double*)xi.p, 12, 1, 0, s);
      launch_resid_mfree(p, fJ, (const double*)xi.p, (const double*)bi.p, (double*)ri.p, 1, sb, (double*)part.p, s);
      if ((rc = check_launch(c, "rk residual"))) return rc;
      if (k == 0 && res_norm) {
        double n2 = 0.0;
        if ((rc = host_sum(c, part, c->L.n_tiles, kPartialSlots, s, n2))) return rc;
        res_norm[n] = std::sqrt(n2);
      }
      launch_to_user(p, iperm, (const double*)ri.p, (double*)bu.p, 12, 1, 0, s);
      launch_scale(N * 12, (double*)bu.p, G * kAlpha[k], s);  // b = -Gamma alpha_k R_l
      launch_fill_zero(xu.p, vu, s);
      double* xp = (double*)xu.p;
      const double* bp = (const double*)bu.p;
      rc = fnlh_relax(c, 1, &sys, &xp, &bp, lin, nullptr, stream);
      if (rc < 0) return rc;
      worst = worse(worst, rc);
      launch_rk_update(true, N * 12, (const double*)q0.p, (const double*)xu.p, qhat, s);
    }
  }
  if ((rc = check_launch(c, "rk update"))) return rc;
  HIPC(c, hipStreamSynchronize(s), "rk sync");
  return worst;
}

}  // extern "C"
