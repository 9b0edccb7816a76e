// Restarted flexible GMRES around the DILU/SGS/Jacobi preconditioner (include/fnlh.h,
// "Krylov solve").  Section "Generalized RK Scheme for The Mean Flow" of the paper notes
// that the ILU(0) approximation of K^-1 serves either as a smoother (fnlh_relax) or as the
// preconditioner of a Krylov method; this is the textbook FGMRES(m) (Saad, Iterative
// Methods for Sparse Linear Systems, 2nd ed., Alg. 9.6) with right preconditioning, for
// up to kMaxBatch systems at once sharing every block read of the preconditioner sweeps
// and the operator products.
//
// Per iteration j (all systems of the cycle still running):
//   z_j = M^-1 v_j (precond_apply: inner sweeps from 0, after a learned step for
//   FNLH_LEARNED), W = -(K + i omega V) z_j (the FP64
//   operator residual with b = 0), one classical Gram-Schmidt pass of W against v_0..v_j
//   (one inner-product launch that also yields ||W||^2, one multi-axpy), a second pass
//   only where the DGKS test asks for it, the Hessenberg column to the host, a complex
//   Givens rotation per system, and v_{j+1} = -W / ||W||.  At the end of a cycle x += Z y (y by back substitution) and the
//   true residual restarts the next cycle.
#include <cmath>
#include <complex>
#include <vector>

#include "ctx.h"

using namespace fnlh;

namespace {

using cd = std::complex<double>;

inline hipStream_t S(void* s) { return (hipStream_t)s; }

struct Bufs {
  std::vector<DevBuf*> all;
  ~Bufs() {
    for (DevBuf* b : all) dfree(*b);
  }
};

// per-system Arnoldi / Givens state of one cycle
struct Cyc {
  std::vector<cd> R;      // upper triangle, column-major (m+1) x m
  std::vector<cd> g;      // rotated right-hand side, m+1
  std::vector<double> c;  // rotation cosines
  std::vector<cd> sn;     // rotation sines
  int k = 0;              // columns built
  bool run = false;
};

// the complex Givens rotation [c s; -conj(s) c] with real c taking (a, b) to (r, 0)
void givens(cd a, cd b, double& c, cd& s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (aa == 0.0) {
    c = 0.0;
    s = std::conj(b) / bb;
    return;
  }
  const double nrm = std::hypot(aa, bb);
  c = aa / nrm;
  s = (a / aa) * std::conj(b) / nrm;
}

}  // namespace

extern "C" {

int fnlh_gmres(fnlh_ctx c, int32_t n, const int32_t* sys, double* const* x, const double* const* b,
               const fnlh_gmres_opts* o, fnlh_gmres_report* rep, double* history, void* stream) {
  if (!c) return FNLH_E_ARG;
  if (!o) return set_err(c, FNLH_E_ARG, "gmres: null options");
  if (n < 1 || n > kMaxBatch) return set_err(c, FNLH_E_ARG, "gmres: 1 <= n <= 16 systems per call");
  if (o->restart < 1 || o->restart > 256 || o->max_iters < 0 || o->inner_sweeps < 1 || !(o->rtol >= 0.0))
    return set_err(c, FNLH_E_ARG, "gmres: need 1 <= restart <= 256, max_iters >= 0, inner_sweeps >= 1, rtol >= 0");
  hipStream_t s = S(stream);
  hipEvent_t e0 = c->ev[0], e1 = c->ev[1];
  HIPC(c, hipEventRecord(e0, s), "event");
  PrecondPlan pp;
  int rc = precond_prepare(c, n, sys, x, b, o->kind, o->inner_sweeps, o->use_graph != 0, s, pp);
  if (rc) return rc;
  const int m = o->restart;
  const int64_t NP = c->L.NP;
  const size_t vb = (size_t)NP * n * 12 * sizeof(double);
  const int64_t vstride = NP * n * 12;
  const int nq = (m + 1) * n;
  const int nblk = mdot_blocks(NP);
  DevBuf V, Z, bz, part, d1, d2, nr, coef;
  Bufs keep{{&V, &Z, &bz, &part, &d1, &d2, &nr, &coef}};
  if ((rc = dalloc(c, V, vb * (m + 1), "alloc gmres basis")) || (rc = dalloc(c, Z, vb * m, "alloc gmres basis")) ||
      (rc = dalloc(c, bz, vb, "alloc gmres")) ||
      (rc = dalloc(c, part, (size_t)nblk * nq * 2 * sizeof(double), "alloc gmres")) ||
      (rc = dalloc(c, d1, (size_t)nq * 2 * sizeof(double), "alloc gmres")) ||
      (rc = dalloc(c, d2, (size_t)nq * 2 * sizeof(double), "alloc gmres")) ||
      (rc = dalloc(c, nr, (size_t)n * 2 * sizeof(double), "alloc gmres")) ||
      (rc = dalloc(c, coef, (size_t)nq * 2 * sizeof(double), "alloc gmres")))
    return rc;
  launch_fill_zero(V.p, V.bytes, s);
  launch_fill_zero(bz.p, bz.bytes, s);
  const DevPattern p = c->pat();
  double* Vp = (double*)V.p;
  double* Zp = (double*)Z.p;
  double* x64 = (double*)c->x64.p;
  const double* b64 = (const double*)c->b64.p;
  auto vec = [&](double* base, int i) { return base + (int64_t)i * vstride; };

  SysBatch all;
  all.n = n;
  for (int k = 0; k < n; ++k) {
    all.orow[k] = sys[k];
    all.vslot[k] = k;
    all.dslot[k] = 0;
  }
  auto sub = [&](const std::vector<char>& on) {
    SysBatch sb;
    sb.n = 0;
    for (int k = 0; k < n; ++k)
      if (on[k]) {
        sb.orow[sb.n] = sys[k];
        sb.vslot[sb.n] = k;
        sb.dslot[sb.n] = 0;
        sb.n++;
      }
    return sb;
  };
  // true residual r = b - A x into v_0 and its norms (host)
  std::vector<double> hbuf((size_t)nq * 2 * 2 + n * 2);
  auto residual = [&](const SysBatch& sb, std::vector<double>& beta) -> int {
    outer_residual_of(c, n, sb, x64, b64, Vp, s);
    launch_mdot(p, n, Vp, vstride, 1, Vp, sb, nq, (double*)part.p, (double*)nr.p, s);  // ||r||^2 per system
    int r2 = check_launch(c, "gmres residual");
    if (r2) return r2;
    HIPC(c, hipMemcpyAsync(hbuf.data(), nr.p, (size_t)sb.n * 2 * sizeof(double), hipMemcpyDeviceToHost, s),
         "read norms");
    HIPC(c, hipStreamSynchronize(s), "gmres sync");
    for (int kk = 0; kk < sb.n; ++kk) beta[sb.vslot[kk]] = std::sqrt(std::max(hbuf[2 * kk], 0.0));
    return FNLH_OK;
  };

  std::vector<double> beta(n, 0.0), n0(n, 0.0);
  std::vector<int> iters(n, 0), restarts(n, 0), status(n, FNLH_NOT_CONVERGED);
  std::vector<char> active(n, 0);
  const int hstride = o->max_iters + 1;
  if ((rc = residual(all, beta))) return rc;
  for (int k = 0; k < n; ++k) {
    n0[k] = beta[k];
    if (history) history[(size_t)k * hstride] = beta[k];
    if (!std::isfinite(beta[k])) {
      status[k] = FNLH_DIVERGED;
    } else if (beta[k] == 0.0 || beta[k] <= o->rtol * n0[k]) {
      status[k] = FNLH_OK;
    } else if (o->max_iters > 0) {
      active[k] = 1;
    }
  }
  std::vector<Cyc> cy(n);
  std::vector<double> h((size_t)nq * 2 * 2);
  while (true) {
    SysBatch cb = sub(active);
    if (cb.n == 0) break;
    // v_0 = r / beta
    KScale sc{};
    for (int kk = 0; kk < cb.n; ++kk) sc.s[kk] = 1.0 / beta[cb.vslot[kk]];
    launch_mscale(p, n, Vp, Vp, sc, cb, s);
    for (int kk = 0; kk < cb.n; ++kk) {
      Cyc& C = cy[cb.vslot[kk]];
      C.R.assign((size_t)(m + 1) * m, cd(0.0));
      C.g.assign(m + 1, cd(0.0));
      C.g[0] = beta[cb.vslot[kk]];
      C.c.assign(m, 0.0);
      C.sn.assign(m, cd(0.0));
      C.k = 0;
      C.run = true;
    }
    std::vector<char> on(active);
    for (int j = 0; j < m; ++j) {
      SysBatch sb = sub(on);
      if (sb.n == 0) break;
      if ((rc = precond_apply(c, pp, n, sb, vec(Vp, j), vec(Zp, j), s))) return rc;
      double* W = vec(Vp, j + 1);
      outer_residual_of(c, n, sb, vec(Zp, j), (const double*)bz.p, W, s);  // W = -A z_j
      // classical Gram-Schmidt, W -= V d with d = V^H W, in one pass; ||W||^2 comes with
      // the products (W is stored as v_{j+1}).  A second pass only for the systems whose
      // W lost more than 1 - 1/sqrt(2) of its norm (the DGKS test).
      launch_mdot(p, n, Vp, vstride, j + 2, W, sb, nq, (double*)part.p, (double*)d1.p, s);
      launch_maxpy(p, n, W, Vp, vstride, j + 1, (const double*)d1.p, -1.0, sb, s);
      if ((rc = check_launch(c, "gmres arnoldi"))) return rc;
      const size_t hn = (size_t)(j + 2) * sb.n * 2;
      HIPC(c, hipMemcpyAsync(h.data(), d1.p, hn * sizeof(double), hipMemcpyDeviceToHost, s), "read hessenberg");
      HIPC(c, hipStreamSynchronize(s), "gmres sync");
      std::vector<cd> hcol((size_t)(j + 1) * sb.n);
      std::vector<double> w2(sb.n), nW(sb.n);
      std::vector<char> again(n, 0);
      bool any_again = false;
      for (int kk = 0; kk < sb.n; ++kk) {
        double s1 = 0.0;
        for (int i = 0; i <= j; ++i) {
          const size_t q = ((size_t)i * sb.n + kk) * 2;
          hcol[(size_t)i * sb.n + kk] = cd(h[q], h[q + 1]);
          s1 += h[q] * h[q] + h[q + 1] * h[q + 1];
        }
        const double nW2 = h[((size_t)(j + 1) * sb.n + kk) * 2];
        nW[kk] = nW2;
        w2[kk] = nW2 - s1;
        if (!(w2[kk] > 0.5 * nW2)) {
          again[sb.vslot[kk]] = 1;
          any_again = true;
        }
      }
      if (any_again) {
        SysBatch sb2 = sub(again);
        launch_mdot(p, n, Vp, vstride, j + 2, W, sb2, nq, (double*)part.p, (double*)d2.p, s);
        launch_maxpy(p, n, W, Vp, vstride, j + 1, (const double*)d2.p, -1.0, sb2, s);
        if ((rc = check_launch(c, "gmres arnoldi"))) return rc;
        const size_t hn2 = (size_t)(j + 2) * sb2.n * 2;
        HIPC(c, hipMemcpyAsync(h.data() + hn, d2.p, hn2 * sizeof(double), hipMemcpyDeviceToHost, s),
             "read hessenberg");
        HIPC(c, hipStreamSynchronize(s), "gmres sync");
        const double* h2 = h.data() + hn;
        for (int k2 = 0; k2 < sb2.n; ++k2) {
          int kk = 0;
          while (sb.vslot[kk] != sb2.vslot[k2]) ++kk;
          double s2 = 0.0;
          for (int i = 0; i <= j; ++i) {
            const size_t q = ((size_t)i * sb2.n + k2) * 2;
            hcol[(size_t)i * sb.n + kk] += cd(h2[q], h2[q + 1]);
            s2 += h2[q] * h2[q] + h2[q + 1] * h2[q + 1];
          }
          w2[kk] = h2[((size_t)(j + 1) * sb2.n + k2) * 2] - s2;
        }
      }
      KScale nx{};
      for (int kk = 0; kk < sb.n; ++kk) {
        const int k = sb.vslot[kk];
        Cyc& C = cy[k];
        // A z_j = -W: the Hessenberg column is minus the Gram-Schmidt coefficients, and
        // h_{j+1,j} = ||W - V d|| = sqrt(||W||^2 - |d|^2) (V orthonormal)
        cd* col = &C.R[(size_t)j * (m + 1)];
        for (int i = 0; i <= j; ++i) col[i] = -hcol[(size_t)i * sb.n + kk];
        // below rounding level of ||A z_j||: A z_j lies in the Krylov space (breakdown)
        const double hnext = w2[kk] > 1e-28 * nW[kk] ? std::sqrt(w2[kk]) : 0.0;
        for (int i = 0; i < j; ++i) {  // earlier rotations
          const cd a = col[i], bq = col[i + 1];
          col[i] = C.c[i] * a + C.sn[i] * bq;
          col[i + 1] = -std::conj(C.sn[i]) * a + C.c[i] * bq;
        }
        double cg;
        cd sg;
        givens(col[j], cd(hnext), cg, sg);
        C.c[j] = cg;
        C.sn[j] = sg;
        col[j] = cg * col[j] + sg * hnext;
        col[j + 1] = 0.0;
        C.g[j + 1] = -std::conj(sg) * C.g[j];
        C.g[j] = cg * C.g[j];
        C.k = j + 1;
        iters[k]++;
        const double res = std::abs(C.g[j + 1]);
        if (history) history[(size_t)k * hstride + iters[k]] = res;
        const bool stop = !(res > o->rtol * n0[k]) || iters[k] >= o->max_iters || !(hnext > 0.0) ||
                          !std::isfinite(res);
        if (stop) {
          on[k] = 0;
          nx.s[kk] = 1.0;
        } else {
          nx.s[kk] = -1.0 / hnext;  // v_{j+1} = A z_j - ... = -W / ||W||
        }
      }
      launch_mscale(p, n, W, W, nx, sb, s);
    }
    // x += Z y, y from R y = g (back substitution), per system of the cycle
    int kmax = 0;
    for (int kk = 0; kk < cb.n; ++kk) kmax = std::max(kmax, cy[cb.vslot[kk]].k);
    std::vector<double> yc((size_t)kmax * cb.n * 2, 0.0);
    for (int kk = 0; kk < cb.n; ++kk) {
      Cyc& C = cy[cb.vslot[kk]];
      std::vector<cd> y(C.k);
      for (int i = C.k - 1; i >= 0; --i) {
        cd t = C.g[i];
        for (int q = i + 1; q < C.k; ++q) t -= C.R[(size_t)q * (m + 1) + i] * y[q];
        y[i] = t / C.R[(size_t)i * (m + 1) + i];
      }
      for (int i = 0; i < C.k; ++i) {
        yc[((size_t)i * cb.n + kk) * 2] = y[i].real();
        yc[((size_t)i * cb.n + kk) * 2 + 1] = y[i].imag();
      }
    }
    if (kmax > 0) {
      HIPC(c, hipMemcpyAsync(coef.p, yc.data(), yc.size() * sizeof(double), hipMemcpyHostToDevice, s), "upload y");
      launch_maxpy(p, n, x64, Zp, vstride, kmax, (const double*)coef.p, 1.0, cb, s);
    }
    if ((rc = residual(cb, beta))) return rc;
    for (int kk = 0; kk < cb.n; ++kk) {
      const int k = cb.vslot[kk];
      restarts[k]++;
      if (!std::isfinite(beta[k])) {
        status[k] = FNLH_DIVERGED;
        active[k] = 0;
      } else if (beta[k] <= o->rtol * n0[k] || beta[k] == 0.0) {
        status[k] = FNLH_OK;
        active[k] = 0;
      } else if (iters[k] >= o->max_iters) {
        status[k] = FNLH_NOT_CONVERGED;
        active[k] = 0;
      }
    }
  }
  launch_to_user_n(p, (const int32_t*)c->iperm.p, x64, x, n, n, 0, s);
  if ((rc = check_launch(c, "gmres final"))) return rc;
  HIPC(c, hipEventRecord(e1, s), "event");
  HIPC(c, hipEventSynchronize(e1), "event sync");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  std::vector<int> counts(2 * n, 0);
  if (pp.learned && (rc = nn_relax_counts(c, n, counts.data(), s))) return rc;
  int worst = FNLH_OK;
  for (int k = 0; k < n; ++k) {
    if (pp.learned && status[k] == FNLH_OK && nn_system_off(c, k)) status[k] = FNLH_FELL_BACK;
    if (rep) {
      rep[k].iters = iters[k];
      rep[k].restarts = restarts[k];
      rep[k].status = status[k];
      rep[k].learned = counts[2 * k];
      rep[k].rel_res = n0[k] > 0.0 ? beta[k] / n0[k] : 0.0;
      rep[k].res0 = n0[k];
      rep[k].t_ms = ms;
    }
    if (status[k] == FNLH_DIVERGED) worst = FNLH_DIVERGED;
    else if (status[k] == FNLH_NOT_CONVERGED && worst != FNLH_DIVERGED) worst = FNLH_NOT_CONVERGED;
    else if (status[k] == FNLH_FELL_BACK && worst == FNLH_OK) worst = FNLH_FELL_BACK;
  }
  return worst;
}

}  // extern "C"
