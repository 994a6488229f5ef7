// (D-)Landweber iteration driver (eqs. (LandweberMeth), (DLandweberMeth)):
//   x_{k+1} = x_k + tau D A'(g - A x_k).
// One iteration is five stream-ordered kernels: residual (fused g - A x with
// FP64 partial norms), transpose (A' or A^T), row forward transform, fused
// column forward/filter/inverse transform, and row inverse transform fused
// with the update x += tau w (and FP64 partials of ||x - f||^2).  Per
// iteration scalars stay on the device as per-workgroup partials and are
// reduced in fixed order once at the end, so the only host crossing is one
// copy of the 2 * iters FP64 scalars.
#include <cmath>
#include <vector>

#include "ar_internal.h"

using namespace ar;

static int ensure_partials(ar_plan_s *p, size_t need_partials, size_t need_scalars) {
  if (need_partials > p->partials_cap) {
    if (p->partials) AR_HIP(hipFree(p->partials));
    p->partials = nullptr;
    p->partials_cap = 0;
    AR_HIP(hipMalloc((void **)&p->partials, need_partials * sizeof(double)));
    p->partials_cap = need_partials;
  }
  if (need_scalars > p->scalars_cap) {
    if (p->scalars) AR_HIP(hipFree(p->scalars));
    p->scalars = nullptr;
    p->scalars_cap = 0;
    AR_HIP(hipMalloc((void **)&p->scalars, need_scalars * sizeof(double)));
    p->scalars_cap = need_scalars;
  }
  return AR_OK;
}

extern "C" int ar_deblur_iterate(ar_plan_t p, const void *g, void *x, int iters, double tau,
                                 int tmode, int precondition, const void *f_true,
                                 double *resnorm_host, double *rre_host, int *best_it_host,
                                 void *stream) {
  if (!p || !g || !x) return fail(AR_EINVAL, "ar_deblur_iterate: null argument");
  if (iters < 0) return fail(AR_EINVAL, "ar_deblur_iterate: iters < 0");
  if (tmode != AR_REBLUR && tmode != AR_ADJOINT)
    return fail(AR_EINVAL, "ar_deblur_iterate: unknown tmode");
  if (!std::isfinite(tau)) return fail(AR_EINVAL, "ar_deblur_iterate: tau must be finite");
  if (g == x || (f_true && (f_true == x || f_true == g)))
    return fail(AR_EALIAS, "ar_deblur_iterate: g, x and f_true must not alias");
  if ((rre_host || best_it_host) && !f_true)
    return fail(AR_EINVAL, "ar_deblur_iterate: RRE outputs need f_true");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (best_it_host) *best_it_host = 0;
  if (iters == 0) return AR_OK;

  const bool want_res = resnorm_host != nullptr;
  const bool want_rre = f_true != nullptr && (rre_host != nullptr || best_it_host != nullptr);
  const int bc = conv_blocks(p, p->n1, p->n2);
  const int bu = precondition ? rows_blocks(p) : axpy_blocks(p);
  const int bf = axpy_blocks(p);
  const size_t need_p = (want_res ? (size_t)iters * bc : 0) + (want_rre ? (size_t)iters * bu + bf : 0);
  const size_t need_s = 2 * (size_t)iters + 1;
  if (want_res || want_rre) {
    int rc = ensure_partials(p, need_p, need_s);
    if (rc != AR_OK) return rc;
  }
  double *res_part = want_res ? p->partials : nullptr;
  double *rre_part = want_rre ? p->partials + (want_res ? (size_t)iters * bc : 0) : nullptr;
  double *f_part = want_rre ? rre_part + (size_t)iters * bu : nullptr;

  int rc = AR_OK;
  if (want_rre && (rc = sumsq_launch(p, f_true, f_part, nullptr, st)) != AR_OK) return rc;
  for (int k = 0; k < iters; ++k) {
    // r = g - A x_k   (+ ||r||^2 partials)
    rc = conv_launch(p, x, p->r, p->w_fwd, 0, 0, p->n1, p->n2, false, g,
                     res_part ? res_part + (size_t)k * bc : nullptr, nullptr, st);
    if (rc != AR_OK) return rc;
    // y = A' r  or  A^T r
    if (tmode == AR_REBLUR) {
      rc = conv_launch(p, p->r, p->y, p->w_rev, 0, 0, p->n1, p->n2, false, nullptr, nullptr,
                       nullptr, st);
    } else {
      rc = conv_launch(p, p->r, p->ext, p->w_rev, -p->q1, -p->q2, p->n1 + 2 * p->q1,
                       p->n2 + 2 * p->q2, true, nullptr, nullptr, nullptr, st, true);
      if (rc == AR_OK) rc = fold_launch(p, p->ext, p->y, st);
    }
    if (rc != AR_OK) return rc;
    double *up = rre_part ? rre_part + (size_t)k * bu : nullptr;
    if (precondition) {
      // x += tau T diag(d) T~ y
      if ((rc = rows_launch(p, p->y, p->c, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st)) != AR_OK)
        return rc;
      if ((rc = cols_launch(p, p->c, p->c, COL_FWD_D_INV, st)) != AR_OK) return rc;
      if ((rc = rows_launch(p, p->c, x, ROW_INV_UPDATE, tau, f_true, up, nullptr, st)) != AR_OK)
        return rc;
    } else {
      if ((rc = axpy_launch(p, x, p->y, tau, f_true, up, nullptr, st)) != AR_OK) return rc;
    }
  }
  if (!(want_res || want_rre)) return AR_OK;
  double *sc = p->scalars;  // [0, iters): ||r_k||^2; [iters, 2 iters): ||x_k - f||^2; [2 iters]: ||f||^2
  if (want_res && (rc = reduce_rows_launch(res_part, iters, bc, sc, st)) != AR_OK) return rc;
  if (want_rre) {
    if ((rc = reduce_rows_launch(rre_part, iters, bu, sc + iters, st)) != AR_OK) return rc;
    if ((rc = reduce_rows_launch(f_part, 1, bf, sc + 2 * (size_t)iters, st)) != AR_OK) return rc;
  }
  std::vector<double> h(2 * (size_t)iters + 1, 0.0);
  AR_HIP(hipMemcpyAsync(h.data(), sc, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  AR_HIP(hipStreamSynchronize(st));
  bool finite = true;
  if (want_res) {
    for (int k = 0; k < iters; ++k) {
      resnorm_host[k] = std::sqrt(h[k]);
      if (!std::isfinite(resnorm_host[k])) finite = false;
    }
  }
  if (want_rre) {
    const double fn = std::sqrt(h[2 * (size_t)iters]);
    int best = 0;
    double bv = 0.0;
    for (int k = 0; k < iters; ++k) {
      const double e = std::sqrt(h[iters + k]) / fn;
      if (rre_host) rre_host[k] = e;
      if (best == 0 || e < bv) {  // first minimiser on ties
        best = k + 1;
        bv = e;
      }
    }
    if (best_it_host) *best_it_host = best;
  }
  if (!finite) return fail(AR_ENONFINITE, "ar_deblur_iterate: residual norm is not finite");
  return AR_OK;
}
