// (D-)Landweber iteration driver (eqs. (LandweberMeth), (DLandweberMeth)):
//   x_{k+1} = x_k + tau D A'(g - A x_k).
// One iteration is five stream-ordered kernels: residual (fused g - A x with
// FP64 partial norms), transpose (A' or A^T), row forward transform, fused
// column forward/filter/inverse transform, and row inverse transform fused
// with the update x += tau w (and FP64 partials of ||x - f||^2).  Per
// iteration scalars stay on the device as per-workgroup partials and are
// reduced in fixed order once at the end, so the only host crossing is one
// copy of the 2 * iters FP64 scalars.  (Capturing long runs into a HIP
// graph was measured slower than direct stream launches: 158 vs 138 us per
// 1024^2 iteration.)
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "ar_internal.h"

using namespace ar;

// Grow the plan's partial-sum and scalar buffers to at least the requested
// sizes.  The plan reserves room for kReserveIters iterations at creation;
// longer runs grow the buffers to twice the need, so that a sequence of
// ever longer runs reallocates rarely (a reallocation frees the old buffer,
// which waits for the device).
static int ensure_partials(ar_plan_s *p, size_t need_partials, size_t need_scalars) {
  if (need_partials > p->partials_cap) {
    const size_t cap = p->partials_cap == 0 ? need_partials : 2 * need_partials;
    if (p->partials) AR_HIP(hipFree(p->partials));
    p->partials = nullptr;
    p->partials_cap = 0;
    AR_HIP(hipMalloc((void **)&p->partials, cap * sizeof(double)));
    p->partials_cap = cap;
  }
  if (need_scalars > p->scalars_cap) {
    const size_t cap = p->scalars_cap == 0 ? need_scalars : 2 * need_scalars;
    if (p->scalars) AR_HIP(hipFree(p->scalars));
    p->scalars = nullptr;
    p->scalars_cap = 0;
    AR_HIP(hipMalloc((void **)&p->scalars, cap * sizeof(double)));
    p->scalars_cap = cap;
  }
  return AR_OK;
}

// Partial sums of one run: [res: iters * bc][upd: iters * bu][f: bf]
static size_t partials_need(const ar_plan_s *p, int iters, bool want_res, bool want_rre,
                            bool precondition) {
  const size_t bc = conv_blocks(p, p->n1, p->n2);
  const size_t bu = precondition ? rows_blocks(p) : axpy_blocks(p);
  const size_t bf = axpy_blocks(p);
  return (want_res ? (size_t)iters * bc : 0) + (want_rre ? (size_t)iters * bu + bf : 0);
}

int ar::iterate_reserve(ar_plan_s *p, int iters) {
  const size_t np = std::max(partials_need(p, iters, true, true, true),
                             partials_need(p, iters, true, true, false));
  return ensure_partials(p, np, 2 * (size_t)iters + 1);
}

namespace {

struct IterArgs {
  const void *g;
  void *x;
  const void *f;
  int iters, tmode, precondition;
  double tau;
  double *res_part, *rre_part, *f_part;
  int bc, bu, bf;
  double *sc;
  bool want_res, want_rre;
};

// The stream-ordered launches of `iters` iterations and the final fixed-order
// reductions of the per-iteration scalars.
int enqueue(ar_plan_s *p, const IterArgs &a, hipStream_t st) {
  int rc = AR_OK;
  if (a.want_rre && (rc = sumsq_launch(p, a.f, a.f_part, nullptr, st)) != AR_OK) return rc;
  const bool fused = a.tmode == AR_REBLUR && conv2_mfma_ok(p);
  for (int k = 0; k < a.iters; ++k) {
    double *rp = a.res_part ? a.res_part + (size_t)k * a.bc : nullptr;
    if (fused) {
      // y = A' (g - A x_k) in one kernel (+ ||r||^2 partials)
      rc = conv2_mfma_launch(p, a.x, a.g, p->y, rp, st);
    } else {
      // r = g - A x_k   (+ ||r||^2 partials), then y = A' r  or  A^T r
      rc = conv_launch(p, a.x, p->r, p->w_fwd, 0, 0, p->n1, p->n2, false, a.g, rp, nullptr, st);
      if (rc == AR_OK && a.tmode == AR_REBLUR) {
        rc = conv_launch(p, p->r, p->y, p->w_rev, 0, 0, p->n1, p->n2, false, nullptr, nullptr,
                         nullptr, st);
      } else if (rc == AR_OK) {
        rc = conv_launch(p, p->r, p->ext, p->w_rev, -p->q1, -p->q2, p->n1 + 2 * p->q1,
                         p->n2 + 2 * p->q2, true, nullptr, nullptr, nullptr, st, true);
        if (rc == AR_OK) rc = fold_launch(p, p->ext, p->y, st);
      }
    }
    if (rc != AR_OK) return rc;
    double *up = a.rre_part ? a.rre_part + (size_t)k * a.bu : nullptr;
    if (a.precondition) {
      // x += tau T diag(d) T~ y
      if ((rc = rows_launch(p, p->y, p->c, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st)) != AR_OK)
        return rc;
      if ((rc = cols_launch(p, p->c, p->c, COL_FWD_D_INV, st)) != AR_OK) return rc;
      if ((rc = rows_launch(p, p->c, a.x, ROW_INV_UPDATE, a.tau, a.f, up, nullptr, st)) != AR_OK)
        return rc;
    } else {
      if ((rc = axpy_launch(p, a.x, p->y, a.tau, a.f, up, nullptr, st)) != AR_OK) return rc;
    }
  }
  // sc: [0, iters): ||r_k||^2; [iters, 2 iters): ||x_k - f||^2; [2 iters]: ||f||^2
  if (a.want_res && (rc = reduce_rows_launch(a.res_part, a.iters, a.bc, a.sc, st)) != AR_OK)
    return rc;
  if (a.want_rre) {
    if ((rc = reduce_rows_launch(a.rre_part, a.iters, a.bu, a.sc + a.iters, st)) != AR_OK)
      return rc;
    if ((rc = reduce_rows_launch(a.f_part, 1, a.bf, a.sc + 2 * (size_t)a.iters, st)) != AR_OK)
      return rc;
  }
  return AR_OK;
}

}  // namespace

int ar::iterate_enqueue(ar_plan_s *p, const void *g, void *x, int iters, hipStream_t st) {
  IterArgs a{};
  a.g = g;
  a.x = x;
  a.iters = iters;
  a.tmode = AR_REBLUR;
  a.precondition = 1;
  a.tau = 1.0;
  return enqueue(p, a, st);
}

namespace {

// Checks shared by both iterate entry points.
int check_args(const char *who, ar_plan_t p, const void *g, void *x, int iters, double tau,
               int tmode, const void *f_true, const double *rre_host, const int *best_it_host) {
  const std::string w(who);
  if (!p || !g || !x) return fail(AR_EINVAL, w + ": null argument");
  if (iters < 0) return fail(AR_EINVAL, w + ": iters < 0");
  if (tmode != AR_REBLUR && tmode != AR_ADJOINT) return fail(AR_EINVAL, w + ": unknown tmode");
  if (tmode == AR_ADJOINT && p->bc != AR_BC_ANTIREFLECTIVE)
    return fail(AR_EUNSUPPORTED, w + ": the exact transpose is Anti-Reflective only");
  if (!std::isfinite(tau)) return fail(AR_EINVAL, w + ": tau must be finite");
  if (g == x || (f_true && (f_true == x || f_true == g)))
    return fail(AR_EALIAS, w + ": g, x and f_true must not alias");
  if ((rre_host || best_it_host) && !f_true) return fail(AR_EINVAL, w + ": RRE outputs need f_true");
  return AR_OK;
}

IterArgs make_args(const ar_plan_s *p, const void *g, void *x, int iters, double tau, int tmode,
                   int precondition, const void *f_true, bool want_res, bool want_rre) {
  IterArgs a{};
  a.g = g;
  a.x = x;
  a.iters = iters;
  a.tmode = tmode;
  a.precondition = precondition ? 1 : 0;
  a.tau = tau;
  a.want_res = want_res;
  a.want_rre = want_rre;
  a.f = a.want_rre ? f_true : nullptr;
  a.bc = conv_blocks(p, p->n1, p->n2);
  a.bu = precondition ? rows_blocks(p) : axpy_blocks(p);
  a.bf = axpy_blocks(p);
  return a;
}

// Partial sums laid out from `part`, reduced scalars at `sc` (device).
void place(IterArgs &a, double *part, double *sc) {
  a.res_part = a.want_res ? part : nullptr;
  a.rre_part = a.want_rre ? part + (a.want_res ? (size_t)a.iters * a.bc : 0) : nullptr;
  a.f_part = a.want_rre ? a.rre_part + (size_t)a.iters * a.bu : nullptr;
  a.sc = sc;
}

}  // namespace

extern "C" int ar_deblur_iterate(ar_plan_t p, const void *g, void *x, int iters, double tau,
                                 int tmode, int precondition, const void *f_true,
                                 double *resnorm_host, double *rre_host, int *best_it_host,
                                 void *stream) {
  int rc = check_args("ar_deblur_iterate", p, g, x, iters, tau, tmode, f_true, rre_host,
                      best_it_host);
  if (rc != AR_OK) return rc;
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (best_it_host) *best_it_host = 0;
  if (iters == 0) return AR_OK;

  IterArgs a = make_args(p, g, x, iters, tau, tmode, precondition, f_true,
                         resnorm_host != nullptr,
                         f_true != nullptr && (rre_host != nullptr || best_it_host != nullptr));
  const size_t need_p = partials_need(p, iters, a.want_res, a.want_rre, a.precondition != 0);
  const size_t need_s = 2 * (size_t)iters + 1;
  if (a.want_res || a.want_rre) {
    rc = ensure_partials(p, need_p, need_s);
    if (rc != AR_OK) return rc;
  }
  place(a, p->partials, p->scalars);

  rc = enqueue(p, a, st);
  if (rc != AR_OK) return rc;
  if (!(a.want_res || a.want_rre)) return AR_OK;
  double *sc = p->scalars;
  std::vector<double> h(2 * (size_t)iters + 1, 0.0);
  AR_HIP(hipMemcpyAsync(h.data(), sc, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  AR_HIP(hipStreamSynchronize(st));
  bool finite = true;
  if (a.want_res) {
    for (int k = 0; k < iters; ++k) {
      resnorm_host[k] = std::sqrt(h[k]);
      if (!std::isfinite(resnorm_host[k])) finite = false;
    }
  }
  if (a.want_rre) {
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

// ---------------------------------------------------------------------------
// Allocation-free variant.  Its per-iteration partial sums and reduced
// scalars live in `scratch`, a file-scope device array (each GPU the library
// runs on holds its own copy until the process ends).  In host code the
// array's name is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that address is handed to kernels and copies.  Nothing in the
// array must start at zero (every partial is written by its kernel before
// the fixed-order reductions read it), so calls do not clear it; calls that
// overlap on one GPU share the array and race.

constexpr size_t kScratchDoubles = size_t(1) << 18;  // 2 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
int scratch_address(int device, double **out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(AR_EINVAL, "ar_deblur_iterate_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    AR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[device] = static_cast<double *>(ptr);
  }
  *out = g_scratch_dev[device];
  return AR_OK;
}

}  // namespace

extern "C" int ar_deblur_iterate_noalloc(ar_plan_t p, const void *g, void *x, int iters,
                                         double tau, int tmode, int precondition,
                                         const void *f_true, double *resnorm_host,
                                         double *rre_host, int *best_it_host, void *stream) {
  int rc = check_args("ar_deblur_iterate_noalloc", p, g, x, iters, tau, tmode, f_true, rre_host,
                      best_it_host);
  if (rc != AR_OK) return rc;
  if (best_it_host && !rre_host)
    return fail(AR_EINVAL, "ar_deblur_iterate_noalloc: best_it needs rre_host (the call keeps "
                           "no host buffer of its own)");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (best_it_host) *best_it_host = 0;
  if (iters == 0) return AR_OK;
  IterArgs a = make_args(p, g, x, iters, tau, tmode, precondition, f_true,
                         resnorm_host != nullptr, f_true != nullptr && rre_host != nullptr);
  const bool scalars = a.want_res || a.want_rre;
  const size_t need_p =
      scalars ? partials_need(p, iters, a.want_res, a.want_rre, a.precondition != 0) : 0;
  const size_t need = scalars ? need_p + 2 * (size_t)iters + 1 : 0;
  if (need > kScratchDoubles)
    return fail(AR_EINVAL, "ar_deblur_iterate_noalloc: this run needs " + std::to_string(need) +
                               " doubles of scratch, the static buffer holds " +
                               std::to_string(kScratchDoubles) +
                               " (run fewer iterations per call)");
  double *base = nullptr;
  if ((rc = scratch_address(p->device, &base)) != AR_OK) return rc;
  place(a, base, base + need_p);
  if ((rc = enqueue(p, a, st)) != AR_OK) return rc;
  if (!scalars) return AR_OK;
  // the reduced sums go straight into the caller's arrays
  double fsq = 0.0;
  if (a.want_res)
    AR_HIP(hipMemcpyAsync(resnorm_host, a.sc, (size_t)iters * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  if (a.want_rre) {
    AR_HIP(hipMemcpyAsync(rre_host, a.sc + iters, (size_t)iters * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    AR_HIP(hipMemcpyAsync(&fsq, a.sc + 2 * (size_t)iters, sizeof(double), hipMemcpyDeviceToHost,
                          st));
  }
  AR_HIP(hipStreamSynchronize(st));
  bool finite = true;
  if (a.want_res) {
    for (int k = 0; k < iters; ++k) {
      resnorm_host[k] = std::sqrt(resnorm_host[k]);
      if (!std::isfinite(resnorm_host[k])) finite = false;
    }
  }
  if (a.want_rre) {
    const double fn = std::sqrt(fsq);
    int best = 0;
    double bv = 0.0;
    for (int k = 0; k < iters; ++k) {
      const double e = std::sqrt(rre_host[k]) / fn;
      rre_host[k] = e;
      if (best == 0 || e < bv) {  // first minimiser on ties
        best = k + 1;
        bv = e;
      }
    }
    if (best_it_host) *best_it_host = best;
  }
  if (!finite)
    return fail(AR_ENONFINITE, "ar_deblur_iterate_noalloc: residual norm is not finite");
  return AR_OK;
}
