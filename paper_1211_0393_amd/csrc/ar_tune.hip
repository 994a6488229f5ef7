// Launch tunables and the autotuner of a plan (gfx950).
//
// The autotuner times each candidate setting of the transform tunables
// (FFT form, lanes per sequence, waves per workgroup, CU-exclusive
// workgroups) on short runs of whole iterations with HIP events, and keeps
// the fastest.  Settings change the
// launch geometry or the FFT factorisation only; every setting computes the
// same transform (up to rounding).
#include <cfloat>
#include <vector>

#include "ar_internal.h"

using namespace ar;

static bool tune_valid(int key, int value) {
  switch (key) {
    case AR_TUNE_ROW_WAVES:
    case AR_TUNE_COL_WAVES:
    case AR_TUNE_ROW_LANES:
    case AR_TUNE_COL_LANES:
      return value == 0 || value == 1 || value == 2 || value == 4;
    case AR_TUNE_ROW_EXCL:
    case AR_TUNE_COL_EXCL:
    case AR_TUNE_FUSE:
      return value == 0 || value == 1;
    case AR_TUNE_ROW_ALGO:
    case AR_TUNE_COL_ALGO:
    case AR_TUNE_BLUR:
      return value == 0 || value == 1 || value == 2;
    default:
      return false;
  }
}

extern "C" int ar_plan_tune(ar_plan_t p, int key, int value) {
  if (!p) return fail(AR_EINVAL, "ar_plan_tune: null plan");
  if (!tune_valid(key, value)) return fail(AR_EINVAL, "ar_plan_tune: bad key or value");
  if (p->bc != AR_BC_ANTIREFLECTIVE && key != AR_TUNE_BLUR && key != AR_TUNE_FUSE)
    return fail(AR_EUNSUPPORTED, "ar_plan_tune: transform tunables are Anti-Reflective only");
  if (key == AR_TUNE_BLUR && value == 2 && !p->mfma_frag_fwd)
    return fail(AR_EUNSUPPORTED, "ar_plan_tune: the matrix-core blur needs an FP32 plan created "
                                 "with q1 <= 10 and q2 <= 8");
  p->tune[key] = value;
  return AR_OK;
}

extern "C" int ar_plan_get_tune(ar_plan_t p, int key, int *value) {
  if (!p || !value) return fail(AR_EINVAL, "ar_plan_get_tune: null argument");
  if (key < 0 || key > AR_TUNE_FUSE) return fail(AR_EINVAL, "ar_plan_get_tune: bad key");
  *value = p->tune[key];
  return AR_OK;
}

namespace {

// Average time (us) of `reps` runs of fn after two warm-up runs.
template <typename F>
int time_us(F &&fn, hipStream_t st, int reps, double *us) {
  hipEvent_t a, b;
  AR_HIP(hipEventCreate(&a));
  AR_HIP(hipEventCreate(&b));
  int rc = AR_OK;
  for (int i = 0; i < 2 && rc == AR_OK; ++i) rc = fn();
  if (rc == AR_OK) {
    (void)hipEventRecord(a, st);
    for (int i = 0; i < reps && rc == AR_OK; ++i) rc = fn();
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    *us = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

extern "C" int ar_plan_autotune(ar_plan_t p, double *best_us, void *stream) {
  if (!p) return fail(AR_EINVAL, "ar_plan_autotune: null plan");
  if (p->bc != AR_BC_ANTIREFLECTIVE)
    return fail(AR_EUNSUPPORTED, "ar_plan_autotune: tunables are Anti-Reflective only");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // The unit timed for every candidate is a short run of whole
  // preconditioned iterations: a kernel's speed depends on what ran before
  // it (its input was just written by another kernel, on other XCDs), which
  // a repetition of the kernel on its own does not show.  Inputs are zero
  // images in buffers owned by this call.
  const size_t bytes = (size_t)p->n1 * p->n2 * p->esize;
  void *g = nullptr, *x = nullptr;
  AR_HIP(hipMalloc(&g, bytes));
  hipError_t e = hipMalloc(&x, bytes);
  if (e != hipSuccess) {
    (void)hipFree(g);
    return hip_fail(e, "hipMalloc");
  }
  int rc = AR_OK;
  if ((e = hipMemsetAsync(g, 0, bytes, st)) != hipSuccess ||
      (e = hipMemsetAsync(x, 0, bytes, st)) != hipSuccess)
    rc = hip_fail(e, "hipMemsetAsync");
  const int reps = 4, iters = 3;
  const int waves[3] = {1, 2, 4}, lanes[3] = {1, 2, 4};
  auto run = [&]() { return iterate_enqueue(p, g, x, iters, st); };
  // one axis at a time: (algo, lanes, waves, excl) keys of that axis
  auto tune_axis = [&](int k_algo, int k_lanes, int k_waves, int k_excl, bool rows,
                       double *best) {
    *best = DBL_MAX;
    int ba = 0, bg = 0, bw = 0, bx = 0;
    for (int a = 1; a <= 2 && rc == AR_OK; ++a) {
      p->tune[k_algo] = a;
      if ((rows ? wave_rows_algo(p) : wave_cols_algo(p)) != a) continue;  // form not available
      for (int gl : lanes)
        for (int w : waves)
          for (int xx = 0; xx < 2 && rc == AR_OK; ++xx) {
            p->tune[k_lanes] = gl;
            p->tune[k_waves] = w;
            p->tune[k_excl] = xx;
            double us = 0;
            rc = time_us(run, st, reps, &us);
            if (rc == AR_OK && us < *best) { *best = us; ba = a; bg = gl; bw = w; bx = xx; }
          }
    }
    p->tune[k_algo] = ba;
    p->tune[k_lanes] = bg;
    p->tune[k_waves] = bw;
    p->tune[k_excl] = bx;
    if (*best == DBL_MAX) *best = 0;  // block-wide engine only
  };
  double best_r = 0, best_c = 0;
  if (rc == AR_OK)
    tune_axis(AR_TUNE_ROW_ALGO, AR_TUNE_ROW_LANES, AR_TUNE_ROW_WAVES, AR_TUNE_ROW_EXCL, true,
              &best_r);
  if (rc == AR_OK)
    tune_axis(AR_TUNE_COL_ALGO, AR_TUNE_COL_LANES, AR_TUNE_COL_WAVES, AR_TUNE_COL_EXCL, false,
              &best_c);
  (void)hipStreamSynchronize(st);
  (void)hipFree(g);
  (void)hipFree(x);
  if (rc != AR_OK) return rc;
  if (best_us) *best_us = (best_c > 0 ? best_c : best_r) / iters;
  return AR_OK;
}

extern "C" int ar_iterate_profile(ar_plan_t p, const void *g, const void *x, int tmode,
                                  int precondition, int reps, double *phase_us, void *stream) {
  if (!p || !g || !x || !phase_us) return fail(AR_EINVAL, "ar_iterate_profile: null argument");
  if (reps < 1) return fail(AR_EINVAL, "ar_iterate_profile: reps < 1");
  if (tmode != AR_REBLUR && tmode != AR_ADJOINT)
    return fail(AR_EINVAL, "ar_iterate_profile: unknown tmode");
  if (tmode == AR_ADJOINT && p->bc != AR_BC_ANTIREFLECTIVE)
    return fail(AR_EUNSUPPORTED, "ar_iterate_profile: the exact transpose is Anti-Reflective only");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)p->n1 * p->n2 * p->esize;
  // work on a private copy of x so the caller's iterate is untouched
  void *xw = nullptr;
  AR_HIP(hipMalloc(&xw, bytes));
  AR_HIP(hipMemcpyAsync(xw, x, bytes, hipMemcpyDeviceToDevice, st));
  // the five phases of one iteration; each is timed as `reps` back-to-back
  // launches between two events (its inputs are left in place by one
  // untimed iteration first, and no timed launch overwrites its own input)
  // with the fused residual and reblur, phase 0 is that kernel and phase 1 empty
  const bool fused = tmode == AR_REBLUR && conv2_mfma_ok(p);
  auto phase = [&](int k) -> int {
    switch (k) {
      case 0:
        if (fused) return conv2_mfma_launch(p, xw, g, p->y, nullptr, st);
        return conv_launch(p, xw, p->r, p->w_fwd, 0, 0, p->n1, p->n2, false, g, nullptr, nullptr,
                           st);
      case 1:
        if (fused) return AR_OK;
        if (tmode == AR_REBLUR)
          return conv_launch(p, p->r, p->y, p->w_rev, 0, 0, p->n1, p->n2, false, nullptr,
                             nullptr, nullptr, st);
        else {
          int rc = conv_launch(p, p->r, p->ext, p->w_rev, -p->q1, -p->q2, p->n1 + 2 * p->q1,
                               p->n2 + 2 * p->q2, true, nullptr, nullptr, nullptr, st, true);
          return rc != AR_OK ? rc : fold_launch(p, p->ext, p->y, st);
        }
      case 2:
        return precondition ? rows_launch(p, p->y, p->c, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st)
                            : AR_OK;
      case 3:  // out of place into r (free after the transpose blur); a periodic
               // plan's half spectra need the wider ext buffer
        return precondition ? cols_launch(p, p->c, p->bc == AR_BC_PERIODIC ? p->ext : p->r,
                                          COL_FWD_D_INV, st)
                            : AR_OK;
      default:
        return precondition
                   ? rows_launch(p, p->c, xw, ROW_INV_UPDATE, 1.0, nullptr, nullptr, nullptr, st)
                   : axpy_launch(p, xw, p->y, 1.0, nullptr, nullptr, nullptr, st);
    }
  };
  hipEvent_t ev[2];
  for (auto &e : ev) AR_HIP(hipEventCreate(&e));
  int rc = AR_OK;
  for (int k = 0; k < 5 && rc == AR_OK; ++k) rc = phase(k);  // untimed iteration
  for (int k = 0; k < 5 && rc == AR_OK; ++k) {
    if (k == 3) rc = phase(2);  // c holds the row pass output again
    if (rc != AR_OK) break;
    rc = phase(k);  // warm-up launch
    (void)hipEventRecord(ev[0], st);
    for (int i = 0; i < reps && rc == AR_OK; ++i) rc = phase(k);
    (void)hipEventRecord(ev[1], st);
    (void)hipEventSynchronize(ev[1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    phase_us[k] = 1e3 * ms / reps;
    if (k >= 2 && !precondition && k < 4) phase_us[k] = 0.0;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  (void)hipFree(xw);
  return rc;
}
