// Launch tunables and the autotuner of a plan (gfx950).
//
// The autotuner times each candidate setting of the transform tunables
// (FFT form, waves per workgroup, CU-exclusive workgroups) on the plan's
// own scratch with HIP events, and keeps the fastest.  Settings change the
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
      return value == 0 || value == 1 || value == 2 || value == 4;
    case AR_TUNE_ROW_EXCL:
    case AR_TUNE_COL_EXCL:
      return value == 0 || value == 1;
    case AR_TUNE_ROW_ALGO:
    case AR_TUNE_COL_ALGO:
    case AR_TUNE_ROW_LANES:
    case AR_TUNE_COL_LANES:
      return value == 0 || value == 1 || value == 2;
    default:
      return false;
  }
}

extern "C" int ar_plan_tune(ar_plan_t p, int key, int value) {
  if (!p) return fail(AR_EINVAL, "ar_plan_tune: null plan");
  if (!tune_valid(key, value)) return fail(AR_EINVAL, "ar_plan_tune: bad key or value");
  p->tune[key] = value;
  return AR_OK;
}

extern "C" int ar_plan_get_tune(ar_plan_t p, int key, int *value) {
  if (!p || !value) return fail(AR_EINVAL, "ar_plan_get_tune: null argument");
  if (key < 0 || key > AR_TUNE_COL_LANES) return fail(AR_EINVAL, "ar_plan_get_tune: bad key");
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
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)p->n1 * p->n2 * p->esize;
  AR_HIP(hipMemsetAsync(p->y, 0, bytes, st));
  const int reps = 5;
  const int waves[3] = {1, 2, 4};
  // rows: forward and inverse pass
  double best_r = DBL_MAX;
  int br_a = 0, br_w = 0, br_x = 0;
  int br_g = 0, bc_g = 0;
  for (int a = 1; a <= 2; ++a) {
    p->tune[AR_TUNE_ROW_ALGO] = a;
    if (wave_rows_algo(p) != a) continue;  // that FFT form is not available here
    for (int gl = 1; gl <= 2; ++gl)
    for (int w : waves)
      for (int x = 0; x < 2; ++x) {
        p->tune[AR_TUNE_ROW_LANES] = gl;
        p->tune[AR_TUNE_ROW_WAVES] = w;
        p->tune[AR_TUNE_ROW_EXCL] = x;
        double us = 0;
        int rc = time_us(
            [&]() {
              int r = rows_launch(p, p->y, p->c, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st);
              return r != AR_OK ? r
                                : rows_launch(p, p->c, p->r, ROW_INV, 0.0, nullptr, nullptr,
                                              nullptr, st);
            },
            st, reps, &us);
        if (rc != AR_OK) return rc;
        if (us < best_r) { best_r = us; br_a = a; br_w = w; br_x = x; br_g = gl; }
      }
  }
  p->tune[AR_TUNE_ROW_ALGO] = br_a;
  p->tune[AR_TUNE_ROW_LANES] = br_g;
  p->tune[AR_TUNE_ROW_WAVES] = br_w;
  p->tune[AR_TUNE_ROW_EXCL] = br_x;
  if (best_r == DBL_MAX) best_r = 0;  // block-wide engine only
  // columns: the fused forward / filter / inverse pass
  double best_c = DBL_MAX;
  int bc_a = 0, bc_w = 0, bc_x = 0;
  for (int a = 1; a <= 2; ++a) {
    p->tune[AR_TUNE_COL_ALGO] = a;
    if (wave_cols_algo(p) != a) continue;
    for (int gl = 1; gl <= 2; ++gl)
    for (int w : waves)
      for (int x = 0; x < 2; ++x) {
        p->tune[AR_TUNE_COL_LANES] = gl;
        p->tune[AR_TUNE_COL_WAVES] = w;
        p->tune[AR_TUNE_COL_EXCL] = x;
        double us = 0;
        int rc = time_us([&]() { return cols_launch(p, p->c, p->c, COL_FWD_D_INV, st); }, st,
                         reps, &us);
        if (rc != AR_OK) return rc;
        if (us < best_c) { best_c = us; bc_a = a; bc_w = w; bc_x = x; bc_g = gl; }
      }
  }
  p->tune[AR_TUNE_COL_ALGO] = bc_a;
  p->tune[AR_TUNE_COL_LANES] = bc_g;
  p->tune[AR_TUNE_COL_WAVES] = bc_w;
  p->tune[AR_TUNE_COL_EXCL] = bc_x;
  if (best_c == DBL_MAX) best_c = 0;
  if (best_us) *best_us = best_r + best_c;
  return AR_OK;
}

extern "C" int ar_iterate_profile(ar_plan_t p, const void *g, const void *x, int tmode,
                                  int precondition, int reps, double *phase_us, void *stream) {
  if (!p || !g || !x || !phase_us) return fail(AR_EINVAL, "ar_iterate_profile: null argument");
  if (reps < 1) return fail(AR_EINVAL, "ar_iterate_profile: reps < 1");
  if (tmode != AR_REBLUR && tmode != AR_ADJOINT)
    return fail(AR_EINVAL, "ar_iterate_profile: unknown tmode");
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
  auto phase = [&](int k) -> int {
    switch (k) {
      case 0:
        return conv_launch(p, xw, p->r, p->w_fwd, 0, 0, p->n1, p->n2, false, g, nullptr, nullptr,
                           st);
      case 1:
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
      case 3:  // out of place into r (free after the transpose blur)
        return precondition ? cols_launch(p, p->c, p->r, COL_FWD_D_INV, st) : AR_OK;
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
