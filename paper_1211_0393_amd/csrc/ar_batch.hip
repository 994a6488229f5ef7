// Batched executor: many independent (D-)Landweber problems of uneven
// sizes, each with its own plan (PSF, eigenvalues lambda, filter d), run
// by batched kernels and one HIP graph launch per call (gfx950).
//
// Grouping.  Blur launches are grouped by the PSF column half-width q2 (the
// compile-time tap width of the convolution kernel); a workgroup table maps
// every workgroup of a group launch to (problem, tile), so problems of any
// size share one launch with equal-sized work items.  Transform launches
// are grouped by image shape: problems of one shape share the FFT tables
// and the launch geometry of the group's first plan, one problem per
// blockIdx.y.  Per-problem pointers live in device job tables that the
// kernels read at run time, so the captured graph stays valid when a later
// call passes other images; it is captured again only when the iteration
// count, tau, the transpose, preconditioning, the requested outputs or a
// launch setting change.
//
// Iteration k of the graph (eqs. (LandweberMeth), (DLandweberMeth)):
//   r = g - A x           one launch per q2 group (FP64 partial norms)
//   y = A' r | A^T r      one launch per q2 group (+ one fold launch)
//   c = rows of T~ y      one launch per shape group
//   c = T d T~ (columns)  one launch per shape group
//   x += tau rows of T c  one launch per shape group (FP64 partials of ||x - f||^2)
// (D = I: one batched update launch instead of the three transform launches.)
// The per-problem scalars are reduced in fixed order inside the graph and
// copied to the host once after it.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "ar_internal.h"

using namespace ar;

namespace {

struct ConvGroup {
  int q2 = 0, q1max = 0;
  std::vector<int> probs;         // problem indices
  int ntiles = 0, ntiles_ext = 0;
  size_t smem = 0, smem_ext = 0;
  size_t tiles_off = 0, tiles_ext_off = 0;  // int2 offsets in the tile table
  int job_off = 0;                // first slot of the group in the conv job arrays
};

struct ShapeGroup {
  int n1 = 0, n2 = 0;
  std::vector<int> probs;
  int job_off = 0;                // first slot in the transform job arrays
};

struct GraphKey {
  int iters = -1, tmode = 0, precondition = 0, want_res = 0, want_rre = 0;
  double tau = 0;
  std::vector<int> tunes;
  const void *part = nullptr;
  bool operator==(const GraphKey &o) const {
    return iters == o.iters && tmode == o.tmode && precondition == o.precondition &&
           want_res == o.want_res && want_rre == o.want_rre && tau == o.tau &&
           tunes == o.tunes && part == o.part;
  }
};

constexpr int kElemB = 64;  // workgroups per problem of the batched elementwise kernels

}  // namespace

struct ar_batch_s {
  int count = 0, dtype = AR_F32, device = 0;
  std::vector<ar_plan_t> plans;
  std::vector<int2> q_at_create;  // (q1, q2) of every plan when the batch was built
  std::vector<int> tiles, tiles_x, tiles_ext, tiles_x_ext;  // per problem
  std::vector<ConvGroup> cg;
  std::vector<ShapeGroup> sg;
  int n1max = 0, n2max = 0, qmax = 0;
  int2 *tiles_dev = nullptr;
  // job tables: one device block and its pinned host mirror
  unsigned char *jobs_dev = nullptr, *jobs_host = nullptr;
  size_t jobs_bytes = 0;
  hipEvent_t jobs_done = nullptr;  // the last upload of the mirror has completed
  bool jobs_pending = false;
  size_t off_cres = 0, off_creb = 0, off_cadj = 0, off_fold = 0;  // ConvJob arrays
  size_t off_xfwd = 0, off_xcol = 0, off_xinv = 0, off_xaxpy = 0, off_xf = 0;  // XJob arrays
  size_t off_rres = 0, off_rrre = 0, off_rf = 0;  // RedJob arrays
  // partial sums and reduced scalars
  double *part = nullptr;
  size_t part_cap = 0;
  double *scal = nullptr;
  size_t scal_cap = 0;
  // capture stream and the cached graph
  hipStream_t cs = nullptr;
  hipGraphExec_t exec = nullptr;
  GraphKey key;
};

namespace {

template <typename J>
J *jarr(ar_batch_s *b, size_t off, bool dev) {
  return reinterpret_cast<J *>((dev ? b->jobs_dev : b->jobs_host) + off);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

std::vector<int> tune_snapshot(const ar_batch_s *b) {
  std::vector<int> t;
  for (const auto &g : b->sg) {
    const ar_plan_s *lead = b->plans[g.probs[0]];
    t.insert(t.end(), lead->tune, lead->tune + 8);
  }
  return t;
}

// Per-problem partial layout for one call: [res: iters * tiles][upd: iters * nblk_upd][f: kElemB]
struct PartLayout {
  std::vector<size_t> res, upd, f;
  std::vector<int> nblk_upd;
  size_t total = 0;
};

PartLayout part_layout(const ar_batch_s *b, int iters, bool want_res, bool want_rre,
                       bool precondition) {
  PartLayout L;
  L.res.assign(b->count, 0);
  L.upd.assign(b->count, 0);
  L.f.assign(b->count, 0);
  L.nblk_upd.assign(b->count, 0);
  for (const auto &g : b->sg) {
    const int nb = precondition ? wave_rows_blocks(b->plans[g.probs[0]]) : kElemB;
    for (int i : g.probs) L.nblk_upd[i] = nb;
  }
  size_t o = 0;
  for (int i = 0; i < b->count; ++i) {
    if (want_res) {
      L.res[i] = o;
      o += (size_t)iters * b->tiles[i];
    }
    if (want_rre) {
      L.upd[i] = o;
      o += (size_t)iters * L.nblk_upd[i];
      L.f[i] = o;
      o += kElemB;
    }
  }
  L.total = o;
  return L;
}

int ensure(double **buf, size_t *cap, size_t need) {
  if (need <= *cap) return AR_OK;
  if (*buf) AR_HIP(hipFree(*buf));
  *buf = nullptr;
  *cap = 0;
  AR_HIP(hipMalloc((void **)buf, need * sizeof(double)));
  *cap = need;
  return AR_OK;
}

// Fill the host mirror of every job table for this call.
void fill_jobs(ar_batch_s *b, const void *const *g, void *const *x, const void *const *f,
               const PartLayout &L, bool want_res, bool want_rre, int iters) {
  ConvJob *cres = jarr<ConvJob>(b, b->off_cres, false);
  ConvJob *creb = jarr<ConvJob>(b, b->off_creb, false);
  ConvJob *cadj = jarr<ConvJob>(b, b->off_cadj, false);
  ConvJob *fold = jarr<ConvJob>(b, b->off_fold, false);
  XJob *xfwd = jarr<XJob>(b, b->off_xfwd, false);
  XJob *xcol = jarr<XJob>(b, b->off_xcol, false);
  XJob *xinv = jarr<XJob>(b, b->off_xinv, false);
  XJob *xaxpy = jarr<XJob>(b, b->off_xaxpy, false);
  XJob *xf = jarr<XJob>(b, b->off_xf, false);
  RedJob *rres = jarr<RedJob>(b, b->off_rres, false);
  RedJob *rrre = jarr<RedJob>(b, b->off_rrre, false);
  RedJob *rf = jarr<RedJob>(b, b->off_rf, false);
  const size_t sstride = 2 * (size_t)iters + 1;
  for (const auto &G : b->cg) {
    for (size_t j = 0; j < G.probs.size(); ++j) {
      const int i = G.probs[j];
      const ar_plan_s *p = b->plans[i];
      ConvJob c{};
      c.n1 = p->n1;
      c.n2 = p->n2;
      c.q1 = p->q1;
      c.q2 = p->q2;
      c.tiles_x = b->tiles_x[i];
      c.nblk = b->tiles[i];
      c.in = x[i];
      c.out = p->r;
      c.gsub = g[i];
      c.w = p->w_fwd;
      c.part = want_res ? b->part + L.res[i] : nullptr;
      cres[G.job_off + j] = c;
      c.in = p->r;
      c.out = p->y;
      c.gsub = nullptr;
      c.w = p->w_rev;
      c.part = nullptr;
      creb[G.job_off + j] = c;
      c.out = p->ext;
      c.tiles_x = b->tiles_x_ext[i];
      c.nblk = b->tiles_ext[i];
      cadj[G.job_off + j] = c;
    }
  }
  for (int i = 0; i < b->count; ++i) {
    const ar_plan_s *p = b->plans[i];
    ConvJob c{};
    c.n1 = p->n1;
    c.n2 = p->n2;
    c.q1 = p->q1;
    c.q2 = p->q2;
    c.in = p->ext;
    c.out = p->y;
    fold[i] = c;
    XJob a{};
    a.n1 = p->n1;
    a.n2 = p->n2;
    a.in = p->y;
    a.out = x[i];
    a.aux = want_rre ? f[i] : nullptr;
    a.part = want_rre ? b->part + L.upd[i] : nullptr;
    a.nblk = kElemB;
    xaxpy[i] = a;
    XJob s{};
    s.n1 = p->n1;
    s.n2 = p->n2;
    s.in = want_rre ? f[i] : nullptr;
    s.part = want_rre ? b->part + L.f[i] : nullptr;
    s.nblk = kElemB;
    xf[i] = s;
    double *sc = b->scal + (size_t)i * sstride;
    rres[i] = RedJob{want_res ? b->part + L.res[i] : nullptr, sc, b->tiles[i], 0};
    rrre[i] = RedJob{want_rre ? b->part + L.upd[i] : nullptr, sc + iters, L.nblk_upd[i], 0};
    rf[i] = RedJob{want_rre ? b->part + L.f[i] : nullptr, sc + 2 * (size_t)iters, kElemB, 0};
  }
  for (const auto &G : b->sg) {
    for (size_t j = 0; j < G.probs.size(); ++j) {
      const int i = G.probs[j];
      const ar_plan_s *p = b->plans[i];
      XJob a{};
      a.n1 = p->n1;
      a.n2 = p->n2;
      a.in = p->y;
      a.out = p->c;
      xfwd[G.job_off + j] = a;
      a.in = p->c;
      a.out = p->c;
      a.aux = p->dT;
      xcol[G.job_off + j] = a;
      a.in = p->c;
      a.out = x[i];
      a.aux = want_rre ? f[i] : nullptr;
      a.part = want_rre ? b->part + L.upd[i] : nullptr;
      a.nblk = L.nblk_upd[i];
      xinv[G.job_off + j] = a;
    }
  }
}

// Upload the host mirror on `st` (the previous upload must have completed
// before the mirror is rewritten: callers wait on jobs_done first).
int upload_jobs(ar_batch_s *b, hipStream_t st) {
  AR_HIP(hipMemcpyAsync(b->jobs_dev, b->jobs_host, b->jobs_bytes, hipMemcpyHostToDevice, st));
  AR_HIP(hipEventRecord(b->jobs_done, st));
  b->jobs_pending = true;
  return AR_OK;
}

int wait_jobs(ar_batch_s *b) {
  if (b->jobs_pending) AR_HIP(hipEventSynchronize(b->jobs_done));
  b->jobs_pending = false;
  return AR_OK;
}

// The launches of `iters` iterations (recorded into the graph).
int record(ar_batch_s *b, int iters, double tau, int tmode, bool precondition, bool want_res,
           bool want_rre, hipStream_t st) {
  int rc = AR_OK;
  const int dt = b->dtype;
  if (want_rre &&
      (rc = sumsq_batch_launch(dt, jarr<XJob>(b, b->off_xf, true), b->count, kElemB, st)) != AR_OK)
    return rc;
  for (int k = 0; k < iters; ++k) {
    for (const auto &G : b->cg) {
      rc = conv_batch_launch(dt, G.q2, jarr<ConvJob>(b, b->off_cres, true) + G.job_off,
                             b->tiles_dev + G.tiles_off, G.ntiles, k, false, G.smem, st);
      if (rc != AR_OK) return rc;
    }
    if (tmode == AR_REBLUR) {
      for (const auto &G : b->cg) {
        rc = conv_batch_launch(dt, G.q2, jarr<ConvJob>(b, b->off_creb, true) + G.job_off,
                               b->tiles_dev + G.tiles_off, G.ntiles, k, false, G.smem, st);
        if (rc != AR_OK) return rc;
      }
    } else {
      for (const auto &G : b->cg) {
        rc = conv_batch_launch(dt, G.q2, jarr<ConvJob>(b, b->off_cadj, true) + G.job_off,
                               b->tiles_dev + G.tiles_ext_off, G.ntiles_ext, k, true, G.smem_ext,
                               st);
        if (rc != AR_OK) return rc;
      }
      rc = fold_batch_launch(dt, jarr<ConvJob>(b, b->off_fold, true), b->count, b->n1max,
                             b->n2max, b->qmax, st);
      if (rc != AR_OK) return rc;
    }
    if (precondition) {
      for (const auto &G : b->sg) {
        const ar_plan_s *lead = b->plans[G.probs[0]];
        const int cnt = (int)G.probs.size();
        rc = wave_rows_launch_batch(lead, jarr<XJob>(b, b->off_xfwd, true) + G.job_off, cnt,
                                    ROW_FWD, 0.0, k, st);
        if (rc != AR_OK) return rc;
        rc = wave_cols_launch_batch(lead, jarr<XJob>(b, b->off_xcol, true) + G.job_off, cnt,
                                    COL_FWD_D_INV, st);
        if (rc != AR_OK) return rc;
        rc = wave_rows_launch_batch(lead, jarr<XJob>(b, b->off_xinv, true) + G.job_off, cnt,
                                    ROW_INV_UPDATE, tau, k, st);
        if (rc != AR_OK) return rc;
      }
    } else {
      rc = axpy_batch_launch(dt, jarr<XJob>(b, b->off_xaxpy, true), b->count, kElemB, tau, k, st);
      if (rc != AR_OK) return rc;
    }
  }
  if (want_res &&
      (rc = reduce_batch_launch(jarr<RedJob>(b, b->off_rres, true), b->count, iters, st)) != AR_OK)
    return rc;
  if (want_rre) {
    if ((rc = reduce_batch_launch(jarr<RedJob>(b, b->off_rrre, true), b->count, iters, st)) !=
        AR_OK)
      return rc;
    if ((rc = reduce_batch_launch(jarr<RedJob>(b, b->off_rf, true), b->count, 1, st)) != AR_OK)
      return rc;
  }
  return AR_OK;
}

int capture(ar_batch_s *b, int iters, double tau, int tmode, bool precondition, bool want_res,
            bool want_rre) {
  if (b->exec) {
    AR_HIP(hipGraphExecDestroy(b->exec));
    b->exec = nullptr;
  }
  AR_HIP(hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed));
  const int rc = record(b, iters, tau, tmode, precondition, want_res, want_rre, b->cs);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cs, &graph);
  if (rc != AR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  const hipError_t e2 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    b->exec = nullptr;
    return hip_fail(e2, "hipGraphInstantiate");
  }
  return AR_OK;
}

void batch_free(ar_batch_s *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  if (b->jobs_done) (void)hipEventDestroy(b->jobs_done);
  if (b->tiles_dev) (void)hipFree(b->tiles_dev);
  if (b->jobs_dev) (void)hipFree(b->jobs_dev);
  if (b->jobs_host) (void)hipHostFree(b->jobs_host);
  if (b->part) (void)hipFree(b->part);
  if (b->scal) (void)hipFree(b->scal);
  delete b;
}

}  // namespace

extern "C" int ar_batch_create(ar_batch_t *out, int count, const ar_plan_t *plans, void *stream) {
  if (!out) return fail(AR_EINVAL, "ar_batch_create: null output");
  *out = nullptr;
  if (!plans || count < 1) return fail(AR_EINVAL, "ar_batch_create: no plans");
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return fail(AR_EINVAL, "ar_batch_create: null plan");
    if (plans[i]->dtype != plans[0]->dtype || plans[i]->device != plans[0]->device)
      return fail(AR_EINVAL, "ar_batch_create: plans differ in dtype or device");
  }
  {
    std::vector<ar_plan_t> s(plans, plans + count);
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end())
      return fail(AR_EINVAL, "ar_batch_create: a plan appears twice");
  }
  if (plans[0]->dtype == AR_F32_BF16X3)
    return fail(AR_EUNSUPPORTED, "ar_batch_create: dense-transform plans are not batched");
  for (int i = 0; i < count; ++i)
    if (plans[i]->bc != AR_BC_ANTIREFLECTIVE)
      return fail(AR_EUNSUPPORTED, "ar_batch_create: batches are Anti-Reflective only");
  for (int i = 0; i < count; ++i)
    if (!wave_rows_ok(plans[i]) || !wave_cols_ok(plans[i]))
      return fail(AR_EUNSUPPORTED, "ar_batch_create: image too large for the batched transform");
  AR_HIP(hipSetDevice(plans[0]->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  ar_batch_s *b = new ar_batch_s();
  b->count = count;
  b->dtype = plans[0]->dtype;
  b->device = plans[0]->device;
  b->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) b->q_at_create.push_back(make_int2(plans[i]->q1, plans[i]->q2));
  b->tiles.resize(count);
  b->tiles_x.resize(count);
  b->tiles_ext.resize(count);
  b->tiles_x_ext.resize(count);
  std::map<int, int> cg_of;                         // q2 -> group
  std::map<std::pair<int, int>, int> sg_of;         // shape -> group
  for (int i = 0; i < count; ++i) {
    const ar_plan_s *p = plans[i];
    b->tiles[i] = conv_tiles(p->n1, p->n2, &b->tiles_x[i]);
    b->tiles_ext[i] = conv_tiles(p->n1 + 2 * p->q1, p->n2 + 2 * p->q2, &b->tiles_x_ext[i]);
    b->n1max = std::max(b->n1max, p->n1);
    b->n2max = std::max(b->n2max, p->n2);
    b->qmax = std::max({b->qmax, p->q1, p->q2});
    auto it = cg_of.find(p->q2);
    if (it == cg_of.end()) {
      it = cg_of.emplace(p->q2, (int)b->cg.size()).first;
      b->cg.emplace_back();
      b->cg.back().q2 = p->q2;
    }
    b->cg[it->second].probs.push_back(i);
    b->cg[it->second].q1max = std::max(b->cg[it->second].q1max, p->q1);
    auto jt = sg_of.find({p->n1, p->n2});
    if (jt == sg_of.end()) {
      jt = sg_of.emplace(std::make_pair(p->n1, p->n2), (int)b->sg.size()).first;
      b->sg.emplace_back();
      b->sg.back().n1 = p->n1;
      b->sg.back().n2 = p->n2;
    }
    b->sg[jt->second].probs.push_back(i);
  }
  // workgroup -> (job, tile) tables, normal and extended grids
  std::vector<int2> tt;
  int off = 0;
  for (auto &G : b->cg) {
    G.job_off = off;
    off += (int)G.probs.size();
    G.tiles_off = tt.size();
    for (size_t j = 0; j < G.probs.size(); ++j)
      for (int t = 0; t < b->tiles[G.probs[j]]; ++t) tt.push_back(make_int2((int)j, t));
    G.ntiles = (int)(tt.size() - G.tiles_off);
    G.tiles_ext_off = tt.size();
    for (size_t j = 0; j < G.probs.size(); ++j)
      for (int t = 0; t < b->tiles_ext[G.probs[j]]; ++t) tt.push_back(make_int2((int)j, t));
    G.ntiles_ext = (int)(tt.size() - G.tiles_ext_off);
    G.smem = conv_batch_smem(b->dtype, G.q1max, G.q2);
    G.smem_ext = conv_batch_smem(b->dtype == AR_F32 ? AR_F32 : AR_F64, G.q1max, G.q2);
    if (G.smem > 64 * 1024) {
      batch_free(b);
      return fail(AR_EUNSUPPORTED, "ar_batch_create: PSF too large for the LDS halo tile");
    }
  }
  off = 0;
  for (auto &G : b->sg) {
    G.job_off = off;
    off += (int)G.probs.size();
  }
  // job table layout
  size_t o = 0;
  auto take = [&](size_t &dst, size_t bytes) {
    o = align_up(o, 64);
    dst = o;
    o += bytes;
  };
  const size_t n = (size_t)count;
  take(b->off_cres, n * sizeof(ConvJob));
  take(b->off_creb, n * sizeof(ConvJob));
  take(b->off_cadj, n * sizeof(ConvJob));
  take(b->off_fold, n * sizeof(ConvJob));
  take(b->off_xfwd, n * sizeof(XJob));
  take(b->off_xcol, n * sizeof(XJob));
  take(b->off_xinv, n * sizeof(XJob));
  take(b->off_xaxpy, n * sizeof(XJob));
  take(b->off_xf, n * sizeof(XJob));
  take(b->off_rres, n * sizeof(RedJob));
  take(b->off_rrre, n * sizeof(RedJob));
  take(b->off_rf, n * sizeof(RedJob));
  b->jobs_bytes = align_up(o, 64);
  hipError_t e = hipMalloc((void **)&b->jobs_dev, b->jobs_bytes);
  if (e == hipSuccess) e = hipHostMalloc((void **)&b->jobs_host, b->jobs_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void **)&b->tiles_dev, std::max<size_t>(tt.size(), 1) * sizeof(int2));
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->tiles_dev, tt.data(), tt.size() * sizeof(int2), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->jobs_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "ar_batch_create");
  }
  std::memset(b->jobs_host, 0, b->jobs_bytes);
  *out = b;
  return AR_OK;
}

extern "C" int ar_batch_destroy(ar_batch_t b) {
  if (!b) return AR_OK;
  AR_HIP(hipSetDevice(b->device));
  (void)hipDeviceSynchronize();
  batch_free(b);
  return AR_OK;
}

extern "C" int ar_batch_iterate(ar_batch_t b, const void *const *g, void *const *x, int iters,
                                double tau, int tmode, int precondition,
                                const void *const *f_true, double *resnorm_host,
                                double *rre_host, int *best_it_host, void *stream) {
  if (!b || !g || !x) return fail(AR_EINVAL, "ar_batch_iterate: null argument");
  if (iters < 0) return fail(AR_EINVAL, "ar_batch_iterate: iters < 0");
  if (tmode != AR_REBLUR && tmode != AR_ADJOINT)
    return fail(AR_EINVAL, "ar_batch_iterate: unknown tmode");
  if (!std::isfinite(tau)) return fail(AR_EINVAL, "ar_batch_iterate: tau must be finite");
  if ((rre_host || best_it_host) && !f_true)
    return fail(AR_EINVAL, "ar_batch_iterate: RRE outputs need f_true");
  for (int i = 0; i < b->count; ++i) {
    if (!g[i] || !x[i] || (f_true && !f_true[i]))
      return fail(AR_EINVAL, "ar_batch_iterate: null image pointer");
    if (g[i] == x[i] || (f_true && (f_true[i] == x[i] || f_true[i] == g[i])))
      return fail(AR_EALIAS, "ar_batch_iterate: g, x and f_true must not alias");
    // the blur groups, their LDS sizes and the extended-grid tile tables
    // were laid out for the half-widths the plans had at ar_batch_create
    if (b->plans[i]->q1 != b->q_at_create[i].x || b->plans[i]->q2 != b->q_at_create[i].y)
      return fail(AR_ESHAPE, "ar_batch_iterate: a plan's PSF half-widths changed since "
                             "ar_batch_create; re-create the batch");
  }
  AR_HIP(hipSetDevice(b->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (best_it_host)
    for (int i = 0; i < b->count; ++i) best_it_host[i] = 0;
  if (iters == 0) return AR_OK;
  const bool want_res = resnorm_host != nullptr;
  const bool want_rre = f_true != nullptr && (rre_host != nullptr || best_it_host != nullptr);
  const PartLayout L = part_layout(b, iters, want_res, want_rre, precondition != 0);
  int rc = wait_jobs(b);
  if (rc != AR_OK) return rc;
  // (re)allocation of the partials or scalars invalidates the graph: the
  // key holds the partial buffer address, and the scalar buffer is only
  // reached through the job tables
  if ((rc = ensure(&b->part, &b->part_cap, std::max<size_t>(L.total, 1))) != AR_OK) return rc;
  if ((rc = ensure(&b->scal, &b->scal_cap, (size_t)b->count * (2 * (size_t)iters + 1))) != AR_OK)
    return rc;
  fill_jobs(b, g, x, f_true, L, want_res, want_rre, iters);
  if ((rc = upload_jobs(b, st)) != AR_OK) return rc;
  GraphKey k;
  k.iters = iters;
  k.tmode = tmode;
  k.precondition = precondition ? 1 : 0;
  k.want_res = want_res;
  k.want_rre = want_rre;
  k.tau = tau;
  k.tunes = tune_snapshot(b);
  k.part = b->part;
  if (!b->exec || !(k == b->key)) {
    b->key = GraphKey{};
    if ((rc = capture(b, iters, tau, tmode, precondition != 0, want_res, want_rre)) != AR_OK)
      return rc;
    b->key = k;
  }
  AR_HIP(hipGraphLaunch(b->exec, st));
  if (!(want_res || want_rre)) return AR_OK;
  const size_t ss = 2 * (size_t)iters + 1;
  std::vector<double> h((size_t)b->count * ss, 0.0);
  AR_HIP(hipMemcpyAsync(h.data(), b->scal, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  AR_HIP(hipStreamSynchronize(st));
  b->jobs_pending = false;
  bool finite = true;
  for (int i = 0; i < b->count; ++i) {
    const double *hs = h.data() + (size_t)i * ss;
    if (want_res)
      for (int kk = 0; kk < iters; ++kk) {
        resnorm_host[(size_t)i * iters + kk] = std::sqrt(hs[kk]);
        if (!std::isfinite(resnorm_host[(size_t)i * iters + kk])) finite = false;
      }
    if (want_rre) {
      const double fn = std::sqrt(hs[2 * (size_t)iters]);
      int best = 0;
      double bv = 0.0;
      for (int kk = 0; kk < iters; ++kk) {
        const double e = std::sqrt(hs[iters + kk]) / fn;
        if (rre_host) rre_host[(size_t)i * iters + kk] = e;
        if (best == 0 || e < bv) {
          best = kk + 1;
          bv = e;
        }
      }
      if (best_it_host) best_it_host[i] = best;
    }
  }
  if (!finite) return fail(AR_ENONFINITE, "ar_batch_iterate: a residual norm is not finite");
  return AR_OK;
}

namespace {

template <typename F>
int time_batch_us(F &&fn, hipStream_t st, int reps, double *us) {
  hipEvent_t a, c;
  AR_HIP(hipEventCreate(&a));
  AR_HIP(hipEventCreate(&c));
  int rc = AR_OK;
  for (int i = 0; i < 2 && rc == AR_OK; ++i) rc = fn();
  if (rc == AR_OK) {
    (void)hipEventRecord(a, st);
    for (int i = 0; i < reps && rc == AR_OK; ++i) rc = fn();
    (void)hipEventRecord(c, st);
    (void)hipEventSynchronize(c);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, c);
    *us = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(c);
  return rc;
}

}  // namespace

extern "C" int ar_batch_autotune(ar_batch_t b, double *best_us, void *stream) {
  if (!b) return fail(AR_EINVAL, "ar_batch_autotune: null batch");
  AR_HIP(hipSetDevice(b->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = wait_jobs(b);
  if (rc != AR_OK) return rc;
  // job tables of a preconditioner application on the plans' own scratch
  // (y -> c -> c -> r), on zeroed inputs
  for (int i = 0; i < b->count; ++i) {
    const ar_plan_s *p = b->plans[i];
    AR_HIP(hipMemsetAsync(p->y, 0, (size_t)p->n1 * p->n2 * p->esize, st));
  }
  XJob *xfwd = jarr<XJob>(b, b->off_xfwd, false);
  XJob *xcol = jarr<XJob>(b, b->off_xcol, false);
  XJob *xinv = jarr<XJob>(b, b->off_xinv, false);
  for (const auto &G : b->sg)
    for (size_t j = 0; j < G.probs.size(); ++j) {
      const ar_plan_s *p = b->plans[G.probs[j]];
      XJob a{};
      a.n1 = p->n1;
      a.n2 = p->n2;
      a.in = p->y;
      a.out = p->c;
      xfwd[G.job_off + j] = a;
      a.in = p->c;
      a.aux = p->dT;
      xcol[G.job_off + j] = a;
      a.aux = nullptr;
      a.out = p->r;  // inverse rows into r (no update)
      xinv[G.job_off + j] = a;
    }
  if ((rc = upload_jobs(b, st)) != AR_OK) return rc;
  const int reps = 5;
  const int waves[3] = {1, 2, 4};
  double total = 0.0;
  for (const auto &G : b->sg) {
    ar_plan_s *lead = b->plans[G.probs[0]];
    const int cnt = (int)G.probs.size();
    XJob *jf = jarr<XJob>(b, b->off_xfwd, true) + G.job_off;
    XJob *jc = jarr<XJob>(b, b->off_xcol, true) + G.job_off;
    XJob *ji = jarr<XJob>(b, b->off_xinv, true) + G.job_off;
    double best_r = DBL_MAX, best_c = DBL_MAX;
    int br[4] = {0, 0, 0, 0}, bc[4] = {0, 0, 0, 0};
    for (int a = 1; a <= 2; ++a) {
      lead->tune[AR_TUNE_ROW_ALGO] = a;
      lead->tune[AR_TUNE_COL_ALGO] = a;
      const bool row_ok = wave_rows_algo(lead) == a, col_ok = wave_cols_algo(lead) == a;
      for (int gl : {1, 2, 4})
      for (int w : waves)
        for (int xx = 0; xx < 2; ++xx) {
          double us = 0;
          lead->tune[AR_TUNE_ROW_LANES] = gl;
          lead->tune[AR_TUNE_COL_LANES] = gl;
          if (row_ok) {
            lead->tune[AR_TUNE_ROW_WAVES] = w;
            lead->tune[AR_TUNE_ROW_EXCL] = xx;
            rc = time_batch_us(
                [&]() {
                  int r = wave_rows_launch_batch(lead, jf, cnt, ROW_FWD, 0.0, 0, st);
                  return r != AR_OK ? r : wave_rows_launch_batch(lead, ji, cnt, ROW_INV, 0.0, 0, st);
                },
                st, reps, &us);
            if (rc != AR_OK) return rc;
            if (us < best_r) { best_r = us; br[0] = a; br[1] = w; br[2] = xx; br[3] = gl; }
          }
          if (col_ok) {
            lead->tune[AR_TUNE_COL_WAVES] = w;
            lead->tune[AR_TUNE_COL_EXCL] = xx;
            rc = time_batch_us(
                [&]() { return wave_cols_launch_batch(lead, jc, cnt, COL_FWD_D_INV, st); }, st,
                reps, &us);
            if (rc != AR_OK) return rc;
            if (us < best_c) { best_c = us; bc[0] = a; bc[1] = w; bc[2] = xx; bc[3] = gl; }
          }
        }
    }
    for (int i : G.probs) {  // every plan of the group runs as the batch does
      ar_plan_s *p = b->plans[i];
      p->tune[AR_TUNE_ROW_ALGO] = br[0];
      p->tune[AR_TUNE_ROW_WAVES] = br[1];
      p->tune[AR_TUNE_ROW_EXCL] = br[2];
      p->tune[AR_TUNE_COL_ALGO] = bc[0];
      p->tune[AR_TUNE_COL_WAVES] = bc[1];
      p->tune[AR_TUNE_COL_EXCL] = bc[2];
      p->tune[AR_TUNE_ROW_LANES] = br[3];
      p->tune[AR_TUNE_COL_LANES] = bc[3];
    }
    total += (best_r < DBL_MAX ? best_r : 0) + (best_c < DBL_MAX ? best_c : 0);
  }
  AR_HIP(hipStreamSynchronize(st));
  b->jobs_pending = false;
  if (best_us) *best_us = total;
  return AR_OK;
}
