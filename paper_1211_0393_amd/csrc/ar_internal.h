// Internal declarations of the AR deblurring library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <utility>

#include "ardeblur.h"

namespace ar {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define AR_HIP(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return ::ar::hip_fail(e_, #call);       \
  } while (0)

// ------------------------------------------------------- global memory

// Global-memory view of a device pointer.  A kernel whose image pointers
// may come from a job table (batched launches) would otherwise reach them
// through generic (flat) instructions, which also count against the LDS
// wait counter, so every LDS wait would wait for outstanding global loads.
template <typename T> using Gl = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ Gl<T> *gmem(T *p) { return (Gl<T> *)p; }

// ---------------------------------------------------------------- complex

template <typename T> struct V2 { T x, y; };
template <typename T> struct V2Native;
template <> struct V2Native<float> { using type = float2; };
template <> struct V2Native<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ V2<T> cmul(V2<T> a, V2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ V2<T> cadd(V2<T> a, V2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ V2<T> csub(V2<T> a, V2<T> b) { return {a.x - b.x, a.y - b.y}; }

// ---------------------------------------------------------------- FFT plan

constexpr int kMaxStages = 24;

// In-place decimation-in-time plan of the wave-per-sequence engine: stage t
// combines sub-transforms of length L[t] with radix R[t] (largest radix
// first); input goes to digit-reversed positions drev[n]; stage twiddles
// e^{-2 pi i k r / (L R)} sit at tw + tw_off[t] + (r - 1) * L[t] + k.
// Either the FFT of length N = M itself (mixed radix, every radix with a
// codelet) or Bluestein's chirp-z form: the length-M DFT as a cyclic
// convolution of power-of-two length N >= 2M - 1 (forward DIT FFT, product
// with the precomputed spectrum bhat of the chirp, inverse via a DIF FFT of
// the conjugate), chirp[j] = e^{-i pi j^2 / M}.
struct WavePlan {
  bool ok = false, bs = false;
  int M = 0, N = 0, nst = 0, twn = 0;
  int R[kMaxStages] = {};
  int L[kMaxStages] = {};
  int tw_off[kMaxStages] = {};
  void *tw = nullptr;     // V2<T>[twn]
  int *drev = nullptr;    // int[N]
  void *chirp = nullptr;  // V2<T>[M]   (Bluestein)
  void *bhat = nullptr;   // V2<T>[N]   (Bluestein; includes 1/N)
};

struct WDesc {
  int M, N, bs, nst, twn;  // twn: total number of twiddles over all stages
  int R[kMaxStages];
  int L[kMaxStages];
  int tw_off[kMaxStages];
};

// Complex FFT of length M = m - 1 used for the DST-I of length m - 2 along
// one image axis of length m.  Stage s has radix radix[s]; ns[s] is the
// product of the radices before it (Stockham stride).  Twiddles are stored
// per stage as e^{-2 pi i k r / (ns R)} at tw + tw_off[s] + k * R + r.
// A radix that has no compiled codelet is run as a generic stage whose
// roots e^{-2 pi i t / R} sit at gen + gen_off[s].
struct FftPlan {
  int m = 0, M = 0, nstages = 0;
  int radix[kMaxStages] = {};
  int ns[kMaxStages] = {};
  int tw_off[kMaxStages] = {};
  int gen_off[kMaxStages] = {};
  void *tw = nullptr;    // V2<T>[]
  void *gen = nullptr;   // V2<T>[]
  void *post = nullptr;  // V2<T>[M+1]: (cos, sin)(pi k / M)
  size_t tw_count = 0, gen_count = 0;
  WavePlan w;            // wave-per-sequence engine, mixed radix (every radix has a codelet)
  WavePlan wb;           // wave-per-sequence engine, Bluestein (any length)
};

// Device-side view passed to kernels by value.
struct FftDesc {
  int M, nstages;
  int radix[kMaxStages];
  int ns[kMaxStages];
  int tw_off[kMaxStages];
  int gen_off[kMaxStages];
};

bool radix_has_codelet(int r);

}  // namespace ar

// ---------------------------------------------------------------- the plan

struct ar_plan_s {
  int n1 = 0, n2 = 0, q1 = 0, q2 = 0, dtype = AR_F32, device = 0;
  size_t esize = 4;          // bytes per image element (storage type)
  size_t csize = 4;          // bytes per element of the compute type
  // device PSF data
  double *H64 = nullptr;     // (2q1+1)(2q2+1) FP64 PSF as given
  double *S64 = nullptr;     // symmetrized PSF, FP64
  void *w_fwd = nullptr;     // correlation weights of A: rot180(H), compute type
  void *w_rev = nullptr;     // weights of A' and of A^T's correlation: H, compute type
  double *lambda = nullptr;  // n1*n2 FP64 eigenvalues
  double *d64 = nullptr;     // n1*n2 FP64 filter
  void *d = nullptr;         // n1*n2 filter in the compute type
  void *dT = nullptr;        // the filter transposed (n2 x n1) in the storage type
  ar::FftPlan fft_row;       // axis i2, length n2
  ar::FftPlan fft_col;       // axis i1, length n1
  // FP32 tables of axis i2 for AR_F32_ACC64 plans: the iteration's fused
  // inverse row pass and update run in FP32 arithmetic (after the filter)
  ar::FftPlan fft_row32;
  // scratch owned by the plan
  void *r = nullptr, *y = nullptr, *c = nullptr;  // n1*n2 dtype each
  void *ext = nullptr;       // (n1+2q1)(n2+2q2) compute type, adjoint correlation
  double *partials = nullptr;  // per-iteration partial sums
  size_t partials_cap = 0;     // doubles
  double *scalars = nullptr;   // reduced per-iteration scalars
  size_t scalars_cap = 0;
  int filter = AR_FILTER_TIKHONOV;
  double filter_param = 1e-2;
  // launch tunables (0 = automatic), set by ar_plan_tune / ar_plan_autotune
  int tune[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // dense transform matrices of AR_F32_BF16X3 as BF16 hi / lo planes (m
  // rows of m padded to a multiple of 32): T~_{n1}, T_{n1}, T~_{n2}, T_{n2};
  // an FP32 n1 x n2 scratch and the planes of one image operand
  void *mat_fwd_col = nullptr, *mat_inv_col = nullptr;
  void *mat_fwd_row = nullptr, *mat_inv_row = nullptr;
  void *dscr = nullptr, *dsplit = nullptr;
  int q1cap = 0, q2cap = 0;    // half-widths the PSF buffers were sized for
  bool strong_sym = false;     // h_{|s1|,|s2|} = h_{s1,s2} (then P(s) = A and the
                               // eigenvalues lambda are those of A itself)
  // boundary conditions (ar_bc); Reflective and Periodic plans run their
  // preconditioner through FFT plans of length n and the DCT twiddles
  // e^{-i pi k/(2n)} (compute type) of each axis
  int bc = AR_BC_ANTIREFLECTIVE;
  // matrix-core blur of FP32 plans: FP16 hi/lo weight fragments of A and A'
  // (scaled by 2^mfma_ew), built per PSF when q1 <= 10 and q2 <= 8
  void *mfma_frag_fwd = nullptr, *mfma_frag_rev = nullptr;
  int mfma_ew = 0;
  ar::FftPlan bc_fft_row, bc_fft_col;
  void *bc_e2_row = nullptr, *bc_e2_col = nullptr;
  float *gains = nullptr;      // last gains of AR_FILTER_GAINS (64 floats)
  void *lscr = nullptr;        // scratch of the learned-filter kernels
};

namespace ar {

// ---------------------------------------------------------------- batches

// One problem of a batched convolution launch (device array).  The blur
// reads `in` (n1 x n2), writes `out` (n1 x n2, or the (n1+2q1) x (n2+2q2)
// extended grid in the compute type for the adjoint's correlation), with
// correlation weights `w` ((2q1+1) x (2q2+1), compute type); `gsub` makes
// it write gsub - A in and FP64 partial norms to part[k * nblk + tile].
struct ConvJob {
  const void *in;
  void *out;
  const void *gsub;
  const void *w;
  double *part;
  int n1, n2, q1, q2;
  int tiles_x, nblk;
};

// One problem of a batched transform / update launch (device array),
// indexed by blockIdx.y: `aux` is d (column pass), f_true (row update) or
// nothing; partial sums go to part[k * nblk + blockIdx.x].
struct XJob {
  const void *in;
  void *out;
  const void *aux;
  double *part;
  int n1, n2, nblk, pad;
};

// Fixed-order sums of rows of per-problem partials: out[r] = sum_c part[r * nblk + c]
struct RedJob {
  const double *part;
  double *out;
  int nblk, pad;
};

// ---------------------------------------------------------------- launchers

// blur kernels (ar_blur.hip)
// out_compute: write the output in the compute type (extended-grid
// intermediate of A^T) instead of the storage type.
int conv_launch(const ar_plan_s *p, const void *in, void *out, const void *w, int o1, int o2,
                int m1, int m2, bool zero_ext, const void *g_minus, double *partial,
                int *nblocks_out, hipStream_t st, bool out_compute = false);
int conv_blocks(const ar_plan_s *p, int m1, int m2);
int fold_launch(const ar_plan_s *p, const void *ext, void *out, hipStream_t st);
// batched blur: every job shares dtype and q2 (the compile-time tap width);
// tiles[b] = (job, tile of that job) for workgroup b; k selects the partials
// of iteration k; ext_mode: correlation onto the zero-extended grid (A^T).
size_t conv_batch_smem(int dtype, int q1max, int q2);
int conv_batch_launch(int dtype, int q2, const ConvJob *jobs, const int2 *tiles, int ntiles, int k,
                      bool ext_mode, size_t smem, hipStream_t st);
int conv_tiles(int m1, int m2, int *tiles_x);
// matrix-core blur of FP32 plans (ar_blur_mfma.hip): FP16x3 products on
// v_mfma_f32_16x16x32_f16; `reverse` selects A' (weights H) over A
constexpr int kMfmaMaxQ1 = 10, kMfmaMaxQ2 = 8;
bool conv_mfma_ok(const ar_plan_s *p);
int conv_mfma_blocks(int m1, int m2);
int mfma_frag_build(ar_plan_s *p, double hmax, hipStream_t st);
int conv_mfma_launch(const ar_plan_s *p, const void *in, void *out, bool reverse,
                     const void *gsub, double *partial, hipStream_t st);
// the residual and the reblur in one matrix-core kernel: y = A' (g - A x)
// with the ||r||^2 partials of conv_mfma_blocks tiles (AR / Reflective plans)
bool conv2_mfma_ok(const ar_plan_s *p);
int conv2_mfma_launch(const ar_plan_s *p, const void *x, const void *g, void *y, double *partial,
                      hipStream_t st);
// batched fold of the extended-grid correlation (in = ext, out = y)
int fold_batch_launch(int dtype, const ConvJob *jobs, int count, int n1max, int n2max,
                      int qmax, hipStream_t st);

// transform kernels (ar_fft.hip)
enum RowMode { ROW_FWD = 0, ROW_INV = 1, ROW_INV_UPDATE = 2 };
enum ColMode { COL_FWD = 0, COL_INV = 1, COL_FWD_D_INV = 2 };
int fft_plan_build(ar::FftPlan &fp, int m, bool cdouble, hipStream_t st);
// longest axis the LDS-resident transform supports for a compute type size
int max_axis_len(size_t csize);
void fft_plan_free(ar::FftPlan &fp);
int rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                const void *f_true, double *partial, int *nblocks_out, hipStream_t st);
int rows_blocks(const ar_plan_s *p);
int cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st);

// wave-per-sequence transform engine (ar_xform.hip)
int wave_plan_build(WavePlan &w, int M, bool cdouble, bool bluestein, hipStream_t st);
void wave_plan_free(WavePlan &w);
bool wave_rows_ok(const ar_plan_s *p);
bool wave_cols_ok(const ar_plan_s *p);
int wave_rows_blocks(const ar_plan_s *p);
// FFT form the wave engine uses for that axis: 1 mixed radix, 2 Bluestein,
// 0 none (the block-wide engine runs instead)
int wave_rows_algo(const ar_plan_s *p);
int wave_cols_algo(const ar_plan_s *p);
int wave_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                     const void *f_true, double *partial, hipStream_t st);
int wave_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st);
// batched forms: `count` problems of the leader's shape and dtype, one per
// blockIdx.y, with the leader's tables and launch settings
int wave_rows_launch_batch(const ar_plan_s *lead, const XJob *jobs, int count, int mode,
                           double tau, int k, hipStream_t st);
int wave_cols_launch_batch(const ar_plan_s *lead, const XJob *jobs, int count, int mode,
                           hipStream_t st);

// length-1024 passes with two or four wavefronts per sequence (ar_x1023.hip):
// storage / compute element sizes ts / cs, W sequences per workgroup (at
// most x1023_cap(G)), smem bytes of dynamic LDS (>= x1023_lds(W, cs)); the
// plan's stage twiddles and post-processing table of that axis
size_t x1023_lds(int W, size_t csize);
int x1023_cap(int G);
// Paired row pass (two rows per complex FFT; W rows per workgroup, W even,
// G = 4 wavefronts per pair; FP64 arithmetic, cs = 8); smem >=
// x1023_pair_lds(W / 2, cs)
size_t x1023_pair_lds(int P, size_t csize);
// Paired column pass (two adjacent columns per complex FFT, W in {2, 4}
// columns per workgroup dividing n2, four wavefronts per pair; FP64
// arithmetic); smem >= x1023_pair_lds(W / 2, cs)
int x1023_cols_pair_launch(size_t ts, size_t cs, const void *in, void *out, int n2, int W,
                           size_t smem, int mode, const void *tw, const void *post, double alpha,
                           double scale, const void *dT, hipStream_t st);
int x1023_rows_pair_launch(size_t ts, size_t cs, const void *in, void *out, int n1, int W, int G,
                           size_t smem, int mode, const void *tw, const void *post, double alpha,
                           double scale, double tau, const void *f_true, double *partial,
                           hipStream_t st);
int x1023_rows_launch(size_t ts, size_t cs, const void *in, void *out, int n1, int W, int G,
                      size_t smem, int mode, const void *tw, const void *post, double alpha,
                      double scale, double tau, const void *f_true, double *partial,
                      const XJob *jobs, int count, int kit, hipStream_t st);
int x1023_cols_launch(size_t ts, size_t cs, const void *in, void *out, int n2, int W, int G,
                      size_t smem, int mode, const void *tw, const void *post, double alpha,
                      double scale, const void *dT, const XJob *jobs, int count, hipStream_t st);

// Reflective (DCT) and Periodic (DFT) preconditioner passes (ar_bc.hip);
// the row and column passes take the modes of the AR passes (a periodic
// plan's column pass only COL_FWD_D_INV, its coefficients being the
// complex half spectra of the rows, bc_coef_elems storage elements)
int bc_setup(ar_plan_s *p, hipStream_t st);
void bc_free(ar_plan_s *p);
int bc_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                   const void *f_true, double *partial, hipStream_t st);
int bc_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st);
int bc_rows_blocks(const ar_plan_s *p);
size_t bc_coef_elems(int bc, int n1, int n2);
int bc_max_axis_len(size_t csize);

// dense BF16x3 MFMA transforms of AR_F32_BF16X3 plans (ar_dense.hip)
int dense_setup(ar_plan_s *p, hipStream_t st);
int dense_blocks(const ar_plan_s *p);
int dense_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                      const void *f_true, double *partial, hipStream_t st);
int dense_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st);

// plan-time and helper kernels (ar_plan.hip)
int spectrum_launch(ar_plan_s *p, hipStream_t st);
int filter_launch(ar_plan_s *p, int filter, double param, hipStream_t st);
// learned-filter kernels (ar_learned.hip)
int gains_filter_launch(ar_plan_s *p, const float *gains, hipStream_t st);
// dT <- transpose of d64 in the storage type (after every filter update)
int filter_transpose_launch(ar_plan_s *p, hipStream_t st);
// `iters` preconditioned reblur iterations on the stream, no scalars (the
// autotuner's unit of work)
int iterate_enqueue(ar_plan_s *p, const void *g, void *x, int iters, hipStream_t st);
int axpy_launch(const ar_plan_s *p, void *x, const void *yv, double tau, const void *f_true,
                double *partial, int *nblocks_out, hipStream_t st);
int axpy_blocks(const ar_plan_s *p);
int reduce_rows_launch(const double *partials, int rows, int cols, double *out, hipStream_t st);
// c <- c * lambda / (lambda^2 + alpha) elementwise in FP64 (coefficient layout)
int tikhonov_scale_launch(const ar_plan_s *p, void *c, double alpha, hipStream_t st);
// host check of strong symmetry (per-axis flips leave H unchanged to 1e-14 max|H|)
bool psf_strongly_symmetric(const double *H, int q1, int q2);
double psf_absmax(const double *H, int taps);
// size the plan's partial-sum and scalar buffers for runs of `iters`
// iterations with residual norms and RRE requested (ar_iterate.hip)
constexpr int kReserveIters = 128;
int iterate_reserve(ar_plan_s *p, int iters);
int sumsq_launch(const ar_plan_s *p, const void *x, double *partial, int *nblocks_out,
                 hipStream_t st);
// batched elementwise kernels: grid (nblk, count); x = job.out, y = job.in,
// f = job.aux
int axpy_batch_launch(int dtype, const XJob *jobs, int count, int nblk, double tau, int k,
                      hipStream_t st);
int sumsq_batch_launch(int dtype, const XJob *jobs, int count, int nblk, hipStream_t st);
int reduce_batch_launch(const RedJob *jobs, int count, int rows, hipStream_t st);
int elem_blocks_n(size_t total);

}  // namespace ar
