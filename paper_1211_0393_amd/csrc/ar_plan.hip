// Plan creation (S0-S2 of the path), FP64 spectrum and filter kernels,
// deterministic reductions and small helper kernels (gfx950).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ar_internal.h"

namespace ar {

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();  // clear the sticky non-fatal error state
  return e == hipErrorOutOfMemory ? AR_ENOMEM : AR_EDEVICE;
}

namespace {

// ------------------------------------------------ PSF preparation (device)

// Symmetrized PSF s = (h + flip_1 h + flip_2 h + flip_1 flip_2 h) / 4
// (Theorem 4, eq. (simmetrizzata2d-bis)) and the correlation weights of the
// blur kernels: A uses rot180(H) (convolution written as a correlation),
// A' uses H itself (the PSF rotated by 180 degrees, convolved).
template <typename T>
__global__ void psf_prep_kernel(const double *__restrict__ H, double *__restrict__ S,
                                T *__restrict__ w_fwd, T *__restrict__ w_rev, int q1, int q2) {
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K1 * K2; e += gridDim.x * blockDim.x) {
    const int a = e / K2, b = e - a * K2;  // a = q1 + s1, b = q2 + s2
    const int fa = K1 - 1 - a, fb = K2 - 1 - b;
    S[e] = (H[fa * K2 + fb] + H[fa * K2 + b] + H[a * K2 + fb] + H[a * K2 + b]) * 0.25;
    w_fwd[e] = T(H[fa * K2 + fb]);
    w_rev[e] = T(H[e]);
  }
}

// cos(a x_k) on the eigenvalue grid of an axis of length n.  AR (Theorem 2
// and the extended grid after it): x_0 = x_{n-1} = 0 and x_k = k pi/(n-1)
// otherwise.  Reflective (Sec. 2.1, the DCT-III algebra): x_k = k pi / n.
__device__ __forceinline__ double grid_cos(int a, int k, int n, int bc) {
  if (bc == AR_BC_REFLECTIVE) {
    if (a == 0 || k == 0) return 1.0;
    const long num = ((long)a * k) % (2L * n);  // cos(pi num / n)
    return cospi((double)num / (double)n);
  }
  if (k == 0 || k == n - 1 || a == 0) return 1.0;
  const long period = 2L * (n - 1);
  const long num = ((long)a * k) % period;  // cos(pi num / (n-1))
  return cospi((double)num / (double)(n - 1));
}

// Cq[a][k2] = w_b-weighted sum over b >= 0 of s[a][b] cos(b x_{k2}),
// w_0 = 1, w_b = 2: the inner sum of eq. (funzione_generatrice).
__global__ void symbol_inner_kernel(const double *__restrict__ S, double *__restrict__ Cq,
                                    int q1, int q2, int n2, int bc) {
  const int K2 = 2 * q2 + 1;
  const int total = (q1 + 1) * n2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int a = e / n2, k2 = e - a * n2;
    const double *row = S + (size_t)(q1 + a) * K2 + q2;
    double acc = row[0];
    for (int b = 1; b <= q2; ++b) acc = fma(2.0 * row[b], grid_cos(b, k2, n2, bc), acc);
    Cq[e] = acc;
  }
}

// lambda[k1][k2] = sum_a w_a cos(a x_{k1}) Cq[a][k2]  (FP64)
__global__ void symbol_outer_kernel(const double *__restrict__ Cq, double *__restrict__ lam,
                                    int q1, int n1, int n2, int bc) {
  const size_t total = (size_t)n1 * n2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int k1 = (int)(e / n2), k2 = (int)(e - (size_t)k1 * n2);
    double acc = Cq[k2];
    for (int a = 1; a <= q1; ++a)
      acc = fma(2.0 * grid_cos(a, k1, n1, bc), Cq[(size_t)a * n2 + k2], acc);
    lam[e] = acc;
  }
}

// Periodic BCs: lambda[k1][k2] = sum_s h_s e^{-2 pi i (k1 s1 / n1 + k2 s2 / n2)}
// (the DFT of the PSF itself, Sec. 4), separably: Cp[a][k2] (complex) over
// s2, then the sum over s1; the plan keeps |lambda| (the filters need only
// the modulus).  Angles are reduced exactly in integers.
__device__ __forceinline__ void unit_root(long num, int n, double *c, double *sn) {
  sincospi(-2.0 * (double)(num % n) / (double)n, sn, c);
}

__global__ void psymbol_inner_kernel(const double *__restrict__ H, double *__restrict__ Cp,
                                     int q1, int q2, int n2) {
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1;
  const int total = K1 * n2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int a = e / n2, k2 = e - a * n2;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < K2; ++b) {
      const long s2 = b - q2;
      double c, sn;
      unit_root((long)k2 * (s2 + n2), n2, &c, &sn);
      const double h = H[a * K2 + b];
      re = fma(h, c, re);
      im = fma(h, sn, im);
    }
    Cp[2 * (size_t)e] = re;
    Cp[2 * (size_t)e + 1] = im;
  }
}

__global__ void psymbol_outer_kernel(const double *__restrict__ Cp, double *__restrict__ lam,
                                     int q1, int n1, int n2) {
  const int K1 = 2 * q1 + 1;
  const size_t total = (size_t)n1 * n2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int k1 = (int)(e / n2), k2 = (int)(e - (size_t)k1 * n2);
    double re = 0.0, im = 0.0;
    for (int a = 0; a < K1; ++a) {
      const long s1 = a - q1;
      double c, sn;
      unit_root((long)k1 * (s1 + n1), n1, &c, &sn);
      const double xr = Cp[2 * ((size_t)a * n2 + k2)], xi = Cp[2 * ((size_t)a * n2 + k2) + 1];
      re = fma(c, xr, fma(-sn, xi, re));
      im = fma(c, xi, fma(sn, xr, im));
    }
    lam[e] = sqrt(re * re + im * im);
  }
}

// Eigenvalue filter (Sec. 4, eq. (TikFilter)); FP64 arithmetic, stored in
// FP64 and in the image dtype.
template <typename T>
__global__ void filter_kernel(const double *__restrict__ lam, double *__restrict__ d64,
                              T *__restrict__ d, size_t total, int kind, double param) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const double l = lam[e];
    double v;
    if (kind == AR_FILTER_TIKHONOV) v = 1.0 / (l * l + param);
    else if (kind == AR_FILTER_THRESHOLD) v = fabs(l) >= param ? 1.0 / (l * l) : 1.0;
    else v = 1.0;
    d64[e] = v;
    d[e] = T(v);
  }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

constexpr int kElemBlocks = 1024;

// x += tau * y, with optional FP64 partial sums of (x - f)^2 (plain Landweber update)
template <typename T>
__global__ __launch_bounds__(256) void axpy_kernel(T *__restrict__ x, const T *__restrict__ y,
                                                   T tau, size_t total,
                                                   const T *__restrict__ f,
                                                   double *__restrict__ partial) {
  __shared__ double red[4];
  double ss = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const T xn = x[e] + tau * y[e];
    x[e] = xn;
    if (f) {
      const double df = (double)xn - (double)f[e];
      ss += df * df;
    }
  }
  if (partial) {
    const double s = block_sum(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const T *__restrict__ x, size_t total,
                                                    double *__restrict__ partial) {
  __shared__ double red[4];
  double ss = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const double v = (double)x[e];
    ss += v * v;
  }
  const double s = block_sum(ss, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[r] = sum_c partials[r * cols + c], fixed order (bitwise reproducible)
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double *__restrict__ partials,
                                                          int cols, double *__restrict__ out) {
  __shared__ double red[4];
  const double *row = partials + (size_t)blockIdx.x * cols;
  double s = 0.0;
  for (int c = threadIdx.x; c < cols; c += blockDim.x) s += row[c];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// Batched forms: blockIdx.y selects the job (x = out, y = in, f = aux).
template <typename T>
__global__ __launch_bounds__(256) void axpy_batch_kernel(const XJob *__restrict__ jobs, T tau,
                                                         int kit) {
  __shared__ double red[4];
  const XJob J = jobs[blockIdx.y];
  T *x = static_cast<T *>(J.out);
  const T *y = static_cast<const T *>(J.in);
  const T *f = static_cast<const T *>(J.aux);
  const size_t total = (size_t)J.n1 * J.n2;
  double ss = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const T xn = x[e] + tau * y[e];
    x[e] = xn;
    if (f) {
      const double df = (double)xn - (double)f[e];
      ss += df * df;
    }
  }
  if (J.part) {
    const double s = block_sum(ss, red);
    if (threadIdx.x == 0) J.part[(size_t)kit * J.nblk + blockIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void sumsq_batch_kernel(const XJob *__restrict__ jobs) {
  __shared__ double red[4];
  const XJob J = jobs[blockIdx.y];
  const T *x = static_cast<const T *>(J.in);
  const size_t total = (size_t)J.n1 * J.n2;
  double ss = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const double v = (double)x[e];
    ss += v * v;
  }
  const double s = block_sum(ss, red);
  if (threadIdx.x == 0 && J.part) J.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void reduce_batch_kernel(const RedJob *__restrict__ jobs) {
  __shared__ double red[4];
  const RedJob J = jobs[blockIdx.y];
  const double *row = J.part + (size_t)blockIdx.x * J.nblk;
  double s = 0.0;
  for (int c = threadIdx.x; c < J.nblk; c += blockDim.x) s += row[c];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) J.out[blockIdx.x] = t;
}

int elem_blocks(size_t total) {
  size_t b = (total + 255) / 256;
  if (b > kElemBlocks) b = kElemBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int spectrum_launch(ar_plan_s *p, hipStream_t st) {
  if (p->csize == 8)
    hipLaunchKernelGGL(psf_prep_kernel<double>, dim3(4), dim3(256), 0, st, p->H64, p->S64,
                       static_cast<double *>(p->w_fwd), static_cast<double *>(p->w_rev), p->q1,
                       p->q2);
  else
    hipLaunchKernelGGL(psf_prep_kernel<float>, dim3(4), dim3(256), 0, st, p->H64, p->S64,
                       static_cast<float *>(p->w_fwd), static_cast<float *>(p->w_rev), p->q1,
                       p->q2);
  AR_HIP(hipGetLastError());
  double *Cq = nullptr;
  if (p->bc == AR_BC_PERIODIC) {
    AR_HIP(hipMalloc((void **)&Cq, 2 * (size_t)(2 * p->q1 + 1) * p->n2 * sizeof(double)));
    hipLaunchKernelGGL(psymbol_inner_kernel, dim3(64), dim3(256), 0, st, p->H64, Cq, p->q1,
                       p->q2, p->n2);
    AR_HIP(hipGetLastError());
    hipLaunchKernelGGL(psymbol_outer_kernel, dim3(1024), dim3(256), 0, st, Cq, p->lambda, p->q1,
                       p->n1, p->n2);
  } else {
    AR_HIP(hipMalloc((void **)&Cq, (size_t)(p->q1 + 1) * p->n2 * sizeof(double)));
    hipLaunchKernelGGL(symbol_inner_kernel, dim3(64), dim3(256), 0, st, p->S64, Cq, p->q1,
                       p->q2, p->n2, p->bc);
    AR_HIP(hipGetLastError());
    hipLaunchKernelGGL(symbol_outer_kernel, dim3(1024), dim3(256), 0, st, Cq, p->lambda, p->q1,
                       p->n1, p->n2, p->bc);
  }
  AR_HIP(hipGetLastError());
  AR_HIP(hipStreamSynchronize(st));
  AR_HIP(hipFree(Cq));
  return AR_OK;
}

// dT[j2][j1] = d64[j1][j2] in the storage type: the column pass reads the
// filter of its column as one contiguous row.  32 x 32 tiles through LDS.
template <typename TS>
__global__ __launch_bounds__(256) void filter_transpose_kernel(const double *__restrict__ d64,
                                                               TS *__restrict__ dT, int n1,
                                                               int n2) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int b1 = blockIdx.y * 32, b2 = blockIdx.x * 32;
  for (int r = ty; r < 32; r += 8) {
    const int j1 = b1 + r, j2 = b2 + tx;
    tile[r][tx] = (j1 < n1 && j2 < n2) ? d64[(size_t)j1 * n2 + j2] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j2 = b2 + r, j1 = b1 + tx;
    if (j1 < n1 && j2 < n2) dT[(size_t)j2 * n1 + j1] = TS(tile[tx][r]);
  }
}

int filter_transpose_launch(ar_plan_s *p, hipStream_t st) {
  const dim3 grid((p->n2 + 31) / 32, (p->n1 + 31) / 32);
  if (p->esize == 8)
    hipLaunchKernelGGL(filter_transpose_kernel<double>, grid, dim3(256), 0, st, p->d64,
                       static_cast<double *>(p->dT), p->n1, p->n2);
  else
    hipLaunchKernelGGL(filter_transpose_kernel<float>, grid, dim3(256), 0, st, p->d64,
                       static_cast<float *>(p->dT), p->n1, p->n2);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int filter_launch(ar_plan_s *p, int filter, double param, hipStream_t st) {
  const size_t total = (size_t)p->n1 * p->n2;
  if (p->csize == 8)
    hipLaunchKernelGGL(filter_kernel<double>, dim3(elem_blocks(total)), dim3(256), 0, st,
                       p->lambda, p->d64, static_cast<double *>(p->d), total, filter, param);
  else
    hipLaunchKernelGGL(filter_kernel<float>, dim3(elem_blocks(total)), dim3(256), 0, st,
                       p->lambda, p->d64, static_cast<float *>(p->d), total, filter, param);
  AR_HIP(hipGetLastError());
  p->filter = filter;
  p->filter_param = param;
  return filter_transpose_launch(p, st);
}

int axpy_blocks(const ar_plan_s *p) { return elem_blocks((size_t)p->n1 * p->n2); }

int elem_blocks_n(size_t total) { return elem_blocks(total); }

int axpy_batch_launch(int dtype, const XJob *jobs, int count, int nblk, double tau, int k,
                      hipStream_t st) {
  if (count == 0) return AR_OK;
  const dim3 grid(nblk, count);
  if (dtype == AR_F64)
    hipLaunchKernelGGL(axpy_batch_kernel<double>, grid, dim3(256), 0, st, jobs, tau, k);
  else
    hipLaunchKernelGGL(axpy_batch_kernel<float>, grid, dim3(256), 0, st, jobs, (float)tau, k);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int sumsq_batch_launch(int dtype, const XJob *jobs, int count, int nblk, hipStream_t st) {
  if (count == 0) return AR_OK;
  const dim3 grid(nblk, count);
  if (dtype == AR_F64)
    hipLaunchKernelGGL(sumsq_batch_kernel<double>, grid, dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL(sumsq_batch_kernel<float>, grid, dim3(256), 0, st, jobs);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int reduce_batch_launch(const RedJob *jobs, int count, int rows, hipStream_t st) {
  if (count == 0 || rows == 0) return AR_OK;
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(rows, count), dim3(256), 0, st, jobs);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int axpy_launch(const ar_plan_s *p, void *x, const void *yv, double tau, const void *f_true,
                double *partial, int *nblocks_out, hipStream_t st) {
  const size_t total = (size_t)p->n1 * p->n2;
  const int blocks = elem_blocks(total);
  if (nblocks_out) *nblocks_out = blocks;
  if (p->dtype == AR_F64)
    hipLaunchKernelGGL(axpy_kernel<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<double *>(x), static_cast<const double *>(yv), tau, total,
                       static_cast<const double *>(f_true), partial);
  else
    hipLaunchKernelGGL(axpy_kernel<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<float *>(x), static_cast<const float *>(yv), (float)tau,
                       total, static_cast<const float *>(f_true), partial);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int sumsq_launch(const ar_plan_s *p, const void *x, double *partial, int *nblocks_out,
                 hipStream_t st) {
  const size_t total = (size_t)p->n1 * p->n2;
  const int blocks = elem_blocks(total);
  if (nblocks_out) *nblocks_out = blocks;
  if (p->dtype == AR_F64)
    hipLaunchKernelGGL(sumsq_kernel<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const double *>(x), total, partial);
  else
    hipLaunchKernelGGL(sumsq_kernel<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const float *>(x), total, partial);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

// Direct Tikhonov solve's filter: for a strongly symmetric PSF the AR matrix
// is T diag(lambda) T~ (Theorems 1-2), so (A'A + alpha I)^{-1} A' with
// A' = A is T diag(lambda / (lambda^2 + alpha)) T~ (eq. (TikFilter) applied
// to lambda); the factor is formed and applied in FP64.
template <typename TS>
__global__ __launch_bounds__(256) void tikhonov_scale_kernel(TS *__restrict__ c,
                                                             const double *__restrict__ lam,
                                                             double alpha, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double l = lam[i];
    c[i] = TS((double)c[i] * (l / (l * l + alpha)));
  }
}

int tikhonov_scale_launch(const ar_plan_s *p, void *c, double alpha, hipStream_t st) {
  const size_t n = (size_t)p->n1 * p->n2;
  const int blocks = elem_blocks(n);
  if (p->esize == 8)
    hipLaunchKernelGGL(tikhonov_scale_kernel<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<double *>(c), p->lambda, alpha, n);
  else
    hipLaunchKernelGGL(tikhonov_scale_kernel<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<float *>(c), p->lambda, alpha, n);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

double psf_absmax(const double *H, int taps) {
  double mx = 0.0;
  for (int e = 0; e < taps; ++e) mx = std::max(mx, std::fabs(H[e]));
  return mx;
}

bool psf_strongly_symmetric(const double *H, int q1, int q2) {
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1;
  double mx = 0.0;
  for (int e = 0; e < K1 * K2; ++e) mx = std::max(mx, std::fabs(H[e]));
  const double tol = 1e-14 * mx;
  for (int a = 0; a < K1; ++a)
    for (int b = 0; b < K2; ++b) {
      const double v = H[a * K2 + b];
      if (std::fabs(v - H[(K1 - 1 - a) * K2 + b]) > tol) return false;
      if (std::fabs(v - H[a * K2 + (K2 - 1 - b)]) > tol) return false;
    }
  return true;
}

int reduce_rows_launch(const double *partials, int rows, int cols, double *out, hipStream_t st) {
  if (rows <= 0) return AR_OK;
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(rows), dim3(256), 0, st, partials, cols, out);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

}  // namespace ar

using namespace ar;


static void plan_free(ar_plan_s *p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  void *bufs[] = {p->H64,         p->S64,         p->w_fwd,        p->w_rev,
                  p->lambda,      p->d64,         p->d,            p->r,
                  p->y,           p->c,           p->ext,          p->partials,
                  p->scalars,     p->gains,       p->lscr,         p->mat_fwd_col,
                  p->mat_inv_col, p->mat_fwd_row, p->mat_inv_row,  p->dscr,
                  p->dsplit,      p->dT,          p->mfma_frag_fwd, p->mfma_frag_rev};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  fft_plan_free(p->fft_row);
  fft_plan_free(p->fft_col);
  fft_plan_free(p->fft_row32);
  bc_free(p);
  delete p;
}

extern "C" int ar_plan_create(ar_plan_t *out, int n1, int n2, const double *psf_host, int q1,
                              int q2, int dtype, int device) {
  return ar_plan_create_bc(out, n1, n2, psf_host, q1, q2, dtype, AR_BC_ANTIREFLECTIVE, device);
}

extern "C" int ar_plan_create_bc(ar_plan_t *out, int n1, int n2, const double *psf_host, int q1,
                                 int q2, int dtype, int bc, int device) {
  if (!out) return fail(AR_EINVAL, "ar_plan_create: out is NULL");
  *out = nullptr;
  if (!psf_host) return fail(AR_EINVAL, "ar_plan_create: psf is NULL");
  if (dtype != AR_F32 && dtype != AR_F64 && dtype != AR_F32_ACC64 && dtype != AR_F32_BF16X3)
    return fail(AR_EINVAL, "ar_plan_create: bad dtype");
  if (bc != AR_BC_ANTIREFLECTIVE && bc != AR_BC_REFLECTIVE && bc != AR_BC_PERIODIC)
    return fail(AR_EINVAL, "ar_plan_create: unknown boundary conditions");
  if (bc != AR_BC_ANTIREFLECTIVE && dtype == AR_F32_BF16X3)
    return fail(AR_EUNSUPPORTED, "ar_plan_create: dense BF16x3 transforms are Anti-Reflective only");
  const size_t esize = dtype == AR_F64 ? 8 : 4;
  const size_t csize = (dtype == AR_F32 || dtype == AR_F32_BF16X3) ? 4 : 8;
  if (q1 < 0 || q2 < 0) return fail(AR_ESHAPE, "ar_plan_create: negative PSF half-width");
  if (n1 < 3 || n2 < 3) return fail(AR_ESHAPE, "ar_plan_create: need n1, n2 >= 3");
  if (q1 > n1 - 3 || q2 > n2 - 3)
    return fail(AR_ESHAPE, "ar_plan_create: AR algebra needs q_j <= n_j - 3");
  const int maxlen = bc == AR_BC_ANTIREFLECTIVE ? max_axis_len(csize) : bc_max_axis_len(csize);
  if (n1 > maxlen || n2 > maxlen)
    return fail(AR_ESHAPE, "ar_plan_create: axis longer than the LDS-resident transform supports");
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1, P = K1 * K2;
  double sum = 0.0;
  for (int e = 0; e < P; ++e) {
    const double v = psf_host[e];
    if (!std::isfinite(v) || v < 0.0)
      return fail(AR_EPSF, "ar_plan_create: PSF entries must be finite and nonnegative");
    sum += v;
  }
  if (std::fabs(sum - 1.0) > 1e-12 * P) return fail(AR_EPSF, "ar_plan_create: PSF must sum to 1");
  int ndev = 0;
  AR_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AR_EINVAL, "ar_plan_create: bad device");
  AR_HIP(hipSetDevice(device));

  ar_plan_s *p = new ar_plan_s();
  p->n1 = n1;
  p->n2 = n2;
  p->q1 = q1;
  p->q2 = q2;
  p->q1cap = q1;
  p->q2cap = q2;
  p->dtype = dtype;
  p->device = device;
  p->strong_sym = psf_strongly_symmetric(psf_host, q1, q2);
  p->bc = bc;
  p->esize = esize;
  p->csize = csize;
  const size_t npx = (size_t)n1 * n2;
  const size_t next = (size_t)(n1 + 2 * q1) * (n2 + 2 * q2);
  int rc = AR_OK;
  auto alloc = [&](void **ptr, size_t bytes) -> bool {
    hipError_t e = hipMalloc(ptr, bytes > 0 ? bytes : 8);
    if (e != hipSuccess) {
      rc = hip_fail(e, "hipMalloc");
      return false;
    }
    return true;
  };
  bool ok = alloc((void **)&p->H64, P * sizeof(double)) && alloc((void **)&p->S64, P * sizeof(double)) &&
            alloc(&p->w_fwd, P * p->csize) && alloc(&p->w_rev, P * p->csize) &&
            alloc((void **)&p->lambda, npx * sizeof(double)) &&
            alloc((void **)&p->d64, npx * sizeof(double)) && alloc(&p->d, npx * p->csize) &&
            alloc(&p->dT, npx * p->esize) &&
            alloc(&p->r, npx * p->esize) && alloc(&p->y, npx * p->esize) &&
            alloc(&p->c, bc_coef_elems(bc, n1, n2) * p->esize) &&
            alloc(&p->ext, std::max(next * p->csize, bc_coef_elems(bc, n1, n2) * p->esize));
  if (!ok) {
    plan_free(p);
    return rc;
  }
  hipStream_t st = nullptr;
  hipError_t e = hipMemcpy(p->H64, psf_host, P * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rc = hip_fail(e, "hipMemcpy(psf)");
    plan_free(p);
    return rc;
  }
  const bool ar = bc == AR_BC_ANTIREFLECTIVE;
  if ((rc = spectrum_launch(p, st)) != AR_OK || (rc = filter_launch(p, AR_FILTER_TIKHONOV, 1e-2, st)) != AR_OK ||
      (ar && (rc = fft_plan_build(p->fft_row, n2, csize == 8, st)) != AR_OK) ||
      (ar && (rc = fft_plan_build(p->fft_col, n1, csize == 8, st)) != AR_OK) ||
      (ar && dtype == AR_F32_ACC64 && (rc = fft_plan_build(p->fft_row32, n2, false, st)) != AR_OK) ||
      (!ar && (rc = bc_setup(p, st)) != AR_OK) ||
      (rc = mfma_frag_build(p, psf_absmax(psf_host, P), st)) != AR_OK ||
      (dtype == AR_F32_BF16X3 && (rc = dense_setup(p, st)) != AR_OK)) {
    plan_free(p);
    return rc;
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    rc = hip_fail(e, "plan setup");
    plan_free(p);
    return rc;
  }
  // per-iteration partial sums for runs of up to kReserveIters iterations
  // with every scalar requested, so that such runs allocate nothing
  if ((rc = iterate_reserve(p, kReserveIters)) != AR_OK) {
    plan_free(p);
    return rc;
  }
  *out = p;
  return AR_OK;
}

extern "C" int ar_plan_set_psf(ar_plan_t p, const double *psf_host, int q1, int q2,
                               void *stream) {
  if (!p || !psf_host) return fail(AR_EINVAL, "ar_plan_set_psf: null argument");
  if (q1 < 0 || q2 < 0 || q1 > p->q1cap || q2 > p->q2cap)
    return fail(AR_ESHAPE, "ar_plan_set_psf: half-widths exceed those of the plan's creation");
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1, P = K1 * K2;
  double sum = 0.0;
  for (int e = 0; e < P; ++e) {
    const double v = psf_host[e];
    if (!std::isfinite(v) || v < 0.0)
      return fail(AR_EPSF, "ar_plan_set_psf: PSF entries must be finite and nonnegative");
    sum += v;
  }
  if (std::fabs(sum - 1.0) > 1e-12 * P) return fail(AR_EPSF, "ar_plan_set_psf: PSF must sum to 1");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  AR_HIP(hipStreamSynchronize(st));  // kernels of the old PSF may still read the buffers
  AR_HIP(hipMemcpy(p->H64, psf_host, P * sizeof(double), hipMemcpyHostToDevice));
  p->q1 = q1;
  p->q2 = q2;
  p->strong_sym = psf_strongly_symmetric(psf_host, q1, q2);
  int rc = spectrum_launch(p, st);
  if (rc != AR_OK) return rc;
  if (p->mfma_frag_fwd && (rc = mfma_frag_build(p, psf_absmax(psf_host, P), st)) != AR_OK)
    return rc;
  rc = p->filter == AR_FILTER_GAINS ? gains_filter_launch(p, p->gains, st)
                                    : filter_launch(p, p->filter, p->filter_param, st);
  if (rc != AR_OK) return rc;
  AR_HIP(hipStreamSynchronize(st));
  return AR_OK;
}

extern "C" int ar_plan_destroy(ar_plan_t p) {
  plan_free(p);
  return AR_OK;
}

extern "C" int ar_precond_set(ar_plan_t p, int filter, double param, const float *gains_dev,
                              void *stream) {
  if (!p) return fail(AR_EINVAL, "ar_precond_set: null plan");
  if (filter == AR_FILTER_GAINS) {
    if (!gains_dev) return fail(AR_EINVAL, "ar_precond_set: the gains filter needs gains");
    if (p->bc != AR_BC_ANTIREFLECTIVE)
      return fail(AR_EUNSUPPORTED, "ar_precond_set: the learned filter is Anti-Reflective only");
    AR_HIP(hipSetDevice(p->device));
    return gains_filter_launch(p, gains_dev, static_cast<hipStream_t>(stream));
  }
  if (filter != AR_FILTER_TIKHONOV && filter != AR_FILTER_THRESHOLD && filter != AR_FILTER_IDENTITY)
    return fail(AR_EINVAL, "ar_precond_set: unknown filter");
  if (filter != AR_FILTER_IDENTITY && !(param > 0.0 && std::isfinite(param)))
    return fail(AR_EINVAL, "ar_precond_set: filter parameter must be finite and > 0");
  AR_HIP(hipSetDevice(p->device));
  return filter_launch(p, filter, param, static_cast<hipStream_t>(stream));
}

extern "C" int ar_psf_normalize(double *psf_host, int q1, int q2) {
  if (!psf_host) return fail(AR_EINVAL, "ar_psf_normalize: psf is NULL");
  if (q1 < 0 || q2 < 0) return fail(AR_ESHAPE, "ar_psf_normalize: negative PSF half-width");
  const int P = (2 * q1 + 1) * (2 * q2 + 1);
  double sum = 0.0;
  for (int e = 0; e < P; ++e) {
    const double v = psf_host[e];
    if (!std::isfinite(v) || v < 0.0)
      return fail(AR_EPSF, "ar_psf_normalize: PSF entries must be finite and nonnegative");
    sum += v;
  }
  if (!(sum > 0.0) || !std::isfinite(sum))
    return fail(AR_EPSF, "ar_psf_normalize: PSF sum must be positive and finite");
  for (int e = 0; e < P; ++e) psf_host[e] /= sum;
  return AR_OK;
}

extern "C" int ar_eigenvalues(ar_plan_t p, double *lambda_dev, void *stream) {
  if (!p || !lambda_dev) return fail(AR_EINVAL, "ar_eigenvalues: null argument");
  AR_HIP(hipSetDevice(p->device));
  AR_HIP(hipMemcpyAsync(lambda_dev, p->lambda, (size_t)p->n1 * p->n2 * sizeof(double),
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return AR_OK;
}

extern "C" int ar_filter_values(ar_plan_t p, double *d_dev, void *stream) {
  if (!p || !d_dev) return fail(AR_EINVAL, "ar_filter_values: null argument");
  AR_HIP(hipSetDevice(p->device));
  AR_HIP(hipMemcpyAsync(d_dev, p->d64, (size_t)p->n1 * p->n2 * sizeof(double),
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return AR_OK;
}

extern "C" const char *ar_last_error(void) { return ar::g_last_error.c_str(); }

extern "C" const char *ar_version(void) { return "ardeblur 0.1 gfx950"; }
