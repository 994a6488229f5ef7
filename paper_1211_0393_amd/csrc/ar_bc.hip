// Transform passes of the preconditioner under the boundary conditions the
// paper compares against (gfx950):
//   * Reflective BCs (Sec. 2.1): for a strongly symmetric PSF the blur lies in
//     the DCT-III algebra, A = R diag(lambda) R^T with R of eq. (Rn) (read as
//     the orthogonal matrix whose transpose is the orthonormal DCT-II); the
//     preconditioner is D = R diag(d) R^T.  Per axis of length N the DCT-II
//     comes from one complex FFT of length N of the even/odd reordering
//     v_t = y_{2t}, v_{N-1-t} = y_{2t+1}:  X_k = Re(e^{-i pi k/(2N)} V_k),
//     c_k = w_k X_k with w_0 = sqrt(1/N), w_k = sqrt(2/N).  The inverse takes
//     V_k = e^{i pi k/(2N)} (X_k - i X_{N-k}) (X_N = 0) back through one FFT
//     (the inverse DFT as the conjugate of the forward DFT of the conjugate)
//     and undoes the reordering.
//   * Periodic BCs (Sec. 2 and Sec. 4): the blur is two-level circulant,
//     diagonalised by the 2-D DFT, and D = F^{-1} diag(d) F with d real and
//     d(-k) = d(k).  Rows go to their half spectrum (k2 = 0..n2/2, complex,
//     kept in the plan's coefficient buffer), columns of the half spectrum are
//     transformed, filtered and transformed back in one pass, and the row
//     inverse rebuilds the full Hermitian row spectrum.
// Every FFT is the block-wide Stockham transform of length N (any N).  Rows
// of a workgroup are contiguous in LDS; columns are interleaved so that a
// wavefront touches consecutive words.
#include <cmath>

#include "ar_internal.h"
#include "ar_stockham.h"

namespace ar {
namespace {

// ------------------------------------------------------- reflective (DCT)

// position in y of element t of the reordered sequence v
__device__ __forceinline__ int dct_src(int t, int N) {
  return t < (N + 1) / 2 ? 2 * t : 2 * (N - 1 - t) + 1;
}
// element of v that holds y_j
__device__ __forceinline__ int dct_pos(int j, int N) { return (j & 1) ? N - 1 - (j >> 1) : j >> 1; }

template <typename T>
__device__ __forceinline__ T dct_w(int k, int N) {
  return k == 0 ? T(sqrt(1.0 / N)) : T(sqrt(2.0 / N));
}

// conj(V_k) of the inverse: e^{-i pi k/(2N)} (X_k + i X_{N-k})
template <typename T>
__device__ __forceinline__ V2<T> dct_inv_in(T xk, T xnk, V2<T> e) {
  return {e.x * xk - e.y * xnk, e.x * xnk + e.y * xk};
}

template <typename T>
__device__ __forceinline__ double block_sum_bc(double v, double *red) {
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

// Row pass (axis i2, length N = n2), B rows per workgroup.  MODE: ROW_FWD
// (y -> c = DCT-II), ROW_INV (c -> DCT-III c), ROW_INV_UPDATE (x += tau
// DCT-III c, FP64 partials of ||x - f||^2).  e2[k] = e^{-i pi k/(2N)}.
template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void dct_rows_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, int N, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, const V2<T> *__restrict__ e2,
    int B, T tau, const TS *__restrict__ f_true, double *__restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)B * N;
  const int row0 = xcd_remap(blockIdx.x, gridDim.x) * B;
  const Layout L{B, N, 1, false};
  for (int idx = threadIdx.x; idx < B * N; idx += blockDim.x) {
    const int s = idx / N, t = idx - s * N;
    const int r = row0 + s;
    V2<T> u{T(0), T(0)};
    if (r < n1) {
      const TS *row = in + (size_t)r * N;
      if (MODE == ROW_FWD) {
        u.x = T(row[dct_src(t, N)]);
      } else {
        const T xk = T(row[t]) / dct_w<T>(t, N);
        const T xnk = t == 0 ? T(0) : T(row[N - t]) / dct_w<T>(N - t, N);
        u = dct_inv_in<T>(xk, xnk, e2[t]);
      }
    }
    bufA[s * N + t] = u;
  }
  __syncthreads();
  const V2<T> *U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  const T invN = T(1) / T(N);
  double ss = 0.0;
  for (int idx = threadIdx.x; idx < B * N; idx += blockDim.x) {
    const int s = idx / N, j = idx - s * N;
    const int r = row0 + s;
    if (r >= n1) continue;
    const size_t o = (size_t)r * N + j;
    if (MODE == ROW_FWD) {
      const V2<T> v = U[s * N + j], e = e2[j];
      out[o] = TS(dct_w<T>(j, N) * (e.x * v.x - e.y * v.y));
    } else {
      const T val = U[s * N + dct_pos(j, N)].x * invN;
      if (MODE == ROW_INV_UPDATE) {
        const TS xn = TS(T(out[o]) + tau * val);
        out[o] = xn;
        if (f_true) {
          const double df = (double)xn - (double)f_true[o];
          ss += df * df;
        }
      } else {
        out[o] = TS(val);
      }
    }
  }
  if (MODE == ROW_INV_UPDATE && partial) {
    double *red = reinterpret_cast<double *>(smem_raw);
    const double sum = block_sum_bc<T>(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
  }
}

// Column pass (axis i1, length N = n1), C interleaved columns per
// workgroup.  MODE: COL_FWD (DCT-II), COL_INV (DCT-III), COL_FWD_D_INV
// (DCT-II, times d, DCT-III: the orthonormal weights cancel, X' = d X).
template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void dct_cols_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int N, int n2, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, const V2<T> *__restrict__ e2,
    int C, const T *__restrict__ dflt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)C * N;
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * C;
  const Layout L{C, 1, C, true};
  const T invN = T(1) / T(N);
  V2<T> *U = bufA;
  if (MODE != COL_INV) {
    for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
      const int t = idx / C, s = idx - t * C;
      const int c = col0 + s;
      bufA[t * C + s] = {c < n2 ? T(in[(size_t)dct_src(t, N) * n2 + c]) : T(0), T(0)};
    }
    __syncthreads();
    U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
    if (MODE == COL_FWD) {
      for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
        const int k = idx / C, s = idx - k * C;
        const int c = col0 + s;
        if (c >= n2) continue;
        const V2<T> v = U[k * C + s], e = e2[k];
        out[(size_t)k * n2 + c] = TS(dct_w<T>(k, N) * (e.x * v.x - e.y * v.y));
      }
      return;
    }
    // X'_k = d_k X_k into the other buffer as real staging
    V2<T> *other = (U == bufA) ? bufB : bufA;
    T *xs = reinterpret_cast<T *>(other);
    for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
      const int k = idx / C, s = idx - k * C;
      const int c = col0 + s;
      const V2<T> v = U[k * C + s], e = e2[k];
      const T dv = c < n2 ? dflt[(size_t)k * n2 + c] : T(0);
      xs[k * C + s] = dv * (e.x * v.x - e.y * v.y);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
      const int k = idx / C, s = idx - k * C;
      const T xk = xs[k * C + s];
      const T xnk = k == 0 ? T(0) : xs[(N - k) * C + s];
      U[k * C + s] = dct_inv_in<T>(xk, xnk, e2[k]);
    }
    __syncthreads();
    U = fft_run<T>(U, other, fd, tw, gen, L);
  } else {
    for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
      const int k = idx / C, s = idx - k * C;
      const int c = col0 + s;
      V2<T> u{T(0), T(0)};
      if (c < n2) {
        const T xk = T(in[(size_t)k * n2 + c]) / dct_w<T>(k, N);
        const T xnk = k == 0 ? T(0) : T(in[(size_t)(N - k) * n2 + c]) / dct_w<T>(N - k, N);
        u = dct_inv_in<T>(xk, xnk, e2[k]);
      }
      bufA[k * C + s] = u;
    }
    __syncthreads();
    U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  }
  for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
    const int j = idx / C, s = idx - j * C;
    const int c = col0 + s;
    if (c >= n2) continue;
    out[(size_t)j * n2 + c] = TS(U[dct_pos(j, N) * C + s].x * invN);
  }
}

// ------------------------------------------------------------ periodic (DFT)

// Row pass (length N = n2, half spectrum width H = N/2 + 1).  ROW_FWD: real
// rows -> half spectra (complex, stored as TS pairs, row stride 2H);
// ROW_INV / ROW_INV_UPDATE: half spectra -> real rows (Hermitian completion,
// inverse DFT, 1/N), optionally x += tau * result with FP64 partials.
template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void pft_rows_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, int N, int H, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, int B, T tau,
    const TS *__restrict__ f_true, double *__restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)B * N;
  const int row0 = xcd_remap(blockIdx.x, gridDim.x) * B;
  const Layout L{B, N, 1, false};
  for (int idx = threadIdx.x; idx < B * N; idx += blockDim.x) {
    const int s = idx / N, k = idx - s * N;
    const int r = row0 + s;
    V2<T> u{T(0), T(0)};
    if (r < n1) {
      if (MODE == ROW_FWD) {
        u.x = T(in[(size_t)r * N + k]);
      } else {
        // conj(Y_k): Y_k = spectrum[k] for k < H, conj(spectrum[N - k]) above
        const TS *sp = in + (size_t)r * 2 * H;
        if (k < H) u = {T(sp[2 * k]), -T(sp[2 * k + 1])};
        else u = {T(sp[2 * (N - k)]), T(sp[2 * (N - k) + 1])};
      }
    }
    bufA[s * N + k] = u;
  }
  __syncthreads();
  const V2<T> *U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  const T invN = T(1) / T(N);
  double ss = 0.0;
  if (MODE == ROW_FWD) {
    for (int idx = threadIdx.x; idx < B * H; idx += blockDim.x) {
      const int s = idx / H, k = idx - s * H;
      const int r = row0 + s;
      if (r >= n1) continue;
      const V2<T> v = U[s * N + k];
      out[(size_t)r * 2 * H + 2 * k] = TS(v.x);
      out[(size_t)r * 2 * H + 2 * k + 1] = TS(v.y);
    }
    return;
  }
  for (int idx = threadIdx.x; idx < B * N; idx += blockDim.x) {
    const int s = idx / N, t = idx - s * N;
    const int r = row0 + s;
    if (r >= n1) continue;
    const T val = U[s * N + t].x * invN;
    const size_t o = (size_t)r * N + t;
    if (MODE == ROW_INV_UPDATE) {
      const TS xn = TS(T(out[o]) + tau * val);
      out[o] = xn;
      if (f_true) {
        const double df = (double)xn - (double)f_true[o];
        ss += df * df;
      }
    } else {
      out[o] = TS(val);
    }
  }
  if (MODE == ROW_INV_UPDATE && partial) {
    double *red = reinterpret_cast<double *>(smem_raw);
    const double sum = block_sum_bc<T>(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
  }
}

// Column pass over the H complex columns of the half spectra (length N =
// n1): DFT, times the real filter d[k1][k2], inverse DFT (1/N), in place.
template <typename TS, typename T>
__global__ __launch_bounds__(256) void pft_cols_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int N, int H, int n2, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, int C,
    const T *__restrict__ dflt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)C * N;
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * C;
  const Layout L{C, 1, C, true};
  for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
    const int t = idx / C, s = idx - t * C;
    const int c = col0 + s;
    V2<T> u{T(0), T(0)};
    if (c < H) u = {T(in[((size_t)t * H + c) * 2]), T(in[((size_t)t * H + c) * 2 + 1])};
    bufA[t * C + s] = u;
  }
  __syncthreads();
  V2<T> *U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  V2<T> *other = (U == bufA) ? bufB : bufA;
  for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
    const int k = idx / C, s = idx - k * C;
    const int c = col0 + s;
    const T dv = c < H ? dflt[(size_t)k * n2 + c] : T(0);
    const V2<T> v = U[k * C + s];
    U[k * C + s] = {dv * v.x, -dv * v.y};  // conj(d Z_k)
  }
  __syncthreads();
  U = fft_run<T>(U, other, fd, tw, gen, L);
  const T invN = T(1) / T(N);
  for (int idx = threadIdx.x; idx < C * N; idx += blockDim.x) {
    const int t = idx / C, s = idx - t * C;
    const int c = col0 + s;
    if (c >= H) continue;
    const V2<T> v = U[t * C + s];
    out[((size_t)t * H + c) * 2] = TS(v.x * invN);
    out[((size_t)t * H + c) * 2 + 1] = TS(-v.y * invN);
  }
}

// e2[k] = e^{-i pi k / (2N)}, k = 0..N-1 (FP64 arithmetic)
template <typename T>
__global__ void dct_twiddle_kernel(V2<T> *e2, int N) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
    double sv, cv;
    sincospi((double)k / (2.0 * N), &sv, &cv);
    e2[k] = {T(cv), T(-sv)};
  }
}

int bc_half(const ar_plan_s *p) { return p->n2 / 2 + 1; }

template <typename TS, typename T>
int bc_rows_t(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
              const void *f_true, double *partial, hipStream_t st) {
  const FftPlan &fp = p->bc_fft_row;
  const int N = p->n2;
  const int B = rows_per_block(N, sizeof(T));
  const int blocks = (p->n1 + B - 1) / B;
  const size_t smem = seq_lds_bytes(B, N, sizeof(T));
  if (smem > kMaxLds) return fail(AR_EUNSUPPORTED, "row transform exceeds LDS");
  const FftDesc fd = make_desc(fp);
  auto tw = static_cast<const V2<T> *>(fp.tw);
  auto gen = static_cast<const V2<T> *>(fp.gen);
  auto e2 = static_cast<const V2<T> *>(p->bc_e2_row);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  const int H = bc_half(p);
  hipError_t e = hipSuccess;
#define AR_BCROWS(KERNEL, ...)                                                             \
  e = allow_lds(KERNEL, smem);                                                             \
  if (e == hipSuccess) {                                                                   \
    hipLaunchKernelGGL(KERNEL, dim3(blocks), dim3(256), smem, st, __VA_ARGS__);            \
    e = hipGetLastError();                                                                 \
  }
  if (p->bc == AR_BC_REFLECTIVE) {
    switch (mode) {
      case ROW_FWD:
        AR_BCROWS((dct_rows_kernel<TS, T, ROW_FWD>), ti, to, p->n1, N, fd, tw, gen, e2, B,
                  T(tau), tf, partial) break;
      case ROW_INV:
        AR_BCROWS((dct_rows_kernel<TS, T, ROW_INV>), ti, to, p->n1, N, fd, tw, gen, e2, B,
                  T(tau), tf, partial) break;
      default:
        AR_BCROWS((dct_rows_kernel<TS, T, ROW_INV_UPDATE>), ti, to, p->n1, N, fd, tw, gen, e2,
                  B, T(tau), tf, partial) break;
    }
  } else {
    switch (mode) {
      case ROW_FWD:
        AR_BCROWS((pft_rows_kernel<TS, T, ROW_FWD>), ti, to, p->n1, N, H, fd, tw, gen, B,
                  T(tau), tf, partial) break;
      case ROW_INV:
        AR_BCROWS((pft_rows_kernel<TS, T, ROW_INV>), ti, to, p->n1, N, H, fd, tw, gen, B,
                  T(tau), tf, partial) break;
      default:
        AR_BCROWS((pft_rows_kernel<TS, T, ROW_INV_UPDATE>), ti, to, p->n1, N, H, fd, tw, gen, B,
                  T(tau), tf, partial) break;
    }
  }
#undef AR_BCROWS
  if (e != hipSuccess) return hip_fail(e, "boundary-condition row pass launch");
  return AR_OK;
}

template <typename TS, typename T>
int bc_cols_t(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  const FftPlan &fp = p->bc_fft_col;
  const int N = p->n1;
  const int C = cols_per_block(N, sizeof(T));
  const int ncols = p->bc == AR_BC_PERIODIC ? bc_half(p) : p->n2;
  const int blocks = (ncols + C - 1) / C;
  const size_t smem = seq_lds_bytes(C, N, sizeof(T));
  if (smem > kMaxLds) return fail(AR_EUNSUPPORTED, "column transform exceeds LDS");
  const FftDesc fd = make_desc(fp);
  auto tw = static_cast<const V2<T> *>(fp.tw);
  auto gen = static_cast<const V2<T> *>(fp.gen);
  auto e2 = static_cast<const V2<T> *>(p->bc_e2_col);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const T *>(p->d);
  hipError_t e = hipSuccess;
#define AR_BCCOLS(KERNEL, ...)                                                             \
  e = allow_lds(KERNEL, smem);                                                             \
  if (e == hipSuccess) {                                                                   \
    hipLaunchKernelGGL(KERNEL, dim3(blocks), dim3(256), smem, st, __VA_ARGS__);            \
    e = hipGetLastError();                                                                 \
  }
  if (p->bc == AR_BC_REFLECTIVE) {
    switch (mode) {
      case COL_FWD:
        AR_BCCOLS((dct_cols_kernel<TS, T, COL_FWD>), ti, to, N, p->n2, fd, tw, gen, e2, C, td)
        break;
      case COL_INV:
        AR_BCCOLS((dct_cols_kernel<TS, T, COL_INV>), ti, to, N, p->n2, fd, tw, gen, e2, C, td)
        break;
      default:
        AR_BCCOLS((dct_cols_kernel<TS, T, COL_FWD_D_INV>), ti, to, N, p->n2, fd, tw, gen, e2, C,
                  td) break;
    }
  } else {
    if (mode != COL_FWD_D_INV)
      return fail(AR_EUNSUPPORTED, "periodic plans apply the column DFT only inside D");
    AR_BCCOLS((pft_cols_kernel<TS, T>), ti, to, N, bc_half(p), p->n2, fd, tw, gen, C, td)
  }
#undef AR_BCCOLS
  if (e != hipSuccess) return hip_fail(e, "boundary-condition column pass launch");
  return AR_OK;
}

}  // namespace

int bc_rows_blocks(const ar_plan_s *p) {
  const int B = rows_per_block(p->n2, p->csize);
  return (p->n1 + B - 1) / B;
}

size_t bc_coef_elems(int bc, int n1, int n2) {
  return bc == AR_BC_PERIODIC ? (size_t)n1 * 2 * (n2 / 2 + 1) : (size_t)n1 * n2;
}

int bc_max_axis_len(size_t csize) {
  int N = 3;
  while (seq_lds_bytes(1, N + 1, csize) <= kMaxLds) ++N;
  return N;
}

int bc_setup(ar_plan_s *p, hipStream_t st) {
  const bool cd = p->csize == 8;
  // FFT plans of length N = n (fft_plan_build builds length m - 1)
  int rc = fft_plan_build(p->bc_fft_row, p->n2 + 1, cd, st);
  if (rc == AR_OK) rc = fft_plan_build(p->bc_fft_col, p->n1 + 1, cd, st);
  if (rc != AR_OK) return rc;
  const size_t cb = cd ? sizeof(double2) : sizeof(float2);
  AR_HIP(hipMalloc(&p->bc_e2_row, (size_t)p->n2 * cb));
  AR_HIP(hipMalloc(&p->bc_e2_col, (size_t)p->n1 * cb));
  if (cd) {
    hipLaunchKernelGGL(dct_twiddle_kernel<double>, dim3(8), dim3(256), 0, st,
                       static_cast<V2<double> *>(p->bc_e2_row), p->n2);
    hipLaunchKernelGGL(dct_twiddle_kernel<double>, dim3(8), dim3(256), 0, st,
                       static_cast<V2<double> *>(p->bc_e2_col), p->n1);
  } else {
    hipLaunchKernelGGL(dct_twiddle_kernel<float>, dim3(8), dim3(256), 0, st,
                       static_cast<V2<float> *>(p->bc_e2_row), p->n2);
    hipLaunchKernelGGL(dct_twiddle_kernel<float>, dim3(8), dim3(256), 0, st,
                       static_cast<V2<float> *>(p->bc_e2_col), p->n1);
  }
  AR_HIP(hipGetLastError());
  return AR_OK;
}

void bc_free(ar_plan_s *p) {
  fft_plan_free(p->bc_fft_row);
  fft_plan_free(p->bc_fft_col);
  if (p->bc_e2_row) (void)hipFree(p->bc_e2_row);
  if (p->bc_e2_col) (void)hipFree(p->bc_e2_col);
  p->bc_e2_row = p->bc_e2_col = nullptr;
}

int bc_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                   const void *f_true, double *partial, hipStream_t st) {
  if (p->dtype == AR_F64)
    return bc_rows_t<double, double>(p, in, out, mode, tau, f_true, partial, st);
  if (p->dtype == AR_F32_ACC64)
    return bc_rows_t<float, double>(p, in, out, mode, tau, f_true, partial, st);
  return bc_rows_t<float, float>(p, in, out, mode, tau, f_true, partial, st);
}

int bc_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  if (p->dtype == AR_F64) return bc_cols_t<double, double>(p, in, out, mode, st);
  if (p->dtype == AR_F32_ACC64) return bc_cols_t<float, double>(p, in, out, mode, st);
  return bc_cols_t<float, float>(p, in, out, mode, st);
}

}  // namespace ar
