// AR transform kernels (gfx950): T~ = T~_{n1} (x) T~_{n2}, T = its inverse,
// and the preconditioner D = T diag(d) T~ (Theorem 1; Sec. 4).
//
// Per axis of length m the transform is an endpoint scaling plus a DST-I of
// length N = m - 2 applied to the interior after removing (forward) or
// adding back (inverse) the linear ramp y_1 p + y_m J p, p_j = 1 - j/(m-1).
// The DST-I Q_N = sqrt(2/(N+1)) [sin(pi j k /(N+1))] is computed from one
// complex FFT of length M = N + 1 per row: the odd extension z of length 2M
// is packed as u_t = z_{2t} + i z_{2t+1}, U = DFT_M(u), and with
// a + ib = U_k, c + id = U_{M-k}, phi = pi k / M,
//   sum_j x_j sin(pi j k / M) = ((d - b) + cos(phi)(a - c) + sin(phi)(b + d)) / 4.
// The FFT is a mixed-radix Stockham transform held in LDS (ping-pong
// buffers); radices with a compiled codelet use straight-line DFTs with
// compile-time roots, any other prime factor runs as a generic O(R) stage.
//
// Row passes (axis i2, contiguous) keep each row contiguous in LDS.  Column
// passes (axis i1) interleave C columns so that a wavefront touches
// consecutive LDS words and consecutive global addresses.  The column pass
// of D fuses forward transform, filter and inverse transform.
#include <cmath>
#include <vector>

#include "ar_codelets.h"
#include "ar_internal.h"
#include "ar_stockham.h"

namespace ar {
namespace {

using namespace cl;

// u_t = z_{2t} + i z_{2t+1} from the real interior x_1..x_N held in `re`
// (x_j at re[s*rss + j*res], j = 1..N; the endpoints are ignored).  When
// `ramp`, x_j is replaced by x_j - e0 p_j - e1 J p_j with e0 = re[.., 0],
// e1 = re[.., m-1].
template <typename T>
__device__ __forceinline__ T odd_ext(const T *row, int res, int tpos, int M) {
  if (tpos == 0 || tpos == M) return T(0);
  if (tpos < M) return row[tpos * res];
  return -row[(2 * M - tpos) * res];
}

template <typename T>
__device__ void pack_u(const T *__restrict__ re, int rss, int res, V2<T> *__restrict__ u,
                       const Layout L, int M, bool ramp, const T *__restrict__ e0,
                       const T *__restrict__ e1) {
  const int total = M * L.nseq;
  const T invM = T(1) / T(M);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int s, t;
    if (L.seq_fast) {
      t = idx / L.nseq;
      s = idx - t * L.nseq;
    } else {
      s = idx / M;
      t = idx - s * M;
    }
    const T *row = re + s * rss;
    T zr = odd_ext(row, res, 2 * t, M);
    T zi = odd_ext(row, res, 2 * t + 1, M);
    if (ramp) {
      // subtract the ramp from the odd extension: x_j - e0 (M-j)/M - e1 j/M,
      // applied with the sign of the extension (x_{2M-j} enters negated)
      const T a0 = e0[s], a1 = e1[s];
      auto rampv = [&](int tp) -> T {
        if (tp == 0 || tp == M) return T(0);
        const int j = tp < M ? tp : 2 * M - tp;
        const T r = a0 * (T(M - j) * invM) + a1 * (T(j) * invM);
        return tp < M ? r : -r;
      };
      zr -= rampv(2 * t);
      zi -= rampv(2 * t + 1);
    }
    u[s * L.ss + t * L.es] = {zr, zi};
  }
}

// DST value k (1..M-1) of a packed sequence whose DFT is U.
template <typename T>
__device__ __forceinline__ T dst_value(const V2<T> *__restrict__ U, int es, int k, int M,
                                       const V2<T> *__restrict__ post, T scale) {
  const V2<T> A = U[k * es], C = U[(M - k) * es];
  const V2<T> cs = post[k];
  return scale * ((C.y - A.y) + cs.x * (A.x - C.x) + cs.y * (A.y + C.y));
}


// ------------------------------------------------------------- row pass

template <typename T>
__device__ __forceinline__ double block_sum256(double v, double *red) {
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

// MODE: ROW_FWD, ROW_INV, ROW_INV_UPDATE (x += tau * T_{n2}-pass output).
// TS: storage type of the images, T: compute type (LDS, tables, arithmetic).
template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void rows_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, int m, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, const V2<T> *__restrict__ post,
    T alpha, T scale, int B, int Mp, T tau, const TS *__restrict__ f_true,
    double *__restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)B * Mp;
  T *e0 = reinterpret_cast<T *>(bufB + (size_t)B * Mp);
  T *e1 = e0 + B;
  const int M = fd.M;
  const int row0 = xcd_remap(blockIdx.x, gridDim.x) * B;
  const int rs = 2 * Mp;  // real staging stride (in T) inside bufB
  T *re = reinterpret_cast<T *>(bufB);
  for (int idx = threadIdx.x; idx < B * m; idx += blockDim.x) {
    const int s = idx / m, t = idx - s * m;
    const int r = row0 + s;
    re[s * rs + t] = r < n1 ? T(in[(size_t)r * m + t]) : T(0);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < B; s += blockDim.x) {
    e0[s] = re[s * rs];
    e1[s] = re[s * rs + m - 1];
  }
  __syncthreads();
  const Layout L{B, Mp, 1, false};
  pack_u<T>(re, rs, 1, bufA, L, M, MODE == ROW_FWD, e0, e1);
  __syncthreads();
  V2<T> *U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  const T invM = T(1) / T(M);
  double ss = 0.0;
  for (int idx = threadIdx.x; idx < B * m; idx += blockDim.x) {
    const int s = idx / m, t = idx - s * m;
    const int r = row0 + s;
    if (r >= n1) continue;
    T val;
    if (MODE == ROW_FWD) {
      if (t == 0) val = alpha * e0[s];
      else if (t == m - 1) val = alpha * e1[s];
      else val = dst_value<T>(U + s * Mp, 1, t, M, post, scale);
    } else {
      const T y0 = e0[s] / alpha, y1 = e1[s] / alpha;
      if (t == 0) val = y0;
      else if (t == m - 1) val = y1;
      else
        val = dst_value<T>(U + s * Mp, 1, t, M, post, scale) + y0 * (T(M - t) * invM) +
              y1 * (T(t) * invM);
    }
    const size_t o = (size_t)r * m + t;
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
    double *red = reinterpret_cast<double *>(smem_raw);  // FFT buffers are dead now
    const double s = block_sum256<T>(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------- column pass

template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void cols_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int m, int n2, FftDesc fd,
    const V2<T> *__restrict__ tw, const V2<T> *__restrict__ gen, const V2<T> *__restrict__ post,
    T alpha, T scale, int C, const T *__restrict__ dflt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = fd.M;
  const int Mp = M;  // interleaved layout: sequence stride 1, element stride C
  V2<T> *bufA = reinterpret_cast<V2<T> *>(smem_raw);
  V2<T> *bufB = bufA + (size_t)C * Mp;
  T *e0 = reinterpret_cast<T *>(bufB + (size_t)C * Mp);
  T *e1 = e0 + C;
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * C;
  // real staging: element t of column s at re[t * C + s] (fits: C*m <= 2*C*M)
  T *re = reinterpret_cast<T *>(bufB);
  for (int idx = threadIdx.x; idx < C * m; idx += blockDim.x) {
    const int t = idx / C, s = idx - t * C;
    const int c = col0 + s;
    re[t * C + s] = c < n2 ? T(in[(size_t)t * n2 + c]) : T(0);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < C; s += blockDim.x) {
    e0[s] = re[s];
    e1[s] = re[(m - 1) * C + s];
  }
  __syncthreads();
  const Layout L{C, 1, C, true};
  const T invM = T(1) / T(M);
  pack_u<T>(re, 1, C, bufA, L, M, MODE != COL_INV, e0, e1);
  __syncthreads();
  V2<T> *U = fft_run<T>(bufA, bufB, fd, tw, gen, L);
  if (MODE == COL_FWD) {
    for (int idx = threadIdx.x; idx < C * m; idx += blockDim.x) {
      const int t = idx / C, s = idx - t * C;
      const int c = col0 + s;
      if (c >= n2) continue;
      T val;
      if (t == 0) val = alpha * e0[s];
      else if (t == m - 1) val = alpha * e1[s];
      else val = dst_value<T>(U + s, C, t, M, post, scale);
      out[(size_t)t * n2 + c] = TS(val);
    }
    return;
  }
  if (MODE == COL_FWD_D_INV) {
    // filtered coefficients into the other buffer as real staging
    V2<T> *other = (U == bufA) ? bufB : bufA;
    T *re2 = reinterpret_cast<T *>(other);
    for (int idx = threadIdx.x; idx < C * m; idx += blockDim.x) {
      const int t = idx / C, s = idx - t * C;
      const int c = col0 + s;
      if (t == 0 || t == m - 1) continue;
      const T dv = c < n2 ? dflt[(size_t)t * n2 + c] : T(0);
      re2[t * C + s] = dv * dst_value<T>(U + s, C, t, M, post, scale);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < C; s += blockDim.x) {
      const int c = col0 + s;
      const T d0 = c < n2 ? dflt[c] : T(0);
      const T d1 = c < n2 ? dflt[(size_t)(m - 1) * n2 + c] : T(0);
      e0[s] = alpha * e0[s] * d0;  // filtered c_0, c_{m-1}
      e1[s] = alpha * e1[s] * d1;
    }
    __syncthreads();
    pack_u<T>(re2, 1, C, U, L, M, false, e0, e1);
    __syncthreads();
    U = fft_run<T>(U, other, fd, tw, gen, L);
  }
  // inverse output: y_0 = c_0 / alpha, y_{m-1} = c_{m-1} / alpha, interior DST + ramp
  for (int idx = threadIdx.x; idx < C * m; idx += blockDim.x) {
    const int t = idx / C, s = idx - t * C;
    const int c = col0 + s;
    if (c >= n2) continue;
    const T y0 = e0[s] / alpha, y1 = e1[s] / alpha;
    T val;
    if (t == 0) val = y0;
    else if (t == m - 1) val = y1;
    else
      val = dst_value<T>(U + s, C, t, M, post, scale) + y0 * (T(M - t) * invM) +
            y1 * (T(t) * invM);
    out[(size_t)t * n2 + c] = TS(val);
  }
}

// ------------------------------------------------------- plan-time tables

template <typename T>
__global__ void tables_kernel(V2<T> *tw, const int *tw_ns, const int *tw_r, const int *tw_base,
                              int nst, V2<T> *post, int M, V2<T> *gen, const int *gen_r,
                              const int *gen_base, int ngen) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int s = 0; s < nst; ++s) {
    const int Ns = tw_ns[s], R = tw_r[s], NR = Ns * R;
    for (int e = tid; e < NR; e += nth) {
      const int k = e / R, r = e - k * R;
      const long kr = ((long)k * r) % NR;
      double sv, cv;
      sincospi(-2.0 * (double)kr / (double)NR, &sv, &cv);
      tw[tw_base[s] + e] = {T(cv), T(sv)};
    }
  }
  for (int k = tid; k <= M; k += nth) {
    double sv, cv;
    sincospi((double)k / (double)M, &sv, &cv);
    post[k] = {T(cv), T(sv)};
  }
  for (int g = 0; g < ngen; ++g) {
    const int R = gen_r[g];
    for (int t = tid; t < R; t += nth) {
      double sv, cv;
      sincospi(-2.0 * (double)t / (double)R, &sv, &cv);
      gen[gen_base[g] + t] = {T(cv), T(sv)};
    }
  }
}

}  // namespace

bool radix_has_codelet(int r) {
  switch (r) {
    case 2: case 3: case 4: case 5: case 7: case 11: case 13: case 17: case 19: case 23:
    case 29: case 31:
      return true;
    default:
      return false;
  }
}

// `cdouble`: tables in double (compute type double) or float.
int fft_plan_build(FftPlan &fp, int m, bool cdouble, hipStream_t st) {
  fp.m = m;
  fp.M = m - 1;
  int M = fp.M;
  std::vector<int> rad;
  // powers of two as radix 4 (and one 2), odd primes ascending; primes
  // without a codelet become generic stages
  while (M % 4 == 0) { rad.push_back(4); M /= 4; }
  while (M % 2 == 0) { rad.push_back(2); M /= 2; }
  for (int p = 3; (long)p * p <= M; p += 2)
    while (M % p == 0) { rad.push_back(p); M /= p; }
  if (M > 1) rad.push_back(M);
  if ((int)rad.size() > kMaxStages) return fail(AR_EUNSUPPORTED, "too many FFT stages");
  fp.nstages = (int)rad.size();
  std::vector<int> tw_ns, tw_r, tw_base, gen_r, gen_base;
  size_t twc = 0, genc = 0;
  int ns = 1;
  for (int s = 0; s < fp.nstages; ++s) {
    fp.radix[s] = rad[s];
    fp.ns[s] = ns;
    fp.tw_off[s] = (int)twc;
    tw_ns.push_back(ns);
    tw_r.push_back(rad[s]);
    tw_base.push_back((int)twc);
    twc += (size_t)ns * rad[s];
    if (!radix_has_codelet(rad[s])) {
      fp.gen_off[s] = (int)genc;
      gen_r.push_back(rad[s]);
      gen_base.push_back((int)genc);
      genc += rad[s];
    }
    ns *= rad[s];
  }
  fp.tw_count = twc;
  fp.gen_count = genc;
  const size_t cb = cdouble ? sizeof(double2) : sizeof(float2);
  AR_HIP(hipMalloc(&fp.tw, (twc > 0 ? twc : 1) * cb));
  AR_HIP(hipMalloc(&fp.post, (size_t)(fp.M + 1) * cb));
  AR_HIP(hipMalloc(&fp.gen, (genc > 0 ? genc : 1) * cb));
  // small integer tables for the table kernel
  const int nst = fp.nstages, ngen = (int)gen_r.size();
  std::vector<int> ints;
  ints.insert(ints.end(), tw_ns.begin(), tw_ns.end());
  ints.insert(ints.end(), tw_r.begin(), tw_r.end());
  ints.insert(ints.end(), tw_base.begin(), tw_base.end());
  ints.insert(ints.end(), gen_r.begin(), gen_r.end());
  ints.insert(ints.end(), gen_base.begin(), gen_base.end());
  int *dints = nullptr;
  AR_HIP(hipMalloc(&dints, (ints.size() + 1) * sizeof(int)));
  AR_HIP(hipMemcpyAsync(dints, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice, st));
  const int *p_ns = dints, *p_r = dints + nst, *p_b = dints + 2 * nst;
  const int *p_gr = dints + 3 * nst, *p_gb = dints + 3 * nst + ngen;
  if (cdouble)
    hipLaunchKernelGGL(tables_kernel<double>, dim3(64), dim3(256), 0, st,
                       static_cast<V2<double> *>(fp.tw), p_ns, p_r, p_b, nst,
                       static_cast<V2<double> *>(fp.post), fp.M,
                       static_cast<V2<double> *>(fp.gen), p_gr, p_gb, ngen);
  else
    hipLaunchKernelGGL(tables_kernel<float>, dim3(64), dim3(256), 0, st,
                       static_cast<V2<float> *>(fp.tw), p_ns, p_r, p_b, nst,
                       static_cast<V2<float> *>(fp.post), fp.M, static_cast<V2<float> *>(fp.gen),
                       p_gr, p_gb, ngen);
  AR_HIP(hipGetLastError());
  AR_HIP(hipStreamSynchronize(st));
  AR_HIP(hipFree(dints));
  int rc = wave_plan_build(fp.w, fp.M, cdouble, false, st);
  if (rc != AR_OK) return rc;
  return wave_plan_build(fp.wb, fp.M, cdouble, true, st);
}

void fft_plan_free(FftPlan &fp) {
  wave_plan_free(fp.w);
  wave_plan_free(fp.wb);
  if (fp.tw) (void)hipFree(fp.tw);
  if (fp.post) (void)hipFree(fp.post);
  if (fp.gen) (void)hipFree(fp.gen);
  fp.tw = fp.post = fp.gen = nullptr;
}

int rows_blocks(const ar_plan_s *p) {
  if (p->bc != AR_BC_ANTIREFLECTIVE) return bc_rows_blocks(p);
  if (p->dtype == AR_F32_BF16X3) return dense_blocks(p);
  if (wave_rows_ok(p)) return wave_rows_blocks(p);
  const int B = rows_per_block(p->fft_row.M, p->csize);
  return (p->n1 + B - 1) / B;
}

int max_axis_len(size_t csize) {
  int M = (int)((kMaxLds - 64 - 2 * csize) / (4 * csize));
  while (M > 2 && seq_lds_bytes(1, M, csize) > kMaxLds) --M;
  return M + 1;
}

template <typename TS, typename T>
static int rows_launch_t(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                         const void *f_true, double *partial, hipStream_t st) {
  const FftPlan &fp = p->fft_row;
  const int m = p->n2, M = fp.M;
  const int B = rows_per_block(M, sizeof(T));
  const int blocks = (p->n1 + B - 1) / B;
  const size_t smem = seq_lds_bytes(B, M, sizeof(T));
  if (smem > kMaxLds) return fail(AR_EUNSUPPORTED, "row transform exceeds LDS");
  const FftDesc fd = make_desc(fp);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(fp.tw);
  auto gen = static_cast<const V2<T> *>(fp.gen);
  auto post = static_cast<const V2<T> *>(fp.post);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  hipError_t e = hipSuccess;
#define AR_ROWS(MODE)                                                                       \
  e = allow_lds(rows_kernel<TS, T, MODE>, smem);                                            \
  if (e == hipSuccess) {                                                                    \
    hipLaunchKernelGGL((rows_kernel<TS, T, MODE>), dim3(blocks), dim3(256), smem, st, ti, to, \
                       p->n1, m, fd, tw, gen, post, alpha, scale, B, M, T(tau), tf, partial); \
    e = hipGetLastError();                                                                  \
  }
  switch (mode) {
    case ROW_FWD: AR_ROWS(ROW_FWD) break;
    case ROW_INV: AR_ROWS(ROW_INV) break;
    default: AR_ROWS(ROW_INV_UPDATE) break;
  }
#undef AR_ROWS
  if (e != hipSuccess) return hip_fail(e, "rows_kernel launch");
  return AR_OK;
}

int rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                const void *f_true, double *partial, int *nblocks_out, hipStream_t st) {
  if (nblocks_out) *nblocks_out = rows_blocks(p);
  if (p->bc != AR_BC_ANTIREFLECTIVE)
    return bc_rows_launch(p, in, out, mode, tau, f_true, partial, st);
  if (p->dtype == AR_F32_BF16X3)
    return dense_rows_launch(p, in, out, mode, tau, f_true, partial, st);
  if (wave_rows_ok(p)) return wave_rows_launch(p, in, out, mode, tau, f_true, partial, st);
  if (p->dtype == AR_F64)
    return rows_launch_t<double, double>(p, in, out, mode, tau, f_true, partial, st);
  if (p->dtype == AR_F32_ACC64)
    return rows_launch_t<float, double>(p, in, out, mode, tau, f_true, partial, st);
  return rows_launch_t<float, float>(p, in, out, mode, tau, f_true, partial, st);
}

template <typename TS, typename T>
static int cols_launch_t(const ar_plan_s *p, const void *in, void *out, int mode,
                         hipStream_t st) {
  const FftPlan &fp = p->fft_col;
  const int m = p->n1, M = fp.M;
  const int C = cols_per_block(M, sizeof(T));
  const int blocks = (p->n2 + C - 1) / C;
  const size_t smem = seq_lds_bytes(C, M, sizeof(T));
  if (smem > kMaxLds) return fail(AR_EUNSUPPORTED, "column transform exceeds LDS");
  const FftDesc fd = make_desc(fp);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(fp.tw);
  auto gen = static_cast<const V2<T> *>(fp.gen);
  auto post = static_cast<const V2<T> *>(fp.post);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const T *>(p->d);
  hipError_t e = hipSuccess;
#define AR_COLS(MODE)                                                                        \
  e = allow_lds(cols_kernel<TS, T, MODE>, smem);                                             \
  if (e == hipSuccess) {                                                                     \
    hipLaunchKernelGGL((cols_kernel<TS, T, MODE>), dim3(blocks), dim3(256), smem, st, ti, to, \
                       m, p->n2, fd, tw, gen, post, alpha, scale, C, td);                    \
    e = hipGetLastError();                                                                   \
  }
  switch (mode) {
    case COL_FWD: AR_COLS(COL_FWD) break;
    case COL_INV: AR_COLS(COL_INV) break;
    default: AR_COLS(COL_FWD_D_INV) break;
  }
#undef AR_COLS
  if (e != hipSuccess) return hip_fail(e, "cols_kernel launch");
  return AR_OK;
}

int cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  if (p->bc != AR_BC_ANTIREFLECTIVE) return bc_cols_launch(p, in, out, mode, st);
  if (p->dtype == AR_F32_BF16X3) return dense_cols_launch(p, in, out, mode, st);
  if (wave_cols_ok(p)) return wave_cols_launch(p, in, out, mode, st);
  if (p->dtype == AR_F64) return cols_launch_t<double, double>(p, in, out, mode, st);
  if (p->dtype == AR_F32_ACC64) return cols_launch_t<float, double>(p, in, out, mode, st);
  return cols_launch_t<float, float>(p, in, out, mode, st);
}

}  // namespace ar

using namespace ar;

extern "C" int ar_transform(ar_plan_t p, const void *x, void *c, void *stream) {
  if (!p || !x || !c) return fail(AR_EINVAL, "ar_transform: null argument");
  if (p->bc == AR_BC_PERIODIC)
    return fail(AR_EUNSUPPORTED, "ar_transform: periodic plans have complex coefficients");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = rows_launch(p, x, c, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st);
  if (rc != AR_OK) return rc;
  return cols_launch(p, c, c, COL_FWD, st);
}

extern "C" int ar_transform_inv(ar_plan_t p, const void *c, void *x, void *stream) {
  if (!p || !x || !c) return fail(AR_EINVAL, "ar_transform_inv: null argument");
  if (p->bc == AR_BC_PERIODIC)
    return fail(AR_EUNSUPPORTED, "ar_transform_inv: periodic plans have complex coefficients");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = cols_launch(p, c, x, COL_INV, st);
  if (rc != AR_OK) return rc;
  return rows_launch(p, x, x, ROW_INV, 0.0, nullptr, nullptr, nullptr, st);
}

extern "C" int ar_precond_solve(ar_plan_t p, const void *y, void *z, void *stream) {
  if (!p || !y || !z) return fail(AR_EINVAL, "ar_precond_solve: null argument");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // Anti-Reflective and Reflective coefficients fit z (in place); periodic
  // half spectra are wider than an image and go through the plan's buffer
  void *w = p->bc == AR_BC_PERIODIC ? p->c : z;
  int rc = rows_launch(p, y, w, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st);
  if (rc != AR_OK) return rc;
  rc = cols_launch(p, w, w, COL_FWD_D_INV, st);
  if (rc != AR_OK) return rc;
  return rows_launch(p, w, z, ROW_INV, 0.0, nullptr, nullptr, nullptr, st);
}

extern "C" int ar_tikhonov_solve(ar_plan_t p, const void *g, void *x, double alpha,
                                 void *stream) {
  if (!p || !g || !x) return fail(AR_EINVAL, "ar_tikhonov_solve: null argument");
  if (!(alpha > 0.0 && std::isfinite(alpha)))
    return fail(AR_EINVAL, "ar_tikhonov_solve: alpha must be finite and > 0");
  if (p->bc == AR_BC_PERIODIC)
    return fail(AR_EUNSUPPORTED, "ar_tikhonov_solve: defined for Anti-Reflective and Reflective "
                                 "plans");
  if (!p->strong_sym)
    return fail(AR_EPSF, "ar_tikhonov_solve: the direct solve needs a strongly symmetric PSF "
                         "(h_{-s1,s2} = h_{s1,-s2} = h_{s1,s2})");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // x = T diag(lambda / (lambda^2 + alpha)) T~ g, every pass in place on x
  int rc = rows_launch(p, g, x, ROW_FWD, 0.0, nullptr, nullptr, nullptr, st);
  if (rc == AR_OK) rc = cols_launch(p, x, x, COL_FWD, st);
  if (rc == AR_OK) rc = tikhonov_scale_launch(p, x, alpha, st);
  if (rc == AR_OK) rc = cols_launch(p, x, x, COL_INV, st);
  if (rc == AR_OK) rc = rows_launch(p, x, x, ROW_INV, 0.0, nullptr, nullptr, nullptr, st);
  return rc;
}
