// Dense AR transforms on MFMA with BF16x3 operands (gfx950).
//
// Per axis of length m the AR transform of Theorem 1 is one m x m matrix:
//   T~ = [ alpha    0        0      ]      T = [ 1/alpha     0      0       ]
//        [ -Q p     Q     -Q J p    ]          [ p/alpha     Q   J p/alpha  ]
//        [ 0        0      alpha    ]          [ 0           0   1/alpha    ]
// (Q the DST-I matrix of eq. (Qn), p_j = 1 - j/(m-1), (J p)_j = j/(m-1)),
// so each pass of the 2-D transform is one GEMM: rows C = Y T~^T, columns
// C = T~ Y (and T for the inverse).  The preconditioner's filter d is
// applied in the epilogue of the forward column GEMM and the update
// x += tau w in the epilogue of the inverse row GEMM.
//
// GEMM: 128 x 128 output tile per workgroup (4 waves, 64 x 64 each), K step
// 32, v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Every FP32 operand
// is split on the fly into hi = bf16(a) and lo = bf16(a - hi) and the
// product is hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-18 relative, is
// dropped), giving ~1e-5 relative accuracy per product.  The matrices are
// built in FP64 on the device and stored as FP32.
#include <cmath>

#include "ar_internal.h"

namespace ar {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int PK = BK + 8;  // LDS row pitch in bf16 (80 bytes)

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

enum Epi { EPI_STORE = 0, EPI_DMUL = 1, EPI_UPDATE = 2 };

// C (M x N) = A (M x K) B (K x N), row-major with leading dimensions.
// EPI_DMUL: C = d .* (A B) with d laid out like C.  EPI_UPDATE: C += tau (A B)
// and, with f, per-workgroup FP64 partial sums of (C - f)^2.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(
    const float *__restrict__ A, long lda, const float *__restrict__ B, long ldb,
    float *__restrict__ C, long ldc, int M, int N, int K, const float *__restrict__ d, float tau,
    const float *__restrict__ f, double *__restrict__ partial, int tiles_n) {
  __shared__ __align__(16) unsigned short Ah[BM * PK], Al[BM * PK], Bh[BN * PK], Bl[BN * PK];
  __shared__ double red[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int i0 = tm * BM, j0 = tn * BN;
  const int wr = wave >> 1, wc = wave & 1;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  // tile loads: A as 128 rows x 32 k (thread: row tid / 8 + 32 u, 4
  // consecutive k), B as 32 k x 128 columns (thread: column tid % 128, 16
  // consecutive k), so that the split halves go to LDS as packed 8- and
  // 16-byte stores ([row][k] for A, [column][k] for B)
  const int bn = tid & 127, bkq = (tid >> 7) * 16;
  for (int k0 = 0; k0 < K; k0 += BK) {
    // global -> registers (clamped addresses, zero outside), all loads first
    float av[16], bv[16];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int row = idx >> 3, c = (idx & 7) * 4;
      const int gi = i0 + row;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gk = k0 + c + e;
        const bool ok = gi < M && gk < K;
        const float v = A[(long)(ok ? gi : 0) * lda + (ok ? gk : 0)];
        av[4 * u + e] = ok ? v : 0.f;
      }
    }
    {
      const int gj = j0 + bn;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int gk = k0 + bkq + e;
        const bool ok = gk < K && gj < N;
        const float v = B[(long)(ok ? gk : 0) * ldb + (ok ? gj : 0)];
        bv[e] = ok ? v : 0.f;
      }
    }
    __syncthreads();  // the previous step's fragments have been read
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int row = idx >> 3, c = (idx & 7) * 4;
      unsigned hw[2], lw[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const float v0 = av[4 * u + 2 * q], v1 = av[4 * u + 2 * q + 1];
        const unsigned short h0 = bf16_bits(v0), h1 = bf16_bits(v1);
        hw[q] = (unsigned)h0 | ((unsigned)h1 << 16);
        lw[q] = (unsigned)bf16_bits(v0 - bf16_val(h0)) |
                ((unsigned)bf16_bits(v1 - bf16_val(h1)) << 16);
      }
      *reinterpret_cast<uint2 *>(&Ah[row * PK + c]) = make_uint2(hw[0], hw[1]);
      *reinterpret_cast<uint2 *>(&Al[row * PK + c]) = make_uint2(lw[0], lw[1]);
    }
    {
      unsigned hw[8], lw[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float v0 = bv[2 * q], v1 = bv[2 * q + 1];
        const unsigned short h0 = bf16_bits(v0), h1 = bf16_bits(v1);
        hw[q] = (unsigned)h0 | ((unsigned)h1 << 16);
        lw[q] = (unsigned)bf16_bits(v0 - bf16_val(h0)) |
                ((unsigned)bf16_bits(v1 - bf16_val(h1)) << 16);
      }
      uint4 *bh4 = reinterpret_cast<uint4 *>(&Bh[bn * PK + bkq]);  // transposed: [n][k]
      uint4 *bl4 = reinterpret_cast<uint4 *>(&Bl[bn * PK + bkq]);
      bh4[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      bh4[1] = make_uint4(hw[4], hw[5], hw[6], hw[7]);
      bl4[0] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
      bl4[1] = make_uint4(lw[4], lw[5], lw[6], lw[7]);
    }
    __syncthreads();
    // lane l: A[i = l % 16][k = 8 (l / 16) + e], B[k = 8 (l / 16) + e][j = l % 16]
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    bf8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = wr * 64 + t * 16 + lr;
      ah[t] = *reinterpret_cast<const bf8 *>(&Ah[r * PK + lk]);
      al[t] = *reinterpret_cast<const bf8 *>(&Al[r * PK + lk]);
      const int cc = wc * 64 + t * 16 + lr;
      bh[t] = *reinterpret_cast<const bf8 *>(&Bh[cc * PK + lk]);
      bl[t] = *reinterpret_cast<const bf8 *>(&Bl[cc * PK + lk]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
      }
  }
  // epilogue: lane l holds D[i = 4 (l / 16) + e][j = l % 16] of each 16 x 16 tile
  double ss = 0.0;
  const int lj = lane & 15, li = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wr * 64 + a * 16 + li + e;
        const int j = j0 + wc * 64 + b * 16 + lj;
        if (i >= M || j >= N) continue;
        const long o = (long)i * ldc + j;
        const float v = acc[a][b][e];
        if (EPI == EPI_STORE) {
          C[o] = v;
        } else if (EPI == EPI_DMUL) {
          C[o] = v * d[o];
        } else {
          const float xn = C[o] + tau * v;
          C[o] = xn;
          if (f) {
            const double df = (double)xn - (double)f[o];
            ss += df * df;
          }
        }
      }
  if (EPI == EPI_UPDATE && partial) {
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// Forward (inv = 0) or inverse (inv = 1) AR transform matrix of length m,
// built in FP64, stored as FP32; transposed with trans = 1.
__global__ __launch_bounds__(256) void ar_matrix_kernel(float *__restrict__ out, int m, int inv,
                                                        int trans) {
  const int N1 = m - 1;  // N + 1 with N = m - 2 interior points
  const double alpha = sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0)));
  const double s = sqrt(2.0 / (double)N1);
  const long total = (long)m * m;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e / m), c = (int)(e - (long)r * m);
    double v = 0.0;
    const bool rin = r > 0 && r < m - 1, cin = c > 0 && c < m - 1;
    auto q = [&](int a, int b) {  // Q entry of interior indices a, b in 1..m-2
      const long t = ((long)a * b) % (2L * N1);
      return s * sinpi((double)t / (double)N1);
    };
    if (!inv) {
      if (r == 0) v = c == 0 ? alpha : 0.0;
      else if (r == m - 1) v = c == m - 1 ? alpha : 0.0;
      else if (cin) v = q(r, c);
      else {
        // -(Q p)_r or -(Q J p)_r
        double acc = 0.0;
        for (int j = 1; j < m - 1; ++j) {
          const double w = c == 0 ? (double)(m - 1 - j) / N1 : (double)j / N1;
          acc += q(r, j) * w;
        }
        v = -acc;
      }
    } else {
      if (c == 0) v = r == 0 ? 1.0 / alpha : (rin ? (double)(m - 1 - r) / N1 / alpha : 0.0);
      else if (c == m - 1) v = r == m - 1 ? 1.0 / alpha : (rin ? (double)r / N1 / alpha : 0.0);
      else v = rin ? q(r, c) : 0.0;
    }
    const long o = trans ? (long)c * m + r : e;
    out[o] = (float)v;
  }
}

template <int EPI>
int gemm_launch(const float *A, long lda, const float *B, long ldb, float *C, long ldc, int M,
                int N, int K, const float *d, float tau, const float *f, double *partial,
                hipStream_t st) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  hipLaunchKernelGGL(gemm_bf16x3_kernel<EPI>, dim3(tiles_m * tiles_n), dim3(256), 0, st, A, lda,
                     B, ldb, C, ldc, M, N, K, d, tau, f, partial, tiles_n);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

}  // namespace

int dense_blocks(const ar_plan_s *p) {
  return ((p->n1 + BM - 1) / BM) * ((p->n2 + BN - 1) / BN);
}

int dense_setup(ar_plan_s *p, hipStream_t st) {
  const size_t b1 = (size_t)p->n1 * p->n1 * sizeof(float);
  const size_t b2 = (size_t)p->n2 * p->n2 * sizeof(float);
  AR_HIP(hipMalloc((void **)&p->mat_fwd_col, b1));
  AR_HIP(hipMalloc((void **)&p->mat_inv_col, b1));
  AR_HIP(hipMalloc((void **)&p->mat_fwdT_row, b2));
  AR_HIP(hipMalloc((void **)&p->mat_invT_row, b2));
  AR_HIP(hipMalloc(&p->dscr, (size_t)p->n1 * p->n2 * sizeof(float)));
  hipLaunchKernelGGL(ar_matrix_kernel, dim3(1024), dim3(256), 0, st, p->mat_fwd_col, p->n1, 0, 0);
  hipLaunchKernelGGL(ar_matrix_kernel, dim3(1024), dim3(256), 0, st, p->mat_inv_col, p->n1, 1, 0);
  hipLaunchKernelGGL(ar_matrix_kernel, dim3(1024), dim3(256), 0, st, p->mat_fwdT_row, p->n2, 0, 1);
  hipLaunchKernelGGL(ar_matrix_kernel, dim3(1024), dim3(256), 0, st, p->mat_invT_row, p->n2, 1, 1);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

// Row passes: out = in T~^T (ROW_FWD), in T^T (ROW_INV), x += tau in T^T
// (ROW_INV_UPDATE, out = x).  in == out goes through the dense scratch.
int dense_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                      const void *f_true, double *partial, hipStream_t st) {
  const int n1 = p->n1, n2 = p->n2;
  const float *A = static_cast<const float *>(in);
  const float *B = mode == ROW_FWD ? p->mat_fwdT_row : p->mat_invT_row;
  if (mode == ROW_INV_UPDATE)
    return gemm_launch<EPI_UPDATE>(A, n2, B, n2, static_cast<float *>(out), n2, n1, n2, n2,
                                   nullptr, (float)tau, static_cast<const float *>(f_true),
                                   partial, st);
  float *C = in == out ? static_cast<float *>(p->dscr) : static_cast<float *>(out);
  int rc = gemm_launch<EPI_STORE>(A, n2, B, n2, C, n2, n1, n2, n2, nullptr, 0.f, nullptr, nullptr,
                                  st);
  if (rc != AR_OK || in != out) return rc;
  AR_HIP(hipMemcpyAsync(out, C, (size_t)n1 * n2 * sizeof(float), hipMemcpyDeviceToDevice, st));
  return AR_OK;
}

// Column passes: out = T~ in (COL_FWD), T in (COL_INV), T (d .* (T~ in))
// (COL_FWD_D_INV, through the dense scratch).
int dense_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  const int n1 = p->n1, n2 = p->n2;
  const float *B = static_cast<const float *>(in);
  float *S = static_cast<float *>(p->dscr);
  if (mode == COL_FWD_D_INV) {
    int rc = gemm_launch<EPI_DMUL>(p->mat_fwd_col, n1, B, n2, S, n2, n1, n2, n1,
                                   static_cast<const float *>(p->d), 0.f, nullptr, nullptr, st);
    if (rc != AR_OK) return rc;
    return gemm_launch<EPI_STORE>(p->mat_inv_col, n1, S, n2, static_cast<float *>(out), n2, n1,
                                  n2, n1, nullptr, 0.f, nullptr, nullptr, st);
  }
  const float *Mx = mode == COL_FWD ? p->mat_fwd_col : p->mat_inv_col;
  float *C = in == out ? S : static_cast<float *>(out);
  int rc = gemm_launch<EPI_STORE>(Mx, n1, B, n2, C, n2, n1, n2, n1, nullptr, 0.f, nullptr,
                                  nullptr, st);
  if (rc != AR_OK || in != out) return rc;
  AR_HIP(hipMemcpyAsync(out, C, (size_t)n1 * n2 * sizeof(float), hipMemcpyDeviceToDevice, st));
  return AR_OK;
}

}  // namespace ar
