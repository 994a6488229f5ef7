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
// Operands are BF16 pairs hi = bf16(a), lo = bf16(a - hi): the matrices are
// built in FP64 on the device and split once when the plan is made; an
// image operand is split once per pass (transposed for the column passes,
// so that both GEMM operands are K-contiguous).  GEMM: 128 x 128 output
// tile per workgroup (8 waves, 64 x 32 each), K step 32, double-buffered
// LDS, three v_mfma_f32_16x16x32_bf16 products per tile pair with FP32
// accumulation.
#include <algorithm>
#include <cmath>

#include "ar_internal.h"

namespace ar {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int PK = BK + 8;  // LDS row pitch in bf16 (80 bytes)
constexpr int KPAD = 32;    // operand rows are padded with zeros to a multiple of this
constexpr int NBUF = 2;     // LDS buffers of the GEMM pipeline
constexpr int GT = 512;     // threads of a GEMM workgroup (8 waves of 64 x 32 outputs)
constexpr int GROUP_M = 4;  // row tiles per group of the workgroup order
constexpr size_t kGemmLds = (size_t)NBUF * 4 * BM * PK * sizeof(unsigned short) + 8 * sizeof(double);

__host__ __device__ inline int kpad(int k) { return (k + KPAD - 1) / KPAD * KPAD; }

__device__ __forceinline__ u16 bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_val(u16 h) { return __uint_as_float((unsigned)h << 16); }

enum Epi { EPI_STORE = 0, EPI_DMUL = 1, EPI_UPDATE = 2 };

// Split an R x C FP32 matrix (leading dimension ldi) into BF16 planes
// hi = bf16(a), lo = bf16(a - hi) with rows of ldo >= C elements (zeros past
// C), as is (trans = 0, R rows) or transposed (trans = 1, C rows of R).
// 32 x 32 tiles through LDS; grid (ceil(ldo_cols / 32), ceil(rows / 32)).
__global__ __launch_bounds__(256) void split_kernel(const float *__restrict__ in, long ldi, int R,
                                                    int C, u16 *__restrict__ hi,
                                                    u16 *__restrict__ lo, long ldo, int trans) {
  __shared__ float t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  // output tile: rows orow0 .. +31, columns ocol0 .. +31
  const int ocol0 = blockIdx.x * 32, orow0 = blockIdx.y * 32;
  const int orows = trans ? C : R, ocols = trans ? R : C;
  if (!trans) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = orow0 + ty + 8 * u, c = ocol0 + tx;
      if (r >= orows || c >= ldo) continue;
      const float v = c < ocols ? in[(long)r * ldi + c] : 0.f;
      const u16 h = bf16_bits(v);
      hi[(long)r * ldo + c] = h;
      lo[(long)r * ldo + c] = bf16_bits(v - bf16_val(h));
    }
    return;
  }
  // transposed: input rows ocol0 .. +31 (< R), input columns orow0 .. +31 (< C)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ir = ocol0 + ty + 8 * u, ic = orow0 + tx;
    t[ty + 8 * u][tx] = (ir < R && ic < C) ? in[(long)ir * ldi + ic] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = orow0 + ty + 8 * u, c = ocol0 + tx;
    if (r >= orows || c >= ldo) continue;
    const float v = t[tx][ty + 8 * u];
    const u16 h = bf16_bits(v);
    hi[(long)r * ldo + c] = h;
    lo[(long)r * ldo + c] = bf16_bits(v - bf16_val(h));
  }
}

// C (M x N) = A B with A given as BF16 planes [M][K] and B as planes [N][K]
// (both K-contiguous, K a multiple of BK with zero padding), row-major C.
// The product is hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-18 relative,
// is dropped), ~1e-5 relative per product, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  128 x 128 tile per workgroup (8 waves, 64 x 32
// each, two per SIMD); the tiles of K-step s + 1 travel global -> registers
// while step s runs from LDS, then go to the other LDS buffer (one barrier
// per step).
// EPI_DMUL: C = d .* (A B) with d laid out like C.  EPI_UPDATE: C += tau (A B)
// and, with f, per-workgroup FP64 partial sums of (C - f)^2.
struct Planes {
  const u16 *hi, *lo;
  long ld;
};

template <int EPI>
__global__ __launch_bounds__(GT) void gemm_b3_kernel(Planes A, Planes B, float *__restrict__ C,
                                                      long ldc, int M, int N, int K,
                                                      const float *__restrict__ d, float tau,
                                                      const float *__restrict__ f,
                                                      double *__restrict__ partial, int tiles_n) {
  extern __shared__ __align__(16) unsigned char gsm[];
  u16(*sm)[4][BM * PK] = reinterpret_cast<u16(*)[4][BM * PK]>(gsm);  // [buffer][Ah, Al, Bh, Bl]
  double *red = reinterpret_cast<double *>(gsm + (size_t)NBUF * 4 * BM * PK * sizeof(u16));
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // tile of this workgroup: consecutive logical ids run on one XCD (ids are
  // dealt round-robin over the 8 XCDs) and walk groups of GROUP_M row tiles
  // column by column, so that the workgroups of an XCD share A rows and B
  // columns in its L2
  int tm, tn;
  {
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, q = b >> 3, g8 = nb >> 3, rem = nb & 7;
    const int L = x * g8 + (x < rem ? x : rem) + q;
    const int tiles_m = nb / tiles_n;
    const int per_group = GROUP_M * tiles_n, grp = L / per_group;
    const int first = grp * GROUP_M, gsize = min(tiles_m - first, GROUP_M);
    const int r = L - grp * per_group;
    tm = first + r % gsize;
    tn = r / gsize;
  }
  const int i0 = tm * BM, j0 = tn * BN;
  const int wr = wave >> 2, wc = wave & 3;  // 64-row half, 32-column quarter
  // this thread's 16-byte chunk of each of the four planes: tile row
  // tid / 4, k offset 8 (tid % 4)
  const int lrow = tid >> 2, lk8 = (tid & 3) * 8;
  const u16 *src[4];
  {
    const int ra = min(i0 + lrow, M - 1), rb = min(j0 + lrow, N - 1);
    src[0] = A.hi + (long)ra * A.ld + lk8;
    src[1] = A.lo + (long)ra * A.ld + lk8;
    src[2] = B.hi + (long)rb * B.ld + lk8;
    src[3] = B.lo + (long)rb * B.ld + lk8;
  }
  // two register stages: the loads of step s + 2 are in flight while step
  // s runs, step s + 1 waits in the other stage for its LDS buffer
  uint4 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;
#define AR_FETCH(S, k0)                                             \
  S##0 = *reinterpret_cast<const uint4 *>(src[0] + (k0));           \
  S##1 = *reinterpret_cast<const uint4 *>(src[1] + (k0));           \
  S##2 = *reinterpret_cast<const uint4 *>(src[2] + (k0));           \
  S##3 = *reinterpret_cast<const uint4 *>(src[3] + (k0))
#define AR_PUT(S, buf)                                                     \
  *reinterpret_cast<uint4 *>(&sm[buf][0][lrow * PK + lk8]) = S##0;         \
  *reinterpret_cast<uint4 *>(&sm[buf][1][lrow * PK + lk8]) = S##1;         \
  *reinterpret_cast<uint4 *>(&sm[buf][2][lrow * PK + lk8]) = S##2;         \
  *reinterpret_cast<uint4 *>(&sm[buf][3][lrow * PK + lk8]) = S##3
  // lane l: A[i = l % 16][k = 8 (l / 16) + e], B[k = 8 (l / 16) + e][j = l % 16]
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  struct Frags { bf8 ah[4], al[4], bh[2], bl[2]; };
  auto frags = [&](int buf, Frags &F) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = (wr * 64 + t * 16 + lr) * PK + lk;
      F.ah[t] = *reinterpret_cast<const bf8 *>(&sm[buf][0][r]);
      F.al[t] = *reinterpret_cast<const bf8 *>(&sm[buf][1][r]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int c = (wc * 32 + t * 16 + lr) * PK + lk;
      F.bh[t] = *reinterpret_cast<const bf8 *>(&sm[buf][2][c]);
      F.bl[t] = *reinterpret_cast<const bf8 *>(&sm[buf][3][c]);
    }
  };
  f4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  // two LDS buffers (step s in buffer s % 2) and two register stages (step
  // s in stage s % 2): step s computes while step s + 1 goes from its stage
  // to the other buffer and step s + 2 is fetched into the freed stage
  const int nk = K / BK;
  AR_FETCH(sa, 0);
  AR_PUT(sa, 0);
  if (nk > 1) {
    AR_FETCH(sb, BK);
  }
  __syncthreads();
  auto mma = [&](int buf) {
    Frags cur;
    frags(buf, cur);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.al[a], cur.bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ah[a], cur.bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ah[a], cur.bh[b], acc[a][b], 0, 0, 0);
      }
  };
  for (int s = 0; s < nk; s += 2) {
    // step s (stage a, buffer 0)
    if (s + 2 < nk) {
      AR_FETCH(sa, (s + 2) * BK);
    }
    mma(0);
    if (s + 1 < nk) {
      AR_PUT(sb, 1);
    }
    __syncthreads();
    if (s + 1 >= nk) break;
    // step s + 1 (stage b, buffer 1)
    if (s + 3 < nk) {
      AR_FETCH(sb, (s + 3) * BK);
    }
    mma(1);
    if (s + 2 < nk) {
      AR_PUT(sa, 0);
    }
    __syncthreads();
  }
#undef AR_FETCH
#undef AR_PUT
  // epilogue: lane l holds D[i = 4 (l / 16) + e][j = l % 16] of each 16 x 16 tile
  double ss = 0.0;
  const int lj = lane & 15, li = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wr * 64 + a * 16 + li + e;
        const int j = j0 + wc * 32 + b * 16 + lj;
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
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < GT / 64; ++w) t += red[w];
      partial[blockIdx.x] = t;
    }
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
int gemm_launch(Planes A, Planes B, float *C, long ldc, int M, int N, int K, const float *d,
                float tau, const float *f, double *partial, hipStream_t st) {
  const int tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
  AR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(gemm_b3_kernel<EPI>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmLds));
  hipLaunchKernelGGL(gemm_b3_kernel<EPI>, dim3(tiles_m * tiles_n), dim3(GT), kGemmLds, st, A, B,
                     C, ldc, M, N, K, d, tau, f, partial, tiles_n);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

// FP32 R x C (leading dimension ldi) -> BF16 planes at `planes` (hi, then lo
// after rows * ldo elements), as is or transposed.
int split_launch(const float *in, long ldi, int R, int C, void *planes, int ldo, bool trans,
                 hipStream_t st) {
  const int orows = trans ? C : R;
  u16 *hi = static_cast<u16 *>(planes), *lo = hi + (size_t)orows * ldo;
  hipLaunchKernelGGL(split_kernel, dim3((ldo + 31) / 32, (orows + 31) / 32), dim3(256), 0, st, in,
                     ldi, R, C, hi, lo, (long)ldo, trans ? 1 : 0);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

Planes planes_of(const void *p, int rows, int ld) {
  const u16 *hi = static_cast<const u16 *>(p);
  return Planes{hi, hi + (size_t)rows * ld, (long)ld};
}

}  // namespace

int dense_blocks(const ar_plan_s *p) {
  return ((p->n1 + BM - 1) / BM) * ((p->n2 + BN - 1) / BN);
}

// The four transform matrices as BF16 planes (split once, here): T~_{n1}
// and T_{n1} for the column passes (A operands, [n1][kpad(n1)]), T~_{n2}
// and T_{n2} for the row passes (B operands [N][K] = the matrices
// themselves, [n2][kpad(n2)]); scratch: the FP32 n1 x n2 filter product and
// the planes of one image operand.
int dense_setup(ar_plan_s *p, hipStream_t st) {
  const int n1 = p->n1, n2 = p->n2, l1 = kpad(n1), l2 = kpad(n2);
  const size_t b1 = 2 * (size_t)n1 * l1 * sizeof(u16), b2 = 2 * (size_t)n2 * l2 * sizeof(u16);
  AR_HIP(hipMalloc(&p->mat_fwd_col, b1));
  AR_HIP(hipMalloc(&p->mat_inv_col, b1));
  AR_HIP(hipMalloc(&p->mat_fwd_row, b2));
  AR_HIP(hipMalloc(&p->mat_inv_row, b2));
  AR_HIP(hipMalloc(&p->dscr, (size_t)n1 * n2 * sizeof(float)));
  const size_t sp = 2 * std::max((size_t)n1 * l2, (size_t)n2 * l1) * sizeof(u16);
  AR_HIP(hipMalloc(&p->dsplit, sp));
  const int mmax = std::max(n1, n2);
  float *tmp = nullptr;
  AR_HIP(hipMalloc((void **)&tmp, (size_t)mmax * mmax * sizeof(float)));
  int rc = AR_OK;
  struct Job { void *dst; int m, inv; } jobs[4] = {
      {p->mat_fwd_col, n1, 0}, {p->mat_inv_col, n1, 1}, {p->mat_fwd_row, n2, 0},
      {p->mat_inv_row, n2, 1}};
  for (const Job &j : jobs) {
    hipLaunchKernelGGL(ar_matrix_kernel, dim3(1024), dim3(256), 0, st, tmp, j.m, j.inv, 0);
    if ((rc = split_launch(tmp, j.m, j.m, j.m, j.dst, kpad(j.m), false, st)) != AR_OK) break;
  }
  hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (rc != AR_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "dense_setup");
  return AR_OK;
}

// Row passes: out = in T~^T (ROW_FWD), in T^T (ROW_INV), x += tau in T^T
// (ROW_INV_UPDATE, out = x).  The input is split into planes first, so
// in == out is allowed.
int dense_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                      const void *f_true, double *partial, hipStream_t st) {
  const int n1 = p->n1, n2 = p->n2, l2 = kpad(n2);
  int rc = split_launch(static_cast<const float *>(in), n2, n1, n2, p->dsplit, l2, false, st);
  if (rc != AR_OK) return rc;
  const Planes A = planes_of(p->dsplit, n1, l2);
  const Planes B = planes_of(mode == ROW_FWD ? p->mat_fwd_row : p->mat_inv_row, n2, l2);
  float *C = static_cast<float *>(out);
  if (mode == ROW_INV_UPDATE)
    return gemm_launch<EPI_UPDATE>(A, B, C, n2, n1, n2, l2, nullptr, (float)tau,
                                   static_cast<const float *>(f_true), partial, st);
  return gemm_launch<EPI_STORE>(A, B, C, n2, n1, n2, l2, nullptr, 0.f, nullptr, nullptr, st);
}

// Column passes: out = T~ in (COL_FWD), T in (COL_INV), T (d .* (T~ in))
// (COL_FWD_D_INV, the filter product through the FP32 scratch).
int dense_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  const int n1 = p->n1, n2 = p->n2, l1 = kpad(n1);
  int rc = split_launch(static_cast<const float *>(in), n2, n1, n2, p->dsplit, l1, true, st);
  if (rc != AR_OK) return rc;
  const Planes B = planes_of(p->dsplit, n2, l1);
  if (mode == COL_FWD_D_INV) {
    float *S = static_cast<float *>(p->dscr);
    rc = gemm_launch<EPI_DMUL>(planes_of(p->mat_fwd_col, n1, l1), B, S, n2, n1, n2, l1,
                               static_cast<const float *>(p->d), 0.f, nullptr, nullptr, st);
    if (rc != AR_OK) return rc;
    if ((rc = split_launch(S, n2, n1, n2, p->dsplit, l1, true, st)) != AR_OK) return rc;
    return gemm_launch<EPI_STORE>(planes_of(p->mat_inv_col, n1, l1), B,
                                  static_cast<float *>(out), n2, n1, n2, l1, nullptr, 0.f,
                                  nullptr, nullptr, st);
  }
  const void *Mx = mode == COL_FWD ? p->mat_fwd_col : p->mat_inv_col;
  return gemm_launch<EPI_STORE>(planes_of(Mx, n1, l1), B, static_cast<float *>(out), n2, n1, n2,
                                l1, nullptr, 0.f, nullptr, nullptr, st);
}

}  // namespace ar
