// Learned preconditioner filter (gfx950): features of a problem, the gains
// filter, and the filter network (forward on BF16 MFMA, backward, Adam).
//
// None of this is in the paper, whose filter is Tikhonov (eq. (TikFilter));
// it replaces the hand-tuned parameter of that filter by a parameter per
// eigenvalue-magnitude bin, predicted from the radial profile of the
// spectrum of the symmetrized PSF (Theorem 2) and a noise estimate of the
// data.
//
// Radial bin (features) of coefficient (k1, k2): with r_j = k_j on interior columns of
// T and 0 on the first and last one, N_j = n_j - 1, (64 rho)^2 =
// 2048 (r1^2 / N1^2 + r2^2 / N2^2) = S / D with S = 2048 (r1^2 N2^2 +
// r2^2 N1^2), D = N1^2 N2^2 (exact 64-bit integers), and bin =
// min(floor(sqrt(S / D)), 63), decided exactly.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ar_internal.h"

namespace ar {
namespace {

constexpr int NB = AR_FNET_BINS, NIN = AR_FNET_IN, NH = AR_FNET_HIDDEN, NPAR = AR_FNET_NPARAM;
// parameter offsets (W stored (out, in) row-major)
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NB * NH;
static_assert(OB3 + NB == NPAR, "parameter layout");

__host__ __device__ inline int radial_bin(int k1, int k2, int n1, int n2) {
  const long long N1 = n1 - 1, N2 = n2 - 1;
  const long long r1 = (k1 == 0 || k1 == n1 - 1) ? 0 : k1;
  const long long r2 = (k2 == 0 || k2 == n2 - 1) ? 0 : k2;
  const long long S = 2048 * (r1 * r1 * N2 * N2 + r2 * r2 * N1 * N1);
  const long long D = N1 * N1 * N2 * N2;
  long long k = (long long)sqrt((double)S / (double)D);
  while (k > 0 && k * k * D > S) --k;
  while ((k + 1) * (k + 1) * D <= S) ++k;
  return k > NB - 1 ? NB - 1 : (int)k;
}

// ------------------------------------------------------------ features

// Per-row partial sums and counts of lambda over the radial bins.
__global__ __launch_bounds__(256) void profile_rows_kernel(const double *__restrict__ lam, int n1,
                                                           int n2, double *__restrict__ psum,
                                                           int *__restrict__ pcnt) {
  __shared__ double s[NB];
  __shared__ int c[NB];
  const int k1 = blockIdx.x;
  if (threadIdx.x < NB) {
    s[threadIdx.x] = 0.0;
    c[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int k2 = threadIdx.x; k2 < n2; k2 += blockDim.x) {
    const size_t e = (size_t)k1 * n2 + k2;
    const int b = radial_bin(k1, k2, n1, n2);
    atomicAdd(&s[b], lam[e]);
    atomicAdd(&c[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    psum[(size_t)k1 * NB + threadIdx.x] = s[threadIdx.x];
    pcnt[(size_t)k1 * NB + threadIdx.x] = c[threadIdx.x];
  }
}

// Bin means in fixed row order (0 for an empty bin).
__global__ void profile_final_kernel(const double *__restrict__ psum, const int *__restrict__ pcnt,
                                     int n1, float *__restrict__ out) {
  const int b = threadIdx.x;
  if (b >= NB) return;
  double s = 0.0;
  long long c = 0;
  for (int k1 = 0; k1 < n1; ++k1) {
    s += psum[(size_t)k1 * NB + b];
    c += pcnt[(size_t)k1 * NB + b];
  }
  out[b] = c > 0 ? (float)(s / (double)c) : 0.f;
}

// 5-point Laplacian on the interior, FP64 arithmetic, stored as float.
template <typename TS>
__global__ __launch_bounds__(256) void laplacian_kernel(const TS *__restrict__ g, int n1, int n2,
                                                        float *__restrict__ L) {
  const int m2 = n2 - 2;
  const size_t total = (size_t)(n1 - 2) * m2;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / m2) + 1, j = (int)(e - (size_t)(i - 1) * m2) + 1;
    const size_t o = (size_t)i * n2 + j;
    const double v = (double)g[o - n2] + (double)g[o + n2] + (double)g[o - 1] + (double)g[o + 1] -
                     4.0 * (double)g[o];
    L[e] = (float)v;
  }
}

// Radix selection (8-bit digits, most significant first) of the element of
// a given rank, on order-preserving 32-bit keys of floats.
struct Sel {
  unsigned prefix, mask, rank, pad;
  float med, mad;
};

__device__ __forceinline__ unsigned fkey(float f) {
  const unsigned u = __float_as_uint(f);
  return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(unsigned k) {
  const unsigned u = (k >> 31) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

__global__ void sel_init_kernel(Sel *sel, unsigned *hist, unsigned rank) {
  const int t = threadIdx.x;
  if (t < 256) hist[t] = 0u;
  if (t == 0) {
    sel->prefix = 0u;
    sel->mask = 0u;
    sel->rank = rank;
  }
}

// mode 0: keys of L; mode 1: keys of |L - med|
__global__ __launch_bounds__(256) void sel_hist_kernel(const float *__restrict__ L, size_t N,
                                                       int mode, const Sel *__restrict__ sel,
                                                       unsigned *__restrict__ hist, int shift) {
  __shared__ unsigned lh[256];
  lh[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned prefix = sel->prefix, mask = sel->mask;
  const float med = sel->med;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (size_t)gridDim.x * blockDim.x) {
    const float v = mode == 0 ? L[e] : fabsf(L[e] - med);
    const unsigned k = fkey(v);
    if ((k & mask) == prefix) atomicAdd(&lh[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  const unsigned c = lh[threadIdx.x];
  if (c) atomicAdd(&hist[threadIdx.x], c);
}

// One digit: find the bucket holding the wanted rank, narrow the prefix,
// clear the histogram; after the last digit store the selected value.
__global__ void sel_pick_kernel(Sel *sel, unsigned *hist, int shift, int mode, int last,
                                unsigned next_rank) {
  if (threadIdx.x != 0) return;
  unsigned cum = 0, rank = sel->rank;
  for (int d = 0; d < 256; ++d) {
    const unsigned c = hist[d];
    if (rank < cum + c) {
      sel->prefix |= (unsigned)d << shift;
      sel->mask |= 255u << shift;
      sel->rank = rank - cum;
      break;
    }
    cum += c;
  }
  for (int d = 0; d < 256; ++d) hist[d] = 0u;
  if (last) {
    const float v = fkey_inv(sel->prefix);
    if (mode == 0) {
      sel->med = v;
      sel->prefix = 0u;
      sel->mask = 0u;
      sel->rank = next_rank;
    } else {
      sel->mad = v;
    }
  }
}

__global__ void noise_final_kernel(const Sel *__restrict__ sel, const double *__restrict__ gn2,
                                   double npx, float *__restrict__ out) {
  if (threadIdx.x != 0) return;
  const double sigma = (double)sel->mad / 0.6745 / sqrt(20.0);
  out[0] = (float)log(sigma * sqrt(npx) / sqrt(gn2[0]));
}

// ------------------------------------------------------------ gains filter

// Eigenvalue bins: edges beta_j = 10^(-4 + j / 16), j = 1..63 (computed on
// the host, passed by value), ebin(lambda) = #{j : |lambda| >= beta_j}.
struct EEdges {
  double b[NB - 1];
};

EEdges eedges() {
  EEdges e;
  for (int j = 1; j < NB; ++j) e.b[j - 1] = std::pow(10.0, -4.0 + j / 16.0);
  return e;
}

__device__ __forceinline__ int ebin(double l, const EEdges &E) {
  const double a = fabs(l);
  int k = 0;
#pragma unroll
  for (int j = 0; j < NB - 1; ++j) k += a >= E.b[j] ? 1 : 0;
  return k;
}

// d = 1 / (lambda^2 + a_b), a_b = 10^(-6 + 6 g_b), b = ebin(lambda); FP64.
template <typename T>
__global__ __launch_bounds__(256) void gains_filter_kernel(const double *__restrict__ lam,
                                                           const float *__restrict__ gains,
                                                           EEdges E, size_t total,
                                                           double *__restrict__ d64,
                                                           T *__restrict__ d) {
  __shared__ double a[NB];
  if (threadIdx.x < NB) a[threadIdx.x] = exp10(-6.0 + 6.0 * (double)gains[threadIdx.x]);
  __syncthreads();
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const double l = lam[e];
    const double v = 1.0 / (l * l + a[ebin(l, E)]);
    d64[e] = v;
    d[e] = T(v);
  }
}

// Label of the plan's filter: g_b = (log10(clip(a_b, 1e-6, 1)) + 6) / 6 with
// a_b = 1 / d(c_b) - c_b^2 at the bin centre c_b = 10^(-4 + (b + 1/2) / 16).
__global__ void gains_label_kernel(int kind, double param, const float *__restrict__ gains,
                                   float *__restrict__ label) {
  const int b = threadIdx.x;
  if (b >= NB) return;
  const double c = exp10(-4.0 + (b + 0.5) / 16.0);
  double a;
  if (kind == AR_FILTER_TIKHONOV) a = param;
  else if (kind == AR_FILTER_THRESHOLD) a = c >= param ? 0.0 : 1.0 - c * c;
  else if (kind == AR_FILTER_GAINS) a = exp10(-6.0 + 6.0 * (double)gains[b]);
  else a = 1.0 - c * c;  // identity: d = 1
  a = a < 1e-6 ? 1e-6 : (a > 1.0 ? 1.0 : a);
  label[b] = (float)((log10(a) + 6.0) / 6.0);
}

// Learned-filter scratch of a plan: [psum n1*64 doubles][pcnt n1*64 ints]
// [Sel][hist 256][g partials kElemMax doubles][g norm^2]
constexpr int kElemMax = 1024;
struct LScr {
  double *psum;
  int *pcnt;
  Sel *sel;
  unsigned *hist;
  double *gpart, *gn2;
};
size_t lscr_bytes(int n1) {
  return (size_t)n1 * NB * (sizeof(double) + sizeof(int)) + 256 + 256 * 4 +
         (kElemMax + 8) * sizeof(double) + 256;
}
LScr lscr_view(const ar_plan_s *p) {
  unsigned char *b = static_cast<unsigned char *>(p->lscr);
  LScr s;
  s.psum = reinterpret_cast<double *>(b);
  b += (size_t)p->n1 * NB * sizeof(double);
  s.pcnt = reinterpret_cast<int *>(b);
  b += (size_t)p->n1 * NB * sizeof(int);
  b = reinterpret_cast<unsigned char *>(((uintptr_t)b + 255) & ~(uintptr_t)255);
  s.sel = reinterpret_cast<Sel *>(b);
  b += 256;
  s.hist = reinterpret_cast<unsigned *>(b);
  b += 256 * 4;
  s.gpart = reinterpret_cast<double *>(b);
  s.gn2 = s.gpart + kElemMax;
  return s;
}
int ensure_lscr(ar_plan_s *p) {
  if (p->lscr) return AR_OK;
  AR_HIP(hipMalloc(&p->lscr, lscr_bytes(p->n1)));
  return AR_OK;
}

int profile_launch(ar_plan_s *p, float *out, hipStream_t st) {
  const LScr s = lscr_view(p);
  hipLaunchKernelGGL(profile_rows_kernel, dim3(p->n1), dim3(256), 0, st, p->lambda, p->n1, p->n2,
                     s.psum, s.pcnt);
  AR_HIP(hipGetLastError());
  hipLaunchKernelGGL(profile_final_kernel, dim3(1), dim3(NB), 0, st, s.psum, s.pcnt, p->n1, out);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

// ------------------------------------------------------------ network

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline unsigned short bf16_rne(float f) {
  unsigned u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

constexpr int kRowsW = 16;          // batch rows per wave
constexpr int kWaves = 2;           // waves per workgroup
constexpr int kPitch = NH + 4;      // LDS row pitch of the activation buffers (floats)

// One layer of 16 rows on the wave's LDS activations: Z = A W^T + b with
// A split into BF16 hi + lo terms and W in BF16 (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation); act 0 = ReLU, 1 = sigmoid.  Lane l holds A[l % 16][4 (l / 16) + e],
// B[4 (l / 16) + e][l % 16] and D[4 (l / 16) + e][l % 16], e = 0..3.
__device__ __forceinline__ void mlp_layer(const float *Ain, float *Aout, int K, int N,
                                          const unsigned short *__restrict__ W,
                                          const float *__restrict__ bias, int act, int lane,
                                          float *__restrict__ zsave, float *__restrict__ ysave,
                                          int row0, int batch, int ldz) {
  const int li = lane & 15, lk = (lane >> 4) * 4;
  const int KS = (K + 15) / 16;
  for (int nt = 0; nt < N / 16; ++nt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int ncol = nt * 16 + li;
    for (int ks = 0; ks < KS; ++ks) {
      s4 ahi, alo, bw;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = ks * 16 + lk + e;
        const float a = k < K ? Ain[li * kPitch + k] : 0.f;
        const unsigned short h = bf16_rne(a);
        const unsigned short lo = bf16_rne(a - bf16_to_f(h));
        ahi[e] = (short)h;
        alo[e] = (short)lo;
        bw[e] = (short)(k < K ? W[(size_t)ncol * K + k] : 0);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bw, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bw, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = lk + e;  // row within the wave's 16
      const float z = acc[e] + bias[ncol];
      const float h = act == 0 ? fmaxf(z, 0.f) : 1.f / (1.f + expf(-z));
      Aout[i * kPitch + ncol] = h;
      const int row = row0 + i;
      if (row < batch) {
        if (zsave) zsave[(size_t)row * ldz + ncol] = z;
        if (ysave) ysave[(size_t)row * ldz + ncol] = h;
      }
    }
  }
}

// Forward pass; with z1/z2 the pre-activations of the hidden layers are
// kept for the backward pass.
__global__ __launch_bounds__(64 * kWaves) void mlp_forward_kernel(
    const float *__restrict__ X, int batch, const unsigned short *__restrict__ wb,
    const float *__restrict__ theta, float *__restrict__ Y, float *__restrict__ z1,
    float *__restrict__ z2) {
  __shared__ float buf[kWaves][2][kRowsW * kPitch];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * kWaves + wave) * kRowsW;
  float *A = buf[wave][0], *Bf = buf[wave][1];
  for (int e = lane; e < kRowsW * NIN; e += 64) {
    const int i = e / NIN, k = e - i * NIN;
    const int row = row0 + i;
    A[i * kPitch + k] = row < batch ? X[(size_t)row * NIN + k] : 0.f;
  }
  __syncthreads();
  mlp_layer(A, Bf, NIN, NH, wb + OW1, theta + OB1, 0, lane, z1, nullptr, row0, batch, NH);
  __syncthreads();
  mlp_layer(Bf, A, NH, NH, wb + OW2, theta + OB2, 0, lane, z2, nullptr, row0, batch, NH);
  __syncthreads();
  mlp_layer(A, Bf, NH, NB, wb + OW3, theta + OB3, 1, lane, nullptr, Y, row0, batch, NB);
}

// Backward pass, per batch row: dZ3 = 2 (y - t) / (B 64) y (1 - y),
// dZ2 = (dZ3 W3) [z2 > 0], dZ1 = (dZ2 W2) [z1 > 0] (FP32, BF16 weights).
__global__ __launch_bounds__(NH) void mlp_back_rows_kernel(
    const float *__restrict__ Y, const float *__restrict__ Tt, const float *__restrict__ z1,
    const float *__restrict__ z2, const unsigned short *__restrict__ wb, int batch,
    float *__restrict__ dz1, float *__restrict__ dz2, float *__restrict__ dz3,
    float *__restrict__ lossrow) {
  __shared__ float s3[NB], s2[NH], red[NH];
  const int b = blockIdx.x, t = threadIdx.x;
  const float scale = 2.f / ((float)batch * (float)NB);
  float sq = 0.f;
  if (t < NB) {
    const float y = Y[(size_t)b * NB + t], e = y - Tt[(size_t)b * NB + t];
    sq = e * e;
    const float g = scale * e * y * (1.f - y);
    s3[t] = g;
    dz3[(size_t)b * NB + t] = g;
  }
  red[t] = sq;
  __syncthreads();
  float acc = 0.f;
  for (int o = 0; o < NB; ++o) acc += s3[o] * bf16_to_f(wb[OW3 + o * NH + t]);
  const float g2 = z2[(size_t)b * NH + t] > 0.f ? acc : 0.f;
  s2[t] = g2;
  dz2[(size_t)b * NH + t] = g2;
  __syncthreads();
  acc = 0.f;
  for (int o = 0; o < NH; ++o) acc += s2[o] * bf16_to_f(wb[OW2 + o * NH + t]);
  dz1[(size_t)b * NH + t] = z1[(size_t)b * NH + t] > 0.f ? acc : 0.f;
  if (t == 0) {
    float s = 0.f;
    for (int k = 0; k < NB; ++k) s += red[k];
    lossrow[b] = s;
  }
}

// Weight and bias gradients: sum over the batch in row order.
__global__ __launch_bounds__(256) void mlp_back_params_kernel(
    const float *__restrict__ X, const float *__restrict__ z1, const float *__restrict__ z2,
    const float *__restrict__ dz1, const float *__restrict__ dz2, const float *__restrict__ dz3,
    int batch, float *__restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NPAR) return;
  const float *dz, *hin;
  int o, i = -1, nout, nin;
  bool relu;
  if (e < OB1) { o = e / NIN; i = e - o * NIN; dz = dz1; hin = X; nout = NH; nin = NIN; relu = false; }
  else if (e < OW2) { o = e - OB1; dz = dz1; hin = X; nout = NH; nin = NIN; relu = false; }
  else if (e < OB2) { const int r = e - OW2; o = r / NH; i = r - o * NH; dz = dz2; hin = z1; nout = NH; nin = NH; relu = true; }
  else if (e < OW3) { o = e - OB2; dz = dz2; hin = z1; nout = NH; nin = NH; relu = true; }
  else if (e < OB3) { const int r = e - OW3; o = r / NH; i = r - o * NH; dz = dz3; hin = z2; nout = NB; nin = NH; relu = true; }
  else { o = e - OB3; dz = dz3; hin = z2; nout = NB; nin = NH; relu = true; }
  float acc = 0.f;
  for (int b = 0; b < batch; ++b) {
    const float d = dz[(size_t)b * nout + o];
    float h = 1.f;
    if (i >= 0) {
      h = hin[(size_t)b * nin + i];
      if (relu) h = fmaxf(h, 0.f);
    }
    acc += d * h;
  }
  grad[e] = acc;
}

__global__ void loss_final_kernel(const float *__restrict__ lossrow, int batch,
                                  float *__restrict__ loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < batch; ++b) s += lossrow[b];
  *loss = (float)(s / ((double)batch * NB));
}

// Adam with bias correction (c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t));
// refreshes the BF16 copy of every parameter.
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ theta, float *__restrict__ m,
                                                   float *__restrict__ v,
                                                   const float *__restrict__ g,
                                                   unsigned short *__restrict__ wb, float lr,
                                                   float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NPAR) return;
  const float ge = g[e];
  const float me = 0.9f * m[e] + 0.1f * ge;
  const float ve = 0.999f * v[e] + 0.001f * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float th = theta[e] - lr * (me * c1) / (sqrtf(ve * c2) + 1e-8f);
  theta[e] = th;
  wb[e] = bf16_rne(th);
}

__global__ void to_bf16_kernel(const float *__restrict__ theta, unsigned short *__restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NPAR) wb[e] = bf16_rne(theta[e]);
}

}  // namespace

int gains_filter_launch(ar_plan_s *p, const float *gains, hipStream_t st) {
  if (!p->gains) AR_HIP(hipMalloc((void **)&p->gains, NB * sizeof(float)));
  if (gains != p->gains)
    AR_HIP(hipMemcpyAsync(p->gains, gains, NB * sizeof(float), hipMemcpyDeviceToDevice, st));
  const size_t total = (size_t)p->n1 * p->n2;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  const EEdges E = eedges();
  if (p->csize == 8)
    hipLaunchKernelGGL(gains_filter_kernel<double>, dim3(blocks), dim3(256), 0, st, p->lambda,
                       p->gains, E, total, p->d64, static_cast<double *>(p->d));
  else
    hipLaunchKernelGGL(gains_filter_kernel<float>, dim3(blocks), dim3(256), 0, st, p->lambda,
                       p->gains, E, total, p->d64, static_cast<float *>(p->d));
  AR_HIP(hipGetLastError());
  p->filter = AR_FILTER_GAINS;
  p->filter_param = 0.0;
  return filter_transpose_launch(p, st);
}

}  // namespace ar

using namespace ar;

// ------------------------------------------------------------ C ABI

extern "C" int ar_features(ar_plan_t p, const void *g, float *feat_dev, void *stream) {
  if (!p || !g || !feat_dev) return fail(AR_EINVAL, "ar_features: null argument");
  if (p->bc != AR_BC_ANTIREFLECTIVE)
    return fail(AR_EUNSUPPORTED, "ar_features: the learned filter is Anti-Reflective only");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ensure_lscr(p);
  if (rc != AR_OK) return rc;
  const LScr s = lscr_view(p);
  if ((rc = profile_launch(p, feat_dev, st)) != AR_OK) return rc;
  // noise estimate: Laplacian into the plan's residual scratch (as float)
  const size_t N = (size_t)(p->n1 - 2) * (p->n2 - 2);
  float *L = static_cast<float *>(p->r);
  const int lb = (int)std::min<size_t>((N + 255) / 256, 4096);
  if (p->dtype == AR_F64)
    hipLaunchKernelGGL(laplacian_kernel<double>, dim3(lb), dim3(256), 0, st,
                       static_cast<const double *>(g), p->n1, p->n2, L);
  else
    hipLaunchKernelGGL(laplacian_kernel<float>, dim3(lb), dim3(256), 0, st,
                       static_cast<const float *>(g), p->n1, p->n2, L);
  AR_HIP(hipGetLastError());
  const unsigned rank = (unsigned)((N - 1) / 2);
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, st, s.sel, s.hist, rank);
  AR_HIP(hipGetLastError());
  const int hb = (int)std::min<size_t>((N + 255) / 256, 1024);
  for (int mode = 0; mode < 2; ++mode)
    for (int d = 3; d >= 0; --d) {
      hipLaunchKernelGGL(sel_hist_kernel, dim3(hb), dim3(256), 0, st, L, N, mode, s.sel, s.hist,
                         8 * d);
      AR_HIP(hipGetLastError());
      hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(64), 0, st, s.sel, s.hist, 8 * d, mode,
                         d == 0 ? 1 : 0, rank);
      AR_HIP(hipGetLastError());
    }
  int nb = 0;
  if ((rc = sumsq_launch(p, g, s.gpart, &nb, st)) != AR_OK) return rc;
  if (nb > kElemMax) return fail(AR_EUNSUPPORTED, "ar_features: too many partial sums");
  if ((rc = reduce_rows_launch(s.gpart, 1, nb, s.gn2, st)) != AR_OK) return rc;
  hipLaunchKernelGGL(noise_final_kernel, dim3(1), dim3(64), 0, st, s.sel, s.gn2,
                     (double)p->n1 * p->n2, feat_dev + NB);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

extern "C" int ar_precond_set_gains(ar_plan_t p, const float *gains_dev, void *stream) {
  if (!p || !gains_dev) return fail(AR_EINVAL, "ar_precond_set_gains: null argument");
  if (p->bc != AR_BC_ANTIREFLECTIVE)
    return fail(AR_EUNSUPPORTED, "ar_precond_set_gains: the learned filter is Anti-Reflective only");
  AR_HIP(hipSetDevice(p->device));
  return gains_filter_launch(p, gains_dev, static_cast<hipStream_t>(stream));
}

extern "C" int ar_gains_label(ar_plan_t p, float *label_dev, void *stream) {
  if (!p || !label_dev) return fail(AR_EINVAL, "ar_gains_label: null argument");
  AR_HIP(hipSetDevice(p->device));
  hipLaunchKernelGGL(gains_label_kernel, dim3(1), dim3(NB), 0, static_cast<hipStream_t>(stream),
                     p->filter, p->filter_param, p->gains, label_dev);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

struct ar_fnet_s {
  int device = 0;
  int t = 0;               // Adam step counter
  float *theta = nullptr;  // FP32 master parameters
  float *m = nullptr, *v = nullptr, *grad = nullptr;
  unsigned short *wb = nullptr;  // BF16 copies
  // per-batch buffers (grown on demand)
  int cap = 0;
  float *y = nullptr, *z1 = nullptr, *z2 = nullptr, *dz1 = nullptr, *dz2 = nullptr,
        *dz3 = nullptr, *lossrow = nullptr, *loss = nullptr;
};

static void fnet_free_batch(ar_fnet_s *n) {
  float *bufs[] = {n->y, n->z1, n->z2, n->dz1, n->dz2, n->dz3, n->lossrow, n->loss};
  for (float *b : bufs)
    if (b) (void)hipFree(b);
  n->y = n->z1 = n->z2 = n->dz1 = n->dz2 = n->dz3 = n->lossrow = n->loss = nullptr;
  n->cap = 0;
}

static int fnet_ensure(ar_fnet_s *n, int batch) {
  if (batch <= n->cap) return AR_OK;
  fnet_free_batch(n);
  const size_t B = (size_t)batch;
  AR_HIP(hipMalloc((void **)&n->y, B * NB * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->z1, B * NH * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->z2, B * NH * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->dz1, B * NH * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->dz2, B * NH * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->dz3, B * NB * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->lossrow, B * sizeof(float)));
  AR_HIP(hipMalloc((void **)&n->loss, sizeof(float)));
  n->cap = batch;
  return AR_OK;
}

static void fnet_free(ar_fnet_s *n) {
  fnet_free_batch(n);
  void *bufs[] = {n->theta, n->m, n->v, n->grad, n->wb};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete n;
}

extern "C" int ar_fnet_create(ar_fnet_t *out, const float *params_host, int device) {
  if (!out) return fail(AR_EINVAL, "ar_fnet_create: null output");
  *out = nullptr;
  if (!params_host) return fail(AR_EINVAL, "ar_fnet_create: null parameters");
  for (int e = 0; e < NPAR; ++e)
    if (!std::isfinite(params_host[e])) return fail(AR_EINVAL, "ar_fnet_create: non-finite parameter");
  int ndev = 0;
  AR_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AR_EINVAL, "ar_fnet_create: bad device");
  AR_HIP(hipSetDevice(device));
  ar_fnet_s *n = new ar_fnet_s();
  n->device = device;
  hipError_t e = hipMalloc((void **)&n->theta, NPAR * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&n->m, NPAR * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&n->v, NPAR * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&n->grad, NPAR * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&n->wb, NPAR * sizeof(unsigned short));
  if (e == hipSuccess) e = hipMemcpy(n->theta, params_host, NPAR * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->m, 0, NPAR * sizeof(float));
  if (e == hipSuccess) e = hipMemset(n->v, 0, NPAR * sizeof(float));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, nullptr, n->theta,
                       n->wb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    const int rc = hip_fail(e, "ar_fnet_create");
    fnet_free(n);
    return rc;
  }
  *out = n;
  return AR_OK;
}

// Parameters from a NumPy .npy file holding one little-endian float32
// vector of AR_FNET_NPARAM entries (format versions 1.0 to 3.0, C order).
static int read_npy_params(const char *path, std::vector<float> &out) {
  FILE *fh = std::fopen(path, "rb");
  if (!fh) return fail(AR_EINVAL, std::string("ar_fnet_load: cannot open ") + path);
  std::vector<unsigned char> buf;
  unsigned char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), fh)) > 0) buf.insert(buf.end(), chunk, chunk + got);
  std::fclose(fh);
  static const unsigned char magic[6] = {0x93, 'N', 'U', 'M', 'P', 'Y'};
  if (buf.size() < 10 || std::memcmp(buf.data(), magic, 6) != 0)
    return fail(AR_EINVAL, "ar_fnet_load: not a .npy file");
  const int major = buf[6];
  size_t hlen, hoff;
  if (major == 1) {
    hlen = buf[8] | (size_t)buf[9] << 8;
    hoff = 10;
  } else if (major == 2 || major == 3) {
    if (buf.size() < 12) return fail(AR_EINVAL, "ar_fnet_load: truncated .npy header");
    hlen = buf[8] | (size_t)buf[9] << 8 | (size_t)buf[10] << 16 | (size_t)buf[11] << 24;
    hoff = 12;
  } else {
    return fail(AR_EINVAL, "ar_fnet_load: unsupported .npy version");
  }
  if (hoff + hlen > buf.size()) return fail(AR_EINVAL, "ar_fnet_load: truncated .npy header");
  std::string h(buf.begin() + hoff, buf.begin() + hoff + hlen);
  std::string compact;
  for (char c : h)
    if (c != ' ') compact += c;
  const std::string shape = "'shape':(" + std::to_string(NPAR) + ",)";
  if (compact.find("'descr':'<f4'") == std::string::npos ||
      compact.find("'fortran_order':False") == std::string::npos ||
      compact.find(shape) == std::string::npos)
    return fail(AR_EINVAL, "ar_fnet_load: expected a C-order <f4 vector of AR_FNET_NPARAM entries");
  const size_t data = hoff + hlen;
  if (buf.size() - data != (size_t)NPAR * sizeof(float))
    return fail(AR_EINVAL, "ar_fnet_load: wrong data size");
  out.resize(NPAR);
  std::memcpy(out.data(), buf.data() + data, (size_t)NPAR * sizeof(float));
  return AR_OK;
}

extern "C" int ar_fnet_load(ar_fnet_t *out, const char *weights_path, int device) {
  if (!out) return fail(AR_EINVAL, "ar_fnet_load: null output");
  *out = nullptr;
  if (!weights_path) return fail(AR_EINVAL, "ar_fnet_load: null path");
  std::vector<float> params;
  const int rc = read_npy_params(weights_path, params);
  if (rc != AR_OK) return rc;
  return ar_fnet_create(out, params.data(), device);
}

extern "C" int ar_fnet_destroy(ar_fnet_t n) {
  if (!n) return AR_OK;
  AR_HIP(hipSetDevice(n->device));
  (void)hipDeviceSynchronize();
  fnet_free(n);
  return AR_OK;
}

extern "C" int ar_fnet_get_params(ar_fnet_t n, float *params_host) {
  if (!n || !params_host) return fail(AR_EINVAL, "ar_fnet_get_params: null argument");
  AR_HIP(hipSetDevice(n->device));
  AR_HIP(hipDeviceSynchronize());
  AR_HIP(hipMemcpy(params_host, n->theta, NPAR * sizeof(float), hipMemcpyDeviceToHost));
  return AR_OK;
}

static int fnet_forward(ar_fnet_s *n, const float *x, float *y, int batch, bool keep,
                        hipStream_t st) {
  const int rows = kWaves * kRowsW;
  const int blocks = (batch + rows - 1) / rows;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(64 * kWaves), 0, st, x, batch, n->wb,
                     n->theta, y, keep ? n->z1 : nullptr, keep ? n->z2 : nullptr);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

extern "C" int ar_fnet_infer(ar_fnet_t n, const float *x_dev, float *y_dev, int batch,
                             void *stream) {
  if (!n || !x_dev || !y_dev) return fail(AR_EINVAL, "ar_fnet_infer: null argument");
  if (batch < 1) return fail(AR_EINVAL, "ar_fnet_infer: batch < 1");
  AR_HIP(hipSetDevice(n->device));
  return fnet_forward(n, x_dev, y_dev, batch, false, static_cast<hipStream_t>(stream));
}

static int fnet_grad(ar_fnet_s *n, const float *x, const float *t, int batch, float *grad,
                     float *loss, hipStream_t st) {
  int rc = fnet_ensure(n, batch);
  if (rc != AR_OK) return rc;
  if ((rc = fnet_forward(n, x, n->y, batch, true, st)) != AR_OK) return rc;
  hipLaunchKernelGGL(mlp_back_rows_kernel, dim3(batch), dim3(NH), 0, st, n->y, t, n->z1, n->z2,
                     n->wb, batch, n->dz1, n->dz2, n->dz3, n->lossrow);
  AR_HIP(hipGetLastError());
  hipLaunchKernelGGL(mlp_back_params_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, x, n->z1,
                     n->z2, n->dz1, n->dz2, n->dz3, batch, grad);
  AR_HIP(hipGetLastError());
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, n->lossrow, batch,
                     loss ? loss : n->loss);
  AR_HIP(hipGetLastError());
  return AR_OK;
}

extern "C" int ar_fnet_grad(ar_fnet_t n, const float *x_dev, const float *t_dev, int batch,
                            float *grad_dev, float *loss_dev, void *stream) {
  if (!n || !x_dev || !t_dev || !grad_dev) return fail(AR_EINVAL, "ar_fnet_grad: null argument");
  if (batch < 1) return fail(AR_EINVAL, "ar_fnet_grad: batch < 1");
  AR_HIP(hipSetDevice(n->device));
  return fnet_grad(n, x_dev, t_dev, batch, grad_dev, loss_dev, static_cast<hipStream_t>(stream));
}

extern "C" int ar_fnet_train_step(ar_fnet_t n, const float *x_dev, const float *t_dev, int batch,
                                  float lr, float *loss_dev, void *stream) {
  if (!n || !x_dev || !t_dev) return fail(AR_EINVAL, "ar_fnet_train_step: null argument");
  if (batch < 1) return fail(AR_EINVAL, "ar_fnet_train_step: batch < 1");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(AR_EINVAL, "ar_fnet_train_step: bad lr");
  AR_HIP(hipSetDevice(n->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = fnet_grad(n, x_dev, t_dev, batch, n->grad, loss_dev, st);
  if (rc != AR_OK) return rc;
  n->t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, n->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, n->t)));
  hipLaunchKernelGGL(adam_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, n->theta, n->m, n->v,
                     n->grad, n->wb, lr, c1, c2);
  AR_HIP(hipGetLastError());
  return AR_OK;
}
