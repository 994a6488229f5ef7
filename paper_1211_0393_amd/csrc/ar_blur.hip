// AR-BC blur kernels: A x, A' r, A^T r (gfx950).
//
// The blur is the convolution g_i = sum_s h_s f_{i-s} (eq. (modello_discreto))
// of the image extended by anti-reflection (Sec. 2.2).  Each workgroup owns a
// TH x TW output tile; it stages the (TH + 2 q1) x (TW + 2 q2) input halo in
// LDS, computing ghost pixels on load from the AR rule (edges: 2 f_1 - f_{1+i};
// corners: the double anti-reflection 4, -2, -2, +1 obtained by applying the
// 1-D rule per axis).  Every thread then produces RY x RX outputs with a
// sliding window over input rows so that one LDS row feeds two output rows;
// PSF weights are workgroup-uniform: FP32 tiles broadcast them from an LDS
// copy, FP64 tiles read them with scalar loads.
//
// The same kernel computes
//   * A x          : weights rot180(H), AR extension, outputs on the FOV;
//   * A' r         : weights H (PSF rotated by 180 degrees, Sec. 4);
//   * C^T r of A^T : weights H, zero outside the FOV, outputs on the extended
//                    grid [-q, n-1+q]; a second kernel folds the ghosts back.
// With `gsub` it writes g - (A x) and per-workgroup FP64 partial sums of the
// squared residual.
#include "ar_halo.h"
#include "ar_internal.h"

namespace ar {
namespace {

constexpr int TX = 16, TY = 16, NT = TX * TY;
constexpr int RX = 4, RY = 2;
constexpr int TW = TX * RX;  // 64 output columns per tile
constexpr int TH = TY * RY;  // 32 output rows per tile

// Bijective remap of the workgroup id so that consecutive logical tiles run
// on the same XCD (workgroups are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, i = b >> 3;
  const int g8 = G >> 3, rem = G & 7;
  const int start = x * g8 + (x < rem ? x : rem);
  return start + i;
}

template <typename T>
__device__ __forceinline__ double block_sum(double v, double *red) {
  // fixed-order reduction: xor-shuffle inside each wave, then wave 0 adds
  // the four wave sums in order
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NT / 64; ++k) s += red[k];
  }
  return s;
}

// Ordering fence: the FMAs that produce `acc` complete before any later
// memory access is issued (the empty asm reads and writes the accumulators
// and clobbers memory); it emits no instruction.
template <typename T, int N>
__device__ __forceinline__ void after(T (&acc)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) asm volatile("" : "+v"(acc[c])::"memory");
}

// TS: storage type of images; T: compute type of the halo tile, weights
// and accumulators (double for FP64 accumulation of FP32 images).
// Q2 >= 0: compile-time column half-width (tap loop fully unrolled).
// Q2 <  0: generic kernel with a runtime column half-width.
template <typename TS, typename T, typename TO, int Q2>
__device__ __forceinline__ void conv_tile(unsigned char *smem_raw, const TS *__restrict__ in,
                                          TO *__restrict__ out, const T *__restrict__ w, int n1,
                                          int n2, int q1, int q2rt, int o1, int o2, int m1, int m2,
                                          int ext_mode, const TS *__restrict__ gsub,
                                          double *__restrict__ partial_slot, int logical,
                                          int tiles_x) {
  constexpr bool GEN = Q2 < 0;
  const int q2 = GEN ? q2rt : Q2;
  const int KW = 2 * q2 + 1;
  const int LW = TW + 2 * q2;
  const int pitch = (LW + 3) & ~3;
  const int LH = TH + 2 * q1;
  T *tile = reinterpret_cast<T *>(smem_raw);
  const Gl<TS> *gin = gmem(in);
  const Gl<T> *gw = gmem(w);

  const int ty_tile = logical / tiles_x, tx_tile = logical - ty_tile * tiles_x;
  const int r0 = ty_tile * TH, c0 = tx_tile * TW;
  const int ib1 = o1 + r0 - q1, ib2 = o2 + c0 - q2;
  const int tid = threadIdx.x;
  const bool inside = ib1 >= 0 && ib2 >= 0 && ib1 + LH <= n1 && ib2 + LW <= n2;
  // stage the halo tile: 4 rows x 64 columns of threads per sweep; each
  // thread first loads a chunk of its elements into registers (clamped,
  // unconditional addresses) and then stores them, so a chunk costs one
  // memory latency instead of one per element
  const int lr = tid >> 6, lc = tid & 63;
  constexpr int CR = 6, CC = 2;  // rows x column-sweeps per chunk
  // the PSF copy for LDS is loaded first, so that its latency overlaps
  // the halo loads
  constexpr int WPT = 4;
  const int P = (2 * q1 + 1) * KW;
  T wpre[WPT];
  constexpr bool kLdsW = !GEN && sizeof(T) != 8;  // weights staged in LDS
  if constexpr (kLdsW) {
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int e = tid + NT * i;
      wpre[i] = gw[e < P ? e : 0];
    }
  }
  for (int a0 = lr; a0 < LH; a0 += 4 * CR) {
    for (int c0 = lc; c0 < LW; c0 += 64 * CC) {
      T vals[CR][CC];
      if (inside) {
#pragma unroll
        for (int i = 0; i < CR; ++i) {
          const int a = a0 + 4 * i < LH ? a0 + 4 * i : a0;
          const Gl<TS> *src = gin + (size_t)(ib1 + a) * n2 + ib2;
#pragma unroll
          for (int j = 0; j < CC; ++j) {
            const int c = c0 + 64 * j < LW ? c0 + 64 * j : c0;
            vals[i][j] = T(src[c]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < CR; ++i)
#pragma unroll
          for (int j = 0; j < CC; ++j)
            vals[i][j] = load_ext<T, TS>(gin, n1, n2, q1, q2, ib1 + a0 + 4 * i, ib2 + c0 + 64 * j,
                                         ext_mode);
      }
#pragma unroll
      for (int i = 0; i < CR; ++i)
#pragma unroll
        for (int j = 0; j < CC; ++j) {
          const int a = a0 + 4 * i, c = c0 + 64 * j;
          if (a < LH && c < LW) tile[a * pitch + c] = vals[i][j];
        }
    }
  }
  if constexpr (kLdsW) {
    T *swr = tile + (size_t)LH * pitch;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int e = tid + NT * i;
      if (e < P) swr[e] = wpre[i];
    }
    for (int e = tid + NT * WPT; e < P; e += NT) swr[e] = gw[e];
  }
  __syncthreads();

  const int tx = tid % TX, ty = tid / TX;
  const int lx = tx * RX, ly = ty * RY;
  T acc0[RX], acc1[RX];
#pragma unroll
  for (int c = 0; c < RX; ++c) { acc0[c] = T(0); acc1[c] = T(0); }

  const int krows = 2 * q1 + 2;
  if constexpr (!GEN) {
    // Software-pipelined sliding window: input row k feeds output row 0
    // with PSF row k and output row 1 with PSF row k - 1.  Rows are taken
    // two at a time (krows = 2 q1 + 2 is even) with ping-pong buffers for
    // the input rows (va, vb) and the PSF rows (wa, wb), so no register
    // copies rotate the window: the next input row is issued before the
    // current row's FMAs, and a PSF row buffer is refilled (broadcast reads
    // of the LDS weight copy) right after its last use.  `after` pins each
    // refill behind the FMAs that read the old contents (a hoisted load needs
    // a third buffer and register copies at the loop edge); indices are
    // clamped.
    constexpr int KWc = 2 * Q2 + 1;
    constexpr int NV = RX + 2 * Q2;
    const T *sw = tile + (size_t)LH * pitch;
    // FP64 tiles read their weights with scalar loads straight from the
    // weight array (workgroup-uniform addresses), which keeps them out of
    // the vector registers and the LDS port; FP32 tiles broadcast them from
    // the LDS copy
    auto wt = [&](int e) -> T {
      if constexpr (sizeof(T) == 8) return gw[e];
      else return sw[e];
    };
    const int klast = 2 * q1;
    T va[NV], vb[NV], wa[KWc], wb[KWc];
    {
      const T *rowp = tile + ly * pitch + lx;
#pragma unroll
      for (int t = 0; t < NV; ++t) va[t] = rowp[t];
#pragma unroll
      for (int b = 0; b < KWc; ++b) wa[b] = wt(b);
    }
    for (int k = 0; k < krows; k += 2) {
      // row k: input in va, PSF row k in wa, PSF row k - 1 in wb
      {
        const T *rowp = tile + (ly + k + 1) * pitch + lx;
#pragma unroll
        for (int t = 0; t < NV; ++t) vb[t] = rowp[t];
      }
      if (k >= 1) {
#pragma unroll
        for (int b = 0; b < KWc; ++b)
#pragma unroll
          for (int c = 0; c < RX; ++c) acc1[c] = fma(wb[b], va[c + b], acc1[c]);
      }
      after(acc1);
      {
        const int wn = k + 1 <= klast ? k + 1 : klast;
#pragma unroll
        for (int b = 0; b < KWc; ++b) wb[b] = wt(wn * KWc + b);
      }
#pragma unroll
      for (int b = 0; b < KWc; ++b)
#pragma unroll
        for (int c = 0; c < RX; ++c) acc0[c] = fma(wa[b], va[c + b], acc0[c]);
      // row k + 1: input in vb, PSF row k + 1 in wb, PSF row k in wa
      after(acc0);
      {
        const int kn = k + 2 < krows ? k + 2 : krows - 1;
        const T *rowp = tile + (ly + kn) * pitch + lx;
#pragma unroll
        for (int t = 0; t < NV; ++t) va[t] = rowp[t];
      }
#pragma unroll
      for (int b = 0; b < KWc; ++b)
#pragma unroll
        for (int c = 0; c < RX; ++c) acc1[c] = fma(wa[b], vb[c + b], acc1[c]);
      after(acc1);
      {
        const int wn = k + 2 <= klast ? k + 2 : klast;
#pragma unroll
        for (int b = 0; b < KWc; ++b) wa[b] = wt(wn * KWc + b);
      }
      if (k + 1 <= klast) {
#pragma unroll
        for (int b = 0; b < KWc; ++b)
#pragma unroll
          for (int c = 0; c < RX; ++c) acc0[c] = fma(wb[b], vb[c + b], acc0[c]);
      }
      after(acc0);
    }
  } else {
    for (int k = 0; k < krows; ++k) {
      const T *rowp = tile + (ly + k) * pitch + lx;
      if (k <= 2 * q1) {
        const T *wr = w + k * KW;
        for (int b = 0; b < KW; ++b) {
          const T wb = wr[b];
#pragma unroll
          for (int c = 0; c < RX; ++c) acc0[c] = fma(wb, rowp[c + b], acc0[c]);
        }
      }
      if (k >= 1) {
        const T *wr = w + (k - 1) * KW;
        for (int b = 0; b < KW; ++b) {
          const T wb = wr[b];
#pragma unroll
          for (int c = 0; c < RX; ++c) acc1[c] = fma(wb, rowp[c + b], acc1[c]);
        }
      }
    }
  }

  double ss = 0.0;
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int oi = r0 + ly + r;
    if (oi >= m1) continue;
#pragma unroll
    for (int c = 0; c < RX; ++c) {
      const int oj = c0 + lx + c;
      if (oj >= m2) continue;
      T val = r == 0 ? acc0[c] : acc1[c];
      const size_t o = (size_t)oi * m2 + oj;
      if (gsub) {
        val = T(gmem(gsub)[o]) - val;
        const TO rs = TO(val);
        ss += (double)rs * (double)rs;
        gmem(out)[o] = rs;
      } else {
        gmem(out)[o] = TO(val);
      }
    }
  }
  if (partial_slot) {
    // the tile is no longer read: reuse LDS for the reduction
    double *red = reinterpret_cast<double *>(smem_raw);
    const double s = block_sum<T>(ss, red);
    if (tid == 0) *gmem(partial_slot) = s;
  }
}

template <typename TS, typename T, typename TO, int Q2>
__global__ __launch_bounds__(NT) void conv_kernel(
    const TS *__restrict__ in, TO *__restrict__ out, const T *__restrict__ w, int n1, int n2,
    int q1, int q2rt, int o1, int o2, int m1, int m2, int zero_ext, const TS *__restrict__ gsub,
    double *__restrict__ partial, int tiles_x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  conv_tile<TS, T, TO, Q2>(smem_raw, in, out, w, n1, n2, q1, q2rt, o1, o2, m1, m2, zero_ext, gsub,
                           partial ? partial + blockIdx.x : nullptr,
                           xcd_remap(blockIdx.x, gridDim.x), tiles_x);
}

// Batched form: workgroup b computes tile tiles[b].y of job tiles[b].x.
// ext_mode: correlation onto the zero-extended grid (the first half of A^T).
template <typename TS, typename T, typename TO, int Q2>
__global__ __launch_bounds__(NT) void conv_batch_kernel(const ConvJob *__restrict__ jobs,
                                                        const int2 *__restrict__ tiles, int k,
                                                        int ext_mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int2 jt = tiles[xcd_remap(blockIdx.x, gridDim.x)];
  const ConvJob J = jobs[jt.x];
  const int q2 = Q2 < 0 ? J.q2 : Q2;
  const int o1 = ext_mode ? -J.q1 : 0, o2 = ext_mode ? -q2 : 0;
  const int m1 = J.n1 - 2 * o1, m2 = J.n2 - 2 * o2;
  conv_tile<TS, T, TO, Q2>(smem_raw, static_cast<const TS *>(J.in), static_cast<TO *>(J.out),
                           static_cast<const T *>(J.w), J.n1, J.n2, J.q1, q2, o1, o2, m1, m2,
                           ext_mode, static_cast<const TS *>(J.gsub),
                           J.part ? J.part + (size_t)k * J.nblk + jt.y : nullptr, jt.y,
                           J.tiles_x);
}


// Fold of the extended-grid correlation back onto the FOV (transpose of the
// AR extension): along each axis a ghost at 1 - t adds 2x to position 1 and
// -1x to position 1 + t, a ghost at n + t adds 2x to n and -1x to n - t.
template <typename TS, typename T>
__device__ __forceinline__ void fold_at(const T *__restrict__ ext, TS *__restrict__ out, int n1,
                                        int n2, int q1, int q2) {
  const int j2 = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j1 = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (j1 >= n1 || j2 >= n2) return;
  const int W = n2 + 2 * q2;
  // per-axis lists (position on the extended grid, weight)
  int e1[40], e2[40];
  float w1[40], w2[40];
  int c1 = 0, c2 = 0;
  auto build = [](int j, int n, int q, int *e, float *wv, int &cnt) {
    e[cnt] = j; wv[cnt] = 1.f; ++cnt;
    if (j == 0)
      for (int t = 1; t <= q; ++t) { e[cnt] = -t; wv[cnt] = 2.f; ++cnt; }
    if (j >= 1 && j <= q) { e[cnt] = -j; wv[cnt] = -1.f; ++cnt; }
    if (j == n - 1)
      for (int t = 1; t <= q; ++t) { e[cnt] = n - 1 + t; wv[cnt] = 2.f; ++cnt; }
    if (j >= n - 1 - q && j <= n - 2) { e[cnt] = 2 * n - 2 - j; wv[cnt] = -1.f; ++cnt; }
  };
  build(j1, n1, q1, e1, w1, c1);
  build(j2, n2, q2, e2, w2, c2);
  T acc = T(0);
  for (int a = 0; a < c1; ++a) {
    const Gl<T> *row = gmem(ext) + (size_t)(e1[a] + q1) * W + q2;
    T s = T(0);
    for (int b = 0; b < c2; ++b) s += T(w2[b]) * row[e2[b]];
    acc += T(w1[a]) * s;
  }
  gmem(out)[(size_t)j1 * n2 + j2] = TS(acc);
}

template <typename TS, typename T>
__global__ __launch_bounds__(256) void fold_kernel(const T *__restrict__ ext, TS *__restrict__ out,
                                                   int n1, int n2, int q1, int q2) {
  fold_at<TS, T>(ext, out, n1, n2, q1, q2);
}

// Batched fold: blockIdx.z selects the job (in = extended grid, out = y).
template <typename TS, typename T>
__global__ __launch_bounds__(256) void fold_batch_kernel(const ConvJob *__restrict__ jobs) {
  const ConvJob J = jobs[blockIdx.z];
  fold_at<TS, T>(static_cast<const T *>(J.in), static_cast<TS *>(J.out), J.n1, J.n2, J.q1, J.q2);
}

template <typename TS, typename T, typename TO>
hipError_t launch_conv_t(const ar_plan_s *p, const void *in, void *out, const void *w, int o1,
                         int o2, int m1, int m2, bool zero_ext, const void *g, double *partial,
                         int blocks, int tiles_x, hipStream_t st) {
  const int q1 = p->q1, q2 = p->q2;
  const int LW = TW + 2 * q2, pitch = (LW + 3) & ~3, LH = TH + 2 * q1;
  size_t smem = ((size_t)LH * pitch + (size_t)(2 * q1 + 1) * (2 * q2 + 1)) * sizeof(T);
  if (smem < 64 * sizeof(double)) smem = 64 * sizeof(double);
  const TS *ti = static_cast<const TS *>(in);
  TO *to = static_cast<TO *>(out);
  const T *tw = static_cast<const T *>(w);
  const TS *tg = static_cast<const TS *>(g);
  const int ze = zero_ext ? EXT_ZERO : plan_ext_mode(p);
#define AR_CONV_CASE(QQ)                                                                      \
  case QQ:                                                                                    \
    hipLaunchKernelGGL((conv_kernel<TS, T, TO, QQ>), dim3(blocks), dim3(NT), smem, st, ti, to, \
                       tw, p->n1, p->n2, q1, q2, o1, o2, m1, m2, ze, tg, partial, tiles_x);   \
    break;
  switch (q2) {
    AR_CONV_CASE(0) AR_CONV_CASE(1) AR_CONV_CASE(2) AR_CONV_CASE(3) AR_CONV_CASE(4)
    AR_CONV_CASE(5) AR_CONV_CASE(6) AR_CONV_CASE(7) AR_CONV_CASE(8) AR_CONV_CASE(9)
    AR_CONV_CASE(10) AR_CONV_CASE(11) AR_CONV_CASE(12) AR_CONV_CASE(13) AR_CONV_CASE(14)
    AR_CONV_CASE(15)
    default:
      hipLaunchKernelGGL((conv_kernel<TS, T, TO, -1>), dim3(blocks), dim3(NT), smem, st, ti, to, tw,
                         p->n1, p->n2, q1, q2, o1, o2, m1, m2, ze, tg, partial, tiles_x);
  }
#undef AR_CONV_CASE
  return hipGetLastError();
}

template <typename TS, typename T, typename TO>
hipError_t launch_conv_batch_t(int q2, const ConvJob *jobs, const int2 *tiles, int ntiles, int k,
                               int ext_mode, size_t smem, hipStream_t st) {
  if (smem < 64 * sizeof(double)) smem = 64 * sizeof(double);
#define AR_CONVB_CASE(QQ)                                                                        \
  case QQ:                                                                                       \
    hipLaunchKernelGGL((conv_batch_kernel<TS, T, TO, QQ>), dim3(ntiles), dim3(NT), smem, st,     \
                       jobs, tiles, k, ext_mode);                                               \
    break;
  switch (q2) {
    AR_CONVB_CASE(0) AR_CONVB_CASE(1) AR_CONVB_CASE(2) AR_CONVB_CASE(3) AR_CONVB_CASE(4)
    AR_CONVB_CASE(5) AR_CONVB_CASE(6) AR_CONVB_CASE(7) AR_CONVB_CASE(8) AR_CONVB_CASE(9)
    AR_CONVB_CASE(10) AR_CONVB_CASE(11) AR_CONVB_CASE(12) AR_CONVB_CASE(13) AR_CONVB_CASE(14)
    AR_CONVB_CASE(15)
    default:
      hipLaunchKernelGGL((conv_batch_kernel<TS, T, TO, -1>), dim3(ntiles), dim3(NT), smem, st,
                         jobs, tiles, k, ext_mode);
  }
#undef AR_CONVB_CASE
  return hipGetLastError();
}

}  // namespace

int conv_tiles(int m1, int m2, int *tiles_x) {
  const int tx = (m2 + TW - 1) / TW;
  if (tiles_x) *tiles_x = tx;
  return ((m1 + TH - 1) / TH) * tx;
}

size_t conv_batch_smem(int dtype, int q1max, int q2) {
  const size_t cs = dtype == AR_F32 ? sizeof(float) : sizeof(double);
  const size_t LH = TH + 2 * (size_t)q1max, LW = TW + 2 * (size_t)q2;
  return (LH * ((LW + 3) & ~(size_t)3) + (2 * (size_t)q1max + 1) * (2 * q2 + 1)) * cs;
}

int conv_batch_launch(int dtype, int q2, const ConvJob *jobs, const int2 *tiles, int ntiles, int k,
                      bool ext_mode, size_t smem, hipStream_t st) {
  if (smem > 64 * 1024) return fail(AR_EUNSUPPORTED, "PSF too large for the LDS halo tile");
  if (ntiles == 0) return AR_OK;
  const int em = ext_mode ? 1 : 0;
  hipError_t e;
  if (dtype == AR_F64)
    e = launch_conv_batch_t<double, double, double>(q2, jobs, tiles, ntiles, k, em, smem, st);
  else if (dtype == AR_F32_ACC64 && ext_mode)
    e = launch_conv_batch_t<float, double, double>(q2, jobs, tiles, ntiles, k, em, smem, st);
  else if (dtype == AR_F32_ACC64)
    e = launch_conv_batch_t<float, double, float>(q2, jobs, tiles, ntiles, k, em, smem, st);
  else
    e = launch_conv_batch_t<float, float, float>(q2, jobs, tiles, ntiles, k, em, smem, st);
  if (e != hipSuccess) return hip_fail(e, "conv_batch_kernel launch");
  return AR_OK;
}

int fold_batch_launch(int dtype, const ConvJob *jobs, int count, int n1max, int n2max, int qmax,
                      hipStream_t st) {
  if (qmax > 36) return fail(AR_EUNSUPPORTED, "adjoint fold supports q <= 36");
  if (count == 0) return AR_OK;
  dim3 grid((n2max + 63) / 64, (n1max + 3) / 4, count);
  if (dtype == AR_F64)
    hipLaunchKernelGGL((fold_batch_kernel<double, double>), grid, dim3(256), 0, st, jobs);
  else if (dtype == AR_F32_ACC64)
    hipLaunchKernelGGL((fold_batch_kernel<float, double>), grid, dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL((fold_batch_kernel<float, float>), grid, dim3(256), 0, st, jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fold_batch_kernel launch");
  return AR_OK;
}

int conv_blocks(const ar_plan_s *p, int m1, int m2) {
  if (conv_mfma_ok(p) && m1 == p->n1 && m2 == p->n2) return conv_mfma_blocks(m1, m2);
  return ((m1 + TH - 1) / TH) * ((m2 + TW - 1) / TW);
}

int conv_launch(const ar_plan_s *p, const void *in, void *out, const void *w, int o1, int o2,
                int m1, int m2, bool zero_ext, const void *g_minus, double *partial,
                int *nblocks_out, hipStream_t st, bool out_compute) {
  if (conv_mfma_ok(p) && o1 == 0 && o2 == 0 && m1 == p->n1 && m2 == p->n2 && !zero_ext &&
      !out_compute && (w == p->w_fwd || w == p->w_rev)) {
    if (nblocks_out) *nblocks_out = conv_mfma_blocks(m1, m2);
    return conv_mfma_launch(p, in, out, w == p->w_rev, g_minus, partial, st);
  }
  const int tiles_x = (m2 + TW - 1) / TW;
  const int blocks = conv_blocks(p, m1, m2);
  const size_t LH = TH + 2 * (size_t)p->q1, LW = TW + 2 * (size_t)p->q2;
  if ((LH * ((LW + 3) & ~(size_t)3) + (2 * (size_t)p->q1 + 1) * (2 * p->q2 + 1)) * p->csize >
      64 * 1024)
    return fail(AR_EUNSUPPORTED, "PSF too large for the LDS halo tile");
  if (nblocks_out) *nblocks_out = blocks;
  hipError_t e;
  if (p->dtype == AR_F64)
    e = launch_conv_t<double, double, double>(p, in, out, w, o1, o2, m1, m2, zero_ext, g_minus,
                                              partial, blocks, tiles_x, st);
  else if (p->dtype == AR_F32_ACC64 && out_compute)
    e = launch_conv_t<float, double, double>(p, in, out, w, o1, o2, m1, m2, zero_ext, g_minus,
                                             partial, blocks, tiles_x, st);
  else if (p->dtype == AR_F32_ACC64)
    e = launch_conv_t<float, double, float>(p, in, out, w, o1, o2, m1, m2, zero_ext, g_minus,
                                            partial, blocks, tiles_x, st);
  else
    e = launch_conv_t<float, float, float>(p, in, out, w, o1, o2, m1, m2, zero_ext, g_minus,
                                           partial, blocks, tiles_x, st);
  if (e != hipSuccess) return hip_fail(e, "conv_kernel launch");
  return AR_OK;
}

int fold_launch(const ar_plan_s *p, const void *ext, void *out, hipStream_t st) {
  if (p->q1 > 36 || p->q2 > 36) return fail(AR_EUNSUPPORTED, "adjoint fold supports q <= 36");
  dim3 grid((p->n2 + 63) / 64, (p->n1 + 3) / 4);
  if (p->dtype == AR_F64)
    hipLaunchKernelGGL((fold_kernel<double, double>), grid, dim3(256), 0, st,
                       static_cast<const double *>(ext), static_cast<double *>(out), p->n1,
                       p->n2, p->q1, p->q2);
  else if (p->dtype == AR_F32_ACC64)
    hipLaunchKernelGGL((fold_kernel<float, double>), grid, dim3(256), 0, st,
                       static_cast<const double *>(ext), static_cast<float *>(out), p->n1,
                       p->n2, p->q1, p->q2);
  else
    hipLaunchKernelGGL((fold_kernel<float, float>), grid, dim3(256), 0, st,
                       static_cast<const float *>(ext), static_cast<float *>(out), p->n1, p->n2,
                       p->q1, p->q2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fold_kernel launch");
  return AR_OK;
}

}  // namespace ar

using namespace ar;

extern "C" int ar_blur_apply(ar_plan_t p, const void *x, void *y, void *stream) {
  if (!p || !x || !y) return fail(AR_EINVAL, "ar_blur_apply: null argument");
  if (x == y) return fail(AR_EALIAS, "ar_blur_apply: x and y must not alias");
  AR_HIP(hipSetDevice(p->device));
  return conv_launch(p, x, y, p->w_fwd, 0, 0, p->n1, p->n2, false, nullptr, nullptr, nullptr,
                     static_cast<hipStream_t>(stream), false);
}

extern "C" int ar_blur_apply_T(ar_plan_t p, const void *r, void *y, int tmode, void *stream) {
  if (!p || !r || !y) return fail(AR_EINVAL, "ar_blur_apply_T: null argument");
  if (r == y) return fail(AR_EALIAS, "ar_blur_apply_T: r and y must not alias");
  AR_HIP(hipSetDevice(p->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (tmode == AR_REBLUR)
    return conv_launch(p, r, y, p->w_rev, 0, 0, p->n1, p->n2, false, nullptr, nullptr, nullptr,
                       st, false);
  if (tmode == AR_ADJOINT) {
    if (p->bc != AR_BC_ANTIREFLECTIVE)
      return fail(AR_EUNSUPPORTED, "ar_blur_apply_T: the exact transpose is Anti-Reflective only");
    int rc = conv_launch(p, r, p->ext, p->w_rev, -p->q1, -p->q2, p->n1 + 2 * p->q1,
                         p->n2 + 2 * p->q2, true, nullptr, nullptr, nullptr, st, true);
    if (rc != AR_OK) return rc;
    return fold_launch(p, p->ext, y, st);
  }
  return fail(AR_EINVAL, "ar_blur_apply_T: unknown tmode");
}
