// Wave-per-sequence AR transform engine (gfx950).
//
// Same mathematics as the block-wide engine (Theorem 1: endpoint scaling,
// ramp removal / restoration, DST-I of length m - 2 through one complex FFT
// of length M = m - 1 on the packed odd extension), organised so that every
// wavefront owns one row (or one column) from global load to global store:
//   * the packed sequence u_t = z_{2t} + i z_{2t+1} is written straight from
//     global memory into the wave's LDS buffer at digit-reversed positions;
//   * the FFT is an in-place mixed-radix decimation-in-time transform, one
//     butterfly per lane per step, largest radix first (its stage needs no
//     twiddles); twiddles of stage t are stored as [r - 1][k] so that lanes
//     with consecutive k read consecutive addresses;
//   * the DST values are formed from U_k and U_{M-k} and stored directly.
// A workgroup holds W waves (W sequences) and synchronises them between FFT
// stages.  The column pass of the preconditioner keeps the filtered
// coefficients in a per-wave LDS staging row and runs the inverse FFT in the
// same workgroup.  Every radix of M must have a codelet; other lengths use
// the block-wide engine.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ar_codelets.h"
#include "ar_internal.h"

namespace ar {
namespace {

using namespace cl;

// ------------------------------------------------------------ DIT stages

// Butterflies are processed NB at a time per lane: indices are clamped so
// that every load of a chunk is unconditional and issued together (one
// memory latency per chunk instead of one per butterfly); only the stores
// are guarded.  In-place is safe: butterflies of one stage touch disjoint
// positions.
template <int R> struct Chunk { static constexpr int value = R <= 4 ? 4 : (R <= 11 ? 2 : 1); };

template <typename T, int R>
__device__ __forceinline__ void dit_bfly(V2<T> *U, int M, int L, const V2<T> *__restrict__ tw,
                                         int lane) {
  constexpr int NB = Chunk<R>::value;
  const int nb = M / R;
  for (int j0 = lane; j0 < nb; j0 += 64 * NB) {
    V2<T> v[NB][R];
    int base[NB];
    bool ok[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int jr = j0 + 64 * c;
      ok[c] = jr < nb;
      const int j = ok[c] ? jr : j0;
      const int g = j / L, k = j - g * L;
      base[c] = g * L * R + k;
      static_for<R>([&](auto r) { v[c][r] = U[base[c] + r * L]; });
      if (L > 1)
        static_for<R - 1>([&](auto r) { v[c][r + 1] = cmul(v[c][r + 1], tw[r * L + k]); });
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (ok[c])
        dft_emit<R, T>(v[c], [&](auto K, V2<T> x) { U[base[c] + decltype(K)::value * L] = x; });
    }
  }
}

template <typename T>
__device__ __forceinline__ void dit_run(V2<T> *U, const WDesc &wd, const V2<T> *__restrict__ tw,
                                     int lane) {
  const int M = wd.M;
  for (int t = 0; t < wd.nst; ++t) {
    const V2<T> *tt = tw + wd.tw_off[t];
    const int L = wd.L[t];
    switch (wd.R[t]) {
      case 2: dit_bfly<T, 2>(U, M, L, tt, lane); break;
      case 3: dit_bfly<T, 3>(U, M, L, tt, lane); break;
      case 4: dit_bfly<T, 4>(U, M, L, tt, lane); break;
      case 5: dit_bfly<T, 5>(U, M, L, tt, lane); break;
      case 7: dit_bfly<T, 7>(U, M, L, tt, lane); break;
      case 11: dit_bfly<T, 11>(U, M, L, tt, lane); break;
      case 13: dit_bfly<T, 13>(U, M, L, tt, lane); break;
      case 17: dit_bfly<T, 17>(U, M, L, tt, lane); break;
      case 19: dit_bfly<T, 19>(U, M, L, tt, lane); break;
      case 23: dit_bfly<T, 23>(U, M, L, tt, lane); break;
      case 29: dit_bfly<T, 29>(U, M, L, tt, lane); break;
      default: dit_bfly<T, 31>(U, M, L, tt, lane); break;
    }
    __syncthreads();
  }
}

// ------------------------------------------------- packing and DST values

// sum_j x_j sin(pi j k / M) * scale from U_k and U_{M-k}, 1 <= k <= M-1
template <typename T>
__device__ __forceinline__ T wdst(const V2<T> *U, int k, int M, const V2<T> *__restrict__ post,
                                  T scale) {
  const V2<T> A = U[k], C = U[M - k];
  const V2<T> cs = post[k];
  return scale * ((C.y - A.y) + cs.x * (A.x - C.x) + cs.y * (A.y + C.y));
}

// Output k of a forward (INV = false) or inverse (INV = true) AR pass of
// length m = M + 1: endpoints from e0/e1, interior from the DST (plus the
// ramp for the inverse).  Loads use a clamped index (branch-free).
template <typename T, bool INV>
__device__ __forceinline__ T wcoef(const V2<T> *U, int k, int M, const V2<T> *__restrict__ post,
                                   T scale, T alpha, T e0, T e1, T invM) {
  const int kc = k < 1 ? 1 : (k > M - 1 ? M - 1 : k);
  const T d = wdst<T>(U, kc, M, post, scale);
  if (!INV) return k == 0 ? alpha * e0 : (k == M ? alpha * e1 : d);
  const T y0 = e0 / alpha, y1 = e1 / alpha;
  const T in = d + y0 * (T(M - k) * invM) + y1 * (T(k) * invM);
  return k == 0 ? y0 : (k == M ? y1 : in);
}

constexpr int kPostChunk = 8;

__device__ __forceinline__ double wg_sum(double v, double *red) {
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

// ------------------------------------------------------- LDS layout

// Workgroup LDS: [twiddles: twn][post: M+1][drev: M ints][U: W x M][aux: W x aux]
template <typename T>
struct WLayout {
  V2<T> *tw, *post, *U;
  int *drev;
  unsigned char *aux;
  __device__ WLayout(unsigned char *raw, int twn, int M, int W, int wave, size_t aux_bytes) {
    tw = reinterpret_cast<V2<T> *>(raw);
    post = tw + twn;
    drev = reinterpret_cast<int *>(post + M + 1);
    size_t off = (size_t)(twn + M + 1) * sizeof(V2<T>) + (size_t)M * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    U = reinterpret_cast<V2<T> *>(raw + off) + (size_t)wave * M;
    off += (size_t)W * M * sizeof(V2<T>);
    aux = raw + off + (size_t)wave * aux_bytes;
  }
};

size_t wlds_bytes(int twn, int M, int W, size_t csize, size_t aux_bytes) {
  size_t off = (size_t)(twn + M + 1) * 2 * csize + (size_t)M * sizeof(int);
  off = (off + 15) & ~(size_t)15;
  return off + (size_t)W * M * 2 * csize + (size_t)W * aux_bytes;
}

constexpr int kTabChunk = 4;   // table elements per thread per batch
constexpr int kRowChunk = 16;  // row elements per lane per batch (covers m <= 1024 at once)

// Twiddle, post and digit-reversal tables into LDS; indices are clamped so
// that all loads of a batch are issued before any store.
template <typename T>
__device__ __forceinline__ void load_tables(const WLayout<T> &Ly, const V2<T> *__restrict__ tw,
                                            int twn, const V2<T> *__restrict__ post, int M,
                                            const int *__restrict__ drev) {
  const int nth = blockDim.x, tid = threadIdx.x;
  const int tot = (twn > M + 1 ? twn : M + 1);
  const int twmax = twn > 0 ? twn - 1 : 0;
  for (int e0 = tid; e0 < tot; e0 += nth * kTabChunk) {
    V2<T> a[kTabChunk], p[kTabChunk];
    int d[kTabChunk];
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c) {
      const int e = e0 + nth * c;
      a[c] = tw[e < twn ? e : twmax];
      p[c] = post[e <= M ? e : M];
      d[c] = drev[e < M ? e : M - 1];
    }
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c) {
      const int e = e0 + nth * c;
      if (e < twn) Ly.tw[e] = a[c];
      if (e <= M) Ly.post[e] = p[c];
      if (e < M) Ly.drev[e] = d[c];
    }
  }
}

// Raw interior values x_j, j = 2t and 2t+1 (mirrored for t beyond M/2),
// of one chunk of the packed sequence, read with clamped indices.
template <typename TSRC, typename T>
__device__ __forceinline__ void pack_load(T (&xr)[kRowChunk], T (&xi)[kRowChunk],
                                          const TSRC *src, long stride, int t0, int M) {
#pragma unroll
  for (int c = 0; c < kRowChunk; ++c) {
    const int t = t0 + 64 * c;
    int j0 = 2 * t, j1 = 2 * t + 1;
    j0 = j0 < M ? j0 : 2 * M - j0;
    j1 = j1 < M ? j1 : 2 * M - j1;
    j0 = (j0 < 1 || j0 > M - 1) ? 1 : j0;  // tau = 0, M (value unused) or t past the end
    j1 = (j1 < 1 || j1 > M - 1) ? 1 : j1;
    xr[c] = T(src[(long)j0 * stride]);
    xi[c] = T(src[(long)j1 * stride]);
  }
}

// z_tau of the odd extension from a loaded raw value (ramp removed if asked)
template <typename T>
__device__ __forceinline__ T zfrom(T x, int tau, int M, bool ramp, T e0, T e1, T invM) {
  const bool zero = (tau == 0) | (tau == M);
  const int j = tau < M ? tau : 2 * M - tau;
  if (ramp) x -= e0 * (T(M - j) * invM) + e1 * (T(j) * invM);
  x = tau < M ? x : -x;
  return zero ? T(0) : x;
}

template <typename T>
__device__ __forceinline__ void pack_store(V2<T> *U, const int *s_drev, const T (&xr)[kRowChunk],
                                           const T (&xi)[kRowChunk], int t0, int M, bool active,
                                           bool ramp, T e0, T e1) {
  const T invM = T(1) / T(M);
#pragma unroll
  for (int c = 0; c < kRowChunk; ++c) {
    const int t = t0 + 64 * c;
    if (t >= M) continue;
    V2<T> u{T(0), T(0)};
    if (active) {
      u.x = zfrom<T>(xr[c], 2 * t, M, ramp, e0, e1, invM);
      u.y = zfrom<T>(xi[c], 2 * t + 1, M, ramp, e0, e1, invM);
    }
    U[s_drev[t]] = u;
  }
}

// Pack the whole sequence (chunk 0 already loaded into xr/xi).
template <typename TSRC, typename T>
__device__ __forceinline__ void pack_rest(V2<T> *U, const int *s_drev, T (&xr)[kRowChunk],
                                          T (&xi)[kRowChunk], const TSRC *src, long stride,
                                          int lane, int M, bool active, bool ramp, T e0, T e1) {
  pack_store<T>(U, s_drev, xr, xi, lane, M, active, ramp, e0, e1);
  for (int t0 = lane + 64 * kRowChunk; t0 < M; t0 += 64 * kRowChunk) {
    pack_load<TSRC, T>(xr, xi, src, stride, t0, M);
    pack_store<T>(U, s_drev, xr, xi, t0, M, active, ramp, e0, e1);
  }
}

// ---------------------------------------------------------------- rows

template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void rows_w_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, int m, WDesc wd,
    const V2<T> *__restrict__ tw, const int *__restrict__ drev, const V2<T> *__restrict__ post,
    T alpha, T scale, T tau, const TS *__restrict__ f_true, double *__restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = wd.M;
  const int W = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = xcd_remap(blockIdx.x, gridDim.x) * W + wave;
  const bool active = row < n1;
  const size_t auxb = MODE == ROW_INV_UPDATE ? 2 * (size_t)m * sizeof(TS) : 0;
  const WLayout<T> Ly(smem_raw, wd.twn, M, W, wave, auxb);
  const TS *src = in + (size_t)(active ? row : 0) * m;
  TS *dst = out + (size_t)(active ? row : 0) * m;
  const TS *fr = f_true ? f_true + (size_t)(active ? row : 0) * m : nullptr;
  TS *sx = reinterpret_cast<TS *>(Ly.aux);
  TS *sf = sx + m;
  // one batch of global loads: this wave's row, x and f (update), tables
  T xr[kRowChunk], xi[kRowChunk];
  pack_load<TS, T>(xr, xi, src, 1, lane, M);
  const T e0 = T(src[0]), e1 = T(src[m - 1]);
  if (MODE == ROW_INV_UPDATE) {
    for (int k0 = lane; k0 < m; k0 += 64 * kRowChunk) {
      TS a[kRowChunk], b[kRowChunk];
#pragma unroll
      for (int c = 0; c < kRowChunk; ++c) {
        const int kr = k0 + 64 * c;
        const int k = kr < m ? kr : m - 1;
        a[c] = dst[k];
        b[c] = fr ? fr[k] : TS(0);
      }
#pragma unroll
      for (int c = 0; c < kRowChunk; ++c) {
        const int k = k0 + 64 * c;
        if (k < m) {
          sx[k] = a[c];
          sf[k] = b[c];
        }
      }
    }
  }
  load_tables<T>(Ly, tw, wd.twn, post, M, drev);
  __syncthreads();
  pack_rest<TS, T>(Ly.U, Ly.drev, xr, xi, src, 1, lane, M, active, MODE == ROW_FWD, e0, e1);
  __syncthreads();
  dit_run<T>(Ly.U, wd, Ly.tw, lane);
  double ss = 0.0;
  if (active) {
    const T invM = T(1) / T(M);
    for (int k0 = lane; k0 < m; k0 += 64 * kPostChunk) {
      T val[kPostChunk];
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int kr = k0 + 64 * c;
        const int k = kr < m ? kr : k0;
        val[c] = wcoef<T, MODE != ROW_FWD>(Ly.U, k, M, Ly.post, scale, alpha, e0, e1, invM);
      }
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int k = k0 + 64 * c;
        if (k >= m) continue;
        if (MODE == ROW_INV_UPDATE) {
          const TS xn = TS(T(sx[k]) + tau * val[c]);
          dst[k] = xn;
          if (fr) {
            const double df = (double)xn - (double)sf[k];
            ss += df * df;
          }
        } else {
          dst[k] = TS(val[c]);
        }
      }
    }
  }
  if (MODE == ROW_INV_UPDATE && partial) {
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem_raw);
    const double s = wg_sum(ss, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------- columns

template <typename TS, typename T, int MODE>
__global__ __launch_bounds__(256) void cols_w_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int m, int n2, WDesc wd,
    const V2<T> *__restrict__ tw, const int *__restrict__ drev, const V2<T> *__restrict__ post,
    T alpha, T scale, const T *__restrict__ dflt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int M = wd.M;
  const int W = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = xcd_remap(blockIdx.x, gridDim.x) * W + wave;
  const bool active = col < n2;
  const size_t auxb = MODE == COL_FWD_D_INV ? (size_t)m * sizeof(T) : 0;
  const WLayout<T> Ly(smem_raw, wd.twn, M, W, wave, auxb);
  T *S = reinterpret_cast<T *>(Ly.aux);
  const long ld = n2;
  const TS *src = in + (active ? col : 0);
  T xr[kRowChunk], xi[kRowChunk];
  pack_load<TS, T>(xr, xi, src, ld, lane, M);
  T e0 = T(src[0]);
  T e1 = T(src[(long)(m - 1) * ld]);
  if (MODE == COL_FWD_D_INV) {
    // filter column into the staging row (overwritten in place below)
    const T *dcol = dflt + (active ? col : 0);
    for (int k0 = lane; k0 < m; k0 += 64 * kRowChunk) {
      T a[kRowChunk];
#pragma unroll
      for (int c = 0; c < kRowChunk; ++c) {
        const int kr = k0 + 64 * c;
        a[c] = dcol[(long)(kr < m ? kr : m - 1) * ld];
      }
#pragma unroll
      for (int c = 0; c < kRowChunk; ++c) {
        const int k = k0 + 64 * c;
        if (k < m) S[k] = a[c];
      }
    }
  }
  load_tables<T>(Ly, tw, wd.twn, post, M, drev);
  __syncthreads();
  pack_rest<TS, T>(Ly.U, Ly.drev, xr, xi, src, ld, lane, M, active, MODE != COL_INV, e0, e1);
  __syncthreads();
  dit_run<T>(Ly.U, wd, Ly.tw, lane);
  const T invM = T(1) / T(M);
  if (MODE == COL_FWD_D_INV) {
    // S[k] <- d_k * (T~ y)_k (same lane reads and writes S[k])
    for (int k0 = lane; k0 < m; k0 += 64 * kPostChunk) {
      T val[kPostChunk];
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int kr = k0 + 64 * c;
        const int k = kr < m ? kr : k0;
        val[c] = wcoef<T, false>(Ly.U, k, M, Ly.post, scale, alpha, e0, e1, invM);
      }
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int k = k0 + 64 * c;
        if (k < m) S[k] = val[c] * S[k];
      }
    }
    __syncthreads();
    e0 = S[0];
    e1 = S[m - 1];
    for (int t0 = lane; t0 < M; t0 += 64 * kRowChunk) {
      pack_load<T, T>(xr, xi, S, 1, t0, M);
      pack_store<T>(Ly.U, Ly.drev, xr, xi, t0, M, active, false, e0, e1);
    }
    __syncthreads();
    dit_run<T>(Ly.U, wd, Ly.tw, lane);
  }
  if (active) {
    for (int k0 = lane; k0 < m; k0 += 64 * kPostChunk) {
      T val[kPostChunk];
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int kr = k0 + 64 * c;
        const int k = kr < m ? kr : k0;
        val[c] = wcoef<T, MODE != COL_FWD>(Ly.U, k, M, Ly.post, scale, alpha, e0, e1, invM);
      }
#pragma unroll
      for (int c = 0; c < kPostChunk; ++c) {
        const int k = k0 + 64 * c;
        if (k < m) out[(long)k * ld + col] = TS(val[c]);
      }
    }
  }
}

// ------------------------------------------------------------- tables

template <typename T>
__global__ void wtables_kernel(V2<T> *tw, const int *R, const int *L, const int *off, int nst) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  for (int s = 0; s < nst; ++s) {
    const int Rs = R[s], Ls = L[s], LR = Rs * Ls;
    const int cnt = (Rs - 1) * Ls;
    for (int e = tid; e < cnt; e += nth) {
      const int r = e / Ls + 1, k = e - (r - 1) * Ls;
      const long kr = ((long)k * r) % LR;
      double sv, cv;
      sincospi(-2.0 * (double)kr / (double)LR, &sv, &cv);
      tw[off[s] + e] = {T(cv), T(sv)};
    }
  }
}

// Waves (sequences) per workgroup: `forced` if it fits, else the largest
// power of two <= 4 whose LDS fits.
int wave_count(size_t fixed, size_t per_wave, int nseq, int forced) {
  if (forced == 1 || forced == 2 || forced == 4) {
    int W = forced;
    while (W > 1 && fixed + (size_t)W * per_wave > 150 * 1024) W >>= 1;
    return W;
  }
  int W = 4;
  while (W > 1 && fixed + (size_t)W * per_wave > 150 * 1024) W >>= 1;
  while (W > 1 && W / 2 >= nseq) W >>= 1;
  return W;
}

// With the exclusive flag the dynamic LDS is padded so that one workgroup
// occupies a CU (the dispatcher then spreads workgroups over all CUs).
size_t excl_pad(size_t smem, int excl) {
  return excl && smem < 81 * 1024 ? 81 * 1024 : smem;
}

constexpr size_t kMaxLdsW = 150 * 1024;

template <typename K>
hipError_t allow_lds_w(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

WDesc make_wdesc(const WavePlan &w) {
  WDesc d{};
  d.M = w.M;
  d.nst = w.nst;
  d.twn = w.twn;
  for (int s = 0; s < kMaxStages; ++s) {
    d.R[s] = w.R[s];
    d.L[s] = w.L[s];
    d.tw_off[s] = w.tw_off[s];
  }
  return d;
}

}  // namespace

// Factor M into codelet radices (4s first, then odd primes), largest radix
// first; build the digit-reversal table and the twiddle tables.
int wave_plan_build(WavePlan &w, int M, bool cdouble, hipStream_t st) {
  w = WavePlan{};
  w.M = M;
  std::vector<int> rad;
  int r = M;
  while (r % 4 == 0) { rad.push_back(4); r /= 4; }
  while (r % 2 == 0) { rad.push_back(2); r /= 2; }
  for (int p = 3; p <= 31 && r > 1; p += 2)
    while (r % p == 0 && cl::has_codelet(p)) { rad.push_back(p); r /= p; }
  if (r != 1 || rad.empty() || (int)rad.size() > kMaxStages) return AR_OK;  // not applicable
  std::sort(rad.begin(), rad.end(), [](int a, int b) { return a > b; });
  w.nst = (int)rad.size();
  int L = 1;
  size_t off = 0;
  std::vector<int> hR, hL, hoff;
  for (int s = 0; s < w.nst; ++s) {
    w.R[s] = rad[s];
    w.L[s] = L;
    w.tw_off[s] = (int)off;
    hR.push_back(rad[s]);
    hL.push_back(L);
    hoff.push_back((int)off);
    off += (size_t)(rad[s] - 1) * L;
    L *= rad[s];
  }
  // digit reversal: natural index n has digits (most significant first)
  // p_0..p_{s-1} in radices R_0..R_{s-1}; its position is sum_t p_t prod_{u<t} R_u
  std::vector<int> drev(M);
  for (int n = 0; n < M; ++n) {
    int rem = n, pos = 0, wpos = 1, wnat = M;
    for (int t = 0; t < w.nst; ++t) {
      wnat /= w.R[t];
      const int d = rem / wnat;
      rem -= d * wnat;
      pos += d * wpos;
      wpos *= w.R[t];
    }
    drev[n] = pos;
  }
  w.twn = (int)off;
  const size_t cb = cdouble ? sizeof(double2) : sizeof(float2);
  AR_HIP(hipMalloc(&w.tw, (off > 0 ? off : 1) * cb));
  AR_HIP(hipMalloc((void **)&w.drev, (size_t)M * sizeof(int)));
  AR_HIP(hipMemcpy(w.drev, drev.data(), (size_t)M * sizeof(int), hipMemcpyHostToDevice));
  std::vector<int> ints;
  ints.insert(ints.end(), hR.begin(), hR.end());
  ints.insert(ints.end(), hL.begin(), hL.end());
  ints.insert(ints.end(), hoff.begin(), hoff.end());
  int *dints = nullptr;
  AR_HIP(hipMalloc(&dints, ints.size() * sizeof(int)));
  AR_HIP(hipMemcpy(dints, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice));
  const int nst = w.nst;
  if (cdouble)
    hipLaunchKernelGGL(wtables_kernel<double>, dim3(32), dim3(256), 0, st,
                       static_cast<V2<double> *>(w.tw), dints, dints + nst, dints + 2 * nst, nst);
  else
    hipLaunchKernelGGL(wtables_kernel<float>, dim3(32), dim3(256), 0, st,
                       static_cast<V2<float> *>(w.tw), dints, dints + nst, dints + 2 * nst, nst);
  AR_HIP(hipGetLastError());
  AR_HIP(hipStreamSynchronize(st));
  AR_HIP(hipFree(dints));
  w.ok = true;
  return AR_OK;
}

void wave_plan_free(WavePlan &w) {
  if (w.tw) (void)hipFree(w.tw);
  if (w.drev) (void)hipFree(w.drev);
  w.tw = nullptr;
  w.drev = nullptr;
  w.ok = false;
}

static size_t rows_aux(const ar_plan_s *p) { return 2 * (size_t)p->n2 * p->esize; }
static size_t cols_aux(const ar_plan_s *p) { return (size_t)p->n1 * p->csize; }

static int rows_waves(const ar_plan_s *p) {
  const int M = p->fft_row.M;
  const size_t fixed = wlds_bytes(p->fft_row.w.twn, M, 0, p->csize, 0);
  return wave_count(fixed, (size_t)M * 2 * p->csize + rows_aux(p), p->n1, p->tune[AR_TUNE_ROW_WAVES]);
}
static int cols_waves(const ar_plan_s *p) {
  const int M = p->fft_col.M;
  const size_t fixed = wlds_bytes(p->fft_col.w.twn, M, 0, p->csize, 0);
  return wave_count(fixed, (size_t)M * 2 * p->csize + cols_aux(p), p->n2, p->tune[AR_TUNE_COL_WAVES]);
}

bool wave_rows_ok(const ar_plan_s *p) {
  return p->fft_row.w.ok &&
         wlds_bytes(p->fft_row.w.twn, p->fft_row.M, 1, p->csize, rows_aux(p)) <= kMaxLdsW;
}
bool wave_cols_ok(const ar_plan_s *p) {
  return p->fft_col.w.ok &&
         wlds_bytes(p->fft_col.w.twn, p->fft_col.M, 1, p->csize, cols_aux(p)) <= kMaxLdsW;
}

int wave_rows_blocks(const ar_plan_s *p) {
  const int W = rows_waves(p);
  return (p->n1 + W - 1) / W;
}

template <typename TS, typename T>
static int wave_rows_t(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                       const void *f_true, double *partial, hipStream_t st) {
  const FftPlan &fp = p->fft_row;
  const int m = p->n2, M = fp.M;
  const int W = rows_waves(p);
  const int blocks = (p->n1 + W - 1) / W;
  const size_t smem = excl_pad(wlds_bytes(fp.w.twn, M, W, sizeof(T), rows_aux(p)),
                               p->tune[AR_TUNE_ROW_EXCL]);
  const WDesc wd = make_wdesc(fp.w);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(fp.w.tw);
  auto post = static_cast<const V2<T> *>(fp.post);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  hipError_t e = hipSuccess;
#define AR_WROWS(MODE)                                                                          \
  e = allow_lds_w(rows_w_kernel<TS, T, MODE>, smem);                                            \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((rows_w_kernel<TS, T, MODE>), dim3(blocks), dim3(64 * W), smem, st, ti,  \
                       to, p->n1, m, wd, tw, fp.w.drev, post, alpha, scale, T(tau), tf, partial); \
    e = hipGetLastError();                                                                      \
  }
  switch (mode) {
    case ROW_FWD: AR_WROWS(ROW_FWD) break;
    case ROW_INV: AR_WROWS(ROW_INV) break;
    default: AR_WROWS(ROW_INV_UPDATE) break;
  }
#undef AR_WROWS
  if (e != hipSuccess) return hip_fail(e, "rows_w_kernel launch");
  return AR_OK;
}

int wave_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                     const void *f_true, double *partial, hipStream_t st) {
  if (p->dtype == AR_F64)
    return wave_rows_t<double, double>(p, in, out, mode, tau, f_true, partial, st);
  if (p->dtype == AR_F32_ACC64)
    return wave_rows_t<float, double>(p, in, out, mode, tau, f_true, partial, st);
  return wave_rows_t<float, float>(p, in, out, mode, tau, f_true, partial, st);
}

template <typename TS, typename T>
static int wave_cols_t(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  const FftPlan &fp = p->fft_col;
  const int m = p->n1, M = fp.M;
  const int W = cols_waves(p);
  const int blocks = (p->n2 + W - 1) / W;
  const size_t smem = excl_pad(wlds_bytes(fp.w.twn, M, W, sizeof(T), cols_aux(p)),
                               p->tune[AR_TUNE_COL_EXCL]);
  const WDesc wd = make_wdesc(fp.w);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(fp.w.tw);
  auto post = static_cast<const V2<T> *>(fp.post);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const T *>(p->d);
  hipError_t e = hipSuccess;
#define AR_WCOLS(MODE)                                                                          \
  e = allow_lds_w(cols_w_kernel<TS, T, MODE>, smem);                                            \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((cols_w_kernel<TS, T, MODE>), dim3(blocks), dim3(64 * W), smem, st, ti,  \
                       to, m, p->n2, wd, tw, fp.w.drev, post, alpha, scale, td);                \
    e = hipGetLastError();                                                                      \
  }
  switch (mode) {
    case COL_FWD: AR_WCOLS(COL_FWD) break;
    case COL_INV: AR_WCOLS(COL_INV) break;
    default: AR_WCOLS(COL_FWD_D_INV) break;
  }
#undef AR_WCOLS
  if (e != hipSuccess) return hip_fail(e, "cols_w_kernel launch");
  return AR_OK;
}

int wave_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  if (p->dtype == AR_F64) return wave_cols_t<double, double>(p, in, out, mode, st);
  if (p->dtype == AR_F32_ACC64) return wave_cols_t<float, double>(p, in, out, mode, st);
  return wave_cols_t<float, float>(p, in, out, mode, st);
}

}  // namespace ar
