// Wave-per-sequence AR transform engine (gfx950).
//
// Same mathematics as the block-wide engine (Theorem 1: endpoint scaling,
// ramp removal / restoration, DST-I of length m - 2 through one complex FFT
// of length M = m - 1 on the packed odd extension u_t = z_{2t} + i z_{2t+1}),
// organised so that every wavefront owns one row (or one column) from global
// load to global store:
//   * the packed sequence is written from registers into the wave's LDS
//     buffer at digit-reversed positions;
//   * the FFT is an in-place decimation-in-time (DIT) transform, one
//     butterfly per lane per step; twiddles of stage t are stored [r - 1][k]
//     so that lanes with consecutive k read consecutive words;
//   * the FFT is either the mixed-radix FFT of length M (every prime factor
//     has a codelet, largest radix first) or Bluestein's chirp-z form:
//     a_j = u_j w_j with w_j = e^{-i pi j^2 / M}, a DIT FFT of power-of-two
//     length N >= 2M - 1, the product with the chirp spectrum, and the
//     inverse FFT as a decimation-in-frequency (DIF) FFT of the conjugate,
//     which leaves its result at digit-reversed positions, so that
//     U_k = w_k conj(D[drev(k)]) needs no extra permutation pass;
//   * the DST values come from U_k and U_{M-k} and are stored directly.
// Twiddle, post-processing and digit-reversal tables are staged in LDS once
// per workgroup; the global loads of a kernel are issued before its first
// barrier.  Two plans are compiled with their stages fixed (every stride,
// bound and table offset a constant): the mixed-radix plan of length 1023
// and the Bluestein plans of power-of-two length 256, 512 and 1024 (FP32
// tables); other lengths run the stage loop of the plan's descriptor.  The column pass of the preconditioner keeps the filtered
// coefficients in a per-wave LDS row and runs the inverse transform in the
// same workgroup.
#include <algorithm>
#include <cmath>
#include <complex>
#include <type_traits>
#include <vector>

#include "ar_codelets.h"
#include "ar_internal.h"

namespace ar {
namespace {

using namespace cl;

// ------------------------------------------------------------ FFT stages

// Butterflies are processed NB at a time per lane: indices are clamped so
// that every load of a chunk is issued together; only the stores are
// guarded.  In place is safe: butterflies of one stage touch disjoint
// positions.
template <int R> struct Chunk { static constexpr int value = R <= 4 ? 4 : (R <= 11 ? 2 : 1); };

// One stage.  DIT: twiddle the inputs, then the DFT.  DIF (the transpose
// of the DIT stage): the DFT, then twiddle the outputs.
template <typename T, int R, bool DIF, int G>
__device__ __forceinline__ void bfly(V2<T> *U, int N, int L, const V2<T> *__restrict__ tw,
                                     int lane) {
  constexpr int NB = Chunk<R>::value;
  constexpr int SL = 64 * G;  // lanes working on one sequence
  // small radices keep their twiddles in registers across the DFT; large
  // ones read them where they are used (register pressure)
  constexpr bool PRE = R <= 11;
  const int nb = N / R;
  // a stage with at most 64 butterflies runs on one wave of the sequence
  // (its other waves wait at the barrier instead of issuing the same
  // instructions for a few lanes each); the working wave alternates between
  // pairs of sequences so that, with waves dealt round-robin to the four
  // SIMDs, every SIMD gets the same share of the stage
  if (G > 1 && nb <= 64) {
    const int wv = threadIdx.x >> 6;
    const int worker = ((wv / G) >> 1) % G;
    lane = wv % G == worker ? (int)(threadIdx.x & 63) : 64 + (int)(threadIdx.x & 63);
  }
  for (int j0 = lane; j0 < nb; j0 += SL * NB) {
    V2<T> v[NB][R];
    V2<T> t[NB][PRE ? R - 1 : 1];
    int base[NB], kk[NB];
    bool ok[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int jr = j0 + SL * c;
      ok[c] = jr < nb;
      const int j = ok[c] ? jr : j0;
      const int g = j / L, k = j - g * L;
      base[c] = g * L * R + k;
      kk[c] = k;
      static_for<R>([&](auto r) { v[c][r] = U[base[c] + r * L]; });
      if (L > 1) {
        if constexpr (PRE) {
          static_for<R - 1>([&](auto r) { t[c][r] = tw[r * L + k]; });
          if constexpr (!DIF)
            static_for<R - 1>([&](auto r) { v[c][r + 1] = cmul(v[c][r + 1], t[c][r]); });
        } else if constexpr (!DIF) {
          static_for<R - 1>([&](auto r) { v[c][r + 1] = cmul(v[c][r + 1], tw[r * L + k]); });
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (!ok[c]) continue;
      if constexpr (!DIF) {
        dft_emit<R, T>(v[c], [&](auto K, V2<T> x) { U[base[c] + decltype(K)::value * L] = x; });
      } else {
        dft_emit<R, T>(v[c], [&](auto K, V2<T> x) {
          constexpr int r = decltype(K)::value;
          if constexpr (r > 0) {
            if (L > 1) {
              if constexpr (PRE) x = cmul(x, t[c][r - 1]);
              else x = cmul(x, tw[(r - 1) * L + kk[c]]);
            }
          }
          U[base[c] + r * L] = x;
        });
      }
    }
  }
}

// Radix sets: a kernel compiled for a set contains only those codelets.
constexpr int rbit(int r) {
  return r == 2 ? 0 : r == 3 ? 1 : r == 4 ? 2 : r == 5 ? 3 : r == 7 ? 4 : r == 11 ? 5 : r == 13 ? 6
       : r == 17 ? 7 : r == 19 ? 8 : r == 23 ? 9 : r == 29 ? 10 : 11;
}
constexpr int kMaskAll = 0xfff;
// M = 1023 = 31 * 11 * 3 (rows or columns of 1024): the three stages are
// fixed at compile time, so every stride, bound and table offset is a
// constant.
constexpr int kPlan1023 = -1;
// Bluestein plans of length N = 2^k (256, 512, 1024 for k = 8, 9, 10): the
// radix-4 stages (and a final radix 2) fixed at compile time, MASK = -k.
constexpr int kPlanBSMin = -10, kPlanBSMax = -8;
constexpr bool is_bs_static(int mask) { return mask >= kPlanBSMin && mask <= kPlanBSMax; }
constexpr bool in_mask(int mask, int r) { return mask >= 0 && ((mask >> rbit(r)) & 1); }
constexpr int plan_n(int mask) { return mask == kPlan1023 ? 1023 : (1 << -mask); }

// The compile-time Bluestein stages from stride L on: radix 4 while N / L
// is a multiple of 4, then radix 2; twiddles of the stage at stride L start
// at L - 1 (the preceding radix-4 stages hold 3 (1 + 4 + ... + L / 4)).
// DIT runs them by increasing L, DIF by decreasing L.
template <typename T, bool DIF, int G, int N, int L>
__device__ __forceinline__ void bs_stages(V2<T> *U, const V2<T> *__restrict__ tw, int lane) {
  constexpr int R = (N / L) % 4 == 0 ? 4 : 2;
  if constexpr (DIF && L * R < N) bs_stages<T, DIF, G, N, L * R>(U, tw, lane);
  bfly<T, R, DIF, G>(U, N, L, tw + (L - 1), lane);
  __syncthreads();
  if constexpr (!DIF && L * R < N) bs_stages<T, DIF, G, N, L * R>(U, tw, lane);
}

// DIT runs stages 0..nst-1 (digit-reversed in, natural out); DIF runs them
// backwards (natural in, digit-reversed out).  Bluestein plans use radices
// 4 and 2 only.
template <typename T, bool DIF, bool BS, int G, int MASK>
__device__ __forceinline__ void fft_run(V2<T> *U, const WDesc &wd, const V2<T> *__restrict__ tw,
                                        int lane) {
  if constexpr (MASK == kPlan1023) {
    // stages (R, L, twiddle offset): (31, 1, 0), (11, 31, 30), (3, 341, 340)
    bfly<T, 31, DIF, G>(U, 1023, 1, tw, lane);
    __syncthreads();
    bfly<T, 11, DIF, G>(U, 1023, 31, tw + 30, lane);
    __syncthreads();
    bfly<T, 3, DIF, G>(U, 1023, 341, tw + 340, lane);
    __syncthreads();
    return;
  }
  if constexpr (is_bs_static(MASK)) {
    bs_stages<T, DIF, G, plan_n(MASK), 1>(U, tw, lane);
    return;
  }
  const int N = wd.N;
  for (int s = 0; s < wd.nst; ++s) {
    const int st = DIF ? wd.nst - 1 - s : s;
    const V2<T> *tt = tw + wd.tw_off[st];
    const int L = wd.L[st];
    if constexpr (BS) {
      if (wd.R[st] == 4)
        bfly<T, 4, DIF, G>(U, N, L, tt, lane);
      else
        bfly<T, 2, DIF, G>(U, N, L, tt, lane);
    } else {
      switch (wd.R[st]) {
        case 2: if constexpr (in_mask(MASK, 2)) bfly<T, 2, DIF, G>(U, N, L, tt, lane); break;
        case 3: if constexpr (in_mask(MASK, 3)) bfly<T, 3, DIF, G>(U, N, L, tt, lane); break;
        case 4: if constexpr (in_mask(MASK, 4)) bfly<T, 4, DIF, G>(U, N, L, tt, lane); break;
        case 5: if constexpr (in_mask(MASK, 5)) bfly<T, 5, DIF, G>(U, N, L, tt, lane); break;
        case 7: if constexpr (in_mask(MASK, 7)) bfly<T, 7, DIF, G>(U, N, L, tt, lane); break;
        case 11: if constexpr (in_mask(MASK, 11)) bfly<T, 11, DIF, G>(U, N, L, tt, lane); break;
        case 13: if constexpr (in_mask(MASK, 13)) bfly<T, 13, DIF, G>(U, N, L, tt, lane); break;
        case 17: if constexpr (in_mask(MASK, 17)) bfly<T, 17, DIF, G>(U, N, L, tt, lane); break;
        case 19: if constexpr (in_mask(MASK, 19)) bfly<T, 19, DIF, G>(U, N, L, tt, lane); break;
        case 23: if constexpr (in_mask(MASK, 23)) bfly<T, 23, DIF, G>(U, N, L, tt, lane); break;
        case 29: if constexpr (in_mask(MASK, 29)) bfly<T, 29, DIF, G>(U, N, L, tt, lane); break;
        default: if constexpr (in_mask(MASK, 31)) bfly<T, 31, DIF, G>(U, N, L, tt, lane); break;
      }
    }
    __syncthreads();
  }
}

// Elements per lane per batch of the sequence-wide loops (1024 per sequence
// at once): G lanes-per-sequence groups of 64 share them.
template <int G> struct RC { static constexpr int value = 16 / G; };
template <int G> struct PC { static constexpr int value = 8 / G; };

// Bluestein middle step, natural order, in place: U_k <- conj(U_k bhat_k)
template <typename T, int G>
__device__ __forceinline__ void bs_mid(V2<T> *U, int N, const V2<T> *__restrict__ bhat, int lane) {
  constexpr int C = RC<G>::value, SL = 64 * G;
  for (int k0 = lane; k0 < N; k0 += SL * C) {
    V2<T> b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int k = k0 + SL * c;
      b[c] = bhat[k < N ? k : k0];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int k = k0 + SL * c;
      if (k < N) {
        const V2<T> z = cmul(U[k], b[c]);
        U[k] = {z.x, -z.y};
      }
    }
  }
}

// The DFT of the packed sequence held in U.
template <typename T, bool BS, int G, int MASK>
__device__ __forceinline__ void fft_full(V2<T> *U, const WDesc &wd, const V2<T> *tw,
                                         const V2<T> *__restrict__ bhat, int lane) {
  fft_run<T, false, BS, G, MASK>(U, wd, tw, lane);
  if constexpr (BS) {
    bs_mid<T, G>(U, wd.N, bhat, lane);
    __syncthreads();
    fft_run<T, true, BS, G, MASK>(U, wd, tw, lane);
  }
}

// ------------------------------------------------- packing and DST values

// U_k of the length-M DFT (1 <= k <= M - 1) from the buffer
template <typename T, bool BS>
__device__ __forceinline__ V2<T> getU(const V2<T> *U, const int *s_drev,
                                      const V2<T> *__restrict__ chirp, int k) {
  if constexpr (!BS) {
    return U[k];
  } else {
    const V2<T> d = U[s_drev[k]];
    return cmul(chirp[k], V2<T>{d.x, -d.y});
  }
}

// sum_j x_j sin(pi j k / M) * scale from U_k and U_{M-k}, 1 <= k <= M-1
template <typename T, bool BS>
__device__ __forceinline__ T wdst(const V2<T> *U, const int *s_drev, const V2<T> *chirp, int k,
                                  int M, const V2<T> *__restrict__ post, T scale) {
  const V2<T> A = getU<T, BS>(U, s_drev, chirp, k);
  const V2<T> C = getU<T, BS>(U, s_drev, chirp, M - k);
  const V2<T> cs = post[k];
  return scale * ((C.y - A.y) + cs.x * (A.x - C.x) + cs.y * (A.y + C.y));
}

// Output k of a forward (INV = false) or inverse (INV = true) AR pass of
// length m = M + 1: endpoints from e0/e1, interior from the DST (plus the
// ramp for the inverse).  Loads use a clamped index (branch-free).
template <typename T, bool INV, bool BS>
__device__ __forceinline__ T wcoef(const V2<T> *U, const int *s_drev, const V2<T> *chirp, int k,
                                   int M, const V2<T> *__restrict__ post, T scale, T alpha, T e0,
                                   T e1, T invM) {
  const int kc = k < 1 ? 1 : (k > M - 1 ? M - 1 : k);
  const T d = wdst<T, BS>(U, s_drev, chirp, kc, M, post, scale);
  if (!INV) return k == 0 ? alpha * e0 : (k == M ? alpha * e1 : d);
  const T y0 = e0 / alpha, y1 = e1 / alpha;
  const T in = d + y0 * (T(M - k) * invM) + y1 * (T(k) * invM);
  return k == 0 ? y0 : (k == M ? y1 : in);
}

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

// Workgroup LDS: [twiddles: twn][post: M+1][drev: N ints][U: W x N][aux: W x aux]
template <typename T>
struct WLayout {
  V2<T> *tw, *post, *U;
  int *drev;
  unsigned char *aux;
  __device__ WLayout(unsigned char *raw, int twn, int M, int N, int W, int wave,
                     size_t aux_bytes) {
    tw = reinterpret_cast<V2<T> *>(raw);
    post = tw + twn;
    drev = reinterpret_cast<int *>(post + M + 1);
    size_t off = (size_t)(twn + M + 1) * sizeof(V2<T>) + (size_t)N * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    U = reinterpret_cast<V2<T> *>(raw + off) + (size_t)wave * N;
    off += (size_t)W * N * sizeof(V2<T>);
    aux = raw + off + (size_t)wave * aux_bytes;
  }
};

size_t wlds_bytes(int twn, int M, int N, int W, size_t csize, size_t aux_bytes) {
  size_t off = (size_t)(twn + M + 1) * 2 * csize + (size_t)N * sizeof(int);
  off = (off + 15) & ~(size_t)15;
  return off + (size_t)W * N * 2 * csize + (size_t)W * aux_bytes;
}

constexpr int kTabChunk = 4;  // table elements per thread per batch

// Twiddle, post and digit-reversal tables into LDS.  One batch holds
// kTabChunk elements of each table per thread; indices are clamped so that
// all loads of a batch are issued before any store, and a kernel issues its
// first batch together with its other global loads (load), stores it after
// them (store), then finishes the tables (rest).
template <typename T>
struct TabChunk {
  V2<T> a[kTabChunk], p[kTabChunk];
  int d[kTabChunk];
  __device__ __forceinline__ void load(int e0, const V2<T> *__restrict__ tw, int twn,
                                       const V2<T> *__restrict__ post, int M,
                                       const int *__restrict__ drev, int N) {
    const int twmax = twn > 0 ? twn - 1 : 0;
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c) {
      const int e = e0 + (int)blockDim.x * c;
      a[c] = tw[e < twn ? e : twmax];
      p[c] = post[e <= M ? e : M];
      d[c] = drev[e < N ? e : N - 1];
    }
  }
  __device__ __forceinline__ void store(const WLayout<T> &Ly, int e0, int twn, int M, int N) const {
#pragma unroll
    for (int c = 0; c < kTabChunk; ++c) {
      const int e = e0 + (int)blockDim.x * c;
      if (e < twn) Ly.tw[e] = a[c];
      if (e <= M) Ly.post[e] = p[c];
      if (e < N) Ly.drev[e] = d[c];
    }
  }
  __device__ __forceinline__ void rest(const WLayout<T> &Ly, const V2<T> *__restrict__ tw, int twn,
                                       const V2<T> *__restrict__ post, int M,
                                       const int *__restrict__ drev, int N) {
    int tot = twn > M + 1 ? twn : M + 1;
    tot = tot > N ? tot : N;
    const int step = (int)blockDim.x * kTabChunk;
    for (int e0 = (int)threadIdx.x + step; e0 < tot; e0 += step) {
      load(e0, tw, twn, post, M, drev, N);
      store(Ly, e0, twn, M, N);
    }
  }
};

// One chunk of the packed sequence: raw interior values x_j for j = 2t and
// 2t + 1 (mirrored past M) and, for Bluestein, the chirp w_t; clamped
// indices so that every load is unconditional.
template <typename TSRC, typename T, bool BS, int G>
struct PackChunk {
  static constexpr int C = RC<G>::value, SL = 64 * G;
  T xr[C], xi[C];
  V2<T> w[BS ? C : 1];
  template <typename P>
  __device__ __forceinline__ void load(P src, long stride, int t0, int M,
                                       const V2<T> *__restrict__ chirp) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = t0 + SL * c;
      int j0 = 2 * t, j1 = 2 * t + 1;
      j0 = j0 < M ? j0 : 2 * M - j0;
      j1 = j1 < M ? j1 : 2 * M - j1;
      j0 = (j0 < 1 || j0 > M - 1) ? 1 : j0;  // tau = 0, M (value unused) or past the end
      j1 = (j1 < 1 || j1 > M - 1) ? 1 : j1;
      xr[c] = T(src[(long)j0 * stride]);
      xi[c] = T(src[(long)j1 * stride]);
      if constexpr (BS) w[c] = chirp[t < M ? t : 0];
    }
  }
};

// z_tau of the odd extension from a loaded raw value (ramp removed if asked)
template <typename T>
__device__ __forceinline__ T zfrom(T x, int tau, int M, bool ramp, T e0, T e1, T invM) {
  const bool zero = (tau == 0) | (tau == M);
  const int j = tau < M ? tau : 2 * M - tau;
  if (ramp) x -= e0 * (T(M - j) * invM) + e1 * (T(j) * invM);
  x = tau < M ? x : -x;
  return zero ? T(0) : x;
}

// Store one chunk at digit-reversed positions; Bluestein zero-pads t >= M.
template <typename TSRC, typename T, bool BS, int G>
__device__ __forceinline__ void pack_store(V2<T> *U, const int *s_drev,
                                           const PackChunk<TSRC, T, BS, G> &pc, int t0, int M,
                                           int N, bool active, bool ramp, T e0, T e1) {
  const T invM = T(1) / T(M);
  constexpr int C = PackChunk<TSRC, T, BS, G>::C;
  // all positions are read before the first store: a store to U could
  // alias the table for the compiler, which would then serialise every
  // read behind the previous store
  int pos[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int t = t0 + 64 * G * c;
    pos[c] = s_drev[t < N ? t : 0];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int t = t0 + 64 * G * c;
    V2<T> u{T(0), T(0)};
    if (active && t < M) {
      u.x = zfrom<T>(pc.xr[c], 2 * t, M, ramp, e0, e1, invM);
      u.y = zfrom<T>(pc.xi[c], 2 * t + 1, M, ramp, e0, e1, invM);
      if constexpr (BS) u = cmul(u, pc.w[c]);
    }
    if (t < N) U[pos[c]] = u;
  }
}

// Pack the whole sequence (chunk 0 already loaded into pc).
template <typename TSRC, typename T, bool BS, int G>
__device__ __forceinline__ void pack_all(V2<T> *U, const int *s_drev,
                                         PackChunk<TSRC, T, BS, G> &pc, const Gl<TSRC> *src,
                                         long stride, int lane, int M, int N, const V2<T> *chirp,
                                         bool active, bool ramp, T e0, T e1) {
  constexpr int step = 64 * G * RC<G>::value;
  pack_store<TSRC, T, BS, G>(U, s_drev, pc, lane, M, N, active, ramp, e0, e1);
  for (int t0 = lane + step; t0 < N; t0 += step) {
    pc.load(src, stride, t0, M, chirp);
    pack_store<TSRC, T, BS, G>(U, s_drev, pc, t0, M, N, active, ramp, e0, e1);
  }
}

// ---------------------------------------------------------------- rows

// Threads per workgroup the kernels are compiled for: 64 G per sequence,
// up to four sequences; with four wavefronts per sequence, two sequences
// (and so 256 registers per lane) unless the kernel computes in FP32 and
// is a Bluestein one, which then needs fewer than 128 registers.
template <typename T, int G, int MASK> struct WgMax {
  static constexpr int value =
      G < 4 ? 256 * G : (sizeof(T) == 4 && MASK != kMaskAll ? 1024 : 512);
};


template <typename TS, typename T, int MODE, bool BS, int G, int MASK>
__global__ __launch_bounds__((WgMax<T, G, MASK>::value)) void rows_w_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, int m, WDesc wd,
    const V2<T> *__restrict__ tw, const int *__restrict__ drev, const V2<T> *__restrict__ post,
    const V2<T> *__restrict__ chirp, const V2<T> *__restrict__ bhat, T alpha, T scale, T tau,
    const TS *__restrict__ f_true, double *__restrict__ partial, const XJob *__restrict__ jobs,
    int kit) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (jobs) {  // batched launch: problem blockIdx.y
    const XJob J = jobs[blockIdx.y];
    in = static_cast<const TS *>(J.in);
    out = static_cast<TS *>(J.out);
    f_true = static_cast<const TS *>(J.aux);
    partial = J.part ? J.part + (size_t)kit * J.nblk : nullptr;
  }
  const int M = MASK == kPlan1023 ? 1023 : wd.M;
  const int N = MASK == kPlan1023 || is_bs_static(MASK) ? plan_n(MASK) : wd.N;
  // G wavefronts per sequence; butterflies and elements are dealt to the
  // 64 G lanes of a sequence interleaved (lane-major across its waves)
  const int W = (blockDim.x >> 6) / G;
  const int wave = (threadIdx.x >> 6) / G;
  const int lane = (threadIdx.x & 63) * G + (threadIdx.x >> 6) % G;
  const int row = xcd_remap(blockIdx.x, gridDim.x) * W + wave;
  const bool active = row < n1;
  const size_t auxb = MODE == ROW_INV_UPDATE ? 2 * (size_t)m * sizeof(TS) : 0;
  const WLayout<T> Ly(smem_raw, wd.twn, M, N, W, wave, auxb);
  const Gl<TS> *src = gmem(in) + (size_t)(active ? row : 0) * m;
  Gl<TS> *dst = gmem(out) + (size_t)(active ? row : 0) * m;
  const Gl<TS> *fr = f_true ? gmem(f_true) + (size_t)(active ? row : 0) * m : nullptr;
  TS *sx = reinterpret_cast<TS *>(Ly.aux);
  TS *sf = sx + m;
  // one batch of global loads: this wave's row, x and f (update), the
  // first table batch; then the LDS stores
  PackChunk<TS, T, BS, G> pc;
  pc.load(src, 1, lane, M, chirp);
  const T e0 = T(src[0]), e1 = T(src[m - 1]);
  constexpr int RCV = RC<G>::value;
  TS ax[RCV], af[RCV];
  if (MODE == ROW_INV_UPDATE) {
#pragma unroll
    for (int c = 0; c < RCV; ++c) {
      const int kr = lane + 64 * G * c;
      const int k = kr < m ? kr : m - 1;
      ax[c] = dst[k];
      af[c] = fr ? fr[k] : TS(0);
    }
  }
  TabChunk<T> tb;
  tb.load(threadIdx.x, tw, wd.twn, post, M, drev, N);
  if (MODE == ROW_INV_UPDATE) {
#pragma unroll
    for (int c = 0; c < RCV; ++c) {
      const int k = lane + 64 * G * c;
      if (k < m) {
        sx[k] = ax[c];
        sf[k] = af[c];
      }
    }
    for (int k0 = lane + 64 * G * RCV; k0 < m; k0 += 64 * G * RCV) {
#pragma unroll
      for (int c = 0; c < RCV; ++c) {
        const int kr = k0 + 64 * G * c;
        const int k = kr < m ? kr : m - 1;
        ax[c] = dst[k];
        af[c] = fr ? fr[k] : TS(0);
      }
#pragma unroll
      for (int c = 0; c < RCV; ++c) {
        const int k = k0 + 64 * G * c;
        if (k < m) {
          sx[k] = ax[c];
          sf[k] = af[c];
        }
      }
    }
  }
  tb.store(Ly, threadIdx.x, wd.twn, M, N);
  tb.rest(Ly, tw, wd.twn, post, M, drev, N);
  __syncthreads();
  pack_all<TS, T, BS, G>(Ly.U, Ly.drev, pc, src, 1, lane, M, N, chirp, active, MODE == ROW_FWD, e0,
                      e1);
  __syncthreads();
  fft_full<T, BS, G, MASK>(Ly.U, wd, Ly.tw, bhat, lane);
  double ss = 0.0;
  if (active) {
    const T invM = T(1) / T(M);
    for (int k0 = lane; k0 < m; k0 += 64 * G * PC<G>::value) {
      T val[PC<G>::value];
#pragma unroll
      for (int c = 0; c < PC<G>::value; ++c) {
        const int kr = k0 + 64 * G * c;
        const int k = kr < m ? kr : k0;
        val[c] = wcoef<T, MODE != ROW_FWD, BS>(Ly.U, Ly.drev, chirp, k, M, Ly.post, scale, alpha,
                                               e0, e1, invM);
      }
#pragma unroll
      for (int c = 0; c < PC<G>::value; ++c) {
        const int k = k0 + 64 * G * c;
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
    if (threadIdx.x == 0) gmem(partial)[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------- columns

// Column block I/O (mixed-radix plans): the W columns of a workgroup are
// read and written row by row by all its threads (thread t always serves
// column t mod W), so one memory instruction covers 64 / W rows of W
// adjacent elements instead of 64 rows of one element.  Row r of column c
// is the odd-extension value z_r: it goes to the real or imaginary half of
// the packed entry u_{r/2} (digit-reversed position) and, negated, to that
// of u_{(2M - r)/2}.
template <typename TS, int C>
struct BlockChunk {
  TS v[C];
  __device__ __forceinline__ void load(const Gl<TS> *col, long ld, int r0, int rstep, int m) {
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const int r = r0 + rstep * i;
      v[i] = col[(long)(r < m ? r : m - 1) * ld];
    }
  }
};

template <typename TS, typename T, int C>
__device__ __forceinline__ void block_scatter(V2<T> *Uc, const int *s_drev,
                                              const BlockChunk<TS, C> &bc, int r0, int rstep,
                                              int M, bool cact, bool ramp, T e0, T e1, T invM) {
  T *Uf = reinterpret_cast<T *>(Uc);
  // positions first (see pack_store), then the stores
  int p0[C], p1[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int r = r0 + rstep * i;
    const int rc = r < M ? r : M;
    const int tm = 2 * M - (r >= 1 && r <= M - 1 ? r : 1);
    p0[i] = 2 * s_drev[rc >> 1] + (rc & 1);
    p1[i] = 2 * s_drev[tm >> 1] + (tm & 1);
  }
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int r = r0 + rstep * i;
    if (r > M) continue;
    T z = T(bc.v[i]);
    if (ramp) z -= e0 * (T(M - r) * invM) + e1 * (T(r) * invM);
    z = (cact && r != 0 && r != M) ? z : T(0);
    Uf[p0[i]] = z;
    if (r >= 1 && r <= M - 1) Uf[p1[i]] = -z;
  }
}

// Rows per thread per batch of block I/O: a column block moves in rows of
// 64 G threads (one per row and column of the block), so 16 / G rows per
// thread cover 1024 rows in one batch with no clamped duplicate loads.
template <int G> struct BlockRows { static constexpr int value = 16 / G; };

template <typename TS, typename T, int MODE, bool BS, int G, int MASK>
__global__ __launch_bounds__((WgMax<T, G, MASK>::value)) void cols_w_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int m, int n2, WDesc wd,
    const V2<T> *__restrict__ tw, const int *__restrict__ drev, const V2<T> *__restrict__ post,
    const V2<T> *__restrict__ chirp, const V2<T> *__restrict__ bhat, T alpha, T scale,
    const TS *__restrict__ dT, const XJob *__restrict__ jobs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (jobs) {  // batched launch: problem blockIdx.y
    const XJob J = jobs[blockIdx.y];
    in = static_cast<const TS *>(J.in);
    out = static_cast<TS *>(J.out);
    dT = static_cast<const TS *>(J.aux);
  }
  // block I/O for mixed-radix plans; Bluestein plans (zero padding, chirp
  // products) pack per wave from strided loads
  constexpr bool BIO = !BS;
  const int M = MASK == kPlan1023 ? 1023 : wd.M;
  const int N = MASK == kPlan1023 || is_bs_static(MASK) ? plan_n(MASK) : wd.N;
  // G wavefronts per sequence; butterflies and elements are dealt to the
  // 64 G lanes of a sequence interleaved (lane-major across its waves)
  const int W = (blockDim.x >> 6) / G;
  const int wave = (threadIdx.x >> 6) / G;
  const int lane = (threadIdx.x & 63) * G + (threadIdx.x >> 6) % G;
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * W;
  const int col = col0 + wave;
  const bool active = col < n2;
  // per-wave staging row: the filter column, then (block I/O) the outputs
  const size_t auxb = (BIO || MODE == COL_FWD_D_INV) ? (size_t)m * sizeof(T) : 0;
  const WLayout<T> Ly(smem_raw, wd.twn, M, N, W, wave, auxb);
  T *S = reinterpret_cast<T *>(Ly.aux);
  const long ld = n2;
  const Gl<TS> *src = gmem(in) + (active ? col : 0);
  T e0 = T(src[0]);
  T e1 = T(src[(long)(m - 1) * ld]);
  const T invM = T(1) / T(M);
  // block I/O: this thread's column of the block and its rows
  const int bc_c = threadIdx.x % W, bc_r0 = threadIdx.x / W, bc_step = blockDim.x / W;
  const bool bc_act = col0 + bc_c < n2;
  const Gl<TS> *bsrc = gmem(in) + (bc_act ? col0 + bc_c : 0);
  V2<T> *const U0 = Ly.U - (size_t)wave * N;
  T *const S0 = reinterpret_cast<T *>(Ly.aux - (size_t)wave * auxb);
  T be0 = T(0), be1 = T(0);
  BlockChunk<TS, BlockRows<G>::value> bch;
  PackChunk<TS, T, BS, G> pc;
  TabChunk<T> tb;
  // the filter of this wave's column: one contiguous row of the transposed
  // filter (stored over the staging row, overwritten in place below)
  constexpr int RCV = RC<G>::value;
  const Gl<TS> *dcol = gmem(dT) + (size_t)(active ? col : 0) * m;
  TS dv[RCV];
  if (MODE == COL_FWD_D_INV) {
#pragma unroll
    for (int c = 0; c < RCV; ++c) {
      const int k = lane + 64 * G * c;
      dv[c] = dcol[k < m ? k : m - 1];
    }
  }
  // one batch of global loads (column or column block, filter, first table
  // batch), then the LDS stores
  if constexpr (BIO) {
    bch.load(bsrc, ld, bc_r0, bc_step, m);
    be0 = T(bsrc[0]);
    be1 = T(bsrc[(long)(m - 1) * ld]);
  } else {
    pc.load(src, ld, lane, M, chirp);
  }
  tb.load(threadIdx.x, tw, wd.twn, post, M, drev, N);
  if (MODE == COL_FWD_D_INV) {
    for (int k0 = lane;;) {
#pragma unroll
      for (int c = 0; c < RCV; ++c) {
        const int k = k0 + 64 * G * c;
        if (k < m) S[k] = T(dv[c]);
      }
      k0 += 64 * G * RCV;
      if (k0 >= m) break;
#pragma unroll
      for (int c = 0; c < RCV; ++c) {
        const int k = k0 + 64 * G * c;
        dv[c] = dcol[k < m ? k : m - 1];
      }
    }
  }
  tb.store(Ly, threadIdx.x, wd.twn, M, N);
  tb.rest(Ly, tw, wd.twn, post, M, drev, N);
  __syncthreads();
  // pass 0: the column with the ramp removed (forward) or as is (inverse)
  if constexpr (BIO) {
    V2<T> *Uc = U0 + (size_t)bc_c * N;
    const bool ramp = MODE != COL_INV;
    block_scatter<TS, T, BlockRows<G>::value>(Uc, Ly.drev, bch, bc_r0, bc_step, M, bc_act, ramp, be0, be1,
                                      invM);
    for (int r0 = bc_r0 + bc_step * BlockRows<G>::value; r0 < m; r0 += bc_step * BlockRows<G>::value) {
      bch.load(bsrc, ld, r0, bc_step, m);
      block_scatter<TS, T, BlockRows<G>::value>(Uc, Ly.drev, bch, r0, bc_step, M, bc_act, ramp, be0, be1,
                                        invM);
    }
  } else {
    pack_all<TS, T, BS, G>(Ly.U, Ly.drev, pc, src, ld, lane, M, N, chirp, active, MODE != COL_INV,
                           e0, e1);
  }
  __syncthreads();
  fft_full<T, BS, G, MASK>(Ly.U, wd, Ly.tw, bhat, lane);
  if constexpr (MODE == COL_FWD_D_INV) {
    // S[k] <- d_k * (T~ y)_k (each lane reads and writes only its own S[k])
    for (int k0 = lane; k0 < m; k0 += 64 * G * PC<G>::value) {
      T val[PC<G>::value];
#pragma unroll
      for (int c = 0; c < PC<G>::value; ++c) {
        const int kr = k0 + 64 * G * c;
        const int k = kr < m ? kr : k0;
        val[c] = wcoef<T, false, BS>(Ly.U, Ly.drev, chirp, k, M, Ly.post, scale, alpha, e0, e1,
                                     invM);
      }
#pragma unroll
      for (int c = 0; c < PC<G>::value; ++c) {
        const int k = k0 + 64 * G * c;
        if (k < m) S[k] = val[c] * S[k];
      }
    }
    __syncthreads();
    // pass 1: the inverse transform of the filtered coefficients
    e0 = S[0];
    e1 = S[m - 1];
    PackChunk<T, T, BS, G> ps;
    for (int t0 = lane; t0 < N; t0 += 64 * G * RC<G>::value) {
      ps.load(S, 1, t0, M, chirp);
      pack_store<T, T, BS, G>(Ly.U, Ly.drev, ps, t0, M, N, active, false, e0, e1);
    }
    __syncthreads();
    fft_full<T, BS, G, MASK>(Ly.U, wd, Ly.tw, bhat, lane);
  }
  // outputs of this wave's column: straight to memory, or (block I/O)
  // through the staging row and then row by row for the whole block
  for (int k0 = lane; k0 < m; k0 += 64 * G * PC<G>::value) {
    T val[PC<G>::value];
#pragma unroll
    for (int c = 0; c < PC<G>::value; ++c) {
      const int kr = k0 + 64 * G * c;
      const int k = kr < m ? kr : k0;
      val[c] = wcoef<T, MODE != COL_FWD, BS>(Ly.U, Ly.drev, chirp, k, M, Ly.post, scale, alpha,
                                             e0, e1, invM);
    }
#pragma unroll
    for (int c = 0; c < PC<G>::value; ++c) {
      const int k = k0 + 64 * G * c;
      if (k >= m) continue;
      if constexpr (BIO) S[k] = val[c];
      else if (active) gmem(out)[(long)k * ld + col] = TS(val[c]);
    }
  }
  if constexpr (BIO) {
    __syncthreads();
    const T *Sc = S0 + (size_t)bc_c * m;
    Gl<TS> *bdst = gmem(out) + col0 + bc_c;
    if (bc_act) {
      for (int r0 = bc_r0; r0 < m; r0 += bc_step * BlockRows<G>::value) {
        T v[BlockRows<G>::value];
#pragma unroll
        for (int i = 0; i < BlockRows<G>::value; ++i) {
          const int r = r0 + bc_step * i;
          v[i] = Sc[r < m ? r : m - 1];
        }
#pragma unroll
        for (int i = 0; i < BlockRows<G>::value; ++i) {
          const int r = r0 + bc_step * i;
          if (r < m) bdst[(long)r * ld] = TS(v[i]);
        }
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

constexpr size_t kMaxLdsW = 150 * 1024;

// Waves (sequences) per workgroup: `forced` if it fits, else the largest
// power of two <= 4 whose LDS fits; never more than `cap`.
int wave_count(size_t fixed, size_t per_wave, int nseq, int forced, int cap) {
  if (forced == 1 || forced == 2 || forced == 4) {
    int W = forced < cap ? forced : cap;
    while (W > 1 && fixed + (size_t)W * per_wave > kMaxLdsW) W >>= 1;
    return W;
  }
  int W = cap;
  while (W > 1 && fixed + (size_t)W * per_wave > kMaxLdsW) W >>= 1;
  while (W > 1 && W / 2 >= nseq) W >>= 1;
  return W;
}

// With the exclusive flag the dynamic LDS is padded so that one workgroup
// occupies a CU (the dispatcher then spreads workgroups over all CUs).
size_t excl_pad(size_t smem, int excl) { return excl && smem < 81 * 1024 ? 81 * 1024 : smem; }

template <typename K>
hipError_t allow_lds_w(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

WDesc make_wdesc(const WavePlan &w) {
  WDesc d{};
  d.M = w.M;
  d.N = w.N;
  d.bs = w.bs ? 1 : 0;
  d.nst = w.nst;
  d.twn = w.twn;
  for (int s = 0; s < kMaxStages; ++s) {
    d.R[s] = w.R[s];
    d.L[s] = w.L[s];
    d.tw_off[s] = w.tw_off[s];
  }
  return d;
}

// In-place iterative radix-2 FFT (host, FP64) of a power-of-two length;
// run once per plan for the chirp spectrum.
void host_fft(std::vector<std::complex<double>> &a) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t k = 0; k < len / 2; ++k) {
      const double ang = -2.0 * M_PI * (double)k / (double)len;
      const std::complex<double> w(std::cos(ang), std::sin(ang));
      for (size_t i = 0; i < n; i += len) {
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

template <typename T>
int upload_complex(void **dst, const std::vector<std::complex<double>> &v) {
  std::vector<V2<T>> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = {T(v[i].real()), T(v[i].imag())};
  AR_HIP(hipMalloc(dst, (h.empty() ? 1 : h.size()) * sizeof(V2<T>)));
  AR_HIP(hipMemcpy(*dst, h.data(), h.size() * sizeof(V2<T>), hipMemcpyHostToDevice));
  return AR_OK;
}

}  // namespace

// Mixed radix: factor M into codelet radices (4s first, then odd primes),
// largest radix first; not applicable when a prime factor exceeds 31.
// Bluestein: N = smallest power of two >= 2M - 1 in radices 4 (and one 2),
// chirp w_j = e^{-i pi j^2 / M} (j^2 reduced mod 2M exactly), and
// bhat = FFT_N(b) / N with b_j = conj(w_j) and b_{N-j} = b_j.
// Both build their digit-reversal and twiddle tables.
int wave_plan_build(WavePlan &w, int M, bool cdouble, bool bluestein, hipStream_t st) {
  w = WavePlan{};
  w.M = M;
  if (M < 2) return AR_OK;
  std::vector<int> rad;
  int N = M;
  if (bluestein) {
    N = 1;
    while (N < 2 * M - 1) N <<= 1;
    int r = N;
    while (r % 4 == 0) { rad.push_back(4); r /= 4; }
    while (r % 2 == 0) { rad.push_back(2); r /= 2; }
  } else {
    int r = M;
    while (r % 4 == 0) { rad.push_back(4); r /= 4; }
    while (r % 2 == 0) { rad.push_back(2); r /= 2; }
    for (int p = 3; p <= 31 && r > 1; p += 2)
      while (r % p == 0 && cl::has_codelet(p)) { rad.push_back(p); r /= p; }
    if (r != 1 || rad.empty()) return AR_OK;  // not applicable
    std::sort(rad.begin(), rad.end(), [](int a, int b) { return a > b; });
  }
  if (rad.empty() || (int)rad.size() > kMaxStages) return AR_OK;
  w.N = N;
  w.bs = bluestein;
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
  w.twn = (int)off;
  // digit reversal: natural index n has digits (most significant first)
  // p_0..p_{s-1} in radices R_0..R_{s-1}; its position is sum_t p_t prod_{u<t} R_u
  std::vector<int> drev(N);
  for (int n = 0; n < N; ++n) {
    int rem = n, pos = 0, wpos = 1, wnat = N;
    for (int t = 0; t < w.nst; ++t) {
      wnat /= w.R[t];
      const int d = rem / wnat;
      rem -= d * wnat;
      pos += d * wpos;
      wpos *= w.R[t];
    }
    drev[n] = pos;
  }
  const size_t cb = cdouble ? sizeof(double2) : sizeof(float2);
  AR_HIP(hipMalloc(&w.tw, (off > 0 ? off : 1) * cb));
  AR_HIP(hipMalloc((void **)&w.drev, (size_t)N * sizeof(int)));
  AR_HIP(hipMemcpy(w.drev, drev.data(), (size_t)N * sizeof(int), hipMemcpyHostToDevice));
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
  if (bluestein) {
    std::vector<std::complex<double>> chirp(M), b(N, 0.0);
    for (int j = 0; j < M; ++j) {
      const long jj = ((long)j * j) % (2L * M);
      const double ang = -M_PI * (double)jj / (double)M;
      chirp[j] = std::complex<double>(std::cos(ang), std::sin(ang));
    }
    for (int j = 0; j < M; ++j) b[j] = std::conj(chirp[j]);
    for (int j = 1; j < M; ++j) b[N - j] = std::conj(chirp[j]);
    host_fft(b);
    for (auto &v : b) v /= (double)N;
    int rc = cdouble ? upload_complex<double>(&w.chirp, chirp)
                     : upload_complex<float>(&w.chirp, chirp);
    if (rc != AR_OK) return rc;
    rc = cdouble ? upload_complex<double>(&w.bhat, b) : upload_complex<float>(&w.bhat, b);
    if (rc != AR_OK) return rc;
  }
  w.ok = true;
  return AR_OK;
}

void wave_plan_free(WavePlan &w) {
  if (w.tw) (void)hipFree(w.tw);
  if (w.drev) (void)hipFree(w.drev);
  if (w.chirp) (void)hipFree(w.chirp);
  if (w.bhat) (void)hipFree(w.bhat);
  w.tw = w.chirp = w.bhat = nullptr;
  w.drev = nullptr;
  w.ok = false;
}

// The compile-time Bluestein plan matching w (FP32 tables only), or 0:
// N = 2^k for k = 8, 9, 10 with the stage layout bs_stages assumes.
static int bs_static_mask(const WavePlan &w) {
  if (!w.bs) return 0;
  int k = 0;
  while ((1 << k) < w.N) ++k;
  if ((1 << k) != w.N || -k < kPlanBSMin || -k > kPlanBSMax) return 0;
  int L = 1;
  for (int s = 0; s < w.nst; ++s) {
    const int R = (w.N / L) % 4 == 0 ? 4 : 2;
    if (w.R[s] != R || w.L[s] != L || w.tw_off[s] != L - 1) return 0;
    L *= R;
  }
  return L == w.N ? -k : 0;
}

// The mixed-radix plan of M = 1023 with the stage layout the fixed-plan
// kernels assume.
static bool is_plan1023(const WavePlan &w) {
  return !w.bs && w.M == 1023 && w.N == 1023 && w.nst == 3 && w.R[0] == 31 && w.R[1] == 11 &&
         w.R[2] == 3 && w.L[0] == 1 && w.L[1] == 31 && w.L[2] == 341 && w.tw_off[0] == 0 &&
         w.tw_off[1] == 30 && w.tw_off[2] == 340;
}

// Wavefronts per sequence from the lanes tunable (0 = one).
static int lanes_of(int v) { return v == 2 || v == 4 ? v : 1; }

static size_t rows_aux(const ar_plan_s *p) { return 2 * (size_t)p->n2 * p->esize; }
static size_t cols_aux(const ar_plan_s *p) { return (size_t)p->n1 * p->csize; }

static bool fits(const WavePlan &w, const ar_plan_s *p, size_t aux) {
  return w.ok && wlds_bytes(w.twn, w.M, w.N, 1, p->csize, aux) <= kMaxLdsW;
}

// FFT form per axis: the tunable (1 mixed radix, 2 Bluestein) when that
// plan exists and fits in LDS, else mixed radix when it does, else Bluestein.
static const WavePlan *pick(const FftPlan &fp, int algo, const ar_plan_s *p, size_t aux) {
  if (algo == 1 && fits(fp.w, p, aux)) return &fp.w;
  if (algo == 2 && fits(fp.wb, p, aux)) return &fp.wb;
  if (fits(fp.w, p, aux)) return &fp.w;
  if (fits(fp.wb, p, aux)) return &fp.wb;
  return nullptr;
}
static const WavePlan *row_plan(const ar_plan_s *p) {
  return pick(p->fft_row, p->tune[AR_TUNE_ROW_ALGO], p, rows_aux(p));
}
static const WavePlan *col_plan(const ar_plan_s *p) {
  return pick(p->fft_col, p->tune[AR_TUNE_COL_ALGO], p, cols_aux(p));
}

// Wavefronts per sequence of an axis from its lanes tunable: 0 (auto) is two
// for the mixed-radix plan of length 1023, one otherwise.
static int axis_lanes(const WavePlan &w, int tune) {
  return tune == 0 ? (is_plan1023(w) ? 2 : 1) : lanes_of(tune);
}

// The length-1024 kernels (two or four wavefronts per sequence) serve the
// mixed-radix plan of length 1023.
static bool use_x1023(const WavePlan &w, int lanes) {
  return is_plan1023(w) && axis_lanes(w, lanes) >= 2;
}

// Sequences per workgroup the kernel of a plan axis was compiled for (the
// host side of WgMax): two with four wavefronts per sequence unless the
// FFT is a Bluestein plan computed in FP32.  The same for every compute
// type of a plan, so that all its row passes share one grid.
static int seq_cap(const ar_plan_s *p, const WavePlan &w, int lanes) {
  if (use_x1023(w, lanes)) return x1023_cap(axis_lanes(w, lanes));
  if (axis_lanes(w, lanes) < 4) return 4;
  return p->csize == 4 && w.bs ? 4 : 2;
}

static int rows_waves(const ar_plan_s *p, const WavePlan &w) {
  const int lanes = p->tune[AR_TUNE_ROW_LANES];
  if (use_x1023(w, lanes))
    return wave_count(0, x1023_lds(1, p->csize), p->n1, p->tune[AR_TUNE_ROW_WAVES],
                      seq_cap(p, w, lanes));
  const size_t fixed = wlds_bytes(w.twn, w.M, w.N, 0, p->csize, 0);
  return wave_count(fixed, (size_t)w.N * 2 * p->csize + rows_aux(p), p->n1,
                    p->tune[AR_TUNE_ROW_WAVES], seq_cap(p, w, lanes));
}
static int cols_waves(const ar_plan_s *p, const WavePlan &w) {
  const int lanes = p->tune[AR_TUNE_COL_LANES];
  if (use_x1023(w, lanes)) {
    // the column blocks of the length-1024 kernels move whole: W divides n2
    int W = wave_count(0, x1023_lds(1, p->csize), p->n2, p->tune[AR_TUNE_COL_WAVES],
                       seq_cap(p, w, lanes));
    while (W > 1 && p->n2 % W) W >>= 1;
    return W;
  }
  const size_t fixed = wlds_bytes(w.twn, w.M, w.N, 0, p->csize, 0);
  return wave_count(fixed, (size_t)w.N * 2 * p->csize + cols_aux(p), p->n2,
                    p->tune[AR_TUNE_COL_WAVES], seq_cap(p, w, lanes));
}

bool wave_rows_ok(const ar_plan_s *p) { return row_plan(p) != nullptr; }
bool wave_cols_ok(const ar_plan_s *p) { return col_plan(p) != nullptr; }

int wave_rows_blocks(const ar_plan_s *p) {
  const int W = rows_waves(p, *row_plan(p));
  return (p->n1 + W - 1) / W;
}

// 1 = mixed radix, 2 = Bluestein, 0 = neither (block-wide engine)
int wave_rows_algo(const ar_plan_s *p) {
  const WavePlan *w = row_plan(p);
  return w ? (w->bs ? 2 : 1) : 0;
}
int wave_cols_algo(const ar_plan_s *p) {
  const WavePlan *w = col_plan(p);
  return w ? (w->bs ? 2 : 1) : 0;
}

template <typename TS, typename T, bool BS, int G, int MASK>
static int wave_rows_t(const ar_plan_s *p, const FftPlan &fp, const WavePlan &w, const void *in,
                       void *out, int mode, double tau, const void *f_true, double *partial,
                       const XJob *jobs, int count, int kit, hipStream_t st) {
  const int m = p->n2, M = w.M;
  // geometry from the plan's own tables, so that the FP32 variant has the
  // same grid (and partial-sum count) as the compute-type one
  const int W = rows_waves(p, *row_plan(p));
  const int blocks = (p->n1 + W - 1) / W;
  const dim3 grid(blocks, count);
  const size_t smem =
      excl_pad(wlds_bytes(w.twn, M, w.N, W, sizeof(T), rows_aux(p)), p->tune[AR_TUNE_ROW_EXCL]);
  const WDesc wd = make_wdesc(w);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(w.tw);
  auto post = static_cast<const V2<T> *>(fp.post);
  auto chirp = static_cast<const V2<T> *>(w.chirp);
  auto bhat = static_cast<const V2<T> *>(w.bhat);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  hipError_t e = hipSuccess;
#define AR_WROWS(MODE)                                                                          \
  e = allow_lds_w(rows_w_kernel<TS, T, MODE, BS, G, MASK>, smem);                                     \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((rows_w_kernel<TS, T, MODE, BS, G, MASK>), grid, dim3(64 * W * G), smem, st,  \
                       ti, to,                                                                  \
                       p->n1, m, wd, tw, w.drev, post, chirp, bhat, alpha, scale, T(tau), tf,    \
                       partial, jobs, kit);                                                     \
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

template <typename TS, typename T>
static int wave_rows_d(const ar_plan_s *p, const FftPlan &fp, const void *in, void *out, int mode,
                       double tau, const void *f_true, double *partial, const XJob *jobs,
                       int count, int kit, hipStream_t st) {
  // the FFT form chosen for the plan, from the tables `fp`
  const WavePlan &w = row_plan(p)->bs ? fp.wb : fp.w;
  const int gl = axis_lanes(w, p->tune[AR_TUNE_ROW_LANES]);
#define AR_R(BS_, MASK_)                                                                       \
  (gl == 4   ? wave_rows_t<TS, T, BS_, 4, MASK_>(p, fp, w, in, out, mode, tau, f_true, partial, \
                                                 jobs, count, kit, st)                         \
   : gl == 2 ? wave_rows_t<TS, T, BS_, 2, MASK_>(p, fp, w, in, out, mode, tau, f_true, partial, \
                                                 jobs, count, kit, st)                         \
             : wave_rows_t<TS, T, BS_, 1, MASK_>(p, fp, w, in, out, mode, tau, f_true, partial, \
                                                 jobs, count, kit, st))
  if (w.bs) {
    if constexpr (std::is_same<T, float>::value) {
      switch (bs_static_mask(w)) {
        case -8: return AR_R(true, -8);
        case -9: return AR_R(true, -9);
        case -10: return AR_R(true, -10);
        default: break;
      }
    }
    return AR_R(true, 0);
  }
  if (is_plan1023(w)) {
    if (gl == 1)
      return wave_rows_t<TS, T, false, 1, kPlan1023>(p, fp, w, in, out, mode, tau, f_true,
                                                     partial, jobs, count, kit, st);
    const int W = rows_waves(p, *row_plan(p));
    const double m = p->n2, M = w.M;
    // Rows in pairs (two per complex FFT, four wavefronts per pair) for the
    // FP64-arithmetic passes.  Their odd DST outputs come from a running
    // sum, which in FP32 arithmetic carries about ten times the rounding of
    // the one-row form (inverse transform 2.7e-6 against 2.7e-7 at 1024^2),
    // so FP32 passes keep the one-row form; in FP64 the transforms stay near
    // 5e-15.  Workgroups of one row (the ROW_WAVES tunable at 1) keep it too.
    if (!jobs && W % 2 == 0 && sizeof(T) == 8) {
      const size_t psmem = excl_pad(x1023_pair_lds(W / 2, sizeof(T)), p->tune[AR_TUNE_ROW_EXCL]);
      return x1023_rows_pair_launch(sizeof(TS), sizeof(T), in, out, p->n1, W, 4, psmem,
                                    mode, w.tw, fp.post,
                                    std::sqrt(m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))),
                                    std::sqrt(2.0 / M) / 4.0, tau, f_true, partial, st);
    }
    const size_t smem = excl_pad(x1023_lds(W, sizeof(T)), p->tune[AR_TUNE_ROW_EXCL]);
    return x1023_rows_launch(sizeof(TS), sizeof(T), in, out, p->n1, W, gl, smem, mode, w.tw,
                             fp.post, std::sqrt(m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))),
                             std::sqrt(2.0 / M) / 4.0, tau, f_true, partial, jobs, count, kit,
                             st);
  }
  return AR_R(false, kMaskAll);
#undef AR_R
}

static int wave_rows_any(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                         const void *f_true, double *partial, const XJob *jobs, int count,
                         int kit, hipStream_t st) {
  if (p->dtype == AR_F64)
    return wave_rows_d<double, double>(p, p->fft_row, in, out, mode, tau, f_true, partial, jobs,
                                       count, kit, st);
  if (p->dtype == AR_F32_ACC64) {
    // the iteration's inverse row pass follows the filter, which does not
    // amplify its rounding: FP32 arithmetic there, FP64 everywhere else
    const WavePlan &w32 = row_plan(p)->bs ? p->fft_row32.wb : p->fft_row32.w;
    if (mode == ROW_INV_UPDATE && w32.ok)
      return wave_rows_d<float, float>(p, p->fft_row32, in, out, mode, tau, f_true, partial,
                                       jobs, count, kit, st);
    return wave_rows_d<float, double>(p, p->fft_row, in, out, mode, tau, f_true, partial, jobs,
                                      count, kit, st);
  }
  return wave_rows_d<float, float>(p, p->fft_row, in, out, mode, tau, f_true, partial, jobs,
                                   count, kit, st);
}

int wave_rows_launch(const ar_plan_s *p, const void *in, void *out, int mode, double tau,
                     const void *f_true, double *partial, hipStream_t st) {
  return wave_rows_any(p, in, out, mode, tau, f_true, partial, nullptr, 1, 0, st);
}

int wave_rows_launch_batch(const ar_plan_s *lead, const XJob *jobs, int count, int mode,
                           double tau, int k, hipStream_t st) {
  if (count == 0) return AR_OK;
  if (!wave_rows_ok(lead)) return fail(AR_EUNSUPPORTED, "batched transform: row length too large");
  return wave_rows_any(lead, nullptr, nullptr, mode, tau, nullptr, nullptr, jobs, count, k, st);
}

template <typename TS, typename T, bool BS, int G, int MASK>
static int wave_cols_t(const ar_plan_s *p, const WavePlan &w, const void *in, void *out, int mode,
                       const XJob *jobs, int count, hipStream_t st) {
  const int m = p->n1, M = w.M;
  const int W = cols_waves(p, w);
  const int blocks = (p->n2 + W - 1) / W;
  const dim3 grid(blocks, count);
  const size_t smem =
      excl_pad(wlds_bytes(w.twn, M, w.N, W, sizeof(T), cols_aux(p)), p->tune[AR_TUNE_COL_EXCL]);
  const WDesc wd = make_wdesc(w);
  const T alpha = T(std::sqrt((double)m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))));
  const T scale = T(std::sqrt(2.0 / M) / 4.0);
  auto tw = static_cast<const V2<T> *>(w.tw);
  auto post = static_cast<const V2<T> *>(p->fft_col.post);
  auto chirp = static_cast<const V2<T> *>(w.chirp);
  auto bhat = static_cast<const V2<T> *>(w.bhat);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const TS *>(p->dT);
  hipError_t e = hipSuccess;
#define AR_WCOLS(MODE)                                                                          \
  e = allow_lds_w(cols_w_kernel<TS, T, MODE, BS, G, MASK>, smem);                                     \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((cols_w_kernel<TS, T, MODE, BS, G, MASK>), grid, dim3(64 * W * G), smem, st,  \
                       ti, to,                                                                  \
                       m, p->n2, wd, tw, w.drev, post, chirp, bhat, alpha, scale, td, jobs);   \
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

template <typename TS, typename T>
static int wave_cols_d(const ar_plan_s *p, const void *in, void *out, int mode, const XJob *jobs,
                       int count, hipStream_t st) {
  const WavePlan &w = *col_plan(p);
  const int gl = axis_lanes(w, p->tune[AR_TUNE_COL_LANES]);
#define AR_C(BS_, MASK_)                                                                       \
  (gl == 4   ? wave_cols_t<TS, T, BS_, 4, MASK_>(p, w, in, out, mode, jobs, count, st)          \
   : gl == 2 ? wave_cols_t<TS, T, BS_, 2, MASK_>(p, w, in, out, mode, jobs, count, st)          \
             : wave_cols_t<TS, T, BS_, 1, MASK_>(p, w, in, out, mode, jobs, count, st))
  if (w.bs) {
    if constexpr (std::is_same<T, float>::value) {
      switch (bs_static_mask(w)) {
        case -8: return AR_C(true, -8);
        case -9: return AR_C(true, -9);
        case -10: return AR_C(true, -10);
        default: break;
      }
    }
    return AR_C(true, 0);
  }
  if (is_plan1023(w)) {
    if (gl == 1) return wave_cols_t<TS, T, false, 1, kPlan1023>(p, w, in, out, mode, jobs, count, st);
    const int W = cols_waves(p, w);
    const double m = p->n1, M = w.M;
    // columns in pairs for FP64 arithmetic (as the row passes)
    if (!jobs && W % 2 == 0 && sizeof(T) == 8) {
      const size_t psmem = excl_pad(x1023_pair_lds(W / 2, sizeof(T)), p->tune[AR_TUNE_COL_EXCL]);
      return x1023_cols_pair_launch(sizeof(TS), sizeof(T), in, out, p->n2, W, psmem, mode, w.tw,
                                    p->fft_col.post,
                                    std::sqrt(m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))),
                                    std::sqrt(2.0 / M) / 4.0, p->dT, st);
    }
    const size_t smem = excl_pad(x1023_lds(W, sizeof(T)), p->tune[AR_TUNE_COL_EXCL]);
    return x1023_cols_launch(sizeof(TS), sizeof(T), in, out, p->n2, W, gl, smem, mode, w.tw,
                             p->fft_col.post, std::sqrt(m * (2.0 * m - 1.0) / (6.0 * (m - 1.0))),
                             std::sqrt(2.0 / M) / 4.0, p->dT, jobs, count, st);
  }
  return AR_C(false, kMaskAll);
#undef AR_C
}

static int wave_cols_any(const ar_plan_s *p, const void *in, void *out, int mode,
                         const XJob *jobs, int count, hipStream_t st) {
  if (p->dtype == AR_F64) return wave_cols_d<double, double>(p, in, out, mode, jobs, count, st);
  if (p->dtype == AR_F32_ACC64)
    return wave_cols_d<float, double>(p, in, out, mode, jobs, count, st);
  return wave_cols_d<float, float>(p, in, out, mode, jobs, count, st);
}

int wave_cols_launch(const ar_plan_s *p, const void *in, void *out, int mode, hipStream_t st) {
  return wave_cols_any(p, in, out, mode, nullptr, 1, st);
}

int wave_cols_launch_batch(const ar_plan_s *lead, const XJob *jobs, int count, int mode,
                           hipStream_t st) {
  if (count == 0) return AR_OK;
  if (!wave_cols_ok(lead))
    return fail(AR_EUNSUPPORTED, "batched transform: column length too large");
  return wave_cols_any(lead, nullptr, nullptr, mode, jobs, count, st);
}

}  // namespace ar
