// Block-wide mixed-radix Stockham FFT held in LDS (gfx950), shared by the
// transform kernels: any length M with a stage per prime factor (compiled
// codelets for radices up to 31, generic O(R) stages otherwise), ping-pong
// buffers, and the launch helpers that size a workgroup's sequences.
#pragma once

#include "ar_codelets.h"
#include "ar_internal.h"

namespace ar {
namespace {

using namespace cl;

// ------------------------------------------------------------ FFT stages

// Element t of sequence s lives at buf[s * ss + t * es].
struct Layout {
  int nseq, ss, es;
  bool seq_fast;  // thread index -> (s fastest) or (t fastest)
};

template <typename T, int R>
__device__ __forceinline__ void stage_fixed(const V2<T> *__restrict__ src, V2<T> *__restrict__ dst,
                                            int M, int Ns, const V2<T> *__restrict__ tw,
                                            const Layout L) {
  const int nb = M / R;
  const int total = nb * L.nseq;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int s, j;
    if (L.seq_fast) {
      j = idx / L.nseq;
      s = idx - j * L.nseq;
    } else {
      s = idx / nb;
      j = idx - s * nb;
    }
    const V2<T> *a = src + s * L.ss;
    V2<T> *b = dst + s * L.ss;
    const int k = j % Ns;
    V2<T> v[R];
    static_for<R>([&](auto r) { v[r] = a[(j + r * nb) * L.es]; });
    if (Ns > 1) {
      const V2<T> *t = tw + k * R;
      static_for<R - 1>([&](auto r) { v[r + 1] = cmul(v[r + 1], t[r + 1]); });
    }
    dft<R, T>(v);
    const int base = (j - k) * R + k;
    static_for<R>([&](auto r) { b[(base + r * Ns) * L.es] = v[r]; });
  }
}

// Radix without a codelet: twiddle in place, then each output is an O(R)
// sum over the butterfly's inputs with the roots e^{-2 pi i t / R}.
template <typename T>
__device__ void stage_generic(V2<T> *__restrict__ src, V2<T> *__restrict__ dst, int M, int R,
                              int Ns, const V2<T> *__restrict__ tw,
                              const V2<T> *__restrict__ roots, const Layout L) {
  const int nb = M / R;
  const int total = M * L.nseq;
  if (Ns > 1) {
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int s, t;
      if (L.seq_fast) {
        t = idx / L.nseq;
        s = idx - t * L.nseq;
      } else {
        s = idx / M;
        t = idx - s * M;
      }
      const int r = t / nb, j = t - r * nb, k = j % Ns;
      if (r == 0) continue;
      V2<T> &e = src[s * L.ss + t * L.es];
      e = cmul(e, tw[k * R + r]);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int s, o;
    if (L.seq_fast) {
      o = idx / L.nseq;
      s = idx - o * L.nseq;
    } else {
      s = idx / M;
      o = idx - s * M;
    }
    const int ro = o / nb, j = o - ro * nb, k = j % Ns;
    const V2<T> *a = src + s * L.ss;
    V2<T> acc{T(0), T(0)};
    int e = 0;
    for (int r = 0; r < R; ++r) {
      const V2<T> x = a[(j + r * nb) * L.es];
      const V2<T> w = roots[e];
      acc.x = fma(x.x, w.x, fma(-x.y, w.y, acc.x));
      acc.y = fma(x.x, w.y, fma(x.y, w.x, acc.y));
      e += ro;
      if (e >= R) e -= R;
    }
    dst[s * L.ss + ((j - k) * R + k + ro * Ns) * L.es] = acc;
  }
}

// Runs all stages; returns the buffer holding the result.
template <typename T>
__device__ V2<T> *fft_run(V2<T> *A, V2<T> *B, const FftDesc &fd, const V2<T> *__restrict__ tw,
                          const V2<T> *__restrict__ gen, const Layout L) {
  const int M = fd.M;
  for (int st = 0; st < fd.nstages; ++st) {
    const int R = fd.radix[st], Ns = fd.ns[st];
    const V2<T> *t = tw + fd.tw_off[st];
    switch (R) {
      case 2: stage_fixed<T, 2>(A, B, M, Ns, t, L); break;
      case 3: stage_fixed<T, 3>(A, B, M, Ns, t, L); break;
      case 4: stage_fixed<T, 4>(A, B, M, Ns, t, L); break;
      case 5: stage_fixed<T, 5>(A, B, M, Ns, t, L); break;
      case 7: stage_fixed<T, 7>(A, B, M, Ns, t, L); break;
      case 11: stage_fixed<T, 11>(A, B, M, Ns, t, L); break;
      case 13: stage_fixed<T, 13>(A, B, M, Ns, t, L); break;
      case 17: stage_fixed<T, 17>(A, B, M, Ns, t, L); break;
      case 19: stage_fixed<T, 19>(A, B, M, Ns, t, L); break;
      case 23: stage_fixed<T, 23>(A, B, M, Ns, t, L); break;
      case 29: stage_fixed<T, 29>(A, B, M, Ns, t, L); break;
      case 31: stage_fixed<T, 31>(A, B, M, Ns, t, L); break;
      default: stage_generic<T>(A, B, M, R, Ns, t, gen + fd.gen_off[st], L); break;
    }
    __syncthreads();
    V2<T> *tmp = A;
    A = B;
    B = tmp;
  }
  return A;
}

FftDesc make_desc(const FftPlan &fp) {
  FftDesc d{};
  d.M = fp.M;
  d.nstages = fp.nstages;
  for (int s = 0; s < kMaxStages; ++s) {
    d.radix[s] = fp.radix[s];
    d.ns[s] = fp.ns[s];
    d.tw_off[s] = fp.tw_off[s];
    d.gen_off[s] = fp.gen_off[s];
  }
  return d;
}

// Rows (columns) per workgroup: enough sequences to give 256 threads work,
// within 63 KiB of LDS when possible; a single long sequence may use up to
// kMaxLds (gfx950 has 160 KiB of LDS per CU).
constexpr size_t kLdsSoft = 63 * 1024, kMaxLds = 150 * 1024;
int seqs_per_block(int M, size_t csize, int target) {
  const size_t cplx = 2 * csize;
  int B = target / (M > 0 ? M : 1);
  if (B < 1) B = 1;
  if (B > 64) B = 64;
  while (B > 1 && 2 * (size_t)B * M * cplx > kLdsSoft) --B;
  return B;
}
int rows_per_block(int M, size_t csize) { return seqs_per_block(M, csize, 2048); }
int cols_per_block(int M, size_t csize) { return seqs_per_block(M, csize, 2048); }

size_t seq_lds_bytes(int B, int M, size_t csize) {
  return 2 * (size_t)B * M * 2 * csize + 2 * (size_t)B * csize + 64;
}

// Raise the dynamic LDS limit of a kernel once when a launch needs more
// than the default 64 KiB.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace
}  // namespace ar
