// Length-1024 AR transform passes (gfx950).
//
// Rows or columns of length m = 1024: the DST-I of length m - 2 through
// one complex FFT of length M = 1023 = 31 * 11 * 3 on the packed odd
// extension u_t = z_{2t} + i z_{2t+1} (Theorem 1: endpoint scaling, ramp
// removal / restoration), the same mathematics as the general
// wave-per-sequence engine with every size fixed at compile time and G = 2
// or 4 wavefronts per sequence.  What differs:
//   * the odd extension z_0 .. z_{2M-1} of a sequence (ramp removed for a
//     forward pass) is staged in LDS in natural order, z_{2M-j} = -z_j
//     written together with z_j; the first (radix-31) stage reads its
//     inputs u_t from there as aligned pairs, so there is no digit-reversal
//     table and no scattered store;
//   * the twiddles of the radix-11 and radix-3 stages and the (cos, sin)
//     factors of the DST post-processing of a lane's outputs sit in
//     registers: one table value per kind is loaded and the others follow
//     by products with compile-time roots of unity (angle addition), so LDS
//     holds only the data and few loads are issued;
//   * rows and columns move as 4-element (rows) or W-column (column
//     blocks) vectors;
//   * the radix-31 output pairs are dealt to the G wavefronts of a
//     sequence (the radix-11 pairs to pairs of wavefronts when G = 4);
//   * the column pass stages its filtered coefficients as the odd extension
//     of the inverse transform's input directly;
//   * in FP64 arithmetic rows and columns may also run in pairs, two per
//     complex FFT of length M (rows1023p_kernel, cols1023p_kernel), which
//     halves the FFTs of a pass.
// Stages (radix, stride L, twiddle offset in the plan's table): (31, 1, 0),
// (11, 31, 30), (3, 341, 340); natural input index n = 33 d0 + 3 d1 + d2
// sits at position d0 + 31 d1 + 341 d2 of the in-place DIT order, so
// radix-31 butterfly j reads u_t for t = 33 r + 3 (j mod 11) + j / 11.
#include <type_traits>

#include "ar_codelets.h"
#include "ar_internal.h"

namespace ar {
namespace {

using namespace cl;

constexpr int kM = 1023;     // FFT length
constexpr int kLen = 1024;   // sequence length m
constexpr int kZ = 2 * kM;   // odd-extension length
constexpr int kWgMax = 512;  // threads per workgroup the kernels are built for

// Output pairs k = lo + 1 .. hi of part P of S (radix R).
template <int R, int S, int P> struct Pairs {
  static constexpr int H = (R - 1) / 2;
  static constexpr int lo = P * H / S, hi = (P + 1) * H / S;
};

// Per-lane constants: stage twiddles and post-processing factors.  The
// radix-11 twiddles e^{-2 pi i k r / 341} of butterfly j11 (k = j11 mod 31)
// for r = 1..5 are loaded and r = 6..10 formed as products; the radix-3
// twiddles e^{-2 pi i j / M} (and their squares) of butterflies
// j = s + 64 G c, and the factors (cos, sin)(pi k / M) of outputs
// k = 4 (s + 64 G c) + i, follow from one table value each and
// compile-time roots.
template <typename T, int G>
struct Regs {
  static constexpr int SL = 64 * G, NQ = 256 / SL, NK = 4 * NQ, C3 = (341 + SL - 1) / SL;
  V2<T> t11[10];
  V2<T> t3[C3][2];
  V2<T> cs[NK];
  __device__ __forceinline__ void load(const V2<T> *__restrict__ tw,
                                       const V2<T> *__restrict__ post, int j11, int s) {
    const int k11 = (j11 < 93 ? j11 : 0) % 31;
#pragma unroll
    for (int r = 0; r < 5; ++r) t11[r] = tw[30 + 31 * r + k11];
    const V2<T> w3 = tw[340 + s];  // e^{-2 pi i s / M}
    const V2<T> p4 = post[4 * s];  // e^{i pi 4 s / M}
#pragma unroll
    for (int r = 5; r < 10; ++r) t11[r] = cmul(t11[4], t11[r - 5]);
    static_for<C3>([&](auto Cc) {
      constexpr int c = decltype(Cc)::value;
      if constexpr (c == 0) {
        t3[c][0] = w3;
      } else {
        constexpr T fx = T(cos2pi(SL * c, kM)), fy = T(-sin2pi(SL * c, kM));
        t3[c][0] = cmul(w3, V2<T>{fx, fy});
      }
      t3[c][1] = cmul(t3[c][0], t3[c][0]);
    });
    static_for<NK>([&](auto Ic) {
      constexpr int idx = decltype(Ic)::value;
      constexpr int q = 4 * SL * (idx / 4) + idx % 4;
      if constexpr (q == 0) {
        cs[idx] = p4;
      } else {
        constexpr T ex = T(cos2pi(q, 2 * kM)), ey = T(sin2pi(q, 2 * kM));
        cs[idx] = cmul(p4, V2<T>{ex, ey});
      }
    });
  }
};

// N consecutive elements from / to global memory: one vector access when
// `vec` (the address is aligned to N elements), else N scalar ones.  The
// image pointers of a call decide `vec` for the whole grid, so the branch
// is uniform.
template <int N, typename T>
__device__ __forceinline__ void vload(T (&d)[N], const Gl<T> *p, bool vec) {
  if constexpr (N == 1) {
    d[0] = p[0];
  } else {
    typedef T V __attribute__((ext_vector_type(N)));
    if (vec) {
      const V v = *(const Gl<V> *)p;
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] = v[i];
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] = p[i];
    }
  }
}
template <int N, typename T>
__device__ __forceinline__ void vstore(Gl<T> *p, const T (&d)[N], bool vec) {
  if constexpr (N == 1) {
    p[0] = d[0];
  } else {
    typedef T V __attribute__((ext_vector_type(N)));
    if (vec) {
      V v;
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = d[i];
      *(Gl<V> *)p = v;
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) p[i] = d[i];
    }
  }
}
template <typename T>
__device__ __forceinline__ bool aligned_to(const void *p, int bytes) {
  return ((size_t)p & (size_t)(bytes - 1)) == 0;
}
// four consecutive LDS words at a 4-aligned index
template <typename T>
__device__ __forceinline__ void lstore4(T *p, const T (&d)[4]) {
  typedef T V __attribute__((ext_vector_type(4)));
  V v;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = d[i];
  *reinterpret_cast<V *>(p) = v;
}

// z_j of the odd extension from the raw value x_j, 0 <= j <= M (ramp
// removed if asked); zero at j = 0 and j = M
template <typename T>
__device__ __forceinline__ T zval(T x, int j, bool ramp, T e0, T e1) {
  const T invM = T(1) / T(kM);
  if (ramp) x -= e0 * (T(kM - j) * invM) + e1 * (T(j) * invM);
  return (j == 0 || j == kM) ? T(0) : x;
}

// Stage the odd extension value of index j (0 <= j <= M) of a sequence.
template <typename T>
__device__ __forceinline__ void zstore(T *Z, int j, T z) {
  Z[j] = z;
  if (j >= 1 && j <= kM - 1) Z[kZ - j] = -z;
}
// The same for j = j0 .. j0 + 3 (j0 a multiple of 4)
template <typename T>
__device__ __forceinline__ void zstore4(T *Z, int j0, const T (&z)[4]) {
  lstore4<T>(Z + j0, z);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (j0 + i >= 1 && j0 + i <= kM - 1) Z[kZ - j0 - i] = -z[i];
}

// Radix-31 stage (stride 1) from the staged odd extension: butterfly j
// (lane j < 33 of every wavefront of the sequence), output pairs of part g.
template <typename T, int G>
__device__ __forceinline__ void st31(V2<T> *U, const V2<T> *Zv, int g, int l64) {
  const bool ok = l64 < 33;
  const int j = ok ? l64 : 0;
  const int jp = 3 * (j % 11) + j / 11;
  V2<T> v[31];
  static_for<31>([&](auto r) { v[r] = Zv[jp + 33 * decltype(r)::value]; });
  V2<T> a[15], b[15];
  dft_odd_ab<31, T>(v, a, b);
  const V2<T> v0 = v[0];
  auto emit = [&](auto K, V2<T> x) {
    if (ok) U[31 * j + decltype(K)::value] = x;
  };
  static_for<G>([&](auto Pc) {
    constexpr int P = decltype(Pc)::value;
    if (g == P) {
      if constexpr (P == 0) dft_odd_zero<31, T>(v0, a, emit);
      dft_odd_pairs<31, Pairs<31, G, P>::lo, Pairs<31, G, P>::hi, T>(v0, a, b, emit);
    }
  });
}

// Radix-11 stage (stride 31), in place; butterfly j < 93 of this lane.  With
// G = 4 the output pairs are split over the two halves of the sequence's
// wavefronts, and a barrier separates all reads from the stores.
template <typename T, int G>
__device__ __forceinline__ void st11(V2<T> *U, const Regs<T, G> &R, int j, int part) {
  const bool ok = j < 93;
  const int jc = ok ? j : 0;
  const int grp = jc / 31, k = jc - 31 * grp;
  const int base = 341 * grp + k;
  V2<T> v[11];
  static_for<11>([&](auto r) { v[r] = U[base + 31 * decltype(r)::value]; });
  static_for<10>([&](auto r) {
    constexpr int q = decltype(r)::value;
    v[q + 1] = cmul(v[q + 1], R.t11[q]);
  });
  auto emit = [&](auto K, V2<T> x) {
    if (ok) U[base + 31 * decltype(K)::value] = x;
  };
  if constexpr (G == 4) {
    V2<T> a[5], b[5];
    dft_odd_ab<11, T>(v, a, b);
    const V2<T> v0 = v[0];
    __syncthreads();
    if (part == 0) {
      dft_odd_zero<11, T>(v0, a, emit);
      dft_odd_pairs<11, Pairs<11, 2, 0>::lo, Pairs<11, 2, 0>::hi, T>(v0, a, b, emit);
    } else {
      dft_odd_pairs<11, Pairs<11, 2, 1>::lo, Pairs<11, 2, 1>::hi, T>(v0, a, b, emit);
    }
  } else {
    dft_emit<11, T>(v, emit);
  }
}

// Radix-3 stage (stride 341), in place; butterflies s + 64 G c.
template <typename T, int G>
__device__ __forceinline__ void st3(V2<T> *U, const Regs<T, G> &R, int s) {
  constexpr int SL = 64 * G, C3 = Regs<T, G>::C3;
  V2<T> v[C3][3];
#pragma unroll
  for (int c = 0; c < C3; ++c) {
    const int j = s + SL * c;
    const int jc = j < 341 ? j : 0;
    v[c][0] = U[jc];
    v[c][1] = cmul(U[jc + 341], R.t3[c][0]);
    v[c][2] = cmul(U[jc + 682], R.t3[c][1]);
  }
#pragma unroll
  for (int c = 0; c < C3; ++c) {
    const int j = s + SL * c;
    if (j < 341)
      dft_emit<3, T>(v[c], [&](auto K, V2<T> x) { U[j + 341 * decltype(K)::value] = x; });
  }
}

// FP64 kernels load the per-lane constants after the radix-31 stage, whose
// 31 inputs and 30 pair sums would otherwise share the registers with them.
template <typename T>
constexpr bool kLateRegs = std::is_same<T, double>::value;

// The FFT of the staged sequence into U (natural order); ends at a barrier.
template <typename T, int G>
__device__ __forceinline__ void fft1023(V2<T> *U, const T *Z, Regs<T, G> &R,
                                        const V2<T> *__restrict__ tw,
                                        const V2<T> *__restrict__ post, int g, int l64, int s) {
  st31<T, G>(U, reinterpret_cast<const V2<T> *>(Z), g, l64);
  if constexpr (kLateRegs<T>) R.load(tw, post, G == 4 ? l64 + 64 * (g & 1) : s, s);
  __syncthreads();
  if constexpr (G == 4) st11<T, G>(U, R, l64 + 64 * (g & 1), g >> 1);
  else st11<T, G>(U, R, s, 0);
  __syncthreads();
  st3<T, G>(U, R, s);
  __syncthreads();
}

// Output k of a forward (INV = false) or inverse (INV = true) pass:
// endpoints from e0 / e1, interior from U_k and U_{M-k} (plus the ramp for
// the inverse).
template <typename T, bool INV>
__device__ __forceinline__ T coef(const V2<T> *U, int k, V2<T> cs, T scale, T alpha, T e0, T e1) {
  const int kc = k < 1 ? 1 : (k > kM - 1 ? kM - 1 : k);
  const V2<T> A = U[kc], C = U[kM - kc];
  const T d = scale * ((C.y - A.y) + cs.x * (A.x - C.x) + cs.y * (A.y + C.y));
  if (!INV) return k == 0 ? alpha * e0 : (k == kM ? alpha * e1 : d);
  const T invM = T(1) / T(kM);
  const T y0 = e0 / alpha, y1 = e1 / alpha;
  const T in = d + y0 * (T(kM - k) * invM) + y1 * (T(k) * invM);
  return k == 0 ? y0 : (k == kM ? y1 : in);
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
  return t;
}

// LDS of one sequence: U (1024 complex), then the staged odd extension with
// a row pitch that spreads the W sequences of a block over the banks.
__host__ __device__ inline int zpitch(int W) { return 2048 + 64 / W; }
// bytes of U and the staging rows of W sequences (or pairs)
__host__ __device__ inline size_t x1023_lds_dev(int W, size_t csize) {
  return (size_t)W * (1024 * 2 * csize + (size_t)zpitch(W) * csize);
}

template <typename T>
struct Lds {
  V2<T> *U;
  T *Z;
  __device__ Lds(unsigned char *raw, int W, int seq) {
    U = reinterpret_cast<V2<T> *>(raw) + (size_t)seq * 1024;
    Z = reinterpret_cast<T *>(raw + (size_t)W * 1024 * sizeof(V2<T>)) + (size_t)seq * zpitch(W);
  }
};

// ---------------------------------------------------------------- rows

// Elements of a row are dealt to the 64 G threads of its sequence in groups
// of four: thread s holds k = 4 (s + 64 G c) + i.
template <typename TS, typename T, int MODE, int G>
__global__ __launch_bounds__(kWgMax) void rows1023_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, const V2<T> *__restrict__ tw,
    const V2<T> *__restrict__ post, T alpha, T scale, T tau, const TS *__restrict__ f_true,
    double *__restrict__ partial, const XJob *__restrict__ jobs, int kit) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (jobs) {  // batched launch: problem blockIdx.y
    const XJob J = jobs[blockIdx.y];
    in = static_cast<const TS *>(J.in);
    out = static_cast<TS *>(J.out);
    f_true = static_cast<const TS *>(J.aux);
    partial = J.part ? J.part + (size_t)kit * J.nblk : nullptr;
  }
  constexpr int SL = 64 * G, NQ = 256 / SL;
  const int W = (blockDim.x >> 6) / G;
  const int wv = threadIdx.x >> 6;
  const int seq = wv / G;
  const int g = __builtin_amdgcn_readfirstlane(wv % G);  // wavefront within the sequence
  const int l64 = threadIdx.x & 63;
  const int s = 64 * g + l64;                             // thread within the sequence
  const int row = xcd_remap(blockIdx.x, gridDim.x) * W + seq;
  const bool active = row < n1;
  const Lds<T> L(smem_raw, W, seq);
  const Gl<TS> *src = gmem(in) + (size_t)(active ? row : 0) * kLen;
  Gl<TS> *dst = gmem(out) + (size_t)(active ? row : 0) * kLen;
  const Gl<TS> *fr = f_true ? gmem(f_true) + (size_t)(active ? row : 0) * kLen : nullptr;
  // every global load first: the row, its endpoints, x and f (update), the
  // lane's constants
  constexpr int VB = 4 * sizeof(TS);
  const bool va_in = aligned_to<TS>(in, VB);
  const bool va_out = aligned_to<TS>(out, VB) && (!f_true || aligned_to<TS>(f_true, VB));
  TS xv[NQ][4], xo[NQ][4], fo[NQ][4];
#pragma unroll
  for (int c = 0; c < NQ; ++c) vload<4>(xv[c], src + 4 * (s + SL * c), va_in);
  const T e0 = T(src[0]), e1 = T(src[kLen - 1]);
  if (MODE == ROW_INV_UPDATE) {
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      vload<4>(xo[c], dst + 4 * (s + SL * c), va_out);
      if (fr) vload<4>(fo[c], fr + 4 * (s + SL * c), va_out);
    }
  }
  Regs<T, G> R;
  if constexpr (!kLateRegs<T>) R.load(tw, post, G == 4 ? l64 + 64 * (g & 1) : s, s);
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int j0 = 4 * (s + SL * c);
    T z[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = zval<T>(T(xv[c][i]), j0 + i, MODE == ROW_FWD, e0, e1);
    zstore4<T>(L.Z, j0, z);
  }
  __syncthreads();
  fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
  double ss = 0.0;
  TS o[NQ][4];
#pragma unroll
  for (int c = 0; c < NQ; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T v = coef<T, MODE != ROW_FWD>(L.U, 4 * (s + SL * c) + i, R.cs[4 * c + i], scale,
                                           alpha, e0, e1);
      if (MODE == ROW_INV_UPDATE) {
        o[c][i] = TS(T(xo[c][i]) + tau * v);
        if (fr) {
          const double df = (double)o[c][i] - (double)fo[c][i];
          ss += df * df;
        }
      } else {
        o[c][i] = TS(v);
      }
    }
  if (active) {
#pragma unroll
    for (int c = 0; c < NQ; ++c) vstore<4>(dst + 4 * (s + SL * c), o[c], va_out);
  } else {
    ss = 0.0;
  }
  if (MODE == ROW_INV_UPDATE && partial) {
    double *red = reinterpret_cast<double *>(smem_raw);
    const double t = block_sum(ss, red);
    if (threadIdx.x == 0) gmem(partial)[blockIdx.x] = t;
  }
}

// ------------------------------------------------------------- columns

// Block I/O: the W columns of a workgroup move as W-element vectors, one
// per row, thread t serving rows t + 64 G W i (one batch covers the 1024
// rows).  Filter values and outputs of a column are dealt like a row's
// elements (k = 4 (s + 64 G c) + i).
template <typename TS, typename T, int MODE, int G, int W>
__global__ __launch_bounds__(kWgMax) void cols1023_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n2, const V2<T> *__restrict__ tw,
    const V2<T> *__restrict__ post, T alpha, T scale, const TS *__restrict__ dT,
    const XJob *__restrict__ jobs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (jobs) {  // batched launch: problem blockIdx.y
    const XJob J = jobs[blockIdx.y];
    in = static_cast<const TS *>(J.in);
    out = static_cast<TS *>(J.out);
    dT = static_cast<const TS *>(J.aux);
  }
  constexpr int SL = 64 * G, NQ = 256 / SL, BT = 64 * G * W, NR = kLen / BT;
  const int wv = threadIdx.x >> 6;
  const int seq = wv / G;
  const int g = __builtin_amdgcn_readfirstlane(wv % G);
  const int l64 = threadIdx.x & 63;
  const int s = 64 * g + l64;
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * W;
  const int col = col0 + seq;
  const bool active = col < n2;
  const long ld = n2;
  const Lds<T> L(smem_raw, W, seq);
  // the block's rows (W columns each), its first and last rows (ramps)
  const int t = threadIdx.x;
  const Gl<TS> *blk = gmem(in) + col0;
  const bool va_in = aligned_to<TS>(in, W * sizeof(TS));
  const bool va_out = aligned_to<TS>(out, W * sizeof(TS));
  const bool va_d = aligned_to<TS>(dT, 4 * sizeof(TS));
  TS bv[NR][W], b0[W], b1[W];
#pragma unroll
  for (int i = 0; i < NR; ++i) vload<W>(bv[i], blk + (long)(t + BT * i) * ld, va_in);
  vload<W>(b0, blk, va_in);
  vload<W>(b1, blk + (long)(kLen - 1) * ld, va_in);
  TS dv[NQ][4];
  if (MODE == COL_FWD_D_INV) {
    const Gl<TS> *dcol = gmem(dT) + (size_t)(active ? col : 0) * kLen;
#pragma unroll
    for (int c = 0; c < NQ; ++c) vload<4>(dv[c], dcol + 4 * (s + SL * c), va_d);
  }
  Regs<T, G> R;
  if constexpr (!kLateRegs<T>) R.load(tw, post, G == 4 ? l64 + 64 * (g & 1) : s, s);
  T e0 = T(0), e1 = T(0);
#pragma unroll
  for (int c = 0; c < W; ++c)
    if (seq == c) {
      e0 = T(b0[c]);
      e1 = T(b1[c]);
    }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    T *Zc = Lds<T>(smem_raw, W, c).Z;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int r = t + BT * i;
      zstore<T>(Zc, r, zval<T>(T(bv[i][c]), r, MODE != COL_INV, T(b0[c]), T(b1[c])));
    }
  }
  __syncthreads();
  fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
  if constexpr (MODE == COL_FWD_D_INV) {
    // d_k (T~ y)_k, staged as the odd extension of the inverse pass's input;
    // its endpoints go to the two spare words past the extension
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      const int k0 = 4 * (s + SL * c);
      T z[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + i;
        const T cf = T(dv[c][i]) * coef<T, false>(L.U, k, R.cs[4 * c + i], scale, alpha, e0, e1);
        z[i] = (k == 0 || k == kM) ? T(0) : cf;
        if (k == 0) L.Z[kZ] = cf;
        if (k == kM) L.Z[kZ + 1] = cf;
      }
      zstore4<T>(L.Z, k0, z);
    }
    __syncthreads();
    e0 = L.Z[kZ];
    e1 = L.Z[kZ + 1];
    fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
  }
  // outputs in natural order over the staging row, then row by row
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int k0 = 4 * (s + SL * c);
    T o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      o[i] = coef<T, MODE != COL_FWD>(L.U, k0 + i, R.cs[4 * c + i], scale, alpha, e0, e1);
    lstore4<T>(L.Z + k0, o);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int r = t + BT * i;
    TS v[W];
#pragma unroll
    for (int c = 0; c < W; ++c) v[c] = TS(Lds<T>(smem_raw, W, c).Z[r]);
    vstore<W>(gmem(out) + col0 + (long)r * ld, v, va_out);
  }
}

// ------------------------------------------------------- rows in pairs

// Two rows a, b of a workgroup share one complex FFT of length n = M.  With
// f the interior of a row (f_0 = f_n = 0) its DST-I X_k = sum_j f_j
// sin(pi j k / n) follows from the length-n DFT Y of
//   y_j = sin(pi j / n) (f_j + f_{n-j}) + (f_j - f_{n-j}) / 2:
// X_{2k} = -Im Y_k, and X_{2k+1} - X_{2k-1} = Re Y_k (X_{-1} = -X_1), so
// the odd outputs are a running sum over k.  The rows ride as the real and
// imaginary parts of w_j = y^a_j + i y^b_j; with W = DFT(w), Y^a_k =
// (W_k + conj W_{n-k}) / 2 and Y^b_k = (W_k - conj W_{n-k}) / (2i).  Half
// the FFTs of the one-row-per-FFT form, no odd extension, and no
// post-processing factors.
//
// sin(pi j / M) for j = j0 .. j0 + 3 from the table value at j0
template <typename T>
__device__ __forceinline__ void sines4(const V2<T> *__restrict__ post, int j0, T (&sv)[4]) {
  const V2<T> p = post[j0];
  sv[0] = p.y;
  static_for<3>([&](auto Ic) {
    constexpr int i = decltype(Ic)::value + 1;
    constexpr T cx = T(cos2pi(i, 2 * kM)), sx = T(sin2pi(i, 2 * kM));
    sv[i] = p.y * cx + p.x * sx;
  });
}

// Inclusive running sum over the SL threads of a pair, in thread order, of
// two values at once; `slot` is G V2 words of LDS for this call alone (a
// second call takes other words, so no barrier separates the two).  Returns
// the thread's inclusive sum and leaves the pair's total in `tot`.
template <typename T, int G>
__device__ __forceinline__ V2<T> pair_scan(V2<T> v, V2<T> *slot, int g, int l64, V2<T> &tot) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T ua = __shfl_up(v.x, off, 64), ub = __shfl_up(v.y, off, 64);
    if (l64 >= off) {
      v.x += ua;
      v.y += ub;
    }
  }
  if (l64 == 63) slot[g] = v;
  __syncthreads();
  V2<T> lo{T(0), T(0)};
  tot = V2<T>{T(0), T(0)};
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const V2<T> t = slot[q];
    if (q < g) {
      lo.x += t.x;
      lo.y += t.y;
    }
    tot.x += t.x;
    tot.y += t.y;
  }
  return V2<T>{v.x + lo.x, v.y + lo.y};
}

template <typename TS, typename T, int MODE, int G>
__global__ __launch_bounds__(kWgMax) void rows1023p_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n1, const V2<T> *__restrict__ tw,
    const V2<T> *__restrict__ post, T alpha, T scale, T tau, const TS *__restrict__ f_true,
    double *__restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int SL = 64 * G, NQ = 256 / SL;
  const int P = (blockDim.x >> 6) / G;  // pairs per workgroup
  const int wv = threadIdx.x >> 6;
  const int pr = wv / G;
  const int g = __builtin_amdgcn_readfirstlane(wv % G);
  const int l64 = threadIdx.x & 63;
  const int s = 64 * g + l64;
  const int ra = xcd_remap(blockIdx.x, gridDim.x) * 2 * P + 2 * pr;
  const bool act_a = ra < n1, act_b = ra + 1 < n1;
  const Lds<T> L(smem_raw, P, pr);
  V2<T> *Wv = reinterpret_cast<V2<T> *>(L.Z);
  V2<T> *slots = reinterpret_cast<V2<T> *>(smem_raw + x1023_lds_dev(P, sizeof(T))) + NQ * G * pr;
  const int rowa = act_a ? ra : 0, rowb = act_b ? ra + 1 : rowa;
  const Gl<TS> *sa = gmem(in) + (size_t)rowa * kLen;
  const Gl<TS> *sb = gmem(in) + (size_t)rowb * kLen;
  constexpr int VB = 4 * sizeof(TS);
  const bool va_in = aligned_to<TS>(in, VB);
  const bool va_out = aligned_to<TS>(out, VB) && (!f_true || aligned_to<TS>(f_true, VB));
  TS xa[NQ][4], xb[NQ][4], ma[NQ][4], mb[NQ][4], oa[NQ][4], ob[NQ][4], fa[NQ][4], fb[NQ][4];
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int q = s + SL * c;
    vload<4>(xa[c], sa + 4 * q, va_in);
    vload<4>(xb[c], sb + 4 * q, va_in);
    vload<4>(ma[c], sa + (kLen - 4) - 4 * q, va_in);
    vload<4>(mb[c], sb + (kLen - 4) - 4 * q, va_in);
  }
  const T e0a = T(sa[0]), e1a = T(sa[kLen - 1]), e0b = T(sb[0]), e1b = T(sb[kLen - 1]);
  Gl<TS> *da = gmem(out) + (size_t)rowa * kLen;
  Gl<TS> *db = gmem(out) + (size_t)rowb * kLen;
  if (MODE == ROW_INV_UPDATE) {
    const Gl<TS> *fra = f_true ? gmem(f_true) + (size_t)rowa * kLen : nullptr;
    const Gl<TS> *frb = f_true ? gmem(f_true) + (size_t)rowb * kLen : nullptr;
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      const int q = s + SL * c;
      vload<4>(oa[c], da + 4 * q, va_out);
      vload<4>(ob[c], db + 4 * q, va_out);
      if (f_true) {
        vload<4>(fa[c], fra + 4 * q, va_out);
        vload<4>(fb[c], frb + 4 * q, va_out);
      }
    }
  }
  Regs<T, G> R;
  if constexpr (!kLateRegs<T>) R.load(tw, post, G == 4 ? l64 + 64 * (g & 1) : s, s);
  // w_j = y^a_j + i y^b_j for the lane's j = 4 q + i (j = M is no input)
  constexpr bool ramp = MODE == ROW_FWD;
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int j0 = 4 * (s + SL * c);
    T sv[4];
    sines4<T>(post, j0, sv);
    V2<T> w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = j0 + i;
      const T fja = zval<T>(T(xa[c][i]), j, ramp, e0a, e1a);
      const T fna = zval<T>(T(ma[c][3 - i]), kM - j, ramp, e0a, e1a);
      const T fjb = zval<T>(T(xb[c][i]), j, ramp, e0b, e1b);
      const T fnb = zval<T>(T(mb[c][3 - i]), kM - j, ramp, e0b, e1b);
      w[i].x = sv[i] * (fja + fna) + T(0.5) * (fja - fna);
      w[i].y = sv[i] * (fjb + fnb) + T(0.5) * (fjb - fnb);
    }
    if (j0 + 3 < kM) {
      T *wp = reinterpret_cast<T *>(Wv + j0);
      lstore4<T>(wp, {w[0].x, w[0].y, w[1].x, w[1].y});
      lstore4<T>(wp + 4, {w[2].x, w[2].y, w[3].x, w[3].y});
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) Wv[j0 + i] = w[i];
    }
  }
  __syncthreads();
  fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
  // outputs k = 4 q + i of both rows: k = 2 kappa from W_kappa and
  // W_{M-kappa} directly, k = 2 kappa + 1 from the running sum of
  // t_kappa = (Re W_kappa + Re W_{M-kappa}, Im W_kappa + Im W_{M-kappa})
  // (halved at kappa = 0).  The sum over all kappa <= 511 is X_M = 0
  // exactly; its computed value is rounding accumulated along the sum, and
  // is removed in proportion to the terms taken (a linear bridge), so the
  // accumulated error is pinned at both ends of the sum.
  const T ps = T(2) * scale;
  const T invM = T(1) / T(kM);
  V2<T> A0[NQ], A1[NQ], C0[NQ], C1[NQ], t0[NQ], t01[NQ], ex[NQ];
  V2<T> carry{T(0), T(0)};
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int q = s + SL * c;
    const int k0 = 2 * q, k1 = 2 * q + 1;
    A0[c] = L.U[k0];
    A1[c] = L.U[k1];
    C0[c] = L.U[k0 == 0 ? 0 : kM - k0];
    C1[c] = L.U[kM - k1];
    const T h0 = k0 == 0 ? T(0.5) : T(1);
    t0[c] = V2<T>{h0 * (A0[c].x + C0[c].x), h0 * (A0[c].y + C0[c].y)};
    t01[c] = V2<T>{t0[c].x + (A1[c].x + C1[c].x), t0[c].y + (A1[c].y + C1[c].y)};
    V2<T> tot;
    const V2<T> inc = pair_scan<T, G>(t01[c], slots + G * c, g, l64, tot);
    ex[c] = V2<T>{carry.x + inc.x - t01[c].x, carry.y + inc.y - t01[c].y};
    carry.x += tot.x;
    carry.y += tot.y;
  }
  double ss = 0.0;
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int q = s + SL * c;
    const T f0 = (T(2 * q) + T(0.5)) * T(1.0 / 512), f1 = (T(2 * q + 1) + T(0.5)) * T(1.0 / 512);
    // DST values (times 4 scale) of k = 4q .. 4q + 3, rows a (x) and b (y)
    V2<T> dv[4];
    dv[0] = V2<T>{ps * (C0[c].y - A0[c].y), ps * (A0[c].x - C0[c].x)};
    dv[1] = V2<T>{ps * (ex[c].x + t0[c].x - f0 * carry.x), ps * (ex[c].y + t0[c].y - f0 * carry.y)};
    dv[2] = V2<T>{ps * (C1[c].y - A1[c].y), ps * (A1[c].x - C1[c].x)};
    dv[3] = V2<T>{ps * (ex[c].x + t01[c].x - f1 * carry.x), ps * (ex[c].y + t01[c].y - f1 * carry.y)};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * q + i;
      T va, vb;
      if (MODE == ROW_FWD) {
        va = k == 0 ? alpha * e0a : (k == kM ? alpha * e1a : dv[i].x);
        vb = k == 0 ? alpha * e0b : (k == kM ? alpha * e1b : dv[i].y);
      } else {
        const T y0a = e0a / alpha, y1a = e1a / alpha, y0b = e0b / alpha, y1b = e1b / alpha;
        const T wl = T(kM - k) * invM, wr = T(k) * invM;
        va = k == 0 ? y0a : (k == kM ? y1a : dv[i].x + y0a * wl + y1a * wr);
        vb = k == 0 ? y0b : (k == kM ? y1b : dv[i].y + y0b * wl + y1b * wr);
      }
      if (MODE == ROW_INV_UPDATE) {
        oa[c][i] = TS(T(oa[c][i]) + tau * va);
        ob[c][i] = TS(T(ob[c][i]) + tau * vb);
        if (f_true) {
          const double dfa = (double)oa[c][i] - (double)fa[c][i];
          const double dfb = (double)ob[c][i] - (double)fb[c][i];
          ss += (act_a ? dfa * dfa : 0.0) + (act_b ? dfb * dfb : 0.0);
        }
      } else {
        oa[c][i] = TS(va);
        ob[c][i] = TS(vb);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const int q = s + SL * c;
    if (act_a) vstore<4>(da + 4 * q, oa[c], va_out);
    if (act_b) vstore<4>(db + 4 * q, ob[c], va_out);
  }
  if (MODE == ROW_INV_UPDATE && partial) {
    double *red = reinterpret_cast<double *>(smem_raw);
    const double t = block_sum(ss, red);
    if (threadIdx.x == 0) gmem(partial)[blockIdx.x] = t;
  }
}

// Post-processing of a paired FFT in U: the DST values (times 4 scale) of
// outputs k = 4 q + i, i = 0..3, of both sequences (x: a, y: b), from the
// even outputs directly and the odd ones by the bridged running sum, for the
// pair's threads s (q = s).  `slot` holds G V2 words for this call.
template <typename T, int G>
__device__ __forceinline__ void pair_dst4(const V2<T> *U, int q, T ps, V2<T> *slot, int g, int l64,
                                          V2<T> (&dv)[4]) {
  const int k0 = 2 * q, k1 = 2 * q + 1;
  const V2<T> A0 = U[k0], A1 = U[k1];
  const V2<T> C0 = U[k0 == 0 ? 0 : kM - k0], C1 = U[kM - k1];
  const T h0 = k0 == 0 ? T(0.5) : T(1);
  const V2<T> t0{h0 * (A0.x + C0.x), h0 * (A0.y + C0.y)};
  const V2<T> t01{t0.x + (A1.x + C1.x), t0.y + (A1.y + C1.y)};
  V2<T> tot;
  const V2<T> inc = pair_scan<T, G>(t01, slot, g, l64, tot);
  const V2<T> ex{inc.x - t01.x, inc.y - t01.y};
  const T f0 = (T(k0) + T(0.5)) * T(1.0 / 512), f1 = (T(k1) + T(0.5)) * T(1.0 / 512);
  dv[0] = V2<T>{ps * (C0.y - A0.y), ps * (A0.x - C0.x)};
  dv[1] = V2<T>{ps * (ex.x + t0.x - f0 * tot.x), ps * (ex.y + t0.y - f0 * tot.y)};
  dv[2] = V2<T>{ps * (C1.y - A1.y), ps * (A1.x - C1.x)};
  dv[3] = V2<T>{ps * (ex.x + t01.x - f1 * tot.x), ps * (ex.y + t01.y - f1 * tot.y)};
}

// w_j = y^a_j + i y^b_j (the pre-weighting above) of the chunk j0 .. j0 + 3
// from two staged sequences Fa, Fb (1024 values each, zero at both ends),
// to the FFT input Wv
template <typename T>
__device__ __forceinline__ void pair_stage4(const T *Fa, const T *Fb, const V2<T> *post, int j0,
                                            V2<T> *Wv) {
  T sv[4];
  sines4<T>(post, j0, sv);
  V2<T> w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = j0 + i;
    const T fja = Fa[j], fna = Fa[kM - j], fjb = Fb[j], fnb = Fb[kM - j];
    w[i].x = sv[i] * (fja + fna) + T(0.5) * (fja - fna);
    w[i].y = sv[i] * (fjb + fnb) + T(0.5) * (fjb - fnb);
  }
  if (j0 + 3 < kM) {
    T *wp = reinterpret_cast<T *>(Wv + j0);
    lstore4<T>(wp, {w[0].x, w[0].y, w[1].x, w[1].y});
    lstore4<T>(wp + 4, {w[2].x, w[2].y, w[3].x, w[3].y});
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) Wv[j0 + i] = w[i];
  }
}

// Column pass in pairs: the W columns of a workgroup (W even) as W / 2
// pairs of adjacent columns, each pair one complex FFT per transform on G
// wavefronts; block I/O of W-column rows as in cols1023_kernel.  LDS per
// pair: U, whose first 2 x 1024 words also hold the two staged columns
// before the FFT, and the staging region Z (FFT input, then the filtered
// coefficients, then the outputs).
template <typename TS, typename T, int MODE, int G, int W>
__global__ __launch_bounds__(kWgMax) void cols1023p_kernel(
    const TS *__restrict__ in, TS *__restrict__ out, int n2, const V2<T> *__restrict__ tw,
    const V2<T> *__restrict__ post, T alpha, T scale, const TS *__restrict__ dT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int P = W / 2, BT = 64 * G * P, NR = kLen / BT;
  static_assert(W % 2 == 0 && G == 4, "pairs of columns on four wavefronts");
  const int wv = threadIdx.x >> 6;
  const int pr = wv / G;
  const int g = __builtin_amdgcn_readfirstlane(wv % G);
  const int l64 = threadIdx.x & 63;
  const int s = 64 * g + l64;  // thread within the pair; chunk q = s
  const int col0 = xcd_remap(blockIdx.x, gridDim.x) * W;
  const long ld = n2;
  const Lds<T> L(smem_raw, P, pr);
  V2<T> *slots = reinterpret_cast<V2<T> *>(smem_raw + x1023_lds_dev(P, sizeof(T))) + 2 * G * pr;
  const int t = threadIdx.x;
  const Gl<TS> *blk = gmem(in) + col0;
  const bool va_in = aligned_to<TS>(in, W * sizeof(TS));
  const bool va_out = aligned_to<TS>(out, W * sizeof(TS));
  const bool va_d = aligned_to<TS>(dT, 4 * sizeof(TS));
  TS bv[NR][W], b0[W], b1[W];
#pragma unroll
  for (int i = 0; i < NR; ++i) vload<W>(bv[i], blk + (long)(t + BT * i) * ld, va_in);
  vload<W>(b0, blk, va_in);
  vload<W>(b1, blk + (long)(kLen - 1) * ld, va_in);
  const int ca = col0 + 2 * pr;  // the pair's columns ca, ca + 1 (n2 % W == 0)
  TS da4[4], db4[4];
  if (MODE == COL_FWD_D_INV) {
    vload<4>(da4, gmem(dT) + (size_t)ca * kLen + 4 * s, va_d);
    vload<4>(db4, gmem(dT) + (size_t)(ca + 1) * kLen + 4 * s, va_d);
  }
  Regs<T, G> R;
  if constexpr (!kLateRegs<T>) R.load(tw, post, G == 4 ? l64 + 64 * (g & 1) : s, s);
  T e0a = T(0), e1a = T(0), e0b = T(0), e1b = T(0);
#pragma unroll
  for (int c = 0; c < W; c += 2)
    if (2 * pr == c) {
      e0a = T(b0[c]);
      e1a = T(b1[c]);
      e0b = T(b0[c + 1]);
      e1b = T(b1[c + 1]);
    }
  // the block's columns, ramp removed for forward passes, to the U region
  // of their pair (column 2p at word 0, column 2p + 1 at word 1024)
#pragma unroll
  for (int c = 0; c < W; ++c) {
    T *Fc = reinterpret_cast<T *>(Lds<T>(smem_raw, P, c / 2).U) + (c & 1) * kLen;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int r = t + BT * i;
      Fc[r] = zval<T>(T(bv[i][c]), r, MODE != COL_INV, T(b0[c]), T(b1[c]));
    }
  }
  __syncthreads();
  V2<T> *Wv = reinterpret_cast<V2<T> *>(L.Z);
  {
    const T *F = reinterpret_cast<const T *>(L.U);
    pair_stage4<T>(F, F + kLen, post, 4 * s, Wv);
  }
  __syncthreads();
  fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
  const T ps = T(2) * scale;
  const T invM = T(1) / T(kM);
  V2<T> dv[4];
  pair_dst4<T, G>(L.U, s, ps, slots, g, l64, dv);
  T oa[4], ob[4];
  if constexpr (MODE == COL_FWD_D_INV) {
    // filtered coefficients d_k (T~ y)_k of both columns to Z, then the
    // inverse transform's input from them (endpoints through the words at
    // k = 0 and k = M)
    T *Fa = L.Z, *Fb = L.Z + kLen;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * s + i;
      const T xa = k == 0 ? alpha * e0a : (k == kM ? alpha * e1a : dv[i].x);
      const T xb = k == 0 ? alpha * e0b : (k == kM ? alpha * e1b : dv[i].y);
      oa[i] = T(da4[i]) * xa;
      ob[i] = T(db4[i]) * xb;
    }
    lstore4<T>(Fa + 4 * s, oa);
    lstore4<T>(Fb + 4 * s, ob);
    __syncthreads();
    e0a = Fa[0];
    e1a = Fa[kM];
    e0b = Fb[0];
    e1b = Fb[kM];
    T ga[4], gb[4], gma[4], gmb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = 4 * s + i;
      ga[i] = (j == 0 || j == kM) ? T(0) : Fa[j];
      gb[i] = (j == 0 || j == kM) ? T(0) : Fb[j];
      gma[i] = (j == 0 || j == kM) ? T(0) : Fa[kM - j];
      gmb[i] = (j == 0 || j == kM) ? T(0) : Fb[kM - j];
    }
    __syncthreads();
    {
      T sv[4];
      sines4<T>(post, 4 * s, sv);
      V2<T> w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w[i].x = sv[i] * (ga[i] + gma[i]) + T(0.5) * (ga[i] - gma[i]);
        w[i].y = sv[i] * (gb[i] + gmb[i]) + T(0.5) * (gb[i] - gmb[i]);
      }
      const int j0 = 4 * s;
      if (j0 + 3 < kM) {
        T *wp = reinterpret_cast<T *>(Wv + j0);
        lstore4<T>(wp, {w[0].x, w[0].y, w[1].x, w[1].y});
        lstore4<T>(wp + 4, {w[2].x, w[2].y, w[3].x, w[3].y});
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) Wv[j0 + i] = w[i];
      }
    }
    __syncthreads();
    fft1023<T, G>(L.U, L.Z, R, tw, post, g, l64, s);
    pair_dst4<T, G>(L.U, s, ps, slots + G, g, l64, dv);
  }
  // outputs of both columns in natural order to Z, then row by row
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 4 * s + i;
    if (MODE == COL_FWD) {
      oa[i] = k == 0 ? alpha * e0a : (k == kM ? alpha * e1a : dv[i].x);
      ob[i] = k == 0 ? alpha * e0b : (k == kM ? alpha * e1b : dv[i].y);
    } else {
      const T y0a = e0a / alpha, y1a = e1a / alpha, y0b = e0b / alpha, y1b = e1b / alpha;
      const T wl = T(kM - k) * invM, wr = T(k) * invM;
      oa[i] = k == 0 ? y0a : (k == kM ? y1a : dv[i].x + y0a * wl + y1a * wr);
      ob[i] = k == 0 ? y0b : (k == kM ? y1b : dv[i].y + y0b * wl + y1b * wr);
    }
  }
  lstore4<T>(L.Z + 4 * s, oa);
  lstore4<T>(L.Z + kLen + 4 * s, ob);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int r = t + BT * i;
    TS v[W];
#pragma unroll
    for (int c = 0; c < W; ++c) v[c] = TS(Lds<T>(smem_raw, P, c / 2).Z[(c & 1) * kLen + r]);
    vstore<W>(gmem(out) + col0 + (long)r * ld, v, va_out);
  }
}

template <typename TS, typename T, int W>
int colsp_t(const void *in, void *out, int n2, size_t smem, int mode, const void *tw,
            const void *post, double alpha, double scale, const void *dT, hipStream_t st) {
  const dim3 grid(n2 / W), block(64 * 4 * (W / 2));
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const TS *>(dT);
  auto ttw = static_cast<const V2<T> *>(tw);
  auto tp = static_cast<const V2<T> *>(post);
  hipError_t e = hipSuccess;
#define AR_X(MODE)                                                                              \
  e = smem > 64 * 1024                                                                          \
          ? hipFuncSetAttribute(                                                                \
                reinterpret_cast<const void *>(cols1023p_kernel<TS, T, MODE, 4, W>),            \
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)                          \
          : hipSuccess;                                                                         \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((cols1023p_kernel<TS, T, MODE, 4, W>), grid, block, smem, st, ti, to,    \
                       n2, ttw, tp, T(alpha), T(scale), td);                                    \
    e = hipGetLastError();                                                                      \
  }
  switch (mode) {
    case COL_FWD: AR_X(COL_FWD) break;
    case COL_INV: AR_X(COL_INV) break;
    default: AR_X(COL_FWD_D_INV) break;
  }
#undef AR_X
  return e == hipSuccess ? AR_OK : hip_fail(e, "cols1023p_kernel launch");
}

template <typename TS, typename T, int G>
int rowsp_t(const void *in, void *out, int n1, int P, size_t smem, int mode, const void *tw,
            const void *post, double alpha, double scale, double tau, const void *f_true,
            double *partial, hipStream_t st) {
  const dim3 grid((n1 + 2 * P - 1) / (2 * P)), block(64 * G * P);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  auto ttw = static_cast<const V2<T> *>(tw);
  auto tp = static_cast<const V2<T> *>(post);
  hipError_t e = hipSuccess;
#define AR_X(MODE)                                                                              \
  e = smem > 64 * 1024 ? hipFuncSetAttribute(                                                   \
                             reinterpret_cast<const void *>(rows1023p_kernel<TS, T, MODE, G>), \
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)            \
                       : hipSuccess;                                                            \
  if (e == hipSuccess) {                                                                        \
    hipLaunchKernelGGL((rows1023p_kernel<TS, T, MODE, G>), grid, block, smem, st, ti, to, n1,   \
                       ttw, tp, T(alpha), T(scale), T(tau), tf, partial);                       \
    e = hipGetLastError();                                                                      \
  }
  switch (mode) {
    case ROW_FWD: AR_X(ROW_FWD) break;
    case ROW_INV: AR_X(ROW_INV) break;
    default: AR_X(ROW_INV_UPDATE) break;
  }
#undef AR_X
  return e == hipSuccess ? AR_OK : hip_fail(e, "rows1023p_kernel launch");
}

template <typename TS, typename T, int G>
int rows_t(const void *in, void *out, int n1, int W, int blocks, size_t smem, int mode,
           const void *tw, const void *post, double alpha, double scale, double tau,
           const void *f_true, double *partial, const XJob *jobs, int count, int kit,
           hipStream_t st) {
  const dim3 grid(blocks, count), block(64 * G * W);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto tf = static_cast<const TS *>(f_true);
  auto ttw = static_cast<const V2<T> *>(tw);
  auto tp = static_cast<const V2<T> *>(post);
  hipError_t e = hipSuccess;
#define AR_X(MODE)                                                                             \
  e = smem > 64 * 1024 ? hipFuncSetAttribute(                                                  \
                             reinterpret_cast<const void *>(rows1023_kernel<TS, T, MODE, G>), \
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)           \
                       : hipSuccess;                                                           \
  if (e == hipSuccess) {                                                                       \
    hipLaunchKernelGGL((rows1023_kernel<TS, T, MODE, G>), grid, block, smem, st, ti, to, n1,   \
                       ttw, tp, T(alpha), T(scale), T(tau), tf, partial, jobs, kit);           \
    e = hipGetLastError();                                                                     \
  }
  switch (mode) {
    case ROW_FWD: AR_X(ROW_FWD) break;
    case ROW_INV: AR_X(ROW_INV) break;
    default: AR_X(ROW_INV_UPDATE) break;
  }
#undef AR_X
  return e == hipSuccess ? AR_OK : hip_fail(e, "rows1023_kernel launch");
}

template <typename TS, typename T, int G, int W>
int cols_t(const void *in, void *out, int n2, int blocks, size_t smem, int mode, const void *tw,
           const void *post, double alpha, double scale, const void *dT, const XJob *jobs,
           int count, hipStream_t st) {
  const dim3 grid(blocks, count), block(64 * G * W);
  auto ti = static_cast<const TS *>(in);
  auto to = static_cast<TS *>(out);
  auto td = static_cast<const TS *>(dT);
  auto ttw = static_cast<const V2<T> *>(tw);
  auto tp = static_cast<const V2<T> *>(post);
  hipError_t e = hipSuccess;
#define AR_X(MODE)                                                                             \
  e = smem > 64 * 1024                                                                         \
          ? hipFuncSetAttribute(                                                               \
                reinterpret_cast<const void *>(cols1023_kernel<TS, T, MODE, G, W>),            \
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)                         \
          : hipSuccess;                                                                        \
  if (e == hipSuccess) {                                                                       \
    hipLaunchKernelGGL((cols1023_kernel<TS, T, MODE, G, W>), grid, block, smem, st, ti, to,    \
                       n2, ttw, tp, T(alpha), T(scale), td, jobs);                             \
    e = hipGetLastError();                                                                     \
  }
  switch (mode) {
    case COL_FWD: AR_X(COL_FWD) break;
    case COL_INV: AR_X(COL_INV) break;
    default: AR_X(COL_FWD_D_INV) break;
  }
#undef AR_X
  return e == hipSuccess ? AR_OK : hip_fail(e, "cols1023_kernel launch");
}

template <typename TS, typename T>
int cols_d(const void *in, void *out, int n2, int W, int G, int blocks, size_t smem, int mode,
           const void *tw, const void *post, double alpha, double scale, const void *dT,
           const XJob *jobs, int count, hipStream_t st) {
#define AR_C(G_, W_)                                                                          \
  cols_t<TS, T, G_, W_>(in, out, n2, blocks, smem, mode, tw, post, alpha, scale, dT, jobs,   \
                        count, st)
  if (G == 4) return W == 2 ? AR_C(4, 2) : AR_C(4, 1);
  return W == 4 ? AR_C(2, 4) : W == 2 ? AR_C(2, 2) : AR_C(2, 1);
#undef AR_C
}

}  // namespace

size_t x1023_lds(int W, size_t csize) {
  return (size_t)W * (1024 * 2 * csize + (size_t)zpitch(W) * csize);
}

int x1023_cap(int G) { return kWgMax / (64 * G); }

// U and staging of P pairs, then 8 running-sum slots (V2) per pair
size_t x1023_pair_lds(int P, size_t csize) { return x1023_lds_dev(P, csize) + 16 * csize * P; }

int x1023_cols_pair_launch(size_t ts, size_t cs, const void *in, void *out, int n2, int W,
                           size_t smem, int mode, const void *tw, const void *post, double alpha,
                           double scale, const void *dT, hipStream_t st) {
  if ((W != 2 && W != 4) || n2 % W || smem < x1023_pair_lds(W / 2, cs))
    return fail(AR_EUNSUPPORTED, "length-1024 paired column pass: bad launch shape");
  if (cs != 8) return fail(AR_EUNSUPPORTED, "length-1024 paired column pass: FP64 arithmetic only");
#define AR_W(TS)                                                                               \
  return W == 4 ? colsp_t<TS, double, 4>(in, out, n2, smem, mode, tw, post, alpha, scale, dT,  \
                                         st)                                                   \
                : colsp_t<TS, double, 2>(in, out, n2, smem, mode, tw, post, alpha, scale, dT, st)
  if (ts == 8) { AR_W(double); }
  AR_W(float);
#undef AR_W
}

int x1023_rows_pair_launch(size_t ts, size_t cs, const void *in, void *out, int n1, int W, int G,
                           size_t smem, int mode, const void *tw, const void *post, double alpha,
                           double scale, double tau, const void *f_true, double *partial,
                           hipStream_t st) {
  if (G != 4 || W < 2 || W % 2 || (W / 2) * G * 64 > kWgMax ||
      smem < x1023_pair_lds(W / 2, cs))
    return fail(AR_EUNSUPPORTED, "length-1024 paired row pass: bad launch shape");
  if (cs != 8) return fail(AR_EUNSUPPORTED, "length-1024 paired row pass: FP64 arithmetic only");
  const int P = W / 2;
  if (ts == 8)
    return rowsp_t<double, double, 4>(in, out, n1, P, smem, mode, tw, post, alpha, scale, tau,
                                      f_true, partial, st);
  return rowsp_t<float, double, 4>(in, out, n1, P, smem, mode, tw, post, alpha, scale, tau,
                                   f_true, partial, st);
}

int x1023_rows_launch(size_t ts, size_t cs, const void *in, void *out, int n1, int W, int G,
                      size_t smem, int mode, const void *tw, const void *post, double alpha,
                      double scale, double tau, const void *f_true, double *partial,
                      const XJob *jobs, int count, int kit, hipStream_t st) {
  if ((G != 2 && G != 4) || W < 1 || W * G * 64 > kWgMax)
    return fail(AR_EUNSUPPORTED, "length-1024 row pass: bad launch shape");
  const int blocks = (n1 + W - 1) / W;
#define AR_D(TS, T)                                                                              \
  return G == 4 ? rows_t<TS, T, 4>(in, out, n1, W, blocks, smem, mode, tw, post, alpha, scale,  \
                                   tau, f_true, partial, jobs, count, kit, st)                   \
                : rows_t<TS, T, 2>(in, out, n1, W, blocks, smem, mode, tw, post, alpha, scale,  \
                                   tau, f_true, partial, jobs, count, kit, st)
  if (ts == 8) { AR_D(double, double); }
  if (cs == 8) { AR_D(float, double); }
  AR_D(float, float);
#undef AR_D
}

int x1023_cols_launch(size_t ts, size_t cs, const void *in, void *out, int n2, int W, int G,
                      size_t smem, int mode, const void *tw, const void *post, double alpha,
                      double scale, const void *dT, const XJob *jobs, int count, hipStream_t st) {
  if ((G != 2 && G != 4) || (W != 1 && W != 2 && W != 4) || W * G * 64 > kWgMax || n2 % W)
    return fail(AR_EUNSUPPORTED, "length-1024 column pass: bad launch shape");
  const int blocks = n2 / W;
  if (ts == 8)
    return cols_d<double, double>(in, out, n2, W, G, blocks, smem, mode, tw, post, alpha, scale,
                                  dT, jobs, count, st);
  if (cs == 8)
    return cols_d<float, double>(in, out, n2, W, G, blocks, smem, mode, tw, post, alpha, scale,
                                 dT, jobs, count, st);
  return cols_d<float, float>(in, out, n2, W, G, blocks, smem, mode, tw, post, alpha, scale, dT,
                              jobs, count, st);
}

}  // namespace ar
