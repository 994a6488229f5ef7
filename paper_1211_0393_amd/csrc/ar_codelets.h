// Straight-line DFT codelets with compile-time roots of unity (gfx950).
// Shared by the transform engines.
#pragma once

#include <utility>

#include "ar_internal.h"

namespace ar {
namespace cl {

// ----------------------------------------------- compile-time roots of unity

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double sin_taylor(double x) {
  double x2 = x * x, term = x, s = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    s += term;
  }
  return s;
}
constexpr double cos_taylor(double x) {
  double x2 = x * x, term = 1.0, s = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    s += term;
  }
  return s;
}
// cos(2 pi num / den) with exact reduction to the first octant.
constexpr double cos2pi(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  const long q = (4 * num) / den, rem = 4 * num - q * den;
  double c = 0, s = 0;
  if (2 * rem <= den) {
    const double th = (kPi / 2) * double(rem) / double(den);
    c = cos_taylor(th);
    s = sin_taylor(th);
  } else {
    const double th = (kPi / 2) * double(den - rem) / double(den);
    c = sin_taylor(th);
    s = cos_taylor(th);
  }
  return q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}
constexpr double sin2pi(long num, long den) { return cos2pi(4 * num - den, 4 * den); }

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ----------------------------------------------------------- DFT codelets

// Forward DFT of odd length R: pairs v_j and v_{R-j} so that each output
// pair (k, R-k) needs (R-1)/2 real-by-complex products for the cosine part
// and as many for the sine part.  Output k is handed to emit(K, value)
// with K = std::integral_constant<int, k> as soon as it is formed, so a
// caller may store it directly (inputs are only read before that point).
// The work is in three pieces so that the output pairs can be dealt to
// several wavefronts: the pair sums and differences (dft_odd_ab), output 0
// (dft_odd_zero) and the output pairs k = K0+1 .. K1 (dft_odd_pairs).
template <int R, typename T>
__device__ __forceinline__ void dft_odd_ab(const V2<T> (&v)[R], V2<T> (&a)[(R - 1) / 2],
                                           V2<T> (&b)[(R - 1) / 2]) {
  static_for<(R - 1) / 2>([&](auto J) {
    constexpr int j = J + 1;
    a[J] = cadd(v[j], v[R - j]);
    b[J] = csub(v[j], v[R - j]);
  });
}

template <int R, typename T, typename Emit>
__device__ __forceinline__ void dft_odd_zero(const V2<T> &v0, const V2<T> (&a)[(R - 1) / 2],
                                             Emit &&emit) {
  V2<T> s0 = v0;
  static_for<(R - 1) / 2>([&](auto J) { s0 = cadd(s0, a[J]); });
  emit(std::integral_constant<int, 0>{}, s0);
}

template <int R, int K0, int K1, typename T, typename Emit>
__device__ __forceinline__ void dft_odd_pairs(const V2<T> &v0, const V2<T> (&a)[(R - 1) / 2],
                                              const V2<T> (&b)[(R - 1) / 2], Emit &&emit) {
  constexpr int H = (R - 1) / 2;
  static_for<K1 - K0>([&](auto KK) {
    constexpr int k = K0 + KK + 1;
    V2<T> C = v0, S{T(0), T(0)};
    static_for<H>([&](auto J) {
      constexpr int j = J + 1;
      constexpr int idx = (j * k) % R;
      constexpr T cv = T(cos2pi(idx, R));
      constexpr T sv = T(sin2pi(idx, R));
      C.x = fma(a[J].x, cv, C.x);
      C.y = fma(a[J].y, cv, C.y);
      if constexpr (J == 0) {
        S.x = b[J].x * sv;
        S.y = b[J].y * sv;
      } else {
        S.x = fma(b[J].x, sv, S.x);
        S.y = fma(b[J].y, sv, S.y);
      }
    });
    // out_k = C - i S, out_{R-k} = C + i S
    emit(std::integral_constant<int, k>{}, V2<T>{C.x + S.y, C.y - S.x});
    emit(std::integral_constant<int, R - k>{}, V2<T>{C.x - S.y, C.y + S.x});
  });
}

template <int R, typename T, typename Emit>
__device__ __forceinline__ void dft_odd(const V2<T> (&v)[R], Emit &&emit) {
  constexpr int H = (R - 1) / 2;
  V2<T> a[H], b[H];
  dft_odd_ab<R, T>(v, a, b);
  const V2<T> v0 = v[0];
  dft_odd_zero<R, T>(v0, a, emit);
  dft_odd_pairs<R, 0, H, T>(v0, a, b, emit);
}

// Forward DFT of the radices with a codelet; outputs through emit(K, value).
template <int R, typename T, typename Emit>
__device__ __forceinline__ void dft_emit(const V2<T> (&v)[R], Emit &&emit) {
  if constexpr (R == 2) {
    emit(std::integral_constant<int, 0>{}, cadd(v[0], v[1]));
    emit(std::integral_constant<int, 1>{}, csub(v[0], v[1]));
  } else if constexpr (R == 4) {
    const V2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const V2<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    emit(std::integral_constant<int, 0>{}, cadd(t0, t2));
    emit(std::integral_constant<int, 2>{}, csub(t0, t2));
    emit(std::integral_constant<int, 1>{}, V2<T>{t1.x + t3.y, t1.y - t3.x});  // t1 - i t3
    emit(std::integral_constant<int, 3>{}, V2<T>{t1.x - t3.y, t1.y + t3.x});  // t1 + i t3
  } else {
    static_assert(R % 2 == 1, "odd radix expected");
    dft_odd<R, T>(v, emit);
  }
}

// In-place forward DFT of the radices with a codelet.
template <int R, typename T>
__device__ __forceinline__ void dft(V2<T> (&v)[R]) {
  V2<T> w[R];
  static_for<R>([&](auto r) { w[r] = v[r]; });
  dft_emit<R, T>(w, [&](auto K, V2<T> x) { v[decltype(K)::value] = x; });
}

// Bijective remap of a workgroup id so that consecutive logical ids run on
// the same XCD (workgroups are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, i = b >> 3;
  const int g8 = G >> 3, rem = G & 7;
  return x * g8 + (x < rem ? x : rem) + i;
}

// Radices with a compiled codelet.
__host__ __device__ constexpr bool has_codelet(int r) {
  return r == 2 || r == 3 || r == 4 || r == 5 || r == 7 || r == 11 || r == 13 || r == 17 ||
         r == 19 || r == 23 || r == 29 || r == 31;
}

}  // namespace cl
}  // namespace ar
