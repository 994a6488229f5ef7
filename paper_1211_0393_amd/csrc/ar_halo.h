// Halo extension rules of the blur kernels (gfx950): the boundary
// conditions of the plan (Anti-Reflective, Sec. 2.2; Reflective, Sec. 2.1;
// Periodic), or zero outside the image.
#pragma once

#include "ar_internal.h"

namespace ar {

// Extension modes of the halo loader: the plan's boundary conditions, or
// zero outside the image (the correlation half of A^T).
enum ExtMode { EXT_AR = 0, EXT_ZERO = 1, EXT_REFLECT = 2, EXT_PERIODIC = 3 };

// Extension rule along one axis, branch-free: position i of an axis of
// length n maps to w0 * f[i0] + w1 * f[i1].  AR (Sec. 2.2): interior
// (i, 1) + (i, 0); before the start (0, 2) + (-i, -1)
// (f_{1-t} = 2 f_1 - f_{1+t}); past the end (n-1, 2) + (2n-2-i, -1)
// (f_{n+t} = 2 f_n - f_{n-t}).  Reflective (Sec. 2.1): f_{1-t} = f_t and
// f_{n+t} = f_{n+1-t}, one term.  Periodic: wrap-around, one term.  `dead`
// marks positions that no stored output consumes (more than q outside) or,
// with zero extension, any position outside the image; they read exactly 0.
struct Rule { int i0, i1; float w0, w1; bool dead; };

__device__ __forceinline__ Rule ar_rule(int i, int n, int q, int mode) {
  Rule r;
  const bool lo = i < 0, hi = i > n - 1;
  r.dead = (i < -q) | (i > n - 1 + q) | ((mode == EXT_ZERO) & (lo | hi));
  if (mode == EXT_REFLECT || mode == EXT_PERIODIC) {
    const int jl = mode == EXT_REFLECT ? -i - 1 : i + n;
    const int jh = mode == EXT_REFLECT ? 2 * n - 1 - i : i - n;
    r.i0 = lo ? jl : (hi ? jh : i);
    r.i1 = r.i0;
    r.w0 = 1.f;
    r.w1 = 0.f;
  } else {
    r.i0 = lo ? 0 : (hi ? n - 1 : i);
    r.i1 = lo ? -i : (hi ? 2 * n - 2 - i : i);
    r.w0 = (lo | hi) ? 2.f : 1.f;
    r.w1 = (lo | hi) ? -1.f : 0.f;
  }
  // keep every address inside the image (the value is discarded when dead)
  r.i0 = r.i0 < 0 ? 0 : (r.i0 > n - 1 ? n - 1 : r.i0);
  r.i1 = r.i1 < 0 ? 0 : (r.i1 > n - 1 ? n - 1 : r.i1);
  return r;
}

// Value of the extended image at (i, j) in the compute type T from
// storage-type pixels: the tensor product of the two 1-D rules (one, two or
// four distinct terms; corners give the double anti-reflection 4, -2, -2, 1).
// All four loads are unconditional so a caller can batch them.
template <typename T, typename TS>
__device__ __forceinline__ T load_ext(const Gl<TS> *__restrict__ in, int n1, int n2, int q1,
                                      int q2, int i, int j, int mode) {
  const Rule a = ar_rule(i, n1, q1, mode), b = ar_rule(j, n2, q2, mode);
  const T x00 = T(in[(size_t)a.i0 * n2 + b.i0]);
  const T x01 = T(in[(size_t)a.i0 * n2 + b.i1]);
  const T x10 = T(in[(size_t)a.i1 * n2 + b.i0]);
  const T x11 = T(in[(size_t)a.i1 * n2 + b.i1]);
  // a term with a zero weight repeats the pixel of a weighted term (i1 == i0
  // there), so evaluating it unconditionally adds an exact zero
  const T v = T(a.w0) * (T(b.w0) * x00 + T(b.w1) * x01) + T(a.w1) * (T(b.w0) * x10 + T(b.w1) * x11);
  return (a.dead | b.dead) ? T(0) : v;
}

// Halo mode of a plan's blur (EXT_ZERO is requested explicitly by A^T).
inline int plan_ext_mode(const ar_plan_s *p) {
  return p->bc == AR_BC_REFLECTIVE ? EXT_REFLECT
                                   : (p->bc == AR_BC_PERIODIC ? EXT_PERIODIC : EXT_AR);
}

}  // namespace ar
