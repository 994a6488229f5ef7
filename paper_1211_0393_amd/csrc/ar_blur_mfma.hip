// AR-BC blur on the matrix cores for FP32 plans (gfx950).
//
// The blur g_i = sum_s h_s f_{i-s} (eq. (modello_discreto)) of the extended
// image is written, per PSF row a, as a banded Toeplitz product: for a
// 16 x 16 block of outputs starting at column j0, out[i][j] += sum_k
// E[i + a][j0 + k] W_a[k][j] with W_a[k][j] = w[a][k - j] for
// 0 <= k - j <= 2 q2 (w the correlation weights), k < 32.  One
// v_mfma_f32_16x16x32_f16 per (block, a) computes it; FP32 accuracy comes
// from splitting both operands into two FP16 terms, v = hi + lo with
// lo = v - hi, and summing hi*hi + hi*lo + lo*hi with FP32 accumulation
// (about 2^-21 relative per product).  FP16 range is kept by exact
// power-of-two scaling: the input tile by 2^ex (its largest magnitude lands
// in [2^13, 2^14)), the weights by 2^ew (the same rule for the largest
// weight, chosen at plan time); the output is multiplied back by
// 2^-(ex + ew).
//
// A workgroup owns a 64 x 32 output tile (four waves of 16 rows, two
// column blocks each).  It stages the (64 + 2 q1) x 48 halo in LDS as two
// FP16 planes (hi, lo) after applying the plan's extension rule on load;
// the weight fragments W_a (hi and lo) are prepared once per PSF and staged
// in LDS by each workgroup, and the A fragment of PSF row a + 1 is obtained
// from row a's by a lane shift.
#include <cmath>

#include "ar_halo.h"
#include "ar_internal.h"

namespace ar {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// Lane r of every 16-lane row takes the value of lane r + 1 (DPP row shift
// left by one); the row's last lane keeps its own, to be replaced.
__device__ __forceinline__ i4 row_up(i4 x) {
  i4 y;
#pragma unroll
  for (int c = 0; c < 4; ++c) y[c] = __builtin_amdgcn_update_dpp(x[c], x[c], 0x101, 0xf, 0xf, false);
  return y;
}

constexpr int MT_H = 64;               // output rows per tile (4 waves x 16)
constexpr int MT_W = 32;               // output columns per tile (2 blocks of 16)
constexpr int MHW = MT_W - 16 + 32;    // halo columns: the last block's 32-wide window
constexpr int MPITCH = MHW + 8;        // 56 halves = 112 bytes: 8 rows hit 8 distinct 16-byte slots

__device__ __forceinline__ int mfma_xcd_remap(int b, int G) {
  const int x = b & 7, i = b >> 3;
  const int g8 = G >> 3, rem = G & 7;
  return x * g8 + (x < rem ? x : rem) + i;
}

// Weight fragments of one PSF: frag[(2 a + part) * 64 + lane] holds, for
// lane l (column j = l % 16, k-group g = l / 16), the eight values
// W_a[8 g + t][j] = w[a][8 g + t - j - (8 - q2)], t = 0..7 (zero outside
// the PSF row), scaled by 2^ew and split into FP16 hi (part 0) and lo
// (part 1).  The offset 8 - q2 places the 32-wide window of a 16-column
// block at an 8-aligned halo column.  rot: the correlation weights are H
// rotated by 180 degrees (A) instead of H itself (A').
__global__ void mfma_frag_kernel(const double *__restrict__ H, int q1, int q2, int rot, int ew,
                                 h8 *__restrict__ frag) {
  const int a = blockIdx.x, lane = threadIdx.x;
  const int j = lane & 15, g = lane >> 4;
  const int K1 = 2 * q1 + 1, K2 = 2 * q2 + 1;
  h8 hi, lo;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int b = 8 * g + t - j - (8 - q2);
    double w = 0.0;
    if (b >= 0 && b < K2) w = rot ? H[(K1 - 1 - a) * K2 + (K2 - 1 - b)] : H[a * K2 + b];
    const double ws = ldexp(w, ew);
    const _Float16 h = (_Float16)(float)ws;
    hi[t] = h;
    lo[t] = (_Float16)(float)(ws - (double)h);
  }
  frag[(2 * a) * 64 + lane] = hi;
  frag[(2 * a + 1) * 64 + lane] = lo;
}

template <int Q1>
__global__ __launch_bounds__(256) void conv_mfma_kernel(
    const float *__restrict__ in, float *__restrict__ out, const h8 *__restrict__ frag, int n1,
    int n2, int q2, int ext_mode, float wscale_inv, const float *__restrict__ gsub,
    double *__restrict__ partial, int tiles_x) {
  constexpr int K1 = 2 * Q1 + 1;
  constexpr int LH = MT_H + 2 * Q1;
  constexpr int HP = MHW / 2;                  // column pairs per halo row
  constexpr int NP = (LH * HP + 255) / 256;    // pairs per thread
  constexpr int NB = 2 * K1 * 64;              // weight fragments (h8) of the tile
  constexpr int NF = (NB + 255) / 256;
  // hi plane and lo plane of the halo (border tiles stage FP32 values here
  // first), and the weight fragments shared by the four waves
  __shared__ __align__(16) _Float16 sbuf[2 * LH * MPITCH];
  __shared__ __align__(16) h8 sfrag[NB];
  __shared__ float redf[4];
  __shared__ double redd[4];
  _Float16 *shi = sbuf, *slo = sbuf + LH * MPITCH;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int logical = mfma_xcd_remap(blockIdx.x, gridDim.x);
  const int ty = logical / tiles_x, tx = logical - ty * tiles_x;
  const int r0 = ty * MT_H, c0 = tx * MT_W;
  // halo origin: Q1 rows above the tile, 8 columns left of it (8-aligned)
  const int ib1 = r0 - Q1, ib2 = c0 - 8;
  const int lo_c = 8 - q2, hi_c = MT_W + 8 + q2;  // halo columns [lo_c, hi_c) carry data
  const int lj = lane & 15, li = (lane >> 4) * 4;

  // Every global load of the tile is issued before the first wait: the
  // weight fragments (for LDS), the residual's g and the halo.
  const Gl<h8> *gf = gmem(frag);
  h8 fr[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + 256 * i;
    fr[i] = gf[e < NB ? e : 0];
  }
  float gv[2][4];
  if (gsub) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int oi = r0 + wave * 16 + li + i, oj = c0 + 16 * blk + lj;
        oi = oi < n1 ? oi : n1 - 1;
        oj = oj < n2 ? oj : n2 - 1;
        gv[blk][i] = gmem(gsub)[(size_t)oi * n2 + oj];
      }
  }
  // Halo as column pairs.  Tiles inside the image load it directly (as
  // aligned pairs when rows have an even length); border tiles under
  // Anti-Reflective or Reflective BCs load the window clamped to the image
  // (every ghost pixel is a combination of pixels in that window) and apply
  // the rule from LDS below; periodic border tiles apply the rule on load
  // (their ghosts come from the far side of the image).
  const Gl<float> *gin = gmem(in);
  const bool inside = ib1 >= 0 && ib2 + lo_c >= 0 && ib1 + LH <= n1 && ib2 + hi_c <= n2;
  const bool wrap = !inside && ext_mode == EXT_PERIODIC;
  float v[NP][2];
  if (!wrap) {
    const bool pairs = (n2 & 1) == 0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = tid + 256 * i;
      const int rr0 = e / HP, cc = 2 * (e - rr0 * HP);
      int ii = ib1 + (rr0 < LH ? rr0 : LH - 1);
      ii = ii < 0 ? 0 : (ii > n1 - 1 ? n1 - 1 : ii);
      const Gl<float> *row = gin + (size_t)ii * n2;
      if (pairs) {
        int jj = ib2 + cc;
        jj = jj < 0 ? 0 : (jj > n2 - 2 ? n2 - 2 : jj);
        const f2 t = *reinterpret_cast<const Gl<f2> *>(row + jj);
        v[i][0] = t[0];
        v[i][1] = t[1];
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          int jj = ib2 + cc + u;
          jj = jj < 0 ? 0 : (jj > n2 - 1 ? n2 - 1 : jj);
          v[i][u] = row[jj];
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = tid + 256 * i;
      const int rr0 = e / HP, cc = 2 * (e - rr0 * HP);
      const int rr = rr0 < LH ? rr0 : LH - 1;
#pragma unroll
      for (int u = 0; u < 2; ++u)
        v[i][u] = load_ext<float, float>(gin, n1, n2, Q1, q2, ib1 + rr, ib2 + cc + u, ext_mode);
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + 256 * i;
    if (e < NB) sfrag[e] = fr[i];
  }

  if (!inside && !wrap) {
    // border tile: the clamped window to LDS as FP32, then every position's
    // extension rule evaluated from it
    float *stage = reinterpret_cast<float *>(sbuf);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = tid + 256 * i;
      if (e < LH * HP) {
        const int rr = e / HP, cc = 2 * (e - rr * HP);
        stage[rr * MHW + cc] = v[i][0];
        stage[rr * MHW + cc + 1] = v[i][1];
      }
    }
    __syncthreads();
    // window position of an image row (column) that the rule references
    // (it lies in the clamped window; the clamp only guards dead positions)
    auto wr = [&](int x) { const int t = x - ib1; return t < 0 ? 0 : (t > LH - 1 ? LH - 1 : t); };
    auto wc = [&](int x) {
      int t = x - ib2;
      // clamped loads put image column c at window column c - ib2 when the
      // window is inside the image; past the image edges the staged values
      // repeat the edge pair, which no rule reads
      return t < 0 ? 0 : (t > MHW - 1 ? MHW - 1 : t);
    };
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = tid + 256 * i;
      const int rr0 = e / HP, cc0 = 2 * (e - rr0 * HP);
      const int rr = rr0 < LH ? rr0 : LH - 1;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cc = cc0 + u;
        const int ii = ib1 + rr, jj = ib2 + cc;
        // pixels of the image keep their loaded value; only ghosts take the rule
        if (ii < 0 || ii > n1 - 1 || jj < 0 || jj > n2 - 1) {
          const Rule ra = ar_rule(ii, n1, Q1, ext_mode), rb = ar_rule(jj, n2, q2, ext_mode);
          const float *s0 = stage + wr(ra.i0) * MHW, *s1 = stage + wr(ra.i1) * MHW;
          const float x = ra.w0 * (rb.w0 * s0[wc(rb.i0)] + rb.w1 * s0[wc(rb.i1)]) +
                          ra.w1 * (rb.w0 * s1[wc(rb.i0)] + rb.w1 * s1[wc(rb.i1)]);
          v[i][u] = (ra.dead | rb.dead) ? 0.f : x;
        }
      }
    }
    __syncthreads();
  }
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int e = tid + 256 * i;
    const int cc0 = 2 * (e % HP);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (!(e < LH * HP && cc0 + u >= lo_c && cc0 + u < hi_c)) v[i][u] = 0.f;
      mx = fmaxf(mx, fabsf(v[i][u]));
    }
  }
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) redf[wave] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(redf[0], redf[1]), fmaxf(redf[2], redf[3]));
  int ex = 0;
  if (mx > 0.f && mx <= 3.0e38f) {
    int E;
    (void)frexpf(mx, &E);
    ex = 14 - E;
    ex = ex > 100 ? 100 : (ex < -100 ? -100 : ex);
  }
  // scaled split into the two planes, two halves per 32-bit store
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int e = tid + 256 * i;
    if (e < LH * HP) {
      const int rr = e / HP, cc = 2 * (e - rr * HP);
      h2 hh, ll;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float xs = ldexpf(v[i][u], ex);
        const _Float16 h = (_Float16)xs;
        hh[u] = h;
        ll[u] = (_Float16)(xs - (float)h);
      }
      *reinterpret_cast<h2 *>(shi + rr * MPITCH + cc) = hh;
      *reinterpret_cast<h2 *>(slo + rr * MPITCH + cc) = ll;
    }
  }
  __syncthreads();

  // 2 blocks x K1 PSF rows x 3 products per wave.  The A fragment of PSF
  // row a + 1 is that of row a moved up by one image row: inside each group
  // of 16 lanes (one fragment row per lane) lane r takes lane r + 1's
  // registers (DPP row shift), and only the group's last lane reads its new
  // row from LDS.
  const int lr = lane & 15, kg = lane >> 4;
  const _Float16 *hrow = shi + (wave * 16 + lr) * MPITCH + kg * 8;
  const _Float16 *lrow = slo + (wave * 16 + lr) * MPITCH + kg * 8;
  i4 ah0 = *reinterpret_cast<const i4 *>(hrow), ah1 = *reinterpret_cast<const i4 *>(hrow + 16);
  i4 al0 = *reinterpret_cast<const i4 *>(lrow), al1 = *reinterpret_cast<const i4 *>(lrow + 16);
  f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < K1; ++a) {
    if (a > 0) {
      ah0 = row_up(ah0);
      ah1 = row_up(ah1);
      al0 = row_up(al0);
      al1 = row_up(al1);
      if (lr == 15) {
        ah0 = *reinterpret_cast<const i4 *>(hrow + a * MPITCH);
        ah1 = *reinterpret_cast<const i4 *>(hrow + a * MPITCH + 16);
        al0 = *reinterpret_cast<const i4 *>(lrow + a * MPITCH);
        al1 = *reinterpret_cast<const i4 *>(lrow + a * MPITCH + 16);
      }
    }
    const h8 bh = sfrag[(2 * a) * 64 + lane], bl = sfrag[(2 * a + 1) * 64 + lane];
    const h8 xh0 = __builtin_bit_cast(h8, ah0), xh1 = __builtin_bit_cast(h8, ah1);
    const h8 xl0 = __builtin_bit_cast(h8, al0), xl1 = __builtin_bit_cast(h8, al1);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl0, bh, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl1, bh, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh0, bl, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh1, bl, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh0, bh, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh1, bh, acc1, 0, 0, 0);
  }

  // lane l holds rows 4 (l / 16) + i, column l % 16 of each 16 x 16 block
  double ss = 0.0;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const f4 acc = blk ? acc1 : acc0;
    const int oj = c0 + 16 * blk + lj;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oi = r0 + wave * 16 + li + i;
      if (oi < n1 && oj < n2) {
        float val = ldexpf(acc[i] * wscale_inv, -ex);
        const size_t o = (size_t)oi * n2 + oj;
        if (gsub) {
          val = gv[blk][i] - val;
          ss += (double)val * (double)val;
        }
        gmem(out)[o] = val;
      }
    }
  }
  if (partial) {
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) redd[wave] = ss;
    __syncthreads();
    if (tid == 0) gmem(partial)[blockIdx.x] = ((redd[0] + redd[1]) + redd[2]) + redd[3];
  }
}

}  // namespace

bool conv_mfma_ok(const ar_plan_s *p) {
  return p->dtype == AR_F32 && p->mfma_frag_fwd != nullptr && p->q1 <= kMfmaMaxQ1 &&
         p->q2 <= kMfmaMaxQ2 && p->tune[AR_TUNE_BLUR] != 1;
}

int conv_mfma_blocks(int m1, int m2) { return ((m1 + MT_H - 1) / MT_H) * ((m2 + MT_W - 1) / MT_W); }

int mfma_frag_build(ar_plan_s *p, double hmax, hipStream_t st) {
  if (p->dtype != AR_F32 || p->q1cap > kMfmaMaxQ1 || p->q2cap > kMfmaMaxQ2) return AR_OK;
  const size_t bytes = (size_t)(2 * p->q1cap + 1) * 2 * 64 * sizeof(h8);
  if (!p->mfma_frag_fwd) {
    AR_HIP(hipMalloc(&p->mfma_frag_fwd, bytes));
    AR_HIP(hipMalloc(&p->mfma_frag_rev, bytes));
  }
  int E = 0;
  if (hmax > 0.0) (void)std::frexp(hmax, &E);
  p->mfma_ew = hmax > 0.0 ? 14 - E : 0;
  hipLaunchKernelGGL(mfma_frag_kernel, dim3(2 * p->q1 + 1), dim3(64), 0, st, p->H64, p->q1, p->q2,
                     1, p->mfma_ew, static_cast<h8 *>(p->mfma_frag_fwd));
  hipLaunchKernelGGL(mfma_frag_kernel, dim3(2 * p->q1 + 1), dim3(64), 0, st, p->H64, p->q1, p->q2,
                     0, p->mfma_ew, static_cast<h8 *>(p->mfma_frag_rev));
  AR_HIP(hipGetLastError());
  return AR_OK;
}

int conv_mfma_launch(const ar_plan_s *p, const void *in, void *out, bool reverse,
                     const void *gsub, double *partial, hipStream_t st) {
  const int tiles_x = (p->n2 + MT_W - 1) / MT_W;
  const int blocks = conv_mfma_blocks(p->n1, p->n2);
  const float wsi = std::ldexp(1.0f, -p->mfma_ew);
  const h8 *frag = static_cast<const h8 *>(reverse ? p->mfma_frag_rev : p->mfma_frag_fwd);
  const float *ti = static_cast<const float *>(in);
  float *to = static_cast<float *>(out);
  const float *tg = static_cast<const float *>(gsub);
  const int em = plan_ext_mode(p);
#define AR_MFMA_CASE(QQ)                                                                      \
  case QQ:                                                                                    \
    hipLaunchKernelGGL((conv_mfma_kernel<QQ>), dim3(blocks), dim3(256), 0, st, ti, to, frag,   \
                       p->n1, p->n2, p->q2, em, wsi, tg, partial, tiles_x);                   \
    break;
  switch (p->q1) {
    AR_MFMA_CASE(0) AR_MFMA_CASE(1) AR_MFMA_CASE(2) AR_MFMA_CASE(3) AR_MFMA_CASE(4)
    AR_MFMA_CASE(5) AR_MFMA_CASE(6) AR_MFMA_CASE(7) AR_MFMA_CASE(8) AR_MFMA_CASE(9)
    AR_MFMA_CASE(10)
    default:
      return fail(AR_EUNSUPPORTED, "matrix-core blur: PSF row half-width above 10");
  }
#undef AR_MFMA_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "conv_mfma_kernel launch");
  return AR_OK;
}

}  // namespace ar
