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
// A workgroup owns a 128 x 32 output tile (eight waves of 16 rows, two
// column blocks each).  It stages the (128 + 2 q1) x 48 halo in LDS as two
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

constexpr int MW = 8;                  // wavefronts per workgroup
constexpr int MT_THREADS = 64 * MW;
constexpr int MT_H = 16 * MW;          // output rows per tile (16 per wavefront)
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
__global__ __launch_bounds__(MT_THREADS) void conv_mfma_kernel(
    const float *__restrict__ in, float *__restrict__ out, const h8 *__restrict__ frag, int n1,
    int n2, int q2, int ext_mode, float wscale_inv, const float *__restrict__ gsub,
    double *__restrict__ partial, int tiles_x) {
  constexpr int K1 = 2 * Q1 + 1;
  constexpr int LH = MT_H + 2 * Q1;
  constexpr int HP = MHW / 2;                  // column pairs per halo row
  constexpr int NP = (LH * HP + MT_THREADS - 1) / MT_THREADS;    // pairs per thread
  constexpr int NB = 2 * K1 * 64;              // weight fragments (h8) of the tile
  constexpr int NF = (NB + MT_THREADS - 1) / MT_THREADS;
  // hi plane and lo plane of the halo (border tiles stage FP32 values here
  // first), and the weight fragments shared by the eight waves
  __shared__ __align__(16) _Float16 sbuf[2 * LH * MPITCH];
  __shared__ __align__(16) h8 sfrag[NB];
  __shared__ float redf[MW];
  __shared__ double redd[MW];
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
    const int e = tid + MT_THREADS * i;
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
  // aligned pairs when rows have an even length); border tiles evaluate the
  // plan's extension rule on load, every position from its (up to four)
  // image pixels (the same arithmetic as a rule applied to staged pixels,
  // and measured faster than staging the window in LDS first).
  const Gl<float> *gin = gmem(in);
  const bool inside = ib1 >= 0 && ib2 + lo_c >= 0 && ib1 + LH <= n1 && ib2 + hi_c <= n2;
  float v[NP][2];
  if (inside) {
    const bool pairs = (n2 & 1) == 0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = tid + MT_THREADS * i;
      const int rr0 = e / HP, cc = 2 * (e - rr0 * HP);
      const Gl<float> *row = gin + (size_t)(ib1 + (rr0 < LH ? rr0 : LH - 1)) * n2;
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
      const int e = tid + MT_THREADS * i;
      const int rr0 = e / HP, cc = 2 * (e - rr0 * HP);
      const int rr = rr0 < LH ? rr0 : LH - 1;
#pragma unroll
      for (int u = 0; u < 2; ++u)
        v[i][u] = load_ext<float, float>(gin, n1, n2, Q1, q2, ib1 + rr, ib2 + cc + u, ext_mode);
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + MT_THREADS * i;
    if (e < NB) sfrag[e] = fr[i];
  }
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int e = tid + MT_THREADS * i;
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
  mx = redf[0];
  for (int w = 1; w < MW; ++w) mx = fmaxf(mx, redf[w]);
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
    const int e = tid + MT_THREADS * i;
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
    if (tid == 0) {
      double t = redd[0];
      for (int w = 1; w < MW; ++w) t += redd[w];
      gmem(partial)[blockIdx.x] = t;
    }
  }
}

// Residual and reblur fused: y = A' (g - A x) for one 128 x 32 tile of y,
// with the residual's ||r||^2 partial over the tile.  The reblur needs r on
// its (64 + 2 q1) x 48 halo; the kernel computes r there itself, in 16 x 16
// blocks of the same banded Toeplitz products (the region [r0 - q1, r0 - q1
// + 16 RB) x [c0 - 8, c0 + 40), from an x halo of 2 q1 more rows and 16 more
// columns), keeps it in LDS, gives the reblur's ghost positions their
// extension rule from r itself, and runs the reblur on it.  Every value is
// computed by the same arithmetic as the two separate kernels (the same
// scales, splits and products), so y equals theirs bitwise; only the FP64
// order of the ||r||^2 partial differs.  Anti-Reflective and Reflective
// extensions only (a periodic ghost lies across the image).
template <int Q1>
__global__ __launch_bounds__(MT_THREADS) void conv2_mfma_kernel(
    const float *__restrict__ in, const float *__restrict__ gsub, float *__restrict__ out,
    const h8 *__restrict__ frag_fwd, const h8 *__restrict__ frag_rev, int n1, int n2, int q2,
    int ext_mode, float wscale_inv, double *__restrict__ partial, int tiles_x) {
  constexpr int K1 = 2 * Q1 + 1;
  constexpr int RB = (MT_H + 2 * Q1 + 15) / 16;  // 16-row blocks of the r region
  constexpr int RH = 16 * RB;                    // rows of the r region
  constexpr int NBLK = 3 * RB;                   // 16 x 16 blocks of the r region
  constexpr int MB = (NBLK + MW - 1) / MW;       // blocks per wave
  constexpr int LH1 = RH + 2 * Q1;               // x halo rows
  constexpr int W1 = 64, P1 = W1 + 8;            // x halo columns and pitch (halves)
  constexpr int HP1 = W1 / 2;
  constexpr int NP1 = (LH1 * HP1 + MT_THREADS - 1) / MT_THREADS;
  constexpr int LH2 = MT_H + 2 * Q1;             // rows of the reblur's halo
  constexpr int HP2 = MHW / 2;
  constexpr int NP2 = (LH2 * HP2 + MT_THREADS - 1) / MT_THREADS;
  constexpr int NB = 2 * K1 * 64;
  constexpr int NF = (NB + MT_THREADS - 1) / MT_THREADS;
  // LDS: the x planes, later (after the r products) the FP32 r region and
  // the reblur's planes; the weight fragments of the current product
  constexpr int XPL = 2 * LH1 * P1 * 2;
  constexpr int RST = RH * MHW * 4;
  constexpr int RPL = 2 * LH2 * MPITCH * 2;
  constexpr int UA = XPL > RST + RPL ? XPL : RST + RPL;
  __shared__ __align__(16) unsigned char sA[UA];
  __shared__ __align__(16) h8 sfrag[NB];
  __shared__ float redf[MW];
  __shared__ double redd[MW];
  _Float16 *xhi = reinterpret_cast<_Float16 *>(sA), *xlo = xhi + LH1 * P1;
  float *rs = reinterpret_cast<float *>(sA);
  _Float16 *shi = reinterpret_cast<_Float16 *>(sA + RST), *slo = shi + LH2 * MPITCH;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int logical = mfma_xcd_remap(blockIdx.x, gridDim.x);
  const int ty = logical / tiles_x, tx = logical - ty * tiles_x;
  const int r0 = ty * MT_H, c0 = tx * MT_W;
  const int rr0 = r0 - Q1, rc0 = c0 - 8;   // r region origin = the reblur halo's origin
  const int xb1 = rr0 - Q1, xb2 = rc0 - 8;  // x halo origin
  const int lo_c = 8 - q2, hi_c = MT_W + 8 + q2;  // reblur halo columns carrying data
  const int lo1 = 8 - q2, hi1 = 56 + q2;          // x halo columns carrying data
  const int lj = lane & 15, li = (lane >> 4) * 4;
  const int lr = lane & 15, kg = lane >> 4;

  // every global load first: both weight sets, g of this wave's r blocks,
  // the x halo
  const Gl<h8> *gff = gmem(frag_fwd), *gfr = gmem(frag_rev);
  h8 ff[NF], fb[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + MT_THREADS * i;
    ff[i] = gff[e < NB ? e : 0];
    fb[i] = gfr[e < NB ? e : 0];
  }
  float gv[MB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int id = wave + MW * m;
    const int rb = (id < NBLK ? id : 0) / 3, cb = (id < NBLK ? id : 0) % 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int oi = rr0 + 16 * rb + li + i, oj = rc0 + 16 * cb + lj;
      oi = oi < 0 ? 0 : (oi > n1 - 1 ? n1 - 1 : oi);
      oj = oj < 0 ? 0 : (oj > n2 - 1 ? n2 - 1 : oj);
      gv[m][i] = gmem(gsub)[(size_t)oi * n2 + oj];
    }
  }
  const Gl<float> *gin = gmem(in);
  const bool inside1 = xb1 >= 0 && xb2 + lo1 >= 0 && xb1 + LH1 <= n1 && xb2 + hi1 <= n2;
  float v[NP1][2];
  {
    const bool pairs = (n2 & 1) == 0;
#pragma unroll
    for (int i = 0; i < NP1; ++i) {
      const int e = tid + MT_THREADS * i;
      const int rw = e / HP1, cc = 2 * (e - rw * HP1);
      int ii = xb1 + (rw < LH1 ? rw : LH1 - 1);
      ii = ii < 0 ? 0 : (ii > n1 - 1 ? n1 - 1 : ii);
      const Gl<float> *row = gin + (size_t)ii * n2;
      if (pairs) {
        int jj = xb2 + cc;
        jj = jj < 0 ? 0 : (jj > n2 - 2 ? n2 - 2 : jj);
        const f2 t = *reinterpret_cast<const Gl<f2> *>(row + jj);
        v[i][0] = t[0];
        v[i][1] = t[1];
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          int jj = xb2 + cc + u;
          jj = jj < 0 ? 0 : (jj > n2 - 1 ? n2 - 1 : jj);
          v[i][u] = row[jj];
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + MT_THREADS * i;
    if (e < NB) sfrag[e] = ff[i];
  }
  // window position of an image row (column) a rule references; the clamp
  // only guards positions whose value is discarded
  auto wrow = [&](int x, int base, int len) {
    const int t = x - base;
    return t < 0 ? 0 : (t > len - 1 ? len - 1 : t);
  };
  if (!inside1) {
    // border tile: the clamped x window as FP32, then every ghost's rule
    float *stage = reinterpret_cast<float *>(sA);
#pragma unroll
    for (int i = 0; i < NP1; ++i) {
      const int e = tid + MT_THREADS * i;
      if (e < LH1 * HP1) {
        const int rw = e / HP1, cc = 2 * (e - rw * HP1);
        stage[rw * W1 + cc] = v[i][0];
        stage[rw * W1 + cc + 1] = v[i][1];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NP1; ++i) {
      const int e = tid + MT_THREADS * i;
      const int rw0 = e / HP1, cc0 = 2 * (e - rw0 * HP1);
      const int rw = rw0 < LH1 ? rw0 : LH1 - 1;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ii = xb1 + rw, jj = xb2 + cc0 + u;
        if (ii < 0 || ii > n1 - 1 || jj < 0 || jj > n2 - 1) {
          const Rule ra = ar_rule(ii, n1, Q1, ext_mode), rb = ar_rule(jj, n2, q2, ext_mode);
          const float *s0 = stage + wrow(ra.i0, xb1, LH1) * W1;
          const float *s1 = stage + wrow(ra.i1, xb1, LH1) * W1;
          const int b0 = wrow(rb.i0, xb2, W1), b1 = wrow(rb.i1, xb2, W1);
          const float xv = ra.w0 * (rb.w0 * s0[b0] + rb.w1 * s0[b1]) +
                           ra.w1 * (rb.w0 * s1[b0] + rb.w1 * s1[b1]);
          v[i][u] = (ra.dead | rb.dead) ? 0.f : xv;
        }
      }
    }
    __syncthreads();
  }
  // scale and split the x halo
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < NP1; ++i) {
    const int e = tid + MT_THREADS * i;
    const int cc0 = 2 * (e % HP1);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (!(e < LH1 * HP1 && cc0 + u >= lo1 && cc0 + u < hi1)) v[i][u] = 0.f;
      mx = fmaxf(mx, fabsf(v[i][u]));
    }
  }
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) redf[wave] = mx;
  __syncthreads();
  mx = redf[0];
  for (int w = 1; w < MW; ++w) mx = fmaxf(mx, redf[w]);
  auto scale_exp = [](float m) {
    int ex = 0;
    if (m > 0.f && m <= 3.0e38f) {
      int E;
      (void)frexpf(m, &E);
      ex = 14 - E;
      ex = ex > 100 ? 100 : (ex < -100 ? -100 : ex);
    }
    return ex;
  };
  const int ex1 = scale_exp(mx);
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int i = 0; i < NP1; ++i) {
    const int e = tid + MT_THREADS * i;
    if (e < LH1 * HP1) {
      const int rw = e / HP1, cc = 2 * (e - rw * HP1);
      h2 hh, ll;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float xs = ldexpf(v[i][u], ex1);
        const _Float16 h = (_Float16)xs;
        hh[u] = h;
        ll[u] = (_Float16)(xs - (float)h);
      }
      *reinterpret_cast<h2 *>(xhi + rw * P1 + cc) = hh;
      *reinterpret_cast<h2 *>(xlo + rw * P1 + cc) = ll;
    }
  }
  __syncthreads();

  // r = g - A x on this wave's 16 x 16 blocks of the r region (block id =
  // wave + MW m: row block id / 3, column block id % 3)
  float rv[MB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int id = wave + MW * m;
    if (id >= NBLK) break;
    const int rb = id / 3, cb = id % 3;
    const _Float16 *hrow = xhi + (16 * rb + lr) * P1 + 16 * cb + kg * 8;
    const _Float16 *lrow = xlo + (16 * rb + lr) * P1 + 16 * cb + kg * 8;
    i4 ah = *reinterpret_cast<const i4 *>(hrow), al = *reinterpret_cast<const i4 *>(lrow);
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < K1; ++a) {
      if (a > 0) {
        ah = row_up(ah);
        al = row_up(al);
        if (lr == 15) {
          ah = *reinterpret_cast<const i4 *>(hrow + a * P1);
          al = *reinterpret_cast<const i4 *>(lrow + a * P1);
        }
      }
      const h8 bh = sfrag[(2 * a) * 64 + lane], bl = sfrag[(2 * a + 1) * 64 + lane];
      const h8 xh = __builtin_bit_cast(h8, ah), xl = __builtin_bit_cast(h8, al);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, bh, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) rv[m][i] = gv[m][i] - ldexpf(acc[i] * wscale_inv, -ex1);
  }
  __syncthreads();  // the x planes and the forward weights are read
  // r to its FP32 region; the reblur's weights to LDS
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int id = wave + MW * m;
    if (id >= NBLK) break;
    const int rb = id / 3, cb = id % 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) rs[(16 * rb + li + i) * MHW + 16 * cb + lj] = rv[m][i];
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    const int e = tid + MT_THREADS * i;
    if (e < NB) sfrag[e] = fb[i];
  }
  __syncthreads();
  // ||r||^2 over the tile's own pixels (rows Q1.., columns 8.. of the region)
  if (partial) {
    double ss = 0.0;
    for (int e = tid; e < MT_H * MT_W; e += MT_THREADS) {
      const int i = e / MT_W, j = e - i * MT_W;
      if (r0 + i < n1 && c0 + j < n2) {
        const double t = (double)rs[(Q1 + i) * MHW + 8 + j];
        ss += t * t;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) redd[wave] = ss;
  }
  // the reblur's halo from r: image positions as computed, ghosts by the
  // extension rule of r, zero outside the data columns
  const bool inside2 = rr0 >= 0 && rc0 + lo_c >= 0 && rr0 + LH2 <= n1 && rc0 + hi_c <= n2;
  float w[NP2][2];
#pragma unroll
  for (int i = 0; i < NP2; ++i) {
    const int e = tid + MT_THREADS * i;
    const int rw0 = e / HP2, cc0 = 2 * (e - rw0 * HP2);
    const int rw = rw0 < LH2 ? rw0 : LH2 - 1;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int cc = cc0 + u;
      float val = rs[rw * MHW + cc];
      if (!inside2) {
        const int ii = rr0 + rw, jj = rc0 + cc;
        if (ii < 0 || ii > n1 - 1 || jj < 0 || jj > n2 - 1) {
          const Rule ra = ar_rule(ii, n1, Q1, ext_mode), rb = ar_rule(jj, n2, q2, ext_mode);
          const float *s0 = rs + wrow(ra.i0, rr0, RH) * MHW;
          const float *s1 = rs + wrow(ra.i1, rr0, RH) * MHW;
          const int b0 = wrow(rb.i0, rc0, MHW), b1 = wrow(rb.i1, rc0, MHW);
          const float xv = ra.w0 * (rb.w0 * s0[b0] + rb.w1 * s0[b1]) +
                           ra.w1 * (rb.w0 * s1[b0] + rb.w1 * s1[b1]);
          val = (ra.dead | rb.dead) ? 0.f : xv;
        }
      }
      w[i][u] = (e < LH2 * HP2 && cc >= lo_c && cc < hi_c) ? val : 0.f;
    }
  }
  mx = 0.f;
#pragma unroll
  for (int i = 0; i < NP2; ++i)
#pragma unroll
    for (int u = 0; u < 2; ++u) mx = fmaxf(mx, fabsf(w[i][u]));
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  __syncthreads();  // redf reuse
  if (lane == 0) redf[wave] = mx;
  __syncthreads();
  mx = redf[0];
  for (int w = 1; w < MW; ++w) mx = fmaxf(mx, redf[w]);
  const int ex2 = scale_exp(mx);
  if (partial && tid == 0) {
    double t = redd[0];
    for (int w = 1; w < MW; ++w) t += redd[w];
    gmem(partial)[blockIdx.x] = t;
  }
#pragma unroll
  for (int i = 0; i < NP2; ++i) {
    const int e = tid + MT_THREADS * i;
    if (e < LH2 * HP2) {
      const int rw = e / HP2, cc = 2 * (e - rw * HP2);
      h2 hh, ll;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float xs = ldexpf(w[i][u], ex2);
        const _Float16 h = (_Float16)xs;
        hh[u] = h;
        ll[u] = (_Float16)(xs - (float)h);
      }
      *reinterpret_cast<h2 *>(shi + rw * MPITCH + cc) = hh;
      *reinterpret_cast<h2 *>(slo + rw * MPITCH + cc) = ll;
    }
  }
  __syncthreads();

  // y = A' r: 2 blocks x K1 PSF rows x 3 products per wave (as conv_mfma_kernel)
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
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const f4 acc = blk ? acc1 : acc0;
    const int oj = c0 + 16 * blk + lj;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oi = r0 + wave * 16 + li + i;
      if (oi < n1 && oj < n2) gmem(out)[(size_t)oi * n2 + oj] = ldexpf(acc[i] * wscale_inv, -ex2);
    }
  }
}

}  // namespace

bool conv_mfma_ok(const ar_plan_s *p) {
  return p->dtype == AR_F32 && p->mfma_frag_fwd != nullptr && p->q1 <= kMfmaMaxQ1 &&
         p->q2 <= kMfmaMaxQ2 && p->tune[AR_TUNE_BLUR] != 1;
}

int conv_mfma_blocks(int m1, int m2) { return ((m1 + MT_H - 1) / MT_H) * ((m2 + MT_W - 1) / MT_W); }

bool conv2_mfma_ok(const ar_plan_s *p) {
  return conv_mfma_ok(p) && p->bc != AR_BC_PERIODIC && p->tune[AR_TUNE_FUSE] == 1;
}

int conv2_mfma_launch(const ar_plan_s *p, const void *x, const void *g, void *y, double *partial,
                      hipStream_t st) {
  const int tiles_x = (p->n2 + MT_W - 1) / MT_W;
  const int blocks = conv_mfma_blocks(p->n1, p->n2);
  const float wsi = std::ldexp(1.0f, -p->mfma_ew);
  const h8 *ff = static_cast<const h8 *>(p->mfma_frag_fwd);
  const h8 *fr = static_cast<const h8 *>(p->mfma_frag_rev);
  const float *tx = static_cast<const float *>(x);
  const float *tg = static_cast<const float *>(g);
  float *ty = static_cast<float *>(y);
  const int em = plan_ext_mode(p);
  if (em != EXT_AR && em != EXT_REFLECT)
    return fail(AR_EUNSUPPORTED, "fused matrix-core residual and reblur: AR or Reflective only");
#define AR_MFMA2_CASE(QQ)                                                                     \
  case QQ:                                                                                    \
    hipLaunchKernelGGL((conv2_mfma_kernel<QQ>), dim3(blocks), dim3(MT_THREADS), 0, st, tx, tg, ty,   \
                       ff, fr, p->n1, p->n2, p->q2, em, wsi, partial, tiles_x);               \
    break;
  switch (p->q1) {
    AR_MFMA2_CASE(0) AR_MFMA2_CASE(1) AR_MFMA2_CASE(2) AR_MFMA2_CASE(3) AR_MFMA2_CASE(4)
    AR_MFMA2_CASE(5) AR_MFMA2_CASE(6) AR_MFMA2_CASE(7) AR_MFMA2_CASE(8) AR_MFMA2_CASE(9)
    AR_MFMA2_CASE(10)
    default:
      return fail(AR_EUNSUPPORTED, "matrix-core blur: PSF row half-width above 10");
  }
#undef AR_MFMA2_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "conv2_mfma_kernel launch");
  return AR_OK;
}

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
    hipLaunchKernelGGL((conv_mfma_kernel<QQ>), dim3(blocks), dim3(MT_THREADS), 0, st, ti, to, frag,   \
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
