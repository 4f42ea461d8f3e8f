// Learned per-element correction to Jacobi, used as the preconditioner of
// flexible CG (not in the paper; a chosen extension of its preconditioned
// CG): for an element with residual r_e and s_e = ||dinv r||_e,
//   x0 = [r, dinv r] / s_e,  h = relu(conv1(x0)),  y = conv2(h),
//   z_L = dinv r + s_e y,    z = M QQ^T (c z_L),
// with 3x3x3 kernels, zero padding at element borders and no bias (the map
// is positively homogeneous in r).  Inputs x0, weights and the hidden
// activations h are rounded to BF16 (RNE); products are accumulated in
// FP32.  Training minimises mean_s ||z_s - e_s||_A^2 / ||e_s||_A^2.
//
// Forward, one workgroup per element: each thread owns positions p; it
// gathers its 54 input neighbours, forms the 32 hidden channels and folds
// them at once into T[p][o] = sum_c W2[c][o] h[c][p] (27 values), so the
// second convolution becomes y[p] = sum_o T[p + o][o] (27 LDS reads instead
// of 864).  Weights are uniform across the wave and are read through the
// scalar cache.
// Backward, a fixed set of workgroups each walking a fixed list of
// elements, the forward recomputed: for N = 7 on the matrix cores (four
// small GEMMs per 32-position tile, see nn_bwd_mfma_n8_kernel), for N = 3
// and 5 in vector FP32 with every thread accumulating the gradient entries
// it owns.  One partial per workgroup, summed in a fixed order afterwards
// (deterministic, no atomics).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <type_traits>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

constexpr int NN_CH = 32;
constexpr int NN_CIN = 2;
constexpr int NN_W1 = NN_CH * NN_CIN * 27;
constexpr int NN_W2 = NN_CH * 27;
constexpr int NN_NP = NN_W1 + NN_W2;
constexpr int NN_THREADS = 256;
constexpr int NN_BWD_BLOCKS = 512;

__device__ inline float bf16r(float x) { return bf16_to_float(float_to_bf16(x)); }

// neighbour of position p = (i,j,k) at offset o, or -1 outside the element
template <int n>
__device__ inline int nbr_of(int i, int j, int k, int o) {
  const int ii = i + (o % 3) - 1, jj = j + (o / 3) % 3 - 1, kk = k + o / 9 - 1;
  if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) return -1;
  return ii + n * (jj + n * kk);
}

// block-wide float sum broadcast to every thread
__device__ inline float block_sum_bcast(float v, float* sred) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  float s = 0.f;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sred[q];
  return s;
}

// Forward: zc = c * z_L for every element (the gather-scatter follows).
template <int N>
__global__ void __launch_bounds__(NN_THREADS)
    nn_fwd_kernel(const float* __restrict__ r, const float* __restrict__ dinv,
                  const uint8_t* __restrict__ mult, const float* __restrict__ W1,
                  const float* __restrict__ W2, float* __restrict__ zc, int E,
                  const State* __restrict__ st, NnDots dd) {
  constexpr int n = N + 1, n3 = n * n * n, PPT = (n3 + NN_THREADS - 1) / NN_THREADS;
  extern __shared__ float sm[];
  float* x0 = sm;           // [2][n3]
  float* T = sm + 2 * n3;   // [n3][27]
  __shared__ float sred[8];
  const int e = blockIdx.x;
  if (e >= E || (st && st->done)) return;
  const int64_t base = (int64_t)e * n3;
  const float alpha = dd.x ? (float)st->alpha : 0.f;
  float rv[PPT], dv[PPT];
  float ss = 0.f;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * NN_THREADS;
    rv[q] = dv[q] = 0.f;
    if (p < n3) {
      rv[q] = r[base + p];
      if (dd.x) {  // the step's vector update (uniform branch)
        rv[q] = rv[q] - alpha * dd.w[base + p];
        const_cast<float*>(r)[base + p] = rv[q];
        dd.x[base + p] = dd.x[base + p] + alpha * dd.p[base + p];
      }
      dv[q] = dinv[base + p] * rv[q];
      ss += dv[q] * dv[q];
    }
  }
  const float s = sqrtf(block_sum_bcast(ss, sred));
  const float inv = s > 0.f ? 1.f / s : 0.f;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * NN_THREADS;
    if (p < n3) {
      x0[p] = bf16r(rv[q] * inv);
      x0[n3 + p] = bf16r(dv[q] * inv);
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * NN_THREADS;
    if (p >= n3) continue;
    const int i = p % n, j = (p / n) % n, k = p / (n * n);
    float xin[54];
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int nb = nbr_of<n>(i, j, k, o);
      xin[o] = nb >= 0 ? x0[nb] : 0.f;
      xin[27 + o] = nb >= 0 ? x0[n3 + nb] : 0.f;
    }
    float t[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) t[o] = 0.f;
#pragma unroll 2
    for (int c = 0; c < NN_CH; ++c) {
      float a = 0.f;
#pragma unroll
      for (int jj = 0; jj < 54; ++jj) a += W1[c * 54 + jj] * xin[jj];
      const float h = bf16r(fmaxf(a, 0.f));
#pragma unroll
      for (int o = 0; o < 27; ++o) t[o] += W2[c * 27 + o] * h;
    }
#pragma unroll
    for (int o = 0; o < 27; ++o) T[p * 27 + o] = t[o];
  }
  __syncthreads();
  double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * NN_THREADS;
    if (p >= n3) continue;
    const int i = p % n, j = (p / n) % n, k = p / (n * n);
    float y = 0.f;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int nb = nbr_of<n>(i, j, k, o);
      if (nb >= 0) y += T[nb * 27 + o];
    }
    const float zl = dv[q] + s * y;
    const uint8_t m = mult[base + p];
    const float zv = m == 1 ? zl : zl / (float)m;
    zc[base + p] = zv;
    if (dd.dots) {
      const double wq = (double)dd.w[base + p], c = cweight(m), cj = c * (double)dv[q];
      dsum[0] += (double)rv[q] * (double)zv;
      dsum[1] += wq * (double)zv;
      dsum[2] += (double)rv[q] * cj;
      dsum[3] += wq * cj;
      dsum[4] += (double)rv[q] * c * (double)rv[q];
    }
  }
  if (dd.dots) {
    __shared__ double dred[16];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double a = block_sum(dsum[k], dred);
      if (threadIdx.x == 0) dd.dots[k * dd.dstride + e] = a;
    }
  }
}

// Forward for N = 7 on the matrix cores (gfx950 v_mfma_f32_32x32x16_bf16),
// both layers as small GEMMs over the 512 positions of an element, computed
// transposed so that positions run along the result columns:
//   layer 1: H[c][p] = relu(sum_k W1[c][k] X[k][p]),  k = (slot, ci), K = 64
//   layer 2: T[o][p] = sum_c W2[c][o] H[c][p],         27 taps -> 32 rows
//   y[p]     = sum_o T[o][p + d_o]                     (zero outside)
//            = sum_g R_g[p + (0, dy_g, dz_g)],  R_g[q] = sum_dx T[(dx,dy_g,dz_g)][q + (dx,0,0)]
// over the 9 groups g = (dy, dz): a tile spans the element's full width in
// i, so the three taps of a group are summed in registers, the i-shifts being
// lane shifts within a row of 8 lanes (DPP), before anything goes to LDS.
// Operand layout of the instruction (lane l, h = l/32): A row l%32 and
// B column l%32, with k = 8h + t; result column l%32, rows
// 8(v/4) + 4h + v%4.  The first layer's result is therefore already the
// second layer's B operand in the same lane (the channel order inside K is
// absorbed into the packed W2), so the hidden tile never leaves registers.
// A tile is 32 positions: 8 along i times 4 along j in one k layer; a wave
// runs its 4 tiles as two interleaved pairs.
//
// LDS, laid out so that every access of a half wave hits 32 distinct banks:
//  * X holds (x0, x1) as one BF16 pair per position in a zero-bordered
//    10^3 grid with row stride 40 and plane stride 400 (the 4 rows of a
//    tile fall into 4 disjoint groups of 8 banks).  The 27 taps sit in the
//    32 input slots so that each operand's two halves are taps whose
//    offsets differ by the same constant in both half waves (1 or 40): an
//    operand is two paired 32-bit loads.
//  * U[g][p] = R_g[p + (0, dy_g, dz_g)]: group g's sum for source q is
//    stored at p = q - (0, dy_g, dz_g) of plane g (9 planes of 512,
//    unpadded).  Stores whose p falls outside the element, and a half wave's
//    unused fifth group, go to a 32-word trash row on the bank they would
//    have used; slots that no source reaches (the convolution's zero border)
//    are cleared once per workgroup and never written.  The sum over groups
//    is then 9 loads of consecutive words per position.
// Second-layer result rows: row R = 8 q + 4 h + t holds, for t < 3, tap dx =
// t - 1 of group g = q + 4 h; the t = 3 rows of q = 0, 1, 2 in half 0 hold
// group 8 (dx = -1, 0, +1); the other rows are padding.  A lane's registers
// v = 4 s + t (s < 4) are then group s + 4 h, and v = 3, 7, 11 group 8 (half
// 0) or padding (half 1).
// 16 KB + 18.1 KB per workgroup, three workgroups per CU; workgroups are
// persistent.  The roundings are the vector kernel's (BF16 inputs, weights
// and h; FP32 accumulation); y is summed by groups here (each group's taps in
// dx order), in tap order there.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef short short2_t __attribute__((ext_vector_type(2)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Persistent workgroups per CU of the MFMA forward: 34.5 KB of LDS each, and
// at most 168 VGPRs, so that three waves share a SIMD.
constexpr int NN_FWD_WG_PER_CU = 3;

namespace nnm {
constexpr int XR = 40, XPL = 400, XWORDS = 10 * XPL;  // bordered input grid
constexpr int UOFF = XWORDS;                          // group planes after X
constexpr int NPL = 9;                                // (dy, dz) groups
constexpr int TRASH = NPL * 512;                      // 32-word trash row
constexpr int UWORDS = TRASH + 32;
constexpr int LDS_BYTES = 4 * (XWORDS + UWORDS);
constexpr int tdx(int o) { return o % 3 - 1; }
constexpr int tdy(int o) { return (o / 3) % 3 - 1; }
constexpr int tdz(int o) { return o / 9 - 1; }
constexpr int xoff(int o) { return tdx(o) + XR * tdy(o) + XPL * tdz(o); }
constexpr int tap_of(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }
// First-layer input slots: slot = 8 ks + 4h + u holds tap in_tap[slot]
// (-1: padding, zero weight).  Slots u = 2m, 2m+1 are read as one pair at
// offsets in_off[8ks + 4h + 2m] + {0, pair_gap(ks)}.
struct InSlots {
  int tap[32];
  int off[32];  // X offset of the pair's first load (even u only)
  constexpr InSlots() : tap(), off() {
    int q = 0;
    // gap-1 pairs: (dx = -1, dx = 0) of every row, then (dx = +1, padding)
    // of the rows dy = +1; gap-40 pairs: (dx = +1, dy = -1 / 0), then
    // two padding slots
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy) {
        tap[q] = tap_of(-1, dy, dz), tap[q + 1] = tap_of(0, dy, dz);
        off[q] = xoff(tap[q]);
        q = next(q);
      }
    for (int dz = -1; dz <= 1; ++dz) {
      tap[q] = tap_of(1, 1, dz), tap[q + 1] = -1;
      off[q] = xoff(tap[q]);
      q = next(q);
    }
    for (int dz = -1; dz <= 1; ++dz) {
      tap[q] = tap_of(1, -1, dz), tap[q + 1] = tap_of(1, 0, dz);
      off[q] = xoff(tap[q]);
      q = next(q);
    }
    tap[q] = tap[q + 1] = -1;
    off[q] = 0;
  }
  // pairs in the order (ks, m, h): fill h = 0 then h = 1 of one (ks, m)
  static constexpr int next(int q) {
    // q = 8ks + 4h + 2m
    const int ks = q / 8, h = (q / 4) % 2, m = (q / 2) % 2;
    if (h == 0) return 8 * ks + 4 + 2 * m;
    return m == 0 ? 8 * ks + 2 : 8 * (ks + 1);
  }
};
constexpr InSlots IN{};
constexpr int pair_gap(int ks) { return ks < 3 ? 1 : XR; }
// second-layer result row -> group (-1: padding) and tap
constexpr int row_group(int R) {
  const int q = R / 8, h = (R / 4) % 2, t = R % 4;
  return t < 3 ? q + 4 * h : (h == 0 && q < 3 ? 8 : -1);
}
constexpr int row_dx(int R) { return R % 4 < 3 ? R % 4 - 1 : R / 8 - 1; }
constexpr int row_tap(int R) {
  return row_group(R) < 0 ? -1
                          : tap_of(row_dx(R), row_group(R) % 3 - 1, row_group(R) / 3 - 1);
}
constexpr int group_dy(int g) { return g % 3 - 1; }
constexpr int group_dz(int g) { return g / 3 - 1; }
// every tap in exactly one row
constexpr bool rows_cover_taps() {
  for (int o = 0; o < 27; ++o) {
    int hits = 0;
    for (int R = 0; R < 32; ++R) hits += row_tap(R) == o;
    if (hits != 1) return false;
  }
  return true;
}
static_assert(rows_cover_taps(), "second-layer rows hold each tap once");
static_assert(NPL * 512 * 4 <= 65535, "group planes reachable by LDS load offsets");
}  // namespace nnm

// Weight operands in the per-lane operand layout, packed once per weight
// update: pk[ks * 64 + lane].  Forward (A operands, ks 0..5): the 4
// first-layer and then 2 second-layer k steps.  First layer: row = channel,
// k = 16 ks + 8h + 2u + ci <-> input slot 8 ks + 4h + u.  Second layer: row =
// result slot, k = 16 ks + 8h + t <-> channel 16 ks + 8(t/4) + 4h + t%4 (the
// first layer's result rows there).  Backward (B operands, column =
// channel, ks 6..11): W1^T over the slots s = 16 (ks - 6) + 8h + t = 32 ci +
// tap, then W2^T over the taps 16 (ks - 10) + 8h + t; taps 27..31 are zero.
__global__ void nn_pack_kernel(const float* __restrict__ W1, const float* __restrict__ W2,
                               bf16x8_t* __restrict__ pk) {
  const int lane = threadIdx.x & 63, ks = threadIdx.x >> 6;  // 12 x 64 threads
  const int row = lane & 31, h = lane >> 5;
  bf16x8_t v;
  for (int t = 0; t < 8; ++t) {
    if (ks >= 10) {
      const int tap = 16 * (ks - 10) + 8 * h + t;
      v[t] = (__bf16)(tap < 27 ? W2[row * 27 + tap] : 0.f);
    } else if (ks >= 6) {
      const int sl = 16 * (ks - 6) + 8 * h + t, ci = sl >> 5, tap = sl & 31;
      v[t] = (__bf16)(tap < 27 ? W1[row * 54 + ci * 27 + tap] : 0.f);
    } else if (ks < 4) {
      const int tap = nnm::IN.tap[8 * ks + 4 * h + (t >> 1)], ci = t & 1;
      v[t] = (__bf16)(tap >= 0 ? W1[row * 54 + ci * 27 + tap] : 0.f);
    } else {
      const int c = 16 * (ks - 4) + 8 * (t >> 2) + 4 * h + (t & 3);
      const int tap = nnm::row_tap(row);
      v[t] = (__bf16)(tap >= 0 ? W2[c * 27 + tap] : 0.f);
    }
  }
  pk[ks * 64 + lane] = v;
}

__global__ void __launch_bounds__(NN_THREADS, NN_FWD_WG_PER_CU)
    nn_fwd_mfma_n8_kernel(const float* __restrict__ r, const float* __restrict__ dinv,
                          const uint8_t* __restrict__ mult, const bf16x8_t* __restrict__ pk,
                          float* __restrict__ zc, int E, const State* __restrict__ st,
                          NnDots dd) {
  using namespace nnm;
  constexpr int n3 = 512;
  extern __shared__ float sm[];
  unsigned* X = (unsigned*)sm;  // bordered BF16-pair grid
  float* U = sm + UOFF;         // 27 tap planes + trash row
  __shared__ float sred2[2][NN_THREADS / 64];
  if (st && st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31;
  // clear once: the borders of X and the unreached slots of U stay 0
  for (int q = tid; q < XWORDS + UWORDS; q += NN_THREADS) sm[q] = 0.f;
  // weight operands (identical for every element)
  bf16x8_t a1[4], a2[2];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) a1[ks] = pk[ks * 64 + lane];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) a2[ks] = pk[(4 + ks) * 64 + lane];
  // Consume the weight loads here: otherwise the first use inside the loop
  // carries a memory-counter wait that, on later elements, waits for the
  // previous element's result stores instead.
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) asm volatile("" ::"v"(__builtin_bit_cast(u32x4_t, a1[ks])));
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) asm volatile("" ::"v"(__builtin_bit_cast(u32x4_t, a2[ks])));
  // this lane's column in the wave's tiles 4*wave + mt
  const int ci_ = c & 7, cj = c >> 3, ck = 2 * wave;
  const int xq = (ci_ + 1) + XR * (cj + 1) + XPL * (ck + 1);
  // im2col pair address per (k step, pair) for the wave's first tile; tile
  // mt adds the constant XPL (mt / 2) + 4 XR (mt % 2)
  int xb[4][2];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int m = 0; m < 2; ++m) xb[ks][m] = xq + IN.off[8 * ks + 4 * h + 2 * m];
  int wa[4][5];  // group-sum store address per (tile, group slot)
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int sg = 0; sg < 5; ++sg) {
      const int g = sg < 4 ? sg + 4 * h : (h == 0 ? 8 : -1);
      const int dy = g >= 0 ? group_dy(g) : 0, dz = g >= 0 ? group_dz(g) : 0;
      const int pj = cj + 4 * (mt & 1) - dy, pk_ = ck + (mt >> 1) - dz;
      const int a = 512 * (g >= 0 ? g : 0) + ci_ + 8 * pj + 64 * pk_;
      const bool live = g >= 0 && (unsigned)pj < 8u && (unsigned)pk_ < 8u;
      wa[mt][sg] = live ? a : TRASH + (a & 31);
    }
  // the lane's neighbours along i inside its row of 8 (outside: zero)
  const bool has_left = ci_ > 0, has_right = ci_ < 7;
  // positions of the sum over taps: p = tid and tid + 256
  const int pi = tid & 7, pj = (tid >> 3) & 7, pk0 = tid >> 6;
  const int xw = (pi + 1) + XR * (pj + 1) + XPL * (pk0 + 1);
  // The next element's r and dinv are loaded while this one is on the matrix
  // cores; its per-wave partial of ||dinv r||^2 goes to the other half of
  // sred2, so one barrier per element serves both the norm and the reuse of U.
  // w for the dots and the update, loaded with r and dinv one element ahead
  // (r stands in when no dots are asked for, so the loop has no branch);
  // with the update, r is updated as it is loaded (r - alpha w) and x, p
  // of the element in hand are loaded with its multiplicities
  const float* __restrict__ wsrc = dd.dots ? dd.w : r;
  const bool upd = dd.x != nullptr;
  const float alpha = upd ? (float)st->alpha : 0.f;
  const float* __restrict__ xsrc = upd ? dd.x : r;
  const float* __restrict__ psrc = upd ? dd.p : r;
  float rv[2] = {0.f, 0.f}, dv[2] = {0.f, 0.f}, wv[2] = {0.f, 0.f};
  auto partial = [&](int slot) {
    float ss = dv[0] * dv[0] + dv[1] * dv[1];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
    if (lane == 0) sred2[slot][wave] = ss;
  };
  if ((int)blockIdx.x < E) {
    const int64_t base = (int64_t)blockIdx.x * n3;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float r0 = r[base + tid + q * NN_THREADS];
      wv[q] = wsrc[base + tid + q * NN_THREADS];
      rv[q] = upd ? r0 - alpha * wv[q] : r0;
      dv[q] = dinv[base + tid + q * NN_THREADS] * rv[q];
    }
    partial(0);
  }
  double dsum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // this workgroup's share of the dots
  int it = 0;
  for (int e = blockIdx.x; e < E; e += gridDim.x, ++it) {
    const int64_t base = (int64_t)e * n3;
    __syncthreads();  // norm partials complete; U no longer read
    const float* sp = sred2[it & 1];
    const float ss = (sp[0] + sp[1]) + (sp[2] + sp[3]);
    const float inv = ss > 0.f ? rsqrtf(ss) : 0.f;
    const float s = ss * inv;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bf16x2_t xv = {(__bf16)(rv[q] * inv), (__bf16)(dv[q] * inv)};
      X[xw + q * 4 * XPL] = __builtin_bit_cast(unsigned, xv);
    }
    __syncthreads();
    // next element (the last one again past the end: loads stay in bounds
    // and branch-free; the values are then unused)
    const int en = min(e + (int)gridDim.x, E - 1);
    float rn[2], dn[2], wn[2];
    {
      const int64_t bn = (int64_t)en * n3;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        rn[q] = r[bn + tid + q * NN_THREADS];
        dn[q] = dinv[bn + tid + q * NN_THREADS];
        wn[q] = wsrc[bn + tid + q * NN_THREADS];
      }
    }
    uint8_t mv[2];
    float xo[2], po[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      mv[q] = mult[base + tid + q * NN_THREADS];
      xo[q] = xsrc[base + tid + q * NN_THREADS];
      po[q] = psrc[base + tid + q * NN_THREADS];
    }
    // raised wave priority for the matrix-core phase: a wave that has begun
    // its MFMA sequence keeps the SIMD's issue slots ahead of waves in their
    // load and store phases (300 learned steps: 60.2 -> 58.9 ms)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int mp = 0; mp < 4; mp += 2) {
      floatx16_t acc[2] = {{0}, {0}};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2) {
          const int mt = mp + t2;
          u32x4_t w;
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const int xa = xb[ks][m] + XPL * (mt >> 1) + 4 * XR * (mt & 1);
            w[2 * m] = X[xa];
            w[2 * m + 1] = X[xa + pair_gap(ks)];
          }
          acc[t2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              a1[ks], __builtin_bit_cast(bf16x8_t, w), acc[t2], 0, 0, 0);
        }
      u32x4_t hb[2][2];
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          // relu after rounding: on BF16 bit patterns a signed 16-bit max
          // with 0 clears exactly the negative values
          typedef float float2_t __attribute__((ext_vector_type(2)));
          const float2_t fv = {acc[t2][v], acc[t2][v + 1]};
          const bf16x2_t hv = __builtin_convertvector(fv, bf16x2_t);
          const short2_t hz = __builtin_elementwise_max(__builtin_bit_cast(short2_t, hv),
                                                        (short2_t){0, 0});
          hb[t2][v >> 3][(v & 7) >> 1] = __builtin_bit_cast(unsigned, hz);
        }
      floatx16_t acc2[2] = {{0}, {0}};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
          acc2[t2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              a2[ks], __builtin_bit_cast(bf16x8_t, hb[t2][ks]), acc2[t2], 0, 0, 0);
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int sg = 0; sg < 5; ++sg) {
          // taps dx = -1, 0, +1 of the group: R_g[q] = T_-1[q - 1] + T_0[q] + T_+1[q + 1]
          const int vm = sg < 4 ? 4 * sg : 3, v0 = sg < 4 ? 4 * sg + 1 : 7,
                    vp = sg < 4 ? 4 * sg + 2 : 11;
          // DPP row_shr:1: lane n takes lane n - 1; row_shl:1: lane n takes lane n + 1.
          // The elements are copied out first: a bit cast of a vector element
          // in place reads element 0 of the vector.
          const float tm = acc2[t2][vm], tp = acc2[t2][vp];
          const float fl = __builtin_bit_cast(
              float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, tm), 0x111, 0xf, 0xf,
                                                 true));
          const float fr = __builtin_bit_cast(
              float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, tp), 0x101, 0xf, 0xf,
                                                 true));
          const float sum = ((has_left ? fl : 0.f) + acc2[t2][v0]) + (has_right ? fr : 0.f);
          U[wa[mp + t2][sg]] = sum;
        }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = tid + q * NN_THREADS;
      float y = 0.f;
#pragma unroll
      for (int g = 0; g < NPL; ++g) y += U[512 * g + p];
      const float zl = dv[q] + s * y;
      // the weight applied to z_L also weights the Jacobi candidate's dots
      // (exact for the power-of-two multiplicities of a box mesh)
      const float cq = mv[q] == 1 ? 1.f : __builtin_amdgcn_rcpf((float)mv[q]);
      const float zv = zl * cq;
      zc[base + p] = zv;
      const double cj = (double)cq * (double)dv[q];
      dsum[0] += (double)rv[q] * (double)zv;
      dsum[1] += (double)wv[q] * (double)zv;
      dsum[2] += (double)rv[q] * cj;
      dsum[3] += (double)wv[q] * cj;
      dsum[4] += (double)rv[q] * (double)cq * (double)rv[q];
      if (upd) {
        const_cast<float*>(r)[base + p] = rv[q];
        dd.x[base + p] = xo[q] + alpha * po[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      wv[q] = wn[q];
      rv[q] = upd ? rn[q] - alpha * wn[q] : rn[q];
      dv[q] = dn[q] * rv[q];
    }
    partial((it + 1) & 1);
  }
  if (dd.dots) {
    __shared__ double dred[16];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double a = block_sum(dsum[k], dred);
      if (tid == 0) dd.dots[k * dd.dstride + blockIdx.x] = a;
    }
  }
}

// Backward: part[blockIdx.x][*] += gradient of sum_p gzl[p] z_L[p] with
// respect to (W1, W2), over the elements blockIdx.x, +gridDim.x, ...
template <int N>
__global__ void __launch_bounds__(NN_THREADS)
    nn_bwd_kernel(const float* __restrict__ r, const float* __restrict__ dinv,
                  const float* __restrict__ gzl, const float* __restrict__ W1,
                  const float* __restrict__ W2, float* __restrict__ part, int E) {
  constexpr int n = N + 1, n3 = n * n * n, PPT = (n3 + NN_THREADS - 1) / NN_THREADS;
  constexpr int QCH = 8;  // channels per pass of the first-layer gradient
  extern __shared__ float sm[];
  float* x0 = sm;                          // [2][n3]
  float* gy = x0 + 2 * n3;                 // [n3]
  float* ga = gy + n3;                     // [QCH][n3]
  bf16_t* hb = (bf16_t*)(ga + QCH * n3);   // [NN_CH][n3] hidden activations (BF16)
  __shared__ float sred[8];
  float acc2[4], acc1[7];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc2[q] = 0.f;
#pragma unroll
  for (int q = 0; q < 7; ++q) acc1[q] = 0.f;
  for (int e = blockIdx.x; e < E; e += gridDim.x) {
    const int64_t base = (int64_t)e * n3;
    float ss = 0.f;
    float rv[PPT], dv[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * NN_THREADS;
      rv[q] = dv[q] = 0.f;
      if (p < n3) {
        rv[q] = r[base + p];
        dv[q] = dinv[base + p] * rv[q];
        ss += dv[q] * dv[q];
      }
    }
    const float s = sqrtf(block_sum_bcast(ss, sred));
    const float inv = s > 0.f ? 1.f / s : 0.f;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * NN_THREADS;
      if (p < n3) {
        x0[p] = bf16r(rv[q] * inv);
        x0[n3 + p] = bf16r(dv[q] * inv);
        gy[p] = s * gzl[base + p];
      }
    }
    __syncthreads();
    // forward recomputation of the hidden layer
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * NN_THREADS;
      if (p >= n3) continue;
      const int i = p % n, j = (p / n) % n, k = p / (n * n);
      float xin[54];
#pragma unroll
      for (int o = 0; o < 27; ++o) {
        const int nb = nbr_of<n>(i, j, k, o);
        xin[o] = nb >= 0 ? x0[nb] : 0.f;
        xin[27 + o] = nb >= 0 ? x0[n3 + nb] : 0.f;
      }
      for (int c = 0; c < NN_CH; ++c) {
        float a = 0.f;
#pragma unroll
        for (int jj = 0; jj < 54; ++jj) a += W1[c * 54 + jj] * xin[jj];
        hb[c * n3 + p] = float_to_bf16(fmaxf(a, 0.f));
      }
    }
    __syncthreads();
    // second-layer weights: gW2[c][o] = sum_q h[c][q] gy[q - o]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + q * NN_THREADS;
      if (idx >= NN_W2) continue;
      const int c = idx / 27, o = idx % 27;
      const int di = (o % 3) - 1, dj = (o / 3) % 3 - 1, dk = o / 9 - 1;
      float a = 0.f;
      for (int kk = 0; kk < n; ++kk) {
        const int k0 = kk - dk;
        if (k0 < 0 || k0 >= n) continue;
        for (int jj = 0; jj < n; ++jj) {
          const int j0 = jj - dj;
          if (j0 < 0 || j0 >= n) continue;
          for (int ii = 0; ii < n; ++ii) {
            const int i0 = ii - di;
            if (i0 < 0 || i0 >= n) continue;
            a += bf16_to_float(hb[c * n3 + ii + n * (jj + n * kk)]) * gy[i0 + n * (j0 + n * k0)];
          }
        }
      }
      acc2[q] += a;
    }
    // first layer, QCH channels at a time: ga = relu'(a1) * sum_o W2[c][o] gy[p - o],
    // gW1[c][ci][o] = sum_p ga[c][p] x0[ci][p + o]
    for (int c0 = 0; c0 < NN_CH; c0 += QCH) {
      __syncthreads();
      for (int q = 0; q < PPT; ++q) {
        const int p = threadIdx.x + q * NN_THREADS;
        if (p >= n3) continue;
        const int i = p % n, j = (p / n) % n, k = p / (n * n);
        float g[27];
#pragma unroll
        for (int o = 0; o < 27; ++o) {
          // gy at p - o (the output that reads h[p] through offset o)
          const int ii = i - ((o % 3) - 1), jj = j - ((o / 3) % 3 - 1), kk = k - (o / 9 - 1);
          g[o] = (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n)
                     ? 0.f
                     : gy[ii + n * (jj + n * kk)];
        }
        for (int cc = 0; cc < QCH; ++cc) {
          const int c = c0 + cc;
          float a = 0.f;
#pragma unroll
          for (int o = 0; o < 27; ++o) a += W2[c * 27 + o] * g[o];
          ga[cc * n3 + p] = bf16_to_float(hb[c * n3 + p]) > 0.f ? a : 0.f;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const int idx = threadIdx.x + q * NN_THREADS;
        if (idx >= NN_W1) continue;
        const int c = idx / 54;
        if (c < c0 || c >= c0 + QCH) continue;
        const int ci = (idx / 27) % 2, o = idx % 27;
        const int di = (o % 3) - 1, dj = (o / 3) % 3 - 1, dk = o / 9 - 1;
        const float* gc = ga + (c - c0) * n3;
        const float* xc = x0 + ci * n3;
        float a = 0.f;
        for (int kk = 0; kk < n; ++kk) {
          const int k1 = kk + dk;
          if (k1 < 0 || k1 >= n) continue;
          for (int jj = 0; jj < n; ++jj) {
            const int j1 = jj + dj;
            if (j1 < 0 || j1 >= n) continue;
            for (int ii = 0; ii < n; ++ii) {
              const int i1 = ii + di;
              if (i1 < 0 || i1 >= n) continue;
              a += gc[ii + n * (jj + n * kk)] * xc[i1 + n * (j1 + n * k1)];
            }
          }
        }
        acc1[q] += a;
      }
    }
    __syncthreads();
  }
  float* pb = part + (int64_t)blockIdx.x * NN_NP;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int idx = threadIdx.x + q * NN_THREADS;
    if (idx < NN_W1) pb[idx] += acc1[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = threadIdx.x + q * NN_THREADS;
    if (idx < NN_W2) pb[NN_W1 + idx] += acc2[q];
  }
}

// Backward for N = 7 on the matrix cores (v_mfma_f32_32x32x16_bf16).  For
// one element, with positions p, hidden channels c, taps o (offsets d_o) and
// input slots s = (ci, o):
//   (1) H^T[p][c]   = relu(sum_s X_s[p] W1[c][s])            forward, recomputed
//   (3) Ga^T[p][c]  = [H[c][p] > 0] sum_o gy[p - d_o] W2[c][o]  gradient at h
//   (2) gW2^T[o][c] += sum_p gy[p - d_o] H[c][p]
//   (4) gW1^T[s][c] += sum_p x_ci[p + d_o] Ga[c][p]
// with X_s[p] = x_ci[p + d_o] and zero values outside the element.  (1) and
// (3) are computed transposed, positions along the result rows: a lane then
// holds one channel's results at 16 positions, which is the B operand that
// (2) and (4) need in the same lane, the 16 positions taken as two K steps in
// the lane's result-row order (a permutation of the summation index that the
// A operand, gathered from LDS, follows).  x, H, gy and Ga enter the matrix
// cores rounded to BF16; products are summed in FP32.
// Tiles of 32 positions (8 along i, 4 along j, one k layer), 16 per element,
// four per wave; workgroups are persistent over elements, each keeps its
// gradient in the accumulators of its four waves and adds them (in wave
// order) to its partial row at the end.
namespace nnb {
constexpr int GR = 10, GP = 100, GW = 1000;  // zero-bordered 10^3 grid of u16
constexpr int XOFF = 0, GOFF = 2 * GW;       // x0, x1 grids, then gy
constexpr int GRID_U16 = 3 * GW;
constexpr int tdx(int o) { return o % 3 - 1; }
constexpr int tdy(int o) { return (o / 3) % 3 - 1; }
constexpr int tdz(int o) { return o / 9 - 1; }
constexpr int toff(int o) { return o < 27 ? tdx(o) + GR * tdy(o) + GP * tdz(o) : 0; }
}  // namespace nnb

__global__ void __launch_bounds__(NN_THREADS)
    nn_bwd_mfma_n8_kernel(const float* __restrict__ r, const float* __restrict__ dinv,
                          const float* __restrict__ gzl, const bf16x8_t* __restrict__ pkb,
                          float* __restrict__ part, int E) {
  using namespace nnb;
  constexpr int n3 = 512;
  __shared__ unsigned short grid[GRID_U16];
  __shared__ float red[48 * 64];
  __shared__ float sred[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, rl = lane & 31;
  for (int q = tid; q < GRID_U16; q += NN_THREADS) grid[q] = 0;
  // weight operands: W1^T (4 K steps) and W2^T (2), column = channel
  bf16x8_t b1[4], b2[2];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) b1[ks] = pkb[ks * 64 + lane];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) b2[ks] = pkb[(4 + ks) * 64 + lane];
  floatx16_t g2 = {0}, g1a = {0}, g1b = {0};
  for (int e = blockIdx.x; e < E; e += gridDim.x) {
    const int64_t base = (int64_t)e * n3;
    float rv[2], dv[2], ss = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = tid + q * NN_THREADS;
      rv[q] = r[base + p];
      dv[q] = dinv[base + p] * rv[q];
      ss += dv[q] * dv[q];
    }
    const float s = sqrtf(block_sum_bcast(ss, sred));  // barriers: the last element is done
    const float inv = s > 0.f ? 1.f / s : 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = tid + q * NN_THREADS;
      const int i = p & 7, j = (p >> 3) & 7, k = p >> 6;
      const int gq = (k + 1) * GP + (j + 1) * GR + (i + 1);
      grid[XOFF + gq] = float_to_bf16(rv[q] * inv);
      grid[XOFF + GW + gq] = float_to_bf16(dv[q] * inv);
      grid[GOFF + gq] = float_to_bf16(s * gzl[base + p]);
    }
    __syncthreads();
#pragma unroll 1
    for (int tq = 0; tq < 4; ++tq) {
      const int t = wave + 4 * tq;
      const int kk = t >> 1, j0 = 4 * (t & 1);
      // (1) and (3): this lane's row is position (rl % 8, j0 + rl / 8, kk)
      const int pc = (kk + 1) * GP + (j0 + (rl >> 3) + 1) * GR + (rl & 7) + 1;
      floatx16_t a1 = {0}, a3 = {0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        u32x4_t w;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          // slots 16 ks + 8 h + 2u, +1: channel ks / 2, taps (16 ks + 8 h + 2u) % 32, +1
          const int o0 = (16 * ks + 2 * u) & 31, o1 = (16 * ks + 8 + 2 * u) & 31;
          const int ci = ks >> 1;
          const int fa = h ? toff(o1) : toff(o0), fb = h ? toff(o1 + 1) : toff(o0 + 1);
          const unsigned lo = grid[XOFF + ci * GW + pc + fa];
          const unsigned hi = grid[XOFF + ci * GW + pc + fb];
          w[u] = lo | (hi << 16);
        }
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, w), b1[ks], a1,
                                                      0, 0, 0);
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        u32x4_t w;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int o0 = 16 * ks + 2 * u, o1 = 16 * ks + 8 + 2 * u;
          const int fa = h ? toff(o1) : toff(o0), fb = h ? toff(o1 + 1) : toff(o0 + 1);
          const unsigned lo = grid[GOFF + pc - fa];
          const unsigned hi = grid[GOFF + pc - fb];
          w[u] = lo | (hi << 16);
        }
        a3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, w), b2[ks], a3,
                                                      0, 0, 0);
      }
      // H = relu (BF16) and Ga = [H > 0] a3 (BF16), as B operands (K steps v < 8, v >= 8)
      u32x4_t hb[2], gb[2];
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const unsigned h0 = a1[v] > 0.f ? float_to_bf16(a1[v]) : 0u;
        const unsigned h1 = a1[v + 1] > 0.f ? float_to_bf16(a1[v + 1]) : 0u;
        const unsigned q0 = h0 ? float_to_bf16(a3[v]) : 0u;
        const unsigned q1 = h1 ? float_to_bf16(a3[v + 1]) : 0u;
        hb[v >> 3][(v & 7) >> 1] = h0 | (h1 << 16);
        gb[v >> 3][(v & 7) >> 1] = q0 | (q1 << 16);
      }
      // (2) and (4): this lane's row is tap rl (rows 27..31 are discarded);
      // K index 8 h + u of step q <-> result row 8 (2q + u / 4) + 4 h + u % 4,
      // i.e. position (4 h + u % 4, j0 + 2 q + u / 4, kk)
      const int ob = toff(rl < 27 ? rl : 13);
      const int pr = (kk + 1) * GP + (j0 + 1) * GR + 4 * h + 1;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        u32x4_t wg, wx0, wx1;
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          const int c0 = pr + (2 * q + (u >> 2)) * GR + (u & 3);
          const unsigned g0 = grid[GOFF + c0 - ob], g1 = grid[GOFF + c0 + 1 - ob];
          const unsigned x00 = grid[XOFF + c0 + ob], x01 = grid[XOFF + c0 + 1 + ob];
          const unsigned x10 = grid[XOFF + GW + c0 + ob], x11 = grid[XOFF + GW + c0 + 1 + ob];
          wg[u >> 1] = g0 | (g1 << 16);
          wx0[u >> 1] = x00 | (x01 << 16);
          wx1[u >> 1] = x10 | (x11 << 16);
        }
        g2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wg),
                                                      __builtin_bit_cast(bf16x8_t, hb[q]), g2, 0, 0, 0);
        g1a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wx0),
                                                       __builtin_bit_cast(bf16x8_t, gb[q]), g1a, 0, 0, 0);
        g1b = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, wx1),
                                                       __builtin_bit_cast(bf16x8_t, gb[q]), g1b, 0, 0, 0);
      }
    }
  }
  // the four waves' gradients, added in wave order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float* rr = red + v * 64 + lane;
        rr[0] = (w ? rr[0] : 0.f) + g2[v];
        rr[16 * 64] = (w ? rr[16 * 64] : 0.f) + g1a[v];
        rr[32 * 64] = (w ? rr[32 * 64] : 0.f) + g1b[v];
      }
    }
    __syncthreads();
  }
  float* pb = part + (int64_t)blockIdx.x * NN_NP;
  for (int q = tid; q < 48 * 64; q += NN_THREADS) {
    const int blk = q >> 10, v = (q >> 6) & 15, l = q & 63;
    const int c = l & 31, o = 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
    if (o >= 27) continue;
    const float val = red[q];
    if (blk == 0) pb[NN_W1 + c * 27 + o] += val;
    else pb[c * 54 + (blk - 1) * 27 + o] += val;
  }
}

// grad[i] = scale * sum_b part[b][i] (fixed order, FP64 accumulation)
__global__ void nn_grad_reduce_kernel(const float* __restrict__ part, int nb, float scale,
                                      float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NN_NP) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += (double)part[(int64_t)b * NN_NP + i];
  grad[i] = (float)(s * scale);
}

__global__ void nn_fill_kernel(float* __restrict__ a, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// d = z - e
__global__ void nn_sub_kernel(const float* __restrict__ z, const float* __restrict__ e,
                              float* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = z[i] - e[i];
}

// g = 2 c Ad / den   (gradient of the loss with respect to z_L)
__global__ void nn_gout_kernel(const float* __restrict__ Ad, const uint8_t* __restrict__ mult,
                               const double* __restrict__ den, float* __restrict__ g, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = (float)(2.0 * (double)Ad[i] / ((double)mult[i] * den[0]));
}

// loss = (1/ns) sum_s num_s / den_s
__global__ void nn_loss_kernel(const double* __restrict__ nd, int ns, double* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < ns; ++q) s += nd[2 * q] / nd[2 * q + 1];
    loss[0] = s / ns;
  }
}

// Adam on the FP32 master weights; Wq receives the BF16-rounded copy
__global__ void nn_adam_kernel(float* __restrict__ W, float* __restrict__ Wq,
                               const float* __restrict__ g, float* __restrict__ m,
                               float* __restrict__ v, float lr, float b1, float b2, float eps,
                               float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NN_NP) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = W[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  W[i] = w;
  Wq[i] = bf16r(w);
}

// training pair: r32 = r64 / ||r64||_c, e32 = (xs - x) / ||r64||_c
__global__ void nn_pair_kernel(const double* __restrict__ r64, const double* __restrict__ xs,
                               const double* __restrict__ x, const double* __restrict__ rr,
                               float* __restrict__ r32, float* __restrict__ e32, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double inv = rr[0] > 0.0 ? 1.0 / sqrt(rr[0]) : 0.0;
  r32[i] = (float)(r64[i] * inv);
  e32[i] = (float)((xs[i] - x[i]) * inv);
}

__global__ void nn_round_kernel(const float* __restrict__ W, float* __restrict__ Wq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NN_NP) Wq[i] = bf16r(W[i]);
}

template <int N>
static size_t fwd_lds() {
  constexpr int n3 = (N + 1) * (N + 1) * (N + 1);
  return sizeof(float) * (2 * n3 + 27 * n3);
}
template <int N>
static size_t bwd_lds() {
  constexpr int n3 = (N + 1) * (N + 1) * (N + 1);
  return sizeof(float) * (2 * n3 + n3 + 8 * n3) + sizeof(bf16_t) * NN_CH * n3;
}

hipError_t launch_nn_fwd(int N, const float* r, const float* dinv, const uint8_t* mult,
                         const float* W1, const float* W2, float* zc, int E, hipStream_t s,
                         const State* st, const void* packed, NnDots dd, int* nparts) {
  if (N == 7) {
    // persistent: NN_FWD_WG_PER_CU workgroups per CU, each walking elements
    // blockIdx.x, +grid, ...
    int dev = 0, ncu = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    const int grid = std::min(E, NN_FWD_WG_PER_CU * std::max(ncu, 1));
    if (nparts) *nparts = grid;
    if (grid <= 0) return hipSuccess;
    if (dd.dots && grid > dd.dstride) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(nn_fwd_mfma_n8_kernel, dim3(grid), dim3(NN_THREADS), nnm::LDS_BYTES, s, r,
                       dinv, mult, (const bf16x8_t*)packed, zc, E, st, dd);
    return hipGetLastError();
  }
  // N = 3 and 5: one workgroup per element (N = 7 takes the matrix-core kernel above)
  if (nparts) *nparts = E;
  if (dd.dots && E > dd.dstride) return hipErrorInvalidConfiguration;
  switch (N) {
#define MX_NN(NN_)                                                                          \
  case NN_:                                                                                 \
    hipLaunchKernelGGL((nn_fwd_kernel<NN_>), dim3(E), dim3(NN_THREADS), fwd_lds<NN_>(), s, r, \
                       dinv, mult, W1, W2, zc, E, st, dd);                                  \
    break;
    MX_NN(3) MX_NN(5)
#undef MX_NN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nn_bwd(int N, const float* r, const float* dinv, const float* gzl,
                         const float* W1, const float* W2, const void* packed, float* part,
                         int nblocks, int E, hipStream_t s) {
  if (N == 7) {
    hipLaunchKernelGGL(nn_bwd_mfma_n8_kernel, dim3(nblocks), dim3(NN_THREADS), 0, s, r, dinv, gzl,
                       (const bf16x8_t*)packed + 6 * 64, part, E);
    return hipGetLastError();
  }
  // N = 3 and 5 (N = 7 takes the matrix-core kernel above)
  switch (N) {
#define MX_NN(NN_)                                                                           \
  case NN_:                                                                                  \
    hipLaunchKernelGGL((nn_bwd_kernel<NN_>), dim3(nblocks), dim3(NN_THREADS), bwd_lds<NN_>(), \
                       s, r, dinv, gzl, W1, W2, part, E);                                    \
    break;
    MX_NN(3) MX_NN(5)
#undef MX_NN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mx

using namespace mx;

struct mxsem_nn {
  mxsem_mesh* mesh = nullptr;
  int cin = NN_CIN, ch = NN_CH;
  float *W = nullptr, *Wq = nullptr, *grad = nullptr, *mo = nullptr, *ve = nullptr;
  float* part = nullptr;  // [NN_BWD_BLOCKS][NN_NP]
  void* packed = nullptr; // [12][64] BF16x8 weight operands of the matrix-core kernels
  float *z = nullptr, *d = nullptr, *Ad = nullptr, *g = nullptr;
  double* nd = nullptr;   // [2 * max samples] numerators / denominators
  double* dots = nullptr; // [5][dstride] per-workgroup flexible-CG dot partials of the forward
  int dstride = 0;
  int nd_cap = 0;         // max_samples of the descriptor
  int nbwd = 0;
  bool counted = false;
};

namespace mx {
// Blocks of a network's workspace: master and BF16-rounded weights,
// gradient, Adam moments, per-workgroup gradient partials of the backward,
// the forward's dot partials, the matrix-core weight operands, four FP32
// work vectors and the per-sample loss terms.  Returns the total; with ws,
// points nn's arrays at the blocks.
static size_t nn_layout(const mxsem_mesh* m, int max_samples, mxsem_nn* nn, char* ws) {
  Layout L;
  const int64_t nl = m->nloc;
  const int nbwd = std::min(NN_BWD_BLOCKS, m->E);
  const int dstride = std::max(m->E, 4096);  // at least every forward grid's workgroup count
  auto put = [&](auto** p, size_t bytes) {
    const size_t o = L.take(bytes);
    if (ws) *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(ws + o);
  };
  float* f = nullptr;
  double* dd = nullptr;
  void* v = nullptr;
  put(ws ? &nn->W : &f, sizeof(float) * NN_NP);
  put(ws ? &nn->Wq : &f, sizeof(float) * NN_NP);
  put(ws ? &nn->grad : &f, sizeof(float) * NN_NP);
  put(ws ? &nn->mo : &f, sizeof(float) * NN_NP);
  put(ws ? &nn->ve : &f, sizeof(float) * NN_NP);
  put(ws ? &nn->part : &f, sizeof(float) * NN_NP * nbwd);
  put(ws ? &nn->dots : &dd, sizeof(double) * 5 * dstride);
  put(ws ? &nn->packed : &v, 16 * 12 * 64);
  put(ws ? &nn->z : &f, sizeof(float) * nl);
  put(ws ? &nn->d : &f, sizeof(float) * nl);
  put(ws ? &nn->Ad : &f, sizeof(float) * nl);
  put(ws ? &nn->g : &f, sizeof(float) * nl);
  put(ws ? &nn->nd : &dd, sizeof(double) * 2 * max_samples);
  if (ws) {
    nn->nbwd = nbwd;
    nn->dstride = dstride;
    nn->nd_cap = max_samples;
  }
  return align256(L.total);
}

static int check_nn_desc(const mxsem_mesh* m, const mxsem_nn_desc* d) {
  MX_CHECK(d->cin == NN_CIN && d->ch == NN_CH, MXSEM_ENOTSUP,
           "nn: the network has 2 input and 32 hidden channels");
  MX_CHECK(d->max_samples >= 1, MXSEM_EINVAL, "nn: max_samples must be >= 1");
  MX_CHECK(m->N == 3 || m->N == 5 || m->N == 7, MXSEM_ENOTSUP,
           "nn: learned preconditioner built for N = 3, 5, 7");
  MX_CHECK(m->dinv32 && m->G32, MXSEM_ENOTSUP, "nn: mesh needs its FP32 view");
  return MXSEM_OK;
}
static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// zc = c z_L(r) (the caller's gather-scatter then gives z = M QQ^T zc);
// with w, also the partials of (r, z)_c and (z, w)_c: nn->dots, *nparts
// per dot, nn->dstride apart
int nn_launch_fwd(mxsem_nn* nn, const float* r, float* zc, hipStream_t s, const State* st,
                  const float* w, int* nparts, const double** dots, int* dstride, float* x,
                  const float* p) {
  if (x && !(w && p && st)) {
    set_error("nn forward: the fused vector update needs w, p and the state");
    return MXSEM_EINVAL;
  }
  mxsem_mesh* m = nn->mesh;
  NnDots dd{w, w ? nn->dots : nullptr, nn->dstride, x, p};
  MX_HIP(launch_nn_fwd(m->N, r, m->dinv32, m->mult, nn->Wq, nn->Wq + NN_W1, zc, m->E, s, st,
                       nn->packed, dd, nparts));
  if (dots) *dots = nn->dots;
  if (dstride) *dstride = nn->dstride;
  return MXSEM_OK;
}

int nn_forward_into(mxsem_nn* nn, const float* r, float* out, hipStream_t s) {
  mxsem_mesh* m = nn->mesh;
  MX_HIP(launch_nn_fwd(m->N, r, m->dinv32, m->mult, nn->Wq, nn->Wq + NN_W1, out, m->E, s,
                       nullptr, nn->packed, NnDots{nullptr, nullptr, 0, nullptr, nullptr}, nullptr));
  MX_HIP(launch_gs_apply(MXSEM_F32, MXSEM_F64, out, m->plan, true, s));
  return MXSEM_OK;
}
}  // namespace mx

extern "C" {

int mxsem_nn_workspace_bytes(const mxsem_mesh* m, const mxsem_nn_desc* d, size_t* bytes) {
  MX_API_BEGIN
  MX_CHECK(m && d && bytes, MXSEM_EINVAL, "nn_workspace_bytes: null argument");
  MX_TRY(check_nn_desc(m, d));
  *bytes = nn_layout(m, d->max_samples, nullptr, nullptr);
  return MXSEM_OK;
  MX_API_END("mxsem_nn_workspace_bytes")
}

int mxsem_nn_create(mxsem_mesh* m, const mxsem_nn_desc* d, void* workspace, size_t ws_bytes,
                    mxsem_nn** out) {
  MX_API_BEGIN
  MX_CHECK(m && d && out, MXSEM_EINVAL, "nn_create: null argument");
  *out = nullptr;
  MX_TRY(check_nn_desc(m, d));
  MX_CHECK(workspace && ((uintptr_t)workspace & 255) == 0, MXSEM_EINVAL,
           "nn_create: workspace must be a 256-byte aligned device pointer");
  MX_CHECK(ws_bytes >= nn_layout(m, d->max_samples, nullptr, nullptr), MXSEM_EINVAL,
           "nn_create: workspace smaller than mxsem_nn_workspace_bytes");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  std::unique_ptr<mxsem_nn> nn(new mxsem_nn());
  nn->mesh = m;
  nn_layout(m, d->max_samples, nn.get(), (char*)workspace);
  hipStream_t s = m->ctx->stream;
  for (float* p : {nn->W, nn->Wq, nn->grad, nn->mo, nn->ve})
    hipLaunchKernelGGL(nn_fill_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, p, (int64_t)NN_NP, 0.f);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(12 * 64), 0, s, nn->Wq, nn->Wq + NN_W1,
                     (bf16x8_t*)nn->packed);
  MX_HIP(hipGetLastError());
  MX_HIP(hipStreamSynchronize(s));
  m->ctx->live += 1;
  nn->counted = true;
  *out = nn.release();
  return MXSEM_OK;
  MX_API_END("mxsem_nn_create")
}

int mxsem_nn_destroy(mxsem_nn* nn) {
  MX_API_BEGIN
  if (!nn) return MXSEM_OK;
  (void)hipSetDevice(nn->mesh->ctx->device);
  if (nn->mesh->ctx->stream) (void)hipStreamSynchronize(nn->mesh->ctx->stream);
  else (void)hipDeviceSynchronize();
  if (nn->mesh->nn == nn) nn->mesh->nn = nullptr;
  if (nn->counted) nn->mesh->ctx->live -= 1;
  delete nn;  // the workspace is the caller's
  return MXSEM_OK;
  MX_API_END("mxsem_nn_destroy")
}

int mxsem_nn_set_params(mxsem_nn* nn, const float* W1, const float* W2) {
  MX_API_BEGIN
  MX_CHECK(nn && W1 && W2, MXSEM_EINVAL, "nn_set_params: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  hipStream_t s = nn->mesh->ctx->stream;
  MX_HIP(hipMemcpyAsync(nn->W, W1, sizeof(float) * NN_W1, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(nn->W + NN_W1, W2, sizeof(float) * NN_W2, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(nn_round_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, nn->W, nn->Wq);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(12 * 64), 0, s, nn->Wq, nn->Wq + NN_W1,
                     (bf16x8_t*)nn->packed);
  for (float* p : {nn->mo, nn->ve})
    hipLaunchKernelGGL(nn_fill_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, p, (int64_t)NN_NP, 0.f);
  MX_HIP(hipGetLastError());
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
  MX_API_END("mxsem_nn_set_params")
}

int mxsem_nn_get_params(mxsem_nn* nn, float* W1, float* W2) {
  MX_API_BEGIN
  MX_CHECK(nn && W1 && W2, MXSEM_EINVAL, "nn_get_params: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  hipStream_t s = nn->mesh->ctx->stream;
  MX_HIP(hipMemcpyAsync(W1, nn->W, sizeof(float) * NN_W1, hipMemcpyDeviceToHost, s));
  MX_HIP(hipMemcpyAsync(W2, nn->W + NN_W1, sizeof(float) * NN_W2, hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
  MX_API_END("mxsem_nn_get_params")
}

int mxsem_nn_forward(mxsem_nn* nn, const float* r, float* z) {
  MX_API_BEGIN
  MX_CHECK(nn && r && z, MXSEM_EINVAL, "nn_forward: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  (void)hipGetLastError();
  return nn_forward_into(nn, r, z, nn->mesh->ctx->stream);
  MX_API_END("mxsem_nn_forward")
}

int mxsem_nn_loss_grad(mxsem_nn* nn, const float* r, const float* e, int nsamp, double* loss_dev,
                       float* grad_dev) {
  MX_API_BEGIN
  MX_CHECK(nn && r && e && nsamp >= 1 && loss_dev, MXSEM_EINVAL, "nn_loss_grad: bad argument");
  mxsem_mesh* m = nn->mesh;
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  hipStream_t s = m->ctx->stream;
  const int64_t nl = m->nloc;
  MX_CHECK(nsamp <= nn->nd_cap, MXSEM_EINVAL,
           "nn_loss_grad: more samples than the network's max_samples");
  hipLaunchKernelGGL(nn_fill_kernel, dim3(nb256((int64_t)NN_NP * nn->nbwd)), dim3(256), 0, s,
                     nn->part, (int64_t)NN_NP * nn->nbwd, 0.f);
  for (int q = 0; q < nsamp; ++q) {
    const float* rq = r + (int64_t)q * nl;
    const float* eq = e + (int64_t)q * nl;
    MX_TRY(nn_forward_into(nn, rq, nn->z, s));
    hipLaunchKernelGGL(nn_sub_kernel, dim3(nb256(nl)), dim3(256), 0, s, nn->z, eq, nn->d, nl);
    MX_TRY(apply_impl(m, MXSEM_F32, nn->d, nn->Ad, 0, s));
    MX_HIP(launch_dot(MXSEM_F32, nn->d, nn->Ad, m->mult, nl, m->part, nn->nd + 2 * q, s));
    MX_TRY(apply_impl(m, MXSEM_F32, eq, nn->g, 0, s));
    MX_HIP(launch_dot(MXSEM_F32, eq, nn->g, m->mult, nl, m->part, nn->nd + 2 * q + 1, s));
    hipLaunchKernelGGL(nn_gout_kernel, dim3(nb256(nl)), dim3(256), 0, s, nn->Ad, m->mult,
                       nn->nd + 2 * q + 1, nn->g, nl);
    MX_HIP(launch_nn_bwd(m->N, rq, m->dinv32, nn->g, nn->Wq, nn->Wq + NN_W1, nn->packed, nn->part, nn->nbwd,
                         m->E, s));
  }
  hipLaunchKernelGGL(nn_grad_reduce_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, nn->part,
                     nn->nbwd, 1.0f / nsamp, nn->grad);
  hipLaunchKernelGGL(nn_loss_kernel, dim3(1), dim3(64), 0, s, nn->nd, nsamp, loss_dev);
  MX_HIP(hipGetLastError());
  if (grad_dev)
    MX_HIP(hipMemcpyAsync(grad_dev, nn->grad, sizeof(float) * NN_NP, hipMemcpyDeviceToDevice, s));
  return MXSEM_OK;
  MX_API_END("mxsem_nn_loss_grad")
}

int mxsem_nn_adam_step(mxsem_nn* nn, const mxsem_adam* o) {
  MX_API_BEGIN
  MX_CHECK(nn && o && o->step >= 1, MXSEM_EINVAL, "nn_adam_step: bad argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  (void)hipGetLastError();
  const float c1 = (float)(1.0 - pow(o->beta1, o->step));
  const float c2 = (float)(1.0 - pow(o->beta2, o->step));
  hipLaunchKernelGGL(nn_adam_kernel, dim3(nb256(NN_NP)), dim3(256), 0, nn->mesh->ctx->stream,
                     nn->W, nn->Wq, nn->grad, nn->mo, nn->ve, (float)o->lr, (float)o->beta1,
                     (float)o->beta2, (float)o->eps, c1, c2);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(12 * 64), 0, nn->mesh->ctx->stream, nn->Wq,
                     nn->Wq + NN_W1, (bf16x8_t*)nn->packed);
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
  MX_API_END("mxsem_nn_adam_step")
}

int mxsem_nn_make_pair(mxsem_mesh* m, const double* b, const double* x, const double* xstar,
                       float* r_out, float* e_out) {
  MX_API_BEGIN
  MX_CHECK(m && b && x && xstar && r_out && e_out, MXSEM_EINVAL, "nn_make_pair: null argument");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  hipStream_t s = m->ctx->stream;
  MX_TRY(apply_impl(m, MXSEM_F64, x, m->tmpb, 0, s));
  MX_HIP(launch_residual(b, m->tmpb, m->tmpa, m->mult, m->nloc, m->part, m->scal + 2, s));
  hipLaunchKernelGGL(nn_pair_kernel, dim3(nb256(m->nloc)), dim3(256), 0, s, m->tmpa, xstar, x,
                     m->scal + 2, r_out, e_out, m->nloc);
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
  MX_API_END("mxsem_nn_make_pair")
}

int mxsem_mesh_attach_nn(mxsem_mesh* m, mxsem_nn* nn) {
  MX_API_BEGIN
  MX_CHECK(m, MXSEM_EINVAL, "mesh_attach_nn: null mesh");
  MX_CHECK(!nn || nn->mesh == m, MXSEM_EINVAL, "mesh_attach_nn: network built for another mesh");
  m->nn = nn;
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_attach_nn")
}

}  // extern "C"
