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
// elements: forward recomputed in LDS, then every thread accumulates the
// gradient entries it owns over all positions and elements; one partial per
// workgroup, summed in a fixed order afterwards (deterministic, no atomics).
#include <math.h>
#include <string.h>

#include <algorithm>
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
                  const State* __restrict__ st) {
  constexpr int n = N + 1, n3 = n * n * n, PPT = (n3 + NN_THREADS - 1) / NN_THREADS;
  extern __shared__ float sm[];
  float* x0 = sm;           // [2][n3]
  float* T = sm + 2 * n3;   // [n3][27]
  __shared__ float sred[8];
  const int e = blockIdx.x;
  if (e >= E || (st && st->done)) return;
  const int64_t base = (int64_t)e * n3;
  float rv[PPT], dv[PPT];
  float ss = 0.f;
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
    zc[base + p] = m == 1 ? zl : zl / (float)m;
  }
}

// Forward for N = 7 on the matrix cores (gfx950 v_mfma_f32_32x32x16_bf16),
// both layers as small GEMMs over the 512 positions of an element, computed
// transposed so that positions run along the result columns:
//   layer 1: H[c][p] = relu(sum_k W1[c][k] X[k][p]),  k = (tap, ci), K = 64
//   layer 2: T[o][p] = sum_c W2[c][o] H[c][p],         27 taps -> 32 rows
//   y[p]     = sum_o T[o][p + d_o]                     (zero outside)
// Operand layout of the instruction (lane l, h = l/32): A row l%32 and
// B column l%32, with k = 8h + t; result column l%32, rows
// 8(v/4) + 4h + v%4.  The first layer's result is therefore already the
// second layer's B operand in the same lane (the channel order inside K is
// absorbed into the packed W2), so the hidden tile never leaves registers.
//
// LDS: X holds (x0, x1) as one BF16 pair per position in a zero-bordered
// 10^3 grid, so every im2col operand is four 32-bit loads at fixed offsets.
// T is written scattered, T[o][q] to slot q - d_o of tap o's plane; each
// plane is a 9^3 (or smaller) box with row stride 9 and layer stride 81
// whose slots outside the element are written but never read, and whose
// in-element slots that no position writes (the convolution's zero padding)
// are cleared once per workgroup.  The sum over taps is then 27 loads at
// fixed offsets per position.  75.5 KB + 4 KB keeps two workgroups per CU.
// Workgroups are persistent over elements.  Same roundings as the vector
// kernel: BF16 inputs, weights and h; FP32 accumulation; y summed in tap
// order.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

namespace nnm {
constexpr int XP = 10;                  // bordered grid edge
constexpr int XWORDS = XP * XP * XP;    // 1000
constexpr int tdx(int o) { return o % 3 - 1; }
constexpr int tdy(int o) { return (o / 3) % 3 - 1; }
constexpr int tdz(int o) { return o / 9 - 1; }
constexpr int ext(int d) { return d != 0 ? 8 : 7; }  // slot span hi - lo per direction
constexpr int lo(int d) { return d > 0 ? -1 : 0; }
constexpr int pmap(int i, int j, int k) { return i + 9 * j + 81 * k; }
constexpr int plane_size(int o) {
  return 1 + ext(tdx(o)) + 9 * ext(tdy(o)) + 81 * ext(tdz(o));
}
// second-layer result slot -> tap (slots 26, 27, 29, 30, 31 are padding)
constexpr int slot_tap(int s) { return s < 26 ? s : (s == 28 ? 26 : -1); }
struct Tables {
  int rof[27];  // read offset of tap o for position p: rof[o] + pmap(p)
  int wof[27];  // write offset of tap o for source position q: wof[o] + pmap(q)
  int size;     // words of all planes
  constexpr Tables() : rof(), wof(), size(0) {
    int b = 0;
    for (int o = 0; o < 27; ++o) {
      rof[o] = b - pmap(lo(tdx(o)), lo(tdy(o)), lo(tdz(o)));
      wof[o] = rof[o] - pmap(tdx(o), tdy(o), tdz(o));
      b += plane_size(o);
    }
    size = b;
  }
};
constexpr Tables TB{};
constexpr int UWORDS = TB.size;
constexpr int LDS_BYTES = 4 * (XWORDS + UWORDS);
static_assert(UWORDS == 18864, "tap planes");
}  // namespace nnm

// Weight operands in the per-lane A layout, packed once per weight update:
// pk[ks * 64 + lane] for the 4 first-layer and then 2 second-layer k steps.
// First layer: row = channel, k = 16 ks + 8h + 2u + ci <-> tap 8 ks + 4h + u.
// Second layer: row = result slot, k = 16 ks + 8h + t <-> channel
// 16 ks + 8(t/4) + 4h + t%4 (the first layer's result rows in that lane).
__global__ void nn_pack_kernel(const float* __restrict__ W1, const float* __restrict__ W2,
                               bf16x8_t* __restrict__ pk) {
  const int lane = threadIdx.x & 63, ks = threadIdx.x >> 6;  // 6 x 64 threads
  const int row = lane & 31, h = lane >> 5;
  bf16x8_t v;
  for (int t = 0; t < 8; ++t) {
    if (ks < 4) {
      const int tap = 8 * ks + 4 * h + (t >> 1), ci = t & 1;
      v[t] = (__bf16)(tap < 27 ? W1[row * 54 + ci * 27 + tap] : 0.f);
    } else {
      const int c = 16 * (ks - 4) + 8 * (t >> 2) + 4 * h + (t & 3);
      const int tap = nnm::slot_tap(row);
      v[t] = (__bf16)(tap >= 0 ? W2[c * 27 + tap] : 0.f);
    }
  }
  pk[ks * 64 + lane] = v;
}

__device__ inline unsigned pack_bf16x2(float lo_, float hi_) {
  return (unsigned)float_to_bf16(lo_) | ((unsigned)float_to_bf16(hi_) << 16);
}

__global__ void __launch_bounds__(NN_THREADS, 2)
    nn_fwd_mfma_n8_kernel(const float* __restrict__ r, const float* __restrict__ dinv,
                          const uint8_t* __restrict__ mult, const bf16x8_t* __restrict__ pk,
                          float* __restrict__ zc, int E, const State* __restrict__ st) {
  using namespace nnm;
  constexpr int n3 = 512;
  extern __shared__ float sm[];
  unsigned* X = (unsigned*)sm;  // [10][10][10] BF16 pairs
  float* U = sm + XWORDS;       // tap planes
  __shared__ float sred[8];
  if (st && st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31;
  // clear both buffers once: borders of X and never-written slots of U stay 0
  for (int q = tid; q < XWORDS + UWORDS; q += NN_THREADS) sm[q] = 0.f;
  // weight operands (identical for every element)
  bf16x8_t a1[4], a2[2];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) a1[ks] = pk[ks * 64 + lane];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) a2[ks] = pk[(4 + ks) * 64 + lane];
  // this lane's first tile (tile 4*wave): i = c%8, j = c/8, k = 2*wave
  const int ci_ = c & 7, cj = c >> 3, ck = 2 * wave;
  const int xq = (ci_ + 1) + XP * (cj + 1) + XP * XP * (ck + 1);
  int xa[4][4];  // im2col load address per (k step, tap quad)
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tap = 8 * ks + 4 * h + u;
      xa[ks][u] = xq + (tap < 27 ? tdx(tap) + XP * tdy(tap) + XP * XP * tdz(tap) : 0);
    }
  const int uq = XWORDS + pmap(ci_, cj, ck);
  int wa[14];  // T store address per result register (v = 13: h = 0 only)
#pragma unroll
  for (int v = 0; v < 14; ++v) {
    const int s0 = 8 * (v >> 2) + (v & 3);
    const int t0 = slot_tap(s0), t1 = slot_tap(s0 + 4);
    wa[v] = uq + (h ? (t1 >= 0 ? TB.wof[t1] : 0) : TB.wof[t0]);
  }
  // positions of the sum over taps: p = tid and tid + 256
  const int pi = tid & 7, pj = (tid >> 3) & 7, pk0 = tid >> 6;
  const int ur = XWORDS + pmap(pi, pj, pk0);
  const int xw = (pi + 1) + XP * (pj + 1) + XP * XP * (pk0 + 1);
  __syncthreads();

  for (int e = blockIdx.x; e < E; e += gridDim.x) {
    const int64_t base = (int64_t)e * n3;
    float rv[2], dv[2];
    float ss = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      rv[q] = r[base + tid + q * NN_THREADS];
      dv[q] = dinv[base + tid + q * NN_THREADS] * rv[q];
      ss += dv[q] * dv[q];
    }
    const float s = sqrtf(block_sum_bcast(ss, sred));
    const float inv = s > 0.f ? 1.f / s : 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) X[xw + q * 4 * XP * XP] = pack_bf16x2(rv[q] * inv, dv[q] * inv);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int xs = XP * XP * (mt >> 1) + 4 * XP * (mt & 1);  // tile shift in X
      const int us = 81 * (mt >> 1) + 36 * (mt & 1);           // tile shift in pmap
      floatx16_t acc = {0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        u32x4_t w;
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = X[xa[ks][u] + xs];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[ks], __builtin_bit_cast(bf16x8_t, w),
                                                      acc, 0, 0, 0);
      }
      bf16x8_t hb[2];
#pragma unroll
      for (int v = 0; v < 16; ++v) hb[v >> 3][v & 7] = (__bf16)fmaxf(acc[v], 0.f);
      floatx16_t acc2 = {0};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
        acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[ks], hb[ks], acc2, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 13; ++v) U[wa[v] - XWORDS + us] = acc2[v];
      if (h == 0) U[wa[13] - XWORDS + us] = acc2[13];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = tid + q * NN_THREADS;
      const float* up = U + (ur - XWORDS) + q * 4 * 81;
      float y = 0.f;
#pragma unroll
      for (int o = 0; o < 27; ++o) y += up[TB.rof[o]];
      const float zl = dv[q] + s * y;
      const uint8_t m = mult[base + p];
      zc[base + p] = m == 1 ? zl : zl / (float)m;
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
                         const State* st, const void* packed) {
  if (N == 7) {
    // persistent: two workgroups per CU, each walking elements blockIdx.x, +grid, ...
    int dev = 0, ncu = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess) err = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    const int grid = std::min(E, 2 * std::max(ncu, 1));
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn_fwd_mfma_n8_kernel, dim3(grid), dim3(NN_THREADS), nnm::LDS_BYTES, s, r,
                       dinv, mult, (const bf16x8_t*)packed, zc, E, st);
    return hipGetLastError();
  }
  switch (N) {
#define MX_NN(NN_)                                                                          \
  case NN_:                                                                                 \
    hipLaunchKernelGGL((nn_fwd_kernel<NN_>), dim3(E), dim3(NN_THREADS), fwd_lds<NN_>(), s, r, \
                       dinv, mult, W1, W2, zc, E, st);                                      \
    break;
    MX_NN(3) MX_NN(5) MX_NN(7)
#undef MX_NN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nn_bwd(int N, const float* r, const float* dinv, const float* gzl,
                         const float* W1, const float* W2, float* part, int nblocks, int E,
                         hipStream_t s) {
  switch (N) {
#define MX_NN(NN_)                                                                           \
  case NN_:                                                                                  \
    hipLaunchKernelGGL((nn_bwd_kernel<NN_>), dim3(nblocks), dim3(NN_THREADS), bwd_lds<NN_>(), \
                       s, r, dinv, gzl, W1, W2, part, E);                                    \
    break;
    MX_NN(3) MX_NN(5) MX_NN(7)
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
  void* packed = nullptr; // [6][64] BF16x8 weight operands of the matrix-core forward
  float *z = nullptr, *d = nullptr, *Ad = nullptr, *g = nullptr;
  double* nd = nullptr;   // [2 * max samples] numerators / denominators
  int nd_cap = 0;
  int nbwd = 0;
  std::vector<void*> allocs;
};

namespace mx {
static int nn_alloc(mxsem_nn* nn, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 256);
  if (e != hipSuccess) {
    set_error(std::string("nn: hipMalloc: ") + hipGetErrorString(e));
    return MXSEM_ENOMEM;
  }
  nn->allocs.push_back(*p);
  return MXSEM_OK;
}
static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// z = M QQ^T (c z_L(r)) into out (FP32)
int nn_launch_fwd(mxsem_nn* nn, const float* r, float* zc, hipStream_t s, const State* st) {
  mxsem_mesh* m = nn->mesh;
  MX_HIP(launch_nn_fwd(m->N, r, m->dinv32, m->mult, nn->Wq, nn->Wq + NN_W1, zc, m->E, s, st,
                       nn->packed));
  return MXSEM_OK;
}

int nn_forward_into(mxsem_nn* nn, const float* r, float* out, hipStream_t s) {
  mxsem_mesh* m = nn->mesh;
  MX_HIP(launch_nn_fwd(m->N, r, m->dinv32, m->mult, nn->Wq, nn->Wq + NN_W1, out, m->E, s,
                       nullptr, nn->packed));
  MX_HIP(launch_gs_apply(MXSEM_F32, MXSEM_F64, out, m->plan, true, s));
  return MXSEM_OK;
}
}  // namespace mx

extern "C" {

int mxsem_nn_create(mxsem_mesh* m, const mxsem_nn_desc* d, mxsem_nn** out) {
  MX_CHECK(m && d && out, MXSEM_EINVAL, "nn_create: null argument");
  MX_CHECK(d->cin == NN_CIN && d->ch == NN_CH, MXSEM_ENOTSUP,
           "nn_create: the network has 2 input and 32 hidden channels");
  MX_CHECK(m->N == 3 || m->N == 5 || m->N == 7, MXSEM_ENOTSUP,
           "nn_create: learned preconditioner built for N = 3, 5, 7");
  MX_CHECK(m->dinv32 && m->G32, MXSEM_ENOTSUP, "nn_create: mesh needs its FP32 view");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  *out = nullptr;
  mxsem_nn* nn = new mxsem_nn();
  nn->mesh = m;
  nn->nbwd = std::min(NN_BWD_BLOCKS, m->E);
  const int64_t nl = m->nloc;
  int rc = MXSEM_OK;
  auto A = [&](void** p, size_t b) {
    if (rc == MXSEM_OK) rc = nn_alloc(nn, p, b);
  };
  A((void**)&nn->W, sizeof(float) * NN_NP);
  A((void**)&nn->Wq, sizeof(float) * NN_NP);
  A((void**)&nn->grad, sizeof(float) * NN_NP);
  A((void**)&nn->mo, sizeof(float) * NN_NP);
  A((void**)&nn->ve, sizeof(float) * NN_NP);
  A((void**)&nn->part, sizeof(float) * NN_NP * nn->nbwd);
  A((void**)&nn->packed, 16 * 6 * 64);
  A((void**)&nn->z, sizeof(float) * nl);
  A((void**)&nn->d, sizeof(float) * nl);
  A((void**)&nn->Ad, sizeof(float) * nl);
  A((void**)&nn->g, sizeof(float) * nl);
  if (rc != MXSEM_OK) {
    mxsem_nn_destroy(nn);
    return rc;
  }
  hipStream_t s = m->ctx->stream;
  for (float* p : {nn->W, nn->Wq, nn->grad, nn->mo, nn->ve})
    hipLaunchKernelGGL(nn_fill_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, p, (int64_t)NN_NP, 0.f);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(6 * 64), 0, s, nn->Wq, nn->Wq + NN_W1,
                     (bf16x8_t*)nn->packed);
  MX_HIP(hipGetLastError());
  MX_HIP(hipStreamSynchronize(s));
  m->ctx->live += 1;
  *out = nn;
  return MXSEM_OK;
}

int mxsem_nn_destroy(mxsem_nn* nn) {
  if (!nn) return MXSEM_OK;
  hipSetDevice(nn->mesh->ctx->device);
  if (nn->mesh->ctx->stream) hipStreamSynchronize(nn->mesh->ctx->stream);
  else hipDeviceSynchronize();
  if (nn->mesh->nn == nn) nn->mesh->nn = nullptr;
  for (void* p : nn->allocs) hipFree(p);
  if (nn->W) nn->mesh->ctx->live -= 1;
  delete nn;
  return MXSEM_OK;
}

int mxsem_nn_set_params(mxsem_nn* nn, const float* W1, const float* W2) {
  MX_CHECK(nn && W1 && W2, MXSEM_EINVAL, "nn_set_params: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  hipStream_t s = nn->mesh->ctx->stream;
  MX_HIP(hipMemcpyAsync(nn->W, W1, sizeof(float) * NN_W1, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(nn->W + NN_W1, W2, sizeof(float) * NN_W2, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(nn_round_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, nn->W, nn->Wq);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(6 * 64), 0, s, nn->Wq, nn->Wq + NN_W1,
                     (bf16x8_t*)nn->packed);
  for (float* p : {nn->mo, nn->ve})
    hipLaunchKernelGGL(nn_fill_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, p, (int64_t)NN_NP, 0.f);
  MX_HIP(hipGetLastError());
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
}

int mxsem_nn_get_params(mxsem_nn* nn, float* W1, float* W2) {
  MX_CHECK(nn && W1 && W2, MXSEM_EINVAL, "nn_get_params: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  hipStream_t s = nn->mesh->ctx->stream;
  MX_HIP(hipMemcpyAsync(W1, nn->W, sizeof(float) * NN_W1, hipMemcpyDeviceToHost, s));
  MX_HIP(hipMemcpyAsync(W2, nn->W + NN_W1, sizeof(float) * NN_W2, hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
}

int mxsem_nn_forward(mxsem_nn* nn, const float* r, float* z) {
  MX_CHECK(nn && r && z, MXSEM_EINVAL, "nn_forward: null argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  (void)hipGetLastError();
  return nn_forward_into(nn, r, z, nn->mesh->ctx->stream);
}

int mxsem_nn_loss_grad(mxsem_nn* nn, const float* r, const float* e, int nsamp, double* loss_dev,
                       float* grad_dev) {
  MX_CHECK(nn && r && e && nsamp >= 1 && loss_dev, MXSEM_EINVAL, "nn_loss_grad: bad argument");
  mxsem_mesh* m = nn->mesh;
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  hipStream_t s = m->ctx->stream;
  const int64_t nl = m->nloc;
  if (nn->nd_cap < nsamp) {
    MX_TRY(nn_alloc(nn, (void**)&nn->nd, sizeof(double) * 2 * nsamp));
    nn->nd_cap = nsamp;
  }
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
    MX_HIP(launch_nn_bwd(m->N, rq, m->dinv32, nn->g, nn->Wq, nn->Wq + NN_W1, nn->part, nn->nbwd,
                         m->E, s));
  }
  hipLaunchKernelGGL(nn_grad_reduce_kernel, dim3(nb256(NN_NP)), dim3(256), 0, s, nn->part,
                     nn->nbwd, 1.0f / nsamp, nn->grad);
  hipLaunchKernelGGL(nn_loss_kernel, dim3(1), dim3(64), 0, s, nn->nd, nsamp, loss_dev);
  MX_HIP(hipGetLastError());
  if (grad_dev)
    MX_HIP(hipMemcpyAsync(grad_dev, nn->grad, sizeof(float) * NN_NP, hipMemcpyDeviceToDevice, s));
  return MXSEM_OK;
}

int mxsem_nn_adam_step(mxsem_nn* nn, const mxsem_adam* o) {
  MX_CHECK(nn && o && o->step >= 1, MXSEM_EINVAL, "nn_adam_step: bad argument");
  MX_HIP(hipSetDevice(nn->mesh->ctx->device));
  (void)hipGetLastError();
  const float c1 = (float)(1.0 - pow(o->beta1, o->step));
  const float c2 = (float)(1.0 - pow(o->beta2, o->step));
  hipLaunchKernelGGL(nn_adam_kernel, dim3(nb256(NN_NP)), dim3(256), 0, nn->mesh->ctx->stream,
                     nn->W, nn->Wq, nn->grad, nn->mo, nn->ve, (float)o->lr, (float)o->beta1,
                     (float)o->beta2, (float)o->eps, c1, c2);
  hipLaunchKernelGGL(nn_pack_kernel, dim3(1), dim3(6 * 64), 0, nn->mesh->ctx->stream, nn->Wq,
                     nn->Wq + NN_W1, (bf16x8_t*)nn->packed);
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
}

int mxsem_nn_make_pair(mxsem_mesh* m, const double* b, const double* x, const double* xstar,
                       float* r_out, float* e_out) {
  MX_CHECK(m && b && x && xstar && r_out && e_out, MXSEM_EINVAL, "nn_make_pair: null argument");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  hipStream_t s = m->ctx->stream;
  MX_TRY(ensure_tmp(m));
  MX_TRY(apply_impl(m, MXSEM_F64, x, m->tmpb, 0, s));
  MX_HIP(launch_residual(b, m->tmpb, m->tmpa, m->mult, m->nloc, m->part, m->scal + 2, s));
  hipLaunchKernelGGL(nn_pair_kernel, dim3(nb256(m->nloc)), dim3(256), 0, s, m->tmpa, xstar, x,
                     m->scal + 2, r_out, e_out, m->nloc);
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
}

int mxsem_mesh_attach_nn(mxsem_mesh* m, mxsem_nn* nn) {
  MX_CHECK(m, MXSEM_EINVAL, "mesh_attach_nn: null mesh");
  MX_CHECK(!nn || nn->mesh == m, MXSEM_EINVAL, "mesh_attach_nn: network built for another mesh");
  m->nn = nn;
  return MXSEM_OK;
}

}  // extern "C"
