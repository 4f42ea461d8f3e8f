// Local spectral-element operator  w_L = sum_ab D_a^T diag(G_ab) D_b u_L + h B u_L
// on hexahedra of order N (the "ax" kernel of the CG loop: local_grad3, the
// geometric-factor multiply and local_grad3_t, Sec. 4.1, CG-loop profiling
// table and its footnote on mxm and accumulations).
//
// Mapping for gfx950: one thread per (i,j) column of an element, n^2
// threads per element, several elements per workgroup (tile size epb),
// workgroup rounded up to whole wave64s.  Each thread keeps its u column
// and the w accumulator column (length n) in registers; the t-direction
// derivative and its transpose therefore never touch LDS.  For each k the
// (i,j) slab of u is staged in LDS for the r/s derivatives, and the slabs
// of G-multiplied r/s components are staged for the transposed sums.
// Global traffic per local dof: u in, six G values in, w out (plus, in the
// solver variant, z in and p in/out for the fused p update) - each a fully
// coalesced n^2-wide stream per k.
#include <hip/hip_ext.h>

#include "common.hpp"

namespace mx {

struct AxApplyArgs {
  const void* u;
  void* w;
  const void* G;
  const void* hB;
  const void* D;
  int E;
};

// Solver variant: p = z + beta p_old (beta from the device state, p
// written back), w = A_L p, and the workgroup's partial sum of p.w.
template <int N, typename T, typename TG, bool SOLVER>
__global__ void __launch_bounds__(256) ax_kernel(const Tile* __restrict__ tiles, const ProbDev* __restrict__ probs,
                          AxApplyArgs apply, int epb) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sD = reinterpret_cast<T*>(smem_raw);
  T* slab = sD + n2;
  __shared__ double sred[16];

  const T* __restrict__ Dg;
  const TG* __restrict__ G;
  const TG* __restrict__ hB;
  const T* __restrict__ U;
  T* __restrict__ Wout;
  const T* __restrict__ Z = nullptr;
  int E, first;
  const ProbDev* P = nullptr;
  if constexpr (SOLVER) {
    const Tile t = tiles[blockIdx.x];
    P = &probs[t.prob];
    if (P->st->done) return;  // uniform across the workgroup
    Dg = (const T*)P->D;
    G = (const TG*)P->G;
    hB = (const TG*)P->hB;
    U = (const T*)P->p;
    Wout = (T*)P->w;
    Z = (const T*)P->z;
    E = P->E;
    first = t.first;
  } else {
    Dg = (const T*)apply.D;
    G = (const TG*)apply.G;
    hB = (const TG*)apply.hB;
    U = (const T*)apply.u;
    Wout = (T*)apply.w;
    E = apply.E;
    first = blockIdx.x * epb;
  }

  const int tid = threadIdx.x;
  for (int q = tid; q < n2; q += blockDim.x) sD[q] = Dg[q];
  const int le = tid / n2;
  const int ij = tid - le * n2;
  const int i = ij % n, j = ij / n;
  const int e = first + le;
  const bool active = (le < epb) && (e < E);
  T* su = slab + le * 3 * n2;
  T* sr = su + n2;
  T* ss = sr + n2;
  __syncthreads();

  T u[n], w[n], Di[n], Dj[n], DiT[n], DjT[n];
#pragma unroll
  for (int l = 0; l < n; ++l) {
    Di[l] = sD[i * n + l];
    Dj[l] = sD[j * n + l];
    DiT[l] = sD[l * n + i];
    DjT[l] = sD[l * n + j];
    w[l] = T(0);
  }
  const int64_t base = (int64_t)e * n3 + ij;
  if (active) {
    if constexpr (SOLVER) {
      const T beta = (T)P->st->beta;
      T* __restrict__ Pw = (T*)P->p;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        T pv = Z[base + k * n2] + beta * U[base + k * n2];
        Pw[base + k * n2] = pv;
        u[k] = pv;
      }
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) u[k] = U[base + k * n2];
    }
  } else {
#pragma unroll
    for (int k = 0; k < n; ++k) u[k] = T(0);
  }

  // Geometric factors of the whole column: loaded before the k loop when
  // they fit in registers, so every load of the element is in flight at
  // once (the workgroup barriers inside the loop would otherwise serialise
  // one HBM round trip per k).
  const TG* __restrict__ Ge = G + (int64_t)e * 6 * n3 + ij;
  constexpr bool PREFETCH = 6 * n * sizeof(T) <= 512;
  T gpre[PREFETCH ? 6 * n : 1];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int k = 0; k < n; ++k)
#pragma unroll
      for (int q = 0; q < 6; ++q)
        gpre[q * n + k] = active ? cvt<T>(Ge[q * n3 + k * n2]) : T(0);
  }
#pragma unroll
  for (int k = 0; k < n; ++k) {
    if (active) su[ij] = u[k];
    __syncthreads();
    if (active) {
      T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        ur += Di[l] * su[j * n + l];
        us += Dj[l] * su[l * n + i];
        ut += sD[k * n + l] * u[l];
      }
      const int off = k * n2;
      T g0, g1, g2, g3, g4, g5;
      if constexpr (PREFETCH) {
        g0 = gpre[0 * n + k];
        g1 = gpre[1 * n + k];
        g2 = gpre[2 * n + k];
        g3 = gpre[3 * n + k];
        g4 = gpre[4 * n + k];
        g5 = gpre[5 * n + k];
      } else {
        g0 = cvt<T>(Ge[0 * n3 + off]);
        g1 = cvt<T>(Ge[1 * n3 + off]);
        g2 = cvt<T>(Ge[2 * n3 + off]);
        g3 = cvt<T>(Ge[3 * n3 + off]);
        g4 = cvt<T>(Ge[4 * n3 + off]);
        g5 = cvt<T>(Ge[5 * n3 + off]);
      }
      const T wr = g0 * ur + g1 * us + g2 * ut;
      const T ws = g1 * ur + g3 * us + g4 * ut;
      const T wt = g2 * ur + g4 * us + g5 * ut;
#pragma unroll
      for (int m = 0; m < n; ++m) w[m] += sD[k * n + m] * wt;
      sr[ij] = wr;
      ss[ij] = ws;
    }
    __syncthreads();
    if (active) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) acc += DiT[l] * sr[j * n + l] + DjT[l] * ss[l * n + i];
      w[k] += acc;
    }
    __syncthreads();
  }

  // (p, QQ^T A_L p)_c = sum_i p_i (A_L p)_i over all local entries, because
  // p is continuous and zero on Dirichlet nodes: the solver takes sigma
  // from the local result, before the gather-scatter.
  double dot = 0.0;
  if (active) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T wv = w[k];
      if (hB) wv += cvt<T>(hB[(int64_t)e * n3 + k * n2 + ij]) * u[k];
      Wout[base + k * n2] = wv;
      if constexpr (SOLVER) dot += (double)u[k] * (double)wv;
    }
  }
  if constexpr (SOLVER) {
    double s = block_sum(dot, sred);
    if (tid == 0) P->part_ax[first / epb] = s;
  }
}

// With ev0/ev1 the launch records its own start and end (hipExtLaunchKernel),
// so the elapsed time between them is the kernel's execution time.
template <int N, typename T, typename TG, bool SOLVER>
static hipError_t launch_one(const Tile* tiles, const ProbDev* probs, const AxApplyArgs& a,
                             int ntiles, int epb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int n = N + 1, n2 = n * n;
  int threads = ((epb * n2 + 63) / 64) * 64;
  if (epb < 1 || threads > 256) return hipErrorInvalidConfiguration;
  size_t shm = sizeof(T) * (n2 + (size_t)epb * 3 * n2);
  if (ev0)
    hipExtLaunchKernelGGL((ax_kernel<N, T, TG, SOLVER>), dim3(ntiles), dim3(threads), (uint32_t)shm,
                          s, ev0, ev1, 0, tiles, probs, a, epb);
  else
    hipLaunchKernelGGL((ax_kernel<N, T, TG, SOLVER>), dim3(ntiles), dim3(threads), shm, s, tiles,
                       probs, a, epb);
  return hipGetLastError();
}

template <typename T, typename TG, bool SOLVER>
static hipError_t dispatch(int N, const Tile* tiles, const ProbDev* probs, const AxApplyArgs& a,
                           int ntiles, int epb, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr) {
  switch (N) {
#define MX_CASE(NN) \
  case NN:          \
    return launch_one<NN, T, TG, SOLVER>(tiles, probs, a, ntiles, epb, s, ev0, ev1);
    MX_CASE(1) MX_CASE(2) MX_CASE(3) MX_CASE(4) MX_CASE(5) MX_CASE(6) MX_CASE(7) MX_CASE(8)
    MX_CASE(9) MX_CASE(10) MX_CASE(11) MX_CASE(12) MX_CASE(13) MX_CASE(14) MX_CASE(15)
#undef MX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// prec: 0 FP64/FP64, 1 FP32/FP32, 2 FP32 vectors with BF16 G
hipError_t launch_ax_apply(int prec, int N, int E, int epb, const void* u, void* w,
                           const void* G, const void* hB, const void* D, hipStream_t s) {
  AxApplyArgs a{u, w, G, hB, D, E};
  int ntiles = (E + epb - 1) / epb;
  switch (prec) {
    case 0: return dispatch<double, double, false>(N, nullptr, nullptr, a, ntiles, epb, s);
    case 1: return dispatch<float, float, false>(N, nullptr, nullptr, a, ntiles, epb, s);
    case 2: return dispatch<float, bf16_t, false>(N, nullptr, nullptr, a, ntiles, epb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ax_solver(int prec, int N, const Tile* tiles, int ntiles, const ProbDev* probs,
                            int epb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  AxApplyArgs a{};
  switch (prec) {
    case 0: return dispatch<double, double, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1);
    case 1: return dispatch<float, float, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1);
    case 2: return dispatch<float, bf16_t, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

// largest epb whose workgroup (rounded to wave64s) fits 256 threads
int max_epb(int N) {
  const int n2 = (N + 1) * (N + 1);
  int e = 1;
  while ((((e + 1) * n2 + 63) / 64) * 64 <= 256) ++e;
  return e;
}

}  // namespace mx
