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

// The six geometric factors of local node `node` (= e n^3 + p).  FP64: the
// master layout [E][6][n^3].  FP32 / BF16: the split layout (a 4-vector of
// rr, rs, rt, ss per node, then a 2-vector of st, tt per node after all
// nloc 4-vectors), i.e. two coalesced vector loads.  G is read once per
// operator application and not again before the next one: non-temporal
// loads keep it from displacing the CG vectors in the last-level cache.
typedef float gf4_t __attribute__((ext_vector_type(4)));
typedef float gf2_t __attribute__((ext_vector_type(2)));
typedef uint16_t gh4_t __attribute__((ext_vector_type(4)));
typedef uint16_t gh2_t __attribute__((ext_vector_type(2)));
template <typename T, typename TG>
__device__ inline void load_g(const gptr<const TG> G, int64_t nloc, int64_t node, int n3, T* g) {
  if constexpr (sizeof(TG) == 8) {
    const int64_t e = node / n3, p = node - e * n3;
    const gptr<const TG> ge = G + e * 6 * n3 + p;
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = (T)__builtin_nontemporal_load(&ge[q * n3]);
  } else if constexpr (sizeof(TG) == 4) {
    const gf4_t a = __builtin_nontemporal_load(&((gptr<const gf4_t>)G)[node]);
    const gf2_t b = __builtin_nontemporal_load(&((gptr<const gf2_t>)(G + 4 * nloc))[node]);
    g[0] = a.x, g[1] = a.y, g[2] = a.z, g[3] = a.w, g[4] = b.x, g[5] = b.y;
  } else {
    const gh4_t a = __builtin_nontemporal_load(&((gptr<const gh4_t>)G)[node]);
    const gh2_t b = __builtin_nontemporal_load(&((gptr<const gh2_t>)(G + 4 * nloc))[node]);
    g[0] = cvt<T>((bf16_t)a.x), g[1] = cvt<T>((bf16_t)a.y), g[2] = cvt<T>((bf16_t)a.z);
    g[3] = cvt<T>((bf16_t)a.w), g[4] = cvt<T>((bf16_t)b.x), g[5] = cvt<T>((bf16_t)b.y);
  }
}

// Synchronisation of one element's threads around its LDS slabs.  When
// n^2 divides 64, no element straddles two wave64s, and the slab exchange
// stays inside one wave: LDS instructions of a wave complete in issue
// order, so a compiler-level wave barrier (no instruction) suffices and the
// elements of a workgroup run unsynchronised.  Otherwise a workgroup
// barrier.
template <int n2>
__device__ inline void elem_sync() {
  if constexpr (64 % n2 == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

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

  gptr<const T> __restrict__ Dg;
  gptr<const TG> __restrict__ G;
  gptr<const TG> __restrict__ hB;
  gptr<const T> __restrict__ U;
  gptr<T> __restrict__ Wout;
  gptr<const T> __restrict__ Z = nullptr;
  int E, first;
  int64_t nloc_all;  // local entries of the whole problem (locates the split G parts)
  const ProbDev* P = nullptr;
  if constexpr (SOLVER) {
    const Tile t = tiles[blockIdx.x];
    P = &probs[t.prob];
    if (gcast(P->st)->done) return;  // uniform across the workgroup
    Dg = gcast((const T*)P->D);
    G = gcast((const TG*)P->G);
    hB = gcast((const TG*)P->hB);
    U = gcast((const T*)P->p);
    Wout = gcast((T*)P->w);
    Z = gcast((const T*)P->z);
    E = P->E;
    nloc_all = P->nloc;
    first = t.first;
  } else {
    Dg = gcast((const T*)apply.D);
    G = gcast((const TG*)apply.G);
    hB = gcast((const TG*)apply.hB);
    U = gcast((const T*)apply.u);
    Wout = gcast((T*)apply.w);
    E = apply.E;
    nloc_all = (int64_t)E * n3;
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
      const T beta = (T)gcast(P->st)->beta;
      gptr<T> __restrict__ Pw = gcast((T*)P->p);
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
  const int64_t gnode = (int64_t)(active ? e : 0) * n3 + ij;  // inactive lanes read element 0
  constexpr bool PREFETCH = 6 * n * sizeof(T) <= 512;
  T gpre[PREFETCH ? 6 * n : 1];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T gk[6];
      load_g<T, TG>(G, nloc_all, gnode + k * n2, n3, gk);
#pragma unroll
      for (int q = 0; q < 6; ++q) gpre[q * n + k] = active ? gk[q] : T(0);
    }
  }
#pragma unroll
  for (int k = 0; k < n; ++k) {
    if (active) su[ij] = u[k];
    elem_sync<n2>();
    if (active) {
      T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        ur += Di[l] * su[j * n + l];
        us += Dj[l] * su[l * n + i];
        ut += sD[k * n + l] * u[l];
      }
      T g0, g1, g2, g3, g4, g5;
      if constexpr (PREFETCH) {
        g0 = gpre[0 * n + k];
        g1 = gpre[1 * n + k];
        g2 = gpre[2 * n + k];
        g3 = gpre[3 * n + k];
        g4 = gpre[4 * n + k];
        g5 = gpre[5 * n + k];
      } else {
        T gk[6];
        load_g<T, TG>(G, nloc_all, gnode + k * n2, n3, gk);
        g0 = gk[0], g1 = gk[1], g2 = gk[2], g3 = gk[3], g4 = gk[4], g5 = gk[5];
      }
      const T wr = g0 * ur + g1 * us + g2 * ut;
      const T ws = g1 * ur + g3 * us + g4 * ut;
      const T wt = g2 * ur + g4 * us + g5 * ut;
#pragma unroll
      for (int m = 0; m < n; ++m) w[m] += sD[k * n + m] * wt;
      sr[ij] = wr;
      ss[ij] = ws;
    }
    elem_sync<n2>();
    if (active) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) acc += DiT[l] * sr[j * n + l] + DjT[l] * ss[l * n + i];
      w[k] += acc;
    }
    elem_sync<n2>();
  }

  // (p, QQ^T A_L p)_c = sum_i p_i (A_L p)_i over all local entries, because
  // p is continuous and zero on Dirichlet nodes: the solver takes sigma
  // from the local result, before the gather-scatter.
  double dot = 0.0;
  if (active) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T wv = w[k];
      if (hB) wv += cvt<T>(__builtin_nontemporal_load(&hB[(int64_t)e * n3 + k * n2 + ij])) * u[k];
      Wout[base + k * n2] = wv;
      if constexpr (SOLVER) dot += (double)u[k] * (double)wv;
    }
  }
  if constexpr (SOLVER) {
    double s = block_sum(dot, sred);
    if (tid == 0) gcast(P->part_ax)[first / epb] = s;
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
