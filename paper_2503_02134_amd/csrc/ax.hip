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
  // solver variant: -1 reads and writes p in place; 0 / 1 (the step's
  // parity) reads p_old from p_alt / p and writes p / p_alt
  int parity;
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
// written back), w = A_L p, and the workgroup's partial sum of p.w,
// accumulated as DotMode DM says.  PB (an ablation of the solver variant):
// p is rounded to the nearest BF16 value before it is stored and used, so
// the whole step works with a direction held in BF16.
template <int N, typename T, typename TG, bool SOLVER, int DM, bool PB = false>
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
    U = gcast((const T*)(apply.parity == 0 ? P->p_alt : P->p));
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
      gptr<T> __restrict__ Pw = gcast((T*)(apply.parity == 1 ? P->p_alt : P->p));
#pragma unroll
      for (int k = 0; k < n; ++k) {
        T pv = Z[base + k * n2] + beta * U[base + k * n2];
        if constexpr (PB) pv = bf16_round(pv);
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
  DotAcc<DM> dot;
  if (active) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T wv = w[k];
      if (hB) wv += cvt<T>(__builtin_nontemporal_load(&hB[(int64_t)e * n3 + k * n2 + ij])) * u[k];
      Wout[base + k * n2] = wv;
      if constexpr (SOLVER) dot.add(u[k], wv);
    }
  }
  if constexpr (SOLVER) {
    double s = dot.block(sred);
    if (tid == 0) gcast(P->part_ax)[first / epb] = s;
  }
}

// Mapping with two columns per thread, for even n with n^2/2 <= 64 (N = 5,
// 9; FP32 vectors): thread (i, jh) of an element owns the columns (i, jh) and
// (i, jh + n/2), so an element takes n^2/2 lanes and never straddles two
// wave64s (for N = 9, 50 lanes per wave; for N = 5, three elements of 18
// lanes per wave).  Every slab exchange is then wave-local (wave barrier,
// no workgroup barrier), where the one-column mapping (n^2 = 100 or 36
// lanes per element) needs workgroup barriers.  Arithmetic and summation
// order per output are those of ax_kernel.
template <int N, typename T>
constexpr bool two_col() {
  return (N == 5 || N == 9) && sizeof(T) == 4;  // FP64 columns do not fit twice in registers
}
template <int N>
constexpr int ax2_epw() {  // elements per wave
  return 64 / ((N + 1) * ((N + 1) / 2));
}

template <int N, typename T, typename TG, bool SOLVER, int DM, bool PB = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) ax2_kernel(const Tile* __restrict__ tiles, const ProbDev* __restrict__ probs,
                           AxApplyArgs apply, int epb) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n, hn = n / 2, TPE = n * hn, EPW = 64 / TPE;
  static_assert(n % 2 == 0 && TPE <= 64, "two columns per thread need even n and n^2/2 <= 64");
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
  int64_t nloc_all;
  const ProbDev* P = nullptr;
  if constexpr (SOLVER) {
    const Tile t = tiles[blockIdx.x];
    P = &probs[t.prob];
    if (gcast(P->st)->done) return;  // uniform across the workgroup
    Dg = gcast((const T*)P->D);
    G = gcast((const TG*)P->G);
    hB = gcast((const TG*)P->hB);
    U = gcast((const T*)(apply.parity == 0 ? P->p_alt : P->p));
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
  const int wave = tid >> 6, lane = tid & 63;
  const int slot = lane / TPE;  // == EPW for the lanes past the wave's last element
  const int tl = lane - slot * TPE;
  const int le = wave * EPW + slot;
  const int i = tl % n, j0 = tl / n, j1 = j0 + hn;
  const int e = first + le;
  const bool active = slot < EPW && le < epb && e < E;
  T* su = slab + (wave * EPW + (slot < EPW ? slot : 0)) * 3 * n2;  // touched by active lanes only
  T* sr = su + n2;
  T* ss = sr + n2;
  __syncthreads();

  T u0[n], u1[n], w0[n], w1[n], Di[n], DiT[n], Dj0[n], Dj1[n], Dj0T[n], Dj1T[n];
#pragma unroll
  for (int l = 0; l < n; ++l) {
    Di[l] = sD[i * n + l];
    DiT[l] = sD[l * n + i];
    Dj0[l] = sD[j0 * n + l];
    Dj1[l] = sD[j1 * n + l];
    Dj0T[l] = sD[l * n + j0];
    Dj1T[l] = sD[l * n + j1];
    w0[l] = T(0);
    w1[l] = T(0);
  }
  const int ij0 = j0 * n + i, ij1 = j1 * n + i;
  const int64_t base0 = (int64_t)e * n3 + ij0, base1 = (int64_t)e * n3 + ij1;
  if (active) {
    if constexpr (SOLVER) {
      const T beta = (T)gcast(P->st)->beta;
      gptr<T> __restrict__ Pw = gcast((T*)(apply.parity == 1 ? P->p_alt : P->p));
#pragma unroll
      for (int k = 0; k < n; ++k) {
        T p0 = Z[base0 + k * n2] + beta * U[base0 + k * n2];
        T p1 = Z[base1 + k * n2] + beta * U[base1 + k * n2];
        if constexpr (PB) {
          p0 = bf16_round(p0);
          p1 = bf16_round(p1);
        }
        Pw[base0 + k * n2] = p0;
        Pw[base1 + k * n2] = p1;
        u0[k] = p0;
        u1[k] = p1;
      }
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) {
        u0[k] = U[base0 + k * n2];
        u1[k] = U[base1 + k * n2];
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < n; ++k) u0[k] = u1[k] = T(0);
  }

  const int64_t g0n = (int64_t)(active ? e : 0) * n3 + ij0;
  const int64_t g1n = (int64_t)(active ? e : 0) * n3 + ij1;
  // G of the next k slab in flight while this one is used (registers for
  // the whole column pair do not fit next to the two columns' u, w and D
  // rows; one slab ahead keeps the kernel at three waves per SIMD, which
  // measured 10% faster than two slabs at two waves)
  constexpr int LA = 1;
  T gbuf[n][12];
#pragma unroll
  for (int k = 0; k < LA && k < n; ++k) {
    load_g<T, TG>(G, nloc_all, g0n + k * n2, n3, gbuf[k]);
    load_g<T, TG>(G, nloc_all, g1n + k * n2, n3, gbuf[k] + 6);
  }
#pragma unroll
  for (int k = 0; k < n; ++k) {
    if (k + LA < n) {
      load_g<T, TG>(G, nloc_all, g0n + (k + LA) * n2, n3, gbuf[k + LA]);
      load_g<T, TG>(G, nloc_all, g1n + (k + LA) * n2, n3, gbuf[k + LA] + 6);
    }
    if (active) {
      su[ij0] = u0[k];
      su[ij1] = u1[k];
    }
    elem_sync<1>();
    if (active) {
      T ur0 = T(0), us0 = T(0), ut0 = T(0), ur1 = T(0), us1 = T(0), ut1 = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const T scol = su[l * n + i];
        ur0 += Di[l] * su[j0 * n + l];
        us0 += Dj0[l] * scol;
        ut0 += sD[k * n + l] * u0[l];
        ur1 += Di[l] * su[j1 * n + l];
        us1 += Dj1[l] * scol;
        ut1 += sD[k * n + l] * u1[l];
      }
      const T* ga = gbuf[k];
      const T* gb = gbuf[k] + 6;
      const T wr0 = ga[0] * ur0 + ga[1] * us0 + ga[2] * ut0;
      const T ws0 = ga[1] * ur0 + ga[3] * us0 + ga[4] * ut0;
      const T wt0 = ga[2] * ur0 + ga[4] * us0 + ga[5] * ut0;
      const T wr1 = gb[0] * ur1 + gb[1] * us1 + gb[2] * ut1;
      const T ws1 = gb[1] * ur1 + gb[3] * us1 + gb[4] * ut1;
      const T wt1 = gb[2] * ur1 + gb[4] * us1 + gb[5] * ut1;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        w0[m] += sD[k * n + m] * wt0;
        w1[m] += sD[k * n + m] * wt1;
      }
      sr[ij0] = wr0;
      ss[ij0] = ws0;
      sr[ij1] = wr1;
      ss[ij1] = ws1;
    }
    elem_sync<1>();
    if (active) {
      T acc0 = T(0), acc1 = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const T rcol = sr[j0 * n + l], rcol1 = sr[j1 * n + l];
        acc0 += DiT[l] * rcol + Dj0T[l] * ss[l * n + i];
        acc1 += DiT[l] * rcol1 + Dj1T[l] * ss[l * n + i];
      }
      w0[k] += acc0;
      w1[k] += acc1;
    }
    elem_sync<1>();
  }

  DotAcc<DM> dot;
  if (active) {
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T wv0 = w0[k], wv1 = w1[k];
      if (hB) {
        wv0 += cvt<T>(__builtin_nontemporal_load(&hB[base0 + k * n2])) * u0[k];
        wv1 += cvt<T>(__builtin_nontemporal_load(&hB[base1 + k * n2])) * u1[k];
      }
      Wout[base0 + k * n2] = wv0;
      Wout[base1 + k * n2] = wv1;
      if constexpr (SOLVER) dot.add2(u0[k], wv0, u1[k], wv1);
    }
  }
  if constexpr (SOLVER) {
    double s = dot.block(sred);
    if (tid == 0) gcast(P->part_ax)[first / epb] = s;
  }
}

// With ev0/ev1 the launch records its own start and end (hipExtLaunchKernel),
// so the elapsed time between them is the kernel's execution time.
template <int N, typename T, typename TG, bool SOLVER, int DM, bool PB>
static hipError_t launch_one(const Tile* tiles, const ProbDev* probs, const AxApplyArgs& a,
                             int ntiles, int epb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                             int cols) {
  constexpr int n = N + 1, n2 = n * n;
  if constexpr (two_col<N, T>()) {
    if (cols != 1) {  // two columns per thread unless one is asked for
      constexpr int EPW = ax2_epw<N>();
      const int waves = (epb + EPW - 1) / EPW;
      if (epb < 1 || waves > 4) return hipErrorInvalidConfiguration;
      const size_t shm = sizeof(T) * (n2 + (size_t)waves * EPW * 3 * n2);
      if (ev0)
        hipExtLaunchKernelGGL((ax2_kernel<N, T, TG, SOLVER, DM, PB>), dim3(ntiles),
                              dim3(64 * waves), (uint32_t)shm, s, ev0, ev1, 0, tiles, probs, a,
                              epb);
      else
        hipLaunchKernelGGL((ax2_kernel<N, T, TG, SOLVER, DM, PB>), dim3(ntiles), dim3(64 * waves),
                           shm, s, tiles, probs, a, epb);
      return hipGetLastError();
    }
  }
  int threads = ((epb * n2 + 63) / 64) * 64;
  if (epb < 1 || threads > 256) return hipErrorInvalidConfiguration;
  size_t shm = sizeof(T) * (n2 + (size_t)epb * 3 * n2);
  if (ev0)
    hipExtLaunchKernelGGL((ax_kernel<N, T, TG, SOLVER, DM, PB>), dim3(ntiles), dim3(threads), (uint32_t)shm,
                          s, ev0, ev1, 0, tiles, probs, a, epb);
  else
    hipLaunchKernelGGL((ax_kernel<N, T, TG, SOLVER, DM, PB>), dim3(ntiles), dim3(threads), shm, s, tiles,
                       probs, a, epb);
  return hipGetLastError();
}

template <typename T, typename TG, bool SOLVER, int DM = DOT_F64, bool PB = false>
static hipError_t dispatch(int N, const Tile* tiles, const ProbDev* probs, const AxApplyArgs& a,
                           int ntiles, int epb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                           int cols) {
  switch (N) {
#define MX_CASE(NN) \
  case NN:          \
    return launch_one<NN, T, TG, SOLVER, DM, PB>(tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
    MX_CASE(1) MX_CASE(2) MX_CASE(3) MX_CASE(4) MX_CASE(5) MX_CASE(6) MX_CASE(7) MX_CASE(8)
    MX_CASE(9) MX_CASE(10) MX_CASE(11) MX_CASE(12) MX_CASE(13) MX_CASE(14) MX_CASE(15)
#undef MX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// prec: 0 FP64/FP64, 1 FP32/FP32, 2 FP32 vectors with BF16 G
hipError_t launch_ax_apply(int prec, int N, int E, int epb, const void* u, void* w,
                           const void* G, const void* hB, const void* D, hipStream_t s, int cols) {
  AxApplyArgs a{u, w, G, hB, D, E};
  int ntiles = (E + epb - 1) / epb;
  switch (prec) {
    case 0: return dispatch<double, double, false>(N, nullptr, nullptr, a, ntiles, epb, s, nullptr, nullptr, cols);
    case 1: return dispatch<float, float, false>(N, nullptr, nullptr, a, ntiles, epb, s, nullptr, nullptr, cols);
    case 2: return dispatch<float, bf16_t, false>(N, nullptr, nullptr, a, ntiles, epb, s, nullptr, nullptr, cols);
    default: return hipErrorInvalidValue;
  }
}

// dm: DotMode of the sigma partials (FP32 vectors with FP32 G; FP64
// vectors and BF16 G take DOT_F64)
hipError_t launch_ax_solver(int prec, int dm, int N, const Tile* tiles, int ntiles,
                            const ProbDev* probs, int epb, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1, int parity, int cols) {
  AxApplyArgs a{};
  a.parity = parity;
  if (prec == 1 && dm == DOT_F32)
    return dispatch<float, float, true, DOT_F32>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
  if (prec == 1 && dm == DOT_DOT2)
    return dispatch<float, float, true, DOT_DOT2>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
  if (dm != DOT_F64) return hipErrorInvalidValue;
  switch (prec) {
    case 0: return dispatch<double, double, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
    case 1: return dispatch<float, float, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
    case 2: return dispatch<float, bf16_t, true>(N, tiles, probs, a, ntiles, epb, s, ev0, ev1, cols);
    case 3:
      return dispatch<float, float, true, DOT_F64, true>(N, tiles, probs, a, ntiles, epb, s, ev0,
                                                         ev1, cols);
    default: return hipErrorInvalidValue;
  }
}

// elements per wave of the two-column mapping (FP32 vectors; 0: N uses the
// one-column mapping only).  Tiles of that many elements suit both mappings.
int ax_wave_elements(int N) {
  if (N == 5) return ax2_epw<5>();
  if (N == 9) return ax2_epw<9>();
  return 0;
}

// largest tile of the two-column mapping: four waves of ax2_epw elements
int max_epb2(int N) {
  const int w = ax_wave_elements(N);
  return w > 0 ? 4 * w : 0;
}

// largest epb whose one-column workgroup (rounded to wave64s) fits 256
// threads
int max_epb(int N) {
  const int n2 = (N + 1) * (N + 1);
  int e = 1;
  while ((((e + 1) * n2 + 63) / 64) * 64 <= 256) ++e;
  return e;
}

}  // namespace mx
