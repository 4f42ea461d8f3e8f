// Shared internal definitions of the mxsem HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>

#include "../../include/mxsem.h"

namespace mx {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* get_error();

// Status of an entry point whose body threw: no C++ exception crosses the C
// boundary (std::bad_alloc becomes MXSEM_ENOMEM, anything else
// MXSEM_EINTERNAL).
inline int api_fail(const char* fn, int code) noexcept {
  try {
    set_error(std::string(fn) + (code == MXSEM_ENOMEM ? ": host allocation failed"
                                                      : ": internal error (C++ exception)"));
  } catch (...) {
  }
  return code;
}
}  // namespace mx

// Every int-returning extern "C" function wraps its body in these two.
#define MX_API_BEGIN try {
#define MX_API_END(fn)                                   \
  }                                                      \
  catch (const std::bad_alloc&) {                        \
    return ::mx::api_fail(fn, MXSEM_ENOMEM);             \
  }                                                      \
  catch (...) {                                          \
    return ::mx::api_fail(fn, MXSEM_EINTERNAL);          \
  }

namespace mx {

#define MX_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::mx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return MXSEM_EHIP;                                                      \
    }                                                                         \
  } while (0)

#define MX_TRY(call)               \
  do {                             \
    int rc_ = (call);              \
    if (rc_ != MXSEM_OK) return rc_; \
  } while (0)

#define MX_CHECK(cond, code, msg)  \
  do {                             \
    if (!(cond)) {                 \
      ::mx::set_error(msg);        \
      return code;                 \
    }                              \
  } while (0)

// ---------------------------------------------------------------- bf16
// Storage of the BF16 geometric factors: the upper 16 bits of an FP32.
typedef uint16_t bf16_t;

__host__ __device__ inline float bf16_to_float(bf16_t b) {
  union {
    uint32_t u;
    float f;
  } v;
  v.u = ((uint32_t)b) << 16;
  return v.f;
}

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__host__ __device__ inline bf16_t float_to_bf16(float f) {
  union {
    uint32_t u;
    float f;
  } v;
  v.f = f;
  uint32_t lsb = (v.u >> 16) & 1u;
  v.u += 0x7FFFu + lsb;
  return (bf16_t)(v.u >> 16);
}

// the nearest BF16 value, as an FP32 (round to nearest even, finite inputs)
__device__ inline float bf16_round(float f) { return bf16_to_float(float_to_bf16(f)); }

template <typename T>
__device__ inline T load_as(const T* p) {
  return *p;
}
template <typename TD, typename TS>
__device__ inline TD cvt(TS v) {
  return (TD)v;
}
template <>
__device__ inline float cvt<float, bf16_t>(bf16_t v) {
  return bf16_to_float(v);
}
template <>
__device__ inline double cvt<double, bf16_t>(bf16_t v) {
  return (double)bf16_to_float(v);
}

// ---------------------------------------------------------------- solver state
// Per-problem scalars of one (P)CG solve, resident in device memory.
struct State {
  double rho;    // (r, z)_c
  double sigma;  // (p, A p)_c
  double alpha, beta;
  double rr;     // (r, r)_c
  double bb;     // (b, b)_c of the (inner) right-hand side
  double tol2;   // tol^2
  double best;   // stagnation reference relative residual
  double res;    // last relative recursive residual
  double zw;     // (z, A p_old)_c (flexible CG)
  double* history;  // nullable [maxit+1]
  int iter, maxit;
  int done;      // 1: this problem's kernels return at once
  int reason;    // MXSEM_CONVERGED ...
  int since;     // iterations since the last 10% improvement
  int fallback;  // learned-PC steps replaced by Jacobi
  int pc;        // mxsem_pc
  int fb_pending;  // flexible CG: this step's z must be replaced by Jacobi
  // PCG with two direction buffers: x is updated every second step with
  // both steps' alpha p; after an even step the update is pending
  int x_pending;
  double alpha_prev;  // alpha of the pending step
};

// A tile: a block of work of one problem (elements, groups or entries);
// aux selects the gather-scatter bucket.
// Device pointers read from device-side structs are generic (flat)
// pointers to the compiler; flat loads count against the LDS counter as
// well, so every LDS wait would also wait for them.  Kernels cast such
// pointers to the global address space, which gives global_load/store.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> gcast(T* p) {
  return (gptr<T>)p;
}

struct Tile {
  int prob;
  int first;
  int aux;
  int pad;
};

// Gather-scatter plan.  Groups of m >= 2 copies of one node are stored in
// buckets of equal m, m copies per group contiguous in idx (ascending local
// index), groups of a bucket in ascending first local index.  Free buckets
// come first (m = 8, 4, 2 at 16-byte aligned offsets, then any other m),
// then buckets of Dirichlet groups, then one bucket with m = 0 that lists
// every Dirichlet entry (one entry per "group") for the mask.
constexpr int MAX_BUCKETS = 16;
struct GsBucket {
  int m;        // copies per group (0: mask list)
  int ngroups;  // groups (entries for the mask list)
  int off;      // first index in idx
  int pad;
};
struct GsPlan {
  const int* idx;
  const int* erank;  // [E] rank of each element for the pairwise order, or null
                     // (then every element is a rank of its own)
  GsBucket bk[MAX_BUCKETS];
  int nfree;    // buckets [0, nfree): free groups
  int nall;     // buckets [nfree, nall): Dirichlet groups; bk[nall]: mask list
  int n3;       // entries per element (locates a copy's element)
  int pad;
};

// Device view of one problem for the iteration kernels.  Vector and
// operator pointers are typed by the kernel instantiation.
struct ProbDev {
  int E, n3;
  int64_t nloc;
  // operator
  const void* G;     // [E][6][n3] in the G type
  const void* hB;    // [E][n3] h*B in the G type or null (Poisson)
  const void* D;     // [n][n] in the vector type
  const void* dinv;  // [nloc] vector type
  const uint8_t* mult;  // [nloc] multiplicity m
  // gather-scatter plan
  GsPlan gs;
  // vectors (vector type); p_alt: the second direction buffer (the
  // search direction of step k is kept in p for even k, p_alt for odd k)
  void *x, *r, *z, *p, *w, *p_alt;
  // FP64 right-hand side of the current (inner) solve and its scale
  const double* rhs64;
  double rhs_scale;  // r = rhs64 * rhs_scale
  // partial sums
  double* part_ax;   // sigma = sum_i p_i (A_L p)_i, per operator tile
  double* part_gs;   // unused by PCG (kept for the flexible-CG dots)
  double* part_u0;   // per update tile: (r,z)_c  (or rr for FCG)
  double* part_u1;   // per update tile: (r,r)_c
  double* part_u2;   // per tile: (z,w)_c (flexible CG)
  int nblk_ax, nblk_gs, nblk_upd;
  int dm;            // DotMode of the partial sums (PCG)
  // box lattice (ne^3 lexicographic elements, lattice global ids, Dirichlet
  // on the whole boundary, n = 8 or 16): elements per direction (else 0),
  // log2 n, 1/ne and 1/ne^2; the PCG vector pass then forms QQ^T w itself
  int box_ne, box_ln;
  float box_rne, box_rne2;
  State* st;
};

constexpr int GS_THREADS = 256;  // gather-scatter workgroup
constexpr int GS_PER_THREAD = 2;
constexpr int GS_CHUNK = GS_THREADS * GS_PER_THREAD;  // items per workgroup
constexpr int GS_PAIRWISE_MAXM = 16;  // largest group of the pairwise summation order
constexpr int GS_ROW_EL = 4;  // elements per row tile of a box lattice (N = 7)
constexpr int UPD_THREADS = 256; // threads per vector-update workgroup
constexpr int UPD_PER_THREAD = 8;  // entries per thread (two 4-wide vectors)
constexpr int UPD_CHUNK = UPD_THREADS * UPD_PER_THREAD;
constexpr int FIN_THREADS = 1024;  // final-reduction workgroup
constexpr int MAX_N = 15;
// accelerator dies (XCDs) of the MI355X: consecutive workgroups of a launch
// are dealt to them in turn, each die with its own L2
constexpr int XCDS = 8;
// stagnation: no 10% improvement of the best relative residual in this many
// iterations (CG residuals on high-contrast coefficients plateau for
// hundreds of iterations before falling again)
constexpr int STAG_WINDOW = 500;

// ---------------------------------------------------------------- reductions
// c = 1/m, the weight of a local copy in the c-weighted dots
__device__ inline double cweight(uint8_t m) { return m == 1 ? 1.0 : 1.0 / (double)m; }

// Deterministic block sum of one value per thread (wave64 shuffles, then
// LDS across waves).  Every thread of the block must call it.  Returns the
// sum on thread 0.
template <typename A>
__device__ inline A block_sum(A v, A* sred) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  A s = 0;
  if (threadIdx.x == 0)
    for (int q = 0; q < nw; ++q) s += sred[q];
  return s;
}

// ---------------------------------------------------------------- dot accumulation
// Accumulation of the dots of an FP32 iteration (the extended-precision
// study of Sec. 5.2.1):
//   DOT_F64   products and sums in FP64 (the mixed recipe);
//   DOT_F32   products and sums in FP32, the working precision;
//   DOT_DOT2  compensated FP32, the Dot2 algorithm of Ogita, Rump and Oishi
//             (2005): each product is split exactly into its rounded value
//             and its error (TwoProduct), the value enters the running sum
//             by TwoSum, whose error joins the product error in a running
//             FP32 correction.  Two partial results (sum, correction) are
//             combined by TwoSum of the sums plus both corrections (the
//             reduction of size-two expansions that the paper applies across
//             ranks, here across lanes, waves and workgroups).  The result is
//             the FP32 rounding of sum + correction.
// A weighted term a c b (c = 1/m) is formed as (a c) b; a c is exact in
// FP32 when m is a power of two (every copy count of a hexahedral box).
enum DotMode { DOT_F64 = 0, DOT_F32 = 1, DOT_DOT2 = 2 };

// Error-free transformations in FP32.  Contraction stays off inside them:
// a product fused into the following sum would lose the error term.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ inline void two_prod(float a, float b, float& p, float& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

struct F2 {
  float s, c;  // running sum and its correction
};
// An F2 travels through one double slot (partial-sum arrays, LDS) as the
// bits of a two-float vector: register moves only.
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ inline double f2_pack(F2 v) {
  const f2v_t t = {v.s, v.c};
  return __builtin_bit_cast(double, t);
}
__device__ inline F2 f2_unpack(double d) {
  const f2v_t t = __builtin_bit_cast(f2v_t, d);
  return F2{t.x, t.y};
}
__device__ inline F2 f2_combine(F2 a, F2 b) {
#pragma clang fp contract(off)
  F2 r;
  float e;
  two_sum(a.s, b.s, r.s, e);
  r.c = (a.c + b.c) + e;
  return r;
}

// Per-thread accumulator; block() reduces over the workgroup and returns
// the workgroup's partial on thread 0, encoded in one double (FP64 and
// FP32 modes: the value; Dot2: the (sum, correction) pair's bits).
template <int DM>
struct DotAcc;
template <>
struct DotAcc<DOT_F64> {
  double s = 0.0;
  template <typename T>
  __device__ void add(T a, T b) { s += (double)a * (double)b; }
  template <typename T>
  __device__ void add2(T a0, T b0, T a1, T b1) { s += (double)a0 * (double)b0 + (double)a1 * (double)b1; }
  template <typename T>
  __device__ void addw(T a, double c, T b) { s += (double)a * c * (double)b; }
  __device__ double block(double* sred) { return block_sum(s, sred); }
};
template <>
struct DotAcc<DOT_F32> {
  float s = 0.f;
  __device__ void add(float a, float b) { s += a * b; }
  __device__ void add2(float a0, float b0, float a1, float b1) { s += a0 * b0; s += a1 * b1; }
  __device__ void addw(float a, double c, float b) { s += (a * (float)c) * b; }
  __device__ double block(double* sred) { return (double)block_sum(s, (float*)sred); }
};
template <>
struct DotAcc<DOT_DOT2> {
  F2 v = {0.f, 0.f};
  __device__ void add(float a, float b) {
#pragma clang fp contract(off)
    float h, r, q;
    two_prod(a, b, h, r);
    two_sum(v.s, h, v.s, q);
    v.c += q + r;
  }
  __device__ void add2(float a0, float b0, float a1, float b1) { add(a0, b0); add(a1, b1); }
  __device__ void addw(float a, double c, float b) {
#pragma clang fp contract(off)
    add(a * (float)c, b);
  }
  __device__ double block(double* sred) {
    F2 x = v;
    for (int off = 32; off > 0; off >>= 1) {
      F2 y;
      y.s = __shfl_down(x.s, off, 64);
      y.c = __shfl_down(x.c, off, 64);
      x = f2_combine(x, y);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) sred[wid] = f2_pack(x);
    __syncthreads();
    F2 t = {0.f, 0.f};
    if (threadIdx.x == 0)
      for (int q = 0; q < nw; ++q) t = f2_combine(t, f2_unpack(sred[q]));
    return f2_pack(t);
  }
};

// Sum of n workgroup partials of mode dm (DOT_F32 or DOT_DOT2) by one
// workgroup of NT threads in a fixed order: thread t combines parts
// t + k NT into accumulator k % 8 (eight independent chains keep eight loads
// in flight), then the eight accumulators pairwise, then the block.  The
// result is an FP32 value.
template <int NT>
__device__ inline double dot_finish(int dm, const gptr<const double> __restrict__ parts, int n,
                                    double* sred) {
  int q = threadIdx.x;
  if (dm == DOT_F32) {
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (; q + 7 * NT < n; q += 8 * NT) {
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] += (float)parts[q + k * NT];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (q + k * NT < n) a[k] += (float)parts[q + k * NT];
    const float s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    return (double)block_sum(s, (float*)sred);
  }
  F2 a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = F2{0.f, 0.f};
  for (; q + 7 * NT < n; q += 8 * NT) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = f2_combine(a[k], f2_unpack(parts[q + k * NT]));
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (q + k * NT < n) a[k] = f2_combine(a[k], f2_unpack(parts[q + k * NT]));
  DotAcc<DOT_DOT2> acc;
  acc.v = f2_combine(f2_combine(f2_combine(a[0], a[1]), f2_combine(a[2], a[3])),
                     f2_combine(f2_combine(a[4], a[5]), f2_combine(a[6], a[7])));
  const F2 t = f2_unpack(acc.block(sred));
  return (double)(t.s + t.c);
}

}  // namespace mx
