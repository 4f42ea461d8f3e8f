// Gather-scatter (direct stiffness summation QQ^T, Sec. 4.2.1), the
// Dirichlet mask, the c-weighted dots (the glsc3 rows of the CG-loop
// profiling table, Sec. 4.1), the fused CG vector pass (the two add2s2
// rows, the preconditioner and the following dots of that table), the
// device-side scalar updates of (P)CG, and the small casts of iterative
// refinement.
//
// Gather-scatter plan: every element-face node belongs to a group (its
// copies, ascending local index).  Groups of free nodes come first, sorted
// by multiplicity, then groups of Dirichlet nodes, whose entries form the
// mask list.  One thread per group: copies are summed in the accumulation
// type (FP64 in every mode of the paper's recipe) in ascending local-index
// order, rounded once to the storage type and written to every copy, so
// the copies stay bitwise equal.  No atomics anywhere: every reduction is a
// fixed tree (wave64 shuffles, LDS, per-tile partials, one final block).
#include <math.h>

#include "common.hpp"

namespace mx {

// ------------------------------------------------------------ gather-scatter
typedef int gi2_t __attribute__((ext_vector_type(2)));
typedef int gi4_t __attribute__((ext_vector_type(4)));

struct GsApi {
  void* v;
  GsPlan plan;
  int bucket;
  int on_z;   // solver variant: sum z instead of w
  int nfin;   // solver variant: leading workgroups that finish sigma (0: none)
  int nprob;  // problems whose sigma they finish (the rest of the nfin do nothing)
  const Tile* ztiles;  // solver variant on z: trailing workgroups forming the Jacobi z
  int nz;
};

template <int NT>
__device__ inline double fixed_sum(const gptr<const double> __restrict__ parts, int n,
                                   double* sred);
__device__ inline void fin_sigma_step(const ProbDev& P, double* sred);

// One thread per group, GS_PER_THREAD groups per thread issued together:
// all index loads, then all value loads, then sums (ascending local index,
// in the accumulation type ACC), then the stores.  m = 0 is the mask list.
// PAIRWISE: the summation order of a pairwise exchange between ranks
// (Sec. 4.2.1), with the elements assigned to ranks by plan->erank (null:
// every element a rank of its own).  Each rank sums its own copies
// (ascending local index), then adds the other ranks' partial sums in
// ascending rank order, and every copy receives its rank's result.  Two
// ranks always agree (a + b = b + a); copies of a node shared by three or
// more ranks may differ in their last bits when the sums are FP32
// (m <= GS_PAIRWISE_MAXM).
// The pairwise order for one group of m copies (local indices ids, ascending).
template <typename T, typename ACC>
__device__ inline void gs_pairwise_group(gptr<T> v, const int* ids, int m,
                                         const gptr<const int> erank, int n3) {
  T a[GS_PAIRWISE_MAXM];
  int rk[GS_PAIRWISE_MAXM];
  for (int k = 0; k < m; ++k) {
    const int i = ids[k];
    a[k] = v[i];
    rk[k] = erank ? erank[i / n3] : i / n3;
  }
  // the ranks holding copies, ascending, with their partial sums
  ACC part[GS_PAIRWISE_MAXM];
  int rl[GS_PAIRWISE_MAXM];
  int nr = 0, last = -1;
  for (int t = 0; t < m; ++t) {
    int best = 0x7fffffff;
    for (int j = 0; j < m; ++j)
      if (rk[j] > last && rk[j] < best) best = rk[j];
    if (best == 0x7fffffff) break;
    ACC ps = ACC(0);
    bool first = true;
    for (int j = 0; j < m; ++j)
      if (rk[j] == best) {
        ps = first ? (ACC)a[j] : ps + (ACC)a[j];
        first = false;
      }
    rl[nr] = best;
    part[nr] = ps;
    ++nr;
    last = best;
  }
  for (int k = 0; k < m; ++k) {
    int own = 0;
    for (int t = 0; t < nr; ++t)
      if (rl[t] == rk[k]) own = t;
    ACC sum = part[own];
    for (int t = 0; t < nr; ++t)
      if (t != own) sum += part[t];
    v[ids[k]] = (T)sum;
  }
}

// Box lattices (ProbDev::box_ne > 0) have tiles of whole elements whose
// groups are found by index arithmetic instead of the index array
// (Tile::aux < 0, Tile::first the first element, Tile::pad the element
// count: four elements at N = 7, one at N = 15).  Element e owns the nodes
// it shares with the elements above it and with none below: the interiors of
// its x+, y+ and z+ faces (2 copies), its three upper edges (4) and its upper
// corner (8); a node on the box boundary is left to the mask list.  A tile lists its
// elements' face groups, then their edge groups, then their corners, so a
// wave mostly does groups of one size.  The copies are the node's entries
// in the elements e + dz ne^2 + dy ne + dx (dx, dy, dz in {0, 1}, 1 across
// an upper face), summed in that lexicographic order, which is ascending
// local index: the order of the index-array groups, so the results are
// bitwise theirs.
// One box tile, one group per thread per pass (56 registers, eight waves
// per SIMD: two groups per thread with all their loads issued together took
// 104 registers and was slower, 38 against 31 us on 32^3 elements, N = 7).
template <typename T, typename ACC, bool PAIRWISE, int N>
__device__ inline void gs_box_tile(gptr<T> v, const ProbDev& P, int e0, int nel) {
  constexpr int n = N + 1, M = N - 1, F = 3 * M * M, ED = 3 * M;
  constexpr int ln = n == 8 ? 3 : 4;
  const int ne = P.box_ne, ne2 = ne * ne;
  // coordinates of the tile's first element (float quotients, corrected)
  int ez = (int)((float)e0 * P.box_rne2);
  ez -= ez * ne2 > e0;
  ez += (ez + 1) * ne2 <= e0;
  const int rem = e0 - ez * ne2;
  int ey = (int)((float)rem * P.box_rne);
  ey -= ey * ne > rem;
  ey += (ey + 1) * ne <= rem;
  const int ex0 = rem - ey * ne, ey0 = ey, ez0 = ez;
  const int nF = nel * F, nE = nel * ED, ntot = nF + nE + nel;
  for (int s = (int)threadIdx.x; s < ntot; s += GS_THREADS) {
    int el, a, b, c, m;
    if (s < nF) {
      el = s / F;
      const int r = s - el * F, f = r / (M * M), uv = r - f * M * M;
      const int u = 1 + uv % M, w = 1 + uv / M;
      a = f == 0 ? N : u;
      b = f == 0 ? u : f == 1 ? N : w;
      c = f == 2 ? N : w;
      m = 2;
    } else if (s < nF + nE) {
      const int s2 = s - nF;
      el = s2 / ED;
      const int r = s2 - el * ED, k = r / M, u = 1 + r % M;
      a = k == 2 ? u : N;
      b = k == 1 ? u : N;
      c = k == 0 ? u : N;
      m = 4;
    } else {
      el = s - nF - nE;
      a = b = c = N;
      m = 8;
    }
    const bool ux = a == N, uy = b == N, uz = c == N;
    // the element's coordinates: the first element's, moved on by el
    int ex = ex0 + el, eyy = ey0, ezz = ez0;
    while (ex >= ne) ex -= ne, ++eyy;
    while (eyy >= ne) eyy -= ne, ++ezz;
    if ((ux && ex == ne - 1) || (uy && eyy == ne - 1) || (uz && ezz == ne - 1)) continue;
    const int e = e0 + el;
    int ids[8];
    int q = 0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          if ((dz && !uz) || (dy && !uy) || (dx && !ux)) continue;
          const int eo = e + dz * ne2 + dy * ne + dx;
          ids[q++] = (eo << (3 * ln)) + (dx ? 0 : a) + ((dy ? 0 : b) << ln) +
                     ((dz ? 0 : c) << (2 * ln));
        }
    if constexpr (PAIRWISE) {
      gs_pairwise_group<T, ACC>(v, ids, m, gcast(P.gs.erank), P.gs.n3);
    } else if (m == 2) {
      const T val = (T)((ACC)v[ids[0]] + (ACC)v[ids[1]]);
      v[ids[0]] = val;
      v[ids[1]] = val;
    } else if (m == 4) {
      const T a0 = v[ids[0]], a1 = v[ids[1]], a2 = v[ids[2]], a3 = v[ids[3]];
      const T val = (T)((((ACC)a0 + (ACC)a1) + (ACC)a2) + (ACC)a3);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[ids[k]] = val;
    } else {
      T av[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) av[k] = v[ids[k]];
      ACC sum = (ACC)av[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) sum += (ACC)av[k];
      const T val = (T)sum;
#pragma unroll
      for (int k = 0; k < 8; ++k) v[ids[k]] = val;
    }
  }
}

// Lattice coordinates of element e of a box problem (float quotients,
// corrected by one either way).
__device__ inline void box_coords(int e, const ProbDev& P, int& ex, int& ey, int& ez) {
  const int ne = P.box_ne, ne2 = ne * ne;
  int z = (int)((float)e * P.box_rne2);
  z -= z * ne2 > e;
  z += (z + 1) * ne2 <= e;
  const int rem = e - z * ne2;
  int y = (int)((float)rem * P.box_rne);
  y -= y * ne > rem;
  y += (y + 1) * ne <= rem;
  ex = rem - y * ne, ey = y, ez = z;
}

// Row tiles of a box lattice at N = 7 (Tile::aux = -2, Tile::first the
// first element, Tile::pad the count).  A row is the n = 8 entries of one
// element at fixed (j, k).  Its owner is the element itself, moved one down
// in y when j = 0 and one down in z when k = 0 (where the box continues
// below).  An owner's rows sit in row slots s = 0..n in each direction: its
// own rows j = s for s = 1..N (and s = 0 on the lower box face) and row
// j = 0 of the element above (s = n, the second copy of line s = N, where
// the box continues above); likewise in z.  A tile is a run of at most
// GS_ROW_EL consecutive elements of one x line of the lattice, one thread
// per (element, row line).  A thread reads its line's copies as whole rows
// (16-byte loads) into registers, and, for the last element of the run,
// entry 0 of the element after it; the rows' end entries pass between the
// run's elements through LDS (one barrier).  It forms each node's sum of
// copies in ACC (lexicographic (dz, dy, dx) order, which is ascending local
// index, so the sums are the index groups' bitwise) or zero on the box
// boundary; an x-face node is formed by the threads on both sides, in the
// same order.  It writes its rows whole, except entry 0 of the run's first
// element when an element precedes it: the run to the left writes that
// column, with its own copies of those nodes.  Every entry has one writer,
// no workgroup uses an entry that another one writes, and the mask list is
// not needed.
constexpr int GS_ROW_N = 8;  // row tiles: n = N + 1
__device__ inline bool row_held(int s, bool lo, bool hi) {
  return s == 0 ? lo : (s == GS_ROW_N ? hi : true);
}
template <typename T, typename ACC>
__device__ inline void gs_row_tile(gptr<T> v, const ProbDev& P, int e0, int nel) {
  constexpr int n = GS_ROW_N, N = n - 1, VW = 16 / (int)sizeof(T), PR = n / VW;
  static_assert(GS_ROW_EL * n * n == GS_THREADS, "one thread per line of the run");
  typedef T VT __attribute__((ext_vector_type(VW)));
  // the end entries of every copy of every line, for the neighbouring elements
  __shared__ T col0[GS_ROW_EL][n * n][4], colN[GS_ROW_EL][n * n][4];
  const int ne = P.box_ne, ne2 = ne * ne;
  int ex0, oy, oz;
  box_coords(e0, P, ex0, oy, oz);
  const bool ylo = oy == 0, yhi = oy + 1 < ne, zlo = oz == 0, zhi = oz + 1 < ne;
  // one thread per (element, z line, y line); lines t = 0..N, line 0 only
  // on the lower box face; line N has a second copy (slot n) where the box
  // continues above
  const int el = (int)threadIdx.x / (n * n), ln = (int)threadIdx.x % (n * n);
  const int ty = ln % n, tz = ln / n;
  const int ex = ex0 + el;
  const bool live = el < nel && (ty > 0 || ylo) && (tz > 0 || zlo);
  const int cy = (ty == N && yhi) ? 2 : 1, cz = (tz == N && zhi) ? 2 : 1, nc = cy * cz;
  const bool xh = ex + 1 < ne;  // a copy of entry N in the element after
  const bool bnd = ty == 0 || tz == 0 || (ty == N && !yhi) || (tz == N && !zhi);
  auto row_at = [&](int e, int c) -> int64_t {  // copy c = 2 dz + dy (dy < cy, dz < cz)
    const int dy = cy == 2 ? (c & 1) : 0, dz = cy == 2 ? (c >> 1) : c;
    const int64_t ee = (int64_t)e0 + e + dy * ne + dz * ne2;
    return ee * (n * n * n) + (dy ? 0 : ty) * n + (dz ? 0 : tz) * (n * n);
  };
  // before the barrier: the rows, the interior sums (entries 1..N-1, no
  // neighbour needed) and the end entries published for the neighbours
  T o[n], a0[4], aN[4], nxt[4];
  if (live) {
    T a[4][n];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nc) {
#pragma unroll
        for (int h = 0; h < PR; ++h) {
          const VT q = *(const VT*)&v[row_at(el, c) + h * VW];
#pragma unroll
          for (int u = 0; u < VW; ++u) a[c][h * VW + u] = q[u];
        }
        // entry 0 of the element after the run: only this run reads or writes it
        if (el == nel - 1 && xh) nxt[c] = v[row_at(nel, c)];
      }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nc) {
        a0[c] = a[c][0];
        aN[c] = a[c][N];
        col0[el][ln][c] = a0[c];
        colN[el][ln][c] = aN[c];
      }
    // the sums in lexicographic (dz, dy, dx) order: ascending local index
#pragma unroll
    for (int i = 1; i < N; ++i) {
      ACC s = (ACC)a[0][i];
#pragma unroll
      for (int c = 1; c < 4; ++c)
        if (c < nc) s += (ACC)a[c][i];
      o[i] = bnd ? T(0) : (T)s;
    }
  }
  __syncthreads();
  if (!live) return;
  T pv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c < nc) {
      pv[c] = el > 0 ? colN[el - 1][ln][c] : T(0);
      if (el + 1 < nel) nxt[c] = col0[el + 1][ln][c];
    }
  if (bnd || ex == 0) {
    o[0] = T(0);
  } else {  // with the element before (formed there too, in the same order)
    ACC s = (ACC)pv[0];
    s += (ACC)a0[0];
#pragma unroll
    for (int c = 1; c < 4; ++c)
      if (c < nc) {
        s += (ACC)pv[c];
        s += (ACC)a0[c];
      }
    o[0] = (T)s;
  }
  if (bnd || !xh) {
    o[N] = T(0);
  } else {
    ACC s = (ACC)aN[0];
    s += (ACC)nxt[0];
#pragma unroll
    for (int c = 1; c < 4; ++c)
      if (c < nc) {
        s += (ACC)aN[c];
        s += (ACC)nxt[c];
      }
    o[N] = (T)s;
  }
  // the rows whole, except entry 0 of the run's first element when an
  // element precedes it (the run to the left writes it); entry N's copies
  // in the element after the run
  const bool skip0 = el == 0 && ex > 0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c < nc) {
      const int64_t r = row_at(el, c);
#pragma unroll
      for (int h = 0; h < PR; ++h) {
        if (h == 0 && skip0) {
#pragma unroll
          for (int u = 1; u < VW; ++u) v[r + u] = o[u];
        } else {
          VT q;
#pragma unroll
          for (int u = 0; u < VW; ++u) q[u] = o[h * VW + u];
          *(VT*)&v[r + h * VW] = q;
        }
      }
      if (el == nel - 1 && xh) v[row_at(nel, c)] = o[N];
    }
}

// The pairwise order on a row tile: the run's elements' groups as box tiles
// form them (no group holds a box-boundary node), then zero the
// box-boundary entries of the rows the run owns.
template <typename T, typename ACC>
__device__ inline void gs_row_pairwise(gptr<T> v, const ProbDev& P, int e0, int nel) {
  constexpr int n = GS_ROW_N, N = n - 1, S = n + 1;
  gs_box_tile<T, ACC, true, N>(v, P, e0, nel);
  const int ne = P.box_ne, ne2 = ne * ne;
  int ex0, oy, oz;
  box_coords(e0, P, ex0, oy, oz);
  const bool ylo = oy == 0, yhi = oy + 1 < ne, zlo = oz == 0, zhi = oz + 1 < ne;
  for (int f = (int)threadIdx.x; f < nel * S * S * n; f += GS_THREADS) {
    const int i = f % n, r = f / n, sy = r % S, sz = (r / S) % S, el = r / (S * S);
    if (!row_held(sy, ylo, yhi) || !row_held(sz, zlo, zhi)) continue;
    const int ex = ex0 + el;
    const bool bnd = sy == 0 || sz == 0 || (sy == N && !yhi) || (sz == N && !zhi) ||
                     (i == 0 && ex == 0) || (i == N && ex + 1 == ne);
    if (bnd) {
      const int64_t ee = (int64_t)e0 + el + (sy == n ? ne : 0) + (sz == n ? ne2 : 0);
      v[ee * (n * n * n) + (sy & (n - 1)) * n + (sz & (n - 1)) * (n * n) + i] = T(0);
    }
  }
}

template <typename T, typename ACC, bool SOLVER, bool PAIRWISE = false>
__global__ void __launch_bounds__(GS_THREADS) gs_kernel(const Tile* __restrict__ tiles,
                                                        const ProbDev* __restrict__ probs,
                                                        GsApi api) {
  const GsPlan* plan;
  gptr<T> __restrict__ v;
  int bucket, first, count = GS_CHUNK;
  if constexpr (SOLVER) {
    // sigma = (p, A p)_c and alpha need only the operator kernel's partial
    // sums, not the gather-scatter: the first nfin workgroups finish them
    // while the others sum copies (nfin is a multiple of XCDS, so the tiles
    // keep their XCD placement)
    if ((int)blockIdx.x < api.nfin) {
      __shared__ double sred[16];
      if ((int)blockIdx.x < api.nprob) fin_sigma_step(probs[blockIdx.x], sred);
      return;
    }
    const int tb = (int)blockIdx.x - api.nfin;
    if (tb >= (int)gridDim.x - api.nfin - api.nz) {
      // z = dinv r where the learned z of this step was rejected
      const Tile t = api.ztiles[tb - ((int)gridDim.x - api.nfin - api.nz)];
      const ProbDev& P = probs[t.prob];
      const gptr<const State> st = gcast((const State*)P.st);
      if (st->done || !st->fb_pending) return;
      const gptr<const T> __restrict__ rr = gcast((const T*)P.r);
      const gptr<const T> __restrict__ dinv = gcast((const T*)P.dinv);
      gptr<T> __restrict__ z = gcast((T*)P.z);
#pragma unroll
      for (int q = 0; q < UPD_PER_THREAD; ++q) {
        const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
        if (i < P.nloc) z[i] = dinv[i] * rr[i];
      }
      return;
    }
    const Tile t = tiles[tb];
    const ProbDev& P = probs[t.prob];
    if (gcast(P.st)->done || (api.nz && gcast(P.st)->fb_pending)) return;
    plan = &P.gs;
    v = gcast((T*)(api.on_z ? P.z : P.w));
    bucket = t.aux;
    first = t.first;
    count = t.pad;
    if (bucket == -2) {  // box lattice at N = 7: row tiles
      if constexpr (PAIRWISE)
        gs_row_pairwise<T, ACC>(v, P, first, count);
      else
        gs_row_tile<T, ACC>(v, P, first, count);
      return;
    }
    if (bucket < 0) {  // box lattice at N = 15: each element's groups by index arithmetic
      gs_box_tile<T, ACC, PAIRWISE, 15>(v, P, first, count);
      return;
    }
  } else {
    plan = &api.plan;
    v = gcast((T*)api.v);
    bucket = api.bucket;
    first = blockIdx.x * GS_CHUNK;
  }
  const GsBucket bk = plan->bk[bucket];
  const gptr<const int> __restrict__ idx = gcast((const int*)plan->idx) + bk.off;
  const int m = bk.m;
  int g[GS_PER_THREAD];
  bool ok[GS_PER_THREAD];
#pragma unroll
  for (int q = 0; q < GS_PER_THREAD; ++q) {
    g[q] = first + q * GS_THREADS + threadIdx.x;
    ok[q] = g[q] < bk.ngroups && g[q] < first + count;
  }
  if (m == 0) {
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) v[idx[g[q]]] = T(0);
  } else if constexpr (PAIRWISE) {
    if (m > GS_PAIRWISE_MAXM) return;  // rejected on the host
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        const gptr<const int> gi = idx + (int64_t)g[q] * m;
        int ids[GS_PAIRWISE_MAXM];
        for (int k = 0; k < m; ++k) ids[k] = gi[k];
        gs_pairwise_group<T, ACC>(v, ids, m, gcast(plan->erank), plan->n3);
      }
  } else if (m == 2) {
    gi2_t ix[GS_PER_THREAD];
    T a0[GS_PER_THREAD], a1[GS_PER_THREAD];
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) ix[q] = ((gptr<const gi2_t>)idx)[g[q]];
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        a0[q] = v[ix[q].x];
        a1[q] = v[ix[q].y];
      }
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        const T val = (T)((ACC)a0[q] + (ACC)a1[q]);
        v[ix[q].x] = val;
        v[ix[q].y] = val;
      }
  } else if (m == 4) {
    gi4_t ix[GS_PER_THREAD];
    T a[GS_PER_THREAD][4];
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) ix[q] = ((gptr<const gi4_t>)idx)[g[q]];
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        a[q][0] = v[ix[q].x];
        a[q][1] = v[ix[q].y];
        a[q][2] = v[ix[q].z];
        a[q][3] = v[ix[q].w];
      }
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        const T val = (T)((((ACC)a[q][0] + (ACC)a[q][1]) + (ACC)a[q][2]) + (ACC)a[q][3]);
        v[ix[q].x] = val;
        v[ix[q].y] = val;
        v[ix[q].z] = val;
        v[ix[q].w] = val;
      }
  } else if (m == 8) {
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        const gi4_t i0 = ((gptr<const gi4_t>)idx)[2 * g[q]];
        const gi4_t i1 = ((gptr<const gi4_t>)idx)[2 * g[q] + 1];
        ACC s = (ACC)v[i0.x];
        s += (ACC)v[i0.y];
        s += (ACC)v[i0.z];
        s += (ACC)v[i0.w];
        s += (ACC)v[i1.x];
        s += (ACC)v[i1.y];
        s += (ACC)v[i1.z];
        s += (ACC)v[i1.w];
        const T val = (T)s;
        v[i0.x] = val; v[i0.y] = val; v[i0.z] = val; v[i0.w] = val;
        v[i1.x] = val; v[i1.y] = val; v[i1.z] = val; v[i1.w] = val;
      }
  } else {
#pragma unroll
    for (int q = 0; q < GS_PER_THREAD; ++q)
      if (ok[q]) {
        const gptr<const int> gi = idx + (int64_t)g[q] * m;
        ACC s = (ACC)v[gi[0]];
        for (int k = 1; k < m; ++k) s += (ACC)v[gi[k]];
        const T val = (T)s;
        for (int k = 0; k < m; ++k) v[gi[k]] = val;
      }
  }
}

// ------------------------------------------------------------ vector pass

template <typename T>
struct V4;
template <>
struct V4<float> {
  typedef float4 type;
};
template <>
struct V4<double> {
  typedef double4 type;
};


// Cache policy of the CG step on gfx950.  Per iteration the solve streams
// about 1.4 GB (FP32) through a 256 MB last-level cache (MALL).  Arrays read
// or written once per iteration and not again before the next iteration (G,
// dinv, multiplicity, x, r) use non-temporal accesses, so that they do not
// displace the vectors that are reused within the iteration (p and w from
// the operator kernel to the update, z from the update to the next operator
// kernel), and so that each kernel's dirty lines reach HBM during that
// kernel instead of being written back during the next one.
template <typename VT, typename T>
__device__ inline void st4_nt(T* dst, const VT& v) {
  typedef T E4 __attribute__((ext_vector_type(4)));
  E4 e = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(e, (E4*)dst);
}
template <typename VT, typename T>
__device__ inline VT ld4_nt(const T* src) {
  typedef T E4 __attribute__((ext_vector_type(4)));
  E4 e = __builtin_nontemporal_load((const E4*)src);
  VT v;
  v.x = e.x, v.y = e.y, v.z = e.z, v.w = e.w;
  return v;
}
__device__ inline uchar4 ld_u8x4_nt(const uint8_t* src) {
  const uint32_t m4 = __builtin_nontemporal_load((const uint32_t*)src);
  uchar4 m;
  m.x = m4 & 255, m.y = (m4 >> 8) & 255, m.z = (m4 >> 16) & 255, m.w = m4 >> 24;
  return m;
}

// Assembled w in the vector pass (box lattices, ProbDev::box_ne > 0).  The
// PCG step of such a problem has no gather-scatter launch for w: the vector
// pass forms QQ^T w and the Dirichlet mask from the operator's local w.  The
// copies of a node are the entries of the elements that share it: along
// each direction in which the node lies on an element face, the neighbour
// across that face, at the opposite face coordinate.  They are summed in
// FP64 in ascending local index, i.e. ascending element, which is the
// lexicographic order of the element offsets (dz, dy, dx) -- the order in
// which the gather-scatter kernel sums the node's group -- and rounded once,
// so every copy gets the same value and the iterates are bitwise those of
// the separate gather-scatter.  A thread's four entries i0..i0+3 lie in one
// row of one element (n = 8 or 16): the row's copies across y and z faces
// are whole rows (one 4-wide load each), and an x face adds one entry per
// such row at the row's first or last slot (never both: n >= 8).
//
// The index work, the loads and the sums of the assembly are split so that
// the vector pass can issue every load of a thread (its own streams and the
// neighbours') before it waits for any: BoxRows holds the clamped addresses
// (a copy that is not needed reads the thread's own row, which is valid) and
// the options, box_load issues the loads, box_sum forms the sums.
struct BoxRows {
  int64_t rs, ry, rz, ryz;  // entry a = 0 of the row in this element, across y, z, both
  int xoff;                 // offset of the x-face copy from a row's entry a = 0
  int a0;
  bool dir_row, xlo, xhi, xlo_dir, xhi_dir;
  bool hy, hz, ylo, zlo;    // copies across y / z faces; the neighbour is the lower one
};
template <typename VT, typename T>
struct BoxVals {
  typedef T E4 __attribute__((ext_vector_type(4)));
  E4 ry, rz, ryz;
  T xs, xy, xz, xyz;
};
// box == false (a problem that is not a box lattice, in a launch that
// assembles the others): every address is the thread's own entries, and
// box_sum returns the thread's own values
__device__ inline BoxRows box_rows(uint32_t i0, const ProbDev& P, bool box) {
  BoxRows R;
  const int ln = P.box_ln, n = 1 << ln, N = n - 1, ne = P.box_ne;
  const uint32_t e = i0 >> (3 * ln);
  const int node = (int)(i0 & ((1u << (3 * ln)) - 1u));
  const int a0 = node & N, row = node >> ln;
  const int b = row & N, c = row >> ln;
  // (ex, ey, ez) of e: quotients by a float reciprocal, corrected by one
  // step (e < 2^24, so the product is off by less than one)
  const int ne2 = ne * ne;
  int ez = (int)((float)e * P.box_rne2);
  ez -= ez * ne2 > (int)e;
  ez += (ez + 1) * ne2 <= (int)e;
  const int rem = (int)e - ez * ne2;
  int ey = (int)((float)rem * P.box_rne);
  ey -= ey * ne > rem;
  ey += (ey + 1) * ne <= rem;
  const int ex = rem - ey * ne;
  const int GL = ne * N;  // lattice index of the far boundary
  const int gy = ey * N + b, gz = ez * N + c, gx0 = ex * N + a0;
  R.a0 = a0;
  R.dir_row = gy == 0 || gy == GL || gz == 0 || gz == GL;
  R.xlo = a0 == 0;
  R.xhi = a0 + 3 == N;
  R.xlo_dir = R.xlo && gx0 == 0;
  R.xhi_dir = R.xhi && gx0 + 3 == GL;
  R.ylo = b == 0;
  R.zlo = c == 0;
  R.hy = !R.dir_row && (b == 0 || b == N);
  R.hz = !R.dir_row && (c == 0 || c == N);
  const int dy = R.ylo ? -1 : 1, cy = R.ylo ? N : 0;
  const int dz = R.zlo ? -1 : 1, cz = R.zlo ? N : 0;
  const int64_t n3 = (int64_t)1 << (3 * ln);
  R.rs = (int64_t)i0 - a0;
  const int64_t ey_e = (int64_t)e + dy * ne, ez_e = (int64_t)e + (int64_t)dz * ne2;
  const int64_t eyz_e = ez_e + dy * ne;
  R.ry = R.hy ? (ey_e << (3 * ln)) + ((int64_t)(cy + (c << ln)) << ln) : R.rs;
  R.rz = R.hz ? (ez_e << (3 * ln)) + ((int64_t)(b + (cz << ln)) << ln) : R.rs;
  R.ryz = (R.hy && R.hz) ? (eyz_e << (3 * ln)) + ((int64_t)(cy + (cz << ln)) << ln) : R.rs;
  const bool xl = R.xlo && !R.xlo_dir, xh = R.xhi && !R.xhi_dir;
  R.xoff = xl ? (int)(N - n3) : xh ? (int)n3 : a0;
  if (!box) {  // box_sum then returns the thread's own values
    R.rs = R.ry = R.rz = R.ryz = i0;
    R.a0 = 0;
    R.xoff = 0;
    R.dir_row = R.xlo = R.xhi = R.xlo_dir = R.xhi_dir = R.hy = R.hz = false;
  }
  return R;
}
template <typename T, typename VT>
__device__ inline void box_load(const gptr<const T> __restrict__ w, const BoxRows& R,
                                BoxVals<VT, T>& V) {
  typedef typename BoxVals<VT, T>::E4 E4;
  V.ry = *((const E4*)&w[R.ry + R.a0]);
  V.rz = *((const E4*)&w[R.rz + R.a0]);
  V.ryz = *((const E4*)&w[R.ryz + R.a0]);
  V.xs = w[R.rs + R.xoff];
  V.xy = w[R.ry + R.xoff];
  V.xz = w[R.rz + R.xoff];
  V.xyz = w[R.ryz + R.xoff];
}
// One copy's row in the running sums: its entries at the four slots and its
// x-face entry (added before slot 0 or after slot 3); first: the node's
// first copy (the sums start from it).
template <typename T>
__device__ inline void box_add(bool on, bool first, bool xl, bool xh, T r0, T r1, T r2, T r3,
                               T xv, double& s0, double& s1, double& s2, double& s3) {
  double t0 = (double)r0;
  if (xl) t0 = (first ? (double)xv : s0 + (double)xv) + t0;
  else t0 = first ? t0 : s0 + t0;
  const double t1 = first ? (double)r1 : s1 + (double)r1;
  const double t2 = first ? (double)r2 : s2 + (double)r2;
  double t3 = first ? (double)r3 : s3 + (double)r3;
  if (xh) t3 += (double)xv;
  s0 = on ? t0 : s0;
  s1 = on ? t1 : s1;
  s2 = on ? t2 : s2;
  s3 = on ? t3 : s3;
}
// wv: the thread's own four local values on entry, the assembled ones on return
template <typename T, typename VT>
__device__ inline void box_sum(const BoxRows& R, const BoxVals<VT, T>& V, VT& wv) {
  if (R.dir_row) {
    wv.x = T(0), wv.y = T(0), wv.z = T(0), wv.w = T(0);
    return;
  }
  const T w0 = wv.x, w1 = wv.y, w2 = wv.z, w3 = wv.w;
  const bool xl = R.xlo && !R.xlo_dir, xh = R.xhi && !R.xhi_dir;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  // rows in ascending element order, (dz, dy) lexicographic: the lower
  // neighbour before this element, the upper one after; at each position one
  // of the four rows (this element's, across y, across z, across both)
#pragma unroll
  for (int qz = 0; qz < 2; ++qz)
#pragma unroll
    for (int qy = 0; qy < 2; ++qy) {
      const bool zn = R.hz && (R.zlo ? qz == 0 : qz == 1);
      const bool yn = R.hy && (R.ylo ? qy == 0 : qy == 1);
      const bool take = (qz == 0 || R.hz) && (qy == 0 || R.hy);
      const bool first = qz == 0 && qy == 0;
      box_add<T>(take && !zn && !yn, first, xl, xh, w0, w1, w2, w3, V.xs, s0, s1, s2, s3);
      box_add<T>(take && !zn && yn, first, xl, xh, V.ry.x, V.ry.y, V.ry.z, V.ry.w, V.xy, s0, s1,
                 s2, s3);
      box_add<T>(take && zn && !yn, first, xl, xh, V.rz.x, V.rz.y, V.rz.z, V.rz.w, V.xz, s0, s1,
                 s2, s3);
      box_add<T>(take && zn && yn, first, xl, xh, V.ryz.x, V.ryz.y, V.ryz.z, V.ryz.w, V.xyz, s0,
                 s1, s2, s3);
    }
  wv.x = R.xlo_dir ? T(0) : (T)s0;
  wv.y = (T)s1;
  wv.z = (T)s2;
  wv.w = R.xhi_dir ? T(0) : (T)s3;
}

// PC: 0 identity, 1 Jacobi, -1 none (z left alone; flexible CG computes it)
// x += alpha p; r -= alpha w; z = M^-1 r; partials (r,z)_c and (r,r)_c.
// Each thread handles UPD_PER_THREAD entries as 4-wide vectors when the
// problem's entry count is a multiple of 4, else one by one (decided per
// problem, so a problem is reduced the same way alone or in a batch).
// par: -1 x += alpha p (p updated in place by the operator kernel); with two
// direction buffers, 0 (even step) leaves x for the next step and records
// alpha as pending, 1 (odd step) adds alpha_prev p (the even step's
// direction, in p) and then alpha p_alt: the same two roundings, in the same
// order, as two steps of the first form.
// ASM: box-lattice problems assemble w here (box_rows / box_load /
// box_sum); the others read the w their gather-scatter launch assembled.
template <typename T, int DM, int PC, bool ASM>
__global__ void __launch_bounds__(UPD_THREADS) update_kernel(const Tile* __restrict__ tiles,
                                                             const ProbDev* __restrict__ probs,
                                                             int par) {
  __shared__ double sred[16];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  const gptr<State> stp = gcast(P.st);
  if (stp->done) return;
  const T alpha = (T)stp->alpha;
  const T alpha0 = par == 1 ? (T)stp->alpha_prev : T(0);
  if (par >= 0 && t.first == 0 && threadIdx.x == 0) {
    // read only by later launches (the next step's update, the host)
    if (par == 0) stp->alpha_prev = stp->alpha;
    stp->x_pending = par == 0 ? 1 : 0;
  }
  gptr<T> __restrict__ x = gcast((T*)P.x);
  gptr<T> __restrict__ r = gcast((T*)P.r);
  gptr<T> __restrict__ z = gcast((T*)P.z);
  const gptr<const T> __restrict__ p = gcast((const T*)P.p);
  const gptr<const T> __restrict__ p1 = gcast((const T*)(par == 1 ? P.p_alt : P.p));
  const gptr<const T> __restrict__ w = gcast((const T*)P.w);
  const gptr<const T> __restrict__ dinv = gcast((const T*)P.dinv);
  const gptr<const uint8_t> __restrict__ mult = gcast(P.mult);
  DotAcc<DM> rz, rr;
  const bool asm_box = ASM && P.box_ne > 0;
  if ((P.nloc & 3) == 0) {
    typedef typename V4<T>::type VT;
#pragma unroll
    for (int q = 0; q < UPD_PER_THREAD / 4; ++q) {
      const int64_t v = (int64_t)t.first / 4 + q * UPD_THREADS + threadIdx.x;
      // box assembly: the neighbour loads issued beside the thread's own,
      // with no branch around them (a copy that is not needed, or an entry
      // past the end, reads a valid address of the thread's own)
      BoxRows br;
      BoxVals<VT, T> bv;
      if constexpr (ASM) {
        br = box_rows((uint32_t)(4 * (4 * v < P.nloc ? v : 0)), P, asm_box);
        box_load<T, VT>(w, br, bv);
      }
      if (4 * v < P.nloc) {
        VT rv = ld4_nt<VT>((const T*)&((const VT*)r)[v]), wv = ((const VT*)w)[v];
        const uchar4 mv = ld_u8x4_nt((const uint8_t*)&((const uchar4*)mult)[v]);
        if (par != 0) {
          VT xv = ld4_nt<VT>((const T*)&((const VT*)x)[v]);
          if (par == 1) {
            const VT pv = ((const VT*)p)[v];
            xv.x += alpha0 * pv.x; xv.y += alpha0 * pv.y; xv.z += alpha0 * pv.z;
            xv.w += alpha0 * pv.w;
          }
          const VT pv = ((const VT*)p1)[v];
          xv.x += alpha * pv.x; xv.y += alpha * pv.y; xv.z += alpha * pv.z; xv.w += alpha * pv.w;
          st4_nt<VT>((T*)&((VT*)x)[v], xv);
        }
        // (the identity for a problem that is not a box lattice)
        if constexpr (ASM) box_sum<T, VT>(br, bv, wv);
        rv.x -= alpha * wv.x; rv.y -= alpha * wv.y; rv.z -= alpha * wv.z; rv.w -= alpha * wv.w;
        st4_nt<VT>((T*)&((VT*)r)[v], rv);
        const double c0 = cweight(mv.x), c1 = cweight(mv.y), c2 = cweight(mv.z),
                     c3 = cweight(mv.w);
        rr.addw(rv.x, c0, rv.x);
        rr.addw(rv.y, c1, rv.y);
        rr.addw(rv.z, c2, rv.z);
        rr.addw(rv.w, c3, rv.w);
        if constexpr (PC >= 0) {
          VT zv = rv;
          if constexpr (PC == 1) {
            const VT dv = ld4_nt<VT>((const T*)&((const VT*)dinv)[v]);
            zv.x = dv.x * rv.x; zv.y = dv.y * rv.y; zv.z = dv.z * rv.z; zv.w = dv.w * rv.w;
          }
          ((VT*)z)[v] = zv;
          rz.addw(rv.x, c0, zv.x);
          rz.addw(rv.y, c1, zv.y);
          rz.addw(rv.z, c2, zv.z);
          rz.addw(rv.w, c3, zv.w);
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < UPD_PER_THREAD; ++q) {
      const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
      if (i < P.nloc) {
        if (par != 0) {
          T xv = x[i];
          if (par == 1) xv += alpha0 * p[i];
          xv += alpha * p1[i];
          x[i] = xv;
        }
        const T rv = r[i] - alpha * w[i];
        r[i] = rv;
        const double c = cweight(mult[i]);
        rr.addw(rv, c, rv);
        if constexpr (PC >= 0) {
          const T zv = (PC == 1) ? dinv[i] * rv : rv;
          z[i] = zv;
          rz.addw(rv, c, zv);
        }
      }
    }
  }
  const double s0 = rz.block(sred);
  const double s1 = rr.block(sred);
  if (threadIdx.x == 0) {
    const int b = t.first / UPD_CHUNK;
    gcast(P.part_u0)[b] = s0;
    gcast(P.part_u1)[b] = s1;
  }
}

// start of a solve: r = rhs64 * scale (cast to T), x = x0 or 0, p = 0,
// z = M^-1 r, partials (r,z)_c and (r,r)_c
template <typename T, int DM, int PC>
__global__ void init_kernel(const Tile* __restrict__ tiles, const ProbDev* __restrict__ probs,
                            const double* __restrict__ x0) {
  __shared__ double sred[16];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  if (gcast(P.st)->done) return;
  gptr<T> __restrict__ x = gcast((T*)P.x);
  gptr<T> __restrict__ r = gcast((T*)P.r);
  gptr<T> __restrict__ z = gcast((T*)P.z);
  gptr<T> __restrict__ p = gcast((T*)P.p);
  const gptr<const T> __restrict__ dinv = gcast((const T*)P.dinv);
  const double scale = P.rhs_scale;
  DotAcc<DM> rz, rr;
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
    if (i < P.nloc) {
      const T rv = (T)(gcast(P.rhs64)[i] * scale);
      r[i] = rv;
      x[i] = x0 ? (T)x0[i] : T(0);
      p[i] = T(0);
      if (P.p_alt) gcast((T*)P.p_alt)[i] = T(0);
      const double c = cweight(gcast(P.mult)[i]);
      rr.addw(rv, c, rv);
      if constexpr (PC >= 0) {
        const T zv = (PC == 1) ? dinv[i] * rv : rv;
        z[i] = zv;
        rz.addw(rv, c, zv);
      }
    }
  }
  const double s0 = rz.block(sred);
  const double s1 = rr.block(sred);
  if (threadIdx.x == 0) {
    const int b = t.first / UPD_CHUNK;
    gcast(P.part_u0)[b] = s0;
    gcast(P.part_u1)[b] = s1;
  }
}

// ------------------------------------------------------------ scalar stages
// sum of parts[0..n) in a fixed order by one workgroup of FIN_THREADS:
// thread t adds parts[t + k*FIN_THREADS] into accumulator k % 8 (eight
// independent chains keep eight loads in flight), then the accumulators,
// then the block.  The order depends only on n.
template <int NT>
__device__ inline double fixed_sum(const gptr<const double> __restrict__ parts, int n,
                                   double* sred) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int q = threadIdx.x;
  for (; q + 7 * NT < n; q += 8 * NT) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += parts[q + k * NT];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (q + k * NT < n) a[k] += parts[q + k * NT];
  const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum(s, sred);
}

// fixed_sum of two arrays of n partials at once (the same order for each,
// so the results are bitwise those of two fixed_sum calls, in one pass of
// loads and one block reduction); sred holds 32 doubles; thread 0 gets both
template <int NT>
__device__ inline void fixed_sum2(const gptr<const double> __restrict__ p0,
                                  const gptr<const double> __restrict__ p1, int n, double* sred,
                                  double& s0, double& s1) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0}, b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int q = threadIdx.x;
  for (; q + 7 * NT < n; q += 8 * NT) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] += p0[q + k * NT];
      b[k] += p1[q + k * NT];
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (q + k * NT < n) {
      a[k] += p0[q + k * NT];
      b[k] += p1[q + k * NT];
    }
  double sa = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  double sb = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
  for (int off = 32; off > 0; off >>= 1) {
    sa += __shfl_down(sa, off, 64);
    sb += __shfl_down(sb, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    sred[wid] = sa;
    sred[16 + wid] = sb;
  }
  __syncthreads();
  s0 = s1 = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) {
      s0 += sred[w];
      s1 += sred[16 + w];
    }
}

// sigma = (p, A p)_c; alpha = rho / sigma; breakdown if sigma <= 0 or not
// finite.  Run by a workgroup of the gather-scatter launch of the same step.
__device__ inline void fin_sigma_step(const ProbDev& P, double* sred) {
  const gptr<State> st = gcast(P.st);
  if (st->done) return;
  const gptr<const double> pa = gcast((const double*)P.part_ax);
  const double sigma = P.dm == DOT_F64 ? fixed_sum<GS_THREADS>(pa, P.nblk_ax, sred)
                                       : dot_finish<GS_THREADS>(P.dm, pa, P.nblk_ax, sred);
  if (threadIdx.x == 0) {
    st->sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
      st->done = 1;
      st->reason = MXSEM_BREAKDOWN;
    } else {
      st->alpha = st->rho / sigma;
    }
  }
}

// After the vector pass.  mode 0 (PCG step): convergence / max-iteration /
// stagnation tests, then beta = rho'/rho.  mode 1: start of a PCG solve.
// mode 2 (flexible CG step): the tests only (beta comes later).  mode 3:
// start of a flexible CG solve (rho comes later).
// End-of-step tests on the recursive residual rr = (r,r)_c: iteration
// count, convergence, non-finite residual, iteration limit, stagnation.
// Returns false when the problem is done (reason set).
__device__ inline bool step_test(const gptr<State> st, double rr) {
  st->rr = rr;
  const int it = st->iter + 1;
  st->iter = it;
  const double res = sqrt(rr / st->bb);
  st->res = res;
  if (st->history) gcast(st->history)[it] = res;
  int reason = 0;
  if (rr <= st->tol2 * st->bb)
    reason = MXSEM_CONVERGED;
  else if (!isfinite(rr))
    reason = MXSEM_BREAKDOWN;
  else if (it >= st->maxit)
    reason = MXSEM_MAX_ITER;
  else if (res < 0.9 * st->best) {
    st->best = res;
    st->since = 0;
  } else if (++st->since >= STAG_WINDOW) {
    reason = MXSEM_STAGNATED;
  }
  if (reason) {
    st->done = 1;
    st->reason = reason;
    return false;
  }
  return true;
}

__global__ void fin_rho_kernel(const ProbDev* __restrict__ probs, int mode) {
  __shared__ double sred[32];
  const ProbDev& P = probs[blockIdx.x];
  const gptr<State> st = gcast(P.st);
  if (st->done) return;
  const gptr<const double> p0 = gcast((const double*)P.part_u0);
  const gptr<const double> p1 = gcast((const double*)P.part_u1);
  double rz, rr;
  if (P.dm == DOT_F64) {
    fixed_sum2<FIN_THREADS>(p0, p1, P.nblk_upd, sred, rz, rr);
  } else {
    rz = dot_finish<FIN_THREADS>(P.dm, p0, P.nblk_upd, sred);
    rr = dot_finish<FIN_THREADS>(P.dm, p1, P.nblk_upd, sred);
  }
  if (threadIdx.x != 0) return;
  st->rr = rr;
  if (mode == 1 || mode == 3) {
    st->bb = rr;
    if (mode == 1) st->rho = rz;
    st->beta = 0.0;
    st->iter = 0;
    st->since = 0;
    st->best = 1.0;
    st->res = rr > 0.0 ? 1.0 : 0.0;
    if (st->history) gcast(st->history)[0] = st->res;
    if (!(rr > 0.0)) {
      st->done = 1;
      st->reason = MXSEM_CONVERGED;
    }
    return;
  }
  if (!step_test(st, rr)) return;
  if (mode == 0) {
    st->beta = rz / st->rho;
    st->rho = rz;
  }
}

// ------------------------------------------------------------ flexible CG
// z = M^-1 r (Jacobi or identity) for flexible CG steps; with only_pending,
// only for problems whose learned z was rejected this step.
template <typename T>
__global__ void __launch_bounds__(UPD_THREADS) zpc_kernel(const Tile* __restrict__ tiles,
                                                          const ProbDev* __restrict__ probs,
                                                          int pc) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  if (gcast(P.st)->done) return;
  const gptr<const T> __restrict__ r = gcast((const T*)P.r);
  const gptr<const T> __restrict__ dinv = gcast((const T*)P.dinv);
  gptr<T> __restrict__ z = gcast((T*)P.z);
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
    if (i < P.nloc) z[i] = pc == MXSEM_PC_IDENTITY ? r[i] : dinv[i] * r[i];
  }
}

// partials (r,z)_c -> part_u0 and (z,w)_c -> part_u2 (w = A p of this step)
template <typename T, typename ACC>
__global__ void __launch_bounds__(UPD_THREADS) fcg_dots_kernel(const Tile* __restrict__ tiles,
                                                               const ProbDev* __restrict__ probs) {
  __shared__ ACC sred[16];
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  if (gcast(P.st)->done) return;
  const gptr<const T> __restrict__ r = gcast((const T*)P.r);
  const gptr<const T> __restrict__ z = gcast((const T*)P.z);
  const gptr<const T> __restrict__ w = gcast((const T*)P.w);
  ACC rz = ACC(0), zw = ACC(0);
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
    if (i < P.nloc) {
      const ACC c = (ACC)cweight(gcast(P.mult)[i]);
      rz += (ACC)r[i] * c * (ACC)z[i];
      zw += (ACC)z[i] * c * (ACC)w[i];
    }
  }
  ACC s0 = block_sum(rz, sred);
  ACC s1 = block_sum(zw, sred);
  if (threadIdx.x == 0) {
    const int b = t.first / UPD_CHUNK;
    gcast(P.part_u0)[b] = (double)s0;
    gcast(P.part_u2)[b] = (double)s1;
  }
}

// beta = -(z, A p_old)_c / (p_old, A p_old)_c, rho = (r,z)_c; init: first
// z of a solve (beta = 0).  With dots (learned step), first the end-of-step
// tests on (r,r)_c (not at init), then the learned z is taken unless it is
// not a descent direction ((r,z)_c <= 0 or non-finite dots), else the
// Jacobi candidate: fb_pending tells the following assembly launch to write
// dinv r, and the fallback is counted.
__global__ void fin_beta_kernel(const ProbDev* __restrict__ probs, int init,
                                const double* __restrict__ dots, int ndots, int dstride) {
  __shared__ double sred[16];
  const ProbDev& P = probs[blockIdx.x];
  const gptr<State> st = gcast(P.st);
  if (st->done) return;
  if (dots) {
    // learned step: the forward summed the dots of both candidates and,
    // past the first step, (r,r)_c of the updated residual
    double d[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) d[k] = fixed_sum<FIN_THREADS>(gcast(dots + k * dstride), ndots, sred);
    if (threadIdx.x != 0) return;
    if (!init && !step_test(st, d[4])) return;
    const bool reject = !(d[0] > 0.0) || !isfinite(d[0]) || (!init && !isfinite(d[1]));
    st->fb_pending = reject ? 1 : 0;
    if (reject) st->fallback += 1;
    st->rho = reject ? d[2] : d[0];
    st->beta = init ? 0.0 : -(reject ? d[3] : d[1]) / st->sigma;
    return;
  }
  double rz = fixed_sum<FIN_THREADS>(gcast((const double*)P.part_u0), P.nblk_upd, sred);
  double zw = fixed_sum<FIN_THREADS>(gcast((const double*)P.part_u2), P.nblk_upd, sred);
  if (threadIdx.x != 0) return;
  st->rho = rz;
  st->beta = init ? 0.0 : -zw / st->sigma;
}

// ------------------------------------------------------------ API kernels
template <typename T, int DM>
__global__ void dot_kernel(const T* __restrict__ a, const T* __restrict__ b,
                           const uint8_t* __restrict__ mult, int64_t n, double* __restrict__ part) {
  __shared__ double sred[16];
  DotAcc<DM> s;
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)blockIdx.x * UPD_CHUNK + q * UPD_THREADS + threadIdx.x;
    if (i < n) s.addw(a[i], cweight(mult[i]), b[i]);
  }
  const double t = s.block(sred);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void final_sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out,
                                 int dm) {
  __shared__ double sred[16];
  const double s = dm == DOT_F64 ? fixed_sum<FIN_THREADS>(gcast(part), n, sred)
                                 : dot_finish<FIN_THREADS>(dm, gcast(part), n, sred);
  if (threadIdx.x == 0) *out = s;
}

template <typename T>
__global__ void precond_kernel(const T* __restrict__ r, T* __restrict__ z,
                               const T* __restrict__ dinv, const int* __restrict__ mask_idx,
                               int64_t n, int pc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = pc == 1 ? dinv[i] * r[i] : r[i];
  (void)mask_idx;
}

// r64 = b - w64, partial (r,r)_c
__global__ void residual_kernel(const double* __restrict__ b, const double* __restrict__ w,
                                double* __restrict__ r, const uint8_t* __restrict__ mult,
                                int64_t n, double* __restrict__ part) {
  __shared__ double sred[16];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)blockIdx.x * UPD_CHUNK + q * UPD_THREADS + threadIdx.x;
    if (i < n) {
      const double v = b[i] - w[i];
      r[i] = v;
      s += v * cweight(mult[i]) * v;
    }
  }
  double t = block_sum(s, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x64 = x64 * keep + s * (double) xT
template <typename T>
__global__ void axpy_cast_kernel(double* __restrict__ x64, const T* __restrict__ xT, double s,
                                 double keep, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x64[i] = (keep == 0.0 ? 0.0 : keep * x64[i]) + s * (double)xT[i];
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

__global__ void mass_kernel(const double* __restrict__ B, const double* __restrict__ f,
                            double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = B[i] * f[i];
}

template <typename TD, typename TS>
__global__ void cast_kernel(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (TD)s[i];
}

__global__ void cast_bf16_kernel(bf16_t* __restrict__ d, const double* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = float_to_bf16((float)s[i]);
}

// FP32 / BF16 copies of the geometric factors in the node-interleaved
// layout the operator kernels read: per local node (e, p) the components
// rr, rs, rt, ss of G as one 4-vector, then (after all E n^3 of those) st,
// tt as one 2-vector.  A thread then loads its node's six factors with two
// coalesced vector loads instead of six scalar ones.
template <typename TG>
__global__ void cast_g_split_kernel(TG* __restrict__ d, const double* __restrict__ G64, int E,
                                    int n3) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nloc = (int64_t)E * n3;
  if (node >= nloc) return;
  const int64_t e = node / n3, p = node - e * n3;
  const double* g = G64 + e * 6 * n3 + p;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if constexpr (sizeof(TG) == 2)
      d[node * 4 + c] = float_to_bf16((float)g[c * n3]);
    else
      d[node * 4 + c] = (TG)g[c * n3];
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if constexpr (sizeof(TG) == 2)
      d[4 * nloc + node * 2 + c] = float_to_bf16((float)g[(4 + c) * n3]);
    else
      d[4 * nloc + node * 2 + c] = (TG)g[(4 + c) * n3];
  }
}

// ------------------------------------------------------------ host launchers
static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// API gather-scatter: free buckets, then either the Dirichlet-group
// buckets (no mask) or the mask list.  io/acc: MXSEM_F64 / MXSEM_F32.
hipError_t launch_gs_apply(int prec_io, int prec_acc, void* v, const GsPlan& plan, bool mask,
                           hipStream_t s, bool pairwise) {
  const int last = mask ? plan.nfree : plan.nall;
  for (int bkt = 0; bkt <= plan.nall; ++bkt) {
    if (bkt >= last && !(mask && bkt == plan.nall)) continue;
    const int ng = plan.bk[bkt].ngroups;
    if (ng == 0) continue;
    GsApi a{v, plan, bkt, 0};
    dim3 g(nblk(ng, GS_CHUNK)), b(GS_THREADS);
    if (pairwise) {
      if (prec_io != MXSEM_F32) return hipErrorInvalidValue;
      if (prec_acc == MXSEM_F64)
        hipLaunchKernelGGL((gs_kernel<float, double, false, true>), g, b, 0, s, nullptr, nullptr, a);
      else
        hipLaunchKernelGGL((gs_kernel<float, float, false, true>), g, b, 0, s, nullptr, nullptr, a);
    } else if (prec_io == MXSEM_F64 && prec_acc == MXSEM_F64)
      hipLaunchKernelGGL((gs_kernel<double, double, false>), g, b, 0, s, nullptr, nullptr, a);
    else if (prec_io == MXSEM_F64 && prec_acc == MXSEM_F32)
      hipLaunchKernelGGL((gs_kernel<double, float, false>), g, b, 0, s, nullptr, nullptr, a);
    else if (prec_io == MXSEM_F32 && prec_acc == MXSEM_F64)
      hipLaunchKernelGGL((gs_kernel<float, double, false>), g, b, 0, s, nullptr, nullptr, a);
    else if (prec_io == MXSEM_F32 && prec_acc == MXSEM_F32)
      hipLaunchKernelGGL((gs_kernel<float, float, false>), g, b, 0, s, nullptr, nullptr, a);
    else
      return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// vector precision: 0 FP64, 1 FP32 (FP64 accumulation), 3 FP32 (FP32 accumulation)
hipError_t launch_gs_solver(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                            hipStream_t s, bool on_z, int sigma_probs, const Tile* ztiles, int nz,
                            bool pairwise) {
  static_assert(GS_THREADS == UPD_THREADS, "the Jacobi-z workgroups use the vector-pass tiles");
  const int nfin = ((sigma_probs + XCDS - 1) / XCDS) * XCDS;
  if (ntiles + nfin + nz == 0) return hipSuccess;
  dim3 g(nfin + ntiles + nz), b(GS_THREADS);
  GsApi a{};
  a.on_z = on_z ? 1 : 0;
  a.nfin = nfin;
  a.nprob = sigma_probs;
  a.ztiles = ztiles;
  a.nz = ztiles ? nz : 0;
  if (pairwise && (vprec == 0 || on_z || nz)) return hipErrorInvalidValue;
  if (pairwise && vprec == 1)
    hipLaunchKernelGGL((gs_kernel<float, double, true, true>), g, b, 0, s, tiles, probs, a);
  else if (pairwise)
    hipLaunchKernelGGL((gs_kernel<float, float, true, true>), g, b, 0, s, tiles, probs, a);
  else if (vprec == 0)
    hipLaunchKernelGGL((gs_kernel<double, double, true>), g, b, 0, s, tiles, probs, a);
  else if (vprec == 1)
    hipLaunchKernelGGL((gs_kernel<float, double, true>), g, b, 0, s, tiles, probs, a);
  else
    hipLaunchKernelGGL((gs_kernel<float, float, true>), g, b, 0, s, tiles, probs, a);
  return hipGetLastError();
}

template <typename T, int DM, bool ASM>
static void upd_dispatch2(int pc, dim3 g, dim3 b, hipStream_t s, const Tile* tiles,
                          const ProbDev* probs, int par) {
  if (pc == MXSEM_PC_JACOBI)
    hipLaunchKernelGGL((update_kernel<T, DM, 1, ASM>), g, b, 0, s, tiles, probs, par);
  else if (pc == MXSEM_PC_IDENTITY)
    hipLaunchKernelGGL((update_kernel<T, DM, 0, ASM>), g, b, 0, s, tiles, probs, par);
  else
    hipLaunchKernelGGL((update_kernel<T, DM, -1, ASM>), g, b, 0, s, tiles, probs, par);
}
template <typename T, int DM>
static void upd_dispatch(int pc, dim3 g, dim3 b, hipStream_t s, const Tile* tiles,
                         const ProbDev* probs, int par, int asm_w) {
  if (asm_w)
    upd_dispatch2<T, DM, true>(pc, g, b, s, tiles, probs, par);
  else
    upd_dispatch2<T, DM, false>(pc, g, b, s, tiles, probs, par);
}

// dm: DotMode of the dots (FP64 vectors: DOT_F64 only)
hipError_t launch_update(int vprec, int pc, const Tile* tiles, int ntiles, const ProbDev* probs,
                         hipStream_t s, int dm, int par, bool asm_w) {
  dim3 g(ntiles), b(UPD_THREADS);
  if (vprec == 0 && dm != DOT_F64) return hipErrorInvalidValue;
  if (par < -1 || par > 1) return hipErrorInvalidValue;
  if (asm_w && vprec != 0 && vprec != 1) return hipErrorInvalidValue;  // FP64 sums only
  const int aw = asm_w ? 1 : 0;
  if (vprec == 0) upd_dispatch<double, DOT_F64>(pc, g, b, s, tiles, probs, par, aw);
  else if (dm == DOT_F64) upd_dispatch<float, DOT_F64>(pc, g, b, s, tiles, probs, par, aw);
  else if (dm == DOT_F32) upd_dispatch<float, DOT_F32>(pc, g, b, s, tiles, probs, par, aw);
  else if (dm == DOT_DOT2) upd_dispatch<float, DOT_DOT2>(pc, g, b, s, tiles, probs, par, aw);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// x += alpha_prev p where the problem's last step left x pending
template <typename T>
__global__ void __launch_bounds__(UPD_THREADS) x_pending_kernel(const Tile* __restrict__ tiles,
                                                                const ProbDev* __restrict__ probs) {
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  const gptr<const State> st = gcast((const State*)P.st);
  if (!st->x_pending) return;
  const T a = (T)st->alpha_prev;
  gptr<T> __restrict__ x = gcast((T*)P.x);
  const gptr<const T> __restrict__ p = gcast((const T*)P.p);
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t i = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
    if (i < P.nloc) x[i] += a * p[i];
  }
}

hipError_t launch_x_pending(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                            hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  if (vprec == 0)
    hipLaunchKernelGGL((x_pending_kernel<double>), dim3(ntiles), dim3(UPD_THREADS), 0, s, tiles,
                       probs);
  else
    hipLaunchKernelGGL((x_pending_kernel<float>), dim3(ntiles), dim3(UPD_THREADS), 0, s, tiles,
                       probs);
  return hipGetLastError();
}

template <typename T, int DM>
static void init_dispatch(int pc, dim3 g, dim3 b, hipStream_t s, const Tile* tiles,
                          const ProbDev* probs, const double* x0) {
  if (pc == MXSEM_PC_JACOBI)
    hipLaunchKernelGGL((init_kernel<T, DM, 1>), g, b, 0, s, tiles, probs, x0);
  else if (pc == MXSEM_PC_IDENTITY)
    hipLaunchKernelGGL((init_kernel<T, DM, 0>), g, b, 0, s, tiles, probs, x0);
  else
    hipLaunchKernelGGL((init_kernel<T, DM, -1>), g, b, 0, s, tiles, probs, x0);
}

hipError_t launch_init(int vprec, int pc, const Tile* tiles, int ntiles, const ProbDev* probs,
                       const double* x0, hipStream_t s, int dm) {
  dim3 g(ntiles), b(UPD_THREADS);
  if (vprec == 0 && dm != DOT_F64) return hipErrorInvalidValue;
  if (vprec == 0) init_dispatch<double, DOT_F64>(pc, g, b, s, tiles, probs, x0);
  else if (dm == DOT_F64) init_dispatch<float, DOT_F64>(pc, g, b, s, tiles, probs, x0);
  else if (dm == DOT_F32) init_dispatch<float, DOT_F32>(pc, g, b, s, tiles, probs, x0);
  else if (dm == DOT_DOT2) init_dispatch<float, DOT_DOT2>(pc, g, b, s, tiles, probs, x0);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fin_rho(const ProbDev* probs, int nprob, int mode, hipStream_t s) {
  hipLaunchKernelGGL(fin_rho_kernel, dim3(nprob), dim3(FIN_THREADS), 0, s, probs, mode);
  return hipGetLastError();
}

hipError_t launch_zpc(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs, int pc,
                      hipStream_t s) {
  if (vprec == 0)
    hipLaunchKernelGGL((zpc_kernel<double>), dim3(ntiles), dim3(UPD_THREADS), 0, s, tiles, probs,
                       pc);
  else
    hipLaunchKernelGGL((zpc_kernel<float>), dim3(ntiles), dim3(UPD_THREADS), 0, s, tiles, probs,
                       pc);
  return hipGetLastError();
}

hipError_t launch_fcg_dots(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                           hipStream_t s) {
  if (vprec == 0)
    hipLaunchKernelGGL((fcg_dots_kernel<double, double>), dim3(ntiles), dim3(UPD_THREADS), 0, s,
                       tiles, probs);
  else if (vprec == 1)
    hipLaunchKernelGGL((fcg_dots_kernel<float, double>), dim3(ntiles), dim3(UPD_THREADS), 0, s,
                       tiles, probs);
  else
    hipLaunchKernelGGL((fcg_dots_kernel<float, float>), dim3(ntiles), dim3(UPD_THREADS), 0, s,
                       tiles, probs);
  return hipGetLastError();
}

hipError_t launch_fin_beta(const ProbDev* probs, int nprob, int init, hipStream_t s,
                           const double* dots, int ndots, int dstride) {
  hipLaunchKernelGGL(fin_beta_kernel, dim3(nprob), dim3(FIN_THREADS), 0, s, probs, init,
                     dots, ndots, dstride);
  return hipGetLastError();
}

// dm: DotMode (FP64 inputs: DOT_F64 only)
hipError_t launch_dot(int prec, const void* a, const void* b, const uint8_t* mult, int64_t n,
                      double* part, double* out, hipStream_t s, int dm) {
  const unsigned nb = nblk(n, UPD_CHUNK);
  dim3 g(nb), t(UPD_THREADS);
  const float* af = (const float*)a;
  const float* bf = (const float*)b;
  if (prec == MXSEM_F64 && dm == DOT_F64)
    hipLaunchKernelGGL((dot_kernel<double, DOT_F64>), g, t, 0, s, (const double*)a,
                       (const double*)b, mult, n, part);
  else if (prec == MXSEM_F64)
    return hipErrorInvalidValue;
  else if (dm == DOT_F64)
    hipLaunchKernelGGL((dot_kernel<float, DOT_F64>), g, t, 0, s, af, bf, mult, n, part);
  else if (dm == DOT_F32)
    hipLaunchKernelGGL((dot_kernel<float, DOT_F32>), g, t, 0, s, af, bf, mult, n, part);
  else if (dm == DOT_DOT2)
    hipLaunchKernelGGL((dot_kernel<float, DOT_DOT2>), g, t, 0, s, af, bf, mult, n, part);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(FIN_THREADS), 0, s, part, (int)nb, out, dm);
  return hipGetLastError();
}

hipError_t launch_precond(int prec, int pc, const void* r, void* z, const void* dinv, int64_t n,
                          hipStream_t s) {
  const unsigned nb = nblk(n, 256);
  if (prec == MXSEM_F64)
    hipLaunchKernelGGL((precond_kernel<double>), dim3(nb), dim3(256), 0, s, (const double*)r,
                       (double*)z, (const double*)dinv, nullptr, n, pc);
  else
    hipLaunchKernelGGL((precond_kernel<float>), dim3(nb), dim3(256), 0, s, (const float*)r,
                       (float*)z, (const float*)dinv, nullptr, n, pc);
  return hipGetLastError();
}

hipError_t launch_residual(const double* b, const double* w, double* r, const uint8_t* mult,
                           int64_t n, double* part, double* out, hipStream_t s) {
  const unsigned nb = nblk(n, UPD_CHUNK);
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(UPD_THREADS), 0, s, b, w, r, mult, n, part);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(FIN_THREADS), 0, s, part, (int)nb, out,
                     (int)DOT_F64);
  return hipGetLastError();
}

hipError_t launch_axpy_cast(int vprec, double* x64, const void* xT, double sc, double keep,
                            int64_t n, hipStream_t s) {
  const unsigned nb = nblk(n, 256);
  if (vprec == 0)
    hipLaunchKernelGGL((axpy_cast_kernel<double>), dim3(nb), dim3(256), 0, s, x64,
                       (const double*)xT, sc, keep, n);
  else
    hipLaunchKernelGGL((axpy_cast_kernel<float>), dim3(nb), dim3(256), 0, s, x64,
                       (const float*)xT, sc, keep, n);
  return hipGetLastError();
}

// Streaming copy, the bandwidth reference of the roofline: a workgroup of
// 256 threads moves 16 KB, four 16-byte vectors per thread, each load and
// store instruction of a wave covering 1 KB of consecutive bytes; all four
// loads are issued before the stores, non-temporal in both directions like
// the operator kernel's streams.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) stream_copy_kernel(const u32x4_t* __restrict__ src,
                                                          u32x4_t* __restrict__ dst, int64_t n16) {
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  u32x4_t v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (i0 + q * 256 < n16) v[q] = __builtin_nontemporal_load(&src[i0 + q * 256]);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (i0 + q * 256 < n16) __builtin_nontemporal_store(v[q], &dst[i0 + q * 256]);
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, hipStream_t s) {
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((n16 + 1023) / 1024)), dim3(256), 0, s,
                     (const u32x4_t*)src, (u32x4_t*)dst, n16);
  return hipGetLastError();
}

// Streaming mix, the bandwidth reference at a kernel's own read:write
// split: dst[i] = src[i] + src[n + i] + ... + src[(K-1) n + i] (16-byte
// words of four FP32, summed left to right), so K bytes are read for every
// byte written.  Same shape as the copy: four output words per thread, every
// load of the thread issued before its adds, non-temporal both ways.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
template <int K>
__global__ void __launch_bounds__(256) stream_mix_kernel(const f32x4_t* __restrict__ src,
                                                         f32x4_t* __restrict__ dst, int64_t n16) {
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  f32x4_t v[4][K];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (i0 + q * 256 < n16)
#pragma unroll
      for (int j = 0; j < K; ++j) v[q][j] = __builtin_nontemporal_load(&src[j * n16 + i0 + q * 256]);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (i0 + q * 256 < n16) {
      f32x4_t t = v[q][0];
#pragma unroll
      for (int j = 1; j < K; ++j) t += v[q][j];
      __builtin_nontemporal_store(t, &dst[i0 + q * 256]);
    }
}

hipError_t launch_stream_mix(const void* src, void* dst, int64_t n16, int k, hipStream_t s) {
  const dim3 g((unsigned)((n16 + 1023) / 1024)), b(256);
  const f32x4_t* a = (const f32x4_t*)src;
  f32x4_t* d = (f32x4_t*)dst;
  switch (k) {
    case 1: hipLaunchKernelGGL(stream_mix_kernel<1>, g, b, 0, s, a, d, n16); break;
    case 2: hipLaunchKernelGGL(stream_mix_kernel<2>, g, b, 0, s, a, d, n16); break;
    case 4: hipLaunchKernelGGL(stream_mix_kernel<4>, g, b, 0, s, a, d, n16); break;
    case 8: hipLaunchKernelGGL(stream_mix_kernel<8>, g, b, 0, s, a, d, n16); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero(double* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_mass(const double* B, const double* f, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(mass_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, B, f, b, n);
  return hipGetLastError();
}

hipError_t launch_cast_f32(float* d, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nblk(n, 256)), dim3(256), 0, s, d, src, n);
  return hipGetLastError();
}

hipError_t launch_cast_g_split(int gprec, void* d, const double* G64, int E, int n3,
                               hipStream_t s) {
  const int64_t nloc = (int64_t)E * n3;
  if (gprec == 1)
    hipLaunchKernelGGL(cast_g_split_kernel<float>, dim3(nblk(nloc, 256)), dim3(256), 0, s,
                       (float*)d, G64, E, n3);
  else
    hipLaunchKernelGGL(cast_g_split_kernel<bf16_t>, dim3(nblk(nloc, 256)), dim3(256), 0, s,
                       (bf16_t*)d, G64, E, n3);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(bf16_t* d, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cast_bf16_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, d, src, n);
  return hipGetLastError();
}

}  // namespace mx
