// Two-level Schwarz / multigrid preconditioner of a box mesh: the solveM
// step of the paper's CG-loop profiling table (70% of the time when
// Nekbone's multigrid is on; Sec. 4.2 finds that its Schwarz weights are
// square roots that must be taken in FP64).  The paper gives none of the
// multigrid algorithm; this is the textbook two-level additive Schwarz
// method with spectral-element local solves:
//
//   z = M QQ^T( ws * FDM_e( ws * r_L ) )  +  P V( P^T r )
//
//   ws      sqrt(1/m) per node (m = copies of the node = overlapping
//           subdomains containing it), the square root taken in FP64 on the
//           host and rounded once to the working precision;
//   FDM_e   exact inverse, by fast diagonalisation, of a separable operator
//           on element e extended by one GLL interval into each neighbour
//           (zero Dirichlet values at the extended ends): per direction the
//           element's 1-D stiffness and mass for its mean length, plus the
//           neighbour's face-node diagonal entries at each shared face; a
//           Dirichlet face node is decoupled.  With A_d s = lambda B_d s,
//           S^T B S = I, the element solve is S diag(1/(kbar (lx+ly+lz) + h))
//           S^T with S = Sz x Sy x Sx;
//   P       trilinear interpolation from the element-vertex lattice;
//   V       one V-cycle of geometric multigrid on the lattice: Galerkin
//           coarse operator P^T A P (27-point stencils), two damped Jacobi
//           sweeps before and after each coarse correction, full-weighting
//           restriction, and the dense inverse of the coarsest level.
//
// Device layout: the Schwarz kernel takes one element per workgroup, one
// thread per (i, j) column holding its n values along k in registers; the
// z-direction contractions are register-only, the x and y ones go through
// the element's values in LDS.  The same pass forms the element's eight
// restricted residual values (FP64).  The lattice kernels are one thread
// per lattice node, in FP64: the coarse problem is small and global.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

// ------------------------------------------------------------------ host set-up
int mg_cube_root(int E) {
  int ne = (int)llround(cbrt((double)E));
  for (int t = std::max(1, ne - 1); t <= ne + 1; ++t)
    if ((int64_t)t * t * t == E) return t;
  return 0;
}

int mg_levels(int ne, int* nu) {
  int nI = ne, l = 0;
  for (;;) {
    nu[l++] = nI - 1;
    const int64_t unk = (int64_t)(nI - 1) * (nI - 1) * (nI - 1);
    if (unk <= MG_COARSEST_MAX || nI % 2 || nI < 4 || l == MG_MAXLEV) break;
    nI /= 2;
  }
  return l;
}

// ne when the mesh is a box lattice: E = ne^3 elements in lexicographic
// order (x fastest), global ids gx + G1 (gy + G1 gz) with gx = ex N + i and
// G1 = ne N + 1, and Dirichlet conditions exactly on the box boundary; else 0
int box_lattice_ne(const mxsem_mesh_desc* d) {
  const int ne = mg_cube_root(d->E);
  if (ne < 1) return 0;
  const int N = d->N, n = N + 1, n3 = n * n * n;
  const int64_t G1 = (int64_t)ne * N + 1;
  for (int e = 0; e < d->E; ++e) {
    const int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const int64_t q = (int64_t)e * n3 + i + n * (j + n * k);
          const int64_t gx = (int64_t)ex * N + i, gy = (int64_t)ey * N + j, gz = (int64_t)ez * N + k;
          if (d->glo[q] != gx + G1 * (gy + G1 * gz)) return 0;
          const bool onb = gx == 0 || gy == 0 || gz == 0 || gx == G1 - 1 || gy == G1 - 1 ||
                           gz == G1 - 1;
          if ((d->bnd[q] != 0) != onb) return 0;
        }
  }
  return ne;
}

int mg_check_box(const mxsem_mesh_desc* d) {
  const int ne = box_lattice_ne(d);
  MX_CHECK(ne >= 2, MXSEM_ENOTSUP,
           "multigrid: needs a box of ne^3 >= 8 elements in lexicographic order with lattice "
           "global ids and Dirichlet conditions on the whole boundary");
  int nu[MG_MAXLEV];
  const int nl = mg_levels(ne, nu);
  MX_CHECK((int64_t)nu[nl - 1] * nu[nl - 1] * nu[nl - 1] <= 4096, MXSEM_ENOTSUP,
           "multigrid: the lattice cannot be coarsened to 4096 unknowns (odd element count)");
  return MXSEM_OK;
}

void mg_layout(mxsem_mesh* m, char* ws, Layout& L) {
  const int ne = mg_cube_root(m->E);
  const int n = m->n, E = m->E;
  const bool f32 = (m->views & (MXSEM_VIEW_F32 | MXSEM_VIEW_BF16)) != 0;
  MgData* g = ws ? m->mg : nullptr;
  auto put = [&](auto** p, size_t bytes) {
    const size_t o = L.take(bytes);
    if (ws) *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(ws + o);
  };
  double* d = nullptr;
  float* f = nullptr;
  put(g ? &g->S64 : &d, sizeof(double) * (size_t)E * 3 * n * n);
  put(g ? &g->lam64 : &d, sizeof(double) * (size_t)E * 3 * n);
  if (f32) {
    put(g ? &g->S32 : &f, sizeof(float) * (size_t)E * 3 * n * n);
    put(g ? &g->lam32 : &f, sizeof(float) * (size_t)E * 3 * n);
  }
  put(g ? &g->kbar : &d, sizeof(double) * E);
  put(g ? &g->ws64 : &d, sizeof(double) * 256);
  put(g ? &g->ws32 : &f, sizeof(float) * 256);
  put(g ? &g->J : &d, sizeof(double) * 2 * n);
  put(g ? &g->corner : &d, sizeof(double) * (size_t)E * 8);
  int* ip = nullptr;
  put(g ? &g->ecorner : &ip, sizeof(int) * (size_t)E * 8);
  put(g ? &g->K : &d, sizeof(double) * (size_t)E * 64);
  int nu[MG_MAXLEV];
  const int nl = mg_levels(ne, nu);
  for (int l = 0; l < nl; ++l) {
    const size_t nn = (size_t)nu[l] * nu[l] * nu[l];
    MgLevel* v = g ? &g->lv[l] : nullptr;
    put(v ? &v->st : &d, sizeof(double) * nn * 27);
    put(v ? &v->b : &d, sizeof(double) * nn);
    put(v ? &v->x : &d, sizeof(double) * nn);
    put(v ? &v->x2 : &d, sizeof(double) * nn);
    put(v ? &v->r : &d, sizeof(double) * nn);
    if (v) v->nu = nu[l];
  }
  const size_t nc = (size_t)nu[nl - 1] * nu[nl - 1] * nu[nl - 1];
  put(g ? &g->cinv : &d, sizeof(double) * nc * nc);
  if (g) {
    g->ne = ne;
    g->nlev = nl;
    g->nc = (int)nc;
  }
}

// Symmetric eigenproblem C = Q diag(w) Q^T by Jacobi rotations (threshold
// sweeps over the upper triangle); C (row-major n x n) is overwritten.
static void sym_eig(int n, std::vector<double>& C, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += C[(size_t)i * n + i] * C[(size_t)i * n + i];
      for (int j = i + 1; j < n; ++j) off += 2.0 * C[(size_t)i * n + j] * C[(size_t)i * n + j];
    }
    if (off <= 1e-30 * (off + diag)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
        // the rotation angle that zeroes C[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double ckp = C[(size_t)k * n + p], ckq = C[(size_t)k * n + q];
          C[(size_t)k * n + p] = cs * ckp - sn * ckq;
          C[(size_t)k * n + q] = sn * ckp + cs * ckq;
        }
        for (int k = 0; k < n; ++k) {
          const double cpk = C[(size_t)p * n + k], cqk = C[(size_t)q * n + k];
          C[(size_t)p * n + k] = cs * cpk - sn * cqk;
          C[(size_t)q * n + k] = sn * cpk + cs * cqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = cs * qkp - sn * qkq;
          Q[(size_t)k * n + q] = sn * qkp + cs * qkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = C[(size_t)i * n + i];
}

// mean length of element e along direction dir: the distance between the
// end nodes of each of its n^2 lines along dir, averaged
static double line_length(const double* xyz, int n, int e, int dir) {
  const int n3 = n * n * n, N = n - 1;
  const double* X = xyz + (size_t)e * 3 * n3;
  double acc = 0.0;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      const int p0 = dir == 0 ? n * (a + n * b) : dir == 1 ? a + n * n * b : a + n * b;
      const int step = dir == 0 ? 1 : dir == 1 ? n : n * n;
      const int p1 = p0 + N * step;
      double s2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double dd = X[(size_t)c * n3 + p1] - X[(size_t)c * n3 + p0];
        s2 += dd * dd;
      }
      acc += sqrt(s2);
    }
  return acc / (n * n);
}

// 1-D fast-diagonalisation pair of one element and direction: the element's
// stiffness (2/l) Ar and mass (l/2) diag(rho), plus at each shared face the
// neighbour's face-node diagonal entries; a Dirichlet face node decoupled
// (A = B = 1 there).  S = B^-1/2 Q with B^-1/2 A B^-1/2 = Q diag(lam) Q^T.
static void fdm_pair(int n, const std::vector<double>& Ar, const double* rho, double l, double llo,
                     double lhi, bool dlo, bool dhi, double* S, double* lam) {
  const int N = n - 1;
  std::vector<double> A((size_t)n * n), B(n), C((size_t)n * n), Q, w;
  for (int i = 0; i < n; ++i) {
    B[i] = 0.5 * l * rho[i];
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = (2.0 / l) * Ar[(size_t)i * n + j];
  }
  if (llo > 0.0) {
    A[0] += (2.0 / llo) * Ar[(size_t)N * n + N];
    B[0] += 0.5 * llo * rho[N];
  }
  if (lhi > 0.0) {
    A[(size_t)N * n + N] += (2.0 / lhi) * Ar[0];
    B[N] += 0.5 * lhi * rho[0];
  }
  for (int q : {dlo ? 0 : -1, dhi ? N : -1}) {
    if (q < 0) continue;
    for (int j = 0; j < n; ++j) A[(size_t)q * n + j] = A[(size_t)j * n + q] = 0.0;
    A[(size_t)q * n + q] = 1.0;
    B[q] = 1.0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = A[(size_t)i * n + j] / sqrt(B[i] * B[j]);
  sym_eig(n, C, w, Q);
  for (int i = 0; i < n; ++i) {
    lam[i] = w[i];
    for (int j = 0; j < n; ++j) S[(size_t)i * n + j] = Q[(size_t)i * n + j] / sqrt(B[i]);
  }
}

static inline int lat(int nu, int I, int J, int K) { return (I - 1) + nu * ((J - 1) + nu * (K - 1)); }
__host__ __device__ inline double hat(int f, int c) {
  const int d = f - 2 * c;
  return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0;
}

// Galerkin stencil of lattice level C from level F: P^T A_F P.
static void rap(int nuf, const std::vector<double>& Af, int nuc, std::vector<double>& Ac) {
  Ac.assign((size_t)nuc * nuc * nuc * 27, 0.0);
  for (int K = 1; K <= nuc; ++K)
    for (int J = 1; J <= nuc; ++J)
      for (int I = 1; I <= nuc; ++I) {
        double* ac = &Ac[(size_t)lat(nuc, I, J, K) * 27];
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int fi = 2 * I + dx, fj = 2 * J + dy, fk = 2 * K + dz;
              const double w = hat(fi, I) * hat(fj, J) * hat(fk, K);
              const double* af = &Af[(size_t)lat(nuf, fi, fj, fk) * 27];
              for (int t = 0; t < 27; ++t) {
                const int gi = fi + t % 3 - 1, gj = fj + (t / 3) % 3 - 1, gk = fk + t / 9 - 1;
                if (gi < 1 || gj < 1 || gk < 1 || gi > nuf || gj > nuf || gk > nuf) continue;
                for (int ck = gk / 2; ck <= (gk + 1) / 2; ++ck)
                  for (int cj = gj / 2; cj <= (gj + 1) / 2; ++cj)
                    for (int ci = gi / 2; ci <= (gi + 1) / 2; ++ci) {
                      if (ci < 1 || cj < 1 || ck < 1 || ci > nuc || cj > nuc || ck > nuc) continue;
                      const double p2 = hat(gi, ci) * hat(gj, cj) * hat(gk, ck);
                      if (p2 == 0.0) continue;
                      ac[(ci - I + 1) + 3 * (cj - J + 1) + 9 * (ck - K + 1)] += w * af[t] * p2;
                    }
              }
            }
      }
}

static double jacobi_damping(int nu, const std::vector<double>& A) {
  double bound = 0.0;
  for (int K = 1; K <= nu; ++K)
    for (int J = 1; J <= nu; ++J)
      for (int I = 1; I <= nu; ++I) {
        const double* a = &A[(size_t)lat(nu, I, J, K) * 27];
        double rs = 0.0;
        for (int t = 0; t < 27; ++t) {
          const int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
          if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
          rs += fabs(a[t]);
        }
        bound = std::max(bound, rs / a[13]);
      }
  return 1.0 / bound;
}

// inverse of an SPD matrix (Gauss-Jordan with the diagonal as pivots)
static bool spd_inverse(int nc, std::vector<double>& A, std::vector<double>& X) {
  X.assign((size_t)nc * nc, 0.0);
  for (int i = 0; i < nc; ++i) X[(size_t)i * nc + i] = 1.0;
  for (int c = 0; c < nc; ++c) {
    const double piv = A[(size_t)c * nc + c];
    if (!(piv > 0.0)) return false;
    for (int j = 0; j < nc; ++j) {
      A[(size_t)c * nc + j] /= piv;
      X[(size_t)c * nc + j] /= piv;
    }
    for (int i = 0; i < nc; ++i) {
      if (i == c) continue;
      const double f = A[(size_t)i * nc + c];
      if (f == 0.0) continue;
      for (int j = 0; j < nc; ++j) {
        A[(size_t)i * nc + j] -= f * A[(size_t)c * nc + j];
        X[(size_t)i * nc + j] -= f * X[(size_t)c * nc + j];
      }
    }
  }
  return true;
}

// ------------------------------------------------------------------ set-up kernels
// u (local FP64) = the order-1 basis function of element corner a (its
// trilinear product) in every element
__global__ void mg_basis_kernel(double* __restrict__ u, const double* __restrict__ J, int n,
                                int64_t nloc, int a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nloc) return;
  const int n3 = n * n * n, p = (int)(q % n3);
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  u[q] = J[2 * i + (a & 1)] * J[2 * j + ((a >> 1) & 1)] * J[2 * k + (a >> 2)];
}

// K[e][b*8 + a] = sum over the element's nodes of basis_b * w  (w = A_L basis_a)
__global__ void mg_elem_restrict_kernel(const double* __restrict__ w, const double* __restrict__ J,
                                        double* __restrict__ K, int E, int n, int a) {
  __shared__ double sred[16];
  const int e = blockIdx.x;
  if (e >= E) return;
  const int n3 = n * n * n;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < n3; p += blockDim.x) {
    const int i = p % n, j = (p / n) % n, k = p / (n * n);
    const double v = w[(int64_t)e * n3 + p];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] += J[2 * i + (b & 1)] * J[2 * j + ((b >> 1) & 1)] * J[2 * k + (b >> 2)] * v;
  }
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const double t = block_sum(acc[b], sred);
    if (threadIdx.x == 0) K[(int64_t)e * 64 + b * 8 + a] = t;
  }
}

int mg_setup(mxsem_mesh* m, const mxsem_mesh_desc* d, hipStream_t s) {
  MgData* g = m->mg;
  const int n = m->n, N = m->N, E = m->E, ne = g->ne;
  // reference 1-D stiffness D^T diag(rho) D, from the library's GLL rule
  std::vector<double> xi(n), rho(n), D((size_t)n * n), Ar((size_t)n * n, 0.0);
  gll_rule(N, xi.data(), rho.data());
  deriv_matrix(N, xi.data(), D.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int l = 0; l < n; ++l) Ar[(size_t)i * n + j] += D[(size_t)l * n + i] * rho[l] * D[(size_t)l * n + j];
  // element lengths and mean coefficients, then the 1-D pairs
  std::vector<double> len((size_t)E * 3), kbar(E), S((size_t)E * 3 * n * n), lam((size_t)E * 3 * n);
  const int n3 = m->n3;
  for (int e = 0; e < E; ++e) {
    for (int dir = 0; dir < 3; ++dir) len[(size_t)e * 3 + dir] = line_length(d->xyz, n, e, dir);
    double kb = 0.0;
    for (int p = 0; p < n3; ++p) kb += d->kcoef ? d->kcoef[(size_t)e * n3 + p] : 1.0;
    kbar[e] = kb / n3;
  }
  const int stride[3] = {1, ne, ne * ne};
  for (int e = 0; e < E; ++e) {
    const int ec[3] = {e % ne, (e / ne) % ne, e / (ne * ne)};
    for (int dir = 0; dir < 3; ++dir) {
      const double llo = ec[dir] > 0 ? len[(size_t)(e - stride[dir]) * 3 + dir] : 0.0;
      const double lhi = ec[dir] < ne - 1 ? len[(size_t)(e + stride[dir]) * 3 + dir] : 0.0;
      fdm_pair(n, Ar, rho.data(), len[(size_t)e * 3 + dir], llo, lhi, ec[dir] == 0,
               ec[dir] == ne - 1, &S[((size_t)e * 3 + dir) * n * n], &lam[((size_t)e * 3 + dir) * n]);
    }
  }
  std::vector<double> ws(256, 0.0);
  std::vector<float> ws32(256, 0.f);
  for (int q = 1; q < 256; ++q) {
    ws[q] = sqrt(1.0 / q);  // FP64 square roots of the Schwarz weights
    ws32[q] = (float)ws[q];
  }
  std::vector<double> Jh((size_t)2 * n);
  for (int i = 0; i < n; ++i) {
    Jh[2 * i] = 0.5 * (1.0 - xi[i]);
    Jh[2 * i + 1] = 0.5 * (1.0 + xi[i]);
  }
  MX_HIP(hipMemcpyAsync(g->S64, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(g->lam64, lam.data(), sizeof(double) * lam.size(), hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(g->kbar, kbar.data(), sizeof(double) * E, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(g->ws64, ws.data(), sizeof(double) * 256, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(g->ws32, ws32.data(), sizeof(float) * 256, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(g->J, Jh.data(), sizeof(double) * Jh.size(), hipMemcpyHostToDevice, s));
  {  // lattice index of every element corner (-1 on the boundary)
    const int nu = ne - 1;
    std::vector<int> ec((size_t)E * 8);
    for (int e = 0; e < E; ++e)
      for (int a = 0; a < 8; ++a) {
        const int I = e % ne + (a & 1), J = (e / ne) % ne + ((a >> 1) & 1), Kk = e / (ne * ne) + (a >> 2);
        ec[(size_t)e * 8 + a] =
            (I < 1 || J < 1 || Kk < 1 || I > nu || J > nu || Kk > nu) ? -1 : lat(nu, I, J, Kk);
      }
    MX_HIP(hipMemcpyAsync(g->ecorner, ec.data(), sizeof(int) * ec.size(), hipMemcpyHostToDevice, s));
    MX_HIP(hipStreamSynchronize(s));  // ec leaves scope
  }
  if (g->S32) {
    MX_HIP(launch_cast_f32(g->S32, g->S64, (int64_t)S.size(), s));
    MX_HIP(launch_cast_f32(g->lam32, g->lam64, (int64_t)lam.size(), s));
  }
  // Galerkin element matrices: the local operator on each corner's basis
  // function (FP64 work vectors x and w of the mesh, unused at set-up)
  double* u = (double*)m->bufs[VP_F64]->x;
  double* w = (double*)m->bufs[VP_F64]->w;
  const unsigned nb = (unsigned)((m->nloc + 255) / 256);
  for (int a = 0; a < 8; ++a) {
    hipLaunchKernelGGL(mg_basis_kernel, dim3(nb), dim3(256), 0, s, u, g->J, n, m->nloc, a);
    MX_HIP(hipGetLastError());
    MX_TRY(apply_impl(m, MXSEM_F64, u, w, MXSEM_LOCAL_ONLY, s));
    hipLaunchKernelGGL(mg_elem_restrict_kernel, dim3(E), dim3(256), 0, s, w, g->J, g->K, E, n, a);
    MX_HIP(hipGetLastError());
  }
  std::vector<double> K((size_t)E * 64);
  MX_HIP(hipMemcpyAsync(K.data(), g->K, sizeof(double) * K.size(), hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  // level 0: element matrices assembled on the vertex lattice (interior nodes)
  std::vector<std::vector<double>> st(g->nlev);
  const int nu0 = g->lv[0].nu;
  st[0].assign((size_t)nu0 * nu0 * nu0 * 27, 0.0);
  for (int e = 0; e < E; ++e) {
    const int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
    for (int b = 0; b < 8; ++b) {
      const int I = ex + (b & 1), J = ey + ((b >> 1) & 1), Kk = ez + (b >> 2);
      if (I < 1 || J < 1 || Kk < 1 || I > nu0 || J > nu0 || Kk > nu0) continue;
      for (int a = 0; a < 8; ++a) {
        const int I2 = ex + (a & 1), J2 = ey + ((a >> 1) & 1), K2 = ez + (a >> 2);
        if (I2 < 1 || J2 < 1 || K2 < 1 || I2 > nu0 || J2 > nu0 || K2 > nu0) continue;
        st[0][(size_t)lat(nu0, I, J, Kk) * 27 + (I2 - I + 1) + 3 * (J2 - J + 1) + 9 * (K2 - Kk + 1)] +=
            K[(size_t)e * 64 + b * 8 + a];
      }
    }
  }
  for (int l = 1; l < g->nlev; ++l) rap(g->lv[l - 1].nu, st[l - 1], g->lv[l].nu, st[l]);
  for (int l = 0; l < g->nlev; ++l) {
    g->lv[l].omega = jacobi_damping(g->lv[l].nu, st[l]);
    MX_HIP(hipMemcpyAsync(g->lv[l].st, st[l].data(), sizeof(double) * st[l].size(),
                          hipMemcpyHostToDevice, s));
  }
  // the coarsest level's dense inverse
  const int nuc = g->lv[g->nlev - 1].nu, nc = g->nc;
  std::vector<double> Ad((size_t)nc * nc, 0.0), X;
  const std::vector<double>& sc = st[g->nlev - 1];
  for (int Kk = 1; Kk <= nuc; ++Kk)
    for (int J = 1; J <= nuc; ++J)
      for (int I = 1; I <= nuc; ++I)
        for (int t = 0; t < 27; ++t) {
          const int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = Kk + t / 9 - 1;
          if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nuc || j2 > nuc || k2 > nuc) continue;
          Ad[(size_t)lat(nuc, I, J, Kk) * nc + lat(nuc, i2, j2, k2)] = sc[(size_t)lat(nuc, I, J, Kk) * 27 + t];
        }
  MX_CHECK(spd_inverse(nc, Ad, X), MXSEM_EMESH, "multigrid: coarsest operator is not positive definite");
  MX_HIP(hipMemcpyAsync(g->cinv, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, s));
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
}

// ------------------------------------------------------------------ apply kernels
// Synchronisation of the element's threads around the LDS exchanges: when
// the element's n^2 threads are one wave (n^2 divides 64), LDS operations of
// the wave complete in order and a compiler-level wave barrier suffices;
// otherwise a workgroup barrier.
template <int n2>
__device__ inline void mg_sync() {
  if constexpr (64 % n2 == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Schwarz part and restriction.  One element per workgroup (n^2 column
// threads, rounded up to whole waves); z_e = ws * S diag(1/Lambda) S^T
// (ws * r_e), corner[e][a] = sum_node J3[node][a] c r (FP64).  The column's
// r and copy counts are loaded first; the element's Sx and Sy are staged in
// LDS (each thread reads the rows and columns it needs there), while Sz and
// the restriction weights J are the same for every lane and are read from
// global memory as scalars (they stay out of the vector registers, which
// keeps several waves per SIMD).  The z direction is register-only, the x and
// y contractions exchange the element's values through LDS.
template <typename T, int N>
__global__ void __launch_bounds__(256)
    mg_schwarz_kernel(const T* __restrict__ r, T* __restrict__ z, const uint8_t* __restrict__ mult,
                      const T* __restrict__ S, const T* __restrict__ lam,
                      const double* __restrict__ kbar, double h, const T* __restrict__ ws,
                      const double* __restrict__ J, double* __restrict__ corner, int E,
                      const State* __restrict__ st) {
  constexpr int n = N + 1, n2 = n * n, n3 = n2 * n;
  __shared__ T buf[n3];
  __shared__ T sS[2 * n2];
  __shared__ T sl[3 * n];
  const int e = blockIdx.x;
  if (e >= E || (st && gcast(st)->done)) return;
  const int tid = threadIdx.x;
  const bool act = tid < n2;
  const int i = act ? tid % n : 0, j = act ? tid / n : 0;
  const int64_t base = (int64_t)e * n3 + i + n * j;
  const T* __restrict__ Se = S + (int64_t)e * 3 * n2;
  const T* __restrict__ Sz = Se + 2 * n2;  // uniform: scalar loads
  T rv[n];
  uint8_t mk[n];
#pragma unroll
  for (int k = 0; k < n; ++k) {
    mk[k] = act ? mult[base + k * n2] : (uint8_t)1;
    rv[k] = act ? r[base + k * n2] : T(0);
  }
  for (int q = tid; q < 2 * n2; q += blockDim.x) sS[q] = Se[q];
  for (int q = tid; q < 3 * n; q += blockDim.x) sl[q] = lam[(int64_t)e * 3 * n + q];
  __syncthreads();
  const T* Sx = sS;
  const T* Sy = sS + n2;
  T v[n];
  double c0 = 0.0, c1 = 0.0;  // sum_k J_k0 c r, sum_k J_k1 c r along this column
#pragma unroll
  for (int k = 0; k < n; ++k) {
    v[k] = ws[mk[k]] * rv[k];
    const double cr = (double)rv[k] * cweight(mk[k]);
    c0 += J[2 * k] * cr;
    c1 += J[2 * k + 1] * cr;
  }
  // forward transform: contract k (registers), then j and i (LDS)
  T u[n];
#pragma unroll
  for (int kk = 0; kk < n; ++kk) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < n; ++k) a += Sz[k * n + kk] * v[k];
    u[kk] = a;
  }
#pragma unroll
  for (int k = 0; k < n; ++k)
    if (act) buf[k * n2 + j * n + i] = u[k];
  mg_sync<n2>();
#pragma unroll
  for (int k = 0; k < n; ++k) {
    T a = T(0);
#pragma unroll
    for (int q = 0; q < n; ++q) a += Sy[q * n + j] * buf[k * n2 + q * n + i];
    v[k] = a;
  }
  mg_sync<n2>();
#pragma unroll
  for (int k = 0; k < n; ++k)
    if (act) buf[k * n2 + j * n + i] = v[k];
  mg_sync<n2>();
  const double kb = kbar[e];
#pragma unroll
  for (int k = 0; k < n; ++k) {
    T a = T(0);
#pragma unroll
    for (int q = 0; q < n; ++q) a += Sx[q * n + i] * buf[k * n2 + j * n + q];
    const T den = (T)(kb * (double)(sl[i] + sl[n + j] + sl[2 * n + k]) + h);
    u[k] = a / den;
  }
  mg_sync<n2>();
  // back transform: i and j (LDS), then k (registers)
#pragma unroll
  for (int k = 0; k < n; ++k)
    if (act) buf[k * n2 + j * n + i] = u[k];
  mg_sync<n2>();
#pragma unroll
  for (int k = 0; k < n; ++k) {
    T a = T(0);
#pragma unroll
    for (int q = 0; q < n; ++q) a += Sx[i * n + q] * buf[k * n2 + j * n + q];
    v[k] = a;
  }
  mg_sync<n2>();
#pragma unroll
  for (int k = 0; k < n; ++k)
    if (act) buf[k * n2 + j * n + i] = v[k];
  mg_sync<n2>();
#pragma unroll
  for (int k = 0; k < n; ++k) {
    T a = T(0);
#pragma unroll
    for (int q = 0; q < n; ++q) a += Sy[j * n + q] * buf[k * n2 + q * n + i];
    u[k] = a;
  }
#pragma unroll
  for (int kk = 0; kk < n; ++kk) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < n; ++k) a += Sz[kk * n + k] * u[k];
    if (act) z[base + kk * n2] = ws[mk[kk]] * a;
  }
  // restriction: corner a = (a0, a1, a2) gets J_i,a0 J_j,a1 sum_k J_k,a2 c r;
  // the eight sums reduced together (wave shuffles, then across waves)
  double cc[8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
    cc[a] = act ? J[2 * i + (a & 1)] * J[2 * j + ((a >> 1) & 1)] * ((a >> 2) ? c1 : c0) : 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 8; ++a) cc[a] += __shfl_down(cc[a], off, 64);
  const int lane = tid & 63, wid = tid >> 6, nw = (int)(blockDim.x >> 6);
  if (nw == 1) {  // lane 0 holds the eight sums
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < 8; ++a) corner[(int64_t)e * 8 + a] = cc[a];
    return;
  }
  __shared__ double sc8[4][8];
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 8; ++a) sc8[wid][a] = cc[a];
  __syncthreads();
  if (tid < 8) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += sc8[q][tid];
    corner[(int64_t)e * 8 + tid] = t;
  }
}

// level-0 right-hand side: each interior vertex sums the corners of its
// elements; with A, also the first Jacobi sweep from x = 0 (x1 = omega b /
// a_diag, the point's own values only)
__global__ void mg_gather_kernel(const double* __restrict__ corner, double* __restrict__ b, int ne,
                                 const State* __restrict__ st, const double* __restrict__ A,
                                 double* __restrict__ x1, double omega) {
  const int nu = ne - 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nu * nu * nu || (st && gcast(st)->done)) return;
  const int I = q % nu + 1, J = (q / nu) % nu + 1, K = q / (nu * nu) + 1;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ex = I - 1 + (a & 1), ey = J - 1 + ((a >> 1) & 1), ez = K - 1 + (a >> 2);
    // vertex (I,J,K) is corner (1-(a&1), ...) of element (ex, ey, ez)
    const int c = (1 - (a & 1)) + 2 * (1 - ((a >> 1) & 1)) + 4 * (1 - (a >> 2));
    s += corner[((int64_t)ex + ne * ((int64_t)ey + ne * ez)) * 8 + c];
  }
  b[q] = s;
  if (A) x1[q] = omega * s / A[(int64_t)q * 27 + 13];
}

__device__ inline double stencil_apply(const double* __restrict__ a, const double* __restrict__ x,
                                       int nu, int I, int J, int K) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
    if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
    s += a[t] * x[(i2 - 1) + nu * ((j2 - 1) + nu * (k2 - 1))];
  }
  return s;
}

// damped Jacobi sweep xo = x + omega D^-1 (b - A x); x == nullptr: x = 0
__global__ void lat_jacobi_kernel(const double* __restrict__ A, const double* __restrict__ b,
                                  const double* __restrict__ x, double* __restrict__ xo, int nu,
                                  double omega, const State* __restrict__ st) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nu * nu * nu || (st && gcast(st)->done)) return;
  const double* a = A + (int64_t)q * 27;
  if (!x) {
    xo[q] = omega * b[q] / a[13];
    return;
  }
  const int I = q % nu + 1, J = (q / nu) % nu + 1, K = q / (nu * nu) + 1;
  xo[q] = x[q] + omega * (b[q] - stencil_apply(a, x, nu, I, J, K)) / a[13];
}

__global__ void lat_residual_kernel(const double* __restrict__ A, const double* __restrict__ b,
                                    const double* __restrict__ x, double* __restrict__ r, int nu,
                                    const State* __restrict__ st) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nu * nu * nu || (st && gcast(st)->done)) return;
  const int I = q % nu + 1, J = (q / nu) % nu + 1, K = q / (nu * nu) + 1;
  r[q] = b[q] - stencil_apply(A + (int64_t)q * 27, x, nu, I, J, K);
}

// bc = P^T r (full weighting); with Ac, also the coarse level's first Jacobi
// sweep from x = 0 (xc1 = omega_c bc / ac_diag, the point's own values only)
__global__ void lat_restrict_kernel(const double* __restrict__ r, double* __restrict__ bc, int nuf,
                                    int nuc, const State* __restrict__ st,
                                    const double* __restrict__ Ac, double* __restrict__ xc1,
                                    double omegac) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nuc * nuc * nuc || (st && gcast(st)->done)) return;
  const int I = q % nuc + 1, J = (q / nuc) % nuc + 1, K = q / (nuc * nuc) + 1;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const double w = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
    s += w * r[(2 * I + dx - 1) + nuf * ((2 * J + dy - 1) + nuf * (2 * K + dz - 1))];
  }
  bc[q] = s;
  if (Ac) xc1[q] = omegac * s / Ac[(int64_t)q * 27 + 13];
}

// x += P xc (trilinear interpolation from the coarser level)
__global__ void lat_prolong_kernel(const double* __restrict__ xc, double* __restrict__ x, int nuf,
                                   int nuc, const State* __restrict__ st) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nuf * nuf * nuf || (st && gcast(st)->done)) return;
  const int I = q % nuf + 1, J = (q / nuf) % nuf + 1, K = q / (nuf * nuf) + 1;
  double s = 0.0;
  for (int ck = K / 2; ck <= (K + 1) / 2; ++ck)
    for (int cj = J / 2; cj <= (J + 1) / 2; ++cj)
      for (int ci = I / 2; ci <= (I + 1) / 2; ++ci) {
        if (ci < 1 || cj < 1 || ck < 1 || ci > nuc || cj > nuc || ck > nuc) continue;
        s += hat(I, ci) * hat(J, cj) * hat(K, ck) * xc[(ci - 1) + nuc * ((cj - 1) + nuc * (ck - 1))];
      }
  x[q] += s;
}

// x = Ainv b on the coarsest level (one workgroup per 4 rows, wave sums)
__global__ void lat_dense_kernel(const double* __restrict__ Ainv, const double* __restrict__ b,
                                 double* __restrict__ x, int nc, const State* __restrict__ st) {
  if (st && gcast(st)->done) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= nc) return;
  double s = 0.0;
  for (int c = lane; c < nc; c += 64) s += Ainv[(int64_t)row * nc + c] * b[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = s;
}

// z += P x0: the coarse correction interpolated to every local node
template <typename T>
__global__ void mg_prolong_kernel(const double* __restrict__ x0, const double* __restrict__ J,
                                  T* __restrict__ z, int ne, int n, int64_t nloc,
                                  const State* __restrict__ st) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nloc || (st && gcast(st)->done)) return;
  const int n3 = n * n * n;
  const int e = (int)(q / n3), p = (int)(q % n3);
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  const int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne), nu = ne - 1;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int I = ex + (a & 1), Jn = ey + ((a >> 1) & 1), K = ez + (a >> 2);
    if (I < 1 || Jn < 1 || K < 1 || I > nu || Jn > nu || K > nu) continue;
    s += J[2 * i + (a & 1)] * J[2 * j + ((a >> 1) & 1)] * J[2 * k + (a >> 2)] *
         x0[(I - 1) + nu * ((Jn - 1) + nu * (K - 1))];
  }
  z[q] = (T)((double)z[q] + s);
}

// Inside a flexible-CG solve: the coarse correction added to every entry of
// z (z += P x0) in the pass that sums the step's dots, (r, z)_c into
// part_u0 and (z, w)_c into part_u2 per vector-pass tile (the partials of
// the flexible-CG dot kernel, in the same layout).
template <typename T, typename ACC, int N>
__global__ void __launch_bounds__(UPD_THREADS)
    mg_prolong_dots_kernel(const Tile* __restrict__ tiles, const ProbDev* __restrict__ probs,
                           const double* __restrict__ x0, const double* __restrict__ J,
                           const int* __restrict__ ecorner) {
  constexpr int n = N + 1, n3 = n * n * n;
  constexpr int NE = UPD_CHUNK / n3 + 2;  // elements a tile can touch
  __shared__ ACC sred[16];
  __shared__ double sJ[2 * n];
  __shared__ double scv[NE * 8];           // corner values of those elements
  const Tile t = tiles[blockIdx.x];
  const ProbDev& P = probs[t.prob];
  if (gcast(P.st)->done) return;
  if (threadIdx.x < 2 * n) sJ[threadIdx.x] = J[threadIdx.x];
  const int e0 = (int)((int64_t)t.first / n3);
  const int nelem = (int)(P.E - e0 < NE ? P.E - e0 : NE);
  for (int q = threadIdx.x; q < nelem * 8; q += UPD_THREADS) {
    const int c = ecorner[(int64_t)e0 * 8 + q];  // lattice index, -1 on the boundary
    scv[q] = c < 0 ? 0.0 : x0[c];
  }
  __syncthreads();
  const gptr<const T> __restrict__ r = gcast((const T*)P.r);
  const gptr<T> __restrict__ z = gcast((T*)P.z);
  const gptr<const T> __restrict__ w = gcast((const T*)P.w);
  const gptr<const uint8_t> __restrict__ mult = gcast(P.mult);
  ACC rz = ACC(0), zw = ACC(0);
#pragma unroll
  for (int q = 0; q < UPD_PER_THREAD; ++q) {
    const int64_t idx = (int64_t)t.first + q * UPD_THREADS + threadIdx.x;
    if (idx < P.nloc) {
      const int e = (int)(idx / n3), p = (int)(idx - (int64_t)e * n3);
      const int i = p % n, j = (p / n) % n, k = p / (n * n);
      const double* cv = scv + (e - e0) * 8;
      // trilinear interpolation, one direction at a time
      const double jx0 = sJ[2 * i], jx1 = sJ[2 * i + 1];
      const double y00 = jx0 * cv[0] + jx1 * cv[1], y10 = jx0 * cv[2] + jx1 * cv[3];
      const double y01 = jx0 * cv[4] + jx1 * cv[5], y11 = jx0 * cv[6] + jx1 * cv[7];
      const double z0 = sJ[2 * j] * y00 + sJ[2 * j + 1] * y10;
      const double z1 = sJ[2 * j] * y01 + sJ[2 * j + 1] * y11;
      const double s = sJ[2 * k] * z0 + sJ[2 * k + 1] * z1;
      const T zn = (T)((double)z[idx] + s);
      z[idx] = zn;
      const ACC c = (ACC)cweight(mult[idx]);
      rz += (ACC)r[idx] * c * (ACC)zn;
      zw += (ACC)zn * c * (ACC)w[idx];
    }
  }
  const ACC s0 = block_sum(rz, sred);
  const ACC s1 = block_sum(zw, sred);
  if (threadIdx.x == 0) {
    const int b = t.first / UPD_CHUNK;
    gcast(P.part_u0)[b] = (double)s0;
    gcast(P.part_u2)[b] = (double)s1;
  }
}

int mg_prolong_dots(const mxsem_mesh* m, const Plan* pl, hipStream_t s) {
  const MgData* g = m->mg;
  const dim3 grid(pl->nt_upd), blk(UPD_THREADS);
  const double* x0 = g->lv[0].x;
  switch (m->N) {
#define MX_PD(NN_)                                                                               \
  case NN_:                                                                                      \
    if (pl->vprec == VP_F64)                                                                     \
      hipLaunchKernelGGL((mg_prolong_dots_kernel<double, double, NN_>), grid, blk, 0, s,         \
                         pl->tiles_upd, pl->probs, x0, g->J, g->ecorner);                        \
    else if (pl->vprec == VP_F32)                                                                \
      hipLaunchKernelGGL((mg_prolong_dots_kernel<float, double, NN_>), grid, blk, 0, s,          \
                         pl->tiles_upd, pl->probs, x0, g->J, g->ecorner);                        \
    else                                                                                         \
      hipLaunchKernelGGL((mg_prolong_dots_kernel<float, float, NN_>), grid, blk, 0, s,           \
                         pl->tiles_upd, pl->probs, x0, g->J, g->ecorner);                        \
    break;
    MX_PD(1) MX_PD(2) MX_PD(3) MX_PD(4) MX_PD(5) MX_PD(6) MX_PD(7) MX_PD(8) MX_PD(9)
    MX_PD(10) MX_PD(11) MX_PD(12) MX_PD(13) MX_PD(14) MX_PD(15)
#undef MX_PD
    default:
      set_error("multigrid: order out of range");
      return MXSEM_ENOTSUP;
  }
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
}

template <typename T>
static hipError_t launch_schwarz(int N, const T* r, T* z, const uint8_t* mult, const T* S,
                                 const T* lam, const double* kbar, double h, const T* ws,
                                 const double* J, double* corner, int E, hipStream_t s,
                                 const State* st) {
  const int n2 = (N + 1) * (N + 1);
  const dim3 t(std::min(256, ((n2 + 63) / 64) * 64));
  switch (N) {
#define MX_MG(NN_)                                                                             \
  case NN_:                                                                                    \
    hipLaunchKernelGGL((mg_schwarz_kernel<T, NN_>), dim3(E), t, 0, s, r, z, mult, S, lam, kbar, \
                       h, ws, J, corner, E, st);                                               \
    break;
    MX_MG(1) MX_MG(2) MX_MG(3) MX_MG(4) MX_MG(5) MX_MG(6) MX_MG(7) MX_MG(8) MX_MG(9)
    MX_MG(10) MX_MG(11) MX_MG(12) MX_MG(13) MX_MG(14) MX_MG(15)
#undef MX_MG
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static inline unsigned lat_blocks(int nn) { return (unsigned)((nn + 255) / 256); }

int mg_apply(mxsem_mesh* m, int vprec, const void* r, void* z, hipStream_t s, const State* st,
             const Plan* pl) {
  MgData* g = m->mg;
  MX_CHECK(g, MXSEM_EINVAL, "multigrid: the mesh was built without MXSEM_VIEW_MG");
  const bool f64 = vprec == VP_F64;
  MX_CHECK(f64 || g->S32, MXSEM_ENOTSUP, "multigrid: mesh has no FP32 view");
  if (f64)
    MX_HIP(launch_schwarz<double>(m->N, (const double*)r, (double*)z, m->mult, g->S64, g->lam64,
                                  g->kbar, m->helm_h, g->ws64, g->J, g->corner, m->E, s, st));
  else
    MX_HIP(launch_schwarz<float>(m->N, (const float*)r, (float*)z, m->mult, g->S32, g->lam32,
                                 g->kbar, m->helm_h, g->ws32, g->J, g->corner, m->E, s, st));
  // the subdomains' contributions summed (FP64 sums), Dirichlet rows zeroed;
  // inside a solve the plan's XCD-ordered tiles, which skip a finished solve
  if (pl)
    MX_HIP(launch_gs_solver(pl->vprec, pl->tiles_gs, pl->nt_gs, pl->probs, s, true, 0, nullptr, 0));
  else
    MX_HIP(launch_gs_apply(f64 ? MXSEM_F64 : MXSEM_F32, MXSEM_F64, z, m->plan, true, s));
  // coarse correction: one V-cycle on the vertex lattice.  The first sweep
  // of each smoothed level starts from x = 0 and needs only the point's own
  // right-hand side, so it is formed where that right-hand side is (the
  // corner gather, the restriction); the other steps couple neighbours and
  // keep launches of their own (fusing the residual into the restriction, or
  // the prolongation into the next sweep, recomputes neighbours' values on
  // grids of a few thousand points and was slower: 137 and 38 us against 6
  // and 10 us on the 32^3 mesh).
  const int L = g->nlev;
  {
    MgLevel& v = g->lv[0];
    const int nu = v.nu;
    hipLaunchKernelGGL(mg_gather_kernel, dim3(lat_blocks(nu * nu * nu)), dim3(256), 0, s, g->corner,
                       v.b, g->ne, st, L > 1 ? (const double*)v.st : nullptr, v.x2, v.omega);
    MX_HIP(hipGetLastError());
  }
  for (int l = 0; l + 1 < L; ++l) {
    MgLevel& v = g->lv[l];
    const int nn = v.nu * v.nu * v.nu;
    hipLaunchKernelGGL(lat_jacobi_kernel, dim3(lat_blocks(nn)), dim3(256), 0, s, v.st, v.b,
                       (const double*)v.x2, v.x, v.nu, v.omega, st);
    hipLaunchKernelGGL(lat_residual_kernel, dim3(lat_blocks(nn)), dim3(256), 0, s, v.st, v.b,
                       (const double*)v.x, v.r, v.nu, st);
    MgLevel& c = g->lv[l + 1];
    const bool csmooth = l + 2 < L;  // the coarser level is smoothed, not solved
    hipLaunchKernelGGL(lat_restrict_kernel, dim3(lat_blocks(c.nu * c.nu * c.nu)), dim3(256), 0, s,
                       (const double*)v.r, c.b, v.nu, c.nu, st,
                       csmooth ? (const double*)c.st : nullptr, c.x2, c.omega);
    MX_HIP(hipGetLastError());
  }
  {
    MgLevel& c = g->lv[L - 1];
    hipLaunchKernelGGL(lat_dense_kernel, dim3((unsigned)((g->nc + 3) / 4)), dim3(256), 0, s,
                       g->cinv, (const double*)c.b, c.x, g->nc, st);
    MX_HIP(hipGetLastError());
  }
  for (int l = L - 2; l >= 0; --l) {
    MgLevel& v = g->lv[l];
    MgLevel& c = g->lv[l + 1];
    const int nn = v.nu * v.nu * v.nu;
    hipLaunchKernelGGL(lat_prolong_kernel, dim3(lat_blocks(nn)), dim3(256), 0, s,
                       (const double*)c.x, v.x, v.nu, c.nu, st);
    hipLaunchKernelGGL(lat_jacobi_kernel, dim3(lat_blocks(nn)), dim3(256), 0, s, v.st, v.b,
                       (const double*)v.x, v.x2, v.nu, v.omega, st);
    hipLaunchKernelGGL(lat_jacobi_kernel, dim3(lat_blocks(nn)), dim3(256), 0, s, v.st, v.b,
                       (const double*)v.x2, v.x, v.nu, v.omega, st);
    MX_HIP(hipGetLastError());
  }
  if (pl) return MXSEM_OK;  // the solve adds the coarse correction in its dot pass
  const unsigned nb = (unsigned)((m->nloc + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(mg_prolong_kernel<double>, dim3(nb), dim3(256), 0, s,
                       (const double*)g->lv[0].x, g->J, (double*)z, g->ne, m->n, m->nloc, st);
  else
    hipLaunchKernelGGL(mg_prolong_kernel<float>, dim3(nb), dim3(256), 0, s,
                       (const double*)g->lv[0].x, g->J, (float*)z, g->ne, m->n, m->nloc, st);
  MX_HIP(hipGetLastError());
  return MXSEM_OK;
}

}  // namespace mx
