/*
 * Plain FP64 CPU oracle for the matrix-free spectral-element (P)CG solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * cpu_baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never links, imports or calls it,
 * and this file includes nothing from the product path.
 *
 * What it computes (paper: "Enabling mixed-precision in spectral element
 * codes"; the paper defers the discretisation to Deville-Fischer-Mund, so the
 * operator steps below are the textbook spectral-element method):
 *   - GLL nodes/weights and the nodal derivative matrix (the tensor-product
 *     basis behind local_grad3 / local_grad3_t, Sec. 4.1, CG-loop profiling
 *     table, its "ax" row and that row's footnote on mxm and accumulations);
 *   - isoparametric geometric factors G and mass B (initialisation, kept in
 *     FP64 per Sec. 5.2);
 *   - the local operator w_L = sum_ab D_a^T diag(G_ab) D_b u_L + h B u_L;
 *   - direct stiffness summation QQ^T (Sec. 4.2.1) and the Dirichlet mask;
 *   - the c-weighted dot glsc3 (CG-loop profiling table, its glsc3 rows);
 *   - the Jacobi diagonal 1/diag(A) (Sec. 5.2, Jacobi paragraph);
 *   - PCG in the order of the CG-loop profiling table (textbook form),
 *     FP64 iterative refinement around an inner PCG, and flexible CG(1).
 *
 * Everything is FP64, compiled with -O2 -fno-fast-math -ffp-contract=off.
 * OpenMP is used only for loops whose iterations are independent (per
 * element / per entry / per gather-scatter group); every reduction (dot
 * product, group sum) runs sequentially in ascending index order.
 *
 * Layouts: a local vector has E*n^3 entries, n = N+1, entry
 * ((e*n + k)*n + j)*n + i for node (i,j,k) of element e (i fastest).
 * xyz is [E][3][n^3]; G is [E][6][n^3] with components rr,rs,rt,ss,st,tt.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EJAC -2   /* non-positive Jacobian determinant */
#define ORC_EMASK -3  /* copies of one global node disagree on the mask */
#define ORC_ENOMEM -4

#define ORC_CONVERGED 1
#define ORC_MAXITER 2
#define ORC_STAGNATED 3
#define ORC_BREAKDOWN 4

#define ORC_PC_IDENTITY 0
#define ORC_PC_JACOBI 1
#define ORC_PC_NN 2

/* ------------------------------------------------------------------------ */
/* O1: Legendre polynomial L_N and the Gauss-Lobatto-Legendre rule.          */
/* ------------------------------------------------------------------------ */

/* L_N(x) and L_{N-1}(x) by the three-term recurrence
 * (k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1}. */
static void legendre_pair(int N, double x, double *LN, double *LNm1) {
  double p0 = 1.0, p1 = x;
  if (N == 0) {
    *LN = 1.0;
    *LNm1 = 0.0;
    return;
  }
  for (int k = 1; k < N; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *LN = p1;
  *LNm1 = p0;
}

/* GLL nodes xi[0..N] (ascending, xi[0]=-1, xi[N]=1) and weights
 * rho_i = 2 / (N (N+1) L_N(xi_i)^2).  The interior nodes are the roots of
 * L'_N, found by Newton's method from the Chebyshev-Lobatto points
 * -cos(pi i / N); L'_N and L''_N come from
 *   (1-x^2) L'_N  = N (L_{N-1} - x L_N)
 *   (1-x^2) L''_N = 2 x L'_N - N (N+1) L_N      (Legendre's equation). */
int orc_gll(int N, double *xi, double *rho) {
  if (N < 1 || N > 32 || !xi || !rho) return ORC_EINVAL;
  xi[0] = -1.0;
  xi[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double x = -cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double L, Lm1;
      legendre_pair(N, x, &L, &Lm1);
      double d1 = N * (Lm1 - x * L) / (1.0 - x * x);
      double d2 = (2.0 * x * d1 - N * (N + 1.0) * L) / (1.0 - x * x);
      double dx = d1 / d2;
      x -= dx;
      if (fabs(dx) < 1e-15) break;
    }
    xi[i] = x;
  }
  /* insertion sort, ascending */
  for (int i = 1; i <= N; ++i) {
    double v = xi[i];
    int j = i - 1;
    while (j >= 0 && xi[j] > v) {
      xi[j + 1] = xi[j];
      --j;
    }
    xi[j + 1] = v;
  }
  for (int i = 0; i <= N; ++i) {
    double L, Lm1;
    legendre_pair(N, xi[i], &L, &Lm1);
    rho[i] = 2.0 / (N * (N + 1.0) * L * L);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O2: nodal derivative matrix, D[i*n + j] = l_j'(xi_i).                     */
/* ------------------------------------------------------------------------ */
int orc_deriv(int N, const double *xi, double *D) {
  if (N < 1 || !xi || !D) return ORC_EINVAL;
  int n = N + 1;
  double *LN = (double *)malloc(sizeof(double) * n);
  if (!LN) return ORC_ENOMEM;
  for (int i = 0; i < n; ++i) {
    double Lm1;
    legendre_pair(N, xi[i], &LN[i], &Lm1);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v;
      if (i != j)
        v = LN[i] / (LN[j] * (xi[i] - xi[j]));
      else if (i == 0)
        v = -N * (N + 1.0) / 4.0;
      else if (i == N)
        v = N * (N + 1.0) / 4.0;
      else
        v = 0.0;
      D[i * n + j] = v;
    }
  free(LN);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Mesh object: FP64 operator data and the gather-scatter groups.             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int E, N, n, n3;
  int64_t nloc;
  double *xi, *rho, *D; /* D[i*n+l] */
  double *G;            /* [E][6][n3] */
  double *B;            /* [E][n3] */
  double helm_h;
  /* gather-scatter: groups of local indices sharing a global id, groups in
   * ascending global id, indices ascending inside each group */
  int64_t ngroups;
  int64_t *goff; /* ngroups+1 */
  int64_t *gidx; /* nloc */
  double *mult;  /* nloc: multiplicity m */
  double *c;     /* nloc: 1/m */
  unsigned char *mask; /* nloc: 1 on Dirichlet entries */
  double *dinv;  /* nloc */
  double mindet;
} orc_mesh;

typedef struct {
  int64_t g, i;
} gpair;

static int gpair_cmp(const void *a, const void *b) {
  const gpair *x = (const gpair *)a, *y = (const gpair *)b;
  if (x->g != y->g) return x->g < y->g ? -1 : 1;
  if (x->i != y->i) return x->i < y->i ? -1 : 1;
  return 0;
}

/* derivatives of a nodal field f (one element, n^3) along r, s, t */
static void grad3(int n, const double *D, const double *f, double *fr,
                  double *fs, double *ft) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double ar = 0.0, as = 0.0, at = 0.0;
        for (int l = 0; l < n; ++l) {
          ar += D[i * n + l] * f[l + n * (j + n * k)];
          as += D[j * n + l] * f[i + n * (l + n * k)];
          at += D[k * n + l] * f[i + n * (j + n * l)];
        }
        int p = i + n * (j + n * k);
        fr[p] = ar;
        fs[p] = as;
        ft[p] = at;
      }
}

/* transpose-derivatives summed: w = Dr^T wr + Ds^T ws + Dt^T wt */
static void grad3_t(int n, const double *D, const double *wr, const double *ws,
                    const double *wt, double *w) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int l = 0; l < n; ++l) {
          a += D[l * n + i] * wr[l + n * (j + n * k)];
          a += D[l * n + j] * ws[i + n * (l + n * k)];
          a += D[l * n + k] * wt[i + n * (j + n * l)];
        }
        w[i + n * (j + n * k)] = a;
      }
}

/* O3: geometric factors for every element. */
static int build_geometry(orc_mesh *m, const double *xyz, const double *kcoef) {
  int n = m->n, n3 = m->n3;
  int bad = 0;
  double mindet = INFINITY;
#pragma omp parallel
  {
    double *buf = (double *)malloc(sizeof(double) * 9 * n3);
    double local_min = INFINITY;
    int local_bad = 0;
#pragma omp for schedule(static)
    for (int e = 0; e < m->E; ++e) {
      const double *X = xyz + (int64_t)e * 3 * n3;
      double *a = buf; /* a[(c*3+d)*n3 + p] = d x_c / d r_d */
      for (int cc = 0; cc < 3; ++cc)
        grad3(n, m->D, X + cc * n3, a + (cc * 3 + 0) * n3, a + (cc * 3 + 1) * n3,
              a + (cc * 3 + 2) * n3);
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            int p = i + n * (j + n * k);
            double J[3][3];
            for (int cc = 0; cc < 3; ++cc)
              for (int d = 0; d < 3; ++d) J[cc][d] = a[(cc * 3 + d) * n3 + p];
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (det < local_min) local_min = det;
            if (!(det > 0.0)) {
              local_bad = 1;
              continue;
            }
            /* inverse: Ji[d][cc] = d r_d / d x_cc = cofactor(cc,d) / det */
            double Ji[3][3];
            Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
            Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
            Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
            Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            double wq = m->rho[i] * m->rho[j] * m->rho[k] * det;
            double kk = kcoef ? kcoef[(int64_t)e * n3 + p] : 1.0;
            static const int ab[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
            for (int q = 0; q < 6; ++q) {
              int ra = ab[q][0], rb = ab[q][1];
              double s = 0.0;
              for (int cc = 0; cc < 3; ++cc) s += Ji[ra][cc] * Ji[rb][cc];
              m->G[((int64_t)e * 6 + q) * n3 + p] = wq * s * kk;
            }
            m->B[(int64_t)e * n3 + p] = wq;
          }
    }
    free(buf);
#pragma omp critical
    {
      if (local_min < mindet) mindet = local_min;
      bad |= local_bad;
    }
  }
  m->mindet = mindet;
  return bad ? ORC_EJAC : ORC_OK;
}

/* O5 set-up: group local entries by global id. */
static int build_groups(orc_mesh *m, const int64_t *glo) {
  int64_t nl = m->nloc;
  gpair *pr = (gpair *)malloc(sizeof(gpair) * nl);
  if (!pr) return ORC_ENOMEM;
  for (int64_t i = 0; i < nl; ++i) {
    pr[i].g = glo[i];
    pr[i].i = i;
  }
  qsort(pr, nl, sizeof(gpair), gpair_cmp);
  int64_t ng = 0;
  for (int64_t i = 0; i < nl; ++i)
    if (i == 0 || pr[i].g != pr[i - 1].g) ++ng;
  m->ngroups = ng;
  m->goff = (int64_t *)malloc(sizeof(int64_t) * (ng + 1));
  m->gidx = (int64_t *)malloc(sizeof(int64_t) * nl);
  if (!m->goff || !m->gidx) {
    free(pr);
    return ORC_ENOMEM;
  }
  int64_t g = -1;
  for (int64_t i = 0; i < nl; ++i) {
    if (i == 0 || pr[i].g != pr[i - 1].g) m->goff[++g] = i;
    m->gidx[i] = pr[i].i;
  }
  m->goff[ng] = nl;
  free(pr);
  for (int64_t q = 0; q < ng; ++q) {
    int64_t cnt = m->goff[q + 1] - m->goff[q];
    for (int64_t t = m->goff[q]; t < m->goff[q + 1]; ++t) {
      m->mult[m->gidx[t]] = (double)cnt;
      m->c[m->gidx[t]] = 1.0 / (double)cnt;
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O4: local operator w_L = A_L u_L                                          */
/* ------------------------------------------------------------------------ */
void orc_ax_local(const orc_mesh *m, const double *u, double *w) {
  int n = m->n, n3 = m->n3;
#pragma omp parallel
  {
    double *t = (double *)malloc(sizeof(double) * 6 * n3);
    double *ur = t, *us = t + n3, *ut = t + 2 * n3;
    double *wr = t + 3 * n3, *ws = t + 4 * n3, *wt = t + 5 * n3;
#pragma omp for schedule(static)
    for (int e = 0; e < m->E; ++e) {
      const double *ue = u + (int64_t)e * n3;
      const double *G = m->G + (int64_t)e * 6 * n3;
      grad3(n, m->D, ue, ur, us, ut);
      for (int p = 0; p < n3; ++p) {
        double grr = G[0 * n3 + p], grs = G[1 * n3 + p], grt = G[2 * n3 + p];
        double gss = G[3 * n3 + p], gst = G[4 * n3 + p], gtt = G[5 * n3 + p];
        wr[p] = grr * ur[p] + grs * us[p] + grt * ut[p];
        ws[p] = grs * ur[p] + gss * us[p] + gst * ut[p];
        wt[p] = grt * ur[p] + gst * us[p] + gtt * ut[p];
      }
      double *we = w + (int64_t)e * n3;
      grad3_t(n, m->D, wr, ws, wt, we);
      if (m->helm_h != 0.0) {
        const double *B = m->B + (int64_t)e * n3;
        for (int p = 0; p < n3; ++p) we[p] += m->helm_h * B[p] * ue[p];
      }
    }
    free(t);
  }
}

/* O5: v <- QQ^T v.  Each group is summed in FP64 in ascending local index
 * order and the sum is written to every copy. */
void orc_gs(const orc_mesh *m, double *v) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < m->ngroups; ++q) {
    double s = 0.0;
    for (int64_t t = m->goff[q]; t < m->goff[q + 1]; ++t) s += v[m->gidx[t]];
    for (int64_t t = m->goff[q]; t < m->goff[q + 1]; ++t) v[m->gidx[t]] = s;
  }
}

/* O6: zero every Dirichlet entry. */
void orc_mask(const orc_mesh *m, double *v) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m->nloc; ++i)
    if (m->mask[i]) v[i] = 0.0;
}

/* O7: assembled apply  w = M QQ^T A_L u */
void orc_apply(const orc_mesh *m, const double *u, double *w) {
  orc_ax_local(m, u, w);
  orc_gs(m, w);
  orc_mask(m, w);
}

/* weighted inner product (a,b)_c = sum_i a_i c_i b_i  (glsc3) */
double orc_dot(const orc_mesh *m, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < m->nloc; ++i) s += a[i] * m->c[i] * b[i];
  return s;
}

/* ------------------------------------------------------------------------ */
/* FP32 reductions of the extended-precision study (Sec. 5.2.1, and the     */
/* gather-scatter modes of Sec. 4.2.1).  The only FP32 routines here: they  */
/* define what the working-precision variants of the dot products and of    */
/* the gather-scatter compute.  Compiled with contraction off, so every     */
/* operation below is one IEEE FP32 operation.                               */
/* ------------------------------------------------------------------------ */

/* TwoSum (Knuth): s = fl(a + b) and e with a + b = s + e exactly. */
static void orc_two_sum(float a, float b, float *s, float *e) {
  const float x = a + b;
  const float z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

/* TwoProduct by a fused multiply-add: p = fl(a b), e = a b - p exactly. */
static void orc_two_prod(float a, float b, float *p, float *e) {
  const float x = a * b;
  *e = fmaf(a, b, -x);
  *p = x;
}

/* Dot2 of Ogita, Rump and Oishi (2005), in index order: the running sum p
 * takes each rounded product by TwoSum; the product errors and the TwoSum
 * errors accumulate in s; the result is fl(p + s). */
float orc_dot2_f32(int64_t n, const float *x, const float *y) {
  float p = 0.f, s = 0.f;
  for (int64_t i = 0; i < n; ++i) {
    float h, r, q;
    orc_two_prod(x[i], y[i], &h, &r);
    orc_two_sum(p, h, &p, &q);
    s = s + (q + r);
  }
  return p + s;
}

/* Recursive FP32 dot in index order: s = fl(s + fl(x_i y_i)). */
float orc_dot_f32(int64_t n, const float *x, const float *y) {
  float s = 0.f;
  for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];
  return s;
}

/* Weighted dot (a, b)_c in the working precision: the terms are
 * (fl(a_i c_i), b_i) with c_i rounded to FP32, then summed by Dot2 (dot2 =
 * 1) or recursively in FP32 (dot2 = 0). */
float orc_dot_c_f32(const orc_mesh *m, int dot2, const float *a, const float *b) {
  float *t = (float *)malloc(sizeof(float) * (size_t)(m->nloc ? m->nloc : 1));
  if (!t) return NAN;
  for (int64_t i = 0; i < m->nloc; ++i) t[i] = a[i] * (float)m->c[i];
  const float r = dot2 ? orc_dot2_f32(m->nloc, t, b) : orc_dot_f32(m->nloc, t, b);
  free(t);
  return r;
}

/* QQ^T on an FP32 vector.  acc64: sums in FP64 (else FP32), rounded once to
 * FP32.  pairwise = 0: one sum per group in ascending local index order,
 * written to every copy.  pairwise = 1: the order of a pairwise exchange
 * between ranks (Sec. 4.2.1): element e belongs to rank erank[e] (erank
 * NULL: rank e); a rank's partial is the sum of its copies in ascending
 * local index; a copy in rank R receives R's partial plus the other ranks'
 * partials in ascending rank order, added left to right.  Groups of up to
 * 64 copies. */
int orc_gs_f32(const orc_mesh *m, float *v, int acc64, int pairwise, const int *erank) {
  for (int64_t q = 0; q < m->ngroups; ++q)
    if (m->goff[q + 1] - m->goff[q] > 64) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < m->ngroups; ++q) {
    const int64_t o = m->goff[q];
    const int cnt = (int)(m->goff[q + 1] - o);
    float val[64], out[64];
    int rank[64];
    for (int k = 0; k < cnt; ++k) {
      const int64_t i = m->gidx[o + k];
      const int64_t e = i / m->n3;
      val[k] = v[i];
      rank[k] = pairwise ? (erank ? erank[e] : (int)e) : 0;
    }
    /* distinct ranks in ascending order and their partial sums */
    int rl[64], nr = 0;
    double pd[64];
    float pf[64];
    for (int k = 0; k < cnt; ++k) {
      int seen = 0;
      for (int t = 0; t < nr; ++t) seen |= rl[t] == rank[k];
      if (!seen) rl[nr++] = rank[k];
    }
    for (int a = 1; a < nr; ++a) /* insertion sort, ascending */
      for (int b = a; b > 0 && rl[b - 1] > rl[b]; --b) {
        const int t = rl[b];
        rl[b] = rl[b - 1];
        rl[b - 1] = t;
      }
    for (int t = 0; t < nr; ++t) {
      int first = 1;
      pd[t] = 0.0;
      pf[t] = 0.f;
      for (int k = 0; k < cnt; ++k)
        if (rank[k] == rl[t]) {
          pd[t] = first ? (double)val[k] : pd[t] + (double)val[k];
          pf[t] = first ? val[k] : pf[t] + val[k];
          first = 0;
        }
    }
    for (int k = 0; k < cnt; ++k) {
      int own = 0;
      for (int t = 0; t < nr; ++t)
        if (rl[t] == rank[k]) own = t;
      double sd = pd[own];
      float sf = pf[own];
      for (int t = 0; t < nr; ++t)
        if (t != own) {
          sd = sd + pd[t];
          sf = sf + pf[t];
        }
      out[k] = acc64 ? (float)sd : sf;
    }
    for (int k = 0; k < cnt; ++k) v[m->gidx[o + k]] = out[k];
  }
  return ORC_OK;
}

/* O8: right-hand side b = M QQ^T (B f) */
void orc_rhs(const orc_mesh *m, const double *f, double *b) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m->nloc; ++i) b[i] = m->B[i] * f[i];
  orc_gs(m, b);
  orc_mask(m, b);
}

/* O9: assembled diagonal of A (before the Dirichlet mask), local diagonal
 *   sum_l D_li^2 Grr(l,j,k) + sum_l D_lj^2 Gss(i,l,k) + sum_l D_lk^2 Gtt(i,j,l)
 *   + 2 D_ii D_jj Grs + 2 D_ii D_kk Grt + 2 D_jj D_kk Gst + h B
 * followed by QQ^T; dinv = 1/diag on free entries and 0 on Dirichlet ones. */
void orc_diag(const orc_mesh *m, double *diag) {
  int n = m->n, n3 = m->n3;
  const double *D = m->D;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < m->E; ++e) {
    const double *G = m->G + (int64_t)e * 6 * n3;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int p = i + n * (j + n * k);
          double s = 0.0;
          for (int l = 0; l < n; ++l) {
            s += D[l * n + i] * D[l * n + i] * G[0 * n3 + l + n * (j + n * k)];
            s += D[l * n + j] * D[l * n + j] * G[3 * n3 + i + n * (l + n * k)];
            s += D[l * n + k] * D[l * n + k] * G[5 * n3 + i + n * (j + n * l)];
          }
          double dii = D[i * n + i], djj = D[j * n + j], dkk = D[k * n + k];
          s += 2.0 * dii * djj * G[1 * n3 + p];
          s += 2.0 * dii * dkk * G[2 * n3 + p];
          s += 2.0 * djj * dkk * G[4 * n3 + p];
          s += m->helm_h * m->B[(int64_t)e * n3 + p];
          diag[(int64_t)e * n3 + p] = s;
        }
  }
  orc_gs(m, diag);
}

/* ------------------------------------------------------------------------ */
/* Mesh creation / destruction / accessors                                   */
/* ------------------------------------------------------------------------ */
void orc_mesh_destroy(orc_mesh *m) {
  if (!m) return;
  free(m->xi);
  free(m->rho);
  free(m->D);
  free(m->G);
  free(m->B);
  free(m->goff);
  free(m->gidx);
  free(m->mult);
  free(m->c);
  free(m->mask);
  free(m->dinv);
  free(m);
}

/* xyz [E][3][n^3], glo [E][n^3] (global node ids), bnd [E][n^3] (nonzero on
 * Dirichlet nodes), kcoef [E][n^3] or NULL (k = 1), helm_h the Helmholtz
 * coefficient (0 for Poisson). */
int orc_mesh_create(int E, int N, const double *xyz, const int64_t *glo,
                    const unsigned char *bnd, const double *kcoef,
                    double helm_h, orc_mesh **out) {
  if (E < 1 || N < 1 || N > 32 || !xyz || !glo || !bnd || !out) return ORC_EINVAL;
  orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
  if (!m) return ORC_ENOMEM;
  m->E = E;
  m->N = N;
  m->n = N + 1;
  m->n3 = m->n * m->n * m->n;
  m->nloc = (int64_t)E * m->n3;
  m->helm_h = helm_h;
  m->xi = (double *)malloc(sizeof(double) * m->n);
  m->rho = (double *)malloc(sizeof(double) * m->n);
  m->D = (double *)malloc(sizeof(double) * m->n * m->n);
  m->G = (double *)malloc(sizeof(double) * 6 * m->nloc);
  m->B = (double *)malloc(sizeof(double) * m->nloc);
  m->mult = (double *)malloc(sizeof(double) * m->nloc);
  m->c = (double *)malloc(sizeof(double) * m->nloc);
  m->mask = (unsigned char *)malloc(m->nloc);
  m->dinv = (double *)malloc(sizeof(double) * m->nloc);
  if (!m->xi || !m->rho || !m->D || !m->G || !m->B || !m->mult || !m->c ||
      !m->mask || !m->dinv) {
    orc_mesh_destroy(m);
    return ORC_ENOMEM;
  }
  int rc = orc_gll(N, m->xi, m->rho);
  if (rc == ORC_OK) rc = orc_deriv(N, m->xi, m->D);
  if (rc == ORC_OK) rc = build_geometry(m, xyz, kcoef);
  if (rc == ORC_OK) rc = build_groups(m, glo);
  if (rc != ORC_OK) {
    orc_mesh_destroy(m);
    return rc;
  }
  for (int64_t i = 0; i < m->nloc; ++i) m->mask[i] = bnd[i] ? 1 : 0;
  for (int64_t q = 0; q < m->ngroups; ++q)
    for (int64_t t = m->goff[q] + 1; t < m->goff[q + 1]; ++t)
      if (m->mask[m->gidx[t]] != m->mask[m->gidx[m->goff[q]]]) {
        orc_mesh_destroy(m);
        return ORC_EMASK;
      }
  orc_diag(m, m->dinv);
  for (int64_t i = 0; i < m->nloc; ++i)
    m->dinv[i] = m->mask[i] ? 0.0 : 1.0 / m->dinv[i];
  *out = m;
  return ORC_OK;
}

int64_t orc_mesh_nloc(const orc_mesh *m) { return m->nloc; }
int orc_max_threads(void) { return omp_get_max_threads(); }
int64_t orc_mesh_ngroups(const orc_mesh *m) { return m->ngroups; }
double orc_mesh_mindet(const orc_mesh *m) { return m->mindet; }

/* copy-out accessors (arrays sized as documented at the struct) */
void orc_mesh_get(const orc_mesh *m, int what, double *out) {
  int64_t nl = m->nloc;
  switch (what) {
    case 0: memcpy(out, m->G, sizeof(double) * 6 * nl); break;
    case 1: memcpy(out, m->B, sizeof(double) * nl); break;
    case 2: memcpy(out, m->mult, sizeof(double) * nl); break;
    case 3: memcpy(out, m->c, sizeof(double) * nl); break;
    case 4: memcpy(out, m->dinv, sizeof(double) * nl); break;
    case 5: memcpy(out, m->D, sizeof(double) * m->n * m->n); break;
    case 6:
      for (int64_t i = 0; i < nl; ++i) out[i] = m->mask[i];
      break;
    default: break;
  }
}

/* ------------------------------------------------------------------------ */
/* Preconditioners (O9 Jacobi, identity) and an optional learned one.        */
/* ------------------------------------------------------------------------ */
typedef struct orc_nn orc_nn;
int orc_nn_apply(const orc_mesh *m, const orc_nn *nn, const double *r, double *z);

static void precond(const orc_mesh *m, int pc, const orc_nn *nn, const double *r,
                    double *z) {
  if (pc == ORC_PC_JACOBI) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->nloc; ++i) z[i] = m->dinv[i] * r[i];
  } else if (pc == ORC_PC_NN && nn) {
    orc_nn_apply(m, nn, r, z);
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->nloc; ++i) z[i] = m->mask[i] ? 0.0 : r[i];
  }
}

typedef struct {
  int iterations;
  int reason;
  int outer;
  int fallback;
  double rel_res_recursive;
  double rel_res_true;
} orc_stats;

/* stagnation: the best relative residual has not improved by >= 10% over
 * 500 consecutive iterations (a CG residual on a high-contrast coefficient
 * can plateau for hundreds of iterations before it falls again) */
typedef struct {
  double ref;
  int since;
} stag_t;
static int stag_update(stag_t *s, double res) {
  if (res < 0.9 * s->ref) {
    s->ref = res;
    s->since = 0;
    return 0;
  }
  return ++s->since >= 500;
}

static double true_rel_res(const orc_mesh *m, const double *b, const double *x,
                           double *tmp, double bnorm) {
  orc_apply(m, x, tmp);
  for (int64_t i = 0; i < m->nloc; ++i) tmp[i] = b[i] - tmp[i];
  return sqrt(orc_dot(m, tmp, tmp)) / bnorm;
}

/* O10: preconditioned CG with the c-weighted inner product.
 *   x = x0 (x0_given) or 0; r = b - A x; z = M^-1 r; p = z; rho = (r,z)_c
 *   loop: w = A p; sigma = (p,w)_c; alpha = rho/sigma;
 *         x += alpha p; r -= alpha w; stop if ||r||_c <= tol ||b||_c;
 *         z = M^-1 r; rho' = (r,z)_c; beta = rho'/rho; p = z + beta p.
 * history (nullable, maxit+1 entries) receives ||r||_c/||b||_c per
 * iteration (entry 0 = initial). */
int orc_pcg(const orc_mesh *m, int pc, const orc_nn *nn, const double *b,
            double *x, int x0_given, double tol, int maxit, double *history,
            orc_stats *st) {
  int64_t nl = m->nloc;
  double *r = (double *)malloc(sizeof(double) * nl);
  double *z = (double *)malloc(sizeof(double) * nl);
  double *p = (double *)malloc(sizeof(double) * nl);
  double *w = (double *)malloc(sizeof(double) * nl);
  if (!r || !z || !p || !w) {
    free(r); free(z); free(p); free(w);
    return ORC_ENOMEM;
  }
  double bnorm = sqrt(orc_dot(m, b, b));
  if (!x0_given) memset(x, 0, sizeof(double) * nl);
  if (x0_given) {
    orc_apply(m, x, w);
    for (int64_t i = 0; i < nl; ++i) r[i] = b[i] - w[i];
  } else {
    memcpy(r, b, sizeof(double) * nl);
  }
  st->iterations = 0;
  st->outer = 0;
  st->fallback = 0;
  st->reason = ORC_MAXITER;
  double res = bnorm > 0 ? sqrt(orc_dot(m, r, r)) / bnorm : 0.0;
  if (history) history[0] = res;
  if (bnorm == 0.0 || res <= tol) {
    st->reason = ORC_CONVERGED;
  } else {
    precond(m, pc, nn, r, z);
    memcpy(p, z, sizeof(double) * nl);
    double rho = orc_dot(m, r, z);
    stag_t sg = {res, 0};
    for (int it = 1; it <= maxit; ++it) {
      orc_apply(m, p, w);
      double sigma = orc_dot(m, p, w);
      if (!(sigma > 0.0) || !isfinite(sigma)) {
        st->reason = ORC_BREAKDOWN;
        break;
      }
      double alpha = rho / sigma;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nl; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * w[i];
      }
      st->iterations = it;
      res = sqrt(orc_dot(m, r, r)) / bnorm;
      if (history) history[it] = res;
      if (res <= tol) {
        st->reason = ORC_CONVERGED;
        break;
      }
      if (stag_update(&sg, res)) {
        st->reason = ORC_STAGNATED;
        break;
      }
      precond(m, pc, nn, r, z);
      double rho_new = orc_dot(m, r, z);
      double beta = rho_new / rho;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nl; ++i) p[i] = z[i] + beta * p[i];
      rho = rho_new;
    }
  }
  st->rel_res_recursive = res;
  st->rel_res_true = bnorm > 0 ? true_rel_res(m, b, x, w, bnorm) : 0.0;
  free(r); free(z); free(p); free(w);
  return ORC_OK;
}

/* O14: flexible CG with one-step truncation (Notay's FCG(1)):
 *   same as PCG except that the new direction is A-orthogonalised against
 *   the previous one, beta = -(z_k, A p_{k-1})_c / (p_{k-1}, A p_{k-1})_c,
 *   so the preconditioner may be any map r -> z.
 * Fallback (the Jacobi fallback of the learned preconditioner, read for the
 * FP32 loop's preconditioner of Sec. 5.2): a z whose (r,z)_c is not
 * positive or not finite, or whose (z, A p)_c is not finite, is replaced by
 * the Jacobi z for that step, the first z included; st->fallback counts the
 * replaced steps. */
int orc_fcg(const orc_mesh *m, int pc, const orc_nn *nn, const double *b,
            double *x, double tol, int maxit, double *history, orc_stats *st) {
  int64_t nl = m->nloc;
  double *r = (double *)malloc(sizeof(double) * nl);
  double *z = (double *)malloc(sizeof(double) * nl);
  double *p = (double *)malloc(sizeof(double) * nl);
  double *w = (double *)malloc(sizeof(double) * nl);
  if (!r || !z || !p || !w) {
    free(r); free(z); free(p); free(w);
    return ORC_ENOMEM;
  }
  double bnorm = sqrt(orc_dot(m, b, b));
  memset(x, 0, sizeof(double) * nl);
  memcpy(r, b, sizeof(double) * nl);
  st->iterations = 0;
  st->outer = 0;
  st->fallback = 0;
  st->reason = ORC_MAXITER;
  double res = bnorm > 0 ? 1.0 : 0.0;
  if (history) history[0] = res;
  if (bnorm == 0.0) {
    st->reason = ORC_CONVERGED;
  } else {
    precond(m, pc, nn, r, z);
    double rho = orc_dot(m, r, z);
    if (!(rho > 0.0) || !isfinite(rho)) {
      /* the first z is held to the same descent test as every later one */
      precond(m, ORC_PC_JACOBI, NULL, r, z);
      rho = orc_dot(m, r, z);
      st->fallback += 1;
    }
    memcpy(p, z, sizeof(double) * nl);
    stag_t sg = {res, 0};
    for (int it = 1; it <= maxit; ++it) {
      orc_apply(m, p, w);
      double sigma = orc_dot(m, p, w);
      if (!(sigma > 0.0) || !isfinite(sigma)) {
        st->reason = ORC_BREAKDOWN;
        break;
      }
      double alpha = rho / sigma;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nl; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * w[i];
      }
      st->iterations = it;
      res = sqrt(orc_dot(m, r, r)) / bnorm;
      if (history) history[it] = res;
      if (res <= tol) {
        st->reason = ORC_CONVERGED;
        break;
      }
      if (stag_update(&sg, res)) {
        st->reason = ORC_STAGNATED;
        break;
      }
      precond(m, pc, nn, r, z);
      double rz = orc_dot(m, r, z);
      double zw = orc_dot(m, z, w);
      if (!(rz > 0.0) || !isfinite(rz) || !isfinite(zw)) {
        /* non-descent direction from a learned map: use Jacobi for this step */
        precond(m, ORC_PC_JACOBI, NULL, r, z);
        rz = orc_dot(m, r, z);
        zw = orc_dot(m, z, w);
        st->fallback += 1;
      }
      double beta = -zw / sigma;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nl; ++i) p[i] = z[i] + beta * p[i];
      rho = rz;
    }
  }
  st->rel_res_recursive = res;
  st->rel_res_true = bnorm > 0 ? true_rel_res(m, b, x, w, bnorm) : 0.0;
  free(r); free(z); free(p); free(w);
  return ORC_OK;
}

/* O13: FP64 iterative refinement around an inner PCG.
 *   x = 0; loop: r = b - A x; s = ||r||_c; stop if s <= tol ||b||_c;
 *   d = PCG(A, r/s) to relative tolerance tau_in; x += s d.
 * The oracle runs the inner solve in FP64.  outer_res (nullable,
 * max_outer+1 entries) receives the true relative residual before each
 * outer step. */
int orc_ir(const orc_mesh *m, int pc, const double *b, double *x, double tol,
           double tau_in, int max_outer, int inner_maxit, double *outer_res,
           orc_stats *st) {
  int64_t nl = m->nloc;
  double *r = (double *)malloc(sizeof(double) * nl);
  double *d = (double *)malloc(sizeof(double) * nl);
  if (!r || !d) {
    free(r); free(d);
    return ORC_ENOMEM;
  }
  double bnorm = sqrt(orc_dot(m, b, b));
  memset(x, 0, sizeof(double) * nl);
  st->iterations = 0;
  st->outer = 0;
  st->fallback = 0;
  st->reason = ORC_MAXITER;
  double res = 0.0;
  for (int o = 0; o <= max_outer; ++o) {
    orc_apply(m, x, r);
    for (int64_t i = 0; i < nl; ++i) r[i] = b[i] - r[i];
    double s = sqrt(orc_dot(m, r, r));
    res = bnorm > 0 ? s / bnorm : 0.0;
    if (outer_res) outer_res[o] = res;
    if (res <= tol) {
      st->reason = ORC_CONVERGED;
      break;
    }
    if (o == max_outer) break;
    for (int64_t i = 0; i < nl; ++i) r[i] /= s;
    orc_stats ist;
    int rc = orc_pcg(m, pc, NULL, r, d, 0, tau_in, inner_maxit, NULL, &ist);
    if (rc != ORC_OK) {
      free(r); free(d);
      return rc;
    }
    st->iterations += ist.iterations;
    st->outer = o + 1;
    for (int64_t i = 0; i < nl; ++i) x[i] += s * d[i];
  }
  st->rel_res_recursive = res;
  st->rel_res_true = res;
  free(r); free(d);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O15: per-element learned correction to Jacobi (flexible-CG preconditioner) */
/*                                                                           */
/* For one element with local residual r_e (n^3 entries) and s_e =           */
/* ||dinv*r||_2 over the element:                                            */
/*   x0 = [r, dinv*r] / s_e                       (2 input channels)         */
/*   a1[c](p) = sum_ci sum_o W1[c][ci][o] x0[ci](p+o)   (3x3x3, zero pad)    */
/*   h = max(a1, 0)                               (ch hidden channels)       */
/*   y(p) = sum_c sum_o W2[c][o] h[c](p+o)                                   */
/*   zL = dinv*r + s_e * y                                                   */
/* and the preconditioned vector is z = M QQ^T (c * zL).  Offsets o index    */
/* (di,dj,dk) in {-1,0,1}^3 as o = (di+1) + 3 (dj+1) + 9 (dk+1).  No bias, so */
/* the map is positively homogeneous in r.                                   */
/* ------------------------------------------------------------------------ */
struct orc_nn {
  int cin, ch;
  double *W1; /* [ch][cin][27] */
  double *W2; /* [ch][27] */
};

int orc_nn_create(int cin, int ch, const double *W1, const double *W2, orc_nn **out) {
  if (cin != 2 || ch < 1 || !W1 || !W2 || !out) return ORC_EINVAL;
  orc_nn *nn = (orc_nn *)calloc(1, sizeof(orc_nn));
  if (!nn) return ORC_ENOMEM;
  nn->cin = cin;
  nn->ch = ch;
  nn->W1 = (double *)malloc(sizeof(double) * ch * cin * 27);
  nn->W2 = (double *)malloc(sizeof(double) * ch * 27);
  if (!nn->W1 || !nn->W2) {
    free(nn->W1); free(nn->W2); free(nn);
    return ORC_ENOMEM;
  }
  memcpy(nn->W1, W1, sizeof(double) * ch * cin * 27);
  memcpy(nn->W2, W2, sizeof(double) * ch * 27);
  *out = nn;
  return ORC_OK;
}

void orc_nn_destroy(orc_nn *nn) {
  if (!nn) return;
  free(nn->W1);
  free(nn->W2);
  free(nn);
}

void orc_nn_set(orc_nn *nn, const double *W1, const double *W2) {
  memcpy(nn->W1, W1, sizeof(double) * nn->ch * nn->cin * 27);
  memcpy(nn->W2, W2, sizeof(double) * nn->ch * 27);
}

/* neighbour index of node (i,j,k) at offset o, or -1 outside the element */
static int nbr(int n, int i, int j, int k, int o) {
  int ii = i + (o % 3) - 1, jj = j + ((o / 3) % 3) - 1, kk = k + (o / 9) - 1;
  if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) return -1;
  return ii + n * (jj + n * kk);
}

/* forward pass of one element; x0 [cin][n3], a1 [ch][n3], y [n3] */
static void nn_elem_forward(const orc_nn *nn, int n, const double *x0, double *a1,
                            double *y) {
  int n3 = n * n * n;
  for (int c = 0; c < nn->ch; ++c)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int ci = 0; ci < nn->cin; ++ci)
            for (int o = 0; o < 27; ++o) {
              int q = nbr(n, i, j, k, o);
              if (q >= 0) s += nn->W1[(c * nn->cin + ci) * 27 + o] * x0[ci * n3 + q];
            }
          a1[c * n3 + i + n * (j + n * k)] = s;
        }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int c = 0; c < nn->ch; ++c)
          for (int o = 0; o < 27; ++o) {
            int q = nbr(n, i, j, k, o);
            if (q >= 0) {
              double hv = a1[c * n3 + q] > 0.0 ? a1[c * n3 + q] : 0.0;
              s += nn->W2[c * 27 + o] * hv;
            }
          }
        y[i + n * (j + n * k)] = s;
      }
}

/* element scale s_e and network input */
static double nn_elem_input(const orc_mesh *m, int e, const double *r, double *x0) {
  int n3 = m->n3;
  double s2 = 0.0;
  for (int p = 0; p < n3; ++p) {
    double v = m->dinv[(int64_t)e * n3 + p] * r[(int64_t)e * n3 + p];
    s2 += v * v;
  }
  double s = sqrt(s2);
  for (int p = 0; p < n3; ++p) {
    double rv = r[(int64_t)e * n3 + p];
    double dv = m->dinv[(int64_t)e * n3 + p] * rv;
    x0[p] = s > 0.0 ? rv / s : 0.0;
    x0[n3 + p] = s > 0.0 ? dv / s : 0.0;
  }
  return s;
}

/* zL (unassembled) and, optionally, the raw network output y */
void orc_nn_local(const orc_mesh *m, const orc_nn *nn, const double *r, double *zL,
                  double *yout) {
  int n3 = m->n3;
#pragma omp parallel
  {
    double *x0 = (double *)malloc(sizeof(double) * 2 * n3);
    double *a1 = (double *)malloc(sizeof(double) * nn->ch * n3);
    double *y = (double *)malloc(sizeof(double) * n3);
#pragma omp for schedule(static)
    for (int e = 0; e < m->E; ++e) {
      double s = nn_elem_input(m, e, r, x0);
      if (s > 0.0)
        nn_elem_forward(nn, m->n, x0, a1, y);
      else
        memset(y, 0, sizeof(double) * n3);
      for (int p = 0; p < n3; ++p) {
        int64_t g = (int64_t)e * n3 + p;
        zL[g] = m->dinv[g] * r[g] + s * y[p];
        if (yout) yout[g] = y[p];
      }
    }
    free(x0); free(a1); free(y);
  }
}

/* z = M QQ^T (c * zL) */
int orc_nn_apply(const orc_mesh *m, const orc_nn *nn, const double *r, double *z) {
  orc_nn_local(m, nn, r, z, NULL);
  for (int64_t i = 0; i < m->nloc; ++i) z[i] *= m->c[i];
  orc_gs(m, z);
  orc_mask(m, z);
  return ORC_OK;
}

/* Loss and gradient over nsamp pairs (R[s], Eerr[s]), each a local vector:
 *   L_s = ||z_s - e_s||_A^2 / ||e_s||_A^2,   ||v||_A^2 = (v, A v)_c,
 *   loss = mean_s L_s.
 * With z = M QQ^T (c * zL), dL_s/dzL = 2 c * A(z_s - e_s) / ||e_s||_A^2,
 * dL/dy = s_e dL/dzL, then the two convolutions are differentiated by the
 * chain rule.  gW1 [ch][cin][27], gW2 [ch][27] receive the mean gradient. */
int orc_nn_loss_grad(const orc_mesh *m, const orc_nn *nn, int nsamp, const double *R,
                     const double *Eerr, double *loss, double *gW1, double *gW2) {
  int64_t nl = m->nloc;
  int n = m->n, n3 = m->n3, ch = nn->ch, cin = nn->cin;
  double *z = (double *)malloc(sizeof(double) * nl);
  double *d = (double *)malloc(sizeof(double) * nl);
  double *Ad = (double *)malloc(sizeof(double) * nl);
  double *Ae = (double *)malloc(sizeof(double) * nl);
  if (!z || !d || !Ad || !Ae) {
    free(z); free(d); free(Ad); free(Ae);
    return ORC_ENOMEM;
  }
  memset(gW1, 0, sizeof(double) * ch * cin * 27);
  memset(gW2, 0, sizeof(double) * ch * 27);
  double total = 0.0;
  double *gw1e = (double *)calloc((size_t)m->E * ch * cin * 27, sizeof(double));
  double *gw2e = (double *)calloc((size_t)m->E * ch * 27, sizeof(double));
  if (!gw1e || !gw2e) {
    free(z); free(d); free(Ad); free(Ae); free(gw1e); free(gw2e);
    return ORC_ENOMEM;
  }
  for (int s = 0; s < nsamp; ++s) {
    const double *r = R + (int64_t)s * nl;
    const double *e = Eerr + (int64_t)s * nl;
    orc_nn_apply(m, nn, r, z);
    for (int64_t i = 0; i < nl; ++i) d[i] = z[i] - e[i];
    orc_apply(m, d, Ad);
    orc_apply(m, e, Ae);
    double num = orc_dot(m, d, Ad), den = orc_dot(m, e, Ae);
    total += num / den;
    /* per-element backward; per-element partial gradients are summed below
     * in ascending element order */
#pragma omp parallel
    {
      double *x0 = (double *)malloc(sizeof(double) * 2 * n3);
      double *a1 = (double *)malloc(sizeof(double) * ch * n3);
      double *y = (double *)malloc(sizeof(double) * n3);
      double *gy = (double *)malloc(sizeof(double) * n3);
      double *ga = (double *)malloc(sizeof(double) * ch * n3);
#pragma omp for schedule(static)
      for (int el = 0; el < m->E; ++el) {
        double *g1 = gw1e + (size_t)el * ch * cin * 27;
        double *g2 = gw2e + (size_t)el * ch * 27;
        memset(g1, 0, sizeof(double) * ch * cin * 27);
        memset(g2, 0, sizeof(double) * ch * 27);
        double se = nn_elem_input(m, el, r, x0);
        if (!(se > 0.0)) continue;
        nn_elem_forward(nn, n, x0, a1, y);
        for (int p = 0; p < n3; ++p) {
          int64_t gI = (int64_t)el * n3 + p;
          gy[p] = se * 2.0 * m->c[gI] * Ad[gI] / den;
        }
        /* layer 2: y(p) = sum_c sum_o W2[c][o] h[c](p+o) */
        for (int c = 0; c < ch; ++c)
          for (int q = 0; q < n3; ++q) ga[c * n3 + q] = 0.0;
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              int p = i + n * (j + n * k);
              for (int c = 0; c < ch; ++c)
                for (int o = 0; o < 27; ++o) {
                  int q = nbr(n, i, j, k, o);
                  if (q < 0) continue;
                  double hv = a1[c * n3 + q] > 0.0 ? a1[c * n3 + q] : 0.0;
                  g2[c * 27 + o] += gy[p] * hv;
                  ga[c * n3 + q] += nn->W2[c * 27 + o] * gy[p];
                }
            }
        /* ReLU */
        for (int c = 0; c < ch; ++c)
          for (int q = 0; q < n3; ++q)
            if (!(a1[c * n3 + q] > 0.0)) ga[c * n3 + q] = 0.0;
        /* layer 1: a1[c](p) = sum_ci sum_o W1[c][ci][o] x0[ci](p+o) */
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              int p = i + n * (j + n * k);
              for (int c = 0; c < ch; ++c)
                for (int ci = 0; ci < cin; ++ci)
                  for (int o = 0; o < 27; ++o) {
                    int q = nbr(n, i, j, k, o);
                    if (q < 0) continue;
                    g1[(c * cin + ci) * 27 + o] += ga[c * n3 + p] * x0[ci * n3 + q];
                  }
            }
      }
      free(x0); free(a1); free(y); free(gy); free(ga);
    }
    for (int el = 0; el < m->E; ++el) {
      for (int t = 0; t < ch * cin * 27; ++t) gW1[t] += gw1e[(size_t)el * ch * cin * 27 + t];
      for (int t = 0; t < ch * 27; ++t) gW2[t] += gw2e[(size_t)el * ch * 27 + t];
    }
  }
  for (int t = 0; t < ch * cin * 27; ++t) gW1[t] /= nsamp;
  for (int t = 0; t < ch * 27; ++t) gW2[t] /= nsamp;
  *loss = total / nsamp;
  free(z); free(d); free(Ad); free(Ae); free(gw1e); free(gw2e);
  return ORC_OK;
}

/* Adam (Kingma & Ba), step t >= 1, bias-corrected moments. */
void orc_adam(int np, double *theta, const double *g, double *mo, double *ve, int t,
              double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int i = 0; i < np; ++i) {
    mo[i] = b1 * mo[i] + (1.0 - b1) * g[i];
    ve[i] = b2 * ve[i] + (1.0 - b2) * g[i] * g[i];
    double mh = mo[i] / c1, vh = ve[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
