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
#define ORC_PC_MG 3

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
typedef struct orc_mg orc_mg;
int orc_nn_apply(const orc_mesh *m, const orc_nn *nn, const double *r, double *z);
void orc_mg_apply(const orc_mesh *m, const orc_mg *mg, const double *r, double *z);

/* z = M^-1 r; pcobj is the network (ORC_PC_NN) or the multigrid
 * preconditioner (ORC_PC_MG) */
static void precond(const orc_mesh *m, int pc, const void *pcobj, const double *r,
                    double *z) {
  if (pc == ORC_PC_JACOBI) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->nloc; ++i) z[i] = m->dinv[i] * r[i];
  } else if (pc == ORC_PC_NN && pcobj) {
    orc_nn_apply(m, (const orc_nn *)pcobj, r, z);
  } else if (pc == ORC_PC_MG && pcobj) {
    orc_mg_apply(m, (const orc_mg *)pcobj, r, z);
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
int orc_pcg(const orc_mesh *m, int pc, const void *nn, const double *b,
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
int orc_fcg(const orc_mesh *m, int pc, const void *nn, const double *b,
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

/* ------------------------------------------------------------------------ */
/* Two-level Schwarz / multigrid preconditioner for box meshes.              */
/*                                                                           */
/* The paper's multigrid preconditioner (solveM in the CG-loop profiling     */
/* table, 70% of the time with it; Sec. 4.2, inspection of the              */
/* preconditioned CG: the Schwarz weights are square roots, and single-      */
/* precision square roots made the mixed solve stagnate) is Nekbone's; the   */
/* paper gives none of its algorithm.  The reading taken is the textbook     */
/* two-level additive Schwarz method (Dryja and Widlund) with the spectral-  */
/* element local solves of hybrid Schwarz/multigrid (Lottes and Fischer):    */
/*                                                                           */
/*   z = M QQ^T( ws * FDM_e( ws * r_L ) )  +  P V( P^T r )                   */
/*                                                                           */
/*  - ws = sqrt(c), c = 1/m: the counting weights of the overlapping        */
/*    subdomains, split symmetrically (square root taken in FP64);           */
/*  - FDM_e: the exact inverse, by fast diagonalisation, of a separable      */
/*    operator on element e extended by one GLL interval into each           */
/*    neighbour with zero Dirichlet values at the extended ends.  Per        */
/*    direction, the 1-D stiffness and mass of the element (mean length l,   */
/*    mean coefficient k) gain at each shared face the face-node diagonal    */
/*    entry of the neighbour's 1-D matrices; at a Dirichlet face the face    */
/*    node is decoupled.  A = k (Bz Bx By Ax + ...) + h Bz By Bx is inverted  */
/*    through the generalised eigenpairs A_d s = lambda B_d s, S^T B S = I;  */
/*  - P: trilinear interpolation from the element-vertex lattice (order 1)  */
/*    to the element's GLL nodes; the coarse operator is Galerkin, P^T A P,  */
/*    assembled from the 8x8 element matrices as a 27-point lattice stencil; */
/*  - V: one V-cycle of geometric multigrid on the lattice: two damped       */
/*    Jacobi sweeps before and after the coarse correction (damping 1 over  */
/*    the row-sum bound of D^-1 A), full-weighting restriction (transpose of */
/*    trilinear interpolation), Galerkin coarse stencils, coarsening by two  */
/*    while the intervals are even and the level has more unknowns than the  */
/*    coarsest limit, and a dense Cholesky solve on the coarsest level.      */
/* The box structure (E = ne^3 elements in lexicographic order, global ids  */
/* on the lattice of GLL nodes, Dirichlet on the whole boundary) gives the  */
/* neighbours and the lattice.                                               */
/* ------------------------------------------------------------------------ */
#define ORC_MG_MAXLEV 12

typedef struct {
  int nI;       /* lattice intervals per direction */
  int nu;       /* unknowns per direction (interior lattice nodes) */
  double *st;   /* [nu^3][27] stencil, offset s = (dx+1) + 3(dy+1) + 9(dz+1) */
  double omega; /* Jacobi damping */
} orc_lvl;

struct orc_mg {
  int ne, n, E;
  double *S;    /* [E][3][n][n]: S[e][d][node][mode] */
  double *lam;  /* [E][3][n] */
  double *kbar; /* [E] */
  double ws[256];
  int nlev;
  orc_lvl lv[ORC_MG_MAXLEV];
  int nc;       /* unknowns of the coarsest level */
  double *L;    /* its dense Cholesky factor, lower triangle [nc][nc] */
};

static int lat_idx(int nu, int I, int J, int K) { return (I - 1) + nu * ((J - 1) + nu * (K - 1)); }

/* eigenvalues and eigenvectors of a symmetric matrix by cyclic Jacobi
 * rotations: A (n x n, destroyed) = Q diag(w) Q^T, Q[i][j] column j */
static void jacobi_eigen(int n, double *A, double *w, double *Q) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[i * n + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) { /* A <- A J (columns p, q) */
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) { /* A <- J^T A (rows p, q) */
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) { /* Q <- Q J */
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

/* mean length of element e along direction d: distance between the two end
 * nodes of each of its n^2 lines along d, averaged */
static double elem_length(const orc_mesh *m, const double *xyz, int e, int d) {
  int n = m->n, N = m->N;
  const double *X = xyz + (int64_t)e * 3 * m->n3;
  double sum = 0.0;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      int p0, p1;
      if (d == 0) { p0 = 0 + n * (a + n * b); p1 = N + n * (a + n * b); }
      else if (d == 1) { p0 = a + n * (0 + n * b); p1 = a + n * (N + n * b); }
      else { p0 = a + n * (b + n * 0); p1 = a + n * (b + n * N); }
      double dx = X[p1] - X[p0], dy = X[m->n3 + p1] - X[m->n3 + p0];
      double dz = X[2 * m->n3 + p1] - X[2 * m->n3 + p0];
      sum += sqrt(dx * dx + dy * dy + dz * dz);
    }
  return sum / (n * n);
}

/* the 1-D extended operator of one element and direction, and its
 * generalised eigenpairs (S = B^-1/2 Q, so S^T B S = I, S^T A S = diag) */
static void fdm_1d(int n, const double *Ar, const double *rho, double l, double llo, double lhi,
                   int dlo, int dhi, double *S, double *lam) {
  int N = n - 1;
  double A[32 * 32], B[32], C[32 * 32], Q[32 * 32];
  for (int i = 0; i < n; ++i) {
    B[i] = 0.5 * l * rho[i];
    for (int j = 0; j < n; ++j) A[i * n + j] = (2.0 / l) * Ar[i * n + j];
  }
  if (llo > 0.0) {
    A[0] += (2.0 / llo) * Ar[N * n + N];
    B[0] += 0.5 * llo * rho[N];
  }
  if (lhi > 0.0) {
    A[N * n + N] += (2.0 / lhi) * Ar[0];
    B[N] += 0.5 * lhi * rho[0];
  }
  int ends[2] = {dlo ? 0 : -1, dhi ? N : -1};
  for (int t = 0; t < 2; ++t) {
    int q = ends[t];
    if (q < 0) continue;
    for (int j = 0; j < n; ++j) A[q * n + j] = A[j * n + q] = 0.0;
    A[q * n + q] = 1.0;
    B[q] = 1.0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i * n + j] = A[i * n + j] / sqrt(B[i] * B[j]);
  jacobi_eigen(n, C, lam, Q);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = Q[i * n + j] / sqrt(B[i]);
}

static void lvl_apply(const orc_lvl *L, const double *x, double *y) {
  int nu = L->nu;
#pragma omp parallel for schedule(static)
  for (int K = 1; K <= nu; ++K)
    for (int J = 1; J <= nu; ++J)
      for (int I = 1; I <= nu; ++I) {
        const double *a = L->st + 27 * (int64_t)lat_idx(nu, I, J, K);
        double s = 0.0;
        for (int t = 0; t < 27; ++t) {
          int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
          if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
          s += a[t] * x[lat_idx(nu, i2, j2, k2)];
        }
        y[lat_idx(nu, I, J, K)] = s;
      }
}

/* trilinear interpolation weight of coarse node c at fine lattice node f
 * (per direction: 1 at f = 2c, 1/2 at f = 2c +- 1) */
static double pw1(int f, int c) {
  int d = f - 2 * c;
  return d == 0 ? 1.0 : (d == 1 || d == -1) ? 0.5 : 0.0;
}

/* Galerkin coarse stencil P^T A_f P of a lattice level (coarse nodes c,
 * fine nodes f = 2c + delta, and every fine stencil neighbour's coarse
 * parents) */
static void lvl_rap(const orc_lvl *F, orc_lvl *Cl) {
  int nuf = F->nu, nuc = Cl->nu;
  memset(Cl->st, 0, sizeof(double) * 27 * (size_t)nuc * nuc * nuc);
  for (int K = 1; K <= nuc; ++K)
    for (int J = 1; J <= nuc; ++J)
      for (int I = 1; I <= nuc; ++I) {
        double *ac = Cl->st + 27 * (int64_t)lat_idx(nuc, I, J, K);
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int fi = 2 * I + dx, fj = 2 * J + dy, fk = 2 * K + dz;
              double w = pw1(fi, I) * pw1(fj, J) * pw1(fk, K);
              const double *af = F->st + 27 * (int64_t)lat_idx(nuf, fi, fj, fk);
              for (int t = 0; t < 27; ++t) {
                int gi = fi + t % 3 - 1, gj = fj + (t / 3) % 3 - 1, gk = fk + t / 9 - 1;
                if (gi < 1 || gj < 1 || gk < 1 || gi > nuf || gj > nuf || gk > nuf) continue;
                double wa = w * af[t];
                for (int ck = gk / 2; ck <= (gk + 1) / 2; ++ck)
                  for (int cj = gj / 2; cj <= (gj + 1) / 2; ++cj)
                    for (int ci = gi / 2; ci <= (gi + 1) / 2; ++ci) {
                      if (ci < 1 || cj < 1 || ck < 1 || ci > nuc || cj > nuc || ck > nuc) continue;
                      double p2 = pw1(gi, ci) * pw1(gj, cj) * pw1(gk, ck);
                      if (p2 == 0.0) continue;
                      int s = (ci - I + 1) + 3 * (cj - J + 1) + 9 * (ck - K + 1);
                      ac[s] += wa * p2;
                    }
              }
            }
      }
}

static double lvl_omega(const orc_lvl *L) {
  int nu = L->nu;
  double mx = 0.0;
  for (int K = 1; K <= nu; ++K)
    for (int J = 1; J <= nu; ++J)
      for (int I = 1; I <= nu; ++I) {
        const double *a = L->st + 27 * (int64_t)lat_idx(nu, I, J, K);
        double s = 0.0;
        for (int t = 0; t < 27; ++t) {
          int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
          if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
          s += fabs(a[t]);
        }
        if (s / a[13] > mx) mx = s / a[13];
      }
  return 1.0 / mx;
}

void orc_mg_destroy(orc_mg *mg) {
  if (!mg) return;
  free(mg->S);
  free(mg->lam);
  free(mg->kbar);
  for (int l = 0; l < mg->nlev; ++l) free(mg->lv[l].st);
  free(mg->L);
  free(mg);
}

/* J[i][a]: the order-1 basis at GLL node i ((1 - xi)/2, (1 + xi)/2) */
static void lin_basis(const orc_mesh *m, double *J) {
  for (int i = 0; i < m->n; ++i) {
    J[2 * i] = 0.5 * (1.0 - m->xi[i]);
    J[2 * i + 1] = 0.5 * (1.0 + m->xi[i]);
  }
}

/* Builds the preconditioner.  ne: elements per direction (E = ne^3); xyz and
 * kcoef (nullable) as given to orc_mesh_create; coarsest_max: largest
 * number of unknowns solved directly.  Returns ORC_EINVAL when the mesh is
 * not a Dirichlet box of lexicographic elements, or when the coarsest level
 * would exceed 4096 unknowns. */
int orc_mg_create(const orc_mesh *m, int ne, const double *xyz, const double *kcoef,
                  int coarsest_max, orc_mg **out) {
  int n = m->n, N = m->N, n3 = m->n3, E = m->E;
  if (ne < 2 || (int64_t)ne * ne * ne != E || !xyz || !out) return ORC_EINVAL;
  /* every node of the domain boundary is Dirichlet: the box faces of the
   * boundary elements */
  for (int e = 0; e < E; ++e) {
    int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          int onb = (ex == 0 && i == 0) || (ex == ne - 1 && i == N) || (ey == 0 && j == 0) ||
                    (ey == ne - 1 && j == N) || (ez == 0 && k == 0) || (ez == ne - 1 && k == N);
          if (onb != m->mask[(int64_t)e * n3 + i + n * (j + n * k)]) return ORC_EINVAL;
        }
  }
  orc_mg *mg = (orc_mg *)calloc(1, sizeof(orc_mg));
  if (!mg) return ORC_ENOMEM;
  mg->ne = ne;
  mg->n = n;
  mg->E = E;
  for (int q = 1; q < 256; ++q) mg->ws[q] = sqrt(1.0 / q);
  mg->S = (double *)malloc(sizeof(double) * (size_t)E * 3 * n * n);
  mg->lam = (double *)malloc(sizeof(double) * (size_t)E * 3 * n);
  mg->kbar = (double *)malloc(sizeof(double) * E);
  double *len = (double *)malloc(sizeof(double) * (size_t)E * 3);
  double *Ar = (double *)malloc(sizeof(double) * n * n);
  if (!mg->S || !mg->lam || !mg->kbar || !len || !Ar) {
    free(len); free(Ar);
    orc_mg_destroy(mg);
    return ORC_ENOMEM;
  }
  /* reference 1-D stiffness D^T diag(rho) D */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += m->D[l * n + i] * m->rho[l] * m->D[l * n + j];
      Ar[i * n + j] = s;
    }
  for (int e = 0; e < E; ++e) {
    for (int d = 0; d < 3; ++d) len[3 * e + d] = elem_length(m, xyz, e, d);
    double kb = 0.0;
    for (int p = 0; p < n3; ++p) kb += kcoef ? kcoef[(int64_t)e * n3 + p] : 1.0;
    mg->kbar[e] = kb / n3;
  }
  for (int e = 0; e < E; ++e) {
    int ec[3] = {e % ne, (e / ne) % ne, e / (ne * ne)};
    int stride[3] = {1, ne, ne * ne};
    for (int d = 0; d < 3; ++d) {
      double llo = ec[d] > 0 ? len[3 * (e - stride[d]) + d] : 0.0;
      double lhi = ec[d] < ne - 1 ? len[3 * (e + stride[d]) + d] : 0.0;
      fdm_1d(n, Ar, m->rho, len[3 * e + d], llo, lhi, ec[d] == 0, ec[d] == ne - 1,
             mg->S + ((size_t)e * 3 + d) * n * n, mg->lam + ((size_t)e * 3 + d) * n);
    }
  }
  free(len);
  free(Ar);
  /* coarse level 0: element-vertex lattice, Galerkin element matrices */
  int nI = ne, nlev = 0;
  for (;;) {
    orc_lvl *L = &mg->lv[nlev];
    L->nI = nI;
    L->nu = nI - 1;
    L->st = (double *)calloc(27 * (size_t)L->nu * L->nu * L->nu, sizeof(double));
    if (!L->st) { mg->nlev = nlev + 1; orc_mg_destroy(mg); return ORC_ENOMEM; }
    ++nlev;
    int nunk = L->nu * L->nu * L->nu;
    if (nunk <= coarsest_max || nI % 2 || nI < 4 || nlev == ORC_MG_MAXLEV) break;
    nI /= 2;
  }
  mg->nlev = nlev;
  {
    double J[64];
    lin_basis(m, J);
    double *u = (double *)malloc(sizeof(double) * m->nloc);
    double *w = (double *)malloc(sizeof(double) * m->nloc);
    double *K = (double *)malloc(sizeof(double) * (size_t)E * 64);
    if (!u || !w || !K) { free(u); free(w); free(K); orc_mg_destroy(mg); return ORC_ENOMEM; }
    for (int a = 0; a < 8; ++a) {
      for (int e = 0; e < E; ++e)
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
              u[(int64_t)e * n3 + i + n * (j + n * k)] =
                  J[2 * i + (a & 1)] * J[2 * j + ((a >> 1) & 1)] * J[2 * k + (a >> 2)];
      orc_ax_local(m, u, w);
      for (int e = 0; e < E; ++e)
        for (int b = 0; b < 8; ++b) {
          double s = 0.0;
          for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i)
                s += J[2 * i + (b & 1)] * J[2 * j + ((b >> 1) & 1)] * J[2 * k + (b >> 2)] *
                     w[(int64_t)e * n3 + i + n * (j + n * k)];
          K[(size_t)e * 64 + b * 8 + a] = s;
        }
    }
    orc_lvl *L0 = &mg->lv[0];
    int nu = L0->nu;
    for (int e = 0; e < E; ++e) {
      int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
      for (int b = 0; b < 8; ++b) {
        int I = ex + (b & 1), Jn = ey + ((b >> 1) & 1), Kn = ez + (b >> 2);
        if (I < 1 || Jn < 1 || Kn < 1 || I > nu || Jn > nu || Kn > nu) continue;
        for (int a = 0; a < 8; ++a) {
          int I2 = ex + (a & 1), J2 = ey + ((a >> 1) & 1), K2 = ez + (a >> 2);
          if (I2 < 1 || J2 < 1 || K2 < 1 || I2 > nu || J2 > nu || K2 > nu) continue;
          int s = (I2 - I + 1) + 3 * (J2 - Jn + 1) + 9 * (K2 - Kn + 1);
          L0->st[27 * (int64_t)lat_idx(nu, I, Jn, Kn) + s] += K[(size_t)e * 64 + b * 8 + a];
        }
      }
    }
    free(u); free(w); free(K);
  }
  for (int l = 1; l < nlev; ++l) lvl_rap(&mg->lv[l - 1], &mg->lv[l]);
  for (int l = 0; l < nlev; ++l) mg->lv[l].omega = lvl_omega(&mg->lv[l]);
  /* coarsest: dense Cholesky */
  orc_lvl *Lc = &mg->lv[nlev - 1];
  int nc = Lc->nu * Lc->nu * Lc->nu;
  if (nc > 4096) { orc_mg_destroy(mg); return ORC_EINVAL; }
  mg->nc = nc;
  mg->L = (double *)calloc((size_t)nc * nc, sizeof(double));
  if (!mg->L) { orc_mg_destroy(mg); return ORC_ENOMEM; }
  {
    int nu = Lc->nu;
    double *Ad = mg->L;
    for (int K = 1; K <= nu; ++K)
      for (int J = 1; J <= nu; ++J)
        for (int I = 1; I <= nu; ++I) {
          int r = lat_idx(nu, I, J, K);
          for (int t = 0; t < 27; ++t) {
            int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
            if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
            Ad[(size_t)r * nc + lat_idx(nu, i2, j2, k2)] = Lc->st[27 * (int64_t)r + t];
          }
        }
    for (int j = 0; j < nc; ++j) { /* in-place Cholesky, lower triangle */
      double d = Ad[(size_t)j * nc + j];
      for (int k = 0; k < j; ++k) d -= Ad[(size_t)j * nc + k] * Ad[(size_t)j * nc + k];
      if (!(d > 0.0)) { orc_mg_destroy(mg); return ORC_EINVAL; }
      d = sqrt(d);
      Ad[(size_t)j * nc + j] = d;
      for (int i = j + 1; i < nc; ++i) {
        double s = Ad[(size_t)i * nc + j];
        for (int k = 0; k < j; ++k) s -= Ad[(size_t)i * nc + k] * Ad[(size_t)j * nc + k];
        Ad[(size_t)i * nc + j] = s / d;
      }
    }
  }
  *out = mg;
  return ORC_OK;
}

/* one V-cycle on lattice level l for right-hand side b; x receives the result */
static void vcycle(const orc_mg *mg, int l, const double *b, double *x) {
  const orc_lvl *L = &mg->lv[l];
  int nu = L->nu, nn = nu * nu * nu;
  if (l == mg->nlev - 1) {
    const double *Lf = mg->L;
    int nc = mg->nc;
    for (int i = 0; i < nc; ++i) { /* L y = b */
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= Lf[(size_t)i * nc + k] * x[k];
      x[i] = s / Lf[(size_t)i * nc + i];
    }
    for (int i = nc - 1; i >= 0; --i) { /* L^T x = y */
      double s = x[i];
      for (int k = i + 1; k < nc; ++k) s -= Lf[(size_t)k * nc + i] * x[k];
      x[i] = s / Lf[(size_t)i * nc + i];
    }
    return;
  }
  double *r = (double *)malloc(sizeof(double) * nn);
  const orc_lvl *C = &mg->lv[l + 1];
  int nuc = C->nu, nnc = nuc * nuc * nuc;
  double *bc = (double *)malloc(sizeof(double) * nnc);
  double *xc = (double *)malloc(sizeof(double) * nnc);
  memset(x, 0, sizeof(double) * nn);
  for (int sweep = 0; sweep < 4; ++sweep) {
    if (sweep == 2) {
      /* coarse correction: r = b - A x, bc = P^T r, x += P V(bc) */
      lvl_apply(L, x, r);
      for (int i = 0; i < nn; ++i) r[i] = b[i] - r[i];
      for (int K = 1; K <= nuc; ++K)
        for (int J = 1; J <= nuc; ++J)
          for (int I = 1; I <= nuc; ++I) {
            double s = 0.0;
            for (int dz = -1; dz <= 1; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                  s += pw1(2 * I + dx, I) * pw1(2 * J + dy, J) * pw1(2 * K + dz, K) *
                       r[lat_idx(nu, 2 * I + dx, 2 * J + dy, 2 * K + dz)];
            bc[lat_idx(nuc, I, J, K)] = s;
          }
      vcycle(mg, l + 1, bc, xc);
      for (int K = 1; K <= nu; ++K)
        for (int J = 1; J <= nu; ++J)
          for (int I = 1; I <= nu; ++I) {
            double s = 0.0;
            for (int ck = K / 2; ck <= (K + 1) / 2; ++ck)
              for (int cj = J / 2; cj <= (J + 1) / 2; ++cj)
                for (int ci = I / 2; ci <= (I + 1) / 2; ++ci) {
                  if (ci < 1 || cj < 1 || ck < 1 || ci > nuc || cj > nuc || ck > nuc) continue;
                  s += pw1(I, ci) * pw1(J, cj) * pw1(K, ck) * xc[lat_idx(nuc, ci, cj, ck)];
                }
            x[lat_idx(nu, I, J, K)] += s;
          }
    }
    /* damped Jacobi: x += omega D^-1 (b - A x) */
    lvl_apply(L, x, r);
    for (int K = 1; K <= nu; ++K)
      for (int J = 1; J <= nu; ++J)
        for (int I = 1; I <= nu; ++I) {
          int q = lat_idx(nu, I, J, K);
          x[q] += L->omega * (b[q] - r[q]) / L->st[27 * (int64_t)q + 13];
        }
  }
  free(r); free(bc); free(xc);
}

/* the Schwarz part before assembly: zL = ws * FDM_e(ws * r) per element */
void orc_mg_schwarz_local(const orc_mesh *m, const orc_mg *mg, const double *r, double *zL) {
  int n = m->n, n3 = m->n3;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < m->E; ++e) {
    double v[4096], u[4096];
    const double *Sx = mg->S + ((size_t)e * 3 + 0) * n * n, *Sy = Sx + n * n, *Sz = Sy + n * n;
    const double *lx = mg->lam + (size_t)e * 3 * n, *ly = lx + n, *lz = ly + n;
    int64_t o = (int64_t)e * n3;
    for (int p = 0; p < n3; ++p) v[p] = mg->ws[(int)m->mult[o + p]] * r[o + p];
    /* u = (Sz x Sy x Sx)^T v, one direction at a time */
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sx[q * n + i] * v[q + n * (j + n * k)];
          u[i + n * (j + n * k)] = s;
        }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sy[q * n + j] * u[i + n * (q + n * k)];
          v[i + n * (j + n * k)] = s;
        }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sz[q * n + k] * v[i + n * (j + n * q)];
          u[i + n * (j + n * k)] = s / (mg->kbar[e] * (lx[i] + ly[j] + lz[k]) + m->helm_h);
        }
    /* back: v = (Sz x Sy x Sx) u */
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sz[k * n + q] * u[i + n * (j + n * q)];
          v[i + n * (j + n * k)] = s;
        }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sy[j * n + q] * v[i + n * (q + n * k)];
          u[i + n * (j + n * k)] = s;
        }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += Sx[i * n + q] * u[q + n * (j + n * k)];
          zL[o + i + n * (j + n * k)] = mg->ws[(int)m->mult[o + i + n * (j + n * k)]] * s;
        }
  }
}

/* restriction to the coarse lattice: rc = P^T r (r continuous, c-weighted
 * over the local copies) */
void orc_mg_restrict(const orc_mesh *m, const orc_mg *mg, const double *r, double *rc) {
  int n = m->n, n3 = m->n3, ne = mg->ne, nu = mg->lv[0].nu;
  double J[64];
  lin_basis(m, J);
  memset(rc, 0, sizeof(double) * nu * nu * nu);
  for (int e = 0; e < m->E; ++e) {
    int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
    for (int b = 0; b < 8; ++b) {
      int I = ex + (b & 1), Jn = ey + ((b >> 1) & 1), Kn = ez + (b >> 2);
      if (I < 1 || Jn < 1 || Kn < 1 || I > nu || Jn > nu || Kn > nu) continue;
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            int64_t q = (int64_t)e * n3 + i + n * (j + n * k);
            s += J[2 * i + (b & 1)] * J[2 * j + ((b >> 1) & 1)] * J[2 * k + (b >> 2)] * m->c[q] * r[q];
          }
      rc[lat_idx(nu, I, Jn, Kn)] += s;
    }
  }
}

/* z += P zc (trilinear interpolation of the coarse lattice values) */
void orc_mg_prolong_add(const orc_mesh *m, const orc_mg *mg, const double *zc, double *z) {
  int n = m->n, n3 = m->n3, ne = mg->ne, nu = mg->lv[0].nu;
  double J[64];
  lin_basis(m, J);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < m->E; ++e) {
    int ex = e % ne, ey = (e / ne) % ne, ez = e / (ne * ne);
    double cv[8];
    for (int b = 0; b < 8; ++b) {
      int I = ex + (b & 1), Jn = ey + ((b >> 1) & 1), Kn = ez + (b >> 2);
      cv[b] = (I < 1 || Jn < 1 || Kn < 1 || I > nu || Jn > nu || Kn > nu)
                  ? 0.0 : zc[lat_idx(nu, I, Jn, Kn)];
    }
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int b = 0; b < 8; ++b)
            s += J[2 * i + (b & 1)] * J[2 * j + ((b >> 1) & 1)] * J[2 * k + (b >> 2)] * cv[b];
          z[(int64_t)e * n3 + i + n * (j + n * k)] += s;
        }
  }
}

/* z = M QQ^T(ws FDM(ws r)) + P V(P^T r) */
void orc_mg_apply(const orc_mesh *m, const orc_mg *mg, const double *r, double *z) {
  int nu = mg->lv[0].nu, nn = nu * nu * nu;
  double *rc = (double *)malloc(sizeof(double) * nn);
  double *zc = (double *)malloc(sizeof(double) * nn);
  orc_mg_schwarz_local(m, mg, r, z);
  orc_gs(m, z);
  orc_mask(m, z);
  orc_mg_restrict(m, mg, r, rc);
  vcycle(mg, 0, rc, zc);
  orc_mg_prolong_add(m, mg, zc, z);
  free(rc);
  free(zc);
}

/* accessors for the pins: levels, their stencils as dense matrices, the
 * coarse correction alone, the per-element 1-D eigenpairs */
int orc_mg_nlev(const orc_mg *mg) { return mg->nlev; }
int orc_mg_level_nu(const orc_mg *mg, int l) { return mg->lv[l].nu; }
double orc_mg_level_omega(const orc_mg *mg, int l) { return mg->lv[l].omega; }
void orc_mg_level_dense(const orc_mg *mg, int l, double *A) {
  const orc_lvl *L = &mg->lv[l];
  int nu = L->nu, nn = nu * nu * nu;
  memset(A, 0, sizeof(double) * (size_t)nn * nn);
  for (int K = 1; K <= nu; ++K)
    for (int J = 1; J <= nu; ++J)
      for (int I = 1; I <= nu; ++I) {
        int r = lat_idx(nu, I, J, K);
        for (int t = 0; t < 27; ++t) {
          int i2 = I + t % 3 - 1, j2 = J + (t / 3) % 3 - 1, k2 = K + t / 9 - 1;
          if (i2 < 1 || j2 < 1 || k2 < 1 || i2 > nu || j2 > nu || k2 > nu) continue;
          A[(size_t)r * nn + lat_idx(nu, i2, j2, k2)] = L->st[27 * (int64_t)r + t];
        }
      }
}
void orc_mg_vcycle(const orc_mg *mg, const double *b, double *x) { vcycle(mg, 0, b, x); }
void orc_mg_eig(const orc_mg *mg, int e, int d, double *S, double *lam) {
  int n = mg->n;
  memcpy(S, mg->S + ((size_t)e * 3 + d) * n * n, sizeof(double) * n * n);
  memcpy(lam, mg->lam + ((size_t)e * 3 + d) * n, sizeof(double) * n);
}
