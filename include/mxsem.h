/*
 * mxsem: matrix-free spectral-element Poisson/Helmholtz (P)CG on one
 * MI355X (gfx950), in FP64, in the paper's mixed FP32/FP64 recipe, inside
 * FP64 iterative refinement, batched over many uneven problems, and with a
 * learned flexible-CG preconditioner.
 *
 * Paper: Y. Chen et al., "Enabling mixed-precision in spectral element
 * codes" (arXiv 2503.02134).  The calls follow the paper's statement of the
 * problem: set up a mesh of E hexahedral elements of order N (Sec. 4,
 * Nekbone solves a Poisson problem on high-order elements; Sec. 5, Neko on
 * hexahedra), apply the matrix-free operator A (Sec. 4.1, CG-loop profiling
 * table, its "ax" row), gather-scatter / direct stiffness summation QQ^T
 * (Sec. 4.2.1), the weighted dot glsc3 (same table, its glsc3 rows), the
 * Jacobi preconditioner 1/diag(A) (Sec. 5.2) and the (P)CG solve with a
 * stopping tolerance (Sec. 6).  The mixed modes keep the gather-scatter sums
 * and the dot products in FP64 while the loop body runs in FP32 (Sec. 4.2.1
 * conclusion, Sec. 5.2, Sec. 6.1.1).
 *
 * Conventions for every call:
 *  - A local vector holds E*(N+1)^3 entries, entry ((e*n+k)*n+j)*n+i for
 *    node (i,j,k) of element e, n = N+1 (i fastest).
 *  - "device" pointers are HIP device memory owned by the caller (for
 *    example torch tensors); they must stay valid until the work queued on
 *    the context stream has finished.  FP64 vectors must be 8-byte aligned,
 *    FP32 vectors 4-byte aligned; 256-byte alignment is best.
 *  - "host" pointers are read or written only during the call.
 *  - The library allocates no device memory.  Everything it keeps on the
 *    device for a mesh, a network, a batch or an autotuning run (operator
 *    data, gather-scatter plan, solver work vectors, launch tables, partial
 *    sums) lives in a workspace the caller allocates (for example a torch
 *    uint8 tensor) and passes to the create call; its size comes from the
 *    matching *_workspace_bytes call, it must be 256-byte aligned and must
 *    outlive the handle.  A workspace smaller than reported is refused with
 *    MXSEM_EINVAL.  Handles own host metadata only; destroy frees that and
 *    never frees caller memory.
 *  - Every call returns 0 (MXSEM_OK) or a negative status; no C++ exception
 *    crosses this boundary and nothing calls exit.  mxsem_last_error()
 *    returns a message for the most recent failure on the calling thread.
 *  - A context (and everything created from it) must be used by one host
 *    thread at a time.
 *  - Calls marked "async" only enqueue work on the context stream.
 */
#ifndef MXSEM_H
#define MXSEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MXSEM_OK 0
#define MXSEM_EINVAL (-1)     /* bad argument: null pointer, size, alignment */
#define MXSEM_ENOTSUP (-2)    /* unsupported order, view or combination      */
#define MXSEM_EHIP (-3)       /* HIP runtime failure (message in last_error) */
#define MXSEM_EBREAKDOWN (-4) /* (p,Ap) <= 0 or non-finite, no fallback left */
#define MXSEM_EINTERNAL (-5)
#define MXSEM_ENOMEM (-6)     /* device or host allocation failed            */
#define MXSEM_EMESH (-7)      /* mesh rejected: |J| <= 0, inconsistent mask,
                                 shared or masked element-interior node      */

/* ---- precisions of vectors and operator data --------------------------- */
typedef enum {
  MXSEM_F64 = 0,       /* FP64 vectors, FP64 geometric factors            */
  MXSEM_F32 = 1,       /* FP32 vectors, FP32 geometric factors            */
  MXSEM_BF16G_F32 = 2  /* FP32 vectors, BF16 geometric factors (and h*B),
                          FP32 accumulation                                */
} mxsem_prec;

/* ---- preconditioners ---------------------------------------------------- */
typedef enum {
  MXSEM_PC_IDENTITY = 0, /* z = r (Sec. 5, identity-preconditioned CG)      */
  MXSEM_PC_JACOBI = 1,   /* z = dinv * r, dinv = 1/diag(A) built in FP64 (Sec. 5.2) */
  MXSEM_PC_LEARNED = 2,  /* z = M QQ^T(c*(dinv*r + s_e NN(r))), needs an
                            attached network and method FCG                */
  MXSEM_PC_MG = 3        /* two-level Schwarz / multigrid (the solveM step of
                            Sec. 4.1's CG-loop table; Sec. 4.2 on its Schwarz
                            weights): z = M QQ^T(ws FDM_e(ws r)) + P V(P^T r),
                            ws = sqrt(1/m) taken in FP64, FDM_e the fast-
                            diagonalisation solve on element e extended by
                            one GLL interval into its neighbours, P trilinear
                            interpolation from the element-vertex lattice, V
                            one geometric V-cycle (damped Jacobi, Galerkin
                            stencils, dense coarsest solve) in FP64.  Needs a
                            mesh built with MXSEM_VIEW_MG; solves run it in
                            flexible CG (one extra dot), single meshes only */
} mxsem_pc;

/* ---- solve modes -------------------------------------------------------- */
typedef enum {
  MXSEM_MODE_FP64 = 0,           /* everything FP64                          */
  MXSEM_MODE_MIXED = 1,          /* the paper's recipe: FP32 loop body and
                                    preconditioner, FP64 gather-scatter sums
                                    and dot products, no refinement        */
  MXSEM_MODE_MIXED_IR = 2,       /* MIXED inner PCG inside FP64 iterative
                                    refinement with FP64 residuals           */
  MXSEM_MODE_MIXED_IR_BF16G = 3, /* as MIXED_IR, inner operator reads BF16 G */
  MXSEM_MODE_FP32_ALL = 4,       /* ablation: FP32 gather-scatter sums and FP32
                                    dot accumulation (the configuration the
                                    paper finds to stagnate)                 */
  MXSEM_MODE_MIXED_IR_BF16P = 5  /* ablation of BF16 operator inputs: as
                                    MIXED_IR, with the inner PCG's direction
                                    p rounded to BF16 (nearest even) each
                                    step, so the operator, sigma and the x
                                    update all see the BF16 value; PCG only */
} mxsem_mode;

typedef enum { MXSEM_METHOD_PCG = 0, MXSEM_METHOD_FCG = 1 } mxsem_method;

/* ---- accumulation of the dot products of the FP32 loop (Sec. 5.2.1) ------ */
typedef enum {
  MXSEM_DOT_DEFAULT = 0, /* the mode's own: FP32 in MXSEM_MODE_FP32_ALL, else FP64 */
  MXSEM_DOT_F64 = 1,     /* FP32 inputs, products and sums in FP64           */
  MXSEM_DOT_F32 = 2,     /* products and sums in FP32                        */
  MXSEM_DOT_DOT2 = 3     /* compensated FP32: the Dot2 algorithm of Ogita,
                            Rump and Oishi (2005) within each thread, partial
                            results (sum, correction) combined by TwoSum
                            across threads and workgroups; the result is
                            the FP32 rounding of sum + correction          */
} mxsem_dot_acc;

/* ---- summation order of the gather-scatter in the solve ------------------ */
typedef enum {
  MXSEM_GS_ORDER_ONE = 0,      /* one sum per node (ascending local index),
                                  written to every copy: the copies stay equal
                                  (what an allreduce-based exchange gives)    */
  MXSEM_GS_ORDER_PAIRWISE = 1  /* the order of a pairwise exchange between
                                  ranks (Sec. 4.2.1), on one GPU: elements are
                                  assigned to ranks (mxsem_mesh_set_ranks; by
                                  default every element is a rank of its own);
                                  each rank sums its own copies of a node in
                                  ascending local index, then adds the other
                                  ranks' partial sums in ascending rank order,
                                  and its copies receive that value.  FP32
                                  vectors, at most 16 copies per node        */
} mxsem_gs_order;

/* termination reasons */
#define MXSEM_CONVERGED 1
#define MXSEM_MAX_ITER 2
#define MXSEM_STAGNATED 3
#define MXSEM_BREAKDOWN 4

/* apply / gather-scatter flags */
#define MXSEM_LOCAL_ONLY 1u /* apply: w = A_L u only (no QQ^T, no mask)      */
#define MXSEM_MASK 2u       /* gather_scatter: also zero Dirichlet entries   */
#define MXSEM_GS_PAIRWISE 4u /* gather_scatter: MXSEM_GS_ORDER_PAIRWISE sums  */

/* mesh views (bitmask): which operator copies to keep on the device */
#define MXSEM_VIEW_F64 1u
#define MXSEM_VIEW_F32 2u
#define MXSEM_VIEW_BF16 4u
#define MXSEM_VIEW_MG 8u   /* also build the multigrid preconditioner: needs a
                              box of ne^3 elements (ne >= 2) in lexicographic
                              order, global ids on the lattice of GLL nodes
                              (id = gx + G1 (gy + G1 gz), G1 = ne N + 1) and
                              Dirichlet conditions on the whole box boundary
                              (else MXSEM_ENOTSUP); about 30 B per local entry */

typedef struct mxsem_ctx mxsem_ctx;
typedef struct mxsem_mesh mxsem_mesh;
typedef struct mxsem_batch mxsem_batch;
typedef struct mxsem_nn mxsem_nn;

/* ---- context ------------------------------------------------------------- */
/* One device and one stream.  hip_stream: a hipStream_t (for example
 * torch.cuda.current_stream().cuda_stream) or NULL for the null stream.
 * Makes hip_device current on the calling thread. */
int mxsem_ctx_create(int hip_device, void *hip_stream, mxsem_ctx **out);
int mxsem_ctx_destroy(mxsem_ctx *ctx);
/* Replace the stream used by later calls (same device). */
int mxsem_ctx_set_stream(mxsem_ctx *ctx, void *hip_stream);

/* ---- reference element --------------------------------------------------- */
/* Gauss-Lobatto-Legendre nodes (ascending, -1..1) and weights for order N,
 * 1 <= N <= 15; host arrays of N+1 entries.  Input generators use the nodes
 * to place mesh points. */
int mxsem_gll(int N, double *xi_host, double *w_host);

/* ---- mesh ---------------------------------------------------------------- */
typedef struct {
  int E;                 /* number of hexahedra, >= 1                       */
  int N;                 /* polynomial order, 1..15                         */
  const double *xyz;     /* host [E][3][n^3] node coordinates               */
  const int64_t *glo;    /* host [E][n^3] global node ids (>= 0)            */
  const uint8_t *bnd;    /* host [E][n^3], nonzero on Dirichlet nodes       */
  const double *kcoef;   /* host [E][n^3] diffusion coefficient, or NULL = 1 */
  double helm_h;         /* Helmholtz coefficient h >= 0 (0: Poisson)       */
  unsigned views;        /* MXSEM_VIEW_* bitmask; F64 is always kept.  The
                            views fix which solve precisions the mesh can
                            run: F32 or BF16 adds the FP32 work vectors     */
} mxsem_mesh_desc;

/* Bytes of device workspace mxsem_mesh_create needs for this description:
 * G, B, dinv in FP64 and in the views' precisions, the gather-scatter plan
 * (so the host sort of glo runs here too), the copy counts, the solver work
 * vectors and partial sums of every precision the views allow, and the
 * launch tables of the mesh's own solves.  About 200 bytes per local entry
 * with all views.  Same errors as mxsem_mesh_create's checks of desc. */
int mxsem_mesh_workspace_bytes(const mxsem_mesh_desc *desc, size_t *bytes);

/* Builds, in FP64 on the device, the geometric factors G (6 per node,
 * times k), the mass B, the multiplicity weight c = 1/m, the gather-scatter
 * plan (host sort of glo), the Dirichlet list and the Jacobi inverse
 * diagonal dinv (0 on Dirichlet nodes); then the FP32 / BF16 copies asked
 * for in views.  workspace: device memory of at least ws_bytes >=
 * mxsem_mesh_workspace_bytes(desc) bytes, 256-byte aligned, owned by the
 * caller and used by the mesh until it is destroyed (MXSEM_EINVAL when null,
 * misaligned or too small).  Synchronous.  Rejects (MXSEM_EMESH) a
 * non-positive Jacobian, copies of one node that disagree on bnd, and
 * element-interior nodes that are shared or Dirichlet. */
int mxsem_mesh_create(mxsem_ctx *ctx, const mxsem_mesh_desc *desc, void *workspace,
                      size_t ws_bytes, mxsem_mesh **out);
int mxsem_mesh_destroy(mxsem_mesh *mesh);

/* Sizes: local entries, gather-scatter groups (shared nodes and free
 * element-face nodes), Dirichlet entries, minimum |J|. */
int mxsem_mesh_info(const mxsem_mesh *mesh, int64_t *nloc, int64_t *ngroups,
                    int64_t *nmasked, double *min_detj);

/* Copy operator data to host arrays (FP64): what = 0 G [E][6][n^3],
 * 1 B [E][n^3], 2 c [E][n^3], 3 dinv [E][n^3], 4 mask [E][n^3] (0/1),
 * 5 D [n][n].  Synchronous. */
int mxsem_mesh_get(const mxsem_mesh *mesh, int what, double *out_host);

/* ---- operator pieces (async) ----------------------------------------------- */
/* w = M QQ^T A_L u (assembled apply, Dirichlet rows zeroed), or with
 * MXSEM_LOCAL_ONLY w = A_L u.  A_L u = sum_ab D_a^T diag(G_ab) D_b u + h B u
 * (tensor-product local_grad3, geometric-factor multiply, local_grad3_t).
 * io selects the vector type and the G copy (the view must exist).  With
 * QQ^T the shared-node sums are accumulated in FP64 for every io. */
int mxsem_apply(mxsem_mesh *mesh, mxsem_prec io, const void *u, void *w, unsigned flags);

/* In place v <- QQ^T v: each shared node's copies are summed in ascending
 * local-index order in acc precision (MXSEM_F64 or MXSEM_F32), rounded once
 * to io and written to every copy.  MXSEM_MASK also zeroes Dirichlet
 * entries.  io: MXSEM_F64 or MXSEM_F32.  MXSEM_GS_PAIRWISE (io MXSEM_F32,
 * at most 16 copies per node, else MXSEM_ENOTSUP): a copy in rank R of a
 * node held by ranks R_1 < R_2 < ... receives S_R + S_{R_a} + S_{R_b} + ...
 * (left to right, the other ranks ascending), S_X the sum of rank X's
 * copies in ascending local index; sums in acc, rounded once to FP32. */
int mxsem_gather_scatter(mxsem_mesh *mesh, mxsem_prec io, mxsem_prec acc, void *v,
                         unsigned flags);

/* *out_dev (device FP64 scalar) = sum_i a_i c_i b_i, c = 1/multiplicity,
 * products and accumulation in FP64 (glsc3).  io: MXSEM_F64 or MXSEM_F32. */
int mxsem_dot(mxsem_mesh *mesh, mxsem_prec io, const void *a, const void *b,
              double *out_dev);

/* As mxsem_dot with the accumulation acc (mxsem_dot_acc; MXSEM_DOT_DEFAULT
 * is FP64).  MXSEM_DOT_F32 and MXSEM_DOT_DOT2 take io MXSEM_F32 and write an
 * FP32 value (widened to FP64) to *out_dev; each term is (a_i c_i) b_i with
 * a_i c_i rounded to FP32 (exact when the multiplicity is a power of two). */
int mxsem_dot_ex(mxsem_mesh *mesh, mxsem_prec io, int acc, const void *a, const void *b,
                 double *out_dev);

/* z = M^-1 r for pc = identity or Jacobi (io MXSEM_F64 / MXSEM_F32), or the
 * learned map (MXSEM_F32, network attached). */
int mxsem_precond(mxsem_mesh *mesh, mxsem_pc pc, mxsem_prec io, const void *r, void *z);

/* Ranks of the pairwise gather-scatter order (Sec. 4.2.1 compares the
 * exchange modes across rank counts; one GPU emulates their summation
 * order): rank_host is a host array [E] of ranks >= 0, or NULL for every
 * element a rank of its own (the default).  Used by MXSEM_GS_PAIRWISE and
 * by solves with gs_order MXSEM_GS_ORDER_PAIRWISE.  The ranks are kept in
 * the mesh's workspace; synchronises the context stream. */
int mxsem_mesh_set_ranks(mxsem_mesh *mesh, const int32_t *rank_host);

/* b = M QQ^T (B f) for a nodal source f (device FP64 vectors). */
int mxsem_mass_rhs(mxsem_mesh *mesh, const double *f, double *b);

/* ---- solve ----------------------------------------------------------------- */
typedef struct {
  int method;         /* mxsem_method                                      */
  int pc;             /* mxsem_pc                                          */
  int mode;           /* mxsem_mode                                        */
  double tol;         /* stop when ||r||_c <= tol ||b||_c                  */
  int max_iter;       /* cap on (inner) iterations in total               */
  double inner_tol;   /* IR modes: relative tolerance of each inner solve  */
  int max_outer;      /* IR modes: cap on refinement steps                 */
  int graph_chunk;    /* iterations per captured HIP graph (>= 1)          */
  int x0_given;       /* 1: start from x (FP64 modes); 0: x = 0            */
  double *history;    /* nullable device FP64 [max_iter+1]: relative
                         recursive residual per iteration                   */
  int dot;            /* mxsem_dot_acc of the loop's dots: PCG, FP32 vectors
                         with FP32 G (MIXED, MIXED_IR, FP32_ALL); otherwise
                         MXSEM_DOT_DEFAULT (or MXSEM_DOT_F64)               */
  int gs_order;       /* mxsem_gs_order of the loop's gather-scatter: PCG in
                         MIXED or FP32_ALL; otherwise MXSEM_GS_ORDER_ONE    */
} mxsem_solve_opts;

typedef struct {
  int iterations;     /* inner (P)CG iterations in total                   */
  int outer;          /* refinement steps (IR modes)                       */
  int reason;         /* MXSEM_CONVERGED / MAX_ITER / STAGNATED / BREAKDOWN */
  int fallback_used;  /* learned PC replaced by Jacobi (steps), or IR fell
                         back to FP64 PCG (1)                              */
  double rel_res;     /* true ||b - A x||_c / ||b||_c in FP64 at exit      */
  double rel_res_recursive; /* last recursive residual of the inner loop   */
  double ms;          /* wall time of the solve on the stream (hipEvents)  */
  double ax_ms;       /* mean duration of the operator kernel of the first
                         iteration of each graph launch (hipEvents around
                         that kernel node), inner loop only               */
  int ax_samples;     /* number of such timed launches                     */
  int pad_;
} mxsem_solve_stats;

/* Solve A x = b.  b, x: device FP64 local vectors (b continuous and masked,
 * e.g. from mxsem_mass_rhs).  Stops at tol, max_iter, stagnation (the best
 * residual has not improved by 10% in 500 iterations) or breakdown.
 * Synchronous on the context stream; fills st. */
int mxsem_solve(mxsem_mesh *mesh, const mxsem_solve_opts *opts, const double *b, double *x,
                mxsem_solve_stats *st);
void mxsem_solve_opts_default(mxsem_solve_opts *opts);

/* ---- batch of independent problems --------------------------------------- */
typedef struct {
  int epb[16];        /* elements per workgroup of the operator kernel per N
                         (0 = library default)                              */
  int cols[16];       /* thread mapping of the operator kernel per N: 0 =
                         library default, 1 = one (i,j) column per thread,
                         2 = two columns per thread (N = 5 and 9 with FP32
                         vectors; FP64 vectors take one column)             */
} mxsem_tuning;

/* Bytes of device workspace mxsem_batch_create needs: the launch tables of
 * the batch's plans (every problem's tiles), overlapped by the autotuning
 * scratch when a tune cache is given. */
int mxsem_batch_workspace_bytes(mxsem_ctx *ctx, int P, mxsem_mesh *const *meshes,
                                const char *tune_cache, size_t *bytes);
/* P meshes on one context solved together: every captured graph chunk
 * launches each stage once per order class over a tile table that spans
 * all problems; problems that have converged become no-ops.  tune_cache:
 * JSON file path for autotuned tiles (nullable = defaults, or the
 * MXSEM_TUNE_CACHE environment variable); a missing entry is tuned in the
 * workspace and added to the file.  workspace: caller device memory of at
 * least mxsem_batch_workspace_bytes bytes, 256-byte aligned, kept until the
 * batch is destroyed; the work vectors are the meshes' own. */
int mxsem_batch_create(mxsem_ctx *ctx, int P, mxsem_mesh *const *meshes,
                       const char *tune_cache, void *workspace, size_t ws_bytes,
                       mxsem_batch **out);
int mxsem_batch_destroy(mxsem_batch *batch);
/* b[p], x[p]: device FP64 vectors per problem; st: host array of P. */
int mxsem_batch_solve(mxsem_batch *batch, const mxsem_solve_opts *opts,
                      const double *const *b, double *const *x, mxsem_solve_stats *st);
/* Bytes of device workspace for mxsem_autotune at (N, E, prec): synthetic
 * u, w, G and D of that size. */
int mxsem_autotune_workspace_bytes(int N, int E, mxsem_prec prec, size_t *bytes);
/* Time the candidate tiles of the operator kernel for one (N, E, prec) on
 * the context's device, on synthetic data in the caller's workspace, and
 * return the fastest (epb[N], cols[N]): every tile size, with both thread
 * mappings where two exist (N = 5, 9 with FP32 vectors).  Synchronous. */
int mxsem_autotune(mxsem_ctx *ctx, int N, int E, mxsem_prec prec, void *workspace,
                   size_t ws_bytes, mxsem_tuning *out);
/* Tiles and thread mapping the library will use for a mesh (after any
 * tuning); EINVAL for a tile that does not fit its mapping's workgroup. */
int mxsem_mesh_set_tuning(mxsem_mesh *mesh, const mxsem_tuning *t);

/* ---- learned preconditioner ------------------------------------------------ */
typedef struct {
  int cin;            /* input channels, must be 2: [r, dinv r] / s_e      */
  int ch;             /* hidden channels (32)                              */
  int max_samples;    /* largest nsamp of mxsem_nn_loss_grad (>= 1)        */
} mxsem_nn_desc;

/* Network z_L = dinv r + s_e * conv2(relu(conv1([r, dinv r]/s_e))), 3x3x3
 * kernels with zero padding at element borders, no bias, s_e = ||dinv r||
 * per element; weights W1 [ch][cin][27], W2 [ch][27] (offset o = (di+1) +
 * 3(dj+1) + 9(dk+1)); BF16 inputs and weights, FP32 accumulation. */
/* Bytes of device workspace mxsem_nn_create needs on this mesh. */
int mxsem_nn_workspace_bytes(const mxsem_mesh *mesh, const mxsem_nn_desc *desc, size_t *bytes);
/* workspace: caller device memory of at least mxsem_nn_workspace_bytes
 * bytes, 256-byte aligned, kept until the network is destroyed. */
int mxsem_nn_create(mxsem_mesh *mesh, const mxsem_nn_desc *desc, void *workspace,
                    size_t ws_bytes, mxsem_nn **out);
int mxsem_nn_destroy(mxsem_nn *nn);
int mxsem_nn_set_params(mxsem_nn *nn, const float *W1_host, const float *W2_host);
int mxsem_nn_get_params(mxsem_nn *nn, float *W1_host, float *W2_host);
/* z = M QQ^T (c * zL(r)) for a device FP32 residual r. Async. */
int mxsem_nn_forward(mxsem_nn *nn, const float *r, float *z);
/* Mean over nsamp pairs of ||z(r_s) - e_s||_A^2 / ||e_s||_A^2 and its
 * gradient (device FP32 grad [ch*cin*27 + ch*27], W1 part first); r, e:
 * device FP32 [nsamp][nloc], 1 <= nsamp <= desc.max_samples (else
 * MXSEM_EINVAL); loss_dev: device FP64 scalar. Async. */
int mxsem_nn_loss_grad(mxsem_nn *nn, const float *r, const float *e, int nsamp,
                       double *loss_dev, float *grad_dev);
typedef struct {
  double lr, beta1, beta2, eps;
  int step;           /* 1-based step count                                */
} mxsem_adam;
/* Adam on the FP32 master weights with the gradient last computed by
 * mxsem_nn_loss_grad. Async. */
int mxsem_nn_adam_step(mxsem_nn *nn, const mxsem_adam *opt);
/* Attach (or with nn = NULL detach) a network as the mesh's learned
 * preconditioner (solves with pc = MXSEM_PC_LEARNED use it). */
int mxsem_mesh_attach_nn(mxsem_mesh *mesh, mxsem_nn *nn);
/* One training pair from an FP64 iterate: r = (b - A x)/||b - A x||_c and
 * e = (xstar - x)/||b - A x||_c as device FP32 vectors (the scaling keeps
 * FP32 in range; the loss is scale-free).  b, x, xstar: device FP64. Async. */
int mxsem_nn_make_pair(mxsem_mesh *mesh, const double *b, const double *x, const double *xstar,
                       float *r_out, float *e_out);

/* ---- bandwidth reference ---------------------------------------------------- */
/* dst = src for `bytes` bytes of device memory (a multiple of 16, both
 * pointers 16-byte aligned, no overlap): a one-pass streaming copy with
 * non-temporal loads and stores, the measured HBM ceiling that the operator
 * kernel's bandwidth is set beside.  Async on the context stream. */
int mxsem_stream_copy(mxsem_ctx *ctx, const void *src, void *dst, size_t bytes);
/* The same reference at a kernel's own read:write split: with n =
 * write_bytes / 16 and k = read_bytes / write_bytes (1, 2, 4 or 8), dst
 * holds n 16-byte words of four FP32 and dst[i] = src[i] + src[n + i] + ...
 * + src[(k-1) n + i], summed left to right in FP32.  Device pointers,
 * 16-byte aligned, write_bytes a positive multiple of 16, read_bytes a
 * multiple of it, no overlap (MXSEM_EINVAL otherwise).  k = 4 is the
 * operator kernel's split (32 bytes read, 8 written per local dof).  Async
 * on the context stream. */
int mxsem_stream_mix(mxsem_ctx *ctx, const void *src, size_t read_bytes, void *dst,
                     size_t write_bytes);

/* ---- diagnostics ------------------------------------------------------------ */
const char *mxsem_status_str(int status);
const char *mxsem_last_error(void);
int mxsem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MXSEM_H */
