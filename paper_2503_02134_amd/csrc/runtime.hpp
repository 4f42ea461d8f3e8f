// Host-side objects of the mxsem library (context, mesh, solver buffers).
#pragma once

#include <vector>

#include "common.hpp"

struct mxsem_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream (may be null)
  hipStream_t capture = nullptr;  // private stream used only for graph capture
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int* pinned_flags = nullptr;    // host-pinned poll buffer
  int live = 0;                   // meshes / batches created from this context
};

namespace mx {

// launchers (defined in the .hip files)
// cols: thread mapping (0 default, 1 one column per thread, 2 two columns
// where the kernel exists: N = 5, 9 with FP32 vectors)
hipError_t launch_ax_apply(int prec, int N, int E, int epb, const void* u, void* w, const void* G,
                           const void* hB, const void* D, hipStream_t s, int cols = 0);
// parity: -1 updates p in place; 0 / 1 the step's parity with two direction
// buffers (see ProbDev::p_alt)
hipError_t launch_ax_solver(int prec, int dm, int N, const Tile* tiles, int ntiles, const ProbDev* probs,
                            int epb, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr, int parity = -1, int cols = 0);
int max_epb(int N);
int ax_wave_elements(int N);
// largest tile of the two-column mapping (0: N has none)
int max_epb2(int N);
// pairwise: the summation order of a pairwise exchange between the mesh's
// ranks (FP32 vectors; see gs_kernel)
hipError_t launch_gs_apply(int prec_io, int prec_acc, void* v, const GsPlan& plan, bool mask,
                           hipStream_t s, bool pairwise = false);
// sigma_probs > 0: the launch also finishes sigma and alpha of problems
// 0..sigma_probs-1 (alpha = rho / sigma, breakdown test) in workgroups of its own.
// ztiles (with on_z): vector-pass tiles of workgroups that set z = dinv r
// where the step's learned z was rejected (fb_pending); the gather-scatter
// tiles of such a problem do nothing.
hipError_t launch_gs_solver(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                            hipStream_t s, bool on_z = false, int sigma_probs = 0,
                            const Tile* ztiles = nullptr, int nz = 0, bool pairwise = false);
hipError_t launch_zpc(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs, int pc,
                      hipStream_t s);
hipError_t launch_fcg_dots(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                           hipStream_t s);
// dots (optional, single problem): the learned forward's partials of the
// learned and the Jacobi candidate's dots (NnDots layout, ndots per dot):
// the step takes the learned z unless it is rejected, then the Jacobi z
// (fb_pending tells the following gather-scatter launch to form it)
hipError_t launch_fin_beta(const ProbDev* probs, int nprob, int init, hipStream_t s,
                           const double* dots = nullptr, int ndots = 0, int dstride = 0);
// The flexible-CG dots of the step, from zc = c z_L before assembly: r
// and w = A p are continuous and zero on Dirichlet nodes, and z = M QQ^T zc
// with the weights c summing to 1 over a node's copies, so
//   (r, z)_c = sum_i r_i zc_i,   (z, w)_c = sum_i w_i zc_i
// over all local entries (equal up to rounding to the dots of the assembled
// z).  The same pass gives the dots of the Jacobi candidate z_J = dinv r
// (continuous already), sum_i r_i c_i z_J,i and sum_i w_i c_i z_J,i, and
// (r,r)_c.  Each workgroup of the forward writes its five partials to
// dots[k * dstride + blockIdx.x], k = 0..4 in that order; dots == nullptr
// skips them.  With x (and p), the forward first applies the step's vector
// update to each element it reads, r -= alpha w and x += alpha p (alpha from
// the state), writes r and x back, and works on the updated r.
struct NnDots {
  const float* w;
  double* dots;
  int dstride;
  float* x;
  const float* p;
};
// nparts (optional): workgroups of the launch, i.e. partials per dot
hipError_t launch_nn_fwd(int N, const float* r, const float* dinv, const uint8_t* mult,
                         const float* W1, const float* W2, float* zc, int E, hipStream_t s,
                         const State* st, const void* packed, NnDots dd, int* nparts);
// dm: DotMode of the dots (FP32 vectors; FP64 vectors take DOT_F64)
// parity: -1 x += alpha p every step; 0 defers x (pending); 1 adds both
// steps' alpha p.  asm_w: box-lattice problems (box_ne > 0) form QQ^T w and
// the mask in this pass (their gather-scatter of w is left out of the step);
// vprec VP_F64 or VP_F32 (FP64 sums).
hipError_t launch_update(int vprec, int pc, const Tile* tiles, int ntiles, const ProbDev* probs,
                         hipStream_t s, int dm = DOT_F64, int parity = -1, bool asm_w = false);
// x += alpha_prev p for the problems whose last step left x pending
hipError_t launch_x_pending(int vprec, const Tile* tiles, int ntiles, const ProbDev* probs,
                            hipStream_t s);
hipError_t launch_init(int vprec, int pc, const Tile* tiles, int ntiles, const ProbDev* probs,
                       const double* x0, hipStream_t s, int dm = DOT_F64);
hipError_t launch_fin_rho(const ProbDev* probs, int nprob, int mode, hipStream_t s);
hipError_t launch_dot(int prec, const void* a, const void* b, const uint8_t* mult, int64_t n,
                      double* part, double* out, hipStream_t s, int dm = DOT_F64);
hipError_t launch_precond(int prec, int pc, const void* r, void* z, const void* dinv, int64_t n,
                          hipStream_t s);
hipError_t launch_residual(const double* b, const double* w, double* r, const uint8_t* mult,
                           int64_t n, double* part, double* out, hipStream_t s);
hipError_t launch_axpy_cast(int vprec, double* x64, const void* xT, double sc, double keep,
                            int64_t n, hipStream_t s);
hipError_t launch_zero(double* x, int64_t n, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, hipStream_t s);
hipError_t launch_stream_mix(const void* src, void* dst, int64_t n16, int k, hipStream_t s);
hipError_t launch_mass(const double* B, const double* f, double* b, int64_t n, hipStream_t s);
hipError_t launch_cast_f32(float* d, const double* src, int64_t n, hipStream_t s);
hipError_t launch_cast_bf16(bf16_t* d, const double* src, int64_t n, hipStream_t s);
hipError_t launch_cast_g_split(int gprec, void* d, const double* G64, int E, int n3,
                               hipStream_t s);
hipError_t launch_geom(int E, int n, const double* xyz, const double* D, const double* wq,
                       const double* kcoef, double* G, double* B, double* detmin, int* nblocks,
                       hipStream_t s);
hipError_t launch_diag(int E, int n, const double* G, const double* B, double h, const double* D,
                       double* diag, hipStream_t s);
hipError_t launch_invert(double* d, int64_t n, hipStream_t s);
hipError_t launch_scale(double* d, const double* src, double h, int64_t n, hipStream_t s);

// host reference-element routines (library's own)
void gll_rule(int N, double* xi, double* w);
void deriv_matrix(int N, const double* xi, double* D);

// vector precision class of a solve
enum VPrec { VP_F64 = 0, VP_F32 = 1, VP_F32ACC = 3 };

// ---------------------------------------------------------------- caller workspaces
// The library allocates no device memory: every device array of a mesh, a
// network, a batch or an autotuning run is a block of a workspace the caller
// allocated (its size comes from the matching *_workspace_bytes call).
// Blocks start on 256-byte boundaries.
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Offsets of the blocks of a workspace, in the order they are taken.
struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t o = align256(total);
    total = o + (bytes ? bytes : 1);
    return o;
  }
};

// A workspace block handed out piece by piece (launch tables of a plan,
// rebuilt in place when the plan is rebuilt).
struct Region {
  char* base = nullptr;
  size_t size = 0, used = 0;
};
// *p = the next 256-aligned piece of `bytes`; MXSEM_EINTERNAL past the end
// (the workspace was sized for every plan the object can build).
int region_take(Region& r, void** p, size_t bytes);

// ---------------------------------------------------------------- multigrid
// Two-level Schwarz / multigrid preconditioner of a box mesh (mg.hip).
constexpr int MG_MAXLEV = 12;
constexpr int MG_COARSEST_MAX = 512;  // unknowns of the directly solved level
struct MgLevel {
  int nu = 0;              // interior lattice nodes per direction
  double omega = 0.0;      // Jacobi damping
  double* st = nullptr;    // [nu^3][27] stencil
  double *b = nullptr, *x = nullptr, *x2 = nullptr, *r = nullptr;  // [nu^3]
};
struct MgData {
  int ne = 0, nlev = 0, nc = 0;
  double *S64 = nullptr, *lam64 = nullptr;  // [E][3][n][n], [E][3][n]
  float *S32 = nullptr, *lam32 = nullptr;
  double* kbar = nullptr;                   // [E] mean coefficient
  double* ws64 = nullptr;                   // [256] sqrt(1/m) (FP64 square roots)
  float* ws32 = nullptr;                    // the same, rounded once to FP32
  double* J = nullptr;                      // [n][2] order-1 basis at the GLL nodes
  double* corner = nullptr;                 // [E][8] restricted residual per element vertex
  int* ecorner = nullptr;                   // [E][8] lattice index of each corner, -1 on the boundary
  double* K = nullptr;                      // [E][64] Galerkin element matrices (set-up)
  double* cinv = nullptr;                   // [nc][nc] inverse of the coarsest operator
  MgLevel lv[MG_MAXLEV];
};
// elements per direction of a box mesh of E elements (0 if E is no cube)
int mg_cube_root(int E);
// the levels' interior node counts per direction for ne elements per direction
int mg_levels(int ne, int* nu);
// blocks of the preconditioner in the mesh workspace (ws == nullptr: sizes only)
void mg_layout(mxsem_mesh* m, char* ws, Layout& L);
// the box structure of a mesh description: MXSEM_OK or MXSEM_ENOTSUP
int mg_check_box(const mxsem_mesh_desc* d);
// ne of a box-lattice mesh (see mg.hip), else 0
int box_lattice_ne(const mxsem_mesh_desc* d);
// builds the preconditioner's data (after the operator data exist)
int mg_setup(mxsem_mesh* m, const mxsem_mesh_desc* d, hipStream_t s);
// z = M^-1 r (vprec VP_F64 or FP32 vectors); st: the solve's state (the
// kernels return at once when it is done), or null.  pl: the solve's plan
// (single problem, z its work vector), or null; with a plan the coarse
// correction is left to mg_prolong_dots, which adds it while it sums the
// flexible-CG dots of the step
struct Plan;
int mg_apply(mxsem_mesh* m, int vprec, const void* r, void* z, hipStream_t s, const State* st,
             const Plan* pl = nullptr);
int mg_prolong_dots(const mxsem_mesh* m, const Plan* pl, hipStream_t s);

// Bytes of the launch tables of one plan over these problems (operator,
// gather-scatter and vector-pass tiles, problem views, states, norms).
size_t plan_table_bytes(mxsem_mesh* const* meshes, int P);

// Workspace bytes of an autotuning run at (N, E, prec).
size_t autotune_bytes(int N, int E, int prec);

// Device work vectors and partial-sum arrays of one problem in one vector
// precision (shared by every launch plan that contains the problem).
struct SolverBufs {
  int vprec = 0;
  void *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *w = nullptr, *p_alt = nullptr;
  double *part_ax = nullptr, *part_gs = nullptr, *part_u0 = nullptr, *part_u1 = nullptr,
         *part_u2 = nullptr;
  int nt_upd = 0, nt_gs = 0;
};

// Operator-kernel launch class: problems of one order N and one tile size.
struct AxClass {
  int N = 0, epb = 1, cols = 0;
  Tile* tiles = nullptr;
  int ntiles = 0;
};

// Launch plan of the (P)CG iteration for a set of problems in one vector
// precision: device problem views and states, tile tables spanning all
// problems, and the cached HIP graph of K iterations.
struct Plan {
  int vprec = 0, P = 0, device = 0;
  std::vector<mxsem_mesh*> meshes;
  std::vector<SolverBufs*> bufs;
  std::vector<int> epb_used;       // tile size per problem when built
  std::vector<int> cols_used;      // thread mapping per problem when built
  std::vector<ProbDev> hprob;      // host copies
  ProbDev* probs = nullptr;        // device [P]
  State* states = nullptr;         // device [P]
  State* hstate = nullptr;         // pinned host [P]
  double* dnorm = nullptr;         // device [P] per-problem scalars
  double* hnorm = nullptr;         // pinned host [P]
  std::vector<AxClass> ax;
  Tile* tiles_gs = nullptr;   // every problem (z in flexible CG, the pairwise order)
  int nt_gs = 0;
  Tile* tiles_gsw = nullptr;  // problems whose PCG step assembles w in the vector pass left out
  int nt_gsw = 0;
  Tile* tiles_upd = nullptr;
  int nt_upd = 0;
  hipGraphExec_t graph = nullptr;
  int graph_k = 0, graph_pc = -1, graph_gprec = -1, graph_method = -1;
  // dot accumulation (DotMode) and gather-scatter order of the captured
  // iteration, set per solve
  int dm = 0, pairwise = 0;
  int graph_dm = -1, graph_pairwise = -1;
  hipEvent_t evA = nullptr, evB = nullptr;
  double ax_ms_sum = 0.0;
  int ax_samples = 0;
  Region tables;  // where the launch tables live (a block of a caller workspace)
};

void plan_destroy(Plan* pl);

}  // namespace mx

struct mxsem_mesh {
  mxsem_ctx* ctx = nullptr;
  int E = 0, N = 0, n = 0, n3 = 0;
  int64_t nloc = 0;
  // box lattice with n = 8 or 16: elements per direction (the PCG step
  // forms QQ^T w in the vector pass), else 0
  int box_ne = 0;
  double helm_h = 0.0;
  unsigned views = 0;
  // device operator data
  double* D64 = nullptr;
  float* D32 = nullptr;
  double* G64 = nullptr;
  float* G32 = nullptr;       // split layout: [nloc] x 4 (rr rs rt ss), then [nloc] x 2 (st tt)
  mx::bf16_t* G16 = nullptr;  // same split layout in BF16
  double* B64 = nullptr;
  double* hB64 = nullptr;
  float* hB32 = nullptr;
  mx::bf16_t* hB16 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  uint8_t* mult = nullptr;
  int* gs_idx = nullptr;
  mx::GsPlan plan{};          // device index array + bucket table (+ element ranks)
  int* erank = nullptr;       // device [E] ranks of the pairwise order, or null
  // host copy, per bucket: the first (smallest) local index of each group
  // in bucket order (mask list: its entries); places solver tiles
  std::vector<std::vector<int32_t>> gs_first;
  int64_t ngroups = 0;        // groups of >= 2 copies
  int nmask_entries = 0;      // Dirichlet entries
  double min_det = 0.0;
  // scratch
  double* part = nullptr;    // [ceil(nloc / UPD_CHUNK) + 64]
  double* scal = nullptr;    // [8] device scalars
  double* tmpa = nullptr;    // FP64 [nloc] work vectors
  double* tmpb = nullptr;
  int epb[16] = {0};
  int cols[16] = {0};         // operator thread mapping per N (0 = default)
  // solver work vectors per vector precision (VP_F32ACC shares VP_F32's)
  mx::SolverBufs* bufs[4] = {nullptr, nullptr, nullptr, nullptr};
  mx::Plan* self_plan[4] = {nullptr, nullptr, nullptr, nullptr};
  mx::Region plan_tables[4];  // workspace blocks of the self plans' tables
  mxsem_nn* nn = nullptr;
  mx::MgData* mg = nullptr;   // multigrid preconditioner (MXSEM_VIEW_MG)
  char* ws = nullptr;         // the caller's workspace (never freed here)
  size_t ws_bytes = 0;
  bool counted = false;
};

namespace mx {
int default_epb(int N);
// the solver work vectors of vprec (MXSEM_ENOTSUP if the mesh's views
// leave that precision out)
int ensure_bufs(mxsem_mesh* m, int vprec, SolverBufs** out);
int mesh_epb(const mxsem_mesh* m);
int mesh_cols(const mxsem_mesh* m);
void mesh_drop_plans(mxsem_mesh* m);
// gather-scatter tiles of problem p, one list per XCD (see solver.hip)
void gs_tiles_by_xcd(const mxsem_mesh* m, int p, std::vector<std::vector<Tile>>& lists);
// bytes of the work vectors and partial sums of one vector precision
size_t solver_bufs_bytes(const mxsem_mesh* m, int vprec);
// carve them from ws + at (layout pass: ws == nullptr only counts)
void carve_solver_bufs(mxsem_mesh* m, int vprec, char* ws, Layout& L);
const void* G_ptr(const mxsem_mesh* m, int gprec);
const void* hB_ptr(const mxsem_mesh* m, int gprec);
int apply_impl(mxsem_mesh* m, int prec, const void* u, void* w, unsigned flags, hipStream_t s);
// largest copy count of a node of the mesh
int max_copies(const mxsem_mesh* m);
// DotMode of an mxsem_dot_acc value (MXSEM_DOT_DEFAULT: fallback)
inline int dot_mode_of(int acc, int fallback) {
  return acc == MXSEM_DOT_F64 ? DOT_F64
         : acc == MXSEM_DOT_F32 ? DOT_F32
         : acc == MXSEM_DOT_DOT2 ? DOT_DOT2
                                 : fallback;
}
// learned preconditioner: forward of an attached network into zc (before
// the gather-scatter); the kernel returns at once when st->done.  With w
// (= A p of the step), also the dot partials of NnDots: *dots, *nparts per
// dot, *dstride apart; with x and p, the step's vector update as well.
int nn_launch_fwd(mxsem_nn* nn, const float* r, float* zc, hipStream_t s, const State* st,
                  const float* w = nullptr, int* nparts = nullptr, const double** dots = nullptr,
                  int* dstride = nullptr, float* x = nullptr, const float* p = nullptr);
}  // namespace mx
