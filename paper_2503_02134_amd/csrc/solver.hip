// (P)CG drivers for one problem or a batch of problems: FP64, the paper's
// mixed FP32/FP64 recipe, FP64 iterative refinement around the mixed inner
// solve, and the FP32-everything ablation.
//
// One PCG iteration (the recurrence of the paper's CG-loop table, Sec. 4.1,
// with the vector operations fused):
//   [ax]   p = z + beta p; w = A_L p; partial (p, A_L p)
//   [gs]   w = M QQ^T w  (FP64 sums in every mixed mode)
//   [fin]  sigma = (p,w)_c; alpha = rho / sigma            (FP64 device scalars)
//   [upd]  x += alpha p; r -= alpha w; z = M^-1 r; partials (r,z)_c, (r,r)_c
//   [fin]  convergence / stagnation tests; beta = rho'/rho
// A launch plan holds, for a set of problems, one tile table per stage that
// spans every problem (the operator stage has one table per order/tile
// class) and per-problem device states; K iterations are captured once into
// a HIP graph that the host relaunches, polling the states once per launch.
// Problems that have stopped make their tiles return at once, so a batch
// runs until its slowest member and each member gets the same result as
// when solved alone with the same tiles (same partial-sum decomposition).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

int vprec_of_mode(int mode) {
  switch (mode) {
    case MXSEM_MODE_FP64: return VP_F64;
    case MXSEM_MODE_FP32_ALL: return VP_F32ACC;
    default: return VP_F32;
  }
}
int gprec_of_mode(int mode) {
  switch (mode) {
    case MXSEM_MODE_FP64: return 0;
    case MXSEM_MODE_MIXED_IR_BF16G: return 2;
    case MXSEM_MODE_MIXED_IR_BF16P: return 3;
    default: return 1;
  }
}

int mesh_epb(const mxsem_mesh* m) { return m->epb[m->N] > 0 ? m->epb[m->N] : default_epb(m->N); }
int mesh_cols(const mxsem_mesh* m) { return m->cols[m->N]; }

int region_take(Region& r, void** p, size_t bytes) {
  const size_t o = align256(r.used);
  if (!r.base || o + bytes > r.size) {
    set_error("workspace block exhausted (sized too small for this plan)");
    return MXSEM_EINTERNAL;
  }
  *p = r.base + o;
  r.used = o + (bytes ? bytes : 1);
  return MXSEM_OK;
}

static int gs_bufs_tiles(const mxsem_mesh* m) {
  int ngs = 0;
  for (int q = 0; q <= m->plan.nall; ++q)
    if (q < m->plan.nfree || q == m->plan.nall)
      ngs += (m->plan.bk[q].ngroups + GS_CHUNK - 1) / GS_CHUNK;
  return ngs;
}

// Work vectors x r z p w (FP64 also p_alt, the second direction buffer) and
// the partial-sum arrays of one vector precision, as blocks of the mesh's
// workspace; with ws, m->bufs[vprec] points at them.
void carve_solver_bufs(mxsem_mesh* m, int vprec, char* ws, Layout& L) {
  const size_t es = vprec == VP_F64 ? 8 : 4;
  const int64_t nl = m->nloc;
  const int nt_gs = gs_bufs_tiles(m);
  const int nt_upd = (int)((nl + UPD_CHUNK - 1) / UPD_CHUNK);
  SolverBufs* b = ws ? new SolverBufs() : nullptr;
  auto put = [&](void** p, size_t bytes) {
    const size_t o = L.take(bytes);
    if (b) *p = ws + o;
  };
  void* dummy = nullptr;
  put(b ? &b->x : &dummy, es * nl);
  put(b ? &b->r : &dummy, es * nl);
  put(b ? &b->z : &dummy, es * nl);
  put(b ? &b->p : &dummy, es * nl);
  put(b ? &b->w : &dummy, es * nl);
  if (vprec == VP_F64) put(b ? &b->p_alt : &dummy, es * nl);
  put(b ? (void**)&b->part_ax : &dummy, sizeof(double) * (m->E + 1));  // any tile size fits
  put(b ? (void**)&b->part_gs : &dummy, sizeof(double) * (nt_gs + 1));
  put(b ? (void**)&b->part_u0 : &dummy, sizeof(double) * (nt_upd + 1));
  put(b ? (void**)&b->part_u1 : &dummy, sizeof(double) * (nt_upd + 1));
  put(b ? (void**)&b->part_u2 : &dummy, sizeof(double) * (nt_upd + nt_gs + 1));
  if (b) {
    b->vprec = vprec;
    b->nt_gs = nt_gs;
    b->nt_upd = nt_upd;
    m->bufs[vprec] = b;
  }
}

int ensure_bufs(mxsem_mesh* m, int vprec, SolverBufs** out) {
  MX_CHECK(m->bufs[vprec], MXSEM_ENOTSUP,
           "solve: the mesh's views leave out this vector precision");
  *out = m->bufs[vprec];
  return MXSEM_OK;
}

void plan_destroy(Plan* pl) {
  if (!pl) return;
  if (pl->graph) (void)hipGraphExecDestroy(pl->graph);
  if (pl->evA) (void)hipEventDestroy(pl->evA);
  if (pl->evB) (void)hipEventDestroy(pl->evB);
  if (pl->hstate) (void)hipHostFree(pl->hstate);
  if (pl->hnorm) (void)hipHostFree(pl->hnorm);
  delete pl;
}

void mesh_drop_plans(mxsem_mesh* m) {
  for (int q = 0; q < 4; ++q) {
    plan_destroy(m->self_plan[q]);
    m->self_plan[q] = nullptr;
  }
}

static int plan_alloc(Plan* pl, void** p, size_t bytes) { return region_take(pl->tables, p, bytes); }

// Gather-scatter tiles of problem p, sorted into one list per XCD.  The
// gather-scatter is the one kernel whose workgroups share cache lines (a
// line of w holds entries of several groups, of several multiplicities),
// and each XCD has its own L2: tiles that touch the same elements should
// run on the same XCD, close together in time.  So the elements are cut
// into XCDS contiguous chunks, each chunk into blocks of about 8K local
// entries, and for every block the groups of every bucket whose first
// copy lies in the block become tiles of that chunk's list, block by
// block.  Tile.pad is the tile's group count (at most GS_CHUNK).  On a box
// lattice the free groups of a block are instead found by index
// arithmetic.  At N = 7 the tiles are runs of at most GS_ROW_EL elements
// along one x line of the lattice, each owning whole rows of the vector
// (Tile.aux = -2, Tile.first the first element, Tile.pad the count); they
// also zero the box boundary, so the mask list is left out.  At N = 15 the
// tiles hold the groups one element owns (Tile.aux = -1) and the mask list
// keeps its index tiles.
void gs_tiles_by_xcd(const mxsem_mesh* m, int p, std::vector<std::vector<Tile>>& lists) {
  const int nx = (int)lists.size();
  const int64_t n3 = m->n3;
  const int eb = (int)std::max<int64_t>(1, 8192 / n3);
  const bool box = m->box_ne > 0, rows = box && m->n == 8;
  const int ne = m->box_ne;
  const int ept = (3 * m->N * m->N - 3 * m->N + 1) <= GS_CHUNK / 4 ? 4 : 1;  // elements per tile
  std::vector<size_t> cur(MAX_BUCKETS, 0);
  for (int e0 = 0; e0 < m->E; e0 += eb) {
    const int e1 = std::min(m->E, e0 + eb);
    const int x = (int)((int64_t)e0 * nx / m->E);
    const int64_t lim = (int64_t)e1 * n3;
    if (rows) {
      for (int e = e0; e < e1;) {
        const int len = std::min({GS_ROW_EL, e1 - e, (e / ne + 1) * ne - e});
        lists[x].push_back(Tile{p, e, -2, len});
        e += len;
      }
    } else if (box) {
      for (int e = e0; e < e1; e += ept) lists[x].push_back(Tile{p, e, -1, std::min(ept, e1 - e)});
    }
    for (int q = 0; q <= m->plan.nall; ++q) {
      if (q >= m->plan.nfree && q < m->plan.nall) continue;  // Dirichlet groups: masked instead
      if (box && q < m->plan.nfree) continue;                  // box tiles above
      if (rows && q == m->plan.nall) continue;                 // the row tiles zero the boundary
      const std::vector<int32_t>& gf = m->gs_first[q];
      size_t g1 = cur[q];
      while (g1 < gf.size() && gf[g1] < lim) ++g1;
      for (size_t f = cur[q]; f < g1; f += GS_CHUNK)
        lists[x].push_back(Tile{p, (int)f, q, (int)std::min<size_t>(GS_CHUNK, g1 - f)});
      cur[q] = g1;
    }
  }
}

// The gather-scatter tile table of a plan: each problem's per-XCD lists,
// interleaved so that workgroup b of a launch runs on XCD b % XCDS, padded
// with empty tiles so that the alignment holds to the end.  w_only: the
// table of the PCG step's gather-scatter of w, which leaves out box-lattice
// problems (their vector pass assembles w).
static void gs_table(mxsem_mesh* const* meshes, int P, std::vector<Tile>& tg, bool w_only = false) {
  std::vector<std::vector<Tile>> gsl(XCDS);
  for (int p = 0; p < P; ++p)
    if (!(w_only && meshes[p]->box_ne > 0)) gs_tiles_by_xcd(meshes[p], p, gsl);
  size_t len = 0;
  for (const auto& l : gsl) len = std::max(len, l.size());
  for (size_t i = 0; i < len; ++i)
    for (int x = 0; x < XCDS; ++x) tg.push_back(i < gsl[x].size() ? gsl[x][i] : Tile{0, 0, 0, 0});
}

size_t plan_table_bytes(mxsem_mesh* const* meshes, int P) {
  std::vector<Tile> tg, tgw;
  gs_table(meshes, P, tg);
  gs_table(meshes, P, tgw, true);
  size_t ax = 0, upd = 0;
  for (int p = 0; p < P; ++p) {
    ax += (size_t)meshes[p]->E;  // at most one tile per element, whatever the tuning
    upd += (size_t)((meshes[p]->nloc + UPD_CHUNK - 1) / UPD_CHUNK);
  }
  // one block per operator class (at most one class per problem), then the
  // gather-scatter and vector-pass tables, problem views, states and norms
  return sizeof(Tile) * ax + 256 * (size_t)(P + 1) + align256(sizeof(Tile) * (tg.size() + 1)) +
         align256(sizeof(Tile) * (tgw.size() + 1)) +
         align256(sizeof(Tile) * (upd + 1)) + align256(sizeof(ProbDev) * P) +
         align256(sizeof(State) * P) + align256(sizeof(double) * P) + 256;
}

// Build the launch plan of P problems (all on one context) in vprec, its
// tables in the workspace block `tables`.
int plan_build(mxsem_mesh* const* meshes, int P, int vprec, Region tables, Plan** out) {
  Plan* pl = new Plan();
  pl->vprec = vprec;
  pl->P = P;
  pl->tables = tables;
  pl->tables.used = 0;
  pl->device = meshes[0]->ctx->device;
  int rc = MXSEM_OK;
  auto fail = [&](int code) {
    plan_destroy(pl);
    return code;
  };
  std::vector<Tile> tg, tgw, tu;
  pl->hprob.resize(P);
  for (int p = 0; p < P; ++p) {
    mxsem_mesh* m = meshes[p];
    SolverBufs* b = nullptr;
    rc = ensure_bufs(m, vprec, &b);
    if (rc != MXSEM_OK) return fail(rc);
    pl->meshes.push_back(m);
    pl->bufs.push_back(b);
    pl->epb_used.push_back(mesh_epb(m));
    pl->cols_used.push_back(mesh_cols(m));
    ProbDev& Q = pl->hprob[p];
    memset(&Q, 0, sizeof(Q));
    Q.E = m->E;
    Q.n3 = m->n3;
    Q.nloc = m->nloc;
    Q.D = vprec == VP_F64 ? (const void*)m->D64 : (const void*)m->D32;
    Q.dinv = vprec == VP_F64 ? (const void*)m->dinv64 : (const void*)m->dinv32;
    Q.mult = m->mult;
    Q.gs = m->plan;
    Q.x = b->x;
    Q.r = b->r;
    Q.z = b->z;
    Q.p = b->p;
    Q.w = b->w;
    Q.p_alt = b->p_alt;
    Q.part_ax = b->part_ax;
    Q.part_gs = b->part_gs;
    Q.part_u0 = b->part_u0;
    Q.part_u1 = b->part_u1;
    Q.part_u2 = b->part_u2;
    Q.nblk_ax = (m->E + pl->epb_used[p] - 1) / pl->epb_used[p];
    Q.nblk_gs = b->nt_gs;
    Q.nblk_upd = b->nt_upd;
    Q.box_ne = m->box_ne;
    Q.box_ln = m->n == 8 ? 3 : 4;
    Q.box_rne = m->box_ne ? 1.0f / (float)m->box_ne : 0.f;
    Q.box_rne2 = m->box_ne ? 1.0f / ((float)m->box_ne * (float)m->box_ne) : 0.f;
    for (int q = 0; q < b->nt_upd; ++q) tu.push_back(Tile{p, q * UPD_CHUNK, 0, 0});
  }
  gs_table(meshes, P, tg);
  gs_table(meshes, P, tgw, true);
  // operator classes (N, tile size, thread mapping)
  typedef std::array<int, 3> AxKey;
  std::vector<AxKey> keys;
  for (int p = 0; p < P; ++p) {
    const AxKey k{meshes[p]->N, pl->epb_used[p], pl->cols_used[p]};
    if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
  }
  std::sort(keys.begin(), keys.end());
  std::vector<std::vector<Tile>> ta(keys.size());
  for (int p = 0; p < P; ++p) {
    const AxKey k{meshes[p]->N, pl->epb_used[p], pl->cols_used[p]};
    const int c = (int)(std::find(keys.begin(), keys.end(), k) - keys.begin());
    const int epb = pl->epb_used[p];
    for (int e = 0; e < meshes[p]->E; e += epb) ta[c].push_back(Tile{p, e, 0, 0});
  }
  for (size_t c = 0; c < keys.size(); ++c) {
    AxClass ac;
    ac.N = keys[c][0];
    ac.epb = keys[c][1];
    ac.cols = keys[c][2];
    ac.ntiles = (int)ta[c].size();
    if ((rc = plan_alloc(pl, (void**)&ac.tiles, sizeof(Tile) * ac.ntiles)) != MXSEM_OK)
      return fail(rc);
    if (hipMemcpy(ac.tiles, ta[c].data(), sizeof(Tile) * ac.ntiles, hipMemcpyHostToDevice) !=
        hipSuccess) {
      set_error("plan: tile upload failed");
      return fail(MXSEM_EHIP);
    }
    pl->ax.push_back(ac);
  }
  pl->nt_gs = (int)tg.size();
  pl->nt_gsw = (int)tgw.size();
  pl->nt_upd = (int)tu.size();
  if ((rc = plan_alloc(pl, (void**)&pl->tiles_gs, sizeof(Tile) * (tg.size() + 1))) != MXSEM_OK ||
      (rc = plan_alloc(pl, (void**)&pl->tiles_gsw, sizeof(Tile) * (tgw.size() + 1))) != MXSEM_OK ||
      (rc = plan_alloc(pl, (void**)&pl->tiles_upd, sizeof(Tile) * (tu.size() + 1))) != MXSEM_OK ||
      (rc = plan_alloc(pl, (void**)&pl->probs, sizeof(ProbDev) * P)) != MXSEM_OK ||
      (rc = plan_alloc(pl, (void**)&pl->states, sizeof(State) * P)) != MXSEM_OK ||
      (rc = plan_alloc(pl, (void**)&pl->dnorm, sizeof(double) * P)) != MXSEM_OK)
    return fail(rc);
  for (int p = 0; p < P; ++p) pl->hprob[p].st = pl->states + p;
  if ((!tg.empty() &&
       hipMemcpy(pl->tiles_gs, tg.data(), sizeof(Tile) * tg.size(), hipMemcpyHostToDevice) !=
           hipSuccess) ||
      (!tgw.empty() &&
       hipMemcpy(pl->tiles_gsw, tgw.data(), sizeof(Tile) * tgw.size(), hipMemcpyHostToDevice) !=
           hipSuccess) ||
      hipMemcpy(pl->tiles_upd, tu.data(), sizeof(Tile) * tu.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipHostMalloc((void**)&pl->hstate, sizeof(State) * P, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&pl->hnorm, sizeof(double) * P, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&pl->evA) != hipSuccess || hipEventCreate(&pl->evB) != hipSuccess) {
    set_error("plan: tile upload / host buffers failed");
    return fail(MXSEM_EHIP);
  }
  *out = pl;
  return MXSEM_OK;
}

bool plan_stale(const Plan* pl) {
  for (int p = 0; p < pl->P; ++p)
    if (pl->epb_used[p] != mesh_epb(pl->meshes[p]) || pl->cols_used[p] != mesh_cols(pl->meshes[p]))
      return true;
  return false;
}

// operator launches of one iteration; skip_first: the first class is
// launched by the caller (timed).  par: the step's parity with two direction
// buffers, -1 with one.
int enqueue_ax(Plan* pl, int gprec, hipStream_t s, bool skip_first, int par = -1) {
  const int kprec = pl->vprec == VP_F64 ? 0 : gprec;
  for (size_t c = skip_first ? 1 : 0; c < pl->ax.size(); ++c) {
    const AxClass& ac = pl->ax[c];
    MX_HIP(launch_ax_solver(kprec, pl->dm, ac.N, ac.tiles, ac.ntiles, pl->probs, ac.epb, s,
                            nullptr, nullptr, par, ac.cols));
  }
  return MXSEM_OK;
}

// The rest of a PCG step after the operator: gather-scatter of w (with
// sigma and alpha finished in the same launch), vector pass, rho/beta and
// the convergence tests.  With FP64 vectors, box-lattice problems skip the
// gather-scatter: their vector pass sums the copies itself, in the same
// order, so the launch only finishes sigma for them (and sums the other
// problems' copies).  On the 32^3, N = 7 mesh this took an FP64 step from
// 101 + 174 us (gather-scatter + vector pass) to 12 + 227 us.  FP32 vectors
// keep the separate gather-scatter: there the neighbour reads cost the
// vector pass 25 us (80 -> 105 us) against 24 us saved (33.5 -> 9.1 us).
static int enqueue_tail(Plan* pl, int pc, hipStream_t s, int par) {
  const bool asm_w = !pl->pairwise && pl->vprec == VP_F64;
  MX_HIP(launch_gs_solver(pl->vprec, asm_w ? pl->tiles_gsw : pl->tiles_gs,
                          asm_w ? pl->nt_gsw : pl->nt_gs, pl->probs, s, false, pl->P, nullptr, 0,
                          pl->pairwise != 0));
  MX_HIP(launch_update(pl->vprec, pc, pl->tiles_upd, pl->nt_upd, pl->probs, s, pl->dm, par, asm_w));
  MX_HIP(launch_fin_rho(pl->probs, pl->P, 0, s));
  return MXSEM_OK;
}

// Two direction buffers (x updated every second step from both steps'
// alpha p) for FP64 vectors: the vector pass moves 16 B/dof less every two
// steps.  With FP32 vectors the second 4 B/dof buffer does not fit beside
// the reused vectors in the 256 MB last-level cache and the gather-scatter
// loses more than the vector pass gains, so they keep one buffer updated in
// place.  With an even K every graph launch starts at an even step.
static bool two_dir(const Plan* pl, int K) { return pl->vprec == VP_F64 && K % 2 == 0; }

// K iterations; the first iteration's operator launches stay outside
static int get_graph(Plan* pl, mxsem_ctx* ctx, int gprec, int pc, int K) {
  if (pl->graph && pl->graph_k == K && pl->graph_pc == pc && pl->graph_gprec == gprec &&
      pl->graph_method == MXSEM_METHOD_PCG && pl->graph_dm == pl->dm &&
      pl->graph_pairwise == pl->pairwise)
    return MXSEM_OK;
  if (pl->graph) {
    MX_HIP(hipGraphExecDestroy(pl->graph));
    pl->graph = nullptr;
  }
  hipStream_t cs = ctx->capture;
  hipGraph_t g = nullptr;
  MX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = MXSEM_OK;
  const bool two_p = two_dir(pl, K);
  for (int k = 0; k < K && rc == MXSEM_OK; ++k) {
    const int par = two_p ? k % 2 : -1;
    if (k > 0) rc = enqueue_ax(pl, gprec, cs, false, par);
    if (rc == MXSEM_OK) rc = enqueue_tail(pl, pc, cs, par);
  }
  hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc != MXSEM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    return MXSEM_EHIP;
  }
  e = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    pl->graph = nullptr;
    return MXSEM_EHIP;
  }
  pl->graph_k = K;
  pl->graph_pc = pc;
  pl->graph_gprec = gprec;
  pl->graph_method = MXSEM_METHOD_PCG;
  pl->graph_dm = pl->dm;
  pl->graph_pairwise = pl->pairwise;
  return MXSEM_OK;
}

// Inner (P)CG on the active problems: r = rhs[p] * scale[p], x = 0,
// relative tolerance tol[p], at most maxit[p] iterations.  Inactive
// problems are marked done and their tiles return at once.
struct Inner {
  std::vector<const double*> rhs;
  std::vector<double> scale, tol;
  std::vector<int> maxit;
  std::vector<char> active;
  double* history = nullptr;  // single-problem plans only
  int dm = DOT_F64;            // DotMode of the dots (PCG)
  int pairwise = 0;             // pairwise gather-scatter order (PCG)
  // results
  std::vector<int> iterations, reason, fallback;
  std::vector<double> res;
};

static int run_inner(Plan* pl, mxsem_ctx* ctx, int gprec, int pc, int K, Inner& in) {
  hipStream_t s = ctx->stream;
  const int P = pl->P;
  int max_launch = 0;
  pl->dm = in.dm;
  pl->pairwise = in.pairwise;
  for (int p = 0; p < P; ++p) {
    State& st = pl->hstate[p];
    memset(&st, 0, sizeof(State));
    st.tol2 = in.tol[p] * in.tol[p];
    st.maxit = in.maxit[p];
    st.history = (P == 1) ? in.history : nullptr;
    st.pc = pc;
    st.done = in.active[p] ? 0 : 1;
    st.reason = in.active[p] ? 0 : MXSEM_CONVERGED;
    ProbDev& Q = pl->hprob[p];
    mxsem_mesh* m = pl->meshes[p];
    const int gp = pl->vprec == VP_F64 ? 0 : gprec;
    Q.rhs64 = in.rhs[p];
    Q.rhs_scale = in.scale[p];
    Q.G = G_ptr(m, gp);
    Q.hB = hB_ptr(m, gp);
    Q.gs = m->plan;  // the element ranks of the pairwise order may have changed
    Q.dm = in.dm;
    if (in.active[p]) max_launch = std::max(max_launch, in.maxit[p] / K + 2);
  }
  MX_HIP(hipMemcpyAsync(pl->probs, pl->hprob.data(), sizeof(ProbDev) * P, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(pl->states, pl->hstate, sizeof(State) * P, hipMemcpyHostToDevice, s));
  MX_HIP(launch_init(pl->vprec, pc, pl->tiles_upd, pl->nt_upd, pl->probs, nullptr, s, in.dm));
  MX_HIP(launch_fin_rho(pl->probs, P, 1, s));
  MX_TRY(get_graph(pl, ctx, gprec, pc, K));
  const int kprec = pl->vprec == VP_F64 ? 0 : gprec;
  const int par0 = two_dir(pl, K) ? 0 : -1;
  for (int l = 0; l < max_launch; ++l) {
    // the chunk's first operator launch of class 0, with its own start/end events
    const AxClass& a0 = pl->ax[0];
    MX_HIP(launch_ax_solver(kprec, pl->dm, a0.N, a0.tiles, a0.ntiles, pl->probs, a0.epb, s,
                            pl->evA, pl->evB, par0, a0.cols));
    MX_TRY(enqueue_ax(pl, gprec, s, true, par0));
    MX_HIP(hipGraphLaunch(pl->graph, s));
    MX_HIP(hipMemcpyAsync(pl->hstate, pl->states, sizeof(State) * P, hipMemcpyDeviceToHost, s));
    MX_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    MX_HIP(hipEventElapsedTime(&ms, pl->evA, pl->evB));
    pl->ax_ms_sum += ms;
    pl->ax_samples += 1;
    bool all = true;
    for (int p = 0; p < P; ++p) all = all && pl->hstate[p].done;
    if (all) break;
  }
  // a problem that stopped after an even step still owes x its last alpha p
  if (par0 == 0) MX_HIP(launch_x_pending(pl->vprec, pl->tiles_upd, pl->nt_upd, pl->probs, s));
  in.iterations.assign(P, 0);
  in.reason.assign(P, 0);
  in.res.assign(P, 0.0);
  for (int p = 0; p < P; ++p) {
    if (!in.active[p]) continue;
    const State& st = pl->hstate[p];
    in.iterations[p] = st.iter;
    in.reason[p] = st.done ? st.reason : MXSEM_MAX_ITER;
    in.res[p] = st.res;
  }
  return MXSEM_OK;
}

// ------------------------------------------------------------------ flexible CG
// z = M^-1 r for a flexible-CG step: the learned map (forward + FP64
// gather-scatter of c z_L) or Jacobi/identity; then (r,z)_c, (z, A p)_c and
// beta.  A rejected learned z is replaced by Jacobi within the same step.
static int enqueue_fcg_z(Plan* pl, int pc, hipStream_t s, bool init) {
  if (pc == MXSEM_PC_LEARNED) {
    // One forward launch applies the step's vector update (x += alpha p,
    // r -= alpha w; not at the start of a solve) and sums (r,r)_c and the
    // step's dots, for the learned z (from c z_L) and for the Jacobi
    // candidate dinv r; the end-of-step tests, beta and the choice between
    // the candidates then come before the assembly, and one launch
    // assembles the learned z or, where it was rejected, writes dinv r.
    mxsem_mesh* m = pl->meshes[0];
    const SolverBufs* b = pl->bufs[0];
    int nparts = 0, dstride = 0;
    const double* dots = nullptr;
    MX_TRY(nn_launch_fwd(m->nn, (const float*)b->r, (float*)b->z, s, pl->hprob[0].st,
                         (const float*)b->w, &nparts, &dots, &dstride,
                         init ? nullptr : (float*)b->x, init ? nullptr : (const float*)b->p));
    MX_HIP(launch_fin_beta(pl->probs, pl->P, init ? 1 : 0, s, dots, nparts, dstride));
    MX_HIP(launch_gs_solver(pl->vprec, pl->tiles_gs, pl->nt_gs, pl->probs, s, true, 0,
                            pl->tiles_upd, pl->nt_upd));
  } else if (pc == MXSEM_PC_MG) {
    // two-level Schwarz / multigrid z (single-problem plans)
    MX_TRY(mg_apply(pl->meshes[0], pl->vprec, pl->bufs[0]->r, pl->bufs[0]->z, s, pl->hprob[0].st,
                    pl));
    MX_TRY(mg_prolong_dots(pl->meshes[0], pl, s));
    MX_HIP(launch_fin_beta(pl->probs, pl->P, init ? 1 : 0, s));
  } else {
    MX_HIP(launch_zpc(pl->vprec, pl->tiles_upd, pl->nt_upd, pl->probs, pc, s));
    MX_HIP(launch_fcg_dots(pl->vprec, pl->tiles_upd, pl->nt_upd, pl->probs, s));
    MX_HIP(launch_fin_beta(pl->probs, pl->P, init ? 1 : 0, s));
  }
  return MXSEM_OK;
}

static int get_graph_fcg(Plan* pl, mxsem_ctx* ctx, int gprec, int pc, int K) {
  if (pl->graph && pl->graph_k == K && pl->graph_pc == pc && pl->graph_gprec == gprec &&
      pl->graph_method == MXSEM_METHOD_FCG && pl->graph_dm == pl->dm &&
      pl->graph_pairwise == pl->pairwise)
    return MXSEM_OK;
  if (pl->graph) {
    MX_HIP(hipGraphExecDestroy(pl->graph));
    pl->graph = nullptr;
  }
  hipStream_t cs = ctx->capture;
  hipGraph_t g = nullptr;
  MX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = MXSEM_OK;
  for (int k = 0; k < K && rc == MXSEM_OK; ++k) {
    if (k > 0) rc = enqueue_ax(pl, gprec, cs, false);
    if (rc != MXSEM_OK) break;
    hipError_t e = launch_gs_solver(pl->vprec, pl->tiles_gs, pl->nt_gs, pl->probs, cs, false, pl->P);
    if (pc != MXSEM_PC_LEARNED) {  // the learned forward does the update and the tests itself
      if (e == hipSuccess) e = launch_update(pl->vprec, -1, pl->tiles_upd, pl->nt_upd, pl->probs, cs);
      if (e == hipSuccess) e = launch_fin_rho(pl->probs, pl->P, 2, cs);
    }
    if (e != hipSuccess) {
      set_error(std::string("flexible CG capture: ") + hipGetErrorString(e));
      rc = MXSEM_EHIP;
      break;
    }
    rc = enqueue_fcg_z(pl, pc, cs, false);
  }
  hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc != MXSEM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    return MXSEM_EHIP;
  }
  e = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    pl->graph = nullptr;
    return MXSEM_EHIP;
  }
  pl->graph_k = K;
  pl->graph_pc = pc;
  pl->graph_gprec = gprec;
  pl->graph_method = MXSEM_METHOD_FCG;
  pl->graph_dm = pl->dm;
  pl->graph_pairwise = pl->pairwise;
  return MXSEM_OK;
}

static int run_inner_fcg(Plan* pl, mxsem_ctx* ctx, int gprec, int pc, int K, Inner& in) {
  hipStream_t s = ctx->stream;
  const int P = pl->P;
  int max_launch = 0;
  pl->dm = DOT_F64;  // flexible CG: FP64 partials (the mode's own accumulation inside them)
  pl->pairwise = 0;
  for (int p = 0; p < P; ++p) {
    State& st = pl->hstate[p];
    memset(&st, 0, sizeof(State));
    st.tol2 = in.tol[p] * in.tol[p];
    st.maxit = in.maxit[p];
    st.history = (P == 1) ? in.history : nullptr;
    st.pc = pc;
    st.done = in.active[p] ? 0 : 1;
    st.reason = in.active[p] ? 0 : MXSEM_CONVERGED;
    ProbDev& Q = pl->hprob[p];
    mxsem_mesh* m = pl->meshes[p];
    const int gp = pl->vprec == VP_F64 ? 0 : gprec;
    Q.rhs64 = in.rhs[p];
    Q.rhs_scale = in.scale[p];
    Q.G = G_ptr(m, gp);
    Q.hB = hB_ptr(m, gp);
    Q.dm = DOT_F64;
    if (in.active[p]) max_launch = std::max(max_launch, in.maxit[p] / K + 2);
  }
  MX_HIP(hipMemcpyAsync(pl->probs, pl->hprob.data(), sizeof(ProbDev) * P, hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(pl->states, pl->hstate, sizeof(State) * P, hipMemcpyHostToDevice, s));
  MX_HIP(launch_init(pl->vprec, -1, pl->tiles_upd, pl->nt_upd, pl->probs, nullptr, s));
  MX_HIP(launch_fin_rho(pl->probs, P, 3, s));
  MX_TRY(enqueue_fcg_z(pl, pc, s, true));
  MX_TRY(get_graph_fcg(pl, ctx, gprec, pc, K));
  const int kprec = pl->vprec == VP_F64 ? 0 : gprec;
  for (int l = 0; l < max_launch; ++l) {
    const AxClass& a0 = pl->ax[0];
    MX_HIP(launch_ax_solver(kprec, pl->dm, a0.N, a0.tiles, a0.ntiles, pl->probs, a0.epb, s,
                            pl->evA, pl->evB, -1, a0.cols));
    MX_TRY(enqueue_ax(pl, gprec, s, true));
    MX_HIP(hipGraphLaunch(pl->graph, s));
    MX_HIP(hipMemcpyAsync(pl->hstate, pl->states, sizeof(State) * P, hipMemcpyDeviceToHost, s));
    MX_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    MX_HIP(hipEventElapsedTime(&ms, pl->evA, pl->evB));
    pl->ax_ms_sum += ms;
    pl->ax_samples += 1;
    bool all = true;
    for (int p = 0; p < P; ++p) all = all && pl->hstate[p].done;
    if (all) break;
  }
  in.iterations.assign(P, 0);
  in.reason.assign(P, 0);
  in.res.assign(P, 0.0);
  in.fallback.assign(P, 0);
  for (int p = 0; p < P; ++p) {
    if (!in.active[p]) continue;
    const State& st = pl->hstate[p];
    in.iterations[p] = st.iter;
    in.reason[p] = st.done ? st.reason : MXSEM_MAX_ITER;
    in.res[p] = st.res;
    in.fallback[p] = st.fallback;
  }
  return MXSEM_OK;
}

// per-problem FP64 scalars, one host synchronisation for all problems
static int norms_of(Plan* pl, mxsem_ctx* ctx, std::vector<double>& out) {
  hipStream_t s = ctx->stream;
  MX_HIP(hipMemcpyAsync(pl->hnorm, pl->dnorm, sizeof(double) * pl->P, hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  out.assign(pl->hnorm, pl->hnorm + pl->P);
  return MXSEM_OK;
}

// r = b - A64 x of problem p, (r,r)_c into pl->dnorm[p] (async); w: work
static int residual64(Plan* pl, int p, const double* b, const double* x, double* r, double* w) {
  mxsem_mesh* m = pl->meshes[p];
  hipStream_t s = m->ctx->stream;
  MX_TRY(apply_impl(m, MXSEM_F64, x, w, 0, s));
  MX_HIP(launch_residual(b, w, r, m->mult, m->nloc, m->part, pl->dnorm + p, s));
  return MXSEM_OK;
}

int get_self_plan(mxsem_mesh* m, int vprec, Plan** out) {
  if (m->self_plan[vprec] && plan_stale(m->self_plan[vprec])) {
    plan_destroy(m->self_plan[vprec]);
    m->self_plan[vprec] = nullptr;
  }
  if (!m->self_plan[vprec]) MX_TRY(plan_build(&m, 1, vprec, m->plan_tables[vprec], &m->self_plan[vprec]));
  *out = m->self_plan[vprec];
  return MXSEM_OK;
}

// Solve every problem of a problem set; get(vprec, &plan) supplies the
// launch plan of the set in a vector precision.
template <typename GetPlan>
static int solve_many(mxsem_ctx* ctx, const std::vector<mxsem_mesh*>& meshes, GetPlan get,
                      const mxsem_solve_opts* o, const double* const* b, double* const* x,
                      mxsem_solve_stats* st) {
  const int P = (int)meshes.size();
  const int mode = o->mode;
  const int vprec = vprec_of_mode(mode);
  const int gprec = gprec_of_mode(mode);
  hipStream_t s = ctx->stream;
  for (int p = 0; p < P; ++p) {
    mxsem_mesh* m = meshes[p];
    if (o->gs_order == MXSEM_GS_ORDER_PAIRWISE)
      MX_CHECK(max_copies(m) <= GS_PAIRWISE_MAXM, MXSEM_ENOTSUP,
               "solve: pairwise gather-scatter order takes at most 16 copies per node");
    if (vprec != VP_F64)
      MX_CHECK(m->dinv32 && (gprec == 2 || m->G32), MXSEM_ENOTSUP, "solve: mesh has no FP32 view");
    if (gprec == 2) MX_CHECK(m->G16, MXSEM_ENOTSUP, "solve: mesh has no BF16 view");
    memset(&st[p], 0, sizeof(mxsem_solve_stats));
  }
  Plan* pl = nullptr;
  MX_TRY(get(vprec, &pl));
  pl->ax_ms_sum = 0.0;
  pl->ax_samples = 0;
  MX_HIP(hipEventRecord(ctx->ev0, s));
  // ||b||_c per problem
  std::vector<double> bnorm;
  for (int p = 0; p < P; ++p)
    MX_HIP(launch_dot(MXSEM_F64, b[p], b[p], meshes[p]->mult, meshes[p]->nloc, meshes[p]->part,
                      pl->dnorm + p, s));
  MX_TRY(norms_of(pl, ctx, bnorm));
  for (double& v : bnorm) v = sqrt(v);
  const bool ir = mode == MXSEM_MODE_MIXED_IR || mode == MXSEM_MODE_MIXED_IR_BF16G ||
                  mode == MXSEM_MODE_MIXED_IR_BF16P;
  const int xv = vprec == VP_F64 ? 0 : 1;
  Inner in;
  in.rhs.assign(P, nullptr);
  in.scale.assign(P, 1.0);
  in.tol.assign(P, o->tol);
  in.maxit.assign(P, o->max_iter);
  in.active.assign(P, 1);
  in.history = o->history;
  in.dm = vprec == VP_F64 ? DOT_F64
                          : dot_mode_of(o->dot, mode == MXSEM_MODE_FP32_ALL ? DOT_F32 : DOT_F64);
  in.pairwise = o->gs_order == MXSEM_GS_ORDER_PAIRWISE ? 1 : 0;
  std::vector<char> fallback(P, 0);
  // the learned and the multigrid preconditioners run in flexible CG (the
  // multigrid one is linear and symmetric, so this is PCG with one more dot)
  const bool fcg = o->method == MXSEM_METHOD_FCG || o->pc == MXSEM_PC_LEARNED ||
                   o->pc == MXSEM_PC_MG;
  auto inner = [&](Plan* q, int gp, Inner& io) {
    return fcg ? run_inner_fcg(q, ctx, gp, o->pc, o->graph_chunk, io)
               : run_inner(q, ctx, gp, o->pc, o->graph_chunk, io);
  };
  std::vector<int> nfb(P, 0);
  if (!ir) {
    std::vector<double> rn(P, 0.0);
    if (o->x0_given) {
      // solve A d = b - A x0 and add d: the iterates of a solve started at x0
      for (int p = 0; p < P; ++p)
        MX_TRY(residual64(pl, p, b[p], x[p], meshes[p]->tmpa, meshes[p]->tmpb));
      MX_TRY(norms_of(pl, ctx, rn));
      for (int p = 0; p < P; ++p) {
        rn[p] = sqrt(rn[p]);
        in.rhs[p] = meshes[p]->tmpa;
        in.tol[p] = rn[p] > 0 ? o->tol * bnorm[p] / rn[p] : o->tol;
      }
    } else {
      for (int p = 0; p < P; ++p) in.rhs[p] = b[p];
    }
    MX_TRY(inner(pl, gprec, in));
    for (int p = 0; p < P; ++p) {
      if (fcg) nfb[p] += in.fallback[p];
      MX_HIP(launch_axpy_cast(xv, x[p], pl->bufs[p]->x, 1.0, o->x0_given ? 1.0 : 0.0,
                              meshes[p]->nloc, s));
      st[p].iterations = in.iterations[p];
      st[p].reason = in.reason[p];
      st[p].rel_res_recursive = in.res[p];
    }
  } else {
    // FP64 iterative refinement: r = b - A64 x; d = inner mixed PCG on r/s; x += s d
    std::vector<int> total(P, 0), outer(P, 0), slow(P, 0), live(P, 1);
    std::vector<double> prev(P, -1.0), rn;
    for (int p = 0; p < P; ++p) {
      if (!o->x0_given) MX_HIP(launch_zero(x[p], meshes[p]->nloc, s));
      st[p].reason = MXSEM_MAX_ITER;
    }
    for (;;) {
      bool any = false;
      for (int p = 0; p < P; ++p)
        if (live[p]) MX_TRY(residual64(pl, p, b[p], x[p], meshes[p]->tmpa, meshes[p]->tmpb));
      MX_TRY(norms_of(pl, ctx, rn));
      for (int p = 0; p < P; ++p) {
        in.active[p] = 0;
        if (!live[p]) continue;
        const double r = sqrt(rn[p]);
        const double rel = bnorm[p] > 0 ? r / bnorm[p] : 0.0;
        if (rel <= o->tol) {
          st[p].reason = MXSEM_CONVERGED;
          live[p] = 0;
          continue;
        }
        if (outer[p] >= o->max_outer || total[p] >= o->max_iter) {
          live[p] = 0;
          continue;
        }
        if (prev[p] > 0 && rel > 0.5 * prev[p]) ++slow[p];
        prev[p] = rel;
        if (slow[p] >= 2) {  // refinement stopped contracting: finish in FP64
          fallback[p] = 1;
          live[p] = 0;
          continue;
        }
        in.active[p] = 1;
        in.rhs[p] = meshes[p]->tmpa;
        in.scale[p] = 1.0 / r;
        in.tol[p] = fmax(o->inner_tol, o->tol * bnorm[p] / r);
        in.maxit[p] = o->max_iter - total[p];
        rn[p] = r;
        any = true;
      }
      if (!any) break;
      MX_TRY(inner(pl, gprec, in));
      for (int p = 0; p < P; ++p) {
        if (!in.active[p]) continue;
        if (fcg) nfb[p] += in.fallback[p];
        MX_HIP(launch_axpy_cast(1, x[p], pl->bufs[p]->x, rn[p], 1.0, meshes[p]->nloc, s));
        total[p] += in.iterations[p];
        st[p].rel_res_recursive = in.res[p];
        ++outer[p];
        if (in.reason[p] == MXSEM_BREAKDOWN) {
          st[p].reason = MXSEM_BREAKDOWN;
          live[p] = 0;
        }
      }
    }
    for (int p = 0; p < P; ++p) {
      st[p].iterations = total[p];
      st[p].outer = outer[p];
    }
    // problems whose refinement stalled: FP64 PCG from the current x
    bool anyf = false;
    for (int p = 0; p < P; ++p) anyf = anyf || fallback[p];
    if (anyf) {
      Plan* p64 = nullptr;
      MX_TRY(get(VP_F64, &p64));
      Inner f;
      f.rhs.assign(P, nullptr);
      f.scale.assign(P, 1.0);
      f.tol.assign(P, o->tol);
      f.maxit.assign(P, 1);
      f.active.assign(P, 0);
      for (int p = 0; p < P; ++p)
        if (fallback[p]) MX_TRY(residual64(p64, p, b[p], x[p], meshes[p]->tmpa, meshes[p]->tmpb));
      std::vector<double> fr;
      MX_TRY(norms_of(p64, ctx, fr));
      for (int p = 0; p < P; ++p) {
        if (!fallback[p]) continue;
        const double r = sqrt(fr[p]);
        f.active[p] = 1;
        f.rhs[p] = meshes[p]->tmpa;
        f.tol[p] = r > 0 ? o->tol * bnorm[p] / r : o->tol;
        f.maxit[p] = std::max(1, o->max_iter - st[p].iterations);
      }
      if (o->pc == MXSEM_PC_MG)
        MX_TRY(run_inner_fcg(p64, ctx, 0, MXSEM_PC_MG, o->graph_chunk, f));
      else
        MX_TRY(run_inner(p64, ctx, 0, o->pc == MXSEM_PC_LEARNED ? MXSEM_PC_JACOBI : o->pc,
                         o->graph_chunk, f));
      for (int p = 0; p < P; ++p) {
        if (!fallback[p]) continue;
        MX_HIP(launch_axpy_cast(0, x[p], p64->bufs[p]->x, 1.0, 1.0, meshes[p]->nloc, s));
        st[p].iterations += f.iterations[p];
        st[p].reason = f.reason[p];
        st[p].fallback_used = 1;
        st[p].rel_res_recursive = f.res[p];
      }
    }
  }
  // true FP64 residuals
  std::vector<double> tr;
  for (int p = 0; p < P; ++p)
    MX_TRY(residual64(pl, p, b[p], x[p], meshes[p]->tmpb, meshes[p]->tmpa));
  MX_TRY(norms_of(pl, ctx, tr));
  MX_HIP(hipEventRecord(ctx->ev1, s));
  MX_HIP(hipEventSynchronize(ctx->ev1));
  float ms = 0.f;
  MX_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  bool breakdown = false;
  for (int p = 0; p < P; ++p) {
    st[p].rel_res = bnorm[p] > 0 ? sqrt(tr[p]) / bnorm[p] : 0.0;
    st[p].ms = ms;
    st[p].ax_samples = pl->ax_samples;
    st[p].ax_ms = pl->ax_samples ? pl->ax_ms_sum / pl->ax_samples : 0.0;
    if (fcg) st[p].fallback_used += nfb[p];
    breakdown = breakdown || st[p].reason == MXSEM_BREAKDOWN;
  }
  if (breakdown) {
    set_error("solve: (p, A p) <= 0 or non-finite");
    return MXSEM_EBREAKDOWN;
  }
  return MXSEM_OK;
}

}  // namespace mx

using namespace mx;

struct mxsem_batch {
  mxsem_ctx* ctx = nullptr;
  std::vector<mxsem_mesh*> meshes;
  mx::Plan* plans[4] = {nullptr, nullptr, nullptr, nullptr};
  mx::Region tables[4];  // workspace blocks of the plans' launch tables
};

namespace mx {
// Layout of a batch workspace: the launch tables of the three plans a batch
// can build (FP64, FP32, FP32 with FP32 sums), overlapped by the autotuning
// scratch that batch_create may need before any plan exists.
static size_t batch_layout(mxsem_mesh* const* meshes, int P, const char* path, size_t* table_bytes) {
  const size_t tb = align256(plan_table_bytes(meshes, P));
  *table_bytes = tb;
  size_t tune = 0;
  if (path && path[0])
    for (int p = 0; p < P; ++p) {
      int e2 = 1;
      while (e2 < meshes[p]->E) e2 <<= 1;
      tune = std::max(tune, autotune_bytes(meshes[p]->N, e2, MXSEM_F32));
    }
  return std::max(3 * tb, tune);
}
static const char* tune_path(const char* tune_cache) {
  return tune_cache ? tune_cache : getenv("MXSEM_TUNE_CACHE");
}
}  // namespace mx

extern "C" {

void mxsem_solve_opts_default(mxsem_solve_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->method = MXSEM_METHOD_PCG;
  o->pc = MXSEM_PC_JACOBI;
  o->mode = MXSEM_MODE_FP64;
  o->tol = 1e-10;
  o->max_iter = 10000;
  o->inner_tol = 1e-4;
  o->max_outer = 10;
  o->graph_chunk = 16;
  o->x0_given = 0;
  o->history = nullptr;
}

int mxsem_precond(mxsem_mesh* m, mxsem_pc pc, mxsem_prec io, const void* r, void* z) {
  MX_API_BEGIN
  MX_CHECK(m && r && z, MXSEM_EINVAL, "precond: null argument");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  if (pc == MXSEM_PC_LEARNED) {
    MX_CHECK(m->nn, MXSEM_EINVAL, "precond: no network attached");
    MX_CHECK(io == MXSEM_F32, MXSEM_ENOTSUP, "precond: the learned map takes FP32 vectors");
    return mxsem_nn_forward(m->nn, (const float*)r, (float*)z);
  }
  if (pc == MXSEM_PC_MG) {
    MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "precond: io must be F64/F32");
    MX_CHECK(r != z, MXSEM_EINVAL, "precond: r and z must not alias for the multigrid map");
    return mg_apply(m, io == MXSEM_F64 ? VP_F64 : VP_F32, r, z, m->ctx->stream, nullptr);
  }
  MX_CHECK(pc == MXSEM_PC_IDENTITY || pc == MXSEM_PC_JACOBI, MXSEM_EINVAL, "precond: unknown pc");
  MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "precond: io must be F64/F32");
  if (io == MXSEM_F32) MX_CHECK(m->dinv32, MXSEM_ENOTSUP, "precond: mesh has no FP32 view");
  const void* dinv = io == MXSEM_F64 ? (const void*)m->dinv64 : (const void*)m->dinv32;
  MX_HIP(launch_precond(io, pc, r, z, dinv, m->nloc, m->ctx->stream));
  return MXSEM_OK;
  MX_API_END("mxsem_precond")
}

static int check_opts(const mxsem_solve_opts* o) {
  MX_CHECK(o->tol >= 0.0 && o->max_iter >= 1 && o->graph_chunk >= 1 && o->graph_chunk <= 256,
           MXSEM_EINVAL, "solve: bad tol / max_iter / graph_chunk");
  MX_CHECK(o->mode >= MXSEM_MODE_FP64 && o->mode <= MXSEM_MODE_MIXED_IR_BF16P, MXSEM_EINVAL,
           "solve: unknown mode");
  MX_CHECK(o->pc == MXSEM_PC_IDENTITY || o->pc == MXSEM_PC_JACOBI || o->pc == MXSEM_PC_LEARNED ||
               o->pc == MXSEM_PC_MG,
           MXSEM_EINVAL, "solve: unknown preconditioner");
  MX_CHECK(o->max_outer >= 0 && o->inner_tol > 0.0 && o->inner_tol < 1.0, MXSEM_EINVAL,
           "solve: bad refinement options");
  MX_CHECK(!o->x0_given || o->mode == MXSEM_MODE_FP64 || o->mode == MXSEM_MODE_MIXED_IR ||
               o->mode == MXSEM_MODE_MIXED_IR_BF16G || o->mode == MXSEM_MODE_MIXED_IR_BF16P,
           MXSEM_ENOTSUP, "solve: x0 is supported in the FP64 and refinement modes");
  MX_CHECK(o->dot >= MXSEM_DOT_DEFAULT && o->dot <= MXSEM_DOT_DOT2, MXSEM_EINVAL,
           "solve: unknown dot accumulation");
  MX_CHECK(o->gs_order == MXSEM_GS_ORDER_ONE || o->gs_order == MXSEM_GS_ORDER_PAIRWISE,
           MXSEM_EINVAL, "solve: unknown gather-scatter order");
  const bool pcg = o->method == MXSEM_METHOD_PCG && o->pc != MXSEM_PC_LEARNED &&
                   o->pc != MXSEM_PC_MG;
  MX_CHECK(o->mode != MXSEM_MODE_MIXED_IR_BF16P || pcg, MXSEM_ENOTSUP,
           "solve: the BF16-direction ablation is for PCG");
  MX_CHECK(o->dot == MXSEM_DOT_DEFAULT || o->dot == MXSEM_DOT_F64 ||
               (pcg && (o->mode == MXSEM_MODE_MIXED || o->mode == MXSEM_MODE_MIXED_IR ||
                        o->mode == MXSEM_MODE_FP32_ALL)),
           MXSEM_ENOTSUP,
           "solve: FP32 and Dot2 dots are for PCG with FP32 vectors and FP32 G");
  MX_CHECK(o->dot != MXSEM_DOT_F64 || o->mode != MXSEM_MODE_FP32_ALL || pcg, MXSEM_ENOTSUP,
           "solve: flexible CG keeps the mode's own dots");
  MX_CHECK(o->gs_order == MXSEM_GS_ORDER_ONE ||
               (pcg && (o->mode == MXSEM_MODE_MIXED || o->mode == MXSEM_MODE_FP32_ALL)),
           MXSEM_ENOTSUP, "solve: the pairwise gather-scatter order is for PCG in MIXED / FP32_ALL");
  return MXSEM_OK;
}

int mxsem_solve(mxsem_mesh* m, const mxsem_solve_opts* o, const double* b, double* x,
                mxsem_solve_stats* st) {
  MX_API_BEGIN
  MX_CHECK(m && o && b && x && st, MXSEM_EINVAL, "solve: null argument");
  MX_TRY(check_opts(o));
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();  // clear any stale error left by other libraries
  memset(st, 0, sizeof(*st));
  if (o->pc == MXSEM_PC_LEARNED) {
    MX_CHECK(m->nn, MXSEM_EINVAL, "solve: the learned preconditioner needs an attached network");
    MX_CHECK(o->mode != MXSEM_MODE_FP64, MXSEM_ENOTSUP,
             "solve: the learned preconditioner runs in the FP32 inner loop");
  }
  MX_CHECK(o->method == MXSEM_METHOD_PCG || o->method == MXSEM_METHOD_FCG, MXSEM_EINVAL,
           "solve: unknown method");
  if (o->pc == MXSEM_PC_MG)
    MX_CHECK(m->mg, MXSEM_EINVAL, "solve: the mesh was built without MXSEM_VIEW_MG");
  std::vector<mxsem_mesh*> ms{m};
  auto get = [m](int vp, Plan** out) { return get_self_plan(m, vp, out); };
  return solve_many(m->ctx, ms, get, o, &b, &x, st);
  MX_API_END("mxsem_solve")
}

// ------------------------------------------------------------------ batch
int mxsem_autotune_cached(mxsem_ctx* ctx, int N, int E, int prec, const char* path, void* ws,
                          size_t ws_bytes, int* epb, int* cols);

static int check_batch_meshes(mxsem_ctx* ctx, int P, mxsem_mesh* const* meshes) {
  MX_CHECK(ctx && meshes && P >= 1, MXSEM_EINVAL, "batch: bad argument");
  for (int p = 0; p < P; ++p) {
    MX_CHECK(meshes[p], MXSEM_EINVAL, "batch: null mesh");
    MX_CHECK(meshes[p]->ctx == ctx, MXSEM_EINVAL, "batch: meshes must share the context");
    for (int q = 0; q < p; ++q)
      MX_CHECK(meshes[q] != meshes[p], MXSEM_EINVAL, "batch: a mesh appears twice");
  }
  return MXSEM_OK;
}

int mxsem_batch_workspace_bytes(mxsem_ctx* ctx, int P, mxsem_mesh* const* meshes,
                                const char* tune_cache, size_t* bytes) {
  MX_API_BEGIN
  MX_CHECK(bytes, MXSEM_EINVAL, "batch_workspace_bytes: null output");
  MX_TRY(check_batch_meshes(ctx, P, meshes));
  size_t tb = 0;
  *bytes = batch_layout(meshes, P, tune_path(tune_cache), &tb);
  return MXSEM_OK;
  MX_API_END("mxsem_batch_workspace_bytes")
}

int mxsem_batch_create(mxsem_ctx* ctx, int P, mxsem_mesh* const* meshes, const char* tune_cache,
                       void* workspace, size_t ws_bytes, mxsem_batch** out) {
  MX_API_BEGIN
  MX_CHECK(out, MXSEM_EINVAL, "batch_create: null output");
  *out = nullptr;
  MX_TRY(check_batch_meshes(ctx, P, meshes));
  const char* path = tune_path(tune_cache);
  size_t tb = 0;
  const size_t need = batch_layout(meshes, P, path, &tb);
  MX_CHECK(workspace && ((uintptr_t)workspace & 255) == 0, MXSEM_EINVAL,
           "batch_create: workspace must be a 256-byte aligned device pointer");
  MX_CHECK(ws_bytes >= need, MXSEM_EINVAL,
           "batch_create: workspace smaller than mxsem_batch_workspace_bytes");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  if (path && path[0]) {
    // one tuned tile per (N, E rounded up to a power of two), FP32 inner
    // loop; a miss is tuned in the workspace (no plan exists yet)
    for (int p = 0; p < P; ++p) {
      mxsem_mesh* m = meshes[p];
      if (m->epb[m->N] > 0) continue;
      int e2 = 1;
      while (e2 < m->E) e2 <<= 1;
      int epb = 0, cols = 0;
      MX_TRY(mxsem_autotune_cached(ctx, m->N, e2, MXSEM_F32, path, workspace, ws_bytes, &epb,
                                   &cols));
      mxsem_tuning t{};
      t.epb[m->N] = epb;
      t.cols[m->N] = cols;
      MX_TRY(mxsem_mesh_set_tuning(m, &t));
    }
  }
  mxsem_batch* bt = new mxsem_batch();
  bt->ctx = ctx;
  bt->meshes.assign(meshes, meshes + P);
  const int vps[3] = {VP_F64, VP_F32, VP_F32ACC};
  for (int q = 0; q < 3; ++q) {
    bt->tables[vps[q]].base = (char*)workspace + q * tb;
    bt->tables[vps[q]].size = tb;
  }
  ctx->live += 1;
  *out = bt;
  return MXSEM_OK;
  MX_API_END("mxsem_batch_create")
}

int mxsem_batch_destroy(mxsem_batch* bt) {
  MX_API_BEGIN
  if (!bt) return MXSEM_OK;
  (void)hipSetDevice(bt->ctx->device);
  if (bt->ctx->stream) (void)hipStreamSynchronize(bt->ctx->stream);
  else (void)hipDeviceSynchronize();
  for (int q = 0; q < 4; ++q) plan_destroy(bt->plans[q]);
  bt->ctx->live -= 1;
  delete bt;
  return MXSEM_OK;
  MX_API_END("mxsem_batch_destroy")
}

int mxsem_batch_solve(mxsem_batch* bt, const mxsem_solve_opts* o, const double* const* b,
                      double* const* x, mxsem_solve_stats* st) {
  MX_API_BEGIN
  MX_CHECK(bt && o && b && x && st, MXSEM_EINVAL, "batch_solve: null argument");
  MX_TRY(check_opts(o));
  MX_CHECK(o->pc != MXSEM_PC_LEARNED && o->pc != MXSEM_PC_MG, MXSEM_ENOTSUP,
           "batch_solve: batches run (flexible) CG with Jacobi or identity");
  MX_CHECK(!o->history, MXSEM_ENOTSUP, "batch_solve: no residual history for batches");
  const int P = (int)bt->meshes.size();
  for (int p = 0; p < P; ++p) MX_CHECK(b[p] && x[p], MXSEM_EINVAL, "batch_solve: null vector");
  MX_HIP(hipSetDevice(bt->ctx->device));
  (void)hipGetLastError();
  auto get = [bt](int vp, Plan** out) -> int {
    if (bt->plans[vp] && plan_stale(bt->plans[vp])) {
      plan_destroy(bt->plans[vp]);
      bt->plans[vp] = nullptr;
    }
    if (!bt->plans[vp]) {
      int rc = plan_build(bt->meshes.data(), (int)bt->meshes.size(), vp, bt->tables[vp],
                          &bt->plans[vp]);
      if (rc != MXSEM_OK) return rc;
    }
    *out = bt->plans[vp];
    return MXSEM_OK;
  };
  return solve_many(bt->ctx, bt->meshes, get, o, b, x, st);
  MX_API_END("mxsem_batch_solve")
}

}  // extern "C"
