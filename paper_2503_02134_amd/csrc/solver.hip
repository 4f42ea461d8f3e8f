// (P)CG drivers: FP64, the paper's mixed FP32/FP64 recipe, FP64 iterative
// refinement around the mixed inner solve, and the FP32-everything
// ablation.  The iteration itself is captured once per (mesh, precision,
// preconditioner, chunk) into a HIP graph of K iterations; the host
// relaunches the graph and polls one device flag per launch.
//
// One iteration (PCG in the order of the paper's CG-loop table, Sec. 4.1,
// with the vector operations fused):
//   [ax]   p = z + beta p; w = A_L p; partial (p,w) over element interiors
//   [gs]   w = M QQ^T w (FP64 sums); partial (p,w)_c over face nodes
//   [fin]  sigma = (p,w)_c; alpha = rho / sigma       (device scalars, FP64)
//   [upd]  x += alpha p; r -= alpha w; z = M^-1 r; partials (r,z)_c, (r,r)_c
//   [fin]  convergence / stagnation tests; beta = rho'/rho
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

static int vprec_of_mode(int mode) {
  switch (mode) {
    case MXSEM_MODE_FP64: return VP_F64;
    case MXSEM_MODE_FP32_ALL: return VP_F32ACC;
    default: return VP_F32;
  }
}
static int gprec_of_mode(int mode) {
  switch (mode) {
    case MXSEM_MODE_FP64: return 0;
    case MXSEM_MODE_MIXED_IR_BF16G: return 2;
    default: return 1;
  }
}

// operator tiles for the mesh's current elements-per-workgroup choice
int retile_ax(mxsem_mesh* m, SolverBufs* b) {
  const int epb = m->epb[m->N] > 0 ? m->epb[m->N] : default_epb(m->N);
  if (epb == b->epb && b->host_prob.nblk_ax == (m->E + epb - 1) / epb) return MXSEM_OK;
  b->epb = epb;
  b->nt_ax = (m->E + epb - 1) / epb;
  std::vector<Tile> ta(b->nt_ax);
  for (int q = 0; q < b->nt_ax; ++q) ta[q] = Tile{0, q * epb, 0, 0};
  MX_HIP(hipMemcpy(b->tiles_ax, ta.data(), sizeof(Tile) * ta.size(), hipMemcpyHostToDevice));
  b->host_prob.nblk_ax = b->nt_ax;
  if (b->graph) {
    MX_HIP(hipGraphExecDestroy(b->graph));
    b->graph = nullptr;
  }
  return MXSEM_OK;
}

int ensure_bufs(mxsem_mesh* m, int vprec, SolverBufs** out) {
  if (m->bufs[vprec]) {
    *out = m->bufs[vprec];
    return retile_ax(m, *out);
  }
  SolverBufs* b = new SolverBufs();
  b->vprec = vprec;
  const size_t es = vprec == VP_F64 ? 8 : 4;
  const int64_t nl = m->nloc;
  b->epb = m->epb[m->N] > 0 ? m->epb[m->N] : default_epb(m->N);
  b->nt_ax = (m->E + b->epb - 1) / b->epb;
  // gather-scatter tiles: free buckets and the mask list
  std::vector<Tile> tg;
  for (int q = 0; q <= m->plan.nall; ++q) {
    if (q >= m->plan.nfree && q < m->plan.nall) continue;
    const int ngq = m->plan.bk[q].ngroups;
    for (int f = 0; f < ngq; f += GS_CHUNK) tg.push_back(Tile{0, f, q, 0});
  }
  b->nt_gs = (int)tg.size();
  b->nt_upd = (int)((nl + UPD_CHUNK - 1) / UPD_CHUNK);
  int rc = MXSEM_OK;
  auto A = [&](void** p, size_t bytes) {
    if (rc == MXSEM_OK) rc = mesh_alloc(m, p, bytes);
  };
  A(&b->x, es * nl);
  A(&b->r, es * nl);
  A(&b->z, es * nl);
  A(&b->p, es * nl);
  A(&b->w, es * nl);
  A((void**)&b->part_ax, sizeof(double) * (m->E + 1));  // any epb fits
  A((void**)&b->part_gs, sizeof(double) * (b->nt_gs + 1));
  A((void**)&b->part_u0, sizeof(double) * (b->nt_upd + 1));
  A((void**)&b->part_u1, sizeof(double) * (b->nt_upd + 1));
  A((void**)&b->part_u2, sizeof(double) * (b->nt_upd + b->nt_gs + 1));
  A((void**)&b->st, sizeof(State));
  A((void**)&b->probs, sizeof(ProbDev));
  A((void**)&b->tiles_ax, sizeof(Tile) * (m->E + 1));
  A((void**)&b->tiles_gs, sizeof(Tile) * (b->nt_gs + 1));
  A((void**)&b->tiles_upd, sizeof(Tile) * (b->nt_upd + 1));
  if (rc != MXSEM_OK) {
    delete b;
    return rc;
  }
  hipStream_t s = m->ctx->stream;
  std::vector<Tile> ta(b->nt_ax), tu(b->nt_upd);
  for (int q = 0; q < b->nt_ax; ++q) ta[q] = Tile{0, q * b->epb, 0, 0};
  for (int q = 0; q < b->nt_upd; ++q) tu[q] = Tile{0, q * UPD_CHUNK, 0, 0};
  MX_HIP(hipMemcpyAsync(b->tiles_ax, ta.data(), sizeof(Tile) * ta.size(), hipMemcpyHostToDevice, s));
  if (!tg.empty())
    MX_HIP(hipMemcpyAsync(b->tiles_gs, tg.data(), sizeof(Tile) * tg.size(), hipMemcpyHostToDevice, s));
  MX_HIP(hipMemcpyAsync(b->tiles_upd, tu.data(), sizeof(Tile) * tu.size(), hipMemcpyHostToDevice, s));
  MX_HIP(hipStreamSynchronize(s));
  ProbDev& P = b->host_prob;
  memset(&P, 0, sizeof(P));
  P.E = m->E;
  P.n3 = m->n3;
  P.nloc = nl;
  P.D = vprec == VP_F64 ? (const void*)m->D64 : (const void*)m->D32;
  P.dinv = vprec == VP_F64 ? (const void*)m->dinv64 : (const void*)m->dinv32;
  P.mult = m->mult;
  P.gs = m->plan;
  P.x = b->x;
  P.r = b->r;
  P.z = b->z;
  P.p = b->p;
  P.w = b->w;
  P.part_ax = b->part_ax;
  P.part_gs = b->part_gs;
  P.part_u0 = b->part_u0;
  P.part_u1 = b->part_u1;
  P.part_u2 = b->part_u2;
  P.nblk_ax = b->nt_ax;
  P.nblk_gs = b->nt_gs;
  P.nblk_upd = b->nt_upd;
  P.st = b->st;
  m->bufs[vprec] = b;
  *out = b;
  return MXSEM_OK;
}

// enqueue one iteration; head = false leaves out the operator kernel (the
// first iteration of a graph chunk launches it outside the graph, between
// two timing events)
static int enqueue_iteration(mxsem_mesh* m, SolverBufs* b, int gprec, int pc, hipStream_t s,
                             bool head = true) {
  const int kprec = b->vprec == VP_F64 ? 0 : gprec;  // operator kernel variant
  if (head) MX_HIP(launch_ax_solver(kprec, m->N, b->tiles_ax, b->nt_ax, b->probs, b->epb, s));
  MX_HIP(launch_gs_solver(b->vprec, b->tiles_gs, b->nt_gs, b->probs, s));
  MX_HIP(launch_fin_sigma(b->probs, 1, s));
  MX_HIP(launch_update(b->vprec, pc, b->tiles_upd, b->nt_upd, b->probs, s));
  MX_HIP(launch_fin_rho(b->probs, 1, 0, s));
  return MXSEM_OK;
}

static int get_graph(mxsem_mesh* m, SolverBufs* b, int gprec, int pc, int K) {
  if (b->graph && b->graph_k == K && b->graph_pc == pc && b->graph_gprec == gprec) return MXSEM_OK;
  if (b->graph) {
    MX_HIP(hipGraphExecDestroy(b->graph));
    b->graph = nullptr;
  }
  hipStream_t cs = m->ctx->capture;
  hipGraph_t g = nullptr;
  if (!b->evA) {
    MX_HIP(hipEventCreate(&b->evA));
    MX_HIP(hipEventCreate(&b->evB));
  }
  MX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = MXSEM_OK;
  for (int k = 0; k < K && rc == MXSEM_OK; ++k) rc = enqueue_iteration(m, b, gprec, pc, cs, k > 0);
  hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc != MXSEM_OK) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    return MXSEM_EHIP;
  }
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    b->graph = nullptr;
    return MXSEM_EHIP;
  }
  b->graph_k = K;
  b->graph_pc = pc;
  b->graph_gprec = gprec;
  return MXSEM_OK;
}

struct InnerResult {
  int iterations = 0;
  int reason = 0;
  double res = 0.0;
};

// One (P)CG solve on the device from r = rhs64 * scale (x = x0 or 0),
// relative tolerance tol, at most maxit iterations.
static int run_pcg(mxsem_mesh* m, SolverBufs* b, int gprec, int pc, const double* rhs64,
                   double scale, const double* x0, double tol, int maxit, int K, double* history,
                   InnerResult* res) {
  hipStream_t s = m->ctx->stream;
  b->host_prob.rhs64 = rhs64;
  b->host_prob.rhs_scale = scale;
  b->host_prob.G = G_ptr(m, b->vprec == VP_F64 ? 0 : gprec);
  b->host_prob.hB = hB_ptr(m, b->vprec == VP_F64 ? 0 : gprec);
  MX_HIP(hipMemcpyAsync(b->probs, &b->host_prob, sizeof(ProbDev), hipMemcpyHostToDevice, s));
  State& st = b->host_state;
  memset(&st, 0, sizeof(st));
  st.tol2 = tol * tol;
  st.maxit = maxit;
  st.history = history;
  st.pc = pc;
  MX_HIP(hipMemcpyAsync(b->st, &st, sizeof(State), hipMemcpyHostToDevice, s));
  MX_HIP(launch_init(b->vprec, pc, b->tiles_upd, b->nt_upd, b->probs, x0, s));
  MX_HIP(launch_fin_rho(b->probs, 1, 1, s));
  MX_TRY(get_graph(m, b, gprec, pc, K));
  int* flag = m->ctx->pinned_flags;
  const int max_launch = maxit / K + 2;
  const int kprec = b->vprec == VP_F64 ? 0 : gprec;
  for (int l = 0; l < max_launch; ++l) {
    // the chunk's first operator kernel, launched with its own start/end
    // events on this stream
    MX_HIP(launch_ax_solver(kprec, m->N, b->tiles_ax, b->nt_ax, b->probs, b->epb, s, b->evA,
                            b->evB));
    MX_HIP(hipGraphLaunch(b->graph, s));
    MX_HIP(hipMemcpyAsync(flag, &b->st->done, sizeof(int), hipMemcpyDeviceToHost, s));
    MX_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    MX_HIP(hipEventElapsedTime(&ms, b->evA, b->evB));
    b->ax_ms_sum += ms;
    b->ax_samples += 1;
    if (flag[0]) break;
  }
  MX_HIP(hipMemcpyAsync(&st, b->st, sizeof(State), hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  res->iterations = st.iter;
  res->reason = st.done ? st.reason : MXSEM_MAX_ITER;
  res->res = st.res;
  return MXSEM_OK;
}

// r = b - A64 x  (FP64 operator with FP64 G); returns ||r||_c via host
static int fp64_residual(mxsem_mesh* m, const double* b, const double* x, double* r,
                         double* norm) {
  hipStream_t s = m->ctx->stream;
  MX_TRY(ensure_tmp(m));
  double* w = (r == m->tmpa) ? m->tmpb : m->tmpa;
  MX_TRY(apply_impl(m, MXSEM_F64, x, w, 0, s));
  MX_HIP(launch_residual(b, w, r, m->mult, m->nloc, m->part, m->scal, s));
  double rr = 0.0;
  MX_HIP(hipMemcpyAsync(&rr, m->scal, sizeof(double), hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  *norm = sqrt(rr);
  return MXSEM_OK;
}

static int host_dot64(mxsem_mesh* m, const double* a, const double* b, double* out) {
  hipStream_t s = m->ctx->stream;
  MX_HIP(launch_dot(MXSEM_F64, a, b, m->mult, m->nloc, m->part, m->scal + 1, s));
  MX_HIP(hipMemcpyAsync(out, m->scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
}

}  // namespace mx

using namespace mx;

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
  MX_CHECK(m && r && z, MXSEM_EINVAL, "precond: null argument");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  if (pc == MXSEM_PC_LEARNED) {
    MX_CHECK(m->nn, MXSEM_EINVAL, "precond: no network attached");
    MX_CHECK(io == MXSEM_F32, MXSEM_ENOTSUP, "precond: the learned map takes FP32 vectors");
    return mxsem_nn_forward(m->nn, (const float*)r, (float*)z);
  }
  MX_CHECK(pc == MXSEM_PC_IDENTITY || pc == MXSEM_PC_JACOBI, MXSEM_EINVAL, "precond: unknown pc");
  MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "precond: io must be F64/F32");
  if (io == MXSEM_F32) MX_CHECK(m->dinv32, MXSEM_ENOTSUP, "precond: mesh has no FP32 view");
  const void* dinv = io == MXSEM_F64 ? (const void*)m->dinv64 : (const void*)m->dinv32;
  MX_HIP(launch_precond(io, pc, r, z, dinv, m->nloc, m->ctx->stream));
  return MXSEM_OK;
}

int mxsem_fcg_solve_impl(mxsem_mesh* m, const mxsem_solve_opts* o, const double* b, double* x,
                         mxsem_solve_stats* st);

int mxsem_solve(mxsem_mesh* m, const mxsem_solve_opts* o, const double* b, double* x,
                mxsem_solve_stats* st) {
  MX_CHECK(m && o && b && x && st, MXSEM_EINVAL, "solve: null argument");
  MX_CHECK(o->tol >= 0.0 && o->max_iter >= 1 && o->graph_chunk >= 1, MXSEM_EINVAL,
           "solve: bad tol / max_iter / graph_chunk");
  MX_CHECK(o->mode >= MXSEM_MODE_FP64 && o->mode <= MXSEM_MODE_FP32_ALL, MXSEM_EINVAL,
           "solve: unknown mode");
  MX_CHECK(o->pc == MXSEM_PC_IDENTITY || o->pc == MXSEM_PC_JACOBI || o->pc == MXSEM_PC_LEARNED,
           MXSEM_EINVAL, "solve: unknown preconditioner");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  (void)hipGetLastError();  // clear any stale error left by other libraries
  memset(st, 0, sizeof(*st));
  if (o->method == MXSEM_METHOD_FCG || o->pc == MXSEM_PC_LEARNED)
    return mxsem_fcg_solve_impl(m, o, b, x, st);
  const int mode = o->mode;
  const int vprec = vprec_of_mode(mode);
  const int gprec = gprec_of_mode(mode);
  if (vprec != VP_F64) MX_CHECK(m->G32 || gprec == 2, MXSEM_ENOTSUP, "solve: mesh has no FP32 view");
  if (gprec == 2) MX_CHECK(m->G16, MXSEM_ENOTSUP, "solve: mesh has no BF16 view");
  MX_CHECK(vprec == VP_F64 || m->dinv32, MXSEM_ENOTSUP, "solve: mesh has no FP32 view");
  MX_CHECK(!o->x0_given || mode == MXSEM_MODE_FP64 || mode == MXSEM_MODE_MIXED_IR ||
               mode == MXSEM_MODE_MIXED_IR_BF16G,
           MXSEM_ENOTSUP, "solve: x0 is supported in the FP64 and refinement modes");
  hipStream_t s = m->ctx->stream;
  SolverBufs* buf = nullptr;
  MX_TRY(ensure_bufs(m, vprec, &buf));
  MX_TRY(ensure_tmp(m));
  buf->ax_ms_sum = 0.0;
  buf->ax_samples = 0;
  MX_HIP(hipEventRecord(m->ctx->ev0, s));
  double bnorm = 0.0;
  MX_TRY(host_dot64(m, b, b, &bnorm));
  bnorm = sqrt(bnorm);
  const bool ir = mode == MXSEM_MODE_MIXED_IR || mode == MXSEM_MODE_MIXED_IR_BF16G;
  if (!ir) {
    InnerResult r;
    const double* x0 = nullptr;
    if (o->x0_given) {
      // solve A d = b - A x0 in FP64 and add: equivalent to starting at x0
      double rn = 0.0;
      MX_TRY(fp64_residual(m, b, x, m->tmpa, &rn));
      MX_TRY(run_pcg(m, buf, gprec, o->pc, m->tmpa, 1.0, x0, o->tol * bnorm / (rn > 0 ? rn : 1.0),
                     o->max_iter, o->graph_chunk, o->history, &r));
      MX_HIP(launch_axpy_cast(vprec == VP_F64 ? 0 : 1, x, buf->x, 1.0, 1.0, m->nloc, s));
    } else {
      MX_TRY(run_pcg(m, buf, gprec, o->pc, b, 1.0, nullptr, o->tol, o->max_iter, o->graph_chunk,
                     o->history, &r));
      MX_HIP(launch_axpy_cast(vprec == VP_F64 ? 0 : 1, x, buf->x, 1.0, 0.0, m->nloc, s));
    }
    st->iterations = r.iterations;
    st->reason = r.reason;
    st->rel_res_recursive = r.res;
  } else {
    // FP64 iterative refinement: r = b - A64 x; d = inner MIXED PCG on r/s; x += s d
    if (!o->x0_given) MX_HIP(launch_zero(x, m->nloc, s));
    int total = 0, outer = 0, slow = 0;
    double prev = -1.0;
    st->reason = MXSEM_MAX_ITER;
    for (;;) {
      double rn = 0.0;
      MX_TRY(fp64_residual(m, b, x, m->tmpa, &rn));
      const double rel = bnorm > 0 ? rn / bnorm : 0.0;
      if (rel <= o->tol) {
        st->reason = MXSEM_CONVERGED;
        break;
      }
      if (outer >= o->max_outer || total >= o->max_iter) break;
      if (prev > 0 && rel > 0.5 * prev) ++slow;
      prev = rel;
      if (slow >= 2) {
        // refinement no longer contracts: finish with FP64 PCG from x
        SolverBufs* b64 = nullptr;
        MX_TRY(ensure_bufs(m, VP_F64, &b64));
        InnerResult r;
        MX_TRY(run_pcg(m, b64, 0, o->pc, m->tmpa, 1.0, nullptr, o->tol * bnorm / rn,
                       o->max_iter - total > 0 ? o->max_iter - total : 1, o->graph_chunk, nullptr,
                       &r));
        MX_HIP(launch_axpy_cast(0, x, b64->x, 1.0, 1.0, m->nloc, s));
        total += r.iterations;
        st->fallback_used = 1;
        st->reason = r.reason;
        st->rel_res_recursive = r.res;
        break;
      }
      InnerResult r;
      const double tin = fmax(o->inner_tol, o->tol * bnorm / rn);
      MX_TRY(run_pcg(m, buf, gprec, o->pc, m->tmpa, 1.0 / rn, nullptr, tin,
                     o->max_iter - total, o->graph_chunk, nullptr, &r));
      MX_HIP(launch_axpy_cast(1, x, buf->x, rn, 1.0, m->nloc, s));
      total += r.iterations;
      st->rel_res_recursive = r.res;
      ++outer;
      if (r.reason == MXSEM_BREAKDOWN) {
        st->reason = MXSEM_BREAKDOWN;
        break;
      }
    }
    st->iterations = total;
    st->outer = outer;
  }
  // true FP64 residual
  double rn = 0.0;
  MX_TRY(fp64_residual(m, b, x, m->tmpb, &rn));
  st->rel_res = bnorm > 0 ? rn / bnorm : 0.0;
  MX_HIP(hipEventRecord(m->ctx->ev1, s));
  MX_HIP(hipEventSynchronize(m->ctx->ev1));
  float ms = 0.f;
  MX_HIP(hipEventElapsedTime(&ms, m->ctx->ev0, m->ctx->ev1));
  st->ms = ms;
  st->ax_samples = buf->ax_samples;
  st->ax_ms = buf->ax_samples ? buf->ax_ms_sum / buf->ax_samples : 0.0;
  if (st->reason == MXSEM_BREAKDOWN) {
    set_error("solve: (p, A p) <= 0 or non-finite");
    return MXSEM_EBREAKDOWN;
  }
  return MXSEM_OK;
}

}  // extern "C"
