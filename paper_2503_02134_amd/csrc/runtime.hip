// Host runtime of the mxsem library: errors, context, reference element,
// mesh set-up (geometry, gather-scatter plan, Jacobi diagonal, precision
// views) and the operator-piece entry points.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

// ---------------------------------------------------------------- reference element
// Legendre L_{m}(x) for m = N-1, N, N+1 by the three-term recurrence.
static void legendre3(int N, double x, double* Lm1, double* L, double* Lp1) {
  double a = 1.0, b = x;  // L_0, L_1
  if (N == 0) {
    *Lm1 = 0.0;
    *L = 1.0;
    *Lp1 = x;
    return;
  }
  for (int k = 1; k <= N; ++k) {
    double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  // now a = L_N, b = L_{N+1}; recover L_{N-1} from the recurrence
  // (N+1) L_{N+1} = (2N+1) x L_N - N L_{N-1}
  *L = a;
  *Lp1 = b;
  *Lm1 = ((2.0 * N + 1.0) * x * a - (N + 1.0) * b) / N;
}

// GLL nodes: zeros of q(x) = L_{N+1}(x) - L_{N-1}(x) = (2N+1)/(N(N+1)) (x^2-1) L_N'(x),
// found by Newton with q'(x) = (2N+1) L_N(x), starting from the
// Chebyshev-Gauss-Lobatto points; weights 2 / (N (N+1) L_N(x_i)^2).
void gll_rule(int N, double* xi, double* w) {
  xi[0] = -1.0;
  xi[N] = 1.0;
  for (int j = 1; j < N; ++j) {
    double x = -cos(M_PI * (double)j / (double)N);
    for (int it = 0; it < 200; ++it) {
      double Lm1, L, Lp1;
      legendre3(N, x, &Lm1, &L, &Lp1);
      const double q = Lp1 - Lm1, dq = (2.0 * N + 1.0) * L;
      const double dx = q / dq;
      x -= dx;
      if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) break;
    }
    xi[j] = x;
  }
  std::sort(xi, xi + N + 1);
  for (int j = 0; j <= N; ++j) {
    double Lm1, L, Lp1;
    legendre3(N, xi[j], &Lm1, &L, &Lp1);
    w[j] = 2.0 / (N * (N + 1.0) * L * L);
  }
}

// D[i][j] = l_j'(x_i) from barycentric weights lambda_j = 1/prod_{k!=j}(x_j-x_k);
// the diagonal makes every row sum to zero (derivative of a constant).
void deriv_matrix(int N, const double* xi, double* D) {
  const int n = N + 1;
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (xi[j] - xi[k]);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
      D[i * n + j] = v;
      diag -= v;
    }
    D[i * n + i] = diag;
  }
}

// ---------------------------------------------------------------- helpers
// Elements per workgroup of the operator kernel (workgroups of at most 256
// threads, rounded up to whole wave64s): one wave's worth for the
// two-column mapping, else the smallest count whose idle lanes are under 5%,
// else the count with the fewest idle lanes.
int default_epb(int N) {
  if (ax_wave_elements(N) > 0) return ax_wave_elements(N);  // one wave per workgroup
  const int n2 = (N + 1) * (N + 1);
  int best = 1;
  double bestw = 1.0;
  for (int e = 1; ((e * n2 + 63) / 64) * 64 <= 256; ++e) {
    const int th = ((e * n2 + 63) / 64) * 64;
    const double waste = (double)(th - e * n2) / th;
    if (waste < 0.05) return e;
    if (waste < bestw - 1e-12) {
      bestw = waste;
      best = e;
    }
  }
  return best;
}

// gprec: 0 FP64, 1 FP32, 2 BF16, 3 FP32 (the BF16-direction ablation)
const void* G_ptr(const mxsem_mesh* m, int gprec) {
  return gprec == 0 ? (const void*)m->G64 : gprec == 2 ? (const void*)m->G16 : (const void*)m->G32;
}
const void* hB_ptr(const mxsem_mesh* m, int gprec) {
  if (m->helm_h == 0.0) return nullptr;
  return gprec == 0 ? (const void*)m->hB64 : gprec == 2 ? (const void*)m->hB16 : (const void*)m->hB32;
}

int max_copies(const mxsem_mesh* m) {
  int mx = 1;
  for (int q = 0; q < m->plan.nall; ++q) mx = std::max(mx, m->plan.bk[q].m);
  return mx;
}

int apply_impl(mxsem_mesh* m, int prec, const void* u, void* w, unsigned flags, hipStream_t s) {
  const int gprec = prec;  // 0 F64, 1 F32, 2 BF16 G with FP32 vectors
  const void* D = prec == MXSEM_F64 ? (const void*)m->D64 : (const void*)m->D32;
  MX_HIP(launch_ax_apply(prec, m->N, m->E, m->epb[m->N] > 0 ? m->epb[m->N] : default_epb(m->N),
                         u, w, G_ptr(m, gprec), hB_ptr(m, gprec), D, s, m->cols[m->N]));
  if (!(flags & MXSEM_LOCAL_ONLY)) {
    MX_HIP(launch_gs_apply(prec == MXSEM_F64 ? MXSEM_F64 : MXSEM_F32, MXSEM_F64, w, m->plan, true,
                           s));
  }
  return MXSEM_OK;
}

}  // namespace mx

using namespace mx;

// ================================================================ C ABI
extern "C" {

const char* mxsem_last_error(void) { return get_error(); }
int mxsem_version(void) { return 10000; }

const char* mxsem_status_str(int st) {
  switch (st) {
    case MXSEM_OK: return "ok";
    case MXSEM_EINVAL: return "invalid argument";
    case MXSEM_ENOTSUP: return "not supported";
    case MXSEM_EHIP: return "HIP runtime error";
    case MXSEM_EBREAKDOWN: return "CG breakdown";
    case MXSEM_EINTERNAL: return "internal error";
    case MXSEM_ENOMEM: return "out of memory";
    case MXSEM_EMESH: return "mesh rejected";
    default: return "unknown status";
  }
}

int mxsem_ctx_create(int hip_device, void* hip_stream, mxsem_ctx** out) {
  MX_API_BEGIN
  MX_CHECK(out, MXSEM_EINVAL, "ctx_create: out is null");
  *out = nullptr;
  int ndev = 0;
  MX_HIP(hipGetDeviceCount(&ndev));
  MX_CHECK(hip_device >= 0 && hip_device < ndev, MXSEM_EINVAL, "ctx_create: bad device index");
  MX_HIP(hipSetDevice(hip_device));
  mxsem_ctx* c = new (std::nothrow) mxsem_ctx();
  MX_CHECK(c, MXSEM_ENOMEM, "ctx_create: host allocation failed");
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->pinned_flags, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error(std::string("ctx_create: ") + hipGetErrorString(e));
    mxsem_ctx_destroy(c);
    return MXSEM_EHIP;
  }

  *out = c;
  return MXSEM_OK;
  MX_API_END("mxsem_ctx_create")
}

int mxsem_ctx_destroy(mxsem_ctx* c) {
  MX_API_BEGIN
  if (!c) return MXSEM_OK;
  MX_CHECK(c->live == 0, MXSEM_EINVAL, "ctx_destroy: meshes or batches of this context are alive");
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->capture) (void)hipStreamDestroy(c->capture);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->pinned_flags) (void)hipHostFree(c->pinned_flags);
  delete c;
  return MXSEM_OK;
  MX_API_END("mxsem_ctx_destroy")
}

int mxsem_ctx_set_stream(mxsem_ctx* c, void* hip_stream) {
  MX_API_BEGIN
  MX_CHECK(c, MXSEM_EINVAL, "ctx_set_stream: null ctx");
  c->stream = (hipStream_t)hip_stream;
  return MXSEM_OK;
  MX_API_END("mxsem_ctx_set_stream")
}

int mxsem_gll(int N, double* xi, double* w) {
  MX_API_BEGIN
  MX_CHECK(N >= 1 && N <= MAX_N, MXSEM_ENOTSUP, "gll: N must be in 1..15");
  MX_CHECK(xi && w, MXSEM_EINVAL, "gll: null output");
  gll_rule(N, xi, w);
  return MXSEM_OK;
  MX_API_END("mxsem_gll")
}

int mxsem_mesh_destroy(mxsem_mesh* m) {
  MX_API_BEGIN
  if (!m) return MXSEM_OK;
  if (m->ctx) {
    (void)hipSetDevice(m->ctx->device);
    if (m->ctx->stream) (void)hipStreamSynchronize(m->ctx->stream);
    else (void)hipDeviceSynchronize();
  }
  mesh_drop_plans(m);
  for (int q = 0; q < 4; ++q) delete m->bufs[q];
  delete m->mg;
  if (m->counted) m->ctx->live -= 1;
  delete m;  // the workspace is the caller's
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_destroy")
}

}  // extern "C"

namespace mx {

static int check_desc(const mxsem_mesh_desc* d) {
  MX_CHECK(d->N >= 1 && d->N <= MAX_N, MXSEM_ENOTSUP, "mesh: N must be in 1..15");
  MX_CHECK(d->E >= 1, MXSEM_EINVAL, "mesh: E must be >= 1");
  MX_CHECK(d->xyz && d->glo && d->bnd, MXSEM_EINVAL, "mesh: xyz, glo, bnd required");
  MX_CHECK(d->helm_h >= 0.0 && isfinite(d->helm_h), MXSEM_EINVAL, "mesh: helm_h < 0");
  const int n = d->N + 1;
  MX_CHECK((int64_t)d->E * n * n * n < (int64_t)INT32_MAX - UPD_CHUNK, MXSEM_ENOTSUP,
           "mesh: more than 2^31 local entries");
  MX_CHECK((d->views & ~(MXSEM_VIEW_F64 | MXSEM_VIEW_F32 | MXSEM_VIEW_BF16 | MXSEM_VIEW_MG)) == 0,
           MXSEM_EINVAL, "mesh: unknown view bits");
  if (d->views & MXSEM_VIEW_MG) MX_TRY(mg_check_box(d));
  return MXSEM_OK;
}

static void mesh_basics(mxsem_mesh* m, const mxsem_mesh_desc* d) {
  m->E = d->E;
  m->N = d->N;
  m->n = d->N + 1;
  m->n3 = m->n * m->n * m->n;
  m->nloc = (int64_t)d->E * m->n3;
  m->helm_h = d->helm_h;
  m->views = d->views | MXSEM_VIEW_F64;
  // the vector pass's box assembly indexes with shifts (n a power of two)
  // and float quotients (E < 2^24), and a thread's four entries hold at most
  // one x-face entry (n >= 8)
  const bool pow2 = m->n == 8 || m->n == 16;
  m->box_ne = (pow2 && d->E < (1 << 24)) ? box_lattice_ne(d) : 0;
}

// Gather-scatter plan on the host (a counting sort of the local entries by
// global id): groups bucketed by copy count (8, 4, 2 first, at 16-byte
// aligned offsets so that a group's indices are one vector load), free
// groups before Dirichlet ones, then the Dirichlet list.  Fills m->plan's
// bucket table, m->gs_first, m->ngroups, m->nmask_entries; the index array
// and the per-entry copy counts go to idx and mult.
static int host_plan(const mxsem_mesh_desc* d, mxsem_mesh* m, std::vector<int32_t>& idx,
                     std::vector<uint8_t>& mult) {
  const int64_t nloc = m->nloc;
  const int64_t* glo = d->glo;
  int64_t gmax = -1;
  for (int64_t i = 0; i < nloc; ++i) {
    MX_CHECK(glo[i] >= 0, MXSEM_EINVAL, "mesh: negative global id");
    gmax = std::max(gmax, glo[i]);
  }
  std::vector<int32_t> order(nloc);
  std::vector<int64_t> gstart;  // group boundaries in `order`
  if (gmax < 4 * nloc + 1024) {
    std::vector<int32_t> cnt(gmax + 2, 0);
    for (int64_t i = 0; i < nloc; ++i) cnt[glo[i] + 1]++;
    for (int64_t g = 0; g <= gmax; ++g) cnt[g + 1] += cnt[g];
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < nloc; ++i) order[pos[glo[i]]++] = (int32_t)i;
    for (int64_t g = 0; g <= gmax; ++g)
      if (cnt[g + 1] > cnt[g]) gstart.push_back(cnt[g]);
  } else {
    for (int64_t i = 0; i < nloc; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [glo](int32_t a, int32_t b) { return glo[a] < glo[b]; });
    for (int64_t t = 0; t < nloc; ++t)
      if (t == 0 || glo[order[t]] != glo[order[t - 1]]) gstart.push_back(t);
  }
  gstart.push_back(nloc);
  const int64_t ng = (int64_t)gstart.size() - 1;
  mult.assign(nloc, 0);
  struct Grp {
    int32_t m, first;  // size, position in `order`
  };
  std::vector<std::vector<Grp>> freeb(256), maskb(256);
  std::vector<int32_t> masklist;
  const uint8_t* bnd = d->bnd;
  int64_t ngroups = 0;
  for (int64_t q = 0; q < ng; ++q) {
    const int64_t a = gstart[q], b = gstart[q + 1];
    const int32_t sz = (int32_t)(b - a);
    MX_CHECK(sz <= 255, MXSEM_ENOTSUP, "mesh: a node shared by more than 255 elements");
    const bool msk = bnd[order[a]] != 0;
    for (int64_t t = a; t < b; ++t) {
      const int32_t li = order[t];
      MX_CHECK((bnd[li] != 0) == msk, MXSEM_EMESH,
               "mesh: copies of a global node disagree on the Dirichlet flag");
      mult[li] = (uint8_t)sz;
      if (msk) masklist.push_back(li);
    }
    if (sz >= 2) {
      (msk ? maskb : freeb)[sz].push_back(Grp{sz, (int32_t)a});
      ++ngroups;
    }
  }
  std::sort(masklist.begin(), masklist.end());
  std::vector<int> morder = {8, 4, 2};
  for (int mm = 255; mm >= 2; --mm)
    if (mm != 8 && mm != 4 && mm != 2) morder.push_back(mm);
  idx.clear();
  GsPlan plan{};
  int nb = 0;
  m->gs_first.assign(MAX_BUCKETS, {});
  auto emit = [&](std::vector<std::vector<Grp>>& bks) -> bool {
    for (int mm : morder) {
      auto& gv = bks[mm];
      if (gv.empty()) continue;
      if (nb >= MAX_BUCKETS - 1) return false;
      std::sort(gv.begin(), gv.end(),
                [&order](const Grp& x, const Grp& y) { return order[x.first] < order[y.first]; });
      while (idx.size() % 4) idx.push_back(0);  // 16-byte aligned bucket start
      plan.bk[nb] = GsBucket{mm, (int)gv.size(), (int)idx.size(), 0};
      std::vector<int32_t>& gf = m->gs_first[nb];
      gf.reserve(gv.size());
      for (const Grp& gr : gv) {
        gf.push_back(order[gr.first]);
        for (int t = 0; t < gr.m; ++t) idx.push_back(order[gr.first + t]);
      }
      ++nb;
    }
    return true;
  };
  MX_CHECK(emit(freeb), MXSEM_ENOTSUP, "mesh: too many distinct node multiplicities");
  plan.nfree = nb;
  MX_CHECK(emit(maskb), MXSEM_ENOTSUP, "mesh: too many distinct node multiplicities");
  plan.nall = nb;
  while (idx.size() % 4) idx.push_back(0);
  plan.bk[nb] = GsBucket{0, (int)masklist.size(), (int)idx.size(), 0};
  idx.insert(idx.end(), masklist.begin(), masklist.end());
  m->gs_first[nb] = masklist;
  m->ngroups = ngroups;
  m->nmask_entries = (int)masklist.size();
  plan.n3 = m->n3;
  plan.erank = nullptr;
  m->plan = plan;
  return MXSEM_OK;
}

// Device arrays used only while a mesh is built (inside the blocks of the
// FP64 work vectors, which no solve has touched yet).
struct SetupTemps {
  double *wq = nullptr, *xyz = nullptr, *k = nullptr, *detmin = nullptr;
  size_t begin = 0, end = 0;  // byte range of the workspace they occupy
};

// Every block of a mesh's workspace in one order: mxsem_mesh_workspace_bytes
// reports the total, mxsem_mesh_create (ws != nullptr) points the mesh's
// arrays at the blocks.  Returns the total in bytes.
static size_t mesh_layout(mxsem_mesh* m, size_t nidx, bool has_k, char* ws, SetupTemps* tmp) {
  Layout L;
  const int64_t nl = m->nloc;
  const int n = m->n;
  const bool h = m->helm_h != 0.0;
  const bool f32 = (m->views & MXSEM_VIEW_F32) != 0, b16 = (m->views & MXSEM_VIEW_BF16) != 0;
  auto put = [&](auto** p, size_t bytes) {
    const size_t o = L.take(bytes);
    if (ws) *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(ws + o);
  };
  put(&m->D64, sizeof(double) * n * n);
  put(&m->D32, sizeof(float) * n * n);
  put(&m->G64, sizeof(double) * 6 * nl);
  put(&m->B64, sizeof(double) * nl);
  if (h) put(&m->hB64, sizeof(double) * nl);
  put(&m->dinv64, sizeof(double) * nl);
  put(&m->mult, (size_t)nl);
  put(&m->gs_idx, sizeof(int) * std::max<size_t>(nidx, 4));
  put(&m->part, sizeof(double) * ((nl + UPD_CHUNK - 1) / UPD_CHUNK + 64));
  put(&m->scal, sizeof(double) * 8);
  put(&m->tmpa, sizeof(double) * nl);
  put(&m->tmpb, sizeof(double) * nl);
  put(&m->erank, sizeof(int) * (size_t)m->E);
  if (f32 || b16) put(&m->dinv32, sizeof(float) * nl);
  if (f32) {
    put(&m->G32, sizeof(float) * 6 * nl);
    if (h) put(&m->hB32, sizeof(float) * nl);
  }
  if (b16) {
    put(&m->G16, sizeof(bf16_t) * 6 * nl);
    if (h) put(&m->hB16, sizeof(bf16_t) * nl);
  }
  const size_t work = align256(L.total);
  carve_solver_bufs(m, VP_F64, ws, L);
  if (f32 || b16) {
    carve_solver_bufs(m, VP_F32, ws, L);
    if (ws) {  // the FP32-sums ablation runs on the same vectors
      m->bufs[VP_F32ACC] = new SolverBufs(*m->bufs[VP_F32]);
      m->bufs[VP_F32ACC]->vprec = VP_F32ACC;
    }
  }
  {
    Layout T;
    T.total = work;
    const size_t owq = T.take(sizeof(double) * n), oxyz = T.take(sizeof(double) * 3 * nl);
    const size_t ok = has_k ? T.take(sizeof(double) * nl) : 0;
    const size_t odet = T.take(sizeof(double) * ((nl + 255) / 256));
    if (ws && tmp) {
      tmp->begin = work;
      tmp->end = T.total;
      tmp->wq = (double*)(ws + owq);
      tmp->xyz = (double*)(ws + oxyz);
      tmp->k = has_k ? (double*)(ws + ok) : nullptr;
      tmp->detmin = (double*)(ws + odet);
    }
    L.total = std::max(L.total, T.total);
  }
  if (m->views & MXSEM_VIEW_MG) {
    if (ws && !m->mg) m->mg = new MgData();
    mg_layout(m, ws, L);
  }
  const size_t tb = plan_table_bytes(&m, 1);
  const int vps[3] = {VP_F64, VP_F32, VP_F32ACC};
  for (int q = 0; q < ((f32 || b16) ? 3 : 1); ++q) {
    const size_t o = L.take(tb);
    if (ws) {
      m->plan_tables[vps[q]].base = ws + o;
      m->plan_tables[vps[q]].size = tb;
    }
  }
  return align256(L.total);
}

__global__ void ws_zero_kernel(uint4* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace mx

extern "C" {

int mxsem_mesh_workspace_bytes(const mxsem_mesh_desc* d, size_t* bytes) {
  MX_API_BEGIN
  MX_CHECK(d && bytes, MXSEM_EINVAL, "mesh_workspace_bytes: null argument");
  MX_TRY(check_desc(d));
  mxsem_mesh tmp;
  mesh_basics(&tmp, d);
  std::vector<int32_t> idx;
  std::vector<uint8_t> mult;
  MX_TRY(host_plan(d, &tmp, idx, mult));
  *bytes = mesh_layout(&tmp, idx.size(), d->kcoef != nullptr, nullptr, nullptr);
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_workspace_bytes")
}

static int mesh_fail(mxsem_mesh* m, int rc) {
  mxsem_mesh_destroy(m);
  return rc;
}

#define MX_MTRY(call)                       \
  do {                                      \
    int rc_ = (call);                       \
    if (rc_ != MXSEM_OK) return mesh_fail(m, rc_); \
  } while (0)
#define MX_MHIP(call)                                                     \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));      \
      return mesh_fail(m, MXSEM_EHIP);                                    \
    }                                                                     \
  } while (0)
#define MX_MCHECK(cond, code, msg) \
  do {                             \
    if (!(cond)) {                 \
      set_error(msg);              \
      return mesh_fail(m, code);   \
    }                              \
  } while (0)

int mxsem_mesh_create(mxsem_ctx* ctx, const mxsem_mesh_desc* d, void* workspace, size_t ws_bytes,
                      mxsem_mesh** out) {
  MX_API_BEGIN
  // every argument is checked before the device is touched
  MX_CHECK(d && out, MXSEM_EINVAL, "mesh_create: null argument");
  *out = nullptr;
  MX_TRY(check_desc(d));
  MX_CHECK(workspace && ((uintptr_t)workspace & 255) == 0, MXSEM_EINVAL,
           "mesh_create: workspace must be a 256-byte aligned device pointer");
  std::unique_ptr<mxsem_mesh> mh(new mxsem_mesh());
  mesh_basics(mh.get(), d);
  // gather-scatter plan (host) and the workspace layout it implies
  std::vector<int32_t> idx;
  std::vector<uint8_t> mult;
  MX_TRY(host_plan(d, mh.get(), idx, mult));
  const size_t need = mesh_layout(mh.get(), idx.size(), d->kcoef != nullptr, nullptr, nullptr);
  MX_CHECK(ws_bytes >= need, MXSEM_EINVAL,
           "mesh_create: workspace smaller than mxsem_mesh_workspace_bytes");
  MX_CHECK(ctx, MXSEM_EINVAL, "mesh_create: null context");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  mxsem_mesh* m = mh.release();
  m->ctx = ctx;
  const int n = m->n;
  const int64_t nloc = m->nloc;
  hipStream_t s = ctx->stream;
  SetupTemps tmp;
  m->ws = (char*)workspace;
  m->ws_bytes = ws_bytes;
  mesh_layout(m, idx.size(), d->kcoef != nullptr, m->ws, &tmp);
  {
    const int64_t n16 = (int64_t)(need / 16);
    hipLaunchKernelGGL(ws_zero_kernel, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 65536)),
                       dim3(256), 0, s, (uint4*)m->ws, n16);
    MX_MHIP(hipGetLastError());
  }

  // reference element
  std::vector<double> xi(n), wq(n), D(n * n);
  gll_rule(d->N, xi.data(), wq.data());
  deriv_matrix(d->N, xi.data(), D.data());
  std::vector<float> D32h(n * n);
  for (int q = 0; q < n * n; ++q) D32h[q] = (float)D[q];
  MX_MHIP(hipMemcpyAsync(m->D64, D.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(m->D32, D32h.data(), sizeof(float) * n * n, hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(tmp.wq, wq.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));

  // geometry (FP64, on the device)
  MX_MHIP(hipMemcpyAsync(tmp.xyz, d->xyz, sizeof(double) * 3 * nloc, hipMemcpyHostToDevice, s));
  if (d->kcoef)
    MX_MHIP(hipMemcpyAsync(tmp.k, d->kcoef, sizeof(double) * nloc, hipMemcpyHostToDevice, s));
  int nbg = 0;
  MX_MHIP(launch_geom(m->E, n, tmp.xyz, m->D64, tmp.wq, tmp.k, m->G64, m->B64, tmp.detmin, &nbg, s));
  std::vector<double> detmin(nbg);
  MX_MHIP(hipMemcpyAsync(detmin.data(), tmp.detmin, sizeof(double) * nbg, hipMemcpyDeviceToHost, s));
  MX_MHIP(hipStreamSynchronize(s));
  double mn = INFINITY;
  for (double v : detmin) mn = fmin(mn, v);
  m->min_det = mn;
  MX_MCHECK(mn > 0.0, MXSEM_EMESH, "mesh_create: non-positive Jacobian determinant");

  // gather-scatter plan and copy counts to the device
  if (!idx.empty())
    MX_MHIP(hipMemcpyAsync(m->gs_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(m->mult, mult.data(), nloc, hipMemcpyHostToDevice, s));
  m->plan.idx = m->gs_idx;

  // Helmholtz term h*B
  if (m->helm_h != 0.0) MX_MHIP(launch_scale(m->hB64, m->B64, m->helm_h, nloc, s));

  // Jacobi: assembled diagonal (FP64), inverse, zero on Dirichlet entries
  MX_MHIP(launch_diag(m->E, n, m->G64, m->B64, m->helm_h, m->D64, m->dinv64, s));
  MX_MHIP(launch_gs_apply(MXSEM_F64, MXSEM_F64, m->dinv64, m->plan, false, s));
  MX_MHIP(launch_invert(m->dinv64, nloc, s));
  {
    GsPlan only_mask = m->plan;  // zero the Dirichlet entries only
    only_mask.nfree = 0;
    MX_MHIP(launch_gs_apply(MXSEM_F64, MXSEM_F64, m->dinv64, only_mask, true, s));
  }

  // lower-precision views (one-time casts)
  if (m->dinv32) MX_MHIP(launch_cast_f32(m->dinv32, m->dinv64, nloc, s));
  if (m->G32) {
    MX_MHIP(launch_cast_g_split(1, m->G32, m->G64, m->E, m->n3, s));
    if (m->hB32) MX_MHIP(launch_cast_f32(m->hB32, m->hB64, nloc, s));
  }
  if (m->G16) {
    MX_MHIP(launch_cast_g_split(2, m->G16, m->G64, m->E, m->n3, s));
    if (m->hB16) MX_MHIP(launch_cast_bf16(m->hB16, m->hB64, nloc, s));
  }
  if (m->mg) MX_MTRY(mg_setup(m, d, s));
  // the set-up temporaries sat in the FP64 work vectors: clear them again
  {
    const size_t end = std::max(tmp.end, (size_t)((char*)m->bufs[VP_F64]->part_ax - m->ws));
    const int64_t n16 = (int64_t)((align256(end) - tmp.begin) / 16);
    hipLaunchKernelGGL(ws_zero_kernel, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 65536)),
                       dim3(256), 0, s, (uint4*)(m->ws + tmp.begin), n16);
    MX_MHIP(hipGetLastError());
  }
  MX_MHIP(hipStreamSynchronize(s));
  for (int q = 0; q < 16; ++q) m->epb[q] = m->cols[q] = 0;
  ctx->live += 1;
  m->counted = true;
  *out = m;
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_create")
}

int mxsem_mesh_info(const mxsem_mesh* m, int64_t* nloc, int64_t* ngroups, int64_t* nmasked,
                    double* min_detj) {
  MX_API_BEGIN
  MX_CHECK(m, MXSEM_EINVAL, "mesh_info: null mesh");
  if (nloc) *nloc = m->nloc;
  if (ngroups) *ngroups = m->ngroups;
  if (nmasked) *nmasked = m->nmask_entries;
  if (min_detj) *min_detj = m->min_det;
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_info")
}

int mxsem_mesh_get(const mxsem_mesh* m, int what, double* out) {
  MX_API_BEGIN
  MX_CHECK(m && out, MXSEM_EINVAL, "mesh_get: null argument");
  hipStream_t s = m->ctx->stream;
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  switch (what) {
    case 0: MX_HIP(hipMemcpyAsync(out, m->G64, sizeof(double) * 6 * m->nloc, hipMemcpyDeviceToHost, s)); break;
    case 1: MX_HIP(hipMemcpyAsync(out, m->B64, sizeof(double) * m->nloc, hipMemcpyDeviceToHost, s)); break;
    case 2:
    case 4: {
      std::vector<uint8_t> mu(m->nloc);
      MX_HIP(hipMemcpyAsync(mu.data(), m->mult, m->nloc, hipMemcpyDeviceToHost, s));
      MX_HIP(hipStreamSynchronize(s));
      if (what == 2) {
        for (int64_t i = 0; i < m->nloc; ++i) out[i] = 1.0 / mu[i];
      } else {
        std::vector<int32_t> idx(m->nmask_entries);
        if (m->nmask_entries)
          MX_HIP(hipMemcpy(idx.data(), m->gs_idx + m->plan.bk[m->plan.nall].off,
                           sizeof(int) * m->nmask_entries, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < m->nloc; ++i) out[i] = 0.0;
        for (int32_t i : idx) out[i] = 1.0;
      }
      return MXSEM_OK;
    }
    case 3: MX_HIP(hipMemcpyAsync(out, m->dinv64, sizeof(double) * m->nloc, hipMemcpyDeviceToHost, s)); break;
    case 5: MX_HIP(hipMemcpyAsync(out, m->D64, sizeof(double) * m->n * m->n, hipMemcpyDeviceToHost, s)); break;
    default: MX_CHECK(false, MXSEM_EINVAL, "mesh_get: unknown field");
  }
  MX_HIP(hipStreamSynchronize(s));
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_get")
}

static int check_prec_view(const mxsem_mesh* m, int prec) {
  MX_CHECK(prec >= MXSEM_F64 && prec <= MXSEM_BF16G_F32, MXSEM_EINVAL, "unknown precision");
  if (prec == MXSEM_F32) MX_CHECK(m->G32, MXSEM_ENOTSUP, "mesh has no FP32 view");
  if (prec == MXSEM_BF16G_F32) MX_CHECK(m->G16, MXSEM_ENOTSUP, "mesh has no BF16 view");
  return MXSEM_OK;
}

int mxsem_apply(mxsem_mesh* m, mxsem_prec io, const void* u, void* w, unsigned flags) {
  MX_API_BEGIN
  MX_CHECK(m && u && w, MXSEM_EINVAL, "apply: null argument");
  MX_CHECK(u != w, MXSEM_EINVAL, "apply: u and w must not alias");
  MX_TRY(check_prec_view(m, io));
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  return apply_impl(m, io, u, w, flags, m->ctx->stream);
  MX_API_END("mxsem_apply")
}

int mxsem_gather_scatter(mxsem_mesh* m, mxsem_prec io, mxsem_prec acc, void* v, unsigned flags) {
  MX_API_BEGIN
  MX_CHECK(m && v, MXSEM_EINVAL, "gather_scatter: null argument");
  MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "gather_scatter: io must be F64/F32");
  MX_CHECK(acc == MXSEM_F64 || acc == MXSEM_F32, MXSEM_EINVAL, "gather_scatter: acc must be F64/F32");
  const bool pairwise = (flags & MXSEM_GS_PAIRWISE) != 0;
  if (pairwise) {
    MX_CHECK(io == MXSEM_F32, MXSEM_ENOTSUP, "gather_scatter: pairwise order takes FP32 vectors");
    MX_CHECK(max_copies(m) <= GS_PAIRWISE_MAXM, MXSEM_ENOTSUP,
             "gather_scatter: pairwise order takes at most 16 copies per node");
  }
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  MX_HIP(launch_gs_apply(io, acc, v, m->plan, (flags & MXSEM_MASK) != 0, m->ctx->stream,
                         pairwise));
  return MXSEM_OK;
  MX_API_END("mxsem_gather_scatter")
}

int mxsem_dot(mxsem_mesh* m, mxsem_prec io, const void* a, const void* b, double* out_dev) {
  MX_API_BEGIN
  MX_CHECK(m && a && b && out_dev, MXSEM_EINVAL, "dot: null argument");
  MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "dot: io must be F64/F32");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  MX_HIP(launch_dot(io, a, b, m->mult, m->nloc, m->part, out_dev, m->ctx->stream));
  return MXSEM_OK;
  MX_API_END("mxsem_dot")
}

int mxsem_dot_ex(mxsem_mesh* m, mxsem_prec io, int acc, const void* a, const void* b,
                 double* out_dev) {
  MX_API_BEGIN
  MX_CHECK(m && a && b && out_dev, MXSEM_EINVAL, "dot_ex: null argument");
  MX_CHECK(io == MXSEM_F64 || io == MXSEM_F32, MXSEM_EINVAL, "dot_ex: io must be F64/F32");
  MX_CHECK(acc >= MXSEM_DOT_DEFAULT && acc <= MXSEM_DOT_DOT2, MXSEM_EINVAL,
           "dot_ex: unknown accumulation");
  const int dm = dot_mode_of(acc, DOT_F64);
  MX_CHECK(io == MXSEM_F32 || dm == DOT_F64, MXSEM_ENOTSUP,
           "dot_ex: FP32 and Dot2 accumulation take FP32 vectors");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  MX_HIP(launch_dot(io, a, b, m->mult, m->nloc, m->part, out_dev, m->ctx->stream, dm));
  return MXSEM_OK;
  MX_API_END("mxsem_dot_ex")
}

int mxsem_stream_copy(mxsem_ctx* ctx, const void* src, void* dst, size_t bytes) {
  MX_API_BEGIN
  MX_CHECK(ctx && src && dst, MXSEM_EINVAL, "stream_copy: null argument");
  MX_CHECK(bytes % 16 == 0 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0,
           MXSEM_EINVAL, "stream_copy: pointers and size must be multiples of 16 bytes");
  MX_CHECK((const char*)src + bytes <= (const char*)dst || (const char*)dst + bytes <= (const char*)src,
           MXSEM_EINVAL, "stream_copy: buffers overlap");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  if (bytes) MX_HIP(launch_stream_copy(src, dst, (int64_t)(bytes / 16), ctx->stream));
  return MXSEM_OK;
  MX_API_END("mxsem_stream_copy")
}

int mxsem_stream_mix(mxsem_ctx* ctx, const void* src, size_t read_bytes, void* dst,
                     size_t write_bytes) {
  MX_API_BEGIN
  MX_CHECK(ctx && src && dst, MXSEM_EINVAL, "stream_mix: null argument");
  MX_CHECK(write_bytes > 0 && write_bytes % 16 == 0 && read_bytes % write_bytes == 0 &&
               ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0,
           MXSEM_EINVAL,
           "stream_mix: 16-byte aligned pointers, write_bytes a positive multiple of 16 and "
           "read_bytes a multiple of write_bytes");
  const size_t k = read_bytes / write_bytes;
  MX_CHECK(k == 1 || k == 2 || k == 4 || k == 8, MXSEM_EINVAL,
           "stream_mix: read_bytes / write_bytes must be 1, 2, 4 or 8");
  MX_CHECK((const char*)src + read_bytes <= (const char*)dst ||
               (const char*)dst + write_bytes <= (const char*)src,
           MXSEM_EINVAL, "stream_mix: buffers overlap");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  MX_HIP(launch_stream_mix(src, dst, (int64_t)(write_bytes / 16), (int)k, ctx->stream));
  return MXSEM_OK;
  MX_API_END("mxsem_stream_mix")
}

int mxsem_mesh_set_ranks(mxsem_mesh* m, const int32_t* rank_host) {
  MX_API_BEGIN
  MX_CHECK(m, MXSEM_EINVAL, "set_ranks: null mesh");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  if (!rank_host) {
    m->plan.erank = nullptr;
    return MXSEM_OK;
  }
  for (int e = 0; e < m->E; ++e)
    MX_CHECK(rank_host[e] >= 0, MXSEM_EINVAL, "set_ranks: ranks must be >= 0");
  hipStream_t s = m->ctx->stream;
  MX_HIP(hipStreamSynchronize(s));  // no queued work may still read the old ranks
  MX_HIP(hipMemcpy(m->erank, rank_host, sizeof(int) * (size_t)m->E, hipMemcpyHostToDevice));
  m->plan.erank = m->erank;
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_set_ranks")
}

int mxsem_mass_rhs(mxsem_mesh* m, const double* f, double* b) {
  MX_API_BEGIN
  MX_CHECK(m && f && b, MXSEM_EINVAL, "mass_rhs: null argument");
  MX_HIP(hipSetDevice(m->ctx->device));
  (void)hipGetLastError();
  hipStream_t s = m->ctx->stream;
  MX_HIP(launch_mass(m->B64, f, b, m->nloc, s));
  MX_HIP(launch_gs_apply(MXSEM_F64, MXSEM_F64, b, m->plan, true, s));
  return MXSEM_OK;
  MX_API_END("mxsem_mass_rhs")
}

}  // extern "C"
