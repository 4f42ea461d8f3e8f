// Host runtime of the mxsem library: errors, context, reference element,
// mesh set-up (geometry, gather-scatter plan, Jacobi diagonal, precision
// views) and the operator-piece entry points.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
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
int mesh_alloc(mxsem_mesh* m, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    return MXSEM_ENOMEM;
  }
  m->allocs.push_back(*p);
  return MXSEM_OK;
}

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

int ensure_tmp(mxsem_mesh* m) {
  if (!m->tmpa) {
    MX_TRY(mesh_alloc(m, (void**)&m->tmpa, sizeof(double) * m->nloc));
    MX_TRY(mesh_alloc(m, (void**)&m->tmpb, sizeof(double) * m->nloc));
  }
  return MXSEM_OK;
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
                         u, w, G_ptr(m, gprec), hB_ptr(m, gprec), D, s));
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
    delete c;
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
  (void)hipSetDevice(m->ctx->device);
  if (m->ctx->stream) (void)hipStreamSynchronize(m->ctx->stream);
  else (void)hipDeviceSynchronize();
  mesh_drop_plans(m);
  for (int q = 0; q < 4; ++q) delete m->bufs[q];
  for (void* p : m->allocs) (void)hipFree(p);
  if (m->counted) m->ctx->live -= 1;
  delete m;
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_destroy")
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

int mxsem_mesh_create(mxsem_ctx* ctx, const mxsem_mesh_desc* d, mxsem_mesh** out) {
  MX_API_BEGIN
  MX_CHECK(ctx && d && out, MXSEM_EINVAL, "mesh_create: null argument");
  *out = nullptr;
  MX_CHECK(d->N >= 1 && d->N <= MAX_N, MXSEM_ENOTSUP, "mesh_create: N must be in 1..15");
  MX_CHECK(d->E >= 1, MXSEM_EINVAL, "mesh_create: E must be >= 1");
  MX_CHECK(d->xyz && d->glo && d->bnd, MXSEM_EINVAL, "mesh_create: xyz, glo, bnd required");
  MX_CHECK(d->helm_h >= 0.0 && isfinite(d->helm_h), MXSEM_EINVAL, "mesh_create: helm_h < 0");
  const int n = d->N + 1, n3 = n * n * n;
  const int64_t nloc = (int64_t)d->E * n3;
  MX_CHECK(nloc < (int64_t)INT32_MAX - UPD_CHUNK, MXSEM_ENOTSUP,
           "mesh_create: more than 2^31 local entries");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  mxsem_mesh* m = new (std::nothrow) mxsem_mesh();
  MX_CHECK(m, MXSEM_ENOMEM, "mesh_create: host allocation failed");
  m->ctx = ctx;
  m->E = d->E;
  m->N = d->N;
  m->n = n;
  m->n3 = n3;
  m->nloc = nloc;
  m->helm_h = d->helm_h;
  m->views = d->views | MXSEM_VIEW_F64;
  hipStream_t s = ctx->stream;

  // reference element
  std::vector<double> xi(n), wq(n), D(n * n);
  gll_rule(d->N, xi.data(), wq.data());
  deriv_matrix(d->N, xi.data(), D.data());
  std::vector<float> D32h(n * n);
  for (int q = 0; q < n * n; ++q) D32h[q] = (float)D[q];
  double* wq_d;
  MX_MTRY(mesh_alloc(m, (void**)&m->D64, sizeof(double) * n * n));
  MX_MTRY(mesh_alloc(m, (void**)&m->D32, sizeof(float) * n * n));
  MX_MTRY(mesh_alloc(m, (void**)&wq_d, sizeof(double) * n));
  MX_MHIP(hipMemcpyAsync(m->D64, D.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(m->D32, D32h.data(), sizeof(float) * n * n, hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(wq_d, wq.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));

  // geometry (FP64, on the device)
  double *xyz_d = nullptr, *k_d = nullptr, *detmin_d = nullptr;
  MX_MTRY(mesh_alloc(m, (void**)&xyz_d, sizeof(double) * 3 * nloc));
  MX_MHIP(hipMemcpyAsync(xyz_d, d->xyz, sizeof(double) * 3 * nloc, hipMemcpyHostToDevice, s));
  if (d->kcoef) {
    MX_MTRY(mesh_alloc(m, (void**)&k_d, sizeof(double) * nloc));
    MX_MHIP(hipMemcpyAsync(k_d, d->kcoef, sizeof(double) * nloc, hipMemcpyHostToDevice, s));
  }
  MX_MTRY(mesh_alloc(m, (void**)&m->G64, sizeof(double) * 6 * nloc));
  MX_MTRY(mesh_alloc(m, (void**)&m->B64, sizeof(double) * nloc));
  const int nb_geom = (int)((nloc + 255) / 256);
  MX_MTRY(mesh_alloc(m, (void**)&detmin_d, sizeof(double) * nb_geom));
  int nbg = 0;
  MX_MHIP(launch_geom(m->E, n, xyz_d, m->D64, wq_d, k_d, m->G64, m->B64, detmin_d, &nbg, s));
  std::vector<double> detmin(nbg);
  MX_MHIP(hipMemcpyAsync(detmin.data(), detmin_d, sizeof(double) * nbg, hipMemcpyDeviceToHost, s));
  MX_MHIP(hipStreamSynchronize(s));
  double mn = INFINITY;
  for (double v : detmin) mn = fmin(mn, v);
  m->min_det = mn;
  MX_MCHECK(mn > 0.0, MXSEM_EMESH, "mesh_create: non-positive Jacobian determinant");

  // gather-scatter plan (host): counting sort of local entries by global id
  const int64_t* glo = d->glo;
  int64_t gmax = -1;
  for (int64_t i = 0; i < nloc; ++i) {
    MX_MCHECK(glo[i] >= 0, MXSEM_EINVAL, "mesh_create: negative global id");
    gmax = std::max(gmax, glo[i]);
  }
  std::vector<int32_t> order(nloc);
  std::vector<int64_t> gstart;  // group boundaries in `order`
  {
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
  }
  const int64_t ng = (int64_t)gstart.size() - 1;
  std::vector<uint8_t> mult(nloc);
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
    MX_MCHECK(sz <= 255, MXSEM_ENOTSUP, "mesh_create: a node shared by more than 255 elements");
    const bool msk = bnd[order[a]] != 0;
    for (int64_t t = a; t < b; ++t) {
      const int32_t li = order[t];
      MX_MCHECK((bnd[li] != 0) == msk, MXSEM_EMESH,
                "mesh_create: copies of a global node disagree on the Dirichlet flag");
      mult[li] = (uint8_t)sz;
      if (msk) masklist.push_back(li);
    }
    if (sz >= 2) {
      (msk ? maskb : freeb)[sz].push_back(Grp{sz, (int32_t)a});
      ++ngroups;
    }
  }
  std::sort(masklist.begin(), masklist.end());
  // bucket order: 8, 4, 2 (vector index loads), then every other m descending
  std::vector<int> morder = {8, 4, 2};
  for (int mm = 255; mm >= 2; --mm)
    if (mm != 8 && mm != 4 && mm != 2) morder.push_back(mm);
  std::vector<int32_t> idx;
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
  MX_MCHECK(emit(freeb), MXSEM_ENOTSUP, "mesh_create: too many distinct node multiplicities");
  plan.nfree = nb;
  MX_MCHECK(emit(maskb), MXSEM_ENOTSUP, "mesh_create: too many distinct node multiplicities");
  plan.nall = nb;
  while (idx.size() % 4) idx.push_back(0);
  plan.bk[nb] = GsBucket{0, (int)masklist.size(), (int)idx.size(), 0};
  idx.insert(idx.end(), masklist.begin(), masklist.end());
  m->gs_first[nb] = masklist;
  m->ngroups = ngroups;
  m->nmask_entries = (int)masklist.size();
  MX_MTRY(mesh_alloc(m, (void**)&m->gs_idx, sizeof(int) * std::max<size_t>(idx.size(), 4)));
  MX_MTRY(mesh_alloc(m, (void**)&m->mult, nloc));
  if (!idx.empty())
    MX_MHIP(hipMemcpyAsync(m->gs_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, s));
  MX_MHIP(hipMemcpyAsync(m->mult, mult.data(), nloc, hipMemcpyHostToDevice, s));
  plan.idx = m->gs_idx;
  plan.n3 = m->n3;
  plan.erank = nullptr;
  m->plan = plan;

  // scratch
  const int64_t nbu = (nloc + UPD_CHUNK - 1) / UPD_CHUNK;
  MX_MTRY(mesh_alloc(m, (void**)&m->part, sizeof(double) * (nbu + 64)));
  MX_MTRY(mesh_alloc(m, (void**)&m->scal, sizeof(double) * 8));

  // Helmholtz term h*B
  if (m->helm_h != 0.0) {
    MX_MTRY(mesh_alloc(m, (void**)&m->hB64, sizeof(double) * nloc));
    MX_MHIP(launch_scale(m->hB64, m->B64, m->helm_h, nloc, s));
  }

  // Jacobi: assembled diagonal (FP64), inverse, zero on Dirichlet entries
  MX_MTRY(mesh_alloc(m, (void**)&m->dinv64, sizeof(double) * nloc));
  MX_MHIP(launch_diag(m->E, n, m->G64, m->B64, m->helm_h, m->D64, m->dinv64, s));
  MX_MHIP(launch_gs_apply(MXSEM_F64, MXSEM_F64, m->dinv64, m->plan, false, s));
  MX_MHIP(launch_invert(m->dinv64, nloc, s));
  {
    GsPlan only_mask = m->plan;  // zero the Dirichlet entries only
    only_mask.nfree = 0;
    MX_MHIP(launch_gs_apply(MXSEM_F64, MXSEM_F64, m->dinv64, only_mask, true, s));
  }

  // lower-precision views (one-time casts)
  if (m->views & (MXSEM_VIEW_F32 | MXSEM_VIEW_BF16)) {
    MX_MTRY(mesh_alloc(m, (void**)&m->dinv32, sizeof(float) * nloc));
    MX_MHIP(launch_cast_f32(m->dinv32, m->dinv64, nloc, s));
  }
  if (m->views & MXSEM_VIEW_F32) {
    MX_MTRY(mesh_alloc(m, (void**)&m->G32, sizeof(float) * 6 * nloc));
    MX_MHIP(launch_cast_g_split(1, m->G32, m->G64, m->E, n * n * n, s));
    if (m->hB64) {
      MX_MTRY(mesh_alloc(m, (void**)&m->hB32, sizeof(float) * nloc));
      MX_MHIP(launch_cast_f32(m->hB32, m->hB64, nloc, s));
    }
  }
  if (m->views & MXSEM_VIEW_BF16) {
    MX_MTRY(mesh_alloc(m, (void**)&m->G16, sizeof(bf16_t) * 6 * nloc));
    MX_MHIP(launch_cast_g_split(2, m->G16, m->G64, m->E, n * n * n, s));
    if (m->hB64) {
      MX_MTRY(mesh_alloc(m, (void**)&m->hB16, sizeof(bf16_t) * nloc));
      MX_MHIP(launch_cast_bf16(m->hB16, m->hB64, nloc, s));
    }
  }
  MX_MHIP(hipStreamSynchronize(s));
  // the coordinates and k are no longer needed on the device
  for (void* p : {(void*)xyz_d, (void*)k_d, (void*)detmin_d}) {
    if (!p) continue;
    (void)hipFree(p);
    m->allocs.erase(std::find(m->allocs.begin(), m->allocs.end(), p));
  }
  for (int q = 0; q < 16; ++q) m->epb[q] = 0;
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
  if (!m->erank) MX_TRY(mesh_alloc(m, (void**)&m->erank, sizeof(int) * (size_t)m->E));
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
