// Autotuner for the operator kernel's tile (elements per workgroup) and
// thread mapping, and the per-mesh tuning entry point.  Candidates are every
// elements-per-workgroup count whose workgroup fits 256 threads, with one
// (i,j) column per thread and, where that kernel exists (N = 5, 9 with FP32
// vectors), with two; each is timed with HIP events over repeated launches
// on synthetic data of the requested (N, E, precision), and the fastest
// wins.
#include <math.h>
#include <stdio.h>

#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace mx {

__global__ void fill_pattern_kernel(float* __restrict__ a, int64_t n, float base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = base + 1e-3f * (float)(i % 977);
}

// Synthetic operator data of the tuning run as blocks of a workspace: u, w,
// G (six factors per node) and D.
struct TuneBlocks {
  size_t u, w, G, D, total;
};
static TuneBlocks tune_blocks(int N, int E, int prec) {
  const int n = N + 1;
  const int64_t nloc = (int64_t)E * n * n * n;
  const size_t vb = prec == MXSEM_F64 ? 8 : 4;
  const size_t gb = prec == MXSEM_F64 ? 8 : prec == MXSEM_F32 ? 4 : 2;
  Layout L;
  TuneBlocks t;
  t.u = L.take(vb * nloc);
  t.w = L.take(vb * nloc);
  t.G = L.take(gb * 6 * nloc);
  t.D = L.take(8 * n * n);
  t.total = align256(L.total);
  return t;
}
size_t autotune_bytes(int N, int E, int prec) { return tune_blocks(N, E, prec).total; }

int autotune_epb(int device, hipStream_t s, int N, int E, int prec, char* ws, int* best_epb,
                 int* best_cols) {
  const int n = N + 1, n3 = n * n * n;
  const int64_t nloc = (int64_t)E * n3;
  const size_t vb = prec == MXSEM_F64 ? 8 : 4;
  const size_t gb = prec == MXSEM_F64 ? 8 : prec == MXSEM_F32 ? 4 : 2;
  const TuneBlocks tb = tune_blocks(N, E, prec);
  void *u = ws + tb.u, *w = ws + tb.w, *G = ws + tb.G, *D = ws + tb.D;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MXSEM_OK;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    set_error("autotune: event creation failed");
    return MXSEM_EHIP;
  }
  // finite synthetic data (values do not affect the timing)
  const size_t words_u = vb * nloc / 4, words_G = gb * 6 * nloc / 4, words_D = 8 * n * n / 4;
  hipLaunchKernelGGL(fill_pattern_kernel, dim3((unsigned)((words_u + 255) / 256)), dim3(256), 0, s,
                     (float*)u, (int64_t)words_u, 0.5f);
  hipLaunchKernelGGL(fill_pattern_kernel, dim3((unsigned)((words_G + 255) / 256)), dim3(256), 0, s,
                     (float*)G, (int64_t)words_G, 0.25f);
  hipLaunchKernelGGL(fill_pattern_kernel, dim3((unsigned)((words_D + 255) / 256)), dim3(256), 0, s,
                     (float*)D, (int64_t)words_D, 0.125f);
  float best = INFINITY;
  *best_epb = default_epb(N);
  *best_cols = 0;
  // the two-column kernel exists for FP32 vectors (FP32 or BF16 G) at N = 5, 9
  const bool two = prec != MXSEM_F64 && ax_wave_elements(N) > 0;
  for (int cols = 1; cols <= (two ? 2 : 1); ++cols) {
    const int emax = cols == 2 ? std::min(max_epb(N), max_epb2(N)) : max_epb(N);
    for (int epb = 1; epb <= emax; ++epb) {
      for (int r = 0; r < 2; ++r) {
        if (launch_ax_apply(prec, N, E, epb, u, w, G, nullptr, D, s, cols) != hipSuccess) {
          cleanup();
          set_error("autotune: launch failed");
          return MXSEM_EHIP;
        }
      }
      const int reps = 5;
      hipError_t err = hipEventRecord(e0, s);
      for (int r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_ax_apply(prec, N, E, epb, u, w, G, nullptr, D, s, cols);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) {
        cleanup();
        set_error(std::string("autotune: timing failed: ") + hipGetErrorString(err));
        return MXSEM_EHIP;
      }
      ms /= reps;
      if (ms < best) {
        best = ms;
        *best_epb = epb;
        *best_cols = two ? cols : 0;
      }
    }
  }
  (void)device;
  cleanup();
  return rc;
}

// Tuning cache: a flat JSON object {"gfx950:N7:E32768:p1": 1, ...}; the
// value is the tile plus 100 times the thread mapping (0, 1 or 2).
static std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = t.substr(i + 1, j - i - 1);
    const size_t c = t.find(':', j);
    if (c == std::string::npos) break;
    out[key] = atoi(t.c_str() + c + 1);
    i = t.find_first_of(",}", c);
    if (i == std::string::npos) break;
  }
  return out;
}

static void write_cache(const char* path, const std::map<std::string, int>& kv) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{");
  bool first = true;
  for (const auto& e : kv) {
    fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", e.first.c_str(), e.second);
    first = false;
  }
  fprintf(f, "\n}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

}  // namespace mx

using namespace mx;

extern "C" {

static int check_tune_args(int N, int E, int prec) {
  MX_CHECK(N >= 1 && N <= MAX_N, MXSEM_ENOTSUP, "autotune: N must be in 1..15");
  MX_CHECK(E >= 1, MXSEM_EINVAL, "autotune: E must be >= 1");
  MX_CHECK(prec >= MXSEM_F64 && prec <= MXSEM_BF16G_F32, MXSEM_EINVAL, "autotune: bad precision");
  MX_CHECK((int64_t)E * (N + 1) * (N + 1) * (N + 1) < (int64_t)INT32_MAX - UPD_CHUNK,
           MXSEM_ENOTSUP, "autotune: more than 2^31 local entries");
  return MXSEM_OK;
}

int mxsem_autotune_workspace_bytes(int N, int E, mxsem_prec prec, size_t* bytes) {
  MX_API_BEGIN
  MX_CHECK(bytes, MXSEM_EINVAL, "autotune_workspace_bytes: null output");
  MX_TRY(check_tune_args(N, E, prec));
  *bytes = autotune_bytes(N, E, prec);
  return MXSEM_OK;
  MX_API_END("mxsem_autotune_workspace_bytes")
}

int mxsem_autotune(mxsem_ctx* ctx, int N, int E, mxsem_prec prec, void* workspace,
                   size_t ws_bytes, mxsem_tuning* out) {
  MX_API_BEGIN
  MX_CHECK(ctx && out, MXSEM_EINVAL, "autotune: null argument");
  MX_TRY(check_tune_args(N, E, prec));
  MX_CHECK(workspace && ((uintptr_t)workspace & 255) == 0, MXSEM_EINVAL,
           "autotune: workspace must be a 256-byte aligned device pointer");
  MX_CHECK(ws_bytes >= autotune_bytes(N, E, prec), MXSEM_EINVAL,
           "autotune: workspace smaller than mxsem_autotune_workspace_bytes");
  MX_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  int best = 0, cols = 0;
  MX_TRY(autotune_epb(ctx->device, ctx->stream, N, E, prec, (char*)workspace, &best, &cols));
  for (int q = 0; q < 16; ++q) out->epb[q] = out->cols[q] = 0;
  out->epb[N] = best;
  out->cols[N] = cols;
  return MXSEM_OK;
  MX_API_END("mxsem_autotune")
}

// Tuned tile for (N, E, prec) from the cache file, autotuned in the given
// workspace and added to the file when missing.
int mxsem_autotune_cached(mxsem_ctx* ctx, int N, int E, int prec, const char* path, void* ws,
                          size_t ws_bytes, int* epb, int* cols) {
  MX_API_BEGIN
  char key[96];
  snprintf(key, sizeof(key), "gfx950:N%d:E%d:p%d", N, E, prec);
  std::map<std::string, int> kv = read_cache(path);
  auto it = kv.find(key);
  if (it != kv.end()) {
    const int e = it->second % 100, c = it->second / 100;
    if (e >= 1 && e <= max_epb(N) && (c <= 1 || (c == 2 && ax_wave_elements(N) > 0))) {
      *epb = e;
      *cols = c;
      return MXSEM_OK;
    }
  }
  mxsem_tuning t{};
  MX_TRY(mxsem_autotune(ctx, N, E, (mxsem_prec)prec, ws, ws_bytes, &t));
  *epb = t.epb[N];
  *cols = t.cols[N];
  kv[key] = *epb + 100 * *cols;
  write_cache(path, kv);
  return MXSEM_OK;
  MX_API_END("mxsem_autotune_cached")
}

int mxsem_mesh_set_tuning(mxsem_mesh* m, const mxsem_tuning* t) {
  MX_API_BEGIN
  MX_CHECK(m && t, MXSEM_EINVAL, "mesh_set_tuning: null argument");
  const int e = t->epb[m->N], c = t->cols[m->N];
  MX_CHECK(e >= 0 && e <= max_epb(m->N), MXSEM_EINVAL,
           "mesh_set_tuning: elements per workgroup out of range for this order");
  MX_CHECK(c >= 0 && c <= 2 && (c < 2 || ax_wave_elements(m->N) > 0), MXSEM_EINVAL,
           "mesh_set_tuning: thread mapping must be 0, 1, or 2 where the order has a "
           "two-column kernel (N = 5, 9)");
  MX_HIP(hipSetDevice(m->ctx->device));
  m->epb[m->N] = e;
  m->cols[m->N] = c;
  mesh_drop_plans(m);  // plans are rebuilt with the new tiles on next use
  return MXSEM_OK;
  MX_API_END("mxsem_mesh_set_tuning")
}

}  // extern "C"
