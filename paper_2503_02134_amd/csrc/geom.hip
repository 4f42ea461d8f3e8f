// Set-up kernels, all FP64 (initialisation stays in double precision and is
// cast once, Sec. 5.2 and Sec. 6.1.1): isoparametric geometric factors and
// mass, the assembled Jacobi diagonal, and the FP32/BF16 copies.
#include <math.h>

#include "common.hpp"

namespace mx {

// One thread per node.  With x_r, x_s, x_t the columns of the Jacobian
// (D applied to the node coordinates along r, s, t), the contravariant
// gradients are grad r = (x_s x x_t)/|J|, grad s = (x_t x x_r)/|J|,
// grad t = (x_r x x_s)/|J|, so
//   G_ab = w_ijk k / |J| * (cross_a . cross_b),  B = w_ijk |J|,
// with w_ijk the tensor GLL weight.  detmin receives a per-block minimum.
__global__ void geom_kernel(int E, int n, const double* __restrict__ xyz,
                            const double* __restrict__ D, const double* __restrict__ wq,
                            const double* __restrict__ kcoef, double* __restrict__ G,
                            double* __restrict__ B, double* __restrict__ detmin) {
  __shared__ double smin[256];
  const int n3 = n * n * n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dmin = INFINITY;
  if (gid < (int64_t)E * n3) {
    const int e = (int)(gid / n3);
    const int p = (int)(gid - (int64_t)e * n3);
    const int i = p % n, j = (p / n) % n, k = p / (n * n);
    double col[3][3];  // col[d][c] = d x_c / d r_d
    for (int c = 0; c < 3; ++c) {
      const double* X = xyz + ((int64_t)e * 3 + c) * n3;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int l = 0; l < n; ++l) {
        a0 += D[i * n + l] * X[l + n * (j + n * k)];
        a1 += D[j * n + l] * X[i + n * (l + n * k)];
        a2 += D[k * n + l] * X[i + n * (j + n * l)];
      }
      col[0][c] = a0;
      col[1][c] = a1;
      col[2][c] = a2;
    }
    double cr[3][3];  // cr[a] = col[a+1] x col[a+2]
    for (int a = 0; a < 3; ++a) {
      const double* u = col[(a + 1) % 3];
      const double* v = col[(a + 2) % 3];
      cr[a][0] = u[1] * v[2] - u[2] * v[1];
      cr[a][1] = u[2] * v[0] - u[0] * v[2];
      cr[a][2] = u[0] * v[1] - u[1] * v[0];
    }
    const double det = col[0][0] * cr[0][0] + col[0][1] * cr[0][1] + col[0][2] * cr[0][2];
    dmin = det;
    const double wijk = wq[i] * wq[j] * wq[k];
    const double kk = kcoef ? kcoef[gid] : 1.0;
    const double s = wijk * kk / det;
    const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int q = 0; q < 6; ++q) {
      const double* ca = cr[pairs[q][0]];
      const double* cb = cr[pairs[q][1]];
      G[((int64_t)e * 6 + q) * n3 + p] = s * (ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2]);
    }
    B[gid] = wijk * det;
  }
  smin[threadIdx.x] = dmin;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) detmin[blockIdx.x] = smin[0];
}

// Local diagonal of sum_ab D_a^T diag(G_ab) D_b + h B at each node:
// only (q = node) terms survive the mixed products, so the cross terms are
// 2 D_ii D_jj G_rs + 2 D_ii D_kk G_rt + 2 D_jj D_kk G_st.
__global__ void diag_kernel(int E, int n, const double* __restrict__ G,
                            const double* __restrict__ B, double h, const double* __restrict__ D,
                            double* __restrict__ diag) {
  const int n3 = n * n * n;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)E * n3) return;
  const int e = (int)(gid / n3);
  const int p = (int)(gid - (int64_t)e * n3);
  const int i = p % n, j = (p / n) % n, k = p / (n * n);
  const double* Ge = G + (int64_t)e * 6 * n3;
  double s = 0.0;
  for (int l = 0; l < n; ++l) {
    const double di = D[l * n + i], dj = D[l * n + j], dk = D[l * n + k];
    s += di * di * Ge[0 * n3 + l + n * (j + n * k)];
    s += dj * dj * Ge[3 * n3 + i + n * (l + n * k)];
    s += dk * dk * Ge[5 * n3 + i + n * (j + n * l)];
  }
  const double dii = D[i * n + i], djj = D[j * n + j], dkk = D[k * n + k];
  s += 2.0 * (dii * djj * Ge[1 * n3 + p] + dii * dkk * Ge[2 * n3 + p] + djj * dkk * Ge[4 * n3 + p]);
  s += h * B[gid];
  diag[gid] = s;
}

__global__ void invert_kernel(double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = 1.0 / d[i];
}

__global__ void scale_kernel(double* __restrict__ d, const double* __restrict__ s, double h,
                             int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = h * s[i];
}

hipError_t launch_geom(int E, int n, const double* xyz, const double* D, const double* wq,
                       const double* kcoef, double* G, double* B, double* detmin, int* nblocks,
                       hipStream_t s) {
  const int64_t tot = (int64_t)E * n * n * n;
  const int nb = (int)((tot + 255) / 256);
  *nblocks = nb;
  hipLaunchKernelGGL(geom_kernel, dim3(nb), dim3(256), 0, s, E, n, xyz, D, wq, kcoef, G, B, detmin);
  return hipGetLastError();
}

hipError_t launch_diag(int E, int n, const double* G, const double* B, double h, const double* D,
                       double* diag, hipStream_t s) {
  const int64_t tot = (int64_t)E * n * n * n;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, E, n, G, B,
                     h, D, diag);
  return hipGetLastError();
}

hipError_t launch_invert(double* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(invert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n);
  return hipGetLastError();
}

hipError_t launch_scale(double* d, const double* src, double h, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, src, h, n);
  return hipGetLastError();
}

}  // namespace mx
