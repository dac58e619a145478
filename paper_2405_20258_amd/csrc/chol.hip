// Per-frequency trace of the logarithm and the frequency quadrature.
//
// The trace is evaluated in the subspace basis as the log of a determinant
// (paper, Implementation section, last paragraph: Tr ln A = ln det A, taken
// from a triangular factorization instead of a diagonalization):
//   F_j = ln det(I - l X_j) + l Tr X_j,   X_j = v^1/2 chi0_s(i w_j) v^1/2.
// I - l X_j is Hermitian positive definite (X_j is negative semidefinite),
// so a Cholesky factor is used: ln det = sum_k ln p_k with p_k the pivots of
// the outer-product elimination B <- B - b_k b_k^H / p_k.
// Then E_c = (1/2 pi) sum_j w_j F_j  (Eq. 1).
//
// At high frequency X_j is small, the pivots are 1 + O(|X|) and ln det and
// l Tr X cancel to second order.  The elimination therefore works on
// B - I: the diagonal holds delta_k = p_k - 1 without the rounding of
// 1 + delta, and F = sum_k [log1p(delta_k) + l X_kk], whose terms are each
// accurate to rounding of their own size.
#include <cmath>

#include "internal.hpp"

namespace ssrpa {

namespace {

// D_j = B_j - I = -c X_j   (interleaved n x n per matrix)
__global__ void build_b_kernel(const double *__restrict__ x, double c, int n,
                               long n_mat, double *__restrict__ b) {
  const long per = (long)n * n;
  const long total = per * n_mat;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    b[2 * idx] = -c * x[2 * idx];
    b[2 * idx + 1] = -c * x[2 * idx + 1];
  }
}

// One elimination step k for every matrix on D = B - I:
// D[i][j] -= conj(D[k][i]) D[k][j] / (1 + D[k][k]) for k < i <= j (upper
// form, row k holds the pivot row; off the diagonal D and B agree).  Block
// (tile, matrix); block 0 of each matrix records delta_k = D[k][k].
__global__ __launch_bounds__(256) void chol_step_kernel(double *__restrict__ b,
                                                        int n, int k,
                                                        double *__restrict__ piv,
                                                        int *__restrict__ flag) {
  const int j_mat = blockIdx.y;
  double2 *B = reinterpret_cast<double2 *>(b) + (long)j_mat * n * n;
  const double dk = B[(long)k * n + k].x;
  const double p = 1.0 + dk;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    piv[(long)j_mat * n + k] = dk;
    if (!(p > 0.0)) *flag = 1;  // every writer stores the same value
  }
  const int m = n - k - 1;
  if (m <= 0 || !(p > 0.0)) return;
  const double inv = 1.0 / p;
  const long total = (long)m * m;
  const double2 *rowk = B + (long)k * n + k + 1;
  for (long idx = blockIdx.x * 256L + threadIdx.x; idx < total;
       idx += (long)gridDim.x * 256L) {
    const int i = (int)(idx / m), j = (int)(idx % m);
    if (j < i) continue;  // upper triangle suffices
    const double2 a = rowk[i], c = rowk[j];
    // conj(a) c / p
    const double re = (a.x * c.x + a.y * c.y) * inv;
    const double im = (a.x * c.y - a.y * c.x) * inv;
    double2 *d = B + (long)(k + 1 + i) * n + k + 1 + j;
    double2 v = *d;
    v.x -= re;
    v.y -= im;
    *d = v;
  }
}

__global__ void logdet_finish_kernel(const double *__restrict__ piv,
                                     const double *__restrict__ x, double c,
                                     int n, int n_mat, double *__restrict__ f) {
  const int j = blockIdx.x;
  if (j >= n_mat) return;
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    // log(1 + delta_k) + c X_kk, with delta_k = p_k - 1 carried exactly
    acc += log1p(piv[(long)j * n + k]) + c * x[2 * ((long)j * n * n + (long)k * n + k)];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) a += red[i];
    f[j] = a;
  }
}

__global__ void quadrature_kernel(const double *__restrict__ w,
                                  const double *__restrict__ f, int n,
                                  double *__restrict__ ec) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += w[j] * f[j];
    ec[0] = s / (2.0 * 3.14159265358979323846);
  }
}

}  // namespace

void trace_log(Context *ctx, const double *x, int n, int n_mat, double coupling,
               double *f, int *flag, hipStream_t s) {
  SSRPA_REQUIRE(n >= 1 && n_mat >= 1, SSRPA_ERR_ARG, "trace_log: empty batch");
  DevBuf b(ctx, sizeof(double) * 2 * (size_t)n * n * n_mat);
  DevBuf piv(ctx, sizeof(double) * (size_t)n * n_mat);
  const long total = (long)n * n * n_mat;
  hipLaunchKernelGGL(build_b_kernel,
                     dim3((unsigned)std::min<long>((total + 255) / 256, 65536)),
                     dim3(256), 0, s, x, coupling, n, (long)n_mat, b.as<double>());
  for (int k = 0; k < n; ++k) {
    const long m = n - k - 1;
    const long work = std::max(1L, (m * m) / 2);
    const int blocks = (int)std::max(1L, std::min((work + 1023) / 1024, 2048L));
    hipLaunchKernelGGL(chol_step_kernel, dim3(blocks, n_mat), dim3(256), 0, s,
                       b.as<double>(), n, k, piv.as<double>(), flag);
  }
  hipLaunchKernelGGL(logdet_finish_kernel, dim3(n_mat), dim3(256), 0, s,
                     piv.as<double>(), x, coupling, n, n_mat, f);
  SSRPA_HIP(hipGetLastError());
  SSRPA_HIP(hipStreamSynchronize(s));  // work buffers are freed on return
}

void quadrature(const double *w, const double *f, int n, double *ec,
                hipStream_t s) {
  hipLaunchKernelGGL(quadrature_kernel, dim3(1), dim3(64), 0, s, w, f, n, ec);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
