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
// D = B - I: the diagonal holds delta_k = p_k - 1 without the rounding of
// 1 + delta, and F = sum_k [log1p(delta_k) + l X_kk], whose terms are each
// accurate to rounding of their own size.
//
// The elimination is blocked over panels of kPb columns (upper form: row k
// of D is the pivot row).  Per panel two launches: the panel kernel
// eliminates the panel's kPb steps inside its rows (each work-group holds
// the kPb x kPb diagonal block and one chunk of the rows' trailing columns
// in LDS), then the update kernel subtracts the panel's rank-kPb product
// from the upper triangle of the trailing block.  A matrix whose pivot is
// not positive is marked failed and skipped from then on; its F is NaN.
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace ssrpa {

namespace {

constexpr int kPb = 32;      // panel width (elimination steps per panel)
constexpr int kPc = 64;      // trailing columns per panel work-group
constexpr int kUt = 32;      // output tile of the trailing update

// D_j = B_j - I = -c X_j   (interleaved n x n per matrix); fail_j = 0.
__global__ void build_b_kernel(const double *__restrict__ x, double c, int n,
                               long n_mat, double *__restrict__ b,
                               int *__restrict__ fail) {
  const long per = (long)n * n;
  const long total = per * n_mat;
  const long t0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  for (long idx = t0; idx < total; idx += (long)gridDim.x * blockDim.x) {
    b[2 * idx] = -c * x[2 * idx];
    b[2 * idx + 1] = -c * x[2 * idx + 1];
  }
  for (long j = t0; j < n_mat; j += (long)gridDim.x * blockDim.x) fail[j] = 0;
}

// Panel k0 .. k0 + nb - 1 of every matrix: grid (chunks, n_mat).  Work-group
// `chunk` owns trailing columns [k0 + nb + chunk kPc, +kPc) of the panel
// rows; every work-group eliminates the diagonal block itself (kPb^3 work),
// so no work-group waits for another.  Step k:
//   D[i][j] -= conj(D[k][i]) D[k][j] / (1 + D[k][k]),  k < i <= j.
// Work-group 0 records delta_k = D[k][k] and marks a non-positive pivot.
__global__ __launch_bounds__(256) void chol_panel_kernel(
    double2 *__restrict__ d, int n, int k0, int nb, double *__restrict__ piv,
    int *__restrict__ fail) {
  __shared__ double2 dd[kPb][kPb + 1];
  __shared__ double2 dc[kPb][kPc + 1];
  const int mat = blockIdx.y;
  if (fail[mat]) return;
  double2 *B = d + (long)mat * n * n;
  const int tid = threadIdx.x;
  const int c0 = k0 + nb + blockIdx.x * kPc;
  const int cw = max(0, min(kPc, n - c0));
  for (int e = tid; e < kPb * kPb; e += 256) {
    const int i = e / kPb, j = e % kPb;
    dd[i][j] = (i < nb && j < nb && j >= i) ? B[(long)(k0 + i) * n + k0 + j]
                                            : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < kPb * kPc; e += 256) {
    const int i = e / kPc, j = e % kPc;
    dc[i][j] = (i < nb && j < cw) ? B[(long)(k0 + i) * n + c0 + j]
                                  : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const double dk = dd[k][k].x;
    const double p = 1.0 + dk;
    if (blockIdx.x == 0 && tid == 0) {
      piv[(long)mat * n + k0 + k] = dk;
      if (!(p > 0.0)) fail[mat] = 1;
    }
    if (!(p > 0.0)) return;  // uniform: every thread read the same pivot
    const double inv = 1.0 / p;
    for (int e = tid; e < kPb * kPb; e += 256) {
      const int i = e / kPb, j = e % kPb;
      if (i > k && j >= i && j < nb) {
        const double2 a = dd[k][i], c = dd[k][j];
        dd[i][j].x -= (a.x * c.x + a.y * c.y) * inv;
        dd[i][j].y -= (a.x * c.y - a.y * c.x) * inv;
      }
    }
    for (int e = tid; e < kPb * kPc; e += 256) {
      const int i = e / kPc, j = e % kPc;
      if (i > k && i < nb && j < cw) {
        const double2 a = dd[k][i], c = dc[k][j];
        dc[i][j].x -= (a.x * c.x + a.y * c.y) * inv;
        dc[i][j].y -= (a.x * c.y - a.y * c.x) * inv;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < kPb * kPc; e += 256) {
    const int i = e / kPc, j = e % kPc;
    if (i < nb && j < cw) B[(long)(k0 + i) * n + c0 + j] = dc[i][j];
  }
}

// Trailing update after panel k0 (width nb): for t0 = k0 + nb <= i <= j < n
//   D[i][j] -= sum_k conj(P[k][i]) P[k][j] / (1 + delta_k),  P = panel rows.
// Grid (upper-triangle tiles of kUt x kUt, n_mat); 256 threads, 2 x 2
// outputs each.
__global__ __launch_bounds__(256) void chol_update_kernel(
    double2 *__restrict__ d, int n, int k0, int nb,
    const double *__restrict__ piv, const int *__restrict__ fail) {
  __shared__ double2 pa[kPb][kUt + 1];
  __shared__ double2 pb[kPb][kUt + 1];
  const int mat = blockIdx.y;
  if (fail[mat]) return;
  double2 *B = d + (long)mat * n * n;
  const int t0 = k0 + nb;
  // tile t -> (ti, tj), ti <= tj, row-major over the upper triangle
  const int nt = (n - t0 + kUt - 1) / kUt;
  int t = blockIdx.x, ti = 0;
  while (t >= nt - ti) {
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int r0 = t0 + ti * kUt, q0 = t0 + tj * kUt;
  const int tid = threadIdx.x;
  for (int e = tid; e < kPb * kUt; e += 256) {
    const int k = e / kUt, c = e % kUt;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (k < nb) {
      const double inv = 1.0 / (1.0 + piv[(long)mat * n + k0 + k]);
      if (r0 + c < n) {
        const double2 v = B[(long)(k0 + k) * n + r0 + c];
        a = make_double2(v.x * inv, -v.y * inv);  // conj(P[k][i]) / p_k
      }
      if (q0 + c < n) b = B[(long)(k0 + k) * n + q0 + c];
    }
    pa[k][c] = a;
    pb[k][c] = b;
  }
  __syncthreads();
  const int ty = tid / 16, tx = tid % 16;
  double2 acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int w = 0; w < 2; ++w) acc[u][w] = make_double2(0.0, 0.0);
  for (int k = 0; k < nb; ++k) {
    const double2 a0 = pa[k][2 * ty], a1 = pa[k][2 * ty + 1];
    const double2 b0 = pb[k][2 * tx], b1 = pb[k][2 * tx + 1];
    const double2 av[2] = {a0, a1}, bv[2] = {b0, b1};
    for (int u = 0; u < 2; ++u)
      for (int w = 0; w < 2; ++w) {
        acc[u][w].x += av[u].x * bv[w].x - av[u].y * bv[w].y;
        acc[u][w].y += av[u].x * bv[w].y + av[u].y * bv[w].x;
      }
  }
  for (int u = 0; u < 2; ++u)
    for (int w = 0; w < 2; ++w) {
      const int i = r0 + 2 * ty + u, j = q0 + 2 * tx + w;
      if (i < n && j < n && j >= i) {
        double2 *o = B + (long)i * n + j;
        double2 v = *o;
        v.x -= acc[u][w].x;
        v.y -= acc[u][w].y;
        *o = v;
      }
    }
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// F_j = sum_k [log1p(delta_k) + c X_kk]; NaN (and *flag = 1) for a matrix
// whose factorization failed.  One work-group of 256 per matrix: strided
// lane sums, a butterfly inside each wave, the four wave sums in order.
__global__ __launch_bounds__(256) void logdet_finish_kernel(
    const double *__restrict__ piv, const double *__restrict__ x, double c,
    int n, int n_mat, const int *__restrict__ fail, double *__restrict__ f,
    int *__restrict__ flag) {
  const int j = blockIdx.x;
  if (j >= n_mat) return;
  __shared__ double red[4];
  if (fail[j]) {
    if (threadIdx.x == 0) {
      f[j] = __builtin_nan("");
      if (flag) *flag = 1;  // every writer stores the same value
    }
    return;
  }
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256)
    acc += log1p(piv[(long)j * n + k]) + c * x[2 * ((long)j * n * n + (long)k * n + k)];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) f[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ec = (1/2 pi) sum_j w_j f_j: one wave, strided lane sums, butterfly.
__global__ __launch_bounds__(64) void quadrature_kernel(
    const double *__restrict__ w, const double *__restrict__ f, int n,
    double *__restrict__ ec) {
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 64) s += w[j] * f[j];
  s = wave_sum(s);
  if (threadIdx.x == 0) ec[0] = s / (2.0 * 3.14159265358979323846);
}

// The whole batch on caller-provided work memory: d (n_mat n^2 complex),
// piv (n_mat n doubles), fail (n_mat ints).
void trace_log_on(const double *x, int n, int n_mat, double coupling,
                  double *f, int *flag, double *d, double *piv, int *fail,
                  hipStream_t s) {
  const long total = (long)n * n * n_mat;
  hipLaunchKernelGGL(build_b_kernel,
                     dim3((unsigned)std::min<long>((total + 255) / 256, 65536)),
                     dim3(256), 0, s, x, coupling, n, (long)n_mat, d, fail);
  double2 *D = reinterpret_cast<double2 *>(d);
  for (int k0 = 0; k0 < n; k0 += kPb) {
    const int nb = std::min(kPb, n - k0);
    const int m = n - k0 - nb;
    const int chunks = std::max(1, (m + kPc - 1) / kPc);
    hipLaunchKernelGGL(chol_panel_kernel, dim3(chunks, n_mat), dim3(256), 0, s,
                       D, n, k0, nb, piv, fail);
    if (m > 0) {
      const long nt = (m + kUt - 1) / kUt;
      hipLaunchKernelGGL(chol_update_kernel,
                         dim3((unsigned)(nt * (nt + 1) / 2), n_mat), dim3(256),
                         0, s, D, n, k0, nb, (const double *)piv,
                         (const int *)fail);
    }
  }
  hipLaunchKernelGGL(logdet_finish_kernel, dim3(n_mat), dim3(256), 0, s,
                     (const double *)piv, x, coupling, n, n_mat,
                     (const int *)fail, f, flag);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace

void trace_log(Context *ctx, const double *x, int n, int n_mat, double coupling,
               double *f, int *flag, hipStream_t s) {
  SSRPA_REQUIRE(n >= 1 && n_mat >= 1, SSRPA_ERR_ARG, "trace_log: empty batch");
  SSRPA_REQUIRE(n_mat <= 65535, SSRPA_ERR_ARG, "trace_log: more than 65535 matrices");
  DevBuf b(ctx, sizeof(double) * 2 * (size_t)n * n * n_mat);
  DevBuf piv(ctx, sizeof(double) * (size_t)n * n_mat + sizeof(int) * (size_t)n_mat);
  int *fail = reinterpret_cast<int *>(piv.as<double>() + (size_t)n * n_mat);
  trace_log_on(x, n, n_mat, coupling, f, flag, b.as<double>(), piv.as<double>(),
               fail, s);
  SSRPA_HIP(hipStreamSynchronize(s));  // work buffers are freed on return
}

void quadrature(const double *w, const double *f, int n, double *ec,
                hipStream_t s) {
  hipLaunchKernelGGL(quadrature_kernel, dim3(1), dim3(64), 0, s, w, f, n, ec);
  SSRPA_HIP(hipGetLastError());
}

// ---- inverse of I - X -------------------------------------------------------
//
// eps^-1 = (I - l X)^-1 for Hermitian X with I - l X positive definite
// (the dielectric matrix of the Implementation section's last paragraph),
// by Gauss-Jordan elimination without pivoting (stable for a positive
// definite matrix).  Step k maps, with old values o and pivot p = o_kk,
//   a_kj = o_kj / p,  a_kk = 1 / p,  a_ik = -o_ik / p,
//   a_ij = o_ij - o_ik o_kj / p          (i, j != k),
// so the n steps leave the inverse in place.  Row and column k are copied
// out before each step so that no work-group reads a value another one has
// already overwritten.

namespace {

__global__ void build_eps_kernel(const double *__restrict__ x, double c, long n,
                                 long n_mat, double *__restrict__ a,
                                 int *__restrict__ fail) {
  const long total = n * n * n_mat;
  const long t0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  for (long idx = t0; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long e = idx % (n * n);
    const bool diag = e / n == e % n;
    a[2 * idx] = (diag ? 1.0 : 0.0) - c * x[2 * idx];
    a[2 * idx + 1] = diag ? 0.0 : -c * x[2 * idx + 1];
  }
  for (long j = t0; j < n_mat; j += (long)gridDim.x * blockDim.x) fail[j] = 0;
}

// rc[mat][0..n) = row k, rc[mat][n..2n) = column k
__global__ void gj_save_kernel(const double2 *__restrict__ a, int n, int k,
                               double2 *__restrict__ rc) {
  const int mat = blockIdx.y;
  const double2 *A = a + (long)mat * n * n;
  double2 *R = rc + (long)mat * 2 * n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gridDim.x * blockDim.x) {
    R[i] = A[(long)k * n + i];
    R[n + i] = A[(long)i * n + k];
  }
}

__global__ void gj_step_kernel(double2 *__restrict__ a, int n, int k,
                               const double2 *__restrict__ rc,
                               int *__restrict__ fail) {
  const int mat = blockIdx.y;
  if (fail[mat]) return;
  const double2 *R = rc + (long)mat * 2 * n;
  const double p = R[k].x;  // real: the matrix stays Hermitian
  if (!(p > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fail[mat] = 1;
    return;
  }
  const double inv = 1.0 / p;
  double2 *A = a + (long)mat * n * n;
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double2 o = A[e];
    double2 r;
    if (i == k && j == k) {
      r = make_double2(inv, 0.0);
    } else if (i == k) {
      r = make_double2(o.x * inv, o.y * inv);
    } else if (j == k) {
      r = make_double2(-o.x * inv, -o.y * inv);
    } else {
      const double2 cik = R[n + i], ckj = R[j];
      r.x = o.x - (cik.x * ckj.x - cik.y * ckj.y) * inv;
      r.y = o.y - (cik.x * ckj.y + cik.y * ckj.x) * inv;
    }
    A[e] = r;
  }
}

__global__ void gj_flag_kernel(const int *__restrict__ fail, int n_mat,
                               int *__restrict__ flag) {
  for (int j = threadIdx.x; j < n_mat; j += blockDim.x)
    if (fail[j]) *flag = 1;  // every writer stores the same value
}

}  // namespace

void inverse_one_minus(Context *ctx, const double *x, int n, int n_mat,
                       double coupling, double *out, int *flag, hipStream_t s) {
  SSRPA_REQUIRE(n >= 1 && n_mat >= 1 && n_mat <= 65535, SSRPA_ERR_ARG,
                "inverse: bad batch");
  DevBuf rc(ctx, sizeof(double2) * 2 * (size_t)n * n_mat + sizeof(int) * n_mat);
  int *fail = reinterpret_cast<int *>(rc.as<double2>() + 2 * (size_t)n * n_mat);
  const long total = (long)n * n * n_mat;
  hipLaunchKernelGGL(build_eps_kernel,
                     dim3((unsigned)std::min<long>((total + 255) / 256, 65536)),
                     dim3(256), 0, s, x, coupling, (long)n, (long)n_mat, out,
                     fail);
  double2 *A = reinterpret_cast<double2 *>(out);
  const unsigned sb = (unsigned)std::max(1, std::min(64, (n + 255) / 256));
  const unsigned ub =
      (unsigned)std::max(1L, std::min<long>(((long)n * n + 255) / 256, 1024));
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(gj_save_kernel, dim3(sb, n_mat), dim3(256), 0, s,
                       (const double2 *)A, n, k, rc.as<double2>());
    hipLaunchKernelGGL(gj_step_kernel, dim3(ub, n_mat), dim3(256), 0, s, A, n, k,
                       (const double2 *)rc.as<double2>(), fail);
  }
  hipLaunchKernelGGL(gj_flag_kernel, dim3(1), dim3(256), 0, s,
                     (const int *)fail, n_mat, flag);
  SSRPA_HIP(hipGetLastError());
  SSRPA_HIP(hipStreamSynchronize(s));  // the work buffer is freed on return
}

// ---- allocation-free form ---------------------------------------------------
//
// Work memory of the batch (D, pivots, failure marks) in a fixed device array
// instead of the context's allocator.  Each device holds its own copy of the
// array; its address is looked up once per device while that device is
// current (noalloc_setup, called when a context is created) and passed to the
// kernels.  Every call on a device shares the array: calls that overlap on one
// device race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

void noalloc_setup(int device) {
  SSRPA_REQUIRE(device >= 0 && device < kMaxDevices, SSRPA_ERR_ARG,
                "device %d beyond the %d devices with a fixed work array",
                device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void *p = nullptr;
  SSRPA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  SSRPA_REQUIRE(p != nullptr, SSRPA_ERR_HIP, "no address for the work array");
  g_scratch_ptr[device] = p;
}

size_t trace_log_noalloc_bytes(int n, int n_mat) {
  return align256(sizeof(double) * 2 * (size_t)n * n * n_mat) +
         align256(sizeof(double) * (size_t)n * n_mat) +
         align256(sizeof(int) * (size_t)n_mat);
}

void trace_log_noalloc(int device, const double *x, int n, int n_mat,
                       double coupling, double *f, int *flag, hipStream_t s) {
  SSRPA_REQUIRE(n >= 1 && n_mat >= 1, SSRPA_ERR_ARG, "trace_log: empty batch");
  SSRPA_REQUIRE(n_mat <= 65535, SSRPA_ERR_ARG, "trace_log: more than 65535 matrices");
  const size_t need = trace_log_noalloc_bytes(n, n_mat);
  SSRPA_REQUIRE(need <= kNoAllocScratchBytes, SSRPA_ERR_ARG,
                "%d matrices of order %d need %zu bytes of work memory, beyond "
                "the fixed %zu-byte array of the allocation-free form",
                n_mat, n, need, kNoAllocScratchBytes);
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (device >= 0 && device < kMaxDevices) base = g_scratch_ptr[device];
  }
  SSRPA_REQUIRE(base, SSRPA_ERR_STATE,
                "work array of device %d not set up (create a context first)",
                device);
  char *b = static_cast<char *>(base);
  double *d = reinterpret_cast<double *>(b);
  b += align256(sizeof(double) * 2 * (size_t)n * n * n_mat);
  double *piv = reinterpret_cast<double *>(b);
  b += align256(sizeof(double) * (size_t)n * n_mat);
  int *fail = reinterpret_cast<int *>(b);
  if (flag) fill_zero(flag, sizeof(int), s);
  // build_b_kernel clears the failure marks; every other word of the array
  // is written before it is read
  trace_log_on(x, n, n_mat, coupling, f, flag, d, piv, fail, s);
}

}  // namespace ssrpa
