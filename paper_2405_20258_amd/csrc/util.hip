// Small layout kernels: zero fill, symmetric scaling, planar <-> interleaved
// conversion and the per-pair energy gaps e_c - e_v.
#include <cstdint>

#include "internal.hpp"

namespace ssrpa {

namespace {

__global__ void fill_zero_kernel(double *p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void fill_zero_bytes_kernel(unsigned char *p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void scale_sym_kernel(double *x, int n, const double *sv,
                                 int inverse) {
  const long total = (long)n * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    double f = sv[r] * sv[c];
    if (inverse) f = 1.0 / f;
    x[2 * idx] *= f;
    x[2 * idx + 1] *= f;
  }
}

__global__ void planar_to_interleaved_kernel(const double *src, int rows,
                                             int cols, int ld, double *dst) {
  const long total = (long)rows * cols;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / cols), c = (int)(idx % cols);
    dst[2 * idx] = src[(long)r * 2 * ld + c];
    dst[2 * idx + 1] = src[(long)r * 2 * ld + ld + c];
  }
}

__global__ void pair_de_kernel(const double *energy, const double *occ,
                               int c_first, int v0, int nvb, int n_c,
                               double *de, double *rowscale) {
  const long total = (long)nvb * n_c;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int v = v0 + (int)(idx / n_c), c = c_first + (int)(idx % n_c);
    if (!occ) {
      de[idx] = energy[c] - energy[v];
      continue;
    }
    // a pair counts once (v below c) and only with unequal occupations
    const double df = occ[v] - occ[c];
    const bool keep = v < c && df != 0.0;
    if (de) de[idx] = keep ? energy[c] - energy[v] : 1.0;
    if (rowscale) rowscale[idx] = keep ? sqrt(df) : 0.0;
  }
}

// de[p] = e_c[c_first + c] - e_v[v0 + v] (two band lists: k and k + q)
__global__ void pair_de2_kernel(const double *e_v, const double *e_c,
                                int c_first, int v0, int nvb, int n_c,
                                double *de) {
  const long total = (long)nvb * n_c;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int v = v0 + (int)(idx / n_c), c = c_first + (int)(idx % n_c);
    de[idx] = e_c[c] - e_v[v];
  }
}

// dst[b][r] = src[b][r] e^{+i 2 pi (g0 . j / N)} for n_b orbitals on the
// grid (x fastest): the valence orbitals shifted by an umklapp vector
__global__ void phase_shift_kernel(const double2 *src, long n_b, int n1, int n2,
                                   int n3, int g1, int g2, int g3,
                                   double2 *dst) {
  const long box = (long)n1 * n2 * n3;
  const long total = box * n_b;
  const double tp = 6.283185307179586476925286766559;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx % box;
    const int j1 = (int)(r % n1), j2 = (int)((r / n1) % n2), j3 = (int)(r / ((long)n1 * n2));
    // phase fraction reduced exactly in integers before the sine and cosine
    const long num = ((long)g1 * j1 * n2 * n3 + (long)g2 * j2 * n1 * n3 +
                      (long)g3 * j3 * n1 * n2) % ((long)n1 * n2 * n3);
    const double ang = tp * (double)num / (double)((long)n1 * n2 * n3);
    double sn, cs;
    sincos(ang, &sn, &cs);
    const double2 a = src[idx];
    dst[idx] = make_double2(a.x * cs - a.y * sn, a.x * sn + a.y * cs);
  }
}

// w[p][:] *= rowscale[p] over planar rows of 2 ld doubles; grid (x: row
// segments, y: rows).
__global__ void scale_rows_kernel(double *w, long rows, int ld,
                                  const double *rowscale, int inverse) {
  const long r = blockIdx.y + (long)gridDim.y * blockIdx.z;
  if (r >= rows) return;
  const double f = inverse ? 1.0 / rowscale[r] : rowscale[r];
  if (f == 1.0) return;
  double *row = w + r * 2L * ld;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * ld;
       i += gridDim.x * blockDim.x)
    row[i] *= f;
}

// planar rows (row stride 2 ld, im at +ld): column j times f[j], j < ncol;
// f[j] = sqrt(max(lam[j], 0)) when from_eigs (scaled by the square roots of
// non-negative eigenvalues)
__global__ void scale_cols_kernel(double *w, long rows, int ld, int ncol,
                                  const double *f, int from_eigs) {
  const long total = rows * ncol;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx / ncol;
    const int j = (int)(idx % ncol);
    const double x = f[j];
    const double m = from_eigs ? sqrt(x > 0.0 ? x : 0.0) : x;
    w[r * 2 * ld + j] *= m;
    w[r * 2 * ld + ld + j] *= m;
  }
}

__global__ void copy_kernel(const double *src, double *dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// 16-byte loads and stores, the access width of the contraction kernels
__global__ void copy16_kernel(const double2 *__restrict__ src,
                              double2 *__restrict__ dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

bool aligned16(const void *p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

unsigned grid_for(long n) {
  return (unsigned)std::max(1L, std::min((n + 255) / 256, 65536L));
}

}  // namespace

void fill_zero(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes % 8 == 0 && ((uintptr_t)p % 8) == 0) {
    const long n = (long)(bytes / 8);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                       (double *)p, n);
  } else {
    hipLaunchKernelGGL(fill_zero_bytes_kernel, dim3(grid_for((long)bytes)),
                       dim3(256), 0, s, (unsigned char *)p, (long)bytes);
  }
  SSRPA_HIP(hipGetLastError());
}

void scale_sym(double *x, int n, const double *sv, int inverse, hipStream_t s) {
  hipLaunchKernelGGL(scale_sym_kernel, dim3(grid_for((long)n * n)), dim3(256), 0,
                     s, x, n, sv, inverse);
  SSRPA_HIP(hipGetLastError());
}

void planar_to_interleaved(const double *src, int rows, int cols, int ld,
                           double *dst, hipStream_t s) {
  hipLaunchKernelGGL(planar_to_interleaved_kernel,
                     dim3(grid_for((long)rows * cols)), dim3(256), 0, s, src,
                     rows, cols, ld, dst);
  SSRPA_HIP(hipGetLastError());
}

void pair_energy_diffs(const double *energy, const double *occ, int c_first,
                       int v0, int nvb, int n_c, double *de, double *rowscale,
                       hipStream_t s) {
  const long total = (long)nvb * n_c;
  hipLaunchKernelGGL(pair_de_kernel, dim3(grid_for(total)), dim3(256), 0, s,
                     energy, occ, c_first, v0, nvb, n_c, de, rowscale);
  SSRPA_HIP(hipGetLastError());
}

void pair_energy_diffs2(const double *e_v, const double *e_c, int c_first,
                        int v0, int nvb, int n_c, double *de, hipStream_t s) {
  hipLaunchKernelGGL(pair_de2_kernel, dim3(grid_for((long)nvb * n_c)), dim3(256),
                     0, s, e_v, e_c, c_first, v0, nvb, n_c, de);
  SSRPA_HIP(hipGetLastError());
}

void phase_shift(const double *src, long n_b, int n1, int n2, int n3,
                 const int *g0, double *dst, hipStream_t s) {
  const long total = (long)n1 * n2 * n3 * n_b;
  hipLaunchKernelGGL(phase_shift_kernel, dim3(grid_for(total)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(src), n_b, n1, n2, n3,
                     g0[0], g0[1], g0[2], reinterpret_cast<double2 *>(dst));
  SSRPA_HIP(hipGetLastError());
}

void scale_rows(double *w, long rows, int ld, const double *rowscale,
                hipStream_t s, bool inverse) {
  if (rows <= 0) return;
  const long ry = std::min<long>(rows, 65535);
  const long rz = (rows + ry - 1) / ry;
  const int bx = std::max(1, std::min(8, (2 * ld + 255) / 256));
  hipLaunchKernelGGL(scale_rows_kernel, dim3(bx, (unsigned)ry, (unsigned)rz),
                     dim3(256), 0, s, w, rows, ld, rowscale, (int)inverse);
  SSRPA_HIP(hipGetLastError());
}

void scale_cols(double *w, long rows, int ld, int ncol, const double *f,
                int from_eigs, hipStream_t s) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(rows * ncol)), dim3(256),
                     0, s, w, rows, ld, ncol, f, from_eigs);
  SSRPA_HIP(hipGetLastError());
}

void copy_interleaved(const double *src, double *dst, size_t n_complex,
                      hipStream_t s) {
  const long n = (long)(2 * n_complex);
  if (aligned16(src) && aligned16(dst)) {
    hipLaunchKernelGGL(copy16_kernel, dim3(grid_for(n / 2)), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(src),
                       reinterpret_cast<double2 *>(dst), n / 2);
  } else {
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, src,
                       dst, n);
  }
  SSRPA_HIP(hipGetLastError());
}

void device_copy16(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const long n = (long)(bytes / 16);
  hipLaunchKernelGGL(copy16_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                     static_cast<const double2 *>(src), static_cast<double2 *>(dst),
                     n);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
