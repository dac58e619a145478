// Real-orbital (Gamma-point) path.
//
// When every orbital is real (c(-G) = conj c(G), time-reversal symmetric
// orbitals at the Gamma point), every pair density rho_vc(r) is real and
// M_vc(-G) = conj M_vc(G).  In the cos/sin basis of the chi0 set,
//   c_G = (e^{iG.r} + e^{-iG.r}) / sqrt 2,  s_G = (e^{iG.r} - e^{-iG.r}) / (sqrt 2 i)
// for the larger member G of each pair {G, -G}, the pair matrix is real,
//   M^c(G) = sqrt 2 Re M(G),  M^s(G) = sqrt 2 Im M(G),
// and chi0 (Eq. 6) is real symmetric: the contractions need a quarter of
// the complex flops.  The basis change is unitary and v(G) = v(-G), so
// eigenvalues, F_j and E_c (Eq. 1) are unchanged.
//
// The pair transform also does half the work: two conduction orbitals are
// packed into one complex orbital phi = psi_c1 + i psi_c2 (in coefficient
// space, before the orbital FFT), the complex pair transform of (psi_v, phi)
// gives F = M_v,c1 + i M_v,c2, and since M(-G) = conj M(G) for both,
//   M_v,c1(G) = (F(G) + conj F(-G)) / 2,  M_v,c2(G) = (F(G) - conj F(-G)) / 2i.
//
// Real contractions on v_mfma_f64_16x16x4f64: a 256-thread block owns a
// 128 x 128 output tile, each wave a 64 x 64 quadrant (4 x 4 MFMA tiles);
// 16-row K chunks staged through LDS with the next chunk prefetched into
// registers; split K with an ordered reduction (deterministic).
#include <cmath>

#include "internal.hpp"
#include "tiles.hpp"

namespace ssrpa {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kRT = 128;   // real output tile
constexpr int kRK = 16;    // K rows per LDS stage
constexpr int kRPad = 2;   // LDS row padding (doubles)

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int l, int e) { return (l >> 4) + 4 * e; }
__device__ __forceinline__ int acc_col(int l) { return l & 15; }


// ---------------------------------------------------------------- SYRK f64
//
// X_w = A^T diag(d_w) A for real A (k rows of stride lda, columns ncol <= ld,
// ld a multiple of 128, zero padded), d_w,p = -4 de_p / (de_p^2 + om_w^2)
// x wscale (or 1 with unit_weight), applied to the B operand while staging.
// Grid (lower-triangle tiles, K splits, frequencies); partial tiles
// [w][split][tile][128][128].
constexpr int kSyrkThreads = 512;   // 8 waves, each a 64 x 32 part of the tile
__global__ __launch_bounds__(kSyrkThreads) void syrk_f64_kernel(
    HerkArgs h, int T, int n_tiles, long kchunk, double *__restrict__ partial) {
  __shared__ double As[kRK][kRT + kRPad];
  __shared__ double Bs[kRK][kRT + kRPad];
  // neighbouring tiles (which share operand panels) on one XCD, in blocks
  // of 8 x 8 tiles
  const int tile_id = xcd_remap(blockIdx.x, n_tiles);
  const int split = blockIdx.y;
  const int om_i = blockIdx.z;
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kRT, J0 = tile.y * kRT;
  const double om = h.unit_weight ? 0.0 : h.omega[om_i];
  const long kbeg = split * kchunk;
  const long kend = min(h.k, kbeg + kchunk);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // 2 x 4 waves of 64 x 32: a 64-row accumulator quadrant per wave would
  // take 128 VGPRs and hold the kernel at 2 waves per SIMD
  const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
  d4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  // staging: 4 double2 per thread; it < 2: A rows, it >= 2: B rows; row
  // r0 + 8 (it & 1), columns 2 c2, 2 c2 + 1 of the 128-wide panel
  const int r0 = threadIdx.x >> 6, c2 = (threadIdx.x & 63) * 2;
  double2 pv[4];
  double pw[2];
  auto fetch = [&](long k0) __attribute__((always_inline)) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const long p = k0 + r0 + 8 * (it & 1);
      const int col0 = it < 2 ? I0 : J0;
      pv[it] = make_double2(0.0, 0.0);
      if (p < kend)
        pv[it] = *reinterpret_cast<const double2 *>(h.a + p * h.lda + col0 + c2);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const long p = k0 + r0 + 8 * q;
      pw[q] = 0.0;
      if (p < kend) {
        if (h.unit_weight) {
          pw[q] = 1.0;
        } else {
          const double de = h.de[p];
          pw[q] = -4.0 * de / (de * de + om * om) * h.wscale;
        }
      }
    }
  };
  fetch(kbeg);
  for (long k0 = kbeg; k0 < kend; k0 += kRK) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int r = r0 + 8 * (it & 1);
      if (it < 2) {
        As[r][c2] = pv[it].x;
        As[r][c2 + 1] = pv[it].y;
      } else {
        const double w = pw[it & 1];
        Bs[r][c2] = pv[it].x * w;
        Bs[r][c2 + 1] = pv[it].y * w;
      }
    }
    __syncthreads();
    if (k0 + kRK < kend) fetch(k0 + kRK);
#pragma unroll
    for (int ks = 0; ks < kRK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const int cl = lane & 15;
      double a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kr][wr + i * 16 + cl];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wc + j * 16 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma64(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double *out = partial + (((long)om_i * gridDim.y + split) * n_tiles + tile_id) *
                              (long)kRT * kRT;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr + i * 16 + acc_row(lane, e);
        const int c = wc + j * 16 + acc_col(lane);
        out[r * kRT + c] = acc[i][j][e];
      }
}

// Sum the split partials in order and write the symmetric matrices as
// interleaved complex (imaginary part 0), both halves.
__global__ void syrk_reduce_kernel(const double *__restrict__ partial, int T,
                                   int n_tiles, int nsplit, int ncol,
                                   double *__restrict__ out, long out_stride,
                                   int beta) {
  const int tile_id = blockIdx.x;
  const int om_i = blockIdx.y;
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kRT, J0 = tile.y * kRT;
  double *o = out + om_i * out_stride;
  for (int e = threadIdx.x; e < kRT * kRT; e += blockDim.x) {
    const int r = e / kRT, c = e % kRT;
    const int g = I0 + r, gp = J0 + c;
    if (g >= ncol || gp >= ncol) continue;
    if (tile.x == tile.y && r < c) continue;
    double sr = 0.0;
    for (int s = 0; s < nsplit; ++s)
      sr += partial[(((long)om_i * nsplit + s) * n_tiles + tile_id) *
                        (long)kRT * kRT + e];
    double *d1 = o + 2L * ((long)g * ncol + gp);
    double *d2 = o + 2L * ((long)gp * ncol + g);
    if (beta) {
      d1[0] += sr;
      if (g != gp) d2[0] += sr;
    } else {
      d1[0] = sr;
      d1[1] = 0.0;
      if (g != gp) {
        d2[0] = sr;
        d2[1] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------- GEMM f64
//
// C = A B for real operands: A m x k (row stride lda), B k x n (row stride
// ldb), C m x n (row stride ldc); k and n multiples of 128 (zero padded).
// Grid: m tiles x n tiles of 128 x 128.
__global__ __launch_bounds__(kSyrkThreads) void gemm_real_f64_kernel(
    const double *__restrict__ A, long lda, const double *__restrict__ B,
    long ldb, double *__restrict__ C, long ldc, long m, int k, int n_tiles) {
  __shared__ double As[kRK][kRT + kRPad];  // [k][m]
  __shared__ double Bs[kRK][kRT + kRPad];  // [k][n]
  const int mt = blockIdx.x / n_tiles, nt = blockIdx.x % n_tiles;
  const long M0 = (long)mt * kRT;
  const int N0 = nt * kRT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // 2 x 4 waves of 64 x 32 (as the SYRK)
  const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
  d4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  // A: 128 rows x 16 k: thread -> (row t/4, k (t%4)*4 .. +4);
  // B: 16 k x 128 cols: thread -> (k t/32, cols (t%32)*4 .. +4)
  const int arow = threadIdx.x >> 2, akq = (threadIdx.x & 3) * 4;
  const int bkr = threadIdx.x >> 5, bcq = (threadIdx.x & 31) * 4;
  double2 av[2], bv[2];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
    const long r = M0 + arow;
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = make_double2(0.0, 0.0);
    if (r < m) {
      const double *src = A + r * lda + k0 + akq;
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = *reinterpret_cast<const double2 *>(src + 2 * x);
    }
    const double *sb = B + (long)(k0 + bkr) * ldb + N0 + bcq;
#pragma unroll
    for (int x = 0; x < 2; ++x) bv[x] = *reinterpret_cast<const double2 *>(sb + 2 * x);
  };
  fetch(0);
  for (int k0 = 0; k0 < k; k0 += kRK) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      As[akq + 2 * x][arow] = av[x].x;
      As[akq + 2 * x + 1][arow] = av[x].y;
      Bs[bkr][bcq + 2 * x] = bv[x].x;
      Bs[bkr][bcq + 2 * x + 1] = bv[x].y;
    }
    __syncthreads();
    if (k0 + kRK < k) fetch(k0 + kRK);
#pragma unroll
    for (int ks = 0; ks < kRK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const int cl = lane & 15;
      double a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kr][wr + i * 16 + cl];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wc + j * 16 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma64(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long r = M0 + wr + i * 16 + acc_row(lane, e);
        const int c = N0 + wc + j * 16 + acc_col(lane);
        if (r < m) C[r * ldc + c] = acc[i][j][e];
      }
}

// ---------------------------------------------------------------- layout

// Packed coefficients: bands [0, nv) copied; packed band nv + q holds
// c_{c0 + 2q} + i c_{c0 + 2q + 1} (the second term only while < n_b).
// Layout: one band per row of n_pw complex values.
__global__ void pack_coeff_kernel(const double2 *__restrict__ c, int n_pw,
                                  int nv, int c0, int n_b, int n_pack,
                                  double2 *__restrict__ out) {
  const long total = (long)(nv + n_pack) * n_pw;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int row = (int)(idx / n_pw), pw = (int)(idx % n_pw);
    if (row < nv) {
      out[idx] = c[(long)row * n_pw + pw];
      continue;
    }
    const int b1 = c0 + 2 * (row - nv), b2 = b1 + 1;
    const double2 x = c[(long)b1 * n_pw + pw];
    double2 y = make_double2(0.0, 0.0);
    if (b2 < n_b) y = c[(long)b2 * n_pw + pw];
    // x + i y
    out[idx] = make_double2(x.x - y.y, x.y + y.x);
  }
}

// Real pair rows from packed ones.  F: rows q = v nc2 + cp (nvb x nc2),
// planar (2 ld doubles).  W: rows p = v n_c + c, ld doubles: column j < nh
// the cos part of G = hpos[j], nh <= j < 2 nh the sin part; the rest 0.
// hpos[j] / hneg[j]: indices of G and -G.
__global__ void unpack_real_kernel(const double *__restrict__ f, int nvb,
                                   int n_c, int nc2, int ld, int nh,
                                   const int *__restrict__ hpos,
                                   const int *__restrict__ hneg,
                                   double *__restrict__ w) {
  const long rows = (long)nvb * n_c;
  const long total = rows * ld;
  const double r2 = 0.70710678118654752440;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long p = idx / ld;
    const int j = (int)(idx % ld);
    double val = 0.0;
    if (j < 2 * nh) {
      const int v = (int)(p / n_c), c = (int)(p % n_c);
      const double *fr = f + ((long)v * nc2 + c / 2) * 2L * ld;
      const int jj = j < nh ? j : j - nh;
      const int gp = hpos[jj], gn = hneg[jj];
      const double ar = fr[gp], ai = fr[ld + gp];  // F(G)
      const double br = fr[gn], bi = fr[ld + gn];  // F(-G)
      const bool second = c & 1, sin_part = j >= nh;
      if (!second)
        val = sin_part ? (ai - bi) * r2 : (ar + br) * r2;
      else
        val = sin_part ? (br - ar) * r2 : (ai + bi) * r2;
    }
    w[idx] = val;
  }
}

// Complex plane-wave pair rows from packed ones (for export): row
// p = v n_c + c, planar ld: M_c1(G) = (F(G) + conj F(-G))/2,
// M_c2(G) = (F(G) - conj F(-G))/2i; neg[g] = index of -G.
__global__ void unpack_pw_kernel(const double *__restrict__ f, int nvb, int n_c,
                                 int nc2, int ld, int n_g,
                                 const int *__restrict__ neg,
                                 double *__restrict__ m) {
  const long total = (long)nvb * n_c * ld;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long p = idx / ld;
    const int g = (int)(idx % ld);
    double re = 0.0, im = 0.0;
    if (g < n_g) {
      const int v = (int)(p / n_c), c = (int)(p % n_c);
      const double *fr = f + ((long)v * nc2 + c / 2) * 2L * ld;
      const int gn = neg[g];
      const double ar = fr[g], ai = fr[ld + g], br = fr[gn], bi = fr[ld + gn];
      if (!(c & 1)) {
        re = 0.5 * (ar + br);
        im = 0.5 * (ai - bi);
      } else {
        // (F - conj F(-G)) / 2i = ((ai + bi) - i (ar - br)) / 2
        re = 0.5 * (ai + bi);
        im = -0.5 * (ar - br);
      }
    }
    m[p * 2L * ld + g] = re;
    m[p * 2L * ld + ld + g] = im;
  }
}

// chi in the plane-wave basis from the real-basis matrix (interleaved,
// imaginary part 0): for G1 = s1 H1, G2 = s2 H2 (s = +-1),
// chi(G1, G2) = [C_cc + i s2 C_cs - i s1 C_sc + s1 s2 C_ss] / 2.
// hj[g] = index j of H in the half list, hs[g] = +1 for G = H, -1 for -H.
__global__ void real_to_pw_sym_kernel(const double *__restrict__ cr, int n,
                                      int nh, const int *__restrict__ hj,
                                      const int *__restrict__ hs,
                                      double *__restrict__ out) {
  const long total = (long)n * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int g1 = (int)(idx / n), g2 = (int)(idx % n);
    const int j1 = hj[g1], j2 = hj[g2];
    const double s1 = hs[g1], s2 = hs[g2];
    auto at = [&](int a, int b) { return cr[2 * ((long)a * n + b)]; };
    const double cc = at(j1, j2), cs = at(j1, nh + j2), sc = at(nh + j1, j2),
                 ss = at(nh + j1, nh + j2);
    out[2 * idx] = 0.5 * (cc + s1 * s2 * ss);
    out[2 * idx + 1] = 0.5 * (s2 * cs - s1 * sc);
  }
}

// Basis vectors to the plane-wave basis: x (planar rows, real part only,
// ld_e) -> y (interleaved n_g x n_eig): y(G) = (a - i s b) / sqrt 2 with
// a = x[hj], b = x[nh + hj], s = hs[G].
__global__ void real_basis_to_pw_kernel(const double *__restrict__ x, int ld_e,
                                        int n_g, int n_eig, int nh,
                                        const int *__restrict__ hj,
                                        const int *__restrict__ hs,
                                        double *__restrict__ y) {
  const long total = (long)n_g * n_eig;
  const double r2 = 0.70710678118654752440;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int g = (int)(idx / n_eig), e = (int)(idx % n_eig);
    const double a = x[(long)hj[g] * 2 * ld_e + e];
    const double b = x[(long)(nh + hj[g]) * 2 * ld_e + e];
    y[2 * idx] = a * r2;
    y[2 * idx + 1] = -hs[g] * b * r2;
  }
}

// Orbitals for export: band n < nv from row n; band n >= nv from packed row
// nv + (n - c0)/2, real or imaginary part (then a real orbital).
__global__ void unpack_orbitals_kernel(const double2 *__restrict__ psi, long box,
                                       int nv, int c0, int n_b,
                                       double2 *__restrict__ out) {
  const long total = (long)n_b * box;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int n = (int)(idx / box);
    const long r = idx % box;
    if (n < nv) {
      out[idx] = psi[(long)n * box + r];
    } else {
      const double2 z = psi[(long)(nv + (n - c0) / 2) * box + r];
      out[idx] = make_double2(((n - c0) & 1) ? z.y : z.x, 0.0);
    }
  }
}

// Largest |c_n(-G) - conj c_n(G)| per work-group (real-orbital check).
__global__ void real_check_kernel(const double2 *__restrict__ c, int n_pw,
                                  int n_b, const int *__restrict__ negpw,
                                  double *__restrict__ blockmax) {
  __shared__ double red[256];
  const long total = (long)n_pw * n_b;
  double m = 0.0;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long row = idx / n_pw;
    const int pw = (int)(idx % n_pw);
    const double2 a = c[idx], b = c[row * n_pw + negpw[pw]];
    m = fmax(m, fmax(fabs(b.x - a.x), fabs(b.y + a.y)));
    m = fmax(m, fmax(fabs(a.x), fabs(a.y)) * 0.0);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

unsigned grid_for(long n) {
  return (unsigned)std::max(1L, std::min((n + 255) / 256, 65536L));
}

struct SyrkPlan {
  int T, n_tiles;
  long nsplit, kchunk;
  size_t bytes;
};

SyrkPlan syrk_plan(const HerkArgs &h) {
  SyrkPlan p{};
  p.T = h.ld / kRT;
  p.n_tiles = p.T * (p.T + 1) / 2;
  const long per_split = (long)p.n_tiles * h.n_omega;
  // resident blocks: 2 per CU (224 VGPRs each)
  const long resident = 512;
  const long kr = std::max(1L, (h.k + kRK - 1) / kRK);
  const long smax =
      std::max(1L, std::min(kr / 8, std::max(4L, 4 * resident / std::max(1L, per_split))));
  long nsplit = 1;
  double best = 0.0;
  for (long sp = 1; sp <= smax; ++sp) {
    const long blocks = per_split * sp;
    const long waves = (blocks + resident - 1) / resident;
    const double fill = (double)blocks / (double)(waves * resident);
    if (fill >= 0.95) {
      nsplit = sp;
      break;
    }
    if (fill > best + 1e-12) {
      best = fill;
      nsplit = sp;
    }
  }
  p.kchunk = ((kr + nsplit - 1) / nsplit) * kRK;
  p.nsplit = std::max(1L, (h.k + p.kchunk - 1) / p.kchunk);
  p.bytes = sizeof(double) * (size_t)kRT * kRT * p.n_tiles * p.nsplit * h.n_omega;
  return p;
}

}  // namespace

size_t syrk_f64_workspace(const HerkArgs &h) { return syrk_plan(h).bytes; }

void syrk(Context *ctx, const HerkArgs &h, double *out, long out_stride,
          int beta, DevBuf &ws, hipStream_t s) {
  SSRPA_REQUIRE(h.ld % kRT == 0 && h.ncol <= h.ld, SSRPA_ERR_ARG,
                "syrk: bad padding");
  SSRPA_REQUIRE(h.n_omega >= 1 && h.n_omega <= 65535, SSRPA_ERR_ARG,
                "syrk: bad frequency count");
  const SyrkPlan p = syrk_plan(h);
  ws.ensure(ctx, p.bytes, s);
  if (h.k > 0) {
    const int ti = (h.timer && h.timer->on) ? h.timer->start(h.stage, s) : -1;
    hipLaunchKernelGGL(syrk_f64_kernel,
                       dim3(p.n_tiles, (unsigned)p.nsplit, h.n_omega), dim3(kSyrkThreads),
                       0, s, h, p.T, p.n_tiles, p.kchunk, ws.as<double>());
    SSRPA_HIP(hipGetLastError());
    if (ti >= 0) h.timer->stop(ti, s);
  } else {
    fill_zero(ws.as(), p.bytes, s);
  }
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(p.n_tiles, h.n_omega), dim3(256), 0,
                     s, ws.as<double>(), p.T, p.n_tiles, (int)p.nsplit, h.ncol, out,
                     out_stride, beta);
  SSRPA_HIP(hipGetLastError());
}

void gemm_real(const double *a, long lda, const double *b, long ldb, double *c,
               long ldc, long m, int k, int n, hipStream_t s) {
  SSRPA_REQUIRE(k % kRT == 0 && n % kRT == 0, SSRPA_ERR_ARG,
                "gemm_real: k and n must be padded to 128");
  if (m <= 0) return;
  const long m_tiles = (m + kRT - 1) / kRT;
  const int n_tiles = n / kRT;
  SSRPA_REQUIRE(m_tiles * n_tiles < (1L << 31), SSRPA_ERR_ARG, "gemm too large");
  hipLaunchKernelGGL(gemm_real_f64_kernel, dim3((unsigned)(m_tiles * n_tiles)),
                     dim3(kSyrkThreads), 0, s, a, lda, b, ldb, c, ldc, m, k, n_tiles);
  SSRPA_HIP(hipGetLastError());
}

void pack_coefficients(const double *coeff, int n_pw, int nv, int c0, int n_b,
                       int n_pack, double *out, hipStream_t s) {
  const long total = (long)(nv + n_pack) * n_pw;
  hipLaunchKernelGGL(pack_coeff_kernel, dim3(grid_for(total)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(coeff), n_pw, nv, c0, n_b,
                     n_pack, reinterpret_cast<double2 *>(out));
  SSRPA_HIP(hipGetLastError());
}

void unpack_real_rows(const double *f, int nvb, int n_c, int ld, int nh,
                      const int *hpos, const int *hneg, double *w,
                      hipStream_t s) {
  const long total = (long)nvb * n_c * ld;
  hipLaunchKernelGGL(unpack_real_kernel, dim3(grid_for(total)), dim3(256), 0, s,
                     f, nvb, n_c, (n_c + 1) / 2, ld, nh, hpos, hneg, w);
  SSRPA_HIP(hipGetLastError());
}

void unpack_pw_rows(const double *f, int nvb, int n_c, int ld, int n_g,
                    const int *neg, double *m, hipStream_t s) {
  const long total = (long)nvb * n_c * ld;
  hipLaunchKernelGGL(unpack_pw_kernel, dim3(grid_for(total)), dim3(256), 0, s, f,
                     nvb, n_c, (n_c + 1) / 2, ld, n_g, neg, m);
  SSRPA_HIP(hipGetLastError());
}

void real_to_pw_sym(const double *cr, int n, int nh, const int *hj,
                    const int *hs, double *out, hipStream_t s) {
  hipLaunchKernelGGL(real_to_pw_sym_kernel, dim3(grid_for((long)n * n)),
                     dim3(256), 0, s, cr, n, nh, hj, hs, out);
  SSRPA_HIP(hipGetLastError());
}

void real_basis_to_pw(const double *x, int ld_e, int n_g, int n_eig, int nh,
                      const int *hj, const int *hs, double *y, hipStream_t s) {
  hipLaunchKernelGGL(real_basis_to_pw_kernel, dim3(grid_for((long)n_g * n_eig)),
                     dim3(256), 0, s, x, ld_e, n_g, n_eig, nh, hj, hs, y);
  SSRPA_HIP(hipGetLastError());
}

void unpack_orbitals(const double *psi, long box, int nv, int c0, int n_b,
                     double *out, hipStream_t s) {
  hipLaunchKernelGGL(unpack_orbitals_kernel, dim3(grid_for((long)n_b * box)),
                     dim3(256), 0, s, reinterpret_cast<const double2 *>(psi), box,
                     nv, c0, n_b, reinterpret_cast<double2 *>(out));
  SSRPA_HIP(hipGetLastError());
}

int real_check_blocks() { return 512; }

void real_check(const double *coeff, int n_pw, int n_b, const int *negpw,
                double *blockmax, hipStream_t s) {
  hipLaunchKernelGGL(real_check_kernel, dim3(real_check_blocks()), dim3(256), 0,
                     s, reinterpret_cast<const double2 *>(coeff), n_pw, n_b,
                     negpw, blockmax);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
