// FFT stage: orbital staging (coefficients -> real-space grid) and the fused
// pair-density transform that produces the plane-wave matrix elements
//   M_vc(G) = <psi_v| e^{iG.r} |psi_c>            (paper, Method, Eq. 3)
// as the grid sum (Omega/N) sum_j conj(psi_v(r_j)) psi_c(r_j) e^{iG.r_j},
// which is exact when the grid satisfies the alias-free bound.
//
// Both transforms use a mixed-radix (4, 2, 3) Stockham FFT that runs on
// batches of lines held in LDS, with natural-order output and twiddles read
// from an LDS table e^{2 pi i t / N}.
#include <cmath>

#include "internal.hpp"

namespace ssrpa {

namespace {

constexpr int kMaxRad = 8;

struct Radices {
  int n;
  int r[kMaxRad];
};

Radices factor(int N) {
  Radices f{};
  int m = N;
  while (m % 4 == 0) { f.r[f.n++] = 4; m /= 4; }
  while (m % 2 == 0) { f.r[f.n++] = 2; m /= 2; }
  while (m % 3 == 0) { f.r[f.n++] = 3; m /= 3; }
  if (m != 1 || f.n > kMaxRad)
    fail(SSRPA_ERR_ARG, "FFT length %d is not of the form 2^i 3^j", N);
  return f;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// i * a
__device__ __forceinline__ double2 cmuli(double2 a) {
  return make_double2(-a.y, a.x);
}

// In-register radix-R DFT, y_k = sum_j v_j e^{+2 pi i jk / R}.
template <int R>
__device__ __forceinline__ void radix_dft(const double2 *v, double2 *y) {
  if constexpr (R == 2) {
    y[0] = cadd(v[0], v[1]);
    y[1] = csub(v[0], v[1]);
  } else if constexpr (R == 4) {
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = cmuli(csub(v[1], v[3]));
    y[0] = cadd(s02, s13);
    y[2] = csub(s02, s13);
    y[1] = cadd(d02, d13);
    y[3] = csub(d02, d13);
  } else {  // R == 3, w = e^{2 pi i / 3}
    const double c = -0.5;
    const double sq = 0.86602540378443864676;  // sqrt(3)/2
    const double2 t1 = cadd(v[1], v[2]);
    const double2 t2 = csub(v[1], v[2]);
    const double2 m = make_double2(v[0].x + c * t1.x, v[0].y + c * t1.y);
    const double2 r = make_double2(-sq * t2.y, sq * t2.x);  // i sq t2
    y[0] = cadd(v[0], t1);
    y[1] = cadd(m, r);
    y[2] = csub(m, r);
  }
}

// One Stockham pass of radix R over `nlines` lines of length N (line stride
// ls) from `in` to `out`; Ns = product of the radices of earlier passes.
// X[k] = sum_j x[j] e^{+2 pi i jk / N}.
template <int R>
__device__ __forceinline__ void stockham_pass(const double2 *in, double2 *out,
                                              int nlines, int ls, int N,
                                              int Ns, const double2 *tw) {
  const int nb = N / R;          // butterflies per line
  const int total = nlines * nb;
  const int stride = N / (Ns * R);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int line = idx / nb;
    const int j = idx - line * nb;
    const int k = j % Ns;
    const double2 *src = in + line * ls + j;
    double2 v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = src[i * nb];
#pragma unroll
    for (int i = 1; i < R; ++i) {
      const int t = (k * i * stride) % N;
      v[i] = cmul(v[i], tw[t]);
    }
    double2 y[R];
    radix_dft<R>(v, y);
    double2 *dst = out + line * ls + (j / Ns) * Ns * R + k;
#pragma unroll
    for (int i = 0; i < R; ++i) dst[i * Ns] = y[i];
  }
}

// Transform the lines in `a` (ping-pong with `b`); returns the buffer that
// holds the result.  Synchronizes the block before and after each pass.
__device__ double2 *lds_fft(double2 *a, double2 *b, int nlines, int ls, int N,
                            const Radices &rad, const double2 *tw) {
  int Ns = 1;
  for (int s = 0; s < rad.n; ++s) {
    __syncthreads();
    const int R = rad.r[s];
    if (R == 4)
      stockham_pass<4>(a, b, nlines, ls, N, Ns, tw);
    else if (R == 2)
      stockham_pass<2>(a, b, nlines, ls, N, Ns, tw);
    else
      stockham_pass<3>(a, b, nlines, ls, N, Ns, tw);
    Ns *= R;
    double2 *t = a; a = b; b = t;
  }
  __syncthreads();
  return a;
}

// ------------------------------------------------------------ orbital FFT

__global__ void scatter_coeff_kernel(const double2 *__restrict__ coeff,
                                     const int *__restrict__ box_index,
                                     int n_pw, int n_b, long box,
                                     double2 *__restrict__ out) {
  const long total = (long)n_pw * n_b;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const long band = i / n_pw;
    const int pw = (int)(i - band * n_pw);
    out[band * box + box_index[pw]] = coeff[i];
  }
}

// Lines: element e of line (o, i) at o*outer + i*inner + e*elem.  A block
// handles `L` consecutive inner indices of one outer index.
__global__ __launch_bounds__(256) void fft_lines_kernel(
    double2 *__restrict__ data, int N, long elem, long inner, int n_inner,
    long outer, Radices rad, const double2 *__restrict__ tw_g, int L,
    double scale) {
  extern __shared__ double2 smem[];
  double2 *tw = smem;
  double2 *a = smem + N;
  double2 *b = a + L * N;
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = tw_g[t];
  const int tiles = (n_inner + L - 1) / L;
  const long o = blockIdx.x / tiles;
  const int i0 = (blockIdx.x % tiles) * L;
  const int nl = min(L, n_inner - i0);
  double2 *base = data + o * outer + i0 * inner;
  const int tot = nl * N;
  if (elem == 1) {
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int line = idx / N, e = idx - line * N;
      a[line * N + e] = base[line * inner + e];
    }
  } else {
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int e = idx / nl, line = idx - e * nl;
      a[line * N + e] = base[line * inner + e * elem];
    }
  }
  double2 *r = lds_fft(a, b, nl, N, N, rad, tw);
  if (elem == 1) {
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int line = idx / N, e = idx - line * N;
      const double2 v = r[line * N + e];
      base[line * inner + e] = make_double2(v.x * scale, v.y * scale);
    }
  } else {
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int e = idx / nl, line = idx - e * nl;
      const double2 v = r[line * N + e];
      base[line * inner + e * elem] = make_double2(v.x * scale, v.y * scale);
    }
  }
}

void fft_lines(double2 *data, int N, long elem, long inner, int n_inner,
               long outer, long n_outer, const double2 *tw, double scale,
               hipStream_t s) {
  const Radices rad = factor(N);
  const int L = 16;
  const int tiles = (n_inner + L - 1) / L;
  const long blocks = n_outer * tiles;
  SSRPA_REQUIRE(blocks < (1L << 31), SSRPA_ERR_ARG, "FFT grid too large");
  const size_t shmem = sizeof(double2) * (N + 2 * L * N);
  hipLaunchKernelGGL(fft_lines_kernel, dim3((unsigned)blocks), dim3(256),
                     shmem, s, data, N, elem, inner, n_inner, outer, rad, tw,
                     L, scale);
  SSRPA_HIP(hipGetLastError());
}

// ------------------------------------------------------- fused pair FFT

constexpr int kPairThreads = 256;
constexpr int kTileV = 8;
constexpr int kTileC = 32;

struct PairGeo {
  int n1, n2, n3, m1;
  int lx;           // x lines per LDS batch
  Radices r1, r2;
};

// Generic fused kernel for grids without a compile-time schedule (N1 != N2,
// or a length outside the staged set): one block per (v, c) pair.  For every
// z-plane j3: pair density of the plane, x transforms (in batches of lx
// lines) pruned to |n1| <= m1, y transforms of those columns, then the z sum
// for the chi0 G vectors is accumulated in registers:
// acc(G) += Y(n1, n2; j3) e^{2 pi i n3 j3 / N3}.
template <int GPT>
__global__ __launch_bounds__(kPairThreads) void pair_fft_kernel(
    const double2 *__restrict__ psi, const double2 *__restrict__ psi_c,
    PairGeo geo, int v0, int nvb, int n_v,
    int n_c, const int *__restrict__ gcol, const double *__restrict__ gscale,
    int n_g, int ld_g, const double2 *__restrict__ tw_g,
    double *__restrict__ w) {
  extern __shared__ double2 smem[];
  const int n1 = geo.n1, n2 = geo.n2;
  const int n3 = geo.n3, m1 = geo.m1, lx = geo.lx;
  const int ny = 2 * m1 + 1;
  double2 *tw1 = smem;
  double2 *tw2 = tw1 + n1;
  double2 *tw3 = tw2 + n2;
  double2 *xa = tw3 + n3;          // lx * n1  (also y ping-pong buffer)
  double2 *xb = xa + lx * n1;      // lx * n1
  double2 *yb = xb + lx * n1;      // ny * n2
  double2 *pz = yb + ny * n2;      // n3: e^{2 pi i k3 j3 / N3} of this plane
  for (int t = threadIdx.x; t < n1 + n2 + n3; t += blockDim.x) smem[t] = tw_g[t];

  // pair of this block: tiles of kTileV valence x kTileC conduction bands
  const int tiles_c = (n_c + kTileC - 1) / kTileC;
  const int tile = blockIdx.x / (kTileV * kTileC);
  const int q = blockIdx.x % (kTileV * kTileC);
  const int vl = (tile / tiles_c) * kTileV + q / kTileC;
  const int c = (tile % tiles_c) * kTileC + q % kTileC;
  if (vl >= nvb || c >= n_c) return;
  const long plane = (long)n1 * n2;
  const long box = plane * n3;
  const double2 *pv = psi + (long)(v0 + vl) * box;
  const double2 *pc = psi_c + (long)(n_v + c) * box;

  int code[GPT];
  double2 acc[GPT];
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int g = threadIdx.x + i * kPairThreads;
    code[i] = g < n_g ? gcol[g] : 0;
    acc[i] = make_double2(0.0, 0.0);
  }

  for (int j3 = 0; j3 < n3; ++j3) {
    const double2 *sv = pv + j3 * plane;
    const double2 *sc = pc + j3 * plane;
    for (int g0 = 0; g0 < n2; g0 += lx) {
      const int nl = min(lx, n2 - g0);
      __syncthreads();
      if (g0 == 0)
        for (int t = threadIdx.x; t < n3; t += blockDim.x) pz[t] = tw3[(t * j3) % n3];
      for (int idx = threadIdx.x; idx < nl * n1; idx += blockDim.x) {
        const double2 a = sv[(long)g0 * n1 + idx];
        const double2 b = sc[(long)g0 * n1 + idx];
        // conj(a) * b
        xa[idx] = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
      }
      const double2 *r = lds_fft(xa, xb, nl, n1, n1, geo.r1, tw1);
      for (int idx = threadIdx.x; idx < nl * ny; idx += blockDim.x) {
        const int line = idx / ny, qq = idx - line * ny;
        int k1 = qq - m1;
        if (k1 < 0) k1 += n1;
        yb[qq * n2 + g0 + line] = r[line * n1 + k1];
      }
    }
    const double2 *ry = lds_fft(yb, xa, ny, n2, n2, geo.r2, tw2);
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int g = threadIdx.x + i * kPairThreads;
      if (g < n_g) {
        const int col = code[i] & 0xFFFFF;
        const int k3 = code[i] >> 20;
        const double2 val = ry[col];
        const double2 t = pz[k3];
        acc[i].x += val.x * t.x - val.y * t.y;
        acc[i].y += val.x * t.y + val.y * t.x;
      }
    }
  }
  double *row = w + ((long)vl * n_c + c) * 2L * ld_g;
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int g = threadIdx.x + i * kPairThreads;
    if (g < n_g) {
      const double sc = gscale[g];
      row[g] = acc[i].x * sc;
      row[ld_g + g] = acc[i].y * sc;
    }
  }
  for (int g = n_g + threadIdx.x; g < ld_g; g += blockDim.x) {
    row[g] = 0.0;
    row[ld_g + g] = 0.0;
  }
}

// LDS ordering between lanes of one wave: a wavefront-scope fence pair
// around a wave barrier (no block-wide barrier needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------- staged pair transform
//
// Two kernels per chunk of pairs (same result as pair_fft_kernel):
//  * pair_plane_kernel forms the pair density conj(psi_v) psi_c of one
//    z-plane at a time and transforms it along x, then along y.  Each line of
//    length N = R1 R2 is split into an R1-point step and an R2-point step
//    computed in registers with one LDS exchange in between (decimation in
//    time: X[ka + R1 kb] = sum_b e^{2 pi i b kb / R2} e^{2 pi i b ka / N}
//    sum_a x[R2 a + b] e^{2 pi i a ka / R1}).  Only |n1| <= m1 survives the x
//    step and only the (n1, n2) columns that hold chi0 vectors are written,
//    to a stage Y[pair][j3][column] in HBM.
//  * pair_z_kernel forms, for every chi0 vector G = (n1, n2, n3),
//    sum_j3 Y[col(G)][j3] e^{2 pi i n3 j3 / N3}, scales it and writes W.

// cos and sin of 2 pi t / R for the register transforms (R divides 16, 12
// or 9); the arguments are compile-time constants after unrolling.
__host__ __device__ constexpr double tw_cos(int R, int t) {
  constexpr double c16[16] = {1.0, 0.9238795325112867, 0.7071067811865476,
                              0.3826834323650898, 0.0, -0.3826834323650898,
                              -0.7071067811865476, -0.9238795325112867, -1.0,
                              -0.9238795325112867, -0.7071067811865476,
                              -0.3826834323650898, 0.0, 0.3826834323650898,
                              0.7071067811865476, 0.9238795325112867};
  constexpr double c12[12] = {1.0, 0.8660254037844386, 0.5, 0.0, -0.5,
                              -0.8660254037844386, -1.0, -0.8660254037844386,
                              -0.5, 0.0, 0.5, 0.8660254037844386};
  constexpr double c9[9] = {1.0, 0.766044443118978, 0.17364817766693036, -0.5,
                            -0.9396926207859084, -0.9396926207859084, -0.5,
                            0.17364817766693036, 0.766044443118978};
  return 16 % R == 0 ? c16[t * (16 / R)]
                     : (12 % R == 0 ? c12[t * (12 / R)] : c9[t * (9 / R)]);
}
__host__ __device__ constexpr double tw_sin(int R, int t) {
  // sin(2 pi t / R) = cos(2 pi (t - R/4) / R), written out for R = 9
  constexpr double s9[9] = {0.0, 0.6427876096865394, 0.984807753012208,
                            0.8660254037844386, 0.3420201433256687,
                            -0.3420201433256687, -0.8660254037844386,
                            -0.984807753012208, -0.6427876096865394};
  return R % 4 == 0 ? tw_cos(R, (t + 3 * (R / 4)) % R)
                    : (12 % R == 0 ? tw_cos(12, ((t * (12 / R)) + 9) % 12)
                                   : s9[t * (9 / R)]);
}

// v e^{2 pi i t / R}, 0 <= t < R; exact for the multiples of pi/2 and pi/4.
template <int R>
__device__ __forceinline__ double2 rot(double2 v, int t) {
  constexpr double h = 0.70710678118654752440;
  if (t == 0) return v;
  if (2 * t == R) return make_double2(-v.x, -v.y);
  if (4 * t == R) return make_double2(-v.y, v.x);
  if (4 * t == 3 * R) return make_double2(v.y, -v.x);
  if (8 * t == R) return make_double2(h * (v.x - v.y), h * (v.x + v.y));
  if (8 * t == 3 * R) return make_double2(-h * (v.x + v.y), h * (v.x - v.y));
  if (8 * t == 5 * R) return make_double2(h * (v.y - v.x), -h * (v.x + v.y));
  if (8 * t == 7 * R) return make_double2(h * (v.x + v.y), h * (v.y - v.x));
  const double c = tw_cos(R, t), s = tw_sin(R, t);
  return make_double2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// In-register DFT of length R in place, y_k = sum_j v_j e^{+2 pi i jk / R};
// R = A B with A, B <= 4 by one Cooley-Tukey split.
template <int R>
__device__ __forceinline__ void dft(double2 *v) {
  if constexpr (R == 2 || R == 3 || R == 4) {
    double2 y[R];
    radix_dft<R>(v, y);
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = y[i];
  } else if constexpr (R > 4) {
    constexpr int A = R % 4 == 0 ? 4 : (R % 3 == 0 ? 3 : 2);
    constexpr int B = R / A;
    static_assert(A * B == R && B <= 4, "register DFT length");
    double2 t[R];  // t[ka * B + b]
#pragma unroll
    for (int b = 0; b < B; ++b) {
      double2 u[A];
#pragma unroll
      for (int a = 0; a < A; ++a) u[a] = v[B * a + b];
      dft<A>(u);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) t[ka * B + b] = rot<R>(u[ka], b * ka);
    }
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      double2 u[B];
#pragma unroll
      for (int b = 0; b < B; ++b) u[b] = t[ka * B + b];
      dft<B>(u);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) v[ka + A * kb] = u[kb];
    }
  }
}


// Lines per wave batch: fewest issue slots per line over the two steps
// (step 1 has R2 items per line, step 2 has R1).
constexpr int pick_lines(int r1, int r2) {
  int best = 1, bn = 1, bd = 1;  // best cost bn / bd
  for (int L = 1; L <= 16; ++L) {
    const int n = (L * r2 + 63) / 64 + (L * r1 + 63) / 64;
    if (n * bd < bn * L || L == 1) { best = L; bn = n; bd = L; }
  }
  return best;
}

// Waves per plane work-group: the x-line batches of a plane should divide
// evenly over the waves (measured: 3 waves for 6 batches at N = 48, 4 for
// 11 at N = 72, against 8 waves: -11 % and -15 % time); small work-groups
// also let more of them share a CU.
constexpr int plane_waves(int n_batches) {
  return n_batches <= 2 ? 2 : ((n_batches % 3 == 0 && n_batches % 4 != 0) ? 3 : 4);
}

template <int R1_, int R2_>
struct LineSplit {
  static constexpr int R1 = R1_, R2 = R2_, N = R1 * R2;
  static constexpr int SB = R2 | 1;      // odd stride between ka rows
  static constexpr int SL = R1 * SB;     // scratch per line
  static constexpr int XS = N | 1;       // odd row stride of the x output
  static constexpr int L = pick_lines(R1, R2);
  static constexpr bool kHoist = L * R2 <= 64;  // one step-1 item per lane
  static constexpr int W = plane_waves((N + L - 1) / L);  // plane kernel
};

// LDS bytes of pair_plane_kernel (tw, column map, nxo x outputs, scratch).
template <class S>
size_t plane_lds_bytes(int ny1, int ny2, int nxo) {
  const size_t cm = ((size_t)ny1 * ny2 * sizeof(int) + 15) / 16 * 16;
  return sizeof(double2) * (S::N + (size_t)nxo * ny1 * S::XS +
                            (size_t)S::W * S::L * S::SL) + cm;
}

// Work-group b -> pair (vl, cl) of a chunk of nvb x ncc pairs and z slab
// zs of nslab.  Work-groups are dealt round-robin to the eight XCDs; on each
// XCD consecutive ones walk an 8 x 8 tile of pairs for one slab of planes,
// then the same tile for the next slab, so the groups resident on one XCD
// share the planes of one slab of eight valence and eight conduction
// orbitals through its L2 (short slabs keep them from drifting apart).
#ifndef SSRPA_PLANE_SLABS
#define SSRPA_PLANE_SLABS 6
#endif
constexpr int kPlaneSlabs = SSRPA_PLANE_SLABS;  // z slabs per pair
__device__ __forceinline__ bool chunk_pair(int b, int nvb, int ncc, int nslab,
                                           int &vl, int &cl, int &zs) {
  const int tiles_c = (ncc + 7) >> 3;
  const int xcd = b & 7, s = b >> 3;
  const int r = s >> 6;
  const int tl = r / nslab;
  zs = r - tl * nslab;
  const int tile = tl * 8 + xcd;
  const int q = s & 63;
  const int tv = tile / tiles_c, tc = tile - tv * tiles_c;
  vl = tv * 8 + (q >> 3);
  cl = tc * 8 + (q & 7);
  return vl < nvb && cl < ncc;
}

// Step 1 of a batch of nl lines: item (line, b) loads x[R2 a + b] through
// `load`, transforms over a, twists by e^{2 pi i b ka / N} and stores to
// scr[line][ka][b].  Step 2: item (line, ka) transforms over b and hands
// X[ka + R1 kb] to `store`.
// With kLineFast the step-1 items run line-fastest (it = b * nl + line), so
// that lanes next to each other load neighbouring lines; the twiddles then
// come from the table.
template <class S, bool kLineFast = false, class Load, class Store>
__device__ __forceinline__ void line_batch(int nl, Load load, Store store,
                                           double2 *scr, const double2 *tw,
                                           const double2 *twh, int lane) {
  for (int it = lane; it < nl * S::R2; it += 64) {
    int line, b;
    if constexpr (kLineFast) {
      b = it / nl;
      line = it - b * nl;
    } else {
      line = it / S::R2;
      b = it - line * S::R2;
    }
    double2 x[S::R1];
#pragma unroll
    for (int a = 0; a < S::R1; ++a) x[a] = load(line, S::R2 * a + b);
    dft<S::R1>(x);
    double2 *d = scr + line * S::SL + b;
    d[0] = x[0];
#pragma unroll
    for (int ka = 1; ka < S::R1; ++ka)
      d[ka * S::SB] =
          cmul(x[ka], (S::kHoist && !kLineFast) ? twh[ka - 1] : tw[b * ka]);
  }
  wave_lds_sync();
  for (int it = lane; it < nl * S::R1; it += 64) {
    const int line = it / S::R1, ka = it - line * S::R1;
    double2 y[S::R2];
    const double2 *s = scr + line * S::SL + ka * S::SB;
#pragma unroll
    for (int b = 0; b < S::R2; ++b) y[b] = s[b];
    dft<S::R2>(y);
#pragma unroll
    for (int kb = 0; kb < S::R2; ++kb) store(line, ka + S::R1 * kb, y[kb]);
  }
  wave_lds_sync();
}

// One work-group per pair of the chunk; it walks the n3 planes.  With
// nxo = 2 the x outputs alternate between two buffers and one block barrier
// per plane suffices; with nxo = 1 a second barrier guards the buffer.
template <int R1, int R2>
__global__ __launch_bounds__((64 * LineSplit<R1, R2>::W)) void pair_plane_kernel(
    const double2 *__restrict__ psi, const double2 *__restrict__ psi_c, int v0,
    int nvb, int n_v, int c0,
    int ncc, int n3, int nslab, int m1, int m2, int nxo, const int *__restrict__ cmap_g,
    int ldy, const double2 *__restrict__ tw_g, double2 *__restrict__ yst) {
  using S = LineSplit<R1, R2>;
  constexpr int N = S::N;
  extern __shared__ double2 smem[];
  const int ny1 = 2 * m1 + 1, ny2 = 2 * m2 + 1;
  double2 *tw = smem;
  double2 *xo0 = tw + N;
  double2 *scr_all = xo0 + nxo * ny1 * S::XS;
  int *cmap = reinterpret_cast<int *>(scr_all + S::W * S::L * S::SL);
  int vl, cl, zs;
  if (!chunk_pair(blockIdx.x, nvb, ncc, nslab, vl, cl, zs)) return;
  const int pz = (n3 + nslab - 1) / nslab;
  const int z0 = zs * pz, z1 = min(n3, z0 + pz);
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = tw_g[t];
  for (int t = threadIdx.x; t < ny1 * ny2; t += blockDim.x) cmap[t] = cmap_g[t];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double2 *scr = scr_all + wave * S::L * S::SL;
  // twiddles of this lane's step-1 item, when each lane has one
  double2 twh[S::R1 > 1 ? S::R1 - 1 : 1];
  if constexpr (S::kHoist) {
    const int b = lane % S::R2;
#pragma unroll
    for (int ka = 1; ka < S::R1; ++ka) twh[ka - 1] = tw_g[b * ka];
  }
  const long plane = (long)N * N;
  const long box = plane * n3;
  const double2 *pv = psi + (long)(v0 + vl) * box;
  const double2 *pc = psi_c + (long)(n_v + c0 + cl) * box;
  double2 *yp = yst + ((long)vl * ncc + cl) * n3 * (long)ldy;
  constexpr int nbx = (N + S::L - 1) / S::L;
  const int nby = (ny1 + S::L - 1) / S::L;
  __syncthreads();
  for (int j3 = z0; j3 < z1; ++j3) {
    double2 *xo = xo0 + (nxo == 2 ? (j3 & 1) : 0) * ny1 * S::XS;
    const double2 *sv = pv + j3 * plane;
    const double2 *sc = pc + j3 * plane;
    for (int bt = wave; bt < nbx; bt += S::W) {
      const int l0 = bt * S::L;
      const int nl = min(S::L, N - l0);
      line_batch<S>(
          nl,
          [&](int line, int j) {
            const long o = (long)(l0 + line) * N + j;
            const double2 a = sv[o], d = sc[o];
            return make_double2(a.x * d.x + a.y * d.y, a.x * d.y - a.y * d.x);
          },
          [&](int line, int k, double2 v) {
            int kk = k + m1;
            if (kk >= N) kk -= N;
            if (kk < ny1) xo[kk * S::XS + l0 + line] = v;
          },
          scr, tw, twh, lane);
    }
    __syncthreads();
    double2 *yo = yp + (long)j3 * ldy;
    for (int bt = wave; bt < nby; bt += S::W) {
      const int r0 = bt * S::L;
      const int nl = min(S::L, ny1 - r0);
      line_batch<S>(
          nl, [&](int line, int j) { return xo[(r0 + line) * S::XS + j]; },
          [&](int line, int k, double2 v) {
            int kk = k + m2;
            if (kk >= N) kk -= N;
            if (kk < ny2) {
              const int col = cmap[(r0 + line) * ny2 + kk];
              if (col >= 0) yo[col] = v;
            }
          },
          scr, tw, twh, lane);
    }
    if (nxo == 1) __syncthreads();
  }
}

// z transform of the stage for N3 = R1 R2: each wave takes L neighbouring
// columns of one pair (four waves per work-group), transforms them along j3
// and writes the chi0 vectors of each column, zcol[col] = (first G, lowest
// n3, highest n3, gap): G = first + n3 - lowest, less one above n3 = 0 in
// the (0, 0) column (gap = 1), which has no G = 0.
constexpr int kZWaves = 4;
template <int R1, int R2>
__global__ __launch_bounds__(64 * kZWaves) void pair_zfft_kernel(
    const double2 *__restrict__ yst, int ncc, int c0, int n_c, int ncol,
    int ldy, int nblk, const int4 *__restrict__ zcol,
    const double *__restrict__ gscale, int n_g, int ld_g,
    const double2 *__restrict__ tw3_g, double *__restrict__ w) {
  using S = LineSplit<R1, R2>;
  constexpr int N = S::N;
  extern __shared__ double2 zsm[];
  double2 *tw = zsm;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double2 *scr = zsm + N + wave * S::L * S::SL;
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t] = tw3_g[t];
  const int q = blockIdx.x / nblk, blk = blockIdx.x - q * nblk;
  const int vl = q / ncc, cl = q - vl * ncc;
  const double2 *yp = yst + (long)q * N * ldy;
  double *row = w + ((long)vl * n_c + c0 + cl) * 2L * ld_g;
  if (blk == 0)
    for (int g = n_g + threadIdx.x; g < ld_g; g += blockDim.x) {
      row[g] = 0.0;
      row[ld_g + g] = 0.0;
    }
  __syncthreads();
  const int cb = (blk * kZWaves + wave) * S::L;
  if (cb >= ncol) return;
  const int nl = min(S::L, ncol - cb);
  const int half = N / 2;
  line_batch<S, true>(
      nl, [&](int line, int j) { return yp[(long)j * ldy + cb + line]; },
      [&](int line, int k, double2 v) {
        const int4 zc = zcol[cb + line];
        const int n3 = k <= half ? k : k - N;
        if (n3 >= zc.y && n3 <= zc.z && !(zc.w && n3 == 0)) {
          const int g = zc.x + n3 - zc.y - (zc.w && n3 > 0 ? 1 : 0);
          const double s = gscale[g];
          row[g] = v.x * s;
          row[ld_g + g] = v.y * s;
        }
      },
      scr, tw, nullptr, lane);
}

// One work-group per pair of the chunk: the z sums of its chi0 vectors
// (direct sum, for N3 without a staged split).
__global__ __launch_bounds__(256) void pair_z_kernel(
    const double2 *__restrict__ yst, int ncc, int c0, int n_c, int n3, int ldy,
    const int *__restrict__ zcode, const double *__restrict__ gscale, int n_g,
    int ld_g, const double2 *__restrict__ tw3_g, double *__restrict__ w) {
  extern __shared__ double2 tw3[];
  for (int t = threadIdx.x; t < n3; t += blockDim.x) tw3[t] = tw3_g[t];
  __syncthreads();
  const int q = blockIdx.x;
  const int vl = q / ncc, cl = q - vl * ncc;
  const double2 *yp = yst + (long)q * n3 * ldy;
  double *row = w + ((long)vl * n_c + c0 + cl) * 2L * ld_g;
  for (int g = threadIdx.x; g < n_g; g += blockDim.x) {
    const int code = zcode[g];
    const int col = code & 0xFFFFF, k3 = code >> 20;
    const double2 *src = yp + col;
    double2 acc = make_double2(0.0, 0.0);
    int t = 0;
#pragma unroll 8
    for (int j3 = 0; j3 < n3; ++j3) {
      const double2 v = src[(long)j3 * ldy];
      const double2 p = tw3[t];
      acc.x += v.x * p.x - v.y * p.y;
      acc.y += v.x * p.y + v.y * p.x;
      t += k3;
      if (t >= n3) t -= n3;
    }
    const double s = gscale[g];
    row[g] = acc.x * s;
    row[ld_g + g] = acc.y * s;
  }
  for (int g = n_g + threadIdx.x; g < ld_g; g += blockDim.x) {
    row[g] = 0.0;
    row[ld_g + g] = 0.0;
  }
}
}  // namespace

void upload_twiddles(System &sys, hipStream_t s) {
  const Geometry &g = sys.geo;
  const int lens[3] = {g.n1, g.n2, g.n3};
  std::vector<double> &tw = sys.fft_tw_host;
  tw.clear();
  for (int d = 0; d < 3; ++d) {
    const int N = lens[d];
    for (int t = 0; t < N; ++t) {
      // exact values at the symmetric points keep the tables symmetric
      const long double ang = 2.0L * 3.14159265358979323846264338327950288L *
                              (long double)t / (long double)N;
      tw.push_back((double)cosl(ang));
      tw.push_back((double)sinl(ang));
    }
  }
  sys.fft_tw = DevBuf(sys.ctx, tw.size() * sizeof(double));
  SSRPA_HIP(hipMemcpyAsync(sys.fft_tw.as(), tw.data(), tw.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
}

void launch_orbital_fft(System &sys, const double *coeff_dev,
                        const int *box_index_dev, hipStream_t s) {
  const Geometry &g = sys.geo;
  const long box = (long)g.n1 * g.n2 * g.n3;
  double2 *psi = sys.psi_r.as<double2>();
  fill_zero(psi, sizeof(double2) * box * sys.n_orb, s);
  const long total = (long)sys.n_pw * sys.n_orb;
  const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(scatter_coeff_kernel, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(coeff_dev),
                     box_index_dev, sys.n_pw, sys.n_orb, box, psi);
  SSRPA_HIP(hipGetLastError());
  const double2 *tw = sys.fft_tw.as<double2>();
  const long plane = (long)g.n1 * g.n2;
  // x lines: contiguous; y lines: stride n1; z lines: stride n1*n2
  fft_lines(psi, g.n1, 1, g.n1, g.n2, plane, (long)sys.n_orb * g.n3, tw, 1.0, s);
  fft_lines(psi, g.n2, g.n1, 1, g.n1, plane, (long)sys.n_orb * g.n3,
            tw + g.n1, 1.0, s);
  fft_lines(psi, g.n3, plane, 1, (int)plane, box, sys.n_orb, tw + g.n1 + g.n2,
            1.0 / std::sqrt(g.volume), s);
}

namespace {

// Staged transform of one valence block: chunks of nvb x ncc pairs.
template <int R1, int R2>
void staged_pairs(System &sys, int v0, int nvb, const double *gscale,
                  double *w, hipStream_t s) {
  using S = LineSplit<R1, R2>;
  const Geometry &g = sys.geo;
  const int ny1 = 2 * g.m1 + 1, ny2 = 2 * g.m2 + 1;
  const size_t ypp = stage_bytes_per_pair(g);
  const int ncc_max = stage_chunk_c(nvb, sys.orb_nc, ypp);
  sys.ystage.ensure(sys.ctx, (size_t)nvb * ncc_max * ypp, s);
  // double-buffer the x outputs when that costs no work-groups per CU
  const size_t l1 = plane_lds_bytes<S>(ny1, ny2, 1);
  const size_t l2 = plane_lds_bytes<S>(ny1, ny2, 2);
  const size_t cu = 160 * 1024;
  SSRPA_REQUIRE(l1 <= cu, SSRPA_ERR_ARG, "pair transform needs %zu bytes of LDS", l1);
  // a second x-output buffer saves one barrier per plane but costs LDS;
  // measured, the extra work-groups per CU win, so it is used only when it
  // costs none of them
  const int nxo = (l2 <= cu && cu / l2 >= cu / l1) ? 2 : 1;
  const size_t lds = nxo == 2 ? l2 : l1;
  auto kern = &pair_plane_kernel<R1, R2>;
  if (lds > 64 * 1024)
    SSRPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
  // valence and conduction orbitals: the system's own, or those of a pair
  // source (k and k + q of a k mesh)
  const double2 *psi = sys.src_psi_v
                            ? reinterpret_cast<const double2 *>(sys.src_psi_v)
                            : sys.psi_r.as<double2>();
  const double2 *psi_c = sys.src_psi_c
                              ? reinterpret_cast<const double2 *>(sys.src_psi_c)
                              : sys.psi_r.as<double2>();
  const double2 *tw = sys.fft_tw.as<double2>();
  double2 *yst = sys.ystage.as<double2>();
  // z: transform the columns when N3 has the same split, else direct sums
  const bool zfft = g.n3 == S::N && 2 * g.m3 + 1 <= g.n3;
  const int nblk = (g.ncol + kZWaves * S::L - 1) / (kZWaves * S::L);
  const size_t zlds = sizeof(double2) * (S::N + (size_t)kZWaves * S::L * S::SL);
  for (int c0 = 0; c0 < sys.orb_nc; c0 += ncc_max) {
    const int ncc = std::min(ncc_max, sys.orb_nc - c0);
    const long tiles = (long)((nvb + 7) / 8) * ((ncc + 7) / 8);
    const int nslab = std::min(kPlaneSlabs, g.n3);
    const long blocks = (tiles + 7) / 8 * 8 * 64 * nslab;
    SSRPA_REQUIRE(blocks < (1L << 31), SSRPA_ERR_ARG, "pair grid too large");
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * S::W), lds, s,
                       psi, psi_c, v0, nvb, sys.orb_c0, c0, ncc, g.n3, nslab, g.m1,
                       g.m2, nxo,
                       sys.cmap.as<int>(), g.ldy, tw, yst);
    SSRPA_HIP(hipGetLastError());
    if (zfft) {
      const long zb = (long)nvb * ncc * nblk;
      SSRPA_REQUIRE(zb < (1L << 31), SSRPA_ERR_ARG, "pair grid too large");
      hipLaunchKernelGGL((pair_zfft_kernel<R1, R2>), dim3((unsigned)zb),
                         dim3(64 * kZWaves), zlds, s, yst, ncc, c0, sys.orb_nc,
                         g.ncol, g.ldy, nblk, sys.zcol.as<int4>(), gscale,
                         g.n_g, g.ld_g, tw + g.n1 + g.n2, w);
    } else {
      hipLaunchKernelGGL(pair_z_kernel, dim3((unsigned)(nvb * ncc)), dim3(256),
                         sizeof(double2) * g.n3, s, yst, ncc, c0, sys.orb_nc, g.n3,
                         g.ldy, sys.zcode.as<int>(), gscale, g.n_g, g.ld_g,
                         tw + g.n1 + g.n2, w);
    }
    SSRPA_HIP(hipGetLastError());
  }
}

template <int A, int B>
struct Split { static constexpr int r1 = A, r2 = B; };

// Grid lengths with a staged schedule (N1 = N2 = R1 R2).
template <class F>
bool staged_dispatch(int n, F &&f) {
  switch (n) {
    case 18: f(Split<6, 3>{}); return true;
    case 24: f(Split<4, 6>{}); return true;
    case 27: f(Split<9, 3>{}); return true;
    case 32: f(Split<4, 8>{}); return true;
    case 36: f(Split<6, 6>{}); return true;
    case 48: f(Split<6, 8>{}); return true;
    case 54: f(Split<9, 6>{}); return true;
    case 64: f(Split<8, 8>{}); return true;
    case 72: f(Split<8, 9>{}); return true;
    case 96: f(Split<12, 8>{}); return true;
    default: return false;
  }
}

}  // namespace

bool staged_grid(const Geometry &g) {
  // the x outputs and the y columns must not wrap around the grid
  return g.n1 == g.n2 && 2 * g.m1 + 1 <= g.n1 && 2 * g.m2 + 1 <= g.n2 &&
         staged_dispatch(g.n1, [](auto) {});
}

void launch_pair_matrix(System &sys, int v0, int nvb, bool scaled, double *w,
                        hipStream_t s) {
  const Geometry &g = sys.geo;
  const double *gscale = sys.sqrtv_d.as<double>();
  if (!scaled) gscale += g.ld_g;  // second half holds Omega/N only
  if (staged_grid(g)) {
    staged_dispatch(g.n1, [&](auto sp) {
      using T = decltype(sp);
      staged_pairs<T::r1, T::r2>(sys, v0, nvb, gscale, w, s);
    });
    return;
  }
  PairGeo pg{};
  pg.n1 = g.n1;
  pg.n2 = g.n2;
  pg.n3 = g.n3;
  pg.m1 = g.m1;
  pg.r1 = factor(g.n1);
  pg.r2 = factor(g.n2);
  const int ny = 2 * g.m1 + 1;
  pg.lx = std::max(16, (ny * g.n2 + 2 * g.n1 - 1) / (2 * g.n1));
  pg.lx = std::min(pg.lx, g.n2);
  if (2 * pg.lx * g.n1 < ny * g.n2) pg.lx = g.n2;  // y ping-pong must fit
  const size_t shmem = sizeof(double2) * (g.n1 + g.n2 + 2 * g.n3 +
                                          2 * pg.lx * g.n1 + ny * g.n2);
  SSRPA_REQUIRE(shmem <= 160 * 1024, SSRPA_ERR_ARG,
                "pair FFT needs %zu bytes of LDS", shmem);
  const int tiles_c = (sys.orb_nc + kTileC - 1) / kTileC;
  const int tiles_v = (nvb + kTileV - 1) / kTileV;
  const long blocks = (long)tiles_v * tiles_c * kTileV * kTileC;
  SSRPA_REQUIRE(blocks < (1L << 31), SSRPA_ERR_ARG, "pair grid too large");
  const int gpt = (g.n_g + kPairThreads - 1) / kPairThreads;
  const double2 *psi = sys.src_psi_v
                            ? reinterpret_cast<const double2 *>(sys.src_psi_v)
                            : sys.psi_r.as<double2>();
  const double2 *psi_c = sys.src_psi_c
                              ? reinterpret_cast<const double2 *>(sys.src_psi_c)
                              : sys.psi_r.as<double2>();
  const int *gcol = sys.gcol.as<int>();
  const double2 *tw = sys.fft_tw.as<double2>();
#define SSRPA_PAIR(G)                                                         \
  do {                                                                        \
    if (shmem > 64 * 1024)                                                    \
      SSRPA_HIP(hipFuncSetAttribute(                                          \
          reinterpret_cast<const void *>(&pair_fft_kernel<G>),                \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));           \
    hipLaunchKernelGGL((pair_fft_kernel<G>), dim3((unsigned)blocks),          \
                       dim3(kPairThreads), shmem, s, psi, psi_c, pg, v0, nvb, \
                       sys.orb_c0, sys.orb_nc, gcol, gscale, g.n_g, g.ld_g, tw, w); \
  } while (0)
  if (gpt <= 2) SSRPA_PAIR(2);
  else if (gpt <= 4) SSRPA_PAIR(4);
  else if (gpt <= 8) SSRPA_PAIR(8);
  else if (gpt <= 16) SSRPA_PAIR(16);
  else if (gpt <= 32) SSRPA_PAIR(32);
  else if (gpt <= 64) SSRPA_PAIR(64);
  else fail(SSRPA_ERR_ARG, "chi0 basis of %d vectors is too large", g.n_g);
#undef SSRPA_PAIR
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
