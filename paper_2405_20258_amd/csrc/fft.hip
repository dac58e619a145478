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

// Compile-time radix schedule (4s, then 2s, then 3s) of a length N.
template <int N>
struct Plan {
  static constexpr int count() {
    if (N <= 0) return 0;
    int m = N, c = 0;
    while (m % 4 == 0) { m /= 4; ++c; }
    while (m % 2 == 0) { m /= 2; ++c; }
    while (m % 3 == 0) { m /= 3; ++c; }
    return c;
  }
  static constexpr int radix(int s) {
    if (N <= 0) return 1;
    int m = N, c = 0;
    while (m % 4 == 0) { if (c == s) return 4; m /= 4; ++c; }
    while (m % 2 == 0) { if (c == s) return 2; m /= 2; ++c; }
    while (m % 3 == 0) { if (c == s) return 3; m /= 3; ++c; }
    return 1;
  }
  static constexpr int ns(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i);
    return p;
  }
};

// The same pass with N, R and Ns known at compile time (line stride N), so
// the index arithmetic reduces to shifts and multiplications.
template <int N, int R, int NS>
__device__ __forceinline__ void stockham_pass_t(const double2 *in, double2 *out,
                                                int nlines, const double2 *tw) {
  constexpr int nb = N / R;
  constexpr int stride = N / (NS * R);
  const int total = nlines * nb;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int line = idx / nb;
    const int j = idx - line * nb;
    const int k = j % NS;
    const double2 *src = in + line * N + j;
    double2 v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = src[i * nb];
#pragma unroll
    for (int i = 1; i < R; ++i) v[i] = cmul(v[i], tw[(k * i * stride) % N]);
    double2 y[R];
    radix_dft<R>(v, y);
    double2 *dst = out + line * N + (j / NS) * NS * R + k;
#pragma unroll
    for (int i = 0; i < R; ++i) dst[i * NS] = y[i];
  }
}

template <int N, int S = 0>
__device__ __forceinline__ double2 *lds_fft_t(double2 *a, double2 *b, int nlines,
                                              const double2 *tw) {
  if constexpr (S == Plan<N>::count()) {
    __syncthreads();
    return a;
  } else {
    __syncthreads();
    stockham_pass_t<N, Plan<N>::radix(S), Plan<N>::ns(S)>(a, b, nlines, tw);
    return lds_fft_t<N, S + 1>(b, a, nlines, tw);
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

// One block per (v, c) pair.  For every z-plane j3: pair density of the
// plane, x transforms (in batches of lx lines) pruned to |n1| <= m1, y
// transforms of those columns, then the z sum for the chi0 G vectors is
// accumulated in registers: acc(G) += Y(n1, n2; j3) e^{2 pi i n3 j3 / N3}.
template <int GPT, int N>
__global__ __launch_bounds__(kPairThreads) void pair_fft_kernel(
    const double2 *__restrict__ psi, PairGeo geo, int v0, int nvb, int n_v,
    int n_c, const int *__restrict__ gcol, const double *__restrict__ gscale,
    int n_g, int ld_g, const double2 *__restrict__ tw_g,
    double *__restrict__ w) {
  extern __shared__ double2 smem[];
  const int n1 = N > 0 ? N : geo.n1, n2 = N > 0 ? N : geo.n2;
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
  const double2 *pc = psi + (long)(n_v + c) * box;

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
      const double2 *r;
      if constexpr (N > 0)
        r = lds_fft_t<N>(xa, xb, nl, tw1);
      else
        r = lds_fft(xa, xb, nl, n1, n1, geo.r1, tw1);
      for (int idx = threadIdx.x; idx < nl * ny; idx += blockDim.x) {
        const int line = idx / ny, qq = idx - line * ny;
        int k1 = qq - m1;
        if (k1 < 0) k1 += n1;
        yb[qq * n2 + g0 + line] = r[line * n1 + k1];
      }
    }
    const double2 *ry;
    if constexpr (N > 0)
      ry = lds_fft_t<N>(yb, xa, ny, tw2);
    else
      ry = lds_fft(yb, xa, ny, n2, n2, geo.r2, tw2);
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

// ---------------------------------------------- wave-synchronous pair FFT

// LDS ordering between lanes of one wave: a wavefront-scope fence pair
// around a wave barrier (no block-wide barrier needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stockham pass executed by the 64 lanes of one wave (line stride N).
template <int N, int R, int NS>
__device__ __forceinline__ void stockham_pass_wave(const double2 *in, double2 *out,
                                                   int nlines, const double2 *tw,
                                                   int lane) {
  constexpr int nb = N / R;
  constexpr int stride = N / (NS * R);
  const int total = nlines * nb;
  for (int idx = lane; idx < total; idx += 64) {
    const int line = idx / nb;
    const int j = idx - line * nb;
    const int k = j % NS;
    const double2 *src = in + line * N + j;
    double2 v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = src[i * nb];
#pragma unroll
    for (int i = 1; i < R; ++i) v[i] = cmul(v[i], tw[(k * i * stride) % N]);
    double2 y[R];
    radix_dft<R>(v, y);
    double2 *dst = out + line * N + (j / NS) * NS * R + k;
#pragma unroll
    for (int i = 0; i < R; ++i) dst[i * NS] = y[i];
  }
}

// Whole transform of `nlines` lines by one wave: pass 0 reads `in0`, the
// last pass writes `outF`, passes in between alternate between bufA (after
// even passes) and bufB (after odd passes).  outF must differ from the
// source of the last pass.
template <int N, int S>
__device__ __forceinline__ void wave_fft(const double2 *in0, double2 *bufA,
                                         double2 *bufB, double2 *outF,
                                         int nlines, const double2 *tw, int lane) {
  constexpr int C = Plan<N>::count();
  const double2 *src = S == 0 ? in0 : ((S - 1) % 2 == 0 ? bufA : bufB);
  double2 *dst = S == C - 1 ? outF : (S % 2 == 0 ? bufA : bufB);
  stockham_pass_wave<N, Plan<N>::radix(S), Plan<N>::ns(S)>(src, dst, nlines, tw,
                                                          lane);
  wave_lds_sync();
  if constexpr (S + 1 < C) wave_fft<N, S + 1>(in0, bufA, bufB, outF, nlines, tw, lane);
}

// buffer that is not the source of the last pass of wave_fft<N>
template <int N>
__device__ __forceinline__ double2 *wave_fft_out(double2 *in0, double2 *bufA,
                                                 double2 *bufB, double2 *spare) {
  constexpr int C = Plan<N>::count();
  if constexpr (C == 1) return bufA;
  const double2 *last_src = (C - 2) % 2 == 0 ? bufA : bufB;
  if (last_src == bufA) return bufB == in0 ? spare : bufB;
  return bufA == in0 ? spare : bufA;
}

template <int N>
constexpr int wave_lines() { return N <= 24 ? 8 : 4; }

// Same result as pair_fft_kernel for N1 = N2 = N: per z-plane, each wave
// transforms its own batches of x lines (private LDS, wave-level ordering
// only), writes the |n1| <= m1 outputs to a shared buffer, then the waves
// transform the y lines the same way; two block barriers per plane.
template <int GPT, int N>
__global__ __launch_bounds__(kPairThreads) void pair_fft_wave_kernel(
    const double2 *__restrict__ psi, PairGeo geo, int v0, int nvb, int n_v,
    int n_c, const int *__restrict__ gcol, const double *__restrict__ gscale,
    int n_g, int ld_g, const double2 *__restrict__ tw_g,
    double *__restrict__ w) {
  constexpr int LW = wave_lines<N>();
  extern __shared__ double2 smem[];
  const int n3 = geo.n3, m1 = geo.m1;
  const int ny = 2 * m1 + 1;
  double2 *tw1 = smem;                 // N   (x and y lengths are equal)
  double2 *tw3 = tw1 + N;              // n3
  double2 *pz = tw3 + n3;              // n3
  double2 *yb = pz + n3;               // ny * N: x outputs, [n1][j2]
  double2 *ry = yb + ny * N;           // ny * N: y outputs, [n1][k2]
  double2 *priv = ry + ny * N;         // 4 waves x 3 x LW x N
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw1[t] = tw_g[t];
  for (int t = threadIdx.x; t < n3; t += blockDim.x) tw3[t] = tw_g[geo.n1 + geo.n2 + t];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double2 *pa = priv + wave * 3 * LW * N;
  double2 *pb = pa + LW * N;
  double2 *pc = pb + LW * N;

  const int tiles_c = (n_c + kTileC - 1) / kTileC;
  const int tile = blockIdx.x / (kTileV * kTileC);
  const int q = blockIdx.x % (kTileV * kTileC);
  const int vl = (tile / tiles_c) * kTileV + q / kTileC;
  const int c = (tile % tiles_c) * kTileC + q % kTileC;
  if (vl >= nvb || c >= n_c) return;
  const long plane = (long)N * N;
  const long box = plane * n3;
  const double2 *pv = psi + (long)(v0 + vl) * box;
  const double2 *pcs = psi + (long)(n_v + c) * box;

  int code[GPT];
  double2 acc[GPT];
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    const int g = threadIdx.x + i * kPairThreads;
    code[i] = g < n_g ? gcol[g] : 0;
    acc[i] = make_double2(0.0, 0.0);
  }
  constexpr int nbx = (N + LW - 1) / LW;
  const int nby = (ny + LW - 1) / LW;
  __syncthreads();
  for (int j3 = 0; j3 < n3; ++j3) {
    const double2 *sv = pv + j3 * plane;
    const double2 *sc = pcs + j3 * plane;
    // x lines: pair density, transform, keep |n1| <= m1
    for (int b = wave; b < nbx; b += 4) {
      const int l0 = b * LW;
      const int nl = min(LW, N - l0);
      for (int idx = lane; idx < nl * N; idx += 64) {
        const double2 a = sv[(long)l0 * N + idx];
        const double2 d = sc[(long)l0 * N + idx];
        pa[idx] = make_double2(a.x * d.x + a.y * d.y, a.x * d.y - a.y * d.x);
      }
      wave_lds_sync();
      double2 *res = wave_fft_out<N>(pa, pb, pc, pc);
      wave_fft<N, 0>(pa, pb, pc, res, nl, tw1, lane);
      for (int idx = lane; idx < nl * ny; idx += 64) {
        const int line = idx / ny, qq = idx - line * ny;
        int k1 = qq - m1;
        if (k1 < 0) k1 += N;
        yb[qq * N + l0 + line] = res[line * N + k1];
      }
      wave_lds_sync();
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n3; t += blockDim.x) pz[t] = tw3[(t * j3) % n3];
    // y lines (one per kept n1): transform from yb straight into ry
    for (int b = wave; b < nby; b += 4) {
      const int q0 = b * LW;
      const int nl = min(LW, ny - q0);
      wave_fft<N, 0>(yb + q0 * N, pa, pb, ry + q0 * N, nl, tw1, lane);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int g = threadIdx.x + i * kPairThreads;
      if (g < n_g) {
        const double2 val = ry[code[i] & 0xFFFFF];
        const double2 t = pz[code[i] >> 20];
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
      const double scl = gscale[g];
      row[g] = acc[i].x * scl;
      row[ld_g + g] = acc[i].y * scl;
    }
  }
  for (int g = n_g + threadIdx.x; g < ld_g; g += blockDim.x) {
    row[g] = 0.0;
    row[ld_g + g] = 0.0;
  }
}

}  // namespace

void upload_twiddles(System &sys) {
  const Geometry &g = sys.geo;
  const int lens[3] = {g.n1, g.n2, g.n3};
  std::vector<double> tw;
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
  SSRPA_HIP(hipMemcpy(sys.fft_tw.as(), tw.data(), tw.size() * sizeof(double),
                      hipMemcpyHostToDevice));
}

void launch_orbital_fft(System &sys, const double *coeff_dev,
                        const int *box_index_dev, hipStream_t s) {
  const Geometry &g = sys.geo;
  const long box = (long)g.n1 * g.n2 * g.n3;
  double2 *psi = sys.psi_r.as<double2>();
  fill_zero(psi, sizeof(double2) * box * sys.n_b, s);
  const long total = (long)sys.n_pw * sys.n_b;
  const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(scatter_coeff_kernel, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(coeff_dev),
                     box_index_dev, sys.n_pw, sys.n_b, box, psi);
  SSRPA_HIP(hipGetLastError());
  const double2 *tw = sys.fft_tw.as<double2>();
  const long plane = (long)g.n1 * g.n2;
  // x lines: contiguous; y lines: stride n1; z lines: stride n1*n2
  fft_lines(psi, g.n1, 1, g.n1, g.n2, plane, (long)sys.n_b * g.n3, tw, 1.0, s);
  fft_lines(psi, g.n2, g.n1, 1, g.n1, plane, (long)sys.n_b * g.n3,
            tw + g.n1, 1.0, s);
  fft_lines(psi, g.n3, plane, 1, (int)plane, box, sys.n_b, tw + g.n1 + g.n2,
            1.0 / std::sqrt(g.volume), s);
}

void launch_pair_matrix(System &sys, int v0, int nvb, bool scaled, double *w,
                        hipStream_t s) {
  const Geometry &g = sys.geo;
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
  const double *gscale = sys.sqrtv_d.as<double>();
  if (!scaled) gscale += g.ld_g;  // second half holds Omega/N only
  const int tiles_c = (sys.n_c + kTileC - 1) / kTileC;
  const int tiles_v = (nvb + kTileV - 1) / kTileV;
  const long blocks = (long)tiles_v * tiles_c * kTileV * kTileC;
  SSRPA_REQUIRE(blocks < (1L << 31), SSRPA_ERR_ARG, "pair grid too large");
  const int gpt = (g.n_g + kPairThreads - 1) / kPairThreads;
  const double2 *psi = sys.psi_r.as<double2>();
  const int *gcol = sys.gcol.as<int>();
  const double2 *tw = sys.fft_tw.as<double2>();
#define SSRPA_PAIR_N(G, NN)                                                  \
  do {                                                                       \
    if constexpr (NN > 0) {                                                  \
      const size_t shw = sizeof(double2) *                                   \
          (NN + 2 * g.n3 + 2 * ny * NN + 4 * 3 * wave_lines<NN>() * NN);     \
      SSRPA_REQUIRE(shw <= 160 * 1024, SSRPA_ERR_ARG, "pair FFT LDS");      \
      if (shw > 64 * 1024)                                                   \
        SSRPA_HIP(hipFuncSetAttribute(                                       \
            reinterpret_cast<const void *>(&pair_fft_wave_kernel<G, NN>),    \
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shw));          \
      hipLaunchKernelGGL((pair_fft_wave_kernel<G, NN>),                      \
                         dim3((unsigned)blocks), dim3(kPairThreads), shw, s, \
                         psi, pg, v0, nvb, sys.n_v, sys.n_c, gcol, gscale,   \
                         g.n_g, g.ld_g, tw, w);                              \
    } else {                                                                 \
      if (shmem > 64 * 1024)                                                 \
        SSRPA_HIP(hipFuncSetAttribute(                                       \
            reinterpret_cast<const void *>(&pair_fft_kernel<G, NN>),         \
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));        \
      hipLaunchKernelGGL((pair_fft_kernel<G, NN>), dim3((unsigned)blocks),   \
                         dim3(kPairThreads), shmem, s, psi, pg, v0, nvb,     \
                         sys.n_v, sys.n_c, gcol, gscale, g.n_g, g.ld_g, tw,  \
                         w);                                                 \
    }                                                                        \
  } while (0)
  // grid lengths with a compile-time schedule (x = y); others run generic
#define SSRPA_PAIR(G)                                                        \
  do {                                                                       \
    const int nn = g.n1 == g.n2 ? g.n1 : 0;                                  \
    if (nn == 24) SSRPA_PAIR_N(G, 24);                                       \
    else if (nn == 32) SSRPA_PAIR_N(G, 32);                                  \
    else if (nn == 36) SSRPA_PAIR_N(G, 36);                                  \
    else if (nn == 48) SSRPA_PAIR_N(G, 48);                                  \
    else if (nn == 64) SSRPA_PAIR_N(G, 64);                                  \
    else if (nn == 72) SSRPA_PAIR_N(G, 72);                                  \
    else SSRPA_PAIR_N(G, 0);                                                 \
  } while (0)
  if (gpt <= 2) SSRPA_PAIR(2);
  else if (gpt <= 4) SSRPA_PAIR(4);
  else if (gpt <= 8) SSRPA_PAIR(8);
  else if (gpt <= 16) SSRPA_PAIR(16);
  else if (gpt <= 32) SSRPA_PAIR(32);
  else if (gpt <= 64) SSRPA_PAIR(64);
  else fail(SSRPA_ERR_ARG, "chi0 basis of %d vectors is too large", g.n_g);
#undef SSRPA_PAIR
#undef SSRPA_PAIR_N
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
