// Reduced-precision forms of the complex contractions (same operands,
// layouts and output as gemm.hip; the precision is a property of the MFMA
// products only, every result leaves in FP64):
//
//  * FP32:   operands rounded to FP32 while staged; v_mfma_f32_16x16x4f32.
//  * BF16x3: each real operand x is split as hi = bf16(x), lo = bf16(x - hi)
//            while staged; a product is hi*hi' + hi*lo' + lo*hi' (the lo*lo'
//            term, ~2^-16 relative, is dropped) on v_mfma_f32_16x16x32_bf16.
//
// Accumulation is FP32 inside a K chunk and FP64 across chunks (and across
// split-K partials and valence blocks), which keeps the FP32 rounding walk
// short: 1024 rows for FP32; 4096 rows for the BF16x3 Gram and projection
// passes, whose split products already carry ~2^-17 relative error per term
// (the longer walk quarters their FP64 flush traffic).
#include <cmath>

#include "internal.hpp"
#include "tiles.hpp"

namespace ssrpa {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4m __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kT = 64;
constexpr int kFlush = 1024;   // K rows accumulated in FP32 before flushing

// 16 x 16 f32 accumulator layout of the 16x16xK f32-output MFMAs: slot e of
// lane l holds row 4 (l/16) + e, column l % 16.
__device__ __forceinline__ int accf_row(int l, int e) { return 4 * (l >> 4) + e; }
__device__ __forceinline__ int accf_col(int l) { return l & 15; }

__device__ __forceinline__ double weight_m(const HerkArgs &h, long p, double om) {
  if (h.unit_weight) return 1.0;
  const double de = h.de[p];
  return -4.0 * de / (de * de + om * om) * h.wscale;
}

// round-to-nearest-even float -> bf16 bits (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}
__device__ __forceinline__ void split_bf16(double x, unsigned short &hi,
                                           unsigned short &lo) {
  hi = f2bf((float)x);
  lo = f2bf((float)(x - (double)bf2f(hi)));
}

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfmabf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 load_bf8(const unsigned short *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf8, v);
}
__device__ __forceinline__ bf8 neg_bf8(bf8 a) {
  uint4 v = __builtin_bit_cast(uint4, a);
  v.x ^= 0x80008000u; v.y ^= 0x80008000u; v.z ^= 0x80008000u; v.w ^= 0x80008000u;
  return __builtin_bit_cast(bf8, v);
}

// ------------------------------------------------- BF16x3 operand staging

constexpr int kKb = 32;         // K rows per stage = one bf16 MFMA
constexpr int kKbP = kKb + 8;   // LDS row length (bf16), 16-byte aligned

// LDS operand tile: [part re/im][hi/lo][column 0..63][k 0..31]
struct alignas(16) BfTile {
  unsigned short v[2][2][kT][kKbP];
};


// ------------------------------------------------------------- GEMM FP32

__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g, int m_tiles,
                                                      int n_tiles) {
  __shared__ float As[2][16][kT + 4];   // [part][k][m]
  __shared__ float Bs[2][16][kT + 4];   // [part][k][n]
  const int total = m_tiles * n_tiles;
  const int b = xcd_remap(blockIdx.x, total);
  const int mt = b / n_tiles, nt = b % n_tiles;
  const long M0 = (long)mt * kT;
  const int N0 = nt * kT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f4 re[2][2], im[2][2];
  d4m Re[2][2], Im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = f4{0, 0, 0, 0}; im[i][j] = f4{0, 0, 0, 0};
      Re[i][j] = d4m{0, 0, 0, 0}; Im[i][j] = d4m{0, 0, 0, 0};
    }
  int since = 0;
  for (int k0 = 0; k0 < g.k; k0 += 16) {
    {
      const int row = threadIdx.x >> 2, part = (threadIdx.x >> 1) & 1;
      const int kq = (threadIdx.x & 1) * 8;
      const long m = M0 + row;
      double v[8];
      if (m < g.m) {
        const double *src = g.a + m * g.lda + part * g.a_im + k0 + kq;
#pragma unroll
        for (int x = 0; x < 8; x += 2) {
          const double2 t = *reinterpret_cast<const double2 *>(src + x);
          v[x] = t.x; v[x + 1] = t.y;
        }
      } else {
#pragma unroll
        for (int x = 0; x < 8; ++x) v[x] = 0.0;
      }
#pragma unroll
      for (int x = 0; x < 8; ++x) As[part][kq + x][row] = (float)v[x];
    }
    {
      const int kr = threadIdx.x >> 4, part = (threadIdx.x >> 3) & 1;
      const int cq = (threadIdx.x & 7) * 8;
      const double *src = g.b + (long)(k0 + kr) * g.ldb + part * g.b_im + N0 + cq;
#pragma unroll
      for (int x = 0; x < 8; x += 2) {
        const double2 t = *reinterpret_cast<const double2 *>(src + x);
        Bs[part][kr][cq + x] = (float)t.x;
        Bs[part][kr][cq + x + 1] = (float)t.y;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4), cl = lane & 15;
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As[0][kr][wr + i * 16 + cl];
        ai[i] = As[1][kr][wr + i * 16 + cl];
        br[i] = Bs[0][kr][wc + i * 16 + cl];
        bi[i] = Bs[1][kr][wc + i * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          re[i][j] = mfma32(ar[i], br[j], re[i][j]);
          re[i][j] = mfma32(-ai[i], bi[j], re[i][j]);
          im[i][j] = mfma32(ar[i], bi[j], im[i][j]);
          im[i][j] = mfma32(ai[i], br[j], im[i][j]);
        }
    }
    __syncthreads();
    since += 16;
    if (since >= kFlush) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            Re[i][j][e] += (double)re[i][j][e];
            Im[i][j][e] += (double)im[i][j][e];
            re[i][j][e] = 0.f;
            im[i][j][e] = 0.f;
          }
      since = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long m = M0 + wr + i * 16 + accf_row(lane, e);
        const int n = N0 + wc + j * 16 + accf_col(lane);
        if (m >= g.m) continue;
        double *cr = g.c + m * g.ldc + n;
        double *ci = cr + g.c_im;
        const double vr = g.alpha * (Re[i][j][e] + (double)re[i][j][e]);
        const double vi = g.alpha * (Im[i][j][e] + (double)im[i][j][e]);
        if (g.beta != 0.0) {
          *cr = vr + g.beta * *cr;
          *ci = vi + g.beta * *ci;
        } else {
          *cr = vr;
          *ci = vi;
        }
      }
}

// ----------------------------------------------------------- GEMM BF16x3

__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(GemmArgs g,
                                                         int m_tiles,
                                                         int n_tiles) {
  __shared__ BfTile At, Bt;   // At: [part][hl][m][k], Bt: [part][hl][n][k]
  const int total = m_tiles * n_tiles;
  const int b = xcd_remap(blockIdx.x, total);
  const int mt = b / n_tiles, nt = b % n_tiles;
  const long M0 = (long)mt * kT;
  const int N0 = nt * kT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int ko = 8 * (lane >> 4), cl = lane & 15;
  f4 re[2][2], im[2][2];
  d4m Re[2][2], Im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = f4{0, 0, 0, 0}; im[i][j] = f4{0, 0, 0, 0};
      Re[i][j] = d4m{0, 0, 0, 0}; Im[i][j] = d4m{0, 0, 0, 0};
    }
  int since = 0;
  for (int k0 = 0; k0 < g.k; k0 += kKb) {
    // A: 64 rows x 32 k x 2 parts; k is contiguous in memory
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;   // 0..1023
      const int part = idx >> 9, row = (idx >> 3) & 63, kq = (idx & 7) * 4;
      const long m = M0 + row;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (m < g.m) {
        const double *src = g.a + m * g.lda + part * g.a_im + k0 + kq;
        const double2 t0 = *reinterpret_cast<const double2 *>(src);
        const double2 t1 = *reinterpret_cast<const double2 *>(src + 2);
        v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        unsigned short hi, lo;
        split_bf16(v[x], hi, lo);
        At.v[part][0][row][kq + x] = hi;
        At.v[part][1][row][kq + x] = lo;
      }
    }
    // B: 32 k rows x 64 columns x 2 parts; transposed into [n][k]
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int part = idx >> 9, kr = (idx >> 4) & 31, cq = (idx & 15) * 4;
      const double *src = g.b + (long)(k0 + kr) * g.ldb + part * g.b_im + N0 + cq;
      const double2 t0 = *reinterpret_cast<const double2 *>(src);
      const double2 t1 = *reinterpret_cast<const double2 *>(src + 2);
      const double v[4] = {t0.x, t0.y, t1.x, t1.y};
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        unsigned short hi, lo;
        split_bf16(v[x], hi, lo);
        Bt.v[part][0][cq + x][kr] = hi;
        Bt.v[part][1][cq + x][kr] = lo;
      }
    }
    __syncthreads();
    bf8 arh[2], arl[2], aih[2], ail[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ma = wr + i * 16 + cl, mb = wc + i * 16 + cl;
      arh[i] = load_bf8(&At.v[0][0][ma][ko]);
      arl[i] = load_bf8(&At.v[0][1][ma][ko]);
      aih[i] = load_bf8(&At.v[1][0][ma][ko]);
      ail[i] = load_bf8(&At.v[1][1][ma][ko]);
      brh[i] = load_bf8(&Bt.v[0][0][mb][ko]);
      brl[i] = load_bf8(&Bt.v[0][1][mb][ko]);
      bih[i] = load_bf8(&Bt.v[1][0][mb][ko]);
      bil[i] = load_bf8(&Bt.v[1][1][mb][ko]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf8 naih = neg_bf8(aih[i]), nail = neg_bf8(ail[i]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // Re += ar br - ai bi
        re[i][j] = mfmabf(arh[i], brh[j], re[i][j]);
        re[i][j] = mfmabf(arh[i], brl[j], re[i][j]);
        re[i][j] = mfmabf(arl[i], brh[j], re[i][j]);
        re[i][j] = mfmabf(naih, bih[j], re[i][j]);
        re[i][j] = mfmabf(naih, bil[j], re[i][j]);
        re[i][j] = mfmabf(nail, bih[j], re[i][j]);
        // Im += ar bi + ai br
        im[i][j] = mfmabf(arh[i], bih[j], im[i][j]);
        im[i][j] = mfmabf(arh[i], bil[j], im[i][j]);
        im[i][j] = mfmabf(arl[i], bih[j], im[i][j]);
        im[i][j] = mfmabf(aih[i], brh[j], im[i][j]);
        im[i][j] = mfmabf(aih[i], brl[j], im[i][j]);
        im[i][j] = mfmabf(ail[i], brh[j], im[i][j]);
      }
    }
    __syncthreads();
    since += kKb;
    if (since >= kFlush) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            Re[i][j][e] += (double)re[i][j][e];
            Im[i][j][e] += (double)im[i][j][e];
            re[i][j][e] = 0.f;
            im[i][j][e] = 0.f;
          }
      since = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long m = M0 + wr + i * 16 + accf_row(lane, e);
        const int n = N0 + wc + j * 16 + accf_col(lane);
        if (m >= g.m) continue;
        double *cr = g.c + m * g.ldc + n;
        double *ci = cr + g.c_im;
        const double vr = g.alpha * (Re[i][j][e] + (double)re[i][j][e]);
        const double vi = g.alpha * (Im[i][j][e] + (double)im[i][j][e]);
        if (g.beta != 0.0) {
          *cr = vr + g.beta * *cr;
          *ci = vi + g.beta * *ci;
        } else {
          *cr = vr;
          *ci = vi;
        }
      }
}

// ------------------------------------------ reduced-precision contractions
//
// The FP32 and BF16x3 HERKs convert each row once per K chunk into a
// K-blocked layout [kb][part][col][rows of the block] with the rows of one
// column contiguous (64 B), so that a lane's MFMA operand (consecutive rows
// of one column) is a single 16-byte load; a Gram kernel then forms
// sum_p conj(a_p[I]) b_p[J] over 128 x 128 tiles of the lower triangle
// (64 x 64 for outputs of at most kGSmallCols columns).
// FP32 accumulators are added into the block's own FP64 partial tile every
// 1024 (FP32) or 4096 (BF16x3) rows, and gram_reduce_kernel sums the
// split-K partials in order and mirrors the Hermitian half (deterministic).
//  * BF16x3: the I operand is the rows as they are, the J operand the rows
//    times d_p; each real part is split hi + lo (bf16) and a product is
//    hi hi' + hi lo' + lo hi'.  For several frequencies the I copy of the
//    whole K range is split once and reused, and the Gram kernel forms
//    each frequency's J operand from it while staging.
//  * FP32: one copy of the rows times sqrt|d_p| (the d_p of one HERK have
//    one sign, restored by the reduction), rounded to FP32; for several
//    frequencies the unweighted rows, d_p applied to the B fragments.

constexpr int kGT = 128;          // Gram tile side (GEMMs; Gram kernels of
                                   // large outputs), also the column
                                   // multiple of the converted copies
constexpr int kGSmallTile = 64;   // Gram tile side of small outputs
constexpr int kGSmallCols = 1024; // largest output side on kGSmallTile tiles
constexpr int kGFlushSteps = 128;  // K steps of 32 rows between FP64 flushes
                                   // (4096 rows)
constexpr int kGColStride = 5;    // uint4 per column in LDS (4 + 1 pad)
constexpr size_t kGChunkBytes = size_t(1) << 30;  // per copy
constexpr size_t kGLds = 2 * 4 * kGT * kGColStride * sizeof(uint4);
// LDS of a Gram block: two operands of `parts` planes of ts columns
constexpr size_t gram_lds(int parts, int ts) {
  return 2 * (size_t)parts * ts * kGColStride * sizeof(uint4);
}

// Splits one copy of a K chunk: the I operand from the rows as they are
// (weighted = 0), the J operand from d_p x (weighted = 1; kGJScale x for a
// unit-weight Gram matrix).  The J copy is rounded independently of the I
// copy, so the dropped lo_I lo_J' products average out; with one copy for
// both they would be lo^2 >= 0 on the diagonal and bias it by ~2^-16/3.
constexpr double kGJScale = 3.0;

// kBoth: one pass writes the unweighted copy to wb and the weighted one to
// wb2 (the two operands of a single-frequency Gram pass), reading each
// element of W once.
template <bool kBoth>
__global__ __launch_bounds__(256) void split_rows_bf16_kernel(
    HerkArgs h, long k0, int nrows, int ldb, int om_i, int weighted,
    uint4 *__restrict__ wb, uint4 *__restrict__ wb2) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int kb = blockIdx.y;
  if (col >= ldb) return;
  const double om = h.unit_weight ? 0.0 : h.omega[om_i];
  unsigned pk[4][16];   // [part][row pair]: two bf16 per word, even row low
  unsigned pk2[4][16];  // weighted copy (kBoth)
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int r = kb * 32 + t;
    // kBoth: x raw and sc the weight; otherwise x already weighted
    double xr = 0.0, xi = 0.0, sc = 1.0;
    if (r < nrows && col < h.ncol) {
      const long p = k0 + r;
      const double w = !(kBoth || weighted)
                           ? 1.0
                           : (h.unit_weight ? kGJScale : weight_m(h, p, om));
      const double *src = h.a + p * h.lda + col;
      if constexpr (kBoth) {
        sc = w;
        xr = src[0];
        xi = src[h.im_off];
      } else {
        xr = src[0] * w;
        xi = src[h.im_off] * w;
      }
    }
    unsigned short v[4];
    split_bf16(xr, v[0], v[1]);
    split_bf16(xi, v[2], v[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (t & 1)
        pk[q][t >> 1] |= (unsigned)v[q] << 16;
      else
        pk[q][t >> 1] = v[q];
    }
    if constexpr (kBoth) {
      unsigned short w[4];
      split_bf16(xr * sc, w[0], w[1]);
      split_bf16(xi * sc, w[2], w[3]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (t & 1)
          pk2[q][t >> 1] |= (unsigned)w[q] << 16;
        else
          pk2[q][t >> 1] = w[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint4 *dst = wb + (((long)kb * 4 + q) * ldb + col) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      dst[u] = make_uint4(pk[q][4 * u], pk[q][4 * u + 1], pk[q][4 * u + 2],
                          pk[q][4 * u + 3]);
    if constexpr (kBoth) {
      uint4 *dst2 = wb2 + (((long)kb * 4 + q) * ldb + col) * 4;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        dst2[u] = make_uint4(pk2[q][4 * u], pk2[q][4 * u + 1], pk2[q][4 * u + 2],
                             pk2[q][4 * u + 3]);
    }
  }
}

// d_p x for the 8 rows of one 16-byte quarter of a column: x rebuilt as
// hi + lo (exact in FP32) from the unweighted split copy, multiplied in FP32
// by the row weights and split again, as split_rows_bf16_kernel does from
// the FP64 rows.  in[4] / out[4]: parts re hi, re lo, im hi, im lo.
__device__ __forceinline__ void reweight_quarter(const uint4 (&in)[4],
                                                 const float *__restrict__ w8,
                                                 uint4 (&out)[4]) {
  unsigned ph[4][4];   // [part][word]
#pragma unroll
  for (int c = 0; c < 2; ++c) {   // re, im
    const unsigned *hi = reinterpret_cast<const unsigned *>(&in[2 * c]);
    const unsigned *lo = reinterpret_cast<const unsigned *>(&in[2 * c + 1]);
#pragma unroll
    for (int wd = 0; wd < 4; ++wd) {
      unsigned short h2[2], l2[2];
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const unsigned short xh = (unsigned short)(hi[wd] >> (16 * hf));
        const unsigned short xl = (unsigned short)(lo[wd] >> (16 * hf));
        // FP32 product: its rounding (2^-24) is far below the lo part's
        // (2^-17), and the split of an FP32 value is exact
        const float y = (bf2f(xh) + bf2f(xl)) * w8[2 * wd + hf];
        h2[hf] = f2bf(y);
        l2[hf] = f2bf(y - bf2f(h2[hf]));
      }
      ph[2 * c][wd] = h2[0] | ((unsigned)h2[1] << 16);
      ph[2 * c + 1][wd] = l2[0] | ((unsigned)l2[1] << 16);
    }
  }
#pragma unroll
  for (int pp = 0; pp < 4; ++pp)
    out[pp] = make_uint4(ph[pp][0], ph[pp][1], ph[pp][2], ph[pp][3]);
}

// kWJ: the J operand is formed while staging from the I copy (unweighted
// split rows) and this frequency's row weights wrow (wj unused), so several
// frequencies share one converted copy of the rows.  kTs: output tile side,
// 128 (4 waves of 64 x 64) or 64 (4 waves of 32 x 32, for small outputs
// whose 128-wide tiles would be mostly padding).
template <int kTs, bool kWJ>
__global__ __launch_bounds__(256, kTs == 128 ? 2 : 4) void gram_bf16x3_kernel(
    const uint4 *__restrict__ wi, const uint4 *__restrict__ wj, int ldb,
    int ncol, int nkb, int T, int n_tiles, int kb_per_split,
    const float *__restrict__ wrow, double *__restrict__ partial) {
  constexpr int kS = kTs / 32;    // 16 x 16 MFMA tiles per wave side
  constexpr int kHc = kTs / 64;   // 64-column halves of a panel
  extern __shared__ uint4 gsm[];
  uint4 *As = gsm;                          // [part][col][kGColStride]
  uint4 *Bs = gsm + 4 * kTs * kGColStride;
  // block -> (split, tile): on 64-wide tiles each XCD takes a contiguous
  // run of (split, tile); on 128-wide tiles each XCD keeps a group of tiles
  // over all splits (measured on 1600 columns: the runs were 17-20 % slower
  // there, and 11 % faster at 400 columns on 64-wide tiles)
  int split, tile_id;
  if constexpr (kTs == kGSmallTile) {
    const int blk = xcd_linear(n_tiles);
    split = blk / n_tiles;
    tile_id = blk - split * n_tiles;
  } else {
    tile_id = xcd_remap(blockIdx.x, n_tiles);
    split = blockIdx.y;
  }
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kTs, J0 = tile.y * kTs;
  const int kb0 = split * kb_per_split;
  const int kb1 = min(nkb, kb0 + kb_per_split);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * (kTs / 2), wc = (wave & 1) * (kTs / 2);
  // dropped sub-tiles are skipped on 64-wide tiles only: on 128-wide tiles
  // the branches cost more than they save (measured on 1600 columns, FP32:
  // 493 against 415 ms for 16 frequencies)
  const unsigned live = live_subtiles<kS>(I0 + wr, J0 + wc, ncol);
  const int q = lane >> 4, cl = lane & 15;
  double *pt = partial + ((long)split * n_tiles + tile_id) * 2L * kTs * kTs;
  f4 re[kS][kS], im[kS][kS];
#pragma unroll
  for (int i = 0; i < kS; ++i)
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      re[i][j] = f4{0, 0, 0, 0};
      im[i][j] = f4{0, 0, 0, 0};
    }
  // partial tiles start zeroed (a fill before the first chunk): every flush
  // adds, so the code has no per-element branches
  // Per-lane offsets; the empty asm statements mark them as redefined on
  // every use, so the compiler rebuilds the flush and staging addresses
  // from them instead of hoisting (and spilling) them.
  int foff = (wr + accf_row(lane, 0)) * kTs + wc + accf_col(lane);
  int soff = (threadIdx.x >> 2) * 4 + (threadIdx.x & 3);
  auto flush = [&]() __attribute__((always_inline)) {
    asm volatile("" : "+v"(foff));
    double *pl = pt + foff;
#pragma unroll
    for (int i = 0; i < kS; ++i)
#pragma unroll
      for (int j = 0; j < kS; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double *p0 = pl + (i * 16 + e) * kTs + j * 16;
          p0[0] += (double)re[i][j][e];
          p0[kTs * kTs] += (double)im[i][j][e];
          re[i][j][e] = 0.f;
          im[i][j][e] = 0.f;
        }
  };
  int steps = 0;
  for (int kb = kb0; kb < kb1; ++kb) {
    __syncthreads();
    asm volatile("" : "+v"(soff));
    const uint4 *si = wi + (long)kb * 16 * ldb + soff;
    const uint4 *sj = wj + (long)kb * 16 * ldb + soff;
    // item it: operand, part, 64-column half hc
    if constexpr (kWJ) {
      (void)sj;
      const float *w8 = wrow + (long)kb * 32 + 8 * (soff & 3);
#pragma unroll
      for (int it = 0; it < 4 * kHc; ++it) {
        const int part = it / kHc, hc = it % kHc;
        const uint4 v = si[(part * ldb + I0 + 64 * hc) * 4];
        const int col = (soff >> 2) + 64 * hc;
        As[(part * kTs + col) * kGColStride + (soff & 3)] = v;
      }
#pragma unroll
      for (int hc = 0; hc < kHc; ++hc) {
        uint4 in[4], out[4];
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) in[pp] = si[(pp * ldb + J0 + 64 * hc) * 4];
        reweight_quarter(in, w8, out);
        const int col = (soff >> 2) + 64 * hc;
#pragma unroll
        for (int pp = 0; pp < 4; ++pp)
          Bs[(pp * kTs + col) * kGColStride + (soff & 3)] = out[pp];
      }
    } else {
#pragma unroll
      for (int it = 0; it < 8 * kHc; ++it) {
        const int op = it / (4 * kHc), part = (it / kHc) % 4, hc = it % kHc;
        const uint4 v =
            (op ? sj : si)[(part * ldb + (op ? J0 : I0) + 64 * hc) * 4];
        const int col = (soff >> 2) + 64 * hc;
        (op ? Bs : As)[(part * kTs + col) * kGColStride + (soff & 3)] = v;
      }
    }
    __syncthreads();
    bf8 a[kS][4];
#pragma unroll
    for (int i = 0; i < kS; ++i)
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
        a[i][pp] = __builtin_bit_cast(
            bf8, As[(pp * kTs + wr + i * 16 + cl) * kGColStride + q]);
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      bf8 b[4];
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
        b[pp] = __builtin_bit_cast(
            bf8, Bs[(pp * kTs + wc + j * 16 + cl) * kGColStride + q]);
      const bf8 nbh = neg_bf8(b[0]), nbl = neg_bf8(b[1]);
#pragma unroll
      for (int i = 0; i < kS; ++i) {
        if (kTs == kGSmallTile && !(live >> (kS * i + j) & 1u)) continue;
        // Re += ar br + ai bi;  Im += ar bi - ai br  (hi*hi + hi*lo + lo*hi)
        re[i][j] = mfmabf(a[i][0], b[0], re[i][j]);
        re[i][j] = mfmabf(a[i][0], b[1], re[i][j]);
        re[i][j] = mfmabf(a[i][1], b[0], re[i][j]);
        re[i][j] = mfmabf(a[i][2], b[2], re[i][j]);
        re[i][j] = mfmabf(a[i][2], b[3], re[i][j]);
        re[i][j] = mfmabf(a[i][3], b[2], re[i][j]);
        im[i][j] = mfmabf(a[i][0], b[2], im[i][j]);
        im[i][j] = mfmabf(a[i][0], b[3], im[i][j]);
        im[i][j] = mfmabf(a[i][1], b[2], im[i][j]);
        im[i][j] = mfmabf(a[i][2], nbh, im[i][j]);
        im[i][j] = mfmabf(a[i][2], nbl, im[i][j]);
        im[i][j] = mfmabf(a[i][3], nbh, im[i][j]);
      }
    }
    if (++steps == kGFlushSteps || kb + 1 == kb1) {
      flush();
      steps = 0;
    }
  }
}

// FP32 form of the Gram pass: one copy wf[kb][part][col][16 floats] (part =
// re, im) of the scaled rows rounded to FP32 (no split, so no bias term);
// in each 16-row block position 4q + s holds row 4s + q, so that lane q's
// 16-byte load carries its rows for the four 16x16x4 MFMA steps.
constexpr int kFFlushSteps = 64;  // 16-row steps between FP64 flushes
constexpr size_t kFLds = 2 * 2 * kGT * kGColStride * sizeof(uint4);

__global__ __launch_bounds__(256) void split_rows_f32_kernel(
    HerkArgs h, long k0, int nrows, int ldb, int om_i, uint4 *__restrict__ wf) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int kb = blockIdx.y;
  if (col >= ldb) return;
  const double om = h.unit_weight ? 0.0 : h.omega[om_i];
  float v[2][16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int r = kb * 16 + t;
    double xr = 0.0, xi = 0.0;
    if (r < nrows && col < h.ncol) {
      const long p = k0 + r;
      const double sc = h.unit_weight ? 1.0 : sqrt(-weight_m(h, p, om));
      const double *src = h.a + p * h.lda + col;
      xr = src[0] * sc;
      xi = src[h.im_off] * sc;
    }
    const int pos = 4 * (t & 3) + (t >> 2);  // row t = 4 s + q -> 4 q + s
    v[0][pos] = (float)xr;
    v[1][pos] = (float)xi;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint4 *dst = wf + (((long)kb * 2 + q) * ldb + col) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      dst[u] = make_uint4(__float_as_uint(v[q][4 * u]), __float_as_uint(v[q][4 * u + 1]),
                          __float_as_uint(v[q][4 * u + 2]),
                          __float_as_uint(v[q][4 * u + 3]));
  }
}

// Per-row weights Delta_p(i omega) of one chunk for the FP32 Gram pass with
// unweighted rows, in the permuted 16-row order of split_rows_f32_kernel
// (position 4 q + s holds row 4 s + q); zero past the chunk.
__global__ __launch_bounds__(256) void row_weights_f32_kernel(
    HerkArgs h, long k0, int nrows, int n_pos, int om_i, float *__restrict__ wp) {
  const int pos = blockIdx.x * 256 + threadIdx.x;
  if (pos >= n_pos) return;
  const int kb = pos >> 4, t = pos & 15;
  const int r = kb * 16 + 4 * (t & 3) + (t >> 2);
  wp[pos] = r < nrows ? (float)weight_m(h, k0 + r, h.omega[om_i]) : 0.0f;
}

// Natural-order row weights of one K chunk for the BF16x3 Gram pass
// (Delta_p(i w) x wscale in FP32); zero past the chunk, up to n_pos.
__global__ __launch_bounds__(256) void row_weights_bf_kernel(
    HerkArgs h, long k0, int nrows, int n_pos, int om_i, float *__restrict__ wp) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n_pos) return;
  wp[r] = r < nrows ? (float)weight_m(h, k0 + r, h.omega[om_i]) : 0.0f;
}

template <int kTs, bool kWeighted>
__global__ __launch_bounds__(256, kTs == 128 ? 2 : 4) void gram_f32_kernel(
    const uint4 *__restrict__ wf, int ldb, int ncol, int nkb, int T, int n_tiles,
    int kb_per_split, const float *__restrict__ wrow,
    double *__restrict__ partial) {
  constexpr int kS = kTs / 32;    // 16 x 16 MFMA tiles per wave side
  constexpr int kHc = kTs / 64;   // 64-column halves of a panel
  extern __shared__ uint4 fsm[];
  uint4 *As = fsm;                          // [part][col][kGColStride]
  uint4 *Bs = fsm + 2 * kTs * kGColStride;
  // block -> (split, tile): on 64-wide tiles each XCD takes a contiguous
  // run of (split, tile); on 128-wide tiles each XCD keeps a group of tiles
  // over all splits (measured on 1600 columns: the runs were 17-20 % slower
  // there, and 11 % faster at 400 columns on 64-wide tiles)
  int split, tile_id;
  if constexpr (kTs == kGSmallTile) {
    const int blk = xcd_linear(n_tiles);
    split = blk / n_tiles;
    tile_id = blk - split * n_tiles;
  } else {
    tile_id = xcd_remap(blockIdx.x, n_tiles);
    split = blockIdx.y;
  }
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kTs, J0 = tile.y * kTs;
  const int kb0 = split * kb_per_split;
  const int kb1 = min(nkb, kb0 + kb_per_split);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * (kTs / 2), wc = (wave & 1) * (kTs / 2);
  // dropped sub-tiles are skipped on 64-wide tiles only: on 128-wide tiles
  // the branches cost more than they save (measured on 1600 columns, FP32:
  // 493 against 415 ms for 16 frequencies)
  const unsigned live = live_subtiles<kS>(I0 + wr, J0 + wc, ncol);
  const int q = lane >> 4, cl = lane & 15;
  double *pt = partial + ((long)split * n_tiles + tile_id) * 2L * kTs * kTs;
  f4 re[kS][kS], im[kS][kS];
#pragma unroll
  for (int i = 0; i < kS; ++i)
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      re[i][j] = f4{0, 0, 0, 0};
      im[i][j] = f4{0, 0, 0, 0};
    }
  int foff = (wr + accf_row(lane, 0)) * kTs + wc + accf_col(lane);
  int soff = (threadIdx.x >> 2) * 4 + (threadIdx.x & 3);
  auto flush = [&]() __attribute__((always_inline)) {
    asm volatile("" : "+v"(foff));
    double *pl = pt + foff;
#pragma unroll
    for (int i = 0; i < kS; ++i)
#pragma unroll
      for (int j = 0; j < kS; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double *p0 = pl + (i * 16 + e) * kTs + j * 16;
          p0[0] += (double)re[i][j][e];
          p0[kTs * kTs] += (double)im[i][j][e];
          re[i][j][e] = 0.f;
          im[i][j][e] = 0.f;
        }
  };
  int steps = 0;
  for (int kb = kb0; kb < kb1; ++kb) {
    __syncthreads();
    asm volatile("" : "+v"(soff));
    const uint4 *src = wf + (long)kb * 8 * ldb + soff;
    // the lane's row weights, loaded with the rows (used after the barrier)
    float wv[4] = {1.0f, 1.0f, 1.0f, 1.0f};
    if constexpr (kWeighted) {
      const float4 w4 = *reinterpret_cast<const float4 *>(wrow + kb * 16 + 4 * q);
      wv[0] = w4.x;
      wv[1] = w4.y;
      wv[2] = w4.z;
      wv[3] = w4.w;
    }
    // item it: operand, part, 64-column half hc
#pragma unroll
    for (int it = 0; it < 4 * kHc; ++it) {
      const int op = it / (2 * kHc), part = (it / kHc) % 2, hc = it % kHc;
      const uint4 v = src[(part * ldb + (op ? J0 : I0) + 64 * hc) * 4];
      const int col = (soff >> 2) + 64 * hc;
      (op ? Bs : As)[(part * kTs + col) * kGColStride + (soff & 3)] = v;
    }
    __syncthreads();
    uint4 a[kS][2];
#pragma unroll
    for (int i = 0; i < kS; ++i)
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
        a[i][pp] = As[(pp * kTs + wr + i * 16 + cl) * kGColStride + q];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      uint4 b[2];
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
        b[pp] = Bs[(pp * kTs + wc + j * 16 + cl) * kGColStride + q];
      float br[4] = {__uint_as_float(b[0].x), __uint_as_float(b[0].y),
                     __uint_as_float(b[0].z), __uint_as_float(b[0].w)};
      float bi[4] = {__uint_as_float(b[1].x), __uint_as_float(b[1].y),
                     __uint_as_float(b[1].z), __uint_as_float(b[1].w)};
      if constexpr (kWeighted) {
        // rows are unweighted: Delta of the lane's row of each MFMA step
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          br[s] *= wv[s];
          bi[s] *= wv[s];
        }
      }
#pragma unroll
      for (int i = 0; i < kS; ++i) {
        if (kTs == kGSmallTile && !(live >> (kS * i + j) & 1u)) continue;
        const float ar[4] = {__uint_as_float(a[i][0].x), __uint_as_float(a[i][0].y),
                             __uint_as_float(a[i][0].z), __uint_as_float(a[i][0].w)};
        const float ai[4] = {__uint_as_float(a[i][1].x), __uint_as_float(a[i][1].y),
                             __uint_as_float(a[i][1].z), __uint_as_float(a[i][1].w)};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          // Re += ar br + ai bi;  Im += ar bi - ai br
          re[i][j] = mfma32(ar[s], br[s], re[i][j]);
          re[i][j] = mfma32(ai[s], bi[s], re[i][j]);
          im[i][j] = mfma32(ar[s], bi[s], im[i][j]);
          im[i][j] = mfma32(ai[s], -br[s], im[i][j]);
        }
      }
    }
    if (++steps == kFFlushSteps || kb + 1 == kb1) {
      flush();
      steps = 0;
    }
  }
}

// BF16x3 GEMM C = A B (beta = 0) for the projection W_s = W C_s: 128 x 128
// output tiles, 4 waves of 64 x 64.  A (FP64 planar rows, k contiguous) is
// split into bf16 hi/lo while it is staged, once per block and K step; B is
// split once per call into the K-blocked layout of the Gram path (the basis
// is small).  A wide N tile reads A ld/128 times instead of ld/64.  FP32
// accumulators are added into C (zeroed first) every kGFlushSteps steps.
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_wide_kernel(
    GemmArgs g, const uint4 *__restrict__ bt, int ldn, int m_tiles,
    int n_tiles) {
  extern __shared__ uint4 wsm[];
  uint4 *As = wsm;                          // [part][row][kGColStride]
  uint4 *Bs = wsm + 4 * kGT * kGColStride;  // [part][col][kGColStride]
  const int total = m_tiles * n_tiles;
  const int t = xcd_remap(blockIdx.x, total);
  const int mt = t / n_tiles, nt = t - mt * n_tiles;
  const long M0 = (long)mt * kGT;
  const int N0 = nt * kGT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  const int q = lane >> 4, cl = lane & 15;
  f4 re[4][4], im[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      re[i][j] = f4{0, 0, 0, 0};
      im[i][j] = f4{0, 0, 0, 0};
    }
  // an opaque zero: the flush addresses are rebuilt at every flush instead
  // of being hoisted out of the K loop (and spilled)
  int zero = 0;
  int soff = (threadIdx.x >> 2) * 4 + (threadIdx.x & 3);
  auto flush = [&]() __attribute__((always_inline)) {
    asm volatile("" : "+v"(zero));
    const int n0 = N0 + wc + accf_col(lane) + zero;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long m = M0 + wr + i * 16 + accf_row(lane, e);
        if (m < g.m) {
          double *cr = g.c + m * g.ldc + n0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (n0 + j * 16 < g.n) {
              cr[j * 16] += g.alpha * (double)re[i][j][e];
              cr[g.c_im + j * 16] += g.alpha * (double)im[i][j][e];
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[i][j][e] = 0.f;
          im[i][j][e] = 0.f;
        }
      }
  };
  const int nkb = g.k / 32;
  int steps = 0;
  for (int kb = 0; kb < nkb; ++kb) {
    __syncthreads();
    asm volatile("" : "+v"(soff));
    // A: thread (row r = soff / 4 (+ 64), q4 = soff % 4) splits the 8 rows
    // k = 32 kb + 8 q4 .. + 7 of its row, real and imaginary parts
#pragma unroll
    for (int hc = 0; hc < 2; ++hc) {
      const int r = (soff >> 2) + 64 * hc, q4 = soff & 3;
      const long m = M0 + r;
      unsigned pk[4][4];
      if (m < g.m) {
        const double *src = g.a + m * g.lda + (long)kb * 32 + q4 * 8;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double2 xr = *reinterpret_cast<const double2 *>(src + 2 * u);
          const double2 xi =
              *reinterpret_cast<const double2 *>(src + g.a_im + 2 * u);
          unsigned short h0, l0, h1, l1, h2, l2, h3, l3;
          split_bf16(xr.x, h0, l0);
          split_bf16(xr.y, h1, l1);
          split_bf16(xi.x, h2, l2);
          split_bf16(xi.y, h3, l3);
          pk[0][u] = h0 | ((unsigned)h1 << 16);
          pk[1][u] = l0 | ((unsigned)l1 << 16);
          pk[2][u] = h2 | ((unsigned)h3 << 16);
          pk[3][u] = l2 | ((unsigned)l3 << 16);
        }
      } else {
#pragma unroll
        for (int pp = 0; pp < 4; ++pp)
#pragma unroll
          for (int u = 0; u < 4; ++u) pk[pp][u] = 0u;
      }
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
        As[(pp * kGT + r) * kGColStride + q4] =
            make_uint4(pk[pp][0], pk[pp][1], pk[pp][2], pk[pp][3]);
    }
    // B: items it = part (it / 2), columns + 64 (it % 2)
    const uint4 *sb = bt + (long)kb * 16 * ldn + soff;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int part = it >> 1, hc = it & 1;
      const uint4 v = sb[(part * ldn + N0 + 64 * hc) * 4];
      const int col = (soff >> 2) + 64 * hc;
      Bs[(part * kGT + col) * kGColStride + (soff & 3)] = v;
    }
    __syncthreads();
    bf8 a[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
        a[i][pp] = __builtin_bit_cast(
            bf8, As[(pp * kGT + wr + i * 16 + cl) * kGColStride + q]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 b[4];
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
        b[pp] = __builtin_bit_cast(
            bf8, Bs[(pp * kGT + wc + j * 16 + cl) * kGColStride + q]);
      const bf8 nih = neg_bf8(b[2]), nil = neg_bf8(b[3]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // Re += ar br - ai bi;  Im += ar bi + ai br  (hi*hi + hi*lo + lo*hi)
        re[i][j] = mfmabf(a[i][0], b[0], re[i][j]);
        re[i][j] = mfmabf(a[i][0], b[1], re[i][j]);
        re[i][j] = mfmabf(a[i][1], b[0], re[i][j]);
        re[i][j] = mfmabf(a[i][2], nih, re[i][j]);
        re[i][j] = mfmabf(a[i][2], nil, re[i][j]);
        re[i][j] = mfmabf(a[i][3], nih, re[i][j]);
        im[i][j] = mfmabf(a[i][0], b[2], im[i][j]);
        im[i][j] = mfmabf(a[i][0], b[3], im[i][j]);
        im[i][j] = mfmabf(a[i][1], b[2], im[i][j]);
        im[i][j] = mfmabf(a[i][2], b[0], im[i][j]);
        im[i][j] = mfmabf(a[i][2], b[1], im[i][j]);
        im[i][j] = mfmabf(a[i][3], b[0], im[i][j]);
      }
    }
    if (++steps == kGFlushSteps || kb + 1 == nkb) {
      flush();
      steps = 0;
    }
  }
}

// FP32 form of the wide GEMM: A rounded to FP32 while staged (in the
// permuted 16-row layout of split_rows_f32_kernel), B split once per call.
__global__ __launch_bounds__(256, 2) void gemm_f32_wide_kernel(
    GemmArgs g, const uint4 *__restrict__ bt, int ldn, int m_tiles,
    int n_tiles) {
  extern __shared__ uint4 fwsm[];
  uint4 *As = fwsm;                          // [part][row][kGColStride]
  uint4 *Bs = fwsm + 2 * kGT * kGColStride;  // [part][col][kGColStride]
  float *Af = reinterpret_cast<float *>(As);
  const int total = m_tiles * n_tiles;
  const int t = xcd_remap(blockIdx.x, total);
  const int mt = t / n_tiles, nt = t - mt * n_tiles;
  const long M0 = (long)mt * kGT;
  const int N0 = nt * kGT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  const int q = lane >> 4, cl = lane & 15;
  f4 re[4][4], im[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      re[i][j] = f4{0, 0, 0, 0};
      im[i][j] = f4{0, 0, 0, 0};
    }
  int zero = 0;
  int soff = (threadIdx.x >> 2) * 4 + (threadIdx.x & 3);
  auto flush = [&]() __attribute__((always_inline)) {
    asm volatile("" : "+v"(zero));
    const int n0 = N0 + wc + accf_col(lane) + zero;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long m = M0 + wr + i * 16 + accf_row(lane, e);
        if (m < g.m) {
          double *cr = g.c + m * g.ldc + n0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (n0 + j * 16 < g.n) {
              cr[j * 16] += g.alpha * (double)re[i][j][e];
              cr[g.c_im + j * 16] += g.alpha * (double)im[i][j][e];
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[i][j][e] = 0.f;
          im[i][j][e] = 0.f;
        }
      }
  };
  const int nkb = g.k / 16;
  int steps = 0;
  for (int kb = 0; kb < nkb; ++kb) {
    __syncthreads();
    asm volatile("" : "+v"(soff));
    // A: thread (row soff / 4 (+ 64), q4 = soff % 4) rounds rows k = 16 kb +
    // 4 q4 + c, c < 4, of its row; row 4 s + q goes to float 4 q + s
#pragma unroll
    for (int hc = 0; hc < 2; ++hc) {
      const int r = (soff >> 2) + 64 * hc, q4 = soff & 3;
      const long m = M0 + r;
      double vr[4] = {0.0, 0.0, 0.0, 0.0}, vi[4] = {0.0, 0.0, 0.0, 0.0};
      if (m < g.m) {
        const double *src = g.a + m * g.lda + (long)kb * 16 + q4 * 4;
        const double2 r0 = *reinterpret_cast<const double2 *>(src);
        const double2 r1 = *reinterpret_cast<const double2 *>(src + 2);
        const double2 i0 = *reinterpret_cast<const double2 *>(src + g.a_im);
        const double2 i1 = *reinterpret_cast<const double2 *>(src + g.a_im + 2);
        vr[0] = r0.x; vr[1] = r0.y; vr[2] = r1.x; vr[3] = r1.y;
        vi[0] = i0.x; vi[1] = i0.y; vi[2] = i1.x; vi[3] = i1.y;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        // k = 4 q4 + c = 4 s + q with s = q4, q = c
        Af[((0 * kGT + r) * kGColStride) * 4 + 4 * c + q4] = (float)vr[c];
        Af[((1 * kGT + r) * kGColStride) * 4 + 4 * c + q4] = (float)vi[c];
      }
    }
    // B: items it = part (it / 2), columns + 64 (it % 2)
    const uint4 *sb = bt + (long)kb * 8 * ldn + soff;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int part = it >> 1, hc = it & 1;
      const uint4 v = sb[(part * ldn + N0 + 64 * hc) * 4];
      const int col = (soff >> 2) + 64 * hc;
      Bs[(part * kGT + col) * kGColStride + (soff & 3)] = v;
    }
    __syncthreads();
    uint4 a[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
        a[i][pp] = As[(pp * kGT + wr + i * 16 + cl) * kGColStride + q];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint4 b[2];
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
        b[pp] = Bs[(pp * kGT + wc + j * 16 + cl) * kGColStride + q];
      const float br[4] = {__uint_as_float(b[0].x), __uint_as_float(b[0].y),
                           __uint_as_float(b[0].z), __uint_as_float(b[0].w)};
      const float bi[4] = {__uint_as_float(b[1].x), __uint_as_float(b[1].y),
                           __uint_as_float(b[1].z), __uint_as_float(b[1].w)};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float ar[4] = {__uint_as_float(a[i][0].x), __uint_as_float(a[i][0].y),
                             __uint_as_float(a[i][0].z), __uint_as_float(a[i][0].w)};
        const float ai[4] = {__uint_as_float(a[i][1].x), __uint_as_float(a[i][1].y),
                             __uint_as_float(a[i][1].z), __uint_as_float(a[i][1].w)};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          // Re += ar br - ai bi;  Im += ar bi + ai br
          re[i][j] = mfma32(ar[s], br[s], re[i][j]);
          re[i][j] = mfma32(ai[s], -bi[s], re[i][j]);
          im[i][j] = mfma32(ar[s], bi[s], im[i][j]);
          im[i][j] = mfma32(ai[s], br[s], im[i][j]);
        }
      }
    }
    if (++steps == kFFlushSteps || kb + 1 == nkb) {
      flush();
      steps = 0;
    }
  }
}

// One block per (tile, 1/kGRedParts of its elements).
constexpr int kGRedParts = 16;
template <int kTs>
__global__ void gram_reduce_kernel(const double *__restrict__ partial,
                                   int n_tiles, int T, int nsplit, int ncol,
                                   double sign, double *__restrict__ out,
                                   int beta) {
  const int tile_id = blockIdx.x;
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kTs, J0 = tile.y * kTs;
  constexpr int per = kTs * kTs / kGRedParts;
  const int e0 = blockIdx.y * per;
  for (int e = e0 + threadIdx.x; e < e0 + per; e += blockDim.x) {
    const int r = e / kTs, c = e % kTs;
    const int g = I0 + r, gp = J0 + c;
    if (g >= ncol || gp >= ncol) continue;
    if (tile.x == tile.y && r < c) continue;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const double *p = partial + ((long)s * n_tiles + tile_id) * 2L * kTs * kTs;
      sr += p[e];
      si += p[kTs * kTs + e];
    }
    sr *= sign;
    si *= sign;
    if (g == gp) si = 0.0;  // the diagonal of A^H D A is real
    double *d1 = out + 2L * ((long)g * ncol + gp);
    double *d2 = out + 2L * ((long)gp * ncol + g);
    if (beta) {
      d1[0] += sr;
      d1[1] += si;
      if (g != gp) {
        d2[0] += sr;
        d2[1] -= si;
      }
    } else {
      d1[0] = sr;
      d1[1] = si;
      if (g != gp) {
        d2[0] = sr;
        d2[1] = -si;
      }
    }
  }
}

}  // namespace

// Work space of the Gram paths: split-K partials and converted rows.
//  * FP32: one copy of a K chunk.
//  * BF16x3, one matrix: an I and a J copy of a K chunk.
//  * BF16x3, several frequencies: the I copy of the whole K range (split
//    once) and the row weights of a K chunk per frequency; the Gram kernel
//    forms the weighted J operand from the I copy while staging it.
struct GramPlan {
  int ts, ncol, ldb, T, n_tiles, nsplit, kb_per_split, rows_step;
  bool resident_i;
  long kc, nchunks;
  size_t partial_bytes, i_bytes, j_bytes, w_bytes;
};

static GramPlan gram_plan(const HerkArgs &h, ssrpa_precision prec) {
  GramPlan p{};
  const bool bf = prec == SSRPA_BF16X3;
  p.rows_step = bf ? 32 : 16;
  // Outputs up to kGSmallCols columns take 64-wide tiles: at N = 400 the
  // 128-wide grid computes 2.0x the lower triangle, the 64-wide one 1.4x
  // (4 resident blocks per CU instead of 2, half the MFMA work per staged
  // byte).
  p.ts = h.ncol <= kGSmallCols ? kGSmallTile : kGT;
  p.ncol = h.ncol;
  p.ldb = round_up(std::max(h.ncol, 1), kGT);
  p.T = round_up(std::max(h.ncol, 1), p.ts) / p.ts;
  p.n_tiles = p.T * (p.T + 1) / 2;
  // 8 bytes per column and row in both forms (4 bf16 parts or 2 floats)
  const size_t row_bytes = (size_t)p.ldb * 8;
  const long kmax = std::max<long>(32, (long)(kGChunkBytes / row_bytes) / 32 * 32);
  const long k32 = std::max<long>(32, (h.k + 31) / 32 * 32);
  p.kc = std::min(kmax, k32);
  p.nchunks = std::max<long>(1, (h.k + p.kc - 1) / p.kc);
  const int nkb = (int)(p.kc / p.rows_step);
  // Split K so that the blocks of one frequency fill whole waves of the
  // resident blocks: the fewest splits whose last wave is at least 95% full
  // (and, from half a wave of tiles, that give two waves or more), else the
  // fullest, within 4 waves.  Split s of every tile covers the same K range,
  // so blocks of one wave share staged rows in L2.  Measured on BF16x3 with
  // 128-wide tiles (512 resident): 496 tiles in two waves of half K beat one
  // wave (55.9 against 57.2 ms); 10 tiles in one wave of 49 splits beat two
  // waves (31.2 against 32.8 ms) and 52 splits (520 blocks, a nearly empty
  // second wave: 35.5 ms).
  // Resident blocks: 256 CUs x (2 on 128-wide tiles; on 64-wide tiles 4 for
  // BF16x3 (VGPRs and LDS), 6 for FP32 (VGPRs)).
  const long kResident = 256L * (p.ts == kGT ? 2 : (bf ? 4 : 6));
  const long min_waves = p.n_tiles >= kResident / 2 ? 2 : 1;
  const int smax = std::max(1, std::min<int>(nkb, (int)(4 * kResident / p.n_tiles)));
  int nsplit = 1;
  double best = 0.0;
  for (int sp = 1; sp <= smax; ++sp) {
    const long blocks = (long)p.n_tiles * sp;
    const long waves = (blocks + kResident - 1) / kResident;
    const double fill = (double)blocks / (double)(waves * kResident);
    if (fill >= 0.95 && waves >= min_waves) {
      nsplit = sp;
      break;
    }
    if (fill > best + 1e-12) {
      best = fill;
      nsplit = sp;
    }
  }
  p.kb_per_split = (nkb + nsplit - 1) / nsplit;
  p.nsplit = (nkb + p.kb_per_split - 1) / p.kb_per_split;
  p.partial_bytes = sizeof(double) * 2L * p.ts * p.ts * p.n_tiles * p.nsplit;
  // several frequencies: the I rows are converted once (BF16x3: unweighted
  // I copy; FP32: unweighted rows, Delta applied to B in the Gram kernel)
  p.resident_i = h.n_omega > 1 && !h.unit_weight;
  p.i_bytes = p.resident_i ? (size_t)(p.nchunks * p.kc) * row_bytes
                           : (size_t)p.kc * row_bytes;
  p.j_bytes = (bf && !p.resident_i) ? (size_t)p.kc * row_bytes : 0;
  p.w_bytes = p.resident_i ? (size_t)p.kc * sizeof(float) : 0;
  return p;
}

// One Gram pass over nkb row blocks: BF16x3 with I operand a and J operand b
// (weighted = J formed from a and the row weights w), or FP32 on the copy a
// (weighted = row weights w applied to B).
template <int kTs>
static void launch_gram(const GramPlan &p, bool bf, bool weighted, const uint4 *a,
                        const uint4 *b, int nkb, const float *w, double *partial,
                        hipStream_t s) {
  const dim3 gg((unsigned)p.n_tiles, (unsigned)p.nsplit);
  if (bf) {
    if (weighted)
      hipLaunchKernelGGL((gram_bf16x3_kernel<kTs, true>), gg, dim3(256),
                         gram_lds(4, kTs), s, a, a, p.ldb, p.ncol, nkb, p.T, p.n_tiles,
                         p.kb_per_split, w, partial);
    else
      hipLaunchKernelGGL((gram_bf16x3_kernel<kTs, false>), gg, dim3(256),
                         gram_lds(4, kTs), s, a, b, p.ldb, p.ncol, nkb, p.T, p.n_tiles,
                         p.kb_per_split, nullptr, partial);
  } else if (weighted) {
    hipLaunchKernelGGL((gram_f32_kernel<kTs, true>), gg, dim3(256), gram_lds(2, kTs),
                       s, a, p.ldb, p.ncol, nkb, p.T, p.n_tiles, p.kb_per_split, w,
                       partial);
  } else {
    hipLaunchKernelGGL((gram_f32_kernel<kTs, false>), gg, dim3(256),
                       gram_lds(2, kTs), s, a, p.ldb, p.ncol, nkb, p.T, p.n_tiles,
                       p.kb_per_split, nullptr, partial);
  }
}

size_t herk_gram_workspace(const HerkArgs &h, ssrpa_precision prec) {
  const GramPlan p = gram_plan(h, prec);
  return p.partial_bytes + p.i_bytes + p.j_bytes + p.w_bytes;
}

void herk_gram(Context *ctx, const HerkArgs &h, ssrpa_precision prec,
               double *out, long out_stride, int beta, DevBuf &ws,
               hipStream_t s) {
  SSRPA_REQUIRE(prec == SSRPA_FP32 || prec == SSRPA_BF16X3, SSRPA_ERR_ARG,
                "herk_gram: FP32 or BF16x3 only");
  const bool bf = prec == SSRPA_BF16X3;
  const GramPlan p = gram_plan(h, prec);
  ws.ensure(ctx, p.partial_bytes + p.i_bytes + p.j_bytes + p.w_bytes, s);
  double *partial = ws.as<double>();
  uint4 *wi = reinterpret_cast<uint4 *>(ws.as<char>() + p.partial_bytes);
  uint4 *wj = reinterpret_cast<uint4 *>(ws.as<char>() + p.partial_bytes + p.i_bytes);
  float *wrow = reinterpret_cast<float *>(ws.as<char>() + p.partial_bytes + p.i_bytes +
                                          p.j_bytes);
  static bool attr = [] {
    SSRPA_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void *>(&gram_bf16x3_kernel<kGT, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram_lds(4, kGT)));
    SSRPA_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void *>(&gram_bf16x3_kernel<kGT, true>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram_lds(4, kGT)));
    return true;
  }();
  (void)attr;
  auto gram = [&](bool weighted, const uint4 *a, const uint4 *b, int nkb,
                  const float *w) {
    if (p.ts == kGT)
      launch_gram<kGT>(p, bf, weighted, a, b, nkb, w, partial, s);
    else
      launch_gram<kGSmallTile>(p, bf, weighted, a, b, nkb, w, partial, s);
  };
  const long blk_stride = 16L * p.ldb;  // uint4 per row block (both forms)
  auto chunk_rows = [&](long c) {
    return (int)std::max<long>(0, std::min(p.kc, h.k - c * p.kc));
  };
  auto split_grid = [&](int nkb) {
    return dim3((unsigned)((p.ldb + 255) / 256), (unsigned)nkb);
  };
  const int ti = (h.timer && h.timer->on) ? h.timer->start(h.stage, s) : -1;
  if (p.resident_i) {
    // both forms hold 8 bytes per column and row, so chunk c starts at the
    // same offset
    HerkArgs hu = h;
    hu.unit_weight = 1;
    for (long c = 0; c < p.nchunks; ++c) {
      const int nkb = (chunk_rows(c) + p.rows_step - 1) / p.rows_step;
      if (nkb == 0) continue;
      if (bf)
        hipLaunchKernelGGL(split_rows_bf16_kernel<false>, split_grid(nkb), dim3(256),
                           0, s, h, c * p.kc, chunk_rows(c), p.ldb, 0, 0,
                           wi + c * (p.kc / 32) * blk_stride, nullptr);
      else
        hipLaunchKernelGGL(split_rows_f32_kernel, split_grid(nkb), dim3(256), 0,
                           s, hu, c * p.kc, chunk_rows(c), p.ldb, 0,
                           wi + c * (p.kc / 32) * blk_stride);
    }
    SSRPA_HIP(hipGetLastError());
  }
  for (int om = 0; om < h.n_omega; ++om) {
    fill_zero(partial, p.partial_bytes, s);
    for (long c = 0; c < p.nchunks; ++c) {
      const long k0 = c * p.kc;
      const int nrows = chunk_rows(c);
      const int nkb = (nrows + p.rows_step - 1) / p.rows_step;
      if (bf) {
        if (p.resident_i) {
          // the J operand is weighted while staged from the resident I copy
          const uint4 *ci = wi + c * (p.kc / 32) * blk_stride;
          const int n_pos = nkb * 32;
          if (nkb > 0)
            hipLaunchKernelGGL(row_weights_bf_kernel, dim3((n_pos + 255) / 256),
                               dim3(256), 0, s, h, k0, nrows, n_pos, om, wrow);
          gram(true, ci, ci, nkb, wrow);
        } else {
          // one matrix: both copies from one read of the rows (weighting J
          // while staged would be redone by every tile of a column; with
          // unit weights the J copy is kGJScale x, rounded independently of
          // the I copy)
          if (nkb > 0)
            hipLaunchKernelGGL(split_rows_bf16_kernel<true>, split_grid(nkb),
                               dim3(256), 0, s, h, k0, nrows, p.ldb, om, 1, wi, wj);
          gram(false, wi, wj, nkb, nullptr);
        }
      } else if (p.resident_i) {
        // unweighted rows converted once; this frequency's Delta per row
        const int n_pos = nkb * 16;
        if (nkb > 0)
          hipLaunchKernelGGL(row_weights_f32_kernel, dim3((n_pos + 255) / 256),
                             dim3(256), 0, s, h, k0, nrows, n_pos, om, wrow);
        gram(true, wi + c * (p.kc / 32) * blk_stride, nullptr, nkb, wrow);
      } else {
        if (nkb > 0)
          hipLaunchKernelGGL(split_rows_f32_kernel, split_grid(nkb), dim3(256), 0,
                             s, h, k0, nrows, p.ldb, om, wi);
        gram(false, wi, nullptr, nkb, nullptr);
      }
      SSRPA_HIP(hipGetLastError());
    }
    // BF16x3 carries the sign in d_p (and a factor kGJScale for unit
    // weights); FP32 used sqrt|d_p| on both sides, or (several
    // frequencies) the signed Delta on one
    const double scale = bf ? (h.unit_weight ? 1.0 / kGJScale : 1.0)
                            : (h.unit_weight || p.resident_i ? 1.0 : -1.0);
    const dim3 rg((unsigned)p.n_tiles, kGRedParts);
    if (p.ts == kGT)
      hipLaunchKernelGGL(gram_reduce_kernel<kGT>, rg, dim3(256), 0, s, partial,
                         p.n_tiles, p.T, p.nsplit, h.ncol, scale,
                         out + om * out_stride, beta);
    else
      hipLaunchKernelGGL(gram_reduce_kernel<kGSmallTile>, rg, dim3(256), 0, s,
                         partial, p.n_tiles, p.T, p.nsplit, h.ncol, scale,
                         out + om * out_stride, beta);
    SSRPA_HIP(hipGetLastError());
  }
  if (ti >= 0) h.timer->stop(ti, s);
}

size_t gemm_bf16x3_wide_workspace(const GemmArgs &g) {
  return (size_t)g.k * round_up(g.n, kGT) * 8;
}

void gemm_bf16x3_wide(Context *ctx, const GemmArgs &g, DevBuf &ws,
                      hipStream_t s) {
  SSRPA_REQUIRE(g.beta == 0.0 && g.k % 32 == 0, SSRPA_ERR_ARG,
                "gemm_bf16x3_wide: beta = 0 and k padded to 32 only");
  const int ldn = round_up(g.n, kGT);
  ws.ensure(ctx, gemm_bf16x3_wide_workspace(g), s);
  uint4 *bt = ws.as<uint4>();
  // B rows (k) split once into [kb][part][n][32]
  HerkArgs hb{};
  hb.a = g.b;
  hb.lda = g.ldb;
  hb.im_off = g.b_im;
  hb.ncol = g.n;
  hb.unit_weight = 1;
  hipLaunchKernelGGL(split_rows_bf16_kernel<false>,
                     dim3((unsigned)((ldn + 255) / 256), (unsigned)(g.k / 32)),
                     dim3(256), 0, s, hb, 0L, g.k, ldn, 0, 0, bt, nullptr);
  // C accumulates its flushes: zero the rows first
  fill_zero(g.c, sizeof(double) * (size_t)g.m * g.ldc, s);
  static bool attr = [] {
    SSRPA_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void *>(&gemm_bf16x3_wide_kernel),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGLds));
    return true;
  }();
  (void)attr;
  const long m_tiles = (g.m + kGT - 1) / kGT;
  const int n_tiles = ldn / kGT;
  SSRPA_REQUIRE(m_tiles * n_tiles < (1L << 31), SSRPA_ERR_ARG, "gemm too large");
  hipLaunchKernelGGL(gemm_bf16x3_wide_kernel, dim3((unsigned)(m_tiles * n_tiles)),
                     dim3(256), kGLds, s, g, bt, ldn, (int)m_tiles, n_tiles);
  SSRPA_HIP(hipGetLastError());
}

size_t gemm_f32_wide_workspace(const GemmArgs &g) {
  return (size_t)g.k * round_up(g.n, kGT) * 8;
}

void gemm_f32_wide(Context *ctx, const GemmArgs &g, DevBuf &ws, hipStream_t s) {
  SSRPA_REQUIRE(g.beta == 0.0 && g.k % 16 == 0, SSRPA_ERR_ARG,
                "gemm_f32_wide: beta = 0 and k padded to 16 only");
  const int ldn = round_up(g.n, kGT);
  ws.ensure(ctx, gemm_f32_wide_workspace(g), s);
  uint4 *bt = ws.as<uint4>();
  HerkArgs hb{};
  hb.a = g.b;
  hb.lda = g.ldb;
  hb.im_off = g.b_im;
  hb.ncol = g.n;
  hb.unit_weight = 1;
  hipLaunchKernelGGL(split_rows_f32_kernel,
                     dim3((unsigned)((ldn + 255) / 256), (unsigned)(g.k / 16)),
                     dim3(256), 0, s, hb, 0L, g.k, ldn, 0, bt);
  fill_zero(g.c, sizeof(double) * (size_t)g.m * g.ldc, s);
  const long m_tiles = (g.m + kGT - 1) / kGT;
  const int n_tiles = ldn / kGT;
  SSRPA_REQUIRE(m_tiles * n_tiles < (1L << 31), SSRPA_ERR_ARG, "gemm too large");
  hipLaunchKernelGGL(gemm_f32_wide_kernel, dim3((unsigned)(m_tiles * n_tiles)),
                     dim3(256), kFLds, s, g, bt, ldn, (int)m_tiles, n_tiles);
  SSRPA_HIP(hipGetLastError());
}

void gemm_mixed_launch(const GemmArgs &g, ssrpa_precision prec, int m_tiles,
                       int n_tiles, hipStream_t s) {
  const dim3 grid((unsigned)(m_tiles * n_tiles));
  if (prec == SSRPA_FP32)
    hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, s, g, m_tiles,
                       n_tiles);
  else
    hipLaunchKernelGGL(gemm_bf16x3_kernel, grid, dim3(256), 0, s, g, m_tiles,
                       n_tiles);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
