// Dense complex contractions on the MFMA units of gfx950.
//
//  * herk:  X_j = A^H diag(d_j) A for a batch of weight vectors d_j, the form
//           of the polarizability sum chi0 = M^H Delta M / Omega (paper,
//           Eq. 6; per valence block, Eq. 15) and of its subspace version
//           chi0_s = M_s^H Delta M_s (Eq. 8).  d_j,p = -4 de_p / (de_p^2 +
//           w_j^2) / Omega, computed from the pair energy gaps while the
//           operand tile is staged, so Delta is never stored.
//  * gemm:  C = alpha A B + beta C, used for the projection M_s = M C_s
//           (Eq. 7) and for small basis updates.
//
// Operands are planar complex: every row holds its real parts, then (at a
// fixed offset) its imaginary parts.  A complex product is four real MFMA
// products: Re = ArBr + AiBi (conjugated A) or ArBr - AiBi, and
// Im = ArBi - AiBr or ArBi + AiBr.
//
// FP64 path: v_mfma_f64_16x16x4f64.  One 256-thread block owns a 64 x 64
// complex output tile; each wave owns a 32 x 32 quadrant (2 x 2 MFMA tiles,
// real and imaginary accumulators).  The K loop stages 16-row chunks of both
// operands through LDS.  HERK computes only lower-triangle tiles and splits K
// over blocks when there are too few tiles; the partial tiles are summed in a
// fixed order by a second kernel that also mirrors the Hermitian upper half,
// so results are deterministic run to run.
#include <cmath>

#include "internal.hpp"
#include "tiles.hpp"

namespace ssrpa {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kT = 64;    // output tile (complex)
constexpr int kKc = 16;   // K rows per LDS stage
constexpr int kPad = 2;   // LDS row padding (doubles)

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output element (row, col) held by lane `l` in accumulator slot e of a
// 16 x 16 f64 MFMA tile: slot e of lane l holds row l/16 + 4e, column l%16.
__device__ __forceinline__ int acc_row(int l, int e) { return (l >> 4) + 4 * e; }
__device__ __forceinline__ int acc_col(int l) { return l & 15; }

// ---------------------------------------------------------------- HERK f64

__global__ __launch_bounds__(256, 3) void herk_f64_kernel(
    HerkArgs h, int n_tiles, long kchunk, double *__restrict__ partial) {
  __shared__ double As[2][kKc][kT + kPad];
  __shared__ double Bs[2][kKc][kT + kPad];
  const int tile_id = xcd_remap(blockIdx.x, n_tiles);
  const int split = blockIdx.y;
  const int om_i = blockIdx.z;
  const int2 tile = tri_tile_blocked(tile_id, h.ld / kT);
  const int I0 = tile.x * kT, J0 = tile.y * kT;
  const double om = h.unit_weight ? 0.0 : h.omega[om_i];
  const long kbeg = split * kchunk;
  const long kend = min(h.k, kbeg + kchunk);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  d4 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = d4{0, 0, 0, 0};
      im[i][j] = d4{0, 0, 0, 0};
    }

  // staging map: 256 threads x 4 loads of double2 cover 2 ops x 2 parts x
  // 16 rows x 64 columns.  The next chunk is fetched into registers while
  // the current one is multiplied.
  const int sr = (threadIdx.x >> 4) & 15;      // k row of this thread's items
  double2 pv[4], pu[4];
  double pde = 0.0;
  auto fetch = [&](long k0) __attribute__((always_inline)) {
    const long p = k0 + sr;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;   // 0..1023
      const int op = idx >> 9;                   // 0: A (rows I), 1: B (cols J)
      const int part = (idx >> 8) & 1;           // 0 re, 1 im
      const int c2 = (idx & 15) * 2;             // column pair (0..30) x2 -> 64
      const int col0 = op ? J0 : I0;
      pv[it] = make_double2(0.0, 0.0);
      pu[it] = make_double2(0.0, 0.0);
      if (p < kend) {
        const double *src = h.a + p * h.lda + part * h.im_off + col0;
        pv[it] = *reinterpret_cast<const double2 *>(src + c2);
        pu[it] = *reinterpret_cast<const double2 *>(src + c2 + 32);
      }
    }
    if (!h.unit_weight && p < kend) pde = h.de[p];
  };
  fetch(kbeg);
  for (long k0 = kbeg; k0 < kend; k0 += kKc) {
    // weight of row sr (B operand): Delta_p(i omega) = -4 de / (de^2 + omega^2)
    double sc = 0.0;
    if (k0 + sr < kend)
      sc = h.unit_weight ? 1.0 : -4.0 * pde / (pde * pde + om * om) * h.wscale;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int op = idx >> 9, part = (idx >> 8) & 1, c2 = (idx & 15) * 2;
      const double s = op ? sc : 1.0;
      double *dst = op ? &Bs[part][sr][0] : &As[part][sr][0];
      dst[c2] = pv[it].x * s;
      dst[c2 + 1] = pv[it].y * s;
      dst[c2 + 32] = pu[it].x * s;
      dst[c2 + 33] = pu[it].y * s;
    }
    __syncthreads();
    if (k0 + kKc < kend) fetch(k0 + kKc);
#pragma unroll
    for (int ks = 0; ks < kKc; ks += 4) {
      const int kr = ks + (lane >> 4);
      const int cl = lane & 15;
      double ar[2], ai[2], br[2], bi[2];
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
          re[i][j] = mfma64(ar[i], br[j], re[i][j]);
          re[i][j] = mfma64(ai[i], bi[j], re[i][j]);
          im[i][j] = mfma64(ar[i], bi[j], im[i][j]);
          im[i][j] = mfma64(-ai[i], br[j], im[i][j]);
        }
    }
    __syncthreads();
  }
  // partial tile: [om][split][tile][part][64][64]
  double *out = partial + (((long)om_i * gridDim.y + split) * n_tiles + tile_id) *
                              2L * kT * kT;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr + i * 16 + acc_row(lane, e);
        const int c = wc + j * 16 + acc_col(lane);
        out[r * kT + c] = re[i][j][e];
        out[kT * kT + r * kT + c] = im[i][j][e];
      }
}

// Two frequencies per block (n_omega >= 2): the K chunk is staged once,
// unweighted, and each frequency's weights Delta_p(i omega_f) scale the B
// fragments in registers, so one staging and its barriers serve twice the
// MFMA work.  Same tiles, split-K and partial layout as herk_f64_kernel.
__global__ __launch_bounds__(256, 2) void herk_f64_pair_kernel(
    HerkArgs h, int n_tiles, long kchunk, double *__restrict__ partial) {
  __shared__ double As[2][kKc][kT + kPad];
  __shared__ double Bs[2][kKc][kT + kPad];
  __shared__ double wk[2][kKc];
  // each XCD takes a contiguous run of (frequency pair, split, tile)
  const int blk = xcd_linear(n_tiles);
  const int per_pair = n_tiles * (int)gridDim.y;
  const int pair = blk / per_pair;
  const int split = (blk - pair * per_pair) / n_tiles;
  const int tile_id = blk - pair * per_pair - split * n_tiles;
  const int om0 = 2 * pair;
  const bool two = om0 + 1 < h.n_omega;
  const int2 tile = tri_tile_blocked(tile_id, h.ld / kT);
  const int I0 = tile.x * kT, J0 = tile.y * kT;
  const double oma = h.omega[om0], omb = two ? h.omega[om0 + 1] : 0.0;
  const long kbeg = split * kchunk;
  const long kend = min(h.k, kbeg + kchunk);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const unsigned live = live_subtiles<2>(I0 + wr, J0 + wc, h.ncol);
  d4 re[2][2][2], im[2][2][2];   // [frequency][i][j]
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        re[f][i][j] = d4{0, 0, 0, 0};
        im[f][i][j] = d4{0, 0, 0, 0};
      }
  const int sr = (threadIdx.x >> 4) & 15;
  double2 pv[4], pu[4];
  double pde = 0.0;
  auto fetch = [&](long k0) __attribute__((always_inline)) {
    const long p = k0 + sr;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int op = idx >> 9, part = (idx >> 8) & 1, c2 = (idx & 15) * 2;
      const int col0 = op ? J0 : I0;
      pv[it] = make_double2(0.0, 0.0);
      pu[it] = make_double2(0.0, 0.0);
      if (p < kend) {
        const double *src = h.a + p * h.lda + part * h.im_off + col0;
        pv[it] = *reinterpret_cast<const double2 *>(src + c2);
        pu[it] = *reinterpret_cast<const double2 *>(src + c2 + 32);
      }
    }
    if (p < kend) pde = h.de[p];
  };
  fetch(kbeg);
  for (long k0 = kbeg; k0 < kend; k0 += kKc) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int op = idx >> 9, part = (idx >> 8) & 1, c2 = (idx & 15) * 2;
      double *dst = op ? &Bs[part][sr][0] : &As[part][sr][0];
      dst[c2] = pv[it].x;
      dst[c2 + 1] = pv[it].y;
      dst[c2 + 32] = pu[it].x;
      dst[c2 + 33] = pu[it].y;
    }
    if ((threadIdx.x & 15) == 0) {
      // Delta_p(i omega) = -4 de / (de^2 + omega^2), zero past the chunk
      const bool in = k0 + sr < kend;
      wk[0][sr] = in ? -4.0 * pde / (pde * pde + oma * oma) * h.wscale : 0.0;
      wk[1][sr] = in ? -4.0 * pde / (pde * pde + omb * omb) * h.wscale : 0.0;
    }
    __syncthreads();
    if (k0 + kKc < kend) fetch(k0 + kKc);
#pragma unroll
    for (int ks = 0; ks < kKc; ks += 4) {
      const int kr = ks + (lane >> 4);
      const int cl = lane & 15;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As[0][kr][wr + i * 16 + cl];
        ai[i] = As[1][kr][wr + i * 16 + cl];
        br[i] = Bs[0][kr][wc + i * 16 + cl];
        bi[i] = Bs[1][kr][wc + i * 16 + cl];
      }
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double w = wk[f][kr];
        const double bw[2] = {br[0] * w, br[1] * w}, biw[2] = {bi[0] * w, bi[1] * w};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (!(live >> (2 * i + j) & 1u)) continue;
            re[f][i][j] = mfma64(ar[i], bw[j], re[f][i][j]);
            re[f][i][j] = mfma64(ai[i], biw[j], re[f][i][j]);
            im[f][i][j] = mfma64(ar[i], biw[j], im[f][i][j]);
            im[f][i][j] = mfma64(-ai[i], bw[j], im[f][i][j]);
          }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    if (f == 1 && !two) break;
    double *out = partial + (((long)(om0 + f) * gridDim.y + split) * n_tiles + tile_id) *
                                2L * kT * kT;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr + i * 16 + acc_row(lane, e);
          const int c = wc + j * 16 + acc_col(lane);
          out[r * kT + c] = re[f][i][j][e];
          out[kT * kT + r * kT + c] = im[f][i][j][e];
        }
  }
}

// Sum split partials in order and write the Hermitian matrix (both halves).
__global__ void herk_reduce_kernel(const double *__restrict__ partial,
                                   int n_tiles, int T,
                                   int nsplit, int ncol, double *__restrict__ out,
                                   long out_stride, int beta) {
  const int tile_id = blockIdx.x;
  const int om_i = blockIdx.y;
  const int2 tile = tri_tile_blocked(tile_id, T);
  const int I0 = tile.x * kT, J0 = tile.y * kT;
  double *o = out + om_i * out_stride;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int r = e / kT, c = e % kT;
    const int g = I0 + r, gp = J0 + c;
    if (g >= ncol || gp >= ncol) continue;
    if (tile.x == tile.y && r < c) continue;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const double *p = partial +
                        (((long)om_i * nsplit + s) * n_tiles + tile_id) * 2L * kT * kT;
      sr += p[e];
      si += p[kT * kT + e];
    }
    if (g == gp) si = 0.0;  // exact: the diagonal of A^H D A is real
    double *d1 = o + 2L * ((long)g * ncol + gp);
    double *d2 = o + 2L * ((long)gp * ncol + g);
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

// ---------------------------------------------------------------- GEMM f64

__global__ __launch_bounds__(256, 3) void gemm_f64_kernel(GemmArgs g, int m_tiles,
                                                      int n_tiles) {
  __shared__ double As[2][kKc][kT + kPad];  // [part][k][m]
  __shared__ double Bs[2][kKc][kT + kPad];  // [part][k][n]
  const int total = m_tiles * n_tiles;
  const int b = xcd_remap(blockIdx.x, total);
  const int mt = b / n_tiles, nt = b % n_tiles;
  const long M0 = (long)mt * kT;
  const int N0 = nt * kT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  d4 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = d4{0, 0, 0, 0};
      im[i][j] = d4{0, 0, 0, 0};
    }
  // A: 64 rows x 16 k x 2 parts = 2048 doubles: thread -> (row, part, 8 k);
  // B: 16 k x 64 cols x 2 parts: thread -> (k, part, 8 cols).  The next K
  // chunk is fetched into registers while the current one is multiplied.
  const int arow = threadIdx.x >> 2, apart = (threadIdx.x >> 1) & 1;
  const int akq = (threadIdx.x & 1) * 8;
  const int bkr = threadIdx.x >> 4, bpart = (threadIdx.x >> 3) & 1;
  const int bcq = (threadIdx.x & 7) * 8;
  double2 av[4], bv[4];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
    const long m = M0 + arow;
#pragma unroll
    for (int x = 0; x < 4; ++x) av[x] = make_double2(0.0, 0.0);
    if (m < g.m) {
      const double *src = g.a + m * g.lda + apart * g.a_im + k0 + akq;
#pragma unroll
      for (int x = 0; x < 4; ++x) av[x] = *reinterpret_cast<const double2 *>(src + 2 * x);
    }
    const double *srcb = g.b + (long)(k0 + bkr) * g.ldb + bpart * g.b_im + N0 + bcq;
#pragma unroll
    for (int x = 0; x < 4; ++x) bv[x] = *reinterpret_cast<const double2 *>(srcb + 2 * x);
  };
  fetch(0);
  for (int k0 = 0; k0 < g.k; k0 += kKc) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      As[apart][akq + 2 * x][arow] = av[x].x;
      As[apart][akq + 2 * x + 1][arow] = av[x].y;
      Bs[bpart][bkr][bcq + 2 * x] = bv[x].x;
      Bs[bpart][bkr][bcq + 2 * x + 1] = bv[x].y;
    }
    __syncthreads();
    if (k0 + kKc < g.k) fetch(k0 + kKc);
#pragma unroll
    for (int ks = 0; ks < kKc; ks += 4) {
      const int kr = ks + (lane >> 4);
      const int cl = lane & 15;
      double ar[2], ai[2], br[2], bi[2];
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
          re[i][j] = mfma64(ar[i], br[j], re[i][j]);
          re[i][j] = mfma64(-ai[i], bi[j], re[i][j]);
          im[i][j] = mfma64(ar[i], bi[j], im[i][j]);
          im[i][j] = mfma64(ai[i], br[j], im[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const long m = M0 + wr + i * 16 + acc_row(lane, e);
        const int n = N0 + wc + j * 16 + acc_col(lane);
        if (m >= g.m) continue;
        double *cr = g.c + m * g.ldc + n;
        double *ci = cr + g.c_im;
        const double vr = g.alpha * re[i][j][e];
        const double vi = g.alpha * im[i][j][e];
        if (g.beta != 0.0) {
          *cr = vr + g.beta * *cr;
          *ci = vi + g.beta * *ci;
        } else {
          *cr = vr;
          *ci = vi;
        }
      }
}

}  // namespace

// reduced-precision launchers (gemm_mixed.hip)
void gemm_mixed_launch(const GemmArgs &g, ssrpa_precision prec, int m_tiles,
                       int n_tiles, hipStream_t s);

// Tiles, K split and partial-tile bytes of an FP64 HERK.  K is split so
// that the blocks fill whole waves of the resident blocks (3 per CU for the
// one-frequency kernel, 2 for the two-frequency one): the fewest splits
// (up to 8, or 4 x the resident blocks) whose last wave is at least 98%
// full, else the fullest, with at least 8 K chunks per split.  (Rounding 512
// blocks up left 1953 medium chi0 tiles at 2.5 waves, 85% full, and the 16
// medium frequencies at 448 of 512; 3 splits fill 95.4% of 8 waves, 7
// splits 98.9% of 18.)
struct HerkF64Plan {
  int T, n_tiles;
  long nsplit, kchunk;
  size_t bytes;
};

static HerkF64Plan herk_f64_plan(const HerkArgs &h) {
  HerkF64Plan p{};
  p.T = h.ld / kT;
  p.n_tiles = p.T * (p.T + 1) / 2;
  const bool pair = h.n_omega >= 2 && !h.unit_weight;
  const long per_split = (long)p.n_tiles * (pair ? (h.n_omega + 1) / 2 : h.n_omega);
  const long resident = pair ? 512 : 768;
  const int kst = kKc;
  const long kr = std::max(1L, (h.k + kst - 1) / kst);
  const long smax =
      std::max(1L, std::min(kr / 8, std::max(8L, 4 * resident / std::max(1L, per_split))));
  long nsplit = 1;
  double best = 0.0;
  for (long sp = 1; sp <= smax; ++sp) {
    const long blocks = per_split * sp;
    const long waves = (blocks + resident - 1) / resident;
    const double fill = (double)blocks / (double)(waves * resident);
    if (fill >= 0.98) {
      nsplit = sp;
      break;
    }
    if (fill > best + 1e-12) {
      best = fill;
      nsplit = sp;
    }
  }
  p.kchunk = ((kr + nsplit - 1) / nsplit) * kst;
  p.nsplit = std::max(1L, (h.k + p.kchunk - 1) / p.kchunk);
  p.bytes = sizeof(double) * 2L * kT * kT * p.n_tiles * p.nsplit * h.n_omega;
  return p;
}

size_t herk_f64_workspace(const HerkArgs &h) { return herk_f64_plan(h).bytes; }

void herk(Context *ctx, const HerkArgs &h, ssrpa_precision prec, double *out,
          long out_stride, int beta, DevBuf &ws, hipStream_t s) {
  SSRPA_REQUIRE(h.ld % kT == 0 && h.ncol <= h.ld, SSRPA_ERR_ARG,
                "herk: bad padding");
  if (prec != SSRPA_FP64) {
    herk_gram(ctx, h, prec, out, out_stride, beta, ws, s);
    return;
  }
  const HerkF64Plan p = herk_f64_plan(h);
  const int T = p.T, n_tiles = p.n_tiles;
  const long nsplit = p.nsplit, kchunk = p.kchunk;
  const size_t need = p.bytes;
  ws.ensure(ctx, need, s);
  DevBuf *wsb = &ws;
  if (h.k > 0) {
    const int ti = (h.timer && h.timer->on) ? h.timer->start(h.stage, s) : -1;
    if (h.n_omega >= 2 && !h.unit_weight)
      hipLaunchKernelGGL(herk_f64_pair_kernel,
                         dim3(n_tiles, (unsigned)nsplit, (h.n_omega + 1) / 2), dim3(256),
                         0, s, h, n_tiles, kchunk, wsb->as<double>());
    else
      hipLaunchKernelGGL(herk_f64_kernel, dim3(n_tiles, (unsigned)nsplit, h.n_omega),
                         dim3(256), 0, s, h, n_tiles, kchunk, wsb->as<double>());
    SSRPA_HIP(hipGetLastError());
    if (ti >= 0) h.timer->stop(ti, s);
  } else {
    fill_zero(wsb->as(), need, s);
  }
  hipLaunchKernelGGL(herk_reduce_kernel, dim3(n_tiles, h.n_omega), dim3(256), 0,
                     s, wsb->as<double>(), n_tiles, T, (int)nsplit, h.ncol,
                     out, out_stride, beta);
  SSRPA_HIP(hipGetLastError());
}

void gemm(Context *ctx, const GemmArgs &g, ssrpa_precision prec, DevBuf &ws,
          hipStream_t s) {
  SSRPA_REQUIRE(g.k % kT == 0 && g.n % kT == 0, SSRPA_ERR_ARG,
                "gemm: k and n must be padded to 64");
  if (g.m <= 0) return;
  if (prec == SSRPA_BF16X3 && g.beta == 0.0) {
    gemm_bf16x3_wide(ctx, g, ws, s);
    return;
  }
  if (prec == SSRPA_FP32 && g.beta == 0.0) {
    gemm_f32_wide(ctx, g, ws, s);
    return;
  }
  const long m_tiles = (g.m + kT - 1) / kT;
  const int n_tiles = g.n / kT;
  SSRPA_REQUIRE(m_tiles * n_tiles < (1L << 31), SSRPA_ERR_ARG, "gemm too large");
  if (prec != SSRPA_FP64) {
    gemm_mixed_launch(g, prec, (int)m_tiles, n_tiles, s);
    return;
  }
  hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)(m_tiles * n_tiles)),
                     dim3(256), 0, s, g, (int)m_tiles, n_tiles);
  SSRPA_HIP(hipGetLastError());
}

}  // namespace ssrpa
