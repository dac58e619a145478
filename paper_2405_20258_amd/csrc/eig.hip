// FP64 Hermitian eigensolver for the static-subspace basis: the n_eig
// eigenpairs of the static v^1/2 chi0 v^1/2 with the largest |eigenvalue|
// (paper, Method: the projector onto the subspace is built from the
// eigenvectors of the static polarizability with the greatest absolute
// eigenvalues).  The matrix is negative semidefinite, so these are the n_eig
// smallest (most negative) eigenvalues.
//
// Steps, all on the GPU:
//  1. Householder reduction A = Q T_c Q^H to Hermitian tridiagonal form, one
//     reflector H_k = I - tau u u^H per column (tau real); step k needs
//     p = tau A' u and the rank-two update A' -= u w^H + w u^H with
//     w = p - (tau/2)(u^H p) u.  The updates are deferred over panels of
//     columns (LAPACK's panel reduction): inside a panel A' is held as the
//     panel-start matrix minus the panel's rank-two terms, and the matrix
//     is updated once per panel.  Reflector k is stored in row k of the
//     work matrix (the part of the row that the reduction no longer needs).
//  2. A diagonal unitary D makes T = D^H T_c D real symmetric with off-
//     diagonal |e_k|.
//  3. Sturm-sequence multisection for the n_eig smallest eigenvalues of T
//     (one wave per eigenvalue, 64 brackets per round).
//  4. Inverse iteration on T - lambda I with a partially pivoted tridiagonal
//     LU (one thread per group of nearly equal eigenvalues; vectors of one
//     group are orthogonalized against each other at every iteration).
//  5. Back-transformation C = Q D Z.
//  6. One Newton-Schulz step C <- C (3I - C^H C) / 2 restores orthonormality
//     to rounding level (the inverse-iteration vectors of different groups
//     are orthogonal only to about eps |T| / gap).
#include <cfloat>
#include <cmath>

#include "internal.hpp"

namespace ssrpa {

namespace {

__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Block-wide sum (blockDim multiple of 64, <= 1024); all threads get it.
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// ------------------------------------------------ Householder reduction
//
// Blocked over panels of kNb columns.  Inside a panel the trailing matrix
// keeps its value A0 from the start of the panel; the current matrix is
//   A' = A0 - sum_i (V_i W_i^H + W_i V_i^H)
// over the panel's earlier reflectors V_i = u_i and their vectors W_i = w_i.
// Step k (slot j = k - k0 of the panel) runs two kernels:
//   col:  finishes step k-1: p = tau (A0 u - V (W^H u) - W (V^H u)) from the
//         hemv partials and w = p - (tau/2)(u^H p) u, where
//         u^H p = tau (u^H A0 u - 2 Re (V^H u)^H (W^H u)) needs no pass over
//         p; then column k of A' from the lower triangle of A0 and the panel
//         vectors (row k keeps its conjugate on the diagonal and x beyond it)
//         and partials of |x|^2;
//   hemv: reflector k from those partials (u = x except u_0 = x_0 - beta;
//         work-group 0 stores u_0, tau, e, d), then A0 u over the lower
//         triangle of the trailing block in strips of 64 x 64 tiles with
//         partials of u^H A0 u, and (in work-groups of their own) the panel
//         products W^H u and V^H u.
// After the panel, her2k applies its rank-2 kNb update to the lower tiles of
// the next trailing block, which is A0 of the next panel.  Only the lower
// triangle is read, so the trailing matrix is read (half of it) once per
// column and rewritten once per panel.
constexpr int kNb = 32;     // panel width; 2 kNb panel products fit 64 slots
constexpr int kHT = 64;     // hemv and her2k tile
constexpr int kStripMax = 8;   // tiles per hemv strip at most
// hemv work-groups resident at once: 2 per CU (256 threads, 2 waves per
// SIMD) on the 256 CUs of the chip
constexpr int kHemvResident = 512;
constexpr int kColTpe = 16;   // threads per element in the col kernel
constexpr int kColRows = 256 / kColTpe;  // elements per col work-group

struct TriWork {
  double2 *a;     // n x n work matrix (interleaved), row-major
  double *tau;    // n
  double *d;      // n   diagonal of T
  double2 *e;     // n   complex off-diagonal of T_c (e[k] = T_c[k+1][k])
  double2 *xs;    // n   x_0 of each step (before the reflector)
  double2 *wb;    // kNb x n: panel vectors W_i by global index
  double2 *prow;  // strips x 64: row partials of the hemv
  double2 *pcol;  // tile rows x ldp: column partials of the hemv
  double2 *pdot;  // tile rows x 64: partials of W^H u (slots < j), V^H u
  double *puau;   // strips: partials of u^H A0 u
  double *pnrm;   // col work-groups: partials of sum_{c > k+1} |x_c|^2
  long ldp;       // row length of pcol
};

// Strips before tile row I: row I has I + 1 tiles in I / sw + 1 strips.
__host__ __device__ inline long strip_prefix(int I, int sw) {
  const long q = I / sw, r = I - q * sw;
  return I + sw * q * (q - 1) / 2 + q * r;
}

// Tiles per hemv strip for a trailing block of nt tile rows: the shortest
// strips (most work-groups, shortest serial chains) for which the strips
// and the nt panel-product groups still fit one round of resident
// work-groups; a second round that holds only a few groups would double
// the step's time.
__host__ __device__ inline int strip_width(int nt) {
  for (int sw = 1; sw < kStripMax; ++sw)
    if (strip_prefix(nt, sw) + nt <= kHemvResident) return sw;
  return kStripMax;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}

// Step k, part col: kColRows elements c = k + kColRows b + e per
// work-group, kColTpe threads (q) per element sharing its sums.  With slot
// j > 0 it first finishes step k-1 (slot j-1, trailing offset k, size
// n - k) and stores W_{j-1}; unless finish_only it then forms x_c = A'[c][k].
__global__ __launch_bounds__(256) void hh_col_kernel(TriWork t, int n, int k,
                                                     int k0, int j,
                                                     int finish_only) {
  constexpr int kPer = kNb / kColTpe;         // panel slots per thread
  __shared__ double red[16];
  __shared__ double2 y[64], yq[4][64], part[kColTpe][kColRows], wsh[kColRows];
  __shared__ double2 vk[kNb], wk[kNb];
  __shared__ double kk[2];
  const int e = threadIdx.x % kColRows, q = threadIdx.x / kColRows;
  const int c = k + blockIdx.x * kColRows + e;
  const bool in = c < n;
  const int jp = j - 1;                       // slot of step k-1
  // sum of the kColTpe parts of element e (after a barrier)
  auto part_sum = [&](int ee) {
    double2 s0 = part[0][ee], s1 = part[1][ee];
#pragma unroll
    for (int g = 2; g < kColTpe; g += 2) {
      s0 = cadd(s0, part[g][ee]);
      s1 = cadd(s1, part[g + 1][ee]);
    }
    return cadd(s0, s1);
  };
  // every load that depends on nothing computed here is issued first
  double2 a_ck = make_double2(0.0, 0.0);
  if (!finish_only && in && q == 0) a_ck = t.a[(long)c * n + k];
  double2 vc[kPer], wc[kPer];                 // V_i[c], W_i[c], i = q + kColTpe s
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int i = q + kColTpe * s;
    vc[s] = make_double2(0.0, 0.0);
    wc[s] = make_double2(0.0, 0.0);
    if (in && i < j) vc[s] = t.a[(long)(k0 + i) * n + c];
    if (in && i < jp) wc[s] = t.wb[(long)i * n + c];
  }
  // V_l[k], W_l[k] for the panel slots l = lane of wave 0
  const int l64 = threadIdx.x & 63;
  const bool w0 = threadIdx.x < 64;
  double2 vke = make_double2(0.0, 0.0), wke = make_double2(0.0, 0.0);
  if (w0 && l64 < j) vke = t.a[(long)(k0 + l64) * n + k];
  if (w0 && l64 < jp) wke = t.wb[(long)l64 * n + k];
  double2 w_own = make_double2(0.0, 0.0);     // w_{j-1}[c]
  if (j > 0) {
    const int mp = n - k;
    const int ntp = (mp + kHT - 1) / kHT;
    const int swp = strip_width(ntp);
    const double taup = t.tau[k - 1];
    const double2 *up = t.a + (long)(k - 1) * n;   // u_{k-1} by global index
    double2 u_c = make_double2(0.0, 0.0), u_k = up[k];
    if (in && q == 0) u_c = up[c];
    // hemv sums of p[r], r = c - k, in kColTpe interleaved parts
    double2 ps = make_double2(0.0, 0.0), ps1 = ps;
    if (in) {
      const int r = c - k, I = r / kHT, rr = r - I * kHT;
      const long b0 = strip_prefix(I, swp), b1 = b0 + I / swp + 1;
      for (long b = b0 + q; b < b1; b += kColTpe) ps = cadd(ps, t.prow[b * kHT + rr]);
      int I2 = I + q;
      for (; I2 + kColTpe < ntp; I2 += 2 * kColTpe) {
        ps = cadd(ps, t.pcol[(long)I2 * t.ldp + r]);
        ps1 = cadd(ps1, t.pcol[(long)(I2 + kColTpe) * t.ldp + r]);
      }
      if (I2 < ntp) ps = cadd(ps, t.pcol[(long)I2 * t.ldp + r]);
      ps = cadd(ps, ps1);
    }
    // the same for r = 0 (w_{j-1}[k] is needed by every work-group)
    double2 p0 = make_double2(0.0, 0.0);
    if (w0) {
      if (l64 == 0) p0 = t.prow[0];
      for (int I2 = l64; I2 < ntp; I2 += 64) p0 = cadd(p0, t.pcol[(long)I2 * t.ldp]);
    }
    // panel products of step k-1, y[s] = W_s^H u, y[jp + s] = V_s^H u, in
    // four parts; the u^H A0 u partials
    const int slot = threadIdx.x & 63, g = threadIdx.x >> 6;
    double2 sy = make_double2(0.0, 0.0), sy1 = sy;
    if (slot < 2 * jp) {
      int I = g;
      for (; I + 4 < ntp; I += 8) {
        sy = cadd(sy, t.pdot[(long)I * 64 + slot]);
        sy1 = cadd(sy1, t.pdot[(long)(I + 4) * 64 + slot]);
      }
      if (I < ntp) sy = cadd(sy, t.pdot[(long)I * 64 + slot]);
    }
    double s0 = 0.0, s1 = 0.0;
    const long nsp = strip_prefix(ntp, swp);
    long bq = threadIdx.x;
    for (; bq + 256 < nsp; bq += 512) {
      s0 += t.puau[bq];
      s1 += t.puau[bq + 256];
    }
    if (bq < nsp) s0 += t.puau[bq];
    yq[g][slot] = cadd(sy, sy1);
    const double uau = block_sum(s0 + s1, red);   // syncs: yq[] is complete
    if (threadIdx.x < 64)
      y[slot] = cadd(cadd(yq[0][slot], yq[1][slot]), cadd(yq[2][slot], yq[3][slot]));
    __syncthreads();
    if (threadIdx.x == 0) {
      double corr = 0.0;
      for (int i = 0; i < jp; ++i)
        corr += y[jp + i].x * y[i].x + y[jp + i].y * y[i].y;
      kk[0] = 0.5 * taup * taup * (uau - 2.0 * corr);
    }
    // panel terms: p -= V_i (W_i^H u) + W_i (V_i^H u), i < jp
#pragma unroll
    for (int s2 = 0; s2 < kPer; ++s2) {
      const int i = q + kColTpe * s2;
      if (i < jp) {
        const double2 y1 = y[i], y2 = y[jp + i];
        const double2 v = vc[s2], w = wc[s2];
        ps.x -= v.x * y1.x - v.y * y1.y + w.x * y2.x - w.y * y2.y;
        ps.y -= v.x * y1.y + v.y * y1.x + w.x * y2.y + w.y * y2.x;
      }
    }
    if (w0) {
      if (l64 < jp) {
        const double2 y1 = y[l64], y2 = y[jp + l64];
        p0.x -= vke.x * y1.x - vke.y * y1.y + wke.x * y2.x - wke.y * y2.y;
        p0.y -= vke.x * y1.y + vke.y * y1.x + wke.x * y2.y + wke.y * y2.x;
      }
      p0.x = wave_sum(p0.x);
      p0.y = wave_sum(p0.y);
    }
    __syncthreads();                          // y[] reads are done
    part[q][e] = ps;
    __syncthreads();
    const double K = kk[0];
    if (q == 0) {
      const double2 tot = part_sum(e);
      if (in) {
        w_own = make_double2(taup * tot.x - K * u_c.x, taup * tot.y - K * u_c.y);
        t.wb[(long)jp * n + c] = w_own;
      }
      wsh[e] = w_own;
    }
    if (threadIdx.x == 0)
      wk[jp] = make_double2(taup * p0.x - K * u_k.x, taup * p0.y - K * u_k.y);
  }
  if (finish_only) return;
  if (w0 && l64 < j) {
    vk[l64] = vke;
    if (l64 < jp) wk[l64] = wke;
  }
  __syncthreads();
  double2 xs = make_double2(0.0, 0.0);
#pragma unroll
  for (int s2 = 0; s2 < kPer; ++s2) {
    const int i = q + kColTpe * s2;
    if (i < j) {
      const double2 wci = i == jp ? wsh[e] : wc[s2];
      const double2 a = cmulc(wk[i], vc[s2]);   // V_i[c] conj(W_i[k])
      const double2 b = cmulc(vk[i], wci);      // W_i[c] conj(V_i[k])
      xs.x += a.x + b.x;
      xs.y += a.y + b.y;
    }
  }
  __syncthreads();                            // part[] reads are done
  part[q][e] = xs;
  __syncthreads();
  double nrm = 0.0;
  if (q == 0 && in) {
    const double2 corr = part_sum(e);
    const double2 x = make_double2(a_ck.x - corr.x, a_ck.y - corr.y);
    if (c == k) {
      t.a[(long)k * n + k] = make_double2(x.x, -x.y);
    } else {
      t.a[(long)k * n + c] = x;
      if (c == k + 1) t.xs[k] = x;
      else nrm = x.x * x.x + x.y * x.y;
    }
  }
  const double tot = block_sum(nrm, red);
  if (threadIdx.x == 0) t.pnrm[blockIdx.x] = tot;
}

// Step k, part hemv: one work-group per strip of up to sw tiles of tile
// row I of the lower triangle of the trailing block (offset o = k + 1, size
// m).  Wave w takes rows 16 w .. 16 w + 15 of the tile row, lane l column l
// of each tile.  Row partials sum A0[r][c] u[c] over the strip; column
// partials sum conj(A0[r][c]) u[r] over the tile's rows (the upper triangle
// by Hermitian symmetry; strictly below the diagonal in diagonal tiles).
// The strip holding the diagonal tile also forms the panel products over its
// rows: slot s < j: conj(W_s) . u, slot j + s: conj(V_s) . u.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void hh_hemv_kernel(TriWork t, int n, int k,
                                                      int k0, int j) {
  __shared__ double red[16];
  __shared__ double2 cs[kStripMax][4][64];
  __shared__ double2 ur_s[kHT];
  const int o = k + 1, m = n - o;
  const int nt = (m + kHT - 1) / kHT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double2 zero = make_double2(0.0, 0.0);
  const long b = blockIdx.x;
  const int sw = strip_width(nt);
  const long nstr = strip_prefix(nt, sw);
  if (b >= nstr) {
    // panel products over rows I*64 .. I*64+63 (work-groups past the
    // strips, only for slot j > 0): 4 threads per product slot, slot s < j:
    // conj(W_s) . u, slot j + s: conj(V_s) . u
    const int I = (int)(b - nstr);
    const int slot = threadIdx.x >> 2, qt = threadIdx.x & 3;
    const int r0 = I * kHT + qt * 16;
    const double2 *u = t.a + (long)k * n + o;
    double2 xv[16], uv[16];
    const double2 *x = slot < j ? t.wb + (long)slot * n + o
                                : t.a + (long)(k0 + slot - j) * n + o;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int r = r0 + rr;
      xv[rr] = make_double2(0.0, 0.0);
      uv[rr] = make_double2(0.0, 0.0);
      if (slot < 2 * j && r < m) xv[rr] = x[r];
      if (r > 0 && r < m) uv[rr] = u[r];
    }
    const double2 x0 = t.xs[k];
    double s = 0.0;
    const int ncb = (m + 1 + kColRows - 1) / kColRows;
    for (int bb = threadIdx.x; bb < ncb; bb += 256) s += t.pnrm[bb];
    const double rest = block_sum(s, red);
    double2 u0 = x0;
    if (m > 1 && rest != 0.0) {
      const double ax0 = hypot(x0.x, x0.y);
      const double nrm = sqrt(rest + ax0 * ax0);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0)
                                   : make_double2(1.0, 0.0);
      u0 = make_double2(x0.x + ph.x * nrm, x0.y + ph.y * nrm);   // x0 - beta
    }
    if (r0 == 0) uv[0] = u0;
    double2 sd = zero;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const double2 qv = cmulc(xv[rr], uv[rr]);
      sd.x += qv.x;
      sd.y += qv.y;
    }
    sd.x += __shfl_xor(sd.x, 1);
    sd.y += __shfl_xor(sd.y, 1);
    sd.x += __shfl_xor(sd.x, 2);
    sd.y += __shfl_xor(sd.y, 2);
    if (qt == 0 && slot < 2 * j) t.pdot[(long)I * 64 + slot] = sd;
    return;
  }
  int lo = 0, hi = nt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (strip_prefix(mid, sw) <= b) lo = mid;
    else hi = mid - 1;
  }
  const int I = lo;
  const int J0 = (int)(b - strip_prefix(I, sw)) * sw;
  const int J1 = min(J0 + sw, I + 1);
  const double2 *u = t.a + (long)k * n + o;
  const double2 *blk = t.a + (long)o * n + o;
  const int rb = I * kHT + wave * 16;
  const int rbu = __builtin_amdgcn_readfirstlane(rb);
  // tile J of the strip: lane's column of the wave's 16 rows (the upper
  // triangle of a diagonal tile is not loaded)
  double2 v[16];
  auto load_tile = [&](int J) __attribute__((always_inline)) {
    const int cj = J * kHT + lane;
    const bool cok = cj < m, diag = J == I;
    const int cjc = cok ? cj : 0;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      // row base is wave-uniform, the lane adds its column
      const double2 *rowp = blk + (long)(rbu + rr) * n;
      const bool ld = cok && rbu + rr < m && (!diag || lane <= wave * 16 + rr);
      v[rr] = ld ? rowp[cjc] : make_double2(0.0, 0.0);
    }
  };
  // loads that need nothing from the reflector go first: u beyond u_0, the
  // first tile, x_0 and the norm partials
  const int rl = I * kHT + lane;
  double2 url = make_double2(0.0, 0.0);
  if (rl > 0 && rl < m) url = u[rl];
  load_tile(J0);
  const double2 x0 = t.xs[k];
  // reflector k: x = row k beyond the diagonal, |x|^2 from the col partials
  double s = 0.0;
  const int ncb = (m + 1 + kColRows - 1) / kColRows;
  for (int bb = threadIdx.x; bb < ncb; bb += 256) s += t.pnrm[bb];
  const double rest = block_sum(s, red);
  const double ax0 = hypot(x0.x, x0.y);
  double tau = 0.0;
  double2 beta = x0, u0 = x0;
  if (m > 1 && rest != 0.0) {
    const double nrm = sqrt(rest + ax0 * ax0);
    const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0)
                                 : make_double2(1.0, 0.0);
    beta = make_double2(-ph.x * nrm, -ph.y * nrm);
    tau = 1.0 / (nrm * (nrm + ax0));
    u0 = make_double2(x0.x - beta.x, x0.y - beta.y);
  }
  // u[0] lives in x0 until work-group 0 stores it, so it is never loaded
  auto uat = [&](int r) {
    double2 w = make_double2(0.0, 0.0);
    if (r > 0 && r < m) w = u[r];
    w.x = r == 0 ? u0.x : w.x;
    w.y = r == 0 ? u0.y : w.y;
    return w;
  };
  if (rl == 0) url = u0;
  ur_s[lane] = url;                           // same in every wave
  double2 acc[16];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) acc[rr] = zero;
  __syncthreads();
  const double2 *ur = ur_s + wave * 16;
#pragma unroll 1
  for (int J = J0; J < J1; ++J) {
    const int cj = J * kHT + lane;
    const bool diag = J == I;
    const double2 uc = uat(cj);
    if (J > J0) load_tile(J);
    double2 csum = zero;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      double2 vr = v[rr], vc = v[rr];
      if (diag && lane == wave * 16 + rr) {
        vr.y = 0.0;                           // real diagonal
        vc = zero;
      }
      acc[rr].x += vr.x * uc.x - vr.y * uc.y;
      acc[rr].y += vr.x * uc.y + vr.y * uc.x;
      const double2 qv = cmulc(vc, ur[rr]);
      csum.x += qv.x;
      csum.y += qv.y;
    }
    cs[J - J0][wave][lane] = csum;
  }
  // reduce the 16 row sums over the 64 lanes: halve the values per lane at
  // each exchange; lane l ends with row (l >> 2) & 15 over lanes l ^ {0..3}
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const bool hb = lane & 32;
    const double2 send = hb ? acc[h] : acc[h + 8];
    const double2 keep = hb ? acc[h + 8] : acc[h];
    acc[h] = make_double2(keep.x + __shfl_xor(send.x, 32), keep.y + __shfl_xor(send.y, 32));
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const bool hb = lane & 16;
    const double2 send = hb ? acc[h] : acc[h + 4];
    const double2 keep = hb ? acc[h + 4] : acc[h];
    acc[h] = make_double2(keep.x + __shfl_xor(send.x, 16), keep.y + __shfl_xor(send.y, 16));
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const bool hb = lane & 8;
    const double2 send = hb ? acc[h] : acc[h + 2];
    const double2 keep = hb ? acc[h + 2] : acc[h];
    acc[h] = make_double2(keep.x + __shfl_xor(send.x, 8), keep.y + __shfl_xor(send.y, 8));
  }
  {
    const bool hb = lane & 4;
    const double2 send = hb ? acc[0] : acc[1];
    const double2 keep = hb ? acc[1] : acc[0];
    acc[0] = make_double2(keep.x + __shfl_xor(send.x, 4), keep.y + __shfl_xor(send.y, 4));
  }
  acc[0].x += __shfl_xor(acc[0].x, 2);
  acc[0].y += __shfl_xor(acc[0].y, 2);
  acc[0].x += __shfl_xor(acc[0].x, 1);
  acc[0].y += __shfl_xor(acc[0].y, 1);
  double uau = 0.0;   // this group's share of u^H A0 u
  if ((lane & 3) == 0) {
    const int r = rb + (lane >> 2);
    t.prow[b * kHT + wave * 16 + (lane >> 2)] = acc[0];
    const double2 uv = uat(r);
    uau += uv.x * acc[0].x + uv.y * acc[0].y;
  }
  __syncthreads();
  for (int jt = wave; J0 + jt < J1; jt += 4) {
    const int J = J0 + jt, cj = J * kHT + lane;
    const double2 tot = cadd(cadd(cs[jt][0][lane], cs[jt][1][lane]),
                             cadd(cs[jt][2][lane], cs[jt][3][lane]));
    t.pcol[(long)I * t.ldp + cj] = tot;
    const double2 uv = uat(cj);
    uau += uv.x * tot.x + uv.y * tot.y;
  }
  const double ut = block_sum(uau, red);
  if (threadIdx.x == 0) {
    t.puau[b] = ut;
    if (b == 0) {
      t.tau[k] = tau;
      t.e[k] = beta;
      t.d[k] = t.a[(long)k * n + k].x;
      t.a[(long)k * n + o] = u0;
    }
  }
}

// End of a panel of nbp reflectors from k0: the lower 64 x 64 tiles of the
// trailing block at s0 = k0 + nbp (diagonal tiles whole) get
// A0 -= sum_i V_i W_i^H + W_i V_i^H.
__global__ __launch_bounds__(256) void hh_her2k_kernel(TriWork t, int n, int k0,
                                                       int nbp, int s0) {
  __shared__ double2 sv[4][8][kHT];   // V rows, W rows, V cols, W cols
  const int m = n - s0;
  const long b = blockIdx.x;
  int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((long)(I + 1) * (I + 2) / 2 <= b) ++I;
  while ((long)I * (I + 1) / 2 > b) --I;
  const int J = (int)(b - (long)I * (I + 1) / 2);
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < nbp; i0 += 8) {
    for (int e = threadIdx.x; e < 4 * 8 * kHT; e += 256) {
      const int arr = e >> 9, ii = (e >> 6) & 7, x = e & 63;
      const int i = i0 + ii;
      const int idx = (arr < 2 ? I : J) * kHT + x;
      double2 v = make_double2(0.0, 0.0);
      if (i < nbp && idx < m)
        v = (arr & 1) ? t.wb[(long)i * n + s0 + idx]
                      : t.a[(long)(k0 + i) * n + s0 + idx];
      sv[arr][ii][x] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      double2 vr[4], wr[4], vc[4], wc[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        vr[a] = sv[0][ii][tr + 16 * a];
        wr[a] = sv[1][ii][tr + 16 * a];
        vc[a] = sv[2][ii][tc + 16 * a];
        wc[a] = sv[3][ii][tc + 16 * a];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double2 p = cmulc(wc[c], vr[a]);   // V[r] conj(W[c])
          const double2 q = cmulc(vc[c], wr[a]);   // W[r] conj(V[c])
          acc[a][c].x += p.x + q.x;
          acc[a][c].y += p.y + q.y;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = I * kHT + tr + 16 * a;
    if (r >= m) continue;
    double2 *row = t.a + (long)(s0 + r) * n + s0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int cc = J * kHT + tc + 16 * c;
      if (cc < m) {
        double2 v = row[cc];
        v.x -= acc[a][c].x;
        v.y -= acc[a][c].y;
        row[cc] = v;
      }
    }
  }
}

__global__ void hh_last_kernel(TriWork t, int n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) t.d[n - 1] = t.a[(long)(n - 1) * n + n - 1].x;
}

// --------------------------------------------------- real tridiagonal T

struct TriReal {
  const double *d;   // n
  double *e;         // n-1, |e_k| (real symmetric off-diagonal)
  double2 *phase;    // n, D = diag(phase)
  double *bounds;    // [lo, hi, tnorm, pivmin]
};

__device__ __forceinline__ double2 unit_mul(double2 a, double2 b) {
  double2 p = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  const double nr = hypot(p.x, p.y);
  return make_double2(p.x / nr, p.y / nr);
}

// |e_k| and the phases phase_{k+1} = phase_k e_k / |e_k| (phase_0 = 1) by
// a prefix product over one work-group of kPhaseThreads threads: each
// thread takes a chunk of consecutive k, the chunk products are scanned in
// LDS, and each thread then walks its chunk from its prefix.  The same pass
// finds the Gershgorin bounds of T, its norm and the pivot minimum.
constexpr int kPhaseThreads = 1024;
__global__ __launch_bounds__(kPhaseThreads) void tri_phase_kernel(
    const double2 *__restrict__ ec, TriReal r, int n) {
  __shared__ double2 sc[kPhaseThreads];
  __shared__ double red[4][kPhaseThreads / 64];
  const int tid = threadIdx.x;
  const int per = (n + kPhaseThreads - 1) / kPhaseThreads;
  const int k0 = min(n, tid * per), k1 = min(n, k0 + per);
  auto unit = [&](int k) {
    const double2 c = ec[k];
    const double ek = hypot(c.x, c.y);
    return ek > 0.0 ? make_double2(c.x / ek, c.y / ek) : make_double2(1.0, 0.0);
  };
  // chunk product of q_k, k in [k0, k1) below n - 1
  double2 loc = make_double2(1.0, 0.0);
  for (int k = k0; k < k1 && k < n - 1; ++k) loc = unit_mul(loc, unit(k));
  sc[tid] = loc;
  __syncthreads();
  for (int off = 1; off < kPhaseThreads; off <<= 1) {
    const double2 v = tid >= off ? unit_mul(sc[tid - off], sc[tid]) : sc[tid];
    __syncthreads();
    sc[tid] = v;
    __syncthreads();
  }
  // phase_k0 = product of the chunks before this one
  double2 ph = tid > 0 ? sc[tid - 1] : make_double2(1.0, 0.0);
  if (tid == 0) r.phase[0] = make_double2(1.0, 0.0);
  double lo = INFINITY, hi = -INFINITY, emax2 = 0.0, tn = 0.0;
  for (int k = k0; k < k1; ++k) {
    double ek = 0.0, ekp = 0.0;
    if (k < n - 1) {
      const double2 c = ec[k];
      ek = hypot(c.x, c.y);
      r.e[k] = ek;
      ph = unit_mul(ph, unit(k));
      r.phase[k + 1] = ph;
      emax2 = fmax(emax2, ek * ek);
    }
    if (k > 0) {
      const double2 c = ec[k - 1];
      ekp = hypot(c.x, c.y);
    }
    const double rad = ekp + ek, dk = r.d[k];
    lo = fmin(lo, dk - rad);
    hi = fmax(hi, dk + rad);
    tn = fmax(tn, fabs(dk) + rad);
  }
  // reductions: min lo, max hi, max tn, max emax2
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    tn = fmax(tn, __shfl_xor(tn, o));
    emax2 = fmax(emax2, __shfl_xor(emax2, o));
  }
  const int w = tid >> 6;
  if ((tid & 63) == 0) {
    red[0][w] = lo;
    red[1][w] = hi;
    red[2][w] = tn;
    red[3][w] = emax2;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < kPhaseThreads / 64; ++i) {
      lo = fmin(lo, red[0][i]);
      hi = fmax(hi, red[1][i]);
      tn = fmax(tn, red[2][i]);
      emax2 = fmax(emax2, red[3][i]);
    }
    const double span = fmax(hi - lo, tn) * 2.0 * DBL_EPSILON + DBL_MIN;
    r.bounds[0] = lo - span;
    r.bounds[1] = hi + span;
    r.bounds[2] = tn;
    r.bounds[3] = fmax(DBL_MIN, DBL_MIN * emax2);
  }
}

// number of eigenvalues of T below sigma
__device__ int sturm_count(const double *d, const double *e, int n,
                           double sigma, double pivmin) {
  double q = d[0] - sigma;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - sigma - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Multisection: one wave per eigenvalue.  Each round evaluates the Sturm
// count at the 63 interior points of 64 equal parts of [lo, hi], one per
// lane, and keeps the part holding eigenvalue i (the count at its left end
// is <= i, at its right end > i); a round narrows the bracket 64-fold
// instead of 2-fold.  lo and hi stay uniform across the wave.
__global__ __launch_bounds__(64) void multisect_kernel(TriReal r, int n,
                                                       int n_eig,
                                                       double *__restrict__ lam) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n_eig) return;
  double lo = r.bounds[0], hi = r.bounds[1];
  const double pivmin = r.bounds[3];
  for (int round = 0; round < 32; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    const double h = (hi - lo) * (1.0 / 64.0);
    const double x = lane < 63 ? lo + h * (lane + 1) : hi;
    const bool above =
        lane == 63 || (x > lo && sturm_count(r.d, r.e, n, x, pivmin) > i);
    const unsigned long long mask = __ballot(above);
    const int first = __ffsll((long long)mask) - 1;   // lane 63 is always set
    const double nlo = first == 0 ? lo : fmin(lo + h * first, hi);
    const double nhi = first == 63 ? hi : fmin(lo + h * (first + 1), hi);
    if (nlo == lo && nhi == hi) break;   // no representable progress
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// ------------------------------------------------------ inverse iteration

struct InvIt {
  const double *d;
  const double *e;
  const double *lam;
  const double *bounds;
  double *z;         // n x ldz (row-major, column j = eigenvector j)
  int ldz;
  double *u0, *u1, *u2, *ml;   // n x ldz each
  unsigned char *pv;           // n x ldz
  double gtol_rel;             // grouping tolerance relative to |T|
};

__device__ __forceinline__ double start_value(int row, int col) {
  unsigned x = (unsigned)row * 2654435761u ^ ((unsigned)col * 2246822519u + 0x9e3779b9u);
  x ^= x >> 15; x *= 2246822519u; x ^= x >> 13; x *= 3266489917u; x ^= x >> 16;
  return (double)(x & 0xFFFFFF) / 8388608.0 - 1.0;  // (-1, 1)
}

// LU of T - lam I with partial pivoting (rows i and i+1 swap when the
// subdiagonal entry is larger); U has bandwidth 2.
__device__ void tri_lu(const InvIt &q, int n, int col, double lam, double tiny) {
  const long ld = q.ldz;
  double r0 = q.d[0] - lam, r1 = n > 1 ? q.e[0] : 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double b = q.e[i];
    const double dn = q.d[i + 1] - lam;
    const double en = (i + 1 < n - 1) ? q.e[i + 1] : 0.0;
    const long o = (long)i * ld + col;
    if (fabs(r0) >= fabs(b)) {
      if (r0 == 0.0) r0 = tiny;
      const double mlt = b / r0;
      q.u0[o] = r0; q.u1[o] = r1; q.u2[o] = 0.0; q.ml[o] = mlt; q.pv[o] = 0;
      r0 = dn - mlt * r1;
      r1 = en;
    } else {
      const double mlt = r0 / b;
      q.u0[o] = b; q.u1[o] = dn; q.u2[o] = en; q.ml[o] = mlt; q.pv[o] = 1;
      r0 = r1 - mlt * dn;
      r1 = -mlt * en;
    }
  }
  if (r0 == 0.0) r0 = tiny;
  const long o = (long)(n - 1) * ld + col;
  q.u0[o] = r0; q.u1[o] = 0.0; q.u2[o] = 0.0; q.ml[o] = 0.0; q.pv[o] = 0;
}

// x <- (T - lam I)^-1 (f x) (x is column col of z); returns ||x|| of the
// result, accumulated during the back substitution with a running scale
// (no overflow for any finite vector).  Both substitutions run in chunks of
// kSolveChunk rows whose coefficients and right-hand sides are loaded before
// the dependent recurrence, so the loads of a chunk overlap instead of each
// waiting behind the previous step.
constexpr int kSolveChunk = 16;
__device__ double tri_solve(const InvIt &q, int n, int col, double f) {
  const long ld = q.ldz;
  double *x = q.z + col;
  const double *ml = q.ml + col, *u0 = q.u0 + col, *u1 = q.u1 + col,
               *u2 = q.u2 + col;
  const unsigned char *pv = q.pv + col;
  // forward: step i pivots rows i, i+1; a carries the updated x[i]
  double a = f * x[0];
  int i = 0;
  for (; i + kSolveChunk < n; i += kSolveChunk) {
    double b[kSolveChunk], m[kSolveChunk];
    unsigned char p[kSolveChunk];
#pragma unroll
    for (int u = 0; u < kSolveChunk; ++u) {
      b[u] = x[(long)(i + 1 + u) * ld];
      m[u] = ml[(long)(i + u) * ld];
      p[u] = pv[(long)(i + u) * ld];
    }
#pragma unroll
    for (int u = 0; u < kSolveChunk; ++u) {
      double aa = a, bb = f * b[u];
      if (p[u]) { const double t = aa; aa = bb; bb = t; }
      x[(long)(i + u) * ld] = aa;
      a = bb - m[u] * aa;
    }
  }
  for (; i < n - 1; ++i) {
    const long o = (long)i * ld;
    double aa = a, bb = f * x[o + ld];
    if (pv[o]) { const double t = aa; aa = bb; bb = t; }
    x[o] = aa;
    a = bb - ml[o] * aa;
  }
  x[(long)(n - 1) * ld] = a;
  // backward: v_i = (x_i - u1_i v_{i+1} - u2_i v_{i+2}) / u0_i, with
  // ||v||^2 = scale^2 ssq
  double xp1 = 0.0, xp2 = 0.0, scale = 0.0, ssq = 1.0;
  auto acc = [&](double v) {
    const double av = fabs(v);
    if (av > scale) {
      const double r = scale / av;
      ssq = 1.0 + ssq * r * r;
      scale = av;
    } else if (av > 0.0) {
      const double r = av / scale;
      ssq += r * r;
    }
  };
  i = n - 1;
  for (; i + 1 >= kSolveChunk; i -= kSolveChunk) {
    double xv[kSolveChunk], c0[kSolveChunk], c1[kSolveChunk], c2[kSolveChunk];
#pragma unroll
    for (int u = 0; u < kSolveChunk; ++u) {
      const long o = (long)(i - u) * ld;
      xv[u] = x[o];
      c0[u] = u0[o];
      c1[u] = u1[o];
      c2[u] = u2[o];
    }
#pragma unroll
    for (int u = 0; u < kSolveChunk; ++u) {
      const double v = (xv[u] - c1[u] * xp1 - c2[u] * xp2) / c0[u];
      x[(long)(i - u) * ld] = v;
      acc(v);
      xp2 = xp1;
      xp1 = v;
    }
  }
  for (; i >= 0; --i) {
    const long o = (long)i * ld;
    const double v = (x[o] - u1[o] * xp1 - u2[o] * xp2) / u0[o];
    x[o] = v;
    acc(v);
    xp2 = xp1;
    xp1 = v;
  }
  return scale * sqrt(ssq);
}

__device__ void scale_col(const InvIt &q, int n, int col, double f) {
  const long ld = q.ldz;
  for (int i = 0; i < n; ++i) q.z[i * ld + col] *= f;
}

__global__ __launch_bounds__(64) void inverse_iteration_kernel(InvIt q, int n, int n_eig) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_eig) return;
  const double tn = q.bounds[2];
  const double gtol = q.gtol_rel * tn;
  // a group starts where the gap to the previous eigenvalue exceeds gtol
  if (j > 0 && q.lam[j] - q.lam[j - 1] <= gtol) return;
  int j1 = j + 1;
  while (j1 < n_eig && q.lam[j1] - q.lam[j1 - 1] <= gtol) ++j1;
  const double tiny = DBL_EPSILON * fmax(tn, DBL_MIN);
  const long ld = q.ldz;
  for (int c = j; c < j1; ++c) {
    // separate exactly equal shifts inside a group by a few ulps of |T|
    const double lam = q.lam[c] + (c - j) * 8.0 * tiny;
    tri_lu(q, n, c, lam, tiny);
    for (int i = 0; i < n; ++i) q.z[i * ld + c] = start_value(i, c);
    // the normalisation of each iterate is folded into the next solve's
    // right-hand side (the solve is linear); a group member is normalised
    // and orthogonalised explicitly against the earlier members
    double f = 1.0;
    for (int it = 0; it < 4; ++it) {
      const double nrm = tri_solve(q, n, c, f);
      f = nrm > 0.0 ? 1.0 / nrm : 1.0;
      if (c > j) {
        scale_col(q, n, c, f);
        for (int o = j; o < c; ++o) {
          double dot = 0.0;
          for (int i = 0; i < n; ++i) dot += q.z[i * ld + o] * q.z[i * ld + c];
          for (int i = 0; i < n; ++i) q.z[i * ld + c] -= dot * q.z[i * ld + o];
        }
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += q.z[i * ld + c] * q.z[i * ld + c];
        f = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
      }
    }
    scale_col(q, n, c, f);
  }
}

// ------------------------------------------------------ back-transform

// C[row][col] = phase[row] z[row][col], planar rows (re at 0, im at +ld_e).
__global__ void phase_apply_kernel(const double *__restrict__ z, int ldz,
                                   const double2 *__restrict__ phase, int n,
                                   int n_eig, double *__restrict__ c, int ld_e,
                                   int rows_pad) {
  const long total = (long)rows_pad * ld_e;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int row = (int)(idx / ld_e), col = (int)(idx % ld_e);
    double re = 0.0, im = 0.0;
    if (row < n && col < n_eig) {
      const double v = z[(long)row * ldz + col];
      const double2 ph = phase[row];
      re = ph.x * v;
      im = ph.y * v;
    }
    c[(long)row * 2 * ld_e + col] = re;
    c[(long)row * 2 * ld_e + ld_e + col] = im;
  }
}

// Blocked back-transformation.  Reflectors k0 .. k0+nb-1 are combined as
// H_k0 H_k0+1 ... H_k0+nb-1 = I - V T V^H with T upper triangular:
// T_jj = tau_j, T_{0:j,j} = -tau_j T_{0:j,0:j} (V_{:,0:j}^H v_j).  Column j of
// V is reflector k0+j: zero in rows <= k0+j, u (stored in row k0+j of the
// work matrix) below.  Blocks are applied last block first, since
// Q = Q_0 Q_1 ... Q_last acts on C from the left.
constexpr int kWy = 32;   // reflectors per block

__device__ __forceinline__ double2 vref(const double2 *a, int n, int k, int r) {
  return r > k ? a[(long)k * n + r] : make_double2(0.0, 0.0);
}

// One block per reflector block: S = V^H V (strict upper part), then T.
__global__ __launch_bounds__(256) void wy_t_kernel(const double2 *__restrict__ a,
                                                   const double *__restrict__ tau,
                                                   int n, double2 *__restrict__ t_all) {
  __shared__ double2 vs[64][kWy + 1];
  __shared__ double2 S[kWy][kWy + 1];
  __shared__ double2 T[kWy][kWy + 1];
  const int b = blockIdx.x;
  const int k0 = b * kWy;
  const int nb = min(kWy, (n - 1) - k0);
  // each thread owns up to 2 (i < j) pairs of the 32 x 32 strict upper part
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  int pi[2], pj[2];
  for (int q = 0; q < 2; ++q) {
    const int id = threadIdx.x + q * 256;   // 0..511 covers 496 pairs
    // decode (i, j) by rows of the upper triangle: row i has kWy - 1 - i pairs
    int ii = 0, rem = id;
    while (ii < kWy - 1 && rem >= kWy - 1 - ii) { rem -= kWy - 1 - ii; ++ii; }
    pi[q] = ii;
    pj[q] = ii + 1 + rem;
  }
  for (int r0 = k0 + 1; r0 < n; r0 += 64) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * kWy; idx += 256) {
      const int j = idx / 64, rr = idx % 64;
      const int r = r0 + rr;
      vs[rr][j] = (j < nb && r < n) ? vref(a, n, k0 + j, r) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      if (pi[q] >= kWy - 1 || pj[q] >= kWy) continue;
      for (int rr = 0; rr < 64; ++rr) {
        const double2 x = vs[rr][pi[q]], y = vs[rr][pj[q]];
        acc[q].x += x.x * y.x + x.y * y.y;   // conj(x) y
        acc[q].y += x.x * y.y - x.y * y.x;
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < 2; ++q)
    if (pi[q] < kWy - 1 && pj[q] < kWy) S[pi[q]][pj[q]] = acc[q];
  for (int idx = threadIdx.x; idx < kWy * kWy; idx += 256)
    T[idx / kWy][idx % kWy] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = tau[k0 + j];
    double2 val = make_double2(0.0, 0.0);
    const int i = threadIdx.x;
    if (i < j) {
      // -tau_j sum_{l=i}^{j-1} T[i][l] S[l][j]
      for (int l = i; l < j; ++l) {
        const double2 tl = T[i][l], sl = S[l][j];
        val.x += tl.x * sl.x - tl.y * sl.y;
        val.y += tl.x * sl.y + tl.y * sl.x;
      }
      val.x *= -tj;
      val.y *= -tj;
    }
    __syncthreads();
    if (i < j) T[i][j] = val;
    if (i == j) T[j][j] = make_double2(tj, 0.0);
    __syncthreads();
  }
  double2 *out = t_all + (long)b * kWy * kWy;
  for (int idx = threadIdx.x; idx < kWy * kWy; idx += 256)
    out[idx] = T[idx / kWy][idx % kWy];
}

// Partial W1 = V^H C over a chunk of rows: part[chunk][j][e].  Chunks hold
// chunk_rows rows (a multiple of kWySub).  The
// reflectors of the block are staged in LDS kWySub rows at a time (zero
// outside their support), so the row loop reads them as broadcasts and only
// the C loads go to memory.
constexpr int kWySub = 64;
constexpr int kWyRows = 64;   // rows per chunk (one partial per chunk)
__global__ __launch_bounds__(256) void wy_vhc_kernel(const double2 *__restrict__ a,
                                                     int n, int k0, int nb,
                                                     int chunk_rows,
                                                     const double *__restrict__ c,
                                                     int ld_e, int n_eig,
                                                     double2 *__restrict__ part) {
  __shared__ double2 vs[kWySub][kWy];
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  const int jg = threadIdx.x >> 6;           // 0..3, 8 reflectors each
  const int chunk = blockIdx.y;
  const int r0 = k0 + 1 + chunk * chunk_rows;
  const int r1 = min(n, r0 + chunk_rows);
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int s0 = r0; s0 < r1; s0 += kWySub) {
    const int m = min(kWySub, r1 - s0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < kWySub * kWy; idx += blockDim.x) {
      const int rr = idx % kWySub, j = idx / kWySub;
      vs[rr][j] = (j < nb && rr < m) ? vref(a, n, k0 + j, s0 + rr)
                                     : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (e < n_eig) {
      const double *cr_p = c + (long)s0 * 2 * ld_e + e;
#pragma unroll 4
      for (int rr = 0; rr < m; ++rr) {
        const double cr = cr_p[(long)rr * 2 * ld_e];
        const double ci = cr_p[(long)rr * 2 * ld_e + ld_e];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double2 v = vs[rr][jg * 8 + q];
          acc[q].x += v.x * cr + v.y * ci;   // conj(v) c
          acc[q].y += v.x * ci - v.y * cr;
        }
      }
    }
  }
  double2 *p = part + (long)chunk * kWy * ld_e;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (e < ld_e) p[(long)(jg * 8 + q) * ld_e + e] = acc[q];
}

// W2 = T (sum over chunks of the partials): w2[j][e].  A block takes
// kTwCols columns e; thread (e, j, h) sums the partials of reflector j over
// the chunks ch = h mod 2, the two halves meet in LDS, then thread (e, j)
// forms row j of T W1.
constexpr int kTwCols = 4;
__global__ __launch_bounds__(256) void wy_tw_kernel(const double2 *__restrict__ part,
                                                    int n_chunks,
                                                    const double2 *__restrict__ t,
                                                    int nb, int ld_e, int n_eig,
                                                    double2 *__restrict__ w2) {
  __shared__ double2 w1[2][kWy][kTwCols];
  const int el = threadIdx.x % kTwCols;
  const int j = (threadIdx.x / kTwCols) % kWy;
  const int h = threadIdx.x / (kTwCols * kWy);   // 0, 1
  const int e = blockIdx.x * kTwCols + el;
  double2 sa = make_double2(0.0, 0.0), sb = sa;
  if (e < n_eig) {
    int ch = h;
    for (; ch + 2 < n_chunks; ch += 4) {
      const double2 v = part[((long)ch * kWy + j) * ld_e + e];
      const double2 u = part[((long)(ch + 2) * kWy + j) * ld_e + e];
      sa.x += v.x;
      sa.y += v.y;
      sb.x += u.x;
      sb.y += u.y;
    }
    if (ch < n_chunks) {
      const double2 v = part[((long)ch * kWy + j) * ld_e + e];
      sa.x += v.x;
      sa.y += v.y;
    }
  }
  w1[h][j][el] = make_double2(sa.x + sb.x, sa.y + sb.y);
  __syncthreads();
  if (h == 0) {
    double2 s = make_double2(0.0, 0.0);
    if (j < nb)
      for (int l = j; l < nb; ++l) {
        const double2 tv = t[j * kWy + l];
        const double2 x = make_double2(w1[0][l][el].x + w1[1][l][el].x,
                                       w1[0][l][el].y + w1[1][l][el].y);
        s.x += tv.x * x.x - tv.y * x.y;
        s.y += tv.x * x.y + tv.y * x.x;
      }
    if (e < ld_e) w2[(long)j * ld_e + e] = s;
  }
}

// C[r][e] -= sum_j v_j[r] W2[j][e] for rows r > k0.
__global__ __launch_bounds__(256) void wy_update_kernel(const double2 *__restrict__ a,
                                                        int n, int k0, int nb,
                                                        const double2 *__restrict__ w2,
                                                        double *__restrict__ c,
                                                        int ld_e, int n_eig) {
  __shared__ double2 vs[4][kWy];
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rl = threadIdx.x >> 6;
  const int r = k0 + 1 + blockIdx.y * 4 + rl;
  if (threadIdx.x < 4 * kWy) {
    const int rr = threadIdx.x / kWy, j = threadIdx.x % kWy;
    const int row = k0 + 1 + blockIdx.y * 4 + rr;
    vs[rr][j] = (j < nb && row < n) ? vref(a, n, k0 + j, row) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (r >= n || e >= n_eig) return;
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < nb; ++j) {
    const double2 v = vs[rl][j], w = w2[(long)j * ld_e + e];
    sr += v.x * w.x - v.y * w.y;
    si += v.x * w.y + v.y * w.x;
  }
  c[(long)r * 2 * ld_e + e] -= sr;
  c[(long)r * 2 * ld_e + ld_e + e] -= si;
}

// B = 1.5 I - 0.5 G  (G interleaved n_eig x n_eig) into planar ld_e x ld_e
__global__ void newton_schulz_coeff_kernel(const double *__restrict__ g,
                                           int n_eig, int ld_e,
                                           double *__restrict__ b) {
  const long total = (long)ld_e * ld_e;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int r = (int)(idx / ld_e), cc = (int)(idx % ld_e);
    double re = 0.0, im = 0.0;
    if (r < n_eig && cc < n_eig) {
      re = -0.5 * g[2L * ((long)r * n_eig + cc)];
      im = -0.5 * g[2L * ((long)r * n_eig + cc) + 1];
      if (r == cc) re += 1.5;
    }
    b[(long)r * 2 * ld_e + cc] = re;
    b[(long)r * 2 * ld_e + ld_e + cc] = im;
  }
}

// Layout of the Householder work buffer: panel vectors W, hemv row,
// column and product partials, u^H A0 u and norm partials.
struct HhSizes {
  int nt_max;
  long strips_max, ldp;
  size_t n_wb, n_prow, n_pcol, n_pdot, n_dbl;
  size_t bytes() const {
    return sizeof(double2) * (n_wb + n_prow + n_pcol + n_pdot) +
           sizeof(double) * n_dbl + 64;
  }
};

HhSizes hh_sizes(int n) {
  HhSizes z;
  z.nt_max = std::max(1, (n - 1 + kHT - 1) / kHT);
  z.strips_max = 0;   // the most strips of any step
  for (int nt = 1; nt <= z.nt_max; ++nt)
    z.strips_max = std::max(z.strips_max, strip_prefix(nt, strip_width(nt)));
  z.ldp = (long)z.nt_max * kHT;
  z.n_wb = (size_t)kNb * n;
  z.n_prow = (size_t)z.strips_max * kHT;
  z.n_pcol = (size_t)z.nt_max * z.ldp;
  z.n_pdot = (size_t)z.nt_max * 64;
  z.n_dbl = (size_t)z.strips_max + (n + kColRows - 1) / kColRows;
  return z;
}

}  // namespace

size_t eig_workspace_bytes(int n) { return hh_sizes(n).bytes(); }

void eig_lowest(Context *ctx, const double *a_in, int n, int n_eig,
                double *eigval, double *basis, int ld_e, int *flag,
                hipStream_t s) {
  (void)flag;
  SSRPA_REQUIRE(n >= 1 && n_eig >= 1 && n_eig <= n, SSRPA_ERR_ARG,
                "eig: bad sizes n=%d n_eig=%d", n, n_eig);
  const int rows_pad = round_up(n, 64);
  DevBuf wa(ctx, sizeof(double2) * (size_t)n * n);
  DevBuf vecs(ctx, sizeof(double) * 2 * (size_t)n + sizeof(double2) * 4 * (size_t)n + 64);
  copy_interleaved(a_in, wa.as<double>(), (size_t)n * n, s);
  TriWork t;
  t.a = wa.as<double2>();
  double *base = vecs.as<double>();
  t.tau = base;
  t.d = base + n;
  t.e = reinterpret_cast<double2 *>(base + 2 * n);
  t.xs = t.e + n;
  double2 *phase = t.xs + n;
  // panel vectors and hemv partials, sized for the first step (m = n - 1)
  const HhSizes hz = hh_sizes(n);
  t.ldp = hz.ldp;
  DevBuf hw(ctx, hz.bytes());
  t.wb = hw.as<double2>();
  t.prow = t.wb + hz.n_wb;
  t.pcol = t.prow + hz.n_prow;
  t.pdot = t.pcol + hz.n_pcol;
  t.puau = reinterpret_cast<double *>(t.pdot + hz.n_pdot);
  t.pnrm = t.puau + hz.strips_max;
  for (int k0 = 0; k0 < n; k0 += kNb) {
    const int kend = std::min(k0 + kNb, n);
    for (int k = k0; k < kend; ++k) {
      const int j = k - k0, m = n - k - 1;
      hipLaunchKernelGGL(hh_col_kernel, dim3((m + 1 + kColRows - 1) / kColRows),
                         dim3(256), 0, s, t, n, k, k0, j, 0);
      if (m == 0) break;
      const int nt = (m + kHT - 1) / kHT;
      // strips, then (slot j > 0) one work-group per tile row for the
      // panel products
      hipLaunchKernelGGL(hh_hemv_kernel,
                         dim3((unsigned)(strip_prefix(nt, strip_width(nt)) +
                                         (j > 0 ? nt : 0))),
                         dim3(256), 0, s, t, n, k, k0, j);
    }
    if (kend < n) {
      // finish w of the panel's last step, then update the next trailing block
      hipLaunchKernelGGL(hh_col_kernel, dim3((n - kend + kColRows - 1) / kColRows),
                         dim3(256), 0, s, t, n, kend, k0, kend - k0, 1);
      const long nt = (n - kend + kHT - 1) / kHT;
      hipLaunchKernelGGL(hh_her2k_kernel, dim3((unsigned)(nt * (nt + 1) / 2)),
                         dim3(256), 0, s, t, n, k0, kend - k0, kend);
    }
  }
  hipLaunchKernelGGL(hh_last_kernel, dim3(1), dim3(64), 0, s, t, n);
  SSRPA_HIP(hipGetLastError());

  DevBuf rw(ctx, sizeof(double) * ((size_t)n + 8));
  TriReal r;
  r.d = t.d;
  r.e = rw.as<double>();
  r.phase = phase;
  r.bounds = rw.as<double>() + n;
  hipLaunchKernelGGL(tri_phase_kernel, dim3(1), dim3(kPhaseThreads), 0, s,
                     (const double2 *)t.e, r, n);
  hipLaunchKernelGGL(multisect_kernel, dim3(n_eig), dim3(64), 0, s, r, n,
                     n_eig, eigval);
  SSRPA_HIP(hipGetLastError());

  // inverse iteration workspace: z, u0, u1, u2, ml (doubles) + pivots
  const int ldz = n_eig;
  const size_t nz = (size_t)n * ldz;
  DevBuf iw(ctx, sizeof(double) * 5 * nz + nz + 64);
  InvIt q;
  q.d = t.d;
  q.e = r.e;
  q.lam = eigval;
  q.bounds = r.bounds;
  q.z = iw.as<double>();
  q.ldz = ldz;
  q.u0 = q.z + nz;
  q.u1 = q.u0 + nz;
  q.u2 = q.u1 + nz;
  q.ml = q.u2 + nz;
  q.pv = reinterpret_cast<unsigned char *>(q.ml + nz);
  // eigenvalues closer than 1e-7 |T| form one group (orthogonalized inside)
  q.gtol_rel = 1e-7;
  hipLaunchKernelGGL(inverse_iteration_kernel, dim3((n_eig + 63) / 64), dim3(64),
                     0, s, q, n, n_eig);
  SSRPA_HIP(hipGetLastError());

  const long tot = (long)rows_pad * ld_e;
  hipLaunchKernelGGL(phase_apply_kernel,
                     dim3((unsigned)std::min<long>((tot + 255) / 256, 65536)),
                     dim3(256), 0, s, q.z, ldz, (const double2 *)phase, n, n_eig,
                     basis, ld_e, rows_pad);
  if (n > 1) {
    const int nblk = (n - 1 + kWy - 1) / kWy;
    const int max_chunks = (n + kWyRows - 1) / kWyRows;
    DevBuf tw(ctx, sizeof(double2) * (size_t)nblk * kWy * kWy);
    DevBuf part(ctx, sizeof(double2) * (size_t)max_chunks * kWy * ld_e);
    DevBuf w2(ctx, sizeof(double2) * (size_t)kWy * ld_e);
    hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s,
                       (const double2 *)t.a, t.tau, n, tw.as<double2>());
    const int ctiles = ld_e / 64;
    for (int b = nblk - 1; b >= 0; --b) {
      const int k0 = b * kWy;
      const int nb = std::min(kWy, (n - 1) - k0);
      const int rows = n - k0 - 1;
      const int chunk_rows = kWyRows;
      const int chunks = (rows + chunk_rows - 1) / chunk_rows;
      hipLaunchKernelGGL(wy_vhc_kernel, dim3(ctiles, chunks), dim3(256), 0, s,
                         (const double2 *)t.a, n, k0, nb, chunk_rows,
                         (const double *)basis, ld_e, n_eig, part.as<double2>());
      hipLaunchKernelGGL(wy_tw_kernel, dim3((ld_e + kTwCols - 1) / kTwCols),
                         dim3(256), 0, s,
                         (const double2 *)part.as<double2>(), chunks,
                         (const double2 *)tw.as<double2>() + (long)b * kWy * kWy,
                         nb, ld_e, n_eig, w2.as<double2>());
      hipLaunchKernelGGL(wy_update_kernel, dim3(ctiles, (rows + 3) / 4), dim3(256),
                         0, s, (const double2 *)t.a, n, k0, nb,
                         (const double2 *)w2.as<double2>(), basis, ld_e, n_eig);
    }
    SSRPA_HIP(hipGetLastError());
    SSRPA_HIP(hipStreamSynchronize(s));
  }

  // Newton-Schulz: C <- C (1.5 I - 0.5 C^H C)
  DevBuf gram(ctx, sizeof(double2) * (size_t)n_eig * n_eig);
  DevBuf coef(ctx, sizeof(double) * 2 * (size_t)ld_e * ld_e);
  DevBuf cnew(ctx, sizeof(double) * 2 * (size_t)rows_pad * ld_e);
  DevBuf ws;
  HerkArgs h{};
  h.a = basis;
  h.lda = 2L * ld_e;
  h.im_off = ld_e;
  h.ncol = n_eig;
  h.ld = ld_e;
  h.k = n;
  h.n_omega = 1;
  h.unit_weight = 1;
  herk(ctx, h, SSRPA_FP64, gram.as<double>(), 0, 0, ws, s);
  const long tc = (long)ld_e * ld_e;
  hipLaunchKernelGGL(newton_schulz_coeff_kernel,
                     dim3((unsigned)std::min<long>((tc + 255) / 256, 65536)),
                     dim3(256), 0, s, gram.as<double>(), n_eig, ld_e,
                     coef.as<double>());
  GemmArgs g{};
  g.a = basis; g.lda = 2L * ld_e; g.a_im = ld_e;
  g.b = coef.as<double>(); g.ldb = 2L * ld_e; g.b_im = ld_e;
  g.c = cnew.as<double>(); g.ldc = 2L * ld_e; g.c_im = ld_e;
  g.m = rows_pad; g.n = ld_e; g.k = ld_e;
  g.alpha = 1.0; g.beta = 0.0;
  DevBuf gws;
  gemm(ctx, g, SSRPA_FP64, gws, s);
  SSRPA_HIP(hipMemcpyAsync(basis, cnew.as(), sizeof(double) * 2 * (size_t)rows_pad * ld_e,
                           hipMemcpyDeviceToDevice, s));
  SSRPA_HIP(hipStreamSynchronize(s));  // work buffers are freed on return
}

}  // namespace ssrpa
