// Host runtime and C ABI of the ssrpa library.
//
// The driver follows the valence-block algorithm of the paper
// (Implementation section, Eqs. 14-15): the pair matrix is produced one block
// of valence bands at a time and its contribution to chi0 accumulated, so the
// memory floor is the resident real-space orbitals; the block loop runs twice
// (static chi0 first, then every frequency in the subspace), and when one
// block covers all valence bands its pair matrix is kept so the pair FFTs run
// only once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <chrono>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <tuple>

#include "internal.hpp"

namespace ssrpa {

void fail(ssrpa_status code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

// Allocation granularity: sizes are rounded up so that cached blocks are
// reusable across slightly different requests.
static size_t round_alloc(size_t bytes) {
  const size_t g = bytes >= (64u << 20) ? (8u << 20) : (bytes >= (1u << 20) ? (1u << 20) : 4096);
  return (bytes + g - 1) / g * g;
}

void Context::trim_locked(size_t need, std::vector<void *> &victims) {
  // largest cached blocks first; the caller frees them outside the lock
  while (!free_blocks.empty() && in_use + cached + need > budget) {
    auto it = std::prev(free_blocks.end());
    victims.push_back(it->second);
    cached -= it->first;
    free_blocks.erase(it);
  }
}

void *Context::alloc(size_t bytes) {
  bytes = round_alloc(bytes == 0 ? 8 : bytes);
  std::vector<void *> victims;
  {
    std::lock_guard<std::mutex> g(mu);
    // reuse a cached block of at least `bytes` and at most 1.25x larger
    auto it = free_blocks.lower_bound(bytes);
    if (it != free_blocks.end() && it->first <= bytes + bytes / 4) {
      void *p = it->second;
      const size_t sz = it->first;
      free_blocks.erase(it);
      cached -= sz;
      in_use += sz;
      high_water = std::max(high_water, in_use);
      // record the actual block size for release
      sizes_[p] = sz;
      return p;
    }
    trim_locked(bytes, victims);
    if (in_use + cached + bytes > budget)
      fail(SSRPA_ERR_NOMEM, "HBM budget exceeded: %zu in use + %zu requested > %zu",
           in_use, bytes, budget);
    in_use += bytes;  // reserved while the lock is released
  }
  // cached blocks are idle (released only after their stream finished); the
  // runtime calls run without the lock so other threads keep allocating
  for (void *v : victims) (void)hipFree(v);
  victims.clear();
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  // The budget is a model: memory held outside this context (other
  // libraries, other processes) can make the device refuse an allocation
  // that fits it.  Then the cached blocks go back to the device, and while
  // other threads of this context keep releasing memory (concurrent
  // solves finishing) the allocation is retried; it fails once no release
  // has come for kOomWaitSeconds, or after kOomGiveUpSeconds in all.
  constexpr double kOomWaitSeconds = 5.0, kOomGiveUpSeconds = 600.0;
  const auto t_start = std::chrono::steady_clock::now();
  while (e != hipSuccess) {
    (void)hipGetLastError();
    uint64_t gen;
    {
      std::lock_guard<std::mutex> g(mu);
      for (auto &fb : free_blocks) victims.push_back(fb.second);
      free_blocks.clear();
      cached = 0;
      gen = release_gen;
    }
    for (void *v : victims) (void)hipFree(v);
    victims.clear();
    e = hipMalloc(&p, bytes);
    if (e == hipSuccess) break;
    (void)hipGetLastError();
    const double waited = std::chrono::duration<double>(
                              std::chrono::steady_clock::now() - t_start).count();
    bool released = false;
    if (waited < kOomGiveUpSeconds) {
      std::unique_lock<std::mutex> lk(mu);
      released = cv_release.wait_for(
          lk, std::chrono::duration<double>(kOomWaitSeconds),
          [&] { return release_gen != gen; });
    }
    if (!released) {
      {
        std::lock_guard<std::mutex> g(mu);
        in_use -= bytes;
      }
      fail(SSRPA_ERR_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    e = hipMalloc(&p, bytes);
  }
  std::lock_guard<std::mutex> g(mu);
  high_water = std::max(high_water, in_use);
  sizes_[p] = bytes;
  return p;
}

void Context::release(void *p, size_t) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu);
  auto it = sizes_.find(p);
  if (it == sizes_.end()) return;
  const size_t sz = it->second;
  sizes_.erase(it);
  in_use -= sz;
  free_blocks.emplace(sz, p);
  cached += sz;
  release_gen += 1;
  cv_release.notify_all();
}

// Error text is kept per calling thread and context, so concurrent callers
// (e.g. serving workers) do not overwrite each other's message.
static std::map<const Context *, std::string> &thread_errors() {
  static thread_local std::map<const Context *, std::string> m;
  return m;
}

void Context::set_error(const std::string &m) { thread_errors()[this] = m; }

std::string Context::error() {
  auto &m = thread_errors();
  auto it = m.find(this);
  return it == m.end() ? std::string() : it->second;
}

Context::~Context() {
  for (auto &fb : free_blocks) (void)hipFree(fb.second);
  for (auto &kv : sizes_) (void)hipFree(kv.first);
}

int StageTimer::start(int stage, hipStream_t s) {
  Rec r{stage, nullptr, nullptr};
  SSRPA_HIP(hipEventCreate(&r.a));
  SSRPA_HIP(hipEventCreate(&r.b));
  SSRPA_HIP(hipEventRecord(r.a, s));
  recs.push_back(r);
  return (int)recs.size() - 1;
}

void StageTimer::stop(int idx, hipStream_t s) {
  (void)hipEventRecord(recs[idx].b, s);
}

void StageTimer::clear() {
  for (auto &r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  recs.clear();
}

DevBuf::DevBuf(Context *ctx, size_t bytes) : ctx_(ctx), bytes_(bytes) {
  ptr_ = ctx->alloc(bytes);
}

DevBuf::~DevBuf() {
  if (ptr_ && ctx_) {
    // a block released while a failed call unwinds may still be read or
    // written by work queued on the call's stream
    sync_api_stream_on_unwind();
    ctx_->release(ptr_, bytes_);
  }
}

ApiStream &api_stream() {
  static thread_local ApiStream a;
  return a;
}

void sync_api_stream_on_unwind() {
  const ApiStream &a = api_stream();
  if (a.set && std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(a.s);
}

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_235(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

void invert3(const double *a, double *inv, double *det) {
  const double d = a[0] * (a[4] * a[8] - a[5] * a[7]) -
                   a[1] * (a[3] * a[8] - a[5] * a[6]) +
                   a[2] * (a[3] * a[7] - a[4] * a[6]);
  *det = d;
  inv[0] = (a[4] * a[8] - a[5] * a[7]) / d;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) / d;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) / d;
  inv[3] = (a[5] * a[6] - a[3] * a[8]) / d;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) / d;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) / d;
  inv[6] = (a[3] * a[7] - a[4] * a[6]) / d;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) / d;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) / d;
}

double gnorm2(const Geometry &g, double n1, double n2, double n3) {
  double v[3];
  for (int c = 0; c < 3; ++c)
    v[c] = n1 * g.recip[c] + n2 * g.recip[3 + c] + n3 * g.recip[6 + c];
  return v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
}

// Validate a description and derive the geometry (no device work).
// qf: the q-point in fractions of the reciprocal vectors (nullptr: q = 0).
// The chi0 set is {G : |G - q|^2 / 2 <= ecut_chi, G != q} with
// v(G - q) = 4 pi / |G - q|^2 (the pair matrix has its bra on the valence
// side, so Eq. (3)'s q + G appears as G - q, see the k-mesh entry points).
Geometry make_geometry(const ssrpa_system_desc *d, const double *qf = nullptr) {
  SSRPA_REQUIRE(d, SSRPA_ERR_ARG, "null system description");
  SSRPA_REQUIRE(d->n_v >= 1 && d->n_c >= 1, SSRPA_ERR_ARG,
                "need at least one valence and one conduction band");
  SSRPA_REQUIRE(d->n_pw >= d->n_v + d->n_c, SSRPA_ERR_ARG,
                "%d bands exceed %d plane waves", d->n_v + d->n_c, d->n_pw);
  SSRPA_REQUIRE(d->miller && d->coeff && d->energy, SSRPA_ERR_ARG,
                "null miller/coeff/energy pointer");
  SSRPA_REQUIRE(d->ecut_chi > 0.0 && std::isfinite(d->ecut_chi), SSRPA_ERR_ARG,
                "ecut_chi must be positive");
  Geometry g{};
  std::memcpy(g.lattice, d->lattice, sizeof(g.lattice));
  double inv[9], det;
  invert3(g.lattice, inv, &det);
  SSRPA_REQUIRE(std::isfinite(det) && std::fabs(det) > 1e-12, SSRPA_ERR_ARG,
                "singular lattice");
  g.volume = std::fabs(det);
  // B = 2 pi A^-T: row j of B is 2 pi times column j of A^-1
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) g.recip[3 * j + c] = 2.0 * kPi * inv[3 * c + j];
  g.n1 = d->fft[0];
  g.n2 = d->fft[1];
  g.n3 = d->fft[2];
  for (int i = 0; i < 3; ++i)
    SSRPA_REQUIRE(is_235(d->fft[i]) && d->fft[i] <= 128 && d->fft[i] >= 2,
                  SSRPA_ERR_ARG, "FFT size %d must be 2^i 3^j in [2, 128]",
                  d->fft[i]);
  // chi0 set: G != 0, |G|^2/2 <= ecut, lexicographic in (n1, n2, n3)
  const double gmax = std::sqrt(2.0 * d->ecut_chi);
  int nb[3];
  for (int i = 0; i < 3; ++i) {
    const double al = std::sqrt(g.lattice[3 * i] * g.lattice[3 * i] +
                                g.lattice[3 * i + 1] * g.lattice[3 * i + 1] +
                                g.lattice[3 * i + 2] * g.lattice[3 * i + 2]);
    nb[i] = (int)std::floor(gmax * al / (2.0 * kPi)) + 1 +
            (qf ? (int)std::ceil(std::fabs(qf[i])) : 0);
    SSRPA_REQUIRE(nb[i] < 512, SSRPA_ERR_ARG, "ecut_chi too large");
  }
  const double q0 = qf ? qf[0] : 0.0, q1 = qf ? qf[1] : 0.0, q2 = qf ? qf[2] : 0.0;
  const bool q_lattice = q0 == std::round(q0) && q1 == std::round(q1) &&
                         q2 == std::round(q2);
  SSRPA_REQUIRE(!qf || (std::isfinite(q0) && std::isfinite(q1) && std::isfinite(q2)),
                SSRPA_ERR_ARG, "non-finite q");
  // a q on the reciprocal lattice is q = 0 (pass it reduced)
  SSRPA_REQUIRE(!q_lattice || (q0 == 0.0 && q1 == 0.0 && q2 == 0.0), SSRPA_ERR_ARG,
                "q is a reciprocal lattice vector: pass q = 0");
  g.q_zero = q_lattice;
  // slab truncation along a3: z_c = |a3|/2, a3 normal to a1 and a2
  g.truncation = d->coulomb_truncation;
  SSRPA_REQUIRE(g.truncation == 0 || g.truncation == 1, SSRPA_ERR_ARG,
                "unknown Coulomb truncation %d", g.truncation);
  double nz[3] = {0, 0, 0}, zc = 0.0;
  if (g.truncation == 1) {
    const double *a3 = g.lattice + 6;
    const double l3 = std::sqrt(a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2]);
    for (int i = 0; i < 2; ++i) {
      const double *ai = g.lattice + 3 * i;
      const double li = std::sqrt(ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2]);
      const double dot = ai[0] * a3[0] + ai[1] * a3[1] + ai[2] * a3[2];
      SSRPA_REQUIRE(std::fabs(dot) <= 1e-10 * li * l3, SSRPA_ERR_ARG,
                    "slab truncation needs a3 normal to a1 and a2");
    }
    for (int c = 0; c < 3; ++c) nz[c] = a3[c] / l3;
    zc = 0.5 * l3;
  }
  g.m1 = g.m2 = g.m3 = 0;
  for (int a = -nb[0]; a <= nb[0]; ++a)
    for (int b = -nb[1]; b <= nb[1]; ++b)
      for (int c = -nb[2]; c <= nb[2]; ++c) {
        if (g.q_zero && a == 0 && b == 0 && c == 0) continue;
        const double g2 = gnorm2(g, a - q0, b - q1, c - q2);
        if (0.5 * g2 <= d->ecut_chi) {
          g.miller_chi.push_back(a);
          g.miller_chi.push_back(b);
          g.miller_chi.push_back(c);
          double v = 4.0 * kPi / g2;
          if (g.truncation == 1) {
            double gv[3];
            for (int q = 0; q < 3; ++q)
              gv[q] = (a - q0) * g.recip[q] + (b - q1) * g.recip[3 + q] +
                      (c - q2) * g.recip[6 + q];
            const double gz = gv[0] * nz[0] + gv[1] * nz[1] + gv[2] * nz[2];
            const double gpar = std::sqrt(std::max(0.0, g2 - gz * gz));
            v *= 1.0 - std::exp(-gpar * zc) * std::cos(gz * zc);
          }
          g.sqrt_v.push_back(std::sqrt(std::max(0.0, v)));
          g.m1 = std::max(g.m1, std::abs(a));
          g.m2 = std::max(g.m2, std::abs(b));
          g.m3 = std::max(g.m3, std::abs(c));
        }
      }
  g.n_g = (int)g.sqrt_v.size();
  SSRPA_REQUIRE(g.n_g >= 1, SSRPA_ERR_ARG, "empty chi0 basis (ecut_chi too small)");
  {
    double smax = 0.0;
    for (double x : g.sqrt_v) smax = std::max(smax, x);
    g.store_scale.resize(g.n_g);
    g.rescale.resize(g.n_g);
    for (int i = 0; i < g.n_g; ++i) {
      const double sv = g.sqrt_v[i];
      const bool tiny = sv <= 1e-6 * smax;
      g.store_scale[i] = tiny ? 1.0 : sv;
      g.rescale[i] = tiny ? sv : 1.0;
      g.rescaled |= tiny;
    }
  }
  g.real = d->real_orbitals != 0;
  SSRPA_REQUIRE(d->real_orbitals == 0 || d->real_orbitals == 1, SSRPA_ERR_ARG,
                "real_orbitals must be 0 or 1");
  // real path: 128-wide contraction tiles
  g.ld_g = round_up(g.n_g, g.real ? 128 : 64);
  if (g.real) {
    std::map<std::tuple<int, int, int>, int> at;
    for (int i = 0; i < g.n_g; ++i)
      at[std::make_tuple(g.miller_chi[3 * i], g.miller_chi[3 * i + 1],
                         g.miller_chi[3 * i + 2])] = i;
    g.neg.resize(g.n_g);
    for (int i = 0; i < g.n_g; ++i) {
      auto it = at.find(std::make_tuple(-g.miller_chi[3 * i], -g.miller_chi[3 * i + 1],
                                        -g.miller_chi[3 * i + 2]));
      SSRPA_REQUIRE(it != at.end(), SSRPA_ERR_ARG, "chi0 set not symmetric");
      g.neg[i] = it->second;
    }
    // the set is lexicographic, so the larger member of {G, -G} has the
    // larger index
    g.nh = g.n_g / 2;
    g.hj.assign(g.n_g, 0);
    g.hs.assign(g.n_g, 0);
    for (int i = 0; i < g.n_g; ++i)
      if (g.neg[i] < i) {
        const int j = (int)g.hpos.size();
        g.hpos.push_back(i);
        g.hneg.push_back(g.neg[i]);
        g.hj[i] = g.hj[g.neg[i]] = j;
        g.hs[i] = 1;
        g.hs[g.neg[i]] = -1;
      }
    SSRPA_REQUIRE((int)g.hpos.size() == g.nh && 2 * g.nh == g.n_g, SSRPA_ERR_ARG,
                  "chi0 set without its G -> -G pairing");
  }
  // alias-free bound N_i >= 2 max|n_psi,i| + max|n_chi,i| + 1
  int mp[3] = {0, 0, 0};
  for (int p = 0; p < d->n_pw; ++p)
    for (int i = 0; i < 3; ++i) mp[i] = std::max(mp[i], std::abs(d->miller[3 * p + i]));
  const int mc[3] = {g.m1, g.m2, g.m3};
  for (int i = 0; i < 3; ++i)
    SSRPA_REQUIRE(d->fft[i] >= 2 * mp[i] + mc[i] + 1, SSRPA_ERR_ALIAS,
                  "FFT size %d along axis %d is below the alias-free bound %d",
                  d->fft[i], i, 2 * mp[i] + mc[i] + 1);
  SSRPA_REQUIRE((long)(2 * g.m1 + 1) * g.n2 < (1 << 20), SSRPA_ERR_ARG,
                "grid too large");
  // columns (n1, n2) of the chi0 set; the set is lexicographic in (n1, n2, n3)
  const int ny2 = 2 * g.m2 + 1;
  g.cmap.assign((size_t)(2 * g.m1 + 1) * ny2, -1);
  g.zcode.resize(g.n_g);
  for (int i = 0; i < g.n_g; ++i) {
    const int a = g.miller_chi[3 * i], b = g.miller_chi[3 * i + 1],
              c = g.miller_chi[3 * i + 2];
    int &col = g.cmap[(size_t)(a + g.m1) * ny2 + b + g.m2];
    if (col < 0) {
      col = g.ncol++;
      // the (0, 0) column skips n3 = 0 (G = 0 is not in the set)
      g.zcol.insert(g.zcol.end(), {i, c, c, (g.q_zero && a == 0 && b == 0) ? 1 : 0});
    }
    g.zcol[4 * col + 2] = c;  // n3 ascends within a column
    g.zcode[i] = col | ((((c % g.n3) + g.n3) % g.n3) << 20);
  }
  g.ldy = round_up(g.ncol, 8);
  return g;
}

size_t bytes_c(size_t n) { return 16 * n; }

}  // namespace

BandSets band_sets(const ssrpa_system_desc *d) {
  BandSets b;
  const int n_b = d->n_v + d->n_c;
  const double *e = d->energy;
  for (int i = 0; i < n_b; ++i)
    SSRPA_REQUIRE(std::isfinite(e[i]), SSRPA_ERR_ARG, "non-finite energy");
  if (!d->occupation) {
    double vmax = -INFINITY, cmin = INFINITY;
    for (int i = 0; i < d->n_v; ++i) vmax = std::max(vmax, e[i]);
    for (int i = d->n_v; i < n_b; ++i) cmin = std::min(cmin, e[i]);
    SSRPA_REQUIRE(cmin > vmax, SSRPA_ERR_ARG,
                  "every conduction energy must lie above every valence energy");
    b.n_val = d->n_v;
    b.c_first = d->n_v;
    b.n_cond = d->n_c;
    return b;
  }
  // partial occupations (Eqs. 4-6): f in [0, 1], non-increasing along the
  // bands, energies non-decreasing, equal energies only with equal f
  const double *f = d->occupation;
  int n_pos = 0, n_full = 0;
  for (int i = 0; i < n_b; ++i) {
    SSRPA_REQUIRE(std::isfinite(f[i]) && f[i] >= 0.0 && f[i] <= 1.0,
                  SSRPA_ERR_ARG, "occupation %d = %g outside [0, 1]", i, f[i]);
    if (i > 0) {
      SSRPA_REQUIRE(f[i] <= f[i - 1], SSRPA_ERR_ARG,
                    "occupations must not increase along the bands (band %d)", i);
      SSRPA_REQUIRE(e[i] >= e[i - 1], SSRPA_ERR_ARG,
                    "energies must be ascending with occupations (band %d)", i);
      SSRPA_REQUIRE(e[i] > e[i - 1] || f[i] == f[i - 1], SSRPA_ERR_ARG,
                    "bands %d and %d have equal energies but different "
                    "occupations", i - 1, i);
    }
    n_pos += f[i] > 0.0;
    n_full += f[i] == 1.0;
  }
  SSRPA_REQUIRE(n_pos == d->n_v, SSRPA_ERR_ARG,
                "n_v = %d but %d bands have a positive occupation", d->n_v, n_pos);
  SSRPA_REQUIRE(n_full < n_b, SSRPA_ERR_ARG, "no band with occupation below 1");
  b.n_val = n_pos;
  b.c_first = n_full;
  b.n_cond = n_b - n_full;
  b.partial = n_pos > n_full;
  return b;
}

namespace {

struct Footprint {
  size_t resident, block, subspace, freq, eig, total;
};

Footprint footprint_of(const ssrpa_system_desc *d, const Geometry &g, int n_eig,
                       int n_freq, int vb, ssrpa_precision prec) {
  Footprint f{};
  const BandSets bs = band_sets(d);
  const size_t nb = (size_t)d->n_v + d->n_c;
  const size_t box = (size_t)g.n1 * g.n2 * g.n3;
  const size_t ng = g.n_g, ldg = g.ld_g;
  const bool full = n_eig >= g.n_g;
  const size_t ne = full ? ng : (size_t)n_eig;
  const size_t lde = full ? ldg : (size_t)round_up(n_eig, 64);
  const size_t pairs = (size_t)vb * bs.n_cond;
  // orbitals on the grid, chi0, per-G tables, and the coefficient copy that
  // lives while the orbitals are staged
  f.resident = bytes_c(nb * box) + bytes_c(ng * ng) + 64 * ldg +
               bytes_c(nb * (size_t)d->n_pw);
  f.block = pairs * (2 * ldg * 8 + 8 + (bs.partial ? 8 : 0));
  if (staged_grid(g)) {
    const size_t ypp = stage_bytes_per_pair(g);
    f.block += (size_t)vb * stage_chunk_c(vb, bs.n_cond, ypp) * ypp;
  }
  f.subspace = full ? 0 : pairs * 2 * lde * 8 + bytes_c(ldg * lde);
  // FP64 split-K partial tiles: the frequency contraction, the
  // Newton-Schulz Gram matrix of the eigensolver and the static pass
  HerkArgs hf{};
  hf.ld = (int)lde;
  hf.ncol = (int)ne;
  hf.k = (long)pairs;
  hf.n_omega = n_freq;
  f.freq = 2 * bytes_c(ne * ne) * n_freq + herk_f64_workspace(hf);
  HerkArgs hn{};
  hn.ld = (int)lde;
  hn.ncol = (int)ne;
  hn.k = (long)ng;
  hn.n_omega = 1;
  hn.unit_weight = 1;
  f.eig = full ? 0 : bytes_c(ng * ng) + eig_workspace_bytes((int)ng) +
                         6 * ng * lde * 8 + 3 * bytes_c(ldg * lde) +
                         herk_f64_workspace(hn);
  HerkArgs hs{};
  hs.ld = (int)ldg;
  hs.ncol = (int)ng;
  hs.k = (long)pairs;
  hs.n_omega = 1;
  size_t stat = herk_f64_workspace(hs);
  if (prec != SSRPA_FP64) {
    // converted rows and 128 x 128 partial tiles of the Gram path
    HerkArgs h{};
    h.ncol = g.n_g;
    h.k = (long)pairs;
    h.n_omega = 1;
    stat = std::max(stat, herk_gram_workspace(h, prec));
    h.ncol = (int)ne;
    h.n_omega = n_freq;
    f.freq += herk_gram_workspace(h, prec);
  }
  // the caching allocator rounds blocks up (<= 12.5%) and reuses blocks up to
  // 25% larger than asked: budget for that slack
  const size_t live = f.resident + f.block + std::max(stat, f.subspace + f.freq + f.eig);
  f.total = live + live / 4 + (128u << 20);
  return f;
}

struct Stream {
  hipStream_t s;
  explicit Stream(void *p) : s(static_cast<hipStream_t>(p)) {}
};

ssrpa_status finish(Context *ctx, const std::exception_ptr &ep) {
  try {
    std::rethrow_exception(ep);
  } catch (const Error &e) {
    if (ctx) ctx->set_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->set_error("host allocation failed");
    return SSRPA_ERR_NOMEM;
  } catch (const std::exception &e) {
    if (ctx) ctx->set_error(e.what());
    return SSRPA_ERR_ARG;
  } catch (...) {
    if (ctx) ctx->set_error("unknown error");
    return SSRPA_ERR_ARG;
  }
}

template <class F>
ssrpa_status guarded(Context *ctx, F &&f) {
  try {
    if (ctx) ctx->set_error("");
    f();
    return SSRPA_OK;
  } catch (...) {
    return finish(ctx, std::current_exception());
  }
}

void set_device(Context *ctx) { SSRPA_HIP(hipSetDevice(ctx->device)); }

// SSRPA_VERBOSE=1: one line on stderr per finished valence block (the block
// is synchronized first), for long solves.
bool verbose() {
  static const bool v = [] {
    const char *e = getenv("SSRPA_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

void block_done(const char *stage, int v0, int nvb, int n_v, hipStream_t s) {
  if (!verbose()) return;
  SSRPA_HIP(hipStreamSynchronize(s));
  fprintf(stderr, "ssrpa: %s: valence bands %d-%d of %d done\n", stage, v0,
          v0 + nvb - 1, n_v);
  fflush(stderr);
}

int resolve_block(System &sys, int requested, int n_eig, int n_freq) {
  if (requested > 0) return std::min(requested, sys.n_v);
  // largest block whose pair matrices fit in the remaining budget
  Context *ctx = sys.ctx;
  size_t free_b;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    free_b = ctx->budget > ctx->in_use ? ctx->budget - ctx->in_use : 0;
  }
  const bool full = n_eig >= sys.geo.n_g;
  const size_t lde = full ? 0 : (size_t)round_up(std::max(n_eig, 1), 64);
  const size_t per_band = (size_t)sys.n_c * (2 * sys.geo.ld_g * 8 + 8 + 2 * lde * 8);
  const size_t reserve = (size_t)1 << 30;
  const size_t avail = free_b > reserve ? free_b - reserve : 0;
  // the pair transform's stage: n_c * ypp per band, at most kStageBytes
  const size_t stage_band = staged_grid(sys.geo)
                                ? (size_t)sys.n_c * stage_bytes_per_pair(sys.geo)
                                : 0;
  size_t nb = avail / std::max<size_t>(per_band + stage_band, 1);
  if (nb * stage_band > kStageBytes)
    nb = avail > kStageBytes ? (avail - kStageBytes) / std::max<size_t>(per_band, 1) : 0;
  int vb = (int)std::min<size_t>(sys.n_v, nb);
  SSRPA_REQUIRE(vb >= 1, SSRPA_ERR_NOMEM,
                "one valence band of pair matrices (%zu bytes) exceeds the budget",
                per_band);
  (void)n_freq;
  return vb;
}

// Pair matrix of one block (cached when one block covers all valence bands).
// Per-G tables of the system's geometry on the device (pair-transform
// columns and scales, s(G) and r(G)), the error flag and the twiddles.  The
// host tables stay in the system for the asynchronous copies.
void upload_geometry(System &sys, hipStream_t s) {
  Context *ctx = sys.ctx;
  const Geometry &g = sys.geo;
  const size_t box = (size_t)g.n1 * g.n2 * g.n3;
  std::vector<int> &code = sys.code_host;
  std::vector<double> &scale = sys.scale_host;
  code.assign(g.n_g, 0);
  // [0, ld_g) s(G) Omega/N, [ld_g, 2 ld_g) Omega/N, then s(G), r(G)
  scale.assign(2 * ((size_t)g.ld_g + g.n_g), 0.0);
  const double on = g.volume / (double)box;
  for (int i = 0; i < g.n_g; ++i) {
    const int a = g.miller_chi[3 * i], b = g.miller_chi[3 * i + 1],
              c = g.miller_chi[3 * i + 2];
    const int col = (a + g.m1) * g.n2 + ((b % g.n2) + g.n2) % g.n2;
    const int k3 = ((c % g.n3) + g.n3) % g.n3;
    code[i] = col | (k3 << 20);
    scale[i] = on * g.store_scale[i];
    scale[g.ld_g + i] = on;
    scale[2 * (size_t)g.ld_g + i] = g.store_scale[i];
    scale[2 * (size_t)g.ld_g + g.n_g + i] = g.rescale[i];
  }
  sys.gcol = DevBuf(ctx, sizeof(int) * g.n_g);
  sys.sqrtv_d = DevBuf(ctx, sizeof(double) * scale.size());
  SSRPA_HIP(hipMemcpyAsync(sys.gcol.as(), code.data(), sizeof(int) * g.n_g,
                           hipMemcpyHostToDevice, s));
  SSRPA_HIP(hipMemcpyAsync(sys.sqrtv_d.as(), scale.data(),
                           sizeof(double) * scale.size(), hipMemcpyHostToDevice, s));
  sys.zcode = DevBuf(ctx, sizeof(int) * g.n_g);
  sys.cmap = DevBuf(ctx, sizeof(int) * g.cmap.size());
  SSRPA_HIP(hipMemcpyAsync(sys.zcode.as(), g.zcode.data(), sizeof(int) * g.n_g,
                           hipMemcpyHostToDevice, s));
  SSRPA_HIP(hipMemcpyAsync(sys.cmap.as(), g.cmap.data(),
                           sizeof(int) * g.cmap.size(), hipMemcpyHostToDevice, s));
  sys.zcol = DevBuf(ctx, sizeof(int) * g.zcol.size());
  SSRPA_HIP(hipMemcpyAsync(sys.zcol.as(), g.zcol.data(),
                           sizeof(int) * g.zcol.size(), hipMemcpyHostToDevice, s));
  sys.dev_flag = DevBuf(ctx, 64);
  fill_zero(sys.dev_flag.as(), 64, s);
  upload_twiddles(sys, s);
}

// Packed pair rows of the real path: F = M_v,c1 + i M_v,c2 for the
// conduction pairs (c1, c2) packed into one orbital (planar complex rows).
void packed_pairs(System &sys, int v0, int nvb, bool scaled, DevBuf &f,
                  hipStream_t s) {
  f.ensure(sys.ctx, (size_t)nvb * sys.orb_nc * 2 * sys.geo.ld_g * sizeof(double), s);
  launch_pair_matrix(sys, v0, nvb, scaled, f.as<double>(), s);
}

// Pair rows of one block: complex planar rows (2 ld_g doubles), or in the
// real path real rows of ld_g doubles in the cos/sin basis.
const double *block_pairs(System &sys, int v0, int nvb, DevBuf &scratch,
                          hipStream_t s) {
  const bool single = sys.sources.empty() && v0 == 0 && nvb == sys.n_v;
  const size_t bytes = (size_t)nvb * sys.n_c * (sys.real ? 1 : 2) *
                       sys.geo.ld_g * sizeof(double);
  if (single && sys.w_cache_valid) return sys.w_cache.as<double>();
  DevBuf &dst = single ? sys.w_cache : scratch;
  dst.ensure(sys.ctx, bytes, s);
  {
    StageScope sc(sys.timer, SSRPA_STAGE_PAIR_FFT, s);
    const Geometry &g = sys.geo;
    if (sys.real) {
      DevBuf f;
      packed_pairs(sys, v0, nvb, true, f, s);
      const int *t = sys.rtab.as<int>();
      unpack_real_rows(f.as<double>(), nvb, sys.n_c, g.ld_g, g.nh, t, t + g.nh,
                       dst.as<double>(), s);
    } else {
      launch_pair_matrix(sys, v0, nvb, true, dst.as<double>(), s);
    }
    if (sys.partial) {
      // rows carry (f_v - f_c)^1/2: every contraction of the block then
      // weighs pair p with (f_v - f_c) Delta_p (Eq. 5 with occupations)
      const long rows = (long)nvb * sys.n_c;
      sys.rowscale.ensure(sys.ctx, sizeof(double) * rows, s);
      pair_energy_diffs(sys.energy_d.as<double>(), sys.occ_d.as<double>(),
                        sys.c_first, v0, nvb, sys.n_c, nullptr,
                        sys.rowscale.as<double>(), s);
      // a real row of ld_g doubles is a "planar" row of half that width
      scale_rows(dst.as<double>(), rows, sys.real ? g.ld_g / 2 : g.ld_g,
                 sys.rowscale.as<double>(), s);
    }
  }
  if (single) sys.w_cache_valid = true;
  return dst.as<double>();
}

// Pair sources: the system's own pairs (one source), or the k-mesh sources.
int n_sources(const System &sys) {
  return sys.sources.empty() ? 1 : (int)sys.sources.size();
}

// Point the pair transform at source i; returns its weight g_k.
double select_source(System &sys, int i) {
  if (sys.sources.empty()) {
    sys.src_psi_v = sys.src_psi_c = nullptr;
    return 1.0;
  }
  const System::PairSource &p = sys.sources[i];
  sys.src_psi_v = p.psi_v;
  sys.src_psi_c = p.psi_c;
  return p.weight;
}

// e_c - e_v for the rows of one block of source i (the occupations of
// partially occupied systems included, see pair_energy_diffs).
void source_energy_diffs(System &sys, int i, int v0, int nvb, double *de,
                         hipStream_t s) {
  if (sys.sources.empty()) {
    pair_energy_diffs(sys.energy_d.as<double>(),
                      sys.partial ? sys.occ_d.as<double>() : nullptr,
                      sys.c_first, v0, nvb, sys.n_c, de, nullptr, s);
  } else {
    const System::PairSource &p = sys.sources[i];
    pair_energy_diffs2(p.e_v, p.e_c, sys.c_first, v0, nvb, sys.n_c, de, s);
  }
}

void static_chi0(System &sys, ssrpa_precision prec, int vb, hipStream_t s) {
  Context *ctx = sys.ctx;
  const Geometry &g = sys.geo;
  if (sys.chibar0.empty())
    sys.chibar0 = DevBuf(ctx, bytes_c((size_t)g.n_g * g.n_g));
  DevBuf scratch, de, ws;
  DevBuf om(ctx, sizeof(double));
  fill_zero(om.as(), sizeof(double), s);
  int blk = 0;
  for (int si = 0; si < n_sources(sys); ++si)
  for (int v0 = 0; v0 < sys.n_v; v0 += vb, ++blk) {
    const double gk = select_source(sys, si);
    const int nvb = std::min(vb, sys.n_v - v0);
    const double *w = block_pairs(sys, v0, nvb, scratch, s);
    de.ensure(ctx, sizeof(double) * (size_t)nvb * sys.n_c, s);
    source_energy_diffs(sys, si, v0, nvb, de.as<double>(), s);
    HerkArgs h{};
    h.a = w;
    h.lda = 2L * g.ld_g;
    h.im_off = g.ld_g;
    h.ncol = g.n_g;
    h.ld = g.ld_g;
    h.k = (long)nvb * sys.n_c;
    h.de = de.as<double>();
    h.omega = om.as<double>();
    h.n_omega = 1;
    h.wscale = gk / g.volume;
    h.timer = &sys.timer;
    h.stage = SSRPA_STAGE_CHI0_HERK;
    if (sys.real) {
      h.lda = g.ld_g;
      h.im_off = 0;
      syrk(ctx, h, sys.chibar0.as<double>(), 0, blk > 0 ? 1 : 0, ws, s);
    } else {
      herk(ctx, h, prec, sys.chibar0.as<double>(), 0, blk > 0 ? 1 : 0, ws, s);
    }
    block_done("static chi0", v0, nvb, sys.n_v, s);
  }
  sys.src_psi_v = sys.src_psi_c = nullptr;
  SSRPA_HIP(hipStreamSynchronize(s));
  sys.have_chi0 = true;
  sys.sub = Subspace();
}

void compute_subspace(System &sys, int n_eig, int kind, hipStream_t s) {
  Context *ctx = sys.ctx;
  const Geometry &g = sys.geo;
  SSRPA_REQUIRE(sys.have_chi0, SSRPA_ERR_STATE,
                "ssrpa_chi0_static must run before ssrpa_subspace");
  SSRPA_REQUIRE(n_eig >= 1 && n_eig <= g.n_g, SSRPA_ERR_ARG,
                "n_eig=%d outside [1, %d]", n_eig, g.n_g);
  SSRPA_REQUIRE(kind == SSRPA_BASIS_SYMMETRIZED || kind == SSRPA_BASIS_CHI0,
                SSRPA_ERR_ARG, "unknown basis kind %d", kind);
  Subspace sub;
  sub.n_eig = n_eig;
  sub.kind = kind;
  // the real path contracts with 128-wide tiles
  sub.ld_e = round_up(n_eig, sys.real ? 128 : 64);
  sub.basis = DevBuf(ctx, sizeof(double) * 2 * (size_t)g.ld_g * sub.ld_e);
  DevBuf ev(ctx, sizeof(double) * n_eig);
  StageScope sc(sys.timer, SSRPA_STAGE_EIGEN, s);
  // s(G) and r(G) in the order of the basis the static matrix is held in
  const double *tab = sys.real ? sys.rscale.as<double>()
                               : sys.sqrtv_d.as<double>() + 2 * (size_t)g.ld_g;
  const double *rs = tab + g.n_g;
  DevBuf tmp;
  const double *a = sys.chibar0.as<double>();
  if (kind == SSRPA_BASIS_CHI0 || g.rescaled) {
    tmp = DevBuf(ctx, bytes_c((size_t)g.n_g * g.n_g));
    copy_interleaved(a, tmp.as<double>(), (size_t)g.n_g * g.n_g, s);
    if (kind == SSRPA_BASIS_CHI0)
      scale_sym(tmp.as<double>(), g.n_g, tab, 1, s);   // chi0 = S^-1 (.) S^-1
    else
      scale_sym(tmp.as<double>(), g.n_g, rs, 0, s);    // R (.) R
    a = tmp.as<double>();
  }
  eig_lowest(ctx, a, g.n_g, n_eig, ev.as<double>(), sub.basis.as<double>(),
             sub.ld_e, sys.dev_flag.as<int>(), s);
  tmp.reset();
  if (kind == SSRPA_BASIS_SYMMETRIZED && g.rescaled) {
    // the projection multiplies the stored rows: W C_s = W_stored (R C_s)
    sub.basis_r = DevBuf(ctx, sub.basis.bytes());
    copy_interleaved(sub.basis.as<double>(), sub.basis_r.as<double>(),
                     sub.basis.bytes() / 16, s);
    scale_rows(sub.basis_r.as<double>(), g.n_g, sub.ld_e, rs, s);
  }
  if (kind == SSRPA_BASIS_CHI0) {
    // v_s = C_s^H v C_s = (V^1/2 C_s)^H (V^1/2 C_s), V^1/2 = S R
    const int le = sub.ld_e;
    DevBuf av(ctx, sub.basis.bytes());
    copy_interleaved(sub.basis.as<double>(), av.as<double>(), sub.basis.bytes() / 16, s);
    scale_rows(av.as<double>(), g.n_g, le, tab, s);
    scale_rows(av.as<double>(), g.n_g, le, rs, s);
    DevBuf vs(ctx, bytes_c((size_t)n_eig * n_eig)), ws;
    HerkArgs h{};
    h.a = av.as<double>();
    h.lda = 2L * le;
    h.im_off = le;
    h.ncol = n_eig;
    h.ld = le;
    h.k = g.n_g;
    h.n_omega = 1;
    h.unit_weight = 1;
    herk(ctx, h, SSRPA_FP64, vs.as<double>(), 0, 0, ws, s);
    // v_s = U diag(l) U^H, Z = U diag(l^1/2): every eigenpair of v_s
    DevBuf lam(ctx, sizeof(double) * n_eig);
    DevBuf z(ctx, sizeof(double) * 2 * (size_t)le * le);
    eig_lowest(ctx, vs.as<double>(), n_eig, n_eig, lam.as<double>(),
               z.as<double>(), le, sys.dev_flag.as<int>(), s);
    scale_cols(z.as<double>(), le, le, n_eig, lam.as<double>(), 1, s);
    // B = S^-1 C_s Z, the operand that turns the stored rows into M C_s Z
    sub.proj = DevBuf(ctx, sub.basis.bytes());
    GemmArgs gm{};
    gm.a = sub.basis.as<double>(); gm.lda = 2L * le; gm.a_im = le;
    gm.b = z.as<double>(); gm.ldb = 2L * le; gm.b_im = le;
    gm.c = sub.proj.as<double>(); gm.ldc = 2L * le; gm.c_im = le;
    gm.m = g.ld_g; gm.n = le; gm.k = le;
    gm.alpha = 1.0; gm.beta = 0.0;
    DevBuf gws;
    gemm(ctx, gm, SSRPA_FP64, gws, s);
    scale_rows(sub.proj.as<double>(), g.n_g, le, tab, s, true);
    SSRPA_HIP(hipStreamSynchronize(s));  // work buffers are freed on return
  }
  sub.eigval.resize(n_eig);
  SSRPA_HIP(hipMemcpyAsync(sub.eigval.data(), ev.as(), sizeof(double) * n_eig,
                           hipMemcpyDeviceToHost, s));
  SSRPA_HIP(hipStreamSynchronize(s));
  for (double x : sub.eigval)
    SSRPA_REQUIRE(std::isfinite(x), SSRPA_ERR_NUMERIC, "eigensolver produced %g", x);
  sys.sub = std::move(sub);
}

// Milliseconds and launch counts per stage from a timer's event pairs.
void read_stage_times(StageTimer &tm, double *ms, int *launches) {
  if (!ms && !launches) return;
  double acc[SSRPA_N_STAGES] = {0};
  int cnt[SSRPA_N_STAGES] = {0};
  for (auto &r : tm.recs) {
    SSRPA_HIP(hipEventSynchronize(r.b));
    float t = 0.f;
    SSRPA_HIP(hipEventElapsedTime(&t, r.a, r.b));
    if (r.stage >= 0 && r.stage < SSRPA_N_STAGES) {
      acc[r.stage] += t;
      cnt[r.stage] += 1;
    }
  }
  for (int i = 0; i < SSRPA_N_STAGES; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
}

struct EcResult {
  double ec = 0.0;
  std::vector<double> f;
};

EcResult energy(System &sys, int n_eig, int n_freq, const double *omega,
                const double *weight, ssrpa_precision prec, int vb,
                double coupling, double *chi_sub, hipStream_t s) {
  Context *ctx = sys.ctx;
  const Geometry &g = sys.geo;
  SSRPA_REQUIRE(n_freq >= 1 && omega && weight, SSRPA_ERR_ARG,
                "need at least one frequency");
  for (int j = 0; j < n_freq; ++j)
    SSRPA_REQUIRE(std::isfinite(omega[j]) && std::isfinite(weight[j]),
                  SSRPA_ERR_ARG, "non-finite frequency or weight");
  const bool full = n_eig >= g.n_g;
  if (!full)
    SSRPA_REQUIRE(sys.sub.n_eig == n_eig && !sys.sub.basis.empty(), SSRPA_ERR_STATE,
                  "no subspace of size %d (call ssrpa_subspace first)", n_eig);
  const int n = full ? g.n_g : n_eig;
  const int ld = full ? g.ld_g : sys.sub.ld_e;
  DevBuf own_chis;
  double *chis = chi_sub;
  if (!chis) {
    own_chis = DevBuf(ctx, bytes_c((size_t)n * n * n_freq));
    chis = own_chis.as<double>();
  }
  DevBuf fw(ctx, sizeof(double) * (3 * (size_t)n_freq + 8));
  double *om_d = fw.as<double>();
  double *w_d = om_d + n_freq;
  double *f_d = w_d + n_freq;
  double *ec_d = f_d + n_freq;
  SSRPA_HIP(hipMemcpyAsync(om_d, omega, sizeof(double) * n_freq,
                           hipMemcpyHostToDevice, s));
  SSRPA_HIP(hipMemcpyAsync(w_d, weight, sizeof(double) * n_freq,
                           hipMemcpyHostToDevice, s));
  DevBuf scratch, de, ws, wsub, gws;
  int blk = 0;
  for (int si = 0; si < n_sources(sys); ++si)
  for (int v0 = 0; v0 < sys.n_v; v0 += vb, ++blk) {
    const double gk = select_source(sys, si);
    const int nvb = std::min(vb, sys.n_v - v0);
    const long rows = (long)nvb * sys.n_c;
    const double *w = block_pairs(sys, v0, nvb, scratch, s);
    de.ensure(ctx, sizeof(double) * rows, s);
    source_energy_diffs(sys, si, v0, nvb, de.as<double>(), s);
    HerkArgs h{};
    const long wcols = sys.real ? 1 : 2;   // real rows hold no imaginary plane
    if (full) {
      h.a = w;
      h.lda = wcols * g.ld_g;
      h.im_off = sys.real ? 0 : g.ld_g;
    } else {
      // W_s = W C_s  (Eq. 7)
      wsub.ensure(ctx, sizeof(double) * wcols * (size_t)rows * ld, s);
      StageScope sc(sys.timer, SSRPA_STAGE_PROJECTION, s);
      if (sys.real) {
        // real basis vectors: the real plane of the stored operand
        gemm_real(w, g.ld_g, sys.sub.projection(), 2L * ld, wsub.as<double>(),
                  ld, rows, g.ld_g, ld, s);
      } else {
        GemmArgs gm{};
        gm.a = w; gm.lda = 2L * g.ld_g; gm.a_im = g.ld_g;
        gm.b = sys.sub.projection();
        gm.ldb = 2L * ld; gm.b_im = ld;
        gm.c = wsub.as<double>(); gm.ldc = 2L * ld; gm.c_im = ld;
        gm.m = rows; gm.n = ld; gm.k = g.ld_g;
        gm.alpha = 1.0; gm.beta = 0.0;
        gemm(ctx, gm, prec, gws, s);
      }
      h.a = wsub.as<double>();
      h.lda = wcols * ld;
      h.im_off = sys.real ? 0 : ld;
    }
    h.ncol = n;
    h.ld = ld;
    h.k = rows;
    h.de = de.as<double>();
    h.omega = om_d;
    h.n_omega = n_freq;
    h.wscale = gk / g.volume;
    h.timer = &sys.timer;
    h.stage = SSRPA_STAGE_FREQ_HERK;
    if (sys.real)
      syrk(ctx, h, chis, 2L * n * n, blk > 0 ? 1 : 0, ws, s);
    else
      herk(ctx, h, prec, chis, 2L * n * n, blk > 0 ? 1 : 0, ws, s);
    block_done("subspace chi0(iw)", v0, nvb, sys.n_v, s);
  }
  sys.src_psi_v = sys.src_psi_c = nullptr;
  if (full && g.rescaled) {
    // full basis: v^1/2 chi0(i w) v^1/2 = R (stored matrix) R
    const double *rs = sys.real ? sys.rscale.as<double>() + g.n_g
                                : sys.sqrtv_d.as<double>() + 2 * (size_t)g.ld_g + g.n_g;
    for (int j = 0; j < n_freq; ++j)
      scale_sym(chis + 2L * n * n * j, n, rs, 0, s);
  }
  fill_zero(sys.dev_flag.as(), sizeof(int), s);
  {
    StageScope sc(sys.timer, SSRPA_STAGE_TRACE_LOG, s);
    trace_log(ctx, chis, n, n_freq, coupling, f_d, sys.dev_flag.as<int>(), s);
    quadrature(w_d, f_d, n_freq, ec_d, s);
  }
  EcResult r;
  r.f.resize(n_freq);
  int flag = 0;
  SSRPA_HIP(hipMemcpyAsync(r.f.data(), f_d, sizeof(double) * n_freq,
                           hipMemcpyDeviceToHost, s));
  SSRPA_HIP(hipMemcpyAsync(&r.ec, ec_d, sizeof(double), hipMemcpyDeviceToHost, s));
  SSRPA_HIP(hipMemcpyAsync(&flag, sys.dev_flag.as(), sizeof(int),
                           hipMemcpyDeviceToHost, s));
  SSRPA_HIP(hipStreamSynchronize(s));
  SSRPA_REQUIRE(flag == 0, SSRPA_ERR_NUMERIC,
                "1 - chi0_s v is not positive definite at some frequency");
  return r;
}

}  // namespace
}  // namespace ssrpa

using namespace ssrpa;

// A k mesh: one system per k-point (orbitals staged on the grid as the
// periodic parts u_nk(r)), their reduced coordinates and weights g_k.
struct ssrpa_kmesh {
  ssrpa_context *ctx = nullptr;
  std::vector<ssrpa_system *> k;
  std::vector<double> kfrac, kweight;
  ssrpa_system_desc d0{};
  std::vector<int32_t> miller0;
  int mp[3] = {0, 0, 0};   // max |n_psi,i| over every k-point
  StageTimer timer;        // stage events of the per-q solves
};

struct ssrpa_ticket {
  std::thread th;
  std::atomic<int> done{0};
  ssrpa_status status = SSRPA_OK;
  double ec = 0.0;
  std::vector<double> f;
};

extern "C" {

const char *ssrpa_status_string(ssrpa_status s) {
  switch (s) {
    case SSRPA_OK: return "ok";
    case SSRPA_ERR_ARG: return "invalid argument";
    case SSRPA_ERR_ALIAS: return "FFT grid below the alias-free bound";
    case SSRPA_ERR_NOMEM: return "out of device memory (HBM budget)";
    case SSRPA_ERR_HIP: return "HIP runtime error";
    case SSRPA_ERR_NUMERIC: return "numerical failure";
    case SSRPA_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}

const char *ssrpa_last_error(const ssrpa_context *ctx) {
  static thread_local std::string copy;
  copy = ctx ? const_cast<ssrpa_context *>(ctx)->error() : std::string();
  return copy.c_str();
}

const char *ssrpa_version(void) { return "0.1.0 gfx950"; }

ssrpa_status ssrpa_context_create(int hip_device, size_t hbm_budget_bytes,
                                  ssrpa_context **out) {
  if (!out) return SSRPA_ERR_ARG;
  *out = nullptr;
  auto *ctx = new (std::nothrow) ssrpa_context();
  if (!ctx) return SSRPA_ERR_NOMEM;
  ssrpa_status st = guarded(ctx, [&] {
    int n = 0;
    SSRPA_HIP(hipGetDeviceCount(&n));
    SSRPA_REQUIRE(hip_device >= 0 && hip_device < n, SSRPA_ERR_ARG,
                  "device %d not present (%d devices)", hip_device, n);
    ctx->device = hip_device;
    SSRPA_HIP(hipSetDevice(hip_device));
    size_t fr = 0, tot = 0;
    SSRPA_HIP(hipMemGetInfo(&fr, &tot));
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    // address of this device's fixed work array (allocation-free entry point)
    noalloc_setup(hip_device);
  });
  if (st != SSRPA_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return SSRPA_OK;
}

ssrpa_status ssrpa_context_destroy(ssrpa_context *ctx) {
  if (!ctx) return SSRPA_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->live_systems > 0) {
      ctx->set_error("systems still alive on this context");
      return SSRPA_ERR_STATE;
    }
  }
  delete ctx;
  return SSRPA_OK;
}

ssrpa_status ssrpa_context_memory(const ssrpa_context *ctx, size_t *in_use,
                                  size_t *high_water) {
  if (!ctx) return SSRPA_ERR_ARG;
  auto *c = const_cast<ssrpa_context *>(ctx);
  std::lock_guard<std::mutex> g(c->mu);
  if (in_use) *in_use = c->in_use + c->cached;
  if (high_water) *high_water = c->high_water;
  return SSRPA_OK;
}

ssrpa_status ssrpa_footprint(const ssrpa_system_desc *desc, int n_eig,
                             int n_freq, ssrpa_precision precision,
                             int valence_block, size_t *bytes) {
  if (!bytes) return SSRPA_ERR_ARG;
  return guarded(nullptr, [&] {
    const Geometry g = make_geometry(desc);
    SSRPA_REQUIRE(n_eig >= 1 && n_freq >= 1, SSRPA_ERR_ARG, "bad n_eig/n_freq");
    const int vb = valence_block > 0 ? std::min(valence_block, desc->n_v) : desc->n_v;
    *bytes = footprint_of(desc, g, n_eig, n_freq, vb, precision).total;
  });
}

ssrpa_status ssrpa_plan_valence_block(const ssrpa_system_desc *desc, int n_eig,
                                      int n_freq, ssrpa_precision precision,
                                      size_t budget_bytes, int *valence_block) {
  if (!valence_block) return SSRPA_ERR_ARG;
  *valence_block = 0;
  return guarded(nullptr, [&] {
    const Geometry g = make_geometry(desc);
    SSRPA_REQUIRE(n_eig >= 1 && n_freq >= 1, SSRPA_ERR_ARG, "bad n_eig/n_freq");
    int lo = 1, hi = desc->n_v, best = 0;
    while (lo <= hi) {
      const int mid = (lo + hi) / 2;
      if (footprint_of(desc, g, n_eig, n_freq, mid, precision).total <= budget_bytes) {
        best = mid;
        lo = mid + 1;
      } else {
        hi = mid - 1;
      }
    }
    SSRPA_REQUIRE(best >= 1, SSRPA_ERR_NOMEM,
                  "even one valence band per block exceeds %zu bytes", budget_bytes);
    *valence_block = best;
  });
}

ssrpa_status ssrpa_system_create(ssrpa_context *ctx, const ssrpa_system_desc *desc,
                                 void *hip_stream, ssrpa_system **out) {
  if (!ctx || !out) return SSRPA_ERR_ARG;
  *out = nullptr;
  ssrpa_system *sys = nullptr;
  hipStream_t s = Stream(hip_stream).s;
  ssrpa_status st = guarded(ctx, [&] {
    set_device(ctx);
    Geometry g = make_geometry(desc);
    // every host-side check and table comes first: no device work is queued
    // before the description has been accepted
    const int n_b = desc->n_v + desc->n_c;
    const BandSets bs = band_sets(desc);
    std::vector<double> energy(desc->energy, desc->energy + n_b);
    const size_t box = (size_t)g.n1 * g.n2 * g.n3;
    std::vector<int> bidx(desc->n_pw);
    for (int p = 0; p < desc->n_pw; ++p) {
      const int a = ((desc->miller[3 * p] % g.n1) + g.n1) % g.n1;
      const int b = ((desc->miller[3 * p + 1] % g.n2) + g.n2) % g.n2;
      const int c = ((desc->miller[3 * p + 2] % g.n3) + g.n3) % g.n3;
      bidx[p] = (c * g.n2 + b) * g.n1 + a;
    }
    {
      std::vector<char> seen(box, 0);
      for (int p = 0; p < desc->n_pw; ++p) {
        SSRPA_REQUIRE(!seen[bidx[p]], SSRPA_ERR_ARG, "duplicate plane wave %d", p);
        seen[bidx[p]] = 1;
      }
    }
    // real orbitals: the plane-wave set holds -G with every G
    std::vector<int> negpw;
    if (g.real) {
      SSRPA_REQUIRE(bs.n_cond >= 1, SSRPA_ERR_ARG, "no conduction band");
      std::vector<int> at(box, -1);
      for (int p = 0; p < desc->n_pw; ++p) at[bidx[p]] = p;
      negpw.resize(desc->n_pw);
      for (int p = 0; p < desc->n_pw; ++p) {
        const int a = ((-desc->miller[3 * p] % g.n1) + g.n1) % g.n1;
        const int b = ((-desc->miller[3 * p + 1] % g.n2) + g.n2) % g.n2;
        const int c = ((-desc->miller[3 * p + 2] % g.n3) + g.n3) % g.n3;
        negpw[p] = at[(c * g.n2 + b) * g.n1 + a];
        SSRPA_REQUIRE(negpw[p] >= 0, SSRPA_ERR_ARG,
                      "real orbitals: plane wave %d has no partner -G", p);
      }
    }
    // from here on device work is queued on s: a failure waits for it
    // before the host sources above and the buffers below are released
    ApiCall call(s);
    sys = new ssrpa_system();
    sys->ctx = ctx;
    sys->geo = std::move(g);
    sys->n_v = bs.n_val;
    sys->n_c = bs.n_cond;
    sys->c_first = bs.c_first;
    sys->partial = bs.partial;
    sys->real = sys->geo.real;
    sys->n_orb = sys->real ? bs.n_val + (bs.n_cond + 1) / 2 : n_b;
    sys->orb_c0 = sys->real ? bs.n_val : bs.c_first;
    sys->orb_nc = sys->real ? (bs.n_cond + 1) / 2 : bs.n_cond;
    sys->n_b = n_b;
    sys->n_pw = desc->n_pw;
    sys->energy = std::move(energy);
    const Geometry &gg = sys->geo;
    sys->energy_d = DevBuf(ctx, sizeof(double) * sys->n_b);
    SSRPA_HIP(hipMemcpyAsync(sys->energy_d.as(), sys->energy.data(),
                             sizeof(double) * sys->n_b, hipMemcpyHostToDevice, s));
    if (bs.partial) {
      sys->occ.assign(desc->occupation, desc->occupation + n_b);
      sys->occ_d = DevBuf(ctx, sizeof(double) * sys->n_b);
      SSRPA_HIP(hipMemcpyAsync(sys->occ_d.as(), sys->occ.data(),
                               sizeof(double) * sys->n_b, hipMemcpyHostToDevice, s));
    }
    upload_geometry(*sys, s);
    // orbital staging: coefficients -> psi(r)
    DevBuf bidx_d(ctx, sizeof(int) * sys->n_pw);
    SSRPA_HIP(hipMemcpyAsync(bidx_d.as(), bidx.data(), sizeof(int) * sys->n_pw,
                             hipMemcpyHostToDevice, s));
    const size_t cbytes = sizeof(double) * 2 * (size_t)sys->n_pw * sys->n_b;
    DevBuf coeff_d;
    const double *cptr = desc->coeff;
    if (!desc->coeff_on_device) {
      coeff_d = DevBuf(ctx, cbytes);
      SSRPA_HIP(hipMemcpyAsync(coeff_d.as(), desc->coeff, cbytes,
                               hipMemcpyHostToDevice, s));
      cptr = coeff_d.as<double>();
    }
    DevBuf packed;
    if (gg.real) {
      // check c(-G) = conj c(G) on the device, then pack two conduction
      // orbitals per complex orbital before the orbital FFT
      DevBuf chk(ctx, sizeof(int) * sys->n_pw + sizeof(double) * real_check_blocks());
      int *negd = chk.as<int>();
      double *bmax = reinterpret_cast<double *>(chk.as<char>() + sizeof(int) * sys->n_pw);
      SSRPA_HIP(hipMemcpyAsync(negd, negpw.data(), sizeof(int) * sys->n_pw,
                               hipMemcpyHostToDevice, s));
      real_check(cptr, sys->n_pw, sys->n_b, negd, bmax, s);
      std::vector<double> hb(real_check_blocks());
      SSRPA_HIP(hipMemcpyAsync(hb.data(), bmax, sizeof(double) * hb.size(),
                               hipMemcpyDeviceToHost, s));
      SSRPA_HIP(hipStreamSynchronize(s));
      double worst = 0.0;
      for (double x : hb) worst = std::max(worst, x);
      SSRPA_REQUIRE(worst <= 1e-10, SSRPA_ERR_ARG,
                    "real_orbitals = 1 but |c(-G) - conj c(G)| reaches %g", worst);
      packed = DevBuf(ctx, sizeof(double) * 2 * (size_t)sys->n_pw * sys->n_orb);
      pack_coefficients(cptr, sys->n_pw, sys->n_v, sys->c_first, sys->n_b,
                        sys->orb_nc, packed.as<double>(), s);
      cptr = packed.as<double>();
      // cos/sin basis tables
      std::vector<int> t;
      t.insert(t.end(), gg.hpos.begin(), gg.hpos.end());
      t.insert(t.end(), gg.hneg.begin(), gg.hneg.end());
      t.insert(t.end(), gg.neg.begin(), gg.neg.end());
      t.insert(t.end(), gg.hj.begin(), gg.hj.end());
      t.insert(t.end(), gg.hs.begin(), gg.hs.end());
      sys->rtab = DevBuf(ctx, sizeof(int) * t.size());
      SSRPA_HIP(hipMemcpyAsync(sys->rtab.as(), t.data(), sizeof(int) * t.size(),
                               hipMemcpyHostToDevice, s));
      std::vector<double> rsc(2 * (size_t)gg.n_g);
      for (int j = 0; j < gg.n_g; ++j) {
        const int gpos = gg.hpos[j < gg.nh ? j : j - gg.nh];
        rsc[j] = gg.store_scale[gpos];
        rsc[gg.n_g + j] = gg.rescale[gpos];
      }
      sys->rscale = DevBuf(ctx, sizeof(double) * rsc.size());
      SSRPA_HIP(hipMemcpyAsync(sys->rscale.as(), rsc.data(), sizeof(double) * rsc.size(),
                               hipMemcpyHostToDevice, s));
      SSRPA_HIP(hipStreamSynchronize(s));  // rsc and t are freed on return
    }
    sys->psi_r = DevBuf(ctx, bytes_c(box * sys->n_orb));
    launch_orbital_fft(*sys, cptr, bidx_d.as<int>(), s);
    SSRPA_HIP(hipStreamSynchronize(s));
  });
  if (st != SSRPA_OK) {
    if (sys) {
      // the system's own buffers may still be targets of queued copies
      (void)hipStreamSynchronize(s);
      delete sys;
    }
    return st;
  }
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->live_systems += 1;
  }
  *out = sys;
  return SSRPA_OK;
}

ssrpa_status ssrpa_system_destroy(ssrpa_system *sys) {
  if (!sys) return SSRPA_ERR_ARG;
  Context *ctx = sys->ctx;
  // every call on the system waited for its own device work before it
  // returned (a failed call included), so its buffers are idle here and go
  // back to the context's cache without a device-wide wait
  (void)hipSetDevice(ctx->device);
  delete sys;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->live_systems -= 1;
  return SSRPA_OK;
}

ssrpa_status ssrpa_system_bands(const ssrpa_system *sys, int *n_val,
                                int *c_first, int *n_cond) {
  if (!sys) return SSRPA_ERR_ARG;
  if (n_val) *n_val = sys->n_v;
  if (c_first) *c_first = sys->c_first;
  if (n_cond) *n_cond = sys->n_c;
  return SSRPA_OK;
}

ssrpa_status ssrpa_chi_gvectors(const ssrpa_system *sys, int *n_g,
                                int32_t *miller) {
  if (!sys || !n_g) return SSRPA_ERR_ARG;
  *n_g = sys->geo.n_g;
  if (miller)
    std::memcpy(miller, sys->geo.miller_chi.data(), sizeof(int32_t) * 3 * sys->geo.n_g);
  return SSRPA_OK;
}

ssrpa_status ssrpa_orbitals_realspace(ssrpa_system *sys, double *psi,
                                      void *hip_stream) {
  if (!sys || !psi) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    const size_t box = (size_t)sys->geo.n1 * sys->geo.n2 * sys->geo.n3;
    if (sys->real)
      unpack_orbitals(sys->psi_r.as<double>(), (long)box, sys->n_v, sys->c_first,
                      sys->n_b, psi, s);
    else
      copy_interleaved(sys->psi_r.as<double>(), psi, box * sys->n_b, s);
    SSRPA_HIP(hipStreamSynchronize(s));
  });
}

ssrpa_status ssrpa_pair_matrix(ssrpa_system *sys, int v0, int n_vb, int scaled,
                               double *m, void *hip_stream) {
  if (!sys || !m) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    SSRPA_REQUIRE(v0 >= 0 && n_vb >= 1 && v0 + n_vb <= sys->n_v, SSRPA_ERR_ARG,
                  "valence range [%d, %d) outside [0, %d)", v0, v0 + n_vb, sys->n_v);
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    const Geometry &g = sys->geo;
    const long rows = (long)n_vb * sys->n_c;
    DevBuf w(sys->ctx, sizeof(double) * 2 * (size_t)rows * g.ld_g);
    if (sys->real) {
      DevBuf f;
      packed_pairs(*sys, v0, n_vb, scaled != 0, f, s);
      unpack_pw_rows(f.as<double>(), n_vb, sys->n_c, g.ld_g, g.n_g,
                     sys->rtab.as<int>() + 2 * g.nh, w.as<double>(), s);
    } else {
      launch_pair_matrix(*sys, v0, n_vb, scaled != 0, w.as<double>(), s);
    }
    planar_to_interleaved(w.as<double>(), (int)rows, g.n_g, g.ld_g, m, s);
    SSRPA_HIP(hipStreamSynchronize(s));
  });
}

ssrpa_status ssrpa_chi0_static(ssrpa_system *sys, ssrpa_precision precision,
                               int valence_block, double *chi0, int symmetrized,
                               void *hip_stream) {
  if (!sys) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    SSRPA_REQUIRE(precision >= SSRPA_FP64 && precision <= SSRPA_BF16X3,
                  SSRPA_ERR_ARG, "unknown precision %d", (int)precision);
    SSRPA_REQUIRE(valence_block >= 0, SSRPA_ERR_ARG, "negative valence block");
    SSRPA_REQUIRE(!sys->real || precision == SSRPA_FP64, SSRPA_ERR_ARG,
                  "real-orbital systems contract in FP64 only");
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    const int vb = resolve_block(*sys, valence_block, 0, 1);
    if (vb < sys->n_v) {
      sys->w_cache.reset();
      sys->w_cache_valid = false;
    }
    static_chi0(*sys, precision, vb, s);
    if (chi0) {
      const Geometry &g = sys->geo;
      // the resident matrix is S chi0 S (S = diag s(G)), in the cos/sin
      // basis on the real path
      if (sys->real) {
        const int *t = sys->rtab.as<int>();
        real_to_pw_sym(sys->chibar0.as<double>(), g.n_g, g.nh, t + 2 * g.nh + g.n_g,
                       t + 2 * g.nh + 2 * g.n_g, chi0, s);
      } else {
        copy_interleaved(sys->chibar0.as<double>(), chi0, (size_t)g.n_g * g.n_g, s);
      }
      const double *tab = sys->sqrtv_d.as<double>() + 2 * (size_t)g.ld_g;
      if (!symmetrized)
        scale_sym(chi0, g.n_g, tab, 1, s);
      else if (g.rescaled)
        scale_sym(chi0, g.n_g, tab + g.n_g, 0, s);
      SSRPA_HIP(hipStreamSynchronize(s));
    }
  });
}

ssrpa_status ssrpa_subspace(ssrpa_system *sys, int n_eig, double *eigval,
                            double *basis, void *hip_stream) {
  return ssrpa_subspace_basis(sys, SSRPA_BASIS_SYMMETRIZED, n_eig, eigval,
                              basis, hip_stream);
}

ssrpa_status ssrpa_subspace_basis(ssrpa_system *sys, ssrpa_basis kind,
                                  int n_eig, double *eigval, double *basis,
                                  void *hip_stream) {
  if (!sys) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    compute_subspace(*sys, n_eig, (int)kind, s);
    if (eigval) std::memcpy(eigval, sys->sub.eigval.data(), sizeof(double) * n_eig);
    if (basis) {
      const Geometry &g = sys->geo;
      if (sys->real) {
        const int *t = sys->rtab.as<int>();
        real_basis_to_pw(sys->sub.basis.as<double>(), sys->sub.ld_e, g.n_g, n_eig,
                         g.nh, t + 2 * g.nh + g.n_g, t + 2 * g.nh + 2 * g.n_g,
                         basis, s);
      } else {
        planar_to_interleaved(sys->sub.basis.as<double>(), g.n_g, n_eig,
                              sys->sub.ld_e, basis, s);
      }
      SSRPA_HIP(hipStreamSynchronize(s));
    }
  });
}

ssrpa_status ssrpa_correlation_energy(ssrpa_system *sys, int n_eig, int n_freq,
                                      const double *omega, const double *weight,
                                      ssrpa_precision precision, int valence_block,
                                      double coupling, double *ec,
                                      double *integrand, double *chi_sub,
                                      void *hip_stream) {
  if (!sys || !ec) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    SSRPA_REQUIRE(precision >= SSRPA_FP64 && precision <= SSRPA_BF16X3,
                  SSRPA_ERR_ARG, "unknown precision %d", (int)precision);
    SSRPA_REQUIRE(n_eig >= 1, SSRPA_ERR_ARG, "n_eig must be >= 1");
    SSRPA_REQUIRE(std::isfinite(coupling), SSRPA_ERR_ARG, "bad coupling");
    SSRPA_REQUIRE(!sys->real || precision == SSRPA_FP64, SSRPA_ERR_ARG,
                  "real-orbital systems contract in FP64 only");
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    const int vb = resolve_block(*sys, valence_block, n_eig, n_freq);
    if (vb < sys->n_v) {
      sys->w_cache.reset();
      sys->w_cache_valid = false;
    }
    EcResult r = energy(*sys, n_eig, n_freq, omega, weight, precision, vb,
                        coupling, chi_sub, s);
    *ec = r.ec;
    if (integrand) std::memcpy(integrand, r.f.data(), sizeof(double) * n_freq);
  });
}

ssrpa_status ssrpa_epsilon_inverse(ssrpa_system *sys, int n_eig, int n_freq,
                                   const double *omega,
                                   ssrpa_precision precision, int valence_block,
                                   double *eps_inv, void *hip_stream) {
  if (!sys || !eps_inv || !omega) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    SSRPA_REQUIRE(precision >= SSRPA_FP64 && precision <= SSRPA_BF16X3,
                  SSRPA_ERR_ARG, "unknown precision %d", (int)precision);
    SSRPA_REQUIRE(n_eig >= 1 && n_freq >= 1, SSRPA_ERR_ARG, "bad sizes");
    SSRPA_REQUIRE(!sys->real || precision == SSRPA_FP64, SSRPA_ERR_ARG,
                  "real-orbital systems contract in FP64 only");
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    const int vb = resolve_block(*sys, valence_block, n_eig, n_freq);
    if (vb < sys->n_v) {
      sys->w_cache.reset();
      sys->w_cache_valid = false;
    }
    // X_j in the subspace (or the full basis), then (I - X_j)^-1 in place;
    // the quadrature weights do not matter here
    const int n = std::min(n_eig, sys->geo.n_g);
    std::vector<double> zero(n_freq, 0.0);
    DevBuf x(sys->ctx, bytes_c((size_t)n * n * n_freq));
    (void)energy(*sys, n_eig, n_freq, omega, zero.data(), precision, vb, 1.0,
                 x.as<double>(), s);
    fill_zero(sys->dev_flag.as(), sizeof(int), s);
    inverse_one_minus(sys->ctx, x.as<double>(), n, n_freq, 1.0, eps_inv,
                      sys->dev_flag.as<int>(), s);
    int flag = 0;
    SSRPA_HIP(hipMemcpyAsync(&flag, sys->dev_flag.as(), sizeof(int),
                             hipMemcpyDeviceToHost, s));
    SSRPA_HIP(hipStreamSynchronize(s));
    SSRPA_REQUIRE(flag == 0, SSRPA_ERR_NUMERIC,
                  "1 - chi0_s v is not positive definite at some frequency");
  });
}

ssrpa_status ssrpa_kmesh_create(ssrpa_context *ctx, int n_k,
                                const ssrpa_system_desc *descs,
                                const double *kfrac, const double *kweight,
                                void *hip_stream, ssrpa_kmesh **out) {
  if (!ctx || !out || !descs || !kfrac || !kweight || n_k < 1) return SSRPA_ERR_ARG;
  *out = nullptr;
  auto *km = new (std::nothrow) ssrpa_kmesh();
  if (!km) return SSRPA_ERR_NOMEM;
  km->ctx = ctx;
  ssrpa_status st = guarded(ctx, [&] {
    const ssrpa_system_desc &a = descs[0];
    for (int i = 0; i < n_k; ++i) {
      const ssrpa_system_desc &d = descs[i];
      SSRPA_REQUIRE(!d.occupation && !d.real_orbitals && !d.coulomb_truncation,
                    SSRPA_ERR_ARG,
                    "k meshes take insulators, complex orbitals and the bare Coulomb kernel");
      SSRPA_REQUIRE(d.n_v == a.n_v && d.n_c == a.n_c && d.ecut_chi == a.ecut_chi &&
                        d.coulomb_truncation == a.coulomb_truncation &&
                        std::memcmp(d.fft, a.fft, sizeof(a.fft)) == 0 &&
                        std::memcmp(d.lattice, a.lattice, sizeof(a.lattice)) == 0,
                    SSRPA_ERR_ARG, "k-point %d differs in cell, grid, cutoff or bands", i);
      SSRPA_REQUIRE(std::isfinite(kweight[i]) && kweight[i] >= 0.0, SSRPA_ERR_ARG,
                    "k weight %d must be non-negative", i);
      for (int c = 0; c < 3; ++c)
        SSRPA_REQUIRE(std::isfinite(kfrac[3 * i + c]), SSRPA_ERR_ARG, "bad k-point");
      for (int p = 0; p < d.n_pw; ++p)
        for (int c = 0; c < 3; ++c)
          km->mp[c] = std::max(km->mp[c], std::abs(d.miller[3 * p + c]));
    }
    SSRPA_REQUIRE(std::any_of(kweight, kweight + n_k, [](double w) { return w > 0.0; }),
                  SSRPA_ERR_ARG, "every k weight is zero");
    km->kfrac.assign(kfrac, kfrac + 3 * (size_t)n_k);
    km->kweight.assign(kweight, kweight + n_k);
    km->d0 = a;
    km->miller0.assign(a.miller, a.miller + 3 * (size_t)a.n_pw);
    km->d0.miller = km->miller0.data();
    km->d0.coeff = nullptr;
    km->d0.energy = nullptr;
    for (int i = 0; i < n_k; ++i) {
      ssrpa_system *sy = nullptr;
      const ssrpa_status s2 = ssrpa_system_create(ctx, &descs[i], hip_stream, &sy);
      if (s2 != SSRPA_OK) fail(s2, "k-point %d: %s", i, ctx->error().c_str());
      km->k.push_back(sy);
    }
  });
  if (st != SSRPA_OK) {
    for (auto *sy : km->k) ssrpa_system_destroy(sy);
    delete km;
    return st;
  }
  *out = km;
  return SSRPA_OK;
}

ssrpa_status ssrpa_kmesh_destroy(ssrpa_kmesh *km) {
  if (!km) return SSRPA_ERR_ARG;
  for (auto *sy : km->k) ssrpa_system_destroy(sy);
  delete km;
  return SSRPA_OK;
}

ssrpa_status ssrpa_kmesh_chi_gvectors(const ssrpa_kmesh *km, const double *q,
                                      int *n_g, int32_t *miller) {
  if (!km || !q || !n_g) return SSRPA_ERR_ARG;
  return guarded(km->ctx, [&] {
    ssrpa_system_desc d = km->d0;
    // the geometry reads the cell, grid, cutoff and G set only
    d.coeff = reinterpret_cast<const double *>(km->miller0.data());
    d.energy = d.coeff;
    const Geometry g = make_geometry(&d, q);
    *n_g = g.n_g;
    if (miller) std::memcpy(miller, g.miller_chi.data(), sizeof(int32_t) * 3 * g.n_g);
  });
}

ssrpa_status ssrpa_kmesh_correlation_energy(
    ssrpa_kmesh *km, const double *q, const int32_t *kq, const int32_t *g0,
    int n_eig, int n_freq, const double *omega, const double *weight,
    double *ec, double *integrand, double *chi0, void *hip_stream) {
  if (!km || !q || !kq || !g0 || !ec || !omega || !weight) return SSRPA_ERR_ARG;
  Context *ctx = km->ctx;
  const int n_k = (int)km->k.size();
  ssrpa_system *qs = nullptr;
  std::vector<DevBuf> shifted;
  hipStream_t s = Stream(hip_stream).s;
  ssrpa_status st = guarded(ctx, [&] {
    set_device(ctx);
    SSRPA_REQUIRE(n_eig >= 1 && n_freq >= 1, SSRPA_ERR_ARG, "bad sizes");
    int g0max[3] = {0, 0, 0};
    for (int i = 0; i < n_k; ++i) {
      if (km->kweight[i] == 0.0) continue;   // a k + q partner only
      SSRPA_REQUIRE(kq[i] >= 0 && kq[i] < n_k, SSRPA_ERR_ARG, "kq[%d] out of range", i);
      for (int c = 0; c < 3; ++c) {
        // k_i + q = k_kq[i] + g0[i]
        const double d = km->kfrac[3 * i + c] + q[c] - km->kfrac[3 * kq[i] + c] - g0[3 * i + c];
        SSRPA_REQUIRE(std::fabs(d) < 1e-9, SSRPA_ERR_ARG,
                      "k_%d + q is not k_%d + g0 (axis %d)", i, kq[i], c);
        g0max[c] = std::max(g0max[c], std::abs(g0[3 * i + c]));
      }
    }
    ssrpa_system_desc d = km->d0;
    // the geometry reads the cell, grid, cutoff and G set only
    d.coeff = reinterpret_cast<const double *>(km->miller0.data());
    d.energy = d.coeff;
    Geometry g = make_geometry(&d, q);
    // no aliasing: products of orbitals of two k-points read at G - g0
    const int nn[3] = {g.n1, g.n2, g.n3}, mc[3] = {g.m1, g.m2, g.m3};
    for (int c = 0; c < 3; ++c)
      SSRPA_REQUIRE(nn[c] >= 2 * km->mp[c] + mc[c] + g0max[c] + 1, SSRPA_ERR_ALIAS,
                    "FFT size %d along axis %d is below the bound %d at this q",
                    nn[c], c, 2 * km->mp[c] + mc[c] + g0max[c] + 1);
    ApiCall call(s);
    qs = new ssrpa_system();
    const ssrpa_system *k0 = km->k[0];
    qs->ctx = ctx;
    qs->geo = std::move(g);
    qs->n_v = k0->n_v;
    qs->n_c = k0->n_c;
    qs->c_first = k0->c_first;
    qs->n_b = k0->n_b;
    qs->n_orb = k0->n_b;
    qs->orb_c0 = k0->c_first;
    qs->orb_nc = k0->n_c;
    qs->timer.on = km->timer.on;
    upload_geometry(*qs, s);
    const Geometry &gg = qs->geo;
    const long box = (long)gg.n1 * gg.n2 * gg.n3;
    shifted.resize(n_k);
    for (int i = 0; i < n_k; ++i) {
      if (km->kweight[i] == 0.0) continue;
      const ssrpa_system *si = km->k[i], *sc = km->k[kq[i]];
      const double *pv = si->psi_r.as<double>();
      const int *gi = g0 + 3 * i;
      if (gi[0] || gi[1] || gi[2]) {
        // u_{k+q} = e^{-iG0.r} u_k': the phase goes on the valence side
        shifted[i] = DevBuf(ctx, 2 * sizeof(double) * box * si->n_v);
        phase_shift(si->psi_r.as<double>(), si->n_v, gg.n1, gg.n2, gg.n3, gi,
                    shifted[i].as<double>(), s);
        pv = shifted[i].as<double>();
      }
      qs->sources.push_back({pv, sc->psi_r.as<double>(), si->energy_d.as<double>(),
                             sc->energy_d.as<double>(), km->kweight[i]});
    }
    const int vb = resolve_block(*qs, 0, n_eig, n_freq);
    static_chi0(*qs, SSRPA_FP64, vb, s);
    if (chi0) {
      // the resident matrix is S chi0 S with S = diag v(G - q)^1/2
      copy_interleaved(qs->chibar0.as<double>(), chi0, (size_t)gg.n_g * gg.n_g, s);
      scale_sym(chi0, gg.n_g, qs->sqrtv_d.as<double>() + 2 * (size_t)gg.ld_g, 1, s);
    }
    if (n_eig < gg.n_g) compute_subspace(*qs, n_eig, SSRPA_BASIS_SYMMETRIZED, s);
    EcResult r = energy(*qs, n_eig, n_freq, omega, weight, SSRPA_FP64, vb, 1.0,
                        nullptr, s);
    *ec = r.ec;
    if (integrand) std::memcpy(integrand, r.f.data(), sizeof(double) * n_freq);
  });
  if (qs) {
    (void)hipStreamSynchronize(s);
    // the stage events outlive the per-q system
    auto &r = qs->timer.recs;
    km->timer.recs.insert(km->timer.recs.end(), r.begin(), r.end());
    r.clear();
    delete qs;
  }
  return st;
}

ssrpa_status ssrpa_device_copy(ssrpa_context *ctx, const void *src, void *dst,
                               size_t bytes, void *hip_stream) {
  if (!ctx) return SSRPA_ERR_ARG;
  return guarded(ctx, [&] {
    set_device(ctx);
    SSRPA_REQUIRE(src && dst && bytes % 16 == 0 &&
                      (reinterpret_cast<uintptr_t>(src) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(dst) & 15) == 0,
                  SSRPA_ERR_ARG, "copy needs 16-byte aligned pointers and sizes");
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    if (bytes) device_copy16(src, dst, bytes, s);
    SSRPA_HIP(hipStreamSynchronize(s));
  });
}

ssrpa_status ssrpa_kmesh_stage_times(ssrpa_kmesh *km, int enable, double *ms,
                                     int *launches) {
  if (!km) return SSRPA_ERR_ARG;
  return guarded(km->ctx, [&] {
    set_device(km->ctx);
    read_stage_times(km->timer, ms, launches);
    km->timer.clear();
    km->timer.on = enable != 0;
  });
}

ssrpa_status ssrpa_trace_log(ssrpa_context *ctx, const double *x, int n,
                             int n_mat, double coupling, double *f,
                             void *hip_stream) {
  if (!ctx || !x || !f) return SSRPA_ERR_ARG;
  return guarded(ctx, [&] {
    set_device(ctx);
    SSRPA_REQUIRE(n >= 1 && n_mat >= 1, SSRPA_ERR_ARG, "empty batch");
    hipStream_t s = Stream(hip_stream).s;
    ApiCall call(s);
    DevBuf fd(ctx, sizeof(double) * n_mat + 64);
    int *flag = reinterpret_cast<int *>(fd.as<double>() + n_mat);
    fill_zero(flag, sizeof(int), s);
    trace_log(ctx, x, n, n_mat, coupling, fd.as<double>(), flag, s);
    int hflag = 0;
    SSRPA_HIP(hipMemcpyAsync(f, fd.as(), sizeof(double) * n_mat,
                             hipMemcpyDeviceToHost, s));
    SSRPA_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    SSRPA_HIP(hipStreamSynchronize(s));
    SSRPA_REQUIRE(hflag == 0, SSRPA_ERR_NUMERIC,
                  "I - c X is not positive definite for some matrix");
  });
}

ssrpa_status ssrpa_trace_log_noalloc(ssrpa_context *ctx, const double *x,
                                     int n, int n_mat, double coupling,
                                     double *f, int *flag, void *hip_stream) {
  if (!ctx || !x || !f) return SSRPA_ERR_ARG;
  try {
    SSRPA_HIP(hipSetDevice(ctx->device));
    trace_log_noalloc(ctx->device, x, n, n_mat, coupling, f, flag,
                      Stream(hip_stream).s);
    return SSRPA_OK;
  } catch (...) {
    return finish(ctx, std::current_exception());
  }
}

ssrpa_status ssrpa_frequency_grid(int n, double omega0, double *omega,
                                  double *weight) {
  if (n < 1 || !(omega0 > 0.0) || !omega || !weight) return SSRPA_ERR_ARG;
  // Gauss-Legendre nodes by Newton's method on P_n, weights
  // 2 / ((1 - x^2) P_n'(x)^2); then the map to [0, inf).
  for (int i = 0; i < n; ++i) {
    long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0L; }
      dp = n * (x * p1 - p0) / (x * x - 1.0L);
      const long double dx = p1 / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    {
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0L; }
      dp = n * (x * p1 - p0) / (x * x - 1.0L);
    }
    const long double wx = 2.0L / ((1.0L - x * x) * dp * dp);
    // ascending order: node i of the loop is the (n-1-i)-th smallest
    const int o = n - 1 - i;
    omega[o] = (double)(omega0 * (1.0L + x) / (1.0L - x));
    weight[o] = (double)(2.0L * omega0 * wx / ((1.0L - x) * (1.0L - x)));
  }
  return SSRPA_OK;
}

ssrpa_status ssrpa_stage_times(ssrpa_system *sys, int enable, double *ms,
                               int *launches) {
  if (!sys) return SSRPA_ERR_ARG;
  return guarded(sys->ctx, [&] {
    set_device(sys->ctx);
    read_stage_times(sys->timer, ms, launches);
    sys->timer.clear();
    sys->timer.on = enable != 0;
  });
}

ssrpa_status ssrpa_correlation_energy_enqueue(ssrpa_system *sys, int n_eig,
                                              int n_freq, const double *omega,
                                              const double *weight,
                                              ssrpa_precision precision,
                                              int valence_block, void *hip_stream,
                                              ssrpa_ticket **ticket) {
  if (!sys || !ticket || !omega || !weight || n_freq < 1) return SSRPA_ERR_ARG;
  auto *t = new (std::nothrow) ssrpa_ticket();
  if (!t) return SSRPA_ERR_NOMEM;
  std::vector<double> om(omega, omega + n_freq), wt(weight, weight + n_freq);
  t->th = std::thread([=]() {
    ssrpa_status st = SSRPA_OK;
    double ec = 0.0;
    std::vector<double> f(n_freq);
    st = ssrpa_chi0_static(sys, precision, valence_block, nullptr, 1, hip_stream);
    if (st == SSRPA_OK && n_eig < sys->geo.n_g)
      st = ssrpa_subspace(sys, n_eig, nullptr, nullptr, hip_stream);
    if (st == SSRPA_OK)
      st = ssrpa_correlation_energy(sys, n_eig, n_freq, om.data(), wt.data(),
                                    precision, valence_block, 1.0, &ec, f.data(),
                                    nullptr, hip_stream);
    t->status = st;
    t->ec = ec;
    t->f = std::move(f);
    t->done.store(1);
  });
  *ticket = t;
  return SSRPA_OK;
}

ssrpa_status ssrpa_ticket_query(ssrpa_ticket *t, int *done) {
  if (!t || !done) return SSRPA_ERR_ARG;
  *done = t->done.load();
  return SSRPA_OK;
}

ssrpa_status ssrpa_ticket_wait(ssrpa_ticket *t, double *ec, double *integrand) {
  if (!t) return SSRPA_ERR_ARG;
  if (t->th.joinable()) t->th.join();
  const ssrpa_status st = t->status;
  if (ec) *ec = t->ec;
  if (integrand && !t->f.empty())
    std::memcpy(integrand, t->f.data(), sizeof(double) * t->f.size());
  delete t;
  return st;
}

}  // extern "C"
