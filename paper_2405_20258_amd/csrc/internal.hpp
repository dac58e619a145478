// Internal declarations of the ssrpa library: runtime objects, device buffer
// ownership and the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ssrpa.h"

namespace ssrpa {

// Error carried from deep inside the runtime to the C ABI boundary, where it
// becomes a status code plus the context's last-error text.
struct Error : std::runtime_error {
  ssrpa_status code;
  Error(ssrpa_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(ssrpa_status code, const char *fmt, ...);

#define SSRPA_HIP(expr)                                                       \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      ::ssrpa::fail(SSRPA_ERR_HIP, "%s failed at %s:%d: %s", #expr, __FILE__, \
                    __LINE__, hipGetErrorString(e_));                         \
  } while (0)

#define SSRPA_REQUIRE(cond, code, ...)              \
  do {                                              \
    if (!(cond)) ::ssrpa::fail((code), __VA_ARGS__); \
  } while (0)

struct Context;

// The HIP stream of the library call running on this thread.  Device work
// of a call is queued on that stream; a call that fails part-way unwinds its
// device buffers while such work may still be queued, so a buffer released
// during exception unwinding first waits for this stream (ApiCall sets it).
struct ApiStream {
  hipStream_t s = nullptr;
  bool set = false;
};
ApiStream &api_stream();
void sync_api_stream_on_unwind();
struct ApiCall {
  ApiStream prev;
  explicit ApiCall(hipStream_t s) : prev(api_stream()) {
    api_stream().s = s;
    api_stream().set = true;
  }
  ~ApiCall() {
    sync_api_stream_on_unwind();
    api_stream() = prev;
  }
};

// Device allocation charged against a context's HBM budget; freed on
// destruction.  Move-only.
class DevBuf {
 public:
  DevBuf() = default;
  DevBuf(Context *ctx, size_t bytes);
  ~DevBuf();
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept { swap(o); }
  DevBuf &operator=(DevBuf &&o) noexcept {
    DevBuf t(std::move(o));
    swap(t);
    return *this;
  }
  void swap(DevBuf &o) noexcept {
    std::swap(ctx_, o.ctx_);
    std::swap(ptr_, o.ptr_);
    std::swap(bytes_, o.bytes_);
  }
  template <class T = void>
  T *as() const { return static_cast<T *>(ptr_); }
  size_t bytes() const { return bytes_; }
  bool empty() const { return ptr_ == nullptr; }
  void reset() { DevBuf t; swap(t); }
  // Grow to at least `bytes` (contents discarded when reallocated).  Work
  // queued on `s` may still use the old block, and a freed block can be
  // handed to another request's stream at once, so `s` is drained first.
  void ensure(Context *ctx, size_t bytes, hipStream_t s) {
    if (bytes_ < bytes || ctx_ != ctx) {
      if (ptr_) SSRPA_HIP(hipStreamSynchronize(s));
      reset();
      *this = DevBuf(ctx, bytes);
    }
  }

 private:
  Context *ctx_ = nullptr;
  void *ptr_ = nullptr;
  size_t bytes_ = 0;
};

// A context owns the device memory budget.  Freed blocks are cached (every
// library call synchronizes its stream before its buffers go out of scope,
// so a returned block is idle) and reused by later allocations; this keeps
// hipFree, which synchronizes the whole device, out of the steady state
// where several requests run concurrently.  budget caps live + cached bytes.
struct Context {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;       // bytes in live allocations
  size_t cached = 0;       // bytes in cached free blocks
  size_t high_water = 0;   // peak of in_use
  int live_systems = 0;    // systems created on this context and not destroyed
  std::multimap<size_t, void *> free_blocks;
  uint64_t release_gen = 0; // counts releases (wakes allocations that wait)
  std::mutex mu;           // guards everything above
  std::condition_variable cv_release;
  void *alloc(size_t bytes);
  void release(void *p, size_t bytes);
  void set_error(const std::string &m);
  std::string error();
  // move cached blocks to `victims` (to be freed) until `need` fits
  void trim_locked(size_t need, std::vector<void *> &victims);
  ~Context();
  std::map<void *, size_t> sizes_;  // live allocations and their block sizes
};

// Geometry of the real-space grid and the chi0 G set, derived once per system.
struct Geometry {
  double lattice[9];
  double recip[9];   // rows b1, b2, b3 with a_i . b_j = 2 pi delta_ij
  double volume;
  int n1, n2, n3;
  int m1, m2, m3;    // max |n_i| over the chi0 set
  int n_g;           // chi0 basis size
  int ld_g;          // n_g rounded up to a multiple of 64 (zero padded)
  std::vector<int32_t> miller_chi;  // n_g x 3
  std::vector<double> sqrt_v;       // v(G)^1/2 per chi0 vector
  // The pair rows are stored scaled by s(G) = v(G)^1/2, except where v(G)
  // is (nearly) zero under a truncated kernel: there s = 1 and the stored
  // matrices are brought to v^1/2 (...) v^1/2 by r(G) = v^1/2 / s.
  // Bare kernel: s = v^1/2, r = 1, rescaled = false.
  std::vector<double> store_scale, rescale;
  bool rescaled = false;
  int truncation = 0;
  bool q_zero = true;   // q = 0: G = 0 left out of the set
  // Real-orbital path: the cos/sin basis.  nh = n_g / 2 pairs {G, -G};
  // hpos[j] / hneg[j] = indices of the larger member G of pair j and of -G;
  // per G: neg = index of -G, hj = its pair, hs = +1 (G = H) or -1.
  bool real = false;
  int nh = 0;
  std::vector<int> hpos, hneg, neg, hj, hs;
  // Columns (n1, n2) that hold chi0 vectors, in order of first appearance:
  // cmap[(n1 + m1) * (2 m2 + 1) + n2 + m2] = column or -1; per G,
  // zcode = column | (n3 mod N3) << 20.  ldy = ncol rounded up to 8.
  // zcol[4 col ..] = (first G of the column, lowest n3, highest n3, 1 for
  // the (0, 0) column, whose n3 = 0 member G = 0 is left out, else 0).
  int ncol = 0, ldy = 0;
  std::vector<int> cmap, zcode, zcol;
};

// Staged pair transform (fft.hip): the pair x-y stage holds n3 * ldy complex
// values per pair and is processed in chunks of at most kStageBytes.
constexpr size_t kStageBytes = size_t(4) << 30;
inline size_t stage_bytes_per_pair(const Geometry &g) {
  return (size_t)g.n3 * g.ldy * 16;
}
// Conduction bands per chunk of a block of nvb valence bands.
inline int stage_chunk_c(int nvb, int n_c, size_t ypp) {
  const size_t per_c = (size_t)nvb * ypp;
  size_t c = kStageBytes / (per_c ? per_c : 1);
  if (c >= (size_t)n_c) return n_c;
  c = c >= 8 ? c / 8 * 8 : (c ? c : 1);
  return (int)c;
}
// true when the staged kernels cover the grid (N1 = N2 with a compiled
// split); other grids use the fused generic kernel, which needs no stage.
bool staged_grid(const Geometry &g);

// Event timing of the stages (ssrpa_stage_times).
struct StageTimer {
  bool on = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  // record the start of a stage on stream s; returns an index for stop()
  int start(int stage, hipStream_t s);
  void stop(int idx, hipStream_t s);
  void clear();
  ~StageTimer() { clear(); }
};

// RAII stage scope: records events only when the timer is on.
struct StageScope {
  StageTimer *t;
  hipStream_t s;
  int idx;
  StageScope(StageTimer &tm, int stage, hipStream_t st)
      : t(&tm), s(st), idx(tm.on ? tm.start(stage, st) : -1) {}
  ~StageScope() { if (idx >= 0) t->stop(idx, s); }
};

// Resident subspace state after ssrpa_subspace.
struct Subspace {
  int n_eig = 0;
  int ld_e = 0;                  // n_eig rounded up to 64
  std::vector<double> eigval;    // host copy, ascending
  DevBuf basis;                  // planar rows: ld_g rows x [re(ld_e) | im(ld_e)]
  DevBuf basis_r;                // rows scaled by r(G) (truncated kernel only)
  // basis kind: 0 eigenvectors of v^1/2 chi0 v^1/2, 1 eigenvectors of chi0
  int kind = 0;
  // kind 1: B = S^-1 C_s Z with v_s = C_s^H v C_s = Z Z^H, the operand of
  // the projection (planar, like basis)
  DevBuf proj;
  // operand of the projection W_s = W_stored (operand)
  const double *projection() const {
    if (kind == 1) return proj.as<double>();
    return (basis_r.empty() ? basis : basis_r).as<double>();
  }
};

// Valence and conduction sets of a description (Method, Eqs. 4-6): bands
// [0, n_val) have f > 0, bands [c_first, n_b) have f < 1; they overlap in
// the partially occupied bands [c_first, n_val).  Insulator: c_first = n_val.
struct BandSets {
  int n_val = 0, c_first = 0, n_cond = 0;
  bool partial = false;
};
// Validate the occupations (or their absence) and energies of a description.
BandSets band_sets(const ssrpa_system_desc *d);

struct System {
  Context *ctx = nullptr;
  Geometry geo;
  // n_v: valence set size; n_c: conduction set size (pair columns);
  // c_first: band index of conduction column 0 (n_v for an insulator)
  int n_v = 0, n_c = 0, n_b = 0, n_pw = 0, c_first = 0;
  bool partial = false;          // partially occupied bands present
  // Orbitals held in psi_r (n_orb of them) and where the pair transform
  // finds its conduction columns: orb_nc orbitals from index orb_c0.
  // Complex orbitals: n_orb = n_b, orb_c0 = c_first, orb_nc = n_c.  Real
  // orbitals: the valence set unpacked, then the conduction set packed two
  // per complex orbital: n_orb = n_v + orb_nc, orb_c0 = n_v,
  // orb_nc = (n_c + 1) / 2.
  int n_orb = 0, orb_c0 = 0, orb_nc = 0;
  // When set, the pair transform takes valence orbital v from src_psi_v + v
  // and conduction orbital orb_c0 + c from src_psi_c (the pair sources of a
  // k mesh at q); otherwise both from psi_r.
  // (complex interleaved grids)
  const double *src_psi_v = nullptr, *src_psi_c = nullptr;
  bool real = false;             // real-orbital (cos/sin basis) path
  // real path tables (ints): hpos, hneg (nh each), neg, hj, hs (n_g each)
  DevBuf rtab;
  // real path: s(G) and r(G) in the order of the cos/sin basis (n_g each)
  DevBuf rscale;
  std::vector<double> energy;
  std::vector<double> occ;       // host occupation factors (partial only)
  DevBuf energy_d;               // n_b doubles
  DevBuf occ_d;                  // n_b doubles (partial only)
  DevBuf rowscale;               // per pair row (f_v - f_c)^1/2 (partial only)
  DevBuf psi_r;                  // n_b x N3 x N2 x N1 complex (interleaved)
  DevBuf gcol;                   // per G: int (column index | n3 mod N3 << 20)
  DevBuf zcode, cmap, zcol;      // Geometry::zcode / cmap / zcol on the device
  DevBuf ystage;                 // x-y stage of the staged pair transform
  // per-G scale tables: [0, ld_g) s(G) Omega/N, [ld_g, 2 ld_g) Omega/N,
  // then s(G) (n_g) and r(G) (n_g)
  DevBuf sqrtv_d;
  DevBuf fft_tw;                 // twiddle tables for N1, N2, N3
  std::vector<double> fft_tw_host;  // their source (kept for the async copy)
  DevBuf chibar0;                // n_g x n_g complex (interleaved), symmetrized
  bool have_chi0 = false;
  Subspace sub;
  // Pair matrix of the last block when a single block covers all valence
  // bands: reused by the second pass (the pair FFTs then run once).
  DevBuf w_cache;
  int w_cache_prec = -1;
  bool w_cache_valid = false;
  // Device-side error flag (non-positive pivot, etc.): int.
  DevBuf dev_flag;
  std::vector<int> code_host;      // sources of the per-G table copies
  std::vector<double> scale_host;
  // Pair sources of a k mesh at q (empty: the system's own pairs).  Each
  // adds the rows of valence orbitals psi_v (energies e_v) against
  // conduction orbitals c_first.. of psi_c (energies e_c), weight g_k.
  struct PairSource {
    const double *psi_v, *psi_c;   // complex interleaved grids
    const double *e_v, *e_c;
    double weight;
  };
  std::vector<PairSource> sources;
  StageTimer timer;
};

// ---------------------------------------------------------------------------
// Kernel launchers (all enqueue on `s`, never synchronize).
// ---------------------------------------------------------------------------

// FFT stage (fft.hip)
void upload_twiddles(System &sys, hipStream_t s);
// psi_r <- orbitals on the grid; box_index_dev[pw] = linear grid index of
// the plane wave's Miller triple (mod N).
void launch_orbital_fft(System &sys, const double *coeff_dev,
                        const int *box_index_dev, hipStream_t s);
// Pair matrix for valence bands [v0, v0+nvb): W rows p = (v - v0) * n_c + c,
// planar layout: row stride 2*ld_g doubles, re at [0, ld_g), im at
// [ld_g, 2 ld_g); the padding columns are written as zeros.
// scaled: multiply by v(G)^1/2 (else plain M).
void launch_pair_matrix(System &sys, int v0, int nvb, bool scaled, double *w,
                        hipStream_t s);

// Contractions (gemm.hip)
struct HerkArgs {
  const double *a;     // planar rows, row stride lda doubles, im at +im_off
  long lda;
  long im_off;
  int ncol;            // output dimension (G or eigen index), <= ld (pad 64)
  int ld;              // padded ncol (multiple of 64)
  long k;              // rows (pairs)
  const double *de;    // per row: e_c - e_v
  const double *omega; // per output matrix: imaginary frequency
  int n_omega;
  double wscale;       // multiplies Delta (1/Omega)
  int unit_weight;     // 1: weights all 1 (Gram matrices), ignore de/omega
  StageTimer *timer = nullptr;  // optional: time the contraction kernel
  int stage = 0;
};
// out_j (+)= A^H diag(d_j) A for every j, written as full Hermitian
// ncol x ncol interleaved complex matrices at out + j * out_stride (doubles).
// beta: 0 overwrite, 1 accumulate.
// ws: caller-owned workspace for split-K partial tiles (grown as needed).
void herk(Context *ctx, const HerkArgs &h, ssrpa_precision prec, double *out,
          long out_stride, int beta, DevBuf &ws, hipStream_t s);
// FP32 and BF16x3 forms of herk (gemm_mixed.hip): rows scaled by
// sqrt|d| and converted once per K chunk, 128 x 128 MFMA Gram tiles; herk
// dispatches to it.  herk_gram_workspace: bytes of ws it needs.
void herk_gram(Context *ctx, const HerkArgs &h, ssrpa_precision prec,
               double *out, long out_stride, int beta, DevBuf &ws,
               hipStream_t s);
size_t herk_gram_workspace(const HerkArgs &h, ssrpa_precision prec);
// Bytes of ws an FP64 herk call needs (its split-K partial tiles).
size_t herk_f64_workspace(const HerkArgs &h);
// C = alpha * A * B + beta * C for complex planar operands:
//   A: m x k rows (row stride lda, im at +a_im), B: k x n (row stride ldb,
//   im at +b_im), C: m x n (row stride ldc, im at +c_im).  k is a multiple of
//   64 (zero padded), n is padded to 64 in all three operands.
struct GemmArgs {
  const double *a; long lda; long a_im;
  const double *b; long ldb; long b_im;
  double *c; long ldc; long c_im;
  long m; int n; int k;
  double alpha, beta;
};
// ws: caller-owned workspace (the BF16x3 path splits B into it; kept alive
// by the caller until the stream is synchronized).
void gemm(Context *ctx, const GemmArgs &g, ssrpa_precision prec, DevBuf &ws,
          hipStream_t s);
// BF16x3 GEMM with 128 x 128 tiles (gemm_mixed.hip), beta = 0.
void gemm_bf16x3_wide(Context *ctx, const GemmArgs &g, DevBuf &ws,
                      hipStream_t s);
size_t gemm_bf16x3_wide_workspace(const GemmArgs &g);
void gemm_f32_wide(Context *ctx, const GemmArgs &g, DevBuf &ws, hipStream_t s);
size_t gemm_f32_wide_workspace(const GemmArgs &g);

// Real-orbital path (real.hip)
// X_w = A^T diag(d_w) A for real A (h.a rows of h.lda doubles; h.ld a
// multiple of 128), written as interleaved complex with imaginary part 0.
void syrk(Context *ctx, const HerkArgs &h, double *out, long out_stride,
          int beta, DevBuf &ws, hipStream_t s);
size_t syrk_f64_workspace(const HerkArgs &h);
// C = A B for real row-major operands; k, n multiples of 128.
void gemm_real(const double *a, long lda, const double *b, long ldb, double *c,
               long ldc, long m, int k, int n, hipStream_t s);
void pack_coefficients(const double *coeff, int n_pw, int nv, int c0, int n_b,
                       int n_pack, double *out, hipStream_t s);
void unpack_real_rows(const double *f, int nvb, int n_c, int ld, int nh,
                      const int *hpos, const int *hneg, double *w,
                      hipStream_t s);
void unpack_pw_rows(const double *f, int nvb, int n_c, int ld, int n_g,
                    const int *neg, double *m, hipStream_t s);
void real_to_pw_sym(const double *cr, int n, int nh, const int *hj,
                    const int *hs, double *out, hipStream_t s);
void real_basis_to_pw(const double *x, int ld_e, int n_g, int n_eig, int nh,
                      const int *hj, const int *hs, double *y, hipStream_t s);
void unpack_orbitals(const double *psi, long box, int nv, int c0, int n_b,
                     double *out, hipStream_t s);
int real_check_blocks();
void real_check(const double *coeff, int n_pw, int n_b, const int *negpw,
                double *blockmax, hipStream_t s);


// Eigensolver (eig.hip): n_eig most negative eigenpairs of a Hermitian n x n
// interleaved matrix (not modified).  eigval: device (n_eig); basis: planar
// rows (ld_rows >= n rows, row stride 2*ld_e, im at +ld_e), padded rows/cols
// zero.
// Bytes of the Householder reduction's work buffer for an n x n matrix
// (besides the n x n work copy), for the footprint model.
size_t eig_workspace_bytes(int n);
void eig_lowest(Context *ctx, const double *a, int n, int n_eig, double *eigval,
                double *basis, int ld_e, int *flag, hipStream_t s);

// Log-determinants (chol.hip): f[j] = ln det(I - c X_j) + c Tr X_j for
// interleaved n x n Hermitian X_j at x + j*n*n; f device (n_mat).  Sets
// *flag (device int) nonzero on a non-positive pivot.
void trace_log(Context *ctx, const double *x, int n, int n_mat, double coupling,
               double *f, int *flag, hipStream_t s);
// out_j = (I - c X_j)^-1 for Hermitian X_j (device, n x n interleaved each);
// *flag (device int) set nonzero where I - c X_j is not positive definite.
void inverse_one_minus(Context *ctx, const double *x, int n, int n_mat,
                       double coupling, double *out, int *flag, hipStream_t s);
// Allocation-free trace_log: work memory in a fixed per-device array of
// kNoAllocScratchBytes (no allocator call); f and flag (nullable) are device
// memory; nothing is synchronized.  noalloc_setup(device) looks the array's
// address up once per device, with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
void noalloc_setup(int device);
size_t trace_log_noalloc_bytes(int n, int n_mat);
void trace_log_noalloc(int device, const double *x, int n, int n_mat,
                       double coupling, double *f, int *flag, hipStream_t s);
// ec[0] = (1/2pi) sum_j w[j] f[j]   (device scalars)
void quadrature(const double *w, const double *f, int n, double *ec,
                hipStream_t s);

// Layout helpers (util.hip)
void fill_zero(void *p, size_t bytes, hipStream_t s);
// interleaved n x n Hermitian, scaled elementwise by s_i s_j
void scale_sym(double *x, int n, const double *sv, int inverse, hipStream_t s);
// planar rows (row stride 2*ld, im at +ld) -> interleaved rows x cols
void planar_to_interleaved(const double *src, int rows, int cols, int ld,
                           double *dst, hipStream_t s);
// de[p] = e_c - e_v for the rows p = (v - v0) n_c + c of a block, band
// c_first + c as conduction band.  With occupations (occ != nullptr), rows
// that do not count (v >= c band, or f_v = f_c) get de = 1 and, when
// rowscale != nullptr, rowscale[p] = (f_v - f_c)^1/2, 0 for those rows.
void pair_energy_diffs(const double *energy, const double *occ, int c_first,
                       int v0, int nvb, int n_c, double *de, double *rowscale,
                       hipStream_t s);
// de[p] = e_c[c_first + c] - e_v[v0 + v] for a block of a pair source.
void pair_energy_diffs2(const double *e_v, const double *e_c, int c_first,
                        int v0, int nvb, int n_c, double *de, hipStream_t s);
// dst = src times e^{+iG0.r} on the grid, n_b orbitals (umklapp shift).
void phase_shift(const double *src, long n_b, int n1, int n2, int n3,
                 const int *g0, double *dst, hipStream_t s);
// Scale column j < ncol of planar rows (stride 2 ld) by f[j], or by
// sqrt(max(f[j], 0)) when from_eigs.
void scale_cols(double *w, long rows, int ld, int ncol, const double *f,
                int from_eigs, hipStream_t s);
// Scale each planar row (2 ld doubles) of w by rowscale[p] (by its
// reciprocal when inverse).
void scale_rows(double *w, long rows, int ld, const double *rowscale,
                hipStream_t s, bool inverse = false);
// Plain streaming copy of `bytes` (a multiple of 16, 16-byte aligned
// pointers) with 16-byte loads and stores.
void device_copy16(const void *src, void *dst, size_t bytes, hipStream_t s);
void copy_interleaved(const double *src, double *dst, size_t n_complex,
                      hipStream_t s);

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace ssrpa

// The opaque handles of the C ABI are the runtime objects themselves.
struct ssrpa_context : ssrpa::Context {};
struct ssrpa_system : ssrpa::System {};
