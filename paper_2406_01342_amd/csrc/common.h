// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/polyclean.h"

namespace pc {

// ----------------------------------------------------------------------------
// Errors: thrown inside the library, converted to pc_status at the ABI.
// ----------------------------------------------------------------------------
struct Error : std::runtime_error {
  pc_status status;
  Error(pc_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void fail(pc_status s, const std::string& msg);
void set_last_error(const std::string& msg);

#define PC_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      ::pc::fail(e_ == hipErrorOutOfMemory ? PC_ERR_OUT_OF_MEMORY : PC_ERR_DEVICE, \
                 std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

#define PC_LAUNCH_CHECK(name)                                                     \
  do {                                                                            \
    hipError_t e_ = hipGetLastError();                                            \
    if (e_ != hipSuccess)                                                         \
      ::pc::fail(PC_ERR_DEVICE, std::string("launch ") + name + ": " +            \
                                    hipGetErrorString(e_));                       \
  } while (0)

#define PC_REQUIRE(cond, msg)                                                     \
  do {                                                                            \
    if (!(cond)) ::pc::fail(PC_ERR_INVALID_ARG, msg);                             \
  } while (0)

// ----------------------------------------------------------------------------
// Complex value types (interleaved, matching complex64 / complex128 buffers).
// ----------------------------------------------------------------------------
// Aligned to its own size, so that a complex value moves in one 64-bit (FP32)
// or 128-bit (FP64) access: LDS then serves a wave's consecutive elements
// without bank conflicts, where two 32-bit halves at an 8-byte stride
// conflicted two ways.
template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R x, y;
};
using c32 = cpx<float>;
using c64 = cpx<double>;

// Spreading tile side in fine-grid cells.  A visibility's footprint (w <= 16
// cells) therefore touches at most the next tile along each axis.
constexpr int kTile = 32;
constexpr int kMaxWidth = 16;

// Spreading register window: a wave's lanes cover a spread_span(W)-wide
// square of cells, the union of the footprints of all visibilities whose
// first cell lies in one spread_block(W)-wide square block.  The plan sorts
// visibilities by that block within each tile.
__host__ __device__ constexpr int spread_span(int W) { return W <= 8 ? 8 : W; }
__host__ __device__ constexpr int spread_block(int W) { return spread_span(W) - W + 1; }

// One spreading work item: an output tile plus the (sub)ranges of sorted
// visibilities that reach it from the tile itself and from its left, upper
// and upper-left neighbours.  slot >= 0 means the tile is split across
// several items and this item writes partial tile `slot`.  FP32 plans with
// kernel widths up to 8 group items by kSpreadQuad, one workgroup of that many
// waves per group: either independent items (combine = 0; tile = -1 marks an
// empty one), or shares of one tile's visibilities (combine = 1, same tile and
// slot) whose LDS tiles the workgroup adds in a fixed order before the single
// write.  Two waves per workgroup (31 KB of LDS) let five workgroups share a
// compute unit, ten waves against the eight that four-wave groups (62 KB)
// allow.
struct SpreadChunk {
  int32_t tile;
  int32_t slot;
  int32_t beg[4];
  int32_t end[4];
  int32_t combine;
  int32_t pad;
};
constexpr int kSpreadQuad = 2;  // waves (items) per workgroup of the grouped spread

// Interpolation work item: the plan-order visibilities [beg, end) whose first
// cells lie in `tile` (a tile's own visibilities, in chunks of at most
// kInterpChunk).
struct InterpItem {
  int32_t tile;
  int32_t beg;
  int32_t end;
  int32_t pad;
};
constexpr int kInterpChunk = 2048;

// A split ("hot") tile: its partial tiles occupy slots [first, first+count).
struct FoldItem {
  int32_t tile;
  int32_t first;
  int32_t count;
  int32_t pad;
};

// Device-side geometry of the fine grid band, passed by value to kernels.
struct GridGeom {
  int32_t n;       // image side
  int32_t M;       // fine grid side
  int32_t W;       // kernel width
  float beta;      // kernel shape
  double beta64;
  int32_t u0, nu;  // band origin / extent along u (cells, multiple of kTile)
  int32_t v0, nv;  // band along v
  int32_t ntu, ntv;
  int32_t wrap;
  double dl;       // pixel step (direction cosine)
};

struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// One active atom of a sparse image: pixel offsets from the phase centre
// (a = i - n/2, b = j - n/2), 1/n(l, m), c = n(l, m) - 1 (the w-term's
// direction factor, <= 0) and the forward weight x / n(l, m).
template <typename R>
struct Atom {
  double a, b;
  double inv_n;
  double c;
  R w;
  R pad;
};

// c = n - 1 = -(l^2 + m^2) / (1 + n), without the
// cancellation of sqrt(1 - r^2) - 1 near the phase centre.
__host__ __device__ inline double n_minus_one(double l, double m) {
  const double r2 = l * l + m * m;
  return -r2 / (1.0 + sqrt(1.0 - r2));
}

// Planes of the w-stacked gridded adjoint (non-coplanar baselines).  The
// factor exp(+2 pi i w_k c) of Eq. adjoint-phi is split as
// exp(2 pi i w_k c_mid) exp(2 pi i w_k c'), c' = c - c_mid in
// [-half, half]; the second factor is spread over planes w_j = w0 + j dw with
// the same ES kernel along w (width W, plane units), so that
//   exp(2 pi i w_k c') ~ sum_j psi((w_k - w_j) / dw) exp(2 pi i w_j c') / Psi(dw c'),
// Psi the kernel's Fourier transform; dw = 1 / (4 half) keeps |dw c'| <= 1/4,
// the band the kernel is designed for at upsampling 2.
struct WStack {
  int nplanes = 0;  // 0: coplanar plan
  double w0 = 0, dw = 0;
  double cmid = 0;
  int nquad = 0;    // Gauss-Legendre nodes on [0, 1] of the Psi integral
};
// Terms of the Chebyshev series of Psi that the w-stacked adjoint's final
// division evaluates (the plan checks the series against the quadrature).
constexpr int kPsiCheb = 40;

// Everything the gridded adjoint's kernels need about one plan, for launches
// that cover the work of several plans at once (FP32 plans).
struct AdjJob {
  GridGeom g;
  const SpreadChunk* chunks;
  const FoldItem* fold;
  const uint8_t* flags;
  const uint32_t* cell;
  const float* off;
  const cpx<float>* vals;
  const int32_t* perm;
  cpx<float>* grid;
  cpx<float>* partials;
  cpx<float>* H;
  float* image;
  const cpx<float>* tw;
  const float* corr;
  float scale;
  int positive;  // max key of max(eta, 0) instead of |eta|
  unsigned long long* maxkey;
  // always NULL (full images), read at run time so that the batched passes
  // compile to the same code as the single-plan ones (bitwise equal results)
  const uint32_t* rows;
};

// Per-kernel instrumentation (optional): launches bracketed by HIP events on
// the launch stream, accumulated per kernel name with the algorithmic bytes
// and work units (visibility-atom pairs, FFT points, ...) of each launch.
struct KStat {
  std::string name;
  int64_t launches = 0;
  double ms = 0, bytes = 0, work = 0;
};

struct Prof {
  bool on = false;
  std::vector<KStat> stats;
  struct Pending {
    int idx;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

}  // namespace pc

// The opaque plan.
struct pc_plan {
  int device = 0;
  int precision = PC_PREC_FP32;
  int64_t L = 0;
  pc::GridGeom g{};
  int64_t n_chunks = 0, n_partials = 0, n_fold = 0, n_interp = 0;
  bool spread_quads = false;  // work items grouped by workgroup (FP32, kernel width <= 8)
  size_t footprint = 0;

  // Per-visibility data in plan (tile-sorted) order.
  int32_t* perm = nullptr;      // sorted index -> caller index
  double* AB = nullptr;         // [2L] (u dl, v dl) turns per pixel, FP64
  double* Cw = nullptr;         // [L] w in wavelengths (NULL: coplanar plan)
  uint32_t* cell = nullptr;     // [L] packed first cell (v << 16 | u), absolute
  void* off = nullptr;          // [2L] float or double: (s_u, s_v) offsets
  // Spreading work list.
  pc::SpreadChunk* chunks = nullptr;
  pc::FoldItem* fold = nullptr;
  uint8_t* tile_flags = nullptr;  // [ntv * ntu]: 1 if the tile holds data
  pc::InterpItem* interp = nullptr;  // interpolation work list
  // Fine grid band, pass-A output, split-tile partials.
  void* grid = nullptr;         // complex [nv][nu]
  void* H = nullptr;            // complex [nv][n]
  void* partials = nullptr;     // complex [n_partials][kTile][kTile]
  // Tables.
  void* twiddle = nullptr;      // complex [M]: exp(+2 pi i t / M)
  void* corr = nullptr;         // real [n]: (-1)^a / psi(a), a = i - n/2
  // Small scratch.
  unsigned long long* maxkey = nullptr;  // packed (|x| bits, ~index)
  uint32_t* rowmask = nullptr;  // a caller's row mask (after the max key)
  int max_positive = 0;  // the key holds max(x, 0) in place of |x| (positivity-constrained solve)
  void* vis_scratch = nullptr;  // complex [L] in plan order (residual etc.)
  pc::WStack ws;                // w-stacking planes (nplanes 0: coplanar)
  void* wvals = nullptr;        // complex [L]: one plane's weighted visibilities
  double* wquad = nullptr;      // [2 nquad] doubles: Psi's Chebyshev series (kPsiCheb terms)
  void* atom_scratch = nullptr; // per-atom staging
  size_t atom_capacity = 0;
  double* red_scratch = nullptr;  // reduction partials
  size_t red_capacity = 0;
  void* image_scratch = nullptr;  // [n][n] float (adjoint image before Psi*)
  size_t image_capacity = 0;
  void* key_scratch = nullptr;    // per-workgroup max keys of the Psi* tiles
  size_t key_capacity = 0;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  pc::Prof prof;
  std::vector<int32_t> chunk_work;  // host copy: visibilities per spreading workgroup

  std::vector<pc::DeviceBuf> owned;
  std::vector<std::pair<hipStream_t, hipEvent_t>> touched;  // see plan_touch
};

namespace pc {

// profile.cpp
struct ProfScope {
  pc_plan* p;
  hipStream_t s;
  const char* name;
  double bytes, work;
  hipEvent_t a = nullptr;
  ProfScope(pc_plan* plan, hipStream_t stream, const char* kname, double b, double w);
  ~ProfScope();
};
void prof_flush(pc_plan* p);
void prof_reset(pc_plan* p);
void prof_release(pc_plan* p);

// plan.cpp
// Per-device pool of device buffers.  Released buffers (a destroyed plan's,
// a finished solver's, scratch that grew) are kept for reuse instead of being
// passed to hipFree, which waits for the whole device: in a serving loop every
// job's end would otherwise drain the other jobs' work.  Buffers are pooled
// by size class (a power of two times 1, 1.25, 1.5 or 1.75, at most 25 %
// slack) up to an eighth of the device's memory; beyond that they are freed.
// pool_trim frees every pooled buffer of a device (returns the bytes).
// The releaser guarantees that no pending work still uses a released buffer.
void* pool_alloc(int device, size_t bytes, size_t* got);
void pool_release(int device, void* ptr, size_t bytes);
size_t pool_class(size_t bytes);
size_t pool_trim(int device);
// Work of a plan's entry points is followed by an event on the call's stream
// (one per stream the plan has seen); destroying the plan waits for these
// events only.
void plan_touch(pc_plan* p, hipStream_t s);
void* dalloc(pc_plan* p, size_t bytes);
void plan_release(pc_plan* p);
void* ensure_atom_scratch(pc_plan* p, size_t bytes);
double* ensure_red_scratch(pc_plan* p, size_t count);
float* ensure_image_scratch(pc_plan* p);  // n^2 floats, grown on first use
unsigned long long* ensure_key_scratch(pc_plan* p, size_t count);  // per-workgroup max keys

// Synthesis dictionary of Gaussian elements (Sect. 4.3; the elements of
// Sect. 6.4): g_s[a][b] = gamma_s t_s[a] t_s[b], t_s the unit-sum 1-D
// Gaussian taps exp(-a^2 / sigma_s^2) of half-width h_s = floor(2 sigma_s)
// (h_s = 0, t = {1}: a single pixel).  Passed to kernels by value.
constexpr int kDictMaxScales = 8;
constexpr int kDictMaxHalf = 32;  // sigma <= 16
constexpr int kDictMaxTaps = 2 * kDictMaxHalf + 1;
struct DictSpec {
  int S;
  int h[kDictMaxScales];
  float gamma[kDictMaxScales];
  float taps[kDictMaxScales][kDictMaxTaps];
};
// Validates sigma/gamma (fails with PC_ERR_INVALID) and fills the taps in FP64
// rounded once to FP32.
DictSpec make_dict(int n_scales, const double* sigma, const double* gamma);
// out[s][i][j] = sum_{a,b} g_s[a][b] img[i + a][j + b] (zero outside), the
// adjoint of the cropped synthesis, with the fused maximum key of |out| (of
// max(out, 0) with positive) over the flat index s n^2 + i n + j in *key.
void dict_analysis(pc_plan* p, const DictSpec& D, const float* img, float* out, bool positive,
                   unsigned long long* key, hipStream_t s);
// img += sum_q w_q g_{s_q} centred on p_q (atoms[q] = s_q n^2 + p_q), cropped.
void dict_synthesis(pc_plan* p, const DictSpec& D, int64_t nS, const int32_t* atoms,
                    const double* w, float* img, hipStream_t s);
// out[q] = (Psi* img)[atoms[q]] in FP64 (the analysis at the active atoms).
void dict_gather(pc_plan* p, const DictSpec& D, int64_t nS, const int32_t* atoms,
                 const float* img, double* out, hipStream_t s);

// kernels_grid.hip
// Image rows taking part in a gridded operator: bit i % 32 of bits[i / 32]
// set for row i (ceil(n / 32) words on the device), count = rows set.  For
// the forward, rows whose bit is clear must be zero and are not read; for
// the adjoint, only the rows set are computed (the others are left as they
// were, and no maximum is formed).
struct RowMask {
  const uint32_t* bits;
  int64_t count;
};
constexpr int kMaxRowWords = 8192 / 32;  // npix <= 8192
template <typename R>
void adjoint_grid(pc_plan* p, const cpx<R>* vis, bool vis_sorted, R* image, R scale,
                  hipStream_t s, const RowMask* rows = nullptr);
// With base (plan order; out_sorted, FP32): vis_out = base - Phi image, and
// with stats (2 p->n_interp doubles) the per-work-item sums of |vis_out|^2
// and Re(conj(base) vis_out), to be summed in order (k_resid_final).
template <typename R>
void forward_grid(pc_plan* p, const R* image, cpx<R>* vis_out, bool out_sorted,
                  hipStream_t s, const RowMask* rows = nullptr, const cpx<R>* base = nullptr,
                  double* stats = nullptr);
// The gridded operators of an APGD step over an active set S (FP32,
// coplanar): its atoms sorted by pixel (pix, nS), the occupied image rows
// (rowlist: row, first atom, end; nrows) and their mask.  Pass B is
// evaluated directly at those rows (forward) or atoms (adjoint), pass A with
// the mask.  forward_grid_set: out (plan order) = base - Phi_S w (Phi_S w
// without base), stats as forward_grid's.  adjoint_grid_set: gout[q] =
// (Phi* vis)[pix[q]] in FP64, vis in plan order.
struct AtomSet {
  int64_t nS;
  const int32_t* pix;
  const int3* rowlist;
  int64_t nrows;
  RowMask rows;
};
void forward_grid_set(pc_plan* p, const AtomSet& as, const double* w, const c32* base,
                      double* stats, c32* out, hipStream_t s);
void adjoint_grid_set(pc_plan* p, const c32* vis, const AtomSet& as, double* gout,
                      hipStream_t s);
// Phi_S* (V - Phi_S x) by the set operators above, atoms in caller order
// (any order, repeats allowed); vis, resid caller order; synchronises.
void restricted_gradient_grid(pc_plan* p, const c32* vis, int64_t natoms, const int32_t* pix,
                              const float* weight, double* grad, c32* resid, hipStream_t s);
void maxkey_read(pc_plan* p, hipStream_t s, double* max_abs, int64_t* argmax);
// Launch tables of the batched adjoint (device copy and pinned staging),
// reused from call to call.
struct BatchCtx {
  unsigned char* dev = nullptr;
  size_t dev_bytes = 0;
  unsigned char* host = nullptr;
  size_t host_bytes = 0;
  hipEvent_t done = nullptr;  // completion of the last call's launches
  bool pending = false;
  void release();
};
// Residuals r = V - Phi_S x of several FP32 plans (direct sums, plan order)
// in one launch over (job, block of 256 visibilities) items; each job rounds
// exactly as forward_atoms does.  Same ctx rules as adjoint_grid_batch.
struct FwdJob {
  const double* AB;
  const double* Cw;  // NULL: coplanar
  const Atom<float>* atoms;
  const cpx<float>* base;
  cpx<float>* out;
  int64_t L;
  int64_t natoms;
};
void forward_residual_batch(BatchCtx& ctx, const std::vector<FwdJob>& jobs, hipStream_t s);
// Restricted adjoints with FP64 totals (adjoint_atoms_acc64) of several
// coplanar FP32 plans in shared launches over (job, workgroup) and (job,
// atom) items, each job rounding exactly as adjoint_atoms_acc64 does: out =
// Phi_S* vis (vis in plan order, or NULL for unit visibilities, the
// point-spread sums); partial holds adjoint_partial_count(p, natoms) doubles
// of the job's own.  Same ctx rules as adjoint_grid_batch.
struct AccJob {
  const pc_plan* p;
  const Atom<float>* atoms;
  int64_t natoms;
  const cpx<float>* vis;
  double* partial;
  double* out;
};
void adjoint_acc64_batch(BatchCtx& ctx, const std::vector<AccJob>& jobs, hipStream_t s);
// Gridded adjoints of several FP32 plans in shared launches (one spread per
// kernel width, one fold, one launch per fine-grid size for each FFT pass).
// vis[j] is in plan order when vis_sorted[j], else in caller order.  The
// plans' max keys hold each image's maximum afterwards.  Calls on one ctx
// must not overlap; the function waits for the previous call's launches
// before it rewrites the tables.
void adjoint_grid_batch(BatchCtx& ctx, pc_plan* const* plans, const c32* const* vis,
                        const bool* vis_sorted, float* const* images, const float* scales, int n,
                        hipStream_t s);
void maxkey_decode(unsigned long long key, double* max_abs, int64_t* argmax);

// batcher.cpp: gridded adjoint of one job through a batcher, which merges
// the requests of jobs on other host threads into shared launches.  Blocks
// until the job's image and maximum are ready; `ms` gets the duration of the
// shared launches.
// With fwd, the residual vis_sorted = fwd->base - Phi_S x (direct sums over
// fwd's atom table) is formed first, in a launch shared with the other
// requests of the batch that carry one.
struct FwdSpec {
  const Atom<float>* atoms;
  int64_t natoms;
  const cpx<float>* base;  // plan order
};
void batcher_adjoint(pc_batcher* b, pc_plan* p, const c32* vis_sorted, float* image,
                     hipStream_t s, double* max_abs, int64_t* argmax, float* ms,
                     const FwdSpec* fwd = nullptr);
// The restricted adjoints `sums` (plan p, work ordered after stream s) in the
// batcher's shared launches; returns when they are done.
void batcher_restricted_adjoints(pc_batcher* b, pc_plan* p, hipStream_t s,
                                 const std::vector<AccJob>& sums);

// kernels_dft.hip
template <typename R>
void forward_sparse(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                    const cpx<R>* vis_base, bool base_sorted, cpx<R>* out, bool out_sorted,
                    hipStream_t s);
template <typename R>
void adjoint_sparse(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                    const int32_t* pix, double* out, hipStream_t s);
// Entries of an atom table for natoms atoms: rounded up to a multiple of 8,
// the padding being zero-weight atoms (the fused pass reads whole groups).
inline int64_t atom_capacity(int64_t natoms) {
  return (std::max<int64_t>(natoms, 1) + 7) / 8 * 8;
}
// Variants on a prepared atom table (the solver keeps one per active set).
// prep_atoms_into fills atom_capacity(natoms) entries.
template <typename R>
void prep_atoms_into(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                     Atom<R>* atoms, hipStream_t s);
template <typename R>
void forward_atoms(pc_plan* p, int64_t natoms, const Atom<R>* atoms, const cpx<R>* vis_base,
                   bool base_sorted, cpx<R>* out, bool out_sorted, hipStream_t s);
template <typename R>
void adjoint_atoms(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                   const Atom<R>* atoms, double* partial, double* out, hipStream_t s);
// Restricted adjoint of plan-order visibilities with FP64 accumulation of the
// FP32 terms (partial: adjoint_partial_count doubles); out[p] in FP64.  vis
// NULL: every visibility is 1 (the point-spread sums, cosines only).
void adjoint_atoms_acc64(pc_plan* p, const cpx<float>* vis, int64_t natoms,
                         const Atom<float>* atoms, double* partial, double* out, hipStream_t s);
template <typename R>
void reduce_partials(pc_plan* p, int64_t natoms, int64_t nwg, const double* partial,
                     const Atom<R>* atoms, double* out, hipStream_t s);
// Forward and restricted adjoint in one pass for 1..64 atoms (FP32):
// r = base - Phi_S w (or Phi_S w when base is NULL), written to r_out when
// given, and the partial sums of Phi_S* r, fused_partial_stride() per atom.
bool fused_supported(int64_t natoms);
int64_t fused_partial_stride(const pc_plan* p, int64_t natoms);
void forward_adjoint_atoms(pc_plan* p, int64_t natoms, const Atom<float>* atoms,
                           const cpx<float>* base, cpx<float>* r_out, double* partial,
                           hipStream_t s, bool caller_order = false);
// g = Phi_S* (V - Phi_S x) with r = V - Phi_S x optionally returned (caller
// order throughout); one pass for 1..64 atoms, else forward then adjoint.
void restricted_gradient(pc_plan* p, const cpx<float>* vis, int64_t natoms, const int32_t* pix,
                         const float* weight, double* out, cpx<float>* resid, hipStream_t s);
// The same with the atom table and partial sums in a fixed per-device array of
// kNoAllocScratchBytes (no device allocation); fails with PC_ERR_UNSUPPORTED
// when restricted_gradient_scratch_bytes exceeds it.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
constexpr int kNoAllocMaxDevices = 64;
size_t restricted_gradient_scratch_bytes(const pc_plan* p, int64_t natoms);
void restricted_gradient_noalloc(pc_plan* p, const cpx<float>* vis, int64_t natoms,
                                 const int32_t* pix, const float* weight, double* out,
                                 cpx<float>* resid, hipStream_t s);
int64_t adjoint_partial_count(const pc_plan* p, int64_t natoms);
// Partials per atom of adjoint_atoms (out == NULL leaves them unsummed).
int64_t adjoint_partial_stride(const pc_plan* p, int64_t natoms);
// Sum of the restricted adjoint's partials (or g_in) fused with one APGD
// step; see kernels_dft.hip.
void reduce_fista(pc_plan* p, int64_t nS, int64_t nwg, const double* partial, const double* g_in,
                  Atom<float>* atoms, double* x, double* y, double* g_out, double* stat,
                  double inv_lip, double thr, double mom, bool positive, hipStream_t s);

}  // namespace pc
