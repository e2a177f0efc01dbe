// Polyatomic Frank-Wolfe LASSO solve (paper Sect. 5.1, Alg. 2) on the GPU.
//
//   eta_0 = Phi* V, lambda_max = ||eta_0||_inf (Eq. lmax), lambda = alpha
//   lambda_max (Eq. lambda), Delta = (1 - delta) lambda_max.
//   for k = 0, 1, ...
//     I  = { j : |eta_k|_j >= ||eta_k||_inf - 2 Delta / (k + 2) }   (1.a)
//     S  = S u I                                                    (1.b)
//     x  = APGD on the LASSO restricted to S, warm-started          (2)
//     S  = supp(x)                                                  (3)
//     r  = V - Phi x, eta_{k+1} = Phi* r, objective and duality gap (4)
//
// Precision: the operator applications (gridded adjoint, direct sparse
// forward and restricted adjoint) are FP32 with FP64 phases; the APGD
// iterates, the step size (power iteration), the objective and the duality
// gap are FP64.  The restricted solve stops when the relative duality gap
// of the restricted problem at the gradient point y is <= tau_k =
// max(tau_min, tau_0 g_k), g_k the full problem's relative gap at the current
// iterate (tested at every step when steps are expensive, else at steps 1,
// 1 + kCheck, ...), returning the proximal step
// taken from y, or at the iteration cap.  Duality gaps use the dual point
// nu = min(1, lambda / ||Phi* r||_inf) r.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <limits>
#include <unordered_map>

#include "common.h"
#include "solver_kernels.h"

namespace pc {

template <typename T>
struct DevArray {
  T* ptr = nullptr;
  int64_t cap = 0;
  size_t bytes = 0;
  int dev = -1;
  void ensure(int64_t n) {
    if (n <= cap && ptr) return;
    int64_t want = std::max<int64_t>(n, std::max<int64_t>(2 * cap, 256));
    // growth mid-solve: queued work may still read the old array, which
    // hipFree waits for
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    PC_HIP(hipGetDevice(&dev));
    size_t got = 0;
    ptr = static_cast<T*>(pool_alloc(dev, want * sizeof(T), &got));
    bytes = got;
    cap = (int64_t)(got / sizeof(T));
  }
  // to the device pool: the owner has waited for its stream (see ~Pfw)
  ~DevArray() { pool_release(dev, ptr, bytes); }
};

// Device FP64 table that keeps its contents when it grows (the old entries
// are copied on the stream before the old allocation is released).
struct KeepDevArray {
  double* ptr = nullptr;
  int64_t cap = 0;
  size_t bytes = 0;
  int dev = -1;
  void ensure(int64_t n, hipStream_t s) {
    if (n <= cap && ptr) return;
    const int64_t want = std::max<int64_t>(n, std::max<int64_t>(2 * cap, 1024));
    PC_HIP(hipGetDevice(&dev));
    size_t got = 0;
    double* np = static_cast<double*>(pool_alloc(dev, want * sizeof(double), &got));
    if (ptr) {
      PC_HIP(hipMemcpyAsync(np, ptr, cap * sizeof(double), hipMemcpyDeviceToDevice, s));
      PC_HIP(hipStreamSynchronize(s));
      pool_release(dev, ptr, bytes);  // the copy above was its last use
    }
    ptr = np;
    bytes = got;
    cap = (int64_t)(got / sizeof(double));
  }
  ~KeepDevArray() { pool_release(dev, ptr, bytes); }
};

constexpr int kCheck = 4;        // APGD convergence test cadence (cheap steps)
// Direct-sum steps over more visibility-atom pairs than this (about 170 us)
// are tested every step, as are gridded ones: the test's reduction and host
// round trip are then small against a step.
constexpr double kCheckEveryPairs = 5e8;
constexpr int64_t kFirstCandidates = 4096;  // candidates read back with their count
// Pinned host staging for uploads and small readbacks.  Its copies are
// asynchronous; `fence` records the stream position of the last use so that
// the buffer is not rewritten while a copy from it may still be pending.
struct Pinned {
  unsigned char* ptr = nullptr;
  size_t cap = 0;
  hipEvent_t fence = nullptr;
  bool armed = false;
  void* get(size_t bytes) {
    if (armed) PC_HIP(hipEventSynchronize(fence));
    armed = false;
    if (bytes > cap) {  // grow geometrically: pinning memory is slow
      const size_t want = std::max<size_t>(bytes, 2 * cap + 4096);
      if (ptr) (void)hipHostFree(ptr);
      ptr = nullptr;
      cap = 0;
      PC_HIP(hipHostMalloc((void**)&ptr, want));
      cap = want;
    }
    return ptr;
  }
  void arm(hipStream_t s) {
    if (!fence) PC_HIP(hipEventCreateWithFlags(&fence, hipEventDisableTiming));
    PC_HIP(hipEventRecord(fence, s));
    armed = true;
  }
  ~Pinned() {
    if (fence) {
      if (armed) (void)hipEventSynchronize(fence);
      (void)hipEventDestroy(fence);
    }
    if (ptr) (void)hipHostFree(ptr);
  }
};

constexpr int kLanczosMax = 12;       // Lanczos steps per active set (cap)
constexpr int kLanczosBatch = 4;      // device steps between host readbacks (cheap steps;
                                      // one when a step is expensive, see kCheckEveryPairs)
constexpr int kGramAtoms = 256;       // default cap of the Gram form (direct sets)
constexpr int kGramChunk = 8;         // Gram-form APGD steps per readback after the first chunk: 2x
constexpr int kGramNewPairs = 16;     // new sums per atom above which the Gram form is skipped
constexpr double kLanczosTol = 1e-2;  // residual bound relative to the estimate
constexpr double kLipMargin = 1.01;

// Largest eigenvalue and its eigenvector of a small symmetric matrix A
// (row-major k x k, overwritten) by cyclic Jacobi rotations.
static double sym_top_eigen(std::vector<double>& A, int k, std::vector<double>& vec) {
  std::vector<double> V((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double q = A[(size_t)i * k + j] * A[(size_t)i * k + j];
        tot += q;
        if (i != j) off += q;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < k; ++r) {  // A <- A J (columns p, q)
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {  // A <- J^T A (rows p, q)
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {  // V <- V J
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = c * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + c * vrq;
        }
      }
  }
  int best = 0;
  for (int i = 1; i < k; ++i)
    if (A[(size_t)i * k + i] > A[(size_t)best * k + best]) best = i;
  vec.resize(k);
  for (int i = 0; i < k; ++i) vec[i] = V[(size_t)i * k + best];
  return A[(size_t)best * k + best];
}

// The plan's fused maximum reports max(eta, 0) for the length of one of a
// positivity-constrained solve's adjoints (a plan serves one solve at a time;
// outside them it reports max |eta|).
struct PositiveMax {
  pc_plan* p;
  PositiveMax(pc_plan* plan, bool on) : p(plan) { p->max_positive = on ? 1 : 0; }
  ~PositiveMax() { p->max_positive = 0; }
};

struct Pfw {
  pc_plan* p;
  hipStream_t s;
  pc_batcher* batcher = nullptr;  // shared-launch adjoints when set
  pc_solve_params prm;
  int64_t L, N;
  DevArray<c32> V, r;
  DevArray<float> eta;
  DevArray<float> dimg;  // dense image of the dictionary's synthesis (kept zero)
  DevArray<int32_t> cand, pix;
  DevArray<unsigned> cand_count;
  DevArray<Atom<float>> atoms;
  DevArray<double> x, y, g, adj_partial, red_partial, scal, stat;
  DevArray<double> lz_Q, lz_w, lz_ab;  // Lanczos basis rows, scratch, alpha/beta
  DevArray<double> lz_out;             // Gram form: {L, steps, theta, rho}, Ritz vector
  // Gram form of the restricted problem: G = Re(Phi_S^H Phi_S) and b = Phi_S^* V.
  // For coplanar arrays G_pq = psf(a_p - a_q, b_p - b_q) / (n_p n_q) with
  // psf(da, db) = sum_k cos 2 pi (A_k da + B_k db), kept per solve by offset.
  // The point-spread sums and b_p stay on the device, in tables indexed by
  // slot; the host keeps the slot of every offset and pixel seen in this
  // solve, and the slot table of the last G (pairs of atoms both there keep
  // theirs), so that G is gathered on the device without a readback.
  std::unordered_map<uint64_t, int32_t> psf_slot;
  std::unordered_map<int32_t, int32_t> b_slot;  // by pixel
  std::vector<int32_t> g_set;                   // the set of the last G, and its slots
  std::vector<int32_t> g_slots;
  KeepDevArray psf_dev, b_dev;
  int64_t n_psf = 0, n_b = 0;
  DevArray<double> gram_blk, psf_partial, asm_blk;
  double *gram_G = nullptr, *gram_b = nullptr, *gram_Q = nullptr;  // inside gram_blk
  DevArray<int> gram_done;  // {passed, step} of the device-side gap test
  int last_inner = 1 + kCheck;  // APGD steps of the last Gram-form solve
  int last_lanczos = 0;         // Lanczos steps of the last step-size estimate
  // candidates of the next exploration selected with step 4's readback
  std::vector<int32_t> pre_I;
  int pre_k = -1;
  bool pre_ok = false;
  DevArray<double> act_blk;  // uploaded [x | pix | row mask] of the active set
  RowMask act_rows{nullptr, 0};  // image rows holding atoms (inside act_blk)
  const int3* act_rowlist = nullptr;  // per occupied row: row, first atom, end
  int64_t act_nrows = 0;
  // partial residual statistics left in red_partial by the last op_forward
  // (its interpolation's work items), 0 when it left none
  int64_t resid_parts = 0;
  DevArray<Atom<float>> off_atoms;
  DevArray<double> b_partial;  // partials of b's sums when batched beside the psf sums
  double v2 = 0;  // ||V||^2
  Pinned up, up_act, down;  // upload staging (Gram form, active set), small readbacks
  std::vector<int32_t> S;
  std::vector<double> xs;
  std::vector<int32_t> pv_set;  // last power-iteration eigenvector (warm start)
  std::vector<double> pv_val;
  double lam = 0, lmax = 0, Delta = 0, eta_inf = 0, P_prev = 0, P = 0, rel_gap = 0, gap = 0;
  int64_t eta_argmax = -1;
  int k = 0, inner_total = 0;
  int64_t grid_thr = 0;  // active-set size from which APGD uses gridded operators
  bool done = false, converged = false;
  bool positive = false;  // x >= 0: signed exploration, one-sided prox and dual scaling
  // Synthesis dictionary (n_scales > 0): atoms s N + p are the columns of
  // Phi Psi; exploration on Psi* eta, APGD through the gridded operators.
  bool ms = false;
  DictSpec dict{};
  int64_t NA = 0;          // atoms in the dictionary (N without one)
  DevArray<float> eta_ms;  // Psi* eta, [S][n][n]
  double adj_ms = 0;
  int adj_calls = 0;
  double t0 = 0;

  // The arrays go back to the device pool after this: wait for the solve's
  // stream first (its own work only, not the whole device).
  ~Pfw() { (void)hipStreamSynchronize(s); }

  Pfw(pc_plan* plan, hipStream_t stream, const pc_solve_params& params)
      : p(plan), s(stream), prm(params), L(plan->L), N((int64_t)plan->g.n * plan->g.n),
        positive(params.positivity != 0), ms(params.n_scales > 0) {
    NA = N;
    if (ms && p->Cw)
      fail(PC_ERR_UNSUPPORTED, "a synthesis dictionary needs a coplanar plan (w = 0)");
    if (ms) {
      dict = make_dict(params.n_scales, params.scale_sigma, params.scale_gamma);
      NA = (int64_t)dict.S * N;
      PC_REQUIRE(NA < ((int64_t)1 << 31), "n_scales * npix^2 must be < 2^31");
    }
    if (params.x0_n > 0) {  // atoms index images on the device: checked here
      std::vector<int32_t> px(params.x0_pix, params.x0_pix + params.x0_n);
      std::sort(px.begin(), px.end());
      PC_REQUIRE(px.front() >= 0 && (int64_t)px.back() < NA,
                 "x0_pix must lie in [0, npix^2) (times n_scales with a dictionary)");
      PC_REQUIRE(std::adjacent_find(px.begin(), px.end()) == px.end(),
                 "x0_pix must not repeat an atom");
    }
  }

  // The exploration image: eta, or Psi* eta with its maximum (which then
  // replaces eta's) under a dictionary.
  float* expl() { return ms ? eta_ms.ptr : eta.ptr; }
  void ms_explore_sync() {
    dict_analysis(p, dict, eta.ptr, eta_ms.ptr, positive, p->maxkey, s);
    maxkey_read(p, s, &eta_inf, &eta_argmax);  // synchronises
  }

  static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
  }

  void adjoint_timed(const c32* vis_sorted, const FwdSpec* fwd = nullptr) {
    PositiveMax pm(p, positive);
    if (batcher) {
      float ms = 0;
      batcher_adjoint(batcher, p, vis_sorted, eta.ptr, s, &eta_inf, &eta_argmax, &ms, fwd);
      adj_ms += ms;
      adj_calls++;
      if (this->ms) ms_explore_sync();
      return;
    }
    PC_HIP(hipEventRecord(p->ev_a, s));
    adjoint_grid<float>(p, vis_sorted, true, eta.ptr, 1.0f, s);
    PC_HIP(hipEventRecord(p->ev_b, s));
    if (this->ms) dict_analysis(p, dict, eta.ptr, eta_ms.ptr, positive, p->maxkey, s);
    double mx;
    int64_t am;
    maxkey_read(p, s, &mx, &am);  // synchronises
    float ms = 0;
    PC_HIP(hipEventElapsedTime(&ms, p->ev_a, p->ev_b));
    adj_ms += ms;
    adj_calls++;
    eta_inf = mx;
    eta_argmax = am;
  }

  // Step 4's dirty residual together with ||r||^2 and Re<V, r>: one host
  // synchronisation for the maximum, the argmax and both statistics.
  // (Off the batcher, the exploration of iteration k_next is selected on the
  // device right after this adjoint, from its maximum, and its candidates come
  // back with the statistics: one host synchronisation for both.)
  void adjoint_and_stats(const c32* vis_sorted, double& r2, double& vr, int k_next) {
    pre_ok = false;
    if (batcher) {  // the batcher synchronises on its own
      adjoint_timed(vis_sorted);
      residual_stats(r2, vr);
      return;
    }
    PositiveMax pm(p, positive);
    PC_HIP(hipEventRecord(p->ev_a, s));
    adjoint_grid<float>(p, vis_sorted, true, eta.ptr, 1.0f, s);
    PC_HIP(hipEventRecord(p->ev_b, s));
    if (ms) dict_analysis(p, dict, eta.ptr, eta_ms.ptr, positive, p->maxkey, s);
    red_partial.ensure(2 * k_resid_blocks(L));
    k_resid(p, L, r.ptr, V.ptr, red_partial.ptr, scal.ptr + kScalResid, s);
    k_select_from_key(p, NA, expl(), p->maxkey, 2.0 * Delta / (k_next + 2), positive,
                      cand_count.ptr, cand.ptr, cand.cap, s);
    const int64_t first = std::min<int64_t>(kFirstCandidates, cand.cap);
    unsigned char* h = (unsigned char*)down.get(28 + first * 4);
    PC_HIP(hipMemcpyAsync(h, p->maxkey, 8, hipMemcpyDeviceToHost, s));
    PC_HIP(hipMemcpyAsync(h + 8, scal.ptr + kScalResid, 16, hipMemcpyDeviceToHost, s));
    PC_HIP(hipMemcpyAsync(h + 24, cand_count.ptr, 4, hipMemcpyDeviceToHost, s));
    PC_HIP(hipMemcpyAsync(h + 28, cand.ptr, first * 4, hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    unsigned long long key;
    double st[2];
    unsigned cnt = 0;
    std::memcpy(&key, h, 8);
    std::memcpy(st, h + 8, 16);
    std::memcpy(&cnt, h + 24, 4);
    if ((int64_t)cnt <= first) {  // else step() selects again with a larger buffer
      pre_I.resize(cnt);
      if (cnt) std::memcpy(pre_I.data(), h + 28, (size_t)cnt * 4);
      pre_k = k_next;
      pre_ok = true;
    }
    maxkey_decode(key, &eta_inf, &eta_argmax);
    r2 = st[0];
    vr = st[1];
    float ms = 0;
    PC_HIP(hipEventElapsedTime(&ms, p->ev_a, p->ev_b));
    adj_ms += ms;
    adj_calls++;
  }

  void read_scal(double* host, int first, int count) {
    PC_HIP(hipMemcpyAsync(host, scal.ptr + first, count * sizeof(double), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
  }

  // Restricted duality gap at the gradient point y from the scalar block
  // ||r_y||^2, Re<V, r_y>, ||y||_1, max |g| (dual point scaled into the
  // feasible set); true when it is within tol of the restricted objective.
  // Under positivity the objective is +inf at a y outside x >= 0: no pass.
  bool gap_test_passes(double tol) {
    double h[5];
    read_scal(h, kScalResid, 5);
    if (positive && h[4] > 0.0) return false;
    const double py = 0.5 * h[0] + lam * h[2];
    const double sc = h[3] <= lam ? 1.0 : lam / h[3];
    const double gy = py - (sc * h[1] - 0.5 * sc * sc * h[0]);
    return gy <= tol * py;
  }

  void residual_stats(double& r2, double& vr) {
    red_partial.ensure(2 * k_resid_blocks(L));
    k_resid(p, L, r.ptr, V.ptr, red_partial.ptr, scal.ptr + kScalResid, s);
    double h[2];
    read_scal(h, kScalResid, 2);
    r2 = h[0];
    vr = h[1];
  }

  // Upload an active set and prepare its atom table (weights from xs_host).
  void load_active(const std::vector<int32_t>& set, const std::vector<double>& xs_host) {
    const int64_t nS = (int64_t)set.size();
    pix.ensure(nS);
    atoms.ensure(atom_capacity(nS));
    x.ensure(nS);
    y.ensure(nS);
    g.ensure(nS);
    adj_partial.ensure(adjoint_partial_count(p, nS));
    act_rows = RowMask{nullptr, 0};
    act_rowlist = nullptr;
    act_nrows = 0;
    if (nS == 0) return;
    // one upload and one kernel: x = y = weights, pix, atom table; the mask
    // of the image rows that hold atoms stays in the block for the gridded
    // operators
    // and the list of occupied rows (the set is sorted by pixel, so each
    // row's atoms are a range)
    const int n = p->g.n;
    int64_t nrows = 0;
    for (int64_t q = 0; q < nS; ++q)
      if (q == 0 || set[q] / n != set[q - 1] / n) ++nrows;
    const int64_t words = (n + 31) / 32, moff = (nS * 12 + 7) / 8 * 8;
    const int64_t loff = moff + words * 4;
    const int64_t bytes = loff + nrows * 12;
    act_blk.ensure((bytes + 7) / 8);
    unsigned char* h = (unsigned char*)up_act.get(bytes);
    std::memcpy(h, xs_host.data(), nS * 8);
    std::memcpy(h + nS * 8, set.data(), nS * 4);
    uint32_t* mask = (uint32_t*)(h + moff);
    std::memset(mask, 0, words * 4);
    int32_t* rl = (int32_t*)(h + loff);
    int64_t r = -1;
    for (int64_t q = 0; q < nS; ++q) {
      const int i = set[q] / n;
      mask[i >> 5] |= 1u << (i & 31);
      if (q == 0 || i != set[q - 1] / n) {
        ++r;
        rl[3 * r] = i;
        rl[3 * r + 1] = (int32_t)q;
      }
      rl[3 * r + 2] = (int32_t)(q + 1);
    }
    PC_HIP(hipMemcpyAsync(act_blk.ptr, h, bytes, hipMemcpyHostToDevice, s));
    up_act.arm(s);
    k_activate(p, nS, act_blk.ptr, x.ptr, y.ptr, pix.ptr, atoms.ptr, s);
    act_rows = RowMask{(const uint32_t*)((const unsigned char*)act_blk.ptr + moff), nrows};
    act_rowlist = (const int3*)((const unsigned char*)act_blk.ptr + loff);
    act_nrows = nrows;
  }

  // Crossover between the direct sums and the gridded operators (restricted
  // to the image rows that hold atoms), per direction, from rates measured on
  // gfx950: the direct sums about 0.45 ps per visibility-atom pair; the
  // gridded operators about 28 ps per visibility (spread or interpolation),
  // 3.4 ps per fine-grid point of the band rows' transforms and 2.7 ps per
  // fine-grid point of the image rows' transforms (at most one row per
  // atom), plus 15 us of launches.
  int64_t grid_crossover() const {
    if (p->Cw) return INT64_MAX / 8;  // no gridded forward with the w-term: direct sums only
    if (prm.grid_atoms > 0) return prm.grid_atoms;
    if (prm.grid_atoms < 0) return INT64_MAX / 8;
    const double M = (double)p->g.M, Ld = (double)L;
    const double per_atom = 0.45e-12 * Ld - 2.7e-12 * M;
    const double fixed = 28e-12 * Ld + 3.4e-12 * (double)p->g.nv * M + 15e-6;
    if (per_atom <= 0 || fixed / per_atom > 1e12) return INT64_MAX / 8;
    return (int64_t)std::ceil(fixed / per_atom);
  }

  // The loaded active set for the gridded operators (not with a
  // dictionary, whose atoms cover several pixels each).
  AtomSet atom_set(int64_t nS) const {
    return AtomSet{nS, pix.ptr, act_rowlist, act_nrows, act_rows};
  }

  void ensure_dimg() {
    if (dimg.ptr) return;
    dimg.ensure(N);
    k_fill(p, N, 0.0f, dimg.ptr, s);
  }

  // out = base - Phi_S w (base = V) or Phi_S w (no base), in plan order.  The
  // direct path takes the weights from the atom table; the gridded one
  // evaluates the set's rows directly (with a dictionary: synthesises the
  // elements into the zero dense image, interpolates, and clears it).
  void op_forward(bool gridded, int64_t nS, const double* w, bool base, c32* out) {
    resid_parts = 0;
    if (!gridded) {
      forward_atoms<float>(p, nS, atoms.ptr, base ? V.ptr : nullptr, true, out, true, s);
      return;
    }
    if (ms) {  // Psi w: weighted elements (overlapping), cleared after use
      ensure_dimg();
      dict_synthesis(p, dict, nS, pix.ptr, w, dimg.ptr, s);
      forward_grid<float>(p, dimg.ptr, out, true, s);
      k_fill(p, N, 0.0f, dimg.ptr, s);
    } else {  // (the residual and its statistics formed by the interpolation itself)
      if (base) red_partial.ensure(2 * std::max<int64_t>(k_resid_blocks(L), p->n_interp));
      forward_grid_set(p, atom_set(nS), w, base ? V.ptr : nullptr,
                       base ? red_partial.ptr : nullptr, out, s);
      resid_parts = base ? p->n_interp : 0;
      return;
    }
    if (base) k_rsub(p, L, V.ptr, out, s);
  }

  // g = Phi_S* r (FP64), directly or as the gridded adjoint sampled at S
  // (eta serves as scratch: it is recomputed after the APGD step; only the
  // rows holding atoms are computed).
  void op_adjoint(bool gridded, int64_t nS, const c32* rr, double* gout) {
    if (!gridded) {
      adjoint_atoms<float>(p, rr, true, nS, atoms.ptr, adj_partial.ptr, gout, s);
      return;
    }
    if (ms) {
      adjoint_grid<float>(p, rr, true, eta.ptr, 1.0f, s);
      dict_gather(p, dict, nS, pix.ptr, eta.ptr, gout, s);
    } else {
      adjoint_grid_set(p, rr, atom_set(nS), gout, s);
    }
  }

  void init(const void* vis_caller) {
    t0 = now();
    grid_thr = grid_crossover();
    V.ensure(L);
    r.ensure(L);
    eta.ensure(N);
    if (ms) eta_ms.ensure(NA);
    scal.ensure(kScalCount);
    cand_count.ensure(1);
    cand.ensure(65536);
    k_gather(p, L, p->perm, (const c32*)vis_caller, V.ptr, s);
    adjoint_timed(V.ptr);
    lmax = eta_inf;
    lam = prm.lambda > 0 ? prm.lambda : prm.alpha * lmax;
    Delta = (1.0 - prm.delta) * lmax;
    // P(0) = ||V||^2 / 2
    PC_HIP(hipMemcpyAsync(r.ptr, V.ptr, L * sizeof(c32), hipMemcpyDeviceToDevice, s));
    double r2, vr;
    residual_stats(r2, vr);
    v2 = r2;
    P_prev = 0.5 * r2;
    P = P_prev;
    const double sc = (eta_inf <= lam) ? 1.0 : lam / eta_inf;
    gap = P - (sc * vr - 0.5 * sc * sc * r2);
    rel_gap = P > 0 ? gap / P : 0.0;
    if (!(lmax > 0) || !(lam > 0)) {  // zero data: x = 0 is the solution
      done = true;
      converged = true;
    } else if (prm.x0_n > 0) {
      warm_start();
    }
  }

  // Residual, dirty residual (and its maximum), objective and duality gap of
  // the iterate (S, xs): step 4 of Alg. 2, also run once for a warm start.
  void assess(int k_next) {
    load_active(S, xs);
    const bool gridded = ms || (int64_t)S.size() >= grid_thr;
    double r2, vr;
    if (batcher && !gridded) {
      // the residual's direct sums run in the batcher's shared launch ahead
      // of the shared adjoint (the atom table holds x / n after load_active)
      const FwdSpec fs{atoms.ptr, (int64_t)S.size(), V.ptr};
      pre_ok = false;
      adjoint_timed(r.ptr, &fs);
      residual_stats(r2, vr);
    } else {
      op_forward(gridded, (int64_t)S.size(), x.ptr, true, r.ptr);
      adjoint_and_stats(r.ptr, r2, vr, k_next);
    }
    double l1 = 0;
    for (double w : xs) l1 += std::fabs(w);
    P = 0.5 * r2 + lam * l1;
    const double sc = (eta_inf <= lam) ? 1.0 : lam / eta_inf;
    gap = P - (sc * vr - 0.5 * sc * sc * r2);
    rel_gap = P > 0 ? gap / P : 0.0;
  }

  // Warm start: the solve continues from x0 (atoms sorted, zero weights
  // dropped) as if it were the previous iterate; lambda_max, lambda and
  // Delta still come from the data alone.  The gap test applies to x0 itself
  // (zero FW iterations when it passes); the improvement test needs an
  // iteration.
  void warm_start() {
    std::vector<std::pair<int32_t, double>> at;
    at.reserve((size_t)prm.x0_n);
    for (int64_t q = 0; q < prm.x0_n; ++q)
      if (prm.x0_w[q] != 0.0) at.push_back({prm.x0_pix[q], prm.x0_w[q]});
    std::sort(at.begin(), at.end());
    S.clear();
    xs.clear();
    for (const auto& a : at) {
      S.push_back(a.first);
      xs.push_back(a.second);
    }
    assess(0);
    P_prev = P;
    // a warm start that already meets the gap tolerance is the answer
    if (prm.rel_gap_tol > 0 && rel_gap <= prm.rel_gap_tol) {
      converged = true;
      done = true;
    }
  }

  int64_t gram_cap() const {  // the Gram-form Lanczos holds its basis in LDS
    // with the w-term Phi_S* Phi_S is no longer a function of pixel offsets
    if (p->Cw) return 0;
    if (prm.gram_atoms > 0) return std::min<int64_t>(prm.gram_atoms, kGramLdsAtoms);
    return prm.gram_atoms < 0 ? 0 : kGramAtoms;
  }

  static uint64_t offset_key(int da, int db) {  // psf(-d) = psf(d): one key for both
    if (da < 0 || (da == 0 && db < 0)) {
      da = -da;
      db = -db;
    }
    return ((uint64_t)(uint32_t)da << 32) | (uint32_t)(db + (1 << 30));
  }

  // G and b for the active set: psf values at offsets not seen before in this
  // solve come from a restricted adjoint of unit visibilities at the offsets,
  // b_p for atoms not seen before from a restricted adjoint of V (both with
  // FP64 totals: the gap test forms ||V - Phi_S y||^2 = ||V||^2 - 2 y.b +
  // y.G y, which cancels), written into per-solve device tables by slot (in
  // the batcher's shared launches when the solve has one).  The host keeps
  // only the slot of each offset and pixel and uploads the slot table with the
  // Lanczos start vector; G, b and that vector are gathered on the device.
  // Returns false (and changes nothing) when the new point-spread sums would
  // cost more than kGramNewPairs operator applications on this set: the
  // operator path is then cheaper for this FW iteration.
  bool build_gram(const std::vector<int32_t>& set) {
    const int64_t nS = (int64_t)set.size();
    const int n = p->g.n;
    std::vector<int> ai(nS), bi(nS);
    std::vector<double> inv_n(nS);
    for (int64_t q = 0; q < nS; ++q) {
      const int i = set[q] / n, j = set[q] - (set[q] / n) * n;
      ai[q] = i - n / 2;
      bi[q] = j - n / 2;
      const double l = ai[q] * p->g.dl, m = bi[q] * p->g.dl;
      inv_n[q] = 1.0 / std::sqrt(1.0 - l * l - m * m);
    }
    // position of each atom in the previous active set (both sets ascending):
    // pairs of atoms that were both there keep their entry of the previous G
    std::vector<int64_t> old(nS, -1);
    for (size_t a = 0, c = 0; a < (size_t)nS && c < g_set.size();) {
      if (set[a] == g_set[c]) {
        old[a] = (int64_t)c;
        ++a;
        ++c;
      } else if (set[a] < g_set[c]) {
        ++a;
      } else {
        ++c;
      }
    }
    // the slot of every pair's offset: kept from the last G, else looked up,
    // a new offset getting the next slot
    std::vector<std::pair<int, int>> miss;
    std::vector<int32_t> slots((size_t)nS * nS);
    const int64_t no = (int64_t)g_set.size();
    for (int64_t a = 0; a < nS; ++a)
      for (int64_t c = a; c < nS; ++c) {
        int32_t sl;
        if (old[a] >= 0 && old[c] >= 0) {
          sl = g_slots[(size_t)old[a] * no + old[c]];
        } else {
          int da = ai[a] - ai[c], db = bi[a] - bi[c];
          const auto ins =
              psf_slot.emplace(offset_key(da, db), (int32_t)(n_psf + (int64_t)miss.size()));
          if (ins.second) {
            if (da < 0 || (da == 0 && db < 0)) {
              da = -da;
              db = -db;
            }
            miss.emplace_back(da, db);
          }
          sl = ins.first->second;
        }
        slots[(size_t)a * nS + c] = sl;
        slots[(size_t)c * nS + a] = sl;
      }
    std::vector<int64_t> bmiss;  // atoms whose b_p is not known yet
    for (int64_t q = 0; q < nS; ++q)
      if (!b_slot.count(set[q])) bmiss.push_back(q);
    const int64_t nm = (int64_t)miss.size(), nb = (int64_t)bmiss.size();
    if (nm + nb > kGramNewPairs * nS) {
      for (const auto& o : miss) psf_slot.erase(offset_key(o.first, o.second));
      return false;
    }
    for (int64_t t = 0; t < nb; ++t) b_slot[set[bmiss[t]]] = (int32_t)(n_b + t);
    // one upload: [offset / atom table | v0 | inv_n | b slots | pair slots]
    const std::vector<double> v0 = lanczos_start(set);
    const size_t tbytes = (size_t)(nm + nb) * sizeof(Atom<float>);
    const size_t abytes = (size_t)(16 * nS + 4 * nS + 4 * nS * nS);
    unsigned char* h = (unsigned char*)up.get(tbytes + abytes);
    Atom<float>* at = (Atom<float>*)h;
    for (int64_t m = 0; m < nm; ++m)
      at[m] = Atom<float>{(double)miss[m].first, (double)miss[m].second, 1.0, 0.0, 0.f, 0.f};
    for (int64_t t = 0; t < nb; ++t) {
      const int64_t q = bmiss[t];
      at[nm + t] = Atom<float>{(double)ai[q], (double)bi[q], inv_n[q], 0.0, 0.f, 0.f};
    }
    unsigned char* blk = h + tbytes;
    std::memcpy(blk, v0.data(), (size_t)nS * 8);
    std::memcpy(blk + 8 * nS, inv_n.data(), (size_t)nS * 8);
    int32_t* bs = (int32_t*)(blk + 16 * nS);
    for (int64_t a = 0; a < nS; ++a) bs[a] = b_slot.at(set[a]);
    std::memcpy(bs + nS, slots.data(), (size_t)nS * nS * 4);
    if (nm + nb > 0) {
      off_atoms.ensure(nm + nb);
      PC_HIP(hipMemcpyAsync(off_atoms.ptr, at, tbytes, hipMemcpyHostToDevice, s));
    }
    asm_blk.ensure((int64_t)((abytes + 7) / 8));
    PC_HIP(hipMemcpyAsync(asm_blk.ptr, blk, abytes, hipMemcpyHostToDevice, s));
    up.arm(s);
    if (nm + nb > 0) {  // new sums, written straight into their slots
      psf_dev.ensure(n_psf + nm, s);
      b_dev.ensure(n_b + nb, s);
      psf_partial.ensure(std::max(adjoint_partial_count(p, nm), adjoint_partial_count(p, nb)));
      if (batcher) {  // in the batcher's shared launches (each sum its own partials)
        b_partial.ensure(adjoint_partial_count(p, nb));
        std::vector<AccJob> sums;
        if (nm)
          sums.push_back(AccJob{p, off_atoms.ptr, nm, nullptr, psf_partial.ptr,
                                psf_dev.ptr + n_psf});
        if (nb)
          sums.push_back(AccJob{p, off_atoms.ptr + nm, nb, V.ptr, b_partial.ptr,
                                b_dev.ptr + n_b});
        batcher_restricted_adjoints(batcher, p, s, sums);
      } else {
        if (nm)  // unit visibilities (none are read): the point-spread sums
          adjoint_atoms_acc64(p, nullptr, nm, off_atoms.ptr, psf_partial.ptr,
                              psf_dev.ptr + n_psf, s);
        if (nb)
          adjoint_atoms_acc64(p, V.ptr, nb, off_atoms.ptr + nm, psf_partial.ptr,
                              b_dev.ptr + n_b, s);
      }
      n_psf += nm;
      n_b += nb;
    }
    g_set = set;
    g_slots.swap(slots);
    // G, b and the Lanczos start vector gathered on the device
    gram_blk.ensure(nS * nS + nS + (int64_t)(kLanczosMax + 1) * nS);
    gram_G = gram_blk.ptr;
    gram_b = gram_G + nS * nS;
    gram_Q = gram_b + nS;
    k_gram_assemble(p, nS, asm_blk.ptr, psf_dev.ptr, b_dev.ptr, gram_G, gram_b, gram_Q, s);
    return true;
  }

  // Lanczos start vector: the previous top Ritz vector on the atoms both sets
  // share (else uniform), normalised.
  std::vector<double> lanczos_start(const std::vector<int32_t>& set) const {
    const int64_t nS = (int64_t)set.size();
    std::vector<double> v0(nS, 1.0 / std::sqrt((double)nS));
    for (size_t a = 0, b = 0; a < pv_set.size() && b < set.size();) {
      if (pv_set[a] == set[b]) {
        v0[b] = pv_val[a];
        ++a;
        ++b;
      } else if (pv_set[a] < set[b]) {
        ++a;
      } else {
        ++b;
      }
    }
    double nrm = 0;
    for (double q : v0) nrm += q * q;
    nrm = std::sqrt(nrm);
    for (double& q : v0) q /= nrm;
    return v0;
  }

  // Upper estimate of the largest eigenvalue of G_S = Re(Phi_S^H Phi_S) by
  // Lanczos iteration with full reorthogonalisation (FP64 on the device; G_S
  // applied as the operator pair, or as the matrix in the Gram form), started
  // from the previous active set's top Ritz vector (lanczos_start).
  // After step j the top Ritz value theta of the tridiagonal T_j and the
  // residual bound rho = beta_j |s_j| (s the Ritz vector in the Lanczos
  // basis) bracket an eigenvalue: |lambda - theta| <= rho.  Stops when
  // rho <= kLanczosTol theta (or at kLanczosMax steps, or on an invariant
  // subspace) and returns theta + rho.
  double top_eigen_bound(const std::vector<int32_t>& set, bool gridded) {
    const int64_t nS = (int64_t)set.size();
    // The recurrence runs on the device (k_lanczos_step); the host reads
    // alpha, beta (and the basis) once per batch of steps and applies the
    // stopping rule to each step of the batch in order, so the result is that
    // of stopping at the first step that meets it.
    const int jmax = (int)std::min<int64_t>(kLanczosMax, nS);  // T is at most nS x nS
    lz_w.ensure(nS);
    lz_ab.ensure(2 * kLanczosMax);
    lz_Q.ensure((int64_t)(kLanczosMax + 1) * nS);
    double* Qd = lz_Q.ptr;
    {
      const std::vector<double> v0 = lanczos_start(set);
      double* h = (double*)up.get(nS * 8);
      std::memcpy(h, v0.data(), nS * 8);
      PC_HIP(hipMemcpyAsync(Qd, h, nS * 8, hipMemcpyHostToDevice, s));
      up.arm(s);
    }
    std::vector<double> svec, Qh;
    double theta = 0, rho = 0;
    int done_steps = 0, kfin = 0;
    // expensive steps are read back one at a time, so that none runs past
    // the one that meets the stopping rule
    const int batch =
        (gridded || (double)L * (double)nS > kCheckEveryPairs) ? 1 : kLanczosBatch;
    while (kfin == 0) {
      const int jend = std::min(jmax, done_steps + batch);
      for (int j = done_steps; j < jend; ++j) {
        double* qj = Qd + (int64_t)j * nS;
        if (!gridded) k_weights(p, nS, qj, atoms.ptr, s);
        if (!gridded && fused_supported(nS)) {  // g = Phi_S* Phi_S q_j in one pass
          forward_adjoint_atoms(p, nS, atoms.ptr, nullptr, nullptr, adj_partial.ptr, s);
          reduce_partials<float>(p, nS, fused_partial_stride(p, nS), adj_partial.ptr, atoms.ptr,
                                 g.ptr, s);
        } else {
          op_forward(gridded, nS, qj, false, r.ptr);
          op_adjoint(gridded, nS, r.ptr, g.ptr);
        }
        k_lanczos_step(p, nS, j, kLanczosMax, Qd, g.ptr, lz_w.ptr, lz_ab.ptr, s);
      }
      const size_t qbytes = (size_t)(jend + 1) * nS * 8;
      const bool basis_now = qbytes <= (512u << 10);  // small: read with the coefficients
      unsigned char* h = (unsigned char*)down.get(16 * kLanczosMax + (basis_now ? qbytes : 0));
      PC_HIP(hipMemcpyAsync(h, lz_ab.ptr, 16 * kLanczosMax, hipMemcpyDeviceToHost, s));
      if (basis_now)
        PC_HIP(hipMemcpyAsync(h + 16 * kLanczosMax, Qd, qbytes, hipMemcpyDeviceToHost, s));
      PC_HIP(hipStreamSynchronize(s));
      const double* alpha = (const double*)h;
      const double* beta = alpha + kLanczosMax;
      for (int j = done_steps; j < jend && kfin == 0; ++j) {
        const int k = j + 1;
        std::vector<double> T((size_t)k * k, 0.0);
        for (int i = 0; i < k; ++i) {
          T[(size_t)i * k + i] = alpha[i];
          if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = beta[i];
        }
        theta = sym_top_eigen(T, k, svec);
        const double bj = beta[j];
        rho = bj * std::fabs(svec[k - 1]);
        const bool invariant = bj <= 1e-14 * std::max(theta, 1e-300) || k >= nS;
        if (invariant || rho <= kLanczosTol * theta || k == kLanczosMax) kfin = k;
        last_lanczos = k;
      }
      if (kfin) {
        Qh.resize((size_t)kfin * nS);
        if (basis_now) {
          std::memcpy(Qh.data(), h + 16 * kLanczosMax, (size_t)kfin * nS * 8);
        } else {
          PC_HIP(hipMemcpyAsync(Qh.data(), Qd, (size_t)kfin * nS * 8,
                                hipMemcpyDeviceToHost, s));
          PC_HIP(hipStreamSynchronize(s));
        }
      }
      done_steps = jend;
    }
    // top Ritz vector as the next warm start
    pv_set = set;
    pv_val.assign(nS, 0.0);
    for (int q = 0; q < kfin; ++q)
      for (int64_t i = 0; i < nS; ++i) pv_val[i] += svec[q] * Qh[(size_t)q * nS + i];
    return theta + rho;
  }

  void step() {
    if (done) return;
    // 1.a polyatomic exploration: threshold in FP64, compared in FP32 (the
    // candidates may already have come back with step 4's statistics)
    const double tau = eta_inf - 2.0 * Delta / (k + 2);
    const float tau_f = (float)tau;
    // the count and the first kFirst candidates come back in one copy pair
    constexpr int64_t kFirst = kFirstCandidates;
    unsigned count = 0;
    std::vector<int32_t> I;
    bool have = false;
    if (pre_ok && pre_k == k) {
      I.swap(pre_I);
      count = (unsigned)I.size();
      have = true;
    }
    pre_ok = false;
    while (!have) {
      k_select(p, NA, expl(), tau_f, positive, cand_count.ptr, cand.ptr, cand.cap, s);
      const int64_t first = std::min<int64_t>(kFirst, cand.cap);
      unsigned char* h = (unsigned char*)down.get(4 + first * 4);
      PC_HIP(hipMemcpyAsync(h, cand_count.ptr, 4, hipMemcpyDeviceToHost, s));
      PC_HIP(hipMemcpyAsync(h + 4, cand.ptr, first * 4, hipMemcpyDeviceToHost, s));
      PC_HIP(hipStreamSynchronize(s));
      std::memcpy(&count, h, 4);
      if ((int64_t)count > cand.cap) {
        cand.ensure(count);
        continue;
      }
      I.resize(count);
      const int64_t head = std::min<int64_t>(count, first);
      if (head) std::memcpy(I.data(), h + 4, head * 4);
      if ((int64_t)count > first) {
        PC_HIP(hipMemcpyAsync(I.data() + first, cand.ptr + first, (count - first) * 4,
                              hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
      }
      have = true;
    }
    std::sort(I.begin(), I.end());
    // 1.b S u I with warm-start weights (new atoms at zero)
    std::vector<int32_t> Sn;
    Sn.reserve(S.size() + I.size());
    std::set_union(S.begin(), S.end(), I.begin(), I.end(), std::back_inserter(Sn));
    std::vector<double> xw(Sn.size(), 0.0);
    for (size_t a = 0, b = 0; a < S.size(); ++a) {
      while (Sn[b] != S[a]) ++b;
      xw[b] = xs[a];
    }
    const int64_t nS = (int64_t)Sn.size();
    load_active(Sn, xw);
    // 2. APGD on the restricted problem
    int inner = 0;
    // small sets: the Gram form (one small kernel per step) when its new
    // point-spread sums are affordable, else the gridded operators from the
    // crossover on, else the direct sums (a crossover set by the caller
    // comes before the Gram form)
    const bool force_grid = ms || (prm.grid_atoms > 0 && nS >= grid_thr);
    const bool gram = !force_grid && nS > 0 && nS <= gram_cap() && build_gram(Sn);
    const bool gridded = !gram && (ms || nS >= grid_thr);
    if (nS > 0) {
      // step constant: on the device for the Gram form (read there by the
      // APGD kernel, no host round trip), else from the host-driven Lanczos
      double lip = 0;
      if (gram) {
        lz_ab.ensure(2 * kLanczosMax);
        lz_out.ensure(4 + nS);
        k_gram_lanczos_full(p, nS, kLanczosMax, kLanczosTol, kLipMargin, gram_G, gram_Q,
                            lz_ab.ptr, lz_out.ptr, lz_out.ptr + 4, s);
      } else {
        lip = top_eigen_bound(Sn, gridded) * kLipMargin;
      }
      k_weights(p, nS, y.ptr, atoms.ptr, s);  // y = x_warm as forward weights
      const double tol = std::max(prm.inner_tol_min, prm.inner_tol0 * rel_gap);
      double t = 1.0;  // FISTA momentum sequence, on the host in FP64
      if (gram) {
        // steps are enqueued in chunks; the kernel applies the gap test and
        // turns the remaining steps into no-ops, and the host reads the
        // outcome (and x) once per chunk
        gram_done.ensure(2);
        k_zero_u32(p, 2, (unsigned*)gram_done.ptr, s);
        int issued = 0, stop = 0;
        unsigned char* h = nullptr;
        while (stop == 0 && issued < prm.inner_max_iter) {
          // first chunk: through one test past the previous solve's stopping
          // step (steps after the passing test are no-ops)
          const int first = std::max(1, last_inner) + kCheck;
          const int chunk = std::min(issued == 0 ? std::min(first, 4 * kGramChunk)
                                                 : 2 * kGramChunk,
                                     prm.inner_max_iter - issued);
          // one launch runs the chunk's steps; the host advances the same
          // momentum recurrence for the next chunk's start
          k_gram_fista(p, nS, gram_G, gram_b, x.ptr, y.ptr, g.ptr, scal.ptr + kScalResid, v2,
                       lz_out.ptr, t, issued, chunk, kCheck, lam, tol, positive, gram_done.ptr,
                       s);
          for (int c = 0; c < chunk; ++c) t = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
          issued += chunk;
          // outcome, x, and the Lanczos result with its Ritz vector
          h = (unsigned char*)down.get(8 + nS * 8 + (4 + nS) * 8);
          PC_HIP(hipMemcpyAsync(h, gram_done.ptr, 8, hipMemcpyDeviceToHost, s));
          PC_HIP(hipMemcpyAsync(h + 8, x.ptr, nS * 8, hipMemcpyDeviceToHost, s));
          PC_HIP(hipMemcpyAsync(h + 8 + nS * 8, lz_out.ptr, (4 + nS) * 8, hipMemcpyDeviceToHost, s));
          PC_HIP(hipStreamSynchronize(s));
          const int* dn = (const int*)h;
          if (dn[0]) stop = dn[1];
        }
        inner = stop ? stop : prm.inner_max_iter;
        last_inner = inner;
        xw.resize(nS);
        std::memcpy(xw.data(), h + 8, nS * 8);
        const double* lz = (const double*)(h + 8 + nS * 8);  // {L, steps, theta, rho}, ritz
        last_lanczos = (int)lz[1];
        pv_set = Sn;
        pv_val.assign(lz + 4, lz + 4 + nS);
      } else {
        stat.ensure(2 * nS);
        // small direct sets: forward and restricted adjoint share one pass
        const bool fused = !gridded && fused_supported(nS);
        const int64_t nwg = fused ? fused_partial_stride(p, nS) : adjoint_partial_stride(p, nS);
        const int every = (gridded || (double)L * (double)nS > kCheckEveryPairs) ? 1 : kCheck;
        for (inner = 1; inner <= prm.inner_max_iter; ++inner) {
          const bool check = (inner - 1) % every == 0;
          if (fused)  // r_y is needed only by the convergence test
            forward_adjoint_atoms(p, nS, atoms.ptr, V.ptr, check ? r.ptr : nullptr,
                                  adj_partial.ptr, s);
          else
            op_forward(gridded, nS, y.ptr, true, r.ptr);
          if (check) {
            if (!fused && resid_parts > 0) {
              k_resid_final(p, (int)resid_parts, red_partial.ptr, scal.ptr + kScalResid, s);
            } else {
              red_partial.ensure(2 * k_resid_blocks(L));
              k_resid(p, L, r.ptr, V.ptr, red_partial.ptr, scal.ptr + kScalResid, s);
            }
          }
          const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
          const double mom = (t - 1.0) / tn;
          t = tn;
          if (!gridded) {  // partial sums of Phi_S* r, summed by the fused step
            if (!fused)
              adjoint_atoms<float>(p, r.ptr, true, nS, atoms.ptr, adj_partial.ptr, nullptr, s);
            reduce_fista(p, nS, nwg, adj_partial.ptr, nullptr, atoms.ptr, x.ptr, y.ptr, g.ptr,
                         stat.ptr, 1.0 / lip, lam / lip, mom, positive, s);
          } else {
            op_adjoint(true, nS, r.ptr, g.ptr);
            reduce_fista(p, nS, 0, nullptr, g.ptr, atoms.ptr, x.ptr, y.ptr, g.ptr, stat.ptr,
                         1.0 / lip, lam / lip, mom, positive, s);
          }
          if (check) {
            k_stat_reduce(p, nS, stat.ptr, scal.ptr, s);
            if (gap_test_passes(tol)) break;
          }
        }
      }
      if (!gram) {
        inner = std::min(inner, prm.inner_max_iter);
        xw.resize(nS);
        double* hx = (double*)down.get(nS * 8);
        PC_HIP(hipMemcpyAsync(hx, x.ptr, nS * 8, hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        std::memcpy(xw.data(), hx, nS * 8);
      }
    }
    inner_total += inner;
    // 3. prune
    S.clear();
    xs.clear();
    for (int64_t a = 0; a < nS; ++a)
      if (xw[a] != 0.0) {
        S.push_back(Sn[a]);
        xs.push_back(xw[a]);
      }
    // 4. residual, dirty residual, objective and gap
    assess(k + 1);
    const double rel_imp = P_prev > 0 ? std::fabs(P - P_prev) / P_prev : 0.0;
    if (prm.log_every > 0 && (k % prm.log_every == 0))
      std::fprintf(stderr,
                   "[pfw] k=%d new=%u active=%zu eta_inf=%.6g obj=%.10g rel_gap=%.3e inner=%d "
                   "lanczos=%d\n",
                   k, count, S.size(), eta_inf, P, rel_gap, inner, last_lanczos);
    P_prev = P;
    ++k;
    if (prm.rel_obj_tol > 0 && rel_imp <= prm.rel_obj_tol) converged = true;
    if (prm.rel_gap_tol > 0 && rel_gap <= prm.rel_gap_tol) converged = true;
    if (converged || k >= prm.max_iter) done = true;
  }

  pc_status fill(pc_solve_result* res) {
    const int64_t na = (int64_t)S.size();
    res->natoms = na;
    res->objective = P;
    res->rel_gap = rel_gap;
    res->lambda = lam;
    res->lambda_max = lmax;
    res->cert_max = lam > 0 ? eta_inf / lam : 0.0;
    res->cert_argmax = eta_argmax;
    res->iters = k;
    res->inner_iters = inner_total;
    res->converged = converged ? 1 : 0;
    res->adjoint_seconds = adj_ms * 1e-3;
    res->adjoint_calls = adj_calls;
    if (prm.want_certificate && res->cert && lam > 0)
      k_scale(p, NA, expl(), (float)(1.0 / lam), res->cert, s);
    PC_HIP(hipStreamSynchronize(s));
    res->seconds = now() - t0;
    if (na > res->capacity) {
      set_last_error("pc_polyclean_solve: result capacity " + std::to_string(res->capacity) +
                     " < natoms " + std::to_string(na));
      return PC_ERR_CAPACITY;
    }
    if (na > 0) {
      std::memcpy(res->pix, S.data(), na * sizeof(int32_t));
      std::memcpy(res->weight, xs.data(), na * sizeof(double));
    }
    return converged ? PC_OK : PC_WARN_NOT_CONVERGED;
  }
};

static void check_params(const pc_solve_params* prm) {
  PC_REQUIRE(prm != nullptr, "params is NULL");
  PC_REQUIRE(prm->max_iter >= 1, "max_iter must be >= 1");
  PC_REQUIRE(prm->delta > 0 && prm->delta <= 1, "delta must be in (0, 1]");
  PC_REQUIRE(prm->lambda > 0 || (prm->alpha > 0 && std::isfinite(prm->alpha)),
             "lambda > 0 or alpha > 0 is required");
  PC_REQUIRE(prm->inner_max_iter >= 1, "inner_max_iter must be >= 1");
  PC_REQUIRE(prm->inner_tol0 >= 0 && prm->inner_tol_min >= 0, "inner tolerances must be >= 0");
  PC_REQUIRE(prm->n_scales >= 0 && prm->n_scales <= kDictMaxScales, "n_scales must be in [0, 8]");
  if (prm->n_scales > 0) (void)make_dict(prm->n_scales, prm->scale_sigma, prm->scale_gamma);
  PC_REQUIRE(prm->x0_n >= 0, "x0_n must be >= 0");
  if (prm->x0_n > 0) {
    PC_REQUIRE(prm->x0_pix != nullptr && prm->x0_w != nullptr, "x0_pix / x0_w are NULL");
    for (int64_t q = 0; q < prm->x0_n; ++q) {
      PC_REQUIRE(std::isfinite(prm->x0_w[q]), "x0_w must be finite");
      PC_REQUIRE(prm->positivity == 0 || prm->x0_w[q] >= 0,
                 "x0_w must be >= 0 under positivity");
    }
  }
}

}  // namespace pc

using namespace pc;

struct pc_solver {
  Pfw pfw;
  pc_solver(pc_plan* p, hipStream_t s, const pc_solve_params& prm) : pfw(p, s, prm) {}
};

static pc_solver* solver_new(pc_plan* plan, const void* vis, const pc_solve_params* prm,
                             void* stream, pc_batcher* batcher) {
  PC_REQUIRE(plan && vis, "NULL argument");
  PC_REQUIRE(plan->precision == PC_PREC_FP32, "solve needs an FP32 plan");
  check_params(prm);
  PC_HIP(hipSetDevice(plan->device));
  auto* sv = new pc_solver(plan, (hipStream_t)stream, *prm);
  sv->pfw.batcher = batcher;
  try {
    sv->pfw.init(vis);
    plan_touch(plan, (hipStream_t)stream);
  } catch (...) {
    delete sv;
    throw;
  }
  return sv;
}

template <typename F>
static pc_status guarded(const char* fn, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(std::string(fn) + ": " + e.what());
    return e.status;
  } catch (const std::exception& e) {
    set_last_error(std::string(fn) + ": " + e.what());
    return PC_ERR_DEVICE;
  }
}

extern "C" {

PC_API void pc_solve_params_default(pc_solve_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->alpha = 0.01;
  p->delta = 0.99;
  p->max_iter = 50;
  p->inner_tol0 = 0.1;
  p->inner_tol_min = 1e-8;
  p->inner_max_iter = 2000;
}

PC_API pc_status pc_polyclean_solve(pc_plan* plan, const void* vis, const pc_solve_params* prm,
                                    pc_solve_result* res, void* stream) {
  return guarded("pc_polyclean_solve", [&] {
    PC_REQUIRE(plan != nullptr && vis != nullptr && res != nullptr, "NULL argument");
    PC_REQUIRE(plan->precision == PC_PREC_FP32, "solve needs an FP32 plan");
    check_params(prm);
    PC_REQUIRE(res->capacity >= 0, "capacity must be >= 0");
    if (res->capacity > 0) PC_REQUIRE(res->pix && res->weight, "result arrays are NULL");
    PC_HIP(hipSetDevice(plan->device));
    Pfw pfw(plan, (hipStream_t)stream, *prm);
    pfw.init(vis);
    while (!pfw.done) pfw.step();
    return pfw.fill(res);
  });
}

PC_API pc_status pc_solver_create(pc_plan* plan, const void* vis, const pc_solve_params* prm,
                                  void* stream, pc_solver** out) {
  return guarded("pc_solver_create", [&] {
    PC_REQUIRE(out != nullptr, "NULL argument");
    *out = nullptr;
    *out = solver_new(plan, vis, prm, stream, nullptr);
    return PC_OK;
  });
}

PC_API pc_status pc_solver_create_batched(pc_plan* plan, const void* vis,
                                          const pc_solve_params* prm, void* stream,
                                          pc_batcher* batcher, pc_solver** out) {
  return guarded("pc_solver_create_batched", [&] {
    PC_REQUIRE(out != nullptr, "NULL argument");
    *out = nullptr;
    *out = solver_new(plan, vis, prm, stream, batcher);
    return PC_OK;
  });
}

PC_API pc_status pc_solver_step(pc_solver* sv, int32_t* done) {
  return guarded("pc_solver_step", [&] {
    PC_REQUIRE(sv != nullptr, "solver is NULL");
    PC_HIP(hipSetDevice(sv->pfw.p->device));
    sv->pfw.step();
    plan_touch(sv->pfw.p, sv->pfw.s);
    if (done) *done = sv->pfw.done ? 1 : 0;
    return PC_OK;
  });
}

PC_API pc_status pc_solver_result(pc_solver* sv, pc_solve_result* res) {
  return guarded("pc_solver_result", [&] {
    PC_REQUIRE(sv != nullptr && res != nullptr, "NULL argument");
    PC_REQUIRE(res->capacity >= 0, "capacity must be >= 0");
    if (res->capacity > 0) PC_REQUIRE(res->pix && res->weight, "result arrays are NULL");
    return sv->pfw.fill(res);
  });
}

PC_API void pc_solver_destroy(pc_solver* sv) { delete sv; }

}  // extern "C"
