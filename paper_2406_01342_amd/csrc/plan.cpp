// Plan construction: host-side FP64 geometry, tile sort, spreading work list,
// kernel correction and twiddle tables, and the device uploads.
//
// Geometry (paper Sect. 2.1-2.2): pixel step dl = fov / n, l_i = (i - n/2) dl,
// m_j = (j - n/2) dl.  The adjoint sum exp(+j 2 pi u_k l_i) with l_i = a dl,
// a = i - n/2, depends on u only through A_k = u_k dl modulo 1 (a is an
// integer), so each visibility sits at the periodic fine-grid coordinate
// X_k = M frac(A_k + 1/2) in cells (M = 2n; the +1/2 puts zero frequency at
// cell M/2 and costs a sign (-1)^a in the output, folded into the correction).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "common.h"

namespace pc {

namespace {
constexpr int kPoolDevices = 64;
struct DevicePool {
  std::mutex mu;
  std::vector<DeviceBuf> free;  // bytes = the size class
  size_t held = 0, cap = 0;
};
DevicePool g_pool[kPoolDevices];
}  // namespace

size_t pool_class(size_t bytes) {
  if (bytes <= 256) return 256;
  int e = 63 - __builtin_clzll((unsigned long long)(bytes - 1));  // 2^e < bytes <= 2^(e+1)
  const size_t step = (size_t)1 << (e - 2);                       // quarters of 2^e
  return (bytes + step - 1) / step * step;
}

size_t pool_trim(int device);

void* pool_alloc(int device, size_t bytes, size_t* got) {
  const size_t cls = pool_class(bytes);
  if (device >= 0 && device < kPoolDevices) {
    DevicePool& P = g_pool[device];
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto it = P.free.begin(); it != P.free.end(); ++it)
      if (it->bytes == cls) {
        void* ptr = it->ptr;
        P.held -= cls;
        P.free.erase(it);
        *got = cls;
        return ptr;
      }
  }
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, cls);
  if (e != hipSuccess && device >= 0 && device < kPoolDevices) {
    // out of memory with buffers parked in the pool: give them back and retry
    (void)hipGetLastError();
    if (pool_trim(device) > 0) e = hipMalloc(&ptr, cls);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(PC_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(cls) + " bytes failed");
  }
  *got = cls;
  return ptr;
}

void pool_release(int device, void* ptr, size_t bytes) {
  if (!ptr) return;
  if (device >= 0 && device < kPoolDevices) {
    DevicePool& P = g_pool[device];
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.cap == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) P.cap = tot / 8;
      else (void)hipGetLastError();
    }
    if (bytes == pool_class(bytes) && P.held + bytes <= P.cap) {
      P.free.push_back({ptr, bytes});
      P.held += bytes;
      return;
    }
  }
  (void)hipFree(ptr);
}

size_t pool_trim(int device) {
  if (device < 0 || device >= kPoolDevices) return 0;
  DevicePool& P = g_pool[device];
  std::vector<DeviceBuf> drop;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    drop.swap(P.free);
    P.held = 0;
  }
  size_t n = 0;
  for (auto& b : drop) {
    (void)hipFree(b.ptr);
    n += b.bytes;
  }
  return n;
}

void plan_touch(pc_plan* p, hipStream_t s) {
  for (auto& t : p->touched)
    if (t.first == s) {
      PC_HIP(hipEventRecord(t.second, s));
      return;
    }
  hipEvent_t ev = nullptr;
  PC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  p->touched.push_back({s, ev});
  PC_HIP(hipEventRecord(ev, s));
}

void* dalloc(pc_plan* p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  size_t got = 0;
  void* ptr = pool_alloc(p->device, bytes, &got);
  p->owned.push_back({ptr, got});
  p->footprint += got;
  return ptr;
}

void plan_release(pc_plan* p) {
  prof_release(p);
  // the plan's own work only (no device-wide wait)
  for (auto& t : p->touched) {
    (void)hipEventSynchronize(t.second);
    (void)hipEventDestroy(t.second);
  }
  p->touched.clear();
  for (auto& b : p->owned) pool_release(p->device, b.ptr, b.bytes);
  p->owned.clear();
  if (p->ev_a) (void)hipEventDestroy(p->ev_a);
  if (p->ev_b) (void)hipEventDestroy(p->ev_b);
}

static void* grow(pc_plan* p, void** slot, size_t* cap, size_t bytes) {
  if (*slot && *cap >= bytes) return *slot;
  if (*slot) {
    for (auto it = p->owned.begin(); it != p->owned.end(); ++it)
      if (it->ptr == *slot) {
        p->footprint -= it->bytes;
        // queued work of the current call may still read the old buffer:
        // hipFree waits for it (growth is rare: scratch reaches its size early)
        (void)hipFree(it->ptr);
        p->owned.erase(it);
        break;
      }
  }
  size_t want = std::max<size_t>(bytes, 4096);
  *slot = dalloc(p, want);
  *cap = want;
  return *slot;
}

void* ensure_atom_scratch(pc_plan* p, size_t bytes) {
  return grow(p, &p->atom_scratch, &p->atom_capacity, bytes);
}

float* ensure_image_scratch(pc_plan* p) {
  return (float*)grow(p, &p->image_scratch, &p->image_capacity,
                      sizeof(float) * (size_t)p->g.n * p->g.n);
}

unsigned long long* ensure_key_scratch(pc_plan* p, size_t count) {
  return (unsigned long long*)grow(p, &p->key_scratch, &p->key_capacity,
                                   sizeof(unsigned long long) * count);
}

double* ensure_red_scratch(pc_plan* p, size_t count) {
  size_t cap = p->red_capacity * sizeof(double);
  void* slot = p->red_scratch;
  void* r = grow(p, &slot, &cap, count * sizeof(double));
  p->red_scratch = static_cast<double*>(r);
  p->red_capacity = cap / sizeof(double);
  return p->red_scratch;
}

// ----------------------------------------------------------------------------
// Host layout: everything pc_plan_create computes before touching the device.
// ----------------------------------------------------------------------------
struct Layout {
  GridGeom g{};
  int64_t L = 0;
  std::vector<int32_t> perm;            // sorted -> caller
  std::vector<double> AB;               // sorted, interleaved (A, B)
  std::vector<double> Cw;               // sorted w in wavelengths (empty: coplanar)
  WStack ws;
  std::vector<uint32_t> cell;           // sorted
  std::vector<double> off;              // sorted, interleaved (s_u, s_v)
  std::vector<SpreadChunk> chunks;
  std::vector<FoldItem> fold;
  std::vector<uint8_t> tile_flags;      // 1 if any footprint reaches the tile
  std::vector<InterpItem> interp;       // interpolation work list
  int64_t n_partials = 0;
  bool quads = false;                   // chunks grouped by workgroup (see SpreadChunk)
  std::vector<int32_t> group_work;      // per workgroup: its longest item's visibilities
};

static double kernel_beta(int W) { return 2.30 * W; }

// Entries of the FFT's two-level twiddle table (matches the kernels' layout).
static int twiddle_entries(int M) { return 64 + std::max(1, M / 64); }

static int kernel_width(double eps) {
  if (!(eps > 0)) eps = 1e-5;
  int W = (int)std::ceil(std::log10(1.0 / eps)) + 1;
  return std::min(std::max(W, 2), kMaxWidth);
}

static void validate(const pc_geometry* g) {
  PC_REQUIRE(g != nullptr, "geometry is NULL");
  PC_REQUIRE(g->nvis > 0, "nvis must be > 0");
  PC_REQUIRE(g->nvis < (int64_t(1) << 31) - 1, "nvis must fit in int32");
  PC_REQUIRE(g->u != nullptr && g->v != nullptr, "u and v must not be NULL");
  PC_REQUIRE(g->npix >= 16 && g->npix <= 8192 && g->npix % 2 == 0,
             "npix must be even and in [16, 8192]");
  PC_REQUIRE(std::isfinite(g->fov_rad) && g->fov_rad > 0, "fov_rad must be finite and > 0");
  PC_REQUIRE(g->uv_units == PC_UV_WAVELENGTHS || g->uv_units == PC_UV_METRES,
             "uv_units must be PC_UV_WAVELENGTHS or PC_UV_METRES");
  if (g->uv_units == PC_UV_METRES)
    PC_REQUIRE(std::isfinite(g->freq_hz) && g->freq_hz > 0, "freq_hz must be > 0 for metres");
  PC_REQUIRE(g->precision == PC_PREC_FP32 || g->precision == PC_PREC_FP64,
             "precision must be PC_PREC_FP32 or PC_PREC_FP64");
  const double dl = g->fov_rad / g->npix;
  const double lmax = (g->npix / 2) * dl;
  PC_REQUIRE(2.0 * lmax * lmax < 1.0, "field of view reaches l^2 + m^2 >= 1");
  if (g->upsamp > 0 && g->upsamp != 2.0) fail(PC_ERR_UNSUPPORTED, "only upsamp = 2 is supported");
  for (int64_t k = 0; k < g->nvis; ++k) {
    if (!std::isfinite(g->u[k]) || !std::isfinite(g->v[k]))
      fail(PC_ERR_INVALID_ARG, "non-finite uv at index " + std::to_string(k));
    if (g->w && !std::isfinite(g->w[k]))
      fail(PC_ERR_INVALID_ARG, "non-finite w at index " + std::to_string(k));
  }
}

static bool has_w(const pc_geometry* g) {
  if (!g->w) return false;
  for (int64_t k = 0; k < g->nvis; ++k)
    if (g->w[k] != 0.0) return true;
  return false;
}

// Planes of the w-stacked adjoint.  The direction factor c = n - 1 spans
// [c_min, 0], c_min at the image corner (a = b = -n/2); planes are dw =
// 1 / (4 half) apart (half = -c_min / 2) and cover [w_min, w_max] (of |w|)
// with W / 2 planes of margin on each side, centred on the range.
static WStack w_planes(const GridGeom& g, double wmin, double wmax) {
  WStack ws;
  const double lmax = (g.n / 2) * g.dl;
  const double cmin = n_minus_one(lmax, lmax);
  const double half = -0.5 * cmin;
  ws.cmid = -half;
  ws.dw = 1.0 / (4.0 * half);
  const double span = (wmax - wmin) / ws.dw;
  PC_REQUIRE(span < 1e6, "w range needs more than 10^6 planes");
  ws.nplanes = (int)std::ceil(span) + g.W + 1;
  ws.w0 = 0.5 * (wmin + wmax) - 0.5 * (ws.nplanes - 1) * ws.dw;
  ws.nquad = g.W + 60;
  return ws;
}

static Layout build_layout(const pc_geometry* geo, bool full) {
  validate(geo);
  const bool with_w = has_w(geo);
  if (with_w && geo->precision != PC_PREC_FP32)
    fail(PC_ERR_UNSUPPORTED, "non-coplanar baselines (w != 0) need an FP32 plan");
  Layout lay;
  const int64_t L = geo->nvis;
  const int n = geo->npix, M = 2 * n, W = kernel_width(geo->nufft_eps);
  const double dl = geo->fov_rad / n;
  const double scale = geo->uv_units == PC_UV_METRES ? geo->freq_hz / 299792458.0 : 1.0;
  GridGeom& g = lay.g;
  g.n = n;
  g.M = M;
  g.W = W;
  g.beta64 = kernel_beta(W);
  g.beta = (float)g.beta64;
  g.dl = dl;
  lay.L = L;

  // Per-visibility phase rates and first cells (unwrapped, in [-W/2, M)).
  std::vector<double> A(L), B(L);
  std::vector<int32_t> c0u(L), c0v(L);
  std::vector<double> su(L), sv(L);
  int64_t lo_u = INT64_MAX, hi_u = INT64_MIN, lo_v = INT64_MAX, hi_v = INT64_MIN;
  for (int64_t k = 0; k < L; ++k) {
    const double a = geo->u[k] * scale * dl, b = geo->v[k] * scale * dl;
    A[k] = a;
    B[k] = b;
    // The gridded adjoint takes Re(h e^{+j2pi(ul + vm + wc)}) = Re(h* e^{+j2pi(-ul - vm - wc)}):
    // a visibility with w < 0 is gridded as its conjugate at (-u, -v, -w), so
    // that the w-planes need only cover [min |w|, max |w|].  The direct sums
    // keep (A, B) as given.
    const bool flip = with_w && geo->w[k] < 0;
    const double ga = flip ? -a : a, gb = flip ? -b : b;
    const double xu = M * (ga + 0.5 - std::floor(ga + 0.5));
    const double xv = M * (gb + 0.5 - std::floor(gb + 0.5));
    const double mu = std::ceil(xu - 0.5 * W), mv = std::ceil(xv - 0.5 * W);
    c0u[k] = (int32_t)mu;
    c0v[k] = (int32_t)mv;
    su[k] = mu - xu;  // in (-W/2, -W/2 + 1]
    sv[k] = mv - xv;
    lo_u = std::min<int64_t>(lo_u, c0u[k]);
    hi_u = std::max<int64_t>(hi_u, c0u[k] + W - 1);
    lo_v = std::min<int64_t>(lo_v, c0v[k]);
    hi_v = std::max<int64_t>(hi_v, c0v[k] + W - 1);
  }
  // Band: a tile-aligned window holding every footprint without wrapping, or
  // the whole periodic grid when footprints cross the grid edge.
  const int T = kTile;
  auto band = [&](int64_t lo, int64_t hi, int32_t& b0, int32_t& nb) {
    if (lo < 0 || hi > M - 1) {
      b0 = 0;
      nb = M;
      return true;
    }
    b0 = (int32_t)(lo / T) * T;
    int64_t b1 = ((hi + 1 + T - 1) / T) * T;
    nb = (int32_t)(std::min<int64_t>(b1, M) - b0);
    return false;
  };
  const bool wu = band(lo_u, hi_u, g.u0, g.nu);
  const bool wv = band(lo_v, hi_v, g.v0, g.nv);
  g.wrap = (wu || wv) ? 1 : 0;
  if (g.wrap) {  // one periodic mode for both axes keeps the kernels simple
    g.u0 = g.v0 = 0;
    g.nu = g.nv = M;
  }
  g.ntu = g.nu / T;
  g.ntv = g.nv / T;
  const int ntu = g.ntu, ntv = g.ntv;
  const int64_t ntiles = (int64_t)ntu * ntv;

  // Tile and spill class of each visibility.  Class order inside a tile:
  // 0 none, 1 spills down (+v) only, 2 spills both ways, 3 spills right (+u)
  // only, so that the sets {down, both}, {both, right}, {both} are ranges.
  std::vector<int64_t> key(L);
  for (int64_t k = 0; k < L; ++k) {
    int32_t cu = ((c0u[k] % M) + M) % M, cv = ((c0v[k] % M) + M) % M;
    int32_t ru = cu - g.u0, rv = cv - g.v0;
    int32_t tu = ru / T, tv = rv / T;
    bool sr = (ru % T) > T - W, sd = (rv % T) > T - W;
    int cls = sd ? (sr ? 2 : 1) : (sr ? 3 : 0);
    key[k] = ((int64_t)tv * ntu + tu) * 4 + cls;
    c0u[k] = cu;
    c0v[k] = cv;
  }
  // Sort by (tile, spill class, first-cell block within the tile): a stable
  // counting sort on the block of the first cell (square blocks of
  // spread_block(W) cells on the absolute fine grid, counted from the tile's
  // first block), then a stable counting sort on (tile, class).  Visibilities
  // sharing a block end up adjacent, which the spreading kernel exploits by
  // accumulating them in registers over one window.
  std::vector<int32_t> order(L);
  {
    const int RB = spread_block(W);
    const int nbk = T / RB + 2;  // blocks a tile's first cells can fall in, per axis
    std::vector<int64_t> c((size_t)nbk * nbk + 1, 0);
    auto local = [&](int64_t k) {
      const int32_t ou = g.u0 + ((c0u[k] - g.u0) / T) * T;
      const int32_t ov = g.v0 + ((c0v[k] - g.v0) / T) * T;
      const int32_t bu = c0u[k] / RB - ou / RB, bv = c0v[k] / RB - ov / RB;
      return (int64_t)bv * nbk + bu;
    };
    for (int64_t k = 0; k < L; ++k) c[local(k) + 1]++;
    for (size_t i = 0; i + 1 < c.size(); ++i) c[i + 1] += c[i];
    for (int64_t k = 0; k < L; ++k) order[c[local(k)]++] = (int32_t)k;
  }
  std::vector<int64_t> cnt(ntiles * 4 + 1, 0);
  for (int64_t k = 0; k < L; ++k) cnt[key[k] + 1]++;
  for (int64_t i = 0; i < ntiles * 4; ++i) cnt[i + 1] += cnt[i];
  std::vector<int64_t> bstart(cnt.begin(), cnt.end());  // class starts
  lay.perm.resize(L);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < L; ++i) {
      const int32_t k = order[i];
      lay.perm[pos[key[k]]++] = k;
    }
  }
  if (with_w) {
    double wmin = INFINITY, wmax = -INFINITY;
    for (int64_t k = 0; k < L; ++k) {  // |w|: negative w is gridded conjugated
      wmin = std::min(wmin, std::fabs(geo->w[k] * scale));
      wmax = std::max(wmax, std::fabs(geo->w[k] * scale));
    }
    lay.ws = w_planes(g, wmin, wmax);
    if (full) {
      lay.Cw.resize(L);
      for (int64_t s = 0; s < L; ++s) lay.Cw[s] = geo->w[lay.perm[s]] * scale;
    }
  }
  if (full) {
    lay.AB.resize(2 * L);
    lay.cell.resize(L);
    lay.off.resize(2 * L);
    for (int64_t s = 0; s < L; ++s) {
      const int32_t k = lay.perm[s];
      lay.AB[2 * s] = A[k];
      lay.AB[2 * s + 1] = B[k];
      lay.cell[s] = ((uint32_t)c0v[k] << 16) | (uint32_t)c0u[k];
      lay.off[2 * s] = su[k];
      lay.off[2 * s + 1] = sv[k];
    }
  }
  // Work list.
  auto tid = [&](int tv, int tu) -> int64_t {
    if (g.wrap) {
      tv = (tv + ntv) % ntv;
      tu = (tu + ntu) % ntu;
    } else if (tv < 0 || tu < 0) {
      return -1;
    }
    return (int64_t)tv * ntu + tu;
  };
  auto cls_beg = [&](int64_t t, int c) { return bstart[t * 4 + c]; };
  // gathered count of each tile: its own visibilities plus the spills of
  // its left, upper and upper-left neighbours
  auto gathered = [&](int tv, int tu, int64_t* rb, int64_t* re) {
    const int64_t t = (int64_t)tv * ntu + tu;
    for (int r = 0; r < 4; ++r) rb[r] = re[r] = 0;
    rb[0] = cls_beg(t, 0);
    re[0] = bstart[t * 4 + 4];  // end of tile t
    const int64_t tl = tid(tv, tu - 1), tup = tid(tv - 1, tu), tul = tid(tv - 1, tu - 1);
    if (tl >= 0 && tl != t) {  // left neighbour: classes both + right
      rb[1] = cls_beg(tl, 2);
      re[1] = bstart[tl * 4 + 4];
    }
    if (tup >= 0 && tup != t) {  // upper neighbour: classes down + both
      rb[2] = cls_beg(tup, 1);
      re[2] = cls_beg(tup, 3);
    }
    if (tul >= 0 && tul != t) {  // upper-left neighbour: class both
      rb[3] = cls_beg(tul, 2);
      re[3] = cls_beg(tul, 3);
    }
    int64_t total = 0;
    for (int r = 0; r < 4; ++r) total += re[r] - rb[r];
    return total;
  };
  // Sub-range [q0, q1) of a tile's gathered sequence (its four ranges
  // concatenated) as an item's four ranges.
  auto sub_ranges = [](const int64_t* rb, const int64_t* re, int64_t q0, int64_t q1,
                       SpreadChunk& ch) {
    int64_t acc = 0;
    for (int r = 0; r < 4; ++r) {
      const int64_t len = re[r] - rb[r];
      const int64_t a = std::max<int64_t>(q0, acc), b = std::min<int64_t>(q1, acc + len);
      if (b > a) {
        ch.beg[r] = (int32_t)(rb[r] + (a - acc));
        ch.end[r] = (int32_t)(rb[r] + (b - acc));
      } else {
        ch.beg[r] = ch.end[r] = 0;
      }
      acc += len;
    }
  };
  auto work = [](const SpreadChunk& c) {
    int64_t w = 0;
    for (int r = 0; r < 4; ++r) w += c.end[r] - c.beg[r];
    return w;
  };
  std::vector<int64_t> totals((size_t)ntiles, 0);
  lay.tile_flags.assign(ntiles, 0);
  for (int tv = 0; tv < ntv; ++tv)
    for (int tu = 0; tu < ntu; ++tu) {
      int64_t rb[4], re[4];
      const int64_t t = (int64_t)tv * ntu + tu;
      totals[t] = gathered(tv, tu, rb, re);
      // Tiles no footprint reaches get no work item and are never written;
      // the first FFT pass reads them as zeros from the occupancy flags.
      lay.tile_flags[t] = totals[t] > 0 ? 1 : 0;
      // interpolation: the tile's own visibilities (first cell inside it)
      for (int64_t q = bstart[t * 4]; q < bstart[t * 4 + 4]; q += kInterpChunk)
        lay.interp.push_back(InterpItem{(int32_t)t, (int32_t)q,
                                        (int32_t)std::min<int64_t>(q + kInterpChunk,
                                                                   bstart[t * 4 + 4]),
                                        0});
    }
  lay.quads = geo->precision == PC_PREC_FP32 && W <= 8;
  if (lay.quads) {
    // Grouped spread: workgroups of G = kSpreadQuad waves.  A tile with at
    // most kq visibilities is one wave's item, packed G to a workgroup with
    // items of similar length; a heavier tile is cut into chunks of at most
    // 4 kq, each shared by the G waves of one workgroup (combine), which write
    // the tile itself when one chunk covers it and a partial tile otherwise.
    // kq is the largest of 1024, 512, ..., 64 that still gives at least 1536
    // workgroups, so that the longest work stays short against the whole
    // launch while the partial tiles to fold stay few.
    constexpr int G = kSpreadQuad;
    const int64_t min_groups = 1536;
    auto groups_for = [&](int64_t kq) {
      int64_t light = 0, heavy = 0;
      for (int64_t t = 0; t < ntiles; ++t) {
        if (totals[t] == 0) continue;
        if (totals[t] <= kq)
          ++light;
        else
          heavy += (totals[t] + 4 * kq - 1) / (4 * kq);
      }
      return heavy + (light + G - 1) / G;
    };
    int64_t kq = 64;
    for (int64_t c = 1024; c >= 64; c /= 2)
      if (groups_for(c) >= min_groups) {
        kq = c;
        break;
      }
    struct Group {
      int64_t work;
      SpreadChunk c[G];
    };
    std::vector<Group> groups;
    std::vector<SpreadChunk> light;
    for (int tv = 0; tv < ntv; ++tv)
      for (int tu = 0; tu < ntu; ++tu) {
        const int64_t t = (int64_t)tv * ntu + tu;
        const int64_t total = totals[t];
        if (total == 0) continue;
        int64_t rb[4], re[4];
        gathered(tv, tu, rb, re);
        if (total <= kq) {
          SpreadChunk c{};
          c.tile = (int32_t)t;
          c.slot = -1;
          sub_ranges(rb, re, 0, total, c);
          light.push_back(c);
          continue;
        }
        const int64_t nch = (total + 4 * kq - 1) / (4 * kq);
        if (nch > 1) {
          lay.fold.push_back(FoldItem{(int32_t)t, (int32_t)lay.n_partials, (int32_t)nch, 0});
        }
        for (int64_t c = 0; c < nch; ++c) {
          const int64_t q0 = total * c / nch, q1 = total * (c + 1) / nch;
          Group gr{};
          gr.work = 0;
          for (int w = 0; w < G; ++w) {
            SpreadChunk& ch = gr.c[w];
            ch.tile = (int32_t)t;
            ch.slot = nch > 1 ? (int32_t)(lay.n_partials + c) : -1;
            ch.combine = 1;
            sub_ranges(rb, re, q0 + (q1 - q0) * w / G, q0 + (q1 - q0) * (w + 1) / G, ch);
            gr.work = std::max(gr.work, work(ch));
          }
          groups.push_back(gr);
        }
        if (nch > 1) lay.n_partials += nch;
      }
    std::stable_sort(light.begin(), light.end(), [&](const SpreadChunk& a, const SpreadChunk& b) {
      return work(a) > work(b);
    });
    for (size_t i = 0; i < light.size(); i += G) {
      Group gr{};
      gr.work = work(light[i]);
      for (int w = 0; w < G; ++w) {
        if (i + w < light.size()) {
          gr.c[w] = light[i + w];
        } else {
          gr.c[w] = SpreadChunk{};
          gr.c[w].tile = -1;
          gr.c[w].slot = -1;
        }
        gr.c[w].combine = 0;
      }
      groups.push_back(gr);
    }
    // longest workgroups first: the dense uv core's work starts before the
    // many short items, which then fill in around it (greedy longest-first)
    std::stable_sort(groups.begin(), groups.end(),
                     [](const Group& a, const Group& b) { return a.work > b.work; });
    for (const Group& gr : groups) {
      for (int w = 0; w < G; ++w) lay.chunks.push_back(gr.c[w]);
      lay.group_work.push_back((int32_t)gr.work);
    }
    return lay;
  }
  // One wave per item (FP64 plans, kernel widths above 8).  Split tiles whose
  // gathered count exceeds kChunk: 256 visibilities keeps the longest item
  // short when few items exist (the spread is then bound by its longest work
  // item); with many items the spread is throughput-bound, and 512 halves the
  // partial tiles to fold.
  int64_t kChunk = 256;
  {
    int64_t items512 = 0;
    for (int64_t t = 0; t < ntiles; ++t)
      if (totals[t] > 0) items512 += (totals[t] + 511) / 512;
    if (items512 >= 7680) kChunk = 512;  // >= 3 waves of work items per wave slot
  }
  for (int tv = 0; tv < ntv; ++tv)
    for (int tu = 0; tu < ntu; ++tu) {
      const int64_t t = (int64_t)tv * ntu + tu;
      const int64_t total = totals[t];
      if (total == 0) continue;
      int64_t rb[4], re[4];
      gathered(tv, tu, rb, re);
      const int64_t nch = std::max<int64_t>(1, (total + kChunk - 1) / kChunk);
      if (nch == 1) {
        SpreadChunk c{};
        c.tile = (int32_t)t;
        c.slot = -1;
        sub_ranges(rb, re, 0, total, c);
        lay.chunks.push_back(c);
        continue;
      }
      FoldItem f{(int32_t)t, (int32_t)lay.n_partials, (int32_t)nch, 0};
      lay.fold.push_back(f);
      for (int64_t c = 0; c < nch; ++c) {
        SpreadChunk ch{};
        ch.tile = (int32_t)t;
        ch.slot = (int32_t)(lay.n_partials + c);
        sub_ranges(rb, re, total * c / nch, total * (c + 1) / nch, ch);
        lay.chunks.push_back(ch);
      }
      lay.n_partials += nch;
    }
  // Longest work items first: the dense uv core's items start before the
  // many short ones, which then fill in around them (greedy longest-first).
  std::stable_sort(lay.chunks.begin(), lay.chunks.end(),
                   [&](const SpreadChunk& a, const SpreadChunk& b) { return work(a) > work(b); });
  for (const SpreadChunk& c : lay.chunks) lay.group_work.push_back((int32_t)work(c));
  return lay;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_q).
static void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// psi(a) = (W/2) int_{-1}^{1} phi(z) cos(pi a W z / M) dz, the Fourier
// transform of the spreading kernel at output frequency a; corr = (-1)^a/psi.
static std::vector<double> correction_table(const GridGeom& g) {
  std::vector<double> x, w;
  gauss_legendre(2 * g.W + 120, x, w);
  std::vector<double> c(g.n);
  for (int i = 0; i < g.n; ++i) {
    const int a = i - g.n / 2;
    double s = 0;
    for (size_t q = 0; q < x.size(); ++q) {
      const double phi = std::exp(g.beta64 * (std::sqrt(1.0 - x[q] * x[q]) - 1.0));
      s += w[q] * phi * std::cos(M_PI * a * g.W * x[q] / g.M);
    }
    const double psi = 0.5 * g.W * s;
    c[i] = ((a & 1) ? -1.0 : 1.0) / psi;
  }
  return c;
}

static size_t layout_bytes(const Layout& lay, int prec) {
  const GridGeom& g = lay.g;
  const size_t cb = prec == PC_PREC_FP64 ? 16 : 8, rb = cb / 2;
  size_t b = 0;
  auto add = [&](size_t x) { b += pool_class(std::max<size_t>(x, 256)); };
  add(lay.L * 4);                            // perm
  add(lay.L * 16);                           // AB
  add(lay.L * 4);                            // cell
  add(lay.L * 2 * rb);                       // off
  add(lay.chunks.size() * sizeof(SpreadChunk));
  add(lay.fold.size() * sizeof(FoldItem));
  add(lay.tile_flags.size());
  add(lay.interp.size() * sizeof(InterpItem));
  add((size_t)g.nu * g.nv * cb);             // grid band
  add((size_t)g.nv * g.n * cb);              // H
  add((size_t)lay.n_partials * kTile * kTile * cb);
  add((size_t)twiddle_entries(g.M) * cb);    // twiddles
  add((size_t)g.n * rb);                     // correction
  add(256 + 4 * kMaxRowWords);               // max key, row mask
  add(lay.L * cb);                           // vis scratch
  if (lay.ws.nplanes > 0) {
    add(lay.L * 8);                          // w
    add(lay.L * cb);                         // one plane's weighted visibilities
    add((size_t)lay.ws.nquad * 16);          // Psi quadrature
  }
  return b;
}

}  // namespace pc

using namespace pc;

extern "C" pc_status pc_device_pool_trim_impl(int32_t device, size_t* released) {
  PC_REQUIRE(device >= 0, "device must be >= 0");
  const size_t n = pool_trim(device);
  if (released) *released = n;
  return PC_OK;
}

extern "C" pc_status pc_plan_footprint_impl(const pc_geometry* geom, size_t* bytes) {
  PC_REQUIRE(bytes != nullptr, "bytes is NULL");
  Layout lay = build_layout(geom, false);
  *bytes = layout_bytes(lay, geom->precision);
  return PC_OK;
}

extern "C" pc_status pc_plan_create_impl(const pc_geometry* geom, void* stream, pc_plan** out) {
  PC_REQUIRE(out != nullptr, "out is NULL");
  *out = nullptr;
  Layout lay = build_layout(geom, true);
  hipStream_t s = (hipStream_t)stream;
  pc_plan* p = new pc_plan();
  try {
    PC_HIP(hipGetDevice(&p->device));
    p->precision = geom->precision;
    p->L = lay.L;
    p->g = lay.g;
    p->n_chunks = (int64_t)lay.chunks.size();
    p->n_partials = lay.n_partials;
    p->n_fold = (int64_t)lay.fold.size();
    p->n_interp = (int64_t)lay.interp.size();
    p->spread_quads = lay.quads;
    p->chunk_work = lay.group_work;
    const GridGeom& g = lay.g;
    const bool f64 = geom->precision == PC_PREC_FP64;
    const size_t cb = f64 ? 16 : 8, rb = cb / 2;
    const int64_t L = lay.L;

    p->perm = (int32_t*)dalloc(p, L * 4);
    p->AB = (double*)dalloc(p, L * 16);
    p->cell = (uint32_t*)dalloc(p, L * 4);
    p->off = dalloc(p, L * 2 * rb);
    p->chunks = (SpreadChunk*)dalloc(p, lay.chunks.size() * sizeof(SpreadChunk));
    p->fold = (FoldItem*)dalloc(p, lay.fold.size() * sizeof(FoldItem));
    p->tile_flags = (uint8_t*)dalloc(p, lay.tile_flags.size());
    p->interp = (InterpItem*)dalloc(p, lay.interp.size() * sizeof(InterpItem));
    p->grid = dalloc(p, (size_t)g.nu * g.nv * cb);
    p->H = dalloc(p, (size_t)g.nv * g.n * cb);
    p->partials = dalloc(p, (size_t)lay.n_partials * kTile * kTile * cb);
    p->twiddle = dalloc(p, (size_t)twiddle_entries(g.M) * cb);
    p->corr = dalloc(p, (size_t)g.n * rb);
    p->maxkey = (unsigned long long*)dalloc(p, 256 + 4 * kMaxRowWords);
    p->rowmask = (uint32_t*)((unsigned char*)p->maxkey + 256);
    p->vis_scratch = dalloc(p, L * cb);
    p->ws = lay.ws;
    if (lay.ws.nplanes > 0) {
      p->Cw = (double*)dalloc(p, L * 8);
      p->wvals = dalloc(p, L * cb);
      p->wquad = (double*)dalloc(p, (size_t)lay.ws.nquad * 16);
    }

    // Host staging of converted tables; copies complete before return.
    PC_HIP(hipMemcpyAsync(p->perm, lay.perm.data(), L * 4, hipMemcpyHostToDevice, s));
    PC_HIP(hipMemcpyAsync(p->AB, lay.AB.data(), L * 16, hipMemcpyHostToDevice, s));
    PC_HIP(hipMemcpyAsync(p->cell, lay.cell.data(), L * 4, hipMemcpyHostToDevice, s));
    std::vector<float> off32;
    if (f64) {
      PC_HIP(hipMemcpyAsync(p->off, lay.off.data(), L * 16, hipMemcpyHostToDevice, s));
    } else {
      off32.resize(2 * L);
      for (int64_t i = 0; i < 2 * L; ++i) off32[i] = (float)lay.off[i];
      PC_HIP(hipMemcpyAsync(p->off, off32.data(), L * 8, hipMemcpyHostToDevice, s));
    }
    if (!lay.chunks.empty())
      PC_HIP(hipMemcpyAsync(p->chunks, lay.chunks.data(), lay.chunks.size() * sizeof(SpreadChunk),
                            hipMemcpyHostToDevice, s));
    PC_HIP(hipMemcpyAsync(p->tile_flags, lay.tile_flags.data(), lay.tile_flags.size(),
                          hipMemcpyHostToDevice, s));
    PC_HIP(hipMemcpyAsync(p->interp, lay.interp.data(), lay.interp.size() * sizeof(InterpItem),
                          hipMemcpyHostToDevice, s));
    if (!lay.fold.empty())
      PC_HIP(hipMemcpyAsync(p->fold, lay.fold.data(), lay.fold.size() * sizeof(FoldItem),
                            hipMemcpyHostToDevice, s));
    // Two-level twiddle table for exp(+2 pi i t / M): lo[q] = exp(2 pi i q / M),
    // q < 64, then hi[j] = exp(2 pi i 64 j / M), j < max(1, M / 64); FP64,
    // rounded once.
    const int ntw = twiddle_entries(g.M);
    std::vector<double> tw64(2 * (size_t)ntw);
    for (int q = 0; q < ntw; ++q) {
      const double t = q < 64 ? (double)q : 64.0 * (q - 64);
      const double ang = 2.0 * M_PI * t / g.M;
      tw64[2 * q] = std::cos(ang);
      tw64[2 * q + 1] = std::sin(ang);
    }
    std::vector<double> wq;
    if (lay.ws.nplanes > 0) {
      PC_HIP(hipMemcpyAsync(p->Cw, lay.Cw.data(), L * 8, hipMemcpyHostToDevice, s));
      // Psi(xi) = (W/2) int_{-1}^{1} phi(z) cos(pi W z xi) dz: the nodes in
      // (0, 1] of an even Gauss-Legendre rule, each weight doubled
      std::vector<double> x, w;
      gauss_legendre(2 * lay.ws.nquad, x, w);
      for (size_t q = 0; q < x.size(); ++q) {
        if (x[q] <= 0) continue;
        const double phi = std::exp(g.beta64 * (std::sqrt(1.0 - x[q] * x[q]) - 1.0));
        wq.push_back(x[q]);
        wq.push_back(g.W * w[q] * phi);
      }
      PC_REQUIRE((int)wq.size() == 2 * lay.ws.nquad, "quadrature nodes");
      // the device evaluates Psi on xi in [-1/4, 1/4] (the range of
      // dw (c' - c_mid)) as a Chebyshev series in 4 xi, interpolated at the
      // Chebyshev points; checked here against the quadrature itself
      auto psi = [&](double xi) {
        double sum = 0.0;
        for (int q = 0; q < lay.ws.nquad; ++q)
          sum += wq[2 * q + 1] * std::cos(M_PI * g.W * wq[2 * q] * xi);
        return sum;
      };
      constexpr int K = kPsiCheb;
      std::vector<double> fv(K), cheb(K, 0.0);
      for (int j = 0; j < K; ++j) fv[j] = psi(0.25 * std::cos(M_PI * (j + 0.5) / K));
      for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int j = 0; j < K; ++j) acc += fv[j] * std::cos(M_PI * k * (j + 0.5) / K);
        cheb[k] = (k == 0 ? 1.0 : 2.0) * acc / K;
      }
      for (int t = 0; t <= 64; ++t) {
        const double x = -1.0 + t / 32.0;
        double b1 = 0.0, b2 = 0.0;
        for (int k = K - 1; k >= 1; --k) {
          const double b0 = 2.0 * x * b1 - b2 + cheb[k];
          b2 = b1;
          b1 = b0;
        }
        const double ser = x * b1 - b2 + cheb[0], ref = psi(0.25 * x);
        PC_REQUIRE(std::fabs(ser - ref) <= 1e-12 * std::fabs(psi(0.0)),
                   "Chebyshev series of the w correction");
      }
      PC_REQUIRE(K <= 2 * lay.ws.nquad, "w correction table size");
      PC_HIP(hipMemcpyAsync(p->wquad, cheb.data(), K * 8, hipMemcpyHostToDevice, s));
      PC_HIP(hipStreamSynchronize(s));  // (cheb is a local)
    }
    std::vector<double> corr64 = correction_table(g);
    std::vector<float> tw32, corr32;
    if (f64) {
      PC_HIP(hipMemcpyAsync(p->twiddle, tw64.data(), ntw * 16, hipMemcpyHostToDevice, s));
      PC_HIP(hipMemcpyAsync(p->corr, corr64.data(), g.n * 8, hipMemcpyHostToDevice, s));
    } else {
      tw32.resize(2 * (size_t)ntw);
      for (size_t i = 0; i < tw32.size(); ++i) tw32[i] = (float)tw64[i];
      corr32.resize(g.n);
      for (int i = 0; i < g.n; ++i) corr32[i] = (float)corr64[i];
      PC_HIP(hipMemcpyAsync(p->twiddle, tw32.data(), ntw * 8, hipMemcpyHostToDevice, s));
      PC_HIP(hipMemcpyAsync(p->corr, corr32.data(), g.n * 4, hipMemcpyHostToDevice, s));
    }
    PC_HIP(hipEventCreate(&p->ev_a));
    PC_HIP(hipEventCreate(&p->ev_b));
    PC_HIP(hipStreamSynchronize(s));
  } catch (...) {
    plan_release(p);
    delete p;
    throw;
  }
  *out = p;
  return PC_OK;
}
