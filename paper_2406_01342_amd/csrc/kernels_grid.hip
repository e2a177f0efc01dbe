// Gridding path of the measurement operator (paper Sect. 5.2: the adjoint and
// forward as type-1 / type-2 non-uniform FFTs).
//
// Adjoint (Eq. adjoint-phi) as four launches:
//   spread   sorted visibilities -> fine-grid band, one workgroup per output
//            tile (kTile x kTile cells) accumulating in LDS; every band tile is
//            written exactly once (no global atomics, no zero-fill pass).  Hot
//            tiles are split into several work items writing partial tiles.
//   fold     sums the partial tiles of split tiles, in a fixed order.
//   pass A   per band row: inverse FFT of length M along u in LDS, keeping the
//            n central frequencies (input pruned to the band, output pruned).
//   pass B   per group of NB image rows: inverse FFT along v in LDS of the
//            pass-A columns, keeping n frequencies, then the apodisation and
//            1/n(l, m) correction, the image write and a fused max |eta|.
// Forward by interpolation (type-2): the same passes transposed with the
// opposite sign, then a w x w gather per visibility.
//
// Non-coplanar baselines (Sect. 2.1, Eq. phi-plane): the adjoint is
// w-stacked (planes and their kernel in the WStack comment).  Per plane, one
// small kernel weights the visibilities by the plane's kernel value (zero
// beyond its reach), the spread and pass A run unchanged, and pass B rotates
// each output pixel by the plane's phase exp(2 pi i w_j c') and adds the real
// part into the image; a last kernel divides by Psi(dw c') and takes the
// maximum.
#include <algorithm>
#include <cstring>
#include <memory>

#include "common.h"
#include "fft_lds.h"

namespace pc {

template <typename R>
__device__ __forceinline__ R es_kernel(R z, R beta) {
  // exponential of semicircle: exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1
  R t = R(1) - z * z;
  if (!(t > R(0))) return R(0);
  if constexpr (sizeof(R) == 4) {
    // hardware square root (about 1 ulp): the correctly rounded expansion
    // costs a dozen more instructions for no gain at this accuracy
    return __expf(beta * (__builtin_amdgcn_sqrtf(t) - 1.0f));
  } else {
    return exp(beta * (sqrt(t) - 1.0));
  }
}

// Tap position relative to an output tile's origin; returns false if the tap
// falls outside the tile.  In periodic (wrap) mode base is in (-W, M - W].
__device__ __forceinline__ bool tap_local(int base, int t, int M, int wrap, int& out) {
  int x = base + t;
  if (wrap && x < 0) x += M;
  out = x;
  return (unsigned)x < (unsigned)kTile;
}

__device__ __forceinline__ int tile_base(int c, int origin, int M, int W, int wrap) {
  int b = c - origin;  // in (-M, M): both are cells of the periodic grid
  if (wrap) {
    if (b < 0) b += M;
    if (b > M - W) b -= M;
  }
  return b;
}

// Spreading layout: one wave per work item owns the output tile in LDS
// (planar re/im, row stride kTile + BS).  Its lanes cover a BS x BS window of
// cells (BS = 8 for kernel widths up to 8, else W): the union of the
// footprints of every visibility whose first cell lies in one RB x RB block
// (RB = BS - W + 1; 3 x 3 first cells for W = 6).  Visibilities are sorted by
// that block, so a run of them shares the window: each lane adds its cell's
// weight times the value into a register, and the sums go to LDS (a plain
// read-add-write: the lanes of one instruction address distinct cells and a
// wave's LDS operations complete in order) only when the block changes.  The
// wave stages 64 visibilities at a time, one per lane: the block key, the
// value, and the kernel weights already shifted onto the window's rows and
// columns (zero outside the visibility's own footprint), so that in the
// accumulation loop a lane reads its two weights at fixed offsets and spends
// one multiply and two FMAs per visibility.  No LDS atomics (whose per-lane
// serialisation made them the bottleneck), and each cell receives its
// contributions in a fixed order, so the result is bitwise reproducible.
// Hot tiles are split across work items upstream.
template <typename R, int W>
struct SpreadCfg {
  static constexpr int BS = spread_span(W);      // window side (cells)
  static constexpr int RB = spread_block(W);     // block side (first cells)
  static constexpr int NPASS = (BS * BS + 63) / 64;
  static constexpr int S = kTile + BS;           // LDS row stride
  static constexpr int TILE = kTile * S;         // reals per plane
  static constexpr int REC = 2 * BS + 4;         // wy[BS], wx[BS], re, im, key, pad
  static constexpr int STG = 64 * REC;
  static constexpr int U = 16;                   // visibilities per inner step
  static constexpr size_t lds_bytes = sizeof(R) * (2 * TILE + STG);
};

// Block key of a window origin (bu, bv) relative to the tile, both in
// (-BS, kTile): one integer, so that a run test is a single comparison.
__device__ __forceinline__ int block_key(int bu, int bv) { return ((bv + 64) << 8) | (bu + 64); }
constexpr int kNoBlock = -1;

// Adds a run's per-cell register sums into the LDS tile and clears them.
// single: the periodic grid is one tile wide, so window cells left of (or
// above) the tile wrap onto its other end.
template <typename R, int W>
__device__ __forceinline__ void spread_flush(int lane, int key, bool single, int M,
                                             R (&accr)[SpreadCfg<R, W>::NPASS],
                                             R (&acci)[SpreadCfg<R, W>::NPASS], R* tre,
                                             R* tim) {
  using C = SpreadCfg<R, W>;
  if (key != kNoBlock) {
    const int bu = (key & 0xff) - 64, bv = (key >> 8) - 64;
#pragma unroll
    for (int ps = 0; ps < C::NPASS; ++ps) {
      const int tap = lane + 64 * ps;
      const int a = tap / C::BS, b = tap - (tap / C::BS) * C::BS;
      int y = bv + a, x = bu + b;
      if (single) {
        y &= kTile - 1;
        x &= kTile - 1;
      }
      if ((C::BS * C::BS % 64 == 0 || tap < C::BS * C::BS) && (unsigned)y < (unsigned)kTile &&
          (unsigned)x < (unsigned)kTile) {
        tre[y * C::S + x] += accr[ps];
        tim[y * C::S + x] += acci[ps];
      }
    }
  }
#pragma unroll
  for (int ps = 0; ps < C::NPASS; ++ps) {
    accr[ps] = R(0);
    acci[ps] = R(0);
  }
}

// One staged visibility as fetched from global memory.
template <typename R>
struct VisIn {
  uint32_t cell;
  R su, sv;
  cpx<R> val;
};

// Position in the sorted arrays of the q-th visibility of a work item whose
// four ranges have cumulative lengths c1 <= c2 <= c3 and offsets b0..b3
// (plain values, so that no reference is selected at run time).
__device__ __forceinline__ int chunk_index(int q, int c1, int c2, int c3, int b0, int b1, int b2,
                                           int b3) {
  const int add = q < c1 ? b0 : (q < c2 ? b1 : (q < c3 ? b2 : b3));
  return q + add;
}

template <typename R>
__device__ __forceinline__ VisIn<R> fetch_vis(int s, const uint32_t* __restrict__ cell,
                                              const R* __restrict__ off,
                                              const cpx<R>* __restrict__ vals,
                                              const int32_t* __restrict__ perm) {
  VisIn<R> v;
  v.cell = cell[s];
  v.su = off[2 * s];
  v.sv = off[2 * s + 1];
  v.val = perm ? vals[perm[s]] : vals[s];
  return v;
}

template <typename R, int W>
__device__ __forceinline__ void spread_body(
    const GridGeom& g, const SpreadChunk& ch, const uint32_t* __restrict__ cell,
    const R* __restrict__ off, const cpx<R>* __restrict__ vals, const int32_t* __restrict__ perm,
    cpx<R>* __restrict__ grid, cpx<R>* __restrict__ partials) {
  using C = SpreadCfg<R, W>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x;
  R* tre = reinterpret_cast<R*>(smem_raw);
  R* tim = tre + C::TILE;
  R* stg = tim + C::TILE;  // [64][REC]
  const int tv = ch.tile / g.ntu, tu = ch.tile - tv * g.ntu;
  const int ov = g.v0 + tv * kTile, ou = g.u0 + tu * kTile;
  const bool single = g.wrap && g.M == kTile;
  const R inv = R(2) / R(W);
  const R beta = sizeof(R) == 4 ? (R)g.beta : (R)g.beta64;
  // cumulative range boundaries
  const int c1 = ch.end[0] - ch.beg[0];
  const int c2 = c1 + ch.end[1] - ch.beg[1];
  const int c3 = c2 + ch.end[2] - ch.beg[2];
  const int total = c3 + ch.end[3] - ch.beg[3];
  const int b0 = ch.beg[0], b1 = ch.beg[1] - c1, b2 = ch.beg[2] - c2, b3 = ch.beg[3] - c3;
  constexpr int NPASS = C::NPASS;
  constexpr int U = C::U;
  // The first batch's global loads go out before the tile is cleared; each
  // later batch's before the current batch's accumulation loop.
  VisIn<R> nx{0u, R(0), R(0), {R(0), R(0)}};
  if (lane < total)
    nx = fetch_vis<R>(chunk_index(lane, c1, c2, c3, b0, b1, b2, b3), cell, off, vals, perm);
  for (int i = lane; i < C::TILE; i += 64) {
    tre[i] = R(0);
    tim[i] = R(0);
  }
  // per-lane window cell (row a, column b) for each pass
  int ia[NPASS], ib[NPASS];
#pragma unroll
  for (int ps = 0; ps < NPASS; ++ps) {
    const int tap = lane + 64 * ps;
    const bool ok = C::BS * C::BS % 64 == 0 || tap < C::BS * C::BS;
    ia[ps] = ok ? tap / C::BS : 0;
    ib[ps] = ok ? C::BS + tap - (tap / C::BS) * C::BS : C::BS;  // wx row follows wy
  }
  int ckey = kNoBlock;
  R accr[NPASS], acci[NPASS];
#pragma unroll
  for (int ps = 0; ps < NPASS; ++ps) accr[ps] = acci[ps] = R(0);
#pragma unroll 1
  for (int base = 0; base < total; base += 64) {
    // stage one visibility per lane: weights shifted onto the window
    const int q = base + lane;
    R* my = stg + lane * C::REC;
    if (q < total) {
      const int cu = (int)(nx.cell & 0xffffu), cv = (int)(nx.cell >> 16);
      const int du = cu % C::RB, dv = cv % C::RB;
      const int bu = tile_base(cu - du, ou, g.M, C::BS, g.wrap);
      const int bv = tile_base(cv - dv, ov, g.M, C::BS, g.wrap);
      // the W taps of each axis land at window positions d .. d + W - 1
      // (d = dv or du < RB); the other BS - W positions are zero
#pragma unroll
      for (int j = 0; j < C::BS; ++j) my[j] = my[C::BS + j] = R(0);
#pragma unroll
      for (int t = 0; t < W; ++t) {
        my[dv + t] = es_kernel<R>((nx.sv + R(t)) * inv, beta);
        my[C::BS + du + t] = es_kernel<R>((nx.su + R(t)) * inv, beta);
      }
      my[2 * C::BS] = nx.val.x;
      my[2 * C::BS + 1] = nx.val.y;
      *reinterpret_cast<int*>(&my[2 * C::BS + 2]) = block_key(bu, bv);  // in the R-sized slot
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (q + 64 < total)
      nx = fetch_vis<R>(chunk_index(q + 64, c1, c2, c3, b0, b1, b2, b3), cell, off, vals, perm);
    const int nb = total - base < 64 ? total - base : 64;
#pragma unroll 1
    for (int v0 = 0; v0 < nb; v0 += U) {
      int key[U];
      R vr[U], vi[U], wg[U][NPASS];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // issue all LDS reads of the step first
        const R* kw = stg + (v0 + u) * C::REC;
        // records past the batch end hold a stale key and stale weights:
        // their key is replaced by kNoBlock below and their weights unused
        key[u] = *reinterpret_cast<const int*>(&kw[2 * C::BS + 2]);
        vr[u] = kw[2 * C::BS];
        vi[u] = kw[2 * C::BS + 1];
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) wg[u][ps] = kw[ia[ps]] * kw[ib[ps]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (v0 + u < nb) {
          const int k = __builtin_amdgcn_readfirstlane(key[u]);
          if (k != ckey) {  // same for every lane of the wave
            spread_flush<R, W>(lane, ckey, single, g.M, accr, acci, tre, tim);
            ckey = k;
          }
#pragma unroll
          for (int ps = 0; ps < NPASS; ++ps) {
            accr[ps] = fma(wg[u][ps], vr[u], accr[ps]);
            acci[ps] = fma(wg[u][ps], vi[u], acci[ps]);
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  spread_flush<R, W>(lane, ckey, single, g.M, accr, acci, tre, tim);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  cpx<R>* dst;
  size_t stride;
  if (ch.slot < 0) {
    dst = grid + (size_t)(tv * kTile) * g.nu + tu * kTile;
    stride = g.nu;
  } else {
    dst = partials + (size_t)ch.slot * kTile * kTile;
    stride = kTile;
  }
  for (int i = lane; i < kTile * kTile; i += 64) {
    const int y = i / kTile, x = i - y * kTile;
    dst[(size_t)y * stride + x] = {tre[y * C::S + x], tim[y * C::S + x]};
  }
}

// FP32 spreading for kernel widths up to 8, four visibilities per step.
//
// The wave's lanes again cover an 8 x 8 window of cells (lane = row a, column
// b), the union of the footprints of the visibilities whose first cell lies
// in one RB x RB block, and a run of visibilities sharing a block accumulates
// in registers.  What differs is how a lane gets its factors.  Each lane
// stages one visibility of a batch of 64 and writes its weights, already
// shifted onto the window, into two transposed tables: wy[a][j] (rows), and
// the column weights times the value as complex pairs, wx[b][j] =
// (wx_j[b] Re v_j, wx_j[b] Im v_j).  Consecutive visibilities j of one table
// row are adjacent, so 128-bit LDS reads hand a lane its factors for four
// visibilities: three reads and eight FMAs per lane for four visibilities
// (instead of two 32-bit weight reads, the broadcast value and key reads, a
// multiply and two FMAs per visibility).  Run boundaries are found once per
// batch (a ballot of "my block differs from my predecessor's"); a group of
// four with no boundary takes the straight path, a group with one flushes
// between its visibilities.  Table rows are padded (68 and 132 floats) so
// that the eight distinct rows a wave reads in one instruction fall in
// distinct banks; the staging writes one row at a time from all lanes.  The
// LDS tile holds interleaved complex cells (one 64-bit read-add-write per
// lane and flush).  Deterministic: each cell receives its terms in a fixed
// order.
// Groups of four visibilities whose LDS reads are issued together.
constexpr int kGroupsAhead = 4;

template <int W>
struct SpreadG {
  static constexpr int BS = 8;                  // window side
  static constexpr int RB = BS - W + 1;         // block side (first cells)
  static constexpr int S = kTile + 4;           // tile row stride (complex cells)
  static constexpr int TR = 68;                 // row-weight table row stride (floats)
  static constexpr int TRX = 132;               // column table row stride (floats)
  static constexpr int TILE_F = 2 * kTile * S;  // floats
  static constexpr int TAB_F = BS * (TR + TRX); // floats
  static constexpr size_t wave_bytes = sizeof(float) * (TILE_F + TAB_F);
  static constexpr size_t lds_bytes = kSpreadQuad * wave_bytes;
};

// Exponential-of-semicircle weight of a tap at distance x (cells) from the
// visibility, in the form the staging evaluates it: with R = W/2,
// phi = exp(beta (sqrt(1 - (x/R)^2) - 1)) = exp2(c1 sqrt(R^2 - x^2) - c0),
// c0 = beta log2(e), c1 = c0 / R.  |x| <= R for every tap of a footprint;
// max(., 0) only absorbs rounding at |x| = R.
__device__ __forceinline__ float es_weight(float x, float R2, float c1, float c0) {
  const float q = fmaxf(fmaf(-x, x, R2), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(c1, __builtin_amdgcn_sqrtf(q), -c0));
}

// Accumulates one work item into the wave's LDS region (its tile, then its
// tables) and leaves the tile there; the caller writes it out.
// perm: NULL when vals is in plan order, else the plan -> caller map.
template <int W>
__device__ __forceinline__ void spread_group_accumulate(
    const GridGeom& g, const SpreadChunk& ch, const uint32_t* __restrict__ cell,
    const float* __restrict__ off, const cpx<float>* __restrict__ vals,
    const int32_t* __restrict__ perm, float* __restrict__ tile, int lane) {
  using C = SpreadG<W>;
  static_assert(W >= 2 && W <= 8, "group spreading covers widths 2..8");
  float* tab = tile + C::TILE_F;        // wy [8][TR]
  float* tabx = tab + C::BS * C::TR;    // wx v as complex pairs [8][TRX]
  const int a = lane >> 3, b = lane & 7;
  const int tv = ch.tile / g.ntu, tu = ch.tile - tv * g.ntu;
  const int ov = g.v0 + tv * kTile, ou = g.u0 + tu * kTile;
  const bool single = g.wrap && g.M == kTile;
  constexpr float R = 0.5f * (float)W;
  const float c0 = g.beta * 1.44269504088896341f;  // beta log2(e)
  const float c1 = c0 / R;
  const int c1n = ch.end[0] - ch.beg[0];
  const int c2n = c1n + ch.end[1] - ch.beg[1];
  const int c3n = c2n + ch.end[2] - ch.beg[2];
  const int total = c3n + ch.end[3] - ch.beg[3];
  const int b0 = ch.beg[0], b1 = ch.beg[1] - c1n, b2 = ch.beg[2] - c2n, b3 = ch.beg[3] - c3n;
  {
    float4* t4 = reinterpret_cast<float4*>(tile);
    for (int i = lane; i < C::TILE_F / 4; i += 64) t4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (total <= 0) return;
  // Loads run ahead through three record buffers (batch k uses buffer k mod 3).
  // The cell, offsets and source index of batch k + 3 and the value of batch
  // k + 2 are issued while batch k is staged and summed; the value of a
  // caller-order input needs its source index, which was issued a batch
  // earlier, so no load waits on one issued just before it.  Lanes past the
  // end load the last record again (no branch around the loads, so that each
  // wait covers exactly the batch it consumes).
  struct Raw {
    uint32_t cell;
    float2 off;
    int32_t ld, sidx;  // the loaded index, and the record's plan position
    cpx<float> val;
  };
  // (for a plan-order input the index load reads the cell array instead and
  // is discarded, so that every path issues the same loads)
  const int32_t* src_arr = perm ? perm : reinterpret_cast<const int32_t*>(cell);
  auto load_pre = [&](Raw& rw, int q) {
    const int sidx = chunk_index(q < total ? q : total - 1, c1n, c2n, c3n, b0, b1, b2, b3);
    rw.cell = cell[sidx];
    rw.off = reinterpret_cast<const float2*>(off)[sidx];
    rw.ld = src_arr[sidx];
    rw.sidx = sidx;
  };
  // (the choice between them is made here, a batch after the index load)
  auto load_val = [&](Raw& rw) { rw.val = vals[perm ? rw.ld : rw.sidx]; };
  Raw rb0, rb1, rb2;
  load_pre(rb0, lane);
  load_val(rb0);
  load_pre(rb1, 64 + lane);
  load_pre(rb2, 128 + lane);
  load_val(rb1);
  const float* rwy = tab + a * C::TR;
  const float* rwx = tabx + b * C::TRX;
  int ckey = kNoBlock;
  float accr = 0.f, acci = 0.f;
  auto flush = [&]() {
    if (ckey != kNoBlock) {
      int y = ((ckey >> 8) - 64) + a, x = ((ckey & 0xff) - 64) + b;
      if (single) {
        y &= kTile - 1;
        x &= kTile - 1;
      }
      if ((unsigned)y < (unsigned)kTile && (unsigned)x < (unsigned)kTile) {
        float2* cp = reinterpret_cast<float2*>(tile) + y * C::S + x;
        float2 o = *cp;
        o.x += accr;
        o.y += acci;
        *cp = o;
      }
    }
    accr = 0.f;
    acci = 0.f;
  };
  // One batch of 64: stage from rk (batch k), reload rk with batch k + 3 and
  // the value of rk2 (batch k + 2), then sum.
  auto batch = [&](int base, Raw& rk, Raw& rk2) {
    const int q = base + lane;
    const bool valid = q < total;
    int key = kNoBlock, du = 0, dv = 0;
    float fy[W], fx[W], vr = 0.f, vi = 0.f;
    if (valid) {
      const int cu = (int)(rk.cell & 0xffffu), cv = (int)(rk.cell >> 16);
      du = cu % C::RB;
      dv = cv % C::RB;
      key = block_key(tile_base(cu - du, ou, g.M, C::BS, g.wrap),
                      tile_base(cv - dv, ov, g.M, C::BS, g.wrap));
      vr = rk.val.x;
      vi = rk.val.y;
      // tap t lies x = s + t cells from the visibility, s in (-R, -R + 1],
      // so |x| <= R (z = x / R in (-1, 1])
#pragma unroll
      for (int t = 0; t < W; ++t) {
        fy[t] = es_weight(rk.off.y + (float)t, R * R, c1, c0);
        fx[t] = es_weight(rk.off.x + (float)t, R * R, c1, c0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < W; ++t) fy[t] = fx[t] = 0.f;
    }
    load_pre(rk, q + 192);
    load_val(rk2);
    // run starts: a valid visibility whose block differs from its predecessor's
    const int prev = __shfl_up(key, 1, 64);
    const bool start = valid && (lane == 0 ? key != ckey : key != prev);
    const unsigned long long runs = __ballot(start);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Every lane writes the same table row at once (consecutive addresses, no
    // bank conflicts): window row a holds tap a - dv of the footprint, or zero
    // outside it, picked by selects over the RB possible shifts.
#pragma unroll
    for (int row = 0; row < C::BS; ++row) {
      float wy = 0.f, wx = 0.f;
#pragma unroll
      for (int d = 0; d < C::RB; ++d) {
        const int t = row - d;
        if (t >= 0 && t < W) {
          wy = dv == d ? fy[t] : wy;
          wx = du == d ? fx[t] : wx;
        }
      }
      tab[row * C::TR + lane] = wy;
      *reinterpret_cast<float2*>(tabx + row * C::TRX + 2 * lane) = make_float2(wx * vr, wx * vi);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int ng = ((total - base < 64 ? total - base : 64) + 3) >> 2;  // groups of four
#pragma unroll 1
    for (int g4 = 0; g4 < ng; g4 += kGroupsAhead) {
      float4 y[kGroupsAhead], xr[kGroupsAhead], xi[kGroupsAhead];
#pragma unroll
      for (int u = 0; u < kGroupsAhead; ++u) {  // every read of these groups first
        y[u] = *reinterpret_cast<const float4*>(rwy + 4 * (g4 + u));
        // (re, im) pairs of visibilities 4g, 4g + 1, then 4g + 2, 4g + 3
        const float4 p01 = *reinterpret_cast<const float4*>(rwx + 8 * (g4 + u));
        const float4 p23 = *reinterpret_cast<const float4*>(rwx + 8 * (g4 + u) + 4);
        xr[u] = make_float4(p01.x, p01.z, p23.x, p23.z);
        xi[u] = make_float4(p01.y, p01.w, p23.y, p23.w);
      }
#pragma unroll
      for (int u = 0; u < kGroupsAhead; ++u) {
        const unsigned bits = (unsigned)(runs >> (4 * (g4 + u))) & 0xfu;
        if (bits == 0u) {  // the group continues the current run
          accr = fmaf(y[u].x, xr[u].x, accr);
          acci = fmaf(y[u].x, xi[u].x, acci);
          accr = fmaf(y[u].y, xr[u].y, accr);
          acci = fmaf(y[u].y, xi[u].y, acci);
          accr = fmaf(y[u].z, xr[u].z, accr);
          acci = fmaf(y[u].z, xi[u].z, acci);
          accr = fmaf(y[u].w, xr[u].w, accr);
          acci = fmaf(y[u].w, xi[u].w, acci);
        } else {
          const int j0 = 4 * (g4 + u);
          if (bits & 1u) {
            flush();
            ckey = __builtin_amdgcn_readlane(key, j0);
          }
          accr = fmaf(y[u].x, xr[u].x, accr);
          acci = fmaf(y[u].x, xi[u].x, acci);
          if (bits & 2u) {
            flush();
            ckey = __builtin_amdgcn_readlane(key, j0 + 1);
          }
          accr = fmaf(y[u].y, xr[u].y, accr);
          acci = fmaf(y[u].y, xi[u].y, acci);
          if (bits & 4u) {
            flush();
            ckey = __builtin_amdgcn_readlane(key, j0 + 2);
          }
          accr = fmaf(y[u].z, xr[u].z, accr);
          acci = fmaf(y[u].z, xi[u].z, acci);
          if (bits & 8u) {
            flush();
            ckey = __builtin_amdgcn_readlane(key, j0 + 3);
          }
          accr = fmaf(y[u].w, xr[u].w, accr);
          acci = fmaf(y[u].w, xi[u].w, acci);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // the three batches of a step run unconditionally (the later ones may be
  // empty: no valid lane, zero weights, no groups), so that the loads in
  // flight are the same on every path and each wait covers just what it needs
#pragma unroll 1
  for (int base = 0; base < total; base += 192) {
    batch(base, rb0, rb2);
    batch(base + 64, rb1, rb0);
    batch(base + 128, rb2, rb1);
  }
  flush();
}

// Output address of a work item's tile: the band tile itself, or its
// partial slot.
__device__ __forceinline__ cpx<float>* spread_dst(const GridGeom& g, const SpreadChunk& ch,
                                                  cpx<float>* grid, cpx<float>* partials,
                                                  size_t& stride) {
  if (ch.slot < 0) {
    const int tv = ch.tile / g.ntu, tu = ch.tile - tv * g.ntu;
    stride = g.nu;
    return grid + (size_t)(tv * kTile) * g.nu + tu * kTile;
  }
  stride = kTile;
  return partials + (size_t)ch.slot * kTile * kTile;
}

// A workgroup of kSpreadQuad waves over as many work items (see
// SpreadChunk): each wave accumulates its item into its own LDS tile;
// independent items are written by their own wave, the shares of a combined
// tile are added in wave order and written once by the whole workgroup.
template <int W>
__device__ __forceinline__ void spread_quad_body(
    const GridGeom& g, const SpreadChunk* __restrict__ quad, const uint32_t* __restrict__ cell,
    const float* __restrict__ off, const cpx<float>* __restrict__ vals,
    const int32_t* __restrict__ perm, cpx<float>* __restrict__ grid,
    cpx<float>* __restrict__ partials) {
  using C = SpreadG<W>;
  constexpr int WAVE_F = C::TILE_F + C::TAB_F;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* region = reinterpret_cast<float*>(smem_raw);
  const SpreadChunk& ch = quad[w];
  const bool combine = quad[0].combine != 0;  // the same for every wave
  if (ch.tile >= 0)
    spread_group_accumulate<W>(g, ch, cell, off, vals, perm, region + w * WAVE_F, lane);
  size_t stride;
  if (!combine) {
    if (ch.tile < 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cpx<float>* dst = spread_dst(g, ch, grid, partials, stride);
    const float4* t4 = reinterpret_cast<const float4*>(region + w * WAVE_F);
    for (int i = lane; i < kTile * kTile / 2; i += 64) {  // two cells per lane and step
      const int y = i / (kTile / 2), x2 = i - y * (kTile / 2);
      *reinterpret_cast<float4*>(dst + (size_t)y * stride + 2 * x2) = t4[(y * C::S) / 2 + x2];
    }
    return;
  }
  __syncthreads();
  cpx<float>* dst = spread_dst(g, quad[0], grid, partials, stride);
  for (int i = threadIdx.x; i < kTile * kTile / 2; i += 64 * kSpreadQuad) {
    const int y = i / (kTile / 2), x2 = i - y * (kTile / 2);
    const int o = (y * C::S) / 2 + x2;
    float4 v = reinterpret_cast<const float4*>(region)[o];
#pragma unroll
    for (int k = 1; k < kSpreadQuad; ++k) {
      const float4 t = reinterpret_cast<const float4*>(region + k * WAVE_F)[o];
      v.x += t.x;
      v.y += t.y;
      v.z += t.z;
      v.w += t.w;
    }
    *reinterpret_cast<float4*>(dst + (size_t)y * stride + 2 * x2) = v;
  }
}

template <int W>
__global__ __launch_bounds__(64 * kSpreadQuad) void spread_quad_kernel(
    GridGeom g, const SpreadChunk* __restrict__ chunks, const uint32_t* __restrict__ cell,
    const float* __restrict__ off, const cpx<float>* __restrict__ vals,
    const int32_t* __restrict__ perm, cpx<float>* __restrict__ grid,
    cpx<float>* __restrict__ partials, unsigned long long* __restrict__ maxkey) {
  // the image maximum that the last pass accumulates starts from zero
  if (blockIdx.x == 0 && threadIdx.x == 0) *maxkey = 0ull;
  spread_quad_body<W>(g, chunks + (size_t)kSpreadQuad * blockIdx.x, cell, off, vals, perm, grid,
                      partials);
}

// One launch over the workgroups of several plans: items[b] = (job, group).
template <int W>
__global__ __launch_bounds__(64 * kSpreadQuad) void spread_quad_batch_kernel(
    const AdjJob* __restrict__ jobs, const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const AdjJob& J = jobs[it.x];
  if (it.y == 0 && threadIdx.x == 0) *J.maxkey = 0ull;  // every job has a group 0
  spread_quad_body<W>(J.g, J.chunks + (size_t)kSpreadQuad * it.y, J.cell, J.off, J.vals, J.perm,
                      J.grid, J.partials);
}

template <typename R, int W>
__global__ __launch_bounds__(64) void spread_kernel(
    GridGeom g, const SpreadChunk* __restrict__ chunks, const uint32_t* __restrict__ cell,
    const R* __restrict__ off, const cpx<R>* __restrict__ vals, const int32_t* __restrict__ perm,
    cpx<R>* __restrict__ grid, cpx<R>* __restrict__ partials,
    unsigned long long* __restrict__ maxkey) {
  // the image maximum that the last pass accumulates starts from zero (reset
  // here rather than by a launch of its own; the pass runs later on the stream)
  if (blockIdx.x == 0 && threadIdx.x == 0) *maxkey = 0ull;
  spread_body<R, W>(g, chunks[blockIdx.x], cell, off, vals, perm, grid, partials);
}

// One launch over the work items of several plans: items[b] = (job, item).
template <int W>
__global__ __launch_bounds__(64) void spread_batch_kernel(const AdjJob* __restrict__ jobs,
                                                          const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const AdjJob& J = jobs[it.x];
  if (it.y == 0 && threadIdx.x == 0) *J.maxkey = 0ull;  // every job has an item 0
  spread_body<float, W>(J.g, J.chunks[it.y], J.cell, J.off, J.vals, J.perm, J.grid, J.partials);
}

// Fold of a split tile: 64 cells per workgroup, kFoldSub threads per cell
// each summing every kFoldSub-th partial (kFoldBurst loads in flight), then the
// sub-sums are added in a fixed order (bitwise reproducible).
constexpr int kFoldSub = 8;
constexpr int kFoldBurst = 4;  // loads in flight per thread

template <typename R>
__device__ __forceinline__ void fold_body(const GridGeom& g, const FoldItem& it,
                                          const cpx<R>* __restrict__ partials,
                                          cpx<R>* __restrict__ grid) {
  __shared__ R sx[kFoldSub][64], sy[kFoldSub][64];
  const int c = threadIdx.x & 63, sub = threadIdx.x >> 6;
  const int i = blockIdx.y * 64 + c;
  const cpx<R>* src = partials + (size_t)it.first * kTile * kTile + i;
  R ax = 0, ay = 0;
  int q = sub;
  for (; q + (kFoldBurst - 1) * kFoldSub < it.count; q += kFoldBurst * kFoldSub) {
    cpx<R> v[kFoldBurst];
#pragma unroll
    for (int u = 0; u < kFoldBurst; ++u) v[u] = src[(size_t)(q + u * kFoldSub) * kTile * kTile];
#pragma unroll
    for (int u = 0; u < kFoldBurst; ++u) {
      ax += v[u].x;
      ay += v[u].y;
    }
  }
  for (; q < it.count; q += kFoldSub) {
    const cpx<R> v = src[(size_t)q * kTile * kTile];
    ax += v.x;
    ay += v.y;
  }
  sx[sub][c] = ax;
  sy[sub][c] = ay;
  __syncthreads();
  if (sub == 0) {
    R tx = 0, ty = 0;
#pragma unroll
    for (int k = 0; k < kFoldSub; ++k) {
      tx += sx[k][c];
      ty += sy[k][c];
    }
    const int tv = it.tile / g.ntu, tu = it.tile - tv * g.ntu;
    cpx<R>* dst = grid + (size_t)(tv * kTile) * g.nu + tu * kTile;
    const int y = i / kTile, x = i - y * kTile;
    dst[(size_t)y * g.nu + x] = {tx, ty};
  }
}

template <typename R>
__global__ __launch_bounds__(64 * kFoldSub) void fold_kernel(GridGeom g,
                                                           const FoldItem* __restrict__ items,
                                                           const cpx<R>* __restrict__ partials,
                                                           cpx<R>* __restrict__ grid) {
  fold_body<R>(g, items[blockIdx.x], partials, grid);
}

__global__ __launch_bounds__(64 * kFoldSub) void fold_batch_kernel(
    const AdjJob* __restrict__ jobs, const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const AdjJob& J = jobs[it.x];
  fold_body<float>(J.g, J.fold[it.y], J.partials, J.grid);
}

// v exp(+2 pi i q / RAD) for a runtime q >= 0 and RAD = 2 or 4: half turns as
// sign changes, quarter turns as a swap of the parts plus sign changes, all
// as selects (the pruned first stage's outputs are band values rotated so).
// Exact; a zero v may come out as -0.
template <typename R, int RAD>
__device__ __forceinline__ cpx<R> turns_pos(cpx<R> v, int q) {
  static_assert(RAD == 2 || RAD == 4, "half or quarter turns");
  if constexpr (RAD == 2) {
    const bool neg = (q & 1) != 0;
    return {neg ? -v.x : v.x, neg ? -v.y : v.y};
  } else {
    q &= 3;
    const bool sw = (q & 1) != 0;
    const R a = sw ? v.y : v.x, b = sw ? v.x : v.y;
    const bool na = ((q + 1) & 2) != 0, nb = (q & 2) != 0;  // q = 1, 2 and q = 2, 3
    return {na ? -a : a, nb ? -b : b};
  }
}

// Pass-A output layout: columns grouped in blocks of KHB, each block stored
// row-major over the band rows, so that a pass-B workgroup reading KHB (or
// fewer) adjacent columns reads one contiguous stretch.
constexpr int kHBLarge = 4;  // block width at fine grids of 8192 and more
template <int M>
constexpr int khb_for() {
  return M >= 8192 ? kHBLarge : 8;
}
template <int KHB>
__device__ __forceinline__ size_t h_index(int row, int col, int nv) {
  return ((size_t)(col / KHB) * nv + row) * KHB + (col % KHB);
}

// Fills the padded LDS buffer from global memory: element idx (< TOTAL) goes
// to buf[pidx(lpos(idx))] and is src[addr(idx)], or zero when addr returns a
// negative value.  Every load of the thread is issued before any result is
// used (masked elements read a fixed valid address and are zeroed by a
// select), so the loads are in flight together instead of one round trip per
// element.
template <typename R, int TOTAL, int NT, typename A, typename P>
__device__ __forceinline__ void gather_to_lds(cpx<R>* buf, const cpx<R>* __restrict__ src,
                                              A addr, P lpos) {
  constexpr int IT = (TOTAL + NT - 1) / NT;
  cpx<R> t[IT];
  int64_t a[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = (int)threadIdx.x + it * NT;
    a[it] = (TOTAL % NT == 0 || idx < TOTAL) ? addr(idx) : -1;
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) t[it] = src[a[it] >= 0 ? a[it] : 0];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = (int)threadIdx.x + it * NT;
    if (TOTAL % NT == 0 || idx < TOTAL)
      buf[pidx(lpos(idx))] = a[it] >= 0 ? t[it] : cpx<R>{R(0), R(0)};
  }
}

// Workgroups are dispatched to the 8 XCDs (each with its own L2) in turn:
// workgroup b runs on XCD b mod 8.  Renumbering so that each XCD receives a
// contiguous range of logical indices keeps neighbouring work (rows that
// share cache lines of the pass-A buffer) inside one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local(int b, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Row masks (see RowMask): copied into LDS by the passes that test a row per
// element; the whole-row passes test their workgroup's rows once.  The pass
// kernels carry a MASKED flag only so that launches with a mask appear under
// their own symbols in traces: the code reads the mask pointer at run time in
// both, exactly as the batched passes do.
__device__ __forceinline__ bool row_set(const uint32_t* bits, int i) {
  return (bits[i >> 5] >> (i & 31)) & 1u;
}
template <int NB>
__device__ __forceinline__ bool any_row_set(const uint32_t* __restrict__ bits, int i0) {
  bool any = false;
#pragma unroll
  for (int b = 0; b < NB; ++b) any |= row_set(bits, i0 + b);
  return any;
}
template <int NT>
__device__ __forceinline__ void rows_to_lds(uint32_t* smask, const uint32_t* __restrict__ bits,
                                            int n) {
  if (bits)
    for (int i = threadIdx.x; i < (n + 31) / 32; i += NT) smask[i] = bits[i];
}

// Pass A of the adjoint: rows of the band grid (fixed v), FFT along u.
// Element m of a row sits at LDS position pidx(b M + m); a thread's elements
// are NT apart, so their positions advance by padded(NT).  The occupancy
// flags of the workgroup's tile rows are read once into LDS: tiles without
// data were never written and are read as zeros.
constexpr int kMaxTileCols = 512;  // fine grids up to 16384 cells per side
template <typename R, int M, int NB, int NT>
__device__ __forceinline__ void passA_adj_body(const GridGeom& g, const cpx<R>* __restrict__ grid,
                                               const uint8_t* __restrict__ tile_flags,
                                               cpx<R>* __restrict__ H,
                                               const cpx<R>* __restrict__ tw, int rowblock,
                                               const uint32_t* __restrict__ rows = nullptr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  __shared__ cpx<R> tws[tw_count(M)];
  constexpr int TR = (NB + kTile - 1) / kTile + 1;  // tile rows a row block can touch
  __shared__ uint8_t sflag[TR][kMaxTileCols];
  __shared__ uint32_t smask[kMaxRowWords];
  rows_to_lds<NT>(smask, rows, g.n);
  constexpr int n = M / 2;
  const int row0 = rowblock * NB;
  const int tr0 = row0 / kTile;
  for (int i = threadIdx.x; i < TR * g.ntu; i += NT) {
    const int r = i / g.ntu, c = i - r * g.ntu;
    sflag[r][c] = (tr0 + r < g.ntv) ? tile_flags[(tr0 + r) * g.ntu + c] : 0;
  }
  load_twiddles<R, M, NT>(tws, tw);  // ends with a barrier
  static_assert((NB * M) % NT == 0 && NT % 16 == 0, "pass-A gather layout");
  // Input pruning as in pass B: with a first radix of 2 or 4 and a band no
  // wider than M / radix columns, the first stage is applied while loading.
  constexpr int RAD0 = first_radix(M);
  constexpr int NBF0 = M / RAD0;
  bool pruned = false;
  if constexpr (RAD0 <= 4) {
    if (g.nu <= NBF0) {  // uniform
      pruned = true;
      constexpr int ITJ = (NB * NBF0 + NT - 1) / NT;
      cpx<R> t[ITJ];
      int rr[ITJ];
#pragma unroll
      for (int it = 0; it < ITJ; ++it) {
        const int e = (int)threadIdx.x + it * NT;
        const int b = e / NBF0, j = e - b * NBF0;
        const int row = row0 + b;
        const int d = g.u0 - j;
        const int r = d > 0 ? (d + NBF0 - 1) / NBF0 : 0;  // first input at or past u0
        const int rel = j + r * NBF0 - g.u0;
        const bool ok = e < NB * NBF0 && row < g.nv && r < RAD0 && (unsigned)rel < (unsigned)g.nu &&
                        sflag[row / kTile - tr0][rel / kTile] != 0;
        const cpx<R> v = grid[ok ? (size_t)row * g.nu + rel : 0];
        t[it] = ok ? v : cpx<R>{R(0), R(0)};
        rr[it] = ok ? r : 0;
      }
#pragma unroll
      for (int it = 0; it < ITJ; ++it) {
        const int e = (int)threadIdx.x + it * NT;
        if ((NB * NBF0) % NT == 0 || e < NB * NBF0) {
          const int b = e / NBF0, j = e - b * NBF0;
#pragma unroll
          for (int s = 0; s < RAD0; ++s)
            buf[pidx(b * M + j * RAD0 + s)] = turns_pos<R, RAD0>(t[it], rr[it] * s);
        }
      }
    }
  }
  if (!pruned) {
    constexpr int IT = NB * M / NT;
    cpx<R> t[IT];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = (int)threadIdx.x + it * NT;
      const int b = idx / M, m = idx - b * M;
      const int row = row0 + b, rel = m - g.u0;
      ok[it] = row < g.nv && (unsigned)rel < (unsigned)g.nu &&
               sflag[row / kTile - tr0][rel / kTile] != 0;
      t[it] = grid[ok[it] ? (size_t)row * g.nu + rel : 0];
    }
    const int p0 = pidx((int)threadIdx.x);
#pragma unroll
    for (int it = 0; it < IT; ++it)
      buf[p0 + it * padded(NT)] = ok[it] ? t[it] : cpx<R>{R(0), R(0)};
  }
  __syncthreads();
  // the n central frequencies f in [-n/2, n/2) go to H column i = f + n/2,
  // stored from the last stage's registers
  auto keep = [](int, int f) { return 4 * f < M || 4 * f >= 3 * M; };
  // (with a row mask, only the columns of the image rows set)
  auto store = [&](int b, int f, cpx<R> v) {
    const int row = row0 + b;
    const int i = f < n / 2 ? f + n / 2 : f - M + n / 2;
    if (row < g.nv && (!rows || row_set(smask, i))) H[h_index<khb_for<M>()>(row, i, g.nv)] = v;
  };
  // a last-stage butterfly j (outputs j + r M/16) keeps the columns
  // i = j + t M/16, t = 0..7: with a row mask, one whose eight columns are all
  // cleared is skipped whole
  auto need = [&](int j) {
    if (!rows) return true;
    bool any = false;
#pragma unroll
    for (int t = 0; t < 8; ++t) any |= row_set(smask, j + t * (M / 16));
    return any;
  };
  if constexpr (RAD0 <= 4) {
    if (pruned)
      lds_fft_store<R, M, NB, NT, +1, RAD0>(buf, tws, keep, store, need);
    else
      lds_fft_store<R, M, NB, NT, +1>(buf, tws, keep, store, need);
  } else {
    lds_fft_store<R, M, NB, NT, +1>(buf, tws, keep, store, need);
  }
}

template <typename R, int M, int NB, int NT, bool MASKED>
__global__ __launch_bounds__(NT) void passA_adj_kernel(GridGeom g, const cpx<R>* __restrict__ grid,
                                                        const uint8_t* __restrict__ tile_flags,
                                                        cpx<R>* __restrict__ H,
                                                        const cpx<R>* __restrict__ tw,
                                                        const uint32_t* __restrict__ rows) {
  passA_adj_body<R, M, NB, NT>(g, grid, tile_flags, H, tw, xcd_local(blockIdx.x, gridDim.x),
                               rows);
}

template <int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passA_batch_kernel(const AdjJob* __restrict__ jobs,
                                                          const int2* __restrict__ items) {
  const int2 it = items[xcd_local(blockIdx.x, gridDim.x)];
  const AdjJob& J = jobs[it.x];
  passA_adj_body<float, M, NB, NT>(J.g, J.grid, J.flags, J.H, J.tw, it.y, J.rows);
}

__device__ __forceinline__ unsigned long long max_key(float a, int idx) {
  return ((unsigned long long)__float_as_uint(a) << 32) | (unsigned long long)(0xffffffffu - (unsigned)idx);
}

// Pass B of the adjoint: NB image rows i; FFT along v of H[:, i]; correction;
// write image rows; fused max |eta| (max(eta, 0) with ``positive``, the
// positivity-constrained solve) with lowest-index ties.
// One w-plane of the w-stacked adjoint: its position, the phase reference
// c_mid, and whether it is the first plane (which writes instead of adding).
struct WPlane {
  double wj, cmid;
  int first;
};

template <typename R, int M, int NB, int NT, bool WACC = false>
__device__ __forceinline__ void passB_adj_body(const GridGeom& g, const cpx<R>* __restrict__ H,
                                               R* __restrict__ image,
                                               const cpx<R>* __restrict__ tw,
                                               const R* __restrict__ corr, R scale,
                                               unsigned long long* __restrict__ maxkey,
                                               int positive, int iblock,
                                               WPlane wp = WPlane{0.0, 0.0, 1},
                                               const uint32_t* __restrict__ rows = nullptr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  __shared__ cpx<R> tws[tw_count(M)];
  constexpr int n = M / 2;
  const int i0 = iblock * NB;
  // with a row mask: workgroups without a row set return at once, the others
  // store only their rows that are set
  unsigned rowbits = (1u << NB) - 1u;
  if (rows) {
    rowbits = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) rowbits |= (unsigned)row_set(rows, i0 + b) << b;
    if (rowbits == 0) return;  // the whole workgroup
  }
  load_twiddles<R, M, NT>(tws, tw);
  // element (m, b): band row m - v0 of column i0 + b of the pass-A buffer,
  // whose KHB-wide column blocks are row-major over the band rows
  static_assert((NB & (NB - 1)) == 0 && NT % NB == 0, "pass-B layout");
  constexpr int IT = (NB * M + NT - 1) / NT;
  constexpr int MSTEP = NT / NB;  // a thread's m advances by this per element
  const int b = (int)threadIdx.x & (NB - 1), m0 = (int)threadIdx.x / NB;
  const int col = i0 + b;
  constexpr int KHB = khb_for<M>();
  const cpx<R>* hcol = H + (size_t)(col / KHB) * g.nv * KHB + (col % KHB);
  // Input pruning: with a first radix of 2 or 4 and a band no longer than
  // M / radix, each first-stage butterfly (inputs j + r M / radix) holds at
  // most one band row, so the stage is applied while loading: output s of
  // butterfly j is that row rotated by r s quarter (or half) turns, exactly
  // what the full stage computes.  The remaining stages follow as usual.
  constexpr int RAD0 = first_radix(M);
  constexpr int NBF0 = M / RAD0;
  bool pruned = false;
  if constexpr (RAD0 <= 4) {
    if (g.nv <= NBF0) {  // uniform
      pruned = true;
      constexpr int ITJ = (NBF0 + MSTEP - 1) / MSTEP;
      cpx<R> t[ITJ];
      int rr[ITJ];
#pragma unroll
      for (int it = 0; it < ITJ; ++it) {
        const int j = m0 + it * MSTEP;
        const int d = g.v0 - j;
        const int r = d > 0 ? (d + NBF0 - 1) / NBF0 : 0;  // first input at or past v0
        const int rel = j + r * NBF0 - g.v0;
        const bool ok = j < NBF0 && r < RAD0 && (unsigned)rel < (unsigned)g.nv;
        const cpx<R> v = hcol[ok ? (size_t)rel * KHB : 0];
        t[it] = ok ? v : cpx<R>{R(0), R(0)};
        rr[it] = ok ? r : 0;
      }
#pragma unroll
      for (int it = 0; it < ITJ; ++it) {
        const int j = m0 + it * MSTEP;
        if (NBF0 % MSTEP == 0 || j < NBF0) {
#pragma unroll
          for (int s = 0; s < RAD0; ++s)
            buf[pidx(b * M + j * RAD0 + s)] = turns_pos<R, RAD0>(t[it], rr[it] * s);
        }
      }
    }
  }
  if (!pruned) {
    cpx<R> t[IT];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int m = m0 + it * MSTEP;
      const int rel = m - g.v0;
      ok[it] = m < M && (unsigned)rel < (unsigned)g.nv;
      t[it] = hcol[ok[it] ? (size_t)rel * KHB : 0];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int m = m0 + it * MSTEP;
      if ((NB * M) % NT == 0 || m < M) buf[pidx(b * M + m)] = ok[it] ? t[it] : cpx<R>{R(0), R(0)};
    }
  }
  __syncthreads();
  unsigned long long best = 0;
  const R dl = (R)g.dl;
  // pixel (i, j) from frequency f = j - n/2 (mod M) of column i, stored from
  // the last stage's registers with the correction and the max key
  auto keep = [](int, int f) { return 4 * f < M || 4 * f >= 3 * M; };
  auto store = [&](int bb, int f, cpx<R> v) {
    if (!((rowbits >> bb) & 1u)) return;
    const int i = i0 + bb;
    const int j = f < n / 2 ? f + n / 2 : f - M + n / 2;
    const R l = (R)(i - n / 2) * dl, mm = (R)(j - n / 2) * dl;
    R inv_n;
    if constexpr (sizeof(R) == 4) {
      inv_n = __builtin_amdgcn_rsqf(R(1) - l * l - mm * mm);
    } else {
      inv_n = R(1) / sqrt(R(1) - l * l - mm * mm);
    }
    if constexpr (WACC) {
      // Re(exp(2 pi i w_j c') v), c' = n - 1 - c_mid, phase in FP64
      double th = wp.wj * (n_minus_one((double)(i - n / 2) * g.dl, (double)(j - n / 2) * g.dl) -
                           wp.cmid);
      th -= rint(th);
      const R sn = (R)__builtin_amdgcn_sinf((float)th), cs = (R)__builtin_amdgcn_cosf((float)th);
      const R val = (v.x * cs - v.y * sn) * (corr[i] * scale) * corr[j] * inv_n;
      R* dst = image + (size_t)i * n + j;
      *dst = wp.first ? val : *dst + val;
      return;
    }
    const R val = v.x * (corr[i] * scale) * corr[j] * inv_n;
    image[(size_t)i * n + j] = val;
    // positive part: +0 for every val <= 0 (never -0, whose bits would win)
    const float kv = positive ? (val > R(0) ? (float)val : 0.0f) : (float)fabs(val);
    const unsigned long long key = max_key(kv, i * n + j);
    best = key > best ? key : best;
  };
  if constexpr (RAD0 <= 4) {
    if (pruned)
      lds_fft_store<R, M, NB, NT, +1, RAD0>(buf, tws, keep, store);
    else
      lds_fft_store<R, M, NB, NT, +1>(buf, tws, keep, store);
  } else {
    lds_fft_store<R, M, NB, NT, +1>(buf, tws, keep, store);
  }
  if constexpr (WACC) return;  // the maximum comes after the last plane
  // block max
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  __shared__ unsigned long long wbest[NT / 64];
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0 && maxkey) {
    unsigned long long m = 0;
    for (int w = 0; w < NT / 64; ++w) m = wbest[w] > m ? wbest[w] : m;
    atomicMax(maxkey, m);
  }
}

template <typename R, int M, int NB, int NT, bool MASKED>
__global__ __launch_bounds__(NT) void passB_adj_kernel(GridGeom g, const cpx<R>* __restrict__ H,
                                                        R* __restrict__ image,
                                                        const cpx<R>* __restrict__ tw,
                                                        const R* __restrict__ corr, R scale,
                                                        unsigned long long* __restrict__ maxkey,
                                                        int positive,
                                                        const uint32_t* __restrict__ rows) {
  passB_adj_body<R, M, NB, NT>(g, H, image, tw, corr, scale, maxkey, positive,
                               xcd_local(blockIdx.x, gridDim.x), WPlane{0.0, 0.0, 1}, rows);
}

template <typename R, int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passB_adj_w_kernel(GridGeom g, const cpx<R>* __restrict__ H,
                                                          R* __restrict__ image,
                                                          const cpx<R>* __restrict__ tw,
                                                          const R* __restrict__ corr, R scale,
                                                          WPlane wp) {
  passB_adj_body<R, M, NB, NT, true>(g, H, image, tw, corr, scale, nullptr, 0,
                                     xcd_local(blockIdx.x, gridDim.x), wp);
}

// Visibility weights of w-plane w_j (plan order): h_k exp(2 pi i w_k c_mid)
// psi((w_k - w_j) / dw) within the kernel's reach |w_k - w_j| <= (W/2) dw,
// zero beyond it; a visibility with w_k < 0 enters as its conjugate at -w_k
// (the plan grids it at (-u, -v)).  perm: NULL when h is in plan order.
__global__ __launch_bounds__(256) void wplane_kernel(int64_t L, const double* __restrict__ Cw,
                                                     const cpx<float>* __restrict__ h,
                                                     const int32_t* __restrict__ perm, double wj,
                                                     double inv_dw, double cmid, float R2,
                                                     float c1, float c0,
                                                     cpx<float>* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const double wk = fabs(Cw[k]);
  const float t = (float)((wk - wj) * inv_dw);
  cpx<float> o{0.f, 0.f};
  if (t * t <= R2) {
    cpx<float> v = h[perm ? perm[k] : k];
    if (Cw[k] < 0.0) v.y = -v.y;
    double ph = wk * cmid;
    ph -= rint(ph);
    const float sn = __builtin_amdgcn_sinf((float)ph), cs = __builtin_amdgcn_cosf((float)ph);
    const float q = fmaxf(fmaf(-t, t, R2), 0.0f);
    const float psi = __builtin_amdgcn_exp2f(fmaf(c1, __builtin_amdgcn_sqrtf(q), -c0));
    o = {psi * (v.x * cs - v.y * sn), psi * (v.x * sn + v.y * cs)};
  }
  out[k] = o;
}

// Last step of the w-stacked adjoint: image /= Psi(dw c') per pixel, and
// the fused maximum key.  Psi(xi) = sum_q W w_q phi(z_q) cos(pi W z_q xi)
// (the quadrature of the kernel's Fourier integral) is evaluated as its
// Chebyshev series in 4 xi (xi = dw (c' - c_mid) lies in [-1/4, 1/4]):
// cheb[k], k < kPsiCheb, by Clenshaw's recurrence in FP64.
__global__ __launch_bounds__(256) void wfinal_kernel(GridGeom g, WStack ws,
                                                     const double* __restrict__ cheb,
                                                     float* __restrict__ image,
                                                     unsigned long long* __restrict__ maxkey,
                                                     int positive) {
  // a grid-stride loop over a capped grid: one atomic per workgroup on the
  // single key, so few workgroups (thousands contending for one address
  // took most of the kernel's time)
  const int n = g.n;
  unsigned long long best = 0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
    const double xi =
        ws.dw * (n_minus_one((double)(i - n / 2) * g.dl, (double)(j - n / 2) * g.dl) - ws.cmid);
    const double x = fmin(fmax(4.0 * xi, -1.0), 1.0);
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = kPsiCheb - 1; k >= 1; --k) {
      const double b0 = fma(2.0 * x, b1, cheb[k] - b2);
      b2 = b1;
      b1 = b0;
    }
    const double psi = fma(x, b1, cheb[0] - b2);
    const float val = (float)((double)image[idx] / psi);
    image[idx] = val;
    const float kv = positive ? (val > 0.f ? val : 0.0f) : fabsf(val);
    const unsigned long long key = max_key(kv, (int)idx);
    best = key > best ? key : best;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  __shared__ unsigned long long wbest[4];
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < 4; ++w) m = wbest[w] > m ? wbest[w] : m;
    atomicMax(maxkey, m);
  }
}

template <int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passB_batch_kernel(const AdjJob* __restrict__ jobs,
                                                          const int2* __restrict__ items) {
  const int2 it = items[xcd_local(blockIdx.x, gridDim.x)];
  const AdjJob& J = jobs[it.x];
  passB_adj_body<float, M, NB, NT>(J.g, J.H, J.image, J.tw, J.corr, J.scale, J.maxkey,
                                   J.positive, it.y, WPlane{0.0, 0.0, 1}, J.rows);
}

// First stage of a forward transform whose input is the n = M/2 central
// frequencies of each sequence (slot m holds frequency m for m < M/4 and
// m - M for m >= 3M/4; the slots between are zero), applied while loading.
// Butterfly j of the first stage (radix RAD0, inputs j + r M/RAD0) then has
// fixed nonzero inputs: for RAD0 >= 4 the r < RAD0/4 and r >= 3 RAD0/4, for
// RAD0 = 2 exactly one (r = 0 when j < M/4, else r = 1).  load(b, c) returns
// the value at central index c = f + n/2 of sequence b; outputs go where the
// full stage writes them (b M + j RAD0 + s).  All loads of a thread are issued
// before the first is used.
template <typename R, int M, int NB, int NT, int SIGN, typename Load>
__device__ __forceinline__ void central_first_stage(cpx<R>* buf, Load load) {
  constexpr int RAD0 = first_radix(M);
  constexpr int NBF0 = M / RAD0;
  constexpr int TOT = NB * NBF0;
  constexpr int IT = (TOT + NT - 1) / NT;
  constexpr int NZ = RAD0 >= 4 ? RAD0 / 2 : 1;  // nonzero inputs per butterfly
  static_assert(M >= 32, "central first stage layout");
  cpx<R> t[IT][NZ];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = (int)threadIdx.x + it * NT;
    const int ee = (TOT % NT == 0 || e < TOT) ? e : 0;  // a valid element for spare lanes
    const int b = ee / NBF0, j = ee - b * NBF0;
    if constexpr (RAD0 == 2) {
      t[it][0] = load(b, j < M / 4 ? j + M / 4 : j - M / 4);
    } else {
#pragma unroll
      for (int q = 0; q < NZ; ++q) {
        const int r = q < RAD0 / 4 ? q : q + RAD0 / 2;   // r in [0, RAD0/4) u [3 RAD0/4, RAD0)
        const int m = j + r * NBF0;
        t[it][q] = load(b, r < RAD0 / 4 ? m + M / 4 : m - 3 * (M / 4));
      }
    }
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = (int)threadIdx.x + it * NT;
    if (TOT % NT == 0 || e < TOT) {
      const int b = e / NBF0, j = e - b * NBF0;
      const int p0 = b * M + j * RAD0;
      if constexpr (RAD0 == 2) {
        const cpx<R> v = t[it][0];
        buf[pidx(p0)] = v;
        buf[pidx(p0 + 1)] = j < M / 4 ? v : cpx<R>{-v.x, -v.y};
      } else if constexpr (RAD0 == 4) {
        // X_s = x_0 + x_3 w^(3 s)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const cpx<R> u = rot<R, 4, SIGN>(t[it][1], (3 * s) & 3);
          buf[pidx(p0 + s)] = {t[it][0].x + u.x, t[it][0].y + u.y};
        }
      } else {
        cpx<R> x[RAD0];
#pragma unroll
        for (int r = 0; r < RAD0; ++r) x[r] = {R(0), R(0)};
#pragma unroll
        for (int q = 0; q < NZ; ++q) x[q < RAD0 / 4 ? q : q + RAD0 / 2] = t[it][q];
        dft<R, RAD0, SIGN>(x);
#pragma unroll
        for (int s = 0; s < RAD0; ++s) buf[pidx(p0 + s)] = x[s];
      }
    }
  }
}

// Forward pass B^T: NB image rows i, pre-correct, FFT along v (sign -1),
// keep the band rows: H[v_rel][i] (the pass-A layout).  The first stage is
// applied while loading (the row's n pixels are the central frequencies) and
// the band rows are stored from the last stage's registers.
template <typename R, int M, int NB, int NT>
__device__ __forceinline__ void passB_fwd_body(const GridGeom& g, const R* __restrict__ image,
                                               cpx<R>* __restrict__ H,
                                               const cpx<R>* __restrict__ tw,
                                               const R* __restrict__ corr, int iblock,
                                               const uint32_t* __restrict__ rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  __shared__ cpx<R> tws[tw_count(M)];
  constexpr int n = M / 2;
  const int i0 = iblock * NB;
  // with a row mask, workgroups of zero rows write nothing (pass A reads
  // those columns of H as zeros)
  if (rows && !any_row_set<NB>(rows, i0)) return;
  load_twiddles<R, M, NT>(tws, tw);
  const R dl = (R)g.dl;
  central_first_stage<R, M, NB, NT, -1>(buf, [&](int b, int j) -> cpx<R> {
    const int i = i0 + b;
    const R l = (R)(i - n / 2) * dl, mm = (R)(j - n / 2) * dl;
    R inv_n;
    if constexpr (sizeof(R) == 4) {
      inv_n = __builtin_amdgcn_rsqf(R(1) - l * l - mm * mm);
    } else {
      inv_n = R(1) / sqrt(R(1) - l * l - mm * mm);
    }
    return {image[(size_t)i * n + j] * corr[i] * corr[j] * inv_n, R(0)};
  });
  __syncthreads();
  constexpr int KHB = khb_for<M>();
  const int v0 = g.v0, nv = g.nv;
  auto keep = [&](int, int f) { return (unsigned)(f - v0) < (unsigned)nv; };
  auto store = [&](int b, int f, cpx<R> v) { H[h_index<KHB>(f - v0, i0 + b, nv)] = v; };
  lds_fft_store<R, M, NB, NT, -1, first_radix(M)>(buf, tws, keep, store);
}

template <typename R, int M, int NB, int NT, bool MASKED>
__global__ __launch_bounds__(NT) void passB_fwd_kernel(GridGeom g, const R* __restrict__ image,
                                                        cpx<R>* __restrict__ H,
                                                        const cpx<R>* __restrict__ tw,
                                                        const R* __restrict__ corr,
                                                        const uint32_t* __restrict__ rows) {
  passB_fwd_body<R, M, NB, NT>(g, image, H, tw, corr, xcd_local(blockIdx.x, gridDim.x), rows);
}

// Forward pass A^T: NB band rows v; FFT along u (sign -1) of H[v][:] placed
// at the n central frequencies (first stage applied while loading); the band
// columns stored from the last stage's registers.
template <typename R, int M, int NB, int NT, bool MASKED>
__global__ __launch_bounds__(NT) void passA_fwd_kernel(GridGeom g, const cpx<R>* __restrict__ H,
                                                        cpx<R>* __restrict__ grid,
                                                        const cpx<R>* __restrict__ tw,
                                                        const uint32_t* __restrict__ rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  __shared__ cpx<R> tws[tw_count(M)];
  __shared__ uint32_t smask[kMaxRowWords];
  rows_to_lds<NT>(smask, rows, g.n);
  load_twiddles<R, M, NT>(tws, tw);  // (its barrier also covers the mask)
  const int row0 = xcd_local(blockIdx.x, gridDim.x) * NB;
  constexpr int KHB = khb_for<M>();
  const int nv = g.nv;
  central_first_stage<R, M, NB, NT, -1>(buf, [&](int b, int c) -> cpx<R> {
    const int row = row0 + b;
    // H column c is image row c: zero, and not read, when the mask clears it;
    // rows past the band (last workgroup) read row 0 and are never stored
    if (rows && !row_set(smask, c)) return {R(0), R(0)};
    return H[h_index<KHB>(row < nv ? row : 0, c, nv)];
  });
  __syncthreads();
  const int u0 = g.u0, nu = g.nu;
  auto keep = [&](int, int f) { return (unsigned)(f - u0) < (unsigned)nu; };
  auto store = [&](int b, int f, cpx<R> v) {
    const int row = row0 + b;
    if (row < nv) grid[(size_t)row * nu + (f - u0)] = v;
  };
  lds_fft_store<R, M, NB, NT, -1, first_radix(M)>(buf, tws, keep, store);
}

// Interpolation: V_k = sum of w x w taps of the fine grid (type-2 gather).
template <typename R, int W>
__global__ __launch_bounds__(256) void interp_kernel(GridGeom g, int64_t L,
                                                     const uint32_t* __restrict__ cell,
                                                     const R* __restrict__ off,
                                                     const cpx<R>* __restrict__ grid,
                                                     const int32_t* __restrict__ perm,
                                                     cpx<R>* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L) return;
  const uint32_t c = cell[s];
  const int cu = (int)(c & 0xffffu), cv = (int)(c >> 16);
  const R su = off[2 * s], sv = off[2 * s + 1];
  const R inv = R(2) / R(W);
  const R beta = sizeof(R) == 4 ? (R)g.beta : (R)g.beta64;
  R ku[W];
#pragma unroll
  for (int t = 0; t < W; ++t) ku[t] = es_kernel<R>((su + R(t)) * inv, beta);
  R ax = 0, ay = 0;
  // rows: not fully unrolled (W^2 loads in flight would exhaust registers for
  // wide kernels); the row weight is evaluated in the loop
#pragma unroll 2
  for (int a = 0; a < W; ++a) {
    const R kva = es_kernel<R>((sv + R(a)) * inv, beta);
    int y = cv + a - g.v0;
    if (g.wrap && y >= g.M) y -= g.M;
    R rx = 0, ry = 0;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      int x = cu + b - g.u0;
      if (g.wrap && x >= g.M) x -= g.M;
      const cpx<R> v = grid[(size_t)y * g.nu + x];
      rx += v.x * ku[b];
      ry += v.y * ku[b];
    }
    ax += rx * kva;
    ay += ry * kva;
  }
  const int64_t d = perm ? perm[s] : s;
  out[d] = {ax, ay};
}

// Interpolation from LDS (FP32, kernel widths up to 16): one workgroup of
// kInterpThreads per work item (InterpItem), a plan-order range of
// visibilities whose first cells lie in one tile.  The workgroup copies the
// tile and the W - 1 cells past its right and lower edges, all that its
// visibilities' footprints reach, into LDS (cells outside the band as zeros;
// with a periodic band, wrapped), then each thread sums the W x W taps of one
// visibility at a time from there, rows of taps in the same order as
// interp_kernel.  With base (plan order, plan-order output), the output is
// base - Phi x: the residual, in the same FP32 subtraction a separate pass
// would do; with stats as well, each work item also writes its sums of
// |r|^2 and Re(conj(base) r) in FP64 to stats[2 item], [2 item + 1] (threads
// combined in a fixed order).
constexpr int kInterpThreads = 256;
template <int W>
struct InterpCfg {
  static constexpr int S = kTile + W - 1;  // region side (cells)
  static constexpr int SP = S | 1;         // row stride (odd)
};

template <int W>
__global__ __launch_bounds__(kInterpThreads) void interp_lds_kernel(GridGeom g,
                                                        const InterpItem* __restrict__ items,
                                                        const uint32_t* __restrict__ cell,
                                                        const float* __restrict__ off,
                                                        const c32* __restrict__ grid,
                                                        const int32_t* __restrict__ perm,
                                                        const c32* __restrict__ base,
                                                        c32* __restrict__ out,
                                                        double* __restrict__ stats) {
  using C = InterpCfg<W>;
  __shared__ float2 reg[C::S * C::SP];
  const InterpItem it = items[blockIdx.x];
  const int tid = (int)threadIdx.x;
  const int tv = it.tile / g.ntu, tu = it.tile - tv * g.ntu;
  const int rv0 = tv * kTile, ru0 = tu * kTile;  // region origin in the band
  for (int e = tid; e < C::S * C::S; e += kInterpThreads) {
    const int y = e / C::S, x = e - y * C::S;
    int rv = rv0 + y, ru = ru0 + x;
    float2 v = make_float2(0.f, 0.f);
    if (g.wrap) {
      if (rv >= g.M) rv -= g.M;
      if (ru >= g.M) ru -= g.M;
    }
    if (rv < g.nv && ru < g.nu) {
      const c32 c = grid[(size_t)rv * g.nu + ru];
      v = make_float2(c.x, c.y);
    }
    reg[y * C::SP + x] = v;
  }
  __syncthreads();
  constexpr float R = 0.5f * (float)W;
  const float c0 = g.beta * 1.44269504088896341f;  // beta log2(e)
  const float c1 = c0 / R;
  const int ou = g.u0 + ru0, ov = g.v0 + rv0;
  double r2 = 0.0, vr = 0.0;
  for (int sidx = it.beg + tid; sidx < it.end; sidx += kInterpThreads) {
    const uint32_t c = cell[sidx];
    const int x = (int)(c & 0xffffu) - ou, y = (int)(c >> 16) - ov;  // in [0, kTile)
    const float2 o = reinterpret_cast<const float2*>(off)[sidx];
    float ku[W];
#pragma unroll
    for (int t = 0; t < W; ++t) ku[t] = es_weight(o.x + (float)t, R * R, c1, c0);
    float ax = 0.f, ay = 0.f;
    const float2* rp = reg + y * C::SP + x;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const float kva = es_weight(o.y + (float)a, R * R, c1, c0);
      float rx = 0.f, ry = 0.f;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const float2 v = rp[a * C::SP + b];
        rx += v.x * ku[b];
        ry += v.y * ku[b];
      }
      ax += rx * kva;
      ay += ry * kva;
    }
    if (base) {
      const c32 v = base[sidx];
      const c32 r = {v.x - ax, v.y - ay};
      out[sidx] = r;
      r2 += (double)r.x * r.x + (double)r.y * r.y;
      vr += (double)v.x * r.x + (double)v.y * r.y;
    } else {
      out[perm ? perm[sidx] : sidx] = {ax, ay};
    }
  }
  if (stats) {
    constexpr int NW = kInterpThreads / 64;
    __shared__ double wsum[2][NW];
    for (int o = 32; o > 0; o >>= 1) {
      r2 += __shfl_xor(r2, o, 64);
      vr += __shfl_xor(vr, o, 64);
    }
    if ((tid & 63) == 0) {
      wsum[0][tid >> 6] = r2;
      wsum[1][tid >> 6] = vr;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NW; ++w) {
        a += wsum[0][w];
        b += wsum[1][w];
      }
      stats[2 * (size_t)blockIdx.x] = a;
      stats[2 * (size_t)blockIdx.x + 1] = b;
    }
  }
}

// Pass B evaluated directly for an active set (the APGD's gridded
// operators).  Its atoms lie on few image rows, a row holding one or two, so
// instead of a length-M transform per row the needed values are sums over
// the atoms or over the band rows with phases e^{-/+2 pi i f q / M} (f = j -
// n/2 the atom's centred column, q = v0 + band row), the product f q reduced
// mod M exactly in integers and the angle (in turns, |t| <= 1/2) taken by the
// hardware sine and cosine.  The apodisation and 1/n factors are applied in
// the order the transform's loading (forward) and epilogue (adjoint) apply
// them.
__device__ __forceinline__ float turns_mod(int f, int q, int M) {
  int t = (f * q) & (M - 1);  // f q mod M (two's complement), f q < 2^31
  if (t >= M / 2) t -= M;
  return (float)t / (float)M;  // exact: M is a power of two
}

__device__ __forceinline__ float inv_n_f32(const GridGeom& g, int i, int j) {
  const float dl = (float)g.dl;
  const float l = (float)(i - g.n / 2) * dl, mm = (float)(j - g.n / 2) * dl;
  return __builtin_amdgcn_rsqf(1.0f - l * l - mm * mm);
}

// Forward: H[band row][i] = sum over the atoms of row i of c e^{-2 pi i f q / M}
// for each occupied row i (rowlist: row, first atom, end), atoms sorted by
// pixel with FP64 weights w.
template <int KHB>
__global__ __launch_bounds__(256) void rows_fwd_direct_kernel(GridGeom g,
                                                              const int3* __restrict__ rowlist,
                                                              const int32_t* __restrict__ pix,
                                                              const double* __restrict__ w,
                                                              const float* __restrict__ corr,
                                                              c32* __restrict__ H) {
  const int3 rl = rowlist[blockIdx.y];
  const int i = rl.x, n = g.n;
  for (int rel = (int)(blockIdx.x * blockDim.x + threadIdx.x); rel < g.nv;
       rel += (int)(gridDim.x * blockDim.x)) {
    const int q = g.v0 + rel;
    float hx = 0.f, hy = 0.f;
    for (int a = rl.y; a < rl.z; ++a) {
      const int j = pix[a] - i * n;
      const float c = (float)w[a] * corr[i] * corr[j] * inv_n_f32(g, i, j);
      const float tt = turns_mod(j - n / 2, q, g.M);
      hx += c * __builtin_amdgcn_cosf(tt);
      hy -= c * __builtin_amdgcn_sinf(tt);
    }
    H[h_index<KHB>(rel, i, g.nv)] = {hx, hy};
  }
}

// Adjoint at the atoms: one 256-thread workgroup per atom, g = Re(sum over
// band rows of H[band row][i] e^{+2 pi i f q / M}) times the corrections, in
// FP64 out (thread sums combined in a fixed order).
template <int KHB>
__global__ __launch_bounds__(256) void atoms_adj_direct_kernel(GridGeom g,
                                                               const int32_t* __restrict__ pix,
                                                               const c32* __restrict__ H,
                                                               const float* __restrict__ corr,
                                                               double* __restrict__ gout) {
  const int a = (int)blockIdx.x, t = (int)threadIdx.x;
  const int pp = pix[a], n = g.n;
  const int i = pp / n, j = pp - i * n;
  float acc = 0.f;
  for (int rel = t; rel < g.nv; rel += 256) {
    const float tt = turns_mod(j - n / 2, g.v0 + rel, g.M);
    const c32 h = H[h_index<KHB>(rel, i, g.nv)];
    acc += h.x * __builtin_amdgcn_cosf(tt) - h.y * __builtin_amdgcn_sinf(tt);
  }
  double d = acc;
  for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
  __shared__ double wsum[4];
  if ((t & 63) == 0) wsum[t >> 6] = d;
  __syncthreads();
  if (t == 0) {
    const double sum = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    const float v = (float)sum * corr[i] * corr[j] * inv_n_f32(g, i, j);
    gout[a] = (double)v;
  }
}

// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------
// Algorithmic bytes of one spread: each visibility's value and its two
// sub-cell offsets read once (4 reals), each band cell written once.
static double spread_bytes(const pc_plan* p, double rb) {
  return p->L * 4.0 * rb + 2.0 * rb * p->g.nu * p->g.nv;
}

template <typename R, int W>
static void launch_spread_w(pc_plan* p, const cpx<R>* vals, const int32_t* perm, hipStream_t s) {
  const double rb = sizeof(R);
  ProfScope ps(p, s, "spread", spread_bytes(p, rb), (double)p->L);
  if constexpr (sizeof(R) == 4 && W <= 8) {
    if (!p->spread_quads) fail(PC_ERR_DEVICE, "spread: the plan's work list is not grouped");
    constexpr size_t lds = SpreadG<W>::lds_bytes;
    static_assert(lds <= 64 * 1024, "grouped spread LDS budget");
    hipLaunchKernelGGL((spread_quad_kernel<W>), dim3((unsigned)(p->n_chunks / kSpreadQuad)),
                       dim3(64 * kSpreadQuad), lds, s, p->g, p->chunks, p->cell,
                       (const float*)p->off, vals, perm, (c32*)p->grid, (c32*)p->partials,
                       p->maxkey);
  } else {
    constexpr size_t lds = SpreadCfg<R, W>::lds_bytes;
    static_assert(lds <= 160 * 1024, "spread LDS budget");
    if (p->spread_quads) fail(PC_ERR_DEVICE, "spread: the plan's work list is grouped");
    if (lds > 64 * 1024)
      PC_HIP(hipFuncSetAttribute((const void*)spread_kernel<R, W>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((spread_kernel<R, W>), dim3((unsigned)p->n_chunks), dim3(64), lds, s, p->g,
                       p->chunks, p->cell, (const R*)p->off, vals, perm, (cpx<R>*)p->grid,
                       (cpx<R>*)p->partials, p->maxkey);
  }
  PC_LAUNCH_CHECK("spread");
}

template <typename R>
static void launch_spread(pc_plan* p, const cpx<R>* vals, const int32_t* perm, hipStream_t s) {
  switch (p->g.W) {
#define PC_W(w) \
  case w:       \
    launch_spread_w<R, w>(p, vals, perm, s); \
    break;
    PC_W(2) PC_W(3) PC_W(4) PC_W(5) PC_W(6) PC_W(7) PC_W(8) PC_W(9) PC_W(10) PC_W(11) PC_W(12)
    PC_W(13) PC_W(14) PC_W(15) PC_W(16)
#undef PC_W
    default:
      fail(PC_ERR_UNSUPPORTED, "kernel width");
  }
  if (p->n_fold > 0) {
    const double tb = 2.0 * sizeof(R) * kTile * kTile;
    ProfScope ps(p, s, "fold", tb * (p->n_partials + p->n_fold), (double)p->n_partials);
    hipLaunchKernelGGL((fold_kernel<R>), dim3((unsigned)p->n_fold, kTile * kTile / 64),
                       dim3(64 * kFoldSub), 0, s, p->g, p->fold,
                       (const cpx<R>*)p->partials, (cpx<R>*)p->grid);
    PC_LAUNCH_CHECK("fold");
  }
}

template <typename R, int W>
static void launch_interp_w(pc_plan* p, const int32_t* perm, cpx<R>* out, hipStream_t s,
                            const cpx<R>* base, double* stats) {
  const double rb = sizeof(R);
  ProfScope ps(p, s, "interp", p->L * (4 + 4 * rb + (base ? 2 * rb : 0)) +
                                   2 * rb * p->g.nu * p->g.nv, (double)p->L);
  if constexpr (sizeof(R) == 4) {
    hipLaunchKernelGGL((interp_lds_kernel<W>), dim3((unsigned)p->n_interp), dim3(kInterpThreads),
                       0, s, p->g,
                       p->interp, p->cell, (const float*)p->off, (const c32*)p->grid, perm,
                       (const c32*)base, (c32*)out, base ? stats : nullptr);
  } else {
    if (base) fail(PC_ERR_UNSUPPORTED, "FP64 interpolation with a base");
    const unsigned nb = (unsigned)((p->L + 255) / 256);
    hipLaunchKernelGGL((interp_kernel<R, W>), dim3(nb), dim3(256), 0, s, p->g, p->L, p->cell,
                       (const R*)p->off, (const cpx<R>*)p->grid, perm, out);
  }
  PC_LAUNCH_CHECK("interp");
}

template <typename R>
static void launch_interp(pc_plan* p, const int32_t* perm, cpx<R>* out, hipStream_t s,
                          const cpx<R>* base = nullptr, double* stats = nullptr) {
  switch (p->g.W) {
#define PC_W(w) \
  case w:       \
    launch_interp_w<R, w>(p, perm, out, s, base, stats); \
    break;
    PC_W(2) PC_W(3) PC_W(4) PC_W(5) PC_W(6) PC_W(7) PC_W(8) PC_W(9) PC_W(10) PC_W(11) PC_W(12)
    PC_W(13) PC_W(14) PC_W(15) PC_W(16)
#undef PC_W
    default:
      fail(PC_ERR_UNSUPPORTED, "kernel width");
  }
}

// Launch shapes per fine-grid size: NB sequences per workgroup, NT threads.
// Pass A keeps about 64 KB (FP32) of LDS per workgroup; pass B up to 128 KB.
template <typename R>
struct Shapes {
  static constexpr int lds_a = 64 * 1024;
  static constexpr int lds_b = 64 * 1024;
};

static void set_lds(const void* kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    PC_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// Sequences per pass-B workgroup: about n/256 (so a launch has >= 256
// workgroups), capped by the LDS budget and at 16.
template <typename R, int M>
constexpr int nb_passB() {
  constexpr int CB = sizeof(cpx<R>);
  constexpr int lim = (M * CB >= Shapes<R>::lds_b) ? 1 : Shapes<R>::lds_b / (M * CB);
  constexpr int want = (M / 2) / 256 < 1 ? 1 : (M / 2) / 256;
  constexpr int a = want < lim ? want : lim;
  return a > 16 ? 16 : a;
}

template <int TOTAL_BUTTERFLIES>
constexpr int nt_for() {
  return TOTAL_BUTTERFLIES >= 1024 ? 1024 : (TOTAL_BUTTERFLIES >= 512 ? 512 : 256);
}

template <typename R, int M>
static void run_passes_adj(pc_plan* p, R* image, R scale, hipStream_t s,
                           const WPlane* wp = nullptr, const RowMask* rows = nullptr,
                           bool pass_b = true) {
  constexpr int CB = sizeof(cpx<R>);
  constexpr int NBA = (M * CB >= Shapes<R>::lds_a) ? 1 : Shapes<R>::lds_a / (M * CB);
  constexpr int NTA = nt_for<NBA * M / 16>();
  constexpr int NBB = nb_passB<R, M>();
  constexpr int NTB = nt_for<NBB * M / 16>();
  const GridGeom& g = p->g;
  const size_t lda = (size_t)padded(NBA * M) * CB, ldb = (size_t)padded(NBB * M) * CB;
  const double nvn = (double)g.nv * g.n * CB;
  // with a row mask: the H columns and image rows of the rows set (the
  // passes appear under names of their own)
  const uint32_t* bits = rows ? rows->bits : nullptr;
  const double nr = rows ? (double)rows->count : (double)g.n;
  const double nvr = (double)g.nv * nr * CB;
  {
    ProfScope ps(p, s, rows ? "passA_adj_rows" : "passA_adj", (double)g.nv * g.nu * CB + nvr,
                 (double)g.nv * M);
#define PC_PASS_A(MASKED)                                                                      \
  set_lds((const void*)passA_adj_kernel<R, M, NBA, NTA, MASKED>, lda);                         \
  hipLaunchKernelGGL((passA_adj_kernel<R, M, NBA, NTA, MASKED>), dim3((g.nv + NBA - 1) / NBA), \
                     dim3(NTA), lda, s, g, (const cpx<R>*)p->grid, p->tile_flags,              \
                     (cpx<R>*)p->H, (const cpx<R>*)p->twiddle, bits)
    if (rows) {
      PC_PASS_A(true);
    } else {
      PC_PASS_A(false);
    }
#undef PC_PASS_A
    PC_LAUNCH_CHECK("passA_adj");
  }
  if (!pass_b) return;  // (the caller evaluates pass B itself)
  if (wp) {  // one w-plane: rotate, add into the image
    set_lds((const void*)passB_adj_w_kernel<R, M, NBB, NTB>, ldb);
    ProfScope ps(p, s, "passB_adj_w", nvn + (double)g.n * g.n * sizeof(R) * (wp->first ? 1 : 2),
                 (double)g.n * M);
    hipLaunchKernelGGL((passB_adj_w_kernel<R, M, NBB, NTB>), dim3((M / 2) / NBB), dim3(NTB), ldb,
                       s, g, (const cpx<R>*)p->H, image, (const cpx<R>*)p->twiddle,
                       (const R*)p->corr, scale, *wp);
    PC_LAUNCH_CHECK("passB_adj_w");
    return;
  }
  ProfScope ps(p, s, rows ? "passB_adj_rows" : "passB_adj",
               nvr + nr * g.n * sizeof(R), nr * M);
#define PC_PASS_B(MASKED)                                                                       \
  set_lds((const void*)passB_adj_kernel<R, M, NBB, NTB, MASKED>, ldb);                          \
  hipLaunchKernelGGL((passB_adj_kernel<R, M, NBB, NTB, MASKED>), dim3((M / 2) / NBB), dim3(NTB), \
                     ldb, s, g, (const cpx<R>*)p->H, image, (const cpx<R>*)p->twiddle,          \
                     (const R*)p->corr, scale, rows ? nullptr : p->maxkey, p->max_positive, bits)
  if (rows) {
    PC_PASS_B(true);
  } else {
    PC_PASS_B(false);
  }
#undef PC_PASS_B
  PC_LAUNCH_CHECK("passB_adj");
}

template <typename R, int M>
static void run_passes_fwd(pc_plan* p, const R* image, hipStream_t s,
                           const RowMask* rows = nullptr, bool pass_b = true) {
  constexpr int CB = sizeof(cpx<R>);
  constexpr int NBA = (M * CB >= Shapes<R>::lds_a) ? 1 : Shapes<R>::lds_a / (M * CB);
  constexpr int NTA = nt_for<NBA * M / 16>();
  constexpr int NBB = nb_passB<R, M>();
  constexpr int NTB = nt_for<NBB * M / 16>();
  const GridGeom& g = p->g;
  const size_t lda = (size_t)padded(NBA * M) * CB, ldb = (size_t)padded(NBB * M) * CB;
  const uint32_t* bits = rows ? rows->bits : nullptr;
  const double nr = rows ? (double)rows->count : (double)g.n;
  const double nvr = (double)g.nv * nr * CB;
  if (pass_b) {  // (else the caller has written the pass-A buffer's columns)
    ProfScope ps(p, s, rows ? "passB_fwd_rows" : "passB_fwd", nvr + nr * g.n * sizeof(R), nr * M);
#define PC_PASS_BF(MASKED)                                                                      \
  set_lds((const void*)passB_fwd_kernel<R, M, NBB, NTB, MASKED>, ldb);                          \
  hipLaunchKernelGGL((passB_fwd_kernel<R, M, NBB, NTB, MASKED>), dim3((M / 2) / NBB), dim3(NTB), \
                     ldb, s, g, image, (cpx<R>*)p->H, (const cpx<R>*)p->twiddle,                \
                     (const R*)p->corr, bits)
    if (rows) {
      PC_PASS_BF(true);
    } else {
      PC_PASS_BF(false);
    }
#undef PC_PASS_BF
    PC_LAUNCH_CHECK("passB_fwd");
  }
  ProfScope ps(p, s, rows ? "passA_fwd_rows" : "passA_fwd", (double)g.nv * g.nu * CB + nvr,
               (double)g.nv * M);
#define PC_PASS_AF(MASKED)                                                                      \
  set_lds((const void*)passA_fwd_kernel<R, M, NBA, NTA, MASKED>, lda);                          \
  hipLaunchKernelGGL((passA_fwd_kernel<R, M, NBA, NTA, MASKED>), dim3((g.nv + NBA - 1) / NBA),  \
                     dim3(NTA), lda, s, g, (const cpx<R>*)p->H, (cpx<R>*)p->grid,               \
                     (const cpx<R>*)p->twiddle, bits)
  if (rows) {
    PC_PASS_AF(true);
  } else {
    PC_PASS_AF(false);
  }
#undef PC_PASS_AF
  PC_LAUNCH_CHECK("passA_fwd");
}

template <typename R>
static void dispatch_M(pc_plan* p, bool adjoint, R* img_out, const R* img_in, R scale,
                       hipStream_t s, const WPlane* wp = nullptr, const RowMask* rows = nullptr,
                       bool pass_b = true) {
  switch (p->g.M) {
#define PC_M(m)                                                     \
  case m:                                                           \
    if (adjoint)                                                    \
      run_passes_adj<R, m>(p, img_out, scale, s, wp, rows, pass_b); \
    else                                                            \
      run_passes_fwd<R, m>(p, img_in, s, rows, pass_b);             \
    return;
    PC_M(32) PC_M(64) PC_M(128) PC_M(256) PC_M(512) PC_M(1024) PC_M(2048) PC_M(4096) PC_M(8192)
#undef PC_M
    case 16384:
      if constexpr (sizeof(R) == 4) {
        if (adjoint)
          run_passes_adj<R, 16384>(p, img_out, scale, s, wp, rows, pass_b);
        else
          run_passes_fwd<R, 16384>(p, img_in, s, rows, pass_b);
        return;
      }
      [[fallthrough]];
    default:
      fail(PC_ERR_UNSUPPORTED, "fine grid size " + std::to_string(p->g.M) +
                                   (sizeof(R) == 8 ? " in FP64" : "") + " is not a supported power of two");
  }
}


void forward_grid_set(pc_plan* p, const AtomSet& as, const double* w, const c32* base,
                      double* stats, c32* out, hipStream_t s) {
  if (p->Cw || p->precision != PC_PREC_FP32)
    fail(PC_ERR_UNSUPPORTED, "gridded set operators need a coplanar FP32 plan");
  const GridGeom& g = p->g;
  {
    ProfScope ps(p, s, "passB_fwd_set", 8.0 * g.nv * as.rows.count + 12.0 * as.nS,
                 (double)g.nv * as.nS);
    const dim3 grid((unsigned)((g.nv + 255) / 256), (unsigned)as.nrows);
    if (g.M >= 8192)
      hipLaunchKernelGGL((rows_fwd_direct_kernel<khb_for<8192>()>), grid, dim3(256), 0, s, g,
                         as.rowlist, as.pix, w, (const float*)p->corr, (c32*)p->H);
    else
      hipLaunchKernelGGL((rows_fwd_direct_kernel<khb_for<4096>()>), grid, dim3(256), 0, s, g,
                         as.rowlist, as.pix, w, (const float*)p->corr, (c32*)p->H);
    PC_LAUNCH_CHECK("rows_fwd_direct");
  }
  dispatch_M<float>(p, false, nullptr, nullptr, 1.0f, s, nullptr, &as.rows, false);
  launch_interp<float>(p, nullptr, out, s, base, stats);
}

void adjoint_grid_set(pc_plan* p, const c32* vis, const AtomSet& as, double* gout,
                      hipStream_t s) {
  if (p->Cw || p->precision != PC_PREC_FP32)
    fail(PC_ERR_UNSUPPORTED, "gridded set operators need a coplanar FP32 plan");
  const GridGeom& g = p->g;
  launch_spread<float>(p, vis, nullptr, s);
  dispatch_M<float>(p, true, nullptr, nullptr, 1.0f, s, nullptr, &as.rows, false);
  ProfScope ps(p, s, "passB_adj_set", 8.0 * g.nv * as.rows.count + 12.0 * as.nS,
               (double)g.nv * as.nS);
  if (g.M >= 8192)
    hipLaunchKernelGGL((atoms_adj_direct_kernel<khb_for<8192>()>), dim3((unsigned)as.nS),
                       dim3(256), 0, s, g, as.pix, (const c32*)p->H, (const float*)p->corr, gout);
  else
    hipLaunchKernelGGL((atoms_adj_direct_kernel<khb_for<4096>()>), dim3((unsigned)as.nS),
                       dim3(256), 0, s, g, as.pix, (const c32*)p->H, (const float*)p->corr, gout);
  PC_LAUNCH_CHECK("atoms_adj_direct");
}

// Small moves of the gridded restricted gradient: caller-order atoms into
// pixel order (weights widened to FP64), the gradient back, and visibilities
// between caller and plan order.
__global__ void atoms_to_set_kernel(int64_t nS, const int32_t* __restrict__ order,
                                    const float* __restrict__ weight, double* __restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nS) w[q] = (double)weight[order[q]];
}
__global__ void set_to_atoms_kernel(int64_t nS, const int32_t* __restrict__ order,
                                    const double* __restrict__ g, double* __restrict__ grad) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nS) grad[order[q]] = g[q];
}
__global__ void vis_to_plan_kernel(int64_t L, const int32_t* __restrict__ perm,
                                   const c32* __restrict__ in, c32* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L) out[k] = in[perm[k]];
}
__global__ void vis_to_caller_kernel(int64_t L, const int32_t* __restrict__ perm,
                                     const c32* __restrict__ in, c32* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L) out[perm[k]] = in[k];
}

void restricted_gradient_grid(pc_plan* p, const c32* vis, int64_t natoms, const int32_t* pix,
                              const float* weight, double* grad, c32* resid, hipStream_t s) {
  if (p->Cw || p->precision != PC_PREC_FP32)
    fail(PC_ERR_UNSUPPORTED, "the gridded restricted gradient needs a coplanar FP32 plan");
  const int64_t L = p->L;
  const unsigned lb = (unsigned)((L + 255) / 256);
  if (natoms == 0) {  // r = V
    if (resid)
      PC_HIP(hipMemcpyAsync(resid, vis, L * sizeof(c32), hipMemcpyDeviceToDevice, s));
    return;
  }
  // the set in pixel order, its occupied rows and their mask, on the host
  const int n = p->g.n;
  std::vector<int32_t> hp((size_t)natoms);
  PC_HIP(hipMemcpyAsync(hp.data(), pix, natoms * 4, hipMemcpyDeviceToHost, s));
  PC_HIP(hipStreamSynchronize(s));
  for (int64_t q = 0; q < natoms; ++q)
    PC_REQUIRE(hp[q] >= 0 && (int64_t)hp[q] < (int64_t)n * n, "pix out of [0, npix^2)");
  std::vector<int32_t> order((size_t)natoms);
  for (int64_t q = 0; q < natoms; ++q) order[q] = (int32_t)q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return hp[a] < hp[b]; });
  const int64_t words = (n + 31) / 32;
  std::vector<int32_t> rl;
  std::vector<uint32_t> mask((size_t)words, 0u);
  for (int64_t q = 0; q < natoms; ++q) {
    const int i = hp[order[q]] / n;
    if (q == 0 || i != hp[order[q - 1]] / n) rl.insert(rl.end(), {i, (int32_t)q, 0});
    rl.back() = (int32_t)(q + 1);
    mask[i >> 5] |= 1u << (i & 31);
  }
  const int64_t nrows = (int64_t)rl.size() / 3;
  // device scratch: [pixel-order pix | order | rows | mask | w | g | V in plan order]
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t o_ord = al(natoms * 4), o_rows = o_ord + al(natoms * 4);
  const size_t o_mask = o_rows + al(nrows * 12), o_w = o_mask + al(words * 4);
  const size_t o_g = o_w + al(natoms * 8), o_v = o_g + al(natoms * 8);
  const size_t total = o_v + al(L * sizeof(c32));
  unsigned char* d = (unsigned char*)ensure_atom_scratch(p, total);
  std::vector<unsigned char> up(o_w);
  for (int64_t q = 0; q < natoms; ++q) ((int32_t*)up.data())[q] = hp[order[q]];
  std::memcpy(up.data() + o_ord, order.data(), natoms * 4);
  std::memcpy(up.data() + o_rows, rl.data(), nrows * 12);
  std::memcpy(up.data() + o_mask, mask.data(), words * 4);
  PC_HIP(hipMemcpyAsync(d, up.data(), o_w, hipMemcpyHostToDevice, s));
  const int32_t* dord = (const int32_t*)(d + o_ord);
  double* w = (double*)(d + o_w);
  double* g = (double*)(d + o_g);
  const unsigned ab = (unsigned)((natoms + 255) / 256);
  hipLaunchKernelGGL(atoms_to_set_kernel, dim3(ab), dim3(256), 0, s, natoms, dord, weight, w);
  PC_LAUNCH_CHECK("atoms_to_set");
  const AtomSet as{natoms, (const int32_t*)d, (const int3*)(d + o_rows), nrows,
                   RowMask{(const uint32_t*)(d + o_mask), nrows}};
  // r = V - Phi_S x in plan order, then Phi_S* r
  c32* vp = (c32*)(d + o_v);
  c32* r = (c32*)p->vis_scratch;
  hipLaunchKernelGGL(vis_to_plan_kernel, dim3(lb), dim3(256), 0, s, L, p->perm, vis, vp);
  PC_LAUNCH_CHECK("vis_to_plan");
  forward_grid_set(p, as, w, vp, nullptr, r, s);
  adjoint_grid_set(p, r, as, g, s);
  hipLaunchKernelGGL(set_to_atoms_kernel, dim3(ab), dim3(256), 0, s, natoms, dord, g, grad);
  PC_LAUNCH_CHECK("set_to_atoms");
  if (resid) {
    hipLaunchKernelGGL(vis_to_caller_kernel, dim3(lb), dim3(256), 0, s, L, p->perm, r, resid);
    PC_LAUNCH_CHECK("vis_to_caller");
  }
  PC_HIP(hipStreamSynchronize(s));  // the host staging above goes out of scope
}

void maxkey_read(pc_plan* p, hipStream_t s, double* max_abs, int64_t* argmax) {
  unsigned long long key = 0;
  PC_HIP(hipMemcpyAsync(&key, p->maxkey, sizeof(key), hipMemcpyDeviceToHost, s));
  PC_HIP(hipStreamSynchronize(s));
  maxkey_decode(key, max_abs, argmax);
}

void maxkey_decode(unsigned long long key, double* max_abs, int64_t* argmax) {
  const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)(key & 0xffffffffu);
  float f;
  std::memcpy(&f, &hi, 4);
  if (max_abs) *max_abs = (double)f;
  if (argmax) *argmax = (int64_t)(0xffffffffu - lo);
}

// The w-stacked adjoint: per plane, weights, spread, pass A and the rotating
// pass B; then the w correction and the maximum.
static void adjoint_grid_w(pc_plan* p, const c32* vis, bool vis_sorted, float* image, float scale,
                           hipStream_t s) {
  const WStack& ws = p->ws;
  const float R = 0.5f * (float)p->g.W;
  const float c0 = (float)(p->g.beta64 * 1.4426950408889634);  // beta log2(e)
  const unsigned nb = (unsigned)((p->L + 255) / 256);
  for (int j = 0; j < ws.nplanes; ++j) {
    const WPlane wp{ws.w0 + j * ws.dw, ws.cmid, j == 0 ? 1 : 0};
    {
      ProfScope ps(p, s, "wplane", p->L * 24.0, (double)p->L);
      hipLaunchKernelGGL(wplane_kernel, dim3(nb), dim3(256), 0, s, p->L, p->Cw, vis,
                         vis_sorted ? nullptr : p->perm, wp.wj, 1.0 / ws.dw, ws.cmid, R * R,
                         c0 / R, c0, (c32*)p->wvals);
      PC_LAUNCH_CHECK("wplane");
    }
    launch_spread<float>(p, (const c32*)p->wvals, nullptr, s);  // also clears the max key
    dispatch_M<float>(p, true, image, nullptr, scale, s, &wp);
  }
  const int64_t N = (int64_t)p->g.n * p->g.n;
  ProfScope ps(p, s, "wfinal", 8.0 * N, (double)N);
  const unsigned nbf = (unsigned)std::min<int64_t>((N + 255) / 256, 1024);
  hipLaunchKernelGGL(wfinal_kernel, dim3(nbf), dim3(256), 0, s, p->g, ws,
                     p->wquad, image, p->maxkey, p->max_positive);
  PC_LAUNCH_CHECK("wfinal");
}

template <typename R>
void adjoint_grid(pc_plan* p, const cpx<R>* vis, bool vis_sorted, R* image, R scale,
                  hipStream_t s, const RowMask* rows) {
  if (p->Cw) {
    if (rows) fail(PC_ERR_UNSUPPORTED, "a row mask with the w-stacked adjoint");
    if constexpr (sizeof(R) == 4) {
      adjoint_grid_w(p, vis, vis_sorted, image, scale, s);
      return;
    }
    fail(PC_ERR_UNSUPPORTED, "w-stacked adjoint of an FP64 plan");
  }
  launch_spread<R>(p, vis, vis_sorted ? nullptr : p->perm, s);  // also clears the max key
  dispatch_M<R>(p, true, image, nullptr, scale, s, nullptr, rows);
}

template <typename R>
void forward_grid(pc_plan* p, const R* image, cpx<R>* vis_out, bool out_sorted, hipStream_t s,
                  const RowMask* rows, const cpx<R>* base, double* stats) {
  if (p->Cw)
    fail(PC_ERR_UNSUPPORTED,
         "the gridded forward operator needs a coplanar plan (w = 0); the direct sums take w");
  if (base && !out_sorted) fail(PC_ERR_INVALID_ARG, "forward_grid: a base needs plan order");
  dispatch_M<R>(p, false, nullptr, image, R(1), s, nullptr, rows);
  launch_interp<R>(p, out_sorted ? nullptr : p->perm, vis_out, s, base, stats);
}

// ----------------------------------------------------------------------------
// Batched adjoint across plans
// ----------------------------------------------------------------------------
namespace {
struct Blob {
  std::vector<unsigned char> bytes;
  template <typename T>
  size_t put(const std::vector<T>& v) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

template <int M>
struct PassShape {
  static constexpr int CB = sizeof(c32);
  static constexpr int NBA = (M * CB >= Shapes<float>::lds_a) ? 1 : Shapes<float>::lds_a / (M * CB);
  static constexpr int NTA = nt_for<NBA * M / 16>();
  static constexpr int NBB = nb_passB<float, M>();
  static constexpr int NTB = nt_for<NBB * M / 16>();
};

int passA_blocks(int M, int nv) {
  switch (M) {
#define PC_M(m) case m: return (nv + PassShape<m>::NBA - 1) / PassShape<m>::NBA;
    PC_M(32) PC_M(64) PC_M(128) PC_M(256) PC_M(512) PC_M(1024) PC_M(2048) PC_M(4096) PC_M(8192)
    PC_M(16384)
#undef PC_M
  }
  return 0;
}

int passB_blocks(int M) {
  switch (M) {
#define PC_M(m) case m: return (m / 2) / PassShape<m>::NBB;
    PC_M(32) PC_M(64) PC_M(128) PC_M(256) PC_M(512) PC_M(1024) PC_M(2048) PC_M(4096) PC_M(8192)
    PC_M(16384)
#undef PC_M
  }
  return 0;
}

template <int M>
void launch_pass_batch(bool passA, const AdjJob* jobs, const int2* items, int nitems,
                       hipStream_t s) {
  using P = PassShape<M>;
  if (passA) {
    const size_t lds = (size_t)padded(P::NBA * M) * P::CB;
    set_lds((const void*)passA_batch_kernel<M, P::NBA, P::NTA>, lds);
    hipLaunchKernelGGL((passA_batch_kernel<M, P::NBA, P::NTA>), dim3(nitems), dim3(P::NTA), lds, s,
                       jobs, items);
    PC_LAUNCH_CHECK("passA_batch");
  } else {
    const size_t lds = (size_t)padded(P::NBB * M) * P::CB;
    set_lds((const void*)passB_batch_kernel<M, P::NBB, P::NTB>, lds);
    hipLaunchKernelGGL((passB_batch_kernel<M, P::NBB, P::NTB>), dim3(nitems), dim3(P::NTB), lds, s,
                       jobs, items);
    PC_LAUNCH_CHECK("passB_batch");
  }
}

void pass_batch(int M, bool passA, const AdjJob* jobs, const int2* items, int nitems,
                hipStream_t s) {
  switch (M) {
#define PC_M(m) case m: launch_pass_batch<m>(passA, jobs, items, nitems, s); return;
    PC_M(32) PC_M(64) PC_M(128) PC_M(256) PC_M(512) PC_M(1024) PC_M(2048) PC_M(4096) PC_M(8192)
    PC_M(16384)
#undef PC_M
  }
  fail(PC_ERR_UNSUPPORTED, "fine grid size");
}

template <int W>
void launch_spread_batch(const AdjJob* jobs, const int2* items, int nitems, hipStream_t s) {
  if constexpr (W <= 8) {  // grouped work lists: items are (job, workgroup)
    constexpr size_t lds = SpreadG<W>::lds_bytes;
    hipLaunchKernelGGL((spread_quad_batch_kernel<W>), dim3(nitems), dim3(64 * kSpreadQuad), lds,
                       s, jobs, items);
  } else {
    constexpr size_t lds = SpreadCfg<float, W>::lds_bytes;
    set_lds((const void*)spread_batch_kernel<W>, lds);
    hipLaunchKernelGGL((spread_batch_kernel<W>), dim3(nitems), dim3(64), lds, s, jobs, items);
  }
  PC_LAUNCH_CHECK("spread_batch");
}

void spread_batch(int W, const AdjJob* jobs, const int2* items, int nitems, hipStream_t s) {
  switch (W) {
#define PC_W(w) case w: launch_spread_batch<w>(jobs, items, nitems, s); return;
    PC_W(2) PC_W(3) PC_W(4) PC_W(5) PC_W(6) PC_W(7) PC_W(8) PC_W(9) PC_W(10) PC_W(11) PC_W(12)
    PC_W(13) PC_W(14) PC_W(15) PC_W(16)
#undef PC_W
  }
  fail(PC_ERR_UNSUPPORTED, "kernel width");
}
}  // namespace

void BatchCtx::release() {
  if (pending && done) (void)hipEventSynchronize(done);
  pending = false;
  if (dev) (void)hipFree(dev);
  if (host) (void)hipHostFree(host);
  if (done) (void)hipEventDestroy(done);
  dev = host = nullptr;
  dev_bytes = host_bytes = 0;
  done = nullptr;
}

void adjoint_grid_batch(BatchCtx& ctx, pc_plan* const* plans, const c32* const* vis,
                        const bool* vis_sorted, float* const* images, const float* scales, int n,
                        hipStream_t s) {
  if (n <= 0) return;
  // w-stacked plans run on their own, ahead of the shared launches
  {
    std::vector<int> flat;
    for (int j = 0; j < n; ++j) {
      PC_REQUIRE(plans[j] && plans[j]->precision == PC_PREC_FP32, "batched adjoint needs FP32 plans");
      if (plans[j]->Cw)
        adjoint_grid<float>(plans[j], vis[j], vis_sorted[j], images[j],
                            scales ? scales[j] : 1.0f, s);
      else
        flat.push_back(j);
    }
    if ((int)flat.size() < n) {
      if (flat.empty()) return;
      std::vector<pc_plan*> fp;
      std::vector<const c32*> fv;
      std::unique_ptr<bool[]> fs(new bool[flat.size()]);
      std::vector<float*> fi;
      std::vector<float> fsc;
      for (size_t q = 0; q < flat.size(); ++q) {
        const int j = flat[q];
        fp.push_back(plans[j]);
        fv.push_back(vis[j]);
        fs[q] = vis_sorted[j];
        fi.push_back(images[j]);
        fsc.push_back(scales ? scales[j] : 1.0f);
      }
      adjoint_grid_batch(ctx, fp.data(), fv.data(), fs.get(), fi.data(), fsc.data(),
                         (int)flat.size(), s);
      return;
    }
  }
  if (!ctx.done) PC_HIP(hipEventCreateWithFlags(&ctx.done, hipEventDisableTiming));
  if (ctx.pending) PC_HIP(hipEventSynchronize(ctx.done));
  // job descriptors and work lists
  std::vector<AdjJob> jobs(n);
  std::vector<std::pair<int32_t, int2>> sitems;  // (work, (job, chunk))
  std::vector<int2> fitems;
  std::vector<int> Ms, Ws;
  for (int j = 0; j < n; ++j) {
    pc_plan* p = plans[j];
    PC_REQUIRE(p && p->precision == PC_PREC_FP32, "batched adjoint needs FP32 plans");
    AdjJob& J = jobs[j];
    J.g = p->g;
    J.chunks = p->chunks;
    J.fold = p->fold;
    J.flags = p->tile_flags;
    J.cell = p->cell;
    J.off = (const float*)p->off;
    J.vals = vis[j];
    J.perm = vis_sorted[j] ? nullptr : p->perm;
    J.grid = (c32*)p->grid;
    J.partials = (c32*)p->partials;
    J.H = (c32*)p->H;
    J.image = images[j];
    J.tw = (const c32*)p->twiddle;
    J.corr = (const float*)p->corr;
    J.scale = scales ? scales[j] : 1.0f;
    J.maxkey = p->maxkey;
    J.positive = p->max_positive;
    J.rows = nullptr;
    // one entry per workgroup: a group of four items, or one item
    for (size_t c = 0; c < p->chunk_work.size(); ++c)
      sitems.push_back({p->chunk_work[c], make_int2(j, (int)c)});
    for (int64_t f = 0; f < p->n_fold; ++f) fitems.push_back(make_int2(j, (int)f));
    if (std::find(Ms.begin(), Ms.end(), p->g.M) == Ms.end()) Ms.push_back(p->g.M);
    if (std::find(Ws.begin(), Ws.end(), p->g.W) == Ws.end()) Ws.push_back(p->g.W);
  }
  // longest spreading items first across all plans
  std::stable_sort(sitems.begin(), sitems.end(),
                   [](const std::pair<int32_t, int2>& a, const std::pair<int32_t, int2>& b) {
                     return a.first > b.first;
                   });
  Blob blob;
  const size_t o_jobs = blob.put(jobs);
  std::vector<size_t> o_spread(Ws.size()), n_spread(Ws.size());
  for (size_t w = 0; w < Ws.size(); ++w) {
    std::vector<int2> it;
    for (auto& e : sitems)
      if (plans[e.second.x]->g.W == Ws[w]) it.push_back(e.second);
    o_spread[w] = blob.put(it);
    n_spread[w] = it.size();
  }
  const size_t o_fold = blob.put(fitems);
  std::vector<size_t> oA(Ms.size()), nA(Ms.size()), oB(Ms.size()), nB(Ms.size());
  for (size_t m = 0; m < Ms.size(); ++m) {
    std::vector<int2> a, b;
    for (int j = 0; j < n; ++j) {
      if (plans[j]->g.M != Ms[m]) continue;
      const int na = passA_blocks(Ms[m], plans[j]->g.nv), nbk = passB_blocks(Ms[m]);
      for (int r = 0; r < na; ++r) a.push_back(make_int2(j, r));
      for (int r = 0; r < nbk; ++r) b.push_back(make_int2(j, r));
    }
    oA[m] = blob.put(a);
    nA[m] = a.size();
    oB[m] = blob.put(b);
    nB[m] = b.size();
  }
  const size_t bytes = blob.bytes.size();
  if (ctx.host_bytes < bytes) {
    if (ctx.host) (void)hipHostFree(ctx.host);
    ctx.host = nullptr;
    ctx.host_bytes = 0;
    PC_HIP(hipHostMalloc((void**)&ctx.host, bytes * 2));
    ctx.host_bytes = bytes * 2;
  }
  if (ctx.dev_bytes < bytes) {
    if (ctx.dev) (void)hipFree(ctx.dev);
    ctx.dev = nullptr;
    ctx.dev_bytes = 0;
    PC_HIP(hipMalloc((void**)&ctx.dev, bytes * 2));
    ctx.dev_bytes = bytes * 2;
  }
  std::memcpy(ctx.host, blob.bytes.data(), bytes);
  PC_HIP(hipMemcpyAsync(ctx.dev, ctx.host, bytes, hipMemcpyHostToDevice, s));
  const AdjJob* djobs = (const AdjJob*)(ctx.dev + o_jobs);
  for (size_t w = 0; w < Ws.size(); ++w)
    if (n_spread[w])
      spread_batch(Ws[w], djobs, (const int2*)(ctx.dev + o_spread[w]), (int)n_spread[w], s);
  if (!fitems.empty()) {
    hipLaunchKernelGGL(fold_batch_kernel, dim3((unsigned)fitems.size(), kTile * kTile / 64),
                       dim3(64 * kFoldSub), 0, s, djobs, (const int2*)(ctx.dev + o_fold));
    PC_LAUNCH_CHECK("fold_batch");
  }
  for (size_t m = 0; m < Ms.size(); ++m)
    if (nA[m]) pass_batch(Ms[m], true, djobs, (const int2*)(ctx.dev + oA[m]), (int)nA[m], s);
  for (size_t m = 0; m < Ms.size(); ++m)
    if (nB[m]) pass_batch(Ms[m], false, djobs, (const int2*)(ctx.dev + oB[m]), (int)nB[m], s);
  PC_HIP(hipEventRecord(ctx.done, s));
  ctx.pending = true;
}

template void adjoint_grid<float>(pc_plan*, const c32*, bool, float*, float, hipStream_t,
                                  const RowMask*);
template void adjoint_grid<double>(pc_plan*, const c64*, bool, double*, double, hipStream_t,
                                   const RowMask*);
template void forward_grid<float>(pc_plan*, const float*, c32*, bool, hipStream_t,
                                  const RowMask*, const c32*, double*);
template void forward_grid<double>(pc_plan*, const double*, c64*, bool, hipStream_t,
                                   const RowMask*, const c64*, double*);

}  // namespace pc
