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
#include <cstring>

#include "common.h"
#include "fft_lds.h"

namespace pc {

template <typename R>
__device__ __forceinline__ R es_kernel(R z, R beta) {
  // exponential of semicircle: exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1
  R t = R(1) - z * z;
  if (!(t > R(0))) return R(0);
  if constexpr (sizeof(R) == 4) {
    return __expf(beta * (__builtin_sqrtf(t) - 1.0f));
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
  int b = c - origin;
  if (wrap) {
    b = ((b % M) + M) % M;
    if (b > M - W) b -= M;
  }
  return b;
}

template <typename R, int W>
__global__ __launch_bounds__(256) void spread_kernel(GridGeom g, const SpreadChunk* __restrict__ chunks,
                                                     const uint32_t* __restrict__ cell,
                                                     const R* __restrict__ off,
                                                     const cpx<R>* __restrict__ vals,
                                                     const int32_t* __restrict__ perm,
                                                     cpx<R>* __restrict__ grid,
                                                     cpx<R>* __restrict__ partials) {
  constexpr int S = kTile + 1;  // padded LDS row stride
  __shared__ R sre[kTile * S];
  __shared__ R sim[kTile * S];
  const SpreadChunk ch = chunks[blockIdx.x];
  for (int i = threadIdx.x; i < kTile * S; i += blockDim.x) {
    sre[i] = R(0);
    sim[i] = R(0);
  }
  __syncthreads();
  const int tv = ch.tile / g.ntu, tu = ch.tile - tv * g.ntu;
  const int ov = g.v0 + tv * kTile, ou = g.u0 + tu * kTile;
  const R inv = R(2) / R(W);
  const R beta = sizeof(R) == 4 ? (R)g.beta : (R)g.beta64;
#pragma unroll 1
  for (int r = 0; r < 4; ++r) {
#pragma unroll 1
    for (int s = ch.beg[r] + (int)threadIdx.x; s < ch.end[r]; s += blockDim.x) {
      const uint32_t c = cell[s];
      const int bu = tile_base((int)(c & 0xffffu), ou, g.M, W, g.wrap);
      const int bv = tile_base((int)(c >> 16), ov, g.M, W, g.wrap);
      const R su = off[2 * s], sv = off[2 * s + 1];
      const cpx<R> val = perm ? vals[perm[s]] : vals[s];
      R ku[W], kv[W];
#pragma unroll
      for (int t = 0; t < W; ++t) {
        ku[t] = es_kernel<R>((su + R(t)) * inv, beta);
        kv[t] = es_kernel<R>((sv + R(t)) * inv, beta);
      }
#pragma unroll
      for (int a = 0; a < W; ++a) {
        int y;
        if (!tap_local(bv, a, g.M, g.wrap, y)) continue;
        const R wr = val.x * kv[a], wi = val.y * kv[a];
#pragma unroll
        for (int b = 0; b < W; ++b) {
          int x;
          if (!tap_local(bu, b, g.M, g.wrap, x)) continue;
          atomicAdd(&sre[y * S + x], wr * ku[b]);
          atomicAdd(&sim[y * S + x], wi * ku[b]);
        }
      }
    }
  }
  __syncthreads();
  if (ch.slot < 0) {
    cpx<R>* dst = grid + (size_t)(tv * kTile) * g.nu + tu * kTile;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
      const int y = i / kTile, x = i - y * kTile;
      dst[(size_t)y * g.nu + x] = {sre[y * S + x], sim[y * S + x]};
    }
  } else {
    cpx<R>* dst = partials + (size_t)ch.slot * kTile * kTile;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
      const int y = i / kTile, x = i - y * kTile;
      dst[i] = {sre[y * S + x], sim[y * S + x]};
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void fold_kernel(GridGeom g, const FoldItem* __restrict__ items,
                                                   const cpx<R>* __restrict__ partials,
                                                   cpx<R>* __restrict__ grid) {
  const FoldItem it = items[blockIdx.x];
  const int tv = it.tile / g.ntu, tu = it.tile - tv * g.ntu;
  cpx<R>* dst = grid + (size_t)(tv * kTile) * g.nu + tu * kTile;
  for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
    R ax = 0, ay = 0;
    for (int q = 0; q < it.count; ++q) {
      const cpx<R> v = partials[(size_t)(it.first + q) * kTile * kTile + i];
      ax += v.x;
      ay += v.y;
    }
    const int y = i / kTile, x = i - y * kTile;
    dst[(size_t)y * g.nu + x] = {ax, ay};
  }
}

// Pass A of the adjoint: rows of the band grid (fixed v), FFT along u.
template <typename R, int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passA_adj_kernel(GridGeom g, const cpx<R>* __restrict__ grid,
                                                        cpx<R>* __restrict__ H,
                                                        const cpx<R>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  constexpr int n = M / 2;
  const int row0 = blockIdx.x * NB;
  for (int idx = threadIdx.x; idx < NB * M; idx += NT) {
    const int b = idx / M, m = idx - b * M;
    const int row = row0 + b;
    cpx<R> v = {R(0), R(0)};
    const int rel = m - g.u0;
    if (row < g.nv && (unsigned)rel < (unsigned)g.nu) v = grid[(size_t)row * g.nu + rel];
    buf[idx] = v;
  }
  __syncthreads();
  lds_fft<R, M, NB, NT, +1>(buf, tw);
  for (int idx = threadIdx.x; idx < NB * n; idx += NT) {
    const int b = idx / n, i = idx - b * n;
    const int row = row0 + b;
    if (row < g.nv) {
      int f = i - n / 2;
      if (f < 0) f += M;
      H[(size_t)row * n + i] = buf[b * M + f];
    }
  }
}

__device__ __forceinline__ unsigned long long max_key(float a, int idx) {
  return ((unsigned long long)__float_as_uint(a) << 32) | (unsigned long long)(0xffffffffu - (unsigned)idx);
}

// Pass B of the adjoint: NB image rows i; FFT along v of H[:, i]; correction;
// write image rows; fused max |eta| with lowest-index ties.
template <typename R, int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passB_adj_kernel(GridGeom g, const cpx<R>* __restrict__ H,
                                                        R* __restrict__ image,
                                                        const cpx<R>* __restrict__ tw,
                                                        const R* __restrict__ corr, R scale,
                                                        unsigned long long* __restrict__ maxkey) {
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  constexpr int n = M / 2;
  const int i0 = blockIdx.x * NB;
  for (int idx = threadIdx.x; idx < NB * M; idx += NT) {
    const int m = idx / NB, b = idx - m * NB;
    const int rel = m - g.v0;
    cpx<R> v = {R(0), R(0)};
    if ((unsigned)rel < (unsigned)g.nv) v = H[(size_t)rel * n + i0 + b];
    buf[b * M + m] = v;
  }
  __syncthreads();
  lds_fft<R, M, NB, NT, +1>(buf, tw);
  unsigned long long best = 0;
  const R dl = (R)g.dl;
  for (int idx = threadIdx.x; idx < NB * n; idx += NT) {
    const int b = idx / n, j = idx - b * n;
    const int i = i0 + b;
    int f = j - n / 2;
    if (f < 0) f += M;
    const R l = (R)(i - n / 2) * dl, mm = (R)(j - n / 2) * dl;
    const R nn = sqrt(R(1) - l * l - mm * mm);
    const R val = buf[b * M + f].x * corr[i] * corr[j] * scale / nn;
    image[(size_t)i * n + j] = val;
    const unsigned long long key = max_key((float)fabs(val), i * n + j);
    best = key > best ? key : best;
  }
  // block max
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  __shared__ unsigned long long wbest[NT / 64];
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < NT / 64; ++w) m = wbest[w] > m ? wbest[w] : m;
    atomicMax(maxkey, m);
  }
}

// Forward pass B^T: NB image rows i, pre-correct, FFT along v (sign -1),
// keep the band rows: Hf[v_rel][i].
template <typename R, int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passB_fwd_kernel(GridGeom g, const R* __restrict__ image,
                                                        cpx<R>* __restrict__ H,
                                                        const cpx<R>* __restrict__ tw,
                                                        const R* __restrict__ corr) {
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  constexpr int n = M / 2;
  const int i0 = blockIdx.x * NB;
  const R dl = (R)g.dl;
  for (int idx = threadIdx.x; idx < NB * M; idx += NT) {
    const int b = idx / M, m = idx - b * M;  // m: frequency slot
    int f = m < n / 2 ? m : m - M;            // signed frequency b
    cpx<R> v = {R(0), R(0)};
    if (f >= -n / 2 && f < n / 2) {
      const int i = i0 + b, j = f + n / 2;
      const R l = (R)(i - n / 2) * dl, mm = (R)(j - n / 2) * dl;
      const R nn = sqrt(R(1) - l * l - mm * mm);
      v.x = image[(size_t)i * n + j] * corr[i] * corr[j] / nn;
    }
    buf[idx] = v;
  }
  __syncthreads();
  lds_fft<R, M, NB, NT, -1>(buf, tw);
  for (int idx = threadIdx.x; idx < NB * g.nv; idx += NT) {
    const int rel = idx / NB, b = idx - rel * NB;
    int m = g.v0 + rel;
    H[(size_t)rel * n + i0 + b] = buf[b * M + m];
  }
}

// Forward pass A^T: band rows v; FFT along u (sign -1) of Hf[v][:] placed at
// the n central frequencies; keep the band columns.
template <typename R, int M, int NB, int NT>
__global__ __launch_bounds__(NT) void passA_fwd_kernel(GridGeom g, const cpx<R>* __restrict__ H,
                                                        cpx<R>* __restrict__ grid,
                                                        const cpx<R>* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem_raw);
  constexpr int n = M / 2;
  const int row0 = blockIdx.x * NB;
  for (int idx = threadIdx.x; idx < NB * M; idx += NT) {
    const int b = idx / M, m = idx - b * M;
    const int row = row0 + b;
    int f = m < n / 2 ? m : m - M;
    cpx<R> v = {R(0), R(0)};
    if (row < g.nv && f >= -n / 2 && f < n / 2) v = H[(size_t)row * n + f + n / 2];
    buf[idx] = v;
  }
  __syncthreads();
  lds_fft<R, M, NB, NT, -1>(buf, tw);
  for (int idx = threadIdx.x; idx < NB * g.nu; idx += NT) {
    const int b = idx / g.nu, rel = idx - b * g.nu;
    const int row = row0 + b;
    if (row < g.nv) grid[(size_t)row * g.nu + rel] = buf[b * M + g.u0 + rel];
  }
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
  R ku[W], kv[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    ku[t] = es_kernel<R>((su + R(t)) * inv, beta);
    kv[t] = es_kernel<R>((sv + R(t)) * inv, beta);
  }
  R ax = 0, ay = 0;
#pragma unroll
  for (int a = 0; a < W; ++a) {
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
    ax += rx * kv[a];
    ay += ry * kv[a];
  }
  const int64_t d = perm ? perm[s] : s;
  out[d] = {ax, ay};
}

__global__ void maxkey_reset_kernel(unsigned long long* k) { *k = 0ull; }

// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------
template <typename R, int W>
static void launch_spread_w(pc_plan* p, const cpx<R>* vals, const int32_t* perm, hipStream_t s) {
  const double rb = sizeof(R);
  ProfScope ps(p, s, "spread", p->L * (4 + 4 * rb) + 2 * rb * p->g.nu * p->g.nv, (double)p->L);
  hipLaunchKernelGGL((spread_kernel<R, W>), dim3((unsigned)p->n_chunks), dim3(256), 0, s, p->g,
                     p->chunks, p->cell, (const R*)p->off, vals, perm, (cpx<R>*)p->grid,
                     (cpx<R>*)p->partials);
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
    hipLaunchKernelGGL((fold_kernel<R>), dim3((unsigned)p->n_fold), dim3(256), 0, s, p->g, p->fold,
                       (const cpx<R>*)p->partials, (cpx<R>*)p->grid);
    PC_LAUNCH_CHECK("fold");
  }
}

template <typename R, int W>
static void launch_interp_w(pc_plan* p, const int32_t* perm, cpx<R>* out, hipStream_t s) {
  const unsigned nb = (unsigned)((p->L + 255) / 256);
  const double rb = sizeof(R);
  ProfScope ps(p, s, "interp", p->L * (4 + 4 * rb) + 2 * rb * p->g.nu * p->g.nv, (double)p->L);
  hipLaunchKernelGGL((interp_kernel<R, W>), dim3(nb), dim3(256), 0, s, p->g, p->L, p->cell,
                     (const R*)p->off, (const cpx<R>*)p->grid, perm, out);
  PC_LAUNCH_CHECK("interp");
}

template <typename R>
static void launch_interp(pc_plan* p, const int32_t* perm, cpx<R>* out, hipStream_t s) {
  switch (p->g.W) {
#define PC_W(w) \
  case w:       \
    launch_interp_w<R, w>(p, perm, out, s); \
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
  static constexpr int lds_b = 128 * 1024;
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
static void run_passes_adj(pc_plan* p, R* image, R scale, hipStream_t s) {
  constexpr int CB = sizeof(cpx<R>);
  constexpr int NBA = (M * CB >= Shapes<R>::lds_a) ? 1 : Shapes<R>::lds_a / (M * CB);
  constexpr int NTA = 256;
  constexpr int NBB = nb_passB<R, M>();
  constexpr int NTB = nt_for<NBB * M / 16>();
  const GridGeom& g = p->g;
  const size_t lda = (size_t)NBA * M * CB, ldb = (size_t)NBB * M * CB;
  const double nvn = (double)g.nv * g.n * CB;
  set_lds((const void*)passA_adj_kernel<R, M, NBA, NTA>, lda);
  {
    ProfScope ps(p, s, "passA_adj", (double)g.nv * g.nu * CB + nvn, (double)g.nv * M);
    hipLaunchKernelGGL((passA_adj_kernel<R, M, NBA, NTA>), dim3((g.nv + NBA - 1) / NBA), dim3(NTA),
                       lda, s, g, (const cpx<R>*)p->grid, (cpx<R>*)p->H, (const cpx<R>*)p->twiddle);
    PC_LAUNCH_CHECK("passA_adj");
  }
  set_lds((const void*)passB_adj_kernel<R, M, NBB, NTB>, ldb);
  ProfScope ps(p, s, "passB_adj", nvn + (double)g.n * g.n * sizeof(R), (double)g.n * M);
  hipLaunchKernelGGL((passB_adj_kernel<R, M, NBB, NTB>), dim3((M / 2) / NBB), dim3(NTB), ldb, s, g,
                     (const cpx<R>*)p->H, image, (const cpx<R>*)p->twiddle, (const R*)p->corr,
                     scale, p->maxkey);
  PC_LAUNCH_CHECK("passB_adj");
}

template <typename R, int M>
static void run_passes_fwd(pc_plan* p, const R* image, hipStream_t s) {
  constexpr int CB = sizeof(cpx<R>);
  constexpr int NBA = (M * CB >= Shapes<R>::lds_a) ? 1 : Shapes<R>::lds_a / (M * CB);
  constexpr int NTA = 256;
  constexpr int NBB = nb_passB<R, M>();
  constexpr int NTB = nt_for<NBB * M / 16>();
  const GridGeom& g = p->g;
  const size_t lda = (size_t)NBA * M * CB, ldb = (size_t)NBB * M * CB;
  const double nvn = (double)g.nv * g.n * CB;
  set_lds((const void*)passB_fwd_kernel<R, M, NBB, NTB>, ldb);
  {
  ProfScope ps(p, s, "passB_fwd", nvn + (double)g.n * g.n * sizeof(R), (double)g.n * M);
  hipLaunchKernelGGL((passB_fwd_kernel<R, M, NBB, NTB>), dim3((M / 2) / NBB), dim3(NTB), ldb, s,
                     g, image, (cpx<R>*)p->H, (const cpx<R>*)p->twiddle, (const R*)p->corr);
  PC_LAUNCH_CHECK("passB_fwd");
  }
  set_lds((const void*)passA_fwd_kernel<R, M, NBA, NTA>, lda);
  ProfScope ps(p, s, "passA_fwd", (double)g.nv * g.nu * CB + nvn, (double)g.nv * M);
  hipLaunchKernelGGL((passA_fwd_kernel<R, M, NBA, NTA>), dim3((g.nv + NBA - 1) / NBA), dim3(NTA),
                     lda, s, g, (const cpx<R>*)p->H, (cpx<R>*)p->grid, (const cpx<R>*)p->twiddle);
  PC_LAUNCH_CHECK("passA_fwd");
}

template <typename R>
static void dispatch_M(pc_plan* p, bool adjoint, R* img_out, const R* img_in, R scale,
                       hipStream_t s) {
  switch (p->g.M) {
#define PC_M(m)                                         \
  case m:                                               \
    if (adjoint)                                        \
      run_passes_adj<R, m>(p, img_out, scale, s);       \
    else                                                \
      run_passes_fwd<R, m>(p, img_in, s);               \
    return;
    PC_M(32) PC_M(64) PC_M(128) PC_M(256) PC_M(512) PC_M(1024) PC_M(2048) PC_M(4096) PC_M(8192)
#undef PC_M
    case 16384:
      if constexpr (sizeof(R) == 4) {
        if (adjoint)
          run_passes_adj<R, 16384>(p, img_out, scale, s);
        else
          run_passes_fwd<R, 16384>(p, img_in, s);
        return;
      }
      [[fallthrough]];
    default:
      fail(PC_ERR_UNSUPPORTED, "fine grid size " + std::to_string(p->g.M) +
                                   (sizeof(R) == 8 ? " in FP64" : "") + " is not a supported power of two");
  }
}

void maxkey_reset(pc_plan* p, hipStream_t s) {
  hipLaunchKernelGGL(maxkey_reset_kernel, dim3(1), dim3(1), 0, s, p->maxkey);
  PC_LAUNCH_CHECK("maxkey_reset");
}

void maxkey_read(pc_plan* p, hipStream_t s, double* max_abs, int64_t* argmax) {
  unsigned long long key = 0;
  PC_HIP(hipMemcpyAsync(&key, p->maxkey, sizeof(key), hipMemcpyDeviceToHost, s));
  PC_HIP(hipStreamSynchronize(s));
  const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)(key & 0xffffffffu);
  float f;
  std::memcpy(&f, &hi, 4);
  if (max_abs) *max_abs = (double)f;
  if (argmax) *argmax = (int64_t)(0xffffffffu - lo);
}

template <typename R>
void adjoint_grid(pc_plan* p, const cpx<R>* vis, bool vis_sorted, R* image, R scale,
                  hipStream_t s) {
  maxkey_reset(p, s);
  launch_spread<R>(p, vis, vis_sorted ? nullptr : p->perm, s);
  dispatch_M<R>(p, true, image, nullptr, scale, s);
}

template <typename R>
void forward_grid(pc_plan* p, const R* image, cpx<R>* vis_out, bool out_sorted, hipStream_t s) {
  dispatch_M<R>(p, false, nullptr, image, R(1), s);
  launch_interp<R>(p, out_sorted ? nullptr : p->perm, vis_out, s);
}

template void adjoint_grid<float>(pc_plan*, const c32*, bool, float*, float, hipStream_t);
template void adjoint_grid<double>(pc_plan*, const c64*, bool, double*, double, hipStream_t);
template void forward_grid<float>(pc_plan*, const float*, c32*, bool, hipStream_t);
template void forward_grid<double>(pc_plan*, const double*, c64*, bool, hipStream_t);

}  // namespace pc
