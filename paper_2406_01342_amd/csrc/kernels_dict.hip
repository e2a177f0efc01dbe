// Synthesis dictionary of Gaussian elements (Sect. 4.3, Eqs. params-synthesis
// and lasso-synthesis; the elements of Sect. 6.4).  The dictionary enters the
// solve only through three image-domain operations around the existing
// gridded operators: Phi Psi theta = forward_grid(synthesis(theta)) and
// Psi* Phi* r = analysis(adjoint_grid(r)), restricted to the active atoms by
// a gather.  All three are HBM/L2-bound stencils with separable taps.
#include <cmath>

#include "common.h"

namespace pc {

DictSpec make_dict(int n_scales, const double* sigma, const double* gamma) {
  PC_REQUIRE(n_scales >= 1 && n_scales <= kDictMaxScales, "n_scales must be in [1, 8]");
  PC_REQUIRE(sigma != nullptr && gamma != nullptr, "dictionary sigma/gamma are NULL");
  DictSpec D{};
  D.S = n_scales;
  for (int s = 0; s < n_scales; ++s) {
    PC_REQUIRE(std::isfinite(sigma[s]) && sigma[s] >= 0 && sigma[s] <= kDictMaxHalf / 2,
               "dictionary sigma must be in [0, 16]");
    PC_REQUIRE(std::isfinite(gamma[s]) && gamma[s] > 0, "dictionary gamma must be > 0");
    const int h = (int)std::floor(2.0 * sigma[s] + 1e-12);
    D.h[s] = h;
    D.gamma[s] = (float)gamma[s];
    if (h == 0) {
      D.taps[s][0] = 1.0f;
      continue;
    }
    double z = 0;
    for (int a = -h; a <= h; ++a) z += std::exp(-(double)a * a / (sigma[s] * sigma[s]));
    for (int a = -h; a <= h; ++a)
      D.taps[s][a + h] = (float)(std::exp(-(double)a * a / (sigma[s] * sigma[s])) / z);
  }
  return D;
}

// One thread copies the taps of the block's scale into LDS with uniform
// indexing into the by-value spec.
__device__ __forceinline__ void load_taps(const DictSpec& D, int s, float* tl) {
  if (threadIdx.x == 0)
    for (int k = 0; k <= 2 * D.h[s]; ++k) tl[k] = D.taps[s][k];
  __syncthreads();
}

// Workgroups are dealt to the XCDs (each with its own L2) round-robin; this
// renumbering gives each XCD a contiguous range of tiles (row-major over the
// image), so that the halo rows two neighbouring tiles share are read into
// one L2.
__device__ __forceinline__ int dict_tile_order(int b, int nb) {
  constexpr int kX = 8;
  const int q = nb / kX, r = nb % kX;
  const int x = b % kX, k = b / kX;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ unsigned long long dict_key(float a, uint32_t idx) {
  return ((unsigned long long)__float_as_uint(a) << 32) | (unsigned long long)(0xffffffffu - idx);
}

// Psi* for one scale on a kTI x kTJ output tile (one workgroup per tile,
// tiles ordered per XCD by dict_tile_order).  The (kTI + 2h) x (kTJ + 2h)
// input window (zeros outside the image) is staged in LDS once; the row pass
// writes (kTI + 2h) x kTJ partial sums to LDS, the column pass forms the
// outputs, scales by gamma_s, stores them coalesced and writes the tile's
// maximum key to keys[tile].  Threads are 4 rows x 64 columns.  Any
// half-width up to kDictMaxHalf (used above 16, where the register version
// would need too many taps and window values per lane).
constexpr int kTI = 64, kTJ = 64;

__global__ __launch_bounds__(256) void dict_tile_kernel(int n, DictSpec D, int s,
                                                        const float* __restrict__ img,
                                                        float* __restrict__ out, int positive,
                                                        unsigned long long* __restrict__ keys) {
  extern __shared__ float sm[];
  __shared__ float tl[kDictMaxTaps];
  __shared__ unsigned long long wbest[4];
  const int h = D.h[s], W = kTJ + 2 * h, R = kTI + 2 * h;
  float* win = sm;           // R x W
  float* mid = sm + R * W;   // R x kTJ
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int tb = dict_tile_order(blockIdx.x, gridDim.x), ntx = (n + kTJ - 1) / kTJ;
  const int i0 = (tb / ntx) * kTI, j0 = (tb - (tb / ntx) * ntx) * kTJ;
  if (threadIdx.x == 0)
    for (int k = 0; k <= 2 * h; ++k) tl[k] = D.taps[s][k];
  for (int r = ty; r < R; r += 4) {
    const int gi = i0 - h + r;
    const bool row_in = gi >= 0 && gi < n;
    for (int c = tx; c < W; c += 64) {
      const int gj = j0 - h + c;
      win[r * W + c] = (row_in && gj >= 0 && gj < n) ? img[(size_t)gi * n + gj] : 0.0f;
    }
  }
  __syncthreads();
  for (int r = ty; r < R; r += 4) {
    const float* w = win + r * W + tx;
    float acc = 0.0f;
    for (int b = 0; b <= 2 * h; ++b) acc += tl[b] * w[b];
    mid[r * kTJ + tx] = acc;
  }
  __syncthreads();
  const size_t N = (size_t)n * n;
  const float g = D.gamma[s];
  unsigned long long best = 0;
  const int gj = j0 + tx;
  for (int r = ty; r < kTI; r += 4) {
    const int gi = i0 + r;
    const float* m = mid + r * kTJ + tx;
    float acc = 0.0f;
    for (int a = 0; a <= 2 * h; ++a) acc += tl[a] * m[a * kTJ];
    if (gi < n && gj < n) {
      const float v = g * acc;
      const size_t e = (size_t)gi * n + gj;
      out[s * N + e] = v;
      const float kv = positive ? (v > 0.0f ? v : 0.0f) : fabsf(v);
      const unsigned long long k = dict_key(kv, (uint32_t)(s * N + e));
      best = k > best ? k : best;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  if (tx == 0) wbest[ty] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wbest[0];
    for (int w = 1; w < 4; ++w) m = wbest[w] > m ? wbest[w] : m;
    keys[tb] = m;
  }
}

// One workgroup per atom: its weighted element added into the image (float
// atomics; elements of nearby atoms overlap).
__global__ __launch_bounds__(256) void dict_synth_kernel(int n, DictSpec D, int64_t nS,
                                                         const int32_t* __restrict__ atoms,
                                                         const double* __restrict__ w,
                                                         float* __restrict__ img) {
  __shared__ float tl[kDictMaxTaps];
  const int64_t q = blockIdx.x;
  const int64_t N = (int64_t)n * n;
  const int64_t a = atoms[q];
  const int s = (int)(a / N);
  const int64_t pix = a - (int64_t)s * N;
  const int i0 = (int)(pix / n), j0 = (int)(pix - (int64_t)(pix / n) * n);
  load_taps(D, s, tl);
  const double wq = w[q];
  if (wq == 0.0) return;  // uniform per workgroup, after the only barrier
  const int h = D.h[s], width = 2 * h + 1;
  const float gw = (float)(wq * (double)D.gamma[s]);
  for (int k = threadIdx.x; k < width * width; k += 256) {
    const int da = k / width - h, db = k - (k / width) * width - h;
    const int i = i0 + da, j = j0 + db;
    if (i >= 0 && i < n && j >= 0 && j < n)
      atomicAdd(img + (size_t)i * n + j, gw * tl[da + h] * tl[db + h]);
  }
}

// One workgroup per atom: (Psi* img) at the atom, summed in FP64.
__global__ __launch_bounds__(256) void dict_gather_kernel(int n, DictSpec D, int64_t nS,
                                                          const int32_t* __restrict__ atoms,
                                                          const float* __restrict__ img,
                                                          double* __restrict__ out) {
  __shared__ float tl[kDictMaxTaps];
  __shared__ double red[4];
  const int64_t q = blockIdx.x;
  const int64_t N = (int64_t)n * n;
  const int64_t a = atoms[q];
  const int s = (int)(a / N);
  const int64_t pix = a - (int64_t)s * N;
  const int i0 = (int)(pix / n), j0 = (int)(pix - (int64_t)(pix / n) * n);
  load_taps(D, s, tl);
  const int h = D.h[s], width = 2 * h + 1;
  double acc = 0.0;
  for (int k = threadIdx.x; k < width * width; k += 256) {
    const int da = k / width - h, db = k - (k / width) * width - h;
    const int i = i0 + da, j = j0 + db;
    if (i >= 0 && i < n && j >= 0 && j < n)
      acc += (double)(tl[da + h] * tl[db + h]) * (double)img[(size_t)i * n + j];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[q] = (((red[0] + red[1]) + red[2]) + red[3]) * (double)D.gamma[s];
}

// The same tile for a compile-time half-width H <= 16 (sigma <= 8, every
// scale of the paper), with the taps in registers and both passes as
// register sliding windows (a lane forms 16 consecutive outputs from 16 + 2H
// reads and 16 (2H + 1) FMAs):
//   vertical:   lane = window column, 16 output rows, reading the image
//               straight from L2 (loads coalesced along the row, all in
//               flight)                               -> mid[kTI][W + 1]
//   horizontal: lane = output row, wave = 16 columns  -> res[kTI][kTJ + 1]
// (odd row strides keep the lanes of the horizontal pass on distinct banks),
// then a coalesced store of res with the block's maximum key written to
// keys[tile] (no atomics; reduced by dict_key_reduce_kernel).  LDS holds only
// mid (res reuses it): kTI (W + 1) floats, W = kTJ + 2H, at most 24.8 KB, so
// that six workgroups share a compute unit.
template <int H>
__global__ __launch_bounds__(256) void dict_tile_h_kernel(int n, DictSpec D, int s,
                                                          const float* __restrict__ img,
                                                          float* __restrict__ out, int positive,
                                                          unsigned long long* __restrict__ keys) {
  constexpr int W = kTJ + 2 * H, T = 2 * H + 1, RB = 16;
  constexpr int MS = W + 1, RS = kTJ + 1;  // padded strides of mid and res
  static_assert(kTI == 64 && kTJ == 64, "one lane per output row, four 16-column waves");
  static_assert(RS <= MS, "res fits in mid");
  __shared__ float mid[kTI * MS];
  __shared__ unsigned long long wbest[4];
  float t[T];
#pragma unroll
  for (int k = 0; k < T; ++k) t[k] = D.taps[s][k];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int tb = dict_tile_order(blockIdx.x, gridDim.x), ntx = (n + kTJ - 1) / kTJ;
  const int i0 = (tb / ntx) * kTI, j0 = (tb - (tb / ntx) * ntx) * kTJ;
  for (int task = threadIdx.x; task < W * (kTI / RB); task += 256) {
    const int c = task % W, g = task / W;
    const int gj = j0 - H + c;
    const bool col_in = gj >= 0 && gj < n;
    float v[RB + 2 * H];
#pragma unroll
    for (int k = 0; k < RB + 2 * H; ++k) {
      const int gi = i0 - H + RB * g + k;
      v[k] = (col_in && gi >= 0 && gi < n) ? img[(size_t)gi * n + gj] : 0.0f;
    }
    float acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int k = 0; k < RB + 2 * H; ++k) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (k - r >= 0 && k - r < T) acc[r] += t[k - r] * v[k];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) mid[(RB * g + r) * MS + c] = acc[r];
  }
  __syncthreads();
  float acc[RB];
  {
    const float* m = mid + tx * MS + RB * ty;
#pragma unroll
    for (int c = 0; c < RB; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int k = 0; k < RB + 2 * H; ++k) {
      const float v = m[k];
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (k - c >= 0 && k - c < T) acc[c] += t[k - c] * v;
    }
  }
  __syncthreads();  // every lane has read mid: res overwrites it
  float* res = mid;
#pragma unroll
  for (int c = 0; c < RB; ++c) res[tx * RS + RB * ty + c] = acc[c];
  __syncthreads();
  const size_t N = (size_t)n * n;
  const float gm = D.gamma[s];
  unsigned long long best = 0;
  const int gj = j0 + tx;
  for (int r = ty; r < kTI; r += 4) {
    const int gi = i0 + r;
    if (gi < n && gj < n) {
      const float v = gm * res[r * RS + tx];
      const size_t e = (size_t)gi * n + gj;
      out[s * N + e] = v;
      const float kv = positive ? (v > 0.0f ? v : 0.0f) : fabsf(v);
      const unsigned long long kk = dict_key(kv, (uint32_t)(s * N + e));
      best = kk > best ? kk : best;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  if (tx == 0) wbest[ty] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = wbest[0];
    for (int w = 1; w < 4; ++w) mx = wbest[w] > mx ? wbest[w] : mx;
    keys[tb] = mx;
  }
}

// *key = max of count per-workgroup keys (one workgroup).
__global__ __launch_bounds__(1024) void dict_key_reduce_kernel(int64_t count,
                                                               const unsigned long long* __restrict__ keys,
                                                               unsigned long long* __restrict__ key) {
  __shared__ unsigned long long wb[16];
  unsigned long long best = 0;
  for (int64_t i = threadIdx.x; i < count; i += 1024) best = keys[i] > best ? keys[i] : best;
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wb[0];
    for (int w = 1; w < 16; ++w) m = wb[w] > m ? wb[w] : m;
    *key = m;
  }
}

using DictTileFn = void (*)(int, DictSpec, int, const float*, float*, int, unsigned long long*);
template <int H>
static DictTileFn tile_fn_upto(int h) {
  if constexpr (H < 0) {
    return nullptr;
  } else {
    return h == H ? dict_tile_h_kernel<H> : tile_fn_upto<H - 1>(h);
  }
}

static void set_lds_bytes(const void* kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    PC_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

void dict_analysis(pc_plan* p, const DictSpec& D, const float* img, float* out, bool positive,
                   unsigned long long* key, hipStream_t s) {
  const int n = p->g.n;
  const size_t N = (size_t)n * n;
  const int64_t nblk = (int64_t)((n + kTJ - 1) / kTJ) * ((n + kTI - 1) / kTI);
  const dim3 grid((unsigned)nblk);
  unsigned long long* keys = ensure_key_scratch(p, (size_t)(nblk * D.S));
  for (int sc = 0; sc < D.S; ++sc) {
    const int h = D.h[sc];
    ProfScope ps(p, s, "dict_analysis", 8.0 * N, (double)N);
    if (h <= 16) {
      hipLaunchKernelGGL(tile_fn_upto<16>(h), grid, dim3(256), 0, s, n, D, sc, img, out,
                         positive ? 1 : 0, keys + sc * nblk);
    } else {
      const size_t lds = sizeof(float) * (size_t)(kTI + 2 * h) * (kTJ + 2 * h + kTJ);
      set_lds_bytes((const void*)dict_tile_kernel, lds);
      hipLaunchKernelGGL(dict_tile_kernel, grid, dim3(256), lds, s, n, D, sc, img, out,
                         positive ? 1 : 0, keys + sc * nblk);
    }
    PC_LAUNCH_CHECK("dict_analysis");
  }
  hipLaunchKernelGGL(dict_key_reduce_kernel, dim3(1), dim3(1024), 0, s, nblk * D.S, keys, key);
  PC_LAUNCH_CHECK("dict_key_reduce");
}

void dict_synthesis(pc_plan* p, const DictSpec& D, int64_t nS, const int32_t* atoms,
                    const double* w, float* img, hipStream_t s) {
  if (nS <= 0) return;
  ProfScope ps(p, s, "dict_synth", 12.0 * nS, (double)nS);
  hipLaunchKernelGGL(dict_synth_kernel, dim3((unsigned)nS), dim3(256), 0, s, p->g.n, D, nS, atoms,
                     w, img);
  PC_LAUNCH_CHECK("dict_synth");
}

void dict_gather(pc_plan* p, const DictSpec& D, int64_t nS, const int32_t* atoms,
                 const float* img, double* out, hipStream_t s) {
  if (nS <= 0) return;
  ProfScope ps(p, s, "dict_gather", 12.0 * nS, (double)nS);
  hipLaunchKernelGGL(dict_gather_kernel, dim3((unsigned)nS), dim3(256), 0, s, p->g.n, D, nS, atoms,
                     img, out);
  PC_LAUNCH_CHECK("dict_gather");
}

}  // namespace pc
