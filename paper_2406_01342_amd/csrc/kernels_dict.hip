// Synthesis dictionary of Gaussian elements (Sect. 3.2, Eqs. params-synthesis
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

// Row pass (one workgroup per image row i, the row staged in LDS):
// tmp[s][i][j] = sum_b t_s[b] img[i][j + b].  Clears the key for the column
// pass that follows on the same stream.
__global__ __launch_bounds__(256) void dict_rows_kernel(int n, DictSpec D,
                                                        const float* __restrict__ img,
                                                        float* __restrict__ tmp,
                                                        unsigned long long* __restrict__ key) {
  extern __shared__ float row[];
  __shared__ float tl[kDictMaxTaps];
  const int i = blockIdx.x;
  if (i == 0 && threadIdx.x == 0) *key = 0ull;
  for (int j = threadIdx.x; j < n; j += 256) row[j] = img[(size_t)i * n + j];
  const size_t N = (size_t)n * n;
  for (int s = 0; s < D.S; ++s) {
    __syncthreads();  // row loaded; previous scale's taps no longer read
    load_taps(D, s, tl);
    const int h = D.h[s];
    for (int j = threadIdx.x; j < n; j += 256) {
      const int b0 = max(-h, -j), b1 = min(h, n - 1 - j);
      float acc = 0.0f;
      for (int b = b0; b <= b1; ++b) acc += tl[b + h] * row[j + b];
      tmp[s * N + (size_t)i * n + j] = acc;
    }
  }
}

__device__ __forceinline__ unsigned long long dict_key(float a, uint32_t idx) {
  return ((unsigned long long)__float_as_uint(a) << 32) | (unsigned long long)(0xffffffffu - idx);
}

// Column pass (grid: x over n^2 / 256 pixel blocks, y = scale):
// out[s][i][j] = gamma_s sum_a t_s[a] tmp[s][i + a][j], loads coalesced along
// j; fused max key.
__global__ __launch_bounds__(256) void dict_cols_kernel(int n, DictSpec D,
                                                        const float* __restrict__ tmp,
                                                        float* __restrict__ out, int positive,
                                                        unsigned long long* __restrict__ key) {
  __shared__ float tl[kDictMaxTaps];
  __shared__ unsigned long long wbest[4];
  const int s = blockIdx.y;
  load_taps(D, s, tl);
  const size_t N = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long best = 0;
  if (e < N) {
    const int i = (int)(e / n), j = (int)(e - (size_t)i * n);
    const int h = D.h[s];
    const int a0 = max(-h, -i), a1 = min(h, n - 1 - i);
    const float* col = tmp + s * N + j;
    float acc = 0.0f;
    for (int a = a0; a <= a1; ++a) acc += tl[a + h] * col[(size_t)(i + a) * n];
    const float v = D.gamma[s] * acc;
    out[s * N + e] = v;
    const float kv = positive ? (v > 0.0f ? v : 0.0f) : fabsf(v);
    best = dict_key(kv, (uint32_t)(s * N + e));
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wbest[0];
    for (int w = 1; w < 4; ++w) m = wbest[w] > m ? wbest[w] : m;
    atomicMax(key, m);
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

void dict_analysis(pc_plan* p, const DictSpec& D, const float* img, float* out, bool positive,
                   unsigned long long* key, hipStream_t s) {
  const int n = p->g.n;
  const size_t N = (size_t)n * n;
  float* tmp = ensure_dict_scratch(p, (size_t)D.S * N);
  {
    ProfScope ps(p, s, "dict_rows", 4.0 * N * (1 + D.S), (double)N * D.S);
    hipLaunchKernelGGL(dict_rows_kernel, dim3(n), dim3(256), n * sizeof(float), s, n, D, img, tmp,
                       key);
    PC_LAUNCH_CHECK("dict_rows");
  }
  ProfScope ps(p, s, "dict_cols", 8.0 * N * D.S, (double)N * D.S);
  hipLaunchKernelGGL(dict_cols_kernel, dim3((unsigned)((N + 255) / 256), D.S), dim3(256), 0, s, n,
                     D, tmp, out, positive ? 1 : 0, key);
  PC_LAUNCH_CHECK("dict_cols");
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
