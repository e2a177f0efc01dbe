// Small kernels of the Polyatomic Frank-Wolfe solve (Alg. 2): visibility
// permutation, FP64 residual reductions for the objective and duality gap,
// candidate selection for the polyatomic exploration, and the single-workgroup
// FP64 vector updates of the APGD (FISTA) restricted solve and of the power
// iteration that estimates its step size.
#include <algorithm>

#include "common.h"
#include "solver_kernels.h"

namespace pc {

__global__ void gather_kernel(int64_t L, const int32_t* __restrict__ perm,
                              const c32* __restrict__ in, c32* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < L) out[s] = in[perm[s]];
}

// Block partials of (sum |r|^2, sum Re(conj(V) r)) in FP64.
__global__ __launch_bounds__(256) void resid_partial_kernel(int64_t L, const c32* __restrict__ r,
                                                            const c32* __restrict__ V,
                                                            double* __restrict__ partial) {
  double a = 0, b = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < L;
       k += (int64_t)gridDim.x * blockDim.x) {
    const c32 x = r[k], v = V[k];
    a += (double)x.x * x.x + (double)x.y * x.y;
    b += (double)v.x * x.x + (double)v.y * x.y;
  }
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa[0];
    partial[2 * blockIdx.x + 1] = sb[0];
  }
}

// Sum of the block partials by one workgroup in a fixed order.
__global__ __launch_bounds__(256) void resid_final_kernel(int nblocks,
                                                          const double* __restrict__ partial,
                                                          double* __restrict__ out) {
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

// Candidates {j : |eta_j| >= tau} (Alg. 2, step 1.a); order is fixed on the
// host by sorting.
__global__ void select_kernel(int64_t N, const float* __restrict__ eta, float tau,
                              unsigned int* __restrict__ count, int32_t* __restrict__ out,
                              int64_t cap) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  if (fabsf(eta[j]) >= tau) {
    const unsigned int q = atomicAdd(count, 1u);
    if ((int64_t)q < cap) out[q] = (int32_t)j;
  }
}

__global__ void zero_u32_kernel(unsigned int* p) { *p = 0u; }

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < NT / 64; ++w) t = fmax(t, sh[w]);
  __syncthreads();
  return t;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < NT / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Forward weights from an FP64 vector: atoms[p].w = x[p] / n_p.
__global__ void weights_kernel(int64_t nS, const double* __restrict__ x,
                               Atom<float>* __restrict__ atoms) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nS) atoms[p].w = (float)(x[p] * atoms[p].inv_n);
}

__global__ void scale_kernel(int64_t N, const float* __restrict__ in, float s,
                             float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) out[j] = in[j] * s;
}

// img[pix[a]] = vals[a] (vals NULL: 0), for the gridded operators on an
// active set.
__global__ void scatter_kernel(int64_t nS, const int32_t* __restrict__ pix,
                               const double* __restrict__ vals, float* __restrict__ img) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a < nS) img[pix[a]] = vals ? (float)vals[a] : 0.0f;
}

__global__ void gather_img_kernel(int64_t nS, const int32_t* __restrict__ pix,
                                  const float* __restrict__ img, double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a < nS) out[a] = (double)img[pix[a]];
}

// scal[kScalYL1] = sum_p stat[p], scal[kScalGmax] = max_p stat[nS + p]
// (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void stat_reduce_kernel(int64_t nS, const double* __restrict__ stat,
                                                           double* __restrict__ scal) {
  __shared__ double sh[16];
  double l1 = 0, mx = 0;
  for (int64_t p = threadIdx.x; p < nS; p += blockDim.x) {
    l1 += stat[p];
    mx = fmax(mx, stat[nS + p]);
  }
  l1 = block_sum<1024>(l1, sh);
  mx = block_max<1024>(mx, sh);
  if (threadIdx.x == 0) {
    scal[kScalYL1] = l1;
    scal[kScalGmax] = mx;
  }
}

__global__ void fill_kernel(int64_t N, float v, float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) out[j] = v;
}

// r = V - r (both in plan order)
__global__ void rsub_kernel(int64_t L, const cpx<float>* __restrict__ V, cpx<float>* __restrict__ r) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L) {
    const cpx<float> v = V[k], m = r[k];
    r[k] = {v.x - m.x, v.y - m.y};
  }
}

// ----------------------------------------------------------------------------
static unsigned blocks(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

void k_gather(pc_plan* p, int64_t L, const int32_t* perm, const c32* in, c32* out, hipStream_t s) {
  ProfScope ps(p, s, "gather", 20.0 * L, (double)L);
  hipLaunchKernelGGL(gather_kernel, dim3(blocks(L, 256)), dim3(256), 0, s, L, perm, in, out);
  PC_LAUNCH_CHECK("gather");
}

int k_resid_blocks(int64_t L) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (L + 255) / 256)); }

void k_resid(pc_plan* p, int64_t L, const c32* r, const c32* V, double* partial, double* out, hipStream_t s) {
  ProfScope ps(p, s, "resid_reduce", 16.0 * L, (double)L);
  const int nb = k_resid_blocks(L);
  hipLaunchKernelGGL(resid_partial_kernel, dim3(nb), dim3(256), 0, s, L, r, V, partial);
  PC_LAUNCH_CHECK("resid_partial");
  hipLaunchKernelGGL(resid_final_kernel, dim3(1), dim3(256), 0, s, nb, partial, out);
  PC_LAUNCH_CHECK("resid_final");
}

void k_select(pc_plan* p, int64_t N, const float* eta, float tau, unsigned* count, int32_t* out, int64_t cap,
              hipStream_t s) {
  ProfScope ps(p, s, "select", 4.0 * N, (double)N);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL(select_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, N, eta, tau, count, out,
                     cap);
  PC_LAUNCH_CHECK("select");
}

void k_weights(pc_plan* p, int64_t nS, const double* x, Atom<float>* atoms, hipStream_t s) {
  if (nS <= 0) return;
  hipLaunchKernelGGL(weights_kernel, dim3(blocks(nS, 256)), dim3(256), 0, s, nS, x, atoms);
  PC_LAUNCH_CHECK("weights");
}

void k_scatter(pc_plan* p, int64_t nS, const int32_t* pix, const double* vals, float* img,
               hipStream_t s) {
  if (nS <= 0) return;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks(nS, 256)), dim3(256), 0, s, nS, pix, vals, img);
  PC_LAUNCH_CHECK("scatter");
}

void k_gather_img(pc_plan* p, int64_t nS, const int32_t* pix, const float* img, double* out,
                  hipStream_t s) {
  if (nS <= 0) return;
  hipLaunchKernelGGL(gather_img_kernel, dim3(blocks(nS, 256)), dim3(256), 0, s, nS, pix, img, out);
  PC_LAUNCH_CHECK("gather_img");
}

void k_stat_reduce(pc_plan* p, int64_t nS, const double* stat, double* scal, hipStream_t s) {
  ProfScope ps(p, s, "stat_reduce", 16.0 * nS, (double)nS);
  hipLaunchKernelGGL(stat_reduce_kernel, dim3(1), dim3(1024), 0, s, nS, stat, scal);
  PC_LAUNCH_CHECK("stat_reduce");
}

void k_fill(pc_plan* p, int64_t N, float v, float* out, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, N, v, out);
  PC_LAUNCH_CHECK("fill");
}

void k_rsub(pc_plan* p, int64_t L, const c32* V, c32* r, hipStream_t s) {
  hipLaunchKernelGGL(rsub_kernel, dim3(blocks(L, 256)), dim3(256), 0, s, L, V, r);
  PC_LAUNCH_CHECK("rsub");
}

void k_scale(pc_plan* p, int64_t N, const float* in, float sc, float* out, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, N, in, sc, out);
  PC_LAUNCH_CHECK("scale");
}

}  // namespace pc
