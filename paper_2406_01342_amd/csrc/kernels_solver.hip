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

// The same sum for many partials (one per interpolation work item): 1024
// threads, each summing every 1024th pair with four pairs' loads in flight
// (pairs q, q + 1024, q + 2048, q + 3072 of each round, added in that order),
// then a tree over the threads.
__global__ __launch_bounds__(1024) void parts_final_kernel(int nparts,
                                                           const double2* __restrict__ partial,
                                                           double* __restrict__ out) {
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < nparts; i += 4 * 1024) {
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = i + u * 1024;
      v[u] = q < nparts ? partial[q] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a += v[u].x;
      b += v[u].y;
    }
  }
  __shared__ double sa[1024], sb[1024];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
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

// Appends j to out[0..cap) for every lane with pred set: one atomic per wave
// (the wave's count, taken by its lowest selecting lane), then each lane
// writes at the base plus the number of selecting lanes below it.
__device__ __forceinline__ void wave_append(bool pred, int32_t j, unsigned int* __restrict__ count,
                                            int32_t* __restrict__ out, int64_t cap) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;  // wave-uniform
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)mask) - 1;
  unsigned int base = 0u;
  if (lane == leader) base = atomicAdd(count, (unsigned int)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (pred) {
    const unsigned int q = base + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
    if ((int64_t)q < cap) out[q] = j;
  }
}

// Candidates {j : |eta_j| >= tau} (Alg. 2, step 1.a), or {j : eta_j >= tau,
// eta_j > 0} under positivity (only positive maxima); order is fixed on the
// host by sorting.
__global__ void select_kernel(int64_t N, const float* __restrict__ eta, float tau, int positive,
                              unsigned int* __restrict__ count, int32_t* __restrict__ out,
                              int64_t cap) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float e = j < N ? eta[j] : 0.0f;
  const bool pick = j < N && (positive ? (e >= tau && e > 0.0f) : fabsf(e) >= tau);
  wave_append(pick, (int32_t)j, count, out, cap);
}

// The same selection with the threshold formed on the device from the fused
// maximum key: tau = max - dec in FP64 (max decoded from the key's high 32
// bits as the host does), rounded once to FP32, so that the next
// exploration's candidates are ready with step 4's readback.
__global__ void select_from_key_kernel(int64_t N, const float* __restrict__ eta,
                                       const unsigned long long* __restrict__ key, double dec,
                                       int positive, unsigned int* __restrict__ count,
                                       int32_t* __restrict__ out, int64_t cap) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float tau = (float)((double)__uint_as_float((unsigned)(key[0] >> 32)) - dec);
  const float e = j < N ? eta[j] : 0.0f;
  const bool pick = j < N && (positive ? (e >= tau && e > 0.0f) : fabsf(e) >= tau);
  wave_append(pick, (int32_t)j, count, out, cap);
}

__global__ void zero_u32_kernel(unsigned int* p) { *p = 0u; }

__global__ void zero_n_u32_kernel(int64_t n, unsigned int* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

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

// dst[0..n) = src[0..n) from global memory into LDS by a 256-thread
// workgroup, eight loads in flight per thread (a plain copy loop waits for
// each load before its LDS store: one memory latency per element).
__device__ __forceinline__ void copy_to_lds(double* dst, const double* __restrict__ src,
                                            int64_t n) {
  int64_t i = threadIdx.x;
  for (; i + 7 * 256 < n; i += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[i + u * 256] = v[u];
  }
  for (; i < n; i += 256) dst[i] = src[i];
}

// (G v)_q for the symmetric G as column q (coalesced across threads), with
// four independent partial sums so that several loads are in flight.
__device__ __forceinline__ double gram_col_dot(const double* __restrict__ G,
                                               const double* __restrict__ v, int64_t nS,
                                               int64_t q) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t p = 0;
  for (; p + 4 <= nS; p += 4) {
    s0 += G[p * nS + q] * v[p];
    s1 += G[(p + 1) * nS + q] * v[p + 1];
    s2 += G[(p + 2) * nS + q] * v[p + 2];
    s3 += G[(p + 3) * nS + q] * v[p + 3];
  }
  for (; p < nS; ++p) s0 += G[p * nS + q] * v[p];
  return (s0 + s1) + (s2 + s3);
}

// Gram form of the restricted problem (small direct sets).  G is the exact
// nS x nS matrix Re(Phi_S^H Phi_S) (symmetric, row-major, FP64) and
// b = Phi_S^* V, so that Phi_S^*(V - Phi_S y) = b - G y.  One APGD step in one
// workgroup: g = b - G y, x+ = soft(y + g / L, lambda / L),
// y+ = x+ + mom (x+ - x), with the step constant L read from lipd[0] (written
// by the Lanczos kernel).  On `check` steps the duality-gap inputs at y are
// stored in stats too: ||V - Phi_S y||^2 = v2 - 2 y.b + y.G y,
// Re<V, V - Phi_S y> = v2 - y.b, ||y||_1 and max |g| (v2 = ||V||^2).
//
// When `check` is set, the restricted duality gap at y is tested: with
// P = ||r_y||^2 / 2 + lambda ||y||_1 and the dual point scaled into the
// feasible set, the step passes when P - D <= tol P; it is still applied, and
// done = {1, iter} is recorded.  G may be an LDS copy; ys is the LDS copy
// of y that the product reads (y itself is kept in step).  Returns with every
// thread past the step's last read of y (the caller synchronises before the
// next step).
__device__ __forceinline__ void gram_fista_step(int64_t nS, const double* __restrict__ G,
                                                const double* __restrict__ b,
                                                double* __restrict__ x, double* __restrict__ y,
                                                double* __restrict__ ys,
                                                double* __restrict__ g_out,
                                                double* __restrict__ stats, double v2,
                                                double inv_lip, double mom, int check, int iter,
                                                double lam, double tol, int positive,
                                                int* __restrict__ done, double* sh) {
  const double thr = lam * inv_lip;
  // under positivity: ||y||_1 = sum y on x >= 0, yneg = max(0, -min y) > 0
  // marks an extrapolated y outside it (objective +inf there: no test), and
  // the dual scaling uses max(g, 0)
  double yGy = 0, yb = 0, yl1 = 0, gmax = 0, yneg = 0;
  for (int64_t q = threadIdx.x; q < nS; q += 256) {
    const double s = gram_col_dot(G, ys, nS, q);  // (G y)_q
    const double gq = b[q] - s;
    const double yq = ys[q];
    g_out[q] = gq;
    yGy += yq * s;
    yb += yq * b[q];
    yl1 += positive ? yq : fabs(yq);
    yneg = fmax(yneg, -yq);
    gmax = fmax(gmax, positive ? gq : fabs(gq));
  }
  bool passed = false;
  if (check) {
    yGy = block_sum<256>(yGy, sh);
    yb = block_sum<256>(yb, sh);
    yl1 = block_sum<256>(yl1, sh);
    gmax = block_max<256>(gmax, sh);
    yneg = block_max<256>(yneg, sh);
    const double r2 = v2 - 2.0 * yb + yGy, vr = v2 - yb;
    const double py = 0.5 * r2 + lam * yl1;
    const double sc = gmax <= lam ? 1.0 : lam / gmax;
    const double gy = py - (sc * vr - 0.5 * sc * sc * r2);
    passed = gy <= tol * py && !(positive && yneg > 0.0);
    if (threadIdx.x == 0) {
      stats[0] = r2;
      stats[1] = vr;
      stats[2] = yl1;
      stats[3] = gmax;
    }
  }
  __syncthreads();  // every thread has read all of y
  for (int64_t q = threadIdx.x; q < nS; q += 256) {
    const double yo = ys[q], xo = x[q];
    const double z = yo + g_out[q] * inv_lip;
    double xn;
    if (positive) {
      xn = z - thr > 0 ? z - thr : 0.0;
    } else {
      const double az = fabs(z) - thr;
      xn = az > 0 ? copysign(az, z) : 0.0;
    }
    const double yn = xn + mom * (xn - xo);
    x[q] = xn;
    y[q] = yn;
    ys[q] = yn;
  }
  if (passed && threadIdx.x == 0) {
    done[1] = iter;
    done[0] = 1;
  }
}

// APGD steps it0 + 1 .. it0 + nsteps of the Gram form in one workgroup, the
// momentum sequence t+ = (1 + sqrt(1 + 4 t^2)) / 2, mom = (t - 1) / t+ carried
// on the device from t0 (the same FP64 recurrence the host advances), the
// gap test on every kcheck-th step.  Steps after a passing test (done[0] set,
// here or by an earlier launch) are skipped.  y is mirrored in LDS for the
// products, and so is G when g_in_lds is set (loaded once for all steps of
// the launch): dynamic LDS of nS (+ nS^2) doubles.
__global__ __launch_bounds__(256) void gram_fista_loop_kernel(
    int64_t nS, const double* __restrict__ G, const double* __restrict__ b,
    double* __restrict__ x, double* __restrict__ y, double* __restrict__ g_out,
    double* __restrict__ stats, double v2, const double* __restrict__ lipd, double t0, int it0,
    int nsteps, int kcheck, double lam, double tol, int positive, int* __restrict__ done,
    int g_in_lds) {
  __shared__ double sh[4];
  extern __shared__ double dyn[];
  double* ys = dyn;
  double* Gl = dyn + nS;
  copy_to_lds(ys, y, nS);
  if (g_in_lds) copy_to_lds(Gl, G, nS * nS);
  __syncthreads();
  const double* Gm = g_in_lds ? Gl : G;
  const double inv_lip = 1.0 / lipd[0];  // step constant from the device
  double t = t0;
  for (int c = 0; c < nsteps; ++c) {
    if (done[0]) return;  // uniform: written before the last barrier
    const int it = it0 + c + 1;
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
    const double mom = (t - 1.0) / tn;
    t = tn;
    gram_fista_step(nS, Gm, b, x, y, ys, g_out, stats, v2, inv_lip, mom, (it - 1) % kcheck == 0,
                    it, lam, tol, positive, done, sh);
    __syncthreads();  // x, y and done written before the next step reads them
  }
}

// Sums of cnt <= kLanczosMax + 1 values over the 256 threads of a workgroup
// (every thread receives the totals); sh holds 4 x (kLanczosMax + 1) doubles.
constexpr int kLzMaxRows = 13;  // the Lanczos basis has at most 12 + 1 rows

__device__ __forceinline__ void block_sum_multi(double* v, int cnt, double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kLzMaxRows; ++q)
    if (q < cnt) {
      double t = v[q];
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      if (lane == 0) sh[wv * kLzMaxRows + q] = t;
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kLzMaxRows; ++q)
    if (q < cnt)
      v[q] = ((sh[q] + sh[kLzMaxRows + q]) + sh[2 * kLzMaxRows + q]) + sh[3 * kLzMaxRows + q];
  __syncthreads();
}

// The part of a Lanczos step after the product: w holds g = G q_j on entry.
// alpha_j = q_j . g, w = g - alpha_j q_j - beta_{j-1} q_{j-1}, then w is
// orthogonalised against q_0..q_j by classical Gram-Schmidt applied twice
// (all projections of a pass reduced together), beta_j = ||w||,
// q_{j+1} = w / beta_j (zero when beta_j = 0); ab[j] = alpha_j,
// ab[kmax + j] = beta_j.  Every thread works on the same indices throughout.
__device__ void lanczos_finish_step(int64_t nS, int j, int kmax, double* __restrict__ Q,
                                    double* __restrict__ w, double* __restrict__ ab,
                                    double* sh) {
  const double* qj = Q + (int64_t)j * nS;
  double v[kLzMaxRows];
  v[0] = 0;
  for (int64_t i = threadIdx.x; i < nS; i += 256) v[0] += qj[i] * w[i];
  block_sum_multi(v, 1, sh);
  const double a = v[0];
  const double bp = j > 0 ? ab[kmax + j - 1] : 0.0;
  const double* qp = j > 0 ? Q + (int64_t)(j - 1) * nS : qj;
  for (int64_t i = threadIdx.x; i < nS; i += 256) w[i] -= a * qj[i] + bp * qp[i];
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int q = 0; q < kLzMaxRows; ++q) v[q] = 0;
    for (int64_t i = threadIdx.x; i < nS; i += 256) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < kLzMaxRows; ++q)
        if (q <= j) v[q] += Q[(int64_t)q * nS + i] * wi;
    }
    block_sum_multi(v, j + 1, sh);
    for (int64_t i = threadIdx.x; i < nS; i += 256) {
      double wi = w[i];
#pragma unroll
      for (int q = 0; q < kLzMaxRows; ++q)
        if (q <= j) wi -= v[q] * Q[(int64_t)q * nS + i];
      w[i] = wi;
    }
  }
  v[0] = 0;
  for (int64_t i = threadIdx.x; i < nS; i += 256) v[0] += w[i] * w[i];
  block_sum_multi(v, 1, sh);
  const double b = sqrt(v[0]);
  if (threadIdx.x == 0) {
    ab[j] = a;
    ab[kmax + j] = b;
  }
  const double inv = b > 0 ? 1.0 / b : 0.0;
  double* qn = Q + (int64_t)(j + 1) * nS;
  for (int64_t i = threadIdx.x; i < nS; i += 256) qn[i] = w[i] * inv;
}

// One Lanczos step on G = Re(Phi_S^H Phi_S) given g = G q_j (the operator
// pair applied by other kernels); Q holds kmax + 1 rows of nS, w is scratch.
__global__ __launch_bounds__(256) void lanczos_step_kernel(int64_t nS, int j, int kmax,
                                                           double* __restrict__ Q,
                                                           const double* __restrict__ g,
                                                           double* __restrict__ w,
                                                           double* __restrict__ ab) {
  __shared__ double sh[4 * kLzMaxRows];
  for (int64_t i = threadIdx.x; i < nS; i += 256) w[i] = g[i];
  lanczos_finish_step(nS, j, kmax, Q, w, ab, sh);
}

// Top eigenpair of the k x k symmetric tridiagonal T (diagonal al[0..k),
// off-diagonal be[0..k-1)), by one wave: Sturm-sequence multisection (each
// of the 64 lanes counts the eigenvalues below its own point of the current
// bracket; kSturmRounds = 6 rounds shrink the Gershgorin bracket by
// 65^6 ~ 7.5e10, far below the 1e-3 residual test and the 1% margin of the
// step constant), then the eigenvector from the three-term recurrence
// (x_0 = 1), normalised.  Every
// lane returns theta and writes nothing; lane 0 stores s[0..k).
__device__ double tridiag_top(const double* al, const double* be, int k, double* s) {
  const int lane = threadIdx.x & 63;
  double lo = al[0], hi = al[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  hi += 1e-300 + 1e-15 * fabs(hi);  // every eigenvalue strictly below hi
  constexpr int kSturmRounds = 6;
  for (int round = 0; round < kSturmRounds; ++round) {
    const double xl = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    int below = 0;  // eigenvalues < xl (signs of the LDL^T pivots of T - xl)
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double off = i > 0 ? be[i - 1] * be[i - 1] / d : 0.0;
      d = al[i] - xl - off;
      if (d == 0.0) d = -1e-300;
      below += d < 0.0;
    }
    // the top eigenvalue lies between the last point with fewer than k
    // eigenvalues below it and the first point with all k below it
    const unsigned long long all_k = __ballot(below >= k);
    const int first = all_k ? __ffsll((long long)all_k) - 1 : 64;
    const double nhi = first < 64 ? __shfl(xl, first, 64) : hi;
    const double nlo = first > 0 ? __shfl(xl, first - 1, 64) : lo;
    lo = nlo;
    hi = nhi;
  }
  const double theta = 0.5 * (lo + hi);
  if (lane == 0) {
    double xm = 0.0, xc = 1.0, nrm = 1.0;
    s[0] = 1.0;
    for (int i = 0; i + 1 < k; ++i) {
      const double xn = ((theta - al[i]) * xc - (i > 0 ? be[i - 1] * xm : 0.0)) / be[i];
      s[i + 1] = xn;
      nrm += xn * xn;
      xm = xc;
      xc = xn;
    }
    nrm = sqrt(nrm);
    for (int i = 0; i < k; ++i) s[i] /= nrm;
  }
  return theta;
}

// The whole Lanczos estimate of the Gram form in one workgroup and without a
// host round trip: steps j = 0.. (Q row 0 holds the unit start vector), and
// after each one the test of the host version: theta = top eigenvalue of
// T_{j+1}, rho = beta_j |s_j|; stop when rho <= tol theta, on an invariant
// subspace (beta_j <= 1e-14 theta, or j + 1 = nS) or at kmax steps.  Writes
// out[0] = (theta + rho) * margin (the APGD step constant), out[1] = steps,
// out[2] = theta, out[3] = rho, and ritz = sum_q s_q q_q (the next start).
//
// The basis rows and w live in dynamic LDS ((kmax + 1) nS + nS doubles), and
// so does G when g_in_lds is set (nS^2 more); Q row 0 is read from Qg.
__global__ __launch_bounds__(256) void gram_lanczos_full_kernel(
    int64_t nS, int kmax, double tol, double margin, const double* __restrict__ Gg,
    const double* __restrict__ Qg, int g_in_lds, double* __restrict__ ab,
    double* __restrict__ out, double* __restrict__ ritz) {
  __shared__ double sh[4 * kLzMaxRows];
  __shared__ double svec[kLzMaxRows];
  __shared__ double res[3];  // theta, rho, stop flag
  extern __shared__ double dyn[];
  double* Q = dyn;
  double* w = Q + (int64_t)(kmax + 1) * nS;
  double* Gl = w + nS;
  copy_to_lds(Q, Qg, nS);
  if (g_in_lds) copy_to_lds(Gl, Gg, nS * nS);
  __syncthreads();
  const double* G = g_in_lds ? Gl : Gg;
  const int jmax = (int)(nS < kmax ? nS : kmax);
  int k = 0;
  for (int j = 0; j < jmax; ++j) {
    const double* qj = Q + (int64_t)j * nS;
    for (int64_t i = threadIdx.x; i < nS; i += 256) w[i] = gram_col_dot(G, qj, nS, i);
    lanczos_finish_step(nS, j, kmax, Q, w, ab, sh);
    __syncthreads();  // ab[j], beta_j and q_{j+1} visible to all
    if (threadIdx.x < 64) {
      const double theta = tridiag_top(ab, ab + kmax, j + 1, svec);
      if (threadIdx.x == 0) {
        const double bj = ab[kmax + j];
        const double rho = bj * fabs(svec[j]);
        const bool invariant = bj <= 1e-14 * fmax(theta, 1e-300) || j + 1 >= nS;
        res[0] = theta;
        res[1] = rho;
        res[2] = (invariant || rho <= tol * theta || j + 1 == kmax) ? 1.0 : 0.0;
      }
    }
    __syncthreads();
    k = j + 1;
    if (res[2] != 0.0) break;
  }
  if (threadIdx.x == 0) {
    out[0] = (res[0] + res[1]) * margin;
    out[1] = (double)k;
    out[2] = res[0];
    out[3] = res[1];
  }
  for (int64_t i = threadIdx.x; i < nS; i += 256) {
    double v = 0;
    for (int q = 0; q < k; ++q) v += svec[q] * Q[(int64_t)q * nS + i];
    ritz[i] = v;
  }
}

// G, b and the Lanczos start vector of the Gram form from one uploaded block
// [v0: nS doubles][inv_n: nS doubles][bslot: nS int32][pslot: nS^2 int32]:
// G[a][c] = psf[pslot[a][c]] inv_n[a] inv_n[c], b[a] = bval[bslot[a]],
// Q0 = v0 (psf and bval hold the solve's point-spread sums and b_p by slot).
__global__ void gram_assemble_kernel(int64_t nS, const unsigned char* __restrict__ blk,
                                     const double* __restrict__ psf,
                                     const double* __restrict__ bval, double* __restrict__ G,
                                     double* __restrict__ b, double* __restrict__ Q0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double* v0 = reinterpret_cast<const double*>(blk);
  const double* inv_n = v0 + nS;
  const int32_t* bslot = reinterpret_cast<const int32_t*>(blk + 16 * nS);
  const int32_t* pslot = bslot + nS;
  if (e < nS * nS) {
    const int64_t a = e / nS, c = e - (e / nS) * nS;
    G[e] = psf[pslot[e]] * inv_n[a] * inv_n[c];
  }
  if (e < nS) {
    b[e] = bval[bslot[e]];
    Q0[e] = v0[e];
  }
}

// Sum over the 64 lanes of a wave (every lane gets the same value: each
// butterfly level adds a commutative pair).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same estimate as gram_lanczos_full_kernel for nS <= kLzWaveAtoms: the
// four waves copy G and the start vector into LDS, then wave 0 alone runs the
// steps, each lane owning rows lane and lane + 64, with every reduction a
// wave butterfly (no workgroup barrier inside a step).  Same recurrence, test
// and outputs; alpha and beta are kept in LDS for the tridiagonal solve and
// copied to ab at the end.
constexpr int kLzWaveAtoms = 128;
__global__ __launch_bounds__(256) void gram_lanczos_wave_kernel(
    int64_t nS, int kmax, double tol, double margin, const double* __restrict__ Gg,
    const double* __restrict__ Qg, double* __restrict__ ab, double* __restrict__ out,
    double* __restrict__ ritz) {
  __shared__ double svec[kLzMaxRows];
  __shared__ double al[kLzMaxRows], be[kLzMaxRows];
  extern __shared__ double dyn[];
  double* Q = dyn;                            // (kmax + 1) rows of nS
  double* G = Q + (int64_t)(kmax + 1) * nS;   // nS x nS
  copy_to_lds(Q, Qg, nS);
  copy_to_lds(G, Gg, nS * nS);
  __syncthreads();
  if (threadIdx.x >= 64) return;  // wave 0 runs the steps
  const int lane = threadIdx.x;
  const int i0 = lane, i1 = lane + 64;
  const bool r0 = i0 < nS, r1 = i1 < nS;
  const int jmax = (int)(nS < kmax ? nS : kmax);
  int k = 0;
  double theta = 0, rho = 0;
  for (int j = 0; j < jmax; ++j) {
    const double* qj = Q + (int64_t)j * nS;
    double w0 = r0 ? gram_col_dot(G, qj, nS, i0) : 0.0;
    double w1 = r1 ? gram_col_dot(G, qj, nS, i1) : 0.0;
    const double q0 = r0 ? qj[i0] : 0.0, q1 = r1 ? qj[i1] : 0.0;
    const double a = wave_sum(q0 * w0 + q1 * w1);
    const double bp = j > 0 ? be[j - 1] : 0.0;
    const double* qp = j > 0 ? Q + (int64_t)(j - 1) * nS : qj;
    w0 -= a * q0 + bp * (r0 ? qp[i0] : 0.0);
    w1 -= a * q1 + bp * (r1 ? qp[i1] : 0.0);
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      double h[kLzMaxRows];
#pragma unroll
      for (int q = 0; q < kLzMaxRows; ++q)
        if (q <= j) {
          const double* Qq = Q + (int64_t)q * nS;
          h[q] = wave_sum((r0 ? Qq[i0] * w0 : 0.0) + (r1 ? Qq[i1] * w1 : 0.0));
        }
#pragma unroll
      for (int q = 0; q < kLzMaxRows; ++q)
        if (q <= j) {
          const double* Qq = Q + (int64_t)q * nS;
          if (r0) w0 -= h[q] * Qq[i0];
          if (r1) w1 -= h[q] * Qq[i1];
        }
    }
    const double b = sqrt(wave_sum(w0 * w0 + w1 * w1));
    const double inv = b > 0 ? 1.0 / b : 0.0;
    double* qn = Q + (int64_t)(j + 1) * nS;
    if (r0) qn[i0] = w0 * inv;
    if (r1) qn[i1] = w1 * inv;
    if (lane == 0) {
      al[j] = a;
      be[j] = b;
    }
    lds_wave_sync();  // q_{j+1}, al, be visible to the wave
    theta = tridiag_top(al, be, j + 1, svec);
    lds_wave_sync();  // svec written by lane 0
    const double bj = be[j];
    rho = bj * fabs(svec[j]);
    const bool invariant = bj <= 1e-14 * fmax(theta, 1e-300) || j + 1 >= nS;
    k = j + 1;
    if (invariant || rho <= tol * theta || j + 1 == kmax) break;
  }
  if (lane == 0) {
    out[0] = (theta + rho) * margin;
    out[1] = (double)k;
    out[2] = theta;
    out[3] = rho;
  }
  for (int q = lane; q < k; q += 64) {
    ab[q] = al[q];
    ab[kmax + q] = be[q];
  }
  for (int64_t i = lane; i < nS; i += 64) {
    double v = 0;
    for (int q = 0; q < k; ++q) v += svec[q] * Q[(int64_t)q * nS + i];
    ritz[i] = v;
  }
}

// An active set from one uploaded block [x: nS doubles][pix: nS int32]:
// x = y = the weights, pix, and the atom table (pixel offsets, 1/n, n - 1,
// forward weight x/n; zero-weight phase-centre padding up to ntotal entries).
__global__ void activate_kernel(int64_t nS, int64_t ntotal, int n, double dl,
                                const unsigned char* __restrict__ blk, double* __restrict__ x,
                                double* __restrict__ y, int32_t* __restrict__ pix,
                                Atom<float>* __restrict__ atoms) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ntotal) return;
  if (p >= nS) {
    atoms[p] = Atom<float>{0.0, 0.0, 1.0, 0.0, 0.f, 0.f};
    return;
  }
  const double xv = reinterpret_cast<const double*>(blk)[p];
  const int q = reinterpret_cast<const int32_t*>(blk + 8 * nS)[p];
  x[p] = xv;
  y[p] = xv;
  pix[p] = q;
  const int qp = q % (n * n);  // the centre pixel of a synthesis-dictionary atom
  const int i = qp / n, j = qp - i * n;
  const double a = (double)(i - n / 2), b = (double)(j - n / 2);
  const double l = a * dl, m = b * dl;
  const double inv_n = 1.0 / sqrt(1.0 - l * l - m * m);
  atoms[p] = Atom<float>{a, b, inv_n, n_minus_one(l, m), (float)(xv * inv_n), 0.f};
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
// scal[kScalYL1] = sum_p stat[p], scal[kScalGmax] = max(0, max_p stat[nS + p]),
// scal[kScalYNeg] = max(0, -min_p stat[p]) (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void stat_reduce_kernel(int64_t nS, const double* __restrict__ stat,
                                                           double* __restrict__ scal) {
  __shared__ double sh[16];
  double l1 = 0, mx = 0, neg = 0;
  for (int64_t p = threadIdx.x; p < nS; p += blockDim.x) {
    l1 += stat[p];
    neg = fmax(neg, -stat[p]);
    mx = fmax(mx, stat[nS + p]);
  }
  l1 = block_sum<1024>(l1, sh);
  mx = block_max<1024>(mx, sh);
  neg = block_max<1024>(neg, sh);
  if (threadIdx.x == 0) {
    scal[kScalYL1] = l1;
    scal[kScalGmax] = mx;
    scal[kScalYNeg] = neg;
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

void k_resid_final(pc_plan* p, int nparts, const double* partial, double* out, hipStream_t s) {
  ProfScope ps(p, s, "resid_final", 16.0 * nparts, (double)nparts);
  hipLaunchKernelGGL(parts_final_kernel, dim3(1), dim3(1024), 0, s, nparts,
                     (const double2*)partial, out);
  PC_LAUNCH_CHECK("resid_final");
}

void k_select_from_key(pc_plan* p, int64_t N, const float* eta, const unsigned long long* key,
                       double dec, bool positive, unsigned* count, int32_t* out, int64_t cap,
                       hipStream_t s) {
  ProfScope ps(p, s, "select", 4.0 * N, (double)N);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL(select_from_key_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, N, eta, key,
                     dec, positive ? 1 : 0, count, out, cap);
  PC_LAUNCH_CHECK("select_from_key");
}

void k_select(pc_plan* p, int64_t N, const float* eta, float tau, bool positive, unsigned* count,
              int32_t* out, int64_t cap, hipStream_t s) {
  ProfScope ps(p, s, "select", 4.0 * N, (double)N);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL(select_kernel, dim3(blocks(N, 256)), dim3(256), 0, s, N, eta, tau,
                     positive ? 1 : 0, count, out, cap);
  PC_LAUNCH_CHECK("select");
}

void k_lanczos_step(pc_plan* p, int64_t nS, int j, int kmax, double* Q, const double* g, double* w,
                    double* ab, hipStream_t s) {
  ProfScope ps(p, s, "lanczos_step", 8.0 * nS * (2.0 * (j + 1) * 2 + 5), (double)nS);
  hipLaunchKernelGGL(lanczos_step_kernel, dim3(1), dim3(256), 0, s, nS, j, kmax, Q, g, w, ab);
  PC_LAUNCH_CHECK("lanczos_step");
}

void k_gram_fista(pc_plan* p, int64_t nS, const double* G, const double* b, double* x, double* y,
                  double* g, double* stats, double v2, const double* lipd, double t0, int it0,
                  int nsteps, int kcheck, double lam, double tol, bool positive, int* done,
                  hipStream_t s) {
  if (nsteps <= 0) return;
  constexpr size_t kLdsMax = 150 * 1024;
  const bool g_in_lds = (size_t)(nS + nS * nS) * 8 <= kLdsMax;
  const size_t lds = (size_t)(nS + (g_in_lds ? nS * nS : 0)) * 8;
  PC_REQUIRE(lds <= kLdsMax, "gram_fista: active set too large for the Gram form");
  PC_HIP(hipFuncSetAttribute((const void*)gram_fista_loop_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax));
  ProfScope ps(p, s, "gram_fista", 8.0 * nS * (nS + 6) * nsteps, (double)nS * nS * nsteps);
  hipLaunchKernelGGL(gram_fista_loop_kernel, dim3(1), dim3(256), lds, s, nS, G, b, x, y, g, stats,
                     v2, lipd, t0, it0, nsteps, kcheck, lam, tol, positive ? 1 : 0, done,
                     g_in_lds ? 1 : 0);
  PC_LAUNCH_CHECK("gram_fista");
}

void k_gram_lanczos_full(pc_plan* p, int64_t nS, int kmax, double tol, double margin,
                         const double* G, const double* Q, double* ab, double* out, double* ritz,
                         hipStream_t s) {
  constexpr size_t kLdsMax = 150 * 1024;
  if (nS <= kLzWaveAtoms && kmax < kLzMaxRows) {  // one wave, basis and G in LDS
    const size_t lds = (size_t)((kmax + 1) * nS + nS * nS) * 8;
    PC_HIP(hipFuncSetAttribute((const void*)gram_lanczos_wave_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax));
    ProfScope ps(p, s, "gram_lanczos", 8.0 * nS * (double)(nS + 30) * 4, (double)nS);
    hipLaunchKernelGGL(gram_lanczos_wave_kernel, dim3(1), dim3(256), lds, s, nS, kmax, tol,
                       margin, G, Q, ab, out, ritz);
    PC_LAUNCH_CHECK("gram_lanczos_wave");
    return;
  }
  // basis rows and w always in LDS; G too when it fits beside them
  const size_t base = (size_t)((kmax + 2) * nS) * 8;
  const bool g_in_lds = base + (size_t)nS * nS * 8 <= kLdsMax;
  const size_t lds = base + (g_in_lds ? (size_t)nS * nS * 8 : 0);
  if (lds > kLdsMax)
    fail(PC_ERR_UNSUPPORTED, "gram_lanczos: active set of " + std::to_string(nS) + " atoms");
  PC_HIP(hipFuncSetAttribute((const void*)gram_lanczos_full_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax));
  ProfScope ps(p, s, "gram_lanczos", 8.0 * nS * (double)(nS + 30) * 4, (double)nS);
  hipLaunchKernelGGL(gram_lanczos_full_kernel, dim3(1), dim3(256), lds, s, nS, kmax, tol, margin,
                     G, Q, g_in_lds ? 1 : 0, ab, out, ritz);
  PC_LAUNCH_CHECK("gram_lanczos_full");
}

void k_gram_assemble(pc_plan* p, int64_t nS, const void* blk, const double* psf,
                     const double* bval, double* G, double* b, double* Q0, hipStream_t s) {
  if (nS <= 0) return;
  hipLaunchKernelGGL(gram_assemble_kernel, dim3(blocks(nS * nS, 256)), dim3(256), 0, s, nS,
                     (const unsigned char*)blk, psf, bval, G, b, Q0);
  PC_LAUNCH_CHECK("gram_assemble");
}

void k_activate(pc_plan* p, int64_t nS, const void* blk, double* x, double* y, int32_t* pix,
                Atom<float>* atoms, hipStream_t s) {
  const int64_t ntotal = atom_capacity(nS);
  hipLaunchKernelGGL(activate_kernel, dim3(blocks(ntotal, 256)), dim3(256), 0, s, nS, ntotal,
                     p->g.n, p->g.dl, (const unsigned char*)blk, x, y, pix, atoms);
  PC_LAUNCH_CHECK("activate");
}

void k_zero_u32(pc_plan* p, int64_t n, unsigned* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_n_u32_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, n, out);
  PC_LAUNCH_CHECK("zero_u32");
}

void k_weights(pc_plan* p, int64_t nS, const double* x, Atom<float>* atoms, hipStream_t s) {
  if (nS <= 0) return;
  hipLaunchKernelGGL(weights_kernel, dim3(blocks(nS, 256)), dim3(256), 0, s, nS, x, atoms);
  PC_LAUNCH_CHECK("weights");
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
