// Direct sparse DFT: the forward operator of a sparse image (Eq.
// phi-discrete restricted to the active atoms) and the adjoint restricted to
// the atoms (Eq. adjoint-phi evaluated at the atoms' pixels only).
//
// The phase of visibility k and atom p is t = A_k a_p + B_k b_p turns, with
// A_k = u_k dl, B_k = v_k dl and integer pixel offsets a_p = i_p - n/2,
// b_p = j_p - n/2.  t is formed and reduced to [-1/2, 1/2] in FP64 (t can
// reach ~10^3 turns, beyond FP32's resolution); the reduced value feeds the
// hardware sine/cosine, whose argument is in revolutions, in FP32.  The FP64
// twin evaluates sin/cos of 2 pi t in double.
//
// Non-coplanar baselines (Sect. 2.1, Eq. phi-plane) add the w-term's phase
// w_k c_p, c_p = n_p - 1, to t, also in FP64 (template flag HW; the plan then
// holds w_k in plan order, the atom table c_p).
#include <algorithm>
#include <cstring>

#include <atomic>
#include <mutex>
#include <string>

#include "common.h"

namespace pc {

template <typename R>
__global__ void atom_prep_kernel(int64_t natoms, int64_t ntotal, int n, double dl,
                                 const int32_t* __restrict__ pix, const R* __restrict__ weight,
                                 Atom<R>* __restrict__ atoms) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ntotal) return;
  if (p >= natoms) {  // padding: the phase-centre pixel with zero weight
    atoms[p] = Atom<R>{0.0, 0.0, 1.0, 0.0, R(0), R(0)};
    return;
  }
  const int q = pix[p];
  const int i = q / n, j = q - i * n;
  const double a = (double)(i - n / 2), b = (double)(j - n / 2);
  const double l = a * dl, m = b * dl;
  const double inv_n = 1.0 / sqrt(1.0 - l * l - m * m);
  Atom<R> at;
  at.a = a;
  at.b = b;
  at.inv_n = inv_n;
  at.c = n_minus_one(l, m);
  at.w = weight ? (R)((double)weight[p] * inv_n) : R(0);
  at.pad = R(0);
  atoms[p] = at;
}

template <typename R>
__device__ __forceinline__ void sincos_turns(double t, R& s, R& c) {
  // t already in [-1/2, 1/2] turns
  if constexpr (sizeof(R) == 4) {
    const float tf = (float)t;
    s = __builtin_amdgcn_sinf(tf);
    c = __builtin_amdgcn_cosf(tf);
  } else {
    double sd, cd;
    sincospi(2.0 * t, &sd, &cd);
    s = sd;
    c = cd;
  }
}

// sum_p w_p exp(-2 pi i t_kp) for one visibility (A, B, C = u dl, v dl, w),
// atoms in order, four at a time; shared by the single-plan and the batched
// forward so that both round identically.
template <typename R, bool HW>
__device__ __forceinline__ void forward_sum(double A, double B, double C, int64_t natoms,
                                            const Atom<R>* __restrict__ atoms, R& re, R& im) {
  re = 0;
  im = 0;
  int64_t p = 0;
  for (; p + 4 <= natoms; p += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const Atom<R> at = atoms[p + q];
      double t = fma(A, at.a, B * at.b);
      if constexpr (HW) t = fma(C, at.c, t);
      t -= rint(t);
      R s, c;
      sincos_turns<R>(t, s, c);
      re = fma(at.w, c, re);
      im = fma(-at.w, s, im);
    }
  }
  for (; p < natoms; ++p) {
    const Atom<R> at = atoms[p];
    double t = fma(A, at.a, B * at.b);
    if constexpr (HW) t = fma(C, at.c, t);
    t -= rint(t);
    R s, c;
    sincos_turns<R>(t, s, c);
    re = fma(at.w, c, re);
    im = fma(-at.w, s, im);
  }
}

// out_k = base_k - sum_p w_p exp(-2 pi i t_kp)   (base NULL: no base term)
// One thread per visibility (plan order); atoms are read with uniform
// (scalar) loads.
template <typename R, bool HW>
__global__ __launch_bounds__(256) void forward_sparse_kernel(
    int64_t L, int64_t natoms, const double* __restrict__ AB, const double* __restrict__ Cw,
    const Atom<R>* __restrict__ atoms,
    const cpx<R>* __restrict__ base, const int32_t* __restrict__ base_perm, R sign_base,
    cpx<R>* __restrict__ out, const int32_t* __restrict__ out_perm) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  R re, im;
  forward_sum<R, HW>(AB[2 * k], AB[2 * k + 1], HW ? Cw[k] : 0.0, natoms, atoms, re, im);
  cpx<R> o;
  if (base) {
    const cpx<R> b = base[base_perm ? base_perm[k] : k];
    o = {sign_base * b.x - re, sign_base * b.y - im};
  } else {
    o = {re, im};
  }
  out[out_perm ? out_perm[k] : k] = o;
}

// Residuals r = V - Phi_S x of several plans in one launch (plan order
// throughout): items[b] = (job, block of 256 visibilities).
__global__ __launch_bounds__(256) void forward_residual_batch_kernel(
    const FwdJob* __restrict__ jobs, const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const FwdJob& J = jobs[it.x];
  const int64_t k = (int64_t)it.y * 256 + threadIdx.x;
  if (k >= J.L) return;
  float re, im;
  if (J.Cw)
    forward_sum<float, true>(J.AB[2 * k], J.AB[2 * k + 1], J.Cw[k], J.natoms, J.atoms, re, im);
  else
    forward_sum<float, false>(J.AB[2 * k], J.AB[2 * k + 1], 0.0, J.natoms, J.atoms, re, im);
  const cpx<float> b = J.base[k];
  J.out[k] = {b.x - re, b.y - im};
}

void forward_residual_batch(BatchCtx& ctx, const std::vector<FwdJob>& jobs, hipStream_t s) {
  if (jobs.empty()) return;
  if (!ctx.done) PC_HIP(hipEventCreateWithFlags(&ctx.done, hipEventDisableTiming));
  if (ctx.pending) PC_HIP(hipEventSynchronize(ctx.done));
  std::vector<int2> items;
  for (size_t j = 0; j < jobs.size(); ++j)
    for (int64_t b = 0; b < (jobs[j].L + 255) / 256; ++b) items.push_back(make_int2((int)j, (int)b));
  const size_t o_items = (jobs.size() * sizeof(FwdJob) + 255) & ~size_t(255);
  const size_t bytes = o_items + items.size() * sizeof(int2);
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
  std::memcpy(ctx.host, jobs.data(), jobs.size() * sizeof(FwdJob));
  std::memcpy(ctx.host + o_items, items.data(), items.size() * sizeof(int2));
  PC_HIP(hipMemcpyAsync(ctx.dev, ctx.host, bytes, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(forward_residual_batch_kernel, dim3((unsigned)items.size()), dim3(256), 0, s,
                     (const FwdJob*)ctx.dev, (const int2*)(ctx.dev + o_items));
  PC_LAUNCH_CHECK("forward_residual_batch");
  PC_HIP(hipEventRecord(ctx.done, s));
  ctx.pending = true;
}

// Restricted adjoint, lanes over atoms.  A workgroup is 4 waves; each wave
// takes a chunk of K consecutive visibilities and up to 64 atoms.  With at
// least 64 atoms each lane owns one atom and the whole wave walks the chunk
// together; with A < 64 atoms (A a power of two) the wave splits into 64/A
// streams over the chunk, combined by a few lane shuffles at the end.  The
// chunk is staged through LDS in rounds of kAdjRound visibilities (one
// coalesced load per lane, double-buffered so that the next round's loads
// are in flight while the current one is summed); the lanes then read each
// visibility as an LDS broadcast and keep private running sums, so there is
// no cross-lane traffic per pair.  The 4 waves' sums are added in LDS and
// written as one partial per (atom, workgroup); a second kernel sums the
// partials in FP64 in a fixed order (bitwise reproducible) and applies 1/n.
constexpr int kAdjRound = 128;

struct AdjShape {
  int lgA;          // log2 atoms per wave
  int64_t ngroups;  // atom groups
  int64_t K;        // visibilities per wave (a multiple of kAdjRound)
  int64_t nwg;      // workgroups per atom group (grid: ngroups x nwg)
};

static AdjShape adjoint_shape(int64_t L, int64_t natoms) {
  AdjShape sh{};
  // at least 2 atoms per wave, so that the 64/A streams (<= 32) times the
  // 4-way unroll of the summing loop tile a round of kAdjRound exactly
  sh.lgA = 1;
  while ((1 << sh.lgA) < natoms && sh.lgA < 6) ++sh.lgA;
  const int64_t A = 1 << sh.lgA;
  sh.ngroups = (natoms + A - 1) / A;
  // about 8192 waves in all (32 per compute unit, 8 per SIMD)
  const int64_t waves = std::max<int64_t>(4, 8192 / sh.ngroups);
  const int64_t K = (L + waves - 1) / waves;
  sh.K = std::max<int64_t>(kAdjRound, (K + kAdjRound - 1) / kAdjRound * kAdjRound);
  sh.nwg = (L + 4 * sh.K - 1) / (4 * sh.K);
  return sh;
}

template <typename R, bool HW>
struct VisRec {
  double A, B;
  cpx<R> h;
};
template <typename R>
struct VisRec<R, true> {
  double A, B, C;
  cpx<R> h;
};

// One pair's term Re(h e^{+2 pi i t}) added to acc; with UNIT h is real (1,
// or 0 for a record past the chunk), so the term is h cos 2 pi t and the sine
// is never formed.
template <typename R, typename A, bool UNIT, bool HW>
__device__ __forceinline__ void adj_pair(const VisRec<R, HW>& v, double a, double b, double c,
                                         A& acc) {
  double t = fma(v.A, a, v.B * b);
  if constexpr (HW) t = fma(v.C, c, t);
  t -= rint(t);
  if constexpr (UNIT) {
    if constexpr (sizeof(R) == 4) {
      acc = fma((A)v.h.x, (A)__builtin_amdgcn_cosf((float)t), acc);
    } else {
      acc = fma((A)v.h.x, (A)cospi(2.0 * t), acc);
    }
  } else {
    R sn, cs;
    sincos_turns<R>(t, sn, cs);
    acc = fma((A)v.h.x, (A)cs, acc);
    acc = fma(-(A)v.h.y, (A)sn, acc);
  }
}

template <typename R, bool UNIT, bool HW>
__device__ __forceinline__ VisRec<R, HW> load_vis(int64_t k, int64_t k1,
                                                  const double* __restrict__ AB,
                                                  const double* __restrict__ Cw,
                                                  const cpx<R>* __restrict__ vis,
                                                  const int32_t* __restrict__ perm) {
  VisRec<R, HW> r{};  // past the chunk: contributes zero
  if (k < k1) {
    r.A = AB[2 * k];
    r.B = AB[2 * k + 1];
    if constexpr (HW) r.C = Cw[k];
    if constexpr (UNIT)
      r.h = {R(1), R(0)};
    else
      r.h = vis[perm ? perm[k] : k];
  }
  return r;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// With UNIT every visibility is 1 (vis is not read): the point-spread sums
// sum_k cos 2 pi (A_k a + B_k b).
// One workgroup's share: atom group grp, visibility chunk wg of the 4 K-long
// chunks (shared by the single-plan and the batched launches, which then
// round identically).
template <typename R, typename Acc, bool UNIT, bool HW>
__device__ __forceinline__ void adjoint_sparse_body(
    int64_t L, int64_t natoms, int lgA, int64_t K, int64_t nwg, const double* __restrict__ AB,
    const double* __restrict__ Cw, const cpx<R>* __restrict__ vis, const int32_t* __restrict__ perm,
    const Atom<R>* __restrict__ atoms, Acc* __restrict__ partial, int64_t grp, int64_t wg) {
  constexpr int T = kAdjRound;
  constexpr int PER = T / 64;  // staged visibilities per lane and round
  static_assert(T % 128 == 0, "a round must hold 4 x 32 visibilities");
  __shared__ VisRec<R, HW> stage[4][2][T];
  __shared__ Acc red[4][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int A = 1 << lgA;
  const int V = 64 >> lgA;
  const int ai = lane & (A - 1), st = lane >> lgA;
  const int64_t p = grp * A + ai;
  const bool live = p < natoms;
  const double a = atoms[live ? p : 0].a, b = atoms[live ? p : 0].b;
  const double c = HW ? atoms[live ? p : 0].c : 0.0;
  const int64_t k0 = (wg * 4 + w) * K;
  const int64_t k1 = k0 + K < L ? k0 + K : L;
  const int nround = k1 > k0 ? (int)((k1 - k0 + T - 1) / T) : 0;
  VisRec<R, HW> nxt[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q)
    nxt[q] = load_vis<R, UNIT, HW>(k0 + q * 64 + lane, k1, AB, Cw, vis, perm);
#pragma unroll
  for (int q = 0; q < PER; ++q) stage[w][0][q * 64 + lane] = nxt[q];
  wave_sync();
  // R accumulators per round (at most T / 4 terms each); with Acc = double
  // each round's four sums are added into FP64 totals, so that FP32 rounding
  // only ever applies to short runs (relative error ~1e-9 on long coherent sums)
  Acc tot0 = 0, tot1 = 0, tot2 = 0, tot3 = 0;
  R acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  for (int j = 0; j < nround; ++j) {
    const int64_t kn = k0 + (int64_t)(j + 1) * T;
    if (j + 1 < nround) {
#pragma unroll
      for (int q = 0; q < PER; ++q)
        nxt[q] = load_vis<R, UNIT, HW>(kn + q * 64 + lane, k1, AB, Cw, vis, perm);
    }
    const VisRec<R, HW>* cur = stage[w][j & 1];
    for (int i = st; i < T; i += 4 * V) {  // 4 V <= T (V <= 32)
      adj_pair<R, R, UNIT, HW>(cur[i], a, b, c, acc0);
      adj_pair<R, R, UNIT, HW>(cur[i + V], a, b, c, acc1);
      adj_pair<R, R, UNIT, HW>(cur[i + 2 * V], a, b, c, acc2);
      adj_pair<R, R, UNIT, HW>(cur[i + 3 * V], a, b, c, acc3);
    }
    if constexpr (sizeof(Acc) != sizeof(R)) {
      tot0 += (Acc)acc0;
      tot1 += (Acc)acc1;
      tot2 += (Acc)acc2;
      tot3 += (Acc)acc3;
      acc0 = acc1 = acc2 = acc3 = 0;
    }
    if (j + 1 < nround) {
#pragma unroll
      for (int q = 0; q < PER; ++q) stage[w][(j + 1) & 1][q * 64 + lane] = nxt[q];
    }
    wave_sync();
  }
  if constexpr (sizeof(Acc) == sizeof(R)) {
    tot0 = acc0;
    tot1 = acc1;
    tot2 = acc2;
    tot3 = acc3;
  }
  Acc acc = (tot0 + tot1) + (tot2 + tot3);
  for (int o = A; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && lane < A && live)
    partial[p * nwg + wg] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

template <typename R, typename Acc, bool UNIT, bool HW>
__global__ __launch_bounds__(256) void adjoint_sparse_kernel(
    int64_t L, int64_t natoms, int lgA, int64_t K, int64_t nwg, const double* __restrict__ AB,
    const double* __restrict__ Cw, const cpx<R>* __restrict__ vis, const int32_t* __restrict__ perm,
    const Atom<R>* __restrict__ atoms, Acc* __restrict__ partial) {
  const int64_t grp = (int64_t)blockIdx.x / nwg, wg = (int64_t)blockIdx.x - grp * nwg;
  adjoint_sparse_body<R, Acc, UNIT, HW>(L, natoms, lgA, K, nwg, AB, Cw, vis, perm, atoms, partial,
                                        grp, wg);
}

// out[p] = (1/n_p) sum_c partial[p][c], FP64, one workgroup per atom.
template <typename P, typename R>
__device__ __forceinline__ void adjoint_sparse_reduce_body(int64_t nwg,
                                                           const P* __restrict__ partial,
                                                           const Atom<R>* __restrict__ atoms,
                                                           double* __restrict__ out, int64_t p) {
  __shared__ double red[4];
  const P* row = partial + p * nwg;
  double s = 0;
  for (int64_t c = threadIdx.x; c < nwg; c += 256) s += (double)row[c];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[p] = (((red[0] + red[1]) + red[2]) + red[3]) * atoms[p].inv_n;
}

template <typename P, typename R>
__global__ __launch_bounds__(256) void adjoint_sparse_reduce_kernel(
    int64_t natoms, int64_t nwg, const P* __restrict__ partial, const Atom<R>* __restrict__ atoms,
    double* __restrict__ out) {
  adjoint_sparse_reduce_body<P, R>(nwg, partial, atoms, out, (int64_t)blockIdx.x);
}

// Restricted adjoints with FP64 totals of several coplanar FP32 plans in one
// launch per kind (unit visibilities or not), then one launch for all their
// final sums: items = (job, workgroup) and (job, atom).
struct AccJobDev {
  const double* AB;
  const cpx<float>* vis;
  const Atom<float>* atoms;
  double* partial;
  double* out;
  int64_t L, natoms, K, nwg;
  int lgA, pad;
};

template <bool UNIT>
__global__ __launch_bounds__(256) void adjoint_acc64_batch_kernel(const AccJobDev* __restrict__ jobs,
                                                                  const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const AccJobDev& J = jobs[it.x];
  const int64_t grp = (int64_t)it.y / J.nwg, wg = (int64_t)it.y - grp * J.nwg;
  adjoint_sparse_body<float, double, UNIT, false>(J.L, J.natoms, J.lgA, J.K, J.nwg, J.AB, nullptr,
                                                  J.vis, nullptr, J.atoms, J.partial, grp, wg);
}

__global__ __launch_bounds__(256) void adjoint_reduce_batch_kernel(const AccJobDev* __restrict__ jobs,
                                                                   const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const AccJobDev& J = jobs[it.x];
  adjoint_sparse_reduce_body<double, float>(J.nwg, J.partial, J.atoms, J.out, (int64_t)it.y);
}

// One APGD step on the restricted problem fused with the restricted
// adjoint's final sum (one workgroup per atom): g_p = (1/n_p) sum_c
// partial[p][c] in FP64 (or g_in[p] when partial is NULL), then the proximal
// gradient step from y and the momentum extrapolation
//   x+ = soft(y + g / L, lambda / L),  y+ = x+ + mom (x+ - x),
// with the new forward weight y+ / n_p.  stat[p] = |y_p| and
// stat[nS + p] = |g_p| (at the gradient point) feed the duality-gap test.
// Under positivity the prox is max(0, z - lambda / L), stat[p] = y_p (signed:
// the test is skipped while some y_p < 0) and stat[nS + p] = max(g_p, 0).
__global__ __launch_bounds__(256) void reduce_fista_kernel(
    int64_t nS, int64_t nwg, const float* __restrict__ partial, const double* __restrict__ g_in,
    Atom<float>* __restrict__ atoms, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ g_out, double* __restrict__ stat, double inv_lip, double thr,
    double mom, int positive) {
  __shared__ double red[4];
  const int64_t p = blockIdx.x;
  double gp;
  if (partial) {
    const float* row = partial + p * nwg;
    double s = 0;
    for (int64_t c = threadIdx.x; c < nwg; c += 256) s += (double)row[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    gp = (((red[0] + red[1]) + red[2]) + red[3]) * atoms[p].inv_n;
  } else {
    gp = g_in[p];
  }
  if (threadIdx.x == 0) {
    const double yo = y[p], xo = x[p];
    const double z = yo + gp * inv_lip;
    double xn;
    if (positive) {
      xn = z - thr > 0 ? z - thr : 0.0;
    } else {
      const double az = fabs(z) - thr;
      xn = az > 0 ? copysign(az, z) : 0.0;
    }
    const double yn = xn + mom * (xn - xo);
    g_out[p] = gp;
    stat[p] = positive ? yo : fabs(yo);
    stat[nS + p] = positive ? fmax(gp, 0.0) : fabs(gp);
    x[p] = xn;
    y[p] = yn;
    atoms[p].w = (float)(yn * atoms[p].inv_n);
  }
}

void reduce_fista(pc_plan* p, int64_t nS, int64_t nwg, const double* partial, const double* g_in,
                  Atom<float>* atoms, double* x, double* y, double* g_out, double* stat,
                  double inv_lip, double thr, double mom, bool positive, hipStream_t s) {
  if (nS <= 0) return;
  ProfScope ps(p, s, "reduce_fista", (double)sizeof(float) * nwg * nS + 64.0 * nS, (double)nS);
  hipLaunchKernelGGL(reduce_fista_kernel, dim3((unsigned)nS), dim3(256), 0, s, nS, nwg,
                     reinterpret_cast<const float*>(partial), g_in, atoms, x, y, g_out, stat,
                     inv_lip, thr, mom, positive ? 1 : 0);
  PC_LAUNCH_CHECK("reduce_fista");
}

template <typename R>
void prep_atoms_into(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                     Atom<R>* atoms, hipStream_t s) {
  if (natoms <= 0) return;
  const int64_t ntotal = atom_capacity(natoms);
  hipLaunchKernelGGL((atom_prep_kernel<R>), dim3((unsigned)((ntotal + 255) / 256)), dim3(256), 0,
                     s, natoms, ntotal, p->g.n, p->g.dl, pix, weight, atoms);
  PC_LAUNCH_CHECK("atom_prep");
}

template <typename R>
void forward_atoms(pc_plan* p, int64_t natoms, const Atom<R>* atoms, const cpx<R>* vis_base,
                   bool base_sorted, cpx<R>* out, bool out_sorted, hipStream_t s) {
  const unsigned nb = (unsigned)((p->L + 255) / 256);
  const double cb = 2.0 * sizeof(R);
  ProfScope ps(p, s, sizeof(R) == 4 ? "forward_sparse" : "forward_sparse_f64",
               p->L * (16 + (p->Cw ? 8 : 0) + cb + (vis_base ? cb : 0)) +
                   (double)natoms * sizeof(Atom<R>),
               (double)p->L * natoms);
  const int32_t* bperm = (vis_base && !base_sorted) ? p->perm : nullptr;
  const int32_t* operm = out_sorted ? nullptr : p->perm;
  if (p->Cw)
    hipLaunchKernelGGL((forward_sparse_kernel<R, true>), dim3(nb), dim3(256), 0, s, p->L, natoms,
                       p->AB, p->Cw, atoms, vis_base, bperm, R(1), out, operm);
  else
    hipLaunchKernelGGL((forward_sparse_kernel<R, false>), dim3(nb), dim3(256), 0, s, p->L, natoms,
                       p->AB, p->Cw, atoms, vis_base, bperm, R(1), out, operm);
  PC_LAUNCH_CHECK("forward_sparse");
}

// Forward and restricted adjoint in one pass, for active sets of at most
// kFusedMaxAtoms atoms (FP32 path).  For each visibility k:
//   r_k = base_k - sum_p w_p e^{-2 pi i t_kp}   (or the sum itself, no base)
// and every atom accumulates Re(r_k e^{+2 pi i t_kp}) with the same phase
// (one FP64 phase and one sin/cos per pair serve both operators).  Lanes run
// over visibilities, atoms are wave-uniform (scalar loads); each lane keeps
// the NB cosines and sines of its current visibility and NB running sums in
// registers.  A wave covers kpw consecutive visibilities and writes one
// partial per atom, partial[p * nwaves + wave] (FP32; summed in FP64 later,
// times 1/n_p, in a fixed order).  r is written only when r_out is given.
// Visibilities are in plan order; base_perm / out_perm (plan -> caller index)
// read the base from and write r to caller order instead.
constexpr int kFusedMaxAtoms = 64;

// One step of the recursive-halving lane reduction (compile-time counts, so
// that the values stay in registers).
template <int CNT, int D>
__device__ __forceinline__ void halve_reduce(float* g, int lane) {
  if constexpr (D >= 1) {
    if constexpr (CNT > 1) {
      constexpr int h = CNT / 2;
      const bool up = (lane & D) != 0;
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const float keep = up ? g[q + h] : g[q];
        const float send = up ? g[q] : g[q + h];
        g[q] = keep + __shfl_xor(send, D, 64);
      }
      halve_reduce<h, D / 2>(g, lane);
    } else {
      g[0] += __shfl_xor(g[0], D, 64);
      halve_reduce<1, D / 2>(g, lane);
    }
  }
}

template <int NB, bool HW>
__global__ __launch_bounds__(256) void forward_adjoint_kernel(
    int64_t L, int natoms, int64_t kpw, int64_t nwaves, const double* __restrict__ AB,
    const double* __restrict__ Cw, const Atom<float>* __restrict__ atoms, const cpx<float>* __restrict__ base,
    const int32_t* __restrict__ base_perm, cpx<float>* __restrict__ r_out,
    const int32_t* __restrict__ out_perm, float* __restrict__ partial) {
  constexpr int P2 = NB <= 8 ? 8 : (NB <= 16 ? 16 : (NB <= 32 ? 32 : 64));  // reduction width
  constexpr int SH = P2 == 8 ? 3 : (P2 == 16 ? 2 : (P2 == 32 ? 1 : 0));   // log2(64 / P2)
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= nwaves) return;  // no workgroup barrier below
  const int64_t k0 = wv * kpw;
  const int64_t k1 = k0 + kpw < L ? k0 + kpw : L;
  float g[P2];
#pragma unroll
  for (int q = 0; q < P2; ++q) g[q] = 0.f;
  // the next group's coordinates and base value are loaded one group ahead
  double An = 0.0, Bn = 0.0, Cn = 0.0;
  cpx<float> vn{0.f, 0.f};
  if (k0 + lane < k1) {
    An = AB[2 * (k0 + lane)];
    Bn = AB[2 * (k0 + lane) + 1];
    if constexpr (HW) Cn = Cw[k0 + lane];
    if (base) vn = base[base_perm ? base_perm[k0 + lane] : k0 + lane];
  }
  for (int64_t kb = k0; kb < k1; kb += 64) {
    const int64_t k = kb + lane;
    const bool live = k < k1;
    const double A = An, B = Bn, C = Cn;
    const cpx<float> v = vn;
    const int64_t kq = k + 64;
    if (kq < k1) {
      An = AB[2 * kq];
      Bn = AB[2 * kq + 1];
      if constexpr (HW) Cn = Cw[kq];
      if (base) vn = base[base_perm ? base_perm[kq] : kq];
    }
    float c[NB], sn[NB];
    float fr = 0.f, fi = 0.f;
    // opaque per iteration: the atom loads stay in the loop (as scalar loads
    // next to their use) instead of being hoisted and kept in spilled SGPRs
    uint64_t ai = reinterpret_cast<uint64_t>(atoms);
    asm volatile("" : "+s"(ai));
    const __attribute__((address_space(4))) Atom<float>* ap =
        reinterpret_cast<const __attribute__((address_space(4))) Atom<float>*>(ai);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      // entries natoms..NB-1 are zero-weight padding (their sums are never stored)
      const double aa = ap[q].a, ab = ap[q].b;
      const float w = ap[q].w;
      double t = fma(A, aa, B * ab);
      if constexpr (HW) t = fma(C, ap[q].c, t);
      t -= rint(t);
      sincos_turns<float>(t, sn[q], c[q]);
      fr = fmaf(w, c[q], fr);
      fi = fmaf(w, sn[q], fi);
    }
    // sum_p w_p e^{-i theta} = fr - i fi
    float rx = base ? v.x - fr : fr;
    float ry = base ? v.y + fi : -fi;
    if (!live) rx = ry = 0.f;
    if (r_out && live) r_out[out_perm ? out_perm[k] : k] = {rx, ry};
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      g[q] = fmaf(rx, c[q], g[q]);
      g[q] = fmaf(-ry, sn[q], g[q]);
    }
  }
  // Sum the P2 values over the 64 lanes by recursive halving: at distance d
  // a lane keeps one half of its values (the upper half when bit d of its
  // index is set) and adds its partner's copy of that half.  Lane l ends with
  // the total of value l >> SH.
  halve_reduce<P2, 32>(g, lane);
  const int idx = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && idx < natoms) partial[(int64_t)idx * nwaves + wv] = g[0];
}

struct FusedShape {
  int nb;          // atoms per pass (template), >= natoms
  int64_t kpw;     // visibilities per wave (a multiple of 64)
  int64_t nwaves;  // waves, one partial each per atom
};

// Waves of forward_adjoint_kernel<NB> resident on the device at once (the
// kernel is register-limited: 3 NB values per lane), from the runtime's
// occupancy calculator; cached per device and NB.
static int64_t fused_resident_waves(int nb, bool hw) {
  constexpr int kDev = 64;
  static std::atomic<int64_t> cache[kDev][2][kFusedMaxAtoms / 8 + 1];  // zero-initialised
  int dev = 0;
  PC_HIP(hipGetDevice(&dev));
  std::atomic<int64_t>& slot = cache[dev < kDev ? dev : 0][hw ? 1 : 0][nb / 8];
  const int64_t known = slot.load(std::memory_order_relaxed);
  if (known > 0) return known;
  const void* fn = nullptr;
  switch (nb) {
#define PC_NB(n) \
  case n:        \
    fn = hw ? (const void*)forward_adjoint_kernel<n, true>      \
            : (const void*)forward_adjoint_kernel<n, false>; \
    break;
    PC_NB(8) PC_NB(16) PC_NB(24) PC_NB(32) PC_NB(40) PC_NB(48) PC_NB(56) PC_NB(64)
#undef PC_NB
    default:
      fail(PC_ERR_UNSUPPORTED, "forward_adjoint_atoms: atoms per pass");
  }
  int blocks = 0, cus = 0;
  PC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 256, 0));
  PC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t waves = std::max<int64_t>(1, (int64_t)blocks * 4 * cus);
  slot.store(waves, std::memory_order_relaxed);
  return waves;
}

static FusedShape fused_shape(const pc_plan* p, int64_t natoms) {
  const int64_t L = p->L;
  FusedShape f{};
  f.nb = (int)((natoms + 7) / 8 * 8);
  // one round of resident waves, each over a contiguous range
  const int64_t target = fused_resident_waves(f.nb, p->Cw != nullptr);
  const int64_t k = (L + target - 1) / target;
  f.kpw = std::max<int64_t>(64, (k + 63) / 64 * 64);
  f.nwaves = (L + f.kpw - 1) / f.kpw;
  return f;
}

bool fused_supported(int64_t natoms) { return natoms >= 1 && natoms <= kFusedMaxAtoms; }

int64_t fused_partial_stride(const pc_plan* p, int64_t natoms) {
  return fused_shape(p, natoms).nwaves;
}

void forward_adjoint_atoms(pc_plan* p, int64_t natoms, const Atom<float>* atoms,
                           const cpx<float>* base, cpx<float>* r_out, double* partial,
                           hipStream_t s, bool caller_order) {
  if (!fused_supported(natoms))
    fail(PC_ERR_INVALID_ARG, "forward_adjoint_atoms: active set of " + std::to_string(natoms) +
                             " atoms (1.." + std::to_string(kFusedMaxAtoms) + " supported)");
  const FusedShape f = fused_shape(p, natoms);
  float* part = reinterpret_cast<float*>(partial);
  ProfScope ps(p, s, "forward_adjoint_sparse",
               p->L * (16.0 + (p->Cw ? 8.0 : 0.0) + (base ? 8.0 : 0.0) + (r_out ? 8.0 : 0.0)) +
                   4.0 * f.nwaves * natoms + (double)sizeof(Atom<float>) * natoms,
               (double)p->L * natoms);
  const unsigned nblk = (unsigned)((f.nwaves + 3) / 4);
  const int32_t* perm = caller_order ? p->perm : nullptr;
  switch (f.nb) {
#define PC_NB(nb)                                                                              \
  case nb:                                                                                     \
    if (p->Cw)                                                                                 \
      hipLaunchKernelGGL((forward_adjoint_kernel<nb, true>), dim3(nblk), dim3(256), 0, s, p->L, \
                         (int)natoms, f.kpw, f.nwaves, p->AB, p->Cw, atoms, base, perm, r_out,  \
                         perm, part);                                                          \
    else                                                                                       \
      hipLaunchKernelGGL((forward_adjoint_kernel<nb, false>), dim3(nblk), dim3(256), 0, s,      \
                         p->L, (int)natoms, f.kpw, f.nwaves, p->AB, p->Cw, atoms, base, perm,   \
                         r_out, perm, part);                                                   \
    break;
    PC_NB(8) PC_NB(16) PC_NB(24) PC_NB(32) PC_NB(40) PC_NB(48) PC_NB(56) PC_NB(64)
#undef PC_NB
    default:
      fail(PC_ERR_UNSUPPORTED, "forward_adjoint_atoms: atoms per pass");
  }
  PC_LAUNCH_CHECK("forward_adjoint_sparse");
}

// out[p] = (1/n_p) sum_c partial[p * nwg + c] for partials stored as R.
template <typename R>
void reduce_partials(pc_plan* p, int64_t natoms, int64_t nwg, const double* partial,
                     const Atom<R>* atoms, double* out, hipStream_t s) {
  if (natoms <= 0) return;
  ProfScope ps(p, s, "adjoint_sparse_reduce", (double)sizeof(R) * nwg * natoms,
               (double)nwg * natoms);
  hipLaunchKernelGGL((adjoint_sparse_reduce_kernel<R, R>), dim3((unsigned)natoms), dim3(256), 0, s,
                     natoms, nwg, reinterpret_cast<const R*>(partial), atoms, out);
  PC_LAUNCH_CHECK("adjoint_sparse_reduce");
}

// Partial-sum buffer size, in doubles (the kernels store R values in it).
int64_t adjoint_partial_count(const pc_plan* p, int64_t natoms) {
  const int64_t na = std::max<int64_t>(natoms, 1);
  int64_t nwg = adjoint_shape(p->L, na).nwg;
  if (fused_supported(na)) nwg = std::max(nwg, fused_shape(p, na).nwaves);
  return nwg * na;  // also holds the fused pass's partials
}

int64_t adjoint_partial_stride(const pc_plan* p, int64_t natoms) {
  return adjoint_shape(p->L, std::max<int64_t>(natoms, 1)).nwg;
}

template <typename R>
void adjoint_atoms(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                   const Atom<R>* atoms, double* partial, double* out, hipStream_t s) {
  if (natoms <= 0) return;
  const AdjShape sh = adjoint_shape(p->L, natoms);
  R* part = reinterpret_cast<R*>(partial);
  {
    ProfScope ps(p, s, sizeof(R) == 4 ? "adjoint_sparse" : "adjoint_sparse_f64",
                 p->L * (16 + (p->Cw ? 8 : 0) + 2.0 * sizeof(R)) * sh.ngroups +
                     (double)sizeof(R) * sh.nwg * natoms,
                 (double)p->L * natoms);
    const dim3 grid((unsigned)(sh.nwg * sh.ngroups));
    const int32_t* perm = vis_sorted ? nullptr : p->perm;
    if (p->Cw)
      hipLaunchKernelGGL((adjoint_sparse_kernel<R, R, false, true>), grid, dim3(256), 0, s, p->L,
                         natoms, sh.lgA, sh.K, sh.nwg, p->AB, p->Cw, vis, perm, atoms, part);
    else
      hipLaunchKernelGGL((adjoint_sparse_kernel<R, R, false, false>), grid, dim3(256), 0, s, p->L,
                         natoms, sh.lgA, sh.K, sh.nwg, p->AB, p->Cw, vis, perm, atoms, part);
    PC_LAUNCH_CHECK("adjoint_sparse");
  }
  if (!out) return;  // the caller sums the partials (fused with its next step)
  reduce_partials<R>(p, natoms, sh.nwg, partial, atoms, out, s);
}

void adjoint_atoms_acc64(pc_plan* p, const c32* vis, int64_t natoms, const Atom<float>* atoms,
                         double* partial, double* out, hipStream_t s) {
  if (natoms <= 0) return;
  const AdjShape sh = adjoint_shape(p->L, natoms);
  const dim3 grid((unsigned)(sh.nwg * sh.ngroups));
  if (vis) {
    ProfScope ps(p, s, "adjoint_sparse_acc64",
                 p->L * (p->Cw ? 32.0 : 24.0) * sh.ngroups + 8.0 * sh.nwg * natoms,
                 (double)p->L * natoms);
    if (p->Cw)
      hipLaunchKernelGGL((adjoint_sparse_kernel<float, double, false, true>), grid, dim3(256), 0,
                         s, p->L, natoms, sh.lgA, sh.K, sh.nwg, p->AB, p->Cw, vis,
                         (const int32_t*)nullptr, atoms, partial);
    else
      hipLaunchKernelGGL((adjoint_sparse_kernel<float, double, false, false>), grid, dim3(256), 0,
                         s, p->L, natoms, sh.lgA, sh.K, sh.nwg, p->AB, p->Cw, vis,
                         (const int32_t*)nullptr, atoms, partial);
    PC_LAUNCH_CHECK("adjoint_sparse_acc64");
  } else {  // unit visibilities: the point-spread sums (coplanar plans only)
    if (p->Cw) fail(PC_ERR_UNSUPPORTED, "point-spread sums of a non-coplanar plan");
    ProfScope ps(p, s, "psf_sums_acc64",
                 p->L * 16.0 * sh.ngroups + 8.0 * sh.nwg * natoms, (double)p->L * natoms);
    hipLaunchKernelGGL((adjoint_sparse_kernel<float, double, true, false>), grid, dim3(256), 0, s,
                       p->L, natoms, sh.lgA, sh.K, sh.nwg, p->AB, p->Cw, (const c32*)nullptr,
                       (const int32_t*)nullptr, atoms, partial);
    PC_LAUNCH_CHECK("psf_sums_acc64");
  }
  ProfScope ps(p, s, "adjoint_sparse_reduce", 8.0 * sh.nwg * natoms, (double)sh.nwg * natoms);
  hipLaunchKernelGGL((adjoint_sparse_reduce_kernel<double, float>), dim3((unsigned)natoms),
                     dim3(256), 0, s, natoms, sh.nwg, (const double*)partial, atoms, out);
  PC_LAUNCH_CHECK("adjoint_sparse_reduce");
}

template <typename R>
void forward_sparse(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                    const cpx<R>* vis_base, bool base_sorted, cpx<R>* out, bool out_sorted,
                    hipStream_t s) {
  Atom<R>* atoms = (Atom<R>*)ensure_atom_scratch(p, atom_capacity(natoms) * sizeof(Atom<R>));
  prep_atoms_into<R>(p, natoms, pix, weight, atoms, s);
  forward_atoms<R>(p, natoms, atoms, vis_base, base_sorted, out, out_sorted, s);
}

// The restricted gradient on caller-provided scratch: `atoms` holds
// atom_capacity(natoms) entries and `partial` adjoint_partial_count doubles.
static void restricted_gradient_on(pc_plan* p, const c32* vis, int64_t natoms,
                                   const int32_t* pix, const float* weight, double* out,
                                   c32* resid, Atom<float>* atoms, double* partial,
                                   hipStream_t s) {
  prep_atoms_into<float>(p, natoms, pix, weight, atoms, s);
  if (fused_supported(natoms)) {
    forward_adjoint_atoms(p, natoms, atoms, vis, resid, partial, s, true);
    reduce_partials<float>(p, natoms, fused_partial_stride(p, natoms), partial, atoms, out, s);
    return;
  }
  // r in caller order (resid) or in plan order (scratch)
  c32* r = resid ? resid : (c32*)p->vis_scratch;
  forward_atoms<float>(p, natoms, atoms, vis, false, r, resid == nullptr, s);
  adjoint_atoms<float>(p, r, resid == nullptr, natoms, atoms, partial, out, s);
}

void restricted_gradient(pc_plan* p, const c32* vis, int64_t natoms, const int32_t* pix,
                         const float* weight, double* out, c32* resid, hipStream_t s) {
  if (natoms == 0) {  // r = V
    if (resid)
      PC_HIP(hipMemcpyAsync(resid, vis, p->L * sizeof(c32), hipMemcpyDeviceToDevice, s));
    return;
  }
  Atom<float>* atoms =
      (Atom<float>*)ensure_atom_scratch(p, atom_capacity(natoms) * sizeof(Atom<float>));
  double* partial = ensure_red_scratch(p, (size_t)adjoint_partial_count(p, natoms));
  restricted_gradient_on(p, vis, natoms, pix, weight, out, resid, atoms, partial, s);
}

// ---------------------------------------------------------------------------
// Allocation-free restricted gradient, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).  The atom
// table and the partial sums, which restricted_gradient keeps in plan scratch
// grown on demand, live here in one fixed device array instead.  Each device
// holds its own copy until the process ends; the host reaches it only through
// the address hipGetSymbolAddress returns on that device.  Every call on a
// device shares the array, so calls that overlap on one device race.  Nothing
// in it needs clearing: each call writes every entry it reads first (the atom
// table by atom_prep_kernel, each partial by the workgroup or wave owning it).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device.
static unsigned char* scratch_on_device() {
  int dev = 0;
  PC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    fail(PC_ERR_UNSUPPORTED, "device index " + std::to_string(dev) + " beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(PC_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

size_t restricted_gradient_scratch_bytes(const pc_plan* p, int64_t natoms) {
  if (natoms <= 0) return 0;
  return round256((size_t)atom_capacity(natoms) * sizeof(Atom<float>)) +
         (size_t)adjoint_partial_count(p, natoms) * sizeof(double);
}

void restricted_gradient_noalloc(pc_plan* p, const c32* vis, int64_t natoms, const int32_t* pix,
                                 const float* weight, double* out, c32* resid, hipStream_t s) {
  if (p->prof.on)
    fail(PC_ERR_INVALID_ARG, "the plan's instrumentation must be off (it creates HIP events)");
  if (natoms == 0) {  // r = V
    if (resid)
      PC_HIP(hipMemcpyAsync(resid, vis, p->L * sizeof(c32), hipMemcpyDeviceToDevice, s));
    return;
  }
  const size_t need = restricted_gradient_scratch_bytes(p, natoms);
  if (need > kNoAllocScratchBytes)
    fail(PC_ERR_UNSUPPORTED, std::to_string(natoms) + " atoms over " + std::to_string(p->L) +
                                 " visibilities need " + std::to_string(need) +
                                 " bytes of scratch, more than the fixed " +
                                 std::to_string(kNoAllocScratchBytes));
  unsigned char* base = scratch_on_device();
  Atom<float>* atoms = reinterpret_cast<Atom<float>*>(base);
  double* partial = reinterpret_cast<double*>(
      base + round256((size_t)atom_capacity(natoms) * sizeof(Atom<float>)));
  restricted_gradient_on(p, vis, natoms, pix, weight, out, resid, atoms, partial, s);
}

template <typename R>
void adjoint_sparse(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                    const int32_t* pix, double* out, hipStream_t s) {
  if (natoms == 0) return;
  Atom<R>* atoms = (Atom<R>*)ensure_atom_scratch(p, atom_capacity(natoms) * sizeof(Atom<R>));
  prep_atoms_into<R>(p, natoms, pix, (const R*)nullptr, atoms, s);
  double* partial = ensure_red_scratch(p, (size_t)adjoint_partial_count(p, natoms));
  adjoint_atoms<R>(p, vis, vis_sorted, natoms, atoms, partial, out, s);
}

void adjoint_acc64_batch(BatchCtx& ctx, const std::vector<AccJob>& jobs, hipStream_t s) {
  std::vector<AccJobDev> dj;
  std::vector<int2> unit_items, vis_items, red_items;
  for (const AccJob& a : jobs) {
    if (a.natoms <= 0) continue;
    PC_REQUIRE(a.p->precision == PC_PREC_FP32 && !a.p->Cw,
               "batched restricted adjoints need coplanar FP32 plans");
    const AdjShape sh = adjoint_shape(a.p->L, a.natoms);
    const int j = (int)dj.size();
    dj.push_back(AccJobDev{a.p->AB, a.vis, a.atoms, a.partial, a.out, a.p->L, a.natoms, sh.K,
                           sh.nwg, sh.lgA, 0});
    std::vector<int2>& dst = a.vis ? vis_items : unit_items;
    for (int64_t b = 0; b < sh.ngroups * sh.nwg; ++b) dst.push_back(make_int2(j, (int)b));
    for (int64_t q = 0; q < a.natoms; ++q) red_items.push_back(make_int2(j, (int)q));
  }
  if (dj.empty()) return;
  if (!ctx.done) PC_HIP(hipEventCreateWithFlags(&ctx.done, hipEventDisableTiming));
  if (ctx.pending) PC_HIP(hipEventSynchronize(ctx.done));
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_unit = up(dj.size() * sizeof(AccJobDev));
  const size_t o_vis = o_unit + up(unit_items.size() * sizeof(int2));
  const size_t o_red = o_vis + up(vis_items.size() * sizeof(int2));
  const size_t bytes = o_red + red_items.size() * sizeof(int2);
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
  std::memcpy(ctx.host, dj.data(), dj.size() * sizeof(AccJobDev));
  if (!unit_items.empty())
    std::memcpy(ctx.host + o_unit, unit_items.data(), unit_items.size() * sizeof(int2));
  if (!vis_items.empty())
    std::memcpy(ctx.host + o_vis, vis_items.data(), vis_items.size() * sizeof(int2));
  std::memcpy(ctx.host + o_red, red_items.data(), red_items.size() * sizeof(int2));
  PC_HIP(hipMemcpyAsync(ctx.dev, ctx.host, bytes, hipMemcpyHostToDevice, s));
  const AccJobDev* d = (const AccJobDev*)ctx.dev;
  if (!unit_items.empty()) {
    hipLaunchKernelGGL((adjoint_acc64_batch_kernel<true>), dim3((unsigned)unit_items.size()),
                       dim3(256), 0, s, d, (const int2*)(ctx.dev + o_unit));
    PC_LAUNCH_CHECK("psf_sums_acc64_batch");
  }
  if (!vis_items.empty()) {
    hipLaunchKernelGGL((adjoint_acc64_batch_kernel<false>), dim3((unsigned)vis_items.size()),
                       dim3(256), 0, s, d, (const int2*)(ctx.dev + o_vis));
    PC_LAUNCH_CHECK("adjoint_sparse_acc64_batch");
  }
  hipLaunchKernelGGL(adjoint_reduce_batch_kernel, dim3((unsigned)red_items.size()), dim3(256), 0,
                     s, d, (const int2*)(ctx.dev + o_red));
  PC_LAUNCH_CHECK("adjoint_reduce_batch");
  PC_HIP(hipEventRecord(ctx.done, s));
  ctx.pending = true;
}

template void forward_sparse<float>(pc_plan*, int64_t, const int32_t*, const float*, const c32*,
                                    bool, c32*, bool, hipStream_t);
template void forward_sparse<double>(pc_plan*, int64_t, const int32_t*, const double*, const c64*,
                                     bool, c64*, bool, hipStream_t);
template void adjoint_sparse<float>(pc_plan*, const c32*, bool, int64_t, const int32_t*, double*,
                                    hipStream_t);
template void adjoint_sparse<double>(pc_plan*, const c64*, bool, int64_t, const int32_t*, double*,
                                     hipStream_t);
template void prep_atoms_into<float>(pc_plan*, int64_t, const int32_t*, const float*, Atom<float>*,
                                     hipStream_t);
template void forward_atoms<float>(pc_plan*, int64_t, const Atom<float>*, const c32*, bool, c32*,
                                   bool, hipStream_t);
template void reduce_partials<float>(pc_plan*, int64_t, int64_t, const double*, const Atom<float>*,
                                     double*, hipStream_t);
template void adjoint_atoms<float>(pc_plan*, const c32*, bool, int64_t, const Atom<float>*,
                                   double*, double*, hipStream_t);

}  // namespace pc
