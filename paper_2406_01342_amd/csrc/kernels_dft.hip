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
#include <algorithm>
#include <cstring>

#include "common.h"

namespace pc {

template <typename R>
__global__ void atom_prep_kernel(int64_t natoms, int n, double dl, const int32_t* __restrict__ pix,
                                 const R* __restrict__ weight, Atom<R>* __restrict__ atoms) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= natoms) return;
  const int q = pix[p];
  const int i = q / n, j = q - i * n;
  const double a = (double)(i - n / 2), b = (double)(j - n / 2);
  const double l = a * dl, m = b * dl;
  const double inv_n = 1.0 / sqrt(1.0 - l * l - m * m);
  Atom<R> at;
  at.a = a;
  at.b = b;
  at.inv_n = inv_n;
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

// out_k = base_k - sum_p w_p exp(-2 pi i t_kp)   (base NULL: no base term)
// One thread per visibility (plan order); atoms are read with uniform
// (scalar) loads.
template <typename R>
__global__ __launch_bounds__(256) void forward_sparse_kernel(
    int64_t L, int64_t natoms, const double* __restrict__ AB, const Atom<R>* __restrict__ atoms,
    const cpx<R>* __restrict__ base, const int32_t* __restrict__ base_perm, R sign_base,
    cpx<R>* __restrict__ out, const int32_t* __restrict__ out_perm) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const double A = AB[2 * k], B = AB[2 * k + 1];
  R re = 0, im = 0;
  int64_t p = 0;
  for (; p + 4 <= natoms; p += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const Atom<R> at = atoms[p + q];
      double t = fma(A, at.a, B * at.b);
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
    t -= rint(t);
    R s, c;
    sincos_turns<R>(t, s, c);
    re = fma(at.w, c, re);
    im = fma(-at.w, s, im);
  }
  cpx<R> o;
  if (base) {
    const cpx<R> b = base[base_perm ? base_perm[k] : k];
    o = {sign_base * b.x - re, sign_base * b.y - im};
  } else {
    o = {re, im};
  }
  out[out_perm ? out_perm[k] : k] = o;
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

template <typename R>
struct VisRec {
  double A, B;
  cpx<R> h;
};

template <typename R>
__device__ __forceinline__ void adj_pair(const VisRec<R>& v, double a, double b, R& acc) {
  double t = fma(v.A, a, v.B * b);
  t -= rint(t);
  R sn, cs;
  sincos_turns<R>(t, sn, cs);
  acc = fma(v.h.x, cs, acc);
  acc = fma(-v.h.y, sn, acc);
}

template <typename R>
__device__ __forceinline__ VisRec<R> load_vis(int64_t k, int64_t k1, const double* __restrict__ AB,
                                              const cpx<R>* __restrict__ vis,
                                              const int32_t* __restrict__ perm) {
  VisRec<R> r{0.0, 0.0, {R(0), R(0)}};  // past the chunk: contributes zero
  if (k < k1) {
    r.A = AB[2 * k];
    r.B = AB[2 * k + 1];
    r.h = vis[perm ? perm[k] : k];
  }
  return r;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__global__ __launch_bounds__(256) void adjoint_sparse_kernel(
    int64_t L, int64_t natoms, int lgA, int64_t K, int64_t nwg, const double* __restrict__ AB,
    const cpx<R>* __restrict__ vis, const int32_t* __restrict__ perm,
    const Atom<R>* __restrict__ atoms, R* __restrict__ partial) {
  constexpr int T = kAdjRound;
  constexpr int PER = T / 64;  // staged visibilities per lane and round
  static_assert(T % 128 == 0, "a round must hold 4 x 32 visibilities");
  __shared__ VisRec<R> stage[4][2][T];
  __shared__ R red[4][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int A = 1 << lgA;
  const int V = 64 >> lgA;
  const int ai = lane & (A - 1), st = lane >> lgA;
  const int64_t grp = (int64_t)blockIdx.x / nwg, wg = (int64_t)blockIdx.x - grp * nwg;
  const int64_t p = grp * A + ai;
  const bool live = p < natoms;
  const double a = atoms[live ? p : 0].a, b = atoms[live ? p : 0].b;
  const int64_t k0 = (wg * 4 + w) * K;
  const int64_t k1 = k0 + K < L ? k0 + K : L;
  const int nround = k1 > k0 ? (int)((k1 - k0 + T - 1) / T) : 0;
  VisRec<R> nxt[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) nxt[q] = load_vis<R>(k0 + q * 64 + lane, k1, AB, vis, perm);
#pragma unroll
  for (int q = 0; q < PER; ++q) stage[w][0][q * 64 + lane] = nxt[q];
  wave_sync();
  R acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  for (int j = 0; j < nround; ++j) {
    const int64_t kn = k0 + (int64_t)(j + 1) * T;
    if (j + 1 < nround) {
#pragma unroll
      for (int q = 0; q < PER; ++q) nxt[q] = load_vis<R>(kn + q * 64 + lane, k1, AB, vis, perm);
    }
    const VisRec<R>* cur = stage[w][j & 1];
    for (int i = st; i < T; i += 4 * V) {  // 4 V <= T (V <= 32)
      adj_pair<R>(cur[i], a, b, acc0);
      adj_pair<R>(cur[i + V], a, b, acc1);
      adj_pair<R>(cur[i + 2 * V], a, b, acc2);
      adj_pair<R>(cur[i + 3 * V], a, b, acc3);
    }
    if (j + 1 < nround) {
#pragma unroll
      for (int q = 0; q < PER; ++q) stage[w][(j + 1) & 1][q * 64 + lane] = nxt[q];
    }
    wave_sync();
  }
  R acc = (acc0 + acc1) + (acc2 + acc3);
  for (int o = A; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && lane < A && live)
    partial[p * nwg + wg] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// out[p] = (1/n_p) sum_c partial[p][c], FP64, one workgroup per atom.
template <typename R>
__global__ __launch_bounds__(256) void adjoint_sparse_reduce_kernel(
    int64_t natoms, int64_t nwg, const R* __restrict__ partial, const Atom<R>* __restrict__ atoms,
    double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t p = blockIdx.x;
  const R* row = partial + p * nwg;
  double s = 0;
  for (int64_t c = threadIdx.x; c < nwg; c += 256) s += (double)row[c];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[p] = (((red[0] + red[1]) + red[2]) + red[3]) * atoms[p].inv_n;
}

// One APGD step on the restricted problem fused with the restricted
// adjoint's final sum (one workgroup per atom): g_p = (1/n_p) sum_c
// partial[p][c] in FP64 (or g_in[p] when partial is NULL), then the proximal
// gradient step from y and the momentum extrapolation
//   x+ = soft(y + g / L, lambda / L),  y+ = x+ + mom (x+ - x),
// with the new forward weight y+ / n_p.  stat[p] = |y_p| and
// stat[nS + p] = |g_p| (at the gradient point) feed the duality-gap test.
__global__ __launch_bounds__(256) void reduce_fista_kernel(
    int64_t nS, int64_t nwg, const float* __restrict__ partial, const double* __restrict__ g_in,
    Atom<float>* __restrict__ atoms, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ g_out, double* __restrict__ stat, double inv_lip, double thr,
    double mom) {
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
    const double az = fabs(z) - thr;
    const double xn = az > 0 ? copysign(az, z) : 0.0;
    const double yn = xn + mom * (xn - xo);
    g_out[p] = gp;
    stat[p] = fabs(yo);
    stat[nS + p] = fabs(gp);
    x[p] = xn;
    y[p] = yn;
    atoms[p].w = (float)(yn * atoms[p].inv_n);
  }
}

void reduce_fista(pc_plan* p, int64_t nS, int64_t nwg, const double* partial, const double* g_in,
                  Atom<float>* atoms, double* x, double* y, double* g_out, double* stat,
                  double inv_lip, double thr, double mom, hipStream_t s) {
  if (nS <= 0) return;
  ProfScope ps(p, s, "reduce_fista", (double)sizeof(float) * nwg * nS + 64.0 * nS, (double)nS);
  hipLaunchKernelGGL(reduce_fista_kernel, dim3((unsigned)nS), dim3(256), 0, s, nS, nwg,
                     reinterpret_cast<const float*>(partial), g_in, atoms, x, y, g_out, stat,
                     inv_lip, thr, mom);
  PC_LAUNCH_CHECK("reduce_fista");
}

template <typename R>
void prep_atoms_into(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                     Atom<R>* atoms, hipStream_t s) {
  if (natoms <= 0) return;
  hipLaunchKernelGGL((atom_prep_kernel<R>), dim3((unsigned)((natoms + 255) / 256)), dim3(256), 0,
                     s, natoms, p->g.n, p->g.dl, pix, weight, atoms);
  PC_LAUNCH_CHECK("atom_prep");
}

template <typename R>
void forward_atoms(pc_plan* p, int64_t natoms, const Atom<R>* atoms, const cpx<R>* vis_base,
                   bool base_sorted, cpx<R>* out, bool out_sorted, hipStream_t s) {
  const unsigned nb = (unsigned)((p->L + 255) / 256);
  const double cb = 2.0 * sizeof(R);
  ProfScope ps(p, s, sizeof(R) == 4 ? "forward_sparse" : "forward_sparse_f64",
               p->L * (16 + cb + (vis_base ? cb : 0)) + (double)natoms * sizeof(Atom<R>),
               (double)p->L * natoms);
  hipLaunchKernelGGL((forward_sparse_kernel<R>), dim3(nb), dim3(256), 0, s, p->L, natoms, p->AB,
                     atoms, vis_base, (vis_base && !base_sorted) ? p->perm : nullptr, R(1), out,
                     out_sorted ? nullptr : p->perm);
  PC_LAUNCH_CHECK("forward_sparse");
}

// Partial-sum buffer size, in doubles (the kernels store R values in it).
int64_t adjoint_partial_count(const pc_plan* p, int64_t natoms) {
  const AdjShape sh = adjoint_shape(p->L, std::max<int64_t>(natoms, 1));
  return sh.nwg * std::max<int64_t>(natoms, 1);
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
                 p->L * (16 + 2.0 * sizeof(R)) * sh.ngroups + (double)sizeof(R) * sh.nwg * natoms,
                 (double)p->L * natoms);
    hipLaunchKernelGGL((adjoint_sparse_kernel<R>), dim3((unsigned)(sh.nwg * sh.ngroups)),
                       dim3(256), 0, s, p->L, natoms, sh.lgA, sh.K, sh.nwg, p->AB, vis,
                       vis_sorted ? nullptr : p->perm, atoms, part);
    PC_LAUNCH_CHECK("adjoint_sparse");
  }
  if (!out) return;  // the caller sums the partials (fused with its next step)
  ProfScope ps(p, s, "adjoint_sparse_reduce", (double)sizeof(R) * sh.nwg * natoms,
               (double)sh.nwg * natoms);
  hipLaunchKernelGGL((adjoint_sparse_reduce_kernel<R>), dim3((unsigned)natoms), dim3(256), 0, s,
                     natoms, sh.nwg, (const R*)part, atoms, out);
  PC_LAUNCH_CHECK("adjoint_sparse_reduce");
}

template <typename R>
void forward_sparse(pc_plan* p, int64_t natoms, const int32_t* pix, const R* weight,
                    const cpx<R>* vis_base, bool base_sorted, cpx<R>* out, bool out_sorted,
                    hipStream_t s) {
  Atom<R>* atoms = (Atom<R>*)ensure_atom_scratch(p, std::max<int64_t>(natoms, 1) * sizeof(Atom<R>));
  prep_atoms_into<R>(p, natoms, pix, weight, atoms, s);
  forward_atoms<R>(p, natoms, atoms, vis_base, base_sorted, out, out_sorted, s);
}

template <typename R>
void adjoint_sparse(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                    const int32_t* pix, double* out, hipStream_t s) {
  if (natoms == 0) return;
  Atom<R>* atoms = (Atom<R>*)ensure_atom_scratch(p, std::max<int64_t>(natoms, 1) * sizeof(Atom<R>));
  prep_atoms_into<R>(p, natoms, pix, (const R*)nullptr, atoms, s);
  double* partial = ensure_red_scratch(p, (size_t)adjoint_partial_count(p, natoms));
  adjoint_atoms<R>(p, vis, vis_sorted, natoms, atoms, partial, out, s);
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
template void adjoint_atoms<float>(pc_plan*, const c32*, bool, int64_t, const Atom<float>*,
                                   double*, double*, hipStream_t);

}  // namespace pc
