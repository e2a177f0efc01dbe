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

// Restricted adjoint, lanes over visibilities: each lane holds kVPT
// visibilities in registers; for each atom (uniform loop, scalar loads) it
// sums Re(h_k exp(+2 pi i t_kp)) over its visibilities in R precision, the
// wave reduces the 64 lane sums, and lane 0 writes the wave's partial to
// partial[p][wave] (atom-major, so the final sum reads contiguously).  The
// per-atom sum over waves is done in FP64 by a second kernel, in a fixed
// order (bitwise reproducible).
constexpr int kVPT = 4;
constexpr int kAdjThreads = 256;
constexpr int kVisChunk = kVPT * kAdjThreads;  // visibilities per workgroup

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename R>
__global__ __launch_bounds__(kAdjThreads) void adjoint_sparse_kernel(
    int64_t L, int64_t natoms, const double* __restrict__ AB, const cpx<R>* __restrict__ vis,
    const int32_t* __restrict__ perm, const Atom<R>* __restrict__ atoms,
    R* __restrict__ partial, int64_t nwaves) {
  const int64_t k0 = (int64_t)blockIdx.x * kVisChunk + threadIdx.x;
  double A[kVPT], B[kVPT];
  R hx[kVPT], hy[kVPT];
#pragma unroll
  for (int i = 0; i < kVPT; ++i) {
    const int64_t k = k0 + (int64_t)i * kAdjThreads;
    if (k < L) {
      A[i] = AB[2 * k];
      B[i] = AB[2 * k + 1];
      const cpx<R> h = vis[perm ? perm[k] : k];
      hx[i] = h.x;
      hy[i] = h.y;
    } else {
      A[i] = B[i] = 0.0;
      hx[i] = hy[i] = R(0);
    }
  }
  const int64_t wave = (int64_t)blockIdx.x * (kAdjThreads / 64) + (threadIdx.x >> 6);
  const bool lane0 = (threadIdx.x & 63) == 0;
  for (int64_t p = 0; p < natoms; ++p) {
    const double a = atoms[p].a, b = atoms[p].b;
    R acc = 0;
#pragma unroll
    for (int i = 0; i < kVPT; ++i) {
      double t = fma(A[i], a, B[i] * b);
      t -= rint(t);
      R s, c;
      sincos_turns<R>(t, s, c);
      acc = fma(hx[i], c, acc);
      acc = fma(-hy[i], s, acc);
    }
    acc = wave_sum<R>(acc);
    if (lane0) partial[p * nwaves + wave] = acc;
  }
}

// out[p] = (1/n_p) sum_w partial[p][w], FP64, one wave per atom.
template <typename R>
__global__ __launch_bounds__(64) void adjoint_sparse_reduce_kernel(
    int64_t natoms, int64_t nwaves, const R* __restrict__ partial,
    const Atom<R>* __restrict__ atoms, double* __restrict__ out) {
  const int64_t p = blockIdx.x;
  const R* row = partial + p * nwaves;
  double s = 0;
  for (int64_t w = threadIdx.x; w < nwaves; w += 64) s += (double)row[w];
  s = wave_sum<double>(s);
  if (threadIdx.x == 0) out[p] = s * atoms[p].inv_n;
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
  const int64_t nwaves = ((p->L + kVisChunk - 1) / kVisChunk) * (kAdjThreads / 64);
  return nwaves * std::max<int64_t>(natoms, 1);
}

template <typename R>
void adjoint_atoms(pc_plan* p, const cpx<R>* vis, bool vis_sorted, int64_t natoms,
                   const Atom<R>* atoms, double* partial, double* out, hipStream_t s) {
  if (natoms <= 0) return;
  const int64_t nblocks = (p->L + kVisChunk - 1) / kVisChunk;
  const int64_t nwaves = nblocks * (kAdjThreads / 64);
  R* part = reinterpret_cast<R*>(partial);
  {
    ProfScope ps(p, s, sizeof(R) == 4 ? "adjoint_sparse" : "adjoint_sparse_f64",
                 p->L * (16 + 2.0 * sizeof(R)) + (double)sizeof(R) * nwaves * natoms,
                 (double)p->L * natoms);
    hipLaunchKernelGGL((adjoint_sparse_kernel<R>), dim3((unsigned)nblocks), dim3(kAdjThreads), 0, s,
                       p->L, natoms, p->AB, vis, vis_sorted ? nullptr : p->perm, atoms, part,
                       nwaves);
    PC_LAUNCH_CHECK("adjoint_sparse");
  }
  ProfScope ps(p, s, "adjoint_sparse_reduce", (double)sizeof(R) * nwaves * natoms,
               (double)nwaves * natoms);
  hipLaunchKernelGGL((adjoint_sparse_reduce_kernel<R>), dim3((unsigned)natoms), dim3(64), 0, s,
                     natoms, nwaves, (const R*)part, atoms, out);
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
