// LDS-resident Stockham FFT for batches of power-of-two sequences.
//
// Each stage of radix R with current sub-transform length Ns reads input
// j + r (M/R), applies the twiddle w^(r k), k = j mod Ns, w = exp(s 2 pi i /
// (Ns R)), does a radix-R DFT in registers and writes output
// (j / Ns) Ns R + k + r Ns (the autosorting Stockham ordering), so the result
// is in natural order without a bit-reversal pass.  Stages: one radix-2^(p mod
// 4) stage first (no twiddles) when p = log2 M is not a multiple of 4, then
// radix-16 stages.  Twiddles exp(+2 pi i t / M) come from a two-level table
// held in LDS: lo[t mod 64] * hi[t / 64], lo[q] = exp(2 pi i q / M) and
// hi[q] = exp(2 pi i 64 q / M), both computed in FP64 on the host and rounded
// once (one extra rounding per twiddle).
#pragma once

#include "common.h"

namespace pc {

template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// exp(SIGN 2 pi i K / N) applied to v, with exact handling of the trivial
// angles (multiples of pi/2) so that no multiplication by 0/1 is emitted.
template <typename R, int N, int SIGN>
__host__ __device__ __forceinline__ cpx<R> rot(cpx<R> v, int K) {
  // cos(2 pi q / 16) for q = 0..4 (first quadrant), as literals so that no
  // table is materialised
  auto c16 = [](int q) -> double {
    return q == 0 ? 1.0
                  : q == 1 ? 0.92387953251128675613
                           : q == 2 ? 0.70710678118654752440
                                    : q == 3 ? 0.38268343236508977173 : 0.0;
  };
  const int k16 = (K * 16 / N) & 15;  // angle in units of 2 pi / 16
  if (k16 == 0) return v;
  if (k16 == 4) return SIGN > 0 ? cpx<R>{-v.y, v.x} : cpx<R>{v.y, -v.x};
  if (k16 == 8) return {-v.x, -v.y};
  if (k16 == 12) return SIGN > 0 ? cpx<R>{v.y, -v.x} : cpx<R>{-v.y, v.x};
  const int q = k16 & 3, quad = k16 >> 2;
  R c = (R)c16(q), s = (R)c16(4 - q);
  // rotate (c, s) by quad quarter turns
  for (int t = 0; t < quad; ++t) {
    R nc = -s, ns = c;
    c = nc;
    s = ns;
  }
  if (SIGN < 0) s = -s;
  return {v.x * c - v.y * s, v.x * s + v.y * c};
}

// In-register DFT of length N (N = 2, 4, 8, 16) with sign SIGN, radix-2 DIT.
template <typename R, int N, int SIGN>
__host__ __device__ __forceinline__ void dft(cpx<R>* x) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2) {
    cpx<R> a = x[0], b = x[1];
    x[0] = {a.x + b.x, a.y + b.y};
    x[1] = {a.x - b.x, a.y - b.y};
  } else {
    cpx<R> e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    dft<R, N / 2, SIGN>(e);
    dft<R, N / 2, SIGN>(o);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
      cpx<R> t = rot<R, N, SIGN>(o[k], k);
      x[k] = {e[k].x + t.x, e[k].y + t.y};
      x[k + N / 2] = {e[k].x - t.x, e[k].y - t.y};
    }
  }
}

constexpr int ilog2(int m) { return m <= 1 ? 0 : 1 + ilog2(m / 2); }
constexpr int first_radix(int m) { return (ilog2(m) % 4) ? (1 << (ilog2(m) % 4)) : 16; }

// Entries of the two-level twiddle table for a transform of length M.
__host__ __device__ constexpr int tw_hi_count(int m) { return m / 64 > 1 ? m / 64 : 1; }
__host__ __device__ constexpr int tw_count(int m) { return 64 + tw_hi_count(m); }

// Copies the two-level table from global memory into LDS (all threads; ends
// with a barrier).
template <typename R, int M, int NT>
__device__ __forceinline__ void load_twiddles(cpx<R>* lds, const cpx<R>* __restrict__ tw) {
  for (int i = threadIdx.x; i < tw_count(M); i += NT) lds[i] = tw[i];
  __syncthreads();
}

// LDS position of element i of the FFT buffers: one padding slot after every
// 16 elements, so that the power-of-two strides of the Stockham stages do not
// map all lanes of a wave onto the same banks.
__host__ __device__ constexpr int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded(int n) { return n + (n >> 4); }

template <typename R, int M>
__device__ __forceinline__ cpx<R> twiddle(const cpx<R>* tws, int t) {
  return cmul(tws[t & 63], tws[64 + (t >> 6)]);
}

// Radix-2 butterfly with twiddle t in fused multiply-adds:
// (a, b) <- (a + t b, a - t b), the difference formed as 2a - (a + t b)
// (six instructions instead of a product, a sum and a difference).
template <typename R>
__host__ __device__ __forceinline__ R fmar(R a, R b, R c) {
  if constexpr (sizeof(R) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

template <typename R>
__host__ __device__ __forceinline__ void bfly_tw(cpx<R>& a, cpx<R>& b, cpx<R> t) {
  const cpx<R> p = {fmar(t.x, b.x, fmar(-t.y, b.y, a.x)), fmar(t.x, b.y, fmar(t.y, b.x, a.y))};
  b = {fmar(R(2), a.x, -p.x), fmar(R(2), a.y, -p.y)};
  a = p;
}

// Twiddled DFT of length N (a power of two) in registers:
// x[f] <- sum_r x[r] (u exp(SIGN 2 pi i f / N))^r, the input twiddles u^r of a
// Stockham stage folded into the transform.  Splitting r into even and odd
// gives two twiddled DFTs of length N/2 with twiddle u^2, joined by
// butterflies with t_f = u exp(SIGN 2 pi i f / N) (t_{f + N/4} = t_f i^SIGN),
// so the stage costs log2(N) squarings and a few constant rotations of u
// instead of N - 2 products forming the powers and N - 1 applying them.
template <typename R, int N, int SIGN>
__host__ __device__ __forceinline__ void dft_tw(cpx<R>* x, cpx<R> u) {
  if constexpr (N > 1) {
    cpx<R> e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    if constexpr (N > 2) {
      const cpx<R> u2 = cmul(u, u);
      dft_tw<R, N / 2, SIGN>(e, u2);
      dft_tw<R, N / 2, SIGN>(o, u2);
    }
    cpx<R> t[N / 2];
#pragma unroll
    for (int f = 0; f < N / 2; ++f) {
      if (N == 2 || f < N / 4) {
        t[f] = rot<R, N, SIGN>(u, f);
      } else {
        const cpx<R> v = t[f - N / 4];
        t[f] = SIGN > 0 ? cpx<R>{-v.y, v.x} : cpx<R>{v.y, -v.x};
      }
    }
#pragma unroll
    for (int f = 0; f < N / 2; ++f) {
      bfly_tw(e[f], o[f], t[f]);
      x[f] = e[f];
      x[f + N / 2] = o[f];
    }
  }
}

template <typename R, int RAD, int M, int NB, int NT, int SIGN, int NS>
__device__ __forceinline__ void fft_stage(cpx<R>* buf, const cpx<R>* tw) {
  constexpr int NBF = M / RAD;
  constexpr int TOT = NB * NBF;
  constexpr int PER = (TOT + NT - 1) / NT;
  // padded positions of the stage's strided reads and writes: when the
  // stride is a multiple of 16 the padding adds a constant per step
  constexpr bool RD_LIN = NBF % 16 == 0;
  constexpr bool WR_LIN = NS % 16 == 0;
  cpx<R> y[PER][RAD];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bi = (int)threadIdx.x + q * NT;
    if (TOT % NT == 0 || bi < TOT) {
      const int b = bi / NBF, j = bi - b * NBF;
      const int k = j & (NS - 1);
      cpx<R> x[RAD];
      const int i0 = b * M + j;
#pragma unroll
      for (int r = 0; r < RAD; ++r)
        x[r] = RD_LIN ? buf[pidx(i0) + r * padded(NBF)] : buf[pidx(i0 + r * NBF)];
      if constexpr (NS > 1) {
        cpx<R> w1 = twiddle<R, M>(tw, k * (M / (NS * RAD)));
        if (SIGN < 0) w1.y = -w1.y;
        dft_tw<R, RAD, SIGN>(x, w1);
      } else {
        dft<R, RAD, SIGN>(x);
      }
#pragma unroll
      for (int r = 0; r < RAD; ++r) y[q][r] = x[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bi = (int)threadIdx.x + q * NT;
    if (TOT % NT == 0 || bi < TOT) {
      const int b = bi / NBF, j = bi - b * NBF;
      const int k = j & (NS - 1);
      const int base = b * M + (j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        if (WR_LIN)
          buf[pidx(base) + r * padded(NS)] = y[q][r];
        else
          buf[pidx(base + r * NS)] = y[q][r];
      }
    }
  }
  __syncthreads();
}

template <typename R, int M, int NB, int NT, int SIGN, int NS>
__device__ __forceinline__ void fft_stages(cpx<R>* buf, const cpx<R>* tw) {
  if constexpr (NS < M) {
    constexpr int RAD = (NS == 1) ? first_radix(M) : 16;
    fft_stage<R, RAD, M, NB, NT, SIGN, NS>(buf, tw);
    fft_stages<R, M, NB, NT, SIGN, NS * RAD>(buf, tw);
  }
}

// The last stage (NS * RAD = M), with each output handed to store(b, f, v)
// (f = frequency index of sequence b) from registers instead of written back
// to LDS, for the outputs keep(f) selects (for RAD = 16 and a keep that tests
// ranges of M / 16, decided per r at compile time).  Butterflies j (outputs
// j + r NS) for which need(j) is false are skipped whole.  No barrier at the
// end.
struct AllNeeded {
  __device__ bool operator()(int) const { return true; }
};

template <typename R, int RAD, int M, int NB, int NT, int SIGN, int NS, typename Keep,
          typename Store, typename Need = AllNeeded>
__device__ __forceinline__ void fft_last_stage(const cpx<R>* buf, const cpx<R>* tw, Keep keep,
                                               Store store, Need need = Need{}) {
  static_assert(NS * RAD == M, "last stage");
  constexpr int NBF = M / RAD;  // == NS: j is its own twiddle index
  constexpr int TOT = NB * NBF;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr bool RD_LIN = NBF % 16 == 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int bi = (int)threadIdx.x + q * NT;
    if (TOT % NT == 0 || bi < TOT) {
      const int b = bi / NBF, j = bi - b * NBF;
      if (!need(j)) continue;
      cpx<R> x[RAD];
      const int i0 = b * M + j;
#pragma unroll
      for (int r = 0; r < RAD; ++r)
        x[r] = RD_LIN ? buf[pidx(i0) + r * padded(NBF)] : buf[pidx(i0 + r * NBF)];
      if constexpr (NS > 1) {
        cpx<R> w1 = twiddle<R, M>(tw, j);
        if (SIGN < 0) w1.y = -w1.y;
        dft_tw<R, RAD, SIGN>(x, w1);
      } else {
        dft<R, RAD, SIGN>(x);
      }
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        const int f = r * NS + j;
        if (keep(r, f)) store(b, f, x[r]);
      }
    }
  }
}

template <typename R, int M, int NB, int NT, int SIGN, int NS, typename Keep, typename Store,
          typename Need>
__device__ __forceinline__ void fft_stages_store(cpx<R>* buf, const cpx<R>* tw, Keep keep,
                                                 Store store, Need need) {
  constexpr int RAD = (NS == 1) ? first_radix(M) : 16;
  if constexpr (NS * RAD < M) {
    fft_stage<R, RAD, M, NB, NT, SIGN, NS>(buf, tw);
    fft_stages_store<R, M, NB, NT, SIGN, NS * RAD>(buf, tw, keep, store, need);
  } else {
    fft_last_stage<R, RAD, M, NB, NT, SIGN, NS>(buf, tw, keep, store, need);
  }
}

// FFT of NB sequences in LDS from stage NS on, the last stage's outputs
// stored through store(b, f, v) for keep(r, f), its butterflies j run only
// where need(j) (see fft_last_stage); the LDS contents are left undefined.
template <typename R, int M, int NB, int NT, int SIGN, int NS = 1, typename Keep, typename Store,
          typename Need = AllNeeded>
__device__ __forceinline__ void lds_fft_store(cpx<R>* buf, const cpx<R>* tw, Keep keep,
                                              Store store, Need need = Need{}) {
  fft_stages_store<R, M, NB, NT, SIGN, NS>(buf, tw, keep, store, need);
}

// In-place FFT of NB sequences of length M stored contiguously in LDS, with
// the twiddle table `tw` in LDS (see load_twiddles).  Must be called by all
// NT threads of the block; ends with a barrier.
template <typename R, int M, int NB, int NT, int SIGN>
__device__ __forceinline__ void lds_fft(cpx<R>* buf, const cpx<R>* tw) {
  fft_stages<R, M, NB, NT, SIGN, 1>(buf, tw);
}

}  // namespace pc
