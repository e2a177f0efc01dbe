// Launchers of the solver's small kernels (kernels_solver.hip).
#pragma once

#include "common.h"

namespace pc {

// Slots of the solver's FP64 device scalar block (read back together).
enum : int {
  kScalResid = 0,  // [0] ||r||^2, [1] Re<V, r>
  kScalYL1 = 2,    // ||y||_1 at the gradient point of the last APGD step
  kScalGmax = 3,   // max_p |(Phi_S^* r)_p| there (max(0, max_p (.)_p) under positivity)
  kScalYNeg = 4,   // max(0, -min_p y_p): > 0 when y lies outside x >= 0
  kScalCount = 5
};

void k_gather(pc_plan* p, int64_t L, const int32_t* perm, const c32* in, c32* out, hipStream_t s);
int k_resid_blocks(int64_t L);
void k_resid(pc_plan* p, int64_t L, const c32* r, const c32* V, double* partial, double* out, hipStream_t s);
void k_select(pc_plan* p, int64_t N, const float* eta, float tau, bool positive, unsigned* count,
              int32_t* out, int64_t cap, hipStream_t s);
// k_select with tau = (max decoded from *key) - dec formed on the device.
void k_select_from_key(pc_plan* p, int64_t N, const float* eta, const unsigned long long* key,
                       double dec, bool positive, unsigned* count, int32_t* out, int64_t cap,
                       hipStream_t s);
void k_weights(pc_plan* p, int64_t nS, const double* x, Atom<float>* atoms, hipStream_t s);
// One Lanczos step (see lanczos_step_kernel): g = G q_j given; writes alpha_j,
// beta_j into ab and q_{j+1} into row j + 1 of Q.
void k_lanczos_step(pc_plan* p, int64_t nS, int j, int kmax, double* Q, const double* g, double* w,
                    double* ab, hipStream_t s);
void k_scale(pc_plan* p, int64_t N, const float* in, float sc, float* out, hipStream_t s);
// Gram form of the restricted problem (see gram_fista_loop_kernel): APGD
// steps it0 + 1 .. it0 + nsteps in one launch from the momentum state t0,
// with the in-kernel duality-gap test on every kcheck-th step.
void k_gram_fista(pc_plan* p, int64_t nS, const double* G, const double* b, double* x, double* y,
                  double* g, double* stats, double v2, const double* lipd, double t0, int it0,
                  int nsteps, int kcheck, double lam, double tol, bool positive, int* done,
                  hipStream_t s);
// The Gram form's Lanczos estimate with its stopping rule on the device: out =
// {step constant, steps, theta, rho}, ritz = the top Ritz vector.
// The basis and scratch live in LDS (G too for up to ~120 atoms): at most
// kGramLdsAtoms atoms.
constexpr int kGramLdsAtoms = 1024;
void k_gram_lanczos_full(pc_plan* p, int64_t nS, int kmax, double tol, double margin,
                         const double* G, const double* Q, double* ab, double* out, double* ritz,
                         hipStream_t s);
void k_zero_u32(pc_plan* p, int64_t n, unsigned* out, hipStream_t s);
// G, b and the Lanczos start vector from one device block (see
// gram_assemble_kernel) and the per-solve point-spread / b tables.
void k_gram_assemble(pc_plan* p, int64_t nS, const void* blk, const double* psf,
                     const double* bval, double* G, double* b, double* Q0, hipStream_t s);
// Active set from one device block [x: nS doubles][pix: nS int32]: x, y, pix
// and the padded atom table (atom_capacity(nS) entries).
void k_activate(pc_plan* p, int64_t nS, const void* blk, double* x, double* y, int32_t* pix,
                Atom<float>* atoms, hipStream_t s);
void k_rsub(pc_plan* p, int64_t L, const c32* V, c32* r, hipStream_t s);
// Sum in order of nparts (|r|^2, Re<V, r>) partial pairs into out[0..1].
void k_resid_final(pc_plan* p, int nparts, const double* partial, double* out, hipStream_t s);
void k_fill(pc_plan* p, int64_t N, float v, float* out, hipStream_t s);
void k_stat_reduce(pc_plan* p, int64_t nS, const double* stat, double* scal, hipStream_t s);

}  // namespace pc
