// Launchers of the solver's small kernels (kernels_solver.hip).
#pragma once

#include "common.h"

namespace pc {

// Slots of the solver's FP64 device scalar block (read back together).
enum : int {
  kScalResid = 0,  // [0] ||r||^2, [1] Re<V, r>
  kScalYL1 = 2,    // ||y||_1 at the gradient point of the last APGD step
  kScalGmax = 3,   // max_p |(Phi_S^* r)_p| there
  kScalCount = 4
};

void k_gather(pc_plan* p, int64_t L, const int32_t* perm, const c32* in, c32* out, hipStream_t s);
int k_resid_blocks(int64_t L);
void k_resid(pc_plan* p, int64_t L, const c32* r, const c32* V, double* partial, double* out, hipStream_t s);
void k_select(pc_plan* p, int64_t N, const float* eta, float tau, unsigned* count, int32_t* out, int64_t cap,
              hipStream_t s);
void k_weights(pc_plan* p, int64_t nS, const double* x, Atom<float>* atoms, hipStream_t s);
void k_scale(pc_plan* p, int64_t N, const float* in, float sc, float* out, hipStream_t s);
// Gridded-operator helpers for large active sets.
void k_scatter(pc_plan* p, int64_t nS, const int32_t* pix, const double* vals, float* img,
               hipStream_t s);
void k_gather_img(pc_plan* p, int64_t nS, const int32_t* pix, const float* img, double* out,
                  hipStream_t s);
void k_rsub(pc_plan* p, int64_t L, const c32* V, c32* r, hipStream_t s);
void k_fill(pc_plan* p, int64_t N, float v, float* out, hipStream_t s);
void k_stat_reduce(pc_plan* p, int64_t nS, const double* stat, double* scal, hipStream_t s);

}  // namespace pc
