// The extern "C" boundary: argument validation, error capture, dispatch.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

extern "C" pc_status pc_plan_footprint_impl(const pc_geometry* geom, size_t* bytes);
extern "C" pc_status pc_plan_create_impl(const pc_geometry* geom, void* stream, pc_plan** out);
extern "C" pc_status pc_device_pool_trim_impl(int32_t device, size_t* released);

namespace pc {

static thread_local std::string g_last_error = "no error";

void set_last_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(pc_status s, const std::string& msg) { throw Error(s, msg); }

template <typename F>
static pc_status guard(const char* fn, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(std::string(fn) + ": " + e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error(std::string(fn) + ": host allocation failed");
    return PC_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_last_error(std::string(fn) + ": " + e.what());
    return PC_ERR_DEVICE;
  } catch (...) {
    set_last_error(std::string(fn) + ": unknown failure");
    return PC_ERR_DEVICE;
  }
}

static void check_plan(const pc_plan* p, int precision) {
  PC_REQUIRE(p != nullptr, "plan is NULL");
  if (p->precision != precision)
    fail(PC_ERR_INVALID_ARG, precision == PC_PREC_FP64
                                 ? "this entry point needs a plan created with PC_PREC_FP64"
                                 : "this entry point needs a plan created with PC_PREC_FP32");
}

static void check_atoms(const pc_plan* p, int64_t natoms, const void* pix, const void* weight,
                        bool need_weight) {
  PC_REQUIRE(natoms >= 0, "natoms must be >= 0");
  PC_REQUIRE(natoms <= (int64_t)p->g.n * p->g.n, "natoms exceeds npix^2");
  if (natoms > 0) {
    PC_REQUIRE(pix != nullptr, "pix is NULL");
    if (need_weight) PC_REQUIRE(weight != nullptr, "weight is NULL");
  }
}

static void set_device(const pc_plan* p) { PC_HIP(hipSetDevice(p->device)); }

// Marks the end of an entry point's work on its stream (plan_touch) when the
// entry point returns, so that pc_plan_destroy can wait for it alone.
struct Touch {
  pc_plan* p;
  hipStream_t s;
  Touch(pc_plan* plan, void* stream) : p(plan), s((hipStream_t)stream) {}
  ~Touch() {
    try {
      plan_touch(p, s);
    } catch (...) {
    }
  }
};

// Launch tables of pc_adjoint_grid_batch, per device (calls are serialised).
constexpr int kMaxDevices = 64;
static std::mutex g_batch_mutex;
static BatchCtx g_batch_ctx[kMaxDevices];

}  // namespace pc

using namespace pc;

extern "C" {

const char* pc_last_error(void) { return g_last_error.c_str(); }

pc_status pc_plan_footprint(const pc_geometry* geom, size_t* bytes) {
  return guard("pc_plan_footprint", [&] { return pc_plan_footprint_impl(geom, bytes); });
}

pc_status pc_plan_create(const pc_geometry* geom, void* stream, pc_plan** out) {
  return guard("pc_plan_create", [&] { return pc_plan_create_impl(geom, stream, out); });
}

pc_status pc_device_pool_trim(int32_t device, size_t* released) {
  return guard("pc_device_pool_trim", [&] {
    PC_REQUIRE(device >= 0, "device must be >= 0");
    int cur = 0;
    PC_HIP(hipGetDevice(&cur));
    PC_HIP(hipSetDevice(device));
    const pc_status st = pc_device_pool_trim_impl(device, released);
    PC_HIP(hipSetDevice(cur));
    return st;
  });
}

void pc_plan_destroy(pc_plan* plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->device);
  plan_release(plan);  // waits for the plan's own recorded work, not the device
  delete plan;
}

pc_status pc_plan_get_info(const pc_plan* p, pc_plan_info* info) {
  return guard("pc_plan_get_info", [&] {
    PC_REQUIRE(p != nullptr && info != nullptr, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->nvis = p->L;
    info->npix = p->g.n;
    info->fine = p->g.M;
    info->kernel_width = p->g.W;
    info->kernel_beta = p->g.beta64;
    info->band_u0 = p->g.u0;
    info->band_nu = p->g.nu;
    info->band_v0 = p->g.v0;
    info->band_nv = p->g.nv;
    info->wraps = p->g.wrap;
    info->tile = kTile;
    info->n_tiles = (int64_t)p->g.ntu * p->g.ntv;
    info->n_chunks = p->n_chunks;
    info->n_partials = p->n_partials;
    info->footprint = p->footprint;
    info->precision = p->precision;
    info->w_planes = p->ws.nplanes;
    info->w_first = p->ws.w0;
    info->w_step = p->ws.dw;
    return PC_OK;
  });
}

pc_status pc_adjoint_grid(pc_plan* p, const void* vis, float* image, double* max_abs,
                          int64_t* argmax, void* stream) {
  return guard("pc_adjoint_grid", [&] {
    check_plan(p, PC_PREC_FP32);
    PC_REQUIRE(vis != nullptr && image != nullptr, "vis and image must not be NULL");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    adjoint_grid<float>(p, (const c32*)vis, false, image, 1.0f, s);
    if (max_abs || argmax) maxkey_read(p, s, max_abs, argmax);
    return PC_OK;
  });
}

pc_status pc_adjoint_grid_ms(pc_plan* p, const void* vis, int32_t n_scales, const double* sigma,
                             const double* gamma, float* images, double* max_abs,
                             int64_t* argmax, void* stream) {
  return guard("pc_adjoint_grid_ms", [&] {
    check_plan(p, PC_PREC_FP32);
    PC_REQUIRE(vis != nullptr && images != nullptr, "vis and images must not be NULL");
    const DictSpec D = make_dict(n_scales, sigma, gamma);
    PC_REQUIRE((int64_t)D.S * p->g.n * p->g.n < ((int64_t)1 << 31),
               "n_scales * npix^2 must be < 2^31");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    // Phi* vis into a plan-owned image (every scale reads all of it), then
    // Psi* into images
    float* eta = ensure_image_scratch(p);
    adjoint_grid<float>(p, (const c32*)vis, false, eta, 1.0f, s);
    dict_analysis(p, D, eta, images, false, p->maxkey, s);
    if (max_abs || argmax) maxkey_read(p, s, max_abs, argmax);
    return PC_OK;
  });
}

pc_status pc_adjoint_grid_f64(pc_plan* p, const void* vis, double* image, double* max_abs,
                              int64_t* argmax, void* stream) {
  return guard("pc_adjoint_grid_f64", [&] {
    check_plan(p, PC_PREC_FP64);
    PC_REQUIRE(vis != nullptr && image != nullptr, "vis and image must not be NULL");
    if (p->g.M > 8192) fail(PC_ERR_UNSUPPORTED, "FP64 twin supports fine grids up to 8192");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    adjoint_grid<double>(p, (const c64*)vis, false, image, 1.0, s);
    if (max_abs || argmax) maxkey_read(p, s, max_abs, argmax);
    return PC_OK;
  });
}

pc_status pc_forward_sparse(pc_plan* p, int64_t natoms, const int32_t* pix, const float* weight,
                            void* vis_out, void* stream) {
  return guard("pc_forward_sparse", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis_out != nullptr, "vis_out is NULL");
    set_device(p);
    Touch touch(p, stream);
    forward_sparse<float>(p, natoms, pix, weight, nullptr, false, (c32*)vis_out, false,
                          (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_forward_sparse_f64(pc_plan* p, int64_t natoms, const int32_t* pix,
                                const double* weight, void* vis_out, void* stream) {
  return guard("pc_forward_sparse_f64", [&] {
    check_plan(p, PC_PREC_FP64);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis_out != nullptr, "vis_out is NULL");
    set_device(p);
    Touch touch(p, stream);
    forward_sparse<double>(p, natoms, pix, weight, nullptr, false, (c64*)vis_out, false,
                           (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_adjoint_sparse_f64(pc_plan* p, const void* vis, int64_t natoms, const int32_t* pix,
                                double* out, void* stream) {
  return guard("pc_adjoint_sparse_f64", [&] {
    check_plan(p, PC_PREC_FP64);
    check_atoms(p, natoms, pix, nullptr, false);
    PC_REQUIRE(vis != nullptr, "vis is NULL");
    if (natoms > 0) PC_REQUIRE(out != nullptr, "out is NULL");
    set_device(p);
    Touch touch(p, stream);
    adjoint_sparse<double>(p, (const c64*)vis, false, natoms, pix, out, (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_dual_certificate_f64(pc_plan* p, const void* vis, int64_t natoms, const int32_t* pix,
                                  const double* weight, double lambda, double* cert,
                                  double* max_abs, int64_t* argmax, void* stream) {
  return guard("pc_dual_certificate_f64", [&] {
    check_plan(p, PC_PREC_FP64);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis != nullptr && cert != nullptr, "vis and cert must not be NULL");
    PC_REQUIRE(std::isfinite(lambda) && lambda > 0, "lambda must be finite and > 0");
    if (p->g.M > 8192) fail(PC_ERR_UNSUPPORTED, "FP64 twin supports fine grids up to 8192");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    c64* r = (c64*)p->vis_scratch;
    forward_sparse<double>(p, natoms, pix, weight, (const c64*)vis, false, r, true, s);
    adjoint_grid<double>(p, r, true, cert, 1.0 / lambda, s);
    if (max_abs || argmax) maxkey_read(p, s, max_abs, argmax);
    return PC_OK;
  });
}

pc_status pc_adjoint_grid_batch(pc_plan* const* plans, const void* const* vis,
                                float* const* images, int32_t njobs, double* max_abs,
                                int64_t* argmax, void* stream) {
  return guard("pc_adjoint_grid_batch", [&] {
    PC_REQUIRE(njobs >= 0, "njobs must be >= 0");
    if (njobs == 0) return PC_OK;
    PC_REQUIRE(plans && vis && images, "NULL argument");
    int dev = -1;
    PC_HIP(hipGetDevice(&dev));
    for (int j = 0; j < njobs; ++j) {
      check_plan(plans[j], PC_PREC_FP32);
      PC_REQUIRE(vis[j] != nullptr && images[j] != nullptr, "vis and image must not be NULL");
      PC_REQUIRE(plans[j]->device == dev, "every plan must live on the current device");
      for (int i = 0; i < j; ++i) PC_REQUIRE(plans[i] != plans[j], "a plan appears twice");
    }
    PC_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index");
    std::lock_guard<std::mutex> lk(g_batch_mutex);
    std::unique_ptr<bool[]> sorted(new bool[njobs]);
    for (int j = 0; j < njobs; ++j) sorted[j] = false;
    hipStream_t s = (hipStream_t)stream;
    adjoint_grid_batch(g_batch_ctx[dev], plans, (const c32* const*)vis, sorted.get(), images,
                       nullptr, njobs, s);
    for (int j = 0; j < njobs; ++j) plan_touch(plans[j], s);
    if (max_abs || argmax) {
      for (int j = 0; j < njobs; ++j)
        maxkey_read(plans[j], s, max_abs ? max_abs + j : nullptr, argmax ? argmax + j : nullptr);
    }
    return PC_OK;
  });
}

pc_status pc_forward_grid(pc_plan* p, const float* image, void* vis_out, void* stream) {
  return guard("pc_forward_grid", [&] {
    check_plan(p, PC_PREC_FP32);
    PC_REQUIRE(image != nullptr && vis_out != nullptr, "image and vis_out must not be NULL");
    set_device(p);
    Touch touch(p, stream);
    forward_grid<float>(p, image, (c32*)vis_out, false, (hipStream_t)stream);
    return PC_OK;
  });
}

// Copies a caller's host row mask into the plan (on the stream) and counts
// its rows; bits past npix must be clear.
static RowMask upload_rows(pc_plan* p, const uint32_t* row_mask, hipStream_t s) {
  PC_REQUIRE(row_mask != nullptr, "row_mask is NULL");
  const int n = p->g.n, words = (n + 31) / 32;
  int64_t count = 0;
  for (int w = 0; w < words; ++w) {
    const uint32_t m = row_mask[w];
    if (w == words - 1 && n % 32) PC_REQUIRE((m >> (n % 32)) == 0, "row_mask has bits past npix");
    count += __builtin_popcount(m);
  }
  PC_HIP(hipMemcpyAsync(p->rowmask, row_mask, (size_t)words * 4, hipMemcpyHostToDevice, s));
  PC_HIP(hipStreamSynchronize(s));  // the caller's array may go away on return
  return RowMask{p->rowmask, count};
}

pc_status pc_forward_grid_rows(pc_plan* p, const float* image, const uint32_t* row_mask,
                               void* vis_out, void* stream) {
  return guard("pc_forward_grid_rows", [&] {
    check_plan(p, PC_PREC_FP32);
    PC_REQUIRE(image != nullptr && vis_out != nullptr, "image and vis_out must not be NULL");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    const RowMask rows = upload_rows(p, row_mask, s);
    forward_grid<float>(p, image, (c32*)vis_out, false, s, rows.count ? &rows : nullptr);
    return PC_OK;
  });
}

pc_status pc_adjoint_grid_rows(pc_plan* p, const void* vis, const uint32_t* row_mask,
                               float* image, void* stream) {
  return guard("pc_adjoint_grid_rows", [&] {
    check_plan(p, PC_PREC_FP32);
    PC_REQUIRE(vis != nullptr && image != nullptr, "vis and image must not be NULL");
    if (p->Cw) fail(PC_ERR_UNSUPPORTED, "row-restricted adjoint of a non-coplanar plan");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    const RowMask rows = upload_rows(p, row_mask, s);
    if (rows.count) adjoint_grid<float>(p, (const c32*)vis, false, image, 1.0f, s, &rows);
    return PC_OK;
  });
}

pc_status pc_restricted_gradient_grid(pc_plan* p, const void* vis, int64_t natoms,
                                      const int32_t* pix, const float* weight, double* grad,
                                      void* resid, void* stream) {
  return guard("pc_restricted_gradient_grid", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis != nullptr, "vis is NULL");
    if (natoms > 0) PC_REQUIRE(grad != nullptr, "grad is NULL");
    PC_REQUIRE(resid == nullptr || resid != vis, "resid must not alias vis");
    if (p->Cw) fail(PC_ERR_UNSUPPORTED, "gridded restricted gradient of a non-coplanar plan");
    set_device(p);
    Touch touch(p, stream);
    restricted_gradient_grid(p, (const c32*)vis, natoms, pix, weight, grad, (c32*)resid,
                             (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_adjoint_sparse(pc_plan* p, const void* vis, int64_t natoms, const int32_t* pix,
                            double* out, void* stream) {
  return guard("pc_adjoint_sparse", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, nullptr, false);
    PC_REQUIRE(vis != nullptr, "vis is NULL");
    if (natoms > 0) PC_REQUIRE(out != nullptr, "out is NULL");
    set_device(p);
    Touch touch(p, stream);
    adjoint_sparse<float>(p, (const c32*)vis, false, natoms, pix, out, (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_restricted_gradient(pc_plan* p, const void* vis, int64_t natoms, const int32_t* pix,
                                 const float* weight, double* grad, void* resid, void* stream) {
  return guard("pc_restricted_gradient", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis != nullptr, "vis is NULL");
    if (natoms > 0) PC_REQUIRE(grad != nullptr, "grad is NULL");
    PC_REQUIRE(resid == nullptr || resid != vis, "resid must not alias vis");
    set_device(p);
    Touch touch(p, stream);
    restricted_gradient(p, (const c32*)vis, natoms, pix, weight, grad, (c32*)resid,
                        (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_restricted_gradient_noalloc(pc_plan* p, const void* vis, int64_t natoms,
                                         const int32_t* pix, const float* weight, double* grad,
                                         void* resid, void* stream) {
  return guard("pc_restricted_gradient_noalloc", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis != nullptr, "vis is NULL");
    if (natoms > 0) PC_REQUIRE(grad != nullptr, "grad is NULL");
    PC_REQUIRE(resid == nullptr || resid != vis, "resid must not alias vis");
    set_device(p);
    restricted_gradient_noalloc(p, (const c32*)vis, natoms, pix, weight, grad, (c32*)resid,
                                (hipStream_t)stream);
    return PC_OK;
  });
}

pc_status pc_dual_certificate(pc_plan* p, const void* vis, int64_t natoms, const int32_t* pix,
                              const float* weight, double lambda, float* cert, double* max_abs,
                              int64_t* argmax, void* stream) {
  return guard("pc_dual_certificate", [&] {
    check_plan(p, PC_PREC_FP32);
    check_atoms(p, natoms, pix, weight, true);
    PC_REQUIRE(vis != nullptr && cert != nullptr, "vis and cert must not be NULL");
    PC_REQUIRE(std::isfinite(lambda) && lambda > 0, "lambda must be finite and > 0");
    set_device(p);
    Touch touch(p, stream);
    hipStream_t s = (hipStream_t)stream;
    c32* r = (c32*)p->vis_scratch;
    // residual in plan order: r = V - Phi x
    forward_sparse<float>(p, natoms, pix, weight, (const c32*)vis, false, r, true, s);
    adjoint_grid<float>(p, r, true, cert, (float)(1.0 / lambda), s);
    if (max_abs || argmax) maxkey_read(p, s, max_abs, argmax);
    return PC_OK;
  });
}

}  // extern "C"
