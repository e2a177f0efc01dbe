/*
 * polyclean.h -- C ABI of the MI355X (gfx950) PolyCLEAN measurement-operator
 * library (libpolyclean.so).
 *
 * Method: Jarret et al. 2024, "PolyCLEAN: Atomic Optimization for
 * Super-Resolution Imaging and Uncertainty Estimation in Radio
 * Interferometry".  The library computes
 *   - the discrete forward operator Phi (Sect. 2.2, Eq. phi-discrete):
 *       V_k = sum_p x_p / n_p * exp(-j 2 pi (u_k l_p + v_k m_p + w_k (n_p - 1))),
 *   - its adjoint Phi* (Sect. 2.2, Eq. adjoint-phi):
 *       eta[i,j] = Re sum_k h_k / n_ij * exp(+j 2 pi (u_k l_i + v_k m_j + w_k (n_ij - 1))),
 *   - the dual certificate mu = Phi*(V - Phi x) / lambda (Sect. 4.2,
 *     Eq. dual_certif),
 *   - the LASSO solve of Eq. lasso by the Polyatomic Frank-Wolfe algorithm
 *     (Sect. 5.1, Alg. 2) with an APGD restricted step,
 * The factor exp(-j 2 pi w (n - 1)) is the w-term of Sect. 2.1 (Eq.
 * phi-plane); with w = 0 (coplanar arrays, or w not given) it is 1.
 *
 * Non-coplanar plans (some w != 0): the direct sums (pc_forward_sparse,
 * pc_adjoint_sparse, pc_restricted_gradient*) add the w phase in FP64; the
 * gridded adjoint (pc_adjoint_grid, pc_dual_certificate, the solve's
 * exploration) is w-stacked: planes w_j = w0 + j dw, dw = 1 / (2 |c_min|)
 * (c_min = n - 1 at the image corner), ceil((max |w| - min |w|) / dw) + W + 1
 * planes (a visibility with w < 0 is gridded as its conjugate at (-u, -v,
 * -w)), each one spread and two FFT passes, so its cost is that many
 * coplanar adjoints.  FP32 plans only; pc_forward_grid, the FP64 twin and
 * the synthesis dictionary need coplanar plans (PC_ERR_UNSUPPORTED).
 *
 * Conventions shared by every entry point
 *   Geometry   (u, v, w) in wavelengths (Sect. 2.1; metres are converted with the
 *              frequency).  Pixel step dl = fov / npix; l_i = (i - npix/2) dl,
 *              m_j = (j - npix/2) dl, so pixel (npix/2, npix/2) is the phase
 *              centre; n_ij = sqrt(1 - l_i^2 - m_j^2).
 *   Images     row-major float [npix][npix]; flat index p = i*npix + j with i
 *              the l (u) axis and j the m (v) axis.
 *   Vis.       interleaved complex (re, im) in the CALLER's order, one
 *              Hermitian half; float pairs (complex64) for FP32 plans, double
 *              pairs (complex128) for the FP64 entry points.
 *   Memory     every buffer argument marked "dev" is device memory on the
 *              plan's GPU; "host" is ordinary host memory.  The caller owns all
 *              input and output buffers; the library never frees them.  The
 *              plan owns its workspace: pc_plan_create allocates what
 *              pc_plan_footprint reports; per-call scratch that depends on the
 *              request (atom tables and partial sums of the direct sums, sized
 *              by the number of atoms; the dirty-image buffer and per-scale
 *              keys of pc_adjoint_grid_ms; the row and atom tables of
 *              pc_restricted_gradient_grid) is added on first use and kept,
 *              and pc_plan_get_info's `footprint` is the total held at the
 *              time.  pc_restricted_gradient_noalloc adds none.
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = the null
 *              stream).  Calls are asynchronous on it, except that any host
 *              scalar output (max_abs, argmax, solve results) synchronises the
 *              stream before returning.  A plan must not be used from two host
 *              threads at once.
 *   Errors     every function returns a pc_status.  Argument errors are
 *              detected on the host before any device work; no C++ exception
 *              crosses the ABI.  pc_last_error() returns a thread-local
 *              message describing the last failure on the calling thread.
 */
#ifndef POLYCLEAN_H
#define POLYCLEAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Symbols are exported from the shared library; nothing else is. */
#if defined(PC_BUILD)
#define PC_API __attribute__((visibility("default")))
#else
#define PC_API
#endif

typedef enum {
  PC_OK = 0,
  PC_WARN_NOT_CONVERGED = 1, /* solve hit max_iter; the result is filled in */
  PC_ERR_INVALID_ARG = -1,   /* a NULL pointer, a bad size or a bad value   */
  PC_ERR_OUT_OF_MEMORY = -2, /* device allocation failed                    */
  PC_ERR_DEVICE = -3,        /* a HIP runtime call or kernel launch failed  */
  PC_ERR_CAPACITY = -4,      /* an output array is too small (see result)   */
  PC_ERR_UNSUPPORTED = -5    /* a valid request the library does not handle */
} pc_status;

enum { PC_UV_WAVELENGTHS = 0, PC_UV_METRES = 1 };
enum { PC_PREC_FP32 = 0, PC_PREC_FP64 = 1 };

typedef struct pc_plan pc_plan;

/* Imaging geometry (Sect. 2.1-2.2).  All pointers are host memory and are
 * only read during pc_plan_create / pc_plan_footprint. */
typedef struct {
  int64_t nvis;          /* L > 0: number of visibilities                     */
  const double* u;       /* [nvis] baseline u (units below)                   */
  const double* v;       /* [nvis] baseline v                                 */
  const double* w;       /* [nvis] or NULL (NULL or all zero: coplanar)       */
  int32_t uv_units;      /* PC_UV_WAVELENGTHS or PC_UV_METRES                 */
  double freq_hz;        /* observing frequency; used only for PC_UV_METRES   */
  int32_t npix;          /* n: image side, even, 16 <= n <= 8192              */
  double fov_rad;        /* field of view (side) in radians, > 0              */
  double nufft_eps;      /* requested gridding accuracy; <= 0 selects 1e-5    */
  double upsamp;         /* fine-grid upsampling sigma; <= 0 selects 2; only 2 */
  int32_t precision;     /* PC_PREC_FP32, or PC_PREC_FP64 for the FP64 twin   */
} pc_geometry;

/* Read-only facts about a plan (for reporting and byte models). */
typedef struct {
  int64_t nvis;
  int32_t npix;
  int32_t fine;          /* M = sigma * n, fine-grid side                     */
  int32_t kernel_width;  /* w, exponential-of-semicircle kernel support       */
  double kernel_beta;    /* beta of phi(z) = exp(beta (sqrt(1 - z^2) - 1))     */
  int32_t band_u0, band_nu; /* occupied fine-grid band along u (cells)        */
  int32_t band_v0, band_nv; /* occupied fine-grid band along v                */
  int32_t wraps;         /* 1 if the band is the whole (periodic) grid        */
  int32_t tile;          /* spreading tile side in cells                      */
  int64_t n_tiles;       /* tiles in the band                                 */
  int64_t n_chunks;      /* spreading work items                              */
  int64_t n_partials;    /* partial tiles folded for split hot tiles          */
  size_t footprint;      /* device bytes owned by the plan                    */
  int32_t precision;
  int32_t w_planes;      /* planes of the w-stacked adjoint (0: coplanar)     */
  double w_first, w_step;/* first plane's w and the plane spacing (wavelengths) */
} pc_plan_info;

/* Device bytes pc_plan_create would allocate for this geometry (host-only
 * computation, used for admission control).  It needs the uv coordinates
 * because the occupied band and the tile work list depend on them. */
PC_API pc_status pc_plan_footprint(const pc_geometry* geom, size_t* bytes);

/* Build a plan on the current HIP device: validates the geometry, computes
 * the per-visibility phases (FP64), the fine-grid cells and offsets, the tile
 * sort and work list, the kernel correction and FFT twiddle tables, and
 * uploads them.  `stream` orders the uploads.  On success *out owns all of it.
 * Errors: PC_ERR_INVALID_ARG (NULL, nvis <= 0, odd or out-of-range npix,
 * fov <= 0, non-finite u, v or w, a field reaching l^2 + m^2 >= 1),
 * PC_ERR_UNSUPPORTED (upsamp != 2; a nonzero w with PC_PREC_FP64),
 * PC_ERR_OUT_OF_MEMORY, PC_ERR_DEVICE. */
PC_API pc_status pc_plan_create(const pc_geometry* geom, void* stream, pc_plan** out);
/* Release a plan.  Waits (on the host) for the work that the plan's entry
 * points queued, as recorded by an event on each stream they were given, and
 * not for the rest of the device; work queued by
 * pc_restricted_gradient_noalloc is not recorded (it creates no event), so
 * its stream must have been synchronised first.  The plan's device buffers go
 * to a per-device pool that later plans and solvers reuse (by size class; the
 * pool keeps at most an eighth of the device's memory and is emptied when an
 * allocation would otherwise fail), so destroying a plan never waits for the
 * whole device.
 *
 * Footprint: pc_plan_footprint and pc_plan_get_info's footprint count what
 * plan creation allocates (each buffer rounded up to its pool size class).
 * Entry points add per-call scratch on first use and keep it: the atom table
 * (40 bytes per atom), the restricted adjoint's partial sums (at most
 * 8 bytes x atoms x a few hundred) and, for pc_adjoint_grid_ms, one npix^2
 * float image; info.footprint then reports the larger total. */
PC_API void pc_plan_destroy(pc_plan* plan);
PC_API pc_status pc_plan_get_info(const pc_plan* plan, pc_plan_info* info);

/* Frees every buffer parked in the device pool of `device` (see
 * pc_plan_destroy), for callers that need the memory elsewhere (another
 * allocator in the process).  hipFree waits for the device.  *released (may
 * be NULL) gets the bytes freed.  Errors: PC_ERR_INVALID_ARG (device < 0),
 * PC_ERR_DEVICE. */
PC_API pc_status pc_device_pool_trim(int32_t device, size_t* released);

/* Per-kernel instrumentation.  While enabled, every kernel the plan launches
 * (operators and solver) is bracketed by HIP events on its stream, and
 * launches, device milliseconds, algorithmic bytes (the minimum data each
 * launch must move) and work units (visibility-atom pairs for the direct
 * DFTs, visibilities for gridding, FFT points for the passes) are summed per
 * kernel name.  Enabling or disabling resets the sums.  Reading a statistic
 * synchronises the device. */
typedef struct {
  char name[48];
  int64_t launches;
  double ms;
  double bytes;
  double work;
} pc_kernel_stat;
PC_API pc_status pc_plan_profile(pc_plan* plan, int32_t enable);
PC_API int32_t pc_plan_kernel_stat_count(pc_plan* plan);
PC_API pc_status pc_plan_kernel_stat(pc_plan* plan, int32_t index, pc_kernel_stat* out);

/* Thread-local description of the last failure (never NULL). */
PC_API const char* pc_last_error(void);

/* ---------------------------------------------------------------------------
 * Operators (FP32 plans)
 * ------------------------------------------------------------------------- */

/* Adjoint Phi* (Eq. adjoint-phi): the full-grid image of `vis`.
 * vis     dev complex64 [nvis], caller order.
 * image   dev float [npix*npix], written entirely.
 * max_abs host double or NULL: max |image|.
 * argmax  host int64 or NULL: lowest flat index attaining max |image|.
 * Method: exponential-of-semicircle gridding on a 2x fine grid, a pruned 2-D
 * inverse FFT and apodisation plus 1/n correction (a type-1 non-uniform FFT,
 * Sect. 5.2).  Relative L2 error against the exact sum ~ nufft_eps. */
PC_API pc_status pc_adjoint_grid(pc_plan* plan, const void* vis, float* image,
                          double* max_abs, int64_t* argmax, void* stream);

/* Forward Phi (Eq. phi-discrete) of a sparse image by direct summation.
 * pix     dev int32 [natoms], flat pixel indices in [0, npix^2).
 * weight  dev float [natoms], pixel values (Jy/pixel).
 * vis_out dev complex64 [nvis], caller order, overwritten.
 * natoms == 0 writes zeros.  Phases are formed and range-reduced in FP64,
 * sin/cos and accumulation are FP32. */
PC_API pc_status pc_forward_sparse(pc_plan* plan, int64_t natoms, const int32_t* pix,
                            const float* weight, void* vis_out, void* stream);

/* Forward Phi of a dense image by interpolation (a type-2 non-uniform FFT,
 * Sect. 5.2): apodisation pre-correction, zero-padded 2-D FFT, gridding-kernel
 * interpolation.  image dev float [npix*npix]; vis_out as above. */
PC_API pc_status pc_forward_grid(pc_plan* plan, const float* image, void* vis_out, void* stream);

/* Row-restricted gridded operators, the gridded form of the restricted
 * operators Phi_S and Phi_S* of the APGD step (Alg. 2 step 2; Sect. 5.2) for
 * an active set S whose atoms lie on the image rows a mask selects: only the
 * transforms of those rows run (their cost scales with the number of rows).
 * row_mask  host uint32 [ceil(npix/32)], bit i % 32 of word i / 32 set for
 *           image row i (pixel index i npix + j); bits past npix must be
 *           clear (-1).  Copied into the plan before the call returns.
 * pc_forward_grid_rows: pc_forward_grid of an image whose rows with a clear
 *   bit are zero (they are not read); the result equals pc_forward_grid's.
 * pc_adjoint_grid_rows: the rows of Phi* vis with a set bit, equal to those
 *   of pc_adjoint_grid's image; the other rows of image are left unchanged,
 *   and no maximum is formed.  An empty mask does nothing.  Coplanar plans
 *   only (-5 for a non-coplanar plan). */
PC_API pc_status pc_forward_grid_rows(pc_plan* plan, const float* image, const uint32_t* row_mask,
                                      void* vis_out, void* stream);
PC_API pc_status pc_adjoint_grid_rows(pc_plan* plan, const void* vis, const uint32_t* row_mask,
                                      float* image, void* stream);

/* The same gradient Phi_S* (V - Phi_S x) by the gridded operators, the form
 * the solve's APGD step takes for large sets (Alg. 2 step 2; Sect. 5.2):
 * interpolation from the fine grid, pass A of the FFT over the band rows,
 * and pass B evaluated directly at the image rows and pixels of S (a row
 * holds few atoms), so the cost is about one gridded operator pair
 * whatever the set's size.  Arguments as pc_restricted_gradient (atoms in
 * any order, repeats allowed); accuracy that of the gridded operators
 * (relative error ~ nufft_eps).  Coplanar plans only (-5 otherwise).  Reads
 * pix back to the host and synchronises the stream before returning. */
PC_API pc_status pc_restricted_gradient_grid(pc_plan* plan, const void* vis, int64_t natoms,
                                             const int32_t* pix, const float* weight,
                                             double* grad, void* resid, void* stream);

/* Restricted adjoint Phi_S* (Eq. adjoint-phi at the pixels of S only), by
 * direct summation: out[p] = Re sum_k vis_k exp(+j2pi(u_k l_p + v_k m_p)) / n_p.
 * vis dev complex64 [nvis] caller order; pix dev int32 [natoms];
 * out dev double [natoms]. */
PC_API pc_status pc_adjoint_sparse(pc_plan* plan, const void* vis, int64_t natoms,
                            const int32_t* pix, double* out, void* stream);

/* Gradient of the data term on the active set, the step that each APGD
 * iteration of the restricted solve takes (Alg. 2, step 2):
 *   r = V - Phi_S x,  grad[p] = Re sum_k r_k exp(+j2pi(u_k l_p + v_k m_p)) / n_p,
 * i.e. Phi_S* (V - Phi_S x), by direct summation.  Up to 64 atoms, one pass
 * evaluates each visibility-atom phase once for both operators; larger sets
 * take pc_forward_sparse then pc_adjoint_sparse.
 * vis dev complex64 [nvis] caller order; pix dev int32 [natoms]; weight dev
 * float [natoms] (the amplitudes x_p); grad dev double [natoms]; resid dev
 * complex64 [nvis] caller order or NULL (not returned; must not alias vis).
 * natoms = 0 gives r = V and no gradient. */
PC_API pc_status pc_restricted_gradient(pc_plan* plan, const void* vis, int64_t natoms,
                                        const int32_t* pix, const float* weight, double* grad,
                                        void* resid, void* stream);

/* pc_restricted_gradient for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and bit-identical results, but the
 * atom table and the partial sums live in a fixed device array of 8 MiB per
 * GPU (held from the first call on that GPU until the process ends) instead
 * of plan scratch grown on demand.  The call makes no device allocation.
 * Limit: 32 B per atom (rounded up to 8 atoms) plus 8 B per atom and
 * partial-sum slot (a few hundred slots per atom at most) must fit the 8 MiB;
 * larger requests return PC_ERR_UNSUPPORTED with the size needed.  Every call
 * on one GPU shares that array, so calls that overlap on one GPU (other
 * streams, other threads) race; serialise them.  The plan's instrumentation
 * (pc_plan_profile) must be off: PC_ERR_INVALID_ARG otherwise. */
PC_API pc_status pc_restricted_gradient_noalloc(pc_plan* plan, const void* vis, int64_t natoms,
                                                const int32_t* pix, const float* weight,
                                                double* grad, void* resid, void* stream);

/* Dual certificate mu = Phi*(V - Phi x) / lambda (Eq. dual_certif) of the
 * sparse image x = (pix, weight).  vis dev complex64 [nvis] caller order;
 * cert dev float [npix*npix]; lambda > 0; max_abs/argmax as for
 * pc_adjoint_grid (of mu). */
PC_API pc_status pc_dual_certificate(pc_plan* plan, const void* vis, int64_t natoms,
                              const int32_t* pix, const float* weight, double lambda,
                              float* cert, double* max_abs, int64_t* argmax,
                              void* stream);

/* ---------------------------------------------------------------------------
 * FP64 twin (plans created with precision = PC_PREC_FP64): the same
 * algorithms entirely in double, for per-stage error reports.
 * vis complex128, images double.  PC_ERR_UNSUPPORTED for fine grids larger
 * than 8192 (the double row no longer fits in one workgroup's LDS).
 * ------------------------------------------------------------------------- */
PC_API pc_status pc_adjoint_grid_f64(pc_plan* plan, const void* vis, double* image,
                              double* max_abs, int64_t* argmax, void* stream);
PC_API pc_status pc_forward_sparse_f64(pc_plan* plan, int64_t natoms, const int32_t* pix,
                                const double* weight, void* vis_out, void* stream);
/* Restricted adjoint in double: vis complex128 [nvis] caller order,
 * out double [natoms]. */
PC_API pc_status pc_adjoint_sparse_f64(pc_plan* plan, const void* vis, int64_t natoms,
                                       const int32_t* pix, double* out, void* stream);
/* Dual certificate in double: vis complex128, weight double, cert double. */
PC_API pc_status pc_dual_certificate_f64(pc_plan* plan, const void* vis, int64_t natoms,
                                         const int32_t* pix, const double* weight,
                                         double lambda, double* cert, double* max_abs,
                                         int64_t* argmax, void* stream);

/* ---------------------------------------------------------------------------
 * Batched gridded adjoint: pc_adjoint_grid for njobs FP32 plans of any sizes
 * on the current device in shared launches (one spreading launch, one fold,
 * one launch per fine-grid size for each FFT pass).  plans, vis, images
 * are host arrays of njobs pointers (vis[j] dev complex64 [nvis_j] caller
 * order, images[j] dev float [npix_j^2]); max_abs / argmax are host arrays
 * of njobs entries or NULL (then the call returns without waiting).  Every
 * image equals that plan's pc_adjoint_grid result bit for bit.  Calls are
 * serialised within the process; a plan must not appear twice in one call.
 * ------------------------------------------------------------------------- */
PC_API pc_status pc_adjoint_grid_batch(pc_plan* const* plans, const void* const* vis,
                                       float* const* images, int32_t njobs, double* max_abs,
                                       int64_t* argmax, void* stream);

/* ---------------------------------------------------------------------------
 * Adjoint of the synthesis form (Sect. 4.3, Eq. lasso-synthesis): images =
 * Psi* Phi* vis for the Gaussian dictionary described at pc_solve_params
 * (n_scales in [1, 8], sigma / gamma host arrays of n_scales doubles).
 * vis: dev complex64 [nvis] caller order; images: dev float
 * [n_scales][npix][npix].  max_abs / argmax (host, or NULL): max over all
 * scales and pixels and the lowest flat index s npix^2 + p attaining it.
 * FP32 plans.  Returns PC_ERR_INVALID_ARG for bad scales.
 * ------------------------------------------------------------------------- */
PC_API pc_status pc_adjoint_grid_ms(pc_plan* plan, const void* vis, int32_t n_scales,
                                    const double* sigma, const double* gamma, float* images,
                                    double* max_abs, int64_t* argmax, void* stream);

/* ---------------------------------------------------------------------------
 * PolyCLEAN solve (Alg. 2)
 * ------------------------------------------------------------------------- */
typedef struct {
  double lambda;          /* > 0: absolute lambda; else alpha * lambda_max    */
  double alpha;           /* lambda = alpha * ||Phi* V||_inf (Eqs. lmax, lambda) */
  double delta;           /* PFW quality in (0, 1] (Alg. 2)                   */
  int32_t max_iter;       /* FW iterations cap (>= 1)                         */
  double rel_obj_tol;     /* stop on relative objective improvement; <= 0 off */
  double rel_gap_tol;     /* stop on relative duality gap; <= 0 off           */
  double inner_tol0;      /* APGD stops when the restricted problem's relative */
  double inner_tol_min;   /*   duality gap <= max(inner_tol_min, inner_tol0 g), */
                          /*   g = the full problem's relative gap at x_k     */
  int32_t inner_max_iter; /* APGD iteration cap per FW iteration              */
  int32_t positivity;     /* 1: x >= 0 (positivity remarks, Sects. 4.1, 5.1): */
                          /*   lambda_max = max(0, max Phi* V), candidates    */
                          /*   only where eta >= tau and eta > 0, the prox    */
                          /*   max(0, z - t), the dual point scaled by the    */
                          /*   largest positive correlation; cert_max is then */
                          /*   max mu (mu may go below -1)                    */
  int32_t want_certificate; /* 1: write mu to result->cert                    */
  int32_t log_every;      /* > 0: print an iteration log line every n iters   */
  int32_t grid_atoms;     /* active-set size from which the APGD step applies */
                          /*   Phi_S and Phi_S* through the gridded operators */
                          /*   (type 2 / type 1, Sect. 5.2) instead of direct */
                          /*   sums: 0 = the built-in cost crossover, < 0 =   */
                          /*   never.  The per-iteration residual and gap use */
                          /*   the gridded forward from 4x that size.         */
  int32_t gram_atoms;     /* direct active sets up to this size solve the     */
                          /*   restricted problem in Gram form: the exact     */
                          /*   G = Re(Phi_S^H Phi_S) (direct sums at pixel    */
                          /*   offsets) and b = Phi_S* V replace the two      */
                          /*   operators in each APGD and Lanczos step: 0 =   */
                          /*   256, < 0 = never, at most 1024.                */
  int32_t n_scales;       /* 0: point atoms (Eq. lasso).  1..8: the synthesis */
                          /*   form (Sect. 4.3, Eq. lasso-synthesis) over the */
                          /*   Gaussian dictionary of Sect. 6.4: element s is */
                          /*   gamma_s g~_s, g~_s[a,b] ~ exp(-(a^2+b^2)/      */
                          /*   sigma_s^2) for |a|,|b| <= floor(2 sigma_s),    */
                          /*   unit l1 norm (sigma_s = 0: one pixel), cropped */
                          /*   at the image border.  Atoms are s npix^2 + p;  */
                          /*   lambda_max = ||Psi* Phi* V||_inf; result->cert */
                          /*   then holds n_scales npix^2 floats (Psi* eta /  */
                          /*   lambda).  The restricted problem always runs   */
                          /*   through the gridded operators.                 */
  double scale_sigma[8];  /* sigma_s in pixels, in [0, 16] (paper: 0, 2, 5, 8) */
  double scale_gamma[8];  /* gamma_s > 0 (paper: 1.2^s)                       */
  const int32_t* x0_pix;  /* warm start (host, read during pc_polyclean_solve / */
  const double* x0_w;     /*   pc_solver_create only): x0_n distinct atoms    */
  int64_t x0_n;           /*   (pixels, or s npix^2 + p) and finite weights   */
                          /*   (>= 0 under positivity); the solve continues   */
                          /*   from this x as its previous iterate (no FW     */
                          /*   iteration if x0 already meets rel_gap_tol).    */
                          /*   lambda_max and lambda still come from the      */
                          /*   data.  x0_n = 0: none                          */
} pc_solve_params;

typedef struct {
  int64_t capacity;       /* in: length of pix/weight                         */
  int32_t* pix;           /* in: host int32 [capacity]; out: active atoms     */
                          /*   (pixels, or s npix^2 + p with a dictionary)    */
  double* weight;         /* in: host double [capacity]; out: their weights   */
  float* cert;            /* in: dev float [npix^2] or NULL                   */
  int64_t natoms;         /* out: atoms in the solution (required if CAPACITY) */
  double objective;       /* out: 1/2 ||V - Phi x||^2 + lambda ||x||_1         */
  double rel_gap;         /* out: relative duality gap at the returned x      */
  double lambda;          /* out: lambda used                                 */
  double lambda_max;      /* out: ||Phi* V||_inf (positivity: max(0, max))    */
  double cert_max;        /* out: ||mu||_inf (positivity: max(0, max mu))     */
  int64_t cert_argmax;    /* out: lowest flat index attaining it (s npix^2 + p */
                          /*   with a dictionary)                             */
  int32_t iters;          /* out: FW iterations run                           */
  int32_t inner_iters;    /* out: total APGD iterations                       */
  int32_t converged;      /* out: 1 if a tolerance test stopped the solve     */
  double seconds;         /* out: wall time of the solve                      */
  double adjoint_seconds; /* out: device time in the adjoint operator         */
  int32_t adjoint_calls;  /* out: number of adjoint applications              */
} pc_solve_result;

/* Fill params with the defaults: alpha 0.01, delta 0.99, max_iter 50,
 * tolerances off, inner_tol0 0.1, inner_tol_min 1e-8, inner_max_iter 2000,
 * point atoms (n_scales 0). */
PC_API void pc_solve_params_default(pc_solve_params* params);

/* Solve the LASSO for the visibilities `vis` (dev complex64 [nvis], caller
 * order).  Returns PC_OK when a tolerance stopped the solve, or
 * PC_WARN_NOT_CONVERGED when max_iter did (result complete in both cases),
 * PC_ERR_CAPACITY if result->capacity < natoms (result->natoms then holds the
 * required size and the other outputs are filled).  Synchronous. */
PC_API pc_status pc_polyclean_solve(pc_plan* plan, const void* vis, const pc_solve_params* params,
                             pc_solve_result* result, void* stream);

/* ---------------------------------------------------------------------------
 * Step-wise solve, for schedulers that interleave several jobs: the same
 * algorithm as pc_polyclean_solve, one Frank-Wolfe iteration per
 * pc_solver_step.  The solver keeps its job's state (sorted visibilities,
 * residual, active set, weights, dirty-residual image) resident in device
 * memory until pc_solver_destroy.  `stream` (given at creation) orders all of
 * the job's work; different jobs may use different streams.
 * ------------------------------------------------------------------------- */
typedef struct pc_solver pc_solver;

/* Validates like pc_polyclean_solve and computes the dirty image,
 * lambda_max and lambda.  vis is read only during this call. */
PC_API pc_status pc_solver_create(pc_plan* plan, const void* vis, const pc_solve_params* params,
                                  void* stream, pc_solver** out);
/* One Frank-Wolfe iteration; *done (host, nullable) becomes 1 once a stop
 * rule has fired (further steps do nothing). */
PC_API pc_status pc_solver_step(pc_solver* solver, int32_t* done);
/* Current iterate as a result (same semantics as pc_polyclean_solve). */
PC_API pc_status pc_solver_result(pc_solver* solver, pc_solve_result* result);
PC_API void pc_solver_destroy(pc_solver* solver);

/* ---------------------------------------------------------------------------
 * Batched serving.  Several solves run at once, each driven by its own host
 * thread on its own stream (pc_solver_step releases nothing and takes no
 * global lock).  Solvers attached to one batcher send their gridded adjoints
 * (the full-grid step 4 of Alg. 2 and the dirty image at creation) through it:
 * requests that meet while the device is busy are merged into shared
 * launches (one spreading launch, one fold, one launch per fine-grid size and
 * FFT pass, whatever the jobs' grid and visibility counts), and the next
 * merged launch starts as soon as the previous one ends.  Each job's result
 * is identical to its result alone: the shared launches run the same
 * per-tile and per-row work as a job's own adjoint.
 * A batcher serves one device; it outlives every solver attached to it.
 * ------------------------------------------------------------------------- */
typedef struct pc_batcher pc_batcher;

typedef struct pc_batcher_stats {
  int64_t batches;      /* shared adjoint launch groups issued */
  int64_t requests;     /* adjoints served */
  int64_t visibilities; /* sum of the served plans' visibility counts */
  int32_t max_batch;    /* most requests merged into one group */
  int32_t pad;
  double seconds;       /* device time of the shared adjoints (HIP events) */
  int64_t forwards;     /* residual forwards (direct sums, step 4) run in
                           shared launches ahead of the adjoints */
  int64_t restricted_adjoints; /* restricted adjoints (point-spread sums and
                           b of new atoms in the Gram form) run in shared
                           launches */
} pc_batcher_stats;

/* Creates a batcher on `device` with a stream of its own (default priority).
 * Allocates its launch tables lazily. */
PC_API pc_status pc_batcher_create(int32_t device, pc_batcher** out);
PC_API pc_status pc_batcher_get_stats(const pc_batcher* batcher, pc_batcher_stats* stats);
PC_API void pc_batcher_destroy(pc_batcher* batcher);
/* pc_solver_create for a solver whose gridded adjoints go through `batcher`
 * (NULL: same as pc_solver_create).  The plan must live on the batcher's
 * device.  May be called concurrently from several threads. */
PC_API pc_status pc_solver_create_batched(pc_plan* plan, const void* vis,
                                          const pc_solve_params* params, void* stream,
                                          pc_batcher* batcher, pc_solver** out);

#ifdef __cplusplus
}
#endif

#endif /* POLYCLEAN_H */
