/*
 * demons.h - C ABI of the gfx950 (MI355X) demons deformable-registration
 * library, libdemons.so.
 *
 * What it computes: multi-scale demons registration as described by Gu et al.,
 * "Implementation and evaluation of various demons deformable image
 * registration algorithms on GPU": each iteration deforms the moving image
 * with the current displacement field by trilinear interpolation (Sec 2.5,
 * interpolation kernel), evaluates one of the demons forces of Eqs 1-6 from
 * the intensity difference and central-difference gradients (Sec 2.1, 2.2,
 * Sec 2.5 gradient and displacement kernels), adds it to the field and
 * smooths the field with a separable Gaussian (Sec 2.1, Sec 2.5 low-pass
 * filter kernel).  Levels run coarse to fine with 2x down-sampling and 2x
 * field up-sampling (Sec 2.3); the relative norm of Sec 2.4 is reduced every
 * iteration and optionally stops a level.
 *
 * Conventions shared by every entry point:
 *   - Volumes are float32 [nz][ny][nx], x fastest (index x + nx*(y + ny*z)).
 *   - A displacement field is three such planes back to back (x, y, z
 *     components), float32, in voxel units.
 *   - A field v registers M onto S when M(x - v(x)) ~= S(x).
 *   - Out-of-grid samples clamp the coordinate; stencils clamp the index.
 *   - Pointers named d_* are DEVICE pointers on the handle's device, owned by
 *     the caller; host pointers are named without the prefix.
 *   - nx*ny*nz must be at most 357,913,941 (a field of 12 bytes per voxel
 *     stays below 4 GiB); larger sizes return DIR_EINVAL.
 *   - All device work is enqueued on the handle's stream.  dir_register,
 *     dir_force and dir_step block until their work is complete; the other
 *     entry points only enqueue (call dir_synchronize before reading their
 *     outputs on the host).  dir_register_async enqueues a whole registration
 *     and returns; while it is in flight the handle refuses further work with
 *     DIR_EBUSY until dir_wait collects it.  Registrations on distinct
 *     handles with distinct streams run concurrently on the device.
 *   - Return value: DIR_OK or a negative dir_status; no exception crosses the
 *     ABI.  After an error the contents of output buffers are unspecified.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef DEMONS_H
#define DEMONS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIR_ABI_VERSION 1
#define DIR_MAX_LEVELS 8
#define DIR_MAX_RADIUS 16
#define DIR_MAX_BATCH 8           /* registrations per dir_register_batch call */
#define DIR_DEFAULT_COMPOSE_ITERS 10

typedef enum {
    DIR_OK = 0,
    DIR_EINVAL = -1,   /* bad argument (null pointer, size, parameter range) */
    DIR_ENOMEM = -2,   /* device or host allocation failed */
    DIR_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed */
    DIR_ENUMERIC = -4, /* a non-finite value appeared in the per-iteration sums */
    DIR_EBUSY = -5     /* a registration is in flight on the handle (dir_wait first) */
} dir_status;

/* Demons force variants (Sec 2.1-2.2).  The Pennec/Wang normalisation factor
 * alpha multiplies D^2 in every denominator of Eqs 1, 3, 4 (giving Eq 5 for
 * DIR_DOUBLE) and 6; alpha = 1 is the paper's unnormalised form.  It is not
 * used by DIR_EVOLVED_PASSIVE (Eq 2). */
typedef enum {
    DIR_PASSIVE = 0,             /* Eq 1: grad of the static image, computed once per level */
    DIR_EVOLVED_PASSIVE = 1,     /* Eq 2: adds |grad| of the undeformed moving image */
    DIR_ACTIVE = 2,              /* Eq 3: grad of the deformed moving image, every iteration */
    DIR_DOUBLE = 3,              /* Eq 4 (Eq 5 with alpha != 1): Eq 1 + Eq 3 */
    DIR_INVERSE_CONSISTENT = 4   /* Eq 6: both images deformed toward each other */
} dir_variant;

/* Units the iteration is written in.  The paper states the method in voxel
 * units (its Gaussian has unit standard deviation, Sec 2.5) while its images
 * have anisotropic voxels (Table 1: about 1.1 x 1.1 x 2.5 mm).  DIR_UNITS_MM
 * writes the same iteration in millimetres, from the voxel sizes spacing_mm
 * (h_x, h_y, h_z) of the input grid (level k has voxels of 2^k h):
 *   - gradients are in intensity per mm;
 *   - the force carries the squared intensity difference over K, the mean
 *     squared voxel size of the level: Eq 1 becomes
 *     dr = D G K / (alpha^2 D^2 + K |G|^2) (Eqs 2-6 likewise, Eq 2 with K
 *     against every squared gradient), dr in mm;
 *   - sigma (and image_sigma) are in mm: the Gaussian has sigma / h_a voxels
 *     along axis a on every level, radius ceil(3 sigma / h_a) per axis unless
 *     `radius` is given;
 *   - the norms of the relative norm (Sec 2.4) are in mm.
 * The output field is in voxels of the input grid either way.  With
 * h = (1, 1, 1) the two units give the same registration. */
typedef enum {
    DIR_UNITS_VOXELS = 0,
    DIR_UNITS_MM = 1
} dir_units;

/* Registration parameters.  Set struct_size = sizeof(dir_params) and zero
 * what is not used (make the struct with = {0}). */
typedef struct {
    int32_t struct_size;
    int32_t variant;                 /* dir_variant */
    double alpha;                    /* > 0; 1.0 = paper form */
    double sigma;                    /* Gaussian standard deviation in voxels (mm with DIR_UNITS_MM), > 0
                                        (Sec 2.5: 1 voxel) */
    int32_t radius;                  /* taps 2R+1 per axis; <= 0 selects ceil(3 sigma) (per axis in mm);
                                        at most DIR_MAX_RADIUS */
    int32_t levels;                  /* 1..DIR_MAX_LEVELS; level k has ceil(n / 2^k) voxels per axis */
    int32_t iters[DIR_MAX_LEVELS];   /* iterations per level, COARSEST FIRST; each >= 0 */
    double eps;                      /* 0: fixed counts; > 0: stop a level once l(n-10) - l(n) <= eps (Sec 2.4) */
    int32_t compose_iters;           /* fixed-point steps of the IC output composition; < 0 selects 10 */
    int32_t storage;                 /* dir_storage of images and fields inside the registration */
    int32_t units;                   /* dir_units; DIR_UNITS_MM needs spacing_mm */
    int32_t reserved;                /* 0 */
    double image_sigma;              /* > 0: every level's static and moving images (each restricted from the
                                        unsmoothed finer level) are smoothed with a Gaussian of this width
                                        (voxels, or mm) and radius ceil(3 width) per axis before the level
                                        runs (Sec 2.5: the low-pass filter kernel smooths images as well as
                                        displacements); 0: no pre-smoothing */
} dir_params;

/* Storage format of the image pyramids, fields and deformed-image buffers
 * inside a registration.  Arithmetic is FP32 and the sums, the relative norm
 * and the intensity difference are FP64 in every format; a 16-bit format
 * halves the bytes each iteration moves at the cost of rounding every stored
 * value (relative 2^-11 for F16, 2^-8 for BF16).  Inputs and the output field
 * stay FP32. */
typedef enum {
    DIR_STORE_F32 = 0,
    DIR_STORE_F16 = 1,   /* IEEE binary16 (range +-65504: intensities and fields fit) */
    DIR_STORE_BF16 = 2   /* bfloat16 (8-bit significand) */
} dir_storage;

/* Optional registration statistics.  Set struct_size = sizeof(dir_stats).
 * history, if not NULL, is a caller-owned host buffer of 4 * history_capacity
 * doubles; per iteration run (levels coarse to fine, packed) it receives
 * sum|dr|, sum|v| (field before the update), mean D^2 and the relative norm
 * l = sum|dr| / sum|v| (NaN while sum|v| = 0). */
typedef struct {
    int32_t struct_size;
    int32_t levels;                     /* written */
    int32_t iters_run[DIR_MAX_LEVELS];  /* written, coarsest first */
    double mse_final;                   /* written: mean D^2 of the last iteration run */
    double relnorm_final;               /* written: l of the last iteration run */
    double *history;                    /* in: host buffer or NULL */
    int32_t history_capacity;           /* in: iterations the buffer holds */
    int32_t history_len;                /* written: iterations stored */
} dir_stats;

typedef struct dir_handle dir_handle;

/* ABI version of the loaded library (DIR_ABI_VERSION it was built with). */
int32_t dir_abi_version(void);

/* Static, never-NULL description of a status code. */
const char *dir_strerror(int32_t code);

/* Text of the last HIP error seen by any handle of this thread ("" if none). */
const char *dir_last_error_message(void);

/* Create a handle on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL selects the null stream).  The handle owns its workspace
 * (image pyramid, ping-pong fields, per-block sums, history), which grows to
 * the largest request and is freed by dir_destroy. */
int32_t dir_create(dir_handle **out, int32_t device, void *stream);

/* Replace the stream work is enqueued on. */
int32_t dir_set_stream(dir_handle *h, void *stream);

/* Free the handle and its workspace.  NULL is accepted. */
int32_t dir_destroy(dir_handle *h);

/* Wait for all work enqueued by this handle. */
int32_t dir_synchronize(dir_handle *h);

/* Capture of whole registrations and lockstep batches into HIP graphs
 * (enable != 0; off by default).  With it on, a registration or batch that
 * needs no host wait (eps = 0, or any asynchronous call) on a handle with a
 * non-null stream and no kernel timing is captured on first use and replayed
 * by later calls whose arguments (pointers, sizes, parameters, spacing) and
 * workspace are unchanged: one graph launch instead of one launch per kernel,
 * with the same kernels, so results are bitwise those of enqueuing the
 * kernels one by one.  It cuts the host's submission time about 7x; on ROCm 7
 * the device time is not shorter (a lone registration runs about 10% longer
 * as a graph), hence the default.  The handle keeps the last captured graph;
 * other calls capture anew. */
int32_t dir_set_graphs(dir_handle *h, int32_t enable);

/* Multi-scale demons registration of d_moving onto d_static (Sec 2.1-2.4).
 * d_static, d_moving: nx*ny*nz floats each.  spacing_mm: host array of three
 * voxel sizes (> 0) or NULL; in voxel units (params->units =
 * DIR_UNITS_VOXELS, the paper's form) it is only validated, in DIR_UNITS_MM
 * it is required and sets the physical units.  d_field_out: 3*nx*ny*nz floats,
 * receives v with M(x - v(x)) ~= S(x) for every variant (for
 * DIR_INVERSE_CONSISTENT the composed full field, see dir_compose).
 * Blocks until complete. */
int32_t dir_register(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                     int32_t nz, const double *spacing_mm, const dir_params *params, float *d_field_out,
                     dir_stats *stats);

/* dir_register without the wait: validates the arguments (same rules and
 * codes as dir_register), enqueues every kernel of the registration on the
 * handle's stream and returns DIR_OK.  d_static, d_moving and d_field_out
 * must stay allocated and unmodified by other work until dir_wait returns;
 * work that produced them on another stream must be ordered before the
 * handle's stream by the caller.  Under the stopping rule (eps > 0) every
 * iteration is enqueued and those after the rule fires return without work,
 * so the result equals dir_register's.  One registration per handle may be
 * in flight. */
int32_t dir_register_async(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                           int32_t nz, const double *spacing_mm, const dir_params *params, float *d_field_out);

/* Wait for the registration enqueued by dir_register_async (or the batch
 * enqueued by dir_register_batch_async) and fill `stats` as dir_register
 * does: NULL, or one entry per registration in flight.  Returns its status
 * (DIR_ENUMERIC for a non-finite sum in any of them) or DIR_EINVAL when
 * none is in flight. */
int32_t dir_wait(dir_handle *h, dir_stats *stats);

/* Deformed image (Sec 2.5 interpolation kernel): d_out(x) = vol(x - v(x)),
 * trilinear, coordinates clamped.  d_field: 3 planes. */
int32_t dir_warp(dir_handle *h, const float *d_vol, const float *d_field, int32_t nx, int32_t ny, int32_t nz,
                 float *d_out);

/* Central-difference gradient (Sec 2.5 gradient kernel): 3 planes
 * (I[i+1] - I[i-1]) / 2 per axis, indices clamped, voxel units. */
int32_t dir_gradient(dir_handle *h, const float *d_img, int32_t nx, int32_t ny, int32_t nz, float *d_grad);

/* Separable Gaussian smoothing (Sec 2.1, Sec 2.5 low-pass filter kernel) of
 * ncomp planes (1..3): weights exp(-j^2/(2 sigma^2)) normalised to unit sum,
 * j in [-R, R], clamped borders.  radius <= 0 selects ceil(3 sigma).
 * d_in and d_out must not overlap. */
int32_t dir_smooth(dir_handle *h, const float *d_in, int32_t ncomp, int32_t nx, int32_t ny, int32_t nz,
                   double sigma, int32_t radius, float *d_out);

/* 2x down-sampling (Sec 2.3): 2x2x2 box mean with children clamped to the
 * grid; d_out has ceil(nx/2) x ceil(ny/2) x ceil(nz/2) voxels. */
int32_t dir_restrict(dir_handle *h, const float *d_in, int32_t nx, int32_t ny, int32_t nz, float *d_out);

/* Field up-sampling to the next finer level (Sec 2.3): cell-centred trilinear
 * interpolation (fine index f at coarse coordinate (f - 0.5) / 2, clamped),
 * values multiplied by 2.  d_coarse: 3 planes of cnx*cny*cnz; d_fine: 3 planes
 * of fnx*fny*fnz. */
int32_t dir_prolong(dir_handle *h, const float *d_coarse, int32_t cnx, int32_t cny, int32_t cnz, float *d_fine,
                    int32_t fnx, int32_t fny, int32_t fnz);

/* One force evaluation (Eqs 1-6) at one level, as inside dir_register:
 * d_updated = v + dr.  For DIR_INVERSE_CONSISTENT d_field is the symmetric
 * half field h (M deformed by x - h, S by x + h).  sums, if not NULL, is a
 * host array receiving sum|dr|, sum|v| and sum D^2 (FP64).  Blocks. */
int32_t dir_force(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                  const float *d_field, int32_t nx, int32_t ny, int32_t nz, float *d_updated, double *sums);

/* One full iteration at one level, exactly as dir_register runs it (same
 * kernels and launch configuration): d_field_out = G_sigma * (v + dr), the
 * Gaussian of dir_smooth applied to the output of dir_force.  sums as in
 * dir_force (over v and dr of this iteration).  d_field_out must not overlap
 * d_field.  Blocks. */
int32_t dir_step(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                 const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma, int32_t radius,
                 float *d_field_out, double *sums);

/* dir_step with the images and field held in a 16-bit storage format, as a
 * registration with params->storage = `storage` holds them: d_static,
 * d_moving and d_field (FP32) are first rounded to that format, the iteration
 * runs with its intermediates stored in it, and d_field_out receives the
 * stored result converted back to FP32.  DIR_STORE_F32 equals dir_step. */
int32_t dir_step_stored(dir_handle *h, int32_t storage, int32_t variant, double alpha, const float *d_static,
                        const float *d_moving, const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma,
                        int32_t radius, float *d_field_out, double *sums);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not allocate while other
 * work is being captured into a HIP graph): dir_step
 * (same arguments, same kernels and launch shapes, so bitwise the same
 * d_field_out and sums, FP32 storage) with every intermediate (the
 * x-smoothed field, the pre-warped images, the per-workgroup sums, the
 * history entry and the level state) in a fixed array of
 * DIR_NOALLOC_SCRATCH_BYTES in device memory that the library holds per
 * device from its first dir_create on that device until the process ends,
 * instead of the handle's workspace.  It calls no allocating routine, creates
 * no timing events and leaves the handle's workspace untouched.  The array
 * takes 12 bytes per voxel for DIR_PASSIVE and DIR_EVOLVED_PASSIVE, 16 for
 * DIR_ACTIVE and DIR_DOUBLE and 20 for DIR_INVERSE_CONSISTENT, plus at most
 * 197 KB of sums: 256x256x100 fits every variant.  A larger volume returns
 * DIR_EINVAL (dir_last_error_message gives the bytes it needs) before any
 * work is enqueued.  Every call on one device shares that device's array and
 * it keeps the last call's contents (each call rewrites what it reads), so
 * calls that overlap on one device (several threads, or handles on
 * different streams) race and must be serialised by the caller.  Blocks
 * until the step is complete (it reads the sums back), so the call itself
 * cannot be recorded into a graph. */
#define DIR_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int32_t dir_step_noalloc(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                         const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma, int32_t radius,
                         float *d_field_out, double *sums);

/* Output field of the inverse-consistent variant from its half field h:
 * w(z) = 2 h(p) with p = z - h(p), p found by K fixed-point updates
 * p <- z - h(p) that start from the first-order inverse p = z - h(z)
 * (K < 0 selects 10; K = 0 gives w(z) = 2 h(z - h(z))).  d_half, d_out:
 * 3 planes, must not overlap. */
int32_t dir_compose(dir_handle *h, const float *d_half, int32_t nx, int32_t ny, int32_t nz, int32_t K,
                    float *d_out);

/* Workspace (device bytes) a handle allocates for a registration with these
 * sizes and parameters; host-only, no device needed.  DIR_EINVAL for
 * parameters dir_register would reject. */
int32_t dir_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const dir_params *params, uint64_t *bytes);

/* Lockstep batch (the iteration of Sec 2.4 and the pyramid of Sec 2.3, run
 * for several pairs at once): `count` (1..DIR_MAX_BATCH) registrations given
 * as host arrays of device pointers d_static[r], d_moving[r] and
 * d_field_out[r], their sizes dims[3r], dims[3r+1], dims[3r+2] (nx, ny, nz;
 * they may differ), spacing_mm (NULL, or three values per registration, only
 * validated as in dir_register) and params[r].  The registrations must agree
 * in levels, iterations per level, sigma, radius, storage, units and
 * image_sigma (and, in DIR_UNITS_MM, spacing); size, variant, alpha, eps and
 * compose_iters may differ.
 *
 * On a pyramid level whose images and fields, over all `count`
 * registrations, fit the device's 256 MB last-level cache (about 8 stored
 * values per voxel each), every iteration of all of them runs as one
 * pre-warp launch (for the variants that have one), one force launch and one
 * smoothing launch (one per tile class when sizes differ: each registration
 * keeps the workgroup layout it has alone): the short, latency-bound launches
 * of coarse levels then carry the work of the whole batch.  A larger level
 * streams from HBM either way and runs registration by registration, so that
 * each kernel finds the field the previous one wrote still in that cache.
 *
 * Each field, its iteration counts and its history are bitwise those
 * dir_register computes alone.  Output fields must be distinct and must not
 * overlap any input.  stats: NULL or an array of `count` (each with
 * struct_size set); DIR_ENUMERIC if any registration's sums turn non-finite.
 * The workspace holds `count` registrations' worth of the largest.  Blocks
 * until complete. */
int32_t dir_register_batch(dir_handle *h, int32_t count, const float *const *d_static,
                           const float *const *d_moving, const int32_t *dims, const double *spacing_mm,
                           const dir_params *params, float *const *d_field_out, dir_stats *stats);

/* The same batch enqueued without waiting (as dir_register_async); dir_wait
 * collects it, with stats NULL or an array of `count`. */
int32_t dir_register_batch_async(dir_handle *h, int32_t count, const float *const *d_static,
                                 const float *const *d_moving, const int32_t *dims, const double *spacing_mm,
                                 const dir_params *params, float *const *d_field_out);

/* Autotuning of launch shapes that leave every result unchanged.  The y/z
 * smoothing kernel (Sec 2.5 low-pass filter) walks z in chunks of 2, 4 or 8
 * planes per workgroup; the depth decides only which workgroup computes which
 * output.  dir_autotune times each depth on the handle's stream at every
 * pyramid level of an nx*ny*nz volume under params (levels, sigma, radius,
 * storage), for launches that carry `count` (1..DIR_MAX_BATCH) registrations
 * as a lockstep batch does, and keeps the fastest for all handles of the
 * process; depths (NULL or params->levels entries, finest first) receives
 * them.  Untuned launches use a fixed rule.  It uses the handle's field
 * buffers as scratch and blocks.  dir_autotune_clear forgets every choice.
 * Thread-safe with respect to registrations on other handles. */
int32_t dir_autotune(dir_handle *h, int32_t nx, int32_t ny, int32_t nz, const dir_params *params, int32_t count,
                     int32_t *depths);
void dir_autotune_clear(void);

/* Request pool (serving).  A pool runs submitted registrations on `slots`
 * handles of its own, each with its own stream, so registrations that arrive
 * while others run overlap with them on the device.  Requests are admitted in
 * arrival order when a slot is free and the workspace all slots then hold
 * stays within max_bytes (0: no limit); a slot keeps its workspace between
 * requests (resident pyramids and fields) and free slots give it back when a
 * request would not fit otherwise.  The pool has no thread of its own: every
 * pool call first collects finished registrations without blocking and admits
 * queued ones.  Results are bitwise those of dir_register on the same inputs.
 * Not thread-safe.
 *
 * dir_pool_submit: queue a registration (arguments as dir_register; the
 *   device buffers must stay valid until its result is taken) and return its
 *   ticket (> 0).  DIR_ENOMEM if it needs more than max_bytes by itself.
 * dir_pool_poll: *done = 1 and the registration's status if it finished (its
 *   result is then taken: stats, if not NULL, receives it without history),
 *   else *done = 0 and DIR_OK.  DIR_EINVAL for an unknown or taken ticket.
 * dir_pool_wait: block until the ticket finishes; its status.
 * dir_pool_stats: workspace held now, the peak held after any admission, the
 *   peak number of registrations running at once, requests queued now. */
typedef struct dir_pool dir_pool;
int32_t dir_pool_create(dir_pool **out, int32_t device, int32_t slots, uint64_t max_bytes);
int32_t dir_pool_destroy(dir_pool *p);
int32_t dir_pool_submit(dir_pool *p, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                        int32_t nz, const double *spacing_mm, const dir_params *params, float *d_field_out,
                        int64_t *ticket);
int32_t dir_pool_progress(dir_pool *p);
int32_t dir_pool_poll(dir_pool *p, int64_t ticket, dir_stats *stats, int32_t *done);
int32_t dir_pool_wait(dir_pool *p, int64_t ticket, dir_stats *stats);
int32_t dir_pool_stats(const dir_pool *p, uint64_t *held_bytes_now, uint64_t *peak_bytes, int32_t *peak_running,
                       int32_t *queued_now);
/* Registrations one slot may run as a lockstep batch (1..DIR_MAX_BATCH;
 * 1, the default, admits requests one by one).  Above 1 the request at the
 * head of the queue is admitted with the queued requests after it that can
 * run in lockstep with it (dir_register_batch: the same levels, iterations,
 * sigma, radius and storage), up to the limit, as one batch on one slot,
 * whose workspace the budget counts.  Results are still bitwise those of
 * dir_register. */
int32_t dir_pool_set_max_batch(dir_pool *p, int32_t max_batch);

/* How well a field registers the pair, the two measures the paper follows
 * over the iterations (Sec 3.2): *mse, the mean of (Im - S)^2, and *cc, the
 * Pearson correlation coefficient of Im and S over all voxels, with
 * Im(x) = M(x - v(x)) sampled in FP64 and every sum in FP64 (NaN when either
 * image is constant).  d_field: 3 planes, or NULL for the undeformed M.
 * Either output may be NULL.  Blocks. */
int32_t dir_similarity(dir_handle *h, const float *d_static, const float *d_moving, const float *d_field, int32_t nx,
                       int32_t ny, int32_t nz, double *mse, double *cc);

/* Per-kernel device timing with HIP events on the handle's stream.
 * Kernels are numbered 0 .. dir_timing_count()-1; dir_timing_name(k) gives
 * the kernel's name (NULL if k is out of range).
 * dir_timing_enable(h, mask) zeroes the totals and, for every kernel k whose
 * bit (1 << k) is set, launches each later instance of k with a start and a
 * stop event that the dispatch stamps at kernel begin and end (so the time is
 * the kernel's own, as a kernel trace reports it); mask 0 stops recording.
 * dir_timing_read returns the accumulated device milliseconds and launch
 * count of kernel k over the launches of blocking calls (dir_register,
 * dir_force) and of calls followed by dir_synchronize;
 * dir_timing_read_level the same restricted to pyramid level `level`
 * (0 = finest; launches outside dir_register count as level 0).  Both return
 * DIR_EINVAL for a NULL handle or an index out of range. */
int32_t dir_timing_count(void);
const char *dir_timing_name(int32_t kernel);
int32_t dir_timing_enable(dir_handle *h, uint64_t kernel_mask);
int32_t dir_timing_read(dir_handle *h, int32_t kernel, double *total_ms, int64_t *launches);
int32_t dir_timing_read_level(dir_handle *h, int32_t kernel, int32_t level, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* DEMONS_H */
