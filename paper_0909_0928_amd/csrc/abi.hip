// C ABI of libdemons (include/demons.h): handle, workspace, argument
// validation, the multi-scale registration loop and per-kernel timing.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <algorithm>
#include <vector>

#include "demons.h"
#include "dir_internal.h"

using namespace dir;

namespace {

thread_local std::string g_last_error;

const char *const kKernelNames[K_COUNT] = {
    "force", "warp", "warp_pair", "smooth_yz", "smooth_x", "finalize", "level_reset",
    "restrict", "prolong", "gradient", "compose", "fill", "convert", "similarity", "warp_mixed",
};

// Bytes allocated past every workspace buffer's size: 16-bit volumes are
// gathered with 8-byte loads that may reach kPad16 bytes past a volume's end.
constexpr size_t kSlackBytes = 256;
static_assert(kSlackBytes >= kPad16, "slack covers the gathers' overreach");

// Device buffer that only grows (`bytes` usable, kSlackBytes more allocated).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need)
    {
        if (need <= bytes) return hipSuccess;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            bytes = 0;
        }
        hipError_t e = hipMalloc(&p, need + kSlackBytes);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

}  // namespace

// Key of a captured registration or lockstep batch: the bytes of the call's
// arguments (pointers, sizes, parameters, voxel sizes) and of every workspace
// and side-stream address its kernels use.  Replaying the graph is only valid
// for an equal key.
using GraphKey = std::vector<unsigned char>;
static_assert(kMaxBatch == DIR_MAX_BATCH, "batch limit of the ABI and of the kernels");

// A registration enqueued by dir_register_async (or dir_register) whose
// statistics have not been collected yet.
struct InFlight {
    bool active = false;
    int count = 1;                  // registrations (a lockstep batch: more than 1)
    int levels = 0;
    int64_t total_iters = 0;
    int64_t hist_off[DIR_MAX_LEVELS] = {};
    size_t hist_stride = 0;         // bytes between registrations' histories
    size_t state_stride = 0;        // bytes between registrations' level states
};

struct dir_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    Timer timer;
    DevBuf pyr_s, pyr_m;           // levels 1.. of the image pyramids, packed
    DevBuf field[3];               // fields, 3 planes each: v and x-smoothed u; scratch for dir_smooth
    DevBuf img_a, img_b;           // pre-warped D (active, double, IC) and P = Im + Is (IC)
    DevBuf img0_s, img0_m;         // finest-level S and M in a 16-bit storage format
    DevBuf pre_s, pre_m;           // every level of S and M pre-smoothed (image_sigma > 0)
    DevBuf partials;               // 3 doubles per force workgroup
    DevBuf history;                // 4 doubles per iteration, per-level fixed offsets
    DevBuf state;                  // one LevelState per level
    InFlight inflight;             // registration enqueued and not yet collected
    bool graphs = false;           // capture registrations into HIP graphs (dir_set_graphs)
    hipGraphExec_t graph_exec = nullptr;  // the last captured registration
    GraphKey graph_key;            // ... and what it was captured for (empty: nothing captured)
    // Side streams on which a batch runs registrations concurrently (created
    // on first use, default priority); the handle's stream forks to them
    // with fork_ev and joins them with side_done.
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork_ev = nullptr;
    // Pinned host buffer the level states and histories of a finished
    // registration (or batch) are copied into, all at once.
    void *stage = nullptr;
    size_t stage_bytes = 0;
};

namespace {

int fail_hip(hipError_t e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
    return e == hipErrorOutOfMemory ? DIR_ENOMEM : DIR_EDEVICE;
}

#define DIR_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return fail_hip(_e, #expr); \
    } while (0)

// Volumes are addressed through buffer resources with 32-bit byte ranges: a
// three-component float field must stay below 4 GiB (nx*ny*nz < 357,913,942).
bool dims_ok(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return false;
    const int64_t n = (int64_t)nx * ny * nz;
    return 12 * n < (int64_t(1) << 32);
}

int resolve_radius(double sigma, int32_t radius)
{
    if (radius > 0) return radius;
    return (int)ceil(3.0 * sigma);
}

// Normalised sampled Gaussian (Sec 2.5 low-pass filter), computed in FP64 and
// rounded to FP32 taps.
GaussTaps make_taps(double sigma, int radius)
{
    GaussTaps t;
    memset(&t, 0, sizeof t);
    t.radius = radius;
    double w[2 * kMaxRadius + 1], sum = 0.0;
    for (int j = -radius; j <= radius; ++j) {
        w[j + radius] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
        sum += w[j + radius];
    }
    for (int j = 0; j <= 2 * radius; ++j) t.w[j] = t.wz[j] = (float)(w[j] / sum);
    return t;
}

// Taps of the y/z smoothing kernel for per-axis widths: y's in w, z's in wz,
// the narrower padded with zero taps to the common radius (a zero tap adds
// an exact zero, so the sums are those of the narrower stencil).
GaussTaps make_taps_yz(double sy, int ry, double sz, int rz)
{
    const GaussTaps ty = make_taps(sy, ry), tz = make_taps(sz, rz);
    GaussTaps t;
    memset(&t, 0, sizeof t);
    t.radius = std::max(ry, rz);
    for (int j = -ry; j <= ry; ++j) t.w[j + t.radius] = ty.w[j + ry];
    for (int j = -rz; j <= rz; ++j) t.wz[j + t.radius] = tz.w[j + rz];
    return t;
}

Dims coarser(Dims d) { return Dims{(d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2}; }

// Round a byte count up to a 256-byte boundary.
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int enter(dir_handle *h)
{
    if (!h) return DIR_EINVAL;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    h->timer.level = 0;
    return DIR_OK;
}

// enter() for calls that enqueue work: refused while a registration is in
// flight on the handle (its workspace is in use until dir_wait).
int enter_idle(dir_handle *h)
{
    int rc = enter(h);
    if (rc != DIR_OK) return rc;
    return h->inflight.active ? DIR_EBUSY : DIR_OK;
}

// Copy device bytes to the host on the handle's stream and wait for them.
int copy_to_host(dir_handle *h, void *dst, const void *src, size_t bytes)
{
    DIR_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
    DIR_TRY(hipStreamSynchronize(h->stream));
    return DIR_OK;
}

// Wait for the stream, then fold completed timing events into the totals.
int finish(dir_handle *h)
{
    DIR_TRY(hipStreamSynchronize(h->stream));
    DIR_TRY(h->timer.harvest());
    return DIR_OK;
}

// ---------------------------------------------------------------------------
// Scratch of dir_step_noalloc: a fixed array in device memory, one copy per
// device, held from the library's first use on that device until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host the
// name is a stand-in, not a device address): dir_create looks up the array's
// address on its device once, and the kernels take that address.
static __device__ __align__(256) unsigned char scratch[DIR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices];  // device address of `scratch` per device (null: not set up)

// With `device` current: look up the address of the device's copy of the
// array, once per device.
int setup_scratch(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return DIR_OK;  // dir_step_noalloc refuses such devices
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return DIR_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = ptr;
    return DIR_OK;
}

void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

}  // namespace

static_assert(dir::kTimerLevels >= DIR_MAX_LEVELS, "timer keeps one slot per pyramid level");

// ---------------------------------------------------------------------------
// Timer
// ---------------------------------------------------------------------------
namespace dir {

hipError_t Timer::take(hipEvent_t *ev)
{
    if (!pool_.empty()) {
        *ev = pool_.back();
        pool_.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

hipError_t Timer::pair(hipEvent_t *start, hipEvent_t *stop)
{
    hipError_t e = take(start);
    if (e != hipSuccess) return e;
    e = take(stop);
    if (e != hipSuccess) pool_.push_back(*start);
    return e;
}

void Timer::record(int k, hipEvent_t start, hipEvent_t stop)
{
    pending_.push_back(Rec{k, level < 0 ? 0 : (level < kTimerLevels ? level : kTimerLevels - 1), start, stop});
}

hipError_t Timer::harvest()
{
    hipError_t err = hipSuccess;
    for (const Rec &r : pending_) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e == hipSuccess) {
            total_ms[r.k][r.level] += ms;
            launches[r.k][r.level] += 1;
        } else if (err == hipSuccess) {
            err = e;
        }
        pool_.push_back(r.a);
        pool_.push_back(r.b);
    }
    pending_.clear();
    return err;
}

void Timer::reset()
{
    for (int k = 0; k < K_COUNT; ++k)
        for (int l = 0; l < kTimerLevels; ++l) {
            total_ms[k][l] = 0.0;
            launches[k][l] = 0;
        }
}

void Timer::release()
{
    for (const Rec &r : pending_) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    pending_.clear();
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
    pool_.clear();
}

}  // namespace dir

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t dir_abi_version(void) { return DIR_ABI_VERSION; }

const char *dir_strerror(int32_t code)
{
    switch (code) {
    case DIR_OK: return "success";
    case DIR_EINVAL: return "invalid argument";
    case DIR_ENOMEM: return "out of memory";
    case DIR_EDEVICE: return "HIP device error";
    case DIR_ENUMERIC: return "non-finite value in the registration sums";
    case DIR_EBUSY: return "a registration is in flight on this handle (collect it with dir_wait)";
    default: return "unknown status code";
    }
}

const char *dir_last_error_message(void) { return g_last_error.c_str(); }

int32_t dir_create(dir_handle **out, int32_t device, void *stream)
{
    if (!out) return DIR_EINVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return fail_hip(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return DIR_EINVAL;
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    const int rc = setup_scratch(device);
    if (rc != DIR_OK) return rc;
    dir_handle *h = new (std::nothrow) dir_handle();
    if (!h) return DIR_ENOMEM;
    h->device = device;
    h->stream = static_cast<hipStream_t>(stream);
    *out = h;
    return DIR_OK;
}

int32_t dir_set_stream(dir_handle *h, void *stream)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    rc = finish(h);  // work already enqueued on the old stream completes first
    h->stream = static_cast<hipStream_t>(stream);
    return rc;
}

int32_t dir_destroy(dir_handle *h)
{
    if (!h) return DIR_OK;
    int rc = enter(h);
    if (rc == DIR_OK) (void)hipStreamSynchronize(h->stream);
    for (hipStream_t sd : h->side) (void)hipStreamSynchronize(sd);
    for (hipStream_t sd : h->side) (void)hipStreamDestroy(sd);
    for (hipEvent_t e : h->side_done) (void)hipEventDestroy(e);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    h->timer.release();
    if (h->stage) (void)hipHostFree(h->stage);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    h->pyr_s.release();
    h->pyr_m.release();
    for (auto &f : h->field) f.release();
    h->img_a.release();
    h->img_b.release();
    h->img0_s.release();
    h->img0_m.release();
    h->pre_s.release();
    h->pre_m.release();
    h->partials.release();
    h->history.release();
    h->state.release();
    delete h;
    return rc;
}

int32_t dir_synchronize(dir_handle *h)
{
    int rc = enter(h);
    if (rc != DIR_OK) return rc;
    return finish(h);
}

int32_t dir_set_graphs(dir_handle *h, int32_t enable)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    h->graphs = enable != 0;
    if (!h->graphs && h->graph_exec) {
        rc = finish(h);
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
        h->graph_key.clear();
    }
    return rc;
}

int32_t dir_timing_count(void) { return K_COUNT; }

const char *dir_timing_name(int32_t kernel)
{
    if (kernel < 0 || kernel >= K_COUNT) return nullptr;
    return kKernelNames[kernel];
}

int32_t dir_timing_enable(dir_handle *h, uint64_t kernel_mask)
{
    int rc = enter(h);
    if (rc != DIR_OK) return rc;
    rc = finish(h);
    h->timer.reset();
    h->timer.mask = kernel_mask;
    return rc;
}

int32_t dir_timing_read(dir_handle *h, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!h || kernel < 0 || kernel >= K_COUNT) return DIR_EINVAL;
    double ms = 0.0;
    int64_t n = 0;
    for (int l = 0; l < kTimerLevels; ++l) {
        ms += h->timer.total_ms[kernel][l];
        n += h->timer.launches[kernel][l];
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    return DIR_OK;
}

int32_t dir_timing_read_level(dir_handle *h, int32_t kernel, int32_t level, double *total_ms, int64_t *launches)
{
    if (!h || kernel < 0 || kernel >= K_COUNT || level < 0 || level >= kTimerLevels) return DIR_EINVAL;
    if (total_ms) *total_ms = h->timer.total_ms[kernel][level];
    if (launches) *launches = h->timer.launches[kernel][level];
    return DIR_OK;
}

int32_t dir_warp(dir_handle *h, const float *d_vol, const float *d_field, int32_t nx, int32_t ny, int32_t nz,
                 float *d_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_vol || !d_field || !d_out || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_warp(c, d_vol, d_field, Dims{nx, ny, nz}, d_out, nullptr, 0));
    return DIR_OK;
}

int32_t dir_gradient(dir_handle *h, const float *d_img, int32_t nx, int32_t ny, int32_t nz, float *d_grad)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_img || !d_grad || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_gradient(c, d_img, Dims{nx, ny, nz}, d_grad));
    return DIR_OK;
}

int32_t dir_smooth(dir_handle *h, const float *d_in, int32_t ncomp, int32_t nx, int32_t ny, int32_t nz,
                   double sigma, int32_t radius, float *d_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_in || !d_out || ncomp < 1 || ncomp > 3 || !dims_ok(nx, ny, nz) || !(sigma > 0.0) || !isfinite(sigma))
        return DIR_EINVAL;
    const int R = resolve_radius(sigma, radius);
    if (R < 0 || R > DIR_MAX_RADIUS) return DIR_EINVAL;
    const Dims d{nx, ny, nz};
    const size_t bytes = sizeof(float) * (size_t)ncomp * (size_t)d.n();
    const char *in = reinterpret_cast<const char *>(d_in);
    const char *out = reinterpret_cast<const char *>(d_out);
    if (in < out + bytes && out < in + bytes) return DIR_EINVAL;  // overlap
    DIR_TRY(h->field[2].ensure(sizeof(float) * 3 * (size_t)d.n()));
    Ctx c{h->stream, &h->timer};
    const GaussTaps taps = make_taps(sigma, R);
    DIR_TRY(launch_smooth_x(c, d_in, ncomp, d, taps, h->field[2].as<float>()));
    DIR_TRY(launch_smooth_yz(c, h->field[2].as<float>(), ncomp, d, taps, d_out, kStoreF32, nullptr, 0, SumsReduce{}));
    return DIR_OK;
}

int32_t dir_restrict(dir_handle *h, const float *d_in, int32_t nx, int32_t ny, int32_t nz, float *d_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_in || !d_out || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    const Dims f{nx, ny, nz};
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_restrict(c, d_in, kStoreF32, f, d_out, kStoreF32, coarser(f)));
    return DIR_OK;
}

int32_t dir_prolong(dir_handle *h, const float *d_coarse, int32_t cnx, int32_t cny, int32_t cnz, float *d_fine,
                    int32_t fnx, int32_t fny, int32_t fnz)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_coarse || !d_fine || !dims_ok(cnx, cny, cnz) || !dims_ok(fnx, fny, fnz)) return DIR_EINVAL;
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_prolong(c, d_coarse, Dims{cnx, cny, cnz}, d_fine, Dims{fnx, fny, fnz}, kStoreF32));
    return DIR_OK;
}

int32_t dir_compose(dir_handle *h, const float *d_half, int32_t nx, int32_t ny, int32_t nz, int32_t K,
                    float *d_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_half || !d_out || !dims_ok(nx, ny, nz) || d_half == d_out) return DIR_EINVAL;
    if (K < 0) K = DIR_DEFAULT_COMPOSE_ITERS;
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_compose(c, d_half, kStoreF32, Dims{nx, ny, nz}, K, d_out));
    return DIR_OK;
}

}  // extern "C"

namespace {

// Device buffers one force evaluation needs at level size d.
int ensure_force_workspace(dir_handle *h, Dims d, int variant, int storage)
{
    const size_t n = (size_t)d.n() * storage_bytes(storage);
    if (variant == kActive || variant == kDouble || variant == kInverseConsistent) DIR_TRY(h->img_a.ensure(n));
    if (variant == kInverseConsistent) DIR_TRY(h->img_b.ensure(sizeof(float) * (size_t)d.n()));  // P: FP32
    DIR_TRY(h->partials.ensure(sizeof(double) * 3 * (size_t)force_blocks(d)));
    return DIR_OK;
}

// Taps that leave a field unchanged (radius 0, weight 1).
GaussTaps identity_taps()
{
    GaussTaps t;
    memset(&t, 0, sizeof t);
    t.radius = 0;
    t.w[0] = t.wz[0] = 1.0f;
    return t;
}

// One iteration's force half for `count` registrations (arrays indexed by
// registration).
struct ForceHalf {
    int count = 1;
    int storage;
    Dims d[kMaxBatch];
    int variant[kMaxBatch];
    float alpha2[kMaxBatch];
    const void *S[kMaxBatch], *M[kMaxBatch], *v[kMaxBatch];
    void *D[kMaxBatch], *P[kMaxBatch];  // pre-warp outputs (workspace)
    void *out[kMaxBatch];
    double *partials[kMaxBatch];
    const int *stop_at[kMaxBatch];
    const Metric *metric = nullptr;     // physical units (the level's), or NULL
};

// The force half of one iteration: one pre-warp launch for the registrations
// whose variant needs deformed-image gradients, then one force launch (u =
// v + dr, x pass of the smoothing with `taps`, per-workgroup sums).
hipError_t force_half(Ctx &c, const ForceHalf &b, const GaussTaps &taps, int n)
{
    PrewarpLaunch w;
    w.count = 0;
    w.storage = b.storage;
    w.n = n;
    unsigned kinds = 0;
    for (int r = 0; r < b.count; ++r) {
        const int v = b.variant[r];
        if (v != kActive && v != kDouble && v != kInverseConsistent) continue;
        const int kind = v == kInverseConsistent ? kPrewarpPair : kPrewarpDiff;
        const int q = w.count++;
        w.kinds[q] = kind;
        kinds |= 1u << kind;
        w.M[q] = b.M[r];
        w.S[q] = b.S[r];
        w.v[q] = b.v[r];
        w.D[q] = b.D[r];
        w.P[q] = b.P[r];
        w.stop_at[q] = b.stop_at[r];
        w.d[q] = b.d[r];
    }
    if (w.count) {
        w.kind = kinds == (1u << kPrewarpDiff) ? kPrewarpDiff
                                               : (kinds == (1u << kPrewarpPair) ? kPrewarpPair : kPrewarpMixed);
        const hipError_t e = launch_prewarp(c, w);
        if (e != hipSuccess) return e;
    }
    ForceLaunch f;
    f.count = b.count;
    f.variant = b.variant[0];
    for (int r = 0; r < b.count; ++r) {
        if (b.variant[r] != b.variant[0]) f.variant = kMixedVariants;
        f.variants[r] = b.variant[r];
        f.alpha2[r] = b.alpha2[r];
        f.S[r] = b.S[r];
        f.M[r] = b.M[r];
        f.v[r] = b.v[r];
        f.D[r] = b.D[r];
        f.P[r] = b.P[r];
        f.out[r] = b.out[r];
        f.partials[r] = b.partials[r];
        f.stop_at[r] = b.stop_at[r];
        f.d[r] = b.d[r];
    }
    f.storage = b.storage;
    f.taps = &taps;
    f.metric = b.metric;
    f.n = n;
    return launch_force(c, f);
}

// Reduction descriptor of one registration's sums at level size d.
SumsReduce sums_reduce_one(double *partials, Dims d, double *hist, LevelState *st, double eps)
{
    SumsReduce r;
    r.count = 1;
    r.partials[0] = partials;
    r.nb[0] = (int)force_blocks(d);
    r.hist[0] = hist;
    r.st[0] = st;
    r.eps[0] = eps;
    r.inv_n[0] = 1.0 / (double)d.n();
    return r;
}

// Buffers one iteration outside a registration works in: the pre-warped
// images D and P, the per-workgroup sums, one history entry, the level state
// and (with taps, or with a 16-bit format) the x-smoothed field u.
struct StepBufs {
    void *D = nullptr, *P = nullptr, *u = nullptr;
    double *partials = nullptr, *history = nullptr;
    LevelState *st = nullptr;
};

// Arguments of one iteration outside a registration (dir_force, dir_step,
// dir_step_stored, dir_step_noalloc).
int check_step_args(int32_t variant, double alpha, const float *S, const float *M, const float *v, int32_t nx,
                    int32_t ny, int32_t nz, float *out, int storage)
{
    if (!S || !M || !v || !out || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    if (variant < kPassive || variant > kInverseConsistent || !(alpha > 0.0) || !isfinite(alpha)) return DIR_EINVAL;
    if (storage < kStoreF32 || storage > kStoreBF16) return DIR_EINVAL;
    const size_t bytes = sizeof(float) * 3 * (size_t)Dims{nx, ny, nz}.n();
    const char *vb = reinterpret_cast<const char *>(v), *ob = reinterpret_cast<const char *>(out);
    if (vb < ob + bytes && ob < vb + bytes) return DIR_EINVAL;  // out must not overlap the field
    return DIR_OK;
}

// The kernels of one iteration in FP32 storage on c's stream: force (with the
// pre-warp its variant needs), then the y/z smoothing and the reduction of the
// sums into b.history (or, without taps, the force alone and the reduction).
hipError_t enqueue_step(Ctx &c, const StepBufs &b, int32_t variant, double alpha, const void *S, const void *M,
                        const void *v, Dims d, const GaussTaps *taps, void *fout, int storage)
{
    hipError_t e = launch_level_reset(c, b.st);
    if (e != hipSuccess) return e;
    SumsReduce red = sums_reduce_one(b.partials, d, b.history, b.st, 0.0);
    red.inv_n[0] = 1.0;  // report the plain sum of D^2
    ForceHalf fh;
    fh.storage = storage;
    fh.d[0] = d;
    fh.variant[0] = variant;
    fh.alpha2[0] = (float)(alpha * alpha);
    fh.S[0] = S;
    fh.M[0] = M;
    fh.v[0] = v;
    fh.D[0] = b.D;
    fh.P[0] = b.P;
    fh.partials[0] = b.partials;
    fh.stop_at[0] = nullptr;
    if (taps) {
        fh.out[0] = b.u;
        e = force_half(c, fh, *taps, 0);
        if (e != hipSuccess) return e;
        return launch_smooth_yz(c, b.u, 3, d, *taps, fout, storage, nullptr, 0, red);
    }
    const GaussTaps id = identity_taps();
    fh.out[0] = fout;
    e = force_half(c, fh, id, 0);
    if (e != hipSuccess) return e;
    return launch_finalize(c, red, 0);
}

// Copy the three sums of the history entry to the host (the stream must be
// complete).
int read_step_sums(dir_handle *h, const double *history, double *sums)
{
    if (!sums) return DIR_OK;
    double e[4];
    const int rc = copy_to_host(h, e, history, sizeof e);
    if (rc != DIR_OK) return rc;
    sums[0] = e[0];
    sums[1] = e[1];
    sums[2] = e[2];  // inv_n = 1: the plain sum of D^2
    return DIR_OK;
}

// dir_force, dir_step and dir_step_stored: one iteration outside a
// registration in the handle's workspace, sums out.  With a 16-bit storage
// format the FP32 inputs are converted first (S, M, v into the workspace) and
// the result converted back.
int single_step(dir_handle *h, int32_t variant, double alpha, const float *S, const float *M, const float *v,
                int32_t nx, int32_t ny, int32_t nz, const GaussTaps *taps, float *out, double *sums,
                int storage = kStoreF32)
{
    int rc = check_step_args(variant, alpha, S, M, v, nx, ny, nz, out, storage);
    if (rc != DIR_OK) return rc;
    const Dims d{nx, ny, nz};
    const size_t n = (size_t)d.n();
    const size_t bytes = sizeof(float) * 3 * n;
    const bool conv = storage != kStoreF32;
    const size_t es = storage_bytes(storage);
    rc = ensure_force_workspace(h, d, variant, storage);
    if (rc != DIR_OK) return rc;
    DIR_TRY(h->history.ensure(sizeof(double) * 4));
    DIR_TRY(h->state.ensure(sizeof(LevelState)));
    if (taps || conv) DIR_TRY(h->field[2].ensure(bytes));
    if (conv) {
        DIR_TRY(h->img0_s.ensure(es * n));
        DIR_TRY(h->img0_m.ensure(es * n));
        DIR_TRY(h->field[0].ensure(es * 3 * n));
        DIR_TRY(h->field[1].ensure(es * 3 * n));
    }
    Ctx c{h->stream, &h->timer};
    const void *Sx = S, *Mx = M, *vx = v;
    void *fout = out;  // where the step leaves its result, in the storage format
    if (conv) {
        DIR_TRY(launch_convert(c, S, kStoreF32, h->img0_s.p, storage, (int64_t)n));
        DIR_TRY(launch_convert(c, M, kStoreF32, h->img0_m.p, storage, (int64_t)n));
        DIR_TRY(launch_convert(c, v, kStoreF32, h->field[0].p, storage, 3 * (int64_t)n));
        Sx = h->img0_s.p;
        Mx = h->img0_m.p;
        vx = h->field[0].p;
        fout = h->field[1].p;
    }
    StepBufs b;
    b.D = h->img_a.p;
    b.P = h->img_b.p;
    b.u = h->field[2].p;
    b.partials = h->partials.as<double>();
    b.history = h->history.as<double>();
    b.st = h->state.as<LevelState>();
    DIR_TRY(enqueue_step(c, b, variant, alpha, Sx, Mx, vx, d, taps, fout, storage));
    if (conv) DIR_TRY(launch_convert(c, fout, storage, out, kStoreF32, 3 * (int64_t)n));
    rc = finish(h);
    if (rc != DIR_OK) return rc;
    return read_step_sums(h, b.history, sums);
}

}  // namespace

extern "C" {

int32_t dir_force(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                  const float *d_field, int32_t nx, int32_t ny, int32_t nz, float *d_updated, double *sums)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    return single_step(h, variant, alpha, d_static, d_moving, d_field, nx, ny, nz, nullptr, d_updated, sums);
}

int32_t dir_step(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                 const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma, int32_t radius,
                 float *d_field_out, double *sums)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!(sigma > 0.0) || !isfinite(sigma)) return DIR_EINVAL;
    const int R = resolve_radius(sigma, radius);
    if (R < 0 || R > DIR_MAX_RADIUS) return DIR_EINVAL;
    const GaussTaps taps = make_taps(sigma, R);
    return single_step(h, variant, alpha, d_static, d_moving, d_field, nx, ny, nz, &taps, d_field_out, sums);
}

int32_t dir_similarity(dir_handle *h, const float *d_static, const float *d_moving, const float *d_field, int32_t nx,
                       int32_t ny, int32_t nz, double *mse, double *cc)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!d_static || !d_moving || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    const Dims d{nx, ny, nz};
    DIR_TRY(h->partials.ensure(sizeof(double) * 6 * (size_t)similarity_blocks(d)));
    DIR_TRY(h->history.ensure(sizeof(double) * 6));
    Ctx c{h->stream, &h->timer};
    DIR_TRY(launch_similarity(c, d_moving, d_static, d_field, d, h->partials.as<double>(), h->history.as<double>()));
    rc = finish(h);
    if (rc != DIR_OK) return rc;
    double e[6];
    rc = copy_to_host(h, e, h->history.p, sizeof e);
    if (rc != DIR_OK) return rc;
    const double n = (double)d.n();
    if (mse) *mse = e[5] / n;
    if (cc) {
        const double cov = n * e[4] - e[0] * e[1], vs = n * e[2] - e[0] * e[0], vm = n * e[3] - e[1] * e[1];
        *cc = (vs > 0.0 && vm > 0.0) ? cov / sqrt(vs * vm) : __builtin_nan("");
    }
    return DIR_OK;
}

int32_t dir_step_stored(dir_handle *h, int32_t storage, int32_t variant, double alpha, const float *d_static,
                        const float *d_moving, const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma,
                        int32_t radius, float *d_field_out, double *sums)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (!(sigma > 0.0) || !isfinite(sigma)) return DIR_EINVAL;
    const int R = resolve_radius(sigma, radius);
    if (R < 0 || R > DIR_MAX_RADIUS) return DIR_EINVAL;
    const GaussTaps taps = make_taps(sigma, R);
    return single_step(h, variant, alpha, d_static, d_moving, d_field, nx, ny, nz, &taps, d_field_out, sums,
                       storage);
}

// dir_step with its intermediates in the library's fixed scratch array: the
// same kernels, launch shapes and reduction order, so the same results; no
// device or host allocation and no timing events.
int32_t dir_step_noalloc(dir_handle *h, int32_t variant, double alpha, const float *d_static, const float *d_moving,
                         const float *d_field, int32_t nx, int32_t ny, int32_t nz, double sigma, int32_t radius,
                         float *d_field_out, double *sums)
{
    // arguments and the scratch size first (host arithmetic only, no device call)
    if (!(sigma > 0.0) || !isfinite(sigma)) return DIR_EINVAL;
    const int R = resolve_radius(sigma, radius);
    if (R < 0 || R > DIR_MAX_RADIUS) return DIR_EINVAL;
    int rc = check_step_args(variant, alpha, d_static, d_moving, d_field, nx, ny, nz, d_field_out, kStoreF32);
    if (rc != DIR_OK) return rc;
    const Dims d{nx, ny, nz};
    // layout: level state, history entry, sums, u, then D and P as the variant needs them
    const size_t n = (size_t)d.n();
    const bool pre = variant == kActive || variant == kDouble || variant == kInverseConsistent;
    const size_t off_hist = align256(sizeof(LevelState));
    const size_t off_part = off_hist + align256(sizeof(double) * 4);
    const size_t off_u = off_part + align256(sizeof(double) * 3 * (size_t)force_blocks(d));
    const size_t off_D = off_u + align256(sizeof(float) * 3 * n);
    const size_t off_P = off_D + (pre ? align256(sizeof(float) * n) : 0);
    const size_t need = off_P + (variant == kInverseConsistent ? align256(sizeof(float) * n) : 0);
    if (need > (size_t)DIR_NOALLOC_SCRATCH_BYTES) {
        char buf[192];
        snprintf(buf, sizeof buf, "dir_step_noalloc: %dx%dx%d needs %zu bytes of scratch, more than its %zu", nx, ny,
                 nz, need, (size_t)DIR_NOALLOC_SCRATCH_BYTES);
        g_last_error = buf;
        return DIR_EINVAL;
    }
    rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    char *base = static_cast<char *>(scratch_of(h->device));
    if (!base) {
        g_last_error = "dir_step_noalloc: no scratch array on this device";
        return DIR_EDEVICE;
    }
    StepBufs b;
    b.st = reinterpret_cast<LevelState *>(base);
    b.history = reinterpret_cast<double *>(base + off_hist);
    b.partials = reinterpret_cast<double *>(base + off_part);
    b.u = base + off_u;
    b.D = pre ? base + off_D : nullptr;
    b.P = variant == kInverseConsistent ? base + off_P : nullptr;
    const GaussTaps taps = make_taps(sigma, R);
    Ctx c{h->stream, nullptr};  // untimed: no events are created
    DIR_TRY(enqueue_step(c, b, variant, alpha, d_static, d_moving, d_field, d, &taps, d_field_out, kStoreF32));
    DIR_TRY(hipStreamSynchronize(h->stream));
    return read_step_sums(h, b.history, sums);
}

}  // extern "C"

namespace {

// Everything one registration, or a lockstep batch of registrations, needs to
// enqueue its kernels: validated arguments and level sizes (arrays indexed by
// registration), the history layout and the workspace strides between
// registrations.
struct RegSizes {
    size_t pyr, img0, pre, field, img_a, img_b, partials, history, state;
    size_t total() const
    {
        return 2 * pyr + 2 * img0 + 2 * pre + 2 * field + img_a + img_b + partials + history + state;
    }
};

struct RegPlan {
    int count = 1;
    const float *S[kMaxBatch], *M[kMaxBatch];
    float *out[kMaxBatch];
    int variant[kMaxBatch], K[kMaxBatch];
    float alpha2[kMaxBatch];
    double eps[kMaxBatch];
    Dims dims[kMaxBatch][DIR_MAX_LEVELS];  // level sizes, finest first
    int storage, L;
    GaussTaps taps, taps_yz;           // field smoothing: x pass (force kernel), y and z passes
    bool mm;                           // physical units (DIR_UNITS_MM)
    double h[3];                       // voxel sizes of the input grid, mm (1 in voxel units)
    Metric metric[DIR_MAX_LEVELS];     // physical units, per level (finest first)
    bool presmooth;                    // image_sigma > 0
    GaussTaps img_x, img_yz;           // the images' pre-smoothing Gaussian
    int iters[DIR_MAX_LEVELS];
    int64_t total_iters;
    int64_t hist_off[DIR_MAX_LEVELS];
    RegSizes stride;  // bytes between registrations in each workspace buffer
};

// Parameter checks of a registration that need no pointers.
int check_register_params(int32_t nx, int32_t ny, int32_t nz, const dir_params *p)
{
    if (!p || !dims_ok(nx, ny, nz)) return DIR_EINVAL;
    if (p->struct_size != (int32_t)sizeof(dir_params)) return DIR_EINVAL;
    if (p->storage < kStoreF32 || p->storage > kStoreBF16) return DIR_EINVAL;
    if (p->variant < kPassive || p->variant > kInverseConsistent) return DIR_EINVAL;
    if (!(p->alpha > 0.0) || !isfinite(p->alpha) || !(p->sigma > 0.0) || !isfinite(p->sigma)) return DIR_EINVAL;
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return DIR_EINVAL;
    if (p->levels < 1 || p->levels > DIR_MAX_LEVELS) return DIR_EINVAL;
    for (int l = 0; l < p->levels; ++l)
        if (p->iters[l] < 0) return DIR_EINVAL;
    if (p->units != DIR_UNITS_VOXELS && p->units != DIR_UNITS_MM) return DIR_EINVAL;
    if (!(p->image_sigma >= 0.0) || !isfinite(p->image_sigma)) return DIR_EINVAL;
    if (p->units == DIR_UNITS_VOXELS) {  // in mm the radii depend on the spacing (checked with it)
        const int R = resolve_radius(p->sigma, p->radius);
        if (R < 0 || R > DIR_MAX_RADIUS) return DIR_EINVAL;
        if (p->image_sigma > 0.0 && resolve_radius(p->image_sigma, 0) > DIR_MAX_RADIUS) return DIR_EINVAL;
    } else if (p->radius > DIR_MAX_RADIUS) {
        return DIR_EINVAL;
    }
    return DIR_OK;
}

// Bytes of every workspace buffer a registration needs (parameters checked).
RegSizes register_sizes(int32_t nx, int32_t ny, int32_t nz, const dir_params *p)
{
    RegSizes z;
    const int L = p->levels;
    int64_t total_iters = 0;
    for (int l = 0; l < L; ++l) total_iters += p->iters[l];
    Dims d{nx, ny, nz};
    const size_t n0 = (size_t)d.n();
    const size_t es = storage_bytes(p->storage);  // bytes per stored value
    size_t pyr = 0, nb = 0;
    for (int k = 0; k < L; ++k) {
        if (k > 0) {
            d = coarser(d);
            pyr += (size_t)d.n();
        }
        nb = std::max(nb, (size_t)force_blocks(d));
    }
    const bool pre = p->variant == kActive || p->variant == kDouble || p->variant == kInverseConsistent;
    z.pyr = L > 1 ? es * pyr : 0;                     // S and M, levels 1..
    z.img0 = p->storage != kStoreF32 ? es * n0 : 0;   // S and M, finest level, 16-bit copies
    z.pre = p->image_sigma > 0.0 ? es * (n0 + pyr) : 0;  // S and M pre-smoothed, every level
    z.field = es * 3 * n0;                            // v and the x-smoothed u
    z.img_a = pre ? es * n0 : 0;                      // D
    z.img_b = p->variant == kInverseConsistent ? sizeof(float) * n0 : 0;  // P, FP32
    z.partials = sizeof(double) * 3 * nb;
    z.history = sizeof(double) * 4 * (size_t)(total_iters > 0 ? total_iters : 1);
    z.state = sizeof(LevelState) * DIR_MAX_LEVELS;
    return z;
}

// Workspace strides of a batch (validated parameters): per buffer, the
// largest registration's size rounded up to 256 bytes.
RegSizes batch_strides(int count, const int32_t *dims, const dir_params *p)
{
    RegSizes z{};
    for (int r = 0; r < count; ++r) {
        const RegSizes zr = register_sizes(dims[3 * r], dims[3 * r + 1], dims[3 * r + 2], &p[r]);
        z.pyr = std::max(z.pyr, align256(zr.pyr));
        z.img0 = std::max(z.img0, align256(zr.img0));
        z.pre = std::max(z.pre, align256(zr.pre));
        z.field = std::max(z.field, align256(zr.field));
        z.img_a = std::max(z.img_a, align256(zr.img_a));
        z.img_b = std::max(z.img_b, align256(zr.img_b));
        z.partials = std::max(z.partials, align256(zr.partials));
        z.history = std::max(z.history, align256(zr.history));
        z.state = std::max(z.state, align256(zr.state));
    }
    return z;
}

}  // namespace

namespace dir {

size_t workspace_now(const dir_handle *h)
{
    size_t b = h->pyr_s.bytes + h->pyr_m.bytes + h->img_a.bytes + h->img_b.bytes + h->img0_s.bytes +
               h->img0_m.bytes + h->pre_s.bytes + h->pre_m.bytes + h->partials.bytes + h->history.bytes +
               h->state.bytes;
    for (const auto &f : h->field) b += f.bytes;
    return b;
}

size_t workspace_after(const dir_handle *h, int32_t nx, int32_t ny, int32_t nz, const dir_params *p)
{
    const RegSizes z = register_sizes(nx, ny, nz, p);
    auto mx = [](size_t a, size_t b) { return a > b ? a : b; };
    return mx(h->pyr_s.bytes, z.pyr) + mx(h->pyr_m.bytes, z.pyr) + mx(h->img0_s.bytes, z.img0) +
           mx(h->img0_m.bytes, z.img0) + mx(h->pre_s.bytes, z.pre) + mx(h->pre_m.bytes, z.pre) +
           mx(h->field[0].bytes, z.field) + mx(h->field[1].bytes, z.field) + h->field[2].bytes +
           mx(h->img_a.bytes, z.img_a) + mx(h->img_b.bytes, z.img_b) + mx(h->partials.bytes, z.partials) +
           mx(h->history.bytes, z.history) + mx(h->state.bytes, z.state);
}

size_t workspace_after_batch(const dir_handle *h, int32_t count, const int32_t *dims, const dir_params *p)
{
    const RegSizes z = batch_strides(count, dims, p);
    const size_t c = (size_t)count;
    auto mx = [c](size_t a, size_t b) { return a > c * b ? a : c * b; };
    return mx(h->pyr_s.bytes, z.pyr) + mx(h->pyr_m.bytes, z.pyr) + mx(h->img0_s.bytes, z.img0) +
           mx(h->img0_m.bytes, z.img0) + mx(h->pre_s.bytes, z.pre) + mx(h->pre_m.bytes, z.pre) +
           mx(h->field[0].bytes, z.field) + mx(h->field[1].bytes, z.field) + h->field[2].bytes +
           mx(h->img_a.bytes, z.img_a) + mx(h->img_b.bytes, z.img_b) + mx(h->partials.bytes, z.partials) +
           mx(h->history.bytes, z.history) + mx(h->state.bytes, z.state);
}

void workspace_release(dir_handle *h)
{
    h->pyr_s.release();
    h->pyr_m.release();
    for (auto &f : h->field) f.release();
    h->img_a.release();
    h->img_b.release();
    h->img0_s.release();
    h->img0_m.release();
    h->pre_s.release();
    h->pre_m.release();
    h->partials.release();
    h->history.release();
    h->state.release();
    if (h->graph_exec) {
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
        h->graph_key.clear();
    }
}

}  // namespace dir

extern "C" int32_t dir_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const dir_params *params, uint64_t *bytes)
{
    if (!bytes) return DIR_EINVAL;
    const int rc = check_register_params(nx, ny, nz, params);
    if (rc != DIR_OK) return rc;
    *bytes = (uint64_t)register_sizes(nx, ny, nz, params).total();
    return DIR_OK;
}

namespace {

// Fill the per-registration entries r of a plan from p (validated).
void plan_entry(RegPlan &pl, int r, const float *S, const float *M, float *out, Dims d, const dir_params *p)
{
    pl.dims[r][0] = d;
    for (int k = 1; k < p->levels; ++k) pl.dims[r][k] = coarser(pl.dims[r][k - 1]);
    pl.S[r] = S;
    pl.M[r] = M;
    pl.out[r] = out;
    pl.variant[r] = p->variant;
    pl.K[r] = p->compose_iters < 0 ? DIR_DEFAULT_COMPOSE_ITERS : p->compose_iters;
    pl.alpha2[r] = (float)(p->alpha * p->alpha);
    pl.eps[r] = p->eps;
}

// The parts of a plan every registration of a batch shares (from p and the
// voxel sizes `spacing`, NULL in voxel units): the Gaussians of the field and
// of the images' pre-smoothing per axis, and in physical units the metric of
// every level.  DIR_EINVAL for a radius beyond DIR_MAX_RADIUS.
int plan_shared(RegPlan &pl, const dir_params *p, const double *spacing)
{
    pl.storage = p->storage;
    pl.L = p->levels;
    pl.mm = p->units == DIR_UNITS_MM;
    if (pl.mm && !spacing) return DIR_EINVAL;
    double sv[3], si[3];
    int rv[3], ri[3];
    for (int a = 0; a < 3; ++a) {
        pl.h[a] = pl.mm ? spacing[a] : 1.0;
        sv[a] = p->sigma / pl.h[a];
        rv[a] = resolve_radius(sv[a], p->radius);
        si[a] = p->image_sigma / pl.h[a];
        ri[a] = p->image_sigma > 0.0 ? resolve_radius(si[a], 0) : 0;
        if (rv[a] > DIR_MAX_RADIUS || ri[a] > DIR_MAX_RADIUS) return DIR_EINVAL;
    }
    pl.taps = make_taps(sv[0], rv[0]);
    pl.taps_yz = pl.mm ? make_taps_yz(sv[1], rv[1], sv[2], rv[2]) : pl.taps;
    pl.presmooth = p->image_sigma > 0.0;
    if (pl.presmooth) {
        pl.img_x = make_taps(si[0], ri[0]);
        pl.img_yz = make_taps_yz(si[1], ri[1], si[2], ri[2]);
    }
    if (pl.mm) {
        // s_a = sqrt(K) / h_a with K the mean squared voxel size; norms in mm
        // with the level's voxel sizes 2^k h_a
        const double K = (pl.h[0] * pl.h[0] + pl.h[1] * pl.h[1] + pl.h[2] * pl.h[2]) / 3.0;
        for (int k = 0; k < pl.L; ++k)
            for (int a = 0; a < 3; ++a) {
                const double sa = sqrt(K) / pl.h[a], hk = ldexp(pl.h[a], k);
                pl.metric[k].gs[a] = (float)(0.5 * sa);
                pl.metric[k].os[a] = (float)sa;
                pl.metric[k].nw[a] = (float)(hk * hk);
            }
    }
    int64_t off = 0;
    for (int k = 0; k < pl.L; ++k) {
        pl.iters[k] = p->iters[k];  // coarsest first
        pl.hist_off[k] = off;
        off += p->iters[k];
    }
    pl.total_iters = off;
    return DIR_OK;
}

// Whether two float ranges of na and nb elements share memory.
bool overlap(const float *a, size_t na, const float *b, size_t nb)
{
    const char *pa = reinterpret_cast<const char *>(a), *pb = reinterpret_cast<const char *>(b);
    return pa < pb + sizeof(float) * nb && pb < pa + sizeof(float) * na;
}

// The output field must not overlap either input.
bool disjoint_io(const float *S, const float *M, const float *out, size_t n)
{
    const char *out_b = reinterpret_cast<const char *>(out);
    for (const float *in : {S, M}) {
        const char *b = reinterpret_cast<const char *>(in);
        if (b < out_b + 3 * sizeof(float) * n && out_b < b + sizeof(float) * n) return false;
    }
    return true;
}

bool spacing_ok(const double *spacing_mm)
{
    if (spacing_mm)
        for (int k = 0; k < 3; ++k)
            if (!(spacing_mm[k] > 0.0) || !isfinite(spacing_mm[k])) return false;
    return true;
}

// Validate the arguments of a registration and size the workspace for it.
int plan_register(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny, int32_t nz,
                  const double *spacing_mm, const dir_params *p, float *d_field_out, RegPlan &pl)
{
    if (!d_static || !d_moving || !d_field_out) return DIR_EINVAL;
    int rc = check_register_params(nx, ny, nz, p);
    if (rc != DIR_OK) return rc;
    if (!spacing_ok(spacing_mm)) return DIR_EINVAL;
    if (!disjoint_io(d_static, d_moving, d_field_out, (size_t)((int64_t)nx * ny * nz))) return DIR_EINVAL;
    rc = plan_shared(pl, p, spacing_mm);
    if (rc != DIR_OK) return rc;

    const RegSizes z = register_sizes(nx, ny, nz, p);
    if (z.pyr) {
        DIR_TRY(h->pyr_s.ensure(z.pyr));
        DIR_TRY(h->pyr_m.ensure(z.pyr));
    }
    if (z.img0) {
        DIR_TRY(h->img0_s.ensure(z.img0));
        DIR_TRY(h->img0_m.ensure(z.img0));
    }
    if (z.pre) {
        DIR_TRY(h->pre_s.ensure(z.pre));
        DIR_TRY(h->pre_m.ensure(z.pre));
    }
    DIR_TRY(h->field[0].ensure(z.field));
    DIR_TRY(h->field[1].ensure(z.field));
    if (z.img_a) DIR_TRY(h->img_a.ensure(z.img_a));
    if (z.img_b) DIR_TRY(h->img_b.ensure(z.img_b));
    DIR_TRY(h->partials.ensure(z.partials));
    DIR_TRY(h->history.ensure(z.history));
    DIR_TRY(h->state.ensure(z.state));

    pl.count = 1;
    plan_entry(pl, 0, d_static, d_moving, d_field_out, Dims{nx, ny, nz}, p);
    pl.stride = z;
    return DIR_OK;
}

// Validate a lockstep batch and size the workspace for it: `count`
// registrations, of sizes dims[3r .. 3r+2] (nx, ny, nz), whose parameters
// agree in everything the iteration schedule and the smoothing depend on
// (levels, iterations per level, sigma, radius, storage); size, variant,
// alpha, eps and the composition steps may differ.  spacing_mm: NULL or
// three values per registration.
int plan_batch(dir_handle *h, int32_t count, const float *const *S, const float *const *M, const int32_t *dims,
               const double *spacing_mm, const dir_params *p, float *const *out, RegPlan &pl)
{
    if (count < 1 || count > DIR_MAX_BATCH || !S || !M || !dims || !p || !out) return DIR_EINVAL;
    size_t n[kMaxBatch];
    for (int r = 0; r < count; ++r) {
        const int32_t nx = dims[3 * r], ny = dims[3 * r + 1], nz = dims[3 * r + 2];
        if (!S[r] || !M[r] || !out[r]) return DIR_EINVAL;
        const int rc = check_register_params(nx, ny, nz, &p[r]);
        if (rc != DIR_OK) return rc;
        if (spacing_mm && !spacing_ok(spacing_mm + 3 * r)) return DIR_EINVAL;
        if (p[r].levels != p[0].levels || p[r].sigma != p[0].sigma || p[r].storage != p[0].storage ||
            p[r].units != p[0].units || p[r].image_sigma != p[0].image_sigma)
            return DIR_EINVAL;
        if (p[0].units == DIR_UNITS_VOXELS ? resolve_radius(p[r].sigma, p[r].radius) !=
                                                 resolve_radius(p[0].sigma, p[0].radius)
                                           : p[r].radius != p[0].radius)
            return DIR_EINVAL;
        if (p[0].units == DIR_UNITS_MM &&
            (!spacing_mm || memcmp(spacing_mm + 3 * r, spacing_mm, 3 * sizeof(double)) != 0))
            return DIR_EINVAL;  // one metric and one Gaussian per launch
        for (int l = 0; l < p[0].levels; ++l)
            if (p[r].iters[l] != p[0].iters[l]) return DIR_EINVAL;
        n[r] = (size_t)((int64_t)nx * ny * nz);
        if (!disjoint_io(S[r], M[r], out[r], n[r])) return DIR_EINVAL;
        for (int q = 0; q < r; ++q) {  // every registration writes a field of its own, read by no other
            if (overlap(out[r], 3 * n[r], out[q], 3 * n[q]) || overlap(out[r], 3 * n[r], S[q], n[q]) ||
                overlap(out[r], 3 * n[r], M[q], n[q]) || overlap(out[q], 3 * n[q], S[r], n[r]) ||
                overlap(out[q], 3 * n[q], M[r], n[r]))
                return DIR_EINVAL;
        }
    }
    const int prc = plan_shared(pl, &p[0], spacing_mm);
    if (prc != DIR_OK) return prc;
    const RegSizes z = batch_strides(count, dims, p);
    const size_t c = (size_t)count;
    if (z.pyr) {
        DIR_TRY(h->pyr_s.ensure(c * z.pyr));
        DIR_TRY(h->pyr_m.ensure(c * z.pyr));
    }
    if (z.img0) {
        DIR_TRY(h->img0_s.ensure(c * z.img0));
        DIR_TRY(h->img0_m.ensure(c * z.img0));
    }
    if (z.pre) {
        DIR_TRY(h->pre_s.ensure(c * z.pre));
        DIR_TRY(h->pre_m.ensure(c * z.pre));
    }
    DIR_TRY(h->field[0].ensure(c * z.field));
    DIR_TRY(h->field[1].ensure(c * z.field));
    if (z.img_a) DIR_TRY(h->img_a.ensure(c * z.img_a));
    if (z.img_b) DIR_TRY(h->img_b.ensure(c * z.img_b));
    DIR_TRY(h->partials.ensure(c * z.partials));
    DIR_TRY(h->history.ensure(c * z.history));
    DIR_TRY(h->state.ensure(c * z.state));

    pl.count = count;
    for (int r = 0; r < count; ++r)
        plan_entry(pl, r, S[r], M[r], out[r], Dims{dims[3 * r], dims[3 * r + 1], dims[3 * r + 2]}, &p[r]);
    pl.stride = z;
    return DIR_OK;
}

// Address of registration r's part of a workspace buffer.
template <class T = void>
T *part(const DevBuf &b, size_t stride, int r)
{
    return reinterpret_cast<T *>(static_cast<char *>(b.p) + stride * (size_t)r);
}

// A batch runs a level in lockstep while the images and fields its
// registrations stream through every iteration (about 8 stored values per
// voxel: S, M, v and u with 3 components each) fit the 256 MB last-level
// cache of an MI355X.  A larger level streams from HBM either way, and then
// (with every finer level) runs registration by registration, on as many
// concurrent streams as registrations fit that cache together: consecutive
// kernels of one registration find the field the previous one wrote still in
// the cache, which a lockstep launch carrying every registration's data would
// have evicted.
constexpr size_t kLockstepBytes = size_t(256) << 20;

bool lockstep_level(int count, int64_t voxels, size_t es)
{
    return count == 1 || 8 * es * (size_t)voxels <= kLockstepBytes;
}

// Registrations of a batch that run a level on their own concurrently: as
// many as that level's images and fields fit the last-level cache together
// (at least 1, at most kMaxLanes).  With FP32 storage a 256x256x100 level
// takes 210 MB and runs alone; with 16-bit storage two run together, which
// measured 14% faster than one after another.
constexpr int kMaxLanes = 4;

int concurrent_lanes(int count, const RegPlan &pl, int k, size_t es)
{
    size_t largest = 0;
    for (int r = 0; r < count; ++r) largest = std::max(largest, 8 * es * (size_t)pl.dims[r][k].n());
    const size_t fit = largest ? kLockstepBytes / largest : 1;
    return (int)std::max<size_t>(1, std::min<size_t>({fit, (size_t)count, (size_t)kMaxLanes}));
}

// Let lanes 1 .. lanes-1 (the handle's side streams, created on first use)
// start after the work enqueued so far on the handle's stream.
int fork_lanes(dir_handle *h, int lanes)
{
    while ((int)h->side.size() < lanes - 1) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        DIR_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        const hipError_t ee = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (ee != hipSuccess) {
            (void)hipStreamDestroy(s);
            return fail_hip(ee, "hipEventCreateWithFlags");
        }
        h->side.push_back(s);
        h->side_done.push_back(e);
    }
    if (!h->fork_ev) DIR_TRY(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
    DIR_TRY(hipEventRecord(h->fork_ev, h->stream));
    for (int l = 0; l < lanes - 1; ++l) DIR_TRY(hipStreamWaitEvent(h->side[l], h->fork_ev, 0));
    return DIR_OK;
}

// Make the handle's stream wait for everything enqueued on lanes 1 .. lanes-1.
int join_lanes(dir_handle *h, int lanes)
{
    for (int l = 0; l < lanes - 1; ++l) {
        DIR_TRY(hipEventRecord(h->side_done[l], h->side[l]));
        DIR_TRY(hipStreamWaitEvent(h->stream, h->side_done[l], 0));
    }
    return DIR_OK;
}

// Registration r of a batch's iteration descriptors, as a batch of one.
ForceHalf one_of(const ForceHalf &b, int r)
{
    ForceHalf o;
    o.count = 1;
    o.storage = b.storage;
    o.d[0] = b.d[r];
    o.variant[0] = b.variant[r];
    o.alpha2[0] = b.alpha2[r];
    o.S[0] = b.S[r];
    o.M[0] = b.M[r];
    o.v[0] = b.v[r];
    o.D[0] = b.D[r];
    o.P[0] = b.P[r];
    o.out[0] = b.out[r];
    o.partials[0] = b.partials[r];
    o.stop_at[0] = b.stop_at[r];
    o.metric = b.metric;
    return o;
}

SumsReduce one_of(const SumsReduce &b, int r)
{
    SumsReduce o = b;
    o.count = 1;
    o.partials[0] = b.partials[r];
    o.hist[0] = b.hist[r];
    o.st[0] = b.st[r];
    o.eps[0] = b.eps[r];
    o.nb[0] = b.nb[r];
    o.inv_n[0] = b.inv_n[r];
    return o;
}

// Enqueue the kernels of a planned registration (or lockstep batch) on the
// handle's stream.  With `poll` (single registrations only), a level run
// under the stopping rule (eps > 0) reads its stop flag every 10 iterations
// and enqueues no further iterations once the rule has fired; otherwise every
// iteration is enqueued and the kernels of iterations after a registration's
// stop return at once.  A batch runs each iteration of all its registrations
// as one pre-warp, one force and one smoothing launch.
int enqueue_register(dir_handle *h, const RegPlan &pl, bool poll)
{
    const int L = pl.L, st_fmt = pl.storage, B = pl.count;
    const GaussTaps &taps = pl.taps, &taps_yz = pl.taps_yz;
    const RegSizes &zs = pl.stride;
    const size_t es = storage_bytes(st_fmt);
    const bool f32 = st_fmt == kStoreF32;
    Ctx c{h->stream, &h->timer};

    // ---- image pyramids in the storage format (Sec 2.3) ----
    // Level 1 is restricted from the caller's FP32 images; with 16-bit
    // storage the finest level itself is a converted copy.  Registrations of
    // a batch that are given the same image (the same device pointer and
    // size) share its pyramid: it is built once.
    const void *Sk[kMaxBatch][DIR_MAX_LEVELS], *Mk[kMaxBatch][DIR_MAX_LEVELS];
    // img[r] -> pyramid pyr[r][.] in pyr_buf's part r (or 16-bit copy img0's part r)
    auto pyramid = [&](const float *const *img, const void *(*pyr)[DIR_MAX_LEVELS], const DevBuf &pyr_buf,
                       const DevBuf &img0) -> int {
        for (int r = 0; r < B; ++r) {
            int same = -1;
            for (int q = 0; q < r && same < 0; ++q)
                if (img[q] == img[r] && pl.dims[q][0].nx == pl.dims[r][0].nx &&
                    pl.dims[q][0].ny == pl.dims[r][0].ny && pl.dims[q][0].nz == pl.dims[r][0].nz)
                    same = q;
            if (same >= 0) {
                for (int k = 0; k < L; ++k) pyr[r][k] = pyr[same][k];
                continue;
            }
            const Dims *dims = pl.dims[r];
            pyr[r][0] = img[r];
            size_t off = 0;
            for (int k = 1; k < L; ++k) {
                char *dst = part<char>(pyr_buf, zs.pyr, r) + es * off;
                h->timer.level = k;
                DIR_TRY(launch_restrict(c, pyr[r][k - 1], k == 1 ? kStoreF32 : st_fmt, dims[k - 1], dst, st_fmt,
                                        dims[k]));
                pyr[r][k] = dst;
                off += (size_t)dims[k].n();
            }
            if (!f32) {
                h->timer.level = 0;
                void *dst = part(img0, zs.img0, r);
                DIR_TRY(launch_convert(c, img[r], kStoreF32, dst, st_fmt, dims[0].n()));
                pyr[r][0] = dst;
            }
        }
        return DIR_OK;
    };
    {
        int rc = pyramid(pl.S, Sk, h->pyr_s, h->img0_s);
        if (rc == DIR_OK) rc = pyramid(pl.M, Mk, h->pyr_m, h->img0_m);
        if (rc != DIR_OK) return rc;
    }

    // ---- optional pre-smoothing of every level's images (Sec 2.5 low-pass
    // filter on images): from the unsmoothed level into pre_buf's part r, in
    // the storage format; the fields' buffers serve as FP32 scratch (they
    // are set up after this).  Shared images are smoothed once.
    auto presmooth = [&](const float *const *img, const void *(*pyr)[DIR_MAX_LEVELS], const DevBuf &pre_buf) -> int {
        const void *done[kMaxBatch][DIR_MAX_LEVELS];
        for (int r = 0; r < B; ++r) {
            int same = -1;
            for (int q = 0; q < r && same < 0; ++q)
                if (img[q] == img[r] && pl.dims[q][0].nx == pl.dims[r][0].nx &&
                    pl.dims[q][0].ny == pl.dims[r][0].ny && pl.dims[q][0].nz == pl.dims[r][0].nz)
                    same = q;
            if (same >= 0) {
                for (int k = 0; k < L; ++k) done[r][k] = pyr[r][k] = done[same][k];
                continue;
            }
            float *ta = part<float>(h->field[0], zs.field, r), *tb = part<float>(h->field[1], zs.field, r);
            size_t off = 0;
            for (int k = 0; k < L; ++k) {
                const Dims d = pl.dims[r][k];
                h->timer.level = k;
                char *dst = part<char>(pre_buf, zs.pre, r) + es * off;
                off += (size_t)d.n();
                if (f32) {
                    DIR_TRY(launch_smooth_x(c, static_cast<const float *>(pyr[r][k]), 1, d, pl.img_x, ta));
                    DIR_TRY(launch_smooth_yz(c, ta, 1, d, pl.img_yz, dst, kStoreF32, nullptr, 0, SumsReduce{}));
                } else {
                    DIR_TRY(launch_convert(c, pyr[r][k], st_fmt, ta, kStoreF32, d.n()));
                    DIR_TRY(launch_smooth_x(c, ta, 1, d, pl.img_x, tb));
                    DIR_TRY(launch_smooth_yz(c, tb, 1, d, pl.img_yz, ta, kStoreF32, nullptr, 0, SumsReduce{}));
                    DIR_TRY(launch_convert(c, ta, kStoreF32, dst, st_fmt, d.n()));
                }
                done[r][k] = pyr[r][k] = dst;
            }
        }
        return DIR_OK;
    };
    if (pl.presmooth) {
        int rc = presmooth(pl.S, Sk, h->pre_s);
        if (rc == DIR_OK) rc = presmooth(pl.M, Mk, h->pre_m);
        if (rc != DIR_OK) return rc;
    }

    // ---- levels, coarse to fine (Sec 2.3) ----
    // With FP32 storage the finest level's field lives in the output field
    // itself, except for the inverse-consistent variant, whose half field is
    // composed into it; 16-bit fields are converted into it at the end.
    void *fa[kMaxBatch], *fb[kMaxBatch], *final_v[kMaxBatch], *v[kMaxBatch], *xs[kMaxBatch];
    LevelState *states[kMaxBatch];
    double *hist[kMaxBatch];
    ForceHalf fh;
    fh.count = B;
    fh.storage = st_fmt;
    h->timer.level = L - 1;
    for (int r = 0; r < B; ++r) {
        fa[r] = part(h->field[0], zs.field, r);
        fb[r] = part(h->field[1], zs.field, r);
        final_v[r] = (pl.variant[r] == kInverseConsistent || !f32) ? nullptr : static_cast<void *>(pl.out[r]);
        v[r] = (L == 1 && final_v[r]) ? final_v[r] : fa[r];
        states[r] = part<LevelState>(h->state, zs.state, r);
        hist[r] = part<double>(h->history, zs.history, r);
        fh.variant[r] = pl.variant[r];
        fh.alpha2[r] = pl.alpha2[r];
        fh.D[r] = part(h->img_a, zs.img_a, r);
        fh.P[r] = part(h->img_b, zs.img_b, r);
        fh.partials[r] = part<double>(h->partials, zs.partials, r);
        DIR_TRY(launch_zero(c, v[r], 3 * pl.dims[r][L - 1].n(), st_fmt));
    }
    SumsReduce red;
    red.count = B;
    // Level k of registration r enqueued on cr: the prolongation into it, the
    // level reset, and its entries of fh and red.
    auto setup_level = [&](Ctx &cr, int r, int k) -> int {
        const int li = L - 1 - k;
        const Dims d = pl.dims[r][k];
        fh.d[r] = d;
        red.nb[r] = (int)force_blocks(d);
        red.inv_n[r] = 1.0 / (double)d.n();
        if (k < L - 1) {
            void *dst = (k == 0 && final_v[r]) ? final_v[r] : (v[r] == fa[r] ? fb[r] : fa[r]);
            DIR_TRY(launch_prolong(cr, v[r], pl.dims[r][k + 1], dst, d, st_fmt));
            v[r] = dst;
        }
        xs[r] = v[r] == fa[r] ? fb[r] : fa[r];  // x-smoothed u of this level
        LevelState *st = states[r] + li;
        DIR_TRY(launch_level_reset(cr, st));
        red.partials[r] = fh.partials[r];
        red.hist[r] = hist[r] + 4 * pl.hist_off[li];
        red.st[r] = st;
        red.eps[r] = pl.eps[r];
        // Without the stopping rule the flag never changes, so the kernels
        // are not given it (each would otherwise read it first).
        fh.stop_at[r] = pl.eps[r] > 0.0 ? &st->stop_at : nullptr;
        fh.S[r] = Sk[r][k];
        fh.M[r] = Mk[r][k];
        fh.v[r] = v[r];
        fh.out[r] = xs[r];
        fh.metric = pl.mm ? &pl.metric[k] : nullptr;
        return DIR_OK;
    };
    // The iterations of level k on cr for the registrations of `f` and `rd`
    // (fields xsv, vv), all in lockstep.
    auto run_level = [&](Ctx &cr, int k, const ForceHalf &f, const SumsReduce &rd, void *const *xsv,
                         void *const *vv) -> int {
        const int li = L - 1 - k, iters = pl.iters[li];
        for (int n = 0; n < iters; ++n) {
            // v -> xs = x-smoothed (v + dr) -> v = y,z-smoothed xs; the
            // smoothing kernel also reduces the sums of this iteration
            DIR_TRY(force_half(cr, f, taps, n));
            DIR_TRY(launch_smooth_yz(cr, f.count, xsv, 3, f.d, taps_yz, vv, st_fmt, f.stop_at, n, rd));
            if (poll && B == 1 && pl.eps[0] > 0.0 && (n + 1) % 10 == 0 && n + 1 < iters) {
                int stop_at = kNeverStopped;
                DIR_TRY(hipMemcpyAsync(&stop_at, &states[0][li].stop_at, sizeof(int), hipMemcpyDeviceToHost,
                                       cr.stream));
                DIR_TRY(hipStreamSynchronize(cr.stream));
                if (stop_at != kNeverStopped) break;
            }
        }
        return DIR_OK;
    };
    // The output field of registration r (FP32).
    auto output = [&](Ctx &cr, int r) -> int {
        h->timer.level = 0;
        const Dims d0 = pl.dims[r][0];
        if (pl.variant[r] == kInverseConsistent) DIR_TRY(launch_compose(cr, v[r], st_fmt, d0, pl.K[r], pl.out[r]));
        else if (!f32) DIR_TRY(launch_convert(cr, v[r], st_fmt, pl.out[r], kStoreF32, 3 * d0.n()));
        return DIR_OK;
    };

    // Levels in lockstep, coarse to fine, while they fit the last-level cache.
    int k = L - 1;
    for (; k >= 0; --k) {
        int64_t voxels = 0;
        for (int r = 0; r < B; ++r) voxels += pl.dims[r][k].n();
        if (!lockstep_level(B, voxels, es)) break;
        h->timer.level = k;
        for (int r = 0; r < B; ++r) {
            const int rc = setup_level(c, r, k);
            if (rc != DIR_OK) return rc;
        }
        const int rc = run_level(c, k, fh, red, xs, v);
        if (rc != DIR_OK) return rc;
    }
    if (k < 0) {
        for (int r = 0; r < B; ++r) {
            const int rc = output(c, r);
            if (rc != DIR_OK) return rc;
        }
        return DIR_OK;
    }

    // The remaining levels (and the output) registration by registration, on
    // as many streams as registrations whose level fits the cache together.
    const int lanes = concurrent_lanes(B, pl, k, es);
    int rc = lanes > 1 ? fork_lanes(h, lanes) : DIR_OK;
    if (rc != DIR_OK) return rc;
    for (int r = 0; r < B && rc == DIR_OK; ++r) {
        Ctx cr{r % lanes == 0 ? h->stream : h->side[r % lanes - 1], &h->timer};
        for (int kk = k; kk >= 0 && rc == DIR_OK; --kk) {
            h->timer.level = kk;
            rc = setup_level(cr, r, kk);
            if (rc == DIR_OK) rc = run_level(cr, kk, one_of(fh, r), one_of(red, r), &xs[r], &v[r]);
        }
        if (rc == DIR_OK) rc = output(cr, r);
    }
    const int jrc = lanes > 1 ? join_lanes(h, lanes) : DIR_OK;  // also after a failure
    return rc != DIR_OK ? rc : jrc;
}

// p: the plan's dir_params, one per registration.
GraphKey graph_key(dir_handle *h, const RegPlan &pl, const dir_params *p)
{
    GraphKey k;
    auto put = [&k](const void *x, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(x);
        k.insert(k.end(), b, b + n);
    };
    put(&pl.count, sizeof pl.count);
    for (int r = 0; r < pl.count; ++r) {
        put(&pl.S[r], sizeof pl.S[r]);
        put(&pl.M[r], sizeof pl.M[r]);
        put(&pl.out[r], sizeof pl.out[r]);
        put(&pl.dims[r][0], sizeof pl.dims[r][0]);
        put(&p[r], sizeof p[r]);
    }
    put(pl.h, sizeof pl.h);
    const DevBuf *bufs[14] = {&h->pyr_s,  &h->pyr_m,  &h->field[0], &h->field[1], &h->field[2],
                              &h->img_a,  &h->img_b,  &h->img0_s,   &h->img0_m,   &h->pre_s,
                              &h->pre_m,  &h->partials, &h->history, &h->state};
    for (const DevBuf *b : bufs) put(&b->p, sizeof b->p);
    for (hipStream_t sd : h->side) put(&sd, sizeof sd);
    return k;
}

// Capture the registration's launches into a graph and instantiate it.
int capture_register(dir_handle *h, const RegPlan &pl, hipGraphExec_t *exec)
{
    DIR_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    const int rc = enqueue_register(h, pl, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != DIR_OK) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail_hip(ei, "hipGraphInstantiate");
    return DIR_OK;
}

// Record an enqueued plan as the handle's registration in flight.
void note_inflight(dir_handle *h, const RegPlan &pl)
{
    InFlight &f = h->inflight;
    f.active = true;
    f.count = pl.count;
    f.levels = pl.L;
    f.total_iters = pl.total_iters;
    for (int li = 0; li < pl.L; ++li) f.hist_off[li] = pl.hist_off[li];
    f.hist_stride = pl.stride.history;
    f.state_stride = pl.stride.state;
}

// Enqueue a validated plan (p: its dir_params, one per registration) and
// record it as in flight.  Without a host wait inside it (no polled stopping
// rule) and without kernel timing, on a handle with graphs on and a non-null
// stream, the launches are captured once into a HIP graph, which is replayed
// while the key stays the same; otherwise they are enqueued one by one.
int submit_plan(dir_handle *h, const RegPlan &pl, const dir_params *p, bool poll)
{
    bool polled = false;
    for (int r = 0; r < pl.count; ++r) polled = polled || (poll && pl.eps[r] > 0.0);
    const bool graph = h->graphs && h->stream != nullptr && h->timer.mask == 0 && !polled;
    if (graph) {
        if (pl.count > 1) {  // the side streams a batch may fork to exist before the key is taken
            int lanes = 1;
            for (int k = 0; k < pl.L; ++k) lanes = std::max(lanes, concurrent_lanes(pl.count, pl, k, storage_bytes(pl.storage)));
            while ((int)h->side.size() < lanes - 1) {
                const int rc = fork_lanes(h, (int)h->side.size() + 2);
                if (rc != DIR_OK) return rc;
            }
        }
        GraphKey key = graph_key(h, pl, p);
        if (!h->graph_exec || key != h->graph_key) {
            if (h->graph_exec) {
                (void)hipGraphExecDestroy(h->graph_exec);
                h->graph_exec = nullptr;
                h->graph_key.clear();
            }
            const int rc = capture_register(h, pl, &h->graph_exec);
            if (rc != DIR_OK) {
                h->graph_exec = nullptr;
                return rc;
            }
            h->graph_key.swap(key);
        }
        DIR_TRY(hipGraphLaunch(h->graph_exec, h->stream));
    } else {
        const int rc = enqueue_register(h, pl, poll);
        if (rc != DIR_OK) return rc;
    }
    note_inflight(h, pl);
    return DIR_OK;
}

// Validate one registration and submit it (submit_plan).
int submit_register(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                    int32_t nz, const double *spacing_mm, const dir_params *p, float *d_field_out, bool poll)
{
    RegPlan pl;
    const int rc = plan_register(h, d_static, d_moving, nx, ny, nz, spacing_mm, p, d_field_out, pl);
    if (rc != DIR_OK) return rc;
    return submit_plan(h, pl, p, poll);
}

// Fill one registration's statistics from its level states and history.
bool fill_stats(const InFlight &f, const LevelState *hs, const double *hh, dir_stats *stats)
{
    bool finite = true;
    int64_t packed = 0;
    double last_mse = 0.0, last_l = __builtin_nan("");
    for (int li = 0; li < f.levels; ++li) {
        for (int n = 0; n < hs[li].iters_run; ++n) {
            const double *e = &hh[(size_t)4 * (f.hist_off[li] + n)];
            if (!isfinite(e[0]) || !isfinite(e[1]) || !isfinite(e[2])) finite = false;
            if (stats && stats->history && packed < stats->history_capacity)
                memcpy(stats->history + 4 * packed, e, sizeof(double) * 4);
            last_mse = e[2];
            last_l = e[3];
            ++packed;
        }
    }
    if (stats) {
        stats->levels = f.levels;
        for (int li = 0; li < DIR_MAX_LEVELS; ++li) stats->iters_run[li] = li < f.levels ? hs[li].iters_run : 0;
        stats->mse_final = last_mse;
        stats->relnorm_final = last_l;
        stats->history_len = (int32_t)(stats->history ? (packed < stats->history_capacity ? packed
                                                                                         : stats->history_capacity)
                                                      : 0);
    }
    return finite;
}

// Wait for the registration (or batch) in flight and fill stats[0 .. count-1]
// (may be NULL) and, if not NULL, status[0 .. count-1] (DIR_OK or
// DIR_ENUMERIC each).  DIR_ENUMERIC if any registration's sums are not
// finite.
int collect_register(dir_handle *h, dir_stats *stats, int32_t *status = nullptr)
{
    const InFlight f = h->inflight;
    h->inflight.active = false;
    // the level states and histories of all registrations: two copies into
    // the pinned stage, one wait
    const size_t sbytes = f.state_stride * (size_t)(f.count - 1) + sizeof(LevelState) * (size_t)f.levels;
    const size_t hoff = (sbytes + 255) & ~(size_t)255;
    const size_t hbytes =
        f.total_iters > 0 ? f.hist_stride * (size_t)(f.count - 1) + sizeof(double) * 4 * (size_t)f.total_iters : 0;
    if (hoff + hbytes > h->stage_bytes) {
        DIR_TRY(hipStreamSynchronize(h->stream));  // the old stage may still be a copy's target
        if (h->stage) (void)hipHostFree(h->stage);
        h->stage = nullptr;
        h->stage_bytes = 0;
        DIR_TRY(hipHostMalloc(&h->stage, hoff + hbytes));
        h->stage_bytes = hoff + hbytes;
    }
    char *stage = static_cast<char *>(h->stage);
    DIR_TRY(hipMemcpyAsync(stage, h->state.p, sbytes, hipMemcpyDeviceToHost, h->stream));
    if (hbytes) DIR_TRY(hipMemcpyAsync(stage + hoff, h->history.p, hbytes, hipMemcpyDeviceToHost, h->stream));
    int rc = finish(h);
    if (rc != DIR_OK) return rc;
    bool finite = true;
    for (int r = 0; r < f.count; ++r) {
        const LevelState *hs = reinterpret_cast<const LevelState *>(stage + f.state_stride * (size_t)r);
        const double *hh = reinterpret_cast<const double *>(stage + hoff + f.hist_stride * (size_t)r);
        const bool ok = fill_stats(f, hs, hh, stats ? &stats[r] : nullptr);
        if (status) status[r] = ok ? DIR_OK : DIR_ENUMERIC;
        if (!ok) finite = false;
    }
    return finite ? DIR_OK : DIR_ENUMERIC;
}

}  // namespace

namespace dir {

int collect_each(dir_handle *h, dir_stats *stats, int32_t *status)
{
    const int rc = enter(h);
    if (rc != DIR_OK) return rc;
    if (!h->inflight.active) return DIR_EINVAL;
    return collect_register(h, stats, status);
}

}  // namespace dir

extern "C" {

int32_t dir_register(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                     int32_t nz, const double *spacing_mm, const dir_params *p, float *d_field_out,
                     dir_stats *stats)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    if (stats && stats->struct_size != (int32_t)sizeof(dir_stats)) return DIR_EINVAL;
    rc = submit_register(h, d_static, d_moving, nx, ny, nz, spacing_mm, p, d_field_out, true);
    if (rc != DIR_OK) return rc;
    return collect_register(h, stats);
}

int32_t dir_register_async(dir_handle *h, const float *d_static, const float *d_moving, int32_t nx, int32_t ny,
                           int32_t nz, const double *spacing_mm, const dir_params *p, float *d_field_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    return submit_register(h, d_static, d_moving, nx, ny, nz, spacing_mm, p, d_field_out, false);
}

int32_t dir_wait(dir_handle *h, dir_stats *stats)
{
    int rc = enter(h);
    if (rc != DIR_OK) return rc;
    if (!h->inflight.active) return DIR_EINVAL;
    if (stats)
        for (int r = 0; r < h->inflight.count; ++r)
            if (stats[r].struct_size != (int32_t)sizeof(dir_stats)) return DIR_EINVAL;
    return collect_register(h, stats);
}

int32_t dir_autotune(dir_handle *h, int32_t nx, int32_t ny, int32_t nz, const dir_params *p, int32_t count,
                     int32_t *depths)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    rc = check_register_params(nx, ny, nz, p);
    if (rc != DIR_OK) return rc;
    if (count < 1 || count > DIR_MAX_BATCH) return DIR_EINVAL;
    const int st = p->storage;
    const size_t es = storage_bytes(st);
    const GaussTaps taps = make_taps(p->sigma, resolve_radius(p->sigma, p->radius));
    Dims d{nx, ny, nz};
    const size_t field = align256(3 * es * (size_t)d.n());  // one registration's finest field
    DIR_TRY(h->field[0].ensure((size_t)count * field));
    DIR_TRY(h->field[1].ensure((size_t)count * field));
    Ctx c{h->stream, nullptr};
    // the depth decides the work distribution only, so the values do not matter: zeros
    DIR_TRY(launch_zero(c, h->field[0].p, (int64_t)(count * field / es), st));
    for (int k = 0; k < p->levels; ++k) {
        if (k > 0) d = coarser(d);
        const void *in[kMaxBatch];
        void *out[kMaxBatch];
        for (int r = 0; r < count; ++r) {
            in[r] = part(h->field[0], field, r);
            out[r] = part(h->field[1], field, r);
        }
        int chosen = 0;
        DIR_TRY(tune_smooth_yz(c, count, in, 3, d, taps, out, st, 3, &chosen));
        if (depths) depths[k] = chosen;
    }
    return DIR_OK;
}

void dir_autotune_clear(void) { clear_smooth_yz_tuning(); }

int32_t dir_register_batch_async(dir_handle *h, int32_t count, const float *const *d_static,
                                 const float *const *d_moving, const int32_t *dims, const double *spacing_mm,
                                 const dir_params *params, float *const *d_field_out)
{
    int rc = enter_idle(h);
    if (rc != DIR_OK) return rc;
    RegPlan pl;
    rc = plan_batch(h, count, d_static, d_moving, dims, spacing_mm, params, d_field_out, pl);
    if (rc != DIR_OK) return rc;
    return submit_plan(h, pl, params, false);
}

int32_t dir_register_batch(dir_handle *h, int32_t count, const float *const *d_static,
                           const float *const *d_moving, const int32_t *dims, const double *spacing_mm,
                           const dir_params *params, float *const *d_field_out, dir_stats *stats)
{
    if (count < 1 || count > DIR_MAX_BATCH) return DIR_EINVAL;
    if (stats)
        for (int r = 0; r < count; ++r)
            if (stats[r].struct_size != (int32_t)sizeof(dir_stats)) return DIR_EINVAL;
    const int rc = dir_register_batch_async(h, count, d_static, d_moving, dims, spacing_mm, params, d_field_out);
    if (rc != DIR_OK) return rc;
    return collect_register(h, stats);
}

}  // extern "C"
