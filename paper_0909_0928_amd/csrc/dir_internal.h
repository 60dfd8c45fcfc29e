// Internal declarations of libdemons: kernel launchers, launch context and
// per-kernel event timing.  Not part of the public ABI (see include/demons.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace dir {

constexpr int kMaxRadius = 16;
constexpr int kBlockX = 64;   // one wavefront along x
constexpr int kBlockY = 4;    // four wavefronts per workgroup

// Variant codes, numerically equal to dir_variant; kMixedVariants selects
// per-registration variants in a lockstep batch.
enum Variant { kMixedVariants = -1, kPassive = 0, kEvolved = 1, kActive = 2, kDouble = 3, kInverseConsistent = 4 };

// Registrations one launch of the per-iteration kernels can carry: a lockstep
// batch runs every iteration of all its registrations as one pre-warp, one
// force and one smoothing launch (one per tile class when their sizes differ).
constexpr int kMaxBatch = 8;

// Storage formats of images and fields inside a registration, numerically
// equal to dir_storage: FP32, IEEE half, bfloat16.
enum Storage { kStoreF32 = 0, kStoreF16 = 1, kStoreBF16 = 2 };
inline unsigned storage_bytes(int st) { return st == kStoreF32 ? 4u : 2u; }

// Bytes a 16-bit volume's buffer reaches past the volume's end, so that the
// 8-byte loads of a 16-bit gather (bpair16) stay in range: the workspace
// allocates them, and the buffer resources of gathered 16-bit volumes
// include them.
constexpr unsigned kPad16 = 8;

// Kernel ids for event timing; names in kKernelNames (abi.hip).
enum KernelId {
    K_FORCE = 0,     // force + x pass of the smoothing + sums (+ last-workgroup reduction)
    K_WARP,          // deformed image (dir_warp) / intensity difference (active, double force)
    K_WARP_PAIR,     // difference and sum of the two deformed images (inverse-consistent)
    K_SMOOTH_YZ,     // y and z passes of the smoothing
    K_SMOOTH_X,      // standalone x pass (dir_smooth)
    K_FINALIZE,      // standalone reduction of the sums (dir_force)
    K_LEVEL_RESET,
    K_RESTRICT,
    K_PROLONG,
    K_GRADIENT,
    K_COMPOSE,
    K_FILL,
    K_CONVERT,       // storage-format conversion (reduced-precision registrations)
    K_SIMILARITY,    // intensity error and correlation coefficient (dir_similarity)
    K_WARP_MIXED,    // pre-warp of a batch that mixes the two kinds above
    K_COUNT
};

struct Dims {
    int nx, ny, nz;
    int64_t n() const { return (int64_t)nx * ny * nz; }
};

// Normalised Gaussian taps w[j + radius], j in [-radius, radius], in FP32.
// wz: the taps of the z pass in the y/z smoothing kernel (equal to w for an
// isotropic Gaussian; for per-axis widths, w holds y's and wz z's, the
// shorter one padded with zero taps to the common radius).
struct GaussTaps {
    float w[2 * kMaxRadius + 1];
    float wz[2 * kMaxRadius + 1];
    int radius;
};

// The force in physical units, written on the voxel grid.  With voxel sizes
// h_a (mm) of the input grid and K = (h_x^2 + h_y^2 + h_z^2) / 3, the force in
// mm (gradients per mm, the squared intensity difference over K) converts to
// voxel units as dr_a = s_a f(D, s * g)_a with s_a = sqrt(K) / h_a, the same on
// every level (both K and h_a^2 scale by 4 per level); g is the voxel central
// difference.  The kernels therefore take gs[a] = s_a / 2 in place of the 1/2
// of the central difference, scale the force component a by s_a, and weight
// the norms behind the relative norm by nw[a] = h_a^2 of the level (mm^2).
struct Metric {
    float gs[3], os[3], nw[3];
};

constexpr int kNeverStopped = 0x7fffffff;

// Device-side state of one resolution level (stopping rule of Sec 2.4).
struct LevelState {
    int stop_at;        // iteration at which the rule fired (kNeverStopped if not)
    int iters_run;      // iterations completed at this level
};

// Where the per-iteration FP64 sums of the force kernel are reduced: the
// kernel that runs next (the y/z smoothing, or the standalone finalize)
// dedicates one workgroup per registration to it.
struct SumsReduce {
    int count = 0;                         // registrations; 0: nothing to reduce
    const double *partials[kMaxBatch];     // 3 * nb doubles each
    double *hist[kMaxBatch];               // level history; entry n at hist[4n]
    LevelState *st[kMaxBatch];
    double eps[kMaxBatch];
    int nb[kMaxBatch];                     // force workgroups of the registration
    double inv_n[kMaxBatch];               // 1 / voxels (the mean of D^2)
};

// Per-kernel HIP-event timing.  A timed launch goes through
// hipExtLaunchKernelGGL with a start and a stop event, which the dispatch
// itself stamps when the kernel begins and ends, so a pair measures the
// kernel's execution and not the stream around it.  Totals are kept per
// pyramid level (0 = finest; `level` is the level whose launches are being
// issued).  Events are recycled from a pool; pairs are read back by harvest()
// after the stream has completed.
constexpr int kTimerLevels = 8;

class Timer {
  public:
    uint64_t mask = 0;
    int level = 0;
    double total_ms[K_COUNT][kTimerLevels] = {};
    int64_t launches[K_COUNT][kTimerLevels] = {};

    bool on(int k) const { return (mask >> k) & 1ull; }
    hipError_t pair(hipEvent_t *start, hipEvent_t *stop);  // two events for one launch
    void record(int k, hipEvent_t start, hipEvent_t stop);  // after the launch was enqueued
    hipError_t harvest();   // stream must be complete
    void reset();
    void release();         // destroy all events

  private:
    struct Rec {
        int k, level;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool_;
    std::vector<Rec> pending_;
    hipError_t take(hipEvent_t *ev);
};

// What every launcher needs: the stream, and the timer to bracket launches.
struct Ctx {
    hipStream_t stream;
    Timer *timer;
};

// Number of workgroups (and FP64 sum slots) of the force kernel for a level.
int64_t force_blocks(Dims d);

// Force kernel for `count` registrations of sizes d[]: u = v + dr (Eqs 1-6),
// its x-smoothing with `taps` (identity taps give u), and the per-workgroup
// FP64 sums.  Every volume is in format `storage`.  Arrays are indexed by
// registration; registrations of one tile width share a launch.
struct ForceLaunch {
    int count = 1;
    int variant;                     // every registration's, or kMixedVariants
    int variants[kMaxBatch];         // per registration, with kMixedVariants
    int storage;
    float alpha2[kMaxBatch];
    const void *S[kMaxBatch], *M[kMaxBatch], *v[kMaxBatch];
    const void *D[kMaxBatch], *P[kMaxBatch];  // from the pre-warp: D (active, double, IC), P = Im + Is (IC)
    Dims d[kMaxBatch];
    const GaussTaps *taps;
    const Metric *metric = nullptr;  // NULL: voxel units (the paper's form); else physical units
    void *out[kMaxBatch];
    double *partials[kMaxBatch];     // 3 * force_blocks(d) doubles each
    const int *stop_at[kMaxBatch];   // skip when *stop_at < n (NULL: never)
    int n;
};

// Pre-warp kinds: D = M(x - v) - S (active, double) or the inverse-consistent
// pair D = Im - Is, P = Im + Is.
enum PrewarpKind { kPrewarpMixed = -1, kPrewarpDiff = 0, kPrewarpPair = 1 };

// One pre-warp launch for `count` registrations of sizes d[] (arrays indexed
// by registration; P only for the pair kind).
struct PrewarpLaunch {
    int count = 1;
    int kind;                        // every registration's, or kPrewarpMixed
    int kinds[kMaxBatch];            // per registration, with kPrewarpMixed
    int storage;
    const void *M[kMaxBatch], *S[kMaxBatch], *v[kMaxBatch];
    void *D[kMaxBatch], *P[kMaxBatch];
    const int *stop_at[kMaxBatch];
    Dims d[kMaxBatch];
    int n;
};

// ---- launchers; each returns the launch status ----------------------------
// `st`, `in_st`, `out_st`: storage format (Storage) of the volume next to it;
// volumes without one are FP32.
hipError_t launch_restrict(Ctx &c, const void *in, int in_st, Dims fine, void *out, int out_st, Dims coarse);
hipError_t launch_prolong(Ctx &c, const void *vc, Dims coarse, void *vf, Dims fine, int st);
hipError_t launch_gradient(Ctx &c, const float *img, Dims d, float *grad);
hipError_t launch_warp(Ctx &c, const float *img, const float *field, Dims d, float *out, const int *stop_at, int n);
hipError_t launch_prewarp(Ctx &c, const PrewarpLaunch &w);
hipError_t launch_force(Ctx &c, const ForceLaunch &f);
hipError_t launch_smooth_x(Ctx &c, const float *in, int ncomp, Dims d, const GaussTaps &taps, float *out);
// y and z passes for `count` registrations of sizes d[] (arrays indexed by
// registration; registrations of one z-chunk depth share a launch); red.count
// is 0 or `count`.
hipError_t launch_smooth_yz(Ctx &c, int count, const void *const *in, int ncomp, const Dims *d,
                            const GaussTaps &taps, void *const *out, int st, const int *const *stop_at, int n,
                            const SumsReduce &red);
inline hipError_t launch_smooth_yz(Ctx &c, const void *in, int ncomp, Dims d, const GaussTaps &taps, void *out,
                                   int st, const int *stop_at, int n, const SumsReduce &red)
{
    return launch_smooth_yz(c, 1, &in, ncomp, &d, taps, &out, st, &stop_at, n, red);
}
hipError_t launch_finalize(Ctx &c, const SumsReduce &red, int n);
// Time the smoothing kernel's z-chunk depths for launches of `count`
// registrations of size d (fields in[], out[] in format st, `reps` timed
// launches per depth, blocking) and keep the fastest for such launches in a
// process-wide table that launch_smooth_yz consults; *chosen receives it.
hipError_t tune_smooth_yz(Ctx &c, int count, const void *const *in, int ncomp, Dims d, const GaussTaps &taps,
                          void *const *out, int st, int reps, int *chosen);
void clear_smooth_yz_tuning();
hipError_t launch_level_reset(Ctx &c, LevelState *st);
hipError_t launch_compose(Ctx &c, const void *h, int h_st, Dims d, int K, float *out);
hipError_t launch_zero(Ctx &c, void *p, int64_t n, int st);
hipError_t launch_convert(Ctx &c, const void *in, int in_st, void *out, int out_st, int64_t n);
int64_t similarity_blocks(Dims d);
// Six FP64 sums (S, Im, S^2, Im^2, S Im, (Im - S)^2) into out[0..5]; v may be NULL.
hipError_t launch_similarity(Ctx &c, const float *M, const float *S, const float *v, Dims d, double *partials,
                             double *out);

}  // namespace dir

// Workspace accounting of a handle (abi.hip), used by the request pool.
#include "demons.h"
namespace dir {
size_t workspace_now(const dir_handle *h);
// Bytes the handle holds after a registration with these parameters
// (each buffer grows to the larger of its current and needed size).
size_t workspace_after(const dir_handle *h, int32_t nx, int32_t ny, int32_t nz, const dir_params *p);
// The same for a lockstep batch (dir_register_batch arguments).
size_t workspace_after_batch(const dir_handle *h, int32_t count, const int32_t *dims, const dir_params *p);
void workspace_release(dir_handle *h);  // free the workspace (no registration may be in flight)
// Collect what is in flight on h (one registration or a batch): stats[r]
// (struct_size set) and status[r] (DIR_OK or DIR_ENUMERIC) per registration;
// the device status of the whole as the return value.
int collect_each(dir_handle *h, dir_stats *stats, int32_t *status);
}  // namespace dir
