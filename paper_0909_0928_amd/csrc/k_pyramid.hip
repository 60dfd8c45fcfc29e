// gfx950 kernels for the image pyramid (Sec 2.3), deformed images (Sec 2.5
// interpolation kernel), plain gradients (Sec 2.5 gradient kernel) and the
// inverse-consistent output composition.
#include <string.h>

#include "device_common.h"

namespace dir {
namespace {

using namespace dev;

// ------------------------------------------------------------------------
// Pyramid (Sec 2.3)
// ------------------------------------------------------------------------
// Si, So: storage formats of the fine input and the coarse output.
template <class Si, class So>
__global__ __launch_bounds__(256) void k_restrict(const void *__restrict__ in, int nx, int ny, int nz,
                                                  void *__restrict__ out, int cx, int cy, int cz, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int i = t.x * kBlockX + threadIdx.x, j = t.y * kBlockY + threadIdx.y, k = t.z;
    if (i >= cx || j >= cy) return;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(in, Si::kBytes * (unsigned)nx * (unsigned)ny * (unsigned)nz);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(out, So::kBytes * (unsigned)cx * (unsigned)cy * (unsigned)cz);
    // FP64 sum, rounded once: coarse images feed intensity differences
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const unsigned row = (unsigned)(nx * (min(2 * j + b, ny - 1) + ny * min(2 * k + c, nz - 1)));
            s += (double)Si::load(rin, Si::kBytes * (row + (unsigned)min(2 * i, nx - 1)), 0) +
                 (double)Si::load(rin, Si::kBytes * (row + (unsigned)min(2 * i + 1, nx - 1)), 0);
        }
    So::store(rout, (float)(0.125 * s), So::kBytes * (unsigned)(i + cx * (j + cy * k)), 0);
}

// FP32 trilinear sample, at a Cell of element offsets, of a volume in format St
// addressed through a buffer resource (soff: byte offset of its plane).
template <class St>
__device__ __forceinline__ float sample_st(__amdgpu_buffer_rsrc_t r, const Cell &c, unsigned soff)
{
    constexpr unsigned E = St::kBytes;
    const float c00 = lerp1(St::load(r, E * c.o000, soff), St::load(r, E * c.o100, soff), c.tx);
    const float c10 = lerp1(St::load(r, E * c.o010, soff), St::load(r, E * c.o110, soff), c.tx);
    const float c01 = lerp1(St::load(r, E * c.o001, soff), St::load(r, E * c.o101, soff), c.tx);
    const float c11 = lerp1(St::load(r, E * c.o011, soff), St::load(r, E * c.o111, soff), c.tx);
    return lerp1(lerp1(c00, c10, c.ty), lerp1(c01, c11, c.ty), c.tz);
}

template <class St>
__global__ __launch_bounds__(256) void k_prolong(const void *__restrict__ vc, int cx, int cy, int cz,
                                                 void *__restrict__ vf, int fx, int fy, int fz, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= fx || y >= fy) return;
    constexpr unsigned E = St::kBytes;
    const unsigned Nc = (unsigned)cx * (unsigned)cy * (unsigned)cz, Nf = (unsigned)fx * (unsigned)fy * (unsigned)fz;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(vc, 3u * E * Nc), rf = make_rsrc(vf, 3u * E * Nf);
    // fine index f sits at coarse coordinate (f - 0.5) / 2
    const Cell c = make_cell(0.5f * x - 0.25f, 0.5f * y - 0.25f, 0.5f * z - 0.25f, cx, cy, cz);
    const unsigned o = E * (unsigned)(x + fx * (y + fy * z));
#pragma unroll
    for (int k = 0; k < 3; ++k) St::store(rf, 2.0f * sample_st<St>(rc, c, (unsigned)k * E * Nc), o, (unsigned)k * E * Nf);
}

__global__ __launch_bounds__(256) void k_gradient(const float *__restrict__ I, int nx, int ny, int nz,
                                                  float *__restrict__ g, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    float a, b, c;
    central_diff(I, x, y, z, nx, ny, nz, a, b, c);
    g[i] = a;
    g[N + i] = b;
    g[2 * N + i] = c;
}

// ------------------------------------------------------------------------
// Deformation (Sec 2.5 interpolation kernel)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_warp(const float *__restrict__ I, const float *__restrict__ v, int nx, int ny,
                                              int nz, float *__restrict__ out, int gx, int gy,
                                              const int *__restrict__ stop_at, int n)
{
    if (stop_at && *stop_at < n) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    out[i] = (float)sample64(I, make_cell_disp(x, y, z, v[i], v[N + i], v[2 * N + i], nx, ny, nz));
}

// Volume size and tiling of one registration of a launch.
struct PlaneGeo {
    int nx, ny, nz;
    int gx, gy;  // x tiles, y tiles
};

// Pre-warp of one iteration for `count` registrations (a lockstep batch; 1
// outside batches), possibly of different sizes: per-registration arguments
// are arrays indexed by registration, and each registration has its own set
// of 64 x 4 workgroups (one per x tile, y tile and z plane; interleaved over
// the XCDs by batch_slot).
struct PrewarpArgs {
    const void *M[kMaxBatch], *S[kMaxBatch], *v[kMaxBatch];
    void *D[kMaxBatch], *P[kMaxBatch];
    const int *stop_at[kMaxBatch];  // skip when *stop_at < n (NULL: never)
    int kind[kMaxBatch];            // read by the mixed instance only
    PlaneGeo geo[kMaxBatch];
    int first[kMaxBatch + 1];       // registration r has first[r + 1] - first[r] workgroups (order: batch_slot)
    int chunk[kXCDs];               // logical start of chunk k (batch_slot)
    int count;
    int n;
};

// Intensity difference for the active and double forces: D = M(x - v) - S(x),
// sampled and subtracted in FP64, rounded once (FP32 for 16-bit storage, see
// bsample32).  The force kernel takes D and
// its gradient from here (grad Im = grad D + grad S), so the gather happens
// once per iteration.  Buffer addressing as in the force kernel; every volume
// in format St.
template <class St>
__device__ __forceinline__ void warp_diff_at(const PrewarpArgs &a, int r, int x, int y, int z)
{
    const int nx = a.geo[r].nx, ny = a.geo[r].ny, nz = a.geo[r].nz;
    constexpr unsigned E = St::kBytes;
    const unsigned nbytes = E * (unsigned)nx * (unsigned)ny * (unsigned)nz;
    constexpr unsigned pad = E == 2 ? kPad16 : 0u;  // M is gathered (bsample32)
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(a.M[r], nbytes + pad), rS = make_rsrc(a.S[r], nbytes),
                                 rv = make_rsrc(a.v[r], 3u * nbytes), rD = make_rsrc(a.D[r], nbytes);
    const unsigned o = E * (unsigned)(x + nx * (y + ny * z));
    const float vx = St::load(rv, o, 0), vy = St::load(rv, o, nbytes), vz = St::load(rv, o, 2u * nbytes);
    if constexpr (E == 4) {
        const double d = bsample64<St>(rM, bcell_disp<E>(x, y, z, vx, vy, vz, nx, ny, nz)) - (double)St::load(rS, o, 0);
        St::store(rD, (float)d, o, 0);
    } else {  // 16-bit storage: FP32 sample (see bsample32)
        St::store(rD, bsample32<St, true>(rM, bcell32<E>(x, y, z, vx, vy, vz, nx, ny, nz)) - St::load(rS, o, 0), o, 0);
    }
}

// Inverse-consistent pair (Sec 2.2, after Eq 6): Im = M(x - h), Is = S(x + h),
// written as D = Im - Is and P = Im + Is (the force needs D and grad P).
// Both formed in FP64 and rounded once (FP32 for 16-bit storage): D to the
// storage format, P to FP32 (P is near twice the background intensity, where
// 16-bit spacing would quantise the gradient the force divides by).
template <class St>
__device__ __forceinline__ void warp_pair_at(const PrewarpArgs &a, int r, int x, int y, int z)
{
    const int nx = a.geo[r].nx, ny = a.geo[r].ny, nz = a.geo[r].nz;
    constexpr unsigned E = St::kBytes;
    const unsigned nbytes = E * (unsigned)nx * (unsigned)ny * (unsigned)nz;
    constexpr unsigned pad = E == 2 ? kPad16 : 0u;  // M and S are gathered (bsample32)
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(a.M[r], nbytes + pad), rS = make_rsrc(a.S[r], nbytes + pad),
                                 rh = make_rsrc(a.v[r], 3u * nbytes), rD = make_rsrc(a.D[r], nbytes),
                                 rP = make_rsrc(a.P[r], (4u / E) * nbytes);
    const unsigned o = E * (unsigned)(x + nx * (y + ny * z));
    const float hx = St::load(rh, o, 0), hy = St::load(rh, o, nbytes), hz = St::load(rh, o, 2u * nbytes);
    if constexpr (E == 4) {
        const double im = bsample64<St>(rM, bcell_disp<E>(x, y, z, hx, hy, hz, nx, ny, nz));
        const double is = bsample64<St>(rS, bcell_disp<E>(x, y, z, -hx, -hy, -hz, nx, ny, nz));
        St::store(rD, (float)(im - is), o, 0);
        StF32::store(rP, (float)(im + is), (4u / E) * o, 0);
    } else {  // 16-bit storage: FP32 samples (see bsample32)
        const float im = bsample32<St, true>(rM, bcell32<E>(x, y, z, hx, hy, hz, nx, ny, nz));
        const float is = bsample32<St, true>(rS, bcell32<E>(x, y, z, -hx, -hy, -hz, nx, ny, nz));
        St::store(rD, im - is, o, 0);
        StF32::store(rP, im + is, (4u / E) * o, 0);
    }
}

// Workgroup -> (registration, x tile, y tile, z plane); false past the volume
// or once the registration's level has stopped.
__device__ __forceinline__ bool prewarp_voxel(const PrewarpArgs &a, int &r, int &x, int &y, int &z)
{
    int lb;  // wave-uniform
    batch_slot(xcd_logical_id(blockIdx.x, gridDim.x), a, r, lb);
    if (a.stop_at[r] && *a.stop_at[r] < a.n) return false;
    const PlaneGeo &t = a.geo[r];
    const int q = lb / t.gx;
    x = (lb - q * t.gx) * kBlockX + threadIdx.x;
    y = (q % t.gy) * kBlockY + threadIdx.y;
    z = q / t.gy;
    return x < t.nx && y < t.ny;
}

template <class St>
__global__ __launch_bounds__(256) void k_warp_diff(PrewarpArgs a)
{
    int r, x, y, z;
    if (prewarp_voxel(a, r, x, y, z)) warp_diff_at<St>(a, r, x, y, z);
}

template <class St>
__global__ __launch_bounds__(256) void k_warp_pair(PrewarpArgs a)
{
    int r, x, y, z;
    if (prewarp_voxel(a, r, x, y, z)) warp_pair_at<St>(a, r, x, y, z);
}

// A batch that mixes the two kinds: each registration's kind (uniform per
// workgroup).
template <class St>
__global__ __launch_bounds__(256) void k_warp_mixed(PrewarpArgs a)
{
    int r, x, y, z;
    if (!prewarp_voxel(a, r, x, y, z)) return;
    if (a.kind[r] == kPrewarpPair) warp_pair_at<St>(a, r, x, y, z);
    else warp_diff_at<St>(a, r, x, y, z);
}

// ------------------------------------------------------------------------
// Inverse-consistent output composition: w(z) = 2 h(p), p = z - h(p)
// ------------------------------------------------------------------------
// h in format St; the output field is FP32.
template <class St>
__global__ __launch_bounds__(256) void k_compose(const void *__restrict__ h, int nx, int ny, int nz, int K,
                                                 float *__restrict__ out, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    constexpr unsigned E = St::kBytes;
    const unsigned N = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const __amdgpu_buffer_rsrc_t H = make_rsrc(h, 3u * E * N);
    // p = (x, y, z) - (hx, hy, hz): the position is kept as the displacement.
    // The first sample, at p = z, gives the starting point p = z - h(z); K
    // updates of p follow, then h at the last p: K + 2 samples.  A sample
    // equal to the one before is a fixed point of the FP32 map, which every
    // later sample repeats, so the loop ends there with the same result.
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    for (int k = 0; k <= K + 1; ++k) {
        float sx, sy, sz;
        bsample3<St>(H, bcell_disp<E>(x, y, z, hx, hy, hz, nx, ny, nz), E * N, sx, sy, sz);
        const bool fixed = sx == hx && sy == hy && sz == hz;
        hx = sx;
        hy = sy;
        hz = sz;
        if (fixed) break;
    }
    const __amdgpu_buffer_rsrc_t O = make_rsrc(out, 12u * N);
    const unsigned o = 4u * (unsigned)(x + nx * (y + ny * z));
    bstore(O, 2.0f * hx, o, 0u);
    bstore(O, 2.0f * hy, o, 4u * N);
    bstore(O, 2.0f * hz, o, 8u * N);
}

// Similarity of S and the deformed M (Sec 3.2 follows registrations by the
// correlation coefficient and the intensity error): per workgroup the FP64
// sums of S, Im, S^2, Im^2, S Im and (Im - S)^2, Im = M(x - v) sampled in FP64;
// the slots (kSimSums arrays of nb) are added up in order by k_similarity_sum.
constexpr int kSimSums = 6;

__global__ __launch_bounds__(256) void k_similarity(const float *__restrict__ M, const float *__restrict__ S,
                                                    const float *__restrict__ v, int nx, int ny, int nz,
                                                    double *__restrict__ partials, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    double acc[kSimSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < nx && y < ny) {
        const unsigned nbytes = 4u * (unsigned)nx * (unsigned)ny * (unsigned)nz;
        const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, nbytes), rS = make_rsrc(S, nbytes);
        const unsigned o = 4u * (unsigned)(x + nx * (y + ny * z));
        float vx = 0.0f, vy = 0.0f, vz = 0.0f;
        if (v) {
            const __amdgpu_buffer_rsrc_t rv = make_rsrc(v, 3u * nbytes);
            vx = bload(rv, o, 0);
            vy = bload(rv, o, nbytes);
            vz = bload(rv, o, 2u * nbytes);
        }
        const double im = bsample64(rM, bcell_disp(x, y, z, vx, vy, vz, nx, ny, nz));
        const double s = (double)bload(rS, o, 0);
        acc[0] = s;
        acc[1] = im;
        acc[2] = s * s;
        acc[3] = im * im;
        acc[4] = s * im;
        acc[5] = (im - s) * (im - s);
    }
    const int tid = threadIdx.x + kBlockX * threadIdx.y;
    block_sum(acc, tid);
    if (tid == 0)
        for (int k = 0; k < kSimSums; ++k) partials[(size_t)k * gridDim.x + blockIdx.x] = acc[k];
}

__global__ __launch_bounds__(256) void k_similarity_sum(const double *__restrict__ partials, int nb,
                                                        double *__restrict__ out)
{
    const int tid = threadIdx.x;
    double acc[kSimSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < nb; b += 256)
        for (int k = 0; k < kSimSums; ++k) acc[k] += partials[(size_t)k * nb + b];
    block_sum(acc, tid);
    if (tid == 0)
        for (int k = 0; k < kSimSums; ++k) out[k] = acc[k];
}

template <class St>
__global__ __launch_bounds__(256) void k_zero(void *__restrict__ p, unsigned n)
{
    const __amdgpu_buffer_rsrc_t r = make_rsrc(p, St::kBytes * n);
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) St::store(r, 0.0f, St::kBytes * i, 0);
}

// Element-wise change of storage format (rounded to nearest even).
template <class Si, class So>
__global__ __launch_bounds__(256) void k_convert(const void *__restrict__ in, void *__restrict__ out, unsigned n)
{
    const __amdgpu_buffer_rsrc_t ri = make_rsrc(in, Si::kBytes * n), ro = make_rsrc(out, So::kBytes * n);
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
        So::store(ro, Si::load(ri, Si::kBytes * i, 0), So::kBytes * i, 0);
}

}  // namespace

namespace {
unsigned grid_stride_blocks(int64_t n)
{
    const int64_t want = (n + 255) / 256;
    return (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
}
}  // namespace

hipError_t launch_zero(Ctx &c, void *p, int64_t n, int st)
{
    const unsigned blocks = grid_stride_blocks(n);
    return timed(c, K_FILL, [&](const Ev &ev) {
        with_storage(st, [&](auto t) {
            using St = typename decltype(t)::type;
            go(c, ev, k_zero<St>, dim3(blocks), dim3(256), p, (unsigned)n);
        });
    });
}

hipError_t launch_convert(Ctx &c, const void *in, int in_st, void *out, int out_st, int64_t n)
{
    const unsigned blocks = grid_stride_blocks(n);
    return timed(c, K_CONVERT, [&](const Ev &ev) {
        with_storage(in_st, [&](auto ti) {
            with_storage(out_st, [&](auto to) {
                using Si = typename decltype(ti)::type;
                using So = typename decltype(to)::type;
                go(c, ev, k_convert<Si, So>, dim3(blocks), dim3(256), in, out, (unsigned)n);
            });
        });
    });
}

hipError_t launch_restrict(Ctx &c, const void *in, int in_st, Dims fine, void *out, int out_st, Dims coarse)
{
    const Grid2 g = plane_grid(coarse);
    return timed(c, K_RESTRICT, [&](const Ev &ev) {
        with_storage(in_st, [&](auto ti) {
            with_storage(out_st, [&](auto to) {
                using Si = typename decltype(ti)::type;
                using So = typename decltype(to)::type;
                go(c, ev, k_restrict<Si, So>, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), in, fine.nx, fine.ny,
                   fine.nz, out, coarse.nx, coarse.ny, coarse.nz, g.gx, g.gy);
            });
        });
    });
}

hipError_t launch_prolong(Ctx &c, const void *vc, Dims coarse, void *vf, Dims fine, int st)
{
    const Grid2 g = plane_grid(fine);
    return timed(c, K_PROLONG, [&](const Ev &ev) {
        with_storage(st, [&](auto t) {
            using St = typename decltype(t)::type;
            go(c, ev, k_prolong<St>, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), vc, coarse.nx, coarse.ny,
               coarse.nz, vf, fine.nx, fine.ny, fine.nz, g.gx, g.gy);
        });
    });
}

hipError_t launch_gradient(Ctx &c, const float *img, Dims d, float *grad)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_GRADIENT, [&](const Ev &ev) {
        go(c, ev, k_gradient, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), img, d.nx, d.ny,
                           d.nz, grad, g.gx, g.gy);
    });
}

hipError_t launch_warp(Ctx &c, const float *img, const float *field, Dims d, float *out, const int *stop_at, int n)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_WARP, [&](const Ev &ev) {
        go(c, ev, k_warp, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), img, field, d.nx,
                           d.ny, d.nz, out, g.gx, g.gy, stop_at, n);
    });
}

hipError_t launch_prewarp(Ctx &c, const PrewarpLaunch &w)
{
    if (w.count < 1 || w.count > kMaxBatch) return hipErrorInvalidValue;
    PrewarpArgs a;
    memset(&a, 0, sizeof a);
    int64_t total = 0;
    for (int r = 0; r < w.count; ++r) {
        const Grid2 g = plane_grid(w.d[r]);
        a.geo[r] = PlaneGeo{w.d[r].nx, w.d[r].ny, w.d[r].nz, g.gx, g.gy};
        a.first[r] = (int)total;
        total += g.blocks;
        a.M[r] = w.M[r];
        a.S[r] = w.S[r];
        a.v[r] = w.v[r];
        a.D[r] = w.D[r];
        a.P[r] = w.P[r];
        a.stop_at[r] = w.stop_at[r];
        a.kind[r] = w.kind == kPrewarpMixed ? w.kinds[r] : w.kind;
    }
    a.first[w.count] = (int)total;
    batch_chunks(a.first, w.count, a.chunk);
    a.count = w.count;
    a.n = w.n;
    const dim3 grid((unsigned)total), block(kBlockX, kBlockY);
    const int k = w.kind == kPrewarpDiff ? K_WARP : (w.kind == kPrewarpPair ? K_WARP_PAIR : K_WARP_MIXED);
    return timed(c, k, [&](const Ev &ev) {
        with_storage(w.storage, [&](auto t) {
            using St = typename decltype(t)::type;
            if (w.kind == kPrewarpDiff) go(c, ev, k_warp_diff<St>, grid, block, a);
            else if (w.kind == kPrewarpPair) go(c, ev, k_warp_pair<St>, grid, block, a);
            else go(c, ev, k_warp_mixed<St>, grid, block, a);
        });
    });
}

int64_t similarity_blocks(Dims d) { return plane_grid(d).blocks; }

hipError_t launch_similarity(Ctx &c, const float *M, const float *S, const float *v, Dims d, double *partials,
                             double *out)
{
    const Grid2 g = plane_grid(d);
    hipError_t e = timed(c, K_SIMILARITY, [&](const Ev &ev) {
        go(c, ev, k_similarity, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), M, S, v, d.nx, d.ny, d.nz,
           partials, g.gx, g.gy);
    });
    if (e != hipSuccess) return e;
    return timed(c, K_SIMILARITY, [&](const Ev &ev) {
        go(c, ev, k_similarity_sum, dim3(1), dim3(256), (const double *)partials, (int)g.blocks, out);
    });
}

hipError_t launch_compose(Ctx &c, const void *h, int h_st, Dims d, int K, float *out)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_COMPOSE, [&](const Ev &ev) {
        with_storage(h_st, [&](auto t) {
            using St = typename decltype(t)::type;
            go(c, ev, k_compose<St>, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), h, d.nx, d.ny, d.nz, K, out,
               g.gx, g.gy);
        });
    });
}

}  // namespace dir
