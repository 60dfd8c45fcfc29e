// gfx950 kernels of the separable Gaussian smoothing (Sec 2.1 regularisation;
// Sec 2.5 low-pass filter, separable in x, y and z).
//
// The x pass runs fused into the force kernel during registration; the
// standalone x pass here serves dir_smooth.  The y and z passes are fused in
// one kernel (z pass into LDS, then y pass out of LDS); each field component
// has its own workgroups.
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>

#include "device_common.h"

namespace dir {
namespace {

using namespace dev;

constexpr int kRowsPerThread = 4;
constexpr int kTileY = kBlockY * kRowsPerThread;  // 16 rows per workgroup

// x pass: each wavefront stages its row segment plus a radius-R halo in LDS.
__global__ __launch_bounds__(256) void k_smooth_x(const float *__restrict__ in, float *__restrict__ out, int ncomp,
                                                  int nx, int ny, int nz, GaussTaps taps, int gx, int gy)
{
    __shared__ float row[kBlockY][kBlockX + 2 * kMaxRadius];
    const Tile t = decode_tile(gx, gy);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x0 = t.x * kBlockX, x = x0 + tx, y = t.y * kBlockY + ty, z = t.z;
    const int R = taps.radius;
    const int N = nx * ny * nz;
    const bool row_ok = y < ny;
    for (int c = 0; c < ncomp; ++c) {
        const float *src = in + (int64_t)c * N + nx * (y + ny * z);
        if (row_ok)
            for (int j = tx; j < kBlockX + 2 * R; j += kBlockX) row[ty][j] = src[clampi(x0 - R + j, nx)];
        __syncthreads();
        if (row_ok && x < nx) {
            float s = 0.0f;
            for (int j = 0; j <= 2 * R; ++j) s = fmaf(taps.w[j], row[ty][tx + j], s);
            out[(int64_t)c * N + nx * (y + ny * z) + x] = s;
        }
        __syncthreads();
    }
}

// z then y within one workgroup: tile of 64 (x) x kTileY (y) x TZ (z) of one
// field component, z taps taps.wz, y taps taps.w.  Phase 1: every thread slides a register window of
// TZ + 2R samples along z for one (x, y) column of the tile plus its y halo
// (rows clamped) and writes the TZ z-smoothed values to LDS.  Phase 2: every
// thread forms 4 consecutive y outputs of one x column for each of the TZ
// planes from 4 + 2R LDS values.
template <int R, int TZ>
struct YZTile {
    static constexpr int ROWS = kTileY + 2 * R;  // tile rows plus y halo
    static_assert(TZ * ROWS * kBlockX * 4 <= 65536, "LDS tile above 64 KB");
};

// Deepest z chunk (8 or 4 planes) whose LDS tile fits in 64 KB.
template <int R>
constexpr int max_tz()
{
    return (kTileY + 2 * R) * kBlockX * 4 * 8 <= 65536 ? 8 : 4;
}

// Volume size and tiling of one registration of a launch.
struct YZGeo {
    int nx, ny, nz;
    int gx, gy, gz;  // x tiles, y tiles, z chunks
};

// One launch serves `count` registrations (a lockstep batch; 1 outside
// batches), possibly of different sizes with the same z-chunk depth:
// per-registration arguments are arrays indexed by registration, and each
// registration has its own range of workgroups.
struct YZArgs {
    const void *in[kMaxBatch];
    void *out[kMaxBatch];
    const int *stop_at[kMaxBatch];  // skip when *stop_at < n (NULL: never)
    YZGeo geo[kMaxBatch];
    int first[kMaxBatch + 1];       // logical workgroups of registration r: first[r] .. first[r + 1] - 1
    int count;
    int n;
};

// With red.count set, the first workgroup of each registration instead adds
// up the FP64 sums the force kernel of this iteration left per workgroup
// (they are complete: that kernel has finished), writes the history entry and
// takes the stopping decision; the smoothing tiles follow it.
template <int R, int TZ, class St>
__global__ __launch_bounds__(256) void k_smooth_yz(YZArgs a, GaussTaps taps, SumsReduce red)
{
    constexpr int ROWS = YZTile<R, TZ>::ROWS;
    __shared__ float zs[TZ][ROWS][kBlockX];
    // workgroup id -> (registration, z chunk, y tile, x tile, component),
    // numbered so that each XCD runs one contiguous range with z chunks
    // fastest, then y tiles: the tiles an XCD has in flight at once form a
    // compact (y, z) block of one x column, whose shared 2R halo planes and
    // rows are then served from that XCD's L2.
    const int g = xcd_logical_id(blockIdx.x, gridDim.x);
    int reg = 0;  // wave-uniform
    while (reg + 1 < a.count && g >= a.first[reg + 1]) ++reg;
    const int lb = g - a.first[reg];
    if (a.stop_at[reg] && *a.stop_at[reg] < a.n) return;
    const int tid = threadIdx.x + kBlockX * threadIdx.y;
    if (red.count && lb == 0) {
        reduce_sums(red.partials[reg], red.nb[reg], red.hist[reg], a.n, red.st[reg], red.eps[reg], red.inv_n[reg],
                    tid);
        return;
    }
    const YZGeo &q = a.geo[reg];
    const int nx = q.nx, ny = q.ny, nz = q.nz, gx = q.gx, gy = q.gy, gz = q.gz;
    const int b = lb - (red.count ? 1 : 0);
    const int tz = b % gz, r1 = b / gz, ty = r1 % gy, r2 = r1 / gy, tx = r2 % gx, c = r2 / gx;
    const void *const in = a.in[reg];
    void *const out = a.out[reg];
    // threadIdx.y is the wavefront index (64 x 4 workgroup): uniform, which
    // lets the row offsets below live in scalar registers
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int x = min(tx * kBlockX + lane, nx - 1);  // lanes past the edge repeat the last column
    const int y_base = ty * kTileY, z0 = tz * TZ;
    constexpr unsigned ES = St::kBytes;
    const unsigned N = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const unsigned rowb = ES * (unsigned)nx, planeb = rowb * (unsigned)ny;
    const __amdgpu_buffer_rsrc_t src = make_rsrc(static_cast<const char *>(in) + (size_t)c * ES * N, ES * N);
    const __amdgpu_buffer_rsrc_t dst = make_rsrc(static_cast<char *>(out) + (size_t)c * ES * N, ES * N);
    const unsigned xb = ES * (unsigned)x;
    float w[2 * R + 1], wz[2 * R + 1];  // y and z taps (equal for an isotropic Gaussian)
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) {
        w[j] = taps.w[j];
        wz[j] = taps.wz[j];
    }
    // byte offsets of the window's planes (clamped), wave-uniform
    unsigned zoff[TZ + 2 * R];
#pragma unroll
    for (int k = 0; k < TZ + 2 * R; ++k) zoff[k] = planeb * (unsigned)clampi(z0 - R + k, nz);

    // phase 1: z pass for rows y_base - R .. y_base + kTileY + R - 1, two rows
    // per step with the loads of both windows issued before any arithmetic
    for (int row = wave; row < ROWS; row += 2 * kBlockY) {
        const int row2 = row + kBlockY;
        const bool two = row2 < ROWS;  // wave-uniform
        const unsigned ra = rowb * (unsigned)clampi(y_base - R + row, ny);
        const unsigned rb = rowb * (unsigned)clampi(y_base - R + (two ? row2 : row), ny);
        float wa[TZ + 2 * R], wb[TZ + 2 * R];
#pragma unroll
        for (int k = 0; k < TZ + 2 * R; ++k) wa[k] = St::load(src, xb, ra + zoff[k]);
        if (two) {
#pragma unroll
            for (int k = 0; k < TZ + 2 * R; ++k) wb[k] = St::load(src, xb, rb + zoff[k]);
        }
#pragma unroll
        for (int k = 0; k < TZ; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) s = fmaf(wz[j], wa[k + j], s);
            zs[k][row][lane] = s;
        }
        if (two) {
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j) s = fmaf(wz[j], wb[k + j], s);
                zs[k][row2][lane] = s;
            }
        }
    }
    __syncthreads();

    // phase 2: y pass, rows y_base + 4 * wave .. + 3
    const int xo = tx * kBlockX + lane;
    const int y0 = y_base + wave * kRowsPerThread;
    if (xo >= nx || y0 >= ny) return;
    const unsigned ob = ES * (unsigned)xo;
    for (int k = 0; k < TZ; ++k) {
        if (z0 + k >= nz) break;
        float v[kRowsPerThread + 2 * R];
#pragma unroll
        for (int j = 0; j < kRowsPerThread + 2 * R; ++j) v[j] = zs[k][wave * kRowsPerThread + j][lane];
        const unsigned zb = planeb * (unsigned)(z0 + k);
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) s = fmaf(w[j], v[q + j], s);
            if (y0 + q < ny) St::store(dst, s, ob, zb + rowb * (unsigned)(y0 + q));
        }
    }
}

// The same tile, 128 columns wide, for 16-bit fields of even nx: each lane
// owns two neighbouring columns, so that every load and store moves both of
// them in one 4-byte access (a 16-bit access moves half the bytes of an FP32
// one for the same cost).  Every output is the same sum in the same order as
// in k_smooth_yz, so the results are identical.  Lanes past the last column
// pair repeat it and store nothing.
template <int R, int TZ>
struct YZTile2 {
    static constexpr int ROWS = kTileY + 2 * R;
    static_assert(TZ * ROWS * 2 * kBlockX * 4 <= 65536, "LDS tile above 64 KB");
};

template <int R, int TZ, class St>
__global__ __launch_bounds__(256) void k_smooth_yz2(YZArgs a, GaussTaps taps, SumsReduce red)
{
    static_assert(St::kBytes == 2, "two 16-bit columns per 4-byte access");
    constexpr int ROWS = YZTile2<R, TZ>::ROWS;
    __shared__ float2 zs[TZ][ROWS][kBlockX];
    const int g = xcd_logical_id(blockIdx.x, gridDim.x);
    int reg = 0;  // wave-uniform
    while (reg + 1 < a.count && g >= a.first[reg + 1]) ++reg;
    const int lb = g - a.first[reg];
    if (a.stop_at[reg] && *a.stop_at[reg] < a.n) return;
    const int tid = threadIdx.x + kBlockX * threadIdx.y;
    if (red.count && lb == 0) {
        reduce_sums(red.partials[reg], red.nb[reg], red.hist[reg], a.n, red.st[reg], red.eps[reg], red.inv_n[reg],
                    tid);
        return;
    }
    const YZGeo &q = a.geo[reg];
    const int nx = q.nx, ny = q.ny, nz = q.nz, gx = q.gx, gy = q.gy, gz = q.gz;
    const int b = lb - (red.count ? 1 : 0);
    const int tz = b % gz, r1 = b / gz, ty = r1 % gy, r2 = r1 / gy, tx = r2 % gx, c = r2 / gx;
    const void *const in = a.in[reg];
    void *const out = a.out[reg];
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int x = min(tx * 2 * kBlockX + 2 * lane, nx - 2);  // first column of the lane's pair
    const int y_base = ty * kTileY, z0 = tz * TZ;
    constexpr unsigned ES = 2;
    const unsigned N = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const unsigned rowb = ES * (unsigned)nx, planeb = rowb * (unsigned)ny;
    const __amdgpu_buffer_rsrc_t src = make_rsrc(static_cast<const char *>(in) + (size_t)c * ES * N, ES * N);
    const __amdgpu_buffer_rsrc_t dst = make_rsrc(static_cast<char *>(out) + (size_t)c * ES * N, ES * N);
    const unsigned xb = ES * (unsigned)x;  // 4-byte aligned: x and nx are even
    float w[2 * R + 1], wz[2 * R + 1];
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) {
        w[j] = taps.w[j];
        wz[j] = taps.wz[j];
    }
    unsigned zoff[TZ + 2 * R];
#pragma unroll
    for (int k = 0; k < TZ + 2 * R; ++k) zoff[k] = planeb * (unsigned)clampi(z0 - R + k, nz);

    // phase 1: z pass for rows y_base - R .. y_base + kTileY + R - 1
    for (int row = wave; row < ROWS; row += kBlockY) {
        const unsigned ra = rowb * (unsigned)clampi(y_base - R + row, ny);
        unsigned pk[TZ + 2 * R];
#pragma unroll
        for (int k = 0; k < TZ + 2 * R; ++k) pk[k] = __builtin_amdgcn_raw_buffer_load_b32(src, xb, ra + zoff[k], 0);
#pragma unroll
        for (int k = 0; k < TZ; ++k) {
            float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) {
                s0 = fmaf(wz[j], St::from_bits(pk[k + j]), s0);
                s1 = fmaf(wz[j], St::from_bits(pk[k + j] >> 16), s1);
            }
            zs[k][row][lane] = make_float2(s0, s1);
        }
    }
    __syncthreads();

    // phase 2: y pass, rows y_base + 4 * wave .. + 3, both columns
    const int xo = tx * 2 * kBlockX + 2 * lane;
    const int y0 = y_base + wave * kRowsPerThread;
    if (xo >= nx || y0 >= ny) return;
    const unsigned ob = ES * (unsigned)xo;
    for (int k = 0; k < TZ; ++k) {
        if (z0 + k >= nz) break;
        float2 v[kRowsPerThread + 2 * R];
#pragma unroll
        for (int j = 0; j < kRowsPerThread + 2 * R; ++j) v[j] = zs[k][wave * kRowsPerThread + j][lane];
        const unsigned zb = planeb * (unsigned)(z0 + k);
#pragma unroll
        for (int qq = 0; qq < kRowsPerThread; ++qq) {
            float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) {
                s0 = fmaf(w[j], v[qq + j].x, s0);
                s1 = fmaf(w[j], v[qq + j].y, s1);
            }
            if (y0 + qq < ny)
                __builtin_amdgcn_raw_buffer_store_b32(St::to_bits(s0) | (St::to_bits(s1) << 16), dst, ob,
                                                      zb + rowb * (unsigned)(y0 + qq), 0);
        }
    }
}

// Two columns per lane: 16-bit storage, even nx, and a depth whose tile fits.
template <int R, int TZ, class St>
constexpr bool yz_two_columns()
{
    return St::kBytes == 2 && TZ * (kTileY + 2 * R) * 2 * kBlockX * 4 <= 65536;
}

// Workgroups below which a launch keeps one column per lane: small launches
// are bound by latency, and halving their workgroups measured slower
// (64x64x25 levels of a six-registration batch).
constexpr int64_t kYZTwoColumnMinBlocks = 1024;

template <int R, int TZ, class St>
void launch_yz_tz(Ctx &c, const Ev &ev, YZArgs a, int ncomp, const GaussTaps &taps, const SumsReduce &red)
{
    if constexpr (yz_two_columns<R, TZ, St>()) {
        bool even = true;
        int64_t blocks2 = 0;
        for (int r = 0; r < a.count; ++r) {
            const YZGeo &q = a.geo[r];
            even = even && q.nx % 2 == 0;
            blocks2 += (int64_t)ceil_div(q.nx, 2 * kBlockX) * ceil_div(q.ny, kTileY) * ceil_div(q.nz, TZ) * ncomp;
        }
        if (even && blocks2 >= kYZTwoColumnMinBlocks) {
            int64_t total = 0;
            for (int r = 0; r < a.count; ++r) {
                YZGeo &q = a.geo[r];
                q.gx = ceil_div(q.nx, 2 * kBlockX);
                q.gy = ceil_div(q.ny, kTileY);
                q.gz = ceil_div(q.nz, TZ);
                a.first[r] = (int)total;
                total += (int64_t)q.gx * q.gy * q.gz * ncomp + (red.count ? 1 : 0);
            }
            a.first[a.count] = (int)total;
            go(c, ev, (k_smooth_yz2<R, TZ, St>), dim3((unsigned)total), dim3(kBlockX, kBlockY), a, taps, red);
            return;
        }
    }

    int64_t total = 0;
    for (int r = 0; r < a.count; ++r) {
        YZGeo &q = a.geo[r];
        q.gx = ceil_div(q.nx, kBlockX);
        q.gy = ceil_div(q.ny, kTileY);
        q.gz = ceil_div(q.nz, TZ);
        a.first[r] = (int)total;
        total += (int64_t)q.gx * q.gy * q.gz * ncomp + (red.count ? 1 : 0);
    }
    a.first[a.count] = (int)total;
    go(c, ev, (k_smooth_yz<R, TZ, St>), dim3((unsigned)total), dim3(kBlockX, kBlockY), a, taps, red);
}

// Workgroups to aim for before the z chunk is made deeper (each chunk re-reads
// 2R halo planes, so deeper chunks cost fewer loads per output).
constexpr int64_t kYZTargetBlocks = 1024;

// z-chunk depth for a registration of size d: the deepest whose tiles still
// number kYZTargetBlocks (or half that for 4).  A 16-bit field of even nx
// takes depth 4 when its two-column tiles are enough for the two-column
// kernel: the autotuner preferred that to depth 8 at 256x256x100.
template <int R, class St>
int yz_depth(Dims d, int ncomp)
{
    if constexpr (yz_two_columns<R, 4, St>()) {
        const int64_t blocks2 =
            (int64_t)ceil_div(d.nx, 2 * kBlockX) * ceil_div(d.ny, kTileY) * ceil_div(d.nz, 4) * ncomp;
        if (d.nx % 2 == 0 && blocks2 >= kYZTwoColumnMinBlocks) return 4;
    }
    const int64_t tiles = (int64_t)ceil_div(d.nx, kBlockX) * ceil_div(d.ny, kTileY) * ncomp;
    if (max_tz<R>() == 8 && tiles * ceil_div(d.nz, 8) >= kYZTargetBlocks) return 8;
    if (tiles * ceil_div(d.nz, 4) >= kYZTargetBlocks / 2) return 4;
    return 2;
}

// Depths measured by tune_smooth_yz, per (size, components, registrations
// per launch, bytes per stored value, radius); process-wide.  The depth only
// decides which workgroup computes which output, never the arithmetic of an
// output, so it leaves every result unchanged.
struct YZKey {
    int nx, ny, nz, ncomp, count, es, R;
    bool operator<(const YZKey &o) const
    {
        return std::tie(nx, ny, nz, ncomp, count, es, R) < std::tie(o.nx, o.ny, o.nz, o.ncomp, o.count, o.es, o.R);
    }
};
std::mutex g_yz_mu;
std::map<YZKey, int> g_yz_depth;

int yz_tuned(const YZKey &k)
{
    std::lock_guard<std::mutex> lock(g_yz_mu);
    const auto it = g_yz_depth.find(k);
    return it == g_yz_depth.end() ? 0 : it->second;
}

template <int R, class St>
hipError_t launch_yz_r(Ctx &c, const YZArgs &a, int ncomp, int tz, const GaussTaps &taps, const SumsReduce &red)
{
    return timed(c, K_SMOOTH_YZ, [&](const Ev &ev) {
        if (tz == 8) launch_yz_tz<R, max_tz<R>(), St>(c, ev, a, ncomp, taps, red);
        else if (tz == 4) launch_yz_tz<R, 4, St>(c, ev, a, ncomp, taps, red);
        else launch_yz_tz<R, 2, St>(c, ev, a, ncomp, taps, red);
    });
}

// One launch for the registrations sel[0 .. k-1], which share depth tz.
template <int R, class St>
hipError_t launch_yz_group(Ctx &c, int n, const void *const *in, int ncomp, const Dims *d, const GaussTaps &taps,
                           void *const *out, const int *const *stop_at, const SumsReduce &red, const int *sel,
                           int k, int tz)
{
    YZArgs a;
    memset(&a, 0, sizeof a);
    SumsReduce rs = red;
    for (int q = 0; q < k; ++q) {
        const int r = sel[q];
        a.in[q] = in[r];
        a.out[q] = out[r];
        a.stop_at[q] = stop_at[r];
        a.geo[q].nx = d[r].nx;
        a.geo[q].ny = d[r].ny;
        a.geo[q].nz = d[r].nz;
        if (red.count) {
            rs.partials[q] = red.partials[r];
            rs.hist[q] = red.hist[r];
            rs.st[q] = red.st[r];
            rs.eps[q] = red.eps[r];
            rs.nb[q] = red.nb[r];
            rs.inv_n[q] = red.inv_n[r];
        }
    }
    a.count = k;
    a.n = n;
    if (red.count) rs.count = k;
    return launch_yz_r<R, St>(c, a, ncomp, tz, taps, rs);
}

// Registrations of one z-chunk depth share a launch; each keeps the tiling it
// has alone.
template <int R, class St>
hipError_t launch_yz_all(Ctx &c, int count, const void *const *in, int ncomp, const Dims *d,
                         const GaussTaps &taps, void *const *out, const int *const *stop_at, int n,
                         const SumsReduce &red)
{
    int tz[kMaxBatch];
    for (int r = 0; r < count; ++r) {
        const int t = yz_tuned(YZKey{d[r].nx, d[r].ny, d[r].nz, ncomp, count, (int)St::kBytes, R});
        tz[r] = t ? t : yz_depth<R, St>(d[r], ncomp);
    }
    bool done[kMaxBatch] = {};
    for (int r = 0; r < count; ++r) {
        if (done[r]) continue;
        int sel[kMaxBatch], k = 0;
        for (int q = r; q < count; ++q)
            if (!done[q] && tz[q] == tz[r]) {
                sel[k++] = q;
                done[q] = true;
            }
        const hipError_t e = launch_yz_group<R, St>(c, n, in, ncomp, d, taps, out, stop_at, red, sel, k, tz[r]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Time every z-chunk depth for `count` registrations of size d (fields in
// and out, `reps` launches each, the fastest launch counting) and keep the
// fastest depth for such launches.
template <int R, class St>
hipError_t tune_yz(Ctx &c, int count, const void *const *in, int ncomp, Dims d, const GaussTaps &taps,
                   void *const *out, int reps, int *chosen)
{
    YZArgs a;
    memset(&a, 0, sizeof a);
    for (int r = 0; r < count; ++r) {
        a.in[r] = in[r];
        a.out[r] = out[r];
        a.geo[r].nx = d.nx;
        a.geo[r].ny = d.ny;
        a.geo[r].nz = d.nz;
    }
    a.count = count;
    SumsReduce none;
    memset(&none, 0, sizeof none);  // count 0: no reduction
    Ev ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&ev.b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev.a);
        return e;
    }
    int best = 0;
    float best_ms = 0.0f;
    const int cands[3] = {2, 4, max_tz<R>() == 8 ? 8 : 0};
    for (int tz : cands) {
        if (!tz) continue;
        float fastest = 0.0f;
        for (int k = 0; k <= reps && e == hipSuccess; ++k) {  // the first launch is not counted
            if (tz == 8) launch_yz_tz<R, max_tz<R>(), St>(c, ev, a, ncomp, taps, none);
            else if (tz == 4) launch_yz_tz<R, 4, St>(c, ev, a, ncomp, taps, none);
            else launch_yz_tz<R, 2, St>(c, ev, a, ncomp, taps, none);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipEventSynchronize(ev.b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
            if (e == hipSuccess && k > 0 && (fastest == 0.0f || ms < fastest)) fastest = ms;
        }
        if (e != hipSuccess) break;
        if (!best || fastest < best_ms) {
            best = tz;
            best_ms = fastest;
        }
    }
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lock(g_yz_mu);
        g_yz_depth[YZKey{d.nx, d.ny, d.nz, ncomp, count, (int)St::kBytes, R}] = best;
    }
    *chosen = best;
    return hipSuccess;
}

}  // namespace

hipError_t tune_smooth_yz(Ctx &c, int count, const void *const *in, int ncomp, Dims d, const GaussTaps &taps,
                          void *const *out, int st, int reps, int *chosen)
{
    if (count < 1 || count > kMaxBatch || reps < 1) return hipErrorInvalidValue;
    auto run = [&](auto tag) -> hipError_t {
        using St = typename decltype(tag)::type;
        switch (taps.radius) {
#define DIR_R(r) \
    case r: return tune_yz<r, St>(c, count, in, ncomp, d, taps, out, reps, chosen);
            DIR_R(0) DIR_R(1) DIR_R(2) DIR_R(3) DIR_R(4) DIR_R(5) DIR_R(6) DIR_R(7) DIR_R(8)
            DIR_R(9) DIR_R(10) DIR_R(11) DIR_R(12) DIR_R(13) DIR_R(14) DIR_R(15) DIR_R(16)
#undef DIR_R
        default: return hipErrorInvalidValue;
        }
    };
    if (st == kStoreF16) return run(Tag<StF16>{});
    if (st == kStoreBF16) return run(Tag<StBF16>{});
    return run(Tag<StF32>{});
}

void clear_smooth_yz_tuning()
{
    std::lock_guard<std::mutex> lock(g_yz_mu);
    g_yz_depth.clear();
}

template <class St>
hipError_t launch_smooth_yz_st(Ctx &c, int count, const void *const *in, int ncomp, const Dims *d,
                               const GaussTaps &taps, void *const *out, const int *const *stop_at, int n,
                               const SumsReduce &red)
{
    switch (taps.radius) {
#define DIR_R(r) \
    case r: return launch_yz_all<r, St>(c, count, in, ncomp, d, taps, out, stop_at, n, red);
        DIR_R(0) DIR_R(1) DIR_R(2) DIR_R(3) DIR_R(4) DIR_R(5) DIR_R(6) DIR_R(7) DIR_R(8)
        DIR_R(9) DIR_R(10) DIR_R(11) DIR_R(12) DIR_R(13) DIR_R(14) DIR_R(15) DIR_R(16)
#undef DIR_R
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_smooth_yz(Ctx &c, int count, const void *const *in, int ncomp, const Dims *d,
                            const GaussTaps &taps, void *const *out, int st, const int *const *stop_at, int n,
                            const SumsReduce &red)
{
    if (count < 1 || count > kMaxBatch || (red.count && red.count != count)) return hipErrorInvalidValue;
    if (st == kStoreF16) return launch_smooth_yz_st<StF16>(c, count, in, ncomp, d, taps, out, stop_at, n, red);
    if (st == kStoreBF16) return launch_smooth_yz_st<StBF16>(c, count, in, ncomp, d, taps, out, stop_at, n, red);
    return launch_smooth_yz_st<StF32>(c, count, in, ncomp, d, taps, out, stop_at, n, red);
}

hipError_t launch_smooth_x(Ctx &c, const float *in, int ncomp, Dims d, const GaussTaps &taps, float *out)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_SMOOTH_X, [&](const Ev &ev) {
        go(c, ev, k_smooth_x, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), in, out, ncomp,
                           d.nx, d.ny, d.nz, taps, g.gx, g.gy);
    });
}

}  // namespace dir
