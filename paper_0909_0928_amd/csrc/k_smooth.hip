// gfx950 kernels of the separable Gaussian smoothing (Sec 2.1 regularisation;
// Sec 2.5 low-pass filter, separable in x, y and z).
//
// The x pass runs fused into the force kernel during registration; the
// standalone x pass here serves dir_smooth.  The y and z passes are fused in
// one kernel (z pass into LDS, then y pass out of LDS); each field component
// has its own workgroups.
#include <string.h>

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
// field component.  Phase 1: every thread slides a register window of
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

// One launch serves `count` registrations of one size (a lockstep batch; 1
// outside batches): per-registration arguments are arrays indexed by
// registration, and the grid holds `per` workgroups per registration.
struct YZArgs {
    const void *in[kMaxBatch];
    void *out[kMaxBatch];
    const int *stop_at[kMaxBatch];  // skip when *stop_at < n (NULL: never)
    int nx, ny, nz;
    int gx, gy, gz;                 // x tiles, y tiles, z chunks
    int n;
    int per;                        // workgroups per registration
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
    const int reg = g / a.per, lb = g - reg * a.per;  // wave-uniform
    if (a.stop_at[reg] && *a.stop_at[reg] < a.n) return;
    const int tid = threadIdx.x + kBlockX * threadIdx.y;
    if (red.count && lb == 0) {
        reduce_sums(red.partials[reg], red.nb, red.hist[reg], a.n, red.st[reg], red.eps[reg], red.inv_n, tid);
        return;
    }
    const int nx = a.nx, ny = a.ny, nz = a.nz, gx = a.gx, gy = a.gy, gz = a.gz;
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
    float w[2 * R + 1];
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) w[j] = taps.w[j];
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
            for (int j = 0; j <= 2 * R; ++j) s = fmaf(w[j], wa[k + j], s);
            zs[k][row][lane] = s;
        }
        if (two) {
#pragma unroll
            for (int k = 0; k < TZ; ++k) {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j) s = fmaf(w[j], wb[k + j], s);
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

template <int R, int TZ, class St>
void launch_yz_tz(Ctx &c, const Ev &ev, YZArgs a, int ncomp, int count, const GaussTaps &taps,
                  const SumsReduce &red)
{
    a.gx = ceil_div(a.nx, kBlockX);
    a.gy = ceil_div(a.ny, kTileY);
    a.gz = ceil_div(a.nz, TZ);
    a.per = a.gx * a.gy * a.gz * ncomp + (red.count ? 1 : 0);
    const int64_t blocks = (int64_t)a.per * count;
    go(c, ev, (k_smooth_yz<R, TZ, St>), dim3((unsigned)blocks), dim3(kBlockX, kBlockY), a, taps, red);
}

// Workgroups to aim for before the z chunk is made deeper (each chunk re-reads
// 2R halo planes, so deeper chunks cost fewer loads per output).
constexpr int64_t kYZTargetBlocks = 1024;

template <int R, class St>
hipError_t launch_yz_r(Ctx &c, const YZArgs &a, int ncomp, int count, const GaussTaps &taps, const SumsReduce &red)
{
    // the depth choice depends on the tiles of one registration
    const int64_t tiles = (int64_t)ceil_div(a.nx, kBlockX) * ceil_div(a.ny, kTileY) * ncomp;
    const bool deep = max_tz<R>() == 8 && tiles * ceil_div(a.nz, 8) >= kYZTargetBlocks;
    return timed(c, K_SMOOTH_YZ, [&](const Ev &ev) {
        if (deep) launch_yz_tz<R, max_tz<R>(), St>(c, ev, a, ncomp, count, taps, red);
        else if (tiles * ceil_div(a.nz, 4) >= kYZTargetBlocks / 2) launch_yz_tz<R, 4, St>(c, ev, a, ncomp, count, taps, red);
        else launch_yz_tz<R, 2, St>(c, ev, a, ncomp, count, taps, red);
    });
}

}  // namespace

template <class St>
hipError_t launch_smooth_yz_st(Ctx &c, const YZArgs &a, int ncomp, int count, const GaussTaps &taps,
                               const SumsReduce &red)
{
    switch (taps.radius) {
#define DIR_R(r) \
    case r: return launch_yz_r<r, St>(c, a, ncomp, count, taps, red);
        DIR_R(0) DIR_R(1) DIR_R(2) DIR_R(3) DIR_R(4) DIR_R(5) DIR_R(6) DIR_R(7) DIR_R(8)
        DIR_R(9) DIR_R(10) DIR_R(11) DIR_R(12) DIR_R(13) DIR_R(14) DIR_R(15) DIR_R(16)
#undef DIR_R
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_smooth_yz(Ctx &c, int count, const void *const *in, int ncomp, Dims d, const GaussTaps &taps,
                            void *const *out, int st, const int *const *stop_at, int n, const SumsReduce &red)
{
    if (count < 1 || count > kMaxBatch || (red.count && red.count != count)) return hipErrorInvalidValue;
    YZArgs a;
    memset(&a, 0, sizeof a);
    for (int r = 0; r < count; ++r) {
        a.in[r] = in[r];
        a.out[r] = out[r];
        a.stop_at[r] = stop_at[r];
    }
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.n = n;
    if (st == kStoreF16) return launch_smooth_yz_st<StF16>(c, a, ncomp, count, taps, red);
    if (st == kStoreBF16) return launch_smooth_yz_st<StBF16>(c, a, ncomp, count, taps, red);
    return launch_smooth_yz_st<StF32>(c, a, ncomp, count, taps, red);
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
