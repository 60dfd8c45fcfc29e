// gfx950 kernel of one demons force step (Eqs 1-6), fused with the x pass of
// the Gaussian smoothing (Sec 2.5 low-pass filter) and the per-workgroup FP64
// sums behind the relative norm of Sec 2.4.
//
// A workgroup of 256 threads owns an x tile of TX voxels (TX = 64, 128 or
// 256; 256/TX rows in flight) and walks `rows_per_block` row steps.  For each
// row it evaluates u = v + dr at the TX tile voxels plus an R-voxel halo on
// both sides (indices clamped, so a halo entry equals u at the clamped
// voxel), stages u in LDS and writes the x-smoothed field.  The per-voxel sums
// sum|dr|, sum|v| and sum D^2 are accumulated in FP64 over the tile voxels
// only, reduced per workgroup in a fixed order and written to per-workgroup
// slots.  The slots are added up, in slot order, by one workgroup of the
// kernel that runs next (no cross-workgroup fences inside this kernel: on a
// multi-XCD device an agent-scope release per workgroup costs an L2
// write-back each).
#include "device_common.h"

namespace dir {
namespace {

using namespace dev;

struct ForceArgs {
    const float *S, *M, *v, *Im, *Is;
    int nx, ny, nz;
    float alpha2;
    float *out;           // x-smoothed u (u itself with identity taps)
    double *partials;     // 3 * gridDim.x doubles: s1[], s2[], sse[]
    const int *stop_at;   // skip when *stop_at < n (NULL: never)
    int n;                // iteration index within the level
    int rows_per_block;
    int gxt;              // x tiles
};

// u = v + dr at voxel (x, y, z) and its contributions |dr|, |v|, D^2.
template <int V>
__device__ __forceinline__ void force_point(const ForceArgs &a, int x, int y, int z, float &u0, float &u1, float &u2,
                                            double &adr, double &av, double &d2)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    const float vx = a.v[i], vy = a.v[N + i], vz = a.v[2 * N + i];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    // intensity difference in FP64, rounded once (see sample64)
    double D64;
    if (V == kInverseConsistent)
        D64 = sample64(a.M, make_cell_disp(x, y, z, vx, vy, vz, nx, ny, nz)) -
              sample64(a.S, make_cell_disp(x, y, z, -vx, -vy, -vz, nx, ny, nz));
    else
        D64 = sample64(a.M, make_cell_disp(x, y, z, vx, vy, vz, nx, ny, nz)) - (double)a.S[i];
    const float D = (float)D64;
    if (V == kInverseConsistent) {
        // Eq 6: g = grad Im + grad Is of the two deformed images
        float ax, ay, az, bx, by, bz;
        central_diff(a.Im, x, y, z, nx, ny, nz, ax, ay, az);
        central_diff(a.Is, x, y, z, nx, ny, nz, bx, by, bz);
        demons_term(D, ax + bx, ay + by, az + bz, a.alpha2, fx, fy, fz);
    } else {
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
        if (V == kPassive || V == kDouble || V == kEvolved) central_diff(a.S, x, y, z, nx, ny, nz, sx, sy, sz);
        if (V == kPassive || V == kDouble) demons_term(D, sx, sy, sz, a.alpha2, fx, fy, fz);  // Eq 1
        if (V == kActive || V == kDouble) {                                                   // Eq 3
            float mx, my, mz, bx, by, bz;
            central_diff(a.Im, x, y, z, nx, ny, nz, mx, my, mz);
            demons_term(D, mx, my, mz, a.alpha2, bx, by, bz);
            fx += bx;
            fy += by;
            fz += bz;
        }
        if (V == kEvolved) {                                                                  // Eq 2
            float mx, my, mz;
            central_diff(a.M, x, y, z, nx, ny, nz, mx, my, mz);
            evolved_term(D, sx, sy, sz, sqrtf(fmaf(mx, mx, fmaf(my, my, mz * mz))), fx, fy, fz);
        }
    }
    u0 = vx + fx;
    u1 = vy + fy;
    u2 = vz + fz;
    adr = (double)sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
    av = (double)sqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
    d2 = D64 * D64;
}

template <int V, int TX>
__global__ __launch_bounds__(256) void k_force_x(ForceArgs a, GaussTaps taps)
{
    if (a.stop_at && *a.stop_at < a.n) return;
    constexpr int W = 256 / TX;
    __shared__ float ul[3][W][TX + 2 * kMaxRadius];
    __shared__ float wl[2 * kMaxRadius + 1];  // taps, read as LDS broadcasts
    const int tid = threadIdx.x;
    if (tid <= 2 * kMaxRadius) wl[tid] = taps.w[tid];  // ordered before use by the row barrier
    const int lane = tid % TX, wrow = tid / TX;
    const int x0 = (blockIdx.x % a.gxt) * TX;
    const int rb = blockIdx.x / a.gxt;
    const int R = taps.radius;
    const int rows = a.ny * a.nz;
    const int N = a.nx * rows;
    double s1 = 0.0, s2 = 0.0, sse = 0.0;

    for (int it = 0; it < a.rows_per_block; ++it) {
        const int r = (rb * a.rows_per_block + it) * W + wrow;  // row index y + ny * z
        const bool row_ok = r < rows;
        if (row_ok) {
            const int y = r % a.ny, z = r / a.ny;
            for (int p = lane; p < TX + 2 * R; p += TX) {
                const int xx = x0 - R + p;
                float u0, u1, u2;
                double adr, av, d2;
                force_point<V>(a, clampi(xx, a.nx), y, z, u0, u1, u2, adr, av, d2);
                ul[0][wrow][p] = u0;
                ul[1][wrow][p] = u1;
                ul[2][wrow][p] = u2;
                if (p >= R && p < TX + R && xx < a.nx) {  // a tile voxel: counted once
                    s1 += adr;
                    s2 += av;
                    sse += d2;
                }
            }
        }
        __syncthreads();
        const int x = x0 + lane;
        if (row_ok && x < a.nx) {
            const int o = x + a.nx * r;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float s = 0.0f;
                for (int j = 0; j <= 2 * R; ++j) s = fmaf(wl[j], ul[c][wrow][lane + j], s);
                a.out[c * N + o] = s;
            }
        }
        __syncthreads();
    }

    // ---- sums: fixed-order workgroup reduction into this workgroup's slots ----
    block_sum3(s1, s2, sse, tid);
    if (tid == 0) {
        const int nb = gridDim.x;
        a.partials[blockIdx.x] = s1;
        a.partials[nb + blockIdx.x] = s2;
        a.partials[2 * nb + blockIdx.x] = sse;
    }
}

__global__ __launch_bounds__(256) void k_finalize(SumsReduce red, int n)
{
    reduce_sums(red.partials, red.nb, red.hist, n, red.st, red.eps, red.inv_n, threadIdx.x);
}

__global__ void k_level_reset(LevelState *st)
{
    if (threadIdx.x == 0) {
        st->stop_at = kNeverStopped;
        st->iters_run = 0;
    }
}

struct ForceGrid {
    int tx, gxt, rows_per_block;
    int64_t blocks;
};

// Workgroups per launch to aim for: volumes with more row steps give each
// workgroup several, which bounds the number of sum slots.
constexpr int64_t kTargetForceBlocks = 8192;

ForceGrid force_grid(Dims d)
{
    ForceGrid g;
    g.tx = d.nx <= 64 ? 64 : (d.nx <= 128 ? 128 : 256);
    const int w = 256 / g.tx;
    g.gxt = ceil_div(d.nx, g.tx);
    const int64_t steps = ((int64_t)d.ny * d.nz + w - 1) / w;  // row steps of the whole volume
    const int64_t per_tile = (kTargetForceBlocks + g.gxt - 1) / g.gxt;
    g.rows_per_block = (int)((steps + per_tile - 1) / per_tile);
    if (g.rows_per_block < 1) g.rows_per_block = 1;
    g.blocks = (int64_t)g.gxt * ((steps + g.rows_per_block - 1) / g.rows_per_block);
    return g;
}

template <int V>
void launch_force_v(Ctx &c, const ForceGrid &g, const ForceArgs &a, const GaussTaps &taps)
{
    const dim3 grid((unsigned)g.blocks), block(256);
    if (g.tx == 64) hipLaunchKernelGGL((k_force_x<V, 64>), grid, block, 0, c.stream, a, taps);
    else if (g.tx == 128) hipLaunchKernelGGL((k_force_x<V, 128>), grid, block, 0, c.stream, a, taps);
    else hipLaunchKernelGGL((k_force_x<V, 256>), grid, block, 0, c.stream, a, taps);
}

}  // namespace

int64_t force_blocks(Dims d) { return force_grid(d).blocks; }

hipError_t launch_force(Ctx &c, const ForceLaunch &f)
{
    const ForceGrid g = force_grid(f.d);
    ForceArgs a;
    a.S = f.S;
    a.M = f.M;
    a.v = f.v;
    a.Im = f.Im;
    a.Is = f.Is;
    a.nx = f.d.nx;
    a.ny = f.d.ny;
    a.nz = f.d.nz;
    a.alpha2 = f.alpha2;
    a.out = f.out;
    a.partials = f.partials;
    a.stop_at = f.stop_at;
    a.n = f.n;
    a.rows_per_block = g.rows_per_block;
    a.gxt = g.gxt;
    return timed(c, K_FORCE, [&] {
        switch (f.variant) {
        case kPassive: launch_force_v<kPassive>(c, g, a, *f.taps); break;
        case kEvolved: launch_force_v<kEvolved>(c, g, a, *f.taps); break;
        case kActive: launch_force_v<kActive>(c, g, a, *f.taps); break;
        case kDouble: launch_force_v<kDouble>(c, g, a, *f.taps); break;
        default: launch_force_v<kInverseConsistent>(c, g, a, *f.taps); break;
        }
    });
}

hipError_t launch_finalize(Ctx &c, const SumsReduce &red, int n)
{
    return timed(c, K_FINALIZE, [&] { hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c.stream, red, n); });
}

hipError_t launch_level_reset(Ctx &c, LevelState *st)
{
    return timed(c, K_LEVEL_RESET, [&] { hipLaunchKernelGGL(k_level_reset, dim3(1), dim3(64), 0, c.stream, st); });
}

}  // namespace dir
