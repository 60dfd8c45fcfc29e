// gfx950 kernels of the demons registration hot path.
//
// Layout: float32 volumes [nz][ny][nx], x fastest; fields are three such
// planes (x, y, z components) in voxel units.  Every kernel maps a 64-wide
// wavefront along x so global loads and stores of a row are coalesced; the
// workgroup is 64 x 4 (four wavefronts on four rows).  Grids are flattened to
// one dimension and decoded per workgroup, so no grid dimension limits apply.
//
// Numerics: FP32 arithmetic, per-voxel sums accumulated in FP64, FP64
// workgroup partials reduced in a fixed order (bitwise reproducible).
#include <math.h>

#include "dir_internal.h"

namespace dir {

namespace {

constexpr float kDenomFloor = 1e-9f;  // force is zero at or below this denominator

__device__ __forceinline__ int clampi(int i, int n) { return min(max(i, 0), n - 1); }

// Cell and weight along one axis for trilinear interpolation with the
// coordinate clamped to [0, n-1] (Sec 2.5 interpolation kernel; explicit
// weights, no hardware filtering).  NaN coordinates clamp to 0.
__device__ __forceinline__ void axis_cell(float p, int n, int &i0, int &i1, float &t)
{
    p = fminf(fmaxf(p, 0.0f), (float)(n - 1));
    int i = (int)p;                  // p >= 0, so truncation is floor
    i = max(min(i, n - 2), 0);       // last cell for p = n-1; n == 1 gives 0
    t = p - (float)i;                // n == 1: p = 0, t = 0
    i0 = i;
    i1 = min(i + 1, n - 1);
}

struct Cell {
    int o000, o100, o010, o110, o001, o101, o011, o111;
    float tx, ty, tz;
};

__device__ __forceinline__ Cell make_cell(float px, float py, float pz, int nx, int ny, int nz)
{
    int x0, x1, y0, y1, z0, z1;
    Cell c;
    axis_cell(px, nx, x0, x1, c.tx);
    axis_cell(py, ny, y0, y1, c.ty);
    axis_cell(pz, nz, z0, z1, c.tz);
    const int r00 = nx * (y0 + ny * z0), r10 = nx * (y1 + ny * z0);
    const int r01 = nx * (y0 + ny * z1), r11 = nx * (y1 + ny * z1);
    c.o000 = r00 + x0;
    c.o100 = r00 + x1;
    c.o010 = r10 + x0;
    c.o110 = r10 + x1;
    c.o001 = r01 + x0;
    c.o101 = r01 + x1;
    c.o011 = r11 + x0;
    c.o111 = r11 + x1;
    return c;
}

__device__ __forceinline__ float lerp1(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ float sample(const float *__restrict__ I, const Cell &c)
{
    const float c00 = lerp1(I[c.o000], I[c.o100], c.tx);
    const float c10 = lerp1(I[c.o010], I[c.o110], c.tx);
    const float c01 = lerp1(I[c.o001], I[c.o101], c.tx);
    const float c11 = lerp1(I[c.o011], I[c.o111], c.tx);
    return lerp1(lerp1(c00, c10, c.ty), lerp1(c01, c11, c.ty), c.tz);
}

__device__ __forceinline__ float trilerp(const float *__restrict__ I, float px, float py, float pz, int nx, int ny,
                                         int nz)
{
    return sample(I, make_cell(px, py, pz, nx, ny, nz));
}

// Decode a flattened workgroup id into (tile x, tile y, z).
struct Tile {
    int x, y, z;
};
__device__ __forceinline__ Tile decode_tile(int gx, int gy)
{
    const int b = blockIdx.x;
    Tile t;
    t.x = b % gx;
    const int r = b / gx;
    t.y = r % gy;
    t.z = r / gy;
    return t;
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Central difference with clamped neighbours (Sec 2.5 gradient kernel).
__device__ __forceinline__ void central_diff(const float *__restrict__ I, int x, int y, int z, int nx, int ny, int nz,
                                             float &gx, float &gy, float &gz)
{
    const int row = nx * (y + ny * z);
    gx = 0.5f * (I[row + min(x + 1, nx - 1)] - I[row + max(x - 1, 0)]);
    gy = 0.5f * (I[nx * (min(y + 1, ny - 1) + ny * z) + x] - I[nx * (max(y - 1, 0) + ny * z) + x]);
    gz = 0.5f * (I[nx * (y + ny * min(z + 1, nz - 1)) + x] - I[nx * (y + ny * max(z - 1, 0)) + x]);
}

// Demons term D g / (alpha^2 D^2 + |g|^2) (Eqs 1, 3, 6; alpha of Eq 5).
__device__ __forceinline__ void demons_term(float D, float gx, float gy, float gz, float alpha2, float &fx, float &fy,
                                            float &fz)
{
    const float den = fmaf(alpha2 * D, D, fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
    if (den <= kDenomFloor) {
        fx = fy = fz = 0.0f;
        return;
    }
    const float s = D / den;
    fx = s * gx;
    fy = s * gy;
    fz = s * gz;
}

// Evolved passive force, Eq 2, with both gradient magnitudes squared in the
// second denominator factor; a = |grad| of the undeformed moving image.
__device__ __forceinline__ void evolved_term(float D, float gx, float gy, float gz, float a, float &fx, float &fy,
                                             float &fz)
{
    const float G2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
    const float a2 = a * a;
    const float den = (fmaf(2.0f * D, D, G2 + a2)) * (G2 + a2);
    if (den <= kDenomFloor) {
        fx = fy = fz = 0.0f;
        return;
    }
    const float s = 4.0f * D * sqrtf(G2) * a / den;
    fx = s * gx;
    fy = s * gy;
    fz = s * gz;
}

// Workgroup sum of three doubles in a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c)
{
    __shared__ double red[3][kBlockX * kBlockY / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    const int tid = threadIdx.x + kBlockX * threadIdx.y;
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
    }
    __syncthreads();
    if (tid == 0) {
        a = red[0][0];
        b = red[1][0];
        c = red[2][0];
        for (int w = 1; w < kBlockX * kBlockY / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
            c += red[2][w];
        }
    }
}

// ------------------------------------------------------------------------
// Pyramid (Sec 2.3)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_restrict(const float *__restrict__ in, int nx, int ny, int nz,
                                                  float *__restrict__ out, int cx, int cy, int cz, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int i = t.x * kBlockX + threadIdx.x, j = t.y * kBlockY + threadIdx.y, k = t.z;
    if (i >= cx || j >= cy) return;
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int row = nx * (min(2 * j + b, ny - 1) + ny * min(2 * k + c, nz - 1));
            s += in[row + min(2 * i, nx - 1)] + in[row + min(2 * i + 1, nx - 1)];
        }
    out[i + cx * (j + cy * k)] = 0.125f * s;
}

__global__ __launch_bounds__(256) void k_prolong(const float *__restrict__ vc, int cx, int cy, int cz,
                                                 float *__restrict__ vf, int fx, int fy, int fz, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= fx || y >= fy) return;
    // fine index f sits at coarse coordinate (f - 0.5) / 2
    const Cell c = make_cell(0.5f * x - 0.25f, 0.5f * y - 0.25f, 0.5f * z - 0.25f, cx, cy, cz);
    const int Nc = cx * cy * cz, Nf = fx * fy * fz;
    const int i = x + fx * (y + fy * z);
    vf[i] = 2.0f * sample(vc, c);
    vf[Nf + i] = 2.0f * sample(vc + Nc, c);
    vf[2 * Nf + i] = 2.0f * sample(vc + 2 * Nc, c);
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
                                              const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    out[i] = trilerp(I, (float)x - v[i], (float)y - v[N + i], (float)z - v[2 * N + i], nx, ny, nz);
}

// Inverse-consistent pair: Im = M(x - h), Is = S(x + h) (Sec 2.2, after Eq 6).
__global__ __launch_bounds__(256) void k_warp_pair(const float *__restrict__ M, const float *__restrict__ S,
                                                   const float *__restrict__ h, int nx, int ny, int nz,
                                                   float *__restrict__ Im, float *__restrict__ Is, int gx, int gy,
                                                   const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    const float hx = h[i], hy = h[N + i], hz = h[2 * N + i];
    Im[i] = trilerp(M, (float)x - hx, (float)y - hy, (float)z - hz, nx, ny, nz);
    Is[i] = trilerp(S, (float)x + hx, (float)y + hy, (float)z + hz, nx, ny, nz);
}

// ------------------------------------------------------------------------
// Force + field update + FP64 workgroup sums (Eqs 1-6; Sec 2.4 norms)
// ------------------------------------------------------------------------
template <int V>
__global__ __launch_bounds__(256) void k_force(const float *__restrict__ S, const float *__restrict__ M,
                                               const float *__restrict__ v, const float *__restrict__ Im,
                                               const float *__restrict__ Is, int nx, int ny, int nz, float alpha2,
                                               float *__restrict__ u, double *__restrict__ partials, int gx, int gy,
                                               const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    double s1 = 0.0, s2 = 0.0, sse = 0.0;
    if (x < nx && y < ny) {
        const int N = nx * ny * nz, i = x + nx * (y + ny * z);
        const float vx = v[i], vy = v[N + i], vz = v[2 * N + i];
        float fx = 0.0f, fy = 0.0f, fz = 0.0f, D;
        if (V == kInverseConsistent) {
            float ax, ay, az, bx, by, bz;
            central_diff(Im, x, y, z, nx, ny, nz, ax, ay, az);
            central_diff(Is, x, y, z, nx, ny, nz, bx, by, bz);
            D = Im[i] - Is[i];
            demons_term(D, ax + bx, ay + by, az + bz, alpha2, fx, fy, fz);
        } else {
            const float im = (V == kPassive || V == kEvolved)
                                 ? trilerp(M, (float)x - vx, (float)y - vy, (float)z - vz, nx, ny, nz)
                                 : Im[i];
            D = im - S[i];
            float sx = 0.0f, sy = 0.0f, sz = 0.0f;
            if (V == kPassive || V == kDouble || V == kEvolved) central_diff(S, x, y, z, nx, ny, nz, sx, sy, sz);
            if (V == kPassive || V == kDouble) demons_term(D, sx, sy, sz, alpha2, fx, fy, fz);
            if (V == kActive || V == kDouble) {
                float mx, my, mz, ax, ay, az;
                central_diff(Im, x, y, z, nx, ny, nz, mx, my, mz);
                demons_term(D, mx, my, mz, alpha2, ax, ay, az);
                fx += ax;
                fy += ay;
                fz += az;
            }
            if (V == kEvolved) {
                float mx, my, mz;
                central_diff(M, x, y, z, nx, ny, nz, mx, my, mz);
                evolved_term(D, sx, sy, sz, sqrtf(fmaf(mx, mx, fmaf(my, my, mz * mz))), fx, fy, fz);
            }
        }
        u[i] = vx + fx;
        u[N + i] = vy + fy;
        u[2 * N + i] = vz + fz;
        s1 = (double)sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
        s2 = (double)sqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
        sse = (double)D * (double)D;
    }
    block_sum3(s1, s2, sse);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double *p = partials + 3 * (int64_t)blockIdx.x;
        p[0] = s1;
        p[1] = s2;
        p[2] = sse;
    }
}

// Fixed-order reduction of the workgroup partials; history entry and the
// stopping rule of Sec 2.4 (l(n-10) - l(n) <= eps).
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(const double *__restrict__ partials, int64_t nblocks,
                                                               double inv_n, double *__restrict__ hist, int n,
                                                               LevelState *__restrict__ st, double eps)
{
    if (st->stop) return;
    __shared__ double red[3][kFinalizeThreads];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t k = threadIdx.x; k < nblocks; k += kFinalizeThreads) {
        a += partials[3 * k];
        b += partials[3 * k + 1];
        c += partials[3 * k + 2];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    red[2][threadIdx.x] = c;
    __syncthreads();
    for (int s = kFinalizeThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] += red[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s1 = red[0][0], s2 = red[1][0], sse = red[2][0];
        const double l = s2 > 0.0 ? s1 / s2 : __builtin_nan("");
        double *e = hist + 4 * (int64_t)n;
        e[0] = s1;
        e[1] = s2;
        e[2] = sse * inv_n;
        e[3] = l;
        st->iters_run = n + 1;
        if (eps > 0.0 && n >= 10) {
            const double l10 = hist[4 * (int64_t)(n - 10) + 3];
            if (!isnan(l) && !isnan(l10) && l10 - l <= eps) st->stop = 1;
        }
    }
}

__global__ void k_level_reset(LevelState *st)
{
    if (threadIdx.x == 0) {
        st->stop = 0;
        st->iters_run = 0;
    }
}

// ------------------------------------------------------------------------
// Gaussian smoothing (Sec 2.1; Sec 2.5 separable low-pass filter)
// ------------------------------------------------------------------------
// x pass: each wavefront stages its row segment plus a radius-R halo in LDS.
__global__ __launch_bounds__(256) void k_smooth_x(const float *__restrict__ in, float *__restrict__ out, int ncomp,
                                                  int nx, int ny, int nz, GaussTaps taps, int gx, int gy,
                                                  const int *__restrict__ stop)
{
    if (stop && *stop) return;
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

// y and z passes: each thread slides a register window of T + 2R samples
// along the axis and writes T consecutive outputs.
template <int R, int T>
__global__ __launch_bounds__(256) void k_smooth_axis(const float *__restrict__ in, float *__restrict__ out, int ncomp,
                                                     int nx, int ny, int nz, int axis, GaussTaps taps, int gx, int gy,
                                                     const int *__restrict__ stop)
{
    if (stop && *stop) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x;
    int y, z, a0, n, stride;
    if (axis == 1) {  // tile y covers kBlockY * T rows; one segment per wavefront
        y = t.y * (kBlockY * T) + threadIdx.y * T;
        z = t.z;
        a0 = y;
        n = ny;
        stride = nx;
    } else {          // tile y covers kBlockY rows; tile z is a segment of T planes
        y = t.y * kBlockY + threadIdx.y;
        z = t.z * T;
        a0 = z;
        n = nz;
        stride = nx * ny;
    }
    if (x >= nx || y >= ny || z >= nz) return;
    const int N = nx * ny * nz;
    float w[2 * R + 1];
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) w[j] = taps.w[j];
    const int base = x + nx * (axis == 1 ? ny * z : y);  // offset with the swept coordinate at 0
    for (int c = 0; c < ncomp; ++c) {
        const float *src = in + (int64_t)c * N + base;
        float *dst = out + (int64_t)c * N + base;
        float win[T + 2 * R];
#pragma unroll
        for (int j = 0; j < T + 2 * R; ++j) win[j] = src[clampi(a0 - R + j, n) * stride];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) s = fmaf(w[j], win[k + j], s);
            if (a0 + k < n) dst[(a0 + k) * stride] = s;
        }
    }
}

// ------------------------------------------------------------------------
// Inverse-consistent output composition: w(z) = 2 h(p), p = z - h(p)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_compose(const float *__restrict__ h, int nx, int ny, int nz, int K,
                                                 float *__restrict__ out, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    float px = (float)x, py = (float)y, pz = (float)z;
    for (int k = 0; k < K; ++k) {
        const Cell c = make_cell(px, py, pz, nx, ny, nz);
        const float hx = sample(h, c), hy = sample(h + N, c), hz = sample(h + 2 * N, c);
        px = (float)x - hx;
        py = (float)y - hy;
        pz = (float)z - hz;
    }
    const Cell c = make_cell(px, py, pz, nx, ny, nz);
    out[i] = 2.0f * sample(h, c);
    out[N + i] = 2.0f * sample(h + N, c);
    out[2 * N + i] = 2.0f * sample(h + 2 * N, c);
}

__global__ __launch_bounds__(256) void k_zero(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0f;
}

// ------------------------------------------------------------------------
// launch helpers
// ------------------------------------------------------------------------
struct Grid2 {
    int gx, gy;
    int64_t blocks;
};

Grid2 plane_grid(Dims d)
{
    Grid2 g;
    g.gx = ceil_div(d.nx, kBlockX);
    g.gy = ceil_div(d.ny, kBlockY);
    g.blocks = (int64_t)g.gx * g.gy * d.nz;
    return g;
}

template <typename F>
hipError_t timed(Ctx &c, int k, F &&launch)
{
    hipEvent_t a = nullptr;
    if (c.timer && c.timer->on(k)) {
        hipError_t e = c.timer->begin(k, c.stream, &a);
        if (e != hipSuccess) return e;
    }
    launch();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a) return c.timer->end(k, c.stream, a);
    return hipSuccess;
}

const dim3 kBlock(kBlockX, kBlockY, 1);

template <int R>
hipError_t launch_axis_r(Ctx &c, const float *in, float *out, int ncomp, Dims d, int axis, const GaussTaps &taps,
                         const int *stop)
{
    constexpr int T = 16;
    int gx = ceil_div(d.nx, kBlockX), gy, gz;
    if (axis == 1) {
        gy = ceil_div(d.ny, kBlockY * T);
        gz = d.nz;
    } else {
        gy = ceil_div(d.ny, kBlockY);
        gz = ceil_div(d.nz, T);
    }
    const int64_t blocks = (int64_t)gx * gy * gz;
    return timed(c, axis == 1 ? K_SMOOTH_Y : K_SMOOTH_Z, [&] {
        hipLaunchKernelGGL((k_smooth_axis<R, T>), dim3((unsigned)blocks), kBlock, 0, c.stream, in, out, ncomp, d.nx,
                           d.ny, d.nz, axis, taps, gx, gy, stop);
    });
}

hipError_t launch_axis(Ctx &c, const float *in, float *out, int ncomp, Dims d, int axis, const GaussTaps &taps,
                       const int *stop)
{
    switch (taps.radius) {
#define DIR_R(r) \
    case r: return launch_axis_r<r>(c, in, out, ncomp, d, axis, taps, stop);
        DIR_R(0) DIR_R(1) DIR_R(2) DIR_R(3) DIR_R(4) DIR_R(5) DIR_R(6) DIR_R(7) DIR_R(8)
        DIR_R(9) DIR_R(10) DIR_R(11) DIR_R(12) DIR_R(13) DIR_R(14) DIR_R(15) DIR_R(16)
#undef DIR_R
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_zero(Ctx &c, float *p, int64_t n)
{
    const int64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    return timed(c, K_FILL, [&] { hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, c.stream, p, n); });
}

int64_t force_blocks(Dims d) { return plane_grid(d).blocks; }

hipError_t launch_restrict(Ctx &c, const float *in, Dims fine, float *out, Dims coarse)
{
    const Grid2 g = plane_grid(coarse);
    return timed(c, K_RESTRICT, [&] {
        hipLaunchKernelGGL(k_restrict, dim3((unsigned)g.blocks), kBlock, 0, c.stream, in, fine.nx, fine.ny, fine.nz,
                           out, coarse.nx, coarse.ny, coarse.nz, g.gx, g.gy);
    });
}

hipError_t launch_prolong(Ctx &c, const float *vc, Dims coarse, float *vf, Dims fine)
{
    const Grid2 g = plane_grid(fine);
    return timed(c, K_PROLONG, [&] {
        hipLaunchKernelGGL(k_prolong, dim3((unsigned)g.blocks), kBlock, 0, c.stream, vc, coarse.nx, coarse.ny,
                           coarse.nz, vf, fine.nx, fine.ny, fine.nz, g.gx, g.gy);
    });
}

hipError_t launch_gradient(Ctx &c, const float *img, Dims d, float *grad)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_GRADIENT, [&] {
        hipLaunchKernelGGL(k_gradient, dim3((unsigned)g.blocks), kBlock, 0, c.stream, img, d.nx, d.ny, d.nz, grad,
                           g.gx, g.gy);
    });
}

hipError_t launch_warp(Ctx &c, const float *img, const float *field, Dims d, float *out, const int *stop)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_WARP, [&] {
        hipLaunchKernelGGL(k_warp, dim3((unsigned)g.blocks), kBlock, 0, c.stream, img, field, d.nx, d.ny, d.nz, out,
                           g.gx, g.gy, stop);
    });
}

hipError_t launch_warp_pair(Ctx &c, const float *M, const float *S, const float *h, Dims d, float *Im, float *Is,
                            const int *stop)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_WARP_PAIR, [&] {
        hipLaunchKernelGGL(k_warp_pair, dim3((unsigned)g.blocks), kBlock, 0, c.stream, M, S, h, d.nx, d.ny, d.nz, Im,
                           Is, g.gx, g.gy, stop);
    });
}

hipError_t launch_force(Ctx &c, int variant, float alpha2, const float *S, const float *M, const float *v,
                        const float *Im, const float *Is, Dims d, float *u, double *partials, const int *stop)
{
    const Grid2 g = plane_grid(d);
    const dim3 grid((unsigned)g.blocks);
    return timed(c, K_FORCE, [&] {
        switch (variant) {
        case kPassive:
            hipLaunchKernelGGL(k_force<kPassive>, grid, kBlock, 0, c.stream, S, M, v, Im, Is, d.nx, d.ny, d.nz,
                               alpha2, u, partials, g.gx, g.gy, stop);
            break;
        case kEvolved:
            hipLaunchKernelGGL(k_force<kEvolved>, grid, kBlock, 0, c.stream, S, M, v, Im, Is, d.nx, d.ny, d.nz,
                               alpha2, u, partials, g.gx, g.gy, stop);
            break;
        case kActive:
            hipLaunchKernelGGL(k_force<kActive>, grid, kBlock, 0, c.stream, S, M, v, Im, Is, d.nx, d.ny, d.nz,
                               alpha2, u, partials, g.gx, g.gy, stop);
            break;
        case kDouble:
            hipLaunchKernelGGL(k_force<kDouble>, grid, kBlock, 0, c.stream, S, M, v, Im, Is, d.nx, d.ny, d.nz,
                               alpha2, u, partials, g.gx, g.gy, stop);
            break;
        default:
            hipLaunchKernelGGL(k_force<kInverseConsistent>, grid, kBlock, 0, c.stream, S, M, v, Im, Is, d.nx, d.ny,
                               d.nz, alpha2, u, partials, g.gx, g.gy, stop);
            break;
        }
    });
}

hipError_t launch_smooth(Ctx &c, const float *in, int ncomp, Dims d, const GaussTaps &taps, float *out, float *tmp,
                         const int *stop)
{
    const Grid2 g = plane_grid(d);
    hipError_t e = timed(c, K_SMOOTH_X, [&] {
        hipLaunchKernelGGL(k_smooth_x, dim3((unsigned)g.blocks), kBlock, 0, c.stream, in, out, ncomp, d.nx, d.ny,
                           d.nz, taps, g.gx, g.gy, stop);
    });
    if (e != hipSuccess) return e;
    e = launch_axis(c, out, tmp, ncomp, d, 1, taps, stop);
    if (e != hipSuccess) return e;
    return launch_axis(c, tmp, out, ncomp, d, 2, taps, stop);
}

hipError_t launch_finalize(Ctx &c, const double *partials, int64_t nblocks, double inv_n, double *hist_level, int n,
                           LevelState *st, double eps)
{
    return timed(c, K_FINALIZE, [&] {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, c.stream, partials, nblocks, inv_n,
                           hist_level, n, st, eps);
    });
}

hipError_t launch_level_reset(Ctx &c, LevelState *st)
{
    return timed(c, K_LEVEL_RESET,
                 [&] { hipLaunchKernelGGL(k_level_reset, dim3(1), dim3(64), 0, c.stream, st); });
}

hipError_t launch_compose(Ctx &c, const float *h, Dims d, int K, float *out)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_COMPOSE, [&] {
        hipLaunchKernelGGL(k_compose, dim3((unsigned)g.blocks), kBlock, 0, c.stream, h, d.nx, d.ny, d.nz, K, out,
                           g.gx, g.gy);
    });
}

}  // namespace dir
