// gfx950 kernels for the image pyramid (Sec 2.3), deformed images (Sec 2.5
// interpolation kernel), plain gradients (Sec 2.5 gradient kernel) and the
// inverse-consistent output composition.
#include "device_common.h"

namespace dir {
namespace {

using namespace dev;

// ------------------------------------------------------------------------
// Pyramid (Sec 2.3)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_restrict(const float *__restrict__ in, int nx, int ny, int nz,
                                                  float *__restrict__ out, int cx, int cy, int cz, int gx, int gy)
{
    const Tile t = decode_tile(gx, gy);
    const int i = t.x * kBlockX + threadIdx.x, j = t.y * kBlockY + threadIdx.y, k = t.z;
    if (i >= cx || j >= cy) return;
    // FP64 sum, rounded once: coarse images feed intensity differences
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int row = nx * (min(2 * j + b, ny - 1) + ny * min(2 * k + c, nz - 1));
            s += (double)in[row + min(2 * i, nx - 1)] + (double)in[row + min(2 * i + 1, nx - 1)];
        }
    out[i + cx * (j + cy * k)] = (float)(0.125 * s);
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
                                              const int *__restrict__ stop_at, int n)
{
    if (stop_at && *stop_at < n) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const int N = nx * ny * nz, i = x + nx * (y + ny * z);
    out[i] = (float)sample64(I, make_cell_disp(x, y, z, v[i], v[N + i], v[2 * N + i], nx, ny, nz));
}

// Intensity difference for the active and double forces: D = M(x - v) - S(x),
// sampled and subtracted in FP64, rounded once.  The force kernel takes D and
// its gradient from here (grad Im = grad D + grad S), so the gather happens
// once per iteration.  Buffer addressing as in the force kernel.
__global__ __launch_bounds__(256) void k_warp_diff(const float *__restrict__ M, const float *__restrict__ S,
                                                   const float *__restrict__ v, int nx, int ny, int nz,
                                                   float *__restrict__ D, int gx, int gy,
                                                   const int *__restrict__ stop_at, int n)
{
    if (stop_at && *stop_at < n) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const unsigned nbytes = 4u * (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, nbytes), rS = make_rsrc(S, nbytes), rv = make_rsrc(v, 3u * nbytes),
                                 rD = make_rsrc(D, nbytes);
    const unsigned o = 4u * (unsigned)(x + nx * (y + ny * z));
    const float vx = bload(rv, o, 0), vy = bload(rv, o, nbytes), vz = bload(rv, o, 2u * nbytes);
    const double d = bsample64(rM, bcell_disp(x, y, z, vx, vy, vz, nx, ny, nz)) - (double)bload(rS, o, 0);
    bstore(rD, (float)d, o, 0);
}

// Inverse-consistent pair (Sec 2.2, after Eq 6): Im = M(x - h), Is = S(x + h),
// written as D = Im - Is and P = Im + Is (the force needs D and grad P).
// Both formed in FP64 and rounded once.
__global__ __launch_bounds__(256) void k_warp_pair(const float *__restrict__ M, const float *__restrict__ S,
                                                   const float *__restrict__ h, int nx, int ny, int nz,
                                                   float *__restrict__ D, float *__restrict__ P, int gx, int gy,
                                                   const int *__restrict__ stop_at, int n)
{
    if (stop_at && *stop_at < n) return;
    const Tile t = decode_tile(gx, gy);
    const int x = t.x * kBlockX + threadIdx.x, y = t.y * kBlockY + threadIdx.y, z = t.z;
    if (x >= nx || y >= ny) return;
    const unsigned nbytes = 4u * (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const __amdgpu_buffer_rsrc_t rM = make_rsrc(M, nbytes), rS = make_rsrc(S, nbytes), rh = make_rsrc(h, 3u * nbytes),
                                 rD = make_rsrc(D, nbytes), rP = make_rsrc(P, nbytes);
    const unsigned o = 4u * (unsigned)(x + nx * (y + ny * z));
    const float hx = bload(rh, o, 0), hy = bload(rh, o, nbytes), hz = bload(rh, o, 2u * nbytes);
    const double im = bsample64(rM, bcell_disp(x, y, z, hx, hy, hz, nx, ny, nz));
    const double is = bsample64(rS, bcell_disp(x, y, z, -hx, -hy, -hz, nx, ny, nz));
    bstore(rD, (float)(im - is), o, 0);
    bstore(rP, (float)(im + is), o, 0);
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
    const unsigned nbytes = 4u * (unsigned)nx * (unsigned)ny * (unsigned)nz;
    const __amdgpu_buffer_rsrc_t H = make_rsrc(h, 3u * nbytes);
    // p = (x, y, z) - (hx, hy, hz): the position is kept as the displacement
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    for (int k = 0; k < K; ++k) bsample3(H, bcell_disp(x, y, z, hx, hy, hz, nx, ny, nz), nbytes, hx, hy, hz);
    float ax, ay, az;
    bsample3(H, bcell_disp(x, y, z, hx, hy, hz, nx, ny, nz), nbytes, ax, ay, az);
    const __amdgpu_buffer_rsrc_t O = make_rsrc(out, 3u * nbytes);
    const unsigned o = 4u * (unsigned)(x + nx * (y + ny * z));
    bstore(O, 2.0f * ax, o, 0u);
    bstore(O, 2.0f * ay, o, nbytes);
    bstore(O, 2.0f * az, o, 2u * nbytes);
}

__global__ __launch_bounds__(256) void k_zero(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0f;
}


}  // namespace

hipError_t launch_zero(Ctx &c, float *p, int64_t n)
{
    const int64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    return timed(c, K_FILL, [&](const Ev &ev) { go(c, ev, k_zero, dim3(blocks), dim3(256), p, n); });
}

hipError_t launch_restrict(Ctx &c, const float *in, Dims fine, float *out, Dims coarse)
{
    const Grid2 g = plane_grid(coarse);
    return timed(c, K_RESTRICT, [&](const Ev &ev) {
        go(c, ev, k_restrict, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), in, fine.nx,
                           fine.ny, fine.nz, out, coarse.nx, coarse.ny, coarse.nz, g.gx, g.gy);
    });
}

hipError_t launch_prolong(Ctx &c, const float *vc, Dims coarse, float *vf, Dims fine)
{
    const Grid2 g = plane_grid(fine);
    return timed(c, K_PROLONG, [&](const Ev &ev) {
        go(c, ev, k_prolong, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), vc, coarse.nx,
                           coarse.ny, coarse.nz, vf, fine.nx, fine.ny, fine.nz, g.gx, g.gy);
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

hipError_t launch_warp_diff(Ctx &c, const float *M, const float *S, const float *v, Dims d, float *D,
                            const int *stop_at, int n)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_WARP, [&](const Ev &ev) {
        go(c, ev, k_warp_diff, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), M, S, v, d.nx,
                           d.ny, d.nz, D, g.gx, g.gy, stop_at, n);
    });
}

hipError_t launch_warp_pair(Ctx &c, const float *M, const float *S, const float *h, Dims d, float *D, float *P,
                            const int *stop_at, int n)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_WARP_PAIR, [&](const Ev &ev) {
        go(c, ev, k_warp_pair, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), M, S, h, d.nx,
                           d.ny, d.nz, D, P, g.gx, g.gy, stop_at, n);
    });
}

hipError_t launch_compose(Ctx &c, const float *h, Dims d, int K, float *out)
{
    const Grid2 g = plane_grid(d);
    return timed(c, K_COMPOSE, [&](const Ev &ev) {
        go(c, ev, k_compose, dim3((unsigned)g.blocks), dim3(kBlockX, kBlockY), h, d.nx, d.ny,
                           d.nz, K, out, g.gx, g.gy);
    });
}

}  // namespace dir
