// gfx950 kernel of one demons force step (Eqs 1-6), fused with the x pass of
// the Gaussian smoothing (Sec 2.5 low-pass filter) and the per-workgroup FP64
// sums behind the relative norm of Sec 2.4.
//
// A workgroup of 256 threads owns an x tile of TX voxels (TX = 64, 128, 256
// or 512; 256/TX rows in flight when TX < 256, and TX/256 voxels per thread
// when TX = 512) and walks `rows_per_block` row steps.  For each
// row it evaluates u = v + dr at the TX tile voxels plus an R-voxel halo on
// both sides where the halo lies inside the row (past a row end the halo is
// the end voxel's u, by index clamping, and is copied, not recomputed: a
// tile spanning the whole row evaluates each voxel once), stages u in LDS
// and writes the x-smoothed field.  The per-voxel sums
// sum|dr|, sum|v| and sum D^2 are accumulated in FP64 over the tile voxels
// only, reduced per workgroup in a fixed order and written to per-workgroup
// slots.  The slots are added up, in slot order, by one workgroup of the
// kernel that runs next (no cross-workgroup fences inside this kernel: on a
// multi-XCD device an agent-scope release per workgroup costs an L2
// write-back each).
#include <string.h>

#include "device_common.h"

namespace dir {
namespace {

using namespace dev;

// Volumes are in the storage format of the kernel instance (StF32, StF16 or
// StBF16); the pointers are untyped.  One launch serves `count` registrations
// (a lockstep batch; 1 outside batches), possibly of different sizes with the
// same tile width TX: per-registration arguments are arrays indexed by
// registration, and each registration has its own set of workgroups
// (interleaved over the XCDs by batch_slot).
// Volume size and workgroup layout of one registration of a launch.
struct Geo {
    int nx, ny, nz;
    int gxt;             // x tiles
    int gy;              // groups of W rows along y
    int rows_per_block;  // row steps per workgroup: consecutive planes z of one y group
    int blocks;          // workgroups
};

struct ForceArgs {
    const void *S[kMaxBatch], *M[kMaxBatch], *v[kMaxBatch];
    const void *Dd[kMaxBatch], *P[kMaxBatch];  // pre-warped D (active, double, IC) and P = Im + Is (IC, always FP32)
    void *out[kMaxBatch];           // x-smoothed u (u itself with identity taps)
    double *partials[kMaxBatch];    // 3 * blocks doubles each: s1[], s2[], sse[]
    const int *stop_at[kMaxBatch];  // skip when *stop_at < n (NULL: never)
    float alpha2[kMaxBatch];
    int variant[kMaxBatch];         // read by the mixed-variant instance only
    Geo geo[kMaxBatch];
    int first[kMaxBatch + 1];       // registration r has first[r + 1] - first[r] workgroups (order: batch_slot)
    int chunk[kXCDs];               // logical start of chunk k (batch_slot)
    int count;
    int n;                          // iteration index within the level
    Metric metric;                  // physical units (instances with MM = true only)
};

// Byte offsets of one wave-uniform row (y, z) and of its stencil neighbour
// rows (indices clamped), plus the lane's x offsets (x and its clamped
// neighbours).  Rows go to the scalar offset of a buffer access, x to the
// vector offset.
struct RowOffsets {
    unsigned c, ym, yp, zm, zp;  // rows (y, z), (y -+ 1, z), (y, z -+ 1)
};
struct LaneOffsets {
    unsigned c, xm, xp;          // x, x - 1, x + 1 (clamped)
};

// Central difference (Sec 2.5 gradient kernel) from a buffer; in physical
// units (MM) each component is scaled by s_a as well (gs = s / 2).
template <class St, bool MM>
__device__ __forceinline__ void cdiff(__amdgpu_buffer_rsrc_t I, const LaneOffsets &lo, const RowOffsets &ro,
                                      const Metric &m, float &gx, float &gy, float &gz)
{
    gx = (MM ? m.gs[0] : 0.5f) * (St::load(I, lo.xp, ro.c) - St::load(I, lo.xm, ro.c));
    gy = (MM ? m.gs[1] : 0.5f) * (St::load(I, lo.c, ro.yp) - St::load(I, lo.c, ro.ym));
    gz = (MM ? m.gs[2] : 0.5f) * (St::load(I, lo.c, ro.zp) - St::load(I, lo.c, ro.zm));
}

// Values of one volume along a lane's column carried from a row step to the
// next (row steps walk z): the centre and the z + 1 neighbour of the last
// step are the z - 1 neighbour and the centre of this one.
struct ZCarry {
    float c, zp;
};

// cdiff that also yields the centre: with `carry` (the previous row step was
// plane z - 1 of the same column) z - 1 and the centre come from zc, else
// they are loaded; zc receives this step's centre and z + 1 value.  The
// loaded values and the arithmetic are those of cdiff.
template <class St, bool MM>
__device__ __forceinline__ void cdiff_carry(__amdgpu_buffer_rsrc_t I, const LaneOffsets &lo, const RowOffsets &ro,
                                            const Metric &m, bool carry, ZCarry &zc, float &gx, float &gy,
                                            float &gz)
{
    float zm;
    if (carry) {
        zm = zc.c;
        zc.c = zc.zp;
    } else {
        zm = St::load(I, lo.c, ro.zm);
        zc.c = St::load(I, lo.c, ro.c);
    }
    gx = (MM ? m.gs[0] : 0.5f) * (St::load(I, lo.xp, ro.c) - St::load(I, lo.xm, ro.c));
    gy = (MM ? m.gs[1] : 0.5f) * (St::load(I, lo.c, ro.yp) - St::load(I, lo.c, ro.ym));
    zc.zp = St::load(I, lo.c, ro.zp);
    gz = (MM ? m.gs[2] : 0.5f) * (zc.zp - zm);
}

// Hardware square root and reciprocal (about 1 ulp): the force's parity
// tolerance is 1e-5 and the norms only feed FP64 sums.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// D g / (alpha^2 D^2 + |g|^2) (Eqs 1, 3, 6; alpha of Eq 5), zero at or below
// the denominator floor.
__device__ __forceinline__ void dterm(float D, float gx, float gy, float gz, float alpha2, float &fx, float &fy,
                                      float &fz)
{
    const float den = fmaf(alpha2 * D, D, fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
    const float s = den > kDenomFloor ? D * fast_rcp(den) : 0.0f;
    fx = s * gx;
    fy = s * gy;
    fz = s * gz;
}

// Eq 2 with both gradient magnitudes squared (see evolved_term).
__device__ __forceinline__ void eterm(float D, float gx, float gy, float gz, float a, float &fx, float &fy, float &fz)
{
    const float G2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
    const float a2 = a * a;
    const float den = (fmaf(2.0f * D, D, G2 + a2)) * (G2 + a2);
    const float s = den > kDenomFloor ? 4.0f * D * fast_sqrt(G2) * a * fast_rcp(den) : 0.0f;
    fx = s * gx;
    fy = s * gy;
    fz = s * gz;
}

struct Bufs {
    __amdgpu_buffer_rsrc_t S, M, v, Dd, P, out;
};

// u = v + dr at voxel (x, y, z) and its contributions |dr|, |v|, D^2.  MM:
// the force in physical units on the voxel grid (see Metric): gradients
// scaled by s, the force component a by s_a, and the norms in mm.
template <int V, class St, bool MM>
__device__ __forceinline__ void force_point(const Geo &q, float alpha2, const Bufs &b, int x, int y, int z,
                                            const RowOffsets &ro, unsigned nbytes, const Metric &m, float &u0,
                                            float &u1, float &u2, double &adr, double &av, double &d2)
{
    const int nx = q.nx, ny = q.ny, nz = q.nz;
    constexpr unsigned ES = St::kBytes;
    LaneOffsets lo;
    lo.c = ES * (unsigned)x;
    lo.xm = ES * (unsigned)max(x - 1, 0);
    lo.xp = ES * (unsigned)min(x + 1, nx - 1);
    const float vx = St::load(b.v, lo.c, ro.c), vy = St::load(b.v, lo.c, ro.c + nbytes),
                vz = St::load(b.v, lo.c, ro.c + 2u * nbytes);
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    // intensity difference: sampled in FP64 here (passive, evolved; FP32 for
    // 16-bit storage) or taken from the pre-warp kernel, which forms it the
    // same way; rounded once
    double D64;
    if constexpr (V == kPassive || V == kEvolved) {
        if constexpr (ES == 4)
            D64 = bsample64<St>(b.M, bcell_disp<ES>(x, y, z, vx, vy, vz, nx, ny, nz)) -
                  (double)St::load(b.S, lo.c, ro.c);
        else  // 16-bit storage: FP32 sample (see bsample32)
            D64 = (double)(bsample32<St, false>(b.M, bcell32<ES>(x, y, z, vx, vy, vz, nx, ny, nz)) -
                           St::load(b.S, lo.c, ro.c));
    } else {
        D64 = (double)St::load(b.Dd, lo.c, ro.c);
    }
    const float D = (float)D64;
    if (V == kInverseConsistent) {
        // Eq 6: g = grad Im + grad Is = grad P of the two deformed images.
        // P is FP32 in every storage format (it sits near twice the
        // background intensity, where 16-bit spacing would quantise grad P).
        constexpr unsigned K4 = 4u / ES;
        const LaneOffsets l4{K4 * lo.c, K4 * lo.xm, K4 * lo.xp};
        const RowOffsets r4{K4 * ro.c, K4 * ro.ym, K4 * ro.yp, K4 * ro.zm, K4 * ro.zp};
        float gx, gy, gz;
        cdiff<StF32, MM>(b.P, l4, r4, m, gx, gy, gz);
        dterm(D, gx, gy, gz, alpha2, fx, fy, fz);
    } else {
        float sx, sy, sz;
        cdiff<St, MM>(b.S, lo, ro, m, sx, sy, sz);
        if (V == kPassive || V == kDouble) dterm(D, sx, sy, sz, alpha2, fx, fy, fz);  // Eq 1
        if (V == kActive || V == kDouble) {                                             // Eq 3
            // grad Im = grad (Im - S) + grad S
            float dx, dy, dz, bx, by, bz;
            cdiff<St, MM>(b.Dd, lo, ro, m, dx, dy, dz);
            dterm(D, dx + sx, dy + sy, dz + sz, alpha2, bx, by, bz);
            fx += bx;
            fy += by;
            fz += bz;
        }
        if (V == kEvolved) {                                                            // Eq 2
            float mx, my, mz;
            cdiff<St, MM>(b.M, lo, ro, m, mx, my, mz);
            eterm(D, sx, sy, sz, fast_sqrt(fmaf(mx, mx, fmaf(my, my, mz * mz))), fx, fy, fz);
        }
    }
    if (MM) {
        fx *= m.os[0];
        fy *= m.os[1];
        fz *= m.os[2];
    }
    u0 = vx + fx;
    u1 = vy + fy;
    u2 = vz + fz;
    if (MM) {
        adr = (double)fast_sqrt(fmaf(m.nw[0] * fx, fx, fmaf(m.nw[1] * fy, fy, m.nw[2] * fz * fz)));
        av = (double)fast_sqrt(fmaf(m.nw[0] * vx, vx, fmaf(m.nw[1] * vy, vy, m.nw[2] * vz * vz)));
    } else {
        adr = (double)fast_sqrt(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
        av = (double)fast_sqrt(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
    }
    d2 = D64 * D64;
}

// force_point for the forces whose stencils are carried in z (active and
// double: S and D; inverse-consistent: P): the same loaded values and the
// same arithmetic, with cs (S) and cd (D, or P) holding the lane's column
// from the previous row step when `carry`.
template <int V, class St, bool MM>
__device__ __forceinline__ void force_point_carry(const Geo &q, float alpha2, const Bufs &b, int x, const RowOffsets &ro,
                                                  unsigned nbytes, const Metric &m, bool carry, ZCarry &cs,
                                                  ZCarry &cd, float &u0, float &u1, float &u2, double &adr,
                                                  double &av, double &d2)
{
    static_assert(V == kActive || V == kDouble || V == kInverseConsistent, "carried stencils");
    constexpr unsigned ES = St::kBytes;
    LaneOffsets lo;
    lo.c = ES * (unsigned)x;
    lo.xm = ES * (unsigned)max(x - 1, 0);
    lo.xp = ES * (unsigned)min(x + 1, q.nx - 1);
    const float vx = St::load(b.v, lo.c, ro.c), vy = St::load(b.v, lo.c, ro.c + nbytes),
                vz = St::load(b.v, lo.c, ro.c + 2u * nbytes);
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    double D64;  // from the pre-warp kernel
    if constexpr (V == kInverseConsistent) {
        D64 = (double)St::load(b.Dd, lo.c, ro.c);
        constexpr unsigned K4 = 4u / ES;  // P is FP32 in every format
        const LaneOffsets l4{K4 * lo.c, K4 * lo.xm, K4 * lo.xp};
        const RowOffsets r4{K4 * ro.c, K4 * ro.ym, K4 * ro.yp, K4 * ro.zm, K4 * ro.zp};
        float gx, gy, gz;
        cdiff_carry<StF32, MM>(b.P, l4, r4, m, carry, cd, gx, gy, gz);
        dterm((float)D64, gx, gy, gz, alpha2, fx, fy, fz);  // Eq 6
    } else {
        float sx, sy, sz, dx, dy, dz, bx, by, bz;
        cdiff_carry<St, MM>(b.S, lo, ro, m, carry, cs, sx, sy, sz);
        cdiff_carry<St, MM>(b.Dd, lo, ro, m, carry, cd, dx, dy, dz);
        D64 = (double)cd.c;
        const float D = (float)D64;
        if (V == kDouble) dterm(D, sx, sy, sz, alpha2, fx, fy, fz);  // Eq 1
        dterm(D, dx + sx, dy + sy, dz + sz, alpha2, bx, by, bz);    // Eq 3: grad Im = grad (Im - S) + grad S
        fx += bx;
        fy += by;
        fz += bz;
    }
    if (MM) {
        fx *= m.os[0];
        fy *= m.os[1];
        fz *= m.os[2];
    }
    u0 = vx + fx;
    u1 = vy + fy;
    u2 = vz + fz;
    if (MM) {
        adr = (double)fast_sqrt(fmaf(m.nw[0] * fx, fx, fmaf(m.nw[1] * fy, fy, m.nw[2] * fz * fz)));
        av = (double)fast_sqrt(fmaf(m.nw[0] * vx, vx, fmaf(m.nw[1] * vy, vy, m.nw[2] * vz * vz)));
    } else {
        adr = (double)fast_sqrt(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
        av = (double)fast_sqrt(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
    }
    d2 = D64 * D64;
}

// Rows in flight per workgroup and the LDS row buffer of a TX-wide tile.
template <int TX>
struct ForceTile {
    static constexpr int LANES = TX < 256 ? TX : 256;  // threads per row
    static constexpr int W = 256 / LANES;               // rows in flight
    using Rows = float[3][W][TX + 2 * kMaxRadius];
};

// The rows of registration `reg` that its logical workgroup `lid` owns.
// RC >= 0: the smoothing radius is RC, known at compile time (taps from the
// kernel arguments, LDS reads issued together); RC < 0: taps.radius, taps
// from LDS.  St: storage format of every volume the kernel reads and writes.
template <int V, int TX, int RC, class St, bool MM>
__device__ __forceinline__ void force_rows(const ForceArgs &a, const GaussTaps &taps, int reg, int lid,
                                           typename ForceTile<TX>::Rows &ul, const float *wl)
{
    constexpr int LANES = ForceTile<TX>::LANES;
    constexpr int W = ForceTile<TX>::W;
    const int tid = threadIdx.x;
    const int lane = tid % LANES, wrow = tid / LANES;
    const Geo &q = a.geo[reg];
    const int x0 = (lid % q.gxt) * TX;
    const int rb = lid / q.gxt;
    const int yb = rb % q.gy, zb = rb / q.gy;  // y group (fastest across workgroups), z chunk
    const int R = RC >= 0 ? RC : taps.radius;
    const int rows = q.ny * q.nz;
    const unsigned N = (unsigned)q.nx * (unsigned)rows;
    constexpr unsigned ES = St::kBytes;
    const unsigned nbytes = ES * N;
    const float alpha2 = a.alpha2[reg];
    Bufs b;
    b.S = make_rsrc(a.S[reg], nbytes);
    b.M = make_rsrc(a.M[reg], nbytes);
    b.v = make_rsrc(a.v[reg], 3u * nbytes);
    b.Dd = make_rsrc(a.Dd[reg], nbytes);
    b.P = make_rsrc(a.P[reg], 4u * N);  // FP32 in every format
    b.out = make_rsrc(a.out[reg], 3u * nbytes);
    double s1 = 0.0, s2 = 0.0, sse = 0.0;
    // The first TX / LANES points of a lane in each row step (all of them
    // unless a row spans several tiles, whose inner halos add up to 2R
    // points) carry their columns' values in z to the next row step: with
    // FP32 storage, for the forces that read two stencils (active, double)
    // or the FP32 sum P (inverse-consistent).  Measured at 512x512x160, the
    // carry took active and double from 314 to 296 us and IC from 279 to
    // 273 us; it left passive unchanged, and for 16-bit storage its registers
    // cost occupancy (passive F16 276 -> 290 us, IC F16 188 -> 203 us).
    constexpr bool CARRY = ES == 4 && (V == kActive || V == kDouble || V == kInverseConsistent);
    constexpr int SLOTS = TX / LANES;
    ZCarry cs[SLOTS], cd[SLOTS];

    for (int it = 0; it < q.rows_per_block; ++it) {
        // row (y, z): the workgroup's row steps walk z, so a row's z +- 1
        // stencil rows and the rows its gathers reach are those of its own
        // neighbouring steps; the same for every lane of a wavefront
        const int y = __builtin_amdgcn_readfirstlane(yb * W + wrow);
        const int z = __builtin_amdgcn_readfirstlane(zb * q.rows_per_block + it);
        const bool row_ok = y < q.ny && z < q.nz;
        const int r = y + q.ny * z;
        if (row_ok) {
            const unsigned rowb = ES * (unsigned)q.nx;  // bytes per row
            RowOffsets ro;
            ro.c = rowb * (unsigned)r;
            ro.ym = rowb * (unsigned)(max(y - 1, 0) + q.ny * z);
            ro.yp = rowb * (unsigned)(min(y + 1, q.ny - 1) + q.ny * z);
            ro.zm = rowb * (unsigned)(y + q.ny * max(z - 1, 0));
            ro.zp = rowb * (unsigned)(y + q.ny * min(z + 1, q.nz - 1));
            // Evaluate only the points of the tile and its halo that lie in
            // the row: a halo slot beyond a row end holds the end voxel's u
            // (clamped index), so the end lanes copy theirs there instead.
            const int p_lo = max(R - x0, 0), p_hi = min(TX + 2 * R, q.nx - x0 + R);
            auto emit = [&](int p, int xx, float u0, float u1, float u2, double adr, double av, double d2) {
                ul[0][wrow][p] = u0;
                ul[1][wrow][p] = u1;
                ul[2][wrow][p] = u2;
                if (xx == 0)
                    for (int q = 0; q < p; ++q) {
                        ul[0][wrow][q] = u0;
                        ul[1][wrow][q] = u1;
                        ul[2][wrow][q] = u2;
                    }
                // slots past the row end up to the last one the x pass reads:
                // min(TX, nx - x0) - 1 + 2R = min(p + R, TX + 2R - 1)
                if (xx == q.nx - 1)
                    for (int q = p + 1; q <= min(p + R, TX + 2 * R - 1); ++q) {
                        ul[0][wrow][q] = u0;
                        ul[1][wrow][q] = u1;
                        ul[2][wrow][q] = u2;
                    }
                if (p >= R && p < TX + R) {  // a tile voxel: counted once
                    s1 += adr;
                    s2 += av;
                    sse += d2;
                }
            };
            if constexpr (CARRY) {
#pragma unroll
                for (int j = 0; j < SLOTS; ++j) {
                    const int p = p_lo + lane + j * LANES;
                    if (p >= p_hi) break;
                    const int xx = x0 - R + p;  // in [0, nx)
                    float u0, u1, u2;
                    double adr, av, d2;
                    force_point_carry<V, St, MM>(q, alpha2, b, xx, ro, nbytes, a.metric, it > 0, cs[j], cd[j], u0, u1,
                                                 u2, adr, av, d2);
                    emit(p, xx, u0, u1, u2, adr, av, d2);
                }
                for (int p = p_lo + lane + SLOTS * LANES; p < p_hi; p += LANES) {  // inner-halo points
                    const int xx = x0 - R + p;
                    float u0, u1, u2;
                    double adr, av, d2;
                    ZCarry ns, nd;
                    force_point_carry<V, St, MM>(q, alpha2, b, xx, ro, nbytes, a.metric, false, ns, nd, u0, u1, u2,
                                                 adr, av, d2);
                    emit(p, xx, u0, u1, u2, adr, av, d2);
                }
            } else {
                for (int p = p_lo + lane; p < p_hi; p += LANES) {
                    const int xx = x0 - R + p;  // in [0, nx)
                    float u0, u1, u2;
                    double adr, av, d2;
                    force_point<V, St, MM>(q, alpha2, b, xx, y, z, ro, nbytes, a.metric, u0, u1, u2, adr, av, d2);
                    emit(p, xx, u0, u1, u2, adr, av, d2);
                }
            }
        }
        __syncthreads();
        const unsigned rowoff = ES * (unsigned)q.nx * (unsigned)r;
#pragma unroll
        for (int xl = lane; xl < TX; xl += LANES) {
            const int x = x0 + xl;
            if (!row_ok || x >= q.nx) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float s = 0.0f;
                if constexpr (RC >= 0) {
                    float u[2 * RC + 1];
#pragma unroll
                    for (int j = 0; j <= 2 * RC; ++j) u[j] = ul[c][wrow][xl + j];
#pragma unroll
                    for (int j = 0; j <= 2 * RC; ++j) s = fmaf(taps.w[j], u[j], s);
                } else {
                    for (int j = 0; j <= 2 * R; ++j) s = fmaf(wl[j], ul[c][wrow][xl + j], s);
                }
                St::store(b.out, s, ES * (unsigned)x, rowoff + (unsigned)c * nbytes);
            }
        }
        __syncthreads();
    }

    // ---- sums: fixed-order workgroup reduction into this workgroup's slots ----
    block_sum3(s1, s2, sse, tid);
    if (tid == 0) {
        const int nb = q.blocks;
        double *p = a.partials[reg];
        p[lid] = s1;
        p[nb + lid] = s2;
        p[2 * nb + lid] = sse;
    }
}

// One workgroup of a force launch.  Logical workgroup ids (XCD-contiguous)
// map to (registration, workgroup) by batch_slot; V = kMixedVariants takes each
// registration's variant from the arguments (a uniform branch per workgroup).
template <int V, int TX, int RC, class St, bool MM>
__global__ __launch_bounds__(256) void k_force_x(ForceArgs a, GaussTaps taps)
{
    __shared__ typename ForceTile<TX>::Rows ul;
    __shared__ float wl[2 * kMaxRadius + 1];  // taps, read as LDS broadcasts
    int reg, lid;  // wave-uniform
    batch_slot(xcd_logical_id(blockIdx.x, gridDim.x), a, reg, lid);
    if (a.stop_at[reg] && *a.stop_at[reg] < a.n) return;
    if (threadIdx.x <= 2 * kMaxRadius) wl[threadIdx.x] = taps.w[threadIdx.x];  // ordered before use by the row barrier
    if constexpr (V != kMixedVariants) {
        force_rows<V, TX, RC, St, MM>(a, taps, reg, lid, ul, wl);
    } else {
        switch (a.variant[reg]) {
        case kPassive: force_rows<kPassive, TX, RC, St, MM>(a, taps, reg, lid, ul, wl); break;
        case kEvolved: force_rows<kEvolved, TX, RC, St, MM>(a, taps, reg, lid, ul, wl); break;
        case kActive: force_rows<kActive, TX, RC, St, MM>(a, taps, reg, lid, ul, wl); break;
        case kDouble: force_rows<kDouble, TX, RC, St, MM>(a, taps, reg, lid, ul, wl); break;
        default: force_rows<kInverseConsistent, TX, RC, St, MM>(a, taps, reg, lid, ul, wl); break;
        }
    }
}


// Workgroup r reduces the sums of registration r.
__global__ __launch_bounds__(256) void k_finalize(SumsReduce red, int n)
{
    const int r = blockIdx.x;
    reduce_sums(red.partials[r], red.nb[r], red.hist[r], n, red.st[r], red.eps[r], red.inv_n[r], threadIdx.x);
}

__global__ void k_level_reset(LevelState *st)
{
    if (threadIdx.x == 0) {
        st->stop_at = kNeverStopped;
        st->iters_run = 0;
    }
}

struct ForceGrid {
    int tx, gxt, gy, rows_per_block;
    int64_t blocks;
};

// Workgroups per launch to aim for: a quarter of the row steps, within
// [256, 8192].  Measured at 256x256x100 (and its pyramid): 25,600 row steps
// run best as 6,400 workgroups of 4 steps (10% faster than one step each).
// Since a lane carries its z-stencil values from step to step, the smaller
// levels gain from longer walks too: in the six-setting batch the 64x64x25
// force launch (400 row steps per registration) went from 13.2-13.8 to
// 11.9-12.1 us with 2 steps per workgroup, and the 128x128x50 one (3,200)
// from 42.5 to 39.5 us with 4 steps (as 800 workgroups per registration,
// in the interleaved order of batch_slot).  The bound also caps the number
// of sum slots.
int64_t target_force_blocks(int64_t steps)
{
    const int64_t t = steps / 4;
    return t < 256 ? 256 : (t > 8192 ? 8192 : t);
}

ForceGrid force_grid(Dims d)
{
    ForceGrid g;
    // the narrowest tile spanning the row (no interior halo), up to 512
    g.tx = d.nx <= 64 ? 64 : (d.nx <= 128 ? 128 : (d.nx <= 256 ? 256 : 512));
    const int w = g.tx < 256 ? 256 / g.tx : 1;
    g.gxt = ceil_div(d.nx, g.tx);
    g.gy = ceil_div(d.ny, w);
    const int64_t steps = (int64_t)g.gy * d.nz;  // row steps of the whole volume
    const int64_t target = target_force_blocks(steps * g.gxt);
    const int64_t per_tile = (target + g.gxt - 1) / g.gxt;
    // planes per workgroup so that the workgroups of one x tile number about per_tile
    g.rows_per_block = (int)(((int64_t)d.nz * g.gy + per_tile - 1) / per_tile);
    if (g.rows_per_block < 1) g.rows_per_block = 1;
    if (g.rows_per_block > d.nz) g.rows_per_block = d.nz;
    g.blocks = (int64_t)g.gxt * g.gy * ceil_div(d.nz, g.rows_per_block);
    return g;
}

template <int V, int RC, class St, bool MM = false>
void launch_force_vr(Ctx &c, const Ev &ev, const ForceGrid &g, const ForceArgs &a, const GaussTaps &taps)
{
    const dim3 grid((unsigned)g.blocks), block(256);
    if (g.tx == 64) go(c, ev, (k_force_x<V, 64, RC, St, MM>), grid, block, a, taps);
    else if (g.tx == 128) go(c, ev, (k_force_x<V, 128, RC, St, MM>), grid, block, a, taps);
    else if (g.tx == 256) go(c, ev, (k_force_x<V, 256, RC, St, MM>), grid, block, a, taps);
    else go(c, ev, (k_force_x<V, 512, RC, St, MM>), grid, block, a, taps);
}

// Radii with their own kernels: 0 (the force alone, FP32 only), and
// ceil(3 sigma) for sigma = 1 and 1.5 voxels; others take the runtime-radius
// kernel, and so does every force in physical units (mm).
template <int V, class St>
void launch_force_vs(Ctx &c, const Ev &ev, const ForceGrid &g, const ForceArgs &a, const GaussTaps &taps, bool mm)
{
    if (mm) {
        launch_force_vr<V, -1, St, true>(c, ev, g, a, taps);
        return;
    }
    switch (taps.radius) {
    case 0:
        if constexpr (St::kBytes == 4) launch_force_vr<V, 0, St>(c, ev, g, a, taps);
        else launch_force_vr<V, -1, St>(c, ev, g, a, taps);
        break;
    case 3: launch_force_vr<V, 3, St>(c, ev, g, a, taps); break;
    case 5: launch_force_vr<V, 5, St>(c, ev, g, a, taps); break;
    default: launch_force_vr<V, -1, St>(c, ev, g, a, taps); break;
    }
}

template <int V>
void launch_force_v(Ctx &c, const Ev &ev, const ForceGrid &g, const ForceArgs &a, const GaussTaps &taps, int storage,
                    bool mm)
{
    if (storage == kStoreF16) launch_force_vs<V, StF16>(c, ev, g, a, taps, mm);
    else if (storage == kStoreBF16) launch_force_vs<V, StBF16>(c, ev, g, a, taps, mm);
    else launch_force_vs<V, StF32>(c, ev, g, a, taps, mm);
}

// One launch for the registrations `sel[0 .. k-1]` of f, which share a tile
// width.
hipError_t launch_force_group(Ctx &c, const ForceLaunch &f, const ForceGrid *g, const int *sel, int k)
{
    ForceArgs a;
    memset(&a, 0, sizeof a);
    int variant = f.variant == kMixedVariants ? f.variants[sel[0]] : f.variant;
    int64_t total = 0;
    for (int q = 0; q < k; ++q) {
        const int r = sel[q];
        a.S[q] = f.S[r];
        a.M[q] = f.M[r];
        a.v[q] = f.v[r];
        a.Dd[q] = f.D[r];
        a.P[q] = f.P[r];
        a.out[q] = f.out[r];
        a.partials[q] = f.partials[r];
        a.stop_at[q] = f.stop_at[r];
        a.alpha2[q] = f.alpha2[r];
        a.variant[q] = f.variant == kMixedVariants ? f.variants[r] : f.variant;
        if (a.variant[q] != variant) variant = kMixedVariants;
        a.geo[q] = Geo{f.d[r].nx, f.d[r].ny, f.d[r].nz, g[r].gxt, g[r].gy, g[r].rows_per_block, (int)g[r].blocks};
        a.first[q] = (int)total;
        total += g[r].blocks;
    }
    a.first[k] = (int)total;
    batch_chunks(a.first, k, a.chunk);
    a.count = k;
    a.n = f.n;
    const bool mm = f.metric != nullptr;
    if (mm) a.metric = *f.metric;
    ForceGrid gl = g[sel[0]];
    gl.blocks = total;  // the launch: every registration's workgroups
    return timed(c, K_FORCE, [&](const Ev &ev) {
        switch (variant) {
        case kPassive: launch_force_v<kPassive>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        case kEvolved: launch_force_v<kEvolved>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        case kActive: launch_force_v<kActive>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        case kDouble: launch_force_v<kDouble>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        case kInverseConsistent: launch_force_v<kInverseConsistent>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        default: launch_force_v<kMixedVariants>(c, ev, gl, a, *f.taps, f.storage, mm); break;
        }
    });
}

}  // namespace

int64_t force_blocks(Dims d) { return force_grid(d).blocks; }

// Registrations whose rows take the same tile width share a launch; each
// keeps the workgroup layout it has alone.
hipError_t launch_force(Ctx &c, const ForceLaunch &f)
{
    if (f.count < 1 || f.count > kMaxBatch) return hipErrorInvalidValue;
    ForceGrid g[kMaxBatch];
    for (int r = 0; r < f.count; ++r) g[r] = force_grid(f.d[r]);
    bool done[kMaxBatch] = {};
    for (int r = 0; r < f.count; ++r) {
        if (done[r]) continue;
        int sel[kMaxBatch], k = 0;
        for (int q = r; q < f.count; ++q)
            if (!done[q] && g[q].tx == g[r].tx) {
                sel[k++] = q;
                done[q] = true;
            }
        const hipError_t e = launch_force_group(c, f, g, sel, k);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_finalize(Ctx &c, const SumsReduce &red, int n)
{
    if (red.count < 1 || red.count > kMaxBatch) return hipErrorInvalidValue;
    return timed(c, K_FINALIZE,
                 [&](const Ev &ev) { go(c, ev, k_finalize, dim3((unsigned)red.count), dim3(256), red, n); });
}

hipError_t launch_level_reset(Ctx &c, LevelState *st)
{
    return timed(c, K_LEVEL_RESET, [&](const Ev &ev) { go(c, ev, k_level_reset, dim3(1), dim3(64), st); });
}

}  // namespace dir
