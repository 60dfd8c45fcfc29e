// Device helpers shared by the gfx950 kernels of libdemons, and the launch
// helpers their host-side launchers use.  Internal header.
//
// Layout: float32 volumes [nz][ny][nx], x fastest; fields are three such
// planes (x, y, z components) in voxel units.  Kernels map a 64-wide
// wavefront along x so a row is read and written with coalesced accesses.
#pragma once

#include <math.h>

#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include "dir_internal.h"

namespace dir {
namespace dev {

constexpr float kDenomFloor = 1e-9f;  // force is zero at or below this denominator

__device__ __forceinline__ int clampi(int i, int n) { return min(max(i, 0), n - 1); }

// Cell and weights along one axis for trilinear interpolation with the
// coordinate clamped to [0, n-1] (Sec 2.5 interpolation kernel; explicit
// weights, no hardware filtering).  The sample lies at i0 + t between i0 and
// i1 = min(i0 + 1, n - 1); w0 = 1 - t is the weight of i0.  A clamped sample
// sits exactly on i0 with t = 0, so border values are reproduced exactly.
//
// The sample position is x - v with x an integer grid index.  Forming x - v
// in FP32 would round it to the ulp of x (7.6e-6 voxel at x = 100); instead v
// is split into floor(v) (exact) and the fraction r = v - floor(v), formed in
// FP64, where it is exact for every FP32 v (in FP32 it is not: for -1/2 < v
// < 0, r = 1 + v lies in a coarser binade than v).  The cell index is then
// integer arithmetic and the weight w0 = r is exact; the FP32 t = 1 - r is
// rounded once.  v is first limited to +-2^20 (NaN becomes -2^20), which
// keeps every index inside the grid.
struct Axis {
    int i0, i1;
    float t;
    double w0;
};

__device__ __forceinline__ Axis axis_disp(int x, float v, int n)
{
    v = fminf(fmaxf(v, -1048576.0f), 1048576.0f);
    const float fv = floorf(v);
    const double r = (double)v - (double)fv;  // exact
    int i = x - (int)fv;  // p = x - v = i - r
    Axis a;
    a.t = 0.0f;
    a.w0 = 1.0;
    if (r > 0.0) {
        i -= 1;
        a.t = (float)(1.0 - r);
        a.w0 = r;
    }
    if (i < 0 || i > n - 1) {  // outside: clamp onto the border sample
        i = i < 0 ? 0 : n - 1;
        a.t = 0.0f;
        a.w0 = 1.0;
    } else if (i == n - 1) {   // p in (n-1, n) would need the next cell: clamp
        a.t = 0.0f;
        a.w0 = 1.0;
    }
    a.i0 = i;
    a.i1 = min(i + 1, n - 1);
    return a;
}

// Same for an FP32 coordinate p that is exact as given (prolongation).
__device__ __forceinline__ Axis axis_coord(float p, int n)
{
    p = fminf(fmaxf(p, 0.0f), (float)(n - 1));
    Axis a;
    a.i0 = min((int)p, n - 1);  // p >= 0, so truncation is floor
    a.i1 = min(a.i0 + 1, n - 1);
    a.t = p - (float)a.i0;      // exact: p carries few fraction bits
    a.w0 = 1.0 - (double)a.t;
    return a;
}

struct Cell {
    int o000, o100, o010, o110, o001, o101, o011, o111;
    float tx, ty, tz;     // FP32 fractional positions
    double wx, wy, wz;    // exact weights of the lower index
};

__device__ __forceinline__ Cell make_cell_axes(const Axis &ax, const Axis &ay, const Axis &az, int nx, int ny)
{
    Cell c;
    const int r00 = nx * (ay.i0 + ny * az.i0), r10 = nx * (ay.i1 + ny * az.i0);
    const int r01 = nx * (ay.i0 + ny * az.i1), r11 = nx * (ay.i1 + ny * az.i1);
    c.o000 = r00 + ax.i0;
    c.o100 = r00 + ax.i1;
    c.o010 = r10 + ax.i0;
    c.o110 = r10 + ax.i1;
    c.o001 = r01 + ax.i0;
    c.o101 = r01 + ax.i1;
    c.o011 = r11 + ax.i0;
    c.o111 = r11 + ax.i1;
    c.tx = ax.t;
    c.ty = ay.t;
    c.tz = az.t;
    c.wx = ax.w0;
    c.wy = ay.w0;
    c.wz = az.w0;
    return c;
}

// Cell of the position (x, y, z) - (vx, vy, vz).
__device__ __forceinline__ Cell make_cell_disp(int x, int y, int z, float vx, float vy, float vz, int nx, int ny,
                                               int nz)
{
    return make_cell_axes(axis_disp(x, vx, nx), axis_disp(y, vy, ny), axis_disp(z, vz, nz), nx, ny);
}

__device__ __forceinline__ Cell make_cell(float px, float py, float pz, int nx, int ny, int nz)
{
    return make_cell_axes(axis_coord(px, nx), axis_coord(py, ny), axis_coord(pz, nz), nx, ny);
}

__device__ __forceinline__ float lerp1(float a, float b, float t) { return fmaf(t, b - a, a); }

// FP32 trilinear sample.
__device__ __forceinline__ float sample(const float *__restrict__ I, const Cell &c)
{
    const float c00 = lerp1(I[c.o000], I[c.o100], c.tx);
    const float c10 = lerp1(I[c.o010], I[c.o110], c.tx);
    const float c01 = lerp1(I[c.o001], I[c.o101], c.tx);
    const float c11 = lerp1(I[c.o011], I[c.o111], c.tx);
    return lerp1(lerp1(c00, c10, c.ty), lerp1(c01, c11, c.ty), c.tz);
}

// FP64 trilinear sample with exact weights.  Used where the sample enters an
// intensity difference: D = Im - S cancels to a few HU on a -1000 HU
// background, and the force's relative error is D's relative error.  FP64 FMA
// issues at the same rate as unpacked FP32 on gfx950.
__device__ __forceinline__ double sample64(const float *__restrict__ I, const Cell &c)
{
    const double ax = c.wx, bx = 1.0 - ax, ay = c.wy, by = 1.0 - ay, az = c.wz, bz = 1.0 - az;
    const double c00 = ax * (double)I[c.o000] + bx * (double)I[c.o100];
    const double c10 = ax * (double)I[c.o010] + bx * (double)I[c.o110];
    const double c01 = ax * (double)I[c.o001] + bx * (double)I[c.o101];
    const double c11 = ax * (double)I[c.o011] + bx * (double)I[c.o111];
    return az * (ay * c00 + by * c10) + bz * (ay * c01 + by * c11);
}

// The dispatcher hands workgroup b to XCD b % 8, and each XCD has its own L2.
// Renumbering so that XCD k runs one contiguous range of logical ids keeps
// spatial neighbours (which share stencil halos and gather rows) in the same
// L2.  A bijection on [0, nb).
constexpr int kXCDs = 8;

__device__ __forceinline__ int xcd_logical_id(int b, int nb)
{
    const int per = nb / kXCDs, rem = nb % kXCDs;
    const int x = b % kXCDs, i = b / kXCDs;
    return x * per + min(x, rem) + i;
}

// Logical workgroup g of a launch over `count` registrations to (reg, lid)
// (A: the launch's arguments, with first[] and chunk[]).  Registration r owns
// b_r = first[r + 1] - first[r] workgroups, cut into kXCDs consecutive chunks
// (chunk k: lids k b_r / kXCDs .. (k + 1) b_r / kXCDs - 1), and the logical
// order runs chunk 0 of every registration, then chunk 1 of every
// registration, and so on (chunk[k]: where chunk k starts, from the host).
// Each XCD's contiguous range of logical ids then holds about an eighth of
// every registration, so registrations of unequal cost (variants) spread
// evenly over the XCDs, while a registration's neighbouring workgroups stay
// together.  chunk[0] < 0 asks for registration-major order instead
// (registration r from first[r]), which keeps more of a small registration
// on one XCD.  Which rows a (reg, lid) covers, and so every result, does not
// depend on the order.  Wave-uniform scalar work on values loaded once.
template <class A>
__device__ __forceinline__ void batch_slot(int g, const A &a, int &reg, int &lid)
{
    reg = 0;
    lid = g;
    if (a.count == 1) return;
    if (a.chunk[0] < 0) {  // registration-major order: registration r at first[r]
        int base = 0;
#pragma unroll
        for (int r = 1; r < kMaxBatch; ++r)
            if (r < a.count && g >= a.first[r]) {
                reg = r;
                base = a.first[r];
            }
        lid = g - base;
        return;
    }
    int b[kMaxBatch];
#pragma unroll
    for (int r = 0; r < kMaxBatch; ++r) b[r] = r < a.count ? a.first[r + 1] - a.first[r] : 0;
    int k = 0, base = 0;
#pragma unroll
    for (int j = 1; j < kXCDs; ++j)
        if (g >= a.chunk[j]) {
            k = j;
            base = a.chunk[j];
        }
    unsigned off = (unsigned)(g - base);
    bool found = false;
#pragma unroll
    for (int r = 0; r < kMaxBatch; ++r) {
        const unsigned lo = ((unsigned)k * (unsigned)b[r]) / kXCDs;
        const unsigned n = ((unsigned)(k + 1) * (unsigned)b[r]) / kXCDs - lo;
        if (!found) {
            if (off < n) {
                reg = r;
                lid = (int)(lo + off);
                found = true;
            } else {
                off -= n;
            }
        }
    }
}

// Raw buffer access: the resource (base, size in bytes) lives in scalar
// registers, a per-lane byte offset in one VGPR and a wave-uniform byte offset
// in an SGPR, so addressing costs no 64-bit vector arithmetic.  Offsets past
// the size read 0 and drop writes (never used on purpose: every offset here
// is in range by construction).
constexpr int kBufferDword3 = 0x00020000;  // 32-bit data format (gfx9-family buffer resource word 3)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferDword3);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

// Storage formats of images and fields.  Arithmetic is FP32 throughout: a
// 16-bit value converts to float exactly on load and a float is rounded to
// nearest-even on store.  kBytes is the element size that every byte offset
// of a volume of that format is scaled by.
struct StF32 {
    static constexpr unsigned kBytes = 4;
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
    {
        return bload(r, voff, soff);
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
    {
        bstore(r, v, voff, soff);
    }
};

// The 16-bit formats also convert to and from their bit patterns (from_bits,
// to_bits), which the smoothing kernel uses to move two values per 4-byte
// access; load and store are those conversions around a 2-byte access.
struct StF16 {  // IEEE binary16
    static constexpr unsigned kBytes = 2;
    static __device__ __forceinline__ float from_bits(unsigned u) { return __half2float(__ushort_as_half((unsigned short)u)); }
    static __device__ __forceinline__ unsigned to_bits(float v) { return __half_as_ushort(__float2half_rn(v)); }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
    {
        return from_bits(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)to_bits(v), r, voff, soff, 0);
    }
};

struct StBF16 {  // bfloat16: the upper half of a binary32
    static constexpr unsigned kBytes = 2;
    static __device__ __forceinline__ float from_bits(unsigned u) { return __uint_as_float((u & 0xffffu) << 16); }
    static __device__ __forceinline__ unsigned to_bits(float v)
    {
        // round to nearest, ties to even, on the 16 bits dropped (finite v)
        unsigned u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return u >> 16;
    }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
    {
        return from_bits(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)to_bits(v), r, voff, soff, 0);
    }
};

// Trilinear cell in byte offsets for buffer access: the lower corner, the
// byte step to the upper neighbour along each axis (0 where the sample was
// clamped onto a single grid point) and the exact weights of the lower
// corner.  Same sample position and weights as make_cell_disp.
struct BCell {
    unsigned o;
    unsigned dx, dy, dz;
    double wx, wy, wz;
};

struct AxisB {
    int i;
    bool step;
    double w0;
};

__device__ __forceinline__ AxisB axis_b(int x, float v, int n)
{
    v = fminf(fmaxf(v, -1048576.0f), 1048576.0f);  // NaN -> -2^20; keeps indices in range
    const float fv = floorf(v);
    const double r = (double)v - (double)fv;         // exact (see axis_disp)
    int i = x - (int)fv;                             // p = x - v = i - r
    AxisB a;
    a.w0 = 1.0;
    if (r > 0.0) {
        i -= 1;
        a.w0 = r;
    }
    a.step = i >= 0 && i <= n - 2;
    if (!a.step) {  // clamped onto the border sample (or the last sample exactly)
        i = min(max(i, 0), n - 1);
        a.w0 = 1.0;
    }
    a.i = i;
    return a;
}

// ES: element size in bytes of the volume the cell addresses.
template <unsigned ES = 4>
__device__ __forceinline__ BCell bcell_disp(int x, int y, int z, float vx, float vy, float vz, int nx, int ny, int nz)
{
    const AxisB ax = axis_b(x, vx, nx), ay = axis_b(y, vy, ny), az = axis_b(z, vz, nz);
    BCell c;
    const unsigned row = ES * (unsigned)nx, plane = row * (unsigned)ny;
    c.o = ES * (unsigned)ax.i + row * (unsigned)ay.i + plane * (unsigned)az.i;
    c.dx = ax.step ? ES : 0u;
    c.dy = ay.step ? row : 0u;
    c.dz = az.step ? plane : 0u;
    c.wx = ax.w0;
    c.wy = ay.w0;
    c.wz = az.w0;
    return c;
}

// The samples at byte offsets o and o + dx (dx 0 or 4) of an FP32 volume from
// one 8-byte load, so that a trilinear gather issues four loads instead of
// eight (the address rate of the gather is what bounds the pre-warp kernel).
// With dx = 0 (an axis clamped onto one grid point) the load ends at o, and
// so never reaches past the volume, except at offset 0, where it reads the
// element after the first; the buffer's range check answers a dword past a
// one-element volume with 0, which is not used.  No branch: a divergent
// path for that one case costs more than the gathers save.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bpair(__amdgpu_buffer_rsrc_t r, unsigned o, unsigned dx, float &lo, float &hi)
{
    const bool back = dx == 0u && o >= 4u;
    const u32x2 p = __builtin_amdgcn_raw_buffer_load_b64(r, back ? o - 4u : o, 0, 0);
    lo = __uint_as_float(back ? p.y : p.x);
    hi = dx ? __uint_as_float(p.y) : lo;
}

// Trilinear FP64 sample through a buffer resource (see sample64) of a volume
// stored in format St.
template <class St = StF32>
__device__ __forceinline__ double bsample64(__amdgpu_buffer_rsrc_t I, const BCell &c)
{
    const double ax = c.wx, bx = 1.0 - ax, ay = c.wy, by = 1.0 - ay, az = c.wz, bz = 1.0 - az;
    const unsigned o = c.o, oy = o + c.dy, oz = o + c.dz, oyz = oz + c.dy;
    if constexpr (St::kBytes == 4) {
        float a0, a1, b0, b1, c0, c1, d0, d1;
        bpair(I, o, c.dx, a0, a1);
        bpair(I, oy, c.dx, b0, b1);
        bpair(I, oz, c.dx, c0, c1);
        bpair(I, oyz, c.dx, d0, d1);
        const double c00 = ax * (double)a0 + bx * (double)a1;
        const double c10 = ax * (double)b0 + bx * (double)b1;
        const double c01 = ax * (double)c0 + bx * (double)c1;
        const double c11 = ax * (double)d0 + bx * (double)d1;
        return az * (ay * c00 + by * c10) + bz * (ay * c01 + by * c11);
    }
    const double c00 = ax * (double)St::load(I, o, 0) + bx * (double)St::load(I, o + c.dx, 0);
    const double c10 = ax * (double)St::load(I, oy, 0) + bx * (double)St::load(I, oy + c.dx, 0);
    const double c01 = ax * (double)St::load(I, oz, 0) + bx * (double)St::load(I, oz + c.dx, 0);
    const double c11 = ax * (double)St::load(I, oyz, 0) + bx * (double)St::load(I, oyz + c.dx, 0);
    return az * (ay * c00 + by * c10) + bz * (ay * c01 + by * c11);
}

// Trilinear cell with FP32 weights, for volumes in a 16-bit storage format.
// Their values are exact in FP32 and their parity bound is the 16-bit
// roundoff (2^-11 or 2^-8), which the FP32 sample's error (about 2^-24 of the
// intensity) leaves far below, so the FP64 sample and its exact-weight split
// are not needed there; the FP32 form costs about a third of the force
// kernel's vector instructions fewer.  Same cell and clamping as axis_b.
struct BCell32 {
    unsigned o;
    unsigned dx, dy, dz;
    float wx, wy, wz;
};

__device__ __forceinline__ void axis_f(int x, float v, int n, int &i, bool &step, float &w0)
{
    v = fminf(fmaxf(v, -1048576.0f), 1048576.0f);  // NaN -> -2^20; keeps indices in range
    const float fv = floorf(v);
    const float r = v - fv;                          // in [0, 1]
    i = x - (int)fv;
    w0 = 1.0f;
    if (r > 0.0f) {
        i -= 1;
        w0 = r;
    }
    step = i >= 0 && i <= n - 2;
    if (!step) {
        i = min(max(i, 0), n - 1);
        w0 = 1.0f;
    }
}

template <unsigned ES>
__device__ __forceinline__ BCell32 bcell32(int x, int y, int z, float vx, float vy, float vz, int nx, int ny, int nz)
{
    int ix, iy, iz;
    bool sx, sy, sz;
    BCell32 c;
    axis_f(x, vx, nx, ix, sx, c.wx);
    axis_f(y, vy, ny, iy, sy, c.wy);
    axis_f(z, vz, nz, iz, sz, c.wz);
    const unsigned row = ES * (unsigned)nx, plane = row * (unsigned)ny;
    c.o = ES * (unsigned)ix + row * (unsigned)iy + plane * (unsigned)iz;
    c.dx = sx ? ES : 0u;
    c.dy = sy ? row : 0u;
    c.dz = sz ? plane : 0u;
    return c;
}

// The 16-bit values at byte offsets o and o + dx (dx 0 or 2) from one 8-byte
// load at the dword boundary at or below o (dword-aligned, unlike a 4-byte
// load at o), so that a trilinear gather issues four loads instead of eight.
__device__ __forceinline__ void bpair16(__amdgpu_buffer_rsrc_t r, unsigned o, unsigned dx, unsigned &lo, unsigned &hi)
{
    const u32x2 p = __builtin_amdgcn_raw_buffer_load_b64(r, o & ~3u, 0, 0);
    const unsigned long long q = ((unsigned long long)p.y << 32) | p.x;
    const unsigned w = (unsigned)(q >> ((o & 2u) * 8u));  // element o in the low half, o + 2 in the high
    lo = w;
    hi = dx ? w >> 16 : w;
}

// FP32 trilinear sample of a volume in format St (16 bits) at a BCell32
// (lower-corner weight w0: w0 * a + (1 - w0) * b per axis).  Paired: each x
// pair comes from one bpair16 load (the volume's buffer must reach kPad16
// bytes past its end).  Measured at 512x512x160 (F16): the pre-warp kernels
// gain from the pairs (the inverse-consistent registration 30.6 -> 30.0 ms),
// the force kernel loses (passive 274 -> 288 us), so only the pre-warps
// take them.
template <class St, bool Paired>
__device__ __forceinline__ float bsample32(__amdgpu_buffer_rsrc_t I, const BCell32 &c)
{
    static_assert(St::kBytes == 2, "16-bit storage formats");
    const unsigned o = c.o, oy = o + c.dy, oz = o + c.dz, oyz = oz + c.dy;
    float a0, a1, b0, b1, e0, e1, f0, f1;
    if constexpr (Paired) {
        unsigned u[8];
        bpair16(I, o, c.dx, u[0], u[1]);
        bpair16(I, oy, c.dx, u[2], u[3]);
        bpair16(I, oz, c.dx, u[4], u[5]);
        bpair16(I, oyz, c.dx, u[6], u[7]);
        a0 = St::from_bits(u[0]), a1 = St::from_bits(u[1]), b0 = St::from_bits(u[2]), b1 = St::from_bits(u[3]);
        e0 = St::from_bits(u[4]), e1 = St::from_bits(u[5]), f0 = St::from_bits(u[6]), f1 = St::from_bits(u[7]);
    } else {
        a0 = St::load(I, o, 0), a1 = St::load(I, o + c.dx, 0), b0 = St::load(I, oy, 0), b1 = St::load(I, oy + c.dx, 0);
        e0 = St::load(I, oz, 0), e1 = St::load(I, oz + c.dx, 0), f0 = St::load(I, oyz, 0);
        f1 = St::load(I, oyz + c.dx, 0);
    }
    const float c00 = fmaf(c.wx, a0 - a1, a1);
    const float c10 = fmaf(c.wx, b0 - b1, b1);
    const float c01 = fmaf(c.wx, e0 - e1, e1);
    const float c11 = fmaf(c.wx, f0 - f1, f1);
    const float d0 = fmaf(c.wy, c00 - c10, c10), d1 = fmaf(c.wy, c01 - c11, c11);
    return fmaf(c.wz, d0 - d1, d1);
}

// FP32 trilinear samples of three planes `plane` bytes apart (a field's
// components) at one cell: the corner offsets are formed once and the plane
// goes to the scalar offset.  Lower-corner weight w0: w0 * a + (1 - w0) * b.
template <class St = StF32>
__device__ __forceinline__ void bsample3(__amdgpu_buffer_rsrc_t I, const BCell &c, unsigned plane, float &s0,
                                         float &s1, float &s2)
{
    const unsigned o = c.o, oy = o + c.dy, oz = o + c.dz, oyz = oz + c.dy;
    const float wx = (float)c.wx, wy = (float)c.wy, wz = (float)c.wz;
    float r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const unsigned so = (unsigned)k * plane;
        const float b00 = St::load(I, o + c.dx, so), b10 = St::load(I, oy + c.dx, so);
        const float b01 = St::load(I, oz + c.dx, so), b11 = St::load(I, oyz + c.dx, so);
        const float c00 = fmaf(wx, St::load(I, o, so) - b00, b00);
        const float c10 = fmaf(wx, St::load(I, oy, so) - b10, b10);
        const float c01 = fmaf(wx, St::load(I, oz, so) - b01, b01);
        const float c11 = fmaf(wx, St::load(I, oyz, so) - b11, b11);
        const float d0 = fmaf(wy, c00 - c10, c10), d1 = fmaf(wy, c01 - c11, c11);
        r[k] = fmaf(wz, d0 - d1, d1);
    }
    s0 = r[0];
    s1 = r[1];
    s2 = r[2];
}

// Decode a flattened workgroup id into (tile x, tile y, z), XCD-contiguous.
struct Tile {
    int x, y, z;
};
__device__ __forceinline__ Tile decode_tile(int gx, int gy)
{
    const int b = xcd_logical_id(blockIdx.x, gridDim.x);
    Tile t;
    t.x = b % gx;
    const int r = b / gx;
    t.y = r % gy;
    t.z = r / gy;
    return t;
}

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

// Sum of three doubles over a 256-thread workgroup in a fixed order (xor
// butterfly within each wavefront, then the four wavefronts in order);
// result valid in thread 0.  `tid` is the flat thread index.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, int tid)
{
    __shared__ double red[3][kBlockX * kBlockY / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
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


// Fixed-order sum of K doubles over a 256-thread workgroup (result in
// thread 0): xor shuffles within each wavefront, then the four wavefront
// sums in order.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], int tid)
{
    __shared__ double red[K][kBlockX * kBlockY / 64];
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][wave] = v[k];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = red[k][0];
            for (int w = 1; w < kBlockX * kBlockY / 64; ++w) v[k] += red[k][w];
        }
}

// Reduction of the force kernel's per-workgroup sums (slots s1[nb], s2[nb],
// sse[nb]) by one 256-thread workgroup: strided partial sums per thread, then
// the fixed-order workgroup sum, so the result is bitwise reproducible.
// Thread 0 writes history entry n of the level (sum|dr|, sum|v|, mean D^2,
// relative norm l = sum|dr| / sum|v|, NaN while sum|v| = 0), the iteration
// count, and applies the stopping rule of Sec 2.4: once n >= 10 and
// l(n-10) - l(n) <= eps the level stops after iteration n.
__device__ __forceinline__ void reduce_sums(const double *__restrict__ partials, int nb, double *hist, int n,
                                            LevelState *st, double eps, double inv_n, int tid)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = tid; k < nb; k += 256) {
        a += partials[k];
        b += partials[nb + k];
        c += partials[2 * nb + k];
    }
    block_sum3(a, b, c, tid);
    if (tid == 0) {
        const double l = b > 0.0 ? a / b : __builtin_nan("");
        double *e = hist + 4 * (int64_t)n;
        e[0] = a;
        e[1] = b;
        e[2] = c * inv_n;
        e[3] = l;
        st->iters_run = n + 1;
        if (eps > 0.0 && n >= 10) {
            const double l10 = hist[4 * (int64_t)(n - 10) + 3];
            if (!isnan(l) && !isnan(l10) && l10 - l <= eps) st->stop_at = n;
        }
    }
}

}  // namespace dev

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// chunk[] of batch_slot for a launch whose registration r owns
// first[r + 1] - first[r] workgroups: the chunk starts of the interleaved
// order when every registration has at least kInterleaveMinBlocks
// workgroups, else registration-major order.  Measured in the six-setting
// batch at 256x256x100: interleaving took the 128x128x50 force launches
// from 47.3 to 45.6 us with 1,600 workgroups per registration (and from
// 42.5 to 39.5 us with 800 of 4 row steps) and the mixed pre-warp from 25.0
// to 21.6 us (3,200), but the 64x64x25 force launch from 13.0 to 14.8 us
// (400 per registration).
constexpr int kInterleaveMinBlocks = 512;

inline void batch_chunks(const int *first, int count, int *chunk)
{
    for (int r = 0; r < count; ++r)
        if (first[r + 1] - first[r] < kInterleaveMinBlocks) {
            chunk[0] = -1;
            return;
        }
    for (int k = 0; k < dev::kXCDs; ++k) {
        unsigned s = 0;
        for (int r = 0; r < count; ++r) s += ((unsigned)k * (unsigned)(first[r + 1] - first[r])) / dev::kXCDs;
        chunk[k] = (int)s;
    }
}

struct Grid2 {
    int gx, gy;
    int64_t blocks;
};

// One 64 x 4 workgroup per (x tile, y tile, z) of a volume.
inline Grid2 plane_grid(Dims d)
{
    Grid2 g;
    g.gx = ceil_div(d.nx, kBlockX);
    g.gy = ceil_div(d.ny, kBlockY);
    g.blocks = (int64_t)g.gx * g.gy * d.nz;
    return g;
}

// Call f(Tag<St>{}) with the storage trait of format code `st` (host side).
template <class T>
struct Tag {
    using type = T;
};
template <class F>
void with_storage(int st, F &&f)
{
    if (st == kStoreF16) f(Tag<dev::StF16>{});
    else if (st == kStoreBF16) f(Tag<dev::StBF16>{});
    else f(Tag<dev::StF32>{});
}

// Start and stop events of one launch; both null when it is not timed.
struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
};

// Enqueue `kernel` on the context's stream with the launch's timing events.
template <typename K, typename... A>
void go(Ctx &c, const Ev &ev, K kernel, dim3 grid, dim3 block, A... args)
{
    hipExtLaunchKernelGGL(kernel, grid, block, 0, c.stream, ev.a, ev.b, 0, args...);
}

// Run `launch(ev)`, which enqueues exactly one kernel through go(); when
// kernel k is timed, ev carries a fresh event pair that the timer collects.
template <typename F>
hipError_t timed(Ctx &c, int k, F &&launch)
{
    Ev ev;
    const bool on = c.timer && c.timer->on(k);
    if (on) {
        hipError_t e = c.timer->pair(&ev.a, &ev.b);
        if (e != hipSuccess) return e;
    }
    launch(ev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (on) c.timer->record(k, ev.a, ev.b);
    return hipSuccess;
}

}  // namespace dir
