/*
 * FP64 CPU oracle for multi-scale demons deformable image registration
 * (Gu et al., "Implementation and evaluation of various demons deformable
 * image registration algorithms on GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the registration computes.  It is called by the tests,
 * by the package smoke check and by the benchmark's CPU-baseline leg, never
 * by the product path, and it shares no code, header or table with the HIP
 * library.  Every step follows the paper in the paper's order; where the
 * paper is silent or garbled the reading taken is stated at the function.
 *
 * Conventions (the same ones the HIP library documents independently):
 *   - volumes are [nz][ny][nx] doubles, x fastest: index x + nx*(y + ny*z);
 *   - a displacement field is three such planes (x, y, z components) in
 *     voxel units, one after the other;
 *   - the field v registers M onto S when M(x - v(x)) = S(x); the paper's
 *     increment dr is added to v (Sec 2.1, Eq 1);
 *   - index and coordinate clamping at the volume border.
 *
 * Reductions are plain serial loops in voxel order so results do not depend
 * on the thread count; element-wise loops may run under OpenMP.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PASSIVE 0
#define ORC_EVOLVED 1
#define ORC_ACTIVE 2
#define ORC_DOUBLE 3
#define ORC_INVERSE_CONSISTENT 4

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENUMERIC (-4)

#define ORC_MAX_LEVELS 8
#define ORC_MAX_RADIUS 16
#define ORC_DENOM_FLOOR 1e-9

static int64_t clampi(int64_t i, int64_t n) { return i < 0 ? 0 : (i > n - 1 ? n - 1 : i); }

static int64_t at(int64_t x, int64_t y, int64_t z, int64_t nx, int64_t ny) { return x + nx * (y + ny * z); }

int orc_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the element-wise loops run on (1 without OpenMP). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Run the element-wise loops on n threads from now on (n >= 1; no effect
 * without OpenMP).  Sums stay serial, so results do not change. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * Trilinear interpolation (Sec 2.5, interpolation kernel).  The paper uses
 * its own full-precision trilinear code rather than hardware filtering.  The
 * paper is silent on samples outside the grid: each coordinate is clamped to
 * [0, n-1] (edge replication).  The cell is i0 = min(floor(p), n-2) with
 * t = p - i0, so the last grid point is reached with t = 1; an axis of
 * length 1 contributes its single value.
 * ------------------------------------------------------------------------ */
static void axis_cell(double p, int64_t n, int64_t *i0, int64_t *i1, double *t)
{
    if (n == 1) { *i0 = 0; *i1 = 0; *t = 0.0; return; }
    if (!(p > 0.0)) p = 0.0;                 /* also maps NaN to 0 */
    if (p > (double)(n - 1)) p = (double)(n - 1);
    int64_t i = (int64_t)floor(p);
    if (i > n - 2) i = n - 2;
    *i0 = i;
    *i1 = i + 1;
    *t = p - (double)i;
}

double orc_trilerp(const double *I, int64_t nx, int64_t ny, int64_t nz, double px, double py, double pz)
{
    int64_t x0, x1, y0, y1, z0, z1;
    double tx, ty, tz;
    axis_cell(px, nx, &x0, &x1, &tx);
    axis_cell(py, ny, &y0, &y1, &ty);
    axis_cell(pz, nz, &z0, &z1, &tz);
    double s = 0.0;
    s += (1 - tx) * (1 - ty) * (1 - tz) * I[at(x0, y0, z0, nx, ny)];
    s += tx * (1 - ty) * (1 - tz) * I[at(x1, y0, z0, nx, ny)];
    s += (1 - tx) * ty * (1 - tz) * I[at(x0, y1, z0, nx, ny)];
    s += tx * ty * (1 - tz) * I[at(x1, y1, z0, nx, ny)];
    s += (1 - tx) * (1 - ty) * tz * I[at(x0, y0, z1, nx, ny)];
    s += tx * (1 - ty) * tz * I[at(x1, y0, z1, nx, ny)];
    s += (1 - tx) * ty * tz * I[at(x0, y1, z1, nx, ny)];
    s += tx * ty * tz * I[at(x1, y1, z1, nx, ny)];
    return s;
}

/* Deformed image (Sec 2.1 and Sec 2.5): out(x) = I(x - sign * v(x)).
 * sign = +1 deforms the moving image by the field; sign = -1 applies the
 * first-order inverse x + v, used for the static image of the
 * inverse-consistent variant (Sec 2.2, text after Eq 6). */
void orc_warp(const double *I, const double *v, int64_t nx, int64_t ny, int64_t nz, double sign, double *out)
{
    const int64_t N = nx * ny * nz;
    const double *vx = v, *vy = v + N, *vz = v + 2 * N;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = at(x, y, z, nx, ny);
                out[i] = orc_trilerp(I, nx, ny, nz, (double)x - sign * vx[i], (double)y - sign * vy[i],
                                     (double)z - sign * vz[i]);
            }
}

/* Image gradient (Sec 2.5, gradient kernel): the separable gradient mask is
 * read as the central difference (I[i+1] - I[i-1]) / 2 per axis in voxel
 * units, neighbour indices clamped.  Output: three planes (d/dx, d/dy, d/dz). */
void orc_gradient(const double *I, int64_t nx, int64_t ny, int64_t nz, double *g)
{
    const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = at(x, y, z, nx, ny);
                g[i] = 0.5 * (I[at(clampi(x + 1, nx), y, z, nx, ny)] - I[at(clampi(x - 1, nx), y, z, nx, ny)]);
                g[N + i] = 0.5 * (I[at(x, clampi(y + 1, ny), z, nx, ny)] - I[at(x, clampi(y - 1, ny), z, nx, ny)]);
                g[2 * N + i] = 0.5 * (I[at(x, y, clampi(z + 1, nz), nx, ny)] - I[at(x, y, clampi(z - 1, nz), nx, ny)]);
            }
}

/* Gaussian low-pass filter weights (Sec 2.5, low-pass filter kernel): the
 * sampled Gaussian exp(-j^2 / (2 sigma^2)) for j in [-R, R], normalised to
 * unit sum.  w has 2R+1 entries, w[j + R] for offset j. */
void orc_gauss_weights(double sigma, int radius, double *w)
{
    double sum = 0.0;
    for (int j = -radius; j <= radius; ++j) {
        w[j + radius] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
        sum += w[j + radius];
    }
    for (int j = 0; j <= 2 * radius; ++j) w[j] /= sum;
}

/* One 1D correlation pass along `axis` (0 = x, 1 = y, 2 = z) with clamped
 * indices. */
static void smooth_pass(const double *in, int64_t nx, int64_t ny, int64_t nz, int axis, const double *w, int radius,
                        double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int j = -radius; j <= radius; ++j) {
                    int64_t k;
                    if (axis == 0) k = at(clampi(x + j, nx), y, z, nx, ny);
                    else if (axis == 1) k = at(x, clampi(y + j, ny), z, nx, ny);
                    else k = at(x, y, clampi(z + j, nz), nx, ny);
                    s += w[j + radius] * in[k];
                }
                out[at(x, y, z, nx, ny)] = s;
            }
}

/* Gaussian smoothing of `ncomp` planes (Sec 2.1 regularisation, Sec 2.5
 * separable convolution): x pass, then y, then z, clamped borders.
 * Returns ORC_EINVAL on bad sigma/radius, ORC_ENOMEM on allocation failure. */
int orc_smooth(const double *in, int ncomp, int64_t nx, int64_t ny, int64_t nz, double sigma, int radius, double *out)
{
    if (!(sigma > 0.0) || radius < 0 || radius > ORC_MAX_RADIUS) return ORC_EINVAL;
    double w[2 * ORC_MAX_RADIUS + 1];
    orc_gauss_weights(sigma, radius, w);
    const int64_t N = nx * ny * nz;
    double *t1 = (double *)malloc(sizeof(double) * N);
    double *t2 = (double *)malloc(sizeof(double) * N);
    if (!t1 || !t2) { free(t1); free(t2); return ORC_ENOMEM; }
    for (int c = 0; c < ncomp; ++c) {
        smooth_pass(in + c * N, nx, ny, nz, 0, w, radius, t1);
        smooth_pass(t1, nx, ny, nz, 1, w, radius, t2);
        smooth_pass(t2, nx, ny, nz, 2, w, radius, out + c * N);
    }
    free(t1);
    free(t2);
    return ORC_OK;
}

/* Coarse grid size for one down-sampling by 2 (Sec 2.3). */
static int64_t coarse_len(int64_t n) { return (n + 1) / 2; }

/* Down-sampling by a factor of 2 per dimension (Sec 2.3).  The paper gives
 * only the factor; the filter read here is the 2x2x2 box mean, children
 * clamped to the grid, coarse size ceil(n/2). */
void orc_restrict(const double *in, int64_t nx, int64_t ny, int64_t nz, double *out)
{
    const int64_t cx = coarse_len(nx), cy = coarse_len(ny), cz = coarse_len(nz);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < cz; ++k)
        for (int64_t j = 0; j < cy; ++j)
            for (int64_t i = 0; i < cx; ++i) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += in[at(clampi(2 * i + a, nx), clampi(2 * j + b, ny), clampi(2 * k + c, nz), nx, ny)];
                out[at(i, j, k, cx, cy)] = s / 8.0;
            }
}

/* Up-sampling of the displacement field to the next finer level (Sec 2.3):
 * cell-centred trilinear interpolation (fine index f sits at coarse
 * coordinate (f - 0.5) / 2), then values multiplied by 2 because one coarse
 * voxel of motion is two fine voxels. */
void orc_prolong(const double *vc, int64_t cx, int64_t cy, int64_t cz, double *vf, int64_t fx, int64_t fy, int64_t fz)
{
    const int64_t Nc = cx * cy * cz, Nf = fx * fy * fz;
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < fz; ++z)
            for (int64_t y = 0; y < fy; ++y)
                for (int64_t x = 0; x < fx; ++x)
                    vf[c * Nf + at(x, y, z, fx, fy)] =
                        2.0 * orc_trilerp(vc + c * Nc, cx, cy, cz, (x - 0.5) / 2.0, (y - 0.5) / 2.0, (z - 0.5) / 2.0);
    }
}

/* Demons force term of Eq 1 / Eq 3, with Pennec's normalisation factor alpha
 * on the squared intensity difference (Sec 2.2, Eq 5):
 *   f = D g / (alpha^2 D^2 + |g|^2).
 * The paper is silent on a vanishing denominator; the force is 0 there
 * (denominator <= 1e-9, in intensity^2 units). */
static void force_term(double D, double gx, double gy, double gz, double alpha, double *fx, double *fy, double *fz)
{
    double den = alpha * alpha * D * D + (gx * gx + gy * gy + gz * gz);
    if (den <= ORC_DENOM_FLOOR) { *fx = *fy = *fz = 0.0; return; }
    *fx = D * gx / den;
    *fy = D * gy / den;
    *fz = D * gz / den;
}

/* Evolved passive force, Eq 2, read with both gradient magnitudes squared in
 * the second denominator factor (the printed one mixes |grad Is|^2 with
 * |grad Im0|, which is not invariant to intensity scaling) and with a = the
 * gradient magnitude of the level's undeformed moving image at x:
 *   e = 4 D G |G| a / ((2 D^2 + |G|^2 + a^2) (|G|^2 + a^2)),  G = grad Is0. */
static void evolved_term(double D, double gx, double gy, double gz, double a, double *fx, double *fy, double *fz)
{
    double G2 = gx * gx + gy * gy + gz * gz;
    double den = (2.0 * D * D + G2 + a * a) * (G2 + a * a);
    if (den <= ORC_DENOM_FLOOR) { *fx = *fy = *fz = 0.0; return; }
    double s = 4.0 * D * sqrt(G2) * a / den;
    *fx = s * gx;
    *fy = s * gy;
    *fz = s * gz;
}

/* Per-level constants of Sec 2.1: grad Is0 is computed once per level
 * (passive, evolved and double force); |grad Im0| once per level (evolved). */
typedef struct {
    double *gs;  /* 3N or NULL */
    double *am;  /* N or NULL */
} level_consts;

static int uses_static_gradient(int variant)
{
    return variant == ORC_PASSIVE || variant == ORC_EVOLVED || variant == ORC_DOUBLE;
}

/* One force evaluation of Eqs 1-6 over the whole level.
 * Inputs: S, M (level images), v (current field, or the half field h of the
 * inverse-consistent variant), per-level constants.
 * Outputs: u = v + dr; sums[0] = sum_x |dr(x)|, sums[1] = sum_x |v(x)|
 * (per-voxel Euclidean norms, for the relative norm of Sec 2.4) and
 * sums[2] = sum_x D(x)^2 (intensity difference before the update). */
static int force_step(int variant, double alpha, const double *S, const double *M, const double *v, int64_t nx,
                      int64_t ny, int64_t nz, const level_consts *lc, double *u, double *sums)
{
    const int64_t N = nx * ny * nz;
    const int need_gm = (variant == ORC_ACTIVE || variant == ORC_DOUBLE || variant == ORC_INVERSE_CONSISTENT);
    const int is_ic = (variant == ORC_INVERSE_CONSISTENT);
    double *Im = (double *)malloc(sizeof(double) * N);
    double *D = (double *)malloc(sizeof(double) * N);
    double *dr = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = need_gm ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    double *Is = is_ic ? (double *)malloc(sizeof(double) * N) : NULL;
    double *gsn = is_ic ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    int rc = ORC_OK;
    if (!Im || !D || !dr || (need_gm && !gm) || (is_ic && (!Is || !gsn))) { rc = ORC_ENOMEM; goto done; }

    /* deformed moving image Im(n); for Eq 6 also the deformed static image Is(n) */
    orc_warp(M, v, nx, ny, nz, +1.0, Im);
    if (need_gm) orc_gradient(Im, nx, ny, nz, gm);
    if (is_ic) {
        orc_warp(S, v, nx, ny, nz, -1.0, Is);
        orc_gradient(Is, nx, ny, nz, gsn);
    }

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double fx = 0, fy = 0, fz = 0, ax = 0, ay = 0, az = 0;
        if (is_ic) {
            /* Eq 6: D = Im(n) - Is(n), g = grad Im(n) + grad Is(n) */
            D[i] = Im[i] - Is[i];
            force_term(D[i], gm[i] + gsn[i], gm[N + i] + gsn[N + i], gm[2 * N + i] + gsn[2 * N + i], alpha, &fx,
                       &fy, &fz);
        } else {
            D[i] = Im[i] - S[i];
            if (variant == ORC_PASSIVE || variant == ORC_DOUBLE) /* Eq 1; first term of Eq 4 / Eq 5 */
                force_term(D[i], lc->gs[i], lc->gs[N + i], lc->gs[2 * N + i], alpha, &fx, &fy, &fz);
            if (variant == ORC_ACTIVE || variant == ORC_DOUBLE) /* Eq 3; second term of Eq 4 / Eq 5 */
                force_term(D[i], gm[i], gm[N + i], gm[2 * N + i], alpha, &ax, &ay, &az);
            if (variant == ORC_EVOLVED) /* Eq 2 */
                evolved_term(D[i], lc->gs[i], lc->gs[N + i], lc->gs[2 * N + i], lc->am[i], &fx, &fy, &fz);
        }
        dr[i] = fx + ax;
        dr[N + i] = fy + ay;
        dr[2 * N + i] = fz + az;
        u[i] = v[i] + dr[i];
        u[N + i] = v[N + i] + dr[N + i];
        u[2 * N + i] = v[2 * N + i] + dr[2 * N + i];
    }

    /* serial sums in voxel order */
    {
        double s1 = 0.0, s2 = 0.0, sse = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            s1 += sqrt(dr[i] * dr[i] + dr[N + i] * dr[N + i] + dr[2 * N + i] * dr[2 * N + i]);
            s2 += sqrt(v[i] * v[i] + v[N + i] * v[N + i] + v[2 * N + i] * v[2 * N + i]);
            sse += D[i] * D[i];
        }
        sums[0] = s1;
        sums[1] = s2;
        sums[2] = sse;
    }
done:
    free(Im);
    free(D);
    free(dr);
    free(gm);
    free(Is);
    free(gsn);
    return rc;
}

static int make_level_consts(int variant, const double *S, const double *M, int64_t nx, int64_t ny, int64_t nz,
                             level_consts *lc)
{
    const int64_t N = nx * ny * nz;
    lc->gs = NULL;
    lc->am = NULL;
    if (uses_static_gradient(variant)) {
        if (!(lc->gs = (double *)malloc(sizeof(double) * 3 * N))) return ORC_ENOMEM;
        orc_gradient(S, nx, ny, nz, lc->gs);
    }
    if (variant == ORC_EVOLVED) {
        double *gm0 = (double *)malloc(sizeof(double) * 3 * N);
        lc->am = (double *)malloc(sizeof(double) * N);
        if (!gm0 || !lc->am) { free(gm0); return ORC_ENOMEM; }
        orc_gradient(M, nx, ny, nz, gm0);
        for (int64_t i = 0; i < N; ++i)
            lc->am[i] = sqrt(gm0[i] * gm0[i] + gm0[N + i] * gm0[N + i] + gm0[2 * N + i] * gm0[2 * N + i]);
        free(gm0);
    }
    return ORC_OK;
}

static void free_level_consts(level_consts *lc)
{
    free(lc->gs);
    free(lc->am);
    lc->gs = NULL;
    lc->am = NULL;
}

static int valid_variant(int variant) { return variant >= ORC_PASSIVE && variant <= ORC_INVERSE_CONSISTENT; }

/* Public single force evaluation: u = v + dr (Eqs 1-6) with the per-level
 * constants computed from S and M as given.  sums as in force_step. */
int orc_force(int variant, double alpha, const double *S, const double *M, const double *v, int64_t nx, int64_t ny,
              int64_t nz, double *u, double *sums)
{
    if (!valid_variant(variant) || !(alpha > 0.0)) return ORC_EINVAL;
    level_consts lc;
    int rc = make_level_consts(variant, S, M, nx, ny, nz, &lc);
    if (rc == ORC_OK) rc = force_step(variant, alpha, S, M, v, nx, ny, nz, &lc, u, sums);
    free_level_consts(&lc);
    return rc;
}

/* Iterations at one resolution level (Sec 2.1, Fig 1a): deform, force,
 * add, Gaussian-smooth the total field, record the relative norm of Sec 2.4.
 *
 * history receives 4 doubles per iteration run: sum|dr|, sum|v| (field before
 * the update), mean squared intensity difference D^2 / N, and the relative
 * norm l = sum|dr| / sum|v| (NaN while sum|v| = 0).
 *
 * Stopping (Sec 2.4; the printed inequality is garbled): with eps > 0 the
 * level stops after iteration n >= 10 when l(n-10) - l(n) <= eps, i.e. when
 * the relative norm has stopped falling over ten iterations; eps = 0 runs the
 * fixed count.  Returns the number of iterations run, or a negative code. */
int orc_iterate(int variant, double alpha, double sigma, int radius, const double *S, const double *M, int64_t nx,
                int64_t ny, int64_t nz, double *v, int iters, double eps, double *history)
{
    if (!valid_variant(variant) || !(alpha > 0.0) || !(sigma > 0.0) || radius < 0 || radius > ORC_MAX_RADIUS ||
        iters < 0 || !(eps >= 0.0))
        return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    level_consts lc;
    double *u = (double *)malloc(sizeof(double) * 3 * N);
    int rc = make_level_consts(variant, S, M, nx, ny, nz, &lc);
    if (!u) rc = ORC_ENOMEM;
    int n = 0;
    for (; rc == ORC_OK && n < iters; ++n) {
        double sums[3];
        rc = force_step(variant, alpha, S, M, v, nx, ny, nz, &lc, u, sums);
        if (rc != ORC_OK) break;
        rc = orc_smooth(u, 3, nx, ny, nz, sigma, radius, v);
        if (rc != ORC_OK) break;
        double l = sums[1] > 0.0 ? sums[0] / sums[1] : NAN;
        history[4 * n + 0] = sums[0];
        history[4 * n + 1] = sums[1];
        history[4 * n + 2] = sums[2] / (double)N;
        history[4 * n + 3] = l;
        if (eps > 0.0 && n >= 10) {
            double l10 = history[4 * (n - 10) + 3];
            if (!isnan(l) && !isnan(l10) && l10 - l <= eps) { ++n; break; }
        }
    }
    free(u);
    free_level_consts(&lc);
    return rc == ORC_OK ? n : rc;
}

/* Output field of the inverse-consistent variant.  The iteration returns the
 * symmetric half field h with M(p - h(p)) = S(p + h(p)) at a match.  Writing
 * z = p + h(p) gives M(z - 2 h(p)) = S(z), so the field in the convention of
 * the other variants is w(z) = 2 h(p) with p = z - h(p).  p is found by
 * fixed-point iteration: it starts at the first-order inverse p = z - h(z)
 * and takes K further updates p <- z - h(p) (reading of Sec 2.2, text after
 * Eq 6). */
void orc_compose(const double *h, int64_t nx, int64_t ny, int64_t nz, int K, double *w)
{
    const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = at(x, y, z, nx, ny);
                /* start: p = z - h(z), h read at the grid point itself */
                double px = (double)x - h[i], py = (double)y - h[N + i], pz = (double)z - h[2 * N + i];
                for (int k = 0; k < K; ++k) {
                    double hx = orc_trilerp(h, nx, ny, nz, px, py, pz);
                    double hy = orc_trilerp(h + N, nx, ny, nz, px, py, pz);
                    double hz = orc_trilerp(h + 2 * N, nx, ny, nz, px, py, pz);
                    px = (double)x - hx;
                    py = (double)y - hy;
                    pz = (double)z - hz;
                }
                w[i] = 2.0 * orc_trilerp(h, nx, ny, nz, px, py, pz);
                w[N + i] = 2.0 * orc_trilerp(h + N, nx, ny, nz, px, py, pz);
                w[2 * N + i] = 2.0 * orc_trilerp(h + 2 * N, nx, ny, nz, px, py, pz);
            }
}

/* ------------------------------------------------------------------------
 * Physical units.  The paper states the method in voxel units (its Gaussian
 * has unit standard deviation, Sec 2.5) while its images have anisotropic
 * voxels (Table 1: about 1.1 x 1.1 x 2.5 mm).  In the physical mode below the
 * same iteration is written in millimetres:
 *   - the gradient is in intensity per mm (central difference over 2 h_a);
 *   - the field, its increment and the norms of Sec 2.4 are in mm; a sample
 *     of the deformed image lies at x - v(x) / h (voxel coordinates);
 *   - the force carries the squared intensity difference over a squared
 *     length, the mean squared voxel size K = (h_x^2 + h_y^2 + h_z^2) / 3 of
 *     the level (the normaliser of the demons force in physical units), so
 *     Eq 1 becomes dr = D G K / (alpha^2 D^2 + K |G|^2) and Eq 2
 *     e = 4 D G |G| a K / ((2 D^2 + K |G|^2 + K a^2) (|G|^2 + a^2))
 *     (a = |grad Im0| per mm);
 *     the zero-force floor applies to the first factor of each denominator
 *     as in voxel units (there K = 1);
 *   - the Gaussian's sigma (and the image pre-smoothing's) is in mm of the
 *     input grid: sigma / h_a voxels along axis a on every level, as the
 *     voxel mode uses sigma voxels on every level; the radius is
 *     ceil(3 sigma / h_a) per axis unless given;
 *   - level k has voxels of 2^k h (2x down-sampling, Sec 2.3), and the field
 *     is carried to the finer level by the same cell-centred interpolation
 *     without the factor 2 (a length in mm does not change with the grid).
 * With h = (1, 1, 1) every step reduces to the voxel-unit one.
 * ------------------------------------------------------------------------ */

/* Per-axis Gaussian smoothing: x pass with sigma[0], radius[0], then y, then
 * z, clamped borders. */
int orc_smooth3(const double *in, int ncomp, int64_t nx, int64_t ny, int64_t nz, const double *sigma,
                const int *radius, double *out)
{
    double w[3][2 * ORC_MAX_RADIUS + 1];
    for (int a = 0; a < 3; ++a) {
        if (!(sigma[a] > 0.0) || radius[a] < 0 || radius[a] > ORC_MAX_RADIUS) return ORC_EINVAL;
        orc_gauss_weights(sigma[a], radius[a], w[a]);
    }
    const int64_t N = nx * ny * nz;
    double *t1 = (double *)malloc(sizeof(double) * N);
    double *t2 = (double *)malloc(sizeof(double) * N);
    if (!t1 || !t2) { free(t1); free(t2); return ORC_ENOMEM; }
    for (int c = 0; c < ncomp; ++c) {
        smooth_pass(in + c * N, nx, ny, nz, 0, w[0], radius[0], t1);
        smooth_pass(t1, nx, ny, nz, 1, w[1], radius[1], t2);
        smooth_pass(t2, nx, ny, nz, 2, w[2], radius[2], out + c * N);
    }
    free(t1);
    free(t2);
    return ORC_OK;
}

/* Gradient in intensity per mm, voxel size h (mm). */
static void gradient_mm(const double *I, int64_t nx, int64_t ny, int64_t nz, const double *h, double *g)
{
    const int64_t N = nx * ny * nz;
    orc_gradient(I, nx, ny, nz, g);
    for (int a = 0; a < 3; ++a)
        for (int64_t i = 0; i < N; ++i) g[a * N + i] /= h[a];
}

/* Deformed image with a field in mm: out(x) = I(x - sign * v(x) / h). */
static void warp_mm(const double *I, const double *v, int64_t nx, int64_t ny, int64_t nz, const double *h, double sign,
                    double *out)
{
    const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = at(x, y, z, nx, ny);
                out[i] = orc_trilerp(I, nx, ny, nz, (double)x - sign * v[i] / h[0], (double)y - sign * v[N + i] / h[1],
                                     (double)z - sign * v[2 * N + i] / h[2]);
            }
}

/* Eq 1 / Eq 3 / Eq 5 in mm (see above). */
static void force_term_mm(double D, const double *G, double alpha, double K, double *f)
{
    const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    const double den = alpha * alpha * D * D + K * G2;
    if (den <= ORC_DENOM_FLOOR) { f[0] = f[1] = f[2] = 0.0; return; }
    for (int a = 0; a < 3; ++a) f[a] = D * G[a] * K / den;
}

/* Eq 2 in mm (see above, numerator and denominator multiplied by K once
 * more); a = |grad Im0| in intensity per mm. */
static void evolved_term_mm(double D, const double *G, double am, double K, double *f)
{
    const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    const double den = (2.0 * D * D + K * G2 + K * am * am) * (K * G2 + K * am * am);
    if (den <= ORC_DENOM_FLOOR) { f[0] = f[1] = f[2] = 0.0; return; }
    const double s = 4.0 * D * sqrt(G2) * am * K * K / den;
    for (int a = 0; a < 3; ++a) f[a] = s * G[a];
}

/* One force evaluation in mm at a level of voxel size h: u = v + dr (mm),
 * sums as in force_step with the norms in mm. */
static int force_step_mm(int variant, double alpha, const double *S, const double *M, const double *v, int64_t nx,
                         int64_t ny, int64_t nz, const double *h, const double *gs, const double *am, double *u,
                         double *sums)
{
    const int64_t N = nx * ny * nz;
    const double K = (h[0] * h[0] + h[1] * h[1] + h[2] * h[2]) / 3.0;
    const int need_gm = (variant == ORC_ACTIVE || variant == ORC_DOUBLE || variant == ORC_INVERSE_CONSISTENT);
    const int is_ic = (variant == ORC_INVERSE_CONSISTENT);
    double *Im = (double *)malloc(sizeof(double) * N);
    double *D = (double *)malloc(sizeof(double) * N);
    double *dr = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = need_gm ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    double *Is = is_ic ? (double *)malloc(sizeof(double) * N) : NULL;
    double *gsn = is_ic ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    int rc = ORC_OK;
    if (!Im || !D || !dr || (need_gm && !gm) || (is_ic && (!Is || !gsn))) { rc = ORC_ENOMEM; goto done; }
    warp_mm(M, v, nx, ny, nz, h, +1.0, Im);
    if (need_gm) gradient_mm(Im, nx, ny, nz, h, gm);
    if (is_ic) {
        warp_mm(S, v, nx, ny, nz, h, -1.0, Is);
        gradient_mm(Is, nx, ny, nz, h, gsn);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double f[3] = {0, 0, 0}, b[3] = {0, 0, 0}, G[3];
        if (is_ic) {
            D[i] = Im[i] - Is[i];
            for (int a = 0; a < 3; ++a) G[a] = gm[a * N + i] + gsn[a * N + i];
            force_term_mm(D[i], G, alpha, K, f);
        } else {
            D[i] = Im[i] - S[i];
            for (int a = 0; a < 3; ++a) G[a] = gs ? gs[a * N + i] : 0.0;
            if (variant == ORC_PASSIVE || variant == ORC_DOUBLE) force_term_mm(D[i], G, alpha, K, f);
            if (variant == ORC_ACTIVE || variant == ORC_DOUBLE) {
                double Gm[3] = {gm[i], gm[N + i], gm[2 * N + i]};
                force_term_mm(D[i], Gm, alpha, K, b);
            }
            if (variant == ORC_EVOLVED) evolved_term_mm(D[i], G, am[i], K, f);
        }
        for (int a = 0; a < 3; ++a) {
            dr[a * N + i] = f[a] + b[a];
            u[a * N + i] = v[a * N + i] + dr[a * N + i];
        }
    }
    {
        double s1 = 0.0, s2 = 0.0, sse = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            s1 += sqrt(dr[i] * dr[i] + dr[N + i] * dr[N + i] + dr[2 * N + i] * dr[2 * N + i]);
            s2 += sqrt(v[i] * v[i] + v[N + i] * v[N + i] + v[2 * N + i] * v[2 * N + i]);
            sse += D[i] * D[i];
        }
        sums[0] = s1;
        sums[1] = s2;
        sums[2] = sse;
    }
done:
    free(Im);
    free(D);
    free(dr);
    free(gm);
    free(Is);
    free(gsn);
    return rc;
}

/* Iterations at one level in mm (orc_iterate in physical units): v in mm,
 * voxel size h, Gaussian widths sigma[a] voxels with radius[a]. */
int orc_iterate_mm(int variant, double alpha, const double *sigma, const int *radius, const double *S, const double *M,
                   int64_t nx, int64_t ny, int64_t nz, const double *h, double *v, int iters, double eps,
                   double *history)
{
    if (!valid_variant(variant) || !(alpha > 0.0) || iters < 0 || !(eps >= 0.0)) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!(h[a] > 0.0) || !(sigma[a] > 0.0) || radius[a] < 0 || radius[a] > ORC_MAX_RADIUS) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    double *u = (double *)malloc(sizeof(double) * 3 * N);
    double *gs = uses_static_gradient(variant) ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    double *am = variant == ORC_EVOLVED ? (double *)malloc(sizeof(double) * N) : NULL;
    double *gm0 = variant == ORC_EVOLVED ? (double *)malloc(sizeof(double) * 3 * N) : NULL;
    int rc = ORC_OK, n = 0;
    if (!u || (uses_static_gradient(variant) && !gs) || (variant == ORC_EVOLVED && (!am || !gm0))) rc = ORC_ENOMEM;
    if (rc == ORC_OK && gs) gradient_mm(S, nx, ny, nz, h, gs);
    if (rc == ORC_OK && am) {
        gradient_mm(M, nx, ny, nz, h, gm0);
        for (int64_t i = 0; i < N; ++i)
            am[i] = sqrt(gm0[i] * gm0[i] + gm0[N + i] * gm0[N + i] + gm0[2 * N + i] * gm0[2 * N + i]);
    }
    for (; rc == ORC_OK && n < iters; ++n) {
        double sums[3];
        rc = force_step_mm(variant, alpha, S, M, v, nx, ny, nz, h, gs, am, u, sums);
        if (rc != ORC_OK) break;
        rc = orc_smooth3(u, 3, nx, ny, nz, sigma, radius, v);
        if (rc != ORC_OK) break;
        double l = sums[1] > 0.0 ? sums[0] / sums[1] : NAN;
        history[4 * n + 0] = sums[0];
        history[4 * n + 1] = sums[1];
        history[4 * n + 2] = sums[2] / (double)N;
        history[4 * n + 3] = l;
        if (eps > 0.0 && n >= 10) {
            double l10 = history[4 * (n - 10) + 3];
            if (!isnan(l) && !isnan(l10) && l10 - l <= eps) { ++n; break; }
        }
    }
    free(u);
    free(gs);
    free(am);
    free(gm0);
    return rc == ORC_OK ? n : rc;
}

/* Multi-scale registration (Sec 2.3, Fig 1a), with the optional physical
 * units above and the optional Gaussian pre-smoothing of the images (Sec 2.5:
 * the low-pass filter kernel smooths images as well as displacement
 * vectors).
 *
 * levels >= 1 resolution levels, level 0 the input grid and level k of size
 * ceil(n / 2^k) per dimension; iters[] lists the iteration counts from the
 * coarsest level to the finest.  The field starts at 0 on the coarsest level
 * and is carried to each finer level by cell-centred interpolation (values
 * times 2 in voxel units).  compose_iters is K of orc_compose for the
 * inverse-consistent variant (ignored otherwise).
 *
 * spacing: NULL or the three voxel sizes in mm; physical != 0 selects the
 * physical units (spacing required), sigma then in mm.  image_sigma > 0
 * smooths every level's S and M (restricted from the unsmoothed finer level)
 * with a Gaussian of that width (voxels, or mm in the physical mode; radius
 * ceil(3 width) per axis) before the level's iterations; 0 disables it.
 *
 * field receives 3 * nx*ny*nz doubles (voxel units, M(x - v(x)) = S(x));
 * history must hold 4 doubles per iteration of sum(iters); iters_run[] gets
 * the iterations run per level (coarse to fine); the history of the levels is
 * packed in that order (sums in mm in the physical mode).  Returns ORC_OK,
 * ORC_EINVAL, ORC_ENOMEM or ORC_ENUMERIC (a non-finite sum in the history). */
int orc_register_ex(const double *S, const double *M, int64_t nx, int64_t ny, int64_t nz, const double *spacing,
                    int physical, double image_sigma, int variant, double alpha, double sigma, int radius, int levels,
                    const int *iters, double eps, int compose_iters, double *field, double *history, int *iters_run)
{
    if (nx < 1 || ny < 1 || nz < 1 || levels < 1 || levels > ORC_MAX_LEVELS || !valid_variant(variant) ||
        compose_iters < 0 || !(image_sigma >= 0.0) || !(sigma > 0.0))
        return ORC_EINVAL;
    if (physical && !spacing) return ORC_EINVAL;
    if (spacing)
        for (int a = 0; a < 3; ++a)
            if (!(spacing[a] > 0.0)) return ORC_EINVAL;
    for (int l = 0; l < levels; ++l)
        if (iters[l] < 0) return ORC_EINVAL;
    /* Gaussian widths in voxels per axis */
    double sv[3], si[3];
    int rv[3], ri[3];
    for (int a = 0; a < 3; ++a) {
        sv[a] = physical ? sigma / spacing[a] : sigma;
        rv[a] = radius > 0 ? radius : (int)ceil(3.0 * sv[a]);
        si[a] = physical ? image_sigma / spacing[a] : image_sigma;
        ri[a] = (int)ceil(3.0 * si[a]);
        if (rv[a] > ORC_MAX_RADIUS || (image_sigma > 0.0 && ri[a] > ORC_MAX_RADIUS)) return ORC_EINVAL;
    }

    int64_t dims[ORC_MAX_LEVELS][3];
    double *Sk[ORC_MAX_LEVELS] = {0}, *Mk[ORC_MAX_LEVELS] = {0};
    double *Ss[ORC_MAX_LEVELS] = {0}, *Ms[ORC_MAX_LEVELS] = {0};  /* pre-smoothed levels */
    dims[0][0] = nx;
    dims[0][1] = ny;
    dims[0][2] = nz;
    for (int k = 1; k < levels; ++k)
        for (int d = 0; d < 3; ++d) dims[k][d] = coarse_len(dims[k - 1][d]);

    int rc = ORC_OK;
    const int64_t N0 = nx * ny * nz;
    double *v = (double *)calloc(3 * N0, sizeof(double));
    double *vt = (double *)calloc(3 * N0, sizeof(double));
    if (!v || !vt) rc = ORC_ENOMEM;
    Sk[0] = (double *)S;
    Mk[0] = (double *)M;
    for (int k = 1; k < levels && rc == ORC_OK; ++k) {
        int64_t Nk = dims[k][0] * dims[k][1] * dims[k][2];
        Sk[k] = (double *)malloc(sizeof(double) * Nk);
        Mk[k] = (double *)malloc(sizeof(double) * Nk);
        if (!Sk[k] || !Mk[k]) { rc = ORC_ENOMEM; break; }
        orc_restrict(Sk[k - 1], dims[k - 1][0], dims[k - 1][1], dims[k - 1][2], Sk[k]);
        orc_restrict(Mk[k - 1], dims[k - 1][0], dims[k - 1][1], dims[k - 1][2], Mk[k]);
    }
    for (int k = 0; k < levels && rc == ORC_OK && image_sigma > 0.0; ++k) {
        const int64_t *d = dims[k];
        int64_t Nk = d[0] * d[1] * d[2];
        Ss[k] = (double *)malloc(sizeof(double) * Nk);
        Ms[k] = (double *)malloc(sizeof(double) * Nk);
        if (!Ss[k] || !Ms[k]) { rc = ORC_ENOMEM; break; }
        rc = orc_smooth3(Sk[k], 1, d[0], d[1], d[2], si, ri, Ss[k]);
        if (rc == ORC_OK) rc = orc_smooth3(Mk[k], 1, d[0], d[1], d[2], si, ri, Ms[k]);
    }

    int64_t hist_off = 0;
    for (int k = levels - 1; k >= 0 && rc == ORC_OK; --k) {
        const int li = levels - 1 - k; /* coarse-to-fine position */
        const int64_t *d = dims[k];
        const double *Sl = image_sigma > 0.0 ? Ss[k] : Sk[k], *Ml = image_sigma > 0.0 ? Ms[k] : Mk[k];
        if (k < levels - 1) {
            const int64_t *dc = dims[k + 1];
            orc_prolong(v, dc[0], dc[1], dc[2], vt, d[0], d[1], d[2]);
            const int64_t n3 = 3 * d[0] * d[1] * d[2];
            if (physical) /* a length in mm: undo the voxel-unit factor 2 */
                for (int64_t i = 0; i < n3; ++i) vt[i] *= 0.5;
            memcpy(v, vt, sizeof(double) * n3);
        }
        int n;
        if (physical) {
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = ldexp(spacing[a], k);  /* 2^k h */
            n = orc_iterate_mm(variant, alpha, sv, rv, Sl, Ml, d[0], d[1], d[2], h, v, iters[li], eps,
                               history + 4 * hist_off);
        } else {
            n = orc_iterate(variant, alpha, sigma, rv[0], Sl, Ml, d[0], d[1], d[2], v, iters[li], eps,
                            history + 4 * hist_off);
        }
        if (n < 0) { rc = n; break; }
        iters_run[li] = n;
        hist_off += n;
    }

    if (rc == ORC_OK) {
        if (physical) /* mm -> voxels of the input grid */
            for (int a = 0; a < 3; ++a)
                for (int64_t i = 0; i < N0; ++i) v[a * N0 + i] /= spacing[a];
        if (variant == ORC_INVERSE_CONSISTENT) orc_compose(v, nx, ny, nz, compose_iters, field);
        else memcpy(field, v, sizeof(double) * 3 * N0);
        for (int64_t i = 0; i < 4 * hist_off; ++i)
            if ((i % 4) != 3 && !isfinite(history[i])) { rc = ORC_ENUMERIC; break; }
    }
    for (int k = 1; k < levels; ++k) { free(Sk[k]); free(Mk[k]); }
    for (int k = 0; k < levels; ++k) { free(Ss[k]); free(Ms[k]); }
    free(v);
    free(vt);
    return rc;
}

/* Multi-scale registration in voxel units without pre-smoothing (the paper's
 * form); see orc_register_ex. */
int orc_register(const double *S, const double *M, int64_t nx, int64_t ny, int64_t nz, int variant, double alpha,
                 double sigma, int radius, int levels, const int *iters, double eps, int compose_iters,
                 double *field, double *history, int *iters_run)
{
    return orc_register_ex(S, M, nx, ny, nz, NULL, 0, 0.0, variant, alpha, sigma, radius, levels, iters, eps,
                           compose_iters, field, history, iters_run);
}
