/*
 * heatcg_oracle.c -- plain, slow, obviously correct CPU reference for the
 * 7-point explicit heat update and for Conjugate Gradient on the 7-point
 * Laplacian.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP path.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no -ffast-math:
 * every sum below is evaluated in the order it is written).
 *
 * Layout of every 3-D array: a[(k*ny + j)*nx + i], i (x) fastest, k (z)
 * slowest -- the paper initialises and partitions the domain in the order
 * k, j, i (Methodology, "Multi-GPU OpenMP Offloading Versions"; the
 * COMPUTE_SINGLE_GPU pseudocode indexes u[k,j,i]).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, k, nx, ny) ((((long)(k)) * (ny) + (j)) * (nx) + (i))

/* Number of OpenMP threads the loops below run on. */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Thread count of the parallel loops that follow (the CPU baseline times
 * the oracle at one thread and at every physical core). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* Wall time of the step loop (oracle_heat_f64) or of the iteration loop
 * (oracle_cg) of the last call, set-up and copies excluded, the way the
 * paper's timer brackets its time loop only (Methodology). */
static double g_loop_seconds = 0.0;
double oracle_last_loop_seconds(void) { return g_loop_seconds; }

/* ------------------------------------------------------------------------ */
/* Heat equation, constant coefficient                                       */
/* ------------------------------------------------------------------------ */

/*
 * One explicit (forward-Euler) step of the heat equation on every interior
 * node, Eq. (4) of "Mathematical Details" with a constant coefficient
 * (kappa = alpha) and no source (f = 0):
 *
 *   u_new = u + r * (sum of the 6 face neighbours - 6 u),  r = alpha dt / h^2
 *
 * The neighbour sum is taken in the fixed order
 *   ((x- + x+) + (y- + y+)) + (z- + z+)
 * and then 6*u is subtracted; the node value is added last.  Boundary nodes
 * (the outermost layer) are Dirichlet nodes and are never written.
 */
void oracle_heat_sweep_f64(const double *u, double *un, long nx, long ny,
                           long nz, double r)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const double c = u[p];
                const double nsum = ((u[p - sx] + u[p + sx]) +
                                     (u[p - sy] + u[p + sy])) +
                                    (u[p - sz] + u[p + sz]);
                const double lap = nsum - 6.0 * c;
                un[p] = c + r * lap;
            }
}

/*
 * `steps` explicit steps with ping-pong buffers and a swap after every step,
 * as in the paper's OpenMP solver (Pseudocode alg:heat3d) and its one-GPU
 * baseline (alg:1gpu-base).  `u` holds u^0 on entry and u^steps on return.
 * The step count is an integer (the paper's `while t < T` with a floating
 * t can take one step more or less).  Returns 0, or -4 when out of memory.
 */
int oracle_heat_f64(double *u, long nx, long ny, long nz, double r, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    double *w = (double *)malloc((size_t)n * sizeof(double));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(double)); /* boundary of w = boundary of u */
    double *a = u, *b = w;
    const double t0 = omp_get_wtime();
    for (long s = 0; s < steps; ++s) {
        oracle_heat_sweep_f64(a, b, nx, ny, nz, r);
        double *t = a;
        a = b;
        b = t;
    }
    g_loop_seconds = omp_get_wtime() - t0;
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(double));
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Heat equation in lower precision (not in the paper, which works in FP64)  */
/* ------------------------------------------------------------------------ */

/*
 * The same step in single precision: every value and every operation is
 * binary32 (x86-64 SSE arithmetic, no excess precision, no contraction), in
 * the order of the FP64 step, with r rounded to binary32 once.
 */
void oracle_heat_sweep_f32(const float *u, float *un, long nx, long ny,
                           long nz, float r)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float c = u[p];
                const float nsum = ((u[p - sx] + u[p + sx]) +
                                    (u[p - sy] + u[p + sy])) +
                                   (u[p - sz] + u[p + sz]);
                const float lap = nsum - 6.0f * c;
                un[p] = c + r * lap;
            }
}

int oracle_heat_f32(float *u, long nx, long ny, long nz, float r, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    float *w = (float *)malloc((size_t)n * sizeof(float));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(float));
    float *a = u, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_sweep_f32(a, b, nx, ny, nz, r);
        float *t = a;
        a = b;
        b = t;
    }
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(float));
    free(w);
    return 0;
}

/*
 * bfloat16: the upper 16 bits of a binary32 (sign, 8-bit exponent, 7
 * stored significand bits).  Widening is exact.  Narrowing rounds to the
 * nearest bfloat16, ties to the even significand; NaN stays a quiet NaN.
 */
float oracle_f32_from_bf16(uint16_t h)
{
    const uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, sizeof f);
    return f;
}

uint16_t oracle_bf16_from_f32(float f)
{
    uint32_t bits;
    memcpy(&bits, &f, sizeof bits);
    if ((bits & 0x7fffffffu) > 0x7f800000u)      /* NaN */
        return (uint16_t)((bits >> 16) | 0x0040u);
    const uint32_t upper = bits >> 16;
    const uint32_t lower = bits & 0xffffu;
    uint32_t out = upper;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u)))
        out = upper + 1u;                        /* carries into the exponent */
    return (uint16_t)out;
}

void oracle_bf16_round_array(const float *in, uint16_t *out, long n)
{
    for (long q = 0; q < n; ++q)
        out[q] = oracle_bf16_from_f32(in[q]);
}

/*
 * One step with bfloat16 storage and binary32 arithmetic: the stored values
 * are widened, the binary32 step above is applied, and the new value is
 * rounded to bfloat16 (round to nearest, ties to even).
 */
void oracle_heat_sweep_bf16(const uint16_t *u, uint16_t *un, long nx, long ny,
                            long nz, float r)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float c = oracle_f32_from_bf16(u[p]);
                const float nsum =
                    ((oracle_f32_from_bf16(u[p - sx]) + oracle_f32_from_bf16(u[p + sx])) +
                     (oracle_f32_from_bf16(u[p - sy]) + oracle_f32_from_bf16(u[p + sy]))) +
                    (oracle_f32_from_bf16(u[p - sz]) + oracle_f32_from_bf16(u[p + sz]));
                const float lap = nsum - 6.0f * c;
                un[p] = oracle_bf16_from_f32(c + r * lap);
            }
}

int oracle_heat_bf16(uint16_t *u, long nx, long ny, long nz, float r, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    uint16_t *w = (uint16_t *)malloc((size_t)n * sizeof(uint16_t));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(uint16_t));
    uint16_t *a = u, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_sweep_bf16(a, b, nx, ny, nz, r);
        uint16_t *t = a;
        a = b;
        b = t;
    }
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(uint16_t));
    free(w);
    return 0;
}

/*
 * bfloat16 storage as offsets from a fixed bfloat16 base (the other remedy
 * for the stagnation of nearest rounding; not in the paper): a node's value
 * is u = base + delta, both stored in bfloat16 and added in binary32.  A
 * step forms u at the node and its six neighbours that way, applies the
 * binary32 step above, and stores the new offset rounded to the nearest
 * bfloat16: delta' = bf16(u' - base) (binary32 subtraction).  The base is
 * never written; as the offsets stay small their ulp is far below the one
 * of u, so the increments that nearest rounding drops on u are kept.  With
 * base = 0 this is the bfloat16 step above.
 */
static float offset_value(const uint16_t *base, const uint16_t *delta, long p)
{
    return oracle_f32_from_bf16(base[p]) + oracle_f32_from_bf16(delta[p]);
}

void oracle_heat_sweep_bf16_offset(const uint16_t *base, const uint16_t *d,
                                   uint16_t *dn, long nx, long ny, long nz, float r)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float c = offset_value(base, d, p);
                const float nsum =
                    ((offset_value(base, d, p - sx) + offset_value(base, d, p + sx)) +
                     (offset_value(base, d, p - sy) + offset_value(base, d, p + sy))) +
                    (offset_value(base, d, p - sz) + offset_value(base, d, p + sz));
                const float lap = nsum - 6.0f * c;
                const float un = c + r * lap;
                dn[p] = oracle_bf16_from_f32(un - oracle_f32_from_bf16(base[p]));
            }
}

int oracle_heat_bf16_offset(const uint16_t *base, uint16_t *delta, long nx, long ny, long nz,
                            float r, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    uint16_t *w = (uint16_t *)malloc((size_t)n * sizeof(uint16_t));
    if (!w)
        return -4;
    memcpy(w, delta, (size_t)n * sizeof(uint16_t));
    uint16_t *a = delta, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_sweep_bf16_offset(base, a, b, nx, ny, nz, r);
        uint16_t *t = a;
        a = b;
        b = t;
    }
    if (a != delta)
        memcpy(delta, a, (size_t)n * sizeof(uint16_t));
    free(w);
    return 0;
}

/*
 * bfloat16 storage with stochastic rounding.  Round to nearest leaves a node
 * unchanged whenever its increment is below half a bfloat16 ulp, which for
 * smooth fields is every step (the sweep stagnates); rounding up with
 * probability equal to the discarded fraction instead makes the rounding
 * unbiased, so small increments accumulate on average.
 *
 * The random bits come from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC 2011), written here from that definition: ten rounds, each
 * multiplying words 0 and 2 of the counter by two constants, recombining
 * high and low halves with the other words and the key, with the key bumped
 * by two Weyl constants between rounds.
 */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/*
 * The 16 random bits of node p (linear index (k*ny + j)*nx + i) at step t
 * under `seed`: nodes are taken in aligned groups of 8; group g = p / 8 draws
 * one Philox4x32-10 block with counter (g low, g high, t low, t high) and key
 * (seed low, seed high); node p takes word (p mod 8) / 2 of the block, its
 * low half when p is even and its high half when p is odd.
 */
uint16_t oracle_sr_bits(uint64_t p, uint64_t t, uint64_t seed)
{
    const uint64_t g = p >> 3;
    const uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)t, (uint32_t)(t >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    const uint32_t w = out[(p & 7u) >> 1];
    return (uint16_t)((p & 1u) ? (w >> 16) : (w & 0xffffu));
}

/*
 * Stochastic rounding of a binary32 to bfloat16 with 16 random bits rho:
 * the magnitude is rounded up exactly when (its discarded 16 bits) + rho
 * carries into the kept part, i.e. with probability (discarded bits)/2^16.
 * Values that are already bfloat16 are unchanged.  NaN stays a quiet NaN.
 */
uint16_t oracle_bf16_sr_from_f32(float f, uint16_t rho)
{
    uint32_t bits;
    memcpy(&bits, &f, sizeof bits);
    if ((bits & 0x7fffffffu) > 0x7f800000u)      /* NaN */
        return (uint16_t)((bits >> 16) | 0x0040u);
    const uint32_t upper = bits >> 16;
    const uint32_t lower = bits & 0xffffu;
    return (uint16_t)(lower + rho >= 0x10000u ? upper + 1u : upper);
}

/* One bfloat16 step as above, rounding each new value stochastically with
 * the bits of its node at step t.  node0 is the linear index of u[0] in the
 * array the bits are keyed to (0 for a whole array; a slab of planes
 * k0.. of a larger array has node0 = k0*nx*ny). */
void oracle_heat_sweep_bf16_sr(const uint16_t *u, uint16_t *un, long nx, long ny,
                               long nz, float r, uint64_t seed, uint64_t t, uint64_t node0)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float c = oracle_f32_from_bf16(u[p]);
                const float nsum =
                    ((oracle_f32_from_bf16(u[p - sx]) + oracle_f32_from_bf16(u[p + sx])) +
                     (oracle_f32_from_bf16(u[p - sy]) + oracle_f32_from_bf16(u[p + sy]))) +
                    (oracle_f32_from_bf16(u[p - sz]) + oracle_f32_from_bf16(u[p + sz]));
                const float lap = nsum - 6.0f * c;
                un[p] = oracle_bf16_sr_from_f32(c + r * lap,
                                                oracle_sr_bits(node0 + (uint64_t)p, t, seed));
            }
}

/* `steps` such steps; step s uses t = step0 + s. */
int oracle_heat_bf16_sr(uint16_t *u, long nx, long ny, long nz, float r, long steps,
                        uint64_t seed, uint64_t step0, uint64_t node0)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    uint16_t *w = (uint16_t *)malloc((size_t)n * sizeof(uint16_t));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(uint16_t));
    uint16_t *a = u, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_sweep_bf16_sr(a, b, nx, ny, nz, r, seed, step0 + (uint64_t)s, node0);
        uint16_t *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(uint16_t));
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Conjugate Gradient on the 7-point Laplacian                               */
/* ------------------------------------------------------------------------ */

/*
 * y = A x for the 7-point operator with zero Dirichlet data outside the box:
 * (A x)_p = 6 x_p - (((x- + x+) + (y- + y+)) + (z- + z+)), a neighbour that
 * falls outside [0,nx) x [0,ny) x [0,nz) counts as 0.  This is the SpMV of
 * the paper's CG case study (Pseudocode alg:spmv, one row per point) with
 * the 7-point stencil in place of the CSR arrays.
 */
void oracle_lap7_apply(const double *x, double *y, long nx, long ny, long nz)
{
    const long sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const double xm = (i > 0) ? x[p - 1] : 0.0;
                const double xp = (i < nx - 1) ? x[p + 1] : 0.0;
                const double ym = (j > 0) ? x[p - sy] : 0.0;
                const double yp = (j < ny - 1) ? x[p + sy] : 0.0;
                const double zm = (k > 0) ? x[p - sz] : 0.0;
                const double zp = (k < nz - 1) ? x[p + sz] : 0.0;
                const double nsum = ((xm + xp) + (ym + yp)) + (zm + zp);
                y[p] = 6.0 * x[p] - nsum;
            }
}

/* Neumaier-compensated running sum (value s, compensation c). */
static void neumaier_add(double *s, double *c, double v)
{
    const double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

/*
 * Dot product a.b in a fixed order that does not depend on the number of
 * threads: one compensated sum per z-plane (index order), then a compensated
 * sum of the plane sums in plane order.
 */
double oracle_dot(const double *a, const double *b, long nx, long ny, long nz)
{
    const long plane = nx * ny;
    double *part = (double *)malloc((size_t)nz * sizeof(double));
    if (!part)
        return NAN;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k) {
        double s = 0.0, c = 0.0;
        const double *pa = a + k * plane, *pb = b + k * plane;
        for (long q = 0; q < plane; ++q)
            neumaier_add(&s, &c, pa[q] * pb[q]);
        part[k] = s + c;
    }
    double s = 0.0, c = 0.0;
    for (long k = 0; k < nz; ++k)
        neumaier_add(&s, &c, part[k]);
    free(part);
    return s + c;
}

/*
 * Textbook (Hestenes-Stiefel) Conjugate Gradient for A x = b, the method of
 * the paper's CG case study (SpMV, dot products, vector updates; Saad 2003):
 *
 *   r = b - A x;  p = r;  rho = r.r
 *   loop:  q = A p;  alpha = rho / (p.q);  x += alpha p;  r -= alpha q;
 *          rho' = r.r;  stop if sqrt(rho') <= tol ||b||;
 *          beta = rho'/rho;  p = r + beta p;  rho = rho'
 *
 * `x` holds the initial guess on entry and the last iterate on return.
 * `hist` (optional, maxit+1 entries) receives ||r_k|| / ||b|| for k = 0..iters.
 * On return *iters is the number of completed iterations and *relres_true is
 * ||b - A x|| / ||b|| recomputed from x.
 * Returns 0 (converged), 1 (maxit reached), -4 (no memory),
 * -6 (p.q <= 0: breakdown), -7 (a scalar went non-finite).
 */
int oracle_cg(const double *b, double *x, long nx, long ny, long nz, double tol,
              long maxit, long *iters, double *relres_true, double *hist)
{
    const long n = nx * ny * nz;
    const size_t bytes = (size_t)n * sizeof(double);
    int status = 1;
    long it = 0;
    *iters = 0;
    *relres_true = 0.0;

    const double bnorm = sqrt(oracle_dot(b, b, nx, ny, nz));
    if (bnorm == 0.0) {
        memset(x, 0, bytes);
        if (hist)
            hist[0] = 0.0;
        return 0;
    }

    double *r = (double *)malloc(bytes), *p = (double *)malloc(bytes),
           *q = (double *)malloc(bytes);
    if (!r || !p || !q) {
        free(r);
        free(p);
        free(q);
        return -4;
    }

    oracle_lap7_apply(x, q, nx, ny, nz);
    for (long t = 0; t < n; ++t)
        r[t] = b[t] - q[t];
    memcpy(p, r, bytes);
    double rho = oracle_dot(r, r, nx, ny, nz);
    if (hist)
        hist[0] = sqrt(rho) / bnorm;

    const double t0 = omp_get_wtime();
    if (sqrt(rho) <= tol * bnorm) {
        status = 0;
    } else {
        while (it < maxit) {
            oracle_lap7_apply(p, q, nx, ny, nz);
            const double pq = oracle_dot(p, q, nx, ny, nz);
            if (!isfinite(pq)) {
                status = -7;
                break;
            }
            if (pq <= 0.0) {
                status = -6;
                break;
            }
            const double alpha = rho / pq;
            for (long t = 0; t < n; ++t) {
                x[t] = x[t] + alpha * p[t];
                r[t] = r[t] - alpha * q[t];
            }
            const double rho_new = oracle_dot(r, r, nx, ny, nz);
            ++it;
            if (hist)
                hist[it] = sqrt(rho_new) / bnorm;
            if (!isfinite(rho_new)) {
                status = -7;
                break;
            }
            if (sqrt(rho_new) <= tol * bnorm) {
                status = 0;
                break;
            }
            const double beta = rho_new / rho;
            for (long t = 0; t < n; ++t)
                p[t] = r[t] + beta * p[t];
            rho = rho_new;
        }
    }
    g_loop_seconds = omp_get_wtime() - t0;

    /* true residual b - A x */
    oracle_lap7_apply(x, q, nx, ny, nz);
    for (long t = 0; t < n; ++t)
        r[t] = b[t] - q[t];
    *relres_true = sqrt(oracle_dot(r, r, nx, ny, nz)) / bnorm;
    *iters = it;
    free(r);
    free(p);
    free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Mixed precision: binary32 inner CG inside binary64 iterative refinement  */
/* ------------------------------------------------------------------------ */

/* y = A x in binary32: 6 x_p - (((x- + x+) + (y- + y+)) + (z- + z+)), each
 * operation rounded to binary32, zero outside the box. */
void oracle_lap7_apply_f32(const float *x, float *y, long nx, long ny, long nz)
{
    const long sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float xm = (i > 0) ? x[p - 1] : 0.0f;
                const float xp = (i < nx - 1) ? x[p + 1] : 0.0f;
                const float ym = (j > 0) ? x[p - sy] : 0.0f;
                const float yp = (j < ny - 1) ? x[p + sy] : 0.0f;
                const float zm = (k > 0) ? x[p - sz] : 0.0f;
                const float zp = (k < nz - 1) ? x[p + sz] : 0.0f;
                const float nsum = ((xm + xp) + (ym + yp)) + (zm + zp);
                y[p] = 6.0f * x[p] - nsum;
            }
}

/* a.b of binary32 vectors, accumulated in binary64 (each product of two
 * binary32 values is exact in binary64), in the order of oracle_dot. */
double oracle_dot_f32(const float *a, const float *b, long nx, long ny, long nz)
{
    const long plane = nx * ny;
    double *part = (double *)malloc((size_t)nz * sizeof(double));
    if (!part)
        return NAN;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k) {
        double s = 0.0, c = 0.0;
        const float *pa = a + k * plane, *pb = b + k * plane;
        for (long q = 0; q < plane; ++q)
            neumaier_add(&s, &c, (double)pa[q] * (double)pb[q]);
        part[k] = s + c;
    }
    double s = 0.0, c = 0.0;
    for (long k = 0; k < nz; ++k)
        neumaier_add(&s, &c, part[k]);
    free(part);
    return s + c;
}

/*
 * Iterative refinement with a binary32 inner CG (the precision direction of
 * the CG case study: the inner solve moves half the bytes, while residuals,
 * solution updates and every dot product stay in binary64):
 *
 *   outer:  r = b - A x (binary64); stop if ||r|| <= tol ||b||;
 *           s = r rounded to binary32;
 *           d = CG in binary32 on A d = s from d = 0 (below);
 *           x = x + d (binary64)
 *   inner:  p = s; rho = s.s;
 *           loop:  q = A p (binary32);  alpha = rho / (p.q)  (binary64,
 *                  then rounded to binary32 for the updates);
 *                  d = d + alpha p;  s = s - alpha q  (binary32);
 *                  rho' = s.s;  stop if sqrt(rho') <= max(inner_tol sqrt(rho_0),
 *                  floor tol ||b||);  beta = rho'/rho (binary64, rounded);
 *                  p = s + beta p;  rho = rho'
 *
 * Dot products of binary32 vectors are accumulated in binary64.  The inner
 * stopping floor (`floor` times the outer target) keeps the last inner solve
 * from reducing the residual far below what the outer test needs.
 *
 * `x` holds the initial guess on entry and the last iterate on return.
 * *iters counts inner iterations over all outer steps (at most maxit);
 * *outer counts outer steps (inner solves); *relres_true is the binary64
 * ||b - A x|| / ||b|| of the returned x.  `inner_hist` (optional, up to
 * max_outer entries) receives the inner iteration count of each outer step.
 * Returns 0 (converged), 1 (maxit reached, or an outer step that did not
 * reduce ||r||), -4 (no memory), -6 (p.q <= 0 on an inner solve's first
 * iteration), -7 (a scalar went non-finite).
 */
int oracle_cg_ir(const double *b, double *x, long nx, long ny, long nz, double tol,
                 long maxit, double inner_tol, double floor_frac, long max_outer,
                 long *iters, long *outer, double *relres_true, long *inner_hist)
{
    const long n = nx * ny * nz;
    *iters = 0;
    *outer = 0;
    *relres_true = 0.0;
    const double bnorm = sqrt(oracle_dot(b, b, nx, ny, nz));
    if (bnorm == 0.0) {
        memset(x, 0, (size_t)n * sizeof(double));
        return 0;
    }
    double *r = (double *)malloc((size_t)n * sizeof(double));
    float *s = (float *)malloc((size_t)n * sizeof(float));
    float *d = (float *)malloc((size_t)n * sizeof(float));
    float *p = (float *)malloc((size_t)n * sizeof(float));
    float *q = (float *)malloc((size_t)n * sizeof(float));
    if (!r || !s || !d || !p || !q) {
        free(r); free(s); free(d); free(p); free(q);
        return -4;
    }
    int status = 1;
    long it = 0;
    double rprev = INFINITY;
    for (;;) {
        oracle_lap7_apply(x, r, nx, ny, nz);
        for (long t = 0; t < n; ++t)
            r[t] = b[t] - r[t];
        const double rnorm = sqrt(oracle_dot(r, r, nx, ny, nz));
        *relres_true = rnorm / bnorm;
        if (!isfinite(rnorm)) { status = -7; break; }
        if (rnorm <= tol * bnorm) { status = 0; break; }
        if (it >= maxit || *outer >= max_outer || rnorm >= rprev) { status = 1; break; }
        rprev = rnorm;

        /* inner solve in binary32 */
        for (long t = 0; t < n; ++t) {
            s[t] = (float)r[t];
            d[t] = 0.0f;
            p[t] = s[t];
        }
        double rho = oracle_dot_f32(s, s, nx, ny, nz);
        const double thresh = fmax(inner_tol * sqrt(rho), floor_frac * tol * bnorm);
        long inner = 0;
        int inner_status = 0;
        while (it < maxit) {
            oracle_lap7_apply_f32(p, q, nx, ny, nz);
            const double pq = oracle_dot_f32(p, q, nx, ny, nz);
            if (!isfinite(pq)) { inner_status = -7; break; }
            if (pq <= 0.0) { inner_status = -6; break; }
            const float alpha = (float)(rho / pq);
            for (long t = 0; t < n; ++t) {
                d[t] = d[t] + alpha * p[t];
                s[t] = s[t] - alpha * q[t];
            }
            const double rho_new = oracle_dot_f32(s, s, nx, ny, nz);
            ++it;
            ++inner;
            if (!isfinite(rho_new)) { inner_status = -7; break; }
            if (sqrt(rho_new) <= thresh) break;
            const float beta = (float)(rho_new / rho);
            for (long t = 0; t < n; ++t)
                p[t] = s[t] + beta * p[t];
            rho = rho_new;
        }
        if (inner_hist)
            inner_hist[*outer] = inner;
        *outer += 1;
        if (inner_status == -7) { status = -7; break; }
        if (inner_status == -6 && inner == 0) { status = -6; break; }
        for (long t = 0; t < n; ++t)
            x[t] = x[t] + (double)d[t];
    }
    *iters = it;
    free(r); free(s); free(d); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Heat equation, variable coefficient with a source (the paper's equation)  */
/* ------------------------------------------------------------------------ */

/*
 * One explicit step of Eq. (1), du/dt = div(kappa grad u) + f, by Eq. (4):
 *
 *   u_new = u + rhs + beta * (D_x + D_y + D_z),   rhs = dt f,  beta = dt/(2h^2)
 *
 * as the heat3d pseudocode stores it (its initialisation loop fills rhs with
 * dt*f and kappa per node; the step adds rhs and beta times the operator).
 * The paper does not spell out D_x.  It is read here as the conservative
 * (flux) difference whose face coefficient is the sum of the coefficients of
 * the face's two nodes, i.e. twice their arithmetic mean -- which is what the
 * 1/2 in beta compensates:
 *
 *   D_x = (k[i] + k[i+1]) (u[i+1] - u[i]) - (k[i-1] + k[i]) (u[i] - u[i-1])
 *
 * and likewise along y and z.  With kappa constant it is 2 kappa times the
 * second difference, i.e. the constant-coefficient step with r = 2 kappa beta.
 * Evaluation order (fixed, no contraction): each D as written, then
 * L = (D_x + D_y) + D_z, then u_new = (u + rhs) + beta * L.  Boundary nodes
 * (the outermost layer) are Dirichlet nodes and are never written; kappa and
 * rhs are read only where the formula reads them.
 */
void oracle_heat_vk_sweep_f64(const double *u, const double *kap,
                              const double *rhs, double *un, long nx, long ny,
                              long nz, double beta)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const double c = u[p], kc = kap[p];
                const double dx = (kc + kap[p + sx]) * (u[p + sx] - c) -
                                  (kap[p - sx] + kc) * (c - u[p - sx]);
                const double dy = (kc + kap[p + sy]) * (u[p + sy] - c) -
                                  (kap[p - sy] + kc) * (c - u[p - sy]);
                const double dz = (kc + kap[p + sz]) * (u[p + sz] - c) -
                                  (kap[p - sz] + kc) * (c - u[p - sz]);
                const double lop = (dx + dy) + dz;
                un[p] = (c + rhs[p]) + beta * lop;
            }
}

/*
 * `steps` variable-coefficient steps with ping-pong buffers and a swap after
 * each (the time loop of the heat3d pseudocode, with an integer step count).
 * kappa and rhs do not change between steps.  Returns 0, or -4 when out of
 * memory.
 */
int oracle_heat_vk_f64(double *u, const double *kap, const double *rhs,
                       long nx, long ny, long nz, double beta, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    double *w = (double *)malloc((size_t)n * sizeof(double));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(double));
    double *a = u, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_vk_sweep_f64(a, kap, rhs, b, nx, ny, nz, beta);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(double));
    free(w);
    return 0;
}

/* The same step in binary32 throughout (beta rounded to binary32 once). */
void oracle_heat_vk_sweep_f32(const float *u, const float *kap,
                              const float *rhs, float *un, long nx, long ny,
                              long nz, float beta)
{
    const long sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 1; k < nz - 1; ++k)
        for (long j = 1; j < ny - 1; ++j)
            for (long i = 1; i < nx - 1; ++i) {
                const long p = IDX(i, j, k, nx, ny);
                const float c = u[p], kc = kap[p];
                const float dx = (kc + kap[p + sx]) * (u[p + sx] - c) -
                                 (kap[p - sx] + kc) * (c - u[p - sx]);
                const float dy = (kc + kap[p + sy]) * (u[p + sy] - c) -
                                 (kap[p - sy] + kc) * (c - u[p - sy]);
                const float dz = (kc + kap[p + sz]) * (u[p + sz] - c) -
                                 (kap[p - sz] + kc) * (c - u[p - sz]);
                const float lop = (dx + dy) + dz;
                un[p] = (c + rhs[p]) + beta * lop;
            }
}

int oracle_heat_vk_f32(float *u, const float *kap, const float *rhs, long nx,
                       long ny, long nz, float beta, long steps)
{
    const long n = nx * ny * nz;
    if (steps <= 0)
        return 0;
    float *w = (float *)malloc((size_t)n * sizeof(float));
    if (!w)
        return -4;
    memcpy(w, u, (size_t)n * sizeof(float));
    float *a = u, *b = w;
    for (long s = 0; s < steps; ++s) {
        oracle_heat_vk_sweep_f32(a, kap, rhs, b, nx, ny, nz, beta);
        float *t = a;
        a = b;
        b = t;
    }
    if (a != u)
        memcpy(u, a, (size_t)n * sizeof(float));
    free(w);
    return 0;
}
