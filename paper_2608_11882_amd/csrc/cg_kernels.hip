// cg_kernels.hip -- Conjugate Gradient on the 7-point Laplacian for gfx950.
//
// The operator is A = 6 I - (face neighbours) with zero data outside the
// box; (A v)_p = 6 v_p - (((x- + x+) + (y- + y+)) + (z- + z+)), evaluated in
// that order without contraction.  CG is the textbook two-reduction form
// (the paper's CG case study: SpMV, dot products, vector updates):
//
//   direction:  p' = r + beta p   (p' = r on the first iteration),
//               q  = A p' on the fly, partial sums of p'.q
//               -> last block: alpha = rho / (p'.q)
//   update:     x += alpha p',  r -= alpha (A p') recomputed from p',
//               partial sums of r.r
//               -> last block: rho' , convergence test, beta = rho'/rho
//
// A p' is never stored: the direction kernel builds p' at the neighbours
// from r and p (the same expression, so the same bits as the value stored
// there), and the update kernel recomputes A p' from p'.  Each iteration
// therefore moves 64 bytes per unknown (r, p read + p' written; x, r, p'
// read + x, r written), against 80 with a stored q.  The z-march is the one
// of the heat kernels: 64 x BY tiles, registers along z, LDS ring in x/y.
//
// Reductions are deterministic: every block reduces its own partial in a
// fixed tree; the last block to arrive (arrival ticket) adds the partials
// in index order and computes the scalars on the device, so no iteration
// needs the host, which only polls the convergence state between batches.

#include "hc_internal.hpp"

#include <climits>

namespace hc {
namespace {

constexpr int kBY = 4;                 // waves per block
constexpr int kThreads = 64 * kBY;
constexpr int kZDepth = 32;            // planes per z-block
constexpr int kLd = kTileX + 2;

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int kXcd = 8;
    const int xcd = bid % kXcd, slot = bid / kXcd;
    const int per = nblk / kXcd, rem = nblk % kXcd;
    return xcd * per + min(xcd, rem) + slot;
}

struct Tile {
    int tx, ty, kb, ke;
};

__device__ __forceinline__ Tile decode_tile(int nx, int ny, int nz) {
    const int ntx = (nx + kTileX - 1) / kTileX;
    const int nty = (ny + kBY - 1) / kBY;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    Tile t;
    t.tx = L % ntx;
    const int rest = L / ntx;
    t.ty = rest % nty;
    t.kb = (rest / nty) * kZDepth;
    t.ke = min(t.kb + kZDepth - 1, nz - 1);
    return t;
}

// Walk a 64 x kBY tile of the box through planes [kb, ke].
//
//  field.at(off)        value of the marched field at the in-box node `off`
//                       (every load is issued unconditionally at a clamped
//                       in-box address; nodes outside the box are then
//                       replaced by 0, the zero Dirichlet data)
//  epi.prefetch(off)    issue the loads the epilogue needs at the own node
//                       `off` of a plane (clamped offset), returned as Pre
//  epi.finish(ok, off, c, nsum, pre)  own node: field value c, the ordered
//                       sum of its six neighbours and the prefetched values;
//                       ok is false off the box
//
// As in the heat kernels no load sits under a branch, and a z-block of
// exactly kZDepth planes is fully unrolled so that the register queue along
// z is renamed rather than copied; kPF planes of field loads and one plane
// of epilogue loads stay in flight.  Shorter z-blocks take a plain loop.
constexpr int kPF = 2;

template <class Field, class Epi>
__device__ __forceinline__ void box_zmarch(int nx, int ny, int nz,
                                           const Tile &t, Field &field,
                                           Epi &epi) {
    constexpr int kRing = 2 * kTileX + 2 * kBY;
    static_assert(kThreads >= kRing, "one thread per ring node");
    using Pre = typename Epi::Pre;
    __shared__ double tile[(kBY + 2) * kLd];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int i0 = t.tx * kTileX, j0 = t.ty * kBY;
    const int i = i0 + lane, j = j0 + w;
    const long long plane = (long long)nx * ny;

    const bool own_in = (i < nx) && (j < ny);
    const long long own = (long long)min(j, ny - 1) * nx + min(i, nx - 1);
    const int own_slot = (w + 1) * kLd + lane + 1;

    const int e = threadIdx.x;
    int ri, rj, rslot;
    if (e < kTileX) {
        ri = i0 + e; rj = j0 - 1; rslot = e + 1;
    } else if (e < 2 * kTileX) {
        ri = i0 + e - kTileX; rj = j0 + kBY; rslot = (kBY + 1) * kLd + (e - kTileX) + 1;
    } else if (e < 2 * kTileX + kBY) {
        ri = i0 - 1; rj = j0 + (e - 2 * kTileX); rslot = (e - 2 * kTileX + 1) * kLd;
    } else if (e < kRing) {
        ri = i0 + kTileX; rj = j0 + (e - 2 * kTileX - kBY);
        rslot = (e - 2 * kTileX - kBY + 1) * kLd + kTileX + 1;
    } else {
        ri = i; rj = j; rslot = -1;
    }
    const bool ring_in = (ri >= 0) && (ri < nx) && (rj >= 0) && (rj < ny);
    const long long ring =
        (long long)max(0, min(rj, ny - 1)) * nx + max(0, min(ri, nx - 1));

    // value at plane k (clamped into the box, 0 outside)
    auto val = [&](int k, long long off, bool in) -> double {
        const int kc = max(0, min(k, nz - 1));
        const double v = field.at((long long)kc * plane + off);
        return (in && k >= 0 && k < nz) ? v : 0.0;
    };
    auto neighbours = [&](double zm, double zp) -> double {
        const double xm = tile[own_slot - 1];
        const double xp = tile[own_slot + 1];
        const double ym = tile[own_slot - kLd];
        const double yp = tile[own_slot + kLd];
        return ((xm + xp) + (ym + yp)) + (zm + zp);
    };
    const int kb = t.kb;

    if (t.ke - kb + 1 == kZDepth) {
        double q[kZDepth + 2];  // q[s]: field at plane kb-1+s of the column
        double rgv[kZDepth];    // ring values of plane kb+s
        Pre pre[kZDepth];
#pragma unroll
        for (int s = 0; s < kPF + 2; ++s) q[s] = val(kb - 1 + s, own, own_in);
#pragma unroll
        for (int s = 0; s < kPF; ++s) rgv[s] = val(kb + s, ring, ring_in);
        pre[0] = epi.prefetch((long long)kb * plane + own);
#pragma unroll
        for (int s = 0; s < kZDepth; ++s) {
            const long long kp = (long long)(kb + s) * plane;
            __syncthreads();
            tile[own_slot] = q[s + 1];
            if (rslot >= 0) tile[rslot] = rgv[s];
            if (s + kPF < kZDepth) rgv[s + kPF] = val(kb + s + kPF, ring, ring_in);
            if (s + 1 < kZDepth) pre[s + 1] = epi.prefetch(kp + plane + own);
            __syncthreads();
            epi.finish(own_in, kp + own, q[s + 1], neighbours(q[s], q[s + 2]), pre[s]);
            if (s + 2 + kPF <= kZDepth + 1) q[s + 2 + kPF] = val(kb + s + 1 + kPF, own, own_in);
        }
        return;
    }

    double zm = val(kb - 1, own, own_in);
    double c = val(kb, own, own_in);
    double zp = val(kb + 1, own, own_in);
    double rc = val(kb, ring, ring_in);
    for (int k = kb; k <= t.ke; ++k) {
        const long long kp = (long long)k * plane;
        const double nn = val(k + 2, own, own_in);
        const double rn = val(min(k + 1, t.ke), ring, ring_in);
        const Pre pr = epi.prefetch(kp + own);
        __syncthreads();
        tile[own_slot] = c;
        if (rslot >= 0) tile[rslot] = rc;
        __syncthreads();
        epi.finish(own_in, kp + own, c, neighbours(zm, zp), pr);
        zm = c;
        c = zp;
        zp = nn;
        rc = rn;
    }
}

// Fixed-order block sum; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

__device__ __forceinline__ void store_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_state(const CGScalars *sc) {
    return __hip_atomic_load(&sc->state, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this block's partials; true in the block that arrives last, after
// which every block's partials are visible to it.
__device__ __forceinline__ bool arrive(CGScalars *sc, double *partial,
                                       int nsum, const double *vals) {
    __shared__ unsigned last;
    if (threadIdx.x == 0) {
        for (int q = 0; q < nsum; ++q)
            store_agent(&partial[(long long)blockIdx.x * nsum + q], vals[q]);
        __threadfence();
        const unsigned t = atomicAdd(&sc->ticket, 1u);
        last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

// In the last block: fixed-order sum of partial[b*nsum + q] over blocks b.
__device__ __forceinline__ double gather(const double *partial, int nsum,
                                         int q) {
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kThreads)
        t += load_agent(&partial[(long long)b * nsum + q]);
    return block_sum(t);
}

__global__ __launch_bounds__(64) void cg_init(CGScalars *sc, double tol) {
    if (threadIdx.x == 0) {
        sc->rho = 0.0;
        sc->pap = 0.0;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->bnorm2 = 0.0;
        sc->tol = tol;
        sc->thresh = 0.0;
        sc->rtrue2 = 0.0;
        sc->iter = 0;
        sc->state = 0;
        sc->ticket = 0u;
    }
}

struct NoPre {};

struct PlainField {
    const double *__restrict__ x;
    __device__ double at(long long o) const { return x[o]; }
};

// p' = r + beta p (p' = r on the first iteration)
struct DirectionField {
    const double *__restrict__ r;
    const double *__restrict__ p;
    double beta;
    int first;
    __device__ double at(long long o) const {
        const double ro = r[o];
        const double po = p[o];
        return first ? ro : ro + beta * po;
    }
};

// mode 0: r = b - A x (stored), rho = r.r, b.b, threshold and state.
// mode 1: true residual only: rtrue2 = |b - A x|^2 (nothing stored).
struct ResidualEpi {
    struct Pre {
        double b;
    };
    const double *__restrict__ b;
    double *__restrict__ r;
    int store;
    double rr = 0.0, bb = 0.0;
    __device__ Pre prefetch(long long o) const { return Pre{b[o]}; }
    __device__ void finish(bool ok, long long o, double c, double nsum, Pre p) {
        const double bo = p.b;
        const double q = 6.0 * c - nsum;
        const double ro = bo - q;
        if (ok) {
            if (store) r[o] = ro;
            rr += ro * ro;
            bb += bo * bo;
        }
    }
};

__global__ __launch_bounds__(kThreads) void cg_residual_f64(
    const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *partial, CGScalars *sc, int nx, int ny,
    int nz, int mode) {
    const Tile t = decode_tile(nx, ny, nz);
    PlainField f{x};
    ResidualEpi epi{b, r, mode == 0 ? 1 : 0};
    box_zmarch(nx, ny, nz, t, f, epi);
    double v[2];
    v[0] = block_sum(epi.rr);
    v[1] = block_sum(epi.bb);
    if (arrive(sc, partial, 2, v)) {
        const double srr = gather(partial, 2, 0);
        const double sbb = gather(partial, 2, 1);
        if (threadIdx.x == 0) {
            if (mode == 0) {
                sc->rho = srr;
                sc->bnorm2 = sbb;
                sc->thresh = sc->tol * sqrt(sbb);
                if (!isfinite(srr) || !isfinite(sbb))
                    sc->state = -7;
                else
                    sc->state = (sqrt(srr) <= sc->thresh) ? 1 : 0;
            } else {
                sc->rtrue2 = srr;
            }
            sc->ticket = 0u;
        }
    }
}

struct DirectionEpi {
    using Pre = NoPre;
    double *__restrict__ pnew;
    double acc = 0.0;
    __device__ Pre prefetch(long long) const { return Pre{}; }
    __device__ void finish(bool ok, long long o, double c, double nsum, Pre) {
        const double q = 6.0 * c - nsum;
        if (ok) {
            __builtin_nontemporal_store(c, pnew + o);
            acc += c * q;
        }
    }
};

__global__ __launch_bounds__(kThreads) void cg_direction_f64(
    const double *__restrict__ r, const double *__restrict__ pold,
    double *__restrict__ pnew, double *partial, CGScalars *sc, int nx, int ny,
    int nz, int first) {
    if (load_state(sc) != 0) return;  // converged or failed: nothing to do
    const Tile t = decode_tile(nx, ny, nz);
    DirectionField f{r, first ? r : pold, first ? 0.0 : sc->beta, first};
    DirectionEpi epi{pnew};
    box_zmarch(nx, ny, nz, t, f, epi);
    double v[1];
    v[0] = block_sum(epi.acc);
    if (arrive(sc, partial, 1, v)) {
        const double pap = gather(partial, 1, 0);
        if (threadIdx.x == 0) {
            sc->pap = pap;
            if (!isfinite(pap))
                sc->state = -7;
            else if (pap <= 0.0)
                sc->state = -6;
            else
                sc->alpha = sc->rho / pap;
            sc->ticket = 0u;
        }
    }
}

// x += alpha p', r -= alpha A p', and r.r of the new residual
struct UpdateEpi {
    struct Pre {
        double x, r;
    };
    double *__restrict__ x;
    double *__restrict__ r;
    double alpha;
    double acc = 0.0;
    __device__ Pre prefetch(long long o) const { return Pre{x[o], r[o]}; }
    __device__ void finish(bool ok, long long o, double c, double nsum, Pre p) {
        const double q = 6.0 * c - nsum;
        const double xn = p.x + alpha * c;
        const double rn = p.r - alpha * q;
        if (ok) {
            x[o] = xn;
            r[o] = rn;
            acc += rn * rn;
        }
    }
};

__global__ __launch_bounds__(kThreads) void cg_update_f64(
    double *__restrict__ x, double *__restrict__ r,
    const double *__restrict__ p, double *partial, CGScalars *sc, int nx,
    int ny, int nz) {
    if (load_state(sc) != 0) return;
    const Tile t = decode_tile(nx, ny, nz);
    PlainField f{p};
    UpdateEpi epi{x, r, sc->alpha};
    box_zmarch(nx, ny, nz, t, f, epi);
    double v[1];
    v[0] = block_sum(epi.acc);
    if (arrive(sc, partial, 1, v)) {
        const double rho_new = gather(partial, 1, 0);
        if (threadIdx.x == 0) {
            sc->iter += 1;
            if (!isfinite(rho_new)) {
                sc->state = -7;
            } else {
                if (sqrt(rho_new) <= sc->thresh) sc->state = 1;
                sc->beta = rho_new / sc->rho;
                sc->rho = rho_new;
            }
            sc->ticket = 0u;
        }
    }
}

struct Lap7Epi {
    using Pre = NoPre;
    double *__restrict__ y;
    __device__ Pre prefetch(long long) const { return Pre{}; }
    __device__ void finish(bool ok, long long o, double c, double nsum, Pre) {
        if (ok) y[o] = 6.0 * c - nsum;
    }
};

__global__ __launch_bounds__(kThreads) void lap7_f64(
    const double *__restrict__ x, double *__restrict__ y, int nx, int ny,
    int nz) {
    const Tile t = decode_tile(nx, ny, nz);
    PlainField f{x};
    Lap7Epi epi{y};
    box_zmarch(nx, ny, nz, t, f, epi);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

long long cg_blocks(int nx, int ny, int nz) {
    const long long ntx = (nx + kTileX - 1) / kTileX;
    const long long nty = (ny + kBY - 1) / kBY;
    const long long nzb = (nz + kZDepth - 1) / kZDepth;
    return ntx * nty * nzb;
}

size_t cg_work_bytes(int nx, int ny, int nz) {
    const size_t n = (size_t)nx * ny * nz;
    const size_t vec = align256(n * sizeof(double));
    const size_t part = align256((size_t)cg_blocks(nx, ny, nz) * 2 * sizeof(double));
    return 3 * vec + part + align256(sizeof(CGScalars));
}

CGWork cg_work_carve(void *base, int nx, int ny, int nz) {
    const size_t n = (size_t)nx * ny * nz;
    const size_t vec = align256(n * sizeof(double));
    const size_t part = align256((size_t)cg_blocks(nx, ny, nz) * 2 * sizeof(double));
    char *c = static_cast<char *>(base);
    CGWork w;
    w.r = reinterpret_cast<double *>(c);
    w.p[0] = reinterpret_cast<double *>(c + vec);
    w.p[1] = reinterpret_cast<double *>(c + 2 * vec);
    w.partial = reinterpret_cast<double *>(c + 3 * vec);
    w.sc = reinterpret_cast<CGScalars *>(c + 3 * vec + part);
    return w;
}

static hipError_t grid_of(int nx, int ny, int nz, dim3 *g) {
    const long long nb = cg_blocks(nx, ny, nz);
    if (nb <= 0 || nb > INT_MAX) return hipErrorInvalidConfiguration;
    *g = dim3((unsigned)nb);
    return hipSuccess;
}

hipError_t launch_cg_init(const CGWork &w, double tol, hipStream_t s) {
    cg_init<<<1, 64, 0, s>>>(w.sc, tol);
    return hipGetLastError();
}

hipError_t launch_cg_residual(const double *b, const double *x,
                              const CGWork &w, int nx, int ny, int nz,
                              int store_r, hipStream_t s) {
    dim3 g;
    hipError_t e = grid_of(nx, ny, nz, &g);
    if (e != hipSuccess) return e;
    cg_residual_f64<<<g, kThreads, 0, s>>>(b, x, w.r, w.partial, w.sc, nx, ny,
                                           nz, store_r ? 0 : 1);
    return hipGetLastError();
}

hipError_t launch_cg_direction(const CGWork &w, int cur, int first, int nx,
                               int ny, int nz, hipStream_t s) {
    dim3 g;
    hipError_t e = grid_of(nx, ny, nz, &g);
    if (e != hipSuccess) return e;
    cg_direction_f64<<<g, kThreads, 0, s>>>(w.r, w.p[cur], w.p[cur ^ 1],
                                            w.partial, w.sc, nx, ny, nz, first);
    return hipGetLastError();
}

hipError_t launch_cg_update(double *x, const CGWork &w, int cur, int nx,
                            int ny, int nz, hipStream_t s) {
    dim3 g;
    hipError_t e = grid_of(nx, ny, nz, &g);
    if (e != hipSuccess) return e;
    cg_update_f64<<<g, kThreads, 0, s>>>(x, w.r, w.p[cur ^ 1], w.partial, w.sc,
                                         nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_lap7_f64(const double *x, double *y, int nx, int ny, int nz,
                           hipStream_t s) {
    dim3 g;
    hipError_t e = grid_of(nx, ny, nz, &g);
    if (e != hipSuccess) return e;
    lap7_f64<<<g, kThreads, 0, s>>>(x, y, nx, ny, nz);
    return hipGetLastError();
}

}  // namespace hc
