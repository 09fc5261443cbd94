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
// read + x, r written), against 80 with a stored q.
//
// The z-march is the heat kernels' one: tiles of 64*VEC*WX (x) by BY (y)
// nodes walk z-blocks of ZB planes with the column in registers and the
// plane in LDS with a one-node ring; loads are issued at clamped in-box
// addresses with out-of-box values replaced by the zero Dirichlet data, and
// full-depth z-blocks are unrolled so that loads stay in flight.
//
// Reductions are deterministic: every block reduces its own partial in a
// fixed tree and stores it with a plain store.  The iteration's two
// reductions are finished by the kernel that needs them: every block of the
// next kernel adds the previous kernel's partials in index order with the
// same tree (so all blocks hold the same bits), computes alpha or beta and
// the convergence test itself, and block 0 records the scalars.  A kernel
// boundary on one stream orders every store before every later load, so no
// fence and no arrival counter is needed inside the iteration: on gfx950 an
// agent-scope release writes back the XCD's L2 and serializes per block,
// which cost more than the sweep itself at a few thousand blocks.  No
// iteration needs the host, which only polls the convergence state between
// batches (after a one-block kernel that finishes the last reduction).  The
// residual kernels, run once per solve or restart, keep a last-block
// arrival ticket.

#include "hc_internal.hpp"

#include <climits>
#include <type_traits>

namespace hc {
namespace {

constexpr int kPF = 2;   // planes of field loads in flight
constexpr int kPFE = 1;  // planes ahead the epilogue's own loads are issued (Epi::kAhead)

// Block order: the hardware deals workgroups to the 8 XCDs round-robin; with
// g > 1, runs of g consecutive tiles (y-neighbours) are dealt to one XCD
// inside windows of 8g blocks (same scheme as the heat kernels).
__device__ __forceinline__ int block_order(int b, int nb, int g) {
    if (g <= 1) return b;
    const int win = 8 * g;
    const int w = b / win;
    if ((w + 1) * win > nb) return b;
    const int o = b - w * win;
    return w * win + (o & 7) * g + (o >> 3);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One access of N bytes as a single load or store.
template <int N> struct Raw;
template <> struct Raw<4> { using T = unsigned int; };
template <> struct Raw<8> { using T = u32x2; };
template <> struct Raw<16> { using T = u32x4; };

template <class T, int VEC>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T *o) {
    using R = typename Raw<VEC * sizeof(T)>::T;
    const R raw = *reinterpret_cast<const R *>(p);
    __builtin_memcpy(o, &raw, sizeof raw);
}

// Store VEC values.  With multi-node lanes the x-edge is a multiple of VEC,
// so a lane is either inside the box or wholly outside it; a lane outside
// stores into its own slot of a sink buffer instead, so no store sits under
// a branch.
template <class T, int VEC>
__device__ __forceinline__ void store_vec(T *__restrict__ p, const T *v, bool nt) {
    using R = typename Raw<VEC * sizeof(T)>::T;
    R raw;
    __builtin_memcpy(&raw, v, sizeof raw);
    if (nt)
        __builtin_nontemporal_store(raw, reinterpret_cast<R *>(p));
    else
        *reinterpret_cast<R *>(p) = raw;
}

// Address of a node: a uniform base (array + plane k, in scalar registers)
// plus the lane's 32-bit byte offset within the plane, the form the
// SGPR-base addressing of global loads and stores takes.  A plane is far
// below 4 GiB, so the offset fits.
template <class T>
__device__ __forceinline__ T *node(T *base, long long plane, int k, unsigned off) {
    return reinterpret_cast<T *>(
        reinterpret_cast<typename std::conditional<std::is_const<T>::value, const char, char>::type *>(
            base + (long long)k * plane) + off);
}

// Offsets are kept in nodes (own, ring) and, for the field's element type
// T, in bytes (own_b, ring_b).
template <class T, int VEC, int WX, int BY>
struct BoxGeom {
    static constexpr int TX = 64 * VEC * WX;
    static constexpr int LD = TX + 2;
    static constexpr int NT = 64 * WX * BY;
    static constexpr int RROW = TX / VEC;  // lanes per tile row
    static_assert(NT >= 2 * RROW + 2 * BY, "one thread per ring element");
    int kb, ke;
    long long plane, own, ring;  // ring: VEC-aligned offset of the ring load
    unsigned own_b, ring_b;      // the same in bytes within the plane
    bool in[VEC];     // own nodes inside the box
    bool lane_in;     // all own nodes inside the box
    bool rin[VEC];    // ring nodes inside the box
    // LDS slots (rows of [left ring][node 0 of every lane] ... [node VEC-1
    // of every lane][right ring]: a wavefront's LDS accesses touch
    // consecutive words); node e of a lane or row piece at slot + e * RROW
    int own_slot, rslot;
    int xm_slot, xp_slot;  // left neighbour of node 0, right one of node VEC-1
    bool rvec;
    int rsel;         // a column node's index within its aligned ring load

    __device__ __forceinline__ BoxGeom(int nx, int ny, int nz, int zdepth, int xcd) {
        const int ntx = (nx + TX - 1) / TX;
        const int nty = (ny + BY - 1) / BY;
        const int L = block_order(blockIdx.x, gridDim.x, xcd);
        const int ty = L % nty;
        const int rest = L / nty;
        const int tx = rest % ntx;
        kb = (rest / ntx) * zdepth;
        ke = min(kb + zdepth - 1, nz - 1);

        const int t = threadIdx.x;
        const int lane = t & 63, w = t >> 6;
        const int wy = w / WX, wx = w % WX;
        const int i0 = tx * TX, j0 = ty * BY;
        const int ia = i0 + (wx * 64 + lane) * VEC;
        const int j = j0 + wy;
        plane = (long long)nx * ny;
        own = (long long)min(j, ny - 1) * nx + min(ia, nx - VEC);
#pragma unroll
        for (int v = 0; v < VEC; ++v) in[v] = (ia + v < nx) && (j < ny);
        lane_in = in[VEC - 1];
        const int gl = wx * 64 + lane;  // lane within the tile row
        const int rowb = (wy + 1) * LD;
        own_slot = rowb + 1 + gl;
        xm_slot = gl == 0 ? rowb : own_slot - 1 + (VEC - 1) * RROW;
        xp_slot = gl == RROW - 1 ? rowb + TX + 1 : own_slot + 1;

        rvec = false;
        rslot = -1;
        rsel = 0;
        int ri = 0, rj = 0;
        if (t < 2 * RROW) {
            const int row = t / RROW, q = t % RROW;
            rj = row == 0 ? j0 - 1 : j0 + BY;
            ri = i0 + q * VEC;
            rslot = (row == 0 ? 0 : (BY + 1) * LD) + 1 + q;
            rvec = true;
#pragma unroll
            for (int v = 0; v < VEC; ++v) rin[v] = (rj >= 0) && (rj < ny) && (ri + v < nx);
            ri = min(ri, nx - VEC);
        } else if (t < 2 * RROW + 2 * BY) {
            const int q = t - 2 * RROW;
            const int row = q % BY, side = q / BY;
            ri = side == 0 ? i0 - 1 : i0 + TX;
            rj = j0 + row;
            rslot = (row + 1) * LD + (side == 0 ? 0 : TX + 1);
            rin[0] = (ri >= 0) && (ri < nx) && (rj < ny);
#pragma unroll
            for (int v = 1; v < VEC; ++v) rin[v] = false;
            ri = max(0, min(ri, nx - 1));
            rsel = ri % VEC;
            ri -= rsel;
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) rin[v] = false;
            ri = min(ia, nx - VEC);
            rj = j;
        }
        ring = (long long)max(0, min(rj, ny - 1)) * nx + ri;
        own_b = (unsigned)(own * (long long)sizeof(T));
        ring_b = (unsigned)(ring * (long long)sizeof(T));
    }
};

// Walk the block's tile through its z-block.
//
//  field.template fetch<V>(k, off, raw)  the loads behind V field values
//                        at the in-box node at byte offset `off` of plane k
//                        (clamped offsets; loads unconditional), into a
//                        Field::Raw<V>
//  field.template make<V>(raw, out)  the V values (type T) from them
//  epi.prefetch(k, off)  the epilogue's own loads for a plane, as Epi::Pre
//  epi.finish(ok, lane_in, k, off, sink, c, nsum, pre)  own nodes: field
//                        values, ordered neighbour sums (type T),
//                        prefetched values; ok[v] false off the box
//  gate()                called by every thread once the first planes'
//                        loads are out (the block's scalars, which `make`
//                        and `finish` may use, are formed meanwhile); the
//                        march ends at once, returning false, when it does
//
// ZPAD: the field's arrays carry one zero plane below plane 0 and one above
// plane nz-1, so planes -1 and nz are read from memory and no plane index
// is ever tested (a uniform test would let the compiler branch around the
// load, and a load under a branch makes it wait for every load in flight).
// UNROLL: take the unrolled path for full-depth z-blocks (false keeps the
// plain loop, for kernels that run once or twice per solve).
template <class T, int VEC, int WX, int BY, int ZB, bool ZPAD, bool UNROLL = true,
          bool EARLY = false, class Field, class Epi, class Gate>
__device__ __forceinline__ bool box_zmarch(int nx, int ny, int nz, int xcd, double *sink,
                                           Field &field, Epi &epi, Gate &gate) {
    using G = BoxGeom<T, VEC, WX, BY>;
    using Pre = typename Epi::Pre;
    using Raw = typename Field::template Raw<VEC>;
    static_assert(G::NT * VEC * sizeof(T) <= kSinkDoubles * sizeof(double),
                  "sink holds one slot per lane");
    __shared__ T tile[(BY + 2) * G::LD];
    const G g(nx, ny, nz, ZB, xcd);
    // a lane outside the box writes its own sink slot of VEC field values
    // (the epilogues store at most that many bytes per lane and vector)
    double *const lane_sink = reinterpret_cast<double *>(
        reinterpret_cast<char *>(sink) + (long long)threadIdx.x * VEC * sizeof(T));

    auto kclamp = [&](int k) { return ZPAD ? k : max(0, min(k, nz - 1)); };
    auto kinside = [&](int k) { return ZPAD || ((k >= 0) && (k < nz)); };
    // column values of plane k (0 outside the box)
    auto col_make = [&](int k, const Raw &raw, T *o) {
        T v[VEC];
        field.template make<VEC>(raw, v);
        const bool kin = kinside(k);
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = (kin && g.in[e]) ? v[e] : T(0);
    };
    auto col = [&](int k, T *o) {
        Raw raw;
        field.template fetch<VEC>(kclamp(k), g.own_b, raw);
        col_make(k, raw, o);
    };
    // one aligned VEC-wide load in every lane; a column node is picked out
    auto ring_make = [&](int k, const Raw &raw, T *o) {
        T v[VEC];
        field.template make<VEC>(raw, v);
        T sel = v[0];
#pragma unroll
        for (int e = 1; e < VEC; ++e) sel = (g.rsel == e) ? v[e] : sel;
        v[0] = sel;
        const bool kin = kinside(k);
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = (kin && g.rin[e]) ? v[e] : T(0);
    };
    auto ringv = [&](int k, T *o) {
        Raw raw;
        field.template fetch<VEC>(kclamp(k), g.ring_b, raw);
        ring_make(k, raw, o);
    };
    auto put = [&](const T *c, const T *rv) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) tile[g.own_slot + e * G::RROW] = c[e];
        if (g.rslot >= 0) {
            tile[g.rslot] = rv[0];
            if (g.rvec) {
#pragma unroll
                for (int e = 1; e < VEC; ++e) tile[g.rslot + e * G::RROW] = rv[e];
            }
        }
    };
    // x neighbours inside the lane come from its registers (the same values
    // the tile holds), the ones across lanes from the tile
    auto nsums = [&](const T *zm, const T *c, const T *zp, T *ns) {
        const T xm0 = tile[g.xm_slot];
        const T xpl = tile[g.xp_slot];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int sl = g.own_slot + e * G::RROW;
            const T xm = e == 0 ? xm0 : c[e - 1];
            const T xp = e == VEC - 1 ? xpl : c[e + 1];
            const T ym = tile[sl - G::LD];
            const T yp = tile[sl + G::LD];
            ns[e] = ((xm + xp) + (ym + yp)) + (zm[e] + zp[e]);
        }
    };
    const int kb = g.kb, ke = g.ke;

    if (UNROLL && ke - kb + 1 == ZB) {
        // Odd z-blocks march downward: a z-block then reads its halo plane
        // at the end of its march when the block below (same XCD, started
        // together) reads it as its own last plane, and at its start when
        // the block above does, so the halo reads tend to find the plane in
        // L2 instead of going back to memory.  (zm + zp is the same sum
        // either way, and the stencil has no other z order.)  pl(s): the
        // plane of queue slot s, the march's s-th column from its start.
        const bool down = ((kb / ZB) & 1) != 0;
        const int k0 = down ? ke + 1 : kb - 1, dz = down ? -1 : 1;
        auto pl = [&](int s) { return k0 + s * dz; };
        T q[ZB + 2][VEC];  // q[s]: column at plane pl(s)
        T rg[ZB][VEC];     // ring values of plane pl(s+1)
        Pre pre[ZB];
        {
            Raw q0[kPF + 2];
            if (!EARLY && !gate()) return false;
#pragma unroll
            for (int s = 0; s < kPF + 2; ++s)
                field.template fetch<VEC>(kclamp(pl(s)), g.own_b, q0[s]);
            if (EARLY && !gate()) return false;
#pragma unroll
            for (int s = 0; s < kPF + 2; ++s) col_make(pl(s), q0[s], q[s]);
        }
#pragma unroll
        for (int s = 0; s < kPF; ++s) ringv(pl(s + 1), rg[s]);
#pragma unroll
        for (int s = 0; s < Epi::kAhead && s < ZB; ++s) pre[s] = epi.prefetch(pl(s + 1), g.own_b);
#pragma unroll
        for (int s = 0; s < ZB; ++s) {
            __syncthreads();
            put(q[s + 1], rg[s]);
            if (s + kPF < ZB) ringv(pl(s + 1 + kPF), rg[s + kPF]);
            if (s + Epi::kAhead < ZB)
                pre[s + Epi::kAhead] = epi.prefetch(pl(s + 1 + Epi::kAhead), g.own_b);
            __syncthreads();
            T ns[VEC];
            nsums(q[s], q[s + 1], q[s + 2], ns);
            epi.finish(g.in, g.lane_in, pl(s + 1), g.own_b, lane_sink, q[s + 1], ns,
                       pre[s]);
            if (s + 2 + kPF <= ZB + 1) col(pl(s + 2 + kPF), q[s + 2 + kPF]);
        }
        return true;
    }

    if (!gate()) return false;
    T zm[VEC], c[VEC], zp[VEC], rc[VEC];
    col(kb - 1, zm);
    col(kb, c);
    col(kb + 1, zp);
    ringv(kb, rc);
    for (int k = kb; k <= ke; ++k) {
        T nn[VEC], rn[VEC];
        col(k + 2, nn);
        ringv(min(k + 1, ke), rn);
        const Pre pr = epi.prefetch(k, g.own_b);
        __syncthreads();
        put(c, rc);
        __syncthreads();
        T ns[VEC];
        nsums(zm, c, zp, ns);
        epi.finish(g.in, g.lane_in, k, g.own_b, lane_sink, c, ns, pr);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            zm[e] = c[e];
            c[e] = zp[e];
            zp[e] = nn[e];
            rc[e] = rn[e];
        }
    }
    return true;
}

// Fixed-order block sum; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[NT / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < NT / 64; ++q) s += red[q];
    __syncthreads();
    return s;
}

// block_sum with the result in every thread.
template <int NT>
__device__ __forceinline__ double block_sum_all(double v) {
    __shared__ double total;
    const double s = block_sum<NT>(v);
    if (threadIdx.x == 0) total = s;
    __syncthreads();
    const double t = total;
    __syncthreads();
    return t;
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
// Block 0 of a kernel may end the solve while later blocks of the same
// kernel start (every block would end it alike from the same partials).
__device__ __forceinline__ void store_state(CGScalars *sc, int v) {
    __hip_atomic_store(&sc->state, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The state read once per block, so that all of its wavefronts take the
// same branch even when block 0 changes it meanwhile.
__device__ __forceinline__ int block_state(const CGScalars *sc) {
    __shared__ int st;
    if (threadIdx.x == 0) st = load_state(sc);
    __syncthreads();
    return st;
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
template <int NT>
__device__ __forceinline__ double gather(const double *partial, int nsum, int q) {
    double t = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += NT)
        t += load_agent(&partial[(long long)b * nsum + q]);
    return block_sum<NT>(t);
}

// The same fixed-order sum of the nb partials a previous kernel stored,
// taken in every block of a later one (result in every thread), and the
// solve's state, read once for the block as block_state does.  A thread
// issues its loads of partials eight at a time, so the block waits about one
// memory latency per eight partials instead of one per partial (blocks on
// the other XCDs wrote most of them, so they come from beyond this XCD's
// L2); the adds keep the index order, so the sum's bits do not depend on
// the unrolling.
template <int NT>
__device__ __forceinline__ double sum_partials(const CGScalars *sc, const double *part, int nb,
                                               int *state) {
    __shared__ double total;
    __shared__ int st;
    // the state's load goes out first, to wait alongside the partials'
    const int s0 = threadIdx.x == 0 ? load_state(sc) : 0;
    double t = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * NT < nb; b += 8 * NT) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[b + q * NT];
#pragma unroll
        for (int q = 0; q < 8; ++q) t += v[q];
    }
    for (; b < nb; b += NT) t += part[b];
    if (threadIdx.x == 0) st = s0;
    // block_sum's first barrier orders the write of st before its reads
    const double s = block_sum<NT>(t);
    if (threadIdx.x == 0) total = s;
    __syncthreads();
    const double r = total;
    *state = st;
    __syncthreads();
    return r;
}

// Iteration k's direction scalars.  On the first iteration of a (re)start
// rho_k is the residual kernel's r.r and beta is 0; otherwise rho_k is the
// sum of the last update's partials (part_u), tested here for convergence
// and finiteness, and beta = rho_k / rho_(k-1).  rho_k goes to slot k&1 for
// the update and the next direction.  False when the solve is over.
template <int NT>
__device__ __forceinline__ bool direction_scalars(CGScalars *sc, const double *part_u, int nb,
                                                  int k, int first, double *beta) {
    if (first) {
        if (block_state(sc) != 0) return false;
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->rslot[k & 1] = sc->rho;
        *beta = 0.0;
        return true;
    }
    int st0;
    const double rho = sum_partials<NT>(sc, part_u, nb, &st0);
    if (st0 != 0) return false;
    const double rho_old = sc->rslot[(k + 1) & 1];
    int state = 0;
    if (!isfinite(rho))
        state = -7;
    else if (sqrt(rho) <= sc->thresh)
        state = 1;
    const double b = rho / rho_old;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rslot[k & 1] = rho;
        sc->rho = rho;
        if (state == 0) sc->beta = b;
        if (state != 0) store_state(sc, state);
    }
    *beta = b;
    return state == 0;
}

// Iteration k's step length alpha = rho_k / (p'.Ap'), p'.Ap' the sum of the
// direction's partials (part_d); breakdown (<= 0) and non-finite values end
// the solve.  Counts the iteration (iter = k + 1) when it goes on.
template <int NT>
__device__ __forceinline__ bool update_scalars(CGScalars *sc, const double *part_d, int nb,
                                               int k, double *alpha) {
    int st0;
    const double pap = sum_partials<NT>(sc, part_d, nb, &st0);
    if (st0 != 0) return false;
    const double rho = sc->rslot[k & 1];
    int state = 0;
    if (!isfinite(pap))
        state = -7;
    else if (pap <= 0.0)
        state = -6;
    const double a = rho / pap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pap = pap;
        if (state == 0) {
            sc->alpha = a;
            sc->aslot[k & 3] = a;
            sc->iter = k + 1;
        } else {
            store_state(sc, state);
        }
    }
    *alpha = a;
    return state == 0;
}

__global__ __launch_bounds__(64) void cg_init(CGScalars *sc, double tol, double inner_tol,
                                              double floor_frac) {
    if (threadIdx.x == 0) {
        sc->rho = 0.0;
        sc->pap = 0.0;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->bnorm2 = 0.0;
        sc->tol = tol;
        sc->thresh = 0.0;
        sc->rtrue2 = 0.0;
        sc->inner_tol = inner_tol;
        sc->floor_frac = floor_frac;
        sc->iter = 0;
        sc->state = 0;
        sc->ticket = 0u;
    }
}

template <class T>
struct PlainField {
    const T *__restrict__ x;
    long long plane;
    template <int V>
    struct Raw {
        T x[V];
    };
    template <int V>
    __device__ void fetch(int k, unsigned off, Raw<V> &o) const {
        load_vec<T, V>(node(x, plane, k, off), o.x);
    }
    template <int V>
    __device__ void make(const Raw<V> &o, T *out) const {
#pragma unroll
        for (int e = 0; e < V; ++e) out[e] = o.x[e];
    }
};

// p' = r + beta p (p' = r on the first iteration)
template <class T>
struct DirectionField {
    const T *__restrict__ r;
    const T *__restrict__ p;
    long long plane;
    T beta;
    int first;
    template <int V>
    struct Raw {
        T r[V], p[V];
    };
    template <int V>
    __device__ void fetch(int k, unsigned off, Raw<V> &o) const {
        load_vec<T, V>(node(r, plane, k, off), o.r);
        load_vec<T, V>(node(p, plane, k, off), o.p);
    }
    template <int V>
    __device__ void make(const Raw<V> &o, T *out) const {
#pragma unroll
        for (int e = 0; e < V; ++e) out[e] = first ? o.r[e] : o.r[e] + beta * o.p[e];
    }
};

// The gate of kernels whose march needs no scalars.
struct Open {
    __device__ bool operator()() const { return true; }
};

struct NoPre {
    int unused;
};

// out = b - A x, with r.r and b.b
// (b is loaded where it is used: this kernel runs once or twice per solve
// and is not worth the registers of a prefetch)
template <int VEC>
struct ResidualEpi {
    using Pre = NoPre;
    static constexpr int kAhead = kPFE;
    const double *__restrict__ b;
    double *__restrict__ r;
    long long plane;
    double rr = 0.0, bb = 0.0;
    __device__ Pre prefetch(int, unsigned) const { return Pre{0}; }
    __device__ void finish(const bool *ok, bool lane_in, int k, unsigned off, double *sink,
                           const double *c, const double *ns, const Pre &) {
        double bo[VEC], ro[VEC];
        load_vec<double, VEC>(node(b, plane, k, off), bo);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const double q = 6.0 * c[e] - ns[e];
            ro[e] = bo[e] - q;
            if (ok[e]) {
                rr += ro[e] * ro[e];
                bb += bo[e] * bo[e];
            }
        }
        store_vec<double, VEC>(lane_in ? node(r, plane, k, off) : sink, ro, false);
    }
};

// Refinement residual: r = b - A x in binary64, its binary32 rounding s
// (the right-hand side of the inner solve) stored, and r.r, s.s, b.b
// accumulated in binary64.
template <int VEC>
struct IRResidualEpi {
    using Pre = NoPre;
    static constexpr int kAhead = kPFE;
    const double *__restrict__ b;
    float *__restrict__ s;
    long long plane;
    double rr = 0.0, ss = 0.0, bb = 0.0;
    __device__ Pre prefetch(int, unsigned) const { return Pre{0}; }
    __device__ void finish(const bool *ok, bool lane_in, int k, unsigned off, double *sink,
                           const double *c, const double *ns, const Pre &) {
        double bo[VEC];
        float so[VEC];
        load_vec<double, VEC>(node(b, plane, k, off), bo);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const double q = 6.0 * c[e] - ns[e];
            const double r = bo[e] - q;
            so[e] = (float)r;
            if (ok[e]) {
                rr += r * r;
                ss += (double)so[e] * (double)so[e];
                bb += bo[e] * bo[e];
            }
        }
        // off is a byte offset into binary64 planes; s holds binary32
        store_vec<float, VEC>(lane_in ? node(s, plane, k, off / 2) : reinterpret_cast<float *>(sink),
                              so, false);
    }
};

template <class T, int VEC>
struct DirectionEpi {
    using Pre = NoPre;
    static constexpr int kAhead = kPFE;
    T *__restrict__ pnew;
    long long plane;
    double acc = 0.0;
    __device__ Pre prefetch(int, unsigned) const { return Pre{0}; }
    __device__ void finish(const bool *ok, bool lane_in, int k, unsigned off, double *sink,
                           const T *c, const T *ns, const Pre &) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T q = T(6) * c[e] - ns[e];
            if (ok[e]) acc += (double)c[e] * (double)q;
        }
        store_vec<T, VEC>(lane_in ? node(pnew, plane, k, off) : reinterpret_cast<T *>(sink), c,
                          true);
    }
};

// How an update kernel treats x.  x is not needed by the iteration itself
// (only r and p are), so its steps can wait and be applied several at a
// time: with XM steps at a time x is read and written every XM-th iteration,
// at the cost of XM-1 more reads of direction vectors then (binary64: 34
// instead of 40 bytes per unknown and iteration on average at XM = 4, 36 at
// XM = 2).  The steps are added one after the other, in iteration order, so
// x takes the same values as with one step per iteration.
//
// XM: 0 updates r only (this iteration's step on x waits); 2 or 4 first
// applies the waiting steps of iterations k-XM+1 .. k-1, then this one's.
template <class T, int VEC, int XM>
struct UpdateEpi {
    static_assert(XM == 0 || XM == 2 || XM == 4, "x steps: 0, 2 or 4");
    static constexpr int NP = XM > 1 ? XM - 1 : 1;  // earlier direction vectors read
    // the four-step form has five loads of its own per plane: they go out
    // two planes ahead (measured 0.5% faster per iteration than one)
    static constexpr int kAhead = XM == 4 ? 2 : kPFE;
    struct Pre {
        T x[XM ? VEC : 1], r[VEC], pp[NP][XM ? VEC : 1];
    };
    T *__restrict__ x;
    T *__restrict__ r;
    const T *__restrict__ pprev[3];  // p_(k-1), p_(k-2), p_(k-3)
    long long plane;
    T alpha;
    T aprev[3];  // alpha_(k-1), alpha_(k-2), alpha_(k-3)
    double acc = 0.0;
    __device__ Pre prefetch(int k, unsigned off) const {
        Pre p;
        if (XM) load_vec<T, VEC>(node(x, plane, k, off), p.x);
        load_vec<T, VEC>(node(r, plane, k, off), p.r);
        if (XM) {
#pragma unroll
            for (int i = 0; i < NP; ++i) load_vec<T, VEC>(node(pprev[i], plane, k, off), p.pp[i]);
        }
        return p;
    }
    __device__ void finish(const bool *ok, bool lane_in, int k, unsigned off, double *sink,
                           const T *c, const T *ns, const Pre &p) {
        T xn[VEC], rn[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T q = T(6) * c[e] - ns[e];
            if (XM) {
                T xv = p.x[e];
#pragma unroll
                for (int i = NP - 1; i >= 0; --i) xv = xv + aprev[i] * p.pp[i][e];
                xn[e] = xv + alpha * c[e];
            }
            rn[e] = p.r[e] - alpha * q;
            if (ok[e]) acc += (double)rn[e] * (double)rn[e];
        }
        T *const sk = reinterpret_cast<T *>(sink);
        if (XM) store_vec<T, VEC>(lane_in ? node(x, plane, k, off) : sk, xn, false);
        store_vec<T, VEC>(lane_in ? node(r, plane, k, off) : sk, rn, false);
    }
};

template <class T, int VEC>
struct Lap7Epi {
    using Pre = NoPre;
    static constexpr int kAhead = kPFE;
    T *__restrict__ y;
    long long plane;
    __device__ Pre prefetch(int, unsigned) const { return Pre{0}; }
    __device__ void finish(const bool *ok, bool lane_in, int k, unsigned off, double *sink,
                           const T *c, const T *ns, const Pre &) {
        (void)ok;
        T out[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) out[e] = T(6) * c[e] - ns[e];
        store_vec<T, VEC>(lane_in ? node(y, plane, k, off) : reinterpret_cast<T *>(sink), out,
                          false);
    }
};

// mode 0: r = b - A x, rho = r.r, b.b, threshold and state.
// mode 1: the true residual |b - A x|^2 of the current x; the vector b - A x
//         goes to `r`, which the driver then points at a dead direction
//         buffer (a restart rebuilds both r and p).
template <int VEC, int WX, int BY, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void cg_residual_f64(
    const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *partial, CGScalars *sc, int nx, int ny,
    int nz, int xcd, double *sink, int mode) {
    constexpr int NT = 64 * WX * BY;
    const long long plane = (long long)nx * ny;
    PlainField<double> f{x, plane};
    ResidualEpi<VEC> epi{b, r, plane};
    Open open;
    box_zmarch<double, VEC, WX, BY, ZB, false, false>(nx, ny, nz, xcd, sink, f, epi, open);
    double v[2];
    v[0] = block_sum<NT>(epi.rr);
    v[1] = block_sum<NT>(epi.bb);
    if (arrive(sc, partial, 2, v)) {
        const double srr = gather<NT>(partial, 2, 0);
        const double sbb = gather<NT>(partial, 2, 1);
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

// Refinement step: r = b - A x (binary64), s = r rounded to binary32 for
// the inner solve.  Outer test ||r|| <= tol ||b|| (state 1); otherwise the
// inner solve starts with rho = s.s and stops at
// max(inner_tol sqrt(rho), floor tol ||b||) (state 0).
template <int VEC, int WX, int BY, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void cg_ir_residual(
    const double *__restrict__ b, const double *__restrict__ x, float *__restrict__ s,
    double *partial, CGScalars *sc, int nx, int ny, int nz, int xcd, double *sink) {
    constexpr int NT = 64 * WX * BY;
    const long long plane = (long long)nx * ny;
    PlainField<double> f{x, plane};
    IRResidualEpi<VEC> epi{b, s, plane};
    Open open;
    box_zmarch<double, VEC, WX, BY, ZB, false, false>(nx, ny, nz, xcd, sink, f, epi, open);
    double v[3];
    v[0] = block_sum<NT>(epi.rr);
    v[1] = block_sum<NT>(epi.ss);
    v[2] = block_sum<NT>(epi.bb);
    if (arrive(sc, partial, 3, v)) {
        const double srr = gather<NT>(partial, 3, 0);
        const double sss = gather<NT>(partial, 3, 1);
        const double sbb = gather<NT>(partial, 3, 2);
        if (threadIdx.x == 0) {
            sc->rtrue2 = srr;
            sc->bnorm2 = sbb;
            const double target = sc->tol * sqrt(sbb);
            if (!isfinite(srr) || !isfinite(sss) || !isfinite(sbb)) {
                sc->state = -7;
            } else if (sqrt(srr) <= target) {
                sc->state = 1;
            } else {
                sc->rho = sss;
                sc->thresh = fmax(sc->inner_tol * sqrt(sss), sc->floor_frac * target);
                sc->state = 0;
            }
            sc->ticket = 0u;
        }
    }
}

// Iteration k (k = iterations completed before it).  partial: the
// direction's partials at [0, nb), the update's at [nb, 2 nb).
template <class T, int VEC, int WX, int BY, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void cg_direction(
    const T *__restrict__ r, const T *__restrict__ pold, T *__restrict__ pnew, double *partial,
    CGScalars *sc, int nx, int ny, int nz, int xcd, double *sink, int first, int k) {
    constexpr int NT = 64 * WX * BY;
    const int nb = (int)gridDim.x;
    const long long plane = (long long)nx * ny;
    DirectionField<T> f{r, first ? r : pold, plane, T(0), first};
    DirectionEpi<T, VEC> epi{pnew, plane};
    // beta is formed while the first planes' loads are out
    auto gate = [&]() {
        double beta;
        if (!direction_scalars<NT>(sc, partial + nb, nb, k, first, &beta)) return false;
        f.beta = first ? T(0) : (T)beta;
        return true;
    };
    if (!box_zmarch<T, VEC, WX, BY, ZB, true, true, true>(nx, ny, nz, xcd, sink, f, epi, gate))
        return;
    const double v = block_sum<NT>(epi.acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// p1, p2, p3: p_(k-1), p_(k-2), p_(k-3), read as UpdateEpi<XM> needs
// (their alphas are in slots (k-i) & 3).
template <class T, int VEC, int WX, int BY, int ZB, int XM>
__global__ __launch_bounds__(64 * WX * BY) void cg_update(
    T *__restrict__ x, T *__restrict__ r, const T *__restrict__ p, const T *p1, const T *p2,
    const T *p3, double *partial, CGScalars *sc, int nx, int ny, int nz, int xcd, double *sink,
    int k) {
    constexpr int NT = 64 * WX * BY;
    const int nb = (int)gridDim.x;
    const long long plane = (long long)nx * ny;
    PlainField<T> f{p, plane};
    UpdateEpi<T, VEC, XM> epi{x, r, {p1, p2, p3}, plane, T(0), {T(0), T(0), T(0)}};
    // alpha is formed while the first planes' loads are out
    auto gate = [&]() {
        double alpha;
        if (!update_scalars<NT>(sc, partial, nb, k, &alpha)) return false;
        epi.alpha = (T)alpha;
        if (XM) {
#pragma unroll
            for (int i = 0; i < UpdateEpi<T, VEC, XM>::NP; ++i)
                epi.aprev[i] = (T)sc->aslot[(k - 1 - i) & 3];
        }
        return true;
    };
    if (!box_zmarch<T, VEC, WX, BY, ZB, true>(nx, ny, nz, xcd, sink, f, epi, gate)) return;
    const double v = block_sum<NT>(epi.acc);
    if (threadIdx.x == 0) partial[nb + blockIdx.x] = v;
}

// One block of the same thread count: finish the last update's reduction
// (the next direction kernel's scalars for iteration k) so that the host
// sees the convergence state.  The direction kernel repeats it with the
// same result.
template <int NT>
__global__ __launch_bounds__(NT) void cg_settle(CGScalars *sc, const double *partial, int nb,
                                                int k) {
    double beta;
    (void)direction_scalars<NT>(sc, partial + nb, nb, k, 0, &beta);
}

template <class T, int VEC, int WX, int BY, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void lap7(
    const T *__restrict__ x, T *__restrict__ y, int nx, int ny, int nz, int xcd, double *sink) {
    const long long plane = (long long)nx * ny;
    PlainField<T> f{x, plane};
    Lap7Epi<T, VEC> epi{y, plane};
    Open open;
    box_zmarch<T, VEC, WX, BY, ZB, false>(nx, ny, nz, xcd, sink, f, epi, open);
}

// x += d (binary64 += widened binary32), four nodes per thread
__global__ __launch_bounds__(256) void ir_axpy(double *__restrict__ x, const float *__restrict__ d,
                                               long long n) {
    const long long stride = (long long)gridDim.x * 256 * 4;
    for (long long i = ((long long)blockIdx.x * 256 + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n) {
#pragma unroll
            for (int e = 0; e < 4; ++e) x[i + e] = x[i + e] + (double)d[i + e];
        } else {
            for (long long e = i; e < n; ++e) x[e] = x[e] + (double)d[e];
        }
    }
}

// A step of x that waited: x += alpha_j p_j (alpha_j from slot j & 3), the
// operation the update kernels apply to x, node by node.
template <class T>
__global__ __launch_bounds__(256) void cg_xstep(T *__restrict__ x, const T *__restrict__ p,
                                                const CGScalars *sc, int j, long long n) {
    const T a = (T)sc->aslot[j & 3];
    const long long stride = (long long)gridDim.x * 256 * 2;
    for (long long i = ((long long)blockIdx.x * 256 + threadIdx.x) * 2; i < n; i += stride) {
        if (i + 2 <= n) {
            x[i] = x[i] + a * p[i];
            x[i + 1] = x[i + 1] + a * p[i + 1];
        } else {
            x[i] = x[i] + a * p[i];
        }
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// Every CG tile shape the library is built with (vec, wx, by, zdepth):
// binary64 vectors, and binary32 vectors of the refinement's inner solve.
#define HC_CG_SHAPES(X)                                                          \
    X(1, 1, 4, 16) X(1, 1, 4, 32) X(1, 4, 4, 16) X(2, 1, 4, 16) X(2, 1, 8, 16)   \
    X(2, 2, 4, 8) X(2, 2, 4, 16) X(2, 2, 4, 32) X(2, 2, 8, 8) X(2, 2, 8, 16)     \
    X(2, 2, 8, 32) X(2, 4, 4, 8) X(2, 4, 4, 16) X(2, 1, 16, 16)
#define HC_CG_SHAPES_F32(X)                                                      \
    X(1, 1, 4, 16) X(1, 4, 4, 16) X(2, 2, 8, 16) X(2, 2, 8, 32) X(2, 4, 4, 16)   \
    X(4, 1, 8, 16) X(4, 1, 8, 32) X(4, 2, 4, 16) X(4, 2, 4, 32) X(4, 2, 8, 16)   \
    X(4, 1, 16, 16) X(4, 4, 4, 16)

#define HC_CG_KEY(V, W, B, Z) (((V * 8 + W) * 32 + B) * 128 + Z)

bool cg_tiling_supported(const CGTiling &t) {
    const int key = HC_CG_KEY(t.vec, t.wx, t.by, t.zdepth);
#define HC_X(V, W, B, Z) if (key == HC_CG_KEY(V, W, B, Z)) return true;
    HC_CG_SHAPES(HC_X)
#undef HC_X
    return false;
}

bool cg_tiling_supported_f32(const CGTiling &t) {
    const int key = HC_CG_KEY(t.vec, t.wx, t.by, t.zdepth);
#define HC_X(V, W, B, Z) if (key == HC_CG_KEY(V, W, B, Z)) return true;
    HC_CG_SHAPES_F32(HC_X)
#undef HC_X
    return false;
}

long long cg_blocks(int nx, int ny, int nz, const CGTiling &t) {
    const long long tx = 64LL * t.vec * t.wx;
    return ((nx + tx - 1) / tx) * ((ny + t.by - 1) / t.by) *
           ((nz + t.zdepth - 1) / t.zdepth);
}

// Partial sums are sized for the smallest tile built (64 x 4 x 8), so one
// workspace serves every shape.
static long long max_blocks(int nx, int ny, int nz) {
    return ((nx + 63) / 64LL) * ((ny + 3) / 4LL) * ((nz + 7) / 8LL);
}

// r and the four direction vectors p0..p3 each carry a zero plane below and
// above the box (see ZPAD).
size_t cg_work_bytes(int nx, int ny, int nz) {
    const size_t plane = (size_t)nx * ny;
    const size_t vec = align256((size_t)(nz + 2) * plane * sizeof(double));
    const size_t part = align256((size_t)max_blocks(nx, ny, nz) * 2 * sizeof(double));
    return 5 * vec + part + align256(sizeof(CGScalars));
}

CGWork cg_work_carve(void *base, int nx, int ny, int nz) {
    const size_t plane = (size_t)nx * ny;
    const size_t vec = align256((size_t)(nz + 2) * plane * sizeof(double));
    const size_t part = align256((size_t)max_blocks(nx, ny, nz) * 2 * sizeof(double));
    char *c = static_cast<char *>(base);
    CGWork w;
    w.r = reinterpret_cast<double *>(c) + plane;
    for (int i = 0; i < 4; ++i) w.p[i] = reinterpret_cast<double *>(c + (1 + i) * vec) + plane;
    w.partial = reinterpret_cast<double *>(c + 5 * vec);
    w.sc = reinterpret_cast<CGScalars *>(c + 5 * vec + part);
    return w;
}

// Refinement workspace: s, p0, p1 (binary32, padded like above), d
// (binary32), three partial sums per block, the scalars.
size_t cg_ir_work_bytes(int nx, int ny, int nz) {
    const size_t plane = (size_t)nx * ny;
    const size_t vec = align256((size_t)(nz + 2) * plane * sizeof(float));
    const size_t part = align256((size_t)max_blocks(nx, ny, nz) * 3 * sizeof(double));
    return 4 * vec + part + align256(sizeof(CGScalars));
}

CGWorkF32 cg_ir_work_carve(void *base, int nx, int ny, int nz) {
    const size_t plane = (size_t)nx * ny;
    const size_t vec = align256((size_t)(nz + 2) * plane * sizeof(float));
    const size_t part = align256((size_t)max_blocks(nx, ny, nz) * 3 * sizeof(double));
    char *c = static_cast<char *>(base);
    CGWorkF32 w;
    w.r = reinterpret_cast<float *>(c) + plane;
    w.p[0] = reinterpret_cast<float *>(c + vec) + plane;
    w.p[1] = reinterpret_cast<float *>(c + 2 * vec) + plane;
    w.d = reinterpret_cast<float *>(c + 3 * vec) + plane;
    w.partial = reinterpret_cast<double *>(c + 4 * vec);
    w.sc = reinterpret_cast<CGScalars *>(c + 4 * vec + part);
    return w;
}

// Launch the kernel KER for the tile shape t out of the shape list LIST.
#define HC_CG_DISPATCH(LIST, KER)                                                 \
    do {                                                                          \
        const long long nb = cg_blocks(nx, ny, nz, t);                            \
        if (nb <= 0 || nb > INT_MAX) return hipErrorInvalidConfiguration;         \
        const dim3 grid((unsigned)nb), block(64 * t.wx * t.by);                   \
        (void)grid;                                                               \
        const int key = HC_CG_KEY(t.vec, t.wx, t.by, t.zdepth);                   \
        bool done = false;                                                        \
        LIST(HC_CG_ONE_##KER)                                                     \
        if (!done) return hipErrorInvalidValue;                                   \
        return hipGetLastError();                                                 \
    } while (0)

#define HC_CG_ONE_RES(V, W, B, Z)                                                 \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        cg_residual_f64<V, W, B, Z><<<grid, block, 0, s>>>(                       \
            b, x, store_r ? w.r : w.p[0], w.partial, w.sc, nx, ny, nz, t.xcd,     \
            sink, store_r ? 0 : 1);                                               \
        done = true;                                                              \
    }
#define HC_CG_ONE_IRRES(V, W, B, Z)                                               \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        cg_ir_residual<V, W, B, Z><<<grid, block, 0, s>>>(                        \
            b, x, w.r, w.partial, w.sc, nx, ny, nz, t.xcd, sink);                 \
        done = true;                                                              \
    }
// (the launchers name pold / pnew, the direction vectors p_(k-1) / p_k, and
// pp[0..2], p_(k-1) .. p_(k-3), for the update; XSTEPS is the update's x
// step count when it applies them)
#define HC_CG_ONE_DIR(V, W, B, Z)                                                 \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        cg_direction<ELEM, V, W, B, Z><<<grid, block, 0, s>>>(                    \
            w.r, pold, pnew, w.partial, w.sc, nx, ny, nz, t.xcd, sink, first, k); \
        done = true;                                                              \
    }
#define HC_CG_ONE_UPD(V, W, B, Z)                                                 \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        if (xsteps == 0)                                                          \
            cg_update<ELEM, V, W, B, Z, 0><<<grid, block, 0, s>>>(                \
                x, w.r, pnew, pp[0], pp[1], pp[2], w.partial, w.sc, nx, ny, nz,   \
                t.xcd, sink, k);                                                  \
        else                                                                      \
            cg_update<ELEM, V, W, B, Z, XSTEPS><<<grid, block, 0, s>>>(           \
                x, w.r, pnew, pp[0], pp[1], pp[2], w.partial, w.sc, nx, ny, nz,   \
                t.xcd, sink, k);                                                  \
        done = true;                                                              \
    }
#define HC_CG_ONE_SETTLE(V, W, B, Z)                                              \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        cg_settle<64 * W * B><<<1, block, 0, s>>>(w.sc, w.partial, (int)nb, k);   \
        done = true;                                                              \
    }
#define HC_CG_ONE_LAP(V, W, B, Z)                                                 \
    if (!done && key == HC_CG_KEY(V, W, B, Z)) {                                  \
        lap7<ELEM, V, W, B, Z><<<grid, block, 0, s>>>(x, y, nx, ny, nz, t.xcd,    \
                                                      sink);                      \
        done = true;                                                              \
    }

hipError_t launch_cg_init(CGScalars *sc, double tol, double inner_tol, double floor_frac,
                          hipStream_t s) {
    cg_init<<<1, 64, 0, s>>>(sc, tol, inner_tol, floor_frac);
    return hipGetLastError();
}

hipError_t launch_cg_residual(const double *b, const double *x, const CGWork &w,
                              int nx, int ny, int nz, int store_r,
                              const CGTiling &t, double *sink, hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES, RES);
}

hipError_t launch_cg_ir_residual(const double *b, const double *x, const CGWorkF32 &w, int nx,
                                 int ny, int nz, const CGTiling &t, double *sink,
                                 hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES, IRRES);
}

#define ELEM double
#define XSTEPS 4
hipError_t launch_cg_direction(const CGWork &w, int first, int k, int nx, int ny, int nz,
                               const CGTiling &t, double *sink, hipStream_t s) {
    const double *pold = w.p[(k - 1) & 3];
    double *pnew = w.p[k & 3];
    HC_CG_DISPATCH(HC_CG_SHAPES, DIR);
}

hipError_t launch_cg_update(double *x, const CGWork &w, int k, int xsteps, int nx, int ny,
                            int nz, const CGTiling &t, double *sink, hipStream_t s) {
    if (xsteps != 0 && xsteps != XSTEPS) return hipErrorInvalidValue;
    const double *pnew = w.p[k & 3];
    const double *pp[3] = {w.p[(k - 1) & 3], w.p[(k - 2) & 3], w.p[(k - 3) & 3]};
    HC_CG_DISPATCH(HC_CG_SHAPES, UPD);
}

hipError_t launch_cg_xstep(double *x, const double *p, const CGScalars *sc, int j, long long n,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 1023) / 1024;
    if (nb > 8192) nb = 8192;
    cg_xstep<double><<<(unsigned)nb, 256, 0, s>>>(x, p, sc, j, n);
    return hipGetLastError();
}

hipError_t launch_cg_settle(const CGWork &w, int k, int nx, int ny, int nz, const CGTiling &t,
                            hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES, SETTLE);
}

hipError_t launch_lap7_f64(const double *x, double *y, int nx, int ny, int nz,
                           const CGTiling &t, double *sink, hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES, LAP);
}
#undef XSTEPS
#undef ELEM

// The binary32 inner solve keeps two direction vectors (p[cur] the last,
// p[cur ^ 1] the one formed now) and takes d's steps two at a time.
#define ELEM float
#define XSTEPS 2
hipError_t launch_cg_direction_f32(const CGWorkF32 &w, int cur, int first, int k, int nx,
                                   int ny, int nz, const CGTiling &t, double *sink,
                                   hipStream_t s) {
    const float *pold = w.p[cur];
    float *pnew = w.p[cur ^ 1];
    HC_CG_DISPATCH(HC_CG_SHAPES_F32, DIR);
}

hipError_t launch_cg_update_f32(const CGWorkF32 &w, int cur, int k, int xstep, int nx, int ny,
                                int nz, const CGTiling &t, double *sink, hipStream_t s) {
    if (xstep != 0 && xstep != 1) return hipErrorInvalidValue;
    float *const x = w.d;
    const int xsteps = xstep ? XSTEPS : 0;
    const float *pnew = w.p[cur ^ 1];
    const float *pp[3] = {w.p[cur], nullptr, nullptr};
    HC_CG_DISPATCH(HC_CG_SHAPES_F32, UPD);
}

hipError_t launch_cg_xstep_f32(float *x, const float *p, const CGScalars *sc, int j, long long n,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 1023) / 1024;
    if (nb > 8192) nb = 8192;
    cg_xstep<float><<<(unsigned)nb, 256, 0, s>>>(x, p, sc, j, n);
    return hipGetLastError();
}

hipError_t launch_cg_settle_f32(const CGWorkF32 &w, int k, int nx, int ny, int nz,
                                const CGTiling &t, hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES_F32, SETTLE);
}

hipError_t launch_lap7_f32(const float *x, float *y, int nx, int ny, int nz, const CGTiling &t,
                           double *sink, hipStream_t s) {
    HC_CG_DISPATCH(HC_CG_SHAPES_F32, LAP);
}
#undef XSTEPS
#undef ELEM

hipError_t launch_ir_axpy(double *x, const float *d, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 1023) / 1024;
    if (nb > 8192) nb = 8192;
    ir_axpy<<<(unsigned)nb, 256, 0, s>>>(x, d, n);
    return hipGetLastError();
}

}  // namespace hc
