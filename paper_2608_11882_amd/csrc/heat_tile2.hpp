#pragma once

// heat_tile2.hpp -- two explicit steps of the 7-point heat update per pass
// over memory (temporal blocking of the z-marching tile), gfx950.  Device
// code only; not exported.
//
// A pass reads u^t and writes u^(t+2); u^(t+1) never leaves the chip.  A
// block owns a tile of VEC*TXL (x) by BY (y) nodes and a run of output
// planes [kb, ke].  Marching up in z, at plane k it
//   1. computes u^(t+1)(k) on the tile and on its one-node ring from the
//      staged u^t(k) (the ring is computed by the threads that load it, from
//      the staged plane and their own u^t(k-1), u^t(k+1)) and stages it;
//   2. computes u^(t+2)(k-1) on the tile from the staged u^(t+1)(k-1) and
//      the registers holding u^(t+1) at k-2, k-1, k, and stores it;
//   3. stages u^t(k+1) in LDS with a two-node ring (the tile, two rows and
//      two columns on each side, and the four corners of the inner ring).
// The u^t and u^(t+1) planes are both double-buffered, so one barrier per
// plane orders every LDS write after the reads of the plane before.
// Every value of u^(t+1) is evaluated with exactly the expression and
// rounding of a single step (heat_tile.hpp), stored values are rounded to
// the storage precision in between, so two steps here are bit-identical to
// two single steps.  The ring of u^(t+1) is computed by two neighbouring
// tiles alike (same inputs, same bits), and the planes just outside [kb, ke]
// by two neighbouring z-runs.
//
// A run of output planes is marched in sub-blocks of exactly ZB planes,
// each fully unrolled, with the register queues carried from one sub-block
// to the next, so the load pipeline fills once per run (the first sub-block
// starts early enough for the last to end at ke); runs shorter than ZB take
// sub-blocks of two planes (and one).  Loads are never
// predicated and are clamped into the array (rows, columns and planes); a
// value read at a clamped address only reaches nodes that are not updated.
// Nodes that are not updated (the Dirichlet layer, lanes past the last
// column or row) keep their value through both steps and are stored back
// unchanged, as in the single-step tile.  Stochastic rounding is not offered
// here (single steps only).

#include "heat_tile.hpp"

namespace hc {
namespace {

template <int VEC, int TXL, int BY>
struct TileGeom2 {
    static constexpr int TX = VEC * TXL;  // tile width in nodes
    static constexpr int LDU = TX + 4;    // row stride of the u^t plane
    static constexpr int LDA = TX + 2;    // row stride of a u^(t+1) plane
    static constexpr int NT = TXL * BY;
    static constexpr int R1N = 2 * TXL + 2 * BY;      // inner ring: rows, columns
    static constexpr int R2N = 2 * TXL + 2 * BY + 4;  // outer ring + inner corners
    static constexpr int U_ELEMS = (BY + 4) * LDU;
    static constexpr int A_ELEMS = (BY + 2) * LDA + 1;  // + one slot no thread reads
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(NT <= 1024, "at most 1024 threads per block");
    static_assert(NT >= R2N, "one thread per ring element");

    int kb, ke, nz;
    long long plane;
    // the lane's own VEC nodes (as in the single-step tile)
    long long own;
    bool st[VEC];
    int own_u, xm_u, xp_u;  // u^t plane: node 0 (node v: + v*TXL), x edges
    int own_a, xm_a, xp_a;  // u^(t+1) plane: the same
    // inner-ring element (u^(t+1) is computed there): a VEC-wide row piece
    // or one column node; threads past R1N hold none (r1on false)
    long long r1;           // aligned load offset
    bool r1on, r1vec;
    int r1sel;
    bool r1st[VEC];
    int r1_u, r1xm_u, r1xp_u;  // its slots in the u^t plane (node v: + v*TXL)
    int r1_a;                  // its slot in the u^(t+1) plane (sink if none)
    // outer-ring element (staged only): row piece, column node or corner
    long long r2;
    bool r2on, r2vec;
    int r2sel;
    int r2_u;

    // thread t of the block that sweeps tile (tx, ty), output planes kb_..ke_
    // (host-callable, so that the offsets can be checked on the CPU)
    __host__ __device__ TileGeom2(int t, int nx, int pitch, int ny, int nz_, int tx, int ty,
                                  int kb_, int ke_) {
        kb = kb_;
        ke = ke_;
        nz = nz_;
        const int gl = t % TXL, wy = t / TXL;
        const int i0 = tx * TX, j0 = 1 + ty * BY;
        const int ia = i0 + gl * VEC, j = j0 + wy;
        plane = (long long)pitch * ny;
        if (ia >= nx)
            own = (long long)(ny - 1) * pitch + (pitch - VEC);
        else
            own = (long long)min(j, ny - 1) * pitch + ia;
#pragma unroll
        for (int v = 0; v < VEC; ++v) st[v] = (ia + v >= 1) && (ia + v <= nx - 2) && (j <= ny - 2);
        {
            const int rb = (wy + 2) * LDU;
            own_u = rb + 2 + gl;
            xm_u = gl == 0 ? rb + 1 : own_u - 1 + (VEC - 1) * TXL;
            xp_u = gl == TXL - 1 ? rb + 2 + TX : own_u + 1;
            const int ab = (wy + 1) * LDA;
            own_a = ab + 1 + gl;
            xm_a = gl == 0 ? ab : own_a - 1 + (VEC - 1) * TXL;
            xp_a = gl == TXL - 1 ? ab + 1 + TX : own_a + 1;
        }

        // inner ring: rows j0-1 and j0+BY (VEC-wide pieces), columns i0-1
        // and i0+TX (one node each)
        r1on = t < R1N;
        r1vec = false;
        r1sel = 0;
        r1 = own;
        r1_u = own_u;
        r1xm_u = xm_u;
        r1xp_u = xp_u;
        r1_a = A_ELEMS - 1;
#pragma unroll
        for (int v = 0; v < VEC; ++v) r1st[v] = false;
        if (t < 2 * TXL) {
            const int row = t / TXL, q = t % TXL;
            const int rj_u = row == 0 ? j0 - 1 : j0 + BY;  // >= 0
            const int rj = min(rj_u, ny - 1);
            const int ib = i0 + q * VEC;
            r1 = (long long)rj * pitch + min(ib, pitch - VEC);
            r1vec = true;
            const int rb = (row == 0 ? 1 : BY + 2) * LDU;
            r1_u = rb + 2 + q;
            r1xm_u = q == 0 ? rb + 1 : r1_u - 1 + (VEC - 1) * TXL;
            r1xp_u = q == TXL - 1 ? rb + 2 + TX : r1_u + 1;
            r1_a = (row == 0 ? 0 : BY + 1) * LDA + 1 + q;
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                r1st[v] = (ib + v >= 1) && (ib + v <= nx - 2) && (rj_u >= 1) && (rj_u <= ny - 2);
        } else if (t < R1N) {
            const int q = t - 2 * TXL;
            const int row = q % BY, side = q / BY;
            const int ri_u = side == 0 ? i0 - 1 : i0 + TX;
            const int ri = max(0, min(ri_u, nx - 1));
            const int rj_u = j0 + row;
            r1sel = ri % VEC;
            r1 = (long long)min(rj_u, ny - 1) * pitch + (ri - r1sel);
            const int rb = (row + 2) * LDU;
            r1_u = rb + (side == 0 ? 1 : 2 + TX);
            r1xm_u = side == 0 ? rb : rb + 2 + (VEC - 1) * TXL + (TXL - 1);
            r1xp_u = side == 0 ? rb + 2 : rb + 3 + TX;
            r1_a = (row + 1) * LDA + (side == 0 ? 0 : 1 + TX);
            r1st[0] = (ri_u >= 1) && (ri_u <= nx - 2) && (rj_u <= ny - 2);
        }

        // outer ring: rows j0-2 and j0+BY+1, columns i0-2 and i0+TX+1, and
        // the corners of the inner ring
        r2on = t < R2N;
        r2vec = false;
        r2sel = 0;
        r2 = own;
        r2_u = own_u;
        if (t < 2 * TXL) {
            const int row = t / TXL, q = t % TXL;
            const int rj = row == 0 ? max(j0 - 2, 0) : min(j0 + BY + 1, ny - 1);
            r2 = (long long)rj * pitch + min(i0 + q * VEC, pitch - VEC);
            r2vec = true;
            r2_u = (row == 0 ? 0 : BY + 3) * LDU + 2 + q;
        } else if (t < 2 * TXL + 2 * BY) {
            const int q = t - 2 * TXL;
            const int row = q % BY, side = q / BY;
            const int ri = max(0, min(side == 0 ? i0 - 2 : i0 + TX + 1, nx - 1));
            r2sel = ri % VEC;
            r2 = (long long)min(j0 + row, ny - 1) * pitch + (ri - r2sel);
            r2_u = (row + 2) * LDU + (side == 0 ? 0 : 3 + TX);
        } else if (t < R2N) {
            const int c = t - 2 * TXL - 2 * BY;
            const int side = c & 1, top = c >> 1;
            const int rj = top == 0 ? j0 - 1 : min(j0 + BY, ny - 1);
            const int ri = max(0, min(side == 0 ? i0 - 1 : i0 + TX, nx - 1));
            r2sel = ri % VEC;
            r2 = (long long)rj * pitch + (ri - r2sel);
            r2_u = (top == 0 ? 1 : BY + 2) * LDU + (side == 0 ? 1 : 2 + TX);
        }
    }
};

// How one block sweeps its run of output planes [kb, ke] with z-blocks of
// zb planes: a march of m sub-blocks from plane `start`, then short runs
// over [rest, ke] (none when rest > ke).  A run of at least zb planes
// starts early enough for its last sub-block to end at ke, unless that
// would reach the Dirichlet plane 0; the planes it adds before kb are
// interior planes that other blocks (or the Boundary kernel) write with the
// same bits.  (Host-callable, so that the plan can be checked on the CPU.)
struct RunPlan {
    int start, m, rest;
};
__host__ __device__ inline RunPlan run_plan(int kb, int ke, int zb) {
    const int R = ke - kb + 1;
    if (R < zb) return {kb, 0, kb};
    const int m = (R + zb - 1) / zb;
    const int start = ke - m * zb + 1;
    if (start >= 1) return {start, m, ke + 1};
    return {kb, R / zb, kb + (R / zb) * zb};
}

// The tile and z-run of this block in a launch over table zt (see
// block_tile; the last z-block of a range is shifted back to zb_full).
//
// xcd < 0 selects slab order: the hardware deals workgroups to the 8 XCDs
// in turn (block id mod 8); XCD q gets the y-tiles [q S, (q+1) S) of every
// x-tile and z-run, S = ceil(nty / 8), and takes them x fastest, then y,
// then z-run, so the tiles one XCD runs side by side are neighbours in x
// and y and read their shared two-node rings through its L2 once.  A slot
// past the last y-tile holds an empty run (the block does nothing).
template <int VEC, int TXL, int BY>
__device__ __forceinline__ TileGeom2<VEC, TXL, BY> block_tile2(int nx, int ny, int nz,
                                                              const ZTable &zt, int ntx,
                                                              int nty, int xcd, int zb_full) {
    int tx, ty, z;
    if (xcd < 0) {
        const int S = (nty + 7) / 8;
        const int i = (int)(blockIdx.x >> 3);
        tx = i % ntx;
        const int rest = i / ntx;
        ty = (int)(blockIdx.x & 7) * S + rest % S;
        z = rest / S;
    } else {
        const int L = block_order(blockIdx.x, gridDim.x, xcd);
        ty = L % nty;
        const int rest = L / nty;
        tx = rest % ntx;
        z = rest / ntx;
    }
    int rg = 0;
    while (rg + 1 < zt.n && z >= zt.first[rg + 1]) ++rg;
    int k0 = zt.kb[rg] + (z - zt.first[rg]) * zt.depth[rg];
    if (zt.depth[rg] == zb_full && zt.ke[rg] - zt.kb[rg] + 1 >= zb_full)
        k0 = min(k0, zt.ke[rg] - zb_full + 1);
    const int k1 = ty < nty ? min(k0 + zt.depth[rg] - 1, zt.ke[rg]) : k0 - 1;
    return TileGeom2<VEC, TXL, BY>((int)threadIdx.x, nx, nx, ny, nz, tx, min(ty, nty - 1), k0,
                                   k1);
}

// A value rounded to storage and back (the state between the two steps is
// a stored state).  Exact for FP64 and FP32.
template <class P, int VEC>
__device__ __forceinline__ void to_storage(typename P::C *v) {
    if constexpr (!std::is_same<typename P::S, typename P::C>::value) {
        typename P::S s[VEC];
        narrow_vec<P, VEC>(v, s, 0, SRKey{});
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = P::widen(s[e]);
    }
}

// Two steps of one tile (geometry g) from u (u^t) into un (u^(t+2)).  tu:
// 2 * TileGeom2::U_ELEMS values of LDS, ta: 2 * TileGeom2::A_ELEMS.
template <class P, int VEC, int TXL, int BY, int PF, int ZB>
__device__ __forceinline__ void heat_tile_sweep2(const typename P::S *__restrict__ u,
                                                 typename P::S *__restrict__ un,
                                                 typename P::C r,
                                                 const TileGeom2<VEC, TXL, BY> &g,
                                                 typename P::C *tu, typename P::C *ta) {
    using C = typename P::C;
    using S = typename P::S;
    using G = TileGeom2<VEC, TXL, BY>;
    static_assert(!P::kStochastic, "stochastic rounding takes single steps");
    static_assert(PF >= 1 && PF <= 4, "prefetch depth 1 to 4");
    const long long plane = g.plane;
    const S *__restrict__ uo = u + g.own;
    const S *__restrict__ u1 = u + g.r1;
    const S *__restrict__ u2 = u + g.r2;
    S *__restrict__ vo = un + g.own;
    const int nzm = g.nz - 1;

    // a VEC-wide aligned load; a column element keeps its node in o[0]
    auto ld = [&](const S *__restrict__ base, int k, bool vec, int sel, C *o) {
        load_vec<P, VEC>(base + (long long)max(0, min(k, nzm)) * plane, o);
        if (!vec) {
            C s = o[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) s = (sel == e) ? o[e] : s;
            o[0] = s;
        }
    };
    // one step at VEC nodes whose node 0 sits at slot s0 of plane t (row
    // stride LD), x neighbours of the end nodes at slots xm / xp; every lane
    // computes, then the mask selects (keeps the LDS reads unconditional)
    auto step = [&](const C *t, int LD, int s0, int xm, int xp, bool vec, const C *zm, const C *c,
                    const C *zp, const bool *upd, C *out) {
        const C xm0 = t[xm], xpl = t[xp];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int sl = s0 + v * TXL;
            const C xmv = v == 0 ? xm0 : (vec ? c[v - 1] : xm0);
            const C xpv = v == VEC - 1 ? xpl : (vec ? c[v + 1] : xpl);
            const C ym = t[sl - LD];
            const C yp = t[sl + LD];
            const C nsum = ((xmv + xpv) + (ym + yp)) + (zm[v] + zp[v]);
            const C lap = nsum - C(6) * c[v];
            C res = c[v] + r * lap;
            asm volatile("" : "+v"(res));
            out[v] = upd[v] ? res : c[v];
        }
    };

    // Iteration s of a sweep whose first output plane is k1 (ka = k1-1+s):
    // compute u^(t+1)(ka) on the tile and its inner ring from the u^t plane
    // staged in tu[s & 1] and, for s >= 2, u^(t+2)(ka-1) from the u^(t+1)
    // plane staged last iteration; then stage u^t(ka+1) into the other u^t
    // plane and issue the loads of later planes.  One barrier per plane:
    // both u^t planes and both u^(t+1) planes alternate, so every LDS write
    // of an iteration goes to a plane the iteration before finished reading.
    // Register queues: qc, q1: u^t at the own nodes / the inner-ring
    // element, plane k1-2+i at index i; q2: the outer-ring element, plane
    // k1-1+i; qa: u^(t+1) at the own nodes, plane k1-1+i.  Loads for later
    // planes go to qc/q1[s+PF+2] and q2[s+PF] while those indices are below
    // qn / rn (the queue lengths of the caller).  s is a constant after
    // unrolling, so every queue index is.
    auto stage_u = [&](C *t, const C *c, const C *e1, const C *e2) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) t[g.own_u + v * TXL] = c[v];
        if (g.r1on) {
            t[g.r1_u] = e1[0];
            if (g.r1vec) {
#pragma unroll
                for (int v = 1; v < VEC; ++v) t[g.r1_u + v * TXL] = e1[v];
            }
        }
        if (g.r2on) {
            t[g.r2_u] = e2[0];
            if (g.r2vec) {
#pragma unroll
                for (int v = 1; v < VEC; ++v) t[g.r2_u + v * TXL] = e2[v];
            }
        }
    };
    auto iter = [&](int k1, int s, int qn, int rn, auto &qc, auto &q1, auto &q2, auto &qa) {
        const int ka = k1 - 1 + s;  // plane of u^(t+1) computed here
        const C *tcu = tu + (s & 1) * G::U_ELEMS;
        C *tnu = tu + ((s + 1) & 1) * G::U_ELEMS;
        C *tcur = ta + (s & 1) * G::A_ELEMS;
        const C *tprev = ta + ((s + 1) & 1) * G::A_ELEMS;
        // u^(t+1)(ka) at the own nodes and the inner-ring element
        const bool zin = ka >= 1 && ka <= g.nz - 2;
        bool upd[VEC], upd1[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            upd[v] = zin && g.st[v];
            upd1[v] = zin && g.r1st[v];
        }
        step(tcu, G::LDU, g.own_u, g.xm_u, g.xp_u, true, qc[s], qc[s + 1], qc[s + 2], upd,
             qa[s]);
        to_storage<P, VEC>(qa[s]);
#pragma unroll
        for (int v = 0; v < VEC; ++v) tcur[g.own_a + v * TXL] = qa[s][v];
        // the inner-ring element, in the threads that hold one (all the
        // lanes of a wavefront agree, but for one wavefront of the block)
        if (g.r1on) {
            C a1[VEC];
            step(tcu, G::LDU, g.r1_u, g.r1xm_u, g.r1xp_u, g.r1vec, q1[s], q1[s + 1], q1[s + 2],
                 upd1, a1);
            to_storage<P, VEC>(a1);
            tcur[g.r1_a] = a1[0];  // a column element writes its one node
            if (g.r1vec) {
#pragma unroll
                for (int v = 1; v < VEC; ++v) tcur[g.r1_a + v * TXL] = a1[v];
            }
        }
        // u^(t+2)(ka-1): its plane of u^(t+1) was staged last iteration
        if (s >= 2) {
            C out[VEC];
            step(tprev, G::LDA, g.own_a, g.xm_a, g.xp_a, true, qa[s - 2], qa[s - 1], qa[s], g.st,
                 out);
            store_vec_nt<P, VEC>(vo + (long long)(ka - 1) * plane, out, 0, SRKey{});
        }
        // stage u^t(ka+1) for the next iteration
        stage_u(tnu, qc[s + 2], q1[s + 2], q2[s + 1]);
        if (s + PF + 2 < qn) {
            ld(uo, k1 + s + PF, true, 0, qc[s + PF + 2]);
            ld(u1, k1 + s + PF, g.r1vec, g.r1sel, q1[s + PF + 2]);
        }
        if (s + PF + 1 < rn) ld(u2, k1 + s + PF, g.r2vec, g.r2sel, q2[s + PF + 1]);
        __syncthreads();
    };
    // the first loads of a sweep from output plane k1, and u^t(k1-1) staged
    // for its first iteration (the barrier also orders it after whatever
    // the block's LDS held before)
    auto prime = [&](int k1, int qn, int rn, auto &qc, auto &q1, auto &q2) {
#pragma unroll
        for (int s = 0; s < PF + 2 && s < qn; ++s) {
            ld(uo, k1 - 2 + s, true, 0, qc[s]);
            ld(u1, k1 - 2 + s, g.r1vec, g.r1sel, q1[s]);
        }
#pragma unroll
        for (int s = 0; s < PF + 1 && s < rn; ++s) ld(u2, k1 - 1 + s, g.r2vec, g.r2sel, q2[s]);
        __syncthreads();
        stage_u(tu, qc[1], q1[1], q2[0]);
        __syncthreads();
    };

    // NB output planes from k1, on their own (short runs: NB = 1, 2)
    auto block = [&](int k1, auto nb_tag) {
        constexpr int NB = decltype(nb_tag)::value;
        C qc[NB + 4][VEC], q1[NB + 4][VEC], q2[NB + 3][VEC], qa[NB + 2][VEC];
        prime(k1, NB + 4, NB + 3, qc, q1, q2);
#pragma unroll
        for (int s = 0; s < NB + 2; ++s) iter(k1, s, NB + 4, NB + 3, qc, q1, q2, qa);
    };
    // m sub-blocks of ZB output planes from k1 as one march: after a
    // sub-block the queues move down by ZB (the next sub-block's planes are
    // the ones already loaded or in flight), so the pipeline is filled once
    // per run.  Loads run PF planes past the end of the run (clamped into
    // the array, never used).
    auto march = [&](int k1, int m) {
        constexpr int QN = ZB + PF + 4, RN = ZB + PF + 3;
        C qc[QN][VEC], q1[QN][VEC], q2[RN][VEC], qa[ZB + 2][VEC];
        prime(k1, QN, RN, qc, q1, q2);
#pragma unroll
        for (int s = 0; s < 2; ++s) iter(k1, s, QN, RN, qc, q1, q2, qa);
        for (int b = 1;; ++b) {
#pragma unroll
            for (int s = 2; s < ZB + 2; ++s) iter(k1, s, QN, RN, qc, q1, q2, qa);
            if (b == m) break;
            k1 += ZB;
#pragma unroll
            for (int i = 2; i < PF + 4; ++i) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    qc[i][v] = qc[i + ZB][v];
                    q1[i][v] = q1[i + ZB][v];
                }
            }
#pragma unroll
            for (int i = 2; i < PF + 3; ++i) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) q2[i][v] = q2[i + ZB][v];
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                qa[0][v] = qa[ZB][v];
                qa[1][v] = qa[ZB + 1][v];
            }
        }
    };
    // runs shorter than a z-block (the Boundary planes): two planes at a
    // time, then one
    auto short_run = [&](int k, int ke) {
        for (; k + 1 <= ke; k += 2) block(k, std::integral_constant<int, 2>{});
        if (k == ke) block(k, std::integral_constant<int, 1>{});
    };

    const RunPlan pl = run_plan(g.kb, g.ke, ZB);
    if (pl.m > 0) march(pl.start, pl.m);
    if (pl.rest <= g.ke) short_run(pl.rest, g.ke);
}

}  // namespace
}  // namespace hc
