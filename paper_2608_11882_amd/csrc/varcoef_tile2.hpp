#pragma once

// varcoef_tile2.hpp -- two explicit steps per pass of the variable-
// coefficient step with a source (the paper's Eq. 1-4 in flux form), gfx950.
// Device code only; not exported.
//
// The two-step tile of heat_tile2.hpp with kappa and rhs beside u: a block
// stages u^t(k) and kappa(k) with the two-node ring, computes u^(t+1)(k) on
// its tile and the one-node ring (kappa is needed at the same nodes as u,
// rhs at the node itself), and computes u^(t+2)(k-1) on the tile; that
// step reads kappa's x and y neighbours at plane k-1.  The march is the
// constant-coefficient one (one barrier per plane, runs of sub-blocks with
// the register queues carried across, run_plan): u^t and u^(t+1) planes
// alternate between two LDS buffers, kappa planes rotate through four (an
// iteration reads kappa at k and k-1 and stages k+1, and the one before
// read k-1 and k-2).  Every value is evaluated with the single step's
// expression (varcoef_kernels.hip), in the same order and precision, so two
// steps here are bit-identical to two single steps.  The geometry
// (TileGeom2) is the constant-coefficient one: kappa and rhs have u's
// layout, so every offset and slot is shared.

#include "heat_tile2.hpp"

namespace hc {
namespace {

// tu: 2 * TileGeom2::U_ELEMS values of LDS (u^t, two planes), tk:
// 4 * U_ELEMS (kappa, four planes), ta: 2 * A_ELEMS (u^(t+1), two planes).
template <class P, int VEC, int TXL, int BY, int PF, int ZB>
__device__ __forceinline__ void vk_tile_sweep2(const typename P::S *__restrict__ u,
                                               const typename P::S *__restrict__ kap,
                                               const typename P::S *__restrict__ rhs,
                                               typename P::S *__restrict__ un,
                                               typename P::C beta,
                                               const TileGeom2<VEC, TXL, BY> &g,
                                               typename P::C *tu, typename P::C *tk,
                                               typename P::C *ta) {
    using C = typename P::C;
    using S = typename P::S;
    using G = TileGeom2<VEC, TXL, BY>;
    static_assert(!P::kStochastic && sizeof(S) == sizeof(C), "FP64 or FP32 storage");
    static_assert(PF >= 1 && PF <= 4, "prefetch depth 1 to 4");
    static_assert(ZB % 4 == 0, "a march keeps the kappa planes' rotation across sub-blocks");
    const long long plane = g.plane;
    const S *__restrict__ uo = u + g.own;
    const S *__restrict__ ko = kap + g.own;
    const S *__restrict__ fo = rhs + g.own;
    const S *__restrict__ u1 = u + g.r1;
    const S *__restrict__ k1p = kap + g.r1;
    const S *__restrict__ f1 = rhs + g.r1;
    const S *__restrict__ u2 = u + g.r2;
    const S *__restrict__ k2p = kap + g.r2;
    S *__restrict__ vo = un + g.own;
    const int nzm = g.nz - 1;

    auto ld = [&](const S *__restrict__ base, int k, bool vec, int sel, C *o) {
        load_vec<P, VEC>(base + (long long)max(0, min(k, nzm)) * plane, o);
        if (!vec) {
            C s = o[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) s = (sel == e) ? o[e] : s;
            o[0] = s;
        }
    };
    auto stage = [&](C *t, int slot, bool vec, const C *v) {
        t[slot] = v[0];
        if (vec) {
#pragma unroll
            for (int e = 1; e < VEC; ++e) t[slot + e * TXL] = v[e];
        }
    };
    // one step at VEC nodes whose node 0 sits at slot s0 of the u plane tv
    // (row stride LDV) and of the kappa plane tkv (row stride G::LDU, slot
    // k0); x neighbours of the end nodes at xm/xp (u) and kxm/kxp (kappa)
    auto step = [&](const C *tv, int LDV, int s0, int xm, int xp, const C *tkv, int k0, int kxm,
                    int kxp, bool vec, const C *zmu, const C *cu, const C *zpu, const C *zmk,
                    const C *ck, const C *zpk, const C *f, const bool *upd, C *out) {
        const C uxm0 = tv[xm], uxpl = tv[xp];
        const C kxm0 = tkv[kxm], kxpl = tkv[kxp];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const C uc = cu[v], kc = ck[v];
            const C uxm = v == 0 ? uxm0 : (vec ? cu[v - 1] : uxm0);
            const C kxm = v == 0 ? kxm0 : (vec ? ck[v - 1] : kxm0);
            const C uxp = v == VEC - 1 ? uxpl : (vec ? cu[v + 1] : uxpl);
            const C kxp = v == VEC - 1 ? kxpl : (vec ? ck[v + 1] : kxpl);
            const int sl = s0 + v * TXL, kl = k0 + v * TXL;
            const C uym = tv[sl - LDV], uyp = tv[sl + LDV];
            const C kym = tkv[kl - G::LDU], kyp = tkv[kl + G::LDU];
            const C dx = (kc + kxp) * (uxp - uc) - (kxm + kc) * (uc - uxm);
            const C dy = (kc + kyp) * (uyp - uc) - (kym + kc) * (uc - uym);
            const C dz = (kc + zpk[v]) * (zpu[v] - uc) - (zmk[v] + kc) * (uc - zmu[v]);
            const C lop = (dx + dy) + dz;
            C res = (uc + f[v]) + beta * lop;
            asm volatile("" : "+v"(res));
            out[v] = upd[v] ? res : uc;
        }
    };
    // u^t and kappa of one plane into their LDS planes: own nodes (c, ck),
    // inner-ring element (e1, e1k), outer-ring element (e2, e2k)
    auto stage_uk = [&](C *t, C *tkk, const C *c, const C *ck, const C *e1, const C *e1k,
                        const C *e2, const C *e2k) {
        stage(t, g.own_u, true, c);
        stage(tkk, g.own_u, true, ck);
        if (g.r1on) {
            stage(t, g.r1_u, g.r1vec, e1);
            stage(tkk, g.r1_u, g.r1vec, e1k);
        }
        if (g.r2on) {
            stage(t, g.r2_u, g.r2vec, e2);
            stage(tkk, g.r2_u, g.r2vec, e2k);
        }
    };

    // Iteration s of a sweep whose first output plane is k1 (ka = k1-1+s),
    // as in heat_tile_sweep2: u^(t+1)(ka) on the tile and its inner ring from
    // the planes staged in tu[s & 1] and tk[s & 3]; for s >= 2, u^(t+2)(ka-1)
    // from the u^(t+1) plane staged last iteration and kappa(ka-1) in
    // tk[(s-1) & 3]; then u^t(ka+1) and kappa(ka+1) staged into tu[(s+1) & 1]
    // and tk[(s+1) & 3], loads of later planes issued, one barrier.
    // Register queues: qc/qk, q1/q1k: u and kappa at the own nodes / the
    // inner-ring element, plane k1-2+i at index i; q2/q2k: the outer-ring
    // element, plane k1-1+i; qf/q1f: rhs at the own nodes / the inner-ring
    // element, plane k1-1+i; qa: u^(t+1) at the own nodes, plane k1-1+i.
    // Loads for later planes go to index s+PF+2 of qc/qk/q1/q1k and s+PF+1
    // of q2/q2k/qf/q1f while below qn / rn.
    auto iter = [&](int k1, int s, int qn, int rn, auto &qc, auto &qk, auto &q1, auto &q1k,
                    auto &q2, auto &q2k, auto &qf, auto &q1f, auto &qa) {
        const int ka = k1 - 1 + s;
        const C *tcu = tu + (s & 1) * G::U_ELEMS;
        C *tnu = tu + ((s + 1) & 1) * G::U_ELEMS;
        const C *kcur = tk + (s & 3) * G::U_ELEMS;
        const C *kprev = tk + ((s + 3) & 3) * G::U_ELEMS;
        C *knext = tk + ((s + 1) & 3) * G::U_ELEMS;
        C *acur = ta + (s & 1) * G::A_ELEMS;
        const C *aprev = ta + ((s + 1) & 1) * G::A_ELEMS;
        const bool zin = ka >= 1 && ka <= g.nz - 2;
        bool upd[VEC], upd1[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            upd[v] = zin && g.st[v];
            upd1[v] = zin && g.r1st[v];
        }
        // u^(t+1)(ka) at the own nodes and the inner-ring element
        step(tcu, G::LDU, g.own_u, g.xm_u, g.xp_u, kcur, g.own_u, g.xm_u, g.xp_u, true, qc[s],
             qc[s + 1], qc[s + 2], qk[s], qk[s + 1], qk[s + 2], qf[s], upd, qa[s]);
#pragma unroll
        for (int v = 0; v < VEC; ++v) acur[g.own_a + v * TXL] = qa[s][v];
        if (g.r1on) {  // the inner-ring element, in the threads that hold one
            C a1[VEC];
            step(tcu, G::LDU, g.r1_u, g.r1xm_u, g.r1xp_u, kcur, g.r1_u, g.r1xm_u, g.r1xp_u,
                 g.r1vec, q1[s], q1[s + 1], q1[s + 2], q1k[s], q1k[s + 1], q1k[s + 2], q1f[s],
                 upd1, a1);
            acur[g.r1_a] = a1[0];
            if (g.r1vec) {
#pragma unroll
                for (int v = 1; v < VEC; ++v) acur[g.r1_a + v * TXL] = a1[v];
            }
        }
        // u^(t+2)(ka-1): u^(t+1) of that plane was staged last iteration,
        // kappa of it the iteration before
        if (s >= 2) {
            C out[VEC];
            step(aprev, G::LDA, g.own_a, g.xm_a, g.xp_a, kprev, g.own_u, g.xm_u, g.xp_u, true,
                 qa[s - 2], qa[s - 1], qa[s], qk[s - 1], qk[s], qk[s + 1], qf[s - 1], g.st, out);
            store_vec_nt<P, VEC>(vo + (long long)(ka - 1) * plane, out, 0, SRKey{});
        }
        // stage u^t(ka+1) and kappa(ka+1) for the next iteration
        stage_uk(tnu, knext, qc[s + 2], qk[s + 2], q1[s + 2], q1k[s + 2], q2[s + 1], q2k[s + 1]);
        if (s + PF + 2 < qn) {
            const int k = k1 + s + PF;
            ld(uo, k, true, 0, qc[s + PF + 2]);
            ld(ko, k, true, 0, qk[s + PF + 2]);
            ld(u1, k, g.r1vec, g.r1sel, q1[s + PF + 2]);
            ld(k1p, k, g.r1vec, g.r1sel, q1k[s + PF + 2]);
        }
        if (s + PF + 1 < rn) {
            const int k = k1 + s + PF;
            ld(u2, k, g.r2vec, g.r2sel, q2[s + PF + 1]);
            ld(k2p, k, g.r2vec, g.r2sel, q2k[s + PF + 1]);
            ld(fo, k, true, 0, qf[s + PF + 1]);
            ld(f1, k, g.r1vec, g.r1sel, q1f[s + PF + 1]);
        }
        __syncthreads();
    };
    // the first loads of a sweep from output plane k1, and u^t(k1-1) and
    // kappa(k1-1) staged for its first iteration (the barrier also orders
    // them after whatever the block's LDS held before)
    auto prime = [&](int k1, int qn, int rn, auto &qc, auto &qk, auto &q1, auto &q1k, auto &q2,
                     auto &q2k, auto &qf, auto &q1f) {
#pragma unroll
        for (int s = 0; s < PF + 2 && s < qn; ++s) {
            ld(uo, k1 - 2 + s, true, 0, qc[s]);
            ld(ko, k1 - 2 + s, true, 0, qk[s]);
            ld(u1, k1 - 2 + s, g.r1vec, g.r1sel, q1[s]);
            ld(k1p, k1 - 2 + s, g.r1vec, g.r1sel, q1k[s]);
        }
#pragma unroll
        for (int s = 0; s < PF + 1 && s < rn; ++s) {
            ld(u2, k1 - 1 + s, g.r2vec, g.r2sel, q2[s]);
            ld(k2p, k1 - 1 + s, g.r2vec, g.r2sel, q2k[s]);
            ld(fo, k1 - 1 + s, true, 0, qf[s]);
            ld(f1, k1 - 1 + s, g.r1vec, g.r1sel, q1f[s]);
        }
        __syncthreads();
        stage_uk(tu, tk, qc[1], qk[1], q1[1], q1k[1], q2[0], q2k[0]);
        __syncthreads();
    };

    // NB output planes from k1, on their own (short runs: NB = 1, 2)
    auto block = [&](int k1, auto nb_tag) {
        constexpr int NB = decltype(nb_tag)::value;
        C qc[NB + 4][VEC], qk[NB + 4][VEC], q1[NB + 4][VEC], q1k[NB + 4][VEC];
        C q2[NB + 3][VEC], q2k[NB + 3][VEC], qf[NB + 3][VEC], q1f[NB + 3][VEC];
        C qa[NB + 2][VEC];
        prime(k1, NB + 4, NB + 3, qc, qk, q1, q1k, q2, q2k, qf, q1f);
#pragma unroll
        for (int s = 0; s < NB + 2; ++s)
            iter(k1, s, NB + 4, NB + 3, qc, qk, q1, q1k, q2, q2k, qf, q1f, qa);
    };
    // m sub-blocks of ZB output planes from k1 as one march (the queues move
    // down by ZB after a sub-block; the pipeline is filled once per run).
    // Step 2 of a sub-block's first iterations reads kappa and rhs one plane
    // further back than the constant-coefficient march keeps, so those
    // queues move from index 1.
    auto march = [&](int k1, int m) {
        constexpr int QN = ZB + PF + 4, RN = ZB + PF + 3;
        C qc[QN][VEC], qk[QN][VEC], q1[QN][VEC], q1k[QN][VEC];
        C q2[RN][VEC], q2k[RN][VEC], qf[RN][VEC], q1f[RN][VEC];
        C qa[ZB + 2][VEC];
        prime(k1, QN, RN, qc, qk, q1, q1k, q2, q2k, qf, q1f);
#pragma unroll
        for (int s = 0; s < 2; ++s) iter(k1, s, QN, RN, qc, qk, q1, q1k, q2, q2k, qf, q1f, qa);
        for (int b = 1;; ++b) {
#pragma unroll
            for (int s = 2; s < ZB + 2; ++s)
                iter(k1, s, QN, RN, qc, qk, q1, q1k, q2, q2k, qf, q1f, qa);
            if (b == m) break;
            k1 += ZB;
#pragma unroll
            for (int i = 1; i < PF + 4; ++i) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    qc[i][v] = qc[i + ZB][v];
                    qk[i][v] = qk[i + ZB][v];
                    q1[i][v] = q1[i + ZB][v];
                    q1k[i][v] = q1k[i + ZB][v];
                }
            }
#pragma unroll
            for (int i = 1; i < PF + 3; ++i) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    q2[i][v] = q2[i + ZB][v];
                    q2k[i][v] = q2k[i + ZB][v];
                    qf[i][v] = qf[i + ZB][v];
                    q1f[i][v] = q1f[i + ZB][v];
                }
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
