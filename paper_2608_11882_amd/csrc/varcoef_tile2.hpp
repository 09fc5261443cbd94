#pragma once

// varcoef_tile2.hpp -- two explicit steps per pass of the variable-
// coefficient step with a source (the paper's Eq. 1-4 in flux form), gfx950.
// Device code only; not exported.
//
// The two-step tile of heat_tile2.hpp with kappa and rhs beside u: a block
// stages u^t(k) and kappa(k) with the two-node ring, computes u^(t+1)(k) on
// its tile and the one-node ring (kappa is needed at the same nodes as u,
// rhs at the node itself), and computes u^(t+2)(k-1) on the tile; that
// step reads kappa's x and y neighbours at plane k-1, so kappa's LDS plane
// is double-buffered like u^(t+1)'s.  Every value is evaluated with the
// single step's expression (varcoef_kernels.hip), in the same order and
// precision, so two steps here are bit-identical to two single steps.  The
// geometry (TileGeom2) is the constant-coefficient one: kappa and rhs have
// u's layout, so every offset and slot is shared.

#include "heat_tile2.hpp"

namespace hc {
namespace {

// tu: TileGeom2::U_ELEMS values of LDS (u^t), tk: 2 * U_ELEMS (kappa, two
// planes), ta: 2 * A_ELEMS (u^(t+1), two planes).
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

    // output planes k1 .. k1+NB-1.  qc/qk, q1/q1k: u and kappa at the own
    // nodes / the inner-ring element, plane k1-2+s; qf, q1f: rhs there,
    // plane k1-1+s; q2/q2k: the outer-ring element, plane k1-1+s; qa:
    // u^(t+1) at the own nodes, plane k1-1+s
    auto block = [&](int k1, auto nb_tag) {
        constexpr int NB = decltype(nb_tag)::value;
        C qc[NB + 4][VEC], qk[NB + 4][VEC], q1[NB + 4][VEC], q1k[NB + 4][VEC];
        C qf[NB + 2][VEC], q1f[NB + 2][VEC], q2[NB + 2][VEC], q2k[NB + 2][VEC];
        C qa[NB + 2][VEC];
#pragma unroll
        for (int s = 0; s < PF + 2 && s < NB + 4; ++s) {
            ld(uo, k1 - 2 + s, true, 0, qc[s]);
            ld(ko, k1 - 2 + s, true, 0, qk[s]);
            ld(u1, k1 - 2 + s, g.r1vec, g.r1sel, q1[s]);
            ld(k1p, k1 - 2 + s, g.r1vec, g.r1sel, q1k[s]);
        }
#pragma unroll
        for (int s = 0; s < PF && s < NB + 2; ++s) {
            ld(fo, k1 - 1 + s, true, 0, qf[s]);
            ld(f1, k1 - 1 + s, g.r1vec, g.r1sel, q1f[s]);
            ld(u2, k1 - 1 + s, g.r2vec, g.r2sel, q2[s]);
            ld(k2p, k1 - 1 + s, g.r2vec, g.r2sel, q2k[s]);
        }
#pragma unroll
        for (int s = 0; s < NB + 2; ++s) {
            const int ka = k1 - 1 + s;  // plane of u^(t+1) computed here
            C *acur = ta + (s & 1) * G::A_ELEMS;
            const C *aprev = ta + ((s + 1) & 1) * G::A_ELEMS;
            C *kcur = tk + (s & 1) * G::U_ELEMS;
            const C *kprev = tk + ((s + 1) & 1) * G::U_ELEMS;
            __syncthreads();  // the last plane's reads of tu, acur and kcur are done
            // stage u^t(ka) and kappa(ka)
            stage(tu, g.own_u, true, qc[s + 1]);
            stage(kcur, g.own_u, true, qk[s + 1]);
            if (g.r1on) {
                stage(tu, g.r1_u, g.r1vec, q1[s + 1]);
                stage(kcur, g.r1_u, g.r1vec, q1k[s + 1]);
            }
            if (g.r2on) {
                stage(tu, g.r2_u, g.r2vec, q2[s]);
                stage(kcur, g.r2_u, g.r2vec, q2k[s]);
            }
            if (s + PF + 2 < NB + 4) {
                ld(uo, k1 + s + PF, true, 0, qc[s + PF + 2]);
                ld(ko, k1 + s + PF, true, 0, qk[s + PF + 2]);
                ld(u1, k1 + s + PF, g.r1vec, g.r1sel, q1[s + PF + 2]);
                ld(k1p, k1 + s + PF, g.r1vec, g.r1sel, q1k[s + PF + 2]);
            }
            if (s + PF < NB + 2) {
                ld(fo, k1 + s + PF - 1, true, 0, qf[s + PF]);
                ld(f1, k1 + s + PF - 1, g.r1vec, g.r1sel, q1f[s + PF]);
                ld(u2, k1 + s + PF - 1, g.r2vec, g.r2sel, q2[s + PF]);
                ld(k2p, k1 + s + PF - 1, g.r2vec, g.r2sel, q2k[s + PF]);
            }
            __syncthreads();
            const bool zin = ka >= 1 && ka <= g.nz - 2;
            bool upd[VEC], upd1[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                upd[v] = zin && g.st[v];
                upd1[v] = zin && g.r1st[v];
            }
            // u^(t+1)(ka) at the own nodes and the inner-ring element
            step(tu, G::LDU, g.own_u, g.xm_u, g.xp_u, kcur, g.own_u, g.xm_u, g.xp_u, true, qc[s],
                 qc[s + 1], qc[s + 2], qk[s], qk[s + 1], qk[s + 2], qf[s], upd, qa[s]);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acur[g.own_a + v * TXL] = qa[s][v];
            if (g.r1on) {  // the inner-ring element, in the threads that hold one
                C a1[VEC];
                step(tu, G::LDU, g.r1_u, g.r1xm_u, g.r1xp_u, kcur, g.r1_u, g.r1xm_u, g.r1xp_u,
                     g.r1vec, q1[s], q1[s + 1], q1[s + 2], q1k[s], q1k[s + 1], q1k[s + 2],
                     q1f[s], upd1, a1);
                acur[g.r1_a] = a1[0];
                if (g.r1vec) {
#pragma unroll
                    for (int v = 1; v < VEC; ++v) acur[g.r1_a + v * TXL] = a1[v];
                }
            }
            // u^(t+2)(ka-1): u^(t+1) and kappa of that plane were staged in
            // the last iteration
            if (s >= 2) {
                C out[VEC];
                step(aprev, G::LDA, g.own_a, g.xm_a, g.xp_a, kprev, g.own_u, g.xm_u, g.xp_u, true,
                     qa[s - 2], qa[s - 1], qa[s], qk[s - 1], qk[s], qk[s + 1], qf[s - 1], g.st,
                     out);
                store_vec_nt<P, VEC>(vo + (long long)(ka - 1) * plane, out, 0, SRKey{});
            }
        }
    };

    if (g.ke - g.kb + 1 >= ZB) {
        for (int k0 = g.kb;; k0 += ZB) {
            const int k1 = min(k0, g.ke - ZB + 1);
            block(k1, std::integral_constant<int, ZB>{});
            if (k1 == g.ke - ZB + 1) break;
        }
    } else {
        // short runs (the Boundary planes): two planes at a time, then one
        int k = g.kb;
        for (; k + 1 <= g.ke; k += 2) block(k, std::integral_constant<int, 2>{});
        if (k == g.ke) block(k, std::integral_constant<int, 1>{});
    }
}

}  // namespace
}  // namespace hc
