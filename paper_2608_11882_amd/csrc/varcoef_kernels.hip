// varcoef_kernels.hip -- the paper's own equation on gfx950: explicit steps
// of du/dt = div(kappa grad u) + f (Eq. 1-4) with a coefficient and a source
// that vary from node to node.
//
// Per interior node (the flux form, face coefficient = sum of the two nodes'
// coefficients, which the 1/2 in beta = dt/(2h^2) compensates):
//   D_x = (k_c + k_x+) (u_x+ - u_c) - (k_x- + k_c) (u_c - u_x-)   (D_y, D_z alike)
//   u_new = (u_c + rhs_c) + beta * ((D_x + D_y) + D_z),   rhs = dt f
// in exactly this order, compiled without contraction, so every node is
// bit-identical to a serial evaluation of the same expression.
//
// The z-marching tile of the constant-coefficient sweep carries a second
// stencil field: kappa is needed at the same seven nodes as u, so it goes
// through the same register queue along z and its own LDS plane with the
// same ring; rhs is needed only at the node itself and is streamed PF planes
// ahead.  One node moves 4 values (u, kappa, rhs in; u_new out): 32 bytes in
// FP64, 16 in FP32, against 16 / 8 for the constant-coefficient step.
//
// Kernels: Interior, Boundary and fused z-marching sweeps (one body, three
// names, as for the constant coefficient), and the one-thread-per-node form.

#include "heat_tile.hpp"

#include <climits>
#include <type_traits>

namespace hc {
namespace {

// Sweep one tile (geometry g) of the variable-coefficient step; tu and tk
// are LDS planes of tile_lds_elems<VEC, TXL, BY>() values each.
template <class P, int VEC, int TXL, int BY, int PF, int ZB>
__device__ __forceinline__ void vk_tile_sweep(const typename P::S *__restrict__ u,
                                              const typename P::S *__restrict__ kap,
                                              const typename P::S *__restrict__ rhs,
                                              typename P::S *__restrict__ un,
                                              typename P::C beta,
                                              const TileGeom<VEC, TXL, BY> &g,
                                              typename P::C *tu, typename P::C *tk) {
    using C = typename P::C;
    using S = typename P::S;
    using G = TileGeom<VEC, TXL, BY>;
    static_assert(!P::kStochastic && sizeof(S) == sizeof(C), "FP64 or FP32 storage");
    static_assert(PF >= 1 && PF <= 4 && PF < ZB, "prefetch depth 1 to 4");
    const long long plane = g.plane;
    const S *__restrict__ uo = u + g.own;
    const S *__restrict__ ko = kap + g.own;
    const S *__restrict__ ro = rhs + g.own;
    const S *__restrict__ ur = u + g.ring;
    const S *__restrict__ kr = kap + g.ring;
    S *__restrict__ vo = un + g.own;
    const int kb = g.kb, ke = g.ke;

    auto ld_ring = [&](const S *__restrict__ base, long long kp, C *o) {
        load_vec<P, VEC>(base + kp, o);
        if (!g.rvec) {
            C sel = o[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) sel = (g.rsel == e) ? o[e] : sel;
            o[0] = sel;
        }
    };
    auto put = [&](C *tile, const C *c, const C *gv) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) tile[g.own_slot + v * TXL] = c[v];
        if (g.rslot >= 0) {
            tile[g.rslot] = gv[0];
            if (g.rvec) {
#pragma unroll
                for (int v = 1; v < VEC; ++v) tile[g.rslot + v * TXL] = gv[v];
            }
        }
    };
    // zm*/c*/zp*: u and kappa of the planes below, at and above; f: rhs
    auto update = [&](const C *zmu, const C *cu, const C *zpu, const C *zmk, const C *ck,
                      const C *zpk, const C *f, C *out) {
        const C uxm0 = tu[g.xm_slot], uxpl = tu[g.xp_slot];
        const C kxm0 = tk[g.xm_slot], kxpl = tk[g.xp_slot];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int sl = g.own_slot + v * TXL;
            const C uc = cu[v], kc = ck[v];
            const C uxm = v == 0 ? uxm0 : cu[v - 1];
            const C kxm = v == 0 ? kxm0 : ck[v - 1];
            const C uxp = v == VEC - 1 ? uxpl : cu[v + 1];
            const C kxp = v == VEC - 1 ? kxpl : ck[v + 1];
            const C uym = tu[sl - G::LD], uyp = tu[sl + G::LD];
            const C kym = tk[sl - G::LD], kyp = tk[sl + G::LD];
            const C dx = (kc + kxp) * (uxp - uc) - (kxm + kc) * (uc - uxm);
            const C dy = (kc + kyp) * (uyp - uc) - (kym + kc) * (uc - uym);
            const C dz = (kc + zpk[v]) * (zpu[v] - uc) - (zmk[v] + kc) * (uc - zmu[v]);
            const C lop = (dx + dy) + dz;
            C res = (uc + f[v]) + beta * lop;
            // computed in every lane, then selected: keeps the LDS reads
            // above unconditional (see the constant-coefficient sweep)
            asm volatile("" : "+v"(res));
            out[v] = g.st[v] ? res : uc;
        }
    };

    if (ke - kb + 1 >= ZB) {
        // sub-blocks of exactly ZB planes, the last shifted back to end at
        // ke (shared planes are computed and written twice, same bits)
        for (int k0 = kb;; k0 += ZB) {
            const int k1 = min(k0, ke - ZB + 1);
            // qu/qk[s]: plane k1-1+s; gu/gk/rh[s]: plane k1+s
            C qu[ZB + 2][VEC], qk[ZB + 2][VEC];
            C gu[ZB][VEC], gk[ZB][VEC], rh[ZB][VEC];
#pragma unroll
            for (int s = 0; s < PF + 2; ++s) {
                load_vec<P, VEC>(uo + (long long)(k1 - 1 + s) * plane, qu[s]);
                load_vec<P, VEC>(ko + (long long)(k1 - 1 + s) * plane, qk[s]);
            }
#pragma unroll
            for (int s = 0; s < PF; ++s) {
                ld_ring(ur, (long long)(k1 + s) * plane, gu[s]);
                ld_ring(kr, (long long)(k1 + s) * plane, gk[s]);
                load_vec<P, VEC>(ro + (long long)(k1 + s) * plane, rh[s]);
            }
#pragma unroll
            for (int s = 0; s < ZB; ++s) {
                const long long kp = (long long)(k1 + s) * plane;
                __syncthreads();  // the previous plane's LDS reads are done
                put(tu, qu[s + 1], gu[s]);
                put(tk, qk[s + 1], gk[s]);
                if (s + PF < ZB) {
                    ld_ring(ur, kp + PF * plane, gu[s + PF]);
                    ld_ring(kr, kp + PF * plane, gk[s + PF]);
                    load_vec<P, VEC>(ro + kp + PF * plane, rh[s + PF]);
                }
                __syncthreads();
                C out[VEC];
                update(qu[s], qu[s + 1], qu[s + 2], qk[s], qk[s + 1], qk[s + 2], rh[s], out);
                store_vec_nt<P, VEC>(vo + kp, out, 0, SRKey{});
                if (s + 2 + PF <= ZB + 1) {
                    load_vec<P, VEC>(uo + kp + (1 + PF) * plane, qu[s + 2 + PF]);
                    load_vec<P, VEC>(ko + kp + (1 + PF) * plane, qk[s + 2 + PF]);
                }
            }
            if (k1 == ke - ZB + 1) break;
        }
        return;
    }

    // generic depth (short ranges): one plane of loads ahead
    C zmu[VEC], cu[VEC], zpu[VEC], zmk[VEC], ck[VEC], zpk[VEC], gu0[VEC], gk0[VEC], f0[VEC];
    load_vec<P, VEC>(uo + (long long)(kb - 1) * plane, zmu);
    load_vec<P, VEC>(uo + (long long)kb * plane, cu);
    load_vec<P, VEC>(uo + (long long)(kb + 1) * plane, zpu);
    load_vec<P, VEC>(ko + (long long)(kb - 1) * plane, zmk);
    load_vec<P, VEC>(ko + (long long)kb * plane, ck);
    load_vec<P, VEC>(ko + (long long)(kb + 1) * plane, zpk);
    ld_ring(ur, (long long)kb * plane, gu0);
    ld_ring(kr, (long long)kb * plane, gk0);
    load_vec<P, VEC>(ro + (long long)kb * plane, f0);
    for (int k = kb; k <= ke; ++k) {
        const long long kp = (long long)k * plane;
        const long long kn = (long long)min(k + 1, ke) * plane;
        C znu[VEC], znk[VEC], gun[VEC], gkn[VEC], fn[VEC];
        load_vec<P, VEC>(uo + (long long)min(k + 2, ke + 1) * plane, znu);
        load_vec<P, VEC>(ko + (long long)min(k + 2, ke + 1) * plane, znk);
        ld_ring(ur, kn, gun);
        ld_ring(kr, kn, gkn);
        load_vec<P, VEC>(ro + kn, fn);
        __syncthreads();
        put(tu, cu, gu0);
        put(tk, ck, gk0);
        __syncthreads();
        C out[VEC];
        update(zmu, cu, zpu, zmk, ck, zpk, f0, out);
        store_vec_nt<P, VEC>(vo + kp, out, 0, SRKey{});
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            zmu[v] = cu[v];
            cu[v] = zpu[v];
            zpu[v] = znu[v];
            zmk[v] = ck[v];
            ck[v] = zpk[v];
            zpk[v] = znk[v];
            gu0[v] = gun[v];
            gk0[v] = gkn[v];
            f0[v] = fn[v];
        }
    }
}

#define HC_VK_KERNEL(NAME)                                                                    \
    template <class P, int VEC, int WX, int BY, int PF, int ZB>                               \
    __global__ __launch_bounds__(64 * WX * BY) void NAME(                                     \
        const typename P::S *__restrict__ u, const typename P::S *__restrict__ kap,           \
        const typename P::S *__restrict__ rhs, typename P::S *__restrict__ un, int nx,        \
        int ny, typename P::C beta, ZTable zt, int ntx, int nty, int xcd) {                   \
        static_assert(64 * WX * BY <= 1024, "at most 1024 threads per block");               \
        __shared__ typename P::C tu[tile_lds_elems<VEC, 64 * WX, BY>()];                      \
        __shared__ typename P::C tk[tile_lds_elems<VEC, 64 * WX, BY>()];                      \
        const auto g = block_tile<VEC, 64 * WX, BY>(nx, ny, zt, ntx, nty, xcd, ZB);           \
        vk_tile_sweep<P, VEC, 64 * WX, BY, PF, ZB>(u, kap, rhs, un, beta, g, tu, tk);         \
    }

// Three entry points with one body, so that profiles name the role.
HC_VK_KERNEL(heat_vk_interior)
HC_VK_KERNEL(heat_vk_boundary)
HC_VK_KERNEL(heat_vk_fused)
#undef HC_VK_KERNEL

// One thread per interior node, every value loaded from memory: the
// straightforward form (the paper's collapse(3) loop over STENCIL).
template <class P>
__global__ __launch_bounds__(256) void heat_vk_plain(
    const typename P::S *__restrict__ u, const typename P::S *__restrict__ kap,
    const typename P::S *__restrict__ rhs, typename P::S *__restrict__ un, int nx, int ny,
    int nz, typename P::C beta) {
    using C = typename P::C;
    const int i = 1 + (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int j = 1 + (int)blockIdx.y * 4 + (int)threadIdx.y;
    const int k = 1 + (int)blockIdx.z;
    if (i > nx - 2 || j > ny - 2 || k > nz - 2) return;
    const long long sy = nx, sz = (long long)nx * ny;
    const long long p = (long long)k * sz + (long long)j * sy + i;
    const C uc = u[p], kc = kap[p];
    const C dx = (kc + kap[p + 1]) * (u[p + 1] - uc) - (kap[p - 1] + kc) * (uc - u[p - 1]);
    const C dy = (kc + kap[p + sy]) * (u[p + sy] - uc) - (kap[p - sy] + kc) * (uc - u[p - sy]);
    const C dz = (kc + kap[p + sz]) * (u[p + sz] - uc) - (kap[p - sz] + kc) * (uc - u[p - sz]);
    const C lop = (dx + dy) + dz;
    un[p] = (uc + rhs[p]) + beta * lop;
}

}  // namespace

// Tile shapes built for the variable-coefficient sweep, per precision:
// X(vec, wx, by, pf, zdepth).  (1, 4, 4, 2, 16) is the fallback for arrays
// that do not allow wide lanes.
#define HC_VK_SHAPES_F64(X)                                                      \
    X(1, 4, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 1, 8, 2, 16) X(2, 2, 8, 2, 16)     \
    X(2, 2, 4, 2, 32) X(2, 4, 4, 2, 16) X(2, 4, 4, 2, 32) X(2, 2, 8, 1, 32)     \
    X(2, 4, 4, 1, 32) X(2, 4, 4, 3, 32)
#define HC_VK_SHAPES_F32(X)                                                      \
    X(1, 4, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 4, 4, 2, 16) X(4, 1, 8, 2, 16)     \
    X(4, 2, 4, 2, 16) X(4, 2, 8, 2, 16) X(4, 4, 4, 2, 16) X(4, 2, 4, 1, 32)     \
    X(1, 4, 4, 2, 32) X(1, 2, 8, 2, 16) X(1, 4, 4, 3, 16)

#define HC_VK_KEY(V, W, B, P, Z) ((((V * 8 + W) * 32 + B) * 8 + P) * 128 + Z)

bool heat_vk_tiling_supported(int dtype, const HeatTiling &t) {
    const int key = HC_VK_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, P, Z) if (key == HC_VK_KEY(V, W, B, P, Z)) return true;
    if (dtype == kDtypeF64) { HC_VK_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_VK_SHAPES_F32(HC_X) }
#undef HC_X
    return false;
}

template <class P>
static hipError_t launch_vk(KernelKind kind, const void *u, const void *kap, const void *rhs,
                            void *un, int nx, int ny, double beta, const ZTable &zt,
                            const HeatTiling &t, hipStream_t s) {
    using S = typename P::S;
    using C = typename P::C;
    const long long nb = heat_tile_blocks(nx, ny, t, zt);
    if (nb <= 0) return hipSuccess;
    if (nb > INT_MAX) return hipErrorInvalidConfiguration;
    const int txw = tile_width(t);
    const int ntx = (nx + txw - 1) / txw;
    const int nty = (ny - 2 + t.by - 1) / t.by;
    const dim3 grid((unsigned)nb), block(64 * t.wx * t.by);
    const S *us = static_cast<const S *>(u);
    const S *ks = static_cast<const S *>(kap);
    const S *rs = static_cast<const S *>(rhs);
    S *uns = static_cast<S *>(un);
    const C b = (C)beta;
    const int shape = HC_VK_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, PF, Z)                                                         \
    if (shape == HC_VK_KEY(V, W, B, PF, Z)) {                                        \
        if (kind == K_VK_INTERIOR)                                                   \
            heat_vk_interior<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(              \
                us, ks, rs, uns, nx, ny, b, zt, ntx, nty, t.xcd);                    \
        else if (kind == K_VK_BOUNDARY)                                              \
            heat_vk_boundary<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(              \
                us, ks, rs, uns, nx, ny, b, zt, ntx, nty, t.xcd);                    \
        else                                                                         \
            heat_vk_fused<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(                 \
                us, ks, rs, uns, nx, ny, b, zt, ntx, nty, t.xcd);                    \
        return hipGetLastError();                                                    \
    }
    if constexpr (std::is_same<P, PrecF64>::value) {
        HC_VK_SHAPES_F64(HC_X)
    } else {
        HC_VK_SHAPES_F32(HC_X)
    }
#undef HC_X
    return hipErrorInvalidValue;
}

hipError_t launch_heat_vk_tile(int dtype, KernelKind kind, const void *u, const void *kap,
                               const void *rhs, void *un, int nx, int ny, double beta,
                               const ZTable &zt, const HeatTiling &t, hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: return launch_vk<PrecF64>(kind, u, kap, rhs, un, nx, ny, beta, zt, t, s);
        case kDtypeF32: return launch_vk<PrecF32>(kind, u, kap, rhs, un, nx, ny, beta, zt, t, s);
        default: return hipErrorInvalidValue;
    }
}

template <class P>
static void vk_plain(const void *u, const void *kap, const void *rhs, void *un, int nx, int ny,
                     int nz, double beta, hipStream_t s) {
    using S = typename P::S;
    using C = typename P::C;
    const dim3 grid((nx - 2 + 63) / 64, (ny - 2 + 3) / 4, nz - 2), block(64, 4);
    heat_vk_plain<P><<<grid, block, 0, s>>>(static_cast<const S *>(u), static_cast<const S *>(kap),
                                            static_cast<const S *>(rhs), static_cast<S *>(un), nx,
                                            ny, nz, (C)beta);
}

hipError_t launch_heat_vk_plain(int dtype, const void *u, const void *kap, const void *rhs,
                                void *un, int nx, int ny, int nz, double beta, hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: vk_plain<PrecF64>(u, kap, rhs, un, nx, ny, nz, beta, s); break;
        case kDtypeF32: vk_plain<PrecF32>(u, kap, rhs, un, nx, ny, nz, beta, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hc
