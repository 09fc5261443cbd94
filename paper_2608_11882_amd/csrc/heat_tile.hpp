#pragma once

// heat_tile.hpp -- the z-marching tile of the 7-point explicit heat update
// (gfx950), shared by the single-problem kernels (heat_kernels.hip) and the
// batched ones (batch_kernels.hip).  Device code only; not exported.
//
// The update is Eq. (4) of the paper with a constant coefficient and no
// source: u_new = u + r * (((x- + x+) + (y- + y+)) + (z- + z+) - 6 u).
// The sum is evaluated in exactly that order and the library is compiled
// without floating-point contraction, so every node is bit-identical to a
// plain serial evaluation of the same expression in the same precision.
//
// Three storage precisions share one kernel body (the Prec traits below):
// FP64 (the paper's precision), FP32, and bfloat16 storage with FP32
// arithmetic (each new value rounded to the nearest bfloat16, ties to even).
//
// Kernel design (2.5-D z-march).  A block owns a tile of VEC*TXL (x) by BY
// (y) nodes -- TXL lanes per row (a multiple of 64, or 16 or 32 so that one
// wavefront covers several short rows), VEC consecutive nodes per lane, 16
// bytes per lane for the wide shapes -- and walks it through a run of planes
// [kb, ke].  Each thread keeps its column's values at k-1, k, k+1 in
// registers, so every stored node is loaded once per z-block.  The current
// plane is staged in LDS (in the arithmetic precision) with a one-node ring
// (two coalesced rows, two columns) for the y neighbours and for the x
// neighbours across lanes; x neighbours inside a lane's VEC nodes come from
// its registers.  An LDS row holds node v of every lane of the row as one
// contiguous run of TXL values (v = 0..VEC-1), so every LDS access of a
// wavefront touches consecutive words (no bank conflicts) and each node
// costs about two LDS reads.  PF planes of loads are in flight while a plane
// is computed.  Results are stored non-temporally: u_new is not read again
// in this step.
//
// Tiles are numbered y fastest, then x, then z-block, and the block ids can
// be regrouped so that runs of y-neighbouring tiles share an XCD's L2 (see
// block_order).

#include "hc_internal.hpp"

#include <type_traits>

namespace hc {

// ---- storage precisions -------------------------------------------------------
struct PrecF64 {
    using S = double;  // stored
    using C = double;  // arithmetic
    static constexpr bool kStochastic = false;
    __device__ static C widen(S v) { return v; }
    __device__ static S narrow(C v) { return v; }
};
struct PrecF32 {
    using S = float;
    using C = float;
    static constexpr bool kStochastic = false;
    __device__ static C widen(S v) { return v; }
    __device__ static S narrow(C v) { return v; }
};
// bfloat16 as its bit pattern: the upper half of a binary32.  Widening is
// exact.  Narrowing uses gfx950's conversion instructions, two values per
// instruction: v_cvt_pk_bf16_f32 rounds to nearest, ties to even, and
// v_cvt_sr_bf16_f32 rounds stochastically -- the magnitude goes up exactly
// when the 16 bits a bfloat16 drops plus the upper 16 bits of its random
// operand carry into the kept part, i.e. with probability (dropped bits) /
// 2^16, which makes the rounding unbiased (values that are already bfloat16
// are kept).  Both keep NaN a NaN.  (Both rules, on every class of finite
// input -- ties, subnormals, values next to the largest finite one -- were
// checked against integer formulas on the device.)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

struct PrecBF16 {
    using S = unsigned short;
    using C = float;
    static constexpr bool kStochastic = false;
    __device__ static C widen(S v) { return __uint_as_float((unsigned)v << 16); }
};
struct PrecBF16SR {
    using S = unsigned short;
    using C = float;
    static constexpr bool kStochastic = true;
    __device__ static C widen(S v) { return PrecBF16::widen(v); }
};

// Key and step of the stochastic rounding (unused by the other precisions).
struct SRKey {
    unsigned k0, k1;  // seed, low and high words
    unsigned t0, t1;  // step index, low and high words
};

namespace {

// Block order.  The hardware deals workgroups to the 8 XCDs round-robin
// (block b runs on XCD b % 8), so consecutive block ids never share an L2.
// With xcd = G > 1 the ids are remapped in windows of 8G blocks: inside a
// window XCD x takes the G consecutive tiles x*G .. x*G+G-1, so runs of G
// neighbouring tiles -- whose halo rows overlap -- are read through one L2,
// while all XCDs still work inside the same window of the array (which keeps
// the DRAM accesses of the whole chip close together).  A last, partial
// window keeps the hardware order.  xcd = 0 or 1: hardware order.
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

// One access of N bytes (2, 4, 8 or 16) as a single load or store.
template <int N> struct Raw;
template <> struct Raw<2> { using T = unsigned short; };
template <> struct Raw<4> { using T = unsigned int; };
template <> struct Raw<8> { using T = u32x2; };
template <> struct Raw<16> { using T = u32x4; };

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of
// two 32x32->64-bit products on counter words 0 and 2, whose halves are
// recombined with words 1 and 3 and the key; the key advances by two Weyl
// constants between rounds.  The key is the same in every lane.
struct U32x4 {
    unsigned x, y, z, w;
};
__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, unsigned k0, unsigned k1) {
    // kept as a loop: unrolled, ten rounds per plane would push the fully
    // unrolled z-march past the compiler's unrolling limit
#pragma unroll 1
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        const U32x4 n = {(unsigned)(p1 >> 32) ^ c.y ^ k0, (unsigned)p1,
                         (unsigned)(p0 >> 32) ^ c.w ^ k1, (unsigned)p0};
        c = n;
    }
    return c;
}

// The 16 random bits of nodes p0 .. p0+VEC-1 (p0 a multiple of VEC, VEC a
// divisor of 8, so all lie in one aligned group of 8 nodes): the group
// g = p0 / 8 draws the block with counter (g, step) and key seed; node p
// takes word (p mod 8) / 2, low half for even p, high half for odd p.  They
// are returned in the upper half of rho[v], where the stochastic conversion
// takes them.
template <int VEC>
__device__ __forceinline__ void sr_bits(long long p0, const SRKey &key, unsigned *rho) {
    const unsigned long long g = (unsigned long long)p0 >> 3;
    const U32x4 w = philox4x32_10({(unsigned)g, (unsigned)(g >> 32), key.t0, key.t1}, key.k0,
                                  key.k1);
    const unsigned wd[4] = {w.x, w.y, w.z, w.w};
    if constexpr (VEC == 8) {  // p0 is a multiple of 8: a fixed assignment
#pragma unroll
        for (int v = 0; v < 8; ++v) rho[v] = (v & 1) ? (wd[v >> 1] & 0xffff0000u) : (wd[v >> 1] << 16);
    } else {
        const unsigned base = (unsigned)p0 & 7u;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const unsigned q = base + v;  // < 8
            const unsigned h = q >> 1;
            const unsigned x = h == 0 ? w.x : h == 1 ? w.y : h == 2 ? w.z : w.w;
            rho[v] = (q & 1u) ? (x & 0xffff0000u) : (x << 16);
        }
    }
}

__device__ __forceinline__ unsigned bf16x2_bits(bf16x2 b) {
    unsigned w;
    __builtin_memcpy(&w, &b, 4);
    return w;
}

// Round VEC new values of nodes p0.. to storage.
template <class P, int VEC>
__device__ __forceinline__ void narrow_vec(const typename P::C *v, typename P::S *o,
                                           long long p0, const SRKey &key) {
    if constexpr (std::is_same<typename P::S, unsigned short>::value) {
        unsigned rho[VEC];
        if constexpr (P::kStochastic) sr_bits<VEC>(p0, key, rho);
#pragma unroll
        for (int e = 0; e < VEC; e += 2) {
            const bool pair = e + 1 < VEC;
            unsigned bits;
            if constexpr (P::kStochastic) {
                bf16x2 b = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2{}, v[e], rho[e], false);
                if (pair) b = __builtin_amdgcn_cvt_sr_bf16_f32(b, v[e + 1], rho[e + 1], true);
                bits = bf16x2_bits(b);
            } else {
                bits = bf16x2_bits(
                    __builtin_convertvector(f32x2{v[e], pair ? v[e + 1] : v[e]}, bf16x2));
            }
            o[e] = (unsigned short)bits;
            if (pair) o[e + 1] = (unsigned short)(bits >> 16);
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = P::narrow(v[e]);
    }
}

template <class P, int VEC>
__device__ __forceinline__ void load_vec(const typename P::S *__restrict__ p,
                                         typename P::C *o) {
    using R = typename Raw<VEC * sizeof(typename P::S)>::T;
    const R raw = *reinterpret_cast<const R *>(p);
    typename P::S s[VEC];
    __builtin_memcpy(s, &raw, sizeof raw);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = P::widen(s[v]);
}

template <class P, int VEC>
__device__ __forceinline__ void store_vec_nt(typename P::S *__restrict__ p,
                                             const typename P::C *v, long long p0,
                                             const SRKey &key) {
    using R = typename Raw<VEC * sizeof(typename P::S)>::T;
    typename P::S s[VEC];
    narrow_vec<P, VEC>(v, s, p0, key);
    R raw;
    __builtin_memcpy(&raw, s, sizeof raw);
    __builtin_nontemporal_store(raw, reinterpret_cast<R *>(p));
}

// Loads are never predicated: a node outside the array is read at a clamped
// in-bounds address instead, and such values only ever reach lanes whose own
// nodes are not updated.  Those lanes store their own (unchanged) values
// back to Dirichlet nodes of un -- the same bits the face copy put there --
// so the store is not predicated either: a lane whose nodes lie in the array
// stores to them, a lane past the last column or row stores to the Dirichlet
// row ny-1.  With no branch around a memory access every wave issues the
// same accesses each plane, and the compiler waits only for the loads a
// plane needs.
//
// A z-range of at least ZB planes takes the fast path, in sub-blocks of
// exactly ZB planes: the march of a sub-block is fully unrolled, so the register queue along z is renamed rather than copied
// (a copy would have to wait for the load in flight) and PF planes of loads
// stay in flight behind the plane being computed.  The last z-block of a
// range is shifted back to a full ZB planes; the planes it shares with the
// block before are computed twice and written twice with identical bits.
// Ranges shorter than ZB (the Boundary planes) take the generic loop.

// LDS row layout (LD values): [left ring column] [node 0 of lanes
// 0..TXL-1] [node 1 of every lane] ... [node VEC-1 of every lane] [right
// ring column]; rows 0 and BY+1 are the ring rows.  Thread t works on lane
// t % TXL of tile row t / TXL.
//
// Rows are `pitch` nodes apart in memory (pitch >= nx, a multiple of VEC;
// the nodes past nx are padding that no update reads).  A lane whose VEC
// nodes reach past nx is not updated there and writes back what it read.
template <int VEC, int TXL, int BY>
struct TileGeom {
    static constexpr int TX = VEC * TXL;       // tile width in nodes
    static constexpr int LD = TX + 2;          // LDS row stride
    static constexpr int NT = TXL * BY;        // threads per block
    static constexpr int RROW = TXL;           // threads per ring row
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(NT >= 2 * RROW + 2 * BY, "one thread per ring element");
    int kb, ke;
    long long plane, own, ring;  // ring: VEC-aligned offset of the ring load
    bool st[VEC];
    int own_slot;          // LDS slot of the lane's node 0 (node v: + v*TXL)
    int xm_slot, xp_slot;  // LDS slots of the left neighbour of node 0 and
                           // the right neighbour of node VEC-1
    int rslot;             // LDS slot of the ring element (node v: + v*TXL)
    bool rvec;  // ring element is a VEC-wide row piece (else one node)
    int rsel;   // the node's index within the aligned VEC-wide ring load

    // Thread t of the block that sweeps tile (tx, ty) of an nx x ny plane
    // with rows `pitch` apart (x-tiles of TX nodes from x = 0, y-tiles of BY
    // rows from y = 1), planes kb_..ke_ (host-callable, so that the offsets
    // can be checked on the CPU).
    __host__ __device__ TileGeom(int t, int nx, int pitch, int ny, int tx, int ty, int kb_,
                                 int ke_) {
        kb = kb_;
        ke = ke_;
        const int gl = t % TXL;      // lane index within the tile row
        const int wy = t / TXL;      // tile row
        const int i0 = tx * TX;
        const int j0 = 1 + ty * BY;  // first updated row of the tile
        const int ia = i0 + gl * VEC;
        const int j = j0 + wy;
        plane = (long long)pitch * ny;
        if (ia >= nx)  // past the last column: Dirichlet row ny-1
            own = (long long)(ny - 1) * pitch + (pitch - VEC);
        else
            own = (long long)min(j, ny - 1) * pitch + ia;
#pragma unroll
        for (int v = 0; v < VEC; ++v) st[v] = (ia + v >= 1) && (ia + v <= nx - 2) && (j <= ny - 2);
        const int rowb = (wy + 1) * LD;
        own_slot = rowb + 1 + gl;
        xm_slot = gl == 0 ? rowb : own_slot - 1 + (VEC - 1) * TXL;
        xp_slot = gl == TXL - 1 ? rowb + TX + 1 : own_slot + 1;

        // ring of the LDS tile: rows j0-1 and j0+BY (VEC nodes per thread,
        // coalesced), then columns i0-1 and i0+TX (one node per thread).
        // Every thread issues one VEC-wide aligned ring load (a column node
        // is taken out of the aligned VEC nodes that hold it), so the load
        // is the same instruction in every lane.
        rvec = false;
        rslot = -1;
        rsel = 0;
        if (t < 2 * RROW) {
            const int row = t / RROW, q = t % RROW;
            const int rj = row == 0 ? j0 - 1 : min(j0 + BY, ny - 1);
            ring = (long long)rj * pitch + min(i0 + q * VEC, pitch - VEC);
            rslot = (row == 0 ? 0 : (BY + 1) * LD) + 1 + q;
            rvec = true;
        } else if (t < 2 * RROW + 2 * BY) {
            const int q = t - 2 * RROW;
            const int row = q % BY, side = q / BY;
            const int ri = max(0, min(side == 0 ? i0 - 1 : i0 + TX, nx - 1));
            rsel = ri % VEC;
            ring = (long long)min(j0 + row, ny - 1) * pitch + (ri - rsel);
            rslot = (row + 1) * LD + (side == 0 ? 0 : TX + 1);
        } else {
            ring = own;
        }
    }
};

// The tile and z-block of this block in a launch over table zt: tiles are
// numbered y fastest (runs of tiles share halo rows), then x, then z-block;
// the last z-block of a range is shifted back to a full zb_full planes.
template <int VEC, int TXL, int BY>
__device__ __forceinline__ TileGeom<VEC, TXL, BY> block_tile(int nx, int ny, const ZTable &zt,
                                                            int ntx, int nty, int xcd,
                                                            int zb_full) {
    const int L = block_order(blockIdx.x, gridDim.x, xcd);
    const int ty = L % nty;
    const int rest = L / nty;
    const int tx = rest % ntx;
    const int z = rest / ntx;
    int rg = 0;
    while (rg + 1 < zt.n && z >= zt.first[rg + 1]) ++rg;
    int k0 = zt.kb[rg] + (z - zt.first[rg]) * zt.depth[rg];
    if (zt.depth[rg] == zb_full && zt.ke[rg] - zt.kb[rg] + 1 >= zb_full)
        k0 = min(k0, zt.ke[rg] - zb_full + 1);
    return TileGeom<VEC, TXL, BY>((int)threadIdx.x, nx, nx, ny, tx, ty, k0,
                                  min(k0 + zt.depth[rg] - 1, zt.ke[rg]));
}

// LDS values a tile of this shape stages (the plane and its ring).
template <int VEC, int TXL, int BY>
constexpr int tile_lds_elems() {
    return (BY + 2) * (VEC * TXL + 2);
}

// Sweep one tile (geometry g) of u into un: planes g.kb .. g.ke, staging
// planes in `tile` (LDS, tile_lds_elems<VEC, TXL, BY>() values).
template <class P, int VEC, int TXL, int BY, int PF, int ZB>
__device__ __forceinline__ void heat_tile_sweep(const typename P::S *__restrict__ u,
                                                typename P::S *__restrict__ un,
                                                typename P::C r,
                                                const TileGeom<VEC, TXL, BY> &g,
                                                const SRKey &key, typename P::C *tile) {
    using C = typename P::C;
    using S = typename P::S;
    using G = TileGeom<VEC, TXL, BY>;
    static_assert(PF >= 1 && PF <= 4 && PF < ZB, "prefetch depth 1 to 4");
    const long long plane = g.plane;
    const S *__restrict__ uo = u + g.own;
    const S *__restrict__ ur = u + g.ring;
    S *__restrict__ vo = un + g.own;
    const int kb = g.kb, ke = g.ke;

    // ring values of plane k: one aligned VEC-wide load in every lane; a
    // column thread keeps the node it needs in o[0]
    auto ld_ring = [&](long long kp, C *o) {
        load_vec<P, VEC>(ur + kp, o);
        if (!g.rvec) {
            C sel = o[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) sel = (g.rsel == e) ? o[e] : sel;
            o[0] = sel;
        }
    };
    auto put = [&](const C *c, const C *gv) {
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
    auto update = [&](const C *zm, const C *c, const C *zp, C *out) {
        const C xm0 = tile[g.xm_slot];
        const C xpl = tile[g.xp_slot];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int sl = g.own_slot + v * TXL;
            const C xm = v == 0 ? xm0 : c[v - 1];
            const C xp = v == VEC - 1 ? xpl : c[v + 1];
            const C ym = tile[sl - G::LD];
            const C yp = tile[sl + G::LD];
            const C nsum = ((xm + xp) + (ym + yp)) + (zm[v] + zp[v]);
            const C lap = nsum - C(6) * c[v];
            C res = c[v] + r * lap;
            // every lane computes the update and then selects, so the LDS
            // reads above stay unconditional: otherwise the compiler sinks
            // them behind a branch per node, each with its own wait
            asm volatile("" : "+v"(res));
            out[v] = g.st[v] ? res : c[v];
        }
    };

    if (ke - kb + 1 >= ZB) {
        // sub-blocks of exactly ZB planes from kb on, the last one shifted
        // back to end at ke (its planes shared with the one before are
        // computed and written twice, with the same bits); a sub-block's
        // first two planes were loaded by the one before and come from cache
        for (int k0 = kb;; k0 += ZB) {
            const int k1 = min(k0, ke - ZB + 1);
            // q[s] = column values of plane k1-1+s, gr[s] = ring of plane k1+s
            C q[ZB + 2][VEC];
            C gr[ZB][VEC];
#pragma unroll
            for (int s = 0; s < PF + 2; ++s)
                load_vec<P, VEC>(uo + (long long)(k1 - 1 + s) * plane, q[s]);
#pragma unroll
            for (int s = 0; s < PF; ++s) ld_ring((long long)(k1 + s) * plane, gr[s]);
#pragma unroll
            for (int s = 0; s < ZB; ++s) {
                const long long kp = (long long)(k1 + s) * plane;
                __syncthreads();  // the previous plane's LDS reads are done
                put(q[s + 1], gr[s]);
                if (s + PF < ZB) ld_ring(kp + PF * plane, gr[s + PF]);
                __syncthreads();
                C out[VEC];
                update(q[s], q[s + 1], q[s + 2], out);
                store_vec_nt<P, VEC>(vo + kp, out, g.own + kp, key);
                if (s + 2 + PF <= ZB + 1)
                    load_vec<P, VEC>(uo + kp + (1 + PF) * plane, q[s + 2 + PF]);
            }
            if (k1 == ke - ZB + 1) break;
        }
        return;
    }

    // generic depth (short ranges): one plane of loads ahead
    C zm[VEC], c[VEC], zp[VEC], g0[VEC];
    load_vec<P, VEC>(uo + (long long)(kb - 1) * plane, zm);
    load_vec<P, VEC>(uo + (long long)kb * plane, c);
    load_vec<P, VEC>(uo + (long long)(kb + 1) * plane, zp);
    ld_ring((long long)kb * plane, g0);
    for (int k = kb; k <= ke; ++k) {
        const long long kp = (long long)k * plane;
        C zn[VEC], gn[VEC];
        load_vec<P, VEC>(uo + (long long)min(k + 2, ke + 1) * plane, zn);
        ld_ring((long long)min(k + 1, ke) * plane, gn);
        __syncthreads();
        put(c, g0);
        __syncthreads();
        C out[VEC];
        update(zm, c, zp, out);
        store_vec_nt<P, VEC>(vo + kp, out, g.own + kp, key);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            zm[v] = c[v];
            c[v] = zp[v];
            zp[v] = zn[v];
            g0[v] = gn[v];
        }
    }
}

}  // namespace
}  // namespace hc
