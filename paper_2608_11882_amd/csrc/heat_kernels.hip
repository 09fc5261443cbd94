// heat_kernels.hip -- 7-point explicit heat update for gfx950 (FP64).
//
// The update is Eq. (4) of the paper with a constant coefficient and no
// source: u_new = u + r * (((x- + x+) + (y- + y+)) + (z- + z+) - 6 u).
// The sum is evaluated in exactly that order and the library is compiled
// without floating-point contraction, so every node is bit-identical to a
// plain serial evaluation of the same expression.
//
// Kernel design (2.5-D z-march).  A block owns a tile of 64 (x) by BY (y)
// nodes and walks it through a run of planes [kb, ke].  Each thread keeps
// its column's values at k-1, k, k+1 in registers, so every stored node is
// loaded once per z-block; the x/y neighbours come from the current plane
// staged in LDS with a one-node ring.  The ring's two rows are coalesced
// 64-wide loads, its two columns are one node per row.  The next plane is
// loaded before the current one is computed, so one plane of loads is
// always in flight per wave.  Results are stored non-temporally: u_new is
// not read again in this step, so it should not evict u from L2.
//
// Block order is XCD-aware: the hardware deals consecutive workgroups to
// the 8 XCDs round-robin, so the block id is remapped to make each XCD walk
// a contiguous run of tiles (neighbouring tiles, whose halos overlap, then
// share one L2).  Tiles are numbered x fastest, then y, then z-block.

#include "hc_internal.hpp"

#include <climits>

namespace hc {
namespace {

constexpr int kLd = kTileX + 2;  // LDS row stride (tile row plus ring)

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    constexpr int kXcd = 8;
    const int xcd = bid % kXcd, slot = bid / kXcd;
    const int per = nblk / kXcd, rem = nblk % kXcd;
    return xcd * per + min(xcd, rem) + slot;
}

// Loads are never predicated: a node outside the array is read at a clamped
// in-bounds address instead, and such values only ever reach lanes whose own
// node is not updated.  Those lanes store their own (unchanged) value back
// to a Dirichlet node of un -- the same bits the face copy put there -- so
// the store is not predicated either.  With no branch around a memory
// access every wave issues the same accesses each plane, and the compiler
// waits only for the loads a plane needs.
//
// A z-block of exactly ZB planes takes the fast path: the march is fully
// unrolled, so the register queue along z is renamed rather than copied
// (a copy would have to wait for the load in flight) and PF planes of loads
// stay in flight behind the plane being computed.  The last z-block of a
// range is shifted back to a full ZB planes; the planes it shares with the
// block before are computed twice and written twice with identical bits.
// Ranges shorter than ZB (the Boundary planes) take the generic loop.

struct TileGeom {
    int kb, ke;
    long long plane, own, ring;
    bool own_st;
    int own_slot, rslot;
};

template <int BY>
__device__ __forceinline__ TileGeom tile_geom(int nx, int ny, const ZTable &zt,
                                              int ntx, int nty, int xcd,
                                              int zb_full) {
    TileGeom g;
    const int L = xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tx = L % ntx;
    const int rest = L / ntx;
    const int ty = rest % nty;
    const int z = rest / nty;
    int rg = 0;
    while (rg + 1 < zt.n && z >= zt.first[rg + 1]) ++rg;
    int kb = zt.kb[rg] + (z - zt.first[rg]) * zt.depth[rg];
    if (zt.depth[rg] == zb_full && zt.ke[rg] - zt.kb[rg] + 1 >= zb_full)
        kb = min(kb, zt.ke[rg] - zb_full + 1);  // full-depth last block
    g.kb = kb;
    g.ke = min(kb + zt.depth[rg] - 1, zt.ke[rg]);

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int i0 = tx * kTileX;
    const int j0 = 1 + ty * BY;  // first updated row of the tile
    const int i = i0 + lane;
    const int j = j0 + w;
    g.plane = (long long)nx * ny;
    g.own = (long long)min(j, ny - 1) * nx + min(i, nx - 1);
    g.own_st = (i >= 1) && (i <= nx - 2) && (j <= ny - 2);
    g.own_slot = (w + 1) * kLd + lane + 1;

    // ring of the LDS tile, one node per thread: rows j0-1 and j0+BY (64
    // nodes each, coalesced), then columns i0-1 and i0+64 (BY nodes each)
    constexpr int kRing = 2 * kTileX + 2 * BY;
    const int e = threadIdx.x;
    int ri, rj, rslot;
    if (e < kTileX) {
        ri = i0 + e; rj = j0 - 1; rslot = e + 1;
    } else if (e < 2 * kTileX) {
        ri = i0 + e - kTileX; rj = j0 + BY; rslot = (BY + 1) * kLd + (e - kTileX) + 1;
    } else if (e < 2 * kTileX + BY) {
        ri = i0 - 1; rj = j0 + (e - 2 * kTileX); rslot = (e - 2 * kTileX + 1) * kLd;
    } else if (e < kRing) {
        ri = i0 + kTileX; rj = j0 + (e - 2 * kTileX - BY);
        rslot = (e - 2 * kTileX - BY + 1) * kLd + kTileX + 1;
    } else {
        ri = i; rj = j; rslot = -1;
    }
    g.ring = (long long)min(rj, ny - 1) * nx + max(0, min(ri, nx - 1));
    g.rslot = rslot;
    return g;
}

// One plane: stage the column value and the ring in LDS, then update.
template <int BY>
__device__ __forceinline__ double plane_update(double *tile, const TileGeom &g,
                                               double zm, double c, double zp,
                                               double ringv, double r) {
    (void)BY;
    const double xm = tile[g.own_slot - 1];
    const double xp = tile[g.own_slot + 1];
    const double ym = tile[g.own_slot - kLd];
    const double yp = tile[g.own_slot + kLd];
    const double nsum = ((xm + xp) + (ym + yp)) + (zm + zp);
    const double lap = nsum - 6.0 * c;
    (void)ringv;
    return g.own_st ? c + r * lap : c;
}

template <int BY, int PF, int ZB>
__device__ __forceinline__ void heat_tile_sweep(const double *__restrict__ u,
                                                double *__restrict__ un, int nx,
                                                int ny, double r,
                                                const ZTable &zt, int ntx,
                                                int nty, int xcd) {
    static_assert(64 * BY >= 2 * kTileX + 2 * BY, "one thread per ring node");
    static_assert(PF >= 1 && PF <= 3, "prefetch depth 1..3");
    __shared__ double tile[(BY + 2) * kLd];
    const TileGeom g = tile_geom<BY>(nx, ny, zt, ntx, nty, xcd, ZB);
    const long long plane = g.plane;
    const double *__restrict__ uo = u + g.own;
    const double *__restrict__ ur = u + g.ring;
    double *__restrict__ vo = un + g.own;
    const int kb = g.kb, ke = g.ke;

    if (ke - kb + 1 == ZB) {
        // q[s] = column value of plane kb-1+s, ring[s] = ring of plane kb+s
        double q[ZB + 2];
        double ring[ZB];
#pragma unroll
        for (int s = 0; s < PF + 2; ++s) q[s] = uo[(long long)(kb - 1 + s) * plane];
#pragma unroll
        for (int s = 0; s < PF; ++s) ring[s] = ur[(long long)(kb + s) * plane];
#pragma unroll
        for (int s = 0; s < ZB; ++s) {
            const long long kp = (long long)(kb + s) * plane;
            __syncthreads();  // the previous plane's LDS reads are done
            tile[g.own_slot] = q[s + 1];
            if (g.rslot >= 0) tile[g.rslot] = ring[s];
            if (s + PF < ZB) ring[s + PF] = ur[kp + PF * plane];
            __syncthreads();
            const double out = plane_update<BY>(tile, g, q[s], q[s + 1], q[s + 2], 0.0, r);
            __builtin_nontemporal_store(out, vo + kp);
            if (s + 2 + PF <= ZB + 1) q[s + 2 + PF] = uo[kp + (1 + PF) * plane];
        }
        return;
    }

    // generic depth (short ranges): one plane of loads ahead
    double zm = uo[(long long)(kb - 1) * plane];
    double c = uo[(long long)kb * plane];
    double zp = uo[(long long)(kb + 1) * plane];
    double g0 = ur[(long long)kb * plane];
    for (int k = kb; k <= ke; ++k) {
        const long long kp = (long long)k * plane;
        const double zn = uo[(long long)min(k + 2, ke + 1) * plane];
        const double gn = ur[(long long)min(k + 1, ke) * plane];
        __syncthreads();
        tile[g.own_slot] = c;
        if (g.rslot >= 0) tile[g.rslot] = g0;
        __syncthreads();
        const double out = plane_update<BY>(tile, g, zm, c, zp, 0.0, r);
        __builtin_nontemporal_store(out, vo + kp);
        zm = c;
        c = zp;
        zp = zn;
        g0 = gn;
    }
}

// Three entry points with one body, so that profiles name the role.
template <int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * BY) void heat_interior_f64(
    const double *__restrict__ u, double *__restrict__ un, int nx, int ny,
    double r, ZTable zt, int ntx, int nty, int xcd) {
    heat_tile_sweep<BY, PF, ZB>(u, un, nx, ny, r, zt, ntx, nty, xcd);
}

template <int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * BY) void heat_boundary_f64(
    const double *__restrict__ u, double *__restrict__ un, int nx, int ny,
    double r, ZTable zt, int ntx, int nty, int xcd) {
    heat_tile_sweep<BY, PF, ZB>(u, un, nx, ny, r, zt, ntx, nty, xcd);
}

template <int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * BY) void heat_fused_f64(
    const double *__restrict__ u, double *__restrict__ un, int nx, int ny,
    double r, ZTable zt, int ntx, int nty, int xcd) {
    heat_tile_sweep<BY, PF, ZB>(u, un, nx, ny, r, zt, ntx, nty, xcd);
}

// One thread per interior node, all seven values loaded from memory: the
// straightforward form (the paper's collapse(3) loop mapped onto a grid).
__global__ __launch_bounds__(256) void heat_plain_f64(
    const double *__restrict__ u, double *__restrict__ un, int nx, int ny,
    int nz, double r) {
    const int i = 1 + (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int j = 1 + (int)blockIdx.y * 4 + (int)threadIdx.y;
    const int k = 1 + (int)blockIdx.z;
    if (i > nx - 2 || j > ny - 2 || k > nz - 2) return;
    const long long sy = nx, sz = (long long)nx * ny;
    const long long p = (long long)k * sz + (long long)j * sy + i;
    const double c = u[p];
    const double nsum = ((u[p - 1] + u[p + 1]) + (u[p - sy] + u[p + sy])) +
                        (u[p - sz] + u[p + sz]);
    const double lap = nsum - 6.0 * c;
    un[p] = c + r * lap;
}

// Copy the outermost layer (the Dirichlet data) of u into un.
__global__ __launch_bounds__(256) void copy_faces_f64(
    const double *__restrict__ u, double *__restrict__ un, int nx, int ny,
    int nz) {
    const long long plane = (long long)nx * ny;
    const long long per_mid = 2LL * nx + 2LL * (ny - 2);  // per inner plane
    const long long total = 2 * plane + (long long)(nz - 2) * per_mid;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
         t < total; t += (long long)gridDim.x * blockDim.x) {
        long long off;
        if (t < 2 * plane) {
            off = (t < plane) ? t : (long long)(nz - 1) * plane + (t - plane);
        } else {
            const long long s = t - 2 * plane;
            const long long k = 1 + s / per_mid;
            const long long q = s % per_mid;
            long long jj, ii;
            if (q < 2LL * nx) {
                jj = (q < nx) ? 0 : ny - 1;
                ii = q % nx;
            } else {
                const long long q2 = q - 2LL * nx;
                jj = 1 + q2 / 2;
                ii = (q2 & 1) ? nx - 1 : 0;
            }
            off = k * plane + jj * nx + ii;
        }
        un[off] = u[off];
    }
}

}  // namespace

int ztable_blocks(const ZTable &zt) { return zt.n > 0 ? zt.first[zt.n] : 0; }

long long heat_tile_blocks(int nx, int ny, int by, const ZTable &zt) {
    const long long ntx = (nx + kTileX - 1) / kTileX;
    const long long nty = (ny - 2 + by - 1) / by;
    return ntx * nty * (long long)ztable_blocks(zt);
}

hipError_t launch_heat_tile_f64(KernelKind kind, const double *u, double *un,
                                int nx, int ny, int nz, double r,
                                const ZTable &zt, const HeatTiling &t,
                                hipStream_t s) {
    (void)nz;
    const long long nb = heat_tile_blocks(nx, ny, t.by, zt);
    if (nb <= 0) return hipSuccess;
    if (nb > INT_MAX) return hipErrorInvalidConfiguration;
    const int ntx = (nx + kTileX - 1) / kTileX;
    const int nty = (ny - 2 + t.by - 1) / t.by;
    const dim3 grid((unsigned)nb), block(64 * t.by);
#define HC_HEAT_LAUNCH(BYV, PFV, ZBV)                                            \
    do {                                                                         \
        if (kind == K_HEAT_INTERIOR)                                             \
            heat_interior_f64<BYV, PFV, ZBV><<<grid, block, 0, s>>>(             \
                u, un, nx, ny, r, zt, ntx, nty, t.xcd);                          \
        else if (kind == K_HEAT_BOUNDARY)                                        \
            heat_boundary_f64<BYV, PFV, ZBV><<<grid, block, 0, s>>>(             \
                u, un, nx, ny, r, zt, ntx, nty, t.xcd);                          \
        else                                                                     \
            heat_fused_f64<BYV, PFV, ZBV><<<grid, block, 0, s>>>(                \
                u, un, nx, ny, r, zt, ntx, nty, t.xcd);                          \
    } while (0)
#define HC_HEAT_CASE(BYV, PFV, ZBV) \
    case (BYV * 100 + PFV * 10000 + ZBV): HC_HEAT_LAUNCH(BYV, PFV, ZBV); break
    switch (t.pf * 10000 + t.by * 100 + t.zdepth) {
        HC_HEAT_CASE(4, 1, 16); HC_HEAT_CASE(4, 1, 32); HC_HEAT_CASE(4, 1, 64);
        HC_HEAT_CASE(4, 2, 16); HC_HEAT_CASE(4, 2, 32); HC_HEAT_CASE(4, 2, 64);
        HC_HEAT_CASE(4, 3, 16); HC_HEAT_CASE(4, 3, 32); HC_HEAT_CASE(4, 3, 64);
        HC_HEAT_CASE(8, 1, 16); HC_HEAT_CASE(8, 1, 32); HC_HEAT_CASE(8, 1, 64);
        HC_HEAT_CASE(8, 2, 16); HC_HEAT_CASE(8, 2, 32); HC_HEAT_CASE(8, 2, 64);
        HC_HEAT_CASE(8, 3, 16); HC_HEAT_CASE(8, 3, 32); HC_HEAT_CASE(8, 3, 64);
        HC_HEAT_CASE(16, 1, 16); HC_HEAT_CASE(16, 1, 32);
        HC_HEAT_CASE(16, 2, 16); HC_HEAT_CASE(16, 2, 32);
        default: return hipErrorInvalidValue;
    }
#undef HC_HEAT_CASE
#undef HC_HEAT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_heat_plain_f64(const double *u, double *un, int nx, int ny,
                                 int nz, double r, hipStream_t s) {
    const dim3 grid((nx - 2 + 63) / 64, (ny - 2 + 3) / 4, nz - 2),
        block(64, 4);
    heat_plain_f64<<<grid, block, 0, s>>>(u, un, nx, ny, nz, r);
    return hipGetLastError();
}

hipError_t launch_copy_faces_f64(const double *u, double *un, int nx, int ny,
                                 int nz, hipStream_t s) {
    const long long total =
        2LL * nx * ny + (long long)(nz - 2) * (2LL * nx + 2LL * (ny - 2));
    long long nb = (total + 255) / 256;
    if (nb > 4096) nb = 4096;
    copy_faces_f64<<<(unsigned)nb, 256, 0, s>>>(u, un, nx, ny, nz);
    return hipGetLastError();
}

}  // namespace hc
