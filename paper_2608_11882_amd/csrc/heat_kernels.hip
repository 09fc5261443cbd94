// heat_kernels.hip -- single-problem kernels of the 7-point explicit heat
// update for gfx950: the Interior / Boundary / fused z-marching sweeps (one
// block per tile and z-block, the tile body in heat_tile.hpp), the
// one-thread-per-node form, and the copy of the Dirichlet layer.

#include "heat_tile.hpp"

#include <climits>
#include <type_traits>

namespace hc {
namespace {

// Three entry points with one body, so that profiles name the role.
template <class P, int VEC, int WX, int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void heat_interior(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un, int nx,
    int ny, typename P::C r, ZTable zt, int ntx, int nty, int xcd, SRKey key) {
    __shared__ typename P::C tile[tile_lds_elems<VEC, 64 * WX, BY>()];
    const auto g = block_tile<VEC, 64 * WX, BY>(nx, ny, zt, ntx, nty, xcd, ZB);
    heat_tile_sweep<P, VEC, 64 * WX, BY, PF, ZB>(u, un, r, g, key, tile);
}

template <class P, int VEC, int WX, int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void heat_boundary(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un, int nx,
    int ny, typename P::C r, ZTable zt, int ntx, int nty, int xcd, SRKey key) {
    __shared__ typename P::C tile[tile_lds_elems<VEC, 64 * WX, BY>()];
    const auto g = block_tile<VEC, 64 * WX, BY>(nx, ny, zt, ntx, nty, xcd, ZB);
    heat_tile_sweep<P, VEC, 64 * WX, BY, PF, ZB>(u, un, r, g, key, tile);
}

template <class P, int VEC, int WX, int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void heat_fused(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un, int nx,
    int ny, typename P::C r, ZTable zt, int ntx, int nty, int xcd, SRKey key) {
    __shared__ typename P::C tile[tile_lds_elems<VEC, 64 * WX, BY>()];
    const auto g = block_tile<VEC, 64 * WX, BY>(nx, ny, zt, ntx, nty, xcd, ZB);
    heat_tile_sweep<P, VEC, 64 * WX, BY, PF, ZB>(u, un, r, g, key, tile);
}

// One thread per interior node, all seven values loaded from memory: the
// straightforward form (the paper's collapse(3) loop mapped onto a grid).
template <class P>
__global__ __launch_bounds__(256) void heat_plain(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un, int nx,
    int ny, int nz, typename P::C r, SRKey key) {
    using C = typename P::C;
    const int i = 1 + (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int j = 1 + (int)blockIdx.y * 4 + (int)threadIdx.y;
    const int k = 1 + (int)blockIdx.z;
    if (i > nx - 2 || j > ny - 2 || k > nz - 2) return;
    const long long sy = nx, sz = (long long)nx * ny;
    const long long p = (long long)k * sz + (long long)j * sy + i;
    const C c = P::widen(u[p]);
    const C nsum = ((P::widen(u[p - 1]) + P::widen(u[p + 1])) +
                    (P::widen(u[p - sy]) + P::widen(u[p + sy]))) +
                   (P::widen(u[p - sz]) + P::widen(u[p + sz]));
    const C lap = nsum - C(6) * c;
    const C out = c + r * lap;
    narrow_vec<P, 1>(&out, &un[p], p, key);
}

// Copy the outermost layer (the Dirichlet data) of u into un.
template <class T>
__global__ __launch_bounds__(256) void copy_faces(const T *__restrict__ u,
                                                  T *__restrict__ un, int nx,
                                                  int ny, int nz) {
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

int tile_width(const HeatTiling &t) { return 64 * t.vec * t.wx; }

long long heat_tile_blocks(int nx, int ny, const HeatTiling &t, const ZTable &zt) {
    const long long tx = tile_width(t);
    const long long ntx = (nx + tx - 1) / tx;
    long long nty = (ny - 2 + t.by - 1) / t.by;
    if (t.xcd < 0) nty = 8 * ((nty + 7) / 8);  // slab order: whole slabs per XCD
    return ntx * nty * (long long)ztable_blocks(zt);
}

// Every tile shape the library is built with, per precision:
// X(vec, wx, by, pf, zdepth).  Arrays that do not allow wide lanes fall
// back to (1, 4, 4, 2, 16), which every list holds.
#define HC_HEAT_SHAPES_F64(X)                                                     \
    X(1, 4, 4, 2, 16) X(1, 1, 4, 1, 16) X(1, 1, 8, 2, 16) X(1, 1, 16, 2, 16)     \
    X(1, 4, 4, 2, 32) X(2, 1, 8, 2, 16) X(2, 1, 16, 2, 32) X(2, 2, 8, 2, 16)     \
    X(2, 2, 8, 2, 32) X(2, 2, 8, 2, 64) X(2, 4, 4, 1, 16) X(2, 4, 4, 2, 16)      \
    X(2, 4, 4, 2, 32) X(2, 4, 4, 2, 64) X(2, 4, 4, 3, 32) X(2, 4, 4, 4, 32)
#define HC_HEAT_SHAPES_F32(X)                                                     \
    X(1, 4, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 1, 8, 2, 32) X(2, 4, 4, 2, 32)      \
    X(4, 1, 8, 2, 32) X(4, 1, 16, 2, 32) X(4, 2, 4, 2, 32) X(4, 2, 8, 2, 16)     \
    X(4, 2, 8, 2, 32) X(4, 4, 4, 2, 16) X(4, 4, 4, 2, 32) X(4, 2, 8, 1, 32)       \
    X(4, 4, 4, 3, 16) X(4, 4, 4, 4, 16)
#define HC_HEAT_SHAPES_BF16(X)                                                    \
    X(1, 4, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 1, 8, 2, 16) X(4, 1, 8, 2, 16)      \
    X(4, 2, 8, 2, 32) X(4, 4, 4, 2, 32) X(8, 1, 4, 2, 32) X(8, 1, 8, 2, 16)      \
    X(8, 1, 8, 2, 32) X(8, 1, 16, 2, 32) X(8, 2, 4, 2, 32) X(8, 2, 8, 2, 32)

#define HC_SHAPE_KEY(V, W, B, P, Z) ((((V * 8 + W) * 32 + B) * 8 + P) * 128 + Z)

bool heat_tiling_supported(int dtype, const HeatTiling &t) {
    const int key = HC_SHAPE_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, P, Z) if (key == HC_SHAPE_KEY(V, W, B, P, Z)) return true;
    if (dtype == 0) { HC_HEAT_SHAPES_F64(HC_X) }
    if (dtype == 1) { HC_HEAT_SHAPES_F32(HC_X) }
    if (dtype == 2 || dtype == 3) { HC_HEAT_SHAPES_BF16(HC_X) }
#undef HC_X
    return false;
}

template <class P>
static hipError_t launch_tile(KernelKind kind, const void *u, void *un, int nx, int ny,
                              double r, const ZTable &zt, const HeatTiling &t,
                              const SRKey &key, hipStream_t s) {
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
    S *uns = static_cast<S *>(un);
    const C rc = (C)r;
    const int shape = HC_SHAPE_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, PF, Z)                                                     \
    if (shape == HC_SHAPE_KEY(V, W, B, PF, Z)) {                                 \
        if (kind == K_HEAT_INTERIOR)                                             \
            heat_interior<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(             \
                us, uns, nx, ny, rc, zt, ntx, nty, t.xcd, key);                  \
        else if (kind == K_HEAT_BOUNDARY)                                        \
            heat_boundary<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(             \
                us, uns, nx, ny, rc, zt, ntx, nty, t.xcd, key);                  \
        else                                                                     \
            heat_fused<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(                \
                us, uns, nx, ny, rc, zt, ntx, nty, t.xcd, key);                  \
        return hipGetLastError();                                                \
    }
    if constexpr (std::is_same<P, PrecF64>::value) {
        HC_HEAT_SHAPES_F64(HC_X)
    } else if constexpr (std::is_same<P, PrecF32>::value) {
        HC_HEAT_SHAPES_F32(HC_X)
    } else {  // both bfloat16 forms
        HC_HEAT_SHAPES_BF16(HC_X)
    }
#undef HC_X
    return hipErrorInvalidValue;
}

static SRKey make_key(unsigned long long seed, unsigned long long step) {
    return {(unsigned)seed, (unsigned)(seed >> 32), (unsigned)step, (unsigned)(step >> 32)};
}

hipError_t launch_heat_tile(int dtype, KernelKind kind, const void *u, void *un, int nx,
                            int ny, double r, const ZTable &zt, const HeatTiling &t,
                            unsigned long long seed, unsigned long long step, hipStream_t s) {
    const SRKey key = make_key(seed, step);
    switch (dtype) {
        case kDtypeF64: return launch_tile<PrecF64>(kind, u, un, nx, ny, r, zt, t, key, s);
        case kDtypeF32: return launch_tile<PrecF32>(kind, u, un, nx, ny, r, zt, t, key, s);
        case kDtypeBF16: return launch_tile<PrecBF16>(kind, u, un, nx, ny, r, zt, t, key, s);
        case kDtypeBF16SR: return launch_tile<PrecBF16SR>(kind, u, un, nx, ny, r, zt, t, key, s);
        default: return hipErrorInvalidValue;
    }
}

template <class P>
static void plain(const void *u, void *un, int nx, int ny, int nz, double r, const SRKey &key,
                  hipStream_t s) {
    using S = typename P::S;
    using C = typename P::C;
    const dim3 grid((nx - 2 + 63) / 64, (ny - 2 + 3) / 4, nz - 2), block(64, 4);
    heat_plain<P><<<grid, block, 0, s>>>(static_cast<const S *>(u), static_cast<S *>(un), nx, ny,
                                         nz, (C)r, key);
}

hipError_t launch_heat_plain(int dtype, const void *u, void *un, int nx, int ny, int nz,
                             double r, unsigned long long seed, unsigned long long step,
                             hipStream_t s) {
    const SRKey key = make_key(seed, step);
    switch (dtype) {
        case kDtypeF64: plain<PrecF64>(u, un, nx, ny, nz, r, key, s); break;
        case kDtypeF32: plain<PrecF32>(u, un, nx, ny, nz, r, key, s); break;
        case kDtypeBF16: plain<PrecBF16>(u, un, nx, ny, nz, r, key, s); break;
        case kDtypeBF16SR: plain<PrecBF16SR>(u, un, nx, ny, nz, r, key, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_faces(int elem_bytes, const void *u, void *un, int nx, int ny, int nz,
                             hipStream_t s) {
    const long long total =
        2LL * nx * ny + (long long)(nz - 2) * (2LL * nx + 2LL * (ny - 2));
    long long nb = (total + 255) / 256;
    if (nb > 4096) nb = 4096;
    switch (elem_bytes) {
        case 8:
            copy_faces<unsigned long long><<<(unsigned)nb, 256, 0, s>>>(
                static_cast<const unsigned long long *>(u), static_cast<unsigned long long *>(un),
                nx, ny, nz);
            break;
        case 4:
            copy_faces<unsigned int><<<(unsigned)nb, 256, 0, s>>>(
                static_cast<const unsigned int *>(u), static_cast<unsigned int *>(un), nx, ny, nz);
            break;
        case 2:
            copy_faces<unsigned short><<<(unsigned)nb, 256, 0, s>>>(
                static_cast<const unsigned short *>(u), static_cast<unsigned short *>(un), nx, ny,
                nz);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hc
