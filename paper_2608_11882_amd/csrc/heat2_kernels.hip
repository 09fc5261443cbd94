// heat2_kernels.hip -- the Interior / Boundary / fused z-marching sweeps of
// the 7-point heat update taking two steps per pass (tile body in
// heat_tile2.hpp), FP64, FP32 and bfloat16 storage with nearest rounding.

#include "heat_tile2.hpp"

#include <climits>
#include <type_traits>

namespace hc {
namespace {

// Blocks of one-node lanes in 64 x 4 tiles are held to 64 VGPRs (eight
// wavefronts per SIMD), so that one fits on a CU beside a block of the
// widest shapes (1024 threads of at most 112 VGPRs each take 448 of a SIMD
// lane's 512): the split form's Boundary kernel runs in that room.
template <int VEC, int WX, int BY>
constexpr int kMinWaves = (VEC == 1 && WX == 1 && BY == 4) ? 8 : 1;

#define HC_HEAT2_KERNEL(NAME)                                                               \
    template <class P, int VEC, int WX, int BY, int PF, int ZB>                             \
    __global__ __launch_bounds__(64 * WX * BY, (kMinWaves<VEC, WX, BY>)) void NAME(         \
        const typename P::S *__restrict__ u, typename P::S *__restrict__ un, int nx,        \
        int ny, int nz, typename P::C r, ZTable zt, int ntx, int nty, int xcd) {            \
        using G = TileGeom2<VEC, 64 * WX, BY>;                                              \
        __shared__ typename P::C tu[2 * G::U_ELEMS];                                        \
        __shared__ typename P::C ta[2 * G::A_ELEMS];                                        \
        const auto g = block_tile2<VEC, 64 * WX, BY>(nx, ny, nz, zt, ntx, nty, xcd, ZB);    \
        heat_tile_sweep2<P, VEC, 64 * WX, BY, PF, ZB>(u, un, r, g, tu, ta);                 \
    }

// Three entry points with one body, so that profiles name the role.
HC_HEAT2_KERNEL(heat2_interior)
HC_HEAT2_KERNEL(heat2_boundary)
HC_HEAT2_KERNEL(heat2_fused)
#undef HC_HEAT2_KERNEL

}  // namespace

// Tile shapes built for the two-step sweep, per precision:
// X(vec, wx, by, pf, zdepth).  (1, 4, 4, 2, 16) is the fallback for arrays
// that do not allow wide lanes; (1, 1, 4, 2, 16) is the Boundary kernel's
// shape in the split form.
#define HC_HEAT2_SHAPES_F64(X)                                                    \
    X(1, 4, 4, 2, 16) X(2, 1, 8, 2, 32) X(2, 1, 16, 2, 16) X(2, 2, 4, 2, 32)     \
    X(2, 2, 8, 2, 16) X(2, 2, 8, 2, 32) X(2, 4, 4, 2, 16) X(2, 2, 4, 2, 64)      \
    X(2, 2, 4, 3, 32) X(2, 1, 8, 2, 64) X(2, 1, 4, 2, 32) X(1, 1, 4, 2, 16)     \
    X(2, 2, 8, 1, 32)
#define HC_HEAT2_SHAPES_F32(X)                                                    \
    X(1, 4, 4, 2, 16) X(2, 2, 8, 2, 16) X(4, 1, 8, 2, 32) X(4, 1, 16, 2, 16)     \
    X(4, 2, 4, 2, 32) X(4, 2, 8, 2, 16) X(4, 2, 4, 2, 64) X(4, 1, 8, 2, 64)      \
    X(4, 2, 4, 3, 32) X(4, 1, 4, 2, 32) X(1, 1, 4, 2, 16)
#define HC_HEAT2_SHAPES_BF16(X)                                                   \
    X(1, 4, 4, 2, 16) X(4, 1, 16, 2, 16) X(4, 1, 8, 2, 32) X(8, 1, 8, 2, 16)     \
    X(8, 1, 4, 2, 32) X(4, 1, 8, 2, 64) X(4, 2, 4, 2, 32) X(4, 1, 4, 2, 32)      \
    X(1, 1, 4, 2, 16)

#define HC_HEAT2_KEY(V, W, B, P, Z) ((((V * 8 + W) * 32 + B) * 8 + P) * 128 + Z)

bool heat2_tiling_supported(int dtype, const HeatTiling &t) {
    const int key = HC_HEAT2_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, P, Z) if (key == HC_HEAT2_KEY(V, W, B, P, Z)) return true;
    if (dtype == kDtypeF64) { HC_HEAT2_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_HEAT2_SHAPES_F32(HC_X) }
    if (dtype == kDtypeBF16) { HC_HEAT2_SHAPES_BF16(HC_X) }
#undef HC_X
    return false;
}

template <class P>
static hipError_t launch2(KernelKind kind, const void *u, void *un, int nx, int ny, int nz,
                          double r, const ZTable &zt, const HeatTiling &t, hipStream_t s) {
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
    const int shape = HC_HEAT2_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, PF, Z)                                                          \
    if (shape == HC_HEAT2_KEY(V, W, B, PF, Z)) {                                      \
        if (kind == K_HEAT2_INTERIOR)                                                 \
            heat2_interior<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(                 \
                us, uns, nx, ny, nz, rc, zt, ntx, nty, t.xcd);                        \
        else if (kind == K_HEAT2_BOUNDARY)                                            \
            heat2_boundary<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(                 \
                us, uns, nx, ny, nz, rc, zt, ntx, nty, t.xcd);                        \
        else                                                                          \
            heat2_fused<P, V, W, B, PF, Z><<<grid, block, 0, s>>>(                    \
                us, uns, nx, ny, nz, rc, zt, ntx, nty, t.xcd);                        \
        return hipGetLastError();                                                     \
    }
    if constexpr (std::is_same<P, PrecF64>::value) {
        HC_HEAT2_SHAPES_F64(HC_X)
    } else if constexpr (std::is_same<P, PrecF32>::value) {
        HC_HEAT2_SHAPES_F32(HC_X)
    } else {
        HC_HEAT2_SHAPES_BF16(HC_X)
    }
#undef HC_X
    return hipErrorInvalidValue;
}

hipError_t launch_heat2_tile(int dtype, KernelKind kind, const void *u, void *un, int nx, int ny,
                             int nz, double r, const ZTable &zt, const HeatTiling &t,
                             hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: return launch2<PrecF64>(kind, u, un, nx, ny, nz, r, zt, t, s);
        case kDtypeF32: return launch2<PrecF32>(kind, u, un, nx, ny, nz, r, zt, t, s);
        case kDtypeBF16: return launch2<PrecBF16>(kind, u, un, nx, ny, nz, r, zt, t, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hc
