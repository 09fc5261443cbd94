// batch_kernels.hip -- many independent heat problems of uneven size
// advanced together, one launch per time step.
//
// The problems' arrays are packed one after another in one buffer (each
// starting on a 64-byte boundary).  A work list holds one entry per
// (problem, x-tile, y-tile, z-block) of the z-marching sweep, in problem
// order and, inside a problem, y-tile fastest, then x-tile, then z-block
// (the order of the single-problem kernels).  The step kernel is persistent:
// a grid sized to fill the chip walks the list with a stride of the grid, so
// at any moment the blocks work on consecutive entries (neighbouring tiles
// of one or two problems) and the list's tail is spread evenly.  Each entry
// runs the same tile body as the single-problem sweep (heat_tile.hpp), so a
// problem in a batch gets the same bits as the problem on its own.  The
// Dirichlet layer is never written.

#include "heat_tile.hpp"

#include <climits>

namespace hc {
namespace {

template <class P, int VEC, int WX, int BY, int PF, int ZB>
__global__ __launch_bounds__(64 * WX * BY) void heat_batch_step(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un,
    const BatchProblem *__restrict__ probs, const BatchItem *__restrict__ items, int nitems) {
    using S = typename P::S;
    using C = typename P::C;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchProblem pr = probs[w.problem];
        const TileGeom<VEC, WX, BY> g(pr.nx, pr.ny, w.tx, w.ty, w.kb, w.ke);
        const S *up = u + pr.offset;
        S *unp = un + pr.offset;
        heat_tile_sweep<P, VEC, WX, BY, PF, ZB>(up, unp, (C)pr.r, g, SRKey{});
    }
}

}  // namespace

// The tile shapes built for the batched sweep, per precision:
// X(vec, wx, by, pf, zdepth).  Narrow tiles suit the small problems.
#define HC_BATCH_SHAPES_F64(X)                                                    \
    X(1, 1, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 1, 4, 2, 16) X(2, 1, 8, 2, 16)      \
    X(2, 1, 8, 2, 32) X(2, 2, 4, 2, 16)
#define HC_BATCH_SHAPES_F32(X)                                                    \
    X(1, 1, 4, 2, 16) X(1, 1, 8, 2, 16) X(2, 1, 4, 2, 16) X(2, 1, 8, 2, 16)      \
    X(2, 1, 8, 2, 32) X(4, 1, 4, 2, 16) X(4, 1, 8, 2, 16) X(2, 2, 4, 2, 16)      \
    X(1, 1, 16, 2, 16)
#define HC_BATCH_SHAPES_BF16(X)                                                   \
    X(1, 1, 4, 2, 16) X(2, 1, 8, 2, 16) X(4, 1, 8, 2, 16) X(8, 1, 4, 2, 16)      \
    X(8, 1, 8, 2, 16)

#define HC_BATCH_KEY(V, W, B, P, Z) ((((V * 8 + W) * 32 + B) * 4 + P) * 128 + Z)

bool batch_tiling_supported(int dtype, const HeatTiling &t) {
    const int key = HC_BATCH_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, P, Z) if (key == HC_BATCH_KEY(V, W, B, P, Z)) return true;
    if (dtype == kDtypeF64) { HC_BATCH_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_BATCH_SHAPES_F32(HC_X) }
    if (dtype == kDtypeBF16) { HC_BATCH_SHAPES_BF16(HC_X) }
#undef HC_X
    return false;
}

template <class P>
static hipError_t launch_batch(const void *u, void *un, const BatchProblem *probs,
                               const BatchItem *items, int nitems, int grid,
                               const HeatTiling &t, hipStream_t s) {
    using S = typename P::S;
    if (nitems <= 0) return hipSuccess;
    const int nb = (grid <= 0 || grid > nitems) ? nitems : grid;
    const dim3 block(64 * t.wx * t.by);
    const S *us = static_cast<const S *>(u);
    S *uns = static_cast<S *>(un);
    const int shape = HC_BATCH_KEY(t.vec, t.wx, t.by, t.pf, t.zdepth);
#define HC_X(V, W, B, PF, Z)                                                     \
    if (shape == HC_BATCH_KEY(V, W, B, PF, Z)) {                                 \
        heat_batch_step<P, V, W, B, PF, Z><<<dim3((unsigned)nb), block, 0, s>>>( \
            us, uns, probs, items, nitems);                                      \
        return hipGetLastError();                                                \
    }
    if constexpr (std::is_same<P, PrecF64>::value) {
        HC_BATCH_SHAPES_F64(HC_X)
    } else if constexpr (std::is_same<P, PrecF32>::value) {
        HC_BATCH_SHAPES_F32(HC_X)
    } else {
        HC_BATCH_SHAPES_BF16(HC_X)
    }
#undef HC_X
    return hipErrorInvalidValue;
}

hipError_t launch_heat_batch(int dtype, const void *u, void *un, const BatchProblem *probs,
                             const BatchItem *items, int nitems, int grid,
                             const HeatTiling &t, hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: return launch_batch<PrecF64>(u, un, probs, items, nitems, grid, t, s);
        case kDtypeF32: return launch_batch<PrecF32>(u, un, probs, items, nitems, grid, t, s);
        case kDtypeBF16: return launch_batch<PrecBF16>(u, un, probs, items, nitems, grid, t, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hc
