// batch_kernels.hip -- many independent heat problems of uneven size
// advanced together, one launch per time step.
//
// The problems' arrays are packed one after another in one buffer (each
// starting on a 64-byte boundary, rows padded to 16 bytes so that every
// problem takes 16-byte lanes).  A work list holds one entry per (problem,
// x-tile, y-tile, run of planes) of the z-marching sweep, grouped by width
// class (below), then in problem order and, inside a problem, y-tile
// fastest, then x-tile, then plane run.
//
// Tile width per problem.  A block has a fixed number of threads NT, but a
// tile row can be 8, 16, 32, 64 or 128 lanes wide (width class 0..4) with
// NT / lanes rows, so one wavefront covers several rows of a narrow problem;
// the host gives each problem the class whose tiles fit its rows best, so
// lanes are rarely left without nodes (which is what costs bandwidth: an
// idle lane issues no useful load).  Every class runs the same tile body as
// the single-problem sweep (heat_tile.hpp), so a problem in a batch gets the
// same bits as the problem on its own; the classes share one LDS buffer.
//
// The step kernel is persistent: a grid sized to fill the chip walks the
// list with a stride of the grid, so at any moment the blocks work on
// consecutive entries (neighbouring tiles of one or two problems) and the
// list's tail is spread evenly; runs of consecutive entries can be dealt to
// one XCD (block_order), so that their shared halo rows meet in one L2.  The
// Dirichlet layer is never written.

#include "batch_class.hpp"
#include "heat_tile.hpp"

#include <climits>

namespace hc {
namespace {

template <int VEC, int NT, int CLS>
constexpr int class_lds() {
    return WidthClass<NT, CLS>::valid
               ? tile_lds_elems<VEC, WidthClass<NT, CLS>::lanes, WidthClass<NT, CLS>::rows>()
               : 0;
}

template <int VEC, int NT>
constexpr int batch_lds() {
    int m = 0;
    const int v[5] = {class_lds<VEC, NT, 0>(), class_lds<VEC, NT, 1>(), class_lds<VEC, NT, 2>(),
                      class_lds<VEC, NT, 3>(), class_lds<VEC, NT, 4>()};
    for (int c = 0; c < 5; ++c) m = v[c] > m ? v[c] : m;
    return m;
}

template <class P, int VEC, int NT, int CLS, int PF, int ZB>
__device__ __forceinline__ void sweep_class(const typename P::S *u, typename P::S *un,
                                            const BatchProblem &pr, const BatchItem &w,
                                            typename P::C *tile) {
    using WC = WidthClass<NT, CLS>;
    if constexpr (WC::valid) {
        const TileGeom<VEC, WC::lanes, WC::rows> g((int)threadIdx.x, pr.nx, pr.pitch, pr.ny, w.tx,
                                                   w.ty, w.kb, w.ke);
        heat_tile_sweep<P, VEC, WC::lanes, WC::rows, PF, ZB>(
            u + pr.offset, un + pr.offset, (typename P::C)pr.r, g, SRKey{}, tile);
    }
}

template <class P, int VEC, int NT, int PF, int ZB>
__global__ __launch_bounds__(NT) void heat_batch_step(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un,
    const BatchProblem *__restrict__ probs, const BatchItem *__restrict__ items, int nitems,
    int xcd) {
    __shared__ typename P::C tile[batch_lds<VEC, NT>()];
    for (int b = blockIdx.x; b < nitems; b += gridDim.x) {
        // runs of xcd consecutive entries (y-neighbouring tiles, which share
        // halo rows) go to the blocks of one XCD
        const int it = block_order(b, nitems, xcd);
        const BatchItem w = items[it];
        const BatchProblem pr = probs[w.problem];
        switch (pr.cls) {  // the same for every thread of the block
            case 0: sweep_class<P, VEC, NT, 0, PF, ZB>(u, un, pr, w, tile); break;
            case 1: sweep_class<P, VEC, NT, 1, PF, ZB>(u, un, pr, w, tile); break;
            case 2: sweep_class<P, VEC, NT, 2, PF, ZB>(u, un, pr, w, tile); break;
            case 3: sweep_class<P, VEC, NT, 3, PF, ZB>(u, un, pr, w, tile); break;
            default: sweep_class<P, VEC, NT, 4, PF, ZB>(u, un, pr, w, tile); break;
        }
    }
}

}  // namespace

bool batch_class_valid(int nt, int cls) {
    if (cls < 0 || cls > 4) return false;
    const int lanes = 8 << cls, rows = nt / lanes;
    return rows >= 4 && nt >= 2 * lanes + 2 * rows + 4;
}

// The block shapes built for the batched sweep, per precision:
// X(vec, threads per block, pf, zdepth); vec nodes make a 16-byte lane.
#define HC_BATCH_SHAPES_F64(X) X(2, 256, 2, 16) X(2, 512, 2, 16) X(2, 512, 3, 16)
#define HC_BATCH_SHAPES_F32(X)                                                    \
    X(4, 256, 2, 16) X(4, 512, 2, 16) X(4, 512, 3, 16) X(4, 512, 2, 32)          \
    X(4, 1024, 2, 16)
#define HC_BATCH_SHAPES_BF16(X) X(8, 256, 2, 16) X(8, 512, 2, 16) X(8, 512, 3, 16)

#define HC_BATCH_KEY(V, N, P, Z) (((V * 2048 + N) * 8 + P) * 128 + Z)

bool batch_tiling_supported(int dtype, const BatchTiling &t) {
    const int key = HC_BATCH_KEY(t.vec, t.threads, t.pf, t.zdepth);
#define HC_X(V, N, P, Z) if (key == HC_BATCH_KEY(V, N, P, Z)) return true;
    if (dtype == kDtypeF64) { HC_BATCH_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_BATCH_SHAPES_F32(HC_X) }
    if (dtype == kDtypeBF16) { HC_BATCH_SHAPES_BF16(HC_X) }
#undef HC_X
    return false;
}

void batch_shapes(int dtype, std::vector<BatchTiling> &out) {
    out.clear();
#define HC_X(V, N, P, Z) out.push_back(BatchTiling{V, N, Z, P, 0, -1});
    if (dtype == kDtypeF64) { HC_BATCH_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_BATCH_SHAPES_F32(HC_X) }
    if (dtype == kDtypeBF16) { HC_BATCH_SHAPES_BF16(HC_X) }
#undef HC_X
}

template <class P>
static hipError_t launch_batch(const void *u, void *un, const BatchProblem *probs,
                               const BatchItem *items, int nitems, int grid,
                               const BatchTiling &t, hipStream_t s) {
    using S = typename P::S;
    if (nitems <= 0) return hipSuccess;
    const int nb = (grid <= 0 || grid > nitems) ? nitems : grid;
    const S *us = static_cast<const S *>(u);
    S *uns = static_cast<S *>(un);
    const int shape = HC_BATCH_KEY(t.vec, t.threads, t.pf, t.zdepth);
#define HC_X(V, N, PF, Z)                                                        \
    if (shape == HC_BATCH_KEY(V, N, PF, Z)) {                                    \
        heat_batch_step<P, V, N, PF, Z><<<dim3((unsigned)nb), dim3(N), 0, s>>>(   \
            us, uns, probs, items, nitems, t.xcd);                               \
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
                             const BatchTiling &t, hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: return launch_batch<PrecF64>(u, un, probs, items, nitems, grid, t, s);
        case kDtypeF32: return launch_batch<PrecF32>(u, un, probs, items, nitems, grid, t, s);
        case kDtypeBF16: return launch_batch<PrecBF16>(u, un, probs, items, nitems, grid, t, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hc
