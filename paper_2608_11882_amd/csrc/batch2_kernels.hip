// batch2_kernels.hip -- the batched sweep taking two steps per pass: the
// same packed buffers, work list and width classes as batch_kernels.hip,
// each work-list entry swept with the two-step tile (heat_tile2.hpp), so a
// launch advances every problem from u^t to u^(t+2) and every problem gets
// the bits of its own single steps.

#include "batch_class.hpp"
#include "heat_tile2.hpp"

#include <climits>

namespace hc {
namespace {

// LDS values of the two-step tile of class CLS: two u^t planes with their
// two-node ring, and two u^(t+1) planes with a one-node ring and a sink.
template <int VEC, int NT, int CLS>
constexpr int class_lds_u() {
    using WC = WidthClass<NT, CLS>;
    return WC::valid ? 2 * (WC::rows + 4) * (VEC * WC::lanes + 4) : 1;
}
template <int VEC, int NT, int CLS>
constexpr int class_lds_a() {
    using WC = WidthClass<NT, CLS>;
    return WC::valid ? 2 * ((WC::rows + 2) * (VEC * WC::lanes + 2) + 1) : 1;
}

template <class P, int VEC, int NT, int CLS, int PF, int ZB>
__device__ __forceinline__ void sweep_class2(const typename P::S *u, typename P::S *un,
                                             const BatchProblem &pr, const BatchItem &w,
                                             typename P::C *tu, typename P::C *ta) {
    using WC = WidthClass<NT, CLS>;
    if constexpr (WC::valid) {
        const TileGeom2<VEC, WC::lanes, WC::rows> g((int)threadIdx.x, pr.nx, pr.pitch, pr.ny,
                                                    pr.nz, w.tx, w.ty, w.kb, w.ke);
        heat_tile_sweep2<P, VEC, WC::lanes, WC::rows, PF, ZB>(
            u + pr.offset, un + pr.offset, (typename P::C)pr.r, g, tu, ta);
    }
}

// One kernel per width class (the class bodies compiled into one kernel
// would share one register allocation, far larger than any of them needs);
// a launch walks the class's slice of the work list.
template <class P, int VEC, int NT, int CLS, int PF, int ZB>
__global__ __launch_bounds__(NT) void heat_batch_step2(
    const typename P::S *__restrict__ u, typename P::S *__restrict__ un,
    const BatchProblem *__restrict__ probs, const BatchItem *__restrict__ items, int nitems,
    int xcd) {
    __shared__ typename P::C tu[class_lds_u<VEC, NT, CLS>()];
    __shared__ typename P::C ta[class_lds_a<VEC, NT, CLS>()];
    for (int b = blockIdx.x; b < nitems; b += gridDim.x) {
        const int it = block_order(b, nitems, xcd);
        const BatchItem w = items[it];
        const BatchProblem pr = probs[w.problem];
        sweep_class2<P, VEC, NT, CLS, PF, ZB>(u, un, pr, w, tu, ta);
    }
}

}  // namespace

// Block shapes built for the two-step batched sweep, per precision (each
// with one kernel per width class; a pass launches one per class present):
// X(vec, threads per block, pf, zdepth); each is also a single-step shape
// (batch_kernels.hip), which takes a last odd step.
#define HC_BATCH2_SHAPES_F64(X) X(2, 512, 2, 16)
#define HC_BATCH2_SHAPES_F32(X) X(4, 256, 2, 16) X(4, 512, 2, 16) X(4, 512, 2, 32) X(4, 1024, 2, 16)
#define HC_BATCH2_SHAPES_BF16(X) X(8, 512, 2, 16)

#define HC_BATCH2_KEY(V, N, P, Z) (((V * 2048 + N) * 8 + P) * 128 + Z)

bool batch2_tiling_supported(int dtype, const BatchTiling &t) {
    const int key = HC_BATCH2_KEY(t.vec, t.threads, t.pf, t.zdepth);
#define HC_X(V, N, P, Z) if (key == HC_BATCH2_KEY(V, N, P, Z)) return true;
    if (dtype == kDtypeF64) { HC_BATCH2_SHAPES_F64(HC_X) }
    if (dtype == kDtypeF32) { HC_BATCH2_SHAPES_F32(HC_X) }
    if (dtype == kDtypeBF16) { HC_BATCH2_SHAPES_BF16(HC_X) }
#undef HC_X
    return false;
}

template <class P, int V, int N, int PF, int Z, int CLS>
static void launch_class(const typename P::S *u, typename P::S *un, const BatchProblem *probs,
                         const BatchItem *items, int n, int grid, int xcd, hipStream_t s) {
    if constexpr (WidthClass<N, CLS>::valid) {
        const int nb = (grid <= 0 || grid > n) ? n : grid;
        heat_batch_step2<P, V, N, CLS, PF, Z><<<dim3((unsigned)nb), dim3(N), 0, s>>>(
            u, un, probs, items, n, xcd);
    }
}

template <class P>
static hipError_t launch_batch2(int cls, const void *u, void *un, const BatchProblem *probs,
                                const BatchItem *items, int n, int grid, const BatchTiling &t,
                                hipStream_t s) {
    using S = typename P::S;
    if (n <= 0) return hipSuccess;
    const S *us = static_cast<const S *>(u);
    S *uns = static_cast<S *>(un);
    const int shape = HC_BATCH2_KEY(t.vec, t.threads, t.pf, t.zdepth);
#define HC_X(V, N, PF, Z)                                                                       \
    if (shape == HC_BATCH2_KEY(V, N, PF, Z)) {                                                  \
        if (!batch_class_valid(N, cls)) return hipErrorInvalidValue;                            \
        switch (cls) {                                                                          \
            case 0: launch_class<P, V, N, PF, Z, 0>(us, uns, probs, items, n, grid, t.xcd, s); break; \
            case 1: launch_class<P, V, N, PF, Z, 1>(us, uns, probs, items, n, grid, t.xcd, s); break; \
            case 2: launch_class<P, V, N, PF, Z, 2>(us, uns, probs, items, n, grid, t.xcd, s); break; \
            case 3: launch_class<P, V, N, PF, Z, 3>(us, uns, probs, items, n, grid, t.xcd, s); break; \
            default: launch_class<P, V, N, PF, Z, 4>(us, uns, probs, items, n, grid, t.xcd, s); break; \
        }                                                                                       \
        return hipGetLastError();                                                               \
    }
    if constexpr (std::is_same<P, PrecF64>::value) {
        HC_BATCH2_SHAPES_F64(HC_X)
    } else if constexpr (std::is_same<P, PrecF32>::value) {
        HC_BATCH2_SHAPES_F32(HC_X)
    } else {
        HC_BATCH2_SHAPES_BF16(HC_X)
    }
#undef HC_X
    return hipErrorInvalidValue;
}

hipError_t launch_heat_batch2(int dtype, int cls, const void *u, void *un,
                              const BatchProblem *probs, const BatchItem *items, int n, int grid,
                              const BatchTiling &t, hipStream_t s) {
    switch (dtype) {
        case kDtypeF64: return launch_batch2<PrecF64>(cls, u, un, probs, items, n, grid, t, s);
        case kDtypeF32: return launch_batch2<PrecF32>(cls, u, un, probs, items, n, grid, t, s);
        case kDtypeBF16: return launch_batch2<PrecBF16>(cls, u, un, probs, items, n, grid, t, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hc
