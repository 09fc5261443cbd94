// Internal declarations shared by the kernel translation units and the C ABI
// layer of libheatcg.so.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace hc {

// Up to this many k-ranges can be swept by one launch (the slab count of
// the Interior/Boundary split is bounded by it).
constexpr int kMaxRanges = 64;

// Work list of a z-marching launch.  Range r covers the planes
// [kb[r], ke[r]] (inclusive), cut into z-blocks of depth[r] planes; the
// z-blocks of range r are numbered first[r] .. first[r+1]-1.
struct ZTable {
    int n;
    int kb[kMaxRanges];
    int ke[kMaxRanges];
    int depth[kMaxRanges];
    int first[kMaxRanges + 1];
};

// Launch shape of the z-marching heat kernels.
struct HeatTiling {
    int vec;      // nodes per lane along x: 1, 2, 4 or 8 (16-byte accesses
                  // at 2 FP64, 4 FP32 or 8 bfloat16 nodes)
    int wx;       // wavefronts per tile row: tile width = 64 * vec * wx
    int by;       // rows per tile
    int zdepth;   // planes per z-block of the Interior / fused kernel
    int pf;       // planes of loads kept in flight: 1 or 2
    int xcd;      // run length of y-neighbouring tiles dealt to one XCD
                  // (0 or 1: hardware order)
};

// Kernel kinds the launches are timed under (same values as hc_kernel_kind).
enum KernelKind {
    K_HEAT_INTERIOR = 0,
    K_HEAT_BOUNDARY = 1,
    K_HEAT_FUSED = 2,
    K_HEAT_PLAIN = 3,
    K_CG_DIRECTION = 4,
    K_CG_UPDATE = 5,
    K_CG_RESIDUAL = 6,
    K_LAP7 = 7,
    K_COPY = 8,
    K_CG32_DIRECTION = 9,
    K_CG32_UPDATE = 10,
    K_IR_RESIDUAL = 11,
    K_IR_UPDATE = 12,
    K_BATCH = 13,
    K_VK_INTERIOR = 14,
    K_VK_BOUNDARY = 15,
    K_VK_FUSED = 16,
    K_VK_PLAIN = 17,
    K_HEAT2_INTERIOR = 18,
    K_HEAT2_BOUNDARY = 19,
    K_HEAT2_FUSED = 20,
    K_VK2_INTERIOR = 21,
    K_VK2_BOUNDARY = 22,
    K_VK2_FUSED = 23,
    K_CG_UPDATE_X = 24,
    K_CG32_UPDATE_X = 25,
    K_COUNT = 26
};

// ---- heat (heat_kernels.hip) ------------------------------------------------
int ztable_blocks(const ZTable &zt);
// Grid size of a z-marching launch over table zt.
long long heat_tile_blocks(int nx, int ny, const HeatTiling &t, const ZTable &zt);
int tile_width(const HeatTiling &t);
// Storage precision codes (0-2: the values of hc_dtype): 0 FP64, 1 FP32,
// 2 bfloat16 storage with FP32 arithmetic rounded to nearest even, 3 the
// same with stochastic rounding (heat_step_sr); 3 shares 2's tile shapes.
constexpr int kDtypeF64 = 0, kDtypeF32 = 1, kDtypeBF16 = 2, kDtypeBF16SR = 3;
inline int dtype_bytes(int dtype) { return dtype == 0 ? 8 : dtype == 1 ? 4 : 2; }
bool heat_tiling_supported(int dtype, const HeatTiling &t);
// u and un hold nodes of the storage type of `dtype`.  seed and step key the
// random bits of the stochastic rounding (ignored by the other precisions).
hipError_t launch_heat_tile(int dtype, KernelKind kind, const void *u, void *un, int nx,
                            int ny, double r, const ZTable &zt, const HeatTiling &t,
                            unsigned long long seed, unsigned long long step, hipStream_t s);
hipError_t launch_heat_plain(int dtype, const void *u, void *un, int nx, int ny, int nz,
                             double r, unsigned long long seed, unsigned long long step,
                             hipStream_t s);
hipError_t launch_copy_faces(int elem_bytes, const void *u, void *un, int nx, int ny, int nz,
                             hipStream_t s);

// ---- two steps per pass (heat2_kernels.hip) ------------------------------------
// FP64, FP32 or bfloat16 (nearest) storage; the tile shapes are those of
// HeatTiling, from a list of their own.  A launch over zt writes u^(t+2) of
// the planes in zt from u^t.
bool heat2_tiling_supported(int dtype, const HeatTiling &t);
hipError_t launch_heat2_tile(int dtype, KernelKind kind, const void *u, void *un, int nx, int ny,
                             int nz, double r, const ZTable &zt, const HeatTiling &t,
                             hipStream_t s);

// ---- variable coefficient and source (varcoef_kernels.hip) ----------------------
// u, kap, rhs and un hold FP64 (dtype 0) or FP32 (dtype 1) nodes; the tile
// shapes are those of HeatTiling, from a list of their own.
bool heat_vk_tiling_supported(int dtype, const HeatTiling &t);
hipError_t launch_heat_vk_tile(int dtype, KernelKind kind, const void *u, const void *kap,
                               const void *rhs, void *un, int nx, int ny, double beta,
                               const ZTable &zt, const HeatTiling &t, hipStream_t s);
hipError_t launch_heat_vk_plain(int dtype, const void *u, const void *kap, const void *rhs,
                                void *un, int nx, int ny, int nz, double beta, hipStream_t s);

// Two steps per pass of the same (varcoef2_kernels.hip).
bool heat_vk2_tiling_supported(int dtype, const HeatTiling &t);
hipError_t launch_heat_vk2_tile(int dtype, KernelKind kind, const void *u, const void *kap,
                                const void *rhs, void *un, int nx, int ny, int nz, double beta,
                                const ZTable &zt, const HeatTiling &t, hipStream_t s);

// ---- batched heat (batch_kernels.hip) ------------------------------------------
// One problem of a batch: its array starts `offset` elements into the packed
// buffers; rows are `pitch` >= nx elements apart (padded to 16 bytes); its
// tiles have rows of 8 << cls lanes (width class cls).
struct BatchProblem {
    long long offset;
    int nx, ny, nz, pitch;
    int cls, pad;
    double r;
};
// One work-list entry: tile (tx, ty) of `problem`, planes kb .. ke.
struct BatchItem {
    int problem;
    unsigned short tx, ty;
    int kb, ke;
};
// Block shape of the batched sweep: vec nodes per lane (16 bytes),
// `threads` per block, z-runs walked in unrolled sub-blocks of `zdepth`
// planes, `pf` planes of loads in flight, runs of `xcd` consecutive
// work-list entries per XCD (0 or 1: hardware order), and the width class
// of every problem (-1: each problem's best fit).  Class c has rows of
// 8 << c lanes, threads >> (3 + c) rows.
struct BatchTiling {
    int vec, threads, zdepth, pf, xcd, cls;
};
bool batch_tiling_supported(int dtype, const BatchTiling &t);
// Whether width class cls exists for blocks of nt threads.
bool batch_class_valid(int nt, int cls);
// Every block shape built for `dtype` (xcd 0, class -1).
void batch_shapes(int dtype, std::vector<BatchTiling> &out);
// The two-step batched sweep (batch2_kernels.hip): its shapes are a subset
// of the single-step ones.
bool batch2_tiling_supported(int dtype, const BatchTiling &t);
// One pass over the n work-list entries `items` of width class cls (all
// of one class).
hipError_t launch_heat_batch2(int dtype, int cls, const void *u, void *un,
                              const BatchProblem *probs, const BatchItem *items, int n, int grid,
                              const BatchTiling &t, hipStream_t s);
// One time step of every problem; grid <= 0 or >= nitems: one block per
// entry, else a persistent grid of `grid` blocks walking the list.
hipError_t launch_heat_batch(int dtype, const void *u, void *un, const BatchProblem *probs,
                             const BatchItem *items, int nitems, int grid,
                             const BatchTiling &t, hipStream_t s);

// ---- CG (cg_kernels.hip) ------------------------------------------------------
// Device-resident scalars of one CG solve.  Written by the last block of
// each reduction kernel, read by the next kernel and (64 bytes) by the host.
struct CGScalars {
    double rho;       // r.r of the current residual
    double pap;       // p.Ap of the current direction
    double alpha;
    double beta;
    double bnorm2;    // b.b
    double tol;       // relative tolerance
    double thresh;    // tol * ||b||
    double rtrue2;    // |b - A x|^2 of the last true-residual pass
    double inner_tol; // refinement: relative reduction of each inner solve
    double floor_frac;// refinement: inner solves stop at floor_frac * tol ||b||
    double rslot[2];  // r.r of iteration k in slot k & 1 (device use)
    double aslot[4];  // alpha of iteration k in slot k & 3 (device use)
    int iter;         // completed iterations
    int state;        // 0 running, 1 converged, -6 breakdown, -7 non-finite
    unsigned ticket;  // arrival counter of the residual kernels (0 between kernels)
    unsigned pad;
};

// r, p[0], p[1] point at plane 0 of vectors that carry one zero plane
// below plane 0 and one above plane nz-1 (cleared by the driver).
struct CGWork {
    double *r;
    double *p[4];      // the direction vector of iteration k is p[k & 3]
    double *partial;   // two doubles per block
    CGScalars *sc;
};

// Refinement (binary32 inner solve): s (the inner residual, first the
// rounded outer residual), p[0], p[1] padded like CGWork's vectors; d the
// inner solution (no padding needed: only read at its own nodes).
struct CGWorkF32 {
    float *r;
    float *p[2];
    float *d;
    double *partial;   // three doubles per block
    CGScalars *sc;
};

// Tile shape of the CG kernels (same meaning as HeatTiling, one plane of
// epilogue loads and two of field loads in flight).
struct CGTiling {
    int vec;
    int wx;
    int by;
    int zdepth;
    int xcd;
};

bool cg_tiling_supported(const CGTiling &t);
bool cg_tiling_supported_f32(const CGTiling &t);
size_t cg_work_bytes(int nx, int ny, int nz);
// Carve a CGWork out of `base` (at least cg_work_bytes bytes).
CGWork cg_work_carve(void *base, int nx, int ny, int nz);
size_t cg_ir_work_bytes(int nx, int ny, int nz);
CGWorkF32 cg_ir_work_carve(void *base, int nx, int ny, int nz);
long long cg_blocks(int nx, int ny, int nz, const CGTiling &t);
hipError_t launch_cg_init(CGScalars *sc, double tol, double inner_tol, double floor_frac,
                          hipStream_t s);
// `sink`: a device buffer of at least kSinkDoubles doubles that lanes outside
// the box store into (never read).
constexpr int kSinkDoubles = 2048;
hipError_t launch_cg_residual(const double *b, const double *x, const CGWork &w,
                              int nx, int ny, int nz, int store_r,
                              const CGTiling &t, double *sink, hipStream_t s);
// Iteration k (iterations completed before it) of the direction and update
// kernels; after a batch, launch_cg_settle(k) with k the next iteration
// finishes the last update's reduction so that the scalars show whether the
// solve has converged.
hipError_t launch_cg_direction(const CGWork &w, int first, int k, int nx, int ny, int nz,
                               const CGTiling &t, double *sink, hipStream_t s);
// xsteps: how many of x's steps the update of iteration k applies: 0 (this
// iteration's step waits) or 4 (those of iterations k-3 .. k, in that
// order).  The direction of iteration k reads p[(k-1)&3] and writes p[k&3].
hipError_t launch_cg_update(double *x, const CGWork &w, int k, int xsteps, int nx, int ny,
                            int nz, const CGTiling &t, double *sink, hipStream_t s);
// x += alpha_j p over n nodes, alpha_j from sc's slot j & 3: a step of x
// that waited (see launch_cg_update).
hipError_t launch_cg_xstep(double *x, const double *p, const CGScalars *sc, int j, long long n,
                           hipStream_t s);
hipError_t launch_cg_settle(const CGWork &w, int k, int nx, int ny, int nz, const CGTiling &t,
                            hipStream_t s);
hipError_t launch_lap7_f64(const double *x, double *y, int nx, int ny, int nz,
                           const CGTiling &t, double *sink, hipStream_t s);
// refinement kernels (t from the binary32 shape list, except the residual,
// whose field is binary64: t from the binary64 list)
hipError_t launch_cg_ir_residual(const double *b, const double *x, const CGWorkF32 &w, int nx,
                                 int ny, int nz, const CGTiling &t, double *sink,
                                 hipStream_t s);
hipError_t launch_cg_direction_f32(const CGWorkF32 &w, int cur, int first, int k, int nx,
                                   int ny, int nz, const CGTiling &t, double *sink,
                                   hipStream_t s);
hipError_t launch_cg_update_f32(const CGWorkF32 &w, int cur, int k, int xstep, int nx, int ny,
                                int nz, const CGTiling &t, double *sink, hipStream_t s);
hipError_t launch_cg_xstep_f32(float *x, const float *p, const CGScalars *sc, int j, long long n,
                               hipStream_t s);
hipError_t launch_cg_settle_f32(const CGWorkF32 &w, int k, int nx, int ny, int nz,
                                const CGTiling &t, hipStream_t s);
hipError_t launch_lap7_f32(const float *x, float *y, int nx, int ny, int nz, const CGTiling &t,
                           double *sink, hipStream_t s);
hipError_t launch_ir_axpy(double *x, const float *d, long long n, hipStream_t s);

// ---- probes (probe.hip) ---------------------------------------------------------
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes,
                             hipStream_t s);

}  // namespace hc
