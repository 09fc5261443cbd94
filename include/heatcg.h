/*
 * heatcg.h -- C ABI of libheatcg.so: the explicit 7-point heat update and
 * Conjugate Gradient on the 7-point Laplacian, for AMD MI355X (gfx950).
 *
 * Paper: "Mathematical Details" (Eqs. 1-6, Pseudocode alg:heat3d), the
 * one-GPU baseline and the Interior / Boundary kernels of the multi-GPU
 * versions (Pseudocodes alg:1gpu-base, alg:interior-kernel,
 * alg:boundary-kernel), and the CG case study (Pseudocode alg:spmv).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer on the current HIP device
 *    (e.g. the data pointer of a contiguous torch CUDA tensor).  The caller
 *    allocates and owns every buffer; the library keeps no pointer after a
 *    call returns.
 *  - 3-D arrays are stored with x fastest and z slowest:
 *    a[(k*ny + j)*nx + i].  This is the paper's u[k, j, i] ordering.
 *  - Arguments are validated before any device work.  On a validation
 *    error nothing is launched and no buffer is touched.
 *  - Return value: HC_OK (0), a positive soft status, or a negative error.
 *    hc_strerror() names a code; hc_last_error_message() gives the detail
 *    of the last failure on the calling thread (e.g. a HIP error string).
 *  - hc_stream_t is a hipStream_t.  NULL means the device's null stream.
 */
#ifndef HEATCG_H
#define HEATCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hc_stream_t;

enum hc_status {
    HC_OK = 0,
    HC_ENOTCONV = 1,     /* CG reached maxit; x holds the last iterate    */
    HC_EINVAL = -1,      /* bad pointer, size, dtype, mode or count        */
    HC_EUNSTABLE = -2,   /* r not finite or outside [0, 1/6]               */
    HC_EALIAS = -3,      /* input and output buffers overlap               */
    HC_ENOMEM = -4,      /* device allocation failed                       */
    HC_EHIP = -5,        /* a HIP runtime call or kernel launch failed     */
    HC_EBREAKDOWN = -6,  /* CG: p.Ap <= 0 (operator not SPD in practice)   */
    HC_ENONFINITE = -7   /* CG: a scalar became NaN or infinite            */
};

/* Element types.  HC_BF16_SR names the stochastic-rounding sweep of
 * heat_step_sr (bfloat16 storage); heat_step_ex does not take it. */
enum hc_dtype { HC_F64 = 0, HC_F32 = 1, HC_BF16 = 2, HC_BF16_SR = 3 };

enum hc_heat_mode {
    HC_HEAT_SPLIT = 0, /* Interior kernel on the caller's stream and the
                          Boundary-plane kernel on a second stream,
                          joined by events every step                      */
    HC_HEAT_FUSED = 1, /* one z-marching kernel over every updated plane   */
    HC_HEAT_PLAIN = 2  /* one thread per node, every neighbour loaded
                          from memory (the straightforward GPU form)      */
};

/*
 * heat_step -- advance the heat equation by `steps` explicit steps.
 *
 * Computes, for every interior node and each step (Eq. 4 with a constant
 * coefficient kappa = alpha and no source, i.e. the 7-point FTCS update):
 *     u_new = u + r * (((x- + x+) + (y- + y+)) + (z- + z+) - 6 u)
 * with r = alpha*dt/h^2, followed by a swap of u and u_new (alg:heat3d).
 *
 *  u       [in/out] nx*ny*nz FP64, device.  u^0 on entry, u^steps on
 *          return.  Its outermost layer holds the Dirichlet data and is
 *          never written (the paper uses zero data, Eq. 5).
 *  u_new   [scratch] nx*ny*nz FP64, device, must not overlap u.  On entry
 *          its outermost layer is overwritten with u's, and it keeps u's
 *          outermost layer on return.  With one step per pass
 *          (hc_heat_set_time_block(1)) it holds u^(steps-1) when steps is
 *          even and >= 2 and u^steps when steps is odd; with two steps per
 *          pass (the default) its interior holds the state before the last
 *          pass or u^steps, and should be taken as unspecified.
 *  nx,ny,nz  stored edge lengths including the Dirichlet layer, each >= 3;
 *          (nx-2)(ny-2)(nz-2) nodes are updated.
 *  r       finite, 0 <= r <= 1/6 (stability and the discrete maximum
 *          principle of the 3-D scheme), else HC_EUNSTABLE.
 *  steps   >= 0; 0 is a no-op.
 *
 * Runs the Interior/Boundary split (HC_HEAT_SPLIT, one slab) and BLOCKS
 * until the result is in u, so kernel faults are reported here.
 */
int heat_step(double *u, double *u_new, int nx, int ny, int nz, double r,
              int steps);

/*
 * heat_step_ex -- heat_step with the element type, kernel form, slab count
 * and stream chosen by the caller.  Enqueues the work on `stream` and
 * returns without waiting (stream order is the only ordering).
 *
 *  dtype  element type of u and u_new:
 *           HC_F64  binary64 storage and arithmetic (the paper's precision);
 *           HC_F32  binary32 storage and arithmetic;
 *           HC_BF16 bfloat16 storage (uint16 bit patterns, the upper half
 *                   of a binary32) with binary32 arithmetic: each node is
 *                   widened exactly, updated in binary32 in the order above,
 *                   and rounded to the nearest bfloat16, ties to even (NaN
 *                   stays NaN).  r is rounded to binary32 for both reduced
 *                   precisions.
 *         Sizes and alignment rules are in elements of that type.
 *  mode   an hc_heat_mode.
 *  parts  number of equal k-slabs the split form treats as separate
 *         subdomains (the paper's decomposition along k, Methodology): the
 *         first and last plane of every slab are Boundary planes, the rest
 *         Interior.  1 <= parts <= min(32, nz-2); must be 1 unless
 *         mode == HC_HEAT_SPLIT.
 *  stream the stream the work is ordered on.  The Boundary kernels run on
 *         an internal stream of the same device that joins `stream` at
 *         every step through events.
 */
int heat_step_ex(void *u, void *u_new, int nx, int ny, int nz, double r,
                 int steps, int dtype, int mode, int parts, hc_stream_t stream);

/*
 * heat_step_streams -- the split form (HC_HEAT_SPLIT) on two streams the
 * caller chooses: the Interior kernels on s_int, the Boundary kernels on
 * s_bnd, joined at every step (the asynchronous Interior / Boundary
 * decomposition of the paper's stream versions, Pseudocodes
 * alg:2gpu-stream and alg:boundary-kernel-async, on one device).
 *
 *  u, u_new, nx, ny, nz, r, steps, dtype, parts  as for heat_step_ex.
 *  s_int  the work is ordered on it: the run starts after its earlier
 *         work, and u holds the result once its work up to here is done.
 *  s_bnd  a stream of the current device (else HC_EINVAL), or s_int
 *         itself (the Boundary kernels then run before the Interior kernel
 *         of each step).  It waits for s_int before the first step and at
 *         the end of every step, so work the caller enqueues on it later
 *         runs after the whole sweep.
 * Enqueues and returns; validation and statuses as for heat_step_ex.
 */
int heat_step_streams(void *u, void *u_new, int nx, int ny, int nz, double r,
                      int steps, int dtype, int parts, hc_stream_t s_int,
                      hc_stream_t s_bnd);

/*
 * heat_step_sr -- heat_step_ex for bfloat16 storage (HC_BF16 layout and
 * rules) with stochastic instead of nearest rounding.  Nearest rounding
 * drops every increment below half a bfloat16 ulp, so smooth fields stall;
 * here each new binary32 value v is rounded up in magnitude with
 * probability (the 16 bits of v a bfloat16 drops) / 2^16, and down
 * otherwise, which makes the rounding unbiased.  Values that are already
 * bfloat16 are kept.  NaN stays a quiet NaN; a value within one bfloat16 ulp
 * of the largest finite one may round to infinity.
 *
 * The 16 random bits of node p = (k*ny + j)*nx + i at step t come from the
 * counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * SC 2011): nodes are taken in aligned groups of 8, group g = p / 8 draws
 * one block with counter words (g mod 2^32, g / 2^32, t mod 2^32, t / 2^32)
 * and key words (seed mod 2^32, seed / 2^32), and node p takes word
 * (p mod 8) / 2 of it, the low half for even p and the high half for odd p.
 * Step s of this call (0 <= s < steps) has t = step0 + s, so a run split
 * over several calls with step0 advanced by the steps already taken gives
 * the same bits as one call.  The result depends on (seed, step0) and on
 * nothing else: not on mode, parts, tile shape or stream.
 */
int heat_step_sr(void *u, void *u_new, int nx, int ny, int nz, double r,
                 int steps, unsigned long long seed, unsigned long long step0,
                 int mode, int parts, hc_stream_t stream);

/*
 * Steps per pass of the constant-coefficient z-marching sweeps (process
 * wide): 1, or 2 (temporal blocking: a pass reads u^t once and writes
 * u^(t+2); u^(t+1) is computed on each tile and its one-node ring in
 * registers and LDS and never stored).  Results do not depend on it: every
 * value of u^(t+1) is evaluated with the same expression and rounding as a
 * single step.  It applies to HC_F64, HC_F32 and HC_BF16 in HC_HEAT_SPLIT
 * and HC_HEAT_FUSED (a last odd step takes a single pass), to heat_vk_step
 * (HC_F64, HC_F32) and to the batch (hc_batch_steps_per_pass); heat_step_sr
 * and HC_HEAT_PLAIN always take single steps.  In the split
 * form with two steps per pass, the Boundary kernel owns the first and last
 * two planes of each slab (the depth of halo two steps need), the Interior
 * kernel the rest.  Default: 2.  HC_EINVAL for other values.
 */
int hc_heat_set_time_block(int steps_per_pass);
int hc_heat_get_time_block(void);

/*
 * Tile shape of the two-step sweep, per dtype (HC_F64, HC_F32, HC_BF16),
 * same fields and rules as hc_heat_set_tiling (all zeros: automatic); the
 * shapes built are listed in heat2_kernels.hip (HC_HEAT2_SHAPES_*).  Here
 * xcd may also be -1: slab order, where each of the 8 XCDs sweeps one
 * eighth of the tile rows (every x-tile of them) z-run by z-run, so the
 * tiles that run side by side on an XCD are neighbours in x and y.
 * hc_heat2_tiling_for reports the shape a two-step sweep of these arrays
 * would run with.
 */
int hc_heat2_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf,
                        int xcd);
int hc_heat2_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth,
                        int *pf, int *xcd);
int hc_heat2_tiling_for(int dtype, int nx, const void *u, const void *u_new,
                        int *vec, int *wx, int *by, int *zdepth, int *pf,
                        int *xcd);

/*
 * Run length of the two-step constant-coefficient sweep, per dtype (HC_F64,
 * HC_F32, HC_BF16): the planes of output each block of the Interior (or
 * fused) kernel marches as one run, its register queues carried from one
 * z-block to the next.  0 (the default) is the automatic choice: 64
 * planes for HC_F64 when a plane has at most 256 tiles (else one z-block),
 * one z-block for HC_F32, 128 planes for HC_BF16; other
 * values are rounded up to a multiple of the tile's zdepth.  Results do
 * not depend on it.
 * hc_heat2_set_zrun returns HC_EINVAL for another dtype or a value outside
 * [0, 2^20]; hc_heat2_get_zrun returns the setting (or HC_EINVAL).
 */
int hc_heat2_set_zrun(int dtype, int planes);
int hc_heat2_get_zrun(int dtype);

/*
 * heat_vk_step -- the paper's own equation: `steps` explicit steps of
 * du/dt = div(kappa grad u) + f with kappa and f varying per node (Eq. 1-4
 * of "Mathematical Details", the time loop of Pseudocode alg:heat3d).  For
 * every interior node and each step, in this order and without contraction:
 *     D_x   = (k + k_x+) (u_x+ - u) - (k_x- + k) (u - u_x-)   (D_y, D_z alike)
 *     u_new = (u + rhs) + beta * ((D_x + D_y) + D_z)
 * i.e. the flux form with the sum of the two nodes' coefficients on each
 * face (twice their mean, which the 1/2 in beta = dt/(2 h^2) compensates),
 * followed by a swap of u and u_new.  With kappa constant it is heat_step
 * with r = 2 kappa beta (up to rounding).
 *
 *  u, u_new  as for heat_step_ex (u^0 in, u^steps out; u_new scratch whose
 *            outermost layer is overwritten with u's).
 *  kappa  [in] nx*ny*nz, device: the coefficient at every node, the
 *         outermost layer included (faces next to the boundary read it).
 *  rhs    [in] nx*ny*nz, device: dt * f at every node (read at interior
 *         nodes only).  kappa and rhs are not written and must not overlap
 *         u or u_new; they may be the same buffer.
 *  beta   dt / (2 h^2); finite and >= 0, else HC_EUNSTABLE.  The step keeps
 *         the discrete maximum principle (rhs = 0) while beta times the sum
 *         of a node's six face coefficients is <= 1: with kappa <= kmax that
 *         is beta <= 1 / (12 kmax), the paper's choice dt = h^2 / (12 kmax)
 *         gives beta = 1 / (24 kmax).  The library does not read kappa to
 *         check it.
 *  dtype  HC_F64 (the paper's precision) or HC_F32 (every array and every
 *         operation binary32, beta rounded to binary32 once).
 *  mode, parts, stream  as for heat_step_ex (HC_HEAT_SPLIT: Interior kernel
 *         on `stream`, Boundary planes on the internal stream).
 * Moves 4 values per updated node and pass (u, kappa, rhs in, u_new out);
 * with two steps per pass (hc_heat_set_time_block(2), the default) a pass
 * takes two steps, with the same bits as single steps.
 * Enqueues and returns; HC_EINVAL, HC_EALIAS as for heat_step_ex.
 */
int heat_vk_step(void *u, void *u_new, const void *kappa, const void *rhs,
                 int nx, int ny, int nz, double beta, int steps, int dtype,
                 int mode, int parts, hc_stream_t stream);

/*
 * Tile shape of the variable-coefficient sweep, per dtype (HC_F64, HC_F32),
 * same fields and rules as hc_heat_set_tiling; the shapes built are listed
 * in varcoef_kernels.hip (HC_VK_SHAPES_*).  All zeros (the default) selects
 * the automatic choice.  hc_heat_vk_tiling_for reports the shape a sweep of
 * these four arrays would run with (the one-node shape when a wide lane does
 * not fit nx or the alignment of any of them).
 */
int hc_heat_vk_set_tiling(int dtype, int vec, int wx, int by, int zdepth,
                          int pf, int xcd);
int hc_heat_vk_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth,
                          int *pf, int *xcd);
int hc_heat_vk_tiling_for(int dtype, int nx, const void *u, const void *u_new,
                          const void *kappa, const void *rhs, int *vec,
                          int *wx, int *by, int *zdepth, int *pf, int *xcd);

/* The same for the two-steps-per-pass variable-coefficient sweep (shapes
 * in varcoef2_kernels.hip, HC_VK2_SHAPES_*). */
int hc_heat_vk2_set_tiling(int dtype, int vec, int wx, int by, int zdepth,
                           int pf, int xcd);
int hc_heat_vk2_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth,
                           int *pf, int *xcd);
int hc_heat_vk2_tiling_for(int dtype, int nx, const void *u, const void *u_new,
                           const void *kappa, const void *rhs, int *vec,
                           int *wx, int *by, int *zdepth, int *pf, int *xcd);

/* Run length of the two-step variable-coefficient sweep, per dtype (HC_F64,
 * HC_F32), with hc_heat2_set_zrun's meaning and errors: 0 (the default) is
 * the automatic choice, 256 planes; other values are rounded up to a
 * multiple of the tile's zdepth.  Results do not depend on it. */
int hc_heat_vk2_set_zrun(int dtype, int planes);
int hc_heat_vk2_get_zrun(int dtype);

/*
 * cg_solve -- solve A x = b with Conjugate Gradient (the CG case study),
 * A the 7-point Laplacian 6 I - (face neighbours) on an n x n x n box with
 * zero Dirichlet data outside the box (no ghost layer is stored).
 *
 *  b      [in]  n^3 FP64, device.
 *  x      [in/out] n^3 FP64, device, must not overlap b: the initial guess
 *         on entry, the last iterate on return.
 *  tol    > 0: stop once ||r_k||_2 <= tol * ||b||_2 (recursive residual);
 *         the true residual ||b - A x|| is then recomputed and, if it is
 *         still above tol * ||b||, the iteration restarts from x (counted
 *         against maxit).
 *  maxit  >= 0 iterations in total.
 *
 * Blocks until done.  Returns HC_OK, HC_ENOTCONV (maxit reached; x holds
 * the last iterate and a later call can resume from it), HC_EBREAKDOWN or
 * HC_ENONFINITE.  ||b|| = 0 sets x = 0 and returns HC_OK.  Uses a
 * workspace the library allocates per device and keeps until unload;
 * hc_cg_last_info() returns the iteration count and true relative
 * residual of the calling thread's last cg_solve.
 */
int cg_solve(const double *b, double *x, int n, double tol, int maxit);

/*
 * cg_solve_ex -- cg_solve on an nx x ny x nz box, with a caller workspace
 * (work may be NULL: the library's own is used) and stream.
 *  work        NULL, or device memory of the current device, 256-byte
 *              aligned (else HC_EINVAL: the solver's scalar block and
 *              partial sums, some updated atomically, sit at multiples of
 *              256 bytes from it), not overlapping b or x.
 *  work_bytes  >= cg_workspace_bytes(nx, ny, nz) when work != NULL.
 *  iters, true_relres  optional outputs (may be NULL).
 * Blocks until done (the host reads the solver's scalars, about a hundred
 * bytes, back once per batch of 16 iterations to test convergence).
 * Solves on one device are serialized: the library's workspace and the
 * host buffer the scalars are read into are shared per device, so a call
 * holds a per-device lock until it returns (a second host thread's solve
 * on the same device waits; solves on different devices run side by
 * side).
 */
int cg_solve_ex(const double *b, double *x, int nx, int ny, int nz, double tol,
                int maxit, void *work, size_t work_bytes, hc_stream_t stream,
                int *iters, double *true_relres);

/* Bytes of device workspace cg_solve_ex needs (0 for invalid sizes): the
 * residual and four direction vectors, each with a zero plane below and
 * above the box, per-block partial sums and the scalar block (about 676 MB
 * at 256^3). */
size_t cg_workspace_bytes(int nx, int ny, int nz);

/*
 * cg_solve_noalloc -- cg_solve_ex for callers that cannot allocate device
 * memory (code next to HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same solver and kernels, with the same
 * results bit for bit as cg_solve_ex with the same tile shape, but its
 * workspace is a fixed array of HC_CG_NOALLOC_BYTES bytes of device memory
 * that the library's code object holds on every GPU it runs on until the
 * process ends.  The call allocates nothing: no hipMalloc, hipFree,
 * hipHostMalloc, stream or event creation (kernel timing through hc_prof_*
 * is not taken for it).
 *
 *  b, x, nx, ny, nz, tol, maxit, stream, iters, true_relres  as cg_solve_ex.
 *  Size limit: cg_workspace_bytes(nx, ny, nz) + 16384 (the store target of
 *  lanes outside the box) must not exceed HC_CG_NOALLOC_BYTES, else
 *  HC_EINVAL before any device work (a 128^3 box needs about 85 MB, the
 *  largest cube is 135^3).
 *
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents; nothing in it is read before the call writes it.  The
 * library holds a per-device lock for the whole call, so calls from several
 * host threads of one process run one after another; calls that overlap on
 * one GPU without that lock (another copy of the library loaded in the same
 * process) would race on the array.  Blocks until done; same statuses as
 * cg_solve_ex.
 */
#define HC_CG_NOALLOC_BYTES (96u << 20)
int cg_solve_noalloc(const double *b, double *x, int nx, int ny, int nz, double tol,
                     int maxit, hc_stream_t stream, int *iters, double *true_relres);

/* Iteration count and true relative residual of this thread's last CG. */
void hc_cg_last_info(int *iters, double *true_relres);

/*
 * hc_lap7_apply -- y = A x with the CG operator above (the SpMV of the CG
 * case study, Pseudocode alg:spmv, one row per node, matrix-free):
 *     y = 6 x - (((x- + x+) + (y- + y+)) + (z- + z+)), outside = 0.
 * x, y: nx*ny*nz FP64 device arrays, not overlapping.  Enqueued on
 * `stream`, does not wait.
 */
int hc_lap7_apply(const double *x, double *y, int nx, int ny, int nz,
                  hc_stream_t stream);

/*
 * hc_copy_probe -- dst[0:bytes) = src[0:bytes) with a streaming kernel of
 * the library's own (the practical HBM ceiling the stencil is compared
 * with).  bytes must be a multiple of 16 and both pointers 16-byte
 * aligned and non-overlapping.  Enqueued on `stream`, does not wait.
 */
int hc_copy_probe(const void *src, void *dst, size_t bytes, hc_stream_t stream);

/*
 * Tile shape of the z-marching heat kernels for element type `dtype` (an
 * hc_dtype), for the whole process (the knob an autotuner turns; results
 * do not depend on it, bit for bit).  A block covers 64*vec*wx nodes along
 * x by `by` rows and walks `zdepth` planes along z.
 *  vec     nodes per lane along x: 1, 2 (FP64), 4 (FP32) or 8 (bfloat16);
 *          a lane of vec > 1 nodes is one access of vec elements, used only
 *          when nx is a multiple of vec and both arrays are aligned to
 *          vec elements, else the shape (1, 4, 4, 16, 2) is used
 *  wx      wavefronts per tile row
 *  by      rows per tile
 *  zdepth  planes per z-block
 *  pf      planes of loads kept in flight ahead of the computed one (1 to 4)
 *  xcd     0..64: runs of this many y-neighbouring tiles are dealt to one
 *          XCD (so their shared halo rows are read through one L2); 0 or 1
 *          keeps the hardware order
 * The shapes built per element type are listed in heat_kernels.hip
 * (HC_HEAT_SHAPES_F64/_F32/_BF16); others, and an unknown dtype, return
 * HC_EINVAL.  All six values zero select the automatic choice (the
 * default): per call, the widest of a short list of measured shapes whose
 * row of tiles is at most 1/8 wider than nx needs.  hc_heat_get_tiling
 * writes the setting (zeros for automatic) through the non-NULL pointers.
 */
int hc_heat_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf,
                       int xcd);
int hc_heat_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth,
                       int *pf, int *xcd);

/*
 * The tile shape heat_step_ex (heat_step_sr for HC_BF16_SR) would run an
 * array of x-edge nx and element type dtype with, for the arrays u and
 * u_new (only their addresses are used, for the lane alignment; NULL counts
 * as aligned): the setting above (HC_BF16_SR uses HC_BF16's) or the
 * automatic choice, then the one-node shape (1, 4, 4, 16, 2) where vec
 * nodes per lane do not fit.  Written through the non-NULL pointers.
 * HC_EINVAL for an unknown dtype or nx < 3.
 */
int hc_heat_tiling_for(int dtype, int nx, const void *u, const void *u_new,
                       int *vec, int *wx, int *by, int *zdepth, int *pf,
                       int *xcd);

/*
 * Tile shape of the CG kernels (and hc_lap7_apply), for the whole process;
 * same meaning as for the heat kernels.  The shapes built are listed in
 * cg_kernels.hip (HC_CG_SHAPES); others return HC_EINVAL.  Results are
 * deterministic for a given shape; the summation tree of the dot products
 * (and so the last bits of the iterates) depends on it.  Default: vec 2,
 * wx 1, by 4, zdepth 16, xcd 8.
 */
int hc_cg_set_tiling(int vec, int wx, int by, int zdepth, int xcd);
void hc_cg_get_tiling(int *vec, int *wx, int *by, int *zdepth, int *xcd);

/* Name of a status code (static string). */
const char *hc_strerror(int code);

/*
 * cg_solve_ir -- the same system solved by iterative refinement around a
 * binary32 inner CG, the precision direction of the CG case study: the
 * inner iterations move 32 bytes per unknown instead of 64, while the
 * residual b - A x, the solution updates and every dot product stay in
 * binary64, so the accuracy reached is that of binary64 CG.
 *
 *   outer:  r = b - A x (binary64); stop when ||r|| <= tol ||b|| (the true
 *           residual: no restart is needed); s = r rounded to binary32;
 *           d = inner CG on A d = s from d = 0; x = x + d (binary64).
 *   inner:  textbook CG with binary32 vectors and arithmetic (operator
 *           6 p - neighbours, updates d + alpha p, s - alpha q, directions
 *           s + beta p), dot products accumulated in binary64, alpha and
 *           beta computed in binary64 and rounded to binary32; it stops at
 *           ||s|| <= max(inner_tol ||s_0||, 0.5 tol ||b||).
 *
 *  b, x, nx, ny, nz, tol   as cg_solve_ex.
 *  maxit      >= 0 inner iterations in total over all outer steps.
 *  inner_tol  relative reduction of each inner solve, < 1; <= 0 selects
 *             1e-5.
 *  work       NULL (the library's cached workspace) or at least
 *             cg_ir_workspace_bytes(nx, ny, nz) bytes of device memory,
 *             256-byte aligned (else HC_EINVAL).  Serialized per device
 *             with the other solves, as cg_solve_ex.
 *  iters, outer, true_relres  optional outputs: inner iterations, outer
 *             steps, binary64 ||b - A x|| / ||b|| of the returned x.
 * Blocks until done.  Returns HC_OK, HC_ENOTCONV (maxit reached, or an
 * outer step that did not reduce ||r||, or 64 outer steps; x holds the last
 * iterate), HC_EBREAKDOWN (p.Ap <= 0 at the start of an inner solve) or
 * HC_ENONFINITE; ||b|| = 0 sets x = 0 and returns HC_OK.
 */
int cg_solve_ir(const double *b, double *x, int nx, int ny, int nz, double tol,
                int maxit, double inner_tol, void *work, size_t work_bytes,
                hc_stream_t stream, int *iters, int *outer, double *true_relres);

/* Bytes of the workspace cg_solve_ir needs (0 for an empty box). */
size_t cg_ir_workspace_bytes(int nx, int ny, int nz);

/*
 * hc_lap7_apply_f32 -- y = A x for binary32 arrays, each operation of
 * 6 x_p - (((x- + x+) + (y- + y+)) + (z- + z+)) rounded to binary32 (the
 * inner operator of cg_solve_ir).  Same rules as hc_lap7_apply.
 */
int hc_lap7_apply_f32(const float *x, float *y, int nx, int ny, int nz,
                      hc_stream_t stream);

/*
 * Tile shape of the binary32 inner CG kernels of cg_solve_ir and of
 * hc_lap7_apply_f32 (same meaning as hc_cg_set_tiling; vec up to 4, i.e.
 * 16-byte lanes, used when nx is a multiple of vec and the vectors are
 * aligned to a lane).  The shapes built are listed in cg_kernels.hip
 * (HC_CG_SHAPES_F32).  Default: vec 4, wx 1, by 8, zdepth 32, xcd 8.
 */
int hc_cg_ir_set_tiling(int vec, int wx, int by, int zdepth, int xcd);
void hc_cg_ir_get_tiling(int *vec, int *wx, int *by, int *zdepth, int *xcd);

/*
 * Batched heat: many independent problems of uneven size advanced together,
 * one launch per time step (each problem's sweep is heat_step's, bit for
 * bit; only its launches are shared).
 *
 * The problems' arrays are packed one after another in one buffer per
 * state.  Problem p (edges nx, ny, nz = dims[3p .. 3p+2]) starts
 * offsets[p] elements in (a multiple of 64 bytes); node (i, j, k) is at
 * offsets[p] + (k*ny + j)*pitches[p] + i, where pitches[p] >= nx rounds nx
 * up to 16 bytes.  Elements i = nx .. pitch-1 of a row are padding: never
 * read by an update, their contents are unspecified on return.
 */
typedef struct hc_batch hc_batch;

/*
 * hc_batch_create -- describe `count` (1 .. 2^20) problems: dims[3*count]
 * edges (each in [3, 2^20], else HC_EINVAL), r[count] coefficients
 * (finite, 0 <= r <= 1/6, else HC_EUNSTABLE), element type dtype (HC_F64,
 * HC_F32 or HC_BF16 with heat_step_ex's arithmetic).  The library copies
 * the description and keeps device tables (the problems, the work list of
 * the current tile shape) and a stream for its graphs, all released by
 * hc_batch_destroy.  The batch belongs to the current device.
 */
int hc_batch_create(int count, const int *dims, const double *r, int dtype,
                    hc_batch **out);
void hc_batch_destroy(hc_batch *b);

/*
 * Packed layout: offsets[count] and pitches[count] (elements; either may be
 * NULL), the total number of elements each state buffer must hold, and the
 * algorithmic bytes of one step of every problem (every stored node read
 * once, every updated node written once; padding not counted).
 */
int hc_batch_layout(const hc_batch *b, long long *offsets, int *pitches,
                    long long *total_elems, double *step_bytes);

/*
 * hc_batch_step -- advance every problem by `steps` steps.
 *  u, u_new  device buffers of total_elems elements, 64-byte aligned, not
 *            overlapping; u holds the states on entry and on return, u_new
 *            is scratch (its Dirichlet layers are first copied from u: the
 *            whole buffer is copied once).
 *  use_graph 0: one kernel launch per step on `stream`; 1: the step loop is
 *            captured once in a HIP graph (kept by the batch for these
 *            buffers, this step count and tile shape) and launched as one
 *            graph, joined to `stream` through events.
 * Each launch runs a persistent kernel whose blocks walk the work list of
 * (problem, x-tile, y-tile, run of planes) entries; with two steps per pass
 * (hc_batch_steps_per_pass) there is one launch per width class and pass,
 * each class's passes in a chain of their own on an internal stream.
 * Enqueued; does not wait.
 */
int hc_batch_step(hc_batch *b, void *u, void *u_new, int steps, int use_graph,
                  hc_stream_t stream);

/*
 * Block shape of the batch (from the list in batch_kernels.hip,
 * HC_BATCH_SHAPES_*): vec nodes per lane (16 bytes), `threads` per block,
 * runs walked in unrolled sub-blocks of zdepth planes, pf planes of loads
 * in flight; `xcd` (0..64): runs of that many consecutive work-list entries
 * dealt to the blocks of one XCD (0 or 1: hardware order);
 * `width_class`: -1 gives every problem the tile width whose tiles cover
 * its nx columns and ny-2 updated rows with the fewest idle threads (the
 * wider on a tie), c = 0..4 gives every problem rows of 8 << c lanes (threads >> (3+c)
 * rows; a class exists when that is at least 4 rows and the tile has one
 * thread per halo element); `grid`: the persistent grid size (0: one block
 * per work-list entry); `item_depth`: the planes per work-list entry (0: a
 * problem's whole column; else near-equal runs of at least
 * max(item_depth, zdepth) planes).  hc_batch_classes writes the width
 * class each problem gets (classes[count]).  A new batch starts with vec
 * 16 / element size, 256 threads for HC_F32 and 512 otherwise, zdepth 16,
 * pf 2, xcd 8, width class -1, grid 0, item_depth 64.
 */
int hc_batch_set_tiling(hc_batch *b, int vec, int threads, int zdepth, int pf,
                        int xcd, int width_class, int grid, int item_depth);
int hc_batch_get_tiling(const hc_batch *b, int *vec, int *threads, int *zdepth,
                        int *pf, int *xcd, int *width_class, int *grid,
                        int *item_depth);
int hc_batch_classes(hc_batch *b, int *classes);

/*
 * hc_batch_autotune -- time every built block shape with each problem's
 * best-fitting width, hardware and XCD-grouped (8) order, whole-column,
 * one-z-block, 32- and 64-plane entries, one block per entry or a
 * persistent grid of 2 blocks per compute unit, and with every width class
 * for all problems, over
 * trial_steps (rounded up to even) steps of the states in u (on two
 * scratch buffers the call allocates and frees; u is not written), time the
 * four fastest again over twice as many steps, twice each, and keep the
 * fastest of those.  Blocks until done; *best_ms (may be NULL) receives its
 * time per step in that second round (hc_batch_tune_result gives the first
 * round's times).  hc_batch_tune_result(b, i, shape8, ms) returns
 * candidate i's setting {vec, threads, zdepth, pf, xcd, width_class, grid,
 * item_depth} and time per step; with i < 0 it returns the number of
 * candidates.
 */
int hc_batch_autotune(hc_batch *b, const void *u, int trial_steps, hc_stream_t stream,
                      double *best_ms);
int hc_batch_tune_result(const hc_batch *b, int index, int *shape8, double *ms_per_step);

/*
 * Steps per pass hc_batch_step takes with the batch's current shape: 2 when
 * hc_heat_set_time_block(2) is in effect (the default) and the shape is
 * built for two steps (HC_BATCH2_SHAPES_* in batch2_kernels.hip; a last odd
 * step then takes one pass), else 1; HC_EINVAL for a NULL batch.  The result
 * of a step does not depend on it.
 */
int hc_batch_steps_per_pass(const hc_batch *b);

/* Detail of the last failure on the calling thread ("" if none). */
const char *hc_last_error_message(void);

/*
 * Kernel timing for measurement.  hc_prof_enable(every) with every >= 1
 * clears the counters and from then on brackets one launch in every `every`
 * of each kernel kind (the middle one of each group, so that no timed CG
 * launch follows the solver's periodic wait for the host) with HIP events
 * on the stream it runs on (the events cost
 * a few microseconds of GPU time each, so sampling keeps the measured run
 * close to an unmeasured one), adding up the algorithmic bytes each timed
 * launch must move; every = 0 stops timing.  hc_prof_read waits for the
 * recorded launches and returns, for one kernel kind, the total duration
 * (ms), the number of timed launches and their algorithmic bytes.
 */
enum hc_kernel_kind {
    HC_K_HEAT_INTERIOR = 0,
    HC_K_HEAT_BOUNDARY = 1,
    HC_K_HEAT_FUSED = 2,
    HC_K_HEAT_PLAIN = 3,
    HC_K_CG_DIRECTION = 4, /* p = r + beta p, A p, p.Ap   */
    HC_K_CG_UPDATE = 5,    /* r -= alpha A p, r.r (x's step waits) */
    HC_K_CG_RESIDUAL = 6,  /* r = b - A x, r.r, b.b      */
    HC_K_LAP7 = 7,
    HC_K_COPY = 8,
    HC_K_CG32_DIRECTION = 9,  /* the same, binary32 (refinement) */
    HC_K_CG32_UPDATE = 10,    /* s -= alpha A p, s.s (d's step waits) */
    HC_K_IR_RESIDUAL = 11,    /* r = b - A x, s = (float) r, sums */
    HC_K_IR_UPDATE = 12,      /* x += d                        */
    HC_K_BATCH = 13,          /* a batch step (graph: all steps) */
    HC_K_VK_INTERIOR = 14,    /* variable coefficient: Interior  */
    HC_K_VK_BOUNDARY = 15,
    HC_K_VK_FUSED = 16,
    HC_K_VK_PLAIN = 17,
    HC_K_HEAT2_INTERIOR = 18, /* two steps per pass            */
    HC_K_HEAT2_BOUNDARY = 19,
    HC_K_HEAT2_FUSED = 20,
    HC_K_VK2_INTERIOR = 21,   /* variable coefficient, two steps */
    HC_K_VK2_BOUNDARY = 22,
    HC_K_VK2_FUSED = 23,
    HC_K_CG_UPDATE_X = 24,    /* HC_K_CG_UPDATE and x's last four steps */
    HC_K_CG32_UPDATE_X = 25,  /* HC_K_CG32_UPDATE and d's last two steps */
    HC_K_COUNT = 26
};
int hc_prof_enable(int every);
int hc_prof_read(int kind, double *total_ms, long long *launches,
                 double *algo_bytes);

#ifdef __cplusplus
}
#endif

#endif /* HEATCG_H */
