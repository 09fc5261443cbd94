// abi.cpp -- the exported C ABI of libheatcg.so (declared in heatcg.h):
// argument validation, per-device streams and events, the time-step loop
// with its Interior/Boundary fork-join, the CG driver and kernel timing.

#include "../../include/heatcg.h"
#include "hc_internal.hpp"

#include <algorithm>
#include <cstdint>
#include <new>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Device memory of cg_solve_noalloc, the entry point for callers that cannot
// allocate: every GPU the library runs on holds its own copy until the
// process ends.  In host code this name is not a device address; the
// address is looked up once per device (scratch_slot) and used instead.
static __device__ __align__(256) unsigned char scratch[HC_CG_NOALLOC_BYTES];

namespace {

using hc::KernelKind;

thread_local std::string g_msg;
thread_local int g_cg_iters = 0;
thread_local double g_cg_relres = 0.0;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_msg = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(HC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HC_TRY(call, what)                         \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ---- tile shape of the heat kernels (settable for tuning) -------------------
std::mutex g_tiling_mu;
// Per storage precision: a shape set by the caller, or all zeros for the
// automatic choice (the default).
hc::HeatTiling g_tiling[3] = {};

hc::HeatTiling current_tiling(int dtype) {
    std::lock_guard<std::mutex> g(g_tiling_mu);
    return g_tiling[dtype];
}

// Automatic choice: candidates per precision, widest tile first, all with
// 16-byte lanes where the width allows, z-blocks of 16-32 planes, two planes
// of loads in flight and runs of 8 y-neighbouring tiles per XCD (the fastest
// shapes of a sweep over the built ones at 512^3 and 1024^3 on MI355X).
// The first candidate whose row of tiles is at most 1/8 wider than the
// narrowest candidate's wins: wide tiles amortise the ring and the block
// set-up, but lanes past the last column do no work.
// The stochastic-rounding form draws one generator block per lane and
// plane, so it favours 8-node lanes even more.
const hc::HeatTiling kAuto[4][5] = {
    {{2, 4, 4, 32, 2, 8}, {2, 2, 8, 16, 2, 8}, {2, 1, 8, 16, 2, 8}, {1, 1, 8, 16, 2, 8}, {}},
    {{4, 4, 4, 16, 2, 8}, {2, 4, 4, 32, 2, 8}, {4, 1, 8, 32, 2, 8}, {2, 1, 8, 32, 2, 8},
     {1, 1, 8, 16, 2, 8}},
    {{8, 1, 8, 16, 2, 8}, {4, 1, 8, 16, 2, 8}, {2, 1, 8, 16, 2, 8}, {1, 1, 8, 16, 2, 8}, {}},
    {{8, 1, 4, 32, 2, 8}, {4, 1, 8, 16, 2, 8}, {2, 1, 8, 16, 2, 8}, {1, 1, 8, 16, 2, 8}, {}},
};

hc::HeatTiling auto_tiling(int dtype, int nx) {
    long long best = -1;
    for (const hc::HeatTiling &c : kAuto[dtype]) {
        if (c.vec == 0) break;
        const long long w = hc::tile_width(c);
        const long long padded = (nx + w - 1) / w * w;
        if (best < 0 || padded < best) best = padded;
    }
    for (const hc::HeatTiling &c : kAuto[dtype]) {
        if (c.vec == 0) break;
        const long long w = hc::tile_width(c);
        if ((nx + w - 1) / w * w * 8 <= best * 9) return c;
    }
    return kAuto[dtype][0];
}

// The shape a sweep of these arrays runs with: the caller's or the automatic
// one, then the one-node shape when vec nodes per lane do not fit (rows that
// are not whole lanes, or arrays not aligned to a lane).
hc::HeatTiling heat_tiling_for(int dtype, int nx, const void *u, const void *un) {
    const int tdt = dtype == hc::kDtypeBF16SR ? hc::kDtypeBF16 : dtype;  // same storage
    hc::HeatTiling til = current_tiling(tdt);
    if (til.vec == 0) til = auto_tiling(dtype, nx);
    const uintptr_t lane_bytes = (uintptr_t)til.vec * (uintptr_t)hc::dtype_bytes(dtype);
    if (til.vec > 1 && ((nx % til.vec) || (reinterpret_cast<uintptr_t>(u) % lane_bytes) ||
                        (reinterpret_cast<uintptr_t>(un) % lane_bytes)))
        til = {1, 4, 4, 16, 2, til.xcd};
    return til;
}

// Tile shape of the variable-coefficient sweep, per precision (FP64, FP32):
// set by the caller, or all zeros for the automatic choice.  Its candidates
// are built in a list of their own (two LDS planes and two register queues
// per tile, so narrower tiles than for the constant coefficient).
hc::HeatTiling g_vk_tiling[2] = {};
// The candidates are the fastest shapes of a sweep over the built ones at
// 512^3 on MI355X (binary32 runs fastest with one-node lanes here).
const hc::HeatTiling kVkAuto[2][4] = {
    {{2, 4, 4, 32, 2, 8}, {2, 2, 8, 16, 2, 8}, {2, 1, 8, 16, 2, 8}, {1, 1, 8, 16, 2, 8}},
    {{1, 4, 4, 16, 2, 8}, {4, 1, 8, 16, 2, 8}, {1, 1, 8, 16, 2, 8}, {}},
};

// Two-step variable-coefficient sweep: shapes of its own, per precision;
// the automatic one is the fastest of a sweep over the built ones (with run
// lengths and block orders) at 512^3 on MI355X: 16-byte lanes, one plane of
// loads ahead (the register queues of u and kappa are long: about 200
// VGPRs, two wavefronts per SIMD), FP64 tiles 128 nodes wide and 8 rows
// tall (512 threads, the most that two wavefronts per SIMD allow; half the
// y-ring per node of 4-row tiles: 7% faster at runs of 256 planes); FP32
// tiles 256 x 4 with two planes of loads ahead in slab order (19% faster
// than the one-z-block, one-plane-ahead shape before the runs).
hc::HeatTiling g_vk2_tiling[2] = {};
const hc::HeatTiling kVk2Auto[2][2] = {
    {{2, 1, 8, 32, 1, 8}, {}},
    {{4, 1, 4, 32, 2, -1}, {}},
};

hc::HeatTiling vk2_tiling_for(int dtype, int nx, const void *const *arrays, int narrays) {
    hc::HeatTiling til;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        til = g_vk2_tiling[dtype];
    }
    if (til.vec == 0) til = kVk2Auto[dtype][0];
    const uintptr_t lane_bytes = (uintptr_t)til.vec * (uintptr_t)hc::dtype_bytes(dtype);
    bool fits = til.vec == 1 || nx % til.vec == 0;
    for (int q = 0; q < narrays && fits; ++q)
        fits = reinterpret_cast<uintptr_t>(arrays[q]) % lane_bytes == 0;
    if (!fits) til = {1, 4, 4, 16, 2, til.xcd};
    return til;
}

hc::HeatTiling vk_tiling_for(int dtype, int nx, const void *const *arrays, int narrays) {
    hc::HeatTiling til;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        til = g_vk_tiling[dtype];
    }
    if (til.vec == 0) {
        long long best = -1;
        for (const hc::HeatTiling &c : kVkAuto[dtype]) {
            if (c.vec == 0) break;
            const long long w = hc::tile_width(c);
            const long long padded = (nx + w - 1) / w * w;
            if (best < 0 || padded < best) best = padded;
        }
        til = kVkAuto[dtype][0];
        for (const hc::HeatTiling &c : kVkAuto[dtype]) {
            if (c.vec == 0) break;
            const long long w = hc::tile_width(c);
            if ((nx + w - 1) / w * w * 8 <= best * 9) {
                til = c;
                break;
            }
        }
    }
    const uintptr_t lane_bytes = (uintptr_t)til.vec * (uintptr_t)hc::dtype_bytes(dtype);
    bool fits = til.vec == 1 || nx % til.vec == 0;
    for (int q = 0; q < narrays && fits; ++q)
        fits = reinterpret_cast<uintptr_t>(arrays[q]) % lane_bytes == 0;
    if (!fits) til = {1, 4, 4, 16, 2, til.xcd};
    return til;
}

// Steps per pass of the z-marching constant-coefficient sweeps (1 or 2;
// two by default: a pass then moves half the bytes per step).  The
// two-step sweep has tile shapes of its own, per storage precision; the
// automatic candidates are the fastest of sweeps over the built ones at
// 512^3 and 1024^3 on MI355X (tiles 256 nodes wide, 8 rows, z-blocks of 32
// planes, slab order: on some boxes it cut the reads the rings miss in L2
// at 1024^3, 5-10% faster than runs of 8 y-tiles per XCD; elsewhere the two
// orders measured within 1-2%).  FP64's widest tile keeps one plane of
// loads ahead (94 VGPRs against 105 with two; 1.5% faster at 512^3, 0.5% at
// 1024^3, in interleaved A/B); FP32 and bfloat16 ran 3-28% slower so.
int g_time_block = 2;
hc::HeatTiling g_tiling2[3] = {};
const hc::HeatTiling kAuto2[3][5] = {
    {{2, 2, 8, 32, 1, -1}, {2, 2, 4, 32, 2, -1}, {2, 1, 8, 32, 2, -1}, {1, 4, 4, 16, 2, 8}, {}},
    {{4, 1, 8, 32, 2, -1}, {4, 2, 4, 32, 2, -1}, {4, 1, 4, 32, 2, -1}, {1, 4, 4, 16, 2, 8}, {}},
    {{4, 1, 8, 32, 2, -1}, {4, 1, 4, 32, 2, -1}, {1, 4, 4, 16, 2, 8}, {}, {}},
};

hc::HeatTiling heat2_tiling_for(int dtype, int nx, const void *u, const void *un) {
    hc::HeatTiling til;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        til = g_tiling2[dtype];
    }
    if (til.vec == 0) {
        long long best = -1;
        for (const hc::HeatTiling &c : kAuto2[dtype]) {
            if (c.vec == 0) break;
            const long long w = hc::tile_width(c);
            const long long padded = (nx + w - 1) / w * w;
            if (best < 0 || padded < best) best = padded;
        }
        til = kAuto2[dtype][0];
        for (const hc::HeatTiling &c : kAuto2[dtype]) {
            if (c.vec == 0) break;
            const long long w = hc::tile_width(c);
            if ((nx + w - 1) / w * w * 8 <= best * 9) {
                til = c;
                break;
            }
        }
    }
    const uintptr_t lane_bytes = (uintptr_t)til.vec * (uintptr_t)hc::dtype_bytes(dtype);
    if (til.vec > 1 && ((nx % til.vec) || (reinterpret_cast<uintptr_t>(u) % lane_bytes) ||
                        (reinterpret_cast<uintptr_t>(un) % lane_bytes)))
        til = {1, 4, 4, 16, 2, til.xcd};
    return til;
}

// Planes of output per block of the two-step constant-coefficient sweep
// (its Interior and fused kernels march them as one run), set per dtype;
// 0 is the automatic choice kAutoZrun, where 0 means one z-block per block.
// Measured on MI355X (interleaved A/B on one box): FP64 runs of two
// z-blocks (64 planes) were 3% faster than one at 512^3, where a plane has
// 128 tiles of 256 x 8 and a column 16 z-blocks, but 5% slower at 1024^3
// (512 tiles a plane), so the automatic choice takes them only for planes
// of at most 256 tiles; FP32 measured alike within noise; the bfloat16
// sweep, bound by its vector ALU work, gains 5-8% from runs of 128 planes
// (fewer pipeline fills, each of which computes two planes of u^(t+1)
// twice).
int g_heat2_zrun[3] = {0, 0, 0};

int heat2_zrun(int dtype, const hc::HeatTiling &t, int nx, int ny) {
    int zr;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        zr = g_heat2_zrun[dtype];
    }
    if (zr <= 0) {
        const long long w = hc::tile_width(t);
        const long long tiles = ((nx + w - 1) / w) * ((ny - 2 + t.by - 1) / t.by);
        zr = dtype == hc::kDtypeBF16 ? 128 : (dtype == hc::kDtypeF64 && tiles <= 256) ? 64 : 0;
    }
    const int zb = t.zdepth;
    return zr <= 0 ? zb : (zr + zb - 1) / zb * zb;
}

// The same for the two-step variable-coefficient sweep (FP64, FP32).
// Measured on MI355X at the paper's 512^3 case: FP64 (128 x 8 tiles) runs
// of 256 planes 4.4% faster than one z-block, 128 planes 3.1%, whole
// columns 2.7%; FP32 (256 x 4 tiles) 256 planes 11% faster, 128 planes 9%;
// 256 planes is the automatic choice for both.
int g_vk2_zrun[2] = {0, 0};

int vk2_zrun(int dtype, const hc::HeatTiling &t) {
    int zr;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        zr = g_vk2_zrun[dtype];
    }
    if (zr <= 0) zr = 256;
    const int zb = t.zdepth;
    return zr <= 0 ? zb : (zr + zb - 1) / zb * zb;
}

int current_time_block() {
    std::lock_guard<std::mutex> g(g_tiling_mu);
    return g_time_block;
}

// Tile shape of the binary64 CG kernels: 256 x 4 tiles of 2-node lanes,
// z-blocks of 16 planes (2048 blocks at 256^3; the fastest built shape
// there on MI355X).
hc::CGTiling g_cg_tiling = {2, 1, 4, 16, 8};

// Tile shape of the refinement's binary32 inner solve: 256 x 8 tiles of
// 4-node (16-byte) lanes, z-blocks of 32 planes (the fastest built shape at
// 256^3 on MI355X).
hc::CGTiling g_cg_ir_tiling = {4, 1, 8, 32, 8};

// The inner solve's shape for these arrays: vec-node lanes need an x-edge
// that is a multiple of vec and arrays aligned to a lane, else the one-node
// shape of the same tile height.
hc::CGTiling cg_ir_tiling_for(int nx, const void *a, const void *b, const void *c,
                              const void *e) {
    hc::CGTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_cg_ir_tiling;
    }
    const uintptr_t lane = (uintptr_t)t.vec * sizeof(float);
    const uintptr_t mis = (reinterpret_cast<uintptr_t>(a) % lane) | (reinterpret_cast<uintptr_t>(b) % lane) |
                          (reinterpret_cast<uintptr_t>(c) % lane) | (reinterpret_cast<uintptr_t>(e) % lane);
    if (t.vec > 1 && ((nx % t.vec) || mis)) t = {1, 1, 4, 16, t.xcd};
    return t;
}

// The CG tile shape for these arrays: two-node lanes need an even x-edge and
// 16-byte aligned vectors, else the one-node shape of the same tile height.
hc::CGTiling cg_tiling_for(int nx, const void *a, const void *b, const void *c) {
    hc::CGTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_cg_tiling;
    }
    const uintptr_t mis = (reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                           reinterpret_cast<uintptr_t>(c)) & 15;
    if (t.vec == 2 && ((nx & 1) || mis)) t = {1, 1, 4, 16, t.xcd};
    return t;
}

// ---- per-device state -------------------------------------------------------
struct DevState {
    bool ready = false;
    hipStream_t aux = nullptr;   // the Boundary kernels' stream
    hipEvent_t ev_main = nullptr, ev_aux = nullptr;
    void *cg_work = nullptr;     // default workspace of cg_solve_ex and cg_solve_ir
    size_t cg_work_size = 0;
    hc::CGScalars *host_sc = nullptr;  // pinned
    double *sink = nullptr;  // store target of lanes outside a CG box
    // Held for the whole of a CG solve: the library's workspace, host_sc
    // and sink are shared by every solve on this device.
    std::mutex cg_mu;
};

constexpr int kMaxDev = 64;
std::mutex g_dev_mu;
DevState g_dev[kMaxDev];

int device_state(DevState **out) {
    int dev = 0;
    HC_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDev) return fail(HC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_dev_mu);
    DevState &d = g_dev[dev];
    if (!d.ready) {
        HC_TRY(hipStreamCreateWithFlags(&d.aux, hipStreamNonBlocking), "hipStreamCreate");
        HC_TRY(hipEventCreateWithFlags(&d.ev_main, hipEventDisableTiming), "hipEventCreate");
        HC_TRY(hipEventCreateWithFlags(&d.ev_aux, hipEventDisableTiming), "hipEventCreate");
        void *h = nullptr;
        HC_TRY(hipHostMalloc(&h, sizeof(hc::CGScalars), hipHostMallocDefault), "hipHostMalloc");
        d.host_sc = static_cast<hc::CGScalars *>(h);
        void *sk = nullptr;
        HC_TRY(hipMalloc(&sk, hc::kSinkDoubles * sizeof(double)), "hipMalloc (sink)");
        d.sink = static_cast<double *>(sk);
        d.ready = true;
    }
    *out = &d;
    return HC_OK;
}

// ---- the fixed workspace of cg_solve_noalloc ----------------------------------------
// Its first kNoallocSinkBytes take the stores of lanes outside the box (the
// CG kernels' sink), the rest is carved like a caller's CG workspace.
constexpr size_t kNoallocSinkBytes = 256 * ((hc::kSinkDoubles * sizeof(double) + 255) / 256);

struct ScratchSlot {
    std::mutex mu;                 // held for a whole solve: one array per device
    bool ready = false;
    unsigned char *ptr = nullptr;  // the array's device address on this device
    hc::CGScalars host;            // the solver's scalars, read back at every poll
};
ScratchSlot g_scratch_slot[kMaxDev];

// The current device's slot; on its first use the device address of
// `scratch` is looked up with that device current (no allocation).
int scratch_slot(ScratchSlot **out) {
    int dev = 0;
    HC_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDev) return fail(HC_EINVAL, "device %d out of range", dev);
    ScratchSlot &sl = g_scratch_slot[dev];
    std::lock_guard<std::mutex> g(sl.mu);
    if (!sl.ready) {
        void *p = nullptr;
        HC_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)");
        if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256 != 0)
            return fail(HC_EHIP, "the fixed CG workspace has no usable device address");
        sl.ptr = static_cast<unsigned char *>(p);
        sl.ready = true;
    }
    *out = &sl;
    return HC_OK;
}

// ---- kernel timing -------------------------------------------------------------
struct Pending {
    int kind;
    hipEvent_t a, b;
    double bytes;
    long long launches;  // launches the events bracket
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_every = 1;                 // time every n-th launch of a kind
long long g_prof_seen[hc::K_COUNT];   // launches of each kind since enable
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
double g_prof_ms[hc::K_COUNT];
long long g_prof_n[hc::K_COUNT];
double g_prof_bytes[hc::K_COUNT];

hipEvent_t pool_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with timing events while profiling is enabled.
class Timed {
  public:
    Timed(KernelKind kind, hipStream_t s, double bytes, long long launches = 1,
          bool allowed = true)
        : kind_(kind), s_(s), bytes_(bytes), launches_(launches) {
        if (!allowed) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on) return;
        // the middle launch of every group of g_prof_every: the CG loop
        // waits for the host after every 16th iteration, and a launch right
        // after such a wait would time the host's enqueue too
        if (g_prof_seen[kind]++ % g_prof_every != g_prof_every / 2) return;
        a_ = pool_event();
        b_ = pool_event();
        if (a_ && b_ && hipEventRecord(a_, s_) == hipSuccess) on_ = true;
    }
    void done() {
        if (!on_) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (hipEventRecord(b_, s_) == hipSuccess)
            g_pending.push_back({(int)kind_, a_, b_, bytes_, launches_});
        on_ = false;
    }

  private:
    KernelKind kind_;
    hipStream_t s_;
    double bytes_;
    long long launches_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool on_ = false;
};

// ---- validation helpers ----------------------------------------------------------
bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

// The pointer must be device memory (or managed memory) of the current
// device whose allocation holds `bytes` bytes from it.  Anything the runtime
// cannot vouch for is rejected, so no kernel is ever launched on a buffer
// that could make it fault.
int check_device_buffer(const void *p, size_t bytes, const char *name) {
    int dev = 0;
    HC_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HC_EINVAL, "%s is not a device pointer (%s)", name, hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(HC_EINVAL, "%s is not device memory (memory type %d)", name, (int)attr.type);
    if (attr.type == hipMemoryTypeDevice && attr.device != dev)
        return fail(HC_EINVAL, "%s lives on device %d, current device is %d", name, attr.device, dev);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void *>(p));
    if (e != hipSuccess || base == nullptr) {
        (void)hipGetLastError();
        return fail(HC_EINVAL, "%s: the size of its allocation is unknown", name);
    }
    const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
    if (reinterpret_cast<uintptr_t>(p) + bytes > end)
        return fail(HC_EINVAL, "%s: its allocation holds %zu bytes from the pointer, %zu needed",
                    name, (size_t)(end - reinterpret_cast<uintptr_t>(p)), bytes);
    return HC_OK;
}

int check_dims(int nx, int ny, int nz, int min_edge, size_t elem, size_t *bytes) {
    if (nx < min_edge || ny < min_edge || nz < min_edge)
        return fail(HC_EINVAL, "edges (%d, %d, %d) must each be >= %d", nx, ny, nz, min_edge);
    const double n = (double)nx * ny * nz;
    if (n * elem > 9.0e15) return fail(HC_EINVAL, "array of %.3g nodes is too large", n);
    *bytes = (size_t)nx * ny * nz * elem;
    return HC_OK;
}

// ---- heat: k-range tables ------------------------------------------------------
void push_range(hc::ZTable &t, int kb, int ke, int depth) {
    if (ke < kb) return;
    const int i = t.n++;
    t.kb[i] = kb;
    t.ke[i] = ke;
    t.depth[i] = depth;
    t.first[i + 1] = t.first[i] + (ke - kb + depth) / depth;
}

hc::ZTable empty_table() {
    hc::ZTable t;
    std::memset(&t, 0, sizeof t);
    return t;
}

// Slab s of `parts` covers the updated planes [a_s, b_s] (k-decomposition).
void slab(int nz, int parts, int s, int *a, int *b) {
    const long long m = nz - 2;
    *a = 1 + (int)((s * m) / parts);
    *b = (int)(((s + 1) * m) / parts);
}

// Bytes a z-marching launch over `t` must move: every stored node of the
// planes it reads (kb-1 .. ke+1 of each range, counted once) plus every
// node it writes.
double tile_algo_bytes(const hc::ZTable &t, int nx, int ny, int nz, size_t elem, int halo = 1) {
    std::vector<char> rd(nz, 0);
    long long written = 0;
    for (int q = 0; q < t.n; ++q) {
        for (int k = std::max(0, t.kb[q] - halo); k <= std::min(nz - 1, t.ke[q] + halo); ++k)
            rd[k] = 1;
        written += t.ke[q] - t.kb[q] + 1;
    }
    long long planes = 0;
    for (char c : rd) planes += c;
    return (double)elem * ((double)planes * nx * ny + (double)written * (nx - 2) * (ny - 2));
}

// The explicit sweep in any of its forms.  With kap == nullptr it is the
// constant-coefficient step with r; otherwise the variable-coefficient step
// with source rhs and beta = r (FP64 or FP32).
// bnd (with own_bnd): the stream of the Boundary kernels in the split form,
// else the library's internal stream; it joins s at every step through
// events.
int heat_run(int dtype, void *u, void *un, int nx, int ny, int nz, double r, int steps, int mode,
             int parts, unsigned long long seed, unsigned long long step0, hipStream_t s,
             const void *kap = nullptr, const void *rhs = nullptr, bool own_bnd = false,
             hipStream_t bnd = nullptr) {
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc) return rc;
    hipStream_t const aux = own_bnd ? bnd : d->aux;
    const bool vk = kap != nullptr;
    const size_t eb = (size_t)hc::dtype_bytes(dtype);
    const void *arrays[4] = {u, un, kap, rhs};
    const hc::HeatTiling til = vk ? vk_tiling_for(dtype, nx, arrays, 4)
                                  : heat_tiling_for(dtype, nx, u, un);
    // algorithmic bytes: u (and kappa) over every node read, rhs and u_new
    // over the updated nodes
    const double fields = vk ? 2.0 : 1.0;
    const double plain_bytes =
        (double)eb * fields * ((double)nx * ny * nz + (double)(nx - 2) * (ny - 2) * (nz - 2));
    const hc::KernelKind k_plain = vk ? hc::K_VK_PLAIN : hc::K_HEAT_PLAIN;
    const hc::KernelKind k_fused = vk ? hc::K_VK_FUSED : hc::K_HEAT_FUSED;
    const hc::KernelKind k_int = vk ? hc::K_VK_INTERIOR : hc::K_HEAT_INTERIOR;
    const hc::KernelKind k_bd = vk ? hc::K_VK_BOUNDARY : hc::K_HEAT_BOUNDARY;

    hc::ZTable tin = empty_table(), tbd = empty_table();
    if (mode == HC_HEAT_SPLIT) {
        for (int q = 0; q < parts; ++q) {
            int a, b;
            slab(nz, parts, q, &a, &b);
            push_range(tin, a + 1, b - 1, til.zdepth);
        }
        for (int q = 0; q < parts; ++q) {
            int a, b;
            slab(nz, parts, q, &a, &b);
            push_range(tbd, a, a, 1);
            if (b != a) push_range(tbd, b, b, 1);
        }
    } else if (mode == HC_HEAT_FUSED) {
        push_range(tin, 1, nz - 2, til.zdepth);
    }
    const long long nb_in = hc::heat_tile_blocks(nx, ny, til, tin);
    const long long nb_bd = hc::heat_tile_blocks(nx, ny, til, tbd);
    if (nb_in > 2147483647LL || nb_bd > 2147483647LL)
        return fail(HC_EINVAL, "grid too large for this tile shape");
    const double bytes_in = fields * tile_algo_bytes(tin, nx, ny, nz, eb);
    const double bytes_bd = fields * tile_algo_bytes(tbd, nx, ny, nz, eb);
    auto tile_launch = [&](hc::KernelKind kind, const hc::ZTable &zt, const void *a, void *b,
                           unsigned long long step, hipStream_t st) {
        return vk ? hc::launch_heat_vk_tile(dtype, kind, a, kap, rhs, b, nx, ny, r, zt, til, st)
                  : hc::launch_heat_tile(dtype, kind, a, b, nx, ny, r, zt, til, seed, step, st);
    };

    // two steps per pass where the sweep allows it (constant coefficient,
    // nearest rounding, z-marching forms); a last odd step takes one pass
    const bool two = dtype != hc::kDtypeBF16SR && mode != HC_HEAT_PLAIN && steps >= 2 &&
                     current_time_block() == 2;
    hc::HeatTiling til2 = {}, til2b = {};
    hc::ZTable tin2 = empty_table(), tbd2 = empty_table();
    double bytes_in2 = 0.0, bytes_bd2 = 0.0;
    if (two) {
        til2 = vk ? vk2_tiling_for(dtype, nx, arrays, 4) : heat2_tiling_for(dtype, nx, u, un);
        if (mode == HC_HEAT_SPLIT) {
            // the first and last two planes of a slab are its Boundary planes
            for (int q = 0; q < parts; ++q) {
                int a, b;
                slab(nz, parts, q, &a, &b);
                if (b - a + 1 >= 5)
                    push_range(tin2, a + 2, b - 2,
                               vk ? vk2_zrun(dtype, til2) : heat2_zrun(dtype, til2, nx, ny));
            }
            for (int q = 0; q < parts; ++q) {
                int a, b;
                slab(nz, parts, q, &a, &b);
                if (b - a + 1 >= 5) {
                    push_range(tbd2, a, a + 1, 2);
                    push_range(tbd2, b - 1, b, 2);
                } else {
                    push_range(tbd2, a, b, b - a + 1);
                }
            }
        } else {
            push_range(tin2, 1, nz - 2, vk ? vk2_zrun(dtype, til2) : heat2_zrun(dtype, til2, nx, ny));
        }
        // The Boundary kernel of the constant-coefficient split form sweeps
        // its planes with 64 x 4 tiles of one-node lanes (256 threads, at most
        // 64 VGPRs, 13 KB of LDS): such a block fits on a CU beside a block of
        // the Interior kernel, so the Boundary kernel runs in what the
        // Interior blocks leave free instead of holding whole CUs of its own
        // while the two kernels share the chip.
        if (!vk) til2b = {1, 1, 4, 16, 2, 8};
        else til2b = til2;
        if (hc::heat_tile_blocks(nx, ny, til2, tin2) > 2147483647LL ||
            hc::heat_tile_blocks(nx, ny, til2b, tbd2) > 2147483647LL)
            return fail(HC_EINVAL, "grid too large for this tile shape");
        bytes_in2 = fields * tile_algo_bytes(tin2, nx, ny, nz, eb, 2);
        bytes_bd2 = fields * tile_algo_bytes(tbd2, nx, ny, nz, eb, 2);
    }
    const hc::KernelKind k2_fused = vk ? hc::K_VK2_FUSED : hc::K_HEAT2_FUSED;
    const hc::KernelKind k2_int = vk ? hc::K_VK2_INTERIOR : hc::K_HEAT2_INTERIOR;
    const hc::KernelKind k2_bd = vk ? hc::K_VK2_BOUNDARY : hc::K_HEAT2_BOUNDARY;
    auto tile2_launch = [&](hc::KernelKind kind, const hc::ZTable &zt, const void *a, void *b,
                            hipStream_t st) {
        const hc::HeatTiling &t = kind == k2_bd ? til2b : til2;
        return vk ? hc::launch_heat_vk2_tile(dtype, kind, a, kap, rhs, b, nx, ny, nz, r, zt, t, st)
                  : hc::launch_heat2_tile(dtype, kind, a, b, nx, ny, nz, r, zt, t, st);
    };

    HC_TRY(hc::launch_copy_faces((int)eb, u, un, nx, ny, nz, s), "copy_faces launch");
    const bool split = (mode == HC_HEAT_SPLIT) && (tbd.n > 0 || tbd2.n > 0);
    if (split) {
        HC_TRY(hipEventRecord(d->ev_main, s), "hipEventRecord");
        HC_TRY(hipStreamWaitEvent(aux, d->ev_main, 0), "hipStreamWaitEvent");
    }
    void *a = u, *b = un;
    for (int st = 0; st < steps;) {
        if (two && steps - st >= 2) {
            if (mode == HC_HEAT_FUSED) {
                Timed tm(k2_fused, s, bytes_in2);
                HC_TRY(tile2_launch(k2_fused, tin2, a, b, s), "heat2_fused launch");
                tm.done();
            } else {
                {
                    Timed tm(k2_bd, aux, bytes_bd2);
                    HC_TRY(tile2_launch(k2_bd, tbd2, a, b, aux), "heat2_boundary launch");
                    tm.done();
                }
                if (tin2.n > 0) {
                    Timed tm(k2_int, s, bytes_in2);
                    HC_TRY(tile2_launch(k2_int, tin2, a, b, s), "heat2_interior launch");
                    tm.done();
                }
                HC_TRY(hipEventRecord(d->ev_main, s), "hipEventRecord");
                HC_TRY(hipEventRecord(d->ev_aux, aux), "hipEventRecord");
                HC_TRY(hipStreamWaitEvent(s, d->ev_aux, 0), "hipStreamWaitEvent");
                HC_TRY(hipStreamWaitEvent(aux, d->ev_main, 0), "hipStreamWaitEvent");
            }
            std::swap(a, b);
            st += 2;
            continue;
        }
        if (mode == HC_HEAT_PLAIN) {
            Timed tm(k_plain, s, plain_bytes);
            HC_TRY(vk ? hc::launch_heat_vk_plain(dtype, a, kap, rhs, b, nx, ny, nz, r, s)
                      : hc::launch_heat_plain(dtype, a, b, nx, ny, nz, r, seed, step0 + st, s),
                   "heat_plain launch");
            tm.done();
        } else if (mode == HC_HEAT_FUSED) {
            Timed tm(k_fused, s, bytes_in);
            HC_TRY(tile_launch(k_fused, tin, a, b, step0 + st, s), "heat_fused launch");
            tm.done();
        } else {
            // the short Boundary kernel goes first, so it is long done when
            // the next step's Interior kernel waits for it
            {
                Timed tm(k_bd, aux, bytes_bd);
                HC_TRY(tile_launch(k_bd, tbd, a, b, step0 + st, aux), "heat_boundary launch");
                tm.done();
            }
            if (tin.n > 0) {
                Timed tm(k_int, s, bytes_in);
                HC_TRY(tile_launch(k_int, tin, a, b, step0 + st, s), "heat_interior launch");
                tm.done();
            }
            // join: the next step needs both halves of this one, in both streams
            HC_TRY(hipEventRecord(d->ev_main, s), "hipEventRecord");
            HC_TRY(hipEventRecord(d->ev_aux, aux), "hipEventRecord");
            HC_TRY(hipStreamWaitEvent(s, d->ev_aux, 0), "hipStreamWaitEvent");
            HC_TRY(hipStreamWaitEvent(aux, d->ev_main, 0), "hipStreamWaitEvent");
        }
        std::swap(a, b);
        ++st;
    }
    if (a != u)
        HC_TRY(hipMemcpyAsync(u, a, (size_t)nx * ny * nz * eb, hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    return HC_OK;
}

// Iterative refinement with a binary32 inner CG: see cg_solve_ir.
int cg_run_ir(const double *b, double *x, int nx, int ny, int nz, double tol, int maxit,
              double inner_tol, void *work, hipStream_t s, int *iters_out, int *outer_out,
              double *relres_out) {
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc) return rc;
    const hc::CGWorkF32 w = hc::cg_ir_work_carve(work, nx, ny, nz);
    const hc::CGTiling t64 = cg_tiling_for(nx, b, x, x);
    const hc::CGTiling t32 = cg_ir_tiling_for(nx, w.r, w.p[0], w.p[1], w.d);
    hc::CGScalars *h = d->host_sc;
    const double n = (double)nx * ny * nz;
    constexpr int kMaxOuter = 64;
    constexpr double kFloor = 0.5;
    *iters_out = 0;
    *outer_out = 0;
    *relres_out = 0.0;

    auto read_scalars = [&]() -> int {
        HC_TRY(hipMemcpyAsync(h, w.sc, sizeof(hc::CGScalars), hipMemcpyDeviceToHost, s),
               "hipMemcpyAsync");
        HC_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        return HC_OK;
    };
    {
        const size_t plane_bytes = (size_t)nx * ny * sizeof(float);
        float *vecs[3] = {w.r, w.p[0], w.p[1]};
        for (float *v : vecs) {
            HC_TRY(hipMemsetAsync(v - (size_t)nx * ny, 0, plane_bytes, s), "hipMemsetAsync");
            HC_TRY(hipMemsetAsync(v + (size_t)nz * nx * ny, 0, plane_bytes, s), "hipMemsetAsync");
        }
    }
    HC_TRY(hc::launch_cg_init(w.sc, tol, inner_tol, kFloor, s), "cg_init launch");
    double rprev = INFINITY;
    int outer = 0;
    int status = HC_ENOTCONV;
    for (;;) {
        {
            Timed tm(hc::K_IR_RESIDUAL, s, 20.0 * n);
            HC_TRY(hc::launch_cg_ir_residual(b, x, w, nx, ny, nz, t64, d->sink, s),
                   "cg_ir_residual launch");
            tm.done();
        }
        if ((rc = read_scalars())) return rc;
        if (h->state == -7) {
            status = fail(HC_ENONFINITE, "non-finite residual after %d outer steps", outer);
            break;
        }
        if (h->bnorm2 == 0.0) {
            HC_TRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s), "hipMemsetAsync");
            HC_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
            *iters_out = h->iter;
            *outer_out = outer;
            return HC_OK;
        }
        const double rnorm = std::sqrt(h->rtrue2);
        if (h->state == 1) {
            status = HC_OK;
            break;
        }
        if (h->iter >= maxit || outer >= kMaxOuter || rnorm >= rprev) break;  // not converged
        rprev = rnorm;
        HC_TRY(hipMemsetAsync(w.d, 0, (size_t)n * sizeof(float), s), "hipMemsetAsync");
        // d takes its steps two at a time (x in cg_run four): iterations
        // start, start+2, ... leave d alone and the next one applies both
        const int start = h->iter;
        int cur = 0, first = 1;
        while (h->state == 0 && h->iter < maxit) {
            const int batch = std::min(16, maxit - h->iter);
            const int k0 = h->iter;
            for (int q = 0; q < batch; ++q) {
                {
                    Timed tm(hc::K_CG32_DIRECTION, s, (first ? 8.0 : 12.0) * n);
                    HC_TRY(hc::launch_cg_direction_f32(w, cur, first, k0 + q, nx, ny, nz, t32,
                                                       d->sink, s),
                           "cg_direction (binary32) launch");
                    tm.done();
                }
                {
                    const int xstep = ((k0 + q - start) & 1) ? 1 : 0;
                    Timed tm(xstep ? hc::K_CG32_UPDATE_X : hc::K_CG32_UPDATE, s,
                             (xstep ? 24.0 : 12.0) * n);
                    HC_TRY(hc::launch_cg_update_f32(w, cur, k0 + q, xstep, nx, ny, nz, t32,
                                                    d->sink, s),
                           "cg_update (binary32) launch");
                    tm.done();
                }
                cur ^= 1;
                first = 0;
            }
            HC_TRY(hc::launch_cg_settle_f32(w, k0 + batch, nx, ny, nz, t32, s),
                   "cg_settle (binary32) launch");
            if ((rc = read_scalars())) return rc;
        }
        ++outer;
        if ((h->iter - start) & 1) {
            // the last completed inner iteration's step on d is still waiting;
            // its direction vector is p[((j - start) & 1) ^ 1]
            const int j = h->iter - 1;
            HC_TRY(hc::launch_cg_xstep_f32(w.d, w.p[((j - start) & 1) ^ 1], w.sc, j,
                                           (long long)n, s),
                   "cg_xstep (binary32) launch");
        }
        if (h->state == -7) {
            status = fail(HC_ENONFINITE, "non-finite inner scalar at iteration %d", h->iter);
            break;
        }
        if (h->state == -6 && h->iter == start) {
            status = fail(HC_EBREAKDOWN, "p.Ap = %g <= 0 at the start of an inner solve", h->pap);
            break;
        }
        {
            Timed tm(hc::K_IR_UPDATE, s, 20.0 * n);
            HC_TRY(hc::launch_ir_axpy(x, w.d, (long long)n, s), "ir_axpy launch");
            tm.done();
        }
    }
    *iters_out = h->iter;
    *outer_out = outer;
    *relres_out = h->bnorm2 > 0.0 ? std::sqrt(h->rtrue2) / std::sqrt(h->bnorm2) : 0.0;
    return status;
}

int validate_heat(const void *u, const void *un, int nx, int ny, int nz, double r, int steps,
                  int dtype, int mode, int parts, size_t *bytes) {
    if (!u || !un) return fail(HC_EINVAL, "u and u_new must be non-NULL");
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    int rc = check_dims(nx, ny, nz, 3, (size_t)hc::dtype_bytes(dtype), bytes);
    if (rc) return rc;
    if (!std::isfinite(r) || r < 0.0 || r > 1.0 / 6.0)
        return fail(HC_EUNSTABLE, "r = %g is outside [0, 1/6]", r);
    if (steps < 0) return fail(HC_EINVAL, "steps = %d < 0", steps);
    if (mode != HC_HEAT_SPLIT && mode != HC_HEAT_FUSED && mode != HC_HEAT_PLAIN)
        return fail(HC_EINVAL, "mode %d unknown", mode);
    const int max_parts = std::min(32, nz - 2);
    if (parts < 1 || parts > max_parts)
        return fail(HC_EINVAL, "parts = %d outside [1, %d]", parts, max_parts);
    if (parts != 1 && mode != HC_HEAT_SPLIT) return fail(HC_EINVAL, "parts > 1 needs the split mode");
    if (mode == HC_HEAT_PLAIN && (nz - 2 > 65535 || ny - 2 > 4 * 65535))
        return fail(HC_EINVAL, "plain mode supports at most 65537 planes");
    if (overlaps(u, *bytes, un, *bytes)) return fail(HC_EALIAS, "u and u_new overlap");
    return HC_OK;
}

// The CG driver.  `sink` (kSinkDoubles doubles of device memory) takes the
// stores of lanes outside the box; `h` (host memory) receives the device
// scalars at every poll; `timing` allows the kernel timing of hc_prof_*.
int cg_run(const double *b, double *x, int nx, int ny, int nz, double tol, int maxit, void *work,
           hipStream_t s, double *sink, hc::CGScalars *h, bool timing, int *iters_out,
           double *relres_out) {
    int rc = HC_OK;
    const hc::CGWork w = hc::cg_work_carve(work, nx, ny, nz);
    const hc::CGTiling til = cg_tiling_for(nx, b, x, w.r);
    const double n = (double)nx * ny * nz;

    auto read_scalars = [&]() -> int {
        HC_TRY(hipMemcpyAsync(h, w.sc, sizeof(hc::CGScalars), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        HC_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        return HC_OK;
    };
    auto residual = [&](int store_r) -> int {
        Timed tm(hc::K_CG_RESIDUAL, s, (store_r ? 24.0 : 16.0) * n, 1, timing);
        HC_TRY(hc::launch_cg_residual(b, x, w, nx, ny, nz, store_r, til, sink, s),
               "cg_residual launch");
        tm.done();
        return HC_OK;
    };

    // the zero planes around r and the four direction vectors
    {
        const size_t plane_bytes = (size_t)nx * ny * sizeof(double);
        double *vecs[5] = {w.r, w.p[0], w.p[1], w.p[2], w.p[3]};
        for (double *v : vecs) {
            HC_TRY(hipMemsetAsync(v - (size_t)nx * ny, 0, plane_bytes, s), "hipMemsetAsync");
            HC_TRY(hipMemsetAsync(v + (size_t)nz * nx * ny, 0, plane_bytes, s), "hipMemsetAsync");
        }
    }
    HC_TRY(hc::launch_cg_init(w.sc, tol, 0.0, 0.0, s), "cg_init launch");
    if ((rc = residual(1))) return rc;
    if ((rc = read_scalars())) return rc;
    if (h->bnorm2 == 0.0) {
        HC_TRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s), "hipMemsetAsync");
        HC_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        *iters_out = 0;
        *relres_out = 0.0;
        return HC_OK;
    }

    // x takes its steps four at a time (see launch_cg_update): after a
    // (re)start at iteration j0 the update of iteration j applies the steps
    // of j-3 .. j when j - j0 is 3 mod 4 and leaves x alone otherwise;
    // steps still waiting when the iteration stops are applied by xsettle,
    // in order, before x is used.  The direction vector of iteration j is
    // p[j & 3].
    const int kBatch = 16;
    int first = 1, restarts = 0;
    int j0 = 0, xdone = 0;
    bool true_done = false;
    auto xsettle = [&]() -> int {
        const int waiting = (h->iter - j0) & 3;
        if (waiting && xdone != h->iter) {
            for (int j = h->iter - waiting; j < h->iter; ++j)
                HC_TRY(hc::launch_cg_xstep(x, w.p[j & 3], w.sc, j, (long long)nx * ny * nz, s),
                       "cg_xstep launch");
            xdone = h->iter;
        }
        return HC_OK;
    };
    for (;;) {
        if (h->state < 0) break;
        if (h->state == 1) {
            if ((rc = xsettle())) return rc;
            if ((rc = residual(0))) return rc;
            if ((rc = read_scalars())) return rc;
            true_done = true;
            if (std::sqrt(h->rtrue2) <= h->thresh || h->iter >= maxit || restarts >= 3) break;
            // residual gap: restart from the current x
            ++restarts;
            true_done = false;
            first = 1;
            j0 = h->iter;
            if ((rc = residual(1))) return rc;
            if ((rc = read_scalars())) return rc;
            continue;
        }
        if (h->iter >= maxit) break;
        const int batch = std::min(kBatch, maxit - h->iter);
        const int k0 = h->iter;
        for (int q = 0; q < batch; ++q) {
            {
                Timed tm(hc::K_CG_DIRECTION, s, (first ? 16.0 : 24.0) * n, 1, timing);
                HC_TRY(hc::launch_cg_direction(w, first, k0 + q, nx, ny, nz, til, sink, s),
                       "cg_direction launch");
                tm.done();
            }
            {
                const int xsteps = ((k0 + q - j0) & 3) == 3 ? 4 : 0;
                Timed tm(xsteps ? hc::K_CG_UPDATE_X : hc::K_CG_UPDATE, s,
                         (xsteps ? 64.0 : 24.0) * n, 1, timing);
                HC_TRY(hc::launch_cg_update(x, w, k0 + q, xsteps, nx, ny, nz, til, sink, s),
                       "cg_update launch");
                tm.done();
            }
            first = 0;
        }
        HC_TRY(hc::launch_cg_settle(w, k0 + batch, nx, ny, nz, til, s), "cg_settle launch");
        if ((rc = read_scalars())) return rc;
    }
    if ((rc = xsettle())) return rc;
    if (!true_done) {
        if ((rc = residual(0))) return rc;
        if ((rc = read_scalars())) return rc;
    }
    *iters_out = h->iter;
    *relres_out = std::sqrt(h->rtrue2) / std::sqrt(h->bnorm2);
    if (h->state == -6) return fail(HC_EBREAKDOWN, "p.Ap = %g <= 0 at iteration %d", h->pap, h->iter);
    if (h->state == -7) return fail(HC_ENONFINITE, "non-finite scalar at iteration %d", h->iter);
    if (h->state == 1 && std::sqrt(h->rtrue2) <= h->thresh) return HC_OK;
    return HC_ENOTCONV;
}


// ---- batched heat ------------------------------------------------------------
// Default batch shapes per precision: 16-byte lanes, each problem with the
// width class that fits its rows, work-list entries of 64 planes; blocks of
// 256 threads for binary32 (the fastest shape for the uneven FP32
// configuration at two steps per pass), 512 otherwise.  The autotuner
// measures all the built ones.
const hc::BatchTiling kBatchDefault[3] = {{2, 512, 16, 2, 8, -1}, {4, 256, 16, 2, 8, -1},
                                          {8, 512, 16, 2, 8, -1}};
constexpr int kBatchDefaultDepth = 64;

}  // namespace

struct hc_batch {
    int device = 0;
    int dtype = 0;
    int count = 0;
    std::vector<int> dims;          // nx, ny, nz per problem
    std::vector<double> r;
    std::vector<long long> offset;  // elements
    std::vector<int> pitch;         // elements between rows
    long long total = 0;            // elements
    double step_bytes = 0.0;        // algorithmic bytes of one step of all problems
    hc::BatchTiling tiling{};
    int grid = 0;                   // persistent blocks (0: one per entry)
    int item_depth = kBatchDefaultDepth;  // planes per work-list entry (0: whole column)
    std::vector<hc::BatchProblem> probs;  // host copy of the problem table
    hc::BatchProblem *d_probs = nullptr;
    hc::BatchItem *d_items = nullptr;
    int nitems = 0, items_cap = 0;
    int cls_first[5] = {}, cls_count[5] = {};  // each width class's slice of the list
    bool items_ok = false;
    hipStream_t gstream = nullptr;  // capture and launch stream of the graph
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the width classes of a two-step pass run side by side on these
    // streams (forked from and joined to the step's stream by events)
    hipStream_t cstream[4] = {};
    hipEvent_t ev_fork = nullptr, ev_join[4] = {};
    hipGraphExec_t gexec = nullptr;
    const void *g_u = nullptr;
    const void *g_un = nullptr;
    int g_steps = -1, g_grid = -1, g_depth = -1;
    long long g_key = 0;
    struct Cand {
        hc::BatchTiling t;
        int grid, depth;
    };
    std::vector<Cand> tune_cand;
    std::vector<double> tune_ms;
};

namespace {

long long batch_shape_key(const hc::BatchTiling &t) {
    return (((((t.vec * 2048LL + t.threads) * 8 + t.pf) * 128 + t.zdepth) * 65 + t.xcd) * 8 +
            (t.cls + 1));
}

// Width class of a problem with nx columns and ny - 2 updated rows, for
// blocks of `threads`: among the valid classes whose tile covers a whole
// row (a row split over x-tiles is read in short segments that straddle
// cache lines), the one whose tiles cover the fewest nodes (the fewest idle
// threads), the wider one on a tie; the widest valid class when no tile
// covers a row.
int batch_auto_class(int nx, int ny, int vec, int threads) {
    int best = -1, widest = -1;
    long long best_a = 0;
    for (int c = 0; c <= 4; ++c) {
        if (!hc::batch_class_valid(threads, c)) continue;
        widest = c;
        const long long tx = (long long)vec * (8 << c), by = threads / (8 << c);
        if (tx < nx) continue;
        const long long a = tx * ((ny - 2 + by - 1) / by * by);
        if (best < 0 || a <= best_a) {
            best = c;
            best_a = a;
        }
    }
    return best >= 0 ? best : widest;
}

// Build the work list of the batch's current shape and upload it.
int batch_items(hc_batch *b) {
    if (b->items_ok) return HC_OK;
    const hc::BatchTiling &t = b->tiling;
    // one list per width class, concatenated widest class first: blocks that
    // run at the same time mostly run one class's code (the classes' unrolled
    // bodies do not all fit the instruction cache), and the smallest tiles
    // come last, where they even out the tail
    std::vector<hc::BatchItem> per_class[5];
    for (int p = 0; p < b->count; ++p) {
        const int nx = b->dims[3 * p], ny = b->dims[3 * p + 1], nz = b->dims[3 * p + 2];
        const int cls = t.cls >= 0 ? t.cls : batch_auto_class(nx, ny, t.vec, t.threads);
        if (!hc::batch_class_valid(t.threads, cls))
            return fail(HC_EINVAL, "width class %d does not exist for %d threads", cls, t.threads);
        b->probs[p].cls = cls;
        const int tx = t.vec * (8 << cls), by = t.threads / (8 << cls);
        const int ntx = (nx + tx - 1) / tx, nty = (ny - 2 + by - 1) / by;
        if (ntx > 65535 || nty > 65535) return fail(HC_EINVAL, "problem %d has too many tiles", p);
        // planes 1 .. nz-2 in nzb near-equal runs of at least `depth`
        // planes (the kernel walks a run in unrolled sub-blocks of zdepth)
        const int m = nz - 2;
        const int depth = b->item_depth > 0 ? std::max(b->item_depth, t.zdepth) : m;
        const int nzb = std::max(1, m / depth);
        for (int z = 0; z < nzb; ++z) {
            const int kb = 1 + (int)((long long)z * m / nzb);
            const int ke = (int)((long long)(z + 1) * m / nzb);
            for (int x = 0; x < ntx; ++x)
                for (int y = 0; y < nty; ++y)
                    per_class[cls].push_back({p, (unsigned short)x, (unsigned short)y, kb, ke});
        }
    }
    // longest runs first within a class (a problem's tiles of one run stay
    // together, in y order): the short runs fill the tail of the launch,
    // 3-4% faster than problem order on the uneven FP32 configuration
    for (auto &v : per_class)
        std::stable_sort(v.begin(), v.end(), [](const hc::BatchItem &a, const hc::BatchItem &c) {
            return a.ke - a.kb > c.ke - c.kb;
        });
    std::vector<hc::BatchItem> items;
    for (int c = 4; c >= 0; --c) {
        b->cls_first[c] = (int)items.size();
        b->cls_count[c] = (int)per_class[c].size();
        items.insert(items.end(), per_class[c].begin(), per_class[c].end());
    }
    if (items.size() > (size_t)INT32_MAX) return fail(HC_EINVAL, "work list too long");
    if ((int)items.size() > b->items_cap) {
        if (b->d_items) HC_TRY(hipFree(b->d_items), "hipFree");
        b->d_items = nullptr;
        b->items_cap = 0;
        if (hipMalloc(&b->d_items, items.size() * sizeof(hc::BatchItem)) != hipSuccess) {
            (void)hipGetLastError();
            b->d_items = nullptr;
            return fail(HC_ENOMEM, "batch work list of %zu entries", items.size());
        }
        b->items_cap = (int)items.size();
    }
    HC_TRY(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(hc::BatchItem),
                     hipMemcpyHostToDevice),
           "hipMemcpy (work list)");
    HC_TRY(hipMemcpy(b->d_probs, b->probs.data(), b->probs.size() * sizeof(hc::BatchProblem),
                     hipMemcpyHostToDevice),
           "hipMemcpy (problem table)");
    b->nitems = (int)items.size();
    b->items_ok = true;
    return HC_OK;
}

void batch_drop_graph(hc_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_steps = -1;
}

// Steps per pass the batch takes with its current shape: two when the
// library's setting asks for two and the shape is built for them.
int batch_time_block(const hc_batch *b) {
    return current_time_block() == 2 && hc::batch2_tiling_supported(b->dtype, b->tiling) ? 2 : 1;
}

// The step loop on stream s: the passes alternate the buffers (a last odd
// step takes one single-step launch), then a copy leaves the result in u
// when it ended in u_new.
int batch_enqueue(hc_batch *b, void *u, void *un, int steps, hipStream_t s) {
    const int eb = hc::dtype_bytes(b->dtype);
    const int tb = batch_time_block(b);
    void *a = u, *c = un;
    int st = 0;
    if (tb == 2 && steps >= 2) {
        // One launch per width class present and pass.  A class touches
        // only its own problems, so each class runs its passes as a chain on
        // a stream of its own: the chains run side by side from the first
        // pass to the last and join once, so no pass waits for the slowest
        // class of the pass before.
        const int passes = steps / 2;
        int used[5], nc = 0;
        for (int k = 4; k >= 0; --k)
            if (b->cls_count[k] > 0) used[nc++] = k;
        if (nc > 1) {
            HC_TRY(hipEventRecord(b->ev_fork, s), "hipEventRecord");
            for (int i = 1; i < nc; ++i)
                HC_TRY(hipStreamWaitEvent(b->cstream[i - 1], b->ev_fork, 0), "hipStreamWaitEvent");
        }
        for (int p = 0; p < passes; ++p) {
            for (int i = 0; i < nc; ++i) {
                const int k = used[i];
                hipStream_t ks = i == 0 ? s : b->cstream[i - 1];
                HC_TRY(hc::launch_heat_batch2(b->dtype, k, a, c, b->d_probs,
                                              b->d_items + b->cls_first[k], b->cls_count[k],
                                              b->grid, b->tiling, ks),
                       "heat_batch2 launch");
            }
            std::swap(a, c);
        }
        for (int i = 1; i < nc; ++i) {
            HC_TRY(hipEventRecord(b->ev_join[i - 1], b->cstream[i - 1]), "hipEventRecord");
            HC_TRY(hipStreamWaitEvent(s, b->ev_join[i - 1], 0), "hipStreamWaitEvent");
        }
        st = 2 * passes;
    }
    for (; st < steps; ++st) {
        HC_TRY(hc::launch_heat_batch(b->dtype, a, c, b->d_probs, b->d_items, b->nitems, b->grid,
                                     b->tiling, s),
               "heat_batch launch");
        std::swap(a, c);
    }
    if (a != u)
        HC_TRY(hipMemcpyAsync(u, a, (size_t)b->total * eb, hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    return HC_OK;
}

int batch_check_device(const hc_batch *b) {
    int dev = 0;
    HC_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != b->device)
        return fail(HC_EINVAL, "batch was created on device %d, current device is %d", b->device, dev);
    return HC_OK;
}

int batch_run(hc_batch *b, void *u, void *un, int steps, int use_graph, hipStream_t s) {
    int rc = batch_items(b);
    if (rc) return rc;
    const int eb = hc::dtype_bytes(b->dtype);
    // u_new takes u's Dirichlet layer (a copy of the whole buffer)
    HC_TRY(hipMemcpyAsync(un, u, (size_t)b->total * eb, hipMemcpyDeviceToDevice, s),
           "hipMemcpyAsync");
    // algorithmic bytes: a pass moves one step's bytes
    const int tb = batch_time_block(b);
    const double run_bytes = b->step_bytes * (steps / tb + steps % tb);
    if (!use_graph) {
        Timed tm(hc::K_BATCH, s, run_bytes, steps);
        if ((rc = batch_enqueue(b, u, un, steps, s))) return rc;
        tm.done();
        return HC_OK;
    }
    const long long key = batch_shape_key(b->tiling) * 2 + (tb - 1);
    if (!b->gexec || b->g_u != u || b->g_un != un || b->g_steps != steps || b->g_key != key ||
        b->g_grid != b->grid || b->g_depth != b->item_depth) {
        batch_drop_graph(b);
        hipGraph_t graph = nullptr;
        HC_TRY(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
        const int erc = batch_enqueue(b, u, un, steps, b->gstream);
        const hipError_t ce = hipStreamEndCapture(b->gstream, &graph);
        if (erc) {
            if (graph) (void)hipGraphDestroy(graph);
            return erc;
        }
        HC_TRY(ce, "hipStreamEndCapture");
        const hipError_t ie = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HC_TRY(ie, "hipGraphInstantiate");
        b->g_u = u;
        b->g_un = un;
        b->g_steps = steps;
        b->g_key = key;
        b->g_grid = b->grid;
        b->g_depth = b->item_depth;
    }
    // join the caller's stream in and out of the graph's stream
    HC_TRY(hipEventRecord(b->ev_in, s), "hipEventRecord");
    HC_TRY(hipStreamWaitEvent(b->gstream, b->ev_in, 0), "hipStreamWaitEvent");
    {
        Timed tm(hc::K_BATCH, b->gstream, run_bytes, steps);
        HC_TRY(hipGraphLaunch(b->gexec, b->gstream), "hipGraphLaunch");
        tm.done();
    }
    HC_TRY(hipEventRecord(b->ev_out, b->gstream), "hipEventRecord");
    HC_TRY(hipStreamWaitEvent(s, b->ev_out, 0), "hipStreamWaitEvent");
    return HC_OK;
}

int batch_check_buffers(const hc_batch *b, const void *u, const void *un) {
    if (!u || !un) return fail(HC_EINVAL, "u and u_new must be non-NULL");
    const size_t bytes = (size_t)b->total * hc::dtype_bytes(b->dtype);
    if (overlaps(u, bytes, un, bytes)) return fail(HC_EALIAS, "u and u_new overlap");
    int rc = check_device_buffer(u, bytes, "u");
    if (rc) return rc;
    rc = check_device_buffer(un, bytes, "u_new");
    if (rc) return rc;
    const uintptr_t a = reinterpret_cast<uintptr_t>(u) | reinterpret_cast<uintptr_t>(un);
    if (a & 63) return fail(HC_EINVAL, "u and u_new must be 64-byte aligned");
    return HC_OK;
}

}  // namespace

extern "C" {

const char *hc_strerror(int code) {
    switch (code) {
        case HC_OK: return "HC_OK";
        case HC_ENOTCONV: return "HC_ENOTCONV";
        case HC_EINVAL: return "HC_EINVAL";
        case HC_EUNSTABLE: return "HC_EUNSTABLE";
        case HC_EALIAS: return "HC_EALIAS";
        case HC_ENOMEM: return "HC_ENOMEM";
        case HC_EHIP: return "HC_EHIP";
        case HC_EBREAKDOWN: return "HC_EBREAKDOWN";
        case HC_ENONFINITE: return "HC_ENONFINITE";
        default: return "HC_UNKNOWN";
    }
}

const char *hc_last_error_message(void) { return g_msg.c_str(); }

int heat_step_ex(void *u, void *u_new, int nx, int ny, int nz, double r, int steps, int dtype,
                 int mode, int parts, hc_stream_t stream) {
    g_msg.clear();
    size_t bytes = 0;
    int rc = validate_heat(u, u_new, nx, ny, nz, r, steps, dtype, mode, parts, &bytes);
    if (rc) return rc;
    if (steps == 0) return HC_OK;
    if ((rc = check_device_buffer(u, bytes, "u"))) return rc;
    if ((rc = check_device_buffer(u_new, bytes, "u_new"))) return rc;
    return heat_run(dtype, u, u_new, nx, ny, nz, r, steps, mode, parts, 0, 0,
                    reinterpret_cast<hipStream_t>(stream));
}

int heat_step_sr(void *u, void *u_new, int nx, int ny, int nz, double r, int steps,
                 unsigned long long seed, unsigned long long step0, int mode, int parts,
                 hc_stream_t stream) {
    g_msg.clear();
    size_t bytes = 0;
    int rc = validate_heat(u, u_new, nx, ny, nz, r, steps, HC_BF16, mode, parts, &bytes);
    if (rc) return rc;
    if (steps == 0) return HC_OK;
    if ((rc = check_device_buffer(u, bytes, "u"))) return rc;
    if ((rc = check_device_buffer(u_new, bytes, "u_new"))) return rc;
    return heat_run(hc::kDtypeBF16SR, u, u_new, nx, ny, nz, r, steps, mode, parts, seed, step0,
                    reinterpret_cast<hipStream_t>(stream));
}

int heat_vk_step(void *u, void *u_new, const void *kappa, const void *rhs, int nx, int ny,
                 int nz, double beta, int steps, int dtype, int mode, int parts,
                 hc_stream_t stream) {
    g_msg.clear();
    if (!kappa || !rhs) return fail(HC_EINVAL, "kappa and rhs must be non-NULL");
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d: the variable-coefficient step takes HC_F64 or HC_F32",
                    dtype);
    if (!std::isfinite(beta) || beta < 0.0)
        return fail(HC_EUNSTABLE, "beta = %g must be finite and >= 0", beta);
    size_t bytes = 0;
    int rc = validate_heat(u, u_new, nx, ny, nz, 0.0, steps, dtype, mode, parts, &bytes);
    if (rc) return rc;
    if (overlaps(kappa, bytes, u, bytes) || overlaps(kappa, bytes, u_new, bytes) ||
        overlaps(rhs, bytes, u, bytes) || overlaps(rhs, bytes, u_new, bytes))
        return fail(HC_EALIAS, "kappa and rhs must not overlap u or u_new");
    if (steps == 0) return HC_OK;
    if ((rc = check_device_buffer(u, bytes, "u"))) return rc;
    if ((rc = check_device_buffer(u_new, bytes, "u_new"))) return rc;
    if ((rc = check_device_buffer(kappa, bytes, "kappa"))) return rc;
    if ((rc = check_device_buffer(rhs, bytes, "rhs"))) return rc;
    return heat_run(dtype, u, u_new, nx, ny, nz, beta, steps, mode, parts, 0, 0,
                    reinterpret_cast<hipStream_t>(stream), kappa, rhs);
}

int heat_step_streams(void *u, void *u_new, int nx, int ny, int nz, double r, int steps,
                      int dtype, int parts, hc_stream_t s_int, hc_stream_t s_bnd) {
    g_msg.clear();
    size_t bytes = 0;
    int rc = validate_heat(u, u_new, nx, ny, nz, r, steps, dtype, HC_HEAT_SPLIT, parts, &bytes);
    if (rc) return rc;
    if (steps == 0) return HC_OK;
    if ((rc = check_device_buffer(u, bytes, "u"))) return rc;
    if ((rc = check_device_buffer(u_new, bytes, "u_new"))) return rc;
    hipStream_t const si = reinterpret_cast<hipStream_t>(s_int);
    hipStream_t const sb = reinterpret_cast<hipStream_t>(s_bnd);
    if (sb != si) {
        int dev = 0, sdev = 0;
        HC_TRY(hipGetDevice(&dev), "hipGetDevice");
        HC_TRY(hipStreamGetDevice(sb, &sdev), "hipStreamGetDevice (s_bnd)");
        if (sdev != dev)
            return fail(HC_EINVAL, "s_bnd belongs to device %d, the current device is %d", sdev,
                        dev);
    }
    return heat_run(dtype, u, u_new, nx, ny, nz, r, steps, HC_HEAT_SPLIT, parts, 0, 0, si,
                    nullptr, nullptr, true, sb);
}

int heat_step(double *u, double *u_new, int nx, int ny, int nz, double r, int steps) {
    int rc = heat_step_ex(u, u_new, nx, ny, nz, r, steps, HC_F64, HC_HEAT_SPLIT, 1, nullptr);
    if (rc != HC_OK || steps == 0) return rc;
    HC_TRY(hipStreamSynchronize(nullptr), "heat_step (kernel execution)");
    return HC_OK;
}

size_t cg_workspace_bytes(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    if ((double)nx * ny * nz * 8.0 > 9.0e15) return 0;
    return hc::cg_work_bytes(nx, ny, nz);
}

// The caller's workspace (checked), or the library's cached one (grown to
// `need` bytes on demand).  Called with d->cg_mu held.
int cg_workspace(DevState *d, const double *b, const double *x, size_t bytes, size_t need,
                 void **work) {
    int rc = HC_OK;
    if (*work) {
        // the carve puts the scalar block and the partial sums (read and
        // written with 8-byte accesses, some of them atomic) at multiples of
        // 256 bytes from the base
        if (reinterpret_cast<uintptr_t>(*work) % 256 != 0)
            return fail(HC_EINVAL, "work must be 256-byte aligned");
        if ((rc = check_device_buffer(*work, need, "work"))) return rc;
        if (overlaps(*work, need, b, bytes) || overlaps(*work, need, x, bytes))
            return fail(HC_EALIAS, "workspace overlaps b or x");
        return HC_OK;
    }
    std::lock_guard<std::mutex> g(g_dev_mu);
    if (d->cg_work_size < need) {
        if (d->cg_work) {
            HC_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
            HC_TRY(hipFree(d->cg_work), "hipFree");
            d->cg_work = nullptr;
            d->cg_work_size = 0;
        }
        if (hipMalloc(&d->cg_work, need) != hipSuccess) {
            (void)hipGetLastError();
            d->cg_work = nullptr;
            return fail(HC_ENOMEM, "CG workspace of %zu bytes", need);
        }
        d->cg_work_size = need;
    }
    *work = d->cg_work;
    return HC_OK;
}

int cg_solve_ex(const double *b, double *x, int nx, int ny, int nz, double tol, int maxit,
                void *work, size_t work_bytes, hc_stream_t stream, int *iters,
                double *true_relres) {
    g_msg.clear();
    g_cg_iters = 0;
    g_cg_relres = 0.0;
    if (!b || !x) return fail(HC_EINVAL, "b and x must be non-NULL");
    size_t bytes = 0;
    int rc = check_dims(nx, ny, nz, 1, 8, &bytes);
    if (rc) return rc;
    if (!std::isfinite(tol) || tol <= 0.0) return fail(HC_EINVAL, "tol = %g must be > 0", tol);
    if (maxit < 0) return fail(HC_EINVAL, "maxit = %d < 0", maxit);
    if (overlaps(b, bytes, x, bytes)) return fail(HC_EALIAS, "b and x overlap");
    const size_t need = hc::cg_work_bytes(nx, ny, nz);
    if (hc::cg_blocks(nx, ny, nz, {1, 1, 4, 8, 0}) > 2147483647LL)
        return fail(HC_EINVAL, "grid too large");
    if (work && work_bytes < need)
        return fail(HC_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, need);
    if ((rc = check_device_buffer(b, bytes, "b"))) return rc;
    if ((rc = check_device_buffer(x, bytes, "x"))) return rc;
    DevState *d = nullptr;
    if ((rc = device_state(&d))) return rc;
    std::lock_guard<std::mutex> solve_lock(d->cg_mu);
    if ((rc = cg_workspace(d, b, x, bytes, need, &work))) return rc;
    int it = 0;
    double rel = 0.0;
    rc = cg_run(b, x, nx, ny, nz, tol, maxit, work, reinterpret_cast<hipStream_t>(stream),
                d->sink, d->host_sc, true, &it, &rel);
    g_cg_iters = it;
    g_cg_relres = rel;
    if (iters) *iters = it;
    if (true_relres) *true_relres = rel;
    return rc;
}

int cg_solve(const double *b, double *x, int n, double tol, int maxit) {
    return cg_solve_ex(b, x, n, n, n, tol, maxit, nullptr, 0, nullptr, nullptr, nullptr);
}

int cg_solve_noalloc(const double *b, double *x, int nx, int ny, int nz, double tol, int maxit,
                     hc_stream_t stream, int *iters, double *true_relres) {
    g_msg.clear();
    if (iters) *iters = 0;
    if (true_relres) *true_relres = 0.0;
    if (!b || !x) return fail(HC_EINVAL, "b and x must be non-NULL");
    size_t bytes = 0;
    int rc = check_dims(nx, ny, nz, 1, 8, &bytes);
    if (rc) return rc;
    if (!std::isfinite(tol) || tol <= 0.0) return fail(HC_EINVAL, "tol = %g must be > 0", tol);
    if (maxit < 0) return fail(HC_EINVAL, "maxit = %d < 0", maxit);
    if (overlaps(b, bytes, x, bytes)) return fail(HC_EALIAS, "b and x overlap");
    const size_t need = kNoallocSinkBytes + hc::cg_work_bytes(nx, ny, nz);
    if (need > (size_t)HC_CG_NOALLOC_BYTES)
        return fail(HC_EINVAL, "a %d x %d x %d box needs %zu bytes of workspace; the fixed one "
                    "holds %zu", nx, ny, nz, need, (size_t)HC_CG_NOALLOC_BYTES);
    if ((rc = check_device_buffer(b, bytes, "b"))) return rc;
    if ((rc = check_device_buffer(x, bytes, "x"))) return rc;
    ScratchSlot *sl = nullptr;
    if ((rc = scratch_slot(&sl))) return rc;
    std::lock_guard<std::mutex> solve_lock(sl->mu);
    double *sink = reinterpret_cast<double *>(sl->ptr);
    void *work = sl->ptr + kNoallocSinkBytes;
    int it = 0;
    double rel = 0.0;
    rc = cg_run(b, x, nx, ny, nz, tol, maxit, work, reinterpret_cast<hipStream_t>(stream), sink,
                &sl->host, false, &it, &rel);
    if (iters) *iters = it;
    if (true_relres) *true_relres = rel;
    return rc;
}

void hc_cg_last_info(int *iters, double *true_relres) {
    if (iters) *iters = g_cg_iters;
    if (true_relres) *true_relres = g_cg_relres;
}

int cg_solve_ir(const double *b, double *x, int nx, int ny, int nz, double tol, int maxit,
                double inner_tol, void *work, size_t work_bytes, hc_stream_t stream, int *iters,
                int *outer, double *true_relres) {
    g_msg.clear();
    if (iters) *iters = 0;
    if (outer) *outer = 0;
    if (true_relres) *true_relres = 0.0;
    if (!b || !x) return fail(HC_EINVAL, "b and x must be non-NULL");
    size_t bytes = 0;
    int rc = check_dims(nx, ny, nz, 1, 8, &bytes);
    if (rc) return rc;
    if (!std::isfinite(tol) || tol <= 0.0) return fail(HC_EINVAL, "tol = %g must be > 0", tol);
    if (maxit < 0) return fail(HC_EINVAL, "maxit = %d < 0", maxit);
    if (!std::isfinite(inner_tol) || inner_tol >= 1.0)
        return fail(HC_EINVAL, "inner_tol = %g must be < 1", inner_tol);
    if (inner_tol <= 0.0) inner_tol = 1e-5;
    if (overlaps(b, bytes, x, bytes)) return fail(HC_EALIAS, "b and x overlap");
    const size_t need = hc::cg_ir_work_bytes(nx, ny, nz);
    if (hc::cg_blocks(nx, ny, nz, {1, 1, 4, 8, 0}) > 2147483647LL)
        return fail(HC_EINVAL, "grid too large");
    if (work && work_bytes < need)
        return fail(HC_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, need);
    if ((rc = check_device_buffer(b, bytes, "b"))) return rc;
    if ((rc = check_device_buffer(x, bytes, "x"))) return rc;
    DevState *d = nullptr;
    if ((rc = device_state(&d))) return rc;
    std::lock_guard<std::mutex> solve_lock(d->cg_mu);
    if ((rc = cg_workspace(d, b, x, bytes, need, &work))) return rc;
    int it = 0, out = 0;
    double rel = 0.0;
    rc = cg_run_ir(b, x, nx, ny, nz, tol, maxit, inner_tol, work,
                   reinterpret_cast<hipStream_t>(stream), &it, &out, &rel);
    if (iters) *iters = it;
    if (outer) *outer = out;
    if (true_relres) *true_relres = rel;
    return rc;
}

size_t cg_ir_workspace_bytes(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    return hc::cg_ir_work_bytes(nx, ny, nz);
}

int hc_lap7_apply_f32(const float *x, float *y, int nx, int ny, int nz, hc_stream_t stream) {
    g_msg.clear();
    if (!x || !y) return fail(HC_EINVAL, "x and y must be non-NULL");
    size_t bytes = 0;
    int rc = check_dims(nx, ny, nz, 1, 4, &bytes);
    if (rc) return rc;
    if (overlaps(x, bytes, y, bytes)) return fail(HC_EALIAS, "x and y overlap");
    if (hc::cg_blocks(nx, ny, nz, {1, 1, 4, 8, 0}) > 2147483647LL)
        return fail(HC_EINVAL, "grid too large");
    if ((rc = check_device_buffer(x, bytes, "x"))) return rc;
    if ((rc = check_device_buffer(y, bytes, "y"))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DevState *d = nullptr;
    if ((rc = device_state(&d))) return rc;
    const hc::CGTiling til = cg_ir_tiling_for(nx, x, y, x, y);
    Timed tm(hc::K_LAP7, s, 8.0 * nx * ny * nz);
    HC_TRY(hc::launch_lap7_f32(x, y, nx, ny, nz, til, d->sink, s), "lap7 (binary32) launch");
    tm.done();
    return HC_OK;
}

int hc_lap7_apply(const double *x, double *y, int nx, int ny, int nz, hc_stream_t stream) {
    g_msg.clear();
    if (!x || !y) return fail(HC_EINVAL, "x and y must be non-NULL");
    size_t bytes = 0;
    int rc = check_dims(nx, ny, nz, 1, 8, &bytes);
    if (rc) return rc;
    if (overlaps(x, bytes, y, bytes)) return fail(HC_EALIAS, "x and y overlap");
    if (hc::cg_blocks(nx, ny, nz, {1, 1, 4, 8, 0}) > 2147483647LL)
        return fail(HC_EINVAL, "grid too large");
    if ((rc = check_device_buffer(x, bytes, "x"))) return rc;
    if ((rc = check_device_buffer(y, bytes, "y"))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DevState *d = nullptr;
    if ((rc = device_state(&d))) return rc;
    const hc::CGTiling til = cg_tiling_for(nx, x, y, x);
    Timed tm(hc::K_LAP7, s, 16.0 * nx * ny * nz);
    HC_TRY(hc::launch_lap7_f64(x, y, nx, ny, nz, til, d->sink, s), "lap7 launch");
    tm.done();
    return HC_OK;
}

int hc_copy_probe(const void *src, void *dst, size_t bytes, hc_stream_t stream) {
    g_msg.clear();
    if (!src || !dst) return fail(HC_EINVAL, "src and dst must be non-NULL");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(HC_EINVAL, "bytes and both pointers must be multiples of 16");
    if (overlaps(src, bytes, dst, bytes)) return fail(HC_EALIAS, "src and dst overlap");
    if (bytes == 0) return HC_OK;
    int rc;
    if ((rc = check_device_buffer(src, bytes, "src"))) return rc;
    if ((rc = check_device_buffer(dst, bytes, "dst"))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Timed tm(hc::K_COPY, s, 2.0 * (double)bytes);
    HC_TRY(hc::launch_copy_probe(src, dst, bytes, s), "copy_probe launch");
    tm.done();
    return HC_OK;
}

int hc_heat_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf, int xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const hc::HeatTiling t = {vec, wx, by, zdepth, pf, xcd};
    if (vec == 0 && wx == 0 && by == 0 && zdepth == 0 && pf == 0 && xcd == 0) {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        g_tiling[dtype] = t;  // automatic choice
        return HC_OK;
    }
    if (!hc::heat_tiling_supported(dtype, t))
        return fail(HC_EINVAL,
                    "tile shape (vec %d, wx %d, by %d, zdepth %d, pf %d) is not built for dtype %d",
                    vec, wx, by, zdepth, pf, dtype);
    if (xcd < 0 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [0, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_tiling[dtype] = t;
    return HC_OK;
}

int hc_heat_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const hc::HeatTiling t = current_tiling(dtype);
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_tiling_for(int dtype, int nx, const void *u, const void *u_new, int *vec, int *wx,
                       int *by, int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16 && dtype != HC_BF16_SR)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    if (nx < 3) return fail(HC_EINVAL, "nx = %d < 3", nx);
    const hc::HeatTiling t = heat_tiling_for(dtype, nx, u, u_new);
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_set_time_block(int steps_per_pass) {
    g_msg.clear();
    if (steps_per_pass != 1 && steps_per_pass != 2)
        return fail(HC_EINVAL, "steps per pass %d: 1 or 2", steps_per_pass);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_time_block = steps_per_pass;
    return HC_OK;
}

int hc_heat_get_time_block(void) { return current_time_block(); }

int hc_heat2_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf, int xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const hc::HeatTiling t = {vec, wx, by, zdepth, pf, xcd};
    if (vec == 0 && wx == 0 && by == 0 && zdepth == 0 && pf == 0 && xcd == 0) {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        g_tiling2[dtype] = t;
        return HC_OK;
    }
    if (!hc::heat2_tiling_supported(dtype, t))
        return fail(HC_EINVAL,
                    "two-step tile shape (vec %d, wx %d, by %d, zdepth %d, pf %d) is not built "
                    "for dtype %d",
                    vec, wx, by, zdepth, pf, dtype);
    if (xcd < -1 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [-1, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_tiling2[dtype] = t;
    return HC_OK;
}

int hc_heat2_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    hc::HeatTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_tiling2[dtype];
    }
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat2_set_zrun(int dtype, int planes) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d has no two-step sweep", dtype);
    if (planes < 0 || planes > (1 << 20)) return fail(HC_EINVAL, "zrun = %d out of range", planes);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_heat2_zrun[dtype] = planes;
    return HC_OK;
}

int hc_heat2_get_zrun(int dtype) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d has no two-step sweep", dtype);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    return g_heat2_zrun[dtype];
}

int hc_heat_vk2_set_zrun(int dtype, int planes) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d has no two-step variable-coefficient sweep", dtype);
    if (planes < 0 || planes > (1 << 20)) return fail(HC_EINVAL, "zrun = %d out of range", planes);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_vk2_zrun[dtype] = planes;
    return HC_OK;
}

int hc_heat_vk2_get_zrun(int dtype) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d has no two-step variable-coefficient sweep", dtype);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    return g_vk2_zrun[dtype];
}

int hc_heat2_tiling_for(int dtype, int nx, const void *u, const void *u_new, int *vec, int *wx,
                        int *by, int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    if (nx < 3) return fail(HC_EINVAL, "nx = %d < 3", nx);
    const hc::HeatTiling t = heat2_tiling_for(dtype, nx, u, u_new);
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_vk2_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf, int xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const hc::HeatTiling t = {vec, wx, by, zdepth, pf, xcd};
    if (vec == 0 && wx == 0 && by == 0 && zdepth == 0 && pf == 0 && xcd == 0) {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        g_vk2_tiling[dtype] = t;
        return HC_OK;
    }
    if (!hc::heat_vk2_tiling_supported(dtype, t))
        return fail(HC_EINVAL,
                    "two-step variable-coefficient tile shape (vec %d, wx %d, by %d, zdepth %d, "
                    "pf %d) is not built for dtype %d",
                    vec, wx, by, zdepth, pf, dtype);
    if (xcd < -1 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [-1, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_vk2_tiling[dtype] = t;
    return HC_OK;
}

int hc_heat_vk2_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth, int *pf,
                           int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    hc::HeatTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_vk2_tiling[dtype];
    }
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_vk2_tiling_for(int dtype, int nx, const void *u, const void *u_new,
                           const void *kappa, const void *rhs, int *vec, int *wx, int *by,
                           int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    if (nx < 3) return fail(HC_EINVAL, "nx = %d < 3", nx);
    const void *arrays[4] = {u, u_new, kappa, rhs};
    const hc::HeatTiling t = vk2_tiling_for(dtype, nx, arrays, 4);
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_vk_set_tiling(int dtype, int vec, int wx, int by, int zdepth, int pf, int xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const hc::HeatTiling t = {vec, wx, by, zdepth, pf, xcd};
    if (vec == 0 && wx == 0 && by == 0 && zdepth == 0 && pf == 0 && xcd == 0) {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        g_vk_tiling[dtype] = t;
        return HC_OK;
    }
    if (!hc::heat_vk_tiling_supported(dtype, t))
        return fail(HC_EINVAL,
                    "variable-coefficient tile shape (vec %d, wx %d, by %d, zdepth %d, pf %d) is "
                    "not built for dtype %d",
                    vec, wx, by, zdepth, pf, dtype);
    if (xcd < 0 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [0, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_vk_tiling[dtype] = t;
    return HC_OK;
}

int hc_heat_vk_get_tiling(int dtype, int *vec, int *wx, int *by, int *zdepth, int *pf, int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    hc::HeatTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_vk_tiling[dtype];
    }
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_heat_vk_tiling_for(int dtype, int nx, const void *u, const void *u_new, const void *kappa,
                          const void *rhs, int *vec, int *wx, int *by, int *zdepth, int *pf,
                          int *xcd) {
    g_msg.clear();
    if (dtype != HC_F64 && dtype != HC_F32)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    if (nx < 3) return fail(HC_EINVAL, "nx = %d < 3", nx);
    const void *arrays[4] = {u, u_new, kappa, rhs};
    const hc::HeatTiling t = vk_tiling_for(dtype, nx, arrays, 4);
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (pf) *pf = t.pf;
    if (xcd) *xcd = t.xcd;
    return HC_OK;
}

int hc_cg_ir_set_tiling(int vec, int wx, int by, int zdepth, int xcd) {
    g_msg.clear();
    const hc::CGTiling t = {vec, wx, by, zdepth, xcd};
    if (!hc::cg_tiling_supported_f32(t))
        return fail(HC_EINVAL, "binary32 CG tile shape (vec %d, wx %d, by %d, zdepth %d) is not built",
                    vec, wx, by, zdepth);
    if (xcd < 0 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [0, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_cg_ir_tiling = t;
    return HC_OK;
}

void hc_cg_ir_get_tiling(int *vec, int *wx, int *by, int *zdepth, int *xcd) {
    hc::CGTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_cg_ir_tiling;
    }
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (xcd) *xcd = t.xcd;
}

int hc_cg_set_tiling(int vec, int wx, int by, int zdepth, int xcd) {
    g_msg.clear();
    const hc::CGTiling t = {vec, wx, by, zdepth, xcd};
    if (!hc::cg_tiling_supported(t))
        return fail(HC_EINVAL, "CG tile shape (vec %d, wx %d, by %d, zdepth %d) is not built", vec,
                    wx, by, zdepth);
    if (xcd < 0 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [0, 64]", xcd);
    std::lock_guard<std::mutex> g(g_tiling_mu);
    g_cg_tiling = t;
    return HC_OK;
}

void hc_cg_get_tiling(int *vec, int *wx, int *by, int *zdepth, int *xcd) {
    hc::CGTiling t;
    {
        std::lock_guard<std::mutex> g(g_tiling_mu);
        t = g_cg_tiling;
    }
    if (vec) *vec = t.vec;
    if (wx) *wx = t.wx;
    if (by) *by = t.by;
    if (zdepth) *zdepth = t.zdepth;
    if (xcd) *xcd = t.xcd;
}

int hc_prof_enable(int every) {
    g_msg.clear();
    if (every < 0) return fail(HC_EINVAL, "every = %d < 0", every);
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (const Pending &p : g_pending) {
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
    for (int k = 0; k < hc::K_COUNT; ++k) {
        g_prof_ms[k] = 0.0;
        g_prof_n[k] = 0;
        g_prof_bytes[k] = 0.0;
        g_prof_seen[k] = 0;
    }
    g_prof_on = (every != 0);
    g_prof_every = every > 0 ? every : 1;
    return HC_OK;
}

int hc_prof_read(int kind, double *total_ms, long long *launches, double *algo_bytes) {
    g_msg.clear();
    if (kind < 0 || kind >= hc::K_COUNT) return fail(HC_EINVAL, "kernel kind %d unknown", kind);
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (const Pending &p : g_pending) {
        HC_TRY(hipEventSynchronize(p.b), "hipEventSynchronize");
        float ms = 0.f;
        HC_TRY(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime");
        g_prof_ms[p.kind] += ms;
        g_prof_n[p.kind] += p.launches;
        g_prof_bytes[p.kind] += p.bytes;
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
    if (total_ms) *total_ms = g_prof_ms[kind];
    if (launches) *launches = g_prof_n[kind];
    if (algo_bytes) *algo_bytes = g_prof_bytes[kind];
    return HC_OK;
}

// ---- batched heat -----------------------------------------------------------------

int hc_batch_create(int count, const int *dims, const double *r, int dtype, hc_batch **out) {
    g_msg.clear();
    if (!out) return fail(HC_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (count < 1 || count > (1 << 20)) return fail(HC_EINVAL, "count = %d outside [1, 2^20]", count);
    if (!dims || !r) return fail(HC_EINVAL, "dims and r must be non-NULL");
    if (dtype != HC_F64 && dtype != HC_F32 && dtype != HC_BF16)
        return fail(HC_EINVAL, "dtype %d is not supported", dtype);
    const int eb = hc::dtype_bytes(dtype);
    const long long align = 64 / eb;  // elements per 64 bytes
    const int row_align = 16 / eb;    // elements per 16 bytes
    for (int p = 0; p < count; ++p) {
        const int nx = dims[3 * p], ny = dims[3 * p + 1], nz = dims[3 * p + 2];
        if (nx < 3 || ny < 3 || nz < 3 || nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20))
            return fail(HC_EINVAL, "problem %d: edges (%d, %d, %d) must each be in [3, 2^20]", p,
                        nx, ny, nz);
        if (!std::isfinite(r[p]) || r[p] < 0.0 || r[p] > 1.0 / 6.0)
            return fail(HC_EUNSTABLE, "problem %d: r = %g is outside [0, 1/6]", p, r[p]);
    }
    hc_batch *b = new (std::nothrow) hc_batch;
    if (!b) return fail(HC_ENOMEM, "batch descriptor");
    b->dtype = dtype;
    b->count = count;
    b->dims.assign(dims, dims + 3 * (size_t)count);
    b->r.assign(r, r + count);
    b->offset.resize(count);
    b->pitch.resize(count);
    long long off = 0;
    double bytes = 0.0;
    std::vector<hc::BatchProblem> probs(count);
    for (int p = 0; p < count; ++p) {
        const int nx = dims[3 * p], ny = dims[3 * p + 1], nz = dims[3 * p + 2];
        const int pitch = (nx + row_align - 1) / row_align * row_align;
        b->offset[p] = off;
        b->pitch[p] = pitch;
        probs[p] = {off, nx, ny, nz, pitch, 0, 0, r[p]};
        const long long n = (long long)pitch * ny * nz;
        off += (n + align - 1) / align * align;
        bytes += (double)eb * ((double)nx * ny * nz + (double)(nx - 2) * (ny - 2) * (nz - 2));
    }
    b->total = off;
    b->step_bytes = bytes;
    b->tiling = kBatchDefault[dtype];
    b->probs = probs;
    int rc = HC_OK;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipMalloc(&b->d_probs, sizeof(hc::BatchProblem) * count) != hipSuccess ||
        hipMemcpy(b->d_probs, probs.data(), sizeof(hc::BatchProblem) * count,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        rc = fail(HC_EHIP, "batch set-up: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < 4 && !rc; ++i) {
        if (hipStreamCreateWithFlags(&b->cstream[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming) != hipSuccess) {
            const hipError_t e = hipGetLastError();
            rc = fail(HC_EHIP, "batch set-up: %s", hipGetErrorString(e));
        }
    }
    if (rc) {
        hc_batch_destroy(b);
        return rc;
    }
    *out = b;
    return HC_OK;
}

void hc_batch_destroy(hc_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_drop_graph(b);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (int i = 0; i < 4; ++i) {
        if (b->ev_join[i]) (void)hipEventDestroy(b->ev_join[i]);
        if (b->cstream[i]) (void)hipStreamDestroy(b->cstream[i]);
    }
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    delete b;
}

int hc_batch_layout(const hc_batch *b, long long *offsets, int *pitches, long long *total_elems,
                    double *step_bytes) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    if (offsets) std::copy(b->offset.begin(), b->offset.end(), offsets);
    if (pitches) std::copy(b->pitch.begin(), b->pitch.end(), pitches);
    if (total_elems) *total_elems = b->total;
    if (step_bytes) *step_bytes = b->step_bytes;
    return HC_OK;
}

int hc_batch_set_tiling(hc_batch *b, int vec, int threads, int zdepth, int pf, int xcd,
                        int width_class, int grid, int item_depth) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    const hc::BatchTiling t = {vec, threads, zdepth, pf, xcd, width_class};
    if (!hc::batch_tiling_supported(b->dtype, t))
        return fail(HC_EINVAL,
                    "batch block shape (vec %d, threads %d, zdepth %d, pf %d) is not built", vec,
                    threads, zdepth, pf);
    if (xcd < 0 || xcd > 64) return fail(HC_EINVAL, "xcd = %d outside [0, 64]", xcd);
    if (width_class != -1 && !hc::batch_class_valid(threads, width_class))
        return fail(HC_EINVAL, "width class %d does not exist for %d threads", width_class,
                    threads);
    if (grid < 0) return fail(HC_EINVAL, "grid = %d < 0", grid);
    if (item_depth < 0) return fail(HC_EINVAL, "item_depth = %d < 0", item_depth);
    if (batch_shape_key(t) != batch_shape_key(b->tiling) || item_depth != b->item_depth)
        b->items_ok = false;
    b->tiling = t;
    b->grid = grid;
    b->item_depth = item_depth;
    return HC_OK;
}

int hc_batch_get_tiling(const hc_batch *b, int *vec, int *threads, int *zdepth, int *pf,
                        int *xcd, int *width_class, int *grid, int *item_depth) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    if (vec) *vec = b->tiling.vec;
    if (threads) *threads = b->tiling.threads;
    if (zdepth) *zdepth = b->tiling.zdepth;
    if (pf) *pf = b->tiling.pf;
    if (xcd) *xcd = b->tiling.xcd;
    if (width_class) *width_class = b->tiling.cls;
    if (grid) *grid = b->grid;
    if (item_depth) *item_depth = b->item_depth;
    return HC_OK;
}

int hc_batch_classes(hc_batch *b, int *classes) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    int rc = batch_check_device(b);
    if (rc) return rc;
    if ((rc = batch_items(b))) return rc;
    if (classes)
        for (int p = 0; p < b->count; ++p) classes[p] = b->probs[p].cls;
    return HC_OK;
}

int hc_batch_step(hc_batch *b, void *u, void *u_new, int steps, int use_graph,
                  hc_stream_t stream) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    if (steps < 0) return fail(HC_EINVAL, "steps = %d < 0", steps);
    int rc = batch_check_device(b);
    if (rc) return rc;
    if ((rc = batch_check_buffers(b, u, u_new))) return rc;
    if (steps == 0) return HC_OK;
    return batch_run(b, u, u_new, steps, use_graph, reinterpret_cast<hipStream_t>(stream));
}

int hc_batch_autotune(hc_batch *b, const void *u, int trial_steps, hc_stream_t stream,
                      double *best_ms) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    if (trial_steps < 1) return fail(HC_EINVAL, "trial_steps = %d < 1", trial_steps);
    int rc = batch_check_device(b);
    if (rc) return rc;
    const size_t bytes = (size_t)b->total * hc::dtype_bytes(b->dtype);
    if ((rc = check_device_buffer(u, bytes, "u"))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // candidates: every built shape, with whole-column, one-z-block, 32-
    // and 64-plane entries, one block per entry or a persistent grid
    int ncu = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
            ncu = prop.multiProcessorCount;
    }
    std::vector<hc::BatchTiling> shapes;
    hc::batch_shapes(b->dtype, shapes);
    std::vector<hc_batch::Cand> cand;
    for (hc::BatchTiling t : shapes) {
        // each problem's best-fitting width, with every order, run length
        // and grid; then every width for all problems, in one setting
        for (int x : {0, 8})
            for (int dep : {0, t.zdepth, 32, 64}) {
                if (dep == 32 && t.zdepth == 32) continue;  // listed as the z-block
                for (int g : {0, 2 * ncu}) {
                    t.xcd = x;
                    t.cls = -1;
                    cand.push_back({t, g, dep});
                }
            }
        for (int c = 0; c <= 4; ++c)
            if (hc::batch_class_valid(t.threads, c)) {
                t.xcd = 8;
                t.cls = c;
                cand.push_back({t, 0, 64});
            }
    }
    void *sa = nullptr, *sb = nullptr;
    if (hipMalloc(&sa, bytes) != hipSuccess || hipMalloc(&sb, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (sa) (void)hipFree(sa);
        return fail(HC_ENOMEM, "autotuner scratch of 2 x %zu bytes", bytes);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const hc::BatchTiling keep_t = b->tiling;
    const int keep_g = b->grid, keep_d = b->item_depth;
    double best = INFINITY;
    size_t best_i = 0;
    b->tune_cand = cand;
    b->tune_ms.assign(cand.size(), INFINITY);
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipFree(sa);
        (void)hipFree(sb);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(HC_EHIP, "hipEventCreate");
    }
    const int tsteps = 2 * ((trial_steps + 1) / 2);
    if (hipMemcpyAsync(sa, u, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sb, sa, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        cleanup();
        return fail(HC_EHIP, "hipMemcpyAsync");
    }
    // milliseconds per step of candidate i over `n` steps (an even count)
    auto trial = [&](size_t i, int n, double *out) -> int {
        b->tiling = cand[i].t;
        b->grid = cand[i].grid;
        b->item_depth = cand[i].depth;
        b->items_ok = false;
        int r = batch_items(b);
        // every trial runs an even number of steps from the states in sa
        // (sa and sb are each other's scratch): warm-up pair, timed steps
        if (!r) r = batch_enqueue(b, sa, sb, 2, s);
        if (!r && hipEventRecord(e0, s) != hipSuccess) r = fail(HC_EHIP, "hipEventRecord");
        if (!r) r = batch_enqueue(b, sa, sb, n, s);
        if (!r && hipEventRecord(e1, s) != hipSuccess) r = fail(HC_EHIP, "hipEventRecord");
        float ms = 0.f;
        if (!r && (hipEventSynchronize(e1) != hipSuccess ||
                   hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = fail(HC_EHIP, "timing a candidate");
        *out = ms / n;
        return r;
    };
    auto bail = [&](int r) {
        b->tiling = keep_t;
        b->grid = keep_g;
        b->item_depth = keep_d;
        b->items_ok = false;
        cleanup();
        return r;
    };
    for (size_t i = 0; i < cand.size(); ++i)
        if ((rc = trial(i, tsteps, &b->tune_ms[i]))) return bail(rc);
    // the four fastest again, each over twice the steps, twice in turn: the
    // best of those (differences of a percent or two decide between them)
    std::vector<size_t> order(cand.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t c) { return b->tune_ms[a] < b->tune_ms[c]; });
    order.resize(std::min<size_t>(4, order.size()));
    for (size_t i : order) {
        if (b->tune_ms[i] < best) {
            best = b->tune_ms[i];
            best_i = i;
        }
    }
    if (order.size() > 1) {
        std::vector<double> again(order.size(), INFINITY);
        for (int rep = 0; rep < 2; ++rep)
            for (size_t q = 0; q < order.size(); ++q) {
                double ms = 0.0;
                if ((rc = trial(order[q], 2 * tsteps, &ms))) return bail(rc);
                again[q] = std::min(again[q], ms);
            }
        size_t bq = 0;
        for (size_t q = 1; q < order.size(); ++q)
            if (again[q] < again[bq]) bq = q;
        best_i = order[bq];
        best = again[bq];
    }
    cleanup();
    b->tiling = cand[best_i].t;
    b->grid = cand[best_i].grid;
    b->item_depth = cand[best_i].depth;
    b->items_ok = false;
    batch_drop_graph(b);
    if (best_ms) *best_ms = best;
    return batch_items(b);
}

int hc_batch_steps_per_pass(const hc_batch *b) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch is NULL");
    return batch_time_block(b);
}

int hc_batch_tune_result(const hc_batch *b, int index, int *shape8, double *ms_per_step) {
    g_msg.clear();
    if (!b) return fail(HC_EINVAL, "batch must be non-NULL");
    if (index < 0) return (int)b->tune_cand.size();
    if (index >= (int)b->tune_cand.size()) return fail(HC_EINVAL, "index %d out of range", index);
    const hc::BatchTiling &t = b->tune_cand[index].t;
    if (shape8) {
        const int v[8] = {t.vec, t.threads, t.zdepth, t.pf, t.xcd, t.cls,
                          b->tune_cand[index].grid, b->tune_cand[index].depth};
        std::copy(v, v + 8, shape8);
    }
    if (ms_per_step) *ms_per_step = b->tune_ms[index];
    return HC_OK;
}

}  // extern "C"
