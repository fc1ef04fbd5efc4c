// api.cpp -- the C ABI declared in include/utfgpu.h.
//
// Argument checks, the frame/head split of the input address, per
// (device, stream) workspaces (control block, tile status words, result
// slots), kernel launches and the synchronous result read-back.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "../../include/utfgpu.h"
#include "device_common.hpp"

// The launchers of every compiled tile geometry (C++ linkage; one build of
// the kernel files per entry of geometries.def).
#define UTF_GEOMETRY(NS, WAVES, ROWS)                                                                             \
    namespace utfgpu {                                                                                            \
    namespace NS {                                                                                                \
    u64 build_tile_bytes();                                                                                       \
    u64 utf8_tiles_for(long long head, long long n);                                                              \
    u64 utf16_tiles_for(long long head, long long m);                                                             \
    hipError_t launch_utf8_tiles(bool convert, const uint8_t *frame, long long head, long long n, uint16_t *out,  \
                                 u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, int schedule,           \
                                 hipStream_t stream);                                                             \
    hipError_t launch_utf16_tiles(bool convert, const uint8_t *frame, long long head, long long m, uint8_t *out,  \
                                  u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, int schedule,          \
                                  hipStream_t stream);                                                            \
    hipError_t launch_utf16_length(const uint8_t *frame, long long head, long long n, u64 *partials, Ctrl *ctrl,  \
                                   u64 *result, hipStream_t stream);                                              \
    hipError_t launch_utf8_length(const uint8_t *frame, long long head, long long m, u64 *partials, Ctrl *ctrl,   \
                                  u64 *result, hipStream_t stream);                                               \
    hipError_t launch_set_result(DevResult *r, int32_t status, u64 count, hipStream_t stream);                    \
    hipError_t launch_set_u64(u64 *r, u64 v, hipStream_t stream);                                                 \
    hipError_t launch_utf8_batch(const uint8_t *frame, long long head, long long n, const int64_t *offsets,       \
                                 u64 k, uint16_t *out, u64 out_cap, int64_t *out_offsets, DevResult *results,     \
                                 u64 *status, Ctrl *ctrl, uint32_t *starts, uint16_t *blockoff, u64 *tilepre,     \
                                 u64 *serr, uint32_t *bad, uint32_t *wavestr, int schedule, hipStream_t stream);  \
    hipError_t launch_utf16_batch(const uint8_t *frame, long long head, long long m, const int64_t *offsets,      \
                                  u64 k, uint8_t *out, u64 out_cap, int64_t *out_offsets, DevResult *results,     \
                                  u64 *status, Ctrl *ctrl, uint32_t *starts, uint16_t *blockoff, u64 *tilepre,    \
                                  u64 *serr, uint32_t *bad, uint32_t *wavestr, int schedule,                      \
                                  hipStream_t stream);                                                            \
    }                                                                                                             \
    }
#include "geometries.def"
#undef UTF_GEOMETRY

using namespace utfgpu;

namespace {

// One compiled geometry: its shape and its launchers.
struct Geometry {
    const char *name;
    uint32_t waves, rows;
    u64 (*tile_bytes)();
    u64 (*utf8_tiles_for)(long long, long long);
    u64 (*utf16_tiles_for)(long long, long long);
    decltype(&utfgpu::g8x4::launch_utf8_tiles) utf8_tiles;
    decltype(&utfgpu::g8x4::launch_utf16_tiles) utf16_tiles;
    decltype(&utfgpu::g8x4::launch_utf8_batch) utf8_batch;
    decltype(&utfgpu::g8x4::launch_utf16_batch) utf16_batch;
};

#define UTF_GEOMETRY(NS, WAVES, ROWS)                                                                         \
    {#NS, WAVES, ROWS, &utfgpu::NS::build_tile_bytes, &utfgpu::NS::utf8_tiles_for,                             \
     &utfgpu::NS::utf16_tiles_for, &utfgpu::NS::launch_utf8_tiles, &utfgpu::NS::launch_utf16_tiles,           \
     &utfgpu::NS::launch_utf8_batch, &utfgpu::NS::launch_utf16_batch},
const Geometry kGeometries[] = {
#include "geometries.def"
};
#undef UTF_GEOMETRY
constexpr int kNumGeometries = (int)(sizeof(kGeometries) / sizeof(kGeometries[0]));

// The length reductions and result writers do not depend on the tile
// geometry: the 8 x 4 build's serve every call.
namespace base = utfgpu::g8x4;

// Tuning table: per operation and input size class, 1 + the geometry index
// (0: the shipped default below).  Written by utfgpu_set_geometry, read once
// per call; UTFGPU_GEOMETRY (an index) overrides it for the whole process.
std::atomic<uint8_t> g_table[UTF_OP_COUNT][UTF_SIZE_CLASSES];

int geometry_index(const char *name) {
    for (int i = 0; i < kNumGeometries; ++i)
        if (std::strcmp(kGeometries[i].name, name) == 0) return i;
    return 0;
}

// Shipped defaults, from timing every build on MI355X over the five script
// mixes (ASCII, Latin, Cyrillic, CJK, emoji) and mixed-script text.
// Conversions of up to 4 MiB (size class <= 22) run fastest in 8 KiB tiles:
// 32 KiB tiles leave most CUs idle there.  Batched UTF-8 calls keep 8 KiB
// tiles up to 16 MiB.  Larger batched UTF-16 calls use the 4 x 4 build:
// serving runs them on several streams beside other look-back kernels, and
// (the likely reading of the measurements) an 8-wave workgroup, which needs
// registers for two 80-VGPR waves on every SIMD of one CU, often finds no
// room on its XCD while later tiles of its own or another kernel wait for
// it, so the wait lasts until the helping path steps in; a 4-wave
// workgroup needs one wave per SIMD and fits beside the others (measured: twice the throughput
// of 8 x 4 for a burst of requests on four streams, against up to 5 % less
// for one call alone).  Everything else: the 8 x 4 build (16 KiB tiles win
// on non-ASCII text and lose more on ASCII).
int shipped_geometry(int op, int c) {
    static const int g4x2 = geometry_index("g4x2");
    static const int g4x4 = geometry_index("g4x4");
    switch (op) {
        case UTF_OP_CONVERT_UTF8:
        case UTF_OP_CONVERT_UTF16LE: return c <= 22 ? g4x2 : 0;
        case UTF_OP_BATCH_UTF16LE: return c <= 22 ? g4x2 : g4x4;
        case UTF_OP_BATCH_UTF8: return c <= 24 ? g4x2 : 0;
        default: return 0;
    }
}

int table_geometry(int op, int c) {
    const int g = (int)g_table[op][c].load(std::memory_order_relaxed) - 1;
    return g >= 0 && g < kNumGeometries ? g : shipped_geometry(op, c);
}

int forced_geometry() {
    static const int g = [] {
        const char *e = std::getenv("UTFGPU_GEOMETRY");
        if (!e || !*e) return -1;
        const int v = std::atoi(e);
        return v >= 0 && v < kNumGeometries ? v : -1;
    }();
    return g;
}

int size_class(u64 bytes) {
    const int c = bytes <= 1 ? 0 : 64 - __builtin_clzll(bytes - 1);   // ceil(log2(bytes))
    return c < UTF_SIZE_CLASSES ? c : UTF_SIZE_CLASSES - 1;
}

const Geometry &geometry_for(int op, u64 bytes) {
    const int f = forced_geometry();
    if (f >= 0) return kGeometries[f];
    return kGeometries[table_geometry(op, size_class(bytes))];
}

// Scan schedule table, laid out like the geometry table (1 + the schedule,
// 0: the shipped default).  The schedule is the order in which the tile
// kernels' workgroups take their tiles: UTF_SCHEDULE_BLOCK, tile = workgroup
// index; UTF_SCHEDULE_TICKET, the next index of a per-call counter taken when
// the workgroup starts.  Both compute the same results.  The shipped default
// is block order everywhere: on MI355X tickets made a 100 000-string batched
// call 9 % (UTF-8) and 16 % (UTF-16) slower, a burst of serving requests on
// four streams 10 % slower with the shipped geometries, and single-buffer
// ASCII conversions 6.5 % slower (the counter's round trip precedes each
// tile's first load).  Ticket order is for concurrency the geometry table
// does not cover: it keeps a burst with 8 x 4 batched UTF-16 calls at
// 790 GB/s where block order halves it.
constexpr int kNumSchedules = UTF_SCHEDULE_COUNT;
static_assert(kScheduleTicket == UTF_SCHEDULE_TICKET, "schedule index");
std::atomic<uint8_t> g_sched[UTF_OP_COUNT][UTF_SIZE_CLASSES];

int table_schedule(int op, int c) {
    const int v = (int)g_sched[op][c].load(std::memory_order_relaxed) - 1;
    return v >= 0 && v < kNumSchedules ? v : UTF_SCHEDULE_BLOCK;
}

int forced_schedule() {
    static const int v = [] {
        const char *e = std::getenv("UTFGPU_SCHEDULE");
        if (!e || !*e) return -1;
        const int x = std::atoi(e);
        return x >= 0 && x < kNumSchedules ? x : -1;
    }();
    return v;
}

int schedule_for(int op, u64 bytes) {
    const int f = forced_schedule();
    return f >= 0 ? f : table_schedule(op, size_class(bytes));
}

}  // namespace

int utfgpu::lookback_spin_limit() {
    static const int limit = [] {
        const char *e = std::getenv("UTFGPU_LOOKBACK_SPINS");
        if (!e || !*e) return kDefaultSpinLimit;
        const int v = std::atoi(e);
        return v < 0 ? 0 : (v > 1 << 20 ? 1 << 20 : v);
    }();
    return limit;
}

u64 utfgpu::epoch_period() {
    static const u64 period = [] {
        constexpr u64 kMax = kEpochMask + 1;
        const char *e = std::getenv("UTFGPU_EPOCH_PERIOD");
        if (!e || !*e) return kMax;
        const long long v = std::atoll(e);
        return v < 2 ? (u64)2 : ((u64)v > kMax ? kMax : (u64)v);
    }();
    return period;
}

static_assert(sizeof(utf_result) == sizeof(DevResult), "result layout");
static_assert(offsetof(utf_result, count) == offsetof(DevResult, count), "result layout");

namespace {

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    Ctrl *ctrl = nullptr;        // device
    DevResult *hres = nullptr;   // pinned host result slot of the synchronous calls
    u64 *hlen = nullptr;         // pinned host length slot
    DevResult *dres = nullptr;   // the same slots as device addresses
    u64 *dlen = nullptr;
    u64 *partials = nullptr;     // device partial sums of the length reductions
    u64 *status = nullptr;       // device tile status words
    u64 status_cap = 0;
    // batched calls
    uint32_t *starts = nullptr;     // string-start bitmap (all zero between calls)
    u64 starts_words = 0;
    uint16_t *blockoff = nullptr;   // per 64-byte block: output offset inside its tile
    u64 blockoff_cap = 0;
    u64 *tilepre = nullptr;         // per tile: output offset
    u64 tilepre_cap = 0;
    u64 *serr = nullptr;            // per string: first error (~0 between calls)
    u64 serr_cap = 0;
    uint32_t *wavestr = nullptr;    // per wave span: owner string of its first position
    u64 wavestr_cap = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

void free_ws(Workspace *w) {
    if (w->ctrl) (void)hipFree(w->ctrl);
    if (w->status) (void)hipFree(w->status);
    if (w->partials) (void)hipFree(w->partials);
    if (w->hres) (void)hipHostFree(w->hres);
    if (w->hlen) (void)hipHostFree(w->hlen);
    if (w->starts) (void)hipFree(w->starts);
    if (w->blockoff) (void)hipFree(w->blockoff);
    if (w->tilepre) (void)hipFree(w->tilepre);
    if (w->serr) (void)hipFree(w->serr);
    if (w->wavestr) (void)hipFree(w->wavestr);
    delete w;
}

hipError_t make_ws(int dev, hipStream_t s, Workspace **out) {
    Workspace *w = new Workspace();
    w->device = dev;
    w->stream = s;
    hipError_t e;
    if ((e = hipMalloc(&w->ctrl, sizeof(Ctrl))) != hipSuccess) goto fail;
    if ((e = hipMalloc(&w->partials, kMaxPartials * sizeof(u64))) != hipSuccess) goto fail;
    // the synchronous calls' results: pinned, coherent host memory that the
    // finalize kernel writes directly (no device-to-host copy per call)
    if ((e = hipHostMalloc(&w->hres, sizeof(DevResult), hipHostMallocCoherent)) != hipSuccess) goto fail;
    if ((e = hipHostMalloc(&w->hlen, sizeof(u64), hipHostMallocCoherent)) != hipSuccess) goto fail;
    if ((e = hipHostGetDevicePointer((void **)&w->dres, w->hres, 0)) != hipSuccess) goto fail;
    if ((e = hipHostGetDevicePointer((void **)&w->dlen, w->hlen, 0)) != hipSuccess) goto fail;
    if ((e = base::launch_ctrl_init(w->ctrl, nullptr, 0, epoch_period(), s)) != hipSuccess) goto fail;
    *out = w;
    return hipSuccess;
fail:
    free_ws(w);
    return e;
}

// Workspace of (current device, stream) with room for `ntiles` status words.
hipError_t get_ws(hipStream_t s, u64 ntiles, Workspace **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    Workspace *w;
    if (it == g_ws.end()) {
        if ((e = make_ws(dev, s, &w)) != hipSuccess) return e;
        g_ws[key] = w;
    } else {
        w = it->second;
    }
    if (ntiles > w->status_cap) {
        // the old array may still be read by work queued on this stream
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (w->status) (void)hipFree(w->status);
        w->status = nullptr;
        w->status_cap = 0;
        u64 cap = ntiles < 4096 ? 4096 : ntiles + ntiles / 4;
        if ((e = hipMalloc(&w->status, cap * kStatusStride * sizeof(u64))) != hipSuccess) return e;
        // clears the new words and points the control block at them
        if ((e = base::launch_ctrl_init(w->ctrl, w->status, cap, epoch_period(), s)) != hipSuccess) return e;
        w->status_cap = cap;
    }
    *out = w;
    return hipSuccess;
}

// Grow a device array to at least `need` elements (new memory filled with
// byte `fill`); the stream is drained first, since queued work may still
// use the old array.
template <class T>
hipError_t grow(T **p, u64 *cap, u64 need, int fill, hipStream_t s) {
    if (need <= *cap) return hipSuccess;
    hipError_t e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const u64 c = need + need / 4 + 64;
    if ((e = hipMalloc(p, c * sizeof(T))) != hipSuccess) return e;
    if ((e = hipMemsetAsync(*p, fill, c * sizeof(T), s)) != hipSuccess) return e;
    *cap = c;
    return hipSuccess;
}

// Batched-call arrays for `ntiles` tiles of `tile_units` positions in
// `waves` wave spans each and `k` strings (block offsets per 32 positions
// cover both directions).
hipError_t get_batch(Workspace *w, u64 ntiles, u64 tile_units, u64 waves, u64 k, hipStream_t s) {
    hipError_t e;
    const u64 positions = ntiles * tile_units + 128;   // every tile and the chunk past the last
    if ((e = grow(&w->starts, &w->starts_words, positions / 32 + 2, 0, s)) != hipSuccess) return e;
    if ((e = grow(&w->blockoff, &w->blockoff_cap, positions / 32 + 2, 0, s)) != hipSuccess) return e;
    if ((e = grow(&w->tilepre, &w->tilepre_cap, ntiles + 1, 0, s)) != hipSuccess) return e;
    if ((e = grow(&w->serr, &w->serr_cap, k + 1, 0xFF, s)) != hipSuccess) return e;
    if ((e = grow(&w->wavestr, &w->wavestr_cap, ntiles * waves + 2, 0, s)) != hipSuccess) return e;
    return hipSuccess;
}

inline utf_result mk(int32_t st, u64 c) {
    utf_result r;
    r.status = st;
    r.count = c;
    return r;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---- argument checks ----------------------------------------------------
int32_t check8(const uint8_t *in, u64 n) {
    if (n == 0) return UTF_OK;
    if (!in) return UTF_ERR_NULL;
    if (n >= UTF_MAX_UTF8_BYTES) return UTF_ERR_TOO_BIG;
    return UTF_OK;
}

int32_t check16(const uint16_t *in, u64 m) {
    if (m == 0) return UTF_OK;
    if (!in) return UTF_ERR_NULL;
    if (reinterpret_cast<uintptr_t>(in) & 1u) return UTF_ERR_ALIGN;
    if (m >= UTF_MAX_UTF16_WORDS) return UTF_ERR_TOO_BIG;
    return UTF_OK;
}

inline const uint8_t *frame_of(const void *p) {
    return reinterpret_cast<const uint8_t *>(reinterpret_cast<uintptr_t>(p) & ~uintptr_t(15));
}
inline long long head_bytes(const void *p) { return (long long)(reinterpret_cast<uintptr_t>(p) & 15u); }


// ---- enqueue helpers (return a negative status or UTF_OK) ----------------
int32_t enqueue_utf8(bool convert, const uint8_t *in, u64 n, uint16_t *out, u64 out_cap, DevResult *res,
                     hipStream_t s, Workspace **wso) {
    const long long head = head_bytes(in);
    const int op = convert ? UTF_OP_CONVERT_UTF8 : UTF_OP_VALIDATE_UTF8;
    const Geometry &g = geometry_for(op, n);
    const u64 nt = g.utf8_tiles_for(head, (long long)n);
    Workspace *w;
    if (get_ws(s, nt, &w) != hipSuccess) return UTF_ERR_HIP;
    if (!res) res = w->dres;
    if (g.utf8_tiles(convert, frame_of(in), head, (long long)n, out, out_cap, w->status, w->ctrl, res,
                     schedule_for(op, n), s) !=
        hipSuccess)
        return UTF_ERR_HIP;
    *wso = w;
    return UTF_OK;
}

int32_t enqueue_utf16(bool convert, const uint16_t *in, u64 m, uint8_t *out, u64 out_cap, DevResult *res,
                      hipStream_t s, Workspace **wso) {
    const long long head = head_bytes(in) / 2;
    const int op = convert ? UTF_OP_CONVERT_UTF16LE : UTF_OP_VALIDATE_UTF16LE;
    const Geometry &g = geometry_for(op, 2 * m);
    const u64 nt = g.utf16_tiles_for(head, (long long)m);
    Workspace *w;
    if (get_ws(s, nt, &w) != hipSuccess) return UTF_ERR_HIP;
    if (!res) res = w->dres;
    if (g.utf16_tiles(convert, frame_of(in), head, (long long)m, out, out_cap, w->status, w->ctrl, res,
                      schedule_for(op, 2 * m), s) !=
        hipSuccess)
        return UTF_ERR_HIP;
    *wso = w;
    return UTF_OK;
}

// ---- the allocation-free entry point --------------------------------------
// Its workspace is a fixed array of device memory: the control block in
// the first 256 bytes, then one status word per tile, kStatusStride words
// apart.  Each device holds its own copy until the process ends.  In host
// code `scratch` only names the symbol; the device address of each
// device's copy comes from hipGetSymbolAddress and is kept per device.
constexpr u64 kNoAllocTiles = 65536;
constexpr u64 kNoAllocCtrlWords = 32;
static_assert(sizeof(Ctrl) <= kNoAllocCtrlWords * sizeof(u64), "control block fits its slot");
__device__ __align__(256) u64 scratch[kNoAllocCtrlWords + kNoAllocTiles * kStatusStride];

constexpr int kMaxDevices = 64;
struct NoAllocState {
    bool ready = false;
    u64 *ptr = nullptr;   // device address of this device's scratch
};
NoAllocState g_noalloc[kMaxDevices];
std::mutex g_noalloc_mu;

// This device's scratch, set up on the first call made on it: its address,
// then its control block and status words initialised on `s`.
hipError_t noalloc_scratch(hipStream_t s, u64 **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocState &st = g_noalloc[dev];
    if (!st.ready) {
        u64 *ptr = nullptr;
        if ((e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        if ((e = base::launch_ctrl_init(reinterpret_cast<Ctrl *>(ptr), ptr + kNoAllocCtrlWords, kNoAllocTiles,
                                        epoch_period(), s)) != hipSuccess)
            return e;
        st.ptr = ptr;
        st.ready = true;
    }
    *out = st.ptr;
    return hipSuccess;
}

// The result of the call just queued on `s`: its finalize kernel writes it
// straight into the workspace's pinned host slot.
utf_result read_result(Workspace *w, hipStream_t s) {
    if (hipStreamSynchronize(s) != hipSuccess) return mk(UTF_ERR_HIP, 0);
    const volatile DevResult *r = w->hres;
    return mk(r->status, r->count);
}

u64 read_len(Workspace *w, hipStream_t s) {
    if (hipStreamSynchronize(s) != hipSuccess) return ~0ull;
    return *(const volatile u64 *)w->hlen;
}

}  // namespace

extern "C" {

utf_result validate_utf8(const uint8_t *in, uint64_t n, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return mk(c, 0);
    if (n == 0) return mk(UTF_OK, 0);
    Workspace *w;
    hipStream_t s = as_stream(stream);
    if ((c = enqueue_utf8(false, in, n, nullptr, 0, nullptr, s, &w)) != UTF_OK) return mk(c, 0);
    return read_result(w, s);
}

utf_result validate_utf16le(const uint16_t *in, uint64_t m, void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return mk(c, 0);
    if (m == 0) return mk(UTF_OK, 0);
    Workspace *w;
    hipStream_t s = as_stream(stream);
    if ((c = enqueue_utf16(false, in, m, nullptr, 0, nullptr, s, &w)) != UTF_OK) return mk(c, 0);
    return read_result(w, s);
}

utf_result convert_utf8_to_utf16le(const uint8_t *in, uint64_t n, uint16_t *out, uint64_t out_cap,
                                   void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return mk(c, 0);
    if (!out && out_cap > 0) return mk(UTF_ERR_NULL, 0);
    if (reinterpret_cast<uintptr_t>(out) & 1u) return mk(UTF_ERR_ALIGN, 0);
    if (n == 0) return mk(UTF_OK, 0);
    Workspace *w;
    hipStream_t s = as_stream(stream);
    if ((c = enqueue_utf8(true, in, n, out, out_cap, nullptr, s, &w)) != UTF_OK) return mk(c, 0);
    return read_result(w, s);
}

utf_result convert_utf16le_to_utf8(const uint16_t *in, uint64_t m, uint8_t *out, uint64_t out_cap,
                                   void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return mk(c, 0);
    if (!out && out_cap > 0) return mk(UTF_ERR_NULL, 0);
    if (m == 0) return mk(UTF_OK, 0);
    Workspace *w;
    hipStream_t s = as_stream(stream);
    if ((c = enqueue_utf16(true, in, m, out, out_cap, nullptr, s, &w)) != UTF_OK) return mk(c, 0);
    return read_result(w, s);
}

uint64_t utf16_length_from_utf8(const uint8_t *in, uint64_t n, void *stream) {
    if (check8(in, n) != UTF_OK) return ~0ull;
    if (n == 0) return 0;
    hipStream_t s = as_stream(stream);
    Workspace *w;
    if (get_ws(s, 0, &w) != hipSuccess) return ~0ull;
    if (base::launch_utf16_length(frame_of(in), head_bytes(in), (long long)n, w->partials, w->ctrl, w->dlen, s) !=
        hipSuccess)
        return ~0ull;
    return read_len(w, s);
}

uint64_t utf8_length_from_utf16le(const uint16_t *in, uint64_t m, void *stream) {
    if (check16(in, m) != UTF_OK) return ~0ull;
    if (m == 0) return 0;
    hipStream_t s = as_stream(stream);
    Workspace *w;
    if (get_ws(s, 0, &w) != hipSuccess) return ~0ull;
    if (base::launch_utf8_length(frame_of(in), head_bytes(in) / 2, (long long)m, w->partials, w->ctrl, w->dlen, s) !=
        hipSuccess)
        return ~0ull;
    return read_len(w, s);
}

int32_t validate_utf8_async(const uint8_t *in, uint64_t n, utf_result *result, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return c;
    if (!result) return UTF_ERR_NULL;
    hipStream_t s = as_stream(stream);
    DevResult *r = reinterpret_cast<DevResult *>(result);
    if (n == 0) return base::launch_set_result(r, UTF_OK, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    return enqueue_utf8(false, in, n, nullptr, 0, r, s, &w);
}

int32_t validate_utf16le_async(const uint16_t *in, uint64_t m, utf_result *result, void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return c;
    if (!result) return UTF_ERR_NULL;
    hipStream_t s = as_stream(stream);
    DevResult *r = reinterpret_cast<DevResult *>(result);
    if (m == 0) return base::launch_set_result(r, UTF_OK, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    return enqueue_utf16(false, in, m, nullptr, 0, r, s, &w);
}

int32_t convert_utf8_to_utf16le_async(const uint8_t *in, uint64_t n, uint16_t *out, uint64_t out_cap,
                                      utf_result *result, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return c;
    if (!result || (!out && out_cap > 0)) return UTF_ERR_NULL;
    if (reinterpret_cast<uintptr_t>(out) & 1u) return UTF_ERR_ALIGN;
    hipStream_t s = as_stream(stream);
    DevResult *r = reinterpret_cast<DevResult *>(result);
    if (n == 0) return base::launch_set_result(r, UTF_OK, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    return enqueue_utf8(true, in, n, out, out_cap, r, s, &w);
}

int32_t convert_utf16le_to_utf8_async(const uint16_t *in, uint64_t m, uint8_t *out, uint64_t out_cap,
                                      utf_result *result, void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return c;
    if (!result || (!out && out_cap > 0)) return UTF_ERR_NULL;
    hipStream_t s = as_stream(stream);
    DevResult *r = reinterpret_cast<DevResult *>(result);
    if (m == 0) return base::launch_set_result(r, UTF_OK, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    return enqueue_utf16(true, in, m, out, out_cap, r, s, &w);
}

int32_t utf16_length_from_utf8_async(const uint8_t *in, uint64_t n, uint64_t *result, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return c;
    if (!result) return UTF_ERR_NULL;
    hipStream_t s = as_stream(stream);
    if (n == 0) return base::launch_set_u64(result, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    if (get_ws(s, 0, &w) != hipSuccess) return UTF_ERR_HIP;
    return base::launch_utf16_length(frame_of(in), head_bytes(in), (long long)n, w->partials, w->ctrl, result, s) ==
                   hipSuccess
               ? UTF_OK
               : UTF_ERR_HIP;
}

int32_t utf8_length_from_utf16le_async(const uint16_t *in, uint64_t m, uint64_t *result, void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return c;
    if (!result) return UTF_ERR_NULL;
    hipStream_t s = as_stream(stream);
    if (m == 0) return base::launch_set_u64(result, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    Workspace *w;
    if (get_ws(s, 0, &w) != hipSuccess) return UTF_ERR_HIP;
    return base::launch_utf8_length(frame_of(in), head_bytes(in) / 2, (long long)m, w->partials, w->ctrl, result, s) ==
                   hipSuccess
               ? UTF_OK
               : UTF_ERR_HIP;
}

int32_t utfgpu_release_workspace(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    int32_t rc = UTF_OK;
    for (auto &kv : g_ws) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(kv.first.first) != hipSuccess) rc = UTF_ERR_HIP;
        if (hipStreamSynchronize(kv.first.second) != hipSuccess) rc = UTF_ERR_HIP;
        free_ws(kv.second);
        (void)hipSetDevice(prev);
    }
    g_ws.clear();
    return rc;
}

int32_t convert_utf8_to_utf16le_batch_async(const uint8_t *in, uint64_t n, const int64_t *offsets, uint64_t k,
                                            uint16_t *out, uint64_t out_cap, int64_t *out_offsets,
                                            utf_result *results, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return c;
    if (!offsets || !out_offsets || (k > 0 && !results)) return UTF_ERR_NULL;
    if (!out && out_cap > 0) return UTF_ERR_NULL;
    if (reinterpret_cast<uintptr_t>(out) & 1u) return UTF_ERR_ALIGN;
    if (k >= UTF_MAX_BATCH_STRINGS) return UTF_ERR_TOO_BIG;
    hipStream_t s = as_stream(stream);
    if (k == 0) {   // no strings partition a non-empty input
        if (n != 0) return UTF_ERR_OFFSETS;
        return base::launch_set_u64(reinterpret_cast<u64 *>(out_offsets), 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    }
    const long long head = n > 0 ? head_bytes(in) : 0;
    const Geometry &g = geometry_for(UTF_OP_BATCH_UTF8, n);
    const u64 nt = n > 0 ? g.utf8_tiles_for(head, (long long)n) : 0;
    Workspace *w;
    if (get_ws(s, nt, &w) != hipSuccess) return UTF_ERR_HIP;
    if (get_batch(w, nt, g.tile_bytes(), g.waves, k, s) != hipSuccess) return UTF_ERR_HIP;
    if (g.utf8_batch(n > 0 ? frame_of(in) : nullptr, head, (long long)n, offsets, k, out, out_cap, out_offsets,
                          reinterpret_cast<DevResult *>(results), w->status, w->ctrl, w->starts,
                          w->blockoff, w->tilepre, w->serr, &w->ctrl->bad, w->wavestr,
                          schedule_for(UTF_OP_BATCH_UTF8, n), s) != hipSuccess)
        return UTF_ERR_HIP;
    return UTF_OK;
}

int32_t convert_utf16le_to_utf8_batch_async(const uint16_t *in, uint64_t m, const int64_t *offsets, uint64_t k,
                                            uint8_t *out, uint64_t out_cap, int64_t *out_offsets,
                                            utf_result *results, void *stream) {
    int32_t c = check16(in, m);
    if (c != UTF_OK) return c;
    if (!offsets || !out_offsets || (k > 0 && !results)) return UTF_ERR_NULL;
    if (!out && out_cap > 0) return UTF_ERR_NULL;
    if (k >= UTF_MAX_BATCH_STRINGS) return UTF_ERR_TOO_BIG;
    hipStream_t s = as_stream(stream);
    if (k == 0) {   // no strings partition a non-empty input
        if (m != 0) return UTF_ERR_OFFSETS;
        return base::launch_set_u64(reinterpret_cast<u64 *>(out_offsets), 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    }
    const long long head = m > 0 ? head_bytes(in) / 2 : 0;
    const Geometry &g = geometry_for(UTF_OP_BATCH_UTF16LE, 2 * m);
    const u64 nt = m > 0 ? g.utf16_tiles_for(head, (long long)m) : 0;
    Workspace *w;
    if (get_ws(s, nt, &w) != hipSuccess) return UTF_ERR_HIP;
    if (get_batch(w, nt, g.tile_bytes() / 2, g.waves, k, s) != hipSuccess) return UTF_ERR_HIP;
    if (g.utf16_batch(m > 0 ? frame_of(in) : nullptr, head, (long long)m, offsets, k, out, out_cap, out_offsets,
                           reinterpret_cast<DevResult *>(results), w->status, w->ctrl, w->starts,
                           w->blockoff, w->tilepre, w->serr, &w->ctrl->bad, w->wavestr,
                           schedule_for(UTF_OP_BATCH_UTF16LE, 2 * m), s) != hipSuccess)
        return UTF_ERR_HIP;
    return UTF_OK;
}

int32_t convert_utf8_to_utf16le_noalloc_async(const uint8_t *in, uint64_t n, uint16_t *out, uint64_t out_cap,
                                              utf_result *result, void *stream) {
    int32_t c = check8(in, n);
    if (c != UTF_OK) return c;
    if (!result || (!out && out_cap > 0)) return UTF_ERR_NULL;
    if (reinterpret_cast<uintptr_t>(out) & 1u) return UTF_ERR_ALIGN;
    hipStream_t s = as_stream(stream);
    DevResult *r = reinterpret_cast<DevResult *>(result);
    if (n == 0) return base::launch_set_result(r, UTF_OK, 0, s) == hipSuccess ? UTF_OK : UTF_ERR_HIP;
    const long long head = head_bytes(in);
    const Geometry &g = geometry_for(UTF_OP_CONVERT_UTF8, n);
    const u64 nt = g.utf8_tiles_for(head, (long long)n);
    if (nt > kNoAllocTiles) return UTF_ERR_TOO_BIG;
    u64 *p = nullptr;
    if (noalloc_scratch(s, &p) != hipSuccess) return UTF_ERR_HIP;
    if (g.utf8_tiles(true, frame_of(in), head, (long long)n, out, out_cap, p + kNoAllocCtrlWords,
                     reinterpret_cast<Ctrl *>(p), r, schedule_for(UTF_OP_CONVERT_UTF8, n), s) != hipSuccess)
        return UTF_ERR_HIP;
    return UTF_OK;
}

const char *utfgpu_version(void) { return "utfgpu 0.2 gfx950"; }

uint64_t utfgpu_tile_bytes(void) { return kGeometries[0].tile_bytes(); }

int32_t utfgpu_geometry_count(void) { return kNumGeometries; }

int32_t utfgpu_geometry(int32_t g, uint32_t *waves, uint32_t *rows, uint64_t *tile_bytes) {
    if (g < 0 || g >= kNumGeometries) return UTF_ERR_ARG;
    if (waves) *waves = kGeometries[g].waves;
    if (rows) *rows = kGeometries[g].rows;
    if (tile_bytes) *tile_bytes = kGeometries[g].tile_bytes();
    return UTF_OK;
}

int32_t utfgpu_set_geometry(int32_t op, int32_t size_class, int32_t g) {
    if (op < 0 || op >= UTF_OP_COUNT || size_class < 0 || size_class >= UTF_SIZE_CLASSES) return UTF_ERR_ARG;
    if (g < -1 || g >= kNumGeometries) return UTF_ERR_ARG;
    g_table[op][size_class].store((uint8_t)(g < 0 ? 0 : g + 1), std::memory_order_relaxed);
    return UTF_OK;
}

int32_t utfgpu_get_geometry(int32_t op, int32_t size_class) {
    if (op < 0 || op >= UTF_OP_COUNT || size_class < 0 || size_class >= UTF_SIZE_CLASSES) return UTF_ERR_ARG;
    const int f = forced_geometry();
    if (f >= 0) return f;
    return table_geometry(op, size_class);
}

int32_t utfgpu_size_class(uint64_t bytes) { return size_class(bytes); }

int32_t utfgpu_set_schedule(int32_t op, int32_t size_class, int32_t schedule) {
    if (op < 0 || op >= UTF_OP_COUNT || size_class < 0 || size_class >= UTF_SIZE_CLASSES) return UTF_ERR_ARG;
    if (schedule < -1 || schedule >= kNumSchedules) return UTF_ERR_ARG;
    g_sched[op][size_class].store((uint8_t)(schedule < 0 ? 0 : schedule + 1), std::memory_order_relaxed);
    return UTF_OK;
}

int32_t utfgpu_get_schedule(int32_t op, int32_t size_class) {
    if (op < 0 || op >= UTF_OP_COUNT || size_class < 0 || size_class >= UTF_SIZE_CLASSES) return UTF_ERR_ARG;
    const int f = forced_schedule();
    return f >= 0 ? f : table_schedule(op, size_class);
}

}  // extern "C"
