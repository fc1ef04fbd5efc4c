// device_common.hpp -- shared device machinery of the gfx950 UTF kernels.
//
// Geometry.  A workgroup is kWaves wave64 waves.  Every lane
// loads kRows 16-byte chunks; the chunks of one row of one wave are
// contiguous (1 KiB per row, coalesced dwordx4 loads), the rows of a wave
// follow each other, and the waves of a workgroup follow each other, so a
// tile is kTileBytes contiguous input bytes.  Tile t is workgroup t.
//
// Buffers are addressed through an aligned "frame": frame = input address
// rounded down to 16 bytes, head = input address - frame.  Input unit i sits
// at frame position head + i.  A chunk is loaded only when it holds at least
// one input unit, so every load stays inside 16-byte blocks that contain
// caller data; positions outside [head, head + n) read as zero.
//
// Output offsets come from an exclusive scan of per-position output widths:
// lanes -> wave (shuffles) -> workgroup (LDS) -> device (decoupled
// look-back over one 64-bit status word per tile: 2 flag bits, 22 epoch
// bits, 40 value bits).  The epoch tags the words written by one call, so
// the status array is never cleared between calls.  A wave that waits too
// long for a predecessor's word computes that tile's aggregate itself and
// publishes it, so no wait depends on the order in which the hardware
// starts workgroups.
//
// Nothing in a tile's path uses a device-scope fence (on gfx950 those write
// back and invalidate the L2) or a shared counter: the result of a call is
// formed by a one-workgroup finalize kernel queued after the tile kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The tile geometry is fixed per build of the kernel files, which are
// compiled once per entry of geometries.def with UTF_GEOM (a namespace),
// UTF_WAVES and UTF_ROWS set; the C ABI picks one build per call.  Without
// them a file builds the default geometry.
#ifndef UTF_GEOM
#define UTF_GEOM g8x4
#define UTF_WAVES 8
#define UTF_ROWS 4
#endif

namespace utfgpu {

constexpr int kWave = 64;
constexpr int kChunk = 16;                         // bytes per lane and row

namespace UTF_GEOM {

// Default: tiles of 32 KiB in workgroups of eight waves; two workgroups fit
// on a CU (the tile kernels are held to 128 VGPRs, four waves per SIMD), so
// one's load latency and look-back wait overlap the other's work.  Smaller
// builds trade per-tile work for more workgroups on small inputs.
constexpr int kWaves = UTF_WAVES;
constexpr int kBlock = kWaves * kWave;             // 512 lanes by default
constexpr int kRows = UTF_ROWS;
constexpr int kGroup = 1;                          // rows staged at a time
constexpr int kRowBytes = kWave * kChunk;          // 1024
constexpr int kWaveBytes = kRows * kRowBytes;      // 4096 by default
constexpr int kTileBytes = kWaves * kWaveBytes;    // 32768 by default
static_assert(kRows % 2 == 0 && kRows >= 2, "rows are scanned in pairs");
static_assert(kBlock <= 1024, "workgroup size");

}  // namespace UTF_GEOM

constexpr int kMaxPartials = 2048;                 // workgroups of the length reductions

// Status codes; the same values as the public header.
enum : uint32_t {
    kOk = 0,
    kTooShort = 1,
    kTooLong = 2,
    kOverlong = 3,
    kTooLarge = 4,
    kSurrogate = 5,
    kHeaderBits = 6,
    kUnpairedHigh = 7,
    kUnpairedLow = 8,
    kOutputTooSmall = 9,
};
constexpr int32_t kErrOffsets = -5;   // batched calls: the offsets array is not a valid partition

typedef uint64_t u64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Device result layout, identical to utf_result.
struct DevResult {
    int32_t status;
    int32_t pad;
    u64 count;
};

// Per-workspace control block, the fields the tiles write each on its own
// 64-byte line.  The last kernel of every call (the finalize kernel, or for
// batched calls the last workgroup of the post kernel) resets the per-call
// fields and advances `epoch`, so each call finds it in the same state.
// Epochs run 1 .. period-1; the call whose finalize would reach `period`
// clears every status word of the workspace and starts again at 1, so a
// status word left by an earlier call never carries the current epoch,
// however many calls (eager or replayed from a captured graph) ran.
struct Ctrl {
    u64 err;        // min over (position << 4 | kind); ~0 when no error
    u64 ticket;     // ticket order: the next tile index to hand out
    u64 done;       // batched calls: post-kernel workgroups finished
    u64 pad0[5];
    u64 total;      // output units of the whole call (written by the last tile)
    uint32_t bad;   // batched calls: the offsets are not a partition of the input
    uint32_t pad_b;
    u64 pad1[6];
    u64 epoch;      // tag of the status words of the current call
    u64 period;     // at most 2^22 (the epoch field of a status word)
    u64 *status;    // the workspace's status words, kStatusStride words apart
    u64 status_cap; // number of status words
    u64 pad2[4];
};

// ------------------------------------------------------------------------
// Agent-scope memory operations (visible across the eight XCDs).
// ------------------------------------------------------------------------
__device__ __forceinline__ u64 ld_agent(u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(u64 *p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void min_agent(u64 *p, u64 v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_agent(u64 *p, u64 expected, u64 desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------
// Wave primitives
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Inclusive prefix sum over the 64 lanes with DPP: shifts by 1, 2, 4 and 8
// lanes within each row of 16 (lanes shifted in from outside the row read
// 0), then the last lane of row 0 / row 2 added to rows 1 / 3, then lane 31
// added to rows 2 and 3.  Six adds, no LDS traffic.  (`lane` is unused: the
// DPP row controls select the lanes.)
constexpr int kDppRowShr = 0x110;     // row_shr:n is kDppRowShr + n
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t /*lane*/) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr + 1, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr + 2, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr + 4, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowShr + 8, 0xF, 0xF, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast15, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast31, 0xC, 0xF, false);
    return v;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ u64 wave_min_u64(u64 v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        u64 t = __shfl_xor(v, d);
        v = t < v ? t : v;
    }
    return v;
}

// LDS written by some lanes of a wave becomes readable by the others.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// a + byte k of b (k = 0..3, a constant after unrolling) in one
// instruction: v_add_u32 with an SDWA byte select on its second source.
// Running slot offsets use it to advance by a per-byte step taken from a
// register that holds the steps of four byte positions.
__device__ __forceinline__ uint32_t add_byte(uint32_t a, uint32_t b, int k) {
    uint32_t d;
    switch (k) {
        case 0:
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
                : "=v"(d) : "v"(a), "v"(b));
            break;
        case 1:
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
                : "=v"(d) : "v"(a), "v"(b));
            break;
        case 2:
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
                : "=v"(d) : "v"(a), "v"(b));
            break;
        default:
            asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
                : "=v"(d) : "v"(a), "v"(b));
            break;
    }
    return d;
}

// LDS byte address of a pointer into a __shared__ array, and LDS pointers
// made from such addresses.  A running store address kept absolute (base
// included) serves each store as its address register as it is; kept as
// an offset from a wave's stage, every store would first add the base.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) T *lptr(uint32_t a) {
    return (__attribute__((address_space(3))) T *)(uintptr_t)a;
}

// A constant in a scalar register.  VOP3 instructions such as v_perm_b32
// take no literal operand on this target, so a constant selector held in
// a vector register is rematerialised with a v_mov wherever the register
// allocator has dropped it; made by s_mov, it costs no vector issue slot.
template <uint32_t kV>
__device__ __forceinline__ uint32_t sconst() {
    uint32_t v;
    asm("s_mov_b32 %0, %1" : "=s"(v) : "i"(kV));
    return v;
}

// bytes k..k+3 of the 8-byte little-endian pair (lo, hi)
__device__ __forceinline__ uint32_t window4(uint32_t lo, uint32_t hi, int k) {
    return k == 0 ? lo : __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)k);
}

// Zero the bytes of the dword at frame position p that fall outside
// [lo, hi).
__device__ __forceinline__ uint32_t keep_range(uint32_t x, long long p, long long lo, long long hi) {
    long long a = lo - p;   // first kept byte
    long long b = hi - p;   // one past the last kept byte
    uint32_t m = 0xFFFFFFFFu;
    if (b <= 0) return 0u;
    if (b < 4) m &= (1u << (8 * b)) - 1u;
    if (a >= 4) return 0u;
    if (a > 0) m &= ~((1u << (8 * a)) - 1u);
    return x & m;
}

// ------------------------------------------------------------------------
// Tile tickets (the ticket-order scan schedule)
// ------------------------------------------------------------------------
// In ticket order a workgroup takes its tile index from a counter in the
// control block, in the order the workgroups start, instead of using the
// workgroup index: every tile before a running tile then belongs to a
// workgroup that has already started, so a look-back never waits on a
// workgroup the hardware has not placed -- which, with several look-back
// kernels in flight on other streams, can happen for a while.  The finalize
// kernel resets the counter.  Run by the whole workgroup; `slot` is a
// __shared__ word.  The tile kernels are compiled for both schedules (a
// template argument, so block order carries no trace of the counter); the
// launchers take the schedule index of the C ABI.
constexpr int kScheduleTicket = 1;
__device__ __forceinline__ u64 take_ticket(Ctrl *ctrl, uint32_t *slot, uint32_t tid) {
    if (tid == 0) *slot = (uint32_t)__hip_atomic_fetch_add(&ctrl->ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return (u64)__builtin_amdgcn_readfirstlane(*slot);   // fewer than 2^32 tiles
}

// ------------------------------------------------------------------------
// Decoupled look-back status words
// ------------------------------------------------------------------------
// Status words sit kStatusStride words apart, so the words a probe reads
// spread over many memory channels instead of hammering a few lines.
constexpr int kStatusStride = 32;   // 256 bytes

constexpr u64 kFlagAggregate = 1ull;
constexpr u64 kFlagPrefix = 2ull;
constexpr u64 kEpochMask = (1ull << 22) - 1;
constexpr u64 kValueMask = (1ull << 40) - 1;
constexpr int kDefaultSpinLimit = 48;   // probes (about 1 us each) before helping

__device__ __forceinline__ u64 pack_status(u64 flag, u64 epoch, u64 value) {
    return (flag << 62) | ((epoch & kEpochMask) << 40) | (value & kValueMask);
}
__device__ __forceinline__ bool status_ready(u64 s, u64 epoch) {
    return (s >> 62) != 0 && ((s >> 40) & kEpochMask) == (epoch & kEpochMask);
}

// Exclusive prefix of tile t (t > 0), run by one whole wave.  A probe
// reads a window of kLookK * 64 predecessors: lane j looks at tiles
// t-1-kLookK*j-k, k = 0..kLookK-1.  The sum runs from the nearest
// predecessor that carries an inclusive prefix, so only the tiles up to
// that one must have published; if none in the window does, their
// aggregates are added and the window moves back.  Knowledge of prefixes
// therefore advances one window per status round trip (about 1.5 us), so
// the window, not the tile size alone, bounds how many tiles per second
// the scan can serve.  If a needed predecessor stays silent for
// `spin_limit` probes, the wave computes its aggregate with `agg(tile)` (a
// wave-wide call returning the same value in every lane) and publishes it
// unless the owner has done so meanwhile.
constexpr int kLookK = 2;

template <class Agg>
__device__ __forceinline__ u64 lookback(u64 *status, long long t, u64 epoch, int spin_limit, Agg agg) {
    const uint32_t lane = lane_id();
    u64 excl = 0;
    for (long long j = t - 1;; j -= (long long)kLookK * kWave) {
        const long long i0 = j - (long long)kLookK * lane;   // nearest tile of the lane
        u64 s[kLookK];
#pragma unroll
        for (int k = 0; k < kLookK; ++k)
            s[k] = i0 - k >= 0 ? ld_agent(status + (i0 - k) * kStatusStride) : pack_status(kFlagPrefix, epoch, 0);
        for (int spins = 0;;) {
            // the lane's nearest prefix kp, whether a tile before it is not
            // ready, the first such tile, and the sum up to the prefix
            int kp = kLookK, fk = kLookK;
            u64 lsum = 0;
#pragma unroll
            for (int k = 0; k < kLookK; ++k) {
                const bool rdy = i0 - k < 0 || status_ready(s[k], epoch);
                if (kp == kLookK) {
                    if (!rdy && fk == kLookK) fk = k;
                    if (rdy) {
                        lsum += s[k] & kValueMask;
                        if ((s[k] >> 62) == kFlagPrefix) kp = k;
                    }
                }
            }
            const u64 pmask = __ballot(kp < kLookK);
            const u64 low = pmask & (~pmask + 1);                 // lane of the nearest prefix
            const u64 need = pmask ? (low << 1) - 1 : ~0ull;      // lanes up to it
            const u64 blocking = __ballot(fk < kLookK) & need;
            if (blocking == 0) {
                excl += wave_sum_u64(((need >> lane) & 1u) ? lsum : 0);
                if (pmask) return excl;
                break;
            }
            if (spins >= spin_limit) {
                const int L = __ffsll((long long)blocking) - 1;
                const int k = (int)readlane((uint32_t)fk, L);
                const long long miss = j - (long long)kLookK * L - k;
                const u64 a = agg(miss);
                u64 old = s[0];
#pragma unroll
                for (int q = 1; q < kLookK; ++q)
                    if (q == k) old = s[q];
                if ((int)lane == L) cas_agent(status + miss * kStatusStride, old, pack_status(kFlagAggregate, epoch, a));
                spins = 0;
            } else {
                __builtin_amdgcn_s_sleep(4);
                ++spins;
            }
#pragma unroll
            for (int k = 0; k < kLookK; ++k)
                if (i0 - k >= 0 && !status_ready(s[k], epoch)) s[k] = ld_agent(status + (i0 - k) * kStatusStride);
        }
    }
}

// Publish tile t's aggregate, resolve its exclusive prefix, publish its
// inclusive prefix.  Run by one whole wave; returns the exclusive prefix.
template <class Agg>
__device__ __forceinline__ u64 resolve_prefix(u64 *status, u64 t, u64 epoch, int spin_limit, u64 tile_total,
                                              Agg agg) {
    const uint32_t lane = lane_id();
    if (t == 0) {
        if (lane == 0) st_agent(status, pack_status(kFlagPrefix, epoch, tile_total));
        return 0;
    }
    if (lane == 0) st_agent(status + t * kStatusStride, pack_status(kFlagAggregate, epoch, tile_total));
    const u64 prefix = lookback(status, (long long)t, epoch, spin_limit, agg);
    if (lane == 0) st_agent(status + t * kStatusStride, pack_status(kFlagPrefix, epoch, prefix + tile_total));
    return prefix;
}

// End of a call: reset the per-call fields of the control block and
// advance the epoch.  The call that would reach the period first clears
// every status word of the workspace (with all `nthreads` threads of the
// calling workgroup) and starts again at epoch 1.  Run by a whole
// workgroup, after every other reader of the per-call fields is done.
__device__ __forceinline__ void reset_control(Ctrl *ctrl, uint32_t tid, uint32_t nthreads) {
    const u64 next = ld_agent(&ctrl->epoch) + 1;
    const bool wrap = next >= ctrl->period;
    __syncthreads();   // every thread has read the epoch before thread 0 advances it
    if (wrap) {
        u64 *st = ctrl->status;
        const u64 cap = ctrl->status_cap;
        for (u64 t = tid; t < cap; t += nthreads) st_agent(st + t * kStatusStride, 0);
    }
    if (tid != 0) return;
    st_agent(&ctrl->err, ~0ull);
    st_agent(&ctrl->total, 0);
    st_agent(&ctrl->ticket, 0);
    st_agent(&ctrl->done, 0);
    ctrl->bad = 0;
    st_agent(&ctrl->epoch, wrap ? 1 : next);
}

// Threads per workgroup of the batched calls' prep and post kernels
// (multiples of the wave size).
constexpr uint32_t kPrepBlock = 256;
constexpr uint32_t kPostBlock = 256;

// Batched calls end in their post kernel: every workgroup counts itself
// done once its threads have read what they need of the control block, and
// the last one resets it (so no separate finalize launch is needed).
__device__ __forceinline__ void batch_call_done(Ctrl *ctrl, uint32_t tid) {
    __shared__ uint32_t s_last;
    __syncthreads();   // every thread of the workgroup has finished its string
    if (tid == 0)
        s_last = __hip_atomic_fetch_add(&ctrl->done, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 (u64)gridDim.x - 1;
    __syncthreads();
    if (s_last) reset_control(ctrl, tid, blockDim.x);
}

// ------------------------------------------------------------------------
// Batched calls
// ------------------------------------------------------------------------
// Batched calls: k strings, string i occupying input units [offsets[i],
// offsets[i+1]).  Outputs are compact: string i's output starts at the sum
// of the length-query values of strings 0..i-1, which is the scan of the
// per-unit widths at offsets[i], so one device-wide scan serves them all.
struct BatchCtx {
    const int64_t *offsets;   // k + 1 boundaries
    u64 k;
    const uint16_t *starts;   // bitmap over frame positions: a non-empty string starts here
    uint16_t *blockoff;       // per block of the frame (64 bytes / 32 words): its output offset inside its tile
    u64 *tilepre;             // per tile: output offset of the tile
    u64 *serr;                // per string: min (position << 4 | kind), ~0 when valid
    const uint32_t *wavestr;  // per wave span: the string owning its first position (one more entry at the end)
};

// The string that owns input unit p: the largest i with offsets[i] <= p
// (an empty string owns no byte, and is never the largest such i).
// Binary search in [lo, hi); returns lo at once when hi <= lo + 1 (which
// offsets that are not a partition can produce: such a call reports
// ERR_OFFSETS for every string, and the search only has to end).
__device__ __forceinline__ u64 owner_string(const int64_t *offsets, u64 lo, u64 hi, long long p) {
    while (hi > lo + 1) {
        const u64 mid = (lo + hi) / 2;
        if (offsets[mid] <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The owner of input unit p lying in wave span w or in the three units
// before it: between the owners of spans w-1 and w+1.  The span owners are
// clamped to [0, k): with offsets that are not a partition some spans have
// no owner and keep a value from an earlier call.
__device__ __forceinline__ u64 owner_near(const BatchCtx &bc, long long w, long long p) {
    const u64 last = bc.k - 1;   // k >= 1 whenever a tile kernel runs
    u64 lo = bc.wavestr[w > 0 ? w - 1 : 0];
    u64 hi1 = (u64)bc.wavestr[w + 1] + 1;
    lo = lo < last ? lo : last;
    hi1 = hi1 < bc.k ? hi1 : bc.k;
    return owner_string(bc.offsets, lo, hi1, p);
}

// ------------------------------------------------------------------------
// Write-out of staged output
// ------------------------------------------------------------------------
// Output addresses are computed as integers; gptr turns one back into a
// pointer in the global address space, so the stores are global_store
// instructions.  (A plain pointer made from an integer is a generic one:
// flat stores, which also count against the LDS wait counter and so hold
// back every later LDS wait of the wave.)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(uintptr_t a) {
    return (__attribute__((address_space(1))) T *)a;
}

// The output occupies bytes [g0, g0 + nbytes) of global memory.  `stage`
// (LDS, dword aligned) holds those bytes starting at stage byte 0.  Whole
// 16-byte aligned global blocks are written with one dwordx4 store each;
// the partial blocks at the two ends are written with stores of kUnit bytes
// so that neighbouring ranges never touch each other's bytes.  Run by
// kThreads threads with index `tid`.
template <int kUnit, int kThreads>
__device__ __forceinline__ void write_out(uint8_t *g0p, u64 nbytes, const uint32_t *stage, uint32_t tid) {
    if (nbytes == 0) return;
    const uintptr_t g0 = (uintptr_t)g0p;
    const uintptr_t g1 = g0 + nbytes;
    const uintptr_t c0 = g0 & ~(uintptr_t)15;
    const uintptr_t cend = (g1 + 15) & ~(uintptr_t)15;
    const uint32_t shift = (uint32_t)((c0 - g0) & 3);   // (c - g0) mod 4 is the same for all blocks
    const uint8_t *sb = (const uint8_t *)stage;
    for (uintptr_t c = c0 + 16 * (uintptr_t)tid; c < cend; c += 16 * kThreads) {
        if (c >= g0 && c + 16 <= g1) {
            const uintptr_t so = c - g0;          // stage byte offset of the block
            const uint32_t *w = stage + (so >> 2);
            u32x4 v;
            if (shift == 0) {
                v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
            } else {
                const uint32_t a0 = w[0], a1 = w[1], a2 = w[2], a3 = w[3], a4 = w[4];
                v.x = __builtin_amdgcn_alignbyte(a1, a0, shift);
                v.y = __builtin_amdgcn_alignbyte(a2, a1, shift);
                v.z = __builtin_amdgcn_alignbyte(a3, a2, shift);
                v.w = __builtin_amdgcn_alignbyte(a4, a3, shift);
            }
            __builtin_nontemporal_store(v, gptr<u32x4>(c));
        } else {
            for (uintptr_t a = c; a < c + 16; a += kUnit) {
                if (a >= g0 && a < g1) {
                    const uintptr_t so = a - g0;
                    if (kUnit == 2)
                        *gptr<uint16_t>(a) = *(const uint16_t *)(sb + so);
                    else
                        *gptr<uint8_t>(a) = sb[so];
                }
            }
        }
    }
}

// Same, for a stage laid out by 16-byte blocks of global memory: global
// byte g sits at stage byte g - (g0 & ~15), so the data starts at stage
// byte g0 & 15 and every whole block is one aligned 16-byte LDS read.
template <int kUnit, int kThreads>
__device__ __forceinline__ void write_out_aligned(uint8_t *g0p, u64 nbytes, const uint32_t *stage, uint32_t tid) {
    if (nbytes == 0) return;
    const uintptr_t g0 = (uintptr_t)g0p;
    const uintptr_t g1 = g0 + nbytes;
    const uintptr_t c0 = g0 & ~(uintptr_t)15;
    const uintptr_t cend = (g1 + 15) & ~(uintptr_t)15;
    const uint8_t *sb = (const uint8_t *)stage;
    for (uintptr_t c = c0 + 16 * (uintptr_t)tid; c < cend; c += 16 * kThreads) {
        const uint32_t so = (uint32_t)(c - c0);
        if (c >= g0 && c + 16 <= g1) {
            const u32x4 v = *(const u32x4 *)(sb + so);
            __builtin_nontemporal_store(v, gptr<u32x4>(c));
        } else {
            for (uint32_t k = 0; k < 16; k += kUnit) {
                const uintptr_t a = c + k;
                if (a >= g0 && a < g1) {
                    if (kUnit == 2)
                        *gptr<uint16_t>(a) = *(const uint16_t *)(sb + so + k);
                    else
                        *gptr<uint8_t>(a) = sb[so + k];
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
// Write-out of a wave's rows with the tail block carried over
// ------------------------------------------------------------------------
// A wave writes its output row by row from a stage laid out by 16-byte
// blocks of global memory (the row's first byte g0 at stage byte g0 & 15).
// The last block of a row is usually shared with the next row, so it is
// not written but carried (16 bytes, the same in every lane) into the next
// row, whose block 0 it completes in registers.  Only the wave's first and last
// blocks are written in part; those take at most eight aligned stores of
// 1/2/4/8 bytes (never below the unit size).
struct Carry {
    uint32_t v[4];
};

// Bytes [a, b) (both inside the 16-byte block at c) from stage bytes
// [a - c + so, b - c + so), with aligned power-of-two stores.
template <int kUnit>
__device__ __forceinline__ void store_part(uintptr_t c, uintptr_t a, uintptr_t b, const uint8_t *sb, uint32_t so) {
#pragma unroll
    for (int sz = kUnit; sz <= 8; sz <<= 1) {   // up to the first 16-byte aligned chunk
        if ((a & (uintptr_t)sz) && a + sz <= b) {
            const uint32_t o = so + (uint32_t)(a - c);
            if (sz == 1) *gptr<uint8_t>(a) = sb[o];
            if (sz == 2) *gptr<uint16_t>(a) = *(const uint16_t *)(sb + o);
            if (sz == 4) *gptr<uint32_t>(a) = *(const uint32_t *)(sb + o);
            if (sz == 8) *gptr<uint64_t>(a) = *(const uint64_t *)(sb + o);
            a += sz;
        }
    }
#pragma unroll
    for (int sz = 8; sz >= kUnit; sz >>= 1) {   // the rest, largest first
        if (a + sz <= b) {
            const uint32_t o = so + (uint32_t)(a - c);
            if (sz == 1) *gptr<uint8_t>(a) = sb[o];
            if (sz == 2) *gptr<uint16_t>(a) = *(const uint16_t *)(sb + o);
            if (sz == 4) *gptr<uint32_t>(a) = *(const uint32_t *)(sb + o);
            if (sz == 8) *gptr<uint64_t>(a) = *(const uint64_t *)(sb + o);
            a += sz;
        }
    }
}

// Block 0 of a row whose first byte is at g0 & 15 = k (1..15): its bytes
// before k come from the carried block.  Wave-uniform k: scalar masks.
__device__ __forceinline__ u32x4 blend_carry(u32x4 b, const Carry &cy, uint32_t k) {
    uint32_t m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int lo = 4 * i;
        m[i] = (int)k >= lo + 4 ? 0xFFFFFFFFu : ((int)k <= lo ? 0u : ((1u << (8 * ((int)k - lo))) - 1u));
    }
    b.x = (cy.v[0] & m[0]) | (b.x & ~m[0]);
    b.y = (cy.v[1] & m[1]) | (b.y & ~m[1]);
    b.z = (cy.v[2] & m[2]) | (b.z & ~m[2]);
    b.w = (cy.v[3] & m[3]) | (b.w & ~m[3]);
    return b;
}

// Write a row's output [g0, g1) except its unfinished last block, which
// goes to `cy`; bytes before `wstart` (the wave's first output byte) are
// never written.  Whole wave, after an LDS sync; the stage holds the row.
// `merge`: the previous row's carried block ends at g0, so block 0 takes
// its bytes before g0 (in registers, on its way to memory or to the next
// carry).  Lane i stores blocks i, i + 64, ...: the first kIters of them
// are read from LDS together and then stored, so the reads' latency is
// paid once per row; a row of more blocks (not produced by the callers'
// stage sizes) finishes in a plain loop.
template <int kUnit, int kIters>
__device__ __forceinline__ void write_row(uintptr_t g0, uintptr_t g1, uintptr_t wstart, uint32_t *stage,
                                          uint32_t lane, Carry &cy, bool merge) {
    const uintptr_t c0 = g0 & ~(uintptr_t)15;
    const uintptr_t lo = c0 > wstart ? c0 : wstart;   // lo < c0 + 16
    const uintptr_t hi = g1 & ~(uintptr_t)15;
    const uint32_t k = (uint32_t)(g0 & 15u);
    merge = merge && k != 0;
    const uint8_t *sb = (const uint8_t *)stage;
    const uint32_t nb = (uint32_t)((hi - c0) >> 4);   // blocks before the carried one
    const bool part0 = c0 < lo;                       // block 0 begins before the wave's bytes
    u32x4 v[kIters];
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
        const uint32_t b = lane + (uint32_t)(kWave * i);
        v[i] = b < nb ? *(const u32x4 *)(sb + 16u * b) : u32x4{0u, 0u, 0u, 0u};
    }
    if (merge && lane == 0) v[0] = blend_carry(v[0], cy, k);
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
        const uint32_t b = lane + (uint32_t)(kWave * i);
        if (b < nb && (b != 0 || !part0)) __builtin_nontemporal_store(v[i], gptr<u32x4>(c0 + 16 * (uintptr_t)b));
    }
    for (uint32_t b = lane + (uint32_t)(kWave * kIters); b < nb; b += kWave)
        __builtin_nontemporal_store(*(const u32x4 *)(sb + 16u * b), gptr<u32x4>(c0 + 16 * (uintptr_t)b));
    if (part0 && nb != 0 && lane == 0) {   // bytes [lo, c0 + 16) of block 0, through the stage
        *(u32x4 *)stage = v[0];
        store_part<kUnit>(c0, lo, c0 + 16, sb, 0);
    }
    if (g1 & 15u) {   // every lane reads the same block; kept in scalar registers
        u32x4 b = *(const u32x4 *)(sb + (uint32_t)(hi - c0));
        if (merge && nb == 0) b = blend_carry(b, cy, k);   // the carried block is block 0
        cy.v[0] = __builtin_amdgcn_readfirstlane(b.x);
        cy.v[1] = __builtin_amdgcn_readfirstlane(b.y);
        cy.v[2] = __builtin_amdgcn_readfirstlane(b.z);
        cy.v[3] = __builtin_amdgcn_readfirstlane(b.w);
    }
}

// Passes of write_row over a stage of kBytes bytes of output plus up to 15
// bytes of block offset.
template <int kBytes>
constexpr int row_write_iters() {
    return ((kBytes + 15) / 16 + kWave - 1) / kWave;
}

// The wave's last unfinished block: bytes [max(block, wstart), gend) from
// the carry.  Lane 0 writes it through block 0 of the stage.
template <int kUnit>
__device__ __forceinline__ void flush_carry(uintptr_t gend, uintptr_t wstart, uint32_t *stage, const Carry &cy,
                                            uint32_t lane) {
    if (!(gend & 15u)) return;
    const uintptr_t c = gend & ~(uintptr_t)15;
    if (lane == 0) *(u32x4 *)stage = u32x4{cy.v[0], cy.v[1], cy.v[2], cy.v[3]};
    wave_lds_sync();
    if (lane == 0) store_part<kUnit>(c, c > wstart ? c : wstart, gend, (const uint8_t *)stage, 0);
}

// ------------------------------------------------------------------------
// Finalize: one workgroup queued after a tile kernel.
// ------------------------------------------------------------------------
enum : int { kFinValidate = 0, kFinConvert = 1, kFinLength = 2 };

namespace UTF_GEOM {
hipError_t launch_finalize(Ctrl *ctrl, DevResult *result, u64 *len_result, int mode, u64 n, u64 out_cap,
                           const u64 *partials, int npartials, hipStream_t stream);
// Set a control block up for a status array of `status_cap` words (all of
// which are cleared): no error, total 0, epoch 1, epochs wrapping at
// `period`.  Used when a workspace is made and when its status array is
// replaced by a larger one.
hipError_t launch_ctrl_init(Ctrl *ctrl, u64 *status, u64 status_cap, u64 period, hipStream_t stream);
}  // namespace UTF_GEOM

// Epoch period of new control blocks: UTFGPU_EPOCH_PERIOD when set (2 ..
// 2^22; small values exercise the wrap), else 2^22.
u64 epoch_period();

// Look-back probes before a wave computes a silent predecessor's aggregate
// itself: UTFGPU_LOOKBACK_SPINS when set (0 exercises the helping path on
// every wait), else kDefaultSpinLimit.
int lookback_spin_limit();

}  // namespace utfgpu
