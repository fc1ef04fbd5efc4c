// device_common.hpp -- shared device machinery of the gfx950 UTF kernels.
//
// Geometry.  A workgroup is 256 lanes (four wave64 waves).  Every lane
// loads kRows 16-byte chunks; the chunks of one row of one wave are
// contiguous (1 KiB per row, coalesced dwordx4 loads), the rows of a wave
// follow each other, and the waves of a workgroup follow each other, so a
// tile is kTileBytes contiguous input bytes.  Tiles are numbered in input
// order by an atomic ticket, which makes the single-pass scan below
// deadlock-free whatever order the hardware starts workgroups in.
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
// the status array is never cleared between calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utfgpu {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kRows = 4;
constexpr int kChunk = 16;
constexpr int kRowBytes = kWave * kChunk;          // 1024
constexpr int kWaveBytes = kRows * kRowBytes;      // 4096
constexpr int kTileBytes = kWaves * kWaveBytes;    // 16384

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

typedef uint64_t u64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Device result layout, identical to utf_result.
struct DevResult {
    int32_t status;
    int32_t pad;
    u64 count;
};

// Per-workspace control block.  Every call leaves it as it found it: the
// last workgroup to finish resets the ticket, the done counter, the error
// word and the total, and advances the epoch.
struct Ctrl {
    u64 ticket;     // next tile number
    u64 done;       // workgroups finished
    u64 err;        // min over (position << 4 | kind); ~0 when no error
    u64 total;      // output units of the whole call
    u64 epoch;      // tag of the status words of the current call
    u64 pad[3];
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
__device__ __forceinline__ u64 add_agent(u64 *p, u64 v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void min_agent(u64 *p, u64 v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (lane >= (uint32_t)d) v += t;
    }
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

// byte k (0..3) of a dword
__device__ __forceinline__ uint32_t byte_of(uint32_t x, int k) { return (x >> (8 * k)) & 0xFFu; }

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
// Decoupled look-back status words
// ------------------------------------------------------------------------
constexpr u64 kFlagAggregate = 1ull;
constexpr u64 kFlagPrefix = 2ull;
constexpr u64 kEpochMask = (1ull << 22) - 1;
constexpr u64 kValueMask = (1ull << 40) - 1;

__device__ __forceinline__ u64 pack_status(u64 flag, u64 epoch, u64 value) {
    return (flag << 62) | ((epoch & kEpochMask) << 40) | (value & kValueMask);
}
__device__ __forceinline__ bool status_ready(u64 s, u64 epoch) {
    return (s >> 62) != 0 && ((s >> 40) & kEpochMask) == (epoch & kEpochMask);
}

// Exclusive prefix of tile t (t > 0): run by one whole wave.  Lane j looks
// at tile t-1-j; once a window of 64 predecessors has published, the sum
// runs from the nearest predecessor that carries an inclusive prefix.
__device__ __noinline__ u64 lookback(u64 *status, long long t, u64 epoch) {
    const uint32_t lane = lane_id();
    u64 excl = 0;
    long long j = t - 1;
    for (;;) {
        long long idx = j - (long long)lane;
        u64 s;
        if (idx >= 0) {
            s = ld_agent(status + idx);
            while (!status_ready(s, epoch)) {
                __builtin_amdgcn_s_sleep(1);
                s = ld_agent(status + idx);
            }
        } else {
            s = pack_status(kFlagPrefix, epoch, 0);
        }
        u64 pmask = __ballot((s >> 62) == kFlagPrefix);
        u64 v = s & kValueMask;
        if (pmask) {
            int k = __ffsll((long long)pmask) - 1;
            if ((int)lane > k) v = 0;
            return excl + wave_sum_u64(v);
        }
        excl += wave_sum_u64(v);
        j -= kWave;
    }
}

// Called by one thread per workgroup after all of the workgroup's global
// effects.  True for the last workgroup of the launch.
__device__ __forceinline__ bool arrive_last(Ctrl *ctrl, u64 nblocks) {
    __threadfence();
    u64 old = __hip_atomic_fetch_add(&ctrl->done, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == nblocks - 1) {
        __threadfence();
        return true;
    }
    return false;
}

__device__ __forceinline__ void reset_ctrl(Ctrl *ctrl) {
    st_agent(&ctrl->ticket, 0);
    st_agent(&ctrl->done, 0);
    st_agent(&ctrl->err, ~0ull);
    st_agent(&ctrl->total, 0);
    st_agent(&ctrl->epoch, ld_agent(&ctrl->epoch) + 1);
    __threadfence();
}

__device__ __forceinline__ void write_result(DevResult *r, uint32_t status, u64 count) {
    r->status = (int32_t)status;
    r->pad = 0;
    r->count = count;
}

// ------------------------------------------------------------------------
// Write-out of a tile's staged output
// ------------------------------------------------------------------------
// The tile's output occupies bytes [g0, g1) of global memory, clamped to
// the caller's capacity.  `stage` (LDS) holds those bytes starting at
// stage byte 0 = global byte g0.  Whole 16-byte aligned global blocks are
// written with one dwordx4 store each; the two partial blocks at the ends
// are written with stores of `unit` bytes so that neighbouring tiles never
// touch each other's bytes.  Run by all 256 lanes.
template <int kUnit>
__device__ __forceinline__ void write_out(uint8_t *g0p, u64 nbytes, const uint32_t *stage, uint32_t tid) {
    if (nbytes == 0) return;
    const uintptr_t g0 = (uintptr_t)g0p;
    const uintptr_t g1 = g0 + nbytes;
    const uintptr_t c0 = g0 & ~(uintptr_t)15;
    const uintptr_t nblk = ((g1 + 15) & ~(uintptr_t)15) - c0;
    const uint32_t shift = (uint32_t)((c0 - g0) & 3);   // (c - g0) mod 4 is the same for all blocks
    const uint8_t *sb = (const uint8_t *)stage;
    for (uintptr_t c = c0 + 16 * (uintptr_t)tid; c < c0 + nblk; c += 16 * kBlock) {
        if (c >= g0 && c + 16 <= g1) {
            const long long so = (long long)(c - g0);          // stage byte offset of the block
            const uint32_t *w = stage + (so >> 2);
            u32x4 v;
            if (shift == 0) {
                v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
            } else {
                uint32_t a0 = w[0], a1 = w[1], a2 = w[2], a3 = w[3], a4 = w[4];
                v.x = __builtin_amdgcn_alignbyte(a1, a0, shift);
                v.y = __builtin_amdgcn_alignbyte(a2, a1, shift);
                v.z = __builtin_amdgcn_alignbyte(a3, a2, shift);
                v.w = __builtin_amdgcn_alignbyte(a4, a3, shift);
            }
            __builtin_nontemporal_store(v, (u32x4 *)c);
        } else {
            for (uintptr_t a = c; a < c + 16; a += kUnit) {
                if (a >= g0 && a < g1) {
                    const uintptr_t so = a - g0;
                    if (kUnit == 2)
                        *(uint16_t *)a = *(const uint16_t *)(sb + so);
                    else
                        *(uint8_t *)a = sb[so];
                }
            }
        }
    }
}

}  // namespace utfgpu
