// utf8_kernels.hip -- UTF-8 validation, UTF-16 length and UTF-8 -> UTF-16LE
// conversion for gfx950 (wave64).
//
// Format (Lemire, "Unicode at Gigabytes per Second", Section 3): leading
// bytes 0xxxxxxx / 110xxxxx / 1110xxxx / 11110xxx start sequences of 1..4
// bytes, continuation bytes are 10xxxxxx, the code point's high bits sit in
// the leading byte.  Validity: rules 1..6 of Section 3.  UTF-16 output: a
// value above U+FFFF becomes a high word D800 + (v-0x10000)>>10 followed by
// a low word DC00 + ((v-0x10000) & 0x3FF).
//
// First error.  The first invalid character starts at the smallest position
// i where a predicate C(i) over bytes i-3..i+3 holds (for a non-continuation
// byte: the character it announces breaks a rule; for a continuation byte:
// none of the three bytes before it announces a character that covers it).
// Every wave first runs a cheap detector -- must(t) != cont(t) with
// must(t) = [b(t-1) >= C0] | [b(t-2) >= E0] | [b(t-3) >= F0], plus the value
// rules checked on every decoded character -- and only a wave where it
// fires evaluates C exactly (over its positions and the three before).
// Both facts are checked on the CPU against the oracle by the test suite.
//
// Output offsets.  A non-continuation byte emits the character's UTF-16
// words: width 1, or 2 for a leading byte >= F0 (a surrogate pair).
// Continuation bytes emit nothing.  Offsets are the exclusive scan of those
// widths, so every tile knows where its output goes without seeing the
// characters of other tiles.
#include "device_common.hpp"

namespace utfgpu {

// Words a tile stage holds.  Valid input needs at most one word per byte of
// the tile plus one: a tile can end with the leading byte of a four-byte
// character (two words) whose continuation bytes lie in the next tile.
// Invalid input can announce up to two words per byte; then only the words
// of the valid prefix (which fit) are kept.
constexpr uint32_t kStageUnits = kTileBytes + 8;

// Byte class of a wave, over its own bytes and the three bytes before it.
enum : uint32_t { kAscii = 0, kUpTo2 = 1, kUpTo3 = 2, kAny = 3 };

// Frame byte q with positions outside [head, end) read as zero.
__device__ __forceinline__ uint32_t frame_byte(const uint8_t *frame, long long q, long long head, long long end) {
    return (q >= head && q < end) ? (uint32_t)frame[q] : 0u;
}

__device__ __forceinline__ bool is_cont(uint32_t b) { return (b & 0xC0u) == 0x80u; }

// Kind of the character announced at non-continuation byte q (0 if it is
// valid), in the order rule 1, rule 2, then rules 4, 5, 6.
__device__ uint32_t lead_kind(const uint8_t *frame, long long q, long long head, long long end) {
    const uint32_t b0 = frame_byte(frame, q, head, end);
    if (b0 < 0x80u) return kOk;
    if (b0 >= 0xF8u) return kHeaderBits;
    const int len = b0 < 0xE0u ? 2 : (b0 < 0xF0u ? 3 : 4);
    uint32_t cp = b0 & (0x7Fu >> len);
    for (int k = 1; k < len; ++k) {
        const uint32_t b = frame_byte(frame, q + k, head, end);
        if (!is_cont(b)) return kTooShort;
        cp = (cp << 6) | (b & 0x3Fu);
    }
    const uint32_t lo = len == 2 ? 0x80u : (len == 3 ? 0x800u : 0x10000u);
    if (cp < lo) return kOverlong;
    if (cp > 0x10FFFFu) return kTooLarge;
    if (cp >= 0xD800u && cp <= 0xDFFFu) return kSurrogate;
    return kOk;
}

// Exact C over frame positions [qlo, qhi): min (position << 4 | kind).
__device__ __noinline__ u64 exact_scan(const uint8_t *frame, long long head, long long end,
                                       long long qlo, long long qhi) {
    if (qlo < head) qlo = head;
    if (qhi > end) qhi = end;
    for (long long q = qlo; q < qhi; ++q) {
        const uint32_t b0 = frame_byte(frame, q, head, end);
        uint32_t kind = kOk;
        if (is_cont(b0)) {
            const uint32_t p1 = frame_byte(frame, q - 1, head, end);
            const uint32_t p2 = frame_byte(frame, q - 2, head, end);
            const uint32_t p3 = frame_byte(frame, q - 3, head, end);
            const bool covered = p1 >= 0xC0u || (p2 >= 0xE0u && is_cont(p1)) ||
                                 (p3 >= 0xF0u && is_cont(p2) && is_cont(p1));
            if (!covered) kind = kTooLong;
        } else {
            kind = lead_kind(frame, q, head, end);
        }
        if (kind != kOk) return ((u64)(q - head) << 4) | kind;
    }
    return ~0ull;
}

// Bit 7 of every byte: byte >= C0, >= E0, >= F0; continuation.
__device__ __forceinline__ uint32_t ge_c0(uint32_t x) { return x & (x << 1); }
__device__ __forceinline__ uint32_t ge_e0(uint32_t x) { return x & (x << 1) & (x << 2); }
__device__ __forceinline__ uint32_t ge_f0(uint32_t x) { return x & (x << 1) & (x << 2) & (x << 3); }
__device__ __forceinline__ uint32_t cont_bits(uint32_t x) { return x & ~(x << 1) & 0x80808080u; }

// Decode the character announced by the non-continuation byte at the low
// byte of `w4` (w4 holds bytes q..q+3).  Sets `bad` when a value rule (or
// rule 1) fails; the words are meaningful only for valid characters.
template <uint32_t kClass>
__device__ __forceinline__ void decode_char(uint32_t w4, uint32_t &u0, uint32_t &u1, uint32_t &two, bool &bad) {
    const uint32_t b = w4 & 0xFFu;
    if (kClass == kUpTo2) {
        const bool l2 = b >= 0xC0u;
        const uint32_t cp = l2 ? (((b & 0x1Fu) << 6) | ((w4 >> 8) & 0x3Fu)) : b;
        bad = l2 && cp < 0x80u;
        u0 = cp;
        u1 = 0;
        two = 0;
        return;
    }
    const uint32_t len = 1u + (b >= 0xC0u) + (b >= 0xE0u) + (b >= 0xF0u);
    const uint32_t c18 = (((w4 >> 8) & 0x3Fu) << 12) | (((w4 >> 16) & 0x3Fu) << 6) | ((w4 >> 24) & 0x3Fu);
    const uint32_t lp = b & (0x7Fu >> (len == 1u ? 0u : len));
    const uint32_t cp = ((lp << 18) | c18) >> (6u * (4u - len));
    const uint32_t lo = len == 1u ? 0u : (len == 2u ? 0x80u : (len == 3u ? 0x800u : 0x10000u));
    bad = (b >= 0xF8u) | (cp < lo) | (cp > 0x10FFFFu) | ((cp & 0xFFFFF800u) == 0xD800u);
    if (kClass == kUpTo3) {
        u0 = cp;
        u1 = 0;
        two = 0;
    } else {
        two = len == 4u;
        u0 = two ? 0xD7C0u + (cp >> 10) : cp;
        u1 = 0xDC00u | (cp & 0x3FFu);
    }
}

// Per-lane view of one tile: the rows of 16 bytes, and the dwords just
// before and after each row's chunk.
struct LaneBytes {
    uint32_t d[kRows][4];
    uint32_t prev[kRows];
    uint32_t next[kRows];
};

__device__ __forceinline__ void load_tile(const uint8_t *frame, long long head, long long end,
                                          long long wbase, uint32_t lane, LaneBytes &t) {
    const bool edge_wave = wbase < head || wbase + kWaveBytes > end;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (q0 < end) v = __builtin_nontemporal_load((const u32x4 *)(frame + q0));
        t.d[r][0] = v.x; t.d[r][1] = v.y; t.d[r][2] = v.z; t.d[r][3] = v.w;
        if (edge_wave && (q0 < head || q0 + 16 > end)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) t.d[r][k] = keep_range(t.d[r][k], q0 + 4 * k, head, end);
        }
    }
    // dwords adjacent to the wave's span
    uint32_t hp = 0, hn = 0;
    if (wbase - 4 >= 0 && wbase - 4 < end)
        hp = keep_range(*(const uint32_t *)(frame + wbase - 4), wbase - 4, head, end);
    if (wbase + kWaveBytes < end)
        hn = keep_range(*(const uint32_t *)(frame + wbase + kWaveBytes), wbase + kWaveBytes, head, end);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t p = __shfl_up(t.d[r][3], 1);
        uint32_t nx = __shfl_down(t.d[r][0], 1);
        const uint32_t p0 = r == 0 ? hp : readlane(t.d[r - 1][3], kWave - 1);
        const uint32_t n63 = r == kRows - 1 ? hn : readlane(t.d[r + 1][0], 0);
        t.prev[r] = lane == 0 ? p0 : p;
        t.next[r] = lane == kWave - 1 ? n63 : nx;
    }
}

__device__ __forceinline__ uint32_t wave_class(const LaneBytes &t, uint32_t lane) {
    uint32_t a80 = 0, aE0 = 0, aF0 = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = t.d[r][k];
            a80 |= x;
            aE0 |= ge_e0(x);
            aF0 |= ge_f0(x);
        }
    if (lane == 0) {   // the three bytes before the wave
        const uint32_t h = t.prev[0] & 0xFFFFFF00u;
        a80 |= h;
        aE0 |= ge_e0(h);
        aF0 |= ge_f0(h);
    }
    if (__ballot((aF0 & 0x80808080u) != 0)) return kAny;
    if (__ballot((aE0 & 0x80808080u) != 0)) return kUpTo3;
    if (__ballot((a80 & 0x80808080u) != 0)) return kUpTo2;
    return kAscii;
}

// Cheap detector over the lane's positions (bit 7 of each byte of the
// result marks must(t) != cont(t)).
template <uint32_t kClass>
__device__ __forceinline__ uint32_t mismatch_bits(const LaneBytes &t) {
    uint32_t mis = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t p = t.prev[r];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = t.d[r][k];
            uint32_t must = __builtin_amdgcn_alignbyte(ge_c0(x), ge_c0(p), 3);
            if (kClass >= kUpTo3) must |= __builtin_amdgcn_alignbyte(ge_e0(x), ge_e0(p), 2);
            if (kClass >= kAny) must |= __builtin_amdgcn_alignbyte(ge_f0(x), ge_f0(p), 1);
            mis |= (must & 0x80808080u) ^ cont_bits(x);
            p = x;
        }
    }
    return mis;
}

// Output width (UTF-16 words) of one 16-byte chunk: one per non-continuation
// byte, one more per byte >= F0.  Zero bytes outside the input count one
// each and are removed by the caller.
__device__ __forceinline__ uint32_t chunk_width16(const uint32_t (&d)[4]) {
    uint32_t w = 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) w = w - __popc(cont_bits(d[k])) + __popc(ge_f0(d[k]) & 0x80808080u);
    return w;
}

__device__ __forceinline__ uint32_t outside_count(long long q0, long long head, long long end) {
    long long a = q0 < head ? head : q0;
    long long b = q0 + 16 > end ? end : q0 + 16;
    long long in = b > a ? b - a : 0;
    return (uint32_t)(16 - in);
}

// Valid-position mask (bit k: position q0+k is an input byte).
__device__ __forceinline__ uint32_t valid_mask16(long long q0, long long head, long long end) {
    if (q0 >= head && q0 + 16 <= end) return 0xFFFFu;
    uint32_t m = 0;
    for (int k = 0; k < 16; ++k)
        if (q0 + k >= head && q0 + k < end) m |= 1u << k;
    return m;
}

// Decode a lane's chunks; write words to the tile stage (when kStore) at
// the tile-local offsets `off[r]`; return whether a value rule failed.
template <uint32_t kClass, bool kStore>
__device__ __forceinline__ bool decode_lane(const LaneBytes &t, const uint32_t (&off)[kRows],
                                            const uint32_t (&vm)[kRows], uint16_t *stage16) {
    bool anybad = false;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t o = off[r];
        const uint32_t cb[4] = {cont_bits(t.d[r][0]), cont_bits(t.d[r][1]), cont_bits(t.d[r][2]),
                                cont_bits(t.d[r][3])};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int dw = k >> 2, bk = k & 3;
            const bool lead = ((cb[dw] >> (8 * bk + 7)) & 1u) == 0u && ((vm[r] >> k) & 1u);
            if (lead) {
                const uint32_t lo = t.d[r][dw];
                const uint32_t hi = dw < 3 ? t.d[r][dw + 1] : t.next[r];
                const uint32_t w4 = window4(lo, hi, bk);
                uint32_t u0, u1, two;
                bool bad;
                decode_char<kClass>(w4, u0, u1, two, bad);
                anybad |= bad;
                if (kStore && o < kStageUnits) {
                    stage16[o] = (uint16_t)u0;
                    if (kClass == kAny && two && o + 1 < kStageUnits) stage16[o + 1] = (uint16_t)u1;
                }
                o += 1 + (kClass == kAny ? two : 0u);
            }
        }
    }
    return anybad;
}

// ASCII rows: every byte is one word (zero-extension).
__device__ __forceinline__ void widen_ascii(const LaneBytes &t, const uint32_t (&off)[kRows], uint16_t *stage16) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[2 * k] = __builtin_amdgcn_perm(0u, t.d[r][k], 0x0c010c00u);
            w[2 * k + 1] = __builtin_amdgcn_perm(0u, t.d[r][k], 0x0c030c02u);
        }
        const uint32_t o = off[r];
        if (o + 16u > kStageUnits) {
            // only reachable after invalid bytes earlier in the tile
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (o + 2 * k < kStageUnits) stage16[o + 2 * k] = (uint16_t)(w[k] & 0xFFFFu);
                if (o + 2 * k + 1 < kStageUnits) stage16[o + 2 * k + 1] = (uint16_t)(w[k] >> 16);
            }
        } else if ((o & 7u) == 0u) {
            u32x4 *dst = (u32x4 *)(stage16 + o);
            dst[0] = u32x4{w[0], w[1], w[2], w[3]};
            dst[1] = u32x4{w[4], w[5], w[6], w[7]};
        } else if ((o & 1u) == 0u) {
            uint32_t *dst = (uint32_t *)(stage16 + o);
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[k] = w[k];
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                stage16[o + 2 * k] = (uint16_t)(w[k] & 0xFFFFu);
                stage16[o + 2 * k + 1] = (uint16_t)(w[k] >> 16);
            }
        }
    }
}

// ------------------------------------------------------------------------
// Validation and conversion: one tile per workgroup.
// ------------------------------------------------------------------------
template <bool kConvert>
__global__ __launch_bounds__(kBlock) void utf8_tile_kernel(
    const uint8_t *__restrict__ frame, long long head, long long n, uint16_t *__restrict__ out,
    u64 out_cap, u64 *__restrict__ status, Ctrl *__restrict__ ctrl, DevResult *__restrict__ result,
    u64 ntiles) {
    constexpr int kStageWords = kConvert ? (kStageUnits / 2 + 4) : 2;   // dwords
    __shared__ uint32_t stage[kStageWords];
    __shared__ uint32_t s_wave_tot[kWaves];
    __shared__ u64 s_tile, s_epoch, s_prefix;
    __shared__ u64 s_err[kWaves];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid >> 6;
    if (tid == 0) {
        s_tile = add_agent(&ctrl->ticket, 1ull);
        s_epoch = ld_agent(&ctrl->epoch);
    }
    __syncthreads();
    const u64 tile = s_tile;
    const u64 epoch = s_epoch;
    const long long end = head + n;
    const long long wbase = (long long)tile * kTileBytes + (long long)wave * kWaveBytes;

    LaneBytes t;
    load_tile(frame, head, end, wbase, lane, t);
    uint32_t cls = wave_class(t, lane);
    // the all-ASCII shortcut writes whole chunks: not for waves at the ends
    if (cls == kAscii && (wbase < head || wbase + kWaveBytes > end)) cls = kUpTo2;

    // widths and in-wave offsets
    uint32_t s[kRows], vm[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
        vm[r] = valid_mask16(q0, head, end);
        s[r] = chunk_width16(t.d[r]) - outside_count(q0, head, end);
    }
    uint32_t off[kRows];
    uint32_t wave_total = 0;
    {
        const uint32_t i01 = wave_incl_scan(s[0] | (s[1] << 16), lane);
        const uint32_t i23 = wave_incl_scan(s[2] | (s[3] << 16), lane);
        const uint32_t t01 = readlane(i01, kWave - 1), t23 = readlane(i23, kWave - 1);
        const uint32_t tot[kRows] = {t01 & 0xFFFFu, t01 >> 16, t23 & 0xFFFFu, t23 >> 16};
        const uint32_t inc[kRows] = {i01 & 0xFFFFu, i01 >> 16, i23 & 0xFFFFu, i23 >> 16};
        uint32_t base = 0;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            off[r] = base + inc[r] - s[r];
            base += tot[r];
        }
        wave_total = base;
    }
    if (lane == 0) s_wave_tot[wave] = wave_total;
    __syncthreads();
    uint32_t wave_off = 0, tile_total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t v = s_wave_tot[w];
        if ((uint32_t)w < wave) wave_off += v;
        tile_total += v;
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) off[r] += wave_off;

    // publish the tile's aggregate early, then resolve its prefix
    if (kConvert && wave == 0) {
        u64 prefix = 0;
        if (tile == 0) {
            if (lane == 0) st_agent(status, pack_status(kFlagPrefix, epoch, tile_total));
        } else {
            if (lane == 0) st_agent(status + tile, pack_status(kFlagAggregate, epoch, tile_total));
            prefix = lookback(status, (long long)tile, epoch);
            if (lane == 0) st_agent(status + tile, pack_status(kFlagPrefix, epoch, prefix + tile_total));
        }
        if (lane == 0) {
            s_prefix = prefix;
            if (tile == ntiles - 1) st_agent(&ctrl->total, prefix + tile_total);
        }
    }

    // decode into the stage, detect errors
    uint16_t *stage16 = (uint16_t *)stage;
    bool flag = false;
    switch (cls) {
        case kAscii:
            if (kConvert) widen_ascii(t, off, stage16);
            break;
        case kUpTo2:
            flag = mismatch_bits<kUpTo2>(t) != 0;
            flag |= decode_lane<kUpTo2, kConvert>(t, off, vm, stage16);
            break;
        case kUpTo3:
            flag = mismatch_bits<kUpTo3>(t) != 0;
            flag |= decode_lane<kUpTo3, kConvert>(t, off, vm, stage16);
            break;
        default:
            flag = mismatch_bits<kAny>(t) != 0;
            flag |= decode_lane<kAny, kConvert>(t, off, vm, stage16);
            break;
    }
    u64 err = ~0ull;
    if (__ballot(flag)) {
        // exact first error over this lane's positions (and, for the first
        // lane, the three positions before the wave)
#pragma unroll 1
        for (int r = 0; r < kRows; ++r) {
            const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
            const long long lo = (r == 0 && lane == 0) ? q0 - 3 : q0;
            const u64 e = exact_scan(frame, head, end, lo, q0 + 16);
            if (e < err) err = e;
        }
        err = wave_min_u64(err);
    }
    if (lane == 0) s_err[wave] = err;
    __syncthreads();

    if (tid == 0) {
        u64 e = s_err[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) e = s_err[w] < e ? s_err[w] : e;
        if (e != ~0ull) min_agent(&ctrl->err, e);
    }
    if (kConvert) {
        const u64 prefix = s_prefix;
        u64 nunits = tile_total < kStageUnits ? tile_total : kStageUnits;
        if (prefix >= out_cap) nunits = 0;
        else if (prefix + nunits > out_cap) nunits = out_cap - prefix;
        write_out<2>((uint8_t *)(out + prefix), 2 * nunits, stage, tid);
    }
    if (tid == 0 && arrive_last(ctrl, ntiles)) {
        const u64 e = ld_agent(&ctrl->err);
        if (e != ~0ull) {
            write_result(result, (uint32_t)(e & 15u), e >> 4);
        } else if (kConvert) {
            const u64 tot = ld_agent(&ctrl->total);
            write_result(result, tot > out_cap ? kOutputTooSmall : kOk, tot);
        } else {
            write_result(result, kOk, (u64)n);
        }
        reset_ctrl(ctrl);
    }
}

// ------------------------------------------------------------------------
// UTF-16 length of UTF-8 (no validation): a plain reduction.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void utf16_length_kernel(
    const uint8_t *__restrict__ frame, long long head, long long n, Ctrl *__restrict__ ctrl,
    u64 *__restrict__ result, u64 nblocks) {
    __shared__ u64 s_sum[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const long long end = head + n;
    u64 acc = 0;
    const long long tbase = (long long)blockIdx.x * kTileBytes + (long long)wave * kWaveBytes;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = tbase + r * kRowBytes + 16 * (long long)lane;
        if (q0 < end) {
            u32x4 v = __builtin_nontemporal_load((const u32x4 *)(frame + q0));
            uint32_t d[4] = {v.x, v.y, v.z, v.w};
            if (q0 < head || q0 + 16 > end)
                for (int k = 0; k < 4; ++k) d[k] = keep_range(d[k], q0 + 4 * k, head, end);
            acc += chunk_width16(d) - outside_count(q0, head, end);
        }
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) s_sum[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        u64 b = 0;
        for (int w = 0; w < kWaves; ++w) b += s_sum[w];
        add_agent(&ctrl->total, b);
        if (arrive_last(ctrl, nblocks)) {
            *result = ld_agent(&ctrl->total);
            reset_ctrl(ctrl);
        }
    }
}

// ------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the C ABI layer).
// ------------------------------------------------------------------------
hipError_t launch_utf8_tiles(bool convert, const uint8_t *frame, long long head, long long n,
                             uint16_t *out, u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result,
                             u64 ntiles, hipStream_t stream) {
    if (convert)
        hipLaunchKernelGGL(utf8_tile_kernel<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, result, ntiles);
    else
        hipLaunchKernelGGL(utf8_tile_kernel<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, result, ntiles);
    return hipGetLastError();
}

hipError_t launch_utf16_length(const uint8_t *frame, long long head, long long n, Ctrl *ctrl, u64 *result,
                               hipStream_t stream) {
    const u64 nblocks = (u64)((head + n + kTileBytes - 1) / kTileBytes);
    hipLaunchKernelGGL(utf16_length_kernel, dim3((unsigned)nblocks), dim3(kBlock), 0, stream, frame, head, n,
                       ctrl, result, nblocks);
    return hipGetLastError();
}

}  // namespace utfgpu

namespace utfgpu {

// Results of empty inputs for the asynchronous calls (a kernel rather than
// a copy from host memory, so the call also works under stream capture).
__global__ void set_result_kernel(DevResult *r, int32_t status, u64 count) {
    if (threadIdx.x == 0) write_result(r, (uint32_t)status, count);
}
__global__ void set_u64_kernel(u64 *r, u64 v) {
    if (threadIdx.x == 0) *r = v;
}

hipError_t launch_set_result(DevResult *r, int32_t status, u64 count, hipStream_t stream) {
    hipLaunchKernelGGL(set_result_kernel, dim3(1), dim3(64), 0, stream, r, status, count);
    return hipGetLastError();
}
hipError_t launch_set_u64(u64 *r, u64 v, hipStream_t stream) {
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, stream, r, v);
    return hipGetLastError();
}

}  // namespace utfgpu
