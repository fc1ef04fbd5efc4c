// utf16_kernels.hip -- UTF-16LE validation, UTF-8 length and UTF-16LE ->
// UTF-8 conversion for gfx950 (wave64).
//
// Format (Lemire, "Unicode at Gigabytes per Second", Section 3): words
// outside D800..DFFF are characters by themselves; a high word D800..DBFF
// must be followed by a low word DC00..DFFF, and the pair stands for
// 0x10000 + ((high & 0x3FF) << 10 | (low & 0x3FF)).  Validation only has to
// look at surrogates.  UTF-8 output follows the byte-length ranges of the
// same section (1 byte up to U+7F, 2 up to U+7FF, 3 up to U+FFFF, 4 above).
//
// Positions here are 16-bit words.  A word's output width is 1, 2 or 3
// bytes, and 2 for each word of a surrogate pair: the high word writes the
// first two bytes of the four-byte sequence and the low word the last two,
// each inside its own slot, so no character's bytes cross a tile's range.
// The first error is the smallest word that is a high surrogate not
// followed by a low one, or a low surrogate not preceded by a high one; it
// depends only on the word and its two neighbours.
//
// Output.  A wave converts one row at a time into its LDS stage, laid out
// by 16-byte blocks of the output (the row's first byte at stage byte
// out & 15), then copies whole blocks out with aligned 16-byte stores.
// Every word stores three bytes at its offset (two in wave classes whose
// words take at most two), in word order, so the bytes past a shorter
// encoding are overwritten by the next word of the lane;
// only the first two bytes of a lane can keep stray bytes (from the
// previous lane's last word), and the lane rewrites them at the end.
#include "device_common.hpp"

namespace utfgpu {
namespace UTF_GEOM {

constexpr int kRowUnits = kRowBytes / 2;       // 512 words per row
constexpr int kWaveUnits = kWaveBytes / 2;     // 2048 words per wave
constexpr int kTileUnits = kTileBytes / 2;     // 32768 words per tile
// one row of output (at most 3 bytes per word) shifted by up to 15 bytes,
// plus the stray bytes past its end
constexpr int kStageBytes16 = 3 * kRowUnits + 32;
constexpr int kStageWords16 = kStageBytes16 / 4;   // a multiple of 4: stages stay 16-byte aligned
constexpr int kWriteIters16 = row_write_iters<3 * kRowUnits>();   // a row: at most three bytes per unit

// Wave classes by the words present: ASCII only; below 0x800; ASCII and
// surrogates only (e.g. English with emoji: two bytes per surrogate word);
// no surrogates; anything.
enum : uint32_t { kAscii16 = 0, kUpTo2B = 1, kQuad16 = 2, kBmp = 3, kAnyUnit = 4 };
__device__ __forceinline__ bool has_sur(uint32_t cls) { return cls == kQuad16 || cls == kAnyUnit; }

// Zero the words of the dword holding frame words p, p+1 that fall
// outside [lo, hi).
__device__ __forceinline__ uint32_t keep_units(uint32_t x, long long p, long long lo, long long hi) {
    const bool k0 = p >= lo && p < hi;
    const bool k1 = p + 1 >= lo && p + 1 < hi;
    return x & ((k0 ? 0x0000FFFFu : 0u) | (k1 ? 0xFFFF0000u : 0u));
}

// Per-lane view of one wave's span: kRows rows of eight words (zero
// outside the input), the dword before the wave (its high word is the word
// before) and the dword after it (its low word is the word after).
struct LaneUnits {
    uint32_t d[kRows][4];
    uint32_t hp, hn;
    bool edge;
};

__device__ __forceinline__ void load_span16(const uint8_t *frame, long long head, long long end, long long wbase,
                                            uint32_t lane, LaneUnits &t) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (q0 < end) v = __builtin_nontemporal_load((const u32x4 *)(frame + 2 * q0));
        t.d[r][0] = v.x; t.d[r][1] = v.y; t.d[r][2] = v.z; t.d[r][3] = v.w;
    }
    t.hp = 0;
    t.hn = 0;
    if (wbase - 2 >= 0 && wbase - 2 < end) t.hp = *(const uint32_t *)(frame + 2 * (wbase - 2));
    if (wbase + kWaveUnits < end) t.hn = *(const uint32_t *)(frame + 2 * (wbase + kWaveUnits));
    // the same dwords in every lane: scalar registers
    t.hp = __builtin_amdgcn_readfirstlane(keep_units(t.hp, wbase - 2, head, end));
    t.hn = __builtin_amdgcn_readfirstlane(keep_units(t.hn, wbase + kWaveUnits, head, end));
    t.edge = wbase < head || wbase + kWaveUnits > end;
    if (t.edge) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
#pragma unroll
            for (int k = 0; k < 4; ++k) t.d[r][k] = keep_units(t.d[r][k], q0 + 2 * k, head, end);
        }
    }
}

// An empty asm per data register: later code cannot reuse comparisons made
// on the words before this point, so their lane masks do not stay live.
__device__ __forceinline__ void fence_units(LaneUnits &t) {
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(t.d[r][k]));
}

// The word before / after the lane's chunk of row r.
__device__ __forceinline__ uint32_t prev_word(const LaneUnits &t, int r, uint32_t lane) {
    const uint32_t p = __shfl_up(t.d[r][3], 1);
    const uint32_t p0 = r == 0 ? t.hp : readlane(t.d[r - 1][3], kWave - 1);
    return (lane == 0 ? p0 : p) >> 16;
}
__device__ __forceinline__ uint32_t next_word(const LaneUnits &t, int r, uint32_t lane) {
    const uint32_t nx = __shfl_down(t.d[r][0], 1);
    const uint32_t n63 = r == kRows - 1 ? t.hn : readlane(t.d[r + 1][0], 0);
    return (lane == kWave - 1 ? n63 : nx) & 0xFFFFu;
}

__device__ __forceinline__ bool is_sur(uint32_t u) { return (u & 0xF800u) == 0xD800u; }
__device__ __forceinline__ bool is_high(uint32_t u) { return (u & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(uint32_t u) { return (u & 0xFC00u) == 0xDC00u; }

// UTF-8 bytes of one word (1 below 0x80, 2 below 0x800, 2 per surrogate
// word, 3 otherwise).
__device__ __forceinline__ uint32_t width8(uint32_t u) {
    return 1u + (u >= 0x80u) + (u >= 0x800u) - (uint32_t)is_sur(u);
}

__device__ __forceinline__ uint32_t chunk_width8(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3) {
    return width8(d0 & 0xFFFFu) + width8(d0 >> 16) + width8(d1 & 0xFFFFu) + width8(d1 >> 16) +
           width8(d2 & 0xFFFFu) + width8(d2 >> 16) + width8(d3 & 0xFFFFu) + width8(d3 >> 16);
}

// Words of the chunk at frame word q0 that lie outside [head, end).
__device__ __forceinline__ uint32_t outside_count8(long long q0, long long head, long long end) {
    const long long a = q0 < head ? head : q0;
    const long long b = q0 + 8 > end ? end : q0 + 8;
    const long long in = b > a ? b - a : 0;
    return (uint32_t)(8 - in);
}

__device__ __forceinline__ uint32_t load_chunk_width8(const uint8_t *frame, long long head, long long end,
                                                      long long q0) {
    if (q0 >= end) return 0;
    const u32x4 v = *(const u32x4 *)(frame + 2 * q0);
    uint32_t d[4] = {v.x, v.y, v.z, v.w};
    if (q0 < head || q0 + 8 > end)
        for (int k = 0; k < 4; ++k) d[k] = keep_units(d[k], q0 + 2 * k, head, end);
    return chunk_width8(d[0], d[1], d[2], d[3]) - outside_count8(q0, head, end);
}

// Aggregate (bytes) of tile `tl`, computed by one wave from global memory:
// used when the tile's own workgroup has not published it.
__device__ __noinline__ u64 tile_width8(const uint8_t *frame, long long head, long long end, long long tl) {
    const uint32_t lane = lane_id();
    u64 acc = 0;
    const long long base = tl * kTileUnits;
    for (int r = 0; r < kTileUnits / kRowUnits; ++r)
        acc += load_chunk_width8(frame, head, end, base + r * kRowUnits + 8 * (long long)lane);
    return wave_sum_u64(acc);
}

// Wave class and the output width (bytes) of each of the lane's rows.
template <bool kWidths>
__device__ __forceinline__ uint32_t survey16(const LaneUnits &t, long long wbase, long long head, long long end,
                                             uint32_t lane, uint32_t (&width)[kRows]) {
    uint32_t a80 = 0, a800 = 0;
    bool sur = false;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = t.d[r][k];
            a80 |= x & 0xFF80FF80u;
            a800 |= x & 0xF800F800u;
            sur = sur || is_sur(x & 0xFFFFu) || is_sur(x >> 16);
        }
    uint32_t cls = kAscii16;
    if (__ballot(sur)) cls = kAnyUnit;
    else if (__ballot(a800 != 0)) cls = kBmp;
    else if (__ballot(a80 != 0)) cls = kUpTo2B;
    if (!kWidths) return cls;
    bool other = false;   // a word >= 0x80 that is not a surrogate
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t w = 8;
        if (cls != kAscii16) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t u0 = t.d[r][k] & 0xFFFFu, u1 = t.d[r][k] >> 16;
                const bool g0 = u0 >= 0x80u, g1 = u1 >= 0x80u;
                w += g0 + g1;
                if (cls >= kBmp) w += (u0 >= 0x800u) + (u1 >= 0x800u);
                if (cls == kAnyUnit) {
                    const bool s0 = is_sur(u0), s1 = is_sur(u1);
                    w -= (uint32_t)s0 + (uint32_t)s1;
                    other = other || (g0 && !s0) || (g1 && !s1);
                }
            }
        }
        if (t.edge) w -= outside_count8(wbase + r * kRowUnits + 8 * (long long)lane, head, end);
        width[r] = w;
    }
    // ASCII and surrogates only: the same widths (two bytes a surrogate
    // word), a cheaper encoder
    if (cls == kAnyUnit && !__ballot(other)) cls = kQuad16;
    return cls;
}

// Whether the lane's words hold an unpaired surrogate: word tests on the
// words with their neighbours, no positions (words outside the input read as
// zero, which pairs with nothing, as the end of the input does).
__device__ __forceinline__ bool lane_has_unpaired(const LaneUnits &t, uint32_t lane) {
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t u[10];
        u[0] = prev_word(t, r, lane);
#pragma unroll
        for (int j = 0; j < 8; ++j) u[j + 1] = (t.d[r][j >> 1] >> (16 * (j & 1))) & 0xFC00u;
        u[9] = next_word(t, r, lane);
        u[0] &= 0xFC00u;
        u[9] &= 0xFC00u;
#pragma unroll
        for (int j = 1; j <= 8; ++j)
            bad |= (u[j] == 0xD800u && u[j + 1] != 0xDC00u) || (u[j] == 0xDC00u && u[j - 1] != 0xD800u);
    }
    return bad;
}

// First unpaired surrogate among the lane's words (position << 4 | kind).
__device__ __forceinline__ u64 lane_first_error16(const LaneUnits &t, long long wbase, long long head,
                                                  long long end, uint32_t lane) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t u[10];
        u[0] = prev_word(t, r, lane);
#pragma unroll
        for (int j = 0; j < 8; ++j) u[j + 1] = (t.d[r][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
        u[9] = next_word(t, r, lane);
        u64 err = ~0ull;
#pragma unroll
        for (int j = 7; j >= 0; --j) {   // backwards: the smallest position is kept
            const long long q = wbase + r * kRowUnits + 8 * (long long)lane + j;
            const uint32_t w = u[j + 1];
            const bool bad_hi = is_high(w) && !is_low(u[j + 2]);
            const bool bad_lo = is_low(w) && !is_high(u[j]);
            if ((bad_hi || bad_lo) && q >= head && q < end)
                err = ((u64)(q - head) << 4) | (bad_hi ? kUnpairedHigh : kUnpairedLow);
        }
        if (err != ~0ull) return err;
    }
    return ~0ull;
}

// ------------------------------------------------------------------------
// Batched calls: a string start ends the pairing (a high word before it and
// a low word at it are both unpaired).
// ------------------------------------------------------------------------
// Start bits of the lane's chunk of row r: bits 0..7 its words, bit 8 the
// word after.  The bitmap covers every tile of the call and 64 words past.
__device__ __forceinline__ uint32_t lane_starts16(const BatchCtx &bc, long long wbase, int r, uint32_t lane) {
    const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
    const long long e = q0 >> 4;
    const uint32_t v = (uint32_t)bc.starts[e] | ((uint32_t)bc.starts[e + 1] << 16);
    return (v >> (uint32_t)(q0 & 15)) & 0x1FFu;
}

// Unpaired words of the lane's chunk of row r as bits 0..7 (words outside
// the input read as zero and pair with nothing).
__device__ __forceinline__ uint32_t unpaired_bits(const LaneUnits &t, int r, uint32_t lane, uint32_t sbits) {
    uint32_t u[10];
    u[0] = prev_word(t, r, lane) & 0xFC00u;
#pragma unroll
    for (int j = 0; j < 8; ++j) u[j + 1] = (t.d[r][j >> 1] >> (16 * (j & 1))) & 0xFC00u;
    u[9] = next_word(t, r, lane) & 0xFC00u;
    uint32_t bad = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool at_start = (sbits >> j) & 1u, next_start = (sbits >> (j + 1)) & 1u;
        const bool bad_hi = u[j + 1] == 0xD800u && (u[j + 2] != 0xDC00u || next_start);
        const bool bad_lo = u[j + 1] == 0xDC00u && (u[j] != 0xD800u || at_start);
        bad |= (uint32_t)(bad_hi || bad_lo) << j;
    }
    return bad;
}

// Each string's first unpaired word among the lane's positions goes to that
// string's error word.
__device__ __forceinline__ void lane_errors_batch(const LaneUnits &t, long long wbase, long long head, long long end,
                                                  uint32_t lane, const BatchCtx &bc) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t sb = lane_starts16(bc, wbase, r, lane);
        uint32_t bad = unpaired_bits(t, r, lane, sb);
        const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
        // select among values, never index the lane's words by a runtime index
        // (that would keep them in memory instead of registers)
        const uint32_t a0 = t.d[r][0], a1 = t.d[r][1], a2 = t.d[r][2], a3 = t.d[r][3];
        int lastj = -100;
        while (bad) {
            const int j = __builtin_ctz(bad);
            bad &= bad - 1u;
            const long long q = q0 + j;
            if (q < head || q >= end) continue;
            // no string starts in (lastj, j]: the same string, already reported
            if (lastj > -100 && ((sb >> (lastj + 1)) & ((1u << (j - lastj)) - 1u)) == 0) continue;
            lastj = j;
            const uint32_t dw = (uint32_t)j >> 1;
            const uint32_t x = dw == 0 ? a0 : (dw == 1 ? a1 : (dw == 2 ? a2 : a3));
            const uint32_t w = (x >> (16 * (j & 1))) & 0xFFFFu;
            const long long pin = q - head;
            const u64 idx = owner_near(bc, wbase / kWaveUnits, pin);
            min_agent(bc.serr + idx,
                      ((u64)(pin - bc.offsets[idx]) << 4) | (is_high(w) ? kUnpairedHigh : kUnpairedLow));
        }
    }
}

// UTF-8 bytes of word u: b0, b1, b2 in output order (only the low byte of
// each is meaningful) and their number; `pv` is the word before (a low
// surrogate takes two bits from it).  No branches.
//
// A surrogate pair hi, lo encodes v = 0x10000 + ((hi & 0x3FF) << 10 |
// (lo & 0x3FF)) in four bytes.  Since the low 12 bits of 0x10000 are zero,
// v >> 12 = 0x10 + ((hi >> 2) & 0xFF): the high word alone gives the first
// two bytes, F0 | (v >> 18) and 80 | ((v >> 12) & 3F); the low word gives
// 80 | (hi & 3) << 4 | ((lo >> 6) & 0xF) and 80 | (lo & 3F).
template <uint32_t kClass>
__device__ __forceinline__ void encode_word(uint32_t u, uint32_t pv, uint32_t &b0, uint32_t &b1, uint32_t &b2,
                                            uint32_t &len) {
    const bool c1 = u >= 0x80u;
    const uint32_t t6 = u >> 6;
    const uint32_t last = (u & 0x3Fu) | 0x80u;            // last byte of a 2- or 3-byte sequence
    b2 = last;
    if (kClass == kQuad16 || kClass == kAnyUnit) {
        const uint32_t v12 = ((u >> 2) & 0xFFu) + 0x10u;
        const uint32_t h0 = (v12 >> 6) | 0xF0u, h1 = (v12 & 0x3Fu) | 0x80u;
        const uint32_t l0 = ((pv & 3u) << 4) | (t6 & 0xFu) | 0x80u;
        const bool hi = (u & 0xFC00u) == 0xD800u;
        const uint32_t s0 = hi ? h0 : l0, s1 = hi ? h1 : last;
        if (kClass == kQuad16) {   // a word >= 0x80 is a surrogate
            b0 = c1 ? s0 : u;
            b1 = s1;
            len = 1u + c1;
            return;
        }
        const bool c2 = u >= 0x800u, sur = (u & 0xF800u) == 0xD800u;
        b0 = c2 ? ((u >> 12) | 0xE0u) : (c1 ? (t6 | 0xC0u) : u);
        b1 = c2 ? ((t6 & 0x3Fu) | 0x80u) : last;
        b0 = sur ? s0 : b0;
        b1 = sur ? s1 : b1;
        len = sur ? 2u : 1u + c1 + c2;
        return;
    }
    b0 = c1 ? (t6 | 0xC0u) : u;                           // 2-byte lead (or the ASCII byte)
    b1 = last;
    if (kClass == kUpTo2B) {
        len = 1u + c1;
        return;
    }
    const bool c2 = u >= 0x800u;
    b0 = c2 ? ((u >> 12) | 0xE0u) : b0;
    b1 = c2 ? ((t6 & 0x3Fu) | 0x80u) : b1;
    len = 1u + c1 + c2;
}

// Word j of the lane's chunk of row r, with j = -1 the word before it.
__device__ __forceinline__ uint32_t word_of(const LaneUnits &t, int r, int j, uint32_t pv) {
    if (j < 0) return pv;
    return (t.d[r][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

// Encode the lane's chunk of row r into the stage at byte offset o, then
// rewrite the lane's first two bytes.  kEdge: the wave reaches outside the
// input, whose words encode to nothing.
template <uint32_t kClass, bool kEdge>
__device__ __forceinline__ void encode_row(const LaneUnits &t, int r, uint32_t o, uint8_t *st, long long wbase,
                                           long long head, long long end, uint32_t lane) {
    const uint32_t pv = has_sur(kClass) ? prev_word(t, r, lane) : 0u;
    uint32_t in = 0xFFu;   // words of the chunk inside the input
    if (kEdge) {
        const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
        in = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (q0 + j >= head && q0 + j < end) in |= 1u << j;
    }
    const uint32_t o0 = o;
    uint32_t ao = lds_addr(st) + o;   // LDS address of the word's first byte
    uint32_t first = 0, nfirst = 0;   // the lane's first two output bytes
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t b0, b1, b2, len;
        encode_word<kClass>(word_of(t, r, j, pv), word_of(t, r, j - 1, pv), b0, b1, b2, len);
        if (kEdge && !((in >> j) & 1u)) len = 0;
        *lptr<uint8_t>(ao) = (uint8_t)b0;
        *lptr<uint8_t>(ao + 1) = (uint8_t)b1;
        if (kClass != kUpTo2B && kClass != kQuad16) *lptr<uint8_t>(ao + 2) = (uint8_t)b2;   // at most two bytes a word there
        if (!kEdge) {
            if (j == 0) {
                first = (b0 & 0xFFu) | ((b1 & 0xFFu) << 8);
                nfirst = len;
            }
            if (j == 1 && nfirst == 1u) first = (first & 0xFFu) | ((b0 & 0xFFu) << 8);
        } else {
            const uint32_t bytes = (b0 & 0xFFu) | ((b1 & 0xFFu) << 8) | ((b2 & 0xFFu) << 16);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if ((uint32_t)k < len && nfirst < 2u) {
                    first |= ((bytes >> (8 * k)) & 0xFFu) << (8 * nfirst);
                    ++nfirst;
                }
            }
        }
        ao += len;
    }
    if (!kEdge) nfirst = 2;   // every word has at least one byte
    wave_lds_sync();          // every lane's stores land before the rewrite
    if (nfirst >= 1u) st[o0] = (uint8_t)first;
    if (nfirst >= 2u) st[o0 + 1] = (uint8_t)(first >> 8);
}

// All-ASCII rows: the low byte of every word.  With the row's first byte at
// stage byte s = 4a + b, lane L owns row bytes [8L, 8L+8) and stores the
// aligned stage dwords 2L + a and 2L + a + 1, which hold row bytes
// [8L - b, 8L - b + 8) (the last b of them from the previous lane).
__device__ __forceinline__ void narrow_row(const LaneUnits &t, int r, uint32_t s, uint32_t *st, uint32_t lane) {
    const uint32_t lo = __builtin_amdgcn_perm(t.d[r][1], t.d[r][0], 0x06040200u);
    const uint32_t hi = __builtin_amdgcn_perm(t.d[r][3], t.d[r][2], 0x06040200u);
    const uint32_t a = s >> 2, b = s & 3u;
    const uint32_t ph = __shfl_up(hi, 1);
    uint32_t *dst = st + 2 * lane + a;
    if (b == 0) {
        dst[0] = lo;
        dst[1] = hi;
    } else {
        dst[0] = __builtin_amdgcn_alignbyte(lo, ph, 4 - b);
        dst[1] = __builtin_amdgcn_alignbyte(hi, lo, 4 - b);
        if (lane == kWave - 1) dst[2] = __builtin_amdgcn_alignbyte(0u, hi, 4 - b);
    }
}

// All-ASCII waves away from the input's ends, with the whole wave's output
// inside the capacity: each lane's eight bytes of a row go straight from
// registers to memory.  With the wave's first output byte at g0 and
// s8 = g0 & 7 (wave-uniform), lane-row q = 64 r + L holds wave bytes
// [8q, 8q + 8) and stores the aligned 8-byte block at g0 - s8 + 8q, which
// holds wave bytes [8q - s8, 8q - s8 + 8): the last s8 bytes of lane-row
// q - 1 (the previous lane, or lane 63 of the previous row) and the first
// 8 - s8 of its own.  The partial blocks at the wave's two ends take byte
// stores, so no byte outside the wave's output is written.
__device__ __forceinline__ void narrow_store_wave(const LaneUnits &t, uint8_t *g0p, uint32_t lane) {
    const uintptr_t g0 = (uintptr_t)g0p;
    const uint32_t s8 = (uint32_t)(g0 & 7u);
    const uint32_t o = 8u - s8;   // the block's first byte in (previous lane-row, own lane-row)
    uint32_t rlo = 0, rhi = 0;    // lane 63's bytes of the previous row
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t lo = __builtin_amdgcn_perm(t.d[r][1], t.d[r][0], 0x06040200u);
        const uint32_t hi = __builtin_amdgcn_perm(t.d[r][3], t.d[r][2], 0x06040200u);
        const uint32_t q = 64u * (uint32_t)r + lane;
        if (s8 == 0) {
            *gptr<uint64_t>(g0 + 8u * q) = (uint64_t)hi << 32 | lo;
            continue;
        }
        uint32_t plo = __shfl_up(lo, 1), phi = __shfl_up(hi, 1);
        if (lane == 0) {
            plo = rlo;
            phi = rhi;
        }
        rlo = readlane(lo, kWave - 1);
        rhi = readlane(hi, kWave - 1);
        uint32_t a, b;
        if (o < 4u) {
            a = __builtin_amdgcn_alignbyte(phi, plo, o);
            b = __builtin_amdgcn_alignbyte(lo, phi, o);
        } else {
            a = __builtin_amdgcn_alignbyte(lo, phi, o - 4u);
            b = __builtin_amdgcn_alignbyte(hi, lo, o - 4u);
        }
        if (q > 0) {
            *gptr<uint64_t>(g0 - s8 + 8u * q) = (uint64_t)b << 32 | a;
        } else {   // head: wave bytes [0, o)
#pragma unroll
            for (uint32_t i = 0; i < 7u; ++i)
                if (i < o) *gptr<uint8_t>(g0 + i) = (uint8_t)((i < 4u ? lo >> (8 * i) : hi >> (8 * (i - 4u))) & 0xFFu);
        }
        if (r == kRows - 1 && lane == kWave - 1) {   // tail: own bytes [o, 8)
#pragma unroll
            for (uint32_t i = 1; i < 8u; ++i)
                if (i >= o)
                    *gptr<uint8_t>(g0 + 8u * q + i) = (uint8_t)((i < 4u ? lo >> (8 * i) : hi >> (8 * (i - 4u))) & 0xFFu);
        }
    }
}

// Batched calls keep each 32-word block's output offset inside its tile in
// 16 bits: a tile emits at most three bytes per word.
static_assert(3 * kTileUnits <= 65536, "16-bit block offsets");

template <bool kConvert, bool kBatch, bool kTicket>
// Six waves per SIMD (at most 80 VGPRs, so three 8-wave workgroups share a
// CU): the kernel waits on loads, barriers and the look-back more than it
// computes, and the third workgroup fills those waits.  It fits without
// spilling VGPRs to scratch because (a) the words pass through an empty asm
// after the survey and after the surrogate check, so the encoders cannot
// reuse those comparisons and keep their lane masks live, and (b) wave 0
// parks its words in LDS while it resolves the tile prefix.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void utf16_tile_kernel(
    const uint8_t *__restrict__ frame, long long head, long long m, uint8_t *__restrict__ out, u64 out_cap,
    u64 *__restrict__ status, Ctrl *__restrict__ ctrl, u64 ntiles, int spin_limit, BatchCtx bc) {
    static_assert(kConvert || !kTicket, "validation has no scan: tiles in block order");
    __shared__ __attribute__((aligned(16))) uint32_t stage[kConvert ? kWaves * kStageWords16 : 4];
    __shared__ uint32_t s_wave_tot[kWaves];
    __shared__ u64 s_prefix;
    __shared__ __attribute__((aligned(16))) uint32_t s_park[kConvert ? kRows * 4 * kWave : 4];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar branches on it
    __shared__ uint32_t s_ticket;
    const u64 tile = kTicket ? take_ticket(ctrl, &s_ticket, tid) : (u64)blockIdx.x;
    const long long end = head + m;
    const long long wbase = (long long)tile * kTileUnits + (long long)wave * kWaveUnits;

    LaneUnits t;
    load_span16(frame, head, end, wbase, lane, t);
    const u64 epoch = kConvert && wave == 0 ? ld_agent(&ctrl->epoch) : 0;   // only wave 0 looks back
    uint32_t width[kRows];
    uint32_t cls = survey16<kConvert>(t, wbase, head, end, lane, width);
    if (cls == kAscii16 && t.edge) cls = kUpTo2B;   // whole-chunk narrowing: not at the ends
    fence_units(t);

    // a wave holding an unpaired surrogate; when an error before it is
    // already known, its output (past the valid prefix) is not written and
    // its first error not located.  When converting, the check runs after
    // the wave total is published (while wave 0 resolves the tile prefix),
    // so it never delays the aggregate that later tiles wait for.
    auto find_unpaired = [&]() -> bool {
        bool lane_bad = false;
        if (has_sur(cls)) {
            if (kBatch) {
#pragma unroll
                for (int r = 0; r < kRows; ++r)
                    lane_bad |= unpaired_bits(t, r, lane, lane_starts16(bc, wbase, r, lane)) != 0;
            } else {
                lane_bad = lane_has_unpaired(t, lane);
            }
        }
        return has_sur(cls) && __ballot(lane_bad) != 0;
    };
    bool unpaired = kConvert ? false : find_unpaired();

    if (kConvert) {
        uint32_t off[kRows], rowbase[kRows + 1];
        rowbase[0] = 0;
#pragma unroll
        for (int p = 0; p < kRows / 2; ++p) {
            const uint32_t s0 = width[2 * p], s1 = width[2 * p + 1];
            const uint32_t inc = wave_incl_scan(s0 | (s1 << 16), lane);
            const uint32_t tot = readlane(inc, kWave - 1);
            off[2 * p] = (inc & 0xFFFFu) - s0;
            rowbase[2 * p + 1] = rowbase[2 * p] + (tot & 0xFFFFu);
            off[2 * p + 1] = (inc >> 16) - s1;
            rowbase[2 * p + 2] = rowbase[2 * p + 1] + (tot >> 16);
        }
        if (lane == 0) s_wave_tot[wave] = rowbase[kRows];
        __syncthreads();
        uint32_t wave_off = 0, tile_total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = s_wave_tot[w];
            if ((uint32_t)w < wave) wave_off += v;
            tile_total += v;
        }
        if (wave == 0) {
            // wave 0's words wait in LDS while it resolves the tile prefix:
            // the look-back's registers then fit beside the rest
            u32x4 *pk = (u32x4 *)s_park;
#pragma unroll
            for (int r = 0; r < kRows; ++r)
                pk[r * kWave + lane] = u32x4{t.d[r][0], t.d[r][1], t.d[r][2], t.d[r][3]};
            asm volatile("" ::: "memory");
            const u64 prefix = resolve_prefix(status, tile, epoch, spin_limit, tile_total, [=](long long tl) {
                return tile_width8(frame, head, end, tl);
            });
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const u32x4 v = pk[r * kWave + lane];
                t.d[r][0] = v.x; t.d[r][1] = v.y; t.d[r][2] = v.z; t.d[r][3] = v.w;
            }
            if (lane == 0) {
                s_prefix = prefix;
                if (tile == ntiles - 1) st_agent(&ctrl->total, prefix + tile_total);
                if (kBatch) bc.tilepre[tile] = prefix;
            }
        }
        if (kBatch && (lane & 3u) == 0) {   // in-tile output offset of every 32-word block
#pragma unroll
            for (int r = 0; r < kRows; ++r)
                bc.blockoff[(wbase + r * kRowUnits + 8 * (long long)lane) >> 5] =
                    (uint16_t)(wave_off + rowbase[r] + off[r]);
        }
        unpaired = find_unpaired();
        fence_units(t);
        __syncthreads();   // the tile prefix is known
        // an error before the wave is already known: its output lies past
        // the valid prefix and is not written (the error word is read only
        // now, off the path that publishes the tile's aggregate)
        const bool moot = !kBatch && unpaired && (long long)(ld_agent(&ctrl->err) >> 4) < wbase - head;
        uint32_t *wst = stage + wave * kStageWords16;
        uint8_t *wst8 = (uint8_t *)wst;
        const u64 base = s_prefix + wave_off;
        const uintptr_t wstart = (uintptr_t)(out + (base < out_cap ? base : out_cap));
        uintptr_t gend = wstart;   // end of the bytes written or carried so far
        Carry cy = {{0u, 0u, 0u, 0u}};
        const bool direct = cls == kAscii16 && base + kWaveUnits <= out_cap;
        if (direct) narrow_store_wave(t, out + base, lane);
#pragma unroll
        for (int r = 0; r < kRows && !moot && !direct; ++r) {
            const u64 b0 = base + rowbase[r];
            u64 b1 = base + rowbase[r + 1];
            if (b1 > out_cap) b1 = out_cap;
            if (b0 >= b1) continue;   // an empty row, or nothing of it fits
            const uintptr_t g0 = (uintptr_t)(out + b0), g1 = (uintptr_t)(out + b1);
            const uint32_t s = (uint32_t)(g0 & 15u);
            if (!t.edge) {
                switch (cls) {
                    case kAscii16: narrow_row(t, r, s, wst, lane); break;
                    case kUpTo2B: encode_row<kUpTo2B, false>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    case kQuad16: encode_row<kQuad16, false>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    case kBmp: encode_row<kBmp, false>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    default: encode_row<kAnyUnit, false>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                }
            } else {   // waves at the ends of the input (never all-ASCII)
                switch (cls) {
                    case kUpTo2B: encode_row<kUpTo2B, true>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    case kQuad16: encode_row<kQuad16, true>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    case kBmp: encode_row<kBmp, true>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                    default: encode_row<kAnyUnit, true>(t, r, s + off[r], wst8, wbase, head, end, lane); break;
                }
            }
            wave_lds_sync();
            write_row<1, kWriteIters16>(g0, g1, wstart, wst, lane, cy, gend > wstart);
            gend = g1;
            wave_lds_sync();
        }
        if (!moot && !direct) flush_carry<1>(gend, wstart, wst, cy, lane);
    }

    if (kBatch) {   // per string
        if (unpaired) lane_errors_batch(t, wbase, head, end, lane, bc);
        return;
    }
    // the first unpaired surrogate, unless an error before the wave is known
    if (unpaired && (long long)(ld_agent(&ctrl->err) >> 4) >= wbase - head) {
        u64 err = lane_first_error16(t, wbase, head, end, lane);
        err = wave_min_u64(err);
        if (lane == 0 && err != ~0ull) min_agent(&ctrl->err, err);
    }
}

__global__ __launch_bounds__(kBlock) void utf8_length_kernel(const uint8_t *__restrict__ frame, long long head,
                                                              long long m, u64 *__restrict__ partials) {
    __shared__ u64 s_sum[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const long long end = head + m;
    const long long nchunks = (end + 7) / 8;
    const long long stride = (long long)gridDim.x * kBlock;
    u64 acc = 0;
    for (long long c = (long long)blockIdx.x * kBlock + tid; c < nchunks; c += 4 * stride) {
        uint32_t w0 = load_chunk_width8(frame, head, end, 8 * c);
        uint32_t w1 = c + stride < nchunks ? load_chunk_width8(frame, head, end, 8 * (c + stride)) : 0;
        uint32_t w2 = c + 2 * stride < nchunks ? load_chunk_width8(frame, head, end, 8 * (c + 2 * stride)) : 0;
        uint32_t w3 = c + 3 * stride < nchunks ? load_chunk_width8(frame, head, end, 8 * (c + 3 * stride)) : 0;
        acc += (u64)w0 + w1 + w2 + w3;
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) s_sum[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        u64 b = 0;
        for (int w = 0; w < kWaves; ++w) b += s_sum[w];
        partials[blockIdx.x] = b;
    }
}

u64 utf16_tiles_for(long long head, long long m) { return (u64)((head + m + kTileUnits - 1) / kTileUnits); }

int partial_blocks(long long units, long long units_per_block);

hipError_t launch_utf16_tiles(bool convert, const uint8_t *frame, long long head, long long m, uint8_t *out,
                              u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, int schedule,
                              hipStream_t stream) {
    const u64 ntiles = utf16_tiles_for(head, m);
    const BatchCtx none = {nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (convert && schedule == kScheduleTicket)
        hipLaunchKernelGGL((utf16_tile_kernel<true, false, true>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    else if (convert)
        hipLaunchKernelGGL((utf16_tile_kernel<true, false, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    else   // no scan: the schedule does not apply
        hipLaunchKernelGGL((utf16_tile_kernel<false, false, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, result, nullptr, convert ? kFinConvert : kFinValidate, (u64)m, out_cap, nullptr,
                           0, stream);
}

// ------------------------------------------------------------------------
// Batched UTF-16LE -> UTF-8
// ------------------------------------------------------------------------
// Output offset (bytes) of input word p: the tile's offset, the offset of
// p's 32-word block inside the tile, and the widths of the block's words
// before p.
__device__ u64 batch_out_offset16(const uint8_t *frame, long long head, long long m, const BatchCtx &bc, u64 total,
                                  int64_t p) {
    if (p >= m) return total;
    const long long q = head + p;
    u64 w = bc.tilepre[q / kTileUnits] + bc.blockoff[q >> 5];
    for (long long c = q & ~31ll; c < q; c += 8) w += load_chunk_width8(frame, head, c + 8 < q ? c + 8 : q, c);
    return w;
}

// Per string: output offsets, result, and the reset of its error word and
// start bit for the next call.
__device__ __forceinline__ void post_string16(const BatchCtx &bc, long long m, int64_t *out_offsets,
                                              DevResult *results, u64 out_cap, bool ok, uint32_t *starts,
                                              long long head, u64 i, u64 oa, u64 ob) {
    const int64_t a = bc.offsets[i];
    out_offsets[i] = (int64_t)oa;
    if (i == bc.k) return;
    const int64_t b = bc.offsets[i + 1];
    if (a >= 0 && b > a && b <= m) {   // the start bit the prep kernel set for this string
        const u64 q = (u64)(head + a);
        atomicAnd(starts + (q >> 5), ~(1u << (q & 31u)));
    }
    const u64 e = bc.serr[i];
    bc.serr[i] = ~0ull;
    results[i].pad = 0;
    if (!ok) {
        results[i].status = kErrOffsets;
        results[i].count = 0;
        return;
    }
    if (e != ~0ull) {
        results[i].status = (int32_t)(e & 15u);
        results[i].count = e >> 4;
    } else {
        results[i].status = ob > out_cap ? (int32_t)kOutputTooSmall : (int32_t)kOk;
        results[i].count = ob - oa;
    }
}

// Thread i <= k: the output offset at offsets[i], shared through LDS (the
// workgroup's last thread also computes the one after its string); then
// string i's offsets and result, and the last workgroup to finish resets
// the control block for the next call.  kPostBlock threads per workgroup.
__global__ __launch_bounds__(kPostBlock) void batch_post16_kernel(const uint8_t *frame, long long head, long long m,
                                                                  BatchCtx bc, Ctrl *ctrl, int64_t *out_offsets,
                                                                  DevResult *results, u64 out_cap,
                                                                  const uint32_t *bad, uint32_t *starts) {
    __shared__ u64 s_off[kPostBlock + 1];
    const uint32_t tid = threadIdx.x;
    const u64 i = (u64)blockIdx.x * kPostBlock + tid;
    const bool ok = *bad == 0;
    const u64 total = ld_agent(&ctrl->total);
    if (i <= bc.k) {
        s_off[tid] = ok ? batch_out_offset16(frame, head, m, bc, total, bc.offsets[i]) : 0;
        if (tid == kPostBlock - 1 && i < bc.k)
            s_off[kPostBlock] = ok ? batch_out_offset16(frame, head, m, bc, total, bc.offsets[i + 1]) : 0;
    }
    __syncthreads();
    if (i <= bc.k)
        post_string16(bc, m, out_offsets, results, out_cap, ok, starts, head, i, s_off[tid],
                      i < bc.k ? s_off[tid + 1] : 0);
    batch_call_done(ctrl, tid);
}

hipError_t launch_batch_prep(const int64_t *offsets, u64 k, long long head, long long n, uint32_t *starts,
                             uint32_t *bad, long long span, uint32_t *wavestr, u64 nspans, hipStream_t stream);

hipError_t launch_utf16_batch(const uint8_t *frame, long long head, long long m, const int64_t *offsets, u64 k,
                              uint8_t *out, u64 out_cap, int64_t *out_offsets, DevResult *results, u64 *status,
                              Ctrl *ctrl, uint32_t *starts, uint16_t *blockoff,
                              u64 *tilepre, u64 *serr, uint32_t *bad, uint32_t *wavestr, int schedule,
                              hipStream_t stream) {
    const u64 ntiles = utf16_tiles_for(head, m);
    hipError_t e = launch_batch_prep(offsets, k, head, m, starts, bad, kWaveUnits, wavestr, ntiles * kWaves, stream);
    if (e != hipSuccess) return e;
    const BatchCtx bc = {offsets, k, (const uint16_t *)starts, blockoff, tilepre, serr, wavestr};
    if (m > 0 && schedule == kScheduleTicket)
        hipLaunchKernelGGL((utf16_tile_kernel<true, true, true>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), bc);
    else if (m > 0)
        hipLaunchKernelGGL((utf16_tile_kernel<true, true, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), bc);
    const unsigned pb = kPostBlock, pg = (unsigned)((k + 1 + pb - 1) / pb);
    hipLaunchKernelGGL(batch_post16_kernel, dim3(pg), dim3(pb), 0, stream, frame, head, m, bc, ctrl, out_offsets,
                       results, out_cap, (const uint32_t *)bad, starts);
    return hipGetLastError();
}

hipError_t launch_utf8_length(const uint8_t *frame, long long head, long long m, u64 *partials, Ctrl *ctrl,
                              u64 *result, hipStream_t stream) {
    const int nb = partial_blocks(head + m, 8LL * kBlock * 4);
    hipLaunchKernelGGL(utf8_length_kernel, dim3(nb), dim3(kBlock), 0, stream, frame, head, m, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, nullptr, result, kFinLength, 0, 0, partials, nb, stream);
}

}  // namespace UTF_GEOM
}  // namespace utfgpu
