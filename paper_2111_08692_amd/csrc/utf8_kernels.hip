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
// Output.  A non-continuation byte emits its character's UTF-16 words:
// width 1, or 2 for a leading byte >= F0 (a surrogate pair); continuation
// bytes emit nothing.  Offsets are the exclusive scan of those widths, so a
// tile places its output without seeing other tiles' characters.  A wave
// converts its span in groups of kGroup rows in two steps: every leading
// byte stores its four-byte window (itself and the next three bytes) in
// LDS at its output slot (a four-byte character also stores a marked copy
// for its low surrogate); then the lanes take aligned 16-byte blocks of the
// output, decode the eight windows of a block and store it whole.  Decoding
// work is thus spent per output word, not per input byte.
#include "device_common.hpp"

namespace utfgpu {
namespace UTF_GEOM {

// Byte class of a wave, over its own bytes and the three bytes before it.
// kQuad: leading bytes only below 0x80 or from F0 on (ASCII text with
// four-byte characters, e.g. emoji), a decode without the 2- and 3-byte forms.
enum : uint32_t { kAscii = 0, kUpTo2 = 1, kUpTo3 = 2, kQuad = 3, kAny = 4 };
// Classes whose waves can hold four-byte characters (two slots each).
constexpr bool has4(uint32_t cls) { return cls >= kQuad; }

// Slots one wave stages at a time (kGroup rows).  Valid input needs at most
// one slot per byte of the group plus one: a group can end with the leading
// byte of a four-byte character (two slots) whose continuation bytes lie
// beyond it.  Invalid input can announce up to two per byte; then only the
// slots of the valid prefix (which fit) are kept.  Decoded words are
// written over the windows, shifted by up to seven words.
constexpr uint32_t kStageSlots = kGroup * kRowBytes + 8;
constexpr int kStageWords = (int)kStageSlots + 8;   // one dword per slot, per wave
constexpr int kWriteIters = row_write_iters<2 * (int)kStageSlots>();   // a row: at most kStageSlots words

__device__ __forceinline__ bool is_cont(uint32_t b) { return (b & 0xC0u) == 0x80u; }

// Kind of the character announced at non-continuation byte b0 followed by
// b1, b2, b3 (0 if it is valid), in the order rule 1, rule 2, then rules
// 4, 5, 6.  Bytes past the end of the input read as zero.
__device__ __forceinline__ uint32_t lead_kind(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
    if (b0 < 0x80u) return kOk;
    if (b0 >= 0xF8u) return kHeaderBits;
    const int len = b0 < 0xE0u ? 2 : (b0 < 0xF0u ? 3 : 4);
    if (!is_cont(b1) || (len > 2 && !is_cont(b2)) || (len > 3 && !is_cont(b3))) return kTooShort;
    uint32_t cp = ((b0 & (0x7Fu >> len)) << 6) | (b1 & 0x3Fu);
    if (len > 2) cp = (cp << 6) | (b2 & 0x3Fu);
    if (len > 3) cp = (cp << 6) | (b3 & 0x3Fu);
    const uint32_t lo = len == 2 ? 0x80u : (len == 3 ? 0x800u : 0x10000u);
    if (cp < lo) return kOverlong;
    if (cp > 0x10FFFFu) return kTooLarge;
    if (cp >= 0xD800u && cp <= 0xDFFFu) return kSurrogate;
    return kOk;
}

// Bit 7 of every zero byte of t.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t t) {
    return ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
}

// Bit 7 of every byte: byte >= C0, >= E0, >= F0; continuation.
__device__ __forceinline__ uint32_t ge_c0(uint32_t x) { return x & (x << 1); }
__device__ __forceinline__ uint32_t ge_e0(uint32_t x) { return x & (x << 1) & (x << 2); }
__device__ __forceinline__ uint32_t ge_f0(uint32_t x) { return x & (x << 1) & (x << 2) & (x << 3); }
__device__ __forceinline__ uint32_t cont_bits(uint32_t x) { return x & ~(x << 1) & 0x80808080u; }

// Bit 7 of each byte of the dword at frame position p that lies outside
// [head, end).
__device__ __forceinline__ uint32_t outside_bits(long long p, long long head, long long end) {
    return ~keep_range(0x80808080u, p, head, end) & 0x80808080u;
}

// Per-lane view of one wave's span: kRows rows of 16 bytes (zero outside
// the input) and the dwords before the first and after the last chunk of
// the wave.  `edge` marks a wave that reaches outside the input.
struct LaneBytes {
    uint32_t d[kRows][4];
    uint32_t hp, hn;
    bool edge;
};

// Keeps the compiler from merging later recomputations of cheap bit tests
// with earlier ones (which would keep dozens of values alive in registers).
__device__ __forceinline__ void fence_values(LaneBytes &t) {
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(t.d[r][k]));
}

__device__ __forceinline__ uint32_t prev_dword(const LaneBytes &t, int r, uint32_t lane) {
    const uint32_t p = __shfl_up(t.d[r][3], 1);
    const uint32_t p0 = r == 0 ? t.hp : readlane(t.d[r - 1][3], kWave - 1);
    return lane == 0 ? p0 : p;
}
__device__ __forceinline__ uint32_t next_dword(const LaneBytes &t, int r, uint32_t lane) {
    const uint32_t nx = __shfl_down(t.d[r][0], 1);
    const uint32_t n63 = r == kRows - 1 ? t.hn : readlane(t.d[r + 1][0], 0);
    return lane == kWave - 1 ? n63 : nx;
}

// Issue the loads of a wave's span (rows and the two adjacent dwords).
__device__ __forceinline__ void issue_span(const uint8_t *frame, long long end, long long wbase, uint32_t lane,
                                           LaneBytes &t) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (q0 < end) v = __builtin_nontemporal_load((const u32x4 *)(frame + q0));
        t.d[r][0] = v.x; t.d[r][1] = v.y; t.d[r][2] = v.z; t.d[r][3] = v.w;
    }
    t.hp = 0;
    t.hn = 0;
    if (wbase - 4 >= 0 && wbase - 4 < end) t.hp = *(const uint32_t *)(frame + wbase - 4);
    if (wbase + kWaveBytes < end) t.hn = *(const uint32_t *)(frame + wbase + kWaveBytes);
}

// Zero everything outside [head, end) once the loads have arrived.
__device__ __forceinline__ void finish_span(long long head, long long end, long long wbase, uint32_t lane,
                                            LaneBytes &t) {
    // the same dwords in every lane: scalar registers
    t.hp = __builtin_amdgcn_readfirstlane(keep_range(t.hp, wbase - 4, head, end));
    t.hn = __builtin_amdgcn_readfirstlane(keep_range(t.hn, wbase + kWaveBytes, head, end));
    t.edge = wbase < head || wbase + kWaveBytes > end;
    if (t.edge) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
            if (q0 < head || q0 + 16 > end) {
#pragma unroll
                for (int k = 0; k < 4; ++k) t.d[r][k] = keep_range(t.d[r][k], q0 + 4 * k, head, end);
            }
        }
    }
}

// Positions of the 16-byte chunk at frame position q0 that lie outside
// [head, end).
__device__ __forceinline__ uint32_t outside_count16(long long q0, long long head, long long end) {
    const long long a = q0 < head ? head : q0;
    const long long b = q0 + 16 > end ? end : q0 + 16;
    return (uint32_t)(16 - (b > a ? b - a : 0));
}

// Continuation bits of dword k of row r, with positions outside the input
// marked as continuations (so they neither emit words nor count).  kEdge:
// whether the wave reaches outside the input (t.edge) is known at compile
// time (kInner, kEdgeWave) or tested per dword (kAnyWave).  The scatter
// steps of single-buffer calls are compiled for inner and edge waves
// apart, so the inner waves' code holds no branch per dword; the batched
// calls test it (compiled twice, they need more registers than the kernel
// has to spare).  The survey needs no such test (see survey_span).
enum : int { kInner = 0, kEdgeWave = 1, kAnyWave = 2 };
template <int kEdge>
__device__ __forceinline__ uint32_t lane_cont_bits(const LaneBytes &t, int r, int k, long long wbase,
                                                   long long head, long long end, uint32_t lane) {
    uint32_t cb = cont_bits(t.d[r][k]);
    if (kEdge == kEdgeWave || (kEdge == kAnyWave && t.edge))
        cb |= outside_bits(wbase + r * kRowBytes + 16 * (long long)lane + 4 * k, head, end);
    return cb;
}

// One pass over the lane's bytes: the wave's byte class (over its bytes
// and the three before it), each row's output width, and the cheap
// detector must(t) != cont(t).
struct Survey {
    uint32_t cls;
    bool mis;
    uint32_t width[kRows];
};

// Batched calls: string starts as bit 7 of each byte of a dword, from four
// bitmap bits (bit j for byte j).
__device__ __forceinline__ uint32_t spread4(uint32_t b) { return ((b & 15u) * 0x10204080u) & 0x80808080u; }

// Bitmap bits of string starts for the lane's chunk of row r: bits 16..31
// for the chunk's positions, bits 0..15 for the 16 positions before.  The
// bitmap covers every tile of the call and 64 positions past them.  Read
// row by row as the survey reaches it (holding every row's bits from the
// start of the kernel cost registers the batched kernel does not have).
__device__ __forceinline__ uint32_t row_start_bits(const BatchCtx &bc, long long wbase, int r, uint32_t lane) {
    const long long ci = (wbase >> 4) + lane + r * (kRowBytes / 16);   // chunk index
    return ((uint32_t)bc.starts[ci] << 16) | (ci >= 1 ? (uint32_t)bc.starts[ci - 1] : 0u);
}

// With kBatch, a string start acts as a buffer end for the detector: a
// leading byte before it announces nothing past it (such an announcement
// is flagged), and a continuation byte at it is covered by nothing.
template <bool kBatch>
__device__ __forceinline__ void survey_span(const LaneBytes &t, long long wbase, long long head, long long end,
                                            uint32_t lane, Survey &sv, const BatchCtx &bc) {
    uint32_t a80 = lane == 0 ? (t.hp & 0xFFFFFF00u) : 0u;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) a80 |= t.d[r][k];
    if (!__ballot((a80 & 0x80808080u) != 0)) {
        // all-ASCII wave (the three bytes before it included): one word per byte
        sv.cls = kAscii;
        sv.mis = false;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            uint32_t w = 16;
            if (t.edge)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    w -= __popc(outside_bits(wbase + r * kRowBytes + 16 * (long long)lane + 4 * k, head, end));
            sv.width[r] = w;
        }
        return;
    }
    uint32_t aE0 = lane == 0 ? ge_e0(t.hp & 0xFFFFFF00u) : 0u;
    uint32_t aF0 = lane == 0 ? ge_f0(t.hp & 0xFFFFFF00u) : 0u;
    uint32_t aMid = 0;   // own bytes C0..EF
    uint32_t mis = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = prev_dword(t, r, lane);
        uint32_t pc0 = ge_c0(p), pe0 = ge_e0(p), pf0 = ge_f0(p);
        const uint32_t sbr = kBatch ? row_start_bits(bc, wbase, r, lane) : 0u;
        uint32_t ps = kBatch ? spread4(sbr >> 12) : 0u;   // starts among the 4 positions before
        uint32_t w = 16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = t.d[r][k];
            const uint32_t c0 = ge_c0(x);
            const uint32_t e0 = c0 & (x << 2);
            const uint32_t f0 = e0 & (x << 3);
            const uint32_t m1 = __builtin_amdgcn_alignbyte(c0, pc0, 3), m2 = __builtin_amdgcn_alignbyte(e0, pe0, 2),
                           m3 = __builtin_amdgcn_alignbyte(f0, pf0, 1);
            const uint32_t cb = cont_bits(x);   // positions outside the input: below
            if (kBatch) {
                const uint32_t s0 = spread4(sbr >> (16 + 4 * k));     // start at t
                const uint32_t s1 = __builtin_amdgcn_alignbyte(s0, ps, 3);  // start at t-1
                const uint32_t s2 = __builtin_amdgcn_alignbyte(s0, ps, 2);  // start at t-2
                const uint32_t x01 = s0 | s1, x012 = x01 | s2;
                const uint32_t mi = (m1 & ~s0) | (m2 & ~x01) | (m3 & ~x012);   // announced within the string
                const uint32_t mc = (m1 & s0) | (m2 & x01) | (m3 & x012);      // announced past its end
                mis |= ((mi & 0x80808080u) ^ cont_bits(x)) | (mc & 0x80808080u);
                ps = s0;
            } else {
                mis |= ((m1 | m2 | m3) & 0x80808080u) ^ cont_bits(x);
            }
            aE0 |= e0;
            aF0 |= f0;
            aMid |= c0 & ~f0;
            w = w - __popc(cb) + __popc(f0 & 0x80808080u);
            pc0 = c0;
            pe0 = e0;
            pf0 = f0;
        }
        sv.width[r] = w;
    }
    // a wave at an end of the input: its positions outside the input hold
    // zero bytes (not continuations), which the rows above counted as
    // characters of one word; they emit nothing
    if (t.edge)
#pragma unroll
        for (int r = 0; r < kRows; ++r) sv.width[r] -= outside_count16(wbase + r * kRowBytes + 16 * (long long)lane, head, end);
    sv.mis = mis != 0;
    if (__ballot((aF0 & 0x80808080u) != 0))
        sv.cls = __ballot((aMid & 0x80808080u) != 0) ? kAny : kQuad;
    else
        sv.cls = __ballot((aE0 & 0x80808080u) != 0) ? kUpTo3 : kUpTo2;
}

// Output width (UTF-16 words) of one 16-byte chunk given its bytes and its
// continuation bits (positions outside the input marked as continuations):
// one per non-continuation byte, one more per byte >= F0.
__device__ __forceinline__ uint32_t chunk_width16(const uint32_t (&d)[4], const uint32_t (&cb)[4]) {
    uint32_t w = 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) w = w - __popc(cb[k]) + __popc(ge_f0(d[k]) & 0x80808080u);
    return w;
}

// Words of the 16-byte chunk at frame position q0 (loaded from memory).
__device__ __forceinline__ uint32_t load_chunk_width16(const uint8_t *frame, long long head, long long end,
                                                       long long q0) {
    if (q0 >= end) return 0;
    const u32x4 v = *(const u32x4 *)(frame + q0);
    uint32_t d[4] = {v.x, v.y, v.z, v.w}, cb[4];
    const bool edge = q0 < head || q0 + 16 > end;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (edge) d[k] = keep_range(d[k], q0 + 4 * k, head, end);
        cb[k] = cont_bits(d[k]) | (edge ? outside_bits(q0 + 4 * k, head, end) : 0u);
    }
    return chunk_width16(d, cb);
}

// Aggregate (words) of tile `tl`, computed by one wave from global memory:
// used when the tile's own workgroup has not published it.
__device__ __noinline__ u64 tile_width16(const uint8_t *frame, long long head, long long end, long long tl) {
    const uint32_t lane = lane_id();
    u64 acc = 0;
    const long long base = tl * kTileBytes;
    for (int r = 0; r < kTileBytes / kRowBytes; ++r)
        acc += load_chunk_width16(frame, head, end, base + r * kRowBytes + 16 * (long long)lane);
    return wave_sum_u64(acc);
}

// ------------------------------------------------------------------------
// Step 1: leading bytes store their windows at their output slots.
// ------------------------------------------------------------------------
// Every byte position of the chunk stores its window, in position order,
// at the slot of the next leading byte (its own slot if it is one); a
// continuation byte's window is thus overwritten by the leading byte that
// follows it in the same lane.  Only the first slot of the lane can keep a
// stray window (from the previous lane's trailing continuation bytes); the
// lane rewrites it at the end.  If the lane's first dword holds no leading
// byte the input is invalid there and every slot of the lane lies past the
// valid prefix, so nothing needs rewriting (waves at the ends of the input
// look for the first leading byte anywhere in the chunk).
//
// The window of a four-byte character's low surrogate is stored with its
// first byte xor 0x70, which maps F0..FF into the continuation range 80..8F
// -- a value no leading byte's window starts with.
//
// kFull (batched calls): an invalid string can end in the lane's first
// dword and a valid one start later in the chunk, so the first leading
// byte is looked for in the whole chunk.
template <uint32_t kClass, bool kFull, int kEdge>
__device__ __forceinline__ void scatter_row_at(const LaneBytes &t, int r, uint32_t gof, uint32_t *wst, long long wbase,
                                               long long head, long long end, uint32_t lane) {
    uint8_t *sb = (uint8_t *)wst;
    constexpr uint32_t kLast = 4u * (kStageSlots - 2);   // invalid input may announce more slots
    const uint32_t base = lds_addr(wst), last = base + kLast;
    uint32_t o = base + 4u * gof;   // LDS address of the slot
    const uint32_t nx_row = next_dword(t, r, lane);
    uint32_t lead0 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = t.d[r][j];
        const uint32_t nx = j < 3 ? t.d[r][j + 1] : nx_row;
        const uint32_t lead = ~lane_cont_bits<kEdge>(t, r, j, wbase, head, end, lane) & 0x80808080u;
        if (j == 0) lead0 = lead;
        const uint32_t f0 = has4(kClass) ? ge_f0(x) & 0x80808080u : 0u;
        // per byte position: 4 (one slot) past a leading byte and 4 more
        // past a byte >= F0; the marked copy's offset, 4 for a byte >= F0
        const uint32_t mark = f0 >> 5;
        const uint32_t step = (lead >> 5) + mark;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t win = window4(x, nx, k);
            const uint32_t a = has4(kClass) ? min(o, last) : o;
            // the marked copy goes to the next slot for a four-byte leading
            // byte, else to this slot, where the plain window replaces it
            if (has4(kClass)) *lptr<uint32_t>(add_byte(a, mark, k)) = win ^ 0x70u;
            *lptr<uint32_t>(a) = win;
            o = add_byte(o, step, k);
        }
    }
    // rewrite the first slot
    uint32_t win = 0;
    bool has = false;
    if (!kFull && (kEdge == kInner || (kEdge == kAnyWave && !t.edge))) {
        has = lead0 != 0;
        const uint32_t p = (uint32_t)__builtin_ctz(lead0 | 0x80000000u) >> 3;   // first leading byte
        win = __builtin_amdgcn_alignbyte(t.d[r][1], t.d[r][0], p);
    } else {
        uint32_t p = 16;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const uint32_t lead = ~lane_cont_bits<kEdge>(t, r, j, wbase, head, end, lane) & 0x80808080u;
            if (lead) p = 4 * j + ((uint32_t)__builtin_ctz(lead) >> 3);
        }
        has = p < 16;
        // select among computed windows, never among the bytes by index
        // (that would keep the bytes in memory instead of registers)
        const uint32_t j = p >> 2, sh = p & 3u;
        const uint32_t a0 = t.d[r][0], a1 = t.d[r][1], a2 = t.d[r][2], a3 = t.d[r][3];
        const uint32_t w0 = __builtin_amdgcn_alignbyte(a1, a0, sh), w1 = __builtin_amdgcn_alignbyte(a2, a1, sh),
                       w2 = __builtin_amdgcn_alignbyte(a3, a2, sh), w3 = __builtin_amdgcn_alignbyte(nx_row, a3, sh);
        win = j == 0 ? w0 : (j == 1 ? w1 : (j == 2 ? w2 : w3));
    }
    if (has) {
        const uint32_t a = has4(kClass) ? min(4u * gof, kLast) : 4u * gof;
        *(uint32_t *)(sb + a) = win;
    }
}
template <uint32_t kClass, bool kFull>
__device__ __forceinline__ void scatter_row(const LaneBytes &t, int r, uint32_t gof, uint32_t *wst, long long wbase,
                                            long long head, long long end, uint32_t lane) {
    if (kFull)
        scatter_row_at<kClass, kFull, kAnyWave>(t, r, gof, wst, wbase, head, end, lane);
    else if (t.edge)
        scatter_row_at<kClass, kFull, kEdgeWave>(t, r, gof, wst, wbase, head, end, lane);
    else
        scatter_row_at<kClass, kFull, kInner>(t, r, gof, wst, wbase, head, end, lane);
}

// ------------------------------------------------------------------------
// Step 2: decode windows into UTF-16 words.
// ------------------------------------------------------------------------
// Word of the window `w` (low byte = leading byte), without branches.
// `bad` is set when a value rule (or rule 1) fails for the character;
// structure (continuation bytes) is checked by the detector.
// Pins two values in registers where they are computed, so that later
// selects between them stay selects.
__device__ __forceinline__ void opaque(uint32_t &a, uint32_t &b) { asm volatile("" : "+v"(a), "+v"(b)); }

// The values of a window's character are sums of its bytes with fixed
// weights, which v_dot4_u32_u8 forms in one instruction (byte k of the
// weight word times byte k of the window, plus a 32-bit addend).  For a
// leading byte b0 and continuation bytes b1, b2, b3 (the marker bits of
// each byte are constants that the addends cancel):
//   two bytes    v2 = 64 b0 + b1 - 0x3080
//   three bytes  v3 = 64 v2 + b2 - 0x20080         = 4096 b0 + 64 b1 + b2 - 0xE2080
//   four bytes   v4 = 4096 v2 + 64 b2 + b3 - 0xC02080
//                   = 2^18 b0 + 4096 b1 + 64 b2 + b3 - 0x3C82080
// each exact (the code point) when the bytes form a character of that
// length.  A marked low-surrogate copy (first byte F0..F4 xor 0x70, i.e.
// 0x70 less) gives v4 smaller by 0x70 << 18, which leaves its low ten bits
// -- all the low surrogate needs -- unchanged.
constexpr uint32_t kWeights2 = 0x00000140u;   // bytes 0, 1 weighted 64, 1
constexpr uint32_t kWeights3 = 0x00010000u;   // byte 2
constexpr uint32_t kWeights4 = 0x01400000u;   // bytes 2, 3 weighted 64, 1

__device__ __forceinline__ uint32_t dot4(uint32_t w, uint32_t weights, uint32_t addend) {
    return __builtin_amdgcn_udot4(w, weights, addend, false);
}

template <uint32_t kClass>
__device__ __forceinline__ uint32_t decode_word(uint32_t w, bool &bad) {
    const uint32_t b0 = w & 0xFFu;
    uint32_t v2 = dot4(w, kWeights2, 0u - 0x3080u);
    if (kClass == kUpTo2) {
        opaque(v2, v2);
        bad |= (w & 0xFEu) == 0xC0u;                          // C0, C1: overlong
        return b0 >= 0xC0u ? v2 : b0;
    }
    if (kClass == kQuad) {   // ASCII, four-byte leading bytes and their marked copies
        const uint32_t v4 = dot4(w, kWeights4, (v2 << 12) - 0xC02080u);
        const bool l4 = b0 >= 0xF0u;
        // rule 1 (F8..FF) and F5..F7 land above U+10FFFF
        bad |= l4 & (v4 - 0x10000u > 0xFFFFFu);
        uint32_t hi = 0xD7C0u + (v4 >> 10), lo = 0xDC00u | (v4 & 0x3FFu);
        opaque(hi, lo);
        return b0 < 0x80u ? b0 : (l4 ? hi : lo);
    }
    uint32_t v3 = dot4(w, kWeights3, (v2 << 6) - 0x20080u);
    opaque(v2, v3);   // computed for every word: selects, not branches
    const bool l3 = b0 >= 0xE0u;
    // a three-byte value below U+0800 (top five bits 0) or a surrogate (11011)
    const bool b3 = __builtin_amdgcn_ubfe(0x08000001u, v3 >> 11, 1) != 0u;
    const uint32_t u = l3 ? v3 : (b0 >= 0xC0u ? v2 : b0);
    if (kClass == kUpTo3) {
        bad |= ((w & 0xFEu) == 0xC0u) | (l3 & b3);
        return u;
    }
    // kAny: four bytes too, and marked low-surrogate copies (80..8F)
    const uint32_t v4 = dot4(w, kWeights4, (v2 << 12) - 0xC02080u);
    const bool l4 = b0 >= 0xF0u;
    bad |= ((w & 0xFEu) == 0xC0u) | (l3 & !l4 & b3) | (l4 & (v4 - 0x10000u > 0xFFFFFu));
    uint32_t hi = 0xD7C0u + (v4 >> 10), lo = 0xDC00u | (v4 & 0x3FFu);
    opaque(hi, lo);
    return l4 ? hi : ((b0 & 0xC0u) == 0x80u ? lo : u);
}

// Group 0 decoded before the tile prefix (and so h) is known, by the waves
// that wait while wave 0 resolves it: each slot's word replaces its window.
// `place_slots` then moves the words to halfword h + s, as decode_slots
// would have stored them.
template <uint32_t kClass>
__device__ __forceinline__ bool decode_slots_early(uint32_t *wst, uint32_t nslots, uint32_t lane) {
    bool bad = false;
    for (uint32_t s = lane; s < nslots; s += kWave) wst[s] = decode_word<kClass>(wst[s], bad);
    return bad;
}

__device__ __forceinline__ void place_slots(uint32_t *wst, uint32_t nslots, uint32_t h, uint32_t lane) {
    constexpr int kU = 2;
    uint16_t *w16 = (uint16_t *)wst;
    for (uint32_t s0 = 0; s0 < nslots; s0 += kU * kWave) {
        uint32_t w[kU];
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            const uint32_t s = s0 + i * kWave + lane;
            w[i] = s < nslots ? wst[s] : 0x20u;   // the word decode_slots gives a slot past the group
        }
#pragma unroll
        for (int i = 0; i < kU; ++i) w16[h + s0 + i * kWave + lane] = (uint16_t)w[i];
    }
}

// Decode the group's slots [0, nslots) in place: slot s's word goes to
// halfword h + s of the stage (lane-strided, so consecutive lanes touch
// consecutive LDS banks).  A pass reads its windows before it writes, and
// its writes land below the windows of later passes.
template <uint32_t kClass>
__device__ __forceinline__ bool decode_slots(uint32_t *wst, uint32_t nslots, uint32_t h, uint32_t lane) {
    constexpr int kU = 2;   // a pass covers 128 slots: little waste on the last one
    uint16_t *w16 = (uint16_t *)wst;
    bool bad = false;
    for (uint32_t s0 = 0; s0 < nslots; s0 += kU * kWave) {
        uint32_t w[kU];
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            const uint32_t s = s0 + i * kWave + lane;
            w[i] = s < nslots ? wst[s] : 0x20u;
        }
        uint32_t u[kU];
#pragma unroll
        for (int i = 0; i < kU; ++i) u[i] = decode_word<kClass>(w[i], bad);
#pragma unroll
        for (int i = 0; i < kU; ++i) w16[h + s0 + i * kWave + lane] = (uint16_t)u[i];
    }
    return bad;
}

// ------------------------------------------------------------------------
// All-ASCII waves: every byte is one word, written straight from registers.
// ------------------------------------------------------------------------
// Bytes q..q+7 (0 < q < 8, wave-uniform) of the 16 bytes a0..a3.
__device__ __forceinline__ void bytes8(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t q,
                                       uint32_t &lo, uint32_t &hi) {
    const uint32_t sh = q & 3u;
    if (q < 4) {
        lo = __builtin_amdgcn_alignbyte(a1, a0, sh);
        hi = __builtin_amdgcn_alignbyte(a2, a1, sh);
    } else {
        lo = __builtin_amdgcn_alignbyte(a2, a1, sh);
        hi = __builtin_amdgcn_alignbyte(a3, a2, sh);
    }
}

__device__ __forceinline__ u32x4 widen8(uint32_t lo, uint32_t hi) {
    return u32x4{__builtin_amdgcn_perm(0u, lo, 0x0c010c00u), __builtin_amdgcn_perm(0u, lo, 0x0c030c02u),
                 __builtin_amdgcn_perm(0u, hi, 0x0c010c00u), __builtin_amdgcn_perm(0u, hi, 0x0c030c02u)};
}

// The wave's words [u0, u0 + kWaveBytes) of `out` (all inside the output
// capacity).  Lane L of row r holds words 1024 r + 16 L .. +16.  With the
// first word at byte s of a 16-byte block, lane L stores the block that
// starts 16 - s bytes into its 32 output bytes and the block that starts
// 32 - s bytes in (finished with the first bytes of the next lane); the
// part blocks at the two ends of the wave take 2-byte stores.  The stores
// are ordinary (cached) ones: each instruction covers every other 16-byte
// block, which the L2 merges into whole lines before they reach HBM.
__device__ __forceinline__ void widen_store_wave(const LaneBytes &t, uint16_t *out, u64 u0, uint32_t lane) {
    uint8_t *g0 = (uint8_t *)(out + u0);
    const uint32_t s = (uint32_t)((uintptr_t)g0 & 15u);   // even
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint8_t *g = g0 + 2 * kRowBytes * r + 32 * lane;
        const uint32_t *d = t.d[r];
        if (s == 0) {
            *(u32x4 *)g = widen8(d[0], d[1]);
            *(u32x4 *)(g + 16) = widen8(d[2], d[3]);
            continue;
        }
        const uint32_t q = 8u - s / 2u;   // first input byte of the block
        uint32_t n0 = __shfl_down(d[0], 1), n1 = __shfl_down(d[1], 1);
        if (r + 1 < kRows) {
            const uint32_t m0 = readlane(t.d[r + 1][0], 0), m1 = readlane(t.d[r + 1][1], 0);
            if (lane == kWave - 1) {
                n0 = m0;
                n1 = m1;
            }
        }
        uint32_t lo, hi;
        bytes8(d[0], d[1], d[2], d[3], q, lo, hi);
        *(u32x4 *)(g + 16 - s) = widen8(lo, hi);
        if (r + 1 < kRows || lane + 1 < kWave) {
            bytes8(d[2], d[3], n0, n1, q, lo, hi);
            *(u32x4 *)(g + 32 - s) = widen8(lo, hi);
        }
        if (r == 0 && lane == 0) {   // head: words 0 .. q-1
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if ((uint32_t)k < q) ((uint16_t *)g)[k] = (uint16_t)((d[k >> 2] >> (8 * (k & 3))) & 0xFFu);
        }
        if (r == kRows - 1 && lane == kWave - 1) {   // tail: words 16 - s/2 .. 15
#pragma unroll
            for (int k = 9; k < 16; ++k)
                if ((uint32_t)k >= 16u - s / 2u)
                    ((uint16_t *)g)[k] = (uint16_t)((d[k >> 2] >> (8 * (k & 3))) & 0xFFu);
        }
    }
}

// ------------------------------------------------------------------------
// Waves of 1- and 2-byte characters: words computed at every position
// ------------------------------------------------------------------------
// The word of the character that starts at a byte is the byte itself
// (ASCII), or for C0..DF its five payload bits above the next byte's six;
// SWAR computes it at all four positions of a dword as two packed 16-bit
// halves (even positions, odd positions).  Every position then stores its
// word, in position order, at the slot of the next leading byte -- the
// order rule of the window scatter above -- so no decode pass is needed.
__device__ __forceinline__ void words2(uint32_t x, uint32_t nx, uint32_t &ce, uint32_t &co) {
    const uint32_t c0 = ge_c0(x) & 0x80808080u;               // leading bytes C0..DF
    const uint32_t p = x & ~(c0 >> 1) & 0x7F7F7F7Fu;           // payload of a leading byte
    const uint32_t q = __builtin_amdgcn_alignbyte(nx, x, 1) & 0x3F3F3F3Fu;   // payload of the next byte
    const uint32_t m = (c0 << 1) - (c0 >> 7);                  // 0xFF for the bytes C0..DF
    const uint32_t se = sconst<0x0c020c00u>(), so = sconst<0x0c030c01u>();
    const uint32_t pe = __builtin_amdgcn_perm(0u, p, se), qe = __builtin_amdgcn_perm(0u, q, se);
    const uint32_t po = __builtin_amdgcn_perm(0u, p, so), qo = __builtin_amdgcn_perm(0u, q, so);
    const uint32_t me = __builtin_amdgcn_perm(0u, m, sconst<0x02020000u>()),
                   mo = __builtin_amdgcn_perm(0u, m, sconst<0x03030101u>());
    ce = (me & ((pe << 6) | qe)) | (~me & pe);
    co = (mo & ((po << 6) | qo)) | (~mo & po);
}

// ------------------------------------------------------------------------
// Validation only: value rules on every leading byte, from its byte and
// the next (SWAR over the dword x, with y = the bytes one position later).
// ------------------------------------------------------------------------
template <uint32_t kClass>
__device__ __forceinline__ uint32_t value_bits(uint32_t x, uint32_t y) {
    uint32_t bad = 0;
    if (kClass != kQuad) {   // kQuad waves hold no leading bytes C0..EF
        bad = zero_bytes((x & 0xFEFEFEFEu) ^ 0xC0C0C0C0u);                  // C0, C1
        if (kClass == kUpTo2) return bad;
        const uint32_t y5 = y << 2;                                          // bit 5 of the next byte
        bad |= zero_bytes(x ^ 0xE0E0E0E0u) & ~y5;                            // E0 80..9F: overlong
        bad |= zero_bytes(x ^ 0xEDEDEDEDu) & y5;                             // ED A0..BF: surrogate
        if (kClass == kUpTo3) return bad;
    }
    const uint32_t y54 = (y << 2) | (y << 3);                                // bit 5 or 4 of the next byte
    bad |= zero_bytes(x ^ 0xF0F0F0F0u) & ~y54;                               // F0 80..8F: overlong
    bad |= zero_bytes(x ^ 0xF4F4F4F4u) & y54;                                // F4 90..BF: too large
    bad |= ((x & 0x7F7F7F7Fu) + 0x0B0B0B0Bu) & x;                            // F5..FF
    return bad & 0x80808080u;
}

// Word at position k (0..3) of a dword from its packed halves.
__device__ __forceinline__ uint32_t word_at2(uint32_t ce, uint32_t co, uint32_t k) {
    return ((k & 1u) ? co : ce) >> (16 * (k >> 1));
}

// Bit 7 of every C0 / C1 byte (overlong two-byte leads).
__device__ __forceinline__ uint32_t overlong2_bits(uint32_t x) {
    return zero_bytes((x & 0xFEFEFEFEu) ^ 0xC0C0C0C0u);
}

// ------------------------------------------------------------------------
// Waves of ASCII and four-byte characters: words computed at every position
// ------------------------------------------------------------------------
// A four-byte character (leading byte A, continuation bytes B, C, D) becomes
// the high surrogate D7C0 + ((A & 07) << 8) + ((B & 3F) << 2) + ((C & 3F) >> 4)
// and the low surrogate DC00 + ((C & 0F) << 6) + (D & 3F).  In 16-bit
// arithmetic, whose wrap-around drops the marker bits of A, B and D:
//   high = A*256 + B*4 + (C >> 4) + E5B8,   low = (C & 0F)*64 + D + DB80.
// Two positions per register in 16-bit halves, as for the 2-byte class.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_h2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

template <uint32_t kSel, uint32_t kMaskSel>
__device__ __forceinline__ void words4_half(uint32_t x, uint32_t y, uint32_t z, uint32_t w, uint32_t mf,
                                            uint32_t &hw, uint32_t &lw) {
    const uint32_t sel = sconst<kSel>();
    const uint32_t a = __builtin_amdgcn_perm(0u, x, sel), b = __builtin_amdgcn_perm(0u, y, sel),
                   c = __builtin_amdgcn_perm(0u, z, sel), d = __builtin_amdgcn_perm(0u, w, sel);
    // multipliers from scalar registers: multiply-adds (v_pk_mad_u16) rather
    // than shifts and adds
    const u16x2 m256 = as_h2(sconst<0x01000100u>()), m4 = as_h2(sconst<0x00040004u>()),
                m64 = as_h2(sconst<0x00400040u>());
    const uint32_t hi = as_u32((as_h2(b) * m4 + (as_h2(a) * m256 + (as_h2(c) >> (unsigned short)4))) +
                               (unsigned short)0xE5B8);
    lw = as_u32((as_h2(c & 0x000F000Fu) * m64 + as_h2(d)) + (unsigned short)0xDB80);
    const uint32_t m = __builtin_amdgcn_perm(0u, mf, sconst<kMaskSel>());
    hw = (m & hi) | (~m & a);   // the byte itself at the other positions
}

// First words (he even positions, ho odd) and low surrogates (le, lo) of
// the four positions of dword x (next dword nx).
__device__ __forceinline__ void words4(uint32_t x, uint32_t nx, uint32_t &he, uint32_t &ho, uint32_t &le,
                                       uint32_t &lo) {
    const uint32_t y = __builtin_amdgcn_alignbyte(nx, x, 1), z = __builtin_amdgcn_alignbyte(nx, x, 2),
                   w = __builtin_amdgcn_alignbyte(nx, x, 3);
    const uint32_t f0 = ge_f0(x) & 0x80808080u;
    const uint32_t mf = (f0 << 1) - (f0 >> 7);   // 0xFF for the bytes >= F0
    words4_half<0x0c020c00u, 0x02020000u>(x, y, z, w, mf, he, le);
    words4_half<0x0c030c01u, 0x03030101u>(x, y, z, w, mf, ho, lo);
}

// Bits 0..3 from bit 7 of bytes 0..3.
__device__ __forceinline__ uint32_t nibble_of(uint32_t m) {
    m >>= 7;
    return (m | (m >> 7) | (m >> 14) | (m >> 21)) & 15u;
}

// Value rules of the leading bytes of every row (kQuad waves): run by
// the waves that wait while wave 0 resolves the tile prefix, so their
// staging after it skips them.
__device__ __forceinline__ bool quad_values_bad(const LaneBytes &t, uint32_t lane) {
    uint32_t bad = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t nx_row = next_dword(t, r, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = t.d[r][j], nx = j < 3 ? t.d[r][j + 1] : nx_row;
            bad |= value_bits<kQuad>(x, __builtin_amdgcn_alignbyte(nx, x, 1));
        }
    }
    return bad != 0;
}

// Stage the lane's chunk of row r (a wave away from the input's ends):
// every position stores its first word at halfword o + slot and its low
// surrogate one halfword further, in position order.  The last positions
// of a lane may leave stray words in the next lane's first two slots; each
// lane rewrites its own first two slots at the end: the first character's
// first word, then its low surrogate or the second character's word.
// Returns whether a value rule failed.
__device__ __forceinline__ bool scatter_quad(const LaneBytes &t, int r, uint32_t o, uint32_t *wst, uint32_t lane,
                                             bool vals) {
    uint16_t *st16 = (uint16_t *)wst;
    const uint32_t nx_row = next_dword(t, r, lane);
    const uint32_t o0 = o;
    uint32_t ob = lds_addr(wst) + 2u * o;   // LDS address of the slot
    uint32_t bad = 0, h0e = 0, h0o = 0, l0e = 0, l0o = 0, h1e = 0, h1o = 0, L = 0, F = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = t.d[r][j];
        const uint32_t nx = j < 3 ? t.d[r][j + 1] : nx_row;
        const uint32_t lead = ~cont_bits(x) & 0x80808080u;
        const uint32_t f0 = ge_f0(x) & 0x80808080u;
        uint32_t he, ho, le, lo;
        words4(x, nx, he, ho, le, lo);
        if (vals) bad |= value_bits<kQuad>(x, __builtin_amdgcn_alignbyte(nx, x, 1));
        if (j == 0) {
            h0e = he; h0o = ho; l0e = le; l0o = lo;
            L = nibble_of(lead);
            F = nibble_of(f0);
        } else if (j == 1) {
            h1e = he; h1o = ho;
            L |= nibble_of(lead) << 4;
        }
        // per byte position: 2 past a leading byte, 2 more past a byte >= F0
        const uint32_t step = (lead >> 6) + (f0 >> 6);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            *lptr<uint16_t>(ob) = (uint16_t)word_at2(he, ho, (uint32_t)k);
            *lptr<uint16_t>(ob + 2) = (uint16_t)word_at2(le, lo, (uint32_t)k);
            ob = add_byte(ob, step, k);
        }
    }
    // a first dword without a leading byte is invalid input: every slot of
    // the lane then lies past the valid prefix
    if (L & 15u) {
        const uint32_t p1 = (uint32_t)__builtin_ctz(L);
        st16[o0] = (uint16_t)word_at2(h0e, h0o, p1);
        const uint32_t rest = L & (L - 1u);
        if ((F >> p1) & 1u) {
            st16[o0 + 1] = (uint16_t)word_at2(l0e, l0o, p1);
        } else if (rest) {   // valid input has its second leading byte right after a one-byte first
            const uint32_t p2 = (uint32_t)__builtin_ctz(rest);
            st16[o0 + 1] = (uint16_t)(p2 < 4 ? word_at2(h0e, h0o, p2) : word_at2(h1e, h1o, p2 - 4));
        }
    }
    return bad != 0;
}

// Words of the dword x (next dword nx) for a wave of class kClass, and
// the value rules of its leading bytes.
template <uint32_t kClass>
__device__ __forceinline__ uint32_t class_words(uint32_t x, uint32_t nx, uint32_t &ce, uint32_t &co) {
    static_assert(kClass == kUpTo2, "words computed in registers: 1- and 2-byte classes");
    words2(x, nx, ce, co);
    return overlong2_bits(x);
}

// Stage the lane's chunk of row r: words at halfword o + slot.  Returns
// whether a value rule failed.  kFull as for scatter_row.
template <uint32_t kClass, bool kFull, int kEdge>
__device__ __forceinline__ bool scatter_words_at(const LaneBytes &t, int r, uint32_t o, uint32_t *wst, long long wbase,
                                                  long long head, long long end, uint32_t lane) {
    uint16_t *st16 = (uint16_t *)wst;
    const uint32_t nx_row = next_dword(t, r, lane);
    const uint32_t o0 = o;
    uint32_t ob = lds_addr(wst) + 2u * o;   // LDS address of the slot
    uint32_t bad = 0, ce0 = 0, co0 = 0, lead0 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = t.d[r][j];
        const uint32_t nx = j < 3 ? t.d[r][j + 1] : nx_row;
        const uint32_t lead = ~lane_cont_bits<kEdge>(t, r, j, wbase, head, end, lane) & 0x80808080u;
        uint32_t ce, co;
        bad |= class_words<kClass>(x, nx, ce, co);
        if (j == 0) {
            ce0 = ce;
            co0 = co;
            lead0 = lead;
        }
        const uint32_t step = lead >> 6;   // per byte position: 2 past a leading byte
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            *lptr<uint16_t>(ob) = (uint16_t)word_at2(ce, co, (uint32_t)k);
            ob = add_byte(ob, step, k);
        }
    }
    // rewrite the first slot (see scatter_row)
    uint32_t v = 0;
    bool has;
    if (!kFull && (kEdge == kInner || (kEdge == kAnyWave && !t.edge))) {
        has = lead0 != 0;
        v = word_at2(ce0, co0, (uint32_t)__builtin_ctz(lead0 | 0x80000000u) >> 3);
    } else {
        uint32_t p = 16;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const uint32_t lead = ~lane_cont_bits<kEdge>(t, r, j, wbase, head, end, lane) & 0x80808080u;
            if (lead) p = 4 * j + ((uint32_t)__builtin_ctz(lead) >> 3);
        }
        has = p < 16;
        const uint32_t j = p >> 2;
        const uint32_t a0 = t.d[r][0], a1 = t.d[r][1], a2 = t.d[r][2], a3 = t.d[r][3];
        const uint32_t x = j == 0 ? a0 : (j == 1 ? a1 : (j == 2 ? a2 : a3));
        const uint32_t y = j == 0 ? a1 : (j == 1 ? a2 : (j == 2 ? a3 : nx_row));
        uint32_t ce, co;
        class_words<kClass>(x, y, ce, co);
        v = word_at2(ce, co, p & 3u);
    }
    if (has) st16[o0] = (uint16_t)v;
    return bad != 0;
}
template <uint32_t kClass, bool kFull>
__device__ __forceinline__ bool scatter_words(const LaneBytes &t, int r, uint32_t o, uint32_t *wst, long long wbase,
                                               long long head, long long end, uint32_t lane) {
    if (kFull) return scatter_words_at<kClass, kFull, kAnyWave>(t, r, o, wst, wbase, head, end, lane);
    return t.edge ? scatter_words_at<kClass, kFull, kEdgeWave>(t, r, o, wst, wbase, head, end, lane)
                  : scatter_words_at<kClass, kFull, kInner>(t, r, o, wst, wbase, head, end, lane);
}

// Words of a wave's leading bytes stored one by one at their slots (`slot`:
// the output word of the lane's chunk of each row), from bytes reloaded
// from memory: the fallback for groups whose slots do not fit the stage,
// which only invalid input produces.  A valid character gets its exact
// words; an invalid one gets some words of its own width.
__device__ __noinline__ void direct_words(const uint8_t *frame, long long head, long long end, long long wbase,
                                          uint32_t lane, u64 s0, u64 s1, u64 s2, u64 s3, uint16_t *out,
                                          u64 out_cap) {
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
        u64 o = r == 0 ? s0 : (r == 1 ? s1 : (r == 2 ? s2 : s3));
        uint32_t b[19];
        for (int i = 0; i < 19; ++i) {
            const long long q = q0 + i;
            b[i] = (q >= head && q < end) ? frame[q] : 0u;
        }
        for (int i = 0; i < 16; ++i) {
            const long long q = q0 + i;
            const uint32_t b0 = b[i], b1 = b[i + 1] & 0x3Fu, b2 = b[i + 2] & 0x3Fu, b3 = b[i + 3] & 0x3Fu;
            if (q < head || q >= end || is_cont(b0)) continue;
            uint32_t w0, w1 = 0;
            bool two = false;
            if (b0 < 0x80u) {
                w0 = b0;
            } else if (b0 < 0xE0u) {
                w0 = ((b0 & 0x1Fu) << 6) | b1;
            } else if (b0 < 0xF0u) {
                w0 = ((b0 & 0x0Fu) << 12) | (b1 << 6) | b2;
            } else {
                const uint32_t cp = ((b0 & 0x07u) << 18) | (b1 << 12) | (b2 << 6) | b3;
                w0 = 0xD7C0u + (cp >> 10);
                w1 = 0xDC00u | (cp & 0x3FFu);
                two = true;
            }
            if (o < out_cap) out[o] = (uint16_t)w0;
            if (two && o + 1 < out_cap) out[o + 1] = (uint16_t)w1;
            o += two ? 2 : 1;
        }
    }
}

// The wave's conversion after the tile prefix is known.  `staged0`: group
// 0 has been staged already.  Returns whether a value rule failed.  Rows
// are written with their unfinished last block carried to the next row.
template <uint32_t kClass, bool kFull>
__device__ __forceinline__ bool convert_wave(const LaneBytes &t, const uint32_t (&gof)[kRows],
                                             const uint32_t (&rowbase)[kRows + 1], u64 base, uint16_t *out,
                                             u64 out_cap, uint32_t *wst, long long wbase, long long head,
                                             long long end, uint32_t lane, bool staged0, bool vals = true,
                                             bool decoded0 = false) {
    bool bad = false;
    uintptr_t wlo = (uintptr_t)(out + (base < out_cap ? base : out_cap));   // lowest byte this wave writes
    uintptr_t gend = wlo;                                                  // end of the bytes done so far
    Carry cy = {{0u, 0u, 0u, 0u}};
#pragma unroll
    for (int g = 0; g < kRows / kGroup; ++g) {
        const u64 u0 = base + rowbase[g * kGroup];
        uint32_t nslots = rowbase[(g + 1) * kGroup] - rowbase[g * kGroup];
        if (nslots > kStageSlots) nslots = kStageSlots;   // only past an error
        u64 u1 = u0 + nslots;
        if (u1 > out_cap) u1 = out_cap;
        const uintptr_t g0 = (uintptr_t)(out + u0), g1 = (uintptr_t)(out + u1);
        if (u0 < u1 && gend != g0) {   // a row cut short before (past an error): finish its block
            flush_carry<2>(gend, wlo, wst, cy, lane);
            wlo = gend;
        }
        const uint32_t h = (uint32_t)(((uintptr_t)(out + u0) >> 1) & 7u);
        if constexpr (kClass == kUpTo2) {   // words straight from the bytes
#pragma unroll
            for (int r = g * kGroup; r < (g + 1) * kGroup; ++r)
                bad |= scatter_words<kClass, kFull>(t, r, h + gof[r], wst, wbase, head, end, lane);
        } else if (kClass == kQuad && !kFull && !t.edge) {
#pragma unroll
            for (int r = g * kGroup; r < (g + 1) * kGroup; ++r) bad |= scatter_quad(t, r, h + gof[r], wst, lane, vals);
        } else {
            if (g > 0 || !staged0)
#pragma unroll
                for (int r = g * kGroup; r < (g + 1) * kGroup; ++r)
                    scatter_row<kClass, kFull>(t, r, gof[r], wst, wbase, head, end, lane);
            wave_lds_sync();
            if (g == 0 && decoded0)
                place_slots(wst, nslots, h, lane);
            else
                bad |= decode_slots<kClass>(wst, nslots, h, lane);   // value rules: even for rows not written
        }
        if (u0 < u1) {
            wave_lds_sync();
            write_row<2, kWriteIters>(g0, g1, wlo, wst, lane, cy, gend == g0 && gend > wlo);
            gend = g1;
        }
        wave_lds_sync();
    }
    flush_carry<2>(gend, wlo, wst, cy, lane);
    return bad;
}

// ------------------------------------------------------------------------
// Exact first error of a lane's chunk (flagged waves only)
// ------------------------------------------------------------------------
// With the bytes in registers -- v = {dword before the chunk, the chunk's
// four dwords, dword after it} -- the smallest position of C is the first
// byte flagged by any of: a continuation byte that no byte in reach
// announces (cont and not must), a leading byte whose announced
// continuation bytes are not all there, a leading byte whose value rules
// fail (from it and the next byte).  Each flag implies C at its position,
// and the first position of C carries one of them, so the first flag is
// the first error.  With `halo`, the leading bytes among the three
// positions before the chunk are examined too (a continuation byte there
// belongs to the previous wave, whose detector fires at it when it is the
// first error).  Returns min (position << 4 | kind) or ~0.  Kept small: it
// runs in few waves, usually with its code not in the instruction cache.
__device__ __noinline__ u64 exact_chunk(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3, uint32_t v4,
                                        uint32_t v5, long long q0, long long head, bool halo) {
    const uint32_t v[6] = {v0, v1, v2, v3, v4, v5};
    uint32_t first = 32;   // byte index into v (chunk position + 4)
#pragma unroll
    for (int i = 4; i >= 0; --i) {   // backwards: the smallest index is kept
        const uint32_t x = v[i], xn = v[i + 1], xp = i > 0 ? v[i - 1] : 0u;
        const uint32_t c0 = ge_c0(x), e0 = ge_e0(x), f0 = ge_f0(x);
        const uint32_t shortb = (c0 & ~cont_bits(__builtin_amdgcn_alignbyte(xn, x, 1))) |
                                (e0 & ~cont_bits(__builtin_amdgcn_alignbyte(xn, x, 2))) |
                                (f0 & ~cont_bits(__builtin_amdgcn_alignbyte(xn, x, 3)));
        const uint32_t lead_bad = (shortb | value_bits<kAny>(x, __builtin_amdgcn_alignbyte(xn, x, 1))) & 0x80808080u;
        uint32_t bad;
        if (i == 0) {
            bad = halo ? lead_bad & 0x80808000u : 0u;
        } else {
            const uint32_t must = __builtin_amdgcn_alignbyte(c0, ge_c0(xp), 3) |
                                  __builtin_amdgcn_alignbyte(e0, ge_e0(xp), 2) |
                                  __builtin_amdgcn_alignbyte(f0, ge_f0(xp), 1);
            bad = lead_bad | (cont_bits(x) & ~must & 0x80808080u);
        }
        if (bad) first = 4 * i + ((uint32_t)__builtin_ctz(bad) >> 3);
    }
    if (first == 32) return ~0ull;
    const uint32_t wi = first >> 2;
    const uint32_t lo = wi == 0 ? v0 : (wi == 1 ? v1 : (wi == 2 ? v2 : (wi == 3 ? v3 : v4)));
    const uint32_t hi = wi == 0 ? v1 : (wi == 1 ? v2 : (wi == 2 ? v3 : (wi == 3 ? v4 : v5)));
    const uint32_t w = __builtin_amdgcn_alignbyte(hi, lo, first & 3u);
    const uint32_t b0 = w & 0xFFu;
    const uint32_t kind = is_cont(b0) ? (uint32_t)kTooLong
                                      : lead_kind(b0, (w >> 8) & 0xFFu, (w >> 16) & 0xFFu, w >> 24);
    return ((u64)(q0 + (long long)first - 4 - head) << 4) | kind;
}

// Batched form of exact_chunk: string starts act as buffer ends (a byte at
// a start continues nothing before it), `sbits` bit i marks a start at
// chunk position i - 16.  Each string's first flagged byte in the chunk is
// reported to that string's error word.
__device__ __forceinline__ void exact_chunk_batch(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3, uint32_t v4,
                                               uint32_t v5, u64 sbits, long long q0, long long head, bool halo,
                                               BatchCtx bc) {
    const uint32_t v[6] = {v0, v1, v2, v3, v4, v5};
    uint32_t badm[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {   // dword i holds chunk positions 4i-4 .. 4i-1
        const uint32_t x = v[i], xn = v[i + 1], xp = i > 0 ? v[i - 1] : 0u;
        const uint32_t sp = spread4((uint32_t)(sbits >> (8 + 4 * i)));    // starts in the dword before
        const uint32_t st = spread4((uint32_t)(sbits >> (12 + 4 * i)));   // starts in this dword
        const uint32_t sn = spread4((uint32_t)(sbits >> (16 + 4 * i)));   // starts in the dword after
        const uint32_t c0 = ge_c0(x), e0 = ge_e0(x), f0 = ge_f0(x);
        // continuation bytes that continue this string (none at a start)
        const uint32_t k1 = cont_bits(__builtin_amdgcn_alignbyte(xn, x, 1)) & ~__builtin_amdgcn_alignbyte(sn, st, 1);
        const uint32_t k2 = cont_bits(__builtin_amdgcn_alignbyte(xn, x, 2)) & ~__builtin_amdgcn_alignbyte(sn, st, 2);
        const uint32_t k3 = cont_bits(__builtin_amdgcn_alignbyte(xn, x, 3)) & ~__builtin_amdgcn_alignbyte(sn, st, 3);
        const uint32_t shortb = (c0 & ~k1) | (e0 & ~k2) | (f0 & ~k3);
        const uint32_t lead_bad = (shortb | value_bits<kAny>(x, __builtin_amdgcn_alignbyte(xn, x, 1))) & 0x80808080u;
        if (i == 0) {
            badm[i] = halo ? lead_bad & 0x80808000u : 0u;
        } else {
            const uint32_t m1 = __builtin_amdgcn_alignbyte(c0, ge_c0(xp), 3),
                           m2 = __builtin_amdgcn_alignbyte(e0, ge_e0(xp), 2),
                           m3 = __builtin_amdgcn_alignbyte(f0, ge_f0(xp), 1);
            const uint32_t s1 = __builtin_amdgcn_alignbyte(st, sp, 3), s2 = __builtin_amdgcn_alignbyte(st, sp, 2);
            const uint32_t mi = (m1 & ~st) | (m2 & ~(st | s1)) | (m3 & ~(st | s1 | s2));
            badm[i] = lead_bad | (cont_bits(x) & ~mi & 0x80808080u);
        }
    }
    int lastpos = -100;   // position of the last report (its string's first flag here)
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        uint32_t m = badm[i];
        while (m) {
            const uint32_t byte = (uint32_t)__builtin_ctz(m) >> 3;
            m &= m - 1;
            const int pos = 4 * i - 4 + (int)byte;          // chunk position
            // no string starts in (lastpos, pos]: same string, already reported
            if (lastpos > -100 && ((sbits >> (17 + lastpos)) & ((1ull << (pos - lastpos)) - 1ull)) == 0) continue;
            lastpos = pos;
            const long long pin = q0 + pos - head;          // input position
            const u64 idx = owner_near(bc, q0 / kWaveBytes, pin);
            // the byte and the three after it, bytes of the next string read as zero
            const uint32_t lo = i == 0 ? v0 : (i == 1 ? v1 : (i == 2 ? v2 : (i == 3 ? v3 : v4)));
            const uint32_t hi = i == 0 ? v1 : (i == 1 ? v2 : (i == 2 ? v3 : (i == 3 ? v4 : v5)));
            uint32_t w = __builtin_amdgcn_alignbyte(hi, lo, byte);
            const uint32_t sw = (uint32_t)(sbits >> (16 + pos)) & 15u;   // starts at pos .. pos+3
            if (sw & 2u) w &= 0x000000FFu;
            else if (sw & 4u) w &= 0x0000FFFFu;
            else if (sw & 8u) w &= 0x00FFFFFFu;
            const uint32_t b0 = w & 0xFFu;
            const uint32_t kind = is_cont(b0) ? (uint32_t)kTooLong
                                              : lead_kind(b0, (w >> 8) & 0xFFu, (w >> 16) & 0xFFu, w >> 24);
            min_agent(bc.serr + idx, ((u64)(pin - bc.offsets[idx]) << 4) | kind);
        }
    }
}

template <uint32_t kClass>
__device__ __forceinline__ bool check_values(const LaneBytes &t, uint32_t lane) {
    uint32_t bad = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t nx_row = next_dword(t, r, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = t.d[r][j];
            const uint32_t nx = j < 3 ? t.d[r][j + 1] : nx_row;
            bad |= value_bits<kClass>(x, __builtin_amdgcn_alignbyte(nx, x, 1));
        }
    }
    return bad != 0;
}

// ------------------------------------------------------------------------
// Validation and conversion: tile t = workgroup t.
// ------------------------------------------------------------------------
// Batched calls keep each 64-byte block's output offset inside its tile in
// 16 bits: a tile emits at most one word per byte.
static_assert(kTileBytes <= 65536, "16-bit block offsets");

template <bool kConvert, bool kBatch, bool kTicket>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void utf8_tile_kernel(
    const uint8_t *__restrict__ frame, long long head, long long n, uint16_t *__restrict__ out, u64 out_cap,
    u64 *__restrict__ status, Ctrl *__restrict__ ctrl, u64 ntiles, int spin_limit, BatchCtx bc) {
    static_assert(kConvert || !kTicket, "validation has no scan: tiles in block order");
    __shared__ __attribute__((aligned(16))) uint32_t stage[kConvert ? kWaves * kStageWords : 4];
    __shared__ uint32_t s_wave_tot[kWaves];
    __shared__ u64 s_prefix;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar branches on it
    const long long end = head + n;
    __shared__ uint32_t s_ticket;
    const u64 tile = kTicket ? take_ticket(ctrl, &s_ticket, tid) : (u64)blockIdx.x;
    const long long wbase = (long long)tile * kTileBytes + (long long)wave * kWaveBytes;
    LaneBytes t;
    issue_span(frame, end, wbase, lane, t);
    const u64 epoch = kConvert && wave == 0 ? ld_agent(&ctrl->epoch) : 0;   // only wave 0 looks back
    finish_span(head, end, wbase, lane, t);
    {
        Survey sv;
        survey_span<kBatch>(t, wbase, head, end, lane, sv, bc);
        // the all-ASCII shortcut widens whole chunks: not for waves at the ends
        const uint32_t cls = (sv.cls == kAscii && t.edge) ? kUpTo2 : sv.cls;
        bool flag = sv.mis;
        fence_values(t);
        // a wave whose detector fired, when an error before it is already
        // known: its output lies past the valid prefix and is not written.
        // The error word is read after the tile prefix is known: read here,
        // its latency would delay the tile's aggregate, which later tiles'
        // look-back waits for.
        const bool flagged = !kBatch && kConvert && __ballot(flag);

        if (kConvert) {
            // in-wave offsets (row-major) and wave total
            uint32_t gof[kRows], rowbase[kRows + 1];
            rowbase[0] = 0;
#pragma unroll
            for (int p = 0; p < kRows / 2; ++p) {
                const uint32_t s0 = sv.width[2 * p], s1 = sv.width[2 * p + 1];
                const uint32_t inc = wave_incl_scan(s0 | (s1 << 16), lane);
                const uint32_t tot = readlane(inc, kWave - 1);
                gof[2 * p] = rowbase[2 * p] + (inc & 0xFFFFu) - s0;
                rowbase[2 * p + 1] = rowbase[2 * p] + (tot & 0xFFFFu);
                gof[2 * p + 1] = rowbase[2 * p + 1] + (inc >> 16) - s1;
                rowbase[2 * p + 2] = rowbase[2 * p + 1] + (tot >> 16);
            }
#pragma unroll
            for (int r = 0; r < kRows; ++r) gof[r] -= rowbase[(r / kGroup) * kGroup];   // offsets inside the group
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
                const u64 prefix = resolve_prefix(status, tile, epoch, spin_limit, tile_total, [=](long long tl) {
                    return tile_width16(frame, head, end, tl);
                });
                if (lane == 0) {
                    s_prefix = prefix;
                    if (tile == ntiles - 1) st_agent(&ctrl->total, prefix + tile_total);
                    if (kBatch) bc.tilepre[tile] = prefix;
                }
            }
            if (kBatch && (lane & 3u) == 0) {   // in-tile output offset of every 64-byte block
                const long long blk = ((wbase >> 4) + lane) >> 2;
#pragma unroll
                for (int r = 0; r < kRows; ++r)
                    bc.blockoff[blk + r * (kRowBytes / 64)] = (uint16_t)(wave_off + rowbase[r] + gof[r]);
            }
            uint32_t *wst = stage + wave * kStageWords;
            // batched calls: a group of an invalid string can announce more
            // slots than the stage holds; the strings after it in the wave
            // still need their words, stored one by one instead
            bool direct = false;
            if (kBatch && has4(cls))
#pragma unroll
                for (int g = 0; g < kRows / kGroup; ++g)
                    direct |= rowbase[(g + 1) * kGroup] - rowbase[g * kGroup] > kStageSlots;
            // ASCII + four-byte waves stage only after the prefix: all waves
            // but wave 0 check their value rules while it resolves it
            const bool quad_pre = !kBatch && cls == kQuad && !t.edge && wave != 0;
            if (quad_pre) flag |= quad_values_bad(t, lane);
            if (!direct) switch (cls) {   // the first group needs no prefix
                case kAscii: break;
                case kUpTo3: scatter_row<kUpTo3, kBatch>(t, 0, gof[0], wst, wbase, head, end, lane); break;
                case kQuad:   // staged after the prefix, except at the ends and in batches
                    if (kBatch || t.edge) scatter_row<kQuad, kBatch>(t, 0, gof[0], wst, wbase, head, end, lane);
                    break;
                default: scatter_row<kAny, kBatch>(t, 0, gof[0], wst, wbase, head, end, lane); break;
            }
            // windows classes: the waves waiting for wave 0 decode that group too
            const bool early = !direct && (cls == kUpTo3 || cls == kAny) && wave != 0;
            if (early) {
                uint32_t n0 = rowbase[kGroup] - rowbase[0];
                if (n0 > kStageSlots) n0 = kStageSlots;
                wave_lds_sync();
                flag |= cls == kUpTo3 ? decode_slots_early<kUpTo3>(wst, n0, lane) : decode_slots_early<kAny>(wst, n0, lane);
            }
            __syncthreads();   // the tile prefix is known
            const u64 base = s_prefix + wave_off;
            const bool moot = flagged && (long long)(ld_agent(&ctrl->err) >> 4) < wbase - head;
            if (direct) {
                static_assert(kRows <= 4, "direct_words takes at most four rows");
                u64 slot[4] = {0, 0, 0, 0};
#pragma unroll
                for (int r = 0; r < kRows; ++r) slot[r] = base + rowbase[(r / kGroup) * kGroup] + gof[r];
                direct_words(frame, head, end, wbase, lane, slot[0], slot[1], slot[2], slot[3], out, out_cap);
                flag = true;
            } else if (!moot) switch (cls) {
                case kAscii:
                    if (base + kWaveBytes <= out_cap)
                        widen_store_wave(t, out, base, lane);
                    else
                        convert_wave<kUpTo2, kBatch>(t, gof, rowbase, base, out, out_cap, wst, wbase, head, end, lane,
                                             false);
                    break;
                case kUpTo2:
                    flag |= convert_wave<kUpTo2, kBatch>(t, gof, rowbase, base, out, out_cap, wst, wbase, head, end, lane,
                                                 true);
                    break;
                case kUpTo3:
                    flag |= convert_wave<kUpTo3, kBatch>(t, gof, rowbase, base, out, out_cap, wst, wbase, head, end, lane,
                                                 true, true, early);
                    break;
                case kQuad:
                    flag |= convert_wave<kQuad, kBatch>(t, gof, rowbase, base, out, out_cap, wst, wbase, head, end, lane,
                                                true, !quad_pre);
                    break;
                default:
                    flag |= convert_wave<kAny, kBatch>(t, gof, rowbase, base, out, out_cap, wst, wbase, head, end, lane,
                                               true, true, early);
                    break;
            }
        } else {
            switch (cls) {
                case kAscii: break;
                case kUpTo2: flag = flag || check_values<kUpTo2>(t, lane); break;
                case kUpTo3: flag = flag || check_values<kUpTo3>(t, lane); break;
                default: flag = flag || check_values<kAny>(t, lane); break;
            }
        }

        // exact first error over this lane's positions (and, for the first
        // lane, the leading bytes among the three positions before the wave),
        // unless an error before the wave is already known
        if (kBatch && __ballot(flag)) {   // per string
            const long long c0 = (wbase >> 4) + lane;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
                const uint32_t p = prev_dword(t, r, lane), nx = next_dword(t, r, lane);
                const long long ci = c0 + r * (kRowBytes / 16);
                const u64 bits = (u64)bc.starts[ci - 1 >= 0 ? ci - 1 : 0] * (ci >= 1) |
                                 ((u64)bc.starts[ci] << 16) | ((u64)bc.starts[ci + 1] << 32);
                exact_chunk_batch(p, t.d[r][0], t.d[r][1], t.d[r][2], t.d[r][3], nx, bits, q0, head,
                                  r == 0 && lane == 0, bc);
            }
        }
        if (!kBatch && __ballot(flag) && (long long)(ld_agent(&ctrl->err) >> 4) >= wbase - 3 - head) {
            u64 err = ~0ull;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const long long q0 = wbase + r * kRowBytes + 16 * (long long)lane;
                const uint32_t p = prev_dword(t, r, lane), nx = next_dword(t, r, lane);
                const u64 e = exact_chunk(p, t.d[r][0], t.d[r][1], t.d[r][2], t.d[r][3], nx, q0, head,
                                          r == 0 && lane == 0);
                if (e < err) err = e;
            }
            err = wave_min_u64(err);
            if (lane == 0 && err != ~0ull) min_agent(&ctrl->err, err);
        }
    }
}

// ------------------------------------------------------------------------
// UTF-16 length of UTF-8 (no validation): per-workgroup partial sums.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void utf16_length_kernel(const uint8_t *__restrict__ frame, long long head,
                                                               long long n, u64 *__restrict__ partials) {
    __shared__ u64 s_sum[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const long long end = head + n;
    const long long nchunks = (end + 15) / 16;
    const long long stride = (long long)gridDim.x * kBlock;
    u64 acc = 0;
    for (long long c = (long long)blockIdx.x * kBlock + tid; c < nchunks; c += 4 * stride) {
        const uint32_t w0 = load_chunk_width16(frame, head, end, 16 * c);
        const uint32_t w1 = c + stride < nchunks ? load_chunk_width16(frame, head, end, 16 * (c + stride)) : 0;
        const uint32_t w2 = c + 2 * stride < nchunks ? load_chunk_width16(frame, head, end, 16 * (c + 2 * stride)) : 0;
        const uint32_t w3 = c + 3 * stride < nchunks ? load_chunk_width16(frame, head, end, 16 * (c + 3 * stride)) : 0;
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

// ------------------------------------------------------------------------
// Finalize (shared by every kernel family)
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void finalize_kernel(Ctrl *ctrl, DevResult *result, u64 *len_result, int mode,
                                                           u64 n, u64 out_cap, const u64 *partials, int npartials) {
    __shared__ u64 s_sum[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    if (mode == kFinLength) {
        u64 acc = 0;
        for (int i = (int)tid; i < npartials; i += kBlock) acc += partials[i];
        acc = wave_sum_u64(acc);
        if (lane == 0) s_sum[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            u64 b = 0;
            for (int w = 0; w < kWaves; ++w) b += s_sum[w];
            *len_result = b;
        }
        return;
    }
    if (tid == 0) {
        const u64 e = ld_agent(&ctrl->err);
        if (e != ~0ull) {
            result->status = (int32_t)(e & 15u);
            result->count = e >> 4;
        } else if (mode == kFinConvert) {
            const u64 tot = ld_agent(&ctrl->total);
            result->status = tot > out_cap ? (int32_t)kOutputTooSmall : (int32_t)kOk;
            result->count = tot;
        } else {
            result->status = kOk;
            result->count = n;
        }
        result->pad = 0;
    }
    reset_control(ctrl, tid, kBlock);   // its barrier orders the reads above before the reset
}

__global__ __launch_bounds__(kBlock) void ctrl_init_kernel(Ctrl *ctrl, u64 *status, u64 status_cap, u64 period) {
    const uint32_t tid = threadIdx.x;
    for (u64 t = (u64)blockIdx.x * kBlock + tid; t < status_cap; t += (u64)gridDim.x * kBlock)
        status[t * kStatusStride] = 0;
    if (blockIdx.x == 0 && tid == 0) {
        ctrl->err = ~0ull;
        ctrl->total = 0;
        ctrl->ticket = 0;
        ctrl->done = 0;
        ctrl->bad = 0;
        ctrl->epoch = 1;
        ctrl->period = period;
        ctrl->status = status;
        ctrl->status_cap = status_cap;
    }
}

// Results of empty inputs for the asynchronous calls (a kernel rather than
// a copy from host memory, so the call also works under stream capture).
__global__ void set_result_kernel(DevResult *r, int32_t status, u64 count) {
    if (threadIdx.x == 0) {
        r->status = status;
        r->pad = 0;
        r->count = count;
    }
}
__global__ void set_u64_kernel(u64 *r, u64 v) {
    if (threadIdx.x == 0) *r = v;
}

// ------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the C ABI layer).
// ------------------------------------------------------------------------
// Input bytes per tile of this build.
u64 build_tile_bytes() { return (u64)kTileBytes; }

u64 utf8_tiles_for(long long head, long long n) {
    // three positions past the end belong to tiles too: a leading byte near
    // the end announces continuation bytes there
    return (u64)((head + n + 3 + kTileBytes - 1) / kTileBytes);
}

hipError_t launch_utf8_tiles(bool convert, const uint8_t *frame, long long head, long long n, uint16_t *out,
                             u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, int schedule,
                             hipStream_t stream) {
    const u64 ntiles = utf8_tiles_for(head, n);
    const BatchCtx none = {nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (convert && schedule == kScheduleTicket)
        hipLaunchKernelGGL((utf8_tile_kernel<true, false, true>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    else if (convert)
        hipLaunchKernelGGL((utf8_tile_kernel<true, false, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    else   // no scan: the schedule does not apply
        hipLaunchKernelGGL((utf8_tile_kernel<false, false, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), none);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, result, nullptr, convert ? kFinConvert : kFinValidate, (u64)n, out_cap, nullptr,
                           0, stream);
}

// ------------------------------------------------------------------------
// Batched UTF-8 -> UTF-16LE
// ------------------------------------------------------------------------
// Thread i < k checks string i's offsets (0 = offsets[0] <= ... <=
// offsets[k] = n; a bad array sets `bad`, a word of the control block that
// is zero between calls), marks its first byte in the start bitmap when it
// is not empty, and owns every wave span (`span` units, frame coordinates)
// whose first position the string holds; positions before the input count
// as position 0 and positions past it as position n - 1.  So an error's
// owner is found among the few strings near its wave, and no thread
// searches.  The 64 threads of a wave then write the owners of all their
// strings' spans together (a string of many spans takes one store per lane
// per 64 spans).  Thread k checks the last offset.  kPrepBlock threads per
// workgroup.
__global__ __launch_bounds__(kPrepBlock) void batch_prep_kernel(const int64_t *offsets, u64 k, long long head,
                                                                long long n, uint32_t *starts, uint32_t *bad,
                                                                long long span, uint32_t *wavestr, u64 nspans) {
    const u64 i = (u64)blockIdx.x * kPrepBlock + threadIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    long long wlo = 1, whi = 0;   // the spans string i owns (none)
    if (i <= k) {
        const int64_t a = offsets[i];
        if (i == 0 && a != 0) atomicOr(bad, 1u);
        if (i == k) {
            if (a != n) atomicOr(bad, 1u);
        } else {
            const int64_t b = offsets[i + 1];
            if (a < 0 || b < a || b > n) {
                atomicOr(bad, 1u);
            } else if (b > a) {
                const u64 q = (u64)(head + a);
                atomicOr(starts + (q >> 5), 1u << (q & 31u));
                wlo = a == 0 ? 0 : (a + head + span - 1) / span;
                whi = b == n ? (long long)nspans : (b + head + span - 1) / span - 1;
            }
        }
    }
#pragma unroll 1
    for (int L = 0; L < kWave; ++L) {   // every lane of the wave takes part
        const long long lo = (long long)(((u64)readlane((uint32_t)((u64)wlo >> 32), L) << 32) |
                                         readlane((uint32_t)wlo, L));
        const long long hi = (long long)(((u64)readlane((uint32_t)((u64)whi >> 32), L) << 32) |
                                         readlane((uint32_t)whi, L));
        const uint32_t owner = readlane((uint32_t)i, L);
        for (long long w = lo + lane; w <= hi; w += kWave) wavestr[w] = owner;
    }
}

// Output offset of input byte p: the tile's offset, the offset of p's
// 64-byte block inside the tile, and the widths of the block's bytes
// before p.
__device__ u64 batch_out_offset(const uint8_t *frame, long long head, long long n, const BatchCtx &bc, u64 total,
                                int64_t p) {
    if (p >= n) return total;
    const long long q = head + p;
    const long long b0 = q & ~63ll;
    u64 w = bc.tilepre[q / kTileBytes] + bc.blockoff[q >> 6];
    for (long long c = b0; c < q; c += 16) {
        const long long e = c + 16 < q ? c + 16 : q;
        w += load_chunk_width16(frame, head, e, c);
    }
    return w;
}

// Per string: output offsets, result, and the reset of its error word and
// start bit for the next call.  `oa` and `ob` are the output offsets at the
// string's first and past its last position (0 when the offsets are bad).
__device__ __forceinline__ void post_string(const BatchCtx &bc, long long n, int64_t *out_offsets,
                                            DevResult *results, u64 out_cap, bool ok, uint32_t *starts,
                                            long long head, u64 i, u64 oa, u64 ob) {
    const int64_t a = bc.offsets[i];
    out_offsets[i] = (int64_t)oa;
    if (i == bc.k) return;
    const int64_t b = bc.offsets[i + 1];
    // the start bit batch_prep_kernel set for this string (same test)
    if (a >= 0 && b > a && b <= n) {
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

// Thread i <= k: the output offset at offsets[i], shared through LDS so
// that each offset is computed once (the workgroup's last thread also
// computes the one after its string); then string i's offsets and result
// (post_string), and the last workgroup to finish resets the control block
// for the next call.  Launched with kPostBlock threads per workgroup.
__global__ __launch_bounds__(kPostBlock) void batch_post_kernel(const uint8_t *frame, long long head, long long n,
                                                                BatchCtx bc, Ctrl *ctrl, int64_t *out_offsets,
                                                                DevResult *results, u64 out_cap,
                                                                const uint32_t *bad, uint32_t *starts) {
    __shared__ u64 s_off[kPostBlock + 1];
    const uint32_t tid = threadIdx.x;
    const u64 i = (u64)blockIdx.x * kPostBlock + tid;
    const bool ok = *bad == 0;
    const u64 total = ld_agent(&ctrl->total);
    if (i <= bc.k) {
        s_off[tid] = ok ? batch_out_offset(frame, head, n, bc, total, bc.offsets[i]) : 0;
        if (tid == kPostBlock - 1 && i < bc.k)
            s_off[kPostBlock] = ok ? batch_out_offset(frame, head, n, bc, total, bc.offsets[i + 1]) : 0;
    }
    __syncthreads();
    if (i <= bc.k)
        post_string(bc, n, out_offsets, results, out_cap, ok, starts, head, i, s_off[tid],
                    i < bc.k ? s_off[tid + 1] : 0);
    batch_call_done(ctrl, tid);
}

// Mark the string starts and index the wave spans (both directions); the
// offsets flag is cleared at the end of the previous call.
hipError_t launch_batch_prep(const int64_t *offsets, u64 k, long long head, long long n, uint32_t *starts,
                             uint32_t *bad, long long span, uint32_t *wavestr, u64 nspans, hipStream_t stream) {
    const unsigned pb = kPrepBlock, pg = (unsigned)((k + 1 + pb - 1) / pb);
    hipLaunchKernelGGL(batch_prep_kernel, dim3(pg), dim3(pb), 0, stream, offsets, k, head, n, starts, bad, span,
                       wavestr, nspans);
    return hipGetLastError();
}

hipError_t launch_utf8_batch(const uint8_t *frame, long long head, long long n, const int64_t *offsets, u64 k,
                             uint16_t *out, u64 out_cap, int64_t *out_offsets, DevResult *results, u64 *status,
                             Ctrl *ctrl, uint32_t *starts, uint16_t *blockoff,
                             u64 *tilepre, u64 *serr, uint32_t *bad, uint32_t *wavestr, int schedule,
                             hipStream_t stream) {
    const unsigned pb = kPostBlock, pg = (unsigned)((k + 1 + pb - 1) / pb);
    const u64 ntiles = utf8_tiles_for(head, n);
    hipError_t e = launch_batch_prep(offsets, k, head, n, starts, bad, kWaveBytes, wavestr, ntiles * kWaves, stream);
    if (e != hipSuccess) return e;
    const BatchCtx bc = {offsets, k, (const uint16_t *)starts, blockoff, tilepre, serr, wavestr};
    if (n > 0 && schedule == kScheduleTicket)
        hipLaunchKernelGGL((utf8_tile_kernel<true, true, true>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), bc);
    else if (n > 0)
        hipLaunchKernelGGL((utf8_tile_kernel<true, true, false>), dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, n, out, out_cap, status, ctrl, ntiles, lookback_spin_limit(), bc);
    hipLaunchKernelGGL(batch_post_kernel, dim3(pg), dim3(pb), 0, stream, frame, head, n, bc, ctrl, out_offsets,
                       results, out_cap, (const uint32_t *)bad, starts);
    return hipGetLastError();
}

int partial_blocks(long long units, long long units_per_block) {
    long long b = (units + units_per_block - 1) / units_per_block;
    if (b < 1) b = 1;
    if (b > kMaxPartials) b = kMaxPartials;
    return (int)b;
}

hipError_t launch_utf16_length(const uint8_t *frame, long long head, long long n, u64 *partials, Ctrl *ctrl,
                               u64 *result, hipStream_t stream) {
    const int nb = partial_blocks(head + n, 16LL * kBlock * 4);
    hipLaunchKernelGGL(utf16_length_kernel, dim3(nb), dim3(kBlock), 0, stream, frame, head, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, nullptr, result, kFinLength, 0, 0, partials, nb, stream);
}

hipError_t launch_finalize(Ctrl *ctrl, DevResult *result, u64 *len_result, int mode, u64 n, u64 out_cap,
                           const u64 *partials, int npartials, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kBlock), 0, stream, ctrl, result, len_result, mode, n,
                       out_cap, partials, npartials);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl *ctrl, u64 *status, u64 status_cap, u64 period, hipStream_t stream) {
    const u64 blocks = (status_cap + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(ctrl_init_kernel, dim3((unsigned)(blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks))),
                       dim3(kBlock), 0, stream, ctrl, status, status_cap, period);
    return hipGetLastError();
}

hipError_t launch_set_result(DevResult *r, int32_t status, u64 count, hipStream_t stream) {
    hipLaunchKernelGGL(set_result_kernel, dim3(1), dim3(64), 0, stream, r, status, count);
    return hipGetLastError();
}
hipError_t launch_set_u64(u64 *r, u64 v, hipStream_t stream) {
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, stream, r, v);
    return hipGetLastError();
}

}  // namespace UTF_GEOM
}  // namespace utfgpu
