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
#include "device_common.hpp"

namespace utfgpu {

constexpr int kRowUnits = kRowBytes / 2;       // 512
constexpr int kWaveUnits = kWaveBytes / 2;     // 2048 words per wave
constexpr int kTileUnits = kTileBytes / 2;     // 32768 words per tile
// bytes one wave stages at a time: at most 3 per word
constexpr uint32_t kStageBytes = 3u * kGroup * kRowUnits;
constexpr int kStageWords16 = (int)kStageBytes / 4 + 4;

enum : uint32_t { kAscii16 = 0, kUpTo2B = 1, kBmp = 2, kAnyUnit = 3 };

// Zero the words of the dword holding frame words p, p+1 that fall
// outside [lo, hi).
__device__ __forceinline__ uint32_t keep_units(uint32_t x, long long p, long long lo, long long hi) {
    const bool k0 = p >= lo && p < hi;
    const bool k1 = p + 1 >= lo && p + 1 < hi;
    return x & ((k0 ? 0x0000FFFFu : 0u) | (k1 ? 0xFFFF0000u : 0u));
}

struct LaneUnits {
    uint32_t d[kRows][4];   // eight words per row, two per dword (low half first)
    uint32_t prev[kRows];   // dword before the chunk (its high half is the word before)
    uint32_t next[kRows];   // dword after the chunk (its low half is the word after)
};

__device__ __forceinline__ void load_span16(const uint8_t *frame, long long head, long long end, long long wbase,
                                            uint32_t lane, LaneUnits &t) {
    const bool edge_wave = wbase < head || wbase + kWaveUnits > end;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (q0 < end) v = __builtin_nontemporal_load((const u32x4 *)(frame + 2 * q0));
        t.d[r][0] = v.x; t.d[r][1] = v.y; t.d[r][2] = v.z; t.d[r][3] = v.w;
        if (edge_wave && (q0 < head || q0 + 8 > end)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) t.d[r][k] = keep_units(t.d[r][k], q0 + 2 * k, head, end);
        }
    }
    uint32_t hp = 0, hn = 0;
    if (wbase - 2 >= 0 && wbase - 2 < end)
        hp = keep_units(*(const uint32_t *)(frame + 2 * (wbase - 2)), wbase - 2, head, end);
    if (wbase + kWaveUnits < end)
        hn = keep_units(*(const uint32_t *)(frame + 2 * (wbase + kWaveUnits)), wbase + kWaveUnits, head, end);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = __shfl_up(t.d[r][3], 1);
        const uint32_t nx = __shfl_down(t.d[r][0], 1);
        const uint32_t p0 = r == 0 ? hp : readlane(t.d[r - 1][3], kWave - 1);
        const uint32_t n63 = r == kRows - 1 ? hn : readlane(t.d[r + 1][0], 0);
        t.prev[r] = lane == 0 ? p0 : p;
        t.next[r] = lane == kWave - 1 ? n63 : nx;
    }
}

__device__ __forceinline__ bool is_sur(uint32_t u) { return (u & 0xF800u) == 0xD800u; }
__device__ __forceinline__ bool is_high(uint32_t u) { return (u & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(uint32_t u) { return (u & 0xFC00u) == 0xDC00u; }

// Any surrogate among the two words of x.
__device__ __forceinline__ bool has_sur(uint32_t x) { return is_sur(x & 0xFFFFu) || is_sur(x >> 16); }

__device__ __forceinline__ uint32_t wave_class16(const LaneUnits &t) {
    uint32_t a80 = 0, a800 = 0;
    bool sur = false;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = t.d[r][k];
            a80 |= x & 0xFF80FF80u;
            a800 |= x & 0xF800F800u;
            sur = sur || has_sur(x);
        }
    if (__ballot(sur)) return kAnyUnit;
    if (__ballot(a800 != 0)) return kBmp;
    if (__ballot(a80 != 0)) return kUpTo2B;
    return kAscii16;
}

// UTF-8 bytes of one word (1 below 0x80, 2 below 0x800, 2 per surrogate
// word, 3 otherwise).
__device__ __forceinline__ uint32_t width8(uint32_t u) {
    return 1u + (u >= 0x80u) + (u >= 0x800u) - (uint32_t)is_sur(u);
}

__device__ __forceinline__ uint32_t chunk_width8(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3) {
    return width8(d0 & 0xFFFFu) + width8(d0 >> 16) + width8(d1 & 0xFFFFu) + width8(d1 >> 16) +
           width8(d2 & 0xFFFFu) + width8(d2 >> 16) + width8(d3 & 0xFFFFu) + width8(d3 >> 16);
}

__device__ __forceinline__ uint32_t outside_count8(long long q0, long long head, long long end) {
    const long long a = q0 < head ? head : q0;
    const long long b = q0 + 8 > end ? end : q0 + 8;
    const long long in = b > a ? b - a : 0;
    return (uint32_t)(8 - in);
}

__device__ __forceinline__ uint32_t valid_mask8(long long q0, long long head, long long end) {
    if (q0 >= head && q0 + 8 <= end) return 0xFFu;
    uint32_t m = 0;
    for (int k = 0; k < 8; ++k)
        if (q0 + k >= head && q0 + k < end) m |= 1u << k;
    return m;
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

// Aggregate (bytes) of tile `tl`, computed by one wave from global memory.
__device__ u64 tile_width8(const uint8_t *frame, long long head, long long end, long long tl) {
    const uint32_t lane = lane_id();
    u64 acc = 0;
    const long long base = tl * kTileUnits;
    for (int r = 0; r < kTileUnits / kRowUnits; ++r)
        acc += load_chunk_width8(frame, head, end, base + r * kRowUnits + 8 * (long long)lane);
    return wave_sum_u64(acc);
}

// Word j (0..7) of a row, with j = -1 and j = 8 reaching into the halo.
__device__ __forceinline__ uint32_t word_at(const LaneUnits &t, int r, int j) {
    if (j < 0) return t.prev[r] >> 16;
    if (j > 7) return t.next[r] & 0xFFFFu;
    return (t.d[r][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

// UTF-8 bytes of word u (packed, first byte lowest) and their number.
// `pv` and `nx` are the words before and after (used by surrogates).
template <uint32_t kClass>
__device__ __forceinline__ uint32_t encode_word(uint32_t u, uint32_t pv, uint32_t nx, uint32_t &len) {
    if (u < 0x80u) {
        len = 1;
        return u;
    }
    if (kClass == kUpTo2B || u < 0x800u) {
        len = 2;
        return (0xC0u | (u >> 6)) | ((0x80u | (u & 0x3Fu)) << 8);
    }
    if (kClass == kBmp || !is_sur(u)) {
        len = 3;
        return (0xE0u | (u >> 12)) | ((0x80u | ((u >> 6) & 0x3Fu)) << 8) | ((0x80u | (u & 0x3Fu)) << 16);
    }
    len = 2;
    if (is_high(u)) {
        const uint32_t cp = 0x10000u + (((u & 0x3FFu) << 10) | (nx & 0x3FFu));
        return (0xF0u | (cp >> 18)) | ((0x80u | ((cp >> 12) & 0x3Fu)) << 8);
    }
    const uint32_t cp = 0x10000u + (((pv & 0x3FFu) << 10) | (u & 0x3FFu));
    return (0x80u | ((cp >> 6) & 0x3Fu)) | ((0x80u | (cp & 0x3Fu)) << 8);
}

// First unpaired surrogate among the lane's words (position << 4 | kind).
__device__ __forceinline__ u64 lane_first_error16(const LaneUnits &t, const uint32_t (&vm)[kRows], long long wbase,
                                                  long long head, uint32_t lane) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t u = word_at(t, r, j);
            const bool bad = ((vm[r] >> j) & 1u) &&
                             ((is_high(u) && !is_low(word_at(t, r, j + 1))) || (is_low(u) && !is_high(word_at(t, r, j - 1))));
            if (bad) {
                const long long q = wbase + r * kRowUnits + 8 * (long long)lane + j;
                return ((u64)(q - head) << 4) | (is_high(u) ? kUnpairedHigh : kUnpairedLow);
            }
        }
    }
    return ~0ull;
}

template <uint32_t kClass>
__device__ __forceinline__ void encode_group(const LaneUnits &t, int r0, const uint32_t (&off)[kRows],
                                             const uint32_t (&vm)[kRows], uint8_t *stage8) {
#pragma unroll
    for (int r = r0; r < r0 + kGroup; ++r) {
        uint32_t o = off[r];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (!((vm[r] >> j) & 1u)) continue;
            const uint32_t u = word_at(t, r, j);
            uint32_t len;
            const uint32_t b = encode_word<kClass>(u, word_at(t, r, j - 1), word_at(t, r, j + 1), len);
            stage8[o] = (uint8_t)b;
            if (len > 1) stage8[o + 1] = (uint8_t)(b >> 8);
            if (len > 2) stage8[o + 2] = (uint8_t)(b >> 16);
            o += len;
        }
    }
}

// ASCII rows: keep the low byte of every word.  In an all-ASCII wave the
// group-local offset of a lane's row is a multiple of 8 bytes.
__device__ __forceinline__ void narrow_group(const LaneUnits &t, int r0, const uint32_t (&off)[kRows],
                                             uint8_t *stage8) {
#pragma unroll
    for (int r = r0; r < r0 + kGroup; ++r) {
        const uint32_t lo = __builtin_amdgcn_perm(t.d[r][1], t.d[r][0], 0x06040200u);
        const uint32_t hi = __builtin_amdgcn_perm(t.d[r][3], t.d[r][2], 0x06040200u);
        uint32_t *dst = (uint32_t *)(stage8 + off[r]);
        dst[0] = lo;
        dst[1] = hi;
    }
}

__device__ __forceinline__ void encode_group_any(uint32_t cls, const LaneUnits &t, int r0,
                                                 const uint32_t (&off)[kRows], const uint32_t (&vm)[kRows],
                                                 uint8_t *stage8) {
    switch (cls) {
        case kAscii16: narrow_group(t, r0, off, stage8); break;
        case kUpTo2B: encode_group<kUpTo2B>(t, r0, off, vm, stage8); break;
        case kBmp: encode_group<kBmp>(t, r0, off, vm, stage8); break;
        default: encode_group<kAnyUnit>(t, r0, off, vm, stage8); break;
    }
}

template <bool kConvert>
__global__ __launch_bounds__(kBlock) void utf16_tile_kernel(const uint8_t *__restrict__ frame, long long head,
                                                             long long m, uint8_t *__restrict__ out, u64 out_cap,
                                                             u64 *__restrict__ status, Ctrl *__restrict__ ctrl,
                                                             u64 ntiles, int spin_limit) {
    __shared__ __attribute__((aligned(16))) uint32_t stage[kConvert ? kWaves * kStageWords16 : 4];
    __shared__ uint32_t s_wave_tot[kWaves];
    __shared__ u64 s_prefix;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid >> 6;
    const u64 tile = blockIdx.x;
    const long long end = head + m;
    const long long wbase = (long long)tile * kTileUnits + (long long)wave * kWaveUnits;

    LaneUnits t;
    load_span16(frame, head, end, wbase, lane, t);
    uint32_t cls = wave_class16(t);
    if (cls == kAscii16 && (wbase < head || wbase + kWaveUnits > end)) cls = kUpTo2B;

    uint32_t vm[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) vm[r] = valid_mask8(wbase + r * kRowUnits + 8 * (long long)lane, head, end);

    u64 err = ~0ull;
    if (cls == kAnyUnit) err = lane_first_error16(t, vm, wbase, head, lane);

    if (kConvert) {
        uint32_t s[kRows], off[kRows], rowbase[kRows + 1];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
            s[r] = chunk_width8(t.d[r][0], t.d[r][1], t.d[r][2], t.d[r][3]) - outside_count8(q0, head, end);
        }
        rowbase[0] = 0;
#pragma unroll
        for (int p = 0; p < kRows / 2; ++p) {
            const uint32_t inc = wave_incl_scan(s[2 * p] | (s[2 * p + 1] << 16), lane);
            const uint32_t tot = readlane(inc, kWave - 1);
            off[2 * p] = rowbase[2 * p] + (inc & 0xFFFFu) - s[2 * p];
            rowbase[2 * p + 1] = rowbase[2 * p] + (tot & 0xFFFFu);
            off[2 * p + 1] = rowbase[2 * p + 1] + (inc >> 16) - s[2 * p + 1];
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
            const u64 epoch = ld_agent(&ctrl->epoch);
            const u64 prefix = resolve_prefix(status, tile, epoch, spin_limit, tile_total, [=](long long tl) {
                return tile_width8(frame, head, end, tl);
            });
            if (lane == 0) {
                s_prefix = prefix;
                if (tile == ntiles - 1) st_agent(&ctrl->total, prefix + tile_total);
            }
        }
        uint8_t *wst8 = (uint8_t *)(stage + wave * kStageWords16);
        uint32_t gof[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) gof[r] = off[r] - rowbase[(r / kGroup) * kGroup];
        encode_group_any(cls, t, 0, gof, vm, wst8);
        __syncthreads();   // the tile prefix is known
        const u64 base = s_prefix + wave_off;
#pragma unroll
        for (int g = 0; g < kRows / kGroup; ++g) {
            if (g > 0) encode_group_any(cls, t, g * kGroup, gof, vm, wst8);
            wave_lds_sync();
            const u64 b0 = base + rowbase[g * kGroup];
            u64 nbytes = rowbase[(g + 1) * kGroup] - rowbase[g * kGroup];
            if (b0 >= out_cap) nbytes = 0;
            else if (b0 + nbytes > out_cap) nbytes = out_cap - b0;
            write_out<1, kWave>(out + b0, nbytes, (const uint32_t *)wst8, lane);
            wave_lds_sync();
        }
    }

    if (cls == kAnyUnit) {
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
                              u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, hipStream_t stream) {
    const u64 ntiles = utf16_tiles_for(head, m);
    if (convert)
        hipLaunchKernelGGL(utf16_tile_kernel<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame, head, m,
                           out, out_cap, status, ctrl, ntiles, lookback_spin_limit());
    else
        hipLaunchKernelGGL(utf16_tile_kernel<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame, head,
                           m, out, out_cap, status, ctrl, ntiles, lookback_spin_limit());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, result, nullptr, convert ? kFinConvert : kFinValidate, (u64)m, out_cap, nullptr,
                           0, stream);
}

hipError_t launch_utf8_length(const uint8_t *frame, long long head, long long m, u64 *partials, Ctrl *ctrl,
                              u64 *result, hipStream_t stream) {
    const int nb = partial_blocks(head + m, 8LL * kBlock * 4);
    hipLaunchKernelGGL(utf8_length_kernel, dim3(nb), dim3(kBlock), 0, stream, frame, head, m, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize(ctrl, nullptr, result, kFinLength, 0, 0, partials, nb, stream);
}

}  // namespace utfgpu
