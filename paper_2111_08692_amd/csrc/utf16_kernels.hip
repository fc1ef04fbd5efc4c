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
constexpr int kWaveUnits = kWaveBytes / 2;     // 2048
constexpr int kTileUnits = kTileBytes / 2;     // 8192
constexpr uint32_t kStageBytes16 = 3u * kTileUnits;

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

__device__ __forceinline__ void load_tile16(const uint8_t *frame, long long head, long long end,
                                            long long wbase, uint32_t lane, LaneUnits &t) {
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
        uint32_t p = __shfl_up(t.d[r][3], 1);
        uint32_t nx = __shfl_down(t.d[r][0], 1);
        const uint32_t p0 = r == 0 ? hp : readlane(t.d[r - 1][3], kWave - 1);
        const uint32_t n63 = r == kRows - 1 ? hn : readlane(t.d[r + 1][0], 0);
        t.prev[r] = lane == 0 ? p0 : p;
        t.next[r] = lane == kWave - 1 ? n63 : nx;
    }
}

__device__ __forceinline__ bool is_sur(uint32_t u) { return (u & 0xF800u) == 0xD800u; }
__device__ __forceinline__ bool is_high(uint32_t u) { return (u & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(uint32_t u) { return (u & 0xFC00u) == 0xDC00u; }

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
            sur = sur || is_sur(x & 0xFFFFu) || is_sur(x >> 16);
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

__device__ __forceinline__ uint32_t chunk_width8(const uint32_t (&d)[4]) {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) w += width8(d[k] & 0xFFFFu) + width8(d[k] >> 16);
    return w;
}

__device__ __forceinline__ uint32_t outside_count8(long long q0, long long head, long long end) {
    long long a = q0 < head ? head : q0;
    long long b = q0 + 8 > end ? end : q0 + 8;
    long long in = b > a ? b - a : 0;
    return (uint32_t)(8 - in);
}

__device__ __forceinline__ uint32_t valid_mask8(long long q0, long long head, long long end) {
    if (q0 >= head && q0 + 8 <= end) return 0xFFu;
    uint32_t m = 0;
    for (int k = 0; k < 8; ++k)
        if (q0 + k >= head && q0 + k < end) m |= 1u << k;
    return m;
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

template <uint32_t kClass, bool kStore>
__device__ __forceinline__ u64 encode_lane(const LaneUnits &t, const uint32_t (&off)[kRows],
                                           const uint32_t (&vm)[kRows], uint8_t *stage8,
                                           long long wbase, long long head, uint32_t lane) {
    u64 err = ~0ull;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t o = off[r];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (!((vm[r] >> j) & 1u)) continue;
            const uint32_t u = word_at(t, r, j);
            const uint32_t pv = word_at(t, r, j - 1);
            const uint32_t nx = word_at(t, r, j + 1);
            if (kClass == kAnyUnit) {
                const bool bad = (is_high(u) && !is_low(nx)) || (is_low(u) && !is_high(pv));
                if (bad && err == ~0ull) {
                    const long long q = wbase + r * kRowUnits + 8 * (long long)lane + j;
                    err = ((u64)(q - head) << 4) | (is_high(u) ? kUnpairedHigh : kUnpairedLow);
                }
            }
            uint32_t len;
            const uint32_t b = encode_word<kClass>(u, pv, nx, len);
            if (kStore) {
                stage8[o] = (uint8_t)b;
                if (len > 1) stage8[o + 1] = (uint8_t)(b >> 8);
                if (len > 2) stage8[o + 2] = (uint8_t)(b >> 16);
            }
            o += len;
        }
    }
    return err;
}

// ASCII rows: keep the low byte of every word.
__device__ __forceinline__ void narrow_ascii(const LaneUnits &t, const uint32_t (&off)[kRows], uint8_t *stage8) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t lo = __builtin_amdgcn_perm(t.d[r][1], t.d[r][0], 0x06040200u);
        const uint32_t hi = __builtin_amdgcn_perm(t.d[r][3], t.d[r][2], 0x06040200u);
        const uint32_t o = off[r];
        if ((o & 3u) == 0u) {
            uint32_t *dst = (uint32_t *)(stage8 + o);
            dst[0] = lo;
            dst[1] = hi;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                stage8[o + k] = (uint8_t)(lo >> (8 * k));
                stage8[o + 4 + k] = (uint8_t)(hi >> (8 * k));
            }
        }
    }
}

template <bool kConvert>
__global__ __launch_bounds__(kBlock) void utf16_tile_kernel(
    const uint8_t *__restrict__ frame, long long head, long long m, uint8_t *__restrict__ out, u64 out_cap,
    u64 *__restrict__ status, Ctrl *__restrict__ ctrl, DevResult *__restrict__ result, u64 ntiles) {
    constexpr int kStageWords = kConvert ? (int)(kStageBytes16 / 4 + 4) : 2;
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
    const long long end = head + m;
    const long long wbase = (long long)tile * kTileUnits + (long long)wave * kWaveUnits;

    LaneUnits t;
    load_tile16(frame, head, end, wbase, lane, t);
    uint32_t cls = wave_class16(t);
    if (cls == kAscii16 && (wbase < head || wbase + kWaveUnits > end)) cls = kUpTo2B;

    uint32_t s[kRows], vm[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = wbase + r * kRowUnits + 8 * (long long)lane;
        vm[r] = valid_mask8(q0, head, end);
        s[r] = chunk_width8(t.d[r]) - outside_count8(q0, head, end);
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

    uint8_t *stage8 = (uint8_t *)stage;
    u64 err = ~0ull;
    switch (cls) {
        case kAscii16:
            if (kConvert) narrow_ascii(t, off, stage8);
            break;
        case kUpTo2B:
            encode_lane<kUpTo2B, kConvert>(t, off, vm, stage8, wbase, head, lane);
            break;
        case kBmp:
            encode_lane<kBmp, kConvert>(t, off, vm, stage8, wbase, head, lane);
            break;
        default:
            err = encode_lane<kAnyUnit, kConvert>(t, off, vm, stage8, wbase, head, lane);
            err = wave_min_u64(err);
            break;
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
        u64 nbytes = tile_total;
        if (prefix >= out_cap) nbytes = 0;
        else if (prefix + nbytes > out_cap) nbytes = out_cap - prefix;
        write_out<1>(out + prefix, nbytes, stage, tid);
    }
    if (tid == 0 && arrive_last(ctrl, ntiles)) {
        const u64 e = ld_agent(&ctrl->err);
        if (e != ~0ull) {
            write_result(result, (uint32_t)(e & 15u), e >> 4);
        } else if (kConvert) {
            const u64 tot = ld_agent(&ctrl->total);
            write_result(result, tot > out_cap ? kOutputTooSmall : kOk, tot);
        } else {
            write_result(result, kOk, (u64)m);
        }
        reset_ctrl(ctrl);
    }
}

__global__ __launch_bounds__(kBlock) void utf8_length_kernel(
    const uint8_t *__restrict__ frame, long long head, long long m, Ctrl *__restrict__ ctrl,
    u64 *__restrict__ result, u64 nblocks) {
    __shared__ u64 s_sum[kWaves];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const long long end = head + m;
    u64 acc = 0;
    const long long tbase = (long long)blockIdx.x * kTileUnits + (long long)wave * kWaveUnits;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const long long q0 = tbase + r * kRowUnits + 8 * (long long)lane;
        if (q0 < end) {
            u32x4 v = __builtin_nontemporal_load((const u32x4 *)(frame + 2 * q0));
            uint32_t d[4] = {v.x, v.y, v.z, v.w};
            if (q0 < head || q0 + 8 > end)
                for (int k = 0; k < 4; ++k) d[k] = keep_units(d[k], q0 + 2 * k, head, end);
            acc += chunk_width8(d) - outside_count8(q0, head, end);
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

hipError_t launch_utf16_tiles(bool convert, const uint8_t *frame, long long head, long long m, uint8_t *out,
                              u64 out_cap, u64 *status, Ctrl *ctrl, DevResult *result, u64 ntiles,
                              hipStream_t stream) {
    if (convert)
        hipLaunchKernelGGL(utf16_tile_kernel<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, result, ntiles);
    else
        hipLaunchKernelGGL(utf16_tile_kernel<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, frame,
                           head, m, out, out_cap, status, ctrl, result, ntiles);
    return hipGetLastError();
}

hipError_t launch_utf8_length(const uint8_t *frame, long long head, long long m, Ctrl *ctrl, u64 *result,
                              hipStream_t stream) {
    const u64 nblocks = (u64)((head + m + kTileUnits - 1) / kTileUnits);
    hipLaunchKernelGGL(utf8_length_kernel, dim3((unsigned)nblocks), dim3(kBlock), 0, stream, frame, head, m,
                       ctrl, result, nblocks);
    return hipGetLastError();
}

u64 utf16_tiles_for(long long head, long long m) { return (u64)((head + m + kTileUnits - 1) / kTileUnits); }

}  // namespace utfgpu
