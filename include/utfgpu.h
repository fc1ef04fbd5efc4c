/*
 * utfgpu.h -- C ABI of the MI355X (gfx950) UTF-8 <-> UTF-16LE library.
 *
 * The library validates UTF-8 and UTF-16LE text and transcodes it in both
 * directions, always validating, as stated in Lemire, "Unicode at Gigabytes
 * per Second" (Section 1: both formats must be validated and converted;
 * Section 5: every transcoding includes validation).  The formats are the
 * ones of Section 3: UTF-8 leading-byte patterns and six validity rules, and
 * UTF-16 with surrogate pairs.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All text and result pointers are DEVICE pointers (memory of the current
 *    HIP device).  The caller owns them; the library never frees them and
 *    never writes to an input.
 *  - `stream` is a hipStream_t passed as `void*`; NULL means the default
 *    stream.  Calls on distinct streams may run concurrently (the library
 *    keeps one workspace per device and stream).  Two calls on the same
 *    stream run in stream order.
 *  - UTF-8 text is a byte array of any alignment.  UTF-16LE text and UTF-16
 *    output are arrays of 16-bit little-endian words and must be 2-byte
 *    aligned.
 *  - Sizes are counted in units of the format: bytes for UTF-8, 16-bit
 *    words for UTF-16.  Inputs may be empty (n == 0); then no kernel runs.
 *  - Synchronous calls return after the result is known (they synchronise
 *    `stream`).  The `_async` forms only enqueue work and write their result
 *    to a device pointer when the stream reaches it.
 *  - Errors never cause writes outside [out, out + out_cap).
 *
 * Result and status codes
 * -----------------------
 *  utf_result.status == UTF_OK (0): `count` is the number of input units
 *      validated (validate_*) or output units written (convert_*).
 *  1..8 (data errors): the input is invalid; `count` is the offset, in input
 *      units, of the first character that cannot be read: the length of the
 *      longest valid prefix.  The kind is the first rule of Section 3 broken
 *      by that character, checked in the order rule 1, rule 3, rule 2, then
 *      rules 4, 5, 6 on the decoded value; for UTF-16 an unpaired high or
 *      low surrogate.
 *  UTF_OUTPUT_TOO_SMALL (9): the input is valid but the conversion needs
 *      more than `out_cap` units; `count` is the number needed.  A data error
 *      takes precedence over this status.
 *  negative values: misuse or runtime failure (null pointer with n > 0,
 *      misaligned UTF-16 pointer, size above the supported maximum, HIP
 *      error); `count` is 0 and nothing was launched unless the status is
 *      UTF_ERR_HIP.
 */
#ifndef UTFGPU_H
#define UTFGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct utf_result {
    int32_t status;
    uint64_t count;
} utf_result;

enum {
    UTF_OK = 0,
    UTF_TOO_SHORT = 1,        /* rule 2: leading byte without enough continuation bytes */
    UTF_TOO_LONG = 2,         /* rule 3: continuation byte without a leading byte */
    UTF_OVERLONG = 3,         /* rule 4: value encoded with more bytes than needed */
    UTF_TOO_LARGE = 4,        /* rule 5: value of 1114112 or more */
    UTF_SURROGATE = 5,        /* rule 6: value in U+D800..U+DFFF */
    UTF_HEADER_BITS = 6,      /* rule 1: byte 0xF8..0xFF */
    UTF_UNPAIRED_HIGH = 7,    /* UTF-16: high surrogate not followed by a low one */
    UTF_UNPAIRED_LOW = 8,     /* UTF-16: low surrogate not preceded by a high one */
    UTF_OUTPUT_TOO_SMALL = 9, /* valid input, output capacity too small */
    UTF_ERR_NULL = -1,
    UTF_ERR_ALIGN = -2,
    UTF_ERR_TOO_BIG = -3,
    UTF_ERR_HIP = -4,
    UTF_ERR_OFFSETS = -5,     /* batched calls: offsets are not a partition of the input */
    UTF_ERR_ARG = -6          /* tuning calls: operation, size class, geometry or schedule out of range */
};

/* Largest supported input: 2^40 - 1 UTF-8 bytes, 2^38 - 1 UTF-16 words. */
#define UTF_MAX_UTF8_BYTES ((uint64_t)1 << 40)
#define UTF_MAX_UTF16_WORDS ((uint64_t)1 << 38)
/* Largest number of strings of one batched call. */
#define UTF_MAX_BATCH_STRINGS ((uint64_t)1 << 31)

/* ---------------------------------------------------------------------- */
/* Validation (Section 3 rules)                                           */
/* ---------------------------------------------------------------------- */

/* Validate n bytes of UTF-8 at `in`.  {UTF_OK, n} or {kind, first error}. */
utf_result validate_utf8(const uint8_t *in, uint64_t n, void *stream);

/* Validate m 16-bit words of UTF-16LE at `in` (2-byte aligned). */
utf_result validate_utf16le(const uint16_t *in, uint64_t m, void *stream);

/* ---------------------------------------------------------------------- */
/* Output lengths                                                         */
/* ---------------------------------------------------------------------- */

/*
 * Number of UTF-16 words the conversion of `in` writes: one per byte that is
 * not a continuation byte (10xxxxxx), plus one more per byte >= 0xF0 (a
 * four-byte character becomes a surrogate pair).  Exact for valid input;
 * defined by the same per-byte count for any input.  Does not validate.
 * Returns UINT64_MAX on misuse or HIP error.
 */
uint64_t utf16_length_from_utf8(const uint8_t *in, uint64_t n, void *stream);

/*
 * Number of UTF-8 bytes the conversion of `in` writes: 1 per word below
 * 0x80, 2 below 0x800, 2 per surrogate word (4 per pair), 3 otherwise.
 * Exact for valid input; same per-word count for any input.  Does not
 * validate.  Returns UINT64_MAX on misuse or HIP error.
 */
uint64_t utf8_length_from_utf16le(const uint16_t *in, uint64_t m, void *stream);

/* ---------------------------------------------------------------------- */
/* Conversions (always validating)                                        */
/* ---------------------------------------------------------------------- */

/*
 * UTF-8 -> UTF-16LE.  `out` has room for `out_cap` words (2-byte aligned;
 * may be NULL when out_cap == 0).  Returns {UTF_OK, words written},
 * {kind, first error} or {UTF_OUTPUT_TOO_SMALL, words needed}.  On a data
 * error, out[0 .. words of the valid prefix) holds the conversion of the
 * valid prefix (cut at out_cap); other output words inside out_cap are
 * unspecified.  On UTF_OUTPUT_TOO_SMALL out[0 .. out_cap) holds the first
 * out_cap words of the conversion.  out_cap >= n always suffices.
 */
utf_result convert_utf8_to_utf16le(const uint8_t *in, uint64_t n, uint16_t *out,
                                   uint64_t out_cap, void *stream);

/*
 * UTF-16LE -> UTF-8, same conventions with `out_cap` in bytes.
 * out_cap >= 3 * m always suffices.
 */
utf_result convert_utf16le_to_utf8(const uint16_t *in, uint64_t m, uint8_t *out,
                                   uint64_t out_cap, void *stream);

/* ---------------------------------------------------------------------- */
/* Asynchronous forms                                                     */
/* ---------------------------------------------------------------------- */

/*
 * Same work as the synchronous calls, enqueued on `stream` without waiting.
 * The result is written to the device pointer `result` (a utf_result, or a
 * uint64_t for the length queries) when the stream reaches it.  The return
 * value is UTF_OK when the work was enqueued, or a negative status (nothing
 * enqueued).  For n == 0 the result is written with a small device copy.
 */
int32_t validate_utf8_async(const uint8_t *in, uint64_t n, utf_result *result, void *stream);
int32_t validate_utf16le_async(const uint16_t *in, uint64_t m, utf_result *result, void *stream);
int32_t utf16_length_from_utf8_async(const uint8_t *in, uint64_t n, uint64_t *result, void *stream);
int32_t utf8_length_from_utf16le_async(const uint16_t *in, uint64_t m, uint64_t *result, void *stream);
int32_t convert_utf8_to_utf16le_async(const uint8_t *in, uint64_t n, uint16_t *out,
                                      uint64_t out_cap, utf_result *result, void *stream);
int32_t convert_utf16le_to_utf8_async(const uint16_t *in, uint64_t m, uint8_t *out,
                                      uint64_t out_cap, utf_result *result, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched conversion (many strings in one call)                          */
/* ---------------------------------------------------------------------- */

/*
 * UTF-8 -> UTF-16LE of k strings packed back to back in `in`: string i is
 * in[offsets[i] .. offsets[i+1]), with offsets[0] == 0 and offsets[k] == n
 * (k + 1 device int64 values, non-decreasing; empty strings allowed).
 * Each string is validated and converted on its own, as by
 * convert_utf8_to_utf16le (Section 3 rules; a string's first byte
 * continues nothing before it and its last character must end inside it),
 * and all of them in one pass over the buffer.
 *
 * Output is compact: string i's words start at out_offsets[i], the sum of
 * utf16_length_from_utf8 of strings 0 .. i-1; out_offsets[k] is the total.
 * `out` has room for `out_cap` words (2-byte aligned).  results[i] (device
 * array of k) is {UTF_OK, words}, {kind, first error inside the string} or
 * {UTF_OUTPUT_TOO_SMALL, words} when the string's words do not all fit
 * below out_cap.  A valid string's words are exact; words in the range of
 * an invalid string are unspecified.  If `offsets` is not a partition of
 * the input every result is {UTF_ERR_OFFSETS, 0} and out_offsets holds 0s
 * (k == 0 with n > 0: the call returns UTF_ERR_OFFSETS and enqueues nothing).
 *
 * Asynchronous on `stream`, like the *_async calls; every pointer except
 * the stream is device memory.  Returns UTF_OK when enqueued, or a negative
 * status.  Work space (a bitmap of string starts, per-string error words,
 * per-tile and per-block offsets) is kept by the library per stream; calls
 * on one stream are ordered, calls on different streams do not share it.
 */
int32_t convert_utf8_to_utf16le_batch_async(const uint8_t *in, uint64_t n, const int64_t *offsets,
                                            uint64_t k, uint16_t *out, uint64_t out_cap,
                                            int64_t *out_offsets, utf_result *results, void *stream);

/*
 * UTF-16LE -> UTF-8 of k strings packed back to back in `in` (2-byte
 * aligned), string i being in[offsets[i] .. offsets[i+1]) in 16-bit units,
 * offsets[0] == 0, offsets[k] == m.  Each string is validated and
 * converted on its own, as by convert_utf16le_to_utf8 (Section 3; a high
 * surrogate at a string's end and a low surrogate at a string's start are
 * unpaired whatever the neighbouring string holds).  out_offsets[i] (bytes)
 * is the sum of utf8_length_from_utf16le of strings 0 .. i-1; results[i]
 * is {UTF_OK, bytes}, {UTF_UNPAIRED_HIGH or _LOW, first error in units
 * inside the string} or {UTF_OUTPUT_TOO_SMALL, bytes}.  Same conventions
 * as the UTF-8 form otherwise.
 */
int32_t convert_utf16le_to_utf8_batch_async(const uint16_t *in, uint64_t m, const int64_t *offsets,
                                            uint64_t k, uint8_t *out, uint64_t out_cap,
                                            int64_t *out_offsets, utf_result *results, void *stream);

/* ---------------------------------------------------------------------- */
/* Allocation-free conversion                                             */
/* ---------------------------------------------------------------------- */

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * same work and results as convert_utf8_to_utf16le_async, with the look-back
 * status words and control block in a fixed array of device memory that the
 * library holds on each device until the process ends (16 MiB + 256 bytes)
 * instead of a per-stream workspace.  The call allocates nothing; its first
 * call on a device looks the array's address up and initialises it with a
 * kernel on `stream`.  At most UTF_NOALLOC_MAX_TILES tiles: with the shipped
 * geometry table, inputs of up to 2 GiB - 64 bytes; a larger input returns
 * UTF_ERR_TOO_BIG and enqueues nothing.  Every call on a device shares that
 * device's array: calls that overlap on one device (different streams, or
 * different host threads, without ordering between them) race and give
 * undefined results; calls ordered on one stream are safe.  Arguments and
 * return value as convert_utf8_to_utf16le_async.
 */
#define UTF_NOALLOC_MAX_TILES 65536
int32_t convert_utf8_to_utf16le_noalloc_async(const uint8_t *in, uint64_t n, uint16_t *out, uint64_t out_cap,
                                              utf_result *result, void *stream);

/* ---------------------------------------------------------------------- */
/* Library state                                                          */
/* ---------------------------------------------------------------------- */

/*
 * Free every workspace the library holds (per device and stream: tile
 * status words, control block, result slots).  Must not overlap with calls
 * in flight.  Later calls allocate again.  Returns UTF_OK or UTF_ERR_HIP.
 */
int32_t utfgpu_release_workspace(void);

/* ---------------------------------------------------------------------- */
/* Tile geometry and its tuning table                                     */
/* ---------------------------------------------------------------------- */

/*
 * The validate and convert kernels are compiled for several tile
 * geometries: a workgroup of `waves` wave64 waves, each lane of which loads
 * `rows` 16-byte chunks, covers `tile_bytes` = waves * rows * 1024 input
 * bytes (UTF-8 bytes, or UTF-16LE bytes: half as many words).  Geometry 0
 * (8 waves x 4 rows, 32 KiB) serves most calls; smaller tiles put more
 * workgroups on small inputs.  Every geometry computes the same results:
 * the choice only changes speed.
 *
 * Which geometry a call uses is looked up in a process-wide table indexed by
 * operation (UTF_OP_*) and input size class: the class of b input bytes is
 * ceil(log2(b)) (0 for b <= 1), clamped to UTF_SIZE_CLASSES - 1; UTF-16
 * inputs count 2 bytes per word and batched calls their whole input.  The
 * table starts at the shipped defaults, measured on MI355X over text of five
 * scripts: conversions of up to 4 MiB (class <= 22; batched UTF-8 calls up
 * to 16 MiB) use 4 waves x 2 rows (8 KiB tiles), larger batched UTF-16LE
 * calls 4 waves x 4 rows (16 KiB tiles, which share CUs better with
 * concurrent calls on other streams), everything else geometry 0.  The
 * environment variable
 * UTFGPU_GEOMETRY, set to a geometry index before the first call, overrides
 * the table for the whole process.  The table is host state: these calls
 * need no GPU, may be made from any thread and take effect on the next
 * call that looks the table up (a call in flight keeps its geometry).
 */
enum {
    UTF_OP_VALIDATE_UTF8 = 0,       /* validate_utf8[_async] */
    UTF_OP_CONVERT_UTF8 = 1,        /* convert_utf8_to_utf16le[_async] */
    UTF_OP_VALIDATE_UTF16LE = 2,    /* validate_utf16le[_async] */
    UTF_OP_CONVERT_UTF16LE = 3,     /* convert_utf16le_to_utf8[_async] */
    UTF_OP_BATCH_UTF8 = 4,          /* convert_utf8_to_utf16le_batch_async */
    UTF_OP_BATCH_UTF16LE = 5,       /* convert_utf16le_to_utf8_batch_async */
    UTF_OP_COUNT = 6
};
#define UTF_SIZE_CLASSES 64

/* Number of compiled geometries (at least 1). */
int32_t utfgpu_geometry_count(void);

/* Shape of geometry g: any of the output pointers may be null.  UTF_OK, or
 * UTF_ERR_ARG if g is out of range. */
int32_t utfgpu_geometry(int32_t g, uint32_t *waves, uint32_t *rows, uint64_t *tile_bytes);

/* Make calls of operation `op` whose input falls in `size_class` use
 * geometry g (-1 restores the shipped default).  UTF_OK or UTF_ERR_ARG. */
int32_t utfgpu_set_geometry(int32_t op, int32_t size_class, int32_t g);

/* The geometry such a call uses now (UTFGPU_GEOMETRY included), or
 * UTF_ERR_ARG. */
int32_t utfgpu_get_geometry(int32_t op, int32_t size_class);

/* The size class of an input of `bytes` bytes. */
int32_t utfgpu_size_class(uint64_t bytes);

/* ---------------------------------------------------------------------- */
/* Scan schedule and its tuning table                                     */
/* ---------------------------------------------------------------------- */

/*
 * The validate and convert kernels find each tile's output offset with a
 * single-pass scan over the tiles (each tile publishes its total and reads
 * its predecessors' totals and prefixes: the decoupled look-back, the
 * device-wide form of the output-offset computation that the paper's
 * sequential loop carries from block to block, Section 4).  The schedule is
 * the order in which workgroups take tiles:
 *   UTF_SCHEDULE_BLOCK   tile = workgroup index (no shared counter);
 *   UTF_SCHEDULE_TICKET  each workgroup takes the next index of a per-call
 *                        counter when it starts, so every tile before a
 *                        running tile belongs to a workgroup that has
 *                        already started and no look-back ever waits on a
 *                        workgroup the hardware has not placed (which
 *                        happens while look-back kernels of other streams
 *                        fill the device).
 * Both compute the same results; tickets cost one atomic round trip before
 * each tile's first load.  Validation has no scan: the entries of the two
 * validate operations are kept but do not change what runs.  A process-wide table (operation, size class, as
 * for the geometry) picks the schedule per call; the shipped default is
 * UTF_SCHEDULE_BLOCK everywhere (faster on MI355X alone and, with the
 * shipped geometries, for four concurrent serving streams).  The
 * environment variable UTFGPU_SCHEDULE, set to a schedule index before the
 * first call, overrides the table for the whole process.  Host state: no
 * GPU needed, any thread, effective from the next call.
 */
enum {
    UTF_SCHEDULE_BLOCK = 0,
    UTF_SCHEDULE_TICKET = 1,
    UTF_SCHEDULE_COUNT = 2
};

/* Make calls of operation `op` whose input falls in `size_class` use scan
 * schedule `schedule` (-1 restores the shipped default).  UTF_OK or
 * UTF_ERR_ARG. */
int32_t utfgpu_set_schedule(int32_t op, int32_t size_class, int32_t schedule);

/* The schedule such a call uses now (UTFGPU_SCHEDULE included), or
 * UTF_ERR_ARG. */
int32_t utfgpu_get_schedule(int32_t op, int32_t size_class);

/* Library version string, e.g. "utfgpu 0.2 gfx950". */
const char *utfgpu_version(void);

/* Input bytes one workgroup of the validate/convert kernels covers in the
 * geometry 0 (a tile of UTF-8 bytes, or of UTF-16LE bytes: half as
 * many words).  Informational: tests use it to place inputs across tile
 * boundaries.  Needs no GPU. */
uint64_t utfgpu_tile_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* UTFGPU_H */
