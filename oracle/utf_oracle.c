/*
 * utf_oracle.c -- plain, slow, scalar reference codec for UTF-8 <-> UTF-16LE.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * What it follows (Lemire, "Unicode at Gigabytes per Second", Section 3):
 *   - UTF-8 leading-byte patterns 0 / 110 / 1110 / 11110 give a sequence of
 *     1 / 2 / 3 / 4 bytes; every following byte of the sequence is a
 *     continuation byte 10xxxxxx; the code point's most significant bits sit
 *     in the leading byte, its least significant bits in the last byte.
 *   - The six validity rules, checked in the paper's order: (1) no byte has
 *     its five most significant bits all ones; (2) a leading byte is followed
 *     by the right number of continuation bytes; (3) a continuation byte needs
 *     a leading byte; (4) shortest form: above U+7F / U+7FF / U+FFFF for
 *     2 / 3 / 4-byte sequences; (5) the value is below 1114112; (6) the value
 *     is not in U+D800..U+DFFF.
 *   - UTF-16: U+0000..D7FF and U+E000..FFFF are one 16-bit word; U+10000..
 *     10FFFF is a high word D800..DBFF followed by a low word DC00..DFFF, the
 *     value being 0x10000 plus the ten low bits of the high word (upper part)
 *     and of the low word (lower part).  Only surrogates need checking.
 *
 * Readings where the paper is silent (each is listed in the design doc):
 *   - The error position is the length of the longest valid prefix, counted
 *     in input units (bytes for UTF-8, 16-bit words for UTF-16): a plain
 *     left-to-right decoder stops at the first character it cannot read.
 *   - The error kind is the first rule, in the paper's numbering with the
 *     structural rules (1, 3, 2) checked before the value rules (4, 5, 6),
 *     that the character at the error position breaks.
 *   - A sequence cut off by the end of the buffer breaks rule 2.
 *   - The length queries return, for any input, the number of output units a
 *     character-by-character conversion would produce if every leading byte
 *     (or word) were read with the length its bit pattern announces; for
 *     valid input this is exactly the number of units a conversion writes.
 *   - UTF-16LE words are assembled from bytes explicitly (low byte first), so
 *     the oracle does not depend on host byte order.
 *
 * Status codes (the oracle's own copy of the convention):
 *   0 OK, 1 TOO_SHORT (rule 2), 2 TOO_LONG (rule 3), 3 OVERLONG (rule 4),
 *   4 TOO_LARGE (rule 5), 5 SURROGATE (rule 6), 6 HEADER_BITS (rule 1),
 *   7 UNPAIRED_HIGH, 8 UNPAIRED_LOW, 9 OUTPUT_TOO_SMALL.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>

enum {
    OR_OK = 0,
    OR_TOO_SHORT = 1,
    OR_TOO_LONG = 2,
    OR_OVERLONG = 3,
    OR_TOO_LARGE = 4,
    OR_SURROGATE = 5,
    OR_HEADER_BITS = 6,
    OR_UNPAIRED_HIGH = 7,
    OR_UNPAIRED_LOW = 8,
    OR_OUTPUT_TOO_SMALL = 9
};

typedef struct {
    int32_t status;
    uint64_t count;
} oracle_result;

/* ------------------------------------------------------------------------ */
/* Reading one character                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Read the UTF-8 character that starts at s[i] (Section 3).  On success store
 * its code point and byte length and return OR_OK; otherwise return the kind
 * of the first rule it breaks.
 */
static int read_utf8_char(const uint8_t *s, size_t n, size_t i,
                          uint32_t *cp_out, int *len_out)
{
    uint8_t lead = s[i];
    int len;
    uint32_t cp;

    /* The leading byte's most significant bits announce the length. */
    if ((lead & 0x80) == 0x00) {
        len = 1;
    } else if ((lead & 0xF8) == 0xF8) {
        return OR_HEADER_BITS;          /* rule 1: 11111xxx */
    } else if ((lead & 0xC0) == 0x80) {
        return OR_TOO_LONG;             /* rule 3: 10xxxxxx with no lead */
    } else if ((lead & 0xE0) == 0xC0) {
        len = 2;                        /* 110xxxxx */
    } else if ((lead & 0xF0) == 0xE0) {
        len = 3;                        /* 1110xxxx */
    } else {
        len = 4;                        /* 11110xxx */
    }

    /* Rule 2: the right number of continuation bytes must follow. */
    for (int k = 1; k < len; k++) {
        if (i + (size_t)k >= n)
            return OR_TOO_SHORT;
        if ((s[i + k] & 0xC0) != 0x80)
            return OR_TOO_SHORT;
    }

    /* Bit layout: leading-byte payload first, then 6 bits per continuation. */
    if (len == 1)
        cp = lead & 0x7F;
    else if (len == 2)
        cp = lead & 0x1F;
    else if (len == 3)
        cp = lead & 0x0F;
    else
        cp = lead & 0x07;
    for (int k = 1; k < len; k++)
        cp = (cp << 6) | (uint32_t)(s[i + k] & 0x3F);

    /* Rule 4: shortest form. */
    if (len == 2 && cp <= 0x7F)
        return OR_OVERLONG;
    if (len == 3 && cp <= 0x7FF)
        return OR_OVERLONG;
    if (len == 4 && cp <= 0xFFFF)
        return OR_OVERLONG;
    /* Rule 5: below 1114112. */
    if (cp >= 1114112)
        return OR_TOO_LARGE;
    /* Rule 6: no surrogate values. */
    if (cp >= 0xD800 && cp <= 0xDFFF)
        return OR_SURROGATE;

    *cp_out = cp;
    *len_out = len;
    return OR_OK;
}

/* Word i of a UTF-16LE byte array: low byte first. */
static uint32_t word_at(const uint8_t *s, size_t i)
{
    return (uint32_t)s[2 * i] | ((uint32_t)s[2 * i + 1] << 8);
}

/*
 * Read the UTF-16 character that starts at word i (Section 3).  A high
 * surrogate must be followed by a low one; a low one may not start a
 * character.
 */
static int read_utf16_char(const uint8_t *s, size_t m, size_t i,
                           uint32_t *cp_out, int *len_out)
{
    uint32_t w = word_at(s, i);
    if (w < 0xD800 || w > 0xDFFF) {
        *cp_out = w;
        *len_out = 1;
        return OR_OK;
    }
    if (w >= 0xDC00)
        return OR_UNPAIRED_LOW;
    if (i + 1 >= m)
        return OR_UNPAIRED_HIGH;
    uint32_t w2 = word_at(s, i + 1);
    if (w2 < 0xDC00 || w2 > 0xDFFF)
        return OR_UNPAIRED_HIGH;
    *cp_out = 0x10000 + (((w & 0x3FF) << 10) | (w2 & 0x3FF));
    *len_out = 2;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Writing one character                                                    */
/* ------------------------------------------------------------------------ */

/* UTF-16 words for a code point: one word, or a surrogate pair. */
static int utf16_words(uint32_t cp, uint16_t w[2])
{
    if (cp < 0x10000) {
        w[0] = (uint16_t)cp;
        return 1;
    }
    uint32_t v = cp - 0x10000;
    w[0] = (uint16_t)(0xD800 | (v >> 10));
    w[1] = (uint16_t)(0xDC00 | (v & 0x3FF));
    return 2;
}

/* UTF-8 bytes for a code point, length chosen by value range. */
static int utf8_bytes(uint32_t cp, uint8_t b[4])
{
    if (cp <= 0x7F) {
        b[0] = (uint8_t)cp;
        return 1;
    }
    if (cp <= 0x7FF) {
        b[0] = (uint8_t)(0xC0 | (cp >> 6));
        b[1] = (uint8_t)(0x80 | (cp & 0x3F));
        return 2;
    }
    if (cp <= 0xFFFF) {
        b[0] = (uint8_t)(0xE0 | (cp >> 12));
        b[1] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
        b[2] = (uint8_t)(0x80 | (cp & 0x3F));
        return 3;
    }
    b[0] = (uint8_t)(0xF0 | (cp >> 18));
    b[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
    b[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
    b[3] = (uint8_t)(0x80 | (cp & 0x3F));
    return 4;
}

/* ------------------------------------------------------------------------ */
/* Validation                                                               */
/* ------------------------------------------------------------------------ */

oracle_result oracle_validate_utf8(const uint8_t *s, uint64_t n)
{
    oracle_result r = {OR_OK, n};
    size_t i = 0;
    while (i < n) {
        uint32_t cp;
        int len;
        int st = read_utf8_char(s, n, i, &cp, &len);
        if (st != OR_OK) {
            r.status = st;
            r.count = i;
            return r;
        }
        i += (size_t)len;
    }
    return r;
}

oracle_result oracle_validate_utf16le(const uint8_t *s, uint64_t m)
{
    oracle_result r = {OR_OK, m};
    size_t i = 0;
    while (i < m) {
        uint32_t cp;
        int len;
        int st = read_utf16_char(s, m, i, &cp, &len);
        if (st != OR_OK) {
            r.status = st;
            r.count = i;
            return r;
        }
        i += (size_t)len;
    }
    return r;
}

/* ------------------------------------------------------------------------ */
/* Length queries                                                           */
/* ------------------------------------------------------------------------ */

/*
 * UTF-16 words produced from a UTF-8 buffer: each leading byte announces a
 * character; 4-byte characters (lead 11110xxx and above) need a surrogate
 * pair, every other character one word.  Continuation bytes add nothing.
 */
uint64_t oracle_utf16_length_from_utf8(const uint8_t *s, uint64_t n)
{
    uint64_t words = 0;
    for (size_t i = 0; i < n; i++) {
        uint8_t b = s[i];
        if ((b & 0xC0) == 0x80)
            continue;
        words += 1;
        if (b >= 0xF0)
            words += 1;
    }
    return words;
}

/*
 * UTF-8 bytes produced from a UTF-16 buffer: 1 byte below U+80, 2 below
 * U+800, 3 for the rest of the basic plane, 4 for a surrogate pair (counted
 * as 2 per surrogate word).
 */
uint64_t oracle_utf8_length_from_utf16le(const uint8_t *s, uint64_t m)
{
    uint64_t bytes = 0;
    for (size_t i = 0; i < m; i++) {
        uint32_t w = word_at(s, i);
        if (w <= 0x7F)
            bytes += 1;
        else if (w <= 0x7FF)
            bytes += 2;
        else if (w >= 0xD800 && w <= 0xDFFF)
            bytes += 2;
        else
            bytes += 3;
    }
    return bytes;
}

/* ------------------------------------------------------------------------ */
/* Conversions                                                              */
/* ------------------------------------------------------------------------ */

/*
 * UTF-8 -> UTF-16LE.  Validate and decode character by character; write the
 * words of every character of the valid prefix.  Output words are stored as
 * little-endian byte pairs in `out` (capacity `cap` words).
 *
 * Result: {OK, words} when valid and it fits; {kind, position} on the first
 * invalid character (out holds the conversion of the valid prefix, cut at
 * cap); {OUTPUT_TOO_SMALL, words needed} when valid but longer than cap (out
 * holds the first cap words of the conversion).
 */
oracle_result oracle_convert_utf8_to_utf16le(const uint8_t *s, uint64_t n,
                                             uint8_t *out, uint64_t cap)
{
    oracle_result r = {OR_OK, 0};
    size_t i = 0;
    uint64_t o = 0;
    while (i < n) {
        uint32_t cp;
        int len;
        int st = read_utf8_char(s, n, i, &cp, &len);
        if (st != OR_OK) {
            r.status = st;
            r.count = i;
            return r;
        }
        uint16_t w[2];
        int k = utf16_words(cp, w);
        for (int j = 0; j < k; j++) {
            if (o < cap) {
                out[2 * o] = (uint8_t)(w[j] & 0xFF);
                out[2 * o + 1] = (uint8_t)(w[j] >> 8);
            }
            o++;
        }
        i += (size_t)len;
    }
    if (o > cap) {
        r.status = OR_OUTPUT_TOO_SMALL;
        r.count = o;
        return r;
    }
    r.count = o;
    return r;
}

/*
 * UTF-16LE -> UTF-8, same conventions; `cap` and the counts are in bytes on
 * the output side and in words on the input side.
 */
oracle_result oracle_convert_utf16le_to_utf8(const uint8_t *s, uint64_t m,
                                             uint8_t *out, uint64_t cap)
{
    oracle_result r = {OR_OK, 0};
    size_t i = 0;
    uint64_t o = 0;
    while (i < m) {
        uint32_t cp;
        int len;
        int st = read_utf16_char(s, m, i, &cp, &len);
        if (st != OR_OK) {
            r.status = st;
            r.count = i;
            return r;
        }
        uint8_t b[4];
        int k = utf8_bytes(cp, b);
        for (int j = 0; j < k; j++) {
            if (o < cap)
                out[o] = b[j];
            o++;
        }
        i += (size_t)len;
    }
    if (o > cap) {
        r.status = OR_OUTPUT_TOO_SMALL;
        r.count = o;
        return r;
    }
    r.count = o;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Many independent strings                                                 */
/* ------------------------------------------------------------------------ */

/*
 * Batched forms: k independent strings, string j occupying input units
 * [offsets[j], offsets[j+1]).  Each string is handled exactly as a single
 * call would handle it.  The output of string j starts at out_offsets[j],
 * which is the sum of the length-query values of strings 0..j-1, and has
 * room for its own length-query value.  out_offsets has k+1 entries and is
 * written by these functions.
 */
void oracle_validate_utf8_batch(const uint8_t *s, const int64_t *offsets,
                                uint64_t k, oracle_result *results)
{
    for (uint64_t j = 0; j < k; j++)
        results[j] = oracle_validate_utf8(s + offsets[j],
                                          (uint64_t)(offsets[j + 1] - offsets[j]));
}

void oracle_validate_utf16le_batch(const uint8_t *s, const int64_t *offsets,
                                   uint64_t k, oracle_result *results)
{
    for (uint64_t j = 0; j < k; j++)
        results[j] = oracle_validate_utf16le(s + 2 * offsets[j],
                                             (uint64_t)(offsets[j + 1] - offsets[j]));
}

void oracle_convert_utf8_to_utf16le_batch(const uint8_t *s,
                                          const int64_t *offsets, uint64_t k,
                                          uint8_t *out, int64_t *out_offsets,
                                          oracle_result *results)
{
    int64_t o = 0;
    for (uint64_t j = 0; j < k; j++) {
        const uint8_t *str = s + offsets[j];
        uint64_t len = (uint64_t)(offsets[j + 1] - offsets[j]);
        uint64_t room = oracle_utf16_length_from_utf8(str, len);
        out_offsets[j] = o;
        results[j] = oracle_convert_utf8_to_utf16le(str, len, out + 2 * o, room);
        o += (int64_t)room;
    }
    out_offsets[k] = o;
}

void oracle_convert_utf16le_to_utf8_batch(const uint8_t *s,
                                          const int64_t *offsets, uint64_t k,
                                          uint8_t *out, int64_t *out_offsets,
                                          oracle_result *results)
{
    int64_t o = 0;
    for (uint64_t j = 0; j < k; j++) {
        const uint8_t *str = s + 2 * offsets[j];
        uint64_t len = (uint64_t)(offsets[j + 1] - offsets[j]);
        uint64_t room = oracle_utf8_length_from_utf16le(str, len);
        out_offsets[j] = o;
        results[j] = oracle_convert_utf16le_to_utf8(str, len, out + o, room);
        o += (int64_t)room;
    }
    out_offsets[k] = o;
}
