/*
 * Oracle for the compressed interest-vector encoding (section "Private
 * Notifications": clients fetch compressed Bloom-filter deltas; the paper
 * gives no format). TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke
 * check and the benchmark's CPU baseline; the product path never links it.
 *
 * Reading taken: Golomb-Rice coding of the gaps between set bits, the usual
 * code for sparse bit sets. Stream, little-endian:
 *   bytes 0-7   m, the vector's length in bits
 *   bytes 8-15  c, the number of set bits
 *   bytes 16-19 k, the Rice parameter: floor(log2(max(1, floor(m / (c + 1)))))
 *   bytes 20-23 zero
 *   then, for the set positions p_0 < ... < p_{c-1} and p_{-1} = -1, the
 *   gap g_i = p_i - p_{i-1} - 1 as floor(g_i / 2^k) one-bits, one zero-bit and
 *   the k low bits of g_i, least significant first; bits fill bytes
 *   least-significant bit first; the last byte's unused bits are zero.
 */
#include <stdint.h>
#include <string.h>

enum { HEADER = 24 };

static int bit_of(const uint8_t *v, uint64_t p) { return (v[p >> 3] >> (p & 7)) & 1; }

static uint32_t rice_k(uint64_t m, uint64_t c)
{
    uint64_t mean = m / (c + 1);
    if (mean < 1)
        mean = 1;
    uint32_t k = 0;
    while ((mean >> (k + 1)) != 0)
        ++k;
    return k;
}

static void put_bit(uint8_t *body, uint64_t at, int b)
{
    if (b)
        body[at >> 3] |= (uint8_t)(1u << (at & 7));
}

/* Encode the m-bit vector v (ceil(m/8) bytes, bit p = byte p>>3, bit p&7).
 * Returns the stream length; writes it into out when it fits in cap (out may
 * be NULL to ask for the length only). */
uint64_t oracle_iv_encode(const uint8_t *v, uint64_t m, uint8_t *out, uint64_t cap)
{
    uint64_t c = 0;
    for (uint64_t p = 0; p < m; ++p)
        c += (uint64_t)bit_of(v, p);
    const uint32_t k = rice_k(m, c);
    uint64_t bits = 0, prev = (uint64_t)-1;
    for (uint64_t p = 0; p < m; ++p)
        if (bit_of(v, p)) {
            const uint64_t g = p - prev - 1;
            bits += (g >> k) + 1 + k;
            prev = p;
        }
    const uint64_t len = HEADER + (bits + 7) / 8;
    if (!out || cap < len)
        return len;
    memset(out, 0, len);
    for (int i = 0; i < 8; ++i) {
        out[i] = (uint8_t)(m >> (8 * i));
        out[8 + i] = (uint8_t)(c >> (8 * i));
    }
    for (int i = 0; i < 4; ++i)
        out[16 + i] = (uint8_t)(k >> (8 * i));
    uint8_t *body = out + HEADER;
    uint64_t at = 0;
    prev = (uint64_t)-1;
    for (uint64_t p = 0; p < m; ++p) {
        if (!bit_of(v, p))
            continue;
        const uint64_t g = p - prev - 1;
        for (uint64_t q = g >> k; q > 0; --q)
            put_bit(body, at++, 1);
        put_bit(body, at++, 0);
        for (uint32_t b = 0; b < k; ++b)
            put_bit(body, at++, (int)((g >> b) & 1));
        prev = p;
    }
    return len;
}

/* Decode a stream into v (ceil(m/8) bytes, m from the header, at most
 * v_bytes). Returns m, or (uint64_t)-1 for a malformed or truncated stream,
 * or when v is too small. */
uint64_t oracle_iv_decode(const uint8_t *s, uint64_t len, uint8_t *v, uint64_t v_bytes)
{
    if (len < HEADER)
        return (uint64_t)-1;
    uint64_t m = 0, c = 0;
    uint32_t k = 0;
    for (int i = 7; i >= 0; --i) {
        m = (m << 8) | s[i];
        c = (c << 8) | s[8 + i];
    }
    for (int i = 3; i >= 0; --i)
        k = (k << 8) | s[16 + i];
    if ((m + 7) / 8 > v_bytes || k > 63 || c > m)
        return (uint64_t)-1;
    memset(v, 0, (m + 7) / 8);
    const uint8_t *body = s + HEADER;
    const uint64_t nbits = (len - HEADER) * 8;
    uint64_t at = 0, prev = (uint64_t)-1;
    for (uint64_t i = 0; i < c; ++i) {
        uint64_t q = 0;
        for (;;) {
            if (at >= nbits)
                return (uint64_t)-1;
            if (!bit_of(body, at++))
                break;
            ++q;
        }
        uint64_t r = 0;
        for (uint32_t b = 0; b < k; ++b) {
            if (at >= nbits)
                return (uint64_t)-1;
            r |= (uint64_t)bit_of(body, at++) << b;
        }
        const uint64_t p = prev + 1 + (q << k) + r;
        if (p >= m)
            return (uint64_t)-1;
        v[p >> 3] |= (uint8_t)(1u << (p & 7));
        prev = p;
    }
    return m;
}
