/*
 * Oracle for the serialized-PIR mask (section "Serialized PIR", steps 6 to 9).
 * TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
 * the CPU-baseline leg of bench.py; the product path never links it.
 *
 * Each server answers a request q with R XOR P, where P = PRNG(p) is a
 * one-time mask of the answer's size drawn from a per-request seed p; the
 * leader XORs the l masked answers and the client removes the l masks. The
 * paper leaves the PRNG open. Reading taken: the ChaCha20 stream cipher
 * (D. J. Bernstein, "ChaCha, a variant of Salsa20", 2008, in the IETF form of
 * RFC 8439: 32-byte key, 32-bit block counter, 96-bit nonce) with the seed as
 * key, an all-zero nonce and the block counter starting at 0; P is the first
 * d * z bytes of that keystream.
 *
 * Written from the cipher's definition: the state is four constant words
 * ("expand 32-byte k"), eight key words, the counter and three nonce words,
 * all little-endian; twenty rounds alternate four column and four diagonal
 * quarter-rounds (a += b; d ^= a; d <<<= 16; c += d; b ^= c; b <<<= 12;
 * a += b; d ^= a; d <<<= 8; c += d; b ^= c; b <<<= 7); the block is the
 * final state plus the initial state, serialized little-endian.
 */
#include <stdint.h>
#include <string.h>

static uint32_t rotl(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

static uint32_t load_le(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static void quarter(uint32_t *x, int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl(x[b], 7);
}

/* One 64-byte keystream block for a 32-byte key, a block counter and a
 * 12-byte nonce. */
void oracle_chacha20_block(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12], uint8_t out[64])
{
    uint32_t s[16], x[16];
    s[0] = 0x61707865u; /* "expa" */
    s[1] = 0x3320646eu; /* "nd 3" */
    s[2] = 0x79622d32u; /* "2-by" */
    s[3] = 0x6b206574u; /* "te k" */
    for (int i = 0; i < 8; ++i)
        s[4 + i] = load_le(key + 4 * i);
    s[12] = counter;
    for (int i = 0; i < 3; ++i)
        s[13 + i] = load_le(nonce + 4 * i);
    memcpy(x, s, sizeof s);
    for (int r = 0; r < 10; ++r) {
        quarter(x, 0, 4, 8, 12);  /* columns */
        quarter(x, 1, 5, 9, 13);
        quarter(x, 2, 6, 10, 14);
        quarter(x, 3, 7, 11, 15);
        quarter(x, 0, 5, 10, 15); /* diagonals */
        quarter(x, 1, 6, 11, 12);
        quarter(x, 2, 7, 8, 13);
        quarter(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) {
        const uint32_t v = x[i] + s[i];
        out[4 * i] = (uint8_t)v;
        out[4 * i + 1] = (uint8_t)(v >> 8);
        out[4 * i + 2] = (uint8_t)(v >> 16);
        out[4 * i + 3] = (uint8_t)(v >> 24);
    }
}

/* len bytes of keystream starting at block `counter`. */
void oracle_chacha20_stream(const uint8_t key[32], const uint8_t nonce[12], uint32_t counter, uint8_t *out,
                            uint64_t len)
{
    uint8_t blk[64];
    for (uint64_t off = 0; off < len; off += 64, ++counter) {
        oracle_chacha20_block(key, counter, nonce, blk);
        const uint64_t take = len - off < 64 ? len - off : 64;
        memcpy(out + off, blk, take);
    }
}

/* The serialized-PIR server answer, step 7: resp[r] ^= P(seed[r]) over
 * row_bytes bytes of each row (resp holds the plain answers on entry). */
void oracle_apply_masks(uint8_t *resp, uint64_t row_bytes, uint32_t B, const uint8_t *seeds)
{
    static const uint8_t zero_nonce[12] = {0};
    uint8_t blk[64];
    for (uint32_t r = 0; r < B; ++r) {
        uint8_t *row = resp + (uint64_t)r * row_bytes;
        uint32_t counter = 0;
        for (uint64_t off = 0; off < row_bytes; off += 64, ++counter) {
            oracle_chacha20_block(seeds + 32ull * r, counter, zero_nonce, blk);
            const uint64_t take = row_bytes - off < 64 ? row_bytes - off : 64;
            for (uint64_t i = 0; i < take; ++i)
                row[off + i] ^= blk[i];
        }
    }
}
