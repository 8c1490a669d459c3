// Host-only driver for the sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer, gcc/g++): exercises the oracle's C code and the
// library's blocked cuckoo table (a detached table: no database, no GPU) on
// seeded inputs, including the edge cases (full tables with dropped items,
// FIFO collection, malformed compressed streams), and requires the library's
// table to equal the oracle's after every sequence. Exit status 0 = every
// check passed; the sanitizers abort the process on the first report.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "talek_pir.h"

extern "C" {
// oracle/ (plain C, built into the same executable)
int oracle_pir_read(const uint8_t *D, uint64_t n, uint64_t bucket_bytes, const uint8_t *req, uint64_t req_stride,
                    uint32_t B, uint8_t *resp, uint32_t nthreads);
void oracle_splitmix64_fill(uint64_t seed, uint64_t count, uint64_t *out);
struct oracle_cuckoo;
oracle_cuckoo *oracle_cuckoo_new(uint64_t n, uint32_t d, uint32_t z, uint64_t capacity, uint64_t seed,
                                 uint32_t max_kicks);
void oracle_cuckoo_free(oracle_cuckoo *c);
uint64_t oracle_cuckoo_insert_many(oracle_cuckoo *c, uint64_t count, const uint64_t *ids, const uint64_t *b1,
                                   const uint64_t *b2, const uint8_t *payloads, int32_t *status, uint64_t *dropped);
const uint8_t *oracle_cuckoo_table(const oracle_cuckoo *c);
uint64_t oracle_cuckoo_live(const oracle_cuckoo *c);
void oracle_cuckoo_slots(const oracle_cuckoo *c, uint64_t *ids, uint8_t *occupied);
int oracle_interest_window(uint64_t m_bits, const uint32_t *pos, const uint64_t *epoch_start, uint32_t last,
                           uint32_t window, uint8_t *out);
void oracle_chacha20_stream(const uint8_t key[32], const uint8_t nonce[12], uint32_t counter, uint8_t *out,
                            uint64_t len);
void oracle_apply_masks(uint8_t *resp, uint64_t row_bytes, uint32_t B, const uint8_t *seeds);
uint64_t oracle_iv_encode(const uint8_t *v, uint64_t m, uint8_t *out, uint64_t cap);
uint64_t oracle_iv_decode(const uint8_t *s, uint64_t len, uint8_t *v, uint64_t v_bytes);

// The detached cuckoo table never stages into a database; these stand in for
// the database half of the library, which needs a GPU.
int pir_db_write_range(pir_db *, uint64_t, uint64_t, const uint8_t *) { return PIR_EINVAL; }
int pir_db_write_bucket(pir_db *, uint64_t, const uint8_t *) { return PIR_EINVAL; }
}

namespace {

int failures = 0;

void check(bool ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

struct Rng {  // test input stream (not the method's randomness)
    uint64_t s;
    uint64_t next()
    {
        uint64_t x;
        oracle_splitmix64_fill(s++, 1, &x);
        return x;
    }
};

void cuckoo_case(uint64_t n, uint32_t d, uint32_t z, uint64_t count, uint64_t capacity, uint32_t max_kicks,
                 uint64_t seed)
{
    Rng r{seed * 7919};
    std::vector<uint64_t> ids(count), b1(count), b2(count);
    std::vector<uint8_t> pay(count * z);
    for (uint64_t i = 0; i < count; ++i) {
        ids[i] = i + 1;
        b1[i] = r.next() % n;
        b2[i] = r.next() % n;
        for (uint32_t k = 0; k < z; ++k)
            pay[i * z + k] = (uint8_t)(r.next() >> 11);
    }
    std::vector<int32_t> st_o(count), st_l(count);
    std::vector<uint64_t> dr_o(count), dr_l(count);
    oracle_cuckoo *o = oracle_cuckoo_new(n, d, z, capacity, seed, max_kicks);
    check(o != nullptr, "oracle table");
    oracle_cuckoo_insert_many(o, count, ids.data(), b1.data(), b2.data(), pay.data(), st_o.data(), dr_o.data());
    pir_cuckoo *c = nullptr;
    check(pir_cuckoo_create_detached(n, d, z, capacity, seed, max_kicks, &c) == PIR_OK, "library table");
    check(pir_cuckoo_insert_many(c, count, ids.data(), b1.data(), b2.data(), pay.data(), st_l.data(),
                                 dr_l.data()) == PIR_OK, "library insert_many");
    check(st_o == st_l && dr_o == dr_l, "insert statuses and dropped ids");
    std::vector<uint8_t> tab(n * d * z);
    check(pir_cuckoo_table(c, tab.data(), tab.size()) == PIR_OK, "library table bytes");
    check(memcmp(tab.data(), oracle_cuckoo_table(o), tab.size()) == 0, "tables equal");
    std::vector<uint64_t> id_l(n * d), id_o(n * d);
    std::vector<uint8_t> oc_l(n * d), oc_o(n * d);
    check(pir_cuckoo_slots(c, id_l.data(), oc_l.data()) == PIR_OK, "library slots");
    oracle_cuckoo_slots(o, id_o.data(), oc_o.data());
    check(id_l == id_o && oc_l == oc_o, "slot ids equal");
    check(pir_cuckoo_live(c) == oracle_cuckoo_live(o), "live counts equal");
    uint64_t staged = 0;
    check(pir_cuckoo_stage(c, &staged) == PIR_EINVAL, "detached table cannot stage");
    uint64_t dropped = 0;
    check(pir_cuckoo_insert(c, 1, n, 0, pay.data(), &dropped) == PIR_ERANGE, "bucket out of range");
    check(pir_cuckoo_table(c, tab.data(), tab.size() - 1) == PIR_EINVAL, "short output");
    pir_cuckoo_destroy(c);
    oracle_cuckoo_free(o);
}

void pir_case(uint64_t n, uint64_t bucket, uint32_t B, uint32_t threads)
{
    Rng r{n * 31 + bucket};
    const uint64_t qb = (n + 7) / 8;
    std::vector<uint8_t> D(n * bucket), q(B * qb), a(B * bucket), b(B * bucket);
    for (auto &x : D)
        x = (uint8_t)r.next();
    for (auto &x : q)
        x = (uint8_t)r.next();
    check(oracle_pir_read(D.data(), n, bucket, q.data(), qb, B, a.data(), 1) == 0, "pir read");
    check(oracle_pir_read(D.data(), n, bucket, q.data(), qb, B, b.data(), threads) == 0, "pir read, threads");
    check(a == b, "threads give the same answers");
    check(oracle_pir_read(D.data(), n, bucket, q.data(), qb - 1, B, b.data(), 1) == -1, "short stride refused");
    std::vector<uint8_t> seeds(32 * B);
    for (auto &x : seeds)
        x = (uint8_t)r.next();
    oracle_apply_masks(a.data(), bucket, B, seeds.data());
    oracle_apply_masks(a.data(), bucket, B, seeds.data());
    check(a == b, "masks cancel");
}

void codec_case(uint64_t m, uint32_t every)
{
    std::vector<uint8_t> v((m + 7) / 8), w((m + 7) / 8);
    Rng r{m + every};
    for (uint64_t p = 0; p < m; ++p)
        if (every && r.next() % every == 0)
            v[p >> 3] |= (uint8_t)(1u << (p & 7));
    const uint64_t len = oracle_iv_encode(v.data(), m, nullptr, 0);
    std::vector<uint8_t> s(len);
    check(oracle_iv_encode(v.data(), m, s.data(), len) == len, "encode");
    check(oracle_iv_decode(s.data(), len, w.data(), w.size()) == m && v == w, "round trip");
    for (uint64_t cut = 0; cut < len; cut += 1 + len / 7)
        (void)oracle_iv_decode(s.data(), cut, w.data(), w.size());   // truncated: refused, no overrun
    std::vector<uint8_t> junk(len + 8);
    for (auto &x : junk)
        x = (uint8_t)r.next();
    (void)oracle_iv_decode(junk.data(), junk.size(), w.data(), w.size());
}

}  // namespace

int main()
{
    cuckoo_case(64, 4, 8, 240, 0, 500, 1);
    cuckoo_case(97, 3, 12, 290, 0, 500, 2);
    cuckoo_case(16, 2, 8, 60, 0, 20, 3);      // overfull: dropped items
    cuckoo_case(64, 2, 8, 400, 80, 500, 4);   // FIFO collection
    cuckoo_case(1024, 4, 32, 3900, 0, 500, 5);
    cuckoo_case(5, 1, 1, 30, 3, 4, 6);
    pir_case(1, 16, 3, 2);
    pir_case(37, 24, 5, 3);
    pir_case(300, 520, 9, 4);
    uint8_t key[32], nonce[12] = {0}, ks[200];
    for (int i = 0; i < 32; ++i)
        key[i] = (uint8_t)i;
    oracle_chacha20_stream(key, nonce, 0, ks, sizeof ks);
    codec_case(64, 3);
    codec_case(1000, 0);
    codec_case(1 << 17, 50);
    codec_case(77, 1);
    std::vector<uint32_t> pos = {1, 5, 200, 5, 9};
    std::vector<uint64_t> starts = {0, 3, 5};
    std::vector<uint8_t> iv(32);
    check(oracle_interest_window(256, pos.data(), starts.data(), 1, 4, iv.data()) == 0, "interest window");
    printf("host driver: %s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
