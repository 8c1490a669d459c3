// Server-side blocked cuckoo table: the DRAM working copy that Write requests
// modify (section "Writing into a Cuckoo Hash Table"; section "Evaluation":
// writes go to the working copy in DRAM, a snapshot is periodically copied to
// the GPU). Changed buckets are tracked and staged into the bound pir_db.
//
// Rules applied to each Write (beta1, beta2, payload), in order:
//   1. if `capacity` messages are live, delete the oldest one (FIFO by write
//      order; its slot bytes become zero) -- the server keeps the latest n
//      messages (section "Server Design");
//   2. store in beta1 if it has a free slot, else in beta2 (lowest free slot);
//   3. both full: one SplitMix64 draw picks beta_e (draw & 1: beta1 / beta2);
//   4. walk: put the item in hand into beta_e if a slot is free; otherwise one
//      draw picks a victim slot (draw % d), the item in hand takes its place,
//      the victim becomes the item in hand and beta_e becomes the victim's
//      other bucket (x == beta1 ? beta2 : beta1). After max_kicks evictions
//      without a free slot the item in hand is dropped: PIR_EFULL.
// The SplitMix64 stream (Steele, Lea, Flood 2014) is seeded with s_cuckoo, so
// every replica that applies the same writes in the same order builds the
// same table (the servers' shared seed s_cuckoo).
#include <string.h>

#include <deque>
#include <new>
#include <vector>

#include "db.h"

namespace {

class SplitMix64 {
  public:
    explicit SplitMix64(uint64_t seed) : x_(seed) {}
    uint64_t operator()()
    {
        x_ += 0x9E3779B97F4A7C15ull;
        uint64_t r = x_;
        r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
        r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
        return r ^ (r >> 31);
    }

  private:
    uint64_t x_;
};

struct Message {
    uint64_t id;
    uint64_t beta1, beta2;
    int64_t where;  // slot index bucket * d + s, -1 when not stored
};

}  // namespace

struct pir_cuckoo {
    pir_db *db = nullptr;
    uint64_t n = 0;
    uint32_t d = 0, z = 0;
    uint64_t capacity = 0;
    uint32_t max_kicks = 500;
    SplitMix64 rng{0};
    std::vector<uint8_t> table;       // n * d * z, bucket-major
    std::vector<int64_t> occupant;    // n * d: message index or -1
    std::vector<Message> msgs;        // every message ever written, in order
    std::deque<uint64_t> order;       // message indices in write order
    uint64_t live = 0;
    std::vector<uint8_t> changed;     // per bucket
    std::vector<uint64_t> changed_list;
    std::vector<uint8_t> carry, spare;

    uint8_t *slot_bytes(uint64_t slot) { return table.data() + slot * z; }

    void touch(uint64_t bucket)
    {
        if (!changed[bucket]) {
            changed[bucket] = 1;
            changed_list.push_back(bucket);
        }
    }

    int first_free(uint64_t bucket) const
    {
        const int64_t *o = occupant.data() + bucket * d;
        for (uint32_t s = 0; s < d; ++s)
            if (o[s] < 0)
                return (int)s;
        return -1;
    }

    void store(uint64_t m, uint64_t bucket, uint32_t s, const uint8_t *bytes)
    {
        const uint64_t slot = bucket * d + s;
        memcpy(slot_bytes(slot), bytes, z);
        occupant[slot] = (int64_t)m;
        msgs[m].where = (int64_t)slot;
        touch(bucket);
    }

    void collect_oldest()
    {
        while (!order.empty() && msgs[order.front()].where < 0)
            order.pop_front();
        if (order.empty())
            return;
        Message &old = msgs[order.front()];
        order.pop_front();
        const uint64_t slot = (uint64_t)old.where;
        memset(slot_bytes(slot), 0, z);
        occupant[slot] = -1;
        old.where = -1;
        live--;
        touch(slot / d);
    }

    int insert(uint64_t id, uint64_t b1, uint64_t b2, const uint8_t *payload, uint64_t *dropped)
    {
        if (b1 >= n || b2 >= n)
            return PIR_ERANGE;
        if (capacity && live >= capacity)
            collect_oldest();
        const uint64_t m = msgs.size();
        msgs.push_back(Message{id, b1, b2, -1});
        order.push_back(m);
        live++;
        for (uint64_t b : {b1, b2}) {
            const int s = first_free(b);
            if (s >= 0) {
                store(m, b, (uint32_t)s, payload);
                return PIR_OK;
            }
        }
        uint64_t bucket = (rng() & 1) ? b2 : b1;
        uint64_t hand = m;
        memcpy(carry.data(), payload, z);
        for (uint32_t kicks = 0;; ++kicks) {
            const int s = first_free(bucket);
            if (s >= 0) {
                store(hand, bucket, (uint32_t)s, carry.data());
                return PIR_OK;
            }
            if (kicks == max_kicks) {
                msgs[hand].where = -1;
                live--;
                if (dropped)
                    *dropped = msgs[hand].id;
                return PIR_EFULL;
            }
            const uint32_t v = (uint32_t)(rng() % d);
            const uint64_t slot = bucket * d + v;
            const uint64_t victim = (uint64_t)occupant[slot];
            memcpy(spare.data(), slot_bytes(slot), z);
            msgs[victim].where = -1;
            store(hand, bucket, v, carry.data());
            carry.swap(spare);
            hand = victim;
            bucket = (bucket == msgs[victim].beta1) ? msgs[victim].beta2 : msgs[victim].beta1;
        }
    }
};

extern "C" {

static int cuckoo_new(pir_db *db, uint64_t n, uint32_t d, uint32_t z, uint64_t capacity, uint64_t s_cuckoo,
                      uint32_t max_kicks, pir_cuckoo **out)
{
    if (!out || n == 0 || d == 0 || z == 0 || n > (1ull << 40) / d)
        return PIR_EINVAL;
    pir_cuckoo *c = new (std::nothrow) pir_cuckoo();
    if (!c)
        return PIR_ENOMEM;
    try {
        c->db = db;
        c->n = n;
        c->d = d;
        c->z = z;
        c->capacity = capacity;
        c->max_kicks = max_kicks;
        c->rng = SplitMix64(s_cuckoo);
        c->table.assign(n * d * (uint64_t)z, 0);
        c->occupant.assign(n * d, -1);
        c->changed.assign(n, 0);
        c->carry.resize(z);
        c->spare.resize(z);
    } catch (...) {
        delete c;
        return PIR_ENOMEM;
    }
    *out = c;
    return PIR_OK;
}

int pir_cuckoo_create(pir_db *db, uint64_t capacity, uint64_t s_cuckoo, uint32_t max_kicks, pir_cuckoo **out)
{
    if (!db)
        return PIR_EINVAL;
    return cuckoo_new(db, db->n, db->d, db->z, capacity, s_cuckoo, max_kicks, out);
}

int pir_cuckoo_create_detached(uint64_t n, uint32_t d, uint32_t msg_bytes, uint64_t capacity, uint64_t s_cuckoo,
                               uint32_t max_kicks, pir_cuckoo **out)
{
    return cuckoo_new(nullptr, n, d, msg_bytes, capacity, s_cuckoo, max_kicks, out);
}

void pir_cuckoo_destroy(pir_cuckoo *c) { delete c; }

int pir_cuckoo_insert(pir_cuckoo *c, uint64_t id, uint64_t beta1, uint64_t beta2, const uint8_t *payload,
                      uint64_t *dropped_id)
{
    if (!c || !payload)
        return PIR_EINVAL;
    try {
        return c->insert(id, beta1, beta2, payload, dropped_id);
    } catch (...) {
        return PIR_ENOMEM;
    }
}

int pir_cuckoo_insert_many(pir_cuckoo *c, uint64_t count, const uint64_t *ids, const uint64_t *beta1,
                           const uint64_t *beta2, const uint8_t *payloads, int32_t *status, uint64_t *dropped)
{
    if (!c || (count && (!ids || !beta1 || !beta2 || !payloads)))
        return PIR_EINVAL;
    try {
        for (uint64_t i = 0; i < count; ++i) {
            uint64_t drop = 0;
            const int rc = c->insert(ids[i], beta1[i], beta2[i], payloads + i * (uint64_t)c->z, &drop);
            if (status)
                status[i] = rc;
            if (dropped)
                dropped[i] = drop;
            if (rc == PIR_ERANGE || rc == PIR_EINVAL)
                return rc;
        }
    } catch (...) {
        return PIR_ENOMEM;
    }
    return PIR_OK;
}

int pir_cuckoo_stage(pir_cuckoo *c, uint64_t *staged)
{
    if (!c || !c->db)
        return PIR_EINVAL;
    const uint64_t cnt = c->changed_list.size();
    const uint64_t row = (uint64_t)c->d * c->z;
    int rc = PIR_OK;
    if (cnt * 2 > c->n) {
        rc = pir_db_write_range(c->db, 0, c->n, c->table.data());
    } else {
        for (uint64_t b : c->changed_list) {
            rc = pir_db_write_bucket(c->db, b, c->table.data() + b * row);
            if (rc != PIR_OK)
                break;
        }
    }
    if (rc != PIR_OK)
        return rc;
    for (uint64_t b : c->changed_list)
        c->changed[b] = 0;
    c->changed_list.clear();
    if (staged)
        *staged = cnt;
    return PIR_OK;
}

int pir_cuckoo_table(const pir_cuckoo *c, uint8_t *out, uint64_t out_bytes)
{
    if (!c || !out || out_bytes < c->table.size())
        return PIR_EINVAL;
    memcpy(out, c->table.data(), c->table.size());
    return PIR_OK;
}

int pir_cuckoo_slots(const pir_cuckoo *c, uint64_t *ids, uint8_t *occupied)
{
    if (!c)
        return PIR_EINVAL;
    for (uint64_t i = 0; i < c->occupant.size(); ++i) {
        const int64_t m = c->occupant[i];
        if (ids)
            ids[i] = m >= 0 ? c->msgs[(uint64_t)m].id : 0;
        if (occupied)
            occupied[i] = m >= 0;
    }
    return PIR_OK;
}

uint64_t pir_cuckoo_live(const pir_cuckoo *c) { return c ? c->live : 0; }

}  // extern "C"
