/*
 * Oracle: reference blocked-cuckoo table with garbage collection, and the
 * server-side global interest vector.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this. It shares no code with the library's own
 * cuckoo table, which is written independently from the same rules.
 *
 * Blocked cuckoo insertion (section "Writing into a Cuckoo Hash Table"; the
 * table shape of section "Server Design": b buckets of d slots of z bytes).
 * Each write carries two candidate buckets beta1, beta2 and z payload bytes.
 * The server, in this order:
 *   1. garbage-collects: if the table already holds `capacity` live messages
 *      (the paper's n, messages kept on the server), the oldest live message
 *      is deleted (its slot bytes become zero). Section "Server Design" keeps
 *      only the latest n messages, collecting the oldest first.
 *   2. stores the message in beta1 if that bucket has a free slot, else in
 *      beta2 if that one has a free slot (lowest free slot index).
 *   3. if both are full, picks beta_e in {beta1, beta2} with randomness derived
 *      from the shared seed s_cuckoo, and
 *   4. repeats: place the item in hand in bucket beta_e if it has space; else
 *      evict a random slot of beta_e, put the item in hand there, take the
 *      evicted item in hand and move to its alternate bucket.
 *
 * Readings where the paper is silent (each is a choice both implementations
 * make identically):
 *   - randomness is one SplitMix64 stream (Steele, Lea, Flood, OOPSLA 2014)
 *     seeded with s_cuckoo and consumed in order: one draw at the first
 *     both-full step (draw & 1: 0 -> beta1, 1 -> beta2), one draw per eviction
 *     (victim slot = draw % d);
 *   - the alternate bucket of an item sitting in bucket x is
 *     (x == beta1 ? beta2 : beta1), so beta1 == beta2 is allowed;
 *   - the loop is bounded: after max_kicks evictions with no free slot the
 *     item in hand is dropped (it leaves the live set) and the insert reports
 *     failure together with the dropped message id;
 *   - an empty or deleted slot holds zero bytes.
 *
 * Global interest vector (section "Private Notifications", maintaining a
 * global interest vector, and its window of Bloom-filter deltas): the server
 * keeps the union (bitwise OR) of the interest vectors written, over a window
 * of the most recent deltas.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* SplitMix64, from its published definition (Steele, Lea, Flood 2014). */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void oracle_splitmix64_fill(uint64_t seed, uint64_t count, uint64_t *out)
{
    uint64_t s = seed;
    for (uint64_t i = 0; i < count; ++i)
        out[i] = splitmix64_next(&s);
}

typedef struct oracle_cuckoo {
    uint64_t n;          /* buckets */
    uint32_t d;          /* slots per bucket */
    uint32_t z;          /* bytes per slot */
    uint64_t capacity;   /* live messages kept; 0 = no garbage collection */
    uint32_t max_kicks;
    uint64_t rng;        /* SplitMix64 state */
    uint8_t *table;      /* n * d * z bytes */
    int64_t *slot_item;  /* n * d entries: item index or -1 */
    uint64_t n_items, cap_items;
    uint64_t *item_id, *item_b1, *item_b2;
    int64_t *item_slot;  /* global slot index, or -1 when not live */
    uint64_t oldest;     /* no live item has an index below this */
    uint64_t live;
    uint8_t *hand, *hand2;
} oracle_cuckoo;

oracle_cuckoo *oracle_cuckoo_new(uint64_t n, uint32_t d, uint32_t z,
                                 uint64_t capacity, uint64_t seed, uint32_t max_kicks)
{
    if (n == 0 || d == 0 || z == 0)
        return NULL;
    oracle_cuckoo *c = (oracle_cuckoo *)calloc(1, sizeof(oracle_cuckoo));
    if (!c)
        return NULL;
    c->n = n;
    c->d = d;
    c->z = z;
    c->capacity = capacity;
    c->max_kicks = max_kicks;
    c->rng = seed;
    c->table = (uint8_t *)calloc(n * d, z);
    c->slot_item = (int64_t *)malloc(sizeof(int64_t) * n * d);
    c->hand = (uint8_t *)malloc(z);
    c->hand2 = (uint8_t *)malloc(z);
    if (!c->table || !c->slot_item || !c->hand || !c->hand2) {
        free(c->table);
        free(c->slot_item);
        free(c->hand);
        free(c->hand2);
        free(c);
        return NULL;
    }
    for (uint64_t i = 0; i < n * d; ++i)
        c->slot_item[i] = -1;
    return c;
}

void oracle_cuckoo_free(oracle_cuckoo *c)
{
    if (!c)
        return;
    free(c->table);
    free(c->slot_item);
    free(c->item_id);
    free(c->item_b1);
    free(c->item_b2);
    free(c->item_slot);
    free(c->hand);
    free(c->hand2);
    free(c);
}

static int grow_items(oracle_cuckoo *c)
{
    if (c->n_items < c->cap_items)
        return 0;
    uint64_t cap = c->cap_items ? c->cap_items * 2 : 1024;
    uint64_t *a = (uint64_t *)realloc(c->item_id, cap * sizeof(uint64_t));
    if (!a) return -1;
    c->item_id = a;
    a = (uint64_t *)realloc(c->item_b1, cap * sizeof(uint64_t));
    if (!a) return -1;
    c->item_b1 = a;
    a = (uint64_t *)realloc(c->item_b2, cap * sizeof(uint64_t));
    if (!a) return -1;
    c->item_b2 = a;
    int64_t *s = (int64_t *)realloc(c->item_slot, cap * sizeof(int64_t));
    if (!s) return -1;
    c->item_slot = s;
    c->cap_items = cap;
    return 0;
}

/* lowest free slot index of bucket b, or -1 */
static int64_t free_slot(const oracle_cuckoo *c, uint64_t b)
{
    for (uint32_t s = 0; s < c->d; ++s)
        if (c->slot_item[b * c->d + s] < 0)
            return (int64_t)s;
    return -1;
}

static void put(oracle_cuckoo *c, uint64_t item, uint64_t bucket, uint64_t s,
                const uint8_t *payload)
{
    uint64_t slot = bucket * c->d + s;
    memcpy(c->table + slot * c->z, payload, c->z);
    c->slot_item[slot] = (int64_t)item;
    c->item_slot[item] = (int64_t)slot;
}

static void delete_oldest(oracle_cuckoo *c)
{
    while (c->oldest < c->n_items && c->item_slot[c->oldest] < 0)
        c->oldest++;
    if (c->oldest >= c->n_items)
        return;
    uint64_t slot = (uint64_t)c->item_slot[c->oldest];
    memset(c->table + slot * c->z, 0, c->z);
    c->slot_item[slot] = -1;
    c->item_slot[c->oldest] = -1;
    c->live--;
    c->oldest++;
}

/* Returns 0 on success, -2 on a bucket out of range, -3 on allocation failure,
 * -5 when the eviction walk hit max_kicks (dropped_id receives the id of the
 * message that was dropped). */
int oracle_cuckoo_insert(oracle_cuckoo *c, uint64_t id, uint64_t b1, uint64_t b2,
                         const uint8_t *payload, uint64_t *dropped_id)
{
    if (b1 >= c->n || b2 >= c->n)
        return -2;
    if (grow_items(c))
        return -3;
    if (c->capacity && c->live >= c->capacity)
        delete_oldest(c);

    uint64_t item = c->n_items++;
    c->item_id[item] = id;
    c->item_b1[item] = b1;
    c->item_b2[item] = b2;
    c->item_slot[item] = -1;
    c->live++;

    int64_t s = free_slot(c, b1);
    if (s >= 0) {
        put(c, item, b1, (uint64_t)s, payload);
        return 0;
    }
    s = free_slot(c, b2);
    if (s >= 0) {
        put(c, item, b2, (uint64_t)s, payload);
        return 0;
    }

    uint64_t be = (splitmix64_next(&c->rng) & 1) ? b2 : b1;
    uint64_t cur = item;
    memcpy(c->hand, payload, c->z);
    for (uint32_t kicks = 0;; ++kicks) {
        s = free_slot(c, be);
        if (s >= 0) {
            put(c, cur, be, (uint64_t)s, c->hand);
            return 0;
        }
        if (kicks == c->max_kicks) {
            c->item_slot[cur] = -1;
            c->live--;
            if (dropped_id)
                *dropped_id = c->item_id[cur];
            return -5;
        }
        uint64_t v = splitmix64_next(&c->rng) % c->d;
        uint64_t slot = be * c->d + v;
        uint64_t victim = (uint64_t)c->slot_item[slot];
        memcpy(c->hand2, c->table + slot * c->z, c->z);
        put(c, cur, be, v, c->hand);
        c->item_slot[victim] = -1;
        uint8_t *t = c->hand;
        c->hand = c->hand2;
        c->hand2 = t;
        cur = victim;
        be = (be == c->item_b1[victim]) ? c->item_b2[victim] : c->item_b1[victim];
    }
}

/* Applies count writes in order. status[i] gets each insert's return code and
 * dropped[i] the dropped id (or 0). Returns the number of failed inserts. */
uint64_t oracle_cuckoo_insert_many(oracle_cuckoo *c, uint64_t count, const uint64_t *ids,
                                   const uint64_t *b1, const uint64_t *b2,
                                   const uint8_t *payloads, int32_t *status,
                                   uint64_t *dropped)
{
    uint64_t failed = 0;
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t drop = 0;
        int rc = oracle_cuckoo_insert(c, ids[i], b1[i], b2[i],
                                      payloads + i * (uint64_t)c->z, &drop);
        if (status)
            status[i] = rc;
        if (dropped)
            dropped[i] = drop;
        if (rc)
            failed++;
    }
    return failed;
}

const uint8_t *oracle_cuckoo_table(const oracle_cuckoo *c) { return c->table; }
uint64_t oracle_cuckoo_live(const oracle_cuckoo *c) { return c->live; }

/* Per slot: the id of the message stored there (0 when empty) and an
 * occupancy flag. */
void oracle_cuckoo_slots(const oracle_cuckoo *c, uint64_t *ids, uint8_t *occupied)
{
    for (uint64_t i = 0; i < c->n * c->d; ++i) {
        int64_t it = c->slot_item[i];
        occupied[i] = it >= 0;
        ids[i] = it >= 0 ? c->item_id[it] : 0;
    }
}

/* Candidate buckets of every message stored (per slot; 0 when empty). */
void oracle_cuckoo_slot_buckets(const oracle_cuckoo *c, uint64_t *b1, uint64_t *b2)
{
    for (uint64_t i = 0; i < c->n * c->d; ++i) {
        int64_t it = c->slot_item[i];
        b1[i] = it >= 0 ? c->item_b1[it] : 0;
        b2[i] = it >= 0 ? c->item_b2[it] : 0;
    }
}

/*
 * Global interest vector over a window of epochs: the OR of every position
 * written in epochs max(0, last - window + 1) .. last. Epoch e's positions are
 * pos[epoch_start[e] .. epoch_start[e + 1]). out receives ceil(m_bits / 8)
 * bytes, bit p at byte p >> 3, bit p & 7. Positions >= m_bits are rejected.
 */
int oracle_interest_window(uint64_t m_bits, const uint32_t *pos,
                           const uint64_t *epoch_start, uint32_t last,
                           uint32_t window, uint8_t *out)
{
    memset(out, 0, (m_bits + 7) / 8);
    if (window == 0)
        return 0;
    uint32_t first = last + 1 >= window ? last + 1 - window : 0;
    for (uint32_t e = first; e <= last; ++e)
        for (uint64_t i = epoch_start[e]; i < epoch_start[e + 1]; ++i) {
            if (pos[i] >= m_bits)
                return -1;
            out[pos[i] >> 3] |= (uint8_t)(1u << (pos[i] & 7));
        }
    return 0;
}
