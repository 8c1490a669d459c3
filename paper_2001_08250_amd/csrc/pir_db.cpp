// C ABI of the XOR-PIR engine: database handle, epoch-published writes,
// reads, and the global interest vector.
#include <string.h>

#include <algorithm>
#include <new>

#include "db.h"

using namespace talek;

namespace talek {

int hip_status(hipError_t e) { return e == hipSuccess ? PIR_OK : PIR_EDEVICE; }

int ensure_device(void **p, uint64_t *cap, uint64_t bytes)
{
    if (bytes <= *cap && *p)
        return PIR_OK;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess)
            return PIR_EDEVICE;
    }
    uint64_t want = std::max<uint64_t>(bytes, 256);
    if (hipMalloc(p, want) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return PIR_ENOMEM;
    }
    *cap = want;
    return PIR_OK;
}

Scratch &scratch_for(pir_db *db, hipStream_t s) { return db->scratch[s]; }

void destroy_stream_graph(Scratch &sc)
{
    if (sc.exec)
        hipGraphExecDestroy(sc.exec);
    sc.exec = nullptr;
    sc.sig.clear();
}

// The event that tracks the readers of buffer b on stream s, created on first
// use. It keeps timing enabled so that a kernel dispatch can record it.
int reader_event(pir_db *db, int b, hipStream_t s, hipEvent_t *ev)
{
    auto it = db->readers[b].find(s);
    if (it == db->readers[b].end()) {
        if (hipEventCreate(ev) != hipSuccess)
            return PIR_EDEVICE;
        db->readers[b].emplace(s, *ev);
    } else {
        *ev = it->second;
    }
    return PIR_OK;
}

int note_reader(pir_db *db, int b, hipStream_t s)
{
    hipEvent_t ev;
    const int rc = reader_event(db, b, s, &ev);
    if (rc != PIR_OK)
        return rc;
    return hipEventRecord(ev, s) == hipSuccess ? PIR_OK : PIR_EDEVICE;
}

// Order `s` after the latest publication; no wait is enqueued when it has
// already completed (the snapshot it wrote is then final for `s` as well).
int wait_published(pir_db *db, hipStream_t s)
{
    if (hipEventQuery(db->published) == hipSuccess)
        return PIR_OK;
    return hipStreamWaitEvent(s, db->published, 0) == hipSuccess ? PIR_OK : PIR_EDEVICE;
}

ReadGeom read_geom(pir_db *db, const void *q, uint64_t qpitch, uint32_t B, void *out, uint64_t out_pitch)
{
    ReadGeom g{};
    g.D = db->buf[db->front];
    g.n = db->n;
    g.stride = db->stride;
    g.Q = q;
    g.qpitch = qpitch;
    g.B = B;
    g.out = out;
    g.out_pitch = out_pitch;
    return g;
}

Plan choose_plan(pir_db *db, uint32_t B)
{
    ReadGeom g = read_geom(db, nullptr, db->qpitch, B, nullptr, db->stride);
    Plan want = db->forced;
    if (want.kind == KIND_AUTO) {
        Plan tuned;
        if (tune_lookup(db->n, B, db->stride, &tuned))
            want = tuned;
    }
    return resolve_plan(g, want, db->num_cus);
}

}  // namespace talek

namespace {

constexpr uint64_t STAGE_BYTES = 64ull << 20;  // pinned staging for bucket writes

#define HIP_TRY(x)                                                                                                 \
    do {                                                                                                           \
        hipError_t e_ = (x);                                                                                       \
        if (e_ != hipSuccess)                                                                                      \
            return PIR_EDEVICE;                                                                                    \
    } while (0)

#define PIR_TRY(x)                                                                                                 \
    do {                                                                                                           \
        int r_ = (x);                                                                                              \
        if (r_ != PIR_OK)                                                                                          \
            return r_;                                                                                             \
    } while (0)

int ensure_back(pir_db *db)
{
    if (db->have_back)
        return PIR_OK;
    const uint64_t bytes = db->rows_alloc * db->stride;
    if (!db->buf[db->front ^ 1]) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return PIR_ENOMEM;
        }
        db->buf[db->front ^ 1] = static_cast<uint8_t *>(p);
    }
    HIP_TRY(hipMemcpyAsync(db->buf[db->front ^ 1], db->buf[db->front], bytes, hipMemcpyDeviceToDevice, db->stream));
    db->have_back = true;
    return PIR_OK;
}

enum { UP_STAGE = 0, UP_POS = 1, UP_MIRROR = 2 };

// Pinned host memory that kernels read in place: *host for the CPU, *dev
// for kernels.
int host_mapped(uint64_t bytes, void **host, void **dev)
{
    *host = *dev = nullptr;
    if (hipHostMalloc(host, std::max<uint64_t>(bytes, 64), hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        *host = nullptr;
        return PIR_ENOMEM;
    }
    if (hipHostGetDevicePointer(dev, *host, 0) != hipSuccess) {
        hipHostFree(*host);
        *host = nullptr;
        return PIR_EDEVICE;
    }
    return PIR_OK;
}

// Block until pinned upload buffer `which` is no longer read by a queued copy.
int wait_upload(pir_db *db, int which)
{
    if (!db->upload_pending[which])
        return PIR_OK;
    HIP_TRY(hipEventSynchronize(db->upload_ev[which]));
    db->upload_pending[which] = false;
    return PIR_OK;
}

int note_upload(pir_db *db, int which)
{
    HIP_TRY(hipEventRecord(db->upload_ev[which], db->stream));
    db->upload_pending[which] = true;
    return PIR_OK;
}

void mark_dirty(pir_db *db, uint64_t b)
{
    if (db->all_dirty || db->dirty_mark[b])
        return;
    db->dirty_mark[b] = 1;
    db->dirty.push_back(b);
}

// Apply the staged rows to the back copy (the kernel reads them straight
// from mapped host memory); afterwards the staging is empty.
int flush_stage(pir_db *db)
{
    if (db->stage_rows == 0)
        return PIR_OK;
    PIR_TRY(ensure_back(db));
    const uint64_t rows = db->stage_rows;
    HIP_TRY(launch_scatter_rows(db->buf[db->front ^ 1], db->stage_map, static_cast<const uint64_t *>(db->stage_idx_map),
                                rows, db->stride, db->stream));
    PIR_TRY(note_upload(db, UP_STAGE));  // the staging rows are refilled only after this
    for (uint64_t i = 0; i < rows; ++i)
        mark_dirty(db, db->stage_idx_host[i]);
    db->stage_rows = 0;
    db->stage_slot.clear();
    return PIR_OK;
}

int stage_row(pir_db *db, uint64_t bucket, const uint8_t *data)
{
    auto it = db->stage_slot.find(bucket);
    uint64_t slot;
    if (it != db->stage_slot.end()) {
        slot = it->second;
    } else {
        if (db->stage_rows == db->stage_cap)
            PIR_TRY(flush_stage(db));
        if (db->stage_rows == 0)
            PIR_TRY(wait_upload(db, UP_STAGE));
        slot = db->stage_rows++;
        db->stage_slot.emplace(bucket, slot);
        db->stage_idx_host[slot] = bucket;
    }
    uint8_t *row = db->stage_host + slot * db->stride;
    memcpy(row, data, db->bucket_bytes);
    if (db->stride > db->bucket_bytes)
        memset(row + db->bucket_bytes, 0, db->stride - db->bucket_bytes);
    return PIR_OK;
}

// Make `s` wait until every reader of buffer `b` recorded so far is done.
int wait_readers(pir_db *db, int b, hipStream_t s)
{
    for (auto &kv : db->readers[b])
        HIP_TRY(hipStreamWaitEvent(s, kv.second, 0));
    return PIR_OK;
}

int interest_alloc(pir_db *db, uint64_t m_bits, uint32_t window)
{
    hipFree(db->iv_ring);
    hipFree(db->iv_global[0]);
    hipFree(db->iv_global[1]);
    db->iv_ring = db->iv_global[0] = db->iv_global[1] = nullptr;
    const uint64_t words = (m_bits + 31) / 32;
    void *p = nullptr;
    if (hipMalloc(&p, words * 4 * window) != hipSuccess)
        return PIR_ENOMEM;
    db->iv_ring = static_cast<uint32_t *>(p);
    for (int i = 0; i < 2; ++i) {
        if (hipMalloc(&p, words * 4) != hipSuccess)
            return PIR_ENOMEM;
        db->iv_global[i] = static_cast<uint32_t *>(p);
    }
    db->m_bits = m_bits;
    db->iv_words = words;
    db->window = window;
    db->pos_pending.clear();
    HIP_TRY(launch_fill_zero(db->iv_ring, words * 4 * window, db->stream));
    HIP_TRY(launch_fill_zero(db->iv_global[0], words * 4, db->stream));
    HIP_TRY(launch_fill_zero(db->iv_global[1], words * 4, db->stream));
    HIP_TRY(hipStreamSynchronize(db->stream));
    return PIR_OK;
}

void free_db(pir_db *db)
{
    if (db->stream)
        (void)hipStreamSynchronize(db->stream);
    for (auto &kv : db->scratch) {
        destroy_stream_graph(kv.second);
        hipFree(kv.second.req);
        hipFree(kv.second.resp);
        hipFree(kv.second.part);
        hipFree(kv.second.aux);
        hipFree(kv.second.keys);
        hipFree(kv.second.leaf_q);
        hipFree(kv.second.host_rows);
        hipFree(kv.second.leaf_out);
    }
    for (int b = 0; b < 3; ++b)
        for (auto &kv : db->readers[b])
            hipEventDestroy(kv.second);
    for (int b = 0; b < 2; ++b) {
        hipFree(db->buf[b]);
        hipFree(db->iv_global[b]);
    }
    hipFree(db->prep);
    hipFree(db->iv_ring);
    if (db->stage_host)
        hipHostFree(db->stage_host);
    if (db->stage_idx_host)
        hipHostFree(db->stage_idx_host);
    if (db->pos_host)
        hipHostFree(db->pos_host);
    if (db->published)
        hipEventDestroy(db->published);
    for (int i = 0; i < 3; ++i)
        if (db->upload_ev[i])
            hipEventDestroy(db->upload_ev[i]);
    if (db->mirror_idx_host)
        hipHostFree(db->mirror_idx_host);
    hipFree(db->codec);
    hipFree(db->codec2);
    hipFree(db->codec3);
    for (auto &ev : db->prof_ev) {
        hipEventDestroy(ev.first);
        hipEventDestroy(ev.second);
    }
    if (db->stream)
        hipStreamDestroy(db->stream);
    if (db->capture_stream)
        hipStreamDestroy(db->capture_stream);
    delete db;
}

}  // namespace

extern "C" {

const char *pir_strerror(int code)
{
    switch (code) {
    case PIR_OK: return "ok";
    case PIR_EINVAL: return "invalid argument";
    case PIR_ERANGE: return "index out of range";
    case PIR_ENOMEM: return "out of memory";
    case PIR_EDEVICE: return "HIP device error";
    case PIR_EFULL: return "cuckoo insertion failed (eviction bound reached)";
    case PIR_EBUSY: return "no memory slot free (admission refused)";
    default: return "unknown error";
    }
}

const char *pir_version(void) { return "talek-pir 0.1 gfx950"; }

int pir_db_create(uint64_t n, uint32_t d, uint32_t msg_bytes, pir_db **out)
{
    if (!out || n == 0 || d == 0 || msg_bytes == 0)
        return PIR_EINVAL;
    const uint64_t bucket = (uint64_t)d * msg_bytes;
    if (bucket > (1ull << 30) || n > (1ull << 40))
        return PIR_EINVAL;
    const uint64_t stride = (bucket + 15) & ~15ull;
    if (stride / 16 > 0xffffffffull || n + 128 > UINT64_MAX / stride)
        return PIR_EINVAL;
    pir_db *db = new (std::nothrow) pir_db();
    if (!db)
        return PIR_ENOMEM;
    db->n = n;
    db->d = d;
    db->z = msg_bytes;
    db->bucket_bytes = bucket;
    db->stride = stride;
    db->qbytes = (n + 7) / 8;
    db->qpitch = (db->qbytes + 15) & ~15ull;
    int rc = PIR_OK;
    do {
        if (hipGetDevice(&db->device) != hipSuccess) { rc = PIR_EDEVICE; break; }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, db->device) == hipSuccess && prop.multiProcessorCount > 0)
            db->num_cus = prop.multiProcessorCount;
        if (hipStreamCreateWithFlags(&db->stream, hipStreamNonBlocking) != hipSuccess) { rc = PIR_EDEVICE; break; }
        if (hipStreamCreateWithFlags(&db->capture_stream, hipStreamNonBlocking) != hipSuccess) {
            rc = PIR_EDEVICE;
            break;
        }
        if (hipEventCreateWithFlags(&db->published, hipEventDisableTiming) != hipSuccess) { rc = PIR_EDEVICE; break; }
        for (int i = 0; i < 3 && rc == PIR_OK; ++i)
            if (hipEventCreateWithFlags(&db->upload_ev[i], hipEventDisableTiming) != hipSuccess)
                rc = PIR_EDEVICE;
        if (rc != PIR_OK)
            break;
        // allocation-free reads: the static scratch of this device and one
        // reader event per snapshot copy, made here so that those reads
        // create nothing
        if ((rc = talek::noalloc_setup(db->device)) != PIR_OK)
            break;
        for (int b = 0; b < 2 && rc == PIR_OK; ++b) {
            hipEvent_t ev = nullptr;
            if (hipEventCreate(&ev) != hipSuccess)
                rc = PIR_EDEVICE;
            else
                db->readers[b].emplace(talek::noalloc_reader_key(db), ev);
        }
        if (rc != PIR_OK)
            break;
        void *p = nullptr;
        db->rows_alloc = talek::padded_db_rows(n);
        if (hipMalloc(&p, db->rows_alloc * stride) != hipSuccess) { rc = PIR_ENOMEM; break; }
        db->buf[0] = static_cast<uint8_t *>(p);
        if (launch_fill_zero(db->buf[0], db->rows_alloc * stride, db->stream) != hipSuccess) {
            rc = PIR_EDEVICE;
            break;
        }
        db->stage_cap = std::max<uint64_t>(1, std::min<uint64_t>(n, STAGE_BYTES / stride));
        if ((rc = host_mapped(db->stage_cap * stride, &p, &db->stage_map)) != PIR_OK)
            break;
        db->stage_host = static_cast<uint8_t *>(p);
        if ((rc = host_mapped(db->stage_cap * sizeof(uint64_t), &p, &db->stage_idx_map)) != PIR_OK)
            break;
        db->stage_idx_host = static_cast<uint64_t *>(p);
        db->dirty_mark.assign(n, 0);
        // the paper's sizes: a vector of about 14 KB at 1M messages and a TTL
        // of 100 write intervals (section "Evaluation", cost of operations)
        if ((rc = interest_alloc(db, 1ull << 17, 100)) != PIR_OK)
            break;
        if (hipEventRecord(db->published, db->stream) != hipSuccess) { rc = PIR_EDEVICE; break; }
        if (hipStreamSynchronize(db->stream) != hipSuccess) { rc = PIR_EDEVICE; break; }
    } while (0);
    if (rc != PIR_OK) {
        (void)hipGetLastError();
        free_db(db);
        return rc;
    }
    *out = db;
    return PIR_OK;
}

void pir_db_destroy(pir_db *db)
{
    if (!db)
        return;
    hipSetDevice(db->device);
    free_db(db);
}

int pir_db_shape(const pir_db *db, uint64_t *n, uint32_t *d, uint32_t *msg_bytes, uint64_t *bucket_bytes)
{
    if (!db)
        return PIR_EINVAL;
    if (n) *n = db->n;
    if (d) *d = db->d;
    if (msg_bytes) *msg_bytes = db->z;
    if (bucket_bytes) *bucket_bytes = db->bucket_bytes;
    return PIR_OK;
}

int pir_db_write_bucket(pir_db *db, uint64_t bucket, const uint8_t *data)
{
    if (!db || !data)
        return PIR_EINVAL;
    if (bucket >= db->n)
        return PIR_ERANGE;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    return stage_row(db, bucket, data);
}

int pir_db_write_range(pir_db *db, uint64_t first, uint64_t count, const uint8_t *data)
{
    if (!db || (count && !data))
        return PIR_EINVAL;
    if (first > db->n || count > db->n - first)
        return PIR_ERANGE;
    if (count == 0)
        return PIR_OK;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    if (count < db->stage_cap / 2) {
        for (uint64_t i = 0; i < count; ++i)
            PIR_TRY(stage_row(db, first + i, data + i * db->bucket_bytes));
        return PIR_OK;
    }
    // Large range: keep write order (staged rows first), then copy straight
    // into the back copy.
    PIR_TRY(flush_stage(db));
    PIR_TRY(ensure_back(db));
    uint8_t *dst = db->buf[db->front ^ 1] + first * db->stride;
    HIP_TRY(hipMemcpy2DAsync(dst, db->stride, data, db->bucket_bytes, db->bucket_bytes, count,
                             hipMemcpyHostToDevice, db->stream));
    HIP_TRY(hipStreamSynchronize(db->stream));
    if (count == db->n) {
        db->all_dirty = true;
    } else {
        for (uint64_t i = 0; i < count; ++i)
            mark_dirty(db, first + i);
    }
    return PIR_OK;
}

// The epoch's dirty bucket indices in mapped pinned memory (device address
// in *dev), for the kernels of the commit that read them in place; the
// caller records UP_MIRROR after the last of them.
static int upload_dirty(pir_db *db, const uint64_t **dev)
{
    const uint64_t cnt = db->dirty.size();
    PIR_TRY(wait_upload(db, UP_MIRROR));
    if (cnt > db->mirror_idx_cap) {
        if (db->mirror_idx_host)
            hipHostFree(db->mirror_idx_host);
        db->mirror_idx_host = nullptr;
        db->mirror_idx_cap = 0;
        void *p = nullptr;
        PIR_TRY(host_mapped(cnt * sizeof(uint64_t), &p, &db->mirror_map));
        db->mirror_idx_host = static_cast<uint64_t *>(p);
        db->mirror_idx_cap = cnt;
    }
    memcpy(db->mirror_idx_host, db->dirty.data(), cnt * sizeof(uint64_t));
    *dev = static_cast<const uint64_t *>(db->mirror_map);
    return PIR_OK;
}

// Leaf databases of preprocessed reads from snapshot buffer b, on the
// handle's stream once the reads still using the old leaves are done: only
// the leaf rows the epoch's dirty buckets feed when those are few (dirty =
// their uploaded indices), else every row.
static int build_prep(pir_db *db, int b, const uint64_t *dirty)
{
    PIR_TRY(wait_readers(db, 2, db->stream));
    if (dirty) {
        HIP_TRY(launch_prep_rows(db->prep_t, db->buf[b], db->stride, db->n, db->prep_Nq, db->prep_Cq, dirty,
                                 db->dirty.size(), db->prep, db->prep_leaf_bytes, db->stream));
        return PIR_OK;
    }
    HIP_TRY(launch_prep_d(db->prep_t, db->buf[b], db->stride, db->n, db->prep_Nq, db->prep_Cq, db->prep,
                          db->prep_leaf_bytes, db->stream));
    return PIR_OK;
}

int pir_epoch_commit(pir_db *db, uint64_t *epoch_out)
{
    if (!db)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    const uint64_t rows = db->stage_rows;
    for (uint64_t i = 0; i < rows; ++i)
        mark_dirty(db, db->stage_idx_host[i]);
    const bool changed = db->all_dirty || !db->dirty.empty();
    const int back = db->front ^ 1;
    if (changed)
        PIR_TRY(ensure_back(db));

    // Interest vector: the open epoch's delta replaces the ring slot of the
    // epoch that leaves the window, and the new global vector (OR of the
    // window) goes with the back copy. The positions go to the kernel sorted
    // by block of COMMIT_IV_WORDS words (counting sort), in mapped host memory.
    PIR_TRY(wait_upload(db, UP_POS));
    const uint64_t npos = db->pos_pending.size();
    const uint64_t nb = (db->iv_words + COMMIT_IV_WORDS - 1) / COMMIT_IV_WORDS;
    if (npos + nb + 1 > db->pos_host_cap) {
        if (db->pos_host)
            hipHostFree(db->pos_host);
        db->pos_host = nullptr;
        db->pos_host_cap = 0;
        void *p = nullptr;
        PIR_TRY(host_mapped((npos + nb + 1) * 4, &p, &db->pos_map));
        db->pos_host = static_cast<uint32_t *>(p);
        db->pos_host_cap = npos + nb + 1;
    }
    uint32_t *start = db->pos_host, *sorted = db->pos_host + nb + 1;
    memset(start, 0, (nb + 1) * 4);
    for (uint32_t p : db->pos_pending)
        ++start[(p >> 5) / COMMIT_IV_WORDS + 1];
    for (uint64_t b = 0; b < nb; ++b)
        start[b + 1] += start[b];
    db->pos_cursor.assign(start, start + nb);
    for (uint32_t p : db->pos_pending)
        sorted[db->pos_cursor[(p >> 5) / COMMIT_IV_WORDS]++] = p;

    // The back copy's vector may still be read by async readers of the
    // buffer it belonged to before the last swap.
    PIR_TRY(wait_readers(db, back, db->stream));
    CommitArgs ca{};
    ca.back = reinterpret_cast<uint4 *>(db->buf[back]);
    ca.rows = static_cast<const uint4 *>(db->stage_map);
    ca.idx = static_cast<const uint64_t *>(db->stage_idx_map);
    ca.nrows = rows;
    ca.stride16 = db->stride / 16;
    ca.global = db->iv_global[back];
    ca.ring = db->iv_ring;
    ca.window = db->window;
    ca.slot = (uint32_t)(db->epoch % db->window);
    ca.words = db->iv_words;
    ca.iv_blocks = nb;
    const uint32_t *pos_dev = static_cast<const uint32_t *>(db->pos_map);
    ca.pos_start = pos_dev;
    ca.pos = pos_dev + nb + 1;
    HIP_TRY(launch_commit(ca, db->stream));
    PIR_TRY(note_upload(db, UP_POS));
    if (rows) {
        PIR_TRY(note_upload(db, UP_STAGE));  // the staging rows are refilled only after this
        db->stage_rows = 0;
        db->stage_slot.clear();
    }
    db->pos_pending.clear();

    if (!changed && !db->have_back) {
        // nothing written: only the interest vector moves. Keep the
        // snapshot where it is and copy the new vector into the front slot.
        PIR_TRY(wait_readers(db, db->front, db->stream));
        HIP_TRY(hipMemcpyAsync(db->iv_global[db->front], db->iv_global[back], db->iv_words * 4,
                               hipMemcpyDeviceToDevice, db->stream));
        HIP_TRY(hipEventRecord(db->published, db->stream));
        db->epoch++;
        if (epoch_out)
            *epoch_out = db->epoch;
        return PIR_OK;
    }
    // publish: swap the copies (the leaf databases of preprocessed reads
    // are brought up to the new snapshot first: the leaf rows that this
    // epoch's buckets feed while those buckets number at most a quarter of
    // the leaf rows, else all of them)
    const bool few = !db->all_dirty && !db->dirty.empty() && db->dirty.size() * 2 <= db->n;
    const uint64_t *dirty_dev = nullptr;
    if (few)
        PIR_TRY(upload_dirty(db, &dirty_dev));
    if (db->prep)
        PIR_TRY(build_prep(db, back, few && db->dirty.size() * 4 <= db->prep_Nq ? dirty_dev : nullptr));
    HIP_TRY(hipEventRecord(db->published, db->stream));
    const int old_front = db->front;
    db->front = back;
    // replay this epoch's buckets into the new back copy once its readers
    // are done
    PIR_TRY(wait_readers(db, old_front, db->stream));
    if (db->all_dirty || db->dirty.size() * 2 > db->n) {
        HIP_TRY(hipMemcpyAsync(db->buf[old_front], db->buf[db->front], db->n * db->stride, hipMemcpyDeviceToDevice,
                               db->stream));
    } else if (few) {
        HIP_TRY(launch_copy_rows(db->buf[old_front], db->buf[db->front], dirty_dev, db->dirty.size(), db->stride,
                                 db->stream));
    }
    if (few)
        PIR_TRY(note_upload(db, UP_MIRROR));
    // no host wait: the rest of the commit runs stream-ordered on the device
    for (uint64_t b : db->dirty)
        db->dirty_mark[b] = 0;
    db->dirty.clear();
    db->all_dirty = false;
    db->epoch++;
    if (epoch_out)
        *epoch_out = db->epoch;
    return PIR_OK;
}

uint64_t pir_epoch(const pir_db *db) { return db ? db->epoch : 0; }

int pir_preprocess_tables(uint32_t levels, uint32_t *leaves, uint8_t *a_cnt, uint8_t *a, uint8_t *d_cnt, uint8_t *d,
                          uint8_t *o_cnt, uint8_t *o_leaf)
{
    PrepTables t;
    if (!leaves || !a_cnt || !a || !d_cnt || !d || !o_cnt || !o_leaf || !prep_tables(levels, &t))
        return PIR_EINVAL;
    *leaves = t.leaves;
    memcpy(a_cnt, t.a_cnt, sizeof t.a_cnt);
    memcpy(a, t.a, sizeof t.a);
    memcpy(d_cnt, t.d_cnt, sizeof t.d_cnt);
    memcpy(d, t.d, sizeof t.d);
    memcpy(o_cnt, t.o_cnt, sizeof t.o_cnt);
    memcpy(o_leaf, t.o_leaf, sizeof t.o_leaf);
    return PIR_OK;
}

int pir_preprocess(pir_db *db, uint32_t levels, uint32_t min_batch)
{
    if (!db || levels > PREP_MAX_LEVELS)
        return PIR_EINVAL;
    if (levels && (db->bucket_bytes % (16ull << levels) != 0))
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    if (db->prep) {
        // the reads still using the old leaves finish before they go
        PIR_TRY(wait_readers(db, 2, db->stream));
        HIP_TRY(hipStreamSynchronize(db->stream));
        HIP_TRY(hipFree(db->prep));
        db->prep = nullptr;
        db->prep_levels = 0;
    }
    if (levels == 0)
        return PIR_OK;
    PrepTables t;
    if (!prep_tables(levels, &t))
        return PIR_EINVAL;
    const uint64_t unit = 32ull << levels;
    const uint64_t Nq = (db->n + unit - 1) / unit * unit >> levels;
    const uint32_t Cq = (uint32_t)(db->bucket_bytes >> levels);
    const uint64_t leaf_bytes = (padded_db_rows(Nq) * Cq + 255) & ~255ull;
    void *p = nullptr;
    if (hipMalloc(&p, leaf_bytes * t.leaves) != hipSuccess) {
        (void)hipGetLastError();
        return PIR_ENOMEM;
    }
    db->prep = static_cast<uint8_t *>(p);
    db->prep_t = t;
    db->prep_levels = levels;
    db->prep_min_batch = min_batch ? min_batch : (256u << levels);
    db->prep_leaf_bytes = leaf_bytes;
    db->prep_Nq = Nq;
    db->prep_Cq = Cq;
    // rows past Nq of every leaf stay zero (the kernels may read them)
    HIP_TRY(launch_fill_zero(db->prep, leaf_bytes * t.leaves, db->stream));
    PIR_TRY(build_prep(db, db->front, nullptr));
    HIP_TRY(hipEventRecord(db->published, db->stream));
    return PIR_OK;
}

// Next timing event pair for a read, or {nullptr, nullptr} when timing is
// off or the record is full.
static int profile_slot(pir_db *db, hipEvent_t *eb, hipEvent_t *ee)
{
    *eb = *ee = nullptr;
    if (!db->prof_on || db->prof_used >= PIR_PROFILE_MAX || (db->prof_count++ % db->prof_every) != 0)
        return PIR_OK;
    if (db->prof_used == db->prof_ev.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        HIP_TRY(hipEventCreate(&a));
        if (hipEventCreate(&b) != hipSuccess) {
            hipEventDestroy(a);
            return PIR_EDEVICE;
        }
        db->prof_ev.emplace_back(a, b);
    }
    *eb = db->prof_ev[db->prof_used].first;
    *ee = db->prof_ev[db->prof_used].second;
    ++db->prof_used;
    return PIR_OK;
}

// Sizes of a preprocessed read of B rows: Bq request blocks of Nq bits
// (Wq words, pitch qpl) per leaf, Cq-byte leaf answers, and the per-leaf
// spans of the request and answer scratch.
struct LeafShape {
    uint32_t Bq;
    uint64_t Nq, Wq, qpl, q_leaf, o_leaf;
    uint32_t Cq;
};

static LeafShape leaf_shape(const pir_db *db, uint32_t B)
{
    LeafShape l{};
    l.Bq = (B + db->prep_t.grid - 1) / db->prep_t.grid;
    l.Nq = db->prep_Nq;
    l.Wq = l.Nq / 32;
    l.Cq = db->prep_Cq;
    l.qpl = (l.Wq * 4 + 15) & ~15ull;                   // leaf request pitch
    l.q_leaf = ((uint64_t)l.Bq * l.qpl + 255) & ~255ull;
    l.o_leaf = ((uint64_t)l.Bq * l.Cq + 255) & ~255ull;
    return l;
}

// Staged entries of all leaves of one read above this many bytes go back to
// leaf request rows and a staging kernel per leaf; split partials of all
// leaves above this many bytes, to a launch per leaf.
constexpr uint64_t PREP_STAGE_MAX = 32ull << 30;
constexpr uint64_t PREP_PARTIAL_MAX = 8ull << 30;

// A preprocessed read's leaf geometry (D, Q and out set per leaf), plan,
// what sc.leaf_q holds per leaf (the 16-bit pair-table entries of its
// request rows when staged, else the rows themselves), the bytes per leaf answer block in
// sc.leaf_out, and whether one launch answers every leaf.
struct LeafRead {
    LeafShape l;
    ReadGeom g;
    Plan p;
    bool staged, fused;
    uint64_t q_leaf, o_leaf;
};

// The request side of every leaf: it depends on the requests only, not on
// the snapshot, so a read enqueues it before it waits for the latest
// publication. Under a pair-table plan one launch stages every leaf's
// table entries straight from the request rows; otherwise the leaves'
// request rows are formed for their reads to stage.
static int prep_requests(pir_db *db, Scratch &sc, const void *q, uint64_t qp, uint32_t B, hipStream_t s,
                         LeafRead *lr)
{
    const PrepTables &t = db->prep_t;
    lr->l = leaf_shape(db, B);
    const LeafShape &l = lr->l;
    ReadGeom &g = lr->g;
    g = ReadGeom{};
    g.n = l.Nq;
    g.stride = l.Cq;
    g.qpitch = l.qpl;
    g.B = l.Bq;
    g.out_pitch = l.Cq;
    Plan want = db->forced;
    if (want.kind == KIND_AUTO) {
        Plan tuned;
        if (tune_lookup(l.Nq, l.Bq, l.Cq, &tuned))
            want = tuned;
    }
    lr->p = resolve_plan(g, want, db->num_cus);
    lr->staged = leaf_staging_supported(g, lr->p, t.leaves) &&
                 m4rw_staging_bytes(g, lr->p, true) * t.leaves <= PREP_STAGE_MAX;
    lr->q_leaf = lr->staged ? m4rw_staging_bytes(g, lr->p, true) : l.q_leaf;
    // one launch for every leaf: the leaves' answers are consecutive row
    // blocks of Bq rows
    const uint64_t split_bytes = lr->p.splits <= 1 ? 0 : (uint64_t)lr->p.splits * l.Bq * l.Cq;
    lr->fused = lr->staged && split_bytes * t.leaves <= PREP_PARTIAL_MAX;
    lr->o_leaf = lr->fused ? (uint64_t)l.Bq * l.Cq : l.o_leaf;
    PIR_TRY(ensure_device(&sc.leaf_q, &sc.leaf_q_cap, lr->q_leaf * t.leaves));
    PIR_TRY(ensure_device(&sc.leaf_out, &sc.leaf_out_cap, lr->o_leaf * t.leaves));
    if (lr->staged)
        HIP_TRY(launch_stage_leaf_pairs(t, q, qp, B, db->n, g, lr->p, sc.leaf_q, lr->q_leaf, s));
    else
        HIP_TRY(launch_prep_q(t, q, qp, B, db->n, l.Bq, l.Wq, sc.leaf_q, l.qpl, l.q_leaf, s));
    return PIR_OK;
}

// Preprocessed read of B rows, whose request side prep_requests enqueued on
// stream s, into out (pitch op): the 7^L leaf products with the
// Four-Russians kernels (one launch for all of them when their entries are
// staged), then the answers from the products (masked in place when keys are
// given). `done` is recorded by the last kernel; eb / ee take the start of
// the first leaf's main kernel and the end of the last one's.
static int prep_read(pir_db *db, Scratch &sc, const LeafRead &lr, uint32_t B, void *out, uint64_t op,
                     const uint32_t *keys, hipStream_t s, hipEvent_t eb, hipEvent_t ee, hipEvent_t done)
{
    const PrepTables &t = db->prep_t;
    ReadGeom g = lr.g;
    if (lr.staged)
        g.staged = static_cast<const uint32_t *>(sc.leaf_q);
    if (lr.fused) {
        g.leaves = t.leaves;
        g.leaf_d_bytes = db->prep_leaf_bytes;
        g.leaf_stage_bytes = lr.q_leaf;
        g.D = db->prep;
        g.out = sc.leaf_out;
        PIR_TRY(ensure_device(&sc.part, &sc.part_cap, partial_bytes(g, lr.p)));
        HIP_TRY(launch_read(g, lr.p, sc.part, s, eb, ee));
    } else {
        PIR_TRY(ensure_device(&sc.part, &sc.part_cap, partial_bytes(g, lr.p)));
        for (uint32_t l = 0; l < t.leaves; ++l) {
            g.D = db->prep + l * db->prep_leaf_bytes;
            uint8_t *lq = static_cast<uint8_t *>(sc.leaf_q) + l * lr.q_leaf;
            if (lr.staged)
                g.staged = reinterpret_cast<const uint32_t *>(lq);
            else
                g.Q = lq;
            g.out = static_cast<uint8_t *>(sc.leaf_out) + l * lr.o_leaf;
            HIP_TRY(launch_read(g, lr.p, sc.part, s, l == 0 ? eb : nullptr, l + 1 == t.leaves ? ee : nullptr));
        }
    }
    HIP_TRY(launch_prep_out(t, sc.leaf_out, lr.o_leaf, B, lr.l.Bq, lr.l.Cq, out, op, s, keys ? nullptr : done));
    if (keys)
        HIP_TRY(launch_mask_rows(nullptr, 0, B, db->stride, out, op, keys, s, done));
    return PIR_OK;
}

static bool use_prep(const pir_db *db, uint32_t B) { return db->prep && B >= db->prep_min_batch; }

// Synchronous read (host rows in and out); seeds = B x 32 bytes of mask
// seeds, or NULL for the plain answers.
static int read_sync(pir_db *db, const uint8_t *req_bits, uint32_t B, const uint8_t *seeds, uint8_t *resp)
{
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    Scratch &sc = scratch_for(db, db->stream);
    PIR_TRY(ensure_device(&sc.req, &sc.req_cap, (uint64_t)B * db->qpitch));
    PIR_TRY(ensure_device(&sc.resp, &sc.resp_cap, (uint64_t)B * db->stride));
    // Host rows move in one contiguous copy each way (a pitched copy from or
    // to pageable memory goes row by row); pitches change on the device.
    const uint64_t qb = db->qbytes, in_bytes = (uint64_t)B * qb, out_bytes = (uint64_t)B * db->bucket_bytes;
    const bool q_direct = qb % 4 == 0, r_direct = db->stride == db->bucket_bytes;
    if (!q_direct || !r_direct)
        PIR_TRY(ensure_device(&sc.host_rows, &sc.host_rows_cap, std::max(q_direct ? 0 : in_bytes,
                                                                           r_direct ? 0 : out_bytes)));
    uint64_t qp = qb;
    if (q_direct) {
        HIP_TRY(hipMemcpyAsync(sc.req, req_bits, in_bytes, hipMemcpyHostToDevice, db->stream));
    } else {
        HIP_TRY(hipMemcpyAsync(sc.host_rows, req_bits, in_bytes, hipMemcpyHostToDevice, db->stream));
        HIP_TRY(hipMemcpy2DAsync(sc.req, db->qpitch, sc.host_rows, qb, qb, B, hipMemcpyDeviceToDevice, db->stream));
        qp = db->qpitch;
    }
    ReadGeom g = read_geom(db, sc.req, qp, B, sc.resp, db->stride);
    if (seeds) {
        PIR_TRY(ensure_device(&sc.keys, &sc.keys_cap, (uint64_t)B * 32));
        HIP_TRY(hipMemcpyAsync(sc.keys, seeds, (uint64_t)B * 32, hipMemcpyHostToDevice, db->stream));
        g.keys = static_cast<const uint32_t *>(sc.keys);
    }
    hipEvent_t eb, ee;
    PIR_TRY(profile_slot(db, &eb, &ee));
    if (use_prep(db, B)) {
        LeafRead lr;
        PIR_TRY(prep_requests(db, sc, sc.req, qp, B, db->stream, &lr));
        PIR_TRY(prep_read(db, sc, lr, B, sc.resp, db->stride, g.keys, db->stream, eb, ee, nullptr));
    } else {
        Plan p = choose_plan(db, B);
        PIR_TRY(ensure_device(&sc.part, &sc.part_cap, partial_bytes(g, p)));
        HIP_TRY(launch_read(g, p, sc.part, db->stream, eb, ee));
    }
    if (r_direct) {
        HIP_TRY(hipMemcpyAsync(resp, sc.resp, out_bytes, hipMemcpyDeviceToHost, db->stream));
    } else {
        HIP_TRY(hipMemcpy2DAsync(sc.host_rows, db->bucket_bytes, sc.resp, db->stride, db->bucket_bytes, B,
                                 hipMemcpyDeviceToDevice, db->stream));
        HIP_TRY(hipMemcpyAsync(resp, sc.host_rows, out_bytes, hipMemcpyDeviceToHost, db->stream));
    }
    HIP_TRY(hipStreamSynchronize(db->stream));
    return PIR_OK;
}

// Stream-ordered read of device rows; d_keys = B x 8 key words on the device
// (4-byte aligned), or NULL.
static int read_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B, const void *d_keys,
                      void *d_resp, uint64_t resp_pitch, void *hip_stream)
{
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    Scratch &sc = scratch_for(db, s);
    const void *q = d_req;
    uint64_t qp = req_pitch;
    // The kernel reads whole 32-bit request words: rows must be 4-byte
    // aligned and the last word of every row must lie inside it.
    if ((reinterpret_cast<uintptr_t>(d_req) & 3) || (req_pitch & 3) || (db->qbytes & 3)) {
        PIR_TRY(ensure_device(&sc.req, &sc.req_cap, (uint64_t)B * db->qpitch));
        HIP_TRY(hipMemcpy2DAsync(sc.req, db->qpitch, d_req, req_pitch, db->qbytes, B, hipMemcpyDeviceToDevice, s));
        q = sc.req;
        qp = db->qpitch;
    }
    // work that needs only the requests goes out before the wait for the
    // latest publication
    const bool prep = use_prep(db, B);
    LeafRead lr;
    if (prep)
        PIR_TRY(prep_requests(db, sc, q, qp, B, s, &lr));
    PIR_TRY(wait_published(db, s));
    const bool direct = !(reinterpret_cast<uintptr_t>(d_resp) & 15) && !(resp_pitch & 15) &&
                        db->stride == db->bucket_bytes;
    void *out = d_resp;
    uint64_t op = resp_pitch;
    if (!direct) {
        PIR_TRY(ensure_device(&sc.resp, &sc.resp_cap, (uint64_t)B * db->stride));
        out = sc.resp;
        op = db->stride;
    }
    ReadGeom g = read_geom(db, q, qp, B, out, op);
    g.keys = static_cast<const uint32_t *>(d_keys);
    hipEvent_t eb, ee, done;
    PIR_TRY(profile_slot(db, &eb, &ee));
    PIR_TRY(reader_event(db, prep ? 2 : db->front, s, &done));
    if (prep) {
        PIR_TRY(prep_read(db, sc, lr, B, out, op, g.keys, s, eb, ee, direct ? done : nullptr));
    } else {
        Plan p = choose_plan(db, B);
        PIR_TRY(ensure_device(&sc.part, &sc.part_cap, partial_bytes(g, p)));
        if (direct)
            g.done = done;  // the read's last kernel marks the end of its use of the snapshot
        HIP_TRY(launch_read(g, p, sc.part, s, eb, ee));
    }
    if (direct)
        return PIR_OK;
    HIP_TRY(hipMemcpy2DAsync(d_resp, resp_pitch, sc.resp, db->stride, db->bucket_bytes, B,
                             hipMemcpyDeviceToDevice, s));
    return hipEventRecord(done, s) == hipSuccess ? PIR_OK : PIR_EDEVICE;
}

int pir_read_batch(pir_db *db, const uint8_t *req_bits, uint32_t B, uint8_t *resp)
{
    if (!db)
        return PIR_EINVAL;
    if (B == 0)
        return PIR_OK;
    if (!req_bits || !resp)
        return PIR_EINVAL;
    return read_sync(db, req_bits, B, nullptr, resp);
}

int pir_read_batch_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B, void *d_resp,
                         uint64_t resp_pitch, void *hip_stream)
{
    if (!db)
        return PIR_EINVAL;
    if (B == 0)
        return PIR_OK;
    if (!d_req || !d_resp || req_pitch < db->qbytes || resp_pitch < db->bucket_bytes)
        return PIR_EINVAL;
    return read_async(db, d_req, req_pitch, B, nullptr, d_resp, resp_pitch, hip_stream);
}

int pir_read_batch_masked(pir_db *db, const uint8_t *req_bits, uint32_t B, const uint8_t *seeds, uint8_t *resp)
{
    if (!db)
        return PIR_EINVAL;
    if (B == 0)
        return PIR_OK;
    if (!req_bits || !seeds || !resp)
        return PIR_EINVAL;
    return read_sync(db, req_bits, B, seeds, resp);
}

int pir_read_batch_masked_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B, const void *d_seeds,
                                void *d_resp, uint64_t resp_pitch, void *hip_stream)
{
    if (!db)
        return PIR_EINVAL;
    if (B == 0)
        return PIR_OK;
    if (!d_req || !d_seeds || !d_resp || req_pitch < db->qbytes || resp_pitch < db->bucket_bytes ||
        (reinterpret_cast<uintptr_t>(d_seeds) & 3))
        return PIR_EINVAL;
    return read_async(db, d_req, req_pitch, B, d_seeds, d_resp, resp_pitch, hip_stream);
}

int pir_xor_combine_async(void *d_out, uint64_t out_pitch, const void *const *d_in, uint32_t l, uint64_t in_pitch,
                          uint32_t B, uint64_t row_bytes, void *hip_stream)
{
    if (B == 0)
        return PIR_OK;
    if (!d_out || !d_in || l == 0 || l > COMBINE_MAX || row_bytes == 0 || (row_bytes & 15) ||
        out_pitch < row_bytes || in_pitch < row_bytes || (out_pitch & 15) || (in_pitch & 15) ||
        (reinterpret_cast<uintptr_t>(d_out) & 15))
        return PIR_EINVAL;
    CombineArgs a{};
    a.out = static_cast<uint4 *>(d_out);
    a.out_row16 = out_pitch / 16;
    for (uint32_t i = 0; i < l; ++i) {
        if (!d_in[i] || (reinterpret_cast<uintptr_t>(d_in[i]) & 15))
            return PIR_EINVAL;
        a.in[i] = static_cast<const uint4 *>(d_in[i]);
    }
    a.in_row16 = in_pitch / 16;
    a.l = l;
    a.B = B;
    a.row16 = row_bytes / 16;
    HIP_TRY(launch_xor_combine(a, static_cast<hipStream_t>(hip_stream)));
    return PIR_OK;
}

int pir_set_plan(pir_db *db, const pir_plan *plan)
{
    if (!db || !plan)
        return PIR_EINVAL;
    Plan p{plan->kind, plan->tile, plan->splits, plan->unroll, plan->flags};
    if (p.kind < KIND_AUTO || p.kind > KIND_M4RW)
        return PIR_EINVAL;
    if (p.kind != KIND_AUTO) {
        ReadGeom g = read_geom(db, nullptr, db->qpitch, std::max<uint32_t>(p.tile, 1), nullptr, db->stride);
        Plan full = resolve_plan(g, p, db->num_cus);
        if (!plan_supported(full))
            return PIR_EINVAL;
    }
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    db->forced = p;
    return PIR_OK;
}

int pir_get_plan(pir_db *db, uint32_t B, pir_plan *plan)
{
    if (!db || !plan)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    Plan p = choose_plan(db, std::max<uint32_t>(B, 1));
    plan->kind = p.kind;
    plan->tile = p.tile;
    plan->splits = p.splits;
    plan->unroll = p.unroll;
    plan->flags = p.flags;
    return PIR_OK;
}

int pir_interest_config(pir_db *db, uint64_t m_bits, uint32_t window_epochs)
{
    if (!db || m_bits == 0 || m_bits > (1ull << 32) || window_epochs == 0 || window_epochs > 4096)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    HIP_TRY(hipStreamSynchronize(db->stream));
    for (int b = 0; b < 2; ++b)
        for (auto &kv : db->readers[b])
            HIP_TRY(hipEventSynchronize(kv.second));
    return interest_alloc(db, m_bits, window_epochs);
}

int pir_interest_add(pir_db *db, const uint32_t *pos, uint32_t k)
{
    if (!db || (k && !pos))
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    for (uint32_t i = 0; i < k; ++i)
        if (pos[i] >= db->m_bits)
            return PIR_ERANGE;
    db->pos_pending.insert(db->pos_pending.end(), pos, pos + k);
    return PIR_OK;
}

int pir_interest_vector(pir_db *db, uint8_t *out, uint64_t out_bytes)
{
    if (!db || !out)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    const uint64_t bytes = (db->m_bits + 7) / 8;
    if (out_bytes < bytes)
        return PIR_EINVAL;
    HIP_TRY(hipSetDevice(db->device));
    HIP_TRY(hipMemcpyAsync(out, db->iv_global[db->front], bytes, hipMemcpyDeviceToHost, db->stream));
    HIP_TRY(hipStreamSynchronize(db->stream));
    return PIR_OK;
}

int pir_interest_vector_encoded(pir_db *db, uint8_t *out, uint64_t out_cap, uint64_t *out_bytes)
{
    if (!db || !out_bytes)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    return encode_interest(db, db->iv_global[db->front], db->m_bits, out, out_cap, out_bytes, db->stream);
}

int pir_interest_delta_encoded(pir_db *db, uint64_t epoch, uint8_t *out, uint64_t out_cap, uint64_t *out_bytes)
{
    if (!db || !out_bytes)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    if (epoch == 0 || epoch > db->epoch || epoch + db->window <= db->epoch)
        return PIR_ERANGE;
    HIP_TRY(hipSetDevice(db->device));
    const uint32_t *slot = db->iv_ring + ((epoch - 1) % db->window) * db->iv_words;
    return encode_interest(db, slot, db->m_bits, out, out_cap, out_bytes, db->stream);
}

int pir_interest_vector_async(pir_db *db, void *d_out, uint64_t out_bytes, void *hip_stream)
{
    if (!db || !d_out)
        return PIR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    const uint64_t bytes = (db->m_bits + 7) / 8;
    if (out_bytes < bytes)
        return PIR_EINVAL;
    HIP_TRY(hipSetDevice(db->device));
    PIR_TRY(wait_published(db, s));
    HIP_TRY(hipMemcpyAsync(d_out, db->iv_global[db->front], bytes, hipMemcpyDeviceToDevice, s));
    return note_reader(db, db->front, s);
}

}  // extern "C"

int pir_profile_enable(pir_db *db, int on)
{
    if (!db || on < 0)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    db->prof_on = on != 0;
    db->prof_every = on > 1 ? (uint32_t)on : 1u;
    db->prof_count = 0;
    db->prof_used = 0;
    return PIR_OK;
}

int pir_profile_collect(pir_db *db, float *ms, uint32_t cap, uint32_t *count)
{
    if (!db || (cap && !ms))
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    HIP_TRY(hipSetDevice(db->device));
    const size_t used = db->prof_used;
    for (size_t i = 0; i < used; ++i) {
        HIP_TRY(hipEventSynchronize(db->prof_ev[i].second));
        if (i < cap)
            HIP_TRY(hipEventElapsedTime(&ms[i], db->prof_ev[i].first, db->prof_ev[i].second));
    }
    if (count)
        *count = (uint32_t)used;
    db->prof_used = 0;
    return PIR_OK;
}
