// Uneven batch streams through the persistent work-queue kernel, captured in
// a HIP graph and replayed while the stream shape, buffers and snapshot stay
// the same (section "Evaluation": reads are batched and forwarded to the GPU;
// the leader may reorder reads).
#include <string.h>

#include <algorithm>
#include <vector>

#include "db.h"

using namespace talek;

namespace {

constexpr uint64_t CHUNK_PARTIAL_BYTES = 256ull << 20;

struct Chunk {
    uint32_t first_batch, n_batches;
    uint32_t first_item, n_items;
    uint32_t n_groups;
    uint64_t part_bytes;
};

uint32_t batch_splits(uint64_t n, uint32_t B, uint32_t n_cg, int num_cus)
{
    const uint64_t n_rt = (B + QUEUE_TILE - 1) / QUEUE_TILE;
    const uint64_t units = n_rt * n_cg;
    const uint64_t nwords = (n + 31) / 32;
    uint64_t s = (2ull * std::max(num_cus, 1) + units - 1) / units;
    s = std::min<uint64_t>(s, std::max<uint64_t>(nwords / 2, 1));
    return (uint32_t)std::max<uint64_t>(s, 1);
}

}  // namespace

extern "C" int pir_read_stream_async(pir_db *db, const void *d_req, uint64_t req_pitch, const uint32_t *sizes,
                                     const uint64_t *req_first, uint32_t n_batches, void *d_resp,
                                     uint64_t resp_pitch, const uint64_t *resp_first, void *hip_stream)
{
    if (!db)
        return PIR_EINVAL;
    if (n_batches == 0)
        return PIR_OK;
    if (!sizes || !d_req || !d_resp)
        return PIR_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_req) & 3) || (req_pitch & 3) || (db->qbytes & 3) ||
        req_pitch < db->qbytes)
        return PIR_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_resp) & 15) || (resp_pitch & 15) || db->stride != db->bucket_bytes ||
        resp_pitch < db->bucket_bytes)
        return PIR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    if (hipSetDevice(db->device) != hipSuccess)
        return PIR_EDEVICE;

    const uint32_t stride16 = (uint32_t)(db->stride / 16);
    const uint32_t n_cg = (stride16 + 255) / 256;
    const uint64_t nwords = (db->n + 31) / 32;

    // Work tables for all chunks.
    std::vector<QueueBatch> batches(n_batches);
    std::vector<QueueItem> items;
    std::vector<Chunk> chunks;
    uint64_t req_row = 0, resp_row = 0;
    Chunk cur{0, 0, 0, 0, 0, 0};
    uint64_t max_part = 0;
    for (uint32_t k = 0; k < n_batches; ++k) {
        const uint32_t B = sizes[k];
        QueueBatch &bt = batches[k];
        memset(&bt, 0, sizeof bt);
        const uint64_t rq = req_first ? req_first[k] : req_row;
        const uint64_t rs = resp_first ? resp_first[k] : resp_row;
        req_row = rq + B;
        resp_row = rs + B;
        bt.q_off = rq * req_pitch;
        bt.out_off = rs * resp_pitch;
        bt.B = B;
        if (B == 0)
            continue;
        bt.n_cg = n_cg;
        bt.n_rt = (B + QUEUE_TILE - 1) / QUEUE_TILE;
        bt.splits = batch_splits(db->n, B, n_cg, db->num_cus);
        bt.words_per_split = (uint32_t)((nwords + bt.splits - 1) / bt.splits);
        bt.splits = (uint32_t)((nwords + bt.words_per_split - 1) / bt.words_per_split);
        const uint64_t part = bt.splits > 1 ? (uint64_t)bt.splits * B * db->stride : 0;
        if (cur.n_batches && cur.part_bytes + part > CHUNK_PARTIAL_BYTES) {
            chunks.push_back(cur);
            cur = Chunk{k, 0, (uint32_t)items.size(), 0, 0, 0};
        }
        if (cur.n_batches == 0) {
            cur.first_batch = k;
            cur.first_item = (uint32_t)items.size();
        }
        bt.part_off = cur.part_bytes;
        bt.group_base = cur.n_groups;
        cur.part_bytes += part;
        cur.n_groups += bt.splits > 1 ? bt.n_rt * n_cg : 0;
        for (uint32_t sp = 0; sp < bt.splits; ++sp)
            for (uint32_t cg = 0; cg < n_cg; ++cg)
                for (uint32_t rt = 0; rt < bt.n_rt; ++rt)
                    items.push_back(QueueItem{k, rt, sp, cg});
        cur.n_batches = k + 1 - cur.first_batch;
        cur.n_items = (uint32_t)items.size() - cur.first_item;
        max_part = std::max(max_part, cur.part_bytes);
    }
    if (cur.n_batches)
        chunks.push_back(cur);
    if (items.empty())
        return PIR_OK;

    Scratch &sc = scratch_for(db, s);
    const uint64_t batch_bytes = batches.size() * sizeof(QueueBatch);
    const uint64_t item_bytes = items.size() * sizeof(QueueItem);
    uint64_t counter_words = 0;
    for (const Chunk &c : chunks)
        counter_words += 1 + c.n_groups;
    const uint64_t aux_bytes = batch_bytes + item_bytes + counter_words * 4;

    void *old_aux = sc.aux, *old_part = sc.part;
    int rc = ensure_device(&sc.aux, &sc.aux_cap, aux_bytes);
    if (rc == PIR_OK)
        rc = ensure_device(&sc.part, &sc.part_cap, std::max<uint64_t>(max_part, 16));
    if (rc != PIR_OK)
        return rc;
    if (sc.aux != old_aux || sc.part != old_part)
        destroy_stream_graph(sc);

    // Signature of everything the captured graph bakes in.
    std::vector<uint64_t> sig;
    sig.reserve(8 + 2 * n_batches);
    sig.push_back(reinterpret_cast<uintptr_t>(db->buf[db->front]));
    sig.push_back(reinterpret_cast<uintptr_t>(d_req));
    sig.push_back(req_pitch);
    sig.push_back(reinterpret_cast<uintptr_t>(d_resp));
    sig.push_back(resp_pitch);
    sig.push_back(reinterpret_cast<uintptr_t>(sc.aux));
    sig.push_back(reinterpret_cast<uintptr_t>(sc.part));
    for (uint32_t k = 0; k < n_batches; ++k) {
        sig.push_back(((uint64_t)batches[k].B << 32) ^ batches[k].q_off);
        sig.push_back(batches[k].out_off);
    }

    if (hipStreamWaitEvent(s, db->published, 0) != hipSuccess)
        return PIR_EDEVICE;
    if (sc.exec && sc.sig == sig) {
        if (hipGraphLaunch(sc.exec, s) != hipSuccess)
            return PIR_EDEVICE;
        return note_reader(db, db->front, s);
    }
    destroy_stream_graph(sc);

    // Upload the tables (stream-ordered on s, before the graph runs).
    std::vector<uint8_t> host(aux_bytes, 0);
    memcpy(host.data(), batches.data(), batch_bytes);
    memcpy(host.data() + batch_bytes, items.data(), item_bytes);
    if (hipMemcpyAsync(sc.aux, host.data(), aux_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return PIR_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess)  // host table is a temporary
        return PIR_EDEVICE;

    uint8_t *aux = static_cast<uint8_t *>(sc.aux);
    const QueueBatch *d_batches = reinterpret_cast<const QueueBatch *>(aux);
    const QueueItem *d_items = reinterpret_cast<const QueueItem *>(aux + batch_bytes);
    uint32_t *d_counters = reinterpret_cast<uint32_t *>(aux + batch_bytes + item_bytes);

    hipStream_t cap = db->capture_stream;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return PIR_EDEVICE;
    hipError_t e = hipSuccess;
    uint64_t cw = 0;
    const uint32_t grid = queue_grid(db->num_cus);
    for (const Chunk &c : chunks) {
        uint32_t *counters = d_counters + cw;
        cw += 1 + c.n_groups;
        if (e == hipSuccess)
            e = launch_fill_zero(counters, (1 + (uint64_t)c.n_groups) * 4, cap);
        QueueGeom g{};
        g.D = db->buf[db->front];
        g.n = db->n;
        g.stride = db->stride;
        g.Q = d_req;
        g.qpitch = req_pitch;
        g.out = d_resp;
        g.out_pitch = resp_pitch;
        g.partials = sc.part;
        g.items = d_items + c.first_item;
        g.batches = d_batches;
        g.head = counters;
        g.done = counters + 1;
        g.n_items = c.n_items;
        if (e == hipSuccess)
            e = launch_queue(g, std::min<uint32_t>(grid, c.n_items), cap);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph)
            hipGraphDestroy(graph);
        return PIR_EDEVICE;
    }
    e = hipGraphInstantiate(&sc.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        sc.exec = nullptr;
        return PIR_EDEVICE;
    }
    sc.sig = sig;
    if (hipGraphLaunch(sc.exec, s) != hipSuccess)
        return PIR_EDEVICE;
    return note_reader(db, db->front, s);
}
