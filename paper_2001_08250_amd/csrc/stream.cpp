// Uneven batch streams (section "Evaluation": read requests are batched and
// forwarded to the GPU; the leader may reorder reads).
//
// Every answer depends only on its own request row and the snapshot, so the
// stream's rows, in order, are cut into launch groups of FUSE_ROWS requests
// (a batch may straddle two groups; the last group takes the rest): one read
// launch per group, with that size's tuned schedule. Full groups keep every
// request tile of the Four-Russians kernel full, and each launch streams the
// database once however many batches it serves. Request rows that are not contiguous are gathered into scratch
// first; response rows that are not contiguous are scattered from scratch
// afterwards. The launch sequence is captured in a HIP graph and replayed
// while the stream shape, buffers and snapshot stay the same.
#include <string.h>

#include <algorithm>
#include <vector>

#include "db.h"

using namespace talek;

namespace {

constexpr uint32_t FUSE_ROWS = 1024;  // requests per launch group

struct Group {
    uint32_t B;
    uint64_t req_row;    // first request row when contiguous
    uint64_t resp_row;   // first response row when contiguous
    bool gather;         // request rows need gathering
    bool scatter;        // response rows need scattering
    uint64_t idx_req;    // offsets (in rows) into the uploaded index lists
    uint64_t idx_resp;
};

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

    // Absolute first rows of every batch.
    std::vector<uint64_t> rq(n_batches), rs(n_batches);
    {
        uint64_t a = 0, b = 0;
        for (uint32_t k = 0; k < n_batches; ++k) {
            rq[k] = req_first ? req_first[k] : a;
            rs[k] = resp_first ? resp_first[k] : b;
            a = rq[k] + sizes[k];
            b = rs[k] + sizes[k];
        }
    }

    // Launch groups, and the row index lists of the groups whose rows are
    // not contiguous.
    std::vector<Group> groups;
    std::vector<uint64_t> idx;
    struct Seg {
        uint32_t k, i0, cnt;  // rows i0 .. i0 + cnt - 1 of batch k
    };
    std::vector<Seg> segs;
    uint32_t k = 0, i0 = 0;
    while (k < n_batches) {
        Group gr{0, 0, 0, false, false, 0, 0};
        segs.clear();
        while (k < n_batches && gr.B < FUSE_ROWS) {
            const uint32_t left = sizes[k] - i0;
            if (left == 0) {
                ++k;
                i0 = 0;
                continue;
            }
            const uint32_t c = std::min<uint32_t>(left, FUSE_ROWS - gr.B);
            const uint64_t q = rq[k] + i0, r = rs[k] + i0;
            if (gr.B == 0) {
                gr.req_row = q;
                gr.resp_row = r;
            } else {
                gr.gather |= q != gr.req_row + gr.B;
                gr.scatter |= r != gr.resp_row + gr.B;
            }
            segs.push_back(Seg{k, i0, c});
            gr.B += c;
            i0 += c;
        }
        if (gr.B == 0)
            continue;
        if (gr.gather || gr.scatter) {
            gr.idx_req = idx.size();
            for (const Seg &sg : segs)
                for (uint32_t i = 0; i < sg.cnt; ++i)
                    idx.push_back(rq[sg.k] + sg.i0 + i);
            gr.idx_resp = idx.size();
            for (const Seg &sg : segs)
                for (uint32_t i = 0; i < sg.cnt; ++i)
                    idx.push_back(rs[sg.k] + sg.i0 + i);
        }
        groups.push_back(gr);
    }
    if (groups.empty())
        return PIR_OK;

    // Scratch: index lists (aux), gathered requests, scattered responses and
    // the largest schedule's partials / staging (part).
    uint64_t req_rows = 0, resp_rows = 0, part = 16;
    std::vector<Plan> plans(groups.size());
    for (size_t i = 0; i < groups.size(); ++i) {
        const Group &gr = groups[i];
        if (gr.gather)
            req_rows = std::max<uint64_t>(req_rows, gr.B);
        if (gr.scatter)
            resp_rows = std::max<uint64_t>(resp_rows, gr.B);
        plans[i] = choose_plan(db, gr.B);
        ReadGeom g = read_geom(db, d_req, req_pitch, gr.B, d_resp, resp_pitch);
        part = std::max<uint64_t>(part, partial_bytes(g, plans[i]));
    }
    const uint64_t idx_bytes = (idx.size() * 8 + 255) & ~255ull;
    const uint64_t req_bytes = (req_rows * db->qpitch + 255) & ~255ull;
    const uint64_t resp_bytes = resp_rows * db->stride;
    Scratch &sc = scratch_for(db, s);
    void *old_aux = sc.aux, *old_part = sc.part;
    int rc = ensure_device(&sc.aux, &sc.aux_cap, std::max<uint64_t>(idx_bytes + req_bytes + resp_bytes, 16));
    if (rc == PIR_OK)
        rc = ensure_device(&sc.part, &sc.part_cap, part);
    if (rc != PIR_OK)
        return rc;
    if (sc.aux != old_aux || sc.part != old_part)
        destroy_stream_graph(sc);
    uint8_t *aux = static_cast<uint8_t *>(sc.aux);
    const uint64_t *d_idx = reinterpret_cast<const uint64_t *>(aux);
    uint8_t *req_scratch = aux + idx_bytes;
    uint8_t *resp_scratch = aux + idx_bytes + req_bytes;

    // Signature of everything the captured graph bakes in.
    std::vector<uint64_t> sig;
    sig.reserve(8 + 4 * groups.size() + idx.size());
    sig.push_back(reinterpret_cast<uintptr_t>(db->buf[db->front]));
    sig.push_back(reinterpret_cast<uintptr_t>(d_req));
    sig.push_back(req_pitch);
    sig.push_back(reinterpret_cast<uintptr_t>(d_resp));
    sig.push_back(resp_pitch);
    sig.push_back(reinterpret_cast<uintptr_t>(sc.aux));
    sig.push_back(reinterpret_cast<uintptr_t>(sc.part));
    for (size_t i = 0; i < groups.size(); ++i) {
        const Group &gr = groups[i];
        const Plan &p = plans[i];
        sig.push_back(((uint64_t)gr.B << 32) | (gr.gather ? 2u : 0u) | (gr.scatter ? 1u : 0u));
        sig.push_back(gr.req_row);
        sig.push_back(gr.resp_row);
        sig.push_back(((uint64_t)p.kind << 56) ^ ((uint64_t)p.tile << 40) ^ ((uint64_t)p.unroll << 32) ^
                      ((uint64_t)p.flags << 16) ^ p.splits);
    }
    sig.insert(sig.end(), idx.begin(), idx.end());

    if (wait_published(db, s) != PIR_OK)
        return PIR_EDEVICE;
    if (sc.exec && sc.sig == sig) {
        if (hipGraphLaunch(sc.exec, s) != hipSuccess)
            return PIR_EDEVICE;
        return note_reader(db, db->front, s);
    }
    destroy_stream_graph(sc);

    if (!idx.empty()) {  // index lists, stream-ordered before the graph runs
        if (hipMemcpyAsync(sc.aux, idx.data(), idx.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)  // idx is a temporary
            return PIR_EDEVICE;
    }

    hipStream_t cap = db->capture_stream;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return PIR_EDEVICE;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < groups.size() && e == hipSuccess; ++i) {
        const Group &gr = groups[i];
        const void *q = static_cast<const uint8_t *>(d_req) + gr.req_row * req_pitch;
        uint64_t qp = req_pitch;
        if (gr.gather) {
            e = launch_move_rows(req_scratch, db->qpitch, nullptr, d_req, req_pitch, d_idx + gr.idx_req, gr.B,
                                 db->qbytes, cap);
            q = req_scratch;
            qp = db->qpitch;
        }
        void *out = static_cast<uint8_t *>(d_resp) + gr.resp_row * resp_pitch;
        uint64_t op = resp_pitch;
        if (gr.scatter) {
            out = resp_scratch;
            op = db->stride;
        }
        if (e == hipSuccess)
            e = launch_read(read_geom(db, q, qp, gr.B, out, op), plans[i], sc.part, cap);
        if (e == hipSuccess && gr.scatter)
            e = launch_move_rows(d_resp, resp_pitch, d_idx + gr.idx_resp, resp_scratch, db->stride, nullptr, gr.B,
                                 db->bucket_bytes, cap);
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
