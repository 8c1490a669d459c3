// Internal definition of the pir_db handle, shared by the host-side sources.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/talek_pir.h"
#include "engine.h"

namespace talek {

// Device scratch owned per HIP stream, so concurrent reads on different
// streams never share partial or restaging buffers.
struct Scratch {
    void *req = nullptr;
    uint64_t req_cap = 0;
    void *resp = nullptr;
    uint64_t resp_cap = 0;
    void *part = nullptr;
    uint64_t part_cap = 0;
    void *aux = nullptr;      // stream index lists and gathered rows
    uint64_t aux_cap = 0;
    void *keys = nullptr;     // mask seeds of a synchronous masked read
    uint64_t keys_cap = 0;
    void *host_rows = nullptr;  // synchronous reads: contiguous rows next to a host copy
    uint64_t host_rows_cap = 0;
    void *leaf_q = nullptr;   // preprocessed reads: leaf requests and products
    uint64_t leaf_q_cap = 0;
    void *leaf_out = nullptr;
    uint64_t leaf_out_cap = 0;
    hipGraphExec_t exec = nullptr;  // captured stream read
    std::vector<uint64_t> sig;      // what the captured graph bakes in
};

int hip_status(hipError_t e);  // hipSuccess -> PIR_OK, else PIR_EDEVICE

// Grow a device buffer to at least `bytes` (contents are not kept).
int ensure_device(void **p, uint64_t *cap, uint64_t bytes);

void destroy_stream_graph(Scratch &sc);

}  // namespace talek

struct pir_db {
    std::recursive_mutex mu;
    int device = 0;
    int num_cus = 256;
    uint64_t n = 0;
    uint32_t d = 0, z = 0;
    uint64_t bucket_bytes = 0;  // d * z
    uint64_t stride = 0;        // bucket_bytes rounded up to 16
    uint64_t qbytes = 0;        // ceil(n / 8)
    uint64_t qpitch = 0;        // internal request pitch (multiple of 16)
    uint64_t rows_alloc = 0;    // device rows per snapshot copy (n plus zero padding)
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;  // graph capture only, never executes

    // double-buffered snapshot: buf[front] is published, buf[front ^ 1] is
    // the back copy that receives staged writes
    uint8_t *buf[2] = {nullptr, nullptr};
    int front = 0;
    bool have_back = false;
    uint64_t epoch = 0;
    hipEvent_t published = nullptr;  // end of the last commit's device work
    // events recorded after async reads, per buffer and per stream; index 2
    // tracks the readers of the preprocessed leaf databases
    std::map<hipStream_t, hipEvent_t> readers[3];

    // staged bucket writes (mapped pinned host rows, `stride` bytes each;
    // the commit kernels read them in place through the *_map pointers)
    uint8_t *stage_host = nullptr;
    uint64_t *stage_idx_host = nullptr;
    void *stage_map = nullptr;
    void *stage_idx_map = nullptr;
    uint64_t stage_cap = 0;   // rows
    uint64_t stage_rows = 0;
    std::unordered_map<uint64_t, uint64_t> stage_slot;
    // buckets changed in the open epoch
    std::vector<uint8_t> dirty_mark;
    std::vector<uint64_t> dirty;
    bool all_dirty = false;

    std::unordered_map<hipStream_t, talek::Scratch> scratch;
    // Its address keys the allocation-free reads' reader events in
    // readers[0] and readers[1] (created with the handle; never a stream).
    char noalloc_key = 0;
    talek::Plan forced{0, 0, 0, 0, 0};

    // interest vector
    uint64_t m_bits = 0;
    uint64_t iv_words = 0;
    uint32_t window = 0;
    uint32_t *iv_ring = nullptr;       // window x iv_words
    uint32_t *iv_global[2] = {nullptr, nullptr};
    std::vector<uint32_t> pos_pending;
    uint32_t *pos_host = nullptr;      // mapped pinned
    void *pos_map = nullptr;
    uint64_t pos_host_cap = 0;         // u32 entries
    std::vector<uint32_t> pos_cursor;  // counting-sort cursors

    // Each mapped pinned buffer is free for the host again once its event
    // (recorded after the kernel that reads it) has completed: 0 = staged
    // rows and indices, 1 = interest positions, 2 = mirror indices.
    hipEvent_t upload_ev[3] = {nullptr, nullptr, nullptr};
    bool upload_pending[3] = {false, false, false};
    uint64_t *mirror_idx_host = nullptr;  // mapped pinned
    void *mirror_map = nullptr;
    // kernel timing (pir_profile_*): event pairs, created on first use
    bool prof_on = false;
    uint32_t prof_every = 1;        // record every prof_every-th read
    uint64_t prof_count = 0;        // reads issued since the enable
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    size_t prof_used = 0;
    // compressed interest vectors: device scratch of the encoder
    void *codec = nullptr, *codec2 = nullptr, *codec3 = nullptr;
    uint64_t codec_cap = 0, codec2_cap = 0, codec3_cap = 0;
    uint64_t mirror_idx_cap = 0;
    // preprocessed reads: the Strassen leaf databases of the published
    // snapshot, rebuilt by every commit that changes it
    uint32_t prep_levels = 0;       // 0 = off
    uint32_t prep_min_batch = 0;    // reads with B >= this take the leaves
    talek::PrepTables prep_t{};
    uint8_t *prep = nullptr;        // prep_t.leaves x prep_leaf_bytes
    uint64_t prep_leaf_bytes = 0;
    uint64_t prep_Nq = 0;           // bucket rows per block (multiple of 32)
    uint32_t prep_Cq = 0;           // bytes per bucket block
};

namespace talek {
// Schedule for a read of B rows on db (forced plan, tuning table, heuristic).
Plan choose_plan(pir_db *db, uint32_t B);
// Geometry of a read of B rows of the published snapshot.
ReadGeom read_geom(pir_db *db, const void *q, uint64_t qpitch, uint32_t B, void *out, uint64_t out_pitch);
// Scratch of a stream (created on first use).
Scratch &scratch_for(pir_db *db, hipStream_t s);
// Order `s` after the latest publication.
int wait_published(pir_db *db, hipStream_t s);
// Device address of the allocation-free reads' static scratch on `device`
// (the current device), taken once per device.
int noalloc_setup(int device);
inline hipStream_t noalloc_reader_key(pir_db *db) { return reinterpret_cast<hipStream_t>(&db->noalloc_key); }
// Compressed stream of the m-bit device vector `words` into host memory (out
// may be NULL: size only); stream-ordered on s, returns when done.
int encode_interest(pir_db *db, const uint32_t *words, uint64_t m, uint8_t *out, uint64_t cap, uint64_t *out_bytes,
                    hipStream_t s);
// Record that stream s reads buffer b (commits wait for it before reusing b).
int note_reader(pir_db *db, int b, hipStream_t s);
int reader_event(pir_db *db, int b, hipStream_t s, hipEvent_t *ev);
// Tuning table lookup: true and *p if an entry exists for (n, B class, stride).
bool tune_lookup(uint64_t n, uint32_t B, uint64_t stride, Plan *p);
}  // namespace talek
