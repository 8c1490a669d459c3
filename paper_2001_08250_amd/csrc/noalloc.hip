// Allocation-free read: pir_read_batch_noalloc_async answers a batch exactly
// as pir_read_batch_async does, but every byte of device scratch it needs
// (split partial answers, the Four-Russians request offsets, restaged request
// and answer rows) lies in one static device array per GPU, so the call
// itself never allocates. Its host code takes the array's device address from
// hipGetSymbolAddress (per device, once, when a handle is created there): in
// host code the array's own name is only a host-side stand-in.
#include <hip/hip_runtime.h>

#include <mutex>

#include "db.h"

using namespace talek;

// The scratch of every allocation-free read on a GPU (each GPU holds its own copy).
static __device__ __align__(256) uint8_t scratch[PIR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES];  // device address of `scratch` on each GPU

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

#define HIP_TRY(x)                                                                                                 \
    do {                                                                                                           \
        if ((x) != hipSuccess)                                                                                     \
            return PIR_EDEVICE;                                                                                    \
    } while (0)
#define PIR_TRY(x)                                                                                                 \
    do {                                                                                                           \
        const int r_ = (x);                                                                                        \
        if (r_ != PIR_OK)                                                                                          \
            return r_;                                                                                             \
    } while (0)

// The handle's schedule for B rows, with its bucket splits halved (and, if
// the Four-Russians offsets alone do not fit, the masked tile kernel taken
// instead) until the read's scratch fits in `cap` bytes. Returns false when
// even one split of the masked kernel needs more.
bool fit_plan(pir_db *db, const ReadGeom &g, uint64_t cap, Plan *out)
{
    Plan p = choose_plan(db, g.B);
    for (int pass = 0; pass < 2; ++pass) {
        while (partial_bytes(g, p) > cap && p.splits > 1) {
            Plan w = p;
            w.splits = p.splits / 2;
            p = resolve_plan(g, w, db->num_cus);
        }
        if (partial_bytes(g, p) <= cap) {
            *out = p;
            return true;
        }
        p = resolve_plan(g, Plan{KIND_MASK, 0, 0, 0, 0}, db->num_cus);
    }
    return false;
}

}  // namespace

namespace talek {

int noalloc_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return PIR_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device])
        return PIR_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return PIR_EDEVICE;
    }
    g_scratch[device] = p;
    return PIR_OK;
}

}  // namespace talek

int pir_read_batch_noalloc_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B, void *d_resp,
                                 uint64_t resp_pitch, void *hip_stream)
{
    if (!db)
        return PIR_EINVAL;
    if (B == 0)
        return PIR_OK;
    if (!d_req || !d_resp || req_pitch < db->qbytes || resp_pitch < db->bucket_bytes)
        return PIR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (db->device >= 0 && db->device < MAX_DEVICES)
            base = g_scratch[db->device];
    }
    if (!base)
        return PIR_EDEVICE;
    // rows the kernels cannot take in place are restaged inside the array
    const bool restage_q = (reinterpret_cast<uintptr_t>(d_req) & 3) || (req_pitch & 3) || (db->qbytes & 3);
    const bool direct = !(reinterpret_cast<uintptr_t>(d_resp) & 15) && !(resp_pitch & 15) &&
                        db->stride == db->bucket_bytes;
    const uint64_t q_bytes = restage_q ? align256((uint64_t)B * db->qpitch) : 0;
    const uint64_t r_bytes = direct ? 0 : align256((uint64_t)B * db->stride);
    if (q_bytes + r_bytes > PIR_NOALLOC_SCRATCH_BYTES)
        return PIR_ERANGE;
    uint8_t *q_area = static_cast<uint8_t *>(base);
    uint8_t *r_area = q_area + q_bytes;
    uint8_t *part = r_area + r_bytes;
    const void *q = restage_q ? q_area : d_req;
    const uint64_t qp = restage_q ? db->qpitch : req_pitch;
    void *out = direct ? d_resp : r_area;
    const uint64_t op = direct ? resp_pitch : db->stride;
    ReadGeom g = read_geom(db, q, qp, B, out, op);
    Plan p;
    if (!fit_plan(db, g, PIR_NOALLOC_SCRATCH_BYTES - q_bytes - r_bytes, &p))
        return PIR_ERANGE;
    // the reader event of the published copy, created with the handle
    auto it = db->readers[db->front].find(noalloc_reader_key(db));
    if (it == db->readers[db->front].end())
        return PIR_EDEVICE;
    hipEvent_t done = it->second;
    HIP_TRY(hipSetDevice(db->device));
    PIR_TRY(wait_published(db, s));
    if (restage_q)
        HIP_TRY(hipMemcpy2DAsync(q_area, db->qpitch, d_req, req_pitch, db->qbytes, B, hipMemcpyDeviceToDevice, s));
    if (direct)
        g.done = done;
    HIP_TRY(launch_read(g, p, part, s));
    if (direct)
        return PIR_OK;
    HIP_TRY(hipMemcpy2DAsync(d_resp, resp_pitch, r_area, db->stride, db->bucket_bytes, B, hipMemcpyDeviceToDevice, s));
    return hipEventRecord(done, s) == hipSuccess ? PIR_OK : PIR_EDEVICE;
}
