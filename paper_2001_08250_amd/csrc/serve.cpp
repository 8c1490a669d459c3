// Serving loop with continuous batching over device lanes (see
// pir_serve_run in talek_pir.h). One dispatcher thread: it admits arrived
// reads while memory slots are free, launches the queued reads as a batch on
// any free lane, retires finished lanes, applies arrived writes to the
// working copy as they come, and publishes them at every epoch boundary.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <thread>
#include <vector>

#include "db.h"

using namespace talek;

namespace {

using Clock = std::chrono::steady_clock;

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *d_req = nullptr;
    void *d_resp = nullptr;
    void *d_iv = nullptr;
    uint8_t *h_resp = nullptr;
    uint8_t *h_iv = nullptr;
    uint32_t *h_rows = nullptr;
    uint32_t *h_rows_dev = nullptr;
    std::vector<uint64_t> reads;
    uint64_t epoch = 0;
    bool busy = false;
};

struct Resources {
    std::vector<Lane> lanes;
    uint8_t *pool = nullptr;
    void *pool_dev = nullptr;
    hipEvent_t start = nullptr;

    ~Resources()
    {
        for (Lane &l : lanes) {
            if (l.stream)
                hipStreamSynchronize(l.stream);
            if (l.done)
                hipEventDestroy(l.done);
            hipFree(l.d_req);
            hipFree(l.d_resp);
            hipFree(l.d_iv);
            if (l.h_resp)
                hipHostFree(l.h_resp);
            if (l.h_iv)
                hipHostFree(l.h_iv);
            if (l.h_rows)
                hipHostFree(l.h_rows);
            if (l.stream)
                hipStreamDestroy(l.stream);
        }
        if (pool)
            hipHostFree(pool);
        if (start)
            hipEventDestroy(start);
    }
};

template <typename T>
int host_alloc(T **p, uint64_t bytes)
{
    void *v = nullptr;
    if (hipHostMalloc(&v, std::max<uint64_t>(bytes, 64), hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        return PIR_ENOMEM;
    }
    *p = static_cast<T *>(v);
    return PIR_OK;
}

int dev_alloc(void **p, uint64_t bytes)
{
    if (hipMalloc(p, std::max<uint64_t>(bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return PIR_ENOMEM;
    }
    return PIR_OK;
}

double nearest_rank(std::vector<double> &v, double q)
{
    if (v.empty())
        return 0.0;
    size_t k = (size_t)std::ceil(q * v.size());
    k = std::min(std::max<size_t>(k, 1), v.size()) - 1;
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

}  // namespace

extern "C" int pir_serve_run(pir_db *db, pir_cuckoo *table, const pir_serve_config *cfg,
                             const pir_serve_trace *tr, pir_serve_result *res)
{
    if (!db || !cfg || !tr || !res)
        return PIR_EINVAL;
    if (cfg->max_batch == 0 || cfg->lanes == 0 || cfg->lanes > 8 || !(cfg->epoch_s > 0))
        return PIR_EINVAL;
    if (tr->n_reads && (!tr->read_t || !tr->read_row || !tr->req_pool || tr->pool_rows == 0))
        return PIR_EINVAL;
    if (tr->n_writes && (!table || !tr->write_t || !tr->write_id || !tr->write_beta1 || !tr->write_beta2 ||
                         !tr->write_payload || (cfg->interest_k && !tr->write_interest)))
        return PIR_EINVAL;
    if (res->n_probe && (!res->probe || !res->probe_resp))
        return PIR_EINVAL;
    for (uint64_t i = 0; i < tr->n_reads; ++i)
        if (tr->read_row[i] >= tr->pool_rows)
            return PIR_ERANGE;
    if (hipSetDevice(db->device) != hipSuccess)
        return PIR_EDEVICE;

    const uint64_t qb = db->qbytes, qp = db->qpitch, bb = db->bucket_bytes;
    const uint64_t iv_bytes = (db->m_bits + 7) / 8;
    const uint32_t MB = cfg->max_batch;
    // a budget below one read's device bytes could never admit a read
    if (cfg->mem_budget && cfg->mem_budget < qp + db->stride)
        return PIR_EBUSY;
    uint64_t slots = (uint64_t)cfg->lanes * MB;
    if (cfg->mem_budget)
        slots = cfg->mem_budget / (qp + db->stride);

    Resources R;
    int rc = host_alloc(&R.pool, tr->pool_rows * qp);
    if (rc != PIR_OK)
        return rc;
    for (uint64_t r = 0; r < tr->pool_rows; ++r) {
        memcpy(R.pool + r * qp, tr->req_pool + r * qb, qb);
        memset(R.pool + r * qp + qb, 0, qp - qb);
    }
    if (hipHostGetDevicePointer(&R.pool_dev, R.pool, 0) != hipSuccess)
        return PIR_EDEVICE;
    R.lanes.resize(cfg->lanes);
    for (Lane &l : R.lanes) {
        if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&l.done) != hipSuccess)
            return PIR_EDEVICE;
        if ((rc = dev_alloc(&l.d_req, MB * qp)) != PIR_OK || (rc = dev_alloc(&l.d_resp, MB * db->stride)) != PIR_OK ||
            (rc = dev_alloc(&l.d_iv, iv_bytes)) != PIR_OK || (rc = host_alloc(&l.h_resp, MB * bb)) != PIR_OK ||
            (rc = host_alloc(&l.h_iv, iv_bytes)) != PIR_OK || (rc = host_alloc(&l.h_rows, MB * 4ull)) != PIR_OK)
            return rc;
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, l.h_rows, 0) != hipSuccess)
            return PIR_EDEVICE;
        l.h_rows_dev = static_cast<uint32_t *>(dp);
        l.reads.reserve(MB);
    }
    if (hipEventCreate(&R.start) != hipSuccess)
        return PIR_EDEVICE;

    std::vector<double> lat(tr->n_reads, -1.0);
    if (res->write_epoch)
        for (uint64_t w = 0; w < tr->n_writes; ++w)
            res->write_epoch[w] = UINT64_MAX;
    std::deque<uint64_t> queue;
    uint64_t next_read = 0, next_write = 0, inflight = 0, completed = 0;
    uint64_t batches = 0, epochs = 0, w_ok = 0, w_fail = 0, max_queue = 0, batched_reads = 0;
    double next_epoch = cfg->epoch_s;
    std::vector<uint8_t> empty_payload;

    // t = 0: host clock and device clock are aligned with one synced event
    if (hipEventRecord(R.start, R.lanes[0].stream) != hipSuccess || hipEventSynchronize(R.start) != hipSuccess)
        return PIR_EDEVICE;
    const Clock::time_point t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };

    auto retire = [&](Lane &l) -> int {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, R.start, l.done) != hipSuccess)
            return PIR_EDEVICE;
        const double t_done = ms / 1000.0;
        for (size_t i = 0; i < l.reads.size(); ++i) {
            const uint64_t rd = l.reads[i];
            lat[rd] = t_done - tr->read_t[rd];
            if (res->read_epoch)
                res->read_epoch[rd] = l.epoch;
            if (res->n_probe) {
                const uint64_t *it = std::lower_bound(res->probe, res->probe + res->n_probe, rd);
                if (it != res->probe + res->n_probe && *it == rd) {
                    const uint64_t k = (uint64_t)(it - res->probe);
                    memcpy(res->probe_resp + k * bb, l.h_resp + i * bb, bb);
                    if (res->probe_iv)
                        memcpy(res->probe_iv + k * iv_bytes, l.h_iv, iv_bytes);
                }
            }
        }
        completed += l.reads.size();
        inflight -= l.reads.size();
        l.reads.clear();
        l.busy = false;
        return PIR_OK;
    };

    while (completed < tr->n_reads) {
        bool progress = false;
        // 1. retire finished lanes
        for (Lane &l : R.lanes) {
            if (!l.busy)
                continue;
            hipError_t q = hipEventQuery(l.done);
            if (q == hipSuccess) {
                if ((rc = retire(l)) != PIR_OK)
                    return rc;
                progress = true;
            } else if (q != hipErrorNotReady) {
                return PIR_EDEVICE;
            }
        }
        double now = now_s();
        // 2. apply the arrived writes to the working copy and stage their
        //    buckets as they come (a few per pass, so reads keep flowing);
        //    the next epoch boundary publishes them
        {
            bool wrote = false;
            while (next_write < tr->n_writes && tr->write_t[next_write] <= now) {
                const uint64_t w = next_write++;
                if (res->write_epoch)
                    res->write_epoch[w] = db->epoch + 1;
                uint64_t dropped = 0;
                const int r = pir_cuckoo_insert(table, tr->write_id[w], tr->write_beta1[w], tr->write_beta2[w],
                                                tr->write_payload + w * db->z, &dropped);
                if (r == PIR_OK)
                    w_ok++;
                else if (r == PIR_EFULL)
                    w_fail++;
                else
                    return r;
                if (cfg->interest_k &&
                    (rc = pir_interest_add(db, tr->write_interest + w * cfg->interest_k, cfg->interest_k)) != PIR_OK)
                    return rc;
                wrote = true;
            }
            if (wrote && table && (rc = pir_cuckoo_stage(table, nullptr)) != PIR_OK)
                return rc;
            if (wrote)
                progress = true;
        }
        // 3. epoch boundary: publish
        if (now >= next_epoch) {
            if ((rc = pir_epoch_commit(db, nullptr)) != PIR_OK)
                return rc;
            epochs++;
            next_epoch += cfg->epoch_s;
            progress = true;
            now = now_s();
        }
        // 4. admit arrived reads while memory slots are free
        while (next_read < tr->n_reads && tr->read_t[next_read] <= now && inflight < slots) {
            queue.push_back(next_read++);
            inflight++;
            progress = true;
        }
        max_queue = std::max<uint64_t>(max_queue, queue.size());
        // 5. launch the queue on a free lane
        if (!queue.empty()) {
            for (Lane &l : R.lanes) {
                if (l.busy || queue.empty())
                    continue;
                const uint32_t B = (uint32_t)std::min<uint64_t>(MB, queue.size());
                for (uint32_t i = 0; i < B; ++i) {
                    const uint64_t rd = queue.front();
                    queue.pop_front();
                    l.reads.push_back(rd);
                    l.h_rows[i] = tr->read_row[rd];
                }
                l.epoch = db->epoch;
                if (launch_gather_rows(l.d_req, qp, R.pool_dev, qp, l.h_rows_dev, B, qb, l.stream) != hipSuccess)
                    return PIR_EDEVICE;
                if ((rc = pir_read_batch_async(db, l.d_req, qp, B, l.d_resp, db->stride, l.stream)) != PIR_OK)
                    return rc;
                if (hipMemcpy2DAsync(l.h_resp, bb, l.d_resp, db->stride, bb, B, hipMemcpyDeviceToHost, l.stream) !=
                    hipSuccess)
                    return PIR_EDEVICE;
                if ((rc = pir_interest_vector_async(db, l.d_iv, iv_bytes, l.stream)) != PIR_OK)
                    return rc;
                if (hipMemcpyAsync(l.h_iv, l.d_iv, iv_bytes, hipMemcpyDeviceToHost, l.stream) != hipSuccess ||
                    hipEventRecord(l.done, l.stream) != hipSuccess)
                    return PIR_EDEVICE;
                l.busy = true;
                batches++;
                batched_reads += B;
                progress = true;
            }
        }
        if (!progress) {
            // idle: nap until the next arrival or epoch, polling lanes often
            double wake = next_epoch;
            if (next_read < tr->n_reads)
                wake = std::min(wake, tr->read_t[next_read]);
            const double nap = std::min(wake - now_s(), 20e-6);
            if (nap > 2e-6)
                std::this_thread::sleep_for(std::chrono::duration<double>(nap));
        }
    }
    const double wall = now_s();
    for (Lane &l : R.lanes)
        if (hipStreamSynchronize(l.stream) != hipSuccess)
            return PIR_EDEVICE;

    if (res->latency_s)
        memcpy(res->latency_s, lat.data(), lat.size() * sizeof(double));
    std::vector<double> sorted(lat);
    res->completed = completed;
    res->batches = batches;
    res->epochs = epochs;
    res->writes_applied = w_ok;
    res->writes_failed = w_fail;
    res->max_queue = max_queue;
    res->wall_s = wall;
    res->reads_per_s = wall > 0 ? completed / wall : 0;
    res->mean_batch = batches ? (double)batched_reads / batches : 0;
    res->p50_s = nearest_rank(sorted, 0.50);
    res->p99_s = nearest_rank(sorted, 0.99);
    res->max_s = sorted.empty() ? 0 : *std::max_element(sorted.begin(), sorted.end());
    return PIR_OK;
}
