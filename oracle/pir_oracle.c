/*
 * Oracle: plain CPU definition of the XOR-PIR server answer.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do. It shares no code, header or table with the HIP library.
 *
 * What it computes (Talek, section "Background: PIR", server step of the
 * l = 3 example; Appendix "Security Proofs", Building Blocks, answer functions
 * A_i of the Chor et al. PIR definition):
 *
 *     resp[r] = XOR over all buckets j in [0, n) with bit_j(req[r]) = 1 of D[j]
 *
 * where D[j] is the j-th bucket (bucket_bytes bytes, row-major, contiguous) and
 * bit_j(v) = (v[j >> 3] >> (j & 7)) & 1 (least-significant bit first inside a
 * request byte). Bits of the last request byte beyond n are ignored. The
 * answer is exact: XOR has no rounding and is order independent.
 *
 * This is the definition written out as a triple loop (request, bucket, byte)
 * with no blocking, fusion or reordering. The optional thread fan-out only
 * splits the request rows between threads; each row is still the same loop.
 */
#include <stdint.h>
#include <string.h>
#include <pthread.h>
#include <stdlib.h>

static int request_bit(const uint8_t *row, uint64_t j)
{
    return (row[j >> 3] >> (j & 7)) & 1;
}

static void answer_one_request(const uint8_t *D, uint64_t n, uint64_t bucket_bytes,
                               const uint8_t *req_row, uint8_t *resp_row)
{
    memset(resp_row, 0, bucket_bytes);
    for (uint64_t j = 0; j < n; ++j) {
        if (!request_bit(req_row, j))
            continue;
        const uint8_t *bucket = D + j * bucket_bytes;
        for (uint64_t k = 0; k < bucket_bytes; ++k)
            resp_row[k] ^= bucket[k];
    }
}

typedef struct {
    const uint8_t *D;
    uint64_t n, bucket_bytes, req_stride;
    const uint8_t *req;
    uint8_t *resp;
    uint32_t row_begin, row_end;
} rows_job;

static void *rows_worker(void *arg)
{
    rows_job *job = (rows_job *)arg;
    for (uint32_t r = job->row_begin; r < job->row_end; ++r)
        answer_one_request(job->D, job->n, job->bucket_bytes,
                           job->req + (uint64_t)r * job->req_stride,
                           job->resp + (uint64_t)r * job->bucket_bytes);
    return NULL;
}

/*
 * D       : n * bucket_bytes bytes.
 * req     : B rows of req_stride bytes (req_stride >= ceil(n / 8)).
 * resp    : B * bucket_bytes bytes, written.
 * nthreads: 0 or 1 = single-threaded; otherwise rows are split over threads.
 * Returns 0, or -1 on a NULL pointer with B > 0 or a too-short req_stride.
 */
int oracle_pir_read(const uint8_t *D, uint64_t n, uint64_t bucket_bytes,
                    const uint8_t *req, uint64_t req_stride, uint32_t B,
                    uint8_t *resp, uint32_t nthreads)
{
    if (B == 0)
        return 0;
    if (!D || !req || !resp || req_stride < (n + 7) / 8)
        return -1;
    if (nthreads <= 1 || B == 1) {
        rows_job job = {D, n, bucket_bytes, req_stride, req, resp, 0, B};
        rows_worker(&job);
        return 0;
    }
    if (nthreads > B)
        nthreads = B;
    pthread_t *tid = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    rows_job *jobs = (rows_job *)calloc(nthreads, sizeof(rows_job));
    if (!tid || !jobs) {
        free(tid);
        free(jobs);
        return -1;
    }
    uint32_t per = B / nthreads, extra = B % nthreads, start = 0;
    for (uint32_t t = 0; t < nthreads; ++t) {
        uint32_t cnt = per + (t < extra ? 1u : 0u);
        jobs[t] = (rows_job){D, n, bucket_bytes, req_stride, req, resp, start, start + cnt};
        start += cnt;
        pthread_create(&tid[t], NULL, rows_worker, &jobs[t]);
    }
    for (uint32_t t = 0; t < nthreads; ++t)
        pthread_join(tid[t], NULL);
    free(tid);
    free(jobs);
    return 0;
}
