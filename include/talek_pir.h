/*
 * talek_pir.h -- C ABI of the MI355X XOR-PIR server engine.
 *
 * One handle (pir_db) is one Talek server's PIR database: a blocked cuckoo
 * table of n buckets, each bucket d slots of msg_bytes bytes (section "Server
 * Design": buckets of equal size, each hash bucket is one PIR block). The
 * engine answers batches of IT-PIR request vectors: for request row r,
 *
 *     resp[r] = XOR of every bucket j (0 <= j < n) whose request bit is 1,
 *
 * bit j of a row being bit (j & 7) of byte (j >> 3), least-significant first.
 * This is the server step of the IT-PIR protocol (section "Background: PIR")
 * and ProcessRead of the server interface (section "Problem Definition",
 * Model). Bits past n in a row's last byte are ignored. Results are exact.
 *
 * Conventions for every call:
 *   - Return value: PIR_OK (0) or a negative pir_status. No exception crosses
 *     the ABI. On a validation error no output is touched.
 *   - Host buffers belong to the caller; the library copies what it needs and
 *     keeps no caller pointer after a call returns.
 *   - Device buffers passed to *_async calls are read/written stream-ordered on
 *     the given HIP stream; the caller keeps them alive until the stream has
 *     passed the call.
 *   - Calls on one handle are serialised internally (a mutex per handle).
 *   - Epochs: writes are staged and become visible to reads issued after the
 *     next pir_epoch_commit (the paper's periodic snapshot of the working copy
 *     into the GPU, section "Evaluation", cost of operations). Reads always
 *     answer from the last published snapshot.
 *   - Device: a handle lives on the HIP device that was current at create.
 *   - Any HIP runtime failure returns PIR_EDEVICE.
 */
#ifndef TALEK_PIR_H
#define TALEK_PIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pir_db pir_db;
typedef struct pir_cuckoo pir_cuckoo;

enum pir_status {
    PIR_OK = 0,
    PIR_EINVAL = -1,  /* bad argument: NULL pointer, zero size, overflow, bad pitch */
    PIR_ERANGE = -2,  /* bucket index >= n, or interest position >= m_bits */
    PIR_ENOMEM = -3,  /* device or pinned host allocation failed */
    PIR_EDEVICE = -4, /* a HIP runtime call failed */
    PIR_EFULL = -5,   /* cuckoo insertion gave up after max_kicks evictions */
    PIR_EBUSY = -6    /* admission refused: no memory slot free */
};

/* Text for a pir_status value (static storage; never NULL). */
const char *pir_strerror(int code);

/* Library version string, e.g. "talek-pir 0.1 gfx950". */
const char *pir_version(void);

/* ---------------------------------------------------------------- database */

/*
 * Create a database of n buckets x d slots x msg_bytes bytes on the current
 * HIP device. The published snapshot starts all-zero (empty slots hold zero
 * bytes). Fails with PIR_EINVAL when n, d or msg_bytes is 0 or n*d*msg_bytes
 * overflows, PIR_ENOMEM when device memory runs out. *out is set only on
 * success. (Section "Writing into a Cuckoo Hash Table": b buckets of d
 * messages of size z.)
 */
int pir_db_create(uint64_t n, uint32_t d, uint32_t msg_bytes, pir_db **out);

/* Free every device and host resource of the handle. NULL is a no-op. Waits
 * for the handle's outstanding work first. */
void pir_db_destroy(pir_db *db);

/* Geometry: n, d, msg_bytes and the bucket size d * msg_bytes. Any output
 * pointer may be NULL. */
int pir_db_shape(const pir_db *db, uint64_t *n, uint32_t *d, uint32_t *msg_bytes,
                 uint64_t *bucket_bytes);

/*
 * Stage the d * msg_bytes bytes of one bucket (ProcessWrite's effect on the
 * table, applied to the next snapshot). A later write to the same bucket in
 * the same epoch wins. PIR_ERANGE if bucket >= n; PIR_EINVAL on NULL data.
 */
int pir_db_write_bucket(pir_db *db, uint64_t bucket, const uint8_t *data);

/* Stage count consecutive buckets starting at first: count * d * msg_bytes
 * bytes, row-major. PIR_ERANGE if first + count > n. */
int pir_db_write_range(pir_db *db, uint64_t first, uint64_t count, const uint8_t *data);

/*
 * Publish every staged bucket write and the open epoch's interest bits: reads
 * issued after this call (on any stream) answer from the new snapshot, reads
 * issued before it finish on the old one. Double-buffered on the device: the
 * staged buckets are written into the back copy, the copies swap, and the
 * same buckets are then replayed into the new back copy once the reads that
 * still use it have finished. Returns the new epoch number in *epoch_out
 * (may be NULL).
 */
int pir_epoch_commit(pir_db *db, uint64_t *epoch_out);

/* Number of epochs published so far. */
uint64_t pir_epoch(const pir_db *db);

/* ------------------------------------------------------------------- reads */

/*
 * Answer B request vectors (ProcessRead, section "Problem Definition";
 * server step 5 of section "Background: PIR").
 *   req_bits: B rows of ceil(n / 8) bytes, row-major, host memory.
 *   resp:     B rows of d * msg_bytes bytes, row-major, host memory, written.
 * Blocks until the answers are in resp. B = 0 is a no-op returning PIR_OK.
 * NULL req_bits or resp with B > 0 -> PIR_EINVAL.
 */
int pir_read_batch(pir_db *db, const uint8_t *req_bits, uint32_t B, uint8_t *resp);

/*
 * Same answer, device memory, asynchronous on a HIP stream (hipStream_t,
 * NULL = the default stream).
 *   d_req:  B rows, row r at d_req + r * req_pitch; req_pitch >= ceil(n / 8).
 *   d_resp: B rows, row r at d_resp + r * resp_pitch; resp_pitch >= d * msg_bytes.
 * Any pitch and alignment is accepted; rows that are not 4-byte (requests) or
 * 16-byte (responses) aligned are restaged through library scratch on the same
 * stream. Returns once the work is enqueued.
 */
int pir_read_batch_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B,
                         void *d_resp, uint64_t resp_pitch, void *hip_stream);

/*
 * Allocation-free variant of pir_read_batch_async, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, the same answers,
 * and no allocation of any kind inside the call. Its device scratch (split
 * partial answers, Four-Russians request offsets, restaged rows) lies in one
 * static device array of PIR_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; the read takes the handle's schedule with its bucket splits
 * reduced (or the masked kernel) until that scratch fits. Preprocessed
 * (Strassen) leaves are not used.
 *   PIR_ERANGE: restaging the rows alone needs more than the array (only
 *     reachable with unaligned rows: B * round_up(ceil(n/8), 16) plus
 *     B * round_up(d * msg_bytes, 16) above PIR_NOALLOC_SCRATCH_BYTES).
 *   PIR_EINVAL: as pir_read_batch_async.
 * Every call on one GPU shares that GPU's array and the handle's reader
 * event of the snapshot copy: calls whose device work overlaps (on any
 * handles or streams of the same GPU) race and give undefined answers; order
 * them on one stream or wait between them.
 */
#define PIR_NOALLOC_SCRATCH_BYTES (32ull << 20)
int pir_read_batch_noalloc_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B,
                                 void *d_resp, uint64_t resp_pitch, void *hip_stream);

/*
 * Uneven batch stream: n_batches batches, batch k holding sizes[k] request
 * rows. Batch k reads request rows req_first[k] .. req_first[k] + sizes[k] - 1
 * of d_req and writes response rows resp_first[k] .. of d_resp (row indices,
 * host arrays; a NULL array means the batches' rows are concatenated in
 * order). Every batch is answered exactly as pir_read_batch_async would
 * answer it. The stream's rows, in order, are cut into launch groups of 1024
 * requests (a batch may straddle two groups; the last group takes the rest:
 * an answer depends only on its own request row and the snapshot), each
 * answered by one read launch with that group's schedule;
 * rows that are not contiguous are gathered into / scattered from library
 * scratch on the stream. The launch sequence is captured in a HIP graph and
 * replayed when the same stream shape, buffers, schedules and snapshot
 * repeat. Requires 4-byte aligned request rows with req_pitch % 4 == 0 and
 * ceil(n/8) % 4 == 0, and 16-byte aligned response rows with
 * resp_pitch % 16 == 0 and d * msg_bytes % 16 == 0 (PIR_EINVAL otherwise).
 * (Section "Evaluation": read requests are batched and forwarded to the GPU;
 * the leader may reorder reads.)
 */
int pir_read_stream_async(pir_db *db, const void *d_req, uint64_t req_pitch,
                          const uint32_t *sizes, const uint64_t *req_first, uint32_t n_batches,
                          void *d_resp, uint64_t resp_pitch, const uint64_t *resp_first,
                          void *hip_stream);

/* ---------------------------------------------------------- serialized PIR */

/*
 * Serialized PIR (section "Serialized PIR", steps 6 and 7): the server answers
 * each request with its IT-PIR answer XORed with a one-time mask of the
 * answer's size, P = PRNG(p), p being the request's seed. The paper leaves
 * the PRNG open; here it is ChaCha20 (D. J. Bernstein, in the form of
 * RFC 8439): the 32-byte seed is the key, the 96-bit nonce is zero, the
 * 32-bit block counter starts at 0, and P is the first d * msg_bytes bytes
 * of the keystream:
 *
 *     resp[r] = (XOR of the buckets selected by req[r]) XOR P(seeds[r]).
 *
 *   seeds: B seeds of 32 bytes, row-major (host memory for the synchronous
 *          call; device memory, 4-byte aligned, for the async one).
 * Every other argument, the validation and the stream rules are those of
 * pir_read_batch / pir_read_batch_async; NULL seeds with B > 0 -> PIR_EINVAL.
 * A seed must not be used for two answers (the mask is a one-time pad).
 */
int pir_read_batch_masked(pir_db *db, const uint8_t *req_bits, uint32_t B, const uint8_t *seeds, uint8_t *resp);
int pir_read_batch_masked_async(pir_db *db, const void *d_req, uint64_t req_pitch, uint32_t B,
                                const void *d_seeds, void *d_resp, uint64_t resp_pitch, void *hip_stream);

/*
 * The leader's combination (section "Serialized PIR", step 8): row r of
 * d_out = XOR over i < l of row r of d_in[i], row_bytes bytes per row, on the
 * given stream. d_in is a host array of l device pointers (1 <= l <= 16);
 * rows start at d_in[i] + r * in_pitch and d_out + r * out_pitch. Requires
 * row_bytes, both pitches and every pointer to be multiples of 16 and pitches
 * >= row_bytes (PIR_EINVAL otherwise). B = 0 is a no-op. No handle: the work
 * runs on the current HIP device.
 */
int pir_xor_combine_async(void *d_out, uint64_t out_pitch, const void *const *d_in, uint32_t l,
                          uint64_t in_pitch, uint32_t B, uint64_t row_bytes, void *hip_stream);

/* --------------------------------------------------------- kernel schedule */

/* Kernel families of the read path. */
enum pir_kernel_kind {
    PIR_KERNEL_AUTO = 0,   /* tuning table, else the built-in heuristic */
    PIR_KERNEL_MASK = 1,   /* branch-free masked XOR (one 3-input op per word) */
    PIR_KERNEL_SKIP = 2,   /* wave-uniform zero-skip of unselected buckets */
    PIR_KERNEL_M4R = 3,    /* Four-Russians: 8-bucket tables in LDS, 4 bytes per lane */
    PIR_KERNEL_M4R_WIDE = 4 /* Four-Russians: 6-bucket tables, or paired 5/4/3-bucket tables (PAIRS
                               flags), in LDS, 16 bytes per lane */
};

/* Plan flags. SHARED_COLUMN (MASK and SKIP families): the four waves of a
 * workgroup stream the same 1 KiB column chunk of D and take four
 * consecutive request tiles, so the chunk is read from L2 once per
 * workgroup instead of once per wave. Bits 8..11 (M4R_WIDE): how many
 * bucket groups ahead D is loaded (0 = 2). ROLLING (M4R_WIDE): table
 * lookups keep a fixed number of LDS reads in flight and the next group's
 * request offsets are fetched during the current one. PAIRS (M4R_WIDE): two
 * 5-bucket tables of 32 entries per step instead of one 6-bucket table,
 * each request folding both lookups in with one 3-input XOR per dword
 * (rolling lookups always). PAIR_G4 / PAIR_G3 (with PAIRS): paired tables of
 * 4 or 3 buckets (16 or 8 entries, 64 or 32 KiB of LDS double-buffered, two
 * workgroups per CU) for batches of tens of requests. HALF_WAVES (with
 * PAIRS, 5-bucket tables or PAIR_G6's 6-bucket ones): 512-byte table
 * entries, each 32-lane half of a wave serving its own request, so a
 * workgroup answers twice the requests from one set of tables (tile =
 * requests per wave, 64 or 32). */
enum {
    PIR_PLAN_SHARED_COLUMN = 1,
    PIR_PLAN_ROLLING = 1 << 12,
    PIR_PLAN_PAIRS = 1 << 13,
    PIR_PLAN_PAIR_G4 = 1 << 14,
    PIR_PLAN_PAIR_G3 = 2 << 14,
    PIR_PLAN_HALF_WAVES = 1 << 16,
    PIR_PLAN_PAIR_G6 = 1 << 17
};

/* A read schedule: kernel family, request tile (requests per wave), bucket
 * splits (0 = heuristic), unroll (MASK/SKIP: buckets loaded ahead; M4R:
 * waves per workgroup; 0 = default), flags. */
typedef struct pir_plan {
    int32_t kind;
    uint32_t tile;
    uint32_t splits;
    uint32_t unroll;
    uint32_t flags;
} pir_plan;

/* Force a schedule for subsequent reads of this handle (kind AUTO restores
 * the automatic choice: MASK up to 16 requests, paired 4-bucket tables up to
 * 128, paired 5-bucket tables up to 256, half-wave paired 6-bucket tables
 * above over rows of 512 bytes or more, unless the tuning table has an
 * entry).
 * PIR_EINVAL for an unsupported combination. */
int pir_set_plan(pir_db *db, const pir_plan *plan);

/* The schedule the next read of B rows would use. */
int pir_get_plan(pir_db *db, uint32_t B, pir_plan *plan);

/*
 * Autotune: time every candidate schedule for batches of B rows on the
 * handle's current snapshot (iters timed launches each, after one warm-up)
 * and record the fastest in the tuning table under (n, B class, bucket
 * bytes). best (may be NULL) receives the winner, best_us its mean time.
 */
int pir_tune(pir_db *db, uint32_t B, uint32_t iters, pir_plan *best, double *best_us);

/* Save / load the tuning table as JSON. Loading merges into the table. */
int pir_tune_save(const char *path);
int pir_tune_load(const char *path);

/*
 * Kernel timing. While enabled (on != 0), every on-th read of this handle
 * issued by pir_read_batch or pir_read_batch_async (on = 1: every read;
 * counting from the enable, the first one included) takes the start and end
 * times of its main read kernel's dispatch (not the request staging or the
 * split reduction) as a HIP event pair on its stream, for the first
 * PIR_PROFILE_MAX recorded reads after the enable; later reads are not
 * recorded. Enabling (or disabling) clears earlier records. on < 0 ->
 * PIR_EINVAL.
 * pir_profile_collect waits for the recorded reads to finish, writes up to
 * cap durations in milliseconds (in issue order) into ms, the number of
 * recorded reads into *count (may be NULL), and clears the records.
 */
enum { PIR_PROFILE_MAX = 4096 };
int pir_profile_enable(pir_db *db, int on);
int pir_profile_collect(pir_db *db, float *ms, uint32_t cap, uint32_t *count);

/* ------------------------------------------------- private notifications */

/*
 * Configure the global interest vector (section "Private Notifications"):
 * m_bits Bloom-filter bits, union over the deltas of the last window_epochs
 * published epochs. Resets the vector. Defaults: 2^17 bits (16 KiB) and 100
 * epochs, the paper's vector size at 1M messages and its TTL of 100 write
 * intervals (section "Evaluation", cost of operations).
 * PIR_EINVAL for m_bits == 0, m_bits > 2^32 or window_epochs == 0.
 */
int pir_interest_config(pir_db *db, uint64_t m_bits, uint32_t window_epochs);

/*
 * OR one write's interest-vector bits into the open epoch's delta: k bit
 * positions, each < m_bits (PIR_ERANGE otherwise, nothing applied). They
 * become visible at the next pir_epoch_commit.
 */
int pir_interest_add(pir_db *db, const uint32_t *pos, uint32_t k);

/*
 * ProcessGetUpdates: copy the published global interest vector (the OR of
 * the window's deltas) into out, ceil(m_bits / 8) bytes, bit p at byte p >> 3,
 * bit p & 7. PIR_EINVAL if out_bytes is smaller.
 */
int pir_interest_vector(pir_db *db, uint8_t *out, uint64_t out_bytes);

/* Device-memory variant of pir_interest_vector, stream-ordered. */
int pir_interest_vector_async(pir_db *db, void *d_out, uint64_t out_bytes, void *hip_stream);

/*
 * Compressed interest vectors for GetUpdates (section "Private
 * Notifications": clients fetch compressed Bloom-filter deltas and keep a
 * window of them). The paper fixes no format; the stream is, little-endian:
 *   bytes 0-7 m, bytes 8-15 c (bits set), bytes 16-19 the Rice parameter
 *   k = floor(log2(max(1, floor(m / (c + 1))))), bytes 20-23 zero, then for
 *   the set positions p_0 < ... < p_{c-1} (p_{-1} = -1) the gaps
 *   g = p_i - p_{i-1} - 1, each as floor(g / 2^k) one-bits, one zero-bit and
 *   the k low bits of g least significant first, packed into bytes least
 *   significant bit first (Golomb-Rice coding).
 * pir_interest_vector_encoded encodes the published global vector;
 * pir_interest_delta_encoded the delta of published epoch `epoch` (the
 * interest bits added before that commit), which must still be in the
 * window: pir_epoch(db) - window < epoch <= pir_epoch(db), else PIR_ERANGE.
 * *out_bytes receives the stream length; out may be NULL to ask for it. If
 * out_cap is smaller than the stream, PIR_EINVAL (with *out_bytes set).
 * Synchronous, ordered after the handle's commits. PIR_EINVAL if the vector
 * has 2^31 or more bits set.
 */
int pir_interest_vector_encoded(pir_db *db, uint8_t *out, uint64_t out_cap, uint64_t *out_bytes);
int pir_interest_delta_encoded(pir_db *db, uint64_t epoch, uint8_t *out, uint64_t out_cap, uint64_t *out_bytes);

/* ------------------------------------------------- server cuckoo table */

/*
 * The server's DRAM working copy: a blocked cuckoo table bound to db (same
 * n, d, msg_bytes), applying Write requests as section "Writing into a Cuckoo
 * Hash Table" describes: delete the oldest message when `capacity` messages
 * are live (0 = never), store in beta1 or else beta2 if either has a free slot
 * (beta1 first, lowest free slot), otherwise walk evictions driven by one
 * SplitMix64 stream seeded with s_cuckoo (one draw & 1 picks beta_e at the
 * first both-full step; each eviction draws once, victim slot = draw % d),
 * giving up after max_kicks evictions. The item in hand at that point is
 * dropped and the call returns PIR_EFULL with its id in *dropped_id.
 * Every bucket the call changes is marked dirty; pir_cuckoo_stage copies the
 * dirty buckets into db's staged writes.
 */
int pir_cuckoo_create(pir_db *db, uint64_t capacity, uint64_t s_cuckoo, uint32_t max_kicks,
                      pir_cuckoo **out);
/* A table with no database bound (host only, no GPU needed): the same rules,
 * pir_cuckoo_stage returns PIR_EINVAL. For replicas that only keep the
 * working copy, and for checking the placement logic on its own. */
int pir_cuckoo_create_detached(uint64_t n, uint32_t d, uint32_t msg_bytes, uint64_t capacity,
                               uint64_t s_cuckoo, uint32_t max_kicks, pir_cuckoo **out);
void pir_cuckoo_destroy(pir_cuckoo *c);

/* One Write: ids are the caller's message ids; payload is msg_bytes bytes. */
int pir_cuckoo_insert(pir_cuckoo *c, uint64_t id, uint64_t beta1, uint64_t beta2,
                      const uint8_t *payload, uint64_t *dropped_id);

/* count Writes in order; status[i] / dropped[i] (either may be NULL) receive
 * each insert's result. Returns PIR_OK, or the first hard error (EINVAL /
 * ERANGE); EFULL results are reported per item only. */
int pir_cuckoo_insert_many(pir_cuckoo *c, uint64_t count, const uint64_t *ids,
                           const uint64_t *beta1, const uint64_t *beta2,
                           const uint8_t *payloads, int32_t *status, uint64_t *dropped);

/* Stage every dirty bucket into the bound database (visible after the next
 * pir_epoch_commit). *staged receives the number of buckets (may be NULL). */
int pir_cuckoo_stage(pir_cuckoo *c, uint64_t *staged);

/* Host working copy, for inspection: n * d * msg_bytes bytes; per-slot message
 * ids (0 = empty) and occupancy (n * d entries each; either may be NULL). */
int pir_cuckoo_table(const pir_cuckoo *c, uint8_t *out, uint64_t out_bytes);
int pir_cuckoo_slots(const pir_cuckoo *c, uint64_t *ids, uint8_t *occupied);
uint64_t pir_cuckoo_live(const pir_cuckoo *c);

/* ----------------------------------------------------------------- serving */

/*
 * Serving loop: an open-loop stream of timed reads and writes is served
 * against db (and its cuckoo working copy `table`) with continuous batching
 * (section "Evaluation": reads are batched and forwarded to the GPU, writes
 * go to the DRAM working copy and are snapshotted into the GPU periodically;
 * section "Private Notifications": each read comes back with the current
 * global interest vector).
 *   - A read arriving at time t is admitted once a memory slot is free (each
 *     in-flight read holds ceil(n/8) request bytes and one response bucket of
 *     device memory; mem_budget bounds the total). Admitted reads queue.
 *     A mem_budget below one read's bytes (the request row at its pitch plus
 *     one response row) could never admit a read: the call returns PIR_EBUSY
 *     before serving anything.
 *   - Whenever one of `lanes` device lanes (each its own HIP stream and
 *     buffers) is free, up to max_batch queued reads leave as one batch: their
 *     request rows are gathered from pinned host memory by a kernel, answered
 *     by the tuned read kernel, and the responses plus the published global
 *     interest vector are copied back. Batches on different lanes overlap on
 *     the device; reads arriving meanwhile join the next batch.
 *   - Writes are applied to the cuckoo table (with their interest bits) and
 *     their buckets staged as they arrive, between batches; every epoch_s
 *     seconds the staged writes are published (pir_epoch_commit), so a write
 *     becomes readable at the first epoch boundary after its arrival. A read
 *     is answered from the snapshot published when its batch launched;
 *     read_epoch reports which.
 *   - max_batch = 1 gives the one-launch-per-read baseline.
 * Latency of a read = device completion of its batch (response and interest
 * vector in host memory) minus its arrival time.
 */
typedef struct pir_serve_config {
    uint32_t max_batch;      /* reads per launch, >= 1 */
    uint32_t lanes;          /* batches in flight, 1..8 */
    uint64_t mem_budget;     /* device bytes for in-flight reads; 0 = lanes * max_batch reads */
    double epoch_s;          /* write publication period, > 0 */
    uint32_t interest_k;     /* interest positions per write (0 = none) */
    uint32_t reserved;
} pir_serve_config;

typedef struct pir_serve_trace {
    uint64_t n_reads;
    const double *read_t;          /* arrival times in seconds, nondecreasing */
    const uint32_t *read_row;      /* pool row carried by each read */
    const uint8_t *req_pool;       /* pool_rows request rows of ceil(n/8) bytes */
    uint64_t pool_rows;
    uint64_t n_writes;
    const double *write_t;         /* arrival times, nondecreasing */
    const uint64_t *write_id;
    const uint64_t *write_beta1;
    const uint64_t *write_beta2;
    const uint8_t *write_payload;  /* n_writes x msg_bytes */
    const uint32_t *write_interest; /* n_writes x interest_k positions (< m_bits) */
} pir_serve_trace;

typedef struct pir_serve_result {
    /* per-read outputs (each may be NULL) */
    double *latency_s;             /* n_reads */
    uint64_t *read_epoch;          /* n_reads: epoch that answered the read */
    uint64_t n_probe;              /* reads whose response is returned */
    const uint64_t *probe;         /* their indices, increasing */
    uint8_t *probe_resp;           /* n_probe x (d * msg_bytes) */
    uint8_t *probe_iv;             /* n_probe x ceil(m_bits / 8), or NULL */
    uint64_t *write_epoch;         /* n_writes: epoch that published the write (UINT64_MAX: never) */
    /* summary, filled by the call */
    uint64_t completed, batches, epochs, writes_applied, writes_failed, max_queue;
    double wall_s, reads_per_s, p50_s, p99_s, max_s, mean_batch;
} pir_serve_result;

int pir_serve_run(pir_db *db, pir_cuckoo *table, const pir_serve_config *cfg,
                  const pir_serve_trace *trace, pir_serve_result *res);

/* ---- Preprocessed reads for large batches ----------------------------------
 *
 * A batch's answers are the GF(2) product of its request bits (B x n) with
 * the snapshot (n x d*msg_bytes); the server side of the method (section
 * "Talek Server", the XOR of the selected buckets) fixes this product, not
 * how it is computed. With preprocessing on, the library applies L levels
 * (1 or 2) of Strassen's block recursion, whose seven block products per
 * level need only XORs over GF(2): the database side of every one of the
 * 7^L leaf products (an XOR of up to 2^L blocks of the snapshot) is formed
 * once and kept up to date by every epoch commit (a commit recomputes the
 * leaf rows its changed buckets feed, or every leaf when they exceed a
 * quarter of the rows), and a read forms the request side of every leaf
 * (under the paired-table kernels: the table offsets of all leaves' request
 * rows in one launch), answers the 7^L leaf products with the usual kernels
 * (in one launch when the offsets were staged together) and XORs them into
 * the answers. The answers are exactly those of the plain definition; a
 * large read does 7^L / 8^L of the plain product's work, at the price of
 * 7^L / 4^L times the snapshot in device memory (1.75 at L = 1, 3.06 at
 * L = 2), the commits' leaf upkeep, and per-read scratch of about
 * 7^L * (n / 2^L / (2G) + 1) * ceil(B / 2^L) * 2 bytes of staged request
 * entries (G = 6 buckets per table for leaves above 256 requests, else 5,
 * 4 or 3) plus the leaves' split partials (4.4 GB and 3.2 GB for 2048
 * requests over 2^22 buckets of 4 KiB at L = 2).
 *
 *   levels:    0 (off, frees the leaves), 1 or 2.
 *   min_batch: reads of B >= min_batch rows take the preprocessed path
 *              (pir_read_batch*, masked or not); 0 selects 256 << levels,
 *              where each leaf product still has a full Four-Russians tile.
 *              The serving loop's batches go through pir_read_batch_async
 *              and take it when they are that large; the uneven-batch
 *              stream keeps the plain path.
 * Errors: PIR_EINVAL for levels > 2 or d * msg_bytes not a multiple of
 * 16 << levels; PIR_ENOMEM when the leaves do not fit. The leaves are built
 * from the published snapshot at once (stream-ordered; reads wait for them).
 */
int pir_preprocess(pir_db *db, uint32_t levels, uint32_t min_batch);

/*
 * The leaf tables of an L-level preprocessing (levels 1 or 2; no handle, no
 * device work), for inspection and tests. Leaf i < 7^L sums the a_cnt[i]
 * request blocks a[4 i .. 4 i + a_cnt[i] - 1] and the d_cnt[i] database
 * blocks d[4 i ..], each block written (row << 4) | col in the 2^L x 2^L
 * grid; answer block b (row * 2^L + col, b < 4^L) is the XOR of the o_cnt[b]
 * leaves o_leaf[16 b ..]. Caller arrays: a_cnt, d_cnt 49 bytes; a, d 196;
 * o_cnt 16; o_leaf 256. *leaves receives 7^L. PIR_EINVAL for other levels or
 * a NULL pointer.
 */
int pir_preprocess_tables(uint32_t levels, uint32_t *leaves, uint8_t *a_cnt, uint8_t *a, uint8_t *d_cnt, uint8_t *d,
                          uint8_t *o_cnt, uint8_t *o_leaf);

#ifdef __cplusplus
}
#endif

#endif /* TALEK_PIR_H */
