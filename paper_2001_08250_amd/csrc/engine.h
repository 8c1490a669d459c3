// Internal interface between the host library and the device kernels.
// Nothing here is part of the C ABI (include/talek_pir.h).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace talek {

// Kernel families (values match enum pir_kernel_kind).
enum Kind : int { KIND_AUTO = 0, KIND_MASK = 1, KIND_SKIP = 2, KIND_M4R = 3, KIND_M4RW = 4 };

// Rows allocated for a database of n buckets: n rounded up to 32 plus 64
// more, all zero beyond n. Kernels may read (never use) any row below this,
// which lets them stream whole 32-bucket request words and prefetch past the
// end of their range without per-row clamping.
inline uint64_t padded_db_rows(uint64_t n) { return ((n + 31) & ~31ull) + 64; }

// Geometry of one read launch. D rows are `stride` bytes apart (stride is
// bucket_bytes rounded up to 16; padding bytes are zero) and
// padded_db_rows(n) rows are readable. Request rows are
// `qpitch` bytes apart, qpitch % 4 == 0, each row readable up to
// round_up(ceil(n/8), 4) bytes. Output rows are `out_pitch` bytes apart,
// out_pitch % 16 == 0, and receive `stride` bytes each.
struct ReadGeom {
    const void *D;
    uint64_t n;
    uint64_t stride;
    const void *Q;
    uint64_t qpitch;
    uint32_t B;
    void *out;
    uint64_t out_pitch;
    // serialized PIR: B x 8 key words (32-byte seeds) of the answers'
    // one-time masks, or none
    const uint32_t *keys = nullptr;
    // Event that the read's last kernel records when it completes (through
    // the dispatch itself, so no separate marker sits in the stream), or none.
    hipEvent_t done = nullptr;
    // Pair-table reads only: offsets already staged in the layout the read's
    // own staging kernel writes (launch_stage_leaf_pairs), or none.
    const uint32_t *staged = nullptr;
    // Pair-table reads of staged offsets only: `leaves` products of this
    // shape in one launch, leaf l's database at D + l * leaf_d_bytes and
    // offsets at staged + l * leaf_stage_bytes, its answers rows l * B ..
    // l * B + B - 1 of out (pitch out_pitch).
    uint32_t leaves = 1;
    uint64_t leaf_d_bytes = 0, leaf_stage_bytes = 0;
};

struct Plan {
    int kind;
    uint32_t tile;     // requests per wave
    uint32_t splits;   // bucket-range splits (1 = none)
    uint32_t unroll;   // buckets loaded ahead (M4R: waves per workgroup)
    uint32_t flags;    // PLAN_SHARED_COLUMN
};
constexpr uint32_t PLAN_SHARED_COLUMN = 1;
constexpr uint32_t PLAN_ROLLING = 1u << 12;
// paired tables of 5 - ((flags >> PLAN_PAIR_G_SHIFT) & 3) buckets each (5, 4 or 3)
constexpr uint32_t PLAN_PAIR_G_SHIFT = 14;
constexpr uint32_t PLAN_PAIRS = 1u << 13;
// with PLAN_PAIRS: 512-byte table entries, one request per 32-lane half wave
// (xorpir_m4rh_kernel); with PLAN_PAIR_G6 too, 6-bucket tables
constexpr uint32_t PLAN_HALF_WAVES = 1u << 16;
constexpr uint32_t PLAN_PAIR_G6 = 1u << 17;

// Device scratch the read needs for split partials: bytes.
uint64_t partial_bytes(const ReadGeom &g, const Plan &p);

// Fill in a complete plan (tile, splits, unroll) for geometry g from a
// partial request (kind may be AUTO; zero fields mean "choose").
Plan resolve_plan(const ReadGeom &g, Plan want, int num_cus);

// Is the (kind, tile, unroll) combination compiled in?
bool plan_supported(const Plan &p);

// Enqueue the read: kernels on `stream`; `partials` must hold
// partial_bytes(g, p) bytes. When ev_begin / ev_end are given they take the
// start and end times of the main read kernel's dispatch (not the staging or
// split-reduction kernels); g.done, when given, is recorded once the read's
// last kernel has completed.
hipError_t launch_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream,
                       hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

// --- epoch writes ------------------------------------------------------
// dst[idx[e]] = src[e] for e < count; each entry `stride` bytes, 16-aligned.
hipError_t launch_scatter_rows(void *dst, const void *src, const uint64_t *idx, uint64_t count,
                               uint64_t stride, hipStream_t stream);
// dst[idx[e]] = src[idx[e]] for e < count.
hipError_t launch_copy_rows(void *dst, const void *src, const uint64_t *idx, uint64_t count,
                            uint64_t stride, hipStream_t stream);

// --- request staging ------------------------------------------------------
// Qt[w * Bp + r] = 32-bit word w of request row r with bits >= n cleared;
// rows B <= r < Bp are zero. Bp % 64 == 0.
hipError_t launch_transpose_requests(const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t *Qt,
                                     uint32_t Bp, hipStream_t stream);

// Qs[g * Bp + r] = (byte g of request row r) << 8 for every 8-bucket group g
// (4 * ceil(n / 32) groups); rows B <= r < Bp are zero. Bp % 64 == 0.
hipError_t launch_stage_group_offsets(const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t *Qs,
                                      uint32_t Bp, hipStream_t stream);

// dst row i = src row rows[i], i < count; pitches multiples of 16, rows of
// round_up(row_bytes, 16) bytes are copied. src and rows may be host-mapped.
// Row copy: dst row (dst_rows ? dst_rows[i] : i) = src row (src_rows ?
// src_rows[i] : i) for i < count, row_bytes bytes each (multiple of 4; rows
// and pitches 4-byte aligned). One workgroup per row.
hipError_t launch_move_rows(void *dst, uint64_t dst_pitch, const uint64_t *dst_rows, const void *src,
                            uint64_t src_pitch, const uint64_t *src_rows, uint64_t count, uint64_t row_bytes,
                            hipStream_t stream);
hipError_t launch_gather_rows(void *dst, uint64_t dst_pitch, const void *src, uint64_t src_pitch,
                              const uint32_t *rows, uint32_t count, uint64_t row_bytes, hipStream_t stream);

// --- interest vector -----------------------------------------------------
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t stream);           // bytes % 4 == 0
// The last step of a read: XOR the bucket splits' partials into the response
// rows (splits > 1), and apply the one-time masks when g.keys is set (fused
// into that reduction, or in place on the rows when there were no splits).
hipError_t launch_split_reduce(const void *partials, uint32_t splits, const ReadGeom &g, hipStream_t stream);
// out row r (pitch out_pitch) = XOR over s < splits of partials[s][r]
// ([splits][B][stride] bytes); `done`, when set, is recorded by the kernel.
hipError_t launch_xor_splits(const void *partials, uint32_t splits, uint32_t B, uint64_t stride, void *out,
                             uint64_t out_pitch, hipStream_t stream, hipEvent_t done);
hipError_t launch_mask_rows(const void *partials, uint32_t splits, uint32_t B, uint64_t stride, void *out,
                            uint64_t out_pitch, const uint32_t *keys, hipStream_t stream, hipEvent_t done = nullptr);

// Leader combine (serialized PIR): out row r = XOR of the l input rows r.
constexpr uint32_t COMBINE_MAX = 16;
struct CombineArgs {
    uint4 *out;
    uint64_t out_row16;
    const uint4 *in[COMBINE_MAX];
    uint64_t in_row16;
    uint32_t l, B;
    uint64_t row16;
};
hipError_t launch_xor_combine(const CombineArgs &a, hipStream_t stream);

// Epoch commit, device half (one launch): staged rows into the back copy and
// the interest-vector update (see commit_kernel).
// Interest-vector words per commit block: a block's 256 threads are 16
// slices of the window, so each thread ORs about window / 16 ring rows, all
// loads in flight at once.
constexpr uint32_t COMMIT_IV_WORDS = 16;
struct CommitArgs {
    uint4 *back;               // back copy
    const uint4 *rows;         // nrows staged rows (stride16 uint4 each), mapped host memory
    const uint64_t *idx;       // their bucket indices, mapped host memory
    uint64_t nrows, stride16;
    uint32_t *global;          // global vector to write (the back copy's)
    uint32_t *ring;            // window x words deltas
    uint32_t window, slot;     // slot = this epoch's delta
    uint64_t words, iv_blocks; // iv_blocks = ceil(words / COMMIT_IV_WORDS)
    const uint32_t *pos;       // positions sorted by block, mapped host memory
    const uint32_t *pos_start; // block b: pos[pos_start[b] .. pos_start[b + 1])
};
hipError_t launch_commit(const CommitArgs &a, hipStream_t stream);



// --- preprocessed reads (Strassen leaves over the Four-Russians kernels) --
constexpr uint32_t PREP_MAX_LEVELS = 2;
constexpr uint32_t PREP_MAX_LEAVES = 49;  // 7^2
constexpr uint32_t PREP_MAX_BLOCKS = 16;  // C blocks at two levels (4 x 4)
// Leaf tables of an L-level recursion: leaf i sums the A blocks a[i][..]
// and the D blocks d[i][..] ((row << 4) | col in the 2^L grid); C block b
// (row * grid + col) is the XOR of the leaves o_leaf[b][..].
struct PrepTables {
    uint32_t leaves, grid;
    uint8_t a_cnt[PREP_MAX_LEAVES], d_cnt[PREP_MAX_LEAVES];
    uint8_t a[PREP_MAX_LEAVES][4], d[PREP_MAX_LEAVES][4];
    uint8_t o_cnt[PREP_MAX_BLOCKS];
    uint8_t o_leaf[PREP_MAX_BLOCKS][16];
};
bool prep_tables(uint32_t levels, PrepTables *t);
// Whether launch_stage_leaf_pairs serves leaf reads of geometry g (n, B, the
// leaf's) under plan p, and the bytes a read of geometry g stages (32-bit
// entries, or the 16-bit entries of staged leaves when half).
bool leaf_staging_supported(const ReadGeom &g, const Plan &p, uint32_t leaves);
uint64_t m4rw_staging_bytes(const ReadGeom &g, const Plan &p, bool half);
// The pair-table entries (16-bit) of every leaf's request rows (leaf i at
// staged + i * leaf_bytes), staged from the B request rows Q (pitch qpitch
// bytes, 4-byte aligned, n bits) of a read.
hipError_t launch_stage_leaf_pairs(const PrepTables &t, const void *Q, uint64_t qpitch, uint32_t B, uint64_t n,
                                   const ReadGeom &g, const Plan &p, void *staged, uint64_t leaf_bytes,
                                   hipStream_t stream);
// Leaf databases: leaf i (leaf_bytes apart, rows Cq bytes) = XOR of its D
// blocks, rows Nq per block (rows >= n of D read as zero).
hipError_t launch_prep_d(const PrepTables &t, const void *D, uint64_t stride, uint64_t n, uint64_t Nq, uint32_t Cq,
                         void *out, uint64_t leaf_bytes, hipStream_t stream);
// The leaf rows x = idx[k] mod Nq (k < count, idx device-readable) of every
// leaf, recomputed from D as launch_prep_d forms them.
hipError_t launch_prep_rows(const PrepTables &t, const void *D, uint64_t stride, uint64_t n, uint64_t Nq, uint32_t Cq,
                            const uint64_t *idx, uint64_t count, void *out, uint64_t leaf_bytes, hipStream_t stream);
// Leaf requests: leaf i (leaf_bytes apart, rows out_pitch bytes, Bq rows of
// Wq words) = XOR of its A blocks of the B request rows (bits >= n zero).
hipError_t launch_prep_q(const PrepTables &t, const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t Bq,
                         uint64_t Wq, void *out, uint64_t out_pitch, uint64_t leaf_bytes, hipStream_t stream);
// Answers: row r < B of `out` = the XOR of the leaf products (Bq x Cq bytes
// each, leaf_bytes apart) that reach each of its blocks; records `done`.
hipError_t launch_prep_out(const PrepTables &t, const void *leaves, uint64_t leaf_bytes, uint32_t B, uint32_t Bq,
                           uint32_t Cq, void *out, uint64_t out_pitch, hipStream_t stream, hipEvent_t done);

}  // namespace talek
