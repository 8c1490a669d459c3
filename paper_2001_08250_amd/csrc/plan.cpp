// Read-schedule selection: kernel family, request tile, bucket splits, unroll.
#include <algorithm>

#include "engine.h"

namespace talek {

bool tile_plan_supported(const Plan &p);
hipError_t launch_tile_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                            hipEvent_t ee);
bool m4r_plan_supported(const Plan &p);
hipError_t launch_m4r_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                           hipEvent_t ee);
uint32_t m4r_tasks(const ReadGeom &g, const Plan &p);
uint64_t m4r_staging_bytes(const ReadGeom &g);
bool m4rw_plan_supported(const Plan &p);
hipError_t launch_m4rw_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                            hipEvent_t ee);
uint32_t m4rw_tasks(const ReadGeom &g, const Plan &p);
uint64_t m4rw_staging_bytes(const ReadGeom &g, const Plan &p, bool half);
uint64_t m4rw_steps(uint64_t n, const Plan &p);

namespace {

constexpr uint64_t PARTIAL_CAP = 256ull << 20;  // bytes of split partials per read
constexpr uint64_t PARTIAL_SOFT = 64ull << 20;  // the tile kernels aim lower (or at 1/64 of D if larger)

uint32_t pow2_at_least(uint32_t x)
{
    uint32_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

}  // namespace

bool plan_supported(const Plan &p)
{
    if (p.kind == KIND_M4R)
        return m4r_plan_supported(p);
    if (p.kind == KIND_M4RW)
        return m4rw_plan_supported(p);
    return tile_plan_supported(p);
}

uint64_t partial_bytes(const ReadGeom &g, const Plan &p)
{
    uint64_t bytes = p.splits <= 1 ? 0 : (uint64_t)p.splits * g.leaves * g.B * g.stride;
    if (p.kind == KIND_M4R)
        bytes += m4r_staging_bytes(g);
    if (p.kind == KIND_M4RW && !(g.staged && (p.flags & PLAN_PAIRS)))
        bytes += m4rw_staging_bytes(g, p, false);
    return bytes;
}

Plan resolve_plan(const ReadGeom &g, Plan want, int num_cus)
{
    Plan p = want;
    if (p.kind == KIND_AUTO) {
        // Small batches stream D with the masked tile kernel. Above 16
        // requests, paired Four-Russians tables shared by the requests of a
        // workgroup win: 4-bucket tables (two workgroups per CU) for one
        // workgroup of up to 128 requests, 5-bucket tables (one workgroup of
        // up to 256 requests per CU) above, where their fewer lookups per
        // request outweigh the larger table builds. A request tile covers
        // the whole batch up to 256 requests (a second tile would build
        // every table again). Above 256 requests over rows of 512 bytes or
        // more, 6-bucket tables of 512-byte entries, a request per half
        // wave, 512 requests a workgroup: 12 buckets per two lookups (73.0
        // against 80.8 ms for 2048 requests over 2^22 rows of 4 KiB; 1.18
        // against 1.32 ms for 512 over 2^20 of 1 KiB).
        if (g.B > 256 && g.stride >= 512) {
            p.kind = KIND_M4RW;
            p.flags = PLAN_PAIRS | PLAN_HALF_WAVES | PLAN_PAIR_G6;
            p.unroll = 8;
            p.tile = 64;
        } else if (g.B > 128) {
            p.kind = KIND_M4RW;
            p.flags = PLAN_PAIRS;
            p.unroll = 8;
            p.tile = 32;
        } else if (g.B > 16) {
            p.kind = KIND_M4RW;
            p.flags = PLAN_PAIRS | (1u << PLAN_PAIR_G_SHIFT);
            p.unroll = 8;
            p.tile = g.B > 64 ? 16 : g.B > 32 ? 8 : 4;
        } else {
            // masked XOR; from 4 to 8 requests the four waves of a workgroup
            // share one 1 KiB column chunk (one wave's tile holds them all),
            // which streams D faster than four chunks per workgroup
            p.kind = KIND_MASK;
            if (g.B >= 4 && g.B <= 8) {
                p.flags = PLAN_SHARED_COLUMN;
                p.unroll = 4;
            }
        }
    }
    const uint64_t nwords = (g.n + 31) / 32;
    const uint32_t stride16 = (uint32_t)(g.stride / 16);
    uint64_t units;  // independent workgroup tasks per split
    uint64_t per_cu = 8;  // workgroups per CU to aim for
    if (p.kind == KIND_M4R) {
        // tile = requests per wave, unroll = waves per workgroup
        if (p.tile == 0)
            p.tile = 32;
        if (p.unroll == 0)
            p.unroll = g.B >= 256 ? 8 : 4;
        units = m4r_tasks(g, Plan{p.kind, p.tile, 1, p.unroll, 0});
        per_cu = 2;  // one 128 KiB LDS table pair per CU at a time
    } else if (p.kind == KIND_M4RW) {
        if (p.tile == 0)
            p.tile = (p.flags & PLAN_HALF_WAVES) ? 64 : g.B > 128 ? 32 : 16;
        if (p.unroll == 0)
            p.unroll = 8;
        units = m4rw_tasks(g, Plan{p.kind, p.tile, 1, p.unroll, p.flags});
        // double-buffered tables of 128 KiB fill a CU's LDS; paired 4- and
        // 3-bucket tables (64 / 32 KiB) let two workgroups share it
        per_cu = ((p.flags & PLAN_PAIRS) && ((p.flags >> PLAN_PAIR_G_SHIFT) & 3u)) ? 2 : 1;
    } else {
        if (p.tile == 0)
            p.tile = g.B <= 16 ? pow2_at_least(std::max<uint32_t>(g.B, 1)) : 16;
        if (p.unroll == 0)
            p.unroll = p.tile <= 2 ? 16 : p.tile >= 16 ? 4 : 8;
        const bool share = p.flags & PLAN_SHARED_COLUMN;
        const uint64_t rows_per_wg = (uint64_t)p.tile * (share ? 4 : 1);
        const uint64_t n_rt = (g.B + rows_per_wg - 1) / rows_per_wg;
        const uint64_t n_cg = share ? (stride16 + 63) / 64 : (stride16 + 255) / 256;
        units = n_rt * n_cg;
    }
    if (p.splits == 0) {
        const uint64_t target = (uint64_t)std::max(num_cus, 1) * per_cu;
        uint64_t s = (target + units - 1) / std::max<uint64_t>(units, 1);
        s = std::min<uint64_t>(s, std::max<uint64_t>(nwords / 2, 1));  // >= 64 buckets per split
        const uint64_t per_split = (uint64_t)g.B * g.stride;
        if (per_split)
            s = std::min<uint64_t>(s, std::max<uint64_t>(PARTIAL_CAP / per_split, 1));
        if (per_split && (p.kind == KIND_MASK || p.kind == KIND_SKIP)) {
            // These kernels stream D at HBM speed, and every split adds a
            // partial answer that is written and read again: halve the
            // splits while the partials exceed 64 MiB and 1/64 of the
            // snapshot, down to two workgroups per CU (at B = 16 over 4 GiB,
            // 1024 splits ran 3% faster than 2048 and 512 7% slower; an
            // uneven 1365 at B = 12 ran 7% slower than 2048).
            const uint64_t cap = std::max<uint64_t>(PARTIAL_SOFT, g.n * g.stride / 64);
            const uint64_t least = ((uint64_t)std::max(num_cus, 1) * 2 + units - 1) / std::max<uint64_t>(units, 1);
            while (s * per_split > cap && s / 2 >= least)
                s /= 2;
        }
        p.splits = (uint32_t)std::max<uint64_t>(s, 1);
    }
    const uint64_t max_splits = p.kind == KIND_M4RW ? m4rw_steps(g.n, p) : nwords;
    p.splits = (uint32_t)std::min<uint64_t>(p.splits, std::max<uint64_t>(max_splits, 1));
    return p;
}

hipError_t launch_split_reduce(const void *partials, uint32_t splits, const ReadGeom &g, hipStream_t stream)
{
    if (g.keys)
        return launch_mask_rows(partials, splits, g.B, g.stride, g.out, g.out_pitch, g.keys, stream, g.done);
    return launch_xor_splits(partials, splits, g.B, g.stride, g.out, g.out_pitch, stream, g.done);
}

hipError_t launch_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t ev_begin,
                       hipEvent_t ev_end)
{
    if (g.B == 0)
        return hipSuccess;
    if (g.leaves != 1 && !(g.leaves > 1 && g.staged && p.kind == KIND_M4RW && (p.flags & PLAN_PAIRS)))
        return hipErrorInvalidValue;
    hipError_t e;
    if (p.kind == KIND_M4R)
        e = launch_m4r_read(g, p, partials, stream, ev_begin, ev_end);
    else if (p.kind == KIND_M4RW)
        e = launch_m4rw_read(g, p, partials, stream, ev_begin, ev_end);
    else
        e = launch_tile_read(g, p, partials, stream, ev_begin, ev_end);
    // without splits the kernel wrote the plain answers: mask them in place
    if (e == hipSuccess && p.splits <= 1) {
        if (g.keys)
            e = launch_mask_rows(nullptr, 0, g.leaves * g.B, g.stride, g.out, g.out_pitch, g.keys, stream, g.done);
        else if (g.done)
            e = hipEventRecord(g.done, stream);
    }
    return e;
}

}  // namespace talek
