// Autotuner for the read schedule: times candidate (kernel family, request
// tile, bucket splits, unroll) combinations on the device for a given
// (n, B class, bucket stride) and keeps the fastest in a process-wide table
// that can be saved to / loaded from JSON.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "db.h"

namespace talek {
namespace {

struct Entry {
    Plan plan;
    double us;
};

using Key = std::tuple<uint64_t, uint32_t, uint64_t>;  // n, B class, stride

std::mutex g_mu;
std::map<Key, Entry> g_table;

uint32_t b_class(uint32_t B)
{
    uint32_t c = 1;
    while (c < B)
        c <<= 1;
    return c;
}

}  // namespace

bool tune_lookup(uint64_t n, uint32_t B, uint64_t stride, Plan *p)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(Key{n, b_class(B), stride});
    if (it == g_table.end())
        return false;
    *p = it->second.plan;
    return true;
}

}  // namespace talek

using namespace talek;

extern "C" {

int pir_tune(pir_db *db, uint32_t B, uint32_t iters, pir_plan *best, double *best_us)
{
    if (!db || B == 0 || iters == 0)
        return PIR_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(db->mu);
    if (hipSetDevice(db->device) != hipSuccess)
        return PIR_EDEVICE;
    Scratch &sc = scratch_for(db, db->stream);
    int rc = ensure_device(&sc.req, &sc.req_cap, (uint64_t)B * db->qpitch);
    if (rc == PIR_OK)
        rc = ensure_device(&sc.resp, &sc.resp_cap, (uint64_t)B * db->stride);
    if (rc != PIR_OK)
        return rc;
    // Request bits for timing: density 1/2 from a fixed linear congruential
    // sequence (the SKIP family's cost depends on the density only).
    std::vector<uint8_t> host((size_t)B * db->qpitch);
    uint64_t x = 0x243F6A8885A308D3ull;
    for (auto &v : host) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        v = (uint8_t)(x >> 56);
    }
    if (hipMemcpy(sc.req, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
        return PIR_EDEVICE;

    ReadGeom g = read_geom(db, sc.req, db->qpitch, B, sc.resp, db->stride);
    std::vector<Plan> cands;
    const uint32_t tiles[] = {1, 2, 4, 8, 16, 24, 32};
    for (int kind : {KIND_MASK, KIND_SKIP}) {
        for (uint32_t t : tiles) {
            if (t > 2 * B && t != 1)
                continue;
            for (uint32_t u : {4u, 8u, 16u})
            for (uint32_t fl : {0u, PLAN_SHARED_COLUMN}) {
                Plan base = resolve_plan(g, Plan{kind, t, 0, u, fl}, db->num_cus);
                for (uint32_t sm : {1u, 2u, 4u}) {
                    for (int dir = 0; dir < 2; ++dir) {
                        if (sm == 1 && dir == 1)
                            continue;
                        Plan p = base;
                        p.splits = dir == 0 ? std::max<uint32_t>(1, base.splits / sm) : base.splits * sm;
                        if (plan_supported(p))
                            cands.push_back(p);
                    }
                }
            }
        }
    }
    for (uint32_t nw : {4u, 8u, 16u}) {
        for (uint32_t t : {16u, 32u, 64u}) {
            if (t * nw > 4 * B && !(t == 16 && nw == 4))
                continue;
            Plan base = resolve_plan(g, Plan{KIND_M4R, t, 0, nw, 0}, db->num_cus);
            for (uint32_t sm : {1u, 2u}) {
                Plan a = base, b = base;
                a.splits = std::max<uint32_t>(1, base.splits / sm);
                b.splits = base.splits * sm;
                if (plan_supported(a))
                    cands.push_back(a);
                if (sm > 1 && plan_supported(b))
                    cands.push_back(b);
            }
        }
    }
    for (uint32_t fl : {PLAN_PAIRS | PLAN_HALF_WAVES | PLAN_PAIR_G6, PLAN_PAIRS | PLAN_HALF_WAVES}) {
        for (uint32_t t : {32u, 64u}) {
            if (t * 8 > 2 * std::max<uint32_t>(B, 32) || g.stride < 512)
                continue;
            Plan base = resolve_plan(g, Plan{KIND_M4RW, t, 0, 8, fl}, db->num_cus);
            for (uint32_t sm : {1u, 2u}) {
                Plan a = base, b = base;
                a.splits = std::max<uint32_t>(1, base.splits / sm);
                b.splits = base.splits * sm;
                if (plan_supported(a))
                    cands.push_back(a);
                if (sm > 1 && plan_supported(b))
                    cands.push_back(b);
            }
        }
    }
    for (uint32_t nw : {4u, 8u, 16u})
    for (uint32_t fl : {2u << 8, 3u << 8, 4u << 8, PLAN_ROLLING, PLAN_ROLLING | (3u << 8), PLAN_PAIRS,
                        PLAN_PAIRS | (3u << 8), PLAN_PAIRS | (1u << PLAN_PAIR_G_SHIFT),
                        PLAN_PAIRS | (2u << PLAN_PAIR_G_SHIFT)}) {
        for (uint32_t t : {4u, 8u, 16u, 32u}) {
            if (t * nw > 8 * std::max<uint32_t>(B, 32))
                continue;
            Plan base = resolve_plan(g, Plan{KIND_M4RW, t, 0, nw, fl}, db->num_cus);
            for (uint32_t sm : {1u, 2u}) {
                Plan a = base, b = base;
                a.splits = std::max<uint32_t>(1, base.splits / sm);
                b.splits = base.splits * sm;
                if (plan_supported(a))
                    cands.push_back(a);
                if (sm > 1 && plan_supported(b))
                    cands.push_back(b);
            }
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return PIR_EDEVICE;
    Plan win{};
    double win_us = 1e30;
    for (const Plan &p : cands) {
        rc = ensure_device(&sc.part, &sc.part_cap, partial_bytes(g, p));
        if (rc != PIR_OK)
            continue;
        if (launch_read(g, p, sc.part, db->stream) != hipSuccess)
            continue;  // warm-up
        hipEventRecord(e0, db->stream);
        for (uint32_t i = 0; i < iters; ++i)
            launch_read(g, p, sc.part, db->stream);
        hipEventRecord(e1, db->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = PIR_EDEVICE;
            break;
        }
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        const double us = 1000.0 * ms / iters;
        if (us < win_us) {
            win_us = us;
            win = p;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == PIR_EDEVICE || win_us >= 1e30)
        return rc == PIR_OK ? PIR_EINVAL : rc;
    {
        std::lock_guard<std::mutex> tl(g_mu);
        g_table[Key{db->n, b_class(B), db->stride}] = Entry{win, win_us};
    }
    if (best) {
        best->kind = win.kind;
        best->tile = win.tile;
        best->splits = win.splits;
        best->unroll = win.unroll;
        best->flags = win.flags;
    }
    if (best_us)
        *best_us = win_us;
    return PIR_OK;
}

int pir_tune_save(const char *path)
{
    if (!path)
        return PIR_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f)
        return PIR_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : g_table) {
        const Plan &p = kv.second.plan;
        fprintf(f,
                "  {\"n\": %llu, \"bclass\": %u, \"stride\": %llu, \"kind\": %d, \"tile\": %u, \"splits\": %u, "
                "\"unroll\": %u, \"flags\": %u, \"us\": %.3f}%s\n",
                (unsigned long long)std::get<0>(kv.first), std::get<1>(kv.first),
                (unsigned long long)std::get<2>(kv.first), p.kind, p.tile, p.splits, p.unroll, p.flags, kv.second.us,
                ++i < g_table.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    fclose(f);
    return PIR_OK;
}

int pir_tune_load(const char *path)
{
    if (!path)
        return PIR_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f)
        return PIR_EINVAL;
    char line[512];
    int rc = PIR_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, "\"bclass\""))
            continue;
        unsigned long long n = 0, stride = 0;
        unsigned bclass = 0, tile = 0, splits = 0, unroll = 0, flags = 0;
        int kind = 0;
        double us = 0;
        const int got = sscanf(line,
                               " {\"n\": %llu, \"bclass\": %u, \"stride\": %llu, \"kind\": %d, \"tile\": %u, "
                               "\"splits\": %u, \"unroll\": %u, \"flags\": %u, \"us\": %lf",
                               &n, &bclass, &stride, &kind, &tile, &splits, &unroll, &flags, &us);
        if (got != 9 || kind < KIND_MASK || kind > KIND_M4RW) {
            rc = PIR_EINVAL;
            continue;
        }
        Plan p{kind, tile, splits, unroll, flags};
        if (!plan_supported(p)) {
            rc = PIR_EINVAL;
            continue;
        }
        g_table[Key{n, bclass, stride}] = Entry{p, us};
    }
    fclose(f);
    return rc;
}

}  // extern "C"
