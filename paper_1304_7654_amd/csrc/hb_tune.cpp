// Autotuner of the batched stage kernel.  The tuning space is the tile shape
// (16 x 15 or 32 x 7 output cells per 256-thread workgroup), the order of
// the tile list (tile rows or tile columns within each block), the XCD-aware
// workgroup renumbering, and the grid: persistent with a number of resident
// workgroups per CU, or one workgroup per tile.  Every candidate runs full pseudo-time iterations on a
// scratch copy of the caller's state, timed with HIP events; the fastest is
// applied.  Results go to a small JSON cache keyed by the device and the
// workload signature (block sizes, N_H, boundary kinds, precision), so a
// later process on the same device and workload applies the choice without
// timing.  The tuning never changes a cell's arithmetic: only which
// workgroup computes which tile, and the order of the per-tile norm
// partials (norms may differ in the last bits, states do not).
#include "hb_internal.hpp"

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

namespace hb {
namespace {

std::string signature(const hb_grid *g) {
    uint64_t h = 1469598103934665603ull;            // FNV-1a over the workload description
    auto mix = [&h](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const BlockDesc &B : g->blk) {
        mix(B.ni); mix(B.nj); mix(B.nh);
        for (int s = 0; s < 4; ++s) mix(B.bc[s]);
    }
    mix(g->solver.precision);
    mix(g->solver.n_stages);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[160];
    snprintf(buf, sizeof(buf), "%s/cu%d/blocks%d/prec%d/%016llx", arch.c_str(), cus, g->nblocks,
             g->solver.precision, (unsigned long long)h);
    return buf;
}

// Cache file: a JSON object with one entry per line,
//   "<key>": {"tile_i": 16, "wg_per_cu": 3, "xcd_order": 1, "tile_order": 0, "stage_ms": 0.4},
bool cache_lookup(const char *path, const std::string &key, hb_tuning *t) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string head = "\"" + key + "\":";
    while (std::getline(f, line)) {
        const size_t p = line.find(head);
        if (p == std::string::npos) continue;
        hb_tuning r{};
        if (sscanf(line.c_str() + p + head.size(),
                   " {\"tile_i\": %d, \"wg_per_cu\": %d, \"xcd_order\": %d, \"tile_order\": %d, "
                   "\"stage_ms\": %lf", &r.tile_i, &r.wg_per_cu, &r.xcd_order, &r.tile_order,
                   &r.stage_ms) == 5) {
            *t = r;
            return true;
        }
    }
    return false;
}

int cache_store(const char *path, const std::string &key, const hb_tuning &t) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        const std::string head = "\"" + key + "\":";
        while (f && std::getline(f, line))
            if (line.find("\": {\"tile_i\"") != std::string::npos && line.find(head) == std::string::npos) {
                while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
                keep.push_back(line);
            }
    }
    char buf[256];
    snprintf(buf, sizeof(buf),
             "  \"%s\": {\"tile_i\": %d, \"wg_per_cu\": %d, \"xcd_order\": %d, \"tile_order\": %d, "
             "\"stage_ms\": %.9g}", key.c_str(), t.tile_i, t.wg_per_cu, t.xcd_order, t.tile_order,
             t.stage_ms);
    keep.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        if (!o) return fail(HB_ERR_ARG, "cannot write the tuning cache");
        o << "{\n";
        for (size_t k = 0; k < keep.size(); ++k) o << keep[k] << (k + 1 < keep.size() ? ",\n" : "\n");
        o << "}\n";
        if (!o) return fail(HB_ERR_ARG, "cannot write the tuning cache");
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(HB_ERR_ARG, "cannot replace the tuning cache");
    return HB_OK;
}

int apply(hb_grid *g, const hb_tuning &t) {
    if (t.wg_per_cu < -1 || t.wg_per_cu > 16 || (t.xcd_order != 0 && t.xcd_order != 1))
        return fail(HB_ERR_ARG, "wg_per_cu must be in [-1, 16] and xcd_order 0 or 1");
    if (t.tile_i != g->tile_ti || t.tile_order != g->tune_order) {
        const int rc = fused_build_tiles(g, t.tile_i, t.tile_order);
        if (rc) return rc;
    } else if (t.tile_i != 16 && t.tile_i != 32) {
        return fail(HB_ERR_ARG, "tile_i must be 16 or 32");
    }
    if (g->tune_wg_per_cu != t.wg_per_cu || g->tune_xcd != t.xcd_order) fused_drop_graph(g);
    g->tune_wg_per_cu = t.wg_per_cu;
    g->tune_xcd = t.xcd_order;
    g->tune_ms = t.stage_ms;
    return HB_OK;
}

}  // namespace

int tune_get(const hb_grid *g, hb_tuning *t) {
    t->tile_i = g->tile_ti;
    t->wg_per_cu = g->tune_wg_per_cu;
    t->xcd_order = g->tune_xcd;
    t->tile_order = g->tune_order;
    t->stage_ms = g->tune_ms;
    return HB_OK;
}

int tune_set(hb_grid *g, const hb_tuning *t) {
    int rc = check_hip(hipDeviceSynchronize(), "sync");
    return rc ? rc : apply(g, *t);
}

int tune_run(hb_grid *g, const double *q, const char *cache_path, int force, hb_tuning *out,
             hipStream_t s) {
    const std::string key = signature(g);
    hb_tuning best{};
    if (cache_path && !force && cache_lookup(cache_path, key, &best)) {
        int rc = tune_set(g, &best);
        if (!rc && out) *out = best;
        return rc;
    }
    double *scratch = nullptr;
    int rc = check_hip(hipMalloc((void **)&scratch, sizeof(double) * g->n_state), "tuning scratch");
    if (rc) return rc;
    std::vector<hb_tuning> cands;
    for (int ti : {16, 32})
        for (int order : {0, 1})
            for (int xcd : {1, 0})
                for (int wg : {0, 2, 1, -1}) cands.push_back(hb_tuning{ti, wg, xcd, order, 0.0});
    best.stage_ms = 1e30;
    for (hb_tuning &c : cands) {
        rc = tune_set(g, &c);
        if (rc) break;
        double ms = 0.0;
        rc = check_hip(hipMemcpyAsync(scratch, q, sizeof(double) * g->n_state, hipMemcpyDeviceToDevice, s),
                       "tuning copy");
        rc = rc ? rc : fused_time_iterations(g, scratch, 1, &ms, s);          // warm-up
        rc = rc ? rc : check_hip(hipMemcpyAsync(scratch, q, sizeof(double) * g->n_state,
                                                hipMemcpyDeviceToDevice, s), "tuning copy");
        rc = rc ? rc : fused_time_iterations(g, scratch, 3, &ms, s);
        if (rc) break;
        c.stage_ms = ms;
        if (ms < best.stage_ms) best = c;
    }
    (void)hipFree(scratch);
    // the timing runs leave the status flag and counters of scratch states
    (void)hipMemsetAsync(g->status_d, 0, sizeof(int), s);
    if (rc) return rc;
    rc = tune_set(g, &best);
    if (!rc && cache_path) rc = cache_store(cache_path, key, best);
    if (!rc && out) *out = best;
    return rc;
}

}  // namespace hb
