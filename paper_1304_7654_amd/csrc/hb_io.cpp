// Restart files: the whole state of a grid (every block and snapshot, the
// public FP64 layout) in one aggregated write, in the spirit of the paper's
// I/O optimisation (§MPI Optimisations, the part on MPI I/O: one collective write of all blocks
// and harmonics instead of one file per process).  Layout (little endian):
//   char[8]  "HBSTATE1"
//   uint64   workload signature (FNV-1a over block sizes, N_H, boundary kinds)
//   int64    iteration counter (caller's)
//   int64    n_state (doubles)
//   int32    nblocks, then per block int32 ni, nj, n_harm
//   double   state[n_state]
//   uint64   FNV-1a of the state bytes
#include "hb_internal.hpp"

#include <cstdio>
#include <cstring>
#include <vector>

namespace hb {
namespace {

uint64_t fnv(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t k = 0; k < n; ++k) {
        h ^= c[k];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t workload_signature(const hb_grid *g) {
    uint64_t h = 1469598103934665603ull;
    for (const BlockDesc &B : g->blk) {
        const int32_t v[7] = {B.ni, B.nj, B.nh, B.bc[0], B.bc[1], B.bc[2], B.bc[3]};
        h = fnv(v, sizeof v, h);
    }
    return h;
}

const char kMagic[8] = {'H', 'B', 'S', 'T', 'A', 'T', 'E', '1'};

}  // namespace

int io_save(hb_grid *g, const double *q, int64_t iteration, const char *path, hipStream_t s) {
    std::vector<double> host(g->n_state);
    int rc = check_hip(hipMemcpyAsync(host.data(), q, sizeof(double) * g->n_state, hipMemcpyDeviceToHost, s),
                       "state copy");
    rc = rc ? rc : check_hip(hipStreamSynchronize(s), "sync");
    if (rc) return rc;
    std::vector<unsigned char> buf;
    auto put = [&buf](const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        buf.insert(buf.end(), c, c + n);
    };
    const uint64_t sig = workload_signature(g);
    const int64_t ns = g->n_state;
    const int32_t nb = g->nblocks;
    put(kMagic, 8);
    put(&sig, 8);
    put(&iteration, 8);
    put(&ns, 8);
    put(&nb, 4);
    for (const BlockDesc &B : g->blk) {
        const int32_t v[3] = {B.ni, B.nj, B.nh};
        put(v, sizeof v);
    }
    put(host.data(), sizeof(double) * host.size());
    const uint64_t sum = fnv(host.data(), sizeof(double) * host.size());
    put(&sum, 8);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(HB_ERR_ARG, "cannot open the restart file for writing");
    const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);       // one aggregated write
    const int cl = std::fclose(f);
    if (w != buf.size() || cl != 0) return fail(HB_ERR_ARG, "restart file write failed");
    if (std::rename(tmp.c_str(), path) != 0) return fail(HB_ERR_ARG, "cannot replace the restart file");
    return HB_OK;
}

int io_load(hb_grid *g, double *q, int64_t *iteration, const char *path, hipStream_t s) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(HB_ERR_ARG, "cannot open the restart file");
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t r;
    while ((r = std::fread(chunk, 1, sizeof chunk, f)) > 0) buf.insert(buf.end(), chunk, chunk + r);
    std::fclose(f);
    const size_t head = 8 + 8 + 8 + 8 + 4 + 12 * (size_t)g->nblocks;
    const size_t need = head + sizeof(double) * (size_t)g->n_state + 8;
    if (buf.size() != need || std::memcmp(buf.data(), kMagic, 8) != 0)
        return fail(HB_ERR_ARG, "not a restart file of this grid (size or magic)");
    uint64_t sig, sum;
    int64_t it, ns;
    int32_t nb;
    std::memcpy(&sig, buf.data() + 8, 8);
    std::memcpy(&it, buf.data() + 16, 8);
    std::memcpy(&ns, buf.data() + 24, 8);
    std::memcpy(&nb, buf.data() + 32, 4);
    if (sig != workload_signature(g) || ns != g->n_state || nb != g->nblocks)
        return fail(HB_ERR_ARG, "restart file of another workload");
    for (int b = 0; b < g->nblocks; ++b) {
        int32_t v[3];
        std::memcpy(v, buf.data() + 36 + 12 * (size_t)b, 12);
        const BlockDesc &B = g->blk[b];
        if (v[0] != B.ni || v[1] != B.nj || v[2] != B.nh)
            return fail(HB_ERR_ARG, "restart file of another workload");
    }
    const unsigned char *data = buf.data() + head;
    std::memcpy(&sum, data + sizeof(double) * (size_t)g->n_state, 8);
    if (sum != fnv(data, sizeof(double) * (size_t)g->n_state))
        return fail(HB_ERR_ARG, "restart file checksum mismatch");
    int rc = check_hip(hipMemcpyAsync(q, data, sizeof(double) * g->n_state, hipMemcpyHostToDevice, s),
                       "state upload");
    rc = rc ? rc : check_hip(hipStreamSynchronize(s), "sync");
    if (!rc && iteration) *iteration = it;
    return rc;
}

}  // namespace hb
