// Restart files and per-snapshot solution files.
//
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

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
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

namespace {

// One solution record per (block, snapshot n): the nodes of snapshot n
// (the body-frame nodes moved by the rigid motion when one is set) and the
// primitives (rho, u, v, p) of every cell:
//   [x (nj+1)(ni+1)][y (nj+1)(ni+1)][rho nj ni][u][v][p]
// grid.y = snapshot; one thread per node (and per cell, cells < nodes).
__global__ void k_sol_record(const BlockDesc *blks, int b, const double *q, const double *xy,
                             Motion mo, double gamma, double *out) {
    const BlockDesc &B = blks[b];
    const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1), nc = (int64_t)B.ni * B.nj;
    const int n = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double *rec = out + (int64_t)n * (2 * nn + 4 * nc);
    if (t < nn) {
        double x = xy[2 * B.node_off + t], y = xy[2 * B.node_off + nn + t];
        if (mo.tab) {
            const double *m = mo.tab + (int64_t)kMotionW * (B.snap_off + n);
            const double rx = x - mo.xp, ry = y - mo.yp;
            x = mo.xp + m[0] * rx - m[1] * ry;
            y = mo.yp + m[3] + m[1] * rx + m[0] * ry;
        }
        rec[t] = x;
        rec[nn + t] = y;
    }
    if (t < nc) {
        const double *qn = q + B.q_off + (int64_t)n * 4 * nc;
        const double rho = qn[t], u = qn[nc + t] / rho, v = qn[2 * nc + t] / rho;
        const double pr = (gamma - 1.0) * (qn[3 * nc + t] - 0.5 * rho * (u * u + v * v));
        double *w = rec + 2 * nn;
        w[t] = rho;
        w[nc + t] = u;
        w[2 * nc + t] = v;
        w[3 * nc + t] = pr;
    }
}

const char kSolMagic[8] = {'H', 'B', 'S', 'O', 'L', 'N', '0', '1'};

}  // namespace

int io_save_solution(hb_grid *g, const double *q, const char *prefix, hipStream_t s) {
    // staging: the records of every block and snapshot, blocks in order
    std::vector<int64_t> off(g->nblocks + 1, 0);
    int max_ns = 0;
    for (int b = 0; b < g->nblocks; ++b) {
        const BlockDesc &B = g->blk[b];
        const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1), nc = (int64_t)B.ni * B.nj;
        off[b + 1] = off[b] + (int64_t)B.ns * (2 * nn + 4 * nc);
        max_ns = std::max(max_ns, (int)B.ns);
    }
    double *stage = nullptr;
    int rc = check_hip(hipMalloc((void **)&stage, sizeof(double) * off[g->nblocks]), "solution staging");
    if (rc) return rc;
    for (int b = 0; b < g->nblocks && !rc; ++b) {
        const BlockDesc &B = g->blk[b];
        const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1);
        hipLaunchKernelGGL(k_sol_record, dim3((unsigned)((nn + 255) / 256), B.ns), dim3(256), 0, s,
                           g->blk_d, b, q, g->xy_d, g->motion, g->flow.gamma, stage + off[b]);
        rc = check_hip(hipGetLastError(), "solution launch");
    }
    std::vector<double> host(off[g->nblocks]);
    rc = rc ? rc : check_hip(hipMemcpyAsync(host.data(), stage, sizeof(double) * host.size(),
                                            hipMemcpyDeviceToHost, s), "solution copy");
    rc = rc ? rc : check_hip(hipStreamSynchronize(s), "sync");
    (void)hipFree(stage);
    if (rc) return rc;
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < max_ns; ++k) {
        // file k: every block with more than k snapshots, one write
        std::vector<unsigned char> buf;
        auto put = [&buf](const void *p, size_t n) {
            const unsigned char *c = static_cast<const unsigned char *>(p);
            buf.insert(buf.end(), c, c + n);
        };
        int32_t nb = 0;
        for (const BlockDesc &B : g->blk) nb += B.ns > k;
        const int32_t kk = k;
        put(kSolMagic, 8);
        put(&kk, 4);
        put(&nb, 4);
        for (int b = 0; b < g->nblocks; ++b) {
            const BlockDesc &B = g->blk[b];
            if (B.ns <= k) continue;
            const int64_t nn = (int64_t)(B.ni + 1) * (B.nj + 1), nc = (int64_t)B.ni * B.nj;
            const int32_t v[4] = {b, B.ni, B.nj, B.nh};
            const double phase = two_pi * k / B.ns;
            put(v, sizeof v);
            put(&phase, 8);
            put(host.data() + off[b] + (int64_t)k * (2 * nn + 4 * nc), sizeof(double) * (2 * nn + 4 * nc));
        }
        const uint64_t sum = fnv(buf.data() + 8, buf.size() - 8);
        put(&sum, 8);
        const std::string path = std::string(prefix) + ".snap" + std::to_string(k);
        const std::string tmp = path + ".tmp";
        FILE *f = std::fopen(tmp.c_str(), "wb");
        if (!f) return fail(HB_ERR_ARG, "cannot open the solution file for writing");
        const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);       // one aggregated write
        const int cl = std::fclose(f);
        if (w != buf.size() || cl != 0) return fail(HB_ERR_ARG, "solution file write failed");
        if (std::rename(tmp.c_str(), path.c_str()) != 0)
            return fail(HB_ERR_ARG, "cannot replace the solution file");
    }
    return HB_OK;
}

}  // namespace hb
