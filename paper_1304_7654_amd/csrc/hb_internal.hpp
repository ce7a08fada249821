// Internal declarations of libhb: the grid object, the device-side block
// descriptor and the launch helpers of each kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hb.h"

namespace hb {

constexpr int kMaxNs = 9;        // N_H <= 4
constexpr int kNsPad = 16;       // padded D (MFMA tile)
constexpr int kAF = 26;          // adjoint terms stored per face and snapshot

// One glued segment of a block side; each hb_cut is listed from both of
// its sides.  Cells start .. start + len - 1 along this side lie against
// the partner block's side `side` from pstart on (reversed: running the
// other way).  Positions along a side are j on the i sides, i on the j
// sides.
struct CutSeg {
    int32_t start, len, blk, side, pstart, rev;
};

// Device-side description of one block.  Offsets index the flat arrays
// of the grid (all blocks concatenated).
struct BlockDesc {
    int32_t ni, nj, ns, nh;
    int32_t bc[4];
    int32_t wake;
    int32_t body;
    int32_t seg_off[4];      // the side's segments: segs[seg_off .. seg_off + seg_cnt), by start
    int32_t seg_cnt[4];
    int32_t rest[4];         // kind of the cells of a CUT side that no segment covers:
                             // 0 (the side is covered), HB_BC_WALL or HB_BC_FARFIELD
    const CutSeg *segs;      // the grid's segment table (device copy in blk_d)
    int32_t snap_off;        // per-snapshot tables: entries snap_off .. +ns
    int32_t d_off;           // D table (kNsPad x kNsPad per block)
    int64_t q_off;           // state (doubles): ns*4*nj*ni
    int64_t cell_off;        // per-cell arrays: nj*ni
    int64_t node_off;        // per-node arrays: (nj+1)*(ni+1)
    int64_t fi_off;          // i-faces: nj*(ni+1)
    int64_t fj_off;          // j-faces: (nj+1)*ni
    int64_t ext_off;         // plain path ghost-extended primitives: ns*4*(nj+4)*(ni+4)
    int64_t fiq_off;         // plain path i-face fluxes: ns*4*nj*(ni+1)
    int64_t fjq_off;         // plain path j-face fluxes: ns*4*(nj+1)*ni
    int64_t part_off;        // plain path norm partials of this block
    int64_t afi_off;         // adjoint: per-face adjoint terms of i-faces, ns*kAF*nj*(ni+1)
    int64_t afj_off;         // adjoint: same for j-faces, ns*kAF*(nj+1)*ni
    int64_t nodeq_off;       // adjoint: node (u, v, T) adjoints, ns*3*(nj+1)*(ni+1)
    double omega_nh;         // omega * N_H (time-step bound of the HB term)
};

// One fused-kernel work item: a tile of cells of one block.  gtab: first
// entry of the tile's halo source table, -1 when every cell of the
// ghost-extended tile is a cell of the block itself.
struct Tile {
    int32_t blk;
    int32_t i0, j0;
    int32_t ns;
    int32_t gtab;
};

// Source of a ghost-extended cell: an interior cell (b, i, j) of some block
// (cell = 1) or the far field (cell = 0), with the parity of the wall
// mirrors met on the way.
struct GSrc {
    int cell;
    int b, i, j;
    int mir;
};

// Geometry and flow constants passed by value to kernels.
struct Consts {
    double gamma, mu, kappa, prandtl, cfl, delta_frac, eps, pinf;
};

// Rigid grid motion for the plain FP64 kernels: per snapshot (block
// snapshot offset + n) kMotionW doubles {cos theta, sin theta, theta_dot,
// h, h_dot, 0, 0, 0}; tab == nullptr is the fixed grid.
constexpr int kMotionW = 8;
struct Motion {
    const double *tab;
    double xp, yp;
};

// Pointers to the FP64 metrics (see metrics kernels for layouts).
template <class T>
struct Metrics {
    const T *SI, *dI;    // [2][nj][ni+1] per block at 2*fi_off
    const T *SJ, *dJ;    // [2][nj+1][ni] per block at 2*fj_off
    const T *V;          // [nj][ni] at cell_off
};

// Per-snapshot tables: free-stream primitives (rho, u, v, p), free-stream
// conserved variables, and c_n = sum_m D[n][m] Q_inf(m).
template <class T>
struct SnapTables {
    const T *ffw;        // [snap][4]
    const T *ffq;        // [snap][4]
    const T *dqinf;      // [snap][4]
};

}  // namespace hb

struct hb_grid {
    int device = 0;
    int nblocks = 0;
    int nbody = 0;
    std::vector<hb::BlockDesc> blk;
    std::vector<hb::CutSeg> segs;                // both sides of every cut, by (block, side, start)
    hb::CutSeg *segs_d = nullptr;
    std::vector<std::vector<double>> xy_host;
    std::vector<int> body_ns, body_off;          // force layout
    hb_flow flow{};
    hb_solver solver{};
    hb::Consts consts{};
    int64_t n_state = 0, n_cells = 0, n_nodes = 0, n_fi = 0, n_fj = 0, n_ext = 0;
    int64_t n_fiq = 0, n_fjq = 0;
    int n_snap = 0;
    int64_t n_forces = 0;
    int64_t total_cs = 0;                          // cell-snapshots

    // device memory
    hb::BlockDesc *blk_d = nullptr;
    double *xy_d = nullptr;
    double *SI_d = nullptr, *dI_d = nullptr, *SJ_d = nullptr, *dJ_d = nullptr;
    double *V_d = nullptr, *C_d = nullptr;
    float *SI_f = nullptr, *dI_f = nullptr, *SJ_f = nullptr, *dJ_f = nullptr, *V_f = nullptr;
    double *D_d = nullptr;
    float *D_f = nullptr;
    double *ffw_d = nullptr, *ffq_d = nullptr, *dqinf_d = nullptr;
    float *ffw_f = nullptr, *ffq_f = nullptr, *dqinf_f = nullptr;
    // scratch
    double *ext_d = nullptr;      // plain path ghost-extended primitives
    double *mot_d = nullptr;      // motion table [snap][kMotionW]
    hb::Motion motion{};          // tab = mot_d while a motion is set
    hb_motion motion_par{};       // the motion last set (time-domain march)
    double *FI_d = nullptr, *FJ_d = nullptr;   // plain path face fluxes [ns][4][faces]
    double *q0_d = nullptr;       // RK base state copy (plain path)
    double *qa_d = nullptr, *qb_d = nullptr;   // stage ping-pong (FP64)
    float *sa_f = nullptr, *sb_f = nullptr;    // stage ping-pong shadows (FP32 bulk)
    float *dtau_f = nullptr;      // fused path: local time step of every cell-snapshot (FP32 bulk)
    double *dtau_d = nullptr;     // the same for the fused FP64 path
    double *partials_d = nullptr; int64_t n_partials = 0;
    double *fpart_d = nullptr;    // force partials [block][kMaxNs][fchunks][3]
    int fchunks = 1;              // 256-face chunks of the longest jmin side
    double *norm_tmp_d = nullptr;
    int *status_d = nullptr;
    int *body_off_d = nullptr, *body_ns_d = nullptr;
    int *body_ptr_d = nullptr, *body_blk_d = nullptr;   // blocks of each body, in block order
    int *ctr_d = nullptr;
    // fused path
    hb::Tile *tiles_d = nullptr;
    int n_tiles = 0;
    // halo source table of the tiles that touch a block side: per tile 512
    // entries (two per thread), each (source element index | mirror << 31,
    // source plane; plane 0 = far field)
    uint32_t *gtab_d = nullptr;
    // the same entries for a rigidly moving grid: (index in xy_d of the x
    // of the wall face's first node, node count of its block) for a moving
    // no-slip wall image, (0, 0) otherwise
    uint32_t *wtab_d = nullptr;
    // 64-bit halo addressing (states of 4 GiB or more, or batched = 2): the
    // source element offset of every halo table entry (0 for far field)
    bool big = false;
    uint64_t *gtab64_d = nullptr;
    int tile_ti = 16, tile_tj = 15;
    int n_cu = 0;
    // tuning of the fused path (hb_set_tuning / hb_autotune)
    int tune_wg_per_cu = 0;      // resident workgroups per CU, 0 = occupancy maximum
    int tune_xcd = 1;            // XCD-aware workgroup renumbering
    int tune_order = 0;          // 0: tiles row by row (j outer), 1: column by column
    double tune_ms = 0.0;        // measured stage time of the applied tuning (0 = not measured)
    hipStream_t cap_stream = nullptr;
    // plain path: the blocks of a stage run on side streams forked from
    // and joined back to the caller's stream (default priority)
    static constexpr int kSide = 8;
    hipStream_t side[kSide] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
    hipGraphExec_t graph_exec = nullptr;
    double *graph_q = nullptr, *graph_norm = nullptr;
    int graph_iters = 0;
    // stage instrumentation
    int prof = 0;
    std::vector<hipEvent_t> prof_ev;     // pairs (start, end), reused
    size_t prof_used = 0;
    // adjoint scratch (allocated on first use)
    double *adj_d = nullptr;
    int64_t n_adj = 0;
    int64_t n_afi = 0, n_afj = 0, n_nodeq = 0;
    double *AFI_d = nullptr, *AFJ_d = nullptr, *NB_d = nullptr, *WBext_d = nullptr;
    double *adj_part_d = nullptr;         // alpha0 partials (n_apart) + 1
    std::vector<int> apart_off;           // first alpha0 partial of each block
    int n_apart = 0;
    double *cf_adj_d = nullptr;           // forward force coefficients (forces adjoint)
    // residual adjoint: far-field code of every ghost-extended cell (0: not a
    // far-field ghost, 1: far field, -1: mirrored far field), blocks at
    // ffc_off; alpha0 partials of the cell-adjoint workgroups at cpart_off
    int8_t *ffc_d = nullptr;
    std::vector<int64_t> ffc_off, cpart_off;
    int64_t n_cpart = 0;
    double *cpart_d = nullptr;
    // coordinate adjoint: per-face sums over snapshots of (S_x, S_y, d_x, d_y)
    // adjoints (i-faces [4][n_fi], then j-faces [4][n_fj]) and the per-cell
    // adjoint of the cell area from the HB source
    double *geo_d = nullptr, *vb_d = nullptr;
    // moving grid: per face and snapshot the adjoint of the face's
    // body-frame midpoint (the face speed's dependence on the nodes)
    double *mb_d = nullptr;
    // adjoint pseudo-time iteration scratch (allocated on first use)
    double *it_lam0_d = nullptr, *it_qbar_d = nullptr, *it_dtv_d = nullptr, *it_part_d = nullptr;
    int64_t n_it_part = 0;
    // time-domain march scratch (allocated on first use)
    double *td_r_d = nullptr, *td_acc_d = nullptr, *td_qs_d = nullptr;
    int *fold_ptr_d = nullptr, *fold_b_d = nullptr, *fold_p_d = nullptr, *fold_m_d = nullptr;
    int *ff_ptr_d = nullptr, *ff_p_d = nullptr, *ff_m_d = nullptr;
    double *ext_adj_d = nullptr;          // ghost-extended primitives for the adjoint
};

namespace hb {

// The segment of side `side` of block B that covers position p (a position
// beyond the side's ends counts as its end cell), or -1.
__host__ __device__ inline int cut_seg_at(const BlockDesc &B, const CutSeg *segs, int side, int p) {
    const int L = side < 2 ? B.nj : B.ni;
    const int pc = p < 0 ? 0 : (p >= L ? L - 1 : p);
    const int o = B.seg_off[side], n = B.seg_cnt[side];
    for (int t = o; t < o + n; ++t)
        if (segs[t].start <= pc && pc < segs[t].start + segs[t].len) return t;
    return -1;
}

// Position p of side `side` of block B is glued: a CUT side covered there
// by a segment (every position of a side with rest[side] == 0).
__host__ __device__ inline bool glued_at(const BlockDesc &B, const CutSeg *segs, int side, int p) {
    return B.bc[side] == HB_BC_CUT && (B.rest[side] == 0 || cut_seg_at(B, segs, side, p) >= 0);
}

// The cell across a cut from ghost layer k (0 nearest) at position p of
// side `side` of block b: the partner block *a and its cell (*i, *j) at
// depth k inside the partner side.  A position beyond the side's ends (a
// corner ghost) continues the end segment; the result may then lie
// outside block *a, whose own side rules apply to it.  On a partly glued
// side the caller checks glued_at first.
__host__ __device__ inline void cut_cell(const BlockDesc *blks, const CutSeg *segs, int b, int side,
                                         int k, int p, int *a, int *i, int *j) {
    const BlockDesc &B = blks[b];
    int q = cut_seg_at(B, segs, side, p);
    if (q < 0) q = B.seg_off[side];
    const CutSeg g = segs[q];
    const int t = p - g.start;
    const int pp = g.pstart + (g.rev ? g.len - 1 - t : t);
    const BlockDesc &A = blks[g.blk];
    *a = g.blk;
    switch (g.side) {
        case 0: *i = k; *j = pp; break;
        case 1: *i = A.ni - 1 - k; *j = pp; break;
        case 2: *i = pp; *j = k; break;
        default: *i = pp; *j = A.nj - 1 - k; break;
    }
}

// rule applications after which a ghost must have reached an interior
// cell or the far field (checked for every ghost at grid creation)
constexpr int kGhostHops = 8;

// ghost.cpp: host-side ghost rules
// wall (optional, 3 ints): the last wall face the resolution mirrored at
// (block, side, position along the side), block -1 for none
GSrc ghost_src(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S, int b, int i, int j,
               int *wall = nullptr);
struct WallFace {
    int64_t node;    // first node of the wall face in block `blk`, -1: no wall image
    int blk;
};
WallFace wall_face(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S, int b, int i, int j);
// every ghost of every block resolves within kGhostHops rule applications
bool ghosts_resolve(const std::vector<BlockDesc> &B, const std::vector<CutSeg> &S);

// error helpers (capi.cpp)
int upload_snapshot_tables(hb_grid *g);
int fail(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);

// metrics.hip
int launch_metrics(hb_grid *g, hipStream_t s);

// plain.hip (FP64 per-block launches)
int64_t plain_partials(const BlockDesc &B);
int plain_residual(hb_grid *g, const double *q, double *r, hipStream_t s);
int plain_rk_iterate(hb_grid *g, double *q, int n_iter, double *resnorm, hipStream_t s);

// fused.hip (batched tile kernel)
int fused_build_tiles(hb_grid *g, int tile_i, int order);
int64_t fused_max_tiles(const hb_grid *g);
int fused_time_iterations(hb_grid *g, double *q, int n_iter, double *ms_per_stage, hipStream_t s);
void fused_drop_graph(hb_grid *g);
// io.cpp
int io_save(hb_grid *g, const double *q, int64_t iteration, const char *path, hipStream_t s);
int io_load(hb_grid *g, double *q, int64_t *iteration, const char *path, hipStream_t s);
int io_save_solution(hb_grid *g, const double *q, const char *prefix, hipStream_t s);
// td.hip
int launch_td_march(hb_grid *g, double *q, double t0, double dt, int n_steps, hipStream_t s);
int td_prepare(hb_grid *g);                       // the march's scratch (hb_prepare)
int launch_td_march_noalloc(hb_grid *g, double *q, double t0, double dt, int n_steps,
                            hipStream_t s);
// tune.cpp
int tune_get(const hb_grid *g, hb_tuning *t);
int tune_set(hb_grid *g, const hb_tuning *t);
int tune_run(hb_grid *g, const double *q, const char *cache_path, int force, hb_tuning *out,
             hipStream_t s);
int fused_residual(hb_grid *g, const double *q, double *r, hipStream_t s);
int fused_rk_iterate(hb_grid *g, double *q, int n_iter, double *resnorm, hipStream_t s);

// forces.hip
int launch_forces(hb_grid *g, const double *q, double *cf, hipStream_t s);

// adjoint.hip
// fill = false: the ghost-extended copy of q is already in place (a caller
// that evaluates several products at one state)
int launch_residual_adjoint(hb_grid *g, const double *q, const double *rbar, double *qbar,
                            double *xybar, double *flowbar, hipStream_t s, bool fill = true);
int launch_forces_adjoint(hb_grid *g, const double *q, const double *cfbar, double *qbar,
                          double *xybar, double *flowbar, hipStream_t s);
int launch_adjoint_iterate(hb_grid *g, const double *q, double *lam, const double *gq,
                           int n_iter, double *resnorm, hipStream_t s);
int adjoint_prepare(hb_grid *g, bool iterate);    // the adjoints' scratch (hb_prepare)

// instrumentation (capi.cpp): event pair around one stage, or no-op
int prof_begin(hb_grid *g, hipStream_t s, hipEvent_t *end);
int prof_end(hipEvent_t end, hipStream_t s);

// reduce.hip
int launch_norm_finalize(hb_grid *g, const double *partials, int64_t n, double *out,
                         int *ctr, hipStream_t s);
int launch_reset_ctr(int *ctr, hipStream_t s);

}  // namespace hb
