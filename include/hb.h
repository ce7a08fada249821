/*
 * hb.h -- C ABI of libhb, an MI355X (gfx950) implementation of the
 * harmonic-balance (HB) Navier-Stokes residual and its explicit
 * Runge-Kutta pseudo-time iteration on structured multi-block grids.
 *
 * The problem statement follows the paper (Jackson & Campobasso, COSA):
 * a structured multi-block grid whose blocks meet at "cuts" (orphan
 * paragraph after the Introduction, and the cut pseudo code in
 * §MPI Optimisations), nharms harmonics per block giving the snapshots
 * n = 0..2*nharms, npde = 4 conserved variables per snapshot (state array
 * q(i, j, ipde, n) in the same section), bodies with lift/drag/moment per
 * snapshot (cl(n, ibody), cd(n, ibody), cm(n, ibody), the force reduction
 * in §MPI Optimisations) and Runge-Kutta steps.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - State layout (public, FP64): blocks one after another; within block b
 *    q[n][v][j][i], n = 0..2*N_H, v = (rho, rho u, rho v, rho E), j = 0..nj-1,
 *    i = 0..ni-1 (i fastest) -- the paper's q(i, j, ipde, n) in C order.
 *    hb_state_size() gives the number of doubles.
 *  - Non-dimensionalisation: rho_inf = 1, c_inf = 1, p_inf = 1/gamma,
 *    |V_inf| = mach, reference length l_ref; angles in radians.
 *  - Residual sign: R*_n = R(Q_n) + V (D Q)_n, with R the net outflow of
 *    the cell and D the HB time-derivative matrix; V dQ/dtau = -R*.
 *  - Device pointers: q, r, rbar, qbar, xybar, flowbar, cf, cfbar, resnorm,
 *    forces are device memory owned by the caller (e.g. torch tensors).  They
 *    must not alias each other unless stated.
 *  - Streams: every call enqueues its work on `stream` (a hipStream_t passed
 *    as void*, NULL = the null stream) and returns without synchronising,
 *    except hb_grid_create, hb_grid_destroy and hb_get_status.
 *  - Errors: a negative return code plus a thread-local message from
 *    hb_last_error().  Argument checks run before any device work, so an
 *    HB_ERR_ARG return leaves every buffer untouched.  No C++ exception
 *    crosses this interface.  A grid handle is not thread-safe.
 */
#ifndef HB_H_
#define HB_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hb_grid hb_grid;   /* opaque, owned by libhb */

enum {
    HB_OK = 0,
    HB_ERR_ARG = -1,          /* invalid argument; nothing was done      */
    HB_ERR_DEVICE = -2,       /* a HIP call failed                       */
    HB_ERR_OOM = -3,          /* device allocation failed                */
    HB_ERR_NONFINITE = -4,    /* a non-finite or non-physical state seen */
    HB_ERR_UNSUPPORTED = -5   /* valid request the library does not do   */
};

/* Boundary kinds, per block side (imin, imax, jmin, jmax). */
enum {
    HB_BC_WALL = 1,       /* no-slip adiabatic wall: ghost k mirrors cell k   */
    HB_BC_FARFIELD = 2,   /* both ghost layers = free stream at alpha(t_n)    */
    HB_BC_PERIODIC = 3,   /* the block wraps onto itself (O-grid in i)        */
    HB_BC_CUT = 4,        /* glued to another block side (see hb_cut)         */
    HB_BC_WAKECUT = 5,    /* jmin only: C-grid wake (cells i < wake_ncells and
                             i >= ni - wake_ncells face each other), wall in
                             between                                         */
    HB_BC_CUT_WALL = 6,   /* partly glued: the cells covered by cut segments
                             are glued, the others are a no-slip wall        */
    HB_BC_CUT_FARFIELD = 7 /* partly glued, the others far field             */
};

enum { HB_FP64 = 0, HB_FP32_BULK = 1 };

/* One structured block.  xy is HOST memory, [2][nj+1][ni+1] (x then y,
 * i fastest), right-handed (i along the body, j outward); it is copied by
 * hb_grid_create.  n_harm = N_H in 0..4 (N_s = 2 N_H + 1 snapshots).
 * body_id >= 0 names the body whose loads this block's wall faces carry;
 * bodies are numbered 0..nbody-1 without gaps, and all blocks of one body
 * share n_harm. */
typedef struct {
    int32_t ni, nj;
    int32_t n_harm;
    const double *xy;
    int32_t bc[4];
    int32_t wake_ncells;
    int32_t body_id;
} hb_block;

/* A cut (the paper's "cuts": block edges whose data are exchanged with the
 * neighbouring block every Runge-Kutta step; the paragraph on the MPI
 * parallelisation that follows the Introduction, and the cut pseudo code of
 * §MPI Optimisations, which sends a cut as a sequence of sections along a
 * block's boundary) glues `len` cells of side `side_a` (0..3 = imin, imax,
 * jmin, jmax) of block blk_a, starting at cell start_a along that side, to
 * `len` cells of side side_b of block blk_b starting at start_b: cell
 * start_a + t against start_b + t, or start_b + len - 1 - t when
 * `reversed` is 1.  Positions along a side are j on the i sides, i on the j
 * sides.  Any two sides may be glued (an imax to a jmin, a jmin to a jmin
 * reversed as the wake of a C-grid cut into wake and profile blocks), also
 * sides of one block.  The ghosts of a glued cell are the other block's
 * interior cells (Jacobi: both read the same stage input); corner ghosts
 * take the i sides first, then the j sides, continuing across a cut in the
 * glued block.  Every side of kind HB_BC_CUT must be covered by its
 * segments exactly once; a side of kind HB_BC_CUT_WALL or
 * HB_BC_CUT_FARFIELD at most once (a block edge made of sections, some
 * glued, the rest wall or far field: the C-grid of several blocks whose
 * wake sections and profile sections share a side); glued blocks have
 * equal n_harm.  HB_ERR_ARG
 * otherwise, for a segment outside its sides, len < 1, reversed not 0 or 1,
 * or cuts around which a corner ghost does not resolve. */
typedef struct {
    int32_t blk_a, side_a, start_a;
    int32_t blk_b, side_b, start_b;
    int32_t len, reversed;
} hb_cut;

/* Free stream and forcing.  alpha(t) = alpha0 + alpha_amp sin(omega t),
 * omega = 2 k_red mach / l_ref; snapshot n is at omega t_n = 2 pi n / N_s.
 * mu = mach l_ref / reynolds (constant), Stokes hypothesis, heat flux
 * -mu/((gamma-1) prandtl) grad(gamma p / rho).  (x_mom, y_mom): moment
 * reference point. */
typedef struct {
    double mach, reynolds, prandtl, gamma;
    double alpha0, alpha_amp, k_red, l_ref;
    double x_mom, y_mom;
} hb_flow;

/* Pseudo-time and scheme settings.
 *   cfl, n_stages (1..8), rk_alpha[n_stages]: Q(k) = Q(0) - a_k (dtau/V) R*(Q(k-1))
 *   precision: HB_FP64, or HB_FP32_BULK (flux, source and time step in
 *     FP32; state, update, norms and forces in FP64)
 *   entropy_delta: Harten fix width as a fraction of the Roe sound speed
 *   limiter_eps: van Albada epsilon
 *   batched: 1 = all blocks in one launch per stage (fused tile kernel,
 *     launch configuration from hb_set_tuning / hb_autotune; its halo
 *     loads use 32-bit byte offsets while the state is below 4 GiB and
 *     64-bit element offsets from 4 GiB on); 2 = the same with 64-bit
 *     offsets at any size (the large-state code on small grids); 0 = plain
 *     per-block launches (separate ghost, face-flux and update kernels,
 *     FP64 only)
 *   graph_iters: iterations captured per HIP graph replay (>= 1) */
typedef struct {
    double cfl;
    int32_t n_stages;
    double rk_alpha[8];
    int32_t precision;
    double entropy_delta, limiter_eps;
    int32_t batched, graph_iters;
} hb_solver;

/* Launch configuration of the batched stage kernel (batched = 1).
 *   tile_i:     threads along i per 256-thread workgroup, 16 or 32; the
 *               output tile is tile_i x (256/tile_i - 1) cells
 *   wg_per_cu:  resident workgroups per CU of the persistent grid
 *               (0 = the occupancy maximum; larger values are capped by it;
 *               -1 = no persistent grid, one workgroup per tile)
 *   xcd_order:  1 = renumber workgroups so that the workgroups of one XCD
 *               (one L2) take consecutive tiles (chunks of grid/8 tiles for
 *               a persistent grid, of 32 tiles for one workgroup per tile)
 *   tile_order: 0 = tiles of a block row by row, 1 = column by column
 *   stage_ms:   measured mean stage time (output; 0 when not measured)
 * The tuning changes which workgroup computes which tile, never a cell's
 * arithmetic: states are bitwise identical across tunings with the same
 * tile_i, and equal to rounding in the norm partial order otherwise. */
typedef struct {
    int32_t tile_i, wg_per_cu, xcd_order, tile_order;
    double stage_ms;
} hb_tuning;

/* Rigid motion of the whole grid (the paper's test case 1 is a heaving and
 * pitching wing, Experimental Setup, Test case 1; the moving-grid equations
 * are the arbitrary Lagrangian-Eulerian finite-volume form).  Snapshot n
 * (omega t_n = 2 pi n / N_s) holds the grid rotated counter-clockwise by
 * theta_n about (x_pivot, y_pivot) and raised by h_n:
 *   theta(t) = pitch_amp sin(omega t + pitch_phase),  h(t) = heave_amp sin(omega t)
 * (radians; heave in grid length units, +y).  Faces carry the flux
 * F.S - (x_t.S) U with the rigid grid velocity x_t at the face midpoint and
 * Roe eigenvalues relative to the face; no-slip walls move with the grid
 * (ghost velocity 2 u_wall - u); the local step uses the velocity relative
 * to the grid; loads are taken on the moved grid with the moment about the
 * reference point carried by the body, lift and drag along alpha0.
 * hb_td_march moves the grid continuously (the motion at each stage time). */
typedef struct {
    double pitch_amp, pitch_phase, heave_amp, x_pivot, y_pivot;
} hb_motion;

/* Build a grid (the paper's problem statement: a structured multi-block
 * grid whose blocks meet at cuts, the paragraph on the MPI parallelisation
 * after the Introduction; N_H harmonics per block, the nharms of the
 * §MPI Optimisations pseudo code, whose snapshots n = 0..2*nharms each
 * carry npde = 4 variables): copies the host arrays, computes the metrics on the device
 * (FP64), allocates all scratch.  Validation (HB_ERR_ARG): nblocks >= 1,
 * ni, nj >= 4, n_harm in [0, 4], known boundary kinds, wake_ncells in
 * [0, ni/2] and only with a WAKECUT jmin, cut sides consistent, bodies
 * numbered without gaps with one n_harm each, every cell area > 0.
 * At most 2^24 cells per block (HB_ERR_ARG otherwise).  Synchronises the current device.  *out is
 * NULL on failure. */
int hb_grid_create(const hb_block *blocks, int32_t nblocks, const hb_cut *cuts,
                   int32_t ncuts, const hb_flow *flow, const hb_solver *solver,
                   hb_grid **out);

/* Free everything hb_grid_create allocated (synchronises).  NULL is a no-op. */
int hb_grid_destroy(hb_grid *g);

/* Doubles in the state: sum over blocks of N_s * 4 * nj * ni.  -1 if g is NULL. */
int64_t hb_state_size(const hb_grid *g);

/* Doubles in a force array: 3 * sum over bodies of N_s(body); -1 if NULL. */
int64_t hb_forces_size(const hb_grid *g);

/* Doubles in the node-coordinate array: sum over blocks 2 (nj+1)(ni+1). */
int64_t hb_xy_size(const hb_grid *g);

/* r = R*(q), the HB residual of every cell and snapshot (public layout):
 * the operator that the paper's Runge-Kutta step (§MPI Optimisations)
 * evaluates over all blocks and harmonics after the cut (halo) exchange.
 * The paper does not print its formula (its HB-formulation section is
 * missing); here R*_n = R(Q_n) + V (D Q)_n with R the net MUSCL/Roe inviscid
 * minus central viscous face flux of the cell and D the time-collocation
 * spectral derivative over the N_s snapshots.
 * q, r: device, hb_state_size() doubles each, must not overlap. */
int hb_residual(hb_grid *g, const double *q, double *r, void *stream);

/* n_iter pseudo-time iterations in place on q (device, public layout): the
 * paper's Runge-Kutta steps (§MPI Optimisations: each step exchanges the cut
 * halos and reduces the loads of every body and harmonic once), here the
 * four-stage scheme Q(k) = Q(0) - a_k (dtau/V) R*(Q(k-1)) with the local
 * pseudo-time step dtau of each cell and snapshot (coefficients and step
 * are not given in the paper; hb_solver sets them).
 * resnorm (device, n_iter doubles, may be NULL): RMS of R*_rho / V over all
 * cells and snapshots at the first stage of each iteration.
 * forces (device, hb_forces_size() doubles, may be NULL): cl, cd, cm of the
 * final state, layout [body][n][3].
 * Non-finite states are flagged in a device status word, read by
 * hb_get_status(). */
int hb_rk_iterate(hb_grid *g, double *q, int32_t n_iter, double *resnorm,
                  double *forces, void *stream);

/* The loads of the paper's force reduction (§MPI Optimisations: cl, cd and
 * cm of every body and harmonic, gathered into one buffer and reduced once
 * per Runge-Kutta step; the paper packs it harmonic-major, here it is
 * body-major because bodies may differ in N_s):
 * cf = (cl, cd, cm) per body and snapshot, layout [body][n][3] (bodies in
 * id order, each with its own N_s); drag along the mean free stream
 * (cos alpha0, sin alpha0), lift normal to it, cm positive nose-up, all on
 * q_inf = mach^2/2 and l_ref.  Wall faces: -(p_w - p_inf) S + tau.S with
 * p_w the adjacent cell's pressure.  FP64. */
int hb_forces(hb_grid *g, const double *q, double *cf, void *stream);

/* Reverse-mode (Jacobian-transpose) products of the residual R* = hb_residual.
 * The paper does not define or use an adjoint; this is the transpose of the
 * linearisation of hb_residual's operator, for gradients of HB-averaged loads
 * with respect to grid and flow parameters:
 *   qbar    = J_Q^T rbar,  J_Q = d R* / d Q        (state size, overwritten)
 *   xybar   = J_X^T rbar,  X = node coordinates    (hb_xy_size(), may be NULL)
 *   flowbar = J_a^T rbar,  a = alpha0              (1 double, may be NULL)
 * The reconstruction is recomputed, nothing is stored between calls.
 * FP64 only (HB_ERR_UNSUPPORTED for an FP32-bulk grid).  With a motion set
 * (hb_set_motion) the products are those of the moving-grid R* (snapshot
 * n's rotated face vectors, face speeds, moving-wall images), the motion
 * held fixed; xybar is then the adjoint of the body-frame nodes (through
 * the face vectors, the face speeds and the wall velocities).  The adjoints'
 * scratch (the inverse ghost map, per-face adjoint terms: 26 doubles per
 * face and snapshot) is allocated by the first adjoint call unless
 * hb_prepare allocated it before. */
int hb_residual_adjoint(hb_grid *g, const double *q, const double *rbar,
                        double *qbar, double *xybar, double *flowbar, void *stream);

/* Reverse-mode products of the force coefficients of hb_forces (the
 * paper's per-body, per-snapshot cl/cd/cm, §MPI Optimisations, force
 * reduction): with cfbar of the hb_forces layout (device), qbar (device,
 * state size), xybar (device, hb_xy_size(), may be NULL) and flowbar
 * (device, 1 double: d/d alpha0, may be NULL) receive (d cf / d .)^T cfbar,
 * overwritten.  Only wall faces contribute; alpha0 enters through the wind
 * axes and the far-field ghosts.  FP64 arithmetic on any grid.  qbar must
 * not alias q.  With a motion set: the moving-grid loads of hb_forces
 * (xybar: body-frame nodes, the moment arm rotating with the body). */
int hb_forces_adjoint(hb_grid *g, const double *q, const double *cfbar,
                      double *qbar, double *xybar, double *flowbar, void *stream);

/* Adjoint pseudo-time iteration at a fixed (converged) state q: n_iter
 * iterations in place on lambda of
 *   lambda(k) = lambda(0) - a_k (dtau/V) (J_Q^T lambda(k-1) + gq),
 * the multistage scheme of hb_rk_iterate (the paper's Runge-Kutta step,
 * §MPI Optimisations) with the same coefficients and the same local steps
 * dtau(q), so it converges as the forward iteration does, to
 * J_Q^T lambda = -gq.  With gq = (dJ/dQ)^T of an objective J, the total
 * derivative of J at a steady state is dJ/dX + lambda^T (d R* / d X) (X = node
 * coordinates or alpha0: hb_residual_adjoint with rbar = lambda).
 * q, gq: device, state size, read only; lambda: device, state size, in/out
 * (must alias neither); resnorm (device, n_iter doubles, may be NULL): RMS
 * over cells, snapshots and variables of (J_Q^T lambda + gq)/V at the first
 * stage of each iteration.  FP64 grids only (HB_ERR_UNSUPPORTED otherwise).
 * With a motion set: the moving-grid products and local steps.
 * Scratch of 2.25 state sizes (and the adjoints' own) is allocated on the
 * first call unless hb_prepare allocated it before. */
int hb_adjoint_iterate(hb_grid *g, const double *q, double *lambda, const double *gq,
                       int32_t n_iter, double *resnorm, void *stream);

/* Scratch that the calls below allocate on their first use, allocated now
 * (synchronously, on the grid's device), so that the later calls allocate
 * nothing: for callers that enqueue them into a HIP graph capture or a
 * serving loop.  The paper defines no such call (it has no device
 * allocator).  what: a bitwise OR of
 *   HB_PREPARE_ADJOINT          hb_residual_adjoint, hb_forces_adjoint
 *   HB_PREPARE_ADJOINT_ITERATE  hb_adjoint_iterate (includes the above;
 *                               FP64 grids only, HB_ERR_UNSUPPORTED otherwise)
 *   HB_PREPARE_TD               hb_td_march
 * Scratch already allocated is kept.  HB_ERR_ARG for NULL or unknown bits,
 * HB_ERR_OOM when the device memory runs out (what was allocated stays
 * with the grid). */
enum {
    HB_PREPARE_ADJOINT = 1,
    HB_PREPARE_ADJOINT_ITERATE = 2,
    HB_PREPARE_TD = 4
};
int hb_prepare(hb_grid *g, int32_t what);

/* Restart files (the paper's aggregated output of all blocks and harmonics,
 * §MPI Optimisations, the part on MPI I/O): hb_save_state writes the whole state q (device,
 * state size) and the caller's iteration counter to `path` in one write
 * (header with a workload signature and the block table, the state in the
 * public layout, a checksum; written to path.tmp, then renamed).
 * hb_load_state reads such a file into q (device) and *iteration (may be
 * NULL); HB_ERR_ARG for a missing file, another workload (signature, block
 * sizes, N_H or boundary kinds differ) or a checksum mismatch.  Both
 * synchronise `stream`. */
int hb_save_state(hb_grid *g, const double *q, int64_t iteration, const char *path, void *stream);
int hb_load_state(hb_grid *g, double *q, int64_t *iteration, const char *path, void *stream);

/* Solution files, one per snapshot (the paper writes one solution file per
 * real harmonic at the end of a run, beside the restart file, and makes
 * each an aggregated parallel write, §MPI Optimisations, the part on MPI
 * I/O): for k = 0 .. max N_s - 1, `<prefix>.snap<k>` holds, in one write,
 * every block with more than k snapshots: its nodes at snapshot k (moved by
 * the rigid motion when one is set) and the primitives (rho, u, v, p) of
 * its cells at snapshot k.  Layout (little endian):
 *   char[8] "HBSOLN01", int32 k, int32 number of blocks in the file,
 *   per block: int32 block index, ni, nj, n_harm; double phase
 *     omega t_k = 2 pi k / N_s; double x[nj+1][ni+1], y[nj+1][ni+1];
 *     double rho[nj][ni], u[nj][ni], v[nj][ni], p[nj][ni],
 *   uint64 FNV-1a of every byte after the magic.
 * q: device, state size.  Each file is written to `<file>.tmp` and renamed.
 * Allocates (and frees) a device staging buffer of the records of all
 * blocks and snapshots; synchronises `stream`.  HB_ERR_ARG for NULL or an
 * empty prefix or a file that cannot be written. */
int hb_save_solution(hb_grid *g, const double *q, const char *prefix, void *stream);

/* Time-domain march: the time-domain counterpart of the HB system (the
 * paper's code solves unsteady flows in the time domain as well as by HB,
 * §Introduction).  n_steps classical fourth-order Runge-Kutta steps of size
 * dt in physical time on V dQ/dt = -R(Q, t), from time t0, with the far
 * field at the instantaneous incidence alpha(t) = alpha0 + alpha_amp
 * sin(omega t); R is the grid's residual path (batched or per-block, FP64
 * or FP32 bulk), the stage combinations FP64.  Grids with n_harm = 0 in
 * every block only (one snapshot per cell; HB_ERR_UNSUPPORTED otherwise).
 * q: device, state size, advanced in place.  dt > 0 is the caller's
 * (stability needs dt below about the smallest local step at CFL 1).
 * Allocates three state-size scratch buffers on the first call, unless
 * hb_prepare allocated them before. */
int hb_td_march(hb_grid *g, double *q, double t0, double dt, int32_t n_steps, void *stream);

/* hb_td_march for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same march, bit for bit, with its three state-size scratch arrays
 * (residual, stage accumulator, stage state) taken from a static device
 * array of 3 x 2^21 doubles (48 MiB) that each GPU the library runs on
 * holds until the process ends, instead of buffers allocated on the first
 * call.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); the grid's own buffers come from hb_grid_create.
 * HB_ERR_ARG when the state exceeds 2^21 doubles (a 1024 x 512 block with
 * n_harm = 0 fits exactly), besides hb_td_march's own checks.  Every call on one GPU shares that GPU's array and may leave any
 * contents in it: calls that overlap on one GPU (several streams or host
 * threads) race and must be serialised by the caller. */
int hb_td_march_noalloc(hb_grid *g, double *q, double t0, double dt, int32_t n_steps,
                        void *stream);

/* Autotune the batched stage kernel (the paper's per-block work, batched
 * over blocks of uneven size and N_H in one launch per Runge-Kutta step,
 * §MPI Optimisations): with cache_path (may be NULL) holding an entry for
 * this device and workload and force = 0, apply it; otherwise time every
 * candidate (tile_i in {16, 32} x tile_order in {0, 1} x xcd_order in
 * {1, 0} x wg_per_cu in {max, 2, 1, -1}) over full pseudo-time iterations on a
 * scratch copy of q (device, state size, not modified), apply the fastest
 * and, with cache_path, store it (JSON, one entry per device/workload key).
 * out (host, may be NULL) receives the applied tuning.  Synchronises;
 * allocates one state-size scratch buffer for the duration of the call.
 * HB_ERR_UNSUPPORTED for a grid with batched = 0. */
int hb_autotune(hb_grid *g, const double *q, const char *cache_path, int32_t force,
                hb_tuning *out, void *stream);

/* Apply (synchronises; a tile change rebuilds the tile list) or read the
 * tuning of a batched grid. */
int hb_set_tuning(hb_grid *g, const hb_tuning *t);
int hb_get_tuning(const hb_grid *g, hb_tuning *t);

/* Replace the node coordinates (device, hb_xy_size() doubles, same layout as
 * the blocks' xy, concatenated) and recompute the metrics on `stream`.  On
 * a moving grid (hb_set_motion) these are the body-frame nodes. */
int hb_set_xy(hb_grid *g, const double *xy, void *stream);

/* Replace the mean incidence alpha0 (radians); takes effect for work
 * enqueued afterwards. */
int hb_set_alpha0(hb_grid *g, double alpha0);

/* Set (m non-NULL with a non-zero amplitude) or clear (NULL, or both
 * amplitudes zero) the rigid grid motion described at hb_motion.  It then
 * applies to hb_residual, hb_rk_iterate, hb_forces and hb_td_march, on the
 * per-block and on the batched path (FP64 and FP32 bulk), and to the
 * adjoints (FP64).
 * HB_ERR_UNSUPPORTED for blocks with walls on an i side (also the wall rest
 * of a partly glued i side); any cuts.  hb_set_xy then sets the body-frame
 * nodes, and the adjoints take the motion.  A moving-wall image takes the
 * velocity of the wall face at which its ghost's resolution mirrors (for a
 * corner ghost across a cut, the glued block's wall face).
 * HB_ERR_ARG for non-finite values.  Drops the batched path's captured
 * iterations (the next hb_rk_iterate captures them again).  Synchronises
 * the current device. */
int hb_set_motion(hb_grid *g, const hb_motion *m);

/* Synchronise and return HB_ERR_NONFINITE if any iteration since the last
 * call met a non-finite residual or a non-positive density or pressure
 * (the flag is then cleared), else HB_OK. */
int hb_get_status(hb_grid *g);

/* Instrumentation for benchmarks.  With enable = 1, hb_rk_iterate runs its
 * stages one launch at a time (no graph replay) and brackets each stage's
 * kernel launches with a pair of HIP events recorded on the caller's stream.
 * hb_stage_stats synchronises on the last event, returns the summed
 * elapsed milliseconds of all bracketed stages and their number since the
 * previous call, and resets both.  Either pointer may be NULL. */
int hb_profile_stages(hb_grid *g, int32_t enable);
int hb_stage_stats(hb_grid *g, double *total_ms, int64_t *stages);

/* Message of the last error on this thread ("" if none). */
const char *hb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HB_H_ */
