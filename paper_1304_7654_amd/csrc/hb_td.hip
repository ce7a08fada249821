// Time-domain march on the GPU: the time-domain counterpart of the HB
// system (the paper's code has both an HB and a time-domain unsteady solver,
// §Introduction and the description of COSA).  Classical fourth-order
// Runge-Kutta in physical time on V dQ/dt = -R(Q, t) for grids with one
// snapshot per cell (N_H = 0 in every block, so the HB source vanishes),
// with the far field at the instantaneous incidence
// alpha(t) = alpha0 + alpha_amp sin(omega t):
//   k_s = -R(Q_s, t + c_s dt) / V,  c = (0, 1/2, 1/2, 1),
//   Q_1 = Q + dt/2 k_0,  Q_2 = Q + dt/2 k_1,  Q_3 = Q + dt k_2,
//   Q <- Q + dt/6 (k_0 + 2 k_1 + 2 k_2 + k_3).
// Every residual is the grid's own residual path (batched or per-block,
// FP64 or FP32 bulk); the stage combinations are FP64.  On a moving grid
// (plain path) the motion table is set to the rigid motion at each stage
// time, as the far field is, and the cell areas stay constant.
#include <mutex>

#include "hb_device.hpp"

namespace hb {
namespace {

// Scratch of the allocation-free march (hb_td_march_noalloc): the residual,
// the stage accumulator and the stage state, three state-size arrays, in a
// file-scope device array that each GPU holds for the life of the process.
// In host code `scratch` names a host-side stand-in, never the device
// memory: host code uses only the address hipGetSymbolAddress returns for
// the device (scratch_address below).  Every call on one GPU shares that
// GPU's array, so calls that overlap on one GPU race.
constexpr int64_t kTdScratchDoubles = 3 * ((int64_t)1 << 21);   // 48 MiB
static __device__ __align__(256) double scratch[kTdScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};

// device address of `scratch` on device `dev`, looked up once per device
// with that device current
int scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HB_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        int cur = 0;
        int rc = check_hip(hipGetDevice(&cur), "hipGetDevice");
        if (!rc && cur != dev) rc = check_hip(hipSetDevice(dev), "hipSetDevice");
        void *p = nullptr;
        if (!rc) rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (cur != dev) {
            const int rc2 = check_hip(hipSetDevice(cur), "hipSetDevice");
            rc = rc ? rc : rc2;
        }
        if (rc) return rc;
        g_scratch_addr[dev] = (double *)p;
    }
    *out = g_scratch_addr[dev];
    return HB_OK;
}

constexpr int kBS = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

// far-field tables of every snapshot at incidence alpha (one snapshot per
// block here, so D Q_inf = 0 stays as uploaded)
__global__ void k_set_far_field(int n_snap, double mach, double gamma, double alpha, double *ffw_d,
                                double *ffq_d, float *ffw_f, float *ffq_f) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_snap) return;
    const double u = mach * cos(alpha), v = mach * sin(alpha), p = 1.0 / gamma;
    const double w[4] = {1.0, u, v, p};
    const double q[4] = {1.0, u, v, p / (gamma - 1.0) + 0.5 * (u * u + v * v)};
    for (int c = 0; c < 4; ++c) {
        ffw_d[4 * k + c] = w[c];
        ffq_d[4 * k + c] = q[c];
        ffw_f[4 * k + c] = (float)w[c];
        ffq_f[4 * k + c] = (float)q[c];
    }
}

// motion table of every snapshot at one time (one snapshot per block here)
__global__ void k_set_motion(int n_snap, double c, double s, double thd, double h, double hd,
                             double *tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_snap) return;
    double *t = tab + (int64_t)kMotionW * k;
    t[0] = c;
    t[1] = s;
    t[2] = thd;
    t[3] = h;
    t[4] = hd;
}

// stage s of one block: acc (+)= w_s R; s < 3: Qs = Q - a_s dt R / V;
// s = 3: Q <- Q - dt/6 acc / V
__global__ void k_td_stage(const BlockDesc *blks, int b, double *q, const double *r, double *acc,
                           double *qs, const double *V, int s, double dt) {
    const BlockDesc &B = blks[b];
    const int64_t plane = (int64_t)B.ni * B.nj;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= plane) return;
    const double iv = 1.0 / V[B.cell_off + t];
    const double ws = (s == 0 || s == 3) ? 1.0 : 2.0;
    const double as = s == 2 ? 1.0 : 0.5;
    for (int v = 0; v < 4; ++v) {
        const int64_t o = B.q_off + (int64_t)v * plane + t;
        const double rv = r[o];
        const double av = (s == 0 ? 0.0 : acc[o]) + ws * rv;
        if (s < 3) {
            acc[o] = av;
            qs[o] = q[o] - as * dt * rv * iv;
        } else {
            q[o] = q[o] - (dt / 6.0) * av * iv;
        }
    }
}

int set_far_field(hb_grid *g, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_set_far_field, dim3(nblk(g->n_snap)), dim3(kBS), 0, s, (int)g->n_snap,
                       g->flow.mach, g->flow.gamma, alpha, g->ffw_d, g->ffq_d, g->ffw_f, g->ffq_f);
    return check_hip(hipGetLastError(), "far-field launch");
}

// rigid motion at time t: theta = A sin(omega t + phi), h = A_h sin(omega t)
int set_motion_at(hb_grid *g, double omega, double t, hipStream_t s) {
    const hb_motion &m = g->motion_par;
    const double th = m.pitch_amp * sin(omega * t + m.pitch_phase);
    hipLaunchKernelGGL(k_set_motion, dim3(nblk(g->n_snap)), dim3(kBS), 0, s, (int)g->n_snap, cos(th),
                       sin(th), omega * m.pitch_amp * cos(omega * t + m.pitch_phase),
                       m.heave_amp * sin(omega * t), omega * m.heave_amp * cos(omega * t), g->mot_d);
    return check_hip(hipGetLastError(), "motion launch");
}

int residual_any(hb_grid *g, const double *q, double *r, hipStream_t s) {
    return g->solver.batched ? fused_residual(g, q, r, s) : plain_residual(g, q, r, s);
}

// the march with caller-chosen scratch: r, acc, qs of n_state doubles each
int td_march(hb_grid *g, double *q, double t0, double dt, int n_steps, double *r, double *acc,
             double *qs, hipStream_t s) {
    const double omega = 2.0 * g->flow.k_red * g->flow.mach / g->flow.l_ref;
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
    int rc = HB_OK;
    for (int it = 0; it < n_steps && !rc; ++it) {
        const double t = t0 + dt * it;
        for (int st = 0; st < 4 && !rc; ++st) {
            const double ts = t + c[st] * dt;
            rc = set_far_field(g, g->flow.alpha0 + g->flow.alpha_amp * sin(omega * ts), s);
            if (!rc && g->motion.tab) rc = set_motion_at(g, omega, ts, s);
            rc = rc ? rc : residual_any(g, st == 0 ? q : qs, r, s);
            for (int b = 0; b < g->nblocks && !rc; ++b) {
                const BlockDesc &B = g->blk[b];
                hipLaunchKernelGGL(k_td_stage, dim3(nblk((int64_t)B.ni * B.nj)), dim3(kBS), 0, s, g->blk_d,
                                   b, q, r, acc, qs, g->V_d, st, dt);
            }
        }
    }
    // the grid's own snapshot (phase 0) far field and motion again
    int rc2 = set_far_field(g, g->flow.alpha0, s);
    if (!rc2 && g->motion.tab) rc2 = set_motion_at(g, omega, 0.0, s);
    rc = rc ? rc : rc2;
    return rc ? rc : check_hip(hipGetLastError(), "td launch");
}

}  // namespace

int td_prepare(hb_grid *g) {
    if (g->td_r_d) return HB_OK;
    int rc = check_hip(hipMalloc((void **)&g->td_r_d, sizeof(double) * g->n_state), "td alloc");
    rc = rc ? rc : check_hip(hipMalloc((void **)&g->td_acc_d, sizeof(double) * g->n_state), "td alloc");
    rc = rc ? rc : check_hip(hipMalloc((void **)&g->td_qs_d, sizeof(double) * g->n_state), "td alloc");
    return rc;
}

int launch_td_march(hb_grid *g, double *q, double t0, double dt, int n_steps, hipStream_t s) {
    const int rc = td_prepare(g);
    if (rc) return rc;
    return td_march(g, q, t0, dt, n_steps, g->td_r_d, g->td_acc_d, g->td_qs_d, s);
}

int launch_td_march_noalloc(hb_grid *g, double *q, double t0, double dt, int n_steps,
                            hipStream_t s) {
    if (3 * g->n_state > kTdScratchDoubles)
        return fail(HB_ERR_ARG, "hb_td_march_noalloc: the state (" + std::to_string(g->n_state) +
                                    " doubles) exceeds the static scratch of " +
                                    std::to_string(kTdScratchDoubles / 3) + " doubles per state copy");
    double *base = nullptr;
    const int rc = scratch_address(g->device, &base);
    if (rc) return rc;
    return td_march(g, q, t0, dt, n_steps, base, base + g->n_state, base + 2 * g->n_state, s);
}

}  // namespace hb
