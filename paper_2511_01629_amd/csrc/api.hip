// api.hip -- host side of the C ABI declared in include/lbm.h.
//
// The context owns (or carves from the caller's workspace) every device
// buffer: two population buffers [Q][N] in the storage type, the uint16
// owner map, the solid-node velocity [d][N] (FP64), a staging area of 4N
// doubles for transfers, device flags and the particle arrays.  A step queues
// three kernels on the context stream: the fused stream-collide-penalize
// update, the per-particle sums (which also clear the indicator), and
// Algorithm 1 with the rasterisation of the new indicator.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_set>
#include <vector>

#include "ctx.h"
#include "lattice.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;

// message of the last lbm_workspace_size / lbm_create failure on this thread
thread_local std::string g_create_err = "no error";
constexpr int PART_DOUBLES = 3 * 7 + 1 + 4 + 3 + 3 + 3 * 5 + 1 + 1 + 4; // X Xn U W Uprev Wprev A, theta, rho a b C, acc, Unext, Ub Y Ys Y2 Dc, dth, Nw, geo
constexpr double CS2 = 1.0 / 3.0;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int storage_bytes(int s) { return s == LBM_F64 ? 8 : s == LBM_F32 ? 4 : 2; }

// Sizes of the slot tables of the fused-sums step (K = 1): per-particle
// tables keyed by the wrapped row and the wavefront index (slot_of).  A scan
// box spans at most ext = ceil(2a) + 7 nodes per axis; the key sizes are
// powers of two at least that many rows and wavefronts, and on a periodic
// axis must divide the period (or cover it), so that no two rows or
// wavefronts of a box share a slot; on a periodic x axis a box must also stay
// 63 nodes short of the period, so that a wavefront never holds nodes of two
// images of one box.  Returns false where the sizes cannot be met (the
// momentum sums then run as a kernel of their own).
struct SlotSizes {
    int Mx, My, Mz;
    int64_t stride;
    size_t bytes; // for `cap` particles
};
bool slot_sizes(const int n[3], const int per[3], int d, int ext, int cap, SlotSizes &z)
{
    auto pow2 = [](int v) {
        int q = 1;
        while (q < v) q <<= 1;
        return q;
    };
    const int wn = (n[0] + 63) / 64;
    const int kwn = std::min(wn, (ext + 62) / 64 + 1 + (per[0] && n[0] % 64 ? 1 : 0));
    z.Mx = pow2(kwn);
    z.My = pow2(ext);
    z.Mz = d == 3 ? pow2(ext) : 1;
    auto axis_ok = [&](int p, int len, int M) { return !p || (ext <= len && (len % M == 0 || M >= len)); };
    bool ok = axis_ok(per[1], n[1], z.My) && (d == 2 || axis_ok(per[2], n[2], z.Mz));
    ok = ok && (!per[0] || (ext + 63 <= n[0] && (wn % z.Mx == 0 || z.Mx >= wn)));
    z.stride = (int64_t)z.Mx * z.My * z.Mz;
    z.bytes = (size_t)cap * (size_t)z.stride * slot_width(d) * sizeof(double);
    const bool coords = n[0] < (1 << 21) && n[1] < (1 << 21) && n[2] < (1 << 21); // packed first nodes
    return ok && coords && z.stride <= 65536 && z.bytes <= ((size_t)1 << 30);
}

struct Layout {
    size_t f0, f1, owner, usol, staging, flags, wall, pd, pf, pi, slots, slots_bytes, total;
};

Layout layout_for(const lbm_config *cfg, int Q, int d, int64_t N)
{
    Layout L;
    size_t off = 0;
    const size_t fbytes = align_up((size_t)Q * N * storage_bytes(cfg->storage));
    const int cap = std::max(cfg->max_particles, 1);
    L.f0 = off;
    off += fbytes;
    L.f1 = off;
    off += fbytes;
    L.owner = off;
    off += align_up((size_t)((N + 1) / 2 * 2) * sizeof(uint16_t));
    L.usol = off;
    off += align_up((size_t)d * N * sizeof(double));
    L.staging = off;
    off += align_up((size_t)4 * N * sizeof(double));
    L.flags = off;
    off += ALIGN;
    L.wall = off;
    off += align_up(2 * 19 * sizeof(double));
    L.pd = off;
    off += align_up((size_t)cap * PART_DOUBLES * sizeof(double));
    L.pf = off;
    off += align_up((size_t)cap * 3 * sizeof(float));
    L.pi = off;
    off += align_up((size_t)cap * 8 * sizeof(int32_t));
    // the slot tables for bodies up to max_radius, when it is given (else the
    // library allocates them at lbm_set_particles)
    L.slots = off;
    L.slots_bytes = 0;
    if (cfg->max_radius > 0 && cfg->K == 1 && !(cfg->rigid_beta > 0) && !cfg->fractional_indicator) {
        const int n[3] = {cfg->n[0], cfg->n[1], d == 3 ? cfg->n[2] : 1};
        const int per[3] = {cfg->periodic[0] != 0, cfg->periodic[1] != 0, d == 3 && cfg->periodic[2] != 0};
        SlotSizes z;
        if (slot_sizes(n, per, d, (int)ceil(2.0 * cfg->max_radius) + 7, cap, z)) {
            L.slots_bytes = align_up(z.bytes);
            off += L.slots_bytes;
        }
    }
    L.total = off;
    return L;
}

int fail(lbm_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hipfail(lbm_ctx *c, hipError_t e, const char *what)
{
    return fail(c, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                                                                                \
    do {                                                                                                               \
        hipError_t e_ = (expr);                                                                                        \
        if (e_ != hipSuccess) return hipfail((c), e_, #expr);                                                          \
    } while (0)

int validate_cfg(const lbm_config *cfg, std::string &why, int &Q, int &d, int64_t &N)
{
    if (!cfg) return why = "cfg is NULL", LBM_EINVAL;
    if (cfg->lattice != LBM_D2Q9 && cfg->lattice != LBM_D3Q19) return why = "unknown lattice", LBM_EINVAL;
    if (cfg->storage < LBM_F64 || cfg->storage > LBM_BF16) return why = "unknown storage", LBM_EINVAL;
    Q = cfg->lattice == LBM_D2Q9 ? 9 : 19;
    d = cfg->lattice == LBM_D2Q9 ? 2 : 3;
    int n[3] = {cfg->n[0], cfg->n[1], d == 3 ? cfg->n[2] : 1};
    for (int k = 0; k < 3; ++k)
        if (n[k] <= 0) return why = "lattice sizes must be positive", LBM_EINVAL;
    N = (int64_t)n[0] * n[1] * n[2];
    // node indices and the [d][N] solid-velocity field use 32-bit offsets;
    // population offsets q N + node switch to 64 bits when Q N >= 2^31
    if ((int64_t)d * N >= ((int64_t)1 << 31)) return why = "d*N must stay below 2^31", LBM_EINVAL;
    if (!(cfg->tau > 0.5)) return why = "tau must exceed 1/2", LBM_EINVAL;
    if (cfg->alpha > 1.0 / cfg->tau * (1.0 + 1e-12)) return why = "alpha must not exceed 1/tau", LBM_EINVAL;
    if (cfg->max_particles < 0 || cfg->max_particles > 65534) return why = "max_particles out of range", LBM_EINVAL;
    if (cfg->K < 1) return why = "K must be >= 1", LBM_EINVAL;
    if (!(cfg->rho_f > 0)) return why = "rho_f must be positive", LBM_EINVAL;
    if (cfg->eps_p <= 0 || cfg->eps_w <= 0 || cfg->delta <= 0) return why = "eps_p, eps_w, delta must be positive", LBM_EINVAL;
    if (!(cfg->rigid_beta >= 0.0 && cfg->rigid_beta <= 1.0)) return why = "rigid_beta must lie in [0, 1]", LBM_EINVAL;
    if (!(cfg->max_radius >= 0.0 && cfg->max_radius < 1e6)) return why = "max_radius must be >= 0 and finite", LBM_EINVAL;
    if (cfg->fractional_indicator && cfg->rigid_beta > 0)
        return why = "the fractional indicator is not defined with the rigid-velocity forcing", LBM_EINVAL;
    // moving walls: one axis (y, or z in 3D), tangential, every other axis periodic
    int wall_axis = 0;
    for (int k = 0; k < 3; ++k)
        for (int s = 0; s < 2; ++s)
            for (int j = 0; j < 3; ++j) {
                const double v = cfg->wall_velocity[k][s][j];
                if (v == 0.0) continue;
                if (!isfinite(v)) return why = "wall velocities must be finite", LBM_EINVAL;
                if (k == 0 || k >= d) return why = "moving walls only on the y axis (or the z axis in 3D)", LBM_EINVAL;
                if (cfg->periodic[k]) return why = "a moving wall needs a wall axis, not a periodic one", LBM_EINVAL;
                if (j == k) return why = "wall velocities must be tangential to the wall", LBM_EINVAL;
                if (wall_axis && wall_axis != k) return why = "moving walls on one axis only", LBM_EINVAL;
                wall_axis = k;
            }
    for (int k = 0; wall_axis && k < d; ++k)
        if (k != wall_axis && !cfg->periodic[k])
            return why = "with moving walls every other axis must be periodic", LBM_EINVAL;
    return LBM_OK;
}

// The axis of the moving walls (validated above) and, per side and
// population, what a population pulled from behind that wall gains:
// 2 w_q (c_q . u_w)/cs^2, the difference of the equilibria of eq. (13) at
// the wall velocity.
template <class L> void wall_terms(const lbm_config *cfg, StepParams &sp, double tab[2][19])
{
    sp.wall_axis = 0;
    for (int k = 1; k < L::D; ++k)
        for (int s = 0; s < 2; ++s)
            for (int j = 0; j < 3; ++j)
                if (cfg->wall_velocity[k][s][j] != 0.0) sp.wall_axis = k;
    for (int s = 0; s < 2; ++s)
        for (int q = 0; q < 19; ++q) {
            tab[s][q] = 0.0;
            if (!sp.wall_axis || q >= L::Q) continue;
            const int c[3] = {L::cx[q], L::cy[q], L::cz[q]};
            double cu = 0.0;
            for (int j = 0; j < L::D; ++j) cu += c[j] * cfg->wall_velocity[sp.wall_axis][s][j];
            tab[s][q] = 2.0 * L::w[q] * cu / CS2;
        }
}

void feq_host(int lattice, double p, const double u[3], double *out)
{
    // eq. (13), evaluated once on the host for the uniform initial state
    static const int c9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    const int Q = lattice == LBM_D2Q9 ? 9 : 19;
    const double w0 = lattice == LBM_D2Q9 ? 4.0 / 9 : 1.0 / 3;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        int c[3];
        if (lattice == LBM_D2Q9) {
            for (int k = 0; k < 3; ++k) c[k] = c9[q][k];
        } else {
            for (int k = 0; k < 3; ++k) c[k] = 0;
            if (q >= 1 && q <= 6) c[(q - 1) / 2] = (q % 2) ? 1 : -1;
            if (q >= 7) {
                static const int ax[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                static const int sg[4][2] = {{1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
                const int e = q - 7;
                c[ax[e / 4][0]] = sg[e % 4][0];
                c[ax[e / 4][1]] = sg[e % 4][1];
            }
        }
        const int s = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        const double w = lattice == LBM_D2Q9 ? (s == 0 ? 4.0 / 9 : s == 1 ? 1.0 / 9 : 1.0 / 36)
                                             : (s == 0 ? 1.0 / 3 : s == 1 ? 1.0 / 18 : 1.0 / 36);
        const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        out[q] = q == 0 ? -(1 - w0) * p / CS2 - w0 * uu / (2 * CS2)
                        : w * (p / CS2 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2));
    }
}

void carve(lbm_ctx *c, const Layout &L)
{
    char *base = (char *)c->ws;
    c->f[0] = c->fws[0] = base + L.f0;
    c->f[1] = c->fws[1] = base + L.f1;
    c->owner = (uint16_t *)(base + L.owner);
    c->usol = (double *)(base + L.usol);
    c->staging = (double *)(base + L.staging);
    c->wall_tab = (double *)(base + L.wall);
    c->sp.wall_tab = c->wall_tab;
    c->flags = (int32_t *)(base + L.flags);
    const int cap = c->cap;
    double *pd = (double *)(base + L.pd);
    auto take = [&](int per) {
        double *p = pd;
        pd += (size_t)cap * per;
        return p;
    };
    c->P.X = take(3);
    c->P.Xn = take(3);
    c->P.theta = take(1);
    c->P.U = take(3);
    c->P.W = take(3);
    c->P.Uprev = take(3);
    c->P.Wprev = take(3);
    c->P.A = take(3);
    c->P.rho_s = take(1);
    c->P.a = take(1);
    c->P.b = take(1);
    c->P.Cc = take(1);
    c->P.acc_d = take(3);
    c->P.Unext = take(3);
    c->P.Y = take(3);
    c->P.Ys = take(3);
    c->P.Y2 = take(3);
    c->P.Ub = take(3);
    c->P.Dc = take(3);
    c->P.dth = take(1);
    c->P.Nw = take(1);
    c->P.geo = take(4);
    c->P.acc_f = (float *)(base + L.pf);
    int32_t *pi = (int32_t *)(base + L.pi);
    c->P.shape = pi;
    c->P.N = pi + cap;
    c->P.lo = pi + 2 * cap;
    c->P.hi = pi + 5 * cap;
    c->ws_slots = L.slots_bytes ? (double *)(base + L.slots) : nullptr;
    c->ws_slots_bytes = L.slots_bytes;
}

} // namespace

// One step queues the lattice update and then, with K = 1 and slots
// (lbm_set_particles sets them up), Algorithm 1 with the new indicator from
// the partial sums the lattice kernel wrote; otherwise the momentum sums
// (which also clear the indicator) and Algorithm 1 with the new indicator
// (K > 1 adds the sub-step integration before it).  With profiling on, each launch is
// timed by a pair of pooled events attached to the kernel's own start and end
// (hipExtLaunchKernelGGL), whose durations are summed per class.
int lbm::step_impl(lbm_ctx *c, int64_t nsteps, double *rec_dev)
{
    std::vector<std::pair<int, size_t>> used; // (kernel class, event pair index)
    size_t next = 0;
    auto timed = [&](int kind, hipError_t (*fn)(lbm_ctx *, void *), void *arg) -> hipError_t {
        if (!c->prof) return fn(c, arg);
        if (2 * next + 2 > c->ev_pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                c->ev_pool.push_back(e);
            }
        }
        c->tev[0] = c->ev_pool[2 * next];
        c->tev[1] = c->ev_pool[2 * next + 1];
        c->tev_used = 0;
        const hipError_t err = fn(c, arg);
        c->tev[0] = c->tev[1] = nullptr;
        if (err != hipSuccess) return err;
        if (c->tev_used) { // a launcher with nothing to do records no events
            used.push_back({kind, next});
            ++next;
        }
        return hipSuccess;
    };
    for (int64_t s = 0; s < nsteps; ++s) {
        ++c->epoch; // the stamp of this step's slots
        void *bufs[2] = {c->f[c->cur], c->f[c->cur ^ 1]};
        HIPCHK(c, timed(0, [](lbm_ctx *cc, void *b) { return launch_stream_collide(cc, ((void **)b)[0], ((void **)b)[1]); },
                        bufs));
        c->cur ^= 1;
        double *rec = rec_dev ? rec_dev + (size_t)s * c->np * REC_STRIDE : nullptr;
        if (c->rp.K == 1 && c->fused) {
            // the lattice kernel took the sums: Algorithm 1 and the indicator from the slots
            HIPCHK(c, timed(2, [](lbm_ctx *cc, void *r) { return launch_rigid_fused(cc, (double *)r); }, rec));
            std::swap(c->P.X, c->P.Xn);
            std::swap(c->P.U, c->P.Unext);
            c->P.Uprev = c->P.U;
        } else if (c->rp.K == 1) {
            HIPCHK(c, timed(1, [](lbm_ctx *cc, void *r) { return launch_reduce(cc, 1, (double *)r); }, rec));
            if (c->sp.beta > 0)
                HIPCHK(c, timed(4, [](lbm_ctx *cc, void *b) { return launch_force(cc, ((void **)b)[0], ((void **)b)[1]); },
                                bufs));
            HIPCHK(c, timed(2, [](lbm_ctx *cc, void *) { return launch_rigid_raster(cc, 1); }, nullptr));
            std::swap(c->P.X, c->P.Xn);
        } else {
            HIPCHK(c, timed(1, [](lbm_ctx *cc, void *r) { return launch_reduce(cc, 1, (double *)r); }, rec));
            if (c->sp.beta > 0)
                HIPCHK(c, timed(4, [](lbm_ctx *cc, void *b) { return launch_force(cc, ((void **)b)[0], ((void **)b)[1]); },
                                bufs));
            HIPCHK(c, timed(2, [](lbm_ctx *cc, void *) { return launch_rigid_substeps(cc); }, nullptr));
            std::swap(c->P.X, c->P.Xn);
            HIPCHK(c, timed(3, [](lbm_ctx *cc, void *) { return launch_rigid_raster(cc, 0); }, nullptr));
        }
        c->step++;
        c->fresh = 0;
        if (c->prof && next >= 512) { // bound the pool: drain what has been recorded
            HIPCHK(c, hipStreamSynchronize(c->stream));
            for (auto &u : used) {
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * u.second], c->ev_pool[2 * u.second + 1]));
                c->prof_ms[u.first] += ms;
                c->prof_cnt[u.first] += 1;
            }
            used.clear();
            next = 0;
        }
    }
    if (c->prof) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (auto &u : used) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * u.second], c->ev_pool[2 * u.second + 1]));
            c->prof_ms[u.first] += ms;
            c->prof_cnt[u.first] += 1;
        }
    }
    return LBM_OK;
}

extern "C" {

int lbm_workspace_size(const lbm_config *cfg, size_t *bytes)
{
    std::string why;
    int Q, d;
    int64_t N;
    if (!bytes) return LBM_EINVAL;
    int rc = validate_cfg(cfg, why, Q, d, N);
    if (rc) return g_create_err = why, rc;
    *bytes = layout_for(cfg, Q, d, N).total;
    return LBM_OK;
}

int lbm_create(const lbm_config *cfg, lbm_ctx **out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    std::string why;
    int Q, d;
    int64_t N;
    int rc = validate_cfg(cfg, why, Q, d, N);
    if (rc) return g_create_err = why, rc;
    lbm_ctx *c = new lbm_ctx();
    c->cfg = *cfg;
    c->Q = Q;
    c->d = d;
    c->geo.nx = cfg->n[0];
    c->geo.ny = cfg->n[1];
    c->geo.nz = d == 3 ? cfg->n[2] : 1;
    c->cfg.n[2] = c->geo.nz;
    c->geo.N = N;
    // 64-bit population offsets in the lattice kernel when Q N >= 2^31;
    // LBM_WIDE_OFFSETS=1 in the environment selects them on any lattice (a
    // testing aid: the two kernels give the same bits)
    {
        const char *w = getenv("LBM_WIDE_OFFSETS");
        c->wide = (int64_t)Q * N >= ((int64_t)1 << 31) || (w && w[0] == '1');
    }
    c->geo.per_x = cfg->periodic[0] != 0;
    c->geo.per_y = cfg->periodic[1] != 0;
    c->geo.per_z = d == 3 && cfg->periodic[2] != 0;
    c->sp.tau = cfg->tau;
    c->sp.omega = 1.0 / cfg->tau;
    c->sp.alpha = cfg->alpha > 0 ? cfg->alpha : 1.0 / cfg->tau;
    c->sp.has_fluid_acc = 0;
    for (int k = 0; k < 3; ++k) {
        c->sp.fluid_acc[k] = k < d ? cfg->fluid_accel[k] : 0.0;
        if (c->sp.fluid_acc[k] != 0.0) c->sp.has_fluid_acc = 1;
    }
    c->sp.penalize_all = cfg->penalize_all != 0;
    c->sp.beta = cfg->rigid_beta;
    c->sp.frac = cfg->fractional_indicator != 0;
    c->rp.frac = c->sp.frac;
    for (int k = 0; k < 3; ++k) {
        c->sp.n[k] = k == 0 ? cfg->n[0] : k == 1 ? cfg->n[1] : (d == 3 ? cfg->n[2] : 1);
        c->sp.per[k] = k < d && cfg->periodic[k] != 0;
    }
    c->sp.stress = cfg->no_stress_penalty == 0;
    if (!c->sp.stress) c->sp.alpha = 0.0; // S of eq. (17) is linear in alpha: off
    c->sp.alpha_tracks_tau = !(cfg->alpha > 0);
    double wall_tab[2][19];
    if (d == 2) wall_terms<D2Q9>(cfg, c->sp, wall_tab);
    else wall_terms<D3Q19>(cfg, c->sp, wall_tab);
    c->grad = nullptr;
    c->fresh = 0;
    c->rp.rho_f = cfg->rho_f;
    for (int k = 0; k < 3; ++k) c->rp.g[k] = k < d ? cfg->g[k] : 0.0;
    c->rp.gmag = sqrt(c->rp.g[0] * c->rp.g[0] + c->rp.g[1] * c->rp.g[1] + c->rp.g[2] * c->rp.g[2]);
    c->rp.eps_p = cfg->eps_p;
    c->rp.eps_w = cfg->eps_w;
    c->rp.delta = cfg->delta;
    c->rp.K = cfg->K;
    c->rp.cform = cfg->collision_form;
    c->rp.gform = cfg->gravity_form;
    c->rp.np = 0;
    c->rp.d = d;
    c->device = cfg->device;
    c->stream = (hipStream_t)cfg->stream;
    c->cap = std::max(cfg->max_particles, 1);
    c->np = 0;
    c->step = 0;
    c->cur = 0;
    c->rec_dev = nullptr;
    c->rec_cap = 0;
    c->slab_mem = nullptr;
    c->slab_bytes = 0;
    c->owner_next = nullptr;
    c->slots = nullptr;
    c->slots_bytes = 0;
    c->slot_stride = c->slot_mx = c->slot_my = c->slot_mz = c->slot_sy = c->slot_sz = c->fused = 0;
    c->epoch = 0;
    c->check_every = cfg->check_every == 0 ? 64 : cfg->check_every;
    c->hflags = nullptr;
    c->poll_ev = nullptr;
    c->poll_pending = 0;
    c->prof = 0;
    c->tev[0] = c->tev[1] = nullptr;
    c->tev_used = 0;
    for (int k = 0; k < LBM_NKERNELS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_cnt[k] = 0;
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) {
        delete c;
        g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return LBM_EDEVICE;
    }
    if ((e = hipHostMalloc((void **)&c->hflags, 2 * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->poll_ev, hipEventDisableTiming)) != hipSuccess) {
        if (c->hflags) (void)hipHostFree(c->hflags);
        delete c;
        g_create_err = std::string("sentinel set-up: ") + hipGetErrorString(e);
        return LBM_EDEVICE;
    }
    const Layout L = layout_for(&c->cfg, Q, d, N);
    if (cfg->workspace) {
        if (cfg->workspace_bytes < L.total || ((uintptr_t)cfg->workspace % ALIGN) != 0) {
            (void)hipHostFree(c->hflags);
            (void)hipEventDestroy(c->poll_ev);
            delete c;
            g_create_err = "workspace too small or not 256-byte aligned";
            return LBM_ENOMEM;
        }
        c->ws = cfg->workspace;
        c->ws_bytes = cfg->workspace_bytes;
        c->own_mem = false;
    } else {
        e = hipMalloc(&c->ws, L.total);
        if (e != hipSuccess) {
            (void)hipHostFree(c->hflags);
            (void)hipEventDestroy(c->poll_ev);
            delete c;
            g_create_err = std::string("hipMalloc: ") + hipGetErrorString(e);
            return LBM_ENOMEM;
        }
        c->ws_bytes = L.total;
        c->own_mem = true;
    }
    carve(c, L);
    c->sp.geo = c->P.geo;
    double u0[3] = {cfg->u0[0], cfg->u0[1], d == 3 ? cfg->u0[2] : 0.0}, fe[19];
    feq_host(cfg->lattice, cfg->p0, u0, fe);
    if ((e = hipMemcpy(c->wall_tab, wall_tab, sizeof(wall_tab), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = launch_init_uniform(c, c->f[0], fe)) != hipSuccess ||
        (e = hipMemsetAsync(c->owner, 0xFF, (size_t)((N + 1) / 2 * 2) * sizeof(uint16_t), c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->flags, 0, ALIGN, c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->P.lo, 0, (size_t)c->cap * 6 * sizeof(int32_t), c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->P.hi, 0xFF, (size_t)c->cap * 3 * sizeof(int32_t), c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
        if (c->own_mem) (void)hipFree(c->ws);
        (void)hipHostFree(c->hflags);
        (void)hipEventDestroy(c->poll_ev);
        delete c;
        g_create_err = std::string("initialisation: ") + hipGetErrorString(e);
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->own_mem) (void)hipFree(c->ws);
    if (c->rec_dev) (void)hipFree(c->rec_dev);
    if (c->slots && c->slots != c->ws_slots) (void)hipFree(c->slots);
    if (c->slab_mem) (void)hipFree(c->slab_mem);
    free_grad(c);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->poll_ev) (void)hipEventDestroy(c->poll_ev);
    if (c->hflags) (void)hipHostFree(c->hflags);
    delete c;
    return LBM_OK;
}

} // extern "C"

namespace {

// The inclusion test of eq. (9) as the device evaluates it (raster_items in
// particles.hip): the same operation order, every product and sum rounded on
// its own (no contraction).
bool host_inside(int shape, double a, double b, double cs, double sn, double dx, double dy, double dz, bool band = false)
{
#pragma clang fp contract(off)
    if (band) { // the fractional indicator's band |r| < R + 1/2 (disks and spheres)
        const double Rh = a + 0.5;
        return (dx * dx + dy * dy) + dz * dz < Rh * Rh;
    }
    if (shape == LBM_DISK) return dx * dx + dy * dy <= a * a;
    if (shape == LBM_SPHERE) return (dx * dx + dy * dy) + dz * dz <= a * a;
    const double xi = cs * dx + sn * dy;
    const double eta = (-sn) * dx + cs * dy;
    return (b * b) * (xi * xi) + (a * a) * (eta * eta) <= (a * a) * (b * b);
}

// Number of nodes each of the n particles would own (lowest index wins),
// counted on the host over each scan box (centre_box of the device: the
// bounding radius plus two nodes, clipped at walls, unwrapped on periodic
// axes).  Lets lbm_set_particles and lbm_load_state reject a body with no
// node before anything on the device changes.
std::vector<int> host_claims(const lbm_ctx *c, const lbm_particle *p, int n)
{
    const Geom &g = c->geo;
    const int nn[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    const int d = c->d;
    std::vector<int> count(n, 0);
    std::unordered_set<int64_t> claimed;
    std::vector<int64_t> mine;
    for (int i = 0; i < n; ++i) {
        const lbm_particle &q = p[i];
        const double b = q.shape == LBM_ELLIPSE ? q.b : q.a;
        const double cs = q.shape == LBM_ELLIPSE ? cos(q.theta) : 1.0, sn = q.shape == LBM_ELLIPSE ? sin(q.theta) : 0.0;
        int lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = hi[k] = 0;
            if (k >= d) continue;
            lo[k] = (int)floor(q.x[k] - q.a) - 2;
            hi[k] = (int)ceil(q.x[k] + q.a) + 2;
            if (!per[k]) {
                lo[k] = std::max(lo[k], 0);
                hi[k] = std::min(hi[k], nn[k] - 1);
            }
        }
        mine.clear();
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const double dz = d == 3 ? (double)z - q.x[2] : 0.0;
                    if (!host_inside(q.shape, q.a, b, cs, sn, (double)x - q.x[0], (double)y - q.x[1], dz,
                                     c->sp.frac != 0))
                        continue;
                    auto wrapn = [](int v, int m) { return v < 0 ? v + m : (v >= m ? v - m : v); };
                    const int64_t id = wrapn(x, nn[0]) + (int64_t)nn[0] * (wrapn(y, nn[1]) + (int64_t)nn[1] * wrapn(z, nn[2]));
                    if (!claimed.count(id)) ++count[i];
                    mine.push_back(id);
                }
        claimed.insert(mine.begin(), mine.end());
    }
    return count;
}

// Host checks of a particle set (everything lbm_set_particles rejects with the
// context unchanged).
int check_particles(lbm_ctx *c, const lbm_particle *p, int32_t n)
{
    if (n < 0 || n > c->cfg.max_particles) return fail(c, LBM_EINVAL, "particle count exceeds max_particles");
    if (n > 0 && !p) return fail(c, LBM_EINVAL, "particles is NULL");
    const int d = c->d;
    const int nn[3] = {c->geo.nx, c->geo.ny, c->geo.nz};
    const int per[3] = {c->geo.per_x, c->geo.per_y, c->geo.per_z};
    for (int i = 0; i < n; ++i) {
        const lbm_particle &q = p[i];
        const bool ok_shape = (d == 2 && (q.shape == LBM_DISK || q.shape == LBM_ELLIPSE)) || (d == 3 && q.shape == LBM_SPHERE);
        if (!ok_shape) return fail(c, LBM_EINVAL, "shape not valid for this lattice");
        if (c->sp.frac && q.shape == LBM_ELLIPSE)
            return fail(c, LBM_EINVAL, "the fractional indicator takes disks and spheres only");
        if (!(q.rho_s > 0) || !isfinite(q.rho_s) || !(q.a >= 1.0) || !isfinite(q.a))
            return fail(c, LBM_EINVAL, "rho_s must be > 0 and a >= 1");
        if (q.shape == LBM_ELLIPSE && !(q.b >= 1.0 && q.b <= q.a)) return fail(c, LBM_EINVAL, "ellipse needs a >= b >= 1");
        if (q.shape == LBM_ELLIPSE && !isfinite(q.theta)) return fail(c, LBM_EINVAL, "non-finite orientation");
        for (int k = 0; k < d; ++k) {
            if (!isfinite(q.x[k])) return fail(c, LBM_EINVAL, "non-finite centre");
            if (per[k]) {
                if (q.a + 2.0 >= 0.5 * nn[k]) return fail(c, LBM_EINVAL, "radius too large for a periodic axis");
                if (q.x[k] < 0 || q.x[k] >= nn[k]) return fail(c, LBM_EINVAL, "centre outside a periodic axis");
            } else if (q.x[k] - q.a < -0.5 || q.x[k] + q.a > nn[k] - 0.5) {
                return fail(c, LBM_EINVAL, "particle crosses a wall");
            }
        }
    }
    const std::vector<int> cnt = host_claims(c, p, n);
    for (int i = 0; i < n; ++i)
        if (cnt[i] == 0)
            return fail(c, LBM_EINVAL, "particle " + std::to_string(i) +
                                           " would own no lattice node (its shape lies inside lower-index particles)");
    return LBM_OK;
}

// Collision constant C_i of sec. 2.3 for the current g and form.
double coll_const(const lbm_ctx *c, const lbm_particle &q)
{
    const double b = q.shape == LBM_ELLIPSE ? q.b : q.a;
    const double V = q.shape == LBM_DISK      ? M_PI * q.a * q.a
                     : q.shape == LBM_ELLIPSE ? M_PI * q.a * b
                                              : 4.0 / 3.0 * M_PI * q.a * q.a * q.a;
    const double Cl = (q.rho_s - c->rp.rho_f) * c->rp.gmag;
    return c->rp.cform == 1 ? Cl : Cl * V;
}

// Upload rho_s and C_i of the current particles (after a change of rho_s or g).
int upload_constants(lbm_ctx *c)
{
    const int cap = c->cap;
    std::vector<double> rho(cap, 1.0), C(cap, 0.0);
    for (int i = 0; i < c->np; ++i) {
        rho[i] = c->host_parts[i].rho_s;
        C[i] = coll_const(c, c->host_parts[i]);
    }
    HIPCHK(c, hipMemcpyAsync(c->P.rho_s, rho.data(), sizeof(double) * cap, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.Cc, C.data(), sizeof(double) * cap, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream)); // the host vectors go out of scope
    return LBM_OK;
}

// Install n checked particles: clear the previous indicator, upload the
// constants, centres, orientations and A = 0, choose the slot layout of the
// fused-sums step.  The caller rasterises and sets the velocities.
int install_particles(lbm_ctx *c, const lbm_particle *p, int32_t n)
{
    const int d = c->d, cap = c->cap;
    if (c->np > 0) HIPCHK(c, launch_raster_clear(c));
    std::vector<double> X(3 * cap, 0), th(cap, 0), z3(3 * cap, 0), a(cap, 1), b(cap, 1);
    std::vector<int32_t> shape(cap, 0);
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) X[3 * i + k] = p[i].x[k];
        th[i] = p[i].theta;
        a[i] = p[i].a;
        b[i] = p[i].shape == LBM_ELLIPSE ? p[i].b : p[i].a;
        shape[i] = p[i].shape;
    }
    const size_t b3 = sizeof(double) * 3 * cap, b1 = sizeof(double) * cap;
    HIPCHK(c, hipMemcpyAsync(c->P.X, X.data(), b3, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.theta, th.data(), b1, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.A, z3.data(), b3, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.a, a.data(), b1, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.b, b.data(), b1, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.shape, shape.data(), sizeof(int32_t) * cap, hipMemcpyHostToDevice, c->stream));
    c->np = n;
    c->host_parts.assign(p, p + n);
    int rc = upload_constants(c); // also waits for the copies above
    if (rc) return rc;
    // fused-sums step (K = 1): the slot tables (slot_sizes), in the
    // workspace when it holds a large enough region, else allocated here
    c->fused = 0;
    // (the forcing pass needs the indicator after the sums; the slots hold
    // node counts, not the weight sums of the fractional indicator)
    if (c->rp.K == 1 && n > 0 && !(c->sp.beta > 0) && !c->sp.frac) {
        const Geom &g = c->geo;
        int ext = 0;
        for (int i = 0; i < n; ++i) ext = std::max(ext, (int)ceil(2.0 * p[i].a) + 7);
        auto lg = [](int v) {
            int k = 0;
            while ((1 << k) < v) ++k;
            return k;
        };
        const int nn[3] = {g.nx, g.ny, g.nz}, per[3] = {g.per_x, g.per_y, g.per_z};
        SlotSizes z;
        if (slot_sizes(nn, per, d, ext, cap, z)) {
            if (z.bytes <= c->ws_slots_bytes) {
                if (c->slots && c->slots != c->ws_slots) HIPCHK(c, hipFree(c->slots));
                c->slots = c->ws_slots;
                c->slots_bytes = c->ws_slots_bytes;
            } else if (c->slots == c->ws_slots || z.bytes > c->slots_bytes) {
                if (c->slots && c->slots != c->ws_slots) HIPCHK(c, hipFree(c->slots));
                c->slots = nullptr;
                c->slots_bytes = 0;
                HIPCHK(c, hipMalloc((void **)&c->slots, z.bytes));
                c->slots_bytes = z.bytes;
            }
            // NaN stamps: no slot counts until a step writes it
            HIPCHK(c, hipMemsetAsync(c->slots, 0xFF, c->slots_bytes, c->stream));
            c->slot_stride = (int)z.stride;
            c->slot_mx = z.Mx - 1;
            c->slot_my = z.My - 1;
            c->slot_mz = z.Mz - 1;
            c->slot_sy = lg(z.Mx);
            c->slot_sz = lg(z.Mx) + lg(z.My);
            c->fused = 1;
        }
    }
    // With fused sums U^{n-1} is read from U itself (U^n goes to Unext,
    // swapped in after the step), so U_prev is an alias of U.  The alias may
    // outlive a later set-up without fused sums; that is harmless because
    // every path leaves U_prev equal to U between steps, and the sums kernel
    // reads U_prev before it writes U.
    if (c->fused) c->P.Uprev = c->P.U;
    return LBM_OK;
}

// U^0 and omega^0 on the current populations (eq. 22a-b), then U^{-1} = U^0
// and omega^{-1} = omega^0 (the start of Algorithm 1).
int measure_initial(lbm_ctx *c)
{
    const size_t b3 = sizeof(double) * 3 * c->cap;
    HIPCHK(c, launch_fields(c, c->f[c->cur], c->usol, nullptr, 1));
    HIPCHK(c, launch_reduce(c, 0, nullptr));
    if (c->P.Uprev != c->P.U) HIPCHK(c, hipMemcpyAsync(c->P.Uprev, c->P.U, b3, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P.Wprev, c->P.W, b3, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

// After the device rasterised: every body must own a node.  The host count
// agrees with the device except where an ellipse boundary passes through a
// node and the two cos/sin differ in the last bit; then the particles are
// taken out again (the context is left with none).
int check_device_claims(lbm_ctx *c)
{
    std::vector<int32_t> Nn(c->cap, 0);
    HIPCHK(c, hipMemcpyAsync(Nn.data(), c->P.N, sizeof(int32_t) * c->cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->np; ++i)
        if (Nn[i] == 0) {
            HIPCHK(c, launch_raster_clear(c));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            c->np = 0;
            c->fused = 0;
            c->host_parts.clear();
            c->fresh = 0;
            return fail(c, LBM_EINVAL, "a particle covers no lattice node on the device (a boundary tie); "
                                       "the context now holds no particles");
        }
    return LBM_OK;
}

// Host side of the sentinel: wait for the queued copy of the device flags
// and report what it read.
int poll_result(lbm_ctx *c)
{
    c->poll_pending = 0;
    HIPCHK(c, hipEventSynchronize(c->poll_ev));
    if (c->hflags[0]) return fail(c, LBM_EUNSTABLE, "velocity non-finite or above 0.3 (sentinel read inside lbm_step)");
    if (c->hflags[1])
        return fail(c, LBM_EDOMAIN, "a particle left the box or lost all its nodes (sentinel read inside lbm_step)");
    return LBM_OK;
}

} // namespace

extern "C" {

int lbm_set_particles(lbm_ctx *c, const lbm_particle *p, int32_t n)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    int rc = check_particles(c, p, n);
    if (rc) return rc;
    free_grad(c); // checkpoints of an earlier differentiated run no longer match
    if ((rc = install_particles(c, p, n))) return rc;
    // indicator and acceleration table (A = 0), U^0, omega^0 on the current populations
    HIPCHK(c, launch_rigid_raster(c, 0));
    if ((rc = measure_initial(c))) return rc;
    if ((rc = check_device_claims(c))) return rc;
    c->fresh = 1;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return c ? fail(c, LBM_EINVAL, "nsteps < 0") : LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const int64_t k = c->check_every;
    if (k <= 0) return step_impl(c, nsteps, nullptr);
    int64_t done = 0;
    while (done < nsteps) {
        const int64_t chunk = std::min(nsteps - done, k - c->step % k);
        int rc = step_impl(c, chunk, nullptr);
        if (rc) return rc;
        done += chunk;
        if (c->step % k) continue;
        // a poll point: read the previous poll (the device has then finished
        // every step but the last chunk), then queue this one
        if (c->poll_pending && (rc = poll_result(c))) return rc;
        HIPCHK(c, hipMemcpyAsync(c->hflags, c->flags, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->poll_ev, c->stream));
        c->poll_pending = 1;
    }
    // a poll that has already completed is read without waiting
    if (c->poll_pending && hipEventQuery(c->poll_ev) == hipSuccess) return poll_result(c);
    return LBM_OK;
}

int lbm_get_fields_device(lbm_ctx *c, double *dev_u, double *dev_p, int32_t *dev_owner)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    if (dev_u || dev_p) {
        // the fields kernel writes both; a NULL one goes to the staging area
        double *du = dev_u ? dev_u : c->staging, *dp = dev_p ? dev_p : c->staging + (size_t)3 * c->geo.N;
        HIPCHK(c, launch_fields(c, c->f[c->cur], du, dp, 0));
    }
    if (dev_owner) HIPCHK(c, launch_owner_to_int(c, dev_owner));
    return LBM_OK;
}

int lbm_set_params(lbm_ctx *c, const double *rho_s, double tau, const double *g)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const bool new_tau = tau > 0.0;
    if (new_tau && !(tau > 0.5 && isfinite(tau))) return fail(c, LBM_EINVAL, "tau must exceed 1/2");
    if (new_tau && !c->sp.alpha_tracks_tau && c->sp.alpha > 1.0 / tau * (1.0 + 1e-12))
        return fail(c, LBM_EINVAL, "the fixed alpha would exceed 1/tau");
    for (int i = 0; rho_s && i < c->np; ++i)
        if (!(rho_s[i] > 0) || !isfinite(rho_s[i])) return fail(c, LBM_EINVAL, "densities must be positive and finite");
    for (int k = 0; g && k < c->d; ++k)
        if (!isfinite(g[k])) return fail(c, LBM_EINVAL, "gravity must be finite");
    free_grad(c);
    if (new_tau) {
        c->cfg.tau = c->sp.tau = tau;
        c->sp.omega = 1.0 / tau;
        if (c->sp.alpha_tracks_tau && c->sp.stress) c->sp.alpha = 1.0 / tau;
    }
    if (g) {
        for (int k = 0; k < 3; ++k) c->cfg.g[k] = c->rp.g[k] = k < c->d ? g[k] : 0.0;
        c->rp.gmag = sqrt(c->rp.g[0] * c->rp.g[0] + c->rp.g[1] * c->rp.g[1] + c->rp.g[2] * c->rp.g[2]);
    }
    for (int i = 0; rho_s && i < c->np; ++i) c->host_parts[i].rho_s = rho_s[i];
    if (c->np == 0) return LBM_OK;
    int rc = upload_constants(c);
    if (rc) return rc;
    HIPCHK(c, launch_write_acc(c));
    // right after the set-up U^{-1} = U^0, which depends on the acceleration
    if (c->fresh && (rc = measure_initial(c))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

} // extern "C"

namespace {

// Layout of a saved state (lbm_save_state).  Everything is little-endian
// host layout; the per-particle block is structure-of-arrays, np entries
// each: rho_s, a, b, shape (as a double), X[3], theta, U^{n-1}[3],
// omega^{n-1}[3], A[3]; the populations follow at f_off.
constexpr char STATE_MAGIC[8] = {'L', 'B', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr int32_t STATE_VERSION = 1;
struct StateHeader {
    char magic[8];
    int32_t version, lattice, storage, n[3], periodic[3], np, fresh, pad;
    int64_t step;
    uint64_t f_off, fbytes, total;
    double tau, g[3];
};
constexpr int PSTATE = 17; // doubles per particle
constexpr size_t STATE_PART_OFF = 256;

size_t state_fbytes(const lbm_ctx *c) { return (size_t)c->Q * c->geo.N * storage_bytes(c->cfg.storage); }

void state_layout(const lbm_ctx *c, int np, size_t &f_off, size_t &total)
{
    f_off = align_up(STATE_PART_OFF + (size_t)np * PSTATE * sizeof(double));
    total = f_off + state_fbytes(c);
}

// offsets (in doubles from the particle block) of the SoA arrays
struct PartOff {
    size_t rho, a, b, shape, X, theta, Up, Wp, A;
};
PartOff part_off(int np)
{
    PartOff o;
    o.rho = 0;
    o.a = (size_t)np;
    o.b = 2 * (size_t)np;
    o.shape = 3 * (size_t)np;
    o.X = 4 * (size_t)np;
    o.theta = 7 * (size_t)np;
    o.Up = 8 * (size_t)np;
    o.Wp = 11 * (size_t)np;
    o.A = 14 * (size_t)np;
    return o;
}

} // namespace

extern "C" {

int lbm_state_size(const lbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return LBM_EINVAL;
    size_t f_off;
    state_layout(c, c->np, f_off, *bytes);
    return LBM_OK;
}

int lbm_save_state(lbm_ctx *c, void *buf)
{
    if (!c || !buf) return c ? fail(c, LBM_EINVAL, "buf is NULL") : LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const int np = c->np;
    StateHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, STATE_MAGIC, 8);
    h.version = STATE_VERSION;
    h.lattice = c->cfg.lattice;
    h.storage = c->cfg.storage;
    for (int k = 0; k < 3; ++k) {
        h.n[k] = k == 0 ? c->geo.nx : k == 1 ? c->geo.ny : c->geo.nz;
        h.periodic[k] = k == 0 ? c->geo.per_x : k == 1 ? c->geo.per_y : c->geo.per_z;
        h.g[k] = c->rp.g[k];
    }
    h.np = np;
    h.fresh = c->fresh;
    h.step = c->step;
    h.tau = c->sp.tau;
    size_t f_off, total;
    state_layout(c, np, f_off, total);
    h.f_off = f_off;
    h.fbytes = state_fbytes(c);
    h.total = total;
    char *out = (char *)buf;
    const PartOff o = part_off(np);
    std::vector<double> cst(4 * (size_t)np);
    for (int i = 0; i < np; ++i) {
        const lbm_particle &q = c->host_parts[i];
        cst[o.rho + i] = q.rho_s;
        cst[o.a + i] = q.a;
        cst[o.b + i] = q.shape == LBM_ELLIPSE ? q.b : q.a;
        cst[o.shape + i] = (double)q.shape;
    }
    double *pb = (double *)(out + STATE_PART_OFF);
    HIPCHK(c, hipMemcpyAsync(out, &h, sizeof(h), hipMemcpyDefault, c->stream));
    if (np > 0) {
        const size_t b3 = sizeof(double) * 3 * np;
        HIPCHK(c, hipMemcpyAsync(pb, cst.data(), cst.size() * sizeof(double), hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(pb + o.X, c->P.X, b3, hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(pb + o.theta, c->P.theta, sizeof(double) * np, hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(pb + o.Up, c->P.Uprev, b3, hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(pb + o.Wp, c->P.Wprev, b3, hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(pb + o.A, c->P.A, b3, hipMemcpyDefault, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(out + f_off, c->f[c->cur], h.fbytes, hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_load_state(lbm_ctx *c, const void *buf)
{
    if (!c || !buf) return c ? fail(c, LBM_EINVAL, "buf is NULL") : LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const char *in = (const char *)buf;
    StateHeader h;
    HIPCHK(c, hipMemcpyAsync(&h, in, sizeof(h), hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (memcmp(h.magic, STATE_MAGIC, 8) || h.version != STATE_VERSION) return fail(c, LBM_EINVAL, "not a saved state");
    const int nn[3] = {c->geo.nx, c->geo.ny, c->geo.nz}, per[3] = {c->geo.per_x, c->geo.per_y, c->geo.per_z};
    bool same = h.lattice == c->cfg.lattice && h.storage == c->cfg.storage;
    for (int k = 0; k < 3; ++k) same = same && h.n[k] == nn[k] && h.periodic[k] == per[k];
    if (!same) return fail(c, LBM_EINVAL, "the state belongs to another lattice, storage or box");
    size_t f_off, total;
    if (h.np < 0 || h.np > c->cfg.max_particles) return fail(c, LBM_EINVAL, "the state holds more particles than max_particles");
    state_layout(c, h.np, f_off, total);
    if (h.f_off != f_off || h.total != total || h.fbytes != state_fbytes(c))
        return fail(c, LBM_EINVAL, "inconsistent state header");
    if (!(h.tau > 0.5) || (!c->sp.alpha_tracks_tau && c->sp.alpha > 1.0 / h.tau * (1.0 + 1e-12)))
        return fail(c, LBM_EINVAL, "the state's tau is not valid for this context");
    const int np = h.np;
    const PartOff o = part_off(np);
    std::vector<double> pb((size_t)np * PSTATE);
    if (np > 0) {
        HIPCHK(c, hipMemcpyAsync(pb.data(), in + STATE_PART_OFF, pb.size() * sizeof(double), hipMemcpyDefault, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    std::vector<lbm_particle> parts(np);
    for (int i = 0; i < np; ++i) {
        lbm_particle &q = parts[i];
        memset(&q, 0, sizeof(q));
        q.shape = (int32_t)pb[o.shape + i];
        q.rho_s = pb[o.rho + i];
        q.a = pb[o.a + i];
        q.b = pb[o.b + i];
        for (int k = 0; k < 3; ++k) q.x[k] = k < c->d ? pb[o.X + 3 * i + k] : 0.0;
        q.theta = pb[o.theta + i];
    }
    // the parameters first (the collision constants depend on g), then the same
    // checks as lbm_set_particles, before anything else changes
    const RigidParams rp0 = c->rp;
    const StepParams sp0 = c->sp;
    c->sp.tau = h.tau;
    c->sp.omega = 1.0 / h.tau;
    if (c->sp.alpha_tracks_tau && c->sp.stress) c->sp.alpha = 1.0 / h.tau;
    for (int k = 0; k < 3; ++k) c->rp.g[k] = k < c->d ? h.g[k] : 0.0;
    c->rp.gmag = sqrt(c->rp.g[0] * c->rp.g[0] + c->rp.g[1] * c->rp.g[1] + c->rp.g[2] * c->rp.g[2]);
    int rc = check_particles(c, parts.data(), np);
    if (rc) {
        c->rp = rp0;
        c->sp = sp0;
        return rc;
    }
    c->cfg.tau = h.tau;
    for (int k = 0; k < 3; ++k) c->cfg.g[k] = c->rp.g[k];
    free_grad(c);
    HIPCHK(c, hipStreamSynchronize(c->stream)); // no poll still pending on the flags
    c->poll_pending = 0;
    if ((rc = install_particles(c, parts.data(), np))) return rc;
    if (np > 0) {
        // U^{n-1} goes to U as well (with fused sums U_prev is U itself; without,
        // the sums read U_prev and overwrite U), omega^{n-1} likewise
        const size_t b3 = sizeof(double) * 3 * np;
        std::vector<double> X(3 * (size_t)np, 0.0);
        for (int i = 0; i < np; ++i)
            for (int k = 0; k < c->d; ++k) X[3 * i + k] = parts[i].x[k];
        HIPCHK(c, hipMemcpyAsync(c->P.X, X.data(), b3, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.theta, pb.data() + o.theta, sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.A, pb.data() + o.A, b3, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.U, pb.data() + o.Up, b3, hipMemcpyHostToDevice, c->stream));
        if (c->P.Uprev != c->P.U)
            HIPCHK(c, hipMemcpyAsync(c->P.Uprev, pb.data() + o.Up, b3, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.W, pb.data() + o.Wp, b3, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.Wprev, pb.data() + o.Wp, b3, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->f[c->cur], in + f_off, h.fbytes, hipMemcpyDefault, c->stream));
    if (np > 0) {
        // the indicator of X^n, theta^n and the acceleration table from A^n
        HIPCHK(c, launch_rigid_raster(c, 0));
        // node counts for the check below (U and omega measured into scratch)
        HIPCHK(c, launch_fields(c, c->f[c->cur], c->usol, nullptr, 1));
        HIPCHK(c, launch_reduce(c, 0, nullptr, 1));
    }
    HIPCHK(c, hipMemsetAsync(c->flags, 0, 2 * sizeof(int32_t), c->stream));
    if ((rc = check_device_claims(c))) return rc;
    c->step = h.step;
    c->fresh = h.fresh;
    return LBM_OK;
}

int lbm_step_record(lbm_ctx *c, int64_t nsteps, double *host_rec)
{
    if (!c || nsteps < 0 || (nsteps > 0 && !host_rec)) return c ? fail(c, LBM_EINVAL, "bad arguments") : LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const size_t need = (size_t)nsteps * std::max(c->np, 1) * REC_STRIDE * sizeof(double);
    if (need > c->rec_cap) {
        if (c->rec_dev) HIPCHK(c, hipFree(c->rec_dev));
        c->rec_dev = nullptr;
        c->rec_cap = 0;
        HIPCHK(c, hipMalloc(&c->rec_dev, need));
        c->rec_cap = need;
    }
    int rc = step_impl(c, nsteps, c->rec_dev);
    if (rc) return rc;
    if (nsteps > 0 && c->np > 0) {
        std::vector<double> full((size_t)nsteps * c->np * REC_STRIDE);
        HIPCHK(c, hipMemcpyAsync(full.data(), c->rec_dev, full.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t r = 0; r < (size_t)nsteps * c->np; ++r)
            for (int k = 0; k < 14; ++k) host_rec[r * 14 + k] = full[r * REC_STRIDE + k];
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return lbm_sync(c);
}

int lbm_sync(lbm_ctx *c)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    int32_t fl[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(fl, c->flags, sizeof(fl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (fl[0]) return fail(c, LBM_EUNSTABLE, "velocity non-finite or above 0.3");
    if (fl[1]) return fail(c, LBM_EDOMAIN, "a particle left the box or lost all its nodes");
    return LBM_OK;
}

int lbm_get_fields(lbm_ctx *c, double *host_u, double *host_p, int32_t *host_owner)
{
    if (!c) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const int64_t N = c->geo.N;
    if (host_u || host_p) {
        double *du = c->staging, *dp = c->staging + (size_t)3 * N;
        HIPCHK(c, launch_fields(c, c->f[c->cur], du, dp, 0));
        if (host_u) HIPCHK(c, hipMemcpyAsync(host_u, du, sizeof(double) * c->d * N, hipMemcpyDeviceToHost, c->stream));
        if (host_p) HIPCHK(c, hipMemcpyAsync(host_p, dp, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (host_owner) {
        int32_t *dow = (int32_t *)c->staging;
        HIPCHK(c, launch_owner_to_int(c, dow));
        HIPCHK(c, hipMemcpyAsync(host_owner, dow, sizeof(int32_t) * N, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return lbm_sync(c);
}

int lbm_get_populations(lbm_ctx *c, double *host_f)
{
    if (!c || !host_f) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const int64_t N = c->geo.N;
    for (int q0 = 0; q0 < c->Q; q0 += 4) {
        const int nq = std::min(4, c->Q - q0);
        HIPCHK(c, launch_populations(c, c->f[c->cur], c->staging, q0, nq));
        HIPCHK(c, hipMemcpyAsync(host_f + (size_t)q0 * N, c->staging, sizeof(double) * nq * N, hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx *c, const double *host_f)
{
    if (!c || !host_f) return LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const int64_t N = c->geo.N;
    // f~ of direction q needs f^n of q and of opp(q): upload both
    for (int q = 0; q < c->Q; ++q) {
        int opp;
        if (c->cfg.lattice == LBM_D2Q9) {
            static const int o9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
            opp = o9[q];
        } else {
            opp = q == 0 ? 0 : (q % 2 ? q + 1 : q - 1);
        }
        HIPCHK(c, hipMemcpyAsync(c->staging, host_f + (size_t)q * N, sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->staging + N, host_f + (size_t)opp * N, sizeof(double) * N, hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, launch_set_populations(c, c->staging, c->f[c->cur], q, 2));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

int lbm_get_particles(lbm_ctx *c, lbm_particle *out, int32_t n)
{
    if (!c || (n > 0 && !out)) return LBM_EINVAL;
    if (n > c->np) return fail(c, LBM_EINVAL, "more particles requested than set");
    (void)hipSetDevice(c->device);
    if (c->np > 0) {
        // measure U and omega on the current populations, into scratch arrays
        // (the step state, U^{n-1} included, stays as it is)
        HIPCHK(c, launch_fields(c, c->f[c->cur], c->usol, nullptr, 1));
        HIPCHK(c, launch_reduce(c, 0, nullptr, 1));
    }
    const int cap = c->cap;
    std::vector<double> X(3 * cap), th(cap), U(3 * cap), W(3 * cap), Up(3 * cap), Wp(3 * cap), A(3 * cap);
    std::vector<int32_t> Nn(cap);
    const size_t b3 = sizeof(double) * 3 * cap;
    HIPCHK(c, hipMemcpyAsync(X.data(), c->P.X, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(th.data(), c->P.theta, sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(U.data(), c->np > 0 ? c->P.Y : c->P.U, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(W.data(), c->np > 0 ? c->P.Ys : c->P.W, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Up.data(), c->P.Uprev, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Wp.data(), c->P.Wprev, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(A.data(), c->P.A, b3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Nn.data(), c->P.N, sizeof(int32_t) * cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i) {
        lbm_particle &q = out[i];
        q = c->host_parts[i];
        for (int k = 0; k < 3; ++k) {
            q.x[k] = X[3 * i + k];
            q.U[k] = U[3 * i + k];
            q.omega[k] = W[3 * i + k];
            q.U_prev[k] = Up[3 * i + k];
            q.omega_prev[k] = Wp[3 * i + k];
            q.A[k] = A[3 * i + k];
        }
        q.theta = th[i];
        q.n_nodes = Nn[i];
    }
    return lbm_sync(c);
}

int lbm_profile(lbm_ctx *c, int32_t enable)
{
    if (!c) return LBM_EINVAL;
    c->prof = enable != 0;
    return LBM_OK;
}

int lbm_profile_read(lbm_ctx *c, double *ms, int64_t *cnt, int32_t reset)
{
    if (!c) return LBM_EINVAL;
    for (int k = 0; k < LBM_NKERNELS; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (cnt) cnt[k] = c->prof_cnt[k];
        if (reset) {
            c->prof_ms[k] = 0.0;
            c->prof_cnt[k] = 0;
        }
    }
    return LBM_OK;
}

int lbm_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if ((!dst || !src) && bytes) return LBM_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src | bytes) % 16) return LBM_EINVAL; // the kernel moves whole 16-byte words
    return launch_copy(dst, src, bytes, (hipStream_t)stream) == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

int lbm_copy_arrays(void *dst, const void *src, int32_t narrays, size_t bytes_per_array, void *stream)
{
    if (narrays < 1 || narrays > 32) return LBM_EINVAL;
    if ((!dst || !src) && bytes_per_array) return LBM_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src | bytes_per_array) % 16) return LBM_EINVAL;
    return launch_copy_arrays(dst, src, narrays, bytes_per_array, (hipStream_t)stream) == hipSuccess ? LBM_OK
                                                                                                    : LBM_EDEVICE;
}

int lbm_get_step(const lbm_ctx *c, int64_t *step)
{
    if (!c || !step) return LBM_EINVAL;
    *step = c->step;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c)
{
    if (!c) return g_create_err.c_str();
    return c->err.c_str();
}

} // extern "C"
