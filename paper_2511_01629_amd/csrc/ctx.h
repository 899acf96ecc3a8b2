// ctx.h -- the context behind the C ABI and the launchers each kernel file
// provides.  Private to the library.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"

// Checkpoint storage of a differentiated run (grad.hip).
struct GradState;

namespace lbm {

// Per-step, per-particle record written by the momentum-sum kernel:
// X[3] theta U^n[3] omega^n[3] A^n[3] N U^{n-1}[3] (pad to 20 doubles).
constexpr int REC_STRIDE = 20;

// Per-particle terms of the adjoint with the fractional indicator, written by
// the rigid adjoint of step n for the lattice adjoint of the same step:
// N_bar (the adjoint of N = sum chi through U^n = sum chi u / N and the mass
// rho_s N), w = (adjoint of U^{n-1}) / N [3], U^{n-1} [3], pad.
constexpr int FRAC_STRIDE = 8;

// Device arrays of the particle state, structure-of-arrays, FP64.
struct PartDev {
    double *X, *Xn, *theta, *U, *W, *Uprev, *Wprev, *A; // [cap*3] (theta [cap]); Xn: next centres
    double *rho_s, *a, *b, *Cc;                    // [cap]; Cc = collision constant C_i
    double *acc_d;                                 // [cap*3] solid-node acceleration (FP64 mode)
    float *acc_f;                                  // [cap*3] the same in FP32
    double *Unext;                                 // [cap*3] U^n written by the fused-sums step (swapped with U)
    double *Ub, *dth;                              // U_bar = (U^n + U^{n-1})/2 [cap*3], theta increment [cap]
    double *Y, *Ys, *Y2, *Dc;                      // [cap*3] sub-step scratch (Dc: summed corrections)
    double *Nw;                                    // [cap] N_i as a weight sum (sum chi, or the node count)
    double *geo;                                   // [cap*4] centre of the current indicator, bounding radius
    int32_t *shape, *N;                            // [cap]
    int32_t *lo, *hi;                              // [cap*3] scan box (unwrapped node coords)
};

// Per-particle partial momentum sums written by the lattice kernel (the
// fused-sums step, K = 1): one slot per (particle, lattice row key, wavefront
// key), each [stamp, lane mask, first node, sums...]; a slot counts for the
// step whose stamp it carries, so nothing is ever cleared.  Slot s of particle i starts
// at slots + (i * stride + s) * width.
// Bound on the particle count (the owner map is 16-bit, FLUID reserved); the
// fused particle kernels keep one reach bit per particle in LDS.
constexpr int MAX_NP = 65536;

// Width of a momentum-sum record in doubles: stamp, lane mask, the packed
// wrapped coordinates of the wavefront's first node (x0 | y << 21 | z << 42),
// then the sums (2D 3, 3D 5).
constexpr int slot_width(int d) { return (d == 2 ? 3 : 5) + 3; }

struct SlotParams {
    double *slots;      // [np][stride][slot_width(d)] records
    int stride;         // slots per particle
    int mx, my, mz;     // wavefront, y and z keys: masks of powers of two
    int sy, sz;         // shifts of the y and z keys
    double stamp;       // this step's stamp
    uint16_t *clear;    // the owner map to reset to FLUID as it is read (in-place steps), or NULL
};

// Everything a kernel needs to know about the lattice.
struct Geom {
    int nx, ny, nz;
    int64_t N;
    int per_x, per_y, per_z;
};

struct StepParams {
    double tau, omega, alpha; // omega = 1/tau
    double fluid_acc[3];
    int has_fluid_acc;
    int penalize_all;
    int alpha_tracks_tau; // alpha = 1/tau (the default) rather than a fixed value
    // moving walls: their axis (1 y, 2 z; 0 none) and, in device memory, per
    // side (low, high) and population, the term 2 w_q (c_q . u_w)/cs^2 that a
    // population pulled from behind that wall gains ([2][19] doubles)
    int wall_axis;
    const double *wall_tab;
    // rigid-velocity forcing (an extension): strength beta (0: off), and
    // whether the penalization source of eq. (17) acts (1: the paper's
    // method; 0: alpha is held at 0, which switches the source off)
    double beta;
    int stress;
    // fractional indicator (an extension, disks and spheres): a node of the
    // band |x - X_i| < R_i + 1/2 carries chi = min(1, R_i + 1/2 - |x - X_i|),
    // which weights its acceleration and penalization; geo holds, per
    // particle, the centre the indicator was built from and R ([cap][4]), and
    // n, per the lattice (for the node coordinates)
    int frac;
    const double *geo;
    int n[3], per[3];
};

// Device pointers of one backward step of Algorithm 1 (see adjoint.hip).
struct AdjArraysHost {
    const double *rec, *Xbar, *Abar, *Upbar;
    double *Xbar_out, *Upbar_out, *uext_d;
    float *uext_f;
    double *acc_d;
    float *acc_f;
    double *rho_g, *g_g;
    // fractional indicator only (else NULL): per particle, the adjoint terms
    // the lattice adjoint adds to chi_bar ([np][FRAC_STRIDE]) and
    // the centre and radius of step n's indicator ([np][4], StepParams::geo)
    double *fpart = nullptr, *geo = nullptr;
};

// Periodic index wrap for an index at most one period out of range.
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

struct RigidParams {
    double rho_f, gmag, g[3];
    double eps_p, eps_w, delta;
    int K, cform, gform, np, d;
    int frac; // the fractional indicator (StepParams::frac)
};

} // namespace lbm

struct lbm_ctx {
    lbm_config cfg;
    int Q, d;
    int wide; // 64-bit population offsets in the lattice kernel (Q N >= 2^31)
    lbm::Geom geo;
    lbm::StepParams sp;
    lbm::RigidParams rp;
    hipStream_t stream;
    int device;
    bool own_mem;
    void *ws;
    size_t ws_bytes;
    void *f[2];   // post-collision populations f~ (ping-pong), [Q][N] raw storage
    int cur;      // f[cur] holds f~ of the last completed step
    void *fws[2]; // the workspace's two population buffers (f[] points elsewhere only
                  // inside a differentiated run)
    uint16_t *owner;      // indicator the next step reads
    uint16_t *owner_next; // NULL: steps update `owner` in place; else the (all FLUID)
                          // buffer the next step's indicator goes to (differentiated runs)
    double *usol;    // [d][N] velocity on solid nodes (written by the lattice kernel unless it takes the sums)
    double *staging; // [4][N] doubles for field/population transfers
    double *wall_tab; // [2][19] moving-wall terms (StepParams::wall_tab)
    int32_t *flags;  // [0] unstable, [1] domain
    // sentinel polling inside lbm_step: every `check_every` steps (absolute step
    // count) the flags are copied to pinned host memory behind an event;
    // the next poll point waits for that event and reads them
    int check_every;
    int32_t *hflags; // pinned host memory, [2]
    hipEvent_t poll_ev;
    int poll_pending;
    lbm::PartDev P;
    int np, cap;
    // fused-sums step (K = 1): slot buffer (library-owned), its layout, the stamp counter
    double *slots;        // the slot tables in use: ws_slots or a library allocation
    size_t slots_bytes;
    double *ws_slots;     // the workspace's slot region (lbm_config.max_radius), or NULL
    size_t ws_slots_bytes;
    int slot_stride, slot_mx, slot_my, slot_mz, slot_sy, slot_sz, fused;
    int64_t epoch;
    int64_t step;
    double *rec_dev;
    size_t rec_cap;
    void *slab_mem; // slab buffers and slot tables of lbm_step_slabs (library-owned)
    size_t slab_bytes;
    std::vector<lbm_particle> host_parts; // inputs of the last lbm_set_particles
    // differentiated run (lbm_forward_checkpointed / lbm_backward)
    GradState *grad;
    int fresh; // no step since the last lbm_set_particles
    // per-kernel event timing (lbm_profile): while tev[0] is set, the next
    // launch through lbm::launch records its own start and end in tev
    int prof;
    hipEvent_t tev[2];
    int tev_used;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[LBM_NKERNELS];
    int64_t prof_cnt[LBM_NKERNELS];
    std::string err;
};

namespace lbm {

// Launch a kernel on the context stream.  While a step is profiled, the
// kernel's own start and end timestamps go to the context's event pair (the
// time between them excludes the dispatch latency an event recorded on the
// stream around the launch would add).
template <typename... Args, typename F>
inline hipError_t launch_shm(lbm_ctx *c, F kernel, dim3 grid, dim3 block, size_t shmem, Args... args)
{
    if (c->tev[0]) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, c->stream, c->tev[0], c->tev[1], 0, args...);
        c->tev_used = 1;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, c->stream, args...);
    }
    return hipGetLastError();
}
template <typename... Args, typename F>
inline hipError_t launch(lbm_ctx *c, F kernel, dim3 grid, dim3 block, Args... args)
{
    return launch_shm(c, kernel, grid, block, 0, args...);
}

// stream_collide.hip
hipError_t launch_stream_collide(lbm_ctx *c, const void *fin, void *fout);
hipError_t launch_init_uniform(lbm_ctx *c, void *fout, const double *feq);
hipError_t launch_fields(lbm_ctx *c, const void *fin, double *u_out, double *p_out, int solid_only);
hipError_t launch_populations(lbm_ctx *c, const void *fin, double *out, int q0, int nq);
hipError_t launch_set_populations(lbm_ctx *c, const double *fn, void *fout, int q0, int nq);
hipError_t launch_force(lbm_ctx *c, const void *fin, void *fout); // rigid-velocity forcing pass

// particles.hip
hipError_t launch_raster_clear(lbm_ctx *c);
hipError_t launch_reduce(lbm_ctx *c, int step, double *rec, int scratch = 0);
hipError_t launch_rigid_raster(lbm_ctx *c, int update);
hipError_t launch_rigid_substeps(lbm_ctx *c);
hipError_t launch_write_acc(lbm_ctx *c); // acceleration table from rho_s, g, A
hipError_t launch_rigid_fused(lbm_ctx *c, double *rec); // Algorithm 1 + raster from the slots
SlotParams slot_params(lbm_ctx *c, bool on);
hipError_t launch_owner_to_int(lbm_ctx *c, int32_t *out);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_copy_arrays(void *dst, const void *src, int na, size_t bytes_per_array, hipStream_t s);

// adjoint.hip
hipError_t launch_adj_lattice(lbm_ctx *c, const void *fprev, const uint16_t *owner, const double *uext_d,
                              const float *uext_f, const double *acc_d, const float *acc_f, const void *lam_in,
                              void *lam_out, double *asol, double *tau_part, const SlotParams &sl,
                              const double *fpart = nullptr, const double *geo = nullptr, int init = 0);
// The particle adjoints read only the constants rho_s, a, b, Cc and shape of P.
hipError_t launch_adj_rigid(lbm_ctx *c, const PartDev &P, const AdjArraysHost &h);
// particle adjoint of step n from the slots (A_bar^n), then, if rigid, the rigid adjoint of step n - 1
hipError_t launch_adj_fused(lbm_ctx *c, const PartDev &P, const AdjArraysHost &h, const SlotParams &sl,
                            double *Abar_n, int rigid);
hipError_t launch_adj_particles(lbm_ctx *c, const PartDev &P, const uint16_t *owner, const double *asol,
                                const double *rec, double *Abar_out, double *rho_g, double *g_g,
                                double *Xbar_n = nullptr);
hipError_t launch_adj_initial(lbm_ctx *c, const PartDev &P, const double *Upbar, double *rho_g, double *g_g);


// api.hip (shared with grad.hip)
int step_impl(lbm_ctx *c, int64_t nsteps, double *rec_dev);
void free_grad(lbm_ctx *c);

} // namespace lbm
