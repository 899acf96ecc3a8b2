// ctx.h -- the context behind the C ABI and the launchers each kernel file
// provides.  Private to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// Device arrays of the particle state, structure-of-arrays, FP64.
struct PartDev {
    double *X, *Xn, *theta, *U, *W, *Uprev, *Wprev, *A; // [cap*3] (theta [cap]); Xn: next centres
    double *rho_s, *a, *b, *Cc;                    // [cap]; Cc = collision constant C_i
    double *acc_d;                                 // [cap*3] solid-node acceleration (FP64 mode)
    float *acc_f;                                  // [cap*3] the same in FP32
    double *sums;                                  // [cap*16] momentum sums of the last reduction
    double *Ub, *dth;                              // U_bar = (U^n + U^{n-1})/2 [cap*3], theta increment [cap]
    double *Y, *Ys, *Y2, *Dc;                      // [cap*3] sub-step scratch (Dc: summed corrections)
    int32_t *shape, *N;                            // [cap]
    int32_t *lo, *hi;                              // [cap*3] scan box (unwrapped node coords)
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
};

struct RigidParams {
    double rho_f, gmag, g[3];
    double eps_p, eps_w, delta;
    int K, cform, gform, np, d;
};

} // namespace lbm

struct lbm_ctx {
    lbm_config cfg;
    int Q, d;
    lbm::Geom geo;
    lbm::StepParams sp;
    lbm::RigidParams rp;
    hipStream_t stream;
    int device;
    bool own_mem;
    void *ws;
    size_t ws_bytes;
    void *f[2]; // post-collision populations f~ (ping-pong), [Q][N] raw storage
    int cur;    // f[cur] holds f~ of the last completed step
    uint16_t *owner;
    double *usol;    // [d][N] velocity on solid nodes (written by the fused kernel)
    double *staging; // [4][N] doubles for field/population transfers
    int32_t *flags;  // [0] unstable, [1] domain
    lbm::PartDev P;
    int np, cap;
    int64_t step;
    double *rec_dev;
    size_t rec_cap;
    std::vector<lbm_particle> host_parts; // inputs of the last lbm_set_particles
    // per-kernel event timing (lbm_profile)
    int prof;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[LBM_NKERNELS];
    int64_t prof_cnt[LBM_NKERNELS];
    std::string err;
};

namespace lbm {

// stream_collide.hip
hipError_t launch_stream_collide(lbm_ctx *c, const void *fin, void *fout);
hipError_t launch_init_uniform(lbm_ctx *c, void *fout, const double *feq);
hipError_t launch_fields(lbm_ctx *c, const void *fin, double *u_out, double *p_out, int solid_only);
hipError_t launch_populations(lbm_ctx *c, const void *fin, double *out, int q0, int nq);
hipError_t launch_set_populations(lbm_ctx *c, const double *fn, void *fout, int q0, int nq);

// particles.hip
hipError_t launch_raster_clear(lbm_ctx *c);
hipError_t launch_reduce(lbm_ctx *c, int step, double *rec);
hipError_t launch_rigid_raster(lbm_ctx *c, int update);
hipError_t launch_rigid_substeps(lbm_ctx *c);
hipError_t launch_owner_to_int(lbm_ctx *c, int32_t *out);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

} // namespace lbm
