/*
 * lbm.h -- C ABI of the MI355X constraint-penalization lattice Boltzmann
 * library (liblbmpen.so), after Millet & Liberge, "Constraint Penalization
 * Method in the Lattice Boltzmann Method (LBM) for Fluid-Structure
 * Interaction", arXiv 2511.01629.
 *
 * One context holds one fictitious-domain simulation on one GPU: a single
 * D2Q9 (or D3Q19) lattice covers fluid and solids alike (sec. 2.1); the solids
 * are the nodes marked by the indicator chi of each rigid particle (eq. 9).
 * lbm_step advances the coupled system by whole time steps:
 *
 *   1. pull streaming with halfway bounce-back walls and periodic axes, then
 *      the velocity-based BGK collision (sec. 2.2, eq. 10 and 13) with the
 *      Guo force (eq. 14) and, on solid nodes, the penalization source
 *      S = w/(2 cs^4) (alpha Pi^neq):(c c - cs^2 I) (eq. 17);
 *   2. per-particle momentum sums U = (1/M) sum u, I omega = sum r x u
 *      (sec. 2.4, eq. 22a-b);
 *   3. Algorithm 1 (sec. 2.4): K-sub-step prediction-correction of the
 *      centres with the repulsive collision forces of sec. 2.3 (eq. 19-21),
 *      the collision acceleration A^{n+1}, and the new indicator.
 *
 * Conventions shared by every call:
 *   - Every function returns an int status: LBM_OK (0) or a negative code
 *     below.  Nothing aborts or throws across the ABI.  lbm_last_error gives
 *     a message for the last failing call on a context (NULL: of the last
 *     failed lbm_create or lbm_workspace_size on the calling thread).
 *   - Pointers named `host_*` or documented as host memory are read or written
 *     by the CPU; the library never keeps them after the call returns.
 *   - Lattice units: node (i, j, k) sits at (i, j, k); a wall axis has walls at
 *     -0.5 and n - 0.5; a periodic axis wraps.
 *   - Work is queued on the context's HIP stream (lbm_config.stream, or the
 *     null stream).  lbm_step returns once queued; every lbm_get_* call and
 *     lbm_sync wait for the stream.
 *   - One context is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument; the context is unchanged            */
    LBM_ENOMEM = -2,    /* device allocation failed, or the workspace is too small */
    LBM_EDEVICE = -3,   /* a HIP call failed                                      */
    LBM_ESTATE = -4,    /* call out of order (e.g. no particles set yet)          */
    LBM_EUNSTABLE = -5, /* a velocity became non-finite or |u| > 0.3 (the sentinel) */
    LBM_EDOMAIN = -6    /* a particle left the box or lost all its nodes          */
};

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
/* population storage: arithmetic is FP64 for LBM_F64 and FP32 otherwise; the
 * particle sums and Algorithm 1 are FP64 in every mode */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3 };
enum { LBM_DISK = 0, LBM_ELLIPSE = 1, LBM_SPHERE = 2 };

typedef struct {
    int32_t lattice;     /* LBM_D2Q9 or LBM_D3Q19                                   */
    int32_t storage;     /* LBM_F64 .. LBM_BF16                                      */
    int32_t n[3];        /* nodes per axis; n[2] is ignored (1) for D2Q9             */
    int32_t periodic[3]; /* 1: periodic axis, 0: halfway bounce-back walls           */
    double tau;          /* BGK relaxation time, > 1/2 (sec. 2.2)                     */
    double alpha;        /* penalization parameter of eq. (17); <= 0 selects 1/tau,
                            the value used throughout sec. 3; must be <= 1/tau        */
    double rho_f;        /* fluid density (1 in lattice units)                        */
    double g[3];         /* gravity acceleration (lattice units)                      */
    double u0[3], p0;    /* initial uniform velocity and pressure (f = f^eq(p0, u0))  */
    double eps_p, eps_w; /* collision stiffness, particle-particle and wall (sec. 2.3) */
    double delta;        /* collision range delta (sec. 2.3)                           */
    int32_t K;           /* Algorithm 1 sub-steps (>= 1)                               */
    int32_t collision_form; /* 0: unit direction, C_i = (rho_s,i - rho_f)|g| V_i;
                               1: the printed form (X_i - X_j), C_i = (rho_s,i - rho_f)|g| */
    int32_t gravity_form;   /* 0: a = (1 - rho_f/rho_s) g on solids; 1: (rho_s/rho_f - 1) g */
    double fluid_accel[3];  /* uniform acceleration on fluid nodes (0 in the paper's cases) */
    int32_t penalize_all;   /* 1: apply the penalization source on every node (testing)   */
    int32_t device;         /* HIP device ordinal                                          */
    void *stream;           /* hipStream_t to queue on, or NULL for the null stream         */
    void *workspace;        /* optional caller-owned device buffer of lbm_workspace_size
                               bytes (e.g. from torch); NULL: the library allocates         */
    size_t workspace_bytes; /* size of `workspace`                                          */
    int32_t max_particles;  /* capacity for lbm_set_particles (sizes the workspace)         */
    double wall_velocity[3][2][3]; /* [axis][low, high wall][component]: velocity of the
                               halfway walls (the plane Couette benchmark of sec. 3.1).  A
                               population bounced off a moving wall gains
                               2 w_q (c_q . u_w)/cs^2 (the difference of the equilibria of
                               eq. 13 at the wall velocity).  Nonzero only on the y axis, or
                               the y or z axis in 3D, tangential (no normal component), with
                               every other axis periodic; all zero: fixed walls.            */
    int32_t check_every;    /* lbm_step reads the device sentinel every this many steps (of the
                               absolute step count); 0 selects 64, a negative value never   */
    double rigid_beta;      /* rigid-velocity forcing, an extension beyond the paper (whose
                               constraint acts through the stress, eq. 17): in [0, 1], 0 off.
                               On the nodes of particle i the acceleration gains
                               2 beta (U_i + omega_i x r - u), u the velocity of eq. (15a) with
                               the gravity acceleration alone, r = x - X_i^n, U_i, omega_i the
                               momentum sums of the same step (eq. 22a-b), so the velocity
                               that enters f^eq and the Guo force is (1 - beta) u +
                               beta (U_i + omega_i x r).  Costs a second pass over the solid
                               nodes (and the separate sums kernel) every step.           */
    int32_t no_stress_penalty; /* 1: leave out the penalization source of eq. (17) (to compare
                               the forcing with the paper's stress penalty); 0: the paper   */
    double max_radius;      /* > 0: the largest bounding radius any lbm_set_particles will
                               use; the workspace then also holds the per-particle
                               momentum-sum slot tables of the K = 1 step (so a caller's
                               workspace owns them).  0, or a larger body later: the
                               library allocates those tables at lbm_set_particles.       */
    int32_t fractional_indicator; /* 1: the fractional indicator, an extension beyond the paper
                               (whose indicator is binary) for gradients in the positions:
                               a node of the band |x - X_i| < R_i + 1/2 belongs to particle i
                               (the lowest id where bands meet) with the weight
                               chi = min(1, R_i + 1/2 - |x - X_i|), which multiplies its
                               acceleration (eq. 5-8) and the penalization strength (eq. 17)
                               and weights the momentum sums (eq. 22a-b:
                               N_i = sum chi, U_i = sum chi u / N_i, omega_i from
                               sum chi r x u and sum chi |r|^2, the tensor in 3D) and the
                               mass M_i = rho_s N_i of Algorithm 1.  Disks and spheres only;
                               not with rigid_beta > 0.  The weights vary smoothly with the
                               centres, so lbm_backward also differentiates through them
                               (lbm_grad_positions).  0: the paper's binary indicator.     */
} lbm_config;

typedef struct {
    int32_t shape;     /* LBM_DISK, LBM_ELLIPSE (2D), LBM_SPHERE (3D)                    */
    double rho_s;      /* solid density, > 0                                             */
    double a, b;       /* radius (disk/sphere: a); ellipse semi-axes a >= b >= 1          */
    double x[3];       /* centre X (lattice units)                                       */
    double theta;      /* 2D orientation of the major axis from +x (radians)              */
    /* outputs of lbm_get_particles (ignored by lbm_set_particles) */
    double U[3], omega[3];           /* U^n, omega^n measured on the current state       */
    double U_prev[3], omega_prev[3]; /* U^{n-1}, omega^{n-1} held for Algorithm 1          */
    double A[3];                     /* collision acceleration A^n of Algorithm 1          */
    int32_t n_nodes;                 /* |Omega_i|, nodes owned now                          */
} lbm_particle;

/* Bytes of device memory a context with this configuration needs (for a
 * caller-provided workspace).  Host pointers only. */
int lbm_workspace_size(const lbm_config *cfg, size_t *bytes);

/* Validate cfg, allocate (or carve the workspace), and initialise every node
 * to f^eq(p0, u0) (eq. 13), also next to moving walls.  Size limit: d*N <
 * 2^31 (node offsets and the [d][N] solid-velocity field are 32-bit); from
 * Q*N >= 2^31 on, the lattice update addresses populations with 64-bit
 * offsets (the same arithmetic, so the same bits; setting LBM_WIDE_OFFSETS=1
 * in the environment before this call selects that kernel on any lattice, a
 * testing aid).  EINVAL: tau <= 1/2,
 * alpha > 1/tau, n <= 0, d*N >= 2^31, unknown lattice/storage, max_particles
 * outside [0, 65534], K < 1, non-positive rho_f, eps_p, eps_w or delta, and
 * moving walls outside their limits (on x, on a periodic axis, on two axes,
 * with a normal component or a non-finite value, or with another axis not
 * periodic).  *out receives the context; it is freed by lbm_destroy. */
int lbm_create(const lbm_config *cfg, lbm_ctx **out);

/* Free the context and everything it allocated (never the caller's workspace). */
int lbm_destroy(lbm_ctx *ctx);

/* Copy n particles in (host array), rasterise the indicator (eq. 9: closed
 * set, the lowest index owns a shared node, FP64 tests with no contraction,
 * minimum image on periodic axes), measure U^0 and omega^0 on the current
 * populations (eq. 22a-b), set U^{-1} = U^0, omega^{-1} = omega^0, A = 0.
 * Any earlier differentiated run is discarded (lbm_backward then gives ESTATE).
 * EINVAL, with the context unchanged: n > max_particles, a bad shape/size, a
 * body crossing a wall, a radius too large for a periodic axis
 * (a + 2 >= n/2), or a body that would own no node (its shape lies inside
 * lower-index bodies; the host counts the nodes each body claims with the
 * inclusion test of the device before anything changes).  Should the device
 * still find a body with no node (an ellipse whose boundary passes through a
 * node, where host and device cos/sin may differ in the last bit), the call
 * returns EINVAL and leaves the context with no particles. */
int lbm_set_particles(lbm_ctx *ctx, const lbm_particle *host_particles, int32_t n);

/* Queue nsteps >= 0 full time steps (stream-collide-penalize, sums,
 * Algorithm 1, re-rasterisation).  With no particles set, only the lattice
 * update runs (pure fluid).
 *
 * Sentinel: the lattice kernel raises a device flag when a node velocity is
 * non-finite or exceeds 0.3 in magnitude (unstable), and the particle kernels
 * one when a centre leaves the box or a body loses all its nodes (domain).
 * After every check_every-th step (absolute count) lbm_step queues a copy of
 * the flags to pinned host memory; at the next such step it waits for that
 * copy (so the host never runs more than 2 check_every steps ahead of the
 * device) and returns LBM_EUNSTABLE or LBM_EDOMAIN, queueing nothing more,
 * if a flag was set: a diverging run stops within 2 check_every steps of the
 * step that tripped it, and its state stays readable.  The particle kernels
 * of the fused K = 1 step skip partner pairs farther apart than
 * R_i + R_j + delta + 0.6, which is exact while the sentinel holds (every
 * |u|, hence every |U_bar|, is at most 0.3); on the steps between a trip and
 * the stop such forces may be missed. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* lbm_step with the lattice cut into nslabs slabs along its last axis (y in
 * 2D, z in 3D), the layout a run over nslabs GPUs would give each GPU,
 * emulated on this one: each slab's populations live in buffers of their
 * own with one halo row (plane) on each side, updated by a kernel of their
 * own and exchanged every step by explicit device copies; each slab writes
 * its solid nodes' momentum sums (eq. 22a-b) to a table of its own, and the
 * tables are merged before Algorithm 1 runs once on the result (the
 * cross-slab particle sums).  The state afterwards equals lbm_step's bit for
 * bit.  The slab buffers are allocated by the library (about 2 Q s N bytes
 * plus a slot table per extra slab) and kept for later calls.  EINVAL:
 * nslabs outside [1, min(64, rows of the split axis)], K > 1, rigid_beta > 0,
 * or a slab buffer of Q*(rows + 2)*plane >= 2^31 elements (the slab kernel's
 * offsets are 32-bit: a larger lattice needs more slabs).
 * Waits for the stream and reports the sentinel like lbm_sync. */
int lbm_step_slabs(lbm_ctx *ctx, int64_t nsteps, int32_t nslabs);

/* As lbm_step, and write a per-step record of every particle into host_rec:
 * nsteps x n x 14 doubles, per particle X[3] theta U[3] omega[3] A[3] N of
 * step n (values before that step's update).  Waits for the stream. */
int lbm_step_record(lbm_ctx *ctx, int64_t nsteps, double *host_rec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * lbm_step_record with no allocation.  The per-step records go through a
 * static device array of LBM_NOALLOC_REC_DOUBLES doubles (8 MiB), one per
 * GPU, held until the process ends, instead of memory the library would
 * allocate; lbm_step_record's results, bit for bit.  EINVAL if nsteps x
 * max(n, 1) x 20 exceeds LBM_NOALLOC_REC_DOUBLES (e.g. 3276 steps of 16
 * particles); ESTATE while lbm_profile is on (it creates events); EDEVICE if
 * the array's address cannot be looked up on this device.  Every
 * context on a GPU shares that GPU's array, which keeps the last call's
 * records: calls that overlap in time on one GPU (other host threads, other
 * streams) race.  Waits for the stream. */
#define LBM_NOALLOC_REC_DOUBLES (1 << 20)
int lbm_step_record_noalloc(lbm_ctx *ctx, int64_t nsteps, double *host_rec);

/* Wait for queued work; report LBM_EUNSTABLE / LBM_EDOMAIN if the device
 * sentinel tripped since the context was created. */
int lbm_sync(lbm_ctx *ctx);

/* Macroscopic fields of the current step (eq. 15a-b), host memory, FP64,
 * node-major: u[N][d] (d = 2 or 3), p[N], owner[N] (-1 = fluid).  Any pointer
 * may be NULL.  N = n[0] n[1] n[2], x fastest. */
int lbm_get_fields(lbm_ctx *ctx, double *host_u, double *host_p, int32_t *host_owner);

/* The same fields into device memory of the context's device (e.g. torch
 * tensors), same layouts; any pointer may be NULL.  Queued on the context
 * stream and not waited for: the caller orders its reads on that stream.
 * The sentinel is not read (lbm_sync does). */
int lbm_get_fields_device(lbm_ctx *ctx, double *dev_u, double *dev_p, int32_t *dev_owner);

/* Populations f^n of the current step (after streaming, before collision),
 * host memory, FP64, direction-major [Q][N]. */
int lbm_get_populations(lbm_ctx *ctx, double *host_f);

/* Replace the populations by host_f ([Q][N] FP64, rounded to the storage
 * type).  Particle state is unchanged; call lbm_set_particles afterwards to
 * re-measure U^0. */
int lbm_set_populations(lbm_ctx *ctx, const double *host_f);

/* Current particle state into host_particles[0..n): centre, orientation, U^n
 * and omega^n measured now, U^{n-1}, omega^{n-1}, A^n, node count. */
int lbm_get_particles(lbm_ctx *ctx, lbm_particle *host_particles, int32_t n);

/* ---- parameters and the state between steps ----
 *
 * lbm_set_params: replace the solid densities (host rho_s[0..np), or NULL to
 * keep them), tau (> 1/2; a value <= 0 keeps it; alpha follows it when alpha
 * <= 0 was given at lbm_create) and the gravity vector (host g[3], or NULL
 * to keep it).  They act from the next step on: the solid-node acceleration
 * (1 - rho_f/rho_s,i) g + A_i (sec. 2.1, 2.4), the collision constants C_i of
 * sec. 2.3 and the BGK rate (eq. 10).  Right after lbm_set_particles (or a
 * load of a state saved then), U^0 and omega^0 are measured again with the
 * new parameters and U^{-1} = U^0, as lbm_set_particles would have.  Any
 * earlier differentiated run is discarded.  EINVAL (nothing changed): tau
 * <= 1/2, a fixed alpha above 1/tau, a non-positive or non-finite density or
 * a non-finite g.  Waits for the stream.
 *
 * lbm_state_size / lbm_save_state / lbm_load_state: the whole state that the
 * next step starts from, as one byte blob (the state Algorithm 1 carries
 * from step to step, sec. 2.4):
 *   header (lattice, storage, sizes, periodic axes, particle count, step
 *   counter, tau, g, whether the state is the one right after
 *   lbm_set_particles); per particle rho_s, a, b, shape, X^n, theta^n,
 *   U^{n-1}, omega^{n-1}, A^n (FP64); then the populations in the storage
 *   type, raw.
 * The indicator is not stored: it is a function of X^n and theta^n (eq. 9)
 * and is rasterised again on load, bit for bit as the step produced it.
 * `buf` may be host or device memory (any address the HIP runtime
 * recognises; unified addressing); lbm_state_size gives its size in bytes.
 * Save waits for the stream.  Load validates the header against the context
 * (same lattice, storage, sizes and periodic axes; particle count <=
 * max_particles; else EINVAL and nothing changes), installs the parameters
 * and the particles (as lbm_set_particles, without measuring U), the
 * populations and the step counter, and clears the sentinel; the sentinel is
 * not stored.  run(2n) equals run(n) + save + load (into this or another
 * context of the same configuration) + run(n), bit for bit.  A loaded state
 * with non-finite populations trips the sentinel on the first step. */
int lbm_set_params(lbm_ctx *ctx, const double *host_rho_s, double tau, const double *host_g);
int lbm_state_size(const lbm_ctx *ctx, size_t *bytes);
int lbm_save_state(lbm_ctx *ctx, void *buf);
int lbm_load_state(lbm_ctx *ctx, const void *buf);

/* ---- differentiated runs (extension beyond the paper) ----
 * Gradients of a loss of the final particle centres with respect to the
 * solid densities rho_s,i, tau (alpha follows it when alpha <= 0 was given),
 * |g| (the direction of g fixed) and the initial centres X^0, by a
 * hand-written adjoint of the step.  With the paper's binary indicator the
 * derivative is that of the step map with the indicator sequence frozen (a
 * binary indicator makes the loss piecewise smooth); with the fractional
 * indicator (lbm_config.fractional_indicator) the node weights are smooth in
 * the centres and the adjoint carries their derivative, so the gradient in
 * X^0 is that of the loss itself (while no node changes owner where two
 * bands meet).
 *
 * lbm_forward_checkpointed: run nsteps >= 1 steps starting right after
 * lbm_set_particles (else ESTATE; K must be 1, rigid_beta 0, the stress
 * penalty on and Q*N < 2^31 -- the lattice adjoint's offsets are 32-bit --
 * else EINVAL, also from lbm_grad_workspace_size), snapshotting the state every `every`
 * steps and keeping every step's particle record (device memory allocated
 * by the library: about (nsteps/every + 1) population buffers plus small
 * records).  Waits for the stream.
 *
 * lbm_backward: host dL_dX (n x 3 doubles, the loss gradient with respect
 * to the final centres) in; host g_rho_s (n), g_tau, g_gmag out (any may be
 * NULL).  Recomputes each segment from its snapshot (`every` extra
 * population buffers) and sweeps the adjoint backwards.  The state at the
 * end of the differentiated run is restored afterwards.  ESTATE without a
 * preceding lbm_forward_checkpointed; may be called repeatedly with other
 * seeds.  The snapshot memory is released by lbm_set_particles or
 * lbm_destroy. */
int lbm_forward_checkpointed(lbm_ctx *ctx, int64_t nsteps, int32_t every);
/* (A differentiated run may also start right after lbm_load_state of a state
 * saved right after lbm_set_particles; lbm_set_params, lbm_set_particles and
 * lbm_load_state discard the run's checkpoints.) */
int lbm_backward(lbm_ctx *ctx, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag);

/* The gradient with respect to the initial centres X^0 from the last
 * lbm_backward or lbm_backward_ws: host g_X0 (n x 3 doubles; the unused axis
 * of a 2D lattice reads 0) out.  With the binary indicator it is the
 * frozen-indicator derivative (the centres move the bodies but no node
 * weight).  ESTATE before a backward sweep of the current particle set;
 * EINVAL for NULL pointers. */
int lbm_grad_positions(lbm_ctx *ctx, double *g_X0);

/* The same two calls with every device buffer they need taken from
 * caller-owned device memory (e.g. torch tensors) instead of the library's
 * allocations: lbm_grad_workspace_size gives, for a run of nsteps steps with
 * checkpoints every `every` steps on the context as it is set up now, the
 * bytes of the forward workspace (the per-step particle records and the
 * snapshots, or every frame when every = 1; it must stay allocated and
 * untouched until the run's last lbm_backward_ws, or until the next
 * differentiated run, lbm_set_particles, lbm_set_params or lbm_load_state)
 * and of the backward workspace (segment frames, adjoint populations and
 * partial sums; needed only during the call).  Each workspace must start on
 * a 256-byte boundary (torch's allocations do; the indicator frames inside are
 * updated with 32-bit atomics).  ENOMEM if a workspace is smaller than that;
 * EINVAL for a NULL or misaligned workspace.  The library frees neither. */
int lbm_grad_workspace_size(lbm_ctx *ctx, int64_t nsteps, int32_t every, size_t *fwd_bytes, size_t *bwd_bytes);
int lbm_forward_checkpointed_ws(lbm_ctx *ctx, int64_t nsteps, int32_t every, void *dev_ws, size_t ws_bytes);
int lbm_backward_ws(lbm_ctx *ctx, const double *dL_dX, double *g_rho_s, double *g_tau, double *g_gmag, void *dev_ws,
                    size_t ws_bytes);

/* Per-kernel timing with HIP events (measurement aid).  While enabled,
 * every kernel lbm_step queues records its own start and end in a pair of
 * events (the kernel's execution, without the dispatch latency), and lbm_step waits
 * for the stream before returning.  lbm_profile_read returns, per kernel
 * class, the summed duration in milliseconds and the launch count since the
 * last reset (reset = 1 clears them afterwards).  Classes, in order:
 * 0 stream-collide-penalize, 1 momentum sums (with the indicator clear; no
 * launches where the lattice kernel takes the sums, which it does with K = 1
 * whenever the set-up found a slot layout), 2 Algorithm 1 with the new
 * indicator (K = 1) or the sub-step integration (K > 1), 3 the indicator
 * after sub-steps (K > 1 only), 4 the rigid-velocity forcing pass
 * (rigid_beta > 0 only).  host_ms and host_count are host arrays of
 * LBM_NKERNELS. */
#define LBM_NKERNELS 5
int lbm_profile(lbm_ctx *ctx, int32_t enable);
int lbm_profile_read(lbm_ctx *ctx, double *host_ms, int64_t *host_count, int32_t reset);

/* Plain device-to-device copy of `bytes` bytes with a streaming kernel of the
 * library (16-byte vector loads/stores), queued on `stream` (hipStream_t or
 * NULL).  dst and src are device pointers, 16-byte aligned, not overlapping;
 * bytes is a multiple of 16 (EINVAL otherwise, and for a NULL pointer with
 * bytes > 0; EDEVICE if the launch fails).  Used as the achievable-bandwidth
 * reference of the measurements. */
int lbm_copy(void *dst, const void *src, size_t bytes, void *stream);

/* The same copy over `narrays` arrays of `bytes_per_array` bytes each, laid
 * out one after another at src and dst (array a at a * bytes_per_array), in
 * one kernel whose threads each move one 16-byte word of every array, loads
 * first: narrays streams read and narrays written together, the access
 * pattern of a lattice update over Q population arrays.  narrays in 1..32
 * (EINVAL otherwise); pointers and bytes_per_array as for lbm_copy.  Used as
 * the bandwidth reference of that pattern in the measurements. */
int lbm_copy_arrays(void *dst, const void *src, int32_t narrays, size_t bytes_per_array, void *stream);

/* Number of completed steps. */
int lbm_get_step(const lbm_ctx *ctx, int64_t *step);

/* Message for the last failing call on ctx (never NULL).  With ctx = NULL:
 * the last lbm_workspace_size or lbm_create failure on the calling thread. */
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
