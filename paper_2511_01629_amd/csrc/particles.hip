// particles.hip -- indicator rasterisation, per-particle momentum sums and
// the rigid-body update (Algorithm 1) for gfx950.  All particle arithmetic is
// FP64.
//
// A step runs two particle kernels after the lattice update, one workgroup
// per particle each:
//
//  k_reduce<STEP>   momentum sums over the particle's scan box (sec. 2.4,
//                   eq. 22a-b); each thread accumulates in a fixed order and a
//                   fixed LDS tree combines the partials, so results are
//                   bitwise reproducible.  The owned nodes are reset to FLUID
//                   as they are read, which clears the indicator.
//  k_rigid_raster   Algorithm 1 (sec. 2.4) for the particle, with the
//                   collision forces of sec. 2.3 (eq. 19-21) summed over the
//                   other particles across the workgroup's lanes, then the
//                   particle's new indicator (sec. 2.1, eq. 9): every node of
//                   its closed shape is claimed with a 16-bit atomic minimum,
//                   so a shared node goes to the lowest index.  The inside
//                   tests are FP64 with explicit round-to-nearest products and
//                   sums, so no contraction moves a node across a boundary.
//
// New centres go to a second buffer (P.Xn), swapped by the host, because every
// workgroup reads all old centres.  With K > 1 sub-steps, one workgroup
// (k_rigid_substeps) integrates all particles together, then k_rigid_raster
// only rasterises.
#include "ctx.h"
#include "lattice.h"

namespace lbm {

__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }

// inside test of eq. (9) on the displacement (dx, dy, dz) from the centre
__device__ __forceinline__ bool inside_shape(int shape, double a, double b, double cs, double sn, double dx, double dy,
                                             double dz)
{
    if (shape == LBM_DISK) return dadd(dmul(dx, dx), dmul(dy, dy)) <= dmul(a, a);
    if (shape == LBM_SPHERE) return dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz)) <= dmul(a, a);
    const double xi = dadd(dmul(cs, dx), dmul(sn, dy));
    const double eta = dadd(dmul(-sn, dx), dmul(cs, dy));
    return dadd(dmul(dmul(b, b), dmul(xi, xi)), dmul(dmul(a, a), dmul(eta, eta))) <= dmul(dmul(a, a), dmul(b, b));
}


// 16-bit atomic minimum through a 32-bit compare-and-swap on the aligned word.
__device__ __forceinline__ void atomic_min_u16(uint16_t *addr, uint16_t val)
{
    uintptr_t a = reinterpret_cast<uintptr_t>(addr);
    unsigned int *word = reinterpret_cast<unsigned int *>(a & ~uintptr_t(3));
    const unsigned int shift = (a & 2) ? 16u : 0u;
    unsigned int old = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
        const unsigned int cur = (old >> shift) & 0xFFFFu;
        if (cur <= val) return;
        const unsigned int nw = (old & ~(0xFFFFu << shift)) | ((unsigned int)val << shift);
        const unsigned int prev = atomicCAS(word, old, nw);
        if (prev == old) return;
        old = prev;
    }
}

struct BoxIter {
    int lo[3], ext[3];
    long cells;
};

__device__ __forceinline__ BoxIter load_box(const PartDev &P, int i, int d)
{
    BoxIter b;
    b.cells = 1;
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = (k < d) ? P.lo[3 * i + k] : 0;
        b.ext[k] = (k < d) ? P.hi[3 * i + k] - P.lo[3 * i + k] + 1 : 1;
        if (b.ext[k] < 0) b.ext[k] = 0;
        b.cells *= b.ext[k];
    }
    return b;
}

__global__ __launch_bounds__(256) void k_raster_clear(uint16_t *__restrict__ owner, PartDev P, Geom g, int d)
{
    const int i = blockIdx.x;
    const BoxIter b = load_box(P, i, d);
    for (long cidx = threadIdx.x; cidx < b.cells; cidx += blockDim.x) {
        const int lx = (int)(cidx % b.ext[0]);
        const int ly = (int)((cidx / b.ext[0]) % b.ext[1]);
        const int lz = (int)(cidx / ((long)b.ext[0] * b.ext[1]));
        const int x = wrap(b.lo[0] + lx, g.nx), y = wrap(b.lo[1] + ly, g.ny), z = wrap(b.lo[2] + lz, g.nz);
        owner[x + g.nx * (y + g.ny * z)] = FLUID;
    }
}

// Per-particle sums over the owned nodes of the scan box.
//  2D: [0] N, [1..2] sum u, [3] sum r x u (z), [4] sum |r|^2
//  3D: [0] N, [1..3] sum u, [4..6] sum r x u, [7..12] inertia xx yy zz xy xz yz
// then U = sum u / N and omega = (sum r x u)/(sum |r|^2) (2D) or I^{-1} L (3D).
//
// STEP = true (inside a time step): every owned node is reset to FLUID once
// read -- a node owned by particle i is read by no other particle's sum, so
// this clears the whole indicator for the next rasterisation -- and the
// quantities Algorithm 1 needs are prepared: U_bar = (U^n + U^{n-1})/2,
// dtheta = (omega^n + omega^{n-1})/2, then U^{n-1} <- U^n, omega^{n-1} <- omega^n.
// rec (optional) receives the step's record (layout REC_STRIDE in ctx.h).
template <int D, bool STEP>
__global__ __launch_bounds__(256) void k_reduce(uint16_t *__restrict__ owner, const double *__restrict__ usol,
                                                 PartDev P, Geom g, double *__restrict__ rec)
{
    constexpr int NS = (D == 2) ? 5 : 13;
    const int i = blockIdx.x;
    const BoxIter b = load_box(P, i, D);
    const double X0 = P.X[3 * i], X1 = P.X[3 * i + 1], X2 = (D == 3) ? P.X[3 * i + 2] : 0.0;
    const int N = (int)g.N;
    double s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = 0.0;
    for (long cidx = threadIdx.x; cidx < b.cells; cidx += blockDim.x) {
        const int lx = (int)(cidx % b.ext[0]);
        const int ly = (int)((cidx / b.ext[0]) % b.ext[1]);
        const int lz = (int)(cidx / ((long)b.ext[0] * b.ext[1]));
        const int xu = b.lo[0] + lx, yu = b.lo[1] + ly, zu = b.lo[2] + lz;
        const int node = wrap(xu, g.nx) + g.nx * (wrap(yu, g.ny) + g.ny * wrap(zu, g.nz));
        if (owner[node] != (uint16_t)i) continue;
        if (STEP) owner[node] = FLUID;
        const double rx = (double)xu - X0, ry = (double)yu - X1;
        const double ux = usol[node], uy = usol[N + node];
        s[0] += 1.0;
        s[1] += ux;
        s[2] += uy;
        if constexpr (D == 2) {
            s[3] += rx * uy - ry * ux;
            s[4] += rx * rx + ry * ry;
        } else {
            const double rz = (double)zu - X2, uz = usol[2 * N + node];
            s[3] += uz;
            s[4] += ry * uz - rz * uy;
            s[5] += rz * ux - rx * uz;
            s[6] += rx * uy - ry * ux;
            const double rr = rx * rx + ry * ry + rz * rz;
            s[7] += rr - rx * rx;
            s[8] += rr - ry * ry;
            s[9] += rr - rz * rz;
            s[10] -= rx * ry;
            s[11] -= rx * rz;
            s[12] -= ry * rz;
        }
    }
    __shared__ double red[NS][256];
#pragma unroll
    for (int k = 0; k < NS; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < NS; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double t[NS];
    for (int k = 0; k < NS; ++k) {
        t[k] = red[k][0];
        P.sums[16 * i + k] = t[k];
    }
    const int cnt = (int)t[0];
    P.N[i] = cnt;
    double U[3] = {0, 0, 0}, W[3] = {0, 0, 0};
    if (cnt > 0) {
        if constexpr (D == 2) {
            U[0] = t[1] / t[0];
            U[1] = t[2] / t[0];
            W[2] = t[3] / t[4];
        } else {
            U[0] = t[1] / t[0];
            U[1] = t[2] / t[0];
            U[2] = t[3] / t[0];
            const double L0 = t[4], L1 = t[5], L2 = t[6];
            const double a = t[7], e = t[8], f = t[9], bxy = t[10], cxz = t[11], dyz = t[12];
            // inverse of the symmetric tensor [[a,b,c],[b,e,d],[c,d,f]] by cofactors
            const double A00 = e * f - dyz * dyz, A01 = cxz * dyz - bxy * f, A02 = bxy * dyz - cxz * e;
            const double A11 = a * f - cxz * cxz, A12 = bxy * cxz - a * dyz, A22 = a * e - bxy * bxy;
            const double det = a * A00 + bxy * A01 + cxz * A02;
            W[0] = (A00 * L0 + A01 * L1 + A02 * L2) / det;
            W[1] = (A01 * L0 + A11 * L1 + A12 * L2) / det;
            W[2] = (A02 * L0 + A12 * L1 + A22 * L2) / det;
        }
    }
    for (int k = 0; k < 3; ++k) {
        P.U[3 * i + k] = U[k];
        P.W[3 * i + k] = W[k];
    }
    if (STEP) {
        if (rec) {
            double *r = rec + REC_STRIDE * i;
            for (int k = 0; k < 3; ++k) {
                r[k] = P.X[3 * i + k];
                r[4 + k] = U[k];
                r[7 + k] = W[k];
                r[10 + k] = P.A[3 * i + k];
                r[14 + k] = P.Uprev[3 * i + k];
            }
            r[3] = P.theta[i];
            r[13] = (double)cnt;
        }
        P.dth[i] = 0.5 * (W[2] + P.Wprev[3 * i + 2]);
        for (int k = 0; k < 3; ++k) {
            P.Ub[3 * i + k] = 0.5 * (U[k] + P.Uprev[3 * i + k]);
            P.Uprev[3 * i + k] = U[k];
            P.Wprev[3 * i + k] = W[k];
        }
    }
}

// Contribution of particle j to the particle-particle force on i at centres
// Yi, Yj (sec. 2.3, eq. 19), minimum image on periodic axes.
__device__ __forceinline__ void pair_force(const double *Yi, const double *Yj, double Ri, double Rj, double Ci,
                                           const RigidParams &rp, const Geom &g, double F[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    double dv[3] = {0, 0, 0};
    for (int k = 0; k < rp.d; ++k) {
        dv[k] = Yi[k] - Yj[k];
        if (per[k]) {
            const double h = 0.5 * n[k];
            if (dv[k] > h) dv[k] -= n[k];
            else if (dv[k] < -h) dv[k] += n[k];
        }
    }
    const double cut = Ri + Rj + rp.delta;
    const double d2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
    if (d2 > cut * cut * (1.0 + 1e-12)) return; // far pair: no square root
    const double dist = sqrt(d2);
    if (dist > cut) return;
    const double s = (cut - dist) / rp.delta;
    const double mag = Ci / rp.eps_p * s * s;
    const double scale = rp.cform == 1 ? mag : mag / dist;
    for (int k = 0; k < rp.d; ++k) F[k] += scale * dv[k];
}

// Particle-wall forces through the mirror particle (sec. 2.3, eq. 20).
__device__ __forceinline__ void wall_force(const double *Yi, double Ri, double Ci, const RigidParams &rp, const Geom &g,
                                           double F[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    for (int k = 0; k < rp.d; ++k) {
        if (per[k]) continue;
        const double walls[2] = {-0.5, n[k] - 0.5};
        for (int s = 0; s < 2; ++s) {
            const double dv = Yi[k] - (2.0 * walls[s] - Yi[k]); // to the mirror particle
            const double dist = fabs(dv);
            if (dist > 2.0 * Ri + rp.delta) continue;
            const double q = (2.0 * Ri + rp.delta - dist) / rp.delta;
            const double mag = Ci / rp.eps_w * q * q;
            F[k] += rp.cform == 1 ? mag * dv : mag * dv / dist;
        }
    }
}

// Solid-node acceleration a_i = b_i g + A_i of the lattice kernel
// (b_i = 1 - rho_f/rho_s,i, or rho_s,i/rho_f - 1 with gravity_form 1).
__device__ __forceinline__ void write_acc(PartDev &P, const RigidParams &rp, int i)
{
    const double bi = rp.gform == 0 ? 1.0 - rp.rho_f / P.rho_s[i] : P.rho_s[i] / rp.rho_f - 1.0;
    for (int k = 0; k < 3; ++k) {
        const double acc = (k < rp.d) ? bi * rp.g[k] + P.A[3 * i + k] : 0.0;
        P.acc_d[3 * i + k] = acc;
        P.acc_f[3 * i + k] = (float)acc;
    }
}

// Claim the nodes of particle i at centre Xc: scan box (bounding radius + 2
// nodes, clipped on wall axes) stored for the sums and the next clear, then a
// 16-bit atomic minimum on every node inside the shape.  Called by the whole
// workgroup; s_X holds the centre.
__device__ void raster_particle(uint16_t *__restrict__ owner, PartDev &P, const Geom &g, int d, int i,
                                const double *s_X, int *s_lo, int *s_hi)
{
    if (threadIdx.x == 0) {
        const int n[3] = {g.nx, g.ny, g.nz};
        const int per[3] = {g.per_x, g.per_y, g.per_z};
        const double R = P.a[i];
        for (int k = 0; k < 3; ++k) {
            int lo = 0, hi = -1; // empty box for a non-finite or runaway centre
            if (k >= d) {
                lo = hi = 0;
            } else if (fabs(s_X[k]) < 1e9) {
                lo = (int)floor(s_X[k] - R) - 2;
                hi = (int)ceil(s_X[k] + R) + 2;
                if (!per[k]) {
                    lo = lo < 0 ? 0 : lo;
                    hi = hi > n[k] - 1 ? n[k] - 1 : hi;
                }
            }
            s_lo[k] = lo;
            s_hi[k] = hi;
            if (k < d) {
                P.lo[3 * i + k] = lo;
                P.hi[3 * i + k] = hi;
            }
        }
    }
    __syncthreads();
    const int ext[3] = {s_hi[0] - s_lo[0] + 1, s_hi[1] - s_lo[1] + 1, s_hi[2] - s_lo[2] + 1};
    if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;
    const long cells = (long)ext[0] * ext[1] * ext[2];
    const int shape = P.shape[i];
    const double a = P.a[i], b = P.b[i];
    double cs = 1.0, sn = 0.0;
    if (shape == LBM_ELLIPSE) {
        cs = cos(P.theta[i]);
        sn = sin(P.theta[i]);
    }
    const double X0 = s_X[0], X1 = s_X[1], X2 = (d == 3) ? s_X[2] : 0.0;
    for (long cidx = threadIdx.x; cidx < cells; cidx += blockDim.x) {
        const int lx = (int)(cidx % ext[0]);
        const int ly = (int)((cidx / ext[0]) % ext[1]);
        const int lz = (int)(cidx / ((long)ext[0] * ext[1]));
        const int xu = s_lo[0] + lx, yu = s_lo[1] + ly, zu = s_lo[2] + lz;
        const double dx = (double)xu - X0, dy = (double)yu - X1, dz = (d == 3) ? (double)zu - X2 : 0.0;
        if (!inside_shape(shape, a, b, cs, sn, dx, dy, dz)) continue;
        const int x = wrap(xu, g.nx), y = wrap(yu, g.ny), z = wrap(zu, g.nz);
        atomic_min_u16(owner + (x + g.nx * (y + g.ny * z)), (uint16_t)i);
    }
}

// One workgroup per particle.  update = 1 (K = 1): Algorithm 1 for particle
// i -- the collision forces at X^n and at the prediction X^n + U_bar summed
// over all other particles in parallel and over the walls, the correction,
// X^{n+1} into P.Xn, A^{n+1}, theta^{n+1} -- then the new indicator of i.
// update = 0: rasterise i at P.X and refresh its acceleration entry.
// The indicator must be all FLUID on entry (cleared by the step-mode sums).
__global__ __launch_bounds__(256) void k_rigid_raster(uint16_t *__restrict__ owner, PartDev P, RigidParams rp, Geom g,
                                                      int update, int32_t *__restrict__ flags)
{
    const int i = blockIdx.x, d = rp.d;
    __shared__ double s_X[3];
    __shared__ int s_lo[3], s_hi[3];
    __shared__ double red[6][256];
    if (update) {
        const double Ri = P.a[i], Ci = P.Cc[i];
        double Xi[3], Yi[3];
        for (int k = 0; k < 3; ++k) {
            Xi[k] = P.X[3 * i + k];
            Yi[k] = Xi[k] + (k < d ? P.Ub[3 * i + k] : 0.0);
        }
        double F0[3] = {0, 0, 0}, F1[3] = {0, 0, 0};
        for (int j = threadIdx.x; j < rp.np; j += blockDim.x) {
            if (j == i) continue;
            double Xj[3], Yj[3];
            for (int k = 0; k < 3; ++k) {
                Xj[k] = P.X[3 * j + k];
                Yj[k] = Xj[k] + (k < d ? P.Ub[3 * j + k] : 0.0);
            }
            const double Rj = P.a[j];
            pair_force(Xi, Xj, Ri, Rj, Ci, rp, g, F0);
            pair_force(Yi, Yj, Ri, Rj, Ci, rp, g, F1);
        }
        for (int k = 0; k < 3; ++k) {
            red[k][threadIdx.x] = F0[k];
            red[3 + k][threadIdx.x] = F1[k];
        }
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double G0[3] = {red[0][0], red[1][0], red[2][0]}, G1[3] = {red[3][0], red[4][0], red[5][0]};
            wall_force(Xi, Ri, Ci, rp, g, G0);
            wall_force(Yi, Ri, Ci, rp, g, G1);
            const double M = P.rho_s[i] * (double)P.N[i];
            const double c = M > 0.0 ? 1.0 / (2.0 * M) : 0.0;
            const int n[3] = {g.nx, g.ny, g.nz};
            const int per[3] = {g.per_x, g.per_y, g.per_z};
            for (int k = 0; k < 3; ++k) {
                if (k >= d) {
                    P.Xn[3 * i + k] = 0.0;
                    s_X[k] = 0.0;
                    continue;
                }
                const double corr = c * (G0[k] + G1[k]) / 2.0;
                double Xw = Yi[k] + corr;
                // A^{n+1} = 2 (X^{n+1} - X^n - U_bar) = 2 * correction displacement
                P.A[3 * i + k] = 2.0 * corr;
                if (per[k]) {
                    if (Xw >= n[k]) Xw -= n[k];
                    else if (Xw < 0.0) Xw += n[k];
                } else if (!(Xw >= -0.5 && Xw <= n[k] - 0.5)) {
                    flags[1] = 1; // centre left the box
                }
                P.Xn[3 * i + k] = Xw;
                s_X[k] = Xw;
            }
            if (P.N[i] == 0) flags[1] = 1;
            if (d == 2) P.theta[i] += P.dth[i];
            write_acc(P, rp, i);
        }
    } else if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) s_X[k] = P.X[3 * i + k];
        write_acc(P, rp, i);
    }
    __syncthreads();
    raster_particle(owner, P, g, d, i, s_X, s_lo, s_hi);
}

// Algorithm 1 with K > 1 sub-steps: every sub-step needs all predicted
// positions, so one workgroup of 1024 threads sweeps the particles with a
// barrier between sub-steps (Jacobi).  Writes P.Xn, A, theta and the
// acceleration table; the indicator is then set by k_rigid_raster(update=0)
// on the swapped positions.
__global__ __launch_bounds__(1024) void k_rigid_substeps(PartDev P, RigidParams rp, Geom g, int32_t *__restrict__ flags)
{
    const int np = rp.np, d = rp.d, K = rp.K;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    for (int i = threadIdx.x; i < np; i += blockDim.x)
        for (int k = 0; k < 3; ++k) {
            P.Y[3 * i + k] = P.X[3 * i + k];
            P.Dc[3 * i + k] = 0.0;
        }
    __syncthreads();
    for (int it = 1; it <= K; ++it) {
        for (int i = threadIdx.x; i < np; i += blockDim.x)
            for (int k = 0; k < 3; ++k) P.Ys[3 * i + k] = P.Y[3 * i + k] + (k < d ? P.Ub[3 * i + k] / (double)K : 0.0);
        __syncthreads();
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            double F0[3] = {0, 0, 0}, F1[3] = {0, 0, 0};
            const double Ri = P.a[i], Ci = P.Cc[i];
            for (int j = 0; j < np; ++j) {
                if (j == i) continue;
                pair_force(P.Y + 3 * i, P.Y + 3 * j, Ri, P.a[j], Ci, rp, g, F0);
                pair_force(P.Ys + 3 * i, P.Ys + 3 * j, Ri, P.a[j], Ci, rp, g, F1);
            }
            wall_force(P.Y + 3 * i, Ri, Ci, rp, g, F0);
            wall_force(P.Ys + 3 * i, Ri, Ci, rp, g, F1);
            const double M = P.rho_s[i] * (double)P.N[i];
            const double c = M > 0.0 ? 1.0 / (2.0 * M) * (1.0 / ((double)K * K)) : 0.0;
            for (int k = 0; k < 3; ++k) {
                const double corr = k < d ? c * (F0[k] + F1[k]) / 2.0 : 0.0;
                P.Y2[3 * i + k] = P.Ys[3 * i + k] + corr;
                P.Dc[3 * i + k] += corr;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < np; i += blockDim.x)
            for (int k = 0; k < 3; ++k) P.Y[3 * i + k] = P.Y2[3 * i + k];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            if (k >= d) {
                P.Xn[3 * i + k] = 0.0;
                continue;
            }
            double Xw = P.Y[3 * i + k];
            P.A[3 * i + k] = 2.0 * P.Dc[3 * i + k];
            if (per[k]) {
                if (Xw >= n[k]) Xw -= n[k];
                else if (Xw < 0.0) Xw += n[k];
            } else if (!(Xw >= -0.5 && Xw <= n[k] - 0.5)) {
                flags[1] = 1;
            }
            P.Xn[3 * i + k] = Xw;
        }
        if (P.N[i] == 0) flags[1] = 1;
        if (d == 2) P.theta[i] += P.dth[i];
        write_acc(P, rp, i);
    }
}

__global__ void k_owner_to_int(const uint16_t *__restrict__ owner, int32_t *__restrict__ out, int64_t N)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const uint16_t o = owner[idx];
    out[idx] = o == FLUID ? -1 : (int32_t)o;
}

// Streaming copy, one 16-byte element per thread (achievable-bandwidth
// reference; the fastest of the copy shapes measured on MI355X).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src, n16);
    return hipGetLastError();
}

hipError_t launch_raster_clear(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_clear, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->P, c->geo, c->d);
    return hipGetLastError();
}

hipError_t launch_reduce(lbm_ctx *c, int step, double *rec)
{
    if (c->np == 0) return hipSuccess;
    dim3 grid(c->np), block(256);
    if (c->d == 2) {
        if (step) hipLaunchKernelGGL((k_reduce<2, true>), grid, block, 0, c->stream, c->owner, c->usol, c->P, c->geo, rec);
        else hipLaunchKernelGGL((k_reduce<2, false>), grid, block, 0, c->stream, c->owner, c->usol, c->P, c->geo, rec);
    } else {
        if (step) hipLaunchKernelGGL((k_reduce<3, true>), grid, block, 0, c->stream, c->owner, c->usol, c->P, c->geo, rec);
        else hipLaunchKernelGGL((k_reduce<3, false>), grid, block, 0, c->stream, c->owner, c->usol, c->P, c->geo, rec);
    }
    return hipGetLastError();
}

hipError_t launch_rigid_raster(lbm_ctx *c, int update)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_rigid_raster, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->P, rp, c->geo, update,
                       c->flags);
    return hipGetLastError();
}

hipError_t launch_rigid_substeps(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_rigid_substeps, dim3(1), dim3(1024), 0, c->stream, c->P, rp, c->geo, c->flags);
    return hipGetLastError();
}

hipError_t launch_owner_to_int(lbm_ctx *c, int32_t *out)
{
    hipLaunchKernelGGL(k_owner_to_int, dim3((unsigned)((c->geo.N + 255) / 256)), dim3(256), 0, c->stream, c->owner, out,
                       c->geo.N);
    return hipGetLastError();
}

} // namespace lbm
