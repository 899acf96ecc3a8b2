// particles.hip -- indicator rasterisation, per-particle momentum sums and
// the rigid-body update (Algorithm 1) for gfx950.  All particle arithmetic is
// FP64.
//
// Indicator (sec. 2.1, eq. 9).  Each particle owns the nodes of its closed
// shape; a node shared by several shapes goes to the lowest index.  A
// particle's previous scan box is cleared to FLUID first (separate kernel),
// then every particle scans a box two nodes wider than its bounding radius
// and takes each node inside its shape with a 16-bit atomic minimum.  The
// inside tests are FP64 with explicit round-to-nearest products and sums, so
// no contraction can move a node across a boundary.
//
// Momentum sums (sec. 2.4, eq. 22a-b).  One workgroup per particle walks its
// scan box; each thread accumulates in a fixed order, then a fixed LDS tree
// combines the 256 partials, so the result is bitwise reproducible.
//
// Algorithm 1 (sec. 2.4) with the collision forces of sec. 2.3 (eq. 19-21).
// One workgroup of 1024 threads: each sub-step evaluates all pair and wall
// forces at the previous and the predicted positions (Jacobi, all particles
// together), with a barrier between sub-steps.
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

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

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

// Compute the new scan box from X (bounding radius + 2 nodes, clipped on
// wall axes), store it, and claim every node inside the shape.
__global__ __launch_bounds__(256) void k_raster_set(uint16_t *__restrict__ owner, PartDev P, Geom g, int d)
{
    const int i = blockIdx.x;
    __shared__ int s_lo[3], s_hi[3];
    if (threadIdx.x == 0) {
        const int n[3] = {g.nx, g.ny, g.nz};
        const int per[3] = {g.per_x, g.per_y, g.per_z};
        const double R = P.a[i];
        for (int k = 0; k < 3; ++k) {
            if (k >= d) {
                s_lo[k] = 0;
                s_hi[k] = 0;
                continue;
            }
            const double Xk = P.X[3 * i + k];
            int lo = 0, hi = -1; // empty box for a non-finite or runaway centre
            if (fabs(Xk) < 1e9) {
                lo = (int)floor(Xk - R) - 2;
                hi = (int)ceil(Xk + R) + 2;
            }
            if (!per[k]) {
                lo = lo < 0 ? 0 : lo;
                hi = hi > n[k] - 1 ? n[k] - 1 : hi;
            }
            s_lo[k] = lo;
            s_hi[k] = hi;
            P.lo[3 * i + k] = lo;
            P.hi[3 * i + k] = hi;
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
    const double X0 = P.X[3 * i], X1 = P.X[3 * i + 1], X2 = (d == 3) ? P.X[3 * i + 2] : 0.0;
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

// Per-particle sums over the owned nodes of the scan box.
//  2D: [0] N, [1..2] sum u, [3] sum r x u (z), [4] sum |r|^2
//  3D: [0] N, [1..3] sum u, [4..6] sum r x u, [7..12] inertia xx yy zz xy xz yz
// then U = sum u / N and omega = (sum r x u)/(sum |r|^2) (2D) or I^{-1} L (3D).
template <int D>
__global__ __launch_bounds__(256) void k_reduce(const uint16_t *__restrict__ owner, const double *__restrict__ usol,
                                                 PartDev P, Geom g)
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
    if (threadIdx.x == 0) {
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
    }
}

// Collision force on particle i with all centres at Y (sec. 2.3, eq. 19-21).
__device__ void coll_force(const PartDev &P, const double *Y, int i, const RigidParams &rp, const Geom &g, double F[3])
{
    const int d = rp.d;
    const double Ri = P.a[i], del = rp.delta, Ci = P.Cc[i];
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    F[0] = F[1] = F[2] = 0.0;
    const double Yi[3] = {Y[3 * i], Y[3 * i + 1], Y[3 * i + 2]};
    for (int j = 0; j < rp.np; ++j) {
        if (j == i) continue;
        const double Rj = P.a[j];
        double dv[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) {
            dv[k] = Yi[k] - Y[3 * j + k];
            if (per[k]) {
                const double h = 0.5 * n[k];
                if (dv[k] > h) dv[k] -= n[k];
                else if (dv[k] < -h) dv[k] += n[k];
            }
        }
        const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (dist > Ri + Rj + del) continue;
        const double s = (Ri + Rj + del - dist) / del;
        const double mag = Ci / rp.eps_p * s * s;
        const double scale = rp.cform == 1 ? mag : mag / dist;
        for (int k = 0; k < d; ++k) F[k] += scale * dv[k];
    }
    for (int k = 0; k < d; ++k) {
        if (per[k]) continue;
        const double walls[2] = {-0.5, n[k] - 0.5};
        for (int s = 0; s < 2; ++s) {
            const double dv = Yi[k] - (2.0 * walls[s] - Yi[k]); // to the mirror particle
            const double dist = fabs(dv);
            if (dist > 2.0 * Ri + del) continue;
            const double q = (2.0 * Ri + del - dist) / del;
            const double mag = Ci / rp.eps_w * q * q;
            F[k] += rp.cform == 1 ? mag * dv : mag * dv / dist;
        }
    }
}

// Algorithm 1 for all particles; update = 0 only refreshes the acceleration
// table (used after lbm_set_particles).  rec: optional per-step record
// [np][14] (X theta U omega A N before the update).
__global__ __launch_bounds__(1024) void k_rigid(PartDev P, RigidParams rp, Geom g, double *__restrict__ rec, int update,
                                                int32_t *__restrict__ flags)
{
    const int np = rp.np, d = rp.d, K = rp.K;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    if (update) {
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            if (rec) {
                double *r = rec + 14 * i;
                for (int k = 0; k < 3; ++k) {
                    r[k] = P.X[3 * i + k];
                    r[4 + k] = P.U[3 * i + k];
                    r[7 + k] = P.W[3 * i + k];
                    r[10 + k] = P.A[3 * i + k];
                }
                r[3] = P.theta[i];
                r[13] = (double)P.N[i];
            }
            for (int k = 0; k < 3; ++k) {
                P.Ub[3 * i + k] = 0.5 * (P.U[3 * i + k] + P.Uprev[3 * i + k]);
                P.Y[3 * i + k] = P.X[3 * i + k];
                P.Dc[3 * i + k] = 0.0;
            }
        }
        __syncthreads();
        for (int it = 1; it <= K; ++it) {
            for (int i = threadIdx.x; i < np; i += blockDim.x)
                for (int k = 0; k < 3; ++k) P.Ys[3 * i + k] = P.Y[3 * i + k] + (k < d ? P.Ub[3 * i + k] / (double)K : 0.0);
            __syncthreads();
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                double F0[3], F1[3];
                coll_force(P, P.Y, i, rp, g, F0);
                coll_force(P, P.Ys, i, rp, g, F1);
                const double M = P.rho_s[i] * (double)P.N[i];
                const double c = (M > 0.0) ? 1.0 / (2.0 * M) * (1.0 / ((double)K * K)) : 0.0;
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
            for (int k = 0; k < d; ++k) {
                const double Xn = P.Y[3 * i + k];
                // A^{n+1} = 2 (X^{n+1} - X^n - U_bar), the bracket being the summed
                // correction displacements (no difference of absolute positions)
                P.A[3 * i + k] = 2.0 * P.Dc[3 * i + k];
                double Xw = Xn;
                if (per[k]) {
                    if (Xw >= n[k]) Xw -= n[k];
                    else if (Xw < 0.0) Xw += n[k];
                } else if (!(Xw >= -0.5 && Xw <= n[k] - 0.5)) {
                    flags[1] = 1; // centre left the box
                }
                P.X[3 * i + k] = Xw;
            }
            if (P.N[i] == 0) flags[1] = 1;
            if (d == 2) P.theta[i] += 0.5 * (P.W[3 * i + 2] + P.Wprev[3 * i + 2]);
            for (int k = 0; k < 3; ++k) {
                P.Uprev[3 * i + k] = P.U[3 * i + k];
                P.Wprev[3 * i + k] = P.W[3 * i + k];
            }
        }
    }
    // acceleration table for the lattice kernel: a_i = b_i g + A_i  (b_i per gravity_form)
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const double bi = rp.gform == 0 ? 1.0 - rp.rho_f / P.rho_s[i] : P.rho_s[i] / rp.rho_f - 1.0;
        for (int k = 0; k < 3; ++k) {
            const double acc = (k < d) ? bi * rp.g[k] + P.A[3 * i + k] : 0.0;
            P.acc_d[3 * i + k] = acc;
            P.acc_f[3 * i + k] = (float)acc;
        }
    }
}

__global__ void k_owner_to_int(const uint16_t *__restrict__ owner, int32_t *__restrict__ out, int64_t N)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const uint16_t o = owner[idx];
    out[idx] = o == FLUID ? -1 : (int32_t)o;
}

// Streaming copy, 16 bytes per thread per iteration (achievable-bandwidth reference).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src, n16);
    return hipGetLastError();
}

hipError_t launch_raster_clear(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_clear, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->P, c->geo, c->d);
    return hipGetLastError();
}

hipError_t launch_raster_set(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_raster_set, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->P, c->geo, c->d);
    return hipGetLastError();
}

hipError_t launch_reduce(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    if (c->d == 2)
        hipLaunchKernelGGL(k_reduce<2>, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->usol, c->P, c->geo);
    else
        hipLaunchKernelGGL(k_reduce<3>, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->usol, c->P, c->geo);
    return hipGetLastError();
}

hipError_t launch_rigid(lbm_ctx *c, double *rec, int update)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_rigid, dim3(1), dim3(1024), 0, c->stream, c->P, rp, c->geo, rec, update, c->flags);
    return hipGetLastError();
}

hipError_t launch_owner_to_int(lbm_ctx *c, int32_t *out)
{
    hipLaunchKernelGGL(k_owner_to_int, dim3((unsigned)((c->geo.N + 255) / 256)), dim3(256), 0, c->stream, c->owner, out,
                       c->geo.N);
    return hipGetLastError();
}

} // namespace lbm
