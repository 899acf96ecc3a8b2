// particles.hip -- indicator rasterisation, per-particle momentum sums and
// the rigid-body update (Algorithm 1) for gfx950.  All particle arithmetic is
// FP64.
//
// The particle side of a step is a few hundred to a few thousand nodes per
// particle: it is bound by memory latency, not bandwidth.  Two launches, one
// workgroup per particle each:
//    k_sums          momentum sums over the scan box (sec. 2.4, eq. 22a-b);
//                    in place, every owned node is reset to FLUID once read
//                    (a node owned by i is matched by no other particle), which
//                    clears the indicator for the next rasterisation.
//    k_rigid_raster  Algorithm 1 (sec. 2.4) for the particle, with the
//                    collision forces of sec. 2.3 (eq. 19-21) summed over the
//                    other particles across lanes, then its new indicator
//                    (sec. 2.1, eq. 9).
// (A single workgroup doing all of it for a few bodies was measured slower:
// it adds up the phases' latency chains on one compute unit.)
//
// Indicator: every node of a particle's closed shape is claimed with a 16-bit
// atomic minimum, so a node shared by two shapes goes to the lower index.  On
// lattices of even width the two nodes of an aligned 32-bit word are claimed
// together by one lane with one compare-and-swap that expects the cleared
// value, so a claim costs one round trip unless another particle touches the
// same word.  The inside tests are FP64 with explicit round-to-nearest
// products and sums, so no contraction moves a node across a boundary.
//
// Indicator buffers: the sums read owner_in; the raster writes owner_out,
// which must be all FLUID.  owner_in == owner_out is the in-place step (the
// sums clear it); distinct buffers keep the old indicator (differentiated runs).
//
// New centres go to a second buffer (P.Xn), swapped by the host, because every
// workgroup reads all old centres.
#include "lattice.h"
#include "node.h"
#include "reduce.h"

namespace lbm {

__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }

// The shape code of the fractional indicator's band |r| < R + 1/2 (disks and
// spheres of radius a; StepParams::frac) for inside_shape.
constexpr int SHAPE_BAND = 16;

// inside test of eq. (9) on the displacement (dx, dy, dz) from the centre
__device__ __forceinline__ bool inside_shape(int shape, double a, double b, double cs, double sn, double dx, double dy,
                                             double dz)
{
    if (shape == SHAPE_BAND) {
        const double Rh = dadd(a, 0.5);
        return dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz)) < dmul(Rh, Rh);
    }
    if (shape == LBM_DISK) return dadd(dmul(dx, dx), dmul(dy, dy)) <= dmul(a, a);
    if (shape == LBM_SPHERE) return dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz)) <= dmul(a, a);
    const double xi = dadd(dmul(cs, dx), dmul(sn, dy));
    const double eta = dadd(dmul(-sn, dx), dmul(cs, dy));
    return dadd(dmul(dmul(b, b), dmul(xi, xi)), dmul(dmul(a, a), dmul(eta, eta))) <= dmul(dmul(a, a), dmul(b, b));
}

// --------------------------------------------------------------- indicator

__device__ __forceinline__ uint32_t min_halves(uint32_t a, uint32_t b)
{
    const uint32_t lo = min(a & 0xFFFFu, b & 0xFFFFu), hi = min(a >> 16, b >> 16);
    return lo | (hi << 16);
}

// Finish lowering the two 16-bit owners of word w to `want` (0xFFFF in a half
// that is not claimed) after a compare-and-swap that expected `exp` returned
// `got`.  Owners only decrease, so the loop ends.
__device__ __forceinline__ void claim_finish(uint32_t *w, uint32_t want, uint32_t exp, uint32_t got)
{
    while (got != exp) {
        const uint32_t nw = min_halves(got, want);
        if (nw == got) return;
        exp = got;
        got = atomicCAS(w, exp, nw);
    }
}

// Claim the nodes of particle i (shape at centre Xc, box [lo, hi]) in owner,
// which holds FLUID wherever no other particle has claimed yet.  The items
// (node pairs on even-width lattices, else single nodes) are spread over nl
// lanes; this lane is `lane`.
template <int U>
__device__ void raster_items(uint16_t *owner, const Geom &g, int d, int i, const double *Xc, int shape, double a,
                             double b, double cs, double sn, const int *lo, const int *hi, int lane, int nl)
{
    if (hi[0] < lo[0] || hi[1] < lo[1] || hi[2] < lo[2]) return;
    const bool pairs = (g.nx & 1) == 0;
    const int step = pairs ? 2 : 1;
    // on an even-width lattice x and wrap(x) have the same parity, so an even
    // unwrapped x starts an aligned word; x - 1 below the box is still a node
    // of the lattice (lo is clipped at 0 on walls, and a periodic box spans
    // less than one period)
    const int xs = pairs ? lo[0] - (lo[0] & 1) : lo[0];
    const int wx = (hi[0] - xs) / step + 1, ey = hi[1] - lo[1] + 1;
    const int items = wx * ey * (hi[2] - lo[2] + 1);
    uint32_t *words = reinterpret_cast<uint32_t *>(owner);
    const uint32_t id = (uint32_t)i;
    const double X0 = Xc[0], X1 = Xc[1], X2 = d == 3 ? Xc[2] : 0.0;
    CellWalk w(wx, ey, lane, nl);
    for (int base = lane; base < items; base += U * nl) {
        uint32_t want[U], got[U];
        int widx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = base + u * nl;
            want[u] = 0xFFFFFFFFu;
            widx[u] = 0;
            const int col = w.lx, ly = w.ly, lz = w.lz;
            w.next();
            if (t < items) {
                const int x0 = xs + step * col, yu = lo[1] + ly, zu = lo[2] + lz;
                const double dy = (double)yu - X1, dz = d == 3 ? (double)zu - X2 : 0.0;
                const int n0 = wrap(x0, g.nx) + g.nx * (wrap(yu, g.ny) + g.ny * wrap(zu, g.nz));
                const bool in0 = inside_shape(shape, a, b, cs, sn, (double)x0 - X0, dy, dz);
                if (pairs) {
                    const bool in1 = inside_shape(shape, a, b, cs, sn, (double)(x0 + 1) - X0, dy, dz);
                    want[u] = (in0 ? id : 0xFFFFu) | ((in1 ? id : 0xFFFFu) << 16);
                } else if (in0) {
                    const uint32_t sh = (n0 & 1) ? 16u : 0u;
                    want[u] = (id << sh) | (0xFFFFu << (16u - sh));
                }
                widx[u] = n0 >> 1;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            got[u] = want[u] != 0xFFFFFFFFu ? atomicCAS(words + widx[u], 0xFFFFFFFFu, want[u]) : 0xFFFFFFFFu;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (want[u] != 0xFFFFFFFFu) claim_finish(words + widx[u], want[u], 0xFFFFFFFFu, got[u]);
    }
}

__global__ __launch_bounds__(256) void k_raster_clear(uint16_t *__restrict__ owner, PartDev P, Geom g)
{
    const int i = blockIdx.x;
    const Box b = make_box(P.lo + 3 * i, P.hi + 3 * i);
    for (int c = threadIdx.x; c < b.cells; c += blockDim.x) {
        int xu, yu, zu, node;
        cell_at(b, c, g, xu, yu, zu, node);
        owner[node] = FLUID;
    }
}

// ------------------------------------------------------------ momentum sums
// Per-particle sums over the owned nodes of the scan box.
//  2D: [0] N, [1..2] sum u, [3] sum r x u (z), [4] sum |r|^2
//  3D: [0] N, [1..3] sum u, [4..6] sum r x u, [7..12] inertia xx yy zz xy xz yz
// then U = sum u / N and omega = (sum r x u)/(sum |r|^2) (2D) or I^{-1} L (3D).
template <int D> struct NSums {
    static constexpr int value = D == 2 ? 5 : 13;
};

// This lane's partial sums over cells lane, lane + nl, ... of box b, with
// the loads of U cells in flight together.  owner_clr (NULL or owner_in):
// reset each owned node to FLUID once read.
template <int D, int U>
__device__ __forceinline__ void cell_sums(const uint16_t *owner_in, uint16_t *owner_clr, const double *__restrict__ usol,
                                          const Geom &g, int i, const double *Xc, const Box &b, int lane, int nl,
                                          double *s, const StepParams *frac, int &count)
{
    const int N = (int)g.N;
    const double X0 = Xc[0], X1 = Xc[1], X2 = D == 3 ? Xc[2] : 0.0;
    CellWalk w(b.ext[0] > 0 ? b.ext[0] : 1, b.ext[1] > 0 ? b.ext[1] : 1, lane, nl);
    for (int base = lane; base < b.cells; base += U * nl) {
        // all loads first (the velocity is read on every cell and used only
        // on owned ones), so their latencies overlap
        const CellWalk w0 = w;
        uint16_t o[U];
        double ux[U], uy[U], uz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int xu, yu, zu;
            const int node = base + u * nl < b.cells ? walk_node(b, w, g, xu, yu, zu) : 0;
            w.next();
            o[u] = owner_in[node];
            ux[u] = usol[node];
            uy[u] = usol[N + node];
            uz[u] = D == 3 ? usol[2 * N + node] : 0.0;
        }
        CellWalk w1 = w0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int xu, yu, zu;
            const int node = walk_node(b, w1, g, xu, yu, zu);
            w1.next();
            if (base + u * nl >= b.cells || o[u] != (uint16_t)i) continue;
            if (owner_clr) owner_clr[node] = FLUID;
            const double rx = (double)xu - X0, ry = (double)yu - X1;
            ++count;
            if (frac) { // the fractional indicator: each sum weighted by chi
                const double w = frac_chi(node, (uint16_t)i, *frac);
                s[0] += w;
                s[1] += w * ux[u];
                s[2] += w * uy[u];
                if constexpr (D == 2) {
                    s[3] += w * (rx * uy[u] - ry * ux[u]);
                    s[4] += w * (rx * rx + ry * ry);
                } else {
                    const double rz = (double)zu - X2;
                    s[3] += w * uz[u];
                    s[4] += w * (ry * uz[u] - rz * uy[u]);
                    s[5] += w * (rz * ux[u] - rx * uz[u]);
                    s[6] += w * (rx * uy[u] - ry * ux[u]);
                    const double rr = rx * rx + ry * ry + rz * rz;
                    s[7] += w * (rr - rx * rx);
                    s[8] += w * (rr - ry * ry);
                    s[9] += w * (rr - rz * rz);
                    s[10] -= w * (rx * ry);
                    s[11] -= w * (rx * rz);
                    s[12] -= w * (ry * rz);
                }
                continue;
            }
            s[0] += 1.0;
            s[1] += ux[u];
            s[2] += uy[u];
            if constexpr (D == 2) {
                s[3] += rx * uy[u] - ry * ux[u];
                s[4] += rx * rx + ry * ry;
            } else {
                const double rz = (double)zu - X2;
                s[3] += uz[u];
                s[4] += ry * uz[u] - rz * uy[u];
                s[5] += rz * ux[u] - rx * uz[u];
                s[6] += rx * uy[u] - ry * ux[u];
                const double rr = rx * rx + ry * ry + rz * rz;
                s[7] += rr - rx * rx;
                s[8] += rr - ry * ry;
                s[9] += rr - rz * rz;
                s[10] -= rx * ry;
                s[11] -= rx * rz;
                s[12] -= ry * rz;
            }
        }
    }
}

// State of particle i before the step, as the closing of the sums needs it.
struct PrevState {
    double X[3], theta, A[3], Uprev[3], Wprev[3];
};

__device__ __forceinline__ PrevState load_prev(const PartDev &P, int i)
{
    PrevState s;
    for (int k = 0; k < 3; ++k) {
        s.X[k] = P.X[3 * i + k];
        s.A[k] = P.A[3 * i + k];
        s.Uprev[k] = P.Uprev[3 * i + k];
        s.Wprev[k] = P.Wprev[3 * i + k];
    }
    s.theta = P.theta[i];
    return s;
}

// From the totals t: N, U^n, omega^n.  STEP (inside a time step): the record
// (layout REC_STRIDE in ctx.h), U_bar = (U^n + U^{n-1})/2, dtheta =
// (omega^n + omega^{n-1})/2 (z component), then U^{n-1} <- U^n, omega^{n-1} <-
// omega^n.  Returns N; Ub (3) and dth receive U_bar and dtheta.
template <int D, bool STEP>
__device__ __forceinline__ int close_sums(PartDev &P, int i, const double *t, int cnt, const PrevState &ps,
                                          double *rec, double *Ub, double &dth)
{
    P.N[i] = cnt;
    P.Nw[i] = t[0]; // the node count, or sum chi
    double U[3] = {0, 0, 0}, W[3] = {0, 0, 0};
    if (cnt > 0 && t[0] != 0.0) {
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
                r[k] = ps.X[k];
                r[4 + k] = U[k];
                r[7 + k] = W[k];
                r[10 + k] = ps.A[k];
                r[14 + k] = ps.Uprev[k];
            }
            r[3] = ps.theta;
            r[13] = t[0];
        }
        dth = 0.5 * (W[2] + ps.Wprev[2]);
        P.dth[i] = dth;
        for (int k = 0; k < 3; ++k) {
            Ub[k] = 0.5 * (U[k] + ps.Uprev[k]);
            P.Ub[3 * i + k] = Ub[k];
            P.Uprev[3 * i + k] = U[k];
            P.Wprev[3 * i + k] = W[k];
        }
    }
    return cnt;
}

// One workgroup of BS threads per particle.
// The sums carry the node count as one more entry (the weight sum s[0] is
// not a count with the fractional indicator).
template <int D, bool STEP, int BS>
__global__ __launch_bounds__(BS) void k_sums(const uint16_t *owner_in, uint16_t *owner_clr,
                                             const double *__restrict__ usol, PartDev P, Geom g,
                                             double *__restrict__ rec, StepParams sp)
{
    constexpr int NS = NSums<D>::value;
    __shared__ double part[BS / WAVE][NS + 1];
    const int i = blockIdx.x;
    const PrevState ps = load_prev(P, i);
    const Box b = make_box(P.lo + 3 * i, P.hi + 3 * i);
    double s[NS + 1];
#pragma unroll
    for (int k = 0; k <= NS; ++k) s[k] = 0.0;
    int count = 0;
    cell_sums<D, UNR>(owner_in, STEP ? owner_clr : nullptr, usol, g, i, ps.X, b, threadIdx.x, BS, s,
                      sp.frac ? &sp : nullptr, count);
    s[NS] = (double)count;
    block_sum<NS + 1, BS>(s, part);
    if (threadIdx.x != 0) return;
    double Ub[3], dth;
    close_sums<D, STEP>(P, i, s, (int)s[NS], ps, rec, Ub, dth);
}

// ------------------------------------------------------- collision forces
// Contribution of particle j to the particle-particle force on i at centres
// Yi, Yj (sec. 2.3, eq. 19), minimum image on periodic axes.
__device__ __forceinline__ void pair_force(const double *Yi, const double *Yj, double Ri, double Rj, double Ci,
                                           const RigidParams &rp, const Geom &g, double F[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    double dv[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= rp.d) continue;
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
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] += scale * dv[k]; // dv = 0 beyond the lattice dimension
}

// Particle-wall forces through the mirror particle (sec. 2.3, eq. 20).
__device__ __forceinline__ void wall_force(const double *Yi, double Ri, double Ci, const RigidParams &rp, const Geom &g,
                                           double F[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= rp.d || per[k]) continue;
        const double walls[2] = {-0.5, n[k] - 0.5};
#pragma unroll
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
__device__ __forceinline__ void write_acc(PartDev &P, const RigidParams &rp, int i, double rho, const double *A)
{
    const double bi = rp.gform == 0 ? 1.0 - rp.rho_f / rho : rho / rp.rho_f - 1.0;
    for (int k = 0; k < 3; ++k) {
        const double acc = (k < rp.d) ? bi * rp.g[k] + A[k] : 0.0;
        P.acc_d[3 * i + k] = acc;
        P.acc_f[3 * i + k] = (float)acc;
    }
}

// Closing of Algorithm 1 for particle i: centre Y after the sub-steps (or the
// single step), summed corrections Dc.  A^{n+1} = 2 * summed corrections;
// wraps periodic axes, flags a centre that left the box or a particle that
// covered no node.  Writes X^{n+1} (to P.Xn and Xout), theta^{n+1} (returned),
// the acceleration table entry.
__device__ __forceinline__ double close_rigid(PartDev &P, const RigidParams &rp, const Geom &g, int i, const double *Y,
                                              const double *Dc, int cnt, double rho, double theta, double dth,
                                              int32_t *flags, double *Xout)
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    double A[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        if (k >= rp.d) {
            P.Xn[3 * i + k] = 0.0;
            P.A[3 * i + k] = 0.0;
            Xout[k] = 0.0;
            continue;
        }
        double Xw = Y[k];
        A[k] = 2.0 * Dc[k];
        P.A[3 * i + k] = A[k];
        if (per[k]) {
            if (Xw >= n[k]) Xw -= n[k];
            else if (Xw < 0.0) Xw += n[k];
        } else if (!(Xw >= -0.5 && Xw <= n[k] - 0.5)) {
            flags[1] = 1; // centre left the box
        }
        P.Xn[3 * i + k] = Xw;
        Xout[k] = Xw;
    }
    if (cnt == 0) flags[1] = 1;
    double th = theta;
    if (rp.d == 2) {
        th = theta + dth;
        P.theta[i] = th;
    }
    write_acc(P, rp, i, rho, A);
    return th;
}

// ----------------------------------------------- many bodies: Algorithm 1
// One workgroup per particle.  update = 1 (K = 1): Algorithm 1 for particle i
// -- the collision forces at X^n and at the prediction X^n + U_bar summed over
// all other particles across lanes and over the walls, the correction, X^{n+1}
// into P.Xn, A^{n+1}, theta^{n+1} -- then the new indicator of i in owner.
// update = 0: rasterise i at P.X and refresh its acceleration entry.
template <int BS>
__global__ __launch_bounds__(BS) void k_rigid_raster(uint16_t *__restrict__ owner, PartDev P, RigidParams rp, Geom g,
                                                     int update, int32_t *__restrict__ flags)
{
    const int i = blockIdx.x, d = rp.d;
    __shared__ double s_X[3], s_cs, s_sn;
    __shared__ int s_lo[3], s_hi[3];
    __shared__ double part[BS / WAVE][6];
    const double Ri = P.a[i], Ci = P.Cc[i], rho = P.rho_s[i], theta = P.theta[i], bi = P.b[i];
    const int shape = P.shape[i];
    double Xi[3], Yi[3];
    for (int k = 0; k < 3; ++k) {
        Xi[k] = P.X[3 * i + k];
        Yi[k] = Xi[k] + (k < d ? P.Ub[3 * i + k] : 0.0);
    }
    if (update) {
        const int cnt = P.N[i];
        const double Nw = P.Nw[i]; // the node count, or sum chi
        const double dth = P.dth[i];
        // orientation of the new indicator, ahead of the force sums (d == 2 only
        // turns; ellipses are 2D)
        const double th1 = d == 2 ? theta + dth : theta;
        const double cs = shape == LBM_ELLIPSE ? cos(th1) : 1.0, sn = shape == LBM_ELLIPSE ? sin(th1) : 0.0;
        double F[6] = {0, 0, 0, 0, 0, 0};
        for (int j = threadIdx.x; j < rp.np; j += BS) {
            if (j == i) continue;
            double Xj[3], Yj[3];
            for (int k = 0; k < 3; ++k) {
                Xj[k] = P.X[3 * j + k];
                Yj[k] = Xj[k] + (k < d ? P.Ub[3 * j + k] : 0.0);
            }
            const double Rj = P.a[j];
            pair_force(Xi, Xj, Ri, Rj, Ci, rp, g, F);
            pair_force(Yi, Yj, Ri, Rj, Ci, rp, g, F + 3);
        }
        block_sum<6, BS>(F, part);
        if (threadIdx.x == 0) {
            wall_force(Xi, Ri, Ci, rp, g, F);
            wall_force(Yi, Ri, Ci, rp, g, F + 3);
            const double M = rho * Nw;
            const double c = M > 0.0 ? 1.0 / (2.0 * M) : 0.0;
            double Y[3], Dc[3];
            for (int k = 0; k < 3; ++k) {
                Dc[k] = k < d ? c * (F[k] + F[3 + k]) / 2.0 : 0.0;
                Y[k] = Yi[k] + Dc[k];
            }
            close_rigid(P, rp, g, i, Y, Dc, cnt, rho, theta, dth, flags, s_X);
            s_cs = cs;
            s_sn = sn;
        }
    } else if (threadIdx.x == 0) {
        double A[3];
        for (int k = 0; k < 3; ++k) {
            s_X[k] = Xi[k];
            A[k] = P.A[3 * i + k];
        }
        write_acc(P, rp, i, rho, A);
        s_cs = shape == LBM_ELLIPSE ? cos(theta) : 1.0;
        s_sn = shape == LBM_ELLIPSE ? sin(theta) : 0.0;
    }
    if (threadIdx.x == 0) {
        centre_box(s_X, Ri, g, d, s_lo, s_hi);
        for (int k = 0; k < 3; ++k) { // unused axes get [0, 0]
            P.lo[3 * i + k] = s_lo[k];
            P.hi[3 * i + k] = s_hi[k];
            P.geo[4 * i + k] = s_X[k]; // the centre this indicator is built from
        }
        P.geo[4 * i + 3] = Ri;
    }
    __syncthreads();
    raster_items<UNR>(owner, g, d, i, s_X, rp.frac ? SHAPE_BAND : shape, Ri, bi, s_cs, s_sn, s_lo, s_hi, threadIdx.x,
                      BS);
}

// Acceleration table a_i = b_i g + A_i of every particle from the current
// rho_s, g and A (after a change of the parameters).
__global__ __launch_bounds__(256) void k_write_acc(PartDev P, RigidParams rp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rp.np) return;
    double A[3];
    for (int k = 0; k < 3; ++k) A[k] = P.A[3 * i + k];
    write_acc(P, rp, i, P.rho_s[i], A);
}

// ------------------------------------- fused-sums step: Algorithm 1 from slots
// K = 1 with the momentum sums taken by the lattice kernel (slot_sums): one
// workgroup per particle i
//  0. waves 1.. test which particles j are close enough to
//     interact at X^n or at the prediction (|X_i - X_j| <= R_i + R_j +
//     delta + 0.6: the lattice sentinel bounds every node speed by 0.3, hence
//     |U_bar| <= 0.3), one bit per j in LDS;
//  1. meanwhile its first wavefront sums i's records of this step (in 3D,
//     with thousands of records, the whole workgroup): lane l takes the
//     records l, l + 64, ... of i's table; one with this step's stamp is
//     shifted to moments about X_i^n by the first node it carries, and the
//     fixed-order sum gives N_i, U_i^n, omega_i^n, the record, U_bar_i and
//     dtheta_i on every lane of wave 0;
//  2. after a barrier the same wavefront visits the particles in reach in
//     index order, sums the count and velocity of j's records of this step
//     (j's box is not needed, which is as well: j's own workgroup is replacing
//     it) for U_j^n and U_bar_j = (U_j^n + U_j^{n-1})/2, and adds the pair
//     forces at X^n and at the prediction;
//  3. lane 0 closes Algorithm 1; after a second barrier the whole workgroup
//     rasterises the new indicator, as k_rigid_raster.
// U^{n-1} of every particle is read from P.U, which nothing writes during the
// launch: U^n goes to P.Unext, and the host swaps the two afterwards.

// Offsets from the centre X of a record's first node (unwrapped: on a
// periodic axis the image nearest to X, which is the scan box's, since a box
// reaches at most ceil(R) + 3 nodes from the centre and the set-up keeps that
// under half a period; in x the wavefront's middle is used, as a wavefront
// reaches 63 nodes further).
__device__ __forceinline__ void slot_offsets(double first, const double *X, const Geom &g, double &dx, double &dy,
                                             double &dz)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(first);
    int x0 = (int)(b & 0x1FFFFFu), y = (int)((b >> 21) & 0x1FFFFFu), z = (int)(b >> 42);
    if (g.per_x) x0 -= g.nx * (int)rint(((double)x0 + 31.5 - X[0]) / g.nx);
    if (g.per_y) y -= g.ny * (int)rint(((double)y - X[1]) / g.ny);
    if (g.per_z) z -= g.nz * (int)rint(((double)z - X[2]) / g.nz);
    dx = (double)x0 - X[0];
    dy = (double)y - X[1];
    dz = (double)z - X[2];
}

// Adds the moments about the particle centre of one slot record (see
// slot_sums) whose first node sits at (X_0 + dx, X_1 + dy, X_2 + dz): 2D
// [N, U (2), L_z, sum |r|^2], 3D [N, U (3), L (3), inertia xx yy zz xy xz yz],
// the moments of the momentum-sum kernel.  A node at lane offset s of the
// slot has r = (s + dx, dy, dz).
template <int D>
__device__ __forceinline__ void add_slot(const double *v, double dx, double dy, double dz, double *c)
{
    double n, s1, s2;
    mask_moments((unsigned long long)__double_as_longlong(v[1]), n, s1, s2);
    const double sxx = s2 + 2.0 * dx * s1 + n * dx * dx; // sum of r_x^2
    if constexpr (D == 2) {
        const double vx = v[3], vy = v[4], vs = v[5];
        c[0] += n;
        c[1] += vx;
        c[2] += vy;
        c[3] += vs + dx * vy - dy * vx;
        c[4] += sxx + n * dy * dy;
    } else {
        const double vx = v[3], vy = v[4], vz = v[5], vsy = v[6], vsz = v[7];
        const double syy = n * dy * dy, szz = n * dz * dz, sx = s1 + n * dx; // sum of r_x
        c[0] += n;
        c[1] += vx;
        c[2] += vy;
        c[3] += vz;
        c[4] += dy * vz - dz * vy;
        c[5] += dz * vx - (vsz + dx * vz);
        c[6] += (vsy + dx * vy) - dy * vx;
        c[7] += syy + szz;
        c[8] += sxx + szz;
        c[9] += sxx + syy;
        c[10] -= dy * sx;
        c[11] -= dz * sx;
        c[12] -= n * dy * dz;
    }
}

template <int D, int BS>
__global__ __launch_bounds__(BS) void k_rigid_fused(uint16_t *__restrict__ owner, PartDev P, RigidParams rp, Geom g,
                                                    SlotParams sl, double *__restrict__ rec, int32_t *__restrict__ flags)
{
    constexpr int NS = NSums<D>::value, W1 = slot_width(D);
    const int i = blockIdx.x, np = rp.np;
    __shared__ double s_X[3], s_cs, s_sn;
    __shared__ int s_lo[3], s_hi[3];
    __shared__ unsigned long long s_reach[MAX_NP / WAVE]; // bit j: particle j is in reach
    const double Ri = P.a[i], bi = P.b[i];
    const int shape = P.shape[i];
    // the particles close enough to interact with i at X^n or at the
    // prediction (|X_i - X_j| <= R_i + R_j + delta + 0.6: the lattice sentinel
    // bounds every node speed by 0.3, hence |U_bar| <= 0.3), tested by waves
    // 1.. while wave 0 sums i's records
    if (threadIdx.x >= WAVE) {
        const int n[3] = {g.nx, g.ny, g.nz};
        const int per[3] = {g.per_x, g.per_y, g.per_z};
        double Xo[3];
        for (int k = 0; k < 3; ++k) Xo[k] = P.X[3 * i + k];
        for (int j0 = 0; j0 < np; j0 += BS - WAVE) { // uniform
            const int j = j0 + (int)threadIdx.x - WAVE;
            bool in = false;
            if (j < np && j != i) {
                double dv2 = 0.0;
                for (int k = 0; k < D; ++k) {
                    double dk = Xo[k] - P.X[3 * j + k];
                    if (per[k]) {
                        const double h = 0.5 * n[k];
                        if (dk > h) dk -= n[k];
                        else if (dk < -h) dk += n[k];
                    }
                    dv2 += dk * dk;
                }
                const double reach = Ri + P.a[j] + rp.delta + 0.6;
                in = dv2 <= reach * reach;
            }
            const unsigned long long m = __ballot(in);
            if ((threadIdx.x & (WAVE - 1)) == 0 && j < np) s_reach[j / WAVE] = m;
        }
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const double Ci = P.Cc[i], rho = P.rho_s[i], theta = P.theta[i];
    double Xi[3];
    for (int k = 0; k < 3; ++k) Xi[k] = P.X[3 * i + k];
    PrevState ps = load_prev(P, i);
    for (int k = 0; k < 3; ++k) ps.Uprev[k] = P.U[3 * i + k]; // U^{n-1}
    int cnt = 0;
    double dth = 0.0, Ub[3] = {0, 0, 0};

    // 1. own sums: every record of i's table (no dependence on the scan box:
    // the loads issue with the particle's own), kept if it carries this
    // step's stamp and shifted to moments about X_i^n by its first node.
    // 2D: wave 0 alone (64 records); 3D (thousands of records): the whole
    // workgroup, then its sum is handed to wave 0.  Either way every lane of
    // wave 0 ends with the same totals.
    double s[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = 0.0;
    if (D == 3 || threadIdx.x < WAVE) {
        const double *si = sl.slots + (size_t)i * sl.stride * W1;
        const int t0 = D == 3 ? (int)threadIdx.x : lane, nt = D == 3 ? BS : WAVE;
        for (int t = t0; t < sl.stride; t += nt) {
            double rv[W1];
#pragma unroll
            for (int m = 0; m < W1; ++m) rv[m] = si[(size_t)t * W1 + m];
            if (rv[0] == sl.stamp) {
                double dx, dy, dz;
                slot_offsets(rv[2], Xi, g, dx, dy, dz);
                add_slot<D>(rv, dx, dy, D == 3 ? dz : 0.0, s);
            }
        }
    }
    if constexpr (D == 3) {
        __shared__ double part[BS / WAVE][NS];
        __shared__ double s_tot[NS];
        block_sum<NS, BS>(s, part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NS; ++k) s_tot[k] = s[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NS; ++k) s[k] = s_tot[k];
    } else if (threadIdx.x < WAVE) {
#pragma unroll
        for (int k = 0; k < NS; ++k) s[k] = wave_sum(s[k]);
    }
    if (threadIdx.x < WAVE) { // wave 0
        cnt = (int)s[0];
        double U[3] = {0, 0, 0}, W[3] = {0, 0, 0};
        if (cnt > 0) {
            if constexpr (D == 2) {
                U[0] = s[1] / s[0];
                U[1] = s[2] / s[0];
                W[2] = s[3] / s[4];
            } else {
                U[0] = s[1] / s[0];
                U[1] = s[2] / s[0];
                U[2] = s[3] / s[0];
                const double L0 = s[4], L1 = s[5], L2 = s[6];
                const double a = s[7], e = s[8], f = s[9], bxy = s[10], cxz = s[11], dyz = s[12];
                const double A00 = e * f - dyz * dyz, A01 = cxz * dyz - bxy * f, A02 = bxy * dyz - cxz * e;
                const double A11 = a * f - cxz * cxz, A12 = bxy * cxz - a * dyz, A22 = a * e - bxy * bxy;
                const double det = a * A00 + bxy * A01 + cxz * A02;
                W[0] = (A00 * L0 + A01 * L1 + A02 * L2) / det;
                W[1] = (A01 * L0 + A11 * L1 + A12 * L2) / det;
                W[2] = (A02 * L0 + A12 * L1 + A22 * L2) / det;
            }
        }
        dth = 0.5 * (W[2] + ps.Wprev[2]);
        for (int k = 0; k < 3; ++k) Ub[k] = 0.5 * (U[k] + ps.Uprev[k]);
        if (lane == 0) {
            P.N[i] = cnt; // (P.Nw and P.geo serve the unfused steps only: the
                          // fused step never runs with the fractional indicator)
            if (rec) {
                double *r = rec + REC_STRIDE * i;
                for (int k = 0; k < 3; ++k) {
                    r[k] = ps.X[k];
                    r[4 + k] = U[k];
                    r[7 + k] = W[k];
                    r[10 + k] = ps.A[k];
                    r[14 + k] = ps.Uprev[k];
                }
                r[3] = ps.theta;
                r[13] = (double)cnt;
            }
            P.dth[i] = dth;
            for (int k = 0; k < 3; ++k) {
                P.Ub[3 * i + k] = Ub[k];
                P.Unext[3 * i + k] = U[k];
                P.W[3 * i + k] = W[k];
                P.Wprev[3 * i + k] = W[k];
            }
        }

    }
    __syncthreads(); // the reach masks are complete
    if (threadIdx.x < WAVE) { // wave 0
        // 2. pair forces with the particles in reach, in index order; the
        // wavefront sums each partner's records for U_j^n, every lane adds
        // the same forces
        double Yi[3];
        for (int k = 0; k < 3; ++k) Yi[k] = Xi[k] + (k < D ? Ub[k] : 0.0);
        double F[6] = {0, 0, 0, 0, 0, 0};
        for (int j0 = 0; j0 < np; j0 += WAVE) { // uniform
            for (unsigned long long m = s_reach[j0 / WAVE]; m; m &= m - 1ull) { // uniform
                const int jj = j0 + __ffsll((long long)m) - 1;
                const double *sj = sl.slots + (size_t)jj * sl.stride * W1;
                double u[4] = {0, 0, 0, 0};
                for (int t = lane; t < sl.stride; t += WAVE) {
                    double rv[W1];
#pragma unroll
                    for (int mm = 0; mm < W1; ++mm) rv[mm] = sj[(size_t)t * W1 + mm];
                    if (rv[0] == sl.stamp) {
                        u[0] += (double)__popcll((unsigned long long)__double_as_longlong(rv[1]));
                        u[1] += rv[3];
                        u[2] += rv[4];
                        if (D == 3) u[3] += rv[5];
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) u[k] = wave_sum(u[k]);
                double Xj[3], Yj[3];
                for (int k = 0; k < 3; ++k) {
                    Xj[k] = P.X[3 * jj + k];
                    const double Uj = (k < D && u[0] > 0.0) ? u[1 + k] / u[0] : 0.0;
                    Yj[k] = Xj[k] + (k < D ? 0.5 * (Uj + P.U[3 * jj + k]) : 0.0);
                }
                const double Rj = P.a[jj];
                pair_force(Xi, Xj, Ri, Rj, Ci, rp, g, F);
                pair_force(Yi, Yj, Ri, Rj, Ci, rp, g, F + 3);
            }
        }

        // 3. close Algorithm 1
        if (lane == 0) {
            wall_force(Xi, Ri, Ci, rp, g, F);
            wall_force(Yi, Ri, Ci, rp, g, F + 3);
            const double M = rho * (double)cnt;
            const double c = M > 0.0 ? 1.0 / (2.0 * M) : 0.0;
            double Y[3], Dc[3];
            for (int k = 0; k < 3; ++k) {
                Dc[k] = k < D ? c * (F[k] + F[3 + k]) / 2.0 : 0.0;
                Y[k] = Yi[k] + Dc[k];
            }
            const double th = close_rigid(P, rp, g, i, Y, Dc, cnt, rho, theta, dth, flags, s_X);
            s_cs = shape == LBM_ELLIPSE ? cos(th) : 1.0;
            s_sn = shape == LBM_ELLIPSE ? sin(th) : 0.0;
            centre_box(s_X, Ri, g, D, s_lo, s_hi);
            for (int k = 0; k < 3; ++k) {
                P.lo[3 * i + k] = s_lo[k];
                P.hi[3 * i + k] = s_hi[k];
            }
        }
    }
    __syncthreads();
    // then the new indicator, by the whole workgroup
    raster_items<UNR>(owner, g, D, i, s_X, shape, Ri, bi, s_cs, s_sn, s_lo, s_hi, threadIdx.x, BS);
}

// Algorithm 1 with K > 1 sub-steps: every sub-step needs all
// predicted positions, so one workgroup of 1024 threads sweeps the particles
// with a barrier between sub-steps (Jacobi).  Writes P.Xn, A, theta and the
// acceleration table; the indicator is then set by k_rigid_raster(update=0)
// on the swapped positions.
__global__ __launch_bounds__(1024) void k_rigid_substeps(PartDev P, RigidParams rp, Geom g, int32_t *__restrict__ flags)
{
    const int np = rp.np, d = rp.d, K = rp.K;
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
            const double M = P.rho_s[i] * P.Nw[i]; // rho_s N_i (N_i = sum chi when fractional)
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
        double Y[3], Dc[3], Xo[3];
        for (int k = 0; k < 3; ++k) {
            Y[k] = P.Y[3 * i + k];
            Dc[k] = P.Dc[3 * i + k];
        }
        close_rigid(P, rp, g, i, Y, Dc, P.N[i], P.rho_s[i], P.theta[i], P.dth[i], flags, Xo);
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

// The same copy over NA arrays at once (array a at a * n16 words of src and
// dst): each thread moves word i of every array, all loads before the first
// store, so that NA streams are read and NA written together, as the lattice
// update reads and writes its Q population arrays.  NA = 0: a runtime count
// na, one array after another per thread.
template <int NA>
__global__ __launch_bounds__(256) void k_copy_arrays(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                                     size_t n16, int na)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    if constexpr (NA > 0) {
        u32x4 v[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) v[a] = __builtin_nontemporal_load(src + (size_t)a * n16 + i);
#pragma unroll
        for (int a = 0; a < NA; ++a) __builtin_nontemporal_store(v[a], dst + (size_t)a * n16 + i);
    } else {
        for (int a = 0; a < na; ++a) dst[(size_t)a * n16 + i] = src[(size_t)a * n16 + i];
    }
}

// ----------------------------------------------------------------- launchers
hipError_t launch_copy_arrays(void *dst, const void *src, int na, size_t bytes_per_array, hipStream_t s)
{
    const size_t n16 = bytes_per_array / 16;
    if (n16 == 0 || na == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(256);
    if (na == 9) hipLaunchKernelGGL(k_copy_arrays<9>, grid, block, 0, s, (u32x4 *)dst, (const u32x4 *)src, n16, na);
    else if (na == 19) hipLaunchKernelGGL(k_copy_arrays<19>, grid, block, 0, s, (u32x4 *)dst, (const u32x4 *)src, n16, na);
    else hipLaunchKernelGGL(k_copy_arrays<0>, grid, block, 0, s, (u32x4 *)dst, (const u32x4 *)src, n16, na);
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_raster_clear, dim3(c->np), dim3(256), 0, c->stream, c->owner, c->P, c->geo);
    return hipGetLastError();
}

// Workgroup size of the per-particle sums: 256 threads cover a 2D scan box in
// one batch of loads; 3D boxes are ~10x larger.
constexpr int SUMS_BS2 = 256, SUMS_BS3 = 512, RIGID_BS = 256;

// step = 1: the sums of a step (clear the indicator, prepare Algorithm 1);
// step = 0: U and omega measured on the current state, into P.U and P.W
// (lbm_set_particles: U^0) or, with scratch = 1, into P.Y and P.Ys, leaving
// the state untouched (lbm_get_particles).
hipError_t launch_reduce(lbm_ctx *c, int step, double *rec, int scratch)
{
    if (c->np == 0) return hipSuccess;
    const uint16_t *oin = c->owner;
    // the rigid-velocity forcing pass reads the indicator after the sums and clears it
    uint16_t *oclr = (c->owner_next || c->sp.beta > 0) ? nullptr : c->owner;
    const dim3 grid(c->np);
    const double *us = c->usol;
    PartDev P = c->P;
    if (!step && scratch) {
        P.U = c->P.Y;
        P.W = c->P.Ys;
    }
    if (c->d == 2)
        return step ? launch(c, k_sums<2, true, SUMS_BS2>, grid, dim3(SUMS_BS2), oin, oclr, us, P, c->geo, rec, c->sp)
                    : launch(c, k_sums<2, false, SUMS_BS2>, grid, dim3(SUMS_BS2), oin, oclr, us, P, c->geo, rec, c->sp);
    return step ? launch(c, k_sums<3, true, SUMS_BS3>, grid, dim3(SUMS_BS3), oin, oclr, us, P, c->geo, rec, c->sp)
                : launch(c, k_sums<3, false, SUMS_BS3>, grid, dim3(SUMS_BS3), oin, oclr, us, P, c->geo, rec, c->sp);
}

hipError_t launch_rigid_raster(lbm_ctx *c, int update)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    uint16_t *out = c->owner_next ? c->owner_next : c->owner;
    return launch(c, k_rigid_raster<RIGID_BS>, dim3(c->np), dim3(RIGID_BS), out, c->P, rp, c->geo, update, c->flags);
}

hipError_t launch_write_acc(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_write_acc, dim3((c->np + 255) / 256), dim3(256), 0, c->stream, c->P, rp);
    return hipGetLastError();
}

hipError_t launch_rigid_substeps(lbm_ctx *c)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    return launch(c, k_rigid_substeps, dim3(1), dim3(1024), c->P, rp, c->geo, c->flags);
}

SlotParams slot_params(lbm_ctx *c, bool on)
{
    SlotParams sl{};
    if (!on || !c->slots || c->np == 0) return sl; // slots == NULL: no fused sums
    sl.slots = c->slots;
    sl.stride = c->slot_stride;
    sl.mx = c->slot_mx;
    sl.my = c->slot_my;
    sl.mz = c->slot_mz;
    sl.sy = c->slot_sy;
    sl.sz = c->slot_sz;
    sl.stamp = (double)c->epoch;
    sl.clear = c->owner_next ? nullptr : c->owner;
    return sl;
}

hipError_t launch_rigid_fused(lbm_ctx *c, double *rec)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    const SlotParams sl = slot_params(c, true);
    if (!sl.slots) return hipErrorInvalidValue;
    uint16_t *out = c->owner_next ? c->owner_next : c->owner;
    if (c->d == 2)
        return launch(c, k_rigid_fused<2, RIGID_BS>, dim3(c->np), dim3(RIGID_BS), out, c->P, rp, c->geo, sl, rec,
                      c->flags);
    return launch(c, k_rigid_fused<3, RIGID_BS>, dim3(c->np), dim3(RIGID_BS), out, c->P, rp, c->geo, sl, rec, c->flags);
}

hipError_t launch_owner_to_int(lbm_ctx *c, int32_t *out)
{
    hipLaunchKernelGGL(k_owner_to_int, dim3((unsigned)((c->geo.N + 255) / 256)), dim3(256), 0, c->stream, c->owner, out,
                       c->geo.N);
    return hipGetLastError();
}

} // namespace lbm
