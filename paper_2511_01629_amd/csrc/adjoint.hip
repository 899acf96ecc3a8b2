// adjoint.hip -- hand-written adjoint of one time step (gfx950).
//
// With the paper's binary indicator the step map is differentiated with the
// indicator sequence frozen (a binary indicator makes the loss piecewise
// smooth in the parameters; the derivative is that of the smooth pieces).
// With the indicator frozen,
// omega^n only advances theta, and theta only moves the indicator, so the
// angular sums carry no derivative: the adjoint of the momentum sums is the
// broadcast u_bar(x) = U_bar_i / N_i onto the nodes of particle i.
//
// One backward step n, given the adjoints of the step's outputs
// (lambda = dL/df~^n, X_bar^{n+1}, A_bar^{n+1}, U_bar of the U^n kept for the
// next step), runs three kernels:
//   k_adj_rigid     Algorithm 1 transposed, one workgroup per particle: the
//                   pair and wall force Jacobians at X^n and at the
//                   prediction, gathered over all particles across lanes;
//                   gives X_bar^n, the adjoint of U^n (for the broadcast) and
//                   of U^{n-1}, and the density and |g| partials of the
//                   collision constant and of 1/(2M).
//   k_adj_lattice   per node: the Jacobian-transpose of the collision
//                   (eq. 10, 13, 14, 15, 17) re-evaluated from the stored
//                   pre-step populations, plus the broadcast u_bar; then the
//                   transpose of the pull, which is a push (streaming is a
//                   permutation).  Writes a_bar on solid nodes and a
//                   per-workgroup partial of dL/dtau.
//   k_adj_particles per particle: A_bar^n = sum of a_bar over its nodes, and
//                   the density and |g| partials through a = b g + A.
// With the fractional indicator (disks and spheres) the weights chi depend
// smoothly on the centres X^n, and the adjoint carries that dependence: per
// node chi_bar gathers the weight's four uses (the acceleration chi (b g + A),
// the penalization chi alpha, the sums chi u and N = sum chi, and, in step 0,
// the initial U^{-1} measured on the same nodes), and X_bar^n receives
// chi_bar dchi/dX summed over the particle's nodes.  The angular sums still
// carry none: omega only turns a disk or sphere, which moves no node weight.
// Where the forward step has momentum-sum slots, the lattice adjoint sums
// a_bar per (particle, slot) record instead of writing it per node, and one
// kernel per particle (k_adj_fused) closes A_bar^n from the records and then
// runs the rigid adjoint of step n - 1: two launches per step instead of
// three.
#include "dispatch.h"
#include "node.h"
#include "reduce.h"

namespace lbm {

// ----------------------------------------------------------- lattice adjoint
// The a_bar of one step's solid nodes summed per (particle, slot) record
// (the slot layout of the forward's momentum sums, slot_of): for each
// distinct key among the lanes, its lowest lane writes [stamp, sum a_bar
// (D)], each a fixed-order wavefront sum.  Called by every lane of the
// wavefront with uniform control flow.
template <int D>
__device__ void slot_abar(bool active, uint16_t own, int x, int y, int z, const double *ab, const SlotParams &sl)
{
    if (__ballot(active) == 0ull) return;
    const uint32_t key = active ? ((uint32_t)own << 16) | slot_of(x, y, z, sl) : 0xFFFFFFFFu;
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const bool mine = key == k;
        const unsigned long long mask = __ballot(mine);
        double v[D];
#pragma unroll
        for (int m = 0; m < D; ++m) v[m] = wave_sum(mine ? ab[m] : 0.0);
        if (lane == leader) {
            double *out = sl.slots + ((size_t)(k >> 16) * sl.stride + (k & 0xFFFFu)) * (D + 1);
            out[0] = sl.stamp;
#pragma unroll
            for (int m = 0; m < D; ++m) out[1 + m] = v[m];
        }
        pending &= ~mask;
    }
}

template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_adj_lattice(const typename S::raw *__restrict__ fprev,
                                                      const uint16_t *__restrict__ owner, const T *__restrict__ acc_tab,
                                                      const T *__restrict__ uext, const T *__restrict__ lam_in,
                                                      T *__restrict__ lam_out, double *__restrict__ asol,
                                                      double *__restrict__ tau_part, Geom g, StepParams sp, int gx,
                                                      unsigned gxm, SlotParams sl, const double *__restrict__ fpart,
                                                      int init)
{
    const int row = div_magic((int)blockIdx.x, gx, gxm), bx = (int)blockIdx.x - row * gx;
    const int x = bx * 256 + (int)threadIdx.x;
    const bool valid = x < g.nx;
    int y, z;
    if (L::D == 2) {
        y = row;
        z = 0;
    } else {
        z = row / g.ny;
        y = row - z * g.ny;
    }
    double tb = 0.0;
    bool solid_node = false;
    uint16_t own_node = FLUID;
    T abn[3] = {0, 0, 0};
    if (valid) {
        const int N = (int)g.N;
        const int idx = row * g.nx + x;
        T f[L::Q];
        const RowPull<L> rp(x, y, z, idx, bx > 0 && bx * 256 + 256 < g.nx, g);
        pull_row<L, S, T>(fprev, rp, f);
        wall_motion<L, T>(f, y, z, g, sp); // the pre-collision populations, moving walls included
        const uint16_t own = owner[idx];
        const bool solid = own != FLUID;
        const bool fr = solid && sp.frac;
        T a[3] = {0, 0, 0}, acc[3] = {0, 0, 0};
        T chi = 1;
        double dchi[3] = {0, 0, 0};
        if (solid) {
            for (int k = 0; k < 3; ++k) acc[k] = a[k] = acc_tab[3 * own + k];
            if (fr) { // the forward's weight, and its derivative in the centre
                chi = (T)frac_chi(idx, own, sp, dchi);
                for (int k = 0; k < 3; ++k) a[k] = chi * acc[k];
            }
        } else if (sp.has_fluid_acc) {
            for (int k = 0; k < 3; ++k) a[k] = (T)sp.fluid_acc[k];
        }
        T u[3], p;
        moments<L, T>(f, a[0], a[1], a[2], u[0], u[1], u[2], p);
        const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const T om = (T)sp.omega, p3 = T(3) * p, u15 = T(1.5) * uu;
        const bool pen = solid || sp.penalize_all;
        const bool frc = solid || sp.has_fluid_acc;
        // Sums over the velocity set leave out the components of c_q that are
        // zero at compile time (CSum, cdot): 0 * v and x + 0 would stay in the
        // code otherwise, though they change at most the sign of a zero.
        T fneq[L::Q], lam[L::Q], fbar[L::Q];
        CSum<T> Pxx, Pyy, Pzz, Pxy, Pxz, Pyz;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const T cu = cdot<L, T>(q, u[0], u[1], u[2]);
            fneq[q] = f[q] - feq_q<L, T>(q, p3, cu, u15);
            lam[q] = lam_in[q * N + idx];
            if (pen) {
                Pxx.add(L::cx[q] != 0, fneq[q]);
                Pyy.add(L::cy[q] != 0, fneq[q]);
                Pzz.add(L::cz[q] != 0, fneq[q]);
                Pxy.add(L::cx[q] * L::cy[q] > 0, fneq[q]);
                Pxy.sub(L::cx[q] * L::cy[q] < 0, fneq[q]);
                Pxz.add(L::cx[q] * L::cz[q] > 0, fneq[q]);
                Pxz.sub(L::cx[q] * L::cz[q] < 0, fneq[q]);
                Pyz.add(L::cy[q] * L::cz[q] > 0, fneq[q]);
                Pyz.sub(L::cy[q] * L::cz[q] < 0, fneq[q]);
            }
        }
        // f~ = f - om fneq + F + S:  f_bar = lam, fneq_bar = -om lam, F_bar = S_bar = lam
        T fnb[L::Q];
        T omb = 0;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            fbar[q] = lam[q];
            fnb[q] = -om * lam[q];
            omb -= lam[q] * fneq[q];
        }
        T sigb = 0;
        if (pen) {
            // S_q = sigma 4.5 w_q (Pi : c c - tr Pi / 3): Pi_bar and sigma_bar
            const T sigma = fr ? (T)((double)chi * sp.alpha) : (T)sp.alpha;
            const T tr3 = (Pxx.v + Pyy.v + Pzz.v) * T(1.0 / 3.0);
            CSum<T> sxx, syy, szz, sxy, sxz, syz;
            T str = 0;
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                const T wl = T(4.5 * L::w[q]) * lam[q];
                sxx.add(L::cx[q] != 0, wl);
                syy.add(L::cy[q] != 0, wl);
                szz.add(L::cz[q] != 0, wl);
                sxy.add(L::cx[q] * L::cy[q] > 0, wl);
                sxy.sub(L::cx[q] * L::cy[q] < 0, wl);
                sxz.add(L::cx[q] * L::cz[q] > 0, wl);
                sxz.sub(L::cx[q] * L::cz[q] < 0, wl);
                syz.add(L::cy[q] * L::cz[q] > 0, wl);
                syz.sub(L::cy[q] * L::cz[q] < 0, wl);
                str += wl;
                CSum<T> diag, off;
                diag.add(L::cx[q] != 0, Pxx.v);
                diag.add(L::cy[q] != 0, Pyy.v);
                diag.add(L::cz[q] != 0, Pzz.v);
                off.add(L::cx[q] * L::cy[q] > 0, Pxy.v);
                off.sub(L::cx[q] * L::cy[q] < 0, Pxy.v);
                off.add(L::cx[q] * L::cz[q] > 0, Pxz.v);
                off.sub(L::cx[q] * L::cz[q] < 0, Pxz.v);
                off.add(L::cy[q] * L::cz[q] > 0, Pyz.v);
                off.sub(L::cy[q] * L::cz[q] < 0, Pyz.v);
                const T PiCC = off.any ? diag.v + T(2) * off.v : diag.v;
                sigb += wl * (PiCC - tr3);
            }
            // trace term acts on the lattice dimensions only (Pzz = 0 in 2D)
            const T t3 = str * T(1.0 / 3.0);
            const T bxx = sigma * (sxx.v - t3), byy = sigma * (syy.v - t3),
                    bzz = (L::D == 3) ? sigma * (szz.v - t3) : T(0);
            const T bxy = sigma * sxy.v, bxz = sigma * sxz.v, byz = sigma * syz.v;
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                CSum<T> diag, off;
                diag.add(L::cx[q] != 0, bxx);
                diag.add(L::cy[q] != 0, byy);
                diag.add(L::cz[q] != 0, bzz);
                off.add(L::cx[q] * L::cy[q] > 0, bxy);
                off.sub(L::cx[q] * L::cy[q] < 0, bxy);
                off.add(L::cx[q] * L::cz[q] > 0, bxz);
                off.sub(L::cx[q] * L::cz[q] < 0, bxz);
                off.add(L::cy[q] * L::cz[q] > 0, byz);
                off.sub(L::cy[q] * L::cz[q] < 0, byz);
                if (diag.any || off.any) fnb[q] += off.any ? diag.v + T(2) * off.v : diag.v;
            }
        }
        T ub[3] = {0, 0, 0}, ab[3] = {0, 0, 0};
        T gamb = 0;
        if (frc) {
            // F_q = gamma w_q [3 (c - u).a + 9 (c.u)(c.a)],  gamma = 1 - om/2
            const T gpre = T(1) - T(0.5) * om;
            const T ua = L::D == 3 ? u[0] * a[0] + u[1] * a[1] + u[2] * a[2] : u[0] * a[0] + u[1] * a[1];
#pragma unroll
            for (int q = 0; q < L::Q; ++q) {
                const int c[3] = {L::cx[q], L::cy[q], L::cz[q]};
                const T ca = cdot<L, T>(q, a[0], a[1], a[2]);
                const T cu = cdot<L, T>(q, u[0], u[1], u[2]);
                const T gl = gpre * T(L::w[q]) * lam[q];
#pragma unroll
                for (int k = 0; k < L::D; ++k) {
                    if (c[k] != 0) {
                        ub[k] += gl * (T(-3) * a[k] + T(9) * ca * T(c[k]));
                        ab[k] += gl * (T(3) * (T(c[k]) - u[k]) + T(9) * cu * T(c[k]));
                    } else {
                        ub[k] += gl * (T(-3) * a[k]);
                        ab[k] += gl * (T(3) * (-u[k]));
                    }
                }
                gamb += T(L::w[q]) * lam[q] * (T(3) * (ca - ua) + T(9) * cu * ca);
            }
        }
        // fneq = f - feq(p, u)
        T pb = 0;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            fbar[q] += fnb[q];
            const T eb = -fnb[q]; // feq_bar
            const int c[3] = {L::cx[q], L::cy[q], L::cz[q]};
            if (q == 0) {
                pb += eb * T(-3.0 * (1.0 - L::w[0]));
#pragma unroll
                for (int k = 0; k < L::D; ++k) ub[k] += eb * T(-3.0 * L::w[0]) * u[k];
            } else {
                const T cu = cdot<L, T>(q, u[0], u[1], u[2]);
                pb += eb * T(3.0 * L::w[q]);
#pragma unroll
                for (int k = 0; k < L::D; ++k)
                    ub[k] += eb * T(L::w[q]) *
                             (c[k] != 0 ? T(3) * T(c[k]) + T(9) * cu * T(c[k]) - T(3) * u[k] : -(T(3) * u[k]));
            }
        }
        // p = (s/3 - w0 |u|^2 / 2) / (1 - w0)
        const T sb = pb * T(1.0 / (3.0 * (1.0 - L::w[0])));
#pragma unroll
        for (int k = 0; k < L::D; ++k) ub[k] += pb * T(-L::w[0] / (1.0 - L::w[0])) * u[k];
        if (solid)
            for (int k = 0; k < L::D; ++k) ub[k] += chi * uext[3 * own + k];
        if (L::D == 2) ub[2] = 0;
        // u = j + a/2
#pragma unroll
        for (int k = 0; k < L::D; ++k) ab[k] += T(0.5) * ub[k];
        // fractional indicator: chi_bar from a = chi acc, sigma = chi alpha,
        // the sums chi u (U_bar / N . u) and N (N_bar), and in step 0 the
        // initial U^{-1} = sum chi (j + chi acc / 2) / N (w = its adjoint / N);
        // then the weight's adjoint share of acc: chi a_bar (+ chi^2 w / 2)
        double xs[3] = {0, 0, 0}, as[3];
        for (int k = 0; k < 3; ++k) as[k] = (double)ab[k];
        if (fr) {
            const double *fp = fpart + FRAC_STRIDE * own;
            double cb = fp[0] + (double)sigb * sp.alpha;
            for (int k = 0; k < L::D; ++k) {
                cb += (double)ab[k] * (double)acc[k] + (double)uext[3 * own + k] * (double)u[k];
                as[k] = (double)chi * (double)ab[k];
                if (init) {
                    cb += fp[1 + k] * ((double)u[k] + 0.5 * (double)chi * (double)acc[k] - fp[4 + k]);
                    as[k] += 0.5 * (double)chi * (double)chi * fp[1 + k];
                }
            }
            for (int k = 0; k < L::D; ++k) xs[k] = cb * dchi[k];
        }
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            if (q > 0) fbar[q] += cdot<L, T>(q, ub[0], ub[1], ub[2]) + sb;
            // transpose of the pull: f_q(x) came from pull_offset(q, x)
            lam_out[rp.at(q)] = fbar[q];
        }
        if (solid && asol) {
            asol[idx] = as[0];
            asol[N + idx] = as[1];
            if (L::D == 3) asol[2 * N + idx] = as[2];
            if (sp.frac) // uniform
                for (int k = 0; k < L::D; ++k) asol[(size_t)(L::D + k) * N + idx] = xs[k];
        }
        solid_node = solid;
        own_node = own;
        for (int k = 0; k < 3; ++k) abn[k] = ab[k];
        // dL/dtau through om = 1/tau, gamma = 1 - 1/(2 tau), and alpha = 1/tau
        const double om2 = sp.omega * sp.omega;
        tb = (double)omb * (-om2) + (double)gamb * (0.5 * om2);
        if (pen && sp.alpha_tracks_tau) tb += (double)sigb * (double)chi * (-om2);
    }
    __shared__ double part[256 / WAVE][1];
    double s[1] = {tb};
    block_sum<1, 256>(s, part);
    if (threadIdx.x == 0) tau_part[blockIdx.x] += s[0];
    if (sl.slots) { // uniform
        const double abd[3] = {(double)abn[0], (double)abn[1], (double)abn[2]};
        slot_abar<L::D>(solid_node, own_node, x, y, z, abd, sl);
    }
}

// --------------------------------------------------------------- rigid adjoint
struct AdjArrays {
    const double *rec;   // step-n record [np][REC_STRIDE]
    const double *Xbar;  // X_bar^{n+1}  [np*3]
    const double *Abar;  // A_bar^{n+1}
    const double *Upbar; // adjoint of U^n as the next step's U^{n-1}
    double *Xbar_out;    // X_bar^n
    double *Upbar_out;   // adjoint of U^{n-1}
    double *uext_d;      // U_bar^n / N per particle (broadcast), [np*3]
    float *uext_f;
    double *acc_d; // a_i of step n
    float *acc_f;
    double *rho_g, *g_g; // accumulated partials per particle
    double *fpart, *geo; // fractional indicator only: see AdjArraysHost
};

__device__ __forceinline__ double particle_volume(int shape, double a, double b)
{
    if (shape == LBM_DISK) return M_PI * a * a;
    if (shape == LBM_ELLIPSE) return M_PI * a * b;
    return 4.0 / 3.0 * M_PI * a * a * a;
}

// J v for the pair-force Jacobian J = dT/dd of T(d) = (C/eps_p) s^2 d/|d|
// (form 0) or (C/eps_p) s^2 d (form 1), s = (cut - |d|)/delta; J is symmetric.
__device__ __forceinline__ void pair_jac_apply(double C, const double *d, double dist, double cut,
                                               const RigidParams &rp, const double *v, double *out)
{
    const double k = C / rp.eps_p, s = (cut - dist) / rp.delta;
    double dh[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
    double a1, a2;
    if (rp.cform == 1) {
        a2 = s * s;
        a1 = -2.0 * s * dist / rp.delta;
    } else {
        a2 = s * s / dist;
        a1 = -2.0 * s / rp.delta - s * s / dist;
    }
    const double dv = dh[0] * v[0] + dh[1] * v[1] + dh[2] * v[2];
    for (int m = 0; m < 3; ++m) out[m] += k * (a1 * dv * dh[m] + a2 * v[m]);
}

// What the transposed Algorithm 1 needs of one particle in step n: its centre
// X^n (Y[0]) and prediction X^n + U_bar^n (Y[1]), the adjoint of its
// correction F_bar = c (X_bar + 2 A_bar)/2 with c = 1/(2 rho N), its radius
// and collision constant.
struct AdjBody {
    double Y[2][3];
    double F[3];
    double R, C;
};

__device__ __forceinline__ void adj_positions(const double *r, int d, AdjBody &b)
{
    for (int k = 0; k < 3; ++k) {
        b.Y[0][k] = r[k];
        b.Y[1][k] = r[k] + (k < d ? 0.5 * (r[4 + k] + r[14 + k]) : 0.0);
    }
}

__device__ __forceinline__ void adj_force_bar(const double *Xb, const double *Ab, double Ni, double rho, int d, double *F)
{
    const double c = Ni > 0 ? 1.0 / (2.0 * rho * Ni) : 0.0;
    for (int k = 0; k < 3; ++k) F[k] = k < d ? 0.5 * c * (Xb[k] + 2.0 * Ab[k]) : 0.0;
}

// Partner i's share of particle j's adjoint: acc[w] += J_ji F_j - J_ij F_i at
// positions w (0: X^n, 1: prediction), unit[w] += the pair force on j per
// unit collision constant.
__device__ __forceinline__ void adj_pair(const AdjBody &bj, const AdjBody &bi, const RigidParams &rp, const Geom &g,
                                         double acc[2][3], double unit[2][3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    const double cut = bi.R + bj.R + rp.delta;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        double dv[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k >= rp.d) continue;
            dv[k] = bj.Y[w][k] - bi.Y[w][k];
            if (per[k]) {
                const double h = 0.5 * n[k];
                if (dv[k] > h) dv[k] -= n[k];
                else if (dv[k] < -h) dv[k] += n[k];
            }
        }
        const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (!(dist <= cut) || dist == 0.0) continue;
        pair_jac_apply(bj.C, dv, dist, cut, rp, bj.F, acc[w]);
        double neg[3] = {0, 0, 0};
        pair_jac_apply(bi.C, dv, dist, cut, rp, bi.F, neg);
        for (int k = 0; k < 3; ++k) acc[w][k] -= neg[k];
        const double s = (cut - dist) / rp.delta;
        const double sc = (rp.cform == 1 ? s * s : s * s / dist) / rp.eps_p;
        for (int k = 0; k < 3; ++k) unit[w][k] += sc * dv[k];
    }
}

// Closing of the transposed Algorithm 1 for particle j once the partner sums
// acc and unit are complete: the wall Jacobians (mirror particle), then
// X_bar^n, the adjoint of U^{n-1}, the broadcast U_bar^n / N, the acceleration
// of the step's nodes; drho and dg receive the density and |g| partials of
// the collision constant and of 1/(2M).  Xbj, Abj, Upbj: X_bar^{n+1}, A_bar^{n+1}
// and the adjoint of U^n of particle j; Nj, Aj: N and A^n of its record rj.
// With the fractional indicator it also leaves the lattice adjoint of step n
// the terms of j's chi_bar (A.fpart) and the indicator's centre (A.geo).
__device__ void adj_rigid_close(int j, const AdjArrays &A, const RigidParams &rp, const Geom &g, const AdjBody &bj,
                                const double *rj, double Nj, const double *Aj, double rho, double V, const double *Xbj,
                                const double *Abj, const double *Upbj, double acc[2][3], double unit[2][3],
                                double &drho, double &dg)
{
    const int d = rp.d;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    const double Rj = bj.R, Cj = bj.C;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k >= d || per[k]) continue;
            const double walls[2] = {-0.5, n[k] - 0.5};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double dv = 2.0 * (bj.Y[w][k] - walls[s]);
                const double dist = fabs(dv);
                if (dist > 2.0 * Rj + rp.delta) continue;
                const double qq = (2.0 * Rj + rp.delta - dist) / rp.delta;
                const double kw = Cj / rp.eps_w;
                double dT, tu;
                if (rp.cform == 1) {
                    dT = kw * (2.0 * qq * qq - 4.0 * qq * dist / rp.delta);
                    tu = qq * qq * dv / rp.eps_w;
                } else {
                    dT = -4.0 * kw * qq / rp.delta;
                    tu = qq * qq * (dv >= 0 ? 1.0 : -1.0) / rp.eps_w;
                }
                acc[w][k] += dT * bj.F[k];
                unit[w][k] += tu;
            }
        }
    }
    const double cj = Nj > 0 ? 1.0 / (2.0 * rho * Nj) : 0.0;
    double corrb_dot_F = 0.0, Cbar = 0.0, UbU = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double corrb = k < d ? Xbj[k] + 2.0 * Abj[k] : 0.0;
        corrb_dot_F += corrb * 0.5 * Cj * (unit[0][k] + unit[1][k]);
        Cbar += bj.F[k] * (unit[0][k] + unit[1][k]);
        const double Xsb = k < d ? Xbj[k] + acc[1][k] : 0.0;
        A.Xbar_out[3 * j + k] = k < d ? Xsb + acc[0][k] : 0.0;
        A.Upbar_out[3 * j + k] = 0.5 * Xsb;
        const double Unb = 0.5 * Xsb + Upbj[k];
        const double ue = Nj > 0 ? Unb / Nj : 0.0;
        A.uext_d[3 * j + k] = ue;
        A.uext_f[3 * j + k] = (float)ue;
        UbU += Unb * rj[4 + k];
        if (A.fpart) {
            A.fpart[FRAC_STRIDE * j + 1 + k] = Nj > 0 ? 0.5 * Xsb / Nj : 0.0;
            A.fpart[FRAC_STRIDE * j + 4 + k] = rj[14 + k];
            A.geo[4 * j + k] = rj[k];
        }
    }
    if (A.fpart) {
        // N enters U^n = sum chi u / N and c = 1/(2 rho N), dc/dN = -c/N
        A.fpart[FRAC_STRIDE * j] = Nj > 0 ? (-UbU - corrb_dot_F * cj) / Nj : 0.0;
        A.geo[4 * j + 3] = Rj;
    }
    // c = 1/(2 rho N): dc/drho = -c/rho;  C = (rho - rho_f)|g| V (form 0) or (rho - rho_f)|g| (form 1)
    const double Vc = rp.cform == 1 ? 1.0 : V;
    drho = corrb_dot_F * (-cj / rho) + Cbar * rp.gmag * Vc;
    dg = Cbar * (rho - rp.rho_f) * Vc;
    // acceleration of the particle's nodes during step n: b g + A^n
    const double bj_ = rp.gform == 0 ? 1.0 - rp.rho_f / rho : rho / rp.rho_f - 1.0;
    for (int k = 0; k < 3; ++k) {
        const double acc_k = k < d ? bj_ * rp.g[k] + Aj[k] : 0.0;
        A.acc_d[3 * j + k] = acc_k;
        A.acc_f[3 * j + k] = (float)acc_k;
    }
}

__device__ __forceinline__ AdjBody load_body(const AdjArrays &A, const PartDev &P, int i, int d)
{
    AdjBody b;
    const double *r = A.rec + REC_STRIDE * i;
    adj_positions(r, d, b);
    adj_force_bar(A.Xbar + 3 * i, A.Abar + 3 * i, r[13], P.rho_s[i], d, b.F);
    b.R = P.a[i];
    b.C = P.Cc[i];
    return b;
}

// Many bodies: one workgroup per particle j, partners across lanes.
__global__ __launch_bounds__(256) void k_adj_rigid(AdjArrays A, PartDev P, RigidParams rp, Geom g)
{
    const int j = blockIdx.x, d = rp.d, np = rp.np;
    __shared__ double part[256 / WAVE][12];
    const AdjBody bj = load_body(A, P, j, d);
    // what the closing needs, loaded up front so its latency overlaps the sums
    const double *rj = A.rec + REC_STRIDE * j;
    double Xbj[3], Abj[3], Upbj[3], Aj[3];
    for (int k = 0; k < 3; ++k) {
        Xbj[k] = A.Xbar[3 * j + k];
        Abj[k] = A.Abar[3 * j + k];
        Upbj[k] = A.Upbar[3 * j + k];
        Aj[k] = rj[10 + k];
    }
    const double Nj = rj[13], rho = P.rho_s[j], V = particle_volume(P.shape[j], P.a[j], P.b[j]);
    const double rg0 = A.rho_g[j], gg0 = A.g_g[j];
    double acc[2][3] = {{0, 0, 0}, {0, 0, 0}}, unit[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int i = threadIdx.x; i < np; i += 256) {
        if (i == j) continue;
        adj_pair(bj, load_body(A, P, i, d), rp, g, acc, unit);
    }
    double s[12];
    for (int w = 0; w < 2; ++w)
        for (int k = 0; k < 3; ++k) {
            s[w * 3 + k] = acc[w][k];
            s[6 + w * 3 + k] = unit[w][k];
        }
    block_sum<12, 256>(s, part);
    if (threadIdx.x != 0) return;
    for (int w = 0; w < 2; ++w)
        for (int k = 0; k < 3; ++k) {
            acc[w][k] = s[w * 3 + k];
            unit[w][k] = s[6 + w * 3 + k];
        }
    double drho, dg;
    adj_rigid_close(j, A, rp, g, bj, rj, Nj, Aj, rho, V, Xbj, Abj, Upbj, acc, unit, drho, dg);
    A.rho_g[j] = rg0 + drho;
    A.g_g[j] = gg0 + dg;
}

// ------------------------------------------------------------ particle adjoint
// A_bar^n_i = sum of a_bar over the nodes of particle i (step n indicator);
// a = b_i g + A_i gives the density and |g| partials.

// This lane's partial sums of the C per-node fields of asol (a_bar, then,
// with the fractional indicator, chi_bar dchi/dX) over the owned cells lane,
// lane + nl, ... of box b, the loads of U cells in flight together; field m
// goes to s[m] for m < D and to s[3 + m - D] after.
template <int D, int C, int U>
__device__ __forceinline__ void cell_abar(const uint16_t *__restrict__ owner, const double *__restrict__ asol,
                                          const Geom &g, int i, const Box &b, int lane, int nl, double *s)
{
    const int N = (int)g.N;
    CellWalk w(b.ext[0] > 0 ? b.ext[0] : 1, b.ext[1] > 0 ? b.ext[1] : 1, lane, nl);
    for (int base = lane; base < b.cells; base += U * nl) {
        uint16_t o[U];
        double v[U][C];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int xu, yu, zu;
            const int node = base + u * nl < b.cells ? walk_node(b, w, g, xu, yu, zu) : 0;
            w.next();
            o[u] = owner[node];
#pragma unroll
            for (int k = 0; k < C; ++k) v[u][k] = asol[(size_t)k * N + node];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * nl >= b.cells || o[u] != (uint16_t)i) continue;
#pragma unroll
            for (int k = 0; k < C; ++k) s[k < D ? k : 3 + k - D] += v[u][k];
        }
    }
}

// Closing for particle i from the totals t: A_bar^n into Abar_out, and the
// density and |g| partials through a = b_i g + A_i.
__device__ __forceinline__ void adj_particle_close(const double *t, double rho, const RigidParams &rp, double *Abar_out,
                                                   double &drho, double &dg, bool store = true)
{
    const double bi = rp.gform == 0 ? 1.0 - rp.rho_f / rho : rho / rp.rho_f - 1.0;
    const double dbdrho = rp.gform == 0 ? rp.rho_f / (rho * rho) : 1.0 / rp.rho_f;
    double ag = 0.0, aghat = 0.0;
    for (int k = 0; k < 3; ++k) {
        if (store) Abar_out[k] = t[k];
        ag += t[k] * rp.g[k];
        aghat += rp.gmag > 0 ? t[k] * rp.g[k] / rp.gmag : 0.0;
    }
    drho = ag * dbdrho;
    dg = bi * aghat;
}

// Box of particle i in step n: around the recorded centre r.
__device__ __forceinline__ Box adj_box(const double *r, double R, const Geom &g, int d)
{
    int lo[3], hi[3];
    centre_box(r, R, g, d, lo, hi);
    return make_box(lo, hi);
}

// C = D: A_bar^n; C = 2 D (fractional indicator): also X_bar^n += the sum of
// chi_bar dchi/dX over the particle's nodes.
template <int D, int C>
__global__ __launch_bounds__(256) void k_adj_particles(const uint16_t *__restrict__ owner,
                                                        const double *__restrict__ asol, const double *__restrict__ rec,
                                                        PartDev P, RigidParams rp, Geom g, double *__restrict__ Abar_out,
                                                        double *__restrict__ rho_g, double *__restrict__ g_g,
                                                        double *__restrict__ Xbar_n)
{
    constexpr int NS = C > D ? 6 : 3;
    __shared__ double part[256 / WAVE][NS];
    const int i = blockIdx.x;
    const Box b = adj_box(rec + REC_STRIDE * i, P.a[i], g, D);
    const double rho = P.rho_s[i], rg0 = rho_g[i], gg0 = g_g[i];
    double s[6] = {0, 0, 0, 0, 0, 0};
    cell_abar<D, C, UNR>(owner, asol, g, i, b, threadIdx.x, 256, s);
    block_sum<NS, 256>(s, part);
    if (threadIdx.x != 0) return;
    double drho, dg;
    adj_particle_close(s, rho, rp, Abar_out + 3 * i, drho, dg);
    rho_g[i] = rg0 + drho;
    g_g[i] = gg0 + dg;
    if (C > D)
        for (int k = 0; k < D; ++k) Xbar_n[3 * i + k] += s[3 + k];
}

// Steps with slots: one workgroup per particle j closes the particle adjoint
// of step n from j's records (A_bar^n_j and its density and |g| partials),
// then, if rigid, runs the rigid adjoint of step n - 1 for j (A: the arrays of
// that step).  The partners in reach (|X_i - X_j| <= R_i + R_j + delta + 0.6
// at X^{n-1}: the prediction moves each body by at most 0.3) are tested by
// waves 1.., one bit per particle in LDS, while wave 0 sums j's records; after one barrier wave 0 sums each partner's records for its
// A_bar^n, which the rigid adjoint needs through the partner's force
// adjoint, in index order; every lane accumulates the same pair terms and
// lane 0 writes.  Abar_n: A_bar^n out.
template <int D, int BS>
__global__ __launch_bounds__(BS) void k_adj_fused(AdjArrays A, PartDev P, RigidParams rp, Geom g, SlotParams sl,
                                                  double *__restrict__ Abar_n, int rigid)
{
    constexpr int W1 = D + 1;
    const int j = blockIdx.x, np = rp.np, lane = threadIdx.x & (WAVE - 1);
    __shared__ unsigned long long s_reach[MAX_NP / WAVE]; // bit i: particle i is in reach
    const double rho = P.rho_s[j], rg0 = A.rho_g[j], gg0 = A.g_g[j];
    const double *rj = A.rec + REC_STRIDE * j;
    double Xj[3];
    for (int k = 0; k < 3; ++k) Xj[k] = rj[k];
    const double Rj = P.a[j];
    // the partners in reach at step n - 1 (positions of its record), tested by
    // waves 1.. while wave 0 sums j's records
    if (rigid && threadIdx.x >= WAVE) {
        const int n[3] = {g.nx, g.ny, g.nz};
        const int per[3] = {g.per_x, g.per_y, g.per_z};
        for (int i0 = 0; i0 < np; i0 += BS - WAVE) { // uniform
            const int i = i0 + (int)threadIdx.x - WAVE;
            bool in = false;
            if (i < np && i != j) {
                double dv2 = 0.0;
                for (int k = 0; k < D; ++k) {
                    double dk = Xj[k] - A.rec[REC_STRIDE * i + k];
                    if (per[k]) {
                        const double h = 0.5 * n[k];
                        if (dk > h) dk -= n[k];
                        else if (dk < -h) dk += n[k];
                    }
                    dv2 += dk * dk;
                }
                const double reach = Rj + P.a[i] + rp.delta + 0.6;
                in = dv2 <= reach * reach;
            }
            const unsigned long long m = __ballot(in);
            if (lane == 0 && i < np) s_reach[i / WAVE] = m;
        }
    }
    // 1. A_bar^n_j from j's records: wave 0 in 2D; the whole workgroup in 3D
    // (thousands of records), its sum then handed to wave 0
    double t[3] = {0, 0, 0}, drho = 0.0, dg = 0.0;
    if (D == 3 || threadIdx.x < WAVE) {
        const double *sj = sl.slots + (size_t)j * sl.stride * W1;
        const int t0 = D == 3 ? (int)threadIdx.x : lane, nt = D == 3 ? BS : WAVE;
        for (int q = t0; q < sl.stride; q += nt) {
            double rv[W1];
#pragma unroll
            for (int m = 0; m < W1; ++m) rv[m] = sj[(size_t)q * W1 + m];
            if (rv[0] == sl.stamp)
#pragma unroll
                for (int m = 0; m < D; ++m) t[m] += rv[1 + m];
        }
    }
    if constexpr (D == 3) {
        __shared__ double part[BS / WAVE][3];
        __shared__ double s_tot[3];
        block_sum<3, BS>(t, part);
        if (threadIdx.x == 0)
            for (int m = 0; m < 3; ++m) s_tot[m] = t[m];
        __syncthreads();
        for (int m = 0; m < 3; ++m) t[m] = s_tot[m];
    } else if (threadIdx.x < WAVE) {
#pragma unroll
        for (int m = 0; m < 3; ++m) t[m] = wave_sum(t[m]);
    }
    if (threadIdx.x < WAVE) { // wave 0
        adj_particle_close(t, rho, rp, Abar_n + 3 * j, drho, dg, lane == 0);
        if (!rigid && lane == 0) {
            A.rho_g[j] = rg0 + drho;
            A.g_g[j] = gg0 + dg;
        }
    }
    if (!rigid) return; // uniform
    __syncthreads();    // the reach masks are complete
    if (threadIdx.x >= WAVE) return;

    // 2. the rigid adjoint of step n - 1 for j, by wave 0
    double Xbj[3], Upbj[3], Aj[3];
    for (int k = 0; k < 3; ++k) {
        Xbj[k] = A.Xbar[3 * j + k];
        Upbj[k] = A.Upbar[3 * j + k];
        Aj[k] = rj[10 + k];
    }
    const double Nj = rj[13], V = particle_volume(P.shape[j], P.a[j], P.b[j]);
    AdjBody bj;
    adj_positions(rj, D, bj);
    adj_force_bar(Xbj, t, Nj, rho, D, bj.F);
    bj.R = Rj;
    bj.C = P.Cc[j];
    double acc[2][3] = {{0, 0, 0}, {0, 0, 0}}, unit[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int i0 = 0; i0 < np; i0 += WAVE) { // uniform
        for (unsigned long long m = s_reach[i0 / WAVE]; m; m &= m - 1ull) { // uniform
            const int ii = i0 + __ffsll((long long)m) - 1;
            const double *si = sl.slots + (size_t)ii * sl.stride * W1;
            double u[3] = {0, 0, 0};
            for (int q = lane; q < sl.stride; q += WAVE) {
                double rv[W1];
#pragma unroll
                for (int mm = 0; mm < W1; ++mm) rv[mm] = si[(size_t)q * W1 + mm];
                if (rv[0] == sl.stamp)
#pragma unroll
                    for (int mm = 0; mm < D; ++mm) u[mm] += rv[1 + mm];
            }
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) u[mm] = wave_sum(u[mm]);
            AdjBody bi;
            const double *ri = A.rec + REC_STRIDE * ii;
            adj_positions(ri, D, bi);
            adj_force_bar(A.Xbar + 3 * ii, u, ri[13], P.rho_s[ii], D, bi.F);
            bi.R = P.a[ii];
            bi.C = P.Cc[ii];
            adj_pair(bj, bi, rp, g, acc, unit);
        }
    }
    if (lane != 0) return;
    double drho2, dg2;
    adj_rigid_close(j, A, rp, g, bj, rj, Nj, Aj, rho, V, Xbj, t, Upbj, acc, unit, drho2, dg2);
    A.rho_g[j] = (rg0 + drho) + drho2;
    A.g_g[j] = (gg0 + dg) + dg2;
}

// U^{-1} = U^0 was measured with a = b g on every node of the particle:
// dU^{-1}/da = 1/2 gives the density and |g| partials of the initial state.
__device__ __forceinline__ void adj_initial_terms(double rho, const double *Upb, const RigidParams &rp, double &drho,
                                                  double &dg)
{
    const double bi = rp.gform == 0 ? 1.0 - rp.rho_f / rho : rho / rp.rho_f - 1.0;
    const double dbdrho = rp.gform == 0 ? rp.rho_f / (rho * rho) : 1.0 / rp.rho_f;
    double ag = 0.0, aghat = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double ab = 0.5 * Upb[k];
        ag += ab * rp.g[k];
        aghat += rp.gmag > 0 ? ab * rp.g[k] / rp.gmag : 0.0;
    }
    drho = ag * dbdrho;
    dg = bi * aghat;
}

__global__ void k_adj_initial(PartDev P, RigidParams rp, const double *__restrict__ Upbar, double *__restrict__ rho_g,
                              double *__restrict__ g_g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rp.np) return;
    double drho, dg;
    adj_initial_terms(P.rho_s[i], Upbar + 3 * i, rp, drho, dg);
    rho_g[i] += drho;
    g_g[i] += dg;
}

// ----------------------------------------------------------------- launchers
hipError_t launch_adj_lattice(lbm_ctx *c, const void *fprev, const uint16_t *owner, const double *uext_d,
                              const float *uext_f, const double *acc_d, const float *acc_f, const void *lam_in,
                              void *lam_out, double *asol, double *tau_part, const SlotParams &sl,
                              const double *fpart, const double *geo, int init)
{
    if (c->sp.frac && (!fpart || !geo || !asol)) return hipErrorInvalidValue;
    const int gx = (c->geo.nx + 255) / 256;
    const unsigned blocks = (unsigned)gx * (unsigned)(c->geo.ny * c->geo.nz);
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        const bool dbl = std::is_same<Tt, double>::value;
        const Tt *acc = dbl ? (const Tt *)acc_d : (const Tt *)acc_f;
        const Tt *uext = dbl ? (const Tt *)uext_d : (const Tt *)uext_f;
        StepParams sp = c->sp;
        sp.geo = geo; // step n's indicator centres (fractional indicator)
        hipLaunchKernelGGL((k_adj_lattice<Lt, St, Tt>), dim3(blocks), dim3(256), 0, c->stream,
                           (const typename St::raw *)fprev, owner, acc, uext, (const Tt *)lam_in, (Tt *)lam_out, asol,
                           tau_part, c->geo, sp, gx, magic_for(gx), sl, fpart, init);
        return hipGetLastError();
    });
}

static AdjArrays adj_arrays(const AdjArraysHost &h)
{
    return AdjArrays{h.rec,    h.Xbar,   h.Abar,  h.Upbar, h.Xbar_out, h.Upbar_out, h.uext_d,
                     h.uext_f, h.acc_d,  h.acc_f, h.rho_g, h.g_g,      h.fpart,     h.geo};
}

hipError_t launch_adj_rigid(lbm_ctx *c, const PartDev &P, const AdjArraysHost &h)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_adj_rigid, dim3(c->np), dim3(256), 0, c->stream, adj_arrays(h), P, rp, c->geo);
    return hipGetLastError();
}

hipError_t launch_adj_particles(lbm_ctx *c, const PartDev &P, const uint16_t *owner, const double *asol,
                                const double *rec, double *Abar_out, double *rho_g, double *g_g, double *Xbar_n)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    const bool fr = c->sp.frac != 0;
    if (fr && !Xbar_n) return hipErrorInvalidValue;
    const dim3 grid(c->np), block(256);
    if (c->d == 2 && !fr)
        hipLaunchKernelGGL((k_adj_particles<2, 2>), grid, block, 0, c->stream, owner, asol, rec, P, rp, c->geo, Abar_out,
                           rho_g, g_g, Xbar_n);
    else if (c->d == 2)
        hipLaunchKernelGGL((k_adj_particles<2, 4>), grid, block, 0, c->stream, owner, asol, rec, P, rp, c->geo, Abar_out,
                           rho_g, g_g, Xbar_n);
    else if (!fr)
        hipLaunchKernelGGL((k_adj_particles<3, 3>), grid, block, 0, c->stream, owner, asol, rec, P, rp, c->geo, Abar_out,
                           rho_g, g_g, Xbar_n);
    else
        hipLaunchKernelGGL((k_adj_particles<3, 6>), grid, block, 0, c->stream, owner, asol, rec, P, rp, c->geo, Abar_out,
                           rho_g, g_g, Xbar_n);
    return hipGetLastError();
}

hipError_t launch_adj_fused(lbm_ctx *c, const PartDev &P, const AdjArraysHost &h, const SlotParams &sl,
                            double *Abar_n, int rigid)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    if (c->d == 2)
        hipLaunchKernelGGL((k_adj_fused<2, 256>), dim3(c->np), dim3(256), 0, c->stream, adj_arrays(h), P, rp, c->geo, sl,
                           Abar_n, rigid);
    else
        hipLaunchKernelGGL((k_adj_fused<3, 256>), dim3(c->np), dim3(256), 0, c->stream, adj_arrays(h), P, rp, c->geo, sl,
                           Abar_n, rigid);
    return hipGetLastError();
}

hipError_t launch_adj_initial(lbm_ctx *c, const PartDev &P, const double *Upbar, double *rho_g, double *g_g)
{
    if (c->np == 0) return hipSuccess;
    RigidParams rp = c->rp;
    rp.np = c->np;
    hipLaunchKernelGGL(k_adj_initial, dim3((c->np + 255) / 256), dim3(256), 0, c->stream, P, rp, Upbar, rho_g, g_g);
    return hipGetLastError();
}

} // namespace lbm
