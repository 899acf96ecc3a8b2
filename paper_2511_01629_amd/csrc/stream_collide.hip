// stream_collide.hip -- the fused lattice update for gfx950.
//
// One thread per node.  Populations live structure-of-arrays, [Q][N] with x
// fastest, in two ping-pong buffers holding post-collision values f~.  A
// thread pulls f_q(x) = f~_q(x - c_q) (sec. 2.2 eq. 10; halfway bounce-back
// f_q(x) = f~_opp(q)(x) when x - c_q lies behind a wall, wrap-around on a
// periodic axis), forms u and p (eq. 15a-b), relaxes towards f^eq (eq. 13),
// adds the Guo force (eq. 14) and, on solid nodes, the penalization source of
// eq. (17), and writes f~ back.  Every population is read once and written
// once: 2 Q s bytes per node, the HBM roofline of the step.
//
// The owner map (uint16, FLUID = 0xFFFF) selects the solid branch; a
// wavefront with no solid node never executes it.  Solid nodes also write
// their velocity (FP64) for the per-particle momentum sums.
#include "ctx.h"
#include "lattice.h"

namespace lbm {

template <class L>
__device__ __forceinline__ void coords(int idx, const Geom &g, int &x, int &y, int &z)
{
    if (L::D == 2) {
        y = idx / g.nx;
        x = idx - y * g.nx;
        z = 0;
    } else {
        int row = idx / g.nx;
        x = idx - row * g.nx;
        z = row / g.ny;
        y = row - z * g.ny;
    }
}

// Source offset of population q pulled into node (x,y,z): the neighbour
// x - c_q (wrapped on periodic axes) or, behind a wall, the opposite
// population of the node itself.
template <class L>
__device__ __forceinline__ int pull_offset(int q, int idx, int x, int y, int z, const Geom &g, int N)
{
    int sx = x - L::cx[q], sy = y - L::cy[q], sz = z - L::cz[q];
    bool wall = false;
    if (L::cx[q] != 0) {
        if (sx < 0) {
            if (g.per_x) sx += g.nx; else wall = true;
        } else if (sx >= g.nx) {
            if (g.per_x) sx -= g.nx; else wall = true;
        }
    }
    if (L::cy[q] != 0) {
        if (sy < 0) {
            if (g.per_y) sy += g.ny; else wall = true;
        } else if (sy >= g.ny) {
            if (g.per_y) sy -= g.ny; else wall = true;
        }
    }
    if (L::D == 3 && L::cz[q] != 0) {
        if (sz < 0) {
            if (g.per_z) sz += g.nz; else wall = true;
        } else if (sz >= g.nz) {
            if (g.per_z) sz -= g.nz; else wall = true;
        }
    }
    return wall ? L::opp[q] * N + idx : q * N + (sx + g.nx * (sy + g.ny * sz));
}

template <class L, class S, class T>
__device__ __forceinline__ void pull(const typename S::raw *__restrict__ fin, int idx, int x, int y, int z,
                                     const Geom &g, int N, T *f)
{
#pragma unroll
    for (int q = 0; q < L::Q; ++q) f[q] = ld<S, T>(fin + pull_offset<L>(q, idx, x, y, z, g, N));
}

// u = sum f c + a/2 and p = (cs^2 sum_{q>0} f - w0 |u|^2 / 2)/(1 - w0)  (eq. 15a-b)
template <class L, class T>
__device__ __forceinline__ void moments(const T *f, T ax, T ay, T az, T &ux, T &uy, T &uz, T &p)
{
    T jx = 0, jy = 0, jz = 0, s = 0;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
        if (L::cx[q] > 0) jx += f[q];
        if (L::cx[q] < 0) jx -= f[q];
        if (L::cy[q] > 0) jy += f[q];
        if (L::cy[q] < 0) jy -= f[q];
        if (L::cz[q] > 0) jz += f[q];
        if (L::cz[q] < 0) jz -= f[q];
        s += f[q];
    }
    ux = jx + T(0.5) * ax;
    uy = jy + T(0.5) * ay;
    uz = (L::D == 3) ? jz + T(0.5) * az : T(0);
    const T uu = ux * ux + uy * uy + uz * uz;
    constexpr double w0 = L::w[0];
    p = (T(1.0 / 3.0) * s - T(0.5 * w0) * uu) * T(1.0 / (1.0 - w0));
}

// f^eq_q of eq. (13) with cs^2 = 1/3: q = 0: -(1-w0) 3p - w0 1.5|u|^2;
// q > 0: w_q (3p + 3 c.u + 4.5 (c.u)^2 - 1.5|u|^2)
template <class L, class T>
__device__ __forceinline__ T feq_q(int q, T p3, T cu, T u15)
{
    if (q == 0) return T(-(1.0 - L::w[0])) * p3 - T(L::w[0]) * u15;
    return T(L::w[q]) * (p3 + T(3) * cu + T(4.5) * cu * cu - u15);
}

// Collision of one node, in place: f holds the pulled populations on entry
// and f~ on return (right side of eq. 10 with F of eq. 14 and, on solid
// nodes, S of eq. 17).  Writes the velocity of solid nodes for the sums.
template <class L, class T>
__device__ __forceinline__ void collide_node(T *f, uint16_t own, const T *__restrict__ acc_tab, const StepParams &sp,
                                             int32_t *__restrict__ flags, double *__restrict__ usol, int idx, int N)
{
    const bool solid = own != FLUID;
    T ax = 0, ay = 0, az = 0;
    if (solid) {
        ax = acc_tab[3 * own + 0];
        ay = acc_tab[3 * own + 1];
        az = acc_tab[3 * own + 2];
    } else if (sp.has_fluid_acc) {
        ax = (T)sp.fluid_acc[0];
        ay = (T)sp.fluid_acc[1];
        az = (T)sp.fluid_acc[2];
    }
    T ux, uy, uz, p;
    moments<L, T>(f, ax, ay, az, ux, uy, uz, p);
    const T uu = ux * ux + uy * uy + uz * uz;
    if (!(uu < T(0.09))) flags[0] = 1; // |u| > 0.3 or not finite
    const T om = (T)sp.omega;
    const T p3 = T(3) * p, u15 = T(1.5) * uu;

    const bool pen = solid || sp.penalize_all;
    const bool frc = solid || sp.has_fluid_acc;
    if (!pen && !frc) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const T cu = T(L::cx[q]) * ux + T(L::cy[q]) * uy + T(L::cz[q]) * uz;
            f[q] = f[q] - om * (f[q] - feq_q<L, T>(q, p3, cu, u15));
        }
        return;
    }
    // solid (or forced) node
    T fneq[L::Q];
    T Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const T cu = T(L::cx[q]) * ux + T(L::cy[q]) * uy + T(L::cz[q]) * uz;
        fneq[q] = f[q] - feq_q<L, T>(q, p3, cu, u15);
        if (L::cx[q] != 0) Pxx += fneq[q];
        if (L::cy[q] != 0) Pyy += fneq[q];
        if (L::cz[q] != 0) Pzz += fneq[q];
        if (L::cx[q] * L::cy[q] > 0) Pxy += fneq[q];
        if (L::cx[q] * L::cy[q] < 0) Pxy -= fneq[q];
        if (L::cx[q] * L::cz[q] > 0) Pxz += fneq[q];
        if (L::cx[q] * L::cz[q] < 0) Pxz -= fneq[q];
        if (L::cy[q] * L::cz[q] > 0) Pyz += fneq[q];
        if (L::cy[q] * L::cz[q] < 0) Pyz -= fneq[q];
    }
    const T al = pen ? (T)sp.alpha : T(0);
    const T trace3 = (Pxx + Pyy + Pzz) * T(1.0 / 3.0);
    const T gpre = T(1) - T(0.5) * om;
    const T ua = ux * ax + uy * ay + uz * az;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const T cx = T(L::cx[q]), cy = T(L::cy[q]), cz = T(L::cz[q]);
        // S_q = alpha w_q / (2 cs^4) Pi^neq : (c c - cs^2 I)   (eq. 17)
        const T PiCC = cx * cx * Pxx + cy * cy * Pyy + cz * cz * Pzz +
                       T(2) * (cx * cy * Pxy + cx * cz * Pxz + cy * cz * Pyz);
        const T Sq = al * T(4.5 * L::w[q]) * (PiCC - trace3);
        // F_q = (1 - 1/(2 tau)) w_q [3 (c - u).a + 9 (c.u)(c.a)]   (eq. 14)
        const T cu = cx * ux + cy * uy + cz * uz;
        const T ca = cx * ax + cy * ay + cz * az;
        const T F = gpre * T(L::w[q]) * (T(3) * (ca - ua) + T(9) * cu * ca);
        f[q] = f[q] - om * fneq[q] + F + Sq;
    }
    if (solid) {
        usol[idx] = (double)ux;
        usol[N + idx] = (double)uy;
        if (L::D == 3) usol[2 * N + idx] = (double)uz;
    }
}

// The lattice update, one node per lane.  Each workgroup covers 256
// consecutive nodes of one row (fixed y, z), so the row and the wall tests of
// y and z are uniform and no index division is needed.  Every population is
// read once (pull) and written once: 2 Q s bytes per node.
//
// Measured alternatives that did not pay on MI355X: two adjacent nodes per
// lane (element-aligned 2-wide loads, or aligned loads with a DPP lane shift
// for the x-shifted directions), two strided nodes per lane, and an XCD-aware
// remap of the workgroup order.
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_stream_collide(const typename S::raw *__restrict__ fin,
                                                         typename S::raw *__restrict__ fout,
                                                         const uint16_t *__restrict__ owner,
                                                         const T *__restrict__ acc_tab, double *__restrict__ usol,
                                                         int32_t *__restrict__ flags, Geom g, StepParams sp, int gx)
{
    const int row = blockIdx.x / gx, bx = blockIdx.x - row * gx; // uniform
    const int x = bx * 256 + (int)threadIdx.x;
    if (x >= g.nx) return;
    int y, z;
    if (L::D == 2) {
        y = row;
        z = 0;
    } else {
        z = row / g.ny;
        y = row - z * g.ny;
    }
    const int N = (int)g.N;
    const int idx = row * g.nx + x;
    T f[L::Q];
    pull<L, S, T>(fin, idx, x, y, z, g, N, f);
    collide_node<L, T>(f, owner[idx], acc_tab, sp, flags, usol, idx, N);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) st<S, T>(fout + q * N + idx, f[q]);
}

// Macroscopic fields of the state held in fin (pull, then eq. 15a-b).
// solid_only: write u of solid nodes into usol ([d][N]) and nothing else;
// otherwise u node-major [N][d] and p [N] for every node.
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_fields(const typename S::raw *__restrict__ fin,
                                                 const uint16_t *__restrict__ owner, const T *__restrict__ acc_tab,
                                                 double *__restrict__ uout, double *__restrict__ pout, int solid_only,
                                                 Geom g, StepParams sp)
{
    const int N = (int)g.N;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const uint16_t own = owner[idx];
    const bool solid = own != FLUID;
    if (solid_only && !solid) return;
    int x, y, z;
    coords<L>(idx, g, x, y, z);
    T f[L::Q];
    pull<L, S, T>(fin, idx, x, y, z, g, N, f);
    T ax = 0, ay = 0, az = 0;
    if (solid) {
        ax = acc_tab[3 * own + 0];
        ay = acc_tab[3 * own + 1];
        az = acc_tab[3 * own + 2];
    } else if (sp.has_fluid_acc) {
        ax = (T)sp.fluid_acc[0];
        ay = (T)sp.fluid_acc[1];
        az = (T)sp.fluid_acc[2];
    }
    T ux, uy, uz, p;
    moments<L, T>(f, ax, ay, az, ux, uy, uz, p);
    if (solid_only) {
        uout[idx] = (double)ux;
        uout[N + idx] = (double)uy;
        if (L::D == 3) uout[2 * N + idx] = (double)uz;
        return;
    }
    uout[(size_t)idx * L::D + 0] = (double)ux;
    uout[(size_t)idx * L::D + 1] = (double)uy;
    if (L::D == 3) uout[(size_t)idx * L::D + 2] = (double)uz;
    pout[idx] = (double)p;
}

// Pulled populations f^n (FP64) of directions [q0, q0+nq) into out[q-q0][N].
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_populations(const typename S::raw *__restrict__ fin, double *__restrict__ out,
                                                      int q0, int nq, Geom g)
{
    const int N = (int)g.N;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    int x, y, z;
    coords<L>(idx, g, x, y, z);
    T f[L::Q];
    pull<L, S, T>(fin, idx, x, y, z, g, N, f);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        if (q >= q0 && q < q0 + nq) out[(size_t)(q - q0) * N + idx] = (double)f[q];
}

// Inverse of the pull: store f~ so that the next pull yields fn.  For node
// x and direction q: f~_q(x) = fn_q(x + c_q) if x + c_q is a node (wrapped),
// else f~_q(x) = fn_opp(q)(x) (the population bounced back into x).
// fn holds directions q and opp(q) at fn[0][N] and fn[1][N].
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_set_populations(const double *__restrict__ fn, typename S::raw *__restrict__ fout,
                                                          int q, Geom g)
{
    const int N = (int)g.N;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    int x, y, z;
    coords<L>(idx, g, x, y, z);
    int cq[3] = {L::cx[q], L::cy[q], L::cz[q]};
    int d[3] = {x + cq[0], y + cq[1], z + cq[2]};
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    bool out = false;
    for (int k = 0; k < L::D; ++k) {
        if (d[k] < 0 || d[k] >= n[k]) {
            if (per[k]) d[k] = (d[k] + n[k]) % n[k];
            else out = true;
        }
    }
    double v = out ? fn[(size_t)N + idx] : fn[d[0] + g.nx * (d[1] + g.ny * d[2])];
    st<S, T>(fout + (size_t)q * N + idx, (T)v);
}

// Uniform initial state f^n = feq everywhere, stored as f~ of the previous step.
struct FeqTab {
    double v[19];
};
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_init_uniform(typename S::raw *__restrict__ fout, FeqTab fe, Geom g)
{
    const int N = (int)g.N;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    int x, y, z;
    coords<L>(idx, g, x, y, z);
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    const int xs[3] = {x, y, z};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int cq[3] = {L::cx[q], L::cy[q], L::cz[q]};
        bool out = false;
        for (int k = 0; k < L::D; ++k) {
            int t = xs[k] + cq[k];
            if ((t < 0 || t >= n[k]) && !per[k]) out = true;
        }
        st<S, T>(fout + (size_t)q * N + idx, (T)(out ? fe.v[L::opp[q]] : fe.v[q]));
    }
}

// ------------------------------------------------------------------ dispatch

template <class F>
static hipError_t dispatch(lbm_ctx *c, F &&fn)
{
    if (c->cfg.lattice == LBM_D2Q9) {
        switch (c->cfg.storage) {
        case LBM_F64: return fn(D2Q9{}, StF64{}, double{});
        case LBM_F32: return fn(D2Q9{}, StF32{}, float{});
        case LBM_F16: return fn(D2Q9{}, StF16{}, float{});
        default: return fn(D2Q9{}, StBF16{}, float{});
        }
    }
    switch (c->cfg.storage) {
    case LBM_F64: return fn(D3Q19{}, StF64{}, double{});
    case LBM_F32: return fn(D3Q19{}, StF32{}, float{});
    case LBM_F16: return fn(D3Q19{}, StF16{}, float{});
    default: return fn(D3Q19{}, StBF16{}, float{});
    }
}

static inline unsigned blocks_for(int64_t N) { return (unsigned)((N + 255) / 256); }

hipError_t launch_stream_collide(lbm_ctx *c, const void *fin, void *fout)
{
    const int gx = (c->geo.nx + 255) / 256;
    const unsigned blocks = (unsigned)gx * (unsigned)(c->geo.ny * c->geo.nz);
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        const Tt *acc = std::is_same<Tt, double>::value ? (const Tt *)c->P.acc_d : (const Tt *)c->P.acc_f;
        hipLaunchKernelGGL((k_stream_collide<Lt, St, Tt>), dim3(blocks), dim3(256), 0, c->stream,
                           (const typename St::raw *)fin, (typename St::raw *)fout, c->owner, acc, c->usol, c->flags,
                           c->geo, c->sp, gx);
        return hipGetLastError();
    });
}

hipError_t launch_fields(lbm_ctx *c, const void *fin, double *u_out, double *p_out, int solid_only)
{
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        const Tt *acc = std::is_same<Tt, double>::value ? (const Tt *)c->P.acc_d : (const Tt *)c->P.acc_f;
        hipLaunchKernelGGL((k_fields<Lt, St, Tt>), dim3(blocks_for(c->geo.N)), dim3(256), 0, c->stream,
                           (const typename St::raw *)fin, c->owner, acc, u_out, p_out, solid_only, c->geo, c->sp);
        return hipGetLastError();
    });
}

hipError_t launch_populations(lbm_ctx *c, const void *fin, double *out, int q0, int nq)
{
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        hipLaunchKernelGGL((k_populations<Lt, St, Tt>), dim3(blocks_for(c->geo.N)), dim3(256), 0, c->stream,
                           (const typename St::raw *)fin, out, q0, nq, c->geo);
        return hipGetLastError();
    });
}

hipError_t launch_set_populations(lbm_ctx *c, const double *fn, void *fout, int q, int)
{
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        hipLaunchKernelGGL((k_set_populations<Lt, St, Tt>), dim3(blocks_for(c->geo.N)), dim3(256), 0, c->stream, fn,
                           (typename St::raw *)fout, q, c->geo);
        return hipGetLastError();
    });
}

hipError_t launch_init_uniform(lbm_ctx *c, void *fout, const double *feq)
{
    FeqTab t;
    for (int q = 0; q < 19; ++q) t.v[q] = q < c->Q ? feq[q] : 0.0;
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        hipLaunchKernelGGL((k_init_uniform<Lt, St, Tt>), dim3(blocks_for(c->geo.N)), dim3(256), 0, c->stream,
                           (typename St::raw *)fout, t, c->geo);
        return hipGetLastError();
    });
}

} // namespace lbm
