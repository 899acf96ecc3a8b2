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
#include "dispatch.h"
#include "node.h"

namespace lbm {

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
        return launch(c, k_stream_collide<Lt, St, Tt>, dim3(blocks), dim3(256), (const typename St::raw *)fin,
                      (typename St::raw *)fout, (const uint16_t *)c->owner, acc, c->usol, c->flags, c->geo, c->sp, gx);
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
