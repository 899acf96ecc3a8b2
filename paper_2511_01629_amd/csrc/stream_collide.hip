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
// wavefront with no solid node never executes it.  Solid nodes also hand
// their velocity to the per-particle momentum sums: as per-slot wavefront
// sums (slot_sums), or, where the step has no slots, as an FP64 field.
#include "dispatch.h"
#include "node.h"
#include "reduce.h"

namespace lbm {

// The lattice update, one node per lane.  Each workgroup covers BS
// consecutive nodes of one row (fixed y, z), so the row and the wall tests of
// y and z are uniform and no index division is needed.  Every population is
// read once (pull) and written once: 2 Q s bytes per node.  BS = 256, or 512
// for D2Q9 in FP64 (512 and 1024 were slower in FP32 and FP16, and capping
// their occupancy below the register limit was slower too).
//
// Measured alternatives that did not pay on MI355X: two adjacent nodes per
// lane (element-aligned 2-wide loads, or aligned loads with a DPP lane shift
// for the x-shifted directions), two strided nodes per lane, and an XCD-aware
// remap of the workgroup order.
//
// With slots (the fused-sums step), the solid nodes also add their momentum
// sums to their particle's slots (keyed wavefront sums, no table lookups) and,
// on in-place steps, reset their owner entry, which no other lane reads.
//
// I: the type of the population offsets q N + node -- int, or int64_t on a
// lattice with Q N >= 2^31 (node indices and the d N velocity field stay
// 32-bit; the same arithmetic, so the same bits, either way).
template <class L, class S, class T, int BS, class I = int>
__global__ __launch_bounds__(BS) void k_stream_collide(const typename S::raw *__restrict__ fin,
                                                         typename S::raw *__restrict__ fout, const uint16_t *owner,
                                                         const T *__restrict__ acc_tab, double *__restrict__ usol,
                                                         int32_t *__restrict__ flags, Geom g, StepParams sp, int gx,
                                                         unsigned gxm, SlotParams sl)
{
    // the row: by the host's reciprocal in 2-byte storage (fewer scalar
    // instructions, which those kernels are short of), by the compiler's
    // division otherwise (measured 1 % faster in FP32)
    const int row = sizeof(typename S::raw) == 2 ? div_magic((int)blockIdx.x, gx, gxm) : (int)blockIdx.x / gx;
    const int bx = (int)blockIdx.x - row * gx; // uniform
    const int x = bx * BS + (int)threadIdx.x;
    const bool valid = x < g.nx;
    int y, z;
    if (L::D == 2) {
        y = row;
        z = 0;
    } else {
        z = row / g.ny;
        y = row - z * g.ny;
    }
    const I N = (I)g.N;
    const int idx = row * g.nx + x;
    uint16_t own = FLUID;
    T ux = 0, uy = 0, uz = 0;
    // the node update.  Rows next to a moving wall take a copy of their own
    // (uniform branch), so that the others carry no wall code: fewer
    // registers in D3Q19 (70 against 90 with the wall term inline), FP32
    // 1 % faster.  The 2D 2-byte kernels, short of instructions, keep the
    // wall term inline: the second copy measured 5-7 % slower there.
    constexpr bool split = !(L::D == 2 && sizeof(typename S::raw) == 2);
    auto update = [&](auto at_wall) {
        T f[L::Q];
        if constexpr (sizeof(typename S::raw) == 2) {
            // 2-byte storage: the row-uniform offsets (the instruction count
            // limits these kernels; measured 4 % faster in FP16, 8 % in BF16)
            own = owner[idx];
            const RowPull<L, I> rp(x, y, z, idx, bx > 0 && bx * BS + BS < g.nx, g);
            pull_row<L, S, T, I>(fin, rp, f);
        } else {
            // 4- and 8-byte storage, bound by HBM: the per-lane offsets measured
            // 3 % (FP32) and 2 % (FP64) faster than the row-uniform ones
            pull<L, S, T, I>(fin, idx, x, y, z, g, N, f);
            own = owner[idx];
        }
        if constexpr (decltype(at_wall)::value || !split) wall_motion<L, T>(f, y, z, g, sp);
        collide_node<L, T>(f, own, acc_tab, sp, flags, usol, idx, (int)N, ux, uy, uz);
        // uniform_at forms a 32-bit byte offset (idx * element size), which
        // the 64-bit-offset lattices (up to 2^30 nodes) can exceed
        if constexpr (std::is_same<I, int>::value) {
#pragma unroll
            for (int q = 0; q < L::Q; ++q) st<S, T>(uniform_at(fout + q * N, idx), f[q]);
        } else {
#pragma unroll
            for (int q = 0; q < L::Q; ++q) st<S, T>(fout + ((I)q * N + idx), f[q]);
        }
    };
    if (valid) {
        if (split && wall_row(y, z, g, sp)) update(std::true_type{}); // uniform
        else update(std::false_type{});
    }
    if (sl.slots) { // uniform
        const bool solid = valid && own != FLUID;
        slot_sums<L::D>(solid, own, x, y, z, (double)ux, (double)uy, (double)uz, sl);
        if (solid && sl.clear) sl.clear[idx] = FLUID;
    }
}

// The 2D update with NS adjacent segments of one row per workgroup, every
// lane issuing the loads of all its NS nodes before it converts any: on a
// lattice whose single-segment grid is at most two rounds of workgroups (the
// cache-resident differentiated workload: 9.25 -> 8.33 us per step on
// 512x1024 in FP32), fewer, longer workgroups finish sooner; on the 2048x4096
// lattice the same kernel is 10 % slower (FP32) and stays unused there.
// Node arithmetic as in k_stream_collide, so the results are the same bits.
template <class L, class S, class T, int BS, int NS>
__global__ __launch_bounds__(BS) void k_stream_collide_multi(const typename S::raw *__restrict__ fin,
                                                           typename S::raw *__restrict__ fout, const uint16_t *owner,
                                                           const T *__restrict__ acc_tab, double *__restrict__ usol,
                                                           int32_t *__restrict__ flags, Geom g, StepParams sp, int gxw,
                                                           unsigned gxm, SlotParams sl)
{
    static_assert(L::D == 2, "2D rows");
    const int row = div_magic((int)blockIdx.x, gxw, gxm);
    const int bw = (int)blockIdx.x - row * gxw; // uniform
    const int y = row, z = 0;
    const int N = (int)g.N;
    using R = decltype(ld_reg<S>(fin));
    R r[NS][L::Q];
    uint16_t own[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int seg = bw * NS + k;
        const int x = seg * BS + (int)threadIdx.x;
        const int idx = row * g.nx + x;
        own[k] = FLUID;
        if (x < g.nx) {
            const RowPull<L> rp(x, y, z, idx, seg > 0 && seg * BS + BS < g.nx, g);
            if (rp.interior) { // uniform
#pragma unroll
                for (int q = 0; q < L::Q; ++q) {
                    const typename S::raw *src = fin + (q * rp.N + rp.rb[L::cy[q] + 1][L::cz[q] + 1] - L::cx[q]);
                    r[k][q] = ld_reg<S>(src + (unsigned)rp.x);
                }
            } else {
#pragma unroll
                for (int q = 0; q < L::Q; ++q) r[k][q] = ld_reg<S>(fin + rp.offset(q));
            }
            own[k] = owner[idx];
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int x = (bw * NS + k) * BS + (int)threadIdx.x;
        const int idx = row * g.nx + x;
        const bool valid = x < g.nx;
        T ux = 0, uy = 0, uz = 0;
        if (valid) {
            T f[L::Q];
#pragma unroll
            for (int q = 0; q < L::Q; ++q) f[q] = from_reg<S, T>(r[k][q]);
            wall_motion<L, T>(f, y, z, g, sp);
            collide_node<L, T>(f, own[k], acc_tab, sp, flags, usol, idx, N, ux, uy, uz);
#pragma unroll
            for (int q = 0; q < L::Q; ++q) st<S, T>(fout + q * N + idx, f[q]);
        }
        if (sl.slots) { // uniform
            const bool solid = valid && own[k] != FLUID;
            slot_sums<L::D>(solid, own[k], x, y, z, (double)ux, (double)uy, (double)uz, sl);
            if (solid && sl.clear) sl.clear[idx] = FLUID;
        }
    }
}

// D3Q19 variant with the source rows staged through LDS, so that every
// global access is a wide aligned vector.  A workgroup of TPB threads owns a
// segment of W = NPL * TPB nodes of one row, NPL = 16 / element size (8 for
// FP16/BF16, 4 FP32, 2 FP64):
//  1. for each population q, lane l loads the 16 bytes at x0 + NPL l of q's
//     source row (row y - c_y, z - c_z, wrapped on periodic axes; behind a
//     y/z wall, the node's own row of the opposite population: halfway
//     bounce-back), plus one halo element outside the segment for the
//     x-shifted populations (x0 - 1 or x0 + W; wrapped, or behind an x wall
//     the bounce-back value of the edge node); all into LDS, with the owner
//     map of the segment;
//  2. lane l collides nodes l, l + TPB, ... (consecutive lanes read
//     consecutive LDS elements) and keeps the results in registers;
//  3. the results go back through LDS and out as 16-byte vectors.
// The arithmetic per node is that of k_stream_collide.  Measured on MI355X it
// beats one node per lane only for D3Q19 in FP32 (6 % on a 256x256x512
// lattice); it is slower for D3Q19 in FP16 (22 %) and FP64 (1.5 %), and for
// D2Q9 in every storage type (10-20 %), where the load / collide / store
// phases of the few resident workgroups overlap less well than a
// one-node-per-lane stream.  Needs nx % NPL == 0 (aligned rows and planes).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class L, class S, class T, int TPB>
__global__ __launch_bounds__(TPB) void k_stream_collide_lds(const typename S::raw *__restrict__ fin,
                                                             typename S::raw *__restrict__ fout,
                                                             const uint16_t *owner, const T *__restrict__ acc_tab,
                                                             double *__restrict__ usol, int32_t *__restrict__ flags,
                                                             Geom g, StepParams sp, int gx, unsigned gxm,
                                                             SlotParams sl)
{
    using raw = typename S::raw;
    constexpr int Q = L::Q, NPL = 16 / (int)sizeof(raw), W = NPL * TPB;
    constexpr int RL = W + NPL; // LDS row: W elements, the two halo slots, padded to 16 bytes
    __shared__ __attribute__((aligned(16))) raw buf[Q * RL];
    __shared__ __attribute__((aligned(16))) uint16_t own_s[W];
    const int row = div_magic((int)blockIdx.x, gx, gxm), seg = (int)blockIdx.x - row * gx; // uniform
    const int x0 = seg * W, Wv = min(W, g.nx - x0);              // Wv: a multiple of NPL
    int y, z;
    if (L::D == 2) {
        y = row;
        z = 0;
    } else {
        z = row / g.ny;
        y = row - z * g.ny;
    }
    const int N = (int)g.N, tid = threadIdx.x, xl = tid * NPL, rbase = row * g.nx;
    const bool mine = xl < Wv;

    // 1. stage: all global loads first, then the LDS writes
    int sh[Q]; // x shift of population q's source (0 behind a y/z wall)
    u32x4 v[Q];
    const raw *hsrc = fin;
    int hslot = -1; // lanes 0 .. Q-1: the halo element of population q = lane
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int sy = y - L::cy[q], sz = z - L::cz[q], sq = q;
        bool wall = false;
        if (L::cy[q] != 0 && (sy < 0 || sy >= g.ny)) {
            if (g.per_y) sy = wrap(sy, g.ny);
            else wall = true;
        }
        if (L::cz[q] != 0 && (sz < 0 || sz >= g.nz)) {
            if (g.per_z) sz = wrap(sz, g.nz);
            else wall = true;
        }
        sh[q] = L::cx[q];
        if (wall) {
            sq = L::opp[q];
            sy = y;
            sz = z;
            sh[q] = 0;
        }
        const raw *src = fin + (size_t)sq * N + (sy + g.ny * sz) * g.nx;
        if (mine) v[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src + x0 + xl));
        if (sh[q] != 0 && tid == q) {
            const int xs = sh[q] > 0 ? x0 - 1 : x0 + Wv;
            if (xs >= 0 && xs < g.nx) hsrc = src + xs;
            else if (g.per_x) hsrc = src + wrap(xs, g.nx);
            else hsrc = fin + (size_t)L::opp[q] * N + rbase + (sh[q] > 0 ? x0 : x0 + Wv - 1); // x wall
            hslot = q * RL + (sh[q] > 0 ? W : W + 1);
        }
    }
    uint32_t ow[NPL / 2];
    if (mine) {
        const uint16_t *op = owner + rbase + x0 + xl;
        if constexpr (NPL == 8) {
            const u32x4 t = *reinterpret_cast<const u32x4 *>(op);
            for (int k = 0; k < 4; ++k) ow[k] = t[k];
        } else if constexpr (NPL == 4) {
            ow[0] = reinterpret_cast<const uint32_t *>(op)[0];
            ow[1] = reinterpret_cast<const uint32_t *>(op)[1];
        } else {
            ow[0] = *reinterpret_cast<const uint32_t *>(op);
        }
    }
    const raw hval = hslot >= 0 ? *hsrc : raw(0);
    if (mine) {
#pragma unroll
        for (int q = 0; q < Q; ++q) *reinterpret_cast<u32x4 *>(buf + q * RL + xl) = v[q];
#pragma unroll
        for (int k = 0; k < NPL / 2; ++k) reinterpret_cast<uint32_t *>(own_s + xl)[k] = ow[k];
    }
    if (hslot >= 0) buf[hslot] = hval;
    __syncthreads();

    // 2. collide nodes tid, tid + TPB, ...
    raw res[NPL][Q];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = tid + k * TPB;
        const bool valid = i < Wv; // consecutive lanes hold consecutive nodes
        uint16_t own = FLUID;
        T ux = 0, uy = 0, uz = 0;
        if (valid) {
            T f[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                int j = i - sh[q];
                j = j < 0 ? W : (j >= Wv ? W + 1 : j);
                f[q] = from_raw<S, T>(buf[q * RL + j]);
            }
            wall_motion<L, T>(f, y, z, g, sp);
            own = own_s[i];
            collide_node<L, T>(f, own, acc_tab, sp, flags, usol, rbase + x0 + i, N, ux, uy, uz);
#pragma unroll
            for (int q = 0; q < Q; ++q) res[k][q] = to_raw<S, T>(f[q]);
        }
        if (sl.slots) { // uniform
            const bool solid = valid && own != FLUID;
            slot_sums<L::D>(solid, own, x0 + i, y, z, (double)ux, (double)uy, (double)uz, sl);
            if (solid && sl.clear) sl.clear[rbase + x0 + i] = FLUID;
        }
    }
    __syncthreads();

    // 3. results back through LDS, out as 16-byte vectors
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = tid + k * TPB;
        if (i >= Wv) continue;
#pragma unroll
        for (int q = 0; q < Q; ++q) buf[q * RL + i] = res[k][q];
    }
    __syncthreads();
    if (mine) {
        const int idx = rbase + x0 + xl;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            __builtin_nontemporal_store(*reinterpret_cast<const u32x4 *>(buf + q * RL + xl),
                                        reinterpret_cast<u32x4 *>(fout + (size_t)q * N + idx));
    }
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
    pull<L, S, T, int64_t>(fin, idx, x, y, z, g, g.N, f); // 64-bit offsets: any lattice size
    wall_motion<L, T>(f, y, z, g, sp);
    T ax = 0, ay = 0, az = 0;
    if (solid) {
        ax = acc_tab[3 * own + 0];
        ay = acc_tab[3 * own + 1];
        az = acc_tab[3 * own + 2];
        if (sp.frac) { // as in collide_node
            const T chi = (T)frac_chi(idx, own, sp);
            ax = chi * ax;
            ay = chi * ay;
            az = chi * az;
        }
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
                                                      int q0, int nq, Geom g, StepParams sp)
{
    const int N = (int)g.N;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    int x, y, z;
    coords<L>(idx, g, x, y, z);
    T f[L::Q];
    pull<L, S, T, int64_t>(fin, idx, x, y, z, g, g.N, f); // 64-bit offsets: any lattice size
    wall_motion<L, T>(f, y, z, g, sp);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        if (q >= q0 && q < q0 + nq) out[(size_t)(q - q0) * N + idx] = (double)f[q];
}

// Inverse of the pull: store f~ so that the next pull yields fn.  For node
// x and direction q: f~_q(x) = fn_q(x + c_q) if x + c_q is a node (wrapped),
// else f~_q(x) = fn_opp(q)(x) (the population bounced back into x), less
// what a moving wall adds to it.
// fn holds directions q and opp(q) at fn[0][N] and fn[1][N].
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_set_populations(const double *__restrict__ fn, typename S::raw *__restrict__ fout,
                                                          int q, Geom g, StepParams sp)
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
    if (out && sp.wall_axis) { // every other axis is periodic: x + c_q lies behind the moving wall
        const int s = sp.wall_axis == 1 ? y + cq[1] : z + cq[2]; // below 0: the low wall; else the high one
        v -= wall_term<L>(L::opp[q], s < 0 ? 0 : 1, sp);
    }
    st<S, T>(fout + (size_t)q * N + idx, (T)v);
}

// Uniform initial state f^n = feq everywhere, stored as f~ of the previous step.
struct FeqTab {
    double v[19];
};
template <class L, class S, class T>
__global__ __launch_bounds__(256) void k_init_uniform(typename S::raw *__restrict__ fout, FeqTab fe, Geom g,
                                                       StepParams sp)
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
        double v = out ? fe.v[L::opp[q]] : fe.v[q];
        if (out && sp.wall_axis) { // less what the moving wall adds to the bounced population
            const int s = xs[sp.wall_axis] + cq[sp.wall_axis];
            v -= wall_term<L>(L::opp[q], s < 0 ? 0 : 1, sp);
        }
        st<S, T>(fout + (size_t)q * N + idx, (T)v);
    }
}

static inline unsigned blocks_for(int64_t N) { return (unsigned)((N + 255) / 256); }

// Rigid-velocity forcing (an extension beyond the paper, lbm_config.rigid_beta
// > 0): after the momentum sums of the step gave U_i^n and omega_i^n, the
// nodes of each particle are collided again with the acceleration
// a_g + 2 beta (U_i + omega_i x r - u), where u is the node's velocity with
// the gravity acceleration a_g alone (eq. 15a) and r = x - X_i^n (nearest
// image): eq. (15a) adds half the acceleration, so the velocity that enters
// the equilibrium and the Guo force is (1 - beta) u + beta (U_i + omega_i x r).
// One workgroup per particle walks its scan box; a node it owns is pulled
// again from the step's input buffer (which the step leaves unchanged),
// collided, written over the lattice kernel's unforced result, and its
// indicator entry reset (the sums left the indicator in place for this pass).
template <class L, class S, class T, int BS>
__global__ __launch_bounds__(BS) void k_force(const typename S::raw *__restrict__ fin,
                                              typename S::raw *__restrict__ fout, uint16_t *owner,
                                              const T *__restrict__ acc_tab, PartDev P, int32_t *__restrict__ flags,
                                              Geom g, StepParams sp)
{
    const int i = blockIdx.x;
    const Box b = make_box(P.lo + 3 * i, P.hi + 3 * i);
    const double X0 = P.X[3 * i], X1 = P.X[3 * i + 1], X2 = L::D == 3 ? P.X[3 * i + 2] : 0.0;
    const double U0 = P.U[3 * i], U1 = P.U[3 * i + 1], U2 = P.U[3 * i + 2];
    const double W0 = P.W[3 * i], W1 = P.W[3 * i + 1], W2 = P.W[3 * i + 2];
    const T ag[3] = {acc_tab[3 * i], acc_tab[3 * i + 1], acc_tab[3 * i + 2]};
    const T beta2 = (T)(2.0 * sp.beta);
    const int N = (int)g.N;
    CellWalk w(b.ext[0] > 0 ? b.ext[0] : 1, b.ext[1] > 0 ? b.ext[1] : 1, threadIdx.x, BS);
    for (int cell = threadIdx.x; cell < b.cells; cell += BS) {
        int xu, yu, zu;
        const int idx = walk_node(b, w, g, xu, yu, zu);
        w.next();
        if (owner[idx] != (uint16_t)i) continue;
        const int x = wrap(xu, g.nx), y = wrap(yu, g.ny), z = wrap(zu, g.nz);
        T f[L::Q];
        pull<L, S, T, int64_t>(fin, idx, x, y, z, g, g.N, f); // 64-bit offsets: any lattice size
        wall_motion<L, T>(f, y, z, g, sp);
        T ux, uy, uz, p;
        moments<L, T>(f, ag[0], ag[1], ag[2], ux, uy, uz, p);
        const double rx = (double)xu - X0, ry = (double)yu - X1, rz = L::D == 3 ? (double)zu - X2 : 0.0;
        const double vx = U0 + (W1 * rz - W2 * ry), vy = U1 + (W2 * rx - W0 * rz), vz = U2 + (W0 * ry - W1 * rx);
        const T acc[3] = {ag[0] + beta2 * ((T)vx - ux), ag[1] + beta2 * ((T)vy - uy),
                          L::D == 3 ? ag[2] + beta2 * ((T)vz - uz) : T(0)};
        collide_node<L, T>(f, 0, acc, sp, flags, nullptr, idx, N, ux, uy, uz);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) st<S, T>(fout + (size_t)q * N + idx, f[q]);
        owner[idx] = FLUID;
    }
}

hipError_t launch_stream_collide(lbm_ctx *c, const void *fin, void *fout)
{
    const SlotParams sl = slot_params(c, c->fused != 0);
    double *usol = sl.slots ? nullptr : c->usol; // the slots replace the velocity field of the sums
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        const Tt *acc = std::is_same<Tt, double>::value ? (const Tt *)c->P.acc_d : (const Tt *)c->P.acc_f;
        if constexpr (Lt::Q == 19 && std::is_same<St, StF32>::value) {
            // staged rows (D3Q19 in FP32, where it measured faster): the largest
            // workgroup (up to 128 threads, for the LDS of 19 populations) whose
            // segment still fits in a row
            constexpr int NPL = 16 / (int)sizeof(typename St::raw);
            if (c->geo.nx % NPL == 0) {
                auto staged = [&](auto tpb) {
                    constexpr int TPB = decltype(tpb)::value, W = NPL * TPB;
                    const int gxs = (c->geo.nx + W - 1) / W;
                    const unsigned bs = (unsigned)gxs * (unsigned)(c->geo.ny * c->geo.nz);
                    return launch(c, k_stream_collide_lds<Lt, St, Tt, TPB>, dim3(bs), dim3(TPB),
                                  (const typename St::raw *)fin, (typename St::raw *)fout, (const uint16_t *)c->owner,
                                  acc, usol, c->flags, c->geo, c->sp, gxs, magic_for(gxs), sl);
                };
                if (c->geo.nx >= 128 * NPL) return staged(std::integral_constant<int, 128>{});
                return staged(std::integral_constant<int, 64>{});
            }
        }
        if constexpr (Lt::D == 2 && sizeof(typename St::raw) <= 4) {
            auto multi = [&](auto ns) {
                constexpr int NS = decltype(ns)::value;
                const int gxw = (c->geo.nx + 256 * NS - 1) / (256 * NS);
                return launch(c, k_stream_collide_multi<Lt, St, Tt, 256, NS>, dim3((unsigned)(gxw * c->geo.ny)),
                              dim3(256), (const typename St::raw *)fin, (typename St::raw *)fout,
                              (const uint16_t *)c->owner, acc, usol, c->flags, c->geo, c->sp, gxw, magic_for(gxw), sl);
            };
            const int64_t blocks1 = (int64_t)((c->geo.nx + 255) / 256) * c->geo.ny;
            if (blocks1 <= 4096 && !c->wide) return multi(std::integral_constant<int, 2>{});
        }
        constexpr bool d2f64 = Lt::D == 2 && sizeof(Tt) == 8;
        constexpr int BS = d2f64 ? 512 : 256;
        // D2Q9 in FP64: at most two 512-thread workgroups per compute unit (an
        // unused LDS reservation of 56 KiB of the 160), 16 waves: measured
        // faster than the 24 its register use would allow
        constexpr size_t shm = d2f64 ? (size_t)56 << 10 : 0;
        const int gx = (c->geo.nx + BS - 1) / BS;
        const unsigned blocks = (unsigned)gx * (unsigned)(c->geo.ny * c->geo.nz);
        if (c->wide) // Q N >= 2^31: 64-bit population offsets
            return launch_shm(c, k_stream_collide<Lt, St, Tt, BS, int64_t>, dim3(blocks), dim3(BS), shm,
                              (const typename St::raw *)fin, (typename St::raw *)fout, (const uint16_t *)c->owner,
                              acc, usol, c->flags, c->geo, c->sp, gx, magic_for(gx), sl);
        return launch_shm(c, k_stream_collide<Lt, St, Tt, BS>, dim3(blocks), dim3(BS), shm,
                          (const typename St::raw *)fin, (typename St::raw *)fout, (const uint16_t *)c->owner, acc,
                          usol, c->flags, c->geo, c->sp, gx, magic_for(gx), sl);
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
                           (const typename St::raw *)fin, out, q0, nq, c->geo, c->sp);
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
                           (typename St::raw *)fout, q, c->geo, c->sp);
        return hipGetLastError();
    });
}

hipError_t launch_force(lbm_ctx *c, const void *fin, void *fout)
{
    if (c->np == 0) return hipSuccess;
    return dispatch(c, [&](auto L, auto S, auto T) {
        using Lt = decltype(L);
        using St = decltype(S);
        using Tt = decltype(T);
        const Tt *acc = std::is_same<Tt, double>::value ? (const Tt *)c->P.acc_d : (const Tt *)c->P.acc_f;
        return launch(c, k_force<Lt, St, Tt, 256>, dim3(c->np), dim3(256), (const typename St::raw *)fin,
                      (typename St::raw *)fout, c->owner, acc, c->P, c->flags, c->geo, c->sp);
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
                           (typename St::raw *)fout, t, c->geo, c->sp);
        return hipGetLastError();
    });
}

} // namespace lbm
