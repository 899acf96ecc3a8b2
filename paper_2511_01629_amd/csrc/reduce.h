// reduce.h -- building blocks of the per-particle kernels: fixed-order
// wavefront and workgroup sums, scan-box iteration.  Private to the library.
//
// The per-particle kernels are bound by memory latency, not bandwidth (a few
// hundred to a few thousand nodes per particle), so each lane issues the
// loads of up to UNR cells before it uses any of them, and partial sums are
// combined with a butterfly over the 64 lanes of a wavefront (every lane ends
// with the same bits) and then across wavefronts through LDS in wave order.
// Nothing depends on timing, so results are bitwise reproducible.
#pragma once
#include "ctx.h"

namespace lbm {

constexpr int WAVE = 64;
constexpr int UNR = 8; // cells whose loads a lane keeps in flight together

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Sum NS values over a workgroup of BS threads; the totals land in thread 0.
// lds must hold BS/64 x NS doubles.  Contains __syncthreads().
template <int NS, int BS>
__device__ __forceinline__ void block_sum(double *s, double (*lds)[NS])
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = wave_sum(s[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NS; ++k) lds[w][k] = s[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            double t = lds[0][k];
            for (int q = 1; q < BS / WAVE; ++q) t += lds[q][k];
            s[k] = t;
        }
}

// A particle's scan box in unwrapped node coordinates.
struct Box {
    int lo[3], ext[3];
    int cells;
};

__device__ __forceinline__ Box make_box(const int *lo, const int *hi)
{
    Box b;
    b.cells = 1;
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = lo[k];
        b.ext[k] = hi[k] - lo[k] + 1 > 0 ? hi[k] - lo[k] + 1 : 0;
        b.cells *= b.ext[k];
    }
    return b;
}

// Scan box of a particle of bounding radius R centred at Xc: two nodes of
// margin, clipped on wall axes; empty (hi < lo) for a non-finite or runaway
// centre.  Unused axes are [0, 0].
__device__ __forceinline__ void centre_box(const double *Xc, double R, const Geom &g, int d, int *lo, int *hi)
{
    const int n[3] = {g.nx, g.ny, g.nz};
    const int per[3] = {g.per_x, g.per_y, g.per_z};
    for (int k = 0; k < 3; ++k) {
        int l = 0, h = -1;
        if (k >= d) {
            l = h = 0;
        } else if (fabs(Xc[k]) < 1e9) {
            l = (int)floor(Xc[k] - R) - 2;
            h = (int)ceil(Xc[k] + R) + 2;
            if (!per[k]) {
                l = l < 0 ? 0 : l;
                h = h > n[k] - 1 ? n[k] - 1 : h;
            }
        }
        lo[k] = l;
        hi[k] = h;
    }
}

// Walks the cells start, start + nl, start + 2 nl, ... of a box of extents
// e0 x e1 x e2 (in x-fastest order) without a division in the loop: the start
// and the stride are decomposed once, then each step adds with carries
// (integer division costs tens of instructions on the GPU, and the
// one-workgroup particle kernels are bound by the ALU work of one CU).
struct CellWalk {
    int lx, ly, lz; // current cell, box-local
    int sx, sy, sz; // the stride nl, decomposed
    int e0, e1;

    __device__ __forceinline__ CellWalk(int ext0, int ext1, int start, int nl) : e0(ext0), e1(ext1)
    {
        int r = start / e0;
        lx = start - r * e0;
        ly = r % e1;
        lz = r / e1;
        r = nl / e0;
        sx = nl - r * e0;
        sy = r % e1;
        sz = r / e1;
    }
    __device__ __forceinline__ void next()
    {
        lx += sx;
        int c = lx >= e0;
        lx -= c ? e0 : 0;
        ly += sy + c;
        c = ly >= e1;
        ly -= c ? e1 : 0;
        lz += sz + c;
    }
};

// Node index of the walker's cell in box b (unwrapped coordinates xu, yu, zu).
__device__ __forceinline__ int walk_node(const Box &b, const CellWalk &w, const Geom &g, int &xu, int &yu, int &zu)
{
    xu = b.lo[0] + w.lx;
    yu = b.lo[1] + w.ly;
    zu = b.lo[2] + w.lz;
    return wrap(xu, g.nx) + g.nx * (wrap(yu, g.ny) + g.ny * wrap(zu, g.nz));
}

// Keyed wavefront sums of the momentum moments of one step's solid nodes
// into the slots (the fused-sums step).  Called by every lane of the
// wavefront with uniform control flow; `active` lanes hold a solid node
// (x, y, z) of particle `own` with velocity u.  The key of a node is its
// particle and its slot: the row of the particle's scan box it lies in and
// the wavefront of the lattice row, counted from the box's first one, so
// every slot has exactly one writing wavefront.  Each distinct key in the
// wavefront is summed with the butterfly (fixed order) and written by its
// lowest lane, with the stamp of the step.  Moments as in the momentum sums:
// 2D [N, u_x, u_y, r x u, |r|^2], 3D [N, u (3), r x u (3), inertia xx yy zz xy xz yz].
template <int D>
__device__ void slot_sums(bool active, uint16_t own, int x, int y, int z, double ux, double uy, double uz,
                          const SlotParams &sp, const Geom &g)
{
    constexpr int NS = D == 2 ? 5 : 13;
    unsigned long long pending = __ballot(active);
    if (pending == 0ull) return;
    const int lane = threadIdx.x & (WAVE - 1);
    uint32_t key = 0xFFFFFFFFu;
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (active) {
        const int i = own;
        const int lo0 = sp.lo[3 * i], lo1 = sp.lo[3 * i + 1], lo2 = sp.lo[3 * i + 2];
        const int hi0 = sp.hi[3 * i], hi1 = sp.hi[3 * i + 1];
        int xu = x, yu = y, zu = z; // unwrapped into the box (it spans less than a period)
        if (g.per_x) xu = xu < lo0 ? xu + g.nx : (xu > hi0 ? xu - g.nx : xu);
        if (g.per_y) yu = yu < lo1 ? yu + g.ny : (yu > hi1 ? yu - g.ny : yu);
        if (D == 3 && g.per_z) {
            const int hi2 = sp.hi[3 * i + 2];
            zu = zu < lo2 ? zu + g.nz : (zu > hi2 ? zu - g.nz : zu);
        }
        const int row = (yu - lo1) + (hi1 - lo1 + 1) * (zu - lo2);
        const int j = ((x / WAVE) - (wrap(lo0, g.nx) / WAVE) + sp.wn) % sp.wn;
        if (row >= 0 && j < sp.kw && row * sp.kw + j < sp.stride) key = ((uint32_t)i << 16) | (uint32_t)(row * sp.kw + j);
        else sp.flags[1] = 1;
        rx = (double)xu - sp.X[3 * i];
        ry = (double)yu - sp.X[3 * i + 1];
        rz = D == 3 ? (double)zu - sp.X[3 * i + 2] : 0.0;
    }
    pending = __ballot(key != 0xFFFFFFFFu);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t k = (uint32_t)__shfl((int)key, leader);
        const bool mine = key == k;
        double v[NS];
        v[0] = mine ? 1.0 : 0.0;
        v[1] = mine ? ux : 0.0;
        v[2] = mine ? uy : 0.0;
        if constexpr (D == 2) {
            v[3] = mine ? rx * uy - ry * ux : 0.0;
            v[4] = mine ? rx * rx + ry * ry : 0.0;
        } else {
            const double rr = rx * rx + ry * ry + rz * rz;
            v[3] = mine ? uz : 0.0;
            v[4] = mine ? ry * uz - rz * uy : 0.0;
            v[5] = mine ? rz * ux - rx * uz : 0.0;
            v[6] = mine ? rx * uy - ry * ux : 0.0;
            v[7] = mine ? rr - rx * rx : 0.0;
            v[8] = mine ? rr - ry * ry : 0.0;
            v[9] = mine ? rr - rz * rz : 0.0;
            v[10] = mine ? -(rx * ry) : 0.0;
            v[11] = mine ? -(rx * rz) : 0.0;
            v[12] = mine ? -(ry * rz) : 0.0;
        }
#pragma unroll
        for (int m = 0; m < NS; ++m) v[m] = wave_sum(v[m]);
        if (lane == leader) {
            double *out = sp.slots + ((size_t)(k >> 16) * sp.stride + (k & 0xFFFFu)) * (NS + 1);
            out[0] = sp.stamp;
#pragma unroll
            for (int m = 0; m < NS; ++m) out[1 + m] = v[m];
        }
        pending &= ~__ballot(mine);
    }
}

// Cell c of box b: unwrapped coordinates and the (wrapped) node index.
__device__ __forceinline__ void cell_at(const Box &b, int c, const Geom &g, int &xu, int &yu, int &zu, int &node)
{
    const int lx = c % b.ext[0], r = c / b.ext[0];
    const int ly = r % b.ext[1], lz = r / b.ext[1];
    xu = b.lo[0] + lx;
    yu = b.lo[1] + ly;
    zu = b.lo[2] + lz;
    node = wrap(xu, g.nx) + g.nx * (wrap(yu, g.ny) + g.ny * wrap(zu, g.nz));
}

} // namespace lbm
