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

// Cross-row step of a wavefront sum, with the gfx950 lane swaps: given v in
// both operands, v_permlane16_swap exchanges the odd 16-lane rows of one with
// the even rows of the other (v_permlane32_swap: the upper half of one with
// the lower half of the other), so the two results hold the two members of
// every row pair (half pair), and their sum is the same, added in the same
// order, on every lane.
template <bool HALVES>
__device__ __forceinline__ double swap_add(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (HALVES) {
        const auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = L[0], l1 = L[1], h0 = H[0], h1 = H[1];
    } else {
        const auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = L[0], l1 = L[1], h0 = H[0], h1 = H[1];
    }
    return __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0)) +
           __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
}

// Sum over the 64 lanes of a wavefront, every lane getting the same bits,
// without an LDS round trip.  Within each row of 16 lanes the partner values
// move over the DPP network: lanes xor 1, xor 2 (quad permutes), then the
// half-row and row mirrors, each step adding a value computed the same way on
// both sides; then rows 0+1 and 2+3, then the two halves (swap_add).  Must be
// called with all 64 lanes active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x141, 0xF, 0xF, false); // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x140, 0xF, 0xF, false); // row_mirror
    return swap_add<true>(swap_add<false>(v));
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

// Slot of a solid node in its particle's table (the fused-sums step).  A
// slot is one wavefront of one lattice row: the row is keyed by its wrapped y
// (and z) modulo powers of two My, Mz, the wavefront by its index in the row
// modulo a power of two Mx.  The sizes are chosen at set-up so that the rows
// and wavefronts of any scan box map to distinct slots (each at least the
// box's extent in rows, or wavefronts it can touch, and on a periodic axis a
// divisor of the period or at least the period), so the key needs nothing
// but the node's coordinates.
__device__ __forceinline__ uint32_t slot_of(int x, int y, int z, const SlotParams &sl)
{
    return (uint32_t)(((z & sl.mz) << sl.sz) | ((y & sl.my) << sl.sy) | ((x >> 6) & sl.mx));
}

// Moments of the bit positions set in a wavefront mask: count, sum and sum
// of squares of the positions (bit-plane popcounts; exact integers).
__device__ __forceinline__ void mask_moments(unsigned long long m, double &n, double &s1, double &s2)
{
    const unsigned long long P[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                                     0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
    long long a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        a += (long long)__popcll(m & P[i]) << i;
        b += (long long)__popcll(m & P[i]) << (2 * i);
#pragma unroll
        for (int j = i + 1; j < 6; ++j) b += (long long)__popcll(m & P[i] & P[j]) << (i + j + 1);
    }
    n = (double)__popcll(m);
    s1 = (double)a;
    s2 = (double)b;
}

// Per-slot sums of one step's solid nodes (the fused-sums step), taken in
// the lattice kernel.  Called by every lane of the wavefront with uniform
// control flow; `active` lanes hold a solid node (x, y, z) of particle own
// with velocity u.  For each distinct (particle, slot) key among the lanes,
// its lowest lane writes the record [stamp, lane mask, first node, sums]: the
// mask gives the count and the lane offsets s = x mod 64 of the nodes, the
// first node is the wavefront's (x0 = x - s, y, z) packed into 64 bits, and
// the sums are 2D [u_x, u_y, s u_y], 3D [u_x, u_y, u_z, s u_y, s u_z], each a
// fixed-order wavefront sum.  The particle kernel shifts these to moments
// about the particle centre.
template <int D>
__device__ void slot_sums(bool active, uint16_t own, int x, int y, int z, double ux, double uy, double uz,
                          const SlotParams &sl)
{
    constexpr int NV = D == 2 ? 3 : 5;
    if (__ballot(active) == 0ull) return;
    const uint32_t key = active ? ((uint32_t)own << 16) | slot_of(x, y, z, sl) : 0xFFFFFFFFu;
    const double s = (double)(x & (WAVE - 1));
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const bool mine = key == k;
        const unsigned long long mask = __ballot(mine);
        double v[NV];
        v[0] = mine ? ux : 0.0;
        v[1] = mine ? uy : 0.0;
        if constexpr (D == 2) {
            v[2] = mine ? s * uy : 0.0;
        } else {
            v[2] = mine ? uz : 0.0;
            v[3] = mine ? s * uy : 0.0;
            v[4] = mine ? s * uz : 0.0;
        }
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = wave_sum(v[m]);
        if (lane == leader) {
            double *out = sl.slots + ((size_t)(k >> 16) * sl.stride + (k & 0xFFFFu)) * slot_width(D);
            const unsigned long long first =
                (unsigned long long)(x & ~(WAVE - 1)) | ((unsigned long long)y << 21) | ((unsigned long long)z << 42);
            out[0] = sl.stamp;
            out[1] = __longlong_as_double((long long)mask);
            out[2] = __longlong_as_double((long long)first);
#pragma unroll
            for (int m = 0; m < NV; ++m) out[3 + m] = v[m];
        }
        pending &= ~mask;
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
