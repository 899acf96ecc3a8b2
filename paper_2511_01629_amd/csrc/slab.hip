// slab.hip -- the step with the lattice split into slabs on one GPU: the
// layout a multi-GPU run would give each GPU, emulated with explicit copies.
//
// The lattice is cut along its last axis (y in 2D, z in 3D; gravity points
// along it in the sedimentation workloads) into S slabs of consecutive rows
// (planes).  Slab s keeps its populations in buffers of its own, [Q][rows_s +
// 2][plane], with one halo row (plane) below and above its rows.  Every step:
//   1. each slab runs the lattice update over its own rows (k_slab_collide:
//      the node arithmetic of k_stream_collide, the pull reading the halo
//      where a source row lies in the neighbouring slab, bounce-back where it
//      lies behind a wall);
//   2. the halos are exchanged: slab s's top row goes to slab s + 1's lower
//      halo and slab s + 1's bottom row to slab s's upper halo (and around
//      the period on a periodic axis), as Q row copies each way;
//   3. the momentum sums of the solid nodes, which every slab wrote to a slot
//      table of its own, are merged into one table (k_merge_slots: records
//      carry the step's stamp and the keys of different rows are distinct) --
//      the cross-slab particle sums; then Algorithm 1 and the new indicator
//      run once over the merged sums, as in the unsplit step.
// The indicator, the solid-node velocity and the particle state stay shared
// (one copy), which a multi-GPU run would replicate.  The results are those
// of the unsplit step bit for bit: every node pulls the same values and
// takes the same arithmetic, every slot record sums the same nodes.
#include <algorithm>
#include <string>

#include "dispatch.h"
#include "node.h"
#include "reduce.h"

using namespace lbm;

namespace lbm {

// One slab: rows [r0, r0 + rows) of the split axis.
struct SlabGeom {
    int r0, rows;     // first global row (y in 2D, z in 3D) and row count
    int plane;        // nodes per row: nx (2D) or nx ny (3D)
    int N;            // population stride of the slab buffer: (rows + 2) plane
    int wall_lo, wall_hi; // the row below / above the slab lies behind a wall
    int gx;           // workgroups per lattice row (of nx nodes)
};

template <class L, class S, class T, int BS>
__global__ __launch_bounds__(BS) void k_slab_collide(const typename S::raw *__restrict__ fin,
                                                     typename S::raw *__restrict__ fout, const uint16_t *owner,
                                                     const T *__restrict__ acc_tab, double *__restrict__ usol,
                                                     int32_t *__restrict__ flags, Geom g, StepParams sp, SlabGeom sg,
                                                     SlotParams sl)
{
    // workgroup -> (lattice row of the slab, segment of BS nodes)
    const int row = (int)blockIdx.x / sg.gx; // row of nx nodes within the slab's rows
    const int bx = (int)blockIdx.x - row * sg.gx;
    const int x = bx * BS + (int)threadIdx.x;
    const bool valid = x < g.nx;
    int y, z, lr; // global y, z; lr: local row (of the split axis) in the slab buffer, 1..rows
    if (L::D == 2) {
        lr = row + 1;
        y = sg.r0 + row;
        z = 0;
    } else {
        const int zl = row / g.ny;
        y = row - zl * g.ny;
        lr = zl + 1;
        z = sg.r0 + zl;
    }
    const int Ng = (int)g.N;
    const int gidx = x + g.nx * (y + g.ny * z);
    const int lidx = x + (L::D == 2 ? g.nx * lr : g.nx * (y + g.ny * lr));
    uint16_t own = FLUID;
    T ux = 0, uy = 0, uz = 0;
    if (valid) {
        T f[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            // source node x - c_q: x and the axis that is not split as on the
            // whole lattice; along the split axis the slab buffer holds the
            // source row (its own rows or a halo) unless it is behind a wall
            const int cs = L::D == 2 ? L::cy[q] : L::cz[q];
            bool wall = (cs > 0 && lr == 1 && sg.wall_lo) || (cs < 0 && lr == sg.rows && sg.wall_hi);
            int sx = x - L::cx[q];
            if (sx < 0) {
                if (g.per_x) sx += g.nx; else wall = true;
            } else if (sx >= g.nx) {
                if (g.per_x) sx -= g.nx; else wall = true;
            }
            int sy = y - L::cy[q];
            if (L::D == 3) {
                if (sy < 0) {
                    if (g.per_y) sy += g.ny; else wall = true;
                } else if (sy >= g.ny) {
                    if (g.per_y) sy -= g.ny; else wall = true;
                }
            }
            const int slr = lr - cs;
            const int src = L::D == 2 ? sx + g.nx * slr : sx + g.nx * (sy + g.ny * slr);
            f[q] = ld<S, T>(fin + (wall ? L::opp[q] * sg.N + lidx : q * sg.N + src));
        }
        own = owner[gidx];
        wall_motion<L, T>(f, y, z, g, sp);
        collide_node<L, T>(f, own, acc_tab, sp, flags, usol, gidx, Ng, ux, uy, uz);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) st<S, T>(fout + q * sg.N + lidx, f[q]);
    }
    if (sl.slots) { // uniform
        const bool solid = valid && own != FLUID;
        slot_sums<L::D>(solid, own, x, y, z, (double)ux, (double)uy, (double)uz, sl);
        if (solid && sl.clear) sl.clear[gidx] = FLUID;
    }
}

// Records of this step's stamp from a slab's slot table into the merged one.
__global__ __launch_bounds__(256) void k_merge_slots(double *__restrict__ dst, const double *__restrict__ src,
                                                     int64_t nrec, int width, double stamp)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec || src[r * width] != stamp) return;
    for (int m = 0; m < width; ++m) dst[r * width + m] = src[r * width + m];
}

} // namespace lbm

namespace {

#define SLABCHK(c, expr)                                                                                               \
    do {                                                                                                               \
        hipError_t e_ = (expr);                                                                                        \
        if (e_ != hipSuccess) {                                                                                        \
            (c)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                                              \
            return LBM_EDEVICE;                                                                                        \
        }                                                                                                              \
    } while (0)

size_t elt_bytes(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }

// Copy `count` consecutive rows of every population between two buffers of
// the given population strides (in elements): rows [src_row, src_row +
// count) of src to rows [dst_row, ...) of dst.
hipError_t copy_rows(lbm_ctx *c, void *dst, int dst_N, int dst_row, const void *src, int src_N, int src_row, int count,
                     int plane)
{
    const size_t e = elt_bytes(c->cfg.storage);
    return hipMemcpy2DAsync((char *)dst + (size_t)dst_row * plane * e, (size_t)dst_N * e,
                            (const char *)src + (size_t)src_row * plane * e, (size_t)src_N * e,
                            (size_t)count * plane * e, (size_t)c->Q, hipMemcpyDeviceToDevice, c->stream);
}

} // namespace

extern "C" int lbm_step_slabs(lbm_ctx *c, int64_t nsteps, int32_t nslabs)
{
    if (!c) return LBM_EINVAL;
    const int d = c->d;
    const int len = d == 2 ? c->geo.ny : c->geo.nz;          // the split axis
    const int per = d == 2 ? c->geo.per_y : c->geo.per_z;
    const int plane = d == 2 ? c->geo.nx : c->geo.nx * c->geo.ny;
    if (nsteps < 0 || nslabs < 1 || nslabs > 64 || nslabs > len)
        return c->err = "nsteps >= 0 and 1 <= nslabs <= min(64, rows of the split axis) required", LBM_EINVAL;
    if (c->sp.beta > 0) return c->err = "the rigid-velocity forcing runs on the unsplit lattice only", LBM_EINVAL;
    if (c->rp.K != 1) return c->err = "slabs are implemented for K = 1", LBM_EINVAL;
    // the slab kernel keeps 32-bit population offsets within a slab buffer
    const int64_t max_rows = len / nslabs + (len % nslabs ? 1 : 0);
    if ((int64_t)c->Q * (max_rows + 2) * plane >= ((int64_t)1 << 31))
        return c->err = "a slab's Q*(rows+2)*plane must stay below 2^31 (32-bit offsets): use more slabs", LBM_EINVAL;
    (void)hipSetDevice(c->device);
    const size_t e = elt_bytes(c->cfg.storage);
    // slabs: rows split as evenly as possible
    std::vector<SlabGeom> sg(nslabs);
    size_t fbytes = 0;
    for (int s = 0, r0 = 0; s < nslabs; ++s) {
        const int rows = len / nslabs + (s < len % nslabs ? 1 : 0);
        sg[s].r0 = r0;
        sg[s].rows = rows;
        sg[s].plane = plane;
        sg[s].N = (rows + 2) * plane;
        sg[s].wall_lo = s == 0 && !per;
        sg[s].wall_hi = s == nslabs - 1 && !per;
        sg[s].gx = (c->geo.nx + 255) / 256;
        r0 += rows;
        fbytes += 2 * (size_t)c->Q * sg[s].N * e;
    }
    const bool fused = c->fused && c->slots && c->np > 0;
    const size_t tbytes = fused ? c->slots_bytes : 0;
    const size_t need = fbytes + (size_t)(nslabs - 1) * tbytes + 256 * (size_t)(2 * nslabs + nslabs);
    if (need > c->slab_bytes) {
        if (c->slab_mem) SLABCHK(c, hipFree(c->slab_mem));
        c->slab_mem = nullptr;
        c->slab_bytes = 0;
        SLABCHK(c, hipMalloc(&c->slab_mem, need));
        c->slab_bytes = need;
    }
    // carve: per slab two population buffers, then the extra slot tables
    std::vector<void *> buf(2 * nslabs);
    std::vector<double *> table(nslabs, nullptr);
    char *p = (char *)c->slab_mem;
    auto take = [&](size_t n) {
        char *q = p;
        p += (n + 255) / 256 * 256;
        return q;
    };
    for (int s = 0; s < nslabs; ++s) {
        buf[2 * s] = take((size_t)c->Q * sg[s].N * e);
        buf[2 * s + 1] = take((size_t)c->Q * sg[s].N * e);
    }
    if (fused) {
        table[0] = c->slots;
        for (int s = 1; s < nslabs; ++s) {
            table[s] = (double *)take(tbytes);
            SLABCHK(c, hipMemsetAsync(table[s], 0xFF, tbytes, c->stream)); // NaN stamps: no record counts
        }
    }
    const int N = (int)c->geo.N;
    void *mono = c->f[c->cur];
    // scatter: each slab's rows and the two neighbouring rows (halos) of the
    // current populations
    auto halos = [&](int cur) -> hipError_t {
        hipError_t err = hipSuccess;
        for (int s = 0; s < nslabs && err == hipSuccess; ++s) {
            const int lo = s > 0 ? s - 1 : (per ? nslabs - 1 : -1);
            const int hi = s < nslabs - 1 ? s + 1 : (per ? 0 : -1);
            if (lo >= 0) // the top row of the slab below into the lower halo
                err = copy_rows(c, buf[2 * s + cur], sg[s].N, 0, buf[2 * lo + cur], sg[lo].N, sg[lo].rows, 1, plane);
            if (err == hipSuccess && hi >= 0) // the bottom row of the slab above into the upper halo
                err = copy_rows(c, buf[2 * s + cur], sg[s].N, sg[s].rows + 1, buf[2 * hi + cur], sg[hi].N, 1, 1, plane);
        }
        return err;
    };
    for (int s = 0; s < nslabs; ++s)
        SLABCHK(c, copy_rows(c, buf[2 * s], sg[s].N, 1, mono, N, sg[s].r0, sg[s].rows, plane));
    SLABCHK(c, halos(0));
    int cur = 0;
    const int64_t nrec = fused ? (int64_t)c->np * c->slot_stride : 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        ++c->epoch;
        for (int s = 0; s < nslabs; ++s) {
            SlotParams sl = slot_params(c, fused);
            if (fused) sl.slots = table[s];
            const hipError_t err = dispatch(c, [&](auto L, auto S, auto T) {
                using Lt = decltype(L);
                using St = decltype(S);
                using Tt = decltype(T);
                const Tt *acc = std::is_same<Tt, double>::value ? (const Tt *)c->P.acc_d : (const Tt *)c->P.acc_f;
                const int rows = Lt::D == 2 ? sg[s].rows : sg[s].rows * c->geo.ny;
                hipLaunchKernelGGL((k_slab_collide<Lt, St, Tt, 256>), dim3((unsigned)(rows * sg[s].gx)), dim3(256),
                                   0, c->stream, (const typename St::raw *)buf[2 * s + cur],
                                   (typename St::raw *)buf[2 * s + (cur ^ 1)], c->owner, acc,
                                   fused ? nullptr : c->usol, c->flags, c->geo, c->sp, sg[s], sl);
                return hipGetLastError();
            });
            SLABCHK(c, err);
        }
        cur ^= 1;
        SLABCHK(c, halos(cur)); // the halo exchange of the step
        if (fused) {
            // the cross-slab sums: every slab's records of this step into one table
            for (int s = 1; s < nslabs; ++s) {
                hipLaunchKernelGGL(k_merge_slots, dim3((unsigned)((nrec + 255) / 256)), dim3(256), 0, c->stream,
                                   table[0], (const double *)table[s], nrec, slot_width(d), (double)c->epoch);
                SLABCHK(c, hipGetLastError());
            }
            SLABCHK(c, launch_rigid_fused(c, nullptr));
            std::swap(c->P.X, c->P.Xn);
            std::swap(c->P.U, c->P.Unext);
            c->P.Uprev = c->P.U;
        } else if (c->np > 0) {
            SLABCHK(c, launch_reduce(c, 1, nullptr));
            SLABCHK(c, launch_rigid_raster(c, 1));
            std::swap(c->P.X, c->P.Xn);
        }
        c->step++;
        c->fresh = 0;
    }
    // gather: the slabs' rows back into the lattice's buffer
    for (int s = 0; s < nslabs; ++s)
        SLABCHK(c, copy_rows(c, mono, N, sg[s].r0, buf[2 * s + cur], sg[s].N, 1, sg[s].rows, plane));
    SLABCHK(c, hipStreamSynchronize(c->stream));
    return lbm_sync(c);
}
