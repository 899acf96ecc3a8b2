// node.h -- per-node device arithmetic shared by the lattice kernels and
// their adjoints: the pull (streaming with halfway bounce-back and wrap),
// the macroscopic moments (eq. 15a-b), the equilibrium (eq. 13) and the
// collision with Guo forcing (eq. 14) and penalization (eq. 17).
#pragma once
#include <type_traits>
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
//
// I is the type of population offsets q N + node: int while Q N < 2^31 (every
// lattice the differentiated run and the slab step take), int64_t above.
template <class L, class I = int>
__device__ __forceinline__ I pull_offset(int q, int idx, int x, int y, int z, const Geom &g, I N)
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
    return wall ? (I)L::opp[q] * N + idx : (I)q * N + (sx + g.nx * (sy + g.ny * sz));
}

// The same offsets for a node of a row-segment kernel (one workgroup per
// segment of a lattice row): the source rows (y - c_y, z - c_z) are uniform
// across the workgroup, so their wrap and wall tests are made once, in scalar
// registers.  A segment that holds neither end of its row and whose source
// rows all exist (`interior`) needs no test per lane: population q of node x
// comes from (source row base + q N - c_x) + x, a uniform pointer plus the
// lane's column.  Other segments test x - 1 and x + 1 per lane and select.
template <class L, class I = int>
struct RowPull {
    int rb[3][3]; // [c_y + 1][c_z + 1]: (sy + ny sz) nx of the source row; -1 behind a wall
    int x, idx;
    I N;
    bool interior;
    const Geom &g;

    // source coordinate v - c on an axis of n nodes: wrapped, or flagged as
    // behind a wall (selects, no branches)
    static __device__ __forceinline__ int src(int v, int c, int n, int per, bool &wall)
    {
        int sv = v - c;
        const bool lo = sv < 0, hi = sv >= n;
        sv += lo ? n : 0;
        sv -= hi ? n : 0;
        wall = (lo || hi) && !per;
        return sv;
    }

    __device__ __forceinline__ RowPull(int x_, int y, int z, int idx_, bool inner_segment, const Geom &g_)
        : x(x_), idx(idx_), N((I)g_.N), g(g_)
    {
        bool walls = false;
#pragma unroll
        for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
            for (int cz = (L::D == 3 ? -1 : 0); cz <= (L::D == 3 ? 1 : 0); ++cz) {
                bool wy, wz = false;
                const int sy = src(y, cy, g.ny, g.per_y, wy);
                const int sz = L::D == 3 ? src(z, cz, g.nz, g.per_z, wz) : 0;
                const bool wall = wy || wz;
                walls = walls || wall;
                rb[cy + 1][cz + 1] = wall ? -1 : (sy + g.ny * sz) * g.nx;
            }
        interior = inner_segment && !walls;
    }
    // offset on any segment
    __device__ __forceinline__ I at(int q) const
    {
        return interior ? (I)q * N + rb[L::cy[q] + 1][L::cz[q] + 1] - L::cx[q] + x : offset(q);
    }
    // general offset (any segment): the column x - c_x tested per lane
    __device__ __forceinline__ I offset(int q) const
    {
        bool wx = false;
        const int s = L::cx[q] != 0 ? src(x, L::cx[q], g.nx, g.per_x, wx) : x;
        const int r = rb[L::cy[q] + 1][L::cz[q] + 1];
        const I a = (I)q * N + r + s, b = (I)L::opp[q] * N + idx;
        const I m = -(I)(r >= 0 && !wx); // branch-free select
        return (a & m) | (b & ~m);
    }
};

// Bounce-back off a moving wall (sec. 3.1 Couette benchmark): a population
// pulled from behind a halfway wall moving with u_w gains the difference of
// the equilibria of eq. (13) at u_w, f^eq_q - f^eq_opp(q) = 2 w_q (c_q . u_w)
// / cs^2.  Moving walls lie on one axis (y or z) and every other axis is
// periodic, so the term depends on the row (y, z) only; rows not next to a
// moving wall skip it.
// The term for population q and the low (side 0) or high wall, in FP64
// (a uniform load, made only on the rows next to a moving wall).
template <class L>
__device__ __forceinline__ double wall_term(int q, int side, const StepParams &sp)
{
    return sp.wall_tab[side * 19 + q];
}

template <class L, class T, int AX>
__device__ __forceinline__ void wall_motion_on(T *f, int v, int n, const StepParams &sp)
{
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
        const int c = AX == 1 ? L::cy[q] : L::cz[q];
        if (c == 0) continue;
        const int s = v - c; // source coordinate on the wall axis
        if (s < 0 || s >= n) f[q] += (T)wall_term<L>(q, s < 0 ? 0 : 1, sp);
    }
}

// Whether row (y, z) lies next to a moving wall (uniform).
__device__ __forceinline__ bool wall_row(int y, int z, const Geom &g, const StepParams &sp)
{
    if (sp.wall_axis == 1) return y == 0 || y == g.ny - 1;
    if (sp.wall_axis == 2) return z == 0 || z == g.nz - 1;
    return false;
}

template <class L, class T>
__device__ __forceinline__ void wall_motion(T *f, int y, int z, const Geom &g, const StepParams &sp)
{
    if (sp.wall_axis == 0) return; // uniform
    const int v = sp.wall_axis == 1 ? y : z, n = sp.wall_axis == 1 ? g.ny : g.nz;
    if (v != 0 && v != n - 1) return; // uniform
    if (L::D == 2 || sp.wall_axis == 1) wall_motion_on<L, T, 1>(f, v, n, sp);
    else wall_motion_on<L, T, 2>(f, v, n, sp);
}

// n / d for a uniform divisor d >= 1 with m = floor(2^32 / d) (2^32 - 1 for
// d = 1) precomputed on the host: the high product is the quotient or one
// less, so one correction gives it exactly (n < 2^31).
__device__ __forceinline__ int div_magic(int n, int d, unsigned m)
{
    int q = (int)__umulhi((unsigned)n, m);
    q += (n - q * d >= d) ? 1 : 0;
    return q;
}
static inline unsigned magic_for(int d) { return d == 1 ? 0xFFFFFFFFu : (unsigned)((1ull << 32) / (unsigned)d); }

// A stored population loaded into a register of its own (2-byte types
// zero-extended to 32 bits, so the compiler does not pack two of them into
// one register, which would need a wait per pair), converted later.
template <class S>
__device__ __forceinline__ auto ld_reg(const typename S::raw *p)
{
    if constexpr (sizeof(typename S::raw) == 2)
        return (uint32_t)__builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p));
    else
        return __builtin_nontemporal_load(p);
}
template <class S, class T, class R>
__device__ __forceinline__ T from_reg(R r)
{
    if constexpr (std::is_same<S, StF16>::value) return (T)__builtin_bit_cast(_Float16, (uint16_t)r);
    else if constexpr (std::is_same<S, StBF16>::value) return __uint_as_float(r << 16);
    else return r;
}

// base + i elements, with base made opaque to the compiler as a wave-uniform
// value and the element offset taken as a 32-bit byte offset (i * sizeof(P)
// < 2^32 for every lattice the library accepts): the access then takes the
// scalar-base form of the global instructions, base in scalar registers plus
// one 32-bit lane offset, instead of a 64-bit address add per access.  The
// byte offset i * sizeof(P) must stay below 2^32.
template <class P>
__device__ __forceinline__ P *uniform_at(P *base, int i)
{
    const uint64_t v = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    // arithmetic on a global (address space 1) pointer, so that the access
    // stays a global one after the integer round trip
    typedef __attribute__((address_space(1))) char gchar;
    gchar *b = (gchar *)(((uint64_t)hi << 32) | lo);
    return (P *)(b + (uint32_t)i * (uint32_t)sizeof(P));
}

// Loads in both branches and the conversion after them, so that no wait for
// the loads is placed at the branch join.
template <class L, class S, class T, class I = int>
__device__ __forceinline__ void pull_row(const typename S::raw *__restrict__ fin, const RowPull<L, I> &rp, T *f)
{
    decltype(ld_reg<S>(fin)) r[L::Q];
    if (rp.interior) { // uniform
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const typename S::raw *src = fin + ((I)q * rp.N + rp.rb[L::cy[q] + 1][L::cz[q] + 1] - L::cx[q]);
            r[q] = ld_reg<S>(uniform_at(src, rp.x));
        }
    } else {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) r[q] = ld_reg<S>(fin + rp.offset(q));
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) f[q] = from_reg<S, T>(r[q]);
}

template <class L, class S, class T, class I = int>
__device__ __forceinline__ void pull(const typename S::raw *__restrict__ fin, int idx, int x, int y, int z,
                                     const Geom &g, I N, T *f)
{
#pragma unroll
    for (int q = 0; q < L::Q; ++q) f[q] = ld<S, T>(fin + pull_offset<L, I>(q, idx, x, y, z, g, N));
}

// A sum whose terms are known at compile time to be present or not (after
// unrolling over q): absent terms are left out instead of added as zeros,
// which IEEE semantics would keep in the code (0 * v and x + 0 are not
// folded, though they change at most the sign of a zero).  Present terms are
// added in the order given.
template <class T>
struct CSum {
    T v = T(0);
    bool any = false;
    __device__ __forceinline__ void add(bool present, T t)
    {
        if (!present) return;
        v = any ? v + t : t;
        any = true;
    }
    __device__ __forceinline__ void sub(bool present, T t)
    {
        if (!present) return;
        v = any ? v - t : -t;
        any = true;
    }
};

// c_q . (vx, vy, vz) without the zero components of c_q
template <class L, class T>
__device__ __forceinline__ T cdot(int q, T vx, T vy, T vz)
{
    CSum<T> r;
    r.add(L::cx[q] > 0, vx);
    r.sub(L::cx[q] < 0, vx);
    r.add(L::cy[q] > 0, vy);
    r.sub(L::cy[q] < 0, vy);
    r.add(L::D == 3 && L::cz[q] > 0, vz);
    r.sub(L::D == 3 && L::cz[q] < 0, vz);
    return r.v;
}

// u = sum f c + a/2 and p = (cs^2 sum_{q>0} f - w0 |u|^2 / 2)/(1 - w0)  (eq. 15a-b)
template <class L, class T>
__device__ __forceinline__ void moments(const T *f, T ax, T ay, T az, T &ux, T &uy, T &uz, T &p)
{
    CSum<T> jx, jy, jz, s;
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
        jx.add(L::cx[q] > 0, f[q]);
        jx.sub(L::cx[q] < 0, f[q]);
        jy.add(L::cy[q] > 0, f[q]);
        jy.sub(L::cy[q] < 0, f[q]);
        jz.add(L::cz[q] > 0, f[q]);
        jz.sub(L::cz[q] < 0, f[q]);
        s.add(true, f[q]);
    }
    ux = jx.v + T(0.5) * ax;
    uy = jy.v + T(0.5) * ay;
    uz = (L::D == 3) ? jz.v + T(0.5) * az : T(0);
    const T uu = ux * ux + uy * uy + uz * uz;
    constexpr double w0 = L::w[0];
    p = (T(1.0 / 3.0) * s.v - T(0.5 * w0) * uu) * T(1.0 / (1.0 - w0));
}

// f^eq_q of eq. (13) with cs^2 = 1/3: q = 0: -(1-w0) 3p - w0 1.5|u|^2;
// q > 0: w_q (3p + 3 c.u + 4.5 (c.u)^2 - 1.5|u|^2)
template <class L, class T>
__device__ __forceinline__ T feq_q(int q, T p3, T cu, T u15)
{
    if (q == 0) return T(-(1.0 - L::w[0])) * p3 - T(L::w[0]) * u15;
    return T(L::w[q]) * (p3 + T(3) * cu + T(4.5) * cu * cu - u15);
}

// Weight of node idx in the fractional indicator of particle own (an
// extension; StepParams::frac): chi = min(1, R + 1/2 - |r|) with r = x - X,
// X the centre the indicator was built from, x the node taken at its
// nearest image on periodic axes; FP64, every product and sum rounded on its
// own (the inclusion test's arithmetic).  dX (optional) receives the
// derivative of chi in the centre: r/|r| where chi < 1, else zero.
__device__ __forceinline__ double frac_chi(int idx, uint16_t own, const StepParams &sp, double *dX = nullptr)
{
    const int x = idx % sp.n[0], yz = idx / sp.n[0];
    const int c[3] = {x, yz % sp.n[1], yz / sp.n[1]};
    double r2 = 0.0, r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double X = sp.geo[4 * own + k];
        int v = c[k];
        if (sp.per[k]) {
            const double half = 0.5 * sp.n[k], dd = (double)v - X;
            v += dd > half ? -sp.n[k] : (dd < -half ? sp.n[k] : 0);
        }
        r[k] = (k < 2 || sp.n[2] > 1) ? __dsub_rn((double)v, X) : 0.0;
        r2 = __dadd_rn(r2, __dmul_rn(r[k], r[k]));
    }
    const double len = sqrt(r2);
    const double v = __dsub_rn(__dadd_rn(sp.geo[4 * own + 3], 0.5), len);
    if (dX) {
        const bool edge = v < 1.0 && len > 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) dX[k] = edge ? r[k] / len : 0.0;
    }
    return v >= 1.0 ? 1.0 : v;
}

// Collision of one node, in place: f holds the pulled populations on entry
// and f~ on return (right side of eq. 10 with F of eq. 14 and, on solid
// nodes, S of eq. 17).  Writes the velocity of solid nodes for the sums
// (unless usol is NULL) and returns the node's velocity u (eq. 15a).
template <class L, class T>
__device__ __forceinline__ void collide_node(T *f, uint16_t own, const T *__restrict__ acc_tab, const StepParams &sp,
                                             int32_t *__restrict__ flags, double *__restrict__ usol, int idx, int N,
                                             T &uxo, T &uyo, T &uzo)
{
    const bool solid = own != FLUID;
    T ax = 0, ay = 0, az = 0;
    T chi = 1;
    if (solid) {
        ax = acc_tab[3 * own + 0];
        ay = acc_tab[3 * own + 1];
        az = acc_tab[3 * own + 2];
        if (sp.frac) { // the force density in proportion to the solid fraction
            chi = (T)frac_chi(idx, own, sp);
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
    uxo = ux;
    uyo = uy;
    uzo = uz;
    const T uu = ux * ux + uy * uy + uz * uz;
    if (!(uu < T(0.09))) flags[0] = 1; // |u| > 0.3 or not finite
    const T om = (T)sp.omega;
    const T p3 = T(3) * p, u15 = T(1.5) * uu;

    const bool pen = solid || sp.penalize_all;
    const bool frc = solid || sp.has_fluid_acc;
    if (!pen && !frc) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const T cu = cdot<L, T>(q, ux, uy, uz);
            f[q] = f[q] - om * (f[q] - feq_q<L, T>(q, p3, cu, u15));
        }
        return;
    }
    // solid (or forced) node
    T fneq[L::Q];
    T Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const T cu = cdot<L, T>(q, ux, uy, uz);
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
    // the penalization strength, in proportion to the solid fraction with the
    // fractional indicator
    const T al = pen ? (solid && sp.frac ? (T)((double)chi * sp.alpha) : (T)sp.alpha) : T(0);
    const T trace3 = (Pxx + Pyy + Pzz) * T(1.0 / 3.0);
    const T gpre = T(1) - T(0.5) * om;
    const T ua = L::D == 3 ? ux * ax + uy * ay + uz * az : ux * ax + uy * ay;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        // S_q = alpha w_q / (2 cs^4) Pi^neq : (c c - cs^2 I)   (eq. 17)
        CSum<T> diag, off;
        diag.add(L::cx[q] != 0, Pxx);
        diag.add(L::cy[q] != 0, Pyy);
        diag.add(L::cz[q] != 0, Pzz);
        off.add(L::cx[q] * L::cy[q] > 0, Pxy);
        off.sub(L::cx[q] * L::cy[q] < 0, Pxy);
        off.add(L::cx[q] * L::cz[q] > 0, Pxz);
        off.sub(L::cx[q] * L::cz[q] < 0, Pxz);
        off.add(L::cy[q] * L::cz[q] > 0, Pyz);
        off.sub(L::cy[q] * L::cz[q] < 0, Pyz);
        const T PiCC = off.any ? diag.v + T(2) * off.v : diag.v;
        const T Sq = al * T(4.5 * L::w[q]) * (PiCC - trace3);
        // F_q = (1 - 1/(2 tau)) w_q [3 (c - u).a + 9 (c.u)(c.a)]   (eq. 14)
        const T cu = cdot<L, T>(q, ux, uy, uz);
        const T ca = cdot<L, T>(q, ax, ay, az);
        const T F = gpre * T(L::w[q]) * (T(3) * (ca - ua) + T(9) * cu * ca);
        f[q] = f[q] - om * fneq[q] + F + Sq;
    }
    if (solid && usol) {
        usol[idx] = (double)ux;
        usol[N + idx] = (double)uy;
        if (L::D == 3) usol[2 * N + idx] = (double)uz;
    }
}

} // namespace lbm
