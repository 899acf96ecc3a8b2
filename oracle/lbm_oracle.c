/*
 * lbm_oracle.c -- plain, slow FP64 CPU oracle of the constraint-penalization
 * lattice Boltzmann step for rigid particles (Millet & Liberge,
 * arXiv 2511.01629).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library: lattice tables are derived
 * here from the velocity vectors, the layout is node-major (AoS), and every
 * formula is written out in the paper's notation.
 *
 * Scalar type.  `real` is double; built with -DORACLE_COMPLEX it is
 * double _Complex, which turns the same code into a complex-step derivative
 * (Squire & Trapp 1998): parameters carry an imaginary perturbation i*h*seed and
 * Im(output)/h is the exact directional derivative.  Every decision (indicator,
 * contact tests, wall tests) is taken on real parts, so the derivative is the
 * one of the discrete step map with the indicator sequence frozen.
 *
 * One step n -> n+1 (the paper's order, section 2):
 *   S1 indicator chi^n from X^n, theta^n              (sec. 2.1, eq. 9)
 *   S2 acceleration a = f/rho on each solid node     (sec. 2.1 eq. 5-8, sec. 2.4 Alg. 1)
 *   S3 macroscopic u, p                               (sec. 2.2, eq. 15a-b)
 *   S4 particle velocities U^n, omega^n               (sec. 2.4, eq. 22a-b)
 *   S5 collision with Guo force and penalization     (sec. 2.2, eq. 10, 13, 14, 17)
 *   S6 streaming (pull), halfway bounce-back walls    (sec. 2.2, eq. 10)
 *   S7 rigid-body update, Algorithm 1                 (sec. 2.3 eq. 19-21, sec. 2.4)
 *
 * Readings of points the paper leaves open (all documented with the design):
 *  - D2Q9 numbering follows the velocity-set figure (1..4 axes, 5..8
 *    diagonals); weights are assigned by speed (4/9, 1/9, 1/36), since the
 *    printed index rule contradicts the figure and is anisotropic.
 *  - Pi^neq = sum_a (f_a - f_a^eq) c_a c_a with pre-collision f and the
 *    half-force velocity (the printed definition lacks the c c factor).
 *  - S_a acts on solid nodes only; alpha defaults to 1/tau (sec. 3 preamble).
 *  - a = (1 - rho_f/rho_s,i) g + A_i on nodes owned by particle i, 0 elsewhere.
 *  - Indicator: closed set, lowest particle id owns a shared node, FP64 with
 *    no fused multiply-add, minimum image on periodic axes.
 *  - M_i = rho_s N_i, I_i = rho_s sum |r|^2 (3D: the discrete tensor),
 *    r = x - X_i.
 *  - Collision force with unit direction and C_i = (rho_s,i - rho_f)|g| V_i
 *    (form 0), or the printed form with the raw centre difference and
 *    C_i = (rho_s,i - rho_f)|g| (form 1).
 *  - theta^{n+1} = theta^n + (omega^n + omega^{n-1})/2 (2D).
 *  - Fractional indicator (an extension for gradients in the positions,
 *    disks and spheres only): chi_i(x) = min(1, R_i + 1/2 - |x - X_i|) on the
 *    band |x - X_i| < R_i + 1/2 (decided on |r|^2 < (R + 1/2)^2 in FP64 from
 *    real parts), the lowest id owning a node of two bands; every use of the
 *    indicator is weighted by chi: a = chi ((1 - rho_f/rho_s) g + A), the
 *    penalization strength chi alpha, and the sums N_i = sum chi,
 *    U_i = sum chi u / N_i, omega from sum chi r x u and sum chi |r|^2 (the
 *    tensor in 3D), M_i = rho_s N_i.  The binary indicator is its limit.
 *
 * Build:  gcc -O2 -std=gnu11 -ffp-contract=off -fopenmp -fPIC -shared
 *         [-DORACLE_COMPLEX] lbm_oracle.c -o liboracle[_cs].so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef ORACLE_COMPLEX
#include <complex.h>
typedef double _Complex real;
#define RE(z) creal(z)
#define IM(z) cimag(z)
#define SQRT(z) csqrt(z)
#else
typedef double real;
#define RE(z) (z)
#define IM(z) (0.0 * (z))
#define SQRT(z) sqrt(z)
#endif

#define QMAX 19
static const double CS2 = 1.0 / 3.0; /* c_s^2 with c = dx/dt = 1 (sec. 2.2) */

/* ------------------------------------------------------------------ lattice */
typedef struct {
    int Q, d;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} lattice_t;

static void lattice_init(lattice_t *L, int kind)
{
    memset(L, 0, sizeof(*L));
    if (kind == 0) {
        /* D2Q9 in the numbering of the velocity-set figure of sec. 2.2 */
        static const int c2[9][2] = {{0, 0},  {1, 0},   {0, 1},  {-1, 0}, {0, -1},
                                     {1, 1},  {-1, 1},  {-1, -1}, {1, -1}};
        L->Q = 9;
        L->d = 2;
        for (int a = 0; a < 9; a++) {
            L->c[a][0] = c2[a][0];
            L->c[a][1] = c2[a][1];
            L->c[a][2] = 0;
        }
    } else {
        /* D3Q19: rest, 6 faces, 12 edges; opposite directions adjacent */
        static const int c3[19][3] = {
            {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
            {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
            {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L->Q = 19;
        L->d = 3;
        for (int a = 0; a < 19; a++)
            for (int k = 0; k < 3; k++) L->c[a][k] = c3[a][k];
    }
    for (int a = 0; a < L->Q; a++) {
        int s = L->c[a][0] * L->c[a][0] + L->c[a][1] * L->c[a][1] + L->c[a][2] * L->c[a][2];
        if (L->d == 2)
            L->w[a] = (s == 0) ? 4.0 / 9.0 : (s == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
        else
            L->w[a] = (s == 0) ? 1.0 / 3.0 : (s == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        for (int b = 0; b < L->Q; b++)
            if (L->c[b][0] == -L->c[a][0] && L->c[b][1] == -L->c[a][1] && L->c[b][2] == -L->c[a][2])
                L->opp[a] = b;
    }
}

/* ------------------------------------------------------- per-node formulas */

/* Equilibrium, sec. 2.2 eq. (13):
 *   f_0^eq = -(1-w_0) p/cs2 - w_0 |u|^2/(2 cs2)
 *   f_a^eq = w_a [ p/cs2 + c.u/cs2 + (c.u)^2/(2 cs2^2) - |u|^2/(2 cs2) ]  */
static void feq_node(const lattice_t *L, real p, const real u[3], real out[QMAX])
{
    real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < L->Q; a++) {
        if (a == 0) {
            out[0] = -(1.0 - L->w[0]) * p / CS2 - L->w[0] * uu / (2.0 * CS2);
        } else {
            real cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
            out[a] = L->w[a] * (p / CS2 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
        }
    }
}

/* Macroscopic fields, sec. 2.2 eq. (15a-b) with dt = 1 and f/rho = a:
 *   u = sum_a f_a c_a + a/2 ;  p = ( cs2 sum_{a!=0} f_a - (w_0/2)|u|^2 ) / (1 - w_0) */
static void macro_node(const lattice_t *L, const real f[QMAX], const real acc[3], real u[3], real *p)
{
    for (int k = 0; k < 3; k++) {
        real s = 0.0;
        for (int a = 0; a < L->Q; a++) s += f[a] * L->c[a][k];
        u[k] = s + 0.5 * acc[k];
    }
    real sf = 0.0;
    for (int a = 1; a < L->Q; a++) sf += f[a];
    real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    *p = (CS2 * sf - 0.5 * L->w[0] * uu) / (1.0 - L->w[0]);
}

/* Guo forcing term, sec. 2.2 eq. (14), with f/rho = a:
 *   F_a = (1 - 1/(2 tau)) w_a [ (c_a - u)/cs2 + (c_a.u) c_a / cs2^2 ] . a   */
static void guo_node(const lattice_t *L, real tau, const real u[3], const real acc[3], real out[QMAX])
{
    real pre = 1.0 - 1.0 / (2.0 * tau);
    for (int a = 0; a < L->Q; a++) {
        real cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
        real s = 0.0;
        for (int k = 0; k < 3; k++) s += ((L->c[a][k] - u[k]) / CS2 + cu * L->c[a][k] / (CS2 * CS2)) * acc[k];
        out[a] = pre * L->w[a] * s;
    }
}

/* Penalization source, sec. 2.2 eq. (17): E = alpha Pi^neq,
 *   S_a = w_a/(2 cs2^2) E : (c_a c_a - cs2 I),  Pi^neq = sum_a (f_a - f_a^eq) c_a c_a */
static void penal_node(const lattice_t *L, real alpha, const real f[QMAX], const real feq[QMAX],
                       real out[QMAX])
{
    real Pi[3][3] = {{0}};
    for (int a = 0; a < L->Q; a++) {
        real fn = f[a] - feq[a];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) Pi[i][j] += fn * L->c[a][i] * L->c[a][j];
    }
    for (int a = 0; a < L->Q; a++) {
        real s = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double cc = L->c[a][i] * L->c[a][j] - (i == j && i < L->d ? CS2 : 0.0);
                s += alpha * Pi[i][j] * cc;
            }
        out[a] = L->w[a] / (2.0 * CS2 * CS2) * s;
    }
}

/* Post-collision populations of one node, the right side of sec. 2.2 eq. (10)
 * with dt = 1:  ft_a = f_a - (f_a - f_a^eq)/tau + F_a + S_a.
 * `solid` switches S on (penalization acts on the solid domain only). */
static void collide_node(const lattice_t *L, real tau, real alpha, int solid, const real f[QMAX],
                         const real acc[3], real ft[QMAX], real u[3], real *p)
{
    real feq[QMAX], F[QMAX], S[QMAX];
    macro_node(L, f, acc, u, p);
    feq_node(L, *p, u, feq);
    guo_node(L, tau, u, acc, F);
    if (solid)
        penal_node(L, alpha, f, feq, S);
    else
        for (int a = 0; a < L->Q; a++) S[a] = 0.0;
    for (int a = 0; a < L->Q; a++) ft[a] = f[a] - (f[a] - feq[a]) / tau + F[a] + S[a];
}

/* ------------------------------------------------------------------ context */
typedef struct {
    int lattice, n[3], periodic[3];
    double tau, alpha, rho_f, g[3], u0[3], p0;
    double eps_p, eps_w, delta;
    int K, collision_form, gravity_form;
    /* test knobs: uniform acceleration on fluid nodes (channel driving), and
     * the penalization source applied on every node */
    double fluid_accel[3];
    int penalize_all;
    /* tangential velocity of the halfway walls, [axis][low, high side][component];
     * moving walls only on the y or z axis, every other axis periodic */
    double wall_u[3][2][3];
    /* rigid-velocity forcing (an extension, not the paper's method): beta in
     * [0, 1], 0 = off; and a switch that leaves out the stress penalization */
    double rigid_beta;
    int no_stress_penalty;
    int fractional; /* 1: the fractional indicator (disks and spheres) */
} ora_cfg;

typedef struct {
    int shape; /* 0 disk, 1 ellipse (2D), 2 sphere (3D) */
    double rho_s, a, b;
    double x[3], theta;
} ora_pin;

typedef struct {
    int shape;
    real rho_s;
    double a, b;
    real X[3], theta;
    real U[3], W[3];         /* U^n, omega^n of the current step (valid after S4) */
    real Uprev[3], Wprev[3]; /* U^{n-1}, omega^{n-1} */
    real A[3];
    int N;       /* owned nodes */
    real Nw;     /* sum of the indicator over them: N, or sum chi (fractional) */
    real sum_r2; /* 2D: sum |r|^2 */
} particle_t;

typedef struct {
    lattice_t L;
    int n[3], periodic[3];
    long N;
    real tau, alpha, g[3];
    int alpha_tracks_tau;
    double rho_f, eps_p, eps_w, delta;
    int K, cform, gform;
    double fluid_accel[3];
    int penalize_all;
    int wall_axis; /* 0: no moving wall; else the axis of the moving walls */
    double wall_u[2][3];
    double beta;           /* rigid-velocity forcing strength (0: off) */
    int no_stress_penalty; /* 1: S of eq. (17) left out */
    int np;
    particle_t *p;
    real *f, *ft, *u, *pr;
    int *owner;
    int fractional;
    real *chi; /* fractional: the owner's chi at each node */
    long step;
    int perturbed;
    /* mask replay: rasterise from recorded centres/orientations */
    long rep_n0, rep_len;
    double *rep_X, *rep_theta;
    /* pending complex-step seeds of the particle densities and centres */
    double *pend_drho, *pend_dX;
    int pend_np;
} ora_ctx;

static long node_index(const ora_ctx *c, int x, int y, int z)
{
    return (long)x + (long)c->n[0] * ((long)y + (long)c->n[1] * (long)z);
}

static double bound_radius(int shape, double a)
{
    (void)shape;
    return a; /* disk/sphere radius, or the semi-major axis of an ellipse */
}

/* Unwrapped coordinate of node index xi along axis k closest to centre Xc. */
static long unwrap_coord(const ora_ctx *c, int k, long xi, double Xc)
{
    if (!c->periodic[k]) return xi;
    double half = 0.5 * c->n[k];
    double d = (double)xi - Xc;
    if (d > half) return xi - c->n[k];
    if (d < -half) return xi + c->n[k];
    return xi;
}

/* Inclusion test of S1, FP64, left-to-right, no contraction (-ffp-contract=off). */
static int inside_shape(int shape, double a, double b, double theta, const double dxyz[3])
{
    double dx = dxyz[0], dy = dxyz[1], dz = dxyz[2];
    if (shape == 0) return dx * dx + dy * dy <= a * a;
    if (shape == 2) return dx * dx + dy * dy + dz * dz <= a * a;
    double cs = cos(theta), sn = sin(theta);
    double xi = cs * dx + sn * dy;
    double eta = -sn * dx + cs * dy;
    return (b * b) * (xi * xi) + (a * a) * (eta * eta) <= (a * a) * (b * b);
}

/* S1: owner(x) = min{ i : x in Omega_i }, else -1 (sec. 2.1 eq. 9).
 * Each particle scans a box two nodes wider than its bounding radius, which
 * contains every node the predicate can accept. */
static void rasterize(ora_ctx *c)
{
    for (long i = 0; i < c->N; i++) c->owner[i] = -1;
    int d = c->L.d;
    for (int i = 0; i < c->np; i++) {
        particle_t *P = &c->p[i];
        double Xc[3] = {0, 0, 0}, th = RE(P->theta);
        long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        if (!c->fractional && c->rep_X && c->step >= c->rep_n0 && c->step < c->rep_n0 + c->rep_len) {
            long s = c->step - c->rep_n0;
            for (int k = 0; k < 3; k++) Xc[k] = c->rep_X[(s * c->np + i) * 3 + k];
            th = c->rep_theta[s * c->np + i];
        } else {
            for (int k = 0; k < 3; k++) Xc[k] = RE(P->X[k]);
        }
        double Rb = bound_radius(P->shape, P->a);
        for (int k = 0; k < d; k++) {
            lo[k] = (long)floor(Xc[k] - Rb) - 2;
            hi[k] = (long)ceil(Xc[k] + Rb) + 2;
            if (!c->periodic[k]) {
                if (lo[k] < 0) lo[k] = 0;
                if (hi[k] > c->n[k] - 1) hi[k] = c->n[k] - 1;
            }
        }
        for (long z = lo[2]; z <= hi[2]; z++)
            for (long y = lo[1]; y <= hi[1]; y++)
                for (long x = lo[0]; x <= hi[0]; x++) {
                    long xu[3] = {x, y, z}, xw[3];
                    double dd[3] = {0, 0, 0};
                    for (int k = 0; k < 3; k++) {
                        xw[k] = xu[k];
                        if (k < d && c->periodic[k]) xw[k] = ((xu[k] % c->n[k]) + c->n[k]) % c->n[k];
                        if (k < d) dd[k] = (double)xu[k] - Xc[k];
                    }
                    long id = node_index(c, (int)xw[0], (int)xw[1], (int)xw[2]);
                    if (c->fractional) {
                        /* the band |r| < R + 1/2, then chi = min(1, R + 1/2 - |r|) */
                        const double Rh = P->a + 0.5;
                        if (!(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2] < Rh * Rh)) continue;
                        if (c->owner[id] >= 0) continue; /* ascending i: lowest id wins */
                        real r2 = 0.0;
                        for (int k = 0; k < d; k++) {
                            real dk = (double)xu[k] - P->X[k];
                            r2 += dk * dk;
                        }
                        real v = Rh - SQRT(r2);
                        c->owner[id] = i;
                        c->chi[id] = RE(v) >= 1.0 ? (real)1.0 : v;
                        continue;
                    }
                    if (!inside_shape(P->shape, P->a, P->b, th, dd)) continue;
                    if (c->owner[id] < 0) c->owner[id] = i; /* ascending i: lowest id wins */
                }
    }
}

/* S2: acceleration f/rho on a node (sec. 2.1 eq. 5-8 and sec. 2.4):
 * gravity minus the hydrostatic part, divided by rho = rho_s, plus the
 * collision acceleration A_i of Algorithm 1; zero on fluid nodes. */
static void node_accel(const ora_ctx *c, long id, real acc[3])
{
    const int owner = c->owner[id];
    acc[0] = acc[1] = acc[2] = 0.0;
    if (owner < 0) {
        for (int k = 0; k < c->L.d; k++) acc[k] = c->fluid_accel[k];
        return;
    }
    const particle_t *P = &c->p[owner];
    real b = (c->gform == 0) ? (1.0 - c->rho_f / P->rho_s) : (P->rho_s / c->rho_f - 1.0);
    for (int k = 0; k < c->L.d; k++) acc[k] = b * c->g[k] + P->A[k];
    if (c->fractional) /* the force density in proportion to the solid fraction */
        for (int k = 0; k < c->L.d; k++) acc[k] = c->chi[id] * acc[k];
}

/* S3 over the whole lattice: u, p at every node from the current f. */
static void macros_all(ora_ctx *c)
{
    const int Q = c->L.Q;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < c->N; i++) {
        real acc[3], u[3], p;
        node_accel(c, i, acc);
        macro_node(&c->L, &c->f[i * Q], acc, u, &p);
        for (int k = 0; k < 3; k++) c->u[i * 3 + k] = u[k];
        c->pr[i] = p;
    }
}

/* Solve the symmetric 3x3 system T w = Lv by Cramer's rule. */
static void solve3(const real T[3][3], const real Lv[3], real w[3])
{
    real det = T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1]) -
               T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0]) +
               T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0]);
    for (int col = 0; col < 3; col++) {
        real M[3][3];
        for (int r = 0; r < 3; r++)
            for (int s = 0; s < 3; s++) M[r][s] = (s == col) ? Lv[r] : T[r][s];
        real dm = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                  M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                  M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        w[col] = dm / det;
    }
}

/* S4: U^n = (1/M) sum rho_s u,  I omega^n = sum r x (rho_s u)  (sec. 2.4,
 * eq. 22a-b), discrete sums over the owned nodes in lexicographic order;
 * rho_s cancels.  r = x - X_i with the unwrapped (minimum-image) node coordinate. */
static void reduce_particles(ora_ctx *c)
{
    const int d = c->L.d;
    int np = c->np;
    real *su = calloc((size_t)np * 3, sizeof(real));
    real *sl = calloc((size_t)np * 3, sizeof(real));
    real *si = calloc((size_t)np * 9, sizeof(real));
    real *sr2 = calloc((size_t)np, sizeof(real));
    real *sw = calloc((size_t)np, sizeof(real));
    int *cnt = calloc((size_t)np, sizeof(int));
    for (int z = 0; z < c->n[2]; z++)
        for (int y = 0; y < c->n[1]; y++)
            for (int x = 0; x < c->n[0]; x++) {
                long id = node_index(c, x, y, z);
                int o = c->owner[id];
                if (o < 0) continue;
                particle_t *P = &c->p[o];
                long xs[3] = {x, y, z};
                real r[3] = {0, 0, 0};
                for (int k = 0; k < d; k++) r[k] = (double)unwrap_coord(c, k, xs[k], RE(P->X[k])) - P->X[k];
                const real *u = &c->u[id * 3];
                const real wt = c->fractional ? c->chi[id] : (real)1.0; /* the node's weight */
                cnt[o]++;
                sw[o] += wt;
                for (int k = 0; k < 3; k++) su[o * 3 + k] += wt * u[k];
                if (d == 2) {
                    sl[o * 3 + 2] += wt * (r[0] * u[1] - r[1] * u[0]);
                    sr2[o] += wt * (r[0] * r[0] + r[1] * r[1]);
                } else {
                    sl[o * 3 + 0] += wt * (r[1] * u[2] - r[2] * u[1]);
                    sl[o * 3 + 1] += wt * (r[2] * u[0] - r[0] * u[2]);
                    sl[o * 3 + 2] += wt * (r[0] * u[1] - r[1] * u[0]);
                    real rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            si[o * 9 + a * 3 + b] += wt * ((a == b ? rr : 0.0) - r[a] * r[b]);
                }
            }
    for (int i = 0; i < np; i++) {
        particle_t *P = &c->p[i];
        P->N = cnt[i];
        P->Nw = sw[i];
        for (int k = 0; k < 3; k++) P->U[k] = 0.0, P->W[k] = 0.0;
        if (cnt[i] == 0 || RE(sw[i]) == 0.0) continue;
        for (int k = 0; k < d; k++) P->U[k] = su[i * 3 + k] / sw[i];
        if (d == 2) {
            P->sum_r2 = sr2[i];
            P->W[2] = sl[i * 3 + 2] / sr2[i];
        } else {
            real T[3][3];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) T[a][b] = si[i * 9 + a * 3 + b];
            solve3(T, &sl[i * 3], P->W);
        }
    }
    free(su);
    free(sl);
    free(si);
    free(sr2);
    free(sw);
    free(cnt);
}

/* Rigid-velocity forcing (an extension beyond the paper, off unless beta > 0):
 * on a node of particle i, the acceleration that moves the velocity of
 * eq. (15a) a fraction beta of the way from the fluid's own velocity u (S3,
 * with the gravity acceleration only) to the rigid motion of the particle,
 * U_i^n + omega_i^n x r with r = x - X_i^n (minimum image) and U^n, omega^n the
 * momentum sums of this step (S4, eq. 22a-b):
 *     a_rig = 2 beta (U_i + omega_i x r - u),
 * since eq. (15a) adds half the acceleration to the velocity, so that
 * u + a_rig/2 = (1 - beta) u + beta (U_i + omega_i x r).  The velocity is
 * then the rigid motion exactly for beta = 1, and the forcing adds no net
 * momentum over the particle (sum of a_rig = 2 beta omega x sum r, zero
 * when the nodes are centred on X_i). */
static void rigid_forcing(const ora_ctx *c, long id, real acc[3])
{
    const int d = c->L.d;
    const particle_t *P = &c->p[c->owner[id]];
    const long xs[3] = {id % c->n[0], (id / c->n[0]) % c->n[1], id / ((long)c->n[0] * c->n[1])};
    real r[3] = {0, 0, 0};
    for (int k = 0; k < d; k++) r[k] = (double)unwrap_coord(c, k, xs[k], RE(P->X[k])) - P->X[k];
    const real wr[3] = {P->W[1] * r[2] - P->W[2] * r[1], P->W[2] * r[0] - P->W[0] * r[2],
                        P->W[0] * r[1] - P->W[1] * r[0]};
    for (int k = 0; k < d; k++) acc[k] += 2.0 * c->beta * (P->U[k] + wr[k] - c->u[id * 3 + k]);
}

/* S5 + S6: collide every node, then pull-stream with halfway bounce-back on
 * wall axes and wrap-around on periodic axes (sec. 2.2 eq. 10). */
static void collide_stream(ora_ctx *c)
{
    const int Q = c->L.Q, d = c->L.d;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < c->N; i++) {
        real acc[3], u[3], p;
        node_accel(c, i, acc);
        if (c->owner[i] >= 0 && c->beta > 0.0) rigid_forcing(c, i, acc);
        int solid = (c->owner[i] >= 0 || c->penalize_all) && !c->no_stress_penalty;
        /* fractional indicator: the penalization in proportion to the solid fraction */
        real alpha = (c->fractional && c->owner[i] >= 0) ? c->chi[i] * c->alpha : c->alpha;
        collide_node(&c->L, c->tau, alpha, solid, &c->f[i * Q], acc, &c->ft[i * Q], u, &p);
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < c->N; i++) {
        long xs[3] = {i % c->n[0], (i / c->n[0]) % c->n[1], i / ((long)c->n[0] * c->n[1])};
        for (int a = 0; a < Q; a++) {
            long src[3];
            int wall = 0;
            for (int k = 0; k < 3; k++) {
                src[k] = xs[k] - (k < d ? c->L.c[a][k] : 0);
                if (src[k] < 0 || src[k] >= c->n[k]) {
                    if (c->periodic[k])
                        src[k] = (src[k] + c->n[k]) % c->n[k];
                    else
                        wall = 1;
                }
            }
            if (wall) {
                c->f[i * Q + a] = c->ft[i * Q + c->L.opp[a]];
                if (c->wall_axis) {
                    /* bounce-back off a moving wall (its other axes are periodic, so
                     * this is the wall crossed): the reflected population gains the
                     * difference of the two equilibria at the wall velocity,
                     * f^eq_a(u_w) - f^eq_opp(u_w) = 2 w_a (c_a . u_w) / cs2 (eq. 13) */
                    const int k = c->wall_axis, side = src[k] < 0 ? 0 : 1;
                    double cu = 0.0;
                    for (int j = 0; j < d; j++) cu += c->L.c[a][j] * c->wall_u[side][j];
                    c->f[i * Q + a] += 2.0 * c->L.w[a] * cu / CS2;
                }
            } else
                c->f[i * Q + a] = c->ft[node_index(c, (int)src[0], (int)src[1], (int)src[2]) * Q + a];
        }
    }
}

/* Collision constant of particle i (sec. 2.3): C = (rho_s - rho_f) g, read as
 * the buoyant weight (rho_s,i - rho_f)|g| V_i (form 0) or literally (form 1). */
static real coll_const(const ora_ctx *c, const particle_t *P)
{
    real gm = SQRT(c->g[0] * c->g[0] + c->g[1] * c->g[1] + c->g[2] * c->g[2]);
    real Cl = (P->rho_s - c->rho_f) * gm;
    if (c->cform == 1) return Cl;
    double V;
    if (P->shape == 0)
        V = M_PI * P->a * P->a;
    else if (P->shape == 1)
        V = M_PI * P->a * P->b;
    else
        V = 4.0 / 3.0 * M_PI * P->a * P->a * P->a;
    return Cl * V;
}

/* Total collision force on particle i with all particles at positions Y
 * (sec. 2.3 eq. 19-21): particle-particle and particle-wall (mirror) terms. */
static void coll_force(const ora_ctx *c, int i, real (*Y)[3], real F[3])
{
    const int d = c->L.d;
    const particle_t *P = &c->p[i];
    real Ci = coll_const(c, P);
    double Ri = bound_radius(P->shape, P->a), del = c->delta;
    F[0] = F[1] = F[2] = 0.0;
    for (int j = 0; j < c->np; j++) {
        if (j == i) continue;
        double Rj = bound_radius(c->p[j].shape, c->p[j].a);
        real dv[3] = {0, 0, 0};
        for (int k = 0; k < d; k++) {
            dv[k] = Y[i][k] - Y[j][k];
            if (c->periodic[k]) {
                double h = 0.5 * c->n[k];
                if (RE(dv[k]) > h) dv[k] -= c->n[k];
                else if (RE(dv[k]) < -h) dv[k] += c->n[k];
            }
        }
        real dist = SQRT(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (RE(dist) > Ri + Rj + del) continue;
        real s = (Ri + Rj + del - dist) / del;
        real mag = Ci / c->eps_p * s * s;
        for (int k = 0; k < d; k++) F[k] += (c->cform == 1) ? mag * dv[k] : mag * dv[k] / dist;
    }
    for (int k = 0; k < d; k++) {
        if (c->periodic[k]) continue;
        double walls[2] = {-0.5, c->n[k] - 0.5};
        for (int s = 0; s < 2; s++) {
            /* mirror centre across the wall plane: Y' = 2w - Y */
            real dv = Y[i][k] - (2.0 * walls[s] - Y[i][k]);
            real dist = (RE(dv) >= 0) ? dv : -dv;
            if (RE(dist) > 2.0 * Ri + del) continue;
            real q = (2.0 * Ri + del - dist) / del;
            real mag = Ci / c->eps_w * q * q;
            F[k] += (c->cform == 1) ? mag * dv : mag * dv / dist;
        }
    }
}

/* S7: Algorithm 1 of sec. 2.4 for all particles simultaneously. */
static void rigid_update(ora_ctx *c)
{
    const int d = c->L.d, np = c->np, K = c->K;
    if (np == 0) return;
    real(*Y)[3] = calloc((size_t)np, sizeof(*Y));
    real(*Ys)[3] = calloc((size_t)np, sizeof(*Ys));
    real(*Ub)[3] = calloc((size_t)np, sizeof(*Ub));
    real(*F0)[3] = calloc((size_t)np, sizeof(*F0));
    real(*F1)[3] = calloc((size_t)np, sizeof(*F1));
    real(*D)[3] = calloc((size_t)np, sizeof(*D)); /* summed corrections */
    for (int i = 0; i < np; i++)
        for (int k = 0; k < 3; k++) {
            Y[i][k] = c->p[i].X[k];
            Ub[i][k] = 0.5 * (c->p[i].U[k] + c->p[i].Uprev[k]);
        }
    for (int it = 1; it <= K; it++) {
        for (int i = 0; i < np; i++)
            for (int k = 0; k < d; k++) Ys[i][k] = Y[i][k] + Ub[i][k] / (double)K; /* prediction */
        for (int i = 0; i < np; i++) {
            coll_force(c, i, Y, F0[i]);
            coll_force(c, i, Ys, F1[i]);
        }
        for (int i = 0; i < np; i++) {
            real M = c->p[i].rho_s * c->p[i].Nw; /* rho_s N_i (N_i = sum chi when fractional) */
            for (int k = 0; k < d; k++) { /* correction */
                real corr = 1.0 / (2.0 * M) * (1.0 / ((double)K * K)) * (F0[i][k] + F1[i][k]) / 2.0;
                Y[i][k] = Ys[i][k] + corr;
                D[i][k] += corr;
            }
        }
    }
    for (int i = 0; i < np; i++) {
        particle_t *P = &c->p[i];
        for (int k = 0; k < d; k++) {
            /* A^{n+1} = 2 (X^{n+1} - X^n - U_bar): the bracket equals the sum of
             * the K correction displacements, taken directly so that no two
             * absolute positions are subtracted */
            P->A[k] = 2.0 * D[i][k];
            P->X[k] = Y[i][k];
            if (c->periodic[k]) {
                if (RE(P->X[k]) >= c->n[k]) P->X[k] -= c->n[k];
                else if (RE(P->X[k]) < 0.0) P->X[k] += c->n[k];
            }
        }
        if (d == 2) P->theta += 0.5 * (P->W[2] + P->Wprev[2]);
        for (int k = 0; k < 3; k++) {
            P->Uprev[k] = P->U[k];
            P->Wprev[k] = P->W[k];
        }
    }
    free(Y);
    free(Ys);
    free(Ub);
    free(F0);
    free(F1);
    free(D);
}

/* ------------------------------------------------------------- public API */

int ora_create(const ora_cfg *cfg, ora_ctx **out)
{
    if (!cfg || !out) return -1;
    if (cfg->lattice != 0 && cfg->lattice != 1) return -1;
    if (!(cfg->tau > 0.5)) return -1;
    ora_ctx *c = calloc(1, sizeof(ora_ctx));
    lattice_init(&c->L, cfg->lattice);
    for (int k = 0; k < 3; k++) {
        c->n[k] = cfg->n[k];
        c->periodic[k] = cfg->periodic[k];
    }
    if (c->L.d == 2) {
        c->n[2] = 1;
        c->periodic[2] = 0;
    }
    for (int k = 0; k < 3; k++)
        if (c->n[k] <= 0) {
            free(c);
            return -1;
        }
    c->N = (long)c->n[0] * c->n[1] * c->n[2];
    c->tau = cfg->tau;
    c->alpha_tracks_tau = !(cfg->alpha > 0);
    c->alpha = c->alpha_tracks_tau ? 1.0 / c->tau : cfg->alpha;
    if (RE(c->alpha) > 1.0 / RE(c->tau) * (1.0 + 1e-12)) {
        free(c);
        return -1;
    }
    c->rho_f = cfg->rho_f;
    for (int k = 0; k < 3; k++) c->g[k] = (k < c->L.d) ? cfg->g[k] : 0.0;
    c->eps_p = cfg->eps_p;
    c->eps_w = cfg->eps_w;
    c->delta = cfg->delta;
    c->K = cfg->K > 0 ? cfg->K : 1;
    c->cform = cfg->collision_form;
    c->gform = cfg->gravity_form;
    for (int k = 0; k < 3; k++) c->fluid_accel[k] = (k < c->L.d) ? cfg->fluid_accel[k] : 0.0;
    c->penalize_all = cfg->penalize_all;
    if (!(cfg->rigid_beta >= 0.0 && cfg->rigid_beta <= 1.0)) {
        free(c);
        return -1;
    }
    c->beta = cfg->rigid_beta;
    c->no_stress_penalty = cfg->no_stress_penalty != 0;
    c->fractional = cfg->fractional != 0;
    /* moving walls: one axis (y or z), tangential velocities, others periodic */
    for (int k = 0; k < 3; k++)
        for (int sd = 0; sd < 2; sd++)
            for (int j = 0; j < 3; j++) {
                if (cfg->wall_u[k][sd][j] == 0.0) continue;
                if (k == 0 || k >= c->L.d || c->periodic[k] || j == k || (c->wall_axis && c->wall_axis != k)) {
                    free(c);
                    return -1;
                }
                c->wall_axis = k;
            }
    if (c->wall_axis) {
        for (int k = 0; k < c->L.d; k++)
            if (k != c->wall_axis && !c->periodic[k]) {
                free(c);
                return -1;
            }
        for (int sd = 0; sd < 2; sd++)
            for (int j = 0; j < 3; j++) c->wall_u[sd][j] = j < c->L.d ? cfg->wall_u[c->wall_axis][sd][j] : 0.0;
    }
    const int Q = c->L.Q;
    c->f = calloc((size_t)c->N * Q, sizeof(real));
    c->ft = calloc((size_t)c->N * Q, sizeof(real));
    c->u = calloc((size_t)c->N * 3, sizeof(real));
    c->pr = calloc((size_t)c->N, sizeof(real));
    c->owner = malloc((size_t)c->N * sizeof(int));
    c->chi = calloc((size_t)c->N, sizeof(real));
    if (!c->f || !c->ft || !c->u || !c->pr || !c->owner || !c->chi) return -2;
    /* initial state: f = f^eq(p0, u0) everywhere */
    real u0[3] = {0, 0, 0}, fe[QMAX];
    for (int k = 0; k < c->L.d; k++) u0[k] = cfg->u0[k];
    feq_node(&c->L, cfg->p0, u0, fe);
    for (long i = 0; i < c->N; i++)
        for (int a = 0; a < Q; a++) c->f[i * Q + a] = fe[a];
    for (long i = 0; i < c->N; i++) c->owner[i] = -1;
    *out = c;
    return 0;
}

void ora_destroy(ora_ctx *c)
{
    if (!c) return;
    free(c->f);
    free(c->ft);
    free(c->u);
    free(c->pr);
    free(c->owner);
    free(c->p);
    free(c->rep_X);
    free(c->rep_theta);
    free(c->pend_drho);
    free(c->pend_dX);
    free(c->chi);
    free(c);
}

/* Complex-step seeds: parameters become value + i*h*seed (tau, |g| along the
 * fixed direction of g, and each rho_s,i).  Call between ora_create and
 * ora_set_particles, since U^0 already depends on the parameters.  In the
 * real build the imaginary part does not exist and the call is rejected. */
int ora_perturb(ora_ctx *c, const double *d_rho_s, int np, double d_tau, double d_gmag, double h,
                const double *d_X)
{
    if (!c) return -1;
#ifdef ORACLE_COMPLEX
    c->tau += I * h * d_tau;
    if (c->alpha_tracks_tau) c->alpha = 1.0 / c->tau;
    double gm = 0.0;
    for (int k = 0; k < 3; k++) gm += RE(c->g[k]) * RE(c->g[k]);
    gm = sqrt(gm);
    if (gm > 0)
        for (int k = 0; k < 3; k++) c->g[k] += I * h * d_gmag * RE(c->g[k]) / gm;
    free(c->pend_drho);
    c->pend_drho = NULL;
    c->pend_np = 0;
    free(c->pend_dX);
    c->pend_dX = NULL;
    if (d_rho_s && np > 0) {
        c->pend_drho = malloc(sizeof(double) * (size_t)np);
        for (int i = 0; i < np; i++) c->pend_drho[i] = h * d_rho_s[i];
        c->pend_np = np;
    }
    if (d_X && np > 0) { /* seeds of the initial centres, [np][3] */
        c->pend_dX = malloc(sizeof(double) * 3 * (size_t)np);
        for (int i = 0; i < 3 * np; i++) c->pend_dX[i] = h * d_X[i];
        c->pend_np = np;
    }
    return 0;
#else
    (void)d_X;
    (void)d_rho_s;
    (void)np;
    (void)d_tau;
    (void)d_gmag;
    (void)h;
    return -1;
#endif
}

/* Copy particles in, rasterise, compute U^0, omega^0 and seed U^{-1} = U^0. */
int ora_set_particles(ora_ctx *c, int np, const ora_pin *pin)
{
    if (!c || np < 0) return -1;
    free(c->p);
    c->np = np;
    c->p = calloc((size_t)(np > 0 ? np : 1), sizeof(particle_t));
    for (int i = 0; i < np; i++) {
        particle_t *P = &c->p[i];
        P->shape = pin[i].shape;
        P->rho_s = pin[i].rho_s;
#ifdef ORACLE_COMPLEX
        if (c->pend_drho && i < c->pend_np) P->rho_s += I * c->pend_drho[i];
#endif
        P->a = pin[i].a;
        P->b = pin[i].b;
        for (int k = 0; k < 3; k++) P->X[k] = (k < c->L.d) ? pin[i].x[k] : 0.0;
#ifdef ORACLE_COMPLEX
        if (c->pend_dX && i < c->pend_np)
            for (int k = 0; k < c->L.d; k++) P->X[k] += I * c->pend_dX[3 * i + k];
#endif
        P->theta = pin[i].theta;
        if (c->fractional && P->shape == 1) return -1; /* disks and spheres only */
    }
    rasterize(c);
    macros_all(c);
    reduce_particles(c);
    for (int i = 0; i < np; i++)
        for (int k = 0; k < 3; k++) {
            c->p[i].Uprev[k] = c->p[i].U[k];
            c->p[i].Wprev[k] = c->p[i].W[k];
        }
    return 0;
}

/* Replay: rasterise step s (absolute step index n0+s) from recorded centres
 * X[s][np][3] and orientations theta[s][np] instead of the live state. */
int ora_set_replay(ora_ctx *c, long n0, long len, const double *X, const double *theta)
{
    free(c->rep_X);
    free(c->rep_theta);
    c->rep_X = NULL;
    c->rep_theta = NULL;
    c->rep_len = 0;
    if (len <= 0 || !X) return 0;
    c->rep_X = malloc(sizeof(double) * (size_t)len * c->np * 3);
    c->rep_theta = malloc(sizeof(double) * (size_t)len * c->np);
    memcpy(c->rep_X, X, sizeof(double) * (size_t)len * c->np * 3);
    memcpy(c->rep_theta, theta, sizeof(double) * (size_t)len * c->np);
    c->rep_n0 = n0;
    c->rep_len = len;
    return 0;
}

/* Per-step record layout (doubles per particle): X[3] theta U[3] W[3] A[3] N */
#define REC_W 14

/* Advance n steps.  If rec (real parts) / rec_im (imaginary parts) are given,
 * record X^n, theta^n, U^n, omega^n, A^n, N^n (sum chi when fractional) of
 * every step. */
int ora_step(ora_ctx *c, long nsteps, double *rec, double *rec_im)
{
    for (long s = 0; s < nsteps; s++) {
        rasterize(c);        /* S1 */
        macros_all(c);       /* S2, S3 */
        reduce_particles(c); /* S4 */
        for (int i = 0; i < c->np; i++) {
            particle_t *P = &c->p[i];
            real v[REC_W] = {P->X[0], P->X[1], P->X[2], P->theta, P->U[0], P->U[1], P->U[2],
                             P->W[0], P->W[1], P->W[2], P->A[0], P->A[1], P->A[2], P->Nw};
            for (int k = 0; k < REC_W; k++) {
                if (rec) rec[(s * c->np + i) * REC_W + k] = RE(v[k]);
                if (rec_im) rec_im[(s * c->np + i) * REC_W + k] = IM(v[k]);
            }
        }
        collide_stream(c); /* S5, S6 */
        rigid_update(c);   /* S7 */
        c->step++;
    }
    return 0;
}

long ora_get_step(const ora_ctx *c) { return c->step; }

/* Populations f^n (pre-collision), node-major [N][Q]. */
int ora_get_f(const ora_ctx *c, double *re, double *im)
{
    long n = c->N * c->L.Q;
    for (long i = 0; i < n; i++) {
        if (re) re[i] = RE(c->f[i]);
        if (im) im[i] = IM(c->f[i]);
    }
    return 0;
}

int ora_set_f(ora_ctx *c, const double *re)
{
    long n = c->N * c->L.Q;
    for (long i = 0; i < n; i++) c->f[i] = re[i];
    return 0;
}

/* Fields of the current state: u[N][3], p[N], owner[N] (S1-S3 evaluated now). */
int ora_get_fields(ora_ctx *c, double *u, double *p, int32_t *owner)
{
    rasterize(c);
    macros_all(c);
    for (long i = 0; i < c->N; i++) {
        if (u)
            for (int k = 0; k < 3; k++) u[i * 3 + k] = RE(c->u[i * 3 + k]);
        if (p) p[i] = RE(c->pr[i]);
        if (owner) owner[i] = c->owner[i];
    }
    return 0;
}

/* Particle state now (doubles per particle): X[3] theta U^n[3] W^n[3]
 * Uprev[3] Wprev[3] A[3] N Nw pad (22 values); U^n, omega^n, N are measured
 * now; Nw is sum chi over the owned nodes (= N for the binary indicator). */
#define PART_W 22
int ora_get_particles(ora_ctx *c, double *re, double *im)
{
    rasterize(c);
    macros_all(c);
    reduce_particles(c);
    for (int i = 0; i < c->np; i++) {
        particle_t *P = &c->p[i];
        real v[PART_W] = {P->X[0],     P->X[1],     P->X[2],     P->theta,    P->U[0],     P->U[1],
                          P->U[2],     P->W[0],     P->W[1],     P->W[2],     P->Uprev[0], P->Uprev[1],
                          P->Uprev[2], P->Wprev[0], P->Wprev[1], P->Wprev[2], P->A[0],     P->A[1],
                          P->A[2],     (double)P->N, P->Nw};
        for (int k = 0; k < PART_W; k++) {
            if (re) re[i * PART_W + k] = (k < 21) ? RE(v[k]) : 0.0;
            if (im) im[i * PART_W + k] = (k < 21) ? IM(v[k]) : 0.0;
        }
    }
    return 0;
}

/* Restore the particle state variables X, theta, U^{n-1}, omega^{n-1}, A
 * (layout of ora_get_particles; real parts) -- used by tests to start the
 * oracle from a given mid-run state together with ora_set_f. */
int ora_load_particles(ora_ctx *c, const double *v, long step)
{
    for (int i = 0; i < c->np; i++) {
        particle_t *P = &c->p[i];
        const double *q = &v[i * PART_W];
        for (int k = 0; k < 3; k++) {
            P->X[k] = q[k];
            P->Uprev[k] = q[10 + k];
            P->Wprev[k] = q[13 + k];
            P->A[k] = q[16 + k];
        }
        P->theta = q[3];
    }
    c->step = step;
    return 0;
}

#ifndef ORACLE_COMPLEX
/* ---- single-node entry points for the pins (real build only) ---- */
int ora_lattice(int kind, int *Q, int *d, int *c, double *w, int *opp)
{
    lattice_t L;
    lattice_init(&L, kind);
    *Q = L.Q;
    *d = L.d;
    for (int a = 0; a < L.Q; a++) {
        for (int k = 0; k < 3; k++) c[a * 3 + k] = L.c[a][k];
        w[a] = L.w[a];
        opp[a] = L.opp[a];
    }
    return 0;
}

int ora_feq(int kind, double p, const double *u, double *out)
{
    lattice_t L;
    lattice_init(&L, kind);
    feq_node(&L, p, u, out);
    return 0;
}

int ora_macro(int kind, const double *f, const double *acc, double *u, double *p)
{
    lattice_t L;
    lattice_init(&L, kind);
    macro_node(&L, f, acc, u, p);
    return 0;
}

int ora_guo(int kind, double tau, const double *u, const double *acc, double *out)
{
    lattice_t L;
    lattice_init(&L, kind);
    guo_node(&L, tau, u, acc, out);
    return 0;
}

int ora_penal(int kind, double alpha, const double *f, const double *feq, double *out)
{
    lattice_t L;
    lattice_init(&L, kind);
    penal_node(&L, alpha, f, feq, out);
    return 0;
}

int ora_collide(int kind, double tau, double alpha, int solid, const double *f, const double *acc, double *ft)
{
    lattice_t L;
    double u[3], p;
    lattice_init(&L, kind);
    collide_node(&L, tau, alpha, solid, f, acc, ft, u, &p);
    return 0;
}

/* Collision force on each particle at the current centres (for the pins). */
int ora_coll_forces(ora_ctx *c, double *F)
{
    real(*Y)[3] = calloc((size_t)(c->np > 0 ? c->np : 1), sizeof(*Y));
    for (int i = 0; i < c->np; i++)
        for (int k = 0; k < 3; k++) Y[i][k] = c->p[i].X[k];
    for (int i = 0; i < c->np; i++) coll_force(c, i, Y, (real *)&F[i * 3]);
    free(Y);
    return 0;
}
#endif
