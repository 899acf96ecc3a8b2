/*
 * sanitize_check.c -- a driver that runs the FP64 oracle (lbm_oracle.c) on
 * small cases under AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure only; see tests/test_oracle_sanitize.py).  It exercises
 * every public entry point: D2Q9 with contacts, an ellipse, a periodic
 * axis, K = 2 sub-steps and the rigid-velocity forcing; D3Q19 spheres; moving
 * walls; the fractional indicator (2D and 3D); mask replay; the single-node entry points (real build).  Built
 * with -DORACLE_COMPLEX it runs the complex-step build on the same cases.  Prints "ok" and exits 0
 * when every call succeeded.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int lattice, n[3], periodic[3];
    double tau, alpha, rho_f, g[3], u0[3], p0;
    double eps_p, eps_w, delta;
    int K, collision_form, gravity_form;
    double fluid_accel[3];
    int penalize_all;
    double wall_u[3][2][3];
    double rigid_beta;
    int no_stress_penalty;
    int fractional;
} ora_cfg;

typedef struct {
    int shape;
    double rho_s, a, b;
    double x[3], theta;
} ora_pin;

typedef struct ora_ctx ora_ctx;
int ora_create(const ora_cfg *cfg, ora_ctx **out);
void ora_destroy(ora_ctx *c);
int ora_set_particles(ora_ctx *c, int np, const ora_pin *pin);
int ora_set_replay(ora_ctx *c, long n0, long len, const double *X, const double *theta);
int ora_step(ora_ctx *c, long nsteps, double *rec, double *rec_im);
int ora_get_f(const ora_ctx *c, double *re, double *im);
int ora_set_f(ora_ctx *c, const double *re);
int ora_get_fields(ora_ctx *c, double *u, double *p, int32_t *owner);
int ora_get_particles(ora_ctx *c, double *re, double *im);
int ora_load_particles(ora_ctx *c, const double *v, long step);
#ifndef ORACLE_COMPLEX /* entry points of the real build only */
int ora_coll_forces(ora_ctx *c, double *F);
int ora_feq(int kind, double p, const double *u, double *out);
int ora_collide(int kind, double tau, double alpha, int solid, const double *f, const double *acc, double *ft);
#endif

static int run(const ora_cfg *cfg, int np, const ora_pin *pins, long steps)
{
    ora_ctx *c = NULL;
    if (ora_create(cfg, &c) || !c) return 1;
    if (ora_set_particles(c, np, pins)) return 2;
    long N = (long)cfg->n[0] * cfg->n[1] * (cfg->lattice ? cfg->n[2] : 1);
    int Q = cfg->lattice ? 19 : 9;
    double *rec = calloc((size_t)steps * np * 14, sizeof(double));
    double *f = calloc((size_t)N * Q, sizeof(double));
    double *u = calloc((size_t)N * 3, sizeof(double)), *p = calloc((size_t)N, sizeof(double));
    int32_t *own = calloc((size_t)N, sizeof(int32_t));
    double *parts = calloc((size_t)np * 22, sizeof(double)), *F = calloc((size_t)np * 3, sizeof(double));
    int rc = ora_step(c, steps, rec, NULL);
    rc |= ora_get_f(c, f, NULL) | ora_set_f(c, f) | ora_get_fields(c, u, p, own);
    rc |= ora_get_particles(c, parts, NULL) | ora_load_particles(c, parts, steps);
#ifndef ORACLE_COMPLEX
    rc |= ora_coll_forces(c, F);
#endif
    /* replay the recorded centres for a few more steps */
    double *X = calloc((size_t)3 * np * 3, sizeof(double)), *th = calloc((size_t)3 * np, sizeof(double));
    for (int s = 0; s < 3; s++)
        for (int i = 0; i < np; i++) {
            for (int k = 0; k < 3; k++) X[(s * np + i) * 3 + k] = parts[i * 22 + k];
            th[s * np + i] = parts[i * 22 + 3];
        }
    rc |= ora_set_replay(c, steps, 3, X, th) | ora_step(c, 3, NULL, NULL);
    ora_destroy(c);
    free(rec), free(f), free(u), free(p), free(own), free(parts), free(F), free(X), free(th);
    return rc;
}

int main(void)
{
    ora_cfg cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.lattice = 0;
    cfg.n[0] = 24, cfg.n[1] = 20, cfg.n[2] = 1;
    cfg.periodic[0] = 1;
    cfg.tau = 0.7, cfg.rho_f = 1.0, cfg.g[1] = -1e-3;
    cfg.eps_p = 2.0, cfg.eps_w = 1.0, cfg.delta = 1.0, cfg.K = 2, cfg.rigid_beta = 0.5;
    ora_pin p2[3] = {{0, 1.5, 3.0, 3.0, {6.0, 8.0, 0}, 0.0},
                     {1, 1.3, 4.0, 2.0, {13.5, 9.0, 0}, 0.7},
                     {0, 1.2, 2.5, 2.5, {22.8, 5.0, 0}, 0.0}};
    int rc = run(&cfg, 3, p2, 12);
    /* D3Q19 spheres, no forcing, K = 1 */
    memset(&cfg, 0, sizeof(cfg));
    cfg.lattice = 1;
    cfg.n[0] = 10, cfg.n[1] = 9, cfg.n[2] = 11;
    cfg.periodic[1] = 1;
    cfg.tau = 0.65, cfg.rho_f = 1.0, cfg.g[2] = -1e-3;
    cfg.eps_p = 2.0, cfg.eps_w = 1.0, cfg.delta = 1.0, cfg.K = 1;
    ora_pin p3[2] = {{2, 1.6, 2.0, 2.0, {3.0, 4.0, 4.0}, 0}, {2, 1.4, 2.2, 2.2, {6.5, 4.5, 6.0}, 0}};
    rc |= run(&cfg, 2, p3, 5) << 4;
    /* moving walls (Couette), one disk */
    memset(&cfg, 0, sizeof(cfg));
    cfg.lattice = 0;
    cfg.n[0] = 16, cfg.n[1] = 12, cfg.n[2] = 1;
    cfg.periodic[0] = 1;
    cfg.tau = 1.0, cfg.rho_f = 1.0, cfg.eps_p = 2.0, cfg.eps_w = 1.0, cfg.delta = 1.0, cfg.K = 1;
    cfg.wall_u[1][0][0] = -0.01, cfg.wall_u[1][1][0] = 0.01;
    ora_pin p1[1] = {{0, 1.0, 3.0, 3.0, {8.0, 6.0, 0}, 0}};
    rc |= run(&cfg, 1, p1, 6) << 8;
    /* the fractional indicator: disks in contact across a periodic axis, then spheres */
    memset(&cfg, 0, sizeof(cfg));
    cfg.lattice = 0;
    cfg.n[0] = 20, cfg.n[1] = 16, cfg.n[2] = 1;
    cfg.periodic[0] = 1;
    cfg.tau = 0.7, cfg.rho_f = 1.0, cfg.g[1] = -1e-3;
    cfg.eps_p = 2.0, cfg.eps_w = 1.0, cfg.delta = 1.0, cfg.K = 1, cfg.fractional = 1;
    ora_pin pf[2] = {{0, 1.5, 3.0, 3.0, {1.2, 8.0, 0}, 0.0}, {0, 1.3, 2.5, 2.5, {6.9, 8.3, 0}, 0.0}};
    rc |= run(&cfg, 2, pf, 6) << 12;
    memset(&cfg, 0, sizeof(cfg));
    cfg.lattice = 1;
    cfg.n[0] = 10, cfg.n[1] = 9, cfg.n[2] = 11;
    cfg.tau = 0.65, cfg.rho_f = 1.0, cfg.g[2] = -1e-3;
    cfg.eps_p = 2.0, cfg.eps_w = 1.0, cfg.delta = 1.0, cfg.K = 1, cfg.fractional = 1;
    rc |= run(&cfg, 2, p3, 4) << 16;
#ifndef ORACLE_COMPLEX
    /* single-node entry points */
    double u[3] = {0.01, -0.02, 0.0}, fe[19], acc[3] = {1e-4, 0, 0}, ft[19];
    rc |= ora_feq(0, 0.001, u, fe) | ora_collide(0, 0.8, 1.25, 1, fe, acc, ft);
    rc |= ora_feq(1, 0.001, u, fe) | ora_collide(1, 0.8, 1.25, 1, fe, acc, ft);
#endif
    if (rc) {
        printf("failed: %d\n", rc);
        return 1;
    }
    printf("ok\n");
    return 0;
}
