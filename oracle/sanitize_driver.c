/*
 * sanitize_driver.c -- runs every entry point of the C oracle (lbm_oracle.c)
 * once on small inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; TEST INFRASTRUCTURE ONLY, like
 * the oracle itself). Covers both collision forms, scalar and tensor
 * permeability, periodic and wall boundaries, a per-cell force field, the
 * local K_eff runs of Sec. 3 (Eq. tensor-kappa), a non-finite state and
 * block averages. Exits non-zero when a result is not finite or a status is
 * unexpected; the sanitizers abort on their own findings.
 *
 * Build: gcc -std=c11 -g -O1 -fsanitize=address,undefined -fno-omit-frame-pointer
 *        -fno-sanitize-recover=all sanitize_driver.c lbm_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny;
    double tau, eps, nu, rho0;
    int32_t walls_y, perm_kind, scheme;
} orc_params;

void orc_init_rest(const orc_params *p, double *f);
void orc_step(const orc_params *p, const double *perm, const double *force, double gx, double gy,
              const double *f, double *fnew);
void orc_moments(const orc_params *p, const double *perm, const double *force, double gx, double gy,
                 const double *f, double *rho_out, double *ux_out, double *uy_out);
void orc_mean_velocity(const orc_params *p, const double *perm, const double *force, double gx,
                       double gy, const double *f, double mean_u[2]);
int orc_run(const orc_params *p, const double *perm, const double *force, double gx, double gy,
            double *f, int64_t max_steps, int32_t check_every, double tol, int64_t *steps_done,
            double mean_u[2]);
int orc_local_keff(const double *kappa_patch, int32_t side, double tau, double eps, double nu,
                   double g, int32_t check_every, double tol, int64_t max_steps, int32_t drive_mask,
                   double keff[4], int64_t steps[2], int32_t status[2]);
void orc_block_average(const double *field, int32_t nx, int32_t ny, int32_t r, double *out);
void orc_lattice(int32_t *ex, int32_t *ey, double *w, int32_t *opp);

static int fail(const char *what)
{
    fprintf(stderr, "sanitize_driver: %s\n", what);
    return 1;
}

int main(void)
{
    const int nx = 7, ny = 5, n = nx * ny;
    double *kap = malloc(sizeof(double) * n), *ten = malloc(sizeof(double) * 4 * n);
    double *force = malloc(sizeof(double) * 2 * n);
    double *f = malloc(sizeof(double) * 9 * n), *g = malloc(sizeof(double) * 9 * n);
    double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n), *uy = malloc(sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        kap[c] = 0.5 + 0.1 * (c % 5);
        ten[4 * c] = kap[c];
        ten[4 * c + 1] = 0.1 * kap[c];
        ten[4 * c + 2] = -0.05 * kap[c];
        ten[4 * c + 3] = 0.7 * kap[c];
        force[2 * c] = 1e-5 * (1 + c % 3);
        force[2 * c + 1] = -1e-5 * (c % 2);
    }
    int32_t ex[9], ey[9], opp[9];
    double w[9];
    orc_lattice(ex, ey, w, opp);
    for (int scheme = 0; scheme < 2; ++scheme)
        for (int walls = 0; walls < 2; ++walls)
            for (int pk = 1; pk <= 4; pk += 3) {
                orc_params p = {nx, ny, 0.8, 0.4, 0.1, 1.0, walls, pk, scheme};
                const double *perm = pk == 1 ? kap : ten;
                orc_init_rest(&p, f);
                for (int s = 0; s < 3; ++s) {
                    orc_step(&p, perm, s == 1 ? force : NULL, 1e-6, 2e-7, f, g);
                    double *t = f; f = g; g = t;
                }
                orc_moments(&p, perm, force, 0.0, 0.0, f, rho, ux, uy);
                double mu[2];
                orc_mean_velocity(&p, perm, NULL, 1e-6, 0.0, f, mu);
                int64_t done = 0;
                int st = orc_run(&p, perm, NULL, 1e-6, 0.0, f, 400, 20, 1e-12, &done, mu);
                if (st != 0 && st != -3) return fail("unexpected run status");
                if (!isfinite(mu[0]) || !isfinite(mu[1]) || !isfinite(rho[0]) || !isfinite(ux[n - 1]) ||
                    !isfinite(uy[n - 1]))
                    return fail("non-finite result");
            }
    /* a non-finite state is reported, not trusted */
    {
        orc_params p = {nx, ny, 0.8, 0.4, 0.1, 1.0, 0, 1, 0};
        orc_init_rest(&p, f);
        f[9 * 3 + 2] = NAN;
        double mu[2];
        int64_t done = 0;
        if (orc_run(&p, kap, NULL, 1e-6, 0.0, f, 50, 10, 1e-9, &done, mu) != -4) return fail("NaN not reported");
    }
    /* local problems, both drives and one drive */
    {
        const int side = 6;
        double patch[36], keff[4];
        int64_t steps[2];
        int32_t status[2];
        for (int c = 0; c < side * side; ++c) patch[c] = exp(0.5 * sin(0.7 * c));
        if (orc_local_keff(patch, side, 0.8, 0.4, 0.1, 1e-6, 20, 1e-9, 20000, 3, keff, steps, status) != 0)
            return fail("local K_eff did not converge");
        if (!(keff[0] > 0.0) || !(keff[3] > 0.0)) return fail("local K_eff not positive");
        (void)orc_local_keff(patch, side, 0.8, 0.4, 0.1, 1e-6, 20, 1e-9, 20000, 2, keff, steps, status);
        if (!isnan(keff[0]) || !(keff[3] > 0.0)) return fail("skipped drive not NaN");
    }
    /* block averages */
    {
        double field[24], out[6];
        for (int i = 0; i < 24; ++i) field[i] = i;
        orc_block_average(field, 6, 4, 2, out);
        if (out[0] != 3.5) return fail("block average");
    }
    free(kap); free(ten); free(force); free(f); free(g); free(rho); free(ux); free(uy);
    printf("sanitize_driver ok\n");
    return 0;
}
