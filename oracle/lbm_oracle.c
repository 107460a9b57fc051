/*
 * lbm_oracle.c -- plain FP64 CPU reference of the upscaled Brinkman lattice
 * Boltzmann method of J. Li and D. Brown, "Upscaled Lattice Boltzmann Method
 * for Simulations of Flows in Heterogeneous Porous Media" (arXiv:1312.0195).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the checker of the HIP path: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it. It shares no code, header, table or helper with the GPU library.
 *
 * Everything is in lattice units (dx = dt = c = 1, c_s^2 = 1/3) and FP64.
 * Populations are stored cell-major, f[(y*nx + x)*9 + a], with the D2Q9
 * velocities and weights of Sec. 2:
 *   e_0 = (0,0)                          w_0 = 4/9
 *   e_a = (cos t, sin t), t = (a-1) pi/2          a = 1..4, w = 1/9
 *   e_a = sqrt2 (cos t, sin t), t = (a-5) pi/2 + pi/4   a = 5..8, w = 1/36
 *
 * One time step is written exactly as the evolution equation states it
 * (collide at x, then move the post-collision value to x + e_a: "push").
 *
 * Two collision operators are provided:
 *   - Shan-Chen form (the paper's method, Sec. 2.2): rho = sum f, j = sum e f,
 *     u from Eq. explicit-u-in-Guo (equal to Eq. u-of-S-C with the drag of
 *     Eq. f_m-depends-on-u), u_eq from Eq. final-ueq-of-S-C, the linear
 *     equilibrium of Eq. feq and the force-free BGK update of Eq.
 *     f-evolution-of-S-C.
 *   - Guo form (Sec. 2.1): u from Eq. explicit-u-in-Guo, f_m from Eq.
 *     f_m-depends-on-u, u_eq = u, equilibrium Eq. feq and the forcing term
 *     F_a of Eq. Fi-of-Guo in Eq. f-evolution-of-Guo.
 * The permeability can be a scalar per cell (Eq. f_m-depends-on-u) or a full
 * 2x2 tensor per cell (Eq. f_m-depends-on-u-and-tensor-k, used on the coarse
 * grid); then the flow velocity of Eq. u-of-S-C is found by solving the 2x2
 * linear system that Eq. u-of-S-C and the tensor drag give together.
 *
 * Boundaries: periodic in x always; in y either periodic or halfway
 * bounce-back walls half a cell outside the first and last rows. The paper
 * only uses periodic boundaries; the walls are this project's reading for
 * channel-type runs.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC lbm_oracle.c -o liblbm_oracle.so -lm
 * (the OpenMP loops only split independent cells; every reduction runs
 * serially in a fixed order, so results do not depend on the thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

typedef struct {
    int32_t nx, ny;
    double tau;   /* BGK relaxation time */
    double eps;   /* porosity epsilon */
    double nu;    /* fluid viscosity nu in the drag term (independent of nu_eff) */
    double rho0;  /* initial density */
    int32_t walls_y;   /* 0: periodic in y; 1: halfway bounce-back walls in y */
    int32_t perm_kind; /* 1: scalar kappa per cell; 4: tensor [kxx kxy kyx kyy] */
    int32_t scheme;    /* 0: Shan-Chen form (the method); 1: Guo form */
} orc_params;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOTCONV = -3, ORC_ENONFINITE = -4 };

int orc_q(void) { return Q; }

/* Lattice constants, exposed so that tests can check them against Sec. 2. */
void orc_lattice(int32_t *ex, int32_t *ey, double *w, int32_t *opp)
{
    for (int a = 0; a < Q; ++a) { ex[a] = EX[a]; ey[a] = EY[a]; w[a] = W[a]; opp[a] = OPP[a]; }
}

/* Rest state f_a = w_a rho0 everywhere (the paper starts from rho0). */
void orc_init_rest(const orc_params *p, double *f)
{
    size_t n = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < n; ++c)
        for (int a = 0; a < Q; ++a) f[c * Q + a] = W[a] * p->rho0;
}

/* Flow velocity u of one cell (Eq. u-of-S-C with the drag force, which for a
 * scalar kappa is Eq. explicit-u-in-Guo), given rho, j and the force G. */
static void flow_velocity(const orc_params *p, const double *perm, double rho, double jx,
                          double jy, double gx, double gy, double *ux, double *uy)
{
    if (p->perm_kind == 1) {
        /* u = (j + dt/2 eps rho G) / (rho (1 + eps dt nu / (2 kappa))) */
        double kappa = perm[0];
        double denom = rho * (1.0 + p->eps * p->nu / (2.0 * kappa));
        *ux = (jx + 0.5 * p->eps * rho * gx) / denom;
        *uy = (jy + 0.5 * p->eps * rho * gy) / denom;
    } else {
        /* rho u = j + rho f_m / 2 with f_m = -eps nu K^{-1} u + eps G, i.e.
         * (I + eps nu K^{-1} / 2) u = (j + eps rho G / 2) / rho. */
        double kxx = perm[0], kxy = perm[1], kyx = perm[2], kyy = perm[3];
        double det = kxx * kyy - kxy * kyx;
        double ixx = kyy / det, ixy = -kxy / det, iyx = -kyx / det, iyy = kxx / det; /* K^{-1} */
        double h = 0.5 * p->eps * p->nu;
        double axx = 1.0 + h * ixx, axy = h * ixy, ayx = h * iyx, ayy = 1.0 + h * iyy;
        double bx = (jx + 0.5 * p->eps * rho * gx) / rho;
        double by = (jy + 0.5 * p->eps * rho * gy) / rho;
        double adet = axx * ayy - axy * ayx;
        *ux = (ayy * bx - axy * by) / adet;
        *uy = (-ayx * bx + axx * by) / adet;
    }
}

/* Force per unit mass f_m (Eq. f_m-depends-on-u, or its tensor form). */
static void drag_force(const orc_params *p, const double *perm, double ux, double uy, double gx,
                       double gy, double *fx, double *fy)
{
    if (p->perm_kind == 1) {
        double kappa = perm[0];
        *fx = -p->eps * p->nu / kappa * ux + p->eps * gx;
        *fy = -p->eps * p->nu / kappa * uy + p->eps * gy;
    } else {
        double kxx = perm[0], kxy = perm[1], kyx = perm[2], kyy = perm[3];
        double det = kxx * kyy - kxy * kyx;
        double ixx = kyy / det, ixy = -kxy / det, iyx = -kyx / det, iyy = kxx / det;
        *fx = -p->eps * p->nu * (ixx * ux + ixy * uy) + p->eps * gx;
        *fy = -p->eps * p->nu * (iyx * ux + iyy * uy) + p->eps * gy;
    }
}

/* Post-collision populations of one cell. */
static void collide_cell(const orc_params *p, const double *perm, double gx, double gy,
                         const double *f, double *fs)
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        jx += EX[a] * f[a];
        jy += EY[a] * f[a];
    }
    double ux, uy;
    flow_velocity(p, perm, rho, jx, jy, gx, gy, &ux, &uy);
    if (p->scheme == 0) {
        /* Shan-Chen form: u_eq = 2 tau u + (1 - 2 tau) j / rho, then BGK. */
        double uex = 2.0 * p->tau * ux + (1.0 - 2.0 * p->tau) * jx / rho;
        double uey = 2.0 * p->tau * uy + (1.0 - 2.0 * p->tau) * jy / rho;
        for (int a = 0; a < Q; ++a) {
            double feq = W[a] * rho * (1.0 + (EX[a] * uex + EY[a] * uey) / CS2);
            fs[a] = f[a] + (feq - f[a]) / p->tau;
        }
    } else {
        /* Guo form: u_eq = u, forcing term F_a with f_m evaluated at u. */
        double fmx, fmy;
        drag_force(p, perm, ux, uy, gx, gy, &fmx, &fmy);
        for (int a = 0; a < Q; ++a) {
            double feq = W[a] * rho * (1.0 + (EX[a] * ux + EY[a] * uy) / CS2);
            double Fa = W[a] * rho * (1.0 - 1.0 / (2.0 * p->tau)) * (EX[a] * fmx + EY[a] * fmy) / CS2;
            fs[a] = f[a] + (feq - f[a]) / p->tau + Fa;
        }
    }
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* One full time step f -> fnew: collide at every cell, then send each
 * post-collision f*_a(x) to x + e_a (periodic wrap, or bounce-back at the y
 * walls, where it returns to x as the opposite population).
 * force: per-cell G as [ny*nx][2] (x, y), or NULL for the uniform (gx, gy). */
void orc_step(const orc_params *p, const double *perm, const double *force, double gx, double gy,
              const double *f, double *fnew)
{
    const int nx = p->nx, ny = p->ny, pk = p->perm_kind;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        double fs[Q];
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double cgx = force ? force[2 * c] : gx;
            double cgy = force ? force[2 * c + 1] : gy;
            collide_cell(p, perm + c * pk, cgx, cgy, f + c * Q, fs);
            for (int a = 0; a < Q; ++a) {
                int xd = wrap(x + EX[a], nx);
                int yd = y + EY[a];
                if (p->walls_y && (yd < 0 || yd >= ny)) {
                    fnew[c * Q + OPP[a]] = fs[a];
                } else {
                    yd = wrap(yd, ny);
                    fnew[((size_t)yd * nx + xd) * Q + a] = fs[a];
                }
            }
        }
    }
}

/* Density, and flow velocity u (Eq. u-of-S-C) of every cell. rho may be NULL. */
void orc_moments(const orc_params *p, const double *perm, const double *force, double gx, double gy,
                 const double *f, double *rho_out, double *ux_out, double *uy_out)
{
    const size_t n = (size_t)p->nx * p->ny;
    const int pk = p->perm_kind;
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; ++c) {
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int a = 0; a < Q; ++a) {
            rho += f[c * Q + a];
            jx += EX[a] * f[c * Q + a];
            jy += EY[a] * f[c * Q + a];
        }
        double cgx = force ? force[2 * c] : gx;
        double cgy = force ? force[2 * c + 1] : gy;
        double ux, uy;
        flow_velocity(p, perm + c * pk, rho, jx, jy, cgx, cgy, &ux, &uy);
        if (rho_out) rho_out[c] = rho;
        ux_out[c] = ux;
        uy_out[c] = uy;
    }
}

/* Volume average of the flow velocity (Sec. 3: the bar over u is a volume
 * average over the domain), summed serially in cell order. */
void orc_mean_velocity(const orc_params *p, const double *perm, const double *force, double gx,
                       double gy, const double *f, double mean_u[2])
{
    const size_t n = (size_t)p->nx * p->ny;
    double *ux = (double *)malloc(n * sizeof(double));
    double *uy = (double *)malloc(n * sizeof(double));
    orc_moments(p, perm, force, gx, gy, f, NULL, ux, uy);
    double sx = 0.0, sy = 0.0;
    for (size_t c = 0; c < n; ++c) { sx += ux[c]; sy += uy[c]; }
    mean_u[0] = sx / (double)n;
    mean_u[1] = sy / (double)n;
    free(ux);
    free(uy);
}

static int valid_params(const orc_params *p)
{
    if (p->nx < 1 || p->ny < 1) return 0;
    if (!(p->tau >= 0.5) || !(p->eps > 0.0) || !(p->nu > 0.0) || !(p->rho0 > 0.0)) return 0;
    if (p->perm_kind != 1 && p->perm_kind != 4) return 0;
    if (p->scheme != 0 && p->scheme != 1) return 0;
    return 1;
}

/* Run from the populations in f (updated in place) for at most max_steps steps.
 * With check_every > 0 the volume-averaged velocity is taken every check_every
 * steps; the run stops once |ubar_k - ubar_{k-1}| <= tol |ubar_k| (tol > 0).
 * mean_u receives the average velocity of the final state.
 * Returns ORC_OK, ORC_ENOTCONV (tol > 0 but not reached), ORC_ENONFINITE. */
int orc_run(const orc_params *p, const double *perm, const double *force, double gx, double gy,
            double *f, int64_t max_steps, int32_t check_every, double tol, int64_t *steps_done,
            double mean_u[2])
{
    if (!valid_params(p)) return ORC_EINVAL;
    const size_t n = (size_t)p->nx * p->ny;
    double *g = (double *)malloc(n * Q * sizeof(double));
    double *cur_f = f, *next_f = g, *tmp;
    double prev[2] = {0.0, 0.0}, cur[2] = {0.0, 0.0};
    int have_prev = 0, status = (tol > 0.0) ? ORC_ENOTCONV : ORC_OK;
    int64_t s = 0;
    while (s < max_steps) {
        orc_step(p, perm, force, gx, gy, cur_f, next_f);
        tmp = cur_f; cur_f = next_f; next_f = tmp;
        ++s;
        if (check_every > 0 && s % check_every == 0) {
            orc_mean_velocity(p, perm, force, gx, gy, cur_f, cur);
            if (!isfinite(cur[0]) || !isfinite(cur[1])) { status = ORC_ENONFINITE; break; }
            if (tol > 0.0 && have_prev) {
                double dx = cur[0] - prev[0], dy = cur[1] - prev[1];
                double dn = sqrt(dx * dx + dy * dy), un = sqrt(cur[0] * cur[0] + cur[1] * cur[1]);
                if (dn <= tol * un) { status = ORC_OK; break; }
            }
            prev[0] = cur[0]; prev[1] = cur[1];
            have_prev = 1;
        }
    }
    if (cur_f != f) memcpy(f, cur_f, n * Q * sizeof(double));
    free(g);
    orc_mean_velocity(p, perm, force, gx, gy, f, mean_u);
    if (status != ORC_ENONFINITE && (!isfinite(mean_u[0]) || !isfinite(mean_u[1]))) status = ORC_ENONFINITE;
    *steps_done = s;
    return status;
}

/* Effective permeability of one periodic side x side subdomain (Sec. 3):
 * two local runs from rest, driven by G1 = (g, 0) and G2 = (0, g), each until
 * the relative change of the mean velocity over check_every steps is <= tol;
 * then Eq. tensor-kappa:
 *   kxx = nu ubar1_x / g, kxy = nu ubar2_x / g,
 *   kyx = nu ubar1_y / g, kyy = nu ubar2_y / g.
 * kappa_patch is [side][side] (x fastest). keff = [kxx, kxy, kyx, kyy];
 * steps[d] and status[d] report each drive. drive_mask bit 0 = x drive,
 * bit 1 = y drive; entries of a skipped drive are set to NaN. */
int orc_local_keff(const double *kappa_patch, int32_t side, double tau, double eps, double nu,
                   double g, int32_t check_every, double tol, int64_t max_steps, int32_t drive_mask,
                   double keff[4], int64_t steps[2], int32_t status[2])
{
    orc_params p;
    p.nx = side; p.ny = side; p.tau = tau; p.eps = eps; p.nu = nu; p.rho0 = 1.0;
    p.walls_y = 0; p.perm_kind = 1; p.scheme = 0;
    if (!valid_params(&p) || !(g > 0.0)) return ORC_EINVAL;
    const size_t n = (size_t)side * side;
    double *f = (double *)malloc(n * Q * sizeof(double));
    int worst = ORC_OK;
    for (int d = 0; d < 2; ++d) {
        double mu[2] = {NAN, NAN};
        steps[d] = 0; status[d] = ORC_OK;
        if (drive_mask & (1 << d)) {
            orc_init_rest(&p, f);
            double gx = (d == 0) ? g : 0.0, gy = (d == 1) ? g : 0.0;
            status[d] = orc_run(&p, kappa_patch, NULL, gx, gy, f, max_steps, check_every, tol,
                                &steps[d], mu);
            if (status[d] != ORC_OK && worst == ORC_OK) worst = status[d];
        }
        /* column d of the tensor holds the response to drive d */
        keff[0 + d] = nu * mu[0] / g; /* kxx (d=0) or kxy (d=1) */
        keff[2 + d] = nu * mu[1] / g; /* kyx (d=0) or kyy (d=1) */
    }
    free(f);
    return worst;
}

/* Average of a [ny][nx] field over r x r blocks -> [ny/r][nx/r], each block
 * summed serially (used to compare fine-grid results with the coarse grid). */
void orc_block_average(const double *field, int32_t nx, int32_t ny, int32_t r, double *out)
{
    int ncx = nx / r, ncy = ny / r;
    for (int J = 0; J < ncy; ++J)
        for (int I = 0; I < ncx; ++I) {
            double s = 0.0;
            for (int y = J * r; y < (J + 1) * r; ++y)
                for (int x = I * r; x < (I + 1) * r; ++x) s += field[(size_t)y * nx + x];
            out[(size_t)J * ncx + I] = s / ((double)r * r);
        }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
