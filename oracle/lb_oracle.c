/*
 * lb_oracle.c -- plain, slow FP64 CPU oracle for one timestep of D3Q19
 * lattice Boltzmann for a symmetric binary fluid (free-energy model).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Every loop runs over lattice sites one at a time, in the order the method
 * states the step (the paper's Ludwig timestep, Sec. 2.1.1: order-parameter
 * gradients, chemical stress, collision, propagation), with no blocking or
 * fusion:
 *
 *   phi(x)      = sum_i g_i(x)                                  (moment)
 *   d_a phi(x)  = [phi(x+e_a) - phi(x-e_a)] / 2                 (7-point FD)
 *   lap phi(x)  = sum_a [phi(x+e_a) + phi(x-e_a) - 2 phi(x)]
 *   mu          = A phi + B phi^3 - kappa lap phi
 *   Pi_ab       = [A/2 phi^2 + 3B/4 phi^4 - kappa phi lap phi
 *                  - kappa/2 |grad phi|^2] delta_ab + kappa d_a phi d_b phi
 *   rho = sum_i f_i,  j = sum_i f_i c_i,  u = j / rho
 *   feq_i = w_i [rho + 3 c_i.j + 9/2 Q_i : (Pi + rho u u)]
 *   geq_i = w_i [phi + 3 phi c_i.u + 9/2 Q_i : ((Gamma mu - phi/3) I + phi u u)]
 *   Q_i   = c_i c_i - I/3
 *   f*_i  = f_i - (f_i - feq_i)/tau_f,   g*_i = g_i - (g_i - geq_i)/tau_g
 *   f_i(x + c_i, t+1) = f*_i(x, t)   (periodic; same for g)
 *
 * Force coupling (coupling = 1; the paper's statement for its Ludwig model,
 * Sec. 2.1.1: the divergence of the chemical stress acts as a body force):
 *
 *   F_a(x)      = - sum_b [Pi_ab(x+e_b) - Pi_ab(x-e_b)] / 2      (central div)
 *   u           = (j + F/2) / rho
 *   feq_i       = w_i rho [1 + 3 c_i.u + 9/2 Q_i : u u]   (no Pi)
 *   geq_i       as above with this u
 *   f*_i        = f_i - (f_i - feq_i)/tau_f
 *                 + (1 - 1/(2 tau_f)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F
 *
 * (Guo, Zheng and Shi's forcing term: the collision adds exactly F to the
 * momentum of every site.)
 *
 * Finite-difference order parameter (order_param = 1): the binary-fluid
 * counterpart of the paper's "Advection" and order-parameter update kernels
 * (Sec. 2.1.1).  There is no g; the state is (f, phi) with phi a field, and
 * phi follows a conservative Cahn-Hilliard update with advection, fluxes on
 * the faces between neighbouring sites (face x + e_a/2 belongs to x):
 *
 *   u_f(x + e_a/2) = [u_a(x) + u_a(x + e_a)] / 2          (u = j/rho of f)
 *   J_a(x + e_a/2) = u_f * (u_f > 0 ? phi(x) : phi(x + e_a))    (upwind)
 *                    - M [mu(x + e_a) - mu(x)]                  (diffusion)
 *   phi(x, t+1)    = phi(x) - sum_a [J_a(x + e_a/2) - J_a(x - e_a/2)]
 *   M              = Gamma (tau_g - 1/2)
 *
 * (the mobility the g scheme above gives, so both schemes solve the same
 * Cahn-Hilliard equation).  mu and Pi from phi(t).  With coupling = 0, f
 * collides with Pi in f^eq as in the first form and u = j/rho of f(t)
 * before collision; with coupling = 1 (the paper's arrangement: the stress
 * divergence acts on the fluid, the order parameter follows finite
 * differences), f collides with the force F = -div Pi as above and the
 * fluxes use the same velocity u = (j + F/2)/rho.
 *
 * The paper does not print these formulas (it names the kernels only); they
 * are the standard free-energy binary-fluid LB model.  The readings taken
 * where the paper is silent (equilibrium form for all i including the rest
 * velocity, 7-point stencil, Gamma entering g^eq directly, initial state) are
 * listed with the design notes of the repository.
 *
 * Storage: a distribution is double[19][N], component-major, with sites in
 * C order (x slowest, z fastest): s = (x*ny + y)*nz + z.  Vectors are
 * double[3][N]; the symmetric tensor Pi is double[6][N] in the order
 * xx, xy, xz, yy, yz, zz.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double A, B, kappa, gamma, tau_f, tau_g, rho0;
    int32_t coupling; /* 0: Pi in f^eq's second moment; 1: force -div Pi */
    int32_t order_param; /* 0: LB distribution g; 1: finite-difference field */
} oracle_params;

#define NVEL 19

/* D3Q19 velocities: rest, the 6 faces, the 12 edges. */
static const int CV[NVEL][3] = {
    { 0, 0, 0},
    { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
    { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0},
    { 1, 0, 1}, {-1, 0,-1}, { 1, 0,-1}, {-1, 0, 1},
    { 0, 1, 1}, { 0,-1,-1}, { 0, 1,-1}, { 0,-1, 1},
};

static double weight(int i)
{
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static long nsites(const oracle_params *p)
{
    return (long)p->nx * p->ny * p->nz;
}

static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Linear index of the site (x, y, z), coordinates taken modulo the extents. */
static long site_index(const oracle_params *p, int x, int y, int z)
{
    return ((long)wrap(x, p->nx) * p->ny + wrap(y, p->ny)) * p->nz + wrap(z, p->nz);
}

static void site_coords(const oracle_params *p, long s, int *x, int *y, int *z)
{
    *z = (int)(s % p->nz);
    *y = (int)((s / p->nz) % p->ny);
    *x = (int)(s / ((long)p->nz * p->ny));
}

/* ---- lattice table, for the identity tests ---------------------------- */

void oracle_lattice(int32_t *c_out /* [19][3] */, double *w_out /* [19] */)
{
    for (int i = 0; i < NVEL; i++) {
        for (int a = 0; a < 3; a++) c_out[3 * i + a] = CV[i][a];
        w_out[i] = weight(i);
    }
}

/* ---- order parameter: phi = sum_i g_i --------------------------------- */

void oracle_order_parameter(const oracle_params *p, const double *g, double *phi)
{
    long n = nsites(p);
    for (long s = 0; s < n; s++) {
        double acc = 0.0;
        for (int i = 0; i < NVEL; i++) acc += g[i * n + s];
        phi[s] = acc;
    }
}

/* ---- order-parameter gradients (7-point central differences) ---------- */

void oracle_gradients(const oracle_params *p, const double *phi,
                      double *grad /* [3][N] */, double *lap /* [N] */)
{
    long n = nsites(p);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        int x, y, z;
        site_coords(p, s, &x, &y, &z);
        double xp = phi[site_index(p, x + 1, y, z)], xm = phi[site_index(p, x - 1, y, z)];
        double yp = phi[site_index(p, x, y + 1, z)], ym = phi[site_index(p, x, y - 1, z)];
        double zp = phi[site_index(p, x, y, z + 1)], zm = phi[site_index(p, x, y, z - 1)];
        double c = phi[s];
        grad[0 * n + s] = 0.5 * (xp - xm);
        grad[1 * n + s] = 0.5 * (yp - ym);
        grad[2 * n + s] = 0.5 * (zp - zm);
        lap[s] = (xp + xm - 2.0 * c) + (yp + ym - 2.0 * c) + (zp + zm - 2.0 * c);
    }
}

/* ---- chemical potential and chemical stress (local) ------------------- */

static void chemical_site(const oracle_params *p, double phi, const double gr[3], double lp,
                          double *mu, double pi[6])
{
    double g2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
    *mu = p->A * phi + p->B * phi * phi * phi - p->kappa * lp;
    double iso = 0.5 * p->A * phi * phi + 0.75 * p->B * phi * phi * phi * phi
               - p->kappa * phi * lp - 0.5 * p->kappa * g2;
    pi[0] = iso + p->kappa * gr[0] * gr[0];
    pi[1] =       p->kappa * gr[0] * gr[1];
    pi[2] =       p->kappa * gr[0] * gr[2];
    pi[3] = iso + p->kappa * gr[1] * gr[1];
    pi[4] =       p->kappa * gr[1] * gr[2];
    pi[5] = iso + p->kappa * gr[2] * gr[2];
}

void oracle_chemical(const oracle_params *p, const double *phi, const double *grad,
                     const double *lap, double *mu /* [N] */, double *pi /* [6][N] */)
{
    long n = nsites(p);
    for (long s = 0; s < n; s++) {
        double gr[3] = {grad[s], grad[n + s], grad[2 * n + s]};
        double m, t[6];
        chemical_site(p, phi[s], gr, lap[s], &m, t);
        mu[s] = m;
        for (int k = 0; k < 6; k++) pi[k * n + s] = t[k];
    }
}

/* ---- equilibria at one site ------------------------------------------- */

/* Full 3x3 matrix of a symmetric tensor stored xx, xy, xz, yy, yz, zz. */
static void sym_to_full(const double t[6], double m[3][3])
{
    m[0][0] = t[0]; m[0][1] = t[1]; m[0][2] = t[2];
    m[1][0] = t[1]; m[1][1] = t[3]; m[1][2] = t[4];
    m[2][0] = t[2]; m[2][1] = t[4]; m[2][2] = t[5];
}

/* Q_i : M = sum_ab (c_ia c_ib - delta_ab/3) M_ab */
static double q_contract(int i, double m[3][3])
{
    double acc = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            acc += ((double)(CV[i][a] * CV[i][b]) - (a == b ? 1.0 / 3.0 : 0.0)) * m[a][b];
    return acc;
}

void oracle_equilibrium_site(const oracle_params *p, double rho, const double j[3],
                             double phi, double mu, const double pi[6],
                             double *feq /* [19] */, double *geq /* [19] */)
{
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double pim[3][3], mf[3][3], mg[3][3];
    sym_to_full(pi, pim);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            mf[a][b] = pim[a][b] + rho * u[a] * u[b];
            mg[a][b] = (a == b ? p->gamma * mu - phi / 3.0 : 0.0) + phi * u[a] * u[b];
        }
    for (int i = 0; i < NVEL; i++) {
        double cj = CV[i][0] * j[0] + CV[i][1] * j[1] + CV[i][2] * j[2];
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = weight(i) * (rho + 3.0 * cj + 4.5 * q_contract(i, mf));
        geq[i] = weight(i) * (phi + 3.0 * phi * cu + 4.5 * q_contract(i, mg));
    }
}

/* ---- force coupling: F = -div Pi (central differences) ---------------- */

void oracle_force(const oracle_params *p, const double *pi /* [6][N] */, double *F /* [3][N] */)
{
    long n = nsites(p);
    /* component of Pi_ab in the xx, xy, xz, yy, yz, zz storage */
    static const int K[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (long s = 0; s < n; s++) {
        int x, y, z;
        site_coords(p, s, &x, &y, &z);
        long nb[3][2] = {
            {site_index(p, x + 1, y, z), site_index(p, x - 1, y, z)},
            {site_index(p, x, y + 1, z), site_index(p, x, y - 1, z)},
            {site_index(p, x, y, z + 1), site_index(p, x, y, z - 1)},
        };
        for (int a = 0; a < 3; a++) {
            double div = 0.0;
            for (int b = 0; b < 3; b++) {
                const double *t = pi + (long)K[a][b] * n;
                div += 0.5 * (t[nb[b][0]] - t[nb[b][1]]);
            }
            F[a * n + s] = -div;
        }
    }
}

/* Force-coupling equilibria at one site from rho, the velocity u, phi, mu. */
void oracle_equilibrium_force_site(const oracle_params *p, double rho, const double u[3],
                                   double phi, double mu, double *feq, double *geq)
{
    double mf[3][3], mg[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            mf[a][b] = rho * u[a] * u[b];
            mg[a][b] = (a == b ? p->gamma * mu - phi / 3.0 : 0.0) + phi * u[a] * u[b];
        }
    for (int i = 0; i < NVEL; i++) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = weight(i) * (rho + 3.0 * rho * cu + 4.5 * q_contract(i, mf));
        geq[i] = weight(i) * (phi + 3.0 * phi * cu + 4.5 * q_contract(i, mg));
    }
}

/* BGK collision with the forcing term, every site (g and gstar may be
 * NULL: f only). */
void oracle_collide_force(const oracle_params *p, const double *f, const double *g,
                          const double *phi, const double *mu, const double *F,
                          double *fstar, double *gstar)
{
    long n = nsites(p);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < NVEL; i++) {
            double fi = f[i * n + s];
            rho += fi;
            for (int a = 0; a < 3; a++) j[a] += fi * CV[i][a];
        }
        double fv[3] = {F[s], F[n + s], F[2 * n + s]};
        double u[3];
        for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * fv[a]) / rho;
        double feq[NVEL], geq[NVEL];
        oracle_equilibrium_force_site(p, rho, u, phi[s], mu[s], feq, geq);
        double pref = 1.0 - 0.5 / p->tau_f;
        for (int i = 0; i < NVEL; i++) {
            double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
            double src = 0.0;
            for (int a = 0; a < 3; a++) src += (3.0 * (CV[i][a] - u[a]) + 9.0 * cu * CV[i][a]) * fv[a];
            double fi = f[i * n + s];
            fstar[i * n + s] = fi - (fi - feq[i]) / p->tau_f + pref * weight(i) * src;
            if (g) gstar[i * n + s] = g[i * n + s] - (g[i * n + s] - geq[i]) / p->tau_g;
        }
    }
}

/* ---- BGK collision at every site (g and gstar may be NULL: f only) ---- */

void oracle_collide(const oracle_params *p, const double *f, const double *g,
                    const double *phi, const double *mu, const double *pi,
                    double *fstar, double *gstar)
{
    long n = nsites(p);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < NVEL; i++) {
            double fi = f[i * n + s];
            rho += fi;
            for (int a = 0; a < 3; a++) j[a] += fi * CV[i][a];
        }
        double t[6];
        for (int k = 0; k < 6; k++) t[k] = pi[k * n + s];
        double feq[NVEL], geq[NVEL];
        oracle_equilibrium_site(p, rho, j, phi[s], mu[s], t, feq, geq);
        for (int i = 0; i < NVEL; i++) {
            double fi = f[i * n + s];
            fstar[i * n + s] = fi - (fi - feq[i]) / p->tau_f;
            if (g) gstar[i * n + s] = g[i * n + s] - (g[i * n + s] - geq[i]) / p->tau_g;
        }
    }
}

/* ---- propagation: out_i(x + c_i) = in_i(x), periodic ------------------ */

void oracle_stream(const oracle_params *p, const double *in, double *out)
{
    long n = nsites(p);
    for (int i = 0; i < NVEL; i++)
        for (long s = 0; s < n; s++) {
            int x, y, z;
            site_coords(p, s, &x, &y, &z);
            long d = site_index(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
            out[i * n + d] = in[i * n + s];
        }
}

/* ---- one full timestep: post-stream state (f, g) -> next one ---------- */

int oracle_step(const oracle_params *p, const double *f, const double *g,
                double *fnew, double *gnew)
{
    long n = nsites(p);
    double *phi = malloc(sizeof(double) * n);
    double *grad = malloc(sizeof(double) * 3 * n);
    double *lap = malloc(sizeof(double) * n);
    double *mu = malloc(sizeof(double) * n);
    double *pi = malloc(sizeof(double) * 6 * n);
    double *fs = malloc(sizeof(double) * NVEL * n);
    double *gs = malloc(sizeof(double) * NVEL * n);
    if (!phi || !grad || !lap || !mu || !pi || !fs || !gs) {
        free(phi); free(grad); free(lap); free(mu); free(pi); free(fs); free(gs);
        return 1;
    }
    oracle_order_parameter(p, g, phi);
    oracle_gradients(p, phi, grad, lap);
    oracle_chemical(p, phi, grad, lap, mu, pi);
    if (p->coupling == 1) {
        double *F = malloc(sizeof(double) * 3 * n);
        if (!F) {
            free(phi); free(grad); free(lap); free(mu); free(pi); free(fs); free(gs);
            return 1;
        }
        oracle_force(p, pi, F);
        oracle_collide_force(p, f, g, phi, mu, F, fs, gs);
        free(F);
    } else {
        oracle_collide(p, f, g, phi, mu, pi, fs, gs);
    }
    oracle_stream(p, fs, fnew);
    oracle_stream(p, gs, gnew);
    free(phi); free(grad); free(lap); free(mu); free(pi); free(fs); free(gs);
    return 0;
}

/* nsteps timesteps in place on (f, g). */
int oracle_run(const oracle_params *p, double *f, double *g, int nsteps)
{
    long n = nsites(p);
    double *f2 = malloc(sizeof(double) * NVEL * n);
    double *g2 = malloc(sizeof(double) * NVEL * n);
    if (!f2 || !g2) { free(f2); free(g2); return 1; }
    for (int t = 0; t < nsteps; t++) {
        if (oracle_step(p, f, g, f2, g2)) { free(f2); free(g2); return 1; }
        memcpy(f, f2, sizeof(double) * NVEL * n);
        memcpy(g, g2, sizeof(double) * NVEL * n);
    }
    free(f2); free(g2);
    return 0;
}

/* ---- initial state: rho = rho0, u = 0, all of phi0 in the rest g ------ */

void oracle_init(const oracle_params *p, const double *phi0, double *f, double *g)
{
    long n = nsites(p);
    for (int i = 0; i < NVEL; i++)
        for (long s = 0; s < n; s++) {
            f[i * n + s] = weight(i) * p->rho0;
            g[i * n + s] = (i == 0) ? phi0[s] : 0.0;
        }
}

/* ---- hydrodynamic moments of a post-stream state ---------------------- */

/* rho, u, phi.  u = j/rho; in the force coupling u = (j + F/2)/rho, the
 * velocity the collision uses, with F = -div Pi of the state's own phi. */
void oracle_moments(const oracle_params *p, const double *f, const double *g,
                    double *rho, double *u /* [3][N] */, double *phi)
{
    long n = nsites(p);
    double *F = NULL;
    if (p->coupling == 1 && u) {
        double *ph = malloc(sizeof(double) * n), *grad = malloc(sizeof(double) * 3 * n);
        double *lap = malloc(sizeof(double) * n), *mu = malloc(sizeof(double) * n);
        double *pi = malloc(sizeof(double) * 6 * n);
        F = malloc(sizeof(double) * 3 * n);
        if (ph && grad && lap && mu && pi && F) {
            oracle_order_parameter(p, g, ph);
            oracle_gradients(p, ph, grad, lap);
            oracle_chemical(p, ph, grad, lap, mu, pi);
            oracle_force(p, pi, F);
        } else {
            free(F);
            F = NULL;
        }
        free(ph); free(grad); free(lap); free(mu); free(pi);
        if (!F) return; /* out of memory: outputs untouched */
    }
    for (long s = 0; s < n; s++) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0}, ph = 0.0;
        for (int i = 0; i < NVEL; i++) {
            r += f[i * n + s];
            for (int a = 0; a < 3; a++) j[a] += f[i * n + s] * CV[i][a];
            ph += g[i * n + s];
        }
        if (F)
            for (int a = 0; a < 3; a++) j[a] += 0.5 * F[a * n + s];
        if (rho) rho[s] = r;
        if (u) for (int a = 0; a < 3; a++) u[a * n + s] = j[a] / r;
        if (phi) phi[s] = ph;
    }
    free(F);
}

/* ---- finite-difference order parameter ------------------------------- */

/* Initial state: f_i = w_i rho0 (rest), phi = phi0. */
void oracle_fd_init(const oracle_params *p, const double *phi0, double *f, double *phi)
{
    long n = nsites(p);
    for (int i = 0; i < NVEL; i++)
        for (long s = 0; s < n; s++) f[i * n + s] = weight(i) * p->rho0;
    memcpy(phi, phi0, sizeof(double) * n);
}

/* Body force F = -div Pi of a phi field (its gradients, mu and Pi first). */
static int force_of_field(const oracle_params *p, const double *phi, double *F)
{
    long n = nsites(p);
    double *grad = malloc(sizeof(double) * 3 * n), *lap = malloc(sizeof(double) * n);
    double *mu = malloc(sizeof(double) * n), *pi = malloc(sizeof(double) * 6 * n);
    int ok = grad && lap && mu && pi;
    if (ok) {
        oracle_gradients(p, phi, grad, lap);
        oracle_chemical(p, phi, grad, lap, mu, pi);
        oracle_force(p, pi, F);
    }
    free(grad); free(lap); free(mu); free(pi);
    return ok ? 0 : 1;
}

/* rho, u of a post-stream f, and phi copied from the field: u = j/rho, or
 * with the force coupling u = (j + F/2)/rho, F = -div Pi of this phi. */
void oracle_fd_moments(const oracle_params *p, const double *f, const double *phi,
                       double *rho, double *u /* [3][N] */, double *phi_out)
{
    long n = nsites(p);
    double *F = NULL;
    if (p->coupling == 1 && u) {
        F = malloc(sizeof(double) * 3 * n);
        if (!F || force_of_field(p, phi, F)) { free(F); return; }  /* out of memory */
    }
    for (long s = 0; s < n; s++) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < NVEL; i++) {
            r += f[i * n + s];
            for (int a = 0; a < 3; a++) j[a] += f[i * n + s] * CV[i][a];
        }
        if (F) for (int a = 0; a < 3; a++) j[a] += 0.5 * F[a * n + s];
        if (rho) rho[s] = r;
        if (u) for (int a = 0; a < 3; a++) u[a * n + s] = j[a] / r;
        if (phi_out) phi_out[s] = phi[s];
    }
    free(F);
}

/* Flux J_a through the face between x and x + e_a, stored at x: J[3][N]. */
void oracle_fd_fluxes(const oracle_params *p, const double *phi, const double *mu,
                      const double *u /* [3][N] */, double *J /* [3][N] */)
{
    long n = nsites(p);
    double M = p->gamma * (p->tau_g - 0.5);
    for (long s = 0; s < n; s++) {
        int x, y, z;
        site_coords(p, s, &x, &y, &z);
        long nb[3] = {site_index(p, x + 1, y, z), site_index(p, x, y + 1, z),
                      site_index(p, x, y, z + 1)};
        for (int a = 0; a < 3; a++) {
            double uf = 0.5 * (u[a * n + s] + u[a * n + nb[a]]);
            double up = uf > 0.0 ? phi[s] : phi[nb[a]];
            J[a * n + s] = uf * up - M * (mu[nb[a]] - mu[s]);
        }
    }
}

/* phi_new(x) = phi(x) - sum_a [J_a(x) - J_a(x - e_a)] (the flux divergence). */
void oracle_fd_update(const oracle_params *p, const double *phi, const double *J,
                      double *phi_new)
{
    long n = nsites(p);
    for (long s = 0; s < n; s++) {
        int x, y, z;
        site_coords(p, s, &x, &y, &z);
        long nm[3] = {site_index(p, x - 1, y, z), site_index(p, x, y - 1, z),
                      site_index(p, x, y, z - 1)};
        double div = 0.0;
        for (int a = 0; a < 3; a++) div += J[a * n + s] - J[a * n + nm[a]];
        phi_new[s] = phi[s] - div;
    }
}

/* One timestep of the finite-difference scheme: (f, phi) -> (fnew, phinew).
 * Returns 1 on allocation failure. */
int oracle_fd_step(const oracle_params *p, const double *f, const double *phi,
                   double *fnew, double *phinew)
{
    long n = nsites(p);
    double *grad = malloc(sizeof(double) * 3 * n);
    double *lap = malloc(sizeof(double) * n);
    double *mu = malloc(sizeof(double) * n);
    double *pi = malloc(sizeof(double) * 6 * n);
    double *u = malloc(sizeof(double) * 3 * n);
    double *J = malloc(sizeof(double) * 3 * n);
    double *fs = malloc(sizeof(double) * NVEL * n);
    if (!grad || !lap || !mu || !pi || !u || !J || !fs) {
        free(grad); free(lap); free(mu); free(pi); free(u); free(J); free(fs);
        return 1;
    }
    oracle_fd_moments(p, f, phi, NULL, u, NULL);
    oracle_gradients(p, phi, grad, lap);
    oracle_chemical(p, phi, grad, lap, mu, pi);
    if (p->coupling == 1) {
        double *F = malloc(sizeof(double) * 3 * n);
        if (!F) {
            free(grad); free(lap); free(mu); free(pi); free(u); free(J); free(fs);
            return 1;
        }
        oracle_force(p, pi, F);
        oracle_collide_force(p, f, NULL, phi, mu, F, fs, NULL);
        free(F);
    } else {
        oracle_collide(p, f, NULL, phi, mu, pi, fs, NULL);
    }
    oracle_stream(p, fs, fnew);
    oracle_fd_fluxes(p, phi, mu, u, J);
    oracle_fd_update(p, phi, J, phinew);
    free(grad); free(lap); free(mu); free(pi); free(u); free(J); free(fs);
    return 0;
}

/* nsteps timesteps in place on (f, phi). */
int oracle_fd_run(const oracle_params *p, double *f, double *phi, int nsteps)
{
    long n = nsites(p);
    double *f2 = malloc(sizeof(double) * NVEL * n);
    double *p2 = malloc(sizeof(double) * n);
    if (!f2 || !p2) { free(f2); free(p2); return 1; }
    for (int t = 0; t < nsteps; t++) {
        int rc = oracle_fd_step(p, f, phi, f2, p2);
        if (rc) { free(f2); free(p2); return rc; }
        memcpy(f, f2, sizeof(double) * NVEL * n);
        memcpy(phi, p2, sizeof(double) * n);
    }
    free(f2); free(p2);
    return 0;
}

/* ---- FP64 pairwise sum (fixed order) ---------------------------------- */

double oracle_sum(const double *x, long n)
{
    if (n <= 0) return 0.0;
    if (n <= 8) {
        double acc = 0.0;
        for (long k = 0; k < n; k++) acc += x[k];
        return acc;
    }
    long h = n / 2;
    return oracle_sum(x, h) + oracle_sum(x + h, n - h);
}

/* ---- thread count (timing only: every parallel loop is over independent
 * sites, so results do not depend on it) ---------------------------------- */

int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
