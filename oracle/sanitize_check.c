/*
 * sanitize_check.c -- drives every entry point of the CPU oracle
 * (lb_oracle.c) on small lattices, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (oracle/build.py: build_sanitize_check).
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself.  A clean run (exit 0, no
 * sanitizer report) shows that no oracle loop reads or writes outside its
 * arrays and that no step hits undefined behaviour, on lattices that include
 * extents 1 and 2 (where x - 1 and x + 1 wrap onto one site), both couplings,
 * both order-parameter schemes and tau != 1.  It also checks the global
 * conservation of mass, order parameter and momentum over the run, so that
 * a silent corruption would fail it too.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny, nz;
    double A, B, kappa, gamma, tau_f, tau_g, rho0;
    int32_t coupling;
    int32_t order_param;
} oracle_params;

#define NVEL 19

void oracle_lattice(int32_t *c_out, double *w_out);
void oracle_stream(const oracle_params *p, const double *in, double *out);
int oracle_run(const oracle_params *p, double *f, double *g, int nsteps);
void oracle_init(const oracle_params *p, const double *phi0, double *f, double *g);
void oracle_moments(const oracle_params *p, const double *f, const double *g, double *rho,
                    double *u, double *phi);
void oracle_fd_init(const oracle_params *p, const double *phi0, double *f, double *phi);
void oracle_fd_moments(const oracle_params *p, const double *f, const double *phi, double *rho,
                       double *u, double *phi_out);
int oracle_fd_run(const oracle_params *p, double *f, double *phi, int nsteps);
double oracle_sum(const double *x, long n);
int oracle_set_threads(int n);

static int failures = 0;

static void expect(int ok, const char *what, const oracle_params *p)
{
    if (!ok) {
        fprintf(stderr, "FAIL %s on %d x %d x %d (coupling %d, order_param %d)\n", what, p->nx,
                p->ny, p->nz, p->coupling, p->order_param);
        failures++;
    }
}

/* A deterministic pseudo-random field in (-amp, amp): a 64-bit LCG
 * (Knuth's MMIX constants); the values only need to be irregular. */
static void fill(double *x, long n, uint64_t seed, double amp)
{
    uint64_t s = seed * 2862933555777941757ULL + 3037000493ULL;
    for (long k = 0; k < n; k++) {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        x[k] = amp * (2.0 * (double)(s >> 11) / 9007199254740992.0 - 1.0);
    }
}

/* Sums of rho, phi and j over the lattice from the moments. */
static void totals(long n, const double *rho, const double *u, const double *phi, double t[5])
{
    for (int k = 0; k < 5; k++) t[k] = 0.0;
    for (long s = 0; s < n; s++) {
        t[0] += rho[s];
        t[1] += phi[s];
        for (int a = 0; a < 3; a++) t[2 + a] += rho[s] * u[a * n + s];
    }
}

static void run_case(int nx, int ny, int nz, int coupling, int order_param)
{
    oracle_params p = {nx, ny, nz, -0.00625, 0.00625, 0.004, 0.5, 0.8, 1.3, 1.0, coupling,
                       order_param};
    const long n = (long)nx * ny * nz;
    double *phi0 = malloc(sizeof(double) * n), *f = malloc(sizeof(double) * NVEL * n);
    double *g = malloc(sizeof(double) * NVEL * n), *phi = malloc(sizeof(double) * n);
    double *rho = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * 3 * n);
    double *ph = malloc(sizeof(double) * n);
    if (!phi0 || !f || !g || !phi || !rho || !u || !ph) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    fill(phi0, n, (uint64_t)(nx * 131 + ny * 17 + nz + 7 * coupling + 3 * order_param), 0.3);
    double t0[5], t1[5];
    if (order_param == 0) {
        oracle_init(&p, phi0, f, g);
        oracle_moments(&p, f, g, rho, u, ph);
        totals(n, rho, u, ph, t0);
        expect(oracle_run(&p, f, g, 6) == 0, "oracle_run", &p);
        oracle_moments(&p, f, g, rho, u, ph);
    } else {
        oracle_fd_init(&p, phi0, f, phi);
        oracle_fd_moments(&p, f, phi, rho, u, ph);
        totals(n, rho, u, ph, t0);
        expect(oracle_fd_run(&p, f, phi, 6) == 0, "oracle_fd_run", &p);
        oracle_fd_moments(&p, f, phi, rho, u, ph);
    }
    totals(n, rho, u, ph, t1);
    /* mass and order parameter exactly conserved up to rounding; the
     * momentum of rho u (u includes F/2 in the force coupling, whose sum
     * over a periodic lattice is zero) likewise */
    const double tol = 1e-11 * (double)n;
    for (int k = 0; k < 5; k++) expect(fabs(t1[k] - t0[k]) <= tol, "conservation", &p);
    /* propagation: L_x steps along every direction return the input */
    fill(f, NVEL * n, 99u + (uint64_t)n, 1.0);
    double *a = malloc(sizeof(double) * NVEL * n), *b = malloc(sizeof(double) * NVEL * n);
    if (!a || !b) exit(2);
    for (long k = 0; k < NVEL * n; k++) a[k] = f[k];
    const int period = nx * ny * nz; /* a multiple of every extent */
    for (int t = 0; t < period && t < 64; t++) {
        oracle_stream(&p, a, b);
        for (long k = 0; k < NVEL * n; k++) a[k] = b[k];
    }
    if (period <= 64)
        for (long k = 0; k < NVEL * n; k++) expect(a[k] == f[k], "stream period", &p);
    expect(isfinite(oracle_sum(f, NVEL * n)), "oracle_sum", &p);
    free(a); free(b);
    free(phi0); free(f); free(g); free(phi); free(rho); free(u); free(ph);
}

int main(void)
{
    int32_t c[NVEL * 3];
    double w[NVEL];
    oracle_lattice(c, w);
    const int shapes[][3] = {{1, 1, 1}, {1, 2, 3}, {2, 2, 2}, {3, 1, 2}, {4, 3, 5}, {6, 5, 7}};
    for (int threads = 1; threads <= 4; threads += 3) {
        oracle_set_threads(threads);
        for (unsigned k = 0; k < sizeof shapes / sizeof shapes[0]; k++)
            for (int coupling = 0; coupling < 2; coupling++)
                for (int op = 0; op < 2; op++)
                    run_case(shapes[k][0], shapes[k][1], shapes[k][2], coupling, op);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitize check ok\n");
    return 0;
}
