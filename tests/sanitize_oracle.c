/* Host sanitizer run of the oracle (test infrastructure): 1D, 2D and 3D grids with CPML, Drude,
 * Lorentz-Bath (per-cell sigma), the learned closure, sources, DFT and energy monitors, stepped
 * and read back through the oracle's C entry points.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer; any report aborts with a nonzero status.  Exit 0 when every call
 * succeeds and every value read back is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void *or_create(int ndim, long nx, long ny, long nz, double courant);
int or_set_boundary(void *g, int axis, int kind, int pml_cells, double R0);
int or_add_drude(void *g, const long *lo, const long *hi, double omega_p, double gamma, double eps_inf);
int or_add_lorentz_bath(void *g, const long *lo, const long *hi, double omega0, double gamma0, double eps_inf,
                        const double *sigma_cells, double sigma, int nb, const double *wj, const double *gj,
                        const double *kj);
int or_add_closure(void *g, const long *lo, const long *hi, double omega0, double gamma0, double eps_inf,
                   const double *sigma_cells, double sigma, double sum_kc, int width, const double *weights,
                   const double *scales);
int or_add_source(void *g, int comp, const long *lo, const long *hi, double omega_c, double width, double amp,
                  const double *profile);
int or_add_dft(void *g, int axis, const long *lo, const long *hi, int nf, const double *omega);
int or_add_energy(void *g, const long *lo, const long *hi, int every);
int or_step(void *g, long nsteps);
int or_get_field(void *g, int comp, double *out);
int or_get_P(void *g, int mi, int c, int level, double *out);
int or_get_Y(void *g, int mi, int c, int level, double *out);
int or_get_hidden(void *g, int mi, int c, double *out);
int or_get_dft(void *g, int id, double *flux, double *raw);
long or_energy_count(void *g, int id);
int or_get_energy(void *g, int id, double *out);
int or_drive_material(void *g, int mi, int c, const double *e_seq, long n, double *p_out);
void or_destroy(void *g);

enum { PML = 0, PERIODIC = 1, CLOSED = 2 };
static int fails = 0;
#define CHECK(x) do { if (!(x)) { fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); fails++; } } while (0)

static void finite(const double *v, long n, const char *what) {
    for (long i = 0; i < n; i++)
        if (!isfinite(v[i])) { fprintf(stderr, "non-finite %s[%ld]\n", what, i); fails++; return; }
}

static double rnd(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) * (1.0 / 16777216.0); }

static void run(int ndim, long nx, long ny, long nz, long steps) {
    const long n = nx * ny * nz;
    void *g = or_create(ndim, nx, ny, nz, 0.5);
    CHECK(g != NULL);
    const int pml = 6;
    for (int a = 0; a < ndim; a++) CHECK(or_set_boundary(g, a, (ndim == 3 && a < 2) ? PERIODIC : PML, pml, 1e-8) == 0);
    const long ax = ndim == 3 ? 2 : 0;            /* the axis the layers stack along */
    const long L = ndim == 3 ? nz : nx;
    long lo[3] = {0, 0, 0}, hi[3] = {nx, ny, nz};
    if (ndim == 2) { lo[1] = pml; hi[1] = ny - pml; }
    /* Drude mirror, Lorentz-Bath slab with per-cell sigma, closure slab */
    lo[ax] = pml + 4; hi[ax] = pml + 7;
    CHECK(or_add_drude(g, lo, hi, 3.0, 0.01, 10.0) == 0);
    long blo[3], bhi[3];
    for (int a = 0; a < 3; a++) { blo[a] = lo[a]; bhi[a] = hi[a]; }
    blo[ax] = pml + 9; bhi[ax] = L / 2;
    long nb_cells = 1;
    for (int a = 0; a < 3; a++) nb_cells *= bhi[a] - blo[a];
    double *sig = malloc(sizeof(double) * nb_cells);
    unsigned seed = 7;
    for (long i = 0; i < nb_cells; i++) sig[i] = 0.01 + 0.09 * rnd(&seed);
    const double wj[5] = {0.9, 0.95, 1.0, 1.05, 1.1}, gj[5] = {0.01, 0.01, 0.01, 0.01, 0.01},
                 kj[5] = {0.03, 0.04, 0.05, 0.04, 0.03};
    CHECK(or_add_lorentz_bath(g, blo, bhi, 1.0, 0.001, 1.2, sig, 0.0, 5, wj, gj, kj) == 0);
    long clo[3], chi[3];
    for (int a = 0; a < 3; a++) { clo[a] = lo[a]; chi[a] = hi[a]; }
    clo[ax] = L / 2 + 2; chi[ax] = L - pml - 6;
    const int width = 8;
    const long nw = width * 7 + width + width * width + width + 5 * width + 5;
    double *w = malloc(sizeof(double) * nw);
    for (long i = 0; i < nw; i++) w[i] = 0.2 * (rnd(&seed) - 0.5);
    const double scales[4] = {1.0, 1.0, 1.0, 1.0};
    CHECK(or_add_closure(g, clo, chi, 1.0, 0.001, 1.0, NULL, 0.05, 0.002, width, w, scales) == 0);
    /* source plane, DFT plane, energy box */
    long slo[3], shi[3];
    for (int a = 0; a < 3; a++) { slo[a] = lo[a]; shi[a] = hi[a]; }
    slo[ax] = pml + 2; shi[ax] = pml + 3;
    CHECK(or_add_source(g, 2 - (ndim == 3 ? 2 : 0), slo, shi, 1.0, 0.5, 1.0, NULL) == 0);
    const double om[16] = {0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6, 1.7, 1.8, 1.9, 2.0};
    long dlo[3], dhi[3];
    for (int a = 0; a < 3; a++) { dlo[a] = lo[a]; dhi[a] = hi[a]; }
    dlo[ax] = L - pml - 3; dhi[ax] = L - pml - 2;
    CHECK(or_add_dft(g, (int)ax, dlo, dhi, 16, om) == 0);
    long elo[3] = {0, 0, 0}, ehi[3] = {nx, ny, nz};
    elo[ax] = pml; ehi[ax] = L - pml;
    if (ndim == 2) { elo[1] = pml; ehi[1] = ny - pml; }
    CHECK(or_add_energy(g, elo, ehi, 3) == 0);
    CHECK(or_step(g, steps) == 0);
    double *f = malloc(sizeof(double) * 9 * n);
    for (int c = 0; c < 9; c++) { CHECK(or_get_field(g, c, f + c * n) == 0); }
    finite(f, 9 * n, "field");
    double *buf = malloc(sizeof(double) * 5 * nb_cells * 4);
    const int c0 = ndim == 3 ? 0 : 2;
    for (int lvl = 0; lvl < 2; lvl++) {
        CHECK(or_get_P(g, 1, c0, lvl, buf) == 0); finite(buf, nb_cells, "P");
        CHECK(or_get_Y(g, 1, c0, lvl, buf) == 0); finite(buf, 5 * nb_cells, "Y");
    }
    CHECK(or_get_hidden(g, 2, c0, buf) == 0);
    double flux[16], raw[16 * 8];
    CHECK(or_get_dft(g, 0, flux, NULL) == 0);
    finite(flux, 16, "flux");
    (void)raw;
    const long ne = or_energy_count(g, 0);
    CHECK(ne == (steps + 2) / 3);
    double *en = malloc(sizeof(double) * 3 * (ne > 0 ? ne : 1));
    CHECK(or_get_energy(g, 0, en) == 0);
    finite(en, 3 * ne, "energy");
    double eseq[64], pout[64];
    for (int i = 0; i < 64; i++) eseq[i] = sin(0.3 * i) * exp(-0.05 * i);
    CHECK(or_drive_material(g, 1, c0, eseq, 64, pout) == 0);
    finite(pout, 64, "driven P");
    free(en); free(buf); free(f); free(w); free(sig);
    or_destroy(g);
}

int main(void) {
    run(1, 120, 1, 1, 400);
    run(2, 48, 40, 1, 150);
    run(3, 4, 6, 60, 80);
    if (fails) { fprintf(stderr, "%d failed checks\n", fails); return 1; }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
