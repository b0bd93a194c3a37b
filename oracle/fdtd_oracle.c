/*
 * FDTD-Bath oracle: a plain, slow FP64 reference of the time step of
 * "FDTD with Auxiliary Bath Fields for Condensed-Phase Polaritonics"
 * (T. E. Li, arXiv 2505.23963).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file.  It shares no code,
 * header, table or helper with the GPU library; the two meet only through
 * the seeded workload descriptions.
 *
 * What it computes, step n -> n+1 (units c = eps0 = mu0 = 1, dx = 1):
 *   1. D^{n+1/2} = D^{n-1/2} + dt [curl H^n - J(t_n)]   (Maxwell curl law for D,
 *      Sec. II; the D line of the 1D loop eq:FDTD-1D), CPML terms added where
 *      the axis is absorbing.
 *   2. E^{n+1/2} = (D^{n+1/2} - P^{n+1/2}) / eps_inf    (D = eps_inf E + P; the
 *      paper writes eps0, eps_inf is the background permittivity).
 *   3. P^{n+3/2} from the three-level recurrences: Lorentz eq:Pz_1D_Lorentz,
 *      Drude (omega0^2 removed from the P^n coefficient, Sec. II.A), and the
 *      Lorentz-Bath update eq:Pz_update-LB followed by the bath update
 *      eq:Yzj_finite_difference, one independent bath per E component (end
 *      of Sec. II.C).
 *   4. H^{n+1} = H^n - dt curl E^{n+1/2}                (dB/dt = -curl E of
 *      Sec. II; the printed 1D H line carries the opposite sign, which makes
 *      the scheme ill-posed, so the curl law is followed).
 *   5. monitors: DFT of the plane fields, and the exact discrete energy.
 *
 * Two extensions of the bath that the paper names as next steps (Sec. V) but
 * does not write out, taken here in their textbook form:
 *   * thermal bath: every damped coordinate (P with gamma0, each Y_j with
 *     gamma_j) gets the Langevin force that the fluctuation-dissipation
 *     relation pairs with its damping, for the effective mass rho =
 *     1/(eps0 sigma omega0^2) of eq:H_full: <eta(t) eta(t')> = (2 gamma kT /
 *     rho) delta(t - t').  Over one step the force is the step average of
 *     white noise, sqrt(2 gamma kT / (rho dt)) xi, with xi independent, of
 *     mean zero and unit variance: xi = sqrt(12) (u - 1/2), u uniform from
 *     the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     SC'11), counter (cell, step, component, variate / 4), key the seed,
 *     variate j for bath mode j and variate N_b for P.  Every second moment
 *     (energies, spectra, equipartition) is that of Gaussian noise.
 *   * anharmonic bath: a quartic term (rho/4) lambda_j Y_j^4 in each mode's
 *     potential, i.e. + lambda_j Y_j^3 on the left of eq:EOM_LorentzBath-2,
 *     taken at level n like omega_j^2 Y_j.
 * Both enter eq:Yzj_finite_difference as one more term f_j = dt^2 (eta_j -
 * lambda_j (Y_j^n)^3) / (1 + gamma_j dt / 2), and, through the substitution
 * of Y_j^{n+1} that gives eq:Pz_update-LB, the P update as - (dt/2) sum_j
 * k_j f_j and + dt^2 eta_P in its bracket.
 *
 * Yee placement, cell (i,j,k), z fastest in memory:
 *   Ex (i+1/2,j,k)  Ey (i,j+1/2,k)  Ez (i,j,k+1/2)
 *   Hx (i,j+1/2,k+1/2)  Hy (i+1/2,j,k+1/2)  Hz (i+1/2,j+1/2,k)
 * A 1D grid runs along x with (Ez, Hy) as in the paper's 1D loop; a 2D grid
 * is the x-y plane with (Ez, Hx, Hy).  Unused axes have extent 1 and are
 * treated as periodic, so every difference along them vanishes.
 *
 * The cell loops of each update run in parallel over the two outer axes
 * (OpenMP, when built with it); every cell's arithmetic is the same as in a serial loop, so the
 * result does not depend on the thread count.  Monitor sums stay serial.
 *
 * Boundaries per axis: periodic (wrap), closed (field values beyond the
 * grid read as zero), or CPML (closed, with a graded absorbing layer).
 *
 * Bloch-periodic axes (the boundary condition the paper applies along y in
 * its 2D runs, Appendix "Simulation details", here with any phase): the
 * field is complex and obeys f(r + L e_a) = exp(i phi_a) f(r), phi_a = k_a L.
 * Every update has real coefficients, so the real and imaginary parts are
 * two real grids of identical set-up (or_pair_bloch) that meet only where a
 * neighbour read crosses a Bloch axis: there part p of exp(+-i phi) (R + i I)
 * is read.  Sources of the imaginary part carry the imaginary part of a
 * complex profile; the flux is Re sum (E~ x conj H~) of the complex DFTs.
 * CPML is the convolutional PML of Roden and Gedney (2000) with kappa = 1,
 * alpha = 0: psi <- b psi + (b - 1) dF, b = exp(-s dt), and the derivative dF
 * is replaced by dF + psi.  The grading is s(d) = s_max (d/L)^3 with
 * s_max = -4 ln(R0) / (2L), d the depth into the layer: E-type nodes sit at
 * integer positions, H-type nodes half a cell further.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { K_DIELECTRIC = 0, K_DRUDE = 1, K_LORENTZ = 2, K_BATH = 3, K_CLOSURE = 4, K_MULTI = 5 };
enum { POLE_LORENTZ = 0, POLE_DRUDE = 1 };
#define MAXPOLE 8
enum { BC_PML = 0, BC_PERIODIC = 1, BC_CLOSED = 2 };

#define MAXMAT 256
#define MAXSRC 16
#define MAXMON 16

typedef struct {
    int kind;
    long lo[3], hi[3], bn[3], ncell;
    double eps_inf, omega0, gamma0;   /* Drude: omega0 holds omega_p, gamma0 holds gamma */
    double *sigma;                    /* per cell of the box */
    int nb;
    double *wj, *gj, *kj;             /* bath frequencies, dampings, couplings */
    double *P[3][2];                  /* [E comp][0: level n+1/2, 1: level n-1/2] */
    double *Y[3][2];                  /* [E comp][level], nb * ncell each */
    /* learned closure */
    int width;
    double *W1, *b1, *W2, *b2, *W3, *b3;
    double scale[4];                  /* s_E, s_P, s_V, s_S */
    double sum_kc;                    /* sum_j k_j c_j kept from the explicit bath */
    double *hid[3];                   /* 4 * ncell per E comp */
    /* sum of Lorentz / Drude terms: P = sum_p P_p, P[c][level] holds np * ncell values (pole-major) */
    int np;
    int pkind[MAXPOLE];
    double pw[MAXPOLE], pg[MAXPOLE], ps[MAXPOLE];   /* omega0 (Drude: omega_p), gamma, sigma */
    /* thermal / anharmonic bath (Sec. V extensions): kT (0: none), Philox key, quartic coefficients */
    double kT;
    uint32_t key[2];
    double *lam;                      /* nb values, or NULL */
    long nupd;                        /* updates taken so far: the step index n of the noise */
} Mat;

typedef struct {
    int comp;
    long lo[3], hi[3];
    double omega_c, width, amp;
    double *profile;                  /* per cell of the box */
} Src;

typedef struct {
    int axis;
    long lo[3], hi[3];
    long npts;
    int nf;
    double *omega;
    double *acc;                      /* [4 fields][npts][nf][re,im]: E_t1, E_t2, H_t1, H_t2 */
} Dft;

typedef struct {
    long lo[3], hi[3];
    int every;
    long nsamp, cap;
    double *out;                      /* [sample][field, P, bath] */
} Energy;

typedef struct Grid {
    int ndim;
    long n[3], ncell;
    double dt;
    int bc[3], pml[3];
    double R0;
    int activeE[3], activeH[3];
    double *E[3], *Eprev[3], *D[3], *H[3];
    double *eps;                      /* eps_inf per cell */
    int *mat;                         /* material index per cell, -1 none */
    long *moff;                       /* cell offset inside its material box */
    double *sE[3], *sH[3];            /* CPML conductivity per axis, E- and H-type nodes */
    double *psiE[3][3], *psiH[3][3];  /* [component][derivative axis] */
    long step;
    /* Bloch pair: the other part's grid, this grid's part (0 real, 1 imaginary), phase per axis */
    struct Grid *twin;
    int part;
    double bph[3];
    int nmat, nsrc, ndft, nen;
    Mat m[MAXMAT];
    Src s[MAXSRC];
    Dft d[MAXMON];
    Energy e[MAXMON];
} Grid;

static long IDX(const Grid *g, long i, long j, long k) { return (i * g->n[1] + j) * g->n[2] + k; }

enum { F_E = 0, F_H = 1 };
static const double *field_of(const Grid *g, int F, int c) { return F == F_E ? g->E[c] : g->H[c]; }

/* value of field F (E or H), component c, at (i,j,k) with the boundary rule of each axis.  On a Bloch
 * pair a read past the upper (lower) end of a periodic axis a picks up exp(+i phi_a) (exp(-i phi_a)):
 * with the own part v and the other part w, part 0 reads Re(e^{i t}(v + i w)) = cos t v - sin t w and
 * part 1 reads Im(e^{i t}(w + i v)) = cos t v + sin t w. */
static double at(const Grid *g, int F, int comp, long i, long j, long k) {
    const double *f = field_of(g, F, comp);
    long c[3] = {i, j, k};
    double t = 0.0;
    for (int a = 0; a < 3; a++) {
        if (c[a] < 0 || c[a] >= g->n[a]) {
            if (g->bc[a] != BC_PERIODIC) return 0.0;
            t += (c[a] < 0 ? -1.0 : 1.0) * g->bph[a];
            c[a] = (c[a] % g->n[a] + g->n[a]) % g->n[a];
        }
    }
    long q = IDX(g, c[0], c[1], c[2]);
    if (!g->twin || t == 0.0) return f[q];
    double w = field_of(g->twin, F, comp)[q];
    return g->part == 0 ? cos(t) * f[q] - sin(t) * w : cos(t) * f[q] + sin(t) * w;
}

static double *zalloc(long n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static double pml_sigma(const Grid *g, int a, double pos) {
    /* conductivity at coordinate pos (cells) along axis a */
    if (g->bc[a] != BC_PML) return 0.0;
    double L = (double)g->pml[a];
    double smax = -4.0 * log(g->R0) / (2.0 * L);
    double d = 0.0;
    if (pos < L) d = L - pos;
    else if (pos > (double)(g->n[a] - 1) - L) d = pos - ((double)(g->n[a] - 1) - L);
    if (d <= 0.0) return 0.0;
    double r = d / L;
    return smax * r * r * r;
}

void *or_create(int ndim, long nx, long ny, long nz, double courant) {
    if (ndim < 1 || ndim > 3) return NULL;
    Grid *g = (Grid *)calloc(1, sizeof(Grid));
    g->ndim = ndim;
    g->n[0] = nx; g->n[1] = ndim >= 2 ? ny : 1; g->n[2] = ndim >= 3 ? nz : 1;
    g->ncell = g->n[0] * g->n[1] * g->n[2];
    g->dt = courant;  /* dx = 1 */
    g->R0 = 1e-8;
    for (int a = 0; a < 3; a++) { g->bc[a] = BC_PERIODIC; g->pml[a] = 0; }
    if (ndim == 1) { g->activeE[2] = 1; g->activeH[1] = 1; }
    else if (ndim == 2) { g->activeE[2] = 1; g->activeH[0] = 1; g->activeH[1] = 1; }
    else for (int c = 0; c < 3; c++) { g->activeE[c] = 1; g->activeH[c] = 1; }
    for (int c = 0; c < 3; c++) {
        if (g->activeE[c]) { g->E[c] = zalloc(g->ncell); g->Eprev[c] = zalloc(g->ncell); g->D[c] = zalloc(g->ncell); }
        if (g->activeH[c]) g->H[c] = zalloc(g->ncell);
    }
    g->eps = zalloc(g->ncell);
    for (long q = 0; q < g->ncell; q++) g->eps[q] = 1.0;
    g->mat = (int *)malloc(sizeof(int) * (size_t)g->ncell);
    g->moff = (long *)malloc(sizeof(long) * (size_t)g->ncell);
    for (long q = 0; q < g->ncell; q++) { g->mat[q] = -1; g->moff[q] = 0; }
    return g;
}

int or_set_boundary(void *gp, int axis, int kind, int pml_cells, double R0) {
    Grid *g = (Grid *)gp;
    if (axis < 0 || axis >= g->ndim) return -1;
    g->bc[axis] = kind;
    g->pml[axis] = pml_cells;
    if (R0 > 0) g->R0 = R0;
    return 0;
}

/* CPML arrays are built once, before the first step */
static void build_pml(Grid *g) {
    for (int a = 0; a < 3; a++) {
        if (g->bc[a] != BC_PML || g->sE[a]) continue;
        g->sE[a] = zalloc(g->n[a]);
        g->sH[a] = zalloc(g->n[a]);
        for (long p = 0; p < g->n[a]; p++) {
            g->sE[a][p] = pml_sigma(g, a, (double)p);
            g->sH[a][p] = pml_sigma(g, a, (double)p + 0.5);
        }
        for (int c = 0; c < 3; c++) {
            if (c == a) continue;
            if (g->activeE[c]) g->psiE[c][a] = zalloc(g->ncell);
            if (g->activeH[c]) g->psiH[c][a] = zalloc(g->ncell);
        }
    }
}

static int box_ok(const Grid *g, const long *lo, const long *hi) {
    for (int a = 0; a < 3; a++)
        if (lo[a] < 0 || hi[a] > g->n[a] || lo[a] >= hi[a]) return 0;
    return 1;
}

static Mat *new_mat(Grid *g, int kind, const long *lo, const long *hi) {
    if (g->nmat >= MAXMAT || !box_ok(g, lo, hi)) return NULL;
    Mat *m = &g->m[g->nmat];
    memset(m, 0, sizeof(Mat));
    m->kind = kind;
    m->ncell = 1;
    for (int a = 0; a < 3; a++) { m->lo[a] = lo[a]; m->hi[a] = hi[a]; m->bn[a] = hi[a] - lo[a]; m->ncell *= m->bn[a]; }
    long q = 0;
    for (long i = lo[0]; i < hi[0]; i++)
        for (long j = lo[1]; j < hi[1]; j++)
            for (long k = lo[2]; k < hi[2]; k++, q++) {
                g->mat[IDX(g, i, j, k)] = g->nmat;
                g->moff[IDX(g, i, j, k)] = q;
            }
    g->nmat++;
    return m;
}

static void set_eps(Grid *g, const Mat *m, double eps_inf) {
    for (long i = m->lo[0]; i < m->hi[0]; i++)
        for (long j = m->lo[1]; j < m->hi[1]; j++)
            for (long k = m->lo[2]; k < m->hi[2]; k++) g->eps[IDX(g, i, j, k)] = eps_inf;
}

static void alloc_P(Grid *g, Mat *m) {
    for (int c = 0; c < 3; c++)
        if (g->activeE[c]) { m->P[c][0] = zalloc(m->ncell); m->P[c][1] = zalloc(m->ncell); }
}

int or_add_dielectric(void *gp, const long *lo, const long *hi, double eps_inf) {
    Grid *g = (Grid *)gp;
    Mat *m = new_mat(g, K_DIELECTRIC, lo, hi);
    if (!m) return -1;
    m->eps_inf = eps_inf;
    set_eps(g, m, eps_inf);
    return 0;
}

int or_add_drude(void *gp, const long *lo, const long *hi, double omega_p, double gamma, double eps_inf) {
    Grid *g = (Grid *)gp;
    Mat *m = new_mat(g, K_DRUDE, lo, hi);
    if (!m) return -1;
    m->eps_inf = eps_inf; m->omega0 = omega_p; m->gamma0 = gamma;
    set_eps(g, m, eps_inf);
    alloc_P(g, m);
    return 0;
}

static Mat *add_lorentz_common(Grid *g, int kind, const long *lo, const long *hi, double omega0, double gamma0,
                               double eps_inf, const double *sigma_cells, double sigma) {
    Mat *m = new_mat(g, kind, lo, hi);
    if (!m) return NULL;
    m->eps_inf = eps_inf; m->omega0 = omega0; m->gamma0 = gamma0;
    set_eps(g, m, eps_inf);
    m->sigma = zalloc(m->ncell);
    for (long q = 0; q < m->ncell; q++) m->sigma[q] = sigma_cells ? sigma_cells[q] : sigma;
    alloc_P(g, m);
    return m;
}

/* nb == 0 gives the plain Lorentz medium, updated by eq:Pz_1D_Lorentz */
int or_add_lorentz_bath(void *gp, const long *lo, const long *hi, double omega0, double gamma0, double eps_inf,
                        const double *sigma_cells, double sigma, int nb, const double *wj, const double *gj,
                        const double *kj) {
    Grid *g = (Grid *)gp;
    Mat *m = add_lorentz_common(g, nb > 0 ? K_BATH : K_LORENTZ, lo, hi, omega0, gamma0, eps_inf, sigma_cells, sigma);
    if (!m) return -1;
    m->nb = nb;
    if (nb > 0) {
        m->wj = zalloc(nb); m->gj = zalloc(nb); m->kj = zalloc(nb);
        memcpy(m->wj, wj, sizeof(double) * (size_t)nb);
        memcpy(m->gj, gj, sizeof(double) * (size_t)nb);
        memcpy(m->kj, kj, sizeof(double) * (size_t)nb);
        for (int c = 0; c < 3; c++)
            if (g->activeE[c]) { m->Y[c][0] = zalloc(nb * m->ncell); m->Y[c][1] = zalloc(nb * m->ncell); }
    }
    return 0;
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds on a 4 x 32-bit counter; a round
 * multiplies counter words 0 and 2 by two fixed constants (full 64-bit products), the new counter is
 * (hi(word 2 product) ^ word 1 ^ key 0, lo(word 2 product), hi(word 0 product) ^ word 3 ^ key 1,
 * lo(word 0 product)), and the key is bumped by two Weyl constants before every round but the first. */
void or_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* the unit-variance variate v of cell q, step n, component c: sqrt(12) (u - 1/2) with
 * u = (x + 1/2) / 2^32 and x lane v % 4 of Philox(counter (q, n, c, v / 4), key) */
static double thermal_variate(const Mat *m, long q, long n, int c, int v) {
    uint32_t ctr[4] = {(uint32_t)q, (uint32_t)n, (uint32_t)c, (uint32_t)(v / 4)}, x[4];
    or_philox(ctr, m->key, x);
    double u = ((double)x[v % 4] + 0.5) * (1.0 / 4294967296.0);
    return (u - 0.5) * 3.4641016151377544;   /* sqrt(12) rounded to double */
}

/* thermal bath of Lorentz-Bath material mi at temperature kT (energy units, >= 0) with the 64-bit
 * seed of its noise (key: low word, high word) */
int or_set_bath_thermal(void *gp, int mi, double kT, uint64_t seed) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || g->m[mi].kind != K_BATH || !(kT >= 0.0) || g->twin) return -1;
    Mat *m = &g->m[mi];
    m->kT = kT;
    m->key[0] = (uint32_t)seed;
    m->key[1] = (uint32_t)(seed >> 32);
    return 0;
}

/* quartic coefficients lambda_j (one per bath mode) of material mi */
int or_set_bath_anharmonic(void *gp, int mi, const double *lam) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || g->m[mi].kind != K_BATH || g->twin) return -1;
    Mat *m = &g->m[mi];
    if (!m->lam) m->lam = zalloc(m->nb);
    memcpy(m->lam, lam, sizeof(double) * (size_t)m->nb);
    return 0;
}

/* Sum of Lorentz and Drude terms in one box (Sec. II.A: realistic susceptibilities are fitted by
 * several such terms): kinds[p] 0 = Lorentz (omega0, gamma, sigma), 1 = Drude (omega_p, gamma); the
 * terms are independent oscillators driven by the same E, and D = eps_inf E + sum_p P_p. */
int or_add_multipole(void *gp, const long *lo, const long *hi, double eps_inf, int np, const int *kinds,
                     const double *omega, const double *gamma, const double *sigma) {
    Grid *g = (Grid *)gp;
    if (np < 1 || np > MAXPOLE) return -1;
    Mat *m = new_mat(g, K_MULTI, lo, hi);
    if (!m) return -1;
    m->eps_inf = eps_inf;
    set_eps(g, m, eps_inf);
    m->np = np;
    for (int pp = 0; pp < np; pp++) {
        m->pkind[pp] = kinds[pp];
        m->pw[pp] = omega[pp];
        m->pg[pp] = gamma[pp];
        m->ps[pp] = kinds[pp] == POLE_DRUDE ? 1.0 : sigma[pp];
    }
    for (int c = 0; c < 3; c++)
        if (g->activeE[c]) { m->P[c][0] = zalloc(np * m->ncell); m->P[c][1] = zalloc(np * m->ncell); }
    return 0;
}

/* Learned bath closure: the bath force term of eq:Pz_update-LB is produced by a
 * recurrent network with 4 hidden states per component-cell.  weights holds
 * W1[width][7], b1[width], W2[width][width], b2[width], W3[5][width], b3[5]
 * (row-major); scales = {s_E, s_P, s_V, s_S}. */
int or_add_closure(void *gp, const long *lo, const long *hi, double omega0, double gamma0, double eps_inf,
                   const double *sigma_cells, double sigma, double sum_kc, int width, const double *weights,
                   const double *scales) {
    Grid *g = (Grid *)gp;
    if (width < 1 || width > 256) return -1;
    Mat *m = add_lorentz_common(g, K_CLOSURE, lo, hi, omega0, gamma0, eps_inf, sigma_cells, sigma);
    if (!m) return -1;
    m->width = width;
    m->sum_kc = sum_kc;
    long nw = (long)width * 7 + width + (long)width * width + width + 5L * width + 5;
    double *w = zalloc(nw);
    memcpy(w, weights, sizeof(double) * (size_t)nw);
    m->W1 = w; m->b1 = m->W1 + width * 7; m->W2 = m->b1 + width; m->b2 = m->W2 + width * width;
    m->W3 = m->b2 + width; m->b3 = m->W3 + 5 * width;
    for (int q = 0; q < 4; q++) m->scale[q] = scales[q];
    for (int c = 0; c < 3; c++)
        if (g->activeE[c]) m->hid[c] = zalloc(4 * m->ncell);
    return 0;
}

int or_add_source(void *gp, int comp, const long *lo, const long *hi, double omega_c, double width, double amp,
                  const double *profile) {
    Grid *g = (Grid *)gp;
    if (g->nsrc >= MAXSRC || !box_ok(g, lo, hi) || comp < 0 || comp > 2 || !g->activeE[comp]) return -1;
    Src *s = &g->s[g->nsrc];
    s->comp = comp; s->omega_c = omega_c; s->width = width; s->amp = amp;
    long nc = 1;
    for (int a = 0; a < 3; a++) { s->lo[a] = lo[a]; s->hi[a] = hi[a]; nc *= hi[a] - lo[a]; }
    s->profile = zalloc(nc);
    for (long q = 0; q < nc; q++) s->profile[q] = profile ? profile[q] : 1.0;
    return g->nsrc++;
}

/* soft current: J(t) = A exp(-(t-t0)^2 / (2 tau^2)) cos(w_c (t - t0)), tau = 1/width, t0 = 5 tau, off after 2 t0 */
static double pulse(const Src *s, double t) {
    double tau = 1.0 / s->width, t0 = 5.0 * tau;
    if (t > 2.0 * t0) return 0.0;
    double u = t - t0;
    return s->amp * exp(-u * u / (2.0 * tau * tau)) * cos(s->omega_c * u);
}

int or_add_dft(void *gp, int axis, const long *lo, const long *hi, int nf, const double *omega) {
    Grid *g = (Grid *)gp;
    if (g->ndft >= MAXMON || !box_ok(g, lo, hi) || axis < 0 || axis >= g->ndim || hi[axis] - lo[axis] != 1) return -1;
    Dft *d = &g->d[g->ndft];
    d->axis = axis; d->nf = nf;
    d->npts = 1;
    for (int a = 0; a < 3; a++) { d->lo[a] = lo[a]; d->hi[a] = hi[a]; d->npts *= hi[a] - lo[a]; }
    d->omega = zalloc(nf);
    memcpy(d->omega, omega, sizeof(double) * (size_t)nf);
    d->acc = zalloc(4 * d->npts * nf * 2);
    return g->ndft++;
}

int or_add_energy(void *gp, const long *lo, const long *hi, int every) {
    Grid *g = (Grid *)gp;
    if (g->nen >= MAXMON || !box_ok(g, lo, hi) || every < 1) return -1;
    Energy *e = &g->e[g->nen];
    for (int a = 0; a < 3; a++) { e->lo[a] = lo[a]; e->hi[a] = hi[a]; }
    e->every = every; e->nsamp = 0; e->cap = 1024;
    e->out = zalloc(3 * e->cap);
    return g->nen++;
}

/* ---------- the curl terms ---------- */

/* For component c the curl is  d_{a1} F_{f1} - d_{a2} F_{f2}  with (c, a1, a2) cyclic. */
static const int CYC[3][2] = {{1, 2}, {2, 0}, {0, 1}};

/* backward difference of H_comp along axis a at cell (i,j,k): H(cell) - H(cell - e_a) */
static double dH(const Grid *g, int comp, int a, long i, long j, long k) {
    if (!g->H[comp]) return 0.0;
    long c[3] = {i, j, k};
    c[a] -= 1;
    return at(g, F_H, comp, i, j, k) - at(g, F_H, comp, c[0], c[1], c[2]);
}

/* forward difference of E_comp along axis a: E(cell + e_a) - E(cell) */
static double dE(const Grid *g, int comp, int a, long i, long j, long k) {
    if (!g->E[comp]) return 0.0;
    long c[3] = {i, j, k};
    c[a] += 1;
    return at(g, F_E, comp, c[0], c[1], c[2]) - at(g, F_E, comp, i, j, k);
}

static void update_D(Grid *g) {
    double dt = g->dt, tn = (double)g->step * dt;
    for (int c = 0; c < 3; c++) {
        if (!g->activeE[c]) continue;
        int a1 = CYC[c][0], a2 = CYC[c][1];
        /* (curl H)_c = d_{a1} H_{a2} - d_{a2} H_{a1} */
#pragma omp parallel for collapse(2) schedule(static)
        for (long i = 0; i < g->n[0]; i++)
            for (long j = 0; j < g->n[1]; j++)
                for (long k = 0; k < g->n[2]; k++) {
                    long q = IDX(g, i, j, k), pos[3] = {i, j, k};
                    double t1 = dH(g, a2, a1, i, j, k);
                    double t2 = dH(g, a1, a2, i, j, k);
                    if (g->psiE[c][a1]) {
                        double b = exp(-g->sE[a1][pos[a1]] * dt);
                        g->psiE[c][a1][q] = b * g->psiE[c][a1][q] + (b - 1.0) * t1;
                        t1 += g->psiE[c][a1][q];
                    }
                    if (g->psiE[c][a2]) {
                        double b = exp(-g->sE[a2][pos[a2]] * dt);
                        g->psiE[c][a2][q] = b * g->psiE[c][a2][q] + (b - 1.0) * t2;
                        t2 += g->psiE[c][a2][q];
                    }
                    g->D[c][q] += dt * (t1 - t2);
                }
    }
    for (int s = 0; s < g->nsrc; s++) {
        Src *src = &g->s[s];
        double J = pulse(src, tn);
        long q = 0;
        for (long i = src->lo[0]; i < src->hi[0]; i++)
            for (long j = src->lo[1]; j < src->hi[1]; j++)
                for (long k = src->lo[2]; k < src->hi[2]; k++, q++)
                    g->D[src->comp][IDX(g, i, j, k)] -= dt * J * src->profile[q];
    }
}

static void update_E(Grid *g) {
    for (int c = 0; c < 3; c++) {
        if (!g->activeE[c]) continue;
        memcpy(g->Eprev[c], g->E[c], sizeof(double) * (size_t)g->ncell);
#pragma omp parallel for schedule(static)
        for (long q = 0; q < g->ncell; q++) {
            double P = 0.0;
            int mi = g->mat[q];
            if (mi >= 0 && g->m[mi].kind == K_MULTI) {
                const Mat *m = &g->m[mi];
                for (int pp = 0; pp < m->np; pp++) P += m->P[c][0][pp * m->ncell + g->moff[q]];
            } else if (mi >= 0 && g->m[mi].P[c][0]) {
                P = g->m[mi].P[c][0][g->moff[q]];
            }
            g->E[c][q] = (g->D[c][q] - P) / g->eps[q];
        }
    }
}

static double tanh_(double x) { return tanh(x); }

/* advance P (and the bath) of one material from level n+1/2 to n+3/2 */
static void update_material(Grid *g, Mat *m) {
    double dt = g->dt, dt2 = dt * dt;
    if (m->kind == K_DIELECTRIC) return;
    if (m->kind == K_MULTI) {
        /* each term follows its own central-difference update: eq:Pz_1D_Lorentz for a Lorentz term, the
         * same with omega0^2 dropped from the P^n coefficient for a Drude term (Sec. II.A) */
        for (int c = 0; c < 3; c++) {
            if (!g->activeE[c]) continue;
#pragma omp parallel for collapse(2) schedule(static)
            for (long i = m->lo[0]; i < m->hi[0]; i++)
                for (long j = m->lo[1]; j < m->hi[1]; j++)
                    for (long k = m->lo[2]; k < m->hi[2]; k++) {
                        long q = ((i - m->lo[0]) * m->bn[1] + (j - m->lo[1])) * m->bn[2] + (k - m->lo[2]);
                        double E = g->E[c][IDX(g, i, j, k)];
                        for (int pp = 0; pp < m->np; pp++) {
                            double *Pn = &m->P[c][0][pp * m->ncell + q], *Pm = &m->P[c][1][pp * m->ncell + q];
                            double w2 = m->pw[pp] * m->pw[pp], gam = m->pg[pp];
                            double A = 1.0 + 0.5 * gam * dt, Pnew;
                            if (m->pkind[pp] == POLE_DRUDE)
                                Pnew = (w2 * dt2 * E + 2.0 * (*Pn) - (1.0 - 0.5 * gam * dt) * (*Pm)) / A;
                            else
                                Pnew = (w2 * dt2 * m->ps[pp] * E - (w2 * dt2 - 2.0) * (*Pn) - (1.0 - 0.5 * gam * dt) * (*Pm)) / A;
                            *Pm = *Pn;
                            *Pn = Pnew;
                        }
                    }
        }
        return;
    }
    for (int c = 0; c < 3; c++) {
        if (!g->activeE[c]) continue;
        double *Pn = m->P[c][0], *Pm = m->P[c][1];
#pragma omp parallel for collapse(2) schedule(static)
        for (long i = m->lo[0]; i < m->hi[0]; i++)
            for (long j = m->lo[1]; j < m->hi[1]; j++)
                for (long k = m->lo[2]; k < m->hi[2]; k++) {
                    long q = ((i - m->lo[0]) * m->bn[1] + (j - m->lo[1])) * m->bn[2] + (k - m->lo[2]);
                    double E = g->E[c][IDX(g, i, j, k)];
                    double Pnew;
                    if (m->kind == K_DRUDE) {
                        double wp2 = m->omega0 * m->omega0, gam = m->gamma0;
                        Pnew = (wp2 * dt2 * E + 2.0 * Pn[q] - (1.0 - 0.5 * gam * dt) * Pm[q]) / (1.0 + 0.5 * gam * dt);
                    } else if (m->kind == K_LORENTZ) {
                        /* eq:Pz_1D_Lorentz */
                        double w02 = m->omega0 * m->omega0, gam = m->gamma0, sg = m->sigma[q];
                        double A = 1.0 + 0.5 * gam * dt;
                        Pnew = (w02 * dt2 * sg * E - (w02 * dt2 - 2.0) * Pn[q] - (1.0 - 0.5 * gam * dt) * Pm[q]) / A;
                    } else if (m->kind == K_BATH) {
                        /* eq:Pz_update-LB with the coefficients of eq:Yzj_finite_difference */
                        double w02 = m->omega0 * m->omega0, g0 = m->gamma0, sg = m->sigma[q];
                        double skc = 0.0, bath = 0.0;
                        /* the thermal and anharmonic term f_j of each mode, and the Langevin force on P */
                        double f[m->nb > 0 ? m->nb : 1], etaP = 0.0;
                        long gq = IDX(g, i, j, k);
                        for (int jb = 0; jb < m->nb; jb++) {
                            double den = 1.0 + 0.5 * m->gj[jb] * dt, force = 0.0;
                            if (m->kT > 0.0)
                                force += sqrt(2.0 * m->gj[jb] * m->kT * w02 * sg / dt) * thermal_variate(m, gq, m->nupd, c, jb);
                            if (m->lam) {
                                double y = m->Y[c][0][jb * m->ncell + q];
                                force -= m->lam[jb] * y * y * y;
                            }
                            f[jb] = dt2 * force / den;
                        }
                        if (m->kT > 0.0) etaP = sqrt(2.0 * g0 * m->kT * w02 * sg / dt) * thermal_variate(m, gq, m->nupd, c, m->nb);
                        for (int jb = 0; jb < m->nb; jb++) {
                            double den = 1.0 + 0.5 * m->gj[jb] * dt;
                            double aj = (2.0 - m->wj[jb] * m->wj[jb] * dt2) / den;
                            double bj = -2.0 / den;
                            double cj = m->kj[jb] * dt / (2.0 * den);
                            skc += m->kj[jb] * cj;
                            bath += m->kj[jb] * (aj * m->Y[c][0][jb * m->ncell + q] + bj * m->Y[c][1][jb * m->ncell + q] + f[jb]);
                        }
                        double A = 1.0 + 0.5 * g0 * dt + 0.5 * dt * skc;
                        Pnew = (w02 * dt2 * sg * E - (w02 * dt2 - 2.0) * Pn[q] - (1.0 - 0.5 * g0 * dt - 0.5 * dt * skc) * Pm[q]
                                - 0.5 * dt * bath + dt2 * etaP) / A;
                        /* bath oscillators, eq:Yzj_finite_difference; level n-1/2 is overwritten by n+3/2 */
                        for (int jb = 0; jb < m->nb; jb++) {
                            double den = 1.0 + 0.5 * m->gj[jb] * dt;
                            double aj = (2.0 - m->wj[jb] * m->wj[jb] * dt2) / den;
                            double bj = -2.0 / den;
                            double cj = m->kj[jb] * dt / (2.0 * den);
                            double *y0 = &m->Y[c][0][jb * m->ncell + q], *y1 = &m->Y[c][1][jb * m->ncell + q];
                            double ynew = aj * (*y0) + (bj + 1.0) * (*y1) + cj * (Pnew - Pm[q]) + f[jb];
                            *y1 = *y0;
                            *y0 = ynew;
                        }
                    } else { /* K_CLOSURE */
                        double w02 = m->omega0 * m->omega0, g0 = m->gamma0, sg = m->sigma[q];
                        double *h = &m->hid[c][4 * q];
                        double x[7], z1[256], z2[256], o[5];
                        int W = m->width;
                        x[0] = E * m->scale[0];
                        x[1] = Pn[q] * m->scale[1];
                        x[2] = (Pn[q] - Pm[q]) / dt * m->scale[2];
                        for (int r = 0; r < 4; r++) x[3 + r] = h[r];
                        for (int u = 0; u < W; u++) {
                            double s = m->b1[u];
                            for (int v = 0; v < 7; v++) s += m->W1[u * 7 + v] * x[v];
                            z1[u] = tanh_(s);
                        }
                        for (int u = 0; u < W; u++) {
                            double s = m->b2[u];
                            for (int v = 0; v < W; v++) s += m->W2[u * W + v] * z1[v];
                            z2[u] = tanh_(s);
                        }
                        for (int u = 0; u < 5; u++) {
                            double s = m->b3[u];
                            for (int v = 0; v < W; v++) s += m->W3[u * W + v] * z2[v];
                            o[u] = s;
                        }
                        double bath_force = o[4] / m->scale[3];   /* stands for (dt/2) sum_j k_j (a_j Y_j^n + b_j Y_j^{n-1}) */
                        double skc = m->sum_kc;
                        double A = 1.0 + 0.5 * g0 * dt + 0.5 * dt * skc;
                        Pnew = (w02 * dt2 * sg * E - (w02 * dt2 - 2.0) * Pn[q] - (1.0 - 0.5 * g0 * dt - 0.5 * dt * skc) * Pm[q]
                                - bath_force) / A;
                        for (int r = 0; r < 4; r++) h[r] += o[r];
                    }
                    Pm[q] = Pn[q];
                    Pn[q] = Pnew;
                }
    }
    m->nupd++;
}

static void update_H(Grid *g) {
    double dt = g->dt;
    for (int c = 0; c < 3; c++) {
        if (!g->activeH[c]) continue;
        int a1 = CYC[c][0], a2 = CYC[c][1];
        /* dH_c/dt = -(curl E)_c = -(d_{a1} E_{a2} - d_{a2} E_{a1}) */
#pragma omp parallel for collapse(2) schedule(static)
        for (long i = 0; i < g->n[0]; i++)
            for (long j = 0; j < g->n[1]; j++)
                for (long k = 0; k < g->n[2]; k++) {
                    long q = IDX(g, i, j, k), pos[3] = {i, j, k};
                    double t1 = g->activeE[a2] ? dE(g, a2, a1, i, j, k) : 0.0;
                    double t2 = g->activeE[a1] ? dE(g, a1, a2, i, j, k) : 0.0;
                    if (g->psiH[c][a1]) {
                        double b = exp(-g->sH[a1][pos[a1]] * dt);
                        g->psiH[c][a1][q] = b * g->psiH[c][a1][q] + (b - 1.0) * t1;
                        t1 += g->psiH[c][a1][q];
                    }
                    if (g->psiH[c][a2]) {
                        double b = exp(-g->sH[a2][pos[a2]] * dt);
                        g->psiH[c][a2][q] = b * g->psiH[c][a2][q] + (b - 1.0) * t2;
                        t2 += g->psiH[c][a2][q];
                    }
                    g->H[c][q] -= dt * (t1 - t2);
                }
    }
}

/* ---------- monitors ---------- */

/* exact discrete energy at time n (fields E^{n-1/2}, E^{n+1/2}, H^n, matter at n+-1/2) */
static void sample_energy(Grid *g, Energy *e) {
    double dt = g->dt, fld = 0.0, pol = 0.0, bath = 0.0;
    for (long i = e->lo[0]; i < e->hi[0]; i++)
        for (long j = e->lo[1]; j < e->hi[1]; j++)
            for (long k = e->lo[2]; k < e->hi[2]; k++) {
                long q = IDX(g, i, j, k);
                for (int c = 0; c < 3; c++) {
                    if (g->activeE[c]) fld += 0.5 * g->eps[q] * g->Eprev[c][q] * g->E[c][q];
                    if (g->activeH[c]) fld += 0.5 * g->H[c][q] * g->H[c][q];
                }
                int mi = g->mat[q];
                if (mi < 0) continue;
                Mat *m = &g->m[mi];
                if (m->kind == K_DIELECTRIC) continue;
                long o = g->moff[q];
                if (m->kind == K_MULTI) {
                    for (int c = 0; c < 3; c++) {
                        if (!g->activeE[c]) continue;
                        for (int pp = 0; pp < m->np; pp++) {
                            double w2 = m->pw[pp] * m->pw[pp];
                            double rho = m->pkind[pp] == POLE_DRUDE ? 1.0 / w2 : 1.0 / (m->ps[pp] * w2);
                            double wr = m->pkind[pp] == POLE_DRUDE ? 0.0 : w2;
                            double p1 = m->P[c][0][pp * m->ncell + o], p0 = m->P[c][1][pp * m->ncell + o];
                            double v = (p1 - p0) / dt;
                            pol += 0.5 * rho * (v * v + wr * p1 * p0);
                        }
                    }
                    continue;
                }
                double rho, w02;
                if (m->kind == K_DRUDE) { rho = 1.0 / (m->omega0 * m->omega0); w02 = 0.0; }
                else { w02 = m->omega0 * m->omega0; rho = 1.0 / (m->sigma[o] * w02); }
                for (int c = 0; c < 3; c++) {
                    if (!g->activeE[c]) continue;
                    double p1 = m->P[c][0][o], p0 = m->P[c][1][o], v = (p1 - p0) / dt;
                    pol += 0.5 * rho * (v * v + w02 * p1 * p0);
                    for (int jb = 0; jb < m->nb; jb++) {
                        double y1 = m->Y[c][0][jb * m->ncell + o], y0 = m->Y[c][1][jb * m->ncell + o];
                        double u = (y1 - y0) / dt;
                        bath += 0.5 * rho * (u * u + m->wj[jb] * m->wj[jb] * y1 * y0);
                    }
                }
            }
    if (e->nsamp == e->cap) {
        e->cap *= 2;
        e->out = (double *)realloc(e->out, sizeof(double) * 3 * (size_t)e->cap);
    }
    e->out[3 * e->nsamp + 0] = fld;
    e->out[3 * e->nsamp + 1] = pol;
    e->out[3 * e->nsamp + 2] = bath;
    e->nsamp++;
}

/* tangential components of a plane normal to axis a, in right-handed order (t1, t2) with t1 x t2 = a */
static void tangents(int a, int *t1, int *t2) { *t1 = CYC[a][0]; *t2 = CYC[a][1]; }

static void accumulate_dft(Grid *g, Dft *d, int fieldE) {
    double dt = g->dt;
    double t = fieldE ? ((double)g->step + 0.5) * dt : ((double)g->step + 1.0) * dt;
    int t1, t2;
    tangents(d->axis, &t1, &t2);
    int comps[2] = {t1, t2};
    long bn1 = d->hi[1] - d->lo[1], bn2 = d->hi[2] - d->lo[2];
#pragma omp parallel for collapse(2) schedule(static)
    for (long i = d->lo[0]; i < d->hi[0]; i++)
        for (long j = d->lo[1]; j < d->hi[1]; j++)
            for (long k = d->lo[2]; k < d->hi[2]; k++) {
                long p = ((i - d->lo[0]) * bn1 + (j - d->lo[1])) * bn2 + (k - d->lo[2]);
                for (int s = 0; s < 2; s++) {
                    int c = comps[s];
                    double val;
                    if (fieldE) {
                        if (!g->activeE[c]) continue;
                        val = g->E[c][IDX(g, i, j, k)];
                    } else {
                        if (!g->activeH[c]) continue;
                        long b[3] = {i, j, k};
                        b[d->axis] -= 1;
                        val = 0.5 * (at(g, F_H, c, b[0], b[1], b[2]) + at(g, F_H, c, i, j, k));
                    }
                    double *acc = &d->acc[(((long)(fieldE ? s : 2 + s) * d->npts + p) * d->nf) * 2];
                    for (int f = 0; f < d->nf; f++) {
                        double ph = d->omega[f] * t;
                        acc[2 * f] += dt * val * cos(ph);
                        acc[2 * f + 1] += dt * val * sin(ph);
                    }
                }
            }
}

/* One step of a grid, or of both parts of a Bloch pair (stepped through part 0): every phase runs on
 * both parts before the next phase, so that reads across a Bloch axis see the other part at the same
 * time level. */
int or_step(void *gp, long nsteps) {
    Grid *g = (Grid *)gp;
    if (g->twin && g->part != 0) return -1;
    Grid *parts[2] = {g, g->twin};
    int np = g->twin ? 2 : 1;
    for (int p = 0; p < np; p++) build_pml(parts[p]);
    for (long s = 0; s < nsteps; s++) {
        for (int p = 0; p < np; p++) update_D(parts[p]);
        for (int p = 0; p < np; p++) {
            Grid *h = parts[p];
            update_E(h);
            for (int e = 0; e < h->nen; e++)
                if (h->step % h->e[e].every == 0) sample_energy(h, &h->e[e]);
            for (int mi = 0; mi < h->nmat; mi++) update_material(h, &h->m[mi]);
            for (int d = 0; d < h->ndft; d++) accumulate_dft(h, &h->d[d], 1);
        }
        for (int p = 0; p < np; p++) update_H(parts[p]);
        for (int p = 0; p < np; p++) {
            for (int d = 0; d < parts[p]->ndft; d++) accumulate_dft(parts[p], &parts[p]->d[d], 0);
            parts[p]->step++;
        }
    }
    return 0;
}

/* Make re and im the real and imaginary parts of one complex grid with Bloch phases phase[a] (radians,
 * k_a n_a) on its periodic axes.  Both grids must have the same shape and boundaries and must not have
 * stepped; their materials and monitors are set up alike by the caller.  Returns 0, or -1. */
int or_pair_bloch(void *rp, void *ip, const double *phase) {
    Grid *re = (Grid *)rp, *im = (Grid *)ip;
    if (re == im || re->twin || im->twin || re->step || im->step) return -1;
    for (int a = 0; a < 3; a++)
        if (re->n[a] != im->n[a] || re->bc[a] != im->bc[a] || (phase[a] != 0.0 && re->bc[a] != BC_PERIODIC)) return -1;
    re->twin = im; im->twin = re;
    re->part = 0; im->part = 1;
    for (int a = 0; a < 3; a++) re->bph[a] = im->bph[a] = phase[a];
    return 0;
}

long or_get_step(void *gp) { return ((Grid *)gp)->step; }

/* threads used by the cell loops (n < 1: leave unchanged); returns the count now in force */
int or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* comp 0..2: E, 3..5: H, 6..8: D; out holds the full grid (zeros for inactive components) */
int or_get_field(void *gp, int comp, double *out) {
    Grid *g = (Grid *)gp;
    double *f = NULL;
    if (comp >= 0 && comp < 3) f = g->E[comp];
    else if (comp >= 3 && comp < 6) f = g->H[comp - 3];
    else if (comp >= 6 && comp < 9) f = g->D[comp - 6];
    else return -1;
    if (f) memcpy(out, f, sizeof(double) * (size_t)g->ncell);
    else memset(out, 0, sizeof(double) * (size_t)g->ncell);
    return 0;
}

/* overwrite a field (comp as in or_get_field) */
int or_set_field(void *gp, int comp, const double *in) {
    Grid *g = (Grid *)gp;
    double *f = NULL;
    if (comp >= 0 && comp < 3) f = g->E[comp];
    else if (comp >= 3 && comp < 6) f = g->H[comp - 3];
    else if (comp >= 6 && comp < 9) f = g->D[comp - 6];
    if (!f) return -1;
    memcpy(f, in, sizeof(double) * (size_t)g->ncell);
    return 0;
}

/* polarization of material mi, E component c, level 0 (n+1/2) or 1 (n-1/2); box-sized output */
int or_get_P(void *gp, int mi, int c, int level, double *out) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->m[mi].P[c][level]) return -1;
    const Mat *m = &g->m[mi];
    memcpy(out, m->P[c][level], sizeof(double) * (size_t)m->ncell);
    for (int pp = 1; m->kind == K_MULTI && pp < m->np; pp++)       /* a multi-term material: the sum */
        for (long q = 0; q < m->ncell; q++) out[q] += m->P[c][level][pp * m->ncell + q];
    return 0;
}

/* one term of a multi-term material: its polarization at a level, box-sized */
int or_get_P_pole(void *gp, int mi, int c, int level, int pole, double *out) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || g->m[mi].kind != K_MULTI || pole < 0 || pole >= g->m[mi].np || !g->m[mi].P[c][level])
        return -1;
    memcpy(out, g->m[mi].P[c][level] + pole * g->m[mi].ncell, sizeof(double) * (size_t)g->m[mi].ncell);
    return 0;
}

int or_set_P_pole(void *gp, int mi, int c, int level, int pole, const double *in) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || g->m[mi].kind != K_MULTI || pole < 0 || pole >= g->m[mi].np || !g->m[mi].P[c][level])
        return -1;
    memcpy(g->m[mi].P[c][level] + pole * g->m[mi].ncell, in, sizeof(double) * (size_t)g->m[mi].ncell);
    return 0;
}

/* bath coordinates, [nb][box cells] */
int or_get_Y(void *gp, int mi, int c, int level, double *out) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->m[mi].Y[c][level]) return -1;
    memcpy(out, g->m[mi].Y[c][level], sizeof(double) * (size_t)(g->m[mi].nb * g->m[mi].ncell));
    return 0;
}

/* closure hidden state [box cells][4] */
int or_get_hidden(void *gp, int mi, int c, double *out) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->m[mi].hid[c]) return -1;
    memcpy(out, g->m[mi].hid[c], sizeof(double) * 4 * (size_t)g->m[mi].ncell);
    return 0;
}

int or_set_P(void *gp, int mi, int c, int level, const double *in) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->m[mi].P[c][level] || g->m[mi].kind == K_MULTI) return -1;
    memcpy(g->m[mi].P[c][level], in, sizeof(double) * (size_t)g->m[mi].ncell);
    return 0;
}

int or_set_Y(void *gp, int mi, int c, int level, const double *in) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->m[mi].Y[c][level]) return -1;
    memcpy(g->m[mi].Y[c][level], in, sizeof(double) * (size_t)(g->m[mi].nb * g->m[mi].ncell));
    return 0;
}

/* Drive material mi with a prescribed field: for each n, E_c of every cell of the box
 * is set to e_seq[n], the material is advanced once, and p_out[n] receives the new
 * polarization (level n+3/2 in grid time) of the first cell of the box. */
int or_drive_material(void *gp, int mi, int c, const double *e_seq, long n, double *p_out) {
    Grid *g = (Grid *)gp;
    if (mi < 0 || mi >= g->nmat || !g->activeE[c]) return -1;
    Mat *m = &g->m[mi];
    for (long s = 0; s < n; s++) {
        for (long i = m->lo[0]; i < m->hi[0]; i++)
            for (long j = m->lo[1]; j < m->hi[1]; j++)
                for (long k = m->lo[2]; k < m->hi[2]; k++) g->E[c][IDX(g, i, j, k)] = e_seq[s];
        update_material(g, m);
        double P = m->P[c][0] ? m->P[c][0][0] : 0.0;
        for (int pp = 1; m->kind == K_MULTI && pp < m->np; pp++) P += m->P[c][0][pp * m->ncell];
        p_out[s] = P;
    }
    return 0;
}

/* flux[f] = Re sum_p (E~ x conj(H~)) . e_axis ; raw (optional) = [4][npts][nf][2] accumulators of this
 * grid (of this part, on a Bloch pair).  On a Bloch pair (asked of part 0) the transforms are those of the
 * complex fields, E~ = E~_re + i E~_im with E~_re, E~_im the transforms of the two parts' series. */
int or_get_dft(void *gp, int id, double *flux, double *raw) {
    Grid *g = (Grid *)gp;
    if (id < 0 || id >= g->ndft) return -1;
    if (g->twin && g->part != 0) {   /* the imaginary part: its accumulators only */
        if (!raw) return -1;
        memcpy(raw, g->d[id].acc, sizeof(double) * 4 * (size_t)g->d[id].npts * (size_t)g->d[id].nf * 2);
        return 0;
    }
    Dft *d = &g->d[id], *di = g->twin ? &g->twin->d[id] : NULL;
    for (int f = 0; f < d->nf; f++) {
        double s = 0.0;
        for (long p = 0; p < d->npts; p++) {
            double v[4][2];   /* complex transform of E_t1, E_t2, H_t1, H_t2 at this point and frequency */
            for (int u = 0; u < 4; u++) {
                const double *r = &d->acc[((u * d->npts + p) * d->nf + f) * 2];
                v[u][0] = r[0];
                v[u][1] = r[1];
                if (di) {   /* + i (transform of the imaginary part) */
                    const double *m = &di->acc[((u * d->npts + p) * d->nf + f) * 2];
                    v[u][0] -= m[1];
                    v[u][1] += m[0];
                }
            }
            /* (E x H*)_a = E_t1 H_t2* - E_t2 H_t1*; real part of u v* = ur vr + ui vi */
            s += (v[0][0] * v[3][0] + v[0][1] * v[3][1]) - (v[1][0] * v[2][0] + v[1][1] * v[2][1]);
        }
        flux[f] = s;
    }
    if (raw) memcpy(raw, d->acc, sizeof(double) * 4 * (size_t)d->npts * (size_t)d->nf * 2);
    return 0;
}

long or_energy_count(void *gp, int id) {
    Grid *g = (Grid *)gp;
    if (id < 0 || id >= g->nen) return -1;
    return g->e[id].nsamp;
}

int or_get_energy(void *gp, int id, double *out) {
    Grid *g = (Grid *)gp;
    if (id < 0 || id >= g->nen) return -1;
    memcpy(out, g->e[id].out, sizeof(double) * 3 * (size_t)g->e[id].nsamp);
    return 0;
}

void or_destroy(void *gp) {
    Grid *g = (Grid *)gp;
    if (!g) return;
    for (int c = 0; c < 3; c++) {
        free(g->E[c]); free(g->Eprev[c]); free(g->D[c]); free(g->H[c]);
        for (int a = 0; a < 3; a++) { free(g->psiE[c][a]); free(g->psiH[c][a]); }
    }
    for (int a = 0; a < 3; a++) { free(g->sE[a]); free(g->sH[a]); }
    free(g->eps); free(g->mat); free(g->moff);
    for (int mi = 0; mi < g->nmat; mi++) {
        Mat *m = &g->m[mi];
        free(m->sigma); free(m->wj); free(m->gj); free(m->kj); free(m->W1);
        for (int c = 0; c < 3; c++) { free(m->P[c][0]); free(m->P[c][1]); free(m->Y[c][0]); free(m->Y[c][1]); free(m->hid[c]); }
    }
    for (int s = 0; s < g->nsrc; s++) free(g->s[s].profile);
    for (int d = 0; d < g->ndft; d++) { free(g->d[d].omega); free(g->d[d].acc); }
    for (int e = 0; e < g->nen; e++) free(g->e[e].out);
    free(g);
}
