/*
 * fdtdb — FDTD-Bath time stepping on one AMD Instinct MI355X (gfx950).
 *
 * The method is the FDTD scheme with auxiliary bath fields of T. E. Li,
 * "FDTD with Auxiliary Bath Fields for Condensed-Phase Polaritonics"
 * (arXiv 2505.23963): a Yee leapfrog (H from curl E, D from curl H,
 * E = (D - P)/eps_inf, Sec. II and eq:FDTD-1D) in which each cell's
 * polarization P follows a Lorentz oscillator coupled to N_b explicit
 * harmonic bath coordinates (eq:EOM_LorentzBath), advanced with the
 * central-difference updates eq:Pz_update-LB and eq:Yzj_finite_difference,
 * one independent bath per E component (end of Sec. II.C).
 *
 * Conventions
 *   Units c = eps0 = mu0 = 1, cell size dx = 1, dt = courant * dx, angular
 *   frequencies.  Cells are indexed (i, j, k) over axes (x, y, z); memory is
 *   C order with z fastest.  Yee placement of cell (i,j,k):
 *     Ex (i+1/2,j,k)  Ey (i,j+1/2,k)  Ez (i,j,k+1/2)
 *     Hx (i,j+1/2,k+1/2)  Hy (i+1/2,j,k+1/2)  Hz (i+1/2,j+1/2,k)
 *   A 1D grid runs along x with (Ez, Hy); a 2D grid is the x-y plane with
 *   (Ez, Hx, Hy); unused axes have extent 1.  Component ids: 0..2 = Ex, Ey,
 *   Ez; 3..5 = Hx, Hy, Hz.
 *   Time: after k full steps, H is at t = k dt; E, D and P at (k + 1/2) dt.
 *   Boxes are half-open cell ranges [lo, hi) per axis.
 *
 * Ownership: the library owns every device buffer it allocates; host arrays
 * passed in are copied before the call returns and never retained; outputs
 * go to caller-owned host buffers.  A grid borrows the caller's HIP stream
 * (or creates its own when given NULL) and never destroys a borrowed stream.
 *
 * Errors: every entry point returns an fdtdb_status; no exception crosses
 * the boundary.  fdtdb_last_error() returns a thread-local message for the
 * last failing call on the calling thread.
 *
 * Threading: calls on one grid must not overlap; distinct grids are
 * independent.
 */
#ifndef FDTDB_H
#define FDTDB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtdb_grid_s *fdtdb_grid;

typedef enum {
    FDTDB_OK = 0,
    FDTDB_E_INVALID = -1,   /* bad argument, box outside the grid, overlapping materials, ... */
    FDTDB_E_NOMEM = -2,     /* device or host allocation failed */
    FDTDB_E_DEVICE = -3,    /* a HIP call failed, or no usable device */
    FDTDB_E_UNSTABLE = -4,  /* parameters violate the explicit-scheme stability bound */
    FDTDB_E_DIVERGED = -5,  /* the watchdog found a non-finite field */
    FDTDB_E_STATE = -6      /* call not allowed in the grid's current state */
} fdtdb_status;

typedef enum { FDTDB_F32 = 0, FDTDB_F64 = 1 } fdtdb_dtype;

/* Boundary per axis.  CLOSED: field values beyond the grid read as zero
 * (electric wall one node past the high end, magnetic wall half a node
 * before the low end; lossless).  PML: the same walls behind a CPML layer of
 * pml_cells cells on both ends.  PERIODIC: wrap-around. */
typedef enum { FDTDB_BC_PML = 0, FDTDB_BC_PERIODIC = 1, FDTDB_BC_CLOSED = 2 } fdtdb_bc;

typedef struct {
    int64_t lo[3], hi[3];
} fdtdb_box;

typedef struct {
    int ndim;                 /* 1, 2 or 3 */
    int64_t n[3];             /* cells per axis (unused axes: 1) */
    double courant;           /* dt / dx; the library checks the vacuum Courant limit 1/sqrt(ndim) */
    fdtdb_dtype dtype;        /* storage precision of the time-stepped state */
    fdtdb_bc bc[3];           /* per axis; unused axes are forced to PERIODIC */
    int pml_cells[3];         /* CPML thickness per axis (used where bc == PML) */
    double pml_R0;            /* nominal CPML reflection (<= 0: 1e-8) */
    void *hip_stream;         /* hipStream_t to enqueue on; NULL: the grid creates its own stream */
} fdtdb_grid_desc;

/* ------------------------------------------------------------------------------------------ grid */

/* Allocate a grid with all fields zero.  Fails with E_INVALID on a bad
 * descriptor, E_UNSTABLE when courant exceeds 1/sqrt(ndim), E_NOMEM/E_DEVICE
 * on allocation or device errors. */
fdtdb_status fdtdb_create_grid(const fdtdb_grid_desc *desc, fdtdb_grid *out);

/* Free every device buffer of the grid; the grid's own stream (if any) is destroyed. */
fdtdb_status fdtdb_destroy_grid(fdtdb_grid g);

/* ------------------------------------------------------------------------------------- materials */
/* Materials are boxes; boxes must not overlap each other, and dispersive
 * boxes must not overlap the CPML layers (E_INVALID).  Materials can only be
 * added before the first fdtdb_step (E_STATE afterwards).  *material_id
 * (nullable) receives the material's index. */

/* Non-dispersive background eps_inf > 0: the constitutive relation D = eps_inf E + P of Sec. II
 * (the E line of eq:FDTD-1D with eps0 replaced by the background permittivity) with P = 0.
 * box: cells of the grid, half-open; eps_inf: the relative permittivity of those cells.  E_INVALID
 * for eps_inf <= 0, a box outside the grid or overlapping another material; E_STATE after the
 * first step. */
fdtdb_status fdtdb_set_eps_inf(fdtdb_grid g, const fdtdb_box *box, double eps_inf, int *material_id);

/* Drude medium: P'' + gamma P' = omega_p^2 E, i.e. the Lorentz model of
 * eq:EOM_Lorentz with omega0^2 dropped from the restoring term and
 * omega0^2 sigma = omega_p^2 (Sec. II.A).  E_UNSTABLE when
 * eps_inf < dt^2 (omega_p^2 + 4 ndim) / 4 (the lossless lattice bound). */
fdtdb_status fdtdb_set_drude(fdtdb_grid g, const fdtdb_box *box, double omega_p, double gamma, double eps_inf,
                             int *material_id);

/* Lorentz-Bath medium (eq:EOM_LorentzBath; parameters of eq:chi_LB):
 *   omega0, gamma0   bright-mode frequency and phenomenological damping
 *   eps_inf          background permittivity (E = (D - P)/eps_inf)
 *   sigma_cells      per-cell oscillator strength over the box, C order (x,y,z),
 *                    box-sized; NULL: sigma_uniform everywhere
 *   n_bath           bath modes per cell and E component (0: plain Lorentz, eq:Pz_1D_Lorentz)
 *   omega_j, gamma_j, k_j  bath frequencies, dampings and couplings (n_bath each)
 * E_UNSTABLE when the lossless lattice bound
 *   eps_inf (4/dt^2 - omega0^2) - omega0^2 sigma_max - 4 ndim (1 - omega0^2 dt^2 / 4) >= 0
 * fails, or when any omega_j dt >= 2 or omega0 dt >= 2. */
fdtdb_status fdtdb_set_lorentz_bath(fdtdb_grid g, const fdtdb_box *box, double omega0, double gamma0,
                                    double eps_inf, const double *sigma_cells, double sigma_uniform, int n_bath,
                                    const double *omega_j, const double *gamma_j, const double *k_j,
                                    int *material_id);

/* Sum of Lorentz and Drude terms on one box (Sec. II.A: realistic susceptibilities are fitted by several
 * such terms).  Term p is kinds[p] = 0, a Lorentz oscillator (eq:EOM_Lorentz with omega0 = omega[p],
 * gamma = gamma[p], oscillator strength sigma[p] > 0), or 1, a Drude term (omega_p = omega[p], gamma[p];
 * sigma[p] unused); every term is driven by the same E and advanced by its own central-difference update
 * (eq:Pz_1D_Lorentz; for a Drude term omega0^2 is dropped from the P^n coefficient), and D = eps_inf E +
 * sum_p P_p.  Arrays of n_terms (1..8) values, copied.  E_UNSTABLE when any omega[p] dt >= 2 or when the
 * lossless lattice bound fails: with X = 4/dt^2, X (eps_inf + sum_p chi_p(X)) >= 4 ndim, chi_p(X) =
 * omega_p^2 sigma_p / (omega_p^2 - X) (Drude: -omega_p^2 / X); one Lorentz term gives the bound of
 * fdtdb_set_lorentz_bath.  Same box rules and E_STATE rule as the other materials. */
fdtdb_status fdtdb_set_multi_term(fdtdb_grid g, const fdtdb_box *box, double eps_inf, int n_terms, const int *kinds,
                                  const double *omega, const double *gamma, const double *sigma, int *material_id);

/* Host-only map of Table 1 (Sec. III): bath form 0 = uniform, 1 = lorentzian,
 * 2 = gaussian.  Frequencies evenly spaced on [omega0 - width/2, omega0 + width/2],
 * gamma_j = bath_gamma, k_b = sqrt(2 dw dephasing / pi) with dw = width/(n_bath-1)
 * (eq:bath_dephasing_value_uniform); the non-uniform forms multiply k_b by
 * sqrt(G^2/(G^2 + (w_j - omega0)^2)) or exp(-(w_j - omega0)^2/(4 G^2)), G = gamma0 + dephasing.
 * Outputs are caller arrays of n_bath doubles.  n_bath >= 2. */
fdtdb_status fdtdb_bath_params(int form, double omega0, double gamma0, int n_bath, double width,
                               double bath_gamma, double dephasing, double *omega_j, double *gamma_j,
                               double *k_j);

/* Replace the explicit bath of Lorentz-Bath material `material_id` by the learned closure: per cell
 * and E component a hidden state h (4 values, starting at zero) and the network
 *   x = [E^{n+1/2} s_E, P^{n+1/2} s_P, (P^{n+1/2} - P^{n-1/2})/dt s_V, h]
 *   z1 = tanh(W1 x + b1), z2 = tanh(W2 z1 + b2), o = W3 z2 + b3     (width 32)
 *   h <- h + o[0:4];  the bath force term of eq:Pz_update-LB, (dt/2) sum_j k_j (a_j Y_j^n + b_j Y_j^{n-1}),
 *   is replaced by o[4] / s_S, while A keeps the exact sum_j k_j c_j of the material's bath.
 * weights: kClosureParams = 1477 floats, row major W1[32][7], b1[32], W2[32][32], b2[32], W3[5][32],
 * b3[5] (copied).  scales: s_E, s_P, s_V, s_S (> 0).  FP32 network arithmetic.  Before the first
 * step only (E_STATE).  E_INVALID unless width == 32 and the material is Lorentz-Bath. */
fdtdb_status fdtdb_set_bath_closure(fdtdb_grid g, int material_id, const float *weights, int width,
                                    const double *scales);

/* Closure hidden state of one E component, [box cells][4] host doubles. */
fdtdb_status fdtdb_get_closure_state(fdtdb_grid g, int material_id, int component, double *out);

/* ---------------------------------------------------------------------------- sources, monitors */

/* Soft current source on E component `component` over `box` (the Gaussian source of the
 * Appendix's simulation details, centred at omega_c with spectral width `width`; the current
 * enters Ampere's law of Sec. II, i.e. the D line of eq:FDTD-1D):
 *   J(t) = amplitude exp(-(t - t0)^2 / (2 tau^2)) cos(omega_c (t - t0)),
 *   tau = 1/width, t0 = 5 tau, J = 0 for t > 2 t0,
 * subtracted in the D update: D^{n+1/2} += -dt J(t_n) profile(cell).  Before the first step only
 * (E_STATE); at most 16 sources (E_INVALID).
 * profile: box-sized per-cell weights (NULL: 1).  The box must lie in one
 * eps_inf (E_INVALID otherwise).  *source_id is nullable. */
fdtdb_status fdtdb_add_source(fdtdb_grid g, int component, const fdtdb_box *box, double omega_c, double width,
                              double amplitude, const double *profile, int *source_id);

/* DFT flux plane normal to `axis` (the flux spectra through a plane behind the structure from
 * which the transmission spectra of Sec. IV are formed, Appendix simulation details), one cell
 * thick (plane->hi[axis] = plane->lo[axis] + 1), through the E nodes at index p0 = plane->lo[axis].
 * omega: nfreq angular frequencies (copied).  Accumulated in FP64:
 *   E~_c(p, w) = dt sum_{n} E_c^{n+1/2}(p) e^{i w (n+1/2) dt}
 *   H~_c(p, w) = dt sum_{n} (1/2)(H_c^{n+1}(p0 - 1/2) + H_c^{n+1}(p0 + 1/2)) e^{i w (n+1) dt}
 * for the two tangential components, and the flux along +axis
 *   Phi(w) = Re sum_p (E~ x conj(H~)) . e_axis. */
fdtdb_status fdtdb_add_dft_flux(fdtdb_grid g, int axis, const fdtdb_box *plane, int nfreq, const double *omega,
                                int *monitor_id);

/* Exact discrete energy over a box, sampled at steps n = 0, every, 2 every, ...
 * (Hamiltonian density eq:H_full in the centred-difference form):
 *   field = sum eps_inf/2 E^{n-1/2}.E^{n+1/2} + 1/2 |H^n|^2
 *   pol   = sum rho/2 [((P^{n+1/2}-P^{n-1/2})/dt)^2 + omega0^2 P^{n+1/2} P^{n-1/2}]
 *   bath  = sum rho/2 sum_j [((Y_j^{n+1/2}-Y_j^{n-1/2})/dt)^2 + omega_j^2 Y_j^{n+1/2} Y_j^{n-1/2}]
 * with rho = 1/(sigma omega0^2) (Drude: 1/omega_p^2).  FP64 sums. */
fdtdb_status fdtdb_add_energy_monitor(fdtdb_grid g, const fdtdb_box *box, int every, int *monitor_id);

/* Bloch-periodic grids (the boundary condition along y of the paper's 2D runs, Appendix "Simulation
 * details", here with any phase): couple two grids, re and im, as the real and imaginary parts of one
 * grid of complex fields with f(r + n_a e_a) = exp(i phase[a]) f(r) on each axis a (phase[a] = k_a n_a
 * in radians; 0 on a periodic axis keeps it plain periodic; phase[a] != 0 needs a periodic axis).
 * Every update has real coefficients, so each part advances by the ordinary step except where a
 * neighbour read crosses a Bloch axis: there it reads part p of exp(+-i phase[a]) (own + i other).
 * Both grids must have the same dimension, shape, boundaries, dtype, Courant number and stream (an im
 * created with a NULL stream gives up its own and takes re's; the stream goes with whichever part is
 * destroyed last), the
 * same set-up of materials and monitors, and no learned closure; sources are per part (the sources
 * of im carry the imaginary part of a complex source profile).  Call after the set-up, before the
 * first step.  Afterwards: fdtdb_step(re, n) advances both parts (E of both, then H of both, every
 * step; direct launches, graph mode unused) and fdtdb_step(im, n) returns E_STATE; fdtdb_dft_flux(re)
 * returns the flux of the complex fields Re sum (E~ x conj H~) with E~ = E~_re + i E~_im (its raw
 * output: re's accumulators), fdtdb_dft_flux(im, id, NULL, raw) only im's accumulators; energies,
 * fields and material state are read per part (the conserved energy is the sum over both parts,
 * so the energy-growth watchdog is off on pairs).  Only the rows whose neighbour read crosses a Bloch
 * axis (E's first row, H's last row along it) read the other part; they run the generic per-cell
 * kernels (in wrap regions four rows deep along z in 3D, y in 2D, when that length is a multiple of
 * 4), every other region the kernels of a real grid; in 2D a Lorentz-Bath material of up to 64 modes
 * that touches the wrap runs as a whole on its own kernel, which reads the other part at the wrap.
 * Destroying one part leaves the other unable to step (E_STATE).  Errors: E_INVALID for mismatched
 * grids, a phase on a non-periodic axis or a flux plane normal to a Bloch axis at its first cell;
 * E_STATE when either grid has stepped, is already paired or holds a learned closure, a bath stored
 * in 16 bits or a thermal or anharmonic bath. */
fdtdb_status fdtdb_pair_bloch(fdtdb_grid re, fdtdb_grid im, const double phase[3]);

/* Storage of a Lorentz-Bath material's bath coordinates Y_j (eq:Yzj_finite_difference; both time
 * levels): FDTDB_BATH_STATE (the grid's state type, the default), FDTDB_BATH_F16 (IEEE binary16 of
 * Y_j * scale) or FDTDB_BATH_BF16 (bfloat16 of Y_j * scale).  A reduced-precision mode beside the
 * method's FP32 state, for baths whose bytes bound the step: E and P are updated in FP64 as always, the
 * bath recurrence of the scaled coordinates in binary32 (its rounding, 6e-8, is far below the format's),
 * and each new Y_j * scale is rounded to the 16-bit format (round to nearest even), which halves the
 * bath's bytes and adds that rounding to every step (its error against the FP64 reference is measured,
 * not bounded by the FP32 bar).  scale (> 0, a power of two keeps it exact) places the
 * coordinates in the format's range (binary16: normal from 6.1e-5 to 65504).  Eight coordinates travel
 * as one 16-byte word ([word][cell] per level and component).  Available for 3D FP32 grids and baths of
 * 16 modes (the component-split kernel), before the first step, on a
 * material without a learned closure, outside Bloch pairs, and with no energy monitor over the
 * material (checked at the first step).  fdtdb_get_bath returns the stored values widened to FP64
 * and divided by scale.  Errors: E_INVALID (bad format, scale, material or grid), E_STATE (after the
 * first step, a closure, a Bloch pair). */
enum { FDTDB_BATH_STATE = 0, FDTDB_BATH_F16 = 1, FDTDB_BATH_BF16 = 2 };
fdtdb_status fdtdb_set_bath_storage(fdtdb_grid g, int material_id, int format, double scale);

/* Thermal bath: the extension the paper names in its outlook (Sec. V, thermal effects in the bath
 * oscillators), taken as Langevin forces.  Every damped coordinate of Lorentz-Bath material
 * material_id (P with gamma0, each Y_j with gamma_j) receives the force that fluctuation-dissipation
 * pairs with its damping for the effective mass rho = 1 / (eps0 sigma omega0^2) of eq:H_full, so that
 * the matter relaxes to the Gibbs state at temperature kT (energy units, same as the fields').  Over
 * one step the force is sqrt(2 gamma kT / (rho dt)) xi with xi = sqrt(12) (u - 1/2), u = (x + 1/2) /
 * 2^32, x a 32-bit word of Philox4x32-10 with counter (linear cell index of the grid, step index n
 * modulo 2^32, E component, variate / 4) and key (seed low word, seed high word), lane variate % 4
 * (a run longer than 2^32 steps repeats its noise); bath mode j
 * takes variate j and P variate N_b.  It enters eq:Yzj_finite_difference as + dt^2 eta_j /
 * (1 + gamma_j dt / 2) and, through the substituted Y_j^{n+1}, eq:Pz_update-LB (and P's own force as
 * + dt^2 eta_P in its bracket).  kT = 0 removes it.  The noise depends only on (seed, cell, step,
 * component), so runs, checkpoints and resumes are reproducible.  Before the first step; a real grid
 * (not a Bloch pair), bath kept in the state type (not 16-bit storage), no learned closure.  Such a
 * material runs on the general E kernel.  Errors: E_INVALID (kT < 0 or not finite, not a Lorentz-Bath
 * material with a bath), E_STATE (after the first step, Bloch pair, 16-bit storage, closure). */
fdtdb_status fdtdb_set_bath_thermal(fdtdb_grid g, int material_id, double kT, uint64_t seed);

/* Anharmonic bath (Sec. V outlook, anharmonicity in the bath oscillators): a quartic term
 * (rho / 4) lambda_j Y_j^4 in the potential of each bath mode, i.e. + lambda_j Y_j^3 on the left of
 * eq:EOM_LorentzBath-2, taken at level n like omega_j^2 Y_j: eq:Yzj_finite_difference gains
 * - dt^2 lambda_j (Y_j^n)^3 / (1 + gamma_j dt / 2), and eq:Pz_update-LB the same term through the
 * substituted Y_j^{n+1}.  lambda: host array of n = N_b values (copied); n = 0 returns to the harmonic
 * bath.  No stability bound is checked for it (the recurrence is nonlinear).  An energy monitor over
 * such a material is refused at the first step (its sum is the harmonic one).  Conditions and errors as
 * for fdtdb_set_bath_thermal, and E_INVALID when n is neither 0 nor N_b or a value is not finite. */
fdtdb_status fdtdb_set_bath_anharmonic(fdtdb_grid g, int material_id, const double *lambda, int n);

/* -------------------------------------------------------------------------------------- stepping */

/* Enqueue nsteps full time steps on the grid's stream and return without
 * waiting.  The first call uploads coefficient tables and fixes the
 * material layout.  Work is replayed from captured HIP graphs when graph
 * mode is on (fdtdb_set_graph). */
fdtdb_status fdtdb_step(fdtdb_grid g, int64_t nsteps);

/* Wait for the grid's stream and run the watchdog: E_DIVERGED when a field holds a non-finite
 * value, or when the total of an energy monitor over every cell outside the CPML layers, sampled
 * after every source has ended (t > 2 t0), exceeds twice its smallest value since then while above
 * 1 % of its value when the sources ended (a passive grid's exact discrete energy cannot grow; the
 * energy check is off on grids with a thermal bath, which feeds energy in, and on Bloch pairs);
 * E_DEVICE on an asynchronous device error. */
fdtdb_status fdtdb_synchronize(fdtdb_grid g);

/* Number of full steps enqueued so far. */
fdtdb_status fdtdb_steps_done(fdtdb_grid g, int64_t *steps);

/* Graph mode: 0 = direct launches; > 0 = capture chunks of this many steps
 * (rounded up to an even count) and replay them. Requires a non-NULL stream. */
fdtdb_status fdtdb_set_graph(fdtdb_grid g, int chunk_steps);

/* Checkpoint and resume of the leapfrog state (Sec. II: H^n, E^{n+1/2}; eq:Pz_update-LB and
 * eq:Yzj_finite_difference: both time levels of P and of every bath coordinate Y_j; the CPML psi
 * of every absorbing cell; the learned closure's hidden state; the FP64 DFT accumulators and
 * their unflushed staging slots; the energy samples so far; probe records; the step counter and
 * source clock).  save_state synchronizes the stream and writes one binary file (host path,
 * overwritten; nothing of the caller's is retained).  load_state reads such a file into a grid
 * built with the same set-up (geometry, dtype, materials and their parameters, sources,
 * monitors, probes, per-cell sigma values and closure weights), after which stepping
 * continues exactly as the saved grid would have: a resumed run equals an uninterrupted one
 * bitwise.  Errors: E_INVALID for null arguments or a file that cannot be opened or written;
 * E_STATE for a file that is not a state file, is truncated, or was written by a grid with
 * another set-up (the grid is then left unchanged); E_DEVICE on a device copy failure. */
fdtdb_status fdtdb_save_state(fdtdb_grid g, const char *path);
fdtdb_status fdtdb_load_state(fdtdb_grid g, const char *path);

/* ------------------------------------------------------------------------------------- read-out */
/* All read-outs synchronize the grid's stream first. */

/* flux: nfreq doubles (nullable when raw is given).  raw (nullable): [4][npts][nfreq][2] doubles,
 * the complex accumulators of E_t1, E_t2, H_t1, H_t2 (t1, t2 cyclic after axis).  Bloch pairs: see
 * fdtdb_pair_bloch. */
fdtdb_status fdtdb_dft_flux(fdtdb_grid g, int monitor_id, double *flux, double *raw);

/* out: capacity x 3 doubles [field, pol, bath]; *n_samples receives the number recorded. */
fdtdb_status fdtdb_energy(fdtdb_grid g, int monitor_id, double *out, int64_t capacity, int64_t *n_samples);

/* Copy a field component (0..5 = Ex, Ey, Ez, Hx, Hy, Hz; zeros for a component the grid does not
 * carry), widened to FP64, into dst: n[0]*n[1]*n[2] doubles in C order.  dst_is_device = 0: dst
 * is host memory; otherwise dst is device memory on the grid's device (the copy runs on the grid's
 * stream; no host round trip).  The call synchronizes the grid's stream before the copy, the whole
 * device before a write to a device destination (work another stream still has pending on dst, such
 * as the fill of a freshly made buffer, finishes first), and the grid's stream after it.  E_INVALID for
 * a null dst or a bad component. */
fdtdb_status fdtdb_get_field(fdtdb_grid g, int component, void *dst, int dst_is_device);

/* Overwrite a field component from n[0]*n[1]*n[2] host doubles (rounded to the storage type). */
fdtdb_status fdtdb_set_field(fdtdb_grid g, int component, const double *in);

/* Polarization of a dispersive material, E component c, at level 0 (P^{n+1/2})
 * or 1 (P^{n-1/2}); box-sized host doubles.  For Drude only the difference
 * level0 - level1 is stored; level 1 then returns zero and level 0 the difference. */
fdtdb_status fdtdb_get_polarization(fdtdb_grid g, int material_id, int component, int level, double *out);

/* One term of a multi-term material (fdtdb_set_multi_term), level as above; box-sized host doubles.  A
 * Drude term stores only its increment P^{n+1/2} - P^{n-1/2} (as fdtdb_set_drude does): level 0 returns the
 * increment, level 1 zeros.  fdtdb_get_polarization of a multi-term material returns the sum of its terms
 * when all are Lorentz terms, else E_INVALID. */
fdtdb_status fdtdb_get_polarization_term(fdtdb_grid g, int material_id, int component, int level, int term,
                                         double *out);

/* Bath coordinates [n_bath][box cells] at level 0 (Y^{n+1/2}) or 1 (Y^{n-1/2}). */
fdtdb_status fdtdb_get_bath(fdtdb_grid g, int material_id, int component, int level, double *out);

/* ---------------------------------------------------------------------------------- diagnostics */

typedef struct {
    int64_t cells;                 /* total cells */
    int64_t dispersive_cells;      /* cells carrying P */
    int64_t bath_cells;            /* cells carrying explicit bath modes */
    double bytes_per_step;         /* algorithmic HBM bytes of one full step (state read once, written once) */
    double bytes_per_step_e;       /* ... of the E/material update alone */
    double bytes_per_step_h;       /* ... of the H update alone */
    int launches_per_step;         /* kernel launches in one step (direct mode) */
} fdtdb_stats;

fdtdb_status fdtdb_get_stats(fdtdb_grid g, fdtdb_stats *out);

/* Per-launch timing.  mode 1: fdtdb_step launches directly (no graph replay) and brackets every
 * E and H launch with HIP events on the grid's stream; mode 2: only the E launches of Lorentz-Bath
 * and learned-closure materials (the launches that dominate a step) are bracketed, so that the
 * others run undisturbed (each bracketed launch adds roughly 7 us of event overhead to a step);
 * 0: off.  fdtdb_kernel_records collects the events.  E_INVALID for other modes. */
fdtdb_status fdtdb_set_profiling(fdtdb_grid g, int mode);

typedef struct {
    int region;                    /* region index (boxes of uniform update kind) */
    int phase;                     /* 0: E / material update, 1: H update */
    int kind;                      /* 0 background, 1 Drude, 2 Lorentz-Bath, 3 learned closure */
    int n_bath;                    /* explicit bath modes per component (kind 2) */
    int pml;                       /* 1 if the region carries CPML terms */
    int64_t cells;                 /* cells updated per launch */
    double bytes;                  /* algorithmic HBM bytes per launch */
    double ms_total;               /* summed event time of the profiled launches */
    int64_t launches;              /* profiled launches */
} fdtdb_kernel_record;

/* Synchronize, fold pending event pairs into the records and copy up to
 * capacity records (two per region) to out; *count receives the number. */
fdtdb_status fdtdb_kernel_records(fdtdb_grid g, fdtdb_kernel_record *out, int capacity, int *count);

/* ------------------------------------------------------------------------------ batched cavities */
/* Many independent 1D cavities (x axis, Ez / Hy, the grid conventions above)
 * of uneven length advanced together.  Each workgroup keeps one segment of one
 * cavity, with a halo of (steps per launch + 1) cells on each side, entirely in
 * registers for several steps per launch (no HBM traffic between those steps),
 * then writes it back; launches are replayed from a captured HIP graph.  The
 * arithmetic is that of the grid path (FP64 registers, FP32 or FP64 storage).
 * Limits: per cavity one Drude medium, one Lorentz-Bath medium with at most 32
 * bath modes, one source cell, one DFT node (frequencies shared by all
 * cavities), one energy box.  CPML of pml_cells cells at both ends of every
 * cavity (0: closed ends).  FP64 storage uses 256-thread workgroups. */
typedef struct fdtdb_batch_s *fdtdb_batch;

/* lengths: ncav cell counts (copied).  Same error model as fdtdb_create_grid.  Check mode for tests:
 * with the environment variable FDTDB_POISON_LDS=1 when the batch is created, every LDS word of the
 * on-chip kernel starts each launch as NaN (results must not change). */
fdtdb_status fdtdb_batch_create(int ncav, const int64_t *lengths, fdtdb_dtype dtype, double courant, int pml_cells,
                                double pml_R0, void *hip_stream, fdtdb_batch *out);
fdtdb_status fdtdb_batch_destroy(fdtdb_batch b);
/* Materials on cells [lo, hi) of cavity cav; same stability checks as the grid calls (ndim = 1). */
fdtdb_status fdtdb_batch_set_drude(fdtdb_batch b, int cav, int64_t lo, int64_t hi, double omega_p, double gamma,
                                   double eps_inf);
fdtdb_status fdtdb_batch_set_lorentz_bath(fdtdb_batch b, int cav, int64_t lo, int64_t hi, double omega0,
                                          double gamma0, double eps_inf, double sigma, int n_bath,
                                          const double *omega_j, const double *gamma_j, const double *k_j);
/* Soft current on Ez at cell x (the pulse of fdtdb_add_source). */
fdtdb_status fdtdb_batch_add_source(fdtdb_batch b, int cav, int64_t x, double omega_c, double width, double amplitude);
/* DFT flux node at cell x (1 <= x < L), the 1D case of fdtdb_add_dft_flux. */
fdtdb_status fdtdb_batch_add_dft_flux(fdtdb_batch b, int cav, int64_t x, int nfreq, const double *omega);
/* Exact discrete energy over cells [lo, hi) every `every` steps (fdtdb_add_energy_monitor). */
fdtdb_status fdtdb_batch_add_energy_monitor(fdtdb_batch b, int cav, int64_t lo, int64_t hi, int every);
/* Tile shape: steps per launch and threads per workgroup (256, 512 or 1024 for FP32; 256 for
 * FP64).  steps_per_launch == 0 runs the autotuner, which times the candidate shapes on scratch
 * copies of the state.  Only before the first step (E_STATE afterwards); the first
 * fdtdb_batch_step autotunes if no shape was set. */
fdtdb_status fdtdb_batch_set_tiling(fdtdb_batch b, int steps_per_launch, int threads_per_block);
fdtdb_status fdtdb_batch_get_tiling(fdtdb_batch b, int *steps_per_launch, int *threads_per_block);
fdtdb_status fdtdb_batch_step(fdtdb_batch b, int64_t nsteps);
fdtdb_status fdtdb_batch_synchronize(fdtdb_batch b);
fdtdb_status fdtdb_batch_steps_done(fdtdb_batch b, int64_t *steps);
/* Read-outs (synchronize first): component 2 (Ez) or 4 (Hy), L doubles; flux nfreq doubles;
 * energy capacity x 3 doubles [field, pol, bath]. */
fdtdb_status fdtdb_batch_get_field(fdtdb_batch b, int cav, int component, double *out);
fdtdb_status fdtdb_batch_dft_flux(fdtdb_batch b, int cav, double *flux);
fdtdb_status fdtdb_batch_energy(fdtdb_batch b, int cav, double *out, int64_t capacity, int64_t *n_samples);
/* fdtdb_batch_energy for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that must not call hipMalloc): the same read-out, the same arguments and results,
 * but the per-sample sums go through a device-resident buffer of the library (one per GPU, 65536
 * samples = 1.5 MiB, held until the process ends) instead of a buffer allocated for the call; it
 * calls no hipMalloc or hipFree.  At most 65536 samples per call (min(n_samples, capacity) above
 * that: E_INVALID, nothing copied).  Every call on one GPU uses that GPU's one buffer: calls that
 * overlap in time on one GPU (several host threads, several batches) race and must be serialized
 * by the caller.  Each call overwrites the part of the buffer it reads back, so nothing needs to
 * be cleared between calls. */
fdtdb_status fdtdb_batch_energy_noalloc(fdtdb_batch b, int cav, double *out, int64_t capacity, int64_t *n_samples);
/* Last error message of the batch calls on this thread. */
const char *fdtdb_batch_last_error(void);

/* ------------------------------------------------------------------- learned-closure training data */
/* Trajectory recorder on a Lorentz-Bath (or closure) material: for each step n < nsteps, row n of
 * the record holds, at each chosen cell, E^{n+1/2} of `component` after the E update of step n and
 * the new polarization P^{n+3/2} of that step (eq:Pz_update-LB), both rounded to FP32.  cells: n
 * flat indices into the material's box (row major, z fastest; copied).  Before the first step only.
 * The record is device memory owned by the grid: n * nsteps * 2 floats. */
fdtdb_status fdtdb_add_probe(fdtdb_grid g, int material_id, int component, int n, const int64_t *cells,
                             int64_t nsteps, int *probe_id);
/* Copy the record out (synchronizes): E and P are [nsteps][n] floats, host buffers, or device
 * buffers when to_device != 0 (written after the whole device has finished its pending work). */
fdtdb_status fdtdb_probe_data(fdtdb_grid g, int probe_id, float *E, float *P, int to_device);

/* Closure trainer (the network of fdtdb_set_bath_closure).  The target along each recorded
 * trajectory is the bath force of eq:Pz_update-LB, (dt/2) sum_j k_j (a_j Y_j^n + b_j Y_j^{n-1}),
 * recomputed in FP64 by running eq:Yzj_finite_difference driven by the recorded P from rest.
 * Inputs are scaled by 1/rms (s_E, s_P, s_V, s_S from the loaded record), the loss is the mean of
 * (o[4] - S s_S)^2, gradients come from truncated backpropagation through time over windows of
 * `window` steps taken in order from step 0 (the hidden state entering a window is carried from
 * the previous window and held constant), and Adam (beta1 0.9, beta2 0.999, eps 1e-8) takes one
 * step per window over all trajectories.  FP32 forward/backward, FP64 gradient sums and master
 * weights. */
typedef struct fdtdb_trainer_s *fdtdb_trainer;
typedef struct {
    int64_t ntraj;          /* trajectories N (recorded cells) */
    int64_t nsteps;         /* recorded steps T per trajectory, a multiple of window */
    int window;             /* truncated-BPTT window W, 1..4096 */
    int activation;         /* 0: tanh (the closure); 1: identity (the linear special case) */
    double dt;              /* time step */
    int n_bath;             /* the explicit bath whose force is learned (arrays copied) */
    const double *omega_j, *gamma_j, *k_j;
    void *hip_stream;       /* borrowed; NULL = default stream */
} fdtdb_trainer_desc;

fdtdb_status fdtdb_trainer_create(const fdtdb_trainer_desc *desc, fdtdb_trainer *out);
fdtdb_status fdtdb_trainer_destroy(fdtdb_trainer t);
/* E, P: [nsteps][ntraj] floats as written by the recorder (host, or device if on_device != 0; device
 * sources are read after the whole device has finished its pending work, on any stream);
 * copied.  Computes the FP64 targets, the scales and the packed inputs. */
fdtdb_status fdtdb_trainer_load(fdtdb_trainer t, const float *E, const float *P, int on_device);
/* s_E, s_P, s_V, s_S (4 doubles, host). */
fdtdb_status fdtdb_trainer_get_scales(fdtdb_trainer t, double *scales);
/* FP64 targets S, [nsteps][ntraj] doubles (host). */
fdtdb_status fdtdb_trainer_get_targets(fdtdb_trainer t, double *S);
/* Weights in the fdtdb_set_bath_closure layout (1477 floats, host; copied); resets Adam. */
fdtdb_status fdtdb_trainer_set_weights(fdtdb_trainer t, const float *weights);
fdtdb_status fdtdb_trainer_get_weights(fdtdb_trainer t, float *weights);
/* Switch the activation used by training.  Going from identity (1) to tanh (0) with weights set,
 * the weights are first rescaled so that the tanh network computes the identity network's
 * function to O(eps^2) (W1, b1, b2 times eps, W3 divided by eps: every pre-activation shrinks by
 * eps, where tanh is linear); Adam's moments restart.  This carries a closure trained in the
 * linear regime (the bath is a linear filter of the polarization history, eq:EOM_LorentzBath-2)
 * into the tanh network.  eps in (0, 1]. */
fdtdb_status fdtdb_trainer_set_activation(fdtdb_trainer t, int activation, double eps);
/* Loss and gradient at the current weights without updating them: the mean over windows of the
 * window loss and of its gradient (1477 doubles, host). */
fdtdb_status fdtdb_trainer_loss_grad(fdtdb_trainer t, double *loss, double *grad);
/* `epochs` passes over the record, learning rate lr * lr_decay^epoch; the mean window loss of
 * each epoch (taken before each window's update) goes to loss_per_epoch[epochs] (may be NULL).
 * An epoch whose loss is not finite or exceeds 100 times the best so far (the learned recurrence
 * ran away) is undone (weights and Adam state restored) and repeated at half the rate; after 12
 * such retries the call returns FDTDB_E_DIVERGED. */
fdtdb_status fdtdb_trainer_train(fdtdb_trainer t, int epochs, double lr, double lr_decay, double *loss_per_epoch);
/* Last error message of the trainer calls on this thread. */
const char *fdtdb_trainer_last_error(void);

/* Last error message on this thread ("" if none). */
const char *fdtdb_last_error(void);

/* Library version string. */
const char *fdtdb_version(void);

/* ------------------------------------------------------------------------------------- memory */
/* Device memory source (not from the paper: an ownership hook for callers with their own device
 * allocator, such as a framework's caching allocator).  Grids, batches and trainers created after
 * the call take every device buffer from alloc(bytes, ctx), which must return memory of the
 * current device, aligned to 256 bytes, or NULL (the creating call then fails with E_NOMEM; a
 * misaligned block is handed back to free and also gives E_NOMEM); they release it through
 * free(ptr, ctx) when destroyed.  Each object keeps the allocator it was created with, so the
 * callbacks and ctx must stay valid until the last such object is destroyed.  Both NULL restores
 * hipMalloc / hipFree (the default).  E_INVALID if exactly one of them is NULL.  Host-only; the
 * setting is process-wide and guarded by a lock. */
typedef void *(*fdtdb_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fdtdb_free_fn)(void *ptr, void *ctx);
fdtdb_status fdtdb_set_allocator(fdtdb_alloc_fn alloc, fdtdb_free_fn free_fn, void *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FDTDB_H */
