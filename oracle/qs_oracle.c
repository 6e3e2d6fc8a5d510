/*
 * qs_oracle.c -- plain FP64 CPU oracle for the linear quasistatic beam-plasma model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python
 * binding) may include, link, load or call this file.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark use it.  It shares no code, header,
 * table or helper with the GPU path.
 *
 * What it computes (San Miguel Claveria et al., "Quasistatic modeling of ultrarelativistic
 * beam-plasma instabilities", Sec. II and Sec. III.D), for one transverse Fourier mode
 * exp(i k.r_perp) at a time, in the paper's normalized units:
 *
 *   plasma response   (d_xi^2 + 1) n_p = rho,  rho = sum_s q_s n_s          Eq. plasma_oscillations_QSA
 *   pseudo-potential  (1 + k^2) Psi = n_p                                   Eq. poisson_QSA (d_y -> i k)
 *   beam continuity   d_tau n_s = d_xi(n0_s u_s) - i k n0_s w_s             Eq. beam_continuity, flux form
 *                                                                            for a xi-dependent n0_s (Sec. III.D)
 *   beam momentum     d_tau (gamma^3 u_s) = -(q_s/m_s) d_xi Psi              Eq. beam_momentum
 *                     d_tau (gamma   w_s) = +(q_s/m_s) i k Psi
 *
 * with u_s, w_s the longitudinal and transverse (along k) velocity perturbations.  Per
 * species the state is n_s (cell centres), pz_s = gamma^3 u_s (interior cell faces) and
 * pt_s = gamma w_s (cell centres).
 *
 * The discretization (the paper gives none; these are the readings written down in the
 * design notes):
 *   - cells j = 0..N-1 of width h, centres (j+1/2)h; the beam front is xi = 0;
 *   - pz_s lives on the interior faces (j+1)h, j = 0..N-2; the two outer faces carry no
 *     flux (n0 = 0 outside the beam);  n0 on a face is the mean of the two centres;
 *   - the plasma oscillator is advanced through each cell with its exact solution for a
 *     cell-constant source, starting from n_p = d_xi n_p = 0 ahead of the front (with the
 *     stationary-front option, from n_p = F, d_xi n_p = 0, F the mode's front value held for
 *     every tau: the boundary value of Sec. III.D and Appendix C);
 *   - classic fourth-order Runge-Kutta in tau, each stage one full march over the beam.
 *
 * Fields (derived from Maxwell's equations under the same quasistatic ordering, neglecting
 * the O(d_tau) transverse beam current):
 *   E_par = -d_xi Psi,  E_perp = -i k (rho - n_p)/(1+k^2),  B_perp = -i k rho/(1+k^2),
 *   so that E_perp - B_perp = i k Psi, the transverse force of Sec. III.D.
 *
 * Everything is double / double complex; no blocking, fusion or reordering.
 *
 * Mutation hooks: the ORC_PLANT_* macros below each plant one deliberate mistake (a sign
 * or index slip, a dropped term).  They are never defined in the oracle's normal build;
 * the pin tests compile variants with one of them defined and check that a pin fails.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DROP_LONGITUDINAL 1 /* drop the gamma^-2 longitudinal term (Eq. CFI_st_master) */
#define ORC_NO_RESTORING 2      /* replace (d_xi^2 + 1) by d_xi^2 (Eq. CFI_st_master_front) */
#define ORC_STEADY_INFLOW 4     /* plasma ahead of the front in equilibrium with cell 0 */
#define ORC_STATIONARY_FRONT 16 /* plasma ahead of the front held at a given n_p, d_xi n_p = 0 */

typedef struct {
    int n_species;
    const double *q;     /* charge per species (units of e) */
    const double *m;     /* mass per species (units of m_e) */
    const double *nb;    /* peak unperturbed density per species (units of n_p) */
    double gamma;        /* common Lorentz factor */
    int n_xi;            /* number of cells */
    double h;            /* cell width */
    const double *shape; /* longitudinal profile at cell centres, NULL = flat top */
    int flags;
} orc_beam;

/* ------------------------------------------------------------------ random numbers */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the i-th output (i = 0, 1, ...) of
 * the generator whose state starts at `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) from the top 53 bits */
double orc_u53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* ------------------------------------------------------------------ profile helpers */

static double shape_at(const orc_beam *b, int j) { return b->shape ? b->shape[j] : 1.0; }

/* unperturbed density of species s at centre j and at face j+1/2 (mean of the centres) */
static double n0_centre(const orc_beam *b, int s, int j) { return b->nb[s] * shape_at(b, j); }
static double n0_face(const orc_beam *b, int s, int j)
{
    return 0.5 * (n0_centre(b, s, j) + n0_centre(b, s, j + 1));
}

/* ------------------------------------------------------------------ plasma march */

/* One causal march of Eq. plasma_oscillations_QSA through the beam for the cell-constant
 * charge density rho[j].  Returns n_p and d_xi n_p at the cell centres and d_xi n_p at the
 * rear face of every cell. */
static void march_from(const orc_beam *b, const double complex *rho, double complex front,
                       double complex *np_c, double complex *dnp_c, double complex *dnp_f)
{
    const int N = b->n_xi;
    const double h = b->h;
    double complex n = 0.0, dn = 0.0; /* unperturbed plasma ahead of the front */
    if (b->flags & ORC_STEADY_INFLOW) n = rho[0];
    if (b->flags & ORC_STATIONARY_FRONT) n = front;
    for (int j = 0; j < N; ++j) {
        const double complex r = rho[j];
        if (b->flags & ORC_NO_RESTORING) {
            /* n'' = r :  n(s) = n + dn s + r s^2/2 */
            double s = 0.5 * h;
            np_c[j] = n + dn * s + 0.5 * r * s * s;
            dnp_c[j] = dn + r * s;
            s = h;
            double complex n1 = n + dn * s + 0.5 * r * s * s;
            double complex d1 = dn + r * s;
            n = n1;
            dn = d1;
        } else {
            /* n'' + n = r :  n(s) = r + (n - r) cos s + dn sin s */
            double s = 0.5 * h;
            np_c[j] = r + (n - r) * cos(s) + dn * sin(s);
            dnp_c[j] = -(n - r) * sin(s) + dn * cos(s);
            s = h;
            double complex n1 = r + (n - r) * cos(s) + dn * sin(s);
            double complex d1 = -(n - r) * sin(s) + dn * cos(s);
            n = n1;
            dn = d1;
        }
        dnp_f[j] = dn;
    }
}

void orc_march(const orc_beam *b, const double complex *rho, double complex *np_c,
               double complex *dnp_c, double complex *dnp_f)
{
    march_from(b, rho, 0.0, np_c, dnp_c, dnp_f);
}

/* ------------------------------------------------------------------ per-species state */

/* state of one mode: for species s, arrays of n_xi complex values each
 *   n [s*N + j]  density perturbation at centre j
 *   pz[s*N + j]  gamma^3 u at face j+1/2 (the last entry, the rear outer face, stays 0)
 *   pt[s*N + j]  gamma w at centre j                                                     */
typedef struct {
    double complex *n, *pz, *pt;
} orc_state;

typedef struct {
    double complex *rho, *np_c, *dnp_c, *dnp_f;
    double complex front; /* the mode's front value in the stored state's units */
} orc_work;

static void charge_density(const orc_beam *b, const orc_state *x, double complex *rho)
{
    const int N = b->n_xi;
    for (int j = 0; j < N; ++j) {
        double complex r = 0.0;
        for (int s = 0; s < b->n_species; ++s) r += b->q[s] * x->n[s * N + j];
        rho[j] = r;
    }
}

/* d/dtau of the state (Eqs. beam_continuity and beam_momentum with Psi from the march) */
static void rates(const orc_beam *b, double k, const orc_state *x, orc_state *dx, orc_work *w)
{
    const int N = b->n_xi;
    const double h = b->h, g = b->gamma;
    const double g3 = g * g * g;
    const double kap = 1.0 / (1.0 + k * k);

    charge_density(b, x, w->rho);
    march_from(b, w->rho, w->front, w->np_c, w->dnp_c, w->dnp_f);

    for (int s = 0; s < b->n_species; ++s) {
        const double qm = b->q[s] / b->m[s];
        for (int j = 0; j < N; ++j) {
            /* longitudinal flux n0 u on the two faces of cell j (zero on the outer faces) */
            double complex f_rear = 0.0, f_front = 0.0;
            if (!(b->flags & ORC_DROP_LONGITUDINAL)) {
#ifdef ORC_PLANT_NONFLUX /* mutation: n0 taken at the cell centre on both faces */
                if (j < N - 1) f_rear = n0_centre(b, s, j) * x->pz[s * N + j] / g3;
                if (j > 0) f_front = n0_centre(b, s, j) * x->pz[s * N + j - 1] / g3;
#else
                if (j < N - 1) f_rear = n0_face(b, s, j) * x->pz[s * N + j] / g3;
                if (j > 0) f_front = n0_face(b, s, j - 1) * x->pz[s * N + j - 1] / g3;
#endif
            }
            double complex psi = kap * w->np_c[j];
            dx->n[s * N + j] = (f_rear - f_front) / h - I * k * n0_centre(b, s, j) * x->pt[s * N + j] / g;
#ifdef ORC_PLANT_TRANS_SIGN /* mutation: sign of the transverse force */
            dx->pt[s * N + j] = -qm * I * k * psi;
#else
            dx->pt[s * N + j] = qm * I * k * psi;
#endif
            if (j < N - 1 && !(b->flags & ORC_DROP_LONGITUDINAL))
#if defined(ORC_PLANT_LONG_SIGN) /* mutation: sign of the longitudinal force */
                dx->pz[s * N + j] = qm * kap * w->dnp_f[j];
#elif defined(ORC_PLANT_FACE_INDEX) /* mutation: the next face's plasma gradient */
                dx->pz[s * N + j] = -qm * kap * w->dnp_f[j + 1];
#else
                dx->pz[s * N + j] = -qm * kap * w->dnp_f[j];
#endif
            else
                dx->pz[s * N + j] = 0.0;
        }
    }
}

/* y = x + a*dx over the whole state */
static void axpy_state(int len, const orc_state *x, double a, const orc_state *dx, orc_state *y)
{
    for (int i = 0; i < len; ++i) {
        y->n[i] = x->n[i] + a * dx->n[i];
        y->pz[i] = x->pz[i] + a * dx->pz[i];
        y->pt[i] = x->pt[i] + a * dx->pt[i];
    }
}

/* one classic RK4 step of length dtau */
static void rk4_step(const orc_beam *b, double k, double dtau, orc_state *x, orc_state *k1,
                     orc_state *k2, orc_state *k3, orc_state *k4, orc_state *tmp, orc_work *w)
{
    const int len = b->n_species * b->n_xi;
    rates(b, k, x, k1, w);
    axpy_state(len, x, 0.5 * dtau, k1, tmp);
    rates(b, k, tmp, k2, w);
    axpy_state(len, x, 0.5 * dtau, k2, tmp);
    rates(b, k, tmp, k3, w);
    axpy_state(len, x, dtau, k3, tmp);
    rates(b, k, tmp, k4, w);
    for (int i = 0; i < len; ++i) {
        x->n[i] += dtau / 6.0 * (k1->n[i] + 2.0 * k2->n[i] + 2.0 * k3->n[i] + k4->n[i]);
        x->pz[i] += dtau / 6.0 * (k1->pz[i] + 2.0 * k2->pz[i] + 2.0 * k3->pz[i] + k4->pz[i]);
        x->pt[i] += dtau / 6.0 * (k1->pt[i] + 2.0 * k2->pt[i] + 2.0 * k3->pt[i] + k4->pt[i]);
    }
}

/* fields of the current state at the cell centres; log2_scale is the power of two the
 * stored state has been divided by.  Writes ln|E|, ln|B|, ln A = ln sqrt(|E|^2+|B|^2). */
static void fields(const orc_beam *b, double k, const orc_state *x, orc_work *w, double log2_scale,
                   double *ln_e, double *ln_b, double *ln_a, double *e_par, double *np_out)
{
    const int N = b->n_xi;
    const double kap = 1.0 / (1.0 + k * k);
    charge_density(b, x, w->rho);
    march_from(b, w->rho, w->front, w->np_c, w->dnp_c, w->dnp_f);
    const double shift = log2_scale * log(2.0);
    for (int j = 0; j < N; ++j) {
        double complex epar = -kap * w->dnp_c[j];
#ifdef ORC_PLANT_EPERP_SIGN /* mutation: sign inside rho - n_p */
        double complex eperp = -I * k * kap * (w->rho[j] + w->np_c[j]);
#else
        double complex eperp = -I * k * kap * (w->rho[j] - w->np_c[j]);
#endif
#ifdef ORC_PLANT_BPERP_NP /* mutation: n_p in place of rho */
        double complex bperp = -I * k * kap * w->np_c[j];
#else
        double complex bperp = -I * k * kap * w->rho[j];
#endif
        double e2 = creal(epar * conj(epar)) + creal(eperp * conj(eperp));
        double b2 = creal(bperp * conj(bperp));
        if (ln_e) ln_e[j] = 0.5 * log(e2) + shift;
        if (ln_b) ln_b[j] = 0.5 * log(b2) + shift;
        if (ln_a) ln_a[j] = 0.5 * log(e2 + b2) + shift;
        if (e_par) { e_par[2 * j] = creal(epar); e_par[2 * j + 1] = cimag(epar); }
        if (np_out) { np_out[2 * j] = creal(w->np_c[j]); np_out[2 * j + 1] = cimag(w->np_c[j]); }
    }
}

/* divide the state by 2^e with e the binary exponent of max_j |Re rho|, |Im rho| */
static void renormalize(const orc_beam *b, orc_state *x, orc_work *w, double *log2_scale)
{
    const int N = b->n_xi, len = b->n_species * N;
    charge_density(b, x, w->rho);
    double mx = 0.0;
    for (int j = 0; j < N; ++j) {
        mx = fmax(mx, fabs(creal(w->rho[j])));
        mx = fmax(mx, fabs(cimag(w->rho[j])));
    }
    if (!(mx > 0.0) || !isfinite(mx)) return;
    int e;
    frexp(mx, &e);
    for (int i = 0; i < len; ++i) {
        x->n[i] = ldexp(creal(x->n[i]), -e) + I * ldexp(cimag(x->n[i]), -e);
        x->pz[i] = ldexp(creal(x->pz[i]), -e) + I * ldexp(cimag(x->pz[i]), -e);
        x->pt[i] = ldexp(creal(x->pt[i]), -e) + I * ldexp(cimag(x->pt[i]), -e);
    }
    *log2_scale += e;
}

/* ------------------------------------------------------------------ public entry points */

static double complex *zalloc(size_t n) { return (double complex *)calloc(n ? n : 1, sizeof(double complex)); }

/*
 * Advance n_modes independent modes by n_steps RK4 steps of dtau.
 *
 * state (interleaved re/im doubles), per mode m, per species s, per cell j:
 *   n [((m*S + s)*N + j)*2 + {0,1}],  same for pz and pt.
 * log2_scale[m]: power of two already divided out of mode m (in/out).
 * renorm: if nonzero, renormalize each mode after every step (exact powers of two).
 * front: with ORC_STATIONARY_FRONT, per mode the complex value F (interleaved re/im, in
 *   unscaled units) that n_p takes ahead of the front at every tau; else ignored (NULL).
 * Outputs, any may be NULL:
 *   ln_e, ln_b  [n_snap][N][n_modes]   fields of the state at the start of each step s
 *               with s % out_every == 0 (n_snap = ceil(n_steps/out_every)); when
 *               n_steps == 0, one snapshot of the current state.
 *   max_ln_a    [n_steps][n_modes]     max over cells of ln A at the start of each step.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int orc_run_modes(const orc_beam *b, int n_modes, const double *k, double dtau, int n_steps,
                  int out_every, double *n_io, double *pz_io, double *pt_io, double *log2_scale,
                  int renorm, double *ln_e, double *ln_b, double *max_ln_a, int n_threads,
                  const double *front)
{
    if (!b || b->n_xi < 1 || b->n_species < 1 || n_modes < 0 || n_steps < 0 || !k) return -1;
    if ((b->flags & ORC_STATIONARY_FRONT) && !front) return -1;
    if (out_every < 1) out_every = 1;
    const int N = b->n_xi, S = b->n_species, len = S * N;
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        orc_state x, k1, k2, k3, k4, tmp;
        orc_state *all[6] = {&x, &k1, &k2, &k3, &k4, &tmp};
        int ok = 1;
        for (int i = 0; i < 6; ++i) {
            all[i]->n = zalloc(len);
            all[i]->pz = zalloc(len);
            all[i]->pt = zalloc(len);
            ok = ok && all[i]->n && all[i]->pz && all[i]->pt;
        }
        orc_work w = {zalloc(N), zalloc(N), zalloc(N), zalloc(N), 0.0};
        double *ln_a = (double *)calloc(N, sizeof(double));
        double *tmp_e = (double *)calloc(N, sizeof(double));
        double *tmp_b = (double *)calloc(N, sizeof(double));
        ok = ok && w.rho && w.np_c && w.dnp_c && w.dnp_f && ln_a && tmp_e && tmp_b;
        if (!ok) {
#pragma omp atomic write
            status = -1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < n_modes; ++m) {
            if (!ok) continue;
            for (int i = 0; i < len; ++i) {
                size_t o = ((size_t)m * len + i) * 2;
                x.n[i] = n_io[o] + I * n_io[o + 1];
                x.pz[i] = pz_io[o] + I * pz_io[o + 1];
                x.pt[i] = pt_io[o] + I * pt_io[o + 1];
            }
            double l2 = log2_scale ? log2_scale[m] : 0.0;
            const double complex f0 =
                (b->flags & ORC_STATIONARY_FRONT) ? front[2 * m] + I * front[2 * m + 1] : 0.0;
            int n_snap_steps = n_steps == 0 ? 1 : n_steps;
            for (int st = 0; st < n_snap_steps; ++st) {
                w.front = f0 * ldexp(1.0, -(int)l2); /* the stored state's units */
                int snap = (st % out_every == 0);
                if ((snap && (ln_e || ln_b)) || (max_ln_a && n_steps > 0)) {
                    fields(b, k[m], &x, &w, l2, tmp_e, tmp_b, ln_a, NULL, NULL);
                    if (snap) {
                        size_t si = (size_t)(st / out_every);
                        for (int j = 0; j < N; ++j) {
                            if (ln_e) ln_e[(si * N + j) * n_modes + m] = tmp_e[j];
                            if (ln_b) ln_b[(si * N + j) * n_modes + m] = tmp_b[j];
                        }
                    }
                    if (max_ln_a && n_steps > 0) {
                        double mx = -INFINITY;
                        for (int j = 0; j < N; ++j) mx = fmax(mx, ln_a[j]);
                        max_ln_a[(size_t)st * n_modes + m] = mx;
                    }
                }
                if (n_steps == 0) break;
                rk4_step(b, k[m], dtau, &x, &k1, &k2, &k3, &k4, &tmp, &w);
                if (renorm) renormalize(b, &x, &w, &l2);
            }
            for (int i = 0; i < len; ++i) {
                size_t o = ((size_t)m * len + i) * 2;
                n_io[o] = creal(x.n[i]);
                n_io[o + 1] = cimag(x.n[i]);
                pz_io[o] = creal(x.pz[i]);
                pz_io[o + 1] = cimag(x.pz[i]);
                pt_io[o] = creal(x.pt[i]);
                pt_io[o + 1] = cimag(x.pt[i]);
            }
            if (log2_scale) log2_scale[m] = l2;
        }
        for (int i = 0; i < 6; ++i) {
            free(all[i]->n);
            free(all[i]->pz);
            free(all[i]->pt);
        }
        free(w.rho);
        free(w.np_c);
        free(w.dnp_c);
        free(w.dnp_f);
        free(ln_a);
        free(tmp_e);
        free(tmp_b);
    }
    return status;
}

/* Diagnostics of one mode's state (same layout as one mode of orc_run_modes):
 * np_c, e_par: complex interleaved [N]; ln_e, ln_b, ln_a: [N].  Any may be NULL.
 * front: the mode's front value (re, im; unscaled) with ORC_STATIONARY_FRONT, else NULL. */
int orc_mode_fields(const orc_beam *b, double k, const double *n_in, const double *pz_in,
                    const double *pt_in, double log2_scale, double *np_c, double *e_par,
                    double *ln_e, double *ln_b, double *ln_a, const double *front)
{
    const int N = b->n_xi, len = b->n_species * N;
    if ((b->flags & ORC_STATIONARY_FRONT) && !front) return -1;
    orc_state x = {zalloc(len), zalloc(len), zalloc(len)};
    orc_work w = {zalloc(N), zalloc(N), zalloc(N), zalloc(N), 0.0};
    if (b->flags & ORC_STATIONARY_FRONT) w.front = (front[0] + I * front[1]) * ldexp(1.0, -(int)log2_scale);
    double *te = (double *)calloc(N, sizeof(double)), *tb = (double *)calloc(N, sizeof(double));
    double *ta = (double *)calloc(N, sizeof(double));
    if (!x.n || !x.pz || !x.pt || !w.rho || !w.np_c || !w.dnp_c || !w.dnp_f || !te || !tb || !ta)
        return -1;
    for (int i = 0; i < len; ++i) {
        x.n[i] = n_in[2 * i] + I * n_in[2 * i + 1];
        x.pz[i] = pz_in[2 * i] + I * pz_in[2 * i + 1];
        x.pt[i] = pt_in[2 * i] + I * pt_in[2 * i + 1];
    }
    fields(b, k, &x, &w, log2_scale, te, tb, ta, e_par, np_c);
    for (int j = 0; j < N; ++j) {
        if (ln_e) ln_e[j] = te[j];
        if (ln_b) ln_b[j] = tb[j];
        if (ln_a) ln_a[j] = ta[j];
    }
    free(x.n); free(x.pz); free(x.pt);
    free(w.rho); free(w.np_c); free(w.dnp_c); free(w.dnp_f);
    free(te); free(tb); free(ta);
    return 0;
}

/* Plain march exposed for the unit tests of the oscillator (complex interleaved arrays). */
int orc_march_io(const orc_beam *b, const double *rho_in, double *np_c, double *dnp_c, double *dnp_f)
{
    const int N = b->n_xi;
    double complex *r = zalloc(N), *a = zalloc(N), *c = zalloc(N), *f = zalloc(N);
    if (!r || !a || !c || !f) return -1;
    for (int j = 0; j < N; ++j) r[j] = rho_in[2 * j] + I * rho_in[2 * j + 1];
    orc_march(b, r, a, c, f);
    for (int j = 0; j < N; ++j) {
        np_c[2 * j] = creal(a[j]); np_c[2 * j + 1] = cimag(a[j]);
        dnp_c[2 * j] = creal(c[j]); dnp_c[2 * j + 1] = cimag(c[j]);
        dnp_f[2 * j] = creal(f[j]); dnp_f[2 * j + 1] = cimag(f[j]);
    }
    free(r); free(a); free(c); free(f);
    return 0;
}

/* Collapse a per-species mode state into the charge and current densities
 *   rho = sum q n,  j_par = sum q n0_face u,  j_perp = sum q n0 w   (complex interleaved [N]). */
int orc_collapse(const orc_beam *b, const double *n_in, const double *pz_in, const double *pt_in,
                 double *rho, double *jpar, double *jperp)
{
    const int N = b->n_xi;
    const double g = b->gamma, g3 = g * g * g;
    for (int j = 0; j < N; ++j) {
        double complex r = 0, a = 0, c = 0;
        for (int s = 0; s < b->n_species; ++s) {
            size_t o = ((size_t)s * N + j) * 2;
            double complex n = n_in[o] + I * n_in[o + 1];
            double complex pz = pz_in[o] + I * pz_in[o + 1];
            double complex pt = pt_in[o] + I * pt_in[o + 1];
            r += b->q[s] * n;
            if (j < N - 1) a += b->q[s] * n0_face(b, s, j) * pz / g3;
            c += b->q[s] * n0_centre(b, s, j) * pt / g;
        }
        rho[2 * j] = creal(r); rho[2 * j + 1] = cimag(r);
        jpar[2 * j] = creal(a); jpar[2 * j + 1] = cimag(a);
        jperp[2 * j] = creal(c); jperp[2 * j + 1] = cimag(c);
    }
    return 0;
}

/* Initial perturbation of one mode, placed on species 0 (only the charge and current
 * densities enter the dynamics).  kind: 0 = random phase noise, 1 = uniform (theta = 0),
 * 2 = impulse at the front (d_tau rho = amp/h in cell 0 at tau = 0+).
 *   noise: rho_j = amp f_j exp(i theta), theta = 2 pi u53(splitmix64(seed, c)),
 *          c = (instance*n_modes_total + mode)*N + j.
 * Outputs n, pz, pt complex interleaved [S*N] (zeroed first). */
int orc_seed_mode(const orc_beam *b, int kind, double amp, double k, uint64_t seed,
                  uint64_t instance, uint64_t mode, uint64_t n_modes_total,
                  double *n_out, double *pz_out, double *pt_out)
{
    const int N = b->n_xi, len = b->n_species * N;
    memset(n_out, 0, sizeof(double) * 2 * len);
    memset(pz_out, 0, sizeof(double) * 2 * len);
    memset(pt_out, 0, sizeof(double) * 2 * len);
    const double q0 = b->q[0];
    if (kind == 0 || kind == 1) {
        for (int j = 0; j < N; ++j) {
            double theta = 0.0;
            if (kind == 0) {
                uint64_t c = (instance * n_modes_total + mode) * (uint64_t)N + (uint64_t)j;
                theta = 2.0 * M_PI * orc_u53(orc_splitmix64(seed, c));
            }
            double complex rho = amp * shape_at(b, j) * cexp(I * theta);
            n_out[2 * j] = creal(rho / q0);
            n_out[2 * j + 1] = cimag(rho / q0);
        }
        return 0;
    }
    if (kind == 2) {
        if (k == 0.0) return -1;
        /* -i k q0 n0 pt / gamma = amp / h  =>  pt = i amp gamma / (h k q0 n0) */
        double n0 = n0_centre(b, 0, 0);
        if (n0 == 0.0) return -1;
        double complex pt = I * amp * b->gamma / (b->h * k * q0 * n0);
        pt_out[0] = creal(pt);
        pt_out[1] = cimag(pt);
        return 0;
    }
    return -1;
}
