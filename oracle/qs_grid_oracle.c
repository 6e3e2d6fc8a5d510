/*
 * qs_grid_oracle.c -- plain FP64 CPU oracle of the finite-width (transverse-grid) form of
 * the linear quasistatic beam-plasma model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product may include, link, load or call this
 * file; it shares no code, header, table or helper with the GPU path.
 *
 * For a beam with a transverse profile the perturbations live on a periodic (x, y) grid
 * instead of a single Fourier mode (Sec. IV.B, where d_y^2 becomes the full transverse
 * Laplacian of Eq. poisson_QSA).  Summed over species (charge density rho, currents j),
 * with Omega(xi, x, y) = sum_s q_s^2 n0_s(xi, x, y) / m_s:
 *
 *   (d_xi^2 + 1) n_p = rho                  per transverse point   Eq. plasma_oscillations_QSA
 *   (1 - Lap_perp) Psi = n_p                per xi slice           Eq. poisson_QSA
 *   d_tau rho   = d_xi j_par - div_perp j_perp                     Eq. beam_continuity (flux form)
 *   d_tau j_par = -gamma^-3 Omega d_xi Psi                         Eq. beam_momentum
 *   d_tau j_perp = +gamma^-1 Omega grad_perp Psi
 *
 * Discretization (readings written down in the design notes): the longitudinal grid,
 * staggering and oscillator propagator of the spectral oracle; transverse points
 * x_i = (i - nx/2) lx/nx (likewise y), periodic; the Helmholtz inverse, gradient and
 * divergence are spectral with this file's own radix-2 FFT: multiplier 1/(1 + kx^2 + ky^2)
 * with k = 2 pi m / l, m in (-n/2, n/2], and i k for derivatives with the Nyquist
 * wavenumber's derivative set to zero; classic RK4 in tau, every stage a full evaluation.
 *
 * Fields at cell centres: E_par = -H[d_xi n_p], E_perp = -grad H[rho - n_p],
 * |B_perp| = |grad H[rho]|, H = (1 - Lap_perp)^-1 (the transverse form of the spectral
 * oracle's fields).
 *
 * Pinned (tests/test_oracle_grid.py): the FFT against a library transform; one transverse
 * Fourier mode in a uniform beam against the spectral oracle; zero density; linearity; the
 * mirror symmetries of the seeds; x <-> y transposition and whole-cell translation of a
 * random problem.  Parity unpinned: the growth of narrow beams beyond these reductions (the
 * paper leaves the geometric factor of the finite-width growth open, Sec. IV.B).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OGR_DROP_LONGITUDINAL 1

typedef struct {
    int nx, ny, n_xi;
    double lx, ly, h, gamma;
    const double *omega;  /* Omega at cell centres, [n_xi][ny][nx] */
    int flags;
} ogr_grid;

uint64_t orc_splitmix64(uint64_t seed, uint64_t i);
double orc_u53(uint64_t x);

/* ------------------------------------------------------------------ FFT */

/* In-place radix-2 decimation-in-time FFT of n = 2^p complex values a[0], a[s], a[2s], ...
 * (Cooley and Tukey 1965): bit-reversal permutation, then butterflies; sign -1 forward. */
static void fft1(double complex *a, int n, int s, int sign)
{
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j |= bit;
        if (i < j) {
            double complex t = a[(size_t)i * s];
            a[(size_t)i * s] = a[(size_t)j * s];
            a[(size_t)j * s] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const double complex w = cexp(I * ang * k);
                const double complex u = a[(size_t)(i + k) * s];
                const double complex v = a[(size_t)(i + k + len / 2) * s] * w;
                a[(size_t)(i + k) * s] = u + v;
                a[(size_t)(i + k + len / 2) * s] = u - v;
            }
    }
}

/* 2D transform of a[y][x]; the inverse includes the 1/(nx ny) factor */
void ogr_fft2(double complex *a, int nx, int ny, int inverse)
{
    const int sign = inverse ? 1 : -1;
    for (int y = 0; y < ny; ++y) fft1(a + (size_t)y * nx, nx, 1, sign);
    for (int x = 0; x < nx; ++x) fft1(a + x, ny, nx, sign);
    if (inverse) {
        const double f = 1.0 / ((double)nx * ny);
        for (size_t i = 0; i < (size_t)nx * ny; ++i) a[i] *= f;
    }
}

static double wavenumber(int i, int n, double l) { return 2.0 * M_PI * (i <= n / 2 ? i : i - n) / l; }
static double derivative_k(int i, int n, double l) { return i == n / 2 ? 0.0 : wavenumber(i, n, l); }

/* out = real part of F^-1[ mult(kx, ky) F(in) ] for one slice, mult one of: */
enum { OP_HELMHOLTZ = 0, OP_DX_HELMHOLTZ = 1, OP_DY_HELMHOLTZ = 2, OP_DX = 3, OP_DY = 4 };

static void spectral_op(const ogr_grid *g, const double *in, double *out, int op, double complex *work)
{
    const int nx = g->nx, ny = g->ny;
    for (size_t i = 0; i < (size_t)nx * ny; ++i) work[i] = in[i];
    ogr_fft2(work, nx, ny, 0);
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const double kx = wavenumber(ix, nx, g->lx), ky = wavenumber(iy, ny, g->ly);
            const double kappa = 1.0 / (1.0 + kx * kx + ky * ky);
            double complex m = 0;
            switch (op) {
            case OP_HELMHOLTZ: m = kappa; break;
            case OP_DX_HELMHOLTZ: m = I * derivative_k(ix, nx, g->lx) * kappa; break;
            case OP_DY_HELMHOLTZ: m = I * derivative_k(iy, ny, g->ly) * kappa; break;
            case OP_DX: m = I * derivative_k(ix, nx, g->lx); break;
            case OP_DY: m = I * derivative_k(iy, ny, g->ly); break;
            }
            work[(size_t)iy * nx + ix] *= m;
        }
    ogr_fft2(work, nx, ny, 1);
    for (size_t i = 0; i < (size_t)nx * ny; ++i) out[i] = creal(work[i]);
}

/* ------------------------------------------------------------------ plasma response */

/* March (d_xi^2 + 1) n_p = rho down every transverse column from n_p = d_xi n_p = 0 at the
 * front, exact for a cell-constant source: n_p at centres, d_xi n_p at centres and at the
 * rear face of each cell. */
static void march(const ogr_grid *g, const double *rho, double *np_c, double *dnp_c, double *dnp_f)
{
    const size_t P = (size_t)g->nx * g->ny;
    const double h = g->h, C = cos(h), S = sin(h), C2 = cos(0.5 * h), S2 = sin(0.5 * h);
    for (size_t p = 0; p < P; ++p) {
        double y = 0.0, v = 0.0;
        for (int j = 0; j < g->n_xi; ++j) {
            const double r = rho[(size_t)j * P + p];
            const double u = y - r;
            if (np_c) np_c[(size_t)j * P + p] = r + C2 * u + S2 * v;
            if (dnp_c) dnp_c[(size_t)j * P + p] = C2 * v - S2 * u;
            const double yn = r + C * u + S * v;
            v = C * v - S * u;
            y = yn;
            if (dnp_f) dnp_f[(size_t)j * P + p] = v;
        }
    }
}

/* ------------------------------------------------------------------ rates and RK4 */

void ogr_rates(const ogr_grid *g, const double *rho, const double *jpar, const double *jx, const double *jy,
               double *drho, double *djpar, double *djx, double *djy)
{
    const size_t P = (size_t)g->nx * g->ny, T = P * g->n_xi;
    double *np_c = calloc(T, sizeof(double)), *dnp_f = calloc(T, sizeof(double));
    double *t1 = calloc(P, sizeof(double)), *t2 = calloc(P, sizeof(double)), *t3 = calloc(P, sizeof(double));
    double *t4 = calloc(P, sizeof(double)), *t5 = calloc(P, sizeof(double));
    double complex *work = calloc(P, sizeof(double complex));
    march(g, rho, np_c, NULL, dnp_f);
    const double ginv = 1.0 / g->gamma;
    const double g3inv = (g->flags & OGR_DROP_LONGITUDINAL) ? 0.0 : 1.0 / (g->gamma * g->gamma * g->gamma);
    for (int j = 0; j < g->n_xi; ++j) {
        const size_t o = (size_t)j * P;
        spectral_op(g, dnp_f + o, t1, OP_HELMHOLTZ, work);     /* d_xi Psi at the rear face */
        spectral_op(g, np_c + o, t2, OP_DX_HELMHOLTZ, work);   /* d_x Psi at the centre */
        spectral_op(g, np_c + o, t3, OP_DY_HELMHOLTZ, work);   /* d_y Psi */
        spectral_op(g, jx + o, t4, OP_DX, work);               /* d_x j_x */
        spectral_op(g, jy + o, t5, OP_DY, work);               /* d_y j_y */
        for (size_t p = 0; p < P; ++p) {
            const double in_front = j > 0 ? jpar[o - P + p] : 0.0;
            drho[o + p] = (jpar[o + p] - in_front) / g->h - (t4[p] + t5[p]);
            if (j < g->n_xi - 1) {
                const double om_face = 0.5 * (g->omega[o + p] + g->omega[o + P + p]);
                djpar[o + p] = -g3inv * om_face * t1[p];
            } else {
                djpar[o + p] = 0.0;   /* no flux through the rear face of the beam */
            }
            djx[o + p] = ginv * g->omega[o + p] * t2[p];
            djy[o + p] = ginv * g->omega[o + p] * t3[p];
        }
    }
    free(np_c); free(dnp_f); free(t1); free(t2); free(t3); free(t4); free(t5); free(work);
}

/* one classic RK4 step of length dtau on the state (rho, jpar, jx, jy) */
void ogr_step(const ogr_grid *g, double dtau, double *rho, double *jpar, double *jx, double *jy)
{
    const size_t T = (size_t)g->nx * g->ny * g->n_xi;
    double *x[4] = {rho, jpar, jx, jy};
    double *k[4][4], *y[4];
    for (int s = 0; s < 4; ++s)
        for (int v = 0; v < 4; ++v) k[s][v] = calloc(T, sizeof(double));
    for (int v = 0; v < 4; ++v) y[v] = calloc(T, sizeof(double));
    const double a[4] = {0.0, 0.5, 0.5, 1.0};
    for (int s = 0; s < 4; ++s) {
        for (int v = 0; v < 4; ++v)
            for (size_t i = 0; i < T; ++i) y[v][i] = x[v][i] + (s ? a[s] * dtau * k[s - 1][v][i] : 0.0);
        ogr_rates(g, y[0], y[1], y[2], y[3], k[s][0], k[s][1], k[s][2], k[s][3]);
    }
    for (int v = 0; v < 4; ++v)
        for (size_t i = 0; i < T; ++i)
            x[v][i] += dtau / 6.0 * (k[0][v][i] + 2.0 * k[1][v][i] + 2.0 * k[2][v][i] + k[3][v][i]);
    for (int s = 0; s < 4; ++s)
        for (int v = 0; v < 4; ++v) free(k[s][v]);
    for (int v = 0; v < 4; ++v) free(y[v]);
}

/* |E|^2 and |B|^2 at cell centres for the charge density rho */
void ogr_fields(const ogr_grid *g, const double *rho, double *e2, double *b2)
{
    const size_t P = (size_t)g->nx * g->ny, T = P * g->n_xi;
    double *np_c = calloc(T, sizeof(double)), *dnp_c = calloc(T, sizeof(double));
    double *d = calloc(P, sizeof(double)), *ep = calloc(P, sizeof(double));
    double *ex = calloc(P, sizeof(double)), *ey = calloc(P, sizeof(double));
    double *bx = calloc(P, sizeof(double)), *by = calloc(P, sizeof(double));
    double complex *work = calloc(P, sizeof(double complex));
    march(g, rho, np_c, dnp_c, NULL);
    for (int j = 0; j < g->n_xi; ++j) {
        const size_t o = (size_t)j * P;
        for (size_t p = 0; p < P; ++p) d[p] = rho[o + p] - np_c[o + p];
        spectral_op(g, dnp_c + o, ep, OP_HELMHOLTZ, work);     /* -E_par */
        spectral_op(g, d, ex, OP_DX_HELMHOLTZ, work);          /* -E_perp */
        spectral_op(g, d, ey, OP_DY_HELMHOLTZ, work);
        spectral_op(g, rho + o, bx, OP_DX_HELMHOLTZ, work);    /* |B_perp| components */
        spectral_op(g, rho + o, by, OP_DY_HELMHOLTZ, work);
        for (size_t p = 0; p < P; ++p) {
            e2[o + p] = ep[p] * ep[p] + ex[p] * ex[p] + ey[p] * ey[p];
            b2[o + p] = bx[p] * bx[p] + by[p] * by[p];
        }
    }
    free(np_c); free(dnp_c); free(d); free(ep); free(ex); free(ey); free(bx); free(by); free(work);
}

/* Run n_steps; at the start of every step s with s % out_every == 0 the fields are written
 * to ln_e/ln_b [snap][T] (natural logs of |E|, |B|), and at the start of every step
 * max_ln_a[s] = ln max over all cells of (|E|^2 + |B|^2)^(1/2).  Any output may be NULL. */
void ogr_run(const ogr_grid *g, double dtau, int n_steps, int out_every, double *rho, double *jpar, double *jx,
             double *jy, double *ln_e, double *ln_b, double *max_ln_a)
{
    const size_t T = (size_t)g->nx * g->ny * g->n_xi;
    double *e2 = calloc(T, sizeof(double)), *b2 = calloc(T, sizeof(double));
    int snap = 0;
    for (int s = 0; s < n_steps; ++s) {
        const int want_snap = ln_e && (s % out_every == 0);
        if (want_snap || max_ln_a) {
            ogr_fields(g, rho, e2, b2);
            double mx = 0.0;
            for (size_t i = 0; i < T; ++i) mx = fmax(mx, e2[i] + b2[i]);
            if (max_ln_a) max_ln_a[s] = 0.5 * log(mx);
            if (want_snap) {
                for (size_t i = 0; i < T; ++i) {
                    ln_e[(size_t)snap * T + i] = 0.5 * log(e2[i]);
                    ln_b[(size_t)snap * T + i] = 0.5 * log(b2[i]);
                }
                ++snap;
            }
        }
        ogr_step(g, dtau, rho, jpar, jx, jy);
    }
    free(e2); free(b2);
}

/* ------------------------------------------------------------------ seeds */

/* Beam charge perturbation of the finite-width seeds, rho[j][iy][ix] with
 * f = longitudinal profile at centre j (NULL = 1), g = exp(-r^2 / (2 sigma_r^2)) (1 when
 * sigma_r <= 0), x_i = (i - nx/2) lx/nx:
 *   kind 0 (noise):    amp (2u - 1) f g
 *   kind 1 (uniform):  amp f g
 *   kind 3 (centroid): offset (x / sigma_r^2) f g + amp (2u - 1) f g
 * u = top 53 bits of SplitMix64 output (j ny + iy) nx + ix of `seed`, over 2^53. */
void ogr_seed(const ogr_grid *g, int kind, double amp, double offset, double sigma_r, const double *f,
              uint64_t seed, double *rho)
{
    const int nx = g->nx, ny = g->ny;
    for (int j = 0; j < g->n_xi; ++j)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const double x = (ix - nx / 2) * g->lx / nx, y = (iy - ny / 2) * g->ly / ny;
                const double gg = sigma_r > 0.0 ? exp(-(x * x + y * y) / (2.0 * sigma_r * sigma_r)) : 1.0;
                const double fg = (f ? f[j] : 1.0) * gg;
                const size_t idx = ((size_t)j * ny + iy) * nx + ix;
                const double u = orc_u53(orc_splitmix64(seed, idx));
                double r = 0.0;
                if (kind == 0) r = amp * (2.0 * u - 1.0) * fg;
                else if (kind == 1) r = amp * fg;
                else if (kind == 3) r = (sigma_r > 0.0 ? offset * x / (sigma_r * sigma_r) : 0.0) * fg + amp * (2.0 * u - 1.0) * fg;
                rho[idx] = r;
            }
}
