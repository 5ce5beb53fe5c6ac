/*
 * gpe_oracle.c -- plain FP64 CPU reference for the 2D split-step Gross-Pitaevskii
 * propagation of arXiv:2404.14401.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; it exists so that the GPU library can be checked against an
 * independent, slow and obviously correct implementation.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Everything is double precision, one operation per loop, in the order the
 * paper states it:
 *   - the GPE and its Hamiltonian split T + V                 (Sec. 2, Eq. 1; Sec. 3.1)
 *   - symmetric split-step: half potential kick, kinetic
 *     propagation in Fourier space, half potential kick       (Sec. 3.1, Eqs. 3-4; the
 *                                                              V/2-T-V/2 ordering of the
 *                                                              same factorisation)
 *   - the FFT imposes periodic boundaries on the grid         (Sec. 3.1)
 *   - the non-linear potential is re-evaluated on the most
 *     recent wave function at every kick                      (Sec. 3.1)
 *   - dimensionless oscillator units, hbar = m = 1            (Sec. 3.2)
 *   - imaginary time dt -> -i dtau, normalise after every
 *     step                                                    (Sec. 3.3)
 *   - optical lattice V0 cos^2(k y)                           (Sec. 5.2, Eq. 9)
 *   - cavity potential V_t + V_p + V_c + V_i                  (Sec. 5.3, Eqs. 10-13)
 *   - cavity field driven by the overlap
 *     <psi| cos kx cos ky |psi>                               (Sec. 5.3, Eq. 14), here as
 *                                                              the driven-damped ODE
 *     d alpha/dt = (i Delta_c - kappa) alpha - i eta Theta, whose fixed point is Eq. 14
 *     with eta standing for N sqrt(V0 U0) and the undressed detuning (cavity = 1);
 *     or Eq. 14 itself, recomputed from the current density before every kick, with
 *     the dispersively shifted detuning of Eq. 15 (cavity = 2).
 *
 * The FFT is an iterative radix-2 Cooley-Tukey transform (bit reversal, then
 * butterflies) with every twiddle factor taken from cos/sin of its own index.
 * A literal O(N^2) DFT is provided next to it so the FFT can be pinned.
 *
 * Conventions: psi is stored row-major [ny][nx] (x fastest); x_i = -Lx/2 + i Lx/Nx;
 * k_j = (2 pi / L)(j - N [j >= N/2]); forward transform exp(-2 pi i jk/N) unscaled,
 * inverse exp(+2 pi i jk/N) scaled by 1/N.
 *
 * OpenMP is used only to run independent rows / columns / instances at once; every
 * reduction is a serial loop in a fixed order, so results do not depend on the
 * thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ problem */

/* Lattice-depth schedule.  kind 0: constant v0.  kind 1: linear ramp from v0 at t0
 * to v1 at t1, clamped outside.  kind 2: piecewise-linear through nknots values
 * placed evenly on [t0, t1], clamped outside. */
typedef struct {
    int kind;
    int nknots;
    double v0, v1, t0, t1;
    const double *knots;
} orc_sched;

typedef struct {
    int nx, ny;
    double lx, ly;
    double dt;
    double g;
    /* harmonic trap 1/2 wx^2 (x-x0)^2 + 1/2 wy^2 (y-y0)^2 (Sec. 5.1) */
    double wx, wy, x0, y0;
    /* lattices Vx(t) cos^2(kx x) and Vy(t) cos^2(ky y) (Sec. 5.2) */
    double kx_lat, ky_lat;
    orc_sched sx, sy;
    /* cavity (Sec. 5.3): the pump is the y lattice, depth Vy(t), wavenumber kc.
     * cavity 0: off; 1: field from the driven-damped ODE (coupling eta); 2: field from
     * the adiabatic expression of Eqs. 14-15 with n_atoms atoms (eta unused) */
    int cavity;
    double vc, kc, delta_c, kappa, eta;
    /* optional extra static potential [ny][nx] (may be NULL) */
    const double *vuser;
    double n_atoms;
    /* on-axis cavity probe of the adiabatic field (Sec. 5.4): strength Omega_c,
     * detuning Delta_p from the pump, phase phi */
    double probe_omega, probe_detuning, probe_phase;
} orc_problem;

/* Propagation state carried between calls. */
typedef struct {
    double t;          /* current real time */
    double alpha_re;   /* cavity field */
    double alpha_im;
    double theta;      /* Theta_n of the current psi */
    double theta_prev; /* Theta_{n-1} */
    int have_theta;    /* 0 before the first real-time step */
} orc_state;

static double sched_eval(const orc_sched *s, double t)
{
    if (s->kind == 0) return s->v0;
    if (s->kind == 1) {
        if (t <= s->t0) return s->v0;
        if (t >= s->t1) return s->v1;
        return s->v0 + (s->v1 - s->v0) * (t - s->t0) / (s->t1 - s->t0);
    }
    /* kind 3: the light shift of a lattice flashed on for t0 <= t < t1, the unit
     * pulse Pi of Sec. 5.2 (v1 outside the pulse) */
    if (s->kind == 3) return (t >= s->t0 && t < s->t1) ? s->v0 : s->v1;
    /* kind 2: knots */
    int m = s->nknots;
    if (m == 1 || t <= s->t0) return s->knots[0];
    if (t >= s->t1) return s->knots[m - 1];
    double u = (t - s->t0) / (s->t1 - s->t0) * (m - 1);
    int i = (int)floor(u);
    if (i >= m - 1) i = m - 2;
    double w = u - i;
    return (1.0 - w) * s->knots[i] + w * s->knots[i + 1];
}

static double xcoord(const orc_problem *p, int i) { return -0.5 * p->lx + i * (p->lx / p->nx); }
static double ycoord(const orc_problem *p, int j) { return -0.5 * p->ly + j * (p->ly / p->ny); }

static double kval(int j, int n, double len)
{
    int m = (j >= n / 2) ? j - n : j;
    return 2.0 * M_PI * m / len;
}

/* External potential at a point (Sec. 5.1-5.3).  Cavity terms: U0|alpha|^2 cos^2(kx)
 * and 2 sqrt(V0 U0) Re(alpha) cos(kx) cos(ky) with V0 the current pump depth. */
static double potential(const orc_problem *p, int i, int j, double t, cplx alpha)
{
    double x = xcoord(p, i), y = ycoord(p, j);
    double v = 0.5 * p->wx * p->wx * (x - p->x0) * (x - p->x0)
             + 0.5 * p->wy * p->wy * (y - p->y0) * (y - p->y0);
    double vx = sched_eval(&p->sx, t), vy = sched_eval(&p->sy, t);
    double cx = cos(p->kx_lat * x), cy = cos(p->ky_lat * y);
    v += vx * cx * cx + vy * cy * cy;
    if (p->cavity) {
        double ccx = cos(p->kc * x), ccy = cos(p->kc * y);
        double a2 = creal(alpha) * creal(alpha) + cimag(alpha) * cimag(alpha);
        v += p->vc * a2 * ccx * ccx;
        v += 2.0 * sqrt(vy * p->vc) * creal(alpha) * ccx * ccy;
    }
    if (p->vuser) v += p->vuser[(size_t)j * p->nx + i];
    return v;
}

/* ---------------------------------------------------------------------- FFT */

/* Literal DFT of one line: X_k = sum_j x_j exp(-+2 pi i jk/n), inverse scaled 1/n. */
void orc_dft1d(const cplx *in, cplx *out, int n, int inverse)
{
    double sgn = inverse ? 1.0 : -1.0;
    for (int k = 0; k < n; k++) {
        cplx s = 0;
        for (int j = 0; j < n; j++) {
            double ang = sgn * 2.0 * M_PI * (double)(((int64_t)j * k) % n) / n;
            s += in[j] * (cos(ang) + I * sin(ang));
        }
        out[k] = inverse ? s / n : s;
    }
}

/* Literal 2D DFT, the double sum written out (tiny grids only). */
void orc_dft2d(const cplx *in, cplx *out, int nx, int ny, int inverse)
{
    double sgn = inverse ? 1.0 : -1.0;
    for (int ky = 0; ky < ny; ky++)
        for (int kx = 0; kx < nx; kx++) {
            cplx s = 0;
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    double ang = sgn * 2.0 * M_PI *
                        ((double)(((int64_t)x * kx) % nx) / nx + (double)(((int64_t)y * ky) % ny) / ny);
                    s += in[(size_t)y * nx + x] * (cos(ang) + I * sin(ang));
                }
            out[(size_t)ky * nx + kx] = inverse ? s / ((double)nx * ny) : s;
        }
}

/* Twiddles w[j] = exp(-2 pi i j / n), j < n/2, each from cos/sin of its own index. */
static cplx *make_twiddles(int n)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(n / 2 > 0 ? n / 2 : 1));
    for (int j = 0; j < n / 2; j++) {
        double ang = -2.0 * M_PI * j / n;
        w[j] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* In-place iterative radix-2 FFT of length n (a power of two). */
static void fft_line(cplx *a, int n, int inverse, const cplx *w)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int j = 0; j < half; j++) {
                cplx tw = inverse ? conj(w[j * step]) : w[j * step];
                cplx u = a[i + j], v = a[i + j + half] * tw;
                a[i + j] = u + v;
                a[i + j + half] = u - v;
            }
    }
    if (inverse)
        for (int i = 0; i < n; i++) a[i] /= n;
}

void orc_fft1d(cplx *a, int n, int inverse)
{
    cplx *w = make_twiddles(n);
    fft_line(a, n, inverse, w);
    free(w);
}

/* 2D transform: every row, then every column. */
void orc_fft2d(cplx *a, int nx, int ny, int inverse)
{
    cplx *wx = make_twiddles(nx), *wy = make_twiddles(ny);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) fft_line(a + (size_t)j * nx, nx, inverse, wx);
#pragma omp parallel
    {
        cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
#pragma omp for schedule(static)
        for (int i = 0; i < nx; i++) {
            for (int j = 0; j < ny; j++) col[j] = a[(size_t)j * nx + i];
            fft_line(col, ny, inverse, wy);
            for (int j = 0; j < ny; j++) a[(size_t)j * nx + i] = col[j];
        }
        free(col);
    }
    free(wx);
    free(wy);
}

/* ------------------------------------------------------------ split step */

/* Potential kick psi <- psi exp(-i (V + g|psi|^2) h) in real time, or
 * psi <- psi exp(-(V + g|psi|^2) h) in imaginary time (Sec. 3.1, Sec. 3.3). */
static void kick(const orc_problem *p, cplx *psi, double t, cplx alpha, double h, int imag)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
            double th = (potential(p, i, j, t, alpha) + p->g * dens) * h;
            if (imag)
                psi[q] *= exp(-th);
            else
                psi[q] *= cos(th) - I * sin(th);
        }
}

/* Kinetic propagation over a full dt in Fourier space: exp(-i k^2 dt / 2)
 * (imaginary time: exp(-k^2 dt / 2)), hbar = m = 1 (Sec. 3.1-3.3). */
static void kinetic(const orc_problem *p, cplx *psi, int imag)
{
    orc_fft2d(psi, p->nx, p->ny, 0);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; j++) {
        double ky = kval(j, p->ny, p->ly);
        for (int i = 0; i < p->nx; i++) {
            double kx = kval(i, p->nx, p->lx);
            double ph = 0.5 * (kx * kx + ky * ky) * p->dt;
            size_t q = (size_t)j * p->nx + i;
            if (imag)
                psi[q] *= exp(-ph);
            else
                psi[q] *= cos(ph) - I * sin(ph);
        }
    }
    orc_fft2d(psi, p->nx, p->ny, 1);
}

/* Reductions over the real-space wave function, dA = dx dy (Sec. 3.3, Sec. 5.3). */
double orc_norm(const orc_problem *p, const cplx *psi)
{
    double s = 0, da = (p->lx / p->nx) * (p->ly / p->ny);
    for (size_t q = 0; q < (size_t)p->nx * p->ny; q++)
        s += creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
    return s * da;
}

/* Theta = integral cos(kc x) cos(kc y) |psi|^2 dx dy  (Sec. 5.3, Eq. 14 numerator). */
double orc_theta(const orc_problem *p, const cplx *psi)
{
    double s = 0, da = (p->lx / p->nx) * (p->ly / p->ny);
    for (int j = 0; j < p->ny; j++) {
        double cy = cos(p->kc * ycoord(p, j));
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
            s += cos(p->kc * xcoord(p, i)) * cy * dens;
        }
    }
    return s * da;
}

/* C = integral cos^2(kc x) |psi|^2 dx dy, the overlap in the dispersive shift
 * (Sec. 5.3, Eq. 15). */
double orc_cos2(const orc_problem *p, const cplx *psi)
{
    double s = 0, da = (p->lx / p->nx) * (p->ly / p->ny);
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
            double c = cos(p->kc * xcoord(p, i));
            s += c * c * dens;
        }
    return s * da;
}

/* The adiabatic cavity field of the density of psi at time t (Sec. 5.3, Eqs. 14-15):
 *   alpha = N sqrt(Vp(t) U0) Theta / (Delta_c~ + i kappa),
 *   Delta_c~ = Delta_c - N U0 C,
 * Theta and C per unit norm (psi describes one atom; N = n_atoms counts them in both
 * the coupling and the shift), U0 = vc, Vp(t) the pump (y lattice) depth.  With the
 * on-axis probe of Sec. 5.4 the field becomes alpha + delta alpha(t),
 *   delta alpha = Omega_c exp(i (Delta_p t + phi)) / (Delta_c~ + i kappa). */
static cplx alpha_adiabatic(const orc_problem *p, const cplx *psi, double t)
{
    double nrm = orc_norm(p, psi);
    double th = orc_theta(p, psi) / nrm, c2 = orc_cos2(p, psi) / nrm;
    double vp = sched_eval(&p->sy, t);
    double dtil = p->delta_c - p->n_atoms * p->vc * c2;
    cplx alpha = p->n_atoms * sqrt(vp * p->vc) * th / (dtil + I * p->kappa);
    cplx dalpha = p->probe_omega * cexp(I * (p->probe_detuning * t + p->probe_phase)) / (dtil + I * p->kappa);
    return alpha + dalpha;
}

void orc_alpha_adiabatic(const orc_problem *p, const cplx *psi, double t, double *out)
{
    cplx a = alpha_adiabatic(p, psi, t);
    out[0] = creal(a);
    out[1] = cimag(a);
}

/* <x>, <y> (unnormalised integrals of x|psi|^2 and y|psi|^2). */
void orc_moments(const orc_problem *p, const cplx *psi, double *mx, double *my)
{
    double sx = 0, sy = 0, da = (p->lx / p->nx) * (p->ly / p->ny);
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
            sx += xcoord(p, i) * dens;
            sy += ycoord(p, j) * dens;
        }
    *mx = sx * da;
    *my = sy * da;
}

/* Cavity-field update over one step: exponential integrator of
 * d alpha/dt = lambda alpha - i eta Theta(t), lambda = i Delta_c - kappa, with the
 * forcing extrapolated to second order, Theta_bar = (3 Theta_n - Theta_{n-1}) / 2:
 *   alpha_{n+1} = e^{lambda dt} alpha_n + (e^{lambda dt} - 1)/lambda * (-i eta Theta_bar).
 * Exact when Theta is constant.  (The adiabatic value of Sec. 5.3, Eq. 14, is this
 * ODE's fixed point.) */
static cplx cavity_advance(const orc_problem *p, cplx alpha, double theta_n, double theta_prev)
{
    cplx lam = I * p->delta_c - p->kappa;
    cplx e = cexp(lam * p->dt);
    double tb = 0.5 * (3.0 * theta_n - theta_prev);
    cplx phi1 = (cabs(lam) > 0) ? (e - 1.0) / lam : p->dt;
    return e * alpha + phi1 * (-I * p->eta * tb);
}

/* Optional per-step observables: for each step n, record
 * {norm, Theta, Re alpha, Im alpha, <x>, <y>} of psi_{n+1}.  */
#define ORC_NOBS 6

static void record(const orc_problem *p, const cplx *psi, cplx alpha, double theta, double *obs)
{
    if (!obs) return;
    obs[0] = orc_norm(p, psi);
    obs[1] = theta;
    obs[2] = creal(alpha);
    obs[3] = cimag(alpha);
    orc_moments(p, psi, &obs[4], &obs[5]);
}

/* Real-time split step, n times (Sec. 3.1):
 *   1. (cavity) alpha_{n+1} from alpha_n, Theta_n, Theta_{n-1}
 *   2. psi' = psi_n exp(-i [V(t_n; alpha_n) + g|psi_n|^2] dt/2)
 *   3. psi* = IFFT2( exp(-i k^2 dt/2) FFT2(psi') )
 *   4. psi_{n+1} = psi* exp(-i [V(t_{n+1}; alpha_{n+1}) + g|psi*|^2] dt/2)
 *   5. (cavity) Theta_{n+1} from psi_{n+1}
 * With the adiabatic field (cavity 2) steps 1 and 5 are replaced by alpha evaluated
 * from the density about to be kicked: alpha(psi_n, t_n) in 2, alpha(psi*, t_{n+1}) in 4.
 * obs (nullable): nsteps * ORC_NOBS doubles. */
int orc_step_real(const orc_problem *p, orc_state *s, cplx *psi, int64_t nsteps, double *obs)
{
    double h = 0.5 * p->dt;
    cplx alpha = s->alpha_re + I * s->alpha_im;
    if (p->cavity == 2) {
        for (int64_t n = 0; n < nsteps; n++) {
            double tn = s->t, tn1 = s->t + p->dt;
            kick(p, psi, tn, alpha_adiabatic(p, psi, tn), h, 0);
            kinetic(p, psi, 0);
            alpha = alpha_adiabatic(p, psi, tn1);
            kick(p, psi, tn1, alpha, h, 0);
            s->t = tn1;
            if (obs) record(p, psi, alpha, orc_theta(p, psi), obs + n * ORC_NOBS);
        }
        s->alpha_re = creal(alpha);
        s->alpha_im = cimag(alpha);
        return 0;
    }
    if (p->cavity && !s->have_theta) {
        s->theta = orc_theta(p, psi);
        s->theta_prev = s->theta;
        s->have_theta = 1;
    }
    for (int64_t n = 0; n < nsteps; n++) {
        double tn = s->t, tn1 = s->t + p->dt;
        cplx alpha1 = alpha;
        if (p->cavity) alpha1 = cavity_advance(p, alpha, s->theta, s->theta_prev);
        kick(p, psi, tn, alpha, h, 0);
        kinetic(p, psi, 0);
        kick(p, psi, tn1, alpha1, h, 0);
        double th = 0;
        if (p->cavity || obs) th = orc_theta(p, psi);
        if (p->cavity) {
            s->theta_prev = s->theta;
            s->theta = th;
        }
        alpha = alpha1;
        s->t = tn1;
        record(p, psi, alpha, th, obs ? obs + n * ORC_NOBS : NULL);
    }
    s->alpha_re = creal(alpha);
    s->alpha_im = cimag(alpha);
    return 0;
}

/* Imaginary-time split step (Sec. 3.3): dt -> -i dtau in every factor, potential
 * frozen at time s->t, then psi <- psi / sqrt(norm).  The ODE cavity field is held
 * fixed; the adiabatic one (cavity 2) is evaluated once per step from the state
 * entering it (the kicks change the density in imaginary time, so one value per step
 * is taken, and a converged state is then a fixed point of the frozen-field step);
 * the state's field afterwards is that of the returned psi. */
int orc_step_imag(const orc_problem *p, orc_state *s, cplx *psi, int64_t nsteps, double *obs)
{
    double h = 0.5 * p->dt;
    cplx alpha = s->alpha_re + I * s->alpha_im;
    size_t npts = (size_t)p->nx * p->ny;
    for (int64_t n = 0; n < nsteps; n++) {
        if (p->cavity == 2) alpha = alpha_adiabatic(p, psi, s->t);
        kick(p, psi, s->t, alpha, h, 1);
        kinetic(p, psi, 1);
        kick(p, psi, s->t, alpha, h, 1);
        double nrm = orc_norm(p, psi);
        double sc = 1.0 / sqrt(nrm);
        for (size_t q = 0; q < npts; q++) psi[q] *= sc;
        if (obs) {
            double *o = obs + n * ORC_NOBS;
            record(p, psi, alpha, orc_theta(p, psi), o);
            o[0] = nrm; /* pre-normalisation norm: -ln(o[0]) / (2 dtau) estimates mu */
        }
    }
    if (p->cavity == 2 && nsteps > 0) {
        /* the field that belongs to the returned state */
        alpha = alpha_adiabatic(p, psi, s->t);
        s->alpha_re = creal(alpha);
        s->alpha_im = cimag(alpha);
    }
    return 0;
}

/* Energy functional of psi at time t (validation, Sec. 5.1):
 *   E_kin = dA/(NxNy) sum_k |k|^2/2 |FFT2(psi)_k|^2
 *   E_pot = dA sum V |psi|^2,  E_int = g/2 dA sum |psi|^4
 *   mu = E_kin + E_pot + 2 E_int; every term divided by the norm.
 * out = {E_kin, E_pot, E_int, E, mu, norm}. */
void orc_energy(const orc_problem *p, const cplx *psi, double t, double alpha_re, double alpha_im,
                double *out)
{
    size_t npts = (size_t)p->nx * p->ny;
    double da = (p->lx / p->nx) * (p->ly / p->ny);
    cplx alpha = alpha_re + I * alpha_im;
    cplx *f = (cplx *)malloc(sizeof(cplx) * npts);
    memcpy(f, psi, sizeof(cplx) * npts);
    orc_fft2d(f, p->nx, p->ny, 0);
    double ek = 0, ep = 0, ei = 0, nrm = 0;
    for (int j = 0; j < p->ny; j++) {
        double ky = kval(j, p->ny, p->ly);
        for (int i = 0; i < p->nx; i++) {
            double kx = kval(i, p->nx, p->lx);
            size_t q = (size_t)j * p->nx + i;
            double a2 = creal(f[q]) * creal(f[q]) + cimag(f[q]) * cimag(f[q]);
            ek += 0.5 * (kx * kx + ky * ky) * a2;
        }
    }
    ek *= da / (double)npts;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
            ep += potential(p, i, j, t, alpha) * dens;
            ei += dens * dens;
            nrm += dens;
        }
    ep *= da;
    ei *= 0.5 * p->g * da;
    nrm *= da;
    free(f);
    out[0] = ek / nrm;
    out[1] = ep / nrm;
    out[2] = ei / nrm;
    out[3] = (ek + ep + ei) / nrm;
    out[4] = (ek + ep + 2.0 * ei) / nrm;
    out[5] = nrm;
}

/* Potential on the whole grid (for tests and plots). */
void orc_potential_grid(const orc_problem *p, double t, double alpha_re, double alpha_im, double *v)
{
    cplx alpha = alpha_re + I * alpha_im;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) v[(size_t)j * p->nx + i] = potential(p, i, j, t, alpha);
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------- adjoint */
/*
 * Discrete adjoint of the real-time split step with respect to the knot values
 * c_m of a piecewise-linear lattice-depth schedule Vx(t) = sum_m c_m w_m(t) (the
 * time-dependent lattice of Sec. 5.2 used as a control).  The paper has no
 * gradient; this is the exact reverse-mode derivative of the discrete map defined
 * by orc_step_real (cavity off), written in the real-gradient convention
 *   G = dL/d(Re psi) + i dL/d(Im psi),  dL = Re sum conj(G) d psi.
 * Per kick psi' = psi e^{-i theta}, theta = (V + g|psi|^2) h:
 *   s = Im(conj(G') psi'),  G = G' e^{+i theta} + 2 g h s psi,  dL/dV(x) = h s(x).
 * Per kinetic propagation psi* = U psi' (U = IFFT2 M FFT2, unitary):
 *   G = IFFT2(conj(M) FFT2(G')).
 * Losses: kind 0, L = 1 - |<target|psi(T)>|^2 with <a|b> = sum conj(a) b dA
 *   (terminal G = -2 c target dA, c = <target|psi(T)>);
 *   kind 1, L = E_kin + E_pot + E_int of psi(T) at time T (norm conserved in real time;
 *   terminal G = 2 dA (T psi + V psi + g|psi|^2 psi)).
 * Forward states are kept as checkpoints every `ckpt` steps; each segment is
 * recomputed forward before it is swept backward, so the gradient is the exact
 * adjoint of this file's own forward map.
 * The controlled lattice is the x lattice (axis 0) or the y lattice (axis 1), the
 * pump of the cavity set-up (Sec. 5.3); dV/dc_m is w_m(t) cos^2(k_lat u) along that
 * axis, plus, with the adiabatic cavity field, the pump's share in the interference
 * lattice and in alpha (see kick_adjoint_cavity; fidelity loss only there).
 */

/* cos^2 of the controlled lattice at grid point (i, j) */
static double control_weight(const orc_problem *p, int axis, int i, int j)
{
    double c = axis == 0 ? cos(p->kx_lat * xcoord(p, i)) : cos(p->ky_lat * ycoord(p, j));
    return c * c;
}

static void hat_weights(const orc_sched *s, double t, int *i0, double *w0, double *w1)
{
    int m = s->nknots;
    if (m == 1 || t <= s->t0) { *i0 = 0; *w0 = 1; *w1 = 0; return; }
    if (t >= s->t1) { *i0 = m - 2; *w0 = 0; *w1 = 1; return; }
    double u = (t - s->t0) / (s->t1 - s->t0) * (m - 1);
    int i = (int)floor(u);
    if (i >= m - 1) i = m - 2;
    *i0 = i;
    *w1 = u - i;
    *w0 = 1.0 - *w1;
}

/* Backward through one kick at time t.  zout is the kick's output; on return z holds
 * its input (reconstructed exactly as zout e^{+i theta}, |z| = |zout|) and G the
 * gradient with respect to it.  Accumulates dL/dc into grad. */
/* Backward through one kick with the adiabatic cavity field (cavity 2).  The field
 * alpha(rho, t) of Eqs. 14-15 depends on the density through Theta^ = Theta/Nrm and
 * C^ = C/Nrm, so besides the local terms the kick has a global one:
 *   A = sum_x s dV/dalpha = 2 U0 alpha S_c + 2 sqrt(Vp U0) S_x    (S_c = sum s cos^2 kx,
 *       S_x = sum s cos kx cos ky, s = Im(conj(G') psi')),
 *   b_T = Re(conj(A) dalpha/dTheta^), b_C = Re(conj(A) dalpha/dC^),
 *   dalpha/dTheta^ = N sqrt(Vp U0)/(D~ + i kappa), dalpha/dC^ = alpha N U0/(D~ + i kappa),
 *   G = G' e^{i theta} + 2 w psi,
 *   w = h [g s + (b_T (cos kx cos ky - Theta^) + b_C (cos^2 kx - C^)) dA / Nrm].
 * Control: the x lattice enters only through h sum s cos^2(kx_lat x); the pump through
 *   h [sum s cos^2(ky_lat y) + (U0/sqrt(Vp U0)) Re(alpha) S_x + Re(conj(A) dalpha/dVp)],
 *   dalpha/dVp = N U0 Theta^ / (2 sqrt(Vp U0) (D~ + i kappa))  (finite for Vp U0 > 0). */
static void kick_adjoint_cavity(const orc_problem *p, int axis, const cplx *zout, cplx *z, cplx *G, double t,
                                double h, double *grad)
{
    double da = (p->lx / p->nx) * (p->ly / p->ny);
    double nrm = orc_norm(p, zout);
    double thn = orc_theta(p, zout) / nrm, c2n = orc_cos2(p, zout) / nrm;
    cplx alpha = alpha_adiabatic(p, zout, t);
    double vp = sched_eval(&p->sy, t), sq = sqrt(vp * p->vc);
    cplx dplus = (p->delta_c - p->n_atoms * p->vc * c2n) + I * p->kappa;
    double s_c = 0, s_x = 0, s_ctl = 0;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double s = cimag(conj(G[q]) * zout[q]);
            double cx = cos(p->kc * xcoord(p, i)), cy = cos(p->kc * ycoord(p, j));
            s_c += s * cx * cx;
            s_x += s * cx * cy;
            s_ctl += s * control_weight(p, axis, i, j);
        }
    cplx A = 2.0 * p->vc * alpha * s_c + 2.0 * sq * s_x;
    cplx a_th = p->n_atoms * sq / dplus, a_c = alpha * p->n_atoms * p->vc / dplus;
    double b_th = creal(conj(A) * a_th), b_c = creal(conj(A) * a_c);
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(zout[q]) * creal(zout[q]) + cimag(zout[q]) * cimag(zout[q]);
            double th = (potential(p, i, j, t, alpha) + p->g * dens) * h;
            cplx e = cos(th) + I * sin(th);
            cplx zin = zout[q] * e;
            double s = cimag(conj(G[q]) * zout[q]);
            double cx = cos(p->kc * xcoord(p, i)), cy = cos(p->kc * ycoord(p, j));
            double w = h * (p->g * s + (b_th * (cx * cy - thn) + b_c * (cx * cx - c2n)) * da / nrm);
            G[q] = G[q] * e + 2.0 * w * zin;
            z[q] = zin;
        }
    double lat_sum = h * s_ctl;
    if (axis == 1) {
        cplx a_v = p->n_atoms * p->vc * thn / (2.0 * sq * dplus);
        lat_sum += h * ((p->vc / sq) * creal(alpha) * s_x + creal(conj(A) * a_v));
    }
    const orc_sched *ctl = axis == 0 ? &p->sx : &p->sy;
    if (grad && ctl->kind == 2) {
        int i0; double w0, w1;
        hat_weights(ctl, t, &i0, &w0, &w1);
        grad[i0] += w0 * lat_sum;
        grad[i0 + 1] += w1 * lat_sum;
    }
}

static void kick_adjoint(const orc_problem *p, int axis, const cplx *zout, cplx *z, cplx *G, double t, double h,
                         double *grad)
{
    if (p->cavity == 2) {
        kick_adjoint_cavity(p, axis, zout, z, G, t, h, grad);
        return;
    }
    double lat_sum = 0;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t q = (size_t)j * p->nx + i;
            double dens = creal(zout[q]) * creal(zout[q]) + cimag(zout[q]) * cimag(zout[q]);
            double th = (potential(p, i, j, t, 0) + p->g * dens) * h;
            cplx e = cos(th) + I * sin(th);
            cplx zin = zout[q] * e;
            double s = cimag(conj(G[q]) * zout[q]);
            G[q] = G[q] * e + 2.0 * p->g * h * s * zin;
            z[q] = zin;
            lat_sum += h * s * control_weight(p, axis, i, j);
        }
    const orc_sched *ctl = axis == 0 ? &p->sx : &p->sy;
    if (grad && ctl->kind == 2) {
        int i0; double w0, w1;
        hat_weights(ctl, t, &i0, &w0, &w1);
        grad[i0] += w0 * lat_sum;
        grad[i0 + 1] += w1 * lat_sum;
    }
}

/* Backward through the kinetic propagation: G <- IFFT2(conj(M) FFT2(G)). */
static void kinetic_adjoint(const orc_problem *p, cplx *G)
{
    orc_fft2d(G, p->nx, p->ny, 0);
    for (int j = 0; j < p->ny; j++) {
        double ky = kval(j, p->ny, p->ly);
        for (int i = 0; i < p->nx; i++) {
            double kx = kval(i, p->nx, p->lx);
            double ph = 0.5 * (kx * kx + ky * ky) * p->dt;
            G[(size_t)j * p->nx + i] *= cos(ph) + I * sin(ph);
        }
    }
    orc_fft2d(G, p->nx, p->ny, 1);
}

int orc_adjoint_axis(const orc_problem *p, int axis, double t0, const cplx *psi0, const cplx *target,
                     int64_t nsteps, int64_t ckpt, int loss_kind, double *loss, double *grad, cplx *psi_final)
{
    const orc_sched *ctl = axis == 0 ? &p->sx : &p->sy;
    if ((axis != 0 && axis != 1) || ctl->kind != 2 || nsteps < 1) return -1;
    /* the cavity: only the adiabatic field, with the fidelity loss */
    if (p->cavity == 1 || (p->cavity == 2 && loss_kind != 0)) return -1;
    if (ckpt < 1) ckpt = 1;
    size_t npts = (size_t)p->nx * p->ny;
    double da = (p->lx / p->nx) * (p->ly / p->ny), h = 0.5 * p->dt;
    int64_t nck = (nsteps + ckpt - 1) / ckpt;
    cplx *ck = (cplx *)malloc(sizeof(cplx) * npts * (size_t)nck);
    cplx *seg = (cplx *)malloc(sizeof(cplx) * npts * (size_t)(ckpt + 1));
    cplx *psi = (cplx *)malloc(sizeof(cplx) * npts);
    cplx *G = (cplx *)malloc(sizeof(cplx) * npts);
    cplx *a = (cplx *)malloc(sizeof(cplx) * npts);
    cplx *b = (cplx *)malloc(sizeof(cplx) * npts);
    orc_state st = {0};

    /* forward sweep, keeping a checkpoint at the start of every segment */
    memcpy(psi, psi0, sizeof(cplx) * npts);
    st.t = t0;
    for (int64_t c = 0; c < nck; c++) {
        memcpy(ck + (size_t)c * npts, psi, sizeof(cplx) * npts);
        int64_t len = (c == nck - 1) ? nsteps - c * ckpt : ckpt;
        orc_step_real(p, &st, psi, len, NULL);
    }
    double T = t0 + nsteps * p->dt;
    if (psi_final) memcpy(psi_final, psi, sizeof(cplx) * npts);

    /* terminal gradient */
    for (int m = 0; m < ctl->nknots; m++) grad[m] = 0;
    if (loss_kind == 0) {
        cplx c = 0;
        for (size_t q = 0; q < npts; q++) c += conj(target[q]) * psi[q];
        c *= da;
        *loss = 1.0 - (creal(c) * creal(c) + cimag(c) * cimag(c));
        for (size_t q = 0; q < npts; q++) G[q] = -2.0 * c * target[q] * da;
    } else {
        double e[6];
        orc_energy(p, psi, T, 0, 0, e);
        *loss = (e[0] + e[1] + e[2]) * e[5];
        memcpy(G, psi, sizeof(cplx) * npts);
        orc_fft2d(G, p->nx, p->ny, 0);
        for (int j = 0; j < p->ny; j++) {
            double ky = kval(j, p->ny, p->ly);
            for (int i = 0; i < p->nx; i++) {
                double kx = kval(i, p->nx, p->lx);
                G[(size_t)j * p->nx + i] *= 0.5 * (kx * kx + ky * ky);
            }
        }
        orc_fft2d(G, p->nx, p->ny, 1);
        double lat_sum = 0;
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                size_t q = (size_t)j * p->nx + i;
                double dens = creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
                G[q] = 2.0 * da * (G[q] + (potential(p, i, j, T, 0) + p->g * dens) * psi[q]);
                lat_sum += da * control_weight(p, axis, i, j) * dens;
            }
        int i0; double w0, w1;
        hat_weights(ctl, T, &i0, &w0, &w1);
        grad[i0] += w0 * lat_sum;
        grad[i0 + 1] += w1 * lat_sum;
    }

    /* backward sweep, segment by segment */
    for (int64_t c = nck - 1; c >= 0; c--) {
        int64_t n0 = c * ckpt;
        int64_t len = (c == nck - 1) ? nsteps - n0 : ckpt;
        memcpy(seg, ck + (size_t)c * npts, sizeof(cplx) * npts);
        orc_state s2 = {0};
        s2.t = t0 + n0 * p->dt;
        for (int64_t k = 0; k < len; k++) {
            memcpy(seg + (size_t)(k + 1) * npts, seg + (size_t)k * npts, sizeof(cplx) * npts);
            orc_step_real(p, &s2, seg + (size_t)(k + 1) * npts, 1, NULL);
        }
        for (int64_t k = len - 1; k >= 0; k--) {
            double tn = t0 + (n0 + k) * p->dt, tn1 = tn + p->dt;
            const cplx *zout = seg + (size_t)(k + 1) * npts;
            /* second kick at t_{n+1}: output psi_{n+1}, input psi* -> a */
            kick_adjoint(p, axis, zout, a, G, tn1, h, grad);
            /* kinetic: psi' = U^H psi* -> b */
            memcpy(b, a, sizeof(cplx) * npts);
            kinetic_adjoint(p, b);
            kinetic_adjoint(p, G);
            /* first kick at t_n: output psi', input psi_n */
            kick_adjoint(p, axis, b, a, G, tn, h, grad);
        }
    }
    free(ck); free(seg); free(psi); free(G); free(a); free(b);
    return 0;
}

/* ------------------------------------------- the paper's printed ordering */
/*
 * Split step in the ordering the paper prints (Sec. 3.1, Eq. 4): the state is kept in
 * Fourier space, psi_k = FFT2(psi) (unscaled), and one step is
 *   psi_k <- e^{T/2} F[ e^{V} F^{-1}[ e^{T/2} psi_k ] ],
 * e^{T/2} = exp(-i k^2 dt / 4) (imaginary time exp(-k^2 dt / 4)), e^{V} the potential
 * kick over the full dt at the step's midpoint t_n + dt/2 on the real-space density
 * after the first kinetic half.  Imaginary time renormalises psi to unit norm after the
 * step (the norm from Parseval).  The cavity field is held fixed (no cavity ODE here).
 */
static void kinetic_half_k(const orc_problem *p, cplx *psik, int imag)
{
    for (int j = 0; j < p->ny; j++) {
        double ky = kval(j, p->ny, p->ly);
        for (int i = 0; i < p->nx; i++) {
            double kx = kval(i, p->nx, p->lx);
            double ph = 0.25 * (kx * kx + ky * ky) * p->dt;
            size_t q = (size_t)j * p->nx + i;
            psik[q] *= imag ? exp(-ph) : cos(ph) - I * sin(ph);
        }
    }
}

static int step_k(const orc_problem *p, orc_state *s, cplx *psik, int64_t nsteps, int imag, double *obs)
{
    size_t npts = (size_t)p->nx * p->ny;
    double da = (p->lx / p->nx) * (p->ly / p->ny);
    cplx alpha = s->alpha_re + I * s->alpha_im;
    for (int64_t n = 0; n < nsteps; n++) {
        double tm = imag ? s->t : s->t + 0.5 * p->dt;
        kinetic_half_k(p, psik, imag);
        orc_fft2d(psik, p->nx, p->ny, 1);
        kick(p, psik, tm, alpha, p->dt, imag);
        orc_fft2d(psik, p->nx, p->ny, 0);
        kinetic_half_k(p, psik, imag);
        double nrm = 0;
        for (size_t q = 0; q < npts; q++) nrm += creal(psik[q]) * creal(psik[q]) + cimag(psik[q]) * cimag(psik[q]);
        nrm *= da / (double)npts;
        if (imag) {
            double sc = 1.0 / sqrt(nrm);
            for (size_t q = 0; q < npts; q++) psik[q] *= sc;
        } else {
            s->t += p->dt;
        }
        if (obs) obs[n] = nrm;
    }
    return 0;
}

/* obs (nullable): nsteps norms (imaginary time: before renormalisation). */
int orc_step_real_k(const orc_problem *p, orc_state *s, cplx *psik, int64_t nsteps, double *obs)
{
    if (p->cavity) return -1;
    return step_k(p, s, psik, nsteps, 0, obs);
}

int orc_step_imag_k(const orc_problem *p, orc_state *s, cplx *psik, int64_t nsteps, double *obs)
{
    if (p->cavity) return -1;
    return step_k(p, s, psik, nsteps, 1, obs);
}

/* Momentum-order populations of a Fourier-space state (Sec. 5.2: the populations of
 * |2 n hbar k> are read off the reciprocal-space amplitude).  psik = FFT2(psi), [ny][nx].
 * The signed bin m along `axis` (0: x, 1: y) belongs to order floor((m + floor(B/2)) / B),
 * B = order_step FFT bins between orders.  out[n + nmax] = fraction of sum |psik|^2 in
 * order n for |n| <= nmax; out[2 nmax + 1] = sum |psik|^2 dx dy / (nx ny) (Parseval). */
int orc_momentum_orders(const orc_problem *p, const cplx *psik, int axis, int order_step, int nmax, double *out)
{
    int n = axis == 0 ? p->nx : p->ny;
    if ((axis != 0 && axis != 1) || order_step < 1 || nmax < 0 || (2 * nmax + 1) * order_step > n) return -1;
    for (int q = 0; q < 2 * nmax + 1; q++) out[q] = 0.0;
    double tot = 0.0;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            int b = axis == 0 ? i : j;
            int m = b >= n / 2 ? b - n : b;
            int ord = (int)floor((double)(m + order_step / 2) / order_step);
            double w = creal(psik[(size_t)j * p->nx + i]) * creal(psik[(size_t)j * p->nx + i]) +
                       cimag(psik[(size_t)j * p->nx + i]) * cimag(psik[(size_t)j * p->nx + i]);
            tot += w;
            if (ord >= -nmax && ord <= nmax) out[ord + nmax] += w;
        }
    for (int q = 0; q < 2 * nmax + 1; q++) out[q] = tot > 0 ? out[q] / tot : 0.0;
    out[2 * nmax + 1] = tot * (p->lx / p->nx) * (p->ly / p->ny) / ((double)p->nx * p->ny);
    return 0;
}

/* The x-lattice control (axis 0). */
int orc_adjoint(const orc_problem *p, double t0, const cplx *psi0, const cplx *target, int64_t nsteps,
                int64_t ckpt, int loss_kind, double *loss, double *grad, cplx *psi_final)
{
    return orc_adjoint_axis(p, 0, t0, psi0, target, nsteps, ckpt, loss_kind, loss, grad, psi_final);
}
