/*
 * Plain FP64 CPU oracle for the staggered-leapfrog lattice evolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * and no header with the GPU library.
 *
 * What is computed (paper, section "Parallel Algorithms", description of the
 * integrator): a staggered leapfrog with a fixed step.  Field values f live at
 * integer times t_n, their derivatives at half times t_n + dt/2.  One step
 * first advances f by a full dt using the derivatives (drift), then evaluates
 * the second derivative from the new field values, then advances the
 * derivatives by dt (kick).  Both updates overwrite the arrays in place.
 *
 * The paper gives no equations of motion.  The ones below are derived from
 * the Friedmann-Robertson-Walker equations for minimally coupled scalar
 * fields (not taken from any program):
 *   evolved variable   f_i = a * phi_i / phi_0   (conformal program field)
 *   time               d tau = sqrt(lambda) phi_0 dt / a  (conformal)
 *   field equation     f_i'' = Lap f_i - dV/df_i + (a''/a) f_i
 *   potential          V = lambda/4 f0^4 + sum_{j>=1} G_j/2 f0^2 fj^2
 *                          + a^2/2 sum_i mu_i^2 f_i^2 + a^4 V0
 *   scale factor       a'' = -a'^2/a + kappa (2/3 Grad + V) / a
 *   constraint (check) a'^2 = kappa rho / 3,  rho = Kin + Grad + V
 * with kappa = 8 pi (phi_0/M_p)^2 and all energies comoving (volume means).
 *
 * Spatial derivatives are nearest-neighbour only: the paper's slab layout keeps
 * exactly one buffer column on each side of a processor's slab, which fixes
 * the stencil radius at one site.  The Laplacian is the (2d+1)-point periodic
 * stencil with spacing dx = L/N; the gradient energy uses forward differences.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math), so rounding is plain IEEE
 * round-to-nearest-even in the order written.
 *
 * Pins (tests/test_oracle_*.py): the Laplacian's Fourier multiplier, the exact
 * discrete dispersion of free modes, the homogeneous quartic (cn) and RK4
 * integrations with expansion and vacuum energy, closed-form kinetic and de
 * Sitter expansion, energy conservation and the Friedmann residual at second
 * order, summation by parts, symmetries, the radius-one reach, and brute force
 * on 4^3 lattices (exact matrix powers; 50-digit arithmetic for the nonlinear
 * case).  The paper prints no values for the resonant regime, so beyond these
 * invariants the nonlinear evolution is parity unpinned except by this oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_FIELDS 3
#define OR_MAX_TERMS 8

/* One term coef * phi_0^e0 phi_1^e1 phi_2^e2 of a user-defined polynomial
 * potential (the model a run names, as the paper's "Overview" section lets
 * every run bring its own potential and derivatives). */
typedef struct {
    double coef;
    int32_t exp[OR_MAX_FIELDS];
    int32_t pad;
} or_term;

typedef struct {
    int32_t dims;       /* 1, 2 or 3 */
    int32_t N;          /* points per edge */
    int32_t nfields;    /* 1..3; field 0 is the inflaton */
    int32_t expansion;  /* 0: a == 1 fixed; 1: self-consistent a(tau) */
    double L;           /* box edge, program units */
    double dt;          /* time step, program units */
    double lambda;      /* quartic self-coupling (1 in program units) */
    double G[OR_MAX_FIELDS];   /* G_j = g_j^2/lambda for j >= 1; G[0] unused */
    double mu2[OR_MAX_FIELDS]; /* mass^2 per field, program units */
    double kappa;       /* 8 pi (phi_0/M_p)^2, used only with expansion */
    double vacuum;      /* V0, the constant term of the physical potential */
    int32_t nterms;     /* > 0: the potential is the polynomial below instead */
    int32_t pad;
    or_term terms[OR_MAX_TERMS];
} or_params;

/* Scalar state at integer step n plus the diagnostics at that step. */
typedef struct {
    int64_t step;
    double tau;
    double a;           /* a^n */
    double adot_half;   /* a'^{n+1/2} */
    double adot;        /* a' at t_n (mean of the two neighbouring half steps) */
    double kin[OR_MAX_FIELDS];
    double grad[OR_MAX_FIELDS];
    double pot;
    double rho;
    double mean[OR_MAX_FIELDS];
    double mean_sq[OR_MAX_FIELDS];
    double resid;       /* (a'^2 - kappa rho/3) / a'^2; 0 without expansion */
} or_state;

static int64_t n_sites(const or_params *p)
{
    int64_t n = 1;
    for (int d = 0; d < p->dims; d++) n *= p->N;
    return n;
}

/* Stride of spatial axis d in C order (axis dims-1 is contiguous). */
static int64_t axis_stride(const or_params *p, int d)
{
    int64_t s = 1;
    for (int e = p->dims - 1; e > d; e--) s *= p->N;
    return s;
}

/* Index of the neighbour of site s one step along axis d, direction dir = +-1,
 * with periodic wrap. */
static int64_t neighbour(const or_params *p, int64_t s, int d, int dir)
{
    int64_t st = axis_stride(p, d);
    int64_t c = (s / st) % p->N;
    int64_t cn = (c + dir + p->N) % p->N;
    return s + (cn - c) * st;
}

/* Discrete Laplacian of one field at one site: sum over axes of
 * (f(x+e) + f(x-e) - 2 f(x)) / dx^2.  The two neighbours of an axis are added
 * first, so mirror-image configurations give bitwise mirror-image results. */
static double lap_at(const or_params *p, const double *f, int64_t s)
{
    double dx = p->L / p->N;
    double acc = 0.0;
    for (int d = 0; d < p->dims; d++) {
        double pair = f[neighbour(p, s, d, +1)] + f[neighbour(p, s, d, -1)];
        acc += pair - 2.0 * f[s];
    }
    return acc / (dx * dx);
}

/* x^e for a small non-negative integer e, as a plain product. */
static double ipow(double x, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; k++) r *= x;
    return r;
}

/* Polynomial potential in the program variables f = a phi: the physical
 * term coef prod_i phi_i^e_i becomes coef a^(4 - D) prod_i f_i^e_i, with D
 * the term's total degree. */
static double poly_pot(const or_params *p, const double *v, double a)
{
    double V = 0.0;
    for (int t = 0; t < p->nterms; t++) {
        int D = 0;
        double mono = p->terms[t].coef;
        for (int i = 0; i < p->nfields; i++) {
            D += p->terms[t].exp[i];
            mono *= ipow(v[i], p->terms[t].exp[i]);
        }
        V += mono * pow(a, 4 - D);
    }
    return V;
}

/* d/df_i of the polynomial potential: each term's exponent of f_i times the
 * product with that exponent lowered by one. */
static double poly_dpot(const or_params *p, const double *v, double a, int i)
{
    double r = 0.0;
    for (int t = 0; t < p->nterms; t++) {
        int ei = p->terms[t].exp[i];
        if (ei == 0) continue;
        int D = 0;
        double mono = p->terms[t].coef * (double)ei;
        for (int j = 0; j < p->nfields; j++) {
            D += p->terms[t].exp[j];
            mono *= ipow(v[j], j == i ? ei - 1 : p->terms[t].exp[j]);
        }
        r += mono * pow(a, 4 - D);
    }
    return r;
}

/* Potential energy density at one site (fields v[0..nfields-1]). */
static double pot_at(const or_params *p, const double *v, double a)
{
    if (p->nterms > 0) return poly_pot(p, v, a);
    double f0sq = v[0] * v[0];
    double V = 0.25 * p->lambda * f0sq * f0sq;
    for (int j = 1; j < p->nfields; j++) V += 0.5 * p->G[j] * f0sq * v[j] * v[j];
    for (int i = 0; i < p->nfields; i++) V += 0.5 * a * a * p->mu2[i] * v[i] * v[i];
    /* a constant V0 of the physical potential is a^4 V0 in conformal variables */
    V += a * a * a * a * p->vacuum;
    return V;
}

/* dV/df_i at one site. */
static double dpot_at(const or_params *p, const double *v, double a, int i)
{
    if (p->nterms > 0) return poly_dpot(p, v, a, i);
    double r;
    if (i == 0) {
        double chisq = 0.0;
        for (int j = 1; j < p->nfields; j++) chisq += p->G[j] * v[j] * v[j];
        r = p->lambda * v[0] * v[0] * v[0] + v[0] * chisq;
    } else {
        r = p->G[i] * v[0] * v[0] * v[i];
    }
    return r + a * a * p->mu2[i] * v[i];
}

static void gather(const or_params *p, const double *f, int64_t ns, int64_t s, double *v)
{
    for (int i = 0; i < p->nfields; i++) v[i] = f[(int64_t)i * ns + s];
}

/* ---- exported building blocks (used by the invariant tests) ---- */

void or_laplacian(const or_params *p, const double *f, double *out)
{
    int64_t ns = n_sites(p);
    for (int64_t s = 0; s < ns; s++) out[s] = lap_at(p, f, s);
}

/* Gradient energy of one field: 1/2 < sum_d (D+_d f)^2 >, forward differences. */
double or_grad_energy(const or_params *p, const double *f)
{
    int64_t ns = n_sites(p);
    double dx = p->L / p->N;
    double acc = 0.0;
    for (int64_t s = 0; s < ns; s++) {
        for (int d = 0; d < p->dims; d++) {
            double df = (f[neighbour(p, s, d, +1)] - f[s]) / dx;
            acc += df * df;
        }
    }
    return 0.5 * acc / (double)ns;
}

/* Volume mean of the potential for fields f[nfields][ns] at scale factor a. */
double or_mean_potential(const or_params *p, const double *f, double a)
{
    int64_t ns = n_sites(p);
    double v[OR_MAX_FIELDS];
    double acc = 0.0;
    for (int64_t s = 0; s < ns; s++) {
        gather(p, f, ns, s, v);
        acc += pot_at(p, v, a);
    }
    return acc / (double)ns;
}

double or_potential_point(const or_params *p, const double *v, double a)
{
    return pot_at(p, v, a);
}

double or_dpotential_point(const or_params *p, const double *v, double a, int32_t i)
{
    return dpot_at(p, v, a, i);
}

/* Scale-factor half-step update.  With y = a'^{n+1/2}, x = a'^{n+3/2} and the
 * time-centred a' taken as (x+y)/2, the leapfrog kick
 *     x = y + dt ( S - ((x+y)/2)^2 / a ),   S = kappa (2/3 Grad + V) / a
 * is the quadratic A x^2 + B x + C = 0 with the coefficients below.  The root
 * that tends to y as dt -> 0 is taken in the form free of cancellation. */
double or_solve_adot(double a, double y, double S, double dt)
{
    double A = dt / (4.0 * a);
    double B = 1.0 + dt * y / (2.0 * a);
    double C = dt * y * y / (4.0 * a) - y - dt * S;
    return -2.0 * C / (B + sqrt(B * B - 4.0 * A * C));
}

static void means(const or_params *p, const double *f, or_state *st)
{
    int64_t ns = n_sites(p);
    for (int i = 0; i < p->nfields; i++) {
        const double *fi = f + (int64_t)i * ns;
        double s1 = 0.0, s2 = 0.0;
        for (int64_t s = 0; s < ns; s++) {
            s1 += fi[s];
            s2 += fi[s] * fi[s];
        }
        st->mean[i] = s1 / (double)ns;
        st->mean_sq[i] = s2 / (double)ns;
    }
}

static void finish_diagnostics(const or_params *p, or_state *st)
{
    double rho = st->pot;
    for (int i = 0; i < p->nfields; i++) rho += st->kin[i] + st->grad[i];
    st->rho = rho;
    if (p->expansion && st->adot != 0.0)
        st->resid = (st->adot * st->adot - p->kappa * rho / 3.0) / (st->adot * st->adot);
    else
        st->resid = 0.0;
}

/*
 * Start-up.  The initial data are the physical program-unit field phi and its
 * time derivative phidot at tau = 0 with a(0) = 1.  The paper stores the
 * derivative half a step ahead of the field but does not say how the first half
 * step is taken; here it is one half kick of the same equations:
 *   f^0     = phi
 *   a'^0    = +sqrt(kappa rho^0 / 3)      (0 without expansion)
 *   f'^0    = phidot + a'^0 phi           (derivative of a*phi at a = 1)
 *   a''^0   = -a'^0^2 + kappa (2/3 Grad^0 + V^0)
 *   pi^{1/2}   = f'^0 + dt/2 (Lap f^0 - dV/df + a''^0 f^0)
 *   a'^{1/2}   = a'^0 + dt/2 a''^0
 * f and pi (both [nfields][N^dims]) are written; st receives step-0 diagnostics.
 */
void or_start(const or_params *p, const double *phi, const double *phidot,
              double *f, double *pi, or_state *st)
{
    int64_t ns = n_sites(p);
    int nf = p->nfields;
    memset(st, 0, sizeof(*st));
    memcpy(f, phi, sizeof(double) * (size_t)(nf * ns));

    st->step = 0;
    st->tau = 0.0;
    st->a = 1.0;
    double gsum = 0.0;
    for (int i = 0; i < nf; i++) {
        const double *fd = phidot + (int64_t)i * ns;
        double k = 0.0;
        for (int64_t s = 0; s < ns; s++) k += fd[s] * fd[s];
        st->kin[i] = 0.5 * k / (double)ns;
        st->grad[i] = or_grad_energy(p, f + (int64_t)i * ns);
        gsum += st->grad[i];
    }
    st->pot = or_mean_potential(p, f, 1.0);
    means(p, f, st);

    double ap0 = 0.0, app0 = 0.0;
    if (p->expansion) {
        double rho0 = st->pot;
        for (int i = 0; i < nf; i++) rho0 += st->kin[i] + st->grad[i];
        ap0 = sqrt(p->kappa * rho0 / 3.0);
        app0 = -ap0 * ap0 + p->kappa * (2.0 / 3.0 * gsum + st->pot);
    }
    st->adot = ap0;
    finish_diagnostics(p, st);

    double v[OR_MAX_FIELDS];
    for (int64_t s = 0; s < ns; s++) {
        gather(p, f, ns, s, v);
        for (int i = 0; i < nf; i++) {
            const double *fi = f + (int64_t)i * ns;
            int64_t k = (int64_t)i * ns + s;
            double fprime = phidot[k] + ap0 * fi[s];
            double force = lap_at(p, fi, s) - dpot_at(p, v, 1.0, i) + app0 * fi[s];
            pi[k] = fprime + 0.5 * p->dt * force;
        }
    }
    st->adot_half = ap0 + 0.5 * p->dt * app0;
}

/*
 * One leapfrog step n -> n+1, in place, in the paper's order:
 *   1. drift:   f^{n+1} = f^n + dt pi^{n+1/2}                (all sites)
 *   2.          a^{n+1} = a^n + dt a'^{n+1/2}
 *   3. volume means of Grad and V at n+1
 *   4. a'^{n+3/2} from the quadratic above; c^{n+1} = a''/a at n+1
 *   5. kick:    pi^{n+3/2} = pi^{n+1/2}
 *                   + dt (Lap f^{n+1} - dV/df(f^{n+1}; a^{n+1}) + c^{n+1} f^{n+1})
 * The drift is pointwise and the kick writes only pi, so updating in place is
 * safe.  Diagnostics at n+1: the kinetic energy uses the time-centred momentum
 * u = (pi^{n+1/2} + pi^{n+3/2})/2 - (abar/a) f with abar the mean of the two
 * half-step a' values.  Without expansion a == 1 and a' == c == 0.
 */
void or_step(const or_params *p, double *f, double *pi, or_state *st)
{
    int64_t ns = n_sites(p);
    int nf = p->nfields;
    double dt = p->dt;

    for (int64_t k = 0; k < (int64_t)nf * ns; k++) f[k] += dt * pi[k];

    double a1 = p->expansion ? st->a + dt * st->adot_half : 1.0;
    double gsum = 0.0;
    for (int i = 0; i < nf; i++) {
        st->grad[i] = or_grad_energy(p, f + (int64_t)i * ns);
        gsum += st->grad[i];
    }
    st->pot = or_mean_potential(p, f, a1);

    double x = 0.0, abar = 0.0, c = 0.0;
    if (p->expansion) {
        double S = p->kappa * (2.0 / 3.0 * gsum + st->pot) / a1;
        x = or_solve_adot(a1, st->adot_half, S, dt);
        abar = 0.5 * (x + st->adot_half);
        c = (S - abar * abar / a1) / a1;
    }

    double v[OR_MAX_FIELDS];
    double ksum[OR_MAX_FIELDS] = {0.0, 0.0, 0.0};
    for (int64_t s = 0; s < ns; s++) {
        gather(p, f, ns, s, v);
        for (int i = 0; i < nf; i++) {
            const double *fi = f + (int64_t)i * ns;
            int64_t k = (int64_t)i * ns + s;
            double force = lap_at(p, fi, s) - dpot_at(p, v, a1, i) + c * fi[s];
            double pnew = pi[k] + dt * force;
            double u = 0.5 * (pi[k] + pnew) - (abar / a1) * fi[s];
            ksum[i] += u * u;
            pi[k] = pnew;
        }
    }

    st->step += 1;
    st->tau += dt;
    st->a = a1;
    st->adot_half = x;
    st->adot = abar;
    for (int i = 0; i < nf; i++) st->kin[i] = 0.5 * ksum[i] / (double)ns;
    means(p, f, st);
    finish_diagnostics(p, st);
}

/* Run nsteps steps; if log is not NULL, log[k] receives the diagnostics after
 * step k+1. */
void or_run(const or_params *p, double *f, double *pi, or_state *st,
            int64_t nsteps, or_state *log)
{
    for (int64_t k = 0; k < nsteps; k++) {
        or_step(p, f, pi, st);
        if (log) log[k] = *st;
    }
}

int32_t or_sizeof_params(void) { return (int32_t)sizeof(or_params); }
int32_t or_sizeof_state(void) { return (int32_t)sizeof(or_state); }
